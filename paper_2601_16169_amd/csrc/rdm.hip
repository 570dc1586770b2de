// Spin-summed reduced density matrices of a normalised vector c, the energy
// gradients by Hellmann-Feynman: dE/dh_pq = rdm1_pq, dE/d(pq|rs) = rdm2_pqrs/2
// (E = ecore + sum h.rdm1 + 1/2 sum (pq|rs) rdm2 for the Hamiltonian of
// Sec. I-II restricted to the product space of Sec. IV).
//
//   rdm1[p,q]     = sum_s <a+_ps a_qs>
//   rdm2[p,q,r,s] = sum_st <a+_ps a+_rt a_st a_qs>
//
// Same-spin parts come from pairs of strings of one spin connected by the
// excitation tables (or equal), weighted by the overlap of the matching rows
// (alpha) or columns (beta) of C: P_a = C C^T, P_b = C^T C, two FP64 MFMA
// GEMMs.  The alpha-beta part is
//   X[pq][rs] = <c| E^a_pq E^b_rs |c> = sum_{K in S} (E^a_qp c)_K (E^b_rs c)_K ,
// a D_a^T D_b product over all determinants; for one alpha string Ia the
// alpha factor is non-zero only on the pairs pq reached by Ia's singles and
// its diagonal, so each workgroup takes one Ia and multiplies a dense
// (pairs of Ia) x (beta chunk) block by the beta factor scattered densely into
// LDS, on FP64 MFMA (v_mfma_f64_16x16x4), accumulating over beta chunks.
// rdm2 receives X[pq][rs] + X[rs][pq] (the beta-alpha term).
#include "sqd_internal.h"

namespace {

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

typedef double double4_t __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4: A[i][k] from lane i + 16 k, B[k][j] from lane j + 16 k;
// lane l, element q of the accumulator holds D[l / 16 + 4 q][l % 16] (checked on
// gfx950; the f32 form of the same shape uses row 4 (l / 16) + q instead).
__device__ __forceinline__ int acc_row(int lane, int q) { return (lane >> 4) + 4 * q; }

// ---------------------------------------------------------------- P = A B^T
// A: M x K, B: N x K (row-major, leading dimension K); P: M x N.  64 x 64
// block tile, four waves of 32 x 32 (2 x 2 MFMA tiles), K steps of 16 in LDS.
__global__ void __launch_bounds__(256)
k_gemm_nt(const double* __restrict__ A, const double* __restrict__ B, double* __restrict__ P, int64_t M, int64_t N,
          int64_t K) {
    __shared__ double As[64][17];
    __shared__ double Bs[64][17];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t m0 = (int64_t)blockIdx.y * 64, n0 = (int64_t)blockIdx.x * 64;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    double4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (double4_t){0.0, 0.0, 0.0, 0.0};
    for (int64_t k0 = 0; k0 < K; k0 += 16) {
        for (int idx = tid; idx < 64 * 16; idx += 256) {
            const int r = idx >> 4, c = idx & 15;
            const int64_t gk = k0 + c;
            As[r][c] = (m0 + r < M && gk < K) ? A[(m0 + r) * K + gk] : 0.0;
            Bs[r][c] = (n0 + r < N && gk < K) ? B[(n0 + r) * K + gk] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 16; ks += 4) {
            double a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[wm + i * 16 + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[wn + j * 16 + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t r = m0 + wm + i * 16 + acc_row(lane, q);
                const int64_t c = n0 + wn + j * 16 + (lane & 15);
                if (r < M && c < N) P[r * N + c] = acc[i][j][q];
            }
}

// ---------------------------------------------------------------- same spin
// One wavefront per string I of one spin; w(J) = P[I][J].  Pairs visited in
// both directions by the symmetric tables.  Updates (Gamma_pqrs = <a+_p a+_r a_s a_q>):
//   diagonal:   rdm1[k][k] += w;  Gamma[k][k][l][l] += w, Gamma[l][k][k][l] -= w (k != l in I)
//   single (i in I, a in J, sign s; spectators k in I, k != i):
//               rdm1[i][a] += s w; Gamma[i][a][k][k] += s w, Gamma[k][k][i][a] += s w,
//               Gamma[k][a][i][k] -= s w, Gamma[i][k][k][a] -= s w
//   double (i < j in I, a < b in J, sign s):
//               Gamma[i][a][j][b] += s w, Gamma[j][b][i][a] += s w,
//               Gamma[j][a][i][b] -= s w, Gamma[i][b][j][a] -= s w
__global__ void __launch_bounds__(256)
k_rdm_same(const uint64_t* __restrict__ str, int nw, int64_t n, const int* __restrict__ s_off,
           const uint64_t* __restrict__ s_ent, const int* __restrict__ d_off, const uint64_t* __restrict__ d_ent,
           const double* __restrict__ P, int norb, double* __restrict__ rdm1, double* __restrict__ rdm2) {
    const int64_t I = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (I >= n) return;
    const int64_t n2 = (int64_t)norb * norb;
    auto G = [&](int p, int q, int r, int s) -> double* { return rdm2 + ((int64_t)p * norb + q) * n2 + r * norb + s; };
    const uint64_t* sI = str + I * nw;
    const double wd = P[I * n + I];
    // diagonal
    for (int k = lane; k < norb; k += 64) {
        if (!str_bit(sI, k)) continue;
        atomicAdd(&rdm1[k * norb + k], wd);
        if (rdm2)
            str_for_each(sI, nw, [&](int l) {
                if (l == k) return;
                atomicAdd(G(k, k, l, l), wd);
                atomicAdd(G(l, k, k, l), -wd);
            });
    }
    for (int e = s_off[I] + lane; e < s_off[I + 1]; e += 64) {
        const uint64_t x = s_ent[e];
        const int64_t J = (int64_t)(x & 0xFFFFFFFFull);
        const int i = SQD_ENT_ORB(x, 0), a = SQD_ENT_ORB(x, 1);
        const double sw = ((x >> 63) ? -1.0 : 1.0) * P[I * n + J];
        atomicAdd(&rdm1[i * norb + a], sw);
        if (rdm2)
            str_for_each(sI, nw, [&](int k) {
                if (k == i) return;
                atomicAdd(G(i, a, k, k), sw);
                atomicAdd(G(k, k, i, a), sw);
                atomicAdd(G(k, a, i, k), -sw);
                atomicAdd(G(i, k, k, a), -sw);
            });
    }
    if (!rdm2) return;
    for (int e = d_off[I] + lane; e < d_off[I + 1]; e += 64) {
        const uint64_t x = d_ent[e];
        const int64_t J = (int64_t)(x & 0xFFFFFFFFull);
        const int i = SQD_ENT_ORB(x, 0), j = SQD_ENT_ORB(x, 1);
        const int a = SQD_ENT_ORB(x, 2), b = SQD_ENT_ORB(x, 3);
        const double sw = ((x >> 63) ? -1.0 : 1.0) * P[I * n + J];
        atomicAdd(G(i, a, j, b), sw);
        atomicAdd(G(j, b, i, a), sw);
        atomicAdd(G(j, a, i, b), -sw);
        atomicAdd(G(i, b, j, a), -sw);
    }
}

// ---------------------------------------------------------------- alpha-beta
constexpr int kKC = 32;        // beta strings per K chunk
constexpr int kMaxNC = 512;    // rs columns per N chunk
constexpr int kMaxTiles = 16;  // output tiles per wave: (32/16) x (512/16) / 4 waves

// One workgroup per alpha string Ia.  U = alpha factor entries of Ia: its
// singles (pair a*norb+i, source row Ja, sign) then its diagonal pairs pp.
__global__ void __launch_bounds__(256)
k_rdm_ab(const double* __restrict__ C, int64_t na, int64_t nb, const uint64_t* __restrict__ astr, int nw,
         const int* __restrict__ a_off, const uint32_t* __restrict__ a_pk, const uint64_t* __restrict__ bstr,
         const int* __restrict__ b_off, const uint32_t* __restrict__ b_pk, int norb, double* __restrict__ rdm2) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int n2 = norb * norb;
    const int npad = (n2 + 15) & ~15;
    const int nc_max = npad < kMaxNC ? npad : kMaxNC;
    double* Bs = reinterpret_cast<double*>(lds_raw);       // [kKC][nc_max]
    double* As = Bs + kKC * nc_max;                        // [32][kKC + 1]
    int* upq = reinterpret_cast<int*>(As + 32 * (kKC + 1));  // [nu_total]
    const int64_t ia = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t* sa = astr + ia * nw;
    const int s0 = a_off[ia], ns = a_off[ia + 1] - s0;
    int ndiag = 0;
    for (int q = 0; q < nw; ++q) ndiag += __popcll(sa[q]);
    const int nu = ns + ndiag;
    // pair index of each U entry
    for (int u = tid; u < nu; u += 256) {
        int pq;
        if (u < ns) {
            pq = (int)((a_pk[s0 + u] >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK);
        } else {
            // the (u - ns)-th occupied orbital p of Ia
            int skip = u - ns, p = -1;
            str_for_each(sa, nw, [&](int k) {
                if (p < 0 && skip-- == 0) p = k;
            });
            pq = p * norb + p;
        }
        upq[u] = pq;
    }
    for (int k = tid; k < kKC * nc_max; k += 256) Bs[k] = 0.0;
    __syncthreads();
    const double* crow = C + ia * nb;
    for (int u0 = 0; u0 < nu; u0 += 32) {
        for (int n0 = 0; n0 < npad; n0 += nc_max) {
            const int nc = (npad - n0) < nc_max ? (npad - n0) : nc_max;
            const int ntiles = 2 * (nc / 16);
            double4_t acc[kMaxTiles];
#pragma unroll
            for (int t = 0; t < kMaxTiles; ++t) acc[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
            for (int64_t b0 = 0; b0 < nb; b0 += kKC) {
                // alpha factor: As[u][k] = sign_u * C[src_u][b0 + k]
                for (int idx = tid; idx < 32 * kKC; idx += 256) {
                    const int u = idx / kKC, k = idx % kKC;
                    double v = 0.0;
                    const int uu = u0 + u;
                    if (uu < nu && b0 + k < nb) {
                        if (uu < ns) {
                            const uint32_t e = a_pk[s0 + uu];
                            v = C[(int64_t)(e & SQD_NBR_MASK) * nb + b0 + k];
                            if (e >> 31) v = -v;
                        } else {
                            v = crow[b0 + k];
                        }
                    }
                    As[u * (kKC + 1) + k] = v;
                }
                // beta factor of this chunk scattered densely: Bs[k][rs - n0]
                for (int idx = tid; idx < kKC * 64; idx += 256) {
                    const int k = idx >> 6, j = idx & 63;
                    const int64_t ib = b0 + k;
                    if (ib >= nb) continue;
                    const int e0 = b_off[ib], e1 = b_off[ib + 1];
                    for (int e = e0 + j; e < e1; e += 64) {
                        const uint32_t x = b_pk[e];
                        const int pair = (int)((x >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK);
                        const int rs = (pair % norb) * norb + pair / norb;   // r = i (in Ib), s = a
                        if (rs < n0 || rs >= n0 + nc) continue;
                        double v = crow[x & SQD_NBR_MASK];
                        if (x >> 31) v = -v;
                        Bs[k * nc_max + (rs - n0)] = v;
                    }
                    for (int jj = j; jj < norb; jj += 64) {
                        if (!str_bit(bstr + ib * nw, jj)) continue;
                        const int rs = jj * norb + jj;
                        if (rs >= n0 && rs < n0 + nc) Bs[k * nc_max + (rs - n0)] = crow[ib];
                    }
                }
                __syncthreads();
#pragma unroll
                for (int t = 0; t < kMaxTiles; ++t) {
                    const int tile = w + 4 * t;
                    if (tile < ntiles) {
                        const int ut = tile & 1, nt = tile >> 1;
#pragma unroll
                        for (int ks = 0; ks < kKC; ks += 4) {
                            const double a = As[(ut * 16 + (lane & 15)) * (kKC + 1) + ks + (lane >> 4)];
                            const double b = Bs[(ks + (lane >> 4)) * nc_max + nt * 16 + (lane & 15)];
                            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
                        }
                    }
                }
                __syncthreads();
                // clear the scattered entries for the next chunk
                for (int idx = tid; idx < kKC * 64; idx += 256) {
                    const int k = idx >> 6, j = idx & 63;
                    const int64_t ib = b0 + k;
                    if (ib >= nb) continue;
                    const int e0 = b_off[ib], e1 = b_off[ib + 1];
                    for (int e = e0 + j; e < e1; e += 64) {
                        const int pair = (int)((b_pk[e] >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK);
                        const int rs = (pair % norb) * norb + pair / norb;
                        if (rs >= n0 && rs < n0 + nc) Bs[k * nc_max + (rs - n0)] = 0.0;
                    }
                    for (int jj = j; jj < norb; jj += 64) {
                        if (!str_bit(bstr + ib * nw, jj)) continue;
                        const int rs = jj * norb + jj;
                        if (rs >= n0 && rs < n0 + nc) Bs[k * nc_max + (rs - n0)] = 0.0;
                    }
                }
                __syncthreads();
            }
            // rdm2[pq][rs] += X, rdm2[rs][pq] += X
#pragma unroll
            for (int t = 0; t < kMaxTiles; ++t) {
                const int tile = w + 4 * t;
                if (tile < ntiles) {
                    const int ut = tile & 1, nt = tile >> 1;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int u = u0 + ut * 16 + acc_row(lane, q);
                        const int rs = n0 + nt * 16 + (lane & 15);
                        const double v = acc[t][q];
                        if (u < nu && rs < n2 && v != 0.0) {
                            const int pq = upq[u];
                            atomicAdd(&rdm2[(int64_t)pq * n2 + rs], v);
                            atomicAdd(&rdm2[(int64_t)rs * n2 + pq], v);
                        }
                    }
                }
            }
        }
    }
}

template <typename T>
__global__ void k_zero(T* __restrict__ p, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = (T)0;
}

__global__ void __launch_bounds__(256) k_transpose_d(const double* __restrict__ in, double* __restrict__ out,
                                                     int64_t rows, int64_t cols) {
    __shared__ double tile[64][65];
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int k = ty; k < 64; k += 4) {
        const int64_t r = r0 + k, c = c0 + tx;
        if (r < rows && c < cols) tile[k][tx] = in[r * cols + c];
    }
    __syncthreads();
    for (int k = ty; k < 64; k += 4) {
        const int64_t c = c0 + k, r = r0 + tx;
        if (r < rows && c < cols) out[c * rows + r] = tile[tx][k];
    }
}

}  // namespace

int sqd_rdm_impl(sqd_ctx* ctx, sqd_space* sp, const double* c, double* rdm1, double* rdm2) {
    int rc = sqd_build_values(ctx, sp);
    if (rc) return rc;
    const spin_tables& A = sp->sp[0];
    const spin_tables& B = sp->sp[1];
    const int64_t na = A.n, nb = B.n;
    const int norb = sp->norb;
    const int64_t n2 = (int64_t)norb * norb;
    hipStream_t s = ctx->stream;
    // scratch: P_a (na^2), P_b (nb^2), C^T (dim)
    const size_t bytes = sizeof(double) * ((size_t)na * na + (size_t)nb * nb + (size_t)sp->dim + 64);
    void* scr = sqd_ctx_scratch(ctx, bytes, &rc);
    if (!scr) return sqd_fail(ctx, SQD_E_OOM, "RDM scratch allocation failed (" + std::to_string(bytes) + " bytes)");
    double* Pa = (double*)scr;
    double* Pb = Pa + na * na;
    double* Ct = Pb + nb * nb;
    hipLaunchKernelGGL(k_zero<double>, dim3(nblk(n2, 256)), dim3(256), 0, s, rdm1, n2);
    if (rdm2) hipLaunchKernelGGL(k_zero<double>, dim3(nblk(n2 * n2, 256)), dim3(256), 0, s, rdm2, n2 * n2);
    // overlaps of alpha rows and of beta columns
    hipLaunchKernelGGL(k_gemm_nt, dim3(nblk(na, 64), nblk(na, 64)), dim3(256), 0, s, c, c, Pa, na, na, nb);
    hipLaunchKernelGGL(k_transpose_d, dim3(nblk(nb, 64), nblk(na, 64)), dim3(256), 0, s, c, Ct, na, nb);
    hipLaunchKernelGGL(k_gemm_nt, dim3(nblk(nb, 64), nblk(nb, 64)), dim3(256), 0, s, Ct, Ct, Pb, nb, nb, na);
    hipLaunchKernelGGL(k_rdm_same, dim3(nblk(na, 4)), dim3(256), 0, s, A.str, sp->nw, na, A.s_off, A.s_ent, A.d_off,
                       A.d_ent, Pa, norb, rdm1, rdm2);
    hipLaunchKernelGGL(k_rdm_same, dim3(nblk(nb, 4)), dim3(256), 0, s, B.str, sp->nw, nb, B.s_off, B.s_ent, B.d_off,
                       B.d_ent, Pb, norb, rdm1, rdm2);
    if (rdm2) {
        const int npad = (int)((n2 + 15) & ~15);
        const int nc_max = npad < kMaxNC ? npad : kMaxNC;
        // LDS: beta chunk, alpha chunk and the pair list of one alpha string
        const size_t maxu = (size_t)A.max_singles + sp->nalpha + 1;
        const size_t lds = sizeof(double) * ((size_t)kKC * nc_max + 32 * (kKC + 1)) + sizeof(int) * maxu;
        if (lds > (size_t)ctx->max_lds) return sqd_fail(ctx, SQD_E_LIMIT, "RDM alpha-beta tile does not fit in LDS");
        hipFuncSetAttribute(reinterpret_cast<const void*>(k_rdm_ab), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
        hipLaunchKernelGGL(k_rdm_ab, dim3((unsigned)na), dim3(256), lds, s, c, na, nb, A.str, sp->nw, A.s_off, A.s_pk,
                           B.str, B.s_off, B.s_pk, norb, rdm2);
    }
    SQD_HIP(ctx, hipGetLastError());
    return SQD_OK;
}
