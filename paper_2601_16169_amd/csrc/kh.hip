// Knowles-Handy form of the alpha-beta term on MFMA (Sec. IV cites Knowles and
// Handy for the three task types).
//
//   D[ia][jb'][bj] = sum_{beta singles jb' <- jb with pair bj} s_b C[ia][jb]
//   G[ia][jb'][e]  = sum_bj D[ia][jb'][bj] (bj|ai_e)          (a real GEMM)
//   sigma[ia'][jb'] += sum_{alpha singles e: ia' <- ia} s_e G[ia][jb'][e]
//
// One workgroup per (source alpha row ia, tile of 64 beta targets): the source
// row of C is staged in LDS, D is built densely in LDS one chunk of pair
// columns at a time, the matching rows of (pq|rs) -- one per alpha single out
// of ia -- are staged beside it, and the 64 x (singles of ia) product is
// accumulated on v_mfma_f64_16x16x4 (FP64) or v_mfma_f32_16x16x4 (FP32).  The
// result for each single e goes to row rev(e) of the intermediate Y (the
// entry of the target row that points back to ia), and the same coalesced
// gather as the direct path adds Y into sigma.
#include <algorithm>

#include "sqd_internal.h"

namespace {

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T> struct mfma;
// Accumulator layout (checked on gfx950): lane l, element q holds D[row][l % 16]
// with row = 4 * (l / 16) + q for the f32 form but row = l / 16 + 4 * q for the
// f64 form.  A[i][k] and B[k][j] come from lane i + 16 k and j + 16 k in both.
template <> struct mfma<double> {
    using acc_t = d4_t;
    static __device__ __forceinline__ int row(int lane, int q) { return (lane >> 4) + 4 * q; }
    static __device__ __forceinline__ acc_t zero() { return (acc_t){0.0, 0.0, 0.0, 0.0}; }
    static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct mfma<float> {
    using acc_t = f4_t;
    static __device__ __forceinline__ int row(int lane, int q) { return 4 * (lane >> 4) + q; }
    static __device__ __forceinline__ acc_t zero() { return (acc_t){0.f, 0.f, 0.f, 0.f}; }
    static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

constexpr int kTile = 64;   // beta targets per workgroup
constexpr int kNE = 32;     // alpha singles per pass (two 16-wide MFMA columns)
constexpr int kKC = 64;     // pair columns of D per chunk

template <typename T>
__global__ void __launch_bounds__(256)
k_ab_kh(const T* __restrict__ C, T* __restrict__ Y, int64_t na, int64_t nb, const int* __restrict__ a_off,
        const uint32_t* __restrict__ a_pk, const int* __restrict__ a_rev, const int* __restrict__ b_off,
        const uint32_t* __restrict__ b_pk, const T* __restrict__ V, int norb, const int* __restrict__ skip) {
    if (skip && *skip) return;
    using M = mfma<T>;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* crow = reinterpret_cast<T*>(lds_raw);          // nb + 1
    T* Dk = crow + ((nb + 1 + 3) & ~3);               // [kTile][kKC + 1]
    T* Vk = Dk + kTile * (kKC + 1);                   // [kKC][kNE + 1]
    __shared__ int epair[kNE];
    const int n2 = norb * norb;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t jb0 = (int64_t)blockIdx.x * kTile;
    for (int64_t ia = blockIdx.y; ia < na; ia += gridDim.y) {
        __syncthreads();
        const T* cr = C + ia * nb;
        for (int k = tid; k < nb; k += 256) crow[k] = cr[k];
        const int e0 = a_off[ia], e1 = a_off[ia + 1];
        for (int p0 = e0; p0 < e1; p0 += kNE) {
            const int ne = (e1 - p0) < kNE ? (e1 - p0) : kNE;
            if (tid < kNE) epair[tid] = (tid < ne) ? (int)((a_pk[p0 + tid] >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK) : -1;
            // wave w owns output tile rows w*16..w*16+15 (targets), both 16-wide columns
            typename M::acc_t acc0 = M::zero(), acc1 = M::zero();
            for (int kc = 0; kc < n2; kc += kKC) {
                __syncthreads();
                for (int k = tid; k < kTile * (kKC + 1); k += 256) Dk[k] = (T)0;
                __syncthreads();
                // scatter D for the chunk: 4 threads per target row
                {
                    const int t = tid >> 2, sub = tid & 3;
                    const int64_t jb = jb0 + t;
                    if (jb < nb) {
                        for (int e = b_off[jb] + sub; e < b_off[jb + 1]; e += 4) {
                            const uint32_t x = b_pk[e];
                            const int pb = (int)((x >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK);
                            if (pb < kc || pb >= kc + kKC) continue;
                            T v = crow[x & SQD_NBR_MASK];
                            if (x >> 31) v = -v;
                            Dk[t * (kKC + 1) + (pb - kc)] = v;
                        }
                    }
                }
                // rows of (pq|rs) for the singles of this pass (symmetric: V[pair][bj])
                for (int k = tid; k < kKC * kNE; k += 256) {
                    const int kk = k / kNE, n = k % kNE;
                    const int pr = epair[n];
                    const int bj = kc + kk;
                    Vk[kk * (kNE + 1) + n] = (pr >= 0 && bj < n2) ? V[(int64_t)pr * n2 + bj] : (T)0;
                }
                __syncthreads();
#pragma unroll 4
                for (int ks = 0; ks < kKC; ks += 4) {
                    const T a = Dk[(w * 16 + (lane & 15)) * (kKC + 1) + ks + (lane >> 4)];
                    const T b0 = Vk[(ks + (lane >> 4)) * (kNE + 1) + (lane & 15)];
                    const T b1 = Vk[(ks + (lane >> 4)) * (kNE + 1) + 16 + (lane & 15)];
                    acc0 = M::op(a, b0, acc0);
                    acc1 = M::op(a, b1, acc1);
                }
            }
            // Y[rev(e)][jb'] = s_e * G[jb'][e]
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int t = w * 16 + M::row(lane, q);
                const int64_t jb = jb0 + t;
                if (jb < nb) {
                    const int n0 = lane & 15, n1 = 16 + (lane & 15);
                    if (n0 < ne) {
                        const uint32_t x = a_pk[p0 + n0];
                        const T v = (x >> 31) ? -acc0[q] : acc0[q];
                        Y[(int64_t)a_rev[p0 + n0] * nb + jb] = v;
                    }
                    if (n1 < ne) {
                        const uint32_t x = a_pk[p0 + n1];
                        const T v = (x >> 31) ? -acc1[q] : acc1[q];
                        Y[(int64_t)a_rev[p0 + n1] * nb + jb] = v;
                    }
                }
            }
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_kh_gather(const T* __restrict__ Y, T* __restrict__ S, int64_t na, int64_t nb, const int* __restrict__ a_off,
            const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int64_t jb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (jb >= nb) return;
    for (int64_t ia = blockIdx.y; ia < na; ia += gridDim.y) {
        T acc = (T)0;
        for (int e = a_off[ia]; e < a_off[ia + 1]; ++e) acc += Y[(int64_t)e * nb + jb];
        S[ia * nb + jb] += acc;
    }
}

// rev[e]: position, in the row of e's neighbour, of the entry pointing back.
int ensure_rev(sqd_ctx* ctx, sqd_space* sp) {
    if (sp->ab_rev) return SQD_OK;
    const spin_tables& A = sp->sp[0];
    std::vector<int> off(A.n + 1);
    std::vector<uint64_t> ent(A.nnz_s > 0 ? A.nnz_s : 1);
    SQD_HIP(ctx, hipMemcpy(off.data(), A.s_off, sizeof(int) * (A.n + 1), hipMemcpyDeviceToHost));
    if (A.nnz_s > 0) SQD_HIP(ctx, hipMemcpy(ent.data(), A.s_ent, sizeof(uint64_t) * A.nnz_s, hipMemcpyDeviceToHost));
    std::vector<int> rev(A.nnz_s > 0 ? A.nnz_s : 1, -1);
    for (int64_t r = 0; r < A.n; ++r)
        for (int e = off[r]; e < off[r + 1]; ++e) {
            const int64_t t = (int64_t)(ent[e] & 0xFFFFFFFFull);
            // rows are sorted by target: binary search row t for r
            int lo = off[t], hi = off[t + 1] - 1;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int64_t v = (int64_t)(ent[mid] & 0xFFFFFFFFull);
                if (v == r) { rev[e] = mid; break; }
                if (v < r) lo = mid + 1; else hi = mid - 1;
            }
            if (rev[e] < 0) return sqd_fail(ctx, SQD_E_STATE, "single excitation table is not symmetric");
        }
    int rc = sqd_alloc(ctx, (void**)&sp->ab_rev, sizeof(int) * rev.size(), &sp->bytes);
    if (rc) return rc;
    SQD_HIP(ctx, hipMemcpy(sp->ab_rev, rev.data(), sizeof(int) * rev.size(), hipMemcpyHostToDevice));
    return SQD_OK;
}

template <typename T>
int launch_kh(sqd_ctx* ctx, sqd_space* sp, const T* C, T* S, T* Y, const T* V, const int* skip) {
    int rc = ensure_rev(ctx, sp);
    if (rc) return rc;
    const spin_tables& A = sp->sp[0];
    const spin_tables& B = sp->sp[1];
    const size_t lds = sizeof(T) * (((size_t)B.n + 1 + 3) / 4 * 4 + (size_t)kTile * (kKC + 1) + (size_t)kKC * (kNE + 1));
    if (lds > (size_t)ctx->max_lds) return sqd_fail(ctx, SQD_E_LIMIT, "KH tile does not fit in LDS");
    hipFuncSetAttribute(reinterpret_cast<const void*>(k_ab_kh<T>), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    const unsigned gy = (unsigned)std::min<int64_t>(A.n, 65535);
    {
        prof_scope ps(ctx, sizeof(T) == 8 ? "k_ab_kh<double>" : "k_ab_kh<float>");
        hipLaunchKernelGGL((k_ab_kh<T>), dim3(nblk(B.n, kTile), gy), dim3(256), lds, ctx->stream, C, Y, A.n, B.n,
                           A.s_off, A.s_pk, sp->ab_rev, B.s_off, B.s_pk, V, sp->norb, skip);
    }
    {
        prof_scope pg(ctx, sizeof(T) == 8 ? "k_kh_gather<double>" : "k_kh_gather<float>");
        hipLaunchKernelGGL((k_kh_gather<T>), dim3(nblk(B.n, 256), gy), dim3(256), 0, ctx->stream, Y, S, A.n, B.n,
                           A.s_off, skip);
    }
    SQD_HIP(ctx, hipGetLastError());
    return SQD_OK;
}

}  // namespace

size_t sqd_kh_bytes(const sqd_space* sp, size_t es) { return (size_t)sp->sp[0].nnz_s * (size_t)sp->sp[1].n * es + 256; }

int sqd_sigma_ab_kh(sqd_ctx* ctx, sqd_space* sp, const void* c, void* sigma, void* y, int fp32, const int* skip) {
    if (fp32)
        return launch_kh<float>(ctx, sp, (const float*)c, (float*)sigma, (float*)y, ctx->eri32, skip);
    return launch_kh<double>(ctx, sp, (const double*)c, (double*)sigma, (double*)y, ctx->eri, skip);
}
