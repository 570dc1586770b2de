// Knowles-Handy form of the alpha-beta term on MFMA (Sec. IV cites Knowles and
// Handy for the three task types).
//
//   D[ia][jb'][bj] = sum_{beta singles jb' <- jb with pair bj} s_b C[ia][jb]
//   G[ia][jb'][e]  = sum_bj D[ia][jb'][bj] (bj|ai_e)          (a real GEMM)
//   sigma[ia'][jb'] += sum_{alpha singles e: ia' <- ia} s_e G[ia][jb'][e]
//
// The K dimension of a tile of 64 beta targets is the union of the pair
// columns bj its singles use (on sampled spaces far fewer than norb^2), and a
// dense map gives, for every (target, column), the source string and sign of
// that single; both are built once per space.  One workgroup per (source
// alpha row ia, tile): D is filled from the map and the row of C one chunk of
// 64 columns at a time, the matching entries of (pq|rs) -- one column per
// alpha single out of ia -- are staged beside it, and the 64 x (singles of
// ia) product is accumulated on v_mfma_f64_16x16x4 (FP64) or
// v_mfma_f32_16x16x4 (FP32).  The result for each single e goes to row rev(e)
// of the intermediate Y (the entry of the target row that points back to ia),
// and a coalesced gather adds Y into sigma.
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

// Per-thread share of one chunk: kDE entries of D, kVE of the (pq|rs) tile.
constexpr int kDE = kTile * kKC / 256;
constexpr int kVE = kKC * kNE / 256;

// STAGE: the source row of C is copied to LDS once per alpha row (when it
// fits); otherwise D reads it from global memory (cached).
template <typename T, bool STAGE>
__global__ void __launch_bounds__(256)
k_ab_kh(const T* __restrict__ C, T* __restrict__ Y, int64_t na, int64_t nb, const int* __restrict__ a_off,
        const uint32_t* __restrict__ a_pk, const int* __restrict__ a_rev, const int* __restrict__ tile_off,
        const int* __restrict__ pairs, const int* __restrict__ map, const T* __restrict__ V, int norb,
        const int* __restrict__ skip) {
    if (skip && *skip) return;
    using M = mfma<T>;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* Dk = reinterpret_cast<T*>(lds_raw);           // [kTile][kKC + 1]
    T* Vk = Dk + kTile * (kKC + 1);                   // [kKC][kNE + 1]
    T* crow = Vk + kKC * (kNE + 1);                   // nb (STAGE)
    const int k0 = tile_off[blockIdx.x], KT = tile_off[blockIdx.x + 1] - k0;
    int* tp = reinterpret_cast<int*>(crow + (STAGE ? nb : 0));   // the tile's KT pair columns
    __shared__ int epair[kNE];
    const int n2 = norb * norb;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t jb0 = (int64_t)blockIdx.x * kTile;
    const int rows = (int)((nb - jb0) < kTile ? (nb - jb0) : kTile);
    const int* __restrict__ tmap = map + (int64_t)kTile * k0;   // [kTile][KT]
    for (int k = tid; k < KT; k += 256) tp[k] = pairs[k0 + k];
    for (int64_t ia = blockIdx.y; ia < na; ia += gridDim.y) {
        const T* __restrict__ cg = C + ia * nb;
        const int e0 = a_off[ia], e1 = a_off[ia + 1];
        if (e1 == e0) continue;   // uniform: no single leaves this row
        __syncthreads();   // the previous row's passes are done with crow, epair and the tiles
        if constexpr (STAGE)
            for (int64_t k = tid; k < nb; k += 256) crow[k] = cg[k];
        const T* cr = STAGE ? crow : cg;
        for (int p0 = e0; p0 < e1; p0 += kNE) {
            const int ne = (e1 - p0) < kNE ? (e1 - p0) : kNE;
            if (p0 != e0) __syncthreads();   // the previous pass has read epair and the tiles
            if (tid < kNE) epair[tid] = (tid < ne) ? (int)((a_pk[p0 + tid] >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK) : -1;
            __syncthreads();   // epair, tp and crow visible
            // registers of the next chunk: map entries and integrals, loaded
            // while the current chunk runs on the matrix cores
            int mv[kDE];
            T vv[kVE];
            auto load = [&](int kc) {
                const int kn = (KT - kc) < kKC ? (KT - kc) : kKC;
#pragma unroll
                for (int u = 0; u < kDE; ++u) {
                    const int k = tid + u * 256, t = k / kKC, kk = k % kKC;
                    mv[u] = (t < rows && kk < kn) ? tmap[(int64_t)t * KT + kc + kk] : 0;
                }
#pragma unroll
                for (int u = 0; u < kVE; ++u) {
                    const int k = tid + u * 256, kk = k / kNE, n = k % kNE;
                    const int pr = epair[n];
                    vv[u] = (pr >= 0 && kk < kn) ? V[(int64_t)pr * n2 + tp[kc + kk]] : (T)0;
                }
            };
            // one 16-wide MFMA column block when this pass has at most 16
            // singles (uniform over the workgroup)
            const bool two = ne > 16;
            typename M::acc_t acc0 = M::zero(), acc1 = M::zero();
            if (KT > 0) load(0);
            for (int kc = 0; kc < KT; kc += kKC) {
                const int kn = (KT - kc) < kKC ? (KT - kc) : kKC;
                __syncthreads();   // the previous chunk's products have read Dk and Vk
#pragma unroll
                for (int u = 0; u < kDE; ++u) {
                    const int k = tid + u * 256, t = k / kKC, kk = k % kKC;
                    const int m = mv[u];
                    T v = (T)0;
                    if (m != 0) {
                        v = cr[(m & 0x7FFFFFFF) - 1];
                        if (m < 0) v = -v;
                    }
                    Dk[t * (kKC + 1) + kk] = v;
                }
#pragma unroll
                for (int u = 0; u < kVE; ++u) {
                    const int k = tid + u * 256, kk = k / kNE, n = k % kNE;
                    Vk[kk * (kNE + 1) + n] = vv[u];
                }
                __syncthreads();
                if (kc + kKC < KT) load(kc + kKC);
                const int ks_end = (kn + 3) & ~3;
                if (two) {
                    for (int ks = 0; ks < ks_end; ks += 4) {
                        const T a = Dk[(w * 16 + (lane & 15)) * (kKC + 1) + ks + (lane >> 4)];
                        const T b0 = Vk[(ks + (lane >> 4)) * (kNE + 1) + (lane & 15)];
                        const T b1 = Vk[(ks + (lane >> 4)) * (kNE + 1) + 16 + (lane & 15)];
                        acc0 = M::op(a, b0, acc0);
                        acc1 = M::op(a, b1, acc1);
                    }
                } else {
                    for (int ks = 0; ks < ks_end; ks += 4) {
                        const T a = Dk[(w * 16 + (lane & 15)) * (kKC + 1) + ks + (lane >> 4)];
                        const T b0 = Vk[(ks + (lane >> 4)) * (kNE + 1) + (lane & 15)];
                        acc0 = M::op(a, b0, acc0);
                    }
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

// Per 64-target beta tile: the ascending union of the pair columns its
// singles use, and the (target, column) -> source map (0 = no single).
int ensure_kh_maps(sqd_ctx* ctx, sqd_space* sp) {
    if (sp->kh_map) return SQD_OK;
    const spin_tables& B = sp->sp[1];
    const int64_t nb = B.n;
    const int ntiles = (int)((nb + kTile - 1) / kTile);
    std::vector<int> off(nb + 1);
    std::vector<uint32_t> pk(B.nnz_s > 0 ? B.nnz_s : 1);
    SQD_HIP(ctx, hipMemcpy(off.data(), B.s_off, sizeof(int) * (nb + 1), hipMemcpyDeviceToHost));
    if (B.nnz_s > 0) SQD_HIP(ctx, hipMemcpy(pk.data(), B.s_pk, sizeof(uint32_t) * B.nnz_s, hipMemcpyDeviceToHost));
    std::vector<int> tile_off(ntiles + 1, 0), pairs, map;
    int64_t cols = 0;
    for (int t = 0; t < ntiles; ++t) {
        const int64_t j0 = (int64_t)t * kTile, j1 = std::min<int64_t>(nb, j0 + kTile);
        std::vector<int> u;
        for (int64_t j = j0; j < j1; ++j)
            for (int e = off[j]; e < off[j + 1]; ++e) u.push_back((int)((pk[e] >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK));
        std::sort(u.begin(), u.end());
        u.erase(std::unique(u.begin(), u.end()), u.end());
        const int K = (int)u.size();
        tile_off[t + 1] = tile_off[t] + K;
        pairs.insert(pairs.end(), u.begin(), u.end());
        const size_t base = map.size();
        map.resize(base + (size_t)kTile * K, 0);
        for (int64_t j = j0; j < j1; ++j)
            for (int e = off[j]; e < off[j + 1]; ++e) {
                const int pr = (int)((pk[e] >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK);
                const int kk = (int)(std::lower_bound(u.begin(), u.end(), pr) - u.begin());
                const uint32_t src = pk[e] & SQD_NBR_MASK;
                map[base + (size_t)(j - j0) * K + kk] = (int)((src + 1) | (pk[e] & 0x80000000u));
            }
        cols += (j1 - j0) * (int64_t)K;
    }
    int rc;
    if ((rc = sqd_alloc(ctx, (void**)&sp->kh_tile_off, sizeof(int) * tile_off.size(), &sp->bytes))) return rc;
    if ((rc = sqd_alloc(ctx, (void**)&sp->kh_pairs, sizeof(int) * std::max<size_t>(pairs.size(), 1), &sp->bytes))) return rc;
    if ((rc = sqd_alloc(ctx, (void**)&sp->kh_map, sizeof(int) * std::max<size_t>(map.size(), 1), &sp->bytes))) return rc;
    SQD_HIP(ctx, hipMemcpy(sp->kh_tile_off, tile_off.data(), sizeof(int) * tile_off.size(), hipMemcpyHostToDevice));
    if (!pairs.empty())
        SQD_HIP(ctx, hipMemcpy(sp->kh_pairs, pairs.data(), sizeof(int) * pairs.size(), hipMemcpyHostToDevice));
    if (!map.empty())
        SQD_HIP(ctx, hipMemcpy(sp->kh_map, map.data(), sizeof(int) * map.size(), hipMemcpyHostToDevice));
    sp->kh_ntiles = ntiles;
    sp->kh_cols = cols;
    int kmax = 0;
    for (int t = 0; t < ntiles; ++t) kmax = std::max(kmax, tile_off[t + 1] - tile_off[t]);
    sp->kh_kmax = kmax;
    return SQD_OK;
}

template <typename T>
int launch_kh(sqd_ctx* ctx, sqd_space* sp, const T* C, T* S, T* Y, const T* V, const int* skip) {
    int rc = ensure_rev(ctx, sp);
    if (rc) return rc;
    if ((rc = ensure_kh_maps(ctx, sp))) return rc;
    const spin_tables& A = sp->sp[0];
    const spin_tables& B = sp->sp[1];
    // tiles + the tile's pair list (+ the source row when two workgroups per
    // CU still fit)
    const size_t base = sizeof(T) * ((size_t)kTile * (kKC + 1) + (size_t)kKC * (kNE + 1)) +
                        sizeof(int) * (size_t)std::max(sp->kh_kmax, 1);
    const size_t staged = base + sizeof(T) * (size_t)B.n;
    const bool stage = staged <= (size_t)ctx->max_lds / 2;
    const size_t lds = stage ? staged : base;
    if (lds > (size_t)ctx->max_lds) return sqd_fail(ctx, SQD_E_LIMIT, "KH tile does not fit in LDS");
    const unsigned gy = (unsigned)std::min<int64_t>(A.n, 65535);
    {
        prof_scope ps(ctx, sizeof(T) == 8 ? "k_ab_kh<double>" : "k_ab_kh<float>");
        if (stage) {
            hipFuncSetAttribute(reinterpret_cast<const void*>(k_ab_kh<T, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            hipLaunchKernelGGL((k_ab_kh<T, true>), dim3(sp->kh_ntiles, gy), dim3(256), lds, ctx->stream, C, Y, A.n,
                               B.n, A.s_off, A.s_pk, sp->ab_rev, sp->kh_tile_off, sp->kh_pairs, sp->kh_map, V,
                               sp->norb, skip);
        } else {
            hipFuncSetAttribute(reinterpret_cast<const void*>(k_ab_kh<T, false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            hipLaunchKernelGGL((k_ab_kh<T, false>), dim3(sp->kh_ntiles, gy), dim3(256), lds, ctx->stream, C, Y,
                               A.n, B.n, A.s_off, A.s_pk, sp->ab_rev, sp->kh_tile_off, sp->kh_pairs, sp->kh_map, V,
                               sp->norb, skip);
        }
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
