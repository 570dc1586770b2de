// Device bodies of the Davidson kernels, shared by the single-space launches
// and the batched launches (davidson.hip).  Grid bodies take their block index
// and block count within their space (bid, nblk); finishing bodies run in one
// block per space.
#pragma once

#include <cmath>
#include <type_traits>

#include "sqd_internal.h"

namespace dav {


constexpr int MM = SQD_MMAX;
constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxBlocks = 512;   // measured on MI355X: 512 beats 1024 and 2048 by 1-3% (fewer partials to reduce)
constexpr int kPstride = MM + 4;   // partial sums per block
constexpr int kStallWindow = 12;   // FP32 phase: iterations without a 10% better residual
constexpr double kStallFrom = 1e-4;  // ... counted once the residual is below this times |theta|
constexpr double kFloor32 = 2e-6;    // 30 FP32 unit roundoffs: FP32 products carry no more digits

enum { DONE_RUNNING = 0, DONE_CONVERGED = 1, DONE_STALLED = 2, DONE_CAP = 3, DONE_SWITCH = 4 };

// Calls f(std::integral_constant<int, NR>) with NR the smallest multiple of 4
// (at most MT) not below cnt.  Loops over the rows of the basis then run to a
// compile-time bound with every load issued before the first use; rows past
// cnt are read from row cnt - 1 (always valid) and weighted by zero.  A
// per-row branch instead makes each load wait for the one before it.
template <int MT, int NR = 4, typename F>
__device__ __forceinline__ void with_rows(int cnt, F&& f) {
    if constexpr (NR >= MT) {
        f(std::integral_constant<int, MT>{});
    } else {
        if (cnt <= NR) f(std::integral_constant<int, NR>{});
        else with_rows<MT, NR + 4>(cnt, f);
    }
}

// Row k of a block of vectors of length n, clamped to the last valid row
// (row 0 when the block is empty).  The vector kernels read basis rows with
// non-temporal loads: the basis (m rows of n) is larger than the caches, and
// what the next kernels reuse (the correction, c, the product's tables) then
// stays cached (4.0e6-determinant workload, same box: FP64 solve 0.227 ->
// 0.216 s, mixed 0.157 -> 0.150 s).
template <typename VT>
__device__ __forceinline__ const VT* row_ptr(const VT* B, int k, int cnt, int64_t n) {
    const int r = k < cnt ? k : cnt - 1;
    return B + (int64_t)(r > 0 ? r : 0) * n;
}

struct dav_state {
    int m;
    int done;
    int iter;
    int collapse;         // number of vectors kept by a pending collapse (0 = none)
    int phase;            // 0: FP32 sigma (mixed mode), 1: FP64 sigma
    int phase_start;      // iteration at which the current phase began
    int kmin;
    int nhist;
    int reortho;          // second Gram-Schmidt projection needed
    int best_it;          // iteration of the smallest residual of the current phase
    int counter[8];       // last-block tickets, one per kernel kind
    double theta;
    double rnorm;
    double tt0;           // |t|^2 before orthogonalisation
    double tinv;          // 1 / |v| of the new basis vector
    double G[MM * MM];
    double y[MM];
    double y_prev[MM];    // previous Ritz vector in the current basis
    double h[MM];
    double qc[2][MM];     // collapse coefficients (columns kept)
    double Gc[4];         // projected matrix after a collapse
    double hc[2];         // Gram-Schmidt coefficients after a collapse
    double hist_r[SQD_HIST];
    double hist_e[SQD_HIST];
    int qn;               // Qp holds the eigenvectors of the leading qn x qn block of G (0: none)
    int xredo;            // locked-vector projection needs a second pass
    double best_r;        // smallest residual of the current phase
    double xc[SQD_MAXLOCK];   // X^T v of the vector being projected
    double xscale;        // scale applied after the projection (1 / |v - X xc|, or 1)
    double Qp[MM * MM];
};

struct dav_params {
    double tol;
    double switch_tol;
    int max_iter;
    int m_max;
    int mixed;
};

// 1/x and 1/sqrt(x) from the hardware estimates refined by two Newton steps
// (each squares the relative error, so two reach FP64 rounding); a dependent
// chain far shorter than IEEE division and square root.
__device__ __forceinline__ double rcp_refined(double x) {
    double r = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int k = 0; k < 2; ++k) r = fma(r, fma(-x, r, 1.0), r);
    return r;
}
__device__ __forceinline__ double rsqrt_refined(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
#pragma unroll
    for (int k = 0; k < 2; ++k) y = fma(y, fma(-h * y, y, 0.5), y);
    return y;
}

// Rotation (c, s) that zeroes the (p, q) entry of a symmetric 2 x 2 block
// [[app, apq], [apq, aqq]] (Rutishauser's smaller-angle choice, written with
// d = aqq - app and e = 2 apq: t = sign(d) e / (|d| + hypot(d, e)), c =
// 1/sqrt(1 + t^2), s = t c; sign(0) = +1).
__device__ __forceinline__ void jacobi_rotation(double app, double aqq, double apq, double& c, double& s) {
    const double d = aqq - app, e = 2.0 * apq;
    const double h2 = d * d + e * e;
    if (!(h2 > 1e-300)) {   // an entry this small is below any convergence test: leave it
        c = 1.0;
        s = 0.0;
        return;
    }
    const double hyp = h2 * rsqrt_refined(h2);
    const double t = (d >= 0.0 ? e : -e) * rcp_refined(fabs(d) + hyp);
    c = rsqrt_refined(1.0 + t * t);
    s = t * c;
}

// Block-wide sums of acc[0..NV) (wave shuffles, then one LDS slot per wave);
// written to partial row `row`.  All NV entries are reduced so that every
// register index is static.
template <int NV>
__device__ void block_to_partial(const double (&acc)[NV], double* __restrict__ partial, int64_t row, int64_t nrows) {
    __shared__ double wred[kWaves][NV];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double v = acc[j];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) wred[w][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int q = 0; q < kWaves; ++q) s += wred[q][threadIdx.x];
        partial[(size_t)threadIdx.x * nrows + row] = s;   // value-major: the reduction reads coalesced
    }
}

// One block of kThreads: out[j] = sum over rows b < nrows of partial[b][j],
// j < NV (thread t takes rows t, t + kThreads, ...; then a fixed tree), so the
// result is deterministic.  The partials come from an earlier launch.
template <int NV>
__device__ void reduce_rows(const double* __restrict__ partial, int nrows, double* out) {
    double acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.0;
    for (int b = threadIdx.x; b < nrows; b += kThreads) {
#pragma unroll
        for (int j = 0; j < NV; ++j) acc[j] += partial[(size_t)j * nrows + b];
    }
    __shared__ double wred[kWaves][NV];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double v = acc[j];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) wred[w][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int q = 0; q < kWaves; ++q) s += wred[q][threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// ---------------------------------------------------------------- kernels

// per-block (min value, first index) of the diagonal
__device__ __forceinline__ void d_argmin(const double* __restrict__ d, int64_t n,
                                                     double* __restrict__ partial, int64_t bid, int64_t nblk) {
    __shared__ double sv[kThreads];
    __shared__ long long si[kThreads];
    double best = INFINITY;
    long long bi = -1;
    for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads) {
        const double v = d[i];
        if (v < best) { best = v; bi = i; }   // ascending i: first minimum kept
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double v = sv[threadIdx.x + s];
            const long long j = si[threadIdx.x + s];
            if (j >= 0 && (si[threadIdx.x] < 0 || v < sv[threadIdx.x] || (v == sv[threadIdx.x] && j < si[threadIdx.x]))) {
                sv[threadIdx.x] = v;
                si[threadIdx.x] = j;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[(size_t)bid * kPstride + 0] = sv[0];
        partial[(size_t)bid * kPstride + 1] = (double)si[0];
    }
}

// largest |x| (MODE 1, lowest index on ties) or smallest value (MODE 0) over
// the per-block partials -> st->kmin; MODE 1 also sums column 2 -> st->tinv = 1/sqrt.
template <int MODE>
__device__ __forceinline__ void f_pick_fin(const double* __restrict__ partial, int nrows, dav_state* st) {
    __shared__ double sv[kThreads], sn[kThreads];
    __shared__ long long si[kThreads];
    double b = MODE ? -1.0 : INFINITY, ss = 0.0;
    long long k = -1;
    for (int q = threadIdx.x; q < nrows; q += kThreads) {
        const double v = partial[(size_t)q * kPstride];
        const long long j = (long long)partial[(size_t)q * kPstride + 1];
        if (MODE) ss += partial[(size_t)q * kPstride + 2];
        const bool better = MODE ? (v > b) : (v < b);
        if (j >= 0 && (k < 0 || better || (v == b && j < k))) { b = v; k = j; }
    }
    sv[threadIdx.x] = b; si[threadIdx.x] = k; sn[threadIdx.x] = ss;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double v = sv[threadIdx.x + s];
            const long long j = si[threadIdx.x + s];
            const bool better = MODE ? (v > sv[threadIdx.x]) : (v < sv[threadIdx.x]);
            if (j >= 0 && (si[threadIdx.x] < 0 || better || (v == sv[threadIdx.x] && j < si[threadIdx.x]))) {
                sv[threadIdx.x] = v;
                si[threadIdx.x] = j;
            }
            sn[threadIdx.x] += sn[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->kmin = (int)(si[0] < 0 ? 0 : si[0]);
        if (MODE) st->tinv = 1.0 / sqrt(sn[0]);
    }
}

// V[0] = start vector (explicit guess, or e_kmin + noise), and |V[0]|^2 partials.
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): a counter-based 64-bit mix.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// Entry i of the library's start noise for counter stream `stream`: uniform of
// zero mean and variance 1e-6 / n, so the noise has norm about 1e-3.  It lets a
// start on e_kmin, which has the spin-flip symmetry of an S_a = S_b space, reach
// a lowest state of the other symmetry.
__device__ __forceinline__ double start_noise(uint64_t stream, int64_t i, int64_t n) {
    const uint64_t r = splitmix64((stream << 40) ^ (uint64_t)i);
    const double uni = (double)(r >> 11) * (1.0 / 9007199254740992.0);   // [0, 1)
    return 1e-3 * sqrt(3.0 / (double)n) * (2.0 * uni - 1.0);
}

// V0 = guess, or e_kmin + noise (the caller's, else start_noise stream 0);
// |V0|^2 partials.
template <typename VT = double>
__device__ __forceinline__ void d_start(const double* __restrict__ guess, const double* __restrict__ noise,
                                                    int64_t n, const dav_state* st, VT* __restrict__ V0,
                                                    double* __restrict__ partial, int64_t bid, int64_t nblk) {
    double acc[1] = {0.0};
    const int64_t kmin = st->kmin;
    for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads) {
        double v;
        if (guess) v = guess[i];
        else v = (i == kmin ? 1.0 : 0.0) + (noise ? noise[i] : start_noise(0, i, n));
        V0[i] = (VT)v;
        acc[0] += v * v;
    }
    block_to_partial<1>(acc, partial, bid, nblk);
}

__device__ __forceinline__ void f_norm_fin(const double* __restrict__ partial, int nrows, dav_state* st) {
    __shared__ double out[1];
    reduce_rows<1>(partial, nrows, out);
    if (threadIdx.x == 0) st->tinv = 1.0 / sqrt(out[0]);
}

// V0 *= tinv; copies into the product input (and its FP32 copy)
template <typename VT = double>
__device__ __forceinline__ void d_scale_copy(VT* __restrict__ V0, int64_t n, const dav_state* st,
                                                         double* __restrict__ cin, float* __restrict__ c32, int64_t bid, int64_t nblk) {
    const double sc = st->tinv;
    for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads) {
        const double v = (double)V0[i] * sc;
        V0[i] = (VT)v;
        cin[i] = v;
        if (c32) c32[i] = (float)v;
    }
}

// Residual, preconditioned correction and the first Gram-Schmidt projection:
// partial columns 0..MT-1: V^T t; MT: |r|^2; MT+1: |t|^2.
template <int MT, typename VT = double>
__device__ __forceinline__ void d_residual(const VT* __restrict__ V, const VT* __restrict__ AV, const double* __restrict__ diag, int64_t n,
           const dav_state* st, double* __restrict__ T, double* __restrict__ partial, int64_t bid, int64_t nblk) {
    if (st->done) return;
    const int m = st->m;
    const double theta = st->theta;
    double acc[MT + 2];
#pragma unroll
    for (int k = 0; k < MT + 2; ++k) acc[k] = 0.0;
    with_rows<MT>(m, [&](auto nr_) {
        constexpr int NR = decltype(nr_)::value;
        double y[NR];
        const VT* vr[NR];
        const VT* ar[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            y[k] = (k < m) ? st->y[k] : 0.0;
            vr[k] = row_ptr(V, k, m, n);
            ar[k] = row_ptr(AV, k, m, n);
        }
        for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads) {
            double v[NR], a[NR];
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                v[k] = __builtin_nontemporal_load(vr[k] + i);
                a[k] = __builtin_nontemporal_load(ar[k] + i);
            }
            const double d = diag[i];
            double x = 0.0, ax = 0.0;
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                x += y[k] * v[k];
                ax += y[k] * a[k];
            }
            const double r = ax - theta * x;
            double den = theta - d;
            if (fabs(den) < 1e-8) den = (den < 0.0) ? -1e-8 : 1e-8;
            const double tv = r / den;
            T[i] = tv;
            acc[MT] += r * r;
            acc[MT + 1] += tv * tv;
#pragma unroll
            for (int k = 0; k < NR; ++k) acc[k] += (k < m) ? v[k] * tv : 0.0;
        }
    });
    block_to_partial<MT + 2>(acc, partial, bid, nblk);
}

// Convergence / cap / phase-switch decisions and the collapse plan.
template <int MT>
__device__ __forceinline__ void f_res_fin(const double* __restrict__ partial, int nrows, dav_state* st, dav_params prm) {
    if (st->done) return;
    __shared__ double out[MT + 2];
    reduce_rows<MT + 2>(partial, nrows, out);
    if (threadIdx.x != 0) return;
    const int m = st->m;
    const double theta = st->theta;
    const double rn = sqrt(out[MT]);
    st->rnorm = rn;
    st->tt0 = out[MT + 1];
    for (int j = 0; j < m; ++j) st->h[j] = out[j];
    const int it = st->iter;
    if (it < SQD_HIST) {
        st->hist_r[it] = rn;
        st->hist_e[it] = theta;
        st->nhist = it + 1;
    }
    st->iter = it + 1;
    int done = DONE_RUNNING;
    // smallest residual of this phase (a new best must improve by 10%)
    if (it == st->phase_start || rn < 0.9 * st->best_r) {
        st->best_r = rn;
        st->best_it = it;
    }
    if (st->phase == 0) {
        // FP32 phase: hand over to FP64 refinement below switch_tol, on
        // reaching tol, below the FP32 floor (kFloor32 |theta|), or once the
        // residual has not improved for kStallWindow iterations after falling
        // below kStallFrom |theta| (a Davidson residual is not monotone: early
        // plateaus and bumps are not the FP32 floor)
        const double at = fabs(theta);
        const bool stall = st->best_r < kStallFrom * at && it - st->best_it >= kStallWindow;
        if (rn < prm.switch_tol || rn <= prm.tol || rn < kFloor32 * at || stall) done = DONE_SWITCH;
    } else if (rn <= prm.tol) {
        done = DONE_CONVERGED;
    }
    if (done == DONE_RUNNING && st->iter >= prm.max_iter) done = DONE_CAP;
    st->done = done;
    st->collapse = 0;
    if (done == DONE_RUNNING && m >= prm.m_max) {
        // keep the Ritz vector and the previous Ritz vector, orthonormalised in
        // the small space: q1 = y, q2 ~ y_prev - (y . y_prev) y
        double* q1 = st->qc[0];
        double* q2 = st->qc[1];
        double dp = 0.0;
        for (int k = 0; k < m; ++k) dp += st->y[k] * st->y_prev[k];
        double nq = 0.0;
        for (int k = 0; k < MM; ++k) {
            q1[k] = (k < m) ? st->y[k] : 0.0;
            q2[k] = (k < m) ? st->y_prev[k] - dp * st->y[k] : 0.0;
            nq += q2[k] * q2[k];
        }
        int keep = 1;
        if (nq > 1e-20 && prm.m_max >= 3) {
            double d2 = 0.0;
            for (int k = 0; k < m; ++k) d2 += q1[k] * q2[k];
            nq = 0.0;
            for (int k = 0; k < m; ++k) {
                q2[k] -= d2 * q1[k];
                nq += q2[k] * q2[k];
            }
            const double inv = 1.0 / sqrt(nq);
            for (int k = 0; k < m; ++k) q2[k] *= inv;
            keep = 2;
        }
        for (int a = 0; a < keep; ++a) {
            double ha = 0.0;
            for (int k = 0; k < m; ++k) ha += st->qc[a][k] * out[k];
            st->hc[a] = ha;
            for (int b = 0; b < keep; ++b) {
                double g = 0.0;
                for (int k = 0; k < m; ++k) {
                    double gk = 0.0;
                    for (int l = 0; l < m; ++l) gk += st->G[k * MM + l] * st->qc[b][l];
                    g += st->qc[a][k] * gk;
                }
                st->Gc[a * 2 + b] = g;
            }
        }
        if (keep == 2) {
            const double g = 0.5 * (st->Gc[1] + st->Gc[2]);
            st->Gc[1] = g;
            st->Gc[2] = g;
        }
        st->collapse = keep;
    }
}

// In-place collapse: V[a] = V qc[a], AV[a] = AV qc[a] for the kept columns a.
// force = 1 (switch to FP64 refinement): keep x = V y only, AV not kept.
template <int MT, typename VT = double>
__device__ __forceinline__ void d_collapse(VT* __restrict__ V, VT* __restrict__ AV, int64_t n, const dav_state* st, int force,
           double* __restrict__ cin, int64_t bid, int64_t nblk) {
    int keep;
    if (force) {
        keep = 1;
    } else {
        if (st->done || !st->collapse) return;
        keep = st->collapse;
    }
    const int m = st->m;
    // an FP32 basis leaves the FP64 refinement's first vector to the caller
    // (it overlaps the FP32 rows still being read): only cin is written
    const bool wv = !(force && sizeof(VT) < sizeof(double));
    const double* q1p = force ? st->y : st->qc[0];
    const double* q2p = st->qc[1];
    with_rows<MT>(m, [&](auto nr_) {
        constexpr int NR = decltype(nr_)::value;
        double q1[NR], q2[NR];
        const VT* vr[NR];
        const VT* ar[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            q1[k] = (k < m) ? q1p[k] : 0.0;
            q2[k] = (k < m) ? q2p[k] : 0.0;
            vr[k] = row_ptr(V, k, m, n);
            ar[k] = row_ptr(AV, k, m, n);
        }
        // every row is read before row 0 or 1 is written: the loads of one
        // element precede its stores, and elements are independent
        for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads) {
            double v[NR];
#pragma unroll
            for (int k = 0; k < NR; ++k) v[k] = __builtin_nontemporal_load(vr[k] + i);
            double x1 = 0.0, x2 = 0.0;
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                x1 += q1[k] * v[k];
                x2 += q2[k] * v[k];
            }
            if (!force) {
                double a[NR];
#pragma unroll
                for (int k = 0; k < NR; ++k) a[k] = __builtin_nontemporal_load(ar[k] + i);
                double a1 = 0.0, a2 = 0.0;
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    a1 += q1[k] * a[k];
                    a2 += q2[k] * a[k];
                }
                AV[i] = (VT)a1;
                if (keep == 2) AV[n + i] = (VT)a2;
            }
            if (wv) {
                V[i] = (VT)x1;
                if (keep == 2) V[n + i] = (VT)x2;
            }
            if (cin) cin[i] = x1;
        }
    });
}

// State after a collapse (force: m = 0, the next dots pass rebuilds G[0][0]).
__device__ __forceinline__ void f_collapse_fin(dav_state* st, int force) {
    if (threadIdx.x != 0) return;
    if (force) {
        st->m = 0;
        st->collapse = 0;
        st->qn = 0;
        return;
    }
    if (st->done || !st->collapse) return;
    const int keep = st->collapse;
    st->m = keep;
    st->qn = 0;
    for (int k = 0; k < MM * MM; ++k) st->G[k] = 0.0;
    st->G[0] = st->Gc[0];
    if (keep == 2) {
        st->G[1] = st->Gc[1];
        st->G[MM] = st->Gc[2];
        st->G[MM + 1] = st->Gc[3];
    }
    for (int k = 0; k < MM; ++k) {
        st->h[k] = (k < keep) ? st->hc[k] : 0.0;
        st->y[k] = (k == 0) ? 1.0 : 0.0;
        st->y_prev[k] = st->y[k];
    }
    st->collapse = 0;
}

// t1 = t - V h; partial columns 0..MT-1: V^T t1; MT: |t1|^2.
template <int MT, typename VT = double>
__device__ __forceinline__ void d_orth1(const VT* __restrict__ V, int64_t n, const dav_state* st, double* __restrict__ T,
        double* __restrict__ partial, int64_t bid, int64_t nblk) {
    if (st->done) return;
    const int m = st->m;
    double acc[MT + 1];
#pragma unroll
    for (int k = 0; k < MT + 1; ++k) acc[k] = 0.0;
    with_rows<MT>(m, [&](auto nr_) {
        constexpr int NR = decltype(nr_)::value;
        double h[NR];
        const VT* vr[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            h[k] = (k < m) ? st->h[k] : 0.0;
            vr[k] = row_ptr(V, k, m, n);
        }
        for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads) {
            double v[NR];
#pragma unroll
            for (int k = 0; k < NR; ++k) v[k] = __builtin_nontemporal_load(vr[k] + i);
            double t = T[i];
#pragma unroll
            for (int k = 0; k < NR; ++k) t -= h[k] * v[k];
            T[i] = t;
            acc[MT] += t * t;
#pragma unroll
            for (int k = 0; k < NR; ++k) acc[k] += (k < m) ? v[k] * t : 0.0;
        }
    });
    block_to_partial<MT + 1>(acc, partial, bid, nblk);
}

template <int MT, typename VT = double>
__device__ __forceinline__ void f_orth1_fin(const double* __restrict__ partial, int nrows, dav_state* st) {
    if (st->done) return;
    __shared__ double out[MT + 1];
    reduce_rows<MT + 1>(partial, nrows, out);
    if (threadIdx.x != 0) return;
    const int m = st->m;
    double hh = 0.0;
    for (int j = 0; j < m; ++j) {
        st->h[j] = out[j];
        hh += out[j] * out[j];
    }
    const double t1 = out[MT];
    const double nrm2 = t1 - hh;
    // a second projection only when the first left an overlap above what
    // the basis rows hold: an FP32 basis is orthonormal to its rounding
    // (6e-8), so a second pass there cannot improve the stored vector unless
    // the first left more than 1e-6 of it
    constexpr double kVisible = sizeof(VT) < sizeof(double) ? 1e-12 : 1e-26;
    st->reortho = (hh > kVisible * t1) ? 1 : 0;
    if (!(nrm2 > 1e-28 * st->tt0) || !(nrm2 > 0.0)) {
        st->done = (st->rnorm <= 0.0) ? DONE_CONVERGED : DONE_STALLED;
    } else {
        st->tinv = 1.0 / sqrt(st->reortho ? nrm2 : t1);
    }
}

template <int MT, typename VT = double>
__device__ __forceinline__ void d_orth2(VT* __restrict__ V, int64_t n, const dav_state* st, const double* __restrict__ T, double* __restrict__ cin,
        float* __restrict__ c32, int64_t bid, int64_t nblk) {
    if (st->done) return;
    const int m = st->m;
    const double sc = st->tinv;
    const bool re = st->reortho != 0;
    VT* vm = V + (int64_t)m * n;
    const bool lo = (st->phase == 0) && c32;
    if (!re) {
        for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads) {
            const double t = T[i] * sc;
            vm[i] = (VT)t;
            cin[i] = t;
            if (lo) c32[i] = (float)t;
        }
        return;
    }
    with_rows<MT>(m, [&](auto nr_) {
        constexpr int NR = decltype(nr_)::value;
        double h[NR];
        const VT* vr[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            h[k] = (k < m) ? st->h[k] : 0.0;
            vr[k] = row_ptr(V, k, m, n);
        }
        for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads) {
            double v[NR];
#pragma unroll
            for (int k = 0; k < NR; ++k) v[k] = __builtin_nontemporal_load(vr[k] + i);
            double t = T[i];
#pragma unroll
            for (int k = 0; k < NR; ++k) t -= h[k] * v[k];
            t *= sc;
            vm[i] = (VT)t;
            cin[i] = t;
            if (lo) c32[i] = (float)t;
        }
    });
}

// AV[m] = S; partial columns 0..m: V[k] . S.
template <int MT, typename VT = double>
__device__ __forceinline__ void d_dots(const VT* __restrict__ V, VT* __restrict__ AV, const double* __restrict__ S, int64_t n,
       const dav_state* st, double* __restrict__ partial, int64_t bid, int64_t nblk) {
    if (st->done) return;
    const int m = st->m;
    double acc[MT + 1];
#pragma unroll
    for (int k = 0; k <= MT; ++k) acc[k] = 0.0;
    VT* avm = AV + (int64_t)m * n;
    const int cnt = m + 1;   // rows 0..m, the new vector included (cnt <= MT)
    with_rows<MT>(cnt, [&](auto nr_) {
        constexpr int NR = decltype(nr_)::value;
        const VT* vr[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) vr[k] = row_ptr(V, k, cnt, n);
        for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads) {
            double v[NR];
#pragma unroll
            for (int k = 0; k < NR; ++k) v[k] = __builtin_nontemporal_load(vr[k] + i);
            const double s = S[i];
            avm[i] = (VT)s;
#pragma unroll
            for (int k = 0; k < NR; ++k) acc[k] += (k < cnt) ? v[k] * s : 0.0;
        }
    });
    block_to_partial<MT + 1>(acc, partial, bid, nblk);
}

// G[:, m] from the partials, m += 1, then the lowest eigenpair of G by
// parallel cyclic Jacobi (round-robin pairs): theta, y (y_prev keeps the old y).
template <int MT>
__device__ __forceinline__ void f_dots_fin(const double* __restrict__ partial, int nrows, dav_state* st) {
    if (st->done) return;
    __shared__ double out[MT + 1];
    reduce_rows<MT + 1>(partial, nrows, out);
    // row stride LS = MM + 1: rows of A, Q and B start in different LDS banks,
    // so the column accesses of the rotations do not all hit one bank
    constexpr int LS = MM + 1;
    __shared__ double A[MM * LS];
    __shared__ double Q[MM * LS];
    __shared__ double B[MM * LS];
    __shared__ double rc[MM / 2], rs[MM / 2];
    __shared__ int rp[MM / 2], rq[MM / 2];
    __shared__ double red[2 * kWaves];
    const int t = threadIdx.x;
    const int m0 = st->m;
    const int m = m0 + 1;
    for (int j = t; j <= m0; j += kThreads) {
        st->G[j * MM + m0] = out[j];
        st->G[m0 * MM + j] = out[j];
    }
    for (int k = t; k < MM; k += kThreads) st->y_prev[k] = st->y[k];
    // Warm start: when Qp diagonalises the leading m0 x m0 block, rotate G by
    // diag(Qp, 1) first; the result is diagonal but for its last row and
    // column, and the sweeps below converge in two or three passes.
    const bool warm = (st->qn == m0) && m0 > 0;
    __syncthreads();
    for (int k = t; k < MM * MM; k += kThreads) {
        const int i = k / MM, j = k % MM;
        double q = (i == j) ? 1.0 : 0.0;
        if (warm && i < m0 && j < m0) q = st->Qp[k];
        Q[i * LS + j] = q;
        A[i * LS + j] = st->G[k];
    }
    if (t == 0) st->m = m;
    __syncthreads();
    if (warm) {
        for (int k = t; k < MM * MM; k += kThreads) {   // B = G Q
            const int i = k / MM, j = k % MM;
            double v = 0.0;
            if (i < m && j < m)
                for (int l = 0; l < m; ++l) v += A[i * LS + l] * Q[l * LS + j];
            B[i * LS + j] = v;
        }
        __syncthreads();
        for (int k = t; k < MM * MM; k += kThreads) {   // A = Q^T B
            const int i = k / MM, j = k % MM;
            double v = 0.0;
            if (i < m && j < m)
                for (int l = 0; l < m; ++l) v += Q[l * LS + i] * B[l * LS + j];
            A[i * LS + j] = v;
        }
        __syncthreads();
        for (int k = t; k < MM * MM; k += kThreads) {   // exact symmetry
            const int i = k / MM, j = k % MM;
            if (i < j && j < m) {
                const double v = 0.5 * (A[i * LS + j] + A[j * LS + i]);
                A[i * LS + j] = v;
                A[j * LS + i] = v;
            }
        }
        __syncthreads();
    }
    if (m > 1) {
        const int n2 = (m + 1) & ~1;
        const int npair = n2 / 2;
        const int lane = t & 63, w = t >> 6;
        for (int sweep = 0; sweep < 50; ++sweep) {
            double off = 0.0, tot = 0.0;
            for (int k = t; k < MM * MM; k += kThreads) {
                const int i = k / MM, j = k % MM;
                if (i < m && j < m) {
                    const double v = A[i * LS + j];
                    tot += v * v;
                    if (i != j) off += v * v;
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                off += __shfl_xor(off, o);
                tot += __shfl_xor(tot, o);
            }
            if (lane == 0) { red[w] = off; red[kWaves + w] = tot; }
            __syncthreads();
            off = 0.0; tot = 0.0;
            for (int q = 0; q < kWaves; ++q) { off += red[q]; tot += red[kWaves + q]; }
            __syncthreads();
            if (off <= 1e-28 * tot || off == 0.0) break;
            for (int step = 0; step < n2 - 1; ++step) {
                // round-robin pairing: index 0 fixed, the others rotate
                if (t < npair) {
                    const int pa = t, pb = n2 - 1 - t;
                    int ia = pa - 1 + step, ib = pb - 1 + step;
                    if (ia >= n2 - 1) ia -= n2 - 1;
                    if (ib >= n2 - 1) ib -= n2 - 1;
                    int p = pa == 0 ? 0 : ia + 1;
                    int q = pb == 0 ? 0 : ib + 1;
                    if (p > q) { const int x = p; p = q; q = x; }
                    double c = 1.0, s = 0.0;
                    if (q < m) {
                        const double apq = A[p * LS + q];
                        if (apq != 0.0) jacobi_rotation(A[p * LS + p], A[q * LS + q], apq, c, s);
                    }
                    rc[t] = c; rs[t] = s; rp[t] = p; rq[t] = q;
                }
                __syncthreads();
                // A <- J^T A J one 2 x 2 block per thread: the pairs are
                // disjoint, so block (P1, P2) depends only on itself
                for (int k = t; k < (MM / 2) * (MM / 2); k += kThreads) {
                    const int b1 = k / (MM / 2), b2 = k % (MM / 2);
                    if (b1 >= npair || b2 >= npair) continue;
                    const int p1 = rp[b1], q1 = rq[b1], p2 = rp[b2], q2 = rq[b2];
                    const bool v1 = q1 < m, v2 = q2 < m;
                    const double c1 = rc[b1], s1 = rs[b1], c2 = rc[b2], s2 = rs[b2];
                    if (s1 == 0.0 && s2 == 0.0) continue;
                    const double app = A[p1 * LS + p2];
                    const double apq = v2 ? A[p1 * LS + q2] : 0.0;
                    const double aqp = v1 ? A[q1 * LS + p2] : 0.0;
                    const double aqq = (v1 && v2) ? A[q1 * LS + q2] : 0.0;
                    const double rpp = c1 * app - s1 * aqp, rpq = c1 * apq - s1 * aqq;
                    const double rqp = s1 * app + c1 * aqp, rqq = s1 * apq + c1 * aqq;
                    A[p1 * LS + p2] = c2 * rpp - s2 * rpq;
                    if (v2) A[p1 * LS + q2] = s2 * rpp + c2 * rpq;
                    if (v1) A[q1 * LS + p2] = c2 * rqp - s2 * rqq;
                    if (v1 && v2) A[q1 * LS + q2] = s2 * rqp + c2 * rqq;
                }
                // Q <- Q J
                for (int k = t; k < (MM / 2) * MM; k += kThreads) {
                    const int pr = k / MM, i = k % MM;
                    if (pr >= npair || i >= m) continue;
                    const int p = rp[pr], q = rq[pr];
                    if (q >= m || rs[pr] == 0.0) continue;
                    const double c = rc[pr], s = rs[pr];
                    const double qp = Q[i * LS + p], qq = Q[i * LS + q];
                    Q[i * LS + p] = c * qp - s * qq;
                    Q[i * LS + q] = s * qp + c * qq;
                }
                __syncthreads();
            }
        }
    }
    for (int k = t; k < MM * MM; k += kThreads) st->Qp[k] = Q[(k / MM) * LS + k % MM];
    if (t == 0) st->qn = m;
    if (t == 0) {
        int kmin = 0;
        for (int k = 1; k < m; ++k)
            if (A[k * LS + k] < A[kmin * LS + kmin]) kmin = k;
        st->theta = A[kmin * LS + kmin];
        double nrm = 0.0;
        for (int k = 0; k < m; ++k) nrm += Q[k * LS + kmin] * Q[k * LS + kmin];
        nrm = 1.0 / sqrt(nrm);
        // sign: keep continuity with the previous Ritz vector
        double dp = 0.0;
        for (int k = 0; k < m; ++k) dp += Q[k * LS + kmin] * st->y_prev[k];
        if (dp < 0.0) nrm = -nrm;
        for (int k = 0; k < MM; ++k) st->y[k] = (k < m) ? Q[k * LS + kmin] * nrm : 0.0;
    }
}

// Final vector x = V y; per-block largest |x| (lowest index on ties) and |x|^2.
template <int MT, typename VT = double>
__device__ __forceinline__ void d_final(const VT* __restrict__ V, int64_t n, const dav_state* st, double* __restrict__ out,
        double* __restrict__ partial, int64_t bid, int64_t nblk) {
    const int m = st->m;
    __shared__ double sv[kThreads], sn[kThreads];
    __shared__ long long si[kThreads];
    double best = -1.0, nrm = 0.0;
    long long bi = -1;
    with_rows<MT>(m, [&](auto nr_) {
        constexpr int NR = decltype(nr_)::value;
        double y[NR];
        const VT* vr[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            y[k] = (k < m) ? st->y[k] : 0.0;
            vr[k] = row_ptr(V, k, m, n);
        }
        for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads) {
            double x = 0.0;
#pragma unroll
            for (int k = 0; k < NR; ++k) x += y[k] * __builtin_nontemporal_load(vr[k] + i);
            out[i] = x;
            nrm += x * x;
            const double a = fabs(x);
            if (a > best) { best = a; bi = i; }
        }
    });
    sv[threadIdx.x] = best; si[threadIdx.x] = bi; sn[threadIdx.x] = nrm;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double v = sv[threadIdx.x + s];
            const long long j = si[threadIdx.x + s];
            if (j >= 0 && (si[threadIdx.x] < 0 || v > sv[threadIdx.x] || (v == sv[threadIdx.x] && j < si[threadIdx.x]))) {
                sv[threadIdx.x] = v;
                si[threadIdx.x] = j;
            }
            sn[threadIdx.x] += sn[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[(size_t)bid * kPstride + 0] = sv[0];
        partial[(size_t)bid * kPstride + 1] = (double)si[0];
        partial[(size_t)bid * kPstride + 2] = sn[0];
    }
}

// sign of the largest entry, read before any rescaling
__device__ __forceinline__ void f_final_sign(const double* __restrict__ out, dav_state* st) {
    if (threadIdx.x == 0) {
        const int64_t k = st->kmin;
        if (out[k] < 0.0) st->tinv = -st->tinv;
    }
}

__device__ __forceinline__ void d_final_scale(double* __restrict__ out, int64_t n, const dav_state* st, int64_t bid, int64_t nblk) {
    const double sc = st->tinv;
    for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads)
        out[i] *= sc;
}

// ---------------------------------------------------------------- locked roots
// Projection of a vector v against nx locked, orthonormal vectors X (the
// roots already found), so that the solve for the next root stays in their
// orthogonal complement.  One classical Gram-Schmidt pass, normalised with
// the norm it predicts; a second pass only when the first removed more than
// half of the squared norm (then the predicted norm is not trusted).

// partial column 0: |v|^2; columns 1..SQD_MAXLOCK: X_k . v (zero past nx)
// v is V itself (vrow = 0) or row st->m of V (the vector just appended).
__device__ __forceinline__ void d_xdots(const double* __restrict__ X, int nx, const double* __restrict__ V,
                                        int vrow, int64_t n, const dav_state* st, int round,
                                        double* __restrict__ partial, int64_t bid, int64_t nblk) {
    if (st->done || (round == 1 && !st->xredo)) return;
    const double* v = vrow ? V + (int64_t)st->m * n : V;
    double acc[1 + SQD_MAXLOCK];
#pragma unroll
    for (int k = 0; k <= SQD_MAXLOCK; ++k) acc[k] = 0.0;
    const double* xr[SQD_MAXLOCK];
#pragma unroll
    for (int k = 0; k < SQD_MAXLOCK; ++k) xr[k] = row_ptr(X, k, nx, n);
    for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads) {
        const double vi = v[i];
        double x[SQD_MAXLOCK];
#pragma unroll
        for (int k = 0; k < SQD_MAXLOCK; ++k) x[k] = xr[k][i];
        acc[0] += vi * vi;
#pragma unroll
        for (int k = 0; k < SQD_MAXLOCK; ++k) acc[1 + k] += (k < nx) ? x[k] * vi : 0.0;
    }
    block_to_partial<1 + SQD_MAXLOCK>(acc, partial, bid, nblk);
}

__device__ __forceinline__ void f_xfin(const double* __restrict__ partial, int nrows, int nx, dav_state* st, int round) {
    if (st->done || (round == 1 && !st->xredo)) return;
    __shared__ double out[1 + SQD_MAXLOCK];
    reduce_rows<1 + SQD_MAXLOCK>(partial, nrows, out);
    if (threadIdx.x != 0) return;
    double cc = 0.0;
    for (int k = 0; k < SQD_MAXLOCK; ++k) {
        st->xc[k] = (k < nx) ? out[1 + k] : 0.0;
        cc += st->xc[k] * st->xc[k];
    }
    const double a2 = out[0], b2 = a2 - cc;
    if (round == 0 && b2 < 0.5 * a2) {
        st->xredo = 1;
        st->xscale = 1.0;
        return;
    }
    if (round == 0) st->xredo = 0;
    if (!(b2 > 1e-28 * a2) || !(b2 > 0.0)) {   // nothing left outside the locked space
        st->done = DONE_STALLED;
        return;
    }
    st->xscale = 1.0 / sqrt(b2);
}

// v = (v - X xc) * xscale; after the last pass also cin (and c32) = v
__device__ __forceinline__ void d_xapply(const double* __restrict__ X, int nx, double* __restrict__ V, int vrow,
                                         int64_t n, const dav_state* st, int round, double* __restrict__ cin,
                                         float* __restrict__ c32, int64_t bid, int64_t nblk) {
    if (st->done || (round == 1 && !st->xredo)) return;
    double* v = vrow ? V + (int64_t)st->m * n : V;
    const bool last = (round == 1) || !st->xredo;
    const double sc = st->xscale;
    double c[SQD_MAXLOCK];
    const double* xr[SQD_MAXLOCK];
#pragma unroll
    for (int k = 0; k < SQD_MAXLOCK; ++k) {
        c[k] = (k < nx) ? st->xc[k] : 0.0;
        xr[k] = row_ptr(X, k, nx, n);
    }
    const bool lo = (st->phase == 0) && c32;
    for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads) {
        double x[SQD_MAXLOCK];
#pragma unroll
        for (int k = 0; k < SQD_MAXLOCK; ++k) x[k] = xr[k][i];
        double t = v[i];
#pragma unroll
        for (int k = 0; k < SQD_MAXLOCK; ++k) t -= c[k] * x[k];
        t *= sc;
        v[i] = t;
        if (last) {
            cin[i] = t;
            if (lo) c32[i] = (float)t;
        }
    }
}

__device__ __forceinline__ void f_set_phase(dav_state* st, int phase, int done) {
    if (threadIdx.x == 0) {
        st->phase = phase;
        st->phase_start = st->iter;
        st->done = done;
    }
}


}  // namespace dav
