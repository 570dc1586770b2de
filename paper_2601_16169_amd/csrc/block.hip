// Block Davidson-Liu for the k lowest roots at once (Sec. I: SQD yields the
// ground and low-lying states from the projected Hamiltonian; Davidson's
// method, cited there, extended to a block of k vectors in the way of Liu's
// block form): one subspace serves all roots, each iteration adds one
// correction per root that has not converged, and restarts keep the k
// current Ritz vectors together with the k of the iteration before (as the
// single-root solver keeps its current and previous Ritz vectors).
//
// One iteration (basis V of m orthonormal vectors, AV = H V, G = V^T H V):
//   eigh       the m x m projected matrix in one workgroup (cyclic Jacobi,
//              round-robin pairs): theta_0 <= ... <= theta_{k-1}, Y = their
//              eigenvectors (m x k).
//   residual   r_j = AV y_j - theta_j V y_j, |r_j|, t_j = r_j / (theta_j - H_II)
//              (|den| < 1e-8 replaced by +-1e-8).
//   host       reads theta and |r_j|: stop when every |r_j| <= tol; restart
//              when the corrections would overflow m_max: Z = orthonormal
//              [Y, Y_prev] (coefficients, m x up to 2k), V <- V Z, AV <- AV Z,
//              G <- Z^T G Z.
//   expand     for each unconverged root, two classical Gram-Schmidt passes of
//              t_j against the current basis (new vectors included); appended
//              when at least 1e-6 of its norm survives.
//   products   AV[new] = H V[new] (FP64, or FP32 off-diagonal terms in the
//              first phase of a mixed solve), then G's new columns V^T AV[new].
// Basis rows are streamed with non-temporal loads (the basis is larger than
// the caches; the corrections and c stay cached).
// All reductions are deterministic: per-block partial sums and one finishing
// workgroup that adds them in block order.
#include <chrono>
#include <cmath>
#include <cstring>

#include "sqd_internal.h"

#include "davidson_body.h"

namespace {

using namespace dav;

constexpr int KB = SQD_MAXLOCK;   // most roots of one block solve
constexpr int kGB = 8;            // basis rows per G-column launch

struct blk_state {
    int m;                 // basis size
    int k;                 // roots
    int slot;              // row the last orthogonalised vector went to
    int accept;            // it was appended
    int kmin[KB];          // start determinants
    double G[MM * MM];
    double Y[MM * KB];     // Y[l * KB + j]: coefficient of basis row l in Ritz vector j
    double Yp[MM * KB];    // the previous iteration's Y (same basis: it only grew since)
    double Z[MM * 2 * KB]; // restart coefficients Z[l * 2KB + c], c < nkeep
    int nkeep;
    double theta[KB];
    double rnorm[KB];
    double h[MM];          // Gram-Schmidt coefficients of the vector being orthogonalised
    double P[MM * KB];     // block projection coefficients P[l * KB + j] = V_l . T_j
    double tn0[KB];        // squared norms of the corrections before any projection
    double hw;             // its squared norm before the first pass
    double t1sq;           // after the first pass
    double scale;          // 1 / predicted norm after the second pass
    double fscale[KB];     // final normalisation with the phase sign
    int fidx[KB];          // index of the largest |x_j| (lowest on ties)
};

// ---------------------------------------------------------------- start
// argmin of the diagonal over indices not already chosen (kmin[0..j))
__global__ void __launch_bounds__(kThreads) k_bargmin(const double* __restrict__ d, int64_t n,
                                                      const blk_state* st, int j, double* __restrict__ partial) {
    __shared__ double sv[kThreads];
    __shared__ long long si[kThreads];
    double best = INFINITY;
    long long bi = -1;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        bool taken = false;
        for (int q = 0; q < j; ++q) taken |= (st->kmin[q] == i);
        const double v = d[i];
        if (!taken && v < best) { best = v; bi = i; }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double v = sv[threadIdx.x + s];
            const long long q = si[threadIdx.x + s];
            if (q >= 0 && (si[threadIdx.x] < 0 || v < sv[threadIdx.x] || (v == sv[threadIdx.x] && q < si[threadIdx.x]))) {
                sv[threadIdx.x] = v;
                si[threadIdx.x] = q;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[(size_t)blockIdx.x * 2 + 0] = sv[0];
        partial[(size_t)blockIdx.x * 2 + 1] = (double)si[0];
    }
}

__global__ void __launch_bounds__(kThreads) k_bargmin_fin(const double* __restrict__ partial, int nrows,
                                                          blk_state* st, int j) {
    if (threadIdx.x != 0) return;
    double b = INFINITY;
    long long k = -1;
    for (int q = 0; q < nrows; ++q) {
        const double v = partial[(size_t)q * 2];
        const long long i = (long long)partial[(size_t)q * 2 + 1];
        if (i >= 0 && (k < 0 || v < b || (v == b && i < k))) { b = v; k = i; }
    }
    st->kmin[j] = (int)(k < 0 ? 0 : k);
}

// T[j] = e_kmin[j] + start noise (counter stream j + 1), j < k
__global__ void __launch_bounds__(kThreads) k_bstart(double* __restrict__ T, int64_t n, const blk_state* st, int k) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        for (int j = 0; j < k; ++j)
            T[(int64_t)j * n + i] = (i == st->kmin[j] ? 1.0 : 0.0) + start_noise((uint64_t)j + 1, i, n);
}

// ---------------------------------------------------------------- Gram-Schmidt of one vector t against V[m_lo..m)
// (m = st->m; the rows below m_lo were projected out already, as a block)
// pass 1 partials: V^T t (rows m_lo..m-1), |t|^2 (column NR)
__global__ void __launch_bounds__(kThreads) k_bo1(const double* __restrict__ V, const double* __restrict__ t,
                                                  int64_t n, const blk_state* st, int m_lo,
                                                  double* __restrict__ partial) {
    const int cnt = st->m - m_lo;
    const double* Vb = V + (int64_t)m_lo * n;
    with_rows<MM>(cnt, [&](auto nr) {
        constexpr int NR = decltype(nr)::value;
        double acc[NR + 1];
#pragma unroll
        for (int l = 0; l <= NR; ++l) acc[l] = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
            const double x = t[i];
            double v[NR];
#pragma unroll
            for (int l = 0; l < NR; ++l) v[l] = __builtin_nontemporal_load(row_ptr(Vb, l, cnt, n) + i);
#pragma unroll
            for (int l = 0; l < NR; ++l) acc[l] += (l < cnt ? v[l] : 0.0) * x;
            acc[NR] += x * x;
        }
        block_to_partial<NR + 1>(acc, partial, blockIdx.x, gridDim.x);
    });
}

// coefficients of pass 1; the reference squared norm for the acceptance test
// is the vector's own (ref < 0) or st->tn0[ref], its norm before the block
// projection
__global__ void __launch_bounds__(kThreads) k_bo1_fin(const double* __restrict__ partial, int nrows, blk_state* st,
                                                      int m_lo, int ref) {
    const int cnt = st->m - m_lo;
    with_rows<MM>(cnt, [&](auto nr) {
        constexpr int NR = decltype(nr)::value;
        __shared__ double out[MM + 1];
        reduce_rows<NR + 1>(partial, nrows, out);
        for (int l = threadIdx.x; l < MM; l += kThreads) st->h[l] = l < cnt ? out[l] : 0.0;
        if (threadIdx.x == 0) st->hw = ref >= 0 ? st->tn0[ref] : out[NR];
    });
}

// t1 = t - V h (in place); pass 2 partials: V^T t1, |t1|^2
__global__ void __launch_bounds__(kThreads) k_bo2(const double* __restrict__ V, double* __restrict__ t, int64_t n,
                                                  const blk_state* st, int m_lo, double* __restrict__ partial) {
    const int cnt = st->m - m_lo;
    const double* Vb = V + (int64_t)m_lo * n;
    with_rows<MM>(cnt, [&](auto nr) {
        constexpr int NR = decltype(nr)::value;
        double h[NR];
#pragma unroll
        for (int l = 0; l < NR; ++l) h[l] = st->h[l];   // zero past cnt
        double acc[NR + 1];
#pragma unroll
        for (int l = 0; l <= NR; ++l) acc[l] = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
            double v[NR];
#pragma unroll
            for (int l = 0; l < NR; ++l) v[l] = __builtin_nontemporal_load(row_ptr(Vb, l, cnt, n) + i);
            double x = t[i];
#pragma unroll
            for (int l = 0; l < NR; ++l) x -= h[l] * (l < cnt ? v[l] : 0.0);
            t[i] = x;
#pragma unroll
            for (int l = 0; l < NR; ++l) acc[l] += (l < cnt ? v[l] : 0.0) * x;
            acc[NR] += x * x;
        }
        block_to_partial<NR + 1>(acc, partial, blockIdx.x, gridDim.x);
    });
}

// second-pass coefficients; the vector is kept when its predicted norm after
// the second pass is above 1e-6 of the reference norm
__global__ void __launch_bounds__(kThreads) k_bo2_fin(const double* __restrict__ partial, int nrows, blk_state* st,
                                                      int m_lo, int m_cap) {
    const int m = st->m, cnt = m - m_lo;
    with_rows<MM>(cnt, [&](auto nr) {
        constexpr int NR = decltype(nr)::value;
        __shared__ double out[MM + 1];
        reduce_rows<NR + 1>(partial, nrows, out);
        for (int l = threadIdx.x; l < MM; l += kThreads) st->h[l] = l < cnt ? out[l] : 0.0;
        if (threadIdx.x == 0) {
            double hh = 0.0;
            for (int l = 0; l < cnt; ++l) hh += out[l] * out[l];
            const double t1sq = out[NR];
            const double t2sq = t1sq - hh;
            const bool ok = (m < m_cap) && t2sq > 1e-12 * st->hw && t2sq > 0.0;
            st->t1sq = t1sq;
            st->scale = ok ? 1.0 / sqrt(t2sq) : 0.0;
            st->accept = ok ? 1 : 0;
            st->slot = m;
            st->m = m + (ok ? 1 : 0);
        }
    });
}

// V[slot] = (t1 - V[m_lo..slot) h2) * scale when accepted
__global__ void __launch_bounds__(kThreads) k_bo3(double* __restrict__ V, const double* __restrict__ t, int64_t n,
                                                  const blk_state* st, int m_lo) {
    if (!st->accept) return;
    const int slot = st->slot, cnt = slot - m_lo;
    const double sc = st->scale;
    const double* Vb = V + (int64_t)m_lo * n;
    double* out = V + (int64_t)slot * n;
    with_rows<MM>(cnt, [&](auto nr) {
        constexpr int NR = decltype(nr)::value;
        double h[NR];
#pragma unroll
        for (int l = 0; l < NR; ++l) h[l] = st->h[l];
        for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
            double v[NR];
#pragma unroll
            for (int l = 0; l < NR; ++l) v[l] = __builtin_nontemporal_load(row_ptr(Vb, l, cnt, n) + i);
            double x = t[i];
#pragma unroll
            for (int l = 0; l < NR; ++l) x -= h[l] * (l < cnt ? v[l] : 0.0);
            out[i] = x * sc;
        }
    });
}

// Block projection of the k candidate rows of T against V[0..m): P = V^T T
// (partials by k_bgcols, stored by k_bpfin), then T -= V P.
template <int NB>
__global__ void __launch_bounds__(kThreads) k_bpfin(const double* __restrict__ partial, int nrows, blk_state* st,
                                                    int l0, int nl, int nc) {
    __shared__ double out[8 * NB];
    reduce_rows<8 * NB>(partial, nrows, out);
    for (int q = threadIdx.x; q < 8 * NB; q += kThreads) {
        const int a = q / NB, b = q % NB;
        if (a < nl && b < nc) st->P[(l0 + a) * KB + b] = out[q];
    }
}

template <int NK>
__global__ void __launch_bounds__(kThreads) k_bproj(const double* __restrict__ V, double* __restrict__ T, int64_t n,
                                                    int m, int nk, const blk_state* st) {
    __shared__ double Ps[MM * NK];
    for (int q = threadIdx.x; q < MM * NK; q += kThreads) Ps[q] = st->P[(q / NK) * KB + q % NK];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        double x[NK];
#pragma unroll
        for (int j = 0; j < NK; ++j) x[j] = j < nk ? T[(int64_t)j * n + i] : 0.0;
        for (int l = 0; l < m; ++l) {
            const double v = __builtin_nontemporal_load(V + (int64_t)l * n + i);
#pragma unroll
            for (int j = 0; j < NK; ++j) x[j] -= Ps[l * NK + j] * v;
        }
#pragma unroll
        for (int j = 0; j < NK; ++j)
            if (j < nk) T[(int64_t)j * n + i] = x[j];
    }
}

// ---------------------------------------------------------------- projected matrix
// partials of V[l0 + a]^T AV[c0 + b] for a < kGB, b < NB (rows and columns
// past the counts read the last valid ones and are dropped by the finisher)
template <int NB>
__global__ void __launch_bounds__(kThreads) k_bgcols(const double* __restrict__ V, const double* __restrict__ AV,
                                                     int64_t n, int l0, int nl, int c0, int nc,
                                                     double* __restrict__ partial) {
    double acc[kGB * NB];
#pragma unroll
    for (int q = 0; q < kGB * NB; ++q) acc[q] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        double v[kGB], w[NB];
#pragma unroll
        for (int a = 0; a < kGB; ++a) v[a] = __builtin_nontemporal_load(V + (int64_t)(l0 + (a < nl ? a : nl - 1)) * n + i);
#pragma unroll
        for (int b = 0; b < NB; ++b) w[b] = AV[(int64_t)(c0 + (b < nc ? b : nc - 1)) * n + i];
#pragma unroll
        for (int a = 0; a < kGB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[a * NB + b] += v[a] * w[b];
    }
    block_to_partial<kGB * NB>(acc, partial, blockIdx.x, gridDim.x);
}

template <int NB>
__global__ void __launch_bounds__(kThreads) k_bgcols_fin(const double* __restrict__ partial, int nrows, blk_state* st,
                                                         int l0, int nl, int c0, int nc) {
    __shared__ double out[kGB * NB];
    reduce_rows<kGB * NB>(partial, nrows, out);
    for (int q = threadIdx.x; q < kGB * NB; q += kThreads) {
        const int a = q / NB, b = q % NB;
        if (a < nl && b < nc) {
            const int r = l0 + a, c = c0 + b;
            st->G[r * MM + c] = out[q];
            st->G[c * MM + r] = out[q];
        }
    }
}

// Lowest k eigenpairs of the m x m matrix G (cyclic Jacobi, round-robin
// pairs; one workgroup).  theta ascending; Y columns normalised.
__global__ void __launch_bounds__(kThreads) k_beigh(blk_state* st) {
    constexpr int LS = MM + 1;
    __shared__ double A[MM * LS];
    __shared__ double Q[MM * LS];
    __shared__ double rc[MM / 2], rs[MM / 2];
    __shared__ int rp[MM / 2], rq[MM / 2];
    __shared__ double red[2 * kWaves];
    __shared__ int order[MM];
    const int t = threadIdx.x;
    const int m = st->m, k = st->k;
    for (int q = t; q < MM * KB; q += kThreads) st->Yp[q] = st->Y[q];
    for (int q = t; q < MM * MM; q += kThreads) {
        const int i = q / MM, j = q % MM;
        A[i * LS + j] = (i < m && j < m) ? st->G[q] : 0.0;
        Q[i * LS + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    // exact symmetry of the stored matrix
    for (int q = t; q < MM * MM; q += kThreads) {
        const int i = q / MM, j = q % MM;
        if (i < j && j < m) {
            const double v = 0.5 * (A[i * LS + j] + A[j * LS + i]);
            A[i * LS + j] = v;
            A[j * LS + i] = v;
        }
    }
    __syncthreads();
    if (m > 1) {
        const int n2 = (m + 1) & ~1;
        const int npair = n2 / 2;
        const int lane = t & 63, w = t >> 6;
        for (int sweep = 0; sweep < 60; ++sweep) {
            double off = 0.0, tot = 0.0;
            for (int q = t; q < MM * MM; q += kThreads) {
                const int i = q / MM, j = q % MM;
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
            if (off <= 1e-30 * tot || off == 0.0) break;
            for (int step = 0; step < n2 - 1; ++step) {
                if (t < npair) {
                    // round-robin: slot 0 fixed, the other n2 - 1 rotate by `step`
                    int a = t == 0 ? 0 : 1 + (t - 1 + step) % (n2 - 1);
                    int b = 1 + (n2 - 2 - t + step) % (n2 - 1);
                    if (a > b) { const int x = a; a = b; b = x; }
                    double c = 1.0, s = 0.0;
                    if (b < m) {
                        const double apq = A[a * LS + b];
                        if (apq != 0.0) jacobi_rotation(A[a * LS + a], A[b * LS + b], apq, c, s);
                    }
                    rc[t] = c; rs[t] = s; rp[t] = a; rq[t] = b;
                }
                __syncthreads();
                for (int q = t; q < (MM / 2) * (MM / 2); q += kThreads) {
                    const int b1 = q / (MM / 2), b2 = q % (MM / 2);
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
                for (int q = t; q < (MM / 2) * MM; q += kThreads) {
                    const int pr = q / MM, i = q % MM;
                    if (pr >= npair || i >= m) continue;
                    const int p = rp[pr], qq = rq[pr];
                    if (qq >= m || rs[pr] == 0.0) continue;
                    const double c = rc[pr], s = rs[pr];
                    const double qp = Q[i * LS + p], qv = Q[i * LS + qq];
                    Q[i * LS + p] = c * qp - s * qv;
                    Q[i * LS + qq] = s * qp + c * qv;
                }
                __syncthreads();
            }
        }
    }
    if (t == 0) {
        // eigenvalues ascending (stable: lowest index on ties)
        for (int i = 0; i < m; ++i) order[i] = i;
        for (int i = 1; i < m; ++i) {
            const int x = order[i];
            const double v = A[x * LS + x];
            int j = i - 1;
            while (j >= 0 && A[order[j] * LS + order[j]] > v) { order[j + 1] = order[j]; --j; }
            order[j + 1] = x;
        }
    }
    __syncthreads();
    for (int q = t; q < MM * KB; q += kThreads) {
        const int l = q / KB, j = q % KB;
        double v = 0.0;
        if (l < m && j < k && j < m) v = Q[l * LS + order[j]];
        st->Y[q] = v;
    }
    if (t < KB) st->theta[t] = (t < k && t < m) ? A[order[t] * LS + order[t]] : 0.0;
}

// ---------------------------------------------------------------- residuals, corrections, Ritz vectors
// For j < k: r_j = AV y_j - theta_j V y_j, T[j] = r_j / (theta_j - diag)
// (guarded); partials |r_j|^2.
template <int K>
__global__ void __launch_bounds__(kThreads) k_bresid(const double* __restrict__ V, const double* __restrict__ AV,
                                                     const double* __restrict__ diag, int64_t n,
                                                     const blk_state* st, double* __restrict__ T,
                                                     double* __restrict__ partial) {
    __shared__ double Ys[MM * K];
    __shared__ double th[K];
    const int m = st->m;
    for (int q = threadIdx.x; q < MM * K; q += kThreads) Ys[q] = st->Y[(q / K) * KB + q % K];
    if (threadIdx.x < K) th[threadIdx.x] = st->theta[threadIdx.x];
    __syncthreads();
    double acc[2 * K];
#pragma unroll
    for (int j = 0; j < 2 * K; ++j) acc[j] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        double x[K], ax[K];
#pragma unroll
        for (int j = 0; j < K; ++j) { x[j] = 0.0; ax[j] = 0.0; }
        for (int l = 0; l < m; ++l) {
            const double v = __builtin_nontemporal_load(V + (int64_t)l * n + i),
                         av = __builtin_nontemporal_load(AV + (int64_t)l * n + i);
#pragma unroll
            for (int j = 0; j < K; ++j) {
                x[j] += Ys[l * K + j] * v;
                ax[j] += Ys[l * K + j] * av;
            }
        }
        const double d = diag[i];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const double r = ax[j] - th[j] * x[j];
            acc[j] += r * r;
            double den = th[j] - d;
            if (fabs(den) < 1e-8) den = den < 0.0 ? -1e-8 : 1e-8;
            const double tv = r / den;
            T[(int64_t)j * n + i] = tv;
            acc[K + j] += tv * tv;
        }
    }
    block_to_partial<2 * K>(acc, partial, blockIdx.x, gridDim.x);
}

template <int K>
__global__ void __launch_bounds__(kThreads) k_bresid_fin(const double* __restrict__ partial, int nrows, blk_state* st) {
    __shared__ double out[2 * K];
    reduce_rows<2 * K>(partial, nrows, out);
    if (threadIdx.x < K) {
        st->rnorm[threadIdx.x] = sqrt(out[threadIdx.x]);
        st->tn0[threadIdx.x] = out[K + threadIdx.x];
    }
}

// Restart coefficients: Z = [Y, Y_prev] orthonormalised column by column
// (two classical Gram-Schmidt passes in coefficient space; a previous Ritz
// vector is dropped when under 1e-3 of it is new), at most kr columns; then
// G <- Z^T G Z.  One workgroup.
__global__ void __launch_bounds__(kThreads) k_bzq(blk_state* st, int kr) {
    __shared__ double Zs[MM * 2 * KB];
    __shared__ double GZ[MM * 2 * KB];
    __shared__ int nk;
    const int m = st->m, k = st->k;
    if (threadIdx.x == 0) {
        for (int q = 0; q < MM * 2 * KB; ++q) Zs[q] = 0.0;
        int nc = 0;
        for (int j = 0; j < k && nc < kr; ++j, ++nc)
            for (int l = 0; l < m; ++l) Zs[l * 2 * KB + nc] = st->Y[l * KB + j];
        for (int j = 0; j < k && nc < kr; ++j) {
            double z[MM];
            for (int l = 0; l < MM; ++l) z[l] = l < m ? st->Yp[l * KB + j] : 0.0;
            double n0 = 0.0;
            for (int l = 0; l < m; ++l) n0 += z[l] * z[l];
            if (!(n0 > 0.0)) continue;
            for (int pass = 0; pass < 2; ++pass)
                for (int c = 0; c < nc; ++c) {
                    double d = 0.0;
                    for (int l = 0; l < m; ++l) d += Zs[l * 2 * KB + c] * z[l];
                    for (int l = 0; l < m; ++l) z[l] -= d * Zs[l * 2 * KB + c];
                }
            double n1 = 0.0;
            for (int l = 0; l < m; ++l) n1 += z[l] * z[l];
            if (n1 <= 1e-6 * n0) continue;
            const double inv = 1.0 / sqrt(n1);
            for (int l = 0; l < m; ++l) Zs[l * 2 * KB + nc] = z[l] * inv;
            ++nc;
        }
        nk = nc;
    }
    __syncthreads();
    const int nc = nk;
    // GZ = G Z (m x nc), then G <- Z^T GZ (nc x nc)
    for (int q = threadIdx.x; q < MM * 2 * KB; q += kThreads) {
        const int l = q / (2 * KB), c = q % (2 * KB);
        double v = 0.0;
        if (l < m && c < nc)
            for (int r = 0; r < m; ++r) v += st->G[l * MM + r] * Zs[r * 2 * KB + c];
        GZ[q] = v;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < MM * MM; q += kThreads) {
        const int a = q / MM, b = q % MM;
        double v = 0.0;
        if (a < nc && b < nc)
            for (int l = 0; l < m; ++l) v += Zs[l * 2 * KB + a] * GZ[l * 2 * KB + b];
        st->G[q] = v;
    }
    for (int q = threadIdx.x; q < MM * 2 * KB; q += kThreads) st->Z[q] = Zs[q];
    if (threadIdx.x == 0) st->nkeep = nc;
}

// X[c] = V z_c, AX[c] = AV z_c for c < nkeep (NK >= nkeep)
template <int NK>
__global__ void __launch_bounds__(kThreads) k_bcombine(const double* __restrict__ V, const double* __restrict__ AV,
                                                       int64_t n, const blk_state* st, double* __restrict__ X,
                                                       double* __restrict__ AX) {
    __shared__ double Zs[MM * NK];
    const int m = st->m, nk = st->nkeep;
    for (int q = threadIdx.x; q < MM * NK; q += kThreads) Zs[q] = st->Z[(q / NK) * 2 * KB + q % NK];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        double x[NK], ax[NK];
#pragma unroll
        for (int c = 0; c < NK; ++c) { x[c] = 0.0; ax[c] = 0.0; }
        for (int l = 0; l < m; ++l) {
            const double v = __builtin_nontemporal_load(V + (int64_t)l * n + i),
                         av = __builtin_nontemporal_load(AV + (int64_t)l * n + i);
#pragma unroll
            for (int c = 0; c < NK; ++c) {
                x[c] += Zs[l * NK + c] * v;
                ax[c] += Zs[l * NK + c] * av;
            }
        }
#pragma unroll
        for (int c = 0; c < NK; ++c)
            if (c < nk) {
                X[(int64_t)c * n + i] = x[c];
                AX[(int64_t)c * n + i] = ax[c];
            }
    }
}

// V[c] = X[c], AV[c] = AX[c] for c < nkeep
__global__ void __launch_bounds__(kThreads) k_bcopy2(double* __restrict__ V, double* __restrict__ AV,
                                                     const double* __restrict__ X, const double* __restrict__ AX,
                                                     int64_t n, const blk_state* st) {
    const int64_t count = (int64_t)st->nkeep * n;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < count; i += (int64_t)gridDim.x * kThreads) {
        V[i] = X[i];
        AV[i] = AX[i];
    }
}

// after a restart: m = nkeep; the Ritz vectors are the first k new basis rows
__global__ void k_brestart_fin(blk_state* st) {
    const int k = st->k;
    for (int q = threadIdx.x; q < MM * KB; q += blockDim.x) {
        const int l = q / KB, j = q % KB;
        st->Y[q] = (l == j && j < k) ? 1.0 : 0.0;
    }
    if (threadIdx.x == 0) st->m = st->nkeep;
}

// final vectors: out[j] = V y_j, and per-block (largest |x|, its index, |x|^2)
template <int K>
__global__ void __launch_bounds__(kThreads) k_bfinal(const double* __restrict__ V, int64_t n, const blk_state* st,
                                                     double* __restrict__ out, double* __restrict__ partial) {
    __shared__ double Ys[MM * K];
    __shared__ double sv[K][kThreads];
    __shared__ long long si[K][kThreads];
    __shared__ double ss[K][kThreads];
    const int m = st->m;
    for (int q = threadIdx.x; q < MM * K; q += kThreads) Ys[q] = st->Y[(q / K) * KB + q % K];
    __syncthreads();
    double best[K], sq[K];
    long long bi[K];
#pragma unroll
    for (int j = 0; j < K; ++j) { best[j] = -1.0; bi[j] = -1; sq[j] = 0.0; }
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        double x[K];
#pragma unroll
        for (int j = 0; j < K; ++j) x[j] = 0.0;
        for (int l = 0; l < m; ++l) {
            const double v = __builtin_nontemporal_load(V + (int64_t)l * n + i);
#pragma unroll
            for (int j = 0; j < K; ++j) x[j] += Ys[l * K + j] * v;
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            out[(int64_t)j * n + i] = x[j];
            sq[j] += x[j] * x[j];
            if (fabs(x[j]) > best[j]) { best[j] = fabs(x[j]); bi[j] = i; }   // ascending i: first kept
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) { sv[j][threadIdx.x] = best[j]; si[j][threadIdx.x] = bi[j]; ss[j][threadIdx.x] = sq[j]; }
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const double v = sv[j][threadIdx.x + s];
                const long long q = si[j][threadIdx.x + s];
                if (q >= 0 && (si[j][threadIdx.x] < 0 || v > sv[j][threadIdx.x] ||
                               (v == sv[j][threadIdx.x] && q < si[j][threadIdx.x]))) {
                    sv[j][threadIdx.x] = v;
                    si[j][threadIdx.x] = q;
                }
                ss[j][threadIdx.x] += ss[j][threadIdx.x + s];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < K) {
        const int j = threadIdx.x;
        partial[((size_t)blockIdx.x * K + j) * 3 + 0] = sv[j][0];
        partial[((size_t)blockIdx.x * K + j) * 3 + 1] = (double)si[j][0];
        partial[((size_t)blockIdx.x * K + j) * 3 + 2] = ss[j][0];
    }
}

template <int K>
__global__ void k_bfinal_fin(const double* __restrict__ partial, int nrows, const double* __restrict__ out,
                             int64_t n, blk_state* st) {
    const int j = threadIdx.x;
    if (j >= K) return;
    double b = -1.0, s = 0.0;
    long long k = -1;
    for (int q = 0; q < nrows; ++q) {
        const double v = partial[((size_t)q * K + j) * 3 + 0];
        const long long i = (long long)partial[((size_t)q * K + j) * 3 + 1];
        s += partial[((size_t)q * K + j) * 3 + 2];
        if (i >= 0 && (k < 0 || v > b || (v == b && i < k))) { b = v; k = i; }
    }
    const double sc = 1.0 / sqrt(s);
    st->fidx[j] = (int)(k < 0 ? 0 : k);
    st->fscale[j] = (k >= 0 && out[(int64_t)j * n + k] < 0.0) ? -sc : sc;
}

__global__ void __launch_bounds__(kThreads) k_bscale(double* __restrict__ out, int64_t n, int k, const blk_state* st) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        for (int j = 0; j < k; ++j) out[(int64_t)j * n + i] *= st->fscale[j];
}

inline int grid_for(int64_t n) {
    int64_t b = (n + kThreads - 1) / kThreads;
    if (b > kMaxBlocks) b = kMaxBlocks;
    if (b < 1) b = 1;
    return (int)b;
}

// Launchers templated on the root count.
template <int K>
void launch_resid(int g, hipStream_t s, const double* V, const double* AV, const double* diag, int64_t n,
                  blk_state* st, double* T, double* part) {
    hipLaunchKernelGGL((k_bresid<K>), dim3(g), dim3(kThreads), 0, s, V, AV, diag, n, st, T, part);
    hipLaunchKernelGGL((k_bresid_fin<K>), dim3(1), dim3(kThreads), 0, s, part, g, st);
}

// Restart onto at most kr vectors: Z, X = V Z, AX = AV Z, V <- X, AV <- AX,
// G <- Z^T G Z, m <- nkeep.
void launch_restart(int g, hipStream_t s, double* V, double* AV, int64_t n, blk_state* st, int kr, double* X,
                    double* AX) {
    hipLaunchKernelGGL(k_bzq, dim3(1), dim3(kThreads), 0, s, st, kr);
    if (kr <= 2) hipLaunchKernelGGL((k_bcombine<2>), dim3(g), dim3(kThreads), 0, s, V, AV, n, st, X, AX);
    else if (kr <= 4) hipLaunchKernelGGL((k_bcombine<4>), dim3(g), dim3(kThreads), 0, s, V, AV, n, st, X, AX);
    else if (kr <= 8) hipLaunchKernelGGL((k_bcombine<8>), dim3(g), dim3(kThreads), 0, s, V, AV, n, st, X, AX);
    else hipLaunchKernelGGL((k_bcombine<16>), dim3(g), dim3(kThreads), 0, s, V, AV, n, st, X, AX);
    hipLaunchKernelGGL(k_bcopy2, dim3(g), dim3(kThreads), 0, s, V, AV, X, AX, n, st);
    hipLaunchKernelGGL(k_brestart_fin, dim3(1), dim3(kThreads), 0, s, st);
}
template <int K>
void launch_final(int g, hipStream_t s, const double* V, int64_t n, blk_state* st, double* out, double* part) {
    hipLaunchKernelGGL((k_bfinal<K>), dim3(g), dim3(kThreads), 0, s, V, n, st, out, part);
    hipLaunchKernelGGL((k_bfinal_fin<K>), dim3(1), dim3(64), 0, s, part, g, out, n, st);
}

template <typename F>
void with_k(int k, F&& f) {
    if (k <= 1) f(std::integral_constant<int, 1>{});
    else if (k <= 2) f(std::integral_constant<int, 2>{});
    else if (k <= 4) f(std::integral_constant<int, 4>{});
    else f(std::integral_constant<int, 8>{});
}

}  // namespace

int sqd_davidson_block_impl(sqd_ctx* ctx, sqd_space* sp, const sqd_davidson_opts* o, int k, double* energies,
                            double* vecs, sqd_report* reps) {
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = sp->dim;
    const int mmax = o->m_max;
    hipStream_t s = ctx->stream;
    int rc = sqd_ensure_diag(ctx, sp);
    if (rc) return rc;
    const double* diag = sp->diag;
    const int kk = k <= 1 ? 1 : (k <= 2 ? 2 : (k <= 4 ? 4 : 8));   // kernel width (>= k)
    // workspace (kept by the context, grown on demand): V, AV (m_max rows),
    // T (kk rows of corrections), X and AX (2 kk rows each, for restarts)
    double *V = nullptr, *AV = nullptr, *T = nullptr, *X = nullptr, *AX = nullptr, *part = nullptr;
    blk_state* st = nullptr;
    std::pair<void**, size_t> req[] = {
        {(void**)&V, sizeof(double) * (size_t)n * mmax},
        {(void**)&AV, sizeof(double) * (size_t)n * mmax},
        {(void**)&T, sizeof(double) * (size_t)n * kk},
        {(void**)&X, sizeof(double) * (size_t)n * 2 * kk},
        {(void**)&AX, sizeof(double) * (size_t)n * 2 * kk},
        {(void**)&part, sizeof(double) * kMaxBlocks * (kGB * KB + 8)},
        {(void**)&st, sizeof(blk_state)},
    };
    size_t total = 0;
    for (auto& r : req) total += (r.second + 255) & ~(size_t)255;
    if (ctx->dav_arena_bytes < total) {
        if (ctx->dav_arena) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(ctx->dav_arena);
            ctx->dav_arena = nullptr;
            ctx->dav_arena_bytes = 0;
        }
        if ((rc = sqd_alloc(ctx, &ctx->dav_arena, total, nullptr))) return rc;
        ctx->dav_arena_bytes = total;
    }
    {
        char* base = static_cast<char*>(ctx->dav_arena);
        size_t off = 0;
        for (auto& r : req) {
            *r.first = base + off;
            off += (r.second + 255) & ~(size_t)255;
        }
    }
    blk_state* hs = new blk_state();
    std::memset(hs, 0, sizeof(blk_state));
    hs->k = k;
    const int g = grid_for(n);
    SQD_HIP(ctx, hipMemcpyAsync(st, hs, sizeof(blk_state), hipMemcpyHostToDevice, s));
    auto fail = [&](int code, const char* what) {
        delete hs;
        return sqd_fail(ctx, code, what);
    };
    auto sync_state = [&]() -> bool {
        return hipMemcpyAsync(hs, st, sizeof(blk_state), hipMemcpyDeviceToHost, s) == hipSuccess &&
               hipStreamSynchronize(s) == hipSuccess;
    };
    // orthogonalise T row j against the basis rows m_lo.. (the rows below were
    // projected out as a block) and append it when accepted
    auto orth_append = [&](const double* tj, int m_lo, int ref) {
        hipLaunchKernelGGL(k_bo1, dim3(g), dim3(kThreads), 0, s, V, tj, n, st, m_lo, part);
        hipLaunchKernelGGL(k_bo1_fin, dim3(1), dim3(kThreads), 0, s, part, g, st, m_lo, ref);
        hipLaunchKernelGGL(k_bo2, dim3(g), dim3(kThreads), 0, s, V, const_cast<double*>(tj), n, st, m_lo, part);
        hipLaunchKernelGGL(k_bo2_fin, dim3(1), dim3(kThreads), 0, s, part, g, st, m_lo, mmax);
        hipLaunchKernelGGL(k_bo3, dim3(g), dim3(kThreads), 0, s, V, tj, n, st, m_lo);
    };
    // two block Gram-Schmidt passes of the kk rows of T against V[0..m)
    auto block_project = [&](int m) {
        for (int pass = 0; pass < 2; ++pass) {
            for (int l0 = 0; l0 < m; l0 += kGB) {
                const int nl = std::min(kGB, m - l0);
                if (kk <= 4) {
                    hipLaunchKernelGGL((k_bgcols<4>), dim3(g), dim3(kThreads), 0, s, V, T, n, l0, nl, 0, kk, part);
                    hipLaunchKernelGGL((k_bpfin<4>), dim3(1), dim3(kThreads), 0, s, part, g, st, l0, nl, kk);
                } else {
                    hipLaunchKernelGGL((k_bgcols<8>), dim3(g), dim3(kThreads), 0, s, V, T, n, l0, nl, 0, kk, part);
                    hipLaunchKernelGGL((k_bpfin<8>), dim3(1), dim3(kThreads), 0, s, part, g, st, l0, nl, kk);
                }
            }
            if (kk <= 4) hipLaunchKernelGGL((k_bproj<4>), dim3(g), dim3(kThreads), 0, s, V, T, n, m, kk, st);
            else hipLaunchKernelGGL((k_bproj<8>), dim3(g), dim3(kThreads), 0, s, V, T, n, m, kk, st);
        }
    };
    // products of the basis rows [m0, m1) and G's columns m0..m1-1 against rows [0, m1)
    auto products = [&](int m0, int m1, int prec) -> int {
        for (int l = m0; l < m1; ++l) {
            int r = (o->product == SQD_PRODUCT_STORED)
                        ? sqd_spmv_impl(ctx, sp, V + (int64_t)l * n, AV + (int64_t)l * n, nullptr)
                        : sqd_sigma_impl(ctx, sp, V + (int64_t)l * n, AV + (int64_t)l * n, prec, SQD_TERM_ALL,
                                         o->ab_path, nullptr, nullptr);
            if (r) return r;
        }
        for (int c0 = m0; c0 < m1; c0 += KB) {
            const int nc = std::min(KB, m1 - c0);
            for (int l0 = 0; l0 < m1; l0 += kGB) {
                const int nl = std::min(kGB, m1 - l0);
                if (nc <= 1) {
                    hipLaunchKernelGGL((k_bgcols<1>), dim3(g), dim3(kThreads), 0, s, V, AV, n, l0, nl, c0, nc, part);
                    hipLaunchKernelGGL((k_bgcols_fin<1>), dim3(1), dim3(kThreads), 0, s, part, g, st, l0, nl, c0, nc);
                } else if (nc <= 4) {
                    hipLaunchKernelGGL((k_bgcols<4>), dim3(g), dim3(kThreads), 0, s, V, AV, n, l0, nl, c0, nc, part);
                    hipLaunchKernelGGL((k_bgcols_fin<4>), dim3(1), dim3(kThreads), 0, s, part, g, st, l0, nl, c0, nc);
                } else {
                    hipLaunchKernelGGL((k_bgcols<8>), dim3(g), dim3(kThreads), 0, s, V, AV, n, l0, nl, c0, nc, part);
                    hipLaunchKernelGGL((k_bgcols_fin<8>), dim3(1), dim3(kThreads), 0, s, part, g, st, l0, nl, c0, nc);
                }
            }
        }
        return hipGetLastError() == hipSuccess ? SQD_OK : SQD_E_HIP;
    };

    // start: the k lowest diagonal determinants plus noise, orthonormalised
    for (int j = 0; j < k; ++j) {
        hipLaunchKernelGGL(k_bargmin, dim3(g), dim3(kThreads), 0, s, diag, n, st, j, part);
        hipLaunchKernelGGL(k_bargmin_fin, dim3(1), dim3(64), 0, s, part, g, st, j);
    }
    hipLaunchKernelGGL(k_bstart, dim3(g), dim3(kThreads), 0, s, T, n, st, k);
    for (int j = 0; j < k; ++j) orth_append(T + (int64_t)j * n, 0, -1);
    if (!sync_state()) return fail(SQD_E_HIP, "block Davidson start failed");
    if (hs->m < k) return fail(SQD_E_STATE, "block Davidson start vectors are linearly dependent");
    const bool mixed = o->mode == SQD_DAV_MIXED;
    int prec = mixed ? SQD_FP32 : SQD_FP64;
    if ((rc = products(0, k, prec))) {
        delete hs;
        return rc;
    }
    int m = k;
    int iter = 0, fp32_iters = 0, switch_iter = -1, nprod = k;
    int status = DONE_CAP;
    double best_r = INFINITY;
    int best_it = 0;
    std::vector<std::vector<double>> hist_r(k), hist_e(k);
    // vectors a restart keeps: the k Ritz vectors and up to k previous ones
    const int kr = std::min(2 * k, mmax - k);
    while (true) {
        hipLaunchKernelGGL(k_beigh, dim3(1), dim3(kThreads), 0, s, st);
        // a restart follows when the corrections could overflow m_max
        const bool restart = m + k > mmax;
        with_k(kk, [&](auto kc) {
            constexpr int K = decltype(kc)::value;
            launch_resid<K>(g, s, V, AV, diag, n, st, T, part);
        });
        if (hipGetLastError() != hipSuccess || !sync_state()) return fail(SQD_E_HIP, "block Davidson iteration failed");
        ++iter;
        if (prec == SQD_FP32) ++fp32_iters;
        double rmax = 0.0;
        int nconv = 0;
        for (int j = 0; j < k; ++j) {
            hist_r[j].push_back(hs->rnorm[j]);
            hist_e[j].push_back(hs->theta[j] + 0.0);
            rmax = std::max(rmax, hs->rnorm[j]);
            if (hs->rnorm[j] <= o->tol) ++nconv;
        }
        if (prec == SQD_FP64 && nconv == k) { status = DONE_CONVERGED; break; }
        if (iter >= o->max_iter) { status = DONE_CAP; break; }
        if (prec == SQD_FP32) {
            // leave FP32 products: below the switch tolerance, at the FP32
            // floor (2e-6 |theta|), or after 12 iterations without a 10% gain
            // once below 1e-4 |theta|
            const double th = std::fabs(hs->theta[k - 1]) + std::fabs(hs->theta[0]);
            if (rmax < 0.9 * best_r) { best_r = rmax; best_it = iter; }
            const bool stall = rmax < kStallFrom * th && iter - best_it >= kStallWindow;
            if (rmax < o->switch_tol || rmax <= o->tol || rmax < kFloor32 * th || stall) {
                // FP64 refinement: restart on the k Ritz vectors and recompute
                // their products in FP64
                switch_iter = iter;
                prec = SQD_FP64;
                launch_restart(g, s, V, AV, n, st, k, X, AX);
                if ((rc = products(0, k, SQD_FP64))) {
                    delete hs;
                    return rc;
                }
                nprod += k;
                m = k;
                best_r = INFINITY;
                continue;
            }
        }
        if (restart) {
            launch_restart(g, s, V, AV, n, st, kr, X, AX);
            if (!sync_state()) return fail(SQD_E_HIP, "block Davidson restart failed");
            m = hs->m;
        }
        // one correction per unconverged root: projected against the current
        // basis as a block, then against each other one by one
        block_project(m);
        for (int j = 0; j < k; ++j)
            if (!(hs->rnorm[j] <= o->tol) || prec == SQD_FP32) orth_append(T + (int64_t)j * n, m, j);
        if (!sync_state()) return fail(SQD_E_HIP, "block Davidson expansion failed");
        const int m1 = hs->m;
        if (m1 == m) { status = DONE_STALLED; break; }
        if ((rc = products(m, m1, prec))) {
            delete hs;
            return rc;
        }
        nprod += m1 - m;
        m = m1;
    }
    // final vectors (normalised, largest |x| positive) and energies
    with_k(kk, [&](auto kc) {
        constexpr int K = decltype(kc)::value;
        launch_final<K>(g, s, V, n, st, X, part);
    });
    hipLaunchKernelGGL(k_bscale, dim3(g), dim3(kThreads), 0, s, X, n, k, st);
    SQD_HIP(ctx, hipMemcpyAsync(vecs, X, sizeof(double) * (size_t)n * k, hipMemcpyDeviceToDevice, s));
    if (!sync_state()) return fail(SQD_E_HIP, "block Davidson final read-back failed");
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int out = SQD_OK;
    for (int j = 0; j < k; ++j) {
        energies[j] = hs->theta[j];
        const bool conv = hs->rnorm[j] <= o->tol && status == DONE_CONVERGED;
        if (!conv) out = SQD_NOT_CONVERGED;
        if (reps) {
            sqd_report* r = reps + j;
            std::memset(r, 0, sizeof(*r));
            r->iterations = iter;
            r->iterations_fp32 = fp32_iters;
            r->switch_iter = switch_iter;
            r->converged = conv ? 1 : 0;
            r->status = status;
            r->energy = hs->theta[j];
            r->residual = hs->rnorm[j];
            r->seconds = secs;
            r->nhist = (int)std::min<size_t>(hist_r[j].size(), SQD_HIST);
            for (int q = 0; q < r->nhist; ++q) {
                r->residual_history[q] = hist_r[j][q];
                r->energy_history[q] = hist_e[j][q];
            }
            r->products = nprod;
        }
    }
    delete hs;
    return out;
}
