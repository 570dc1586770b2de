// Davidson-Liu for the lowest root, entirely on the device (Sec. III names
// moving the whole iteration -- vector updates, dot products, norms,
// Gram-Schmidt -- to the GPU as the alternative to offloading only the
// product; Sec. VI lists those steps; Sec. I cites the algorithm).
//
// All control state (basis size m, projected matrix G, Ritz pair, flags) lives
// in device memory; every kernel reads it and returns at once when the solve
// has ended, so the host can enqueue several iterations (or replay a captured
// graph) between polls.  Grid reductions are deterministic: each block writes
// its partial sums and the last block to finish (atomic ticket) sums them in
// block order and updates the state.
//
// One iteration (m basis vectors V, AV = H V, G = V^T A V, Ritz pair theta, y):
//   residual   x = V y, Ax = AV y, r = Ax - theta x, t = r / (theta - H_II)
//              (|den| < 1e-8 replaced by +-1e-8); partials of |r|^2, |t|^2 and
//              h = V^T t (first classical Gram-Schmidt pass) in the same sweep.
//              Last block: convergence / cap / phase-switch decisions.
//   collapse   (only when m == m_max) V[0] = V y, AV[0] = AV y in place.
//   orth1      t1 = t - V h, partials of h2 = V^T t1 and |t1|^2 (second pass).
//   orth2      v = (t1 - V h2) / |t1 - V h2| -> V[m] and the product input.
//   sigma      AV[m] = H v (FP64, or FP32 off-diagonal terms in mixed mode).
//   dots       G[:, m] = V^T AV[m]; last block: m += 1 and a parallel cyclic
//              Jacobi eigen-solve of G for the next (theta, y).
#include <chrono>
#include <cmath>
#include <cstring>

#include "sqd_internal.h"

namespace {

constexpr int MM = SQD_MMAX;
constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxBlocks = 2048;
constexpr int kPstride = MM + 4;   // partial sums per block

enum { DONE_RUNNING = 0, DONE_CONVERGED = 1, DONE_STALLED = 2, DONE_CAP = 3, DONE_SWITCH = 4 };

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
    int pad_;
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
};

struct dav_params {
    double tol;
    double switch_tol;
    int max_iter;
    int m_max;
    int mixed;
};

// Partial sums written by other blocks of the same launch.  The last block
// reads them after the ticket's fence; this CU's vector cache cannot hold
// stale copies (nothing in the launch read them before, and the cache is
// invalidated at launch), so plain loads are used: they issue in parallel.
__device__ __forceinline__ double ld_part(const double* p) { return *p; }

// Returns true in exactly one block: the last to arrive.  Every block must call it.
__device__ bool last_block(int* counter) {
    __shared__ int amlast;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const int prev = atomicAdd(counter, 1);
        amlast = (prev == (int)gridDim.x - 1);
    }
    __syncthreads();
    if (amlast) __threadfence();
    return amlast != 0;
}

// Block-wide sums of acc[0..NV) (wave shuffles, then one LDS slot per wave);
// written to partial row blockIdx.x.  All NV entries are reduced so that every
// register index is static.
template <int NV>
__device__ void block_to_partial(const double (&acc)[NV], double* __restrict__ partial) {
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
        partial[(size_t)blockIdx.x * kPstride + threadIdx.x] = s;
    }
}

// In the last block: out[j] = sum over blocks of partial[b][cols[j]] for
// j < ncol.  One wave per column (lanes stride the blocks, then shuffles);
// fixed order, so the result is deterministic.  Ends with a barrier.
__device__ void partials_to_out(const double* __restrict__ partial, int nblocks, const int* cols, int ncol,
                                double* out) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int j = w; j < ncol; j += kWaves) {
        const int c = cols[j];
        double s = 0.0;
        int b = lane;
        for (; b + 192 < nblocks; b += 256)   // four independent loads in flight
            s += (ld_part(&partial[(size_t)b * kPstride + c]) + ld_part(&partial[(size_t)(b + 64) * kPstride + c])) +
                 (ld_part(&partial[(size_t)(b + 128) * kPstride + c]) +
                  ld_part(&partial[(size_t)(b + 192) * kPstride + c]));
        for (; b < nblocks; b += 64) s += ld_part(&partial[(size_t)b * kPstride + c]);
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
        if (lane == 0) out[j] = s;
    }
    __syncthreads();
}

// ---------------------------------------------------------------- kernels

// argmin of the diagonal (lowest index on ties) -> st->kmin
__global__ void __launch_bounds__(kThreads) k_argmin(const double* __restrict__ d, int64_t n, dav_state* st,
                                                     double* __restrict__ partial) {
    __shared__ double sv[kThreads];
    __shared__ long long si[kThreads];
    double best = INFINITY;
    long long bi = -1;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
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
        partial[(size_t)blockIdx.x * kPstride + 0] = sv[0];
        partial[(size_t)blockIdx.x * kPstride + 1] = (double)si[0];
    }
    if (last_block(&st->counter[0])) {
        double b = INFINITY;
        long long k = -1;
        for (unsigned q = threadIdx.x; q < gridDim.x; q += kThreads) {
            const double v = ld_part(&partial[(size_t)q * kPstride]);
            const long long j = (long long)ld_part(&partial[(size_t)q * kPstride + 1]);
            if (j >= 0 && (k < 0 || v < b || (v == b && j < k))) { b = v; k = j; }
        }
        sv[threadIdx.x] = b;
        si[threadIdx.x] = k;
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
            st->kmin = (int)(si[0] < 0 ? 0 : si[0]);
            st->counter[0] = 0;
        }
    }
}

// V[0] = start vector (explicit guess, or e_kmin + noise); pass 1 normalises it.
__global__ void __launch_bounds__(kThreads) k_start(const double* __restrict__ guess, const double* __restrict__ noise,
                                                    int64_t n, dav_state* st, double* __restrict__ V0,
                                                    double* __restrict__ partial, int pass) {
    if (pass == 0) {
        double acc[1] = {0.0};
        const int64_t kmin = st->kmin;
        for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
            double v;
            if (guess) v = guess[i];
            else v = (i == kmin ? 1.0 : 0.0) + (noise ? noise[i] : 0.0);
            V0[i] = v;
            acc[0] += v * v;
        }
        block_to_partial<1>(acc, partial);
        if (last_block(&st->counter[1])) {
            __shared__ double out[1];
            const int cols[1] = {0};
            partials_to_out(partial, gridDim.x, cols, 1, out);
            if (threadIdx.x == 0) {
                st->tinv = 1.0 / sqrt(out[0]);
                st->counter[1] = 0;
            }
        }
    } else {
        const double sc = st->tinv;
        for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
            V0[i] *= sc;
    }
}

__global__ void k_copy_vec(const double* __restrict__ a, double* __restrict__ b, float* __restrict__ b32, int64_t n,
                           const int* __restrict__ skip) {
    if (skip && *skip) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        b[i] = a[i];
        if (b32) b32[i] = (float)a[i];
    }
}

// Residual, preconditioned correction and the first Gram-Schmidt projection.
template <int MT>
__global__ void __launch_bounds__(kThreads)
k_residual(const double* __restrict__ V, const double* __restrict__ AV, const double* __restrict__ diag, int64_t n,
           dav_state* st, dav_params prm, double* __restrict__ T, double* __restrict__ partial) {
    if (st->done) return;
    const int m = st->m;
    const double theta = st->theta;
    double acc[MT + 2];
#pragma unroll
    for (int k = 0; k < MT + 2; ++k) acc[k] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        double x = 0.0, ax = 0.0;
#pragma unroll
        for (int k = 0; k < MT; ++k)
            if (k < m) {
                const double yk = st->y[k];
                x += yk * V[(int64_t)k * n + i];
                ax += yk * AV[(int64_t)k * n + i];
            }
        const double r = ax - theta * x;
        double den = theta - diag[i];
        if (fabs(den) < 1e-8) den = (den < 0.0) ? -1e-8 : 1e-8;
        const double tv = r / den;
        T[i] = tv;
        acc[MT] += r * r;
        acc[MT + 1] += tv * tv;
#pragma unroll
        for (int k = 0; k < MT; ++k)
            if (k < m) acc[k] += V[(int64_t)k * n + i] * tv;
    }
    block_to_partial<MT + 2>(acc, partial);
    if (last_block(&st->counter[2])) {
        __shared__ double out[MT + 2];
        __shared__ int cols[MT + 2];
        if (threadIdx.x < m) cols[threadIdx.x] = threadIdx.x;
        if (threadIdx.x == 0) { cols[m] = MT; cols[m + 1] = MT + 1; }
        __syncthreads();
        partials_to_out(partial, gridDim.x, cols, m + 2, out);
        if (threadIdx.x == 0) {
            const double rn = sqrt(out[m]);
            st->rnorm = rn;
            st->tt0 = out[m + 1];
            for (int j = 0; j < m; ++j) st->h[j] = out[j];
            const int it = st->iter;
            if (it < SQD_HIST) {
                st->hist_r[it] = rn;
                st->hist_e[it] = theta;
                st->nhist = it + 1;
            }
            st->iter = it + 1;
            int done = DONE_RUNNING;
            if (st->phase == 0) {
                // FP32 phase: hand over to FP64 refinement below switch_tol, on
                // reaching tol, or when the residual stops falling
                const int inphase = st->iter - st->phase_start;
                const bool stall = inphase >= 6 && it >= 5 && it - 5 < SQD_HIST && rn > 0.7 * st->hist_r[it - 5];
                if (rn < prm.switch_tol || rn <= prm.tol || stall) done = DONE_SWITCH;
            } else if (rn <= prm.tol) {
                done = DONE_CONVERGED;
            }
            if (done == DONE_RUNNING && st->iter >= prm.max_iter) done = DONE_CAP;
            st->done = done;
            st->collapse = 0;
            if (done == DONE_RUNNING && m >= prm.m_max) {
                // keep the Ritz vector and the previous Ritz vector (orthonormalised
                // in the small space): q1 = y, q2 ~ y_prev - (y.y_prev) y
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
                    // second projection for orthogonality in the small space
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
                // projected matrix and Gram-Schmidt coefficients in the kept basis
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
            st->counter[2] = 0;
        }
    }
}

// In-place collapse: V[a] = V qc[a], AV[a] = AV qc[a] for the kept columns a.
// force = 1 (switch to FP64 refinement): keep x = V y only, AV not kept, and
// the next dots pass rebuilds G[0][0].
template <int MT>
__global__ void __launch_bounds__(kThreads)
k_collapse(double* __restrict__ V, double* __restrict__ AV, int64_t n, dav_state* st, int force,
           double* __restrict__ cin) {
    int keep;
    if (force) {
        keep = 1;
    } else {
        if (st->done || !st->collapse) return;
        keep = st->collapse;
    }
    const int m = st->m;
    const double* q1 = force ? st->y : st->qc[0];
    const double* q2 = st->qc[1];
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        double x1 = 0.0, x2 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int k = 0; k < MT; ++k)
            if (k < m) {
                const double v = V[(int64_t)k * n + i];
                x1 += q1[k] * v;
                x2 += q2[k] * v;
                if (!force) {
                    const double av = AV[(int64_t)k * n + i];
                    a1 += q1[k] * av;
                    a2 += q2[k] * av;
                }
            }
        V[i] = x1;
        if (keep == 2) V[n + i] = x2;
        if (!force) {
            AV[i] = a1;
            if (keep == 2) AV[n + i] = a2;
        }
        if (cin) cin[i] = x1;
    }
    if (last_block(&st->counter[3])) {
        if (threadIdx.x == 0) {
            if (force) {
                st->m = 0;
            } else {
                st->m = keep;
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
            }
            st->collapse = 0;
            st->counter[3] = 0;
        }
    }
}

template <int MT>
__global__ void __launch_bounds__(kThreads)
k_orth1(const double* __restrict__ V, int64_t n, dav_state* st, double* __restrict__ T, double* __restrict__ partial) {
    if (st->done) return;
    const int m = st->m;
    double acc[MT + 1];
#pragma unroll
    for (int k = 0; k < MT + 1; ++k) acc[k] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        double t = T[i];
#pragma unroll
        for (int k = 0; k < MT; ++k)
            if (k < m) t -= st->h[k] * V[(int64_t)k * n + i];
        T[i] = t;
        acc[MT] += t * t;
#pragma unroll
        for (int k = 0; k < MT; ++k)
            if (k < m) acc[k] += V[(int64_t)k * n + i] * t;
    }
    block_to_partial<MT + 1>(acc, partial);
    if (last_block(&st->counter[4])) {
        __shared__ double out[MT + 1];
        __shared__ int cols[MT + 1];
        if (threadIdx.x < m) cols[threadIdx.x] = threadIdx.x;
        if (threadIdx.x == 0) cols[m] = MT;
        __syncthreads();
        partials_to_out(partial, gridDim.x, cols, m + 1, out);
        if (threadIdx.x == 0) {
            double hh = 0.0;
            for (int j = 0; j < m; ++j) {
                st->h[j] = out[j];
                hh += out[j] * out[j];
            }
            const double t1 = out[m];
            const double nrm2 = t1 - hh;
            // a second projection only when the first left a visible overlap
            st->reortho = (hh > 1e-26 * t1) ? 1 : 0;
            if (!(nrm2 > 1e-28 * st->tt0) || !(nrm2 > 0.0)) {
                st->done = (st->rnorm <= 0.0) ? DONE_CONVERGED : DONE_STALLED;
            } else {
                st->tinv = 1.0 / sqrt(st->reortho ? nrm2 : t1);
            }
            st->counter[4] = 0;
        }
    }
}

template <int MT>
__global__ void __launch_bounds__(kThreads)
k_orth2(double* __restrict__ V, int64_t n, dav_state* st, const double* __restrict__ T, double* __restrict__ cin,
        float* __restrict__ c32) {
    if (st->done) return;
    const int m = st->m;
    const double sc = st->tinv;
    const bool re = st->reortho != 0;
    double* vm = V + (int64_t)m * n;
    const bool lo = (st->phase == 0) && c32;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        double t = T[i];
        if (re) {
#pragma unroll
            for (int k = 0; k < MT; ++k)
                if (k < m) t -= st->h[k] * V[(int64_t)k * n + i];
        }
        t *= sc;
        vm[i] = t;
        cin[i] = t;
        if (lo) c32[i] = (float)t;
    }
}

// AV[m] = S; G[k][m] = G[m][k] = V[k] . S for k <= m; m += 1.
template <int MT>
__global__ void __launch_bounds__(kThreads)
k_dots(const double* __restrict__ V, double* __restrict__ AV, const double* __restrict__ S, int64_t n, dav_state* st,
       double* __restrict__ partial) {
    if (st->done) return;
    const int m = st->m;
    double acc[MT + 1];
#pragma unroll
    for (int k = 0; k <= MT; ++k) acc[k] = 0.0;
    double* avm = AV + (int64_t)m * n;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const double s = S[i];
        avm[i] = s;
#pragma unroll
        for (int k = 0; k <= MT; ++k)
            if (k <= m) acc[k] += V[(int64_t)k * n + i] * s;
    }
    block_to_partial<MT + 1>(acc, partial);
    if (last_block(&st->counter[5])) {
        __shared__ double out[MT + 1];
        __shared__ int cols[MT + 1];
        if (threadIdx.x <= m) cols[threadIdx.x] = threadIdx.x;
        __syncthreads();
        partials_to_out(partial, gridDim.x, cols, m + 1, out);
        if (threadIdx.x == 0) {
            for (int j = 0; j <= m; ++j) {
                st->G[j * MM + m] = out[j];
                st->G[m * MM + j] = out[j];
            }
            st->m = m + 1;
            st->counter[5] = 0;
        }
    }
}

// Lowest eigenpair of G (m x m) by parallel cyclic Jacobi in one wavefront:
// theta, y; the previous y is kept as y_prev (padded with a zero).
__global__ void __launch_bounds__(64) k_eig(dav_state* st, int ignore_done) {
    if (!ignore_done && st->done) return;
    __shared__ double A[MM * MM];
    __shared__ double Q[MM * MM];
    __shared__ double rc[MM / 2], rs[MM / 2];
    __shared__ int rp[MM / 2], rq[MM / 2];
    const int t = threadIdx.x;
    const int m = st->m;
    for (int k = t; k < MM; k += 64) st->y_prev[k] = st->y[k];
    for (int k = t; k < MM * MM; k += 64) {
        A[k] = st->G[k];
        Q[k] = ((k / MM) == (k % MM)) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (m > 1) {
        const int n2 = (m + 1) & ~1;
        const int npair = n2 / 2;
        for (int sweep = 0; sweep < 50; ++sweep) {
            double off = 0.0, tot = 0.0;
            for (int k = t; k < m * m; k += 64) {
                const int i = k / m, j = k % m;
                const double v = A[i * MM + j];
                tot += v * v;
                if (i != j) off += v * v;
            }
            for (int o = 32; o > 0; o >>= 1) {
                off += __shfl_xor(off, o);
                tot += __shfl_xor(tot, o);
            }
            if (off <= 1e-28 * tot || off == 0.0) break;
            for (int step = 0; step < n2 - 1; ++step) {
                if (t < npair) {
                    // round-robin pairing: player 0 fixed, the others rotate
                    const int pa = t, pb = n2 - 1 - t;
                    int p = pa == 0 ? 0 : ((pa - 1 + step) % (n2 - 1)) + 1;
                    int q = pb == 0 ? 0 : ((pb - 1 + step) % (n2 - 1)) + 1;
                    if (p > q) { const int x = p; p = q; q = x; }
                    double c = 1.0, s = 0.0;
                    if (q < m) {
                        const double apq = A[p * MM + q];
                        if (apq != 0.0) {
                            const double tau = (A[q * MM + q] - A[p * MM + p]) / (2.0 * apq);
                            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                            c = 1.0 / sqrt(1.0 + tt * tt);
                            s = tt * c;
                        }
                    }
                    rc[t] = c; rs[t] = s; rp[t] = p; rq[t] = q;
                }
                __syncthreads();
                for (int k = t; k < npair * m; k += 64) {   // rows: A <- J^T A
                    const int pr = k / m, j = k % m;
                    const int p = rp[pr], q = rq[pr];
                    if (q >= m) continue;
                    const double c = rc[pr], s = rs[pr];
                    const double ap = A[p * MM + j], aq = A[q * MM + j];
                    A[p * MM + j] = c * ap - s * aq;
                    A[q * MM + j] = s * ap + c * aq;
                }
                __syncthreads();
                for (int k = t; k < npair * m; k += 64) {   // columns: A <- A J, Q <- Q J
                    const int pr = k / m, i = k % m;
                    const int p = rp[pr], q = rq[pr];
                    if (q >= m) continue;
                    const double c = rc[pr], s = rs[pr];
                    const double ap = A[i * MM + p], aq = A[i * MM + q];
                    A[i * MM + p] = c * ap - s * aq;
                    A[i * MM + q] = s * ap + c * aq;
                    const double qp = Q[i * MM + p], qq = Q[i * MM + q];
                    Q[i * MM + p] = c * qp - s * qq;
                    Q[i * MM + q] = s * qp + c * qq;
                }
                __syncthreads();
            }
        }
    }
    if (t == 0) {
        int kmin = 0;
        for (int k = 1; k < m; ++k)
            if (A[k * MM + k] < A[kmin * MM + kmin]) kmin = k;
        st->theta = A[kmin * MM + kmin];
        double nrm = 0.0;
        for (int k = 0; k < m; ++k) nrm += Q[k * MM + kmin] * Q[k * MM + kmin];
        nrm = 1.0 / sqrt(nrm);
        // sign: keep continuity with the previous Ritz vector
        double dp = 0.0;
        for (int k = 0; k < m; ++k) dp += Q[k * MM + kmin] * st->y_prev[k];
        if (dp < 0.0) nrm = -nrm;
        for (int k = 0; k < MM; ++k) st->y[k] = (k < m) ? Q[k * MM + kmin] * nrm : 0.0;
    }
}

// Final vector x = V y with its norm and largest-|x| entry (lowest index on ties).
template <int MT>
__global__ void __launch_bounds__(kThreads)
k_final(const double* __restrict__ V, int64_t n, dav_state* st, double* __restrict__ out, double* __restrict__ partial) {
    const int m = st->m;
    __shared__ double sv[kThreads], sn[kThreads];
    __shared__ long long si[kThreads];
    double best = -1.0, nrm = 0.0;
    long long bi = -1;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        double x = 0.0;
#pragma unroll
        for (int k = 0; k < MT; ++k)
            if (k < m) x += st->y[k] * V[(int64_t)k * n + i];
        out[i] = x;
        nrm += x * x;
        const double a = fabs(x);
        if (a > best) { best = a; bi = i; }
    }
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
        partial[(size_t)blockIdx.x * kPstride + 0] = sv[0];
        partial[(size_t)blockIdx.x * kPstride + 1] = (double)si[0];
        partial[(size_t)blockIdx.x * kPstride + 2] = sn[0];
    }
    if (last_block(&st->counter[6])) {
        double bv = -1.0, ss = 0.0;
        long long k = -1;
        for (unsigned q = threadIdx.x; q < gridDim.x; q += kThreads) {
            const double v = ld_part(&partial[(size_t)q * kPstride]);
            const long long j = (long long)ld_part(&partial[(size_t)q * kPstride + 1]);
            ss += ld_part(&partial[(size_t)q * kPstride + 2]);
            if (j >= 0 && (k < 0 || v > bv || (v == bv && j < k))) { bv = v; k = j; }
        }
        __syncthreads();
        sv[threadIdx.x] = bv; si[threadIdx.x] = k; sn[threadIdx.x] = ss;
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
            st->kmin = (int)(si[0] < 0 ? 0 : si[0]);
            st->tinv = 1.0 / sqrt(sn[0]);
            st->counter[6] = 0;
        }
    }
}

// sign of the largest entry, read before any rescaling
__global__ void k_final_sign(const double* __restrict__ out, dav_state* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int64_t k = st->kmin;
        if (out[k] < 0.0) st->tinv = -st->tinv;
    }
}

__global__ void k_final_scale(double* __restrict__ out, int64_t n, const dav_state* st) {
    const double sc = st->tinv;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        out[i] *= sc;
}

__global__ void k_set_phase(dav_state* st, int phase, int done) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->phase = phase;
        st->phase_start = st->iter;
        st->done = done;
    }
}

inline int grid_for(int64_t n) {
    int64_t b = (n + kThreads - 1) / kThreads;
    if (b > kMaxBlocks) b = kMaxBlocks;
    if (b < 1) b = 1;
    return (int)b;
}

// Launch helpers templated on the compile-time basis bound.
template <int MT>
struct dav_launch {
    static void residual(int g, hipStream_t s, const double* V, const double* AV, const double* d, int64_t n,
                         dav_state* st, dav_params p, double* T, double* part) {
        hipLaunchKernelGGL((k_residual<MT>), dim3(g), dim3(kThreads), 0, s, V, AV, d, n, st, p, T, part);
    }
    static void collapse(int g, hipStream_t s, double* V, double* AV, int64_t n, dav_state* st, int force, double* cin) {
        hipLaunchKernelGGL((k_collapse<MT>), dim3(g), dim3(kThreads), 0, s, V, AV, n, st, force, cin);
    }
    static void orth1(int g, hipStream_t s, const double* V, int64_t n, dav_state* st, double* T, double* part) {
        hipLaunchKernelGGL((k_orth1<MT>), dim3(g), dim3(kThreads), 0, s, V, n, st, T, part);
    }
    static void orth2(int g, hipStream_t s, double* V, int64_t n, dav_state* st, const double* T, double* cin, float* c32) {
        hipLaunchKernelGGL((k_orth2<MT>), dim3(g), dim3(kThreads), 0, s, V, n, st, T, cin, c32);
    }
    static void dots(int g, hipStream_t s, const double* V, double* AV, const double* S, int64_t n, dav_state* st,
                     double* part) {
        hipLaunchKernelGGL((k_dots<MT>), dim3(g), dim3(kThreads), 0, s, V, AV, S, n, st, part);
    }
    static void final_(int g, hipStream_t s, const double* V, int64_t n, dav_state* st, double* out, double* part) {
        hipLaunchKernelGGL((k_final<MT>), dim3(g), dim3(kThreads), 0, s, V, n, st, out, part);
    }
};

}  // namespace

// Workspace of one solve.
struct dav_work {
    double* V = nullptr;
    double* AV = nullptr;
    double* T = nullptr;
    double* cin = nullptr;
    double* sout = nullptr;
    float* c32 = nullptr;
    double* partial = nullptr;
    dav_state* st = nullptr;
    dav_state* st_host = nullptr;  // pinned
};

static void free_work(dav_work& w) {
    void* ps[] = {w.V, w.AV, w.T, w.cin, w.sout, w.c32, w.partial, w.st};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    if (w.st_host) (void)hipHostFree(w.st_host);
    w = dav_work();
}

template <int MT>
static int davidson_run(sqd_ctx* ctx, sqd_space* sp, const sqd_davidson_opts* o, double* energy, double* vec,
                        sqd_report* rep, dav_work& w, const dav_params& prm) {
    using L = dav_launch<MT>;
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = sp->dim;
    hipStream_t s = ctx->stream;
    int rc = sqd_ensure_diag(ctx, sp);
    if (rc) return rc;
    const double* diag = sp->diag;
    const int g = grid_for(n);
    std::memset(w.st_host, 0, sizeof(dav_state));
    w.st_host->phase = prm.mixed ? 0 : 1;
    w.st_host->y[0] = 1.0;
    if (hipMemcpyAsync(w.st, w.st_host, sizeof(dav_state), hipMemcpyHostToDevice, s) != hipSuccess)
        return sqd_hip_fail(ctx, hipGetLastError(), "state upload");
    // start vector, its product, G[0][0]
    if (!o->guess_dev) hipLaunchKernelGGL(k_argmin, dim3(g), dim3(kThreads), 0, s, diag, n, w.st, w.partial);
    hipLaunchKernelGGL(k_start, dim3(g), dim3(kThreads), 0, s, o->guess_dev, o->guess_noise_dev, n, w.st, w.V,
                       w.partial, 0);
    hipLaunchKernelGGL(k_start, dim3(g), dim3(kThreads), 0, s, o->guess_dev, o->guess_noise_dev, n, w.st, w.V,
                       w.partial, 1);
    hipLaunchKernelGGL(k_copy_vec, dim3(g), dim3(kThreads), 0, s, w.V, w.cin, w.c32, n, nullptr);
    const int* skip = &w.st->done;
    int prec = prm.mixed ? SQD_FP32 : SQD_FP64;
    if ((rc = sqd_sigma_impl(ctx, sp, w.cin, w.sout, prec, SQD_TERM_ALL, o->ab_path, prm.mixed ? w.c32 : nullptr,
                             skip)))
        return rc;
    L::dots(g, s, w.V, w.AV, w.sout, n, w.st, w.partial);
    hipLaunchKernelGGL(k_eig, dim3(1), dim3(64), 0, s, w.st, 0);
    if (hipGetLastError() != hipSuccess) return sqd_fail(ctx, SQD_E_HIP, "launch failed in Davidson start");

    int enqueued = 0;
    int switch_iter = -1;
    int final_done = DONE_CAP;
    while (true) {
        // enqueue check_every iterations, then poll the device flag; kernels of
        // iterations past the end return at once
        for (int k = 0; k < o->check_every; ++k) {
            L::residual(g, s, w.V, w.AV, diag, n, w.st, prm, w.T, w.partial);
            L::collapse(g, s, w.V, w.AV, n, w.st, 0, nullptr);
            L::orth1(g, s, w.V, n, w.st, w.T, w.partial);
            L::orth2(g, s, w.V, n, w.st, w.T, w.cin, prec == SQD_FP32 ? w.c32 : nullptr);
            if ((rc = sqd_sigma_impl(ctx, sp, w.cin, w.sout, prec, SQD_TERM_ALL, o->ab_path,
                                     prec == SQD_FP32 ? w.c32 : nullptr, skip)))
                return rc;
            L::dots(g, s, w.V, w.AV, w.sout, n, w.st, w.partial);
            hipLaunchKernelGGL(k_eig, dim3(1), dim3(64), 0, s, w.st, 0);
            ++enqueued;
        }
        if (hipGetLastError() != hipSuccess) return sqd_fail(ctx, SQD_E_HIP, "launch failed in Davidson loop");
        if (hipMemcpyAsync(w.st_host, w.st, sizeof(dav_state), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return sqd_fail(ctx, SQD_E_HIP, "Davidson state read-back failed");
        const int done = w.st_host->done;
        if (done == DONE_RUNNING) {
            if (enqueued > o->max_iter + 8) { final_done = DONE_CAP; break; }
            continue;
        }
        if (done == DONE_SWITCH) {
            // FP64 refinement: collapse onto the current Ritz vector, recompute
            // its product in FP64, rebuild G[0][0] and continue
            switch_iter = w.st_host->iter;
            prec = SQD_FP64;
            L::collapse(g, s, w.V, w.AV, n, w.st, 1, w.cin);
            hipLaunchKernelGGL(k_set_phase, dim3(1), dim3(64), 0, s, w.st, 1, DONE_RUNNING);
            if ((rc = sqd_sigma_impl(ctx, sp, w.cin, w.sout, SQD_FP64, SQD_TERM_ALL, o->ab_path, nullptr, skip)))
                return rc;
            L::dots(g, s, w.V, w.AV, w.sout, n, w.st, w.partial);
            hipLaunchKernelGGL(k_eig, dim3(1), dim3(64), 0, s, w.st, 0);
            continue;
        }
        final_done = done;
        break;
    }
    L::final_(g, s, w.V, n, w.st, vec, w.partial);
    hipLaunchKernelGGL(k_final_sign, dim3(1), dim3(64), 0, s, vec, w.st);
    hipLaunchKernelGGL(k_final_scale, dim3(g), dim3(kThreads), 0, s, vec, n, w.st);
    if (hipMemcpyAsync(w.st_host, w.st, sizeof(dav_state), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return sqd_fail(ctx, SQD_E_HIP, "Davidson final read-back failed");
    const dav_state& h = *w.st_host;
    *energy = h.theta;
    if (rep) {
        std::memset(rep, 0, sizeof(*rep));
        rep->iterations = h.iter;
        rep->iterations_fp32 = prm.mixed ? (switch_iter >= 0 ? switch_iter : h.iter) : 0;
        rep->switch_iter = switch_iter;
        rep->converged = (final_done == DONE_CONVERGED) ? 1 : 0;
        rep->status = final_done;
        rep->nhist = h.nhist;
        rep->energy = h.theta;
        rep->residual = h.rnorm;
        for (int k = 0; k < h.nhist && k < SQD_HIST; ++k) {
            rep->residual_history[k] = h.hist_r[k];
            rep->energy_history[k] = h.hist_e[k];
        }
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return final_done == DONE_CONVERGED ? SQD_OK : SQD_NOT_CONVERGED;
}

int sqd_davidson_impl(sqd_ctx* ctx, sqd_space* sp, const sqd_davidson_opts* o, double* energy, double* vec,
                      sqd_report* rep) {
    const int64_t n = sp->dim;
    const int mmax = o->m_max;
    dav_work w;
    int rc = SQD_OK;
#define DAV_ALLOC(ptr, bytes)                                                     \
    do {                                                                          \
        if ((rc = sqd_alloc(ctx, (void**)&(ptr), (bytes), nullptr))) {            \
            free_work(w);                                                         \
            return rc;                                                            \
        }                                                                         \
    } while (0)
    DAV_ALLOC(w.V, sizeof(double) * (size_t)n * mmax);
    DAV_ALLOC(w.AV, sizeof(double) * (size_t)n * mmax);
    DAV_ALLOC(w.T, sizeof(double) * n);
    DAV_ALLOC(w.cin, sizeof(double) * n);
    DAV_ALLOC(w.sout, sizeof(double) * n);
    if (o->mode == SQD_DAV_MIXED) DAV_ALLOC(w.c32, sizeof(float) * n);
    DAV_ALLOC(w.partial, sizeof(double) * kMaxBlocks * kPstride);
    DAV_ALLOC(w.st, sizeof(dav_state));
#undef DAV_ALLOC
    if (hipHostMalloc((void**)&w.st_host, sizeof(dav_state), hipHostMallocDefault) != hipSuccess) {
        free_work(w);
        return sqd_fail(ctx, SQD_E_OOM, "pinned host allocation failed");
    }
    dav_params prm;
    prm.tol = o->tol;
    prm.switch_tol = o->switch_tol;
    prm.max_iter = o->max_iter;
    prm.m_max = mmax;
    prm.mixed = o->mode == SQD_DAV_MIXED;
    if (mmax <= 8) rc = davidson_run<8>(ctx, sp, o, energy, vec, rep, w, prm);
    else if (mmax <= 16) rc = davidson_run<16>(ctx, sp, o, energy, vec, rep, w, prm);
    else if (mmax <= 24) rc = davidson_run<24>(ctx, sp, o, energy, vec, rep, w, prm);
    else rc = davidson_run<32>(ctx, sp, o, energy, vec, rep, w, prm);
    free_work(w);
    return rc;
}
