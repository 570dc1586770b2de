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
constexpr int kMaxBlocks = 2048;
constexpr int kPstride = MM + 4;   // partial sums per block

enum { DONE_RUNNING = 0, DONE_CONVERGED = 1, DONE_STALLED = 2, DONE_CAP = 3, DONE_SWITCH = 4 };

struct dav_state {
    int m;
    int done;
    int iter;
    int collapse;
    int phase;            // 0: FP32 sigma (mixed mode), 1: FP64 sigma
    int phase_start;      // iteration at which the current phase began
    int kmin;
    int nhist;
    int counter[8];       // last-block tickets, one per kernel kind
    double theta;
    double rnorm;
    double tt0;           // |t|^2 before orthogonalisation
    double tinv;          // 1 / |v| of the new basis vector
    double h0new;         // y . h after a collapse
    double G[MM * MM];
    double y[MM];
    double h[MM];
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

__device__ __forceinline__ double ld_agent(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

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

// Block-wide sum of nv values per thread into red[0..nv): red has nv*kThreads slots.
__device__ void block_sum(double* vals, int nv, double* red) {
    const int t = threadIdx.x;
    for (int j = 0; j < nv; ++j) red[j * kThreads + t] = vals[j];
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (t < s)
            for (int j = 0; j < nv; ++j) red[j * kThreads + t] += red[j * kThreads + t + s];
        __syncthreads();
    }
}

// Sum partial[b][j] over blocks b for j < nv, in block order; result in out[j].
__device__ void reduce_partials(const double* partial, int nblocks, int nv, double* out, double* red) {
    const int t = threadIdx.x;
    for (int j = 0; j < nv; ++j) {
        double s = 0.0;
        for (int b = t; b < nblocks; b += kThreads) s += ld_agent(&partial[(size_t)b * kPstride + j]);
        red[t] = s;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if (t < w) red[t] += red[t + w];
            __syncthreads();
        }
        if (t == 0) out[j] = red[0];
        __syncthreads();
    }
}


// Sum of acc[0..nv) over the block (wave shuffles, then one LDS slot per wave);
// thread 0 writes the sums to partial row blockIdx.x at columns col0..col0+nv.
// (all NV entries are reduced so that every register index is static)
template <int NV>
__device__ void block_to_partial(const double (&acc)[NV], double* __restrict__ partial) {
    __shared__ double wred[kThreads / 64][NV];
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
        for (int q = 0; q < kThreads / 64; ++q) s += wred[q][threadIdx.x];
        partial[(size_t)blockIdx.x * kPstride + threadIdx.x] = s;
    }
}

// Sum partial[b][col0 + j] over blocks b (block order within each thread's
// stride, then a fixed tree), for j < nv; result in out[j] (shared).
__device__ void partials_to_out(const double* __restrict__ partial, int nblocks, int nv, int col0, double* out) {
    __shared__ double red[kThreads];
    const int t = threadIdx.x;
    for (int j = 0; j < nv; ++j) {
        double s = 0.0;
        for (int b = t; b < nblocks; b += kThreads) s += ld_agent(&partial[(size_t)b * kPstride + col0 + j]);
        red[t] = s;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if (t < w) red[t] += red[t + w];
            __syncthreads();
        }
        if (t == 0) out[j] = red[0];
        __syncthreads();
    }
}

// Parallel cyclic Jacobi on the symmetric m x m matrix in A (LDS, row stride MM);
// Q receives the eigenvectors (columns).  Whole block participates.
__device__ void jacobi_eig(double* A, double* Q, int m, double* rot_c, double* rot_s, int* rp, int* rq,
                           double* scratch) {
    const int t = threadIdx.x;
    for (int k = t; k < MM * MM; k += kThreads) Q[k] = ((k / MM) == (k % MM)) ? 1.0 : 0.0;
    __syncthreads();
    if (m <= 1) return;
    const int n2 = (m + 1) & ~1;
    const int npair = n2 / 2;
    for (int sweep = 0; sweep < 40; ++sweep) {
        // convergence: off-diagonal Frobenius mass against the whole matrix
        double off = 0.0, tot = 0.0;
        for (int k = t; k < m * m; k += kThreads) {
            const int i = k / m, j = k % m;
            const double v = A[i * MM + j];
            tot += v * v;
            if (i != j) off += v * v;
        }
        scratch[t] = off;
        scratch[kThreads + t] = tot;
        __syncthreads();
        for (int s = kThreads / 2; s > 0; s >>= 1) {
            if (t < s) {
                scratch[t] += scratch[t + s];
                scratch[kThreads + t] += scratch[kThreads + t + s];
            }
            __syncthreads();
        }
        const double offs = scratch[0], tots = scratch[kThreads];
        __syncthreads();
        if (offs <= 1e-32 * tots || offs == 0.0) break;
        for (int step = 0; step < n2 - 1; ++step) {
            if (t < npair) {
                // round-robin pairing: player 0 fixed, the others rotate
                auto player = [&](int pos) { return pos == 0 ? 0 : ((pos - 1 + step) % (n2 - 1)) + 1; };
                int p = player(t), q = player(n2 - 1 - t);
                if (p > q) { int x = p; p = q; q = x; }
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
                rot_c[t] = c; rot_s[t] = s; rp[t] = p; rq[t] = q;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int k = t; k < npair * m; k += kThreads) {
                const int pr = k / m, j = k % m;
                const int p = rp[pr], q = rq[pr];
                if (q >= m) continue;
                const double c = rot_c[pr], s = rot_s[pr];
                const double ap = A[p * MM + j], aq = A[q * MM + j];
                A[p * MM + j] = c * ap - s * aq;
                A[q * MM + j] = s * ap + c * aq;
            }
            __syncthreads();
            // columns: A <- A J, Q <- Q J
            for (int k = t; k < npair * m; k += kThreads) {
                const int pr = k / m, i = k % m;
                const int p = rp[pr], q = rq[pr];
                if (q >= m) continue;
                const double c = rot_c[pr], s = rot_s[pr];
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

// Lowest eigenpair of st->G (m x m) into st->theta, st->y.  Whole block.
__device__ void ritz_update(dav_state* st, int m) {
    __shared__ double A[MM * MM];
    __shared__ double Q[MM * MM];
    __shared__ double rc[MM], rs[MM];
    __shared__ int rp[MM], rq[MM];
    __shared__ double scr[2 * kThreads];
    const int t = threadIdx.x;
    for (int k = t; k < MM * MM; k += kThreads) A[k] = st->G[k];
    __syncthreads();
    jacobi_eig(A, Q, m, rc, rs, rp, rq, scr);
    if (t == 0) {
        int kmin = 0;
        for (int k = 1; k < m; ++k)
            if (A[k * MM + k] < A[kmin * MM + kmin]) kmin = k;
        st->theta = A[kmin * MM + kmin];
        double nrm = 0.0;
        for (int k = 0; k < m; ++k) nrm += Q[k * MM + kmin] * Q[k * MM + kmin];
        nrm = 1.0 / sqrt(nrm);
        for (int k = 0; k < MM; ++k) st->y[k] = (k < m) ? Q[k * MM + kmin] * nrm : 0.0;
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
        if (v < best || (v == best && i < bi)) { best = v; bi = i; }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double v = sv[threadIdx.x + s];
            const long long j = si[threadIdx.x + s];
            if (j >= 0 && (v < sv[threadIdx.x] || (v == sv[threadIdx.x] && (si[threadIdx.x] < 0 || j < si[threadIdx.x])))) {
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
        if (threadIdx.x == 0) {
            double b = INFINITY;
            long long k = 0;
            for (unsigned q = 0; q < gridDim.x; ++q) {
                const double v = ld_agent(&partial[(size_t)q * kPstride]);
                const long long j = (long long)ld_agent(&partial[(size_t)q * kPstride + 1]);
                if (j >= 0 && (v < b || (v == b && j < k))) { b = v; k = j; }
            }
            st->kmin = (int)k;
            st->counter[0] = 0;
        }
    }
}

// V[0] = start vector (explicit guess, or e_kmin + noise), normalised; also the product input.
__global__ void __launch_bounds__(kThreads) k_start(const double* __restrict__ guess, const double* __restrict__ noise,
                                                    int64_t n, dav_state* st, double* __restrict__ V0,
                                                    double* __restrict__ partial, int pass) {
    __shared__ double red[kThreads];
    if (pass == 0) {
        double s = 0.0;
        const int64_t kmin = st->kmin;
        for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
            double v;
            if (guess) v = guess[i];
            else v = (i == kmin ? 1.0 : 0.0) + (noise ? noise[i] : 0.0);
            V0[i] = v;
            s += v * v;
        }
        double vals[1] = {s};
        block_sum(vals, 1, red);
        if (threadIdx.x == 0) partial[(size_t)blockIdx.x * kPstride] = red[0];
        if (last_block(&st->counter[1])) {
            double out[1];
            __shared__ double red2[kThreads];
            reduce_partials(partial, gridDim.x, 1, out, red2);
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

__global__ void __launch_bounds__(kThreads)
k_residual(const double* __restrict__ V, const double* __restrict__ AV, const double* __restrict__ diag, int64_t n,
           dav_state* st, dav_params prm, double* __restrict__ T, double* __restrict__ partial) {
    if (st->done) return;
    const int m = st->m;
    const double theta = st->theta;
    double y[MM];
#pragma unroll
    for (int k = 0; k < MM; ++k) y[k] = st->y[k];
    double acc[MM + 2];
#pragma unroll
    for (int k = 0; k < MM + 2; ++k) acc[k] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        double v[MM];
        double x = 0.0, ax = 0.0;
#pragma unroll
        for (int k = 0; k < MM; ++k) {
            if (k < m) {
                v[k] = V[(int64_t)k * n + i];
                x += y[k] * v[k];
                ax += y[k] * AV[(int64_t)k * n + i];
            }
        }
        const double r = ax - theta * x;
        double den = theta - diag[i];
        if (fabs(den) < 1e-8) den = (den < 0.0) ? -1e-8 : 1e-8;
        const double tv = r / den;
        T[i] = tv;
        acc[MM] += r * r;
        acc[MM + 1] += tv * tv;
#pragma unroll
        for (int k = 0; k < MM; ++k)
            if (k < m) acc[k] += v[k] * tv;
    }
    // columns 0..m-1: V^T t; column MM: |r|^2; column MM+1: |t|^2
    block_to_partial<MM + 2>(acc, partial);
    if (last_block(&st->counter[2])) {
        __shared__ double out[MM + 2];
        partials_to_out(partial, gridDim.x, m, 0, out);
        partials_to_out(partial, gridDim.x, 2, MM, out + MM);
        if (threadIdx.x == 0) {
            const double rn = sqrt(out[MM]);
            st->rnorm = rn;
            st->tt0 = out[MM + 1];
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
            st->collapse = (done == DONE_RUNNING && m >= prm.m_max) ? 1 : 0;
            double h0 = 0.0;
            for (int j = 0; j < m; ++j) h0 += st->y[j] * out[j];
            st->h0new = h0;
            st->counter[2] = 0;
        }
    }
}

// In-place V[0] = V y, AV[0] = AV y when a collapse is pending (or forced).
__global__ void __launch_bounds__(kThreads)
k_collapse(double* __restrict__ V, double* __restrict__ AV, int64_t n, dav_state* st, int force, int with_av,
           double* __restrict__ cin, float* __restrict__ c32) {
    if (!force && (st->done || !st->collapse)) return;
    const int m = st->m;
    double y[MM];
#pragma unroll
    for (int k = 0; k < MM; ++k) y[k] = st->y[k];
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        double x = 0.0, ax = 0.0;
#pragma unroll
        for (int k = 0; k < MM; ++k)
            if (k < m) {
                x += y[k] * V[(int64_t)k * n + i];
                if (with_av) ax += y[k] * AV[(int64_t)k * n + i];
            }
        V[i] = x;
        if (with_av) AV[i] = ax;
        if (cin) cin[i] = x;
        if (c32) c32[i] = (float)x;
    }
    if (last_block(&st->counter[3])) {
        if (threadIdx.x == 0) {
            if (force) {
                st->m = 0;          // the next dots pass rebuilds G[0][0]
            } else {
                st->m = 1;
                for (int k = 0; k < MM * MM; ++k) st->G[k] = 0.0;
                st->G[0] = st->theta;
                st->h[0] = st->h0new;
                for (int k = 0; k < MM; ++k) st->y[k] = (k == 0) ? 1.0 : 0.0;
            }
            st->collapse = 0;
            st->counter[3] = 0;
        }
    }
}

__global__ void __launch_bounds__(kThreads)
k_orth1(const double* __restrict__ V, int64_t n, dav_state* st, double* __restrict__ T, double* __restrict__ partial) {
    if (st->done) return;
    const int m = st->m;
    double h[MM];
#pragma unroll
    for (int k = 0; k < MM; ++k) h[k] = st->h[k];
    double acc[MM + 1];
#pragma unroll
    for (int k = 0; k < MM + 1; ++k) acc[k] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        double v[MM];
        double t = T[i];
#pragma unroll
        for (int k = 0; k < MM; ++k)
            if (k < m) {
                v[k] = V[(int64_t)k * n + i];
                t -= h[k] * v[k];
            }
        T[i] = t;
        acc[MM] += t * t;
#pragma unroll
        for (int k = 0; k < MM; ++k)
            if (k < m) acc[k] += v[k] * t;
    }
    block_to_partial<MM + 1>(acc, partial);
    if (last_block(&st->counter[4])) {
        __shared__ double out[MM + 1];
        partials_to_out(partial, gridDim.x, m, 0, out);
        partials_to_out(partial, gridDim.x, 1, MM, out + MM);
        if (threadIdx.x == 0) {
            double hh = 0.0;
            for (int j = 0; j < m; ++j) {
                st->h[j] = out[j];
                hh += out[j] * out[j];
            }
            const double nrm2 = out[MM] - hh;
            if (!(nrm2 > 1e-28 * st->tt0) || !(nrm2 > 0.0)) {
                st->done = (st->rnorm <= 0.0) ? DONE_CONVERGED : DONE_STALLED;
            } else {
                st->tinv = 1.0 / sqrt(nrm2);
            }
            st->counter[4] = 0;
        }
    }
}

__global__ void __launch_bounds__(kThreads)
k_orth2(double* __restrict__ V, int64_t n, dav_state* st, const double* __restrict__ T, double* __restrict__ cin,
        float* __restrict__ c32) {
    if (st->done) return;
    const int m = st->m;
    const double sc = st->tinv;
    double h[MM];
#pragma unroll
    for (int k = 0; k < MM; ++k) h[k] = st->h[k];
    double* vm = V + (int64_t)m * n;
    const bool lo = (st->phase == 0);
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        double t = T[i];
#pragma unroll
        for (int k = 0; k < MM; ++k)
            if (k < m) t -= h[k] * V[(int64_t)k * n + i];
        t *= sc;
        vm[i] = t;
        cin[i] = t;
        if (lo && c32) c32[i] = (float)t;
    }
}

// AV[m] = S; G[k][m] = G[m][k] = V[k] . S for k <= m; then m += 1 and Ritz update.
__global__ void __launch_bounds__(kThreads)
k_dots(const double* __restrict__ V, double* __restrict__ AV, const double* __restrict__ S, int64_t n, dav_state* st,
       double* __restrict__ partial, int ignore_done) {
    if (!ignore_done && st->done) return;
    const int m = st->m;
    double acc[MM + 1];
#pragma unroll
    for (int k = 0; k <= MM; ++k) acc[k] = 0.0;
    double* avm = AV + (int64_t)m * n;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const double s = S[i];
        avm[i] = s;
#pragma unroll
        for (int k = 0; k <= MM; ++k)
            if (k <= m) acc[k] += V[(int64_t)k * n + i] * s;
    }
    block_to_partial<MM + 1>(acc, partial);
    if (last_block(&st->counter[5])) {
        __shared__ double out[MM + 1];
        partials_to_out(partial, gridDim.x, m + 1, 0, out);
        if (threadIdx.x == 0) {
            for (int j = 0; j <= m; ++j) {
                st->G[j * MM + m] = out[j];
                st->G[m * MM + j] = out[j];
            }
            st->m = m + 1;
            st->counter[5] = 0;
        }
        __syncthreads();
        ritz_update(st, m + 1);
    }
}

// Final vector x = V y, normalised, largest-|x| entry positive (lowest index on ties).
__global__ void __launch_bounds__(kThreads)
k_final(const double* __restrict__ V, int64_t n, dav_state* st, double* __restrict__ out, double* __restrict__ partial,
        int pass) {
    const int m = st->m;
    if (pass == 0) {
        __shared__ double sv[kThreads], sn[kThreads];
        __shared__ long long si[kThreads];
        double y[MM];
#pragma unroll
        for (int k = 0; k < MM; ++k) y[k] = st->y[k];
        double best = -1.0, nrm = 0.0;
        long long bi = -1;
        for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
            double x = 0.0;
#pragma unroll
            for (int k = 0; k < MM; ++k)
                if (k < m) x += y[k] * V[(int64_t)k * n + i];
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
                if (v > sv[threadIdx.x] || (v == sv[threadIdx.x] && j >= 0 && j < si[threadIdx.x])) {
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
            if (threadIdx.x == 0) {
                double b = -1.0, s = 0.0;
                long long k = -1;
                for (unsigned q = 0; q < gridDim.x; ++q) {
                    const double v = ld_agent(&partial[(size_t)q * kPstride]);
                    const long long j = (long long)ld_agent(&partial[(size_t)q * kPstride + 1]);
                    s += ld_agent(&partial[(size_t)q * kPstride + 2]);
                    if (v > b || (v == b && j >= 0 && j < k)) { b = v; k = j; }
                }
                st->kmin = (int)k;
                double sc = 1.0 / sqrt(s);
                st->tinv = sc;
                st->counter[6] = 0;
            }
        }
    }
}

// sign of the largest entry, read before any rescaling
__global__ void k_final_sign(const double* __restrict__ out, dav_state* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int64_t k = st->kmin;
        if (k >= 0 && out[k] < 0.0) st->tinv = -st->tinv;
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

int sqd_davidson_impl(sqd_ctx* ctx, sqd_space* sp, const sqd_davidson_opts* o, double* energy, double* vec,
                      sqd_report* rep) {
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = sp->dim;
    const int mmax = o->m_max;
    hipStream_t s = ctx->stream;
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
    auto fail = [&](int code) { free_work(w); return code; };
    if ((rc = sqd_ensure_diag(ctx, sp))) return fail(rc);
    const double* diag = sp->diag;
    const int g = grid_for(n);
    dav_params prm;
    prm.tol = o->tol;
    prm.switch_tol = o->switch_tol;
    prm.max_iter = o->max_iter;
    prm.m_max = mmax;
    prm.mixed = o->mode == SQD_DAV_MIXED;

    std::memset(w.st_host, 0, sizeof(dav_state));
    w.st_host->phase = prm.mixed ? 0 : 1;
    if (hipMemcpyAsync(w.st, w.st_host, sizeof(dav_state), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(sqd_hip_fail(ctx, hipGetLastError(), "state upload"));
    // start vector
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
        return fail(rc);
    hipLaunchKernelGGL(k_dots, dim3(g), dim3(kThreads), 0, s, w.V, w.AV, w.sout, n, w.st, w.partial, 0);
    if (hipGetLastError() != hipSuccess) return fail(sqd_fail(ctx, SQD_E_HIP, "launch failed in Davidson start"));

    int enqueued = 0;
    int switch_iter = -1;
    int fp32_iters = 0;
    int final_done = DONE_CAP;
    while (true) {
        // enqueue check_every iterations, then poll the device flag
        for (int k = 0; k < o->check_every; ++k) {
            hipLaunchKernelGGL(k_residual, dim3(g), dim3(kThreads), 0, s, w.V, w.AV, diag, n, w.st, prm, w.T, w.partial);
            hipLaunchKernelGGL(k_collapse, dim3(g), dim3(kThreads), 0, s, w.V, w.AV, n, w.st, 0, 1, nullptr, nullptr);
            hipLaunchKernelGGL(k_orth1, dim3(g), dim3(kThreads), 0, s, w.V, n, w.st, w.T, w.partial);
            hipLaunchKernelGGL(k_orth2, dim3(g), dim3(kThreads), 0, s, w.V, n, w.st, w.T, w.cin, w.c32);
            if ((rc = sqd_sigma_impl(ctx, sp, w.cin, w.sout, prec, SQD_TERM_ALL, o->ab_path,
                                     prec == SQD_FP32 ? w.c32 : nullptr, skip)))
                return fail(rc);
            hipLaunchKernelGGL(k_dots, dim3(g), dim3(kThreads), 0, s, w.V, w.AV, w.sout, n, w.st, w.partial, 0);
            ++enqueued;
        }
        if (hipGetLastError() != hipSuccess) return fail(sqd_fail(ctx, SQD_E_HIP, "launch failed in Davidson loop"));
        if (hipMemcpyAsync(w.st_host, w.st, sizeof(dav_state), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(sqd_fail(ctx, SQD_E_HIP, "Davidson state read-back failed"));
        const int done = w.st_host->done;
        if (done == DONE_RUNNING) {
            if (enqueued > o->max_iter + 8) { final_done = DONE_CAP; break; }
            continue;
        }
        if (done == DONE_SWITCH) {
            // FP64 refinement: collapse onto the current Ritz vector, recompute
            // its product in FP64, rebuild G[0][0] and continue.
            fp32_iters = w.st_host->iter;
            switch_iter = w.st_host->iter;
            prec = SQD_FP64;
            hipLaunchKernelGGL(k_collapse, dim3(g), dim3(kThreads), 0, s, w.V, w.AV, n, w.st, 1, 0, w.cin, nullptr);
            hipLaunchKernelGGL(k_set_phase, dim3(1), dim3(64), 0, s, w.st, 1, DONE_RUNNING);
            if ((rc = sqd_sigma_impl(ctx, sp, w.cin, w.sout, SQD_FP64, SQD_TERM_ALL, o->ab_path, nullptr, skip)))
                return fail(rc);
            hipLaunchKernelGGL(k_dots, dim3(g), dim3(kThreads), 0, s, w.V, w.AV, w.sout, n, w.st, w.partial, 0);
            continue;
        }
        final_done = done;
        break;
    }
    // final vector
    hipLaunchKernelGGL(k_final, dim3(g), dim3(kThreads), 0, s, w.V, n, w.st, vec, w.partial, 0);
    hipLaunchKernelGGL(k_final_sign, dim3(1), dim3(64), 0, s, vec, w.st);
    hipLaunchKernelGGL(k_final_scale, dim3(g), dim3(kThreads), 0, s, vec, n, w.st);
    if (hipMemcpyAsync(w.st_host, w.st, sizeof(dav_state), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(sqd_fail(ctx, SQD_E_HIP, "Davidson final read-back failed"));
    const dav_state& h = *w.st_host;
    *energy = h.theta;
    if (rep) {
        std::memset(rep, 0, sizeof(*rep));
        rep->iterations = h.iter;
        rep->iterations_fp32 = prm.mixed ? (switch_iter >= 0 ? fp32_iters : h.iter) : 0;
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
    free_work(w);
    return final_done == DONE_CONVERGED ? SQD_OK : SQD_NOT_CONVERGED;
}
