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
//   sigma      AV[m] = H v (FP64, or FP32 off-diagonal terms in mixed mode,
//              whose FP32 phase keeps V and AV in FP32).
//   dots       G[:, m] = V^T AV[m]; last block: m += 1 and a parallel cyclic
//              Jacobi eigen-solve of G for the next (theta, y).
#include <chrono>
#include <cmath>
#include <cstring>

#include "sqd_internal.h"

#include "davidson_body.h"

namespace {

using namespace dav;

// ---- single-space launches of the device bodies (davidson_body.h)
__global__ void __launch_bounds__(kThreads) k_argmin(const double* __restrict__ d, int64_t n, double* __restrict__ partial) {
    d_argmin(d, n, partial, blockIdx.x, gridDim.x);
}
template <int MODE>
__global__ void __launch_bounds__(kThreads) k_pick_fin(const double* __restrict__ partial, int nrows, dav_state* st) {
    f_pick_fin<MODE>(partial, nrows, st);
}
template <typename VT>
__global__ void __launch_bounds__(kThreads) k_start(const double* __restrict__ guess, const double* __restrict__ noise,
                                                    int64_t n, const dav_state* st, VT* __restrict__ V0,
                                                    double* __restrict__ partial) {
    d_start<VT>(guess, noise, n, st, V0, partial, blockIdx.x, gridDim.x);
}
__global__ void __launch_bounds__(kThreads) k_norm_fin(const double* __restrict__ partial, int nrows, dav_state* st) {
    f_norm_fin(partial, nrows, st);
}
template <typename VT>
__global__ void __launch_bounds__(kThreads) k_scale_copy(VT* __restrict__ V0, int64_t n, const dav_state* st,
                                                         double* __restrict__ cin, float* __restrict__ c32) {
    d_scale_copy<VT>(V0, n, st, cin, c32, blockIdx.x, gridDim.x);
}
// dst = src and the |src|^2 partials (the FP64 refinement's first vector,
// normalised afterwards by k_norm_fin and k_scale_copy)
__global__ void __launch_bounds__(kThreads) k_copy_norm(const double* __restrict__ src, double* __restrict__ dst,
                                                        int64_t n, double* __restrict__ partial) {
    double acc[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const double v = src[i];
        dst[i] = v;
        acc[0] += v * v;
    }
    block_to_partial<1>(acc, partial, blockIdx.x, gridDim.x);
}
template <int MT, typename VT>
__global__ void __launch_bounds__(kThreads) k_residual(const VT* __restrict__ V, const VT* __restrict__ AV,
                                                       const double* __restrict__ diag, int64_t n, const dav_state* st,
                                                       double* __restrict__ T, double* __restrict__ partial) {
    d_residual<MT, VT>(V, AV, diag, n, st, T, partial, blockIdx.x, gridDim.x);
}
template <int MT>
__global__ void __launch_bounds__(kThreads) k_res_fin(const double* __restrict__ partial, int nrows, dav_state* st,
                                                      dav_params prm) {
    f_res_fin<MT>(partial, nrows, st, prm);
}
template <int MT, typename VT>
__global__ void __launch_bounds__(kThreads) k_collapse(VT* __restrict__ V, VT* __restrict__ AV, int64_t n,
                                                       const dav_state* st, int force, double* __restrict__ cin) {
    d_collapse<MT, VT>(V, AV, n, st, force, cin, blockIdx.x, gridDim.x);
}
__global__ void k_collapse_fin(dav_state* st, int force) { f_collapse_fin(st, force); }
template <int MT, typename VT>
__global__ void __launch_bounds__(kThreads) k_orth1(const VT* __restrict__ V, int64_t n, const dav_state* st,
                                                    double* __restrict__ T, double* __restrict__ partial) {
    d_orth1<MT, VT>(V, n, st, T, partial, blockIdx.x, gridDim.x);
}
template <int MT, typename VT>
__global__ void __launch_bounds__(kThreads) k_orth1_fin(const double* __restrict__ partial, int nrows, dav_state* st) {
    f_orth1_fin<MT, VT>(partial, nrows, st);
}
template <int MT, typename VT>
__global__ void __launch_bounds__(kThreads) k_orth2(VT* __restrict__ V, int64_t n, const dav_state* st,
                                                    const double* __restrict__ T, double* __restrict__ cin,
                                                    float* __restrict__ c32) {
    d_orth2<MT, VT>(V, n, st, T, cin, c32, blockIdx.x, gridDim.x);
}
template <int MT, typename VT>
__global__ void __launch_bounds__(kThreads) k_dots(const VT* __restrict__ V, VT* __restrict__ AV,
                                                   const double* __restrict__ S, int64_t n, const dav_state* st,
                                                   double* __restrict__ partial) {
    d_dots<MT, VT>(V, AV, S, n, st, partial, blockIdx.x, gridDim.x);
}
template <int MT>
__global__ void __launch_bounds__(kThreads) k_dots_fin(const double* __restrict__ partial, int nrows, dav_state* st) {
    f_dots_fin<MT>(partial, nrows, st);
}
template <int MT, typename VT>
__global__ void __launch_bounds__(kThreads) k_final(const VT* __restrict__ V, int64_t n, const dav_state* st,
                                                    double* __restrict__ out, double* __restrict__ partial) {
    d_final<MT, VT>(V, n, st, out, partial, blockIdx.x, gridDim.x);
}
__global__ void k_final_sign(const double* __restrict__ out, dav_state* st) { f_final_sign(out, st); }
__global__ void __launch_bounds__(kThreads) k_final_scale(double* __restrict__ out, int64_t n, const dav_state* st) {
    d_final_scale(out, n, st, blockIdx.x, gridDim.x);
}
__global__ void k_set_phase(dav_state* st, int phase, int done) { f_set_phase(st, phase, done); }
__global__ void __launch_bounds__(kThreads) k_xdots(const double* __restrict__ X, int nx, const double* __restrict__ V,
                                                    int vrow, int64_t n, const dav_state* st, int round,
                                                    double* __restrict__ partial) {
    d_xdots(X, nx, V, vrow, n, st, round, partial, blockIdx.x, gridDim.x);
}
__global__ void __launch_bounds__(kThreads) k_xfin(const double* __restrict__ partial, int nrows, int nx,
                                                   dav_state* st, int round) {
    f_xfin(partial, nrows, nx, st, round);
}
__global__ void __launch_bounds__(kThreads) k_xapply(const double* __restrict__ X, int nx, double* __restrict__ V,
                                                     int vrow, int64_t n, const dav_state* st, int round,
                                                     double* __restrict__ cin, float* __restrict__ c32) {
    d_xapply(X, nx, V, vrow, n, st, round, cin, c32, blockIdx.x, gridDim.x);
}

// Project V0 (vrow 0) or the appended row V[m] (vrow 1) against the nx locked
// vectors X and normalise it; cin (and c32 in the FP32 phase) receive it.
void lock_project(int g, hipStream_t s, const double* X, int nx, double* V, int vrow, int64_t n, dav_state* st,
                  double* cin, float* c32, double* part) {
    for (int round = 0; round < 2; ++round) {
        hipLaunchKernelGGL(k_xdots, dim3(g), dim3(kThreads), 0, s, X, nx, V, vrow, n, st, round, part);
        hipLaunchKernelGGL(k_xfin, dim3(1), dim3(kThreads), 0, s, part, g, nx, st, round);
        hipLaunchKernelGGL(k_xapply, dim3(g), dim3(kThreads), 0, s, X, nx, V, vrow, n, st, round, cin, c32);
    }
}

inline int grid_for(int64_t n) {
    int64_t b = (n + kThreads - 1) / kThreads;
    if (b > kMaxBlocks) b = kMaxBlocks;
    if (b < 1) b = 1;
    return (int)b;
}

// Launch helpers templated on the compile-time basis bound and the storage
// type of the basis V and its products AV (FP64; FP32 in the FP32 phase of a
// mixed solve, where FP32 products carry no more digits and the passes over
// the basis move half the bytes).
template <int MT, typename VT>
struct dav_launch {
    static void residual(int g, hipStream_t s, const VT* V, const VT* AV, const double* d, int64_t n, dav_state* st,
                         dav_params p, double* T, double* part) {
        hipLaunchKernelGGL((k_residual<MT, VT>), dim3(g), dim3(kThreads), 0, s, V, AV, d, n, st, T, part);
        hipLaunchKernelGGL((k_res_fin<MT>), dim3(1), dim3(kThreads), 0, s, part, g, st, p);
    }
    static void collapse(int g, hipStream_t s, VT* V, VT* AV, int64_t n, dav_state* st, int force, double* cin) {
        hipLaunchKernelGGL((k_collapse<MT, VT>), dim3(g), dim3(kThreads), 0, s, V, AV, n, st, force, cin);
        hipLaunchKernelGGL(k_collapse_fin, dim3(1), dim3(64), 0, s, st, force);
    }
    static void orth1(int g, hipStream_t s, const VT* V, int64_t n, dav_state* st, double* T, double* part) {
        hipLaunchKernelGGL((k_orth1<MT, VT>), dim3(g), dim3(kThreads), 0, s, V, n, st, T, part);
        hipLaunchKernelGGL((k_orth1_fin<MT, VT>), dim3(1), dim3(kThreads), 0, s, part, g, st);
    }
    static void orth2(int g, hipStream_t s, VT* V, int64_t n, dav_state* st, const double* T, double* cin, float* c32) {
        hipLaunchKernelGGL((k_orth2<MT, VT>), dim3(g), dim3(kThreads), 0, s, V, n, st, T, cin, c32);
    }
    static void dots(int g, hipStream_t s, const VT* V, VT* AV, const double* S, int64_t n, dav_state* st,
                     double* part) {
        hipLaunchKernelGGL((k_dots<MT, VT>), dim3(g), dim3(kThreads), 0, s, V, AV, S, n, st, part);
        hipLaunchKernelGGL((k_dots_fin<MT>), dim3(1), dim3(kThreads), 0, s, part, g, st);
    }
    static void final_(int g, hipStream_t s, const VT* V, int64_t n, dav_state* st, double* out, double* part) {
        hipLaunchKernelGGL((k_final<MT, VT>), dim3(g), dim3(kThreads), 0, s, V, n, st, out, part);
        hipLaunchKernelGGL((k_pick_fin<1>), dim3(1), dim3(kThreads), 0, s, part, g, st);
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

// One solve; with nx > 0 locked vectors X (orthonormal, nx x n) every basis
// vector is kept orthogonal to them, giving the lowest root of their
// orthogonal complement.
template <int MT>
static int davidson_run(sqd_ctx* ctx, sqd_space* sp, const sqd_davidson_opts* o, double* energy, double* vec,
                        sqd_report* rep, dav_work& w, const dav_params& prm, const double* X, int nx) {
    using L = dav_launch<MT, double>;
    using L32 = dav_launch<MT, float>;
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
    if (!o->guess_dev) {
        hipLaunchKernelGGL(k_argmin, dim3(g), dim3(kThreads), 0, s, diag, n, w.partial);
        hipLaunchKernelGGL((k_pick_fin<0>), dim3(1), dim3(kThreads), 0, s, w.partial, g, w.st);
    }
    // the FP32 phase of a mixed solve keeps its basis in FP32, in the first
    // halves of the FP64 buffers (not with locked roots, whose projections
    // work on FP64 rows)
    bool basis32 = prm.mixed && nx == 0;
    float* V32 = reinterpret_cast<float*>(w.V);
    float* AV32 = reinterpret_cast<float*>(w.AV);
    if (basis32) {
        hipLaunchKernelGGL(k_start<float>, dim3(g), dim3(kThreads), 0, s, o->guess_dev, o->guess_noise_dev, n, w.st,
                           V32, w.partial);
        hipLaunchKernelGGL(k_norm_fin, dim3(1), dim3(kThreads), 0, s, w.partial, g, w.st);
        hipLaunchKernelGGL(k_scale_copy<float>, dim3(g), dim3(kThreads), 0, s, V32, n, w.st, w.cin, w.c32);
    } else {
        hipLaunchKernelGGL(k_start<double>, dim3(g), dim3(kThreads), 0, s, o->guess_dev, o->guess_noise_dev, n, w.st,
                           w.V, w.partial);
        if (nx > 0) {
            lock_project(g, s, X, nx, w.V, 0, n, w.st, w.cin, w.c32, w.partial);
        } else {
            hipLaunchKernelGGL(k_norm_fin, dim3(1), dim3(kThreads), 0, s, w.partial, g, w.st);
            hipLaunchKernelGGL(k_scale_copy<double>, dim3(g), dim3(kThreads), 0, s, w.V, n, w.st, w.cin, w.c32);
        }
    }
    const int* skip = &w.st->done;
    int prec = prm.mixed ? SQD_FP32 : SQD_FP64;
    // the product: matrix-free (FP64, or FP32 off-diagonal terms from the
    // FP32 copy of the input), or the stored H (FP64)
    auto product = [&](int p) -> int {
        if (o->product == SQD_PRODUCT_STORED) return sqd_spmv_impl(ctx, sp, w.cin, w.sout, skip);
        return sqd_sigma_impl(ctx, sp, w.cin, w.sout, p, SQD_TERM_ALL, o->ab_path,
                              p == SQD_FP32 ? w.c32 : nullptr, skip);
    };
    if ((rc = product(prec))) return rc;
    if (basis32) L32::dots(g, s, V32, AV32, w.sout, n, w.st, w.partial);
    else L::dots(g, s, w.V, w.AV, w.sout, n, w.st, w.partial);
    if (hipGetLastError() != hipSuccess) return sqd_fail(ctx, SQD_E_HIP, "launch failed in Davidson start");

    int enqueued = 0;
    int switch_iter = -1;
    int final_done = DONE_CAP;
    while (true) {
        // enqueue check_every iterations, then poll the device flag; kernels of
        // iterations past the end return at once
        for (int k = 0; k < o->check_every; ++k) {
            if (basis32) {
                L32::residual(g, s, V32, AV32, diag, n, w.st, prm, w.T, w.partial);
                L32::collapse(g, s, V32, AV32, n, w.st, 0, nullptr);
                L32::orth1(g, s, V32, n, w.st, w.T, w.partial);
                L32::orth2(g, s, V32, n, w.st, w.T, w.cin, w.c32);
                if ((rc = product(prec))) return rc;
                L32::dots(g, s, V32, AV32, w.sout, n, w.st, w.partial);
            } else {
                L::residual(g, s, w.V, w.AV, diag, n, w.st, prm, w.T, w.partial);
                L::collapse(g, s, w.V, w.AV, n, w.st, 0, nullptr);
                L::orth1(g, s, w.V, n, w.st, w.T, w.partial);
                L::orth2(g, s, w.V, n, w.st, w.T, w.cin, prec == SQD_FP32 ? w.c32 : nullptr);
                if (nx > 0)
                    lock_project(g, s, X, nx, w.V, 1, n, w.st, w.cin, prec == SQD_FP32 ? w.c32 : nullptr, w.partial);
                if ((rc = product(prec))) return rc;
                L::dots(g, s, w.V, w.AV, w.sout, n, w.st, w.partial);
            }
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
            if (basis32) {
                // x = V y from the FP32 basis into cin, then V[0] = x / |x|
                // in FP64 (the FP32 rows are not orthonormal to FP64 accuracy)
                L32::collapse(g, s, V32, AV32, n, w.st, 1, w.cin);
                hipLaunchKernelGGL(k_copy_norm, dim3(g), dim3(kThreads), 0, s, w.cin, w.V, n, w.partial);
                hipLaunchKernelGGL(k_norm_fin, dim3(1), dim3(kThreads), 0, s, w.partial, g, w.st);
                hipLaunchKernelGGL(k_scale_copy<double>, dim3(g), dim3(kThreads), 0, s, w.V, n, w.st, w.cin,
                                   nullptr);
                basis32 = false;
            } else {
                L::collapse(g, s, w.V, w.AV, n, w.st, 1, w.cin);
            }
            hipLaunchKernelGGL(k_set_phase, dim3(1), dim3(64), 0, s, w.st, 1, DONE_RUNNING);
            if ((rc = product(SQD_FP64))) return rc;
            L::dots(g, s, w.V, w.AV, w.sout, n, w.st, w.partial);
            continue;
        }
        final_done = done;
        break;
    }
    if (basis32) L32::final_(g, s, V32, n, w.st, vec, w.partial);
    else L::final_(g, s, w.V, n, w.st, vec, w.partial);
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
                      sqd_report* rep, int nroots_) {
    const int64_t n = sp->dim;
    const int mmax = o->m_max;
    dav_work w;
    int rc = SQD_OK;
    // The vectors live in an arena the context keeps (grown on demand) across
    // calls, so repeated solves (finite differences, the sampling loop) do not
    // allocate the m_max x dim basis every time.
    std::pair<void**, size_t> req[] = {
        {(void**)&w.V, sizeof(double) * (size_t)n * mmax},
        {(void**)&w.AV, sizeof(double) * (size_t)n * mmax},
        {(void**)&w.T, sizeof(double) * n},
        {(void**)&w.cin, sizeof(double) * n},
        {(void**)&w.sout, sizeof(double) * n},
        {(void**)&w.c32, o->mode == SQD_DAV_MIXED ? sizeof(float) * n : 0},
        {(void**)&w.partial, sizeof(double) * kMaxBlocks * kPstride},
        {(void**)&w.st, sizeof(dav_state)},
    };
    size_t total = 0;
    for (auto& r : req) total += (r.second + 255) & ~(size_t)255;
    if (ctx->dav_arena_bytes < total) {
        if (ctx->dav_arena) {
            (void)hipStreamSynchronize(ctx->stream);
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
            *r.first = r.second ? base + off : nullptr;
            off += (r.second + 255) & ~(size_t)255;
        }
    }
    if (!ctx->dav_state_host &&
        hipHostMalloc((void**)&ctx->dav_state_host, sizeof(dav_state), hipHostMallocDefault) != hipSuccess) {
        ctx->dav_state_host = nullptr;
        return sqd_fail(ctx, SQD_E_OOM, "pinned host allocation failed");
    }
    w.st_host = static_cast<dav_state*>(ctx->dav_state_host);
    dav_params prm;
    prm.tol = o->tol;
    prm.switch_tol = o->switch_tol;
    prm.max_iter = o->max_iter;
    prm.m_max = mmax;
    prm.mixed = o->mode == SQD_DAV_MIXED;
    const int nroots = nroots_ > 0 ? nroots_ : 1;
    for (int j = 0; j < nroots; ++j) {
        double* vj = vec + (int64_t)j * n;
        sqd_report* rj = rep ? rep + j : nullptr;
        int rj_rc;
        if (mmax <= 8) rj_rc = davidson_run<8>(ctx, sp, o, energy + j, vj, rj, w, prm, vec, j);
        else if (mmax <= 16) rj_rc = davidson_run<16>(ctx, sp, o, energy + j, vj, rj, w, prm, vec, j);
        else if (mmax <= 24) rj_rc = davidson_run<24>(ctx, sp, o, energy + j, vj, rj, w, prm, vec, j);
        else rj_rc = davidson_run<32>(ctx, sp, o, energy + j, vj, rj, w, prm, vec, j);
        if (rj_rc < 0) return rj_rc;
        if (rj_rc != SQD_OK) rc = rj_rc;
    }
    return rc;
}
