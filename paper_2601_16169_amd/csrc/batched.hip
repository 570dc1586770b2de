// Many independent SQD spaces solved together (the batches of uneven string
// counts that the sampling loop of Sec. I produces; load balance across task
// groups is the paper's scaling limiter, Sec. VI).
//
// * Every sigma term of every space runs in ONE launch: the work units are
//   (space, tile) pairs -- row blocks for the same-spin kernel, pair chunks for
//   the alpha-beta kernel -- ordered longest-first and pulled by persistent
//   workgroups from an atomic queue; the cheaper uniform passes (transposes,
//   gathers, vector kernels) stride over their unit lists statically.
// * The Davidson state of each space stays on the device; the vector kernels
//   of all spaces run in one launch each and the small per-space work runs in
//   one workgroup per space.  A space that has converged (or reached its cap
//   or its precision switch) skips its units.
// * One whole iteration of all spaces (FP32 and FP64 variants) is captured once
//   as a hipGraph and replayed; the host polls a device count of running
//   spaces every check_every replays.
// The kernels are the same device bodies as the single-space path
// (sigma_body.h, davidson_body.h).
#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>

#include "davidson_body.h"
#include "sigma_body.h"

using namespace dav;

namespace {

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Per-space descriptor (device copy).
struct bdesc {
    int64_t n, na, nb;
    int nblk;        // vector-kernel blocks of this space
    int part0;       // first partial row
    int ntx, nty;    // transpose tiles of C (na x nb): x over nb, y over na
    double* V;
    double* AV;
    double* T;
    double* cin;
    double* sout;
    float* c32;
    const double* diag;
    dav_state* st;
    double* out;
    const double* noise;
    // sigma scratch
    double* Ct;
    double* Yt;
    double* Y64;
    float* Ct32;
    float* Yt32;
    float* S32;
    float* Y32;
    const int* a_off;
    const int* a_order;   // alpha rows, heaviest first (gather order)
    const int* abs_src;   // source string of each alpha-beta chunk (source-grouped spaces)
    ss_args<double> bb64, aa64;
    ss_args<float> bb32, aa32;
    abg_args<double> ab64;
    abg_args<float> ab32;
};

__device__ __forceinline__ const ss_args<double>& ssa(const bdesc& d, int which, double) { return which ? d.aa64 : d.bb64; }
__device__ __forceinline__ const ss_args<float>& ssa(const bdesc& d, int which, float) { return which ? d.aa32 : d.bb32; }
__device__ __forceinline__ const abg_args<double>& aba(const bdesc& d, double) { return d.ab64; }
__device__ __forceinline__ const abg_args<float>& aba(const bdesc& d, float) { return d.ab32; }

__global__ void kb_reset(int* counters, int n) {
    if (threadIdx.x < n) counters[threadIdx.x] = 0;
}

// Pull the next unit index from the queue (whole block).
__device__ __forceinline__ int next_unit(int* counter) {
    __shared__ int u_sh;
    if (threadIdx.x == 0) u_sh = atomicAdd(counter, 1);
    __syncthreads();
    const int u = u_sh;
    __syncthreads();
    return u;
}

// ---------------------------------------------------------------- sigma terms
template <typename T, int R>
__global__ void __launch_bounds__(1024) kb_same_spin(const bdesc* __restrict__ D, int which, const int2* __restrict__ units,
                                                     int nunits, int* counter, const T* __restrict__ jk, int norb) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    while (true) {
        const int u = next_unit(counter);
        if (u >= nunits) break;
        const bdesc& d = D[units[u].x];
        if (d.st->done) continue;
        ss_block<T, R>(ssa(d, which, T()), jk, norb, units[u].y, lds_raw);
        __syncthreads();
    }
}

template <typename T, int G>
__global__ void __launch_bounds__(1024) kb_ab_grouped(const bdesc* __restrict__ D, const int2* __restrict__ units,
                                                      int nunits, int* counter, const T* __restrict__ V, int norb) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    while (true) {
        const int u = next_unit(counter);
        if (u >= nunits) break;
        const bdesc& d = D[units[u].x];
        if (d.st->done) continue;
        abg_block<T, G>(aba(d, T()), V, norb, units[u].y, lds_raw);
        __syncthreads();
    }
}

// The spaces of the longest rows with their alpha singles grouped by source
// string (abs_block; the chunks in ab64/ab32.grp, their sources in abs_src).
template <typename T, int GS>
__global__ void __launch_bounds__(1024) kb_ab_srcgrouped(const bdesc* __restrict__ D, const int2* __restrict__ units,
                                                         int nunits, int* counter, const T* __restrict__ V, int norb) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    while (true) {
        const int u = next_unit(counter);
        if (u >= nunits) break;
        const bdesc& d = D[units[u].x];
        if (d.st->done) continue;
        abs_block<T, GS>(aba(d, T()), d.abs_src, V, norb, units[u].y, lds_raw);
        __syncthreads();
    }
}

// which 0: C -> C^T (rows na, cols nb); which 1: Y^T -> sigma (rows nb, cols na)
template <typename T>
__global__ void __launch_bounds__(256) kb_transpose(const bdesc* __restrict__ D, int which, const int2* __restrict__ units,
                                                    int nunits) {
    __shared__ T tile[64][65];
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const bdesc& d = D[units[u].x];
        if (d.st->done) continue;
        const int t = units[u].y;
        const T* in;
        T* out;
        int64_t rows, cols, ty, tx;
        if (which == 0) {
            in = (const T*)(sizeof(T) == 8 ? (const void*)d.cin : (const void*)d.c32);
            out = (T*)(sizeof(T) == 8 ? (void*)d.Ct : (void*)d.Ct32);
            rows = d.na; cols = d.nb; ty = t / d.ntx; tx = t % d.ntx;
        } else {
            in = (const T*)(sizeof(T) == 8 ? (const void*)d.Yt : (const void*)d.Yt32);
            out = (T*)(sizeof(T) == 8 ? (void*)d.sout : (void*)d.S32);
            rows = d.nb; cols = d.na; ty = t % d.ntx; tx = t / d.ntx;
        }
        transpose_tile<T, T, false>(in, out, rows, cols, ty, tx, tile);
        __syncthreads();
    }
}

// One unit per (space, alpha row); STAGED: rows assembled in LDS (gather_row).
template <typename T, bool STAGED>
__global__ void __launch_bounds__(256) kb_gather(const bdesc* __restrict__ D, const int2* __restrict__ units, int nunits) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* row = STAGED ? reinterpret_cast<T*>(lds_raw) : nullptr;
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const bdesc& d = D[units[u].x];
        if (d.st->done) continue;
        const T* Y = (const T*)(sizeof(T) == 8 ? (const void*)d.Y64 : (const void*)d.Y32);
        T* S = (T*)(sizeof(T) == 8 ? (void*)d.sout : (void*)d.S32);
        gather_row<T>(Y, S, d.nb, d.ab64.ldy, d.ab64.bperm, d.a_off, d.a_order[units[u].y], row);
    }
}

// sout = diag * cin + (double) S32  (FP32 path)
__global__ void __launch_bounds__(256) kb_combine(const bdesc* __restrict__ D, const int2* __restrict__ units, int nunits) {
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const bdesc& d = D[units[u].x];
        if (d.st->done) continue;
        for (int64_t i = (int64_t)units[u].y * 256 + threadIdx.x; i < d.n; i += (int64_t)d.nblk * 256)
            d.sout[i] = d.diag[i] * d.cin[i] + (double)d.S32[i];
    }
}

// ---------------------------------------------------------------- Davidson
// VT: storage of the basis V and its products AV (float in the FP32 phase of a
// mixed batch, held in the first halves of the FP64 buffers)
template <int MT, typename VT>
__global__ void __launch_bounds__(kThreads) kb_residual(const bdesc* __restrict__ D, const int2* __restrict__ units,
                                                        int nunits, double* __restrict__ partial) {
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const bdesc& d = D[units[u].x];
        d_residual<MT, VT>(reinterpret_cast<const VT*>(d.V), reinterpret_cast<const VT*>(d.AV), d.diag, d.n, d.st, d.T,
                           partial + (size_t)d.part0 * kPstride, units[u].y, d.nblk);
        __syncthreads();
    }
}
template <int MT>
__global__ void __launch_bounds__(kThreads) kb_res_fin(const bdesc* __restrict__ D, double* __restrict__ partial,
                                                       dav_params prm) {
    const bdesc& d = D[blockIdx.x];
    f_res_fin<MT>(partial + (size_t)d.part0 * kPstride, d.nblk, d.st, prm);
}
// force: 0 pending restarts; 1 spaces at their precision switch
template <int MT, typename VT>
__global__ void __launch_bounds__(kThreads) kb_collapse(const bdesc* __restrict__ D, const int2* __restrict__ units,
                                                        int nunits, int force) {
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const bdesc& d = D[units[u].x];
        if (force && d.st->done != DONE_SWITCH) continue;
        d_collapse<MT, VT>(reinterpret_cast<VT*>(d.V), reinterpret_cast<VT*>(d.AV), d.n, d.st, force,
                           force ? d.cin : nullptr, units[u].y, d.nblk);
    }
}
// Spaces at their switch: V[0] = cin (the Ritz vector formed from an FP32
// basis) and its |.|^2 partials, normalised by kb_norm_fin / kb_scale_copy.
__global__ void __launch_bounds__(kThreads) kb_copy_norm(const bdesc* __restrict__ D, const int2* __restrict__ units,
                                                         int nunits, double* __restrict__ partial) {
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const bdesc& d = D[units[u].x];
        if (d.st->done != DONE_SWITCH) continue;
        double acc[1] = {0.0};
        for (int64_t i = (int64_t)units[u].y * kThreads + threadIdx.x; i < d.n; i += (int64_t)d.nblk * kThreads) {
            const double v = d.cin[i];
            d.V[i] = v;
            acc[0] += v * v;
        }
        block_to_partial<1>(acc, partial + (size_t)d.part0 * kPstride, units[u].y, d.nblk);
        __syncthreads();
    }
}
__global__ void kb_collapse_fin(const bdesc* __restrict__ D, int force) {
    const bdesc& d = D[blockIdx.x];
    if (force) {
        if (d.st->done != DONE_SWITCH) return;
        f_collapse_fin(d.st, 1);
        f_set_phase(d.st, 1, DONE_RUNNING);
        return;
    }
    f_collapse_fin(d.st, 0);
}
template <int MT, typename VT>
__global__ void __launch_bounds__(kThreads) kb_orth1(const bdesc* __restrict__ D, const int2* __restrict__ units,
                                                     int nunits, double* __restrict__ partial) {
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const bdesc& d = D[units[u].x];
        d_orth1<MT, VT>(reinterpret_cast<const VT*>(d.V), d.n, d.st, d.T, partial + (size_t)d.part0 * kPstride,
                        units[u].y, d.nblk);
        __syncthreads();
    }
}
template <int MT, typename VT>
__global__ void __launch_bounds__(kThreads) kb_orth1_fin(const bdesc* __restrict__ D, double* __restrict__ partial) {
    const bdesc& d = D[blockIdx.x];
    f_orth1_fin<MT, VT>(partial + (size_t)d.part0 * kPstride, d.nblk, d.st);
}
template <int MT, typename VT>
__global__ void __launch_bounds__(kThreads) kb_orth2(const bdesc* __restrict__ D, const int2* __restrict__ units,
                                                     int nunits, int lowp) {
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const bdesc& d = D[units[u].x];
        d_orth2<MT, VT>(reinterpret_cast<VT*>(d.V), d.n, d.st, d.T, d.cin, lowp ? d.c32 : nullptr, units[u].y, d.nblk);
    }
}
template <int MT, typename VT>
__global__ void __launch_bounds__(kThreads) kb_dots(const bdesc* __restrict__ D, const int2* __restrict__ units,
                                                    int nunits, double* __restrict__ partial) {
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const bdesc& d = D[units[u].x];
        d_dots<MT, VT>(reinterpret_cast<const VT*>(d.V), reinterpret_cast<VT*>(d.AV), d.sout, d.n, d.st,
                       partial + (size_t)d.part0 * kPstride, units[u].y, d.nblk);
        __syncthreads();
    }
}
template <int MT>
__global__ void __launch_bounds__(kThreads) kb_dots_fin(const bdesc* __restrict__ D, double* __restrict__ partial) {
    const bdesc& d = D[blockIdx.x];
    f_dots_fin<MT>(partial + (size_t)d.part0 * kPstride, d.nblk, d.st);
}
__global__ void __launch_bounds__(kThreads) kb_argmin(const bdesc* __restrict__ D, const int2* __restrict__ units,
                                                      int nunits, double* __restrict__ partial) {
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const bdesc& d = D[units[u].x];
        d_argmin(d.diag, d.n, partial + (size_t)d.part0 * kPstride, units[u].y, d.nblk);
        __syncthreads();
    }
}
template <int MODE>
__global__ void __launch_bounds__(kThreads) kb_pick_fin(const bdesc* __restrict__ D, double* __restrict__ partial) {
    const bdesc& d = D[blockIdx.x];
    f_pick_fin<MODE>(partial + (size_t)d.part0 * kPstride, d.nblk, d.st);
}
// Start vector of space b: e_kmin plus start_noise of counter stream b;
// |V0|^2 partials.
template <typename VT>
__global__ void __launch_bounds__(kThreads) kb_start(const bdesc* __restrict__ D, const int2* __restrict__ units,
                                                     int nunits, double* __restrict__ partial) {
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const int b = units[u].x;
        const bdesc& d = D[b];
        const int64_t kmin = d.st->kmin;
        double acc[1] = {0.0};
        for (int64_t i = (int64_t)units[u].y * kThreads + threadIdx.x; i < d.n; i += (int64_t)d.nblk * kThreads) {
            const double v = (i == kmin ? 1.0 : 0.0) + start_noise((uint64_t)b, i, d.n);
            reinterpret_cast<VT*>(d.V)[i] = (VT)v;
            acc[0] += v * v;
        }
        block_to_partial<1>(acc, partial + (size_t)d.part0 * kPstride, units[u].y, d.nblk);
        __syncthreads();
    }
}
// sel 1: only the spaces at their precision switch
__global__ void __launch_bounds__(kThreads) kb_norm_fin(const bdesc* __restrict__ D, double* __restrict__ partial,
                                                        int sel) {
    const bdesc& d = D[blockIdx.x];
    if (sel && d.st->done != DONE_SWITCH) return;
    f_norm_fin(partial + (size_t)d.part0 * kPstride, d.nblk, d.st);
}
template <typename VT>
__global__ void __launch_bounds__(kThreads) kb_scale_copy(const bdesc* __restrict__ D, const int2* __restrict__ units,
                                                          int nunits, int lowp, int sel) {
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const bdesc& d = D[units[u].x];
        if (sel && d.st->done != DONE_SWITCH) continue;
        d_scale_copy<VT>(reinterpret_cast<VT*>(d.V), d.n, d.st, d.cin, lowp ? d.c32 : nullptr, units[u].y, d.nblk);
    }
}
// b32: spaces still in the FP32 phase (stopped by their cap) hold an FP32 basis
template <int MT>
__global__ void __launch_bounds__(kThreads) kb_final(const bdesc* __restrict__ D, const int2* __restrict__ units,
                                                     int nunits, double* __restrict__ partial, int b32) {
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const bdesc& d = D[units[u].x];
        if (b32 && d.st->phase == 0)
            d_final<MT, float>(reinterpret_cast<const float*>(d.V), d.n, d.st, d.out,
                               partial + (size_t)d.part0 * kPstride, units[u].y, d.nblk);
        else
            d_final<MT, double>(d.V, d.n, d.st, d.out, partial + (size_t)d.part0 * kPstride, units[u].y, d.nblk);
        __syncthreads();
    }
}
__global__ void kb_final_sign(const bdesc* __restrict__ D) {
    const bdesc& d = D[blockIdx.x];
    f_final_sign(d.out, d.st);
}
__global__ void __launch_bounds__(kThreads) kb_final_scale(const bdesc* __restrict__ D, const int2* __restrict__ units,
                                                           int nunits) {
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const bdesc& d = D[units[u].x];
        d_final_scale(d.out, d.n, d.st, units[u].y, d.nblk);
    }
}
// number of spaces still running -> *count
__global__ void kb_count_running(const bdesc* __restrict__ D, int nspace, int* count) {
    __shared__ int c;
    if (threadIdx.x == 0) c = 0;
    __syncthreads();
    for (int b = threadIdx.x; b < nspace; b += blockDim.x)
        if (D[b].st->done == DONE_RUNNING) atomicAdd(&c, 1);
    __syncthreads();
    if (threadIdx.x == 0) *count = c;
}

// ---------------------------------------------------------------- host plan
struct unit_list {
    int2* dev = nullptr;
    int n = 0;
};

struct batch_plan {
    int nspace = 0;
    std::vector<bdesc> host;
    bdesc* D = nullptr;
    unit_list vec, tr, ss_bb, ss_aa, abg, abg2, gath;
    int* counters = nullptr;
    int* count_dev = nullptr;
    int* count_host = nullptr;
    double* partial = nullptr;
    dav_state* states = nullptr;
    int R = 0, G = 0, Rf = 0;
    int G2 = 0;                // pair group of the spaces with shorter rows (0: one class)
    int GS = 0;                // the first class grouped by source string, GS singles per chunk (0: by pair)
    size_t lds_abs64 = 0, lds_abs32 = 0;
    size_t lds_ss64 = 0, lds_ss32 = 0, lds_ab64 = 0, lds_ab32 = 0, lds_ab64_2 = 0, lds_ab32_2 = 0;
    size_t gather_lds64 = 0;   // FP64 row bytes of the staged gather (0: in-place gather)
    int grid_persist = 0;
};

template <typename F>
void lds_attr(F f, size_t bytes) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(f), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

constexpr int kGridCap = 4096;

// The alpha-beta chunks of the second class (spaces whose rows allow a
// larger pair group than the longest rows of the batch).
template <typename T>
void launch_ab_class2(batch_plan& p, hipStream_t s, dim3 gp, int nw_ab, const T* V, int norb, int* counter) {
    if (!p.G2 || p.abg2.n == 0) return;
    const size_t lds = sizeof(T) == 8 ? p.lds_ab64_2 : p.lds_ab32_2;
#define SQD_AB2_LAUNCH(GG)                                                                                       \
    case GG:                                                                                                     \
        hipLaunchKernelGGL((kb_ab_grouped<T, GG>), gp, dim3(64 * nw_ab), lds, s, p.D, p.abg2.dev, p.abg2.n, counter, \
                           V, norb);                                                                             \
        break;
    switch (p.G2) {
        SQD_AB2_LAUNCH(2)
        SQD_AB2_LAUNCH(4)
        SQD_AB2_LAUNCH(8)
    }
#undef SQD_AB2_LAUNCH
}

// The first class grouped by source string.
template <typename T>
void launch_ab_src(batch_plan& p, hipStream_t s, dim3 gp, int nw_ab, const T* V, int norb, int* counter) {
    const size_t lds = sizeof(T) == 8 ? p.lds_abs64 : p.lds_abs32;
#define SQD_ABS_LAUNCH(GG)                                                                                      \
    case GG:                                                                                                    \
        hipLaunchKernelGGL((kb_ab_srcgrouped<T, GG>), gp, dim3(64 * nw_ab), lds, s, p.D, p.abg.dev, p.abg.n,      \
                           counter, V, norb);                                                                   \
        break;
    switch (p.GS) {
        SQD_ABS_LAUNCH(2)
        SQD_ABS_LAUNCH(3)
        SQD_ABS_LAUNCH(4)
        SQD_ABS_LAUNCH(8)
    }
#undef SQD_ABS_LAUNCH
}

// Launch the sigma of every running space (precision prec) into its sout.
template <int R, int G, int RF>
int batched_sigma(sqd_ctx* ctx, batch_plan& p, hipStream_t s, int prec, int nw_ss, int nw_ab) {
    const int norb = ctx->norb;
    const dim3 gp(p.grid_persist);
    hipLaunchKernelGGL(kb_reset, dim3(1), dim3(64), 0, s, p.counters, 8);
    auto sgrid = [&](int n) { return dim3((unsigned)std::max(1, std::min(n, kGridCap))); };
    if (prec == SQD_FP64) {
        hipLaunchKernelGGL((kb_transpose<double>), sgrid(p.tr.n), dim3(256), 0, s, p.D, 0, p.tr.dev, p.tr.n);
        hipLaunchKernelGGL((kb_same_spin<double, R>), gp, dim3(64 * nw_ss), p.lds_ss64, s, p.D, 1, p.ss_aa.dev, p.ss_aa.n,
                           p.counters + 0, ctx->jk64, norb);
        hipLaunchKernelGGL((kb_transpose<double>), sgrid(p.tr.n), dim3(256), 0, s, p.D, 1, p.tr.dev, p.tr.n);
        hipLaunchKernelGGL((kb_same_spin<double, R>), gp, dim3(64 * nw_ss), p.lds_ss64, s, p.D, 0, p.ss_bb.dev, p.ss_bb.n,
                           p.counters + 1, ctx->jk64, norb);
        if (p.GS) launch_ab_src<double>(p, s, gp, nw_ab, ctx->eri, norb, p.counters + 2);
        else
            hipLaunchKernelGGL((kb_ab_grouped<double, G>), gp, dim3(64 * nw_ab), p.lds_ab64, s, p.D, p.abg.dev,
                               p.abg.n, p.counters + 2, ctx->eri, norb);
        launch_ab_class2<double>(p, s, gp, nw_ab, ctx->eri, norb, p.counters + 6);
        if (p.gather_lds64)
            hipLaunchKernelGGL((kb_gather<double, true>), sgrid(p.gath.n), dim3(256), p.gather_lds64, s, p.D,
                               p.gath.dev, p.gath.n);
        else
            hipLaunchKernelGGL((kb_gather<double, false>), sgrid(p.gath.n), dim3(256), 0, s, p.D, p.gath.dev,
                               p.gath.n);
    } else {
        hipLaunchKernelGGL((kb_transpose<float>), sgrid(p.tr.n), dim3(256), 0, s, p.D, 0, p.tr.dev, p.tr.n);
        hipLaunchKernelGGL((kb_same_spin<float, RF>), gp, dim3(64 * nw_ss), p.lds_ss32, s, p.D, 1, p.ss_aa.dev,
                           p.ss_aa.n, p.counters + 3, ctx->jk32, norb);
        hipLaunchKernelGGL((kb_transpose<float>), sgrid(p.tr.n), dim3(256), 0, s, p.D, 1, p.tr.dev, p.tr.n);
        hipLaunchKernelGGL((kb_same_spin<float, RF>), gp, dim3(64 * nw_ss), p.lds_ss32, s, p.D, 0, p.ss_bb.dev,
                           p.ss_bb.n, p.counters + 4, ctx->jk32, norb);
        if (p.GS) launch_ab_src<float>(p, s, gp, nw_ab, ctx->eri32, norb, p.counters + 5);
        else
            hipLaunchKernelGGL((kb_ab_grouped<float, G>), gp, dim3(64 * nw_ab), p.lds_ab32, s, p.D, p.abg.dev,
                               p.abg.n, p.counters + 5, ctx->eri32, norb);
        launch_ab_class2<float>(p, s, gp, nw_ab, ctx->eri32, norb, p.counters + 7);
        if (p.gather_lds64)
            hipLaunchKernelGGL((kb_gather<float, true>), sgrid(p.gath.n), dim3(256), p.gather_lds64 / 2, s, p.D,
                               p.gath.dev, p.gath.n);
        else
            hipLaunchKernelGGL((kb_gather<float, false>), sgrid(p.gath.n), dim3(256), 0, s, p.D, p.gath.dev,
                               p.gath.n);
        hipLaunchKernelGGL(kb_combine, sgrid(p.vec.n), dim3(256), 0, s, p.D, p.vec.dev, p.vec.n);
    }
    return SQD_OK;
}

template <int MT, int R, int G, int RF>
int batched_run(sqd_ctx* ctx, batch_plan& p, const sqd_davidson_opts* o, double* energies, sqd_report* reps,
                hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const bool mixed = o->mode == SQD_DAV_MIXED;
    dav_params prm;
    prm.tol = o->tol;
    prm.switch_tol = o->switch_tol;
    prm.max_iter = o->max_iter;
    prm.m_max = o->m_max;
    prm.mixed = mixed;
    const int nw_ss = ctx->tune[SQD_TUNE_SS_WAVES] ? ctx->tune[SQD_TUNE_SS_WAVES]
                                                   : ((R == 8 || p.lds_ss64 > (size_t)ctx->max_lds / 2) ? 16 : 8);
    // measured on MI355X (the batched tuner's choice on 64 spaces of 200-3000 strings)
    const int nw_ab = ctx->tune[SQD_TUNE_AB_WAVES] ? ctx->tune[SQD_TUNE_AB_WAVES] : 8;
    lds_attr(kb_same_spin<double, R>, p.lds_ss64);
    lds_attr(kb_same_spin<float, RF>, p.lds_ss32);
    lds_attr(kb_ab_grouped<double, G>, p.lds_ab64);
    lds_attr(kb_ab_grouped<float, G>, p.lds_ab32);
    switch (p.GS) {
        case 2: lds_attr(kb_ab_srcgrouped<double, 2>, p.lds_abs64); lds_attr(kb_ab_srcgrouped<float, 2>, p.lds_abs32); break;
        case 3: lds_attr(kb_ab_srcgrouped<double, 3>, p.lds_abs64); lds_attr(kb_ab_srcgrouped<float, 3>, p.lds_abs32); break;
        case 4: lds_attr(kb_ab_srcgrouped<double, 4>, p.lds_abs64); lds_attr(kb_ab_srcgrouped<float, 4>, p.lds_abs32); break;
        case 8: lds_attr(kb_ab_srcgrouped<double, 8>, p.lds_abs64); lds_attr(kb_ab_srcgrouped<float, 8>, p.lds_abs32); break;
        default: break;
    }
    switch (p.G2) {
        case 2: lds_attr(kb_ab_grouped<double, 2>, p.lds_ab64_2); lds_attr(kb_ab_grouped<float, 2>, p.lds_ab32_2); break;
        case 4: lds_attr(kb_ab_grouped<double, 4>, p.lds_ab64_2); lds_attr(kb_ab_grouped<float, 4>, p.lds_ab32_2); break;
        case 8: lds_attr(kb_ab_grouped<double, 8>, p.lds_ab64_2); lds_attr(kb_ab_grouped<float, 8>, p.lds_ab32_2); break;
        default: break;
    }
    const int ns = p.nspace;
    auto sgrid = [&](int n) { return dim3((unsigned)std::max(1, std::min(n, kGridCap))); };
    // initial states
    {
        std::vector<dav_state> h(ns);
        for (int b = 0; b < ns; ++b) {
            std::memset(&h[b], 0, sizeof(dav_state));
            h[b].phase = mixed ? 0 : 1;
            h[b].y[0] = 1.0;
        }
        SQD_HIP(ctx, hipMemcpyAsync(p.states, h.data(), sizeof(dav_state) * ns, hipMemcpyHostToDevice, s));
        SQD_HIP(ctx, hipStreamSynchronize(s));
    }
    // start vectors e_argmin(H_II), their products, G[0][0]
    hipLaunchKernelGGL(kb_argmin, sgrid(p.vec.n), dim3(kThreads), 0, s, p.D, p.vec.dev, p.vec.n, p.partial);
    hipLaunchKernelGGL((kb_pick_fin<0>), dim3(ns), dim3(kThreads), 0, s, p.D, p.partial);
    // a mixed batch keeps the basis of its FP32 phase in FP32
    if (mixed) {
        hipLaunchKernelGGL(kb_start<float>, sgrid(p.vec.n), dim3(kThreads), 0, s, p.D, p.vec.dev, p.vec.n, p.partial);
        hipLaunchKernelGGL(kb_norm_fin, dim3(ns), dim3(kThreads), 0, s, p.D, p.partial, 0);
        hipLaunchKernelGGL(kb_scale_copy<float>, sgrid(p.vec.n), dim3(kThreads), 0, s, p.D, p.vec.dev, p.vec.n, 1, 0);
        batched_sigma<R, G, RF>(ctx, p, s, SQD_FP32, nw_ss, nw_ab);
        hipLaunchKernelGGL((kb_dots<MT, float>), sgrid(p.vec.n), dim3(kThreads), 0, s, p.D, p.vec.dev, p.vec.n,
                           p.partial);
    } else {
        hipLaunchKernelGGL(kb_start<double>, sgrid(p.vec.n), dim3(kThreads), 0, s, p.D, p.vec.dev, p.vec.n,
                           p.partial);
        hipLaunchKernelGGL(kb_norm_fin, dim3(ns), dim3(kThreads), 0, s, p.D, p.partial, 0);
        hipLaunchKernelGGL(kb_scale_copy<double>, sgrid(p.vec.n), dim3(kThreads), 0, s, p.D, p.vec.dev, p.vec.n, 0, 0);
        batched_sigma<R, G, RF>(ctx, p, s, SQD_FP64, nw_ss, nw_ab);
        hipLaunchKernelGGL((kb_dots<MT, double>), sgrid(p.vec.n), dim3(kThreads), 0, s, p.D, p.vec.dev, p.vec.n,
                           p.partial);
    }
    hipLaunchKernelGGL((kb_dots_fin<MT>), dim3(ns), dim3(kThreads), 0, s, p.D, p.partial);
    SQD_HIP(ctx, hipGetLastError());
    SQD_HIP(ctx, hipStreamSynchronize(s));

    // one iteration of every space, captured once per precision (the FP32
    // one on the FP32 basis)
    auto record_vt = [&](int prec, auto vt) {
        using VT = decltype(vt);
        hipLaunchKernelGGL((kb_residual<MT, VT>), sgrid(p.vec.n), dim3(kThreads), 0, s, p.D, p.vec.dev, p.vec.n,
                           p.partial);
        hipLaunchKernelGGL((kb_res_fin<MT>), dim3(ns), dim3(kThreads), 0, s, p.D, p.partial, prm);
        hipLaunchKernelGGL((kb_collapse<MT, VT>), sgrid(p.vec.n), dim3(kThreads), 0, s, p.D, p.vec.dev, p.vec.n, 0);
        hipLaunchKernelGGL(kb_collapse_fin, dim3(ns), dim3(64), 0, s, p.D, 0);
        hipLaunchKernelGGL((kb_orth1<MT, VT>), sgrid(p.vec.n), dim3(kThreads), 0, s, p.D, p.vec.dev, p.vec.n,
                           p.partial);
        hipLaunchKernelGGL((kb_orth1_fin<MT, VT>), dim3(ns), dim3(kThreads), 0, s, p.D, p.partial);
        hipLaunchKernelGGL((kb_orth2<MT, VT>), sgrid(p.vec.n), dim3(kThreads), 0, s, p.D, p.vec.dev, p.vec.n,
                           prec == SQD_FP32 ? 1 : 0);
        batched_sigma<R, G, RF>(ctx, p, s, prec, nw_ss, nw_ab);
        hipLaunchKernelGGL((kb_dots<MT, VT>), sgrid(p.vec.n), dim3(kThreads), 0, s, p.D, p.vec.dev, p.vec.n,
                           p.partial);
        hipLaunchKernelGGL((kb_dots_fin<MT>), dim3(ns), dim3(kThreads), 0, s, p.D, p.partial);
    };
    auto record = [&](int prec) {
        if (prec == SQD_FP32) record_vt(prec, 0.0f);
        else record_vt(prec, 0.0);
    };
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipGraph_t graph[2] = {nullptr, nullptr};
    for (int k = 0; k < 2; ++k) {
        const int prec = k == 0 ? SQD_FP32 : SQD_FP64;
        if (prec == SQD_FP32 && !mixed) continue;
        SQD_HIP(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        record(prec);
        SQD_HIP(ctx, hipStreamEndCapture(s, &graph[k]));
        SQD_HIP(ctx, hipGraphInstantiate(&exec[k], graph[k], nullptr, nullptr, 0));
    }
    int phase = mixed ? 0 : 1;
    int replays = 0;
    std::vector<int> switch_iter(ns, -1);
    int rc = SQD_OK;
    while (true) {
        for (int k = 0; k < o->check_every; ++k) {
            if (hipGraphLaunch(exec[phase], s) != hipSuccess) {
                rc = sqd_fail(ctx, SQD_E_HIP, "graph launch failed");
                break;
            }
            ++replays;
        }
        if (rc) break;
        hipLaunchKernelGGL(kb_count_running, dim3(1), dim3(256), 0, s, p.D, ns, p.count_dev);
        if (hipMemcpyAsync(p.count_host, p.count_dev, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = sqd_fail(ctx, SQD_E_HIP, "batched poll failed");
            break;
        }
        if (*p.count_host > 0 && replays <= o->max_iter + 8) continue;
        if (phase == 0) {
            // FP64 refinement of every space at its switch: collapse onto the
            // Ritz vector, FP64 product, rebuild G[0][0]
            std::vector<dav_state> h(ns);
            SQD_HIP(ctx, hipMemcpy(h.data(), p.states, sizeof(dav_state) * ns, hipMemcpyDeviceToHost));
            for (int b = 0; b < ns; ++b)
                if (h[b].done == DONE_SWITCH) switch_iter[b] = h[b].iter;
            // the Ritz vector from the FP32 basis into cin, then V[0] = it,
            // normalised in FP64
            hipLaunchKernelGGL((kb_collapse<MT, float>), sgrid(p.vec.n), dim3(kThreads), 0, s, p.D, p.vec.dev, p.vec.n,
                               1);
            hipLaunchKernelGGL(kb_copy_norm, sgrid(p.vec.n), dim3(kThreads), 0, s, p.D, p.vec.dev, p.vec.n, p.partial);
            hipLaunchKernelGGL(kb_norm_fin, dim3(ns), dim3(kThreads), 0, s, p.D, p.partial, 1);
            hipLaunchKernelGGL(kb_scale_copy<double>, sgrid(p.vec.n), dim3(kThreads), 0, s, p.D, p.vec.dev, p.vec.n,
                               0, 1);
            hipLaunchKernelGGL(kb_collapse_fin, dim3(ns), dim3(64), 0, s, p.D, 1);
            batched_sigma<R, G, RF>(ctx, p, s, SQD_FP64, nw_ss, nw_ab);
            hipLaunchKernelGGL((kb_dots<MT, double>), sgrid(p.vec.n), dim3(kThreads), 0, s, p.D, p.vec.dev, p.vec.n,
                               p.partial);
            hipLaunchKernelGGL((kb_dots_fin<MT>), dim3(ns), dim3(kThreads), 0, s, p.D, p.partial);
            phase = 1;
            replays = 0;
            continue;
        }
        break;
    }
    for (int k = 0; k < 2; ++k) {
        if (exec[k]) (void)hipGraphExecDestroy(exec[k]);
        if (graph[k]) (void)hipGraphDestroy(graph[k]);
    }
    if (rc) return rc;
    hipLaunchKernelGGL((kb_final<MT>), sgrid(p.vec.n), dim3(kThreads), 0, s, p.D, p.vec.dev, p.vec.n, p.partial,
                       mixed ? 1 : 0);
    hipLaunchKernelGGL((kb_pick_fin<1>), dim3(ns), dim3(kThreads), 0, s, p.D, p.partial);
    hipLaunchKernelGGL(kb_final_sign, dim3(ns), dim3(64), 0, s, p.D);
    hipLaunchKernelGGL(kb_final_scale, sgrid(p.vec.n), dim3(kThreads), 0, s, p.D, p.vec.dev, p.vec.n);
    SQD_HIP(ctx, hipGetLastError());
    std::vector<dav_state> h(ns);
    SQD_HIP(ctx, hipMemcpyAsync(h.data(), p.states, sizeof(dav_state) * ns, hipMemcpyDeviceToHost, s));
    SQD_HIP(ctx, hipStreamSynchronize(s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int all_conv = 1;
    for (int b = 0; b < ns; ++b) {
        energies[b] = h[b].theta;
        const int conv = h[b].done == DONE_CONVERGED;
        all_conv &= conv;
        if (reps) {
            sqd_report& r = reps[b];
            std::memset(&r, 0, sizeof(r));
            r.iterations = h[b].iter;
            r.switch_iter = switch_iter[b];
            r.iterations_fp32 = mixed ? (switch_iter[b] >= 0 ? switch_iter[b] : h[b].iter) : 0;
            r.converged = conv;
            r.status = h[b].done;
            r.nhist = h[b].nhist;
            r.energy = h[b].theta;
            r.residual = h[b].rnorm;
            for (int k = 0; k < h[b].nhist && k < SQD_HIST; ++k) {
                r.residual_history[k] = h[b].hist_r[k];
                r.energy_history[k] = h[b].hist_e[k];
            }
            r.seconds = secs;
        }
    }
    return all_conv ? SQD_OK : SQD_NOT_CONVERGED;
}

int pick_R(sqd_ctx* ctx, int64_t max_cols, int norb, size_t es, int forced) {
    for (int R : {8, 4, 2, 1}) {
        if (forced && R != forced) continue;
        if (((size_t)(max_cols + 1) * R + (size_t)norb * norb * R) * es <= (size_t)ctx->max_lds) return R;
    }
    return 0;
}

int pick_G(sqd_ctx* ctx, int64_t max_nb, int norb) {
    auto bytes = [&](int G) { return (size_t)(max_nb + 1) * G * 8 + (size_t)norb * norb * 8; };
    const int forced = ctx->tune[SQD_TUNE_AB_GROUP];
    if (forced) return bytes(forced) <= (size_t)ctx->max_lds ? forced : 0;
    for (int G : {8, 4, 2}) if (bytes(G) <= (size_t)ctx->max_lds / 2) return G;
    for (int G : {8, 4, 2, 1}) if (bytes(G) <= (size_t)ctx->max_lds) return G;
    return 0;
}

}  // namespace

int sqd_davidson_batched_impl(sqd_ctx* ctx, int nspace, sqd_space* const* spaces, const sqd_davidson_opts* o,
                              double* energies, double* const* vecs, sqd_report* reps) {
    const int norb = ctx->norb;
    batch_plan p;
    p.nspace = nspace;
    int rc = SQD_OK;
    int64_t max_nb = 0, max_na = 0;
    for (int b = 0; b < nspace; ++b) {
        max_na = std::max(max_na, spaces[b]->sp[0].n);
        max_nb = std::max(max_nb, spaces[b]->sp[1].n);
        if ((rc = sqd_ensure_diag(ctx, spaces[b]))) return rc;
    }
    const int64_t max_cols = std::max(max_na, max_nb);
    p.R = pick_R(ctx, max_cols, norb, 8, ctx->tune[SQD_TUNE_SS_ROWS]);
    p.Rf = p.R;
    p.G = pick_G(ctx, max_nb, norb);
    if (!p.R || !p.Rf || !p.G) return sqd_fail(ctx, SQD_E_LIMIT, "batched tiles do not fit in LDS");
    // spaces whose own rows allow a larger pair group than the batch's
    // longest rows form a second class with its own launch (cfg-4-like
    // batches: beta rows of 200-3000 strings, groups of four below about
    // 2400 strings and of two above); a forced group size keeps one class
    std::vector<char> cls2(nspace, 0);
    int64_t max_nb2 = 0;
    if (!ctx->tune[SQD_TUNE_AB_GROUP]) {
        for (int b = 0; b < nspace; ++b)
            if (pick_G(ctx, spaces[b]->sp[1].n, norb) > p.G) {
                cls2[b] = 1;
                max_nb2 = std::max(max_nb2, spaces[b]->sp[1].n);
            }
        if (max_nb2 > 0) p.G2 = pick_G(ctx, max_nb2, norb);
        // where the longest rows leave pair groups of one or two, that class
        // groups its singles by source string instead (as the single-space
        // product does)
        if (p.G <= 2 && ctx->tune[SQD_TUNE_AB_VARIANT] != 1) {
            const size_t n2 = (size_t)norb * norb;
            for (int G : {8, 4, 3, 2})
                if ((size_t)(max_nb + 1) * 8 + (size_t)G * n2 * 8 <= (size_t)ctx->max_lds) { p.GS = G > p.G ? G : 0; break; }
        }
    }
    p.lds_ss64 = ((size_t)(max_cols + 1) * p.R + (size_t)norb * norb * p.R) * 8;
    p.lds_ss32 = ((size_t)(max_cols + 1) * p.R + (size_t)norb * norb * p.R) * 4;
    p.lds_ab64 = ((size_t)(max_nb + 1) * p.G + (size_t)norb * norb) * 8;
    p.lds_ab32 = ((size_t)(max_nb + 1) * p.G + (size_t)norb * norb) * 4;
    p.lds_ab64_2 = ((size_t)(max_nb2 + 1) * p.G2 + (size_t)norb * norb) * 8;
    p.lds_abs64 = ((size_t)(max_nb + 1) + (size_t)p.GS * norb * norb) * 8;
    p.lds_abs32 = ((size_t)(max_nb + 1) + (size_t)p.GS * norb * norb) * 4;
    p.lds_ab32_2 = ((size_t)(max_nb2 + 1) * p.G2 + (size_t)norb * norb) * 4;
    p.gather_lds64 = (size_t)max_nb * 8 <= (size_t)(64 * 1024) ? (size_t)max_nb * 8 : 0;
    p.grid_persist = ctx->num_cu * 2;
    const bool mixed = o->mode == SQD_DAV_MIXED;
    const int mmax = o->m_max;
    // Every device buffer of the plan is a slice of one arena that the context
    // keeps (grown on demand) across calls: a batch of dozens of spaces needs
    // hundreds of buffers, and allocating and freeing them per call costs more
    // than a short solve.  Slices are requested first and bound to the arena
    // once its size is known.
    std::vector<std::pair<void**, size_t>> req;
    auto want = [&](void** ptr, size_t bytes) { req.push_back({ptr, bytes}); };
    p.host.resize(nspace);
    int part = 0;
    std::vector<int2> vec, tr, ssbb, ssaa, abg, abg2, gath;
    std::vector<std::pair<double, int>> order;  // longest-first by sigma work
    for (int b = 0; b < nspace; ++b) {
        sqd_space* sp = spaces[b];
        const spin_tables& A = sp->sp[0];
        const spin_tables& B = sp->sp[1];
        if (cls2[b]) rc = sqd_ensure_ab_groups(ctx, sp, p.G2);
        else rc = p.GS ? sqd_ensure_ab_source_groups(ctx, sp, p.GS) : sqd_ensure_ab_groups(ctx, sp, p.G);
        if (rc) return rc;
        bdesc& d = p.host[b];
        std::memset(&d, 0, sizeof(d));
        d.n = sp->dim;
        d.na = A.n;
        d.nb = B.n;
        d.nblk = (int)std::max<int64_t>(1, std::min<int64_t>((d.n + kThreads - 1) / kThreads, kMaxBlocks));
        d.part0 = part;
        part += d.nblk;
        d.ntx = (int)nblk(d.nb, 64);
        d.nty = (int)nblk(d.na, 64);
        const int64_t ldy = (int64_t)B.nslices * 64;
        want((void**)&d.V, sizeof(double) * d.n * mmax);
        want((void**)&d.AV, sizeof(double) * d.n * mmax);
        want((void**)&d.T, sizeof(double) * d.n);
        want((void**)&d.cin, sizeof(double) * d.n);
        want((void**)&d.sout, sizeof(double) * d.n);
        want((void**)&d.Ct, sizeof(double) * d.n);
        want((void**)&d.Yt, sizeof(double) * d.n);
        want((void**)&d.Y64, sizeof(double) * (A.nnz_s * ldy + 1));
        if (mixed) {
            want((void**)&d.c32, sizeof(float) * d.n);
            want((void**)&d.Ct32, sizeof(float) * d.n);
            want((void**)&d.Yt32, sizeof(float) * d.n);
            want((void**)&d.S32, sizeof(float) * d.n);
            want((void**)&d.Y32, sizeof(float) * (A.nnz_s * ldy + 1));
        }
        for (int j = 0; j < d.nblk; ++j) vec.push_back(make_int2(b, j));
        for (int t = 0; t < d.ntx * d.nty; ++t) tr.push_back(make_int2(b, t));
        for (int64_t k = 0; k < d.na; ++k) gath.push_back(make_int2(b, (int)k));
        const double work = (double)(B.nnz_s + B.nnz_d) * A.n + (double)(A.nnz_s + A.nnz_d) * B.n +
                            (double)A.nnz_s * B.nnz_s;
        order.emplace_back(-work, b);
    }
    // longest-first: spaces by sigma work, their tiles in order
    std::sort(order.begin(), order.end());
    for (auto& ob : order) {
        const int b = ob.second;
        const bdesc& d = p.host[b];
        for (int64_t r = 0; r < (d.na + p.R - 1) / p.R; ++r) ssbb.push_back(make_int2(b, (int)r));
        for (int64_t r = 0; r < (d.nb + p.R - 1) / p.R; ++r) ssaa.push_back(make_int2(b, (int)r));
        const int nch = (!cls2[b] && p.GS) ? spaces[b]->abs_nchunks : spaces[b]->ab_nchunks;
        for (int c = 0; c < nch; ++c) (cls2[b] ? abg2 : abg).push_back(make_int2(b, c));
    }
    want((void**)&p.partial, sizeof(double) * (size_t)part * kPstride);
    want((void**)&p.states, sizeof(dav_state) * nspace);
    want((void**)&p.counters, sizeof(int) * 8);
    want((void**)&p.count_dev, sizeof(int));
    want((void**)&p.D, sizeof(bdesc) * nspace);
    std::pair<std::vector<int2>*, unit_list*> lists[7] = {{&vec, &p.vec}, {&tr, &p.tr}, {&ssbb, &p.ss_bb},
                                                          {&ssaa, &p.ss_aa}, {&abg, &p.abg}, {&abg2, &p.abg2},
                                                          {&gath, &p.gath}};
    for (auto& l : lists) {
        l.second->n = (int)l.first->size();
        if (l.first->empty()) l.first->push_back(make_int2(0, 0));
        want((void**)&l.second->dev, sizeof(int2) * l.first->size());
    }
    size_t total = 0;
    for (auto& r : req) total += (r.second + 255) & ~(size_t)255;
    if (ctx->batch_arena_bytes < total) {
        if (ctx->batch_arena) {
            (void)hipStreamSynchronize(ctx->stream);
            (void)hipFree(ctx->batch_arena);
            ctx->batch_arena = nullptr;
            ctx->batch_arena_bytes = 0;
        }
        if ((rc = sqd_alloc(ctx, &ctx->batch_arena, total, nullptr))) return rc;
        ctx->batch_arena_bytes = total;
    }
    {
        char* base = static_cast<char*>(ctx->batch_arena);
        size_t off = 0;
        for (auto& r : req) {
            *r.first = base + off;
            off += (r.second + 255) & ~(size_t)255;
        }
    }
    for (int b = 0; b < nspace; ++b) {
        sqd_space* sp = spaces[b];
        const spin_tables& A = sp->sp[0];
        const spin_tables& B = sp->sp[1];
        bdesc& d = p.host[b];
        const int64_t ldy = (int64_t)B.nslices * 64;
        d.diag = sp->diag;
        d.out = vecs[b];
        d.noise = nullptr;
        d.a_off = A.s_off;
        d.a_order = sp->ab_row_order;
        d.st = p.states + b;
        // same-spin: BB on C (rows alpha, columns beta, diagonal fused), AA on C^T
        d.aa64 = ss_args<double>{d.Ct, d.Yt, B.n, A.n, A.perm_ss, A.nslices, A.sl_s_off, A.sl_d_off, A.sell_s_pk,
                                 A.sell_s_v64, A.sell_d_nbr, A.sell_d_v64, B.str, B.nw, nullptr, 0};
        d.bb64 = ss_args<double>{d.cin, d.sout, A.n, B.n, B.perm_ss, B.nslices, B.sl_s_off, B.sl_d_off, B.sell_s_pk,
                                 B.sell_s_v64, B.sell_d_nbr, B.sell_d_v64, A.str, A.nw, sp->diag, 1};
        d.aa32 = ss_args<float>{d.Ct32, d.Yt32, B.n, A.n, A.perm_ss, A.nslices, A.sl_s_off, A.sl_d_off, A.sell_s_pk,
                                A.sell_s_v32, A.sell_d_nbr, A.sell_d_v32, B.str, B.nw, nullptr, 0};
        d.bb32 = ss_args<float>{d.c32, d.S32, A.n, B.n, B.perm_ss, B.nslices, B.sl_s_off, B.sl_d_off, B.sell_s_pk,
                                B.sell_s_v32, B.sell_d_nbr, B.sell_d_v32, A.str, A.nw, nullptr, 1};
        const bool src = !cls2[b] && p.GS;
        const int* grp = src ? sp->abs_grp : sp->ab_grp;
        const int* cpair = src ? nullptr : sp->ab_chunk_pair;
        d.abs_src = src ? sp->abs_src : nullptr;
        d.ab64 = abg_args<double>{d.cin, d.Y64, B.n, ldy, grp, cpair, A.s_pk, B.perm_ab, B.nslices, B.sl_ab_off,
                                  B.sell_ab_pk};
        d.ab32 = abg_args<float>{d.c32, d.Y32, B.n, ldy, grp, cpair, A.s_pk, B.perm_ab, B.nslices, B.sl_ab_off,
                                 B.sell_ab_pk};
    }
    if (!ctx->batch_count_host &&
        hipHostMalloc((void**)&ctx->batch_count_host, sizeof(int), hipHostMallocDefault) != hipSuccess) {
        ctx->batch_count_host = nullptr;
        return sqd_fail(ctx, SQD_E_OOM, "pinned allocation failed");
    }
    p.count_host = ctx->batch_count_host;
    for (auto& l : lists)
        SQD_HIP(ctx, hipMemcpy(l.second->dev, l.first->data(), sizeof(int2) * l.first->size(),
                               hipMemcpyHostToDevice));
    SQD_HIP(ctx, hipMemcpy(p.D, p.host.data(), sizeof(bdesc) * nspace, hipMemcpyHostToDevice));
    // a private stream for graph capture, ordered after the context's stream
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&ev) != hipSuccess)
        return sqd_fail(ctx, SQD_E_HIP, "stream creation failed");
    (void)hipEventRecord(ev, ctx->stream);
    (void)hipStreamWaitEvent(s, ev, 0);
    // the FP32 same-spin kernel stages as many rows as the FP64 one
    auto run = [&](auto mt) -> int {
        constexpr int MT = decltype(mt)::value;
        auto with_g = [&](auto rr) -> int {
            constexpr int R = decltype(rr)::value;
            switch (p.G) {
                case 8: return batched_run<MT, R, 8, R>(ctx, p, o, energies, reps, s);
                case 4: return batched_run<MT, R, 4, R>(ctx, p, o, energies, reps, s);
                case 2: return batched_run<MT, R, 2, R>(ctx, p, o, energies, reps, s);
                default: return batched_run<MT, R, 1, R>(ctx, p, o, energies, reps, s);
            }
        };
        switch (p.R) {
            case 8: return with_g(std::integral_constant<int, 8>());
            case 4: return with_g(std::integral_constant<int, 4>());
            case 2: return with_g(std::integral_constant<int, 2>());
            default: return with_g(std::integral_constant<int, 1>());
        }
    };
    if (mmax <= 16) rc = run(std::integral_constant<int, 16>());
    else rc = run(std::integral_constant<int, 32>());
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(s);
    return rc;
}
