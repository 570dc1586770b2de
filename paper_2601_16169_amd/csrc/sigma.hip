// sigma = H c on the product space (Sec. II matrix-free product; Sec. IV the
// three task types of the Slater-Condon rules: alpha-alpha, beta-beta and one
// alpha plus one beta excitation).
//
// Terms and kernels (all owner-computes, no atomics, deterministic):
//   DIAG  H_II c_I, fused into the beta-beta kernel's epilogue (FP64 always).
//   BB    same-spin kernel on C (rows = alpha strings, columns = beta strings):
//         sigma[ia, jb] += sum over beta singles/doubles (jb <- kb) of
//         H^bb(jb, kb; Ia) c[ia, kb].  A workgroup stages R rows of C in LDS
//         (layout [column][row], plus a zero slot for padding) and the
//         cross-spin term W_a[pq] = sum_{k in Ia} (pq|kk) of those rows; each
//         lane owns one target column of a 64-row slice of the sliced table
//         and walks its entries (coalesced 64-wide table reads).
//   AA    the same kernel on C^T (one tiled transpose each way), i.e. the
//         beta-beta machinery applied with the spins swapped.
//   AB    sigma[ia', jb'] += sum_{alpha singles ia' <- ia (pair ai, s_a)}
//         sum_{beta singles jb' <- jb (pair bj, s_b)} s_a s_b (ai|bj) c[ia, jb]:
//         a workgroup per target alpha row stages KC source rows of C and the
//         KC rows s_a (ai|..) of the (pq|rs) matrix in LDS (interleaved so one
//         lane reads all KC values of a column with wide loads), lanes own
//         beta targets and accumulate in registers across all alpha sources.
#include "sigma_body.h"

namespace {

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <typename T> struct vec2;
template <> struct vec2<double> { using type = double2; };
template <> struct vec2<float> { using type = float2; };

// ---------------------------------------------------------------- diagonal
// ua[ia*norb + q] = sum_{p in Ia} (pp|qq)
__global__ void k_ua(const uint64_t* __restrict__ astr, int nw, int64_t na, int norb,
                     const double* __restrict__ jdiag, double* __restrict__ ua) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= na * norb) return;
    const int64_t ia = k / norb;
    const int q = (int)(k % norb);
    double acc = 0.0;
    str_for_each(astr + ia * nw, nw, [&](int p) { acc += jdiag[p * norb + q]; });
    ua[k] = acc;
}

// H_II = ecore + E_a(Ia) + E_b(Ib) + sum_{p in Ia, q in Ib} (pp|qq)
__global__ void k_diag(const double* __restrict__ ea, const double* __restrict__ eb, const double* __restrict__ ua,
                       const uint64_t* __restrict__ bstr, int nw, int64_t na, int64_t nb, int norb, double ecore,
                       double* __restrict__ diag) {
    const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= na * nb) return;
    const int64_t ia = d / nb, ib = d % nb;
    const double* u = ua + ia * norb;
    double acc = ecore + ea[ia] + eb[ib];
    str_for_each(bstr + ib * nw, nw, [&](int q) { acc += u[q]; });
    diag[d] = acc;
}

// ---------------------------------------------------------------- transposes
// out[c][r] (=|+=) in[r][c], in is rows x cols; 64x64 tiles through LDS.
template <typename TI, typename TO, bool ADD>
__global__ void __launch_bounds__(256) k_transpose(const TI* __restrict__ in, TO* __restrict__ out, int64_t rows,
                                                   int64_t cols, const int* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ TI tile[64][65];
    transpose_tile<TI, TO, ADD>(in, out, rows, cols, blockIdx.y, blockIdx.x, tile);
}

template <typename TI, typename TO>
__global__ void k_convert(const TI* __restrict__ in, TO* __restrict__ out, int64_t n, const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = (TO)in[k];
}

template <typename T>
__global__ void k_fill(T* __restrict__ out, int64_t n, T v, const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = v;
}

// sigma = (diag ? diag*c : 0) + (accumulate ? sigma : 0) + (double)s32
__global__ void k_combine(const double* __restrict__ diag, const double* __restrict__ c,
                          const float* __restrict__ s32, double* __restrict__ sigma, int64_t n,
                          const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double v = s32 ? (double)s32[k] : 0.0;
    if (diag) v += diag[k] * c[k];
    sigma[k] = v;
}

__global__ void k_diag_apply(const double* __restrict__ diag, const double* __restrict__ c, double* __restrict__ s,
                             int64_t n, int accumulate, const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double v = diag[k] * c[k];
    if (accumulate) v += s[k];
    s[k] = v;
}


// ---------------------------------------------------------------- same-spin
// X: nrows x ncols (row = string of the other spin, column = string of the
// excited spin).  Y (=|+=) sum over the column spin's singles and doubles.
// LDS: xs[(ncols+1)*R] as [col][r]; ws[norb2*R] as [pq][r].
template <typename T, int R>
__global__ void __launch_bounds__(1024)
k_same_spin(ss_args<T> a, const T* __restrict__ jk, int norb, const int* __restrict__ skip) {
    if (skip && *skip) return;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    ss_block<T, R>(a, jk, norb, blockIdx.x, lds_raw);
}

// ---------------------------------------------------------------- alpha-beta
// One workgroup per target alpha row ia' (blockIdx.x) and group of beta slices
// (blockIdx.y).  LDS: cs[(nb+1)*KC] as [col][k]; vs[norb2*KC] as [pq][k].
template <typename T, int KC, int MAXJ>
__global__ void __launch_bounds__(1024)
k_ab_direct(const T* __restrict__ C, T* __restrict__ S, int64_t na, int64_t nb, const int* __restrict__ a_off,
            const uint32_t* __restrict__ a_pk, const int* __restrict__ bperm, int nbslices,
            const int* __restrict__ bsl_off, const uint32_t* __restrict__ bs_pk, const T* __restrict__ V, int norb,
            const int* __restrict__ skip) {
    if (skip && *skip) return;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* cs = reinterpret_cast<T*>(lds_raw);
    const int norb2 = norb * norb;
    T* vs = cs + (nb + 1) * KC;
    const int64_t ia = blockIdx.x;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63, nw = nthr >> 6;
    const int slice_base = blockIdx.y * nw * MAXJ;
    const int a0 = a_off[ia], a1 = a_off[ia + 1];
    T acc[MAXJ];
#pragma unroll
    for (int j = 0; j < MAXJ; ++j) acc[j] = (T)0;
    for (int k0 = a0; k0 < a1; k0 += KC) {
        __syncthreads();
        {
            const T* rows[KC];
#pragma unroll
            for (int k = 0; k < KC; ++k)
                rows[k] = (k0 + k < a1) ? C + (int64_t)(a_pk[k0 + k] & SQD_NBR_MASK) * nb : nullptr;
            stage_rows<T, KC>(cs, rows, (int)nb);
        }
        for (int idx = tid; idx < KC * norb2; idx += nthr) {
            const int k = idx / norb2, pq = idx - k * norb2;
            T v = (T)0;
            if (k0 + k < a1) {
                const uint32_t e = a_pk[k0 + k];
                const int pair = (int)((e >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK);
                v = V[(int64_t)pair * norb2 + pq];
                if (e >> 31) v = -v;
            }
            vs[lds_cols<T, KC>::idx(pq, k)] = v;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < MAXJ; ++j) {
            const int sl = slice_base + j * nw + wave;
            if (sl < nbslices) {
                const int c0 = bsl_off[sl], c1 = bsl_off[sl + 1];
                T a = acc[j];
                auto one = [&](uint32_t e) {
                    const int nbr = (int)(e & SQD_NBR_MASK);
                    const int pair = (int)((e >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK);
                    T cr[KC], vr[KC];
                    lds_cols<T, KC>::load(cs, nbr, cr);
                    lds_cols<T, KC>::load(vs, pair, vr);
                    T t = (T)0;
#pragma unroll
                    for (int k = 0; k < KC; ++k) t += vr[k] * cr[k];
                    a += (e >> 31) ? -t : t;
                };
                int col = c0;
                for (; col + 8 <= c1; col += 8) {   // eight table entries in flight
                    uint32_t b8[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) b8[u] = bs_pk[(int64_t)(col + u) * 64 + lane];
#pragma unroll
                    for (int u = 0; u < 8; ++u) one(b8[u]);
                }
                if (col + 4 <= c1) {
                    uint32_t b4[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) b4[u] = bs_pk[(int64_t)(col + u) * 64 + lane];
#pragma unroll
                    for (int u = 0; u < 4; ++u) one(b4[u]);
                    col += 4;
                }
                for (; col < c1; ++col) one(bs_pk[(int64_t)col * 64 + lane]);
                acc[j] = a;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < MAXJ; ++j) {
        const int sl = slice_base + j * nw + wave;
        if (sl < nbslices) {
            const int tb = bperm[sl * 64 + lane];
            if (tb < nb) {
                const int64_t o = ia * nb + tb;
                S[o] += acc[j];
            }
        }
    }
}


// ---------------------------------------------------------------- alpha-beta, grouped by alpha pair
// (body and layout: abg_block); a coalesced gather then adds
// sigma[ia'][jb'] += sum_{e in row ia'} Y[e][slot(jb')].
template <typename T, int G>
__global__ void __launch_bounds__(1024)
k_ab_grouped(abg_args<T> a, const T* __restrict__ V, int norb, const int* __restrict__ skip) {
    if (skip && *skip) return;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    abg_block<T, G>(a, V, norb, blockIdx.x, lds_raw);
}

// ---------------------------------------------------------------- alpha-beta, grouped by source string
// (body and layout: abs_block); the same gather follows.
template <typename T, int GS>
__global__ void __launch_bounds__(1024)
k_ab_srcgrouped(abg_args<T> a, const int* __restrict__ chunk_src, const T* __restrict__ V, int norb,
                const int* __restrict__ skip) {
    if (skip && *skip) return;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    abs_block<T, GS>(a, chunk_src, V, norb, blockIdx.x, lds_raw);
}

// sigma[ia][perm(p)] += sum_{e = a_off[ia]}^{a_off[ia+1]-1} Y[e][p] (gather_row),
// one workgroup per alpha row; STAGED: the row is assembled in LDS first.
template <typename T, bool STAGED>
__global__ void __launch_bounds__(1024)
k_ab_gather(const T* __restrict__ Y, T* __restrict__ S, int64_t na, int64_t nb, int64_t ldy,
            const int* __restrict__ bperm, const int* __restrict__ a_off, const int* __restrict__ order,
            const int* __restrict__ skip) {
    if (skip && *skip) return;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* row = STAGED ? reinterpret_cast<T*>(lds_raw) : nullptr;
    for (int64_t k = blockIdx.x; k < na; k += gridDim.x)
        gather_row<T>(Y, S, nb, ldy, bperm, a_off, order[k], row);
}

// Longest alpha-beta output row assembled in LDS by the gather (larger rows are
// added in place, with scattered read-modify-writes of sigma).
constexpr int64_t kGatherStageBytes = 128 * 1024;

constexpr int kAbMaxJ = 8;

// Raise a kernel's dynamic-LDS limit once per kernel (largest size seen).
template <typename F>
void set_lds(F f, int bytes) {
    static std::vector<std::pair<const void*, int>> seen;
    const void* key = reinterpret_cast<const void*>(f);
    for (auto& kv : seen)
        if (kv.first == key) {
            if (kv.second >= bytes) return;
            kv.second = bytes;
            (void)hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
            return;
        }
    seen.emplace_back(key, bytes);
    (void)hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

int pick_rows(sqd_ctx* ctx, int64_t nrows, int64_t ncols, int norb, size_t es) {
    const int forced = ctx->tune[SQD_TUNE_SS_ROWS];
    const int cands[4] = {8, 4, 2, 1};
    for (int R : cands) {
        if (forced && R != forced) continue;
        const size_t lds = ((size_t)(ncols + 1) * R + (size_t)norb * norb * R) * es;
        if (lds > (size_t)ctx->max_lds) continue;
        // enough row blocks to occupy (nearly) every compute unit
        if (!forced && R > 1 && (nrows + R - 1) / R < (int64_t)ctx->num_cu * 9 / 10) continue;
        return R;
    }
    return 0;
}

int pick_chunk(sqd_ctx* ctx, int64_t nb, int norb, size_t es) {
    const int forced = ctx->tune[SQD_TUNE_AB_CHUNK];
    const int cands[4] = {8, 4, 2, 1};
    for (int K : cands) {
        if (forced && K != forced) continue;
        const size_t lds = ((size_t)(nb + 1) + (size_t)norb * norb) * K * es;
        if (lds <= (size_t)ctx->max_lds) return K;
    }
    return 0;
}

// The spin_tables that own the arrays of t (an alias of the other spin's
// tables when both spins have the same strings).
spin_tables& owner(sqd_space* sp, const spin_tables& t) {
    if (&t == &sp->sp[1] && t.alias) return sp->sp[0];
    return const_cast<spin_tables&>(t);
}

// Windowed same-spin kernel: forced on or off by SQD_TUNE_SS_WINDOW, else used
// when fewer than four rows fit in one workgroup's LDS.  Measured on MI355X
// on norb-36 spaces of n strings per spin (same-spin beta-beta / alpha-alpha
// terms, ms, row-staged against windowed): FP64 with two rows staged, n =
// 4000: 1.41 / 1.55 against 1.00 / 0.91; n = 8000: 5.75 / 6.18 against 4.64 /
// 3.99; one row, n = 16000: 48.6 / 50.8 against 23.6 / 21.5.  FP32 with four
// rows staged, n = 6000: 1.29 / 1.44 against 1.56 / 1.48; n = 8000: 2.25 /
// 2.50 against 2.53 / 2.35; two rows, n = 10000: 5.41 / 5.82 against 4.65 /
// 4.23; n = 16000: 15.0 / 16.0 against 12.9 / 11.0.
bool use_window(sqd_ctx* ctx, int64_t nrows, int64_t ncols, int norb, size_t es) {
    const int mode = ctx->tune[SQD_TUNE_SS_WINDOW];
    if (mode == 1) return false;
    if (mode >= 2) return true;
    if (ctx->tune[SQD_TUNE_SS_ROWS]) return false;
    const size_t lds4 = ((size_t)(ncols + 1) * 4 + (size_t)norb * norb * 4) * es;
    return lds4 > (size_t)ctx->max_lds && nrows >= 2;
}

// colmajor: X and Y hold the transposes (the alpha-alpha term read from C and
// added into sigma directly).
// The alpha-alpha term runs column-major on C (no transposes) when a staged
// column of C is a whole 64-byte piece: the windowed kernel (8 FP64 or 16
// FP32 rows) and the row-staged kernel with 8 FP64 rows (measured on MI355X:
// 4.0e6 workload, sigma FP64 0.878 -> 0.867 ms; FP32 with 8 rows, 32-byte
// pieces: no change; FP32 with 2 rows of the 2.56e8 workload, 8-byte pieces:
// alpha-alpha with its transposes 17.1 ms, in place 20.8 ms); otherwise the
// transposes around the row-major kernel.
bool aa_in_place(sqd_ctx* ctx, int64_t nb, int64_t na, int norb, size_t es) {
    if (use_window(ctx, nb, na, norb, es)) return true;
    return (size_t)pick_rows(ctx, nb, na, norb, es) * es >= 64;
}

template <typename T>
int launch_same_spin(sqd_ctx* ctx, sqd_space* sp, const T* X, T* Y, int64_t nrows, int64_t ncols,
                     const spin_tables& col, const spin_tables& row, const T* jk, int norb, const double* diag,
                     int accumulate, const int* skip, const char* timer_name, int colmajor = 0) {
    const size_t es = sizeof(T);
    if (use_window(ctx, nrows, ncols, norb, es)) {
        // the windowed kernel ends in slot order, so the diagonal (scattered
        // reads of diag and X there) goes in the coalesced pass that places
        // its output, or in one of its own (2.56e8 workload: beta-beta with
        // the diagonal fused in the kernel 35.5 ms, without 28.1 ms)
        int diag_done = 0;
        int rc = sqd_same_spin_windowed(ctx, sp, owner(sp, col), owner(sp, row), X, Y, nrows, ncols, colmajor,
                                        accumulate, sizeof(T) == 4, sizeof(T) == 8 ? diag : nullptr, &diag_done,
                                        skip, timer_name);
        if (rc || !diag || diag_done) return rc;
        if constexpr (sizeof(T) == 8) {
            prof_scope pd(ctx, "k_diag_apply");
            const int64_t n = nrows * ncols;
            hipLaunchKernelGGL(k_diag_apply, dim3(nblk(n, 256)), dim3(256), 0, ctx->stream, diag, X, Y, n, 1, skip);
            SQD_HIP(ctx, hipGetLastError());
        }
        return SQD_OK;
    }
    const int R = pick_rows(ctx, nrows, ncols, norb, es);
    if (R == 0) return sqd_fail(ctx, SQD_E_LIMIT, "same-spin row does not fit in LDS (too many strings)");
    const size_t lds = ((size_t)(ncols + 1) * R + (size_t)norb * norb * R) * es;
    // measured on MI355X: 16 waves hide the table latency best with 8 staged
    // rows, and whenever the LDS leaves room for one workgroup per CU only
    // (long rows: the table is then streamed once per row from the caches)
    int nw = ctx->tune[SQD_TUNE_SS_WAVES] ? ctx->tune[SQD_TUNE_SS_WAVES]
                                          : ((R == 8 || lds > (size_t)ctx->max_lds / 2) ? 16 : 8);
    const dim3 grid(nblk(nrows, R)), block(64 * nw);
    const T* sv = nullptr; const T* dv = nullptr;
    if constexpr (sizeof(T) == 8) { sv = (const T*)col.sell_s_v64; dv = (const T*)col.sell_d_v64; }
    else { sv = (const T*)col.sell_s_v32; dv = (const T*)col.sell_d_v32; }
    ss_args<T> args{X, Y, nrows, ncols, col.perm_ss, col.nslices, col.sl_s_off, col.sl_d_off, col.sell_s_pk, sv,
                    col.sell_d_nbr, dv, row.str, row.nw, diag, accumulate, colmajor};
    prof_scope ps(ctx, timer_name);
#define SQD_SS_LAUNCH(RR)                                                                                    \
    case RR:                                                                                                 \
        set_lds(k_same_spin<T, RR>, (int)lds);                                                               \
        hipLaunchKernelGGL((k_same_spin<T, RR>), grid, block, lds, ctx->stream, args, jk, norb, skip);       \
        break;
    switch (R) {
        SQD_SS_LAUNCH(1)
        SQD_SS_LAUNCH(2)
        SQD_SS_LAUNCH(4)
        SQD_SS_LAUNCH(8)
    }
#undef SQD_SS_LAUNCH
    SQD_HIP(ctx, hipGetLastError());
    return SQD_OK;
}

template <typename T>
int launch_ab_direct(sqd_ctx* ctx, const sqd_space* sp, const T* C, T* S, const T* V, const int* skip) {
    const spin_tables& A = sp->sp[0];
    const spin_tables& B = sp->sp[1];
    const size_t es = sizeof(T);
    const int KC = pick_chunk(ctx, B.n, sp->norb, es);
    if (KC == 0) return sqd_fail(ctx, SQD_E_LIMIT, "alpha-beta source row does not fit in LDS");
    int nw = ctx->tune[SQD_TUNE_AB_WAVES] ? ctx->tune[SQD_TUNE_AB_WAVES] : 8;
    // fewer waves when there are few slices
    while (nw > 4 && (int64_t)nw * 2 > B.nslices && ctx->tune[SQD_TUNE_AB_WAVES] == 0) nw >>= 1;
    const int groups = (B.nslices + nw * kAbMaxJ - 1) / (nw * kAbMaxJ);
    const size_t lds = ((size_t)(B.n + 1) + (size_t)sp->norb * sp->norb) * KC * es;
    const dim3 grid((unsigned)A.n, (unsigned)groups), block(64 * nw);
    prof_scope ps(ctx, sizeof(T) == 8 ? "k_ab_direct<double>" : "k_ab_direct<float>");
#define SQD_AB_LAUNCH(KK)                                                                                    \
    case KK:                                                                                                 \
        set_lds(k_ab_direct<T, KK, kAbMaxJ>, (int)lds);                                                      \
        hipLaunchKernelGGL((k_ab_direct<T, KK, kAbMaxJ>), grid, block, lds, ctx->stream, C, S, A.n, B.n,   \
                           A.s_off, A.s_pk, B.perm_ab, B.nslices, B.sl_ab_off, B.sell_ab_pk, V, sp->norb,  \
                           skip);                                                                            \
        break;
    switch (KC) {
        SQD_AB_LAUNCH(1)
        SQD_AB_LAUNCH(2)
        SQD_AB_LAUNCH(4)
        SQD_AB_LAUNCH(8)
    }
#undef SQD_AB_LAUNCH
    SQD_HIP(ctx, hipGetLastError());
    return SQD_OK;
}


// Entries per chunk of the grouped alpha-beta kernel: the most source rows of
// C (FP64) that fit in LDS next to one row of (pq|rs).
int ab_group_size(sqd_ctx* ctx, const sqd_space* sp) {
    const size_t nb = (size_t)sp->sp[1].n, n2 = (size_t)sp->norb * sp->norb;
    const int forced = ctx->tune[SQD_TUNE_AB_GROUP];
    auto bytes = [&](int G) { return (nb + 1) * G * sizeof(double) + n2 * sizeof(double); };
    if (forced) return bytes(forced) <= (size_t)ctx->max_lds ? forced : 0;
    // largest group that leaves room for two workgroups per compute unit (one
    // stages while the other computes), else the largest that fits
    for (int G : {8, 4, 2}) if (bytes(G) <= (size_t)ctx->max_lds / 2) return G;
    for (int G : {8, 4, 2, 1}) if (bytes(G) <= (size_t)ctx->max_lds) return G;
    return 0;
}

// Gather order: heaviest alpha rows first, so that the rows with the most
// singles start together on different compute units.
int ensure_ab_row_order(sqd_ctx* ctx, sqd_space* sp) {
    if (sp->ab_row_order) return SQD_OK;
    const spin_tables& A = sp->sp[0];
    std::vector<int> off(A.n + 1);
    SQD_HIP(ctx, hipMemcpy(off.data(), A.s_off, sizeof(int) * (A.n + 1), hipMemcpyDeviceToHost));
    std::vector<int> order(A.n);
    for (int64_t r = 0; r < A.n; ++r) order[r] = (int)r;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return off[x + 1] - off[x] > off[y + 1] - off[y]; });
    int rc;
    if ((rc = sqd_alloc(ctx, (void**)&sp->ab_row_order, sizeof(int) * (A.n + 1), &sp->bytes))) return rc;
    SQD_HIP(ctx, hipMemcpy(sp->ab_row_order, order.data(), sizeof(int) * A.n, hipMemcpyHostToDevice));
    return SQD_OK;
}

// Group the alpha singles (CSR positions) by orbital pair, padded to chunks of G.
int ensure_ab_groups_impl(sqd_ctx* ctx, sqd_space* sp, int G) {
    if (sp->ab_G == G && sp->ab_grp) return SQD_OK;
    if (G <= 0) return sqd_fail(ctx, SQD_E_LIMIT, "alpha-beta group does not fit in LDS");
    const spin_tables& A = sp->sp[0];
    std::vector<uint32_t> pk(A.nnz_s);
    if (A.nnz_s > 0)
        SQD_HIP(ctx, hipMemcpy(pk.data(), A.s_pk, sizeof(uint32_t) * A.nnz_s, hipMemcpyDeviceToHost));
    const int npair = sp->norb * sp->norb;
    std::vector<std::vector<int>> by(npair);
    for (int64_t e = 0; e < A.nnz_s; ++e) by[(pk[e] >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK].push_back((int)e);
    std::vector<int> grp, cp;
    for (int p = 0; p < npair; ++p) {
        const auto& v = by[p];
        for (size_t k = 0; k < v.size(); k += G) {
            for (int r = 0; r < G; ++r) grp.push_back(k + r < v.size() ? v[k + r] : -1);
            cp.push_back(p);
        }
    }
    if (sp->ab_grp) { (void)hipFree(sp->ab_grp); sp->ab_grp = nullptr; }
    if (sp->ab_chunk_pair) { (void)hipFree(sp->ab_chunk_pair); sp->ab_chunk_pair = nullptr; }
    int rc;
    if ((rc = ensure_ab_row_order(ctx, sp))) return rc;
    if ((rc = sqd_alloc(ctx, (void**)&sp->ab_grp, sizeof(int) * (grp.size() + 1), &sp->bytes))) return rc;
    if ((rc = sqd_alloc(ctx, (void**)&sp->ab_chunk_pair, sizeof(int) * (cp.size() + 1), &sp->bytes))) return rc;
    if (!grp.empty()) {
        SQD_HIP(ctx, hipMemcpy(sp->ab_grp, grp.data(), sizeof(int) * grp.size(), hipMemcpyHostToDevice));
        SQD_HIP(ctx, hipMemcpy(sp->ab_chunk_pair, cp.data(), sizeof(int) * cp.size(), hipMemcpyHostToDevice));
    }
    sp->ab_G = G;
    sp->ab_nchunks = (int)cp.size();
    return SQD_OK;
}

// Singles per chunk of the source-grouped kernel: the most (ai|..) rows that
// fit in LDS beside one FP64 source row (0: fewer than two).
int ab_source_group_size(sqd_ctx* ctx, const sqd_space* sp) {
    const size_t nb = (size_t)sp->sp[1].n, n2 = (size_t)sp->norb * sp->norb;
    auto bytes = [&](int G) { return (nb + 1) * sizeof(double) + (size_t)G * n2 * sizeof(double); };
    for (int G : {8, 4, 3, 2}) if (bytes(G) <= (size_t)ctx->max_lds) return G;
    return 0;
}

// The source-grouped kernel is taken where the pair-grouped chunks would
// hold one or two source rows, or when forced (SQD_TUNE_AB_VARIANT 3).
// Every chunk walks the whole beta table, so grouping more singles per chunk
// cuts the table stream as well as the staging; measured on MI355X
// (alpha-beta FP64 / FP32): 16000-string rows (pair groups of one) 24.8 /
// 14.5 -> 13.8 / 8.5 ms, the full-CI 14-orbital space (pair groups of two,
// 49 singles per source) 6.1 / 4.7 -> 3.6 / 2.8 ms, while on the 4.0e6
// workload (pair groups of four, 17 singles per source) the pair groups win
// (278 against 333 us).
bool ab_use_source_groups(sqd_ctx* ctx, const sqd_space* sp) {
    const int variant = ctx->tune[SQD_TUNE_AB_VARIANT];
    if (variant == 3) return ab_source_group_size(ctx, sp) > 0;
    if (variant != 0 || ctx->tune[SQD_TUNE_AB_GROUP]) return false;
    const int G = ab_group_size(ctx, sp);
    return G >= 1 && G <= 2 && ab_source_group_size(ctx, sp) > G;
}

// Group the alpha singles (CSR positions) by source string, padded to chunks of G.
int ensure_ab_source_groups(sqd_ctx* ctx, sqd_space* sp, int G) {
    if (sp->abs_G == G && sp->abs_grp) return SQD_OK;
    const spin_tables& A = sp->sp[0];
    std::vector<uint32_t> pk(A.nnz_s);
    if (A.nnz_s > 0)
        SQD_HIP(ctx, hipMemcpy(pk.data(), A.s_pk, sizeof(uint32_t) * A.nnz_s, hipMemcpyDeviceToHost));
    std::vector<std::vector<int>> by(A.n);
    for (int64_t e = 0; e < A.nnz_s; ++e) by[pk[e] & SQD_NBR_MASK].push_back((int)e);
    std::vector<int> grp, cs;
    for (int64_t j = 0; j < A.n; ++j) {
        const auto& v = by[j];
        for (size_t k = 0; k < v.size(); k += G) {
            for (int r = 0; r < G; ++r) grp.push_back(k + r < v.size() ? v[k + r] : -1);
            cs.push_back((int)j);
        }
    }
    if (sp->abs_grp) { (void)hipFree(sp->abs_grp); sp->abs_grp = nullptr; }
    if (sp->abs_src) { (void)hipFree(sp->abs_src); sp->abs_src = nullptr; }
    int rc;
    if ((rc = sqd_alloc(ctx, (void**)&sp->abs_grp, sizeof(int) * (grp.size() + 1), &sp->bytes))) return rc;
    if ((rc = sqd_alloc(ctx, (void**)&sp->abs_src, sizeof(int) * (cs.size() + 1), &sp->bytes))) return rc;
    if (!grp.empty()) {
        SQD_HIP(ctx, hipMemcpy(sp->abs_grp, grp.data(), sizeof(int) * grp.size(), hipMemcpyHostToDevice));
        SQD_HIP(ctx, hipMemcpy(sp->abs_src, cs.data(), sizeof(int) * cs.size(), hipMemcpyHostToDevice));
    }
    sp->abs_G = G;
    sp->abs_nchunks = (int)cs.size();
    return SQD_OK;
}

// Y bytes of the grouped alpha-beta path (0 if it is not to be used).
size_t ab_grouped_bytes(sqd_ctx* ctx, const sqd_space* sp, size_t es) {
    const int variant = ctx->tune[SQD_TUNE_AB_VARIANT];
    if (variant == 2) return 0;
    if (ab_group_size(ctx, sp) == 0 && !ab_use_source_groups(ctx, sp)) return 0;
    const size_t bytes = (size_t)sp->sp[0].nnz_s * (size_t)sp->sp[1].nslices * 64 * es;
    const size_t cap = (size_t)64 << 30;   // keep the intermediate below 64 GiB
    if (variant == 0 && bytes > cap) return 0;
    return bytes + 256;
}

template <typename T>
int launch_ab_grouped(sqd_ctx* ctx, sqd_space* sp, const T* C, T* S, T* Y, const T* V, const int* skip) {
    const spin_tables& A = sp->sp[0];
    const spin_tables& B = sp->sp[1];
    int rc;
    if (ab_use_source_groups(ctx, sp)) {
        const int GS = ab_source_group_size(ctx, sp);
        if ((rc = ensure_ab_row_order(ctx, sp)) || (rc = ensure_ab_source_groups(ctx, sp, GS))) return rc;
        if (sp->abs_nchunks > 0) {
            const size_t lds = ((size_t)(B.n + 1) + (size_t)GS * sp->norb * sp->norb) * sizeof(T);
            const int nw = ctx->tune[SQD_TUNE_AB_WAVES] ? ctx->tune[SQD_TUNE_AB_WAVES] : 16;
            abg_args<T> args{C, Y, B.n, (int64_t)B.nslices * 64, sp->abs_grp, nullptr, A.s_pk, B.perm_ab,
                             B.nslices, B.sl_ab_off, B.sell_ab_pk};
            prof_scope ps(ctx, sizeof(T) == 8 ? "k_ab_srcgrouped<double>" : "k_ab_srcgrouped<float>");
#define SQD_ABS_LAUNCH(GG)                                                                                    \
    case GG:                                                                                                  \
        set_lds(k_ab_srcgrouped<T, GG>, (int)lds);                                                            \
        hipLaunchKernelGGL((k_ab_srcgrouped<T, GG>), dim3(sp->abs_nchunks), dim3(64 * nw), lds, ctx->stream,    \
                           args, sp->abs_src, V, sp->norb, skip);                                             \
        break;
            switch (GS) {
                SQD_ABS_LAUNCH(2)
                SQD_ABS_LAUNCH(3)
                SQD_ABS_LAUNCH(4)
                SQD_ABS_LAUNCH(8)
            }
#undef SQD_ABS_LAUNCH
        }
    } else {
    const int G = ab_group_size(ctx, sp);
    if ((rc = ensure_ab_groups_impl(ctx, sp, G))) return rc;
    if (sp->ab_nchunks > 0) {
        const size_t lds = ((size_t)(B.n + 1) * G + (size_t)sp->norb * sp->norb) * sizeof(T);
        // measured on MI355X: 16 waves for FP64, and for FP32 when few rows
        // share each table entry (G <= 2: the loop is latency-bound)
        const int nw = ctx->tune[SQD_TUNE_AB_WAVES] ? ctx->tune[SQD_TUNE_AB_WAVES]
                                                    : ((sizeof(T) == 8 || G <= 2) ? 16 : 8);
        abg_args<T> args{C, Y, B.n, (int64_t)B.nslices * 64, sp->ab_grp, sp->ab_chunk_pair, A.s_pk, B.perm_ab,
                         B.nslices, B.sl_ab_off, B.sell_ab_pk};
        prof_scope ps(ctx, sizeof(T) == 8 ? "k_ab_grouped<double>" : "k_ab_grouped<float>");
#define SQD_ABG_LAUNCH(GG)                                                                                   \
    case GG:                                                                                                 \
        set_lds(k_ab_grouped<T, GG>, (int)lds);                                                              \
        hipLaunchKernelGGL((k_ab_grouped<T, GG>), dim3(sp->ab_nchunks), dim3(64 * nw), lds, ctx->stream, args, \
                           V, sp->norb, skip);                                                               \
        break;
        switch (G) {
            SQD_ABG_LAUNCH(1)
            SQD_ABG_LAUNCH(2)
            SQD_ABG_LAUNCH(4)
            SQD_ABG_LAUNCH(8)
        }
#undef SQD_ABG_LAUNCH
    }
    }
    const unsigned gx = (unsigned)std::min<int64_t>(A.n, 1 << 20);
    prof_scope ps(ctx, sizeof(T) == 8 ? "k_ab_gather<double>" : "k_ab_gather<float>");
    const int64_t ldy = (int64_t)B.nslices * 64;
    const int64_t row_bytes = B.n * (int64_t)sizeof(T);
    if (A.n == 0 || B.n == 0) return SQD_OK;
    // measured on MI355X (4.0e6-determinant workload): 1024 threads per row
    // for FP64, 512 for FP32
    const dim3 gblock(sizeof(T) == 8 ? 1024 : 512);
    if (row_bytes <= std::min<int64_t>(kGatherStageBytes, (int64_t)ctx->max_lds)) {
        set_lds(k_ab_gather<T, true>, (int)row_bytes);
        hipLaunchKernelGGL((k_ab_gather<T, true>), dim3(gx), gblock, (size_t)row_bytes, ctx->stream, Y, S, A.n,
                           B.n, ldy, B.perm_ab, A.s_off, sp->ab_row_order, skip);
    } else {
        hipLaunchKernelGGL((k_ab_gather<T, false>), dim3(gx), gblock, 0, ctx->stream, Y, S, A.n, B.n, ldy,
                           B.perm_ab, A.s_off, sp->ab_row_order, skip);
    }
    SQD_HIP(ctx, hipGetLastError());
    return SQD_OK;
}

}  // namespace

int sqd_ensure_ab_groups(sqd_ctx* ctx, sqd_space* sp, int G) { return ensure_ab_groups_impl(ctx, sp, G); }
int sqd_ensure_ab_source_groups(sqd_ctx* ctx, sqd_space* sp, int G) {
    int rc = ensure_ab_row_order(ctx, sp);
    return rc ? rc : ensure_ab_source_groups(ctx, sp, G);
}

int sqd_ensure_diag(sqd_ctx* ctx, sqd_space* sp) {
    int rc = sqd_build_values(ctx, sp);
    if (rc) return rc;
    if (sp->diag_version == ctx->ham_version) return SQD_OK;
    const spin_tables& A = sp->sp[0];
    const spin_tables& B = sp->sp[1];
    if (!sp->diag) {
        if ((rc = sqd_alloc(ctx, (void**)&sp->diag, sizeof(double) * (sp->dim + 1), &sp->bytes))) return rc;
        if ((rc = sqd_alloc(ctx, (void**)&sp->ua, sizeof(double) * (A.n * sp->norb + 1), &sp->bytes))) return rc;
    }
    hipLaunchKernelGGL(k_ua, dim3(nblk(A.n * sp->norb, 256)), dim3(256), 0, ctx->stream, A.str, sp->nw, A.n,
                       sp->norb, ctx->jdiag, sp->ua);
    hipLaunchKernelGGL(k_diag, dim3(nblk(sp->dim, 256)), dim3(256), 0, ctx->stream, A.e_same, B.e_same, sp->ua,
                       B.str, sp->nw, A.n, B.n, sp->norb, ctx->ecore, sp->diag);
    SQD_HIP(ctx, hipGetLastError());
    sp->diag_version = ctx->ham_version;
    return SQD_OK;
}

int sqd_sigma_auto_path(sqd_ctx* ctx, const sqd_space* sp, int precision) {
    (void)sp; (void)precision;
    if (ctx->tune[SQD_TUNE_AB_PATH]) return ctx->tune[SQD_TUNE_AB_PATH];
    return SQD_AB_DIRECT;
}

// True when a product with these arguments would allocate, copy or
// synchronise nothing: the space's values and diagonal are current and the
// alpha-beta path's per-space schedule exists.  (The context scratch is
// checked separately, by its size.)
bool sqd_sigma_prepared(sqd_ctx* ctx, const sqd_space* sp, int precision, unsigned mask, int ab_path) {
    if (sp->values_version != ctx->ham_version || sp->diag_version != ctx->ham_version) return false;
    const size_t es0 = precision == SQD_FP64 ? 8 : 4;
    for (int spin = 0; spin < 2; ++spin) {   // windowed same-spin tables of either spin
        if (!(mask & (spin == 0 ? SQD_TERM_AA : SQD_TERM_BB))) continue;
        const spin_tables& col = sp->sp[spin].alias ? sp->sp[0] : sp->sp[spin];
        const spin_tables& row = sp->sp[1 - spin].alias ? sp->sp[0] : sp->sp[1 - spin];
        if (use_window(ctx, sp->sp[1 - spin].n, sp->sp[spin].n, sp->norb, es0)) {
            const int W = sqd_window_count(ctx, sp->sp[spin].n);
            if (W == 0 || col.win_W != W || col.win_values_version != ctx->ham_version || !row.wg64 ||
                row.wg_version != ctx->ham_version || (W > 1 && sp->win_P_bytes < sqd_window_scratch_bytes(sp)))
                return false;
        }
    }
    if (!(mask & SQD_TERM_AB)) return true;
    if (ab_path == SQD_AB_AUTO) ab_path = sqd_sigma_auto_path(ctx, sp, precision);
    if (ab_path == SQD_AB_KH) return sp->kh_map != nullptr && sp->ab_rev != nullptr;
    const size_t es = precision == SQD_FP64 ? 8 : 4;
    if (ab_grouped_bytes(ctx, sp, es) == 0) return true;   // row-staged kernel: nothing per space
    if (ab_use_source_groups(ctx, sp))
        return sp->abs_grp != nullptr && sp->abs_G == ab_source_group_size(ctx, sp) && sp->ab_row_order != nullptr;
    return sp->ab_grp != nullptr && sp->ab_G == ab_group_size(ctx, sp) && sp->ab_row_order != nullptr;
}

// True when the arrays that a space's first product builds exist for a
// product with these arguments: the diagonal, and for same-spin rows too long
// to stage four whole the windowed tables of the column spin, the cross-spin
// table of the row spin and the partial-sum scratch.  (Their values may still
// be stale: those are refreshed in place.)
bool sqd_space_built_for(sqd_ctx* ctx, const sqd_space* sp, int precision, unsigned mask) {
    if (!sp->diag || !sp->ua) return false;
    const size_t es = precision == SQD_FP64 ? 8 : 4;
    for (int spin = 0; spin < 2; ++spin) {
        if (!(mask & (spin == 0 ? SQD_TERM_AA : SQD_TERM_BB))) continue;
        const spin_tables& col = sp->sp[spin].alias ? sp->sp[0] : sp->sp[spin];
        const spin_tables& row = sp->sp[1 - spin].alias ? sp->sp[0] : sp->sp[1 - spin];
        if (use_window(ctx, sp->sp[1 - spin].n, sp->sp[spin].n, sp->norb, es)) {
            const int W = sqd_window_count(ctx, sp->sp[spin].n);
            if (W == 0 || col.win_W != W || !row.wg64 || (W > 1 && sp->win_P_bytes < sqd_window_scratch_bytes(sp)))
                return false;
        }
    }
    return true;
}

// Context scratch (grown on demand): FP64 path 2*dim doubles, FP32 path 4*dim floats.
static int space_scratch_get(sqd_ctx* ctx, sqd_space* sp, size_t bytes, void** out) {
    (void)sp;
    int rc = SQD_E_OOM;
    void* p = sqd_ctx_scratch(ctx, bytes, &rc);
    if (!p) {
        if (rc == SQD_E_STATE)
            return sqd_fail(ctx, rc, "product scratch of " + std::to_string(bytes) +
                                         " bytes not allocated before the stream capture");
        return sqd_fail(ctx, SQD_E_OOM, "scratch allocation failed (" + std::to_string(bytes) + " bytes)");
    }
    *out = p;
    return SQD_OK;
}

int sqd_sigma_impl(sqd_ctx* ctx, sqd_space* sp, const double* c, double* sigma, int precision, unsigned mask,
                   int ab_path, const float* c32_in, const int* skip, void* ext_scratch, size_t ext_bytes) {
    int rc = sqd_ensure_diag(ctx, sp);
    if (rc) return rc;
    // a caller-provided scratch: the row-staged alpha-beta kernel (no
    // intermediate) and nothing taken from the context
    auto scratch_get = [&](size_t bytes, void** out) -> int {
        if (!ext_scratch) return space_scratch_get(ctx, sp, bytes, out);
        if (bytes > ext_bytes)
            return sqd_fail(ctx, SQD_E_LIMIT, "product needs " + std::to_string(bytes) + " scratch bytes, " +
                                                  std::to_string(ext_bytes) + " available");
        *out = ext_scratch;
        return SQD_OK;
    };
    const spin_tables& A = sp->sp[0];
    const spin_tables& B = sp->sp[1];
    const int64_t na = A.n, nb = B.n, dim = sp->dim;
    const int norb = sp->norb;
    if (ab_path == SQD_AB_AUTO) ab_path = sqd_sigma_auto_path(ctx, sp, precision);
    const double* diag = (mask & SQD_TERM_DIAG) ? sp->diag : nullptr;
    const unsigned g = nblk(dim, 256);
    const dim3 tgrid(nblk(nb, 64), nblk(na, 64)), tgridT(nblk(na, 64), nblk(nb, 64));
    if (precision == SQD_FP64) {
        void* scr = nullptr;
        const size_t ybytes = (!(mask & SQD_TERM_AB) || ext_scratch) ? 0
                              : (ab_path == SQD_AB_KH ? sqd_kh_bytes(sp, 8) : ab_grouped_bytes(ctx, sp, 8));
        if ((rc = scratch_get(sizeof(double) * 2 * (dim + 64) + ybytes, &scr))) return rc;
        double* Ct = (double*)scr;
        double* Yt = Ct + dim + 64;
        double* Yab = Yt + dim + 64;
        // beta-beta (with the diagonal) writes sigma first, so that its
        // scattered stores need no read of sigma; the alpha-alpha term reads
        // the columns of C and adds into sigma (row-staged kernel with eight
        // rows, and the windowed kernel through its placing pass), or comes
        // back through a coalesced transpose that adds
        bool written = false;
        if (mask & SQD_TERM_BB) {
            if ((rc = launch_same_spin<double>(ctx, sp, c, sigma, na, nb, B, A, ctx->jk64, norb, diag, 0, skip,
                                               "k_same_spin<double>[bb]")))
                return rc;
            written = true;
        } else if (diag) {
            hipLaunchKernelGGL(k_diag_apply, dim3(g), dim3(256), 0, ctx->stream, diag, c, sigma, dim, 0, skip);
            written = true;
        }
        if ((mask & SQD_TERM_AA) && aa_in_place(ctx, nb, na, norb, 8)) {
            // beta rows read from the columns of C, added into sigma
            if ((rc = launch_same_spin<double>(ctx, sp, c, sigma, nb, na, A, B, ctx->jk64, norb, nullptr,
                                               written ? 1 : 0, skip, "k_same_spin<double>[aa]", 1)))
                return rc;
            written = true;
        } else if (mask & SQD_TERM_AA) {
            {
                prof_scope pt(ctx, "k_transpose<double>");
                hipLaunchKernelGGL((k_transpose<double, double, false>), tgrid, dim3(256), 0, ctx->stream, c, Ct, na,
                                   nb, skip);
            }
            if ((rc = launch_same_spin<double>(ctx, sp, Ct, Yt, nb, na, A, B, ctx->jk64, norb, nullptr, 0, skip,
                                               "k_same_spin<double>[aa]"))) return rc;
            {
                prof_scope pt(ctx, "k_transpose<double>");
                if (written)
                    hipLaunchKernelGGL((k_transpose<double, double, true>), tgridT, dim3(256), 0, ctx->stream, Yt,
                                       sigma, nb, na, skip);
                else
                    hipLaunchKernelGGL((k_transpose<double, double, false>), tgridT, dim3(256), 0, ctx->stream, Yt,
                                       sigma, nb, na, skip);
            }
            written = true;
        }
        if (!written) hipLaunchKernelGGL(k_fill<double>, dim3(g), dim3(256), 0, ctx->stream, sigma, dim, 0.0, skip);
        if (mask & SQD_TERM_AB) {
            if (ab_path == SQD_AB_KH) {
                if ((rc = sqd_sigma_ab_kh(ctx, sp, c, sigma, Yab, 0, skip))) return rc;
            } else if (ybytes) {
                if ((rc = launch_ab_grouped<double>(ctx, sp, c, sigma, Yab, ctx->eri, skip))) return rc;
            } else if ((rc = launch_ab_direct<double>(ctx, sp, c, sigma, ctx->eri, skip))) {
                return rc;
            }
        }
        SQD_HIP(ctx, hipGetLastError());
        return SQD_OK;
    }
    // FP32 off-diagonal terms
    void* scr = nullptr;
    const size_t ybytes = (!(mask & SQD_TERM_AB) || ext_scratch) ? 0
                          : (ab_path == SQD_AB_KH ? sqd_kh_bytes(sp, 4) : ab_grouped_bytes(ctx, sp, 4));
    if ((rc = scratch_get(sizeof(float) * 4 * (dim + 64) + ybytes, &scr))) return rc;
    float* C32 = (float*)scr;
    float* Ct32 = C32 + dim + 64;
    float* Yt32 = Ct32 + dim + 64;
    float* S32 = Yt32 + dim + 64;
    float* Yab = S32 + dim + 64;
    const float* Cin = c32_in;
    if (!Cin) {
        hipLaunchKernelGGL((k_convert<double, float>), dim3(g), dim3(256), 0, ctx->stream, c, C32, dim, skip);
        Cin = C32;
    }
    bool written = false;
    if (mask & SQD_TERM_BB) {
        if ((rc = launch_same_spin<float>(ctx, sp, Cin, S32, na, nb, B, A, ctx->jk32, norb, nullptr, 0, skip,
                                          "k_same_spin<float>[bb]")))
            return rc;
        written = true;
    }
    if ((mask & SQD_TERM_AA) && aa_in_place(ctx, nb, na, norb, 4)) {
        if ((rc = launch_same_spin<float>(ctx, sp, Cin, S32, nb, na, A, B, ctx->jk32, norb, nullptr, written ? 1 : 0,
                                          skip, "k_same_spin<float>[aa]", 1)))
            return rc;
        written = true;
    } else if (mask & SQD_TERM_AA) {
        {
            prof_scope pt(ctx, "k_transpose<float>");
            hipLaunchKernelGGL((k_transpose<float, float, false>), tgrid, dim3(256), 0, ctx->stream, Cin, Ct32, na, nb,
                               skip);
        }
        if ((rc = launch_same_spin<float>(ctx, sp, Ct32, Yt32, nb, na, A, B, ctx->jk32, norb, nullptr, 0, skip,
                                              "k_same_spin<float>[aa]"))) return rc;
        {
            prof_scope pt(ctx, "k_transpose<float>");
            if (written)
                hipLaunchKernelGGL((k_transpose<float, float, true>), tgridT, dim3(256), 0, ctx->stream, Yt32, S32, nb,
                                   na, skip);
            else
                hipLaunchKernelGGL((k_transpose<float, float, false>), tgridT, dim3(256), 0, ctx->stream, Yt32, S32, nb,
                                   na, skip);
        }
        written = true;
    }
    if (!written) hipLaunchKernelGGL(k_fill<float>, dim3(g), dim3(256), 0, ctx->stream, S32, dim, 0.0f, skip);
    if (mask & SQD_TERM_AB) {
        if (ab_path == SQD_AB_KH) {
            if ((rc = sqd_sigma_ab_kh(ctx, sp, Cin, S32, Yab, 1, skip))) return rc;
        } else if (ybytes) {
            if ((rc = launch_ab_grouped<float>(ctx, sp, Cin, S32, Yab, ctx->eri32, skip))) return rc;
        } else if ((rc = launch_ab_direct<float>(ctx, sp, Cin, S32, ctx->eri32, skip))) {
            return rc;
        }
    }
    hipLaunchKernelGGL(k_combine, dim3(g), dim3(256), 0, ctx->stream, diag, c, S32, sigma, dim, skip);
    SQD_HIP(ctx, hipGetLastError());
    return SQD_OK;
}
