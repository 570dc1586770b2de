// Same-spin term (Sec. IV: the alpha-alpha and beta-beta task types) for rows
// too long to stage several whole in LDS.
//
// The row-staged kernel (sigma_body.h) keeps R rows of C in LDS and walks the
// column spin's whole sliced table once per row block; when a row alone fills
// the LDS (R = 1), every row streams the whole table through the caches.
// Here the source strings of the column spin are dealt into W interleaved
// windows (window w: the sources j with j mod W = w, local index j / W): a
// workgroup stages R rows x one window of C and walks that window's part of
// the table, for all windows in turn, so the table is streamed once per R
// rows.  Every window's part keeps the targets in the order of the whole
// sliced table (rows sorted by total length), so a lane owns the same targets
// in every window; interleaving spreads each target's sources evenly over the
// windows, which keeps the 64-lane slices of every part nearly as tight as
// the whole table's.  A lane's partial sums go to a scratch row in slot order
// (coalesced, read back by the same lane in the next window); the last
// window leaves them there too, and a coalesced pass places the targets
// (adding the diagonal for row-major output).  The cross-spin part of the
// singles comes from a per-string table wg[pq][s] = sum_{k in s} (pq|kk) of
// the row spin (global memory) instead of an LDS copy per row, held with the
// strings fastest so that a lane reads the values of its row block for one
// pair as one 64-byte piece (2.56e8-determinant workload, same-spin terms:
// FP64 26.2 / 23.2 -> 24.0 / 21.4 ms, FP32 16.1 / 13.4 -> 12.9 / 11.0 ms
// against eight scattered loads per single from wg[s][pq]).  Neighbours of
// the doubles are local indices below the window width, held as 16-bit
// values (same workload: 26.9 -> 26.2 ms FP64 beta-beta, 3% on each term).
#include <algorithm>
#include <numeric>

#include "sqd_internal.h"

#include "sigma_body.h"

namespace {

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// strings of the cross-spin table, padded to whole 16-string blocks (the
// rows staged per workgroup, 8 or 16, read one aligned 64-byte piece)
inline int64_t sqd_wtable_ld(int64_t n) { return (n + 15) / 16 * 16; }

// wg[pq * ldw + s] = sum over occupied k of s (ascending) of jk[k * norb2 + pq]
// (zero for the padding strings n <= s < ldw)
__global__ void k_wtable(const uint64_t* __restrict__ str, int nw, int64_t n, int64_t ldw, int norb,
                         const double* __restrict__ jk, double* __restrict__ w64, float* __restrict__ w32) {
    const int norb2 = norb * norb;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ldw * norb2) return;
    const int pq = (int)(idx / ldw);
    const int64_t s = idx - (int64_t)pq * ldw;
    double acc = 0.0;
    if (s < n) str_for_each(str + s * nw, nw, [&](int k) { acc += jk[(int64_t)k * norb2 + pq]; });
    w64[idx] = acc;
    w32[idx] = (float)acc;
}

template <typename T>
__global__ void k_win_values(const int* __restrict__ csr, int64_t m, const T* __restrict__ v, T* __restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int src = csr[k];
    out[k] = (src >= 0) ? v[src] : (T)0;
}

template <typename T>
struct win_args {
    const T* X;                 // nrows x ncols
    T* Y;
    T* P;                       // partial sums: nrows x (nslices * 64), slot order
    int64_t nrows, ncols;
    int W, width, nslices;
    const int* perm;            // nslices * 64: target of each slot (n = padding)
    const int* s_off;           // W x (nslices + 1)
    const int* d_off;
    const uint32_t* s_pk;
    const T* s_val;
    const uint16_t* d_nbr;
    const T* d_val;
    const T* wg;                // row spin: norb2 x ldw (strings padded to ldw)
    int64_t ldw;
    int norb;
    int colmajor;               // X, Y hold the transposes: (row, col) at col * nrows + row
    int accumulate;             // Y += (else Y =)
    int slot_out;               // the last window also writes P (slot order); Y is left alone
};

// One workgroup per block of R rows; windows in turn.  LDS: xs[(width + 1) * R]
// in the lds_cols<T, R> layout (column width is the zero slot).  The loop
// over a slice's entries waits on the table, which streams from beyond the
// L2, so the partial sums of the earlier windows and the first batch of
// doubles are loaded before the singles, and each single's successor loads
// while its cross-spin terms are read (measured on MI355X, 2.56e8-determinant
// workload, beta-beta FP64: 30.7 -> 27.9 ms; double-buffering the doubles
// batches as well needs more than the 128 VGPRs of 16 waves per CU).
template <typename T, int R>
__global__ void __launch_bounds__(1024) k_same_spin_win(win_args<T> a, const int* __restrict__ skip) {
    if (skip && *skip) return;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* xs = reinterpret_cast<T*>(lds_raw);
    using L = lds_cols<T, R>;
    constexpr int kD = 8;   // doubles per batch
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63, nw = nthr >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * R;
    const int norb2 = a.norb * a.norb;
    const int64_t ldp = (int64_t)a.nslices * 64;
    // rows past the end read the last row (their results are not stored)
    auto rowc = [&](int r) -> int64_t { return row0 + r < a.nrows ? row0 + r : a.nrows - 1; };
    for (int w = 0; w < a.W; ++w) {
        // sources w, w + W, w + 2W, ... as local columns 0, 1, 2, ...
        const int len = (int)((a.ncols - w + a.W - 1) / a.W);
        __syncthreads();   // the previous window is done with xs
        for (int c0 = tid; c0 <= a.width; c0 += 2 * nthr) {
            T v[2][R];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int c = c0 + u * nthr;
                const int cc = c < len ? c : 0;
                const int64_t src = w + (int64_t)cc * a.W;
#pragma unroll
                for (int r = 0; r < R; ++r)
                    v[u][r] = a.colmajor ? a.X[src * a.nrows + rowc(r)] : a.X[rowc(r) * a.ncols + src];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int c = c0 + u * nthr;
                if (c > a.width) continue;
#pragma unroll
                for (int r = 0; r < R; ++r)
                    xs[L::idx(c, r)] = (c < len && row0 + r < a.nrows) ? v[u][r] : (T)0;
            }
        }
        __syncthreads();
        const int* so = a.s_off + (int64_t)w * (a.nslices + 1);
        const int* dof = a.d_off + (int64_t)w * (a.nslices + 1);
        const bool first = (w == 0), last = (w == a.W - 1);
        for (int sl = wave; sl < a.nslices; sl += nw) {
            const int64_t slot = (int64_t)sl * 64 + lane;
            T acc[R], prev[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                acc[r] = (T)0;
                prev[r] = first ? (T)0 : __builtin_nontemporal_load(a.P + rowc(r) * ldp + slot);
            }
            const int d0 = dof[sl], d1 = dof[sl + 1];
            const int nfull = (d1 - d0) / kD;
            int nA[kD];
            T vA[kD];
            auto load = [&](int k, int (&nb)[kD], T (&v)[kD]) {
                const uint16_t* pn = a.d_nbr + (int64_t)k * 64 + lane;
                const T* pv = a.d_val + (int64_t)k * 64 + lane;
#pragma unroll
                for (int u = 0; u < kD; ++u) {
                    nb[u] = pn[u * 64];
                    v[u] = pv[u * 64];
                }
            };
            auto use = [&](const int (&nb)[kD], const T (&v)[kD]) {
#pragma unroll
                for (int u = 0; u < kD; u += 2) {
                    T x0[R], x1[R];
                    L::load(xs, nb[u], x0);
                    L::load(xs, nb[u + 1], x1);
#pragma unroll
                    for (int r = 0; r < R; ++r) acc[r] += v[u] * x0[r];
#pragma unroll
                    for (int r = 0; r < R; ++r) acc[r] += v[u + 1] * x1[r];
                    __builtin_amdgcn_sched_barrier(0);   // two entries' LDS reads at a time
                }
            };
            if (nfull > 0) load(d0, nA, vA);
            // singles: the next entry loads while the cross-spin terms of
            // the current one are read
            const int s0 = so[sl], s1 = so[sl + 1];
            uint32_t en = 0;
            T vn = (T)0;
            if (s0 < s1) {
                en = a.s_pk[(int64_t)s0 * 64 + lane];
                vn = a.s_val[(int64_t)s0 * 64 + lane];
            }
            for (int k = s0; k < s1; ++k) {
                const uint32_t e = en;
                const T v = vn;
                if (k + 1 < s1) {
                    en = a.s_pk[(int64_t)(k + 1) * 64 + lane];
                    vn = a.s_val[(int64_t)(k + 1) * 64 + lane];
                }
                const int pair = (int)((e >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK);
                // the R values of the row block for this pair: 64
                // contiguous bytes (row0 is a multiple of R, ldw of 16)
                T wv[R];
                {
                    using V4 = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
                    constexpr int kP = (int)(16 / sizeof(T));
                    const V4* wp = reinterpret_cast<const V4*>(a.wg + (int64_t)pair * a.ldw + row0);
#pragma unroll
                    for (int q = 0; q < R / kP; ++q) {
                        const V4 x = wp[q];
                        const T* xv = reinterpret_cast<const T*>(&x);
#pragma unroll
                        for (int i = 0; i < kP; ++i) wv[q * kP + i] = xv[i];
                    }
                }
                T xr[R];
                L::load(xs, (int)(e & SQD_NBR_MASK), xr);
                const bool neg = (e >> 31) != 0;
#pragma unroll
                for (int r = 0; r < R; ++r) acc[r] += (v + (neg ? -wv[r] : wv[r])) * xr[r];
            }
            for (int b = 0; b < nfull; ++b) {
                if (b > 0) load(d0 + b * kD, nA, vA);
                use(nA, vA);
            }
            for (int k = d0 + nfull * kD; k < d1; ++k) {
                const int nb1 = a.d_nbr[(int64_t)k * 64 + lane];
                const T v1 = a.d_val[(int64_t)k * 64 + lane];
                T xr[R];
                L::load(xs, nb1, xr);
#pragma unroll
                for (int r = 0; r < R; ++r) acc[r] += v1 * xr[r];
            }
            // the lane keeps its slot in every window: partial sums in slot
            // order (its own earlier writes, read back in program order;
            // non-temporal, so that the scratch of all row blocks in flight,
            // larger than the caches, does not evict the table: 2.56e8
            // workload, same box, 28.0 -> 26.6-27.1 ms per same-spin term);
            // with slot_out the last window writes P as well, for the
            // coalesced pass that places the targets; else it writes them
            const int t = a.perm[slot];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t row = row0 + r;
                if (row >= a.nrows) continue;
                const T val = acc[r] + prev[r];
                if (!last || a.slot_out) {
                    __builtin_nontemporal_store(val, a.P + row * ldp + slot);
                } else if (t < a.ncols) {
                    const int64_t o = a.colmajor ? (int64_t)t * a.nrows + row : row * a.ncols + t;
                    a.Y[o] = a.accumulate ? a.Y[o] + val : val;
                }
            }
        }
    }
}

// Row-major output of the windowed kernel from the slot-ordered sums in P:
// Y[row][t] (=|+=) P[row][islot[t]] (+ diag * X, the FP64 diagonal term).
// One workgroup per row: the reads of P stay within one row (in the L2 after
// their first touch), everything else is coalesced.  Scattered stores of the
// targets straight from the last window cost more (2.56e8-determinant
// workload, beta-beta: FP64 23.9 ms against 20.5 ms with the stores in slot
// order, FP32 12.9 against 9.9 ms).
template <typename T>
__global__ void __launch_bounds__(256) k_win_unperm(const T* __restrict__ P, int64_t ldp, const int* __restrict__ islot,
                                                    const T* __restrict__ X, const double* __restrict__ diag,
                                                    T* __restrict__ Y, int64_t nrows, int64_t ncols, int accumulate,
                                                    const int* __restrict__ skip) {
    if (skip && *skip) return;
    for (int64_t row = blockIdx.x; row < nrows; row += gridDim.x) {
        const T* prow = P + row * ldp;
        for (int64_t t = threadIdx.x; t < ncols; t += blockDim.x) {
            const int64_t o = row * ncols + t;
            T v = prow[islot[t]];
            if (diag) v += (T)(diag[o] * (double)X[o]);
            if (accumulate) v += Y[o];
            Y[o] = v;
        }
    }
}

// The same with the scratch row staged in LDS first (coalesced reads, each
// line of P fetched once), for rows of ldp * sizeof(T) bytes up to the LDS
// size: the gathers straight from P re-fetch lines evicted by the other rows
// in flight (2.56e8-determinant workload, beta-beta placing pass: FP64 1.76
// -> 0.74 ms, FP32 1.26 -> 0.35 ms).
template <typename T>
__global__ void __launch_bounds__(1024) k_win_unperm_lds(const T* __restrict__ P, int64_t ldp,
                                                         const int* __restrict__ islot, const T* __restrict__ X,
                                                         const double* __restrict__ diag, T* __restrict__ Y,
                                                         int64_t nrows, int64_t ncols, int accumulate,
                                                         const int* __restrict__ skip) {
    if (skip && *skip) return;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* ps = reinterpret_cast<T*>(lds_raw);
    constexpr int kB = 8;
    const int64_t step = (int64_t)blockDim.x * kB;
    for (int64_t row = blockIdx.x; row < nrows; row += gridDim.x) {
        const T* prow = P + row * ldp;
        __syncthreads();   // the previous row's reads of ps are done
        for (int64_t q0 = threadIdx.x; q0 < ldp; q0 += step) {
            T v[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int64_t q = q0 + (int64_t)u * blockDim.x;
                v[u] = q < ldp ? __builtin_nontemporal_load(prow + q) : (T)0;
            }
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int64_t q = q0 + (int64_t)u * blockDim.x;
                if (q < ldp) ps[q] = v[u];
            }
        }
        __syncthreads();
        for (int64_t t = threadIdx.x; t < ncols; t += blockDim.x) {
            const int64_t o = row * ncols + t;
            T v = ps[islot[t]];
            if (diag) v += (T)(diag[o] * (double)X[o]);
            if (accumulate) v += Y[o];
            Y[o] = v;
        }
    }
}

// Column-major output (Y[t * nrows + row]) from the slot-ordered sums in P:
// 64 x 64 tiles of (rows, slots) through LDS, each target's 64 rows read
// and written as 64 contiguous values.  The last window's adds into 64-byte
// pieces of scattered targets cost more (2.56e8-determinant workload,
// alpha-alpha term adding into sigma: FP64 24.1 ms against 19.2 + 1.9 ms,
// FP32 14.4 against 10.2 + 0.9 ms).
template <typename T>
__global__ void __launch_bounds__(256) k_win_unperm_t(const T* __restrict__ P, int64_t ldp, const int* __restrict__ perm,
                                                      T* __restrict__ Y, int64_t nrows, int64_t ncols, int accumulate,
                                                      const int* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ T tile[64][65];
    const int64_t s0 = (int64_t)blockIdx.x * 64, r0 = (int64_t)blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const int64_t r = r0 + i;
        tile[i][tx] = r < nrows ? P[r * ldp + s0 + tx] : (T)0;
    }
    __syncthreads();
    const int64_t r = r0 + tx;
    for (int j = ty; j < 64; j += 4) {
        const int t = perm[s0 + j];
        if (t < ncols && r < nrows) {
            const int64_t o = (int64_t)t * nrows + r;
            const T v = tile[tx][j];
            Y[o] = accumulate ? Y[o] + v : v;
        }
    }
}

// Build the windowed tables of spin t for W interleaved windows (host pass
// over the canonical CSR, which lists for every string its in-set
// neighbours); targets in the order of the whole sliced table (perm_ss).
int build_window_tables(sqd_ctx* ctx, sqd_space* sp, spin_tables& t, int W) {
    sqd_free_window_tables(&t);
    const int64_t n = t.n;
    const int ns = t.nslices;
    const int width = (int)((n + W - 1) / W);
    std::vector<int> soff(n + 1), doff(n + 1), dnbr(t.nnz_d > 0 ? t.nnz_d : 1), perm((size_t)ns * 64);
    std::vector<uint32_t> spk(t.nnz_s > 0 ? t.nnz_s : 1);
    SQD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    SQD_HIP(ctx, hipMemcpy(soff.data(), t.s_off, sizeof(int) * (n + 1), hipMemcpyDeviceToHost));
    SQD_HIP(ctx, hipMemcpy(doff.data(), t.d_off, sizeof(int) * (n + 1), hipMemcpyDeviceToHost));
    SQD_HIP(ctx, hipMemcpy(perm.data(), t.perm_ss, sizeof(int) * perm.size(), hipMemcpyDeviceToHost));
    if (t.nnz_s > 0) SQD_HIP(ctx, hipMemcpy(spk.data(), t.s_pk, sizeof(uint32_t) * t.nnz_s, hipMemcpyDeviceToHost));
    if (t.nnz_d > 0) SQD_HIP(ctx, hipMemcpy(dnbr.data(), t.d_nbr, sizeof(int) * t.nnz_d, hipMemcpyDeviceToHost));
    // slot of every target (perm_ss lists each target once, padding = n)
    std::vector<int> islot(n > 0 ? n : 1, -1);
    for (size_t q = 0; q < perm.size(); ++q)
        if (perm[q] >= 0 && perm[q] < n) {
            if (islot[perm[q]] >= 0) return sqd_fail(ctx, SQD_E_STATE, "target listed twice in the sliced table");
            islot[perm[q]] = (int)q;
        }
    for (int64_t r = 0; r < n; ++r)
        if (islot[r] < 0) return sqd_fail(ctx, SQD_E_STATE, "target missing from the sliced table");
    // per (window, target) entry counts, then slice widths per window
    std::vector<int> cs((size_t)W * n, 0), cd((size_t)W * n, 0);
    for (int64_t r = 0; r < n; ++r) {
        for (int e = soff[r]; e < soff[r + 1]; ++e) cs[(size_t)((spk[e] & SQD_NBR_MASK) % W) * n + r] += 1;
        for (int e = doff[r]; e < doff[r + 1]; ++e) cd[(size_t)(dnbr[e] % W) * n + r] += 1;
    }
    std::vector<int> so((size_t)W * (ns + 1)), dof((size_t)W * (ns + 1));
    int64_t tot_s = 0, tot_d = 0;
    for (int w = 0; w < W; ++w) {
        so[(size_t)w * (ns + 1)] = (int)tot_s;
        dof[(size_t)w * (ns + 1)] = (int)tot_d;
        for (int sl = 0; sl < ns; ++sl) {
            int ms = 0, md = 0;
            for (int l = 0; l < 64; ++l) {
                const int tg = perm[(size_t)sl * 64 + l];
                if (tg < n) {
                    ms = std::max(ms, cs[(size_t)w * n + tg]);
                    md = std::max(md, cd[(size_t)w * n + tg]);
                }
            }
            tot_s += ms;
            tot_d += md;
            so[(size_t)w * (ns + 1) + sl + 1] = (int)tot_s;
            dof[(size_t)w * (ns + 1) + sl + 1] = (int)tot_d;
        }
    }
    if ((tot_s + tot_d) * 64 >= (1LL << 31)) return sqd_fail(ctx, SQD_E_LIMIT, "windowed table exceeds 2^31 slots");
    if (width >= 65535) return sqd_fail(ctx, SQD_E_LIMIT, "window width exceeds 16-bit local indices");
    // slots: a target's entries of window w in CSR order; padding points at
    // the zero column (local index width)
    std::vector<uint32_t> hs_pk((size_t)tot_s * 64 + 1);
    std::vector<uint16_t> hd_nbr((size_t)tot_d * 64 + 1);
    std::vector<int> hs_csr((size_t)tot_s * 64 + 1, -1), hd_csr((size_t)tot_d * 64 + 1, -1);
    for (int w = 0; w < W; ++w)
        for (int sl = 0; sl < ns; ++sl) {
            const int sb = so[(size_t)w * (ns + 1) + sl], se = so[(size_t)w * (ns + 1) + sl + 1];
            const int db = dof[(size_t)w * (ns + 1) + sl], de = dof[(size_t)w * (ns + 1) + sl + 1];
            for (int l = 0; l < 64; ++l) {
                const int tg = perm[(size_t)sl * 64 + l];
                int col = sb;
                if (tg < n)
                    for (int e = soff[tg]; e < soff[tg + 1]; ++e) {
                        const uint32_t src = spk[e] & SQD_NBR_MASK;
                        if ((int)(src % W) != w) continue;
                        hs_pk[(size_t)col * 64 + l] = (src / W) | (spk[e] & ~SQD_NBR_MASK);
                        hs_csr[(size_t)col * 64 + l] = e;
                        ++col;
                    }
                for (; col < se; ++col) hs_pk[(size_t)col * 64 + l] = (uint32_t)width;
                col = db;
                if (tg < n)
                    for (int e = doff[tg]; e < doff[tg + 1]; ++e) {
                        const int src = dnbr[e];
                        if (src % W != w) continue;
                        hd_nbr[(size_t)col * 64 + l] = (uint16_t)(src / W);
                        hd_csr[(size_t)col * 64 + l] = e;
                        ++col;
                    }
                for (; col < de; ++col) hd_nbr[(size_t)col * 64 + l] = (uint16_t)width;
            }
        }
    int rc;
    int64_t bytes = 0;
    const size_t S = (size_t)tot_s * 64 + 1, D = (size_t)tot_d * 64 + 1;
    if ((rc = sqd_alloc(ctx, (void**)&t.win_s_off, sizeof(int) * so.size(), &bytes)) ||
        (rc = sqd_alloc(ctx, (void**)&t.win_d_off, sizeof(int) * dof.size(), &bytes)) ||
        (rc = sqd_alloc(ctx, (void**)&t.win_s_pk, sizeof(uint32_t) * S, &bytes)) ||
        (rc = sqd_alloc(ctx, (void**)&t.win_s_csr, sizeof(int) * S, &bytes)) ||
        (rc = sqd_alloc(ctx, (void**)&t.win_d_nbr, sizeof(uint16_t) * D, &bytes)) ||
        (rc = sqd_alloc(ctx, (void**)&t.win_d_csr, sizeof(int) * D, &bytes)) ||
        (rc = sqd_alloc(ctx, (void**)&t.win_s_v64, sizeof(double) * S, &bytes)) ||
        (rc = sqd_alloc(ctx, (void**)&t.win_s_v32, sizeof(float) * S, &bytes)) ||
        (rc = sqd_alloc(ctx, (void**)&t.win_d_v64, sizeof(double) * D, &bytes)) ||
        (rc = sqd_alloc(ctx, (void**)&t.win_d_v32, sizeof(float) * D, &bytes)) ||
        (rc = sqd_alloc(ctx, (void**)&t.win_islot, sizeof(int) * islot.size(), &bytes))) {
        sqd_free_window_tables(&t);
        return rc;
    }
    SQD_HIP(ctx, hipMemcpy(t.win_s_off, so.data(), sizeof(int) * so.size(), hipMemcpyHostToDevice));
    SQD_HIP(ctx, hipMemcpy(t.win_d_off, dof.data(), sizeof(int) * dof.size(), hipMemcpyHostToDevice));
    SQD_HIP(ctx, hipMemcpy(t.win_s_pk, hs_pk.data(), sizeof(uint32_t) * S, hipMemcpyHostToDevice));
    SQD_HIP(ctx, hipMemcpy(t.win_s_csr, hs_csr.data(), sizeof(int) * S, hipMemcpyHostToDevice));
    SQD_HIP(ctx, hipMemcpy(t.win_d_nbr, hd_nbr.data(), sizeof(uint16_t) * D, hipMemcpyHostToDevice));
    SQD_HIP(ctx, hipMemcpy(t.win_d_csr, hd_csr.data(), sizeof(int) * D, hipMemcpyHostToDevice));
    SQD_HIP(ctx, hipMemcpy(t.win_islot, islot.data(), sizeof(int) * islot.size(), hipMemcpyHostToDevice));
    t.win_W = W;
    t.win_width = width;
    t.win_values_version = -1;
    t.win_bytes = bytes;
    sp->bytes += bytes;
    return SQD_OK;
}

// values of the windowed slots from the canonical CSR values (per Hamiltonian)
int window_values(sqd_ctx* ctx, spin_tables& t) {
    if (t.win_values_version == ctx->ham_version) return SQD_OK;
    int s_cols = 0, d_cols = 0;
    SQD_HIP(ctx, hipMemcpy(&s_cols, t.win_s_off + (size_t)t.win_W * (t.nslices + 1) - 1, sizeof(int),
                           hipMemcpyDeviceToHost));
    SQD_HIP(ctx, hipMemcpy(&d_cols, t.win_d_off + (size_t)t.win_W * (t.nslices + 1) - 1, sizeof(int),
                           hipMemcpyDeviceToHost));
    const int64_t S = (int64_t)s_cols * 64, D = (int64_t)d_cols * 64;
    hipStream_t s = ctx->stream;
    if (S > 0) {
        hipLaunchKernelGGL(k_win_values<double>, dim3(nblk(S, 256)), dim3(256), 0, s, t.win_s_csr, S, t.s_val64,
                           t.win_s_v64);
        hipLaunchKernelGGL(k_win_values<float>, dim3(nblk(S, 256)), dim3(256), 0, s, t.win_s_csr, S, t.s_val32,
                           t.win_s_v32);
    }
    if (D > 0) {
        hipLaunchKernelGGL(k_win_values<double>, dim3(nblk(D, 256)), dim3(256), 0, s, t.win_d_csr, D, t.d_val64,
                           t.win_d_v64);
        hipLaunchKernelGGL(k_win_values<float>, dim3(nblk(D, 256)), dim3(256), 0, s, t.win_d_csr, D, t.d_val32,
                           t.win_d_v32);
    }
    SQD_HIP(ctx, hipGetLastError());
    SQD_HIP(ctx, hipStreamSynchronize(s));
    t.win_values_version = ctx->ham_version;
    return SQD_OK;
}

int window_wtable(sqd_ctx* ctx, sqd_space* sp, spin_tables& t) {
    if (t.wg64 && t.wg_version == ctx->ham_version) return SQD_OK;
    const int64_t m = sqd_wtable_ld(t.n) * (int64_t)sp->norb * sp->norb;
    int rc;
    if (!t.wg64) {
        int64_t bytes = 0;
        if ((rc = sqd_alloc(ctx, (void**)&t.wg64, sizeof(double) * (m + 1), &bytes)) ||
            (rc = sqd_alloc(ctx, (void**)&t.wg32, sizeof(float) * (m + 1), &bytes)))
            return rc;
        t.win_bytes += bytes;
        sp->bytes += bytes;
    }
    hipLaunchKernelGGL(k_wtable, dim3(nblk(m, 256)), dim3(256), 0, ctx->stream, t.str, t.nw, t.n,
                       sqd_wtable_ld(t.n), sp->norb, ctx->jk64, t.wg64, t.wg32);
    SQD_HIP(ctx, hipGetLastError());
    t.wg_version = ctx->ham_version;
    return SQD_OK;
}

template <typename F>
void set_lds_attr(F f, int bytes) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(f), hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <typename T, int R>
int launch_win(sqd_ctx* ctx, sqd_space* sp, spin_tables& col, spin_tables& row, const T* X, T* Y, int64_t nrows,
               int64_t ncols, int colmajor, int accumulate, const double* diag, const int* skip, const char* timer,
               int* diag_done) {
    const T* sv;
    const T* dv;
    const T* wg;
    if constexpr (sizeof(T) == 8) { sv = (const T*)col.win_s_v64; dv = (const T*)col.win_d_v64; wg = (const T*)row.wg64; }
    else { sv = (const T*)col.win_s_v32; dv = (const T*)col.win_d_v32; wg = (const T*)row.wg32; }
    // the output goes through P in slot order (P exists when W > 1) and a
    // coalesced pass places it
    const int slot_out = col.win_W > 1 ? 1 : 0;
    win_args<T> a{X, Y, (T*)sp->win_P, nrows, ncols, col.win_W, col.win_width, col.nslices, col.perm_ss,
                  col.win_s_off, col.win_d_off, col.win_s_pk, sv, col.win_d_nbr, dv, wg, sqd_wtable_ld(row.n),
                  sp->norb, colmajor, accumulate, slot_out};
    const size_t lds = (size_t)(col.win_width + 1) * R * sizeof(T);
    set_lds_attr(k_same_spin_win<T, R>, (int)lds);
    {
        prof_scope ps(ctx, timer);
        hipLaunchKernelGGL((k_same_spin_win<T, R>), dim3(nblk(nrows, R)), dim3(1024), lds, ctx->stream, a, skip);
    }
    if (slot_out && colmajor) {
        prof_scope pu(ctx, "k_win_unperm");
        const dim3 tg((unsigned)col.nslices, nblk(nrows, 64));
        hipLaunchKernelGGL((k_win_unperm_t<T>), tg, dim3(256), 0, ctx->stream, (const T*)sp->win_P,
                           (int64_t)col.nslices * 64, col.perm_ss, Y, nrows, ncols, accumulate, skip);
    } else if (slot_out) {
        const double* dg = sizeof(T) == 8 ? diag : nullptr;
        prof_scope pu(ctx, "k_win_unperm");
        const int64_t ldp = (int64_t)col.nslices * 64;
        const size_t rb = (size_t)ldp * sizeof(T);
        if (rb <= (size_t)ctx->max_lds) {
            set_lds_attr(k_win_unperm_lds<T>, (int)rb);
            const int per_cu = std::max<int>(1, (int)((size_t)ctx->max_lds / rb));
            const unsigned g = (unsigned)std::min<int64_t>(nrows, (int64_t)ctx->num_cu * per_cu);
            hipLaunchKernelGGL((k_win_unperm_lds<T>), dim3(g), dim3(1024), rb, ctx->stream, (const T*)sp->win_P, ldp,
                               col.win_islot, X, dg, Y, nrows, ncols, accumulate, skip);
        } else {
            const unsigned g = (unsigned)std::min<int64_t>(nrows, 1 << 20);
            hipLaunchKernelGGL((k_win_unperm<T>), dim3(g), dim3(256), 0, ctx->stream, (const T*)sp->win_P, ldp,
                               col.win_islot, X, dg, Y, nrows, ncols, accumulate, skip);
        }
        if (dg && diag_done) *diag_done = 1;
    }
    SQD_HIP(ctx, hipGetLastError());
    return SQD_OK;
}

}  // namespace

// rows staged per windowed workgroup: the window width is set by 8 FP64 rows;
// FP32 stages 16 rows of the same width in the same LDS, which halves its
// table stream per row (2.56e8-determinant workload, beta-beta FP32 windowed:
// 18.4 -> 16.9 ms)
constexpr int kWinRows = 8;
constexpr int kWinRows32 = 16;

void sqd_free_window_tables(spin_tables* t) {
    void* ptrs[] = {t->win_s_off, t->win_d_off, t->win_s_pk, t->win_d_nbr, t->win_s_csr, t->win_d_csr,
                    t->win_s_v64, t->win_s_v32, t->win_d_v64, t->win_d_v32, t->wg64, t->wg32, t->win_islot};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    t->win_s_off = t->win_d_off = t->win_s_csr = t->win_d_csr = nullptr;
    t->win_d_nbr = nullptr;
    t->win_islot = nullptr;
    t->win_s_pk = nullptr;
    t->win_s_v64 = t->win_d_v64 = t->wg64 = nullptr;
    t->win_s_v32 = t->win_d_v32 = t->wg32 = nullptr;
    t->win_W = t->win_width = 0;
    t->win_values_version = t->wg_version = -1;
    t->win_bytes = 0;
}

// Windows for rows of ncols strings: the fewest whose R staged FP64 rows fit
// the LDS of one workgroup (or of the width set by SQD_TUNE_SS_WINDOW).  FP32
// products use the same windows (with twice the rows), so both precisions
// share one set of tables.
int sqd_window_count(sqd_ctx* ctx, int64_t ncols) {
    int64_t wmax = (int64_t)(ctx->max_lds / (sizeof(double) * kWinRows)) - 1;
    if (ctx->tune[SQD_TUNE_SS_WINDOW] >= 64) wmax = std::min<int64_t>(wmax, ctx->tune[SQD_TUNE_SS_WINDOW]);
    if (wmax < 64) return 0;
    return (int)std::max<int64_t>(1, (ncols + wmax - 1) / wmax);
}

size_t sqd_window_scratch_bytes(const sqd_space* sp) {
    size_t b = 0;
    for (int spin = 0; spin < 2; ++spin) {   // rows of one spin x slots of the other
        const spin_tables& col = sp->sp[spin].alias ? sp->sp[0] : sp->sp[spin];
        b = std::max(b, (size_t)sp->sp[1 - spin].n * (size_t)col.nslices * 64 * sizeof(double));
    }
    return b;
}

int sqd_same_spin_windowed(sqd_ctx* ctx, sqd_space* sp, spin_tables& col, spin_tables& row, const void* X, void* Y,
                           int64_t nrows, int64_t ncols, int colmajor, int accumulate, int fp32, const double* diag,
                           int* diag_done, const int* skip, const char* timer) {
    const int W = sqd_window_count(ctx, ncols);
    if (W == 0) return sqd_fail(ctx, SQD_E_LIMIT, "same-spin window does not fit in LDS");
    const bool cap = sqd_capturing(ctx);
    int rc;
    if (col.win_W != W) {
        if (cap) return sqd_fail(ctx, SQD_E_STATE, "windowed tables not built before the capture");
        if ((rc = build_window_tables(ctx, sp, col, W))) return rc;
    }
    if (col.win_values_version != ctx->ham_version || !row.wg64 || row.wg_version != ctx->ham_version) {
        if (cap) return sqd_fail(ctx, SQD_E_STATE, "windowed values not built before the capture");
        if ((rc = window_values(ctx, col)) || (rc = window_wtable(ctx, sp, row))) return rc;
    }
    // partial sums between windows: one scratch per space, kept
    const size_t pb = sqd_window_scratch_bytes(sp);
    if (W > 1 && sp->win_P_bytes < pb) {
        if (cap) return sqd_fail(ctx, SQD_E_STATE, "windowed scratch not allocated before the capture");
        SQD_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (sp->win_P) {
            (void)hipFree(sp->win_P);
            sp->bytes -= (int64_t)sp->win_P_bytes;
            sp->win_P = nullptr;
            sp->win_P_bytes = 0;
        }
        if ((rc = sqd_alloc(ctx, &sp->win_P, pb, &sp->bytes))) return rc;
        sp->win_P_bytes = pb;
    }
    if (fp32)
        return launch_win<float, kWinRows32>(ctx, sp, col, row, (const float*)X, (float*)Y, nrows, ncols, colmajor,
                                             accumulate, nullptr, skip, timer, diag_done);
    return launch_win<double, kWinRows>(ctx, sp, col, row, (const double*)X, (double*)Y, nrows, ncols, colmajor,
                                          accumulate, diag, skip, timer, diag_done);
}
