// Device bodies of the sigma kernels, shared by the single-space launches
// (sigma.hip) and the batched persistent launches (davidson.hip).  Each body
// processes one work unit (a block index of its own launch shape) of one
// space described by an argument struct.
#pragma once

#include <type_traits>

#include "sqd_internal.h"

// LDS layout of R values per column c (staged rows of C, or rows of the
// cross-spin table): column c owns R * sizeof(T) bytes at c * R.  Lanes read
// whole columns at random c in 16-byte pieces; when a column is two or four
// 16-byte pieces, the pieces are stored XOR-permuted by bits of c above those
// that already select the bank group, so that for any piece index the 64
// lanes spread over all LDS banks instead of a quarter or half of them.
template <typename T, int R>
struct lds_cols {
    static constexpr int kE = 16 / (int)sizeof(T);                 // elements per 16-byte piece
    static constexpr int kU = (R * (int)sizeof(T)) / 16;           // pieces per column (0: under 16 bytes)
    static constexpr bool kSwz = (kU == 2 || kU == 4);
    __device__ static __forceinline__ int swz(int64_t c) {
        return kU == 4 ? (int)((c >> 2) & 3) : (int)((c >> 3) & 1);
    }
    __device__ static __forceinline__ int64_t idx(int64_t c, int r) {
        if constexpr (kSwz) return c * R + (((r / kE) ^ swz(c)) * kE) + (r % kE);
        else return c * R + r;
    }
    __device__ static __forceinline__ void load(const T* __restrict__ xs, int64_t c, T (&v)[R]) {
        if constexpr (kSwz) {
            const int f = swz(c);
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const T* src = xs + c * R + ((u ^ f) * kE);
#pragma unroll
                for (int w = 0; w < kE; ++w) v[u * kE + w] = src[w];
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = xs[c * R + r];
        }
    }
};

// Stage R rows of length ncols (row r starts at rows[r], or zeros when null;
// rows[0] is never null) into LDS in the lds_cols<T, R> layout; column ncols
// is zero.  Each thread takes four columns per pass and issues all 4R loads
// before any store: null rows read row 0 and are zeroed by a select, columns
// past the end read the last column and are not stored, so no load sits
// behind a branch.
template <typename T, int R>
__device__ __forceinline__ void stage_rows(T* __restrict__ xs, const T* const (&rows)[R], int ncols) {
    using L = lds_cols<T, R>;
    constexpr int kCols = 4;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const T* src[R];
    bool ok[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        ok[r] = rows[r] != nullptr;
        src[r] = ok[r] ? rows[r] : rows[0];
    }
    for (int col0 = tid; col0 < ncols; col0 += kCols * nthr) {
        T v[kCols][R];
#pragma unroll
        for (int u = 0; u < kCols; ++u) {
            const int c = min(col0 + u * nthr, ncols - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) v[u][r] = src[r][c];
        }
#pragma unroll
        for (int u = 0; u < kCols; ++u) {
            const int c = col0 + u * nthr;
            if (c < ncols) {
#pragma unroll
                for (int r = 0; r < R; ++r) xs[L::idx(c, r)] = ok[r] ? v[u][r] : (T)0;
            }
        }
    }
    if (tid < R) xs[(int64_t)ncols * R + tid] = (T)0;
}

// Stage rows row0 .. row0+R-1 of X held column-major (element (row, col) at
// col * nrows + row) into LDS in the lds_cols<T, R> layout; column ncols is
// zero.  A thread reads the R consecutive values of a column (one or two
// cache lines), two columns per pass with all loads before any store.
template <typename T, int R>
__device__ __forceinline__ void stage_cols(T* __restrict__ xs, const T* __restrict__ X, int64_t nrows, int64_t row0,
                                           int64_t ncols) {
    using L = lds_cols<T, R>;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const bool full = row0 + R <= nrows;   // uniform over the workgroup
    for (int64_t c0 = tid; c0 < ncols; c0 += 2 * nthr) {
        T v[2][R];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int64_t c = c0 + u * nthr < ncols ? c0 + u * nthr : ncols - 1;
            const T* src = X + c * nrows + row0;
            if (full) {
                if constexpr (R * sizeof(T) % 16 == 0) {
                    if ((reinterpret_cast<uintptr_t>(src) & 15) == 0) {   // 16-byte pieces
                        using V4 = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
                        constexpr int kP = (int)(16 / sizeof(T));
#pragma unroll
                        for (int q = 0; q < R / kP; ++q) {
                            const V4 x = reinterpret_cast<const V4*>(src)[q];
                            const T* xv = reinterpret_cast<const T*>(&x);
#pragma unroll
                            for (int i = 0; i < kP; ++i) v[u][q * kP + i] = xv[i];
                        }
                        continue;
                    }
                }
#pragma unroll
                for (int r = 0; r < R; ++r) v[u][r] = src[r];
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) v[u][r] = (row0 + r < nrows) ? src[r] : (T)0;
            }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int64_t c = c0 + u * nthr;
            if (c < ncols) {
#pragma unroll
                for (int r = 0; r < R; ++r) xs[L::idx(c, r)] = v[u][r];
            }
        }
    }
    if (tid < R) xs[ncols * R + tid] = (T)0;
}

// ---------------------------------------------------------------- same spin
template <typename T>
struct ss_args {
    const T* X;            // nrows x ncols
    T* Y;
    int64_t nrows, ncols;
    const int* perm;       // sliced table of the column spin
    int nslices;
    const int* sl_s_off;
    const int* sl_d_off;
    const uint32_t* s_pk;
    const T* s_val;
    const int* d_nbr;
    const T* d_val;
    const uint64_t* row_str;   // strings of the row spin (cross-spin term), nw words each
    int nw;
    const double* diag;        // fused DIAG term (or null)
    int accumulate;
    int colmajor;              // X, Y (and diag) hold the transposes: (row, col) at col * nrows + row
};

// Rows blk*R .. blk*R+R-1: Y (=|+=) same-spin singles and doubles of the column
// spin.  LDS: xs[(ncols+1)*R] as [col][r]; ws[norb2*R] as [pq][r].
template <typename T, int R>
__device__ __forceinline__ void ss_block(const ss_args<T>& a, const T* __restrict__ jk, int norb, int64_t blk,
                                         unsigned char* lds_raw) {
    T* xs = reinterpret_cast<T*>(lds_raw);
    const int norb2 = norb * norb;
    const int64_t ncols = a.ncols, nrows = a.nrows;
    T* ws = xs + (ncols + 1) * R;
    const int64_t row0 = blk * R;
    const int nthr = blockDim.x;
    const int tid = threadIdx.x;
    if (a.colmajor) {
        stage_cols<T, R>(xs, a.X, nrows, row0, ncols);
    } else {
        const T* rows[R];
#pragma unroll
        for (int r = 0; r < R; ++r) rows[r] = (row0 + r < nrows) ? a.X + (row0 + r) * ncols : nullptr;
        stage_rows<T, R>(xs, rows, (int)ncols);
    }
    // cross-spin term of the staged rows: ws[pq][r] = sum_{k in row string} (pq|kk),
    // summed over k in increasing order; every (pq|kk) is loaded (no load
    // behind a branch) and unoccupied k contribute an exact zero
    for (int idx = tid; idx < R * norb2; idx += nthr) {
        const int r = idx / norb2, pq = idx - r * norb2;
        const int64_t row = row0 + r;
        T acc = (T)0;
        for (int q = 0; q < a.nw; ++q) {
            const uint64_t x = (row < nrows) ? a.row_str[row * a.nw + q] : 0ull;
            const int kend = min(norb - 64 * q, 64);
            const T* jq = jk + (int64_t)(64 * q) * norb2 + pq;
            int k = 0;
            for (; k + 4 <= kend; k += 4) {
                T v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = jq[(int64_t)(k + u) * norb2];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if ((x >> (k + u)) & 1ull) acc += v[u];
            }
            for (; k < kend; ++k)
                if ((x >> k) & 1ull) acc += jq[(int64_t)k * norb2];
        }
        ws[lds_cols<T, R>::idx(pq, r)] = acc;
    }
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63, nw = nthr >> 6;
    for (int sl = wave; sl < a.nslices; sl += nw) {
        T acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = (T)0;
        const int s0 = a.sl_s_off[sl], s1 = a.sl_s_off[sl + 1];
        const int d0 = a.sl_d_off[sl], d1 = a.sl_d_off[sl + 1];
        // table entries in flight: sixteen for FP32, whose entries are half
        // the bytes and whose LDS reads are cheaper; eight for FP64 (measured
        // on MI355X: sixteen is slower there, with one row or eight)
        constexpr int kD = sizeof(T) == 4 ? 16 : 8;
        // with one or two staged rows (long rows: the table streams from
        // beyond the L2) the first batch of doubles loads while the singles
        // run (2.56e8 workload, FP32 same-spin: 16.0 -> 14.7 ms; with eight
        // rows it only costs registers: FP32 90 -> 106 us on the 4.0e6 one)
        constexpr bool kPre = R <= 2;
        int nbP[kPre ? kD : 1];
        T vP[kPre ? kD : 1];
        const bool pre = kPre && d0 + kD <= d1;
        if constexpr (kPre) {
            if (pre) {
#pragma unroll
                for (int u = 0; u < kD; ++u) {
                    nbP[u] = a.d_nbr[(int64_t)(d0 + u) * 64 + lane];
                    vP[u] = a.d_val[(int64_t)(d0 + u) * 64 + lane];
                }
            }
        }
        auto single = [&](uint32_t e, T v) {
            const int nbr = (int)(e & SQD_NBR_MASK);
            const int pair = (int)((e >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK);
            T xr[R], wr[R];
            lds_cols<T, R>::load(xs, nbr, xr);
            lds_cols<T, R>::load(ws, pair, wr);
            const bool neg = (e >> 31) != 0;
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += (v + (neg ? -wr[r] : wr[r])) * xr[r];
        };
        int k = s0;
        for (; k + 4 <= s1; k += 4) {   // four table entries in flight
            uint32_t e[4];
            T v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                e[u] = a.s_pk[(int64_t)(k + u) * 64 + lane];
                v[u] = a.s_val[(int64_t)(k + u) * 64 + lane];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) single(e[u], v[u]);
        }
        for (; k < s1; ++k) single(a.s_pk[(int64_t)k * 64 + lane], a.s_val[(int64_t)k * 64 + lane]);
        auto dbl = [&](int nbr, T v) {
            T xr[R];
            lds_cols<T, R>::load(xs, nbr, xr);
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += v * xr[r];
        };
        k = d0;
        if constexpr (kPre) {
            if (pre) {
#pragma unroll
                for (int u = 0; u < kD; ++u) dbl(nbP[u], vP[u]);
                k += kD;
            }
        }
        for (; k + kD <= d1; k += kD) {
            int nbd[kD];
            T v[kD];
#pragma unroll
            for (int u = 0; u < kD; ++u) {
                nbd[u] = a.d_nbr[(int64_t)(k + u) * 64 + lane];
                v[u] = a.d_val[(int64_t)(k + u) * 64 + lane];
            }
#pragma unroll
            for (int u = 0; u < kD; ++u) dbl(nbd[u], v[u]);
        }
        if constexpr (kD > 8) {
            if (k + 8 <= d1) {
                int nb8[8];
                T v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    nb8[u] = a.d_nbr[(int64_t)(k + u) * 64 + lane];
                    v[u] = a.d_val[(int64_t)(k + u) * 64 + lane];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) dbl(nb8[u], v[u]);
                k += 8;
            }
        }
        for (; k + 4 <= d1; k += 4) {
            int nb4[4];
            T v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                nb4[u] = a.d_nbr[(int64_t)(k + u) * 64 + lane];
                v[u] = a.d_val[(int64_t)(k + u) * 64 + lane];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) dbl(nb4[u], v[u]);
        }
        for (; k < d1; ++k) dbl(a.d_nbr[(int64_t)k * 64 + lane], a.d_val[(int64_t)k * 64 + lane]);
        const int t = a.perm[sl * 64 + lane];
        if constexpr (R * sizeof(T) % 16 == 0) {
            // column-major output of a whole row block: R consecutive values
            // of the target's column in 16-byte pieces
            T* yp = a.Y + (int64_t)t * nrows + row0;
            if (a.colmajor && !a.diag && t < ncols && row0 + R <= nrows &&
                (reinterpret_cast<uintptr_t>(yp) & 15) == 0) {
                using V4 = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
                constexpr int kP = (int)(16 / sizeof(T));
                V4 old[R / kP];
                if (a.accumulate) {
#pragma unroll
                    for (int q = 0; q < R / kP; ++q) old[q] = reinterpret_cast<const V4*>(yp)[q];
                }
#pragma unroll
                for (int q = 0; q < R / kP; ++q) {
                    V4 y;
                    T* yv = reinterpret_cast<T*>(&y);
                    const T* ov = reinterpret_cast<const T*>(&old[q]);
#pragma unroll
                    for (int i = 0; i < kP; ++i) yv[i] = acc[q * kP + i] + (a.accumulate ? ov[i] : (T)0);
                    reinterpret_cast<V4*>(yp)[q] = y;
                }
                continue;
            }
        }
        if (t < ncols) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t row = row0 + r;
                if (row < nrows) {
                    const int64_t o = a.colmajor ? (int64_t)t * nrows + row : row * ncols + t;
                    T val = acc[r];
                    if (a.diag) val += (T)(a.diag[o] * (double)xs[lds_cols<T, R>::idx(t, r)]);
                    if (a.accumulate) val += a.Y[o];
                    a.Y[o] = val;
                }
            }
        }
    }
}

// ---------------------------------------------------------------- alpha-beta, grouped
// The alpha single entries e (CSR position in the target row's list; source
// row src(e), pair ai(e), sign s(e)) are grouped by pair ai and cut into chunks
// of G entries that share ai.  One unit per chunk stages the G source rows of C
// in LDS (lds_cols layout) and the row (ai|..) of the (pq|rs) matrix, then
// walks the sliced beta singles table once for all G rows:
//   Y[e][slot(jb')] = s(e) * sum_{beta singles jb' <- jb (pair bj, s_b)} s_b (ai|bj) C[src(e)][jb]
// Y is written in slot order (slice * 64 + lane), so each wave stores 64
// consecutive values, with non-temporal stores (read once, by the gather);
// the gather maps slots back to beta strings.
template <typename T>
struct abg_args {
    const T* C;
    T* Y;                     // nnz_alpha_singles x ldy, columns in sliced (slot) order
    int64_t nb;
    int64_t ldy;              // 64 x number of beta slices
    const int* grp;           // chunks x G CSR positions (-1 = padding)
    const int* chunk_pair;
    const uint32_t* a_pk;     // alpha singles (gather form)
    const int* bperm;         // sliced beta singles
    int nbslices;
    const int* bsl_off;
    const uint32_t* bs_pk;
};

template <typename T, int G>
__device__ __forceinline__ void abg_block(const abg_args<T>& a, const T* __restrict__ V, int norb, int64_t chunk,
                                          unsigned char* lds_raw) {
    T* xs = reinterpret_cast<T*>(lds_raw);
    const int norb2 = norb * norb;
    const int64_t nb = a.nb;
    T* vrow = xs + (nb + 1) * G;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int pair = a.chunk_pair[chunk];
    int e[G];
    T sgn[G];
#pragma unroll
    for (int r = 0; r < G; ++r) {
        e[r] = a.grp[chunk * G + r];
        sgn[r] = (e[r] >= 0 && (a.a_pk[e[r]] >> 31)) ? (T)-1 : (T)1;
    }
    {
        const T* rows[G];
#pragma unroll
        for (int r = 0; r < G; ++r) rows[r] = (e[r] >= 0) ? a.C + (int64_t)(a.a_pk[e[r]] & SQD_NBR_MASK) * nb : nullptr;
        stage_rows<T, G>(xs, rows, (int)nb);
    }
    for (int q = tid; q < norb2; q += nthr) vrow[q] = V[(int64_t)pair * norb2 + q];
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63, nw = nthr >> 6;
    for (int sl = wave; sl < a.nbslices; sl += nw) {
        T acc[G];
#pragma unroll
        for (int r = 0; r < G; ++r) acc[r] = (T)0;
        const int c0 = a.bsl_off[sl], c1 = a.bsl_off[sl + 1];
        auto one = [&](uint32_t b) {
            const int nbr = (int)(b & SQD_NBR_MASK);
            const int pb = (int)((b >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK);
            T v = vrow[pb];
            if (b >> 31) v = -v;
            T xr[G];
            lds_cols<T, G>::load(xs, nbr, xr);
#pragma unroll
            for (int r = 0; r < G; ++r) acc[r] += v * xr[r];
        };
        int col = c0;
        constexpr int kD = G <= 2 ? 16 : 8;   // table entries in flight (more when few rows share each)
        for (; col + kD <= c1; col += kD) {
            uint32_t bd[kD];
#pragma unroll
            for (int u = 0; u < kD; ++u) bd[u] = a.bs_pk[(int64_t)(col + u) * 64 + lane];
#pragma unroll
            for (int u = 0; u < kD; ++u) one(bd[u]);
        }
        if constexpr (kD > 8) {
            if (col + 8 <= c1) {
                uint32_t b8[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) b8[u] = a.bs_pk[(int64_t)(col + u) * 64 + lane];
#pragma unroll
                for (int u = 0; u < 8; ++u) one(b8[u]);
                col += 8;
            }
        }
        if (col + 4 <= c1) {
            uint32_t b4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) b4[u] = a.bs_pk[(int64_t)(col + u) * 64 + lane];
#pragma unroll
            for (int u = 0; u < 4; ++u) one(b4[u]);
            col += 4;
        }
        for (; col < c1; ++col) one(a.bs_pk[(int64_t)col * 64 + lane]);
        // padding lanes read only the zero column: their value is zero
        const int64_t slot = (int64_t)sl * 64 + lane;
#pragma unroll
        for (int r = 0; r < G; ++r)
            if (e[r] >= 0) __builtin_nontemporal_store(sgn[r] * acc[r], a.Y + (int64_t)e[r] * a.ldy + slot);
    }
}

// The same Y from chunks of up to GS alpha singles that share their source
// string (chunk_src): one staged row of C serves GS pairs, whose (ai|..) rows
// are staged beside it.  Where a row of C fills most of the LDS (long rows,
// where the pair-grouped chunks hold one single) this reads 8 bytes of LDS
// per table entry for C and 8 per single for the integral, (8 + 8 GS) / GS
// bytes per connection instead of 16, and stages each source row once per GS
// singles.  Same products and summation order as abg_block.
template <typename T, int GS>
__device__ __forceinline__ void abs_block(const abg_args<T>& a, const int* __restrict__ chunk_src,
                                          const T* __restrict__ V, int norb, int64_t chunk, unsigned char* lds_raw) {
    T* xs = reinterpret_cast<T*>(lds_raw);   // the source row, column nb zero
    const int norb2 = norb * norb;
    const int64_t nb = a.nb;
    T* vrows = xs + (nb + 1);                // GS rows of (ai|..), row g at g * norb2
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int64_t src = chunk_src[chunk];
    int e[GS], pr[GS];
    T sgn[GS];
#pragma unroll
    for (int g = 0; g < GS; ++g) {
        e[g] = a.grp[chunk * GS + g];
        const uint32_t x = e[g] >= 0 ? a.a_pk[e[g]] : 0u;
        sgn[g] = (x >> 31) ? (T)-1 : (T)1;
        pr[g] = (int)((x >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK);
    }
    const T* crow = a.C + src * nb;
    for (int64_t k = tid; k < nb; k += nthr) xs[k] = crow[k];
    if (tid == 0) xs[nb] = (T)0;
    for (int q = tid; q < GS * norb2; q += nthr) {
        const int g = q / norb2, r = q - g * norb2;
        vrows[q] = e[g] >= 0 ? V[(int64_t)pr[g] * norb2 + r] : (T)0;
    }
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63, nw = nthr >> 6;
    for (int sl = wave; sl < a.nbslices; sl += nw) {
        T acc[GS];
#pragma unroll
        for (int g = 0; g < GS; ++g) acc[g] = (T)0;
        const int c0 = a.bsl_off[sl], c1 = a.bsl_off[sl + 1];
        auto one = [&](uint32_t b) {
            const int nbr = (int)(b & SQD_NBR_MASK);
            const int pb = (int)((b >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK);
            T x = xs[nbr];
            if (b >> 31) x = -x;   // (-v) x = v (-x) exactly
#pragma unroll
            for (int g = 0; g < GS; ++g) acc[g] += vrows[g * norb2 + pb] * x;
        };
        int col = c0;
        // table entries in flight: sixteen while GS rows leave the registers
        // for them (with GS = 8 FP64 sixteen entries spilled)
        constexpr int kD = GS <= 3 ? 16 : 8;
        for (; col + kD <= c1; col += kD) {
            uint32_t bd[kD];
#pragma unroll
            for (int u = 0; u < kD; ++u) bd[u] = a.bs_pk[(int64_t)(col + u) * 64 + lane];
#pragma unroll
            for (int u = 0; u < kD; ++u) one(bd[u]);
        }
        if (kD > 8 && col + 8 <= c1) {
            uint32_t b8[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) b8[u] = a.bs_pk[(int64_t)(col + u) * 64 + lane];
#pragma unroll
            for (int u = 0; u < 8; ++u) one(b8[u]);
            col += 8;
        }
        if (col + 4 <= c1) {
            uint32_t b4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) b4[u] = a.bs_pk[(int64_t)(col + u) * 64 + lane];
#pragma unroll
            for (int u = 0; u < 4; ++u) one(b4[u]);
            col += 4;
        }
        for (; col < c1; ++col) one(a.bs_pk[(int64_t)col * 64 + lane]);
        // padding lanes read only the zero column: their value is zero
        const int64_t slot = (int64_t)sl * 64 + lane;
#pragma unroll
        for (int g = 0; g < GS; ++g)
            if (e[g] >= 0) __builtin_nontemporal_store(sgn[g] * acc[g], a.Y + (int64_t)e[g] * a.ldy + slot);
    }
}

// sigma[ia][perm(p)] += sum_{e in row ia} Y[e][p] over all slots p of row ia,
// one workgroup per row: each thread reads two adjacent slots with
// one vector load (ldy is a multiple of 64), eight rows of Y in flight.  Y is
// written once and read once, so both sides bypass the caches' retention
// (non-temporal accesses): the tables and C of the next kernels stay cached
// (4.0e6-determinant workload, same box: gather 142 -> 103 us, the beta-beta
// kernel after it 192 -> 176 us).  With `row` (LDS, nb values) the sums are
// placed by target first and the row of sigma is then updated with coalesced
// accesses; without it (rows too long for LDS) each sum is added in place.
template <typename T>
__device__ __forceinline__ void gather_row(const T* __restrict__ Y, T* __restrict__ S, int64_t nb, int64_t ldy,
                                           const int* __restrict__ bperm, const int* __restrict__ a_off, int64_t ia,
                                           T* row) {
    typedef T T2 __attribute__((ext_vector_type(2)));
    constexpr int kU = 8;
    const int e0 = a_off[ia], e1 = a_off[ia + 1];
    T* srow = S + ia * nb;
    for (int64_t p = 2 * (int64_t)threadIdx.x; p < ldy; p += 2 * (int64_t)blockDim.x) {
        T a0 = (T)0, a1 = (T)0;
        for (int e = e0; e < e1; e += kU) {
            T2 v[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u)
                v[u] = (e + u < e1) ? __builtin_nontemporal_load(reinterpret_cast<const T2*>(Y + (int64_t)(e + u) * ldy + p))
                                    : T2{(T)0, (T)0};
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                a0 += v[u].x;
                a1 += v[u].y;
            }
        }
        const int t0 = bperm[p], t1 = bperm[p + 1];
        if (row) {
            if (t0 < nb) row[t0] = a0;
            if (t1 < nb) row[t1] = a1;
        } else {
            if (t0 < nb) srow[t0] += a0;
            if (t1 < nb) srow[t1] += a1;
        }
    }
    if (row) {
        __syncthreads();
        for (int64_t j = threadIdx.x; j < nb; j += blockDim.x) srow[j] += row[j];
        __syncthreads();
    }
}

// out[c][r] (=|+=) in[r][c] for the 64 x 64 tile (ty, tx); in is rows x cols.
template <typename TI, typename TO, bool ADD>
__device__ __forceinline__ void transpose_tile(const TI* __restrict__ in, TO* __restrict__ out, int64_t rows,
                                               int64_t cols, int64_t ty, int64_t tx_, TI (*tile)[65]) {
    const int64_t r0 = ty * 64, c0 = tx_ * 64;
    const int tx = threadIdx.x & 63, tyy = threadIdx.x >> 6, ny = blockDim.x >> 6;
    for (int k = tyy; k < 64; k += ny) {
        const int64_t r = r0 + k, c = c0 + tx;
        if (r < rows && c < cols) tile[k][tx] = in[r * cols + c];
    }
    __syncthreads();
    for (int k = tyy; k < 64; k += ny) {
        const int64_t c = c0 + k, r = r0 + tx;
        if (r < rows && c < cols) {
            TO v = (TO)tile[tx][k];
            if (ADD) v += out[c * rows + r];
            out[c * rows + r] = v;
        }
    }
}
