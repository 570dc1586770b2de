// Excitation tables on the device (Sec. IV-A persistent configuration data and
// Sec. V-A flattened per-string excitation lists, offset + entries).
//
// For each string of a sorted set, the in-set single (i -> a) and double
// (i < j -> a < b) excitations are enumerated one wavefront per string, lanes
// over candidates; each candidate target is looked up by binary search in the
// sorted strings; the found entries are compacted into CSR rows, sorted inside
// each row by target index (canonical order) and packed.  The integral-
// dependent same-spin values are computed per entry afterwards, so that a new
// Hamiltonian does not rebuild the structure.
#include <rocprim/device/device_radix_sort.hpp>

#include "sqd_internal.h"

namespace {

// A string of NW 64-bit words (word q: orbitals 64q .. 64q+63) held in registers.
template <int NW>
struct wstr {
    uint64_t w[NW];
    __device__ __forceinline__ void flip(int k) { w[k >> 6] ^= 1ull << (k & 63); }
};

template <int NW>
__device__ __forceinline__ wstr<NW> load_str(const uint64_t* __restrict__ s, int64_t r) {
    wstr<NW> x;
#pragma unroll
    for (int q = 0; q < NW; ++q) x.w[q] = s[r * NW + q];
    return x;
}

// Binary search of the ascending strings (as NW-word integers, word NW-1 most
// significant) for key.
template <int NW>
__device__ __forceinline__ int64_t find_string(const uint64_t* __restrict__ s, int64_t n, const wstr<NW>& key) {
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        const int64_t mid = (lo + hi) >> 1;
        int c = 0;
#pragma unroll
        for (int q = NW - 1; q >= 0; --q) {
            const uint64_t v = s[mid * NW + q];
            if (c == 0 && v != key.w[q]) c = v < key.w[q] ? -1 : 1;
        }
        if (c == 0) return mid;
        if (c < 0) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

// Occupied / virtual orbital lists of string s, built by one wavefront (lane =
// orbital within a word) into LDS, each ascending.
template <int NW>
__device__ __forceinline__ void orbital_lists(const wstr<NW>& s, int norb, uint8_t* occ, uint8_t* vir) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    int no = 0, nv = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        const int orb = 64 * q + lane;
        const bool in = orb < norb;
        const bool o = in && ((s.w[q] >> lane) & 1ull);
        const uint64_t bo = __ballot(o);
        const uint64_t bv = __ballot(in && !o);
        if (o) occ[no + __popcll(bo & below)] = (uint8_t)orb;
        if (in && !o) vir[nv + __popcll(bv & below)] = (uint8_t)orb;
        no += __popcll(bo);
        nv += __popcll(bv);
    }
}

// (-1)^(occupied orbitals below k) as 0 / 1
template <int NW>
__device__ __forceinline__ int parity_below(const wstr<NW>& s, int k) {
    int c = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        const int lo = 64 * q;
        if (k >= lo + 64) c += __popcll(s.w[q]);
        else if (k > lo) c += __popcll(s.w[q] & ((~0ull) >> (64 - (k - lo))));
    }
    return c & 1;
}

// Sign of a+_a a_i applied to s (a_i first).
template <int NW>
__device__ __forceinline__ int single_sign(wstr<NW> s, int i, int a) {
    int p = parity_below(s, i);
    s.flip(i);
    p ^= parity_below(s, a);
    return p;  // 1 = negative
}

// Sign of a+_a a+_b a_j a_i applied to s (a_i, a_j, a+_b, a+_a in that order).
template <int NW>
__device__ __forceinline__ int double_sign(wstr<NW> s, int i, int j, int a, int b) {
    int p = parity_below(s, i);
    s.flip(i);
    p ^= parity_below(s, j);
    s.flip(j);
    p ^= parity_below(s, b);
    s.flip(b);
    p ^= parity_below(s, a);
    return p;
}

// Waves per block and LDS slots for the (x < y) orbital pairs of one string:
// C(64, 2) for one-word strings, C(128, 2) (one wave per block) for two.
template <int NW> struct enum_shape;
template <> struct enum_shape<1> { static constexpr int kWaves = 4, kPairs = 2016; };
template <> struct enum_shape<2> { static constexpr int kWaves = 1, kPairs = 8128; };

// KIND 0: singles, 1: doubles.  MODE 0: count, 1: fill.
template <int KIND, int MODE, int NW>
__global__ void __launch_bounds__(64 * enum_shape<NW>::kWaves)
k_enum(const uint64_t* __restrict__ str, int64_t n, int norb, int nel,
       int* __restrict__ counts, const int* __restrict__ off,
       uint64_t* __restrict__ keys, uint32_t* __restrict__ payload) {
    constexpr int WPB = enum_shape<NW>::kWaves, NP = enum_shape<NW>::kPairs;
    __shared__ uint8_t s_occ[WPB][64 * NW];
    __shared__ uint8_t s_vir[WPB][64 * NW];
    __shared__ uint16_t s_op[WPB][KIND == 1 ? NP : 1];
    __shared__ uint16_t s_vp[WPB][KIND == 1 ? NP : 1];
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * WPB + w;
    // every wave reaches both barriers; waves past the end do no work
    const bool valid = row < n;
    wstr<NW> s;
#pragma unroll
    for (int q = 0; q < NW; ++q) s.w[q] = 0ull;
    if (valid) s = load_str<NW>(str, row);
    const int nvir = norb - nel;
    uint8_t* occ = s_occ[w];
    uint8_t* vir = s_vir[w];
    if (valid) orbital_lists<NW>(s, norb, occ, vir);
    int npo = 0, npv = 0;
    if (KIND == 1) {
        npo = nel * (nel - 1) / 2;
        npv = nvir * (nvir - 1) / 2;
    }
    __syncthreads();
    if (KIND == 1 && valid) {
        for (int k = lane; k < npo; k += 64) {
            // decode k -> (x < y) in row-major upper-triangle order
            int x = 0, rem = k;
            while (rem >= nel - 1 - x) { rem -= nel - 1 - x; ++x; }
            s_op[w][k] = (uint16_t)(occ[x] | (occ[x + 1 + rem] << 8));
        }
        for (int k = lane; k < npv; k += 64) {
            int x = 0, rem = k;
            while (rem >= nvir - 1 - x) { rem -= nvir - 1 - x; ++x; }
            s_vp[w][k] = (uint16_t)(vir[x] | (vir[x + 1 + rem] << 8));
        }
    }
    __syncthreads();
    if (!valid) return;
    const int64_t ncand = (KIND == 0) ? (int64_t)nel * nvir : (int64_t)npo * npv;
    int found = 0;
    const int base = (MODE == 1) ? off[row] : 0;
    for (int64_t c0 = 0; c0 < ncand; c0 += 64) {
        const int64_t c = c0 + lane;
        int64_t tgt = -1;
        int i = 0, j = 0, a = 0, b = 0;
        if (c < ncand) {
            wstr<NW> t = s;
            if (KIND == 0) {
                i = occ[c / nvir];
                a = vir[c % nvir];
                t.flip(i);
                t.flip(a);
            } else {
                const uint16_t op = s_op[w][c / npv];
                const uint16_t vp = s_vp[w][c % npv];
                i = op & 0xFF; j = op >> 8; a = vp & 0xFF; b = vp >> 8;
                t.flip(i);
                t.flip(j);
                t.flip(a);
                t.flip(b);
            }
            tgt = find_string<NW>(str, n, t);
        }
        const bool hit = tgt >= 0;
        const uint64_t m = __ballot(hit);
        if (MODE == 1 && hit) {
            const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
            const int pos = base + found + __popcll(m & below);
            keys[pos] = ((uint64_t)row << 17) | (uint64_t)tgt;
            uint32_t neg = (KIND == 0) ? (uint32_t)single_sign<NW>(s, i, a)
                                       : (uint32_t)double_sign<NW>(s, i, j, a, b);
            payload[pos] = (uint32_t)i | ((uint32_t)j << 7) | ((uint32_t)a << 14) |
                           ((uint32_t)b << 21) | (neg << 31);
        }
        found += __popcll(m);
    }
    if (MODE == 0 && lane == 0) counts[row] = found;
}

// Exclusive scan of n ints into off[0..n] with off[n] = total (one block).
__global__ void __launch_bounds__(1024) k_scan(const int* __restrict__ in, int64_t n, int* __restrict__ out,
                                               long long* __restrict__ total) {
    __shared__ long long part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t b = t * chunk, e = (b + chunk < n) ? b + chunk : n;
    long long s = 0;
    for (int64_t k = b; k < e; ++k) s += in[k];
    part[t] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        long long v = (t >= o) ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    long long run = part[t] - s;
    for (int64_t k = b; k < e; ++k) {
        out[k] = (int)run;
        run += in[k];
    }
    if (t == 1023) {
        out[n] = (int)part[1023];
        *total = part[1023];
    }
}

template <int KIND>
__global__ void k_pack(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ payload,
                       int64_t nnz, int norb, uint64_t* __restrict__ ent, uint32_t* __restrict__ pk,
                       int* __restrict__ nbr) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const uint64_t tgt = keys[e] & SQD_NBR_MASK;
    const uint32_t p = payload[e];
    const uint64_t i = p & 127, j = (p >> 7) & 127, a = (p >> 14) & 127, b = (p >> 21) & 127;
    const uint64_t neg = p >> 31;
    if (KIND == 0) {
        ent[e] = tgt | (i << 32) | (a << 39) | (neg << 63);
        const uint32_t pair = (uint32_t)(a * norb + i);
        pk[e] = (uint32_t)tgt | (pair << SQD_PAIR_SHIFT) | ((uint32_t)neg << 31);
    } else {
        ent[e] = tgt | (i << 32) | (j << 39) | (a << 46) | (b << 53) | (neg << 63);
        nbr[e] = (int)tgt;
    }
}

// Row lengths -> sort keys for the sliced layouts (longest rows first).
__global__ void k_len_keys(const int* __restrict__ off_a, const int* __restrict__ off_b, int64_t n,
                           uint32_t* __restrict__ keys, int* __restrict__ rows) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int len = off_a[r + 1] - off_a[r];
    if (off_b) len += off_b[r + 1] - off_b[r];
    keys[r] = 0x7FFFFFFFu - (uint32_t)len;
    rows[r] = (int)r;
}

// Per-slice maximum row lengths; perm is padded to nslices*64 with n.
__global__ void k_slice_max(const int* __restrict__ perm, int64_t n, int nslices,
                            const int* __restrict__ off_a, const int* __restrict__ off_b,
                            int* __restrict__ max_a, int* __restrict__ max_b) {
    const int sl = blockIdx.x;
    const int lane = threadIdx.x;
    const int r = perm[sl * 64 + lane];
    int la = 0, lb = 0;
    if (r < n) {
        la = off_a[r + 1] - off_a[r];
        if (off_b) lb = off_b[r + 1] - off_b[r];
    }
    for (int o = 32; o > 0; o >>= 1) {
        la = max(la, __shfl_xor(la, o));
        lb = max(lb, __shfl_xor(lb, o));
    }
    if (lane == 0) {
        max_a[sl] = la;
        if (max_b) max_b[sl] = lb;
    }
}

__global__ void k_pad_perm(const int* __restrict__ sorted_rows, int64_t n, int total, int* __restrict__ perm) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= total) return;
    perm[k] = (k < n) ? sorted_rows[k] : (int)n;
}

// Fill a sliced table: slot (slice, col, lane) takes CSR entry col of row
// perm[slice*64+lane] or a padding entry pointing at the zero slot n.
__global__ void k_sell_fill_pk(const int* __restrict__ perm, int64_t n, int nslices,
                               const int* __restrict__ sl_off, const int* __restrict__ off,
                               const uint32_t* __restrict__ pk, uint32_t* __restrict__ sell_pk,
                               int* __restrict__ sell_csr) {
    const int sl = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int r = perm[sl * 64 + lane];
    const int ncol = sl_off[sl + 1] - sl_off[sl];
    const int len = (r < n) ? off[r + 1] - off[r] : 0;
    for (int col = threadIdx.x >> 6; col < ncol; col += blockDim.x >> 6) {
        const int64_t pos = ((int64_t)sl_off[sl] + col) * 64 + lane;
        if (col < len) {
            const int src = off[r] + col;
            sell_pk[pos] = pk[src];
            if (sell_csr) sell_csr[pos] = src;
        } else {
            sell_pk[pos] = (uint32_t)n;   // neighbour = zero slot, pair 0, positive
            if (sell_csr) sell_csr[pos] = -1;
        }
    }
}

// Order each target's entries in the sliced alpha-beta table by pair index,
// so that lanes reading column k of a slice tend to look up nearby (often
// equal) integrals.  Padding stays at the end of each lane's column list.
__global__ void k_sell_sort_pairs(const int* __restrict__ perm, int64_t n, int nslices,
                                  const int* __restrict__ sl_off, const int* __restrict__ off,
                                  uint32_t* __restrict__ sell_pk) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)nslices * 64) return;
    const int sl = (int)(q >> 6), lane = (int)(q & 63);
    const int r = perm[q];
    if (r >= n) return;
    const int len = off[r + 1] - off[r];
    uint32_t* col = sell_pk + (int64_t)sl_off[sl] * 64 + lane;
    auto key = [](uint32_t x) { return (x >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK; };
    for (int i = 1; i < len; ++i) {   // insertion sort over the lane's entries (strided by 64)
        const uint32_t x = col[(int64_t)i * 64];
        int j = i - 1;
        while (j >= 0 && key(col[(int64_t)j * 64]) > key(x)) {
            col[(int64_t)(j + 1) * 64] = col[(int64_t)j * 64];
            --j;
        }
        col[(int64_t)(j + 1) * 64] = x;
    }
}

__global__ void k_sell_fill_nbr(const int* __restrict__ perm, int64_t n, int nslices,
                                const int* __restrict__ sl_off, const int* __restrict__ off,
                                const int* __restrict__ nbr, int* __restrict__ sell_nbr,
                                int* __restrict__ sell_csr) {
    const int sl = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int r = perm[sl * 64 + lane];
    const int ncol = sl_off[sl + 1] - sl_off[sl];
    const int len = (r < n) ? off[r + 1] - off[r] : 0;
    for (int col = threadIdx.x >> 6; col < ncol; col += blockDim.x >> 6) {
        const int64_t pos = ((int64_t)sl_off[sl] + col) * 64 + lane;
        if (col < len) {
            sell_nbr[pos] = nbr[off[r] + col];
            sell_csr[pos] = off[r] + col;
        } else {
            sell_nbr[pos] = (int)n;
            sell_csr[pos] = -1;
        }
    }
}

// ---- integral-dependent values ----

// e_same[r] = sum_{i in s} h_ii + 1/2 sum_{i,j in s} [(ii|jj) - (ij|ji)]
__global__ void k_same_energy(const uint64_t* __restrict__ str, int nw, int64_t n, int norb,
                              const double* __restrict__ h, const double* __restrict__ eri,
                              double* __restrict__ e) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint64_t* s = str + r * nw;
    const int64_t n2 = (int64_t)norb * norb;
    double acc = 0.0;
    str_for_each(s, nw, [&](int i) {
        acc += h[i * norb + i];
        str_for_each(s, nw, [&](int j) {
            acc += 0.5 * (eri[(int64_t)(i * norb + i) * n2 + j * norb + j] -
                          eri[(int64_t)(i * norb + j) * n2 + j * norb + i]);
        });
    });
    e[r] = acc;
}

// single (row string s, i -> a in the neighbour): sign * [h_ai + sum_{k in s}((ai|kk) - (ak|ki))]
__global__ void k_single_values(const uint64_t* __restrict__ str, int nw, const int* __restrict__ off, int64_t n,
                                const uint64_t* __restrict__ ent, int norb,
                                const double* __restrict__ h, const double* __restrict__ eri,
                                double* __restrict__ v64, float* __restrict__ v32) {
    const int64_t r = (int64_t)blockIdx.x;
    if (r >= n) return;
    const uint64_t* s = str + r * nw;
    const int64_t n2 = (int64_t)norb * norb;
    for (int e = off[r] + threadIdx.x; e < off[r + 1]; e += blockDim.x) {
        const uint64_t x = ent[e];
        const int i = SQD_ENT_ORB(x, 0), a = SQD_ENT_ORB(x, 1);
        double acc = h[a * norb + i];
        str_for_each(s, nw, [&](int k) {
            acc += eri[(int64_t)(a * norb + i) * n2 + k * norb + k] -
                   eri[(int64_t)(a * norb + k) * n2 + k * norb + i];
        });
        if (x >> 63) acc = -acc;
        v64[e] = acc;
        v32[e] = (float)acc;
    }
}

// double (i < j -> a < b): sign * [(ai|bj) - (aj|bi)]
__global__ void k_double_values(const uint64_t* __restrict__ ent, int64_t nnz, int norb,
                                const double* __restrict__ eri, double* __restrict__ v64,
                                float* __restrict__ v32) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const uint64_t x = ent[e];
    const int i = SQD_ENT_ORB(x, 0), j = SQD_ENT_ORB(x, 1);
    const int a = SQD_ENT_ORB(x, 2), b = SQD_ENT_ORB(x, 3);
    const int64_t n2 = (int64_t)norb * norb;
    double v = eri[(int64_t)(a * norb + i) * n2 + b * norb + j] - eri[(int64_t)(a * norb + j) * n2 + b * norb + i];
    if (x >> 63) v = -v;
    v64[e] = v;
    v32[e] = (float)v;
}

template <typename T>
__global__ void k_sell_values(const int* __restrict__ sell_csr, int64_t m, const T* __restrict__ v,
                              T* __restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int src = sell_csr[k];
    out[k] = (src >= 0) ? v[src] : (T)0;
}

inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Sort (key, value) pairs with rocPRIM's device radix sort; end_bit bits of key used.
template <typename K, typename V>
int radix_sort(sqd_ctx* ctx, K* keys, V* vals, int64_t n, int end_bit) {
    if (n <= 1) return SQD_OK;
    K* k2 = nullptr; V* v2 = nullptr; void* tmp = nullptr; size_t tmpb = 0;
    SQD_HIP(ctx, hipMalloc(&k2, sizeof(K) * n));
    SQD_HIP(ctx, hipMalloc(&v2, sizeof(V) * n));
    SQD_HIP(ctx, rocprim::radix_sort_pairs(nullptr, tmpb, keys, k2, vals, v2, (size_t)n, 0u, (unsigned)end_bit,
                                           ctx->stream));
    SQD_HIP(ctx, hipMalloc(&tmp, tmpb > 0 ? tmpb : 1));
    SQD_HIP(ctx, rocprim::radix_sort_pairs(tmp, tmpb, keys, k2, vals, v2, (size_t)n, 0u, (unsigned)end_bit, ctx->stream));
    SQD_HIP(ctx, hipMemcpyAsync(keys, k2, sizeof(K) * n, hipMemcpyDeviceToDevice, ctx->stream));
    SQD_HIP(ctx, hipMemcpyAsync(vals, v2, sizeof(V) * n, hipMemcpyDeviceToDevice, ctx->stream));
    SQD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    hipFree(k2); hipFree(v2); hipFree(tmp);
    return SQD_OK;
}

// Build one kind (singles or doubles) of canonical CSR table.
template <int KIND>
int build_kind(sqd_ctx* ctx, sqd_space* sp, spin_tables& t, int** off_out, uint64_t** ent_out,
               uint32_t** pk_out, int** nbr_out, int64_t* nnz_out) {
    const int norb = sp->norb;
    int* counts = nullptr;
    long long* dtot = nullptr;
    SQD_HIP(ctx, hipMalloc(&counts, sizeof(int) * (t.n + 1)));
    SQD_HIP(ctx, hipMalloc(&dtot, sizeof(long long)));
    int* off = nullptr;
    int rc = sqd_alloc(ctx, (void**)&off, sizeof(int) * (t.n + 1), &sp->bytes);
    if (rc) return rc;
    uint64_t* keys_ = nullptr;
    uint32_t* pay_ = nullptr;
    auto launch_enum = [&](int mode) {
        const int wpb = t.nw == 1 ? enum_shape<1>::kWaves : enum_shape<2>::kWaves;
        const dim3 grid(nblocks(t.n, wpb)), block(64 * wpb);
        int* cnt = mode == 0 ? counts : nullptr;
        const int* of = mode == 0 ? nullptr : off;
        uint64_t* ky = mode == 0 ? nullptr : keys_;
        uint32_t* py = mode == 0 ? nullptr : pay_;
        if (t.nw == 1) {
            if (mode == 0) hipLaunchKernelGGL((k_enum<KIND, 0, 1>), grid, block, 0, ctx->stream, t.str, t.n, norb, t.nel, cnt, of, ky, py);
            else hipLaunchKernelGGL((k_enum<KIND, 1, 1>), grid, block, 0, ctx->stream, t.str, t.n, norb, t.nel, cnt, of, ky, py);
        } else {
            if (mode == 0) hipLaunchKernelGGL((k_enum<KIND, 0, 2>), grid, block, 0, ctx->stream, t.str, t.n, norb, t.nel, cnt, of, ky, py);
            else hipLaunchKernelGGL((k_enum<KIND, 1, 2>), grid, block, 0, ctx->stream, t.str, t.n, norb, t.nel, cnt, of, ky, py);
        }
    };
    launch_enum(0);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, ctx->stream, counts, t.n, off, dtot);
    long long total = 0;
    SQD_HIP(ctx, hipMemcpyAsync(&total, dtot, sizeof(long long), hipMemcpyDeviceToHost, ctx->stream));
    SQD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    SQD_HIP(ctx, hipGetLastError());
    if (total >= (1LL << 31) - 64LL * 1024) {
        hipFree(counts); hipFree(dtot);
        return sqd_fail(ctx, SQD_E_LIMIT, "excitation table exceeds 2^31 entries");
    }
    const int64_t nnz = total;
    uint64_t* keys = nullptr; uint32_t* pay = nullptr;
    SQD_HIP(ctx, hipMalloc(&keys, sizeof(uint64_t) * (nnz + 1)));
    SQD_HIP(ctx, hipMalloc(&pay, sizeof(uint32_t) * (nnz + 1)));
    keys_ = keys;
    pay_ = pay;
    launch_enum(1);
    SQD_HIP(ctx, hipGetLastError());
    rc = radix_sort(ctx, keys, pay, nnz, 34);   // (row << 17 | target): rows, then targets
    if (rc) return rc;
    uint64_t* ent = nullptr; uint32_t* pk = nullptr; int* nbr = nullptr;
    if ((rc = sqd_alloc(ctx, (void**)&ent, sizeof(uint64_t) * (nnz + 1), &sp->bytes))) return rc;
    if (KIND == 0) {
        if ((rc = sqd_alloc(ctx, (void**)&pk, sizeof(uint32_t) * (nnz + 1), &sp->bytes))) return rc;
    } else {
        if ((rc = sqd_alloc(ctx, (void**)&nbr, sizeof(int) * (nnz + 1), &sp->bytes))) return rc;
    }
    if (nnz > 0)
        hipLaunchKernelGGL((k_pack<KIND>), dim3(nblocks(nnz, 256)), dim3(256), 0, ctx->stream,
                           keys, pay, nnz, norb, ent, pk, nbr);
    SQD_HIP(ctx, hipGetLastError());
    SQD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    hipFree(keys); hipFree(pay); hipFree(counts); hipFree(dtot);
    *off_out = off; *ent_out = ent; *pk_out = pk; *nbr_out = nbr; *nnz_out = nnz;
    return SQD_OK;
}

// Sorted row order (longest first) padded to whole 64-row slices.
int make_perm(sqd_ctx* ctx, sqd_space* sp, spin_tables& t, const int* off_a, const int* off_b,
              int** perm_out) {
    const int nslices = (int)((t.n + 63) / 64);
    uint32_t* keys = nullptr; int* rows = nullptr; int* perm = nullptr;
    SQD_HIP(ctx, hipMalloc(&keys, sizeof(uint32_t) * t.n));
    SQD_HIP(ctx, hipMalloc(&rows, sizeof(int) * t.n));
    int rc = sqd_alloc(ctx, (void**)&perm, sizeof(int) * nslices * 64, &sp->bytes);
    if (rc) return rc;
    hipLaunchKernelGGL(k_len_keys, dim3(nblocks(t.n, 256)), dim3(256), 0, ctx->stream, off_a, off_b, t.n, keys, rows);
    rc = radix_sort(ctx, keys, rows, t.n, 32);
    if (rc) return rc;
    hipLaunchKernelGGL(k_pad_perm, dim3(nblocks(nslices * 64, 256)), dim3(256), 0, ctx->stream, rows, t.n,
                       nslices * 64, perm);
    SQD_HIP(ctx, hipGetLastError());
    SQD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    hipFree(keys); hipFree(rows);
    *perm_out = perm;
    return SQD_OK;
}

// Slice offsets (units of 64 entries) from per-slice maxima.
int slice_offsets(sqd_ctx* ctx, sqd_space* sp, int nslices, const int* maxes, int** sl_off, int64_t* total) {
    long long* dtot = nullptr;
    SQD_HIP(ctx, hipMalloc(&dtot, sizeof(long long)));
    int rc = sqd_alloc(ctx, (void**)sl_off, sizeof(int) * (nslices + 1), &sp->bytes);
    if (rc) return rc;
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, ctx->stream, maxes, (int64_t)nslices, *sl_off, dtot);
    long long tot = 0;
    SQD_HIP(ctx, hipMemcpyAsync(&tot, dtot, sizeof(long long), hipMemcpyDeviceToHost, ctx->stream));
    SQD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    hipFree(dtot);
    if (tot * 64 >= (1LL << 31)) return sqd_fail(ctx, SQD_E_LIMIT, "sliced table exceeds 2^31 slots");
    *total = tot;
    return SQD_OK;
}

}  // namespace

int sqd_build_spin_tables(sqd_ctx* ctx, sqd_space* sp, int spin, const uint64_t* host_str, int64_t n, int nel) {
    spin_tables& t = sp->sp[spin];
    t.n = n;
    t.nel = nel;
    t.nw = sp->nw;
    int rc = sqd_alloc(ctx, (void**)&t.str, sizeof(uint64_t) * (n > 0 ? n : 1) * t.nw, &sp->bytes);
    if (rc) return rc;
    SQD_HIP(ctx, hipMemcpyAsync(t.str, host_str, sizeof(uint64_t) * n * t.nw, hipMemcpyHostToDevice, ctx->stream));
    int* dummy_nbr = nullptr; uint32_t* dummy_pk = nullptr;
    if ((rc = build_kind<0>(ctx, sp, t, &t.s_off, &t.s_ent, &t.s_pk, &dummy_nbr, &t.nnz_s))) return rc;
    if ((rc = build_kind<1>(ctx, sp, t, &t.d_off, &t.d_ent, &dummy_pk, &t.d_nbr, &t.nnz_d))) return rc;

    // same-spin sliced layout: rows sorted by singles + doubles
    t.nslices = (int)((n + 63) / 64);
    if ((rc = make_perm(ctx, sp, t, t.s_off, t.d_off, &t.perm_ss))) return rc;
    int *mx_s = nullptr, *mx_d = nullptr;
    SQD_HIP(ctx, hipMalloc(&mx_s, sizeof(int) * (t.nslices + 1)));
    SQD_HIP(ctx, hipMalloc(&mx_d, sizeof(int) * (t.nslices + 1)));
    hipLaunchKernelGGL(k_slice_max, dim3(t.nslices), dim3(64), 0, ctx->stream, t.perm_ss, n, t.nslices, t.s_off,
                       t.d_off, mx_s, mx_d);
    int64_t tot_s = 0, tot_d = 0;
    if ((rc = slice_offsets(ctx, sp, t.nslices, mx_s, &t.sl_s_off, &tot_s))) return rc;
    if ((rc = slice_offsets(ctx, sp, t.nslices, mx_d, &t.sl_d_off, &tot_d))) return rc;
    t.sell_ss_entries = (tot_s + tot_d) * 64;
    int* csr_s = nullptr; int* csr_d = nullptr;
    if ((rc = sqd_alloc(ctx, (void**)&t.sell_s_pk, sizeof(uint32_t) * (tot_s * 64 + 1), &sp->bytes))) return rc;
    if ((rc = sqd_alloc(ctx, (void**)&t.sell_d_nbr, sizeof(int) * (tot_d * 64 + 1), &sp->bytes))) return rc;
    if ((rc = sqd_alloc(ctx, (void**)&csr_s, sizeof(int) * (tot_s * 64 + 1), &sp->bytes))) return rc;
    if ((rc = sqd_alloc(ctx, (void**)&csr_d, sizeof(int) * (tot_d * 64 + 1), &sp->bytes))) return rc;
    if ((rc = sqd_alloc(ctx, (void**)&t.sell_s_v64, sizeof(double) * (tot_s * 64 + 1), &sp->bytes))) return rc;
    if ((rc = sqd_alloc(ctx, (void**)&t.sell_s_v32, sizeof(float) * (tot_s * 64 + 1), &sp->bytes))) return rc;
    if ((rc = sqd_alloc(ctx, (void**)&t.sell_d_v64, sizeof(double) * (tot_d * 64 + 1), &sp->bytes))) return rc;
    if ((rc = sqd_alloc(ctx, (void**)&t.sell_d_v32, sizeof(float) * (tot_d * 64 + 1), &sp->bytes))) return rc;
    hipLaunchKernelGGL(k_sell_fill_pk, dim3(t.nslices), dim3(256), 0, ctx->stream, t.perm_ss, n, t.nslices,
                       t.sl_s_off, t.s_off, t.s_pk, t.sell_s_pk, csr_s);
    hipLaunchKernelGGL(k_sell_fill_nbr, dim3(t.nslices), dim3(256), 0, ctx->stream, t.perm_ss, n, t.nslices,
                       t.sl_d_off, t.d_off, t.d_nbr, t.sell_d_nbr, csr_d);
    SQD_HIP(ctx, hipGetLastError());

    // alpha-beta sliced singles: rows sorted by singles count
    if ((rc = make_perm(ctx, sp, t, t.s_off, nullptr, &t.perm_ab))) return rc;
    hipLaunchKernelGGL(k_slice_max, dim3(t.nslices), dim3(64), 0, ctx->stream, t.perm_ab, n, t.nslices, t.s_off,
                       nullptr, mx_s, nullptr);
    int64_t tot_ab = 0;
    if ((rc = slice_offsets(ctx, sp, t.nslices, mx_s, &t.sl_ab_off, &tot_ab))) return rc;
    t.sell_ab_entries = tot_ab * 64;
    if ((rc = sqd_alloc(ctx, (void**)&t.sell_ab_pk, sizeof(uint32_t) * (tot_ab * 64 + 1), &sp->bytes))) return rc;
    hipLaunchKernelGGL(k_sell_fill_pk, dim3(t.nslices), dim3(256), 0, ctx->stream, t.perm_ab, n, t.nslices,
                       t.sl_ab_off, t.s_off, t.s_pk, t.sell_ab_pk, nullptr);
    hipLaunchKernelGGL(k_sell_sort_pairs, dim3((unsigned)(((int64_t)t.nslices * 64 + 255) / 256)), dim3(256), 0,
                       ctx->stream, t.perm_ab, n, t.nslices, t.sl_ab_off, t.s_off, t.sell_ab_pk);
    SQD_HIP(ctx, hipGetLastError());
    SQD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    hipFree(mx_s); hipFree(mx_d);

    // value arrays (CSR order)
    if ((rc = sqd_alloc(ctx, (void**)&t.s_val64, sizeof(double) * (t.nnz_s + 1), &sp->bytes))) return rc;
    if ((rc = sqd_alloc(ctx, (void**)&t.s_val32, sizeof(float) * (t.nnz_s + 1), &sp->bytes))) return rc;
    if ((rc = sqd_alloc(ctx, (void**)&t.d_val64, sizeof(double) * (t.nnz_d + 1), &sp->bytes))) return rc;
    if ((rc = sqd_alloc(ctx, (void**)&t.d_val32, sizeof(float) * (t.nnz_d + 1), &sp->bytes))) return rc;
    if ((rc = sqd_alloc(ctx, (void**)&t.e_same, sizeof(double) * (n + 1), &sp->bytes))) return rc;
    t.sell_csr_s = csr_s;
    t.sell_csr_d = csr_d;
    // host-side maxima for kernel launch shapes
    std::vector<int> off_h(n + 1);
    SQD_HIP(ctx, hipMemcpy(off_h.data(), t.s_off, sizeof(int) * (n + 1), hipMemcpyDeviceToHost));
    t.max_singles = 0;
    for (int64_t r = 0; r < n; ++r) t.max_singles = std::max(t.max_singles, off_h[r + 1] - off_h[r]);
    SQD_HIP(ctx, hipMemcpy(off_h.data(), t.d_off, sizeof(int) * (n + 1), hipMemcpyDeviceToHost));
    t.max_doubles = 0;
    for (int64_t r = 0; r < n; ++r) t.max_doubles = std::max(t.max_doubles, off_h[r + 1] - off_h[r]);
    return SQD_OK;
}

int sqd_build_values(sqd_ctx* ctx, sqd_space* sp) {
    if (sp->values_version == ctx->ham_version) return SQD_OK;
    const int norb = sp->norb;
    for (int spin = 0; spin < 2; ++spin) {
        spin_tables& t = sp->sp[spin];
        if (t.alias) continue;
        if (t.n > 0) {
            hipLaunchKernelGGL(k_same_energy, dim3(nblocks(t.n, 128)), dim3(128), 0, ctx->stream, t.str, t.nw, t.n,
                               norb, ctx->h, ctx->eri, t.e_same);
            hipLaunchKernelGGL(k_single_values, dim3((unsigned)t.n), dim3(64), 0, ctx->stream, t.str, t.nw, t.s_off,
                               t.n, t.s_ent, norb, ctx->h, ctx->eri, t.s_val64, t.s_val32);
        }
        if (t.nnz_d > 0)
            hipLaunchKernelGGL(k_double_values, dim3(nblocks(t.nnz_d, 256)), dim3(256), 0, ctx->stream, t.d_ent,
                               t.nnz_d, norb, ctx->eri, t.d_val64, t.d_val32);
        int s_slots = 0, d_slots = 0;
        SQD_HIP(ctx, hipMemcpy(&s_slots, t.sl_s_off + t.nslices, sizeof(int), hipMemcpyDeviceToHost));
        SQD_HIP(ctx, hipMemcpy(&d_slots, t.sl_d_off + t.nslices, sizeof(int), hipMemcpyDeviceToHost));
        const int64_t S = (int64_t)s_slots * 64, D = (int64_t)d_slots * 64;
        if (S > 0) {
            hipLaunchKernelGGL(k_sell_values<double>, dim3(nblocks(S, 256)), dim3(256), 0, ctx->stream, t.sell_csr_s, S,
                               t.s_val64, t.sell_s_v64);
            hipLaunchKernelGGL(k_sell_values<float>, dim3(nblocks(S, 256)), dim3(256), 0, ctx->stream, t.sell_csr_s, S,
                               t.s_val32, t.sell_s_v32);
        }
        if (D > 0) {
            hipLaunchKernelGGL(k_sell_values<double>, dim3(nblocks(D, 256)), dim3(256), 0, ctx->stream, t.sell_csr_d, D,
                               t.d_val64, t.sell_d_v64);
            hipLaunchKernelGGL(k_sell_values<float>, dim3(nblocks(D, 256)), dim3(256), 0, ctx->stream, t.sell_csr_d, D,
                               t.d_val32, t.sell_d_v32);
        }
        SQD_HIP(ctx, hipGetLastError());
    }
    SQD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    sp->values_version = ctx->ham_version;
    return SQD_OK;
}

void sqd_free_spin_tables(spin_tables* t) {
    if (t->alias) { *t = spin_tables(); return; }
    sqd_free_window_tables(t);
    void* ptrs[] = {t->str, t->s_off, t->s_ent, t->d_off, t->d_ent, t->s_pk, t->d_nbr, t->s_val64, t->s_val32,
                    t->d_val64, t->d_val32, t->e_same, t->perm_ss, t->sl_s_off, t->sl_d_off, t->sell_s_pk,
                    t->sell_s_v64, t->sell_s_v32, t->sell_d_nbr, t->sell_d_v64, t->sell_d_v32, t->perm_ab,
                    t->sl_ab_off, t->sell_ab_pk, t->sell_csr_s, t->sell_csr_d};
    for (void* p : ptrs)
        if (p) hipFree(p);
    *t = spin_tables();
}
