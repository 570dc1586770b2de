// Internal declarations of libsqd (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/sqd.h"

// gather form of a single excitation: neighbour (17 bits) | orbital pair
// a * norb + i (14 bits, norb <= 128) | negative sign (bit 31)
#define SQD_MAXN 131071          // strings per spin (17-bit neighbour field)
#define SQD_NBR_MASK 0x1FFFFu
#define SQD_PAIR_SHIFT 17
#define SQD_PAIR_MASK 0x3FFFu
#define SQD_WAVE 64
#define SQD_MAXORB 128           // orbitals: strings of one or two 64-bit words

// canonical table entries (sqd_get_tables): target | o0 << 32 | o1 << 39 |
// o2 << 46 | o3 << 53 | negative << 63, orbitals in 7-bit fields; singles
// (o0, o1) = (i, a), doubles (o0, o1, o2, o3) = (i, j, a, b)
#define SQD_ENT_ORB(x, f) ((int)(((x) >> (32 + 7 * (f))) & 127u))

struct sqd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int tune[SQD_TUNE_COUNT] = {};
    int max_lds = 65536;          // bytes of LDS a workgroup may allocate
    int num_cu = 256;
    // Hamiltonian
    int norb = 0;
    double ecore = 0.0;
    int ham_version = 0;
    double* h = nullptr;          // norb^2
    double* eri = nullptr;        // norb^4 (also the norb^2 x norb^2 matrix V)
    float* eri32 = nullptr;
    double* jk64 = nullptr;       // Jk[k*norb2 + pq] = (pq|kk)
    float* jk32 = nullptr;
    double* jdiag = nullptr;      // J[p*norb+q] = (pp|qq)
    std::vector<double> h_host, eri_host;
    // scratch shared by products on this context; once a call has been
    // captured into a graph with it (scratch_captured) a grown scratch does
    // not free the old buffer, which the graph may still use: it is retired
    // and freed only by sqd_release_workspace / sqd_destroy
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    bool scratch_captured = false;
    std::vector<void*> scratch_retired;
    // spaces built on this context (sqd_destroy releases their device memory)
    std::vector<sqd_space*> spaces;
    // workspace of the batched solver (grown on demand, kept across calls)
    void* batch_arena = nullptr;
    size_t batch_arena_bytes = 0;
    int* batch_count_host = nullptr;   // pinned
    // workspace of the single-space Davidson solver (grown on demand)
    void* dav_arena = nullptr;
    size_t dav_arena_bytes = 0;
    void* dav_state_host = nullptr;    // pinned
    // per-kernel HIP-event timers (sqd_profile)
    bool profiling = false;
    struct prof_rec { const char* name; hipEvent_t a, b; };
    std::vector<prof_rec> prof;
    std::vector<hipEvent_t> prof_pool;
};

// Records HIP events on the context's stream around the launches in its scope
// while profiling is on (sqd_profile); names must be string literals.
struct prof_scope {
    sqd_ctx* ctx;
    const char* name;
    hipEvent_t a = nullptr;
    static hipEvent_t take(sqd_ctx* c) {
        if (!c->prof_pool.empty()) {
            hipEvent_t e = c->prof_pool.back();
            c->prof_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    prof_scope(sqd_ctx* c, const char* n) : ctx(c), name(n) {
        if (ctx->profiling && (a = take(ctx))) (void)hipEventRecord(a, ctx->stream);
    }
    ~prof_scope() {
        if (!a) return;
        hipEvent_t b = take(ctx);
        if (!b) return;
        (void)hipEventRecord(b, ctx->stream);
        ctx->prof.push_back({name, a, b});
    }
};

// Per-spin tables of one string set (Sec. V-A flattened lists).
struct spin_tables {
    int64_t n = 0;                // strings
    int nel = 0;
    int nw = 1;                   // 64-bit words per string (word q: orbitals 64q .. 64q+63)
    uint64_t* str = nullptr;      // ascending strings, nw words each
    // canonical CSR (rows = source strings, entries sorted by target)
    int* s_off = nullptr;         // n+1
    uint64_t* s_ent = nullptr;    // packed canonical singles
    int* d_off = nullptr;
    uint64_t* d_ent = nullptr;
    int64_t nnz_s = 0, nnz_d = 0;
    // gather form of the singles: nbr | pair << 19 | negative << 31
    uint32_t* s_pk = nullptr;
    int* d_nbr = nullptr;
    // integral-dependent values (rebuilt when the Hamiltonian changes)
    double* s_val64 = nullptr; float* s_val32 = nullptr;
    double* d_val64 = nullptr; float* d_val32 = nullptr;
    double* e_same = nullptr;     // same-spin diagonal energy per string
    // sliced (SELL-64) copies for the same-spin kernel, rows sorted by length
    int nslices = 0;
    int* perm_ss = nullptr;       // nslices*64, padded with n
    int* sl_s_off = nullptr;      // nslices+1 (units of 64 entries)
    int* sl_d_off = nullptr;
    uint32_t* sell_s_pk = nullptr;
    double* sell_s_v64 = nullptr; float* sell_s_v32 = nullptr;
    int* sell_d_nbr = nullptr;
    double* sell_d_v64 = nullptr; float* sell_d_v32 = nullptr;
    // sliced singles for the alpha-beta kernel (rows sorted by singles count)
    int* perm_ab = nullptr;
    int* sl_ab_off = nullptr;
    uint32_t* sell_ab_pk = nullptr;
    int* sell_csr_s = nullptr;    // CSR index of each sliced slot (-1 = padding)
    int* sell_csr_d = nullptr;
    int64_t sell_ss_entries = 0, sell_ab_entries = 0;
    int max_singles = 0, max_doubles = 0;
    bool alias = false;           // arrays owned by the other spin
    // windowed sliced tables for rows too long to stage whole (window.hip):
    // the source strings are dealt into win_W interleaved windows (source j in
    // window j mod W, local index j / W, at most win_width per window); part w
    // lists, per target in the perm_ss order, the entries of window w
    int win_W = 0, win_width = 0, win_values_version = -1;
    int* win_s_off = nullptr;     // win_W * (nslices + 1) slot-column offsets (units of 64)
    int* win_d_off = nullptr;
    uint32_t* win_s_pk = nullptr; // local source | pair << 17 | negative << 31
    uint16_t* win_d_nbr = nullptr; // local source (below the window width)
    int* win_islot = nullptr;     // n: slot of each target in the perm_ss order
    int* win_s_csr = nullptr;     // CSR index of each slot (-1: padding)
    int* win_d_csr = nullptr;
    double* win_s_v64 = nullptr; float* win_s_v32 = nullptr;
    double* win_d_v64 = nullptr; float* win_d_v32 = nullptr;
    int64_t win_bytes = 0;
    // cross-spin table of these strings as the row spin: wg[pq * ldw + s] =
    // sum_{k in s} (pq|kk) (FP64 and FP32; ldw = n rounded up to 16, zero
    // past n), per Hamiltonian version
    double* wg64 = nullptr; float* wg32 = nullptr;
    int wg_version = -1;
};

struct sqd_space {
    sqd_ctx* ctx = nullptr;       // null once the context was destroyed (orphan)
    int norb = 0;
    int nw = 1;                   // 64-bit words per string
    int nalpha = 0, nbeta = 0;
    spin_tables sp[2];            // 0 alpha, 1 beta
    int values_version = -1;      // ham_version the values were built for
    int64_t dim = 0;
    int64_t bytes = 0;
    // diagonal cache (FP64), per Hamiltonian version
    double* diag = nullptr;
    int diag_version = -1;
    double* ua = nullptr;         // na x norb: sum_{p in Ia} (pp|qq)
    // alpha singles grouped by orbital pair for the grouped alpha-beta kernel
    int ab_G = 0;                 // entries per chunk (0 = not built)
    int ab_nchunks = 0;
    int* ab_grp = nullptr;        // ab_nchunks * ab_G CSR positions (-1 = padding)
    int* ab_chunk_pair = nullptr; // pair index of each chunk
    int* ab_rev = nullptr;        // alpha singles: entry of the neighbour's row pointing back
    int* ab_row_order = nullptr;  // alpha rows by decreasing number of singles (gather order)
    // the same singles grouped by source string (rows too long for two
    // staged sources: one staged source row serves several pairs)
    int abs_G = 0;
    int abs_nchunks = 0;
    int* abs_grp = nullptr;       // abs_nchunks * abs_G CSR positions (-1 = padding)
    int* abs_src = nullptr;       // source alpha string of each chunk
    // Knowles-Handy beta tiles (64 targets each): the union of the pair columns
    // their singles use, and for every (target, column) the source of that
    // single (0: none, else source + 1, bit 31 = negative sign)
    int kh_ntiles = 0;
    int* kh_tile_off = nullptr;   // ntiles + 1 offsets into kh_pairs
    int* kh_pairs = nullptr;      // ascending pair indices per tile
    int* kh_map = nullptr;        // tile t: 64 x K_t entries at 64 * kh_tile_off[t]
    int64_t kh_cols = 0;          // sum over tiles of (targets in tile) x K_t
    int kh_kmax = 0;              // largest K_t
    // stored H (CSR of H restricted to S; built on request, per Hamiltonian version)
    int64_t* h_rowptr = nullptr;  // dim + 1
    int* h_col = nullptr;         // nnz column indices
    double* h_val = nullptr;      // nnz values
    int64_t h_nnz = 0;
    int64_t h_bytes = 0;
    int h_version = -1;
    int64_t h_xcd_rows[9] = {};   // row ranges of equal element counts, one per XCD
    // partial sums of the windowed same-spin kernel (rows x slots, FP64-sized)
    void* win_P = nullptr;
    size_t win_P_bytes = 0;
};

// ---- helpers (api.hip) ----
int sqd_fail(sqd_ctx* ctx, int code, const std::string& msg);
int sqd_hip_fail(sqd_ctx* ctx, hipError_t e, const char* what);
int sqd_alloc(sqd_ctx* ctx, void** p, size_t bytes, int64_t* counter);
void* sqd_ctx_scratch(sqd_ctx* ctx, size_t bytes, int* rc);
bool sqd_capturing(sqd_ctx* ctx);

#define SQD_HIP(ctx, call)                                              \
    do {                                                                \
        hipError_t _e = (call);                                         \
        if (_e != hipSuccess) return sqd_hip_fail((ctx), _e, #call);    \
    } while (0)

// ---- noalloc.hip ----
int sqd_noalloc_init(int device);   // device address of the static product scratch

// ---- tables.hip ----
int sqd_build_spin_tables(sqd_ctx* ctx, sqd_space* sp, int spin, const uint64_t* host_str,
                          int64_t n, int nel);   // host_str: n x sp->nw words
int sqd_build_values(sqd_ctx* ctx, sqd_space* sp);   // integral-dependent parts
void sqd_free_spin_tables(spin_tables* t);

// ---- sigma.hip ----
int sqd_ensure_diag(sqd_ctx* ctx, sqd_space* sp);
int sqd_sigma_impl(sqd_ctx* ctx, sqd_space* sp, const double* c, double* sigma,
                   int precision, unsigned mask, int ab_path, const float* c32_in,
                   const int* skip_flag, void* ext_scratch = nullptr, size_t ext_bytes = 0);
int sqd_sigma_auto_path(sqd_ctx* ctx, const sqd_space* sp, int precision);
bool sqd_sigma_prepared(sqd_ctx* ctx, const sqd_space* sp, int precision, unsigned mask, int ab_path);
int sqd_ensure_ab_groups(sqd_ctx* ctx, sqd_space* sp, int G);
// the alpha singles grouped by source string, chunks of G (for the batched solver)
int sqd_ensure_ab_source_groups(sqd_ctx* ctx, sqd_space* sp, int G);

// ---- kh.hip ----
size_t sqd_kh_bytes(const sqd_space* sp, size_t es);
int sqd_sigma_ab_kh(sqd_ctx* ctx, sqd_space* sp, const void* c, void* sigma, void* y, int fp32,
                    const int* skip_flag);

// ---- window.hip ----
// Same-spin term for rows too long to stage whole: X (nrows x ncols) times the
// column spin's tables, by windows of source strings; Y written, or added to
// with accumulate.  col / row: the owning spin_tables of the column and row
// spins.  diag (FP64, row-major, or null): where the output is placed by the
// coalesced pass after the kernel, that pass adds diag * X too and sets
// *diag_done; otherwise the caller adds the diagonal.
int sqd_same_spin_windowed(sqd_ctx* ctx, sqd_space* sp, spin_tables& col, spin_tables& row, const void* X, void* Y,
                           int64_t nrows, int64_t ncols, int colmajor, int accumulate, int fp32, const double* diag,
                           int* diag_done, const int* skip, const char* timer);
void sqd_free_window_tables(spin_tables* t);
bool sqd_space_built_for(sqd_ctx* ctx, const sqd_space* sp, int precision, unsigned mask);
int sqd_window_count(sqd_ctx* ctx, int64_t ncols);    // 0: a window does not fit
size_t sqd_window_scratch_bytes(const sqd_space* sp);

// ---- stored.hip ----
int sqd_store_h_impl(sqd_ctx* ctx, sqd_space* sp, int64_t* nnz_out);
int sqd_spmv_impl(sqd_ctx* ctx, sqd_space* sp, const double* x, double* y, const int* skip_flag);
void sqd_release_stored_h(sqd_space* sp);

// ---- davidson.hip ----
int sqd_davidson_impl(sqd_ctx* ctx, sqd_space* sp, const sqd_davidson_opts* o, double* energy, double* vec,
                      sqd_report* rep, int nroots);

// ---- block.hip ----
int sqd_davidson_block_impl(sqd_ctx* ctx, sqd_space* sp, const sqd_davidson_opts* o, int nroots,
                            double* energies, double* vecs, sqd_report* reps);

// ---- rdm.hip ----
int sqd_rdm_impl(sqd_ctx* ctx, sqd_space* sp, const double* c, double* rdm1, double* rdm2);

// ---- batched.hip ----
int sqd_davidson_batched_impl(sqd_ctx* ctx, int nspace, sqd_space* const* spaces,
                              const sqd_davidson_opts* o, double* energies,
                              double* const* vecs, sqd_report* reps);

// ---- device helpers shared by kernels ----
__device__ __forceinline__ int dev_popc(uint64_t x) { return __popcll(x); }

// bit k of a string of nw words
__device__ __forceinline__ bool str_bit(const uint64_t* s, int k) { return (s[k >> 6] >> (k & 63)) & 1ull; }

// f(k) for every occupied orbital k of a string of nw words, ascending
template <typename F>
__device__ __forceinline__ void str_for_each(const uint64_t* s, int nw, F&& f) {
    for (int q = 0; q < nw; ++q)
        for (uint64_t x = s[q]; x; x &= x - 1) f(64 * q + __ffsll((unsigned long long)x) - 1);
}
