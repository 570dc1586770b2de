// C-ABI entry points of libsqd: context, integrals, string spaces, products,
// eigensolver and RDM calls.  Argument checking happens here; the work is in
// tables.hip, sigma.hip, kh.hip, davidson.hip, rdm.hip and batched.hip.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "sqd_internal.h"

#define SQD_VERSION_STRING "libsqd 0.1 gfx950"

int sqd_fail(sqd_ctx* ctx, int code, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return code;
}

int sqd_hip_fail(sqd_ctx* ctx, hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return sqd_fail(ctx, SQD_E_OOM, std::string("device allocation failed: ") + what);
    return sqd_fail(ctx, SQD_E_HIP, std::string(hipGetErrorString(e)) + " in " + what);
}

int sqd_alloc(sqd_ctx* ctx, void** p, size_t bytes, int64_t* counter) {
    hipError_t e = hipMalloc(p, bytes > 0 ? bytes : 16);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return sqd_fail(ctx, SQD_E_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    if (counter) *counter += (int64_t)bytes;
    return SQD_OK;
}

bool sqd_capturing(sqd_ctx* ctx) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(ctx->stream, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return cs != hipStreamCaptureStatusNone;
}

// Context scratch of at least `bytes`.  Under stream capture nothing is
// allocated or freed: the scratch must already be large enough (else
// SQD_E_STATE), and it is marked as referenced by a graph.  A later growth
// then retires the old buffer instead of freeing it.
void* sqd_ctx_scratch(sqd_ctx* ctx, size_t bytes, int* rc) {
    if (sqd_capturing(ctx)) {
        if (ctx->scratch_bytes < bytes) {
            if (rc) *rc = SQD_E_STATE;
            return nullptr;
        }
        ctx->scratch_captured = true;
        return ctx->scratch;
    }
    if (ctx->scratch_bytes >= bytes) return ctx->scratch;
    if (ctx->scratch) {
        (void)hipStreamSynchronize(ctx->stream);
        if (ctx->scratch_captured) ctx->scratch_retired.push_back(ctx->scratch);
        else (void)hipFree(ctx->scratch);
        ctx->scratch = nullptr;
        ctx->scratch_bytes = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        if (rc) *rc = SQD_E_OOM;
        return nullptr;
    }
    ctx->scratch = p;
    ctx->scratch_bytes = bytes;
    return p;
}

// Jk[k*norb2 + pq] = (pq|kk); jdiag[p*norb + q] = (pp|qq)
__global__ void k_jtables(const double* __restrict__ eri, int norb, double* __restrict__ jk64,
                          float* __restrict__ jk32, double* __restrict__ jdiag, float* __restrict__ eri32) {
    const int n2 = norb * norb;
    const int64_t n4 = (int64_t)n2 * n2;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n4) eri32[idx] = (float)eri[idx];
    if (idx < (int64_t)norb * n2) {
        const int k = (int)(idx / n2), pq = (int)(idx % n2);
        const double v = eri[(int64_t)pq * n2 + k * norb + k];
        jk64[idx] = v;
        jk32[idx] = (float)v;
    }
    if (idx < n2) {
        const int p = (int)(idx / norb), q = (int)(idx % norb);
        jdiag[idx] = eri[(int64_t)(p * norb + p) * n2 + q * norb + q];
    }
}

static void free_ham(sqd_ctx* ctx) {
    void* ps[] = {ctx->h, ctx->eri, ctx->eri32, ctx->jk64, ctx->jk32, ctx->jdiag};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    ctx->h = ctx->eri = ctx->jk64 = ctx->jdiag = nullptr;
    ctx->eri32 = ctx->jk32 = nullptr;
}

static void free_scratch(sqd_ctx* ctx) {
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    for (void* p : ctx->scratch_retired) (void)hipFree(p);
    ctx->scratch_retired.clear();
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
    ctx->scratch_captured = false;
}

// Device memory of a space (the host struct stays).
static void space_release_device(sqd_space* sp) {
    sqd_release_stored_h(sp);
    sqd_free_spin_tables(&sp->sp[1]);
    sqd_free_spin_tables(&sp->sp[0]);
    void* ptrs[] = {sp->diag, sp->ua, sp->ab_grp, sp->ab_chunk_pair, sp->ab_rev, sp->kh_tile_off, sp->kh_pairs,
                    sp->kh_map, sp->ab_row_order, sp->win_P, sp->abs_grp, sp->abs_src};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    sp->diag = sp->ua = nullptr;
    sp->ab_grp = sp->ab_chunk_pair = sp->ab_rev = sp->kh_tile_off = sp->kh_pairs = sp->kh_map = nullptr;
    sp->ab_row_order = nullptr;
    sp->abs_grp = sp->abs_src = nullptr;
    sp->abs_G = sp->abs_nchunks = 0;
    sp->win_P = nullptr;
    sp->win_P_bytes = 0;
    sp->ab_G = 0;
    sp->kh_ntiles = 0;
}

extern "C" {

const char* sqd_version(void) { return SQD_VERSION_STRING; }

int sqd_create(int device, void* hip_stream, sqd_ctx** out) {
    if (!out) return SQD_E_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return SQD_E_HIP;
    }
    if (device < 0 || device >= ndev) return SQD_E_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return SQD_E_HIP;
    sqd_ctx* ctx = new sqd_ctx();
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        ctx->num_cu = prop.multiProcessorCount;
        ctx->max_lds = (int)prop.sharedMemPerBlock;
    }
    int lds_optin = 0;
    if (hipDeviceGetAttribute(&lds_optin, hipDeviceAttributeSharedMemPerBlockOptin, device) == hipSuccess &&
        lds_optin > ctx->max_lds)
        ctx->max_lds = lds_optin;
    (void)hipGetLastError();
    // the no-allocation product's static scratch: its address on this device
    // (a failure surfaces as SQD_E_STATE from sqd_sigma_noalloc)
    (void)sqd_noalloc_init(device);
    *out = ctx;
    return SQD_OK;
}

void sqd_destroy(sqd_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    // spaces still open: release their device memory and orphan them, so that
    // a later sqd_space_free only deletes the host struct
    for (sqd_space* sp : ctx->spaces) {
        space_release_device(sp);
        sp->ctx = nullptr;
    }
    ctx->spaces.clear();
    free_ham(ctx);
    free_scratch(ctx);
    if (ctx->batch_arena) (void)hipFree(ctx->batch_arena);
    if (ctx->batch_count_host) (void)hipHostFree(ctx->batch_count_host);
    if (ctx->dav_arena) (void)hipFree(ctx->dav_arena);
    if (ctx->dav_state_host) (void)hipHostFree(ctx->dav_state_host);
    for (auto& r : ctx->prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : ctx->prof_pool) (void)hipEventDestroy(e);
    delete ctx;
}

const char* sqd_last_error(const sqd_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int sqd_synchronize(sqd_ctx* ctx) {
    if (!ctx) return SQD_E_INVALID_ARG;
    SQD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return SQD_OK;
}

int sqd_set_tuning(sqd_ctx* ctx, int key, int value) {
    if (!ctx) return SQD_E_INVALID_ARG;
    if (key < 0 || key >= SQD_TUNE_COUNT) return sqd_fail(ctx, SQD_E_INVALID_ARG, "unknown tuning key");
    static const int allowed[SQD_TUNE_COUNT][5] = {
        {0, 1, 2, 4, 8}, {0, 1, 2, 4, 8}, {0, 4, 8, 16, -1}, {0, 4, 8, 16, -1}, {0, 1, 2, -1, -1}, {0, 32, 64, -1, -1},
        {0, 1, 2, 3, -1}, {0, 1, 2, 4, 8}, {0, 1, 2, -1, -1}};
    bool ok = false;
    for (int v : allowed[key]) ok |= (v == value);
    // same-spin windows: also an explicit window width (a multiple of 64)
    if (key == SQD_TUNE_SS_WINDOW && value >= 64 && value <= 65536 && value % 64 == 0) ok = true;
    if (!ok) return sqd_fail(ctx, SQD_E_INVALID_ARG, "tuning value not allowed for key " + std::to_string(key));
    ctx->tune[key] = value;
    return SQD_OK;
}

int sqd_release_workspace(sqd_ctx* ctx) {
    if (!ctx) return SQD_E_INVALID_ARG;
    SQD_HIP(ctx, hipSetDevice(ctx->device));
    SQD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    free_scratch(ctx);
    if (ctx->batch_arena) (void)hipFree(ctx->batch_arena);
    if (ctx->dav_arena) (void)hipFree(ctx->dav_arena);
    ctx->batch_arena = nullptr;
    ctx->batch_arena_bytes = 0;
    ctx->dav_arena = nullptr;
    ctx->dav_arena_bytes = 0;
    return SQD_OK;
}

int sqd_profile(sqd_ctx* ctx, int enable) {
    if (!ctx) return SQD_E_INVALID_ARG;
    ctx->profiling = enable != 0;
    return SQD_OK;
}

int sqd_profile_report(sqd_ctx* ctx, char* buf, int len) {
    if (!ctx || !buf || len < 1) return SQD_E_INVALID_ARG;
    SQD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::vector<std::pair<std::string, std::pair<int, double>>> agg;
    for (auto& r : ctx->prof) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, r.a, r.b);
        bool found = false;
        for (auto& kv : agg)
            if (kv.first == r.name) {
                kv.second.first += 1;
                kv.second.second += ms;
                found = true;
                break;
            }
        if (!found) agg.push_back({r.name, {1, (double)ms}});
        ctx->prof_pool.push_back(r.a);
        ctx->prof_pool.push_back(r.b);
    }
    ctx->prof.clear();
    std::string out;
    for (auto& kv : agg)
        out += kv.first + " " + std::to_string(kv.second.first) + " " + std::to_string(kv.second.second) + "\n";
    std::strncpy(buf, out.c_str(), (size_t)len - 1);
    buf[len - 1] = 0;
    return SQD_OK;
}

int sqd_get_tuning(const sqd_ctx* ctx, int key, int* value) {
    if (!ctx || !value || key < 0 || key >= SQD_TUNE_COUNT) return SQD_E_INVALID_ARG;
    *value = ctx->tune[key];
    return SQD_OK;
}

int sqd_set_hamiltonian(sqd_ctx* ctx, int norb, const double* h, const double* eri, double ecore) {
    if (!ctx) return SQD_E_INVALID_ARG;
    if (norb < 1 || norb > SQD_MAXORB) return sqd_fail(ctx, SQD_E_NORB, "norb must be in [1, 128]");
    if (!h || !eri) return sqd_fail(ctx, SQD_E_INVALID_ARG, "null integral pointer");
    if (!std::isfinite(ecore)) return sqd_fail(ctx, SQD_E_INVALID_ARG, "ecore not finite");
    const int64_t n2 = (int64_t)norb * norb, n4 = n2 * n2;
    double mx = 0.0;
    for (int64_t k = 0; k < n2; ++k) {
        if (!std::isfinite(h[k])) return sqd_fail(ctx, SQD_E_INVALID_ARG, "h not finite");
        mx = std::max(mx, std::fabs(h[k]));
    }
    for (int64_t k = 0; k < n4; ++k) {
        if (!std::isfinite(eri[k])) return sqd_fail(ctx, SQD_E_INVALID_ARG, "eri not finite");
        mx = std::max(mx, std::fabs(eri[k]));
    }
    const double tol = 1e-12 * std::max(mx, 1e-300);
    for (int p = 0; p < norb; ++p)
        for (int q = 0; q < norb; ++q)
            if (std::fabs(h[p * norb + q] - h[q * norb + p]) > tol)
                return sqd_fail(ctx, SQD_E_ASYMMETRIC, "h is not symmetric");
    for (int p = 0; p < norb; ++p)
        for (int q = 0; q < norb; ++q)
            for (int r = 0; r < norb; ++r)
                for (int s = 0; s < norb; ++s) {
                    const double v = eri[((int64_t)(p * norb + q) * norb + r) * norb + s];
                    const double v1 = eri[((int64_t)(q * norb + p) * norb + r) * norb + s];
                    const double v2 = eri[((int64_t)(p * norb + q) * norb + s) * norb + r];
                    const double v3 = eri[((int64_t)(r * norb + s) * norb + p) * norb + q];
                    if (std::fabs(v - v1) > tol || std::fabs(v - v2) > tol || std::fabs(v - v3) > tol)
                        return sqd_fail(ctx, SQD_E_ASYMMETRIC, "(pq|rs) lacks the 8-fold symmetry");
                }
    SQD_HIP(ctx, hipSetDevice(ctx->device));
    SQD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    // from here until success the context holds no usable integrals: norb 0
    // makes every space fail its norb check (SQD_E_STATE) if a step fails
    if (ctx->norb != norb) free_ham(ctx);
    ctx->norb = 0;
    int rc;
    if (!ctx->h) {
        if ((rc = sqd_alloc(ctx, (void**)&ctx->h, sizeof(double) * n2, nullptr))) return rc;
        if ((rc = sqd_alloc(ctx, (void**)&ctx->eri, sizeof(double) * n4, nullptr))) return rc;
        if ((rc = sqd_alloc(ctx, (void**)&ctx->eri32, sizeof(float) * n4, nullptr))) return rc;
        if ((rc = sqd_alloc(ctx, (void**)&ctx->jk64, sizeof(double) * n2 * norb, nullptr))) return rc;
        if ((rc = sqd_alloc(ctx, (void**)&ctx->jk32, sizeof(float) * n2 * norb, nullptr))) return rc;
        if ((rc = sqd_alloc(ctx, (void**)&ctx->jdiag, sizeof(double) * n2, nullptr))) return rc;
    }
    SQD_HIP(ctx, hipMemcpy(ctx->h, h, sizeof(double) * n2, hipMemcpyHostToDevice));
    SQD_HIP(ctx, hipMemcpy(ctx->eri, eri, sizeof(double) * n4, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_jtables, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, ctx->stream, ctx->eri, norb,
                       ctx->jk64, ctx->jk32, ctx->jdiag, ctx->eri32);
    SQD_HIP(ctx, hipGetLastError());
    SQD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->h_host.assign(h, h + n2);
    ctx->eri_host.assign(eri, eri + n4);
    ctx->norb = norb;
    ctx->ecore = ecore;
    ctx->ham_version += 1;
    return SQD_OK;
}

// strings of nw words (word q: orbitals 64q .. 64q+63): no bit >= norb, nel
// bits set, strictly ascending as integers (word nw-1 most significant)
static int validate_strings(sqd_ctx* ctx, const uint64_t* s, int nw, int64_t n, int nel, int norb,
                            const char* which) {
    for (int64_t k = 0; k < n; ++k) {
        const uint64_t* x = s + k * nw;
        int pop = 0;
        for (int q = 0; q < nw; ++q) {
            const int lo = 64 * q;
            const uint64_t mask = (norb >= lo + 64) ? ~0ull : (norb <= lo ? 0ull : ((1ull << (norb - lo)) - 1));
            if (x[q] & ~mask)
                return sqd_fail(ctx, SQD_E_NORB, std::string(which) + " string has a bit >= norb at " + std::to_string(k));
            pop += __builtin_popcountll(x[q]);
        }
        if (pop != nel)
            return sqd_fail(ctx, SQD_E_POPCOUNT, std::string(which) + " string has the wrong electron count at " + std::to_string(k));
        if (k > 0) {
            const uint64_t* y = x - nw;
            int cmp = 0;
            for (int q = nw - 1; q >= 0 && cmp == 0; --q)
                if (x[q] != y[q]) cmp = x[q] > y[q] ? 1 : -1;
            if (cmp <= 0)
                return sqd_fail(ctx, SQD_E_UNSORTED, std::string(which) + " strings not strictly ascending at " + std::to_string(k));
        }
    }
    return SQD_OK;
}

static int build_space_impl(sqd_ctx* ctx, int nalpha, int nbeta, int nw, const uint64_t* astr, int64_t na,
                            const uint64_t* bstr, int64_t nb, sqd_space** out) {
    if (!ctx || !out) return SQD_E_INVALID_ARG;
    *out = nullptr;
    if (ctx->norb == 0) return sqd_fail(ctx, SQD_E_STATE, "call sqd_set_hamiltonian before sqd_build_space");
    const int norb = ctx->norb;
    if (nw < 1 || nw > 2) return sqd_fail(ctx, SQD_E_INVALID_ARG, "strings take 1 or 2 words");
    if (norb > 64 * nw)
        return sqd_fail(ctx, SQD_E_NORB, "norb > 64 needs two-word strings (sqd_build_space_words)");
    if (!astr || !bstr || na < 1 || nb < 1) return sqd_fail(ctx, SQD_E_INVALID_ARG, "empty or null string list");
    if (na > SQD_MAXN || nb > SQD_MAXN) return sqd_fail(ctx, SQD_E_LIMIT, "more than 131071 strings per spin");
    if ((double)na * (double)nb >= 1099511627776.0) return sqd_fail(ctx, SQD_E_LIMIT, "dimension >= 2^40");
    if (nalpha < 0 || nalpha > norb || nbeta < 0 || nbeta > norb)
        return sqd_fail(ctx, SQD_E_POPCOUNT, "electron count outside [0, norb]");
    int rc;
    if ((rc = validate_strings(ctx, astr, nw, na, nalpha, norb, "alpha"))) return rc;
    if ((rc = validate_strings(ctx, bstr, nw, nb, nbeta, norb, "beta"))) return rc;
    SQD_HIP(ctx, hipSetDevice(ctx->device));
    sqd_space* sp = new sqd_space();
    sp->ctx = ctx;
    sp->norb = norb;
    sp->nw = nw;
    sp->nalpha = nalpha;
    sp->nbeta = nbeta;
    sp->dim = na * nb;
    if ((rc = sqd_build_spin_tables(ctx, sp, 0, astr, na, nalpha))) {
        sqd_space_free(sp);
        return rc;
    }
    const bool same = (na == nb) && (nalpha == nbeta) && std::memcmp(astr, bstr, sizeof(uint64_t) * na * nw) == 0;
    if (same) {
        sp->sp[1] = sp->sp[0];
        sp->sp[1].alias = true;
    } else if ((rc = sqd_build_spin_tables(ctx, sp, 1, bstr, nb, nbeta))) {
        sqd_space_free(sp);
        return rc;
    }
    ctx->spaces.push_back(sp);
    if ((rc = sqd_build_values(ctx, sp)) || (rc = sqd_ensure_diag(ctx, sp))) {
        sqd_space_free(sp);
        return rc;
    }
    *out = sp;
    return SQD_OK;
}

int sqd_build_space(sqd_ctx* ctx, int nalpha, int nbeta, const uint64_t* astr, int64_t na, const uint64_t* bstr,
                    int64_t nb, sqd_space** out) {
    return build_space_impl(ctx, nalpha, nbeta, 1, astr, na, bstr, nb, out);
}

int sqd_build_space_words(sqd_ctx* ctx, int nalpha, int nbeta, int nwords, const uint64_t* astr, int64_t na,
                          const uint64_t* bstr, int64_t nb, sqd_space** out) {
    return build_space_impl(ctx, nalpha, nbeta, nwords, astr, na, bstr, nb, out);
}

void sqd_space_free(sqd_space* sp) {
    if (!sp) return;
    sqd_ctx* ctx = sp->ctx;
    if (ctx) {   // orphans (context destroyed) hold no device memory
        (void)hipSetDevice(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        space_release_device(sp);
        auto& v = ctx->spaces;
        v.erase(std::remove(v.begin(), v.end(), sp), v.end());
    }
    delete sp;
}

int sqd_space_info(const sqd_space* sp, sqd_space_info_t* out) {
    if (!sp || !out) return SQD_E_INVALID_ARG;
    if (!sp->ctx) return SQD_E_STATE;
    std::memset(out, 0, sizeof(*out));
    out->norb = sp->norb;
    out->nalpha = sp->nalpha;
    out->nbeta = sp->nbeta;
    out->na = sp->sp[0].n;
    out->nb = sp->sp[1].n;
    out->dim = sp->dim;
    for (int s = 0; s < 2; ++s) {
        out->nnz_single[s] = sp->sp[s].nnz_s;
        out->nnz_double[s] = sp->sp[s].nnz_d;
    }
    const int64_t na = out->na, nb = out->nb;
    out->conn_terms[0] = sp->dim;
    out->conn_terms[1] = (sp->sp[0].nnz_s + sp->sp[0].nnz_d) * nb;
    out->conn_terms[2] = (sp->sp[1].nnz_s + sp->sp[1].nnz_d) * na;
    out->conn_terms[3] = sp->sp[0].nnz_s * sp->sp[1].nnz_s;
    out->conn_per_sigma = out->conn_terms[0] + out->conn_terms[1] + out->conn_terms[2] + out->conn_terms[3];
    out->device_bytes = sp->bytes;
    out->kh_columns = sp->kh_cols;
    return SQD_OK;
}

int sqd_get_tables(const sqd_space* sp, int spin, int kind, int64_t* offsets, uint64_t* entries) {
    if (!sp || !offsets || (spin != 0 && spin != 1) || (kind != SQD_SINGLES && kind != SQD_DOUBLES))
        return SQD_E_INVALID_ARG;
    if (!sp->ctx) return SQD_E_STATE;
    sqd_ctx* ctx = sp->ctx;
    const spin_tables& t = sp->sp[spin];
    SQD_HIP(ctx, hipSetDevice(ctx->device));
    SQD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::vector<int> off(t.n + 1);
    SQD_HIP(ctx, hipMemcpy(off.data(), kind == SQD_SINGLES ? t.s_off : t.d_off, sizeof(int) * (t.n + 1),
                           hipMemcpyDeviceToHost));
    for (int64_t k = 0; k <= t.n; ++k) offsets[k] = off[k];
    const int64_t nnz = kind == SQD_SINGLES ? t.nnz_s : t.nnz_d;
    if (nnz > 0) {
        if (!entries) return sqd_fail(ctx, SQD_E_INVALID_ARG, "null entries pointer");
        SQD_HIP(ctx, hipMemcpy(entries, kind == SQD_SINGLES ? t.s_ent : t.d_ent, sizeof(uint64_t) * nnz,
                               hipMemcpyDeviceToHost));
    }
    return SQD_OK;
}

int sqd_diag(sqd_ctx* ctx, const sqd_space* spc, double* diag) {
    if (!ctx || !spc || !diag) return SQD_E_INVALID_ARG;
    sqd_space* sp = const_cast<sqd_space*>(spc);
    if (sp->ctx != ctx) return sqd_fail(ctx, SQD_E_INVALID_ARG, "space belongs to another context");
    if (ctx->norb != sp->norb) return sqd_fail(ctx, SQD_E_STATE, "integrals changed norb since the space was built");
    SQD_HIP(ctx, hipSetDevice(ctx->device));
    int rc = sqd_ensure_diag(ctx, sp);
    if (rc) return rc;
    SQD_HIP(ctx, hipMemcpyAsync(diag, sp->diag, sizeof(double) * sp->dim, hipMemcpyDeviceToDevice, ctx->stream));
    return SQD_OK;
}

int sqd_sigma(sqd_ctx* ctx, const sqd_space* spc, const double* c, double* sigma, int precision, unsigned mask,
              int ab_path) {
    if (!ctx || !spc || !c || !sigma) return SQD_E_INVALID_ARG;
    sqd_space* sp = const_cast<sqd_space*>(spc);
    if (sp->ctx != ctx) return sqd_fail(ctx, SQD_E_INVALID_ARG, "space belongs to another context");
    if (ctx->norb != sp->norb) return sqd_fail(ctx, SQD_E_STATE, "integrals changed norb since the space was built");
    if (precision != SQD_FP64 && precision != SQD_FP32) return sqd_fail(ctx, SQD_E_INVALID_ARG, "bad precision");
    if (mask == 0 || (mask & ~SQD_TERM_ALL)) return sqd_fail(ctx, SQD_E_INVALID_ARG, "bad terms mask");
    if (ab_path < SQD_AB_AUTO || ab_path > SQD_AB_KH) return sqd_fail(ctx, SQD_E_INVALID_ARG, "bad ab_path");
    if (c == sigma) return sqd_fail(ctx, SQD_E_INVALID_ARG, "c and sigma must be distinct buffers");
    SQD_HIP(ctx, hipSetDevice(ctx->device));
    if (sqd_capturing(ctx) && !sqd_sigma_prepared(ctx, sp, precision, mask, ab_path))
        return sqd_fail(ctx, SQD_E_STATE,
                        "sqd_sigma under stream capture needs an earlier identical eager call on this space");
    return sqd_sigma_impl(ctx, sp, c, sigma, precision, mask, ab_path, nullptr, nullptr);
}

void sqd_davidson_default_opts(sqd_davidson_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-8;
    o->max_iter = 200;
    o->m_max = 24;
    o->mode = SQD_DAV_FP64;
    o->switch_tol = 1e-4;
    o->ab_path = SQD_AB_AUTO;
    o->check_every = 4;
    o->product = SQD_PRODUCT_MATRIX_FREE;
}

static int check_opts(sqd_ctx* ctx, const sqd_davidson_opts* o) {
    if (!o) return sqd_fail(ctx, SQD_E_INVALID_ARG, "null options");
    if (!(o->tol > 0.0) || o->max_iter < 1 || o->m_max < 2 || o->m_max > SQD_MMAX || o->check_every < 1 ||
        (o->mode != SQD_DAV_FP64 && o->mode != SQD_DAV_MIXED) || o->ab_path < 0 || o->ab_path > 2 ||
        (o->mode == SQD_DAV_MIXED && !(o->switch_tol > 0.0)) ||
        (o->product != SQD_PRODUCT_MATRIX_FREE && o->product != SQD_PRODUCT_STORED))
        return sqd_fail(ctx, SQD_E_INVALID_ARG, "invalid Davidson options");
    if (o->product == SQD_PRODUCT_STORED && o->mode != SQD_DAV_FP64)
        return sqd_fail(ctx, SQD_E_INVALID_ARG, "the stored-H product is FP64 only");
    return SQD_OK;
}

int sqd_davidson(sqd_ctx* ctx, const sqd_space* spc, const sqd_davidson_opts* o, double* energy, double* vec,
                 sqd_report* rep) {
    if (!ctx || !spc || !energy || !vec) return SQD_E_INVALID_ARG;
    int rc = check_opts(ctx, o);
    if (rc) return rc;
    sqd_space* sp = const_cast<sqd_space*>(spc);
    if (sp->ctx != ctx) return sqd_fail(ctx, SQD_E_INVALID_ARG, "space belongs to another context");
    if (ctx->norb != sp->norb) return sqd_fail(ctx, SQD_E_STATE, "integrals changed norb since the space was built");
    if (o->product == SQD_PRODUCT_STORED && (!sp->h_val || sp->h_version != ctx->ham_version))
        return sqd_fail(ctx, SQD_E_STATE, "no current stored H on this space (call sqd_store_hamiltonian)");
    SQD_HIP(ctx, hipSetDevice(ctx->device));
    return sqd_davidson_impl(ctx, sp, o, energy, vec, rep, 1);
}

int sqd_davidson_roots(sqd_ctx* ctx, const sqd_space* spc, const sqd_davidson_opts* o, int nroots,
                       double* energies, double* vecs, sqd_report* reps) {
    if (!ctx || !spc || !energies || !vecs) return SQD_E_INVALID_ARG;
    if (nroots < 1 || nroots > SQD_MAXLOCK) return sqd_fail(ctx, SQD_E_INVALID_ARG, "nroots must be 1..SQD_MAXLOCK");
    int rc = check_opts(ctx, o);
    if (rc) return rc;
    sqd_space* sp = const_cast<sqd_space*>(spc);
    if (sp->ctx != ctx) return sqd_fail(ctx, SQD_E_INVALID_ARG, "space belongs to another context");
    if (ctx->norb != sp->norb) return sqd_fail(ctx, SQD_E_STATE, "integrals changed norb since the space was built");
    if ((int64_t)nroots > sp->dim) return sqd_fail(ctx, SQD_E_INVALID_ARG, "more roots than determinants");
    if (o->product == SQD_PRODUCT_STORED && (!sp->h_val || sp->h_version != ctx->ham_version))
        return sqd_fail(ctx, SQD_E_STATE, "no current stored H on this space (call sqd_store_hamiltonian)");
    SQD_HIP(ctx, hipSetDevice(ctx->device));
    return sqd_davidson_impl(ctx, sp, o, energies, vecs, reps, nroots);
}

int sqd_davidson_block(sqd_ctx* ctx, const sqd_space* spc, const sqd_davidson_opts* o, int nroots,
                       double* energies, double* vecs, sqd_report* reps) {
    if (!ctx || !spc || !energies || !vecs) return SQD_E_INVALID_ARG;
    if (nroots < 1 || nroots > SQD_MAXLOCK) return sqd_fail(ctx, SQD_E_INVALID_ARG, "nroots must be 1..SQD_MAXLOCK");
    int rc = check_opts(ctx, o);
    if (rc) return rc;
    if (o->m_max < 2 * nroots) return sqd_fail(ctx, SQD_E_INVALID_ARG, "block Davidson needs m_max >= 2 nroots");
    sqd_space* sp = const_cast<sqd_space*>(spc);
    if (sp->ctx != ctx) return sqd_fail(ctx, SQD_E_INVALID_ARG, "space belongs to another context");
    if (ctx->norb != sp->norb) return sqd_fail(ctx, SQD_E_STATE, "integrals changed norb since the space was built");
    if ((int64_t)nroots > sp->dim) return sqd_fail(ctx, SQD_E_INVALID_ARG, "more roots than determinants");
    if (o->product == SQD_PRODUCT_STORED && (!sp->h_val || sp->h_version != ctx->ham_version))
        return sqd_fail(ctx, SQD_E_STATE, "no current stored H on this space (call sqd_store_hamiltonian)");
    SQD_HIP(ctx, hipSetDevice(ctx->device));
    return sqd_davidson_block_impl(ctx, sp, o, nroots, energies, vecs, reps);
}

int sqd_davidson_batched(sqd_ctx* ctx, int nspace, const sqd_space* const* spaces, const sqd_davidson_opts* o,
                         double* energies, double* const* vecs, sqd_report* reps) {
    if (!ctx || nspace < 1 || !spaces || !energies || !vecs) return SQD_E_INVALID_ARG;
    int rc = check_opts(ctx, o);
    if (rc) return rc;
    if (o->product != SQD_PRODUCT_MATRIX_FREE)
        return sqd_fail(ctx, SQD_E_INVALID_ARG, "batched solves use the matrix-free product");
    std::vector<sqd_space*> sps(nspace);
    for (int b = 0; b < nspace; ++b) {
        if (!spaces[b] || !vecs[b]) return sqd_fail(ctx, SQD_E_INVALID_ARG, "null space or vector");
        sps[b] = const_cast<sqd_space*>(spaces[b]);
        if (sps[b]->ctx != ctx) return sqd_fail(ctx, SQD_E_INVALID_ARG, "space belongs to another context");
        if (sps[b]->norb != ctx->norb) return sqd_fail(ctx, SQD_E_STATE, "norb mismatch");
    }
    SQD_HIP(ctx, hipSetDevice(ctx->device));
    return sqd_davidson_batched_impl(ctx, nspace, sps.data(), o, energies, vecs, reps);
}

int sqd_rdm(sqd_ctx* ctx, const sqd_space* spc, const double* c, double* rdm1, double* rdm2) {
    if (!ctx || !spc || !c || !rdm1) return SQD_E_INVALID_ARG;
    sqd_space* sp = const_cast<sqd_space*>(spc);
    if (sp->ctx != ctx) return sqd_fail(ctx, SQD_E_INVALID_ARG, "space belongs to another context");
    if (ctx->norb != sp->norb) return sqd_fail(ctx, SQD_E_STATE, "integrals changed norb since the space was built");
    SQD_HIP(ctx, hipSetDevice(ctx->device));
    return sqd_rdm_impl(ctx, sp, c, rdm1, rdm2);
}

}  // extern "C"
