// Stored-H mode: H restricted to S evaluated once into CSR on the device and
// applied by a sparse matrix-vector product in every Davidson iteration (the
// second of the two methods of Sec. II: compute the matrix elements one time,
// keep them, and reuse them, trading memory for the recomputation the
// matrix-free product does).
//
// Row d = (ia, ib) lists, in this order: the diagonal, the alpha singles and
// alpha doubles of ia (columns ia' * nb + ib), the beta singles and beta
// doubles of ib (columns ia * nb + ib'), and the alpha x beta singles pairs
// (columns ia' * nb + ib').  Each in-set connection appears exactly once (a
// string pair at Hamming distance 2 is a single, at 4 a double), so the row
// length is 1 + A(ia) + B(ib) + sa(ia) sb(ib), with A = singles + doubles and
// s = singles of each spin, and the row pointer has a closed form in per-spin
// prefix sums.  Values come from the same per-string tables as the
// matrix-free kernels: same-spin singles add the cross-spin term
// sum_{k in other string} (pq|kk), alpha-beta pairs are s_a s_b (ai|bj).
//
// The product y = H x streams 12 bytes per stored element (int32 column and
// FP64 value) from HBM: a plain bandwidth-bound kernel, one wavefront per row.
#include <algorithm>

#include "sqd_internal.h"

namespace {

constexpr int kRowsPerBlock = 4;   // wavefronts (rows) per 256-thread workgroup

struct store_args {
    int64_t na, nb;
    const int* as_off; const uint32_t* as_pk; const double* as_val;
    const int* ad_off; const int* ad_nbr; const double* ad_val;
    const int* bs_off; const uint32_t* bs_pk; const double* bs_val;
    const int* bd_off; const int* bd_nbr; const double* bd_val;
    const uint64_t* astr; const uint64_t* bstr;
    int nw;                    // words per string
    const double* jk;          // jk[k * norb2 + pq] = (pq|kk)
    const double* V;           // (pq|rs) as a norb2 x norb2 matrix
    int norb;
    const double* diag;
    const int64_t* rp;
    int* col;
    double* val;
};

// sum over occupied k of the string (nw words), in increasing k, of (pq|kk)
__device__ __forceinline__ double cross_spin(const double* __restrict__ jk, int norb2, const uint64_t* s, int nw,
                                             int pair) {
    double w = 0.0;
    str_for_each(s, nw, [&](int k) { w += jk[(int64_t)k * norb2 + pair]; });
    return w;
}

// row pointer: rp[d] = RA[ia] + ib (1 + A(ia)) + PB[ib] + sa(ia) PSB[ib]
__global__ void k_store_rowptr(const int64_t* __restrict__ RA, const int64_t* __restrict__ PB,
                               const int64_t* __restrict__ PSB, const int* __restrict__ as_off,
                               const int* __restrict__ ad_off, int64_t na, int64_t nb, int64_t* __restrict__ rp) {
    const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t dim = na * nb;
    if (d > dim) return;
    if (d == dim) { rp[d] = RA[na]; return; }
    const int64_t ia = d / nb, ib = d - ia * nb;
    const int64_t sa = as_off[ia + 1] - as_off[ia];
    const int64_t A1 = 1 + sa + (ad_off[ia + 1] - ad_off[ia]);
    rp[d] = RA[ia] + ib * A1 + PB[ib] + sa * PSB[ib];
}

__global__ void __launch_bounds__(256) k_store_fill(store_args a) {
    const int lane = threadIdx.x & 63;
    const int norb2 = a.norb * a.norb;
    const int64_t dim = a.na * a.nb;
    for (int64_t d = (int64_t)blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6); d < dim;
         d += (int64_t)gridDim.x * kRowsPerBlock) {
        const int64_t ia = d / a.nb, ib = d - ia * a.nb;
        const int sa0 = a.as_off[ia], nsa = a.as_off[ia + 1] - sa0;
        const int da0 = a.ad_off[ia], nda = a.ad_off[ia + 1] - da0;
        const int sb0 = a.bs_off[ib], nsb = a.bs_off[ib + 1] - sb0;
        const int db0 = a.bd_off[ib], ndb = a.bd_off[ib + 1] - db0;
        const int64_t e1 = 1 + nsa, e2 = e1 + nda, e3 = e2 + nsb, e4 = e3 + ndb;
        const int64_t e5 = e4 + (int64_t)nsa * nsb;
        const int64_t base = a.rp[d];
        const uint64_t* sa_str = a.astr + ia * a.nw;
        const uint64_t* sb_str = a.bstr + ib * a.nw;
        for (int64_t e = lane; e < e5; e += 64) {
            int64_t c;
            double v;
            if (e == 0) {
                c = d;
                v = a.diag[d];
            } else if (e < e1) {            // alpha single: ia' <- ia, beta string fixed
                const int p = sa0 + (int)(e - 1);
                const uint32_t pk = a.as_pk[p];
                const int pair = (int)((pk >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK);
                const double w = cross_spin(a.jk, norb2, sb_str, a.nw, pair);
                v = a.as_val[p] + ((pk >> 31) ? -w : w);
                c = (int64_t)(pk & SQD_NBR_MASK) * a.nb + ib;
            } else if (e < e2) {            // alpha double
                const int p = da0 + (int)(e - e1);
                v = a.ad_val[p];
                c = (int64_t)a.ad_nbr[p] * a.nb + ib;
            } else if (e < e3) {            // beta single: ib' <- ib, alpha string fixed
                const int p = sb0 + (int)(e - e2);
                const uint32_t pk = a.bs_pk[p];
                const int pair = (int)((pk >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK);
                const double w = cross_spin(a.jk, norb2, sa_str, a.nw, pair);
                v = a.bs_val[p] + ((pk >> 31) ? -w : w);
                c = ia * a.nb + (int64_t)(pk & SQD_NBR_MASK);
            } else if (e < e4) {            // beta double
                const int p = db0 + (int)(e - e3);
                v = a.bd_val[p];
                c = ia * a.nb + a.bd_nbr[p];
            } else {                        // one alpha and one beta single
                const int k = (int)(e - e4);
                const int ka = k / nsb, kb = k - ka * nsb;
                const uint32_t pa = a.as_pk[sa0 + ka], pb = a.bs_pk[sb0 + kb];
                const int qa = (int)((pa >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK);
                const int qb = (int)((pb >> SQD_PAIR_SHIFT) & SQD_PAIR_MASK);
                v = a.V[(int64_t)qa * norb2 + qb];
                if ((pa ^ pb) >> 31) v = -v;
                c = (int64_t)(pa & SQD_NBR_MASK) * a.nb + (int64_t)(pb & SQD_NBR_MASK);
            }
            a.col[base + e] = (int)c;
            a.val[base + e] = v;
        }
    }
}

struct xcd_rows {
    int64_t r[9];
};

// y[r] = sum_k val[k] x[col[k]]: one wavefront per row, four 64-entry blocks
// of the row in flight per lane; the matrix stream is read non-temporally so
// that the cached lines of x stay resident.  The rows are cut into eight
// ranges of equal element counts, one per XCD (workgroup k runs on XCD k mod
// 8 and walks range k mod 8), so that the rows in flight on one XCD share
// their alpha string and the rows of x they gather from stay in that XCD's
// L2.
__global__ void __launch_bounds__(256) k_spmv(const int64_t* __restrict__ rp, const int* __restrict__ col,
                                              const double* __restrict__ val, const double* __restrict__ x,
                                              double* __restrict__ y, xcd_rows xr, const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63;
    const int xcd = (int)(blockIdx.x & 7);
    const int64_t j = blockIdx.x >> 3, nj = gridDim.x >> 3;
    const int64_t r0 = xr.r[xcd], r1 = xr.r[xcd + 1];
    for (int64_t r = r0 + j * kRowsPerBlock + (threadIdx.x >> 6); r < r1; r += nj * kRowsPerBlock) {
        const int64_t k1 = rp[r + 1];
        int64_t k = rp[r] + lane;
        double acc = 0.0;
        for (; k + 192 < k1; k += 256) {
            int c[4];
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                c[u] = __builtin_nontemporal_load(col + k + 64 * u);
                v[u] = __builtin_nontemporal_load(val + k + 64 * u);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) acc += v[u] * x[c[u]];
        }
        for (; k < k1; k += 64) acc += __builtin_nontemporal_load(val + k) * x[__builtin_nontemporal_load(col + k)];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) y[r] = acc;
    }
}

unsigned fill_grid(int64_t rows) {
    const int64_t b = (rows + kRowsPerBlock - 1) / kRowsPerBlock;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 1 << 16));
}

}  // namespace

void sqd_release_stored_h(sqd_space* sp) {
    void* ptrs[] = {sp->h_rowptr, sp->h_col, sp->h_val};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    sp->bytes -= sp->h_bytes;
    sp->h_rowptr = nullptr;
    sp->h_col = nullptr;
    sp->h_val = nullptr;
    sp->h_nnz = 0;
    sp->h_bytes = 0;
    sp->h_version = -1;
}

int sqd_store_h_impl(sqd_ctx* ctx, sqd_space* sp, int64_t* nnz_out) {
    int rc = sqd_ensure_diag(ctx, sp);
    if (rc) return rc;
    const spin_tables& A = sp->sp[0];
    const spin_tables& B = sp->sp[1];
    const int64_t na = A.n, nb = B.n, dim = sp->dim;
    if (dim >= 2147483647LL) return sqd_fail(ctx, SQD_E_LIMIT, "stored H needs dim < 2^31 (int32 columns)");
    // per-spin counts -> prefix sums of the closed-form row lengths
    std::vector<int> as(na + 1), ad(na + 1), bs(nb + 1), bd(nb + 1);
    SQD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    SQD_HIP(ctx, hipMemcpy(as.data(), A.s_off, sizeof(int) * (na + 1), hipMemcpyDeviceToHost));
    SQD_HIP(ctx, hipMemcpy(ad.data(), A.d_off, sizeof(int) * (na + 1), hipMemcpyDeviceToHost));
    SQD_HIP(ctx, hipMemcpy(bs.data(), B.s_off, sizeof(int) * (nb + 1), hipMemcpyDeviceToHost));
    SQD_HIP(ctx, hipMemcpy(bd.data(), B.d_off, sizeof(int) * (nb + 1), hipMemcpyDeviceToHost));
    std::vector<int64_t> PB(nb + 1), PSB(nb + 1), RA(na + 1);
    PB[0] = PSB[0] = 0;
    for (int64_t j = 0; j < nb; ++j) {
        PB[j + 1] = PB[j] + (bs[j + 1] - bs[j]) + (bd[j + 1] - bd[j]);
        PSB[j + 1] = PSB[j] + (bs[j + 1] - bs[j]);
    }
    RA[0] = 0;
    for (int64_t i = 0; i < na; ++i) {
        const int64_t sa = as[i + 1] - as[i], A1 = 1 + sa + (ad[i + 1] - ad[i]);
        RA[i + 1] = RA[i] + nb * A1 + PB[nb] + sa * PSB[nb];
    }
    const int64_t nnz = RA[na];
    // (re)allocate
    sqd_release_stored_h(sp);
    const size_t bytes = sizeof(int64_t) * (dim + 1) + (sizeof(int) + sizeof(double)) * (size_t)nnz;
    if ((rc = sqd_alloc(ctx, (void**)&sp->h_rowptr, sizeof(int64_t) * (dim + 1), nullptr)) ||
        (rc = sqd_alloc(ctx, (void**)&sp->h_col, sizeof(int) * (size_t)nnz, nullptr)) ||
        (rc = sqd_alloc(ctx, (void**)&sp->h_val, sizeof(double) * (size_t)nnz, nullptr))) {
        sqd_release_stored_h(sp);
        return sqd_fail(ctx, SQD_E_OOM, "stored H of " + std::to_string(nnz) + " elements (" +
                                            std::to_string(bytes) + " bytes) does not fit");
    }
    sp->h_bytes = (int64_t)bytes;
    sp->bytes += sp->h_bytes;
    int64_t *dRA = nullptr, *dPB = nullptr, *dPSB = nullptr;
    if ((rc = sqd_alloc(ctx, (void**)&dRA, sizeof(int64_t) * (na + 1), nullptr)) ||
        (rc = sqd_alloc(ctx, (void**)&dPB, sizeof(int64_t) * (nb + 1), nullptr)) ||
        (rc = sqd_alloc(ctx, (void**)&dPSB, sizeof(int64_t) * (nb + 1), nullptr))) {
        if (dRA) (void)hipFree(dRA);
        if (dPB) (void)hipFree(dPB);
        sqd_release_stored_h(sp);
        return rc;
    }
    hipError_t e = hipMemcpy(dRA, RA.data(), sizeof(int64_t) * (na + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dPB, PB.data(), sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dPSB, PSB.data(), sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_store_rowptr, dim3((unsigned)((dim + 256) / 256)), dim3(256), 0, ctx->stream, dRA, dPB,
                           dPSB, A.s_off, A.d_off, na, nb, sp->h_rowptr);
        store_args a{na, nb, A.s_off, A.s_pk, A.s_val64, A.d_off, A.d_nbr, A.d_val64,
                     B.s_off, B.s_pk, B.s_val64, B.d_off, B.d_nbr, B.d_val64,
                     A.str, B.str, sp->nw, ctx->jk64, ctx->eri, sp->norb, sp->diag, sp->h_rowptr, sp->h_col,
                     sp->h_val};
        hipLaunchKernelGGL(k_store_fill, dim3(fill_grid(dim)), dim3(256), 0, ctx->stream, a);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    }
    (void)hipFree(dRA);
    (void)hipFree(dPB);
    (void)hipFree(dPSB);
    if (e != hipSuccess) {
        sqd_release_stored_h(sp);
        return sqd_hip_fail(ctx, e, "stored H build");
    }
    sp->h_nnz = nnz;
    // row ranges of equal element counts for the eight XCDs (binary search
    // on the row pointer)
    sp->h_xcd_rows[0] = 0;
    sp->h_xcd_rows[8] = dim;
    for (int q = 1; q < 8; ++q) {
        const int64_t target = nnz * q / 8;
        int64_t lo = sp->h_xcd_rows[q - 1], hi = dim;   // first row whose start is >= target
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            int64_t v = 0;
            e = hipMemcpy(&v, sp->h_rowptr + mid, sizeof(int64_t), hipMemcpyDeviceToHost);
            if (e != hipSuccess) {
                sqd_release_stored_h(sp);
                return sqd_hip_fail(ctx, e, "stored H row ranges");
            }
            if (v < target) lo = mid + 1; else hi = mid;
        }
        sp->h_xcd_rows[q] = lo;
    }
    sp->h_version = ctx->ham_version;
    if (nnz_out) *nnz_out = nnz;
    return SQD_OK;
}

int sqd_spmv_impl(sqd_ctx* ctx, sqd_space* sp, const double* x, double* y, const int* skip) {
    if (!sp->h_val || sp->h_version != ctx->ham_version)
        return sqd_fail(ctx, SQD_E_STATE, "no current stored H on this space (call sqd_store_hamiltonian)");
    prof_scope ps(ctx, "k_spmv");
    // eight workgroups of four rows per CU, a multiple of the 8 XCDs
    const int64_t want = std::max<int64_t>(1, (sp->dim + kRowsPerBlock - 1) / kRowsPerBlock);
    const unsigned grid = (unsigned)(8 * std::max<int64_t>(1, std::min<int64_t>(ctx->num_cu, (want + 7) / 8)));
    xcd_rows xr;
    for (int q = 0; q < 9; ++q) xr.r[q] = sp->h_xcd_rows[q];
    hipLaunchKernelGGL(k_spmv, dim3(grid), dim3(256), 0, ctx->stream, sp->h_rowptr, sp->h_col, sp->h_val, x, y, xr,
                       skip);
    SQD_HIP(ctx, hipGetLastError());
    return SQD_OK;
}

extern "C" {

int sqd_store_hamiltonian(sqd_ctx* ctx, const sqd_space* spc, int64_t* nnz_out) {
    if (!ctx || !spc) return SQD_E_INVALID_ARG;
    sqd_space* sp = const_cast<sqd_space*>(spc);
    if (sp->ctx != ctx) return sqd_fail(ctx, SQD_E_INVALID_ARG, "space belongs to another context");
    if (ctx->norb != sp->norb) return sqd_fail(ctx, SQD_E_STATE, "integrals changed norb since the space was built");
    SQD_HIP(ctx, hipSetDevice(ctx->device));
    return sqd_store_h_impl(ctx, sp, nnz_out);
}

int sqd_release_hamiltonian(sqd_ctx* ctx, const sqd_space* spc) {
    if (!ctx || !spc) return SQD_E_INVALID_ARG;
    sqd_space* sp = const_cast<sqd_space*>(spc);
    if (sp->ctx != ctx) return sqd_fail(ctx, SQD_E_INVALID_ARG, "space belongs to another context");
    SQD_HIP(ctx, hipSetDevice(ctx->device));
    SQD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    sqd_release_stored_h(sp);
    return SQD_OK;
}

int sqd_spmv(sqd_ctx* ctx, const sqd_space* spc, const double* c, double* sigma) {
    if (!ctx || !spc || !c || !sigma) return SQD_E_INVALID_ARG;
    sqd_space* sp = const_cast<sqd_space*>(spc);
    if (sp->ctx != ctx) return sqd_fail(ctx, SQD_E_INVALID_ARG, "space belongs to another context");
    if (ctx->norb != sp->norb) return sqd_fail(ctx, SQD_E_STATE, "integrals changed norb since the space was built");
    if (c == sigma) return sqd_fail(ctx, SQD_E_INVALID_ARG, "c and sigma must be distinct buffers");
    SQD_HIP(ctx, hipSetDevice(ctx->device));
    return sqd_spmv_impl(ctx, sp, c, sigma, nullptr);
}

int sqd_get_stored_hamiltonian(const sqd_space* spc, int64_t* rowptr, int32_t* cols, double* vals) {
    if (!spc || !rowptr) return SQD_E_INVALID_ARG;
    sqd_space* sp = const_cast<sqd_space*>(spc);
    sqd_ctx* ctx = sp->ctx;
    if (!ctx) return SQD_E_STATE;
    if (!sp->h_val || sp->h_version != ctx->ham_version)
        return sqd_fail(ctx, SQD_E_STATE, "no current stored H on this space");
    SQD_HIP(ctx, hipSetDevice(ctx->device));
    SQD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    SQD_HIP(ctx, hipMemcpy(rowptr, sp->h_rowptr, sizeof(int64_t) * (sp->dim + 1), hipMemcpyDeviceToHost));
    if (sp->h_nnz > 0) {
        if (!cols || !vals) return sqd_fail(ctx, SQD_E_INVALID_ARG, "null column or value pointer");
        SQD_HIP(ctx, hipMemcpy(cols, sp->h_col, sizeof(int) * (size_t)sp->h_nnz, hipMemcpyDeviceToHost));
        SQD_HIP(ctx, hipMemcpy(vals, sp->h_val, sizeof(double) * (size_t)sp->h_nnz, hipMemcpyDeviceToHost));
    }
    return SQD_OK;
}

}  // extern "C"
