/*
 * CPU oracle for the SQD Hamiltonian -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this file's library.  The product path (libsqd) never does.
 *
 * What it computes (Sec. I: configurations as occupation bit-strings; Sec. II:
 * the matrix-free product with the Hamiltonian, each H_ij recomputed from the
 * integrals with a sign; Sec. IV: the alpha x beta product space):
 *
 *   H = Ecore + sum_{pq,s} h_pq a+_{ps} a_{qs}
 *             + 1/2 sum_{pqrs,s,t} (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs}
 *
 * (real orbitals, chemists' notation), written in spin-orbitals P = p (alpha) or norb + p (beta):
 *
 *   H = Ecore + sum_{PQ} h_PQ [sP==sQ] a+_P a_Q
 *             + 1/2 sum_{PQRS} (pq|rs) [sP==sQ][sR==sS] a+_P a+_R a_S a_Q .
 *
 * A determinant |I> is a_{P1}+ a_{P2}+ ... |0> with P1 < P2 < ..., i.e. all
 * alpha creators (ascending) to the left of all beta creators (ascending);
 * its bit pattern D has bit p set for occupied alpha orbital p and bit
 * norb + q for occupied beta orbital q (2 norb <= 256 bits, four 64-bit
 * words).  A string of norb <= 128 orbitals is given as nw = 1 or 2 64-bit
 * words, word w holding orbitals 64 w .. 64 w + 63.  A matrix element
 * <I| op |J> is obtained by applying the ladder operators of op to D_J one at
 * a time, right to left, each contributing (-1)^(number of occupied
 * spin-orbitals below it), and comparing the result with D_I.  Every H_IJ is
 * the sum of coefficient * <I|op|J> over exactly the operator strings that can
 * map J to I; no Slater-Condon closed form and no factorised alpha/beta table
 * is used, so the result is the plain definition of sigma = P H P c.
 *
 * The same enumeration accumulates the spin-summed reduced density matrices
 *   gamma_pq = sum_s <a+_{ps} a_{qs}>,
 *   Gamma_pqrs = sum_{s,t} <a+_{ps} a+_{rt} a_{st} a_{qs}>,
 * so that E = Ecore + sum h.gamma + 1/2 sum (pq|rs) Gamma.
 *
 * Pair classes (for per-term output): DIAG (I == J), AA (only the alpha
 * strings differ), BB (only the beta strings differ), AB (both differ).
 *
 * Neighbour search (a pre-filter only): for every alpha string the in-set
 * alpha strings at Hamming distance 2 or 4 are found by a brute-force scan;
 * likewise for beta.  A connected J must combine such neighbours (or the same
 * string) with at most two spin-orbital differences in total.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NWD 4   /* 64-bit words of a determinant bit pattern (2 norb <= 256) */
typedef struct { uint64_t w[NWD]; } u256;

#define OR_DIAG 1u
#define OR_AA 2u
#define OR_BB 4u
#define OR_AB 8u

typedef struct {
    int norb;
    int nw;               /* 64-bit words per string */
    int64_t na, nb;
    const uint64_t* astr;
    const uint64_t* bstr;
    const double* h;
    const double* eri;
    double ecore;
    /* neighbour lists: CSR, indices of strings at Hamming distance 2 or 4 */
    int64_t* aoff; int64_t* aidx;
    int64_t* boff; int64_t* bidx;
} prob_t;

static int bit_get(const u256* d, int k) { return (int)((d->w[k >> 6] >> (k & 63)) & 1u); }
static void bit_flip(u256* d, int k) { d->w[k >> 6] ^= 1ull << (k & 63); }
static int bits_equal(const u256* a, const u256* b) {
    for (int q = 0; q < NWD; ++q)
        if (a->w[q] != b->w[q]) return 0;
    return 1;
}

/* number of set bits below position k */
static int count_below(const u256* d, int k) {
    int c = 0;
    for (int q = 0; q < (k >> 6); ++q) c += __builtin_popcountll(d->w[q]);
    if (k & 63) c += __builtin_popcountll(d->w[k >> 6] & ((1ull << (k & 63)) - 1));
    return c;
}

/* apply a_k: returns 0 if the orbital is empty; updates *d and *sign */
static int op_annihilate(u256* d, int k, int* sign) {
    if (!bit_get(d, k)) return 0;
    if (count_below(d, k) & 1) *sign = -*sign;
    bit_flip(d, k);
    return 1;
}

/* apply a+_k: returns 0 if the orbital is already occupied */
static int op_create(u256* d, int k, int* sign) {
    if (bit_get(d, k)) return 0;
    if (count_below(d, k) & 1) *sign = -*sign;
    bit_flip(d, k);
    return 1;
}

/* <I| a+_P a_Q |J> */
static int me1(u256 I, u256 J, int P, int Q) {
    int s = 1;
    u256 d = J;
    if (!op_annihilate(&d, Q, &s)) return 0;
    if (!op_create(&d, P, &s)) return 0;
    return bits_equal(&d, &I) ? s : 0;
}

/* <I| a+_P a+_R a_S a_Q |J> : a_Q acts first, then a_S, a+_R, a+_P */
static int me2(u256 I, u256 J, int P, int Q, int R, int S) {
    int s = 1;
    u256 d = J;
    if (!op_annihilate(&d, Q, &s)) return 0;
    if (!op_annihilate(&d, S, &s)) return 0;
    if (!op_create(&d, R, &s)) return 0;
    if (!op_create(&d, P, &s)) return 0;
    return bits_equal(&d, &I) ? s : 0;
}

/* positions of the set bits of x, ascending; returns their count */
static int bits_of(u256 x, int* out) {
    int n = 0;
    for (int q = 0; q < NWD; ++q)
        for (uint64_t v = x.w[q]; v; v &= v - 1) out[n++] = 64 * q + __builtin_ctzll(v);
    return n;
}

/* Hamming distance of two strings of nw words */
static int str_dist(const uint64_t* a, const uint64_t* b, int nw) {
    int d = 0;
    for (int q = 0; q < nw; ++q) d += __builtin_popcountll(a[q] ^ b[q]);
    return d;
}

/* Visit every operator string that maps J to I.  For the one-body part the
 * visitor gets (P, Q, -1, -1, sign); for the two-body part (P, Q, R, S, sign).
 * The two-body strings a+_P a+_R a_S a_Q with result I must annihilate the
 * spin-orbitals of J not in I plus spectators, and create those of I not in J
 * plus the same spectators; all orderings are visited. */
typedef void (*visit_fn)(void* ctx, int P, int Q, int R, int S, int sign);

static void for_each_term(u256 I, u256 J, visit_fn fn, void* ctx) {
    u256 x, jn, in, both;
    int nd2 = 0;
    for (int q = 0; q < NWD; ++q) {
        x.w[q] = I.w[q] ^ J.w[q];
        jn.w[q] = J.w[q] & ~I.w[q];
        in.w[q] = I.w[q] & ~J.w[q];
        both.w[q] = I.w[q] & J.w[q];
        nd2 += __builtin_popcountll(x.w[q]);
    }
    if (nd2 > 4) return;
    int hole[2], part[2], com[64 * NWD];
    int nh = bits_of(jn, hole);   /* in J, not in I: annihilated */
    int np = bits_of(in, part);   /* in I, not in J: created */
    int nc = bits_of(both, com);
    if (nh != np) return;
    /* one-body */
    if (nh == 0) {
        for (int k = 0; k < nc; ++k) {
            int s = me1(I, J, com[k], com[k]);
            if (s) fn(ctx, com[k], com[k], -1, -1, s);
        }
    } else if (nh == 1) {
        int s = me1(I, J, part[0], hole[0]);
        if (s) fn(ctx, part[0], hole[0], -1, -1, s);
    }
    /* two-body: choose the annihilated pair {Q,S} and created pair {P,R} */
    if (nh == 2) {
        int qs[2][2] = {{hole[0], hole[1]}, {hole[1], hole[0]}};
        int pr[2][2] = {{part[0], part[1]}, {part[1], part[0]}};
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                int P = pr[b][0], R = pr[b][1], Q = qs[a][0], S = qs[a][1];
                int s = me2(I, J, P, Q, R, S);
                if (s) fn(ctx, P, Q, R, S, s);
            }
    } else if (nh == 1) {
        for (int k = 0; k < nc; ++k) {
            int sp = com[k];
            int qs[2][2] = {{hole[0], sp}, {sp, hole[0]}};
            int pr[2][2] = {{part[0], sp}, {sp, part[0]}};
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    int P = pr[b][0], R = pr[b][1], Q = qs[a][0], S = qs[a][1];
                    int s = me2(I, J, P, Q, R, S);
                    if (s) fn(ctx, P, Q, R, S, s);
                }
        }
    } else if (nh == 0) {
        for (int k = 0; k < nc; ++k)
            for (int l = 0; l < nc; ++l) {
                if (k == l) continue;
                int Q = com[k], S = com[l];
                /* created pair must be {Q,S} again, both orders */
                int s1 = me2(I, J, Q, Q, S, S);
                if (s1) fn(ctx, Q, Q, S, S, s1);
                int s2 = me2(I, J, S, Q, Q, S);
                if (s2) fn(ctx, S, Q, Q, S, s2);
            }
    }
}

typedef struct { const prob_t* pb; double acc; } hctx_t;

static void hvisit(void* vctx, int P, int Q, int R, int S, int sign) {
    hctx_t* c = (hctx_t*)vctx;
    int n = c->pb->norb;
    int sP = P >= n, sQ = Q >= n;
    int p = P % n, q = Q % n;
    if (R < 0) {
        if (sP == sQ) c->acc += sign * c->pb->h[p * n + q];
        return;
    }
    int sR = R >= n, sS = S >= n;
    int r = R % n, s = S % n;
    if (sP == sQ && sR == sS)
        c->acc += 0.5 * sign * c->pb->eri[((size_t)(p * n + q) * n + r) * n + s];
}

/* D: bit p for alpha orbital p, bit norb + q for beta orbital q */
static u256 det_bits(const prob_t* pb, int64_t ia, int64_t ib) {
    u256 d;
    memset(&d, 0, sizeof(d));
    const uint64_t* a = pb->astr + ia * pb->nw;
    const uint64_t* b = pb->bstr + ib * pb->nw;
    for (int p = 0; p < pb->norb; ++p) {
        if ((a[p >> 6] >> (p & 63)) & 1u) bit_flip(&d, p);
        if ((b[p >> 6] >> (p & 63)) & 1u) bit_flip(&d, pb->norb + p);
    }
    return d;
}

static double h_elem(const prob_t* pb, int64_t ia, int64_t ib, int64_t ja, int64_t jb) {
    hctx_t c = {pb, 0.0};
    u256 I = det_bits(pb, ia, ib), J = det_bits(pb, ja, jb);
    for_each_term(I, J, hvisit, &c);
    if (bits_equal(&I, &J)) c.acc += pb->ecore;
    return c.acc;
}

/* brute-force neighbour lists: strings at Hamming distance 2 or 4 */
static void build_nbrs(const uint64_t* s, int64_t n, int nw, int64_t** off_out, int64_t** idx_out) {
    int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
    off[0] = 0;
    int64_t* cnt = (int64_t*)calloc(n, sizeof(int64_t));
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j) {
            int d = str_dist(s + i * nw, s + j * nw, nw);
            if (d == 2 || d == 4) ++c;
        }
        cnt[i] = c;
    }
    for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + cnt[i];
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (off[n] > 0 ? off[n] : 1));
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = off[i];
        for (int64_t j = 0; j < n; ++j) {
            int d = str_dist(s + i * nw, s + j * nw, nw);
            if (d == 2 || d == 4) idx[c++] = j;
        }
    }
    free(cnt);
    *off_out = off; *idx_out = idx;
}

static void prob_init(prob_t* pb, int norb, int nw, const uint64_t* astr, int64_t na,
                      const uint64_t* bstr, int64_t nb, const double* h, const double* eri,
                      double ecore) {
    pb->norb = norb; pb->nw = nw; pb->na = na; pb->nb = nb; pb->astr = astr; pb->bstr = bstr;
    pb->h = h; pb->eri = eri; pb->ecore = ecore;
    build_nbrs(astr, na, nw, &pb->aoff, &pb->aidx);
    build_nbrs(bstr, nb, nw, &pb->boff, &pb->bidx);
}

/* the string word count norb needs, or 0 when norb is outside [1, 128] */
static int words_for(int norb, int nw) {
    if (norb < 1 || norb > 128 || nw < 1 || nw > 2 || norb > 64 * nw) return 0;
    return nw;
}

static void prob_free(prob_t* pb) {
    free(pb->aoff); free(pb->aidx); free(pb->boff); free(pb->bidx);
}

/* Visit every (J, class) connected to row I = (ia, ib). */
typedef void (*pair_fn)(void* ctx, int64_t ja, int64_t jb, unsigned cls);

static void for_each_neighbour(const prob_t* pb, int64_t ia, int64_t ib, pair_fn fn, void* ctx) {
    fn(ctx, ia, ib, OR_DIAG);
    for (int64_t k = pb->aoff[ia]; k < pb->aoff[ia + 1]; ++k)
        fn(ctx, pb->aidx[k], ib, OR_AA);
    for (int64_t k = pb->boff[ib]; k < pb->boff[ib + 1]; ++k)
        fn(ctx, ia, pb->bidx[k], OR_BB);
    for (int64_t k = pb->aoff[ia]; k < pb->aoff[ia + 1]; ++k) {
        int64_t ja = pb->aidx[k];
        if (str_dist(pb->astr + ia * pb->nw, pb->astr + ja * pb->nw, pb->nw) != 2) continue;
        for (int64_t l = pb->boff[ib]; l < pb->boff[ib + 1]; ++l) {
            int64_t jb = pb->bidx[l];
            if (str_dist(pb->bstr + ib * pb->nw, pb->bstr + jb * pb->nw, pb->nw) != 2) continue;
            fn(ctx, ja, jb, OR_AB);
        }
    }
}

typedef struct {
    const prob_t* pb; int64_t ia, ib; const double* c; unsigned mask; double acc;
} sctx_t;

static void sigma_visit(void* vctx, int64_t ja, int64_t jb, unsigned cls) {
    sctx_t* s = (sctx_t*)vctx;
    if (!(s->mask & cls)) return;
    double hij = h_elem(s->pb, s->ia, s->ib, ja, jb);
    s->acc += hij * s->c[ja * s->pb->nb + jb];
}

static double sigma_row(const prob_t* pb, int64_t row, const double* c, unsigned mask) {
    sctx_t s = {pb, row / pb->nb, row % pb->nb, c, mask, 0.0};
    for_each_neighbour(pb, s.ia, s.ib, sigma_visit, &s);
    return s.acc;
}

/* ---------------------------------------------------------------- exports */

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* sigma = (P H P c) restricted to the pair classes in mask; all rows. */
int oracle_sigma(int norb, int nw, const uint64_t* astr, int64_t na, const uint64_t* bstr, int64_t nb,
                 const double* h, const double* eri, double ecore,
                 const double* c, double* sigma, unsigned mask) {
    if (!words_for(norb, nw)) return -1;
    prob_t pb;
    prob_init(&pb, norb, nw, astr, na, bstr, nb, h, eri, ecore);
    int64_t dim = na * nb;
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < dim; ++r) sigma[r] = sigma_row(&pb, r, c, mask);
    prob_free(&pb);
    return 0;
}

/* sigma at selected rows only: out[k] = sigma[rows[k]] */
int oracle_sigma_rows(int norb, int nw, const uint64_t* astr, int64_t na, const uint64_t* bstr, int64_t nb,
                      const double* h, const double* eri, double ecore,
                      const double* c, const int64_t* rows, int64_t nrows, double* out,
                      unsigned mask) {
    if (!words_for(norb, nw)) return -1;
    prob_t pb;
    prob_init(&pb, norb, nw, astr, na, bstr, nb, h, eri, ecore);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nrows; ++k) out[k] = sigma_row(&pb, rows[k], c, mask);
    prob_free(&pb);
    return 0;
}

/* diagonal H_II for all rows */
int oracle_diag(int norb, int nw, const uint64_t* astr, int64_t na, const uint64_t* bstr, int64_t nb,
                const double* h, const double* eri, double ecore, double* diag) {
    if (!words_for(norb, nw)) return -1;
    prob_t pb;
    pb.norb = norb; pb.nw = nw; pb.na = na; pb.nb = nb; pb.astr = astr; pb.bstr = bstr;
    pb.h = h; pb.eri = eri; pb.ecore = ecore;
    int64_t dim = na * nb;
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < dim; ++r) diag[r] = h_elem(&pb, r / nb, r % nb, r / nb, r % nb);
    return 0;
}

typedef struct { const prob_t* pb; int64_t ia, ib; double* H; int64_t dim; } dctx_t;

static void dense_visit(void* vctx, int64_t ja, int64_t jb, unsigned cls) {
    (void)cls;
    dctx_t* d = (dctx_t*)vctx;
    int64_t row = d->ia * d->pb->nb + d->ib, col = ja * d->pb->nb + jb;
    d->H[row * d->dim + col] = h_elem(d->pb, d->ia, d->ib, ja, jb);
}

/* dense H_S (dim x dim, row-major); the caller zero-fills H */
int oracle_dense(int norb, int nw, const uint64_t* astr, int64_t na, const uint64_t* bstr, int64_t nb,
                 const double* h, const double* eri, double ecore, double* H) {
    if (!words_for(norb, nw)) return -1;
    prob_t pb;
    prob_init(&pb, norb, nw, astr, na, bstr, nb, h, eri, ecore);
    int64_t dim = na * nb;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < dim; ++r) {
        dctx_t d = {&pb, r / nb, r % nb, H, dim};
        for_each_neighbour(&pb, d.ia, d.ib, dense_visit, &d);
    }
    prob_free(&pb);
    return 0;
}

/* ------------------------------------------------------------------ RDMs */

typedef struct { int norb; double w; double* g1; double* g2; } rctx_t;

static void rdm_visit(void* vctx, int P, int Q, int R, int S, int sign) {
    rctx_t* c = (rctx_t*)vctx;
    int n = c->norb;
    int sP = P >= n, sQ = Q >= n;
    int p = P % n, q = Q % n;
    if (R < 0) {
        if (sP == sQ) c->g1[p * n + q] += c->w * sign;
        return;
    }
    int sR = R >= n, sS = S >= n;
    int r = R % n, s = S % n;
    if (sP == sQ && sR == sS)
        c->g2[((size_t)(p * n + q) * n + r) * n + s] += c->w * sign;
}

typedef struct { const prob_t* pb; int64_t ia, ib; const double* c; rctx_t* r; } rpctx_t;

static void rdm_pair_visit(void* vctx, int64_t ja, int64_t jb, unsigned cls) {
    (void)cls;
    rpctx_t* d = (rpctx_t*)vctx;
    const prob_t* pb = d->pb;
    double ci = d->c[d->ia * pb->nb + d->ib], cj = d->c[ja * pb->nb + jb];
    d->r->w = ci * cj;
    if (d->r->w == 0.0) return;
    u256 I = det_bits(pb, d->ia, d->ib), J = det_bits(pb, ja, jb);
    for_each_term(I, J, rdm_visit, d->r);
}

/* 1-RDM (norb^2) and 2-RDM (norb^4), spin-summed, for a normalised c:
 * rdm1[p,q] = sum_s <a+_ps a_qs>, rdm2[p,q,r,s] = sum_st <a+_ps a+_rt a_st a_qs>. */
int oracle_rdm(int norb, int nw, const uint64_t* astr, int64_t na, const uint64_t* bstr, int64_t nb,
               const double* c, double* rdm1, double* rdm2) {
    if (!words_for(norb, nw)) return -1;
    prob_t pb;
    prob_init(&pb, norb, nw, astr, na, bstr, nb, NULL, NULL, 0.0);
    int64_t dim = na * nb;
    size_t n2 = (size_t)norb * norb, n4 = n2 * n2;
    memset(rdm1, 0, sizeof(double) * n2);
    memset(rdm2, 0, sizeof(double) * n4);
    #pragma omp parallel
    {
        double* g1 = (double*)calloc(n2, sizeof(double));
        double* g2 = (double*)calloc(n4, sizeof(double));
        rctx_t rc = {norb, 0.0, g1, g2};
        #pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < dim; ++r) {
            rpctx_t d = {&pb, r / nb, r % nb, c, &rc};
            for_each_neighbour(&pb, d.ia, d.ib, rdm_pair_visit, &d);
        }
        #pragma omp critical
        {
            for (size_t k = 0; k < n2; ++k) rdm1[k] += g1[k];
            for (size_t k = 0; k < n4; ++k) rdm2[k] += g2[k];
        }
        free(g1); free(g2);
    }
    prob_free(&pb);
    return 0;
}

/* single matrix element, for spot checks */
double oracle_h_elem(int norb, int nw, const uint64_t* astr, int64_t na, const uint64_t* bstr, int64_t nb,
                     const double* h, const double* eri, double ecore,
                     int64_t ia, int64_t ib, int64_t ja, int64_t jb) {
    prob_t pb;
    pb.norb = norb; pb.nw = nw; pb.na = na; pb.nb = nb; pb.astr = astr; pb.bstr = bstr;
    pb.h = h; pb.eri = eri; pb.ecore = ecore;
    return h_elem(&pb, ia, ib, ja, jb);
}

/* ----------------------------------------------------------- memoised H
 * The same elements, evaluated once into CSR (rows I, every visited J, the
 * diagonal first), so that a Davidson run on a large space pays the
 * definition-based evaluation only once.  Pass 1 counts (rowptr), pass 2 fills. */

typedef struct { const prob_t* pb; int64_t n; } cctx_t;
static void count_visit(void* vctx, int64_t ja, int64_t jb, unsigned cls) {
    (void)ja; (void)jb; (void)cls;
    ((cctx_t*)vctx)->n += 1;
}

int oracle_csr_count(int norb, int nw, const uint64_t* astr, int64_t na, const uint64_t* bstr, int64_t nb,
                     int64_t* rowptr) {
    if (!words_for(norb, nw)) return -1;
    prob_t pb;
    prob_init(&pb, norb, nw, astr, na, bstr, nb, NULL, NULL, 0.0);
    int64_t dim = na * nb;
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t r = 0; r < dim; ++r) {
        cctx_t c = {&pb, 0};
        for_each_neighbour(&pb, r / nb, r % nb, count_visit, &c);
        rowptr[r + 1] = c.n;
    }
    rowptr[0] = 0;
    for (int64_t r = 0; r < dim; ++r) rowptr[r + 1] += rowptr[r];
    prob_free(&pb);
    return 0;
}

typedef struct { const prob_t* pb; int64_t ia, ib, pos; int32_t* cols; double* vals; } fctx_t;
static void fill_visit(void* vctx, int64_t ja, int64_t jb, unsigned cls) {
    (void)cls;
    fctx_t* f = (fctx_t*)vctx;
    f->cols[f->pos] = (int32_t)(ja * f->pb->nb + jb);
    f->vals[f->pos] = h_elem(f->pb, f->ia, f->ib, ja, jb);
    f->pos += 1;
}

int oracle_csr_fill(int norb, int nw, const uint64_t* astr, int64_t na, const uint64_t* bstr, int64_t nb,
                    const double* h, const double* eri, double ecore,
                    const int64_t* rowptr, int32_t* cols, double* vals) {
    if (!words_for(norb, nw)) return -1;
    if (na * nb >= 2147483647LL) return -2;
    prob_t pb;
    prob_init(&pb, norb, nw, astr, na, bstr, nb, h, eri, ecore);
    int64_t dim = na * nb;
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t r = 0; r < dim; ++r) {
        fctx_t f = {&pb, r / nb, r % nb, rowptr[r], cols, vals};
        for_each_neighbour(&pb, f.ia, f.ib, fill_visit, &f);
    }
    prob_free(&pb);
    return 0;
}

/* y = H x with the memoised rows */
int oracle_csr_matvec(int64_t dim, const int64_t* rowptr, const int32_t* cols, const double* vals,
                      const double* x, double* y) {
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t r = 0; r < dim; ++r) {
        double acc = 0.0;
        for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k) acc += vals[k] * x[cols[k]];
        y[r] = acc;
    }
    return 0;
}
