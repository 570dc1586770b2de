/*
 * libsqd -- MI355X (gfx950) hot path of sample-based quantum diagonalization.
 *
 * The library evaluates sigma = H c over the product space S = S_alpha x S_beta
 * of sampled alpha and beta occupation strings (Sec. I: configurations as
 * bit-strings; Sec. IV: the alpha x beta index space and the three task types
 * of the Slater-Condon rules), runs a Davidson eigensolver for the lowest root
 * entirely on the GPU (Sec. III names moving the whole Davidson iteration to
 * the device as the alternative to offloading only the product; Sec. VI lists
 * its steps), and forms reduced density matrices for energy gradients.
 *
 * Hamiltonian (real orbitals, chemists' notation; the paper names the
 * second-quantized Hamiltonian and the Slater-Condon rules, Sec. I-II):
 *   H = ecore + sum_pq h_pq E_pq + 1/2 sum_pqrs (pq|rs) sum_st a+_ps a+_rt a_st a_qs
 * Determinants: |Ia Ib> = prod_{p in Ia, asc} a+_pa prod_{q in Ib, asc} a+_qb |0>
 * (all alpha creators left of all beta creators).
 *
 * Conventions shared by every entry point:
 *  - a string is a uint64 with bit p set when orbital p is occupied
 *    (norb <= 64), or, for norb <= 128, two uint64 words, word q holding
 *    orbitals 64 q .. 64 q + 63 (sqd_build_space_words): the bit_length
 *    packing of Sec. IV-A, with up to 64 orbitals per word;
 *  - string lists are strictly ascending; the vector index of determinant
 *    (ia, ib) is d = ia * nb + ib (alpha-major, the ia-outer / ib-inner loop
 *    order of Sec. IV-A);
 *  - pointers named *_dev are device pointers on the context's device,
 *    owned by the caller; pointers named *_host are host pointers;
 *  - work is enqueued on the context's stream; calls return after enqueueing
 *    unless stated otherwise;
 *  - every call returns an int status: 0 = SQD_OK, > 0 = warning, < 0 = error.
 *    No exception crosses the ABI.  sqd_last_error() gives the message of the
 *    last failing call on a context.
 *  - a context is not thread-safe; distinct contexts may be used concurrently.
 */
#ifndef SQD_H
#define SQD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define SQD_OK 0
#define SQD_NOT_CONVERGED 1     /* warning: outputs hold the best Ritz pair   */
#define SQD_E_INVALID_ARG (-1)  /* null pointer, bad size or option           */
#define SQD_E_UNSORTED (-2)     /* string list not strictly ascending          */
#define SQD_E_POPCOUNT (-3)     /* a string has the wrong electron count       */
#define SQD_E_NORB (-4)         /* norb outside [1, 128], a bit >= norb, or
                                   norb > 64 with one-word strings           */
#define SQD_E_ASYMMETRIC (-5)   /* integrals lack the required symmetry        */
#define SQD_E_OOM (-6)          /* device allocation failed                    */
#define SQD_E_HIP (-7)          /* HIP runtime error                           */
#define SQD_E_STATE (-8)        /* call order violated (e.g. no Hamiltonian)   */
#define SQD_E_LIMIT (-9)        /* size beyond a documented library limit      */

/* ---- sigma term selection (Sec. IV: the three task types) -------------- */
#define SQD_TERM_DIAG 1u  /* H_II c_I                                        */
#define SQD_TERM_AA 2u    /* pairs differing only in the alpha string          */
#define SQD_TERM_BB 4u    /* pairs differing only in the beta string           */
#define SQD_TERM_AB 8u    /* one alpha and one beta excitation                 */
#define SQD_TERM_ALL 15u

/* arithmetic of the off-diagonal sigma terms */
#define SQD_FP64 0
#define SQD_FP32 1        /* FP32 storage and accumulation; the diagonal term
                             and the output stay FP64                          */

/* alpha-beta algorithm */
#define SQD_AB_AUTO 0
#define SQD_AB_DIRECT 1   /* LDS-staged gather over alpha x beta singles       */
#define SQD_AB_KH 2       /* Knowles-Handy: D build, MFMA GEMM with (pq|rs), gather */

/* Davidson precision modes */
#define SQD_DAV_FP64 0
#define SQD_DAV_MIXED 1   /* FP32 sigma (and an FP32 basis) until ||r|| < switch_tol, then FP64 refinement */

/* Davidson product (Sec. II: the two methods of the CPU code) */
#define SQD_PRODUCT_MATRIX_FREE 0   /* every H_IJ recomputed in each product (sqd_sigma)  */
#define SQD_PRODUCT_STORED 1        /* H computed once and reused (sqd_store_hamiltonian,
                                       sqd_spmv); FP64 only                                */

#define SQD_MMAX 32       /* largest Davidson subspace (m_max)                 */
#define SQD_MAXLOCK 8     /* most roots of one sqd_davidson_roots call         */
#define SQD_HIST 512      /* residual history kept in the report               */

/* table kinds for sqd_get_tables */
#define SQD_SINGLES 0
#define SQD_DOUBLES 1

/* tuning keys for sqd_set_tuning */
#define SQD_TUNE_SS_ROWS 0     /* rows staged per same-spin workgroup: 1,2,4,8 (0 = auto) */
#define SQD_TUNE_AB_CHUNK 1    /* alpha sources staged per alpha-beta pass: 1,2,4,8 (0 = auto) */
#define SQD_TUNE_AB_WAVES 2    /* waves per alpha-beta workgroup: 4, 8 or 16 (0 = auto) */
#define SQD_TUNE_SS_WAVES 3    /* waves per same-spin workgroup: 4, 8 or 16 (0 = auto) */
#define SQD_TUNE_AB_PATH 4     /* default alpha-beta path for SQD_AB_AUTO */
#define SQD_TUNE_KH_TILE 5     /* beta targets per KH tile: 32 or 64 (0 = auto) */
#define SQD_TUNE_AB_VARIANT 6  /* direct alpha-beta kernel: 1 grouped by alpha pair (with an
                                  intermediate of nnz_singles_alpha x nb values and a gather),
                                  2 staged per target row (no intermediate), 3 grouped by
                                  source string (the same intermediate; auto takes it where
                                  one FP64 source row is all a pair group can stage);
                                  0 = auto */
#define SQD_TUNE_AB_GROUP 7    /* alpha singles per grouped alpha-beta unit: 1,2,4,8 (0 = auto) */
#define SQD_TUNE_SS_WINDOW 8   /* same-spin term by windows of source strings (rows of C too
                                  long for four to fit in LDS): 0 auto, 1 never, 2 always,
                                  or a window width (multiple of 64, <= 65536; always) */
#define SQD_TUNE_COUNT 9

typedef struct sqd_ctx sqd_ctx;      /* opaque, library-owned */
typedef struct sqd_space sqd_space;  /* opaque, library-owned */

typedef struct {
    int norb, nalpha, nbeta;
    int64_t na, nb, dim;
    int64_t nnz_single[2];   /* [0] alpha, [1] beta: in-set single excitations  */
    int64_t nnz_double[2];   /* in-set double excitations                       */
    int64_t conn_per_sigma;  /* connected (I,J) pairs visited by one full sigma,
                                the diagonal included                           */
    int64_t conn_terms[4];   /* the same split as DIAG, AA, BB, AB              */
    int64_t device_bytes;    /* device memory held by the space                 */
    int64_t kh_columns;      /* Knowles-Handy GEMM size: sum over 64-target beta
                                tiles of targets x active pair columns (0 until
                                the KH path has run on the space); its GEMM does
                                2 x kh_columns x nnz_single[0] flops           */
} sqd_space_info_t;

typedef struct {
    double tol;                  /* stop when ||H x - theta x||_2 <= tol, ||x|| = 1 */
    int max_iter;                /* iterations (sigma products) cap              */
    int m_max;                   /* subspace size before collapse, 2..SQD_MMAX   */
    int mode;                    /* SQD_DAV_FP64 or SQD_DAV_MIXED                */
    double switch_tol;           /* mixed: leave FP32 sigma when ||r|| < switch_tol */
    int ab_path;                 /* SQD_AB_*                                      */
    const double* guess_noise_dev; /* optional (dim): start = e_argmin(H_II) + noise; when both this
                                      and guess_dev are NULL the library adds its own noise of norm
                                      about 1e-3 (SplitMix64 counter stream 0), so that the start is
                                      not confined to one spin-flip symmetry sector */
    const double* guess_dev;       /* optional (dim): explicit start vector; overrides */
    int check_every;             /* host polls the device convergence flag every k
                                    iterations (>= 1); iterations past convergence
                                    are skipped on the device                    */
    int product;                 /* SQD_PRODUCT_*: the stored H needs a current
                                    sqd_store_hamiltonian on the space and mode
                                    SQD_DAV_FP64; batched solves take MATRIX_FREE */
} sqd_davidson_opts;

typedef struct {
    int iterations;              /* Davidson iterations (one sigma each)          */
    int iterations_fp32;         /* of which with FP32 sigma                      */
    int switch_iter;             /* iteration at which FP64 refinement began (-1) */
    int converged;               /* 1 if ||r|| <= tol                             */
    int status;                  /* device end state: 1 converged, 2 stalled, 3 cap */
    int nhist;
    double energy;               /* lowest Ritz value (includes ecore)            */
    double residual;             /* final ||r||_2                                 */
    double seconds;              /* wall time of the solve, diagonal included     */
    double residual_history[SQD_HIST];
    double energy_history[SQD_HIST];
    int products;                /* products H v evaluated (the block solver adds
                                    up to one per unconverged root per iteration) */
} sqd_report;

/* ---- context ----------------------------------------------------------- */

/* Create a context on HIP device `device`; all work is enqueued on
 * `hip_stream` (a hipStream_t, or NULL for the default stream).  The stream
 * must outlive the context. */
int sqd_create(int device, void* hip_stream, sqd_ctx** out);
/* Synchronise the stream and free everything the context owns.  Spaces still
 * open on it lose their device memory and become orphans: any call on an
 * orphan returns SQD_E_STATE (or SQD_E_INVALID_ARG where a context is passed),
 * and sqd_space_free on it only frees its small host record.  HIP graphs
 * captured from calls on the context must not be replayed afterwards. */
void sqd_destroy(sqd_ctx* ctx);
/* Message of the last failing call on ctx (never NULL; empty if none). */
const char* sqd_last_error(const sqd_ctx* ctx);
/* Library version string. */
const char* sqd_version(void);
/* Block the host until all work enqueued by ctx has finished. */
int sqd_synchronize(sqd_ctx* ctx);
/* Set a tuning parameter (SQD_TUNE_*); value 0 restores the automatic choice. */
int sqd_set_tuning(sqd_ctx* ctx, int key, int value);
int sqd_get_tuning(const sqd_ctx* ctx, int key, int* value);
/* Free the device workspaces the context keeps between calls (the product
 * and Davidson scratch, and the batched solver's arena, which holds every
 * vector of every space of the last batch); the next call that needs them
 * allocates them again.  Synchronises the context's stream.  HIP graphs that
 * captured sqd_sigma on this context must not be replayed afterwards. */
int sqd_release_workspace(sqd_ctx* ctx);
/* Per-kernel timers: while enabled, the single-space calls record HIP events
 * on the context's stream around each kernel they launch (the batched solver,
 * which replays captured graphs, records none). */
int sqd_profile(sqd_ctx* ctx, int enable);
/* Synchronise, write one line per kernel name, "name calls total_ms\n", into
 * buf (NUL-terminated, truncated to len), and clear the records. */
int sqd_profile_report(sqd_ctx* ctx, char* buf, int len);

/* ---- Hamiltonian (Sec. II: integrals provided in an input file; Sec. V-A:
 * integrals held as raw arrays indexed by orbital pair) ------------------ */

/* Copy the integrals (host pointers) to the device.
 *   h   : norb*norb, row-major, h[p*norb+q] = h_pq
 *   eri : norb^4, (pq|rs) at ((p*norb+q)*norb+r)*norb+s
 * Checks h = h^T and (pq|rs) = (qp|rs) = (pq|sr) = (rs|pq) to
 * 1e-12 * max|value| (else SQD_E_ASYMMETRIC).  Spaces built on ctx pick up
 * new integrals at their next use; spaces built for another norb fail every
 * later call with SQD_E_STATE.  If the copy fails after the checks, the
 * context holds no integrals (as before the first call) and every space
 * fails with SQD_E_STATE until a call succeeds. */
int sqd_set_hamiltonian(sqd_ctx* ctx, int norb, const double* h_host,
                        const double* eri_host, double ecore);

/* ---- space: strings and excitation tables (Sec. IV-A configuration cache,
 * Sec. V-A flattened excitation lists) ---------------------------------- */

/* Validate the strings (strictly ascending, popcount == nalpha / nbeta, no bit
 * >= norb), upload them and build on the device the per-string single and
 * double excitation tables with fermionic signs.  astr_host / bstr_host are
 * host arrays of na / nb one-word strings (norb <= 64).  Requires
 * sqd_set_hamiltonian first (for norb).  Limits: na, nb <= 131071; na*nb <
 * 2^40.  The space is owned by the library; free it with sqd_space_free
 * before destroying ctx. */
int sqd_build_space(sqd_ctx* ctx, int nalpha, int nbeta,
                    const uint64_t* astr_host, int64_t na,
                    const uint64_t* bstr_host, int64_t nb, sqd_space** out);
/* The same for strings of nwords (1 or 2) uint64 words each, word q holding
 * orbitals 64 q .. 64 q + 63, string k at astr_host[k * nwords ..]; order is
 * that of the strings read as integers (word nwords - 1 most significant).
 * norb > 64 needs nwords = 2 (SQD_E_NORB otherwise).  Every later call works
 * on the space as on a one-word space; the products stage norb^2 integral
 * rows in LDS, so for norb near 128 the longest string lists that fit are
 * shorter (SQD_E_LIMIT names it). */
int sqd_build_space_words(sqd_ctx* ctx, int nalpha, int nbeta, int nwords,
                          const uint64_t* astr_host, int64_t na,
                          const uint64_t* bstr_host, int64_t nb, sqd_space** out);
/* Free a space: its device memory (synchronising the context's stream) and
 * its host record.  On an orphan (its context destroyed) only the host
 * record is freed.  NULL is a no-op. */
void sqd_space_free(sqd_space* space);
/* Sizes and table counts of a space (SQD_E_STATE on an orphan). */
int sqd_space_info(const sqd_space* space, sqd_space_info_t* out);

/* Copy one table to the host in canonical order: rows by source string,
 * entries by target index ascending.  spin 0 = alpha, 1 = beta; kind
 * SQD_SINGLES or SQD_DOUBLES.  offsets_host has n+1 int64 slots (CSR),
 * entries_host has nnz uint64 slots packed as (7-bit orbital fields)
 *   singles: target | i << 32 | a << 39 | negative << 63
 *   doubles: target | i << 32 | j << 39 | a << 46 | b << 53 | negative << 63
 * where i (< j) are annihilated in the source, a (< b) created, and the sign is
 * <target| a+_a a_i |source> or <target| a+_a a+_b a_j a_i |source>.
 * Synchronous. */
int sqd_get_tables(const sqd_space* space, int spin, int kind,
                   int64_t* offsets_host, uint64_t* entries_host);

/* ---- products ---------------------------------------------------------- */

/* diag_dev[d] = H_dd for every determinant (dim doubles): the diagonal of
 * the Hamiltonian restricted to S (Sec. II: every matrix element recomputed
 * from the integrals; here the zero-difference Slater-Condon case). */
int sqd_diag(sqd_ctx* ctx, const sqd_space* space, double* diag_dev);

/* sigma_dev = (selected terms of H) c_dev, both dim doubles, distinct buffers:
 * the matrix-free product of Sec. II (every H_IJ recomputed from the
 * integrals, nothing stored per determinant), split into the three task types
 * of Sec. IV (alpha-alpha, beta-beta, one alpha plus one beta excitation)
 * plus the diagonal.  precision SQD_FP64 or SQD_FP32 (off-diagonal terms in
 * FP32 with FP32 accumulation; the diagonal term and the result in FP64).
 * terms_mask is a non-zero OR of SQD_TERM_*.  ab_path selects the alpha-beta
 * algorithm.
 * The first call for a space and precision may allocate and synchronise (the
 * grouped alpha-beta schedule, the context's scratch); later identical calls
 * only enqueue kernels on the context's stream, so they can be captured in a
 * HIP graph.  Under capture the call allocates nothing: it returns
 * SQD_E_STATE unless an identical eager call came first.  The scratch is
 * shared by the graph and eager calls on the same context (do not run them
 * concurrently); eager calls that need a larger scratch later keep the
 * captured buffer alive until sqd_release_workspace or sqd_destroy, after
 * which the graph must not be replayed.  A later call that changes how the
 * space's alpha singles are grouped (another SQD_TUNE_AB_* setting, or a
 * batched solve that includes the space) rebuilds that schedule: graphs
 * captured on the space before must then not be replayed either. */
int sqd_sigma(sqd_ctx* ctx, const sqd_space* space, const double* c_dev,
              double* sigma_dev, int precision, unsigned terms_mask, int ab_path);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid the allocator): the
 * product of sqd_sigma with no allocation.  Its scratch (the transposed input
 * and output of the alpha-alpha term, and the FP32 copies of the FP32 path) is
 * a static device array of SQD_NOALLOC_SCRATCH_BYTES that every GPU the
 * library runs on holds until the process ends; the alpha-beta term uses the
 * row-staged kernel, which needs no intermediate.  Arguments as sqd_sigma
 * (ab_path fixed to that kernel).  Limits: dim <= SQD_NOALLOC_MAX_DIM, and a
 * source row of C plus one norb^2 integral row must fit in one workgroup's LDS
 * (as for SQD_TUNE_AB_VARIANT 2); beyond either SQD_E_LIMIT, before anything
 * is enqueued.  Where a same-spin term takes the windowed kernel (rows too
 * long to stage four whole in LDS), its tables are built by the space's first
 * sqd_sigma call with that term and precision; until then SQD_E_STATE, before
 * anything is enqueued.  After a Hamiltonian change the first call refreshes the
 * space's values in place (kernels and a synchronisation; under capture it
 * returns SQD_E_STATE instead).  All calls on one GPU share the array and it
 * keeps the last call's contents (every word the product reads is written by
 * the same call first): calls that overlap in time on one GPU -- on other
 * streams or contexts -- race, and must be serialised by the caller. */
#define SQD_NOALLOC_SCRATCH_BYTES (256ull << 20)
#define SQD_NOALLOC_MAX_DIM 16777152LL   /* (SQD_NOALLOC_SCRATCH_BYTES - 1024) / 16 */
int sqd_sigma_noalloc(sqd_ctx* ctx, const sqd_space* space, const double* c_dev, double* sigma_dev,
                      int precision, unsigned terms_mask);

/* ---- stored-H mode (Sec. II: the CPU code's second method, the Hamiltonian
 * matrix computed one time, stored, and reused in every Davidson iteration,
 * against the matrix-free product that saves memory by recomputing) ------ */

/* Evaluate H restricted to S once into CSR on the device and keep it with the
 * space (replacing an earlier one).  Row d = ia * nb + ib holds the diagonal
 * first, then the alpha singles and doubles of ia (columns ia' * nb + ib), the
 * beta singles and doubles of ib (columns ia * nb + ib'), then the alpha x
 * beta singles pairs (ia' * nb + ib', alpha-major); every in-set connection
 * once, values as the matrix-free product uses them.  Storage: 8 (dim + 1) +
 * 12 nnz bytes (int64 row pointer, int32 column, FP64 value), nnz =
 * sum over rows of 1 + A(ia) + B(ib) + sa(ia) sb(ib) (A, B: singles plus
 * doubles of each spin; sa, sb: singles), i.e. conn_per_sigma of
 * sqd_space_info.  nnz_out (optional host pointer) receives nnz.  Errors:
 * SQD_E_LIMIT (dim >= 2^31), SQD_E_OOM (does not fit; nothing is kept).
 * The stored H belongs to the Hamiltonian version it was built for: after
 * sqd_set_hamiltonian every use returns SQD_E_STATE until it is rebuilt.
 * Synchronous. */
int sqd_store_hamiltonian(sqd_ctx* ctx, const sqd_space* space, int64_t* nnz_out);
/* Free the stored H of a space (no-op if none).  Synchronises the stream. */
int sqd_release_hamiltonian(sqd_ctx* ctx, const sqd_space* space);
/* sigma_dev = H c_dev from the stored H (all terms, FP64; dim doubles each,
 * distinct caller-owned buffers): a sparse product bound by HBM bandwidth,
 * 12 bytes per stored element.  SQD_E_STATE without a current stored H.
 * Only enqueues work, so it can be captured in a HIP graph. */
int sqd_spmv(sqd_ctx* ctx, const sqd_space* space, const double* c_dev, double* sigma_dev);
/* Host copy of the stored H: rowptr_host (dim + 1), cols_host and vals_host
 * (nnz each).  Synchronous. */
int sqd_get_stored_hamiltonian(const sqd_space* space, int64_t* rowptr_host, int32_t* cols_host,
                               double* vals_host);

/* ---- eigensolver (Sec. I, Sec. VI: Davidson for the lowest eigenpair) --- */

/* Fill opts with the defaults: tol 1e-8, max_iter 200, m_max 24, FP64,
 * switch_tol 1e-4, AUTO path, no guess, check_every 4, matrix-free product. */
void sqd_davidson_default_opts(sqd_davidson_opts* opts);

/* Lowest eigenpair of H restricted to S.  energy_host receives the energy
 * (ecore included); vec_dev (dim doubles, caller-owned) the normalised
 * eigenvector with its largest-magnitude entry positive.  rep (optional)
 * receives the report.  Synchronous.  Returns SQD_NOT_CONVERGED (warning) if
 * the tolerance was not reached; the outputs then hold the last Ritz pair. */
int sqd_davidson(sqd_ctx* ctx, const sqd_space* space, const sqd_davidson_opts* opts,
                 double* energy_host, double* vec_dev, sqd_report* rep);

/* The nroots lowest eigenpairs (1 <= nroots <= SQD_MAXLOCK), one after another:
 * root j is the lowest root of the orthogonal complement of roots 0..j-1,
 * every basis vector of its solve being projected against them (locking;
 * classical Gram-Schmidt, repeated when it removes over half the norm).
 * energies_host[nroots]; vecs_dev (nroots x dim doubles, row j = root j,
 * caller-owned) normalised, largest-magnitude entry positive; reps[nroots]
 * optional.  Root accuracy: each solve stops at opts->tol; the locked roots
 * enter later solves with their residual error.  Synchronous.  Returns
 * SQD_NOT_CONVERGED if any root missed the tolerance. */
int sqd_davidson_roots(sqd_ctx* ctx, const sqd_space* space, const sqd_davidson_opts* opts, int nroots,
                       double* energies_host, double* vecs_dev, sqd_report* reps);

/* The nroots lowest eigenpairs (1 <= nroots <= SQD_MAXLOCK) together, by block
 * Davidson-Liu (Sec. I: the ground and low-lying states of the projected
 * Hamiltonian; Davidson's method extended to a block of vectors): one
 * subspace for all roots, one correction per unconverged root per iteration
 * (two classical Gram-Schmidt passes; kept when over 1e-6 of its norm
 * survives), restarts on the nroots current Ritz vectors when the next
 * corrections would exceed m_max (which must be >= 2 nroots).  Start: the
 * nroots lowest diagonal determinants plus noise of norm about 1e-3
 * (SplitMix64 counter streams 1..nroots).  Stops when every root's residual
 * is <= tol.  Mixed mode: FP32 off-diagonal products until the largest
 * residual drops below switch_tol (or the FP32 floor), then a restart on the
 * Ritz vectors with FP64 products.  opts->guess_dev and guess_noise_dev are
 * ignored.  energies_host[nroots] ascending; vecs_dev (nroots x dim doubles,
 * row j = root j, caller-owned) normalised, largest-magnitude entry
 * positive; reps[nroots] optional (shared iteration and product counts,
 * per-root residual and history).  The small projected eigenproblem, the
 * orthogonalisation and the residuals run on the device; the host reads the
 * Ritz values and residual norms once per iteration.  Synchronous.  Returns
 * SQD_NOT_CONVERGED if any root missed the tolerance. */
int sqd_davidson_block(sqd_ctx* ctx, const sqd_space* space, const sqd_davidson_opts* opts, int nroots,
                       double* energies_host, double* vecs_dev, sqd_report* reps);

/* Many independent spaces built on the same context (same integrals) solved
 * together, each for its lowest root (Sec. I: the sampling loop yields many
 * configuration sets; Sec. II/IV: the same matrix-free product per space;
 * Sec. VI: load imbalance across uneven task groups): one persistent launch per sigma term over a work queue of
 * (space, tile) units ordered longest-first, and the Davidson iteration of all
 * spaces captured once in a hipGraph and replayed.  energies_host[nspace],
 * vecs_dev[nspace] (each that space's dim), reps[nspace] optional.
 * Synchronous. */
int sqd_davidson_batched(sqd_ctx* ctx, int nspace, const sqd_space* const* spaces,
                         const sqd_davidson_opts* opts, double* energies_host,
                         double* const* vecs_dev, sqd_report* reps);

/* ---- reduced density matrices (Hellmann-Feynman gradients) ------------- */

/* For a normalised c_dev (dim doubles):
 *   rdm1_dev[p*n+q]           = sum_s <c| a+_ps a_qs |c>
 *   rdm2_dev[((p*n+q)*n+r)*n+s] = sum_st <c| a+_ps a+_rt a_st a_qs |c>
 * so that E = ecore + sum h.rdm1 + 1/2 sum (pq|rs) rdm2, dE/dh_pq = rdm1_pq and
 * dE/d(pq|rs) = rdm2_pqrs / 2 (per element).  rdm1_dev has norb^2 doubles,
 * rdm2_dev norb^4 (NULL skips it).  The alpha-beta part of rdm2 is a
 * D_alpha^T D_beta product over all determinants on FP64 MFMA. */
int sqd_rdm(sqd_ctx* ctx, const sqd_space* space, const double* c_dev,
            double* rdm1_dev, double* rdm2_dev);

#ifdef __cplusplus
}
#endif
#endif /* SQD_H */
