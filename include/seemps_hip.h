/*
 * seemps_hip.h -- C ABI of the MI355X (gfx950) library for applying a matrix
 * product operator (MPO) to a matrix product state (MPS) and compressing the
 * result with the two-site variational sweep.
 *
 * Paper: "SeeMPS" (arXiv 2601.16734).  Each entry point names the passage
 * that defines its operation.
 *
 * Conventions shared by every call
 *   - Tensors are real.  An MPS site tensor is A[k][chi_l][d][chi_r] and an MPO
 *     site tensor is B[k][D_l][d_out][d_in][D_r], both dense C order, with open
 *     ends (first and last bond dimension 1)  (Sec. 2.1, Sec. 2.2).
 *   - Handles are opaque.  The caller owns every handle it receives and frees
 *     it with the matching *_destroy call; the library owns the device memory
 *     behind a handle.  Host pointers passed in are read during the call and
 *     never retained.  Inputs are never modified.
 *   - Every call returns an smps_status.  On failure nothing is written to
 *     *out (it is set to NULL where it is a handle) and smps_last_error(ctx)
 *     returns a message.  Nothing throws across this boundary.
 *   - All device work is ordered on the stream given to smps_ctx_create.
 *     Calls that return host values (scalars, shapes, reads) synchronise
 *     that stream before returning.
 *   - One context must not be used from two host threads at once.
 *   - Handles are checked on entry: NULL, a destroyed handle (or a pointer the
 *     library never returned) and a handle of another context are refused
 *     with SMPS_EINVAL, and destroying such a pointer returns SMPS_EINVAL.
 *     (A new handle can reuse a destroyed one's address; the check cannot
 *     tell those apart.)  Destroying a context destroys the handles it still
 *     owns.
 */
#ifndef SEEMPS_HIP_H
#define SEEMPS_HIP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct smps_ctx smps_ctx;
typedef struct smps_mps smps_mps;
typedef struct smps_mpo smps_mpo;

typedef enum {
    SMPS_OK = 0,
    SMPS_EINVAL = -1,       /* bad argument: shapes do not chain, NULL handle, bad strategy */
    SMPS_ENOMEM = -2,       /* device allocation failed or a workspace limit was exceeded */
    SMPS_EHIP = -3,         /* a HIP runtime call failed */
    SMPS_ENUMERIC = -4,     /* non-finite values met in a factorization */
    SMPS_EUNSUPPORTED = -5, /* valid request the library does not handle */
    SMPS_ENODEV = -6        /* the call needs a device and the context is a planning context */
} smps_status;

/* storage type of host data handed to *_create */
enum { SMPS_F64 = 0, SMPS_F32 = 1 };

/* arithmetic of the contractions; factorizations, discarded-weight sums and
   norms are always FP64 */
enum {
    SMPS_PREC_FP64 = 0,    /* FP64 MFMA, FP64 accumulation */
    SMPS_PREC_FP32 = 1,    /* FP32 MFMA, FP32 accumulation */
    SMPS_PREC_BF16X3 = 2,  /* x = hi + lo in bf16, product hi*hi + hi*lo + lo*hi, FP32 accumulation */
    SMPS_PREC_BF16 = 3     /* one bf16 product, FP32 accumulation */
};

/* truncation rule (Sec. 2.3) */
enum {
    SMPS_TRUNC_REL_NORM2 = 0,  /* smallest r >= 1 with sum_{j>=r} s_j^2 <= tol * sum_j s_j^2 */
    SMPS_TRUNC_REL_SV = 1      /* keep s_j > tol * s_0 (at least one) */
};

/* factorization of the two-site tensor */
enum {
    SMPS_FACT_SVD = 0,        /* exact one-sided Jacobi SVD */
    SMPS_FACT_RSVD_MLP = 1,   /* randomized SVD sized by the rank predictor, exact SVD as fallback */
    SMPS_FACT_RSVD_PREV = 2,  /* randomized SVD sized by the bond's previous kept rank, exact fallback */
    SMPS_FACT_RSVD_FIXED = 3  /* randomized SVD with the sketch sized by the bond cap alone (no rank
                                 estimate: r = min(max_bond, m, n)), exact fallback; the baseline that
                                 the two estimates are measured against */
};
/* Randomized factorization (single-problem path only): Gaussian range finder
   (Halko, Martinsson & Tropp 2011, Alg. 4.1 with oversampling 16) on a sketch
   of k = r + 16 rows drawn from Philox4x64-10 (counter (block, step, 0, 0)),
   orthonormalised by two Gram passes (k x k Jacobi eigenproblems), then the
   SVD of the projected matrix (Rayleigh-Ritz) through its k x k Gram matrix.  r is the predicted rank: ceil(exp(output)) of the rank predictor on
   the bond's previous spectrum (RSVD_MLP), or the bond's previous kept rank
   (RSVD_PREV); for those two the step is exact when r >= min(max_bond, m, n)
   (a rank at the cap cannot meet the tolerance).  RSVD_FIXED takes
   r = min(max_bond, m, n).  Every mode is exact when k >= min(m, n).  The discarded weight
   ||theta||^2 - sum_{j<r} s_j^2 is exact; the step is accepted when it is at
   most tol * ||theta||^2 (relative-norm rule) and r <= k - 8, else the exact
   SVD replaces it.  The first left-to-right pass is always exact (no previous
   spectrum to predict from). */

/* Compression strategy (Sec. 2.3): maximum bond, tolerance, rule, and the
   number of sweeps of the variational search. */
typedef struct {
    int max_bond;      /* >= 1 */
    double tol;        /* >= 0 */
    int trunc_mode;    /* SMPS_TRUNC_* */
    int max_sweeps;    /* >= 1; a sweep is a left-to-right and a right-to-left pass */
    double sweep_tol;  /* 0: always run max_sweeps; > 0: stop once the relative change of
                          ||psi||^2 over a sweep falls below it (one host sync per sweep;
                          the batched entry point always runs max_sweeps) */
    int precision;     /* SMPS_PREC_* */
    int factorization; /* SMPS_FACT_* */
} smps_strategy;

/* Diagnostics of the last mpo_apply / simplify on a context. */
typedef struct {
    double error_bound;   /* sum over steps of sqrt(discarded weight): the accumulated
                             truncation-error bound kept with the state (Sec. 2.3) */
    double discarded;     /* sum over steps of the discarded weight */
    double norm;          /* Frobenius norm of the result's centre tensor (FP64) */
    int sweeps_done;
    int steps;            /* two-site updates performed (site-updates) */
    int rsvd_accepted;    /* randomized factorizations accepted */
    int rsvd_fallbacks;   /* randomized factorizations replaced by the exact SVD */
    int jacobi_sweeps;    /* Jacobi sweeps summed over the exact factorizations of the sweep */
    int reserved;
} smps_apply_info;

/* ---- context ---------------------------------------------------------------
 * device: HIP ordinal.  hip_stream: a hipStream_t (may be NULL for the null
 * stream) on which all work of this context is enqueued; the caller keeps it
 * alive for the lifetime of the context. */
int smps_ctx_create(int device, void *hip_stream, smps_ctx **out);
/* A planning context: no device is used, so it works on a host without a GPU.
 * Handles made in it hold shapes only (tensor data are not read), argument
 * validation and smps_plan_apply / smps_plan_apply_batched work, and every
 * call that would compute, read or copy device data returns SMPS_ENODEV
 * after its arguments have been validated. */
int smps_ctx_create_planning(smps_ctx **out);
int smps_ctx_destroy(smps_ctx *ctx);
const char *smps_last_error(const smps_ctx *ctx);
/* Bytes of device workspace the context currently holds (grow-only arena). */
int smps_ctx_workspace_bytes(const smps_ctx *ctx, size_t *bytes);
/* Upper bound on the workspace arena, in bytes (0 = none, the default).  A
 * call whose workspace would exceed it fails with SMPS_ENOMEM before any
 * device work; an arena already above a new limit is released. */
int smps_ctx_set_workspace_limit(smps_ctx *ctx, size_t bytes);
/* Exact split of a two-site tensor in the single-problem sweep (Sec. 2.3):
 *   SMPS_SPLIT_AUTO (default): the method measured fastest for the size --
 *     at present the one-sided Jacobi SVD for every size;
 *   SMPS_SPLIT_JACOBI: the one-sided Jacobi SVD for every step;
 *   SMPS_SPLIT_GRAM: vectors of at most 128 elements go through the Gram
 *     matrix H = X^T X, its Householder tridiagonal form and a
 *     divide-and-conquer eigensolver (the kept rows are eigenvectors of H,
 *     the singular values the norms ||X v_i||); longer vectors use the
 *     one-sided Jacobi SVD.
 * Batched launches always use the one-sided Jacobi SVD.  Unknown method:
 * SMPS_EINVAL. */
enum { SMPS_SPLIT_AUTO = 0, SMPS_SPLIT_JACOBI = 1, SMPS_SPLIT_GRAM = 2 };
int smps_ctx_set_split(smps_ctx *ctx, int method);
/* Per-phase kernel timing of the single-problem sweep, with HIP events
   recorded on the context stream around every launch (enabling it adds two
   event records per launch).  Categories:
     0 = factorizations (every split of the sweep),
     1 = contractions (every GEMM and MPO-site launch),
     2 = the splits of the largest square two-site tensor of the run (the
         bulk steps; also in 0),
     3 = contractions that build the X tensors of a sweep step (also in 1),
     4 = the two-site products theta (also in 1),
     5 = the environment updates after a split (also in 1),
     6 = every other launch (copies, fills, bond bookkeeping, norms).
   Contractions outside a sweep step (canonical form of the guess, warm-start
   rotations, the final projection) count in 1 only.  on != 0 enables it and
   clears the counters; smps_ctx_kernel_time returns the accumulated
   milliseconds and the number of timed launches of a category since then. */
int smps_ctx_set_profiling(smps_ctx *ctx, int on);
int smps_ctx_kernel_time(smps_ctx *ctx, int category, double *total_ms, long long *launches);

/* ---- MPS (Sec. 2.1, Eq. general-MPS) ---------------------------------------
 * L >= 1 sites; phys[L] local dimensions; bonds[L+1] with bonds[0] =
 * bonds[L] = 1.  tensors[k] points to bonds[k]*phys[k]*bonds[k+1] host values
 * of type dtype (C order); a NULL entry gives zeros.  Stored as FP64. */
int smps_mps_create(smps_ctx *ctx, int L, const int *phys, const int *bonds, int dtype,
                    const void *const *tensors, smps_mps **out);
/* Same, from device memory: tensors[k] are device pointers of type dtype; the
   data are copied on the context stream. */
int smps_mps_create_device(smps_ctx *ctx, int L, const int *phys, const int *bonds, int dtype,
                           const void *const *tensors, smps_mps **out);
int smps_mps_destroy(smps_mps *mps);
/* Shape query.  phys and bonds may be NULL; center = -1 unless the MPS is in
   canonical form with that isometry centre (Sec. 2.3). */
int smps_mps_shape(const smps_mps *mps, int *L, int *phys, int *bonds, int *center);
/* Copy site tensor `site` (FP64, C order) into host_out; count must equal its size. */
int smps_mps_read(smps_ctx *ctx, const smps_mps *mps, int site, double *host_out, size_t count);
/* Shape and site read-back of an operator: pout / pin (L ints each), bonds
   (L+1 ints), any may be NULL; site k is (bonds[k], pout[k], pin[k],
   bonds[k+1]) doubles in C order and count must equal that size. */
int smps_mpo_shape(const smps_mpo *mpo, int *L, int *pout, int *pin, int *bonds);
int smps_mpo_read(smps_ctx *ctx, const smps_mpo *mpo, int site, double *host_out, size_t count);
/* Device pointer of site tensor `site` (FP64, C order, owned by the handle). */
int smps_mps_device_ptr(const smps_mps *mps, int site, const double **ptr);

/* ---- MPO (Sec. 2.2, Eq. MPO) -------------------------------------------------
 * phys_out[L], phys_in[L]; bonds[L+1] with ends 1; tensors[k] has
 * bonds[k]*phys_out[k]*phys_in[k]*bonds[k+1] values [D_l][out][in][D_r]. */
int smps_mpo_create(smps_ctx *ctx, int L, const int *phys_out, const int *phys_in, const int *bonds,
                    int dtype, const void *const *tensors, smps_mpo **out);
int smps_mpo_destroy(smps_mpo *mpo);

/* ---- apply + compress (Sec. 2.4.2; Sec. 2.3 Eq. simplification; Sec. 2.5) ----
 * Returns in *out a new MPS psi approximating U v: the minimiser of
 * ||psi - U v||^2 over MPS with the strategy's bond limit, found by two-site
 * sweeps from the guess v (right-canonicalised).  psi is canonical with centre
 * 0 and is not normalised.  trunc_err (nullable) receives the accumulated
 * error bound.  Validation: L equal, phys_in(U) == phys(v), strategy fields in
 * range -> SMPS_EINVAL; non-finite two-site tensor -> SMPS_ENUMERIC. */
int smps_mpo_apply(smps_ctx *ctx, const smps_mpo *U, const smps_mps *v, const smps_strategy *strategy,
                   smps_mps **out, double *trunc_err);
/* Compression of v itself (Eq. simplification with phi = v): identical to
   smps_mpo_apply with the identity operator. */
int smps_simplify(smps_ctx *ctx, const smps_mps *v, const smps_strategy *strategy,
                  smps_mps **out, double *trunc_err);
/* Diagnostics of the last apply/simplify call on ctx. */
int smps_last_info(const smps_ctx *ctx, smps_apply_info *info);
/* Per-step log of the last apply/simplify: for step i (in sweep order),
   deltas[i] = discarded weight, ranks[i] = kept rank, spectra[i*32 + j] =
   j-th largest singular value (0 beyond the rank of the two-site tensor).
   Any pointer may be NULL; max_steps bounds the copy; *steps receives the
   number of steps available. */
int smps_last_log(const smps_ctx *ctx, int max_steps, double *deltas, int *ranks, double *spectra,
                  int *steps);
/* Factorization used at each step of the last single-problem apply/simplify:
   0 exact SVD, +k randomized with sketch k accepted, -k randomized with sketch k
   rejected and replaced by the exact SVD.  max_steps bounds the copy; *steps
   receives the number of steps available. */
int smps_last_factor_log(const smps_ctx *ctx, int max_steps, int *kinds, int *steps);
/* Per step of the last single-problem apply: the number of one-sided Jacobi
   sweeps that applied a rotation in its exact factorization (0 for randomized
   steps and for factorizations too large for the LDS-resident kernel).  Same
   copy contract as smps_last_log. */
int smps_last_jacobi_log(const smps_ctx *ctx, int max_steps, int *sweeps, int *steps);

/* Compression of a linear combination (Sec. 2.4.1, Eq. mps-sum-opt):
   *out ~ sum_l w[l] U[l] v[l], the minimiser over MPS of bond <= max_bond of
   || psi - sum_l w[l] U[l] v[l] ||^2 by the same two-site sweep as mpo_apply,
   with one set of three-layer environments per term (the local minimiser is
   the weighted sum of the terms' projections).  n >= 1 terms; w: n finite
   host doubles; U: n operator handles, or NULL, or NULL entries (identity);
   v: n state handles sharing L and the physical dimensions (operators must be
   square, as in mpo_apply).  The guess is v[0] (its bonds are the starting
   bonds).  Single-problem path; the result is canonical at site 0 and owned
   by the caller.  Errors: SMPS_EINVAL for bad arguments, otherwise as
   smps_mpo_apply. */
int smps_combine(smps_ctx *ctx, int n, const double *w, const smps_mpo *const *U, const smps_mps *const *v,
                 const smps_strategy *strategy, smps_mps **out, double *trunc_err);

/* Operator utilities (Sec. 2.4.1-2.4.3), built on mpo_apply / simplify:
 *   smps_mpo_transpose: new operator with the out and in indices of every site
 *       exchanged (in real arithmetic, the adjoint); caller owns *out.
 *   smps_mpo_apply_right: v @ U, the operator applied from the right
 *       (Sec. 2.4.2), computed as mpo_apply(U^T, v); same contract as mpo_apply.
 *   smps_mpo_list_apply: U[n-1] ... U[1] U[0] v applied one operator at a
 *       time, compressing after each product (Sec. 2.4.3); *trunc_err
 *       (nullable) receives the sum of the steps' error bounds.
 *   smps_mpo_simplify: compression of an operator (simplify_mpo, Sec. 2.4.1):
 *       the sites read as an MPS of site dimension out*in, compressed by
 *       simplify under the strategy, and returned as a new operator. */
int smps_mpo_transpose(smps_ctx *ctx, const smps_mpo *U, smps_mpo **out);
int smps_mpo_apply_right(smps_ctx *ctx, const smps_mps *v, const smps_mpo *U, const smps_strategy *strategy,
                         smps_mps **out, double *trunc_err);
int smps_mpo_list_apply(smps_ctx *ctx, int n, const smps_mpo *const *U, const smps_mps *v,
                        const smps_strategy *strategy, smps_mps **out, double *trunc_err);
int smps_mpo_simplify(smps_ctx *ctx, const smps_mpo *U, const smps_strategy *strategy, smps_mpo **out,
                      double *trunc_err);

/* Complex arithmetic (complex MPS / MPO; Sec. 2.1-2.4 with complex tensors).
 * Handles of complex states and operators are separate types.  Tensors are
 * complex128 in C order, the real and imaginary parts interleaved (re, im):
 * a site of `count` complex entries is 2 * count doubles; index orders are the
 * real path's ((chi_l, d, chi_r) and (D_l, d_out, d_in, D_r)).
 *   smps_zmps_create / smps_zmpo_create: copy host tensors to the device;
 *       smps_zmps_read copies one site back (count = complex entries).
 *   smps_zmpo_apply: psi ~ U v, compressed by the two-site variational sweep
 *       with the bra conjugated in the environments and a complex one-sided
 *       Jacobi SVD per split; strategy as for smps_mpo_apply but FP64 and the
 *       exact factorization only (SMPS_EUNSUPPORTED otherwise), square
 *       operator sites matching the state; two-site tensors must fit the
 *       factorization's LDS (about 9000 complex entries, SMPS_EUNSUPPORTED
 *       beyond); *out has its centre at site 0 and is not normalised;
 *       *trunc_err (nullable) receives the error bound; smps_last_info reports
 *       norm, steps and discarded weight.
 *   smps_zscprod: <a, b> = sum conj(a) b (Sec. 2.4.4), real and imaginary
 *       parts written to *re, *im. */
typedef struct smps_zmps smps_zmps;
typedef struct smps_zmpo smps_zmpo;
int smps_zmps_create(smps_ctx *ctx, int L, const int *phys, const int *bonds, const double *const *tensors,
                     smps_zmps **out);
int smps_zmps_destroy(smps_zmps *mps);
int smps_zmps_shape(const smps_zmps *mps, int *L, int *phys, int *bonds);
int smps_zmps_read(smps_ctx *ctx, const smps_zmps *mps, int site, double *host_out, size_t count);
int smps_zmpo_create(smps_ctx *ctx, int L, const int *pout, const int *pin, const int *bonds,
                     const double *const *tensors, smps_zmpo **out);
int smps_zmpo_destroy(smps_zmpo *mpo);
int smps_zmpo_apply(smps_ctx *ctx, const smps_zmpo *U, const smps_zmps *v, const smps_strategy *strategy,
                    smps_zmps **out, double *trunc_err);
int smps_zscprod(smps_ctx *ctx, const smps_zmps *a, const smps_zmps *b, double *re, double *im);

/* Ground-state search by two-site DMRG (Sec. 3.1.1).  H: a real symmetric
 * operator with pout == pin == the guess's physical dimensions.  guess: any
 * nonzero MPS of that shape (not modified; it is right-canonicalised and
 * normalised on a copy).  Each two-site update finds the lowest eigenpair of
 * the effective operator L[k] W_k W_{k+1} R[k+2] by Lanczos with at most
 * krylov_dim vectors (2..128; full re-orthogonalisation), then splits the pair
 * with the exact SVD under the strategy's max_bond / tol / trunc_mode.  A sweep
 * is a left-to-right and a right-to-left pass; strategy->max_sweeps sweeps run,
 * or fewer when sweep_tol > 0 and the relative change of the energy over a
 * sweep falls below it.  The computation is FP64 throughout (precision and
 * factorization must be SMPS_PREC_FP64 / SMPS_FACT_SVD).  On success *out (caller owns it)
 * is the normalised state with isometry centre 0 and *energy the Ritz value of
 * the last update.  Two-site tensors with more than 2048 rows or columns are
 * rejected with SMPS_EUNSUPPORTED. */
int smps_dmrg(smps_ctx *ctx, const smps_mpo *H, const smps_mps *guess, const smps_strategy *strategy,
              int krylov_dim, smps_mps **out, double *energy);

/* Batched apply: n independent (U[i], v[i]) problems of arbitrary length and
   bonds under one strategy, advanced together bond step by bond step; the
   launch sequence is captured once in a HIP graph per batch shape and replayed.
   out[i] as for smps_mpo_apply; trunc_err (nullable) has n entries. */
int smps_mpo_apply_batched(smps_ctx *ctx, int n, const smps_mpo *const *U, const smps_mps *const *v,
                           const smps_strategy *strategy, smps_mps **out, double *trunc_err);
/* The same with a bond cap per problem: max_bonds[i] (>= 1) replaces
   strategy->max_bond for problem i, so that chains compressed at different
   caps share one batch (one graph).  max_bonds NULL: the strategy's cap for
   every problem (= smps_mpo_apply_batched). */
int smps_mpo_apply_batched_caps(smps_ctx *ctx, int n, const smps_mpo *const *U, const smps_mps *const *v,
                                const int *max_bonds, const smps_strategy *strategy, smps_mps **out,
                                double *trunc_err);

/* ---- planning (host only) ------------------------------------------------------
 * What smps_mpo_apply (one problem) or smps_mpo_apply_batched (n problems)
 * would allocate and enqueue for these handles and strategy (Sec. 2.5
 * sweep), computed on the host: nothing is allocated on or sent to a device,
 * in either kind of context.  Same validation and the same refusals as the
 * apply: SMPS_EUNSUPPORTED for two-site tensors beyond 2048 rows or columns
 * and for a batch whose graph would exceed the kernel limit, SMPS_ENOMEM for
 * a workspace above the context's limit; *info is filled before such a
 * refusal, so the sizes that caused it can be read. */
typedef struct {
    size_t workspace_bytes;  /* device workspace of the call */
    long long steps;         /* two-site updates, summed over the problems */
    long long operations;    /* operations of the recorded sequence(s) */
    long long launches;      /* batched: merged launches; single problem: = operations */
    long long graph_kernels; /* batched: kernels the captured graph holds (upper bound); else 0 */
    size_t descriptor_bytes; /* batched: descriptor arrays uploaded with the graph; else 0 */
} smps_plan_info;
int smps_plan_apply(smps_ctx *ctx, const smps_mpo *U, const smps_mps *v, const smps_strategy *strategy,
                    smps_plan_info *info);
/* max_bonds: as for smps_mpo_apply_batched_caps (NULL: the strategy's cap). */
int smps_plan_apply_batched(smps_ctx *ctx, int n, const smps_mpo *const *U, const smps_mps *const *v,
                            const int *max_bonds, const smps_strategy *strategy, smps_plan_info *info);

/* ---- scalar product and norm (Sec. 2.4.4) -------------------------------------
 * scprod: <a, b> by the transfer-matrix sweep, O(L chi^3 d), FP64.
 * norm: ||a|| -- from the centre tensor when a is canonical (O(d chi^2)),
 * otherwise sqrt(scprod(a, a)). */
int smps_scprod(smps_ctx *ctx, const smps_mps *a, const smps_mps *b, double *out);
int smps_norm(smps_ctx *ctx, const smps_mps *a, double *out);

/* ---- scalar product without allocation -----------------------------------------
 * For callers that cannot allocate device memory: code being captured into a
 * HIP graph, serving loops that must not call hipMalloc, harnesses that forbid
 * it.  Same transfer-matrix sweep and the same products as smps_scprod, but
 * its workspace is a fixed 4 MiB device array of the library (one per device,
 * held until the process ends) instead of the context's grow-only arena, and
 * the result is written to device memory instead of the host:
 *   out_dev: device address of one double, owned by the caller; written
 *            stream-ordered on the context's stream (no host synchronisation;
 *            the caller synchronises before reading it).
 * Limit: 2 * max_k(chi_a[k] chi_b[k]) + max_k(chi_a[k] d_k chi_b[k+1]) doubles
 * (each part rounded up to 256 bytes) must fit in 4 MiB -- e.g. chi <= 256
 * at d = 2 -- else SMPS_ENOMEM and nothing is launched.  No allocation of any
 * kind happens inside the call.  Every call on one device shares that
 * device's array: calls that overlap on one device (different streams or
 * contexts, or host threads) race and must be serialised by the caller. */
int smps_scprod_noalloc(smps_ctx *ctx, const smps_mps *a, const smps_mps *b, double *out_dev);

/* ---- learned rank predictor for the randomized factorization ------------------
 * A 32-64-64-1 ReLU network with bf16 weights (FP32 master copy, FP32
 * accumulation).  Input: the 32 largest log(s_j / s_0) of a bond's spectrum in
 * the previous sweep (padded with log(1e-30)); output: log of the kept rank.
 * Training runs on the device with the library's own forward, backward and
 * Adam kernels.
 *   feats: n x 32 host floats; labels: n host floats (log rank).
 *   smps_rank_mlp_init: seed the weights (deterministic in seed).
 *   smps_rank_mlp_train: `epochs` passes of mini-batch Adam (batch, lr);
 *       *final_loss receives the mean loss of the last epoch.
 *   smps_rank_mlp_predict: out[n] = predicted log rank.
 *   smps_rank_mlp_get / set: the FP32 master parameters in the order
 *       W1[64x32], b1[64], W2[64x64], b2[64], W3[1x64], b3[1] (6337 floats). */
int smps_rank_mlp_init(smps_ctx *ctx, unsigned long long seed);
int smps_rank_mlp_train(smps_ctx *ctx, int n, const float *feats, const float *labels, int epochs, int batch,
                        float lr, float *final_loss);
int smps_rank_mlp_predict(smps_ctx *ctx, int n, const float *feats, float *out);
int smps_rank_mlp_get(const smps_ctx *ctx, float *params, int count);
int smps_rank_mlp_set(smps_ctx *ctx, const float *params, int count);
/* Training pairs from the last single-problem apply/simplify: for every step
   whose bond was factorized before in that call, feats (32 floats) are the
   predictor inputs built from the previous factorization's spectrum and the
   label is log(kept rank) of this step.  feats: max_pairs x 32, labels:
   max_pairs (either may be NULL to query *count, the number available). */
int smps_rank_training_pairs(const smps_ctx *ctx, int max_pairs, float *feats, float *labels, int *count);
/* One forward + backward of the loss on a host batch, returning the loss and
   the gradient w.r.t. the FP32 master parameters (same order as _get); used to
   check the hand-written backward kernels. */
int smps_rank_mlp_grad(smps_ctx *ctx, int n, const float *feats, const float *labels, float *loss,
                       float *grad, int count);

/* ---- GEMM tile autotuner --------------------------------------------------------
 * Each dense product runs with one of four output tiles (64x64, 64x32, 32x64,
 * 32x32, ids 0-3).  The process-wide table maps (precision, operand/result
 * types, transposes, power-of-two buckets of the M and N allocation caps) to
 * the fastest tile; products without an entry use 64x64.  The tile never
 * changes result bits (every tile sums each output in the same k order).
 *   smps_autotune_apply: record the products one apply + compression of
 *       (U, v, strategy) would launch, time the four tiles on each distinct
 *       shape (reps launches each, synthetic operands) and store the best;
 *       *tuned (nullable) receives the number of shapes timed.
 *   smps_autotune_gemm: the same for one M x N x K product (types SMPS_F64 /
 *       SMPS_F32, ta/tb/tc as in the library's products); *best_tile nullable.
 *   smps_autotune_save / _load: the table as JSON (one entry per line; load
 *       merges); smps_autotune_clear empties it; smps_autotune_entries counts. */
int smps_autotune_apply(smps_ctx *ctx, const smps_mpo *U, const smps_mps *v, const smps_strategy *strategy,
                        int reps, int *tuned);
int smps_autotune_gemm(smps_ctx *ctx, int precision, int M, int N, int K, int ta, int tb, int tc, int a_type,
                       int b_type, int c_type, int reps, int *best_tile);
int smps_autotune_save(smps_ctx *ctx, const char *path);
int smps_autotune_load(smps_ctx *ctx, const char *path);
int smps_autotune_clear(smps_ctx *ctx);
int smps_autotune_entries(const smps_ctx *ctx, int *count);

#ifdef __cplusplus
}
#endif

#endif /* SEEMPS_HIP_H */
