/*
 * sppc.h - C ABI of the SPPC eigensolver on one MI355X (gfx950).
 *
 * Subspace Projection with Perturbative Corrections (SPPC): the k lowest
 * eigenpairs of a large sparse symmetric H = H0 + V, where H0 = diag(H0hat, 0)
 * and H0hat is the leading n0 x n0 block (the small configuration space,
 * Sec. II eqs. split/split2).  The subspace is spanned by the zero-padded
 * eigenvectors of H0hat and their perturbative corrections (eq. exp_seq2,
 * solved in the small space, eqs. sm_first and sm_lin_proj), and the
 * approximations are the Rayleigh-Ritz pairs of that subspace (eq. tilde_H,
 * Alg. 2), judged by the relative residual ||Hz - theta z|| / |theta| (eq. rrn).
 *
 * Conventions for every entry point:
 *   - every pointer named *_dev is device memory owned by the caller and must
 *     stay valid for the lifetime of the context that uses it; *_host is host
 *     memory owned by the caller;
 *   - blocks of vectors are row-major n x b (the b values of one row are
 *     contiguous, leading dimension b);
 *   - all work is enqueued on the stream given to sppc_setup; entry points that
 *     return host values synchronise that stream;
 *   - return codes are sppc_status values; no C++ exception crosses this ABI;
 *     sppc_last_error() gives a readable message for the last failure;
 *   - a context is used by one host thread at a time.
 */
#ifndef SPPC_H_
#define SPPC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPPC_OK = 0,
  SPPC_E_ARG = 1,           /* invalid argument or shape */
  SPPC_E_HIP = 2,           /* a HIP runtime call failed */
  SPPC_E_NOMEM = 3,         /* device allocation failed */
  SPPC_E_SINGULAR_E0 = 4,   /* some wanted E_k^(0) is zero: eq. sm_first divides by it */
  SPPC_E_BREAKDOWN = 5,     /* the subspace could not be extended (every new direction dropped) */
  SPPC_E_NOCONV = 6,        /* iteration limit reached; the best pairs are still written */
  SPPC_E_NAN = 7            /* a NaN or Inf appeared */
} sppc_status;

typedef enum { SPPC_F64 = 0, SPPC_F32 = 1 } sppc_dtype;

/* Shift of the small-space corrections in eq. sm_first and eq. sm_lin_proj. */
typedef enum {
  SPPC_SHIFT_E0 = 0,    /* E_k^(0), the zeroth-order energy (the paper's recursion, eq. exp_seq2) */
  SPPC_SHIFT_RITZ = 1   /* theta_k, the Ritz value of the step before: (H0hat - theta_k) x1 = b1 and
                           x2 = -b2 / theta_k, with the same right-hand side and E^(p) (a variant the
                           paper does not take; it stagnates earlier on the synthetic workloads) */
} sppc_shift;

typedef enum {
  SPPC_PREC_FP64 = 0,   /* every product in float64 */
  SPPC_PREC_MIXED = 1   /* block products with H: float32 X, float32 products accumulated in
                           float64 (the diagonal term in float64), until the largest relative
                           residual falls below 1e-4, float64 after that.  H Psi^(0), the
                           small-space solves (inner_tol 1e-6 by default), basis, projected matrix,
                           orthonormalisation, Rayleigh-Ritz and the final residual check are
                           float64; a float64 refinement follows when the check fails */
} sppc_precision;

typedef enum {
  SPPC_CORR_PERTURBATIVE = 0, /* Psi^(p) of eq. exp_seq2 for every wanted pair (Alg. 2 step 6) */
  SPPC_CORR_JACOBI = 1,       /* continuation: t_i = -(I - z_i z_i^T) (diag(H) - theta_i)^-1 r_i */
  SPPC_CORR_MPNN = 2,         /* continuation: learned diagonal scaling of the Jacobi step */
  SPPC_CORR_SMALL = 3,        /* continuation: t_i = -(I - z_i z_i^T) M_i r_i with M_i = (H0hat - theta_i)^-1
                                 on the small-space rows (deflated CG to a loose tolerance plus the
                                 exact deflated terms) and (diag(H) - theta_i)^-1 on the other rows */
  SPPC_CORR_RMMDIIS = 4       /* continuation of the SPPC + RMM-DIIS hybrid (Sec. V-VI): after the
                                 perturbative steps every unconverged Ritz pair is refined on its own
                                 by RMM-DIIS (Pulay's DIIS over the pair's iterates of the current sweep,
                                 at most 5, then the residual-minimising step along
                                 (diag(H) - theta)^-1 r or the learned step (rmm_precond); one product
                                 with H per pair and iteration, the pairs batched), in sweeps of 4
                                 with Rayleigh-Ritz on the refined vectors between them; once the
                                 largest residual has not halved over three sweeps the Davidson
                                 continuation with the diagonal step takes over from the refined Ritz
                                 vectors; at most max_cont iterations and steps in all; the final
                                 check takes Rayleigh-Ritz on the refined vectors, and if its true
                                 residuals miss the tolerance the float64 refinement follows
                                 (refine_precond), as after a mixed solve.  sppc_solve only (not a block for sppc_correct); not a
                                 refine_precond */
} sppc_corr_kind;

/* Upper triangle (diagonal included) of the symmetric H, CSR, device memory. */
typedef struct {
  int64_t n;                /* order of H */
  int64_t nnz;              /* stored entries (upper triangle with the diagonal) */
  const int64_t* row_ptr_dev; /* [n+1] */
  const int32_t* col_dev;   /* [nnz], columns >= row, ascending within a row */
  const void* val_dev;      /* [nnz], float64 or float32 */
  sppc_dtype val_type;
} sppc_csr;

typedef struct {
  double tol;          /* convergence: every rrn_i < tol (eq. rrn); default 1e-6 */
  int maxiter;         /* highest perturbation order of pure SPPC (Alg. 2 input); default 30 */
  int p_switch;        /* after this many SPPC steps switch to the continuation (0 = never) ; 15 */
  int max_cont;        /* continuation steps at most (RMM-DIIS iterations and the Davidson steps after
                          its hand-over together); the float64 refinement after a failed check has
                          a budget of its own of the same size; default 200 */
  int m_max;           /* basis columns kept (2k..512); the continuation restarts beyond it.  0 (the
                          default) = automatic: k (p_switch + 1) rounded up to 16 with the RMM-DIIS
                          continuation (which restarts the basis at every sweep), else 512 */
  int n_deflate;       /* eigenpairs of H0hat computed and deflated in the small solves (k..28);
                          0 (the default) = min(3k, 28, n0) with small solves to 1e-9 or tighter (the
                          float64 default), min(2k, 28, n0) with looser ones (the mixed default); with
                          pair_index j at least j + 2 */
  double tau_drop;     /* new column dropped when sin(angle to the basis) <= tau_drop */
  double inner_tol;    /* relative residual of the small-space solves; 0 = 1e-12 (FP64) / 1e-6 (MIXED) */
  double h0_tol;       /* residual of the H0hat eigenpairs, relative to max(1,|E|); default 1e-12.
                          The pairs beyond the wanted ones (kept only to deflate the small solves)
                          stop at max(h0_tol, 1e-3 inner_tol): 1e-9 in the mixed form */
  int precision;       /* sppc_precision; MIXED adds a float64 refinement when the final check fails */
  int precond;         /* sppc_corr_kind used by the continuation (JACOBI, MPNN, SMALL or RMMDIIS); JACOBI */
  int final_check;     /* explicit float64 H Z, Rayleigh-Ritz on span Z, true residual */
  int verbose;         /* per-iteration line on stderr */
  int panel_width;     /* block products with H over column panels of this many columns (<= 65536),
                          so that the gathered rows of X stay in L2: -1 = automatic (when a k-column
                          block of X exceeds 8 MiB and n < 2^24), 0 = off.  The panel copy stores a
                          column in 24 bits: an explicit width with n >= 2^24 is refused by
                          sppc_setup (SPPC_E_ARG), and the automatic choice then keeps the row-wise
                          products over the full CSR */
  int refine_precond;  /* continuation kind of the float64 refinement after a failed check of a mixed
                          solve or of the SPPC + RMM-DIIS hybrid; SMALL */
  double precond_tol;  /* relative residual of the small-space solve inside SMALL; 1e-3 */
  int auto_switch;     /* 1: switch to the continuation before p_switch once SPPC stagnates: after a
                          step the smallest sine of the angle between a new correction vector and
                          the basis is below 1e-4 (Fig. 3), or the largest rrn has not halved over
                          the last three steps (detection left open by the paper, Sec. VII); takes
                          effect only with p_switch > 0; 0 (default): switch at p_switch only */
  int corr_shift;      /* sppc_shift of the perturbative corrections in sppc_solve; SPPC_SHIFT_E0 */
  int pair_index;      /* -1 (default): Alg. 2, the k lowest pairs together.  j = 0..26 with k = 1:
                          Alg. 1 for the j-th eigenpair alone (j = 0 the lowest): the zeroth order is
                          the j-th eigenpair of H0hat, the subspace the span of its own corrections,
                          the approximation the lowest Ritz pair of that subspace (which may move to a
                          lower eigenvalue, Sec. VI).  n_deflate (default at least j + 2, at most 28)
                          must exceed j; sppc_get(what = 0) then lists E_j^(0) first */
  int rmm_precond;     /* step of the RMM-DIIS continuation: SPPC_CORR_JACOBI (the diagonal step,
                          default) or SPPC_CORR_MPNN (the learned correction of the diagonal step,
                          weights from sppc_mpnn_set_weights; a pair falls back to the diagonal step
                          for good as soon as the iterate a learned step produced has a relative
                          residual not below 0.9x that of the iterate the step started from) */
} sppc_opts;

typedef struct {
  int iterations;      /* SPPC steps p reached */
  int cont_steps;      /* continuation steps (refinement steps included) */
  int refine_steps;    /* float64 refinement steps after a failed check of a mixed-precision solve or
                          of the float64 SPPC + RMM-DIIS hybrid */
  int mpnn_steps;      /* continuation steps that used the learned preconditioner */
  int64_t n_spmv;      /* products of H with one vector (k per SPPC step, Sec. IV.C; a learned step
                          adds the network's two per pair) */
  int64_t spmm_calls;  /* block products with H (kernel launches) */
  int64_t spmm_cols;   /* sum of their block widths */
  int basis_size;      /* columns of the final basis */
  int cg_iterations;   /* small-space solver iterations, summed over steps */
  int h0_iterations;   /* iterations of the H0hat eigensolver */
  int converged;       /* 1 if every pair met tol (after the final check when enabled) */
  double t_setup_ms;   /* device format, H0hat extraction, zeroth order */
  double t_solve_ms;   /* iteration loop + final check */
  double t_spmm_ms;    /* time inside the block-product kernels with H (HIP events) */
  double t_small_ms;   /* time inside the small-space solves */
  double t_ortho_ms;   /* block Gram-Schmidt + Cholesky-QR */
  double t_rr_ms;      /* projected matrix, eigensolve, Ritz vectors, residuals */
  double spmm_alg_bytes; /* algorithmic bytes of the counted products with H: the stored upper
                            triangle once (values as read: float32 when lossless or mixed;
                            int32 columns; int64 row pointers) + X read + Y written */
  double t_h0_ms;      /* time inside products with H0hat outside the small solves */
  int mpnn_fallbacks;  /* pairs that the true residual sent back to the diagonal step */
  int64_t workspace_peak; /* bytes of the caller's workspace in use at the peak so far (0 without one) */
  int rmm_iterations;  /* RMM-DIIS iterations of the SPPC + RMM-DIIS hybrid (counted in cont_steps) */
  int rmm_handover;    /* 1 if stagnated RMM-DIIS sweeps handed over to the Davidson continuation with
                          the diagonal step (the largest residual did not halve over three sweeps) */
} sppc_stats;

typedef struct sppc_ctx sppc_ctx;

/* Fills *opts with the defaults listed above.  Returns SPPC_E_ARG for NULL. */
sppc_status sppc_default_opts(sppc_opts* opts);

/*
 * Bytes of device workspace that sppc_setup followed by sppc_solve needs for this problem and these
 * options (arguments as sppc_setup): the arrays the context keeps (the device copies of H, H0hat,
 * the basis Q and H Q of m_max columns, the blocks, the RMM-DIIS histories or the learned
 * preconditioner's arrays when the options use them) plus the largest set of setup temporaries
 * alive at one time.  It runs the checks of sppc_setup and reads H's row pointer of the first row
 * outside the small space (one 8-byte copy from the device); it allocates nothing.  The entry
 * count of the full matrix is bounded by twice the stored entries, and for float64 values both
 * outcomes of the float32-exactness check are covered, so the figure is an upper bound.
 * Errors: as sppc_setup's argument checks (the message in sppc_setup_error()).
 */
sppc_status sppc_workspace_size(const sppc_csr* H, const int64_t* level_offsets_host, int n_levels,
                                int n_small_levels, int k, const sppc_opts* opts, size_t* bytes);

/*
 * Builds a context for the k lowest eigenpairs of H (Alg. 2 input).
 *   H                 upper CSR in device memory (see sppc_csr)
 *   level_offsets_host  [n_levels+1] host array, 0 = first row of each level, last = n
 *   n_small_levels    the leading levels that form the small space: n0 = level_offsets[n_small_levels]
 *                     (H0hat = H[0:n0, 0:n0], eq. split2)
 *   k                 wanted pairs, 1 <= k <= 16, k <= n_deflate <= n0
 *   opts              NULL for the defaults
 *   workspace_dev, workspace_bytes
 *                     device memory owned by the caller (at least sppc_workspace_size bytes) from
 *                     which every device array of the context is taken, setup temporaries
 *                     included; it must stay valid and unused by anything else until
 *                     sppc_destroy.  NULL: the library allocates (hipMalloc, returned by
 *                     sppc_destroy; see sppc_set_memory_cache).
 *   stream            hipStream_t (as void*), NULL for the default stream
 * Work: device copy of H in both triangles (float32 values when every value is
 * float32-exact, else float64), H0hat, the n_deflate lowest eigenpairs of
 * H0hat (eq. EP_small), and step p = 0 of Alg. 2 (basis Psi^(0), one block
 * product with H, Rayleigh-Ritz).  Errors: SPPC_E_ARG, SPPC_E_NOMEM (also when a
 * workspace is too small), SPPC_E_HIP, SPPC_E_SINGULAR_E0 (*out is then NULL).
 */
sppc_status sppc_setup(sppc_ctx** out, const sppc_csr* H, const int64_t* level_offsets_host,
                       int n_levels, int n_small_levels, int k, const sppc_opts* opts, void* workspace_dev,
                       size_t workspace_bytes, void* stream);

/*
 * Y = H X for the matrix of the context (the paper's cost unit, Sec. IV.C).
 *   X_dev   row-major n x b, float64 (xt = SPPC_F64) or float32 (SPPC_F32)
 *   Y_dev   row-major n x b, float64
 *   b       1..32 (widths above 16 take the row-wise kernel over the full CSR)
 * float64 X uses the float64 values; float32 X uses the float32 values with
 * float32 products accumulated in float64.  Asynchronous on the context stream.
 */
sppc_status sppc_spmm(sppc_ctx* ctx, const void* X_dev, sppc_dtype xt, double* Y_dev, int b);

/*
 * Y = H X read from the upper triangle alone (Sec. IV.C's product with the symmetric H; no
 * context, no mirrored copy): the strictly lower half is applied as the transpose of the stored
 * entries, each adding its share to a row of Y by a float64 atomic add.  Streams half the matrix
 * bytes of the full-storage product at the price of those scattered adds.
 *   H       the caller's upper CSR (as for sppc_setup), float64 or float32 values; only read
 *   X_dev   row-major n x b, float64 (xt = SPPC_F64) or float32 (SPPC_F32), only read
 *   Y_dev   row-major n x b, float64, overwritten (zeroed, then accumulated); must not overlap X, and
 *           must be ordinary device memory (hipMalloc or a torch tensor): the float64 atomic adds run
 *           in the device's caches and memory, not across PCIe
 *   b       1..32
 *   stream  hipStream_t (as void*), NULL for the default stream; asynchronous on it
 * float64 X: float64 products of the values as stored.  float32 X: each value rounded to float32,
 * float32 products, float64 sums.  The order of the float64 sums depends on scheduling, so two
 * calls can differ in the last bits.  Allocates nothing.  Errors: SPPC_E_ARG (message in
 * sppc_setup_error()), SPPC_E_HIP.
 */
sppc_status sppc_spmm_upper(const sppc_csr* H, const void* X_dev, sppc_dtype xt, double* Y_dev, int b,
                            void* stream);

/*
 * Y = H X exactly as sppc_spmm, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): this call allocates
 * nothing.  When the context holds the column-panel copy of H and X is not already in the layout
 * its kernels read (b in {4, 8, 16} columns per row, 16-byte aligned), X is copied to a row stride
 * B = 4, 8 or 16 in the library's static device scratch array (32 MiB per device, held until the
 * process ends) instead of the context's buffer; n * B * sizeof(X element) beyond 32 MiB is
 * rejected with SPPC_E_ARG.  Every call on one device shares that array and it keeps the last
 * call's contents: calls that overlap on one device (several streams or threads) race.
 * Arguments, layout and errors as sppc_spmm.
 */
sppc_status sppc_spmm_noalloc(sppc_ctx* ctx, const void* X_dev, sppc_dtype xt, double* Y_dev, int b);

/*
 * Computes the next block of new directions into the context (not yet in the basis):
 *   SPPC_CORR_PERTURBATIVE: E_k^(p) and Psi_k^(p) for every wanted pair from
 *     eq. exp_seq (first line) and eq. exp_seq2, with H Psi^(p-1) taken from
 *     the stored H Q (eq. HPsip) and V Psi = H Psi - H0 Psi (eq. avoid_SpMV2);
 *     complement rows by eq. sm_first, small-space rows by eq. sm_lin_proj
 *     (minimum-norm solution orthogonal to psi_k).
 *   SPPC_CORR_JACOBI / SPPC_CORR_MPNN / SPPC_CORR_SMALL: preconditioned residuals of
 *     the current unconverged Ritz pairs (Sec. V continuation; the pending block is
 *     n x (number of unconverged pairs)).
 *   shifts_host  [k] host array or NULL.  PERTURBATIVE only: sigma_k replaces E_k^(0) in eq. sm_first
 *     (x2 = -b2 / sigma_k) and eq. sm_lin_proj ((H0hat - sigma_k) x1 = b1 - (b1^T psi_k) psi_k,
 *     minimum-norm, x1 orthogonal to psi_k); the right-hand side of eq. exp_seq2 and E^(p) are
 *     unchanged.  NULL is the paper's E^(0).  Each sigma_k must be finite, nonzero and at most the
 *     largest deflated eigenvalue E_D^(0) of H0hat (sppc_get what = 0), so that the deflated CG
 *     operator is positive definite; the Ritz values theta_k always are.
 * Errors: SPPC_E_ARG (e.g. PERTURBATIVE after the basis was restarted, shifts out of range or given
 * to a continuation kind), SPPC_E_SINGULAR_E0 (a zero shift), SPPC_E_HIP.
 */
sppc_status sppc_correct(sppc_ctx* ctx, int kind, const double* shifts_host);

/*
 * Appends the pending block to the basis and extracts new Ritz pairs:
 * block Gram-Schmidt twice + Cholesky-QR twice (eqs. blkGS, QR, Qp), one block
 * product with H, the new rows and columns of T = Q^T H Q (eq. proj), the k
 * lowest eigenpairs of T and the residual norms (eq. rrn).
 *   theta_host, rrn_host  [k] outputs (may be NULL); n_added_host: columns appended.
 * Synchronises the stream.  Errors: SPPC_E_BREAKDOWN (nothing appended), SPPC_E_NAN, SPPC_E_HIP.
 */
sppc_status sppc_rayleigh_ritz(sppc_ctx* ctx, double* theta_host, double* rrn_host,
                               int* n_added_host);

/*
 * The whole method: Alg. 2 until every rrn_i < tol or p = p_switch (or maxiter;
 * with auto_switch also once SPPC stagnates), then the continuation chosen by
 * opts.precond (a preconditioned basis expansion, or the per-pair RMM-DIIS
 * refinement of the SPPC + RMM-DIIS hybrid, Sec. V-VI), then (if enabled) the
 * final float64 check and, in mixed precision, the float64 refinement.  Outputs:
 *   evals_host  [k] ascending
 *   evecs_dev   row-major n x k float64 (may be NULL)
 *   rrn_host    [k] relative residuals (may be NULL)
 *   stats       may be NULL
 * Returns SPPC_OK, or SPPC_E_NOCONV with the best pairs written.
 */
sppc_status sppc_solve(sppc_ctx* ctx, double* evals_host, double* evecs_dev, double* rrn_host,
                       sppc_stats* stats);

/*
 * Copies internal state for inspection (tests):
 *   what = 0: E^(0) [n_deflate] (host)          what = 1: Ritz values of the last step [k] (host)
 *   what = 2: basis size m (as double, host)    what = 3: Q, row-major n x m (device, ld = m)
 *   what = 4: H Q, row-major n x m (device)     what = 5: pending block, row-major n x k (device)
 *   what = 6: T, m x m (host, row-major)        what = 7: angles of the last appended block [k] (host)
 *   what = 8: E^(p) table [(p+1) x k] (host)    what = 9: H0hat eigenvectors, row-major n0 x n_deflate (device)
 *   what = 10: Ritz vectors Z, n x k (device)   what = 11: residuals R = H Z - Z diag(theta), n x k (device)
 * `count` is the capacity of dst in doubles.  Errors: SPPC_E_ARG.
 */
sppc_status sppc_get(sppc_ctx* ctx, int what, double* dst, int64_t count);

/* ------------------------------------------------------------------ learned preconditioner
 *
 * A 2-layer message-passing network over the graph of H (hidden width 32) scales the diagonal
 * step of the continuation row by row.  For a Ritz pair (theta, x) with residual r:
 *   f = [r / rms(r), (d - theta)/(1 + |theta|), lambda],  g = A f,  A = H - diag(d),
 *   lambda = min(max(level - n_small_levels + 1, 0), 2) / 2  (0 on the small-space levels, 1/2 on the
 *            first level outside them, 1 beyond: the same for any number of levels)
 *   h = tanh(Ws f + Wn g + b1),  o = ws.h + A (wn.h) + b2,
 *   t = tJ (1 + o) with the diagonal step tJ = r / (d - theta) (|d - theta| >= 1e-2 max(1,|theta|)),
 *   t~ = t - x (x^T t);  the continuation direction is -t~.  A zero network is the diagonal step.
 * Parameters (float32, 289): Ws[32x3] | Wn[32x3] | b1[32] | ws[32] | wn[32] | b2, row-major.
 * The solver uses them rounded to bfloat16, with float32 arithmetic; the products with H are float64.
 */
#define SPPC_MPNN_NPARAM 289

/* Weights for SPPC_CORR_MPNN (host, 289 floats, copied).  Non-finite weights make every pair use
 * the diagonal step.  During the continuation a pair whose true residual did not fall below 0.9x
 * its value at its previous learned step uses the diagonal step from then on. */
sppc_status sppc_mpnn_set_weights(sppc_ctx* ctx, const float* w_host);

/*
 * Evaluates the network for S (1..32) samples on the matrix of the context.
 *   w_host        289 parameters (host)
 *   R_dev, X_dev  n x S row-major: residuals and unit Ritz vectors (device)
 *   theta_host    [S] Ritz values
 *   Q_dev, m      optional basis (n x m row-major, orthonormal columns spanning every x_s, device):
 *                 the output is then projected as t - Q (Q^T t), the part that enlarges the basis.
 *                 NULL / 0: t - x (x^T t).  m <= 512.
 *   E_dev         n x S targets, or NULL (then no loss / gradient)
 *   T_dev         n x S projected output (device), or NULL
 *   loss_host     [S] per-sample loss 1 - cos^2(projected output, e), or NULL
 *   grad_host     [289] gradient of the mean loss, or NULL
 *   f64           1: float64 arithmetic and exact weights (gradient checks); 0: float32 arithmetic
 *                 with bfloat16-rounded weights (the solver's form)
 * Errors: SPPC_E_ARG (S out of range, missing arrays, loss/grad requested without E).
 */
sppc_status sppc_mpnn_eval(sppc_ctx* ctx, const float* w_host, int S, const double* R_dev, const double* X_dev,
                           const double* theta_host, const double* Q_dev, int m, const double* E_dev,
                           double* T_dev, double* loss_host, double* grad_host, int f64);

/*
 * One training step on the GPU: forward, backward (one more product with H), and an Adam update
 * (beta 0.9 / 0.999) of the float32 master weights.  Arguments as in sppc_mpnn_eval.
 *   state_dev  device float[4 x 289]: weights | first moments | second moments | bfloat16 copy
 *   step       Adam step count (>= 1); loss_host: mean loss of the batch before the update (or NULL)
 */
sppc_status sppc_mpnn_train_step(sppc_ctx* ctx, float* state_dev, int S, const double* R_dev, const double* X_dev,
                                 const double* theta_host, const double* Q_dev, int m, const double* E_dev,
                                 float lr, int step, double* loss_host);

/* Training targets E = (I - Q Q^T) Psi (n x S, device) for the exact eigenvectors Psi (n x S, device)
 * and the basis Q (n x m, orthonormal columns, device): the part of each eigenvector that a
 * subspace expansion still has to supply.  A direction that the Davidson step of Sec. V
 * orthogonalises against Q adds psi_s to the span exactly when it is parallel to E[:, s]. */
sppc_status sppc_mpnn_target(sppc_ctx* ctx, int S, const double* Q_dev, int m, const double* Psi_dev,
                             double* E_dev);

const char* sppc_last_error(const sppc_ctx* ctx);

/* Message of the last failure in sppc_setup (no context exists then). */
const char* sppc_setup_error(void);

/* Waits for the context's stream, then gives every device and pinned allocation of the context
 * back to the library's memory cache.  NULL is ignored. */
void sppc_destroy(sppc_ctx* ctx);

/*
 * Device memory the library allocates itself (contexts set up without a workspace) is returned
 * with hipFree when it is given back, unless this cache is enabled: with bytes_per_device > 0 a
 * block given back by sppc_destroy or by setup is kept and handed to the next request of the same
 * rounded size (2 MiB granules) on the same device, up to that many bytes (and at most 3/4 of the
 * device's memory) per device.  Repeated setups of one problem size then allocate nothing
 * (hipMalloc/hipFree stall the host, and VRAM freed recently is cleared by the driver before it is
 * handed out again, about a second per 100 GB), but PyTorch's allocator cannot see or trim the
 * cached blocks.  An allocation that fails empties the cache of its device and is tried once more.
 * 0 (the default) disables the cache and frees what it holds.  Returns the previous limit.
 * Thread-safe.
 */
size_t sppc_set_memory_cache(size_t bytes_per_device);

/* Frees every block the cache holds (of every device) now; returns the number of bytes freed.
 * Thread-safe; blocks in use by live contexts are not affected. */
size_t sppc_release_cached_memory(void);

#ifdef __cplusplus
}
#endif
#endif /* SPPC_H_ */
