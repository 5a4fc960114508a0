// common.h - shared declarations of the SPPC HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <stdexcept>
#include <string>

namespace sppc {

// Error carried from the host engine to the C ABI boundary.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// A failed HIP call throws SPPC_E_HIP, or SPPC_E_NOMEM when memory (or the caller's workspace) ran out.
#define SPPC_HIP(call)                                                                 \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::sppc::Error(e_ == hipErrorOutOfMemory ? 3 : 2,                           \
                          std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

#define SPPC_LAUNCH_CHECK() SPPC_HIP(hipGetLastError())

constexpr int WAVE = 64;

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- memory (memory.hip)

// Device memory: from the active caller workspace (WsScope) when there is one, else from the
// library (hipMalloc, or the optional cache of freed blocks).  dev_alloc_tmp marks a temporary of a
// setup phase (taken from the workspace's top end).  A block may be given back only once the stream
// that last used it has been synchronised.  Pinned host memory always comes from the library.
struct Workspace;
Workspace* ws_create(void* base, size_t bytes);
void ws_destroy(Workspace* w);
size_t ws_peak(const Workspace* w);
struct WsScope {
  Workspace* prev;
  explicit WsScope(Workspace* w);
  ~WsScope();
  WsScope(const WsScope&) = delete;
  WsScope& operator=(const WsScope&) = delete;
};
hipError_t dev_alloc(void** p, size_t bytes);
hipError_t dev_alloc_tmp(void** p, size_t bytes);
void dev_free(void* p);
hipError_t pinned_alloc(void** p, size_t bytes);
void pinned_free(void* p);
template <class T>
inline hipError_t dev_malloc(T** p, size_t bytes) {
  return dev_alloc((void**)p, bytes);
}
template <class T>
inline hipError_t dev_malloc_tmp(T** p, size_t bytes) {
  return dev_alloc_tmp((void**)p, bytes);
}
// bytes one device array of `bytes` takes in a workspace (256-byte granules)
inline size_t ws_bytes(size_t bytes) { return (std::max<size_t>(bytes, 1) + 255) / 256 * 256; }

// ---------------------------------------------------------------- sparse (kernels_sparse.hip)

// Full symmetric CSR on the device (both triangles, columns ascending in each row).
// Row-block x column-panel copy of H for the block product with large n (n < 2^24).  Rows are
// cut into blocks of RB = 256 (one workgroup each) and columns into panels of PW (a panel of X
// is small enough to stay in one XCD's L2).  The off-diagonal entries of a block form one
// stream ordered by (panel, row, column), padded with zero entries to a multiple of 8; an
// entry is a word (column | row-in-block << 24) and a value.  The diagonal is kept apart (dg).
struct PanelH {
  int64_t n = 0;
  int nblocks = 0;
  int RB = 0;                 // rows per block
  int P = 0;                  // panels
  int PW = 0;                 // columns per panel (<= 65536)
  int64_t* bstart = nullptr;  // [nblocks + 1]: first entry of each block (multiples of 8)
  int32_t* bcount = nullptr;  // [nblocks]: entries of each block, without the padding
  uint32_t* ent = nullptr;    // column | row-in-block << 24
  float* val32 = nullptr;
  double* val64 = nullptr;
  double* dg = nullptr;       // [n] diagonal of H
  void* xpad = nullptr;       // [n x 16] doubles: X copied to row stride B when needed
};

struct DevCSR {
  int64_t n = 0;
  int64_t nnz = 0;
  int64_t* rp = nullptr;       // [n+1] row begin
  int64_t* rend = nullptr;     // [n] optional row end (sub-matrix views); nullptr = rp[i+1]
  int32_t* col = nullptr;
  double* val64 = nullptr;     // float64 values (nullptr when val32 is exact and enough)
  float* val32 = nullptr;      // float32 values
  const PanelH* panel = nullptr;  // optional panel copy used by the plain products (b <= 16)
};

// Setup: build the full CSR from the upper triangle.  Returns nnz of the full matrix.
void build_full_csr(int64_t n, int64_t nnz_up, const int64_t* up_rp, const int32_t* up_col,
                    const void* up_val, int val_is_f32, DevCSR& out, int* d_flags,
                    bool want64, bool want32, bool& exact32, hipStream_t s);
// The caller's upper triangle (diagonal included, columns ascending), borrowed.
struct UpperCSR {
  int64_t n = 0;
  const int64_t* rp = nullptr;
  const int32_t* col = nullptr;
  const float* val32 = nullptr;   // one of the two
  const double* val64 = nullptr;
};
// Y[n x b] (ldy) = H X from the upper triangle alone: the transposed half by float64 atomic adds
// (Y is zeroed first); X float32 (xf32) or float64.
void spmm_upper(const UpperCSR& U, const void* X, bool xf32, int64_t ldx, double* Y, int64_t ldy, int b,
                hipStream_t s);
// Row ends of the leading n0 x n0 block (columns < n0) of the full CSR.
void build_block_view(const DevCSR& full, int64_t n0, int64_t* rend, hipStream_t s);
// rend[i] = end of the entries of row i with column < c0, for rows i < nrows of the full CSR.
void row_ends_below(const DevCSR& full, int64_t nrows, int64_t c0, int64_t* rend, hipStream_t s);
// Panel copy of a full CSR (ascending columns per row); values as stored in the CSR.
// Device memory is allocated with hipMalloc and owned by the caller (release_panel).
void build_panel(const DevCSR& H, int PW, PanelH& out, hipStream_t s);
void release_panel(PanelH& p);
// Workspace bytes of the builders: arrays kept by the context and setup temporaries.
struct BuildBytes {
  size_t persist = 0, temp = 0;
};
BuildBytes full_csr_bytes(int64_t n, int64_t nnz_up, bool want64, bool want32);
BuildBytes panel_bytes(int64_t n, int64_t nnz_full, bool v64, bool v32);
BuildBytes view_bytes(int64_t n0, int64_t nnz0, bool v64, bool v32);
// out[0..n] = exclusive prefix sums of a[0..n) (out[n] = total); bsum holds cdiv(n, 1024) + 1.
void scan_exclusive(int64_t n, const int32_t* a, int64_t* out, int64_t* bsum, hipStream_t s);
// Contiguous copy of a block view (rows [0, n0), columns < n0); hipMalloc'd arrays.
void compact_view(const DevCSR& V, DevCSR& out, hipStream_t s);
// diag(H) from the full CSR.
void extract_diag(const DevCSR& H, double* diag, hipStream_t s);

// Y[n x b] = H X (- shift_c X[:,c] when shift != nullptr), row-major with leading dims.
// X float64 with float64 or float32-exact values.
// stage (optional, stage_bytes long): where the panel kernels put the padded copy of X when the
// caller's X is not in their layout (default: the panel's own buffer).
void spmm_f64(const DevCSR& H, const double* X, int64_t ldx, double* Y, int64_t ldy, int b,
              const double* shift, hipStream_t s, void* stage = nullptr, size_t stage_bytes = 0);
// Chebyshev filter step: Y = ea * (H X - ec X) + eb * Zo   (Zo must be non-null)
void spmm_cheb(const DevCSR& H, const double* X, int64_t ldx, double* Y, int64_t ldy, int b, double ea,
               double ec, double eb, const double* Zo, int64_t ldz, hipStream_t s);
// max_i (h_ii + sum_{j != i} |h_ij|) into *out (device); tmp holds n doubles
void gershgorin_upper(const DevCSR& H, double* tmp, double* out, hipStream_t s);
// Mixed: float32 values and float32 X, float32 products accumulated in float64.  With diag
// (the diagonal of H) and X64 (float64 X) the diagonal entries are skipped in the float32 sum and
// diag * X64 is added in float64: the diagonal product is the largest term of a row.
void spmm_f32(const DevCSR& H, const float* X, int64_t ldx, double* Y, int64_t ldy, int b,
              const double* shift, hipStream_t s, const double* diag = nullptr, const double* X64 = nullptr,
              int64_t ldx64 = 0, void* stage = nullptr, size_t stage_bytes = 0);
// Device address (on the current device) and size of the library's static scratch array used by
// the allocation-free block product; looked up once per device.
void* noalloc_scratch(size_t* bytes);

// ---------------------------------------------------------------- dense (kernels_dense.hip)

// C[m x b] (ldc) = beta*C + alpha * A[n x m]^T B[n x b]   (A lda, B ldb, row-major)
// work: partial sums, at least gemm_tn_work(n, m, b) doubles.
int64_t gemm_tn_work(int64_t n, int m, int b);
void gemm_tn(int64_t n, int m, int b, const double* A, int64_t lda, const double* B, int64_t ldb,
             double* C, int64_t ldc, double alpha, double beta, double* work, hipStream_t s);
// Y[n x b] (ldy) = beta*Y + alpha * A[n x m] C[m x b]   (C row-major, ldc)
void gemm_nn(int64_t n, int m, int b, const double* A, int64_t lda, const double* C, int64_t ldc,
             double* Y, int64_t ldy, double alpha, double beta, hipStream_t s);
// One pass over A for two products: Y1[n x b1] (ldy1) = beta1*Y1 + A C[:, 0:b1] and
// Y2[n x b2] (ldy2) = beta2*Y2 + A C[:, b1:b1+b2], with b1 + b2 <= 32 (C row-major, ldc).
void gemm_nn2(int64_t n, int m, int b1, int b2, const double* A, int64_t lda, const double* C, int64_t ldc,
              double* Y1, int64_t ldy1, double beta1, double* Y2, int64_t ldy2, double beta2, hipStream_t s);
// Same with float32 output (mixed-precision staging of SpMM inputs).
void copy_to_f32(int64_t n, int b, const double* X, int64_t ldx, float* Y, int64_t ldy, hipStream_t s);
// Y[r, c] = X[r, c] for a sub-block (row-major)
void copy_block(int64_t n, int b, const double* X, int64_t ldx, double* Y, int64_t ldy, hipStream_t s);
// Y1[:, c] = X1[:, c], Y2[:, c] = X2[:, c] for the columns c (< b <= 32) whose bit is set in mask,
// one pass for all of them (leading dimension ld for the four arrays).
void copy_cols2(int64_t n, int b, uint32_t mask, const double* X1, double* Y1, const double* X2, double* Y2,
                int64_t ld, hipStream_t s);
void fill_zero(int64_t count, double* p, hipStream_t s);
// R = HZ - Z diag(theta) and partial sums of squares of R's columns into out[b] (sum of squares).
void residual_block(int64_t n, int b, const double* Z, int64_t ldz, const double* HZ, int64_t ldhz,
                    const double* theta, double* R, int64_t ldr, double* sumsq, double* work,
                    hipStream_t s);
// sum of squares of each column of X: out[b]
void colsumsq(int64_t n, int b, const double* X, int64_t ldx, double* out, double* work, hipStream_t s);
// Psi[r, c] = W[r, c] / E0[c] for r in [r0, n)   (complement rows, eq. sm_first)
void complement_rows(int64_t r0, int64_t n, int b, const double* W, int64_t ldw, const double* E0,
                     double* Psi, int64_t ldp, hipStream_t s);
// Y[r, c] = a*X[r, c] + Y[r, c]*beta
void axpby_block(int64_t n, int b, double a, const double* X, int64_t ldx, double beta, double* Y,
                 int64_t ldy, hipStream_t s);
// Jacobi continuation block for the active pairs: T[:, a] = R[:, idx[a]] / clamp(d - theta[idx[a]])
void jacobi_block(int64_t n, int na, const int* idx, const double* R, int64_t ldr, const double* diag,
                  const double* theta, double* T, int64_t ldt, hipStream_t s);
// T[:, a] = -(T[:, a] - Z[:, idx[a]] * dots[a])
void project_out_block(int64_t n, int na, const int* idx, const double* Z, int64_t ldz,
                       const double* dots, double* T, int64_t ldt, hipStream_t s);
// dots[a] = Z[:, idx[a]]^T T[:, a]
void paired_dots(int64_t n, int na, const int* idx, const double* Z, int64_t ldz, const double* T,
                 int64_t ldt, double* dots, double* work, hipStream_t s);

// ---------------------------------------------------------------- small (kernels_small.hip)

// Lowest nwant eigenpairs of symmetric S (m x m, row-major lds): w[nwant] ascending,
// V row-major m x nwant (ldv).  Single workgroup.  scratch >= eig_scratch(m, nwant) doubles.
int64_t eig_scratch(int m, int nwant);
void sym_eig_lowest(int m, int nwant, const double* S, int64_t lds, double* w, double* V,
                    int64_t ldv, double* scratch, hipStream_t s);

// Orthonormalisation helpers (block of width b <= 32):
// Step 1: from G = Phi^T Phi (b x b) and the squared norms of the original columns, drop
// columns with sin(angle) <= tau, pivoted Cholesky of the rest; with rel > 0 a column whose
// Schur complement falls to rel times its own diagonal of G is dropped as dependent on the
// pivots taken (0 keeps it while it exceeds tau^2 times its original squared norm).  Outputs:
//   M[b x b] (row-major, columns >= kept are zero) with Phi1 = Phi M, R1[b x b] (Phi[:,kept] =
//   Phi1 R1 restricted), perm/kept count in info[0..], angles[b].
void cholqr_first(int b, const double* G, const double* psi_sumsq, double tau, double rel, double* M,
                  double* Rfac, double* angles, int* info, hipStream_t s);
// Step 2: G2 = Phi1^T Phi1 (kept x kept) -> M2 = R2^-1 and Rtot = R2 * R1 (kept x b in the
// original column order); info[1] := 1 if the Cholesky failed.
void cholqr_second(int b, const double* G2, double* M2, double* Rfac, int* info, hipStream_t s);

// T bookkeeping
void t_extend(int m_old, int kn, const double* X, int64_t ldx, double* T, int64_t ldt, hipStream_t s);
void t_set_diag(int m, const double* theta, double* T, int64_t ldt, hipStream_t s);
void t_from_full(int m, const double* X, int64_t ldx, double* T, int64_t ldt, hipStream_t s);
// Coefficients of the raw correction in the basis: G[(m_old + kn) x k] = [C; Rtot]
void store_coef(int m_old, int kn, int k, const double* C, int64_t ldc, const double* Rtot,
                double* G, int64_t ldg, hipStream_t s);
// A = G^(p-1), B = sum_{l=0}^{p-2} G^(l) diag(E^(p-l)); also E^(p) from T (see kernels_small.hip)
void build_correction_coefs(int p, int k, int m, const double* Ghist, int64_t gstride, int64_t ldg,
                            const int* m_hist, double* Etab, const double* T, int64_t ldt,
                            const double* E0, double* A, double* B, hipStream_t s);
// x1 add-back coefficients for the deflated small solves
// out[j][a] = c[j][a] / (w[j] - theta[a]) (theta device, na values): deflated terms of the
// theta-shifted small-space solve
void deflate_shift(int D, int na, const double* w, const double* theta, const double* c, int64_t ldc, double* out,
                   int64_t ldo, hipStream_t s);
// shift (device, [k], optional): sigma_kk in place of E_kk^(0) = w[kk] in the denominators
void deflate_coefs(int D, int k, const double* w, const double* shift, const double* c, int64_t ldc, double* out,
                   int64_t ldo, hipStream_t s);
// element-wise small: C = C1 + C2 (m x b)
void add_small(int count, const double* a, double* b, hipStream_t s);
// sign fix: make the largest-magnitude entry of each column positive (n x b, row-major)
void sign_fix_columns(int64_t n, int b, double* X, int64_t ldx, double* work, hipStream_t s);
// argmin selection of the nsel smallest entries of d[0..n) (ties by index): idx[nsel]
void select_smallest(int64_t n, const double* d, int nsel, int* idx, hipStream_t s);
// X[r, c] = (r == idx[c])
void unit_block(int64_t n, int b, const int* idx, double* X, int64_t ldx, hipStream_t s);

// ---------------------------------------------------------------- small-space solver (kernels_cg.hip)
int64_t cg_work_doubles(int64_t n0);
// Row bounds of the CG iteration blocks (once per H0hat); rowb has 257 entries, tmp 2 (n0 + 2)
// doubles.
void cg_prepare(const DevCSR& H0, int64_t n0, int64_t* rowb, double* tmp, hipStream_t s);
// Deflated CG for the k small-space systems (b in r on entry, solution in x); ccoef = Ps^T b.
// Products in float64 (float32-stored values are widened).  host_flag: two ints of pinned memory.
int cg_solve(const DevCSR& H0, int64_t n0, int k, int D, const double* shift, const double* Ps,
             const int64_t* rowb, double* x, double* r, double* work, double* ccoef, int maxit, double tol,
             int* host_flag, hipStream_t s);
// ---------------------------------------------------------------- RMM-DIIS (kernels_rmmdiis.hip)
int diis_max_depth();
// alpha[a][0..L) = Pulay's DIIS coefficients of pair a from its residual Gram matrix A[a] (D x D)
void diis_coefficients(int k, int L, int D, const double* A, double* alpha, hipStream_t s);
// xb[:, a] = sum_l alpha[a][l] Xh_l[:, a] (slots of n x k), the same for H x
void diis_combine(int64_t n, int k, int L, int D, const double* alpha, const double* Xh, const double* HXh,
                  double* xb, double* hxb, hipStream_t s);
// X[:, a], HX[:, a] divided by sqrt(ss[a])
void columns_to_unit(int64_t n, int k, const double* ss, double* X, double* HX, hipStream_t s);
// Xn = xb + lam t, HXn = hxb + lam ht with lam[a] = -rd[a] / uu[a]
void min_residual_step(int64_t n, int k, const double* rd, const double* uu, const double* xb, const double* hxb,
                       const double* t, const double* ht, double* Xn, double* HXn, hipStream_t s);
// A[a][i][l] = A[a][l][i] = g[a]
void gram_set(int k, int D, int i, int l, const double* g, double* A, hipStream_t s);
// out[c] = X[:, c]^T Y[:, c]
void coldots(int64_t n, int b, const double* X, int64_t ldx, const double* Y, int64_t ldy, double* out,
             double* work, hipStream_t s);
void fill_block_zero(int64_t n, int b, double* Y, int64_t ldy, hipStream_t s);
// Y[:, a] = X[:, idx[a]]   /   Y[:, idx[a]] = alpha X[:, a] (idx[a] < 0 skipped)
void gather_cols(int64_t n, int S, const int* idx, const double* X, int64_t ldx, double* Y, int64_t ldy,
                 hipStream_t s);
void scatter_cols(int64_t n, int S, const int* idx, const double* X, int64_t ldx, double* Y, int64_t ldy,
                  double alpha, hipStream_t s);

// ---------------------------------------------------------------- learned preconditioner (kernels_mpnn.hip)
int mpnn_nparam();
void mpnn_prepare(const DevCSR& H, const double* diag, const int64_t* level_off_dev, int L, int nsmall, double* lev,
                  double* Ad, double* A1, double* Al, double* tmp, hipStream_t s);
int64_t mpnn_work_doubles(int64_t n, int S);
// Optional basis for the output projection t - Q (Q^T t) (training against the part of the
// exact eigenvector outside the basis); work holds mpnn_basis_work_doubles(n, m) doubles.
struct MpnnBasis {
  const double* Q;
  int64_t ldq;
  int m;
  double* work;
};
int64_t mpnn_basis_work_doubles(int64_t n, int m);
template <typename T>
void mpnn_run(const DevCSR& H, const double* diag, const double* lev, const double* Ad, const double* A1,
              const double* Al, const T* w, int S, const double* R, int64_t ldr, const double* X, int64_t ldx,
              const double* theta_dev, const double* E, double* T_out, double* grad_out, double* loss_dev,
              double* work, const MpnnBasis* basis, hipStream_t s, bool project = true);
void mpnn_adam(float* w, float* m, float* v, const double* g, float lr, int step, float* wq, hipStream_t s);
void mpnn_round_bf16(int cnt, const float* w, float* wq, double* wd, hipStream_t s);
void mpnn_target(int64_t n, int S, const MpnnBasis& B, const double* Psi, double* E, hipStream_t s);

}  // namespace sppc
