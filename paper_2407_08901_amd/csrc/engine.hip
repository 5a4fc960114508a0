// engine.hip - host driver of SPPC on one GPU and the C ABI (include/sppc.h).
//
// Step structure (Alg. 2):
//   setup      device format of H, H0hat view, zeroth order (eq. EP_small), p = 0
//   correct    E^(p), Psi^(p) (eq. exp_seq, eq. exp_seq2) from the stored basis:
//              H Psi^(p-1) = HQ G^(p-1) (eq. HPsip, raw corrections kept as basis
//              coefficients), V Psi = H Psi - H0 Psi (eq. avoid_SpMV2), complement rows by
//              eq. sm_first, small-space rows by a deflated CG for eq. sm_lin_proj
//   append+RR  block Gram-Schmidt twice, Cholesky-QR twice (eqs. blkGS, QR, Qp), one block
//              product with H, new rows/columns of T (eq. proj), lowest eigenpairs of T,
//              residual norms (eq. rrn)
// After p_switch SPPC steps (or earlier, once SPPC stagnates, with auto_switch) either the basis
// keeps growing with preconditioned residual blocks (Davidson continuation) or each pair is
// refined on its own by RMM-DIIS (the hybrid of Sec. V-VI).  A final float64 check follows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "common.h"
#include "sppc.h"

namespace sppc {

constexpr int KB = 32;   // widest block handled by one product / orthonormalisation
constexpr int NWMAX = 64;

// Device arrays of a context (or, with temp, of one setup phase).  A counting arena allocates
// nothing: it adds up the workspace bytes its requests would take (the size query runs the same
// allocation code as the setup).
struct Arena {
  std::vector<void*> ptrs;
  bool temp = false;
  bool counting = false;
  size_t counted = 0;
  template <class T>
  T* alloc(size_t count) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (counting) {
      counted += ws_bytes(bytes);
      return nullptr;
    }
    hipError_t e = temp ? dev_alloc_tmp(&p, bytes) : dev_alloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(SPPC_E_NOMEM, "allocation of " + std::to_string(bytes) + " bytes of device memory failed" +
                                    std::string(" (device memory, or the caller's workspace, is exhausted)"));
    }
    ptrs.push_back(p);
    return (T*)p;
  }
  void release() {
    for (void* p : ptrs) dev_free(p);
    ptrs.clear();
  }
  ~Arena() { release(); }
};

struct Basis {
  int64_t n = 0;
  int ldq = 0;   // columns allocated (row stride of Q and HQ)
  int m = 0;     // columns in use
  double* Q = nullptr;
  double* HQ = nullptr;
  double* T = nullptr;  // ldq x ldq
};

enum Cat { C_SPMM = 0, C_SMALL, C_ORTHO, C_RR, C_H0, C_NCAT };

struct EventTimer {
  std::vector<hipEvent_t> pool;
  struct Rec { hipEvent_t a, b; int cat; };
  std::vector<Rec> open;
  hipStream_t s = nullptr;
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e;
    SPPC_HIP(hipEventCreate(&e));
    return e;
  }
  size_t begin(int cat) {
    Rec r{get(), get(), cat};
    SPPC_HIP(hipEventRecord(r.a, s));
    open.push_back(r);
    return open.size() - 1;
  }
  void end(size_t i) { SPPC_HIP(hipEventRecord(open[i].b, s)); }
  void collect(double* acc) {  // stream must be synchronised
    for (auto& r : open) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) acc[r.cat] += ms;
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    open.clear();
  }
  ~EventTimer() {
    for (auto& r : open) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace sppc

using namespace sppc;

struct sppc_ctx {
  hipStream_t s = nullptr;
  sppc_opts o{};
  int64_t n = 0, n0 = 0;
  int k = 0, D = 0;
  std::vector<int64_t> loff;
  Arena arena;
  DevCSR H, H0;
  PanelH panel;
  double* diag = nullptr;
  bool exact32 = false;
  double* E0 = nullptr;      // [D]
  double* Psihat = nullptr;  // n0 x D
  std::vector<double> E0h;
  Basis B;
  double *Psi = nullptr, *Phi = nullptr, *Wb = nullptr, *Z = nullptr, *HZ = nullptr, *R = nullptr;
  float* X32 = nullptr;
  double *C1 = nullptr, *C2 = nullptr, *Gm = nullptr, *M1 = nullptr, *M2 = nullptr, *Rt = nullptr;
  double *Vrr = nullptr, *theta = nullptr, *sumsq = nullptr, *psi2 = nullptr, *angles = nullptr;
  double *Xt = nullptr, *Acoef = nullptr, *Bcoef = nullptr, *dots = nullptr, *work = nullptr;
  // The next perturbative step's W = H Psi^(p-1) - sum E Psi (in Wb) and its coefficients (Acoef,
  // Bcoef) formed in the Rayleigh-Ritz passes of the step before: valid for step w_next while the
  // basis holds w_m columns.  Cq = [V | -B] and Ch = [V | A] are the right-hand sides of those passes.
  double *Cq = nullptr, *Ch = nullptr;
  int w_next = -1, w_m = -1;
  double* eigscr = nullptr;
  int *info = nullptr, *idx = nullptr, *mhist_dev = nullptr;
  double *cx = nullptr, *cr = nullptr,
         *ccoef = nullptr, *ctmp = nullptr, *cgpart = nullptr;
  int64_t* cg_rowb = nullptr;
  double* cshift = nullptr;  // shifts of the theta-shifted small-space solves
  int cg_blocks = 1;
  double* Ghist = nullptr;
  int64_t gstride = 0;
  int maxhist = 0;
  double* Etab = nullptr;
  std::vector<int> mhist;
  int p = 0;
  bool restarted = false;
  bool refining = false;  // float64 residual refinement after a mixed-precision solve
  bool f64_products = false;  // mixed precision: the block products have switched to float64
  int pend_b = 0, pend_kind = -1;
  int nw_last = 0;  // width of Z/HZ/R from the last Rayleigh-Ritz
  // RMM-DIIS state (allocated at its first use): history slots of x, H x, R (D x n x k), the
  // residual Gram matrices (k x D x D), coefficients, work blocks and column scalars
  double *rd_Xh = nullptr, *rd_HXh = nullptr, *rd_Rh = nullptr, *rd_A = nullptr, *rd_al = nullptr;
  double *rd_xb = nullptr, *rd_hxb = nullptr, *rd_rb = nullptr, *rd_t = nullptr, *rd_ht = nullptr, *rd_u = nullptr;
  double* rd_sc = nullptr;
  std::vector<double> theta_h, rrn_h, angles_h;
  int last_added = 0;
  // learned preconditioner
  bool mp_ready = false, mp_have_w = false, mp_invalid = false;
  int64_t* loff_dev = nullptr;
  double *mp_lev = nullptr, *mp_Ad = nullptr, *mp_A1 = nullptr, *mp_Al = nullptr, *mp_work = nullptr;
  double *mp_sel = nullptr, *mp_th = nullptr, *mp_grad = nullptr, *mp_loss = nullptr, *mp_wd = nullptr;
  float *mp_w = nullptr, *mp_wq = nullptr;
  int mp_S = 0;
  double* mp_bwork = nullptr;  // basis-projection workspace (training)
  int64_t mp_bwork_cap = 0;
  std::vector<int> mp_fallback;     // per pair: 1 = use the diagonal step
  std::vector<double> mp_prev_rrn;  // residual when the learned step was last used (0 = not used)
  sppc_stats st{};
  std::string err;
  double* pin = nullptr;  // pinned host staging
  int* pin_i = nullptr;
  EventTimer tm;
  double tacc[C_NCAT] = {0, 0, 0, 0, 0};
  int64_t nnz_up = 0;  // stored upper-triangle entries of the input
  int nsmall = 0;      // leading levels that form the small space
  Workspace* ws = nullptr;  // the caller's workspace (nullptr: library-allocated memory)
};

namespace sppc {
namespace {

thread_local std::string g_setup_err;

inline double* Gh(sppc_ctx* c, int l) { return c->Ghist + (int64_t)l * c->gstride; }

// Algorithmic bytes of one block product with H: the upper triangle once (values as the kernel
// reads them: float32 when stored losslessly or in mixed mode, int32 columns), the row pointers,
// X read (in mixed mode float32 X for the sum and float64 X for the diagonal) and Y written.
double spmm_alg_bytes(const sppc_ctx* c, int b, bool xf32) {
  const double vb = (xf32 || !c->H.val64) ? 4.0 : 8.0;
  const double xb = xf32 ? 4.0 + 8.0 : 8.0;  // mixed: float32 X gathered, float64 X for the diagonal
  return (double)c->nnz_up * (vb + 4.0) + (double)(c->n + 1) * 8.0 + (double)c->n * b * (xb + 8.0);
}

// Y = A X on the operator of the basis: the whole H (mixed or float64) or H0hat.  Products
// with H are counted and timed (kernel only) in the statistics.
struct Op {
  sppc_ctx* c;
  const DevCSR* A;
  bool mixed;
  bool isH;
  void operator()(const double* X, int64_t ldx, double* Y, int64_t ldy, int b, hipStream_t s) const;
};

void sync(sppc_ctx* c) { SPPC_HIP(hipStreamSynchronize(c->s)); }

void Op::operator()(const double* X, int64_t ldx, double* Y, int64_t ldy, int b, hipStream_t s) const {
  if (mixed) copy_to_f32(A->n, b, X, ldx, c->X32, b, s);
  const size_t t0 = c->tm.begin(isH ? C_SPMM : C_H0);
  if (mixed)
    spmm_f32(*A, c->X32, b, Y, ldy, b, nullptr, s, isH ? c->diag : nullptr, isH ? X : nullptr, ldx);
  else
    spmm_f64(*A, X, ldx, Y, ldy, b, nullptr, s);
  c->tm.end(t0);
  if (isH) {
    c->st.n_spmv += b;
    c->st.spmm_calls += 1;
    c->st.spmm_cols += b;
    c->st.spmm_alg_bytes += spmm_alg_bytes(c, b, mixed);
  }
}

void to_host(sppc_ctx* c, const double* dev, int count, double* host) {
  SPPC_HIP(hipMemcpyAsync(c->pin, dev, sizeof(double) * count, hipMemcpyDeviceToHost, c->s));
  sync(c);
  memcpy(host, c->pin, sizeof(double) * count);
}

// Rayleigh-Ritz on the basis: nw lowest pairs, Ritz vectors Z, H Z, residual R, norms.
// with_next (nw = k, main basis): the passes over Q and H Q that form Z = Q V and H Z = H Q V also
// form the next perturbative step's W = H Q A - Q B from the coefficients already in Acoef, Bcoef.
void rayleigh_ritz(sppc_ctx* c, Basis& b, int nw, bool with_next = false) {
  hipStream_t s = c->s;
  const size_t t0 = c->tm.begin(C_RR);
  sym_eig_lowest(b.m, nw, b.T, b.ldq, c->theta, c->Vrr, nw, c->eigscr, s);
  if (with_next) {
    const int k = c->k, w2 = nw + k;
    copy_block(b.m, nw, c->Vrr, nw, c->Cq, w2, s);
    copy_block(b.m, nw, c->Vrr, nw, c->Ch, w2, s);
    axpby_block(b.m, k, -1.0, c->Bcoef, k, 0.0, c->Cq + nw, w2, s);
    copy_block(b.m, k, c->Acoef, k, c->Ch + nw, w2, s);
    gemm_nn2(b.n, b.m, nw, k, b.Q, b.ldq, c->Cq, w2, c->Z, nw, 0.0, c->Wb, k, 0.0, s);
    gemm_nn2(b.n, b.m, nw, k, b.HQ, b.ldq, c->Ch, w2, c->HZ, nw, 0.0, c->Wb, k, 1.0, s);
  } else {
    gemm_nn(b.n, b.m, nw, b.Q, b.ldq, c->Vrr, nw, c->Z, nw, 1.0, 0.0, s);
    gemm_nn(b.n, b.m, nw, b.HQ, b.ldq, c->Vrr, nw, c->HZ, nw, 1.0, 0.0, s);
  }
  residual_block(b.n, nw, c->Z, nw, c->HZ, nw, c->theta, c->R, nw, c->sumsq, c->work, s);
  c->tm.end(t0);
  SPPC_HIP(hipMemcpyAsync(c->pin, c->theta, sizeof(double) * nw, hipMemcpyDeviceToHost, s));
  SPPC_HIP(hipMemcpyAsync(c->pin + NWMAX, c->sumsq, sizeof(double) * nw, hipMemcpyDeviceToHost, s));
  sync(c);
  c->tm.collect(c->tacc);
  c->theta_h.assign(c->pin, c->pin + nw);
  c->rrn_h.resize(nw);
  for (int i = 0; i < nw; ++i) {
    const double th = c->theta_h[i];
    const double rn = std::sqrt(std::max(c->pin[NWMAX + i], 0.0));
    c->rrn_h[i] = rn / (std::fabs(th) > 1e-300 ? std::fabs(th) : 1.0);
    if (!std::isfinite(th) || !std::isfinite(rn)) throw Error(SPPC_E_NAN, "NaN/Inf in the Ritz pairs");
  }
  c->nw_last = nw;
}

// Block Gram-Schmidt (twice) + Cholesky-QR (twice) of the n x bw block P against the basis,
// append the kept columns, multiply them by the operator and extend T.  Returns the number
// of appended columns.  If coef_slot >= 0 the coefficients [C; R] of P in the new basis are
// stored in the history slot (P = Q C + q R).
// HP (optional): H P already known; H Q_new then follows by the same transformation as Q_new
// instead of a product with H.
int ortho_append(sppc_ctx* c, Basis& b, const double* P, int bw, const Op& op, int coef_slot,
                 const double* HP = nullptr) {
  hipStream_t s = c->s;
  const int64_t n = b.n;
  const int m = b.m;
  if (bw < 1 || bw > KB) throw Error(SPPC_E_ARG, "block width must be 1..32");
  c->w_next = -1;  // Wb is scratch here
  size_t t0 = c->tm.begin(C_ORTHO);
  colsumsq(n, bw, P, bw, c->psi2, c->work, s);
  copy_block(n, bw, P, bw, c->Phi, bw, s);
  if (m > 0) {
    gemm_tn(n, m, bw, b.Q, b.ldq, c->Phi, bw, c->C1, bw, 1.0, 0.0, c->work, s);
    gemm_nn(n, m, bw, b.Q, b.ldq, c->C1, bw, c->Phi, bw, -1.0, 1.0, s);
    gemm_tn(n, m, bw, b.Q, b.ldq, c->Phi, bw, c->C2, bw, 1.0, 0.0, c->work, s);
    gemm_nn(n, m, bw, b.Q, b.ldq, c->C2, bw, c->Phi, bw, -1.0, 1.0, s);
    add_small(m * bw, c->C2, c->C1, s);
  }
  gemm_tn(n, bw, bw, c->Phi, bw, c->Phi, bw, c->Gm, bw, 1.0, 0.0, c->work, s);
  // appended to a basis, a column that depends on the block's own pivots (its Schur complement at
  // the rounding of the Gram matrix, below 1e-12 of its Gram diagonal: a remaining part of 1e-6 of
  // its norm) is dropped, or it would be normalised from rounding into a direction that is not
  // orthogonal to Q.  An empty basis keeps such columns (they are then random directions of the
  // block, as in the filtered subspace iteration of the zeroth order)
  cholqr_first(bw, c->Gm, c->psi2, c->o.tau_drop, m > 0 ? 1e-12 : 0.0, c->M1, c->Rt, c->angles, c->info, s);
  c->tm.end(t0);
  SPPC_HIP(hipMemcpyAsync(c->pin_i, c->info, sizeof(int) * 2, hipMemcpyDeviceToHost, s));
  SPPC_HIP(hipMemcpyAsync(c->pin, c->angles, sizeof(double) * bw, hipMemcpyDeviceToHost, s));
  sync(c);
  // never more basis columns than rows
  const int kept = std::min(c->pin_i[0], std::max(0, (int)std::min<int64_t>(b.ldq, n) - m));
  c->angles_h.assign(c->pin, c->pin + bw);
  if (kept > 0) {
    t0 = c->tm.begin(C_ORTHO);
    gemm_nn(n, bw, kept, c->Phi, bw, c->M1, bw, c->Wb, kept, 1.0, 0.0, s);
    gemm_tn(n, kept, kept, c->Wb, kept, c->Wb, kept, c->Gm, bw, 1.0, 0.0, c->work, s);
    cholqr_second(bw, c->Gm, c->M2, c->Rt, c->info, s);
    gemm_nn(n, kept, kept, c->Wb, kept, c->M2, bw, b.Q + m, b.ldq, 1.0, 0.0, s);
    if (HP) {
      // H Phi is H P minus the projections (m = 0 here: H P itself), then the two Cholesky factors
      if (m > 0) throw Error(SPPC_E_ARG, "ortho_append: H P only for an empty basis");
      gemm_nn(n, bw, kept, HP, bw, c->M1, bw, c->Psi, kept, 1.0, 0.0, s);
      gemm_nn(n, kept, kept, c->Psi, kept, c->M2, bw, b.HQ + m, b.ldq, 1.0, 0.0, s);
    }
    c->tm.end(t0);
    if (!HP) op(b.Q + m, b.ldq, b.HQ + m, b.ldq, kept, s);
    t0 = c->tm.begin(C_RR);
    gemm_tn(n, m + kept, kept, b.Q, b.ldq, b.HQ + m, b.ldq, c->Xt, kept, 1.0, 0.0, c->work, s);
    if (op.mixed && &b == &c->B && !c->restarted && m >= c->k) {
      // float32 products: the rows of T against Psi^(0) (the first k columns, whose H Psi^(0)
      // is a float64 product) are taken as (H Psi^(0))^T Q_new instead.  They are all that
      // E^(p) reads (eq. exp_seq with eq. avoid_SpMV2), and the perturbative orders are far
      // smaller than the float32 errors of H Q_new.
      gemm_tn(n, c->k, kept, b.HQ, b.ldq, b.Q + m, b.ldq, c->Xt, kept, 1.0, 0.0, c->work, s);
    }
    t_extend(m, kept, c->Xt, kept, b.T, b.ldq, s);
    c->tm.end(t0);
  }
  if (coef_slot >= 0) store_coef(m, kept, c->k, c->C1, bw, c->Rt, Gh(c, coef_slot), c->k, s);
  b.m = m + kept;
  return kept;
}

void restart_basis(sppc_ctx* c, Basis& b, int keep) {
  // basis <- the current Ritz vectors (Z, H Z of width nw_last), T <- diag(theta)
  hipStream_t s = c->s;
  copy_block(b.n, keep, c->Z, c->nw_last, b.Q, b.ldq, s);
  copy_block(b.n, keep, c->HZ, c->nw_last, b.HQ, b.ldq, s);
  t_set_diag(keep, c->theta, b.T, b.ldq, s);
  b.m = keep;
}

// Preconditioned residual block for the listed Ritz pairs: t = -(I - z z^T) (d - theta)^-1 r.
void jacobi_expansion(sppc_ctx* c, int64_t n, const double* diag, const std::vector<int>& act, int nw) {
  hipStream_t s = c->s;
  const int na = (int)act.size();
  for (int a = 0; a < na; ++a) c->pin_i[8 + a] = act[a];
  SPPC_HIP(hipMemcpyAsync(c->idx, c->pin_i + 8, sizeof(int) * na, hipMemcpyHostToDevice, s));
  jacobi_block(n, na, c->idx, c->R, nw, diag, c->theta, c->Psi, na, s);
  paired_dots(n, na, c->idx, c->Z, nw, c->Psi, na, c->dots, c->work, s);
  project_out_block(n, na, c->idx, c->Z, nw, c->dots, c->Psi, na, s);
  sync(c);  // pin_i is reused by later steps
}

// The n_deflate lowest eigenpairs of H0hat by Chebyshev-filtered subspace iteration: a block
// of nb >= n_deflate vectors (started at unit vectors on the smallest diagonal entries) is
// repeatedly multiplied by a Chebyshev polynomial of H0hat that damps [theta_nb, upper
// Gershgorin bound] and grows what lies below, then Rayleigh-Ritz on the block.
void zeroth_order(sppc_ctx* c) {
  hipStream_t s = c->s;
  const int64_t n0 = c->n0;
  const int D = c->D;
  const int nb = (int)std::min<int64_t>(n0, KB);
  Arena tmp;
  tmp.temp = true;
  Basis sb;
  sb.n = n0;
  sb.ldq = nb;
  sb.Q = tmp.alloc<double>((size_t)n0 * nb);
  sb.HQ = tmp.alloc<double>((size_t)n0 * nb);
  sb.T = tmp.alloc<double>((size_t)nb * nb);
  double* h0diag = tmp.alloc<double>(n0);
  double* gtmp = tmp.alloc<double>(n0 + 1);
  copy_block(n0, 1, c->diag, 1, h0diag, 1, s);
  gershgorin_upper(c->H0, gtmp, gtmp + n0, s);
  double bup = 0.0;
  SPPC_HIP(hipMemcpyAsync(c->pin, gtmp + n0, sizeof(double), hipMemcpyDeviceToHost, s));
  sync(c);
  bup = c->pin[0];
  Op op{c, &c->H0, false, false};
  select_smallest(n0, h0diag, nb, c->idx, s);
  unit_block(n0, nb, c->idx, c->Psi, nb, s);
  ortho_append(c, sb, c->Psi, nb, op, -1);
  const double tol = c->o.h0_tol;
  // The eigenpairs kept only for the deflation of the small solves (beyond the wanted ones) need the
  // accuracy of those solves, not more: a residual 1e-3 times their tolerance (1e-9 for the mixed
  // form's 1e-6; the float64 form's 1e-12 keeps h0_tol)
  const int nwant = std::max(c->k, c->o.pair_index + 1);
  const double inner = c->o.inner_tol > 0.0 ? c->o.inner_tol
                                            : (c->o.precision == SPPC_PREC_MIXED ? 1e-6 : 1e-12);
  const double tol_defl = std::max(tol, 1e-3 * inner);
  int it = 0;
  for (;; ++it) {
    const int nw = sb.m;
    rayleigh_ritz(c, sb, nw);
    double worst = 0.0;
    for (int i = 0; i < std::min(D, nw); ++i) {
      const double r = std::sqrt(std::max(0.0, c->pin[NWMAX + i])) / std::max(1.0, std::fabs(c->theta_h[i]));
      worst = std::max(worst, i < nwant ? r : r * (tol / tol_defl));
    }
    if ((worst <= tol && nw >= D) || nw == n0) break;
    if (it >= 400) throw Error(SPPC_E_BREAKDOWN, "eigensolver for H0hat did not converge");
    // filter interval [a, bup], scaled so that the lowest Ritz value maps to ~1
    const double a = c->theta_h[nw - 1], a0 = c->theta_h[0];
    const double bb = std::max(bup, a + 1e-3 * std::max(1.0, std::fabs(a)));
    const double e = 0.5 * (bb - a), cc = 0.5 * (bb + a);
    double sigma = e / (a0 - cc);
    const double tau = 2.0 / sigma;
    // degree: the lowest Ritz value grows by T_deg(y0) against the damped interval; keep that
    // below e^25 (~7e10) so the block keeps the accuracy of its slowest wanted directions
    const double y0 = std::max(1.0 + 1e-12, (cc - a0) / e);
    const int deg = std::max(12, std::min(64, (int)(25.0 / std::acosh(y0))));
    double* buf[4] = {c->Z, c->Psi, c->R, c->HZ};
    int i0 = 0, i1 = 1;  // Y_{j-1}, Y_j
    // Y_1 = sigma/e (H - cc) Y_0  (Z holds the Ritz vectors, ld nw)
    spmm_cheb(c->H0, buf[0], nw, buf[1], nw, nw, sigma / e, cc, 0.0, buf[0], nw, s);
    for (int j = 2; j <= deg; ++j) {
      const double sn = 1.0 / (tau - sigma);
      int nxt = 0;
      while (nxt == i0 || nxt == i1) ++nxt;
      spmm_cheb(c->H0, buf[i1], nw, buf[nxt], nw, nw, 2.0 * sn / e, cc, -sigma * sn, buf[i0], nw, s);
      i0 = i1;
      i1 = nxt;
      sigma = sn;
    }
    sb.m = 0;
    const int kept = ortho_append(c, sb, buf[i1], nw, op, -1);
    if (kept < D) throw Error(SPPC_E_BREAKDOWN, "H0hat eigensolver lost directions in the filter");
  }
  c->st.h0_iterations = it;
  if (c->nw_last < D) throw Error(SPPC_E_ARG, "n_deflate exceeds the available eigenpairs of H0hat");
  copy_block(1, D, c->theta, D, c->E0, D, s);
  copy_block(n0, D, c->Z, c->nw_last, c->Psihat, D, s);
  sign_fix_columns(n0, D, c->Psihat, D, c->work, s);
  c->E0h.assign(c->theta_h.begin(), c->theta_h.begin() + D);
  sync(c);
  tmp.release();
}

// Deflated CG on (H0hat - E_k) restricted to the complement of the deflated eigenvectors,
// for all k columns at once (one kernel per iteration), then the exact deflated terms: the
// minimum-norm solution of eq. sm_lin_proj orthogonal to psi_k.  b1 in c->cr (n0 x k);
// result into Psi rows [0, n0).  Float64 products in both precisions: float32 products in these
// solves cost the mixed form continuation steps (measured), the product with H0hat is small.
// shift (device, [k], optional): sigma_k in place of E_k^(0) (the theta-shifted variant); the CG
// operator H0hat - sigma_k stays positive definite on the complement of the deflated vectors when
// sigma_k <= E_D^(0) < E_{D+1}^(0).
void small_solve(sppc_ctx* c, const double* shift = nullptr) {
  hipStream_t s = c->s;
  const int64_t n0 = c->n0;
  const int k = c->k, D = c->D;
  const bool mixed = c->o.precision == SPPC_PREC_MIXED;
  double tol = c->o.inner_tol;
  if (tol <= 0.0) tol = mixed ? 1e-6 : 1e-12;
  const double* sig = shift ? shift : c->E0;
  c->st.cg_iterations += cg_solve(c->H0, n0, k, D, sig, c->Psihat, c->cg_rowb, c->cx, c->cr, c->cgpart,
                                  c->ccoef, 5000, tol, c->pin_i + 4, s);
  deflate_coefs(D, k, c->E0, shift, c->ccoef, k, c->ctmp, k, s);
  gemm_nn(n0, D, k, c->Psihat, D, c->ctmp, k, c->cx, k, 1.0, 1.0, s);
  copy_block(n0, k, c->cx, k, c->Psi, k, s);
}

// shifts_host (optional, [k]): sigma_k in place of E_k^(0) in eq. sm_first and eq. sm_lin_proj (the
// right-hand side of eq. exp_seq2 and E^(p) are unchanged); each must lie below E_D^(0) so that the
// small-space operator is positive definite on the complement of the deflated eigenvectors.
void correct_perturbative(sppc_ctx* c, const double* shifts_host = nullptr) {
  if (c->restarted) throw Error(SPPC_E_ARG, "perturbative corrections need the unrestarted basis");
  if (c->p + 1 >= c->maxhist) throw Error(SPPC_E_ARG, "perturbation order limit reached");
  hipStream_t s = c->s;
  const int k = c->k;
  const int64_t n = c->n, n0 = c->n0;
  Basis& b = c->B;
  const double* sig = c->E0;
  if (shifts_host) {
    const double top = c->E0h[c->D - 1];
    for (int i = 0; i < k; ++i) {
      const double v = shifts_host[i];
      if (!std::isfinite(v) || v > top)
        throw Error(SPPC_E_ARG, "shifts must be finite and at most the largest deflated eigenvalue of H0hat");
      if (std::fabs(v) < 1e-10 * std::max(1.0, std::fabs(top)))
        throw Error(SPPC_E_SINGULAR_E0, "a zero shift: eq. sm_first divides by it");
      c->pin[3 * NWMAX + i] = v;
    }
    SPPC_HIP(hipMemcpyAsync(c->cshift, c->pin + 3 * NWMAX, sizeof(double) * k, hipMemcpyHostToDevice, s));
    sig = c->cshift;
  }
  c->p += 1;
  const int p = c->p;
  size_t t0 = c->tm.begin(C_SMALL);
  // W = H Psi^(p-1) - sum_l E^(p-l) Psi^(l)  (eq. HPsip with the stored H Q); usually formed
  // already by the Rayleigh-Ritz passes of step p - 1
  if (!(c->w_next == p && c->w_m == b.m)) {
    build_correction_coefs(p, k, b.m, c->Ghist, c->gstride, k, c->mhist_dev, c->Etab, b.T, b.ldq, c->E0,
                           c->Acoef, c->Bcoef, s);
    gemm_nn(n, b.m, k, b.HQ, b.ldq, c->Acoef, k, c->Wb, k, 1.0, 0.0, s);
    gemm_nn(n, b.m, k, b.Q, b.ldq, c->Bcoef, k, c->Wb, k, -1.0, 1.0, s);
  }
  c->w_next = -1;
  // complement rows: x2 = -b2 / E^(0) with b2 = -W2 (H0 is zero there), eq. sm_first
  complement_rows(n0, n, k, c->Wb, k, sig, c->Psi, k, s);
  // small space: b1 = -W1 + H0hat Psi^(p-1)_1 (eq. exp_seq2 with eq. avoid_SpMV2)
  gemm_nn(n0, b.m, k, b.Q, b.ldq, c->Acoef, k, c->cx, k, 1.0, 0.0, s);
  spmm_f64(c->H0, c->cx, k, c->cr, k, k, nullptr, s);
  axpby_block(n0, k, -1.0, c->Wb, k, 1.0, c->cr, k, s);
  small_solve(c, shifts_host ? c->cshift : nullptr);
  if (shifts_host) sync(c);  // the pinned shifts are reused by later steps
  c->tm.end(t0);
  c->pend_b = k;
  c->pend_kind = SPPC_CORR_PERTURBATIVE;
}

// Arrays of the learned preconditioner: the static inputs (A is the context's arena, or a counting
// one) and the work of S samples.
void alloc_mpnn_static(sppc_ctx* c, Arena& A) {
  const int64_t n = c->n;
  const int L = (int)c->loff.size() - 1;
  c->loff_dev = A.alloc<int64_t>(L + 1);
  c->mp_lev = A.alloc<double>(n);
  c->mp_Ad = A.alloc<double>(n);
  c->mp_A1 = A.alloc<double>(n);
  c->mp_Al = A.alloc<double>(n);
  c->mp_grad = A.alloc<double>(512);
  c->mp_loss = A.alloc<double>(64);
  c->mp_th = A.alloc<double>(64);
  c->mp_wd = A.alloc<double>(512);
  c->mp_w = A.alloc<float>(512);
  c->mp_wq = A.alloc<float>(512);
}
void alloc_mpnn_samples(sppc_ctx* c, Arena& A, int S) {
  c->mp_work = A.alloc<double>((size_t)mpnn_work_doubles(c->n, S));
  c->mp_sel = A.alloc<double>((size_t)c->n * S * 3);
}

// Static inputs of the learned preconditioner and workspace for S samples (lazy).
void mpnn_ensure(sppc_ctx* c, int S) {
  hipStream_t s = c->s;
  const int64_t n = c->n;
  if (!c->mp_ready) {
    const int L = (int)c->loff.size() - 1;
    alloc_mpnn_static(c, c->arena);
    SPPC_HIP(hipMemcpy(c->loff_dev, c->loff.data(), sizeof(int64_t) * (L + 1), hipMemcpyHostToDevice));
    Arena tmpA;
    tmpA.temp = true;
    double* tmp = tmpA.alloc<double>((size_t)6 * n);
    mpnn_prepare(c->H, c->diag, c->loff_dev, L, c->nsmall, c->mp_lev, c->mp_Ad, c->mp_A1, c->mp_Al, tmp, s);
    sync(c);
    tmpA.release();
    c->mp_ready = true;
  }
  if (S > c->mp_S) {
    // sized for all k pairs at once (the solver's calls never need more, so they allocate once;
    // only the training entry points may ask for up to 32 samples)
    const int Sa = std::max(S, c->k);
    alloc_mpnn_samples(c, c->arena, Sa);
    c->mp_S = Sa;
  }
}

// Basis argument of the training entry points (NULL / m = 0: project against x only).
const MpnnBasis* mpnn_basis(sppc_ctx* c, const double* Q_dev, int m, MpnnBasis& B) {
  if (!Q_dev || m <= 0) return nullptr;
  if (m > 512) throw Error(SPPC_E_ARG, "basis wider than 512 columns");
  const int64_t need = mpnn_basis_work_doubles(c->n, m);
  if (need > c->mp_bwork_cap) {  // sized once for the widest basis
    c->mp_bwork_cap = mpnn_basis_work_doubles(c->n, 512);
    c->mp_bwork = c->arena.alloc<double>((size_t)c->mp_bwork_cap);
  }
  B = MpnnBasis{Q_dev, m, m, c->mp_bwork};
  return &B;
}

void upload_theta(sppc_ctx* c, const double* th, int S) {
  for (int i = 0; i < S; ++i) c->pin[3 * NWMAX + i] = th[i];
  SPPC_HIP(hipMemcpyAsync(c->mp_th, c->pin + 3 * NWMAX, sizeof(double) * S, hipMemcpyHostToDevice, c->s));
  sync(c);
}

// Continuation step with the small-space preconditioner: t_a = -(I - z z^T) M_a r_a where M_a is
// (H0hat - theta_a)^-1 on the rows of the small space (deflated CG to precond_tol, plus the exact
// terms of the D deflated eigenvectors of H0hat) and the diagonal step (diag(H) - theta_a)^-1 on
// the other rows.  On the complement of the deflated vectors H0hat - theta_a is positive
// definite: a Ritz value theta_a >= lambda_a(H) <= E_a(H0hat) < E_{D+1} by interlacing.
void small_expansion(sppc_ctx* c, const std::vector<int>& act) {
  hipStream_t s = c->s;
  const int na = (int)act.size(), k = c->k, D = c->D;
  const int64_t n = c->n, n0 = c->n0;
  for (int a = 0; a < na; ++a) {
    c->pin_i[8 + a] = act[a];
    c->pin[3 * NWMAX + a] = c->theta_h[act[a]];
  }
  SPPC_HIP(hipMemcpyAsync(c->idx, c->pin_i + 8, sizeof(int) * na, hipMemcpyHostToDevice, s));
  SPPC_HIP(hipMemcpyAsync(c->cshift, c->pin + 3 * NWMAX, sizeof(double) * na, hipMemcpyHostToDevice, s));
  jacobi_block(n, na, c->idx, c->R, k, c->diag, c->theta, c->Psi, na, s);
  gather_cols(n0, na, c->idx, c->R, k, c->cr, na, s);
  c->st.cg_iterations += cg_solve(c->H0, n0, na, D, c->cshift, c->Psihat, c->cg_rowb, c->cx, c->cr, c->cgpart,
                                  c->ccoef, 1000, c->o.precond_tol, c->pin_i + 4, s);
  deflate_shift(D, na, c->E0, c->cshift, c->ccoef, na, c->ctmp, na, s);
  gemm_nn(n0, D, na, c->Psihat, D, c->ctmp, na, c->cx, na, 1.0, 1.0, s);
  copy_block(n0, na, c->cx, na, c->Psi, na, s);
  paired_dots(n, na, c->idx, c->Z, k, c->Psi, na, c->dots, c->work, s);
  project_out_block(n, na, c->idx, c->Z, k, c->dots, c->Psi, na, s);
  sync(c);
}

void correct_continuation(sppc_ctx* c, int kind) {
  if (kind == SPPC_CORR_MPNN && !c->mp_have_w) throw Error(SPPC_E_ARG, "no weights for the learned preconditioner");
  std::vector<int> act;
  for (int i = 0; i < c->k; ++i)
    if (!(c->rrn_h[i] < c->o.tol)) act.push_back(i);
  if (act.empty()) { c->pend_b = 0; return; }
  if (c->nw_last != c->k) throw Error(SPPC_E_ARG, "no Ritz pairs available");
  Basis& b = c->B;
  size_t t0 = c->tm.begin(C_SMALL);
  if (b.m + (int)act.size() > b.ldq) {
    restart_basis(c, b, c->k);
    c->restarted = true;
  }
  if (kind == SPPC_CORR_SMALL)
    small_expansion(c, act);
  else
    jacobi_expansion(c, c->n, c->diag, act, c->k);
  if (kind == SPPC_CORR_MPNN && !c->mp_invalid) {
    // the true residual judges the learned step: a pair whose residual did not fall below 0.9x
    // its value at the previous learned step uses the diagonal step from then on
    if ((int)c->mp_fallback.size() != c->k) {
      c->mp_fallback.assign(c->k, 0);
      c->mp_prev_rrn.assign(c->k, 0.0);
    }
    for (int i = 0; i < c->k; ++i)
      if (c->mp_prev_rrn[i] > 0.0 && !(c->rrn_h[i] < 0.9 * c->mp_prev_rrn[i])) c->mp_fallback[i] = 1;
    std::vector<int> sel, pos;
    for (int a = 0; a < (int)act.size(); ++a)
      if (!c->mp_fallback[act[a]]) { sel.push_back(act[a]); pos.push_back(a); }
    if (!sel.empty()) {
      const int S = (int)sel.size(), na = (int)act.size();
      const int64_t n = c->n;
      mpnn_ensure(c, S);
      hipStream_t s = c->s;
      for (int a = 0; a < S; ++a) c->pin_i[8 + a] = sel[a];
      SPPC_HIP(hipMemcpyAsync(c->idx, c->pin_i + 8, sizeof(int) * S, hipMemcpyHostToDevice, s));
      double* Rs = c->mp_sel;
      double* Zs = Rs + n * S;
      double* Ts = Zs + n * S;
      gather_cols(n, S, c->idx, c->R, c->k, Rs, S, s);
      gather_cols(n, S, c->idx, c->Z, c->k, Zs, S, s);
      std::vector<double> th(S);
      for (int a = 0; a < S; ++a) th[a] = c->theta_h[sel[a]];
      upload_theta(c, th.data(), S);
      mpnn_run<float>(c->H, c->diag, c->mp_lev, c->mp_Ad, c->mp_A1, c->mp_Al, c->mp_wq, S, Rs, S, Zs, S,
                      c->mp_th, nullptr, Ts, nullptr, nullptr, c->mp_work, nullptr, s);
      c->st.n_spmv += 2 * S;  // the network's two aggregations are products with H
      // a non-finite or vanishing learned direction falls back to the diagonal step
      colsumsq(n, S, Ts, S, c->sumsq, c->work, s);
      SPPC_HIP(hipMemcpyAsync(c->pin + 2 * NWMAX, c->sumsq, sizeof(double) * S, hipMemcpyDeviceToHost, s));
      sync(c);
      for (int a = 0; a < S; ++a) {
        const double nn = c->pin[2 * NWMAX + a];
        if (std::isfinite(nn) && nn > 0.0) {
          c->pin_i[8 + a] = pos[a];
          c->mp_prev_rrn[sel[a]] = c->rrn_h[sel[a]];
        } else {
          c->pin_i[8 + a] = -1;
          c->mp_fallback[sel[a]] = 1;
        }
      }
      SPPC_HIP(hipMemcpyAsync(c->idx, c->pin_i + 8, sizeof(int) * S, hipMemcpyHostToDevice, s));
      scatter_cols(n, S, c->idx, Ts, S, c->Psi, na, -1.0, s);
      sync(c);
      c->st.mpnn_steps += 1;
    }
  }
  c->tm.end(t0);
  c->pend_b = (int)act.size();
  c->pend_kind = kind;
}

// Mixed precision: block products use float32 X and float32 products until the largest
// relative residual falls below this, float64 afterwards.  The float32 products put relative
// errors of about 1e-7 into H Q, and through T into the high perturbative orders E^(p); near a
// residual of 1e-4 those orders stop improving the basis (measured on the four-level workloads:
// the residual stalls at 1e-5 instead of falling to 6e-6 by p = 15).
constexpr double kMixedF64Below = 1e-4;

int append_and_rr(sppc_ctx* c) {
  Basis& b = c->B;
  const bool mixed = c->o.precision == SPPC_PREC_MIXED;
  Op op{c, &c->H, mixed && !c->refining && !c->f64_products, true};
  int added = 0;
  bool pert = false;
  if (c->pend_b > 0) {
    pert = c->pend_kind == SPPC_CORR_PERTURBATIVE;
    added = ortho_append(c, b, c->Psi, c->pend_b, op, pert ? c->p : -1);
    if (pert) {
      c->mhist.push_back(b.m);
      c->pin_i[40] = b.m;
      SPPC_HIP(hipMemcpyAsync(c->mhist_dev + c->p, c->pin_i + 40, sizeof(int), hipMemcpyHostToDevice, c->s));
    }
  }
  c->pend_b = 0;
  c->last_added = added;
  // when another perturbative step may follow, its coefficients depend only on T and the stored
  // history, so its W is formed in the same passes as Z and H Z
  const sppc_opts& o = c->o;
  const int last_p = o.p_switch > 0 ? std::min(o.p_switch, o.maxiter) : o.maxiter;
  const bool with_next = pert && !c->restarted && c->p < last_p && c->p + 1 < c->maxhist;
  if (with_next)
    build_correction_coefs(c->p + 1, c->k, b.m, c->Ghist, c->gstride, c->k, c->mhist_dev, c->Etab, b.T, b.ldq,
                           c->E0, c->Acoef, c->Bcoef, c->s);
  rayleigh_ritz(c, b, c->k, with_next);
  if (with_next) {
    c->w_next = c->p + 1;
    c->w_m = b.m;
  }
  if (mixed && !c->f64_products) {
    double mx = 0.0;
    for (int i = 0; i < c->k; ++i) mx = std::max(mx, c->rrn_h[i]);
    if (mx < kMixedF64Below) c->f64_products = true;
  }
  return added;
}

void final_check(sppc_ctx* c) {
  hipStream_t s = c->s;
  const int k = c->k;
  const int64_t n = c->n;
  c->w_next = -1;  // Wb is scratch here
  size_t t0 = c->tm.begin(C_SPMM);
  spmm_f64(c->H, c->Z, k, c->Wb, k, k, nullptr, s);
  c->tm.end(t0);
  c->st.n_spmv += k;
  c->st.spmm_calls += 1;
  c->st.spmm_cols += k;
  c->st.spmm_alg_bytes += spmm_alg_bytes(c, k, false);
  t0 = c->tm.begin(C_RR);
  gemm_tn(n, k, k, c->Z, k, c->Wb, k, c->Gm, k, 1.0, 0.0, c->work, s);
  t_from_full(k, c->Gm, k, c->Xt, k, s);
  sym_eig_lowest(k, k, c->Xt, k, c->theta, c->Vrr, k, c->eigscr, s);
  gemm_nn(n, k, k, c->Z, k, c->Vrr, k, c->Phi, k, 1.0, 0.0, s);
  gemm_nn(n, k, k, c->Wb, k, c->Vrr, k, c->HZ, k, 1.0, 0.0, s);
  copy_block(n, k, c->Phi, k, c->Z, k, s);
  residual_block(n, k, c->Z, k, c->HZ, k, c->theta, c->R, k, c->sumsq, c->work, s);
  c->tm.end(t0);
  SPPC_HIP(hipMemcpyAsync(c->pin, c->theta, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  SPPC_HIP(hipMemcpyAsync(c->pin + NWMAX, c->sumsq, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  sync(c);
  c->tm.collect(c->tacc);
  for (int i = 0; i < k; ++i) {
    c->theta_h[i] = c->pin[i];
    c->rrn_h[i] = std::sqrt(std::max(0.0, c->pin[NWMAX + i])) / std::max(std::fabs(c->pin[i]), 1e-300);
  }
}

void log_step(sppc_ctx* c, const char* phase) {
  if (!c->o.verbose) return;
  double mx = 0.0, mn = 1.0;
  for (double r : c->rrn_h) mx = std::max(mx, r);
  for (double a : c->angles_h) mn = std::min(mn, a);
  fprintf(stderr, "[sppc] %s p=%d m=%d added=%d max_rrn=%.3e min_angle=%.2e theta0=%.15g\n", phase, c->p,
          c->B.m, c->last_added, mx, mn, c->theta_h.empty() ? 0.0 : c->theta_h[0]);
}

double max_rrn(const sppc_ctx* c) {
  double mx = 0.0;
  for (double r : c->rrn_h) mx = std::max(mx, r);
  return mx;
}

// The automatic switch (the paper leaves its detection open, Sec. VII): SPPC has stagnated once a
// new correction vector lies almost in the basis (sine of its angle to the basis below 1e-4, the
// collapse of Fig. 3) or once the largest residual has not halved over the last three steps.
// top[j] is the largest rrn after the j-th step of this call (top[0]: before the first).
bool sppc_stagnates(const sppc_ctx* c, const std::vector<double>& top) {
  double mn = 1.0;
  for (double a : c->angles_h) mn = std::min(mn, a);
  if (mn < 1e-4) return true;
  const size_t h = top.size();
  return h >= 4 && !(top[h - 1] < 0.5 * top[h - 4]);
}

// The hand-over of the RMM-DIIS refinement to the Davidson continuation: top[0] is the largest
// residual at the switch, top[s] the largest after sweep s.  It has stagnated when that residual
// has not halved since three sweeps before (the residual clause of the SPPC rule above).  An
// interior pair whose minimal-residual step along the diagonally preconditioned residual turns
// orthogonal to the residual (H - theta and the preconditioner both indefinite) gains nothing
// from further sweeps.
bool rmm_stagnates(const std::vector<double>& top) {
  const size_t h = top.size();
  return h >= 4 && !(top[h - 1] < 0.5 * top[h - 4]);
}

bool all_converged(sppc_ctx* c) {
  for (int i = 0; i < c->k; ++i)
    if (!(c->rrn_h[i] < c->o.tol)) return false;
  return true;
}

// The arrays of a context that do not depend on what setup finds in H (A: the context's arena, or a
// counting one).
void alloc_buffers(sppc_ctx* c, Arena& A) {
  const sppc_opts& o = c->o;
  const int k = c->k;
  const int64_t n = c->n;
  const int mm = o.m_max;
  const int last_p = (o.p_switch > 0) ? std::min(o.p_switch, o.maxiter) : o.maxiter;
  const bool mixed = o.precision == SPPC_PREC_MIXED;
  c->B.Q = A.alloc<double>((size_t)n * mm);
  c->B.HQ = A.alloc<double>((size_t)n * mm);
  c->B.T = A.alloc<double>((size_t)mm * mm);
  c->Psi = A.alloc<double>((size_t)n * KB);
  c->Phi = A.alloc<double>((size_t)n * KB);
  c->Wb = A.alloc<double>((size_t)n * KB);
  c->Z = A.alloc<double>((size_t)n * KB);
  c->HZ = A.alloc<double>((size_t)n * KB);
  c->R = A.alloc<double>((size_t)n * KB);
  if (mixed) c->X32 = A.alloc<float>((size_t)n * KB);
  const int mbig = std::max(mm, 512);
  c->C1 = A.alloc<double>((size_t)mbig * KB);
  c->C2 = A.alloc<double>((size_t)mbig * KB);
  c->Xt = A.alloc<double>((size_t)mbig * KB);
  c->Acoef = A.alloc<double>((size_t)mbig * KB);
  c->Bcoef = A.alloc<double>((size_t)mbig * KB);
  c->Cq = A.alloc<double>((size_t)mbig * KB);
  c->Ch = A.alloc<double>((size_t)mbig * KB);
  c->Gm = A.alloc<double>(KB * KB);
  c->M1 = A.alloc<double>(KB * KB);
  c->M2 = A.alloc<double>(KB * KB);
  c->Rt = A.alloc<double>(KB * KB);
  c->Vrr = A.alloc<double>((size_t)mbig * NWMAX);
  c->theta = A.alloc<double>(NWMAX);
  c->sumsq = A.alloc<double>(NWMAX);
  c->psi2 = A.alloc<double>(KB);
  c->angles = A.alloc<double>(KB);
  c->dots = A.alloc<double>(KB);
  c->work = A.alloc<double>((size_t)std::max({gemm_tn_work(n, mbig, KB), gemm_tn_work(c->n0, mbig, KB),
                                               2 * cdiv(n, 256) * KB + KB + 64}));
  c->eigscr = A.alloc<double>((size_t)eig_scratch(mbig, NWMAX));
  c->info = A.alloc<int>(8);
  c->idx = A.alloc<int>(64);
  c->maxhist = last_p + 2;
  c->mhist_dev = A.alloc<int>(c->maxhist + 1);
  c->gstride = (int64_t)mm * k;
  c->Ghist = A.alloc<double>((size_t)c->gstride * c->maxhist);
  c->Etab = A.alloc<double>((size_t)(c->maxhist + 1) * k);
  const int64_t n0 = c->n0;
  c->E0 = A.alloc<double>(c->D);
  c->Psihat = A.alloc<double>((size_t)n0 * c->D);
  c->cx = A.alloc<double>((size_t)n0 * KB);
  c->cr = A.alloc<double>((size_t)n0 * KB);
  c->cgpart = A.alloc<double>((size_t)cg_work_doubles(n0));
  c->cg_rowb = A.alloc<int64_t>(257);
  c->cshift = A.alloc<double>(KB);
  c->ccoef = A.alloc<double>((size_t)KB * KB);
  c->ctmp = A.alloc<double>((size_t)KB * KB);
}

// Columns per panel of the column-panel copy of H (0: none): opts.panel_width, or automatically
// 1 MiB of float64 X per panel when a k-column block of X exceeds 8 MiB and n < 2^24.
int choose_panel_width(const sppc_opts& o, int64_t n, int k) {
  int pw = o.panel_width;
  if (pw < 0) {
    const int64_t xbytes = n * (int64_t)k * 8;
    pw = 0;
    if (xbytes > ((int64_t)8 << 20) && n < ((int64_t)1 << 24)) {
      int64_t w = ((int64_t)1 << 20) / ((int64_t)k * 8);  // 1 MiB of float64 X per panel
      int64_t p2 = 1024;
      while (p2 * 2 <= w && p2 * 2 <= 65536) p2 *= 2;
      pw = (int)p2;
    }
  }
  return pw;
}

// Checks the problem and the options and fixes the sizes of the context (no device work).
void configure(sppc_ctx* c, const sppc_csr* Hin, const int64_t* loff, int L, int nsmall, int k) {
  if (!Hin || !loff || L < 1 || nsmall < 1 || nsmall > L) throw Error(SPPC_E_ARG, "bad level partition");
  if (Hin->n < 1 || !Hin->row_ptr_dev || !Hin->col_dev || !Hin->val_dev) throw Error(SPPC_E_ARG, "bad H");
  if (Hin->n >= (int64_t)1 << 31) throw Error(SPPC_E_ARG, "n must be < 2^31");
  c->loff.assign(loff, loff + L + 1);
  if (c->loff[0] != 0 || c->loff[L] != Hin->n) throw Error(SPPC_E_ARG, "level offsets must run 0..n");
  for (int l = 0; l < L; ++l)
    if (c->loff[l + 1] <= c->loff[l]) throw Error(SPPC_E_ARG, "levels must be non-empty and ascending");
  c->n = Hin->n;
  c->nnz_up = Hin->nnz;
  c->n0 = c->loff[nsmall];
  c->nsmall = nsmall;
  c->k = k;
  sppc_opts& o = c->o;
  if (k < 1 || k > 16 || k > c->n0) throw Error(SPPC_E_ARG, "k must be 1..16 and <= n0");
  const int pj = o.pair_index;
  if (pj < -1 || pj > 26 || (pj >= 0 && (k != 1 || pj >= c->n0)))
    throw Error(SPPC_E_ARG, "pair_index must be -1, or 0..26 (below n0) with k = 1 (Alg. 1)");
  if (o.n_deflate <= 0) {
    // tight small solves (the float64 form's 1e-12) take fewer CG iterations with more deflated
    // directions; inexact ones (1e-6) gain nothing from them, and their deflation-only eigenpairs stop
    // at 1e-9 (zeroth_order), which with more of them costs continuation steps (measured at k = 8)
    const double inner = o.inner_tol > 0.0 ? o.inner_tol : (o.precision == SPPC_PREC_MIXED ? 1e-6 : 1e-12);
    const int mult = inner <= 1e-9 ? 3 : 2;
    o.n_deflate = std::min<int64_t>(std::min(std::max(mult * k, pj + 2), 28), c->n0);
  }
  if (o.n_deflate < k || o.n_deflate > 28 || o.n_deflate > c->n0) throw Error(SPPC_E_ARG, "n_deflate must be in [k, min(28, n0)]");
  if (pj >= o.n_deflate) throw Error(SPPC_E_ARG, "n_deflate must exceed pair_index");
  c->D = o.n_deflate;
  if (o.m_max == 0) {
    // automatic: the RMM-DIIS continuation restarts the basis on the k refined vectors at every
    // sweep, so the perturbative steps alone fill it (k columns per step, rounded up to 16 so that
    // the rows stay 128-byte multiples); the Davidson continuations grow it past the switch: 512
    const int lp = (o.p_switch > 0) ? std::min(o.p_switch, o.maxiter) : o.maxiter;
    if (o.precond == SPPC_CORR_RMMDIIS && o.p_switch > 0 && lp >= 0)
      o.m_max = (int)std::min<int64_t>(512, std::max<int64_t>(2 * k, ((int64_t)k * (lp + 1) + 15) / 16 * 16));
    else
      o.m_max = 512;
  }
  if (o.m_max < 2 * k || o.m_max > 512) throw Error(SPPC_E_ARG, "m_max must be in [2k, 512]");
  if (o.panel_width < -1 || o.panel_width > 65536) throw Error(SPPC_E_ARG, "panel_width must be -1, 0 or 1..65536");
  if (o.panel_width > 0 && c->n >= ((int64_t)1 << 24))
    throw Error(SPPC_E_ARG, "the column-panel copy stores a column in 24 bits: panel_width needs n < 2^24");
  if (o.precond != SPPC_CORR_JACOBI && o.precond != SPPC_CORR_MPNN && o.precond != SPPC_CORR_SMALL &&
      o.precond != SPPC_CORR_RMMDIIS)
    throw Error(SPPC_E_ARG, "continuation must be JACOBI, MPNN, SMALL or RMMDIIS");
  if (o.corr_shift != SPPC_SHIFT_E0 && o.corr_shift != SPPC_SHIFT_RITZ)
    throw Error(SPPC_E_ARG, "corr_shift must be SPPC_SHIFT_E0 or SPPC_SHIFT_RITZ");
  if (o.rmm_precond != SPPC_CORR_JACOBI && o.rmm_precond != SPPC_CORR_MPNN)
    throw Error(SPPC_E_ARG, "the RMM-DIIS step preconditioner must be JACOBI or MPNN");
  if (o.refine_precond != SPPC_CORR_JACOBI && o.refine_precond != SPPC_CORR_MPNN &&
      o.refine_precond != SPPC_CORR_SMALL)
    throw Error(SPPC_E_ARG, "refinement preconditioner must be JACOBI, MPNN or SMALL");
  if (!(o.precond_tol > 0.0) || o.precond_tol >= 1.0) throw Error(SPPC_E_ARG, "precond_tol must be in (0, 1)");
  if (!(o.tol > 0) || !(o.tau_drop >= 0) || !(o.inner_tol >= 0) || !(o.h0_tol > 0)) throw Error(SPPC_E_ARG, "bad tolerances");
  if (o.precision != SPPC_PREC_FP64 && o.precision != SPPC_PREC_MIXED) throw Error(SPPC_E_ARG, "bad precision");
  if (o.auto_switch != 0 && o.auto_switch != 1) throw Error(SPPC_E_ARG, "auto_switch must be 0 or 1");
  const int last_p = (o.p_switch > 0) ? std::min(o.p_switch, o.maxiter) : o.maxiter;
  if (last_p < 0) throw Error(SPPC_E_ARG, "maxiter must be >= 0");
  if ((int64_t)k * (last_p + 1) > o.m_max) throw Error(SPPC_E_ARG, "m_max < k * (perturbation order + 1)");
}

void setup_impl(sppc_ctx* c, const sppc_csr* Hin, const int64_t* loff, int L, int nsmall, int k) {
  configure(c, Hin, loff, L, nsmall, k);
  sppc_opts& o = c->o;
  const int pj = o.pair_index;
  hipStream_t s = c->s;
  const bool mixed = o.precision == SPPC_PREC_MIXED;
  // device address of the static scratch of the allocation-free block product (once per device)
  (void)noalloc_scratch(nullptr);

  // device format of H
  Arena& A = c->arena;
  int* dflags = A.alloc<int>(4);
  bool exact = false;
  // first pass decides which value arrays are stored: float32 alone when lossless
  {
    const bool in32 = Hin->val_type == SPPC_F32;
    // validation + exactness happen inside; request float64 storage unless exact
    DevCSR tmp;
    build_full_csr(c->n, Hin->nnz, Hin->row_ptr_dev, Hin->col_dev, Hin->val_dev, in32 ? 1 : 0, tmp, dflags,
                   /*want64=*/false, /*want32=*/true, exact, s);
    if (exact) {
      c->H = tmp;
    } else {
      dev_free(tmp.val32);
      tmp.val32 = nullptr;
      dev_free(tmp.rp);
      dev_free(tmp.col);
      DevCSR t2;
      build_full_csr(c->n, Hin->nnz, Hin->row_ptr_dev, Hin->col_dev, Hin->val_dev, 0, t2, dflags, true, mixed,
                     exact, s);
      c->H = t2;
    }
    A.ptrs.push_back(c->H.rp);
    A.ptrs.push_back(c->H.col);
    if (c->H.val64) A.ptrs.push_back(c->H.val64);
    if (c->H.val32) A.ptrs.push_back(c->H.val32);
  }
  c->exact32 = exact;
  c->H0 = c->H;
  c->H0.n = c->n0;
  c->H0.panel = nullptr;
  {
    // column-panel copy for the block products with H
    const int pw = choose_panel_width(o, c->n, k);
    if (pw > 0) {
      build_panel(c->H, pw, c->panel, s);
      for (void* q : {(void*)c->panel.bstart, (void*)c->panel.bcount, (void*)c->panel.ent, (void*)c->panel.val64,
                      (void*)c->panel.val32, (void*)c->panel.dg, c->panel.xpad})
        if (q) A.ptrs.push_back(q);
      c->H.panel = &c->panel;
    }
  }
  c->H0.rend = A.alloc<int64_t>(c->n0);
  build_block_view(c->H, c->n0, c->H0.rend, s);
  {
    // H0hat as its own contiguous CSR (no gaps where the rows continue beyond column n0)
    DevCSR v = c->H0;
    compact_view(v, c->H0, s);
    A.ptrs.push_back(c->H0.rp);
    A.ptrs.push_back(c->H0.col);
    if (c->H0.val64) A.ptrs.push_back(c->H0.val64);
    if (c->H0.val32) A.ptrs.push_back(c->H0.val32);
  }
  c->diag = A.alloc<double>(c->n);
  extract_diag(c->H, c->diag, s);

  // buffers
  const int64_t n = c->n;
  const int mm = o.m_max;
  c->B.n = n;
  c->B.ldq = mm;
  alloc_buffers(c, A);
  const int64_t n0 = c->n0;
  cg_prepare(c->H0, n0, c->cg_rowb, c->cgpart, s);
  SPPC_HIP(pinned_alloc((void**)&c->pin, sizeof(double) * 4 * NWMAX));
  SPPC_HIP(pinned_alloc((void**)&c->pin_i, sizeof(int) * 128));
  c->tm.s = s;

  // zeroth order
  zeroth_order(c);
  if (pj > 0) {
    // Alg. 1 for pair pj: its zeroth order (E_pj^(0), psi_pj) goes first, so the single wanted pair
    // starts from it and its small solves project psi_pj out; the deflation and its exact terms
    // treat the D eigenvectors alike in any order
    std::swap(c->E0h[0], c->E0h[pj]);
    SPPC_HIP(hipMemcpy(c->E0, c->E0h.data(), sizeof(double) * c->D, hipMemcpyHostToDevice));
    copy_block(c->n0, 1, c->Psihat + pj, c->D, c->cx, 1, s);
    copy_block(c->n0, 1, c->Psihat, c->D, c->Psihat + pj, c->D, s);
    copy_block(c->n0, 1, c->cx, 1, c->Psihat, c->D, s);
    sync(c);
  }
  const double scale = std::max(1.0, std::fabs(c->E0h.back()));
  for (int j = 0; j < k; ++j)
    if (std::fabs(c->E0h[j]) < 1e-10 * scale)
      throw Error(SPPC_E_SINGULAR_E0, "E^(0) is zero for a wanted pair: eq. sm_first divides by it");

  // p = 0: basis Psi^(0) = [psihat; 0], H Psi^(0), T, Rayleigh-Ritz (Alg. 2 steps 2-4)
  Basis& b = c->B;
  fill_block_zero(n, k, b.Q, b.ldq, s);
  copy_block(n0, k, c->Psihat, c->D, b.Q, b.ldq, s);
  {
    // H Psi^(0): Psi^(0) vanishes below row n0, so only the entries of H in columns < n0 (the
    // leading entries of each row) take part: a row-wise product over those, float64 also in mixed
    // precision (E^(p) reads H Psi^(0)).  With levels coupled only to adjacent levels that is a small
    // fraction of H; the rows without such entries get zero.
    Arena tmp;
    tmp.temp = true;
    int64_t* rend = tmp.alloc<int64_t>(n);
    row_ends_below(c->H, n, n0, rend, s);
    DevCSR Hc = c->H;
    Hc.rend = rend;
    Hc.panel = nullptr;
    spmm_f64(Hc, b.Q, b.ldq, b.HQ, b.ldq, k, nullptr, s);
    c->st.n_spmv += k;
    sync(c);
    tmp.release();
  }
  gemm_tn(n, k, k, b.Q, b.ldq, b.HQ, b.ldq, c->Xt, k, 1.0, 0.0, c->work, s);
  t_from_full(k, c->Xt, k, b.T, b.ldq, s);
  b.m = k;
  // G^(0) = I (Psi^(0) is the first block of the basis); E^(0), E^(1) = 0 (eq. first_PC)
  std::vector<double> I0((size_t)k * k, 0.0);
  for (int j = 0; j < k; ++j) I0[(size_t)j * k + j] = 1.0;
  SPPC_HIP(hipMemcpy(Gh(c, 0), I0.data(), sizeof(double) * k * k, hipMemcpyHostToDevice));
  std::vector<double> e01((size_t)2 * k, 0.0);
  for (int j = 0; j < k; ++j) e01[j] = c->E0h[j];
  SPPC_HIP(hipMemcpy(c->Etab, e01.data(), sizeof(double) * 2 * k, hipMemcpyHostToDevice));
  c->mhist.assign(1, k);
  int mk = k;
  SPPC_HIP(hipMemcpy(c->mhist_dev, &mk, sizeof(int), hipMemcpyHostToDevice));
  c->p = 0;
  c->angles_h.assign(k, 1.0);
  rayleigh_ritz(c, b, k);
  log_step(c, "sppc");
}

// SPPC + RMM-DIIS (Sec. V-VI): after the perturbative steps each unconverged Ritz pair is
// refined on its own by RMM-DIIS, the k pairs batched into one block product with H per
// iteration.  Each iteration combines a pair's history by Pulay's DIIS, normalises the
// combination xb, stops the pair when its residual meets the tolerance (Z, H Z and theta keep
// xb), and otherwise steps along t = (diag(H) - theta)^-1 R with the step length that minimises
// the residual along t; the new iterate joins the history.  A sweep of at most RMM_SWEEP
// iterations holds at most RMM_SWEEP + 1 iterates, so only that many history slots exist (at
// n = 7.7M and k = 16 one slot of the three histories is 3 GB); a full history would restart
// from xb.  The final check then takes Rayleigh-Ritz on the span of the refined vectors.
// Returns the number of iterations (at most cap <= RMM_SWEEP).
constexpr int RMM_SWEEP = 4;

// The learned step of RMM-DIIS: for the listed pairs (unit iterates xb, residuals rb, Rayleigh
// quotients th_host) the direction tJ (1 + o) of the network replaces the diagonal step tJ already
// in t.  Returns the pairs that took it (their rrn before the step in mp_prev_rrn): the caller judges
// each by the true residual of the iterate the step produced.  A pair whose learned direction is not
// finite keeps the diagonal step from then on.
std::vector<int> rmm_learned_step(sppc_ctx* c, const std::vector<int>& act, const std::vector<double>& rrn_now,
                                  const double* th_host, const double* rb, const double* xb, double* t) {
  hipStream_t s = c->s;
  const int k = c->k;
  const int64_t n = c->n;
  if ((int)c->mp_fallback.size() != k) {
    c->mp_fallback.assign(k, 0);
    c->mp_prev_rrn.assign(k, 0.0);
  }
  std::vector<int> sel, used;
  for (int a : act)
    if (!c->mp_fallback[a]) sel.push_back(a);
  if (sel.empty()) return used;
  const int S = (int)sel.size();
  mpnn_ensure(c, S);
  for (int a = 0; a < S; ++a) c->pin_i[8 + a] = sel[a];
  SPPC_HIP(hipMemcpyAsync(c->idx, c->pin_i + 8, sizeof(int) * S, hipMemcpyHostToDevice, s));
  double* Rs = c->mp_sel;
  double* Zs = Rs + n * S;
  double* Ts = Zs + n * S;
  gather_cols(n, S, c->idx, rb, k, Rs, S, s);
  gather_cols(n, S, c->idx, xb, k, Zs, S, s);
  std::vector<double> th(S);
  for (int a = 0; a < S; ++a) th[a] = th_host[sel[a]];
  upload_theta(c, th.data(), S);
  mpnn_run<float>(c->H, c->diag, c->mp_lev, c->mp_Ad, c->mp_A1, c->mp_Al, c->mp_wq, S, Rs, S, Zs, S, c->mp_th,
                  nullptr, Ts, nullptr, nullptr, c->mp_work, nullptr, s, /*project=*/false);
  c->st.n_spmv += 2 * S;  // the network's two aggregations are products with H
  colsumsq(n, S, Ts, S, c->sumsq, c->work, s);
  SPPC_HIP(hipMemcpyAsync(c->pin + 2 * NWMAX, c->sumsq, sizeof(double) * S, hipMemcpyDeviceToHost, s));
  sync(c);
  for (int a = 0; a < S; ++a) {
    const double nn = c->pin[2 * NWMAX + a];
    if (std::isfinite(nn) && nn > 0.0) {
      c->pin_i[8 + a] = sel[a];
      c->mp_prev_rrn[sel[a]] = rrn_now[sel[a]];
      used.push_back(sel[a]);
    } else {
      c->pin_i[8 + a] = -1;
      c->mp_fallback[sel[a]] = 1;
    }
  }
  SPPC_HIP(hipMemcpyAsync(c->idx, c->pin_i + 8, sizeof(int) * S, hipMemcpyHostToDevice, s));
  scatter_cols(n, S, c->idx, Ts, S, t, k, 1.0, s);
  // idx is read again by the caller: restore the identity map of the k pairs
  for (int a = 0; a < k; ++a) c->pin_i[8 + a] = a;
  SPPC_HIP(hipMemcpyAsync(c->idx, c->pin_i + 8, sizeof(int) * k, hipMemcpyHostToDevice, s));
  sync(c);
  c->st.mpnn_steps += 1;
  return used;
}

// The RMM-DIIS arrays (A: the context's arena, or a counting one): RMM_SWEEP + 1 history slots of
// the iterates, their products with H and their residuals, and the per-iteration blocks.
void alloc_rmm(sppc_ctx* c, Arena& A) {
  const int k = c->k;
  const int D = diis_max_depth();
  const int NS = std::min(D, RMM_SWEEP + 1);
  const int64_t slot = c->n * k;
  c->rd_Xh = A.alloc<double>((size_t)NS * slot);
  c->rd_HXh = A.alloc<double>((size_t)NS * slot);
  c->rd_Rh = A.alloc<double>((size_t)NS * slot);
  c->rd_A = A.alloc<double>((size_t)k * D * D);
  c->rd_al = A.alloc<double>((size_t)k * D);
  c->rd_xb = A.alloc<double>((size_t)slot);
  c->rd_hxb = A.alloc<double>((size_t)slot);
  c->rd_rb = A.alloc<double>((size_t)slot);
  c->rd_t = A.alloc<double>((size_t)slot);
  c->rd_ht = A.alloc<double>((size_t)slot);
  c->rd_u = A.alloc<double>((size_t)slot);
  c->rd_sc = A.alloc<double>(8 * 64);
}

int rmm_diis_sweep(sppc_ctx* c, int cap) {
  hipStream_t s = c->s;
  const int k = c->k;
  const int64_t n = c->n;
  const int D = diis_max_depth();            // leading size of the Gram matrices
  const int NS = std::min(D, RMM_SWEEP + 1);  // history slots
  const sppc_opts& o = c->o;
  if (c->nw_last != k) throw Error(SPPC_E_ARG, "no Ritz pairs available");
  if (cap < 0 || cap > RMM_SWEEP) throw Error(SPPC_E_ARG, "RMM-DIIS sweep longer than its history");
  const int64_t slot = n * k;
  if (!c->rd_Xh) alloc_rmm(c, c->arena);
  double *xb = c->rd_xb, *hxb = c->rd_hxb, *rb = c->rd_rb, *t = c->rd_t, *ht = c->rd_ht, *u = c->rd_u;
  double *ss = c->rd_sc, *th = ss + 64, *ssr = ss + 128, *uu = ss + 192, *rd = ss + 256, *g = ss + 320;
  double *th2 = ss + 384, *ss2 = ss + 448;
  double *Xh = c->rd_Xh, *HXh = c->rd_HXh, *Rh = c->rd_Rh;
  for (int a = 0; a < k; ++a) c->pin_i[8 + a] = a;
  SPPC_HIP(hipMemcpyAsync(c->idx, c->pin_i + 8, sizeof(int) * k, hipMemcpyHostToDevice, s));
  // slot 0: the Ritz pairs of the switch
  copy_block(n, k, c->Z, k, Xh, k, s);
  copy_block(n, k, c->HZ, k, HXh, k, s);
  residual_block(n, k, Xh, k, HXh, k, c->theta, Rh, k, ssr, c->work, s);
  gram_set(k, D, 0, 0, ssr, c->rd_A, s);
  int L = 1, iters = 0;
  std::vector<char> done(k);
  for (int a = 0; a < k; ++a) done[a] = c->rrn_h[a] < o.tol;
  Op op{c, &c->H, false, true};
  const bool learned = o.rmm_precond == SPPC_CORR_MPNN && c->mp_have_w && !c->mp_invalid;
  std::vector<double> rrn_now(k, 0.0), th_now(k, 0.0);
  for (int it = 0;; ++it) {
    size_t t0 = c->tm.begin(C_SMALL);
    diis_coefficients(k, L, D, c->rd_A, c->rd_al, s);
    diis_combine(n, k, L, D, c->rd_al, Xh, HXh, xb, hxb, s);
    colsumsq(n, k, xb, k, ss, c->work, s);
    columns_to_unit(n, k, ss, xb, hxb, s);
    coldots(n, k, xb, k, hxb, k, th, c->work, s);
    residual_block(n, k, xb, k, hxb, k, th, rb, k, ssr, c->work, s);
    c->tm.end(t0);
    SPPC_HIP(hipMemcpyAsync(c->pin, th, sizeof(double) * k, hipMemcpyDeviceToHost, s));
    SPPC_HIP(hipMemcpyAsync(c->pin + NWMAX, ssr, sizeof(double) * k, hipMemcpyDeviceToHost, s));
    sync(c);
    bool all = true;
    uint32_t fin = 0;  // pairs that stop here: their xb and H xb go to Z and H Z in one pass
    for (int a = 0; a < k; ++a) {
      if (done[a]) continue;
      const double thv = c->pin[a];
      const double r = std::sqrt(std::max(0.0, c->pin[NWMAX + a])) / std::max(std::fabs(thv), 1e-300);
      rrn_now[a] = r;
      th_now[a] = thv;
      if (r < o.tol || it >= cap) {
        fin |= 1u << a;
        c->theta_h[a] = thv;
        c->rrn_h[a] = r;
        done[a] = 1;
      } else {
        all = false;
      }
    }
    copy_cols2(n, k, fin, xb, c->Z, hxb, c->HZ, k, s);
    if (all) break;
    ++iters;
    // the step of minimal residual along the preconditioned residual (one product with H)
    t0 = c->tm.begin(C_SMALL);
    jacobi_block(n, k, c->idx, rb, k, c->diag, th, t, k, s);
    c->tm.end(t0);
    std::vector<int> took;  // pairs whose step this iteration was the learned one
    if (learned) {
      std::vector<int> act;
      for (int a = 0; a < k; ++a)
        if (!done[a]) act.push_back(a);
      t0 = c->tm.begin(C_SMALL);
      took = rmm_learned_step(c, act, rrn_now, th_now.data(), rb, xb, t);
      c->tm.end(t0);
    }
    op(t, k, ht, k, k, s);
    t0 = c->tm.begin(C_SMALL);
    residual_block(n, k, t, k, ht, k, th, u, k, uu, c->work, s);  // u = H t - theta t
    coldots(n, k, rb, k, u, k, rd, c->work, s);
    int dst = L;
    if (L >= NS) {  // restart the history from xb
      copy_block(n, k, xb, k, Xh, k, s);
      copy_block(n, k, hxb, k, HXh, k, s);
      copy_block(n, k, rb, k, Rh, k, s);
      gram_set(k, D, 0, 0, ssr, c->rd_A, s);
      dst = 1;
    }
    double *Xn = Xh + dst * slot, *HXn = HXh + dst * slot, *Rn = Rh + dst * slot;
    min_residual_step(n, k, rd, uu, xb, hxb, t, ht, Xn, HXn, s);
    colsumsq(n, k, Xn, k, ss2, c->work, s);
    columns_to_unit(n, k, ss2, Xn, HXn, s);
    coldots(n, k, Xn, k, HXn, k, th2, c->work, s);
    residual_block(n, k, Xn, k, HXn, k, th2, Rn, k, g, c->work, s);
    if (!took.empty()) {
      // the true residual judges the learned step at once: a pair whose new iterate's residual is not
      // below 0.9x that of the iterate it started from takes the diagonal step from now on
      SPPC_HIP(hipMemcpyAsync(c->pin, th2, sizeof(double) * k, hipMemcpyDeviceToHost, s));
      SPPC_HIP(hipMemcpyAsync(c->pin + NWMAX, g, sizeof(double) * k, hipMemcpyDeviceToHost, s));
      sync(c);
      for (int a : took) {
        const double r = std::sqrt(std::max(0.0, c->pin[NWMAX + a])) / std::max(std::fabs(c->pin[a]), 1e-300);
        if (!(r < 0.9 * c->mp_prev_rrn[a])) c->mp_fallback[a] = 1;
      }
    }
    gram_set(k, D, dst, dst, g, c->rd_A, s);
    for (int l = 0; l < dst; ++l) {
      coldots(n, k, Rn, k, Rh + l * slot, k, g, c->work, s);
      gram_set(k, D, dst, l, g, c->rd_A, s);
    }
    c->tm.end(t0);
    L = dst + 1;
  }
  for (int a = 0; a < k; ++a) c->pin[a] = c->theta_h[a];
  SPPC_HIP(hipMemcpyAsync(c->theta, c->pin, sizeof(double) * k, hipMemcpyHostToDevice, s));
  sync(c);
  return iters;
}

// Sweeps of at most 4 RMM-DIIS iterations per pair; between sweeps, Rayleigh-Ritz on the span of
// the k refined vectors (the subspace rotation of multi-pair RMM-DIIS: it separates pairs whose
// eigenvalues are close, which a single-vector iteration resolves only slowly).  The rotation
// needs no product: the refined vectors carry H x.  The basis restarts on them.  Once the sweeps
// stagnate (rmm_stagnates) *handover is set and the basis restarts on the refined Ritz vectors
// with their products taken afresh (the H x carried through the DIIS combinations has drifted
// from H Z by rounding, and Rayleigh-Ritz on drifted columns cannot see below that drift); the
// Davidson continuation goes on from there.  Returns the number of iterations.
int rmm_diis_phase(sppc_ctx* c, bool* handover) {
  const sppc_opts& o = c->o;
  const int k = c->k;
  Op op{c, &c->H, false, true};
  int total = 0;
  std::vector<double> top{max_rrn(c)};
  *handover = false;
  for (bool first = true;; first = false) {
    if (!first) {
      c->B.m = 0;
      const int kept = ortho_append(c, c->B, c->Z, k, op, -1, c->HZ);
      if (kept < k) throw Error(SPPC_E_BREAKDOWN, "RMM-DIIS: the refined vectors became linearly dependent");
      rayleigh_ritz(c, c->B, k);
      c->restarted = true;
      top.push_back(max_rrn(c));
      if (!all_converged(c) && rmm_stagnates(top)) {
        // the products of the continuation's basis (float32 X in mixed precision until its
        // residuals fall below kMixedF64Below)
        Op opc{c, &c->H, o.precision == SPPC_PREC_MIXED && !c->refining && !c->f64_products, true};
        c->B.m = 0;
        if (ortho_append(c, c->B, c->Z, k, opc, -1, nullptr) < k)
          throw Error(SPPC_E_BREAKDOWN, "RMM-DIIS: the refined vectors became linearly dependent");
        rayleigh_ritz(c, c->B, k);
        *handover = true;
        break;
      }
    }
    if (all_converged(c) || total >= o.max_cont) break;
    total += std::max(1, rmm_diis_sweep(c, std::min(RMM_SWEEP, o.max_cont - total)));
  }
  return total;
}

sppc_status solve_impl(sppc_ctx* c, double* evals, double* evecs, double* rrn, sppc_stats* st) {
  const auto t0 = std::chrono::steady_clock::now();
  sppc_opts& o = c->o;
  const int last_p = (o.p_switch > 0) ? std::min(o.p_switch, o.maxiter) : o.maxiter;
  bool conv = all_converged(c);
  std::vector<double> top;  // largest rrn after each SPPC step of this call (automatic switch)
  top.push_back(max_rrn(c));
  while (!conv && c->p < last_p && !c->restarted) {
    std::vector<double> sh;
    if (o.corr_shift == SPPC_SHIFT_RITZ) sh.assign(c->theta_h.begin(), c->theta_h.begin() + c->k);
    correct_perturbative(c, sh.empty() ? nullptr : sh.data());
    const int added = append_and_rr(c);
    log_step(c, "sppc");
    conv = all_converged(c);
    if (added == 0 && !conv) break;  // stagnation: no new direction
    top.push_back(max_rrn(c));
    if (o.auto_switch && !conv && o.p_switch > 0 && sppc_stagnates(c, top)) break;
  }
  c->st.iterations = c->p;
  int cont = 0;
  // the Davidson continuation: the default after the switch, and where RMM-DIIS stagnates
  bool davidson = o.p_switch > 0 && o.precond != SPPC_CORR_RMMDIIS;
  int kind = o.precond;
  if (o.p_switch > 0 && o.precond == SPPC_CORR_RMMDIIS) {
    if (!conv) {
      bool handover = false;
      cont = rmm_diis_phase(c, &handover);
      c->st.rmm_iterations = cont;
      c->st.rmm_handover = handover ? 1 : 0;
      log_step(c, "rmmdiis");
      conv = all_converged(c);
      if (handover && !conv) {
        log_step(c, "handover");
        davidson = true;
        kind = SPPC_CORR_JACOBI;
      }
    }
  }
  if (davidson) {
    std::vector<double> hist;  // max residual per continuation step (mixed hand-over test)
    while (!conv && cont < o.max_cont) {
      correct_continuation(c, kind);
      const int added = append_and_rr(c);
      ++cont;
      log_step(c, "cont");
      conv = all_converged(c);
      if (added == 0 && !conv) break;
      // mixed precision: the loop runs until its residuals (which carry the float32 noise of
      // H Q, far below the tolerance here) meet the tolerance, and the float64 check decides;
      // once they stop falling (the noise floor) it hands over to the float64 refinement
      if (!conv && o.precision == SPPC_PREC_MIXED && o.final_check) {
        double mx = 0.0;
        for (int i = 0; i < c->k; ++i) mx = std::max(mx, c->rrn_h[i]);
        hist.push_back(mx);
        const size_t h = hist.size();
        if (h > 4 && !(mx < 0.5 * hist[h - 5])) break;
      }
    }
  }
  if (o.final_check) {
    final_check(c);
    log_step(c, "final");
    conv = all_converged(c);
    // mixed precision: the float32 products limit what the loop's residuals can see; restart on
    // the checked Ritz vectors (float64 H Z) and continue with float64 products until the true
    // residual meets the tolerance.  The float64 SPPC + RMM-DIIS hybrid takes the same path: its
    // residuals come from the H x carried through the DIIS combinations, which can sit just below
    // the tolerance while the checked ones sit just above it
    const bool rmm64 = o.precond == SPPC_CORR_RMMDIIS && o.precision != SPPC_PREC_MIXED;
    if (!conv && (o.precision == SPPC_PREC_MIXED || rmm64) && o.p_switch > 0) {
      // New basis columns get float64 products.  The basis is kept at first (its float32-product
      // columns still span the directions found so far); the loop's residuals carry the float32
      // noise, so each round ends with the float64 check, which decides convergence.  The
      // float32 columns also bound the accuracy the kept basis can reach: once a round fails to
      // halve the checked residual (or after two rounds) the basis restarts on the checked Ritz
      // vectors, whose H Z is exact, and continues with float64 products only.
      c->refining = true;
      int ref = 0;
      bool clean = false, stalled = false;
      double last = 0.0;
      for (int i = 0; i < c->k; ++i) last = std::max(last, c->rrn_h[i]);
      for (int round = 0; !conv && ref < o.max_cont; ++round) {
        // (after RMM-DIIS the basis does not hold the refined vectors: restart at once)
        if (!clean && (stalled || round >= 2 || o.precond == SPPC_CORR_RMMDIIS)) {
          restart_basis(c, c->B, c->k);
          c->restarted = true;
          clean = true;
        }
        // a kept-basis round cannot see below the float32 noise: at most 4 steps before checking
        const int cap = clean ? o.max_cont : 4;
        for (int st = 0; st < cap && ref < o.max_cont; ++st) {
          correct_continuation(c, o.refine_precond);
          const int added = append_and_rr(c);
          ++ref;
          ++cont;
          log_step(c, "refine");
          conv = all_converged(c);
          if (conv || added == 0) break;
        }
        final_check(c);
        log_step(c, "final");
        conv = all_converged(c);
        double now = 0.0;
        for (int i = 0; i < c->k; ++i) now = std::max(now, c->rrn_h[i]);
        stalled = !(now < 0.5 * last);
        last = now;
        if (clean && stalled && !conv) break;
      }
      c->st.refine_steps = ref;
    }
  }
  c->st.cont_steps = cont;
  c->st.converged = conv;
  c->st.mpnn_fallbacks = 0;
  for (int f : c->mp_fallback) c->st.mpnn_fallbacks += f ? 1 : 0;
  c->st.workspace_peak = (int64_t)ws_peak(c->ws);
  c->st.basis_size = c->B.m;
  const int k = c->k;
  if (evals) memcpy(evals, c->theta_h.data(), sizeof(double) * k);
  if (rrn) memcpy(rrn, c->rrn_h.data(), sizeof(double) * k);
  if (evecs) {
    copy_block(c->n, k, c->Z, c->nw_last, evecs, k, c->s);
    sync(c);
  }
  c->st.t_solve_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  c->st.t_spmm_ms = c->tacc[C_SPMM];
  c->st.t_small_ms = c->tacc[C_SMALL];
  c->st.t_ortho_ms = c->tacc[C_ORTHO];
  c->st.t_rr_ms = c->tacc[C_RR];
  c->st.t_h0_ms = c->tacc[C_H0];
  if (st) *st = c->st;
  return conv ? SPPC_OK : SPPC_E_NOCONV;
}

// Workspace bytes of a context for sppc_setup followed by sppc_solve with its options: the arrays it
// keeps plus the largest set of setup temporaries alive at one time, phase by phase as setup_impl
// allocates them (the builders' sizes from the same expressions as their allocations, the other
// arrays by a counting run of the same allocation code).  For float64 input both outcomes of the
// float32-exactness check are covered.  The training entry points' basis projection is not.
size_t workspace_bytes(sppc_ctx* c, const sppc_csr* Hin) {
  const sppc_opts& o = c->o;
  const int k = c->k;
  const int64_t n = c->n, n0 = c->n0;
  const bool mixed = o.precision == SPPC_PREC_MIXED;
  const bool in32 = Hin->val_type == SPPC_F32;
  int64_t up0 = 0;  // upper entries of the rows of the small space (bounds H0hat's entries)
  SPPC_HIP(hipMemcpy(&up0, Hin->row_ptr_dev + n0, sizeof(int64_t), hipMemcpyDeviceToHost));
  const int64_t nnz_full = 2 * Hin->nnz, nnz0 = 2 * up0;
  size_t best = 0;
  for (int exact = in32 ? 1 : 0; exact < 2; ++exact) {
    size_t base = ws_bytes(sizeof(int) * 4), peak = 0;
    const BuildBytes f1 = full_csr_bytes(n, Hin->nnz, false, true);
    peak = std::max(peak, base + f1.persist + f1.temp);
    size_t csr = f1.persist;
    bool v64 = false, v32 = true;
    if (!exact) {  // the float32 copy is dropped and the CSR built again with float64 values
      const BuildBytes f2 = full_csr_bytes(n, Hin->nnz, true, mixed);
      peak = std::max(peak, base + f2.persist + f2.temp);
      csr = f2.persist;
      v64 = true;
      v32 = mixed;
    }
    base += csr;
    if (choose_panel_width(o, n, k) > 0) {
      const BuildBytes pb = panel_bytes(n, nnz_full, v64, v32);
      peak = std::max(peak, base + pb.persist + pb.temp);
      base += pb.persist;
    }
    base += ws_bytes(sizeof(int64_t) * n0);  // row ends of the H0hat view
    const BuildBytes vb = view_bytes(n0, nnz0, v64, v32);
    peak = std::max(peak, base + vb.persist + vb.temp);
    base += vb.persist + ws_bytes(sizeof(double) * n);  // + diag(H)
    Arena cnt;
    cnt.counting = true;
    alloc_buffers(c, cnt);
    base += cnt.counted;
    const int64_t nb = std::min<int64_t>(n0, KB);  // the zeroth order's temporaries
    peak = std::max(peak, base + 2 * ws_bytes(8 * n0 * nb) + ws_bytes(8 * nb * nb) + ws_bytes(8 * n0) +
                              ws_bytes(8 * (n0 + 1)));
    peak = std::max(peak, base + ws_bytes(sizeof(int64_t) * n));  // row ends of the p = 0 product
    Arena sv;  // arrays the solve adds
    sv.counting = true;
    size_t sv_tmp = 0;
    if (o.precond == SPPC_CORR_RMMDIIS && o.p_switch > 0) alloc_rmm(c, sv);
    if (o.precond == SPPC_CORR_MPNN || o.refine_precond == SPPC_CORR_MPNN ||
        (o.precond == SPPC_CORR_RMMDIIS && o.rmm_precond == SPPC_CORR_MPNN)) {
      alloc_mpnn_static(c, sv);
      alloc_mpnn_samples(c, sv, k);
      sv_tmp = ws_bytes(sizeof(double) * 6 * n);
    }
    peak = std::max(peak, base + sv.counted + sv_tmp);
    best = std::max(best, peak);
  }
  return best + 4096;  // the start of the workspace is rounded up to 256 bytes
}

template <class F>
sppc_status guarded(sppc_ctx* c, F&& f) {
  WsScope scope(c ? c->ws : nullptr);
  try {
    return f();
  } catch (const Error& e) {
    if (c) c->err = e.what();
    return (sppc_status)e.code;
  } catch (const std::exception& e) {
    if (c) c->err = e.what();
    return SPPC_E_ARG;
  }
}

}  // namespace
}  // namespace sppc

// ============================================================================ C ABI
extern "C" {

sppc_status sppc_default_opts(sppc_opts* o) {
  if (!o) return SPPC_E_ARG;
  memset(o, 0, sizeof(*o));
  o->tol = 1e-6;
  o->maxiter = 30;
  o->p_switch = 15;
  o->max_cont = 200;
  o->m_max = 0;  // automatic
  o->n_deflate = 0;
  o->tau_drop = 1e-10;
  o->inner_tol = 0.0;  // automatic: 1e-12 (float64), 1e-6 (mixed)
  o->h0_tol = 1e-12;
  o->precision = SPPC_PREC_FP64;
  o->precond = SPPC_CORR_JACOBI;
  o->refine_precond = SPPC_CORR_SMALL;
  o->precond_tol = 1e-3;
  o->final_check = 1;
  o->verbose = 0;
  o->panel_width = -1;
  o->corr_shift = SPPC_SHIFT_E0;
  o->pair_index = -1;
  o->rmm_precond = SPPC_CORR_JACOBI;
  return SPPC_OK;
}

sppc_status sppc_workspace_size(const sppc_csr* H, const int64_t* level_offsets_host, int n_levels,
                                int n_small_levels, int k, const sppc_opts* opts, size_t* bytes) {
  if (!bytes) return SPPC_E_ARG;
  *bytes = 0;
  sppc_ctx c;
  if (opts) c.o = *opts; else sppc_default_opts(&c.o);
  const sppc_status st = guarded(&c, [&]() {
    configure(&c, H, level_offsets_host, n_levels, n_small_levels, k);
    *bytes = workspace_bytes(&c, H);
    return SPPC_OK;
  });
  if (st != SPPC_OK) g_setup_err = c.err;
  return st;
}

sppc_status sppc_setup(sppc_ctx** out, const sppc_csr* H, const int64_t* level_offsets_host, int n_levels,
                       int n_small_levels, int k, const sppc_opts* opts, void* workspace_dev,
                       size_t workspace_bytes, void* stream) {
  if (!out) return SPPC_E_ARG;
  *out = nullptr;
  if (workspace_dev && workspace_bytes < 4096) {
    g_setup_err = "workspace smaller than 4096 bytes";
    return SPPC_E_ARG;
  }
  sppc_ctx* c = new (std::nothrow) sppc_ctx();
  if (!c) return SPPC_E_NOMEM;
  if (opts) c->o = *opts; else sppc_default_opts(&c->o);
  c->s = (hipStream_t)stream;
  if (workspace_dev) c->ws = ws_create(workspace_dev, workspace_bytes);
  const auto t0 = std::chrono::steady_clock::now();
  sppc_status st = guarded(c, [&]() {
    setup_impl(c, H, level_offsets_host, n_levels, n_small_levels, k);
    return SPPC_OK;
  });
  if (st != SPPC_OK) {
    g_setup_err = c->err;
    sppc_destroy(c);
    return st;
  }
  c->st.t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  c->st.workspace_peak = (int64_t)ws_peak(c->ws);
  *out = c;
  return SPPC_OK;
}

sppc_status sppc_spmm(sppc_ctx* c, const void* X, sppc_dtype xt, double* Y, int b) {
  if (!c || !X || !Y || b < 1 || b > 32) return SPPC_E_ARG;
  return guarded(c, [&]() {
    if (xt == SPPC_F32) {
      if (!c->H.val32) throw Error(SPPC_E_ARG, "float32 values are not stored (H is not float32-exact)");
      spmm_f32(c->H, (const float*)X, b, Y, b, b, nullptr, c->s);
    } else {
      spmm_f64(c->H, (const double*)X, b, Y, b, b, nullptr, c->s);
    }
    return SPPC_OK;
  });
}

sppc_status sppc_spmm_noalloc(sppc_ctx* c, const void* X, sppc_dtype xt, double* Y, int b) {
  if (!c || !X || !Y || b < 1 || b > 32) return SPPC_E_ARG;
  return guarded(c, [&]() {
    size_t cap = 0;
    void* stage = noalloc_scratch(&cap);
    if (xt == SPPC_F32) {
      if (!c->H.val32) throw Error(SPPC_E_ARG, "float32 values are not stored (H is not float32-exact)");
      spmm_f32(c->H, (const float*)X, b, Y, b, b, nullptr, c->s, nullptr, nullptr, 0, stage, cap);
    } else {
      spmm_f64(c->H, (const double*)X, b, Y, b, b, nullptr, c->s, stage, cap);
    }
    return SPPC_OK;
  });
}

sppc_status sppc_spmm_upper(const sppc_csr* H, const void* X, sppc_dtype xt, double* Y, int b, void* stream) {
  sppc_ctx c;
  const sppc_status st = guarded(&c, [&]() {
    if (!H || !X || !Y || b < 1 || b > 32) throw Error(SPPC_E_ARG, "bad argument");
    if (H->n < 0 || H->n >= (int64_t)1 << 31 || (H->n > 0 && (!H->row_ptr_dev || !H->col_dev || !H->val_dev)))
      throw Error(SPPC_E_ARG, "bad H");
    if ((H->val_type != SPPC_F32 && H->val_type != SPPC_F64) || (xt != SPPC_F32 && xt != SPPC_F64))
      throw Error(SPPC_E_ARG, "bad value type");
    UpperCSR U;
    U.n = H->n;
    U.rp = H->row_ptr_dev;
    U.col = H->col_dev;
    if (H->val_type == SPPC_F32) U.val32 = (const float*)H->val_dev;
    else U.val64 = (const double*)H->val_dev;
    spmm_upper(U, X, xt == SPPC_F32, b, Y, b, b, (hipStream_t)stream);
    return SPPC_OK;
  });
  if (st != SPPC_OK) g_setup_err = c.err;
  return st;
}

sppc_status sppc_correct(sppc_ctx* c, int kind, const double* shifts_host) {
  if (!c) return SPPC_E_ARG;
  return guarded(c, [&]() {
    if (kind == SPPC_CORR_PERTURBATIVE) correct_perturbative(c, shifts_host);
    else if (shifts_host) throw Error(SPPC_E_ARG, "shifts apply to the perturbative correction only");
    else if (kind == SPPC_CORR_JACOBI || kind == SPPC_CORR_MPNN || kind == SPPC_CORR_SMALL)
      correct_continuation(c, kind);
    else throw Error(SPPC_E_ARG, "unknown correction kind");
    return SPPC_OK;
  });
}

sppc_status sppc_rayleigh_ritz(sppc_ctx* c, double* theta, double* rrn, int* n_added) {
  if (!c) return SPPC_E_ARG;
  return guarded(c, [&]() {
    const bool had = c->pend_b > 0;
    const int added = append_and_rr(c);
    if (theta) memcpy(theta, c->theta_h.data(), sizeof(double) * c->k);
    if (rrn) memcpy(rrn, c->rrn_h.data(), sizeof(double) * c->k);
    if (n_added) *n_added = added;
    return (had && added == 0) ? SPPC_E_BREAKDOWN : SPPC_OK;
  });
}

sppc_status sppc_solve(sppc_ctx* c, double* evals, double* evecs, double* rrn, sppc_stats* st) {
  if (!c) return SPPC_E_ARG;
  return guarded(c, [&]() { return solve_impl(c, evals, evecs, rrn, st); });
}

sppc_status sppc_get(sppc_ctx* c, int what, double* dst, int64_t count) {
  if (!c || !dst) return SPPC_E_ARG;
  return guarded(c, [&]() {
    auto need = [&](int64_t x) { if (count < x) throw Error(SPPC_E_ARG, "destination too small"); };
    const int64_t n = c->n;
    const int m = c->B.m, k = c->k;
    switch (what) {
      case 0: need(c->D); memcpy(dst, c->E0h.data(), sizeof(double) * c->D); break;
      case 1: need(k); memcpy(dst, c->theta_h.data(), sizeof(double) * k); break;
      case 2: need(1); dst[0] = m; break;
      case 3: need(n * m); copy_block(n, m, c->B.Q, c->B.ldq, dst, m, c->s); sync(c); break;
      case 4: need(n * m); copy_block(n, m, c->B.HQ, c->B.ldq, dst, m, c->s); sync(c); break;
      case 5: need(n * k); copy_block(n, c->pend_b > 0 ? c->pend_b : k, c->Psi, c->pend_b > 0 ? c->pend_b : k, dst,
                                      c->pend_b > 0 ? c->pend_b : k, c->s); sync(c); break;
      case 6: {
        need((int64_t)m * m);
        std::vector<double> h((size_t)m * c->B.ldq);
        SPPC_HIP(hipMemcpy(h.data(), c->B.T, sizeof(double) * m * c->B.ldq, hipMemcpyDeviceToHost));
        for (int i = 0; i < m; ++i) memcpy(dst + (int64_t)i * m, h.data() + (int64_t)i * c->B.ldq, sizeof(double) * m);
        break;
      }
      case 7: need((int64_t)c->angles_h.size()); memcpy(dst, c->angles_h.data(), sizeof(double) * c->angles_h.size()); break;
      case 8: need((int64_t)(c->p + 1) * k);
        SPPC_HIP(hipMemcpy(dst, c->Etab, sizeof(double) * (c->p + 1) * k, hipMemcpyDeviceToHost)); break;
      case 9: need(c->n0 * c->D); copy_block(c->n0, c->D, c->Psihat, c->D, dst, c->D, c->s); sync(c); break;
      case 10: need(n * k); copy_block(n, k, c->Z, c->nw_last, dst, k, c->s); sync(c); break;
      case 11: need(n * k); copy_block(n, k, c->R, c->nw_last, dst, k, c->s); sync(c); break;
      default: throw Error(SPPC_E_ARG, "unknown item");
    }
    return SPPC_OK;
  });
}

sppc_status sppc_mpnn_set_weights(sppc_ctx* c, const float* w_host) {
  if (!c || !w_host) return SPPC_E_ARG;
  return guarded(c, [&]() {
    mpnn_ensure(c, 1);
    bool finite = true;
    for (int i = 0; i < SPPC_MPNN_NPARAM; ++i) finite = finite && std::isfinite(w_host[i]);
    c->mp_invalid = !finite;  // every pair then takes the diagonal step
    SPPC_HIP(hipMemcpy(c->mp_w, w_host, sizeof(float) * SPPC_MPNN_NPARAM, hipMemcpyHostToDevice));
    mpnn_round_bf16(SPPC_MPNN_NPARAM, c->mp_w, c->mp_wq, nullptr, c->s);
    sync(c);
    c->mp_have_w = true;
    c->mp_fallback.assign(c->k, 0);
    c->mp_prev_rrn.assign(c->k, 0.0);
    return SPPC_OK;
  });
}

sppc_status sppc_mpnn_eval(sppc_ctx* c, const float* w_host, int S, const double* R_dev, const double* X_dev,
                           const double* theta_host, const double* Q_dev, int m, const double* E_dev,
                           double* T_dev, double* loss_host, double* grad_host, int f64) {
  if (!c || !w_host || S < 1 || S > 32 || !R_dev || !X_dev || !theta_host || m < 0) return SPPC_E_ARG;
  if ((loss_host || grad_host) && !E_dev) return SPPC_E_ARG;
  return guarded(c, [&]() {
    mpnn_ensure(c, S);
    hipStream_t s = c->s;
    MpnnBasis B;
    const MpnnBasis* bp = mpnn_basis(c, Q_dev, m, B);
    SPPC_HIP(hipMemcpy(c->mp_w, w_host, sizeof(float) * SPPC_MPNN_NPARAM, hipMemcpyHostToDevice));
    upload_theta(c, theta_host, S);
    double* grad = grad_host ? c->mp_grad : nullptr;
    double* lossd = loss_host ? c->mp_loss : nullptr;
    const double* E = (grad || lossd) ? E_dev : nullptr;
    if (f64) {
      std::vector<double> wd(w_host, w_host + SPPC_MPNN_NPARAM);
      SPPC_HIP(hipMemcpy(c->mp_wd, wd.data(), sizeof(double) * SPPC_MPNN_NPARAM, hipMemcpyHostToDevice));
      mpnn_run<double>(c->H, c->diag, c->mp_lev, c->mp_Ad, c->mp_A1, c->mp_Al, c->mp_wd, S, R_dev, S, X_dev, S,
                       c->mp_th, E, T_dev, c->mp_grad, c->mp_loss, c->mp_work, bp, s);
    } else {
      mpnn_round_bf16(SPPC_MPNN_NPARAM, c->mp_w, c->mp_wq, nullptr, s);
      mpnn_run<float>(c->H, c->diag, c->mp_lev, c->mp_Ad, c->mp_A1, c->mp_Al, c->mp_wq, S, R_dev, S, X_dev, S,
                      c->mp_th, E, T_dev, c->mp_grad, c->mp_loss, c->mp_work, bp, s);
    }
    sync(c);
    if (loss_host) SPPC_HIP(hipMemcpy(loss_host, c->mp_loss, sizeof(double) * S, hipMemcpyDeviceToHost));
    if (grad_host) SPPC_HIP(hipMemcpy(grad_host, c->mp_grad, sizeof(double) * SPPC_MPNN_NPARAM, hipMemcpyDeviceToHost));
    return SPPC_OK;
  });
}

sppc_status sppc_mpnn_train_step(sppc_ctx* c, float* state_dev, int S, const double* R_dev, const double* X_dev,
                                 const double* theta_host, const double* Q_dev, int m, const double* E_dev,
                                 float lr, int step, double* loss_host) {
  if (!c || !state_dev || S < 1 || S > 32 || !R_dev || !X_dev || !theta_host || !E_dev || step < 1 || m < 0)
    return SPPC_E_ARG;
  return guarded(c, [&]() {
    mpnn_ensure(c, S);
    hipStream_t s = c->s;
    MpnnBasis B;
    const MpnnBasis* bp = mpnn_basis(c, Q_dev, m, B);
    float* w = state_dev;
    float* mo = w + SPPC_MPNN_NPARAM;
    float* v = mo + SPPC_MPNN_NPARAM;
    float* wq = v + SPPC_MPNN_NPARAM;
    upload_theta(c, theta_host, S);
    mpnn_round_bf16(SPPC_MPNN_NPARAM, w, wq, nullptr, s);
    mpnn_run<float>(c->H, c->diag, c->mp_lev, c->mp_Ad, c->mp_A1, c->mp_Al, wq, S, R_dev, S, X_dev, S, c->mp_th,
                    E_dev, nullptr, c->mp_grad, c->mp_loss, c->mp_work, bp, s);
    mpnn_adam(w, mo, v, c->mp_grad, lr, step, wq, s);
    if (loss_host) {
      std::vector<double> lv(S);
      SPPC_HIP(hipMemcpyAsync(lv.data(), c->mp_loss, sizeof(double) * S, hipMemcpyDeviceToHost, s));
      sync(c);
      double tot = 0.0;
      for (double x : lv) tot += x;
      *loss_host = tot / S;
    }
    return SPPC_OK;
  });
}

sppc_status sppc_mpnn_target(sppc_ctx* c, int S, const double* Q_dev, int m, const double* Psi_dev,
                             double* E_dev) {
  if (!c || S < 1 || S > 32 || !Q_dev || m < 1 || !Psi_dev || !E_dev) return SPPC_E_ARG;
  return guarded(c, [&]() {
    mpnn_ensure(c, S);
    MpnnBasis B;
    mpnn_target(c->n, S, *mpnn_basis(c, Q_dev, m, B), Psi_dev, E_dev, c->s);
    sync(c);
    return SPPC_OK;
  });
}

const char* sppc_last_error(const sppc_ctx* c) { return c ? c->err.c_str() : "null context"; }

const char* sppc_setup_error(void) { return g_setup_err.c_str(); }

void sppc_destroy(sppc_ctx* c) {
  if (!c) return;
  if (c->s) (void)hipStreamSynchronize(c->s); else (void)hipDeviceSynchronize();
  pinned_free(c->pin);
  pinned_free(c->pin_i);
  Workspace* ws = c->ws;
  {
    WsScope scope(ws);  // arrays in the caller's workspace go back to it, the others to the library
    c->arena.release();
    delete c;
  }
  ws_destroy(ws);
}

}  // extern "C"
