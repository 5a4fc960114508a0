// kernels_rmmdiis.hip - the per-pair RMM-DIIS refinement of the SPPC + RMM-DIIS hybrid (Sec. V-VI).
//
// Every wanted pair is refined on its own (one product with H per pair and iteration, the k
// pairs batched into one block product).  The history of pair a is kept in slots of n x k blocks
// (column a of each slot): iterates x_l (unit norm), H x_l and residuals R_l = H x_l - theta_l x_l,
// with the Gram matrix A_a[i][l] = R_i . R_l of the residuals (k x D x D).
#include "common.h"

namespace sppc {

namespace {

inline unsigned grid1(int64_t count) { return (unsigned)cdiv(count > 0 ? count : 1, 256); }

constexpr int DIIS_MAX = 16;

// Pulay's DIIS: the a minimising a^T A a subject to sum(a) = 1, from the bordered system
// [[A, 1], [1^T, 0]] [a; mu] = [0; 1] by Gaussian elimination with partial pivoting, one thread
// per pair.  A is scaled to a unit largest diagonal first (the minimiser does not depend on its
// scale, and the residuals shrink to ~1e-10 against the unit border).  A pivot below 1e-14
// (residuals of converging iterates grow parallel) leaves the latest iterate alone: a = e_{L-1}.
__global__ __launch_bounds__(64) void k_diis_coef(int k, int L, int D, const double* __restrict__ A,
                                                  double* __restrict__ alpha) {
  __shared__ double M[16][DIIS_MAX + 1][DIIS_MAX + 2];
  const int a = threadIdx.x;
  if (a >= k) return;
  double (*m)[DIIS_MAX + 2] = M[a];
  const double* Aa = A + (int64_t)a * D * D;
  const int N = L + 1;
  double scale = 0.0;
  for (int i = 0; i < L; ++i) scale = fmax(scale, Aa[i * D + i]);
  const double rs = scale > 0.0 ? 1.0 / scale : 0.0;
  for (int i = 0; i < L; ++i)
    for (int l = 0; l < L; ++l) m[i][l] = Aa[i * D + l] * rs;
  for (int i = 0; i < L; ++i) {
    m[i][L] = 1.0;
    m[L][i] = 1.0;
    m[i][N] = 0.0;
  }
  m[L][L] = 0.0;
  m[L][N] = 1.0;
  bool ok = scale > 0.0;
  for (int c = 0; c < N && ok; ++c) {
    int p = c;
    for (int r = c + 1; r < N; ++r)
      if (fabs(m[r][c]) > fabs(m[p][c])) p = r;
    if (!(fabs(m[p][c]) > 1e-14)) {
      ok = false;
      break;
    }
    if (p != c)
      for (int j = c; j <= N; ++j) {
        const double tmp = m[c][j];
        m[c][j] = m[p][j];
        m[p][j] = tmp;
      }
    const double inv = 1.0 / m[c][c];
    for (int r = c + 1; r < N; ++r) {
      const double f = m[r][c] * inv;
      if (f != 0.0)
        for (int j = c; j <= N; ++j) m[r][j] -= f * m[c][j];
    }
  }
  double* out = alpha + (int64_t)a * D;
  if (ok) {
    double x[DIIS_MAX + 1];
    for (int r = N - 1; r >= 0; --r) {
      double v = m[r][N];
      for (int j = r + 1; j < N; ++j) v -= m[r][j] * x[j];
      x[r] = v / m[r][r];
    }
    for (int l = 0; l < L; ++l) out[l] = x[l];
  } else {
    for (int l = 0; l < L; ++l) out[l] = l == L - 1 ? 1.0 : 0.0;
  }
}

// xb[:, a] = sum_l alpha[a][l] Xh_l[:, a], and the same for H x
__global__ void k_hist_combine(int64_t n, int k, int L, int D, const double* __restrict__ alpha,
                               const double* __restrict__ Xh, const double* __restrict__ HXh,
                               double* __restrict__ xb, double* __restrict__ hxb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  const int a = (int)(e % k);
  const double* al = alpha + (int64_t)a * D;
  const int64_t slot = n * k;
  double x = 0.0, hx = 0.0;
  for (int l = 0; l < L; ++l) {
    x = fma(al[l], Xh[l * slot + e], x);
    hx = fma(al[l], HXh[l * slot + e], hx);
  }
  xb[e] = x;
  hxb[e] = hx;
}

// X[:, a] /= sqrt(ss[a]) and HX[:, a] /= sqrt(ss[a])
__global__ void k_col_unit(int64_t n, int k, const double* __restrict__ ss, double* __restrict__ X,
                           double* __restrict__ HX) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  const double r = 1.0 / sqrt(ss[e % k]);
  X[e] *= r;
  HX[e] *= r;
}

// the step of minimal residual along t: lam = -(Rb . u) / (u . u), u = H t - theta t;
// Xn = xb + lam t, HXn = H xb + lam H t
__global__ void k_col_step(int64_t n, int k, const double* __restrict__ rd, const double* __restrict__ uu,
                           const double* __restrict__ xb, const double* __restrict__ hxb,
                           const double* __restrict__ t, const double* __restrict__ ht, double* __restrict__ Xn,
                           double* __restrict__ HXn) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  const int a = (int)(e % k);
  const double lam = uu[a] > 0.0 ? -rd[a] / uu[a] : 0.0;
  Xn[e] = fma(lam, t[e], xb[e]);
  HXn[e] = fma(lam, ht[e], hxb[e]);
}

// A_a[i][l] = A_a[l][i] = g[a]
__global__ void k_gram_set(int k, int D, int i, int l, const double* __restrict__ g, double* __restrict__ A) {
  const int a = threadIdx.x;
  if (a >= k) return;
  A[(int64_t)a * D * D + i * D + l] = g[a];
  A[(int64_t)a * D * D + l * D + i] = g[a];
}

}  // namespace

int diis_max_depth() { return DIIS_MAX; }

void diis_coefficients(int k, int L, int D, const double* A, double* alpha, hipStream_t s) {
  if (k < 1 || k > 16 || L < 1 || L > D || D > DIIS_MAX) throw Error(1, "diis: k <= 16, 1 <= L <= D <= 16");
  k_diis_coef<<<1, 64, 0, s>>>(k, L, D, A, alpha);
  SPPC_LAUNCH_CHECK();
}

void diis_combine(int64_t n, int k, int L, int D, const double* alpha, const double* Xh, const double* HXh,
                  double* xb, double* hxb, hipStream_t s) {
  k_hist_combine<<<grid1(n * k), 256, 0, s>>>(n, k, L, D, alpha, Xh, HXh, xb, hxb);
  SPPC_LAUNCH_CHECK();
}

void columns_to_unit(int64_t n, int k, const double* ss, double* X, double* HX, hipStream_t s) {
  k_col_unit<<<grid1(n * k), 256, 0, s>>>(n, k, ss, X, HX);
  SPPC_LAUNCH_CHECK();
}

void min_residual_step(int64_t n, int k, const double* rd, const double* uu, const double* xb, const double* hxb,
                       const double* t, const double* ht, double* Xn, double* HXn, hipStream_t s) {
  k_col_step<<<grid1(n * k), 256, 0, s>>>(n, k, rd, uu, xb, hxb, t, ht, Xn, HXn);
  SPPC_LAUNCH_CHECK();
}

void gram_set(int k, int D, int i, int l, const double* g, double* A, hipStream_t s) {
  k_gram_set<<<1, 64, 0, s>>>(k, D, i, l, g, A);
  SPPC_LAUNCH_CHECK();
}

}  // namespace sppc
