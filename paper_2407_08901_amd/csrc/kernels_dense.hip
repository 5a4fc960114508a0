// kernels_dense.hip - tall-skinny dense passes over the basis (row-major, float64).
//
// Q and H Q are n x m_max row-major (the m used columns of a row are contiguous), so a
// row tile is a set of contiguous segments and a new block of columns can be read by
// the sparse product in place.  Reductions over rows write one partial per row chunk
// and are summed in a fixed order (deterministic results).
#include "common.h"

namespace sppc {

namespace {

// rows per partial sum in gemm_tn: enough chunks to fill the chip, at most 2048 rows each
inline int64_t tn_chunk(int64_t n) {
  int64_t c = (n / 512 + 31) / 32 * 32;
  return c < 32 ? 32 : (c > 2048 ? 2048 : c);
}
constexpr int TN_MT = 64;       // columns of A per block
constexpr int TN_RT = 32;       // rows per LDS tile

// partial[chunk][i][j] = sum_{r in chunk} A[r][i0+i] B[r][j]
__global__ __launch_bounds__(256) void k_gemm_tn(int64_t n, int m, int b, const double* __restrict__ A,
                                                 int64_t lda, const double* __restrict__ B, int64_t ldb,
                                                 double* __restrict__ part, int64_t chunk) {
  __shared__ double As[TN_RT][TN_MT];
  __shared__ double Bs[TN_RT][33];
  const int t = threadIdx.x;
  const int i = t & 63;
  const int jg = t >> 6;
  const int i0 = blockIdx.y * TN_MT;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = min<int64_t>(n, r0 + chunk);
  double acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0.0;
  for (int64_t rt = r0; rt < r1; rt += TN_RT) {
    const int nr = (int)min<int64_t>(TN_RT, r1 - rt);
#pragma unroll
    for (int q = 0; q < (TN_RT * TN_MT) / 256; ++q) {
      const int e = t + 256 * q;
      const int rr = e >> 6, ii = e & 63;
      double v = 0.0;
      if (rr < nr && i0 + ii < m) v = A[(rt + rr) * lda + i0 + ii];
      As[rr][ii] = v;
    }
    for (int e = t; e < TN_RT * 32; e += 256) {
      const int rr = e >> 5, jj = e & 31;
      double v = 0.0;
      if (rr < nr && jj < b) v = B[(rt + rr) * ldb + jj];
      Bs[rr][jj] = v;
    }
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < TN_RT; ++rr) {
      const double a = As[rr][i];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] = fma(a, Bs[rr][jg + 4 * q], acc[q]);
    }
    __syncthreads();
  }
  if (i0 + i < m) {
    double* out = part + ((int64_t)blockIdx.x * m + i0 + i) * b;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int j = jg + 4 * q;
      if (j < b) out[j] = acc[q];
    }
  }
}

// one wave per output element: lanes stride over the chunks, fixed-order tree sum
__global__ void k_reduce_partials(int64_t nchunks, int m, int b, const double* __restrict__ part,
                                  double* __restrict__ C, int64_t ldc, double alpha, double beta) {
  const int64_t e = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (e >= (int64_t)m * b) return;
  const int64_t mb = (int64_t)m * b;
  double s = 0.0;
  for (int64_t c = lane; c < nchunks; c += 64) s += part[c * mb + e];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) {
    const int i = (int)(e / b), j = (int)(e % b);
    double* dst = C + (int64_t)i * ldc + j;
    *dst = beta == 0.0 ? alpha * s : beta * (*dst) + alpha * s;
  }
}

constexpr int NN_RB = 64;  // rows per block
constexpr int NN_IT = 64;  // inner tile

__global__ __launch_bounds__(256) void k_gemm_nn(int64_t n, int m, int b, const double* __restrict__ A,
                                                 int64_t lda, const double* __restrict__ C, int64_t ldc,
                                                 double* __restrict__ Y, int64_t ldy, double alpha,
                                                 double beta) {
  __shared__ double As[NN_RB][NN_IT + 1];
  __shared__ double Cs[NN_IT][33];
  const int t = threadIdx.x;
  const int r = t >> 2;
  const int jq = t & 3;
  const int64_t row0 = (int64_t)blockIdx.x * NN_RB;
  const int nr = (int)min<int64_t>(NN_RB, n - row0);
  double acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0.0;
  for (int i0 = 0; i0 < m; i0 += NN_IT) {
    const int ni = min(NN_IT, m - i0);
#pragma unroll
    for (int q = 0; q < (NN_RB * NN_IT) / 256; ++q) {
      const int e = t + 256 * q;
      const int rr = e >> 6, ii = e & 63;
      double v = 0.0;
      if (rr < nr && ii < ni) v = A[(row0 + rr) * lda + i0 + ii];
      As[rr][ii] = v;
    }
    for (int e = t; e < NN_IT * 32; e += 256) {
      const int ii = e >> 5, jj = e & 31;
      double v = 0.0;
      if (ii < ni && jj < b) v = C[(int64_t)(i0 + ii) * ldc + jj];
      Cs[ii][jj] = v;
    }
    __syncthreads();
#pragma unroll 8
    for (int ii = 0; ii < NN_IT; ++ii) {
      const double a = As[r][ii];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] = fma(a, Cs[ii][jq + 4 * q], acc[q]);
    }
    __syncthreads();
  }
  if (r < nr) {
    double* y = Y + (row0 + r) * ldy;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int j = jq + 4 * q;
      if (j < b) y[j] = beta == 0.0 ? alpha * acc[q] : beta * y[j] + alpha * acc[q];
    }
  }
}

// ---------------------------------------------------------------- column reductions
// rows per partial sum of the column reductions
inline int64_t cr_chunk(int64_t n) {
  int64_t c = (n / 256 + 255) / 256 * 256;
  return c < 256 ? 256 : (c > 4096 ? 4096 : c);
}

// mode 0: sum X^2 ; mode 1: R = HZ - Z theta and sum R^2 ; mode 2: sum Z[:,idx[a]] * T[:,a]
template <int MODE>
__global__ __launch_bounds__(256) void k_colreduce(int64_t n, int b, const double* __restrict__ X,
                                                   int64_t ldx, const double* __restrict__ Y,
                                                   int64_t ldy, const double* __restrict__ theta,
                                                   const int* __restrict__ idx, double* __restrict__ R,
                                                   int64_t ldr, double* __restrict__ part, int64_t chunk) {
  __shared__ double sh[256];
  const int t = threadIdx.x;
  const int B2 = b <= 1 ? 1 : b <= 2 ? 2 : b <= 4 ? 4 : b <= 8 ? 8 : b <= 16 ? 16 : 32;
  const int tc = t % B2, tr = t / B2, nrt = 256 / B2;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = min<int64_t>(n, r0 + chunk);
  double s = 0.0;
  if (tc < b) {
    for (int64_t r = r0 + tr; r < r1; r += nrt) {
      double v;
      if (MODE == 0) {
        v = X[r * ldx + tc];
        s = fma(v, v, s);
      } else if (MODE == 1) {
        v = Y[r * ldy + tc] - X[r * ldx + tc] * theta[tc];
        R[r * ldr + tc] = v;
        s = fma(v, v, s);
      } else {
        s = fma(X[r * ldx + idx[tc]], Y[r * ldy + tc], s);
      }
    }
  }
  sh[t] = s;
  __syncthreads();
  for (int o = 128; o >= B2; o >>= 1) {
    if (t < o) sh[t] += sh[t + o];
    __syncthreads();
  }
  if (t < b) part[(int64_t)blockIdx.x * b + t] = sh[t];
}

// one wave per column, lanes stride over the chunks, fixed-order tree sum
__global__ void k_colreduce_final(int64_t nchunks, int b, const double* __restrict__ part,
                                  double* __restrict__ out) {
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= b) return;
  double s = 0.0;
  for (int64_t c = lane; c < nchunks; c += 64) s += part[c * b + j];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) out[j] = s;
}

__global__ void k_copy_block(int64_t n, int b, const double* __restrict__ X, int64_t ldx,
                             double* __restrict__ Y, int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * b) return;
  const int64_t r = e / b;
  const int c = (int)(e % b);
  Y[r * ldy + c] = X[r * ldx + c];
}

__global__ void k_copy_f32(int64_t n, int b, const double* __restrict__ X, int64_t ldx,
                           float* __restrict__ Y, int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * b) return;
  const int64_t r = e / b;
  const int c = (int)(e % b);
  Y[r * ldy + c] = (float)X[r * ldx + c];
}

__global__ void k_fill_zero(int64_t count, double* __restrict__ p) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = 0.0;
}

__global__ void k_complement(int64_t r0, int64_t n, int b, const double* __restrict__ W, int64_t ldw,
                             const double* __restrict__ E0, double* __restrict__ P, int64_t ldp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (n - r0) * b) return;
  const int64_t r = r0 + e / b;
  const int c = (int)(e % b);
  P[r * ldp + c] = W[r * ldw + c] / E0[c];
}

__global__ void k_axpby(int64_t n, int b, double a, const double* __restrict__ X, int64_t ldx,
                        double beta, double* __restrict__ Y, int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * b) return;
  const int64_t r = e / b;
  const int c = (int)(e % b);
  double* y = Y + r * ldy + c;
  *y = beta == 0.0 ? a * X[r * ldx + c] : a * X[r * ldx + c] + beta * (*y);
}

__global__ void k_jacobi(int64_t n, int na, const int* __restrict__ idx, const double* __restrict__ R,
                         int64_t ldr, const double* __restrict__ diag, const double* __restrict__ theta,
                         double* __restrict__ T, int64_t ldt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * na) return;
  const int64_t r = e / na;
  const int a = (int)(e % na);
  const int i = idx[a];
  const double th = theta[i];
  const double floor_ = 1e-2 * fmax(1.0, fabs(th));
  double den = diag[r] - th;
  if (fabs(den) < floor_) den = den >= 0.0 ? floor_ : -floor_;
  T[r * ldt + a] = R[r * ldr + i] / den;
}

__global__ void k_project_out(int64_t n, int na, const int* __restrict__ idx, const double* __restrict__ Z,
                              int64_t ldz, const double* __restrict__ dots, double* __restrict__ T,
                              int64_t ldt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * na) return;
  const int64_t r = e / na;
  const int a = (int)(e % na);
  double* t = T + r * ldt + a;
  *t = -(*t - Z[r * ldz + idx[a]] * dots[a]);
}

inline int64_t grid1(int64_t count) { return cdiv(count > 0 ? count : 1, 256); }

}  // namespace

int64_t gemm_tn_work(int64_t n, int m, int b) { return cdiv(n > 0 ? n : 1, tn_chunk(n)) * (int64_t)m * b; }

void gemm_tn(int64_t n, int m, int b, const double* A, int64_t lda, const double* B, int64_t ldb,
             double* C, int64_t ldc, double alpha, double beta, double* work, hipStream_t s) {
  if (m <= 0 || b <= 0) return;
  if (b > 32) throw Error(1, "gemm_tn: b must be <= 32");
  const int64_t chunk = tn_chunk(n);
  const int64_t nch = cdiv(n > 0 ? n : 1, chunk);
  if (n > 0) {
    dim3 grid((unsigned)nch, (unsigned)cdiv(m, TN_MT));
    k_gemm_tn<<<grid, 256, 0, s>>>(n, m, b, A, lda, B, ldb, work, chunk);
  } else {
    k_fill_zero<<<grid1((int64_t)m * b), 256, 0, s>>>((int64_t)m * b, work);
  }
  k_reduce_partials<<<cdiv((int64_t)m * b, 4), 256, 0, s>>>(nch, m, b, work, C, ldc, alpha, beta);
  SPPC_LAUNCH_CHECK();
}

void gemm_nn(int64_t n, int m, int b, const double* A, int64_t lda, const double* C, int64_t ldc,
             double* Y, int64_t ldy, double alpha, double beta, hipStream_t s) {
  if (n <= 0 || b <= 0) return;
  if (b > 32) throw Error(1, "gemm_nn: b must be <= 32");
  k_gemm_nn<<<cdiv(n, NN_RB), 256, 0, s>>>(n, m, b, A, lda, C, ldc, Y, ldy, alpha, beta);
  SPPC_LAUNCH_CHECK();
}

void copy_to_f32(int64_t n, int b, const double* X, int64_t ldx, float* Y, int64_t ldy, hipStream_t s) {
  k_copy_f32<<<grid1(n * b), 256, 0, s>>>(n, b, X, ldx, Y, ldy);
  SPPC_LAUNCH_CHECK();
}

void copy_block(int64_t n, int b, const double* X, int64_t ldx, double* Y, int64_t ldy, hipStream_t s) {
  if (n * b == 0) return;
  k_copy_block<<<grid1(n * b), 256, 0, s>>>(n, b, X, ldx, Y, ldy);
  SPPC_LAUNCH_CHECK();
}

void fill_zero(int64_t count, double* p, hipStream_t s) {
  if (count <= 0) return;
  k_fill_zero<<<grid1(count), 256, 0, s>>>(count, p);
  SPPC_LAUNCH_CHECK();
}

void residual_block(int64_t n, int b, const double* Z, int64_t ldz, const double* HZ, int64_t ldhz,
                    const double* theta, double* R, int64_t ldr, double* sumsq, double* work,
                    hipStream_t s) {
  const int64_t ch = cr_chunk(n), nch = cdiv(n > 0 ? n : 1, ch);
  k_colreduce<1><<<nch, 256, 0, s>>>(n, b, Z, ldz, HZ, ldhz, theta, nullptr, R, ldr, work, ch);
  k_colreduce_final<<<cdiv(b, 4), 256, 0, s>>>(nch, b, work, sumsq);
  SPPC_LAUNCH_CHECK();
}

void colsumsq(int64_t n, int b, const double* X, int64_t ldx, double* out, double* work, hipStream_t s) {
  const int64_t ch = cr_chunk(n), nch = cdiv(n > 0 ? n : 1, ch);
  k_colreduce<0><<<nch, 256, 0, s>>>(n, b, X, ldx, nullptr, 0, nullptr, nullptr, nullptr, 0, work, ch);
  k_colreduce_final<<<cdiv(b, 4), 256, 0, s>>>(nch, b, work, out);
  SPPC_LAUNCH_CHECK();
}

void paired_dots(int64_t n, int na, const int* idx, const double* Z, int64_t ldz, const double* T,
                 int64_t ldt, double* dots, double* work, hipStream_t s) {
  const int64_t ch = cr_chunk(n), nch = cdiv(n > 0 ? n : 1, ch);
  k_colreduce<2><<<nch, 256, 0, s>>>(n, na, Z, ldz, T, ldt, nullptr, idx, nullptr, 0, work, ch);
  k_colreduce_final<<<cdiv(na, 4), 256, 0, s>>>(nch, na, work, dots);
  SPPC_LAUNCH_CHECK();
}

void complement_rows(int64_t r0, int64_t n, int b, const double* W, int64_t ldw, const double* E0,
                     double* Psi, int64_t ldp, hipStream_t s) {
  if (n <= r0) return;
  k_complement<<<grid1((n - r0) * b), 256, 0, s>>>(r0, n, b, W, ldw, E0, Psi, ldp);
  SPPC_LAUNCH_CHECK();
}

void axpby_block(int64_t n, int b, double a, const double* X, int64_t ldx, double beta, double* Y,
                 int64_t ldy, hipStream_t s) {
  if (n * b == 0) return;
  k_axpby<<<grid1(n * b), 256, 0, s>>>(n, b, a, X, ldx, beta, Y, ldy);
  SPPC_LAUNCH_CHECK();
}

void jacobi_block(int64_t n, int na, const int* idx, const double* R, int64_t ldr, const double* diag,
                  const double* theta, double* T, int64_t ldt, hipStream_t s) {
  k_jacobi<<<grid1(n * na), 256, 0, s>>>(n, na, idx, R, ldr, diag, theta, T, ldt);
  SPPC_LAUNCH_CHECK();
}

void project_out_block(int64_t n, int na, const int* idx, const double* Z, int64_t ldz,
                       const double* dots, double* T, int64_t ldt, hipStream_t s) {
  k_project_out<<<grid1(n * na), 256, 0, s>>>(n, na, idx, Z, ldz, dots, T, ldt);
  SPPC_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- small-space solver helpers
namespace {

__global__ __launch_bounds__(256) void k_coldots(int64_t n, int b, const double* __restrict__ X,
                                                 int64_t ldx, const double* __restrict__ Y, int64_t ldy,
                                                 double* __restrict__ part, int64_t chunk) {
  __shared__ double sh[256];
  const int t = threadIdx.x;
  const int B2 = b <= 1 ? 1 : b <= 2 ? 2 : b <= 4 ? 4 : b <= 8 ? 8 : b <= 16 ? 16 : 32;
  const int tc = t % B2, tr = t / B2, nrt = 256 / B2;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = min<int64_t>(n, r0 + chunk);
  double s = 0.0;
  if (tc < b)
    for (int64_t r = r0 + tr; r < r1; r += nrt) s = fma(X[r * ldx + tc], Y[r * ldy + tc], s);
  sh[t] = s;
  __syncthreads();
  for (int o = 128; o >= B2; o >>= 1) {
    if (t < o) sh[t] += sh[t + o];
    __syncthreads();
  }
  if (t < b) part[(int64_t)blockIdx.x * b + t] = sh[t];
}

__global__ void k_cg_precond(int64_t n0, int k, const double* __restrict__ diag,
                             const double* __restrict__ shift, const double* __restrict__ r,
                             double* __restrict__ z) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n0 * k) return;
  const int64_t i = e / k;
  const int c = (int)(e % k);
  const double sh = shift[c];
  const double fl = 1e-2 * fmax(1.0, fabs(sh));
  const double den = fmax(fabs(diag[i] - sh), fl);
  z[e] = r[e] / den;
}

__global__ void k_cg_xr(int64_t n0, int k, double* __restrict__ x, double* __restrict__ r,
                        const double* __restrict__ p, const double* __restrict__ q,
                        const double* __restrict__ rz, const double* __restrict__ pq,
                        const int* __restrict__ active) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n0 * k) return;
  const int c = (int)(e % k);
  if (!active[c]) return;
  const double a = pq[c] != 0.0 ? rz[c] / pq[c] : 0.0;
  x[e] = fma(a, p[e], x[e]);
  r[e] = fma(-a, q[e], r[e]);
}

__global__ void k_cg_p(int64_t n0, int k, double* __restrict__ p, const double* __restrict__ z,
                       const double* __restrict__ rzn, const double* __restrict__ rzo,
                       const int* __restrict__ active) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n0 * k) return;
  const int c = (int)(e % k);
  if (!active[c]) return;
  const double bt = rzo[c] != 0.0 ? rzn[c] / rzo[c] : 0.0;
  p[e] = fma(bt, p[e], z[e]);
}

__global__ void k_cg_check(int k, const double* __restrict__ rr, const double* __restrict__ bb,
                           double tol2, int* __restrict__ active, int* __restrict__ nactive,
                           double* __restrict__ rzn, double* __restrict__ rzo) {
  if (threadIdx.x != 0) return;
  int na = 0;
  for (int c = 0; c < k; ++c) {
    if (active[c] && !(rr[c] > tol2 * bb[c])) active[c] = 0;
    na += active[c];
  }
  *nactive = na;
  if (rzn) for (int c = 0; c < k; ++c) rzo[c] = rzn[c];
}

__global__ void k_cg_init(int k, const double* __restrict__ bb, int* __restrict__ active,
                          int* __restrict__ nactive) {
  if (threadIdx.x != 0) return;
  int na = 0;
  for (int c = 0; c < k; ++c) {
    active[c] = bb[c] > 0.0;
    na += active[c];
  }
  *nactive = na;
}

}  // namespace

void coldots(int64_t n, int b, const double* X, int64_t ldx, const double* Y, int64_t ldy, double* out,
             double* work, hipStream_t s) {
  const int64_t ch = cr_chunk(n), nch = cdiv(n > 0 ? n : 1, ch);
  k_coldots<<<nch, 256, 0, s>>>(n, b, X, ldx, Y, ldy, work, ch);
  k_colreduce_final<<<cdiv(b, 4), 256, 0, s>>>(nch, b, work, out);
  SPPC_LAUNCH_CHECK();
}

void cg_precond(int64_t n0, int k, const double* diag, const double* shift, const double* r, double* z,
                hipStream_t s) {
  k_cg_precond<<<grid1(n0 * k), 256, 0, s>>>(n0, k, diag, shift, r, z);
  SPPC_LAUNCH_CHECK();
}

void cg_update_xr(int64_t n0, int k, double* x, double* r, const double* p, const double* q,
                  const double* rz, const double* pq, const int* active, hipStream_t s) {
  k_cg_xr<<<grid1(n0 * k), 256, 0, s>>>(n0, k, x, r, p, q, rz, pq, active);
  SPPC_LAUNCH_CHECK();
}

void cg_update_p(int64_t n0, int k, double* p, const double* z, const double* rzn, const double* rzo,
                 const int* active, hipStream_t s) {
  k_cg_p<<<grid1(n0 * k), 256, 0, s>>>(n0, k, p, z, rzn, rzo, active);
  SPPC_LAUNCH_CHECK();
}

void cg_check(int k, const double* rr, const double* bb, double tol2, int* active, int* nactive,
              double* rzn, double* rzo, hipStream_t s) {
  k_cg_check<<<1, 64, 0, s>>>(k, rr, bb, tol2, active, nactive, rzn, rzo);
  SPPC_LAUNCH_CHECK();
}

void cg_init(int k, const double* bb, int* active, int* nactive, hipStream_t s) {
  k_cg_init<<<1, 64, 0, s>>>(k, bb, active, nactive);
  SPPC_LAUNCH_CHECK();
}

namespace {
__global__ void k_gather_cols(int64_t n, int S, const int* __restrict__ idx, const double* __restrict__ X,
                              int64_t ldx, double* __restrict__ Y, int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * S) return;
  const int64_t r = e / S;
  const int a = (int)(e % S);
  Y[r * ldy + a] = X[r * ldx + idx[a]];
}

__global__ void k_scatter_cols(int64_t n, int S, const int* __restrict__ idx, const double* __restrict__ X,
                               int64_t ldx, double* __restrict__ Y, int64_t ldy, double alpha) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * S) return;
  const int64_t r = e / S;
  const int a = (int)(e % S);
  const int j = idx[a];
  if (j >= 0) Y[r * ldy + j] = alpha * X[r * ldx + a];
}

__global__ void k_zero_block(int64_t n, int b, double* __restrict__ Y, int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * b) return;
  Y[(e / b) * ldy + (e % b)] = 0.0;
}
}  // namespace

void gather_cols(int64_t n, int S, const int* idx, const double* X, int64_t ldx, double* Y, int64_t ldy,
                 hipStream_t s) {
  k_gather_cols<<<grid1(n * S), 256, 0, s>>>(n, S, idx, X, ldx, Y, ldy);
  SPPC_LAUNCH_CHECK();
}

void scatter_cols(int64_t n, int S, const int* idx, const double* X, int64_t ldx, double* Y, int64_t ldy,
                  double alpha, hipStream_t s) {
  k_scatter_cols<<<grid1(n * S), 256, 0, s>>>(n, S, idx, X, ldx, Y, ldy, alpha);
  SPPC_LAUNCH_CHECK();
}

void fill_block_zero(int64_t n, int b, double* Y, int64_t ldy, hipStream_t s) {
  if (n * b == 0) return;
  k_zero_block<<<grid1(n * b), 256, 0, s>>>(n, b, Y, ldy);
  SPPC_LAUNCH_CHECK();
}

}  // namespace sppc
