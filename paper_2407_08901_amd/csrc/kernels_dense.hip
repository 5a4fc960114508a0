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
// ---------------------------------------------------------------- MFMA tall-skinny products
// v_mfma_f64_16x16x4f64 (wave64): lane l supplies A[l%16][l/16] and B[l/16][l%16] of a
// 16x4 by 4x16 product and holds D[l/16 + 4v][l%16], v = 0..3, of the 16x16 accumulator.
typedef double v2d __attribute__((ext_vector_type(2)));
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ inline v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int TN_COLS = 64;  // columns of A per workgroup (4 tiles of 16)

// partial[chunk][i][j] = sum_{r in chunk} A[r][i] B[r][j] for the 64 columns i of blockIdx.y.
// The reduction dimension of the MFMA is the row index: each wave takes 4 rows per step
// (rows r0 + 16 t + 4 w .. +3 for wave w), 4 column tiles of A and NT column tiles of B.
template <int NT>
__global__ __launch_bounds__(256) void k_gemm_tn(int64_t n, int m, int b, const double* __restrict__ A,
                                                 int64_t lda, const double* __restrict__ B, int64_t ldb,
                                                 double* __restrict__ part, int64_t chunk) {
  __shared__ double red[2][64][16 * NT];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int rl = lane >> 4, cl = lane & 15;
  const int i0 = blockIdx.y * TN_COLS;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = min<int64_t>(n, r0 + chunk);
  v4d acc[4][NT];
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) acc[ti][tj] = v4d{0.0, 0.0, 0.0, 0.0};
  bool icol[4];
#pragma unroll
  for (int ti = 0; ti < 4; ++ti) icol[ti] = i0 + 16 * ti + cl < m;
  bool jcol[NT];
#pragma unroll
  for (int tj = 0; tj < NT; ++tj) jcol[tj] = 16 * tj + cl < b;
  for (int64_t rt = r0; rt < r1; rt += 32) {
    double a[2][4], bv[2][NT];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t r = rt + 16 * u + 4 * w + rl;
      const bool rin = r < r1;
      const double* ar = A + r * lda + i0 + cl;
      const double* br = B + r * ldb + cl;
#pragma unroll
      for (int ti = 0; ti < 4; ++ti) a[u][ti] = (rin && icol[ti]) ? ar[16 * ti] : 0.0;
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) bv[u][tj] = (rin && jcol[tj]) ? br[16 * tj] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < NT; ++tj) acc[ti][tj] = mfma16(a[u][ti], bv[u][tj], acc[ti][tj]);
  }
  // sum the 4 waves' accumulators in a fixed order: (w0 + w2) + (w1 + w3)
  for (int ti = 0; ti < 4; ++ti) {
    if (w >= 2) {
#pragma unroll
      for (int tj = 0; tj < NT; ++tj)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[w - 2][lane][tj * 4 + v] = acc[ti][tj][v];
    }
    __syncthreads();
    if (w < 2) {
#pragma unroll
      for (int tj = 0; tj < NT; ++tj)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[ti][tj][v] += red[w][lane][tj * 4 + v];
    }
    __syncthreads();
    if (w == 1) {
#pragma unroll
      for (int tj = 0; tj < NT; ++tj)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[0][lane][tj * 4 + v] = acc[ti][tj][v];
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) {
        const int j = 16 * tj + cl;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + 16 * ti + rl + 4 * v;
          if (i < m && j < b)
            part[((int64_t)blockIdx.x * m + i) * b + j] = acc[ti][tj][v] + red[0][lane][tj * 4 + v];
        }
      }
    }
    __syncthreads();
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

constexpr int NN_ROWS = 128;  // rows per workgroup: 4 waves x 2 tiles of 16

// Y = beta Y + alpha A C: the reduction dimension of the MFMA is the column index i of A.  In
// step st of a 16-column slab, k-slot q of the MFMA is column i0 + 4 q + st when the rows of A
// allow 32-byte loads (VEC: a lane reads its 4 columns of a row at once), else i0 + 4 st + q.
// Columns j >= split of the product go to Y2 (column j - split, ld ldy2, beta2) instead, so that
// two products with the same A share its pass.
template <int NT, bool VEC>
__global__ __launch_bounds__(256) void k_gemm_nn(int64_t n, int m, int b, const double* __restrict__ A,
                                                 int64_t lda, const double* __restrict__ C, int64_t ldc,
                                                 double* __restrict__ Y, int64_t ldy, double alpha,
                                                 double beta, int split, double* __restrict__ Y2,
                                                 int64_t ldy2, double beta2) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int q = lane >> 4, cl = lane & 15;
  const int64_t rbase = (int64_t)blockIdx.x * NN_ROWS + 32 * w;
  v4d acc[2][NT];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) acc[mt][tj] = v4d{0.0, 0.0, 0.0, 0.0};
  bool rin[2];
  const double* arow[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const int64_t r = rbase + 16 * mt + cl;
    rin[mt] = r < n;
    arow[mt] = A + (rin[mt] ? r : 0) * lda;
  }
  bool jcol[NT];
#pragma unroll
  for (int tj = 0; tj < NT; ++tj) jcol[tj] = 16 * tj + cl < b;
  for (int i0 = 0; i0 < m; i0 += 16) {
    double a[4][2], c[4][NT];
    if constexpr (VEC) {
      // slot q of step st is column i0 + 4 q + st: a lane's 4 columns of a row are one 32-byte
      // load, and the 16 columns of a row one 128-byte segment (lda >= m rounded up to 16)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        const v2d lo = rin[mt] ? *(const v2d*)(arow[mt] + i0 + 4 * q) : v2d{0.0, 0.0};
        const v2d hi = rin[mt] ? *(const v2d*)(arow[mt] + i0 + 4 * q + 2) : v2d{0.0, 0.0};
        a[0][mt] = lo.x;
        a[1][mt] = lo.y;
        a[2][mt] = hi.x;
        a[3][mt] = hi.y;
      }
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int i = i0 + 4 * q + st;
        const bool iin = i < m;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) a[st][mt] = iin ? a[st][mt] : 0.0;
#pragma unroll
        for (int tj = 0; tj < NT; ++tj)
          c[st][tj] = (iin && jcol[tj]) ? C[(int64_t)i * ldc + 16 * tj + cl] : 0.0;
      }
    } else {
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int i = i0 + 4 * st + q;
        const bool iin = i < m;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) a[st][mt] = (iin && rin[mt]) ? arow[mt][i] : 0.0;
#pragma unroll
        for (int tj = 0; tj < NT; ++tj)
          c[st][tj] = (iin && jcol[tj]) ? C[(int64_t)i * ldc + 16 * tj + cl] : 0.0;
      }
    }
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int tj = 0; tj < NT; ++tj) acc[mt][tj] = mfma16(a[st][mt], c[st][tj], acc[mt][tj]);
  }
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) {
      const int j = 16 * tj + cl;
      if (j >= b) continue;
      const bool second = j >= split;
      double* const yb = second ? Y2 + (j - split) : Y + j;
      const int64_t ld = second ? ldy2 : ldy;
      const double bt = second ? beta2 : beta;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = rbase + 16 * mt + q + 4 * v;
        if (r < n) {
          double* y = yb + r * ld;
          *y = bt == 0.0 ? alpha * acc[mt][tj][v] : bt * (*y) + alpha * acc[mt][tj][v];
        }
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

// Y1[:, c] = X1[:, c] and Y2[:, c] = X2[:, c] for the columns c whose bit is set in mask (leading
// dimension ld for all four): one pass over the rows, whatever the number of columns
__global__ void k_copy_cols2(int64_t n, int b, uint32_t mask, const double* __restrict__ X1,
                             double* __restrict__ Y1, const double* __restrict__ X2, double* __restrict__ Y2,
                             int64_t ld) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * b) return;
  const int c = (int)(e % b);
  if (!((mask >> c) & 1u)) return;
  const int64_t o = (e / b) * ld + c;
  Y1[o] = X1[o];
  Y2[o] = X2[o];
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
    dim3 grid((unsigned)nch, (unsigned)cdiv(m, TN_COLS));
    if (b <= 16)
      k_gemm_tn<1><<<grid, 256, 0, s>>>(n, m, b, A, lda, B, ldb, work, chunk);
    else
      k_gemm_tn<2><<<grid, 256, 0, s>>>(n, m, b, A, lda, B, ldb, work, chunk);
  } else {
    k_fill_zero<<<grid1((int64_t)m * b), 256, 0, s>>>((int64_t)m * b, work);
  }
  k_reduce_partials<<<cdiv((int64_t)m * b, 4), 256, 0, s>>>(nch, m, b, work, C, ldc, alpha, beta);
  SPPC_LAUNCH_CHECK();
}

namespace {
void gemm_nn_launch(int64_t n, int m, int b, const double* A, int64_t lda, const double* C, int64_t ldc,
                    double* Y, int64_t ldy, double alpha, double beta, int split, double* Y2, int64_t ldy2,
                    double beta2, hipStream_t s) {
  if (n <= 0 || b <= 0) return;
  if (b > 32) throw Error(1, "gemm_nn: b must be <= 32");
  // 32-byte row loads when the rows of A are 32-byte aligned and hold m rounded up to 16 columns
  const bool vec = lda % 4 == 0 && ((uintptr_t)A & 31) == 0 && lda >= (int64_t)((m + 15) / 16) * 16;
  const unsigned g = (unsigned)cdiv(n, NN_ROWS);
  if (b <= 16) {
    if (vec) k_gemm_nn<1, true><<<g, 256, 0, s>>>(n, m, b, A, lda, C, ldc, Y, ldy, alpha, beta, split, Y2, ldy2, beta2);
    else k_gemm_nn<1, false><<<g, 256, 0, s>>>(n, m, b, A, lda, C, ldc, Y, ldy, alpha, beta, split, Y2, ldy2, beta2);
  } else {
    if (vec) k_gemm_nn<2, true><<<g, 256, 0, s>>>(n, m, b, A, lda, C, ldc, Y, ldy, alpha, beta, split, Y2, ldy2, beta2);
    else k_gemm_nn<2, false><<<g, 256, 0, s>>>(n, m, b, A, lda, C, ldc, Y, ldy, alpha, beta, split, Y2, ldy2, beta2);
  }
  SPPC_LAUNCH_CHECK();
}
}  // namespace

void gemm_nn(int64_t n, int m, int b, const double* A, int64_t lda, const double* C, int64_t ldc,
             double* Y, int64_t ldy, double alpha, double beta, hipStream_t s) {
  gemm_nn_launch(n, m, b, A, lda, C, ldc, Y, ldy, alpha, beta, b, nullptr, 0, 0.0, s);
}

void gemm_nn2(int64_t n, int m, int b1, int b2, const double* A, int64_t lda, const double* C, int64_t ldc,
              double* Y1, int64_t ldy1, double beta1, double* Y2, int64_t ldy2, double beta2, hipStream_t s) {
  if (b1 < 1 || b2 < 1) throw Error(1, "gemm_nn2: both parts need columns");
  gemm_nn_launch(n, m, b1 + b2, A, lda, C, ldc, Y1, ldy1, 1.0, beta1, b1, Y2, ldy2, beta2, s);
}

void copy_to_f32(int64_t n, int b, const double* X, int64_t ldx, float* Y, int64_t ldy, hipStream_t s) {
  k_copy_f32<<<grid1(n * b), 256, 0, s>>>(n, b, X, ldx, Y, ldy);
  SPPC_LAUNCH_CHECK();
}

void copy_cols2(int64_t n, int b, uint32_t mask, const double* X1, double* Y1, const double* X2, double* Y2,
                int64_t ld, hipStream_t s) {
  if (n * b == 0 || mask == 0) return;
  if (b > 32 || ld < b) throw Error(1, "copy_cols2: at most 32 columns within the leading dimension");
  k_copy_cols2<<<grid1(n * b), 256, 0, s>>>(n, b, mask, X1, Y1, X2, Y2, ld);
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


}  // namespace

void coldots(int64_t n, int b, const double* X, int64_t ldx, const double* Y, int64_t ldy, double* out,
             double* work, hipStream_t s) {
  const int64_t ch = cr_chunk(n), nch = cdiv(n > 0 ? n : 1, ch);
  k_coldots<<<nch, 256, 0, s>>>(n, b, X, ldx, Y, ldy, work, ch);
  k_colreduce_final<<<cdiv(b, 4), 256, 0, s>>>(nch, b, work, out);
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
