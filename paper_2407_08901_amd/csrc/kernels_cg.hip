// kernels_cg.hip - the small-space solves of the perturbative correction (eq. sm_lin_proj).
//
// For every wanted pair c the singular system (H0hat - E_c) x = b_c - (b_c^T psi_c) psi_c is
// solved for its minimum-norm solution orthogonal to psi_c.  The D lowest eigenvectors of
// H0hat (Ps, n0 x D) are deflated: preconditioned CG runs on the complement, where
// H0hat - E_c is positive definite, and the deflated directions are added back exactly
// by the caller.  All k systems advance together, sharing one product with H0hat per
// iteration.
//
// The right-hand side is projected once onto the complement; H0hat - E_c maps the complement
// into itself (its deflated directions are eigenvectors), so plain CG iterates stay there and
// need only the k-wide dot products p.q and r.r per iteration.  The final x is projected once
// more to remove rounding drift.
//
// One iteration is two kernels; the kernel boundaries are the only grid-wide barriers.  Every
// block re-adds the previous kernel's per-block partial sums in the same fixed order, so the
// CG scalars are identical on all blocks and bit-reproducible.  The product kernel forms the
// new search direction p = r + beta p_old on the fly for every row it gathers (p is double
// buffered), so no separate direction update is needed.  Scalars are double-buffered by
// iteration parity; once no column is active every kernel returns at entry (the host polls
// the count every few iterations).
#include "common.h"

namespace sppc {

namespace {

constexpr int CG_MAXK = 16;
constexpr int CG_MAXD = 28;
constexpr int PW = 1024;       // partial width of the reduction phase (>= 2k + 2Dk)
constexpr int R1 = 16;         // rows per block of the product kernel
constexpr int CH = 64;         // rows per LDS chunk of the projections

// device scalars: [parity][...]
struct CGScal {
  double rr[2][CG_MAXK];
  double bb[CG_MAXK];
  int act[2][CG_MAXK];
  int nact[2];
  int iters;
};

struct CGArgs {
  int64_t n0;
  int k, D;
  const int64_t* rp;
  const int64_t* rend;
  const int32_t* col;
  const double* v64;
  const float* v32;
  const double* diag;
  const double* shift;  // E_c
  const double* Ps;     // n0 x D
  double *x, *r, *q;    // n0 x k
  double *pa, *pb;      // search directions, double-buffered
  double* part1;        // nb1 x k   (p.q)
  double* part2;        // nb2 x k   (r.r)
  double* partP;        // nb2 x Dk  (Ps^T y)
  int nb1, nb2;
  double* ccoef;        // D x k: Ps^T b (for the add-back)
  CGScal* sc;
  double tol2;
};

// tot[e] = sum_b part[b*stride + e] for e < w, fixed order (4 interleaved partial sums)
__device__ void reduce_parts(const double* __restrict__ part, int nb, int64_t stride, int w, double* tot) {
  for (int e = threadIdx.x; e < w; e += blockDim.x) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int b2 = 0;
    for (; b2 + 3 < nb; b2 += 4) {
      s0 += part[(int64_t)b2 * stride + e];
      s1 += part[(int64_t)(b2 + 1) * stride + e];
      s2 += part[(int64_t)(b2 + 2) * stride + e];
      s3 += part[(int64_t)(b2 + 3) * stride + e];
    }
    for (; b2 < nb; ++b2) s0 += part[(int64_t)b2 * stride + e];
    tot[e] = (s0 + s1) + (s2 + s3);
  }
  __syncthreads();
}

// tot[c] = sum_b part[b*CG_MAXK + c] for c < w <= CG_MAXK, all threads of the block: thread t
// sums the blocks b = t/16, t/16 + nt/16, ... of column t%16, then a fixed-order tree.
__device__ void reduce_cols(const double* __restrict__ part, int nb, int w, double* red, double* tot) {
  const int t = threadIdx.x, nt = blockDim.x;
  const int c = t % CG_MAXK;
  double s = 0.0;
  if (c < w)
    for (int b2 = t / CG_MAXK; b2 < nb; b2 += nt / CG_MAXK) s += part[(int64_t)b2 * CG_MAXK + c];
  red[t] = s;
  __syncthreads();
  for (int o = nt / 2; o >= CG_MAXK; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  if (t < w) tot[t] = red[t];
  __syncthreads();
}

// Column sums over rows [r0, r1) of X[r][c] * Y[r][c] -> out[c]; block of 1024 threads.
__device__ void block_coldot(const double* __restrict__ X, const double* __restrict__ Y, int64_t r0,
                             int64_t r1, int k, double* red, double* out) {
  const int t = threadIdx.x, nt = blockDim.x;
  const int tc = t % CG_MAXK, tr = t / CG_MAXK;
  double s = 0.0;
  if (tc < k)
    for (int64_t r = r0 + tr; r < r1; r += nt / CG_MAXK) s = fma(X[r * k + tc], Y[r * k + tc], s);
  red[t] = s;
  __syncthreads();
  for (int o = nt / 2; o >= CG_MAXK; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  if (t < k) out[t] = red[t];
  __syncthreads();
}

// Block partials over rows [r0, r1): Ps^T Y -> out[0 .. Dk) and, if psx, Ps^T X -> out[Dk .. 2Dk);
// rows staged through LDS (one output per thread, 2Dk <= 896 < 1024 threads).
__device__ void block_psT(const double* __restrict__ Ps, const double* __restrict__ X,
                          const double* __restrict__ Y, int64_t r0, int64_t r1, int D, int k, bool psx,
                          double* sh_ps, double* sh_x, double* sh_y, double* out) {
  const int t = threadIdx.x, nt = blockDim.x;
  const int Dk = D * k;
  const int nout = psx ? 2 * Dk : Dk;
  double acc = 0.0;
  const bool second = t >= Dk;
  const int ee = second ? t - Dk : t;
  const int d = ee / k, c = ee % k;
  for (int64_t c0 = r0; c0 < r1; c0 += CH) {
    const int nr = (int)min<int64_t>(CH, r1 - c0);
    for (int e = t; e < CH * CG_MAXD; e += nt) {
      const int rr = e / CG_MAXD, dd = e % CG_MAXD;
      sh_ps[e] = (rr < nr && dd < D) ? Ps[(c0 + rr) * D + dd] : 0.0;
    }
    for (int e = t; e < CH * CG_MAXK; e += nt) {
      const int rr = e / CG_MAXK, cc = e % CG_MAXK;
      const bool ok = rr < nr && cc < k;
      sh_x[e] = ok ? X[(c0 + rr) * k + cc] : 0.0;
      sh_y[e] = ok ? Y[(c0 + rr) * k + cc] : 0.0;
    }
    __syncthreads();
    if (t < nout) {
      const double* src = second ? sh_x : sh_y;
      for (int rr = 0; rr < nr; ++rr) acc = fma(sh_ps[rr * CG_MAXD + d], src[rr * CG_MAXK + c], acc);
    }
    __syncthreads();
  }
  if (t < nout) out[t] = acc;
}

inline __device__ void rows_of(int64_t n0, int blk, int nb, int64_t& r0, int64_t& r1) {
  r0 = n0 * blk / nb;
  r1 = n0 * (blk + 1) / nb;
}

// ---- partial Ps^T y over the rows of block b (nb2 blocks)
__global__ __launch_bounds__(1024) void k_cg_psT(CGArgs a, const double* Y) {
  __shared__ double sh_ps[CH * CG_MAXD], sh_x[CH * CG_MAXK], sh_y[CH * CG_MAXK];
  int64_t r0, r1;
  rows_of(a.n0, blockIdx.x, a.nb2, r0, r1);
  block_psT(a.Ps, Y, Y, r0, r1, a.D, a.k, false, sh_ps, sh_x, sh_y, a.partP + (int64_t)blockIdx.x * PW);
}

// ---- Y -= Ps (Ps^T Y) from the partials; optionally also: coef = Ps^T Y, zero X, r.r partials
__global__ __launch_bounds__(1024) void k_cg_project(CGArgs a, double* Y, double* coef, int start) {
  __shared__ double tot[PW], red[1024];
  const int k = a.k, D = a.D, Dk = D * k, t = threadIdx.x;
  reduce_parts(a.partP, a.nb2, PW, Dk, tot);
  if (coef && blockIdx.x == 0)
    for (int e = t; e < Dk; e += blockDim.x) coef[e] = tot[e];
  int64_t r0, r1;
  rows_of(a.n0, blockIdx.x, a.nb2, r0, r1);
  for (int64_t e = r0 * k + t; e < r1 * k; e += blockDim.x) {
    const int64_t row = e / k;
    const int c = (int)(e % k);
    double v = Y[e];
    for (int d = 0; d < D; ++d) v -= a.Ps[row * D + d] * tot[d * k + c];
    Y[e] = v;
    if (start) {
      a.x[e] = 0.0;
      a.pb[e] = 0.0;
    }
  }
  if (start) {
    __syncthreads();
    block_coldot(Y, Y, r0, r1, k, red, a.part2 + (int64_t)blockIdx.x * CG_MAXK);
  }
}

// ---- iteration, K1: beta, convergence; p = r + beta p_old (on the fly); q = (H0hat - E) p ;
//      partial p.q.  One wave per row.
template <int B, typename VT, bool F32P>
__global__ __launch_bounds__(256) void k_cg_spmm(CGArgs a, int par, int first, const double* __restrict__ pold,
                                                 double* __restrict__ pnew) {
  const int t = threadIdx.x;
  const int k = a.k;
  if (!first && a.sc->nact[par ^ 1] == 0) {
    if (blockIdx.x == 0 && t == 0) a.sc->nact[par] = 0;
    return;
  }
  __shared__ double tot[CG_MAXK], be[CG_MAXK], pqw[4][CG_MAXK], red[256];
  __shared__ int act[CG_MAXK];
  reduce_cols(a.part2, a.nb2, k, red, tot);
  if (t < k) {
    const double rrn = tot[t];
    const double rro = first ? rrn : a.sc->rr[par ^ 1][t];
    const double bb = first ? rrn : a.sc->bb[t];
    const int was = first ? (rrn > 0.0) : a.sc->act[par ^ 1][t];
    const int now = was && (rrn > a.tol2 * bb);
    act[t] = now;
    be[t] = (now && rro != 0.0) ? rrn / rro : 0.0;
    if (blockIdx.x == 0) {
      a.sc->rr[par][t] = now ? rrn : rro;
      a.sc->act[par][t] = now;
      if (first) a.sc->bb[t] = rrn;
    }
  }
  __syncthreads();
  if (blockIdx.x == 0 && t == 0) {
    int na = 0;
    for (int c = 0; c < k; ++c) na += act[c];
    a.sc->nact[par] = na;
    if (first) a.sc->iters = 0;
    if (na) a.sc->iters += 1;
  }
  constexpr int G = 64 / B;
  const int lane = t & 63, g = lane / B, cc = lane % B, w = t >> 6;
  const VT* val = sizeof(VT) == 8 ? (const VT*)a.v64 : (const VT*)a.v32;
  const bool ca = cc < k && act[cc < k ? cc : 0];
  const double bc = cc < k ? be[cc] : 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * R1, r1 = min<int64_t>(a.n0, r0 + R1);
  double pq = 0.0;
  for (int64_t row = r0 + w; row < r1; row += 4) {
    const int64_t beg = a.rp[row], end = a.rend ? a.rend[row] : a.rp[row + 1];
    double acc = 0.0;
    for (int64_t base = beg; base < end; base += 64) {
      const int cnt = (int)min<int64_t>(64, end - base);
      int32_t mc = 0;
      VT mv = VT(0);
      if (lane < cnt) { mc = a.col[base + lane]; mv = val[base + lane]; }
      for (int s0 = 0; s0 < cnt; s0 += G) {
        const int e = s0 + g;
        const int32_t cl = __shfl(mc, e);
        const VT vv = __shfl(mv, e);
        if (e < cnt && ca) {
          const int64_t o = (int64_t)cl * k + cc;
          const double pn = fma(bc, pold[o], a.r[o]);
          if constexpr (F32P) {
            acc += (double)((float)vv * (float)pn);  // float32 product, float64 accumulation
          } else {
            acc = fma((double)vv, pn, acc);
          }
        }
      }
    }
    for (int o = B; o < 64; o <<= 1) acc += __shfl_xor(acc, o);
    if (g == 0 && cc < k) {
      const int64_t o = row * k + cc;
      if (ca) {
        const double pv = fma(bc, pold[o], a.r[o]);
        const double qv = acc - a.shift[cc] * pv;
        pnew[o] = pv;
        a.q[o] = qv;
        pq = fma(pv, qv, pq);
      } else {
        pnew[o] = pold[o];
      }
    }
  }
  if (g == 0) pqw[w][cc] = pq;
  __syncthreads();
  if (t < k) a.part1[(int64_t)blockIdx.x * CG_MAXK + t] = (pqw[0][t] + pqw[1][t]) + (pqw[2][t] + pqw[3][t]);
}

// ---- iteration, K2: alpha ; x += alpha p ; r -= alpha q ; partial r.r
__global__ __launch_bounds__(1024) void k_cg_update(CGArgs a, int par, const double* __restrict__ p) {
  if (a.sc->nact[par] == 0) return;
  __shared__ double tot[CG_MAXK], red[1024], al[CG_MAXK];
  const int k = a.k, t = threadIdx.x;
  reduce_cols(a.part1, a.nb1, k, red, tot);
  if (t < k) {
    const double s = tot[t];
    al[t] = (a.sc->act[par][t] && s != 0.0) ? a.sc->rr[par][t] / s : 0.0;
  }
  __syncthreads();
  int64_t r0, r1;
  rows_of(a.n0, blockIdx.x, a.nb2, r0, r1);
  for (int64_t e = r0 * k + t; e < r1 * k; e += blockDim.x) {
    const double av = al[e % k];
    if (av != 0.0) {
      a.x[e] = fma(av, p[e], a.x[e]);
      a.r[e] = fma(-av, a.q[e], a.r[e]);
    }
  }
  __syncthreads();
  block_coldot(a.r, a.r, r0, r1, k, red, a.part2 + (int64_t)blockIdx.x * CG_MAXK);
}

}  // namespace

// doubles reserved for the device scalars (64-byte multiple)
constexpr int64_t SC_D = (int64_t)((sizeof(CGScal) + 63) / 64) * 8;

int64_t cg_work_doubles(int64_t n0) {
  const int64_t nb1 = cdiv(n0, R1), nb2 = std::min<int64_t>(256, cdiv(n0, 64));
  return nb1 * CG_MAXK + nb2 * CG_MAXK + nb2 * PW + SC_D + 2 * n0 * CG_MAXK;
}

// b in r (n0 x k) on entry; x returns the CG solution on the deflated complement and
// ccoef = Ps^T b.  Returns the number of iterations (synchronises the stream).
int cg_solve(const DevCSR& H0, int64_t n0, int k, int D, const double* diag, const double* shift,
             const double* Ps, double* x, double* r, double* z, double* p, double* q, double* work,
             double* ccoef, int maxit, double tol, bool f32prod, int* host_flag, hipStream_t s) {
  (void)diag;
  (void)z;
  (void)p;
  if (k < 1 || k > CG_MAXK || D < 1 || D > CG_MAXD) throw Error(1, "cg: k <= 16 and D <= 28 required");
  if (f32prod && !H0.val32) throw Error(1, "cg: float32 products need float32 values");
  const int nb1 = (int)cdiv(n0, R1);
  const int nb2 = (int)std::min<int64_t>(256, cdiv(n0, 64));
  double* part1 = work;
  double* part2 = part1 + (int64_t)nb1 * CG_MAXK;
  double* partP = part2 + (int64_t)nb2 * CG_MAXK;
  CGScal* sc = (CGScal*)(partP + (int64_t)nb2 * PW);
  double* pa = (double*)sc + SC_D;
  double* pb = pa + n0 * CG_MAXK;
  CGArgs a{n0, k, D, H0.rp, H0.rend, H0.col, H0.val64, H0.val32, diag, shift, Ps, x, r, q, pa, pb,
           part1, part2, partP, nb1, nb2, ccoef, sc, tol * tol};
  // r <- P b (ccoef = Ps^T b), x = 0, p_old = 0, partial r.r
  k_cg_psT<<<nb2, 1024, 0, s>>>(a, r);
  k_cg_project<<<nb2, 1024, 0, s>>>(a, r, ccoef, 1);
  SPPC_LAUNCH_CHECK();
  const bool f64 = H0.val64 != nullptr;
  int it = 0;
  for (it = 1; it <= maxit; ++it) {
    const int par = it & 1;
    const double* pold = (it & 1) ? pb : pa;
    double* pnew = (it & 1) ? pa : pb;
    const int first = it == 1;
#define SPPC_CG_LAUNCH(BB)                                                                     \
  if (f32prod) k_cg_spmm<BB, float, true><<<nb1, 256, 0, s>>>(a, par, first, pold, pnew);       \
  else if (f64) k_cg_spmm<BB, double, false><<<nb1, 256, 0, s>>>(a, par, first, pold, pnew);    \
  else k_cg_spmm<BB, float, false><<<nb1, 256, 0, s>>>(a, par, first, pold, pnew);
    if (k <= 4) {
      SPPC_CG_LAUNCH(4)
    } else if (k <= 8) {
      SPPC_CG_LAUNCH(8)
    } else {
      SPPC_CG_LAUNCH(16)
    }
#undef SPPC_CG_LAUNCH
    k_cg_update<<<nb2, 1024, 0, s>>>(a, par, pnew);
    if (it % 16 == 0 || it == maxit) {
      SPPC_LAUNCH_CHECK();
      SPPC_HIP(hipMemcpyAsync(host_flag, &sc->nact[par], sizeof(int), hipMemcpyDeviceToHost, s));
      SPPC_HIP(hipStreamSynchronize(s));
      if (*host_flag == 0) break;
    }
  }
  // x <- P x (removes the drift into the deflated directions)
  k_cg_psT<<<nb2, 1024, 0, s>>>(a, x);
  k_cg_project<<<nb2, 1024, 0, s>>>(a, x, nullptr, 0);
  SPPC_LAUNCH_CHECK();
  SPPC_HIP(hipMemcpyAsync(host_flag, &sc->iters, sizeof(int), hipMemcpyDeviceToHost, s));
  SPPC_HIP(hipStreamSynchronize(s));
  return *host_flag;
}

}  // namespace sppc
