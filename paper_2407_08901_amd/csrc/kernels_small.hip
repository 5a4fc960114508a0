// kernels_small.hip - single-workgroup kernels on the small matrices of the method:
// the projected matrix T = Q^T H Q and its lowest eigenpairs (Rayleigh-Ritz, eq. tilde_H),
// the Cholesky factors of the block QR (eq. QR), and the coefficient bookkeeping of the
// perturbative recursion (eq. exp_seq, eq. exp_seq2).
#include "common.h"

namespace sppc {

namespace {

constexpr int EIG_THREADS = 1024;
constexpr int EIG_LDS_M = 128;

__device__ inline double block_sum(double v, double* sh) {
  // sh: >= 16 doubles; all threads of the (1024-thread) block call this
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = blockDim.x >> 6;
  for (int i = 0; i < nw; ++i) s += sh[i];
  return s;
}

// Sum over the 64 lanes of a wave, returned to every lane, with DPP moves instead of the
// LDS-routed lane shuffles (about 100 cycles of dependent latency instead of about 900):
// prefix sums within rows of 16 lanes (shifts 1, 2, 4, 8; lanes without a source add 0), then
// lane 15 of rows 0 and 2 into rows 1 and 3, lane 31 into rows 2 and 3, and lane 63 is read.
template <int CTRL, int ROWS>
__device__ inline double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, true);
  return __hiloint2double(hi, lo);
}
__device__ inline double wave_sum(double v) {
  v += dpp_move<0x111, 0xF>(v);  // row_shr:1
  v += dpp_move<0x112, 0xF>(v);  // row_shr:2
  v += dpp_move<0x114, 0xF>(v);  // row_shr:4
  v += dpp_move<0x118, 0xF>(v);  // row_shr:8
  v += dpp_move<0x142, 0xA>(v);  // row_bcast:15 into rows 1, 3
  v += dpp_move<0x143, 0xC>(v);  // row_bcast:31 into rows 2, 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// a / b from the hardware reciprocal refined by one Newton-Raphson step, a few ulp from the
// rounded quotient: the Sturm counts and the shifted solves of inverse iteration sit on long
// chains of dependent divisions and do not need the correctly rounded one.  b is nonzero and
// finite at every call (both callers clamp their pivots away from zero); below 1e-290 the
// reciprocal could overflow, and the plain division is taken.
__device__ inline double quick_div(double a, double b) {
  if (fabs(b) < 1e-290) return a / b;
  double r = __builtin_amdgcn_rcp(b);
  r = fma(r, fma(-b, r, 1.0), r);
  return a * r;
}

// Sturm count: number of eigenvalues of the tridiagonal (d, e) smaller than x.  The pivots are
// kept at least 1e-290 in magnitude, so the reciprocal needs no guard.
__device__ inline double rcp_div(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(r, fma(-b, r, 1.0), r);
  return a * r;
}
__device__ int sturm_count(int m, const double* d, const double* e2, double x, double pivmin) {
  pivmin = fmax(pivmin, 1e-290);
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  int i = 1;
  // the operands of 8 steps are loaded ahead of the dependent chain
  for (; i + 8 <= m; i += 8) {
    double dd[8], ee[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      dd[u] = d[i + u] - x;
      ee[u] = e2[i + u - 1];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      q = dd[u] - rcp_div(ee[u], q);
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
    }
  }
  for (; i < m; ++i) {
    q = d[i] - x - rcp_div(e2[i - 1], q);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// Solve (Tri - lam I) y = y in place by Gaussian elimination with partial pivoting on the
// tridiagonal (two superdiagonals appear after interchanges).  Work arrays u0,u1,u2,l [m], piv [m].
__device__ void tri_shifted_solve(int m, const double* d, const double* e, double lam, double epsp,
                                  double* u0, double* u1, double* u2, double* l, unsigned char* piv,
                                  double* y, bool factor) {
  if (factor) {
    double ca = d[0] - lam;
    double cb = m > 1 ? e[0] : 0.0;
    for (int k = 0; k < m - 1; ++k) {
      const double sub = e[k];
      const double na = d[k + 1] - lam;
      const double nb = (k + 1 < m - 1) ? e[k + 1] : 0.0;
      if (fabs(ca) >= fabs(sub)) {
        if (ca == 0.0) ca = epsp;
        const double mult = quick_div(sub, ca);
        u0[k] = ca; u1[k] = cb; u2[k] = 0.0; l[k] = mult; piv[k] = 0;
        ca = na - mult * cb;
        cb = nb;
      } else {
        const double mult = quick_div(ca, sub);
        u0[k] = sub; u1[k] = na; u2[k] = nb; l[k] = mult; piv[k] = 1;
        ca = cb - mult * na;
        cb = -mult * nb;
      }
    }
    if (fabs(ca) < epsp) ca = ca >= 0.0 ? epsp : -epsp;
    u0[m - 1] = ca;
    for (int k = 0; k < m - 1; ++k)
      if (fabs(u0[k]) < epsp) u0[k] = u0[k] >= 0.0 ? epsp : -epsp;
  }
  for (int k = 0; k < m - 1; ++k) {
    if (piv[k]) {
      const double t = y[k];
      y[k] = y[k + 1];
      y[k + 1] = t;
    }
    y[k + 1] -= l[k] * y[k];
  }
  y[m - 1] = quick_div(y[m - 1], u0[m - 1]);
  if (m >= 2) y[m - 2] = quick_div(y[m - 2] - u1[m - 2] * y[m - 1], u0[m - 2]);
  for (int k = m - 3; k >= 0; --k) y[k] = quick_div(y[k] - u1[k] * y[k + 1] - u2[k] * y[k + 2], u0[k]);
}

__device__ void normalize(int m, double* y) {
  double s = 0.0, mx = 0.0;
  for (int i = 0; i < m; ++i) mx = fmax(mx, fabs(y[i]));
  if (mx == 0.0) return;
  const double rmx = 1.0 / mx;
  for (int i = 0; i < m; ++i) { y[i] *= rmx; s += y[i] * y[i]; }
  s = 1.0 / sqrt(s);
  for (int i = 0; i < m; ++i) y[i] *= s;
}

// scratch layout (doubles): A[m*m] | d[m] | e[m] | e2[m] | beta[m] | Y[nw*m] | u0,u1,u2,l [nw*m each] | piv
__global__ __launch_bounds__(EIG_THREADS) void k_sym_eig(int m, int nw, const double* __restrict__ S,
                                                         int64_t lds, double* __restrict__ wout,
                                                         double* __restrict__ V, int64_t ldv,
                                                         double* __restrict__ scr) {
  __shared__ double vsh[512];
  __shared__ double vsh2[512];
  __shared__ double psh[4][512];
  __shared__ double wsh[512];
  __shared__ double red[16];
  __shared__ double sc[4];
  __shared__ double Alds[EIG_LDS_M * EIG_LDS_M];  // the working matrix when it fits
  // d, e and beta of the steps taken in LDS (j >= o): a global store in the step would make the
  // next barrier wait for it
  __shared__ double dej[3][EIG_LDS_M];
  const int t = threadIdx.x;
  double* A = scr;  // the working matrix in global memory (ld m) while it does not fit in LDS
  double* d = scr + (int64_t)m * m;
  double* e = d + m;
  double* e2 = e + m;
  double* beta = e2 + m;
  double* Y = beta + m;
  double* u0 = Y + (int64_t)nw * m;
  double* u1 = u0 + (int64_t)nw * m;
  double* u2 = u1 + (int64_t)nw * m;
  double* lm = u2 + (int64_t)nw * m;
  unsigned char* piv = (unsigned char*)(lm + (int64_t)nw * m);

  // Rows and columns >= o live in LDS (stride EIG_LDS_M); the rest in global memory (stride m).
  // Step j of the reduction touches only [j, m)^2, so the trailing block moves to LDS once it fits
  // and every later step (and the Householder vectors it stores) stays there.
  // (2-D loops throughout: rows by thread group, columns by lane, so no index is divided)
  const int tg = t >> 8, tc = t & 255;
  int o = m;
  if (m <= EIG_LDS_M) {
    for (int r = tg; r < m; r += EIG_THREADS / 256)
      for (int c = tc; c < m; c += 256) Alds[r * EIG_LDS_M + c] = S[(int64_t)r * lds + c];
    o = 0;
  } else {
    for (int r = tg; r < m; r += EIG_THREADS / 256)
      for (int c = tc; c < m; c += 256) A[(int64_t)r * m + c] = S[(int64_t)r * lds + c];
  }
  __syncthreads();

  // ---- Householder tridiagonalisation (the lower part; A stays symmetric)
  // The rank-2 update of step j - 1 is not applied in a pass of its own: step j applies it to
  // row j as it forms its Householder vector, and to the rest of the trailing block in the same
  // pass that forms A v (each element read and written once per step instead of read twice and
  // written once, and one barrier less); the last 2 x 2 block takes the last step's update at
  // the end.  up/wsh hold v and w of step j - 1 (index 0 = row j), vc the vector of step j.
  bool pend = false;
  for (int j = 0; j + 2 < m; ++j) {
    double* const vc = (j & 1) ? vsh2 : vsh;
    const double* const up = (j & 1) ? vsh : vsh2;
    if (o > j && m - j <= EIG_LDS_M) {
      // the trailing block moves to LDS, with the pending update of step j - 1
      const int len0 = m - j;
      for (int r = tg; r < len0; r += EIG_THREADS / 256) {
        const double ur = pend ? up[r] : 0.0, wr = pend ? wsh[r] : 0.0;
        for (int c = tc; c < len0; c += 256)
          Alds[r * EIG_LDS_M + c] = A[(int64_t)(j + r) * m + j + c] - (ur * wsh[c] + wr * up[c]);
      }
      __syncthreads();
      o = j;
      pend = false;
    }
    double* const base = j >= o ? Alds : A;
    const int ld = j >= o ? EIG_LDS_M : m;
    const int off = j >= o ? o : 0;
    const int len = m - 1 - j;
    // row j, columns j+1.. == column j below the diagonal (with the pending update).  Wave 0 forms
    // the Householder vector alone (no block-wide reduction), the other waves wait at the barrier.
    const double* xr = base + (int64_t)(j - off) * ld + (j + 1 - off);
    if (t < 64) {
      const double u0 = pend ? up[0] : 0.0, w0 = pend ? wsh[0] : 0.0;
      double part = 0.0;
      for (int i = 1 + t; i < len; i += 64) {
        const double x = xr[i] - (u0 * wsh[1 + i] + w0 * up[1 + i]);
        part += x * x;
      }
      part = wave_sum(part);
      const double sigma = part;
      const double alpha = xr[0] - (u0 * wsh[1] + w0 * up[1]);
      double b = 0.0, v0 = 1.0, ej = alpha;
      if (sigma > 0.0) {
        const double mu = sqrt(alpha * alpha + sigma);
        v0 = alpha <= 0.0 ? alpha - mu : -sigma / (alpha + mu);
        b = 2.0 * v0 * v0 / (sigma + v0 * v0);
        ej = mu;
      }
      if (t == 0) {
        const double dj = base[(int64_t)(j - off) * ld + (j - off)] - 2.0 * u0 * w0;
        if (j >= o) {
          dej[0][j - o] = dj;
          dej[1][j - o] = ej;
          dej[2][j - o] = b;
        } else {
          d[j] = dj;
          e[j] = ej;
          beta[j] = b;
        }
        sc[0] = b;
      }
      const double rv0 = 1.0 / v0;
      for (int i = t; i < len; i += 64) {
        const double x = i == 0 ? alpha : xr[i] - (u0 * wsh[1 + i] + w0 * up[1 + i]);
        vc[i] = i == 0 ? 1.0 : (b == 0.0 ? 0.0 : x * rv0);
      }
    }
    __syncthreads();
    const double b = sc[0];
    // keep v for the back-transformation in row j (no longer needed otherwise)
    for (int i = t; i < len; i += EIG_THREADS) base[(int64_t)(j - off) * ld + (j + 1 - off) + i] = vc[i];
    if (j >= o) {
      // trailing block in LDS (len <= 128): apply the pending update of step j - 1 and form
      // p = b * A_tr v in one pass.  Thread (lg, i) owns column i and the rows l = lg mod 8;
      // p_i in 8 partial sums
      const int i = t & 127, lg = t >> 7;
      double* pp = &psh[0][0];  // [8][128]
      double* ci = base + (int64_t)(j + 1 - off) * ld + (j + 1 - off) + i;
      if (i < len) {
        double s0 = 0.0;
        if (pend) {
          const double ui = up[1 + i], wi = wsh[1 + i];
          for (int l = lg; l < len; l += 8) {
            const double a0 = ci[(int64_t)l * ld] - (up[1 + l] * wi + wsh[1 + l] * ui);
            ci[(int64_t)l * ld] = a0;
            s0 += a0 * vc[l];
          }
        } else {
          for (int l = lg; l < len; l += 8) s0 += ci[(int64_t)l * ld] * vc[l];
        }
        pp[lg * 128 + i] = s0;
      }
      __syncthreads();  // every read of the previous step's w is done
      if (t < 64) {
        double kp = 0.0;
        for (int i2 = t; i2 < len; i2 += 64) {
          double pi = 0.0;
#pragma unroll
          for (int g8 = 0; g8 < 8; ++g8) pi += pp[g8 * 128 + i2];
          pi *= b;
          wsh[i2] = pi;
          kp += pi * vc[i2];
        }
        kp = wave_sum(kp);
        const double K = 0.5 * b * kp;
        for (int i2 = t; i2 < len; i2 += 64) wsh[i2] -= K * vc[i2];
      }
      pend = true;
    } else {
      // trailing block in global memory: apply the pending update of step j - 1 and form
      // p = b * A_tr v in one pass (4 row groups x 256 columns)
      const int grp = t >> 8, tl = t & 255;
      const int l0 = (len * grp) / 4, l1 = (len * (grp + 1)) / 4;
      for (int i = tl; i < len; i += 256) {
        double* col = base + (int64_t)(j + 1 - off) * ld + (j + 1 - off) + i;
        const double ui = pend ? up[1 + i] : 0.0, wi = pend ? wsh[1 + i] : 0.0;
        double s0 = 0.0, s1 = 0.0;
        int l = l0;
        if (pend) {
          for (; l + 1 < l1; l += 2) {
            const double a0 = col[(int64_t)l * ld] - (up[1 + l] * wi + wsh[1 + l] * ui);
            const double a1 = col[(int64_t)(l + 1) * ld] - (up[2 + l] * wi + wsh[2 + l] * ui);
            col[(int64_t)l * ld] = a0;
            col[(int64_t)(l + 1) * ld] = a1;
            s0 += a0 * vc[l];
            s1 += a1 * vc[l + 1];
          }
          for (; l < l1; ++l) {
            const double a0 = col[(int64_t)l * ld] - (up[1 + l] * wi + wsh[1 + l] * ui);
            col[(int64_t)l * ld] = a0;
            s0 += a0 * vc[l];
          }
        } else {
          for (; l + 1 < l1; l += 2) {
            s0 += col[(int64_t)l * ld] * vc[l];
            s1 += col[(int64_t)(l + 1) * ld] * vc[l + 1];
          }
          for (; l < l1; ++l) s0 += col[(int64_t)l * ld] * vc[l];
        }
        psh[grp][i] = s0 + s1;
      }
      __syncthreads();  // every read of the previous step's w is done
      // w = p - (b/2)(v^T p) v, by wave 0 (zero when b = 0: the update is then empty)
      if (t < 64) {
        double kp = 0.0;
        for (int i = t; i < len; i += 64) {
          const double pi = b * (psh[0][i] + psh[1][i] + psh[2][i] + psh[3][i]);
          wsh[i] = pi;
          kp += pi * vc[i];
        }
        kp = wave_sum(kp);
        const double K = 0.5 * b * kp;
        for (int i = t; i < len; i += 64) wsh[i] -= K * vc[i];
      }
      pend = true;
    }
    __syncthreads();
  }
  for (int j = o + t; j + 2 < m; j += EIG_THREADS) {
    d[j] = dej[0][j - o];
    e[j] = dej[1][j - o];
    beta[j] = dej[2][j - o];
  }
  if (t == 0) {
    // the last 2 x 2 block is in LDS (o <= m - 2 whenever m >= 3; o = 0 when m <= EIG_LDS_M),
    // with the pending update of the last step (its v and w, index 0 = row m - 2)
    const double* lb = Alds + (int64_t)(m >= 2 ? m - 2 - o : 0) * EIG_LDS_M + (m >= 2 ? m - 2 - o : 0);
    if (m >= 2) {
      const double* vl = ((m - 3) & 1) ? vsh2 : vsh;
      const double v0 = pend ? vl[0] : 0.0, v1 = pend ? vl[1] : 0.0;
      const double w0 = pend ? wsh[0] : 0.0, w1 = pend ? wsh[1] : 0.0;
      d[m - 2] = lb[0] - 2.0 * v0 * w0;
      d[m - 1] = lb[EIG_LDS_M + 1] - 2.0 * v1 * w1;
      e[m - 2] = lb[EIG_LDS_M] - (v1 * w0 + w1 * v0);
      beta[m - 2] = 0.0;
    } else {
      d[0] = lb[0];
    }
    e[m - 1] = 0.0;
    beta[m - 1] = 0.0;
  }
  __syncthreads();
  for (int i = t; i < m; i += EIG_THREADS) e2[i] = e[i] * e[i];
  // the Householder vectors held in LDS (rows j >= o) move to A, so that LDS can hold the
  // inverse-iteration work arrays
  for (int j = o; j + 2 < m; ++j) {
    const int len = m - 1 - j;
    for (int i = t; i < len; i += EIG_THREADS)
      A[(int64_t)j * m + j + 1 + i] = Alds[(int64_t)(j - o) * EIG_LDS_M + (j + 1 - o) + i];
  }
  o = m;
  __syncthreads();
  if ((int64_t)nw * m * 41 <= (int64_t)sizeof(Alds)) {
    Y = Alds;
    u0 = Y + (int64_t)nw * m;
    u1 = u0 + (int64_t)nw * m;
    u2 = u1 + (int64_t)nw * m;
    lm = u2 + (int64_t)nw * m;
    piv = (unsigned char*)(lm + (int64_t)nw * m);
  }

  // ---- eigenvalues by bisection (one thread per wanted eigenvalue); d, e, e2 copied to LDS
  double* dl = psh[0];
  double* el = psh[1];
  double* e2l = psh[2];
  for (int i = t; i < m; i += EIG_THREADS) {
    dl[i] = d[i];
    el[i] = e[i];
    e2l[i] = e2[i];
  }
  if (t == 0) {
    double tn = 0.0;
    for (int i = 0; i < m; ++i)
      tn = fmax(tn, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i < m - 1 ? fabs(e[i]) : 0.0));
    sc[2] = fmax(tn, 1e-300);
  }
  __syncthreads();
  const double tn = sc[2];
  // Multisection: one wave per wanted eigenvalue; in each round the 64 lanes evaluate the Sturm
  // count at 64 interior points of the current interval, which shrinks 65-fold (counts are
  // monotone in x, so the crossing is found by a ballot).
  {
    double lo = dl[0], hi = dl[0], maxe2 = 0.0;
    for (int i = 0; i < m; ++i) {
      const double r = (i > 0 ? fabs(el[i - 1]) : 0.0) + (i < m - 1 ? fabs(el[i]) : 0.0);
      lo = fmin(lo, dl[i] - r);
      hi = fmax(hi, dl[i] + r);
      if (i < m - 1) maxe2 = fmax(maxe2, e2l[i]);
    }
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, maxe2);
    const int wv0 = t >> 6, ln0 = t & 63;
    for (int idx = wv0; idx < nw; idx += EIG_THREADS / 64) {
      double a = lo - 1e-14 * tn - 1e-300, bb = hi + 1e-14 * tn + 1e-300;
      for (int it = 0; it < 40; ++it) {
        if (bb - a <= 2.220446049250313e-16 * fmax(fabs(a), fabs(bb)) + pivmin) break;
        const double h = (bb - a) / 65.0;
        const double x = a + (ln0 + 1) * h;
        const bool le = x < bb && sturm_count(m, dl, e2l, x, pivmin) <= idx;
        const unsigned long long bal = __ballot(le);
        // lanes 0..L-1 have count <= idx (monotone); the eigenvalue lies in [x_{L-1}, x_L]
        const int L = __popcll(bal);
        const double na = L > 0 ? a + L * h : a;
        const double nbv = L < 64 ? a + (L + 1) * h : bb;
        if (!(na < nbv) || (na == a && nbv == bb)) break;
        a = na;
        bb = fmin(nbv, bb);
      }
      if (ln0 == 0) wsh[idx] = 0.5 * (a + bb);
    }
  }
  __syncthreads();

  // ---- eigenvectors of the tridiagonal by inverse iteration, one thread per vector
  const double epsp = 2.220446049250313e-16 * tn;
  if (t < nw) {
    double* y = Y + (int64_t)t * m;
    double lam = wsh[t];
    // repeated eigenvalues: separate the shifts slightly so the vectors differ
    int rep = 0;
    for (int c2 = t - 1; c2 >= 0 && wsh[t] - wsh[c2] < 10.0 * epsp; --c2) ++rep;
    lam += 10.0 * epsp * rep;
    uint32_t h = 0x9E3779B9u * (uint32_t)(t + 1);
    for (int i = 0; i < m; ++i) {
      h ^= h << 13; h ^= h >> 17; h ^= h << 5;
      y[i] = 0.5 + (double)(h & 0xFFFFFF) / (double)0x1000000;
    }
    double* U0 = u0 + (int64_t)t * m;
    double* U1 = u1 + (int64_t)t * m;
    double* U2 = u2 + (int64_t)t * m;
    double* Lm = lm + (int64_t)t * m;
    unsigned char* Pv = piv + (int64_t)t * m;
    for (int it = 0; it < 2; ++it) {  // the shift is the eigenvalue to a few ulp: two solves suffice
      tri_shifted_solve(m, dl, el, lam, epsp, U0, U1, U2, Lm, Pv, y, it == 0);
      normalize(m, y);
    }
  }
  __syncthreads();
  // vectors of close eigenvalues: classical Gram-Schmidt twice against the earlier members
  // of their cluster (the whole block works on one vector at a time)
  {
    const double ctol = 1e-3 * tn;
    const int wv = t >> 6, ln = t & 63;
    for (int c = 1; c < nw; ++c) {
      int c0 = c;
      while (c0 > 0 && wsh[c0] - wsh[c0 - 1] <= ctol) --c0;
      if (c0 == c) continue;  // uniform across the block
      double* y = Y + (int64_t)c * m;
      for (int pass = 0; pass < 2; ++pass) {
        // dots with the previous members: one wave per member
        for (int c2 = c0 + wv; c2 < c; c2 += EIG_THREADS / 64) {
          const double* y2 = Y + (int64_t)c2 * m;
          double sdot = 0.0;
          for (int i = ln; i < m; i += 64) sdot += y[i] * y2[i];
          for (int o = 32; o > 0; o >>= 1) sdot += __shfl_xor(sdot, o);
          if (ln == 0) vsh[c2] = sdot;
        }
        __syncthreads();
        for (int i = t; i < m; i += EIG_THREADS) {
          double v = y[i];
          for (int c2 = c0; c2 < c; ++c2) v -= vsh[c2] * Y[(int64_t)c2 * m + i];
          y[i] = v;
        }
        __syncthreads();
        double part = 0.0;
        for (int i = t; i < m; i += EIG_THREADS) part += y[i] * y[i];
        const double nrm = sqrt(block_sum(part, red));
        for (int i = t; i < m; i += EIG_THREADS) y[i] = nrm > 0.0 ? y[i] / nrm : 0.0;
        __syncthreads();
      }
    }
  }
  __syncthreads();

  // ---- back-transformation V = H_0 H_1 ... H_{m-3} Y ; one wave per eigenvector column.  The
  // Householder vectors go back to LDS, packed after Y, when both fit (v_j of length m-1-j at
  // offset j (m-1) - j (j-1)/2): each of the m sequential steps then reads LDS, not L2.
  const int64_t yl = (Y == Alds) ? (int64_t)nw * m : 0;
  const int64_t hvn = m >= 3 ? (int64_t)(m - 1) * m / 2 - 1 : 0;
  double* hv = nullptr;
  if (yl + hvn <= (int64_t)(sizeof(Alds) / sizeof(double))) {
    hv = Alds + yl;
    for (int j = tg; j + 2 < m; j += EIG_THREADS / 256) {
      const int len = m - 1 - j;
      double* dst = hv + (int64_t)j * (m - 1) - (int64_t)j * (j - 1) / 2;
      for (int i = tc; i < len; i += 256) dst[i] = A[(int64_t)j * m + j + 1 + i];
    }
    __syncthreads();
  }
  // Each wave applies all reflectors to its own columns, so the steps need no barrier; lane ln
  // always handles the entries e = ln (mod 64) of its column, so no entry passes between lanes.
  double* bl = psh[3];  // beta, read by every wave at every step
  for (int i = t; i < m; i += EIG_THREADS) bl[i] = beta[i];
  __syncthreads();
  const int wv = t >> 6, ln = t & 63;
  for (int c = wv; c < nw; c += EIG_THREADS / 64) {
    double* y = Y + (int64_t)c * m;
    for (int j = m - 3; j >= 0; --j) {
      const double b = bl[j];
      if (b == 0.0) continue;
      const double* v = hv ? hv + (int64_t)j * (m - 1) - (int64_t)j * (j - 1) / 2 : A + (int64_t)j * m + j + 1;
      const int e0 = j + 1 + ((ln - (j + 1)) & 63);  // v[e - j - 1] pairs with y[e], e in [j + 1, m)
      double s = 0.0;
      for (int e = e0; e < m; e += 64) s += v[e - j - 1] * y[e];
      s = wave_sum(s) * b;
      for (int e = e0; e < m; e += 64) y[e] -= s * v[e - j - 1];
    }
  }
  __syncthreads();
  // ---- sign convention (largest-magnitude entry positive) and output
  for (int c = wv; c < nw; c += EIG_THREADS / 64) {
    const double* y = Y + (int64_t)c * m;
    double best = -1.0;
    int bi = 0;
    for (int i = ln; i < m; i += 64) {
      const double a = fabs(y[i]);
      if (a > best) { best = a; bi = i; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o);
      const int oi = __shfl_xor(bi, o);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const double sgn = y[bi] < 0.0 ? -1.0 : 1.0;
    for (int i = ln; i < m; i += 64) V[(int64_t)i * ldv + c] = sgn * y[i];
    if (ln == 0) wout[c] = wsh[c];
  }
}

// ---------------------------------------------------------------- Cholesky-QR factors
constexpr int KB = 32;

// Pivoted Cholesky of G restricted to the columns whose angle exceeds tau (one wave, LDS).
// rel > 0: a column whose Schur complement (what remains of it after the pivots taken) has fallen
// to rel times its own Gram diagonal is dropped as dependent on those pivots.  The complement of a
// Gram matrix carries rounding of about b eps times that diagonal (b <= 32), so below ~1e-14 it is
// noise; normalised, it becomes a direction that is not orthogonal to the basis the block was
// projected against (the second pass orthonormalises the block only within itself).
__global__ __launch_bounds__(64) void k_cholqr_first(int b, const double* __restrict__ G,
                                                     const double* __restrict__ psi2, double tau, double rel,
                                                     double* __restrict__ M, double* __restrict__ Rfac,
                                                     double* __restrict__ angles, int* __restrict__ info) {
  __shared__ double W[KB][KB + 1];
  __shared__ double L[KB][KB + 1];
  __shared__ double Ri[KB][KB + 1];
  __shared__ int perm[KB];
  __shared__ int cand[KB];
  __shared__ double gd[KB];
  __shared__ int best_sh, stop_sh;
  __shared__ double r_sh;
  const int t = threadIdx.x;
  for (int e = t; e < b * b; e += 64) {
    W[e / b][e % b] = G[e];
    L[e / b][e % b] = 0.0;
  }
  if (t < b) {
    const double pn = psi2[t] > 0.0 ? psi2[t] : 1.0;
    const double a = sqrt(fmax(G[t * b + t], 0.0) / pn);
    angles[t] = a;
    cand[t] = a > tau;
    gd[t] = G[t * b + t];
  }
  __syncthreads();
  int s = 0;
  while (s < b) {
    if (t == 0) {
      int best = -1;
      double bv = 0.0;
      for (int i = 0; i < b; ++i) {
        if (cand[i] && !(W[i][i] > rel * gd[i])) cand[i] = 0;  // dependent on the pivots
        if (cand[i] && W[i][i] > bv) { bv = W[i][i]; best = i; }
      }
      int stop = best < 0;
      if (!stop) {
        const double pn = psi2[best] > 0.0 ? psi2[best] : 1.0;
        stop = !(bv > tau * tau * pn);
      }
      best_sh = best;
      stop_sh = stop;
      r_sh = stop ? 1.0 : sqrt(bv);
    }
    __syncthreads();
    if (stop_sh) break;
    const int best = best_sh;
    const double r = r_sh;
    if (t < b) L[t][s] = (cand[t] || t == best) ? W[t][best] / r : 0.0;
    __syncthreads();
    if (t == 0) {
      cand[best] = 0;
      perm[s] = best;
    }
    __syncthreads();
    for (int e = t; e < b * b; e += 64) {
      const int i = e / b, j = e % b;
      if (cand[i] && cand[j]) W[i][j] -= L[i][s] * L[j][s];
    }
    __syncthreads();
    ++s;
  }
  // R1[a][c] = L[perm[c]][a]; column c of R1^-1 by back substitution (one lane per column)
  if (t < s) {
    const int c = t;
    for (int a = 0; a < s; ++a) Ri[a][c] = 0.0;
    Ri[c][c] = 1.0 / L[perm[c]][c];
    for (int a = c - 1; a >= 0; --a) {
      double acc = 0.0;
      for (int q = a + 1; q <= c; ++q) acc += L[perm[q]][a] * Ri[q][c];
      Ri[a][c] = -acc / L[perm[a]][a];
    }
  }
  __syncthreads();
  for (int e = t; e < b * b; e += 64) M[e] = 0.0;
  __syncthreads();
  for (int e = t; e < s * s; e += 64) {
    const int a = e / s, c = e % s;
    M[perm[a] * b + c] = Ri[a][c];
  }
  // Rfac (b x b, rows >= s zero): Phi[:, j] ~= Phi1 Rfac[:, j]
  for (int e = t; e < b * b; e += 64) {
    const int a = e / b, j = e % b;
    Rfac[e] = (a < s) ? L[j][a] : 0.0;
  }
  if (t == 0) {
    info[0] = s;
    info[1] = 0;
  }
}

// Cholesky of G2 (s x s, leading dim b), M2 = R2^-1 (ld b), Rfac <- R2 * Rfac (s x b).
__global__ __launch_bounds__(64) void k_cholqr_second(int b, const double* __restrict__ G2,
                                                      double* __restrict__ M2, double* __restrict__ Rfac,
                                                      int* __restrict__ info) {
  __shared__ double R[KB][KB + 1];
  __shared__ double Mi[KB][KB + 1];
  __shared__ double F[KB][KB + 1];
  __shared__ int fail_sh;
  const int t = threadIdx.x;
  const int s = info[0];
  for (int e = t; e < KB * KB; e += 64) R[e / KB][e % KB] = 0.0;
  if (t == 0) fail_sh = 0;
  __syncthreads();
  for (int j = 0; j < s; ++j) {
    if (t == 0) {
      double dsum = G2[j * b + j];
      for (int q = 0; q < j; ++q) dsum -= R[q][j] * R[q][j];
      if (!(dsum > 0.0)) { fail_sh = 1; dsum = 1e-300; }
      R[j][j] = sqrt(dsum);
    }
    __syncthreads();
    if (t > j && t < s) {
      double v = G2[j * b + t];
      for (int q = 0; q < j; ++q) v -= R[q][j] * R[q][t];
      R[j][t] = v / R[j][j];
    }
    __syncthreads();
  }
  if (t < s) {
    const int c = t;
    for (int a = 0; a < s; ++a) Mi[a][c] = 0.0;
    Mi[c][c] = 1.0 / R[c][c];
    for (int a = c - 1; a >= 0; --a) {
      double acc = 0.0;
      for (int q = a + 1; q <= c; ++q) acc += R[a][q] * Mi[q][c];
      Mi[a][c] = -acc / R[a][a];
    }
  }
  for (int e = t; e < s * b; e += 64) F[e / b][e % b] = Rfac[e];
  __syncthreads();
  for (int e = t; e < s * s; e += 64) M2[(e / s) * b + (e % s)] = Mi[e / s][e % s];
  for (int e = t; e < s * b; e += 64) {
    const int a = e / b, j = e % b;
    double acc = 0.0;
    for (int q = a; q < s; ++q) acc += R[a][q] * F[q][j];
    Rfac[e] = acc;
  }
  if (t == 0) info[1] = fail_sh;
}

// ---------------------------------------------------------------- T bookkeeping
__global__ void k_t_extend(int m_old, int kn, const double* __restrict__ X, int64_t ldx,
                           double* __restrict__ T, int64_t ldt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int mt = m_old + kn;
  if (e >= (int64_t)mt * kn) return;
  const int i = (int)(e / kn), j = (int)(e % kn);
  const int cj = m_old + j;
  if (i < m_old) {
    const double v = X[(int64_t)i * ldx + j];
    T[(int64_t)i * ldt + cj] = v;
    T[(int64_t)cj * ldt + i] = v;
  } else {
    const int a = i - m_old;
    T[(int64_t)i * ldt + cj] = 0.5 * (X[(int64_t)i * ldx + j] + X[(int64_t)(m_old + j) * ldx + a]);
  }
}

__global__ void k_t_full(int m, const double* __restrict__ X, int64_t ldx, double* __restrict__ T,
                         int64_t ldt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * m) return;
  const int i = (int)(e / m), j = (int)(e % m);
  T[(int64_t)i * ldt + j] = 0.5 * (X[(int64_t)i * ldx + j] + X[(int64_t)j * ldx + i]);
}

__global__ void k_t_diag(int m, const double* __restrict__ th, double* __restrict__ T, int64_t ldt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * m) return;
  const int i = (int)(e / m), j = (int)(e % m);
  T[(int64_t)i * ldt + j] = i == j ? th[i] : 0.0;
}

__global__ void k_store_coef(int m_old, int kn, int k, const double* __restrict__ C, int64_t ldc,
                             const double* __restrict__ Rt, double* __restrict__ G, int64_t ldg) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)(m_old + kn) * k) return;
  const int i = (int)(e / k), j = (int)(e % k);
  G[(int64_t)i * ldg + j] = i < m_old ? C[(int64_t)i * ldc + j] : Rt[(int64_t)(i - m_old) * ldc + j];
}

// E^(p)_j = G^(p-1)[:, j]^T (T[:, j] - E0_j e_j)  (eq. exp_seq, first line: Psi^(p-1)^T V Psi^(0)
// with Psi^(l) = Q G^(l), Q^T H Psi^(0) = T[:, 0:k] and Q^T H0 Psi^(0) = E0 on the first k rows);
// A = G^(p-1), B = sum_{l=0}^{p-2} G^(l) diag(E^(p-l)), both m x k (zero-padded rows).
__global__ void k_corr_coefs(int p, int k, int m, const double* __restrict__ Gh, int64_t gstride,
                             int64_t ldg, const int* __restrict__ mh, double* __restrict__ Et,
                             const double* __restrict__ T, int64_t ldt, const double* __restrict__ E0,
                             double* __restrict__ A, double* __restrict__ B) {
  __shared__ double Ep[32];
  const int t = threadIdx.x;
  const double* Gp = Gh + (int64_t)(p - 1) * gstride;
  const int mp = mh[p - 1];
  if (t < k) {
    double s = 0.0;
    for (int i = 0; i < mp; ++i) s += Gp[(int64_t)i * ldg + t] * T[(int64_t)i * ldt + t];
    s -= E0[t] * Gp[(int64_t)t * ldg + t];
    Ep[t] = s;
    Et[(int64_t)p * k + t] = s;
  }
  __syncthreads();
  for (int64_t e = t; e < (int64_t)m * k; e += blockDim.x) {
    const int i = (int)(e / k), j = (int)(e % k);
    A[e] = i < mp ? Gp[(int64_t)i * ldg + j] : 0.0;
    double s = 0.0;
    for (int l = 0; l + 2 <= p; ++l) {
      const double El = (l == 0) ? Ep[j] : Et[(int64_t)(p - l) * k + j];
      if (i < mh[l]) s += El * Gh[(int64_t)l * gstride + (int64_t)i * ldg + j];
    }
    B[e] = s;
  }
}

// out[j][kk] = c[j][kk] / (w[j] - sigma_kk) for the deflated j != kk (psi_kk is projected out),
// sigma_kk = shift[kk] when given, else E_kk^(0) = w[kk]
__global__ void k_deflate_coefs(int D, int k, const double* __restrict__ w, const double* __restrict__ shift,
                                const double* __restrict__ c, int64_t ldc, double* __restrict__ out, int64_t ldo) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= D * k) return;
  const int j = e / k, kk = e % k;
  const double Ek = shift ? shift[kk] : w[kk];
  const double dj = w[j] - Ek;
  double v = 0.0;
  if (j != kk && fabs(dj) > 1e-12 * fmax(1.0, fabs(Ek))) v = c[(int64_t)j * ldc + kk] / dj;
  out[(int64_t)j * ldo + kk] = v;
}

// out[j][a] = c[j][a] / (w[j] - theta[a]) for every deflated j (shifted small-space solve)
__global__ void k_deflate_shift(int D, int na, const double* __restrict__ w, const double* __restrict__ theta,
                                const double* __restrict__ c, int64_t ldc, double* __restrict__ out,
                                int64_t ldo) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= D * na) return;
  const int j = e / na, a = e % na;
  const double th = theta[a];
  const double dj = w[j] - th;
  double v = 0.0;
  if (fabs(dj) > 1e-12 * fmax(1.0, fabs(th))) v = c[(int64_t)j * ldc + a] / dj;
  out[(int64_t)j * ldo + a] = v;
}

__global__ void k_add(int count, const double* __restrict__ a, double* __restrict__ b) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) b[e] += a[e];
}

// per-chunk max |x| (first index on ties) for each column
__global__ __launch_bounds__(256) void k_colargmax(int64_t n, int b, const double* __restrict__ X,
                                                   int64_t ldx, double* __restrict__ pv,
                                                   int64_t* __restrict__ pi) {
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  const int c = blockIdx.y;
  const int64_t r0 = (int64_t)blockIdx.x * 4096;
  const int64_t r1 = min<int64_t>(n, r0 + 4096);
  double best = -1.0;
  int64_t bi = r0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
    const double a = fabs(X[r * ldx + c]);
    if (a > best) { best = a; bi = r; }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < (unsigned)o) {
      const double ov = sv[threadIdx.x + o];
      const int64_t oi = si[threadIdx.x + o];
      if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x])) {
        sv[threadIdx.x] = ov;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pv[(int64_t)c * gridDim.x + blockIdx.x] = sv[0];
    pi[(int64_t)c * gridDim.x + blockIdx.x] = si[0];
  }
}

__global__ void k_colsign(int64_t nch, int b, const double* __restrict__ X, int64_t ldx,
                          const double* __restrict__ pv, const int64_t* __restrict__ pi,
                          double* __restrict__ sgn) {
  const int c = threadIdx.x;
  if (c >= b) return;
  double best = -1.0;
  int64_t bi = 0;
  for (int64_t q = 0; q < nch; ++q) {
    const double v = pv[(int64_t)c * nch + q];
    const int64_t i = pi[(int64_t)c * nch + q];
    if (v > best || (v == best && i < bi)) { best = v; bi = i; }
  }
  sgn[c] = X[bi * ldx + c] < 0.0 ? -1.0 : 1.0;
}

__global__ void k_colscale(int64_t n, int b, double* __restrict__ X, int64_t ldx,
                           const double* __restrict__ sgn) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * b) return;
  const int64_t r = e / b;
  const int c = (int)(e % b);
  X[r * ldx + c] *= sgn[c];
}

__global__ void k_select_smallest(int64_t n, const double* __restrict__ d, int nsel, int* __restrict__ idx) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  // pass q takes the smallest (value, index) pair above the one taken by pass q - 1
  double pv = -INFINITY;
  int pi = -1;
  for (int q = 0; q < nsel; ++q) {
    double best = INFINITY;
    int bi = 0x7fffffff;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
      const double v = d[i];
      const bool above = v > pv || (v == pv && (int)i > pi);
      if (above && (v < best || (v == best && (int)i < bi))) { best = v; bi = (int)i; }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
      if (threadIdx.x < (unsigned)o) {
        const double ov = sv[threadIdx.x + o];
        const int oi = si[threadIdx.x + o];
        if (ov < sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x])) {
          sv[threadIdx.x] = ov;
          si[threadIdx.x] = oi;
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) idx[q] = si[0];
    pv = sv[0];
    pi = si[0];
    __syncthreads();
  }
}

__global__ void k_unit_block(int64_t n, int b, const int* __restrict__ idx, double* __restrict__ X,
                             int64_t ldx) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * b) return;
  const int64_t r = e / b;
  const int c = (int)(e % b);
  X[r * ldx + c] = (r == idx[c]) ? 1.0 : 0.0;
}

inline int64_t g1(int64_t count) { return cdiv(count > 0 ? count : 1, 256); }

}  // namespace

int64_t eig_scratch(int m, int nwant) {
  return (int64_t)m * m + 4LL * m + 5LL * nwant * m + cdiv((int64_t)nwant * m, 8) + 64;
}

void sym_eig_lowest(int m, int nwant, const double* S, int64_t lds, double* w, double* V, int64_t ldv,
                    double* scratch, hipStream_t s) {
  if (m < 1 || m > 512 || nwant < 1 || nwant > m || nwant > 64)
    throw Error(1, "sym_eig_lowest: need 1 <= nwant <= min(m, 64), m <= 512");
  k_sym_eig<<<1, EIG_THREADS, 0, s>>>(m, nwant, S, lds, w, V, ldv, scratch);
  SPPC_LAUNCH_CHECK();
}

void cholqr_first(int b, const double* G, const double* psi_sumsq, double tau, double rel, double* M,
                  double* Rfac, double* angles, int* info, hipStream_t s) {
  if (b < 1 || b > KB) throw Error(1, "cholqr: block width must be 1..32");
  k_cholqr_first<<<1, 64, 0, s>>>(b, G, psi_sumsq, tau, rel, M, Rfac, angles, info);
  SPPC_LAUNCH_CHECK();
}

void cholqr_second(int b, const double* G2, double* M2, double* Rfac, int* info, hipStream_t s) {
  k_cholqr_second<<<1, 64, 0, s>>>(b, G2, M2, Rfac, info);
  SPPC_LAUNCH_CHECK();
}

void t_extend(int m_old, int kn, const double* X, int64_t ldx, double* T, int64_t ldt, hipStream_t s) {
  k_t_extend<<<g1((int64_t)(m_old + kn) * kn), 256, 0, s>>>(m_old, kn, X, ldx, T, ldt);
  SPPC_LAUNCH_CHECK();
}

void t_from_full(int m, const double* X, int64_t ldx, double* T, int64_t ldt, hipStream_t s) {
  k_t_full<<<g1((int64_t)m * m), 256, 0, s>>>(m, X, ldx, T, ldt);
  SPPC_LAUNCH_CHECK();
}

void t_set_diag(int m, const double* theta, double* T, int64_t ldt, hipStream_t s) {
  k_t_diag<<<g1((int64_t)m * m), 256, 0, s>>>(m, theta, T, ldt);
  SPPC_LAUNCH_CHECK();
}

void store_coef(int m_old, int kn, int k, const double* C, int64_t ldc, const double* Rtot, double* G,
                int64_t ldg, hipStream_t s) {
  k_store_coef<<<g1((int64_t)(m_old + kn) * k), 256, 0, s>>>(m_old, kn, k, C, ldc, Rtot, G, ldg);
  SPPC_LAUNCH_CHECK();
}

void build_correction_coefs(int p, int k, int m, const double* Ghist, int64_t gstride, int64_t ldg,
                            const int* m_hist, double* Etab, const double* T, int64_t ldt,
                            const double* E0, double* A, double* B, hipStream_t s) {
  k_corr_coefs<<<1, 256, 0, s>>>(p, k, m, Ghist, gstride, ldg, m_hist, Etab, T, ldt, E0, A, B);
  SPPC_LAUNCH_CHECK();
}

void deflate_coefs(int D, int k, const double* w, const double* shift, const double* c, int64_t ldc, double* out,
                   int64_t ldo, hipStream_t s) {
  k_deflate_coefs<<<g1((int64_t)D * k), 256, 0, s>>>(D, k, w, shift, c, ldc, out, ldo);
  SPPC_LAUNCH_CHECK();
}

void deflate_shift(int D, int na, const double* w, const double* theta, const double* c, int64_t ldc, double* out,
                   int64_t ldo, hipStream_t s) {
  k_deflate_shift<<<g1((int64_t)D * na), 256, 0, s>>>(D, na, w, theta, c, ldc, out, ldo);
  SPPC_LAUNCH_CHECK();
}

void add_small(int count, const double* a, double* b, hipStream_t s) {
  if (count <= 0) return;
  k_add<<<g1(count), 256, 0, s>>>(count, a, b);
  SPPC_LAUNCH_CHECK();
}

void sign_fix_columns(int64_t n, int b, double* X, int64_t ldx, double* work, hipStream_t s) {
  const int64_t nch = cdiv(n > 0 ? n : 1, 4096);
  double* pv = work;
  int64_t* pi = (int64_t*)(work + nch * b);
  double* sg = work + 2 * nch * b;
  k_colargmax<<<dim3((unsigned)nch, (unsigned)b), 256, 0, s>>>(n, b, X, ldx, pv, pi);
  k_colsign<<<1, 64, 0, s>>>(nch, b, X, ldx, pv, pi, sg);
  k_colscale<<<g1(n * b), 256, 0, s>>>(n, b, X, ldx, sg);
  SPPC_LAUNCH_CHECK();
}

void select_smallest(int64_t n, const double* d, int nsel, int* idx, hipStream_t s) {
  k_select_smallest<<<1, 1024, 0, s>>>(n, d, nsel, idx);
  SPPC_LAUNCH_CHECK();
}

void unit_block(int64_t n, int b, const int* idx, double* X, int64_t ldx, hipStream_t s) {
  k_unit_block<<<g1(n * b), 256, 0, s>>>(n, b, idx, X, ldx);
  SPPC_LAUNCH_CHECK();
}

}  // namespace sppc
