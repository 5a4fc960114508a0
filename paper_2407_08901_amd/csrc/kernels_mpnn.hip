// kernels_mpnn.hip - learned preconditioner for the continuation: a 2-layer message-passing
// network over the graph of H that corrects the diagonal (Jacobi) step for each Ritz pair.
//
//   f = [r / rms(r), (d - theta)/(1 + |theta|), lambda(level)],  g = A f,  A = H - diag(d)
//   lambda = min(max(level - n_small_levels + 1, 0), 2) / 2 (0 in the small space, 1/2 next to it, 1 beyond)
//   h = tanh(Ws f + Wn g + b1)   (32 hidden units, per row, in registers; never written to HBM)
//   o = ws.h + A (wn.h) + b2 ;   t = tJ (1 + o),  tJ = r / (d - theta) (clamped) ;  t~ = t - x (x.t)
//
// The messages g reduce to one block product per application: A (r / rms(r)) -- the other two
// feature columns are affine in theta and use A d, A 1 and A level, computed once.  Layer 2
// needs A u with u = wn.h.  Training adds one more product, A dL/do (A is symmetric).  All
// row sums over samples are deterministic per-block partials added in a fixed order.
// Parameters: Ws[32x3] | Wn[32x3] | b1[32] | ws[32] | wn[32] | b2  (289).
#include "common.h"

namespace sppc {

namespace {

constexpr int HID = 32;
constexpr int NPAR = 289;

__device__ inline double clamp_den(double den, double theta) {
  const double fl = 1e-2 * fmax(1.0, fabs(theta));
  return fabs(den) < fl ? (den >= 0.0 ? fl : -fl) : den;
}

// static per-row inputs of the network
struct Static {
  const double* d;    // diag(H)
  const double* lev;  // level / (L-1)
  const double* Ad;   // A d
  const double* A1;   // A 1
  const double* Al;   // A lev
};

// Y[r][s] = X[r][s] / scale[s]
__global__ void k_scale_cols(int64_t n, int S, const double* __restrict__ X, int64_t ldx,
                             const double* __restrict__ sumsq, double* __restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * S) return;
  const int64_t r = e / S;
  const int s = (int)(e % S);
  double sr = sqrt(sumsq[s] / (double)n);
  if (!(sr > 0.0)) sr = 1.0;
  Y[e] = X[r * ldx + s] / sr;
}

// layer 1 + the row parts of layer 2: u = wn.h, hs = ws.h   (HF = H fr, the full product)
template <typename T>
__global__ __launch_bounds__(256) void k_mpnn_layer1(int64_t n, int S, Static st, const T* __restrict__ w,
                                                     const double* __restrict__ fr,
                                                     const double* __restrict__ HF,
                                                     const double* __restrict__ theta, double* __restrict__ u,
                                                     double* __restrict__ hs) {
  __shared__ T wsh[NPAR];
  for (int i = threadIdx.x; i < NPAR; i += blockDim.x) wsh[i] = w[i];
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * S) return;
  const int64_t r = e / S;
  const int s = (int)(e % S);
  const double th = theta[s], sth = 1.0 + fabs(th);
  const double d = st.d[r];
  const T f0 = (T)fr[e], f1 = (T)((d - th) / sth), f2 = (T)st.lev[r];
  const T g0 = (T)(HF[e] - d * fr[e]), g1 = (T)((st.Ad[r] - th * st.A1[r]) / sth), g2 = (T)st.Al[r];
  T su = 0, sh = 0;
#pragma unroll 8
  for (int j = 0; j < HID; ++j) {
    const T pre = wsh[j * 3] * f0 + wsh[j * 3 + 1] * f1 + wsh[j * 3 + 2] * f2 + wsh[96 + j * 3] * g0 +
                  wsh[96 + j * 3 + 1] * g1 + wsh[96 + j * 3 + 2] * g2 + wsh[192 + j];
    const T h = tanh(pre);
    su += wsh[256 + j] * h;
    sh += wsh[224 + j] * h;
  }
  u[e] = (double)su;
  hs[e] = (double)sh;
}

// t = tJ (1 + o), o = hs + (H u - d u) + b2 ; also tJ for the backward pass
template <typename T>
__global__ void k_mpnn_out(int64_t n, int S, const double* __restrict__ d, const T* __restrict__ w,
                           const double* __restrict__ R, int64_t ldr, const double* __restrict__ theta,
                           const double* __restrict__ hs, const double* __restrict__ u,
                           const double* __restrict__ Hu, double* __restrict__ t, double* __restrict__ tJ) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * S) return;
  const int64_t r = e / S;
  const int s = (int)(e % S);
  const double th = theta[s];
  const double o = hs[e] + (Hu[e] - d[r] * u[e]) + (double)w[288];
  const double tj = R[r * ldr + s] / clamp_den(d[r] - th, th);
  t[e] = tj * (1.0 + o);
  if (tJ) tJ[e] = tj;
}

// Y[r][s] = a[s] * X[r][s] + b[s] * Z[r][s]   (per-column coefficients, device)
__global__ void k_comb_cols(int64_t n, int S, const double* __restrict__ a, const double* __restrict__ X,
                            int64_t ldx, const double* __restrict__ b, const double* __restrict__ Z, int64_t ldz,
                            double* __restrict__ Y, int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * S) return;
  const int64_t r = e / S;
  const int s = (int)(e % S);
  Y[r * ldy + s] = a[s] * X[r * ldx + s] + b[s] * Z[r * ldz + s];
}

// loss pieces -> coefficients of dL/dt~ = ca e + cb t~ ; loss per sample
__global__ void k_loss_coef(int S, const double* __restrict__ c1, const double* __restrict__ c2,
                            const double* __restrict__ c3, double* __restrict__ ca, double* __restrict__ cb,
                            double* __restrict__ lossv, double inv_scale) {
  const int s = threadIdx.x;
  if (s >= S) return;
  const double q = c2[s] * c3[s];
  lossv[s] = 1.0 - c1[s] * c1[s] / q;
  ca[s] = -2.0 * c1[s] / q * inv_scale;
  cb[s] = 2.0 * c1[s] * c1[s] / (c2[s] * q) * inv_scale;
}

// gradient partials: one item (row, sample) per 32 threads (lane = hidden unit)
template <typename T>
__global__ __launch_bounds__(256) void k_mpnn_grad(int64_t n, int S, Static st, const T* __restrict__ w,
                                                   const double* __restrict__ fr, const double* __restrict__ HF,
                                                   const double* __restrict__ theta,
                                                   const double* __restrict__ dO, const double* __restrict__ HdO,
                                                   double* __restrict__ part, int64_t items_per_block) {
  __shared__ T wsh[NPAR];
  __shared__ double red[8][HID][10];
  for (int i = threadIdx.x; i < NPAR; i += blockDim.x) wsh[i] = w[i];
  __syncthreads();
  const int j = threadIdx.x & 31, slot = threadIdx.x >> 5;
  double acc[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) acc[q] = 0.0;
  const int64_t i0 = (int64_t)blockIdx.x * items_per_block;
  const int64_t i1 = min<int64_t>(n * S, i0 + items_per_block);
  for (int64_t e = i0 + slot; e < i1; e += 8) {
    const int64_t r = e / S;
    const int s = (int)(e % S);
    const double th = theta[s], sth = 1.0 + fabs(th);
    const double d = st.d[r];
    const T f0 = (T)fr[e], f1 = (T)((d - th) / sth), f2 = (T)st.lev[r];
    const T g0 = (T)(HF[e] - d * fr[e]), g1 = (T)((st.Ad[r] - th * st.A1[r]) / sth), g2 = (T)st.Al[r];
    const T pre = wsh[j * 3] * f0 + wsh[j * 3 + 1] * f1 + wsh[j * 3 + 2] * f2 + wsh[96 + j * 3] * g0 +
                  wsh[96 + j * 3 + 1] * g1 + wsh[96 + j * 3 + 2] * g2 + wsh[192 + j];
    const T h = tanh(pre);
    const T dov = (T)dO[e];
    const T duv = (T)(HdO[e] - d * dO[e]);   // dL/du = A dL/do
    const T dpre = (dov * wsh[224 + j] + duv * wsh[256 + j]) * ((T)1 - h * h);
    acc[0] += (double)(dpre * f0);
    acc[1] += (double)(dpre * f1);
    acc[2] += (double)(dpre * f2);
    acc[3] += (double)(dpre * g0);
    acc[4] += (double)(dpre * g1);
    acc[5] += (double)(dpre * g2);
    acc[6] += (double)dpre;
    acc[7] += (double)(dov * h);
    acc[8] += (double)(duv * h);
    acc[9] += (double)dov;  // db2 (only lane 0's copy is used)
  }
#pragma unroll
  for (int q = 0; q < 10; ++q) red[slot][j][q] = acc[q];
  __syncthreads();
  if (slot == 0) {
    double tot[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) {
      double v = 0.0;
      for (int sl = 0; sl < 8; ++sl) v += red[sl][j][q];
      tot[q] = v;
    }
    double* out = part + (int64_t)blockIdx.x * NPAR;
    out[j * 3] = tot[0];
    out[j * 3 + 1] = tot[1];
    out[j * 3 + 2] = tot[2];
    out[96 + j * 3] = tot[3];
    out[96 + j * 3 + 1] = tot[4];
    out[96 + j * 3 + 2] = tot[5];
    out[192 + j] = tot[6];
    out[224 + j] = tot[7];
    out[256 + j] = tot[8];
    if (j == 0) out[288] = tot[9];
  }
}

__global__ void k_sum_parts(int64_t nb, const double* __restrict__ part, double* __restrict__ g) {
  const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= NPAR) return;
  double s = 0.0;
  for (int64_t b = lane; b < nb; b += 64) s += part[b * NPAR + i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) g[i] = s;
}

// Adam on the float32 master weights; the network uses their bfloat16 rounding
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const double* __restrict__ g, float lr, float b1, float b2, float eps, int step,
                       float* __restrict__ wq) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPAR) return;
  const float gi = (float)g[i];
  m[i] = b1 * m[i] + (1.f - b1) * gi;
  v[i] = b2 * v[i] + (1.f - b2) * gi * gi;
  const float mh = m[i] / (1.f - powf(b1, (float)step));
  const float vh = v[i] / (1.f - powf(b2, (float)step));
  w[i] -= lr * mh / (sqrtf(vh) + eps);
  if (wq) {
    // round to bfloat16 (nearest even) and back
    uint32_t bits = __float_as_uint(w[i]);
    const uint32_t lsb = (bits >> 16) & 1u;
    bits += 0x7FFFu + lsb;
    wq[i] = __uint_as_float(bits & 0xFFFF0000u);
  }
}

__global__ void k_round_bf16(int cnt, const float* __restrict__ w, float* __restrict__ wq, double* __restrict__ wd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  uint32_t bits = __float_as_uint(w[i]);
  const uint32_t lsb = (bits >> 16) & 1u;
  bits += 0x7FFFu + lsb;
  const float q = __uint_as_float(bits & 0xFFFF0000u);
  if (wq) wq[i] = q;
  if (wd) wd[i] = (double)q;
}

// static inputs: lev, and the row sums A d, A 1, A lev from full products
__global__ void k_static(int64_t n, const double* __restrict__ d, const double* __restrict__ lev,
                         const double* __restrict__ P, double* __restrict__ Ad, double* __restrict__ A1,
                         double* __restrict__ Al) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  // P = H [d, 1, lev] row-major n x 3
  Ad[r] = P[r * 3] - d[r] * d[r];
  A1[r] = P[r * 3 + 1] - d[r];
  Al[r] = P[r * 3 + 2] - d[r] * lev[r];
}

__global__ void k_pack3(int64_t n, const double* __restrict__ d, const double* __restrict__ lev,
                        double* __restrict__ P) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  P[r * 3] = d[r];
  P[r * 3 + 1] = 1.0;
  P[r * 3 + 2] = lev[r];
}

// level feature: the level counted from the small space, clipped: 0 on the small-space levels, 1/2
// on the first level outside it, 1 beyond (the same values for any number of levels)
__global__ void k_levels(int64_t n, int L, int nsmall, const int64_t* __restrict__ off, double* __restrict__ lev) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  int l = 0;
  while (l + 1 < L && off[l + 1] <= r) ++l;
  const int rel = l - nsmall + 1;
  lev[r] = 0.5 * (double)(rel < 0 ? 0 : rel > 2 ? 2 : rel);
}

__global__ void k_fill_const(int S, double v, double* __restrict__ out) {
  const int i = threadIdx.x;
  if (i < S) out[i] = v;
}

__global__ void k_neg(int S, const double* __restrict__ in, double* __restrict__ out) {
  const int i = threadIdx.x;
  if (i < S) out[i] = -in[i];
}

__global__ void k_mul(int64_t cnt, const double* __restrict__ a, double* __restrict__ b) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < cnt) b[e] *= a[e];
}

inline int64_t gg(int64_t c) { return cdiv(c > 0 ? c : 1, 256); }

}  // namespace

int mpnn_nparam() { return NPAR; }

// Static inputs: lev[n], Ad[n], A1[n], Al[n]; tmp >= 6n doubles.
void mpnn_prepare(const DevCSR& H, const double* diag, const int64_t* level_off_dev, int L, int nsmall, double* lev,
                  double* Ad, double* A1, double* Al, double* tmp, hipStream_t s) {
  const int64_t n = H.n;
  k_levels<<<gg(n), 256, 0, s>>>(n, L, nsmall, level_off_dev, lev);
  k_pack3<<<gg(n), 256, 0, s>>>(n, diag, lev, tmp);
  spmm_f64(H, tmp, 3, tmp + 3 * n, 3, 3, nullptr, s);
  k_static<<<gg(n), 256, 0, s>>>(n, diag, lev, tmp + 3 * n, Ad, A1, Al);
  SPPC_LAUNCH_CHECK();
}

// Workspace layout (n x S doubles each): fr | HF | u | hs | Hu | t | tJ | dO | HdO  (9 n S)
// + small: sumsq[S], th[S], c1..c3[S], ca, cb, lossv, xdt[S], grad partials.
int64_t mpnn_work_doubles(int64_t n, int S) {
  const int64_t items = n * S;
  const int64_t nblk = cdiv(items, 8 * 64);
  return 9 * items + 16 * 64 + nblk * NPAR + NPAR + 64;
}

// Forward (and, with E, the loss gradient) for S samples.  R, X: n x S (leading dims ldr, ldx),
// theta_dev[S].  T_out (n x S, ld S): the projected output t~ (or nullptr).  grad_out (device,
// 289 doubles, mean over samples) and loss_dev (S doubles) when E != nullptr.
// Y := Y - Q (Q^T Y) for Y n x S (ld S) and a basis Q n x m (ld ldq) with orthonormal columns.
static void project_basis(int64_t n, int S, const MpnnBasis& B, double* Y, hipStream_t s) {
  double* C = B.work;
  double* gw = B.work + (int64_t)B.m * 32;
  for (int c0 = 0; c0 < S; c0 += 32) {
    const int bs = S - c0 < 32 ? S - c0 : 32;
    gemm_tn(n, B.m, bs, B.Q, B.ldq, Y + c0, S, C, bs, 1.0, 0.0, gw, s);
    gemm_nn(n, B.m, bs, B.Q, B.ldq, C, bs, Y + c0, S, -1.0, 1.0, s);
  }
}

int64_t mpnn_basis_work_doubles(int64_t n, int m) { return (int64_t)m * 32 + gemm_tn_work(n, m, 32); }

template <typename T>
void mpnn_run(const DevCSR& H, const double* diag, const double* lev, const double* Ad, const double* A1,
              const double* Al, const T* w, int S, const double* R, int64_t ldr, const double* X, int64_t ldx,
              const double* theta_dev, const double* E, double* T_out, double* grad_out, double* loss_dev,
              double* work, const MpnnBasis* basis, hipStream_t s, bool project) {
  const int64_t n = H.n;
  const int64_t items = n * S;
  if (!project && E) throw Error(1, "mpnn_run: the loss needs the projected output");
  double* fr = work;
  double* HF = fr + items;
  double* u = HF + items;
  double* hs = u + items;
  double* Hu = hs + items;
  double* t = Hu + items;
  double* tJ = t + items;
  double* dO = tJ + items;
  double* HdO = dO + items;
  double* sm = HdO + items;
  double* sumsq = sm;
  double* c1 = sm + 64;
  double* c2 = sm + 128;
  double* c3 = sm + 192;
  double* ca = sm + 256;
  double* cb = sm + 320;
  double* lossv = sm + 384;
  double* xdt = sm + 448;
  double* one = sm + 512;
  double* mxdt = sm + 576;
  double* part = sm + 16 * 64;
  Static st{diag, lev, Ad, A1, Al};
  // the two aggregations: with the bfloat16 weights (T = float) their products take float32 X when
  // float32 values are stored (float32 products, float64 sums; the network's inputs need no more),
  // the float32 copy of X in tJ's space, which k_mpnn_out fills only after both
  auto hprod = [&](const double* Xd, double* Yd) {
    if constexpr (sizeof(T) == 4) {
      if (H.val32) {
        float* x32 = (float*)tJ;
        copy_to_f32(n, S, Xd, S, x32, S, s);
        spmm_f32(H, x32, S, Yd, S, S, nullptr, s);
        return;
      }
    }
    spmm_f64(H, Xd, S, Yd, S, S, nullptr, s);
  };
  colsumsq(n, S, R, ldr, sumsq, part, s);
  k_scale_cols<<<gg(items), 256, 0, s>>>(n, S, R, ldr, sumsq, fr);
  hprod(fr, HF);
  k_mpnn_layer1<T><<<gg(items), 256, 0, s>>>(n, S, st, w, fr, HF, theta_dev, u, hs);
  hprod(u, Hu);
  k_mpnn_out<T><<<gg(items), 256, 0, s>>>(n, S, diag, w, R, ldr, theta_dev, hs, u, Hu, t, tJ);
  // t~ = t - x (x.t), or t - Q (Q^T t) with a basis
  k_fill_const<<<1, 64, 0, s>>>(S, 1.0, one);
  if (!project) {
    // unprojected t = tJ (1 + o) (the step of a single-vector refinement)
  } else if (basis) {
    project_basis(n, S, *basis, t, s);
  } else {
    coldots(n, S, X, ldx, t, S, xdt, part, s);
    k_neg<<<1, 64, 0, s>>>(S, xdt, mxdt);
    k_comb_cols<<<gg(items), 256, 0, s>>>(n, S, one, t, S, mxdt, X, ldx, t, S);
  }
  if (T_out) copy_block(n, S, t, S, T_out, S, s);
  if (E) {
    coldots(n, S, t, S, E, S, c1, part, s);
    coldots(n, S, t, S, t, S, c2, part, s);
    coldots(n, S, E, S, E, S, c3, part, s);
    k_loss_coef<<<1, 64, 0, s>>>(S, c1, c2, c3, ca, cb, lossv, 1.0 / S);
    // dL/dt~ = ca e + cb t~ -> dO ; then through the projection and t = tJ (1 + o)
    k_comb_cols<<<gg(items), 256, 0, s>>>(n, S, ca, E, S, cb, t, S, dO, S);
    if (basis) {
      project_basis(n, S, *basis, dO, s);
    } else {
      coldots(n, S, X, ldx, dO, S, xdt, part, s);
      k_neg<<<1, 64, 0, s>>>(S, xdt, mxdt);
      k_comb_cols<<<gg(items), 256, 0, s>>>(n, S, one, dO, S, mxdt, X, ldx, dO, S);
    }
    k_mul<<<gg(items), 256, 0, s>>>(items, tJ, dO);
    spmm_f64(H, dO, S, HdO, S, S, nullptr, s);
    const int64_t ipb = 8 * 64;
    const int64_t nblk = cdiv(items, ipb);
    k_mpnn_grad<T><<<nblk, 256, 0, s>>>(n, S, st, w, fr, HF, theta_dev, dO, HdO, part, ipb);
    k_sum_parts<<<cdiv(NPAR, 4), 256, 0, s>>>(nblk, part, grad_out);
    if (loss_dev) copy_block(1, S, lossv, S, loss_dev, S, s);
  }
  SPPC_LAUNCH_CHECK();
}

template void mpnn_run<float>(const DevCSR&, const double*, const double*, const double*, const double*,
                              const double*, const float*, int, const double*, int64_t, const double*, int64_t,
                              const double*, const double*, double*, double*, double*, double*,
                              const MpnnBasis*, hipStream_t, bool);
template void mpnn_run<double>(const DevCSR&, const double*, const double*, const double*, const double*,
                               const double*, const double*, int, const double*, int64_t, const double*,
                               int64_t, const double*, const double*, double*, double*, double*, double*,
                               const MpnnBasis*, hipStream_t, bool);

void mpnn_adam(float* w, float* m, float* v, const double* g, float lr, int step, float* wq, hipStream_t s) {
  k_adam<<<cdiv(NPAR, 256), 256, 0, s>>>(w, m, v, g, lr, 0.9f, 0.999f, 1e-8f, step, wq);
  SPPC_LAUNCH_CHECK();
}

void mpnn_round_bf16(int cnt, const float* w, float* wq, double* wd, hipStream_t s) {
  k_round_bf16<<<cdiv(cnt, 256), 256, 0, s>>>(cnt, w, wq, wd);
  SPPC_LAUNCH_CHECK();
}

// E = (I - Q Q^T) Psi  (n x S, ld S): the part of each exact eigenvector outside the basis.
void mpnn_target(int64_t n, int S, const MpnnBasis& B, const double* Psi, double* E, hipStream_t s) {
  copy_block(n, S, Psi, S, E, S, s);
  project_basis(n, S, B, E, s);
}

}  // namespace sppc
