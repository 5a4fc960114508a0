// kernels_cg.hip - the small-space solves of the perturbative correction (eq. sm_lin_proj).
//
// For every wanted pair c the singular system (H0hat - E_c) x = b_c - (b_c^T psi_c) psi_c is
// solved for its minimum-norm solution orthogonal to psi_c.  The D lowest eigenvectors of
// H0hat (Ps, n0 x D) are deflated: CG runs on the complement, where H0hat - E_c is positive
// definite, and the deflated directions are added back exactly by the caller.  All k
// systems advance together, sharing one product with H0hat per iteration.
//
// The right-hand side is projected once onto the complement; H0hat - E_c maps the complement
// into itself (its deflated directions are eigenvectors), so the CG iterates stay there.  The
// final x is projected once more to remove rounding drift.
//
// The iteration is the single-reduction form of CG (Chronopoulos and Gear): with w = A r the
// two inner products r.r and w.r of one iteration are formed together, so one kernel per
// iteration suffices and the kernel boundary is the only grid-wide barrier.  The kernel
// re-adds the previous kernel's per-block partial sums (same fixed order on every block, so
// the CG scalars are identical everywhere and bit-reproducible), updates p, s, x, r of its own
// rows and forms w = A r_new, evaluating r_new = r - alpha (w + beta s_old) at every gathered
// row.  r, w and s are double-buffered by iteration parity.  Rows are split over the blocks by
// nonzero count (level-0 rows of H0hat have far more entries than level-1 rows).
#include "common.h"

namespace sppc {

namespace {

constexpr int CG_MAXK = 16;
constexpr int CG_MAXD = 28;
constexpr int PW = 1024;       // partial width of the projection phase (>= 2Dk)
constexpr int CH = 64;         // rows per LDS chunk of the projections
constexpr int NB = 256;        // blocks of the iteration kernel
constexpr int NT = 1024;       // threads per block of the iteration kernel

// device scalars, double-buffered by iteration parity
struct CGScal {
  double gam[2][CG_MAXK];  // r.r of the iteration's residual
  double alp[2][CG_MAXK];  // step length
  double bb[CG_MAXK];      // r.r of the projected right-hand side
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
  const double* shift;  // E_c
  const double* Ps;     // n0 x D
  const int64_t* rowb;  // [NB + 1] row bounds of the iteration blocks
  double* x;            // n0 x k
  double* r0;           // n0 x k: the right-hand side, projected in place
  double* G[2];         // by iteration parity: per row (r_j, w_j = A r_j, s_{j-1} = A p_{j-1}), 3k values
  double* p;
  double* z;            // n0 x k: A s (pipelined form only)
  double* part[2];      // NB x 2*CG_MAXK partial (r.r, w.r) by parity
  double* partP;        // nb2 x PW   (Ps^T y)
  int nb2;
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

// ---- Y -= Ps (Ps^T Y) from the partials; optionally also: coef = Ps^T Y, and (start) zero
// x, p and s_{-1}
__global__ __launch_bounds__(1024) void k_cg_project(CGArgs a, double* Y, double* coef, int start) {
  __shared__ double tot[PW];
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
      a.p[e] = 0.0;
      const int64_t g = row * 3 * k + c;
      a.G[0][g] = v;          // r_0
      a.G[0][g + 2 * k] = 0.0;  // s_{-1}
      a.z[e] = 0.0;
    }
  }
}

// ---- one CG iteration (j >= 0) or, with INIT, w_0 = A r_0 and the partials of (r.r, w.r).
// Kernel j reads r_j, w_j (buffer j&1), s_{j-1} (buffer (j&1)^1), p_{j-1}, x_j and the partials
// of kernel j-1; it writes p_j, s_j (buffer j&1), x_{j+1}, r_{j+1}, w_{j+1} (buffer (j&1)^1) and
// its partials (buffer j&1).
//
// A block owns a row range (H0hat is a contiguous CSR) and takes it in chunks of RCH rows.  The
// product is entry-parallel: each wave streams windows of 64 entries of the chunk (one coalesced
// load), groups of B lanes take B consecutive entries, lane c gathers column c of the rows of
// (r, w, s) named by the entries, and runs of entries of one row are summed in a register and
// added to the row's LDS accumulator when the run ends.  Then every (row, column) of the chunk is
// updated by one thread.
constexpr int RCH = 128;

// entries [win, win + 64) of a chunk: columns, values and the row (last r with soff[r] <= e)
template <typename VT>
__device__ inline void cg_window(const int32_t* __restrict__ col, const VT* __restrict__ val, int64_t e0,
                                 const int* soff, int nr, int ne, int e, int& mc, VT& mv, int& mr) {
  mc = 0;
  mv = VT(0);
  mr = 0;
  if (e < ne) {
    mc = col[e0 + e];
    mv = val[e0 + e];
    int lo = 0, hi = nr - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (soff[mid] <= e) lo = mid; else hi = mid - 1;
    }
    mr = lo;
  }
}

template <int B, typename VT>
__device__ inline void cg_runs(int win, int ne, int g, int c, bool cok, int mr, VT mv, const double* xv,
                               double* acc_s) {
  int cur_r = __shfl(mr, g * B);
  double cur = 0.0;
#pragma unroll
  for (int q = 0; q < B; ++q) {
    const int src = g * B + q;
    const VT vv = __shfl(mv, src);
    const int rr = __shfl(mr, src);
    if (win + src < ne) {
      if (rr != cur_r) {
        if (cok) atomicAdd(&acc_s[cur_r * CG_MAXK + c], cur);
        cur = 0.0;
        cur_r = rr;
      }
      cur = fma((double)vv, xv[q], cur);
    }
  }
  if (win + g * B < ne && cok) atomicAdd(&acc_s[cur_r * CG_MAXK + c], cur);
}

template <int B, typename VT, bool INIT, bool PIPE>
__global__ __launch_bounds__(NT) void k_cg_iter(CGArgs a, int j) {
  const int t = threadIdx.x;
  const int k = a.k;
  const int par = INIT ? 1 : (j & 1);
  const double* __restrict__ partin = a.part[par ^ 1];
  __shared__ double red[NT];
  __shared__ double al[CG_MAXK], be[CG_MAXK];
  __shared__ double acc_s[RCH * CG_MAXK];
  __shared__ int soff[RCH + 1];
  __shared__ int nact_s;
  if (!INIT && j > 0 && a.sc->nact[par ^ 1] == 0) {
    if (blockIdx.x == 0 && t == 0) a.sc->nact[par] = 0;
    return;
  }
  const int lane = t & 63, wv = t >> 6;
  const int g = lane / B, c = lane % B;
  const bool cok = c < k;
  // the triple (r, w, s) of a row is contiguous, so a gathered row of the three is one segment
  const int k3 = 3 * k;
  const double* __restrict__ rj = a.G[INIT ? 0 : par];
  const double* __restrict__ wj = rj + k;
  const double* __restrict__ sm = rj + 2 * k;
  double* __restrict__ rn = a.G[INIT ? 0 : par ^ 1];
  double* __restrict__ wn = rn + k;
  double* __restrict__ sj = rn + 2 * k;
  const VT* __restrict__ val = sizeof(VT) == 8 ? (const VT*)a.v64 : (const VT*)a.v32;
  // own-row phase mapping: column oc, row slots os and os + NT/16 of each chunk
  const int oc = t % CG_MAXK, os = t / CG_MAXK;
  constexpr int OS = NT / CG_MAXK;
  static_assert(2 * OS == RCH, "two row slots per thread and chunk");
  double sg = 0.0, sd = 0.0;
  double alpha = 0.0, beta = 0.0, oal = 0.0, obe = 0.0;
  const double osh = oc < k ? a.shift[oc] : 0.0;
  const int64_t rb0 = a.rowb[blockIdx.x], rb1 = a.rowb[blockIdx.x + 1];
  bool first = true;
  for (int64_t c0 = rb0; c0 < rb1 || (first && !INIT); c0 += RCH) {
    const int nr = (int)max<int64_t>(0, min<int64_t>(RCH, rb1 - c0));
    // operands that do not depend on this iteration's scalars are requested first
    const int64_t e0 = nr > 0 ? a.rp[c0] : 0;
    const int rpv = (t <= nr && nr > 0) ? (int)(a.rp[c0 + t] - e0) : 0;
    double orj[2] = {0.0, 0.0}, owj[2] = {0.0, 0.0}, osm[2] = {0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int rl = os + OS * u;
      if (oc < k && rl < nr) {
        const int64_t og = (c0 + rl) * k3 + oc;
        orj[u] = rj[og];
        if (!INIT) {
          owj[u] = wj[og];
          osm[u] = sm[og];
        }
      }
    }
    if (!INIT && first) {
      // (r.r, w.r) of iteration j from the NB partials of the previous kernel, in a fixed order:
      // lane sums over blocks, the two half-waves, then the 16 waves in turn
      const int v = t % (2 * CG_MAXK);
      double sacc = 0.0;
      for (int b2 = t / (2 * CG_MAXK); b2 < NB; b2 += NT / (2 * CG_MAXK))
        sacc += partin[(int64_t)b2 * 2 * CG_MAXK + v];
      sacc += __shfl_xor(sacc, 32);
      if ((t & 63) < 2 * CG_MAXK) red[(t >> 6) * 2 * CG_MAXK + v] = sacc;
      __syncthreads();
      if (t < 2 * CG_MAXK) {
        double tot = 0.0;
        for (int w2 = 0; w2 < NT / 64; ++w2) tot += red[w2 * 2 * CG_MAXK + t];
        red[NT - 2 * CG_MAXK + t] = tot;
      }
      __syncthreads();
      if (t < 2 * CG_MAXK) red[t] = red[NT - 2 * CG_MAXK + t];
      __syncthreads();
      if (t < k) {
        const double gg = red[t], d = red[CG_MAXK + t];
        double al_ = 0.0, be_ = 0.0, gkeep;
        int now;
        if (j == 0) {
          now = gg > 0.0 && d != 0.0;
          al_ = now ? gg / d : 0.0;
          gkeep = gg;
          if (blockIdx.x == 0) a.sc->bb[t] = gg;
        } else {
          const double gold = a.sc->gam[par ^ 1][t];
          const double aold = a.sc->alp[par ^ 1][t];
          now = a.sc->act[par ^ 1][t] && gg > a.tol2 * a.sc->bb[t];
          if (now) {
            be_ = gg / gold;
            const double den = d - be_ * gg / aold;
            al_ = den != 0.0 ? gg / den : 0.0;
            if (den == 0.0) {
              now = 0;
              be_ = 0.0;
            }
          }
          gkeep = now ? gg : gold;
        }
        al[t] = al_;
        be[t] = be_;
        if (blockIdx.x == 0) {
          a.sc->gam[par][t] = gkeep;
          a.sc->alp[par][t] = now ? al_ : 0.0;
          a.sc->act[par][t] = now;
        }
        red[t] = now;
      }
      __syncthreads();
      if (t == 0) {
        int na = 0;
        for (int cc = 0; cc < k; ++cc) na += red[cc] != 0.0;
        nact_s = na;
        if (blockIdx.x == 0) {
          a.sc->nact[par] = na;
          if (j == 0) a.sc->iters = 0;
          if (na) a.sc->iters += 1;
        }
      }
      __syncthreads();
      if (nact_s == 0) return;
      alpha = cok ? al[c] : 0.0;
      beta = cok ? be[c] : 0.0;
      oal = oc < k ? al[oc] : 0.0;
      obe = oc < k ? be[oc] : 0.0;
    }
    first = false;
    if (nr == 0) break;
    if (t <= nr) soff[t] = rpv;
    for (int i = t; i < RCH * CG_MAXK; i += NT) acc_s[i] = 0.0;
    __syncthreads();
    const int ne = soff[nr];
    // two windows per trip (one for 16-lane groups): their gathers are in flight together
    constexpr int WT = B <= 8 ? 2 : 1;
    for (int win = wv * 64; win < ne; win += WT * NT) {
      const int win2 = WT == 2 ? win + NT : ne;  // ne: an empty second window
      int mc1, mr1, mc2, mr2;
      VT mv1, mv2;
      cg_window<VT>(a.col, val, e0, soff, nr, ne, win + lane, mc1, mv1, mr1);
      cg_window<VT>(a.col, val, e0, soff, nr, ne, win2 + lane, mc2, mv2, mr2);
      double xv1[B], xv2[B];
#pragma unroll
      for (int q = 0; q < B; ++q) {
        const int src = g * B + q;
        const int cl1 = __shfl(mc1, src);
        const int cl2 = __shfl(mc2, src);
        double v1 = 0.0, v2 = 0.0;
        // pipelined form: the product is A w_j, which needs no scalar of this iteration
        if (win + src < ne && cok) {
          const int64_t og = (int64_t)cl1 * k3 + c;
          v1 = INIT ? rj[og] : PIPE ? wj[og] : rj[og] - alpha * (wj[og] + beta * sm[og]);
        }
        if (win2 + src < ne && cok) {
          const int64_t og = (int64_t)cl2 * k3 + c;
          v2 = INIT ? rj[og] : PIPE ? wj[og] : rj[og] - alpha * (wj[og] + beta * sm[og]);
        }
        xv1[q] = v1;
        xv2[q] = v2;
      }
      cg_runs<B, VT>(win, ne, g, c, cok, mr1, mv1, xv1, acc_s);
      cg_runs<B, VT>(win2, ne, g, c, cok, mr2, mv2, xv2, acc_s);
    }
    __syncthreads();
    if (oc < k) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int rl = os + OS * u;
        if (rl < nr) {
          const int64_t o = (c0 + rl) * k + oc;
          const int64_t og = (c0 + rl) * k3 + oc;
          double rnew, wv2;
          if (INIT) {
            rnew = orj[u];
            wv2 = acc_s[rl * CG_MAXK + oc] - osh * rnew;
          } else if (!PIPE) {
            const double pv = orj[u] + obe * a.p[o];
            const double sv = owj[u] + obe * osm[u];
            a.p[o] = pv;
            sj[og] = sv;
            a.x[o] = fma(oal, pv, a.x[o]);
            rnew = orj[u] - oal * sv;
            rn[og] = rnew;
            wv2 = acc_s[rl * CG_MAXK + oc] - osh * rnew;
          } else {
            // pipelined CG: q = A w_j, z = q + beta z, s = w + beta s, p = r + beta p,
            // x += alpha p, r -= alpha s, w -= alpha z
            const double q = acc_s[rl * CG_MAXK + oc] - osh * owj[u];
            const double zv = q + obe * a.z[o];
            const double sv = owj[u] + obe * osm[u];
            const double pv = orj[u] + obe * a.p[o];
            a.z[o] = zv;
            a.p[o] = pv;
            sj[og] = sv;
            a.x[o] = fma(oal, pv, a.x[o]);
            rnew = orj[u] - oal * sv;
            rn[og] = rnew;
            wv2 = owj[u] - oal * zv;
          }
          wn[og] = wv2;
          sg = fma(rnew, rnew, sg);
          sd = fma(wv2, rnew, sd);
        }
      }
    }
    __syncthreads();
  }
  // block partials in a fixed order: the four lanes of a column within a wave, then the waves
  sg += __shfl_xor(sg, 16);
  sg += __shfl_xor(sg, 32);
  sd += __shfl_xor(sd, 16);
  sd += __shfl_xor(sd, 32);
  if ((t & 63) < CG_MAXK) {
    red[(t >> 6) * 2 * CG_MAXK + oc] = sg;
    red[(t >> 6) * 2 * CG_MAXK + CG_MAXK + oc] = sd;
  }
  __syncthreads();
  if (t < 2 * CG_MAXK) {
    double tot = 0.0;
    for (int w2 = 0; w2 < NT / 64; ++w2) tot += red[w2 * 2 * CG_MAXK + t];
    a.part[par][(int64_t)blockIdx.x * 2 * CG_MAXK + t] = tot;
  }
}

// ---- row bounds of the iteration blocks: equal shares of (entries + 8 per row)
__global__ void k_row_cost(int64_t n0, const int64_t* __restrict__ rp, const int64_t* __restrict__ rend,
                           int32_t* __restrict__ cost) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n0) cost[i] = (int32_t)((rend ? rend[i] : rp[i + 1]) - rp[i] + 8);
}

__global__ void k_row_bounds(int64_t n0, const int64_t* __restrict__ pre, int64_t* __restrict__ rowb) {
  const int b = threadIdx.x;
  if (b > NB) return;
  if (b == 0) { rowb[0] = 0; return; }
  if (b == NB) { rowb[NB] = n0; return; }
  const int64_t target = pre[n0] * b / NB;
  int64_t lo = 0, hi = n0;  // first row whose prefix reaches the target
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (pre[mid] < target) lo = mid + 1; else hi = mid;
  }
  rowb[b] = lo;
}

}  // namespace

// doubles reserved for the device scalars (64-byte multiple)
constexpr int64_t SC_D = (int64_t)((sizeof(CGScal) + 63) / 64) * 8;

int64_t cg_work_doubles(int64_t n0) {
  const int64_t nb2 = std::min<int64_t>(256, cdiv(n0, 64));
  return 2 * NB * 2 * CG_MAXK + nb2 * PW + SC_D + 8 * n0 * CG_MAXK + (NB + 1) + 2 * (n0 + 2);
}

// Row bounds for the iteration blocks (once per H0hat); tmp holds 2 (n0 + 2) doubles.
void cg_prepare(const DevCSR& H0, int64_t n0, int64_t* rowb, double* tmp, hipStream_t s) {
  int32_t* cost = (int32_t*)tmp;
  int64_t* pre = (int64_t*)(tmp + (n0 + 2) / 2 + 1);
  int64_t* bsum = pre + n0 + 1;
  (void)bsum;
  k_row_cost<<<cdiv(n0 > 0 ? n0 : 1, 256), 256, 0, s>>>(n0, H0.rp, H0.rend, cost);
  SPPC_LAUNCH_CHECK();
  scan_exclusive(n0, cost, pre, bsum, s);
  k_row_bounds<<<1, NB + 1 > 1024 ? 1024 : NB + 1, 0, s>>>(n0, pre, rowb);
  SPPC_LAUNCH_CHECK();
}

// b in r (n0 x k) on entry; x returns the CG solution on the deflated complement and
// ccoef = Ps^T b.  Returns the number of iterations (synchronises the stream).
int cg_solve(const DevCSR& H0, int64_t n0, int k, int D, const double* shift, const double* Ps,
             const int64_t* rowb, double* x, double* r, double* work, double* ccoef, int maxit, double tol,
             int* host_flag, hipStream_t s) {
  if (k < 1 || k > CG_MAXK || D < 1 || D > CG_MAXD) throw Error(1, "cg: k <= 16 and D <= 28 required");
  if (H0.rend) throw Error(1, "cg: H0hat must be a contiguous CSR");
  if (n0 * (int64_t)RCH >= ((int64_t)1 << 31)) throw Error(1, "cg: n0 too large for 32-bit chunk offsets");
  const int nb2 = (int)std::min<int64_t>(256, cdiv(n0, 64));
  double* part0 = work;
  double* part1 = part0 + NB * 2 * CG_MAXK;
  double* partP = part1 + NB * 2 * CG_MAXK;
  CGScal* sc = (CGScal*)(partP + (int64_t)nb2 * PW);
  double* vec = (double*)sc + SC_D;
  const int64_t vs = n0 * CG_MAXK;
  CGArgs a{n0, k, D, H0.rp, H0.rend, H0.col, H0.val64, H0.val32, shift, Ps, rowb, x,
           r, {vec, vec + 3 * vs}, vec + 6 * vs, vec + 7 * vs, {part0, part1}, partP, nb2, sc, tol * tol};
  // r <- P b (ccoef = Ps^T b), x = p = s_{-1} = 0
  k_cg_psT<<<nb2, 1024, 0, s>>>(a, r);
  k_cg_project<<<nb2, 1024, 0, s>>>(a, r, ccoef, 1);
  SPPC_LAUNCH_CHECK();
  const bool f64 = H0.val64 != nullptr;
  // the pipelined form (one gathered vector per entry) for loose tolerances; its recursively
  // updated residual drifts from the true one, so tight tolerances keep the classical form
  const bool pipe = tol >= 1e-9;
#define SPPC_CG_LAUNCH(BB, INIT, J)                                                \
  if (INIT) {                                                                       \
    if (f64) k_cg_iter<BB, double, true, false><<<NB, NT, 0, s>>>(a, J);            \
    else k_cg_iter<BB, float, true, false><<<NB, NT, 0, s>>>(a, J);                 \
  } else if (pipe) {                                                                \
    if (f64) k_cg_iter<BB, double, false, true><<<NB, NT, 0, s>>>(a, J);            \
    else k_cg_iter<BB, float, false, true><<<NB, NT, 0, s>>>(a, J);                 \
  } else {                                                                          \
    if (f64) k_cg_iter<BB, double, false, false><<<NB, NT, 0, s>>>(a, J);           \
    else k_cg_iter<BB, float, false, false><<<NB, NT, 0, s>>>(a, J);                \
  }
#define SPPC_CG_STEP(INIT, J)      \
  if (k <= 4) {                    \
    SPPC_CG_LAUNCH(4, INIT, J)     \
  } else if (k <= 8) {             \
    SPPC_CG_LAUNCH(8, INIT, J)     \
  } else {                         \
    SPPC_CG_LAUNCH(16, INIT, J)    \
  }
  SPPC_CG_STEP(true, 0)
  // The active count is read back after every 16 iterations without draining the stream: the
  // host waits for the count of the batch before the one just queued, so the GPU always has a
  // batch to run.  Iterations queued after convergence return at once.
  hipEvent_t ev[2] = {nullptr, nullptr};
  auto cleanup = [&]() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  };
  try {
    SPPC_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    SPPC_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    int batch = 0;
    for (int j = 0; j < maxit; ++j) {
      SPPC_CG_STEP(false, j)
      if ((j + 1) % 16 == 0 || j + 1 == maxit) {
        SPPC_LAUNCH_CHECK();
        SPPC_HIP(hipMemcpyAsync(host_flag + (batch & 1), &sc->nact[j & 1], sizeof(int), hipMemcpyDeviceToHost, s));
        SPPC_HIP(hipEventRecord(ev[batch & 1], s));
        if (batch > 0) {
          SPPC_HIP(hipEventSynchronize(ev[(batch - 1) & 1]));
          if (host_flag[(batch - 1) & 1] == 0) break;
        }
        ++batch;
      }
    }
  } catch (...) {
    (void)hipStreamSynchronize(s);
    cleanup();
    throw;
  }
  cleanup();
#undef SPPC_CG_STEP
#undef SPPC_CG_LAUNCH
  // x <- P x (removes the drift into the deflated directions)
  k_cg_psT<<<nb2, 1024, 0, s>>>(a, x);
  k_cg_project<<<nb2, 1024, 0, s>>>(a, x, nullptr, 0);
  SPPC_LAUNCH_CHECK();
  SPPC_HIP(hipMemcpyAsync(host_flag, &sc->iters, sizeof(int), hipMemcpyDeviceToHost, s));
  SPPC_HIP(hipStreamSynchronize(s));
  return *host_flag;
}

}  // namespace sppc
