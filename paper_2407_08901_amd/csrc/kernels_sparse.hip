// kernels_sparse.hip - device format of H and the block product Y = H X.
//
// H arrives as its upper triangle (CSR, columns >= row).  The product needs both
// triangles: the transposed half would otherwise be a scatter with float64
// atomics (k of them per stored entry), which costs more HBM/L2 traffic than
// streaming the mirrored entries and is not deterministic.  So setup mirrors the
// strict upper triangle into a full CSR with ascending columns per row, with no
// atomics in the arithmetic and a deterministic entry order.
#include "common.h"

#include <algorithm>
#include <vector>

namespace sppc {

namespace {

// -------------------------------------------------------------------------- setup

template <typename VT>
__global__ void k_validate_count(int64_t n, const int64_t* __restrict__ rp,
                                 const int32_t* __restrict__ col, const VT* __restrict__ val,
                                 int32_t* __restrict__ lower_cnt, int* __restrict__ flags) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= n) return;
  const int64_t b = rp[row], e = rp[row + 1];
  int bad = 0, inexact = 0, nonfinite = 0;
  if (e < b) bad = 1;
  for (int64_t t = b + lane; t < e; t += 64) {
    const int32_t c = col[t];
    if (c < row || c >= n) bad = 1;
    if (t > b && col[t - 1] >= c) bad = 1;
    const double v = (double)val[t];
    if (!isfinite(v)) nonfinite = 1;
    if ((double)(float)v != v) inexact = 1;
    if (c != row && c < n && c > row) atomicAdd(&lower_cnt[c], 1);
  }
  if (bad) atomicOr(&flags[0], 1);
  if (inexact) atomicOr(&flags[1], 1);
  if (nonfinite) atomicOr(&flags[2], 1);
}

// exclusive scan of int32 counts into int64, three phases
constexpr int SCAN_BLOCK = 1024;

__global__ void k_scan_blocks(int64_t n, const int32_t* __restrict__ a, int64_t* __restrict__ bsum) {
  __shared__ int64_t sh[SCAN_BLOCK / 64];
  const int64_t i = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
  int64_t v = i < n ? a[i] : 0;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t s = 0;
    for (int w = 0; w < SCAN_BLOCK / 64; ++w) s += sh[w];
    bsum[blockIdx.x] = s;
  }
}

__global__ void k_scan_sums(int64_t nb, int64_t* __restrict__ bsum) {
  // single block: sequential chunks of blockDim.x, exclusive in place
  __shared__ int64_t sh[1024];
  int64_t carry = 0;
  for (int64_t base = 0; base < nb; base += blockDim.x) {
    const int64_t i = base + threadIdx.x;
    const int64_t v = i < nb ? bsum[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < (int)blockDim.x; o <<= 1) {
      int64_t t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nb) bsum[i] = carry + sh[threadIdx.x] - v;
    const int64_t tot = sh[blockDim.x - 1];
    __syncthreads();
    carry += tot;
  }
}

__global__ void k_scan_final(int64_t n, const int32_t* __restrict__ a, const int64_t* __restrict__ bsum,
                             int64_t* __restrict__ out) {
  __shared__ int64_t sh[SCAN_BLOCK];
  const int64_t i = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
  const int64_t v = i < n ? a[i] : 0;
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < SCAN_BLOCK; o <<= 1) {
    int64_t t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < n) out[i] = bsum[blockIdx.x] + sh[threadIdx.x] - v;
  if (i == n - 1) out[n] = bsum[blockIdx.x] + sh[threadIdx.x];
}

void scan_exclusive_impl(int64_t n, const int32_t* a, int64_t* out, int64_t* bsum, hipStream_t s) {
  const int64_t nb = cdiv(n, SCAN_BLOCK);
  k_scan_blocks<<<nb, SCAN_BLOCK, 0, s>>>(n, a, bsum);
  k_scan_sums<<<1, 1024, 0, s>>>(nb, bsum);
  k_scan_final<<<nb, SCAN_BLOCK, 0, s>>>(n, a, bsum, out);
  SPPC_LAUNCH_CHECK();
}

__global__ void k_full_rowptr(int64_t n, const int64_t* __restrict__ lower_rp,
                              const int64_t* __restrict__ up_rp, int64_t* __restrict__ full_rp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= n) full_rp[i] = lower_rp[i] + up_rp[i];
}

template <typename VT>
__global__ void k_fill(int64_t n, const int64_t* __restrict__ up_rp, const int32_t* __restrict__ up_col,
                       const VT* __restrict__ up_val, const int64_t* __restrict__ lower_rp,
                       const int64_t* __restrict__ full_rp, int32_t* __restrict__ fillc,
                       int32_t* __restrict__ full_col, double* __restrict__ full_v64,
                       float* __restrict__ full_v32, int32_t* __restrict__ tmp_col,
                       double* __restrict__ tmp_val) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= n) return;
  const int64_t b = up_rp[row], e = up_rp[row + 1];
  const int64_t nlow = lower_rp[row + 1] - lower_rp[row];
  const int64_t dst = full_rp[row] + nlow;
  for (int64_t t = b + lane; t < e; t += 64) {
    const int32_t c = up_col[t];
    const double v = (double)up_val[t];
    const int64_t o = dst + (t - b);
    full_col[o] = c;
    if (full_v64) full_v64[o] = v;
    if (full_v32) full_v32[o] = (float)v;
    if (c != row) {
      const int32_t slot = atomicAdd(&fillc[c], 1);
      const int64_t q = lower_rp[c] + slot;
      tmp_col[q] = (int32_t)row;
      tmp_val[q] = v;
    }
  }
}

// The mirrored entries of a row arrive in arbitrary order; place each at its rank
// (column indices in a row are unique), which is deterministic.
__global__ void k_sort_lower(int64_t n, const int64_t* __restrict__ lower_rp,
                             const int64_t* __restrict__ full_rp, const int32_t* __restrict__ tmp_col,
                             const double* __restrict__ tmp_val, int32_t* __restrict__ full_col,
                             double* __restrict__ full_v64, float* __restrict__ full_v32) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= n) return;
  const int64_t b = lower_rp[row], e = lower_rp[row + 1];
  const int64_t L = e - b;
  const int64_t dst = full_rp[row];
  for (int64_t t = lane; t < L; t += 64) {
    const int32_t key = tmp_col[b + t];
    int64_t rank = 0;
    for (int64_t f = 0; f < L; ++f) rank += tmp_col[b + f] < key;
    full_col[dst + rank] = key;
    const double v = tmp_val[b + t];
    if (full_v64) full_v64[dst + rank] = v;
    if (full_v32) full_v32[dst + rank] = (float)v;
  }
}

__global__ void k_block_view(int64_t n0, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                             int64_t* __restrict__ rend) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n0) return;
  int64_t lo = rp[i], hi = rp[i + 1];  // first position with col >= n0
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (col[mid] < n0) lo = mid + 1; else hi = mid;
  }
  rend[i] = lo;
}

__global__ void k_diag(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                       const double* __restrict__ v64, const float* __restrict__ v32,
                       double* __restrict__ diag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t lo = rp[i], hi = rp[i + 1];
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (col[mid] < i) lo = mid + 1; else hi = mid;
  }
  double d = 0.0;
  if (lo < rp[i + 1] && col[lo] == i) d = v64 ? v64[lo] : (double)v32[lo];
  diag[i] = d;
}

// -------------------------------------------------------------------------- SpMM
//
// One wave per row.  The wave loads 64 (column, value) pairs of its row at a time
// (coalesced stream), then groups of B lanes take one nonzero each: the B lanes of a
// group read the B contiguous entries of the gathered row of X (one 8*B-byte segment)
// and accumulate into one float64 register per lane.  The groups are summed with
// cross-lane shuffles at the end of the row.
template <int B, typename VT, typename XT>
__global__ __launch_bounds__(256) void k_spmm(int64_t n, const int64_t* __restrict__ rp,
                                              const int64_t* __restrict__ rend,
                                              const int32_t* __restrict__ col,
                                              const VT* __restrict__ val, const XT* __restrict__ X,
                                              int64_t ldx, double* __restrict__ Y, int64_t ldy, int b,
                                              const double* __restrict__ shift, double ea, double ec,
                                              double eb, const double* __restrict__ Zo, int64_t ldz,
                                              const double* __restrict__ dg, const double* __restrict__ X64,
                                              int64_t ldx64) {
  constexpr int G = 64 / B;
  const int lane = threadIdx.x & 63;
  const int g = lane / B;
  const int c = lane % B;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const int64_t beg = rp[row];
  const int64_t end = rend ? rend[row] : rp[row + 1];
  const bool colok = c < b;
  double acc = 0.0;
  for (int64_t base = beg; base < end; base += 64) {
    const int cnt = (int)min<int64_t>(64, end - base);
    int32_t mc = 0;
    VT mv = VT(0);
    if (lane < cnt) {
      mc = __builtin_nontemporal_load(&col[base + lane]);
      mv = __builtin_nontemporal_load(&val[base + lane]);
    }
#pragma unroll 4
    for (int s0 = 0; s0 < cnt; s0 += G) {
      const int e = s0 + g;
      const int32_t cc = __shfl(mc, e);
      const VT vv = __shfl(mv, e);
      if (e < cnt && colok && !(dg && cc == row)) {
        const XT xv = X[(int64_t)cc * ldx + c];
        if constexpr (sizeof(XT) == 4) {
          acc += (double)(vv * xv);            // float32 product, float64 accumulation
        } else {
          acc = fma((double)vv, (double)xv, acc);
        }
      }
    }
  }
#pragma unroll
  for (int o = B; o < 64; o <<= 1) acc += __shfl_xor(acc, o);
  if (g == 0 && colok) {
    if (dg) acc = fma(dg[row], X64[row * ldx64 + c], acc);  // diagonal term in float64
    if (shift) acc -= shift[c] * (double)X[row * ldx + c];
    if (Zo) acc = ea * (acc - ec * (double)X[row * ldx + c]) + eb * Zo[row * ldz + c];
    Y[row * ldy + c] = acc;
  }
}

template <typename VT, typename XT>
void launch_spmm(const DevCSR& H, const VT* val, const XT* X, int64_t ldx, double* Y, int64_t ldy,
                 int b, const double* shift, hipStream_t s, double ea = 0.0, double ec = 0.0,
                 double eb = 0.0, const double* Zo = nullptr, int64_t ldz = 0, const double* dg = nullptr,
                 const double* X64 = nullptr, int64_t ldx64 = 0) {
  if (b < 1 || b > 32) throw Error(1, "spmm: block width must be 1..32");
  if (H.n == 0) return;
  const int64_t grid = cdiv(H.n, 4);
#define SPPC_SPMM_CASE(BB)                                                                        \
  k_spmm<BB, VT, XT><<<grid, 256, 0, s>>>(H.n, H.rp, H.rend, H.col, val, X, ldx, Y, ldy, b, shift, ea, ec, \
                                          eb, Zo, ldz, dg, X64, ldx64);                                     \
  break;
  switch (b <= 1 ? 1 : b <= 2 ? 2 : b <= 4 ? 4 : b <= 8 ? 8 : b <= 16 ? 16 : 32) {
    case 1: SPPC_SPMM_CASE(1)
    case 2: SPPC_SPMM_CASE(2)
    case 4: SPPC_SPMM_CASE(4)
    case 8: SPPC_SPMM_CASE(8)
    case 16: SPPC_SPMM_CASE(16)
    default: SPPC_SPMM_CASE(32)
  }
#undef SPPC_SPMM_CASE
  SPPC_LAUNCH_CHECK();
}

// rows [0, n0) restricted to columns < n0 (the row ends of the view), copied contiguously
__global__ void k_view_count(int64_t n0, const int64_t* __restrict__ rp, const int64_t* __restrict__ rend,
                             int32_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n0) cnt[i] = (int32_t)(rend[i] - rp[i]);
}

__global__ void k_view_fill(int64_t n0, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                            const double* __restrict__ v64, const float* __restrict__ v32,
                            const int64_t* __restrict__ nrp, int32_t* __restrict__ ncol,
                            double* __restrict__ n64, float* __restrict__ n32) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= n0) return;
  const int64_t b = rp[row], len = nrp[row + 1] - nrp[row], d = nrp[row];
  for (int64_t t = lane; t < len; t += 64) {
    ncol[d + t] = col[b + t];
    if (n64) n64[d + t] = v64[b + t];
    if (n32) n32[d + t] = v32[b + t];
  }
}

// ------------------------------------------------------------------ panel format
//
// Block product over the row-block x column-panel copy (PanelH).  One workgroup per row
// block; all workgroups sweep the panels in the same order, so the panel of X that the
// resident workgroups gather from stays in L2.  Each wave owns RB/4 consecutive rows, whose
// entries in one panel are contiguous; the wave streams them in windows of 64 (one coalesced
// load of columns and values).  Group g of B lanes takes the B consecutive entries
// g*B .. g*B+B-1 of the window, lane c reading column c of each gathered row of X, and sums runs
// of entries of the same row in a register; a run is added to the row's LDS accumulator
// when it ends.  Runs that straddle two groups meet in the same LDS add instruction.
template <int B, typename VT, typename XT>
__global__ __launch_bounds__(256) void k_spmm_panel(int64_t n, int RB, int P, int PW,
                                                    const int32_t* __restrict__ off,
                                                    const int64_t* __restrict__ bstart,
                                                    const uint16_t* __restrict__ pcol,
                                                    const VT* __restrict__ pval, const XT* __restrict__ X,
                                                    int64_t ldx, double* __restrict__ Y, int64_t ldy, int b,
                                                    int blk0, const double* __restrict__ dg,
                                                    const double* __restrict__ X64, int64_t ldx64) {
  constexpr int E = B;  // entries per group and window: 64/B groups share the 64 entries
  extern __shared__ double ysh[];  // RB * B accumulators, then RB + 1 ints
  int* soff = (int*)(ysh + (size_t)RB * B);
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int g = lane / B, c = lane % B;
  const int64_t blk = blk0 + (int64_t)blockIdx.x;
  const int64_t row0 = blk * RB;
  const int nr = (int)min<int64_t>(RB, n - row0);
  const int32_t* boff = off + blk * ((int64_t)P * RB + 1);
  const VT* bval = pval + bstart[blk];
  const uint16_t* bcol = pcol + bstart[blk];
  const int WR = RB / 4;
  const int R0 = w * WR, R1 = R0 + WR;
  const bool colok = c < b;
  for (int i = t; i < RB * B; i += 256) ysh[i] = 0.0;
  for (int p = 0; p < P; ++p) {
    __syncthreads();  // previous panel's offsets are no longer read; accumulators zeroed
    for (int i = t; i <= RB; i += 256) soff[i] = boff[(int64_t)p * RB + i];
    __syncthreads();
    const int a = soff[R0], z = soff[R1];
    const XT* Xp = X + (int64_t)p * PW * ldx + c;
    // the window after the current one is loaded while the current one is processed; the
    // matrix is read once, streaming (nontemporal), so it does not evict the panel of X
    int nc = 0;
    VT nv = VT(0);
    if (a + lane < z) {
      nc = (int)__builtin_nontemporal_load(&bcol[a + lane]);
      nv = __builtin_nontemporal_load(&bval[a + lane]);
    }
    for (int win = a; win < z; win += 64) {
      const int e = win + lane;
      const int mc = nc;
      const VT mv = nv;
      int mr = R0;
      if (e < z) {
        // row of entry e: last r in [R0, R1) with soff[r] <= e
        int lo = R0, hi = R1 - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (soff[mid] <= e) lo = mid; else hi = mid - 1;
        }
        mr = lo;
      }
      XT xv[E];
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int src = g * E + q;
        const int cc = __shfl(mc, src);
        bool use = win + src < z && colok;
        if (dg && use) use = (int64_t)p * PW + cc != row0 + __shfl(mr, src);  // diagonal: float64 below
        xv[q] = use ? Xp[(int64_t)cc * ldx] : XT(0);
      }
      // loads return in issue order: the next window is requested after the gathers, so
      // waiting for the gathered values does not wait for the (HBM) window load
      asm volatile("" ::: "memory");
      if (e + 64 < z) {
        nc = (int)__builtin_nontemporal_load(&bcol[e + 64]);
        nv = __builtin_nontemporal_load(&bval[e + 64]);
      }
      int cur_r = __shfl(mr, g * E);
      double cur = 0.0;
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int src = g * E + q;
        const VT vv = __shfl(mv, src);
        const int rr = __shfl(mr, src);
        if (win + src < z) {
          if (rr != cur_r) {
            atomicAdd(&ysh[cur_r * B + c], cur);
            cur = 0.0;
            cur_r = rr;
          }
          if constexpr (sizeof(XT) == 4) {
            cur += (double)(vv * xv[q]);  // float32 product, float64 accumulation
          } else {
            cur = fma((double)vv, (double)xv[q], cur);
          }
        }
      }
      if (win + g * E < z) atomicAdd(&ysh[cur_r * B + c], cur);
    }
  }
  __syncthreads();
  for (int i = t; i < nr * B; i += 256) {
    const int rr = i / B, cc = i % B;
    if (cc < b) {
      double y = ysh[i];
      if (dg) y = fma(dg[row0 + rr], X64[(row0 + rr) * ldx64 + cc], y);
      Y[(row0 + rr) * ldy + cc] = y;
    }
  }
}

// Workgroups of one launch start together and sweep the panels in step; when the blocks do
// not all fit on the device at once they are split into rounds of at most the resident count,
// one launch each, so that a later round does not start at staggered times.
template <int B, typename VT, typename XT>
void spmm_panel_rounds(const PanelH& P, const VT* val, const XT* X, int64_t ldx, double* Y, int64_t ldy, int b,
                       hipStream_t s, const double* dg, const double* X64, int64_t ldx64) {
  const size_t lds = sizeof(double) * (size_t)P.RB * B + sizeof(int) * (size_t)(P.RB + 1);
  static int resident = 0;  // per instantiation, computed once per process
  if (resident == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    SPPC_HIP(hipGetDevice(&dev));
    SPPC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    SPPC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_spmm_panel<B, VT, XT>, 256, lds));
    resident = std::max(1, cus * std::max(1, per_cu));
  }
  const int cap = resident;
  const int rounds = (int)cdiv(P.nblocks, cap);
  const int per = (int)cdiv(P.nblocks, rounds);  // equal rounds
  for (int r0 = 0; r0 < P.nblocks; r0 += per) {
    const int nb = std::min(per, P.nblocks - r0);
    k_spmm_panel<B, VT, XT><<<nb, 256, lds, s>>>(P.n, P.RB, P.P, P.PW, P.off, P.bstart, P.col, val, X, ldx, Y,
                                                 ldy, b, r0, dg, X64, ldx64);
  }
  SPPC_LAUNCH_CHECK();
}

template <typename VT, typename XT>
void launch_spmm_panel(const PanelH& P, const VT* val, const XT* X, int64_t ldx, double* Y, int64_t ldy, int b,
                       hipStream_t s, const double* dg = nullptr, const double* X64 = nullptr,
                       int64_t ldx64 = 0) {
  if (b <= 4)
    spmm_panel_rounds<4, VT, XT>(P, val, X, ldx, Y, ldy, b, s, dg, X64, ldx64);
  else if (b <= 8)
    spmm_panel_rounds<8, VT, XT>(P, val, X, ldx, Y, ldy, b, s, dg, X64, ldx64);
  else
    spmm_panel_rounds<16, VT, XT>(P, val, X, ldx, Y, ldy, b, s, dg, X64, ldx64);
}

// first entry of row [b, e) with column >= key (columns ascending)
__device__ inline int64_t lower_col(const int32_t* __restrict__ col, int64_t b, int64_t e, int64_t key) {
  while (b < e) {
    const int64_t mid = (b + e) >> 1;
    if (col[mid] < key) b = mid + 1; else e = mid;
  }
  return b;
}

// cnt[blk][p*RB + r] = entries of row r of block blk in panel p (one wave per row; the lane
// that holds the last entry of a panel run writes its length)
__global__ void k_panel_count(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                              int RB, int P, int PW, int32_t* __restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= n) return;
  const int64_t b = rp[row], e = rp[row + 1];
  const int64_t blk = row / RB;
  const int rl = (int)(row - blk * RB);
  for (int64_t t = b + lane; t < e; t += 64) {
    const int p = col[t] / PW;
    if (t + 1 == e || col[t + 1] / PW != p) {
      const int64_t st = lower_col(col, b, t, (int64_t)p * PW);
      cnt[blk * ((int64_t)P * RB) + (int64_t)p * RB + rl] = (int32_t)(t - st + 1);
    }
  }
}

// relative offsets per block from the global exclusive scan of the counts
__global__ void k_panel_offsets(int nblocks, int64_t per_block, const int64_t* __restrict__ gscan,
                                int32_t* __restrict__ off, int64_t* __restrict__ bstart) {
  const int64_t blk = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > per_block) return;
  const int64_t base = gscan[blk * per_block];
  off[blk * (per_block + 1) + i] = (int32_t)(gscan[blk * per_block + i] - base);
  if (i == 0) {
    bstart[blk] = base;
    if (blk + 1 == nblocks) bstart[nblocks] = gscan[(int64_t)nblocks * per_block];
  }
}

template <typename VT>
__global__ void k_panel_fill(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                             const VT* __restrict__ val, int RB, int P, int PW, const int32_t* __restrict__ off,
                             const int64_t* __restrict__ bstart, uint16_t* __restrict__ pcol,
                             VT* __restrict__ pval) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= n) return;
  const int64_t b = rp[row], e = rp[row + 1];
  const int64_t blk = row / RB;
  const int rl = (int)(row - blk * RB);
  const int64_t per = (int64_t)P * RB + 1;
  for (int64_t t = b + lane; t < e; t += 64) {
    const int c = col[t];
    const int p = c / PW;
    const int64_t st = lower_col(col, b, t, (int64_t)p * PW);
    const int64_t dst = bstart[blk] + off[blk * per + (int64_t)p * RB + rl] + (t - st);
    pcol[dst] = (uint16_t)(c - p * PW);
    pval[dst] = val[t];
  }
}

// upper Gershgorin bound of each row: d_i + sum_{j != i} |a_ij|
__global__ void k_gersh(int64_t n, const int64_t* __restrict__ rp, const int64_t* __restrict__ rend,
                        const int32_t* __restrict__ col, const double* __restrict__ v64,
                        const float* __restrict__ v32, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const int64_t b = rp[row], e = rend ? rend[row] : rp[row + 1];
  double s = 0.0;
  for (int64_t t = b + lane; t < e; t += 64) {
    const double v = v64 ? v64[t] : (double)v32[t];
    s += col[t] == row ? v : fabs(v);
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) out[row] = s;
}

__global__ void k_max_reduce(int64_t n, const double* __restrict__ x, double* __restrict__ out) {
  __shared__ double sh[1024];
  double m = -INFINITY;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, x[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < (unsigned)o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

}  // namespace

void gershgorin_upper(const DevCSR& H, double* tmp, double* out, hipStream_t s) {
  k_gersh<<<cdiv(H.n, 4), 256, 0, s>>>(H.n, H.rp, H.rend, H.col, H.val64, H.val32, tmp);
  k_max_reduce<<<1, 1024, 0, s>>>(H.n, tmp, out);
  SPPC_LAUNCH_CHECK();
}

void spmm_cheb(const DevCSR& H, const double* X, int64_t ldx, double* Y, int64_t ldy, int b, double ea,
               double ec, double eb, const double* Zo, int64_t ldz, hipStream_t s) {
  if (H.val64)
    launch_spmm<double, double>(H, H.val64, X, ldx, Y, ldy, b, nullptr, s, ea, ec, eb, Zo, ldz);
  else
    launch_spmm<float, double>(H, H.val32, X, ldx, Y, ldy, b, nullptr, s, ea, ec, eb, Zo, ldz);
}

void build_full_csr(int64_t n, int64_t nnz_up, const int64_t* up_rp, const int32_t* up_col,
                    const void* up_val, int val_is_f32, DevCSR& out, int* d_flags, bool want64,
                    bool want32, bool& exact32, hipStream_t s) {
  int32_t *lower_cnt = nullptr, *fillc = nullptr, *tmp_col = nullptr;
  int64_t *lower_rp = nullptr, *bsum = nullptr;
  double* tmp_val = nullptr;
  auto cleanup = [&]() {
    hipFree(lower_cnt); hipFree(fillc); hipFree(tmp_col); hipFree(lower_rp); hipFree(bsum);
    hipFree(tmp_val);
  };
  try {
    SPPC_HIP(hipMalloc(&lower_cnt, sizeof(int32_t) * (n + 1)));
    SPPC_HIP(hipMalloc(&fillc, sizeof(int32_t) * (n + 1)));
    SPPC_HIP(hipMalloc(&lower_rp, sizeof(int64_t) * (n + 1)));
    SPPC_HIP(hipMalloc(&bsum, sizeof(int64_t) * (cdiv(n, SCAN_BLOCK) + 1)));
    SPPC_HIP(hipMemsetAsync(lower_cnt, 0, sizeof(int32_t) * (n + 1), s));
    SPPC_HIP(hipMemsetAsync(fillc, 0, sizeof(int32_t) * (n + 1), s));
    SPPC_HIP(hipMemsetAsync(d_flags, 0, sizeof(int) * 4, s));
    const int64_t grid_w = cdiv(n, 4);
    if (val_is_f32)
      k_validate_count<float><<<grid_w, 256, 0, s>>>(n, up_rp, up_col, (const float*)up_val, lower_cnt, d_flags);
    else
      k_validate_count<double><<<grid_w, 256, 0, s>>>(n, up_rp, up_col, (const double*)up_val, lower_cnt, d_flags);
    SPPC_LAUNCH_CHECK();
    int h_flags[4];
    SPPC_HIP(hipMemcpyAsync(h_flags, d_flags, sizeof(h_flags), hipMemcpyDeviceToHost, s));
    SPPC_HIP(hipStreamSynchronize(s));
    if (h_flags[0]) throw Error(1, "H: upper CSR expected (columns >= row, < n, strictly ascending)");
    if (h_flags[2]) throw Error(7, "H: NaN or Inf among the values");
    exact32 = val_is_f32 || !h_flags[1];
    scan_exclusive_impl(n, lower_cnt, lower_rp, bsum, s);
    int64_t nlow = 0;
    SPPC_HIP(hipMemcpyAsync(&nlow, lower_rp + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPPC_HIP(hipStreamSynchronize(s));
    const int64_t nnz = nnz_up + nlow;
    out.n = n;
    out.nnz = nnz;
    SPPC_HIP(hipMalloc(&out.rp, sizeof(int64_t) * (n + 1)));
    SPPC_HIP(hipMalloc(&out.col, sizeof(int32_t) * (nnz > 0 ? nnz : 1)));
    if (want64) SPPC_HIP(hipMalloc(&out.val64, sizeof(double) * (nnz > 0 ? nnz : 1)));
    if (want32) SPPC_HIP(hipMalloc(&out.val32, sizeof(float) * (nnz > 0 ? nnz : 1)));
    SPPC_HIP(hipMalloc(&tmp_col, sizeof(int32_t) * (nlow > 0 ? nlow : 1)));
    SPPC_HIP(hipMalloc(&tmp_val, sizeof(double) * (nlow > 0 ? nlow : 1)));
    k_full_rowptr<<<cdiv(n + 1, 256), 256, 0, s>>>(n, lower_rp, up_rp, out.rp);
    if (val_is_f32)
      k_fill<float><<<grid_w, 256, 0, s>>>(n, up_rp, up_col, (const float*)up_val, lower_rp, out.rp, fillc,
                                           out.col, out.val64, out.val32, tmp_col, tmp_val);
    else
      k_fill<double><<<grid_w, 256, 0, s>>>(n, up_rp, up_col, (const double*)up_val, lower_rp, out.rp,
                                            fillc, out.col, out.val64, out.val32, tmp_col, tmp_val);
    k_sort_lower<<<grid_w, 256, 0, s>>>(n, lower_rp, out.rp, tmp_col, tmp_val, out.col, out.val64,
                                        out.val32);
    SPPC_LAUNCH_CHECK();
    SPPC_HIP(hipStreamSynchronize(s));
  } catch (...) {
    cleanup();
    throw;
  }
  cleanup();
}

void build_block_view(const DevCSR& full, int64_t n0, int64_t* rend, hipStream_t s) {
  if (n0 == 0) return;
  k_block_view<<<cdiv(n0, 256), 256, 0, s>>>(n0, full.rp, full.col, rend);
  SPPC_LAUNCH_CHECK();
}

void compact_view(const DevCSR& V, DevCSR& out, hipStream_t s) {
  const int64_t n0 = V.n;
  if (!V.rend) throw Error(1, "compact_view: not a block view");
  int32_t* cnt = nullptr;
  int64_t* bsum = nullptr;
  auto cleanup = [&]() { hipFree(cnt); hipFree(bsum); };
  try {
    out = DevCSR{};
    out.n = n0;
    SPPC_HIP(hipMalloc(&cnt, sizeof(int32_t) * (n0 + 1)));
    SPPC_HIP(hipMalloc(&bsum, sizeof(int64_t) * (cdiv(n0 + 1, SCAN_BLOCK) + 1)));
    SPPC_HIP(hipMalloc(&out.rp, sizeof(int64_t) * (n0 + 1)));
    k_view_count<<<cdiv(n0 > 0 ? n0 : 1, 256), 256, 0, s>>>(n0, V.rp, V.rend, cnt);
    SPPC_LAUNCH_CHECK();
    scan_exclusive_impl(n0, cnt, out.rp, bsum, s);
    int64_t nnz = 0;
    SPPC_HIP(hipMemcpyAsync(&nnz, out.rp + n0, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPPC_HIP(hipStreamSynchronize(s));
    out.nnz = nnz;
    SPPC_HIP(hipMalloc(&out.col, sizeof(int32_t) * (nnz > 0 ? nnz : 1)));
    if (V.val64) SPPC_HIP(hipMalloc(&out.val64, sizeof(double) * (nnz > 0 ? nnz : 1)));
    if (V.val32) SPPC_HIP(hipMalloc(&out.val32, sizeof(float) * (nnz > 0 ? nnz : 1)));
    k_view_fill<<<cdiv(n0 > 0 ? n0 : 1, 4), 256, 0, s>>>(n0, V.rp, V.col, V.val64, V.val32, out.rp, out.col,
                                                          out.val64, out.val32);
    SPPC_LAUNCH_CHECK();
    SPPC_HIP(hipStreamSynchronize(s));
  } catch (...) {
    cleanup();
    (void)hipFree(out.rp); (void)hipFree(out.col); (void)hipFree(out.val64); (void)hipFree(out.val32);
    out = DevCSR{};
    throw;
  }
  cleanup();
}

void extract_diag(const DevCSR& H, double* diag, hipStream_t s) {
  k_diag<<<cdiv(H.n, 256), 256, 0, s>>>(H.n, H.rp, H.col, H.val64, H.val32, diag);
  SPPC_LAUNCH_CHECK();
}

void build_panel(const DevCSR& H, int PW, int RB, PanelH& out, hipStream_t s) {
  if (PW < 1 || PW > 65536 || RB < 64 || RB % 64 != 0) throw Error(1, "panel: bad width or block size");
  const int64_t n = H.n;
  out.n = n;
  out.RB = RB;
  out.PW = PW;
  out.P = (int)cdiv(n, PW);
  out.nblocks = (int)cdiv(n, RB);
  const int64_t per = (int64_t)out.P * RB;
  const int64_t total = per * out.nblocks;
  if (total >= ((int64_t)1 << 31)) throw Error(1, "panel: too many (row, panel) pairs");
  int32_t* cnt = nullptr;
  int64_t *gscan = nullptr, *bsum = nullptr;
  auto cleanup = [&]() { hipFree(cnt); hipFree(gscan); hipFree(bsum); };
  try {
    SPPC_HIP(hipMalloc(&cnt, sizeof(int32_t) * total));
    SPPC_HIP(hipMalloc(&gscan, sizeof(int64_t) * (total + 1)));
    SPPC_HIP(hipMalloc(&bsum, sizeof(int64_t) * (cdiv(total, SCAN_BLOCK) + 1)));
    SPPC_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * total, s));
    const int64_t grid_w = cdiv(n, 4);
    k_panel_count<<<grid_w, 256, 0, s>>>(n, H.rp, H.col, RB, out.P, PW, cnt);
    scan_exclusive_impl(total, cnt, gscan, bsum, s);
    SPPC_HIP(hipMalloc(&out.off, sizeof(int32_t) * (per + 1) * out.nblocks));
    SPPC_HIP(hipMalloc(&out.bstart, sizeof(int64_t) * (out.nblocks + 1)));
    // a block holds fewer than 2^31 entries: RB rows of at most n columns each
    if ((int64_t)RB * n >= ((int64_t)1 << 31)) {
      int64_t big = 0;
      // checked after the scan: the largest block
      std::vector<int64_t> hs(out.nblocks + 1);
      SPPC_HIP(hipStreamSynchronize(s));
      for (int q = 0; q <= out.nblocks; ++q)
        SPPC_HIP(hipMemcpy(&hs[q], gscan + (int64_t)q * per, sizeof(int64_t), hipMemcpyDeviceToHost));
      for (int q = 0; q < out.nblocks; ++q) big = std::max(big, hs[q + 1] - hs[q]);
      if (big >= ((int64_t)1 << 31)) throw Error(1, "panel: block with 2^31 entries");
    }
    dim3 g2((unsigned)cdiv(per + 1, 256), (unsigned)out.nblocks);
    k_panel_offsets<<<g2, 256, 0, s>>>(out.nblocks, per, gscan, out.off, out.bstart);
    const int64_t nnz = H.nnz;
    SPPC_HIP(hipMalloc(&out.col, sizeof(uint16_t) * (nnz > 0 ? nnz : 1)));
    if (H.val64) {
      SPPC_HIP(hipMalloc(&out.val64, sizeof(double) * (nnz > 0 ? nnz : 1)));
      k_panel_fill<double><<<grid_w, 256, 0, s>>>(n, H.rp, H.col, H.val64, RB, out.P, PW, out.off, out.bstart,
                                                   out.col, out.val64);
    }
    if (H.val32) {
      SPPC_HIP(hipMalloc(&out.val32, sizeof(float) * (nnz > 0 ? nnz : 1)));
      k_panel_fill<float><<<grid_w, 256, 0, s>>>(n, H.rp, H.col, H.val32, RB, out.P, PW, out.off, out.bstart,
                                                 out.col, out.val32);
    }
    SPPC_LAUNCH_CHECK();
    SPPC_HIP(hipStreamSynchronize(s));
  } catch (...) {
    cleanup();
    release_panel(out);
    throw;
  }
  cleanup();
}

void scan_exclusive(int64_t n, const int32_t* a, int64_t* out, int64_t* bsum, hipStream_t s) {
  scan_exclusive_impl(n, a, out, bsum, s);
}

void release_panel(PanelH& p) {
  (void)hipFree(p.off);
  (void)hipFree(p.bstart);
  (void)hipFree(p.col);
  (void)hipFree(p.val32);
  (void)hipFree(p.val64);
  p = PanelH{};
}

void spmm_f64(const DevCSR& H, const double* X, int64_t ldx, double* Y, int64_t ldy, int b,
              const double* shift, hipStream_t s) {
  if (H.panel && !shift && b >= 1 && b <= 16 && H.n > 0) {
    if (H.val64)
      launch_spmm_panel<double, double>(*H.panel, H.panel->val64, X, ldx, Y, ldy, b, s);
    else
      launch_spmm_panel<float, double>(*H.panel, H.panel->val32, X, ldx, Y, ldy, b, s);
    return;
  }
  if (H.val64)
    launch_spmm<double, double>(H, H.val64, X, ldx, Y, ldy, b, shift, s);
  else
    launch_spmm<float, double>(H, H.val32, X, ldx, Y, ldy, b, shift, s);
}

void spmm_f32(const DevCSR& H, const float* X, int64_t ldx, double* Y, int64_t ldy, int b,
              const double* shift, hipStream_t s, const double* diag, const double* X64, int64_t ldx64) {
  if (!H.val32) throw Error(1, "spmm_f32: no float32 values");
  if (diag && !X64) throw Error(1, "spmm_f32: the float64 diagonal term needs float64 X");
  if (H.panel && !shift && b >= 1 && b <= 16 && H.n > 0) {
    launch_spmm_panel<float, float>(*H.panel, H.panel->val32, X, ldx, Y, ldy, b, s, diag, X64, ldx64);
    return;
  }
  launch_spmm<float, float>(H, H.val32, X, ldx, Y, ldy, b, shift, s, 0.0, 0.0, 0.0, nullptr, 0, diag, X64, ldx64);
}

}  // namespace sppc
