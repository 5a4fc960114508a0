// kernels_sparse.hip - device format of H and the block product Y = H X.
//
// H arrives as its upper triangle (CSR, columns >= row).  The product needs both
// triangles: the transposed half would otherwise be a scatter with float64
// atomics (k of them per stored entry), which costs more HBM/L2 traffic than
// streaming the mirrored entries and is not deterministic.  So setup mirrors the
// strict upper triangle into a full CSR with ascending columns per row, with no
// atomics in the arithmetic and a deterministic entry order.
#include "common.h"

#include <mutex>
#include <string>

#include <algorithm>
#include <vector>

namespace sppc {

namespace {

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// -------------------------------------------------------------------------- setup

// One wave per row: checks the upper CSR (columns >= row, < n, strictly ascending), whether
// every value is float32-exact and finite, and counts the row's strict-upper entries.
template <typename VT>
__global__ void k_validate_count(int64_t n, const int64_t* __restrict__ rp,
                                 const int32_t* __restrict__ col, const VT* __restrict__ val,
                                 int32_t* __restrict__ su_cnt, int* __restrict__ flags) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= n) return;
  const int64_t b = rp[row], e = rp[row + 1];
  int bad = 0, inexact = 0, nonfinite = 0;
  if (e < b || e - b > n - row) bad = 1;
  for (int64_t t = b + lane; t < e && !bad; t += 64) {
    const int32_t c = col[t];
    if (c < row || c >= n) bad = 1;
    if (t > b && col[t - 1] >= c) bad = 1;
    const double v = (double)val[t];
    if (!isfinite(v)) nonfinite = 1;
    if ((double)(float)v != v) inexact = 1;
  }
  if (lane == 0) su_cnt[row] = bad ? 0 : (int32_t)((e - b) - ((e > b && col[b] == row) ? 1 : 0));
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

// The mirror of the strict upper triangle is a stable sort of its entries by column: entry (r, c)
// of the upper triangle becomes entry (c, r) of the lower one, and a stable sort of the entries,
// taken in row order, by column leaves every lower row with its columns ascending.  The sort is
// a least-significant-digit radix sort (digits of at most 8 bits): per pass, a histogram of
// each tile of RS_TILE entries, an exclusive scan of the (digit, tile) counts in digit-major
// order, and a scatter in which each wave of a tile ranks its part of the tile round by round (a
// digit's peers in a round come from ballots over the digit's bits, and a wave's runs follow
// those of the waves before it), so every entry keeps its order among equal digits.  No global
// atomics, and the result does not depend on scheduling.
constexpr int RS_WAVES = 4;                 // waves per tile
constexpr int RS_WTILE = 2048;              // entries per wave
constexpr int RS_TILE = RS_WAVES * RS_WTILE;
constexpr int RS_ROUNDS = RS_WTILE / 64;

// strict-upper entries in row order: key = column, row, value (TT: float when only float32 values
// are kept)
template <typename VT, typename TT>
__global__ void k_extract_upper(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                const VT* __restrict__ val, const int64_t* __restrict__ su_off,
                                int32_t* __restrict__ key, int32_t* __restrict__ rowi, TT* __restrict__ v) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= n) return;
  const int64_t e = rp[row + 1];
  int64_t b = rp[row];
  if (e > b && col[b] == row) ++b;  // the diagonal (first, since columns ascend from row)
  const int64_t o = su_off[row];
  if (su_off[row + 1] - o != e - b) return;  // (cannot happen for a valid input)
  for (int64_t t = b + lane; t < e; t += 64) {
    key[o + (t - b)] = col[t];
    rowi[o + (t - b)] = (int32_t)row;
    v[o + (t - b)] = (TT)val[t];
  }
}

// counts of digit (key >> shift) & mask per tile, digit-major: cnt[d * ntile + tile]
__global__ __launch_bounds__(256) void k_rs_hist(int64_t m, const int32_t* __restrict__ key, int shift, int mask,
                                                 int64_t ntile, int32_t* __restrict__ cnt) {
  __shared__ int h[256];
  const int t = threadIdx.x;
  h[t] = 0;
  __syncthreads();
  const int64_t i0 = (int64_t)blockIdx.x * RS_TILE;
  const int64_t i1 = min<int64_t>(m, i0 + RS_TILE);
  for (int64_t i = i0 + t; i < i1; i += 256) atomicAdd(&h[((uint32_t)key[i] >> shift) & mask], 1);
  __syncthreads();
  if (t <= mask) cnt[(int64_t)t * ntile + blockIdx.x] = h[t];
}

// One workgroup of RS_WAVES waves per tile; wave w holds entries [w RS_WTILE, (w + 1) RS_WTILE)
// of it.  Entry i of the tile goes to off[d * ntile + tile] + (its rank among the tile's entries
// with digit d), ranks taken in tile order.  The tile is first reordered by digit in LDS
// (stable), then written out in that order, so consecutive lanes write consecutive positions of
// one digit's run and the stores coalesce: a tile of 8192 entries holds runs of 32 entries on
// average for 256 digits (a one-wave tile of 2048 left runs of 8, 32-byte stores of each array).
template <typename TT>
__global__ __launch_bounds__(64 * RS_WAVES) void k_rs_scatter(int64_t m, const int32_t* __restrict__ kin,
                                                              const int32_t* __restrict__ rin,
                                                              const TT* __restrict__ vin,
                                                              int32_t* __restrict__ kout, int32_t* __restrict__ rout,
                                                              TT* __restrict__ vout, int shift, int bits,
                                                              int64_t ntile, const int32_t* __restrict__ cnt,
                                                              const int64_t* __restrict__ off) {
  __shared__ int64_t gbase[256];           // first global position of each digit's run of this tile
  __shared__ int lbase[256];               // first position of each digit's run in the reordered tile
  __shared__ int wnext[RS_WAVES][256];     // per wave: its count of each digit, then its cursor
  __shared__ int wsum[RS_WAVES];
  __shared__ int32_t sk[RS_TILE], sr[RS_TILE];
  __shared__ TT sv[RS_TILE];
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int mask = (1 << bits) - 1;
  const int64_t i0 = (int64_t)blockIdx.x * RS_TILE;
  const int nt = (int)min<int64_t>(RS_TILE, m - i0);
  const int wb = w * RS_WTILE;  // this wave's first entry in the tile
  int32_t kk[RS_ROUNDS], rr[RS_ROUNDS];
  TT vv[RS_ROUNDS];
#pragma unroll
  for (int q = 0; q < RS_ROUNDS; ++q) {
    const int i = wb + q * 64 + lane;
    const bool ok = i < nt;
    kk[q] = ok ? kin[i0 + i] : 0;
    rr[q] = ok ? rin[i0 + i] : 0;
    vv[q] = ok ? vin[i0 + i] : TT(0);
  }
  for (int i = t; i < RS_WAVES * 256; i += 64 * RS_WAVES) (&wnext[0][0])[i] = 0;
  __syncthreads();
  // (1) each wave counts its digits
#pragma unroll
  for (int q = 0; q < RS_ROUNDS; ++q)
    if (wb + q * 64 + lane < nt) atomicAdd(&wnext[w][((uint32_t)kk[q] >> shift) & mask], 1);
  __syncthreads();
  // (2) thread d (< 256): the tile's count of digit d, an exclusive scan over the digits (a wave
  // scan, then the totals of the waves before), and each wave's cursor after the waves before it
  {
    int tot = 0;
    if (t < 256)
      for (int v = 0; v < RS_WAVES; ++v) tot += wnext[v][t];
    int inc = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    if (lane == 63 && t < 256) wsum[w] = inc;
    __syncthreads();
    if (t < 256) {
      int before = 0;
      for (int v = 0; v < w; ++v) before += wsum[v];
      const int run = before + inc - tot;
      lbase[t] = run;
      gbase[t] = t <= mask ? off[(int64_t)t * ntile + blockIdx.x] : 0;
      int c = run;
      for (int v = 0; v < RS_WAVES; ++v) {
        const int cv = wnext[v][t];
        wnext[v][t] = c;
        c += cv;
      }
    }
  }
  __syncthreads();
  // (3) ranking within each wave, in rounds of 64 entries in order
  const unsigned long long below = (1ull << lane) - 1ull;
  int* lnext = wnext[w];
#pragma unroll
  for (int q = 0; q < RS_ROUNDS; ++q) {
    const bool ok = wb + q * 64 + lane < nt;
    const int d = ((uint32_t)kk[q] >> shift) & mask;
    unsigned long long peers = __ballot(ok);
#pragma unroll
    for (int bb = 0; bb < 8; ++bb) {
      if (bb < bits) {
        const unsigned long long bal = __ballot((d >> bb) & 1);
        peers &= ((d >> bb) & 1) ? bal : ~bal;
      }
    }
    // the lowest peer advances the digit's cursor after every lane has read it (one wave: its
    // LDS accesses take effect in program order)
    const int lp = lnext[d] + __popcll(peers & below);
    if (ok) {
      sk[lp] = kk[q];
      sr[lp] = rr[q];
      sv[lp] = vv[q];
      if ((peers & below) == 0) lnext[d] += __popcll(peers);
    }
  }
  __syncthreads();
  for (int i = t; i < nt; i += 64 * RS_WAVES) {
    const int32_t k = sk[i];
    const int d = ((uint32_t)k >> shift) & mask;
    const int64_t pos = gbase[d] + (i - lbase[d]);
    kout[pos] = k;
    rout[pos] = sr[i];
    vout[pos] = sv[i];
  }
}

// first index of each column's run in the sorted keys: lower_rp[c] for c in [0, n]
__global__ void k_run_starts(int64_t m, int64_t n, const int32_t* __restrict__ key, int64_t* __restrict__ lrp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > m) return;
  const int64_t lo = i == 0 ? 0 : (int64_t)key[i - 1] + 1;  // columns whose run starts at i
  const int64_t hi = i == m ? n : (int64_t)key[i];
  for (int64_t c = lo; c <= hi; ++c) lrp[c] = i;
}

// full row = mirrored entries (columns ascending, all < row) followed by the upper row
template <typename VT, typename TT>
__global__ void k_fill(int64_t n, const int64_t* __restrict__ up_rp, const int32_t* __restrict__ up_col,
                       const VT* __restrict__ up_val, const int64_t* __restrict__ lower_rp,
                       const int32_t* __restrict__ lrow, const TT* __restrict__ lval,
                       const int64_t* __restrict__ full_rp, int32_t* __restrict__ full_col,
                       double* __restrict__ full_v64, float* __restrict__ full_v32) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= n) return;
  const int64_t lb = lower_rp[row], nl = lower_rp[row + 1] - lb;
  const int64_t dst = full_rp[row];
  for (int64_t t = lane; t < nl; t += 64) {
    full_col[dst + t] = lrow[lb + t];
    const double v = (double)lval[lb + t];
    if (full_v64) full_v64[dst + t] = v;
    if (full_v32) full_v32[dst + t] = (float)v;
  }
  const int64_t b = up_rp[row], e = up_rp[row + 1];
  for (int64_t t = b + lane; t < e; t += 64) {
    const int64_t o = dst + nl + (t - b);
    full_col[o] = up_col[t];
    const double v = (double)up_val[t];
    if (full_v64) full_v64[o] = v;
    if (full_v32) full_v32[o] = (float)v;
  }
}

// rend[i] = the end of the entries of row i with column < c0 (columns ascending), rows i < nrows
__global__ void k_block_view(int64_t nrows, int64_t c0, const int64_t* __restrict__ rp,
                             const int32_t* __restrict__ col, int64_t* __restrict__ rend) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  int64_t lo = rp[i], hi = rp[i + 1];  // first position with col >= c0
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (col[mid] < c0) lo = mid + 1; else hi = mid;
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

// Wide blocks of float64 X (B = 16 or 32; b and ld even, X 16-byte aligned): groups of B/2
// lanes take one nonzero each and read two columns per lane (16-byte loads), so a wave holds
// 128/B nonzeros per step, twice as many as k_spmm.  Same epilogues as k_spmm (no diagonal term).
template <int B, typename VT>
__global__ __launch_bounds__(256) void k_spmm_wide(int64_t n, const int64_t* __restrict__ rp,
                                                   const int64_t* __restrict__ rend,
                                                   const int32_t* __restrict__ col,
                                                   const VT* __restrict__ val, const double* __restrict__ X,
                                                   int64_t ldx, double* __restrict__ Y, int64_t ldy, int b,
                                                   const double* __restrict__ shift, double ea, double ec,
                                                   double eb, const double* __restrict__ Zo, int64_t ldz) {
  constexpr int L = B / 2;   // lanes per nonzero
  constexpr int G = 64 / L;  // nonzeros per step
  const int lane = threadIdx.x & 63;
  const int g = lane / L;
  const int c = (lane % L) * 2;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const int64_t beg = rp[row];
  const int64_t end = rend ? rend[row] : rp[row + 1];
  double a0 = 0.0, a1 = 0.0;
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
      if (e < cnt && c < b) {  // b even: c < b covers both columns
        const f64x2 xv = *(const f64x2*)(X + (int64_t)cc * ldx + c);
        a0 = fma((double)vv, xv.x, a0);
        a1 = fma((double)vv, xv.y, a1);
      }
    }
  }
#pragma unroll
  for (int o = L; o < 64; o <<= 1) {
    a0 += __shfl_xor(a0, o);
    a1 += __shfl_xor(a1, o);
  }
  if (g == 0) {
    double acc[2] = {a0, a1};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int cq = c + q;
      if (cq < b) {
        double y = acc[q];
        if (shift) y -= shift[cq] * X[row * ldx + cq];
        if (Zo) y = ea * (y - ec * X[row * ldx + cq]) + eb * Zo[row * ldz + cq];
        Y[row * ldy + cq] = y;
      }
    }
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
  if constexpr (sizeof(XT) == 8) {
    if (b > 8 && b % 2 == 0 && !dg && ldx % 2 == 0 && ((uintptr_t)X & 15) == 0) {
      if (b <= 16)
        k_spmm_wide<16, VT><<<grid, 256, 0, s>>>(H.n, H.rp, H.rend, H.col, val, X, ldx, Y, ldy, b, shift, ea, ec,
                                                 eb, Zo, ldz);
      else
        k_spmm_wide<32, VT><<<grid, 256, 0, s>>>(H.n, H.rp, H.rend, H.col, val, X, ldx, Y, ldy, b, shift, ea, ec,
                                                 eb, Zo, ldz);
      SPPC_LAUNCH_CHECK();
      return;
    }
  }
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
// Block product over the row-block x column-panel stream (PanelH).  One workgroup per block of
// RB = 256 rows.  The block's off-diagonal entries are one contiguous stream ordered by (panel,
// row, column); each entry is a 32-bit word (column | row-in-block << 24) and a value.  The
// NW waves take tiles of the stream in turn, so the workgroup sweeps the panels in order and,
// with all workgroups of a launch starting together, the panels of X they gather from stay in
// L2 (the gathers are most of the product's time: without them it runs 1.5x faster).
//
// Inside a tile, group g of G lanes takes U = 8 consecutive entries (two vector loads of words
// and values per lane, shared by the G lanes); lane h of the group gathers columns
// [h*CPL, h*CPL + CPL) (CPL = 4) of each entry's row of X with 16-byte loads and adds the products
// to the row's LDS accumulators (native float64 LDS adds).  In one add instruction the groups
// hold entries 8 apart, which lie in different rows, so the adds rarely collide.  The words and
// values of the tile D steps ahead are requested after the gathers of the current one.  X is
// read from a copy with row stride B (16-byte aligned); the diagonal is not in the stream and is
// added in float64 at the end: dg * X64 when X64 is given, else the product in the precision of
// X.

template <typename VT> struct ValLoad;
template <> struct ValLoad<float> {
  static __device__ inline void load(const float* p, float (&v)[8]) {
    const f32x4 a = __builtin_nontemporal_load((const f32x4*)p);
    const f32x4 b = __builtin_nontemporal_load((const f32x4*)p + 1);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  }
};
template <> struct ValLoad<double> {
  static __device__ inline void load(const double* p, double (&v)[8]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const f64x2 a = __builtin_nontemporal_load((const f64x2*)p + i);
      v[2 * i] = a.x;
      v[2 * i + 1] = a.y;
    }
  }
};

struct f64x4 {
  f64x2 lo, hi;
};
template <typename XT> struct XRow;  // CPL = 4 columns of one row of X (16 or 32 bytes)
template <> struct XRow<float> {
  static constexpr int CPL = 4;
  typedef f32x4 V;
  static __device__ inline V load(const float* p) { return *(const f32x4*)p; }
  static __device__ inline float get(const V& v, int j) { return v[j]; }
};
template <> struct XRow<double> {
  static constexpr int CPL = 4;
  typedef f64x4 V;
  static __device__ inline V load(const double* p) { return V{*(const f64x2*)p, *((const f64x2*)p + 1)}; }
  static __device__ inline double get(const V& v, int j) { return j < 2 ? v.lo[j] : v.hi[j - 2]; }
};

constexpr int PANEL_RB = 256;  // rows per block: the row index is stored in 8 bits
constexpr int PANEL_U = 8;     // consecutive entries per lane group and tile
template <typename VT>
__device__ inline void panel_load(const uint32_t* __restrict__ ent, const VT* __restrict__ pval, int64_t e,
                                  int64_t s1, u32x4& wa, u32x4& wb, VT (&v)[PANEL_U]) {
  if (e < s1) {
    wa = __builtin_nontemporal_load((const u32x4*)(ent + e));
    wb = __builtin_nontemporal_load((const u32x4*)(ent + e) + 1);
    ValLoad<VT>::load(pval + e, v);
  } else {
    wa = u32x4{0u, 0u, 0u, 0u};  // column 0: the gathers stay in bounds, the adds are masked
    wb = wa;
  }
}

template <int B, int NW, int D, typename VT, typename XT>
__global__ __launch_bounds__(NW * 64) void k_spmm_panel(int64_t n, const int64_t* __restrict__ bstart,
                                                    const int32_t* __restrict__ bcount,
                                                    const uint32_t* __restrict__ ent,
                                                    const VT* __restrict__ pval, const XT* __restrict__ Xc,
                                                    double* __restrict__ Y, int64_t ldy, int b, int blk0,
                                                    const double* __restrict__ dg,
                                                    const double* __restrict__ X64, int64_t ldx64) {
  typedef XRow<XT> XR;
  constexpr int CPL = XR::CPL;
  constexpr int G = B / CPL;       // lanes per entry
  constexpr int NG = 64 / G;       // entry groups per wave
  constexpr int U = PANEL_U;
  constexpr int T = NG * U;        // entries per wave tile
  constexpr int YS = B + 1;        // LDS row stride in doubles (odd: spreads the rows over banks)
  constexpr int RB = PANEL_RB;
  constexpr int NT = NW * 64;      // threads
  __shared__ double ysh[RB * YS];
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int g = lane / G, h = lane % G;
  const int64_t blk = blk0 + (int64_t)blockIdx.x;
  const int64_t row0 = blk * RB;
  const int nr = (int)min<int64_t>(RB, n - row0);
  for (int i = t; i < RB * YS; i += NT) ysh[i] = 0.0;
  __syncthreads();
  const int64_t s0 = bstart[blk];
  const int64_t s1 = s0 + bcount[blk];
  const XT* xb = Xc + h * CPL;
  const int64_t step = (int64_t)NW * T;
  int64_t e0 = s0 + (int64_t)w * T + g * U;  // this lane group's chunk of the current tile
  // words and values of the next D tiles are in flight; chunks start at multiples of 8 and each
  // block's stream is padded to 8, so a chunk that starts before s1 is inside the allocation
  u32x4 wa[D], wb[D];
  VT v[D][U];
#pragma unroll
  for (int d = 0; d < D; ++d) panel_load(ent, pval, e0 + d * step, s1, wa[d], wb[d], v[d]);
  int64_t tb = s0 + (int64_t)w * T;
  while (tb < s1) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if (tb >= s1) break;
      const uint32_t wd[U] = {wa[d].x, wa[d].y, wa[d].z, wa[d].w, wb[d].x, wb[d].y, wb[d].z, wb[d].w};
      typename XR::V xv[U];
#pragma unroll
      for (int q = 0; q < U; ++q) xv[q] = XR::load(xb + (int64_t)(wd[q] & 0xFFFFFFu) * B);
      VT cv[U];
#pragma unroll
      for (int q = 0; q < U; ++q) cv[q] = v[d][q];
      // loads return in issue order: the tile D steps ahead is requested after the gathers
      asm volatile("" ::: "memory");
      panel_load(ent, pval, e0 + D * step, s1, wa[d], wb[d], v[d]);
#pragma unroll
      for (int q = 0; q < U; ++q) {
        if (e0 + q < s1) {
          double* yr = ysh + (int)(wd[q] >> 24) * YS + h * CPL;
#pragma unroll
          for (int j = 0; j < CPL; ++j) {
            if constexpr (sizeof(XT) == 4) {
              atomicAdd(yr + j, (double)(cv[q] * XR::get(xv[q], j)));  // float32 product, float64 sum
            } else {
              atomicAdd(yr + j, (double)cv[q] * XR::get(xv[q], j));
            }
          }
        }
      }
      tb += step;
      e0 += step;
    }
  }
  __syncthreads();
  for (int i = t; i < nr * B; i += NT) {
    const int rr = i / B, cc = i % B;
    if (cc < b) {
      const int64_t row = row0 + rr;
      double y = ysh[rr * YS + cc];
      if (X64) {
        y = fma(dg[row], X64[row * ldx64 + cc], y);
      } else if constexpr (sizeof(XT) == 4) {
        y += (double)((float)dg[row] * Xc[row * B + cc]);
      } else {
        y = fma(dg[row], Xc[row * B + cc], y);
      }
      Y[row * ldy + cc] = y;
    }
  }
}

// Xp[r][c] = X[r][c] for c < b, row stride B
template <typename XT>
__global__ void k_pad_copy(int64_t n, int b, const XT* __restrict__ X, int64_t ldx, XT* __restrict__ Xp, int B) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * B) return;
  const int64_t r = i / B;
  const int c = (int)(i % B);
  if (c < b) Xp[i] = X[r * ldx + c];
}

// Workgroups of one launch start together and sweep the panels in step.  The blocks run in
// rounds of exactly BPC workgroups per compute unit, one launch each: every CU then carries the
// same load, so the workgroups progress at the same rate and stay within a few panels of each
// other (an uneven round lets the workgroups on busier CUs fall behind, and the gathers of
// X then miss L2).
template <int B, int NW, int D, typename VT, typename XT>
void spmm_panel_rounds(const PanelH& P, const VT* val, const XT* Xc, double* Y, int64_t ldy, int b, int bpc,
                       hipStream_t s, const double* X64, int64_t ldx64) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    SPPC_HIP(hipGetDevice(&dev));
    SPPC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    cus = std::max(1, cus);
  }
  const int per = cus * bpc;
  for (int r0 = 0; r0 < P.nblocks; r0 += per) {
    const int nb = std::min(per, P.nblocks - r0);
    k_spmm_panel<B, NW, D, VT, XT><<<nb, NW * 64, 0, s>>>(P.n, P.bstart, P.bcount, P.ent, val, Xc, Y, ldy, b, r0, P.dg,
                                                       X64, ldx64);
  }
  SPPC_LAUNCH_CHECK();
}

// X is read from a copy with row stride B when the caller's X is not in that layout: the copy goes
// to `stage` (stage_bytes long) when given, else to the panel's own buffer.
template <int B, typename VT, typename XT>
void spmm_panel_b(const PanelH& P, const VT* val, const XT* X, int64_t ldx, double* Y, int64_t ldy, int b,
                  hipStream_t s, const double* X64, int64_t ldx64, void* stage, size_t stage_bytes) {
  const XT* Xc = X;
  if (ldx != B || ((uintptr_t)X & 15) != 0) {
    XT* xp = (XT*)P.xpad;
    if (stage) {
      const size_t need = (size_t)P.n * B * sizeof(XT);
      if (need > stage_bytes)
        throw Error(1, "the padded copy of X (" + std::to_string(need) + " bytes) exceeds the " +
                           std::to_string(stage_bytes) + "-byte scratch; pass X with " + std::to_string(B) +
                           " columns per row, 16-byte aligned, or use sppc_spmm");
      xp = (XT*)stage;
    }
    k_pad_copy<XT><<<(unsigned)cdiv(P.n * B, 256), 256, 0, s>>>(P.n, b, X, ldx, xp, B);
    Xc = xp;
  }
  // Two launch shapes, words and values two tiles ahead in both: one-wave workgroups, four per
  // CU, or two-wave workgroups, two (float64 X) or four (float32 X) per CU.  Measured per product
  // (ms, one-wave / two-wave):
  //   n = 7.72M, d = 300:  b = 4: 17.7 / 29.2 (float64 X), 14.0 / 21.1 (float32);
  //                        b = 8: 20.6 / 34.4, 18.5 / 25.5;  b = 16: two-wave 13-15% slower
  //   n = 1.17M, d = 200:  b = 4: 1.53 / 1.90 (float64);  b = 8: 1.86 / 1.88 (float64),
  //                        1.79 / 1.72 (float32);  b = 16: 2.79 / 2.64 (float64), 2.74 / 2.10
  // The shape follows the rows, not the width of this product: a narrow product gathers as many
  // rows of X as a wide one.  One-wave workgroups when X at width 16 would exceed the 256 MB MALL
  // (its rows then come from HBM at longer latency, and more rows in flight per CU pay), and for
  // float64 X of width <= 8.
  if ((int64_t)P.n * 16 * (int64_t)sizeof(XT) > ((int64_t)256 << 20) || (sizeof(XT) == 8 && B <= 8))
    spmm_panel_rounds<B, 1, 2, VT, XT>(P, val, Xc, Y, ldy, b, 4, s, X64, ldx64);
  else
    spmm_panel_rounds<B, 2, 2, VT, XT>(P, val, Xc, Y, ldy, b, sizeof(XT) == 4 ? 4 : 2, s, X64, ldx64);
}

template <typename VT, typename XT>
void launch_spmm_panel(const PanelH& P, const VT* val, const XT* X, int64_t ldx, double* Y, int64_t ldy, int b,
                       hipStream_t s, const double* X64 = nullptr, int64_t ldx64 = 0, void* stage = nullptr,
                       size_t stage_bytes = 0) {
  if (b <= 4)
    spmm_panel_b<4, VT, XT>(P, val, X, ldx, Y, ldy, b, s, X64, ldx64, stage, stage_bytes);
  else if (b <= 8)
    spmm_panel_b<8, VT, XT>(P, val, X, ldx, Y, ldy, b, s, X64, ldx64, stage, stage_bytes);
  else
    spmm_panel_b<16, VT, XT>(P, val, X, ldx, Y, ldy, b, s, X64, ldx64, stage, stage_bytes);
}

// first entry of row [b, e) with column >= key (columns ascending)
__device__ inline int64_t lower_col(const int32_t* __restrict__ col, int64_t b, int64_t e, int64_t key) {
  while (b < e) {
    const int64_t mid = (b + e) >> 1;
    if (col[mid] < key) b = mid + 1; else e = mid;
  }
  return b;
}

// Off-diagonal entries of each block of PANEL_RB rows, padded to a multiple of 8 (one thread
// per row, one workgroup per block); flags[0] is set when a block holds 2^31 - 8 or more.
__global__ __launch_bounds__(256) void k_panel_bcount(int64_t n, const int64_t* __restrict__ rp,
                                                      const int32_t* __restrict__ col, int32_t* __restrict__ bcount,
                                                      int32_t* __restrict__ padded, int* __restrict__ flags) {
  __shared__ int64_t sh[4];
  const int64_t row = (int64_t)blockIdx.x * PANEL_RB + threadIdx.x;
  int64_t len = 0;
  if (row < n) {
    const int64_t b = rp[row], e = rp[row + 1];
    const int64_t d = lower_col(col, b, e, row);
    len = (e - b) - ((d < e && col[d] == row) ? 1 : 0);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) len += __shfl_xor(len, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = len;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t tot = sh[0] + sh[1] + sh[2] + sh[3];
    if (tot >= ((int64_t)1 << 31) - 8) atomicOr(&flags[0], 1);
    bcount[blockIdx.x] = (int32_t)min<int64_t>(tot, ((int64_t)1 << 31) - 8);
    padded[blockIdx.x] = (bcount[blockIdx.x] + 7) & ~7;
  }
}

// Writes the stream of one block (one workgroup of 16 waves per block; a wave takes every 16th
// row, 64 consecutive entries at a time), in chunks of PANEL_PC panels: (1) the off-diagonal
// entries of each (panel, row) of the chunk are counted in LDS, (2) a block-wide exclusive scan
// in (panel, row) order gives each run's offset, (3) every entry goes to its run's offset plus
// its index in the run (the run start comes from a ballot over the window, carried across
// windows).  Each row keeps a cursor in LDS, so no row is searched.  The diagonal goes to dg
// instead (when dg is given).  A wave takes its rows one after the other, and a row holds few
// entries in one chunk (about 10 at n = 7.7M), so the kernel waits on one load round trip per row
// and chunk: wide chunks (128 panels, 128 KB of LDS counters) keep the number of chunks small.
constexpr int PANEL_PC = 128;
constexpr int PANEL_FT = 1024;  // threads of the fill kernel

// rows whose first window a wave requests together (n = 7.72M, float32 values: 45.7 ms with 1, 38.2
// with 4, 34.1 with 8; 256 rows per block, 16 per wave); 4 with float64 values, which keep 8 windows
// in flight only by spilling registers
template <typename VT>
constexpr int panel_ru() { return sizeof(VT) == 4 ? 8 : 4; }

template <typename VT>
__global__ __launch_bounds__(PANEL_FT) void k_panel_fill(int64_t n, const int64_t* __restrict__ rp,
                                                         const int32_t* __restrict__ col,
                                                         const VT* __restrict__ val, int PW, int P,
                                                         const int64_t* __restrict__ bstart,
                                                         uint32_t* __restrict__ ent, VT* __restrict__ pval,
                                                         double* __restrict__ dg) {
  constexpr int NWV = PANEL_FT / 64;
  constexpr int PER = PANEL_PC * PANEL_RB / PANEL_FT;  // counters per thread in the scan
  constexpr int RU = panel_ru<VT>();
  __shared__ int cnt[PANEL_PC * PANEL_RB];
  __shared__ int64_t cur[PANEL_RB];   // next entry of each row
  __shared__ int64_t rend[PANEL_RB];  // end of each row
  __shared__ int64_t dpos[PANEL_RB];  // position of the row's diagonal entry (or -1)
  __shared__ int sh[NWV];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * PANEL_RB;
  const int nr = (int)min<int64_t>(PANEL_RB, n - row0);
  for (int r = threadIdx.x; r < PANEL_RB; r += PANEL_FT) {
    cur[r] = r < nr ? rp[row0 + r] : 0;
    rend[r] = r < nr ? rp[row0 + r + 1] : 0;
    if (r < nr) {
      const int64_t b = rp[row0 + r], e = rp[row0 + r + 1];
      const int64_t d = lower_col(col, b, e, row0 + r);
      dpos[r] = (d < e && col[d] == row0 + r) ? d : -1;
    }
  }
  int64_t base = bstart[blockIdx.x];
  // A wave takes its rows RU at a time: the first 64-entry window of each of the RU rows is
  // requested before any is used (a row holds a few dozen entries of a chunk, so one window
  // usually covers it), and the rare further windows of a row follow one by one.
  for (int p0 = 0; p0 < P; p0 += PANEL_PC) {
    const int64_t c1 = min<int64_t>((int64_t)(p0 + PANEL_PC) * PW, n);
    for (int i = threadIdx.x; i < PANEL_PC * PANEL_RB; i += PANEL_FT) cnt[i] = 0;
    __syncthreads();
    // (1) counts; the chunk of a row is [cur, first entry with column >= c1)
    for (int rb = w; rb < nr; rb += NWV * RU) {
      int64_t ts[RU], es[RU];
      int cs[RU];
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int r = rb + u * NWV;
        ts[u] = r < nr ? cur[r] : 0;
        es[u] = r < nr ? rend[r] : 0;
      }
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int64_t t = ts[u] + lane;
        cs[u] = t < es[u] ? col[t] : (int)n;
      }
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int r = rb + u * NWV;
        if (r >= nr) break;  // uniform over the wave
        const int64_t row = row0 + r, e = es[u];
        int64_t t0 = ts[u];
        int c = cs[u];
        while (true) {
          const bool in = c < c1;
          if (in && c != row) atomicAdd(&cnt[(c / PW - p0) * PANEL_RB + r], 1);
          if (__ballot(!in)) break;  // columns ascend: the chunk ends in this window
          t0 += 64;
          if (t0 >= e) break;
          const int64_t t = t0 + lane;
          c = t < e ? col[t] : (int)n;
        }
      }
    }
    __syncthreads();
    // (2) exclusive scan in (panel, row) order: thread i owns PER consecutive counters
    int* mine = cnt + threadIdx.x * PER;
    int loc = 0;
    for (int q = 0; q < PER; ++q) loc += mine[q];
    int inc = loc;
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(inc, o);
      if (lane >= o) inc += u;
    }
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    int before = 0, tot = 0;
    for (int i = 0; i < NWV; ++i) {
      if (i < w) before += sh[i];
      tot += sh[i];
    }
    int run = before + inc - loc;
    for (int q = 0; q < PER; ++q) {
      const int v = mine[q];
      mine[q] = run;
      run += v;
    }
    __syncthreads();
    // (3) placement
    for (int rb = w; rb < nr; rb += NWV * RU) {
      int64_t ts[RU], es[RU];
      int cs[RU];
      VT vs[RU];
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int r = rb + u * NWV;
        ts[u] = r < nr ? cur[r] : 0;
        es[u] = r < nr ? rend[r] : 0;
      }
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int64_t t = ts[u] + lane;
        const bool ok = t < es[u];
        cs[u] = ok ? col[t] : (int)n;
        vs[u] = ok ? val[t] : VT(0);
      }
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int r = rb + u * NWV;
        if (r >= nr) break;  // uniform over the wave
        const int64_t row = row0 + r, e = es[u];
        int64_t t0 = ts[u];
        if (t0 >= e) continue;  // the row is done (cur[r] == e already)
        const int64_t dp = dpos[r];
        int64_t rs = t0;  // start of the run that continues into the next window
        int pr = -1;      // its panel
        int c = cs[u];
        VT vv = vs[u];
        while (true) {
          const int64_t t = t0 + lane;
          const bool in = c < c1;
          const int p = in ? c / PW : 0x7fffffff;
          const int pprev = __shfl_up(p, 1);
          const bool start = in && (lane == 0 ? p != pr : p != pprev);
          const unsigned long long m = __ballot(start);
          const unsigned long long mm = m & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
          const int64_t st = mm ? t0 + (63 - __builtin_clzll(mm)) : rs;
          if (in) {
            if (c == row) {
              if (dg) dg[row] = (double)vv;
            } else {
              const int64_t idx = t - st - ((dp >= st && dp < t) ? 1 : 0);
              const int64_t dst = base + cnt[(p - p0) * PANEL_RB + r] + idx;
              ent[dst] = (uint32_t)c | ((uint32_t)r << 24);
              pval[dst] = vv;
            }
          }
          const unsigned long long nin = __ballot(in);
          if (nin != ~0ull) {  // the chunk ends in this window: next chunk starts at the first lane out
            if (lane == 0) cur[r] = t0 + __builtin_popcountll(nin);
            break;
          }
          rs = __shfl(st, 63);
          pr = __shfl(p, 63);
          t0 += 64;
          if (t0 >= e) {
            if (lane == 0) cur[r] = e;
            break;
          }
          const int64_t t2 = t0 + lane;
          const bool ok = t2 < e;
          c = ok ? col[t2] : (int)n;
          vv = ok ? val[t2] : VT(0);
        }
      }
    }
    __syncthreads();  // cnt and cur are rewritten by the next chunk
    base += tot;
  }
}

// Zero the padding slots of each block's stream, [bstart + bcount, bstart[blk + 1]), and with an
// empty stream the whole cap.
__global__ void k_panel_pad(int nb, const int64_t* __restrict__ bstart, const int32_t* __restrict__ bcount,
                            int64_t cap, uint32_t* __restrict__ ent, double* __restrict__ v64,
                            float* __restrict__ v32) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int64_t e1 = b + 1 < nb ? bstart[b + 1] : max<int64_t>(bstart[nb], cap);
  for (int64_t e = bstart[b] + bcount[b]; e < e1; ++e) {
    ent[e] = 0u;
    if (v64) v64[e] = 0.0;
    if (v32) v32[e] = 0.0f;
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

template <typename VT, typename TT>
void mirror_and_fill(int64_t n, int64_t m, const int64_t* up_rp, const int32_t* up_col, const VT* up_val,
                     const int64_t* su_off, DevCSR& out, int64_t* lower_rp, int32_t* key[2], int32_t* rowi[2],
                     TT* v[2], int32_t* cnt, int64_t* off, int64_t* bsum, hipStream_t s) {
  const int64_t grid_w = cdiv(n, 4);
  k_extract_upper<VT, TT><<<grid_w, 256, 0, s>>>(n, up_rp, up_col, up_val, su_off, key[0], rowi[0], v[0]);
  int cur = 0;
  if (m > 0) {
    int kb = 1;  // bits of the largest column index
    while (kb < 31 && ((int64_t)1 << kb) < n) ++kb;
    const int passes = (kb + 7) / 8;
    const int64_t ntile = cdiv(m, RS_TILE);
    for (int p = 0, shift = 0; p < passes; ++p) {
      const int bits = std::min(8, (kb - shift + (passes - p) - 1) / (passes - p));
      k_rs_hist<<<ntile, 256, 0, s>>>(m, key[cur], shift, (1 << bits) - 1, ntile, cnt);
      scan_exclusive_impl(ntile << bits, cnt, off, bsum, s);
      k_rs_scatter<TT><<<ntile, 64 * RS_WAVES, 0, s>>>(m, key[cur], rowi[cur], v[cur], key[cur ^ 1], rowi[cur ^ 1],
                                                       v[cur ^ 1],
                                            shift, bits, ntile, cnt, off);
      cur ^= 1;
      shift += bits;
    }
  }
  k_run_starts<<<cdiv(m + 1, 256), 256, 0, s>>>(m, n, key[cur], lower_rp);
  k_full_rowptr<<<cdiv(n + 1, 256), 256, 0, s>>>(n, lower_rp, up_rp, out.rp);
  k_fill<VT, TT><<<grid_w, 256, 0, s>>>(n, up_rp, up_col, up_val, lower_rp, rowi[cur], v[cur], out.rp, out.col,
                                        out.val64, out.val32);
  SPPC_LAUNCH_CHECK();
}

void build_full_csr(int64_t n, int64_t nnz_up, const int64_t* up_rp, const int32_t* up_col,
                    const void* up_val, int val_is_f32, DevCSR& out, int* d_flags, bool want64,
                    bool want32, bool& exact32, hipStream_t s) {
  int32_t *su_cnt = nullptr, *cnt = nullptr;
  int64_t *su_off = nullptr, *lower_rp = nullptr, *bsum = nullptr, *off = nullptr;
  int32_t* key[2] = {nullptr, nullptr};
  int32_t* rowi[2] = {nullptr, nullptr};
  void* v[2] = {nullptr, nullptr};
  auto cleanup = [&]() {
    dev_free(su_cnt); dev_free(cnt); dev_free(su_off); dev_free(lower_rp); dev_free(bsum); dev_free(off);
    for (int i = 0; i < 2; ++i) { dev_free(key[i]); dev_free(rowi[i]); dev_free(v[i]); }
  };
  try {
    SPPC_HIP(dev_malloc_tmp(&su_cnt, sizeof(int32_t) * (n + 1)));
    SPPC_HIP(dev_malloc_tmp(&su_off, sizeof(int64_t) * (n + 1)));
    SPPC_HIP(dev_malloc_tmp(&lower_rp, sizeof(int64_t) * (n + 1)));
    SPPC_HIP(hipMemsetAsync(d_flags, 0, sizeof(int) * 4, s));
    const int64_t grid_w = cdiv(n, 4);
    if (val_is_f32)
      k_validate_count<float><<<grid_w, 256, 0, s>>>(n, up_rp, up_col, (const float*)up_val, su_cnt, d_flags);
    else
      k_validate_count<double><<<grid_w, 256, 0, s>>>(n, up_rp, up_col, (const double*)up_val, su_cnt, d_flags);
    SPPC_LAUNCH_CHECK();
    int h_flags[4];
    SPPC_HIP(hipMemcpyAsync(h_flags, d_flags, sizeof(h_flags), hipMemcpyDeviceToHost, s));
    SPPC_HIP(hipStreamSynchronize(s));
    if (h_flags[0]) throw Error(1, "H: upper CSR expected (columns >= row, < n, strictly ascending)");
    if (h_flags[2]) throw Error(7, "H: NaN or Inf among the values");
    exact32 = val_is_f32 || !h_flags[1];
    SPPC_HIP(dev_malloc_tmp(&bsum, sizeof(int64_t) * (cdiv(n, SCAN_BLOCK) + 1)));
    scan_exclusive_impl(n, su_cnt, su_off, bsum, s);
    int64_t m = 0;  // strict-upper entries = mirrored entries
    SPPC_HIP(hipMemcpyAsync(&m, su_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPPC_HIP(hipStreamSynchronize(s));
    const int64_t nnz = nnz_up + m;
    out.n = n;
    out.nnz = nnz;
    SPPC_HIP(dev_malloc(&out.rp, sizeof(int64_t) * (n + 1)));
    SPPC_HIP(dev_malloc(&out.col, sizeof(int32_t) * (nnz > 0 ? nnz : 1)));
    if (want64) SPPC_HIP(dev_malloc(&out.val64, sizeof(double) * (nnz > 0 ? nnz : 1)));
    if (want32) SPPC_HIP(dev_malloc(&out.val32, sizeof(float) * (nnz > 0 ? nnz : 1)));
    // sort buffers (twice: the passes alternate between them) and the digit counts
    const int64_t ms = m > 0 ? m : 1;
    const size_t vb = want64 ? sizeof(double) : sizeof(float);
    for (int i = 0; i < 2; ++i) {
      SPPC_HIP(dev_malloc_tmp(&key[i], sizeof(int32_t) * ms));
      SPPC_HIP(dev_malloc_tmp(&rowi[i], sizeof(int32_t) * ms));
      SPPC_HIP(dev_alloc_tmp(&v[i], vb * ms));
    }
    const int64_t ncnt = (cdiv(ms, RS_TILE) << 8) + 1;
    SPPC_HIP(dev_malloc_tmp(&cnt, sizeof(int32_t) * ncnt));
    SPPC_HIP(dev_malloc_tmp(&off, sizeof(int64_t) * (ncnt + 1)));
    dev_free(bsum);
    bsum = nullptr;
    SPPC_HIP(dev_malloc_tmp(&bsum, sizeof(int64_t) * (cdiv(std::max(ncnt, n + 1), SCAN_BLOCK) + 1)));
    if (want64) {
      double* vv[2] = {(double*)v[0], (double*)v[1]};
      if (val_is_f32)
        mirror_and_fill<float, double>(n, m, up_rp, up_col, (const float*)up_val, su_off, out, lower_rp, key, rowi,
                                       vv, cnt, off, bsum, s);
      else
        mirror_and_fill<double, double>(n, m, up_rp, up_col, (const double*)up_val, su_off, out, lower_rp, key,
                                        rowi, vv, cnt, off, bsum, s);
    } else {
      float* vv[2] = {(float*)v[0], (float*)v[1]};
      if (val_is_f32)
        mirror_and_fill<float, float>(n, m, up_rp, up_col, (const float*)up_val, su_off, out, lower_rp, key, rowi,
                                      vv, cnt, off, bsum, s);
      else
        mirror_and_fill<double, float>(n, m, up_rp, up_col, (const double*)up_val, su_off, out, lower_rp, key,
                                       rowi, vv, cnt, off, bsum, s);
    }
    SPPC_HIP(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipStreamSynchronize(s);
    cleanup();
    throw;
  }
  cleanup();
}

void build_block_view(const DevCSR& full, int64_t n0, int64_t* rend, hipStream_t s) {
  row_ends_below(full, n0, n0, rend, s);
}

void row_ends_below(const DevCSR& full, int64_t nrows, int64_t c0, int64_t* rend, hipStream_t s) {
  if (nrows <= 0) return;
  k_block_view<<<cdiv(nrows, 256), 256, 0, s>>>(nrows, c0, full.rp, full.col, rend);
  SPPC_LAUNCH_CHECK();
}

void compact_view(const DevCSR& V, DevCSR& out, hipStream_t s) {
  const int64_t n0 = V.n;
  if (!V.rend) throw Error(1, "compact_view: not a block view");
  int32_t* cnt = nullptr;
  int64_t* bsum = nullptr;
  auto cleanup = [&]() { dev_free(cnt); dev_free(bsum); };
  try {
    out = DevCSR{};
    out.n = n0;
    SPPC_HIP(dev_malloc_tmp(&cnt, sizeof(int32_t) * (n0 + 1)));
    SPPC_HIP(dev_malloc_tmp(&bsum, sizeof(int64_t) * (cdiv(n0 + 1, SCAN_BLOCK) + 1)));
    SPPC_HIP(dev_malloc(&out.rp, sizeof(int64_t) * (n0 + 1)));
    k_view_count<<<cdiv(n0 > 0 ? n0 : 1, 256), 256, 0, s>>>(n0, V.rp, V.rend, cnt);
    SPPC_LAUNCH_CHECK();
    scan_exclusive_impl(n0, cnt, out.rp, bsum, s);
    int64_t nnz = 0;
    SPPC_HIP(hipMemcpyAsync(&nnz, out.rp + n0, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPPC_HIP(hipStreamSynchronize(s));
    out.nnz = nnz;
    SPPC_HIP(dev_malloc(&out.col, sizeof(int32_t) * (nnz > 0 ? nnz : 1)));
    if (V.val64) SPPC_HIP(dev_malloc(&out.val64, sizeof(double) * (nnz > 0 ? nnz : 1)));
    if (V.val32) SPPC_HIP(dev_malloc(&out.val32, sizeof(float) * (nnz > 0 ? nnz : 1)));
    k_view_fill<<<cdiv(n0 > 0 ? n0 : 1, 4), 256, 0, s>>>(n0, V.rp, V.col, V.val64, V.val32, out.rp, out.col,
                                                          out.val64, out.val32);
    SPPC_LAUNCH_CHECK();
    SPPC_HIP(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipStreamSynchronize(s);
    cleanup();
    (void)dev_free(out.rp); (void)dev_free(out.col); (void)dev_free(out.val64); (void)dev_free(out.val32);
    out = DevCSR{};
    throw;
  }
  cleanup();
}

void extract_diag(const DevCSR& H, double* diag, hipStream_t s) {
  k_diag<<<cdiv(H.n, 256), 256, 0, s>>>(H.n, H.rp, H.col, H.val64, H.val32, diag);
  SPPC_LAUNCH_CHECK();
}

void build_panel(const DevCSR& H, int PW, PanelH& out, hipStream_t s) {
  const int64_t n = H.n;
  if (PW < 1 || PW > 65536) throw Error(1, "panel: bad width");
  if (n < 1 || n >= ((int64_t)1 << 24)) throw Error(1, "panel: n must be in [1, 2^24)");
  out.n = n;
  out.RB = PANEL_RB;
  out.PW = PW;
  out.P = (int)cdiv(n, PW);
  out.nblocks = (int)cdiv(n, PANEL_RB);
  int32_t* padded = nullptr;
  int64_t* bsum = nullptr;
  int* flags = nullptr;
  auto cleanup = [&]() { (void)dev_free(padded); (void)dev_free(bsum); (void)dev_free(flags); };
  try {
    const int nb = out.nblocks;
    SPPC_HIP(dev_malloc_tmp(&padded, sizeof(int32_t) * nb));
    SPPC_HIP(dev_malloc_tmp(&bsum, sizeof(int64_t) * (cdiv(nb, SCAN_BLOCK) + 1)));
    SPPC_HIP(dev_malloc(&out.bcount, sizeof(int32_t) * nb));
    SPPC_HIP(dev_malloc(&out.bstart, sizeof(int64_t) * (nb + 1)));
    SPPC_HIP(dev_malloc(&out.dg, sizeof(double) * n));
    SPPC_HIP(dev_malloc(&out.xpad, sizeof(double) * 16 * n));
    SPPC_HIP(hipMemsetAsync(out.dg, 0, sizeof(double) * n, s));
    SPPC_HIP(dev_malloc_tmp(&flags, sizeof(int)));
    SPPC_HIP(hipMemsetAsync(flags, 0, sizeof(int), s));
    k_panel_bcount<<<nb, 256, 0, s>>>(n, H.rp, H.col, out.bcount, padded, flags);
    scan_exclusive_impl(nb, padded, out.bstart, bsum, s);
    int64_t total = 0;
    int flag = 0;
    SPPC_HIP(hipMemcpyAsync(&total, out.bstart + nb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPPC_HIP(hipMemcpyAsync(&flag, flags, sizeof(int), hipMemcpyDeviceToHost, s));
    SPPC_HIP(hipStreamSynchronize(s));
    if (flag) throw Error(1, "panel: a block of rows holds 2^31 entries or more");
    const int64_t cap = std::max<int64_t>(total, 8);
    SPPC_HIP(dev_malloc(&out.ent, sizeof(uint32_t) * cap));
    if (H.val64) SPPC_HIP(dev_malloc(&out.val64, sizeof(double) * cap));
    if (H.val32) SPPC_HIP(dev_malloc(&out.val32, sizeof(float) * cap));
    // the fill writes every entry; the up to 7 padding slots of each block get column 0, row 0 and
    // value 0 (a cap of 8 beyond an empty stream included)
    k_panel_pad<<<cdiv(nb, 256), 256, 0, s>>>(nb, out.bstart, out.bcount, cap, out.ent, out.val64, out.val32);
    if (H.val64)
      k_panel_fill<double><<<nb, PANEL_FT, 0, s>>>(n, H.rp, H.col, H.val64, PW, out.P, out.bstart, out.ent,
                                                    out.val64, out.dg);
    if (H.val32)
      k_panel_fill<float><<<nb, PANEL_FT, 0, s>>>(n, H.rp, H.col, H.val32, PW, out.P, out.bstart, out.ent,
                                                   out.val32, H.val64 ? nullptr : out.dg);
    SPPC_LAUNCH_CHECK();
    SPPC_HIP(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipStreamSynchronize(s);
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
  (void)dev_free(p.bstart);
  (void)dev_free(p.bcount);
  (void)dev_free(p.ent);
  (void)dev_free(p.val32);
  (void)dev_free(p.val64);
  (void)dev_free(p.dg);
  (void)dev_free(p.xpad);
  p = PanelH{};
}

void spmm_f64(const DevCSR& H, const double* X, int64_t ldx, double* Y, int64_t ldy, int b,
              const double* shift, hipStream_t s, void* stage, size_t stage_bytes) {
  if (H.panel && !shift && b >= 1 && b <= 16 && H.n > 0) {
    if (H.val64)
      launch_spmm_panel<double, double>(*H.panel, H.panel->val64, X, ldx, Y, ldy, b, s, nullptr, 0, stage,
                                        stage_bytes);
    else
      launch_spmm_panel<float, double>(*H.panel, H.panel->val32, X, ldx, Y, ldy, b, s, nullptr, 0, stage,
                                       stage_bytes);
    return;
  }
  if (H.val64)
    launch_spmm<double, double>(H, H.val64, X, ldx, Y, ldy, b, shift, s);
  else
    launch_spmm<float, double>(H, H.val32, X, ldx, Y, ldy, b, shift, s);
}

void spmm_f32(const DevCSR& H, const float* X, int64_t ldx, double* Y, int64_t ldy, int b,
              const double* shift, hipStream_t s, const double* diag, const double* X64, int64_t ldx64,
              void* stage, size_t stage_bytes) {
  if (!H.val32) throw Error(1, "spmm_f32: no float32 values");
  if (diag && !X64) throw Error(1, "spmm_f32: the float64 diagonal term needs float64 X");
  if (H.panel && !shift && b >= 1 && b <= 16 && H.n > 0) {
    // the panel stream holds the diagonal apart: diag * X64 in float64 when given, else the
    // float32 product as for the other entries
    launch_spmm_panel<float, float>(*H.panel, H.panel->val32, X, ldx, Y, ldy, b, s, diag ? X64 : nullptr,
                                    ldx64, stage, stage_bytes);
    return;
  }
  launch_spmm<float, float>(H, H.val32, X, ldx, Y, ldy, b, shift, s, 0.0, 0.0, 0.0, nullptr, 0, diag, X64, ldx64);
}

// ---------------------------------------------------------------- workspace sizes
// Bytes the builders above take from a workspace (each array rounded up to 256 bytes), from the same
// expressions as their allocations.  nnz_up bounds the strict-upper entries.
BuildBytes full_csr_bytes(int64_t n, int64_t nnz_up, bool want64, bool want32) {
  BuildBytes b;
  const int64_t m = std::max<int64_t>(nnz_up, 1);
  const int64_t nnz = std::max<int64_t>(nnz_up + m, 1);
  b.persist = ws_bytes(8 * (n + 1)) + ws_bytes(4 * nnz) + (want64 ? ws_bytes(8 * nnz) : 0) +
              (want32 ? ws_bytes(4 * nnz) : 0);
  const int64_t vb = want64 ? 8 : 4;
  const int64_t ncnt = (cdiv(m, RS_TILE) << 8) + 1;
  b.temp = ws_bytes(4 * (n + 1)) + 2 * ws_bytes(8 * (n + 1)) + ws_bytes(8 * (cdiv(n, SCAN_BLOCK) + 1)) +
           2 * (2 * ws_bytes(4 * m) + ws_bytes(vb * m)) + ws_bytes(4 * ncnt) + ws_bytes(8 * (ncnt + 1)) +
           ws_bytes(8 * (cdiv(std::max(ncnt, n + 1), SCAN_BLOCK) + 1));
  return b;
}

BuildBytes panel_bytes(int64_t n, int64_t nnz_full, bool v64, bool v32) {
  BuildBytes b;
  const int64_t nb = cdiv(n, PANEL_RB);
  const int64_t cap = std::max<int64_t>(nnz_full + 7 * nb, 8);
  b.persist = ws_bytes(4 * nb) + ws_bytes(8 * (nb + 1)) + ws_bytes(8 * n) + ws_bytes(8 * 16 * n) + ws_bytes(4 * cap) +
              (v64 ? ws_bytes(8 * cap) : 0) + (v32 ? ws_bytes(4 * cap) : 0);
  b.temp = ws_bytes(4 * nb) + ws_bytes(8 * (cdiv(nb, SCAN_BLOCK) + 1)) + ws_bytes(4);
  return b;
}

BuildBytes view_bytes(int64_t n0, int64_t nnz0, bool v64, bool v32) {
  BuildBytes b;
  const int64_t z = std::max<int64_t>(nnz0, 1);
  b.persist = ws_bytes(8 * (n0 + 1)) + ws_bytes(4 * z) + (v64 ? ws_bytes(8 * z) : 0) + (v32 ? ws_bytes(4 * z) : 0);
  b.temp = ws_bytes(4 * (n0 + 1)) + ws_bytes(8 * (cdiv(n0 + 1, SCAN_BLOCK) + 1));
  return b;
}

// ---------------------------------------------------------------- allocation-free staging
// Device scratch of sppc_spmm_noalloc: the padded copy of X that the panel kernels read when the
// caller's X is not already in that layout.  Each device holds its own copy of this array for the
// life of the process; host code uses only the address found by hipGetSymbolAddress (the name
// itself is a host-side stand-in).  Calls that overlap on one device share it and race.
namespace {
constexpr size_t kNoallocScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Looks up (once per device, with that device current) the device address of the scratch array.
void* noalloc_scratch(size_t* bytes) {
  int dev = 0;
  SPPC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error(1, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    SPPC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(2, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  if (bytes) *bytes = kNoallocScratchBytes;
  return g_scratch_ptr[dev];
}

}  // namespace sppc
