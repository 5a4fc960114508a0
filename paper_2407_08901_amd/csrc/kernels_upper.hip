// kernels_upper.hip - the block product Y = H X read from the stored upper triangle alone.
//
// The paper's cost unit is the product with H (Sec. IV.C); H is symmetric and the caller keeps
// its upper triangle only.  The solver's own products read a mirrored full-storage copy (both
// triangles, built once at setup), which streams every off-diagonal entry twice per product but
// writes each output row once.  This kernel is the other trade: it streams the upper triangle
// once (half the matrix bytes, no mirror in memory) and pays for the lower triangle with a
// scatter: every stored entry (r, j > r, v) adds v X[r] to row j of Y by a float64 atomic add.
//
// One wave per row r, lane c of a group of B lanes owns column c of the block.  A batch of 64
// entries is loaded coalesced (one per lane) and broadcast by shuffles, 64/B entries per step:
// the gather of X[j] feeds row r's sum in a register, the scatter of v X[r] goes to Y[j].  Row r's
// sum is itself added atomically (other rows' scatters reach Y[r] concurrently), so Y is zeroed
// first and the order of the float64 sums depends on scheduling (not bit-reproducible).
// float32 X: values rounded to float32, float32 products, float64 sums.
#include "common.h"

namespace sppc {

namespace {

// Native float64 add at the memory side (global_atomic_add_f64): Y is ordinary device memory.
__device__ __forceinline__ void add_f64(double* p, double v) { unsafeAtomicAdd(p, v); }

template <int B, typename VT, typename XT>
__global__ __launch_bounds__(256) void k_spmm_upper(int64_t n, const int64_t* __restrict__ rp,
                                                    const int32_t* __restrict__ col,
                                                    const VT* __restrict__ val, const XT* __restrict__ X,
                                                    int64_t ldx, double* __restrict__ Y, int64_t ldy, int b) {
  constexpr int G = 64 / B;
  const int lane = threadIdx.x & 63;
  const int g = lane / B;
  const int c = lane % B;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const int64_t beg = rp[row], end = rp[row + 1];
  const bool colok = c < b;
  const XT xr = colok ? X[row * ldx + c] : XT(0);
  double acc = 0.0;
  for (int64_t base = beg; base < end; base += 64) {
    const int cnt = (int)min<int64_t>(64, end - base);
    int32_t mc = 0;
    VT mv = VT(0);
    if (lane < cnt) {
      mc = __builtin_nontemporal_load(&col[base + lane]);
      mv = __builtin_nontemporal_load(&val[base + lane]);
    }
    for (int s0 = 0; s0 < cnt; s0 += G) {
      const int e = s0 + g;
      const int32_t j = __shfl(mc, e);
      const VT v = __shfl(mv, e);
      if (e < cnt && colok) {
        const XT xj = X[(int64_t)j * ldx + c];
        if constexpr (sizeof(XT) == 4) {
          const float vf = (float)v;
          acc += (double)(vf * xj);
          if (j != row) add_f64(&Y[(int64_t)j * ldy + c], (double)(vf * xr));
        } else {
          acc = fma((double)v, xj, acc);
          if (j != row) add_f64(&Y[(int64_t)j * ldy + c], (double)v * xr);
        }
      }
    }
  }
#pragma unroll
  for (int o = B; o < 64; o <<= 1) acc += __shfl_xor(acc, o);
  if (g == 0 && colok) add_f64(&Y[row * ldy + c], acc);
}

template <typename VT, typename XT>
void launch_upper(int64_t n, const int64_t* rp, const int32_t* col, const VT* val, const XT* X, int64_t ldx,
                  double* Y, int64_t ldy, int b, hipStream_t s) {
  fill_block_zero(n, b, Y, ldy, s);
  const int64_t grid = cdiv(n, 4);
  switch (b <= 4 ? 4 : b <= 8 ? 8 : b <= 16 ? 16 : 32) {
    case 4: k_spmm_upper<4, VT, XT><<<grid, 256, 0, s>>>(n, rp, col, val, X, ldx, Y, ldy, b); break;
    case 8: k_spmm_upper<8, VT, XT><<<grid, 256, 0, s>>>(n, rp, col, val, X, ldx, Y, ldy, b); break;
    case 16: k_spmm_upper<16, VT, XT><<<grid, 256, 0, s>>>(n, rp, col, val, X, ldx, Y, ldy, b); break;
    default: k_spmm_upper<32, VT, XT><<<grid, 256, 0, s>>>(n, rp, col, val, X, ldx, Y, ldy, b); break;
  }
  SPPC_LAUNCH_CHECK();
}

}  // namespace

void spmm_upper(const UpperCSR& U, const void* X, bool xf32, int64_t ldx, double* Y, int64_t ldy, int b,
                hipStream_t s) {
  if (b < 1 || b > 32) throw Error(1, "spmm: block width must be 1..32");
  if (U.n == 0) return;
  if (U.val32) {
    if (xf32) launch_upper<float, float>(U.n, U.rp, U.col, U.val32, (const float*)X, ldx, Y, ldy, b, s);
    else launch_upper<float, double>(U.n, U.rp, U.col, U.val32, (const double*)X, ldx, Y, ldy, b, s);
  } else {
    if (xf32) launch_upper<double, float>(U.n, U.rp, U.col, U.val64, (const float*)X, ldx, Y, ldy, b, s);
    else launch_upper<double, double>(U.n, U.rp, U.col, U.val64, (const double*)X, ldx, Y, ldy, b, s);
  }
}

}  // namespace sppc
