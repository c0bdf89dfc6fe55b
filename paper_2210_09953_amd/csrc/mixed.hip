// mixed.hip -- Rademacher sketch P = Theta X on FP16 matrix cores for FP32 X.
//
// Section 5 asks for the sketch to be computed more accurately than the
// working precision; here X is FP32 and the products run at FP16 rate while
// keeping ~22 bits of X:
//   * Theta entries are +-1, exact in FP16 (the 1/sqrt(k) goes on P).
//   * Each FP32 x is scaled by a power of two 2^s chosen per column and
//     split into x 2^s ~ hi + lo with hi = fp16(x 2^s), lo = fp16(x 2^s - hi)
//     (the difference is exact in FP32), so |x - (hi + lo) 2^-s| <=
//     ~2^-22 |max of the column|.  s keeps the column's running maximum in
//     [2^14, 2^15) (no FP16 overflow) and only decreases, so values rescale
//     rarely; P's error budget is relative to the column norm anyway.
//   * v_mfma_f32_16x16x32_f16 accumulates Theta hi + Theta lo in FP32; the
//     FP32 accumulators are flushed into FP64 totals every 1024 rows and
//     whenever a column's scale changes, then the per-split FP64 partials are
//     reduced in a fixed order (sketch_reduce_kernel).
// A workgroup owns 256 rows of Theta and 64 columns of X (8 waves x 32
// Theta rows), so every converted X element feeds 256 Theta rows.  Stages
// of 128 rows of X: global loads for the next stage are issued before the
// matrix-core loop of the current one.  Theta comes from the Philox bits
// directly: the A operand (16 Theta rows x 32 X rows) is packed from bits
// with integer ops, 0x3C00 | sign << 15 per FP16 entry.
#include "common.h"
#include "theta.h"
#include "kernels.h"

namespace rcq {

constexpr int kMxRows = 128;    // rows of X per stage
constexpr int kMxTheta = 256;   // Theta rows per workgroup
constexpr int kMxCols = 64;     // columns of X per workgroup
constexpr int kMxLd = kMxRows + 8;  // LDS row stride (halves) of the transposed X tile
constexpr int kMxFlushStages = 8;

typedef uint32_t u4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float pow2f(int s) {
  return __int_as_float((s + 127) << 23);
}

template <int NB>  // column tiles of 16 in this workgroup's column slice
__global__ __launch_bounds__(512, 1) void sketch_mixed_kernel(
    const float* __restrict__ X, int64_t m, int n, int64_t ldx, uint64_t seed, int ktiles,
    int nh, int64_t rows_per_split, int kpad, int npad, double* __restrict__ part) {
  constexpr int NPW = NB * 16;
  __shared__ __align__(16) _Float16 xhi[kMxCols][kMxLd];
  __shared__ __align__(16) _Float16 xlo[kMxCols][kMxLd];
  __shared__ __align__(16) uint32_t zb[2][4][kMxRows];  // [philox block][word][x row]
  __shared__ int rexp[kMxCols];       // running exponent of the column maximum
  __shared__ int flush_flag;

  const int bid = blockIdx.x;
  const int xcd = bid & 7, slot = bid >> 3;
  const int tps = ktiles * nh;
  const int jt = slot % tps;
  const int t = jt % ktiles, h = jt / ktiles;
  const int s = (slot / tps) * 8 + xcd;

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  const int c0 = h * kMxCols;              // first column of the slice
  const int theta0 = t * kMxTheta;         // first Theta row of the workgroup
  const int64_t r_begin = static_cast<int64_t>(s) * rows_per_split;
  const int64_t r_end = (r_begin + rows_per_split < m) ? r_begin + rows_per_split : m;

  // Loader mapping: column group cg (2 columns), 8 consecutive rows.
  const int cg = tid >> 4, sub = tid & 15;
  float xv[2][8];

  auto load_stage = [&](int64_t r0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int c = c0 + 2 * cg + q;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t r = r0 + 8 * sub + e;
        xv[q][e] = (r < r_end && c < n && 2 * cg + q < NPW) ? X[r + static_cast<int64_t>(c) * ldx] : 0.f;
      }
    }
  };

  f4 acc[2][NB];
  double tot[2][NB][4];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      acc[rt][b] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) tot[rt][b][v] = 0.0;
    }
  // Exponent currently applied to each of this lane's accumulator columns.
  int cur_s[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) cur_s[b] = 0;

  if (tid < kMxCols) rexp[tid] = -1000;
  if (tid == 0) flush_flag = 0;

  auto flush = [&]() {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const double inv = static_cast<double>(pow2f(-cur_s[b]));
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) tot[rt][b][v] += static_cast<double>(acc[rt][b][v]) * inv;
        acc[rt][b] = f4{0.f, 0.f, 0.f, 0.f};
      }
    }
  };

  int stage = 0;
  if (r_begin < r_end) load_stage(r_begin);
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kMxRows, ++stage) {
    __syncthreads();  // previous stage's tiles are consumed
    // Column maxima of this stage: 16 lanes (one DPP row) share a column.
    float cmax[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      float mx = 0.f;
#pragma unroll
      for (int e = 0; e < 8; ++e) mx = fmaxf(mx, fabsf(xv[q][e]));
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 16));
      cmax[q] = mx;
    }
    if (sub == 0) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int cl = 2 * cg + q;
        if (cmax[q] > 0.f) {
          const int e = ((__float_as_int(cmax[q]) >> 23) & 0xff) - 127;
          const int old = rexp[cl];
          if (e > old) {
            rexp[cl] = e;
            flush_flag = 1;
          }
        }
      }
    }
    // Theta bits for the stage: 128 x rows x 2 Philox blocks.
    if (tid < 2 * kMxRows) {
      const int xr = tid & (kMxRows - 1), blk = tid >> 7;
      const int64_t r = r0 + xr;
      Words w = Words{0u, 0u, 0u, 0u};
      if (r < r_end) w = radem_words(seed, r, static_cast<uint32_t>((theta0 >> 7) + blk));
      zb[blk][0][xr] = w.w0;
      zb[blk][1][xr] = w.w1;
      zb[blk][2][xr] = w.w2;
      zb[blk][3][xr] = w.w3;
    }
    __syncthreads();
    // Split this thread's values into hi + lo with the column's scale.
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int cl = 2 * cg + q;
      int ex = rexp[cl];
      int sc = 14 - ex;
      sc = sc > 126 ? 126 : (sc < -126 ? -126 : sc);
      const float f = pow2f(sc);
      _Float16 hv[8], lv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float y = xv[q][e] * f;
        const _Float16 hi = static_cast<_Float16>(y);
        hv[e] = hi;
        lv[e] = static_cast<_Float16>(y - static_cast<float>(hi));
      }
      *reinterpret_cast<u4v*>(&xhi[cl][8 * sub]) = *reinterpret_cast<u4v*>(hv);
      *reinterpret_cast<u4v*>(&xlo[cl][8 * sub]) = *reinterpret_cast<u4v*>(lv);
    }
    // Prefetch the next stage while this one is consumed.
    if (r0 + kMxRows < r_end) load_stage(r0 + kMxRows);
    __syncthreads();
    // Scale changes or periodic flush: fold FP32 sums into FP64 totals.
    const bool periodic = (stage % kMxFlushStages) == 0;
    if (flush_flag || periodic) {
      flush();
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        int sc = 14 - rexp[16 * b + l16];
        cur_s[b] = sc > 126 ? 126 : (sc < -126 ? -126 : sc);
      }
    }
    // Matrix-core loop: 4 steps of 32 rows.
#pragma unroll
    for (int ks = 0; ks < kMxRows / 32; ++ks) {
      h8 a[2];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        const int r = 32 * wave + 16 * rt + l16;  // local Theta row
        const int blk = r >> 7, wd = (r & 127) >> 5, bit = r & 31;
        const u4v w0 = *reinterpret_cast<const u4v*>(&zb[blk][wd][32 * ks + 8 * lg]);
        const u4v w1 = *reinterpret_cast<const u4v*>(&zb[blk][wd][32 * ks + 8 * lg + 4]);
        uint32_t pk[4];
        pk[0] = 0x3C003C00u | (((w0.x >> bit) & 1u) << 15) | (((w0.y >> bit) & 1u) << 31);
        pk[1] = 0x3C003C00u | (((w0.z >> bit) & 1u) << 15) | (((w0.w >> bit) & 1u) << 31);
        pk[2] = 0x3C003C00u | (((w1.x >> bit) & 1u) << 15) | (((w1.y >> bit) & 1u) << 31);
        pk[3] = 0x3C003C00u | (((w1.z >> bit) & 1u) << 15) | (((w1.w >> bit) & 1u) << 31);
        a[rt] = *reinterpret_cast<h8*>(pk);
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const h8 bh = *reinterpret_cast<const h8*>(&xhi[16 * b + l16][32 * ks + 8 * lg]);
        const h8 bl = *reinterpret_cast<const h8*>(&xlo[16 * b + l16][32 * ks + 8 * lg]);
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
          acc[rt][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[rt], bh, acc[rt][b], 0, 0, 0);
          acc[rt][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[rt], bl, acc[rt][b], 0, 0, 0);
        }
      }
    }
    __syncthreads();
    if (tid == 0) flush_flag = 0;
  }
  flush();
  // part[s][c][i] (ld kpad); D element v of lane group lg is Theta row 4 lg + v.
  double* dst = part + static_cast<int64_t>(s) * npad * kpad;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = theta0 + 32 * wave + 16 * rt + 4 * lg + v;
        const int c = c0 + 16 * b + l16;
        dst[static_cast<int64_t>(c) * kpad + i] = tot[rt][b][v];
      }
}

hipError_t launch_sketch_mixed(const float* X, int64_t m, int n, int64_t ldx, int k, uint64_t seed,
                               const SketchPlan& pl, double* part, double* P, int64_t ldp,
                               hipStream_t st) {
  const int nh = static_cast<int>(ceil_div(n, kMxCols));
  const int npw = static_cast<int>((nh > 1) ? kMxCols : round_up(n, 16));
  const int nb = npw / 16;
  const dim3 grid(pl.nsplit * pl.ktiles * nh), block(512);
#define RCQ_MX_CASE(NBV)                                                                          \
  case NBV:                                                                                       \
    sketch_mixed_kernel<NBV><<<grid, block, 0, st>>>(X, m, n, ldx, seed, pl.ktiles, nh,           \
                                                     pl.rows_per_split, pl.kpad, pl.npad, part);  \
    break;
  switch (nb) {
    RCQ_MX_CASE(1) RCQ_MX_CASE(2) RCQ_MX_CASE(3) RCQ_MX_CASE(4)
    default: return hipErrorInvalidValue;
  }
#undef RCQ_MX_CASE
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sketch_reduce(part, pl, k, n, 1.0 / sqrt(static_cast<double>(k)), P, ldp, st);
}

}  // namespace rcq
