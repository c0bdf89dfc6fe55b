// tall.hip -- the passes over the tall matrix after the sketch.
//
// trsm_kernel: Q = X R^{-1} (Algorithm 2 step 3, Algorithm 3 step 4) by
// forward substitution on every row, the operation whose row-wise backward
// error bound |dR| <= 1.1 u n |R| (Higham Thm 8.5, as used in Section 5.1)
// gives eq. (main1).  R is never inverted: each 16-column panel first takes
// the update X_b - Q_{<b} R_{<b,b} on 16x16x4 matrix cores (the same sums
// as the substitution, in another order), then solves its 16 x 16 diagonal
// block by plain substitution with true division.  A wave owns 16 rows and
// keeps all of its computed Q entries in registers (the B operand layout),
// so X is read once and Q written once.  The product is set up transposed
// (panel columns x rows) so that loads and stores of X and Q walk 16
// consecutive rows of a column; the A operand's rows are permuted so that
// each lane group holds 4 consecutive panel columns for the diagonal solve.
// Works in place (Q == X).
//
// trmm_kernel: Q = Q1 T for the upper triangular T = R'^{-1} (the second
// solve as a product; R' is well conditioned).
//
// gram_kernel: A = Q^T Q (Algorithm 3 step 2), split-K over rows on matrix
// cores in the working precision, FP64 partial sums per split (FP32 sums are
// folded into FP64 every 2048 rows); per-split partials are reduced in a
// fixed order by gram_reduce_kernel.
#include "common.h"
#include "kernels.h"

namespace rcq {

// Copies panel b (rows 0..16b+15 x 16 columns) of the packed R array to
// registers (staging toward LDS): thread t holds elements t, t+256, ...
template <typename T, int NB>
__device__ __forceinline__ void panel_fetch(const T* __restrict__ pan, int b, T (&st)[NB]) {
  const T* pb = pan + 256 * (b * (b + 1) / 2);
#pragma unroll
  for (int q = 0; q < NB; ++q)
    if (q <= b) st[q] = pb[threadIdx.x + 256 * q];
}
template <typename T, int NB>
__device__ __forceinline__ void panel_store(T* __restrict__ buf, int b, const T (&st)[NB]) {
#pragma unroll
  for (int q = 0; q < NB; ++q)
    if (q <= b) buf[threadIdx.x + 256 * q] = st[q];
}

// Rows per wave: 16 x RB (two 16-row blocks share every A operand in FP32;
// FP64 keeps one to stay within the register file).
#ifndef RCQ_F32_ROW_BLOCKS
#define RCQ_F32_ROW_BLOCKS 1
#endif
template <typename T>
struct RowBlocks {
  static constexpr int value = sizeof(T) == 4 ? RCQ_F32_ROW_BLOCKS : 1;
};

template <typename T, int NB>
__global__ __launch_bounds__(256) void trsm_kernel(const T* X, int64_t m, int n, int64_t ldx,
                                                   const T* __restrict__ pan, T* Q, int64_t ldq) {
  typedef typename Acc4<T>::type A4;
  constexpr int RB = RowBlocks<T>::value;
  __shared__ T tq[4][RB][16][4];
  __shared__ T pbuf[2][256 * NB];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * 64 * RB + wave * 16 * RB + l16;
  // A rows permuted so that D element v of lane group lg is panel column 4 lg + v.
  const int acol = arow_for_blocked_d<T>(l16);
  T qa[RB][4 * NB];
  T stg[NB];

  panel_fetch<T, NB>(pan, 0, stg);
  panel_store<T, NB>(pbuf[0], 0, stg);
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const T* pb = pbuf[b & 1];
    if (b + 1 < NB) panel_fetch<T, NB>(pan, b + 1, stg);  // overlap with this panel
    A4 D[RB], E[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int64_t row = row0 + 16 * rb;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = 16 * b + 4 * lg + v;
        D[rb][v] = (row < m && col < n) ? X[row + static_cast<int64_t>(col) * ldx] : T(0);
        E[rb][v] = T(0);
      }
    }
    // D <- X_b^T - R_{<b,b}^T Q_{<b}^T (A = -R^T block, B = Q^T block), two chains.
#pragma unroll
    for (int s = 0; s < 4 * (NB - 1); s += 2)
      if (s < 4 * b) {
        const T a0 = pb[(4 * s + lg) * 16 + acol];
        const T a1 = pb[(4 * (s + 1) + lg) * 16 + acol];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          D[rb] = mfma16x16x4(a0, qa[rb][s], D[rb]);
          E[rb] = mfma16x16x4(a1, qa[rb][s + 1], E[rb]);
        }
      }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) D[rb][v] += E[rb][v];

    // Diagonal block (its diagonal holds 1/R_jj): lane group gs substitutes
    // its 4 columns, the solved 16 x 4 piece goes through LDS into the B
    // layout (which is also the register copy of Q for later panels), and
    // one matrix-core product subtracts it from the panel's later columns.
    const T* dgb = pb + 16 * b * 16;
#pragma unroll
    for (int gs = 0; gs < 4; ++gs) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        T x[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          T t = D[rb][v];
#pragma unroll
          for (int vp = 0; vp < v; ++vp) t -= x[vp] * dgb[(4 * gs + vp) * 16 + 4 * gs + v];
          x[v] = t * dgb[(4 * gs + v) * 16 + 4 * gs + v];
        }
        if (lg == gs) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            D[rb][v] = x[v];
            tq[wave][rb][l16][v] = x[v];
          }
        }
      }
      wave_sync();
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) qa[rb][4 * b + gs] = tq[wave][rb][l16][lg];
      wave_sync();
      if (gs < 3) {
        const T a = (acol > 4 * gs + 3) ? -dgb[(4 * gs + lg) * 16 + acol] : T(0);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) D[rb] = mfma16x16x4(a, qa[rb][4 * b + gs], D[rb]);
      }
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int64_t row = row0 + 16 * rb;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = 16 * b + 4 * lg + v;
        if (row < m && col < n) Q[row + static_cast<int64_t>(col) * ldq] = D[rb][v];
      }
    }
    if (b + 1 < NB) {
      panel_store<T, NB>(pbuf[(b + 1) & 1], b + 1, stg);
      __syncthreads();
    }
  }
}

template <typename T>
static hipError_t trsm_dispatch(int nb, const T* X, int64_t m, int n, int64_t ldx, const T* pan,
                                T* Q, int64_t ldq, hipStream_t st) {
  const unsigned grid = static_cast<unsigned>(ceil_div(m, 64 * RowBlocks<T>::value));
#define RCQ_TR_CASE(NBV)                                                       \
  case NBV:                                                                    \
    trsm_kernel<T, NBV><<<grid, 256, 0, st>>>(X, m, n, ldx, pan, Q, ldq);      \
    break;
  switch (nb) {
    RCQ_TR_CASE(1) RCQ_TR_CASE(2) RCQ_TR_CASE(3) RCQ_TR_CASE(4) RCQ_TR_CASE(5) RCQ_TR_CASE(6)
    RCQ_TR_CASE(7) RCQ_TR_CASE(8) RCQ_TR_CASE(9) RCQ_TR_CASE(10) RCQ_TR_CASE(11) RCQ_TR_CASE(12)
    RCQ_TR_CASE(13) RCQ_TR_CASE(14) RCQ_TR_CASE(15) RCQ_TR_CASE(16)
    default: return hipErrorInvalidValue;
  }
#undef RCQ_TR_CASE
  return hipGetLastError();
}

hipError_t launch_trsm(const void* X, bool f32, int64_t m, int n, int64_t ldx, const void* pan,
                       void* Q, int64_t ldq, hipStream_t st) {
  if (m == 0) return hipSuccess;
  const int nb = static_cast<int>(ceil_div(n, 16));
  if (f32)
    return trsm_dispatch<float>(nb, static_cast<const float*>(X), m, n, ldx,
                                static_cast<const float*>(pan), static_cast<float*>(Q), ldq, st);
  return trsm_dispatch<double>(nb, static_cast<const double*>(X), m, n, ldx,
                               static_cast<const double*>(pan), static_cast<double*>(Q), ldq, st);
}

// ----------------------------------------------------------------------------
// Q = Q1 T for an upper triangular T (T = R'^{-1}, Algorithm 3 step 4 as a
// product: R' comes from the Cholesky factor of the Gram of a well
// conditioned Q1, so its inverse is safe to form).  Same layout as the
// solve: a wave loads its 16 rows of Q1 into registers first (so the
// product can overwrite them), then each 16-column output panel is a chain
// of 16x16x4 matrix-core products with no diagonal solve.
// FULL = false: Q <- Q T for upper triangular T (panel b holds rows 0..16b+15).
// FULL = true:  Q <- C + Q B for a dense n x n B (panel b holds all rows);
// C (ld ldc) may be null.  Both work in place.
template <typename T, int NB, bool FULL>
__global__ __launch_bounds__(256) void trmm_kernel(T* Q, int64_t m, int n, int64_t ldq,
                                                   const T* __restrict__ pan,
                                                   const T* __restrict__ C, int64_t ldc) {
  typedef typename Acc4<T>::type A4;
  constexpr int RB = RowBlocks<T>::value;
  __shared__ T pbuf[2][256 * NB];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * 64 * RB + wave * 16 * RB + l16;
  const int acol = arow_for_blocked_d<T>(l16);
  T qa[RB][4 * NB];
  T stg[NB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int64_t row = row0 + 16 * rb;
#pragma unroll
    for (int s = 0; s < 4 * NB; ++s) {
      const int col = 4 * s + lg;
      qa[rb][s] = (row < m && col < n) ? Q[row + static_cast<int64_t>(col) * ldq] : T(0);
    }
  }
  auto fetch = [&](int b) {
    if (FULL) {
      const T* pb = pan + 256 * NB * b;
#pragma unroll
      for (int q = 0; q < NB; ++q) stg[q] = pb[threadIdx.x + 256 * q];
    } else {
      panel_fetch<T, NB>(pan, b, stg);
    }
  };
  auto store = [&](T* buf, int b) {
    if (FULL) {
#pragma unroll
      for (int q = 0; q < NB; ++q) buf[threadIdx.x + 256 * q] = stg[q];
    } else {
      panel_store<T, NB>(buf, b, stg);
    }
  };
  fetch(0);
  store(pbuf[0], 0);
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const T* pb = pbuf[b & 1];
    if (b + 1 < NB) fetch(b + 1);
    A4 D[RB], E[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        D[rb][v] = T(0);
        E[rb][v] = T(0);
      }
#pragma unroll
    for (int s = 0; s < 4 * NB; s += 2)
      if (FULL || s < 4 * (b + 1)) {
        const T a0 = pb[(4 * s + lg) * 16 + acol];
        const T a1 = pb[(4 * (s + 1) + lg) * 16 + acol];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          D[rb] = mfma16x16x4(a0, qa[rb][s], D[rb]);
          E[rb] = mfma16x16x4(a1, qa[rb][s + 1], E[rb]);
        }
      }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int64_t row = row0 + 16 * rb;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = 16 * b + 4 * lg + v;
        if (row < m && col < n) {
          T y = D[rb][v] + E[rb][v];
          if (C) y += C[row + static_cast<int64_t>(col) * ldc];
          Q[row + static_cast<int64_t>(col) * ldq] = y;
        }
      }
    }
    if (b + 1 < NB) {
      store(pbuf[(b + 1) & 1], b + 1);
      __syncthreads();
    }
  }
}

template <typename T, bool FULL>
static hipError_t trmm_dispatch(int nb, T* Q, int64_t m, int n, int64_t ldq, const T* pan,
                                const T* C, int64_t ldc, hipStream_t st) {
  const unsigned grid = static_cast<unsigned>(ceil_div(m, 64 * RowBlocks<T>::value));
#define RCQ_TM_CASE(NBV)                                                            \
  case NBV:                                                                         \
    trmm_kernel<T, NBV, FULL><<<grid, 256, 0, st>>>(Q, m, n, ldq, pan, C, ldc);     \
    break;
  switch (nb) {
    RCQ_TM_CASE(1) RCQ_TM_CASE(2) RCQ_TM_CASE(3) RCQ_TM_CASE(4) RCQ_TM_CASE(5) RCQ_TM_CASE(6)
    RCQ_TM_CASE(7) RCQ_TM_CASE(8) RCQ_TM_CASE(9) RCQ_TM_CASE(10) RCQ_TM_CASE(11) RCQ_TM_CASE(12)
    RCQ_TM_CASE(13) RCQ_TM_CASE(14) RCQ_TM_CASE(15) RCQ_TM_CASE(16)
    default: return hipErrorInvalidValue;
  }
#undef RCQ_TM_CASE
  return hipGetLastError();
}

hipError_t launch_trmm(void* Q, bool f32, int64_t m, int n, int64_t ldq, const void* pan,
                       hipStream_t st) {
  if (m == 0) return hipSuccess;
  const int nb = static_cast<int>(ceil_div(n, 16));
  if (f32)
    return trmm_dispatch<float, false>(nb, static_cast<float*>(Q), m, n, ldq,
                                       static_cast<const float*>(pan), nullptr, 0, st);
  return trmm_dispatch<double, false>(nb, static_cast<double*>(Q), m, n, ldq,
                                      static_cast<const double*>(pan), nullptr, 0, st);
}

hipError_t launch_gemm_add(void* Q, bool f32, int64_t m, int n, int64_t ldq, const void* pan,
                           const void* C, int64_t ldc, hipStream_t st) {
  if (m == 0) return hipSuccess;
  const int nb = static_cast<int>(ceil_div(n, 16));
  if (f32)
    return trmm_dispatch<float, true>(nb, static_cast<float*>(Q), m, n, ldq,
                                      static_cast<const float*>(pan), static_cast<const float*>(C),
                                      ldc, st);
  return trmm_dispatch<double, true>(nb, static_cast<double*>(Q), m, n, ldq,
                                     static_cast<const double*>(pan), static_cast<const double*>(C),
                                     ldc, st);
}

// ----------------------------------------------------------------------------
// Gram A = Q^T Q.  One wave per 64 x 64 block of the upper triangle; rows
// staged through LDS 32 at a time; products on matrix cores in the working
// precision.  FP64 data accumulates in FP64.  FP32 data accumulates in FP32
// for at most kGrFlush rows, then the sums are added into the workgroup's
// own FP64 partial in memory (written by this workgroup only: deterministic).
constexpr int kGrFlush = 2048;
template <typename T>
struct GramRows {
  static constexpr int value = sizeof(T) == 4 ? 32 : 16;
};

// CROSS = false: A = Q^T Q, upper 64 x 64 blocks.  CROSS = true: C = Q^T B
// for a second tall matrix B (ld ldb), all blocks (used by the adjoint).
template <typename T, int NBB, bool CROSS>
__global__ __launch_bounds__(64 * (CROSS ? NBB * NBB : NBB * (NBB + 1) / 2)) void gram_kernel(
    const T* __restrict__ Q, int64_t m, int n, int64_t ldq, int64_t rows_per_split,
    double* __restrict__ gpart, const T* __restrict__ B, int64_t ldb) {
  typedef typename Acc4<T>::type A4;
  constexpr int NP = 64 * NBB;
  constexpr int NW = CROSS ? NBB * NBB : NBB * (NBB + 1) / 2;
  constexpr int kGrRows = GramRows<T>::value;
  // Column-major staging: rows of a column are contiguous (conflict-free
  // stores of the coalesced loads); the row stride kLd = kGrRows + 4 words
  // spreads the 16 columns x 4 rows of an operand read over distinct banks.
  constexpr int kLd = kGrRows + 4;
  __shared__ T qs[NP][kLd];
  __shared__ T bs[CROSS ? NP : 1][CROSS ? kLd : 1];
  const int s = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  int bi = 0, bj = 0, cnt = 0;
  if (CROSS) {
    bi = wave % NBB;
    bj = wave / NBB;
  } else {
    for (int j = 0; j < NBB; ++j)
      for (int i = 0; i <= j; ++i) {
        if (cnt == wave) {
          bi = i;
          bj = j;
        }
        ++cnt;
      }
  }
  const int64_t r_begin = static_cast<int64_t>(s) * rows_per_split;
  const int64_t r_end = (r_begin + rows_per_split < m) ? r_begin + rows_per_split : m;
  double* dst = gpart + static_cast<int64_t>(s) * NP * NP;
  A4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[a][b][v] = T(0);
  bool first = true;
  // Element (a, b, v) of this lane sits at dst + lane_off + constant; the
  // offset is laundered at each flush so the 64 addresses are not kept live
  // across the row loop.
  const int64_t lane_off = (64 * bi + drow<T>(lg, 0)) + static_cast<int64_t>(64 * bj + l16) * NP;
#define RCQ_GRAM_FLUSH()                                                        \
  do {                                                                          \
    int64_t lo = lane_off;                                                      \
    asm volatile("" : "+v"(lo));                                                \
    double* base = dst + lo;                                                    \
    _Pragma("unroll") for (int a = 0; a < 4; ++a)                               \
    _Pragma("unroll") for (int b = 0; b < 4; ++b)                               \
    _Pragma("unroll") for (int v = 0; v < 4; ++v) {                             \
      double* p = base + (16 * a + (drow<T>(lg, v) - drow<T>(lg, 0))) +         \
                  static_cast<int64_t>(16 * b) * NP;                            \
      const double val = static_cast<double>(acc[a][b][v]);                     \
      *p = first ? val : *p + val;                                              \
      acc[a][b][v] = T(0);                                                      \
      if (v == 3 && b == 3) __builtin_amdgcn_sched_barrier(0);                  \
    }                                                                           \
    first = false;                                                              \
  } while (0)
  // FP32: register prefetch of the next stage (kGrRows x NP values over
  // NW*64 threads).  FP64 (accumulators twice as large): direct staging.
  constexpr bool kPre = sizeof(T) == 4 && !CROSS;
  constexpr int PER = kPre ? (kGrRows * NP + NW * 64 - 1) / (NW * 64) : 1;
  T pre[PER];
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = threadIdx.x + q * NW * 64;
      const int jj = idx % kGrRows, c = idx / kGrRows;
      const int64_t r = r0 + jj;
      pre[q] = (idx < kGrRows * NP && r < r_end && c < n) ? Q[r + static_cast<int64_t>(c) * ldq] : T(0);
    }
  };
  if (kPre && r_begin < r_end) fetch(r_begin);
  int64_t since = 0;
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kGrRows) {
    __syncthreads();
    if (kPre) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int idx = threadIdx.x + q * NW * 64;
        if (idx < kGrRows * NP) qs[idx / kGrRows][idx % kGrRows] = pre[q];
      }
    } else {
      for (int idx = threadIdx.x; idx < kGrRows * NP; idx += NW * 64) {
        const int jj = idx % kGrRows, c = idx / kGrRows;
        const int64_t r = r0 + jj;
        const bool in = r < r_end && c < n;
        qs[c][jj] = in ? Q[r + static_cast<int64_t>(c) * ldq] : T(0);
        if (CROSS) bs[c][jj] = in ? B[r + static_cast<int64_t>(c) * ldb] : T(0);
      }
    }
    __syncthreads();
    if (kPre && r0 + kGrRows < r_end) fetch(r0 + kGrRows);
#pragma unroll
    for (int ks = 0; ks < kGrRows / 4; ++ks) {
      T av[4], bv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        av[t] = qs[64 * bi + 16 * t + l16][4 * ks + lg];
        bv[t] = CROSS ? bs[64 * bj + 16 * t + l16][4 * ks + lg] : qs[64 * bj + 16 * t + l16][4 * ks + lg];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mfma16x16x4(av[a], bv[b], acc[a][b]);
    }
    since += kGrRows;
    if (sizeof(T) == 4 && since >= kGrFlush) {
      RCQ_GRAM_FLUSH();
      since = 0;
    }
  }
  RCQ_GRAM_FLUSH();
#undef RCQ_GRAM_FLUSH
}
template <typename T, bool CROSS>
static hipError_t gram_dispatch(const T* Q, int64_t m, int n, int64_t ldq, const GramPlan& gp,
                                double* gpart, const T* B, int64_t ldb, hipStream_t st) {
  const unsigned grid = static_cast<unsigned>(gp.nsplit);
  auto nw = [](int b) { return CROSS ? b * b : b * (b + 1) / 2; };
  switch (gp.nbb) {
    case 1: gram_kernel<T, 1, CROSS><<<grid, 64 * nw(1), 0, st>>>(Q, m, n, ldq, gp.rows_per_split, gpart, B, ldb); break;
    case 2: gram_kernel<T, 2, CROSS><<<grid, 64 * nw(2), 0, st>>>(Q, m, n, ldq, gp.rows_per_split, gpart, B, ldb); break;
    case 3: gram_kernel<T, 3, CROSS><<<grid, 64 * nw(3), 0, st>>>(Q, m, n, ldq, gp.rows_per_split, gpart, B, ldb); break;
    case 4: gram_kernel<T, 4, CROSS><<<grid, 64 * nw(4), 0, st>>>(Q, m, n, ldq, gp.rows_per_split, gpart, B, ldb); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gram(const void* Q, bool f32, int64_t m, int n, int64_t ldq, const GramPlan& gp,
                       double* gpart, hipStream_t st) {
  if (f32)
    return gram_dispatch<float, false>(static_cast<const float*>(Q), m, n, ldq, gp, gpart, nullptr, 0, st);
  return gram_dispatch<double, false>(static_cast<const double*>(Q), m, n, ldq, gp, gpart, nullptr, 0, st);
}

hipError_t launch_cross_gram(const void* A, const void* B, bool f32, int64_t m, int n, int64_t lda,
                             int64_t ldb, const GramPlan& gp, double* gpart, hipStream_t st) {
  if (f32)
    return gram_dispatch<float, true>(static_cast<const float*>(A), m, n, lda, gp, gpart,
                                      static_cast<const float*>(B), ldb, st);
  return gram_dispatch<double, true>(static_cast<const double*>(A), m, n, lda, gp, gpart,
                                     static_cast<const double*>(B), ldb, st);
}

}  // namespace rcq
