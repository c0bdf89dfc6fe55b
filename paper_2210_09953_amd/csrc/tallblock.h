// tallblock.h -- workgroup-level bodies of the generic tall solve and
// product (trsm_kernel, trmm_kernel in tall.hip), shared with the
// persistent batched engine (batched.hip), which runs them as tasks.
#pragma once
#include "common.h"

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

// LDS of trsm_block (one 256-thread workgroup).
template <typename T, int NB>
struct TrsmLds {
  T tq[4][RowBlocks<T>::value][16][4];
  T pbuf[2][256 * NB];
};

// Rows 64 RB blk .. 64 RB blk + 64 RB - 1 of Q = X R^{-1} (trsm_kernel's
// work for workgroup blk); all 256 threads of the calling workgroup take
// part, and its LDS is `sh`.
//
// SK (the column-oriented update): panels 0..s0-1 are already solved and sit
// in Q.  They are loaded from there straight into the operand layout of the
// later updates and neither solved again nor stored; X then holds columns
// 16 s0 .. n-1.  Without SK, s0 is ignored.
template <typename T, int NB, bool SK = false>
__device__ __forceinline__ void trsm_block(const T* X, int64_t m, int n, int64_t ldx,
                                           const T* __restrict__ pan, T* Q, int64_t ldq,
                                           int64_t blk, TrsmLds<T, NB>& sh, int s0 = 0) {
  typedef typename Acc4<T>::type A4;
  constexpr int RB = RowBlocks<T>::value;
  auto& tq = sh.tq;
  auto& pbuf = sh.pbuf;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  const int64_t row0 = blk * 64 * RB + wave * 16 * RB + l16;
  // A rows permuted so that D element v of lane group lg is panel column 4 lg + v.
  const int acol = arow_for_blocked_d<T>(l16);
  T qa[RB][4 * NB];
  T stg[NB];

  // X of the next panel is loaded one panel ahead (its latency overlaps the
  // current panel's work; loads are not moved across the barriers).
  // Whole workgroup inside the matrix: no per-element bounds checks.
  const bool full = blk * 64 * RB + 64 * RB <= m && n == 16 * NB;
  T xn[RB][4];
  auto load_x = [&](int b) {
    if constexpr (SK) {
      if (b < s0) {
        // a solved panel: lane group lg takes columns 4 v + lg (the operand
        // layout qa[4 b + v])
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const int64_t row = row0 + 16 * rb;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int col = 16 * b + 4 * v + lg;
            xn[rb][v] = (full || row < m) ? Q[row + static_cast<int64_t>(col) * ldq] : T(0);
          }
        }
        return;
      }
    }
    const int cb = 16 * (SK ? b - s0 : b);  // panel b's first column in X
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int64_t row = row0 + 16 * rb;
      if (full) {
        const T* xb = X + row + static_cast<int64_t>(4 * lg) * ldx;
#pragma unroll
        for (int v = 0; v < 4; ++v) xn[rb][v] = xb[static_cast<int64_t>(cb + v) * ldx];
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = 16 * b + 4 * lg + v;
          xn[rb][v] = (row < m && col < n)
                          ? X[row + static_cast<int64_t>(cb + 4 * lg + v) * ldx] : T(0);
        }
      }
    }
  };
  load_x(0);
  panel_fetch<T, NB>(pan, 0, stg);
  panel_store<T, NB>(pbuf[0], 0, stg);
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const T* pb = pbuf[b & 1];
    if (SK && b < s0) {
      // already solved: into the operand registers as loaded
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) qa[rb][4 * b + v] = xn[rb][v];
      if (b + 1 < NB) {
        panel_fetch<T, NB>(pan, b + 1, stg);
        load_x(b + 1);
        panel_store<T, NB>(pbuf[(b + 1) & 1], b + 1, stg);
        __syncthreads();
      }
      continue;
    }
    A4 D[RB], E[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        D[rb][v] = xn[rb][v];
        E[rb][v] = T(0);
      }
    if (b + 1 < NB) {
      panel_fetch<T, NB>(pan, b + 1, stg);  // overlap with this panel
      load_x(b + 1);
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
      if (full) {
        T* qb = Q + row + static_cast<int64_t>(4 * lg) * ldq;
#pragma unroll
        for (int v = 0; v < 4; ++v) qb[static_cast<int64_t>(16 * b + v) * ldq] = D[rb][v];
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = 16 * b + 4 * lg + v;
          if (row < m && col < n) Q[row + static_cast<int64_t>(col) * ldq] = D[rb][v];
        }
      }
    }
    if (b + 1 < NB) {
      panel_store<T, NB>(pbuf[(b + 1) & 1], b + 1, stg);
      __syncthreads();
    }
  }
}


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
__device__ __forceinline__ void trmm_block(T* Q, int64_t m, int n, int64_t ldq,
                                           const T* __restrict__ pan, const T* __restrict__ C,
                                           int64_t ldc, int64_t blk, T (&pbuf)[2][256 * NB]) {
  typedef typename Acc4<T>::type A4;
  constexpr int RB = RowBlocks<T>::value;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  const int64_t row0 = blk * 64 * RB + wave * 16 * RB + l16;
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


}  // namespace rcq
