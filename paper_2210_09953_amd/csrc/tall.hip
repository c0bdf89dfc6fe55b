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
// gram_kernel: A = Q^T Q (Algorithm 3 step 2), split-K over rows with FP64
// matrix-core accumulation; one wave per 64 x 64 block of the upper
// triangle, rows staged through LDS; per-split partials are reduced in a
// fixed order by gram_reduce_kernel.
#include "common.h"
#include "kernels.h"

namespace rcq {

template <typename T, int NB>
__global__ __launch_bounds__(256) void trsm_kernel(const T* X, int64_t m, int n, int64_t ldx,
                                                   const T* __restrict__ pan, T* Q, int64_t ldq) {
  typedef typename Acc4<T>::type A4;
  __shared__ T tr[4][16][17];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  const int64_t row = static_cast<int64_t>(blockIdx.x) * 64 + wave * 16 + l16;
  // A rows permuted so that D element v of lane group lg is panel column 4 lg + v.
  const int acol = arow_for_blocked_d<T>(l16);
  const bool rok = row < m;
  T qa[4 * NB];

#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const T* pb = pan + 256 * (b * (b + 1) / 2);
    A4 D;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int col = 16 * b + 4 * lg + v;
      D[v] = (rok && col < n) ? X[row + static_cast<int64_t>(col) * ldx] : T(0);
    }
    // D <- X_b^T - R_{<b,b}^T Q_{<b}^T  (A = -R^T block, B = Q^T block)
#pragma unroll
    for (int s = 0; s < 4 * (NB - 1); ++s)
      if (s < 4 * b) D = mfma16x16x4(pb[(4 * s + lg) * 16 + acol], qa[s], D);

    // Diagonal block: column c = 4*lg + v of the panel lives in lane group lg.
    const T* dgb = pb + 16 * b * 16;
#pragma unroll
    for (int gs = 0; gs < 4; ++gs) {
      if (lg == gs) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          T x = D[v];
#pragma unroll
          for (int vp = 0; vp < v; ++vp) x -= D[vp] * dgb[(4 * gs + vp) * 16 + 4 * gs + v];
          D[v] = x / dgb[(4 * gs + v) * 16 + 4 * gs + v];
        }
      }
      if (gs < 3) {
        T q[4];
#pragma unroll
        for (int vp = 0; vp < 4; ++vp) q[vp] = __shfl(D[vp], l16 + 16 * gs, 64);
        if (lg > gs) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            T x = D[v];
#pragma unroll
            for (int vp = 0; vp < 4; ++vp) x -= q[vp] * dgb[(4 * gs + vp) * 16 + 4 * lg + v];
            D[v] = x;
          }
        }
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int col = 16 * b + 4 * lg + v;
      if (rok && col < n) Q[row + static_cast<int64_t>(col) * ldq] = D[v];
    }
    if (b + 1 < NB) {
#pragma unroll
      for (int v = 0; v < 4; ++v) tr[wave][4 * lg + v][l16] = D[v];
      wave_sync();
#pragma unroll
      for (int s = 0; s < 4; ++s) qa[4 * b + s] = tr[wave][4 * s + lg][l16];
      wave_sync();
    }
  }
}

template <typename T>
static hipError_t trsm_dispatch(int nb, const T* X, int64_t m, int n, int64_t ldx, const T* pan,
                                T* Q, int64_t ldq, hipStream_t st) {
  const unsigned grid = static_cast<unsigned>(ceil_div(m, 64));
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
constexpr int kGrRows = 16;

template <typename T, int NBB>
__global__ __launch_bounds__(640) void gram_kernel(const T* __restrict__ Q, int64_t m, int n,
                                                   int64_t ldq, int64_t rows_per_split,
                                                   double* __restrict__ gpart) {
  constexpr int NP = 64 * NBB;
  constexpr int NW = NBB * (NBB + 1) / 2;
  __shared__ double qs[kGrRows][NP + 1];
  const int s = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  // wave -> upper block (bi, bj), bi <= bj
  int bi = 0, bj = 0, cnt = 0;
  for (int j = 0; j < NBB; ++j)
    for (int i = 0; i <= j; ++i) {
      if (cnt == wave) {
        bi = i;
        bj = j;
      }
      ++cnt;
    }
  const int64_t r_begin = static_cast<int64_t>(s) * rows_per_split;
  const int64_t r_end = (r_begin + rows_per_split < m) ? r_begin + rows_per_split : m;
  d4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  for (int64_t r0 = r_begin; r0 < r_end; r0 += kGrRows) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < kGrRows * NP; idx += NW * 64) {
      const int jj = idx % kGrRows, c = idx / kGrRows;
      const int64_t r = r0 + jj;
      qs[jj][c] = (r < r_end && c < n) ? static_cast<double>(Q[r + static_cast<int64_t>(c) * ldq]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kGrRows / 4; ++ks) {
      double av[4], bv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        av[t] = qs[4 * ks + lg][64 * bi + 16 * t + l16];
        bv[t] = qs[4 * ks + lg][64 * bj + 16 * t + l16];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mfma16x16x4(av[a], bv[b], acc[a][b]);
    }
  }
  double* dst = gpart + static_cast<int64_t>(s) * NP * NP;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 64 * bi + 16 * a + drow<double>(lg, v);
        const int c = 64 * bj + 16 * b + l16;
        dst[r + static_cast<int64_t>(c) * NP] = acc[a][b][v];
      }
}

template <typename T>
static hipError_t gram_dispatch(const T* Q, int64_t m, int n, int64_t ldq, const GramPlan& gp,
                                double* gpart, hipStream_t st) {
  const unsigned grid = static_cast<unsigned>(gp.nsplit);
  switch (gp.nbb) {
    case 1: gram_kernel<T, 1><<<grid, 64, 0, st>>>(Q, m, n, ldq, gp.rows_per_split, gpart); break;
    case 2: gram_kernel<T, 2><<<grid, 192, 0, st>>>(Q, m, n, ldq, gp.rows_per_split, gpart); break;
    case 3: gram_kernel<T, 3><<<grid, 384, 0, st>>>(Q, m, n, ldq, gp.rows_per_split, gpart); break;
    case 4: gram_kernel<T, 4><<<grid, 640, 0, st>>>(Q, m, n, ldq, gp.rows_per_split, gpart); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gram(const void* Q, bool f32, int64_t m, int n, int64_t ldq, const GramPlan& gp,
                       double* gpart, hipStream_t st) {
  if (f32) return gram_dispatch<float>(static_cast<const float*>(Q), m, n, ldq, gp, gpart, st);
  return gram_dispatch<double>(static_cast<const double*>(Q), m, n, ldq, gp, gpart, st);
}

}  // namespace rcq
