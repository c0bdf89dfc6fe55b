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
// solve as a product; R' is well conditioned); trmm_bf3_kernel does the FP32
// case on bf16 matrix cores with FP32-accurate three-way splits.
//
// gram_kernel: A = Q^T Q (Algorithm 3 step 2), split-K over rows on matrix
// cores in the working precision, FP64 partial sums per split (FP32 sums are
// folded into FP64 every 2048 rows); per-split partials are reduced in a
// fixed order by gram_reduce_kernel.
#include <utility>

#include "common.h"
#include "kernels.h"
#include "tallblock.h"

namespace rcq {

// bf16 x 8 matrix-core operand, and the exact split of an FP32 value into
// three bf16 parts (bit patterns in the high halves): h keeps the top 8
// significand bits, d the next 8 of the remainder, l the last 8.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4v_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void split3(float x, uint32_t& h, uint32_t& d, uint32_t& l) {
  h = __float_as_uint(x) & 0xFFFF0000u;
  const float r = x - __uint_as_float(h);
  d = __float_as_uint(r) & 0xFFFF0000u;
  l = __float_as_uint(r - __uint_as_float(d));
}
constexpr int kG3Rows = 32;  // Gram rows per stage = K of one bf16 matrix-core step

template <typename T, int NB, bool SK = false>
__global__ __launch_bounds__(256) void trsm_kernel(const T* X, int64_t m, int n, int64_t ldx,
                                                   const T* __restrict__ pan, T* Q, int64_t ldq,
                                                   int s0 = 0) {
  __shared__ TrsmLds<T, NB> sh;
  trsm_block<T, NB, SK>(X, m, n, ldx, pan, Q, ldq, blockIdx.x, sh, s0);
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

// Q = Q1 T (or C + Q B) by trmm_block, one 64 RB-row block per workgroup.
template <typename T, int NB, bool FULL>
__global__ __launch_bounds__(256) void trmm_kernel(T* Q, int64_t m, int n, int64_t ldq,
                                                   const T* __restrict__ pan,
                                                   const T* __restrict__ C, int64_t ldc) {
  __shared__ T pbuf[2][256 * NB];
  trmm_block<T, NB, FULL>(Q, m, n, ldq, pan, C, ldc, blockIdx.x, pbuf);
}

// Direct global -> LDS operand staging for the tall bf16 x 3 kernels.  A
// panel of `bytes` bytes is copied as 1 KiB wave-instructions (16 bytes per
// lane) dealt round-robin to the kTallWaves waves of the workgroup; every wave issues
// the same number of instructions (the surplus ones read the panel's first
// KiB into a 1 KiB sink), so the wait counts below are compile-time facts.
// Waves per workgroup of the tall bf16 x 3 kernels (16 rows each): one
// staged copy of the operand panels serves 16 kTallWaves rows.
constexpr int kTallWaves = 8;
__host__ __device__ constexpr int dma_kib(int bytes) { return (bytes + 1023) / 1024; }
__host__ __device__ constexpr int dma_per_wave(int bytes) {
  return (dma_kib(bytes) + kTallWaves - 1) / kTallWaves;
}

__device__ __forceinline__ void dma_panel(const unsigned char* __restrict__ src, int bytes,
                                          unsigned char* slot, unsigned char* sink, int wave,
                                          int lane) {
  const int w = dma_kib(bytes);
#pragma unroll
  for (int i = 0; i < dma_per_wave(bytes); ++i) {
    const int j = wave + kTallWaves * i;
    const bool live = j < w;
    const unsigned char* g = src + (live ? 1024 * j : 0) + 16 * lane;
    unsigned char* l = live ? slot + 1024 * j : sink;
    __builtin_amdgcn_global_load_lds(g, l, 16, 0, 0);
  }
}

// Compute units of the current device (queried once per device).
static int device_cus() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cus[dev] == 0) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
      c = 256;
    cus[dev] = c;
  }
  return cus[dev];
}

// One 16-byte direct global -> LDS load per lane: lane L's bytes land at
// slot + 16 L.
__device__ __forceinline__ void dma16(const void* src, void* slot) {
  __builtin_amdgcn_global_load_lds(src, slot, 16, 0, 0);
}

// s_waitcnt vmcnt(N).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// f(integral_constant<int, 0>), ..., f(integral_constant<int, N - 1>): a loop
// whose index is a compile-time constant in the body.
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Workgroup barrier without a memory fence (the fence would wait for every
// outstanding load, including the staging of later panels); LDS visibility
// comes from the explicit vmcnt / lgkmcnt waits before it.
__device__ __forceinline__ void wg_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// ----------------------------------------------------------------------------
// Q = Q1 T for FP32 Q1 on bf16 matrix cores (the FP32 second solve).  Both
// operands are split exactly into three bf16 parts (split3: T in advance by
// make_bf3_panels, Q1 rows when loaded) and each 32-column chunk of the
// product takes the six significant bf16 products, summed from zero on the
// matrix cores and added to the output in FP32 with round-to-nearest vector
// adds.  A wave keeps its 16 rows of Q1, split, in registers (96 registers
// for n = 256), so the product works in place.  Panel b of T (output columns
// 16b..16b+15, chunks 0..b/2) is staged in LDS two panels ahead by direct
// global -> LDS loads.
typedef unsigned int u4b_t __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr int bf3_panel_offset(int b) {
  // sum over b' < b of (b'/2 + 1) chunks of 3 KiB
  return 3072 * ((b & 1) ? ((b + 1) / 2) * ((b + 1) / 2) : (b / 2) * (b / 2 + 1));
}

// Bytes of panel b of T (chunks 0..b/2 of 3 KiB).
__host__ __device__ constexpr int trmm_bf3_psize(int b) { return (b / 2 + 1) * 3072; }

// FULL, persistence and blk0 as for trsm_bf3_kernel (FULL: n = 32 NCH).
template <int NB, bool FULL>
__global__ __launch_bounds__(64 * kTallWaves) void trmm_bf3_kernel(float* Q, int64_t m, int n, int64_t ldq,
                                                       const unsigned char* __restrict__ pan3,
                                                       int64_t blk0) {
  constexpr int NCH = (NB + 1) / 2;
  constexpr int PMAX = NCH * 3072;
  constexpr int SLOT = dma_kib(PMAX) * 1024;
  constexpr bool persist = FULL && NB % 4 == 0;
  constexpr int NSL = persist ? 4 : 3;
  constexpr int64_t kTile = 16 * kTallWaves;
  // NSL panel slots (panel b in slot b % NSL, staged two panels ahead), a
  // sink, and (whole tiles) two chunk slots of 2 KiB per wave
  __shared__ __align__(1024) unsigned char ring[NSL * SLOT + 1024 + (FULL ? 2 * 2048 * kTallWaves : 0)];
  auto xslot = [&](int sl) -> float* {
    return reinterpret_cast<float*>(ring + NSL * SLOT + 1024 + sl * 2048 * kTallWaves +
                                    2048 * (threadIdx.x >> 6));
  };
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  const int64_t ntiles = persist ? m / kTile : 0;
  int64_t tile = blk0 + blockIdx.x;
  // Q1 row l16 of this wave, columns 32 ch + 8 lg + e.  Chunk ch is loaded
  // with the staging of output panel 2 ch, the first that needs it (two
  // panels ahead), and split into its three bf16 planes just before that
  // panel; the loads overlap the earlier panels.  Ragged tiles load
  // registers, clamping the row and column: rows past m are never stored,
  // and columns past n meet zero rows of T.  In place: panel b overwrites
  // columns 16b..16b+15 of rows that this lane has already loaded.
  float xq[NCH][8];
  constexpr bool full = FULL;
  // Strides and the panel base laundered per tile (as in trsm_bf3_kernel).
  int64_t ldqv = ldq;
  const unsigned char* panv = pan3;
  // Whole tiles stage chunk ch in LDS by two direct loads per wave: load i,
  // lane L = 16 e' + 4 g + q brings rows 4q..4q+3 of column 32 ch + 8 g +
  // 4 i + e', so that the reads of element e (float 256 (e / 4) + 64 (e % 4)
  // + 16 lg + l16) fall in distinct banks.
  const int qcol = 8 * ((lane >> 2) & 3) + (lane >> 4);
  auto load_chunk = [&](int64_t t, int ch) {
    if (full) {
      const float* qt = Q + t * kTile + wave * 16 + 4 * (lane & 3);
#pragma unroll
      for (int i = 0; i < 2; ++i)
        dma16(qt + static_cast<int64_t>(32 * ch + 4 * i + qcol) * ldqv, xslot(ch % 2) + 256 * i);
    } else {
      const int64_t r = t * kTile + wave * 16 + l16;
      const float* qrow = Q + (r < m ? r : m - 1);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int col = 32 * ch + 8 * lg + e;
        xq[ch][e] = qrow[static_cast<int64_t>(col < n ? col : n - 1) * ldqv];
      }
    }
  };
  u4b_t qb[NCH][3];
  auto split_chunk = [&](int ch) {
    if (full) {
      const float* xl = xslot(ch % 2) + 16 * lg + l16;
#pragma unroll
      for (int e = 0; e < 8; ++e) xq[ch][e] = xl[256 * (e / 4) + 64 * (e % 4)];
    }
    uint32_t hp[8], dp[8], lp[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) split3(xq[ch][e], hp[e], dp[e], lp[e]);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      qb[ch][0][w] = __builtin_amdgcn_perm(hp[2 * w + 1], hp[2 * w], 0x07060302u);
      qb[ch][1][w] = __builtin_amdgcn_perm(dp[2 * w + 1], dp[2 * w], 0x07060302u);
      qb[ch][2][w] = __builtin_amdgcn_perm(lp[2 * w + 1], lp[2 * w], 0x07060302u);
    }
  };
  auto stage = [&](int b, int sl) {
    dma_panel(panv + bf3_panel_offset(b), trmm_bf3_psize(b), ring + SLOT * sl, ring + NSL * SLOT,
              wave, lane);
  };
  stage(0, 0);
  load_chunk(tile, 0);
  if (NB > 1) stage(1, 1);
  bool first = true;
  while (true) {
    asm volatile("" : "+s"(ldqv), "+s"(panv));
    const int64_t row = tile * kTile + wave * 16 + l16;
    const int64_t next = tile + gridDim.x;
    const bool has_next = persist && next < ntiles;
    static_for<NB>([&](auto bc) {
      constexpr int b = decltype(bc)::value;
      // Panel b (and, for even b, chunk b/2) has landed once the memory
      // operations issued after them are all that remain: 4 stores per
      // earlier panel, and per later panel its staging plus, for even
      // panels, the 2 loads of its chunk (see trsm_bf3_kernel).
      if (full) {
        constexpr bool staged = (b + 1 < NB) || persist;  // at panel b - 1
        constexpr int d1 = staged ? dma_per_wave(trmm_bf3_psize((b + 1) % NB)) +
                                        (((b + 1) % 2 == 0) ? 2 : 0)
                                  : 0;
        if (b >= 2) {
          wait_vmcnt<d1 + 8>();
        } else if (first) {
          wait_vmcnt<(b == 0) ? d1 : d1 + 4>();
        } else {
          wait_vmcnt<d1 + 8>();
        }
      } else {
        wait_vmcnt<0>();
      }
      wg_barrier();
      if (b + 2 < NB) {
        stage(b + 2, (b + 2) % NSL);
        if ((b & 1) == 0) load_chunk(tile, b / 2 + 1);
      } else if (persist) {
        stage(b + 2 - NB, (b + 2) % NSL);
        if ((b & 1) == 0) load_chunk(has_next ? next : tile, 0);
      }
      // Every staging load of this panel precedes its stores (wait counts).
      asm volatile("" ::: "memory");
      if ((b & 1) == 0) split_chunk(b / 2);
      const u4b_t* pa = reinterpret_cast<const u4b_t*>(ring + SLOT * (b % NSL)) + lane;
      // One chain per chunk (independent, so the matrix cores pipeline them),
      // each from zero; products grouped by T plane: d with d, h; l with h;
      // h with l, d, h.
      f4 c4[NCH];
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) c4[ch] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int tp = 1; tp < 4; ++tp) {
        const int tpl = tp % 3;  // planes in the order d, l, h
        bf8 tv[NCH];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
          if (ch <= b / 2) tv[ch] = __builtin_bit_cast(bf8, pa[(3 * ch + tpl) * 64]);
        const int nq = (tpl == 1) ? 2 : (tpl == 2 ? 1 : 3);
#pragma unroll
        for (int iq = 0; iq < 3; ++iq)
          if (iq < nq) {
            // d: (d, h)->planes 1, 0;  l: plane 0;  h: planes 2, 1, 0
            const int qp = (tpl == 1) ? (iq == 0 ? 1 : 0) : (tpl == 2 ? 0 : 2 - iq);
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
              if (ch <= b / 2)
                c4[ch] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    tv[ch], __builtin_bit_cast(bf8, qb[ch][qp]), c4[ch], 0, 0, 0);
          }
      }
      f4 D = c4[0];
#pragma unroll
      for (int ch = 1; ch < NCH; ++ch)
        if (ch <= b / 2) D += c4[ch];
      float* qout = Q + row;
      if (full) {
        float* qo = qout + static_cast<int64_t>(drow<float>(lg, 0)) * ldqv;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          qo[static_cast<int64_t>(16 * b + drow<float>(lg, v) - drow<float>(lg, 0)) * ldqv] = D[v];
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = 16 * b + drow<float>(lg, v);
          if (row < m && col < n) qout[static_cast<int64_t>(col) * ldqv] = D[v];
        }
      }
    });
    if (!has_next) break;
    tile = next;
    first = false;
  }
  // The last tile's two extra stagings must land before the workgroup's LDS
  // is released.
  if (persist) wait_vmcnt<0>();
}

// ----------------------------------------------------------------------------
// Q = X R^{-1} for FP32 X on bf16 matrix cores (the FP32 and mixed solves).
// Blocked forward substitution over 16-column subpanels: subpanel b first
// takes the update D = X_b - Q_{<b} R_{<b,b} (the same sums as the row-wise
// substitution, regrouped), then is multiplied by the inverse Tb of its
// 16 x 16 diagonal block (formed in FP64 by make_trsm_bf3_panels_kernel).
// Both products split their FP32 operands exactly into three bf16 parts and
// take the six significant products (as in trmm_bf3_kernel), so each is as
// accurate as an FP32 product.  Applying Tb costs a backward error of about
// u || |Tb| |Rbb| || |D| instead of substitution's u |Q_b| |Rbb| (Higham Thm
// 8.5, the bound Section 5.1 builds on); when the panels flag a block whose
// || |Tb| |Rbb| || is large, every block takes one refinement step, E += Tb^T
// (D - Rbb^T E), with the residual from the six significant products (FP32
// accurate) and the correction from the three leading ones: the backward
// error is then u |D| + O(u^2 || |Tb| |Rbb| ||^2) |D|, as for substitution
// while u cond(Rbb) << 1.  The transposed setup (panel columns x rows)
// makes the solved block, as the 16x16 matrix cores return it, directly the
// operand of the later updates: a wave keeps its 16 rows of Q split in
// registers (two subpanels per 32-wide chunk, in the column order the panels
// are packed in), so X is read once and Q written once, with no LDS round
// trip.  Subpanel b's operands are staged in LDS two subpanels ahead by
// direct global -> LDS loads.  Works in place (Q == X: a wave reads all of
// its rows before it writes).
typedef short s4b_t __attribute__((ext_vector_type(4)));

// Bytes of subpanel b of the solve's panels that are staged: (b+1)/2 chunks
// and the diagonal block's inverse, plus the block itself when refining.
__host__ __device__ constexpr int trsm_bf3_psize(int b, bool rf) {
  return ((b + 1) / 2) * 3072 + (rf ? 3072 : 1536);
}

// SK (the column-oriented update): subpanels 0..s0-1 are already solved and
// sit in Q; they are read from there as the operand of the later updates,
// neither solved again nor stored.  X then points at the first column of
// subpanel s0 (the new columns), and subpanel b >= s0 is read from its column
// 16 (b - s0).  Without SK, s0 is ignored and X holds all n columns.
//
// FULL: whole tiles of 16 kTallWaves rows below m, n = 16 NB, NB >= 4 (no
// bounds checks, so the wait counts are exact).  When NB % 4 == 0 the panel
// ring has four slots, a tile's panels fill whole ring cycles, and each
// workgroup loops over tiles blockIdx.x, + gridDim.x, ...: the next tile's
// first two panels (and X subpanels) are staged during the last two of the
// current one.  Otherwise a workgroup solves tile blk0 + blockIdx.x, with
// bounds checks unless FULL.
//
// The refinement is a separate instance (RF): both are launched, and the one
// that does not match the panels' flags returns at once, so that the plain
// instance keeps its registers.
template <int NB, bool FULL, bool RF, bool SK = false>
__global__ __launch_bounds__(64 * kTallWaves) void trsm_bf3_kernel(const float* X, int64_t m, int n,
                                                       int64_t ldx,
                                                       const unsigned char* __restrict__ pan3,
                                                       float* Q, int64_t ldq, int64_t blk0,
                                                       int s0 = 0) {
  constexpr int NCH = (NB + 1) / 2;
  constexpr int PMAX = trsm_bf3_psize(NB - 1, RF);
  constexpr int SLOT = dma_kib(PMAX) * 1024;
  constexpr bool persist = FULL && NB % 4 == 0;
  constexpr int NSL = persist ? 4 : 3;
  constexpr int64_t kTile = 16 * kTallWaves;
  // NSL panel slots (panel b in slot b % NSL, staged two panels ahead), a
  // sink, and (whole tiles) NSL X slots of 1 KiB per wave
  __shared__ __align__(1024) unsigned char ring[NSL * SLOT + 1024 + (FULL ? NSL * 1024 * kTallWaves : 0)];
  auto xslot = [&](int sl) -> float* {
    return reinterpret_cast<float*>(ring + NSL * SLOT + 1024 + sl * 1024 * kTallWaves +
                                    1024 * (threadIdx.x >> 6));
  };
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  const int64_t ntiles = persist ? m / kTile : 0;
  int64_t tile = blk0 + blockIdx.x;
  constexpr bool full = FULL;
  // X row of this lane at columns 16 b + 4 lg + v: the layout of the solved
  // values.  Subpanel b is loaded with the staging of its panel, two
  // subpanels ahead, so the loads overlap the earlier subpanels.  Whole
  // tiles stage it in LDS by one direct load per wave: lane L = 16 v + 4 g
  // + q brings rows 4q..4q+3 of column 16 b + 4 g + v, so that the reads
  // (float 64 v + 16 lg + l16) fall in distinct banks.  Ragged tiles load
  // registers, clamping row and column (rows past m are never stored;
  // columns past n meet zero panel entries).
  float xd[NB][4];
  // Strides and the panel base as loop-carried copies: laundered at the top
  // of every tile, so that the compiler recomputes the per-panel offsets
  // instead of holding all of them in registers across the tile loop.
  int64_t ldxv = ldx, ldqv = ldq;
  const unsigned char* panv = pan3;
  const int xcol = 4 * ((lane >> 2) & 3) + (lane >> 4);
  auto load_x = [&](int64_t t, int b, int sl) {
    // subpanel b's first column and stride (solved ones from Q under SK)
    const float* src = X + static_cast<int64_t>(16 * b) * ldxv;
    int64_t ld = ldxv;
    if constexpr (SK) {
      const bool solved = b < s0;
      ld = solved ? ldqv : ldxv;
      src = solved ? Q + static_cast<int64_t>(16 * b) * ldqv
                   : X + static_cast<int64_t>(16 * (b - s0)) * ldxv;
    }
    if (full) {
      dma16(src + t * kTile + wave * 16 + 4 * (lane & 3) + static_cast<int64_t>(xcol) * ld,
            xslot(sl));
    } else {
      const int64_t r = t * kTile + wave * 16 + l16;
      const float* xrow = src + (r < m ? r : m - 1);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = 4 * lg + v;
        xd[b][v] = xrow[static_cast<int64_t>(col < n - 16 * b ? col : n - 1 - 16 * b) * ld];
      }
    }
  };
  u4b_t qb[NCH][3];
  auto stage = [&](int b, int sl) {
    dma_panel(panv + trsm_bf3_panel_offset(b), trsm_bf3_psize(b, RF), ring + SLOT * sl,
              ring + NSL * SLOT, wave, lane);
  };
  // bf16 planes of four FP32 values, two per 32-bit word (element 0 low).
  auto split4 = [](const f4& x, uint32_t (&h)[2], uint32_t (&d)[2], uint32_t (&l)[2]) {
    uint32_t hp[4], dp[4], lp[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) split3(x[e], hp[e], dp[e], lp[e]);
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      h[w] = __builtin_amdgcn_perm(hp[2 * w + 1], hp[2 * w], 0x07060302u);
      d[w] = __builtin_amdgcn_perm(dp[2 * w + 1], dp[2 * w], 0x07060302u);
      l[w] = __builtin_amdgcn_perm(lp[2 * w + 1], lp[2 * w], 0x07060302u);
    }
  };
  auto as_s4 = [](const uint32_t (&w)[2]) {
    const uint2 u = make_uint2(w[0], w[1]);
    return __builtin_bit_cast(s4b_t, u);
  };
  // One refinement flag per subpanel: any set one refines every block.
  bool refine = false;
  {
    const int* fl = reinterpret_cast<const int*>(pan3 + trsm_bf3_flags_offset(n));
#pragma unroll
    for (int b = 0; b < NB; ++b) refine |= fl[b] != 0;
    refine = __builtin_amdgcn_readfirstlane(refine ? 1 : 0) != 0;
  }
  if (refine != RF) return;
  stage(0, 0);
  load_x(tile, 0, 0);
  if (NB > 1) {
    stage(1, 1);
    load_x(tile, 1, 1);
  }
  bool first = true;
  while (true) {
    asm volatile("" : "+s"(ldxv), "+s"(ldqv), "+s"(panv));
    const int64_t row = tile * kTile + wave * 16 + l16;
    const int64_t next = tile + gridDim.x;
    const bool has_next = persist && next < ntiles;
    static_for<NB>([&](auto bc) {
      constexpr int b = decltype(bc)::value;
      // Subpanel b's panel and X values have landed once the memory
      // operations issued after them are all that remain, in issue order:
      // 4 stores per earlier subpanel, and per later one its staging and
      // one X load (whole tiles only; a ragged tile may skip stores and
      // waits for everything).  Persistent workgroups stage two panels
      // past the end of every tile (the next tile's first two, or a
      // harmless repeat of this tile's on the last one).
      if (full) {
        constexpr bool staged = (b + 1 < NB) || persist;  // at subpanel b - 1
        constexpr int d1 = staged ? dma_per_wave(trsm_bf3_psize((b + 1) % NB, RF)) + 1 : 0;
        if (SK) {
          // Subpanels below s0 store nothing: count the store groups of the
          // two subpanels before b (of the previous tile, for b < 2 after
          // the first), or of subpanel 0 for b = 1 on the first tile.
          int ns;
          if (b >= 2 || !first)
            ns = static_cast<int>((b + NB - 2) % NB >= s0) + static_cast<int>((b + NB - 1) % NB >= s0);
          else
            ns = (b == 0) ? 0 : static_cast<int>(s0 == 0);
          ns = __builtin_amdgcn_readfirstlane(ns);
          if (ns == 2)
            wait_vmcnt<d1 + 8>();
          else if (ns == 1)
            wait_vmcnt<d1 + 4>();
          else
            wait_vmcnt<d1>();
        } else if (b >= 2) {
          wait_vmcnt<d1 + 8>();
        } else if (first) {
          wait_vmcnt<(b == 0) ? d1 : d1 + 4>();
        } else {
          wait_vmcnt<d1 + 8>();
        }
      } else {
        wait_vmcnt<0>();
      }
      wg_barrier();
      if (b + 2 < NB) {
        stage(b + 2, (b + 2) % NSL);
        load_x(tile, b + 2, (b + 2) % NSL);
      } else if (persist) {
        stage(b + 2 - NB, (b + 2) % NSL);
        load_x(has_next ? next : tile, b + 2 - NB, (b + 2) % NSL);
      }
      // The wait counts take every staging load of this subpanel to precede
      // its stores: keep the compiler from interleaving them.
      asm volatile("" ::: "memory");
      const int nc = (b + 1) / 2;
      const unsigned char* slot = ring + SLOT * (b % NSL);
      const u4b_t* pa = reinterpret_cast<const u4b_t*>(slot) + lane;
      if (full) {
        const float* xl = xslot(b % NSL) + 16 * lg + l16;
#pragma unroll
        for (int v = 0; v < 4; ++v) xd[b][v] = xl[64 * v];
      }
      f4 D = f4{xd[b][0], xd[b][1], xd[b][2], xd[b][3]};
      f4 E = D;  // a solved subpanel (SK, b < s0) as read
      if (!(SK && b < s0)) {
        if (nc > 0) {
          // One chain per chunk, each from zero; products grouped by R plane:
          // d with d, h; l with h; h with l, d, h.
          f4 c4[NCH];
#pragma unroll
          for (int p = 0; p < NCH; ++p) c4[p] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int tp = 1; tp < 4; ++tp) {
            const int tpl = tp % 3;  // planes in the order d, l, h
            bf8 tv[NCH];
#pragma unroll
            for (int p = 0; p < NCH; ++p)
              if (p < nc) tv[p] = __builtin_bit_cast(bf8, pa[(3 * p + tpl) * 64]);
            const int nq = (tpl == 1) ? 2 : (tpl == 2 ? 1 : 3);
#pragma unroll
            for (int iq = 0; iq < 3; ++iq)
              if (iq < nq) {
                const int qp = (tpl == 1) ? (iq == 0 ? 1 : 0) : (tpl == 2 ? 0 : 2 - iq);
#pragma unroll
                for (int p = 0; p < NCH; ++p)
                  if (p < nc)
                    c4[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        tv[p], __builtin_bit_cast(bf8, qb[p][qp]), c4[p], 0, 0, 0);
              }
          }
#pragma unroll
          for (int p = 0; p < NCH; ++p)
            if (p < nc) D += c4[p];
        }
        // Diagonal block: Q_b = Tb^T D on 16x16x16 matrix cores; D as returned
        // is the B operand (K = 4 lg + v).
        uint32_t dh[2], dd[2], dl[2];
        split4(D, dh, dd, dl);
        const uint2* pd = reinterpret_cast<const uint2*>(slot + 3072 * nc) + lane;
        const s4b_t th = __builtin_bit_cast(s4b_t, pd[0]);
        const s4b_t td = __builtin_bit_cast(s4b_t, pd[64]);
        const s4b_t tl = __builtin_bit_cast(s4b_t, pd[128]);
        E = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(td, as_s4(dd), f4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        E = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(tl, as_s4(dh), E, 0, 0, 0);
        E = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(th, as_s4(dl), E, 0, 0, 0);
        E = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(td, as_s4(dh), E, 0, 0, 0);
        E = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(th, as_s4(dd), E, 0, 0, 0);
        E = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(th, as_s4(dh), E, 0, 0, 0);
        if (RF) {
          // -Rbb^T E (smallest products first), then the residual and the
          // correction Tb^T r from its two leading planes.
          uint32_t fh[2], fd[2], fl[2];
          split4(E, fh, fd, fl);
          const s4b_t rh = __builtin_bit_cast(s4b_t, pd[192]);
          const s4b_t rd = __builtin_bit_cast(s4b_t, pd[256]);
          const s4b_t rl = __builtin_bit_cast(s4b_t, pd[320]);
          f4 F = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(rd, as_s4(fd), f4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
          F = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(rl, as_s4(fh), F, 0, 0, 0);
          F = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(rh, as_s4(fl), F, 0, 0, 0);
          F = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(rd, as_s4(fh), F, 0, 0, 0);
          F = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(rh, as_s4(fd), F, 0, 0, 0);
          F = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(rh, as_s4(fh), F, 0, 0, 0);
          const f4 res = D + F;
          uint32_t gh[2], gd[2], gl[2];
          split4(res, gh, gd, gl);
          f4 C = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(td, as_s4(gh), f4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
          C = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(th, as_s4(gd), C, 0, 0, 0);
          C = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(th, as_s4(gh), C, 0, 0, 0);
          E += C;
        }
        float* qout = Q + row;
        if (full) {
          float* qo = qout + static_cast<int64_t>(4 * lg) * ldqv;
#pragma unroll
          for (int v = 0; v < 4; ++v) qo[static_cast<int64_t>(16 * b + v) * ldqv] = E[v];
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int col = 16 * b + 4 * lg + v;
            if (row < m && col < n) qout[static_cast<int64_t>(col) * ldqv] = E[v];
          }
        }
      }
      // Keep Q_b split for the later updates: words 0-1 of chunk b/2 for even
      // b (words 2-3 zero until b + 1 is solved), words 2-3 for odd b.
      uint32_t eh[2], ed[2], el[2];
      split4(E, eh, ed, el);
      if ((b & 1) == 0) {
        qb[b / 2][0] = u4b_t{eh[0], eh[1], 0u, 0u};
        qb[b / 2][1] = u4b_t{ed[0], ed[1], 0u, 0u};
        qb[b / 2][2] = u4b_t{el[0], el[1], 0u, 0u};
      } else {
        qb[b / 2][0][2] = eh[0]; qb[b / 2][0][3] = eh[1];
        qb[b / 2][1][2] = ed[0]; qb[b / 2][1][3] = ed[1];
        qb[b / 2][2][2] = el[0]; qb[b / 2][2][3] = el[1];
      }
    });
    if (!has_next) break;
    tile = next;
    first = false;
  }
  // The last tile's two extra stagings must land before the workgroup's LDS
  // is released.
  if (persist) wait_vmcnt<0>();
}

hipError_t launch_trsm(const void* X, bool f32, int64_t m, int n, int64_t ldx, const void* pan,
                       void* Q, int64_t ldq, hipStream_t st) {
  if (m == 0) return hipSuccess;
  const int nb = static_cast<int>(ceil_div(n, 16));
  if (f32) {
    // pan holds bf16 x 3 subpanels (make_trsm_bf3_panels_kernel)
    // Whole tiles on the unchecked instance (which stages X by 16-byte
    // direct loads: X 16-byte aligned, ldx a multiple of 4), the ragged rest
    // (or every tile, when n is not a multiple of 16) on the checked one.
    // With nb % 4 == 0 the whole tiles are shared out to one persistent
    // workgroup per compute unit.
    const int64_t tiles = ceil_div(m, 16 * kTallWaves);
    const bool aligned = (ldx % 4) == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0;
    const int64_t nfull = (n % 16 == 0 && nb >= 4 && aligned) ? m / (16 * kTallWaves) : 0;
    const int64_t gfull = (nb % 4 == 0) ? std::min<int64_t>(nfull, device_cus()) : nfull;
    const float* x = static_cast<const float*>(X);
    float* q = static_cast<float*>(Q);
    const unsigned char* p3 = static_cast<const unsigned char*>(pan);
#define RCQ_S3_RF(NBV, RFV)                                                                \
  do {                                                                                     \
    if (nfull > 0)                                                                         \
      trsm_bf3_kernel<NBV, true, RFV><<<static_cast<unsigned>(gfull), 64 * kTallWaves, 0,  \
                                        st>>>(x, m, n, ldx, p3, q, ldq, 0);                \
    if (tiles > nfull)                                                                     \
      trsm_bf3_kernel<NBV, false, RFV><<<static_cast<unsigned>(tiles - nfull),             \
                                         64 * kTallWaves, 0, st>>>(x, m, n, ldx, p3, q,    \
                                                                   ldq, nfull);            \
  } while (0)
#define RCQ_S3_CASE(NBV)  \
  case NBV:               \
    RCQ_S3_RF(NBV, false); \
    RCQ_S3_RF(NBV, true);  \
    break;
    switch (nb) {
      RCQ_S3_CASE(1) RCQ_S3_CASE(2) RCQ_S3_CASE(3) RCQ_S3_CASE(4) RCQ_S3_CASE(5) RCQ_S3_CASE(6)
      RCQ_S3_CASE(7) RCQ_S3_CASE(8) RCQ_S3_CASE(9) RCQ_S3_CASE(10) RCQ_S3_CASE(11)
      RCQ_S3_CASE(12) RCQ_S3_CASE(13) RCQ_S3_CASE(14) RCQ_S3_CASE(15) RCQ_S3_CASE(16)
      default: return hipErrorInvalidValue;
    }
#undef RCQ_S3_CASE
#undef RCQ_S3_RF
    return hipGetLastError();
  }
  return trsm_dispatch<double>(nb, static_cast<const double*>(X), m, n, ldx,
                               static_cast<const double*>(pan), static_cast<double*>(Q), ldq, st);
}

hipError_t launch_trsm_append(const void* Xv, bool f32, int64_t m, int n, int64_t ldx,
                              const void* pan, void* Qv, int64_t ldq, int s0, hipStream_t st) {
  if (m == 0) return hipSuccess;
  const int nb = static_cast<int>(ceil_div(n, 16));
  if (s0 < 0 || s0 >= nb) return hipErrorInvalidValue;
  if (!f32) {
    const unsigned grid = static_cast<unsigned>(ceil_div(m, 64 * RowBlocks<double>::value));
    const double* X = static_cast<const double*>(Xv);
    const double* pd = static_cast<const double*>(pan);
    double* Q = static_cast<double*>(Qv);
#define RCQ_SD_CASE(NBV)                                                                     \
  case NBV:                                                                                  \
    trsm_kernel<double, NBV, true><<<grid, 256, 0, st>>>(X, m, n, ldx, pd, Q, ldq, s0);      \
    break;
    switch (nb) {
      RCQ_SD_CASE(1) RCQ_SD_CASE(2) RCQ_SD_CASE(3) RCQ_SD_CASE(4) RCQ_SD_CASE(5) RCQ_SD_CASE(6)
      RCQ_SD_CASE(7) RCQ_SD_CASE(8) RCQ_SD_CASE(9) RCQ_SD_CASE(10) RCQ_SD_CASE(11)
      RCQ_SD_CASE(12) RCQ_SD_CASE(13) RCQ_SD_CASE(14) RCQ_SD_CASE(15) RCQ_SD_CASE(16)
      default: return hipErrorInvalidValue;
    }
#undef RCQ_SD_CASE
    return hipGetLastError();
  }
  const float* X = static_cast<const float*>(Xv);
  float* Q = static_cast<float*>(Qv);
  // As launch_trsm's FP32 branch; the whole-tile instance also stages the
  // solved subpanels from Q by 16-byte direct loads.
  const int64_t tiles = ceil_div(m, 16 * kTallWaves);
  const bool aligned = (ldx % 4) == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0 &&
                       (ldq % 4) == 0 && (reinterpret_cast<uintptr_t>(Q) & 15) == 0;
  const int64_t nfull = (n % 16 == 0 && nb >= 4 && aligned) ? m / (16 * kTallWaves) : 0;
  const int64_t gfull = (nb % 4 == 0) ? std::min<int64_t>(nfull, device_cus()) : nfull;
  const unsigned char* p3 = static_cast<const unsigned char*>(pan);
#define RCQ_SA_RF(NBV, RFV)                                                                  \
  do {                                                                                       \
    if (nfull > 0)                                                                           \
      trsm_bf3_kernel<NBV, true, RFV, true><<<static_cast<unsigned>(gfull), 64 * kTallWaves, \
                                              0, st>>>(X, m, n, ldx, p3, Q, ldq, 0, s0);     \
    if (tiles > nfull)                                                                       \
      trsm_bf3_kernel<NBV, false, RFV, true><<<static_cast<unsigned>(tiles - nfull),         \
                                               64 * kTallWaves, 0, st>>>(X, m, n, ldx, p3,   \
                                                                         Q, ldq, nfull, s0); \
  } while (0)
#define RCQ_SA_CASE(NBV)   \
  case NBV:                \
    RCQ_SA_RF(NBV, false); \
    RCQ_SA_RF(NBV, true);  \
    break;
  switch (nb) {
    RCQ_SA_CASE(1) RCQ_SA_CASE(2) RCQ_SA_CASE(3) RCQ_SA_CASE(4) RCQ_SA_CASE(5) RCQ_SA_CASE(6)
    RCQ_SA_CASE(7) RCQ_SA_CASE(8) RCQ_SA_CASE(9) RCQ_SA_CASE(10) RCQ_SA_CASE(11)
    RCQ_SA_CASE(12) RCQ_SA_CASE(13) RCQ_SA_CASE(14) RCQ_SA_CASE(15) RCQ_SA_CASE(16)
    default: return hipErrorInvalidValue;
  }
#undef RCQ_SA_CASE
#undef RCQ_SA_RF
  return hipGetLastError();
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
  if (f32) {
    // pan holds bf16 x 3 panels (make_bf3_panels)
    // Whole tiles on the unchecked instance (n a multiple of 32, n >= 64; Q
    // staged by 16-byte direct loads: 16-byte aligned, ldq a multiple of 4;
    // one persistent workgroup per compute unit when nb % 4 == 0), the rest
    // on the checked one.
    const int64_t tiles = ceil_div(m, 16 * kTallWaves);
    const bool aligned = (ldq % 4) == 0 && (reinterpret_cast<uintptr_t>(Q) & 15) == 0;
    const int64_t nfull = (n % 32 == 0 && nb >= 4 && aligned) ? m / (16 * kTallWaves) : 0;
    const int64_t gfull = (nb % 4 == 0) ? std::min<int64_t>(nfull, device_cus()) : nfull;
    float* q = static_cast<float*>(Q);
    const unsigned char* p3 = static_cast<const unsigned char*>(pan);
#define RCQ_T3_CASE(NBV)                                                                   \
  case NBV:                                                                                \
    if (nfull > 0)                                                                         \
      trmm_bf3_kernel<NBV, true><<<static_cast<unsigned>(gfull), 64 * kTallWaves, 0, st>>>( \
          q, m, n, ldq, p3, 0);                                                            \
    if (tiles > nfull)                                                                     \
      trmm_bf3_kernel<NBV, false><<<static_cast<unsigned>(tiles - nfull), 64 * kTallWaves, \
                                    0, st>>>(q, m, n, ldq, p3, nfull);                     \
    break;
    switch (nb) {
      RCQ_T3_CASE(1) RCQ_T3_CASE(2) RCQ_T3_CASE(3) RCQ_T3_CASE(4) RCQ_T3_CASE(5) RCQ_T3_CASE(6)
      RCQ_T3_CASE(7) RCQ_T3_CASE(8) RCQ_T3_CASE(9) RCQ_T3_CASE(10) RCQ_T3_CASE(11)
      RCQ_T3_CASE(12) RCQ_T3_CASE(13) RCQ_T3_CASE(14) RCQ_T3_CASE(15) RCQ_T3_CASE(16)
      default: return hipErrorInvalidValue;
    }
#undef RCQ_T3_CASE
    return hipGetLastError();
  }
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
    const T* __restrict__ Q, int64_t m, int n, int64_t ldq, int64_t rows_per_split, int npg,
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
  double* dst = gpart + static_cast<int64_t>(s) * npg * npg;
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
  const int64_t lane_off = (64 * bi + drow<T>(lg, 0)) + static_cast<int64_t>(64 * bj + l16) * npg;
#define RCQ_GRAM_FLUSH()                                                        \
  do {                                                                          \
    int64_t lo = lane_off;                                                      \
    asm volatile("" : "+v"(lo));                                                \
    double* base = dst + lo;                                                    \
    _Pragma("unroll") for (int a = 0; a < 4; ++a)                               \
    _Pragma("unroll") for (int b = 0; b < 4; ++b)                               \
    _Pragma("unroll") for (int v = 0; v < 4; ++v) {                             \
      double* p = base + (16 * a + (drow<T>(lg, v) - drow<T>(lg, 0))) +         \
                  static_cast<int64_t>(16 * b) * npg;                           \
      const double val = static_cast<double>(acc[a][b][v]);                     \
      *p = first ? val : *p + val;                                              \
      acc[a][b][v] = T(0);                                                      \
      if (v == 3 && b == 3) __builtin_amdgcn_sched_barrier(0);                  \
    }                                                                           \
    first = false;                                                              \
  } while (0)
  // Register prefetch of the next stage (kGrRows x NP values over NW*64
  // threads): its loads overlap this stage's products.  FP64 with ten
  // waves (three per SIMD) has no registers to spare and stages directly.
  constexpr bool kPre = !CROSS && (sizeof(T) == 4 || NBB <= 3);
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
// ----------------------------------------------------------------------------
// Gram A = Q^T Q for FP32 Q on bf16 matrix cores.  Every FP32 entry splits
// exactly into three bf16 parts (split3), and
//   q q' ~ h h' + h d' + d h' + h l' + l h' + d d'
// drops only terms below 2^-24 |q q'| (d l', l d', l l'), so each product is
// as accurate as an FP32 product; the six bf16 products of a pair cost less
// than one FP32 matrix-core product.  The matrix cores sum one 32-row step
// from zero (a long accumulation inside the bf16 matrix-core instruction
// drifts: ||Q^T Q - I|| ~ 1e-5 was measured at 4e6 rows), and each step's
// FP32 result is added into FP64 accumulators held in registers.  A row
// split's sums therefore carry one FP32 rounding per step relative to that
// step's own terms: a column whose norm sits in a few rows (one large entry)
// loses nothing to the later, smaller steps, as it would in an FP32 running
// sum.  The partial is written once, at the end of the split.
//
// One workgroup owns one set of rows and the whole upper triangle of 16 x 16
// sub-tiles.  With NB = n / 16 column blocks, wave w owns the pair of row
// blocks w and NB - 1 - w: sub-tiles (w, c) for c >= w and (NB - 1 - w, c)
// for c >= NB - 1 - w, NB + 1 of them for every wave (17 FP64 accumulators,
// 136 registers, for n = 256 in 8 waves: two waves per SIMD, so nothing
// spills), every column block read once per wave for both rows.  Each row of
// Q is fetched and split exactly once.  Stages of 32 rows are double
// buffered in LDS as three bf16 planes laid out as the matrix-core operands:
// 16-byte chunks (8 rows of one column), chunk-major with a row of chunks per
// 8 rows; the operand reads (16 consecutive columns per lane group) and the
// split's writes (16 consecutive columns per 16 lanes) are free of bank
// conflicts.  The next stage's loads are issued before the current stage's
// products.
template <int NB64>
struct PairGram {
  static constexpr int kNB = 4 * NB64;            // 16-column blocks
  static constexpr int kWaves = kNB / 2;          // one pair of row blocks each
  static constexpr int kAcc = kNB + 1;            // sub-tiles per wave
  static constexpr int kCols = 64 * NB64;
  // Chunk row stride (16-byte units): a multiple of 16 chunks, so that an
  // operand read (16 consecutive chunks per lane group, the four groups a
  // stride apart) is free of bank conflicts on gfx950 (a stride of 2 mod 16
  // costs 4 extra cycles per read, measured).
  static constexpr int kStr = kCols;
  static constexpr int kBuf = 3 * 4 * kStr;       // chunks per stage buffer
  static constexpr int kTasks = 4 * kCols;        // 8-row pieces per stage
  static constexpr int kPer = kTasks / (64 * kWaves);
  static_assert(kPer * 64 * kWaves == kTasks, "whole tasks per thread");
  static constexpr size_t kLds = 2 * kBuf * 16;
};

// Sub-tile t of the wave that owns row blocks W and NB - 1 - W: the row block
// and the column block.
template <int NB, int W>
__device__ __forceinline__ constexpr int pg_row(int t) {
  return t < NB - W ? W : NB - 1 - W;
}
template <int NB, int W>
__device__ __forceinline__ constexpr int pg_col(int t) {
  return t < NB - W ? W + t : (NB - 1 - W) + (t - (NB - W));
}

template <int NB64>
__global__ __launch_bounds__(64 * PairGram<NB64>::kWaves) void gram_bf3_kernel(
    const float* __restrict__ Q, int64_t m, int n, int64_t ldq, int64_t rows_per_split, int npg,
    double* __restrict__ gpart) {
  typedef PairGram<NB64> G;
  constexpr int NB = G::kNB;
  extern __shared__ __align__(16) u4v_t qs3[];
  const int s = blockIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  // Workgroup s takes the 32-row stages s, s + G, s + 2G, ... (G = the
  // grid): at any time the workgroups read one contiguous band of rows.  Its
  // partial sums these stages in that order.
  (void)rows_per_split;
  const int64_t nstage = (m + kG3Rows - 1) / kG3Rows;
  const int64_t sstep = gridDim.x;
  const int64_t r_end = m;
  double* dst = gpart + static_cast<int64_t>(s) * npg * npg;

  d4 acc[G::kAcc];
#pragma unroll
  for (int i = 0; i < G::kAcc; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
  // The empty asm pins each sum to its place in the instruction stream:
  // otherwise the FP64 adds of a stage sink below all of its products, and
  // every chain's FP32 result stays live until then.
  auto add_step = [](d4& a, const f4& c) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double x = a[v] + static_cast<double>(c[v]);
      asm volatile("" : "+v"(x));
      a[v] = x;
    }
  };

  // Loads: task t = (column 16 (t / 64) + t % 16, rows 8 ((t / 16) % 4) ..),
  // kPer tasks per thread: lane groups of 16 write 16 consecutive chunks.
  // Columns past n read column n - 1 and are zeroed, so that only the last
  // stage (rows past m) takes the element-wise path: no divergent branches.
  float pre[G::kPer][8];
  const bool vec = ((ldq & 3) == 0) && ((reinterpret_cast<uintptr_t>(Q) & 15) == 0);
  const float* colp[G::kPer];  // first row of the task's 8 in row 0's stage
  bool liveq[G::kPer];
#pragma unroll
  for (int q = 0; q < G::kPer; ++q) {
    const int t = threadIdx.x + 64 * G::kWaves * q;
    const int c = 16 * (t >> 6) + (t & 15), g = (t >> 4) & 3;
    liveq[q] = c < n;
    colp[q] = Q + static_cast<int64_t>(c < n ? c : n - 1) * ldq + 8 * g;
  }
  auto fetch = [&](int64_t r0) {
    const int64_t rem = r_end - r0;  // rows left from r0 (>= 1)
    if (vec && rem >= kG3Rows) {
#pragma unroll
      for (int q = 0; q < G::kPer; ++q) {
        const float4 f0 = reinterpret_cast<const float4*>(colp[q] + r0)[0];
        const float4 f1 = reinterpret_cast<const float4*>(colp[q] + r0)[1];
        pre[q][0] = f0.x; pre[q][1] = f0.y; pre[q][2] = f0.z; pre[q][3] = f0.w;
        pre[q][4] = f1.x; pre[q][5] = f1.y; pre[q][6] = f1.z; pre[q][7] = f1.w;
      }
    } else {
      // the last stage (or unaligned Q): rows clamped to m - 1, then zeroed
      const int lim = static_cast<int>(rem < kG3Rows ? rem : kG3Rows);
#pragma unroll
      for (int q = 0; q < G::kPer; ++q) {
        const int t = threadIdx.x + 64 * G::kWaves * q;
        const int g8 = 8 * ((t >> 4) & 3);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int o = g8 + e < lim ? e : lim - 1 - g8;
          const float v = colp[q][r0 + o];
          pre[q][e] = g8 + e < lim ? v : 0.f;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < G::kPer; ++q)
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (!liveq[q]) pre[q][e] = 0.f;
  };
  auto stage_in = [&](u4v_t* buf) {
#pragma unroll
    for (int q = 0; q < G::kPer; ++q) {
      const int t = threadIdx.x + 64 * G::kWaves * q;
      const int c = 16 * (t >> 6) + (t & 15), g = (t >> 4) & 3;
      uint32_t hp[8], dp[8], lp[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) split3(pre[q][e], hp[e], dp[e], lp[e]);
      u4v_t hv, dv, lv;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        hv[w] = __builtin_amdgcn_perm(hp[2 * w + 1], hp[2 * w], 0x07060302u);
        dv[w] = __builtin_amdgcn_perm(dp[2 * w + 1], dp[2 * w], 0x07060302u);
        lv[w] = __builtin_amdgcn_perm(lp[2 * w + 1], lp[2 * w], 0x07060302u);
      }
      buf[(0 * 4 + g) * G::kStr + c] = hv;
      buf[(1 * 4 + g) * G::kStr + c] = dv;
      buf[(2 * 4 + g) * G::kStr + c] = lv;
    }
  };
  // Operands of the 16 columns starting at c0: lane (l16, lg) holds rows
  // 8 lg .. 8 lg + 7 of column c0 + l16, in each plane.
  auto opnd = [&](const u4v_t* buf, int p, int c0) {
    return __builtin_bit_cast(bf8, buf[(p * 4 + lg) * G::kStr + c0 + l16]);
  };
  // Six significant bf16 products of a sub-tile, from zero, smallest first.
  auto prod6 = [](const bf8& ah, const bf8& ad, const bf8& al, const bf8& bh, const bf8& bd,
                  const bf8& bl) {
    f4 c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ad, bd, f4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ad, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bd, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
  };
  // One wave's stages, its pair of row blocks a compile-time fact (the
  // accumulators stay in registers).
  auto run = [&](auto wc) {
    constexpr int W = decltype(wc)::value;
    constexpr int R0 = W, R1 = NB - 1 - W;
    int cur = 0;
    for (int64_t j = s; j < nstage; j += sstep) {
      const bool more = j + sstep < nstage;
      if (more) fetch((j + sstep) * kG3Rows);
      const u4v_t* buf = qs3 + cur * G::kBuf;
      const bf8 a0h = opnd(buf, 0, 16 * R0), a0d = opnd(buf, 1, 16 * R0), a0l = opnd(buf, 2, 16 * R0);
      const bf8 a1h = opnd(buf, 0, 16 * R1), a1d = opnd(buf, 1, 16 * R1), a1l = opnd(buf, 2, 16 * R1);
      static_for<NB - R0>([&](auto cc) {
        constexpr int c = R0 + decltype(cc)::value;
        // one column block in flight (bounds the live operand registers)
        __builtin_amdgcn_sched_barrier(0);
        const bf8 bh = c == R0 ? a0h : (c == R1 ? a1h : opnd(buf, 0, 16 * c));
        const bf8 bd = c == R0 ? a0d : (c == R1 ? a1d : opnd(buf, 1, 16 * c));
        const bf8 bl = c == R0 ? a0l : (c == R1 ? a1l : opnd(buf, 2, 16 * c));
        add_step(acc[c - R0], prod6(a0h, a0d, a0l, bh, bd, bl));
        if constexpr (c >= R1) add_step(acc[(NB - W) + (c - R1)], prod6(a1h, a1d, a1l, bh, bd, bl));
      });
      if (more) stage_in(qs3 + (cur ^ 1) * G::kBuf);
      __syncthreads();
      cur ^= 1;
    }
    // The split's partial: sub-tile t at rows 16 pg_row(t) + 4 lg + v,
    // column 16 pg_col(t) + l16.
    static_for<G::kAcc>([&](auto tc) {
      constexpr int t = decltype(tc)::value;
      double* base = dst + (16 * pg_row<NB, W>(t) + drow<float>(lg, 0)) +
                     static_cast<int64_t>(16 * pg_col<NB, W>(t) + l16) * npg;
#pragma unroll
      for (int v = 0; v < 4; ++v) base[drow<float>(lg, v) - drow<float>(lg, 0)] = acc[t][v];
    });
  };
  if (s < nstage) {
    fetch(static_cast<int64_t>(s) * kG3Rows);
    stage_in(qs3);
  }
  __syncthreads();
  static_for<G::kWaves>([&](auto wc) {
    if (wave == decltype(wc)::value) run(wc);
  });
}

template <typename T, bool CROSS>
static hipError_t gram_dispatch(const T* Q, int64_t m, int n, int64_t ldq, const GramPlan& gp,
                                double* gpart, const T* B, int64_t ldb, hipStream_t st) {
  const unsigned grid = static_cast<unsigned>(gp.nsplit);
  auto nw = [](int b) { return CROSS ? b * b : b * (b + 1) / 2; };
  switch (gp.nbb) {
    case 1: gram_kernel<T, 1, CROSS><<<grid, 64 * nw(1), 0, st>>>(Q, m, n, ldq, gp.rows_per_split, gp.npg, gpart, B, ldb); break;
    case 2: gram_kernel<T, 2, CROSS><<<grid, 64 * nw(2), 0, st>>>(Q, m, n, ldq, gp.rows_per_split, gp.npg, gpart, B, ldb); break;
    case 3: gram_kernel<T, 3, CROSS><<<grid, 64 * nw(3), 0, st>>>(Q, m, n, ldq, gp.rows_per_split, gp.npg, gpart, B, ldb); break;
    case 4: gram_kernel<T, 4, CROSS><<<grid, 64 * nw(4), 0, st>>>(Q, m, n, ldq, gp.rows_per_split, gp.npg, gpart, B, ldb); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gram(const void* Q, bool f32, int64_t m, int n, int64_t ldq, const GramPlan& gp,
                       double* gpart, hipStream_t st) {
  if (f32) {
    const int nb64 = static_cast<int>(ceil_div(n, 64));
    if (gp.npg < 64 * nb64) return hipErrorInvalidValue;
    const float* Qf = static_cast<const float*>(Q);
#define RCQ_G3_CASE(NB)                                                                      \
  case NB: {                                                                                 \
    const hipError_t e = hipFuncSetAttribute(                                                \
        reinterpret_cast<const void*>(&gram_bf3_kernel<NB>),                                 \
        hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(PairGram<NB>::kLds));   \
    if (e != hipSuccess) return e;                                                           \
    gram_bf3_kernel<NB><<<gp.nsplit, 64 * PairGram<NB>::kWaves, PairGram<NB>::kLds, st>>>(  \
        Qf, m, n, ldq, gp.rows_per_split, gp.npg, gpart);                                    \
    break;                                                                                   \
  }
    switch (nb64) {
      RCQ_G3_CASE(1) RCQ_G3_CASE(2) RCQ_G3_CASE(3) RCQ_G3_CASE(4)
      default: return hipErrorInvalidValue;
    }
#undef RCQ_G3_CASE
    return hipGetLastError();
  }
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
