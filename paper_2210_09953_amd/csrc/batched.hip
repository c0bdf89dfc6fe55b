// batched.hip -- persistent batched RCholeskyQR: one launch factors many
// independent tall-skinny problems (for example the panels of a block Krylov
// method, Section 3.2), each by Algorithm 2 or 3 with a Rademacher sketch.
//
// Work is a queue of tasks in phase-major order:
//   A  sketch chunk   (instance i, row chunk c, 64 Theta rows g): P_c
//   B  small QR       (instance i): P = sum_c P_c / sqrt(k), Householder,
//                      sign fix, R_s, solve panels
//   C  solve chunk    (instance i, row chunk c): Q1 = X R_s^{-1} on the
//                      chunk's rows, then (2 passes) G_c = Q1_c^T Q1_c
//   D  Cholesky       (instance i): G = sum_c G_c, R' = chol(G), R = R' R_s,
//                      T = R'^{-1}, product panels
//   E  product chunk  (instance i, row chunk c): Q = Q1 T
// A persistent workgroup takes the next task from an atomic counter, waits
// (bounded spin) until the instance's previous phase has completed, runs the
// task and counts it done with an agent-scope release.  A task only waits on
// tasks earlier in the queue, each held by a running workgroup that waits on
// nothing later, so the queue drains whatever the grid size.  A spin that
// exceeds its bound sets the engine's error word and every workgroup exits
// normally.
//
// Arithmetic: Theta is the Rademacher operator of theta.h (bit for bit the
// one of the single-problem path); X (FP32) is split exactly into three bf16
// planes, so each product with the +-1 entries is exact; 32-row steps are
// summed from zero on bf16 matrix cores in FP32 and added into FP64.  The
// small QR (FP64 Householder as LAPACK's xGEQR2, sign-fixed) and the
// Cholesky (FP64, upper) run in one workgroup per instance; the tall solve
// and product are the generic FP32 matrix-core blocks of tall.hip
// (trsm_block: blocked forward substitution with true division on the
// diagonal blocks); the Gram takes exact FP32 matrix-core products per
// 32-row step, summed into FP64.
#include <math.h>
#include <stddef.h>

#include <type_traits>

#include "../../include/rcholqr.h"
#include "common.h"
#include "kernels.h"
#include "tallblock.h"
#include "theta.h"

namespace rcq {

typedef unsigned int u4v_t __attribute__((ext_vector_type(4)));

constexpr int kBThreads = 256;
constexpr int kMaxKB = 384;      // largest k the engine takes
// X and Q are addressed with 32-bit byte offsets (buffer instructions):
// each holds at most 2^30 elements (4 GiB) with its leading dimension.
constexpr int64_t kBMaxElems = int64_t{1} << 30;

// Device layout of one instance's scratch (byte offsets from its region).
struct BLayout {
  int64_t Pp, P, Rs, pan, Gp, G, T, pan2, total;
  int nchunk, nb;  // row chunks; 16-column blocks
  int nh;          // sketch tasks per 16-column block: halves of the Theta rows
};

// Row tiles of Theta (16 rows each) per sketch task: at most 12 (the FP32
// accumulators of a wave); k > 192 is split into two halves.
constexpr int kBSketchTiles = 12;
constexpr int kBXtLd = 128 + 4;  // row stride (floats) of a wave's X tile in LDS

__host__ __device__ inline int64_t b_align(int64_t x) { return (x + 255) & ~int64_t{255}; }

__host__ __device__ inline BLayout b_layout(int64_t m, int n, int k, int passes, int64_t chunk) {
  BLayout L{};
  L.nb = n / 16;
  L.nchunk = static_cast<int>((m + chunk - 1) / chunk);
  L.nh = (k / 16 + kBSketchTiles - 1) / kBSketchTiles;
  const int64_t kpad = k;  // P_c partials: k x n, column-major
  const int64_t pe = 256 * static_cast<int64_t>(L.nb) * (L.nb + 1) / 2;  // panel elements
  int64_t off = 0;
  L.Pp = off; off += b_align(L.nchunk * kpad * n * 8);
  L.P = off; off += b_align(static_cast<int64_t>(k) * n * 8);
  L.Rs = off; off += b_align(static_cast<int64_t>(n) * n * 8);
  L.pan = off; off += b_align(pe * 4);
  if (passes == 2) {
    L.Gp = off; off += b_align(L.nchunk * static_cast<int64_t>(n) * n * 8);
    L.G = off; off += b_align(static_cast<int64_t>(n) * n * 8);
    L.T = off; off += b_align(static_cast<int64_t>(n) * n * 8);
    L.pan2 = off; off += b_align(pe * 4);
  }
  L.total = off;
  return L;
}

// Problem checks of the batched engine (0 = usable).
__host__ __device__ inline bool b_valid(const rcholqr_problem& p) {
  return p.X && p.Q && p.R && p.n >= 16 && p.n <= 128 && p.n % 16 == 0 && p.k % 16 == 0 &&
         p.k >= p.n && p.k <= kMaxKB && p.m >= p.n && p.ldx >= p.m && p.ldq >= p.m && p.ldr >= p.n &&
         p.ldx * p.n <= kBMaxElems && p.ldq * p.n <= kBMaxElems;
}

struct BInst {
  const float* X;
  float* Q;
  double* R;
  int64_t m, ldx, ldq, ldr;
  uint64_t seed;
  int n, k;
  BLayout L;
  int64_t base;            // byte offset of the instance's region in the workspace
  int64_t tA, tC;          // first task of the instance in phases A and C/E
};

struct BHeader {
  int counter;       // next task
  int error;         // 0; bit 0: a wait exceeded its bound; 2: workspace too small
  int batch, passes;
  int64_t chunk;     // rows per chunk
  int64_t nA, nC;    // tasks in phase A, and in each of phases C and E
  int64_t total_bytes;
  // the first wait that exceeded its bound: instance, phase, count seen,
  // count needed (diagnostics for the status call)
  int stall_inst, stall_phase, stall_seen, stall_need;
};

// Workspace: header | done[batch][8] | status[batch] | inst[batch] | regions
__host__ __device__ inline int64_t b_done_off() { return 256; }
__host__ __device__ inline int64_t b_status_off(int batch) {
  return b_align(b_done_off() + 32ll * batch);
}
__host__ __device__ inline int64_t b_inst_off(int batch) {
  return b_align(b_status_off(batch) + 4ll * batch);
}
__host__ __device__ inline int64_t b_region_off(int batch) {
  return b_align(b_inst_off(batch) + static_cast<int64_t>(sizeof(BInst)) * batch);
}

// ---------------------------------------------------------------------------
// Setup: per-instance layouts, task offsets, counters (no memset: the kernel
// writes every word the engine reads).
__global__ __launch_bounds__(kBThreads) void batched_setup_kernel(
    const rcholqr_problem* __restrict__ probs, int batch, int passes, int64_t chunk,
    unsigned char* __restrict__ ws, int64_t ws_bytes) {
  BHeader* h = reinterpret_cast<BHeader*>(ws);
  int* done = reinterpret_cast<int*>(ws + b_done_off());
  int* status = reinterpret_cast<int*>(ws + b_status_off(batch));
  BInst* inst = reinterpret_cast<BInst*>(ws + b_inst_off(batch));
  for (int i = threadIdx.x; i < 8 * batch; i += blockDim.x) done[i] = 0;
  if (threadIdx.x == 0) {
    int64_t off = b_region_off(batch), tA = 0, tC = 0;
    for (int i = 0; i < batch; ++i) {
      const rcholqr_problem p = probs[i];
      BInst b{};
      b.X = static_cast<const float*>(p.X);
      b.Q = static_cast<float*>(p.Q);
      b.R = p.R;
      b.m = p.m;
      b.ldx = p.ldx;
      b.ldq = p.ldq;
      b.ldr = p.ldr;
      b.seed = p.seed;
      b.n = static_cast<int>(p.n);
      b.k = static_cast<int>(p.k);
      const bool ok = b_valid(p);
      status[i] = ok ? 0 : RCHOLQR_BATCH_INVALID;
      if (ok) {
        b.L = b_layout(p.m, b.n, b.k, passes, chunk);
      } else {
        b.L = BLayout{};
      }
      b.base = off;
      b.tA = tA;
      b.tC = tC;
      off += b.L.total;
      tA += static_cast<int64_t>(b.L.nchunk) * b.L.nb * b.L.nh;
      tC += b.L.nchunk;
      inst[i] = b;
    }
    h->counter = 0;
    h->error = (off > ws_bytes) ? 2 : 0;
    h->stall_inst = -1;
    h->stall_phase = -1;
    h->stall_seen = 0;
    h->stall_need = 0;
    h->batch = batch;
    h->passes = passes;
    h->chunk = chunk;
    h->nA = tA;
    h->nC = tC;
    h->total_bytes = off;
    if (off > ws_bytes)
      for (int i = 0; i < batch; ++i) status[i] = RCHOLQR_BATCH_INVALID;
  }
}

// Instance whose task range [first(i), first(i+1)) holds task u (binary
// search over the per-instance offsets, which are nondecreasing).
// The table is read through the constant address space: it is written by
// the setup kernel only, so the persistent kernel may read it with scalar
// loads (scalar cache) instead of a chain of vector loads.
#define RCQ_K __attribute__((address_space(4)))
template <bool PHASE_A>
__device__ inline int b_find(const BInst* inst, int batch, int64_t u) {
  const RCQ_K BInst* kinst = (const RCQ_K BInst*)(inst);
  int lo = 0, hi = batch - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int64_t f = PHASE_A ? kinst[mid].tA : kinst[mid].tC;
    if (f <= u) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Sum of v over the workgroup (all threads get it); red holds 4 doubles.
__device__ inline double b_block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// v as lane 0 of the wave holds it, in scalar registers (for values that
// every lane loaded from the same address and that steer a loop with
// barriers: the branch is then visibly uniform).
__device__ inline double b_uniform(double v) {
  const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(v));
  const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(u));
  const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(u >> 32));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

__device__ inline int64_t b_uniform(int64_t v) {
  const unsigned long long u = static_cast<unsigned long long>(v);
  const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(u));
  const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(u >> 32));
  return static_cast<int64_t>((static_cast<unsigned long long>(hi) << 32) | lo);
}
__device__ inline int b_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// The task bodies are separate functions, so the pointers they get (from
// the problem table and the workspace) have no known address space and
// would be accessed with flat instructions, which also count against the
// LDS counter: every LDS wait would then wait for the rows loaded ahead.
// gp() states that they point to global memory.
#define RCQ_G __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ RCQ_G T* gp(T* p) {
  return (RCQ_G T*)(p);
}

// Row range [r_begin, r_end) of chunk c, in scalar registers.
__device__ inline void b_chunk_rows(const BInst& b, int c, const unsigned char* ws, int64_t& r_begin,
                                    int64_t& r_end) {
  const int64_t chunk = b_uniform(gp(reinterpret_cast<const BHeader*>(ws))->chunk);
  const int64_t m = b_uniform(gp(&b)->m);
  r_begin = static_cast<int64_t>(c) * chunk;
  r_end = (r_begin + chunk < m) ? r_begin + chunk : m;
}


// Addressing of a 16-row block of a column-major FP32 matrix with buffer
// instructions: a descriptor for the whole matrix (scalar registers), the
// lane's byte offset (row + 4 lg ld) 4 in one 32-bit register, and the
// column's byte offset c ld 4 as the scalar offset.  A lane whose row is
// past m loads row m - 1 instead (a select on the loaded value would make
// the compiler wait for each load where it is issued); such rows are never
// stored, and the Gram zeroes them when it stages them.
struct BMat {
  __amdgpu_buffer_rsrc_t r;
  int ld4;  // leading dimension in bytes
};
__device__ __forceinline__ BMat b_mat(const float* p, int64_t ld, int64_t n) {
  // the base and size in scalar registers (a descriptor the compiler cannot
  // prove uniform is rebuilt around every access); dword 3: 32-bit data
  // format, as the gfx9 family's raw buffers take it
  float* base = reinterpret_cast<float*>(b_uniform(reinterpret_cast<int64_t>(p)));
  const int bytes = __builtin_amdgcn_readfirstlane(static_cast<int>(static_cast<uint32_t>(ld * n * 4)));
  return BMat{__builtin_amdgcn_make_buffer_rsrc(base, 0, bytes, 0x00020000),
              __builtin_amdgcn_readfirstlane(static_cast<int>(ld * 4))};
}
__device__ __forceinline__ int b_lane_off(int64_t row, int64_t m, const BMat& A, int lgmul) {
  const int lg = (threadIdx.x & 63) >> 4;
  const int r = static_cast<int>(row < m ? row : m - 1);
  return r * 4 + lgmul * lg * A.ld4;
}
__device__ __forceinline__ float b_ld(const BMat& A, int off, int col) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(A.r, off, col * A.ld4, 0));
}
__device__ __forceinline__ void b_st(const BMat& A, int off, int col, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), A.r, off, col * A.ld4, 0);
}

// LDS of the engine: one union over the phases (about 72 KB: two
// workgroups per CU).
constexpr int kBPanMax = 256 * 8 * 9 / 2;   // solve / product panels, n = 128
constexpr int kBQsLd = 128 + 4;             // Gram tile row stride (floats)
constexpr int kBPackMax = 128 * 129 / 2;    // packed upper n x n, n = 128
struct BLds {
  union {
    struct {                                 // A: the block of P_c (FP64), X tiles
      double p[16 * kBSketchTiles * 16];
      float xt[4][16][kBXtLd];                 // per wave: 16 columns x 128 rows
    } a;
    struct {                                 // C, E: panels, exchange tiles, Gram rows
      float pan[kBPanMax];
      float tq[4][16][4];
      float qs[64][kBQsLd];
    } c;
    struct {                                 // B: one 16-column panel of P
      double V[16][kMaxKB];
      double tau[16];
    } q;
    struct {                                 // D: G / R' / T packed, a column per wave
      double g[kBPackMax];
      double col[4][128];
    } d;
  };
  double red[8];
  int flag;
};

typedef __bf16 bbf8 __attribute__((ext_vector_type(8)));

__device__ inline void b_split3(float x, uint32_t& h, uint32_t& d, uint32_t& l) {
  h = __float_as_uint(x) & 0xFFFF0000u;
  const float r = x - __uint_as_float(h);
  d = __float_as_uint(r) & 0xFFFF0000u;
  l = __float_as_uint(r - __uint_as_float(d));
}

// ---------------------------------------------------------------------------
// A: columns 16 g .. 16 g + 15 of P_c = Theta_c X_c (the rows of chunk c),
// row tiles j0 .. j0 + KT - 1 of Theta (16 rows each).  The chunk's 128-row blocks (one
// Rademacher block each) go round-robin to the waves, so every wave streams
// different rows: it loads its block straight into the B-operand layout of
// the 16x16x32 bf16 product (lane: column 16 g + l16, rows 8 lg .. 8 lg + 7
// of each 32-row step), splits it exactly into three bf16 planes in
// registers and multiplies them with the +-1 A operand of every row tile
// (products exact), summing in FP32 over its blocks; the next block is
// loaded while the current one is used.  The four waves' sums are added in
// FP64 through LDS in wave order.
template <int KT>
__device__ __noinline__ void b_sketch_task(const BInst& b, int c, int g, int j0, unsigned char* ws,
                                           BLds& sh) {
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63, l16 = lane & 15, lg = lane >> 4;
  int64_t r_begin, r_end;
  b_chunk_rows(b, c, ws, r_begin, r_end);
  const int n = b_uniform(gp(&b)->n), k = b_uniform(gp(&b)->k);
  const int64_t ldx = b_uniform(gp(&b)->ldx);
  const uint64_t seed = static_cast<uint64_t>(b_uniform(static_cast<int64_t>(gp(&b)->seed)));
  const BMat X = b_mat(b.X, ldx, n);
  f4 acc[KT];
#pragma unroll
  for (int j = 0; j < KT; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
  // A block is loaded with row-contiguous loads (load i: column i / 2, rows
  // 64 (i & 1) + lane: two cache lines per instruction), stored to the
  // wave's LDS tile and read back in the B-operand layout (rows 8 lg ..
  // 8 lg + 7 of column l16).
  const int coff = __builtin_amdgcn_readfirstlane(static_cast<int>(static_cast<uint32_t>(16 * g * ldx * 4)));
  auto load_blk = [&](int64_t r0, float (&xv)[32]) {
#pragma unroll
    for (int i = 0; i < 32; ++i)
      xv[i] = __builtin_bit_cast(
          float, __builtin_amdgcn_raw_buffer_load_b32(
                     X.r, 4 * lane,
                     __builtin_amdgcn_readfirstlane(static_cast<int>(
                         static_cast<uint32_t>(coff + (i >> 1) * X.ld4 + (r0 + 64 * (i & 1)) * 4))),
                     0));
  };
  float (*xt)[kBXtLd] = sh.a.xt[wave];
  float xn[32];
  const int64_t first = r_begin + 128 * wave;
  if (first < r_end) load_blk(first, xn);
  for (int64_t r0 = first; r0 < r_end; r0 = b_uniform(r0 + 512)) {
    // the block to LDS (rows past the end of the matrix, which read other
    // data, as zeros), then the next block's loads
    if (r0 + 128 > r_end) {
#pragma unroll
      for (int i = 0; i < 32; ++i)
        xt[i >> 1][64 * (i & 1) + lane] = (r0 + 64 * (i & 1) + lane < r_end) ? xn[i] : 0.f;
    } else {
#pragma unroll
      for (int i = 0; i < 32; ++i) xt[i >> 1][64 * (i & 1) + lane] = xn[i];
    }
    wave_sync();
    if (r0 + 512 < r_end) load_blk(r0 + 512, xn);
    // Rademacher words of the block: the four lane groups need the same
    // Theta rows, so lane group lg computes tiles lg, lg + 4, ... (one
    // Philox call per row) and the others read them with a cross-lane permute
    const int64_t blk = r0 >> 7;
    constexpr int TR = (KT + 3) / 4;
    Words w[TR];
#pragma unroll
    for (int i = 0; i < TR; ++i) {
      const int j = lg + 4 * i;
      w[i] = (j < KT) ? radem_words(seed, 16 * (j0 + j) + l16, blk) : Words{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // B operands: the three planes of rows 8 lg .. 8 lg + 7
      const f4 x0 = *reinterpret_cast<const f4*>(&xt[l16][32 * q + 8 * lg]);
      const f4 x1 = *reinterpret_cast<const f4*>(&xt[l16][32 * q + 8 * lg + 4]);
      uint32_t hp[8], dp[8], lp[8];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        b_split3(x0[e], hp[e], dp[e], lp[e]);
        b_split3(x1[e], hp[4 + e], dp[4 + e], lp[4 + e]);
      }
      u4v_t hv, dv, lv;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        hv[t] = __builtin_amdgcn_perm(hp[2 * t + 1], hp[2 * t], 0x07060302u);
        dv[t] = __builtin_amdgcn_perm(dp[2 * t + 1], dp[2 * t], 0x07060302u);
        lv[t] = __builtin_amdgcn_perm(lp[2 * t + 1], lp[2 * t], 0x07060302u);
      }
      const bbf8 bh = __builtin_bit_cast(bbf8, hv), bd = __builtin_bit_cast(bbf8, dv),
                 bl = __builtin_bit_cast(bbf8, lv);
#pragma unroll
      for (int j = 0; j < KT; ++j) {
        const Words& wj = w[j >> 2];
        const uint32_t wown = (q == 0) ? wj.w0 : (q == 1) ? wj.w1 : (q == 2) ? wj.w2 : wj.w3;
        const uint32_t wq = static_cast<uint32_t>(__shfl(static_cast<int>(wown), l16 + 16 * (j & 3)));
        // Row 8 lg + u of the step has step offset 4 t + e with
        // t = 2 lg + (u >> 2), e = u & 3, i.e. bit 8 e + t of the word
        // (theta.h's layout): after y = wq >> 2 lg, rows u = 0..3 sit at
        // bits 0, 8, 16, 24 and rows 4..7 at bits 1, 9, 17, 25.  Each byte
        // of s0 (s1) is the high byte of the bf16 +-1 of one row, 0x3F or
        // 0xBF (0x3F80 is +1 in bf16); the permutes pair them with the low
        // bytes 0x80 in row order.
        const uint32_t y = wq >> (2 * lg);
        const uint32_t s0 = ((y << 7) & 0x80808080u) | 0x3F3F3F3Fu;
        const uint32_t s1 = ((y << 6) & 0x80808080u) | 0x3F3F3F3Fu;
        u4v_t av;
        av[0] = __builtin_amdgcn_perm(s0, 0x80808080u, 0x05000400u);
        av[1] = __builtin_amdgcn_perm(s0, 0x80808080u, 0x07000600u);
        av[2] = __builtin_amdgcn_perm(s1, 0x80808080u, 0x05000400u);
        av[3] = __builtin_amdgcn_perm(s1, 0x80808080u, 0x07000600u);
        const bbf8 a = __builtin_bit_cast(bbf8, av);
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl, acc[j], 0, 0, 0);
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bd, acc[j], 0, 0, 0);
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh, acc[j], 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);  // one step's planes live at a time
    }
    wave_sync();  // the tile is rewritten by the next block
  }
  // sum of the waves' partials in FP64, in wave order; lane (l16, lg) holds
  // Theta rows 16 (j0 + j) + 4 lg + v and X column 16 g + l16
  constexpr int kr = 16 * KT;
  double* red = sh.a.p;  // kr x 16, element (row, col) at row + kr col
#pragma unroll
  for (int wv = 0; wv < 4; ++wv) {
    if (wave == wv)
#pragma unroll
      for (int j = 0; j < KT; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double& t = red[(16 * j + 4 * lg + v) + kr * l16];
          t = (wv == 0 ? 0.0 : t) + static_cast<double>(acc[j][v]);
        }
    __syncthreads();
  }
  // P_c is column-major with leading dimension k
  RCQ_G double* Pc = gp(reinterpret_cast<double*>(ws + b.base + b.L.Pp)) + static_cast<int64_t>(c) * k * n;
  for (int e = threadIdx.x; e < 16 * kr; e += kBThreads) {
    const int r = e % kr, col = e / kr;
    Pc[(16 * j0 + r) + static_cast<int64_t>(16 * g + col) * k] = red[e];
  }
  __syncthreads();  // the LDS is reused by the next task
}

// ---------------------------------------------------------------------------
// B: P = sum_c P_c / sqrt(k), Householder QR (FP64), sign fix, R_s, panels.
// Blocked by 16-column panels: a panel of P sits in LDS while its 16
// reflectors are formed (LAPACK's dlarfg convention, v_j = 1 implied), then
// each wave applies them to 4 trailing columns at a time, held in registers
// (rows spread over the lanes), so a trailing column makes one round trip to
// memory per panel.
__device__ __noinline__ void b_qr_task(const BInst& b, int i, unsigned char* ws, BLds& sh, int* status,
                                       int passes) {
  const int n = b_uniform(b.n), k = b_uniform(b.k);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t kpad = k;
  const int nchunk = b_uniform(b.L.nchunk);
  const RCQ_G double* Pp = gp(reinterpret_cast<const double*>(ws + b.base + b.L.Pp));
  RCQ_G double* P = gp(reinterpret_cast<double*>(ws + b.base + b.L.P));
  RCQ_G double* Rs = gp(reinterpret_cast<double*>(ws + b.base + b.L.Rs));
  RCQ_G float* pan = gp(reinterpret_cast<float*>(ws + b.base + b.L.pan));
  RCQ_G double* R = gp(b.R);
  const int64_t ldr = b.ldr;
  const double scale = 1.0 / sqrt(static_cast<double>(k));
  for (int64_t e = tid; e < static_cast<int64_t>(k) * n; e += kBThreads) {
    const int64_t r = e % k, col = e / k;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += Pp[(static_cast<int64_t>(c) * n + col) * kpad + r];
    P[r + col * k] = s * scale;
  }
  __syncthreads();
  auto& V = sh.q.V;
  for (int c0 = 0; c0 < n; c0 += 16) {
    const int rows = k - c0;  // panel rows c0 .. k-1 (local row r = global row c0 + r)
    for (int e = tid; e < 16 * rows; e += kBThreads) {
      const int r = e % rows, cc = e / rows;
      V[cc][r] = P[(c0 + r) + static_cast<int64_t>(c0 + cc) * k];
    }
    __syncthreads();
    for (int jj = 0; jj < 16; ++jj) {
      // alpha is read before the block sum, whose barriers order every read
      // before the diagonal is overwritten with beta
      const double alpha = b_uniform(V[jj][jj]);
      double ss = 0.0;
      for (int r = jj + 1 + tid; r < rows; r += kBThreads) ss += V[jj][r] * V[jj][r];
      const double xnorm2 = b_uniform(b_block_sum(ss, sh.red));
      double tau = 0.0, beta = alpha, scal = 0.0;
      if (xnorm2 > 0.0) {
        beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      for (int r = jj + 1 + tid; r < rows; r += kBThreads) V[jj][r] *= scal;
      if (tid == 0) {
        V[jj][jj] = beta;
        sh.q.tau[jj] = tau;
      }
      __syncthreads();
      // the panel's later columns (wave w: columns jj + 1 + w, + 4, ...)
      if (tau != 0.0)
        for (int c = jj + 1 + wave; c < 16; c += 4) {
          double d = (lane == 0) ? V[c][jj] : 0.0;
          for (int r = jj + 1 + lane; r < rows; r += 64) d += V[jj][r] * V[c][r];
          d = wave_sum(d) * tau;
          if (lane == 0) V[c][jj] -= d;
          for (int r = jj + 1 + lane; r < rows; r += 64) V[c][r] -= d * V[jj][r];
        }
      __syncthreads();
    }
    // the panel's R rows back to P (on and above the diagonal)
    for (int e = tid; e < 256; e += kBThreads) {
      const int r = e & 15, cc = e >> 4;
      if (r <= cc) P[(c0 + r) + static_cast<int64_t>(c0 + cc) * k] = V[cc][r];
    }
    // trailing columns c0 + 16 .. n - 1, four per wave at a time; rows
    // lane + 64 t of the panel (t < 6 covers k <= 384)
    for (int cb = c0 + 16 + 4 * wave; cb < n; cb += 16) {
      double a[4][6];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int t = 0; t < 6; ++t) {
          const int r = lane + 64 * t;
          a[q][t] = (cb + q < n && r < rows) ? P[(c0 + r) + static_cast<int64_t>(cb + q) * k] : 0.0;
        }
      for (int jj = 0; jj < 16; ++jj) {
        const double tau = sh.q.tau[jj];
        double v[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) {
          const int r = lane + 64 * t;
          v[t] = (r < jj || r >= rows) ? 0.0 : (r == jj) ? 1.0 : V[jj][r];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double d = 0.0;
#pragma unroll
          for (int t = 0; t < 6; ++t) d += v[t] * a[q][t];
          d = wave_sum(d) * tau;
#pragma unroll
          for (int t = 0; t < 6; ++t) a[q][t] -= d * v[t];
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int t = 0; t < 6; ++t) {
          const int r = lane + 64 * t;
          if (cb + q < n && r < rows) P[(c0 + r) + static_cast<int64_t>(cb + q) * k] = a[q][t];
        }
    }
    __syncthreads();
  }
  // R_s = D R with D = sign(diag R) (positive diagonal); status 1 for a zero
  // or non-finite diagonal
  int bad = 0;
  for (int e = tid; e < n * n; e += kBThreads) {
    const int r = e % n, col = e / n;
    const double dr = P[r + static_cast<int64_t>(r) * k];
    const double sg = (dr < 0.0) ? -1.0 : 1.0;
    Rs[r + col * n] = (r <= col) ? sg * P[r + static_cast<int64_t>(col) * k] : 0.0;
  }
  if (tid < n) {
    const double dr = P[tid + static_cast<int64_t>(tid) * k];
    if (!(dr != 0.0) || !isfinite(dr)) bad = 1;
  }
  if (bad) atomicMax(status + i, RCHOLQR_SKETCH_RANK);
  __syncthreads();
  // solve panels (make_panels_kernel's layout: panel b rows 0..16b+15 of
  // columns 16b..16b+15, row-major; above the diagonal block -R, in it R
  // with 1/R_jj on the diagonal)
  const int nb = b_uniform(b.L.nb);
  const int64_t pe = 256 * static_cast<int64_t>(nb) * (nb + 1) / 2;
  for (int64_t e = tid; e < pe; e += kBThreads) {
    int pb = 0;
    while (256ll * (pb + 1) * (pb + 2) / 2 <= e) ++pb;
    const int64_t off = e - 256ll * pb * (pb + 1) / 2;
    const int r = static_cast<int>(off / 16), cc = static_cast<int>(off % 16);
    const int col = 16 * pb + cc;
    double v;
    if (r < 16 * pb) {
      v = -Rs[r + col * n];
    } else {
      v = (r <= col) ? Rs[r + col * n] : 0.0;
      if (r == col) v = 1.0 / v;
    }
    pan[e] = static_cast<float>(v);
  }
  if (passes == 1)
    for (int e = tid; e < n * n; e += kBThreads) {
      const int r = e % n, col = e / n;
      R[r + col * ldr] = Rs[r + col * n];
    }
}

// Loads the packed panels (256 NB (NB + 1) / 2 floats) into LDS.
template <int NB>
__device__ __forceinline__ void b_panels_to_lds(const RCQ_G float* __restrict__ pan, float* lds) {
  constexpr int kE = 256 * NB * (NB + 1) / 2;
  for (int e = threadIdx.x; e < kE; e += kBThreads) lds[e] = pan[e];
}

// X rows in the solve's register layout (xr[4 b + v] = X[row][16 b + 4 lg + v];
// off = b_lane_off(row, m, X, 4)).
template <int NB>
__device__ __forceinline__ void b_load_rows(const BMat& X, int off, float (&xr)[4 * NB]) {
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) xr[4 * b + v] = b_ld(X, off, 16 * b + v);
}
// Q1 rows in the B-operand layout (qa[s] = Q1[row][4 s + lg]; off =
// b_lane_off(row, m, Q, 1)).
template <int NB>
__device__ __forceinline__ void b_load_qa(const BMat& Q, int off, float (&qa)[4 * NB]) {
#pragma unroll
  for (int s = 0; s < 4 * NB; ++s) qa[s] = b_ld(Q, off, 4 * s);
}

// The wave's 16 rows of Q1 = X R^{-1}: xr holds the rows of X
// (xr[4 b + v] = X[row][16 b + 4 lg + v]), the panels are in LDS (pl,
// make_panels layout), tq is the wave's exchange tile.  Q1 is written to Q
// (qoff: the lane's b_lane_off; FULL: every row of the block is below m,
// else rows >= m are skipped) and left in qa (qa[s] = Q1[row][4 s + lg], the
// B-operand layout).  Once panel b has taken its X values, their registers
// are reloaded with the rows of the next block (xoff, when `next`), so the
// loads run a block ahead without a second copy.  Same arithmetic as
// trsm_block, without barriers.
template <int NB, bool FULL>
__device__ __forceinline__ void b_solve16(float (&xr)[4 * NB], const float* pl, float (&qa)[4 * NB],
                                          float (*tq)[4], const BMat& Q, int qoff, bool in,
                                          const BMat& X, int xoff, bool next) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, lg = lane >> 4;
  const int acol = arow_for_blocked_d<float>(l16);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const float* pb = pl + 256 * (b * (b + 1) / 2);
    f4 D = f4{xr[4 * b], xr[4 * b + 1], xr[4 * b + 2], xr[4 * b + 3]};
    if (next)
#pragma unroll
      for (int v = 0; v < 4; ++v) xr[4 * b + v] = b_ld(X, xoff, 16 * b + v);
    f4 E = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4 * (NB - 1); s += 2)
      if (s < 4 * b) {
        D = mfma16x16x4(pb[(4 * s + lg) * 16 + acol], qa[s], D);
        E = mfma16x16x4(pb[(4 * (s + 1) + lg) * 16 + acol], qa[s + 1], E);
        if ((s & 7) == 6) __builtin_amdgcn_sched_barrier(0);
      }
    D += E;
    const float* dgb = pb + 16 * b * 16;
#pragma unroll
    for (int gs = 0; gs < 4; ++gs) {
      float x[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float t = D[v];
#pragma unroll
        for (int vp = 0; vp < v; ++vp) t -= x[vp] * dgb[(4 * gs + vp) * 16 + 4 * gs + v];
        x[v] = t * dgb[(4 * gs + v) * 16 + 4 * gs + v];
      }
      if (lg == gs) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          D[v] = x[v];
          tq[l16][v] = x[v];
        }
      }
      wave_sync();
      qa[4 * b + gs] = tq[l16][lg];
      wave_sync();
      if (gs < 3) {
        const float a = (acol > 4 * gs + 3) ? -dgb[(4 * gs + lg) * 16 + acol] : 0.f;
        D = mfma16x16x4(a, qa[4 * b + gs], D);
      }
    }
    if (FULL || in)
#pragma unroll
      for (int v = 0; v < 4; ++v) b_st(Q, qoff, 16 * b + v, D[v]);
    // one panel's operands live at a time (unrolled, the scheduler would
    // hoist every panel's LDS loads and spill)
    __builtin_amdgcn_sched_barrier(0);
  }
}

// ---------------------------------------------------------------------------
// C: Q1 rows of chunk c (64-row blocks, 16 rows per wave, panels in LDS),
// then (2 passes) their Gram G_c = Q1_c^T Q1_c from the solved rows, which
// go through an LDS tile: each wave owns upper 16 x 16 tiles of G_c, takes
// their FP32 matrix-core products in one chain per tile over 4 blocks (256
// rows), and folds the chain into the chunk's FP64 partial in memory (the
// first fold stores, the later ones are FP64 atomic adds: this workgroup
// alone writes the partial, so the order of the additions is fixed).
// FP64 accumulators in registers would cost 8 VGPRs per tile and spill at
// n >= 64, and a spill reload waits for every row loaded ahead.
constexpr int kBGramFold = 4;  // blocks per FP32 chain

template <int NB>
__device__ __noinline__ void b_solve_task(const BInst& b, int c, unsigned char* ws, BLds& sh, int passes) {
  constexpr int N = 16 * NB;
  constexpr int kTiles = NB * (NB + 1) / 2;
  constexpr int kPerWave = (kTiles + 3) / 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  int64_t r_begin, r_end;
  b_chunk_rows(b, c, ws, r_begin, r_end);
  const int64_t m = b_uniform(b.m), ldx = b_uniform(b.ldx), ldq = b_uniform(b.ldq);
  const BMat X = b_mat(b.X, ldx, N), Q = b_mat(b.Q, ldq, N);
  RCQ_G double* Gc = gp(reinterpret_cast<double*>(ws + b.base + b.L.Gp)) + static_cast<int64_t>(c) * N * N;
  b_panels_to_lds<NB>(gp(reinterpret_cast<const float*>(ws + b.base + b.L.pan)), sh.c.pan);
  const bool gram = passes == 2;
  f4 acc[kPerWave];
  int ti[kPerWave], tj[kPerWave];
#pragma unroll
  for (int s = 0; s < kPerWave; ++s) {
    acc[s] = f4{0.f, 0.f, 0.f, 0.f};
    int idx = wave + 4 * s, a = 0;
    while (idx >= NB - a && a < NB) {
      idx -= NB - a;
      ++a;
    }
    ti[s] = __builtin_amdgcn_readfirstlane(a);
    tj[s] = __builtin_amdgcn_readfirstlane(a + idx);
  }
  int pending = 0;      // blocks in the FP32 chains
  bool stored = false;  // the partial holds a first fold
  auto fold = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < kPerWave; ++s)
      if (wave + 4 * s < kTiles) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          RCQ_G double* g = Gc + (16 * ti[s] + 4 * lg + v) + static_cast<int64_t>(16 * tj[s] + l16) * N;
          if (stored)
            __builtin_amdgcn_global_atomic_fadd_f64(g, static_cast<double>(acc[s][v]));
          else
            *g = static_cast<double>(acc[s][v]);
        }
        acc[s] = f4{0.f, 0.f, 0.f, 0.f};
      }
    if (!stored) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // stores before the adds
    stored = true;
    pending = 0;
  };
  // one 64-row block: solve (16 rows per wave), then the Gram of its rows
  auto block = [&](auto full, int64_t r0, float (&xr)[4 * NB]) {
    const int64_t row = r0 + 16 * wave + l16;
    const bool next = r0 + 64 < r_end;
    float qa[4 * NB];
    b_solve16<NB, decltype(full)::value>(xr, sh.c.pan, qa, sh.c.tq[wave], Q, b_lane_off(row, m, Q, 4),
                                         row < m, X, b_lane_off(row + 64, m, X, 4), next);
    if (!gram) return;
    const bool in = row < m;
#pragma unroll
    for (int s = 0; s < 4 * NB; ++s) sh.c.qs[16 * wave + l16][4 * s + lg] = in ? qa[s] : 0.f;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kPerWave; ++s) {
      if (wave + 4 * s < kTiles) {
#pragma unroll
        for (int kk = 0; kk < 16; ++kk)
          acc[s] = mfma16x16x4(sh.c.qs[4 * kk + lg][16 * ti[s] + l16], sh.c.qs[4 * kk + lg][16 * tj[s] + l16],
                               acc[s]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    if (++pending == kBGramFold) fold();
  };
  float xr[4 * NB];
  b_load_rows<NB>(X, b_lane_off(r_begin + 16 * wave + l16, m, X, 4), xr);
  __syncthreads();  // panels in LDS
  // full blocks, then the block that holds row m - 1 (if it is partial)
  const int64_t r_full = r_begin + ((r_end - r_begin) / 64) * 64;
  for (int64_t r0 = r_begin; r0 < r_full; r0 += 64) block(std::true_type{}, r0, xr);
  if (r_full < r_end) block(std::false_type{}, r_full, xr);
  if (gram && (pending > 0 || !stored)) fold();
}

// ---------------------------------------------------------------------------
// D: G = sum_c G_c, R' = chol(G) (upper), R = R' R_s, T = R'^{-1}, product
// panels.  G, R' and T share one packed upper triangle in LDS (column j at
// j (j + 1) / 2): the Cholesky is right-looking, the inverse is formed in
// place column by column (T(0:j, j) = -T(j, j) T(0:j, 0:j) R'(0:j, j), as
// LAPACK's xTRTI2).
__device__ inline int b_pk(int r, int c) { return c * (c + 1) / 2 + r; }

__device__ __noinline__ void b_chol_task(const BInst& b, int i, unsigned char* ws, BLds& sh, int* status) {
  const int n = b_uniform(b.n), tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nchunk = b_uniform(b.L.nchunk);
  const RCQ_G double* Gp = gp(reinterpret_cast<const double*>(ws + b.base + b.L.Gp));
  const RCQ_G double* Rs = gp(reinterpret_cast<const double*>(ws + b.base + b.L.Rs));
  RCQ_G float* pan2 = gp(reinterpret_cast<float*>(ws + b.base + b.L.pan2));
  RCQ_G double* R = gp(b.R);
  const int64_t ldr = b.ldr;
  double* g = sh.d.g;
  // upper triangle of G (the partials hold the upper 16 x 16 blocks)
  for (int c = wave; c < n; c += 4)
    for (int r = lane; r <= c; r += 64) {
      double s = 0.0;
      for (int ch = 0; ch < nchunk; ++ch) s += Gp[static_cast<int64_t>(ch) * n * n + r + c * n];
      g[b_pk(r, c)] = s;
    }
  __syncthreads();
  // G = R'^T R': step j scales row j by 1 / r_jj, then updates the trailing
  // upper triangle (the diagonal entry becomes r_jj during that update,
  // which does not read it)
  int fail = -1;
  for (int j = 0; j < n; ++j) {
    const double d = b_uniform(g[b_pk(j, j)]);
    if (!(d > 0.0) || !isfinite(d)) {
      fail = j;
      break;
    }
    const double rjj = sqrt(d);
    for (int l = j + 1 + tid; l < n; l += kBThreads) g[b_pk(j, l)] /= rjj;
    __syncthreads();
    for (int c = j + 1 + wave; c < n; c += 4) {
      const double gjc = g[b_pk(j, c)];
      for (int a = j + 1 + lane; a <= c; a += 64) g[b_pk(a, c)] -= g[b_pk(j, a)] * gjc;
    }
    if (tid == 0) g[b_pk(j, j)] = rjj;
    __syncthreads();
  }
  if (fail >= 0) {
    if (tid == 0) atomicMax(status + i, RCHOLQR_CHOL_BREAKDOWN + fail);
    return;
  }
  // R = R' R_s (both upper triangular): wave w forms columns w, w + 4, ...
  // with column c of R_s in its LDS slot
  for (int c = wave; c < n; c += 4) {
    for (int l = lane; l <= c; l += 64) sh.d.col[wave][l] = Rs[l + c * n];
    wave_sync();
    for (int r = lane; r < n; r += 64) {
      double s = 0.0;
      for (int l = r; l <= c; ++l) s += g[b_pk(r, l)] * sh.d.col[wave][l];
      R[r + static_cast<int64_t>(c) * ldr] = (r <= c) ? s : 0.0;
    }
    wave_sync();
  }
  __syncthreads();
  // T = R'^{-1} in place, column by column
  for (int j = 0; j < n; ++j) {
    for (int l = tid; l < j; l += kBThreads) sh.d.col[0][l] = g[b_pk(l, j)];
    __syncthreads();
    const double tjj = 1.0 / g[b_pk(j, j)];
    for (int r = tid; r < j; r += kBThreads) {
      double s = 0.0;
      for (int l = r; l < j; ++l) s += g[b_pk(r, l)] * sh.d.col[0][l];
      g[b_pk(r, j)] = -tjj * s;
    }
    __syncthreads();
    if (tid == 0) g[b_pk(j, j)] = tjj;
  }
  __syncthreads();
  // product panels (make_panels_kernel's layout with +T above the diagonal)
  const int nb = b_uniform(b.L.nb);
  const int64_t pe = 256 * static_cast<int64_t>(nb) * (nb + 1) / 2;
  for (int64_t e = tid; e < pe; e += kBThreads) {
    int pb = 0;
    while (256ll * (pb + 1) * (pb + 2) / 2 <= e) ++pb;
    const int64_t off = e - 256ll * pb * (pb + 1) / 2;
    const int r = static_cast<int>(off / 16), col = 16 * pb + static_cast<int>(off % 16);
    pan2[e] = static_cast<float>((r <= col) ? g[b_pk(r, col)] : 0.0);
  }
}

// E: Q = Q1 T on the rows of chunk c (in place; panels in LDS, 16 rows per
// wave, the next block's rows loaded ahead).
template <int NB>
__device__ __noinline__ void b_product_task(const BInst& b, int c, unsigned char* ws, BLds& sh) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  const int acol = arow_for_blocked_d<float>(l16);
  int64_t r_begin, r_end;
  b_chunk_rows(b, c, ws, r_begin, r_end);
  const int64_t m = b_uniform(b.m), ldq = b_uniform(b.ldq);
  const BMat Q = b_mat(b.Q, ldq, 16 * NB);
  b_panels_to_lds<NB>(gp(reinterpret_cast<const float*>(ws + b.base + b.L.pan2)), sh.c.pan);
  auto block = [&](auto full, int64_t r0, float (&qn)[4 * NB]) {
    const int64_t row = r0 + 16 * wave + l16;
    float qa[4 * NB];
#pragma unroll
    for (int e = 0; e < 4 * NB; ++e) qa[e] = qn[e];
    if (r0 + 64 < r_end) b_load_qa<NB>(Q, b_lane_off(row + 64, m, Q, 1), qn);
    const int qoff = b_lane_off(row, m, Q, 4);
    const bool in = row < m;
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) {
      const float* pb = sh.c.pan + 256 * (bb * (bb + 1) / 2);
      f4 D = f4{0.f, 0.f, 0.f, 0.f}, E = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 4 * NB; s += 2)
        if (s < 4 * (bb + 1)) {
          D = mfma16x16x4(pb[(4 * s + lg) * 16 + acol], qa[s], D);
          E = mfma16x16x4(pb[(4 * (s + 1) + lg) * 16 + acol], qa[s + 1], E);
          if ((s & 7) == 6) __builtin_amdgcn_sched_barrier(0);
        }
      if (decltype(full)::value || in)
#pragma unroll
        for (int v = 0; v < 4; ++v) b_st(Q, qoff, 16 * bb + v, D[v] + E[v]);
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  float qn[4 * NB];
  b_load_qa<NB>(Q, b_lane_off(r_begin + 16 * wave + l16, m, Q, 1), qn);
  __syncthreads();
  const int64_t r_full = r_begin + ((r_end - r_begin) / 64) * 64;
  for (int64_t r0 = r_begin; r0 < r_full; r0 += 64) block(std::true_type{}, r0, qn);
  if (r_full < r_end) block(std::false_type{}, r_full, qn);
}

#define RCQ_B_NB_SWITCH(NBV, CALL) \
  switch (NBV) {                   \
    case 1: CALL(1); break;        \
    case 2: CALL(2); break;        \
    case 3: CALL(3); break;        \
    case 4: CALL(4); break;        \
    case 5: CALL(5); break;        \
    case 6: CALL(6); break;        \
    case 7: CALL(7); break;        \
    case 8: CALL(8); break;        \
    default: break;                \
  }

// ---------------------------------------------------------------------------
// The queue loop has no thread-divergent branch: the dequeue, the wait and
// the completion count run in wave 0 as a whole (wave-uniform branch; lane 0
// alone adds to the counters, every lane takes lane 0's result), and every
// value that steers the loop is made scalar with readfirstlane.  A block
// guarded by threadIdx.x == 0 at the end of the body and another at its top
// would be merged across the back edge by the compiler into a second loop
// latch taken by thread 0 alone: the other lanes would then pass the
// barriers and rerun the previous task without a new one being dequeued.
// A wait is bounded in wall-clock time (s_memrealtime, 100 MHz): past the
// bound the engine's error word is set, the stall is recorded and every
// workgroup leaves the loop.
__global__ __launch_bounds__(kBThreads, 2) void batched_persistent_kernel(unsigned char* ws,
                                                                       long long wait_ticks) {
  __shared__ BLds sh;
  __shared__ int s_task, s_stop;
  BHeader* h = reinterpret_cast<BHeader*>(ws);
  int* done = reinterpret_cast<int*>(ws + b_done_off());
  const int batch = __builtin_amdgcn_readfirstlane(h->batch);
  const int passes = __builtin_amdgcn_readfirstlane(h->passes);
  int* status = reinterpret_cast<int*>(ws + b_status_off(batch));
  const BInst* inst = reinterpret_cast<const BInst*>(ws + b_inst_off(batch));
  const int64_t nA = h->nA, nC = h->nC;
  const int64_t nB = batch, nD = (passes == 2) ? batch : 0, nE = (passes == 2) ? nC : 0;
  const int total = __builtin_amdgcn_readfirstlane(static_cast<int>(nA + nB + nC + nD + nE));
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int one = ((threadIdx.x & 63) == 0) ? 1 : 0;  // lane 0's increment
  for (;;) {
    if (wave == 0) {
      const int t = __builtin_amdgcn_readfirstlane(atomicAdd(&h->counter, one));
      const int e = __builtin_amdgcn_readfirstlane(
          __hip_atomic_load(&h->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      s_task = t;
      s_stop = e;
    }
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(s_task);
    const int stop = __builtin_amdgcn_readfirstlane(s_stop);
    __syncthreads();  // s_task, s_stop are rewritten below
    if (t >= total || stop != 0) break;
    // decode (phase, instance, chunk, group)
    int ph, i = 0, c = 0, g = 0;
    int64_t u = t;
    const RCQ_K BInst* kinst = (const RCQ_K BInst*)(inst);
    if (u < nA) {
      ph = 0;
      i = b_find<true>(inst, batch, u);
      const int64_t loc = u - kinst[i].tA;
      const int ng = kinst[i].L.nb * kinst[i].L.nh;
      c = static_cast<int>(loc / ng);
      g = static_cast<int>(loc % ng);
    } else if ((u -= nA) < nB) {
      ph = 1;
      i = static_cast<int>(u);
    } else if ((u -= nB) < nC) {
      ph = 2;
      i = b_find<false>(inst, batch, u);
      c = static_cast<int>(u - kinst[i].tC);
    } else if ((u -= nC) < nD) {
      ph = 3;
      i = static_cast<int>(u);
    } else {
      u -= nD;
      ph = 4;
      i = b_find<false>(inst, batch, u);
      c = static_cast<int>(u - kinst[i].tC);
    }
    ph = __builtin_amdgcn_readfirstlane(ph);
    i = __builtin_amdgcn_readfirstlane(i);
    c = __builtin_amdgcn_readfirstlane(c);
    g = __builtin_amdgcn_readfirstlane(g);
    const BInst& b = inst[i];
    // dependency: the instance's previous phase complete
    if (wave == 0) {
      int failed = 0;
      if (ph > 0) {
        const int need = __builtin_amdgcn_readfirstlane(
            (ph == 1) ? b.L.nchunk * b.L.nb * b.L.nh : (ph == 3) ? b.L.nchunk : 1);
        int* cnt = done + 8 * i + (ph - 1);
        const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
        int seen = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT));
        while (seen < need) {
          __builtin_amdgcn_s_sleep(8);
          const int err = __builtin_amdgcn_readfirstlane(
              __hip_atomic_load(&h->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
          if (err != 0) {
            failed = 1;
            break;
          }
          if (static_cast<long long>(__builtin_amdgcn_s_memrealtime() - t0) > wait_ticks) {
            const int prev = __builtin_amdgcn_readfirstlane(
                __hip_atomic_fetch_or(&h->error, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            if (prev == 0 && one) {
              h->stall_inst = i;
              h->stall_phase = ph;
              h->stall_seen = seen;
              h->stall_need = need;
            }
            failed = 1;
            break;
          }
          seen = __builtin_amdgcn_readfirstlane(
              __hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT));
        }
      }
      s_stop = failed;
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(s_stop) != 0) break;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const bool live = __builtin_amdgcn_readfirstlane(status[i]) != RCHOLQR_BATCH_INVALID;
    const int nb = __builtin_amdgcn_readfirstlane(b.L.nb);
    if (live) {
      if (ph == 0) {
        // k = 3 n (the engine's shapes) has its own instance; other
        // multiples of 16 use the next larger one (zero rows of Theta are
        // not generated: KT only bounds the loops)
        // task g: 16-column block g / nh, half g % nh of the row tiles
        // (the first half takes the odd tile)
        const int nh = __builtin_amdgcn_readfirstlane(b.L.nh);
        const int kt = __builtin_amdgcn_readfirstlane(b.k) / 16;
        const int half = g % nh, first = (kt + 1) / 2;
        const int j0 = (nh == 1 || half == 0) ? 0 : first;
        const int cnt = (nh == 1) ? kt : (half == 0 ? first : kt - first);
        switch (cnt) {
#define RCQ_B_SK(KTV) case KTV: b_sketch_task<KTV>(b, c, g / nh, j0, ws, sh); break;
          RCQ_B_SK(1) RCQ_B_SK(2) RCQ_B_SK(3) RCQ_B_SK(4) RCQ_B_SK(5) RCQ_B_SK(6) RCQ_B_SK(7)
          RCQ_B_SK(8) RCQ_B_SK(9) RCQ_B_SK(10) RCQ_B_SK(11) RCQ_B_SK(12)
#undef RCQ_B_SK
          default: break;
        }
      } else if (ph == 1) {
        b_qr_task(b, i, ws, sh, status, passes);
      } else if (ph == 2) {
#define RCQ_B_C(NBV) b_solve_task<NBV>(b, c, ws, sh, passes)
        RCQ_B_NB_SWITCH(nb, RCQ_B_C)
#undef RCQ_B_C
      } else if (ph == 3) {
        b_chol_task(b, i, ws, sh, status);
      } else {
#define RCQ_B_E(NBV) b_product_task<NBV>(b, c, ws, sh)
        RCQ_B_NB_SWITCH(nb, RCQ_B_E)
#undef RCQ_B_E
      }
    }
    // every thread's writes are released before the task is counted done
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (wave == 0)
      __hip_atomic_fetch_add(done + 8 * i + ph, one, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// Host side.
int64_t batched_engine_bytes(const rcholqr_problem* probs, int batch, int passes,
                             int64_t chunk) {
  int64_t off = b_region_off(batch);
  for (int i = 0; i < batch; ++i)
    if (b_valid(probs[i]))
      off += b_layout(probs[i].m, static_cast<int>(probs[i].n), static_cast<int>(probs[i].k),
                      passes, chunk).total;
  return off;
}

hipError_t launch_batched_engine(const rcholqr_problem* probs_dev, int batch, int passes,
                                 int64_t chunk, void* ws, int64_t ws_bytes, int grid,
                                 long long wait_ticks, hipStream_t st) {
  batched_setup_kernel<<<1, kBThreads, 0, st>>>(probs_dev, batch, passes, chunk,
                                                static_cast<unsigned char*>(ws), ws_bytes);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  batched_persistent_kernel<<<grid, kBThreads, 0, st>>>(static_cast<unsigned char*>(ws),
                                                        wait_ticks);
  return hipGetLastError();
}

int batched_engine_grid() {
  int dev = 0, cus = 256, per = 1;
  if (hipGetDevice(&dev) == hipSuccess) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && c > 0)
      cus = c;
  }
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per, reinterpret_cast<const void*>(&batched_persistent_kernel), kBThreads, 0) !=
          hipSuccess ||
      per < 1)
    per = 1;
  return cus * per;
}

int64_t batched_engine_status_offset(int batch) { return b_status_off(batch); }

int64_t batched_engine_stall_offset() { return offsetof(BHeader, stall_inst); }

}  // namespace rcq
