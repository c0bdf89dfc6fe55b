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

#include "../../include/rcholqr.h"
#include "common.h"
#include "kernels.h"
#include "tallblock.h"
#include "theta.h"

namespace rcq {

typedef unsigned int u4v_t __attribute__((ext_vector_type(4)));

constexpr int kBThreads = 256;
constexpr int kBSteps = 32;      // rows per sketch / Gram step
constexpr int kBGroup = 64;      // Theta rows per sketch task

// Device layout of one instance's scratch (byte offsets from its region).
struct BLayout {
  int64_t Pp, P, Rs, pan, Gp, G, T, pan2, total;
  int nchunk, ngroup, nb;
};

__host__ __device__ inline int64_t b_align(int64_t x) { return (x + 255) & ~int64_t{255}; }

__host__ __device__ inline BLayout b_layout(int64_t m, int n, int k, int passes, int64_t chunk) {
  BLayout L{};
  L.nb = n / 16;
  L.nchunk = static_cast<int>((m + chunk - 1) / chunk);
  L.ngroup = (k + kBGroup - 1) / kBGroup;
  const int64_t kpad = static_cast<int64_t>(kBGroup) * L.ngroup;
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
         p.k >= p.n && p.k <= 384 && p.m >= p.n && p.ldx >= p.m && p.ldq >= p.m && p.ldr >= p.n;
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
      tA += static_cast<int64_t>(b.L.nchunk) * b.L.ngroup;
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
template <bool PHASE_A>
__device__ inline int b_find(const BInst* inst, int batch, int64_t u) {
  int lo = 0, hi = batch - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int64_t f = PHASE_A ? inst[mid].tA : inst[mid].tC;
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

// Row range [r_begin, r_end) of chunk c, in scalar registers.
__device__ inline void b_chunk_rows(const BInst& b, int c, const unsigned char* ws, int64_t& r_begin,
                                    int64_t& r_end) {
  const int64_t chunk = b_uniform(reinterpret_cast<const BHeader*>(ws)->chunk);
  const int64_t m = b_uniform(b.m);
  r_begin = static_cast<int64_t>(c) * chunk;
  r_end = (r_begin + chunk < m) ? r_begin + chunk : m;
}

__device__ inline double b_wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// LDS of the engine: the largest phase (the sketch's double-buffered planes).
struct BLds {
  union {
    u4v_t planes[2][3 * 4 * 128];       // sketch: bf16 planes of 32 rows x n
    TrsmLds<float, 8> trsm;
    float pbuf[2][256 * 8];              // product
    float qs[kBSteps][128 + 4];          // Gram: FP32 rows
    double v[kMaxK];                     // Householder vector
  };
  double red[8];
  double tau;
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
// A: P_c rows 64 g .. 64 g + 63 (wave w: 16 Theta rows) for the rows of
// chunk c.  Per 32-row step the chunk's X rows are split into three bf16
// planes in LDS, laid out as B operands (16-byte chunk = 8 rows of one
// column); a lane's A operand holds +-1 for 8 rows of its Theta row, built
// from the Rademacher words of that row.
template <int NB>
__device__ __noinline__ void b_sketch_task(const BInst& b, int c, int g, unsigned char* ws, BLds& sh) {
  constexpr int N = 16 * NB;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  int64_t r_begin, r_end;
  b_chunk_rows(b, c, ws, r_begin, r_end);
  const int trow = kBGroup * g + 16 * wave + l16;  // this lane's Theta row
  const bool tlive = trow < b.k;
  d4 acc[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  // staging tasks: (column, 8-row group) pairs, 4 N per step
  constexpr int kTasks = 4 * N;
  constexpr int kPer = (kTasks + kBThreads - 1) / kBThreads;
  float pre[kPer][8];
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int t = threadIdx.x + kBThreads * q;
      const int col = 16 * (t >> 6) + (t & 15), grp = (t >> 4) & 3;
      const int64_t r = r0 + 8 * grp;
      const bool live = t < kTasks;
      const float* src = b.X + static_cast<int64_t>(live ? col : 0) * b.ldx + r;
#pragma unroll
      for (int e = 0; e < 8; ++e) pre[q][e] = (live && r + e < r_end) ? src[e] : 0.f;
    }
  };
  auto stage_in = [&](u4v_t* buf) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int t = threadIdx.x + kBThreads * q;
      if (t < kTasks) {
        const int col = 16 * (t >> 6) + (t & 15), grp = (t >> 4) & 3;
        uint32_t hp[8], dp[8], lp[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) b_split3(pre[q][e], hp[e], dp[e], lp[e]);
        u4v_t hv, dv, lv;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          hv[w] = __builtin_amdgcn_perm(hp[2 * w + 1], hp[2 * w], 0x07060302u);
          dv[w] = __builtin_amdgcn_perm(dp[2 * w + 1], dp[2 * w], 0x07060302u);
          lv[w] = __builtin_amdgcn_perm(lp[2 * w + 1], lp[2 * w], 0x07060302u);
        }
        buf[(0 * 4 + grp) * N + col] = hv;
        buf[(1 * 4 + grp) * N + col] = dv;
        buf[(2 * 4 + grp) * N + col] = lv;
      }
    }
  };
  Words w{0u, 0u, 0u, 0u};
  int64_t wblk = -1;
  int cur = 0;
  if (r_begin < r_end) {
    fetch(r_begin);
    stage_in(sh.planes[0]);
  }
  __syncthreads();
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kBSteps) {
    const bool more = r0 + kBSteps < r_end;
    if (more) fetch(r0 + kBSteps);
    const int64_t blk = r0 >> 7;
    if (blk != wblk) {
      w = tlive ? radem_words(b.seed, trow, blk) : Words{0u, 0u, 0u, 0u};
      wblk = blk;
    }
    const int q = static_cast<int>((r0 >> 5) & 3);
    const uint32_t wq = (q == 0) ? w.w0 : (q == 1) ? w.w1 : (q == 2) ? w.w2 : w.w3;
    // rows 8 lg + u of the step: offset 4 t + e with t = 2 lg + (u >> 2),
    // e = u & 3, at bit 8 e + t (theta.h's layout); 0x3F80 is +1 in bf16
    u4v_t av;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      uint32_t e2[2];
#pragma unroll
      for (int h2 = 0; h2 < 2; ++h2) {
        const int u = 2 * d + h2;
        const uint32_t bit = (wq >> (8 * (u & 3) + 2 * lg + (u >> 2))) & 1u;
        e2[h2] = tlive ? (0x3F80u | (bit << 15)) : 0u;
      }
      av[d] = e2[0] | (e2[1] << 16);
    }
    const bbf8 a = __builtin_bit_cast(bbf8, av);
    const u4v_t* buf = sh.planes[cur];
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const bbf8 bh = __builtin_bit_cast(bbf8, buf[(0 * 4 + lg) * N + 16 * t + l16]);
      const bbf8 bd = __builtin_bit_cast(bbf8, buf[(1 * 4 + lg) * N + 16 * t + l16]);
      const bbf8 bl = __builtin_bit_cast(bbf8, buf[(2 * 4 + lg) * N + 16 * t + l16]);
      f4 s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl, f4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
      s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bd, s, 0, 0, 0);
      s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh, s, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[t][v] += static_cast<double>(s[v]);
    }
    if (more) stage_in(sh.planes[cur ^ 1]);
    __syncthreads();
    cur ^= 1;
  }
  // P_c is column-major with leading dimension kpad; lane (l16, lg) holds
  // Theta rows 4 lg + v of the wave's 16 and X column 16 t + l16.
  const int64_t kpad = static_cast<int64_t>(kBGroup) * b.L.ngroup;
  double* Pc = reinterpret_cast<double*>(ws + b.base + b.L.Pp) + static_cast<int64_t>(c) * kpad * N;
#pragma unroll
  for (int t = 0; t < NB; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      Pc[(kBGroup * g + 16 * wave + 4 * lg + v) + static_cast<int64_t>(16 * t + l16) * kpad] = acc[t][v];
}

// ---------------------------------------------------------------------------
// B: P = sum_c P_c / sqrt(k), Householder QR (FP64), sign fix, R_s, panels.
__device__ __noinline__ void b_qr_task(const BInst& b, int i, unsigned char* ws, BLds& sh, int* status,
                          int passes) {
  const int n = b_uniform(b.n), k = b_uniform(b.k);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t kpad = static_cast<int64_t>(kBGroup) * b.L.ngroup;
  const double* Pp = reinterpret_cast<const double*>(ws + b.base + b.L.Pp);
  double* P = reinterpret_cast<double*>(ws + b.base + b.L.P);
  double* Rs = reinterpret_cast<double*>(ws + b.base + b.L.Rs);
  float* pan = reinterpret_cast<float*>(ws + b.base + b.L.pan);
  const double scale = 1.0 / sqrt(static_cast<double>(k));
  for (int64_t e = tid; e < static_cast<int64_t>(k) * n; e += kBThreads) {
    const int64_t r = e % k, col = e / k;
    double s = 0.0;
    for (int c = 0; c < b.L.nchunk; ++c) s += Pp[(static_cast<int64_t>(c) * n + col) * kpad + r];
    P[r + col * k] = s * scale;
  }
  __syncthreads();
  // Householder reflectors H_j = I - tau v v^T with v_j = 1 (LAPACK's dlarfg
  // convention); v in LDS, R on and above P's diagonal.
  int bad = 0;
  for (int j = 0; j < n; ++j) {
    // alpha is read before the block sum, whose barriers order every read
    // before thread 0 overwrites the diagonal with beta
    const double alpha = b_uniform(P[j + static_cast<int64_t>(j) * k]);
    double ss = 0.0;
    for (int r = j + 1 + tid; r < k; r += kBThreads) ss += P[r + static_cast<int64_t>(j) * k] * P[r + static_cast<int64_t>(j) * k];
    const double xnorm2 = b_uniform(b_block_sum(ss, sh.red));
    double tau = 0.0, beta = alpha, scal = 0.0;
    if (xnorm2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    for (int r = j + 1 + tid; r < k; r += kBThreads) sh.v[r] = P[r + static_cast<int64_t>(j) * k] * scal;
    if (tid == 0) {
      sh.v[j] = 1.0;
      P[j + static_cast<int64_t>(j) * k] = beta;
    }
    __syncthreads();
    // trailing columns, wave w takes columns j + 1 + w, + 4, ...
    if (tau != 0.0)
      for (int l = j + 1 + wave; l < n; l += 4) {
        double* col = P + static_cast<int64_t>(l) * k;
        double d = 0.0;
        for (int r = j + lane; r < k; r += 64) d += sh.v[r] * col[r];
        d = b_wave_sum(d) * tau;
        for (int r = j + lane; r < k; r += 64) col[r] -= d * sh.v[r];
      }
    __syncthreads();
  }
  // R_s = D R with D = sign(diag R) (positive diagonal); status 1 for a zero
  // or non-finite diagonal
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
  const int nb = b.L.nb;
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
      b.R[r + col * b.ldr] = Rs[r + col * n];
    }
}

template <int NB>
__device__ __noinline__ void b_gram_chunk(const BInst& b, int c, int64_t r_begin, int64_t r_end,
                                          unsigned char* ws, BLds& sh);

// ---------------------------------------------------------------------------
// C: Q1 rows of chunk c by trsm_block, then (2 passes) their Gram G_c.
template <int NB>
__device__ __noinline__ void b_solve_task(const BInst& b, int c, unsigned char* ws, BLds& sh, int passes) {
  constexpr int N = 16 * NB;
  int64_t r_begin, r_end;
  b_chunk_rows(b, c, ws, r_begin, r_end);
  const float* pan = reinterpret_cast<const float*>(ws + b.base + b.L.pan);
  for (int64_t blk = r_begin / 64; blk * 64 < r_end; ++blk) {
    trsm_block<float, NB>(b.X, b.m, N, b.ldx, pan, b.Q, b.ldq, blk,
                          *reinterpret_cast<TrsmLds<float, NB>*>(&sh.trsm));
    __syncthreads();
  }
  if (passes != 2) return;
  // The chunk's Q1 rows were written by this workgroup: make them visible
  // to all its waves before the Gram reads them back.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  b_gram_chunk<NB>(b, c, r_begin, r_end, ws, sh);
}

// G_c = Q1_c^T Q1_c for the rows [r_begin, r_end) of chunk c: exact FP32
// matrix-core products, each 32-row step from zero, summed into FP64.
template <int NB>
__device__ __noinline__ void b_gram_chunk(const BInst& b, int c, int64_t r_begin, int64_t r_end,
                                          unsigned char* ws, BLds& sh) {
  constexpr int N = 16 * NB;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  constexpr int kTiles = NB * (NB + 1) / 2;
  constexpr int kPerWave = (kTiles + 3) / 4;
  d4 acc[kPerWave];
  int ti[kPerWave], tj[kPerWave];
#pragma unroll
  for (int s = 0; s < kPerWave; ++s) {
    acc[s] = d4{0.0, 0.0, 0.0, 0.0};
    int idx = wave + 4 * s, a = 0;
    while (idx >= NB - a && a < NB) {
      idx -= NB - a;
      ++a;
    }
    ti[s] = a;
    tj[s] = a + idx;
  }
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kBSteps) {
    for (int e = threadIdx.x; e < kBSteps * N; e += kBThreads) {
      const int rr = e % kBSteps, col = e / kBSteps;
      const int64_t r = r0 + rr;
      sh.qs[rr][col] = (r < r_end) ? b.Q[r + static_cast<int64_t>(col) * b.ldq] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kPerWave; ++s) {
      if (wave + 4 * s < kTiles) {
        f4 cc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < kBSteps / 4; ++kk) {
          const float av = sh.qs[4 * kk + lg][16 * ti[s] + l16];
          const float bv = sh.qs[4 * kk + lg][16 * tj[s] + l16];
          cc = mfma16x16x4(av, bv, cc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[s][v] += static_cast<double>(cc[v]);
      }
    }
    __syncthreads();
  }
  double* Gc = reinterpret_cast<double*>(ws + b.base + b.L.Gp) + static_cast<int64_t>(c) * N * N;
#pragma unroll
  for (int s = 0; s < kPerWave; ++s)
    if (wave + 4 * s < kTiles)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Gc[(16 * ti[s] + 4 * lg + v) + static_cast<int64_t>(16 * tj[s] + l16) * N] = acc[s][v];
}

// ---------------------------------------------------------------------------
// D: G = sum_c G_c, R' = chol(G) (upper), R = R' R_s, T = R'^{-1}, panels.
__device__ __noinline__ void b_chol_task(const BInst& b, int i, unsigned char* ws, BLds& sh, int* status) {
  const int n = b_uniform(b.n), tid = threadIdx.x;
  const double* Gp = reinterpret_cast<const double*>(ws + b.base + b.L.Gp);
  double* G = reinterpret_cast<double*>(ws + b.base + b.L.G);
  double* T = reinterpret_cast<double*>(ws + b.base + b.L.T);
  const double* Rs = reinterpret_cast<const double*>(ws + b.base + b.L.Rs);
  float* pan2 = reinterpret_cast<float*>(ws + b.base + b.L.pan2);
  // upper triangle of G (partials hold the upper 16 x 16 blocks)
  for (int e = tid; e < n * n; e += kBThreads) {
    const int r = e % n, col = e / n;
    if ((r >> 4) <= (col >> 4)) {
      double s = 0.0;
      for (int c = 0; c < b.L.nchunk; ++c) s += Gp[static_cast<int64_t>(c) * n * n + e];
      G[e] = s;
    }
  }
  if (tid == 0) sh.flag = 0;
  __syncthreads();
  // right-looking Cholesky on the upper triangle: G = R'^T R'
  for (int j = 0; j < n; ++j) {
    const double d = b_uniform(G[j + j * n]);
    if (!(d > 0.0) || !isfinite(d)) {
      if (tid == 0) {
        atomicMax(status + i, RCHOLQR_CHOL_BREAKDOWN + j);
        sh.flag = 1;
      }
      __syncthreads();
      break;
    }
    const double rjj = sqrt(d);
    __syncthreads();
    for (int l = j + tid; l < n; l += kBThreads) G[j + l * n] = (l == j) ? rjj : G[j + l * n] / rjj;
    __syncthreads();
    const int w = n - 1 - j;  // trailing order
    for (int e = tid; e < w * w; e += kBThreads) {
      const int a = j + 1 + e % w, c2 = j + 1 + e / w;
      if (a <= c2) G[a + c2 * n] -= G[j + a * n] * G[j + c2 * n];
    }
    __syncthreads();
  }
  if (__builtin_amdgcn_readfirstlane(sh.flag)) return;
  // R = R' R_s (both upper triangular)
  for (int e = tid; e < n * n; e += kBThreads) {
    const int r = e % n, col = e / n;
    double s = 0.0;
    for (int l = r; l <= col; ++l) s += G[r + l * n] * Rs[l + col * n];
    b.R[r + static_cast<int64_t>(col) * b.ldr] = (r <= col) ? s : 0.0;
  }
  // T = R'^{-1}: column j by back substitution
  for (int j = tid; j < n; j += kBThreads) {
    for (int r = n - 1; r >= 0; --r) {
      double t = 0.0;
      if (r <= j) {
        double s = (r == j) ? 1.0 : 0.0;
        for (int l = r + 1; l <= j; ++l) s -= G[r + l * n] * T[l + j * n];
        t = s / G[r + r * n];
      }
      T[r + j * n] = t;
    }
  }
  __syncthreads();
  // product panels (make_panels_kernel's layout with +T above the diagonal)
  const int nb = b.L.nb;
  const int64_t pe = 256 * static_cast<int64_t>(nb) * (nb + 1) / 2;
  for (int64_t e = tid; e < pe; e += kBThreads) {
    int pb = 0;
    while (256ll * (pb + 1) * (pb + 2) / 2 <= e) ++pb;
    const int64_t off = e - 256ll * pb * (pb + 1) / 2;
    const int r = static_cast<int>(off / 16), col = 16 * pb + static_cast<int>(off % 16);
    pan2[e] = static_cast<float>((r <= col) ? T[r + col * n] : 0.0);
  }
}

// E: Q = Q1 T on the rows of chunk c.
template <int NB>
__device__ __noinline__ void b_product_task(const BInst& b, int c, unsigned char* ws, BLds& sh) {
  int64_t r_begin, r_end;
  b_chunk_rows(b, c, ws, r_begin, r_end);
  const float* pan2 = reinterpret_cast<const float*>(ws + b.base + b.L.pan2);
  float(&pbuf)[2][256 * NB] = *reinterpret_cast<float(*)[2][256 * NB]>(&sh.pbuf[0][0]);
  for (int64_t blk = r_begin / 64; blk * 64 < r_end; ++blk) {
    trmm_block<float, NB, false>(b.Q, b.m, 16 * NB, b.ldq, pan2, nullptr, 0, blk, pbuf);
    __syncthreads();
  }
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
    if (u < nA) {
      ph = 0;
      i = b_find<true>(inst, batch, u);
      const int64_t loc = u - inst[i].tA;
      const int ng = inst[i].L.ngroup;
      c = static_cast<int>(loc / ng);
      g = static_cast<int>(loc % ng);
    } else if ((u -= nA) < nB) {
      ph = 1;
      i = static_cast<int>(u);
    } else if ((u -= nB) < nC) {
      ph = 2;
      i = b_find<false>(inst, batch, u);
      c = static_cast<int>(u - inst[i].tC);
    } else if ((u -= nC) < nD) {
      ph = 3;
      i = static_cast<int>(u);
    } else {
      u -= nD;
      ph = 4;
      i = b_find<false>(inst, batch, u);
      c = static_cast<int>(u - inst[i].tC);
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
            (ph == 1) ? b.L.nchunk * b.L.ngroup : (ph == 3) ? b.L.nchunk : 1);
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
#define RCQ_B_A(NBV) b_sketch_task<NBV>(b, c, g, ws, sh)
        RCQ_B_NB_SWITCH(nb, RCQ_B_A)
#undef RCQ_B_A
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
