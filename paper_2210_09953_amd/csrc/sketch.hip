// sketch.hip -- Algorithm 2 step 1, P = Theta X, with Theta generated on the
// fly (Section 2) and never written to memory.
//
// Dense embeddings (Gaussian, Rademacher): a split-K GEMM on FP64 matrix
// cores.  Each workgroup owns 64 rows of Theta (4 waves x 16) and all n
// columns, and streams a contiguous range of rows of X: per stage it stages
// 16 rows of X in LDS (coalesced column segments, FP32 widened exactly to
// FP64), regenerates the matching 64 x 16 block of Theta in LDS, and issues
// 16x16x4 FP64 MFMAs.  Every Theta entry is generated exactly once.  The
// workgroups that share a row range run on the same XCD (L2) so that X is
// fetched from HBM about once.  Per-split FP64 partials are summed in a
// fixed order by sketch_reduce (deterministic).
//
// CountSketch: P[h(j), :] += s(j) X[j, :].  Rows are grouped in tiles of
// 256; count_prep sorts each tile's rows by bucket (stable, once per call),
// so that count_accum can add every bucket's rows in row order without
// atomics: one thread per bucket per tile, into an LDS accumulator.
#include "common.h"
#include "theta.h"
#include "kernels.h"

namespace rcq {

// ----------------------------------------------------------------------------
// Theta export for tests.
__global__ void theta_debug_kernel(int kind, int k, int64_t m, uint64_t seed, int64_t i0,
                                   int64_t ni, int64_t j0, int64_t nj, double* out) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= ni * nj) return;
  const int64_t ii = idx % ni, jj = idx / ni;
  const int64_t i = i0 + ii, j = j0 + jj;
  double v;
  if (kind == kGaussian) {
    double z0, z1;
    gauss_pair(seed, j, static_cast<uint32_t>(i >> 1), z0, z1);
    v = (i & 1) ? z1 : z0;
  } else if (kind == kRademacher) {
    const Words w = radem_words(seed, static_cast<int>(i), j >> 7);
    v = radem_bit(w, static_cast<int>(j & 127)) ? -1.0 : 1.0;
  } else if (kind == kSRHT) {
    const uint64_t sr = srht_row(seed, static_cast<int>(i), srht_log2(m));
    const Words w = srht_words(seed, sr, srht_walsh(sr), j >> 7);
    v = radem_bit(w, static_cast<int>(j & 127)) ? -1.0 : 1.0;
  } else {
    int h, neg;
    count_hash(seed, j, k, h, neg);
    v = (h == i) ? (neg ? -1.0 : 1.0) : 0.0;
  }
  out[idx] = v;
}

// ----------------------------------------------------------------------------
// Dense sketch.
constexpr int kSkRows = 16;  // rows of X per LDS stage

template <typename TX, int NB>
__global__ __launch_bounds__(256, 2) void sketch_dense_kernel(const TX* __restrict__ X, int64_t m,
                                                           int n, int64_t ldx, int kind,
                                                           uint64_t seed, int ktiles,
                                                           int64_t rows_per_split, int kpad,
                                                           double* __restrict__ part) {
  constexpr int NP = NB * 16;
  // Stages of 16 rows, double buffered: while the matrix cores work on
  // stage i, the X loads of stage i + 2 are in flight in registers and stage
  // i + 1 (its X and this wave's Theta block) is already in LDS.
  __shared__ double xs[2][kSkRows][NP + 1];
  __shared__ double zs[2][4][kSkRows][16];

  // XCD-aware decode: workgroup ids are dealt round-robin to the 8 XCDs;
  // consecutive ids on one XCD walk the Theta tiles of one row range.
  const int bid = blockIdx.x;
  const int xcd = bid & 7, slot = bid >> 3;
  const int t = slot % ktiles;
  const int s = (slot / ktiles) * 8 + xcd;

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  const int ibase = t * 64 + wave * 16;  // first Theta row of this wave
  const int64_t r_begin = static_cast<int64_t>(s) * rows_per_split;
  const int64_t r_end = (r_begin + rows_per_split < m) ? r_begin + rows_per_split : m;

  d4 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = d4{0.0, 0.0, 0.0, 0.0};
  Words rw{0u, 0u, 0u, 0u};  // Rademacher words of this lane's Theta row
  int64_t rblk = -1;

  // X prefetch: element e of thread t is row t % 16, column t / 16 + 16 e.
  const int pjj = threadIdx.x & 15, pc0 = threadIdx.x >> 4;
  TX pre[NB];
  auto fetch = [&](int64_t r0) {
    const int64_t row = r0 + pjj;
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int c = pc0 + 16 * e;
      pre[e] = (row < r_end && c < n) ? X[row + static_cast<int64_t>(c) * ldx] : TX(0);
    }
  };
  auto put = [&](int buf) {
#pragma unroll
    for (int e = 0; e < NB; ++e) xs[buf][pjj][pc0 + 16 * e] = static_cast<double>(pre[e]);
  };
  // Theta(ibase:ibase+16, r0:r0+16) for this wave.
  auto gen = [&](int64_t r0, int buf) {
    if (kind == kGaussian) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int pi = lane + 64 * h;  // 128 pairs: 8 row pairs x 16 columns
        const int ip = pi & 7, jj = pi >> 3;
        const int64_t row = r0 + jj;
        double z0 = 0.0, z1 = 0.0;
        if (row < r_end) gauss_pair(seed, row, static_cast<uint32_t>((ibase >> 1) + ip), z0, z1);
        zs[buf][wave][jj][2 * ip] = z0;
        zs[buf][wave][jj][2 * ip + 1] = z1;
      }
    } else {
      // Lane: Theta row ibase + (lane & 15), rows jj0..jj0+3 of the stage.
      // The row's words cover a 128-row block of X; a 16-row stage never
      // straddles two blocks (stages start at multiples of 16).
      const int ii = lane & 15, jj0 = 4 * (lane >> 4);
      const int64_t blk = r0 >> 7;
      if (blk != rblk) {
        rw = radem_words(seed, ibase + ii, blk);
        rblk = blk;
      }
      const int o = static_cast<int>(r0 & 127) + jj0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = r0 + jj0 + e;
        zs[buf][wave][jj0 + e][ii] = (row < r_end) ? (radem_bit(rw, o + e) ? -1.0 : 1.0) : 0.0;
      }
    }
  };
  if (r_begin < r_end) {
    fetch(r_begin);
    put(0);
    gen(r_begin, 0);
    if (r_begin + kSkRows < r_end) fetch(r_begin + kSkRows);
  }
  __syncthreads();
  int cur = 0;
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kSkRows) {
#pragma unroll
    for (int ks = 0; ks < kSkRows / 4; ++ks) {
      const double a = zs[cur][wave][4 * ks + lg][l16];
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] = mfma16x16x4(a, xs[cur][4 * ks + lg][16 * b + l16], acc[b]);
    }
    const int64_t r1 = r0 + kSkRows;
    if (r1 < r_end) {
      put(cur ^ 1);
      gen(r1, cur ^ 1);
      if (r1 + kSkRows < r_end) fetch(r1 + kSkRows);
    }
    __syncthreads();
    cur ^= 1;
  }
  // Partial layout: part[s][c][i], ld = kpad, for c < NP.
  double* dst = part + static_cast<int64_t>(s) * NP * kpad;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      dst[static_cast<int64_t>(16 * b + l16) * kpad + ibase + drow<double>(lg, v)] = acc[b][v];
}

// P(i, c) = scale * sum_s part[s][c][i], s ascending.
__global__ void sketch_reduce_kernel(const double* __restrict__ part, int nsplit, int k, int n,
                                     int kpad, int npad, double scale, double* __restrict__ P,
                                     int64_t ldp) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(k) * n) return;
  const int i = static_cast<int>(idx % k), c = static_cast<int>(idx / k);
  const int64_t stride = static_cast<int64_t>(npad) * kpad;
  const double* p = part + static_cast<int64_t>(c) * kpad + i;
  P[i + c * ldp] = scale * ordered_sum(p, nsplit, stride);
}

// ----------------------------------------------------------------------------
// CountSketch.
constexpr int kCsTile = 256;
constexpr int kCsCols = 8;

// For each tile of 256 rows: key(t) = (h(j) << 9) | (s(j) << 8) | t, stored
// at the row's position in the tile sorted by bucket (stable in t).  Rows
// past m get bucket 0x7ff and sort last.
__global__ __launch_bounds__(256) void count_prep_kernel(int64_t m, int k, uint64_t seed,
                                                         uint32_t* __restrict__ keys) {
  __shared__ int hs[kCsTile];
  const int t = threadIdx.x;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kCsTile + t;
  int h = 0x7ff, neg = 0;
  if (j < m) count_hash(seed, j, k, h, neg);
  hs[t] = h;
  __syncthreads();
  int pos = 0;
  for (int u = 0; u < kCsTile; ++u) {
    const int hu = hs[u];
    pos += (hu < h) || (hu == h && u < t);
  }
  keys[static_cast<int64_t>(blockIdx.x) * kCsTile + pos] =
      (static_cast<uint32_t>(h) << 9) | (static_cast<uint32_t>(neg) << 8) | static_cast<uint32_t>(t);
}

template <typename TX>
__global__ __launch_bounds__(256) void count_accum_kernel(const TX* __restrict__ X, int64_t m,
                                                          int n, int64_t ldx, int k,
                                                          const uint32_t* __restrict__ keys,
                                                          int64_t tiles_per_split, int kpad,
                                                          int npad, double* __restrict__ part) {
  extern __shared__ double smem[];
  double* acc = smem;                     // [kpad][kCsCols]
  double* xs = smem + kpad * kCsCols;     // [kCsTile][kCsCols + 1]
  __shared__ uint32_t ks[kCsTile];
  const int panel = blockIdx.x;           // columns panel*8 .. panel*8+7
  const int s = blockIdx.y;
  const int c0 = panel * kCsCols;
  const int t = threadIdx.x;
  for (int idx = t; idx < kpad * kCsCols; idx += 256) acc[idx] = 0.0;
  const int64_t ntile = ceil_div(m, kCsTile);
  const int64_t tb = s * tiles_per_split;
  const int64_t te = (tb + tiles_per_split < ntile) ? tb + tiles_per_split : ntile;
  for (int64_t tile = tb; tile < te; ++tile) {
    __syncthreads();
    const int64_t row = tile * kCsTile + t;
#pragma unroll
    for (int c = 0; c < kCsCols; ++c) {
      double v = 0.0;
      if (row < m && c0 + c < n) v = static_cast<double>(X[row + static_cast<int64_t>(c0 + c) * ldx]);
      xs[t * (kCsCols + 1) + c] = v;
    }
    ks[t] = keys[tile * kCsTile + t];
    __syncthreads();
    const uint32_t key = ks[t];
    const int h = static_cast<int>(key >> 9);
    const bool head = (h < k) && (t == 0 || static_cast<int>(ks[t - 1] >> 9) != h);
    if (head) {
      double sum[kCsCols];
#pragma unroll
      for (int c = 0; c < kCsCols; ++c) sum[c] = 0.0;
      for (int p = t; p < kCsTile && static_cast<int>(ks[p] >> 9) == h; ++p) {
        const uint32_t kp = ks[p];
        const int src = static_cast<int>(kp & 255u);
        const bool neg = (kp >> 8) & 1u;
#pragma unroll
        for (int c = 0; c < kCsCols; ++c) {
          const double x = xs[src * (kCsCols + 1) + c];
          sum[c] += neg ? -x : x;
        }
      }
#pragma unroll
      for (int c = 0; c < kCsCols; ++c) acc[h * kCsCols + c] += sum[c];
    }
  }
  __syncthreads();
  double* dst = part + static_cast<int64_t>(s) * npad * kpad;
  for (int idx = t; idx < k * kCsCols; idx += 256) {
    const int i = idx % k, c = idx / k;
    if (c0 + c < npad) dst[static_cast<int64_t>(c0 + c) * kpad + i] = acc[i * kCsCols + c];
  }
}

// ----------------------------------------------------------------------------
// Host-side launchers.

hipError_t launch_theta_debug(int kind, int k, int64_t m, uint64_t seed, int64_t i0, int64_t ni,
                              int64_t j0, int64_t nj, double* out, hipStream_t st) {
  const int64_t total = ni * nj;
  if (total == 0) return hipSuccess;
  theta_debug_kernel<<<static_cast<unsigned>(ceil_div(total, 256)), 256, 0, st>>>(
      kind, k, m, seed, i0, ni, j0, nj, out);
  return hipGetLastError();
}

template <typename TX>
static hipError_t dense_dispatch(int nb, const TX* X, int64_t m, int n, int64_t ldx, int kind,
                                 uint64_t seed, const SketchPlan& pl, double* part,
                                 hipStream_t st) {
  const dim3 grid(pl.nsplit * pl.ktiles), block(256);
#define RCQ_SK_CASE(NBV)                                                                         \
  case NBV:                                                                                      \
    sketch_dense_kernel<TX, NBV><<<grid, block, 0, st>>>(X, m, n, ldx, kind, seed, pl.ktiles,    \
                                                         pl.rows_per_split, pl.kpad, part);      \
    break;
  switch (nb) {
    RCQ_SK_CASE(1) RCQ_SK_CASE(2) RCQ_SK_CASE(3) RCQ_SK_CASE(4) RCQ_SK_CASE(5) RCQ_SK_CASE(6)
    RCQ_SK_CASE(7) RCQ_SK_CASE(8) RCQ_SK_CASE(9) RCQ_SK_CASE(10) RCQ_SK_CASE(11) RCQ_SK_CASE(12)
    RCQ_SK_CASE(13) RCQ_SK_CASE(14) RCQ_SK_CASE(15) RCQ_SK_CASE(16)
    default: return hipErrorInvalidValue;
  }
#undef RCQ_SK_CASE
  return hipGetLastError();
}

hipError_t launch_sketch_partials(const void* X, bool x_is_f32, int64_t m, int n, int64_t ldx,
                                  int k, int kind, uint64_t seed, const SketchPlan& pl,
                                  double* part, uint32_t* keys, hipStream_t st) {
  hipError_t e;
  if (kind == kSRHT) return launch_sketch_srht_partials(X, x_is_f32, m, n, ldx, k, seed, pl, part, st);
  if (kind == kCountSketch) {
    const int64_t ntile = ceil_div(m, kCsTile);
    count_prep_kernel<<<static_cast<unsigned>(ntile), kCsTile, 0, st>>>(m, k, seed, keys);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const dim3 grid(static_cast<unsigned>(ceil_div(n, kCsCols)), pl.nsplit);
    const size_t shm = (static_cast<size_t>(pl.kpad) * kCsCols + kCsTile * (kCsCols + 1)) * sizeof(double);
    static bool attr_done = false;
    if (!attr_done) {
      const int mx = static_cast<int>((static_cast<size_t>(kMaxK) * kCsCols + kCsTile * (kCsCols + 1)) * sizeof(double));
      if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(count_accum_kernel<float>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, mx)) != hipSuccess)
        return e;
      if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(count_accum_kernel<double>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, mx)) != hipSuccess)
        return e;
      attr_done = true;
    }
    if (x_is_f32)
      count_accum_kernel<float><<<grid, 256, shm, st>>>(static_cast<const float*>(X), m, n, ldx, k,
                                                        keys, pl.rows_per_split / kCsTile, pl.kpad,
                                                        pl.npad, part);
    else
      count_accum_kernel<double><<<grid, 256, shm, st>>>(static_cast<const double*>(X), m, n, ldx,
                                                         k, keys, pl.rows_per_split / kCsTile,
                                                         pl.kpad, pl.npad, part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  } else {
    const int nb = static_cast<int>(ceil_div(n, 16));
    if (x_is_f32)
      e = dense_dispatch<float>(nb, static_cast<const float*>(X), m, n, ldx, kind, seed, pl, part, st);
    else
      e = dense_dispatch<double>(nb, static_cast<const double*>(X), m, n, ldx, kind, seed, pl, part, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_sketch(const void* X, bool x_is_f32, int64_t m, int n, int64_t ldx, int k,
                         int kind, uint64_t seed, const SketchPlan& pl, double* part,
                         uint32_t* keys, double* P, int64_t ldp, hipStream_t st) {
  const hipError_t e = launch_sketch_partials(X, x_is_f32, m, n, ldx, k, kind, seed, pl, part, keys, st);
  if (e != hipSuccess) return e;
  const double scale = (kind == kCountSketch) ? 1.0 : 1.0 / sqrt(static_cast<double>(k));
  return launch_sketch_reduce(part, pl, k, n, scale, P, ldp, st);
}

// Theta = I (the test-only embedding): P = X, FP32 values promoted exactly.
template <typename TX>
__global__ void sketch_identity_kernel(const TX* __restrict__ X, int64_t m, int n, int64_t ldx,
                                       double* __restrict__ P, int64_t ldp) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= m * n) return;
  const int64_t i = idx % m, c = idx / m;
  P[i + c * ldp] = static_cast<double>(X[i + c * ldx]);
}

hipError_t launch_sketch_identity(const void* X, bool x_is_f32, int64_t m, int n, int64_t ldx,
                                  double* P, int64_t ldp, hipStream_t st) {
  const unsigned grid = static_cast<unsigned>(ceil_div(m * n, 256));
  if (x_is_f32)
    sketch_identity_kernel<float><<<grid, 256, 0, st>>>(static_cast<const float*>(X), m, n, ldx, P, ldp);
  else
    sketch_identity_kernel<double><<<grid, 256, 0, st>>>(static_cast<const double*>(X), m, n, ldx, P, ldp);
  return hipGetLastError();
}

hipError_t launch_sketch_reduce(const double* part, const SketchPlan& pl, int k, int n,
                                double scale, double* P, int64_t ldp, hipStream_t st) {
  const int64_t total = static_cast<int64_t>(k) * n;
  sketch_reduce_kernel<<<static_cast<unsigned>(ceil_div(total, 256)), 256, 0, st>>>(
      part, pl.nsplit, k, n, pl.kpad, pl.npad, scale, P, ldp);
  return hipGetLastError();
}

}  // namespace rcq
