// srht.hip -- the SRHT sketch P = Theta X by blocked fast Walsh-Hadamard
// transforms, in one pass over X (Section 2: the SRHT costs O(m n log m)
// through the fast transform; Section 3.3).
//
// Theta = sqrt(m'/k) S H D with the raw entry d_j (-1)^popcount(s_i & j)
// (theta.h).  Split a row index as j = 256 j1 + j2 and a sample as
// s = 256 s1 + s2; the parity splits the same way, so
//   sum_j d_j (-1)^popcount(s & j) X_j
//     = sum_j1 (-1)^popcount(s1 & j1) Y_j1[s2],
//   Y_j1 = H_256 (d .* X rows 256 j1 .. 256 j1 + 255),
// the 256-point Walsh-Hadamard transform (Sylvester order) of one sign-
// flipped row block.  A workgroup streams a range of row blocks for 16
// columns: each block is transformed (8 butterfly levels, 4 in registers
// over 16 consecutive rows, a padded LDS transpose, 4 more over rows 16
// apart), written to LDS, and every sample i adds +-Y[s2_i] to its FP64 sum.
// Per element: 8 additions for the transform and k/256 for the samples,
// against k multiply-adds for a dense sketch.  All arithmetic is FP64 (FP32
// X is promoted exactly), so the transform and the sums over blocks round
// at 2^-53; the per-range sums are reduced in a fixed order afterwards.
#include "common.h"
#include "kernels.h"
#include "theta.h"

namespace rcq {

constexpr int kFwB = 256;      // rows per transform block
constexpr int kFwC = 16;       // columns per workgroup
constexpr int kFwZLd = 272;    // doubles per column of the transpose buffer (2176 B)
constexpr int kFwYLd = 257;    // doubles per column of the transformed block
constexpr int kFwDChunk = 32;  // blocks per table of d words

// LDS of one workgroup.  Both block buffers are padded so that their
// accesses are affine (immediate offsets).  Row r of a column of z sits at
// 17 (r >> 4) + (r & 15), so 16 consecutive rows (written by one lane) and
// rows 16 apart (read by 16 lanes) both spread over the banks without
// conflicts.  y is column-major with an odd stride, so that the 16 columns
// of one sample's row, read by 16 lanes, fall in distinct banks; the two
// samples of a half-wave can still share banks, and its writes pair two
// columns on one bank group.  (17-double rows, conflict-free for the
// writes, measured 0.43 ms slower: two samples of a half-wave then collide
// far more often.)
struct FwhtLds {
  double z[kFwC][kFwZLd];        // first-stage results
  double y[kFwC][kFwYLd];        // transformed block
  double sg[kMaxK];              // +-1 of each sample for the current block
  int s2[kMaxK];                 // low 8 bits of each sample
  uint32_t dt[kFwDChunk][2][4];  // d words of the next 32 blocks (two halves each)
};

// Splits of the row blocks for k, n (the workspace layout uses the same).
void srht_sketch_plan(int64_t m, int k, int n, SketchPlan& sp) {
  const int64_t nblk = ceil_div(m, kFwB);
  const int ncg = static_cast<int>(ceil_div(n, kFwC));
  int64_t ns = ceil_div(512, ncg);  // about two workgroups per compute unit
  if (ns > nblk) ns = nblk;
  if (ns < 1) ns = 1;
  const int64_t bps = ceil_div(nblk, ns);
  sp.rows_per_split = bps * kFwB;
  sp.nsplit = static_cast<int>(ceil_div(nblk, bps));
  sp.ktiles = 0;
  sp.kpad = static_cast<int>(round_up(k, 16));
  sp.npad = static_cast<int>(round_up(n, 16));
}

// Workgroup (column group blockIdx.x, row range blockIdx.y).  KR >= k / 16:
// the samples per thread in the accumulation.
// VEC: X 16-byte aligned with ld a multiple of 16 bytes (whole blocks load
// by 16-byte vectors).
template <typename TX, int KR, bool VEC>
__global__ __launch_bounds__(256, 2) void srht_fwht_kernel(const TX* __restrict__ X, int64_t m,
                                                           int n, int64_t ldx, int k,
                                                           uint64_t seed, int L,
                                                           int64_t blocks_per_split, int kpad,
                                                           int npad, double* __restrict__ part) {
  extern __shared__ __align__(16) unsigned char fw_smem[];
  FwhtLds& sh = *reinterpret_cast<FwhtLds*>(fw_smem);
  const int t = threadIdx.x;
  const int cg = blockIdx.x, s = blockIdx.y;
  const int c0 = kFwC * cg;
  const int64_t nblk = (m + kFwB - 1) / kFwB;
  const int64_t b0 = static_cast<int64_t>(s) * blocks_per_split;
  const int64_t b1 = b0 + blocks_per_split < nblk ? b0 + blocks_per_split : nblk;

  // Transform role: column c, rows 16 u .. 16 u + 15 of a block.
  const int c = t >> 4, u = t & 15;
  const int col = c0 + c < n ? c0 + c : n - 1;
  const bool col_live = c0 + c < n;
  const TX* xcol = X + static_cast<int64_t>(col) * ldx + 16 * u;
  // Accumulation role: column cc, samples sgp + 16 r.
  const int cc = t & 15, sgp = t >> 4;

  // Samples: s2 into LDS; s1 (the high part) kept by the thread that forms
  // the signs of samples t, t + 256, ...
  // Slots k .. 16 KR - 1 (no sample) read Y[0] with sign 0, so that the
  // accumulation below has no per-sample condition.
  constexpr int kSgPer = kMaxK / 256;
  uint64_t s1[kSgPer];
#pragma unroll
  for (int q = 0; q < kSgPer; ++q) {
    const int i = t + 256 * q;
    s1[q] = 0;
    if (i < k) {
      const uint64_t sv = srht_row(seed, i, L);
      sh.s2[i] = static_cast<int>(sv & (kFwB - 1));
      s1[q] = sv >> 8;
    } else if (i < 16 * KR) {
      sh.s2[i] = 0;
      sh.sg[i] = 0.0;
    }
  }
  // d words of blocks blk .. blk + 31 (two Philox draws each, one per
  // 128-row half), drawn by the 64 lanes of wave 0 in one pass.
  auto d_table = [&](int64_t blk) {
    if (t < 2 * kFwDChunk) {
      const int64_t b = blk + (t >> 1);
      if (b < b1) {
        const Words w = theta_words(seed, 2 * b + (t & 1), 0u, kTagSrhtD);
        uint32_t* d = sh.dt[t >> 1][t & 1];
        d[0] = w.w0;
        d[1] = w.w1;
        d[2] = w.w2;
        d[3] = w.w3;
      }
    }
  };

  // Rows of the block starting at row r0 (zero past m).
  TX xn[16];
  auto load = [&](int64_t blk) {
    const int64_t r0 = blk * kFwB;
    if (r0 + kFwB <= m) {
      if (VEC) {
        typedef TX v2 __attribute__((ext_vector_type(16 / sizeof(TX))));
        constexpr int W = 16 / sizeof(TX);
#pragma unroll
        for (int e = 0; e < 16; e += W) {
          const v2 f = *reinterpret_cast<const v2*>(xcol + r0 + e);
#pragma unroll
          for (int w = 0; w < W; ++w) xn[e + w] = f[w];
        }
      } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) xn[e] = xcol[r0 + e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t r = r0 + 16 * u + e;
        xn[e] = r < m ? xcol[r0 + e] : TX(0);
      }
    }
  };

  double acc[KR];
#pragma unroll
  for (int r = 0; r < KR; ++r) acc[r] = 0.0;

  if (b0 < b1) load(b0);
  __syncthreads();  // the sample table
  // Up to 48 samples per thread, the LDS index of each sample's Y entry is
  // formed once and kept (the accumulation then issues independent reads);
  // with more samples it is formed from the s2 table every block.
  constexpr bool kKeep = KR <= 48;
  int yo[kKeep ? KR : 1];
  if (kKeep) {
#pragma unroll
    for (int r = 0; r < KR; ++r) {
      const int v = sh.s2[sgp + 16 * r];
      yo[r] = 8 * (kFwYLd * cc + v);  // byte offset in y
    }
  }
  for (int64_t blk = b0; blk < b1; ++blk) {
    // The thread's indices as fresh values each block: the LDS addresses
    // below are then formed where they are used, not kept in registers
    // across the loop.
    int tt = t;
    asm volatile("" : "+v"(tt));
    const int uu = tt & 15;
    if (((blk - b0) & (kFwDChunk - 1)) == 0) {
      // the previous table's last reads are behind the block's first barrier
      d_table(blk);
      __syncthreads();
    }
    // 1. this block's rows (signs d_j applied), next block's loads issued
    double x[16];
    {
      // row 16 u + e of the block: half u >> 3, word (u & 7) >> 1, bit
      // 8 e' + t' with t' = 4 (u & 1) + (e >> 2), e' = e & 3 (radem_bit's
      // layout); bit b set -> the sign bit of the value flipped
      const uint32_t w = sh.dt[(blk - b0) & (kFwDChunk - 1)][uu >> 3][(uu & 7) >> 1] >>
                         (4 * (uu & 1));
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int b = 8 * (e & 3) + (e >> 2);
        const uint32_t flip = (w << (31 - b)) & 0x80000000u;
        const double v = col_live ? static_cast<double>(xn[e]) : 0.0;
        const uint64_t vb = static_cast<uint64_t>(__double_as_longlong(v)) ^
                            (static_cast<uint64_t>(flip) << 32);
        x[e] = __longlong_as_double(static_cast<long long>(vb));
      }
    }
    if (blk + 1 < b1) load(blk + 1);
    // 2. butterflies over the low four row bits, in registers
#pragma unroll
    for (int st = 1; st < 16; st <<= 1)
#pragma unroll
      for (int e = 0; e < 16; ++e)
        if ((e & st) == 0) {
          const double a = x[e], b = x[e + st];
          x[e] = a + b;
          x[e + st] = a - b;
        }
#pragma unroll
    for (int e = 0; e < 16; ++e) sh.z[c][17 * uu + e] = x[e];
    __syncthreads();
    // 3. rows u + 16 q, butterflies over the high four row bits; the
    // transformed block to LDS and the samples' signs for this block
#pragma unroll
    for (int q = 0; q < 16; ++q) x[q] = sh.z[c][17 * q + uu];
#pragma unroll
    for (int st = 1; st < 16; st <<= 1)
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if ((q & st) == 0) {
          const double a = x[q], b = x[q + st];
          x[q] = a + b;
          x[q + st] = a - b;
        }
#pragma unroll
    for (int q = 0; q < 16; ++q) sh.y[c][uu + 16 * q] = x[q];
#pragma unroll
    for (int q = 0; q < kSgPer; ++q) {
      const int i = tt + 256 * q;
      if (i < k)
        sh.sg[i] = (__builtin_popcountll(s1[q] & static_cast<uint64_t>(blk)) & 1) ? -1.0 : 1.0;
    }
    __syncthreads();
    // 4. every sample adds +-Y[s2]
    const int ccl = tt & 15, sgl = tt >> 4;
    const char* yb = reinterpret_cast<const char*>(sh.y);
#pragma unroll
    for (int r = 0; r < KR; ++r) {
      const int i = sgl + 16 * r;
      int o;
      if (kKeep) {
        o = yo[r];
      } else {
        o = 8 * (kFwYLd * ccl + sh.s2[i]);
      }
      acc[r] = __builtin_fma(sh.sg[i], *reinterpret_cast<const double*>(yb + o), acc[r]);
      // sixteen samples' reads in flight at a time (bounds the registers)
      if ((r & 15) == 15) __builtin_amdgcn_sched_barrier(0);
    }
  }
  double* dst = part + (static_cast<int64_t>(s) * npad + c0 + cc) * kpad;
#pragma unroll
  for (int r = 0; r < KR; ++r) {
    const int i = sgp + 16 * r;
    if (i < k) dst[i] = acc[r];
  }
}

hipError_t launch_sketch_srht_partials(const void* X, bool x_is_f32, int64_t m, int n,
                                       int64_t ldx, int k, uint64_t seed, const SketchPlan& pl,
                                       double* part, hipStream_t st) {
  if (k < 1 || k > kMaxK || n < 1) return hipErrorInvalidValue;
  const int64_t nblk = ceil_div(m, kFwB);
  const int64_t bps = pl.rows_per_split / kFwB;
  if (pl.rows_per_split % kFwB != 0 || bps < 1 || ceil_div(nblk, bps) != pl.nsplit ||
      pl.kpad < k || pl.npad < static_cast<int>(round_up(n, kFwC)))
    return hipErrorInvalidValue;
  const int L = srht_log2(m);
  const dim3 grid(static_cast<unsigned>(ceil_div(n, kFwC)), static_cast<unsigned>(pl.nsplit));
  const size_t esz = x_is_f32 ? sizeof(float) : sizeof(double);
  const bool vec = (reinterpret_cast<uintptr_t>(X) & 15) == 0 && ((ldx * esz) & 15) == 0;
  hipError_t e = hipSuccess;
#define RCQ_FW(TX, KRV, VV)                                                                    \
  do {                                                                                         \
    const void* fn = reinterpret_cast<const void*>(&srht_fwht_kernel<TX, KRV, VV>);            \
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,                    \
                            static_cast<int>(sizeof(FwhtLds)));                                \
    if (e != hipSuccess) return e;                                                             \
    srht_fwht_kernel<TX, KRV, VV><<<grid, 256, sizeof(FwhtLds), st>>>(                         \
        static_cast<const TX*>(X), m, n, ldx, k, seed, L, bps, pl.kpad, pl.npad, part);        \
  } while (0)
#define RCQ_FW_V(TX, KRV)   \
  if (vec)                  \
    RCQ_FW(TX, KRV, true);  \
  else                      \
    RCQ_FW(TX, KRV, false);
#define RCQ_FW_K(TX)        \
  if (k <= 256) {           \
    RCQ_FW_V(TX, 16)        \
  } else if (k <= 512) {    \
    RCQ_FW_V(TX, 32)        \
  } else if (k <= 768) {    \
    RCQ_FW_V(TX, 48)        \
  } else {                  \
    RCQ_FW_V(TX, 64)        \
  }
  if (x_is_f32) {
    RCQ_FW_K(float)
  } else {
    RCQ_FW_K(double)
  }
#undef RCQ_FW_K
#undef RCQ_FW_V
#undef RCQ_FW
  return hipGetLastError();
}

}  // namespace rcq
