// mixed.hip -- Rademacher sketch P = Theta X for FP32 X on int8 matrix cores
// (the +-1 entries are exact in int8; the SRHT sketch takes the blocked fast
// transform of srht.hip in every precision).
//
// Section 5 asks for the sketch to be computed more accurately than the
// working precision.  Here the products Theta X are exact integer sums:
//   * Theta entries are +-1, exact in int8 (the 1/sqrt(k) goes on P).
//   * Each column of X is quantised to integers q = rint(x 2^s), with a power
//     of two 2^s that keeps the column's running maximum in [2^20, 2^22), so
//     |x - q 2^-s| <= 2^-21 max|x| over the rows seen; q is split into three
//     signed bytes, q = 2^16 h + 2^8 d + l.
//   * v_mfma_i32_16x16x64_i8 accumulates Theta h, Theta d and Theta l in
//     three int32 accumulators, exactly (|sum| < 2^31 for up to 2^24 rows).
//   * A column's accumulators are folded into its FP64 partial only when the
//     column's scale has to grow (rare: the maximum must double twice) and
//     at the end: part += (2^16 H + 2^8 D + L) 2^-s, exact in FP64.
// The only rounding in P is therefore the quantisation of X and the FP64
// sum over row splits: the result is bitwise reproducible.
//
// Quantiser: y = fma(x, 2^s, 1.5 2^23) holds rint(x 2^s) + 2^22 in its
// mantissa; adding 0x408080 - 0x4B000000 to its bits leaves 0 in the top
// byte and l + 128, d + 128, h + 128 in the low three bytes, and XOR 0x80
// per byte turns each into its signed digit.  A non-finite x leaves a
// non-zero top byte, which marks the workgroup's partials NaN.
//
// Theta from Philox bits: a Rademacher draw of Theta row i covers 128 rows
// of X, with rows 4t..4t+3 of each 32 at bit t of the four bytes of a word
// (theta.h), so one rotate, one AND and one byte permute give four +-1
// bytes of an A operand.
//
// Work split: a workgroup of wt x wc waves streams one row split of X in
// stages of 128 rows (one Philox block) for Tg = 64 wt Theta rows and
// Cg = 16 CT wc columns.  Per stage every thread quantises 16 rows of one
// column into three LDS digit planes and threads 0..Tg-1 draw their Theta
// row's words; then each wave (TT = 4 Theta tiles x CT column tiles, 3 TT CT
// int32 tiles) issues two matrix-core steps of 64 rows.  The matrix-core
// K slot (lane group g, byte 4t + e) carries row 16g + 4t + e of the step in
// both operands.
#include "common.h"
#include "theta.h"
#include "kernels.h"

namespace rcq {

constexpr int kQBlock = 128;                 // rows of X per Philox block
constexpr int kQZs = 5;                      // LDS words per Theta row and block (4 + pad)
constexpr float kQMagic = 12582912.0f;       // 1.5 * 2^23
constexpr uint32_t kQDigitBias = 0xB5408080u;  // 0x408080 - 0x4B000000 (mod 2^32)
constexpr int kQUnset = -100000;             // column scale not chosen yet

typedef int i4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float pow2f(int s) { return __int_as_float((s + 127) << 23); }

__device__ __forceinline__ uint32_t bperm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

// Maximum over aligned groups of G (8 or 16) consecutive lanes, with DPP
// lane swaps (quad swaps, then mirrors within 8- and 16-lane rows).
template <int G>
__device__ __forceinline__ float group_max(float v) {
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false)));
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false)));
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, false)));
  if (G == 16)
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x140, 0xF, 0xF, false)));
  return v;
}

// TT, CT: Theta and column tiles (16) per wave.  SB: Philox blocks (128
// rows) per stage.  NSL: quantiser task slots per thread.  FULL: the tasks
// fill every slot of every thread (no per-slot guards) and the stage's
// matrix-core steps are interleaved with the next stage's quantisation.
template <int TT, int CT, int SB, int NSL, bool FULL>
__global__ __launch_bounds__(512, 1) void sketch_i8_kernel(
    const float* __restrict__ X, int64_t m, int n, int64_t ldx, int k, uint64_t seed, int wt,
    int wc, int ktiles, int nh, int64_t rows_per_split, int kpad, int npad,
    double* __restrict__ part) {
  constexpr int S = kQBlock * SB;  // rows per stage
  constexpr int KS = S / 64;       // matrix-core steps per stage
  // LDS bytes per column of a digit plane: 2 mod 16 chunks of 16 bytes, so
  // that a matrix-core operand read (16 columns x 4 row chunks of 16 bytes)
  // is free of bank conflicts on gfx950 (a stride of 1 mod 16 chunks costs 4
  // extra cycles per read, measured).
  constexpr int LD = S + 32;
  constexpr int G = S / 16;        // quantiser row groups per column
  extern __shared__ __align__(16) unsigned char smem[];
  const int Tg = wt * TT * 16, Cg = wc * CT * 16;
  const int dig_sz = 3 * Cg * LD;           // bytes of one digit buffer
  const int zb_sz = Tg * SB * kQZs;         // words of one Philox buffer
  unsigned char* dig = smem;                                           // [2][3][Cg][LD]
  uint32_t* zb = reinterpret_cast<uint32_t*>(smem + 2 * dig_sz);      // [2][SB][Tg][kQZs]
  int* colexp = reinterpret_cast<int*>(zb + 2 * zb_sz);               // [2][Cg]
  int* badflag = colexp + 2 * Cg;

  // XCD-aware decode: ids are dealt round-robin to the 8 XCDs; consecutive
  // ids on one XCD walk the Theta and column groups of one row split.
  const int bid = blockIdx.x;
  const int xcd = bid & 7, slot = bid >> 3;
  const int tps = ktiles * nh;
  const int jt = slot % tps;
  const int tgi = jt % ktiles, h = jt / ktiles;
  const int s = (slot / tps) * 8 + xcd;

  const int nthr = static_cast<int>(blockDim.x);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  const int wrow = wave % wt, wcol = wave / wt;
  const int c0 = h * Cg, theta0 = tgi * Tg;
  // Split s takes the stages s, s + nsplit, s + 2 nsplit, ...: at any time
  // the running workgroups read one contiguous band of rows (long runs per
  // column).  rows_per_split bounds the rows a split sums (int32 range).
  (void)rows_per_split;
  const int64_t sstride = static_cast<int64_t>(gridDim.x / (ktiles * nh)) * S;
  const int64_t r_begin = static_cast<int64_t>(s) * S;
  const int64_t r_end = m;
  const int ntask = G * Cg;  // quantiser task: 16 rows (group g) of one column
  const bool vec = ((ldx & 3) == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);

  if (tid < 2 * Cg) colexp[tid] = kQUnset;
  if (tid == 0) *badflag = 0;

  // Quantiser state: NSL task slots per thread.  Task (column group cg,
  // lane g of the column's G lanes) covers the 4-row groups G v + g (v < 4) of the
  // stage, so that each load instruction reads 16 G contiguous bytes of a
  // column.  A task's column is fixed, so its scale exponent sq persists
  // across stages.  Columns past n read column n - 1 (their sums are never
  // used).
  float xv[NSL][16];
  int sq[NSL];
  int qcol[NSL], qg[NSL];
  const float* qsrc[NSL];
#pragma unroll
  for (int sl = 0; sl < NSL; ++sl) {
    sq[sl] = kQUnset;
    const int task = tid + sl * nthr;
    // The four column groups of a wave take columns 2 apart (within each
    // 16 columns, bits b3 b2 b1 b0 of the group become b3 b1 b0 b2), so that
    // their digit writes (column stride 72 words) fall in distinct banks.
    const int cg = task / G;
    qcol[sl] = (G == 16)
                   ? ((cg & ~15) | ((cg & 3) << 1) | ((cg >> 2) & 1) | (cg & 8))
                   : cg;
    qg[sl] = task % G;
    const int c = (c0 + qcol[sl] < n) ? c0 + qcol[sl] : n - 1;
    qsrc[sl] = X + static_cast<int64_t>(c) * ldx + 4 * qg[sl];
  }
  uint32_t orv = 0;

  // Load slot sl's rows of the stage starting at row r0 (nothing past the
  // split; rows past it read as zero).
  auto load_slot = [&](int sl, int64_t r0) {
    if (!FULL && tid + sl * nthr >= ntask) return;
    if (r0 >= r_end) return;
    const float* src = qsrc[sl] + r0;
    if (vec && r0 + S <= r_end) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float4 f = *reinterpret_cast<const float4*>(src + 4 * G * v);
        xv[sl][4 * v] = f.x;
        xv[sl][4 * v + 1] = f.y;
        xv[sl][4 * v + 2] = f.z;
        xv[sl][4 * v + 3] = f.w;
      }
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t off = 4 * G * v + e;
          xv[sl][4 * v + e] = (r0 + 4 * qg[sl] + off < r_end) ? src[off] : 0.f;
        }
    }
  };
  auto load_stage = [&](int64_t r0) {
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) load_slot(sl, r0);
  };

  // Quantiser, first part: the column's stage maximum (every lane of the
  // column's group agrees on it), scale growth, and the scale of slot sl.
  auto qscale = [&](int sl, int buf) -> float {
    float mx = 0.f;
#pragma unroll
    for (int e = 0; e < 16; ++e) mx = fmaxf(mx, fabsf(xv[sl][e]));
    mx = group_max<G>(mx);
    const int ex = static_cast<int>((__float_as_uint(mx) >> 23) & 0xffu) - 127;
    const int sn = min(max(20 - ex, -126), 126);
    const int sc = sq[sl];
    const bool grow = (mx > 0.f) & ((sc == kQUnset) | (ex >= 22 - sc));
    sq[sl] = grow ? sn : sc;
    if (qg[sl] == 0) colexp[buf * Cg + qcol[sl]] = sq[sl];
    return pow2f(sq[sl] == kQUnset ? 0 : sq[sl]);
  };
  // Quantiser, second part: rows 4 (G v + g) .. + 3 of slot sl into the three
  // digit planes of buffer buf.
  auto qdigits = [&](int sl, int v, float f, int buf) {
    uint32_t u[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      u[e] = __float_as_uint(__builtin_fmaf(xv[sl][4 * v + e], f, kQMagic)) + kQDigitBias;
    orv |= u[0] | u[1] | u[2] | u[3];
    const uint32_t r01 = bperm(u[1], u[0], 0x05010400u);
    const uint32_t r23 = bperm(u[3], u[2], 0x05010400u);
    const uint32_t s01 = bperm(u[1], u[0], 0x0C0C0602u);
    const uint32_t s23 = bperm(u[3], u[2], 0x0C0C0602u);
    uint32_t* d = reinterpret_cast<uint32_t*>(dig + buf * dig_sz + qcol[sl] * LD +
                                              4 * (G * v + qg[sl]));
    d[0] = bperm(r23, r01, 0x05040100u) ^ 0x80808080u;
    d[Cg * LD / 4] = bperm(r23, r01, 0x07060302u) ^ 0x80808080u;
    d[2 * Cg * LD / 4] = bperm(s23, s01, 0x05040100u) ^ 0x80808080u;
  };
  auto quantise = [&](int sl, int buf) {
    if (!FULL && tid + sl * nthr >= ntask) return;
    const float f = qscale(sl, buf);
#pragma unroll
    for (int v = 0; v < 4; ++v) qdigits(sl, v, f, buf);
  };

  // Philox words of the stage starting at row r0 into buffer buf: draw c is
  // Theta row theta0 + c % Tg, block (r0 >> 7) + c / Tg.  The block size is a
  // multiple of Tg, so a thread always draws row theta0 + tid % Tg.
  auto draw = [&](int64_t r0, int buf) {
    for (int c = tid; c < Tg * SB; c += nthr) {
      const int r = c % Tg, sb = c / Tg;
      const int i = theta0 + r;
      Words w{0u, 0u, 0u, 0u};
      if (i < k) w = radem_words(seed, i, (r0 >> 7) + sb);
      uint32_t* z = zb + buf * zb_sz + (sb * Tg + r) * kQZs;
      z[0] = w.w0;
      z[1] = w.w1;
      z[2] = w.w2;
      z[3] = w.w3;
    }
  };

  i4v acc[3][TT][CT];
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int tt = 0; tt < TT; ++tt)
#pragma unroll
      for (int b = 0; b < CT; ++b) acc[p][tt][b] = i4v{0, 0, 0, 0};
  int cur_s[CT];
  bool written[CT];
#pragma unroll
  for (int b = 0; b < CT; ++b) {
    cur_s[b] = kQUnset;
    written[b] = false;
  }

  // Fold column tile b's integer sums into the FP64 partials (exact: each
  // sum is below 2^31, so 2^16 H + 2^8 D + L is below 2^48).
  auto fold = [&](int b, bool nan_out) {
    const double sc = (cur_s[b] == kQUnset) ? 1.0 : static_cast<double>(pow2f(-cur_s[b]));
    const int c = c0 + wcol * CT * 16 + 16 * b + l16;
    double* dst = part + (static_cast<int64_t>(s) * npad + c) * kpad + theta0 + wrow * TT * 16;
#pragma unroll
    for (int tt = 0; tt < TT; ++tt) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double val = (65536.0 * static_cast<double>(acc[2][tt][b][v]) +
                      256.0 * static_cast<double>(acc[1][tt][b][v]) +
                      static_cast<double>(acc[0][tt][b][v])) * sc;
        if (nan_out) val = __builtin_nan("");
        double* p = dst + 16 * tt + 4 * lg + v;
        *p = written[b] ? *p + val : val;
      }
#pragma unroll
      for (int p = 0; p < 3; ++p) acc[p][tt][b] = i4v{0, 0, 0, 0};
    }
    written[b] = true;
  };

  // Register t of this lane's A operand holds rows 4t..4t+3 of its 16-row
  // slot, whose Theta bits sit at bit b = 4 (lg & 1) + t of the four bytes
  // of one word.  Masking that bit leaves selector bytes 0 or 2^b, and the
  // byte permute maps 0 to 0x01 (+1) and every 2^b to 0xFF (-1): bytes 1
  // and 2 of the low source and byte 0 of the high source are 0xFF, byte 1's
  // sign bit is set (selector 8), and selectors of 13 and more give 0xFF.
  uint32_t amask[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) amask[t] = 0x01010101u << (4 * (lg & 1) + t);

  // A operand of Theta tile tt for matrix-core step ks (rows 64 ks .. 64 ks
  // + 63 of the stage in buffer buf).
  auto agen = [&](int ks, int buf, int tt) -> i4v {
    const uint32_t w = zb[buf * zb_sz + ((ks >> 1) * Tg + wrow * TT * 16 + 16 * tt + l16) * kQZs +
                          2 * (ks & 1) + (lg >> 1)];
    i4v a;
#pragma unroll
    for (int t = 0; t < 4; ++t) a[t] = static_cast<int>(bperm(0xFFFFFFFFu, 0xFFFFFF01u, w & amask[t]));
    return a;
  };
  // B operands (three digit planes) of column tile b for step ks.
  auto bload = [&](int ks, int buf, int b, i4v* bp) {
    const unsigned char* d =
        dig + buf * dig_sz + (wcol * CT * 16 + 16 * b + l16) * LD + 64 * ks + 16 * lg;
#pragma unroll
    for (int p = 0; p < 3; ++p) bp[p] = *reinterpret_cast<const i4v*>(d + p * Cg * LD);
  };
  auto mma3 = [&](const i4v& a, const i4v* bp, int tt, int b) {
#pragma unroll
    for (int p = 0; p < 3; ++p)
      acc[p][tt][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, bp[p], acc[p][tt][b], 0, 0, 0);
  };

  __syncthreads();
  int64_t r0 = r_begin;
  int cur = 0;
  if (r0 < r_end) {
    load_stage(r0);
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) quantise(sl, 0);
    draw(r0, 0);
  }
  __syncthreads();
  if (r0 + sstride < r_end) load_stage(r0 + sstride);
  for (; r0 < r_end; r0 += sstride, cur ^= 1) {
    // Columns whose scale grew for this stage: fold at the old scale.
#pragma unroll
    for (int b = 0; b < CT; ++b) {
      const int ns = colexp[cur * Cg + wcol * CT * 16 + 16 * b + l16];
      if (ns != cur_s[b]) {
        if (cur_s[b] != kQUnset) fold(b, false);
        cur_s[b] = ns;
      }
    }
    // This stage's matrix-core steps, with the next stage's quantisation
    // in between (on the last stage it works on stale registers into the
    // idle buffer, which is never read).
    if (FULL) {
      // KS steps of TT CT groups of 3 matrix-core instructions.  Between
      // groups goes the vector work, fenced so that the compiler keeps the
      // interleaving: the next step's A operands (last TT groups of a step),
      // the next stage's quantisation (steps 0 .. NSL-1, one task slot per
      // step) and its Philox draw (step NSL, two rounds per group).  B
      // operands are loaded one column tile ahead (two buffers).
      static_assert(!FULL || (KS >= NSL + 1 && CT % 2 == 0 && TT * CT >= 6),
                    "FULL layout");
      constexpr int NG = TT * CT;
      i4v a[2][TT], bq[2][3];
#pragma unroll
      for (int tt = 0; tt < TT; ++tt) a[0][tt] = agen(0, cur, tt);
      bload(0, cur, 0, bq[0]);
      float fq = 0.f;
      const int pr = tid % Tg, psb = tid / Tg;  // this thread's Philox draw
      PhiloxState ph;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
        for (int j = 0; j < NG; ++j) {
          const int b = j / TT, tt = j % TT;
          mma3(a[ks & 1][tt], bq[b & 1], tt, b);
          if (tt == 0 && b + 1 < CT) bload(ks, cur, b + 1, bq[(b + 1) & 1]);
          if (j == NG - 1 && ks + 1 < KS) bload(ks + 1, cur, 0, bq[0]);
          if (ks < NSL) {
            if (j == 0) fq = qscale(ks, cur ^ 1);
            if (j >= 1 && j <= 4) qdigits(ks, j - 1, fq, cur ^ 1);
            // This slot's registers are free again: fetch its rows of the
            // stage after next, a whole stage ahead of their use.
            if (j == 5) load_slot(ks, r0 + 2 * sstride);
          } else if (ks == NSL) {
            if (j == 0) {
              const uint64_t blk = static_cast<uint64_t>((r0 + sstride) >> 7) + psb;
              // words (blk, row, RADE)
              ph = PhiloxState{static_cast<uint32_t>(blk), static_cast<uint32_t>(blk >> 32),
                               static_cast<uint32_t>(theta0 + pr), kTagRadem,
                               static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32)};
            }
            if (j < 5) {
              philox_round(ph);
              philox_round(ph);
            }
            if (j == 5) {
              uint32_t* z = zb + (cur ^ 1) * zb_sz + (psb * Tg + pr) * kQZs;
              z[0] = ph.c0;
              z[1] = ph.c1;
              z[2] = ph.c2;
              z[3] = ph.c3;
            }
          }
          if (ks + 1 < KS && j >= NG - TT) {
            const int t2 = j - (NG - TT);
            a[(ks + 1) & 1][t2] = agen(ks + 1, cur, t2);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        i4v a[TT];
#pragma unroll
        for (int tt = 0; tt < TT; ++tt) a[tt] = agen(ks, cur, tt);
#pragma unroll
        for (int b = 0; b < CT; ++b) {
          i4v bp[3];
          bload(ks, cur, b, bp);
#pragma unroll
          for (int tt = 0; tt < TT; ++tt) mma3(a[tt], bp, tt, b);
        }
        if (ks < NSL) {
          quantise(ks, cur ^ 1);
          load_slot(ks, r0 + 2 * sstride);
        }
      }
#pragma unroll
      for (int sl = KS; sl < NSL; ++sl) {
        quantise(sl, cur ^ 1);
        load_slot(sl, r0 + 2 * sstride);
      }
    }
    if (!FULL) draw(r0 + sstride, cur ^ 1);
    if (orv >> 24) *badflag = 1;
    __syncthreads();
  }
  const bool bad = *badflag != 0;
#pragma unroll
  for (int b = 0; b < CT; ++b) fold(b, bad);
}

// Launch plan of the int8 sketch for (k, n).
struct I8Plan {
  int tt, ct, sb, wt, wc, ktiles, nh, kpad, npad;
  bool full;  // four Theta waves x two column waves of two tiles: one task per thread
};

// Layout of the interleaved kernel for k > 384, n > 32: 256 Theta rows x 64
// columns per workgroup of 8 waves, each wave kQMainTT x kQMainCT tiles.
constexpr int kQMainTT = 2, kQMainCT = 4;

static I8Plan i8_plan(int k, int n) {
  I8Plan p{};
  if (k > 384 && n > 32) {
    p.tt = kQMainTT;
    p.ct = kQMainCT;
    p.wc = 64 / (16 * p.ct);
    p.wt = 8 / p.wc;
    p.full = true;
    p.sb = 2;
    p.ktiles = static_cast<int>(ceil_div(k, 16 * p.tt * p.wt));
  } else {
    p.tt = 4;
    p.ct = (n <= 16) ? 1 : 2;
    p.wc = (n > 16 * p.ct) ? 2 : 1;
    const int kt = static_cast<int>(ceil_div(k, 16 * p.tt));
    // Waves along Theta: 1, 2 or 4 (at most 8 waves), fewest padded tiles.
    int best_wt = 1, best_slots = 1 << 30;
    for (int wt = 1; wt <= 8 / p.wc && wt <= 4; wt *= 2) {
      const int slots = wt * static_cast<int>(ceil_div(kt, wt));
      if (slots <= best_slots) {
        best_slots = slots;
        best_wt = wt;
      }
    }
    p.wt = best_wt;
    p.ktiles = static_cast<int>(ceil_div(kt, p.wt));
    if (p.ct > p.wt) p.ct = 1;  // at most two quantiser tasks per thread
    p.full = false;
    p.sb = 1;
  }
  const int cg = 16 * p.ct * p.wc;
  p.nh = static_cast<int>(ceil_div(n, cg));
  p.kpad = 16 * p.tt * p.wt * p.ktiles;
  p.npad = cg * p.nh;
  return p;
}

static size_t i8_lds_bytes(const I8Plan& p) {
  const int tg = 16 * p.tt * p.wt, cg = 16 * p.ct * p.wc, ld = kQBlock * p.sb + 32;
  return static_cast<size_t>(2 * 3 * cg * ld + 2 * tg * p.sb * kQZs * 4 + 2 * cg * 4 + 16);
}

void mixed_sketch_plan(int64_t m, int k, int n, SketchPlan& sp) {
  const I8Plan p = i8_plan(k, n);
  sp.ktiles = p.ktiles;
  sp.kpad = p.kpad;
  sp.npad = p.npad;
  // Splits (multiples of 8, for the XCD decode) chosen so that the grid
  // fills whole rounds of one workgroup per CU; at most 2^23 rows a split
  // keeps the int32 sums exact.
  const int64_t stage = kQBlock * p.sb;
  const int64_t tps = static_cast<int64_t>(p.ktiles) * p.nh;
  const int64_t maxs = round_up(ceil_div(m, stage), 8);
  const int64_t mins = round_up(ceil_div(m, int64_t{1} << 23), 8);
  int64_t best = mins > 8 ? mins : 8;
  double best_eff = -1.0;
  for (int64_t ns = best; ns <= 512 && ns <= maxs; ns += 8) {
    const int64_t w = ns * tps;
    const double eff = static_cast<double>(w) / (256.0 * ceil_div(w, 256));
    const double score = eff - ((w < 512) ? 0.5 : 0.0) - 1e-4 * static_cast<double>(w / 256);
    if (score > best_eff + 1e-9) {
      best_eff = score;
      best = ns;
    }
  }
  sp.nsplit = static_cast<int>(best);
  sp.rows_per_split = round_up(ceil_div(m, sp.nsplit), stage);
}

hipError_t launch_sketch_mixed_partials(const float* X, int64_t m, int n, int64_t ldx, int k,
                                        uint64_t seed, const SketchPlan& pl, double* part,
                                        hipStream_t st, int kind) {
  if (kind == kSRHT) return launch_sketch_srht_partials(X, true, m, n, ldx, k, seed, pl, part, st);
  if (kind != kRademacher) return hipErrorInvalidValue;
  const I8Plan p = i8_plan(k, n);
  // every thread draws one Theta row: the block is a multiple of Tg
  const int tt = p.full ? kQMainTT : 4;
  if ((64 * p.wt * p.wc) % (16 * tt * p.wt) != 0) return hipErrorInvalidValue;
  if (p.ktiles != pl.ktiles || p.kpad != pl.kpad || p.npad != pl.npad ||
      (pl.rows_per_split % (kQBlock * p.sb)) != 0 || (pl.nsplit % 8) != 0 ||
      pl.rows_per_split > (int64_t{1} << 23))
    return hipErrorInvalidValue;
  const size_t shm = i8_lds_bytes(p);
  const dim3 grid(pl.nsplit * p.ktiles * p.nh), block(64 * p.wt * p.wc);
  hipError_t e = hipSuccess;
#define RCQ_I8(TTV, CTV, SBV, NSLV, FV)                                                        \
  do {                                                                                         \
    const void* fn = reinterpret_cast<const void*>(&sketch_i8_kernel<TTV, CTV, SBV, NSLV, FV>); \
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,                    \
                            static_cast<int>(shm));                                            \
    if (e != hipSuccess) return e;                                                             \
    sketch_i8_kernel<TTV, CTV, SBV, NSLV, FV><<<grid, block, shm, st>>>(                       \
        X, m, n, ldx, k, seed, p.wt, p.wc, p.ktiles, p.nh, pl.rows_per_split, pl.kpad, pl.npad, \
        part);                                                                                 \
  } while (0)
  if (p.full)
    RCQ_I8(kQMainTT, kQMainCT, 2, 2, true);
  else if (p.ct == 2)
    RCQ_I8(4, 2, 1, 2, false);
  else
    RCQ_I8(4, 1, 1, 2, false);
#undef RCQ_I8
  return hipGetLastError();
}

hipError_t launch_sketch_mixed(const float* X, int64_t m, int n, int64_t ldx, int k, uint64_t seed,
                               const SketchPlan& pl, double* part, double* P, int64_t ldp,
                               hipStream_t st, int kind) {
  const hipError_t e = launch_sketch_mixed_partials(X, m, n, ldx, k, seed, pl, part, st, kind);
  if (e != hipSuccess) return e;
  return launch_sketch_reduce(part, pl, k, n, 1.0 / sqrt(static_cast<double>(k)), P, ldp, st);
}

}  // namespace rcq
