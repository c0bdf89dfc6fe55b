// theta.h -- on-the-fly sketching matrix Theta for gfx950.
//
// Theta (k x m) is never stored (Section 2: a seeded random number generator
// makes the embedding's memory negligible; Algorithm 2 takes Theta as a
// function handle).  Column j of Theta belongs to row j of X, so a kernel
// streaming rows of X regenerates exactly the Theta columns it needs.
//
// Generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key =
// (lo32 seed, hi32 seed), counter = (lo32 a, hi32 a, b, stream tag):
//   Gaussian   : a = j, b = pair index: Theta rows 2b, 2b+1 of column j via
//                Box-Muller (1958).
//   Rademacher : a = j >> 7, b = Theta row i: one bit for each of the 128
//                columns 128a..128a+127 of row i (bit 1 -> -1).  Column
//                offset r = 32q + 4t + e (q < 4, t < 8, e < 4) is bit
//                8e + t of word q, so that four consecutive columns sit at
//                the same bit of the four bytes of a word.
//   CountSketch: a = j, b = 0: h(j) = (w0 * k) >> 32, s(j) = w1 & 1 ? -1 : +1.
// The Box-Muller transform uses only IEEE +, -, *, /, sqrt and explicit fma
// in a fixed order (contraction disabled here), so that its bits are the
// same on any conforming machine:
//   u1 = ((w0:w1 >> 11) + 1) 2^-53 in (0, 1],  u2 = (w2:w3 >> 11) 2^-53,
//   rho = sqrt(-2 ln u1), z_2b = rho cos(2 pi u2), z_2b+1 = rho sin(2 pi u2)
// with ln from the atanh series after an exponent split, and sin/cos of
// 2 pi u2 from an exact quadrant reduction on the 53-bit integer and
// Taylor series on [-pi/4, pi/4].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rcq {

constexpr uint32_t kTagGauss = 0x47415553u;  // "GAUS"
constexpr uint32_t kTagRadem = 0x52414445u;  // "RADE"
constexpr uint32_t kTagCount = 0x434F554Eu;  // "COUN"
constexpr uint32_t kTagSrhtD = 0x53524844u;  // "SRHD"
constexpr uint32_t kTagSrhtS = 0x53524853u;  // "SRHS"

struct Words {
  uint32_t w0, w1, w2, w3;
};

// Full 32 x 32 -> 64-bit product in one instruction (the compiler would
// otherwise split it into separate low and high multiplies).
__device__ __forceinline__ uint64_t mul_wide(uint32_t a, uint32_t b) {
  uint64_t r;
  asm("v_mad_u64_u32 %0, vcc, %1, %2, 0" : "=v"(r) : "v"(a), "s"(b) : "vcc");
  return r;
}

// Philox counter and key while the rounds run.
struct PhiloxState {
  uint32_t c0, c1, c2, c3, k0, k1;
};

// One Philox4x32 round and key bump.  Round multipliers and Weyl key
// increments are the published Philox4x32 constants.
__device__ __forceinline__ void philox_round(PhiloxState& p) {
  // One 32 x 32 -> 64-bit product each (a single v_mad_u64_u32).
  const uint64_t p0 = mul_wide(p.c0, 0xD2511F53u);
  const uint64_t p1 = mul_wide(p.c2, 0xCD9E8D57u);
  const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ p.c1 ^ p.k0;
  const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ p.c3 ^ p.k1;
  p.c0 = n0;
  p.c1 = static_cast<uint32_t>(p1);
  p.c2 = n2;
  p.c3 = static_cast<uint32_t>(p0);
  p.k0 += 0x9E3779B9u;
  p.k1 += 0xBB67AE85u;
}

// Ten Philox rounds.
__device__ __forceinline__ Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1) {
  PhiloxState p{c0, c1, c2, c3, k0, k1};
#pragma unroll
  for (int r = 0; r < 10; ++r) philox_round(p);
  return Words{p.c0, p.c1, p.c2, p.c3};
}

__device__ __forceinline__ Words theta_words(uint64_t seed, int64_t j, uint32_t block,
                                             uint32_t tag) {
  const uint64_t uj = static_cast<uint64_t>(j);
  return philox4x32_10(static_cast<uint32_t>(uj), static_cast<uint32_t>(uj >> 32), block, tag,
                       static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
}

// Natural log of a finite x > 0 (see the file comment).
__device__ __forceinline__ double bm_log(double x) {
#pragma clang fp contract(off)
  int64_t bits = __double_as_longlong(x);
  int ex = static_cast<int>((bits >> 52) & 0x7ff);
  if (ex == 0) {  // subnormal input: bring into the normal range
    x = x * 0x1p54;
    bits = __double_as_longlong(x);
    ex = static_cast<int>((bits >> 52) & 0x7ff) - 54;
  }
  ex -= 1023;
  double f = __longlong_as_double((bits & 0x000fffffffffffffll) | 0x3ff0000000000000ll);
  if (f >= 0x1.6a09e667f3bcdp+0) {
    f = f * 0.5;
    ex += 1;
  }
  const double s = (f - 1.0) / (f + 1.0);
  const double s2 = s * s;
  // 1/(2i+1), i = 0..12, correctly rounded
  double p = 0x1.47ae147ae147bp-5;
  p = __fma_rn(p, s2, 0x1.642c8590b2164p-5);
  p = __fma_rn(p, s2, 0x1.8618618618618p-5);
  p = __fma_rn(p, s2, 0x1.af286bca1af28p-5);
  p = __fma_rn(p, s2, 0x1.e1e1e1e1e1e1ep-5);
  p = __fma_rn(p, s2, 0x1.1111111111111p-4);
  p = __fma_rn(p, s2, 0x1.3b13b13b13b14p-4);
  p = __fma_rn(p, s2, 0x1.745d1745d1746p-4);
  p = __fma_rn(p, s2, 0x1.c71c71c71c71cp-4);
  p = __fma_rn(p, s2, 0x1.2492492492492p-3);
  p = __fma_rn(p, s2, 0x1.999999999999ap-3);
  p = __fma_rn(p, s2, 0x1.5555555555555p-2);
  p = __fma_rn(p, s2, 1.0);
  const double half_log = s * p;
  const double lnf = half_log + half_log;
  const double e = static_cast<double>(ex);
  return e * 0x1.62e42fee00000p-1 + (e * 0x1.a39ef35793c76p-33 + lnf);
}

// (sin, cos) of 2 pi b 2^-53 for an integer b in [0, 2^53).
__device__ __forceinline__ void bm_sincos2pi(uint64_t b, double& sn, double& cs) {
#pragma clang fp contract(off)
  const uint64_t quad = (b + (1ull << 50)) >> 51;
  const int64_t red = static_cast<int64_t>(b) - static_cast<int64_t>(quad << 51);
  const double x = (static_cast<double>(red) * 0x1p-51) * 0x1.921fb54442d18p+0;
  const double x2 = x * x;
  // (-1)^i / (2i+1)!, i = 1..9
  double ps = -0x1.2f49b46814157p-57;
  ps = __fma_rn(ps, x2, 0x1.952c77030ad4ap-49);
  ps = __fma_rn(ps, x2, -0x1.ae7f3e733b81fp-41);
  ps = __fma_rn(ps, x2, 0x1.6124613a86d09p-33);
  ps = __fma_rn(ps, x2, -0x1.ae64567f544e4p-26);
  ps = __fma_rn(ps, x2, 0x1.71de3a556c734p-19);
  ps = __fma_rn(ps, x2, -0x1.a01a01a01a01ap-13);
  ps = __fma_rn(ps, x2, 0x1.1111111111111p-7);
  ps = __fma_rn(ps, x2, -0x1.5555555555555p-3);
  const double s = __fma_rn(x * x2, ps, x);
  // (-1)^i / (2i)!, i = 2..10
  double pc = 0x1.e542ba4020225p-62;
  pc = __fma_rn(pc, x2, -0x1.6827863b97d97p-53);
  pc = __fma_rn(pc, x2, 0x1.ae7f3e733b81fp-45);
  pc = __fma_rn(pc, x2, -0x1.93974a8c07c9dp-37);
  pc = __fma_rn(pc, x2, 0x1.1eed8eff8d898p-29);
  pc = __fma_rn(pc, x2, -0x1.27e4fb7789f5cp-22);
  pc = __fma_rn(pc, x2, 0x1.a01a01a01a01ap-16);
  pc = __fma_rn(pc, x2, -0x1.6c16c16c16c17p-10);
  pc = __fma_rn(pc, x2, 0x1.5555555555555p-5);
  const double c = __fma_rn(x2 * x2, pc, __fma_rn(-0.5, x2, 1.0));
  switch (static_cast<int>(quad & 3)) {
    case 0: sn = s; cs = c; break;
    case 1: sn = c; cs = -s; break;
    case 2: sn = -s; cs = -c; break;
    default: sn = -c; cs = s; break;
  }
}

// Gaussian pair (rows 2b, 2b+1) of Theta column j.
__device__ __forceinline__ void gauss_pair(uint64_t seed, int64_t j, uint32_t b, double& z0,
                                           double& z1) {
#pragma clang fp contract(off)
  const Words w = theta_words(seed, j, b, kTagGauss);
  const uint64_t a = ((static_cast<uint64_t>(w.w0) << 32) | w.w1) >> 11;
  const uint64_t bb = ((static_cast<uint64_t>(w.w2) << 32) | w.w3) >> 11;
  const double u1 = static_cast<double>(a + 1) * 0x1p-53;
  const double rho = __dsqrt_rn(-2.0 * bm_log(u1));
  double sn, cs;
  bm_sincos2pi(bb, sn, cs);
  z0 = rho * cs;
  z1 = rho * sn;
}

// Rademacher words of Theta row i for columns 128 blk .. 128 blk + 127.
__device__ __forceinline__ Words radem_words(uint64_t seed, int i, int64_t blk) {
  return theta_words(seed, blk, static_cast<uint32_t>(i), kTagRadem);
}

// Rademacher bit (1 -> -1) of column offset r (0..127) within a block.
__device__ __forceinline__ uint32_t radem_bit(const Words& w, int r) {
  const int q = r >> 5, t = (r & 31) >> 2, e = r & 3;
  const uint32_t word = (q == 0) ? w.w0 : (q == 1) ? w.w1 : (q == 2) ? w.w2 : w.w3;
  return (word >> (8 * e + t)) & 1u;
}

// SRHT, Theta = sqrt(m'/k) S H D (m' = 2^L >= m, X padded with zero rows):
// D the diagonal of signs d_j, H the Sylvester-Hadamard matrix normalised by
// 1/sqrt(m') (H_sj = (-1)^popcount(s & j)), S the sampling of k rows s_i,
// uniform on [0, m') and independent.  Raw entry: d_j (-1)^popcount(s_i & j),
// with 1/sqrt(k) on P as for the other dense kinds.  d_j of the 128 columns
// of block blk are the bits of the words (blk, 0, SRHD) in radem_bit's
// layout; s_i is the top L bits of the 64-bit word (i, 0, SRHS).
__host__ __device__ inline int srht_log2(int64_t m) {
  int L = 0;
  while ((int64_t{1} << L) < m) ++L;
  return L;
}

__device__ __forceinline__ uint64_t srht_row(uint64_t seed, int i, int L) {
  const Words w = theta_words(seed, i, 0u, kTagSrhtS);
  const uint64_t x = (static_cast<uint64_t>(w.w1) << 32) | w.w0;
  return (L == 0) ? 0 : (x >> (64 - L));
}

// (-1)^popcount(s & r) for the 128 offsets r of a block, in radem_bit's
// layout (bit 8e + t of word q is offset 32q + 4t + e): parity is linear in
// r, so a word is a byte pattern over t, a byte mask over e and a constant
// over q.
__device__ __forceinline__ Words srht_walsh(uint64_t s) {
  const uint32_t se = static_cast<uint32_t>(s) & 3u, st = (static_cast<uint32_t>(s) >> 2) & 7u;
  const uint32_t sq = (static_cast<uint32_t>(s) >> 5) & 3u;
  uint32_t bt = 0u, em = 0u;
  for (uint32_t t = 0; t < 8; ++t) bt |= (__builtin_popcount(st & t) & 1u) << t;
  for (uint32_t e = 0; e < 4; ++e)
    if (__builtin_popcount(se & e) & 1u) em |= 0xFFu << (8 * e);
  const uint32_t base = bt * 0x01010101u ^ em;
  return {base, (sq & 1u) ? ~base : base, (sq & 2u) ? ~base : base,
          (__builtin_popcount(sq) & 1u) ? ~base : base};
}

// SRHT words of Theta row i (sample s, Walsh pattern wal of s) for block blk.
__device__ __forceinline__ Words srht_words(uint64_t seed, uint64_t s, const Words& wal,
                                            int64_t blk) {
  const Words d = theta_words(seed, blk, 0u, kTagSrhtD);
  const uint32_t hi =
      (__builtin_popcountll(s & (static_cast<uint64_t>(blk) << 7)) & 1) ? 0xFFFFFFFFu : 0u;
  return {d.w0 ^ wal.w0 ^ hi, d.w1 ^ wal.w1 ^ hi, d.w2 ^ wal.w2 ^ hi, d.w3 ^ wal.w3 ^ hi};
}

// CountSketch bucket and sign of column j.
__device__ __forceinline__ void count_hash(uint64_t seed, int64_t j, int k, int& h, int& neg) {
  const Words w = theta_words(seed, j, 0u, kTagCount);
  h = static_cast<int>((static_cast<uint64_t>(w.w0) * static_cast<uint64_t>(k)) >> 32);
  neg = static_cast<int>(w.w1 & 1u);
}

}  // namespace rcq
