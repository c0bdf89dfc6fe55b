// common.h -- shared device helpers for the gfx950 kernels (wave64, MFMA).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rcq {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

constexpr int kWave = 64;

// 16x16x4 matrix-core products.  Operand layouts (lane l, l16 = l % 16,
// lg = l / 16):  A(16x4): A[l16][lg];  B(4x16): B[lg][l16];
// D(16x16): element v holds D[drow(lg, v)][l16], where the row index is
// lg + 4 v for the FP64 product and 4 lg + v for the FP32 one (measured on
// gfx950 with a one-hot probe).
// Wave index within the workgroup as a wave-uniform (scalar) value, so that
// branches on it are scalar branches and not exec-masked divergent code.
__device__ __forceinline__ int wave_index() {
  return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
}

__device__ __forceinline__ d4 mfma16x16x4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16x16x4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T>
__device__ __forceinline__ constexpr int drow(int lg, int v) {
  return sizeof(T) == 8 ? lg + 4 * v : 4 * lg + v;
}
// A-operand row that makes D element v of lane group lg hold row 4 lg + v.
template <typename T>
__device__ __forceinline__ constexpr int arow_for_blocked_d(int l16) {
  return sizeof(T) == 8 ? 4 * (l16 & 3) + (l16 >> 2) : l16;
}

template <typename T>
struct Acc4;
template <>
struct Acc4<double> {
  typedef d4 type;
};
template <>
struct Acc4<float> {
  typedef f4 type;
};

// Sum over the 64 lanes of a wave, every lane gets it (fixed order:
// deterministic).  Within each row of 16 lanes by DPP moves (exchange with
// lane ^ 1, ^ 2, then the mirror images within 8 and 16 lanes, which pair
// lanes holding equal partial sums), then the four row sums read from
// lanes 0, 16, 32, 48.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ double read_lane(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ __forceinline__ float read_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Sum over a block; every thread gets the result.  `red` must hold at least
// blockDim.x / 64 values.  Contains two barriers.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  T s = T(0);
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

// Orders LDS traffic among the lanes of one wave (lanes run in lockstep;
// the fences keep the compiler and the memory model from reordering).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Status word: the first nonzero code written wins.
__device__ __forceinline__ void set_status(int* status, int code) {
  atomicCAS(status, 0, code);
}

__host__ __device__ constexpr int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ constexpr int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// sum_{s < ns} p[s * stride] added in order of s (the fixed order that makes
// the split-K reductions reproducible), with the loads of 16 terms issued
// together.
__device__ __forceinline__ double ordered_sum(const double* __restrict__ p, int ns,
                                              int64_t stride) {
  double sum = 0.0;
  int s = 0;
  for (; s + 16 <= ns; s += 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = p[static_cast<int64_t>(s + u) * stride];
#pragma unroll
    for (int u = 0; u < 16; ++u) sum += v[u];
  }
  for (; s < ns; ++s) sum += p[static_cast<int64_t>(s) * stride];
  return sum;
}

}  // namespace rcq
