// col.hip -- the small steps of column-oriented RCholeskyQR (Algorithm 4,
// Section 3.2) for one new block of b columns after j0 factored ones:
//   * the projection of the block's sketch on the previous sketch basis:
//     R_{1:j0, block} = S_{1:j0}^T P_block (the least-squares solution, S
//     having orthonormal columns) and W = P_block - S_{1:j0} R_{1:j0, block},
//   * the triangular factor of the tall step: [Q_{1:j0}, X_block] T^{-1} =
//     [Q_{1:j0}, (X_block - Q_{1:j0} R_{1:j0, block}) R_bb^{-1}] with T the
//     identity on the first j0 columns and R's new columns after them, so the
//     tall solve of Algorithm 2 does step 5 and leaves Q_{1:j0} as it is.
#include "common.h"
#include "kernels.h"

namespace rcq {

// One workgroup per column c of the block: P(:, c) into LDS, the j0
// coefficients by coalesced wave dot products (written to R(0:j0, j0 + c)),
// then W(:, c) = P(:, c) - S r in place over P.
__global__ __launch_bounds__(256) void col_project_kernel(const double* __restrict__ S,
                                                          int64_t lds, int j0,
                                                          double* __restrict__ P, int k,
                                                          double* __restrict__ R, int64_t ldr) {
  __shared__ double pc[kMaxK];
  __shared__ double rc[kMaxN];
  const int c = blockIdx.x, t = threadIdx.x, wave = t >> 6, lane = t & 63;
  double* pcol = P + static_cast<int64_t>(c) * k;
  for (int i = t; i < k; i += 256) pc[i] = pcol[i];
  __syncthreads();
  for (int l = wave; l < j0; l += 4) {
    const double* sl = S + static_cast<int64_t>(l) * lds;
    double a = 0.0;
    for (int i = lane; i < k; i += 64) a += sl[i] * pc[i];
    a = wave_sum(a);
    if (lane == 0) {
      rc[l] = a;
      R[l + static_cast<int64_t>(j0 + c) * ldr] = a;
    }
  }
  __syncthreads();
  for (int i = t; i < k; i += 256) {
    double w = pc[i];
    for (int l = 0; l < j0; ++l) w -= S[i + static_cast<int64_t>(l) * lds] * rc[l];
    pcol[i] = w;
  }
}

// T (nt x nt, ld nt): the identity on columns 0..j0-1, the upper part of R's
// columns j0..nt-1 after them.
__global__ __launch_bounds__(256) void col_make_t_kernel(const double* __restrict__ R,
                                                         int64_t ldr, int j0, int nt,
                                                         double* __restrict__ T) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= nt * nt) return;
  const int r = idx % nt, c = idx / nt;
  T[idx] = (c < j0) ? ((r == c) ? 1.0 : 0.0) : ((r <= c) ? R[r + static_cast<int64_t>(c) * ldr] : 0.0);
}

hipError_t launch_col_project(const double* S, int64_t lds, int j0, double* P, int k, int b,
                              double* R, int64_t ldr, hipStream_t st) {
  if (j0 == 0) return hipSuccess;
  col_project_kernel<<<b, 256, 0, st>>>(S, lds, j0, P, k, R, ldr);
  return hipGetLastError();
}

hipError_t launch_col_make_t(const double* R, int64_t ldr, int j0, int nt, double* T,
                             hipStream_t st) {
  col_make_t_kernel<<<static_cast<unsigned>(ceil_div(nt * nt, 256)), 256, 0, st>>>(R, ldr, j0,
                                                                                    nt, T);
  return hipGetLastError();
}

}  // namespace rcq
