// rr.hip -- the steps of rank-revealing RCholeskyQR (Algorithm 7, Section 4)
// around the shared sketch, Householder and tall-solve kernels:
//   * column norms D of X (split partials in FP64, reduced in split order),
//   * the normalised sketch P D^{-1},
//   * the rank-revealing QR of that sketch: Householder with column pivoting
//     (largest remaining column norm, first on ties) applied to the n x n R
//     factor of P D^{-1} -- P D^{-1} = S R with orthonormal S, so pivots and
//     R are those of the sketch itself -- in one workgroup,
//   * the rank rule (step 3) with ||R||_2 from a power iteration, R <- R_{1:r,:}
//     Pi^T D Pi (the normalisation undone), and the triangular factor of the
//     solve of step 4 (R_{1:r,1:r} Pi^T D Pi, identity on the dropped columns),
//   * the gather X Pi (the tall solve then runs in place on it).
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace rcq {

constexpr int kRrSplits = 256;  // row splits of the column norms

// part[s * n + c] = sum of X(r, c)^2 over rows r of split s (FP64); one wave
// per column, 4 columns per workgroup.
template <typename T>
__global__ __launch_bounds__(256) void colnorm_partial_kernel(const T* __restrict__ X, int64_t m,
                                                              int n, int64_t ldx,
                                                              int64_t rows_per_split,
                                                              double* __restrict__ part) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + wave, s = blockIdx.y;
  if (c >= n) return;
  const int64_t r0 = static_cast<int64_t>(s) * rows_per_split;
  const int64_t r1 = (r0 + rows_per_split < m) ? r0 + rows_per_split : m;
  const T* col = X + static_cast<int64_t>(c) * ldx;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t r = r0 + lane;
  for (; r + 192 < r1; r += 256) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double x = static_cast<double>(col[r + 64 * u]);
      acc[u] += x * x;
    }
  }
  for (; r < r1; r += 64) {
    const double x = static_cast<double>(col[r]);
    acc[0] += x * x;
  }
  const double t = wave_sum((acc[0] + acc[1]) + (acc[2] + acc[3]));
  if (lane == 0) part[static_cast<int64_t>(s) * n + c] = t;
}

// d[c] = sqrt(sum over splits in order); P(:, c) /= d[c] (a zero column stays
// zero).  One thread per column.
__global__ void colnorm_scale_kernel(const double* __restrict__ part, int nsplit, int n,
                                     double* __restrict__ d, double* __restrict__ P, int k,
                                     int64_t ldp) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double s = 0.0;
  for (int i = 0; i < nsplit; ++i) s += part[static_cast<int64_t>(i) * n + c];
  const double dc = sqrt(s);
  d[c] = dc;
  const double inv = (dc > 0.0) ? 1.0 / dc : 0.0;
  double* pc = P + static_cast<int64_t>(c) * ldp;
  for (int i = 0; i < k; ++i) pc[i] *= inv;
}

// Householder QR with column pivoting of the n x n upper triangular Rp (ld
// n).  W (n x n, row-major scratch) is the working matrix; thread c owns
// column c.  Step j: the remaining column of largest norm over rows j..
// (norms carried from the previous step's update, first index on ties) is
// swapped to j, reflected (alpha = -sign(x_j) ||x||), and the reflector is
// applied to the columns right of it.  Out: Rt (ld n, column-major, positive
// diagonal: rows flipped with alpha), piv.
__global__ __launch_bounds__(256) void qrcp_kernel(const double* __restrict__ Rp, int n,
                                                   double* __restrict__ W,
                                                   double* __restrict__ Rt, int* __restrict__ piv) {
  __shared__ double v[kMaxN];
  __shared__ double nrm2[kMaxN];
  __shared__ double sgn[kMaxN];
  __shared__ int pcol[kMaxN];
  __shared__ int pivot;
  __shared__ double hb[2];  // beta, alpha
  const int c = threadIdx.x, lane = c & 63;
  if (c < n) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
      const double x = (i <= c) ? Rp[i + static_cast<int64_t>(c) * n] : 0.0;
      W[static_cast<int64_t>(i) * n + c] = x;
      s += x * x;
    }
    nrm2[c] = s;
    pcol[c] = c;
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    // pivot: wave 0 scans the candidates c >= j (4 per lane), largest norm,
    // lowest index among equal ones
    if (c < 64) {
      double best = -1.0;
      int bi = n;
      for (int q = 0; q < 4; ++q) {
        const int cc = lane + 64 * q;
        if (cc >= j && cc < n && nrm2[cc] > best) {
          best = nrm2[cc];
          bi = cc;
        }
      }
      double mx = best;
      for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
      int cand = (best == mx) ? bi : n;
      for (int off = 32; off >= 1; off >>= 1) cand = min(cand, __shfl_xor(cand, off));
      if (lane == 0) pivot = cand;
    }
    __syncthreads();
    const int p = pivot;
    if (p != j) {
      // swap columns j and p (rows 0..n-1), their norms and labels
      for (int i = c; i < n; i += blockDim.x) {
        const double a = W[static_cast<int64_t>(i) * n + j];
        W[static_cast<int64_t>(i) * n + j] = W[static_cast<int64_t>(i) * n + p];
        W[static_cast<int64_t>(i) * n + p] = a;
      }
      if (c == 0) {
        const double t = nrm2[j];
        nrm2[j] = nrm2[p];
        nrm2[p] = t;
        const int l = pcol[j];
        pcol[j] = pcol[p];
        pcol[p] = l;
      }
    }
    __syncthreads();
    // reflector of column j (rows j..n-1), from its norm (already known)
    for (int i = j + c; i < n; i += blockDim.x) v[i] = W[static_cast<int64_t>(i) * n + j];
    __syncthreads();
    if (c == 0) {
      const double x0 = v[j];
      const double nr = sqrt(nrm2[j]);
      const double alpha = (x0 >= 0.0) ? -nr : nr;
      const double v0 = x0 - alpha;
      const double vtv = v0 * v0 + (nrm2[j] - x0 * x0);
      v[j] = v0;
      hb[0] = (vtv > 0.0 && nr > 0.0) ? 2.0 / vtv : 0.0;
      hb[1] = (nr > 0.0) ? alpha : x0;
      sgn[j] = (hb[1] < 0.0) ? -1.0 : 1.0;
    }
    __syncthreads();
    const double beta = hb[0];
    if (c > j && c < n) {
      double w = 0.0;
      for (int i = j; i < n; ++i) w += v[i] * W[static_cast<int64_t>(i) * n + c];
      const double f = beta * w;
      double s = 0.0;
      for (int i = j; i < n; ++i) {
        const double x = W[static_cast<int64_t>(i) * n + c] - f * v[i];
        W[static_cast<int64_t>(i) * n + c] = x;
        if (i > j) s += x * x;
      }
      nrm2[c] = s;  // norm over rows j+1.. for the next pivot
    } else if (c == j) {
      W[static_cast<int64_t>(j) * n + j] = hb[1];
      for (int i = j + 1; i < n; ++i) W[static_cast<int64_t>(i) * n + j] = 0.0;
    }
    __syncthreads();
  }
  if (c < n) {
    for (int i = 0; i < n; ++i)
      Rt[i + static_cast<int64_t>(c) * n] = (i <= c) ? sgn[i] * W[static_cast<int64_t>(i) * n + c] : 0.0;
    piv[c] = pcol[c];
  }
}

// Step 3 (rank: least r with ||Rt_{r:,r:}||_F <= tau ||Rt||_2, the 2-norm by
// 64 power-iteration steps on Rt^T Rt) and the outputs: R (ld ldr) =
// Rt_{1:r,:} diag(d[piv]) (rows >= r zero), Rs (ld n) the factor of the
// solve (that block on 1:r, identity on the dropped columns), rank.  The
// status word keeps only the non-finite flag (rank deficiency is expected).
__global__ __launch_bounds__(256) void rr_finish_kernel(const double* __restrict__ Rt, int n,
                                                        double tau, const double* __restrict__ d,
                                                        const int* __restrict__ piv,
                                                        double* __restrict__ R, int64_t ldr,
                                                        double* __restrict__ Rs,
                                                        int* __restrict__ rank,
                                                        int* __restrict__ status) {
  __shared__ double x[kMaxN], y[kMaxN], red[4];
  __shared__ double tail[kMaxN + 1];
  __shared__ int rr;
  const int t = threadIdx.x;
  if (t < n) x[t] = 1.0;
  __syncthreads();
  double sigma = 0.0;
  for (int it = 0; it < 64; ++it) {
    // y = Rt x, x = Rt^T y / ||Rt^T y||
    if (t < n) {
      double s = 0.0;
      for (int c = t; c < n; ++c) s += Rt[t + static_cast<int64_t>(c) * n] * x[c];
      y[t] = s;
    }
    __syncthreads();
    double z = 0.0;
    if (t < n)
      for (int i = 0; i <= t; ++i) z += Rt[i + static_cast<int64_t>(t) * n] * y[i];
    const double zz = block_sum(z * z, red);
    const double yy = block_sum((t < n) ? y[t] * y[t] : 0.0, red);
    sigma = sqrt(yy);  // ||Rt x|| with ||x|| = 1 after the first step
    const double inv = (zz > 0.0) ? 1.0 / sqrt(zz) : 0.0;
    __syncthreads();
    if (t < n) x[t] = z * inv;
    __syncthreads();
  }
  // ||Rt x|| for the final unit x
  if (t < n) {
    double s = 0.0;
    for (int c = t; c < n; ++c) s += Rt[t + static_cast<int64_t>(c) * n] * x[c];
    y[t] = s;
  }
  const double yy = block_sum((t < n) ? y[t] * y[t] : 0.0, red);
  sigma = fmax(sigma, sqrt(yy));
  // row sums of squares, suffix sums in order
  if (t < n) {
    double s = 0.0;
    for (int c = t; c < n; ++c) {
      const double a = Rt[t + static_cast<int64_t>(c) * n];
      s += a * a;
    }
    y[t] = s;
  }
  __syncthreads();
  if (t == 0) {
    tail[n] = 0.0;
    for (int i = n - 1; i >= 0; --i) tail[i] = tail[i + 1] + y[i];
    int r = n;
    for (int q = 0; q <= n; ++q)
      if (sqrt(tail[q]) <= tau * sigma) {
        r = q;
        break;
      }
    rr = r;
    *rank = r;
    bool bad = !isfinite(sigma);
    for (int c = 0; c < n; ++c) bad = bad || !isfinite(d[c]);
    *status = bad ? 2 : 0;
  }
  __syncthreads();
  const int r = rr;
  for (int idx = t; idx < n * n; idx += blockDim.x) {
    const int i = idx % n, c = idx / n;
    const double v = (i < r && i <= c) ? Rt[i + static_cast<int64_t>(c) * n] * d[piv[c]] : 0.0;
    R[i + static_cast<int64_t>(c) * ldr] = v;
    Rs[idx] = (i < r && c < r) ? v : ((i == c) ? 1.0 : 0.0);
  }
}

// Q(:, j) = X(:, piv[j]) for the n columns.
template <typename T>
__global__ __launch_bounds__(256) void gather_cols_kernel(const T* __restrict__ X, int64_t m,
                                                          int64_t ldx, const int* __restrict__ piv,
                                                          T* __restrict__ Q, int64_t ldq) {
  const int j = blockIdx.y;
  const T* src = X + static_cast<int64_t>(piv[j]) * ldx;
  T* dst = Q + static_cast<int64_t>(j) * ldq;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; r < m; r += stride)
    dst[r] = src[r];
}

size_t rr_extra_bytes(int n) {
  const size_t nn = static_cast<size_t>(n) * n * sizeof(double);
  return static_cast<size_t>(kRrSplits) * n * sizeof(double)  // norm partials
         + n * sizeof(double)                                 // d
         + 3 * nn                                             // W, Rt, Rs
         + 2 * n * sizeof(int) + 256;                         // piv, rank
}

hipError_t launch_rr_steps(const void* X, bool f32, int64_t m, int n, int64_t ldx, double* P,
                           int k, const double* Rp, double tau, unsigned char* extra,
                           double* R, int64_t ldr, int* piv_out, int* rank_out, int* status,
                           double** Rs_out, hipStream_t st, int stage) {
  double* part = reinterpret_cast<double*>(extra);
  double* d = part + static_cast<size_t>(kRrSplits) * n;
  double* W = d + n;
  double* Rt = W + static_cast<size_t>(n) * n;
  double* Rs = Rt + static_cast<size_t>(n) * n;
  *Rs_out = Rs;
  if (stage == 0) {
    // column norms of X and the normalised sketch
    const int64_t rows = ceil_div(m, static_cast<int64_t>(kRrSplits));
    const dim3 grid(static_cast<unsigned>(ceil_div(n, 4)), kRrSplits);
    if (f32)
      colnorm_partial_kernel<float><<<grid, 256, 0, st>>>(static_cast<const float*>(X), m, n, ldx,
                                                           rows, part);
    else
      colnorm_partial_kernel<double><<<grid, 256, 0, st>>>(static_cast<const double*>(X), m, n,
                                                            ldx, rows, part);
    colnorm_scale_kernel<<<1, 256, 0, st>>>(part, kRrSplits, n, d, P, k, k);
    return hipGetLastError();
  }
  qrcp_kernel<<<1, 256, 0, st>>>(Rp, n, W, Rt, piv_out);
  rr_finish_kernel<<<1, 256, 0, st>>>(Rt, n, tau, d, piv_out, R, ldr, Rs, rank_out, status);
  return hipGetLastError();
}

hipError_t launch_gather_cols(const void* X, bool f32, int64_t m, int n, int64_t ldx,
                              const int* piv, void* Q, int64_t ldq, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(std::min<int64_t>(ceil_div(m, 256), 64)), n);
  if (f32)
    gather_cols_kernel<float><<<grid, 256, 0, st>>>(static_cast<const float*>(X), m, ldx, piv,
                                                     static_cast<float*>(Q), ldq);
  else
    gather_cols_kernel<double><<<grid, 256, 0, st>>>(static_cast<const double*>(X), m, ldx, piv,
                                                      static_cast<double*>(Q), ldq);
  return hipGetLastError();
}

}  // namespace rcq
