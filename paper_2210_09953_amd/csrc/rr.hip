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

// d[c] = sqrt(sum of the split partials, a fixed-order block reduction);
// P(:, c) /= d[c] (a zero column stays zero).  One workgroup per column.
__global__ __launch_bounds__(256) void colnorm_scale_kernel(const double* __restrict__ part,
                                                            int nsplit, int n,
                                                            double* __restrict__ d,
                                                            double* __restrict__ P, int k,
                                                            int64_t ldp) {
  __shared__ double red[4];
  const int c = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  for (int i = t; i < nsplit; i += 256) s += part[static_cast<int64_t>(i) * n + c];
  s = block_sum(s, red);
  const double dc = sqrt(s);
  if (t == 0) d[c] = dc;
  const double inv = (dc > 0.0) ? 1.0 / dc : 0.0;
  double* pc = P + static_cast<int64_t>(c) * ldp;
  for (int i = t; i < k; i += 256) pc[i] *= inv;
}

// Householder QR with column pivoting of the n x n upper triangular Rp (ld
// n).  W (n x n, row-major scratch) is the working matrix; column c belongs
// to the four threads c + 256 q, thread q taking rows 64 q .. 64 q + 63; the
// four partial sums of a column are added in q order.  Step j: the
// remaining column of largest norm over rows j.. (carried from the previous
// step's update, first index on ties) is swapped to j, reflected (alpha =
// -sign(x_j) ||x||), and the reflector is applied to the columns right of
// it.  Out: Rt (ld n, column-major, positive diagonal: rows flipped with
// alpha), the same factor row-major in W, piv.
constexpr int kQcpThreads = 4 * kMaxN;

__global__ __launch_bounds__(kQcpThreads) void qrcp_kernel(const double* __restrict__ Rp, int n,
                                                           double* __restrict__ W,
                                                           double* __restrict__ Rt,
                                                           int* __restrict__ piv) {
  __shared__ double v[kMaxN];
  __shared__ double nrm2[kMaxN];
  __shared__ double sgn[kMaxN];
  __shared__ double qpart[4][kMaxN];
  __shared__ int pcol[kMaxN];
  __shared__ int pivot;
  __shared__ double hb[2];  // beta, alpha
  const int tid = threadIdx.x, c = tid & (kMaxN - 1), q = tid >> 8, lane = tid & 63;
  const int i0 = 64 * q;
  const bool col = c < n;
  // start: W = Rp (upper part), column norms
  {
    double s = 0.0;
    if (col)
      for (int u = 0; u < 64; ++u) {
        const int i = i0 + u;
        if (i < n) {
          const double x = (i <= c) ? Rp[i + static_cast<int64_t>(c) * n] : 0.0;
          W[static_cast<int64_t>(i) * n + c] = x;
          s += x * x;
        }
      }
    qpart[q][c] = s;
  }
  __syncthreads();
  if (tid < kMaxN && tid < n) {
    nrm2[tid] = ((qpart[0][tid] + qpart[1][tid]) + qpart[2][tid]) + qpart[3][tid];
    pcol[tid] = tid;
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    // pivot: wave 0 scans the candidates c >= j (4 per lane), largest norm,
    // lowest index among equal ones
    if (tid < 64) {
      double best = -1.0;
      int bi = n;
      for (int qq = 0; qq < 4; ++qq) {
        const int cc = lane + 64 * qq;
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
      for (int i = tid; i < n; i += kQcpThreads) {
        const double a = W[static_cast<int64_t>(i) * n + j];
        W[static_cast<int64_t>(i) * n + j] = W[static_cast<int64_t>(i) * n + p];
        W[static_cast<int64_t>(i) * n + p] = a;
      }
      if (tid == 0) {
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
    for (int i = j + tid; i < n; i += kQcpThreads) v[i] = W[static_cast<int64_t>(i) * n + j];
    __syncthreads();
    if (tid == 0) {
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
    // this thread's rows of the trailing part: max(j, i0) .. min(n, i0 + 64)
    const int lo = (j > i0) ? j : i0, hi = (i0 + 64 < n) ? i0 + 64 : n;
    const bool upd = col && c > j;
    {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      if (upd) {
        int i = lo;
        for (; i + 3 < hi; i += 4) {
          a0 += v[i] * W[static_cast<int64_t>(i) * n + c];
          a1 += v[i + 1] * W[static_cast<int64_t>(i + 1) * n + c];
          a2 += v[i + 2] * W[static_cast<int64_t>(i + 2) * n + c];
          a3 += v[i + 3] * W[static_cast<int64_t>(i + 3) * n + c];
        }
        for (; i < hi; ++i) a0 += v[i] * W[static_cast<int64_t>(i) * n + c];
      }
      qpart[q][c] = (a0 + a1) + (a2 + a3);
    }
    __syncthreads();
    {
      const double f = upd ? beta * (((qpart[0][c] + qpart[1][c]) + qpart[2][c]) + qpart[3][c]) : 0.0;
      __syncthreads();
      double s0 = 0.0, s1 = 0.0;
      if (upd) {
        int i = lo;
        for (; i + 1 < hi; i += 2) {
          const double x = W[static_cast<int64_t>(i) * n + c] - f * v[i];
          const double y = W[static_cast<int64_t>(i + 1) * n + c] - f * v[i + 1];
          W[static_cast<int64_t>(i) * n + c] = x;
          W[static_cast<int64_t>(i + 1) * n + c] = y;
          if (i > j) s0 += x * x;
          s1 += y * y;  // i + 1 > j
        }
        for (; i < hi; ++i) {
          const double x = W[static_cast<int64_t>(i) * n + c] - f * v[i];
          W[static_cast<int64_t>(i) * n + c] = x;
          if (i > j) s0 += x * x;
        }
      } else if (col && c == j) {
        for (int i = lo; i < hi; ++i) W[static_cast<int64_t>(i) * n + j] = (i == j) ? hb[1] : 0.0;
      }
      qpart[q][c] = s0 + s1;
    }
    __syncthreads();
    if (tid < n && tid > j)  // norm over rows j+1.. for the next pivot
      nrm2[tid] = ((qpart[0][tid] + qpart[1][tid]) + qpart[2][tid]) + qpart[3][tid];
    __syncthreads();
  }
  if (col) {
    for (int u = 0; u < 64; ++u) {
      const int i = i0 + u;
      if (i < n) {
        const double a = (i <= c) ? sgn[i] * W[static_cast<int64_t>(i) * n + c] : 0.0;
        Rt[i + static_cast<int64_t>(c) * n] = a;
        W[static_cast<int64_t>(i) * n + c] = a;
      }
    }
    if (q == 0) piv[c] = pcol[c];
  }
}

// Step 3 (rank: least r with ||Rt_{r:,r:}||_F <= tau ||Rt||_2, the 2-norm by
// 64 power-iteration steps on Rt^T Rt) and the outputs: R (ld ldr) =
// Rt_{1:r,:} diag(d[piv]) (rows >= r zero), Rs (ld n) the factor of the
// solve (that block on 1:r, identity on the dropped columns), rank.  The
// status word keeps only the non-finite flag (rank deficiency is expected).
// Rt is read column-major for the products Rt x and row-major (Rw) for
// Rt^T y, so that both are coalesced; output entry t of either product is
// the sum of four quarter sums (threads t + 256 q over indices 64 q ..
// 64 q + 63) added in q order.
constexpr int kFinThreads = 4 * kMaxN;

__global__ __launch_bounds__(kFinThreads) void rr_finish_kernel(
    const double* __restrict__ Rt, const double* __restrict__ Rw, int n, double tau,
    const double* __restrict__ d, const int* __restrict__ piv, double* __restrict__ R,
    int64_t ldr, double* __restrict__ Rs, int* __restrict__ rank, int* __restrict__ status) {
  __shared__ double x[kMaxN], y[kMaxN], qp[4][kMaxN], red[kFinThreads / 64];
  __shared__ double tail[kMaxN + 1];
  __shared__ int rr;
  const int tid = threadIdx.x, t = tid & (kMaxN - 1), q = tid >> 8;
  const int c0 = 64 * q, c1 = (c0 + 64 < n) ? c0 + 64 : n;
  const bool live = t < n;
  // quarter q of row t of Rt times x: columns max(t, c0) .. c1 (upper part)
  auto row_part = [&](bool sq) -> double {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (live) {
      int c = (t > c0) ? t : c0;
      for (; c + 3 < c1; c += 4) {
        const double r0 = Rt[t + static_cast<int64_t>(c) * n];
        const double r1 = Rt[t + static_cast<int64_t>(c + 1) * n];
        const double r2 = Rt[t + static_cast<int64_t>(c + 2) * n];
        const double r3 = Rt[t + static_cast<int64_t>(c + 3) * n];
        a0 += r0 * (sq ? r0 : x[c]);
        a1 += r1 * (sq ? r1 : x[c + 1]);
        a2 += r2 * (sq ? r2 : x[c + 2]);
        a3 += r3 * (sq ? r3 : x[c + 3]);
      }
      for (; c < c1; ++c) {
        const double r0 = Rt[t + static_cast<int64_t>(c) * n];
        a0 += r0 * (sq ? r0 : x[c]);
      }
    }
    return (a0 + a1) + (a2 + a3);
  };
  // y = Rt x, every thread gets ||y||^2
  auto mul_rt = [&]() -> double {
    qp[q][t] = row_part(false);
    __syncthreads();
    double yt = 0.0;
    if (q == 0 && live) {
      yt = ((qp[0][t] + qp[1][t]) + qp[2][t]) + qp[3][t];
      y[t] = yt;
    }
    return block_sum(yt * yt, red);  // its barriers also publish y
  };
  if (tid < n) x[tid] = 1.0;
  __syncthreads();
  double sigma = 0.0;
  for (int it = 0; it < 64; ++it) {
    // y = Rt x, x = Rt^T y / ||Rt^T y||
    const double yy = mul_rt();
    sigma = sqrt(yy);  // ||Rt x|| with ||x|| = 1 after the first step
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (live) {
      // quarter q of column t of Rt times y: rows c0 .. min(c1, t + 1)
      const int i1 = (c1 < t + 1) ? c1 : t + 1;
      int i = c0;
      for (; i + 3 < i1; i += 4) {
        a0 += Rw[static_cast<int64_t>(i) * n + t] * y[i];
        a1 += Rw[static_cast<int64_t>(i + 1) * n + t] * y[i + 1];
        a2 += Rw[static_cast<int64_t>(i + 2) * n + t] * y[i + 2];
        a3 += Rw[static_cast<int64_t>(i + 3) * n + t] * y[i + 3];
      }
      for (; i < i1; ++i) a0 += Rw[static_cast<int64_t>(i) * n + t] * y[i];
    }
    qp[q][t] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    const double z = (q == 0 && live) ? ((qp[0][t] + qp[1][t]) + qp[2][t]) + qp[3][t] : 0.0;
    const double zz = block_sum(z * z, red);
    const double inv = (zz > 0.0) ? 1.0 / sqrt(zz) : 0.0;
    if (q == 0 && live) x[t] = z * inv;
    __syncthreads();
  }
  // ||Rt x|| for the final unit x
  sigma = fmax(sigma, sqrt(mul_rt()));
  // row sums of squares, suffix sums in order
  qp[q][t] = row_part(true);
  __syncthreads();
  if (q == 0 && live) y[t] = ((qp[0][t] + qp[1][t]) + qp[2][t]) + qp[3][t];
  const int bad = __syncthreads_or((tid < n && !isfinite(d[tid])) ? 1 : 0);
  if (tid == 0) {
    tail[n] = 0.0;
    for (int i = n - 1; i >= 0; --i) tail[i] = tail[i + 1] + y[i];
    int r = n;
    for (int k = 0; k <= n; ++k)
      if (sqrt(tail[k]) <= tau * sigma) {
        r = k;
        break;
      }
    rr = r;
    *rank = r;
    *status = (bad || !isfinite(sigma)) ? 2 : 0;
  }
  __syncthreads();
  const int r = rr;
  for (int idx = tid; idx < n * n; idx += kFinThreads) {
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
    colnorm_scale_kernel<<<n, 256, 0, st>>>(part, kRrSplits, n, d, P, k, k);
    return hipGetLastError();
  }
  qrcp_kernel<<<1, kQcpThreads, 0, st>>>(Rp, n, W, Rt, piv_out);
  rr_finish_kernel<<<1, kFinThreads, 0, st>>>(Rt, W, n, tau, d, piv_out, R, ldr, Rs, rank_out,
                                              status);
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
