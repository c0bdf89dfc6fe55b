// rr.hip -- the steps of rank-revealing RCholeskyQR (Algorithm 7, Section 4)
// around the shared sketch, Householder and tall-solve kernels:
//   * column norms D of X (split partials of power-of-two scaled sums of
//     squares, so that no column overflows or underflows; reduced in split
//     order),
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

// Column norms without overflow or underflow: a sum of squares is kept as a
// pair (ssq, e) meaning ssq * 4^(e - 1023), e a biased FP64 exponent.  FP64
// entries are scaled by the power of two of the largest exponent seen so far
// (as the scaled sums of LAPACK's norm routines, with powers of two so that
// scaling is exact); FP32 entries square into the FP64 range unscaled
// (e = 1023).  kEmpty marks a sum with no non-zero term.
constexpr int kEmpty = -4096;

struct Ssq {
  double s;
  int e;
};

__device__ __forceinline__ void ssq_add(Ssq& a, double x) {
  const int ex = static_cast<int>((__double_as_longlong(x) >> 52) & 0x7ff);
  if (x != 0.0) {
    if (ex > a.e) {
      a.s = (a.e == kEmpty) ? 0.0 : ldexp(a.s, 2 * (a.e - ex));
      a.e = ex;
    }
    const double y = ldexp(x, 1023 - a.e);
    a.s += y * y;
  }
}

// a.s * 4^(a.e - e) for e >= a.e.
__device__ __forceinline__ double ssq_at(const Ssq& a, int e) {
  return (a.e == kEmpty) ? 0.0 : ldexp(a.s, 2 * (a.e - e));
}

// part[s * n + c] = the scaled sum of squares of X(r, c) over the rows r of
// split s and epart[s * n + c] its exponent; one wave per column, 4 columns
// per workgroup.
template <typename T>
__global__ __launch_bounds__(256) void colnorm_partial_kernel(const T* __restrict__ X, int64_t m,
                                                              int n, int64_t ldx,
                                                              int64_t rows_per_split,
                                                              double* __restrict__ part,
                                                              int* __restrict__ epart) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + wave, s = blockIdx.y;
  if (c >= n) return;
  const int64_t r0 = static_cast<int64_t>(s) * rows_per_split;
  const int64_t r1 = (r0 + rows_per_split < m) ? r0 + rows_per_split : m;
  const T* col = X + static_cast<int64_t>(c) * ldx;
  Ssq acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = Ssq{0.0, sizeof(T) == 8 ? kEmpty : 1023};
  auto add = [&](Ssq& a, T v) {
    if constexpr (sizeof(T) == 8) {
      ssq_add(a, v);
    } else {
      const double x = static_cast<double>(v);
      a.s += x * x;
    }
  };
  int64_t r = r0 + lane;
  for (; r + 192 < r1; r += 256) {
#pragma unroll
    for (int u = 0; u < 4; ++u) add(acc[u], col[r + 64 * u]);
  }
  for (; r < r1; r += 64) add(acc[0], col[r]);
  // the lane's pairs at its largest exponent, then the wave's
  int e = acc[0].e;
#pragma unroll
  for (int u = 1; u < 4; ++u) e = max(e, acc[u].e);
  double t = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u) t += ssq_at(acc[u], e);
  int ew = e;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) ew = max(ew, __shfl_xor(ew, off));
  const double tw = wave_sum(ssq_at(Ssq{t, e}, ew));
  if (lane == 0) {
    part[static_cast<int64_t>(s) * n + c] = tw;
    epart[static_cast<int64_t>(s) * n + c] = ew;
  }
}

// d[c] = the norm from the split pairs (their largest exponent, then a
// fixed-order block reduction); P(:, c) /= d[c] (a zero column stays zero).
// One workgroup per column.
__global__ __launch_bounds__(256) void colnorm_scale_kernel(const double* __restrict__ part,
                                                            const int* __restrict__ epart,
                                                            int nsplit, int n,
                                                            double* __restrict__ d,
                                                            double* __restrict__ P, int k,
                                                            int64_t ldp) {
  __shared__ double red[4];
  __shared__ int emax[4];
  const int c = blockIdx.x, t = threadIdx.x;
  int e = kEmpty;
  for (int i = t; i < nsplit; i += 256) e = max(e, epart[static_cast<int64_t>(i) * n + c]);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) e = max(e, __shfl_xor(e, off));
  if ((t & 63) == 0) emax[t >> 6] = e;
  __syncthreads();
  e = max(max(emax[0], emax[1]), max(emax[2], emax[3]));
  double s = 0.0;
  for (int i = t; i < nsplit; i += 256)
    s += ssq_at(Ssq{part[static_cast<int64_t>(i) * n + c], epart[static_cast<int64_t>(i) * n + c]},
                e);
  s = block_sum(s, red);
  const double dc = (e == kEmpty) ? 0.0 : ldexp(sqrt(s), e - 1023);
  if (t == 0) d[c] = dc;
  const double inv = (dc > 0.0) ? 1.0 / dc : 0.0;
  double* pc = P + static_cast<int64_t>(c) * ldp;
  for (int i = t; i < k; i += 256) pc[i] *= inv;
}

// Householder QR with column pivoting of the n x n upper triangular Rp (ld
// n).  W (n x n, row-major scratch) is the working matrix, kept in its
// original column order: column c belongs to the four threads c + 256 q,
// thread q taking the rows i = q mod 4, and the pivoted order is kept as a
// permutation (pos: position of a column, colat: column at a position).
// Step j: among the columns at positions >= j, the one of largest norm over
// rows j.. (recomputed from the previous update, lowest position on ties)
// goes to position j; its reflector (alpha = -sign(x_j) ||x||) is applied to
// the columns still unplaced.  Three barriers a step: after the reflector
// load, after the products, after the update.  Out: Rt (ld n, column-major,
// pivoted order, positive diagonal: rows flipped with alpha), the same
// factor row-major in Rw, piv.
constexpr int kQcpThreads = 4 * kMaxN;
constexpr int kQcRows = 16;  // rows per thread kept in registers within a step

__global__ __launch_bounds__(kQcpThreads) void qrcp_kernel(const double* __restrict__ Rp, int n,
                                                           double* __restrict__ W,
                                                           double* __restrict__ Rt,
                                                           double* __restrict__ Rw,
                                                           int* __restrict__ piv) {
  __shared__ double v[kMaxN];
  __shared__ double sgn[kMaxN];
  __shared__ double dotp[4][kMaxN];  // reflector products, by row class
  __shared__ double nrmp[4][kMaxN];  // squared norms below the current row, by row class
  __shared__ int pos[kMaxN];
  __shared__ int colat[kMaxN];
  const int tid = threadIdx.x, c = tid & (kMaxN - 1), q = tid >> 8, lane = tid & 63;
  const bool col = c < n;
  {
    double s = 0.0;
    if (col)
      for (int i = q; i < n; i += 4) {
        const double x = (i <= c) ? Rp[i + static_cast<int64_t>(c) * n] : 0.0;
        W[static_cast<int64_t>(i) * n + c] = x;
        s += x * x;
      }
    nrmp[q][c] = s;
    if (tid < kMaxN) {
      pos[tid] = tid;
      colat[tid] = tid;
    }
  }
  bool placed = false;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    // pivot, found by every wave alike (4 columns a lane)
    double best = -1.0;
    int bpos = n;
    for (int qq = 0; qq < 4; ++qq) {
      const int cc = lane + 64 * qq;
      if (cc < n) {
        const int pc = pos[cc];
        if (pc >= j) {
          double a = ((nrmp[0][cc] + nrmp[1][cc]) + nrmp[2][cc]) + nrmp[3][cc];
          if (!(a >= 0.0)) a = -0.5;  // a NaN norm takes the lowest priority
          if (a > best || (a == best && pc < bpos)) {
            best = a;
            bpos = pc;
          }
        }
      }
    }
    double mx = best;
    for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    int cand = (best == mx) ? bpos : n;
    for (int off = 32; off >= 1; off >>= 1) cand = min(cand, __shfl_xor(cand, off));
    const int p = colat[cand];
    const double nr2 = ((nrmp[0][p] + nrmp[1][p]) + nrmp[2][p]) + nrmp[3][p];
    for (int i = j + tid; i < n; i += kQcpThreads) v[i] = W[static_cast<int64_t>(i) * n + p];
    __syncthreads();
    const double x0 = v[j];
    const double nr = sqrt(nr2);
    const double alpha = (x0 >= 0.0) ? -nr : nr;
    const double v0 = x0 - alpha;
    const double vtv = v0 * v0 + (nr2 - x0 * x0);
    const double beta = (vtv > 0.0 && nr > 0.0) ? 2.0 / vtv : 0.0;
    const double rjj = (nr > 0.0) ? alpha : x0;
    if (tid == 0) {
      sgn[j] = (rjj < 0.0) ? -1.0 : 1.0;
      const int cj = colat[j], pp = pos[p];
      pos[cj] = pp;
      colat[pp] = cj;
      pos[p] = j;
      colat[j] = p;
    }
    const bool is_p = col && c == p;
    const bool upd = col && !placed && !is_p;
    placed = placed || is_p;
    const int is = j + ((q - j) & 3);  // this thread's first row >= j
    // the first kQcRows of this thread's rows stay in registers from the
    // products to the update (one read of W per row and step for them)
    double wc[kQcRows];
    {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      if (upd) {
#pragma unroll
        for (int u = 0; u < kQcRows; ++u) {
          const int i = is + 4 * u;
          const double w = (i < n) ? W[static_cast<int64_t>(i) * n + c] : 0.0;
          wc[u] = w;
          const double t = ((i < n) ? ((i == j) ? v0 : v[i]) : 0.0) * w;
          if ((u & 3) == 0) a0 += t;
          else if ((u & 3) == 1) a1 += t;
          else if ((u & 3) == 2) a2 += t;
          else a3 += t;
        }
        for (int i = is + 4 * kQcRows; i < n; i += 4) a0 += v[i] * W[static_cast<int64_t>(i) * n + c];
      }
      dotp[q][c] = (a0 + a1) + (a2 + a3);
    }
    __syncthreads();
    {
      double s0 = 0.0, s1 = 0.0;
      if (upd) {
        const double f = beta * (((dotp[0][c] + dotp[1][c]) + dotp[2][c]) + dotp[3][c]);
#pragma unroll
        for (int u = 0; u < kQcRows; ++u) {
          const int i = is + 4 * u;
          if (i < n) {
            const double x = wc[u] - f * ((i == j) ? v0 : v[i]);
            W[static_cast<int64_t>(i) * n + c] = x;
            // row j is final after this step and leaves the norm
            const double x2 = (i > j) ? x * x : 0.0;
            if (u & 1)
              s1 += x2;
            else
              s0 += x2;
          }
        }
        for (int i = is + 4 * kQcRows; i < n; i += 4) {
          const double x = W[static_cast<int64_t>(i) * n + c] - f * v[i];
          W[static_cast<int64_t>(i) * n + c] = x;
          s0 += x * x;
        }
      } else if (is_p) {
        for (int i = is; i < n; i += 4) W[static_cast<int64_t>(i) * n + c] = (i == j) ? rjj : 0.0;
      }
      nrmp[q][c] = s0 + s1;
    }
    __syncthreads();
  }
  if (col) {
    const int jc = pos[c];
    for (int i = q; i < n; i += 4) {
      const double a = (i <= jc) ? sgn[i] * W[static_cast<int64_t>(i) * n + c] : 0.0;
      Rt[i + static_cast<int64_t>(jc) * n] = a;
      Rw[static_cast<int64_t>(i) * n + jc] = a;
    }
    if (q == 0) piv[jc] = c;
  }
}

// Step 3, the rank: least r with ||Rt_{r:,r:}||_F <= tau ||Rt||_2, the
// 2-norm by at most 64 power-iteration steps on Rt^T Rt, fewer once the
// estimate has settled (kept in *sigma_out for the
// strong RRQR step).  The status word keeps only the non-finite flag (rank
// deficiency is expected).
// Rt is read column-major for the products Rt x and row-major (Rw) for
// Rt^T y, so that both are coalesced; output entry t of either product is
// the sum of four quarter sums (threads t + 256 q over indices 64 q ..
// 64 q + 63) added in q order.
constexpr int kFinThreads = 4 * kMaxN;

__global__ __launch_bounds__(kFinThreads) void rr_rank_kernel(
    const double* __restrict__ Rt, const double* __restrict__ Rw, int n, double tau,
    const double* __restrict__ d, double* __restrict__ sigma_out, int* __restrict__ rank,
    int* __restrict__ status) {
  __shared__ double x[kMaxN], y[kMaxN], qp[4][kMaxN], red[kFinThreads / 64];
  __shared__ double tail[kMaxN + 1];
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
    // y = Rt x, x = Rt^T y / ||Rt^T y||; stop once ||Rt x|| has settled to
    // 1e-12 relative (every thread holds the same block sums, so all stop
    // together)
    const double yy = mul_rt();
    const double prev = sigma;
    sigma = sqrt(yy);  // ||Rt x|| with ||x|| = 1 after the first step
    if (it >= 8 && fabs(sigma - prev) <= 1e-12 * sigma) break;
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
    *rank = r;
    *sigma_out = sigma;
    *status = (bad || !isfinite(sigma)) ? 2 : 0;
  }
}

// The outputs of step 3: R (ld ldr) = Rt_{1:r,:} diag(d[piv]) (rows >= r
// zero) and Rs (ld n), the factor of the solve: that block on 1:r, the
// identity on the dropped columns.
__global__ __launch_bounds__(256) void rr_out_kernel(const double* __restrict__ Rt, int n,
                                                     const double* __restrict__ d,
                                                     const int* __restrict__ piv,
                                                     const int* __restrict__ rank,
                                                     double* __restrict__ R, int64_t ldr,
                                                     double* __restrict__ Rs) {
  const int r = *rank;
  for (int idx = blockIdx.x * 256 + threadIdx.x; idx < n * n; idx += gridDim.x * 256) {
    const int i = idx % n, c = idx / n;
    const double v = (i < r && i <= c) ? Rt[i + static_cast<int64_t>(c) * n] * d[piv[c]] : 0.0;
    R[i + static_cast<int64_t>(c) * ldr] = v;
    Rs[idx] = (i < r && c < r) ? v : ((i == c) ? 1.0 : 0.0);
  }
}

// Strong RRQR (Gu and Eisenstat's swaps, with parameter f) on the pivoted
// factor for k = the rank of the rule: while the largest rho_ij^2 =
// (R11^{-1} R12)_ij^2 + ||R22 e_j||^2 ||e_i^T R11^{-1}||^2 (first in
// row-major order on ties) exceeds f^2, columns i and k + j trade places
// (and their labels in piv) and R is triangularised again by Householder
// steps from column i on (earlier columns are untouched), rows made
// positive.  At most 4n swaps.  Rw (row-major) is worked in place, Ri holds
// R11^{-1} (row-major); after a swap Rt is refreshed and the rank rule is
// applied again with the same ||R||_2 (the swaps keep the singular values).
constexpr int kSrThreads = 4 * kMaxN;

__global__ __launch_bounds__(kSrThreads) void srrqr_kernel(double* __restrict__ Rt,
                                                           double* __restrict__ Rw,
                                                           double* __restrict__ Ri, int n,
                                                           double tau, double f,
                                                           const double* __restrict__ sigma,
                                                           int* __restrict__ piv,
                                                           int* __restrict__ rank) {
  __shared__ double part[4][kMaxN];
  __shared__ double w2[kMaxN], g2[kMaxN], v[kMaxN], sgn[kMaxN], tail[kMaxN + 1];
  __shared__ double wbest[kSrThreads / 64];
  __shared__ int wkey[kSrThreads / 64];
  __shared__ double hb;
  const int tid = threadIdx.x, c = tid & (kMaxN - 1), q = tid >> 8;
  const int lane = tid & 63, wave = tid >> 6;
  const int k = *rank;
  if (k <= 0 || k >= n) return;
  auto at = [n](int i, int j) { return static_cast<int64_t>(i) * n + j; };
  bool swapped = false;
  for (int it = 0; it < 4 * n; ++it) {
    // Ri = R11^{-1}, row i from rows i+1.. (four row classes per column)
    for (int i = k - 1; i >= 0; --i) {
      double a = 0.0;
      if (c > i && c < k)
        for (int l = i + 1 + ((q - i - 1) & 3); l <= c; l += 4) a += Rw[at(i, l)] * Ri[at(l, c)];
      part[q][c] = a;
      __syncthreads();
      if (q == 0 && c >= i && c < k) {
        const double rii = Rw[at(i, i)];
        Ri[at(i, c)] =
            (c == i) ? 1.0 / rii : -(((part[0][c] + part[1][c]) + part[2][c]) + part[3][c]) / rii;
      }
      __syncthreads();
    }
    // squared row norms of R11^{-1}, squared column norms of R22
    {
      double s = 0.0;
      if (c < k)
        for (int l = c + ((q - c) & 3); l < k; l += 4) {
          const double x = Ri[at(c, l)];
          s += x * x;
        }
      else if (c < n)
        for (int l = k + ((q - k) & 3); l < n; l += 4) {
          const double x = Rw[at(l, c)];
          s += x * x;
        }
      part[q][c] = s;
    }
    __syncthreads();
    if (q == 0 && c < n) {
      const double s = ((part[0][c] + part[1][c]) + part[2][c]) + part[3][c];
      if (c < k)
        w2[c] = s;
      else
        g2[c] = s;
    }
    __syncthreads();
    // the largest rho^2: thread (c, q) takes column c of R12 and rows i = q mod 4
    double best = -1.0;
    int bkey = n * n;
    if (c >= k && c < n)
      for (int i = q; i < k; i += 4) {
        double a0 = 0.0, a1 = 0.0;
        int l = i;
        for (; l + 1 < k; l += 2) {
          a0 += Ri[at(i, l)] * Rw[at(l, c)];
          a1 += Ri[at(i, l + 1)] * Rw[at(l + 1, c)];
        }
        if (l < k) a0 += Ri[at(i, l)] * Rw[at(l, c)];
        const double a = a0 + a1;
        const double r2 = a * a + w2[i] * g2[c];
        if (r2 > best) {  // rows rise within a thread: the first of equal values stays
          best = r2;
          bkey = i * n + c;
        }
      }
    {
      double mx = best;
      for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
      int key = (best == mx) ? bkey : n * n;
      for (int off = 32; off >= 1; off >>= 1) key = min(key, __shfl_xor(key, off));
      if (lane == 0) {
        wbest[wave] = mx;
        wkey[wave] = key;
      }
    }
    __syncthreads();
    double gb = -1.0;
    int gk = n * n;
    for (int w = 0; w < kSrThreads / 64; ++w)
      if (wbest[w] > gb || (wbest[w] == gb && wkey[w] < gk)) {
        gb = wbest[w];
        gk = wkey[w];
      }
    __syncthreads();  // wbest and wkey are rewritten by the next round
    if (!(gb > f * f) || gk >= n * n) break;
    const int si = gk / n, sc = gk % n;
    if (tid < n) {
      const double a = Rw[at(tid, si)];
      Rw[at(tid, si)] = Rw[at(tid, sc)];
      Rw[at(tid, sc)] = a;
    }
    if (tid == 0) {
      const int p = piv[si];
      piv[si] = piv[sc];
      piv[sc] = p;
    }
    __syncthreads();
    // Householder from column si on, no pivoting
    for (int j = si; j < n; ++j) {
      for (int l = j + tid; l < n; l += kSrThreads) v[l] = Rw[at(l, j)];
      __syncthreads();
      if (wave == 0) {
        double s = 0.0;
        for (int l = j + lane; l < n; l += 64) s += v[l] * v[l];
        s = wave_sum(s);
        if (lane == 0) hb = s;
      }
      __syncthreads();
      const double nr2 = hb, x0 = v[j];
      const double nr = sqrt(nr2);
      const double alpha = (x0 >= 0.0) ? -nr : nr;
      const double v0 = x0 - alpha;
      const double vtv = v0 * v0 + (nr2 - x0 * x0);
      const double beta = (vtv > 0.0 && nr > 0.0) ? 2.0 / vtv : 0.0;
      const double rjj = (nr > 0.0) ? alpha : x0;
      if (tid == 0) sgn[j] = (rjj < 0.0) ? -1.0 : 1.0;
      const int is = j + ((q - j) & 3);
      const bool upd = c > j && c < n;
      {
        double a0 = 0.0, a1 = 0.0;
        if (upd) {
          int l = is;
          if (l == j) {
            a0 = v0 * Rw[at(j, c)];
            l += 4;
          }
          for (; l + 4 < n; l += 8) {
            a0 += v[l] * Rw[at(l, c)];
            a1 += v[l + 4] * Rw[at(l + 4, c)];
          }
          if (l < n) a0 += v[l] * Rw[at(l, c)];
        }
        part[q][c] = a0 + a1;
      }
      __syncthreads();
      if (upd) {
        const double fj = beta * (((part[0][c] + part[1][c]) + part[2][c]) + part[3][c]);
        for (int l = is; l < n; l += 4) Rw[at(l, c)] -= fj * ((l == j) ? v0 : v[l]);
      } else if (c == j) {
        for (int l = is; l < n; l += 4) Rw[at(l, j)] = (l == j) ? rjj : 0.0;
      }
      __syncthreads();
    }
    if (c < n)
      for (int l = si + ((q - si) & 3); l < n; l += 4) Rw[at(l, c)] *= sgn[l];
    __syncthreads();
    swapped = true;
  }
  if (!swapped) return;
  for (int idx = tid; idx < n * n; idx += kSrThreads)
    Rt[(idx % n) * static_cast<int64_t>(n) + idx / n] = Rw[idx];
  {
    double s = 0.0;
    if (c < n)
      for (int l = c + ((q - c) & 3); l < n; l += 4) {
        const double x = Rw[at(c, l)];
        s += x * x;
      }
    part[q][c] = s;
  }
  __syncthreads();
  if (tid == 0) {
    const double lim = tau * *sigma;
    tail[n] = 0.0;
    for (int i = n - 1; i >= 0; --i)
      tail[i] = tail[i + 1] + (((part[0][i] + part[1][i]) + part[2][i]) + part[3][i]);
    int r = n;
    for (int t = 0; t <= n; ++t)
      if (sqrt(tail[t]) <= lim) {
        r = t;
        break;
      }
    *rank = r;
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

// Second pass (Algorithm 3 steps 2-3 on the r columns of Q): R(0:r, :) <-
// U R(0:r, :) with U (ld ldu) upper triangular r x r.  One workgroup per
// column of R; the column is read into LDS before it is overwritten.
__global__ __launch_bounds__(256) void left_upper_kernel(const double* __restrict__ U,
                                                         int64_t ldu, int r,
                                                         double* __restrict__ R, int64_t ldr) {
  __shared__ double col[kMaxN];
  const int c = blockIdx.x, t = threadIdx.x;
  double* rc = R + static_cast<int64_t>(c) * ldr;
  if (t < r) col[t] = rc[t];
  __syncthreads();
  if (t < r) {
    double s = 0.0;
    for (int l = t; l < r; ++l) s += U[t + static_cast<int64_t>(l) * ldu] * col[l];
    rc[t] = s;
  }
}

hipError_t launch_left_upper(const double* U, int64_t ldu, int r, double* R, int64_t ldr, int n,
                             hipStream_t st) {
  left_upper_kernel<<<n, 256, 0, st>>>(U, ldu, r, R, ldr);
  return hipGetLastError();
}

size_t rr_extra_bytes(int n) {
  const size_t nn = static_cast<size_t>(n) * n * sizeof(double);
  return static_cast<size_t>(kRrSplits) * n * sizeof(double)  // norm partials
         + static_cast<size_t>(kRrSplits) * n * sizeof(double)  // their exponents (int)
         + n * sizeof(double)                                 // d
         + 5 * nn                                             // W, Rt, Rs, Rw, Ri
         + 256                                                // ||R||_2
         + 2 * n * sizeof(int) + 256;                         // piv, rank
}

hipError_t launch_rr_steps(const void* X, bool f32, int64_t m, int n, int64_t ldx, double* P,
                           int k, const double* Rp, double tau, double f, unsigned char* extra,
                           double* R, int64_t ldr, int* piv_out, int* rank_out, int* status,
                           double** Rs_out, hipStream_t st, int stage) {
  double* part = reinterpret_cast<double*>(extra);
  int* epart = reinterpret_cast<int*>(part + static_cast<size_t>(kRrSplits) * n);
  double* d = part + 2 * static_cast<size_t>(kRrSplits) * n;
  double* W = d + n;
  double* Rt = W + static_cast<size_t>(n) * n;
  double* Rs = Rt + static_cast<size_t>(n) * n;
  double* Rw = Rs + static_cast<size_t>(n) * n;
  double* Ri = Rw + static_cast<size_t>(n) * n;
  double* sig = Ri + static_cast<size_t>(n) * n;
  *Rs_out = Rs;
  if (stage == 0) {
    // column norms of X and the normalised sketch
    const int64_t rows = ceil_div(m, static_cast<int64_t>(kRrSplits));
    const dim3 grid(static_cast<unsigned>(ceil_div(n, 4)), kRrSplits);
    if (f32)
      colnorm_partial_kernel<float><<<grid, 256, 0, st>>>(static_cast<const float*>(X), m, n, ldx,
                                                           rows, part, epart);
    else
      colnorm_partial_kernel<double><<<grid, 256, 0, st>>>(static_cast<const double*>(X), m, n,
                                                            ldx, rows, part, epart);
    colnorm_scale_kernel<<<n, 256, 0, st>>>(part, epart, kRrSplits, n, d, P, k, k);
    return hipGetLastError();
  }
  qrcp_kernel<<<1, kQcpThreads, 0, st>>>(Rp, n, W, Rt, Rw, piv_out);
  rr_rank_kernel<<<1, kFinThreads, 0, st>>>(Rt, Rw, n, tau, d, sig, rank_out, status);
  if (f > 0.0)
    srrqr_kernel<<<1, kSrThreads, 0, st>>>(Rt, Rw, Ri, n, tau, f, sig, piv_out, rank_out);
  const unsigned out_blocks = static_cast<unsigned>(std::min<int64_t>(ceil_div(n * n, 256), 256));
  rr_out_kernel<<<out_blocks, 256, 0, st>>>(Rt, n, d, piv_out, rank_out, R, ldr, Rs);
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
