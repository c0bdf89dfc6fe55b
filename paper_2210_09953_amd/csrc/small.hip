// small.hip -- the FP64 small-matrix steps (Section 5: minor operations in
// higher precision), all on the GPU:
//   * Householder QR of the k x n sketch P (Algorithm 2 step 2; Householder
//     is the choice of the numerical experiments, Section 6.1), blocked in
//     16-column panels with the compact WY form H_1..H_16 = I - V T V^T:
//     one workgroup factors a panel in LDS, then one workgroup per
//     16-column block of the trailing matrix applies (I - V T^T V^T) on
//     matrix cores.  The sign fix D = sign(diag R) gives R_s = D R with a
//     positive diagonal; S = (H_1 ... H_n)[I; 0] D on request.
//   * Cholesky of the n x n Gram, upper factor A = R'^T R' (Algorithm 3
//     step 3), blocked right-looking in 32-column panels, one workgroup.
//   * R = R' R_s, panel packing of R for the tall solve, Gram reduction.
#include "common.h"
#include "kernels.h"

namespace rcq {

// ----------------------------------------------------------------------------
// Householder panel.  A (k x n, ld k) holds the matrix being factored; on
// exit columns p0..p0+15 hold R above the diagonal (diagonal = alpha) and
// the tail of each reflector v below it; v's leading entry goes to v0[],
// 2/(v^T v) to beta[], and the panel's 16 x 16 T to Tp.
// One wave per panel column, its rows (lane + 64 q) in registers.  Step j:
// the waves right of j apply reflector j (read from LDS) to their column,
// and wave j + 1 then forms reflector j + 1 from its updated column and
// publishes it in LDS: one barrier per reflector.  The wave that forms the
// next reflector raises its issue priority for the step, as the others'
// updates are off the critical path.  Reflector j sits at vsh[j Ls + r] for
// all 64 RPL rows (zero from row L on, so no reads are guarded), with the
// stride Ls = 4 (mod 32) doubles so that the 16 reflectors' entries of one
// row fall in distinct banks for the V^T V step.
// RPL = rows per lane (L <= 64 RPL).
__host__ __device__ constexpr int hh_panel_ld(int rpl) { return 64 * rpl + 4; }
template <int RPL>
__global__ __launch_bounds__(1024) void hh_panel_kernel(double* __restrict__ A, int k, int n,
                                                        int p0, double* __restrict__ v0g,
                                                        double* __restrict__ betag,
                                                        double* __restrict__ Tp) {
  extern __shared__ double vsh[];  // [16][Ls]: reflector j = vsh[j Ls + r] (0 above row j)
  __shared__ double sc[kHhPanel][3];
  __shared__ double y[kHhPanel][kHhPanel];
  __shared__ double ypart[8][kHhPanel][kHhPanel + 1];
  const int L = k - p0;
  constexpr int Ls = hh_panel_ld(RPL);
  const int nbp = (n - p0 < kHhPanel) ? n - p0 : kHhPanel;
  const int tid = threadIdx.x, wave = wave_index(), lane = tid & 63;
  const bool own = wave < nbp;
  double xr[RPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int r = lane + 64 * q;
    xr[q] = (own && r < L) ? A[(p0 + r) + static_cast<int64_t>(p0 + wave) * k] : 0.0;
  }
  // Wave j: reflector from its column (rows >= j), diagonal becomes alpha.
  auto reflect = [&](int j) {
    // rows >= L hold zeros; rows above j are all in q = 0 (j < 16)
    double tq[4] = {lane > j ? xr[0] * xr[0] : 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 1; q < RPL; ++q) tq[q & 3] += xr[q] * xr[q];
    const double t = wave_sum((tq[0] + tq[1]) + (tq[2] + tq[3]));
    const double x0 = read_lane(xr[0], j);  // j < 16: row j is lane j, q = 0
    const double nrm = sqrt(x0 * x0 + t);
    const double alpha = (x0 >= 0.0) ? -nrm : nrm;
    const double v0 = x0 - alpha;
    const double vtv = v0 * v0 + t;
    const double beta = (vtv > 0.0) ? 2.0 / vtv : 0.0;
    vsh[j * Ls + lane] = (lane < j) ? 0.0 : ((lane == j) ? v0 : xr[0]);
#pragma unroll
    for (int q = 1; q < RPL; ++q) vsh[j * Ls + lane + 64 * q] = xr[q];
    if (lane == j) xr[0] = alpha;
    if (lane == 0) {
      sc[j][0] = alpha;
      sc[j][1] = v0;
      sc[j][2] = beta;
    }
  };
  if (wave == 0 && nbp > 0) reflect(0);
  __syncthreads();
  for (int j = 0; j < nbp; ++j) {
    if (wave > j && own) {
      const bool next = wave == j + 1;
      if (next) __builtin_amdgcn_s_setprio(2);
      const double* vj = vsh + j * Ls;
      double wq[4] = {0.0, 0.0, 0.0, 0.0};
      double vr[RPL];
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        vr[q] = vj[lane + 64 * q];
        wq[q & 3] += vr[q] * xr[q];
      }
      const double w = wave_sum((wq[0] + wq[1]) + (wq[2] + wq[3]));
      const double f = sc[j][2] * w;
#pragma unroll
      for (int q = 0; q < RPL; ++q) xr[q] -= f * vr[q];
      if (next) {
        reflect(j + 1);
        __builtin_amdgcn_s_setprio(0);
      }
    }
    __syncthreads();
  }
  // y = V^T V (strict upper part used) on FP64 matrix cores: wave w sums the
  // rows of its chunk (A(a, r) = V(r, a), B(r, b) = V(r, b)); partials are
  // added in a fixed order (w + 8 into w, then w = 0..7).
  {
    const int l16 = lane & 15, lg = lane >> 4;
    const int chunk = ((L + 63) / 64) * 4;  // rows per wave, a multiple of 4
    const int rb = wave * chunk;
    d4 yp = d4{0.0, 0.0, 0.0, 0.0};
    for (int r0 = rb; r0 < rb + chunk; r0 += 4) {
      const int r = r0 + lg;
      const double av = (r < L && l16 < nbp) ? vsh[l16 * Ls + r] : 0.0;
      yp = mfma16x16x4(av, av, yp);
    }
    // waves 8..15 hand their partials to waves 0..7 (LDS for 8 partials)
    if (wave >= 8)
#pragma unroll
      for (int v = 0; v < 4; ++v) ypart[wave - 8][drow<double>(lg, v)][l16] = yp[v];
    __syncthreads();
    if (wave < 8)
#pragma unroll
      for (int v = 0; v < 4; ++v) yp[v] += ypart[wave][drow<double>(lg, v)][l16];
    __syncthreads();
    if (wave < 8)
#pragma unroll
      for (int v = 0; v < 4; ++v) ypart[wave][drow<double>(lg, v)][l16] = yp[v];
  }
  __syncthreads();
  if (tid < kHhPanel * kHhPanel) {
    const int a = tid >> 4, b = tid & 15;
    double sum = 0.0;
    for (int w = 0; w < 8; ++w) sum += ypart[w][a][b];
    y[a][b] = (a < b && b < nbp) ? sum : 0.0;
  }
  __syncthreads();
  // T upper (compact WY of the panel): T^{-1} = diag(1 / beta) + strict
  // upper part of V^T V, so column j of T follows by back substitution:
  // T(j, j) = beta_j, T(i, j) = -beta_i sum_{i < l <= j} y(i, l) T(l, j).
  // Lane j of wave 0 forms column j (entries below it stay zero).
  if (wave == 0 && lane < kHhPanel) {
    const int j = lane;
    double t[kHhPanel];
#pragma unroll
    for (int i = kHhPanel - 1; i >= 0; --i) {
      double ac[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int l = i + 1; l < kHhPanel; ++l) ac[l & 3] += y[i][l] * t[l];
      const double acc = (ac[0] + ac[1]) + (ac[2] + ac[3]);
      const double bi = (i < nbp) ? sc[i][2] : 0.0;
      t[i] = (j >= nbp || i > j) ? 0.0 : ((i == j) ? bi : -bi * acc);
    }
#pragma unroll
    for (int i = 0; i < kHhPanel; ++i) Tp[i + kHhPanel * j] = t[i];
  }
  if (tid < nbp) {
    v0g[p0 + tid] = sc[tid][1];
    betag[p0 + tid] = sc[tid][2];
  }
  if (own) {
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int r = lane + 64 * q;
      if (r < L) A[(p0 + r) + static_cast<int64_t>(p0 + wave) * k] = xr[q];
    }
  }
}

// M(p0:k, c_begin + 16 blockIdx.x + 0..15) <- (I - V T' V^T) M(...) with
// T' = T^T (trans = 1, factorisation) or T (trans = 0, forming S).  One
// workgroup of 16 waves per 16-column block; the L = k - p0 rows go in tiles
// of 16, tile g to wave g % 16 (TPW tiles per wave, L <= 256 TPW).  All on
// FP64 matrix cores: each wave sums W_w = V(rows_w, :)^T M(rows_w, :) over
// its tiles, the 16 partials are added in LDS in wave order, every wave forms
// Y = T' W and then M(rows_w, :) - V(rows_w, :) Y, with the M values it read
// for the first product kept in registers as the accumulator.  V is read
// from A (its tail below the diagonal) and v0[] (its leading entries).
// A wave reads and writes its 16 x 16 tiles of M and V four columns per
// instruction, each column's 16 rows a full 128-byte line (the operand
// layouts would touch 16 lines per instruction), and turns them into
// operands and back through its own LDS buffer.
constexpr int kHuLd = kHhPanel + 1;  // LDS row stride (doubles) of tiles and partials
template <int TPW>
__global__ __launch_bounds__(1024) void hh_update_kernel(const double* __restrict__ A, int k,
                                                         int n, int p0, const double* __restrict__ v0g,
                                                         const double* __restrict__ Tp, int trans,
                                                         double* __restrict__ M, int64_t ldm,
                                                         int c_begin, int c_end) {
  __shared__ double wp[16][kHhPanel][kHuLd];
  __shared__ double wsum[kHhPanel][kHuLd];
  __shared__ double tiles[16][2][kHhPanel][kHuLd];  // per wave: M, V tile as [column][row]
  const int L = k - p0;
  const int nref = (n - p0 < kHhPanel) ? n - p0 : kHhPanel;  // reflectors of the panel
  const int wave = wave_index(), lane = threadIdx.x & 63, l16 = lane & 15, lg = lane >> 4;
  const int cb = c_begin + kHhPanel * blockIdx.x;
  // Tile loads: load q reads column 4 q + lc, row lr.  Every address is
  // clamped into range and issued unconditionally, so that a wave's loads
  // are in flight together (a select on a loaded value becomes an
  // exec-masked branch holding the load, and a wait for it); V's structure
  // (zero above row i, v0[i] on it, the stored tail below) is applied by 0/1
  // factors (inputs are finite; a non-finite one is reported by the status
  // word).  M's clamped rows and columns need no mask: V is zero on those
  // rows and such outputs are never stored.
  const int lr = lane & 15, lc = lane >> 4;
  int64_t mcol[4], vcol[4];
  double v0q[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = 4 * q + lc, mc = cb + c, ic = c < nref ? c : nref - 1;
    mcol[q] = static_cast<int64_t>(mc < c_end ? mc : c_end - 1) * ldm;
    vcol[q] = static_cast<int64_t>(p0 + ic) * k;
    v0q[q] = v0g[p0 + ic];
  }
  auto load_tile = [&](int t, double* mld, double* vld) {
    const int r = 16 * (wave + 16 * t) + lr, rc = p0 + (r < L ? r : L - 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = 4 * q + lc;
      const bool ok = r < L && c < nref;
      mld[q] = M[rc + mcol[q]];
      vld[q] = A[rc + vcol[q]] * ((ok && r > c) ? 1.0 : 0.0) + v0q[q] * ((ok && r == c) ? 1.0 : 0.0);
    }
  };
  double (*mt)[kHuLd] = tiles[wave][0];
  double (*vt)[kHuLd] = tiles[wave][1];
  double mreg[TPW][4], va[TPW][4];
  d4 w = d4{0.0, 0.0, 0.0, 0.0};
  double mld[4], vld[4];
  load_tile(0, mld, vld);
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      mt[4 * q + lc][lr] = mld[q];
      vt[4 * q + lc][lr] = vld[q];
    }
    if (t + 1 < TPW) load_tile(t + 1, mld, vld);
    wave_sync();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      // A(i, kk) = V(r0 + kk, i), B(kk, j) = M(r0 + kk, j), r0 = 16 g + 4 s;
      // and the second product's A(rr, kk) = -V(16 g + rr, 4 s + kk)
      mreg[t][s] = mt[l16][4 * s + lg];
      w = mfma16x16x4(vt[l16][4 * s + lg], mreg[t][s], w);
      va[t][s] = -vt[4 * s + lg][l16];
    }
    wave_sync();
  }
  double ta[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int l = 4 * s + lg;
    ta[s] = trans ? Tp[l + kHhPanel * l16] : Tp[l16 + kHhPanel * l];  // T'(l16, l)
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) wp[wave][drow<double>(lg, v)][l16] = w[v];
  __syncthreads();
  if (threadIdx.x < kHhPanel * kHhPanel) {
    const int i = threadIdx.x >> 4, j = threadIdx.x & 15;
    double sum = 0.0;
    for (int ww = 0; ww < 16; ++ww) sum += wp[ww][i][j];
    wsum[i][j] = sum;
  }
  __syncthreads();
  // Y = T' W; element v of y holds Y(lg + 4 v, l16), which is the B operand
  // of step v of the second product.
  d4 y = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < 4; ++s) y = mfma16x16x4(ta[s], wsum[4 * s + lg][l16], y);
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    // C(rr, j) = M(16 g + rr, j): element v (row lg + 4 v) was read in step v
    d4 acc = d4{mreg[t][0], mreg[t][1], mreg[t][2], mreg[t][3]};
#pragma unroll
    for (int s = 0; s < 4; ++s) acc = mfma16x16x4(va[t][s], y[s], acc);
    // back to the load layout through the wave's tile buffer: full-line stores
#pragma unroll
    for (int v = 0; v < 4; ++v) mt[l16][drow<double>(lg, v)] = acc[v];
    wave_sync();
    const int r = 16 * (wave + 16 * t) + lr;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int col = cb + 4 * q + lc;
      const double val = mt[4 * q + lc][lr];
      if (r < L && col < c_end) M[(p0 + r) + static_cast<int64_t>(col) * ldm] = val;
    }
    wave_sync();
  }
}

__global__ void set_identity_kernel(double* S, int64_t lds, int k, int n) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(k) * n) return;
  const int i = static_cast<int>(idx % k), c = static_cast<int>(idx / k);
  S[i + c * lds] = (i == c) ? 1.0 : 0.0;
}

// Sign fix and status.  Rs (n x n, ld n) = D triu(A); R (optional, ld ldr)
// gets the same; S columns (optional) scaled by D.  Status: 2 if any R entry
// is not finite (non-finite input), 1 if a diagonal is 0; every block adds
// its finding with an integer atomic max into the status word, which
// reset_status_kernel zeroes before the factorisation.  Blocks 0..nb_r-1
// cover R, the rest cover S.
__global__ void reset_status_kernel(int* status) { *status = 0; }

// Column scaling before the factorisation: column c of A (k x n, ld k) is
// multiplied by 2^-e_c, e_c the exponent of its largest magnitude (0 for a
// zero or non-finite column), so that the sums of squares inside the
// reflectors neither underflow nor overflow.  Power-of-two scaling changes
// no rounding in the normal range and Householder QR commutes with it
// (QR(A D) = Q (R D)), so R is the same bits; hh_finalize_kernel multiplies
// column c of R back by 2^e_c.  One workgroup per column.
__global__ __launch_bounds__(256) void hh_colscale_kernel(double* __restrict__ A, int k,
                                                          int* __restrict__ cexp) {
  __shared__ double red[4];
  const int c = blockIdx.x;
  double* col = A + static_cast<int64_t>(c) * k;
  double mx = 0.0;
  bool bad = false;
  for (int i = threadIdx.x; i < k; i += 256) {
    const double a = fabs(col[i]);
    bad |= !isfinite(a);
    mx = fmax(mx, a);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  const bool anybad = __syncthreads_or(bad);
  if (lane == 0) red[wave] = mx;
  __syncthreads();
  mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  int e = 0;
  if (!anybad && mx > 0.0) {
    int ex = 0;
    (void)frexp(mx, &ex);
    e = ex - 1;  // mx 2^-e in [1, 2)
  }
  if (threadIdx.x == 0) cexp[c] = e;
  if (e != 0)
    for (int i = threadIdx.x; i < k; i += 256) col[i] = ldexp(col[i], -e);
}

__global__ __launch_bounds__(256) void hh_finalize_kernel(const double* __restrict__ A, int k,
                                                          int n, const int* __restrict__ cexp,
                                                          double* __restrict__ Rs,
                                                          double* __restrict__ R, int64_t ldr,
                                                          double* __restrict__ S, int64_t lds,
                                                          int nb_r, int* __restrict__ status) {
  __shared__ int worst;
  if (threadIdx.x == 0) worst = 0;
  __syncthreads();
  int code = 0;
  if (static_cast<int>(blockIdx.x) < nb_r) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx < n * n) {
      const int r = idx % n, c = idx / n;
      double v = 0.0;
      if (r <= c) {
        const double d = (A[r + static_cast<int64_t>(r) * k] < 0.0) ? -1.0 : 1.0;
        v = ldexp(d * A[r + static_cast<int64_t>(c) * k], cexp[c]);
        if (!isfinite(v)) code = 2;
        else if (r == c && !(v > 0.0)) code = 1;
      }
      Rs[r + c * n] = v;
      if (R) R[r + c * ldr] = v;
    }
  } else if (S) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x - nb_r) * 256 + threadIdx.x;
    if (idx < static_cast<int64_t>(k) * n) {
      const int i = static_cast<int>(idx % k), c = static_cast<int>(idx / k);
      const double d = (A[c + static_cast<int64_t>(c) * k] < 0.0) ? -1.0 : 1.0;
      S[i + c * lds] *= d;
    }
  }
  if (code) atomicMax(&worst, code);
  __syncthreads();
  if (threadIdx.x == 0 && worst) atomicMax(status, worst);
}

hipError_t launch_householder(double* A, int k, int n, double* V0, double* beta, double* T,
                              double* S, int64_t lds, double* Rs, double* R, int64_t ldr,
                              int* status, hipStream_t st) {
  hipError_t e;
  static bool attr_done = false;
  if (!attr_done) {
    const void* pk[] = {reinterpret_cast<const void*>(hh_panel_kernel<4>),
                        reinterpret_cast<const void*>(hh_panel_kernel<8>),
                        reinterpret_cast<const void*>(hh_panel_kernel<12>),
                        reinterpret_cast<const void*>(hh_panel_kernel<16>)};
    for (int i = 0; i < 4; ++i) {
      e = hipFuncSetAttribute(pk[i], hipFuncAttributeMaxDynamicSharedMemorySize,
                              static_cast<int>(kHhPanel * hh_panel_ld(16) * sizeof(double)));
      if (e != hipSuccess) return e;
    }
    attr_done = true;
  }
  reset_status_kernel<<<1, 1, 0, st>>>(status);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int npan = static_cast<int>(ceil_div(n, kHhPanel));
  // the column exponents live after the panels' T blocks (hh_t_bytes)
  int* cexp = reinterpret_cast<int*>(T + static_cast<int64_t>(npan) * kHhPanel * kHhPanel);
  hh_colscale_kernel<<<n, 256, 0, st>>>(A, k, cexp);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // Rows per lane of the one-wave-per-column kernels, from the panel height.
#define RCQ_HH_RPL(L, STMT)                            \
  do {                                                 \
    const int rows_ = (L);                             \
    if (rows_ <= 256) {                                \
      constexpr int RPL = 4;                           \
      STMT;                                            \
    } else if (rows_ <= 512) {                         \
      constexpr int RPL = 8;                           \
      STMT;                                            \
    } else if (rows_ <= 768) {                         \
      constexpr int RPL = 12;                          \
      STMT;                                            \
    } else {                                           \
      constexpr int RPL = 16;                          \
      STMT;                                            \
    }                                                  \
  } while (0)
  for (int p = 0; p < npan; ++p) {
    const int p0 = p * kHhPanel;
    RCQ_HH_RPL(k - p0, (hh_panel_kernel<RPL><<<1, 1024, kHhPanel * hh_panel_ld(RPL) * sizeof(double), st>>>(
                           A, k, n, p0, V0, beta, T + p * kHhPanel * kHhPanel)));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int cstart = p0 + kHhPanel;
    if (cstart < n) {
      const int nblk = static_cast<int>(ceil_div(n - cstart, kHhPanel));
      RCQ_HH_RPL(k - p0, (hh_update_kernel<RPL / 4><<<nblk, 1024, 0, st>>>(
                             A, k, n, p0, V0, T + p * kHhPanel * kHhPanel, 1, A, k, cstart, n)));
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  if (S) {
    const int64_t tot = static_cast<int64_t>(k) * n;
    set_identity_kernel<<<static_cast<unsigned>(ceil_div(tot, 256)), 256, 0, st>>>(S, lds, k, n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int p = npan - 1; p >= 0; --p) {
      const int p0 = p * kHhPanel;
      const int nblk = static_cast<int>(ceil_div(n - p0, kHhPanel));
      RCQ_HH_RPL(k - p0, (hh_update_kernel<RPL / 4><<<nblk, 1024, 0, st>>>(
                             A, k, n, p0, V0, T + p * kHhPanel * kHhPanel, 0, S, lds, p0, n)));
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
#undef RCQ_HH_RPL
  const int nb_r = static_cast<int>(ceil_div(n * n, 256));
  const int nb_s = S ? static_cast<int>(ceil_div(static_cast<int64_t>(k) * n, 256)) : 0;
  hh_finalize_kernel<<<nb_r + nb_s, 256, 0, st>>>(A, k, n, cexp, Rs, R, ldr, S, lds, nb_r,
                                                  status);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Cholesky, upper, in place on G (ld ldg); only the upper triangle is read
// and written.  Right-looking in 16-column panels with the whole upper
// triangle held in registers as 16 x 16 tiles (tile (i, j), i <= j, belongs
// to wave (tile index) % 8 of one 512-thread workgroup):
//   1. one wave factors the diagonal tile in registers (a lane per column,
//      pivots and rows shared by lane reads) and, by the same elimination
//      on the identity, forms W^T = R_PP^{-T};
//   2. the owners of row P's tiles form R_Pj = W^T G_Pj on FP64 matrix cores
//      (a tile's accumulator layout is the B operand's) and publish them;
//   3. the owners of the trailing tiles subtract R_Pi^T R_Pj on matrix cores.
// Status 1000 + j at the first pivot that is not positive and finite (only
// if the status word is still 0).
constexpr int kChTiles = (kMaxN / 16) * (kMaxN / 16 + 1) / 2;  // 136
constexpr int kChWaves = 8;
constexpr int kChPerWave = (kChTiles + kChWaves - 1) / kChWaves;  // 17

__global__ __launch_bounds__(64 * kChWaves) void chol_kernel(double* __restrict__ G, int n, int ldg,
                                                    int* __restrict__ status) {
  __shared__ double dgb[16][17];        // diagonal tile being factored
  __shared__ double wl[16][17];         // W^T, W = R_PP^{-1}
  __shared__ double rp[16][kMaxN + 1];  // row panel R_P,: (16 x n)
  __shared__ double xt[kChWaves][16][17];  // per wave: a tile on its way to or from G
  __shared__ int fail;
  const int tid = threadIdx.x, wave = wave_index(), lane = tid & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  const int nt = (n + 15) / 16;
  const int ntile = nt * (nt + 1) / 2;
  if (tid == 0) fail = 0;
  // Tile index -> (i, j), column-major over the upper triangle.  Lane u of
  // each wave decodes the wave's u-th tile once, packed as i | j << 8 | (not
  // a tile) << 16; the loops below read it back with a lane read.
  int tcode = 1 << 16;
  if (lane < kChPerWave) {
    int t = wave + kChWaves * lane, tj = 0;
    const bool live = t < ntile;
    while (t > tj) {
      t -= tj + 1;
      ++tj;
    }
    tcode = t | (tj << 8) | (live ? 0 : 1 << 16);
  }
  auto decode = [&](int u, int& ti, int& tj) -> bool {
    const int code = __builtin_amdgcn_readlane(tcode, u);
    ti = code & 255;
    tj = (code >> 8) & 255;
    return (code >> 16) == 0;
  };
  // Tiles move between G and the accumulators through the wave's LDS tile
  // xt[column][row]: a load or store covers four columns of 16 rows (full
  // 128-byte lines), where the accumulator layout would touch 16 lines.
  // Loads come from clamped addresses in the upper triangle (an element
  // below the diagonal reads its mirror image), unconditionally and with the
  // mask applied by 0/1 factors, so that they are all in flight together (a
  // select on a loaded value is compiled into a branch and a wait per load).
  // Padding beyond n is the identity.
  double (*xw)[17] = xt[wave];
  auto load_tile = [&](int u, double* x) {
    int ti, tj;
    const bool live = decode(u, ti, tj);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 16 * ti + l16, c = 16 * tj + 4 * q + lg;
      const int rc = r < n ? r : n - 1, cc = c < n ? c : n - 1;
      const bool inb = r < n && c < n;
      const double g = G[(rc < cc ? rc : cc) + static_cast<int64_t>(rc < cc ? cc : rc) * ldg];
      x[q] = g * ((live && inb && r <= c) ? 1.0 : 0.0) + ((live && !inb && r == c) ? 1.0 : 0.0);
    }
  };
  d4 acc[kChPerWave];
  double xl[4];
  load_tile(0, xl);
#pragma unroll
  for (int u = 0; u < kChPerWave; ++u) {
#pragma unroll
    for (int q = 0; q < 4; ++q) xw[4 * q + lg][l16] = xl[q];
    if (u + 1 < kChPerWave) load_tile(u + 1, xl);
    wave_sync();
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = xw[l16][drow<double>(lg, v)];
    wave_sync();
  }
  for (int P = 0; P < nt; ++P) {
    // 1. the diagonal tile to LDS (its owner), then wave 0 factors it.
    const int tdiag = P * (P + 1) / 2 + P;
#pragma unroll
    for (int u = 0; u < kChPerWave; ++u)
      if (wave + kChWaves * u == tdiag)
#pragma unroll
        for (int v = 0; v < 4; ++v) dgb[drow<double>(lg, v)][l16] = acc[u][v];
    __syncthreads();
    if (wave == 0 && lane < 32) {
      // Lanes 0..15 hold column c = lane of the tile, lanes 16..31 column
      // c = lane - 16 of the identity, 16 values each in registers.  The
      // elimination that turns the tile into R (row j scaled by 1 / r_jj,
      // rows below it reduced) turns the identity into R^{-T} = W^T; the
      // pivot and row j reach every lane by lane reads.
      const bool apart = lane < 16;
      const int c = lane & 15;
      double col[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) col[i] = apart ? dgb[i][c] : ((i == c) ? 1.0 : 0.0);
      double dn = read_lane(col[0], 0);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const double d = dn;
        const bool ok = (d > 0.0) && isfinite(d);
        // 1 / sqrt(d) from the hardware estimate and two Newton steps
        // (y <- y (3/2 - d y^2 / 2), each squaring the relative error): a
        // few dependent FMAs instead of a correctly rounded square root and
        // division on this serial chain.
        const double dd = ok ? d : 1.0;
        const double hd = 0.5 * dd;
        double ri = __builtin_amdgcn_rsq(dd);
        ri *= __builtin_fma(-hd, ri * ri, 1.5);
        ri *= __builtin_fma(-hd, ri * ri, 1.5);
        if (!ok && lane == 0 && fail == 0 && 16 * P + j < n) fail = 16 * P + j + 1;
        // row j: R(j, c) = A(j, c) / sqrt(d), lane j's own entry giving
        // d / sqrt(d) = sqrt(d); the identity part is scaled whole.  Rows i > j:
        // A(i, c) -= R(j, i) R(j, c).  Only entries on or above the diagonal
        // are ever read (pivots and R(j, i) with j < i), so the tile part's
        // lanes update below the diagonal too instead of masking.
        col[j] *= ri;
        if (j + 1 < 16) dn = read_lane(__builtin_fma(-col[j], col[j], col[j + 1]), j + 1);
#pragma unroll
        for (int i = j + 1; i < 16; ++i) col[i] = __builtin_fma(-read_lane(col[j], i), col[j], col[i]);
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        if (apart)
          dgb[i][c] = (i <= c) ? col[i] : 0.0;
        else
          wl[i][c] = col[i];  // W^T(i, c)
      }
    }
    __syncthreads();
    if (fail) break;
    // 2. row P: diagonal tile <- R_PP; R_Pj = W^T G_Pj for j > P.
#pragma unroll
    for (int u = 0; u < kChPerWave; ++u) {
      int ti, tj;
      if (!decode(u, ti, tj) || ti != P) continue;
      if (tj == P) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rr = drow<double>(lg, v);
          acc[u][v] = (rr <= l16) ? dgb[rr][l16] : 0.0;
        }
      } else {
        d4 y = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int sk = 0; sk < 4; ++sk)  // A(M = l16, K = 4 sk + lg) = W^T(l16, 4 sk + lg)
          y = mfma16x16x4(wl[l16][4 * sk + lg], acc[u][sk], y);
        acc[u] = y;
#pragma unroll
        for (int v = 0; v < 4; ++v) rp[drow<double>(lg, v)][16 * tj + l16] = y[v];
      }
    }
    __syncthreads();
    // 3. trailing tiles (i, j), P < i <= j: G_ij -= R_Pi^T R_Pj.
#pragma unroll
    for (int u = 0; u < kChPerWave; ++u) {
      int ti, tj;
      if (!decode(u, ti, tj) || ti <= P) continue;
#pragma unroll
      for (int sk = 0; sk < 4; ++sk) {
        const double a = -rp[4 * sk + lg][16 * ti + l16];  // A(M = l16, K) = R_Pi(K, l16)
        const double bb = rp[4 * sk + lg][16 * tj + l16];  // B(K, N = l16) = R_Pj(K, l16)
        acc[u] = mfma16x16x4(a, bb, acc[u]);
      }
    }
    // the next panel's first barrier orders these updates before its reads
  }
  __syncthreads();
  if (!fail) {
#pragma unroll
    for (int u = 0; u < kChPerWave; ++u) {
      int ti, tj;
      if (!decode(u, ti, tj)) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) xw[l16][drow<double>(lg, v)] = acc[u][v];
      wave_sync();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 16 * ti + l16, c = 16 * tj + 4 * q + lg;
        const double x = xw[4 * q + lg][l16];
        if (r < n && c < n && r <= c) G[r + static_cast<int64_t>(c) * ldg] = x;
      }
      wave_sync();
    }
  }
  if (tid == 0 && fail) atomicCAS(status, 0, 1000 + fail - 1);
}

hipError_t launch_cholesky(double* G, int n, int ldg, int* status, hipStream_t st) {
  chol_kernel<<<1, 64 * kChWaves, 0, st>>>(G, n, ldg, status);
  return hipGetLastError();
}

// C = A B for upper triangular A, B (strict lower part of C set to 0).
__global__ __launch_bounds__(256) void triu_product_kernel(const double* __restrict__ A,
                                                           int64_t lda,
                                                           const double* __restrict__ B,
                                                           int64_t ldb, double* __restrict__ C,
                                                           int64_t ldc, int n) {
  // C(:, c) = triu(A) B(:, c) for upper triangular A, B; block c, thread r.
  __shared__ double bc[kMaxN];
  const int c = blockIdx.x, r = threadIdx.x;
  if (r < n) bc[r] = (r <= c) ? B[r + static_cast<int64_t>(c) * ldb] : 0.0;
  __syncthreads();
  if (r >= n) return;
  double s = 0.0;
  if (r <= c) {
    int l = r;
    for (; l + 8 <= c + 1; l += 8) {
      double a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = A[r + static_cast<int64_t>(l + u) * lda];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += a[u] * bc[l + u];
    }
    for (; l <= c; ++l) s += A[r + static_cast<int64_t>(l) * lda] * bc[l];
  }
  C[r + static_cast<int64_t>(c) * ldc] = s;
}

hipError_t launch_triu_product(const double* A, int64_t lda, const double* B, int64_t ldb,
                               double* C, int64_t ldc, int n, hipStream_t st) {
  triu_product_kernel<<<static_cast<unsigned>(n), 256, 0, st>>>(A, lda, B, ldb, C, ldc, n);
  return hipGetLastError();
}

__global__ void copy_upper_kernel(const double* __restrict__ A, int64_t lda, double* __restrict__ B,
                                  int64_t ldb, int n) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int r = idx % n, c = idx / n;
  B[r + c * ldb] = (r <= c) ? A[r + c * lda] : 0.0;
}

hipError_t launch_copy_upper(const double* A, int64_t lda, double* B, int64_t ldb, int n,
                             hipStream_t st) {
  copy_upper_kernel<<<static_cast<unsigned>(ceil_div(n * n, 256)), 256, 0, st>>>(A, lda, B, ldb, n);
  return hipGetLastError();
}

// Panel packing for the tall passes.  Panel b (16 columns 16b..16b+15)
// holds rows 0..16b+15 row-major (16 entries per row): the upper triangle
// of R in the diagonal block, and above it R times offdiag_sign: -1 for the
// solve (its matrix-core update subtracts), +1 for the triangular product.
// Columns past n are padded with the identity.
template <typename T>
__global__ void make_panels_kernel(const double* __restrict__ R, int64_t ldr, int n,
                                   T* __restrict__ pan, int64_t total, double offdiag_sign) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  // locate panel b: offset(b) = 256 b (b+1) / 2
  int b = 0;
  while (256ll * (b + 1) * (b + 2) / 2 <= idx) ++b;
  const int64_t off = idx - 256ll * b * (b + 1) / 2;
  const int r = static_cast<int>(off / 16), c = static_cast<int>(off % 16);
  const int col = 16 * b + c;
  double v;
  if (r < 16 * b) {
    v = (col < n && r < n) ? offdiag_sign * R[r + col * ldr] : 0.0;
  } else {
    if (col < n && r < n)
      v = (r <= col) ? R[r + col * ldr] : 0.0;
    else
      v = (r == col) ? 1.0 : 0.0;
    if (r == col && offdiag_sign < 0.0) v = 1.0 / v;  // the solve multiplies by 1/R_jj
  }
  pan[idx] = static_cast<T>(v);
}

// Operand panels of an upper triangular R (n x n, ld ldr) for the FP32 solve
// trsm_bf3_kernel.  Subpanel b (output columns 16b..16b+15) holds
//  - (b+1)/2 update chunks: chunk p covers Q columns 32p..32p+31 in the
//    order in which the solved values sit in registers: K = 8 lg + e is
//    column 32p + 4lg + e for e < 4 and 32p + 16 + 4lg + (e - 4) for e >= 4.
//    Lane (lg, l16) holds -R(col(K), 16b + l16) where col(K) < 16b (else 0),
//    FP32 split exactly into three bf16 planes: 3 planes x 64 lanes x 16 B;
//  - the inverse Tb of the 16 x 16 diagonal block (FP64 substitution, then
//    FP32, split): lane (lg, l16) holds Tb(4 lg + e, l16), e < 4: 3 planes x
//    64 lanes x 8 B;
//  - the block itself, negated, in the same layout: -Rbb(4 lg + e, l16),
//    the operand of the solve's refinement residual D - Rbb^T E.
// Columns past n are zero (their solved values are zero).  Block b also
// writes flags[b] = 1 when a = || |Tb| |Rbb| ||_inf exceeds max(n, 32).
// Applying Tb costs a backward error of about a u |q_b| |Rbb| on a row,
// against the n u |q| |R| of row-wise substitution (Higham Thm 8.5): up to
// a = n the block inverse stays within that bound (a is 12 - 36 on the
// graded test matrices), beyond it the solve adds one refinement step on
// that launch.  One 64-thread block per subpanel.
__device__ __forceinline__ void split3_bits(double v, uint32_t& h, uint32_t& d, uint32_t& l) {
  const float x = static_cast<float>(v);
  h = __float_as_uint(x) & 0xFFFF0000u;
  const float r = x - __uint_as_float(h);
  d = __float_as_uint(r) & 0xFFFF0000u;
  l = __float_as_uint(r - __uint_as_float(d));
}

__global__ __launch_bounds__(64) void make_trsm_bf3_panels_kernel(const double* __restrict__ R,
                                                                  int64_t ldr, int n,
                                                                  unsigned char* __restrict__ pan3,
                                                                  int* __restrict__ flags) {
  __shared__ double rb[16][17];  // the diagonal block (identity past n)
  __shared__ double tb[16][17];
  __shared__ double amp[16];
  const int b = blockIdx.x, lane = threadIdx.x;
  const int l16 = lane & 15, lg = lane >> 4;
  const int c0 = 16 * b;
  // Every global load is issued unconditionally from a clamped in-range
  // address with its mask applied afterwards by 0/1 factors, so that a
  // lane's loads are in flight together (a select on a loaded value is
  // compiled into a branch and a wait per load); the serial steps below
  // then read the block from LDS.
  auto rat = [&](int r, int c) -> double {
    return R[(r < n ? r : n - 1) + static_cast<int64_t>(c < n ? c : n - 1) * ldr];
  };
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int i = 4 * lg + e, j = l16;
    const bool in = c0 + j < n && i <= j;
    rb[i][j] = rat(c0 + i, c0 + j) * (in ? 1.0 : 0.0) + ((c0 + j >= n && i == j) ? 1.0 : 0.0);
  }
  __syncthreads();
  if (lane < 16) {
    // column j = lane of Tb by back substitution (upper triangular)
    const int j = lane;
    for (int i = 15; i >= 0; --i) {
      double t = 0.0;
      if (i <= j && c0 + j < n) {
        if (i == j) {
          t = 1.0 / rb[j][j];
        } else {
          double s = 0.0;
          for (int l = i + 1; l <= j; ++l) s += rb[i][l] * tb[l][j];
          t = -s / rb[i][i];
        }
      }
      tb[i][j] = t;
    }
  }
  __syncthreads();
  const int nc = (b + 1) / 2;
  unsigned char* base = pan3 + trsm_bf3_panel_offset(b);
  const int col = c0 + l16;
  constexpr int kMaxChunks = (kMaxN / 16 + 1) / 2;
  double rv[kMaxChunks][8];
#pragma unroll
  for (int p = 0; p < kMaxChunks; ++p)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 32 * p + (e < 4 ? 4 * lg + e : 16 + 4 * lg + (e - 4));
      const bool in = p < nc && k < c0 && col < n;
      const double x = -rat(in ? k : 0, col);
      rv[p][e] = in ? x : 0.0;
    }
#pragma unroll
  for (int p = 0; p < kMaxChunks; ++p) {
    if (p >= nc) break;
    uint32_t hp[8], dp[8], lp[8];
    for (int e = 0; e < 8; ++e) split3_bits(rv[p][e], hp[e], dp[e], lp[e]);
    unsigned char* dst = base + 3072 * p;
    for (int w = 0; w < 4; ++w) {
      reinterpret_cast<uint32_t*>(dst + 16 * lane)[w] = (hp[2 * w] >> 16) | (hp[2 * w + 1] & 0xFFFF0000u);
      reinterpret_cast<uint32_t*>(dst + 1024 + 16 * lane)[w] = (dp[2 * w] >> 16) | (dp[2 * w + 1] & 0xFFFF0000u);
      reinterpret_cast<uint32_t*>(dst + 2048 + 16 * lane)[w] = (lp[2 * w] >> 16) | (lp[2 * w + 1] & 0xFFFF0000u);
    }
  }
  unsigned char* dd = base + 3072 * nc;
  for (int part = 0; part < 2; ++part) {
    uint32_t hp[4], dp[4], lp[4];
    for (int e = 0; e < 4; ++e) {
      const int i = 4 * lg + e;
      double v;
      if (part == 0)
        v = tb[i][l16];
      else
        v = (i <= l16 && c0 + l16 < n) ? -rb[i][l16] : 0.0;
      split3_bits(v, hp[e], dp[e], lp[e]);
    }
    unsigned char* dq = dd + 1536 * part;
    for (int w = 0; w < 2; ++w) {
      reinterpret_cast<uint32_t*>(dq + 8 * lane)[w] = (hp[2 * w] >> 16) | (hp[2 * w + 1] & 0xFFFF0000u);
      reinterpret_cast<uint32_t*>(dq + 512 + 8 * lane)[w] = (dp[2 * w] >> 16) | (dp[2 * w + 1] & 0xFFFF0000u);
      reinterpret_cast<uint32_t*>(dq + 1024 + 8 * lane)[w] = (lp[2 * w] >> 16) | (lp[2 * w + 1] & 0xFFFF0000u);
    }
  }
  // Row i of |Tb| |Rbb| (both upper triangular), its largest sum decides.
  if (lane < 16) {
    const int i = lane;
    double rs = 0.0;
    for (int j = i; j < 16; ++j) {
      double t = 0.0;
      for (int l = i; l <= j; ++l) t += fabs(tb[i][l]) * fabs(rb[l][j]);
      rs += t;
    }
    amp[i] = rs;
  }
  __syncthreads();
  if (lane == 0) {
    double a = 0.0;
    for (int i = 0; i < 16; ++i) a = fmax(a, amp[i]);
    // NaN (a failed factorisation) also asks for the refinement: harmless
    flags[b] = (a <= fmax(32.0, static_cast<double>(n))) ? 0 : 1;
  }
}

hipError_t launch_make_panels(const double* R, int64_t ldr, int n, bool f32, void* pan,
                              hipStream_t st, bool negate) {
  const int64_t total = panel_elems(n);
  const unsigned grid = static_cast<unsigned>(ceil_div(total, 256));
  const double sg = negate ? -1.0 : 1.0;
  if (f32 && negate) {
    // FP32 solve: bf16 x 3 operand panels with inverted diagonal blocks
    unsigned char* p3 = static_cast<unsigned char*>(pan);
    make_trsm_bf3_panels_kernel<<<static_cast<unsigned>(ceil_div(n, 16)), 64, 0, st>>>(
        R, ldr, n, p3, reinterpret_cast<int*>(p3 + trsm_bf3_flags_offset(n)));
    return hipGetLastError();
  }
  if (f32)
    make_panels_kernel<float><<<grid, 256, 0, st>>>(R, ldr, n, static_cast<float*>(pan), total, sg);
  else
    make_panels_kernel<double><<<grid, 256, 0, st>>>(R, ldr, n, static_cast<double*>(pan), total, sg);
  return hipGetLastError();
}

// bf16 x 3 operand panels of an upper triangular T (n x n, ld ldt) for
// trmm_bf3_kernel: panel b, chunk ch <= b/2, plane p (h, d, l), lane
// (lg, l16) holds the 8 values T(32 ch + 8 lg + e, 16 b + l16), e < 8, of
// FP32(T) split exactly into three bf16 parts, as 16 bytes.  Entries below
// the diagonal or past n are 0, except 1 on the diagonal past n.
__global__ void make_bf3_panels_kernel(const double* __restrict__ T, int64_t ldt, int n, int nb,
                                       unsigned char* __restrict__ pan3) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // (b, ch, lane)
  // panel b has (b/2 + 1) chunks of 64 lanes
  int b = 0, base = 0;
  while (b < nb && base + 64 * (b / 2 + 1) <= idx) {
    base += 64 * (b / 2 + 1);
    ++b;
  }
  if (b >= nb) return;
  const int rem = idx - base, ch = rem / 64, lane = rem % 64;
  const int l16 = lane & 15, lg = lane >> 4;
  const int col = 16 * b + l16;
  uint32_t hp[8], dp[8], lp[8];
  for (int e = 0; e < 8; ++e) {
    const int k = 32 * ch + 8 * lg + e;
    double v;
    if (k < n && col < n)
      v = (k <= col) ? T[k + static_cast<int64_t>(col) * ldt] : 0.0;
    else
      v = (k == col) ? 1.0 : 0.0;
    const float x = static_cast<float>(v);
    hp[e] = __float_as_uint(x) & 0xFFFF0000u;
    const float r = x - __uint_as_float(hp[e]);
    dp[e] = __float_as_uint(r) & 0xFFFF0000u;
    lp[e] = __float_as_uint(r - __uint_as_float(dp[e]));
  }
  // chunk ch of panel b: 3 planes x 64 lanes x 16 bytes
  unsigned char* dst = pan3 + 3072 * (base / 64 + ch);
  for (int w = 0; w < 4; ++w) {
    reinterpret_cast<uint32_t*>(dst + 16 * lane)[w] = (hp[2 * w] >> 16) | (hp[2 * w + 1] & 0xFFFF0000u);
    reinterpret_cast<uint32_t*>(dst + 1024 + 16 * lane)[w] = (dp[2 * w] >> 16) | (dp[2 * w + 1] & 0xFFFF0000u);
    reinterpret_cast<uint32_t*>(dst + 2048 + 16 * lane)[w] = (lp[2 * w] >> 16) | (lp[2 * w + 1] & 0xFFFF0000u);
  }
}

int64_t bf3_panel_bytes(int n) {
  const int nb = static_cast<int>(ceil_div(n, 16));
  int64_t chunks = 0;
  for (int b = 0; b < nb; ++b) chunks += b / 2 + 1;
  return 3072 * chunks;
}

hipError_t launch_make_bf3_panels(const double* T, int64_t ldt, int n, void* pan3, hipStream_t st) {
  const int nb = static_cast<int>(ceil_div(n, 16));
  const int64_t lanes = bf3_panel_bytes(n) / 3072 * 64;
  make_bf3_panels_kernel<<<static_cast<unsigned>(ceil_div(lanes, 256)), 256, 0, st>>>(
      T, ldt, n, nb, static_cast<unsigned char*>(pan3));
  return hipGetLastError();
}

hipError_t launch_set_identity(double* A, int64_t lda, int rows, int cols, hipStream_t st) {
  const int64_t tot = static_cast<int64_t>(rows) * cols;
  set_identity_kernel<<<static_cast<unsigned>(ceil_div(tot, 256)), 256, 0, st>>>(A, lda, rows, cols);
  return hipGetLastError();
}

// G(r, c) = sum_s gpart[s](r, c) for r <= c < n (ld npg), s ascending.
__global__ void gram_reduce_kernel(const double* __restrict__ gpart, int nsplit, int npg, int n,
                                   double* __restrict__ G) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int r = idx % n, c = idx / n;
  if (r > c) return;
  const int64_t stride = static_cast<int64_t>(npg) * npg;
  const double* p = gpart + r + static_cast<int64_t>(c) * npg;
  const double s = ordered_sum(p, nsplit, stride);
  G[r + c * npg] = s;
}

hipError_t launch_gram_reduce(const double* gpart, const GramPlan& gp, int n, double* G,
                              hipStream_t st) {
  gram_reduce_kernel<<<static_cast<unsigned>(ceil_div(n * n, 256)), 256, 0, st>>>(gpart, gp.nsplit,
                                                                                   gp.npg, n, G);
  return hipGetLastError();
}

// C(r, c) = sum_s gpart[s](r, c) for all r, c < n (ld npg).
__global__ void gram_reduce_full_kernel(const double* __restrict__ gpart, int nsplit, int npg, int n,
                                        double* __restrict__ G) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int r = idx % n, c = idx / n;
  const int64_t stride = static_cast<int64_t>(npg) * npg;
  const double* p = gpart + r + static_cast<int64_t>(c) * npg;
  const double s = ordered_sum(p, nsplit, stride);
  G[r + c * npg] = s;
}

hipError_t launch_gram_reduce_full(const double* gpart, const GramPlan& gp, int n, double* G,
                                   hipStream_t st) {
  gram_reduce_full_kernel<<<static_cast<unsigned>(ceil_div(n * n, 256)), 256, 0, st>>>(
      gpart, gp.nsplit, gp.npg, n, G);
  return hipGetLastError();
}

// Small step of the adjoint of the positive-diagonal thin QR X = Q R:
//   M = R dR^T - dQ^T Q (C = dQ^T Q given), N = copyltu(M) (the lower
//   triangle of M mirrored to the upper one), and Rrev = J R^T J, the upper
//   triangular matrix whose row-wise solve gives dX = Y R^{-T} on
//   column-reversed views.  All n x n, FP64.  dR may be null (zero).
__global__ void adjoint_small_kernel(const double* __restrict__ R, const double* __restrict__ dR,
                                     int64_t lddr, const double* __restrict__ C, int ldc, int n,
                                     double* __restrict__ Nm, double* __restrict__ Rrev) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int a = idx % n, b = idx / n;
  // N(a, b) = M(max, min)
  const int i = (a >= b) ? a : b, j = (a >= b) ? b : a;
  double s = 0.0;  // (R dR^T)(i, j) = sum_{l >= i} R(i, l) dR(j, l), dR(j, l) = 0 for l < j
  if (dR)
    for (int l = i; l < n; ++l) s += R[i + l * n] * dR[j + l * lddr];
  Nm[a + b * n] = s - C[i + j * ldc];
  // Rrev(a, b) = R(n-1-b, n-1-a)
  Rrev[a + b * n] = R[(n - 1 - b) + (n - 1 - a) * n];
}

hipError_t launch_adjoint_small(const double* R, const double* dR, int64_t lddr,
                                const double* C, int ldc, int n, double* Nm, double* Rrev,
                                hipStream_t st) {
  adjoint_small_kernel<<<static_cast<unsigned>(ceil_div(n * n, 256)), 256, 0, st>>>(
      R, dR, lddr, C, ldc, n, Nm, Rrev);
  return hipGetLastError();
}

// Dense panel packing: panel b holds all rows 0..16 NB - 1 of columns
// 16b..16b+15, row-major, zero-padded.
template <typename T>
__global__ void make_dense_panels_kernel(const double* __restrict__ B, int64_t ldb, int n,
                                         T* __restrict__ pan, int np) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = 16ll * np;
  if (idx >= per * (np / 16)) return;
  const int b = static_cast<int>(idx / per);
  const int64_t off = idx - per * b;
  const int r = static_cast<int>(off / 16), c = static_cast<int>(off % 16);
  const int col = 16 * b + c;
  pan[idx] = static_cast<T>((r < n && col < n) ? B[r + col * ldb] : 0.0);
}

hipError_t launch_make_dense_panels(const double* B, int64_t ldb, int n, bool f32, void* pan,
                                    hipStream_t st) {
  const int np = static_cast<int>(round_up(n, 16));
  const int64_t total = dense_panel_elems(n);
  const unsigned grid = static_cast<unsigned>(ceil_div(total, 256));
  if (f32)
    make_dense_panels_kernel<float><<<grid, 256, 0, st>>>(B, ldb, n, static_cast<float*>(pan), np);
  else
    make_dense_panels_kernel<double><<<grid, 256, 0, st>>>(B, ldb, n, static_cast<double*>(pan), np);
  return hipGetLastError();
}

}  // namespace rcq
