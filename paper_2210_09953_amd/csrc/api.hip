// api.hip -- the C ABI declared in include/rcholqr.h: argument checks,
// workspace layout, and the launch sequence of Algorithms 2 and 3.
//
// Launch sequence of rcholqr_factor (all on the caller's stream, no host
// synchronisation, no allocation):
//   sketch partials -> fixed-order reduction (x 1/sqrt(k))       P = Theta X
//   blocked Householder on P, sign fix, status word               R_s (, S)
//   panel packing of R_s, tall solve                              Q1 = X R_s^{-1}
//   passes = 2: Gram partials of Q1 -> reduction -> Cholesky (status)
//               -> R = R' R_s -> panel packing of R' -> solve in place
//                                                                 Q = Q1 R'^{-1}
#include <math.h>
#include <algorithm>
#include <mutex>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/rcholqr.h"
#include "common.h"
#include "kernels.h"

using namespace rcq;

namespace {

struct Layout {
  SketchPlan sp;
  GramPlan gp;
  size_t status, part, keys, P, v0, beta, T, Rs, pan, Tinv, gpart, G, total;
};

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// Sketch kinds of rcholqr_factor: the four embeddings, and Theta = I
// (test only; k = m, not with the mixed precision).
bool valid_kind(int kind) { return (kind >= 0 && kind <= 3) || kind == kIdentity; }

bool valid_dims(int64_t m, int64_t n, int64_t k) {
  return n >= 1 && n <= kMaxN && m >= n && k >= n && k <= kMaxK;
}

Layout make_layout(int64_t m, int64_t n, int64_t k, int kind, int passes, int prec) {
  Layout L{};
  SketchPlan& sp = L.sp;
  sp.npad = static_cast<int>(round_up(n, 16));
  if (kind == kIdentity) {
    // Theta = I: P is X itself, no partial sums.
    sp.nsplit = 0;
    sp.ktiles = 0;
    sp.kpad = static_cast<int>(k);
    sp.rows_per_split = m;
  } else if (kind == kSRHT) {
    // blocked fast transform (srht.hip), every precision
    srht_sketch_plan(m, static_cast<int>(k), static_cast<int>(n), sp);
  } else if (prec == kPrecMixed) {
    // int8 matrix-core sketch (mixed.hip) chooses its own tiles and splits.
    mixed_sketch_plan(m, static_cast<int>(k), static_cast<int>(n), sp);
  } else if (kind == kCountSketch) {
    const int panels = static_cast<int>(ceil_div(n, 8));
    const int64_t ntile = ceil_div(m, 256);
    int64_t ns = ceil_div(1024, panels);
    if (ns > ntile) ns = ntile;
    if (ns < 1) ns = 1;
    sp.rows_per_split = round_up(ceil_div(m, ns), 256);
    sp.nsplit = static_cast<int>(ceil_div(m, sp.rows_per_split));
    sp.ktiles = 0;
    sp.kpad = static_cast<int>(round_up(k, 16));
  } else {
    sp.ktiles = static_cast<int>(ceil_div(k, 64));
    sp.kpad = 64 * sp.ktiles;
    int64_t ns = ceil_div(1024, sp.ktiles);
    const int64_t maxs = ceil_div(m, 16);
    if (ns > maxs) ns = maxs;
    ns = round_up(ns < 8 ? 8 : ns, 8);
    sp.rows_per_split = round_up(ceil_div(m, ns), 16);
    sp.nsplit = static_cast<int>(ns);
  }
  GramPlan& gp = L.gp;
  gp.nbb = static_cast<int>(ceil_div(n, 64));
  gp.npg = 128 * static_cast<int>(ceil_div(n, 128));  // ld of the partials: whole 128-blocks
  if (prec == kPrecF64) {
    // Row splits for the FP64 Gram: a multiple of 8, at most 256.
    const int64_t maxs = round_up(ceil_div(m, 16), 8);
    const int64_t ns = maxs < 256 ? maxs : 256;
    gp.rows_per_split = round_up(ceil_div(m, ns), 16);
    gp.nsplit = static_cast<int>(ns);
  } else {
    // FP32 Gram on bf16 matrix cores: one workgroup per row split holds the
    // whole triangle; as many splits as workgroups fit on the 256 CUs at
    // once (fewer, waves per CU, for wider n), each of at least 256 rows.
    const int nb64 = static_cast<int>(ceil_div(n, 64));
    const int64_t per_cu = nb64 >= 3 ? 1 : (nb64 == 2 ? 2 : 6);
    int64_t ns = 256 * per_cu;
    const int64_t maxs = ceil_div(m, 256);
    if (ns > maxs) ns = maxs < 1 ? 1 : maxs;
    gp.rows_per_split = round_up(ceil_div(m, ns), 32);
    gp.nsplit = static_cast<int>(ceil_div(m, gp.rows_per_split));
  }

  const size_t esz = (prec == kPrecF64) ? sizeof(double) : sizeof(float);
  size_t off = 0;
  L.status = off; off += 256;
  L.part = off; off += align256(static_cast<size_t>(sp.nsplit) * sp.kpad * sp.npad * sizeof(double));
  L.keys = off;
  if (kind == kCountSketch) off += align256(static_cast<size_t>(round_up(m, 256)) * sizeof(uint32_t));
  L.P = off; off += align256(static_cast<size_t>(k) * n * sizeof(double));
  L.v0 = off; off += align256(static_cast<size_t>(n) * sizeof(double));
  L.beta = off; off += align256(static_cast<size_t>(n) * sizeof(double));
  L.T = off; off += align256(hh_t_bytes(static_cast<int>(n)));
  L.Rs = off; off += align256(static_cast<size_t>(n) * n * sizeof(double));
  (void)esz;
  {
    const int64_t pb = panel_elems(static_cast<int>(n)) * static_cast<int64_t>(sizeof(double));
    int64_t p3 = bf3_panel_bytes(static_cast<int>(n));
    // the solve's panels, the 1 KiB its staging may read past them, flags
    if (trsm_bf3_ws_bytes(static_cast<int>(n)) > p3) p3 = trsm_bf3_ws_bytes(static_cast<int>(n));
    L.pan = off; off += align256(static_cast<size_t>(pb > p3 ? pb : p3));
  }
  L.Tinv = off; off += align256(static_cast<size_t>(n) * n * sizeof(double));
  L.gpart = off;
  if (passes == 2) off += align256(static_cast<size_t>(gp.nsplit) * gp.npg * gp.npg * sizeof(double));
  L.G = off; off += align256(static_cast<size_t>(gp.npg) * gp.npg * sizeof(double));
  L.total = off;
  return L;
}

// Gram partials of the second rank-revealing pass: the largest over the
// possible ranks r = 1..n of the r-column plan.
size_t rr_second_gram_bytes(int64_t m, int64_t n, int prec) {
  size_t most = 0;
  for (int64_t r = 1; r <= n; ++r) {
    const GramPlan gp = make_layout(m, r, r, kGaussian, 2, prec).gp;
    const size_t b = align256(static_cast<size_t>(gp.nsplit) * gp.npg * gp.npg * sizeof(double));
    if (b > most) most = b;
  }
  return most;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

#define RCQ_TRY(expr)                              \
  do {                                             \
    if ((expr) != hipSuccess) return RCHOLQR_ERR_HIP; \
  } while (0)

// Phase-boundary events (see rcholqr_profile_enable).
constexpr int kRing = 256;
constexpr int kEv = RCHOLQR_NPHASES + 1;
struct Profiler {
  bool on = false;
  hipEvent_t ev[kRing][kEv];
  bool used[kRing][kEv];
  int head = 0, count = 0;
};
Profiler g_prof;

// Records boundary `b` of the current call (no-op when profiling is off).
void prof_mark(int b, hipStream_t st) {
  if (!g_prof.on) return;
  const int slot = g_prof.head;
  if (hipEventRecord(g_prof.ev[slot][b], st) == hipSuccess) g_prof.used[slot][b] = true;
}
void prof_begin(hipStream_t st) {
  if (!g_prof.on) return;
  for (int b = 0; b < kEv; ++b) g_prof.used[g_prof.head][b] = false;
  prof_mark(0, st);
}
void prof_end() {
  if (!g_prof.on) return;
  g_prof.head = (g_prof.head + 1) % kRing;
  if (g_prof.count < kRing) ++g_prof.count;
}

}  // namespace

extern "C" {

size_t rcholqr_workspace_bytes(int64_t m, int64_t n, int64_t k, int sketch_kind, int passes,
                               int precision) {
  if (!valid_dims(m, n, k) || !valid_kind(sketch_kind) || passes < 1 || passes > 2 ||
      precision < 0 || precision > 2)
    return 0;
  if (sketch_kind == kIdentity && (k != m || precision == kPrecMixed)) return 0;
  return make_layout(m, n, k, sketch_kind, passes, precision).total;
}

}  // extern "C"

namespace {

// Validation shared by the single and batched entry points (0 or -arg).
int check_factor_args(const void* X, int64_t m, int64_t n, int64_t ldx, int64_t k,
                      int sketch_kind, int passes, int precision, const void* Q, int64_t ldq,
                      const double* R, int64_t ldr, const double* S, int64_t lds) {
  if (!X) return -1;
  if (n < 1 || n > kMaxN) return -3;
  if (m < n) return -2;
  if (ldx < m) return -4;
  if (k < n || k > kMaxK) return -5;
  if (!valid_kind(sketch_kind)) return -7;
  if (sketch_kind == kIdentity && k != m) return -5;
  if (passes < 1 || passes > 2) return -8;
  if (precision < 0 || precision > 2) return -9;
  if (precision == kPrecMixed && sketch_kind != kRademacher && sketch_kind != kSRHT) return -9;
  if (!Q) return -10;
  if (ldq < m) return -11;
  if (!R) return -12;
  if (ldr < n) return -13;
  if (S && lds < k) return -15;
  return 0;
}

// The launch sequence of Algorithm 2 / 3 for one problem on one stream.
int factor_one(const void* X, int64_t m, int64_t n, int64_t ldx, int64_t k, uint64_t seed,
               int sketch_kind, int passes, int precision, void* Q, int64_t ldq, double* R,
               int64_t ldr, double* S, int64_t lds, double* Rs, double* Rp, void* ws,
               const Layout& L, hipStream_t st, bool profile) {
  const bool f32 = precision != kPrecF64;
  const int ni = static_cast<int>(n), ki = static_cast<int>(k);
  int* status = at<int>(ws, L.status);
  double* P = at<double>(ws, L.P);
  double* Rsw = at<double>(ws, L.Rs);
  void* pan = at<void>(ws, L.pan);
  if (profile) prof_begin(st);
  if (sketch_kind == kIdentity)
    RCQ_TRY(launch_sketch_identity(X, f32, m, ni, ldx, P, k, st));
  else if (precision == kPrecMixed)
    RCQ_TRY(launch_sketch_mixed(static_cast<const float*>(X), m, ni, ldx, ki, seed, L.sp,
                                at<double>(ws, L.part), P, k, st, sketch_kind));
  else
    RCQ_TRY(launch_sketch(X, f32, m, ni, ldx, ki, sketch_kind, seed, L.sp, at<double>(ws, L.part),
                          at<uint32_t>(ws, L.keys), P, k, st));
  if (profile) prof_mark(1, st);
  RCQ_TRY(launch_householder(P, ki, ni, at<double>(ws, L.v0), at<double>(ws, L.beta),
                             at<double>(ws, L.T), S, lds, Rsw, passes == 1 ? R : nullptr, ldr,
                             status, st));
  if (Rs) RCQ_TRY(launch_copy_upper(Rsw, n, Rs, n, ni, st));
  RCQ_TRY(launch_make_panels(Rsw, n, ni, f32, pan, st));
  if (profile) prof_mark(2, st);
  RCQ_TRY(launch_trsm(X, f32, m, ni, ldx, pan, Q, ldq, st));
  if (profile) prof_mark(3, st);
  if (passes == 1) {
    if (profile) prof_end();
    return 0;
  }
  double* G = at<double>(ws, L.G);
  RCQ_TRY(launch_gram(Q, f32, m, ni, ldq, L.gp, at<double>(ws, L.gpart), st));
  RCQ_TRY(launch_gram_reduce(at<double>(ws, L.gpart), L.gp, ni, G, st));
  if (profile) prof_mark(4, st);
  RCQ_TRY(launch_cholesky(G, ni, L.gp.npg, status, st));
  RCQ_TRY(launch_triu_product(G, L.gp.npg, Rsw, n, R, ldr, ni, st));
  if (Rp) RCQ_TRY(launch_copy_upper(G, L.gp.npg, Rp, n, ni, st));
  // T = R'^{-1} by the row-wise solve applied to the identity (FP64), then
  // the second solve as the triangular product Q = Q1 T in place.
  double* Tinv = at<double>(ws, L.Tinv);
  RCQ_TRY(launch_set_identity(Tinv, n, ni, ni, st));
  RCQ_TRY(launch_make_panels(G, L.gp.npg, ni, false, pan, st));
  RCQ_TRY(launch_trsm(Tinv, false, ni, ni, n, pan, Tinv, n, st));
  if (f32)
    RCQ_TRY(launch_make_bf3_panels(Tinv, n, ni, pan, st));
  else
    RCQ_TRY(launch_make_panels(Tinv, n, ni, false, pan, st, false));
  if (profile) prof_mark(5, st);
  RCQ_TRY(launch_trmm(Q, f32, m, ni, ldq, pan, st));
  if (profile) {
    prof_mark(6, st);
    prof_end();
  }
  return 0;
}

// Streams and fork/join events of the batched entry point, one set per
// device (created on the first call on that device, with it current;
// default priority, non-blocking; no device memory is allocated).  Creation
// is serialised; calls that use one device's pool from several host threads
// at once must be serialised by the caller (they share the fork/join events).
constexpr int kPool = 8;
constexpr int kPoolDevices = 64;
struct Pool {
  bool ready = false;
  hipStream_t s[kPool];
  hipEvent_t fork, join[kPool];
};
Pool g_pool[kPoolDevices];
std::mutex g_pool_mutex;

// The current device's pool (created if needed), or nullptr on failure.
Pool* ensure_pool() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kPoolDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_pool_mutex);
  Pool& p = g_pool[dev];
  if (p.ready) return &p;
  for (int i = 0; i < kPool; ++i) {
    if (hipStreamCreateWithFlags(&p.s[i], hipStreamNonBlocking) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&p.join[i], hipEventDisableTiming) != hipSuccess) return nullptr;
  }
  if (hipEventCreateWithFlags(&p.fork, hipEventDisableTiming) != hipSuccess) return nullptr;
  p.ready = true;
  return &p;
}

size_t batched_offset(const rcholqr_problem* probs, int i, int kind, int passes, int precision) {
  size_t off = 0;
  for (int j = 0; j < i; ++j)
    off += align256(make_layout(probs[j].m, probs[j].n, probs[j].k, kind, passes, precision).total);
  return off;
}

}  // namespace

namespace rcq {
// Plain 16-byte-vector device copy: the byte-count reference for HBM counters.
__global__ __launch_bounds__(256) void hbm_copy_kernel(const uint4* __restrict__ src,
                                                       uint4* __restrict__ dst, int64_t n16) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n16;
       i += stride)
    dst[i] = src[i];
}
}  // namespace rcq

extern "C" {

int rcholqr_factor(const void* X, int64_t m, int64_t n, int64_t ldx, int64_t k, uint64_t seed,
                   int sketch_kind, int passes, int precision, void* Q, int64_t ldq, double* R,
                   int64_t ldr, double* S, int64_t lds, double* Rs, double* Rp, void* ws,
                   size_t ws_bytes, void* stream) {
  const int bad = check_factor_args(X, m, n, ldx, k, sketch_kind, passes, precision, Q, ldq, R,
                                    ldr, S, lds);
  if (bad) return bad;
  if (!ws) return -18;
  const Layout L = make_layout(m, n, k, sketch_kind, passes, precision);
  if (ws_bytes < L.total) return -19;
  return factor_one(X, m, n, ldx, k, seed, sketch_kind, passes, precision, Q, ldq, R, ldr, S, lds,
                    Rs, Rp, ws, L, static_cast<hipStream_t>(stream), true);
}

size_t rcholqr_batched_workspace_bytes(const rcholqr_problem* probs, int batch, int sketch_kind,
                                       int passes, int precision) {
  if (!probs || batch < 1) return 0;
  for (int i = 0; i < batch; ++i)
    if (!valid_dims(probs[i].m, probs[i].n, probs[i].k)) return 0;
  if (sketch_kind < 0 || sketch_kind > 3 || passes < 1 || passes > 2 || precision < 0 ||
      precision > 2)
    return 0;
  return batched_offset(probs, batch, sketch_kind, passes, precision);
}

int rcholqr_factor_batched(const rcholqr_problem* probs, int batch, int sketch_kind, int passes,
                           int precision, void* ws, size_t ws_bytes, void* stream) {
  if (!probs) return -1;
  if (batch < 1) return -2;
  if (sketch_kind < 0 || sketch_kind > 3) return -3;
  if (passes < 1 || passes > 2) return -4;
  if (precision < 0 || precision > 2) return -5;
  for (int i = 0; i < batch; ++i) {
    const rcholqr_problem& p = probs[i];
    if (check_factor_args(p.X, p.m, p.n, p.ldx, p.k, sketch_kind, passes, precision, p.Q, p.ldq,
                          p.R, p.ldr, nullptr, 0) != 0)
      return RCHOLQR_ERR_BATCH_ENTRY - i;
  }
  if (!ws) return -6;
  if (ws_bytes < batched_offset(probs, batch, sketch_kind, passes, precision)) return -7;
  Pool* pool = ensure_pool();
  if (!pool) return RCHOLQR_ERR_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int used = batch < kPool ? batch : kPool;
  RCQ_TRY(hipEventRecord(pool->fork, st));
  for (int q = 0; q < used; ++q) RCQ_TRY(hipStreamWaitEvent(pool->s[q], pool->fork, 0));
  size_t off = 0;
  int rc = 0;
  for (int i = 0; i < batch && rc == 0; ++i) {
    const rcholqr_problem& p = probs[i];
    const Layout L = make_layout(p.m, p.n, p.k, sketch_kind, passes, precision);
    rc = factor_one(p.X, p.m, p.n, p.ldx, p.k, p.seed, sketch_kind, passes, precision, p.Q,
                    p.ldq, p.R, p.ldr, nullptr, 0, nullptr, nullptr,
                    static_cast<char*>(ws) + off, L, pool->s[i % kPool], false);
    off += align256(L.total);
  }
  // Join every forked stream even after a failed launch, so that a stream
  // capture in progress is left well formed.
  for (int q = 0; q < used; ++q) {
    RCQ_TRY(hipEventRecord(pool->join[q], pool->s[q]));
    RCQ_TRY(hipStreamWaitEvent(st, pool->join[q], 0));
  }
  return rc;
}

int rcholqr_batched_status(const rcholqr_problem* probs, int batch, int sketch_kind, int passes,
                           int precision, const void* ws, int* info) {
  if (!probs || batch < 1 || !ws || !info) return -1;
  if (hipDeviceSynchronize() != hipSuccess) return RCHOLQR_ERR_HIP;
  size_t off = 0;
  for (int i = 0; i < batch; ++i) {
    const Layout L = make_layout(probs[i].m, probs[i].n, probs[i].k, sketch_kind, passes, precision);
    if (hipMemcpy(&info[i], static_cast<const char*>(ws) + off + L.status, sizeof(int),
                  hipMemcpyDeviceToHost) != hipSuccess)
      return RCHOLQR_ERR_HIP;
    off += align256(L.total);
  }
  return 0;
}

namespace {
struct BwdLayout {
  GramPlan gp;
  size_t pan, Tinv, Rw, Nm, Rrev, Cm, gpart, total;
};
BwdLayout make_bwd_layout(int64_t m, int64_t n) {
  BwdLayout L{};
  L.gp = make_layout(m, n, n, kGaussian, 2, kPrecF64).gp;
  size_t off = 256;
  const int ni = static_cast<int>(n);
  int64_t pe = panel_elems(ni) > dense_panel_elems(ni) ? panel_elems(ni) : dense_panel_elems(ni);
  pe *= static_cast<int64_t>(sizeof(double));
  if (bf3_panel_bytes(ni) > pe) pe = bf3_panel_bytes(ni);
  if (trsm_bf3_ws_bytes(ni) > pe) pe = trsm_bf3_ws_bytes(ni);
  L.pan = off; off += align256(static_cast<size_t>(pe));
  L.Tinv = off; off += align256(static_cast<size_t>(n) * n * sizeof(double));
  L.Rw = off; off += align256(static_cast<size_t>(n) * n * sizeof(double));
  L.Nm = off; off += align256(static_cast<size_t>(n) * n * sizeof(double));
  L.Rrev = off; off += align256(static_cast<size_t>(n) * n * sizeof(double));
  L.Cm = off; off += align256(static_cast<size_t>(L.gp.npg) * L.gp.npg * sizeof(double));
  L.gpart = off; off += align256(static_cast<size_t>(L.gp.nsplit) * L.gp.npg * L.gp.npg * sizeof(double));
  L.total = off;
  return L;
}
}  // namespace

size_t rcholqr_backward_workspace_bytes(int64_t m, int64_t n, int precision) {
  if (n < 1 || n > kMaxN || m < n || precision < 0 || precision > 2) return 0;
  return make_bwd_layout(m, n).total;
}

int rcholqr_backward(const void* X, int64_t m, int64_t n, int64_t ldx, const double* Rs,
                     const double* Rp, const void* dQ, int64_t lddq, const double* dR,
                     int64_t lddr, int precision, void* dX, int64_t lddx, void* ws,
                     size_t ws_bytes, void* stream) {
  if (!X) return -1;
  if (n < 1 || n > kMaxN) return -3;
  if (m < n) return -2;
  if (ldx < m) return -4;
  if (!Rs) return -5;
  if (!Rp) return -6;
  if (!dQ) return -7;
  if (lddq < m) return -8;
  if (dR && lddr < n) return -10;
  if (precision < 0 || precision > 2) return -11;
  if (!dX) return -12;
  if (lddx < m) return -13;
  if (!ws) return -14;
  const BwdLayout L = make_bwd_layout(m, n);
  if (ws_bytes < L.total) return -15;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool f32 = precision != kPrecF64;
  const int ni = static_cast<int>(n);
  void* pan = at<void>(ws, L.pan);
  double* Tinv = at<double>(ws, L.Tinv);
  double* Rw = at<double>(ws, L.Rw);
  double* Nm = at<double>(ws, L.Nm);
  double* Rrev = at<double>(ws, L.Rrev);
  double* Cm = at<double>(ws, L.Cm);
  // Q recomputed into dX exactly as the forward pass formed it.
  RCQ_TRY(launch_make_panels(Rs, n, ni, f32, pan, st));
  RCQ_TRY(launch_trsm(X, f32, m, ni, ldx, pan, dX, lddx, st));
  RCQ_TRY(launch_set_identity(Tinv, n, ni, ni, st));
  RCQ_TRY(launch_make_panels(Rp, n, ni, false, pan, st));
  RCQ_TRY(launch_trsm(Tinv, false, ni, ni, n, pan, Tinv, n, st));
  if (f32)
    RCQ_TRY(launch_make_bf3_panels(Tinv, n, ni, pan, st));
  else
    RCQ_TRY(launch_make_panels(Tinv, n, ni, false, pan, st, false));
  RCQ_TRY(launch_trmm(dX, f32, m, ni, lddx, pan, st));
  // dQ^T Q, then M, N = copyltu(M) and J R^T J in FP64.
  RCQ_TRY(launch_triu_product(Rp, n, Rs, n, Rw, n, ni, st));
  RCQ_TRY(launch_cross_gram(dQ, dX, f32, m, ni, lddq, lddx, L.gp, at<double>(ws, L.gpart), st));
  RCQ_TRY(launch_gram_reduce_full(at<double>(ws, L.gpart), L.gp, ni, Cm, st));
  RCQ_TRY(launch_adjoint_small(Rw, dR, lddr, Cm, L.gp.npg, ni, Nm, Rrev, st));
  // Y = dQ + Q N (in place over Q).
  RCQ_TRY(launch_make_dense_panels(Nm, n, ni, f32, pan, st));
  RCQ_TRY(launch_gemm_add(dX, f32, m, ni, lddx, pan, dQ, lddq, st));
  // dX = Y R^{-T}: row-wise substitution with J R^T J on column-reversed views.
  RCQ_TRY(launch_make_panels(Rrev, n, ni, f32, pan, st));
  const size_t esz = f32 ? sizeof(float) : sizeof(double);
  void* dX_rev = static_cast<char*>(dX) + static_cast<size_t>(n - 1) * lddx * esz;
  RCQ_TRY(launch_trsm(dX_rev, f32, m, ni, -lddx, pan, dX_rev, -lddx, st));
  return 0;
}

int rcholqr_device_copy(const void* src, void* dst, size_t bytes, void* stream) {
  if (!src || (reinterpret_cast<uintptr_t>(src) & 15)) return -1;
  if (!dst || (reinterpret_cast<uintptr_t>(dst) & 15)) return -2;
  if (bytes & 15) return -3;
  const int64_t n16 = static_cast<int64_t>(bytes / 16);
  if (n16 == 0) return 0;
  const int blocks = static_cast<int>(std::min<int64_t>((n16 + 255) / 256, 8192));
  hbm_copy_kernel<<<blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(
      static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16);
  return hipGetLastError() == hipSuccess ? 0 : RCHOLQR_ERR_HIP;
}

int rcholqr_profile_enable(int on) {
  if (on && !g_prof.on) {
    for (int i = 0; i < kRing; ++i)
      for (int b = 0; b < kEv; ++b) {
        if (hipEventCreate(&g_prof.ev[i][b]) != hipSuccess) return RCHOLQR_ERR_HIP;
        g_prof.used[i][b] = false;
      }
    g_prof.on = true;
    g_prof.head = g_prof.count = 0;
  } else if (!on && g_prof.on) {
    for (int i = 0; i < kRing; ++i)
      for (int b = 0; b < kEv; ++b) (void)hipEventDestroy(g_prof.ev[i][b]);
    g_prof.on = false;
  }
  return 0;
}

int rcholqr_profile_read(double* ms) {
  if (!ms) return -1;
  for (int p = 0; p < RCHOLQR_NPHASES; ++p) ms[p] = 0.0;
  if (!g_prof.on) return 0;
  const int n = g_prof.count;
  for (int c = 0; c < n; ++c) {
    const int slot = (g_prof.head - 1 - c + kRing) % kRing;
    for (int p = 0; p < RCHOLQR_NPHASES; ++p) {
      if (!g_prof.used[slot][p] || !g_prof.used[slot][p + 1]) continue;
      if (hipEventSynchronize(g_prof.ev[slot][p + 1]) != hipSuccess) return RCHOLQR_ERR_HIP;
      float t = 0.f;
      if (hipEventElapsedTime(&t, g_prof.ev[slot][p], g_prof.ev[slot][p + 1]) != hipSuccess)
        return RCHOLQR_ERR_HIP;
      ms[p] += t;
    }
  }
  g_prof.count = 0;
  return n;
}

// Reduced RCholeskyQR: one (k + l)-row sketch pass, two fixed-order
// reductions (P with 1/sqrt(k), Y = L X with 1/sqrt(l) straight into Z),
// Householder on P, Z = Y R^{-1} in place by the FP64 row solve.
size_t rcholqr_reduced_workspace_bytes(int64_t m, int64_t n, int64_t k, int64_t l, int sketch_kind,
                                       int precision) {
  if (!valid_dims(m, n, k) || l < 1 || k + l > kMaxK || sketch_kind < 0 || sketch_kind > 1 ||
      precision < 0 || precision > 2)
    return 0;
  return make_layout(m, n, k + l, sketch_kind, 1, precision).total;
}

int rcholqr_reduced(const void* X, int64_t m, int64_t n, int64_t ldx, int64_t k, int64_t l,
                    uint64_t seed, int sketch_kind, int precision, double* Z, int64_t ldz,
                    double* R, int64_t ldr, double* S, int64_t lds, void* ws, size_t ws_bytes,
                    void* stream) {
  if (!X) return -1;
  if (n < 1 || n > kMaxN) return -3;
  if (m < n) return -2;
  if (ldx < m) return -4;
  if (k < n || k > kMaxK) return -5;
  if (l < 1 || k + l > kMaxK) return -6;
  if (sketch_kind != kGaussian && sketch_kind != kRademacher) return -8;
  if (precision < 0 || precision > 2) return -9;
  if (precision == kPrecMixed && sketch_kind != kRademacher && sketch_kind != kSRHT) return -9;
  if (!Z) return -10;
  if (ldz < l) return -11;
  if (!R) return -12;
  if (ldr < n) return -13;
  if (S && lds < k) return -15;
  if (!ws) return -16;
  const int64_t kl = k + l;
  const Layout L = make_layout(m, n, kl, sketch_kind, 1, precision);
  if (ws_bytes < L.total) return -17;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int ni = static_cast<int>(n), ki = static_cast<int>(k), li = static_cast<int>(l);
  double* part = at<double>(ws, L.part);
  double* P = at<double>(ws, L.P);  // room for (k + l) x n; P uses k x n, ld k
  if (precision == kPrecMixed)
    RCQ_TRY(launch_sketch_mixed_partials(static_cast<const float*>(X), m, ni, ldx,
                                         static_cast<int>(kl), seed, L.sp, part, st));
  else
    RCQ_TRY(launch_sketch_partials(X, precision != kPrecF64, m, ni, ldx, static_cast<int>(kl),
                                   sketch_kind, seed, L.sp, part, at<uint32_t>(ws, L.keys), st));
  RCQ_TRY(launch_sketch_reduce(part, L.sp, ki, ni, 1.0 / sqrt(static_cast<double>(k)), P, k, st));
  RCQ_TRY(launch_sketch_reduce(part + k, L.sp, li, ni, 1.0 / sqrt(static_cast<double>(l)), Z, ldz,
                               st));
  double* Rsw = at<double>(ws, L.Rs);
  RCQ_TRY(launch_householder(P, ki, ni, at<double>(ws, L.v0), at<double>(ws, L.beta),
                             at<double>(ws, L.T), S, lds, Rsw, R, ldr, at<int>(ws, L.status), st));
  void* pan = at<void>(ws, L.pan);
  RCQ_TRY(launch_make_panels(Rsw, n, ni, false, pan, st));
  RCQ_TRY(launch_trsm(Z, false, l, ni, ldz, pan, Z, ldz, st));
  return 0;
}

// Rank-revealing RCholeskyQR: sketch, column norms and P D^{-1},
// Householder of P D^{-1}, column-pivoted QR of its R, rank rule and the
// factors, gather X Pi into Q, tall solve in place.
size_t rcholqr_rr_workspace_bytes(int64_t m, int64_t n, int64_t k, int sketch_kind,
                                  int precision, int passes) {
  if (!valid_dims(m, n, k) || sketch_kind < 0 || sketch_kind > 3 || precision < 0 ||
      precision > 2 || passes < 1 || passes > 2)
    return 0;
  return align256(make_layout(m, n, k, sketch_kind, 1, precision).total) +
         align256(rr_extra_bytes(static_cast<int>(n))) +
         (passes == 2 ? rr_second_gram_bytes(m, n, precision) : 0);
}

int rcholqr_rr(const void* X, int64_t m, int64_t n, int64_t ldx, int64_t k, uint64_t seed,
               int sketch_kind, int precision, int passes, double tau, double f, void* Q,
               int64_t ldq, double* R, int64_t ldr, int* piv, int* rank, void* ws,
               size_t ws_bytes, void* stream) {
  if (!X) return -1;
  if (n < 1 || n > kMaxN) return -3;
  if (m < n) return -2;
  if (ldx < m) return -4;
  if (k < n || k > kMaxK) return -5;
  if (sketch_kind < 0 || sketch_kind > 3) return -7;
  if (precision < 0 || precision > 2) return -8;
  if (precision == kPrecMixed && sketch_kind != kRademacher && sketch_kind != kSRHT) return -8;
  if (passes < 1 || passes > 2) return -9;
  if (!(tau >= 0.0) || !isfinite(tau)) return -10;
  if (!(f == 0.0 || (f > 1.0 && isfinite(f)))) return -11;
  if (!Q) return -12;
  if (ldq < m) return -13;
  if (!R) return -14;
  if (ldr < n) return -15;
  if (!piv) return -16;
  if (!rank) return -17;
  if (!ws) return -18;
  const Layout L = make_layout(m, n, k, sketch_kind, 1, precision);
  const size_t extra_off = align256(L.total);
  const size_t gram_off = extra_off + align256(rr_extra_bytes(static_cast<int>(n)));
  if (ws_bytes < gram_off + (passes == 2 ? rr_second_gram_bytes(m, n, precision) : 0)) return -19;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool f32 = precision != kPrecF64;
  const int ni = static_cast<int>(n), ki = static_cast<int>(k);
  double* P = at<double>(ws, L.P);
  unsigned char* extra = at<unsigned char>(ws, extra_off);
  int* status = at<int>(ws, L.status);
  if (precision == kPrecMixed)
    RCQ_TRY(launch_sketch_mixed(static_cast<const float*>(X), m, ni, ldx, ki, seed, L.sp,
                                at<double>(ws, L.part), P, k, st, sketch_kind));
  else
    RCQ_TRY(launch_sketch(X, f32, m, ni, ldx, ki, sketch_kind, seed, L.sp, at<double>(ws, L.part),
                          at<uint32_t>(ws, L.keys), P, k, st));
  double* Rsolve = nullptr;
  RCQ_TRY(launch_rr_steps(X, f32, m, ni, ldx, P, ki, nullptr, tau, f, extra, R, ldr, piv, rank,
                          status, &Rsolve, st, 0));
  double* Rsw = at<double>(ws, L.Rs);
  RCQ_TRY(launch_householder(P, ki, ni, at<double>(ws, L.v0), at<double>(ws, L.beta),
                             at<double>(ws, L.T), nullptr, k, Rsw, nullptr, ldr, status, st));
  RCQ_TRY(launch_rr_steps(X, f32, m, ni, ldx, P, ki, Rsw, tau, f, extra, R, ldr, piv, rank,
                          status, &Rsolve, st, 1));
  // r is read back (the call's one synchronisation) so that step 4 touches
  // only the r kept columns: X Pi_{:,1:r} gathered into Q, solved in place
  // with the leading r x r block of the solve's factor (about m r^2 work).
  int r = 0;
  RCQ_TRY(hipMemcpyAsync(&r, rank, sizeof(int), hipMemcpyDeviceToHost, st));
  RCQ_TRY(hipStreamSynchronize(st));
  if (r < 1 || r > ni) return 0;
  RCQ_TRY(launch_gather_cols(X, f32, m, r, ldx, piv, Q, ldq, st));
  void* pan = at<void>(ws, L.pan);
  RCQ_TRY(launch_make_panels(Rsolve, n, r, f32, pan, st));
  RCQ_TRY(launch_trsm(Q, f32, m, r, ldq, pan, Q, ldq, st));
  if (passes == 1) return 0;
  // RRRCholeskyQR2: one Cholesky QR pass (Algorithm 3 steps 2-4) over the r
  // kept columns of Q.
  const GramPlan gp = make_layout(m, r, r, kGaussian, 2, precision).gp;
  double* G = at<double>(ws, L.G);
  RCQ_TRY(launch_gram(Q, f32, m, r, ldq, gp, at<double>(ws, gram_off), st));
  RCQ_TRY(launch_gram_reduce(at<double>(ws, gram_off), gp, r, G, st));
  RCQ_TRY(launch_cholesky(G, r, gp.npg, status, st));
  RCQ_TRY(launch_left_upper(G, gp.npg, r, R, ldr, ni, st));
  double* Tinv = at<double>(ws, L.Tinv);
  RCQ_TRY(launch_set_identity(Tinv, r, r, r, st));
  RCQ_TRY(launch_make_panels(G, gp.npg, r, false, pan, st));
  RCQ_TRY(launch_trsm(Tinv, false, r, r, r, pan, Tinv, r, st));
  if (f32)
    RCQ_TRY(launch_make_bf3_panels(Tinv, r, r, pan, st));
  else
    RCQ_TRY(launch_make_panels(Tinv, r, r, false, pan, st, false));
  RCQ_TRY(launch_trmm(Q, f32, m, r, ldq, pan, st));
  return 0;
}

size_t rcholqr_col_block_workspace_bytes(int64_t m, int64_t j0, int64_t b, int64_t k,
                                         int sketch_kind, int precision) {
  const int64_t nt = j0 + b;
  if (j0 < 0 || b < 1 || !valid_dims(m, nt, k) || sketch_kind < 0 || sketch_kind > 3 ||
      precision < 0 || precision > 2)
    return 0;
  const Layout Lb = make_layout(m, b, k, sketch_kind, 1, precision);
  const Layout Ln = make_layout(m, nt, k, sketch_kind, 1, precision);
  return align256(Lb.total) + align256(static_cast<size_t>(nt) * nt * sizeof(double)) +
         (Ln.Tinv - Ln.pan);
}

int rcholqr_col_block(const void* Xb, int64_t m, int64_t j0, int64_t b, int64_t ldx, int64_t k,
                      uint64_t seed, int sketch_kind, int precision, void* Q, int64_t ldq,
                      double* S, int64_t lds, double* R, int64_t ldr, void* ws,
                      size_t ws_bytes, void* stream) {
  const int64_t nt = j0 + b;
  if (!Xb) return -1;
  if (j0 < 0) return -3;
  if (b < 1 || nt > kMaxN) return -4;
  if (m < nt) return -2;
  if (ldx < m) return -5;
  if (k < nt || k > kMaxK) return -6;
  if (sketch_kind < 0 || sketch_kind > 3) return -8;
  if (precision < 0 || precision > 2) return -9;
  if (precision == kPrecMixed && sketch_kind != kRademacher && sketch_kind != kSRHT) return -9;
  if (!Q) return -10;
  if (ldq < m) return -11;
  if (!S) return -12;
  if (lds < k) return -13;
  if (!R) return -14;
  if (ldr < nt) return -15;
  if (!ws) return -16;
  if (ws_bytes < rcholqr_col_block_workspace_bytes(m, j0, b, k, sketch_kind, precision))
    return -17;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool f32 = precision != kPrecF64;
  const size_t esz = f32 ? sizeof(float) : sizeof(double);
  const int bi = static_cast<int>(b), ji = static_cast<int>(j0), ni = static_cast<int>(nt);
  const int ki = static_cast<int>(k);
  const Layout Lb = make_layout(m, b, k, sketch_kind, 1, precision);
  double* P = at<double>(ws, Lb.P);
  double* T = at<double>(ws, align256(Lb.total));
  void* pan = at<void>(ws, align256(Lb.total) + align256(static_cast<size_t>(nt) * nt * sizeof(double)));
  int* status = at<int>(ws, Lb.status);
  // step 2: P_b = Theta X_b (the same Theta as for the whole X)
  if (precision == kPrecMixed)
    RCQ_TRY(launch_sketch_mixed(static_cast<const float*>(Xb), m, bi, ldx, ki, seed, Lb.sp,
                                at<double>(ws, Lb.part), P, k, st, sketch_kind));
  else
    RCQ_TRY(launch_sketch(Xb, f32, m, bi, ldx, ki, sketch_kind, seed, Lb.sp,
                          at<double>(ws, Lb.part), at<uint32_t>(ws, Lb.keys), P, k, st));
  // steps 3-4: coefficients on the previous S, then the QR of the remainder
  RCQ_TRY(launch_col_project(S, lds, ji, P, ki, bi, R, ldr, st));
  RCQ_TRY(launch_householder(P, ki, bi, at<double>(ws, Lb.v0), at<double>(ws, Lb.beta),
                             at<double>(ws, Lb.T), S + j0 * lds, lds, at<double>(ws, Lb.Rs),
                             R + j0 + j0 * ldr, ldr, status, st));
  // step 5: Q_b = (X_b - Q_{1:j0} R_{1:j0,b}) R_bb^{-1}, Q_{1:j0} read and
  // never rewritten: one pass of the tall solve over [Q_{1:j0}, X_b] with T
  // (the identity on columns 0..j0-1, R's columns after) that takes its
  // leading 16 s0 columns as solved.  A j0 that is not a multiple of 16
  // shares a 16-column subpanel with X_b: X_b is copied into Q first and that
  // subpanel solved in place (its old columns meet the identity, which
  // reproduces them).
  char* qb = static_cast<char*>(Q) + static_cast<size_t>(j0) * ldq * esz;
  const int s0 = ji / 16;
  const void* xs = Xb;
  int64_t ldxs = ldx;
  if (ji % 16 != 0 || static_cast<const void*>(qb) == Xb) {
    if (static_cast<const void*>(qb) != Xb)
      RCQ_TRY(hipMemcpy2DAsync(qb, ldq * esz, Xb, ldx * esz, m * esz, b, hipMemcpyDeviceToDevice,
                               st));
    xs = static_cast<const char*>(Q) + static_cast<size_t>(16 * s0) * ldq * esz;
    ldxs = ldq;
  }
  RCQ_TRY(launch_col_make_t(R, ldr, ji, ni, T, st));
  RCQ_TRY(launch_make_panels(T, nt, ni, f32, pan, st));
  RCQ_TRY(launch_trsm_append(xs, f32, m, ni, ldxs, pan, Q, ldq, s0, st));
  return 0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// rcholqr_factor_noalloc: rcholqr_factor with its workspace in a
// library-owned device array.  `scratch` names a host-side stand-in in host
// code; the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// only that address is ever passed to kernels.
namespace {
constexpr size_t kScratchBytes = size_t{256} << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
struct ScratchSlot {
  std::once_flag once;
  void* ptr = nullptr;
  hipError_t err = hipSuccess;
};
ScratchSlot g_scratch[kMaxDevices];

// The current device's scratch address (resolved on its first use there).
int scratch_of_current_device(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return RCHOLQR_ERR_HIP;
  ScratchSlot& sl = g_scratch[dev];
  std::call_once(sl.once, [&sl]() {
    void* p = nullptr;
    sl.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (sl.err == hipSuccess) sl.ptr = p;
  });
  if (sl.err != hipSuccess || sl.ptr == nullptr) return RCHOLQR_ERR_HIP;
  *out = sl.ptr;
  return 0;
}
}  // namespace

extern "C" {

size_t rcholqr_noalloc_max_bytes(void) { return kScratchBytes; }

int rcholqr_factor_noalloc(const void* X, int64_t m, int64_t n, int64_t ldx, int64_t k,
                           uint64_t seed, int sketch_kind, int passes, int precision, void* Q,
                           int64_t ldq, double* R, int64_t ldr, void* stream) {
  const int bad = check_factor_args(X, m, n, ldx, k, sketch_kind, passes, precision, Q, ldq, R,
                                    ldr, nullptr, 0);
  if (bad) return bad;
  const Layout L = make_layout(m, n, k, sketch_kind, passes, precision);
  if (L.total > kScratchBytes) return RCHOLQR_ERR_NOALLOC_SIZE;
  void* ws = nullptr;
  const int rc = scratch_of_current_device(&ws);
  if (rc != 0) return rc;
  return factor_one(X, m, n, ldx, k, seed, sketch_kind, passes, precision, Q, ldq, R, ldr, nullptr,
                    0, nullptr, nullptr, ws, L, static_cast<hipStream_t>(stream), true);
}

int rcholqr_noalloc_status(int* info) {
  if (!info) return -1;
  void* ws = nullptr;
  const int rc = scratch_of_current_device(&ws);
  if (rc != 0) return rc;
  if (hipDeviceSynchronize() != hipSuccess) return RCHOLQR_ERR_HIP;
  if (hipMemcpy(info, ws, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return RCHOLQR_ERR_HIP;
  return 0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Persistent batched engine: host entry points and the chunk-size tuning.
namespace {
// Rows per tall task by the batch's largest n (16, 32, ..., 128).
constexpr int64_t kChunkDefault = 8192;
// Bound of one dependency wait in the engine: 2 s of the 100 MHz clock.
constexpr long long kWaitTicks = 200000000ll;
constexpr int64_t kChunkCandidates[] = {1024, 2048, 4096, 8192, 16384};
int64_t g_chunk[9] = {kChunkDefault, kChunkDefault, kChunkDefault, kChunkDefault, kChunkDefault,
                      kChunkDefault, kChunkDefault, kChunkDefault, kChunkDefault};
std::mutex g_chunk_mutex;

int chunk_slot(int64_t max_n) {
  const int64_t s = (max_n + 15) / 16;
  return static_cast<int>(s < 1 ? 1 : (s > 8 ? 8 : s));
}

bool valid_chunk(int64_t c) { return c > 0 && c % 128 == 0 && c <= (int64_t{1} << 24); }

int write_chunk_table(const char* path) {
  FILE* f = fopen(path, "w");
  if (!f) return -1;
  fprintf(f, "{\"batched_engine_chunk_rows\": {");
  for (int s = 1; s <= 8; ++s)
    fprintf(f, "%s\"%d\": %lld", s > 1 ? ", " : "", 16 * s, static_cast<long long>(g_chunk[s]));
  fprintf(f, "}}\n");
  return fclose(f) == 0 ? 0 : -1;
}
}  // namespace

extern "C" {

int rcholqr_init(const char* tune_path) {
  std::lock_guard<std::mutex> lock(g_chunk_mutex);
  for (int s = 0; s <= 8; ++s) g_chunk[s] = kChunkDefault;
  if (!tune_path) return 0;
  FILE* f = fopen(tune_path, "r");
  if (!f) return -1;
  char buf[4096];
  const size_t len = fread(buf, 1, sizeof(buf) - 1, f);
  fclose(f);
  buf[len] = 0;
  const char* p = strstr(buf, "\"batched_engine_chunk_rows\"");
  if (!p) return -1;
  p = strchr(p, '{');
  if (!p) return -1;
  // entries "<n>": rows, up to the closing brace
  int read = 0;
  while (*p && *p != '}') {
    const char* q = strchr(p, '"');
    if (!q) break;
    const long nval = strtol(q + 1, nullptr, 10);
    const char* colon = strchr(q + 1, ':');
    if (!colon) return -1;
    char* end = nullptr;
    const long long rows = strtoll(colon + 1, &end, 10);
    if (end == colon + 1 || nval < 16 || nval > 128 || nval % 16 != 0 || !valid_chunk(rows))
      return -1;
    g_chunk[nval / 16] = rows;
    ++read;
    p = end;
    while (*p == ' ' || *p == ',' || *p == '\n') ++p;
  }
  return read > 0 ? 0 : -1;
}

int64_t rcholqr_batched_engine_chunk(int64_t max_n) {
  std::lock_guard<std::mutex> lock(g_chunk_mutex);
  return g_chunk[chunk_slot(max_n)];
}

size_t rcholqr_batched_engine_workspace_bytes(const rcholqr_problem* probs_host, int batch,
                                              int passes, int64_t chunk_rows) {
  if (!probs_host || batch < 1 || passes < 1 || passes > 2) return 0;
  if (chunk_rows == 0) {
    int64_t mx = 16;
    for (int i = 0; i < batch; ++i) mx = std::max<int64_t>(mx, probs_host[i].n);
    chunk_rows = rcholqr_batched_engine_chunk(mx);
  }
  if (!valid_chunk(chunk_rows)) return 0;
  return static_cast<size_t>(batched_engine_bytes(probs_host, batch, passes, chunk_rows));
}

int rcholqr_factor_batched_engine(const rcholqr_problem* probs_dev, int batch, int sketch_kind,
                                  int passes, int64_t chunk_rows, void* ws, size_t ws_bytes,
                                  void* stream) {
  if (!probs_dev) return -1;
  if (batch < 1) return -2;
  if (sketch_kind != kRademacher) return -3;
  if (passes < 1 || passes > 2) return -4;
  if (chunk_rows != 0 && !valid_chunk(chunk_rows)) return -5;
  if (!ws) return -6;
  if (ws_bytes < static_cast<size_t>(batched_engine_status_offset(batch))) return -7;
  // chunk_rows = 0 needs the batch's largest n, which lives on the device:
  // the default table entry for n = 128 is used (the caller passes the
  // value it sized the workspace with, as rcholqr_batched_engine_chunk gives)
  if (chunk_rows == 0) chunk_rows = rcholqr_batched_engine_chunk(128);
  RCQ_TRY(launch_batched_engine(probs_dev, batch, passes, chunk_rows, ws,
                                static_cast<int64_t>(ws_bytes), batched_engine_grid(),
                                kWaitTicks, static_cast<hipStream_t>(stream)));
  return 0;
}

int rcholqr_batched_engine_status(int batch, const void* ws, int* info) {
  if (batch < 1 || !ws || !info) return -1;
  if (hipDeviceSynchronize() != hipSuccess) return RCHOLQR_ERR_HIP;
  int hdr[2] = {0, 0};
  if (hipMemcpy(hdr, ws, sizeof(hdr), hipMemcpyDeviceToHost) != hipSuccess) return RCHOLQR_ERR_HIP;
  if (hdr[1] & 1) {
    int stall[4] = {0, 0, 0, 0};
    if (hipMemcpy(stall, static_cast<const char*>(ws) + batched_engine_stall_offset(), sizeof(stall),
                  hipMemcpyDeviceToHost) == hipSuccess)
      fprintf(stderr,
              "rcholqr batched engine: a wait exceeded its bound (instance %d, phase %d, "
              "%d of %d tasks of the previous phase counted)\n",
              stall[0], stall[1], stall[2], stall[3]);
  }
  if (hipMemcpy(info, static_cast<const char*>(ws) + batched_engine_status_offset(batch),
                sizeof(int) * batch, hipMemcpyDeviceToHost) != hipSuccess)
    return RCHOLQR_ERR_HIP;
  return (hdr[1] & 1) ? RCHOLQR_ERR_ENGINE : 0;
}

int rcholqr_batched_engine_tune(const rcholqr_problem* probs_host, const rcholqr_problem* probs_dev,
                                int batch, int sketch_kind, int passes, void* ws, size_t ws_bytes,
                                const char* save_path, void* stream) {
  if (!probs_host) return -1;
  if (!probs_dev) return -2;
  if (batch < 1) return -3;
  if (sketch_kind != kRademacher) return -4;
  if (passes < 1 || passes > 2) return -5;
  if (!ws) return -6;
  int64_t mx = 16;
  for (int i = 0; i < batch; ++i) mx = std::max<int64_t>(mx, probs_host[i].n);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  RCQ_TRY(hipEventCreate(&e0));
  RCQ_TRY(hipEventCreate(&e1));
  float best_ms = 1e30f;
  int64_t best = -1;
  for (const int64_t c : kChunkCandidates) {
    if (static_cast<size_t>(batched_engine_bytes(probs_host, batch, passes, c)) > ws_bytes) continue;
    float ms_sum = 0.f;
    bool ok = true;
    for (int rep = 0; rep < 3 && ok; ++rep) {
      ok = launch_batched_engine(probs_dev, batch, passes, c, ws, static_cast<int64_t>(ws_bytes),
                                 batched_engine_grid(), kWaitTicks, st) == hipSuccess;  // warm
      ok = ok && hipEventRecord(e0, st) == hipSuccess;
      ok = ok && launch_batched_engine(probs_dev, batch, passes, c, ws, static_cast<int64_t>(ws_bytes),
                                       batched_engine_grid(), kWaitTicks, st) == hipSuccess;
      ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
      float ms = 0.f;
      ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
      ms_sum += ms;
    }
    if (ok && ms_sum < best_ms) {
      best_ms = ms_sum;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best < 0) return -7;
  {
    std::lock_guard<std::mutex> lock(g_chunk_mutex);
    g_chunk[chunk_slot(mx)] = best;
    if (save_path && write_chunk_table(save_path) != 0) return -1;
  }
  return 0;
}

int rcholqr_status(const void* ws, int* info) {
  if (!ws || !info) return -1;
  if (hipDeviceSynchronize() != hipSuccess) return RCHOLQR_ERR_HIP;
  if (hipMemcpy(info, ws, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return RCHOLQR_ERR_HIP;
  return 0;
}

int rcholqr_sketch(const void* X, int64_t m, int64_t n, int64_t ldx, int64_t k, uint64_t seed,
                   int sketch_kind, int precision, double* P, int64_t ldp, void* ws,
                   size_t ws_bytes, void* stream) {
  if (!X) return -1;
  if (n < 1 || n > kMaxN) return -3;
  if (m < n) return -2;
  if (ldx < m) return -4;
  if (k < n || k > kMaxK) return -5;
  if (sketch_kind < 0 || sketch_kind > 3) return -7;
  if (precision < 0 || precision > 2) return -8;
  if (precision == kPrecMixed && sketch_kind != kRademacher && sketch_kind != kSRHT) return -8;
  if (!P) return -9;
  if (ldp < k) return -10;
  if (!ws) return -11;
  const Layout L = make_layout(m, n, k, sketch_kind, 1, precision);
  if (ws_bytes < L.total) return -12;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (precision == kPrecMixed)
    RCQ_TRY(launch_sketch_mixed(static_cast<const float*>(X), m, static_cast<int>(n), ldx,
                                static_cast<int>(k), seed, L.sp, at<double>(ws, L.part), P, ldp, st,
                                sketch_kind));
  else
    RCQ_TRY(launch_sketch(X, precision != kPrecF64, m, static_cast<int>(n), ldx, static_cast<int>(k),
                          sketch_kind, seed, L.sp, at<double>(ws, L.part), at<uint32_t>(ws, L.keys),
                          P, ldp, st));
  return 0;
}

int rcholqr_debug_theta(int sketch_kind, int64_t k, int64_t m, uint64_t seed, int64_t i0,
                        int64_t ni, int64_t j0, int64_t nj, double* out, void* stream) {
  if (sketch_kind < 0 || sketch_kind > 3) return -1;
  if (k < 1 || k > kMaxK) return -2;
  if (m < 1) return -3;
  if (i0 < 0 || ni < 0 || i0 + ni > k) return -5;
  if (j0 < 0 || nj < 0) return -8;
  if (ni * nj > (int64_t(1) << 26)) return -7;
  if (!out && ni * nj > 0) return -9;
  RCQ_TRY(launch_theta_debug(sketch_kind, static_cast<int>(k), m, seed, i0, ni, j0, nj, out,
                             static_cast<hipStream_t>(stream)));
  return 0;
}

int rcholqr_trsm(const void* X, int64_t m, int64_t n, int64_t ldx, const double* R, int64_t ldr,
                 int precision, void* Q, int64_t ldq, void* ws, size_t ws_bytes, void* stream) {
  if (!X) return -1;
  if (n < 1 || n > kMaxN) return -3;
  if (m < n) return -2;
  if (ldx < m) return -4;
  if (!R) return -5;
  if (ldr < n) return -6;
  if (precision < 0 || precision > 2) return -7;
  if (!Q) return -8;
  if (ldq < m) return -9;
  if (!ws) return -10;
  const Layout L = make_layout(m, n, n, kGaussian, 2, precision);
  if (ws_bytes < L.total) return -11;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool f32 = precision != kPrecF64;
  void* pan = at<void>(ws, L.pan);
  RCQ_TRY(launch_make_panels(R, ldr, static_cast<int>(n), f32, pan, st));
  RCQ_TRY(launch_trsm(X, f32, m, static_cast<int>(n), ldx, pan, Q, ldq, st));
  return 0;
}

const char* rcholqr_error_string(int code) {
  if (code == 0) return "success";
  if (code == RCHOLQR_ERR_HIP) return "HIP launch or runtime error";
  if (code == RCHOLQR_ERR_ENGINE) return "batched engine stopped on a bounded wait (a task's dependency never completed)";
  if (code == RCHOLQR_BATCH_INVALID) return "batched engine refused the problem (n, k, m or leading dimensions outside its rules, or a workspace that is too small)";
  if (code == RCHOLQR_ERR_NOALLOC_SIZE)
    return "problem needs more workspace than the no-allocation entry point holds";
  if (code < 0) return "invalid argument (the -code-th argument, 1-based)";
  if (code == RCHOLQR_SKETCH_RANK) return "zero diagonal in the sketch R (rank-deficient X or failed embedding)";
  if (code == RCHOLQR_NONFINITE) return "non-finite value in X";
  if (code >= RCHOLQR_CHOL_BREAKDOWN) return "Cholesky breakdown of Q^T Q (status - 1000 = column)";
  return "unknown code";
}

}  // extern "C"
