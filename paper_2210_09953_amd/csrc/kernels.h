// kernels.h -- internal launch interface between the C-ABI driver and the
// kernel translation units.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

struct rcholqr_problem;  // include/rcholqr.h

namespace rcq {

constexpr int kGaussian = 0;
constexpr int kRademacher = 1;
constexpr int kCountSketch = 2;
constexpr int kSRHT = 3;
// Test-only embedding Theta = I (k = m): the sketch is X itself.
constexpr int kIdentity = 99;

constexpr int kPrecF64 = 0;
constexpr int kPrecF32 = 1;
constexpr int kPrecMixed = 2;

constexpr int kMaxN = 256;
constexpr int kMaxK = 1024;
constexpr int kHhPanel = 16;  // Householder panel width

// Split-K plan of the sketch.
struct SketchPlan {
  int nsplit;              // row ranges (multiple of 8 for the dense kernels)
  int ktiles;              // 64-row tiles of Theta (dense kernels)
  int kpad;                // padded k of the partials
  int npad;                // padded n of the partials
  int64_t rows_per_split;  // rows of X per range
};

struct GramPlan {
  int nsplit;
  int nbb;                 // 64-column blocks
  int npg;                 // 64 * nbb
  int64_t rows_per_split;
};

// sketch.hip
hipError_t launch_theta_debug(int kind, int k, int64_t m, uint64_t seed, int64_t i0, int64_t ni,
                              int64_t j0, int64_t nj, double* out, hipStream_t st);
hipError_t launch_sketch(const void* X, bool x_is_f32, int64_t m, int n, int64_t ldx, int k,
                         int kind, uint64_t seed, const SketchPlan& pl, double* part,
                         uint32_t* keys, double* P, int64_t ldp, hipStream_t st);
// Theta = I: P = X promoted to FP64 (k = m rows).
hipError_t launch_sketch_identity(const void* X, bool x_is_f32, int64_t m, int n, int64_t ldx,
                                  double* P, int64_t ldp, hipStream_t st);
hipError_t launch_sketch_reduce(const double* part, const SketchPlan& pl, int k, int n,
                                double scale, double* P, int64_t ldp, hipStream_t st);
// The split partials of the sketch without the reduction (rows 0..k-1 of
// each split's partial, layout as in launch_sketch_reduce).
hipError_t launch_sketch_partials(const void* X, bool x_is_f32, int64_t m, int n, int64_t ldx,
                                  int k, int kind, uint64_t seed, const SketchPlan& pl,
                                  double* part, uint32_t* keys, hipStream_t st);
void mixed_sketch_plan(int64_t m, int k, int n, SketchPlan& sp);
// srht.hip: the SRHT sketch's partials by blocked fast Walsh-Hadamard
// transforms (X FP32 or FP64), and its plan.
void srht_sketch_plan(int64_t m, int k, int n, SketchPlan& sp);
hipError_t launch_sketch_srht_partials(const void* X, bool x_is_f32, int64_t m, int n,
                                       int64_t ldx, int k, uint64_t seed, const SketchPlan& pl,
                                       double* part, hipStream_t st);
// kind: kRademacher (int8 matrix cores) or kSRHT (the blocked fast transform).
hipError_t launch_sketch_mixed(const float* X, int64_t m, int n, int64_t ldx, int k, uint64_t seed,
                               const SketchPlan& pl, double* part, double* P, int64_t ldp,
                               hipStream_t st, int kind = kRademacher);
hipError_t launch_sketch_mixed_partials(const float* X, int64_t m, int n, int64_t ldx, int k,
                                        uint64_t seed, const SketchPlan& pl, double* part,
                                        hipStream_t st, int kind = kRademacher);

// rr.hip (rank-revealing variant).  stage 0: column norms d of X and P <-
// P D^{-1} (P k x n, ld k); stage 1: column-pivoted QR of Rp (n x n), rank,
// the strong RRQR swaps with parameter f (none for f = 0), R (ld ldr), piv,
// rank, status, and *Rs_out = the solve's n x n factor.
size_t rr_extra_bytes(int n);
hipError_t launch_rr_steps(const void* X, bool f32, int64_t m, int n, int64_t ldx, double* P,
                           int k, const double* Rp, double tau, double f, unsigned char* extra,
                           double* R, int64_t ldr, int* piv_out, int* rank_out, int* status,
                           double** Rs_out, hipStream_t st, int stage);
// R(0:r, 0:n) <- U R(0:r, 0:n), U upper triangular r x r (second pass).
hipError_t launch_left_upper(const double* U, int64_t ldu, int r, double* R, int64_t ldr, int n,
                             hipStream_t st);
hipError_t launch_gather_cols(const void* X, bool f32, int64_t m, int n, int64_t ldx,
                              const int* piv, void* Q, int64_t ldq, hipStream_t st);

// col.hip (column-oriented variant): R(0:j0, j0:j0+b) = S(:, 0:j0)^T P and
// P <- P - S(:, 0:j0) R(0:j0, j0:j0+b) (P k x b, ld k); T (nt x nt) for the
// tall step.
hipError_t launch_col_project(const double* S, int64_t lds, int j0, double* P, int k, int b,
                              double* R, int64_t ldr, hipStream_t st);
hipError_t launch_col_make_t(const double* R, int64_t ldr, int j0, int nt, double* T,
                             hipStream_t st);

// small.hip
// Bytes of the T argument of launch_householder: the panels' 16 x 16 T
// blocks and the n column exponents of its column scaling.
inline size_t hh_t_bytes(int n) {
  return static_cast<size_t>((n + kHhPanel - 1) / kHhPanel) * kHhPanel * kHhPanel * sizeof(double) +
         static_cast<size_t>(n) * sizeof(int);
}
hipError_t launch_householder(double* A, int k, int n, double* V, double* beta, double* T,
                              double* S, int64_t lds, double* Rs, double* R, int64_t ldr,
                              int* status, hipStream_t st);
hipError_t launch_cholesky(double* G, int n, int ldg, int* status, hipStream_t st);
hipError_t launch_triu_product(const double* A, int64_t lda, const double* B, int64_t ldb,
                               double* C, int64_t ldc, int n, hipStream_t st);
hipError_t launch_copy_upper(const double* A, int64_t lda, double* B, int64_t ldb, int n,
                             hipStream_t st);
hipError_t launch_make_panels(const double* R, int64_t ldr, int n, bool f32, void* pan,
                              hipStream_t st, bool negate = true);
hipError_t launch_set_identity(double* A, int64_t lda, int rows, int cols, hipStream_t st);
int64_t bf3_panel_bytes(int n);
hipError_t launch_make_bf3_panels(const double* T, int64_t ldt, int n, void* pan3, hipStream_t st);
hipError_t launch_gram_reduce_full(const double* gpart, const GramPlan& gp, int n, double* G,
                                   hipStream_t st);
hipError_t launch_adjoint_small(const double* R, const double* dR, int64_t lddr,
                                const double* C, int ldc, int n, double* Nm, double* Rrev,
                                hipStream_t st);
hipError_t launch_make_dense_panels(const double* B, int64_t ldb, int n, bool f32, void* pan,
                                    hipStream_t st);
hipError_t launch_gram_reduce(const double* gpart, const GramPlan& gp, int n, double* G,
                              hipStream_t st);

// tall.hip
hipError_t launch_trsm(const void* X, bool f32, int64_t m, int n, int64_t ldx, const void* pan,
                       void* Q, int64_t ldq, hipStream_t st);
// Q = [Q_{1:16 s0}, X] R^{-1} where the first 16 s0 columns of Q are already
// solved (R's leading block the identity): they are read, not written; X
// (ld ldx) holds columns 16 s0 .. n-1; pan as for launch_trsm.
hipError_t launch_trsm_append(const void* X, bool f32, int64_t m, int n, int64_t ldx,
                              const void* pan, void* Q, int64_t ldq, int s0, hipStream_t st);
hipError_t launch_gram(const void* Q, bool f32, int64_t m, int n, int64_t ldq,
                       const GramPlan& gp, double* gpart, hipStream_t st);
hipError_t launch_trmm(void* Q, bool f32, int64_t m, int n, int64_t ldq, const void* pan,
                       hipStream_t st);
hipError_t launch_gemm_add(void* Q, bool f32, int64_t m, int n, int64_t ldq, const void* pan,
                           const void* C, int64_t ldc, hipStream_t st);
hipError_t launch_cross_gram(const void* A, const void* B, bool f32, int64_t m, int n, int64_t lda,
                             int64_t ldb, const GramPlan& gp, double* gpart, hipStream_t st);

inline int64_t dense_panel_elems(int n) {
  const int64_t nb = (n + 15) / 16;
  return 256 * nb * nb;
}

// Byte offset of subpanel b in the FP32 solve's bf16 x 3 panels: subpanel
// b' holds (b'+1)/2 chunks of 3072 bytes and a 3072-byte diagonal part (the
// block's inverse and the block itself, 1536 bytes each).
__host__ __device__ inline int64_t trsm_bf3_panel_offset(int b) {
  return 3072 * static_cast<int64_t>(b / 2) * ((b + 1) / 2) + 3072 * static_cast<int64_t>(b);
}
__host__ __device__ inline int64_t trsm_bf3_panel_bytes(int n) {
  return trsm_bf3_panel_offset((n + 15) / 16);
}
// The solve's refinement flags (one int per subpanel, at most 16) sit past
// the panels and the 1 KiB the staging may read beyond them.
__host__ __device__ inline int64_t trsm_bf3_flags_offset(int n) {
  return trsm_bf3_panel_bytes(n) + 1024;
}
inline int64_t trsm_bf3_ws_bytes(int n) { return trsm_bf3_flags_offset(n) + 64; }

inline int64_t panel_elems(int n) {
  const int64_t nb = (n + 15) / 16;
  return 256 * nb * (nb + 1) / 2;
}

// Persistent batched engine (batched.hip).
int64_t batched_engine_bytes(const rcholqr_problem* probs, int batch, int passes, int64_t chunk);
hipError_t launch_batched_engine(const rcholqr_problem* probs_dev, int batch, int passes,
                                 int64_t chunk, void* ws, int64_t ws_bytes, int grid,
                                 long long wait_ticks, hipStream_t st);
int batched_engine_grid();
int64_t batched_engine_status_offset(int batch);
int64_t batched_engine_stall_offset();

}  // namespace rcq
