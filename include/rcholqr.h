/*
 * rcholqr.h -- C ABI of librcholqr.so, the MI355X (gfx950) randomized
 * Cholesky QR library.
 *
 * The method is Balabanov, "Randomized Cholesky QR factorizations":
 *   Algorithm 2 (RCholeskyQR, passes = 1):
 *       P = Theta X;  [S, R] = QR(P);  Q = X R^{-1}
 *   Algorithm 3 (RCholeskyQR2, passes = 2):
 *       Algorithm 2, then A = Q^T Q;  R' = chol(A);  R <- R' R;  Q <- Q R'^{-1}
 * for a tall-and-skinny X (m x n, n << m, Section 1), with Theta a k x m
 * oblivious subspace embedding (Section 2) that is never stored: its
 * entries are regenerated on the fly from a counter-based generator
 * (Philox4x32-10) keyed by the seed, as Section 2 and Algorithm 2 allow
 * ("provided as a function handle", "seeded random number generator").
 *
 * Conventions shared by every entry point:
 *   - Matrices are column-major (Fortran) with a leading dimension >= rows.
 *   - Unless stated otherwise, pointers are DEVICE pointers on the current
 *     HIP device; the caller owns all memory.  The library never allocates
 *     or frees device memory inside these calls: all scratch space is the
 *     caller's workspace buffer, sized by rcholqr_workspace_bytes().
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Calls only enqueue work; they do not synchronise.  Numerical outcomes
 *     are written to a status word inside the workspace and read with
 *     rcholqr_status() after the stream has been synchronised.
 *   - R factors have a positive diagonal (R_s after a sign fix of the
 *     Householder R, R' from Cholesky), so the 2-pass (Q, R) is the unique
 *     thin QR of a full-rank X.
 *   - Return value: 0 on success; -i if argument i (1-based) is invalid
 *     (LAPACK style); RCHOLQR_ERR_HIP if a launch failed.
 *   - Results are bitwise reproducible run to run (no floating-point
 *     atomics; every reduction has a fixed order).
 */
#ifndef RCHOLQR_H
#define RCHOLQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Sketching embeddings (Section 2): rescaled Gaussian (entries z/sqrt(k),
 * z ~ N(0,1) by Box-Muller), Rademacher (+-1/sqrt(k)), CountSketch (one
 * +-1 per column of Theta at a hashed row, no scaling), SRHT (subsampled
 * randomized Hadamard transform sqrt(m'/k) S H D, m' = 2^ceil(log2 m): random
 * signs D, the normalised Sylvester-Hadamard matrix H, k rows sampled
 * uniformly and independently; entries d_j (-1)^popcount(s_i & j) / sqrt(k),
 * formed on the fly, so no transform of X is stored). */
enum rcholqr_sketch_kind {
  RCHOLQR_GAUSSIAN = 0,
  RCHOLQR_RADEMACHER = 1,
  RCHOLQR_COUNTSKETCH = 2,
  RCHOLQR_SRHT = 3,
  /* Test only, rcholqr_factor (and rcholqr_factor_noalloc) alone: Theta = I
   * with k = m (so m <= 1024), F64 or F32 precision.  Algorithm 2 then
   * reduces to Householder QR of X itself: R_s is the R of X with a
   * positive diagonal and Q = X R_s^{-1} its thin Q, which LAPACK's QR
   * fixes up to rounding. */
  RCHOLQR_IDENTITY_TESTONLY = 99
};

/* Working precision of the dominant (tall) operations.
 *   F64:   X, Q FP64; sketch on FP64 matrix cores.
 *   F32:   X, Q FP32; sketch accumulated in FP64; solves and Gram with
 *          FP32 accuracy on bf16 matrix cores (each FP32 operand split
 *          exactly into three bf16 parts, six products kept).
 *   MIXED: X, Q FP32; the Rademacher sketch computed exactly on int8
 *          matrix cores (each column of X rounded to a 24-bit fixed-point
 *          value under a power-of-two scale, three byte planes times the +-1
 *          entries, integer sums folded into FP64); solves and Gram as F32.
 *          Requires RCHOLQR_RADEMACHER or RCHOLQR_SRHT.
 * The SRHT sketch, in every precision, is formed by blocked fast
 * Walsh-Hadamard transforms in FP64 (one pass over X).
 * In every precision the small k x n QR, the Cholesky factorisation and
 * the R' R_s product run in FP64 on the GPU (Section 5: minor operations
 * in higher precision). */
enum rcholqr_precision {
  RCHOLQR_F64 = 0,
  RCHOLQR_F32 = 1,
  RCHOLQR_MIXED = 2
};

/* Numerical status codes written to the workspace status word. */
#define RCHOLQR_OK 0
#define RCHOLQR_SKETCH_RANK 1    /* zero diagonal in the sketch R (X rank deficient or Theta failed to embed) */
#define RCHOLQR_NONFINITE 2      /* non-finite value in X (seen through the sketch) */
#define RCHOLQR_CHOL_BREAKDOWN 1000 /* + j: non-positive pivot at column j (0-based) of chol(Q^T Q) */
#define RCHOLQR_BATCH_INVALID 3  /* batched engine: the problem was refused (see its checks) */

#define RCHOLQR_ERR_HIP (-1000)

/* Bytes of device workspace rcholqr_factor needs for this problem
 * (0 if the arguments are invalid). */
size_t rcholqr_workspace_bytes(int64_t m, int64_t n, int64_t k, int sketch_kind,
                               int passes, int precision);

/* Factor X = Q R by Algorithm 2 (passes = 1) or Algorithm 3 (passes = 2).
 *
 *  X      [in]  m x n, ldx >= m; FP64 if precision == F64, else FP32.
 *               Read only.
 *  m, n   1 <= n <= 256, n <= m.
 *  k      sketch rows, n <= k <= 1024 (the configurations use k = 3n).
 *  seed   Philox key; Theta is a deterministic function of (kind, k, seed).
 *  Q      [out] m x n, ldq >= m, same dtype as X.  Must not overlap X.
 *               passes = 1: Q is well conditioned and Theta Q ~ S is
 *               orthonormal (not Q^T Q = I).  passes = 2: Q^T Q ~ I.
 *  R      [out] n x n FP64, ldr >= n; upper triangle written, strict lower
 *               triangle set to zero.  passes = 2: R = R' R_s.
 *  S      [out, optional] k x n FP64, lds >= k: the orthonormal factor of
 *               the sketch P = S R_s (Algorithm 2 output); NULL to skip.
 *  Rs, Rp [out, optional] n x n FP64 (ld = n): the sketch R_s and the
 *               Cholesky factor R' (passes = 2), as saved for the adjoint;
 *               NULL to skip.
 *  ws     [in/out] workspace of at least rcholqr_workspace_bytes() bytes,
 *               256-byte aligned.  Holds the status word.
 * Outputs are unspecified when the status word is nonzero. */
int rcholqr_factor(const void* X, int64_t m, int64_t n, int64_t ldx, int64_t k,
                   uint64_t seed, int sketch_kind, int passes, int precision,
                   void* Q, int64_t ldq, double* R, int64_t ldr, double* S,
                   int64_t lds, double* Rs, double* Rp, void* ws,
                   size_t ws_bytes, void* stream);

/* Reduced RCholeskyQR (Algorithm 5, Section 3.3): the l x n projection
 * Z = L Q of the well-conditioned Q factor without forming Q.  One pass over
 * X forms P = Theta X and Y = L X, then [S, R] = QR(P) (Householder, positive
 * diagonal) and Z = Y R^{-1} (row-wise forward substitution, FP64).
 *
 * L is the extractor of rows k .. k+l-1 of the same counter-based operator as
 * Theta (same seed and kind, independent rows), scaled by 1/sqrt(l): an
 * oblivious embedding of its own.  Theta is exactly the k-row operator of
 * rcholqr_factor with the same seed and kind.
 *
 *  X      [in]  m x n, column-major, ld ldx >= m; FP64 for RCHOLQR_F64,
 *               FP32 for RCHOLQR_F32 and RCHOLQR_MIXED (device pointer).
 *  k, l   sketch rows (n <= k) and extractor rows (l >= 1), k + l <= 1024.
 *  seed, sketch_kind   RCHOLQR_GAUSSIAN or RCHOLQR_RADEMACHER (a CountSketch
 *               maps every column of X to one row, so its rows are not
 *               independent: refused); MIXED requires RADEMACHER.
 *  Z      [out] l x n FP64, ld ldz >= l.     R [out] n x n FP64 upper, ld ldr.
 *  S      [out, optional] k x n FP64, S = P R^{-1} (orthonormal), ld lds >= k.
 *  ws     workspace of rcholqr_reduced_workspace_bytes(m, n, k, l, kind,
 *         precision) bytes; its first word is the status (as rcholqr_factor:
 *         1 rank-deficient sketch, 2 non-finite X).
 * Returns 0, -i for invalid argument i (1-based), or RCHOLQR_ERR_HIP.
 * Asynchronous on `stream`; allocates nothing. */
size_t rcholqr_reduced_workspace_bytes(int64_t m, int64_t n, int64_t k, int64_t l,
                                       int sketch_kind, int precision);
int rcholqr_reduced(const void* X, int64_t m, int64_t n, int64_t ldx, int64_t k,
                    int64_t l, uint64_t seed, int sketch_kind, int precision,
                    double* Z, int64_t ldz, double* R, int64_t ldr, double* S,
                    int64_t lds, void* ws, size_t ws_bytes, void* stream);

/* Rank-revealing RCholeskyQR (Algorithm 7, Section 4): X Pi ~ Q R with Q
 * (m x r) well-conditioned and R (r x n) upper trapezoidal, for any X
 * (numerically rank-deficient included).  Steps: P = Theta X; D = diag of
 * the column norms of X; the rank-revealing QR of P D^{-1} (Householder with
 * column pivoting: largest remaining column norm, the first on ties,
 * followed for f > 0 by the strong RRQR swaps of Gu and Eisenstat for k = the
 * rank the rule gives: while some rho_ij^2 = (R11^{-1} R12)_ij^2 +
 * ||R22 e_j||^2 ||e_i^T R11^{-1}||^2 exceeds f^2, the largest is swapped in
 * and R triangularised again, at most 4n times); r = the least r with
 * ||R_{r+1:n,r+1:n}||_F <= tau ||R||_2 (again after any swap); Q = X Pi_{:,1:r}
 * (R_{1:r,1:r} Pi^T D Pi)^{-1} by the tall forward substitution; R <-
 * R_{1:r,:} Pi^T D Pi.  With passes = 2 (RRRCholeskyQR2, Section 4) one
 * Cholesky QR pass follows on the r columns of Q: G = Q^T Q = R'^T R',
 * Q <- Q R'^{-1}, R <- R' R (Algorithm 3 steps 2-4).
 *
 *  X, m, n, ldx, k, seed, sketch_kind, precision  as rcholqr_factor.
 *  passes 1 (Algorithm 7) or 2 (with the Cholesky QR pass).
 *  tau    truncation tolerance (>= 0).
 *  f      strong RRQR parameter: 0 (column pivoting alone) or > 1 (the
 *         paper's experiments use 1.5).
 *  Q      [out] m x n buffer (ld ldq >= m, FP64 or FP32 as X): columns 0..r-1
 *         hold Q; columns r.. are not written.  The call reads r back to the
 *         host before the tall steps (they touch only the r kept columns), so
 *         it waits for the stream once.
 *  R      [out] n x n FP64 (ld ldr): rows 0..r-1 hold R, rows r.. are zero.
 *  piv    [out] n int32 on the device: column j of X Pi is column piv[j] of X.
 *  rank   [out] one int32 on the device: r.
 *  ws     rcholqr_rr_workspace_bytes(m, n, k, kind, precision, passes)
 *         bytes; status word 0, 2 for non-finite X, or 1000 + j when the
 *         second pass's Cholesky breaks down at column j.
 * Returns 0, -i for invalid argument i (1-based), or RCHOLQR_ERR_HIP. */
size_t rcholqr_rr_workspace_bytes(int64_t m, int64_t n, int64_t k, int sketch_kind,
                                  int precision, int passes);
int rcholqr_rr(const void* X, int64_t m, int64_t n, int64_t ldx, int64_t k,
               uint64_t seed, int sketch_kind, int precision, int passes, double tau,
               double f, void* Q, int64_t ldq, double* R, int64_t ldr, int* piv,
               int* rank, void* ws, size_t ws_bytes, void* stream);

/* Column-oriented RCholeskyQR (Algorithm 4, Section 3.2), one block per
 * call: with Q_{1:j0}, S_{1:j0} and R_{1:j0,1:j0} from the calls for the
 * previous blocks (j0 = 0 for the first), factor the next b columns X_b
 * (which an application such as a block Krylov method builds from Q_{1:j0}):
 *   P_b = Theta X_b (the same Theta as for the whole matrix);
 *   R_{1:j0,b} = S_{1:j0}^T P_b (the least-squares solution for orthonormal
 *   S); [S_b, R_bb] = QR(P_b - S_{1:j0} R_{1:j0,b}) (Householder, FP64);
 *   Q_b = (X_b - Q_{1:j0} R_{1:j0,b}) R_bb^{-1} by the tall forward
 *   substitution.  Block by block this computes what Algorithm 2 computes
 *   on the whole matrix.
 *
 *  Xb     [in]  m x b, ld ldx >= m, FP64 or FP32 as the precision; may be
 *               Q's own columns j0..j0+b-1 (then nothing is copied).
 *  j0, b  columns already factored and the block width; j0 + b <= 256,
 *         j0 + b <= k <= 1024, m >= j0 + b.
 *  seed, sketch_kind, precision   as rcholqr_factor (the same for every
 *         block of one factorisation).
 *  Q      [in/out] m x (j0 + b), ld ldq: columns 0..j0-1 in (left as they
 *         are), columns j0.. out.
 *  S      [in/out] k x (j0 + b) FP64, ld lds >= k: columns 0..j0-1 in.
 *  R      [in/out] (j0 + b) x (j0 + b) FP64 upper, ld ldr: columns 0..j0-1
 *         in; the new columns (rows 0..j0+b-1) out.
 *  ws     rcholqr_col_block_workspace_bytes(m, j0, b, k, kind, precision)
 *         bytes; status word as rcholqr_factor (1: the remainder of the
 *         block's sketch is rank deficient).
 * Returns 0, -i for invalid argument i (1-based), or RCHOLQR_ERR_HIP. */
size_t rcholqr_col_block_workspace_bytes(int64_t m, int64_t j0, int64_t b, int64_t k,
                                         int sketch_kind, int precision);
int rcholqr_col_block(const void* Xb, int64_t m, int64_t j0, int64_t b, int64_t ldx,
                      int64_t k, uint64_t seed, int sketch_kind, int precision, void* Q,
                      int64_t ldq, double* S, int64_t lds, double* R, int64_t ldr,
                      void* ws, size_t ws_bytes, void* stream);

/* Read the status word of a workspace used by a completed call
 * (synchronises the current device).  *info receives 0, 1, 2 or 1000 + j.
 * Returns 0 or RCHOLQR_ERR_HIP. */
int rcholqr_status(const void* ws, int* info);

/* Stage entry point: the sketch alone, P = Theta X (k x n FP64, ldp >= k),
 * scaled by 1/sqrt(k) for the dense embeddings (Algorithm 2 step 1).
 * Same argument rules as rcholqr_factor; ws sized for the same problem. */
int rcholqr_sketch(const void* X, int64_t m, int64_t n, int64_t ldx, int64_t k,
                   uint64_t seed, int sketch_kind, int precision, double* P,
                   int64_t ldp, void* ws, size_t ws_bytes, void* stream);

/* Test-only export of raw Theta entries (before 1/sqrt(k) scaling):
 * out[ii + jj*ni] = Theta(i0+ii, j0+jj) for 0 <= ii < ni, 0 <= jj < nj, as
 * FP64 (Gaussian z, +-1, or the CountSketch column: s(j) at row h(j),
 * zero elsewhere).  m is the row count of the X that Theta is for (only the
 * SRHT depends on it, through m').  Lets tests compare Theta with the oracle
 * bit for bit.  Requires m >= 1, 0 <= i0, i0+ni <= k, 0 <= j0,
 * ni*nj <= 2^26. */
int rcholqr_debug_theta(int sketch_kind, int64_t k, int64_t m, uint64_t seed,
                        int64_t i0, int64_t ni, int64_t j0, int64_t nj,
                        double* out, void* stream);

/* Test-only: Q = X R^{-1} by the library's tall triangular solve for an
 * upper triangular FP64 R (n x n, ld = ldr, positive diagonal), in the
 * working precision of `precision` (F64: FP64 X/Q; F32/MIXED: FP32).
 * Q may equal X (in place).  ws sized by rcholqr_workspace_bytes(m, n, n,
 * RCHOLQR_GAUSSIAN, 2, precision). */
int rcholqr_trsm(const void* X, int64_t m, int64_t n, int64_t ldx,
                 const double* R, int64_t ldr, int precision, void* Q,
                 int64_t ldq, void* ws, size_t ws_bytes, void* stream);

/* Batched factorisation of independent problems (for example the panels of
 * a block Krylov method, Section 3.2) with one sketch kind, pass count and
 * precision.  `probs` is a HOST array of `batch` descriptors; every X, Q, R
 * inside is a device pointer with the same rules as rcholqr_factor (R is
 * n x n FP64, Q has X's dtype).  Instance i uses its own slice of `ws`
 * (size rcholqr_batched_workspace_bytes()).  The call fans the instances
 * out over an internal pool of 8 non-blocking streams forked from and
 * joined back to `stream` with events, performs no allocation, memset or
 * synchronisation, and can therefore be captured into a HIP graph and
 * replayed (each device's pool is created on the first call on that device,
 * outside any capture; calls on one device from several host threads at
 * once must be serialised by the caller, since they share its pool).
 * Returns 0, -i for an invalid argument i, RCHOLQR_ERR_BATCH_ENTRY - j if
 * problem j is invalid, or RCHOLQR_ERR_HIP. */
typedef struct rcholqr_problem {
  const void* X;
  int64_t m, n, ldx, k;
  uint64_t seed;
  void* Q;
  int64_t ldq;
  double* R;
  int64_t ldr;
} rcholqr_problem;
#define RCHOLQR_ERR_BATCH_ENTRY (-2000000)
size_t rcholqr_batched_workspace_bytes(const rcholqr_problem* probs, int batch,
                                       int sketch_kind, int passes, int precision);
int rcholqr_factor_batched(const rcholqr_problem* probs, int batch,
                           int sketch_kind, int passes, int precision, void* ws,
                           size_t ws_bytes, void* stream);
/* Status words of a completed batched call (synchronises): info[i] for
 * problem i, same codes as rcholqr_status. */
int rcholqr_batched_status(const rcholqr_problem* probs, int batch,
                           int sketch_kind, int passes, int precision,
                           const void* ws, int* info);

/* Persistent batched engine: many independent problems in ONE kernel
 * launch (plus a one-block setup launch), with no per-problem launches, no
 * allocation, no memset and no host synchronisation, so the call can be
 * captured into a HIP graph and replayed.  Workgroups (as many as are
 * resident at once) take tasks from a queue in device memory:
 *   sketch chunks (P_c = Theta X_c for row chunks c and 64 Theta rows at a
 *   time), then per problem the FP64 Householder QR of P = sum_c P_c and
 *   the solve panels, then solve chunks (Q1 = X R_s^{-1}, and for 2 passes
 *   the chunk's Gram G_c), then per problem the FP64 Cholesky of
 *   G = sum_c G_c with R = R' R_s, then product chunks (Q = Q1 R'^{-1}).
 * A task waits (bounded spin) for its problem's previous phase; every
 * reduction has a fixed order, so results are reproducible run to run.
 * Problems: FP32 X and Q (column-major), FP64 R; n in {16, 32, ..., 128},
 * k a multiple of 16 with n <= k <= 384, m >= n; sketch RCHOLQR_RADEMACHER
 * (the same Theta, bit for bit, as rcholqr_factor with that seed); passes 1
 * or 2.  X, Q and R are read and written as in rcholqr_factor (Q must not
 * overlap X).  The products of X with the +-1 entries are exact (X split
 * into three bf16 parts) and summed in FP32 per 32 rows, then in FP64; the
 * solves and the Gram run on FP32 matrix cores (exact products), the small
 * steps in FP64.
 *
 *  probs_dev   DEVICE array of `batch` descriptors (the same struct as the
 *              stream-pool entry); a problem outside the rules above gets
 *              status RCHOLQR_BATCH_INVALID and is skipped.
 *  chunk_rows  rows per tall task, a positive multiple of 128; 0 takes the
 *              value rcholqr_batched_engine_chunk(max n) returns (the
 *              tuned one once rcholqr_init has loaded a tuning file).
 *  ws          at least rcholqr_batched_engine_workspace_bytes(probs_host,
 *              batch, passes, chunk_rows) bytes, computed from a HOST copy
 *              of the same descriptors with the same chunk_rows; a smaller
 *              buffer makes every status RCHOLQR_BATCH_INVALID (the engine
 *              sees the size on the device).
 * rcholqr_batched_engine_status (synchronises) copies the per-problem
 * status words (0, 1, 1000 + j, or RCHOLQR_BATCH_INVALID) to info and
 * returns RCHOLQR_ERR_ENGINE if the engine stopped on a bounded wait.
 * Returns 0, -i for an invalid argument i, or RCHOLQR_ERR_HIP. */
#define RCHOLQR_ERR_ENGINE (-4000)
int64_t rcholqr_batched_engine_chunk(int64_t max_n);
size_t rcholqr_batched_engine_workspace_bytes(const rcholqr_problem* probs_host, int batch,
                                              int passes, int64_t chunk_rows);
int rcholqr_factor_batched_engine(const rcholqr_problem* probs_dev, int batch,
                                  int sketch_kind, int passes, int64_t chunk_rows,
                                  void* ws, size_t ws_bytes, void* stream);
int rcholqr_batched_engine_status(int batch, const void* ws, int* info);

/* Tuning of the engine's rows per tall task (a project-written autotuner).
 * rcholqr_batched_engine_tune times the engine on the given batch for each
 * candidate chunk (1024 ... 16384 rows whose workspace fits in ws_bytes),
 * keeps the fastest for the batch's largest n, and, when save_path is not
 * NULL, writes the table of tuned values as JSON
 * ({"batched_engine_chunk_rows": {"<max n>": rows, ...}}).  It synchronises
 * the device.  rcholqr_init(path) loads such a file (NULL: built-in
 * defaults), once, before other calls; the table is read-only afterwards.
 * Both return 0, -1 for an unreadable or malformed file / unwritable path,
 * -i for another invalid argument, or RCHOLQR_ERR_HIP. */
int rcholqr_init(const char* tune_path);
int rcholqr_batched_engine_tune(const rcholqr_problem* probs_host,
                                const rcholqr_problem* probs_dev, int batch,
                                int sketch_kind, int passes, void* ws, size_t ws_bytes,
                                const char* save_path, void* stream);

/* Reverse-mode derivative of the 2-pass factorisation (the positive-diagonal
 * thin QR X = Q R, which Algorithm 3 returns; the paper does not treat
 * derivatives).  Given dQ (m x n) and dR (n x n, upper triangle used),
 *     M = R dR^T - dQ^T Q,   N = copyltu(M) (lower triangle mirrored up),
 *     dX = (dQ + Q N) R^{-T}.
 * Q is not stored by the forward call: it is recomputed from X and the
 * saved R_s, R' (the `Rs`, `Rp` outputs of rcholqr_factor with passes = 2)
 * by the same kernels, so it equals the forward Q bit for bit.  The final
 * R^{-T} is applied by row-wise substitution (R = R' R_s is formed in FP64).
 *  X      [in]  m x n, ldx >= m, FP64 (precision F64) or FP32 (F32/MIXED).
 *  Rs, Rp [in]  n x n FP64, ld = n, upper triangular.
 *  dQ     [in]  m x n, lddq >= m, same dtype as X.
 *  dR     [in, optional] n x n FP64, ld lddr >= n; NULL means zero.
 *  dX     [out] m x n, lddx >= m, same dtype as X; must not overlap X or dQ.
 *  ws     workspace of rcholqr_backward_workspace_bytes(m, n, precision).
 * Returns 0, -i for the i-th invalid argument, or RCHOLQR_ERR_HIP. */
size_t rcholqr_backward_workspace_bytes(int64_t m, int64_t n, int precision);
int rcholqr_backward(const void* X, int64_t m, int64_t n, int64_t ldx,
                     const double* Rs, const double* Rp, const void* dQ,
                     int64_t lddq, const double* dR, int64_t lddr, int precision,
                     void* dX, int64_t lddx, void* ws, size_t ws_bytes,
                     void* stream);

/* Phase timing.  rcholqr_profile_enable(1) creates a ring of HIP events
 * (no device memory is allocated); while enabled, every rcholqr_factor call
 * records one event at each phase boundary on its own stream:
 *   0 sketch (Theta X and its reduction)   1 small QR (Householder, sign fix)
 *   2 first solve (Q1 = X R_s^{-1})        3 Gram (Q1^T Q1 and its reduction)
 *   4 Cholesky and R = R' R_s               5 second solve (Q = Q1 R'^{-1})
 * rcholqr_profile_read() waits for the recorded calls, adds their phase
 * durations into ms[0..5] (milliseconds, summed over calls), returns the
 * number of calls, and clears the record.  At most 256 calls are kept
 * between reads (older ones are dropped).  rcholqr_profile_enable(0) frees
 * the events.  Returns RCHOLQR_ERR_HIP on a runtime error.  Not thread safe. */
#define RCHOLQR_NPHASES 6
int rcholqr_profile_enable(int on);
int rcholqr_profile_read(double* ms);

/* Plain device-to-device copy of `bytes` bytes (a multiple of 16) from src
 * to dst (device pointers, 16-byte aligned, not overlapping) on `stream`,
 * 16 bytes per lane.  It is the known-size reference against which hardware
 * byte counters (FETCH_SIZE, WRITE_SIZE) of the other kernels are scaled to
 * HBM bytes.  Returns -1/-2 for a null or misaligned src/dst, -3 if bytes is
 * not a multiple of 16, RCHOLQR_ERR_HIP if the launch failed. */
int rcholqr_device_copy(const void* src, void* dst, size_t bytes, void* stream);

/* rcholqr_factor for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * launch sequence and kernels as rcholqr_factor with passes, kind and
 * precision as there (so the same Q and R, bit for bit), but the workspace
 * is a library-owned device array of rcholqr_noalloc_max_bytes() bytes
 * (256 MiB; every GPU the library runs on holds its own copy until the
 * process ends), not a caller buffer.  The call allocates, frees and
 * clears nothing: every word the kernels read is written first in the same
 * call (the status word included).
 *
 *  X, m, n, ldx, k, seed, sketch_kind, passes, precision, Q, ldq, R, ldr
 *         as rcholqr_factor (no S, R_s or R' outputs).
 * Returns 0, -i for invalid argument i (1-based), RCHOLQR_ERR_NOALLOC_SIZE
 * when the problem's workspace (rcholqr_workspace_bytes) exceeds the array,
 * or RCHOLQR_ERR_HIP.  Calls on one GPU share its array and each keeps the
 * last call's contents: calls that overlap in time on one GPU (two streams,
 * two host threads) race and give undefined results; serialise them.
 * rcholqr_noalloc_status() reads the status word of the last completed
 * call on the current device (it synchronises the device). */
#define RCHOLQR_ERR_NOALLOC_SIZE (-3000)
size_t rcholqr_noalloc_max_bytes(void);
int rcholqr_factor_noalloc(const void* X, int64_t m, int64_t n, int64_t ldx,
                           int64_t k, uint64_t seed, int sketch_kind, int passes,
                           int precision, void* Q, int64_t ldq, double* R,
                           int64_t ldr, void* stream);
int rcholqr_noalloc_status(int* info);

/* Human-readable text for a return code or status value. */
const char* rcholqr_error_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* RCHOLQR_H */
