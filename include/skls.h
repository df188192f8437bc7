/*
 * skls -- sparse-embedding sketching and least squares on AMD MI355X (gfx950).
 *
 * C ABI of the library libskls.so.  The operations follow Clarkson & Woodruff,
 * "Low Rank Approximation and Regression in Input Sparsity Time"
 * (arXiv:1207.6365); each declaration cites the part of the paper that defines
 * what it computes.
 *
 * Conventions shared by every entry point:
 *  - Pointers documented as "device" address GPU memory of the current HIP
 *    device; "host" pointers address CPU memory.  All device buffers (inputs,
 *    outputs, workspace) belong to the caller; the library allocates and frees
 *    no device memory.  Workspace sizes come from the *_workspace queries; a
 *    workspace may be reused between calls once the previous call on it has
 *    completed in stream order.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is enqueued on it in order.  Calls marked "asynchronous" return before the
 *    GPU finishes; the others synchronise `stream` before returning.
 *  - Indices are 0-based (the paper writes [n] = {1..n}).  Rows i in [0, n),
 *    buckets in [0, t).
 *  - Errors are returned as skls_status.  Nothing aborts and no C++ exception
 *    crosses the ABI.  skls_last_error() gives a message for the calling thread.
 *    On an error return no work has been enqueued, except SKLS_ERR_DEVICE
 *    (a HIP call failed), SKLS_ERR_RANK and SKLS_ERR_NOCONV (detected after
 *    GPU work ran; outputs then hold what the documentation of the call says).
 *  - Nothing here is thread-safe with respect to two calls that share a
 *    workspace or output buffer; calls on distinct buffers may run concurrently.
 */
#ifndef SKLS_H
#define SKLS_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define SKLS_API __attribute__((visibility("default")))
#else
#define SKLS_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SKLS_F64 = 0,  /* IEEE binary64 */
  SKLS_F32 = 1,  /* IEEE binary32 */
  SKLS_BF16 = 2  /* bfloat16 (upper half of a binary32), read-only inputs */
} skls_dtype;

typedef enum {
  SKLS_OK = 0,
  SKLS_ERR_ARG = 1,        /* null pointer, bad enum or option value */
  SKLS_ERR_SHAPE = 2,      /* inconsistent or unsupported sizes */
  SKLS_ERR_DTYPE = 3,      /* unsupported combination of types */
  SKLS_ERR_RANK = 4,       /* the sketch is numerically rank deficient */
  SKLS_ERR_NOCONV = 5,     /* the iteration did not certify within max_iter */
  SKLS_ERR_WORKSPACE = 6,  /* workspace missing or smaller than required */
  SKLS_ERR_DEVICE = 7,     /* a HIP runtime call or kernel launch failed */
  SKLS_ERR_NOTIMPL = 8     /* operation not provided by the library */
} skls_status;

typedef enum { SKLS_DENSE = 0, SKLS_CSR = 1 } skls_layout;

/*
 * Input matrix A (n x d), read-only, device memory.
 *  dense: row-major, element (i, j) at val[i * ld + j], ld >= d.
 *  CSR:   row i holds entries row_ptr[i] .. row_ptr[i+1]-1 of col_idx / val;
 *         row_ptr has n+1 entries, row_ptr[0] = 0, row_ptr[n] = nnz, and is
 *         int32 (row_ptr_64 = 0) or int64 (row_ptr_64 = 1).  Column indices lie
 *         in [0, d); order within a row is free, repeats are summed.
 * The library requires n < 2^31 and d < 2^31.
 */
typedef struct {
  int32_t layout;          /* skls_layout */
  int32_t dtype;           /* skls_dtype of val */
  int64_t n, d;
  int64_t ld;              /* dense: elements between consecutive rows */
  int64_t nnz;             /* CSR: number of stored entries */
  const void* row_ptr;     /* CSR: device, int32 or int64 [n+1] */
  int32_t row_ptr_64;      /* CSR: 1 if row_ptr is int64 */
  int32_t reserved;
  const int32_t* col_idx;  /* CSR: device [nnz] */
  const void* val;         /* device: dense n*ld or CSR nnz values */
} skls_matrix;

/* Human-readable name of a status code (static string). */
SKLS_API const char* skls_status_str(int32_t status);
/* Message describing the last error returned on the calling thread ("" if none). */
SKLS_API const char* skls_last_error(void);
/* Library version string. */
SKLS_API const char* skls_version(void);

/*
 * Hash and sign of the sparse embedding S = Phi D (Section 2): for global rows
 * i = start .. start+n-1, bucket[i-start] = h(i) in [0, t) and sign[i-start] =
 * the diagonal entry of D, +1 or -1.  Drawn from SplitMix64 (Steele, Lea &
 * Flood 2014) output i of stream `seed`: h = ((z >> 32) * t) >> 32, sign = -1
 * iff bit 0 of z is set.  Bit-exact and identical on every device.
 * bucket: device int32[n]; sign: device int8[n] (either may be NULL).
 * Requires 1 <= t < 2^31, n >= 0.  Asynchronous.
 */
SKLS_API int32_t skls_hash(int64_t n, int64_t t, uint64_t seed, int64_t start, int32_t* bucket, int8_t* sign,
                  void* stream);

/*
 * Sketch-apply variants (Section 2; the O(nnz(A)) product of the main theorem
 * of Section 3 and of the regression theorem of Section 7).
 *  SKLS_SKETCH_AUTO      library default for the layout and sizes
 *  SKLS_SKETCH_ATOMIC    stream rows in storage order; scatter-add each entry
 *                        into S*A with device-wide atomics (S*A zeroed first)
 *  SKLS_SKETCH_SORTED    group rows by bucket (counting sort of h), then one
 *                        wavefront reduces each bucket's rows in increasing
 *                        row order and writes its row of S*A once; results are
 *                        reproducible bit for bit from run to run when no
 *                        bucket holds more than 128 rows.  CSR inputs need
 *                        d * sizeof(out) <= 12288 bytes.
 *  SKLS_SKETCH_BINNED    group rows into bins of consecutive buckets; one
 *                        block keeps a bin's rows of S*A in LDS, adds the
 *                        bin's rows into them with LDS atomics and writes
 *                        them once (float results depend on the order of the
 *                        additions).  Needs d * sizeof(out) <= 32768 bytes.
 * AUTO picks BINNED for CSR inputs and SORTED for dense inputs with at most
 * 256 rows per bucket on average (BINNED above that), and ATOMIC where the
 * chosen one does not apply.  An explicitly requested variant that does not
 * support the shape fails with SKLS_ERR_SHAPE.
 */
enum { SKLS_SKETCH_AUTO = 0, SKLS_SKETCH_ATOMIC = 1, SKLS_SKETCH_SORTED = 2, SKLS_SKETCH_BINNED = 3 };

/* Bytes of workspace skls_sketch needs for this input, t and variant. */
SKLS_API int32_t skls_sketch_workspace(const skls_matrix* A, int64_t t, int32_t variant, size_t* bytes);

/*
 * SA = S A and Sb = S b with S = Phi D (Section 2): row h(i) of SA accumulates
 * sign(i) * A[i, :], and Sb[h(i)] accumulates sign(i) * b[i].  When w is not
 * NULL the learned value w[i] replaces sign(i) (h stays the hashed bucket).
 *  A:      input matrix (F64, F32 or BF16 values).
 *  b:      device vector [n] of type b_dtype (F64 or F32), or NULL.
 *  t:      sketch rows, 1 <= t < 2^31.
 *  seed:   64-bit stream of the hash (see skls_hash).
 *  w:      device float32 [n] or NULL.
 *  SA:     device, t x d row-major (leading dimension d), type out_dtype (F64
 *          or F32); every element is written.
 *  Sb:     device [t] of type out_dtype, or NULL (required iff b != NULL).
 *  Sums are accumulated in out_dtype.  Asynchronous.
 */
SKLS_API int32_t skls_sketch(const skls_matrix* A, const void* b, int32_t b_dtype, int64_t t, uint64_t seed,
                    const float* w, int32_t variant, void* SA, void* Sb, int32_t out_dtype, void* ws,
                    size_t ws_bytes, void* stream);

/*
 * The same sketch of a block of rows that starts at global row `row_start`:
 * row i of A is hashed as row row_start + i (h, sign and, for CSR, nothing
 * else changes), so the sketches of consecutive row blocks A_1, A_2, ... of a
 * taller matrix, each with its own row_start, sum to the sketch of the whole
 * (S A = sum_g S A_g: Phi D acts on each row independently, Section 2).  b and
 * w are indexed by the block's own rows.  row_start >= 0; other arguments as
 * for skls_sketch.  Asynchronous.
 */
SKLS_API int32_t skls_sketch_rows(const skls_matrix* A, int64_t row_start, const void* b, int32_t b_dtype, int64_t t,
                                  uint64_t seed, const float* w, int32_t variant, void* SA, void* Sb,
                                  int32_t out_dtype, void* ws, size_t ws_bytes, void* stream);

/*
 * Reusable bucket plans.  The buckets h(i) depend only on (seed, i, t)
 * (Section 2), so the grouping of the rows by bucket that the SORTED and
 * BINNED variants build can be kept and reused for every matrix with the same
 * rows: any dense matrix with the same n, or a CSR matrix with the same row
 * pointers (values and columns may change).  skls_sketch_plan builds it into
 * a caller-owned device buffer and fills the host descriptor; each
 * skls_sketch_planned call then runs only the reduce.
 */
typedef struct {
  int64_t n, d, t;
  int64_t row_start;  /* global index of the first row (as skls_sketch_rows) */
  uint64_t seed;
  int32_t layout;     /* skls_layout of the matrix the plan was built for */
  int32_t row_ptr_64;
  int32_t variant;    /* the variant that will run (AUTO resolved) */
  int32_t out_dtype;  /* F64 or F32 */
  int64_t bytes;      /* bytes of the device plan (0 for ATOMIC, which has none) */
  int64_t reserved[2];
} skls_sketch_plan_desc;

/* Bytes of the device plan for this input shape, t, variant and output type. */
SKLS_API int32_t skls_sketch_plan_workspace(const skls_matrix* A, int64_t t, int32_t variant, int32_t out_dtype,
                                            size_t* bytes);
/*
 * Build the plan of A's rows (row pointers for CSR; nothing of the values)
 * for (row_start, t, seed, variant, out_dtype) into `plan` (device, plan_bytes
 * from the query) and fill `desc` (host).  Asynchronous.
 */
SKLS_API int32_t skls_sketch_plan(const skls_matrix* A, int64_t row_start, int64_t t, uint64_t seed,
                                  int32_t variant, int32_t out_dtype, void* plan, size_t plan_bytes,
                                  skls_sketch_plan_desc* desc, void* stream);
/*
 * SA = S A (and Sb = S b) with a plan from skls_sketch_plan.  A must have the
 * plan's n, d, layout and row pointer width, and (CSR) the same row pointer
 * contents as when the plan was built; results are then those of skls_sketch
 * with the plan's arguments.  For CSR inputs with b, b[i] is gathered per
 * row during the reduce (the plan holds no values).  The plan is only read:
 * several calls may share it.  Asynchronous.
 */
SKLS_API int32_t skls_sketch_planned(const skls_matrix* A, const void* b, int32_t b_dtype, const float* w, void* SA,
                                     void* Sb, const skls_sketch_plan_desc* desc, const void* plan,
                                     size_t plan_bytes, void* stream);

/*
 * skls_sketch without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  The bucket plan is kept in a fixed array of
 * SKLS_NOALLOC_SCRATCH_BYTES bytes that the library holds on each device it
 * runs on until the process ends; the call allocates nothing.  Arguments and
 * results as for skls_sketch.  Inputs whose plan needs more than that
 * (skls_sketch_workspace) are rejected with SKLS_ERR_WORKSPACE.  Every call
 * on a device shares that device's array: calls that overlap on one device
 * (other streams or host threads) race and must be serialised by the caller.
 * Asynchronous.
 */
#define SKLS_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
SKLS_API int32_t skls_sketch_noalloc(const skls_matrix* A, const void* b, int32_t b_dtype, int64_t t, uint64_t seed,
                                     const float* w, int32_t variant, void* SA, void* Sb, int32_t out_dtype,
                                     void* stream);

/*
 * Generalized sparse embedding (Section 5, the construction): a hash h sends
 * each row i to one of q groups; group g applies its own matrix B^(g), the
 * stack of `a` independent sparse embeddings sqrt(1/a) Phi_j D_j onto v
 * rows each.  S = blockdiag(B^(1), ..., B^(q)) P has t = a q v rows and
 * exactly `a` nonzeros +-1/sqrt(a) per column.
 * Randomness: h(i) = bucket of output i of the stream `seed` reduced to
 * [0, q) (as in skls_hash); copy j (0-based) hashes row i to
 * h_j(i) in [0, v) with sign from output i of the stream
 * seed + (j + 1) * 0xD1B54A32D192ED03 (mod 2^64).
 * Row order of SA: copy-major, row j q v + h(i) v + h_j(i) (a permutation of
 * the block-diagonal order; norms and the R of a QR of S A do not change).
 *  q, v:   groups and rows per copy, q v < 2^31; a: copies, 1 <= a <= 256.
 *  SA:     device, (a q v) x d row-major, type out_dtype; Sb: (a q v) or NULL.
 *  variant, ws: as for skls_sketch with t = q v (one copy at a time).
 * Each copy is one pass over A, so the cost is a times that of skls_sketch.
 * Asynchronous.
 */
SKLS_API int32_t skls_sketch_general_workspace(const skls_matrix* A, int64_t q, int64_t v, int32_t variant,
                                               size_t* bytes);
SKLS_API int32_t skls_sketch_general(const skls_matrix* A, const void* b, int32_t b_dtype, int64_t q, int64_t v,
                                     int32_t a, uint64_t seed, int32_t variant, void* SA, void* Sb,
                                     int32_t out_dtype, void* ws, size_t ws_bytes, void* stream);

/*
 * Triangular factor of a QR factorisation of a tall matrix (Section 7 solves
 * the sketched regression through the QR factorisation of S A, as R^{-1} Q^T S b;
 * Section 6 uses the same R as the change of basis that makes S A R^{-1}
 * orthonormal).  Computed as the Cholesky factor of the Gram matrix M^T M
 * formed in float64 on the matrix cores (CholeskyQR): in exact arithmetic this
 * is the R of M = QR with a positive diagonal.
 *  M:     device, m x d row-major (leading dimension d), F64 or F32, m >= d,
 *         d <= 8192.
 *  R:     device float64 d x d row-major, upper triangular (zeros below).
 *  Rinv:  device float64 d x d row-major, the inverse of R, or NULL.
 *  Returns SKLS_ERR_RANK (R, Rinv then unspecified) when a pivot of the Gram
 *  matrix is not positive or some R_kk <= 4 sqrt(d * 2^-52) sqrt(G_kk), G = M^T M
 *  (R_kk / sqrt(G_kk) is the sine of the angle between column k and the
 *  columns before it, so the test does not depend on column scaling; a
 *  Gram-based factor cannot resolve smaller angles).  Synchronous.
 */
SKLS_API int32_t skls_qr_r_workspace(int64_t m, int64_t d, size_t* bytes);
SKLS_API int32_t skls_qr_r(const void* M, int32_t dtype, int64_t m, int64_t d, double* R, double* Rinv, void* ws,
                  size_t ws_bytes, void* stream);

/* Options of skls_lstsq.  Zero-initialise, then set fields. */
typedef struct {
  int64_t t;            /* sketch rows (t >= d) */
  uint64_t seed;        /* hash stream */
  double delta;         /* target: ||A x - b|| <= (1 + delta) min ||A x - b||; 0 -> 1e-6 */
  double sigma_lb;      /* assumed lower bound on sigma_min(A R^{-1}); 0 -> 0.5 */
  int32_t max_iter;     /* LSQR iterations (total over refinements); 0 -> 100 */
  int32_t precision;    /* 0: float64 arithmetic in every pass ("plain");
                           1: mixed -- float32 LSQR passes with float64
                              residual refinement */
  int32_t sketch_only;  /* 1: return the sketch-and-solve x~ without iterating */
  int32_t variant;      /* sketch variant (SKLS_SKETCH_*) */
  const float* w;       /* learned sketch values (device float32 [n]) or NULL */
  const double* x0;     /* device float64 [d] or NULL: start the iteration here instead of at the
                           sketch-and-solve x~ (Section 7.7 starts from any x(0) whose error is at
                           most that of x = 0); the sketch still provides R */
  int32_t max_retries;  /* extra attempts with a new sketch when one fails (0: none): a sketch whose
                           S A is rank deficient, or an iteration that does not certify within
                           max_iter.  Attempt r uses seed + r * 0x9E3779B97F4A7C15 (mod 2^64); the
                           failure probability of a sparse embedding (Section 3) then drops
                           geometrically with the attempts */
  int32_t second_stage; /* 0: factor S A directly.  m > 0 (d <= m <= t, m <= 65536): factor
                           Pi1 A = F (S A) instead, F the m x t sign matrix of skls_second_stage
                           (stream seed), and take x~ from F S b.  sigma_lb should then reflect the
                           wider spread of F (about 1 - sqrt(d / m) for the smallest singular value
                           of F restricted to the range of S A) */
} skls_lstsq_opts;

typedef struct {
  int32_t iterations;     /* LSQR iterations run */
  int32_t refinements;    /* outer float64 residual refinements (mixed) */
  int32_t certified;      /* 1 if the stopping certificate holds at the result */
  int32_t retries;        /* attempts after the first (each with a new sketch) */
  double resid_norm;      /* ||b - A x|| at the result (float64 accumulation) */
  double grad_norm;       /* ||R^{-T} A^T (b - A x)|| at the result */
  double ratio_bound;     /* certified bound on ||Ax-b|| / min ||Ax-b|| (given sigma_lb) */
  double ms_sketch, ms_qr, ms_iter;  /* phase times (device events) */
} skls_lstsq_info;

SKLS_API int32_t skls_lstsq_workspace(const skls_matrix* A, const skls_lstsq_opts* opts, size_t* bytes);

/*
 * Least squares min_x ||A x - b||_2 (Section 7).  Sketch-and-solve (regression
 * theorem of Section 7) gives x~ = argmin ||S A x - S b|| through the R of S A;
 * unless sketch_only, LSQR (Paige & Saunders 1982) on M = A R^{-1} started at
 * x~ -- the R-preconditioned Krylov (conjugate-gradient type) iteration of Section 7.7 -- runs until the
 * certificate ||M^T r|| <= sigma_lb * sqrt(D / (1 + D)) ||r|| with
 * D = (1 + delta)^2 - 1 holds for r = b - A x evaluated with float64
 * accumulation; this certifies ratio <= 1 + delta when sigma_min(M) >= sigma_lb.
 *  A:    dense or CSR input (F64, F32 or BF16 values).
 *  b:    device float64 [n].
 *  x:    device float64 [d], output.
 *  info: host, may be NULL.
 * With max_retries, a failed attempt is repeated with a new seed (info->retries).
 * Returns SKLS_ERR_RANK if S A is rank deficient (x unspecified) and
 * SKLS_ERR_NOCONV if max_iter ran out (x = last iterate).  Synchronous.
 */
SKLS_API int32_t skls_lstsq(const skls_matrix* A, const double* b, const skls_lstsq_opts* opts, double* x,
                   skls_lstsq_info* info, void* ws, size_t ws_bytes, void* stream);

/*
 * Second sketch stage (Section 6: Pi1 = F S, the sparse embedding followed by
 * a dense Johnson-Lindenstrauss map; the composition facts of Section 8 keep
 * the embedding property of the product): given S A and
 * S b (t rows), FSA = F (S A) and FSb = F (S b) with F the m x t matrix whose
 * entry (i, r) is -1 / sqrt(m) when bit b(r mod 64) of SplitMix64 output
 * i * ceil(t / 64) + floor(r / 64) of the stream seed ^ 0x7374616765327369 is
 * set, else +1 / sqrt(m); b(c) = 32 floor(c / 32) + 16 (c mod 2) + 15 -
 * floor((c mod 32) / 2), a fixed order of the word's bits.
 *  SA:   device [t x d] row-major, dtype F64 or F32.  Each entry is rounded to
 *        float32 and then to bfloat16 (round to nearest even each); the products
 *        with the signs are summed in float32 over splits of the t rows and the
 *        splits in float64.
 *  Sb:   device [t] of the same dtype, or NULL (then FSb is not written).  F S b
 *        is summed in float64 from Sb as given.
 *  FSA:  device float64 [m x d] row-major, output.  FSb: device float64 [m].
 *  Requires 1 <= d <= 8192, 1 <= m <= 65536, 1 <= t < 2^31.  Asynchronous.
 */
SKLS_API int32_t skls_second_stage_workspace(int64_t t, int64_t d, int64_t m, size_t* bytes);
SKLS_API int32_t skls_second_stage(const void* SA, const void* Sb, int32_t dtype, int64_t t, int64_t d, int64_t m,
                                   uint64_t seed, double* FSA, double* FSb, void* ws, size_t ws_bytes,
                                   void* stream);

/*
 * Approximate leverage scores (Section 6, theorem on approximating all leverage
 * scores): scores[i] = || A[i, :] R^{-1} Pi2 ||^2 where R is the triangular
 * factor of S A (S from t, seed) and Pi2 is a d x k Johnson-Lindenstrauss
 * matrix (device float64, row-major).  Pi2 = NULL uses the d x k matrix of
 * signs / sqrt(k) with the sign of entry e from bit 0 of output e of the
 * stream seed ^ 0x6C65766572616765 (the projection of skls_low_rank).  The
 * products A T, T = R^{-1} Pi2, are accumulated in float32.
 *  scores: device float32 [n].
 * Returns SKLS_ERR_RANK if S A is rank deficient.  Synchronous.
 */
SKLS_API int32_t skls_leverage_workspace(const skls_matrix* A, int64_t t, int32_t k, size_t* bytes);
SKLS_API int32_t skls_leverage_scores(const skls_matrix* A, int64_t t, uint64_t seed, int32_t k, const double* Pi2,
                             float* scores, void* ws, size_t ws_bytes, void* stream);

/*
 * The same scores from a triangular factor the caller already has (Section 6:
 * any R for which A R^{-1} is well conditioned, such as the R of S A that
 * skls_qr_r or a least-squares solve produced): scores[i] = ||A[i, :] R^{-1}
 * Pi2||^2, R^{-1} by the doubling inverse of skls_qr_r.
 *  R:    device float64 d x d row-major, upper triangular, nonzero diagonal
 *        (entries below the diagonal are not read).
 *  Pi2:  device float64 d x k, or NULL for the seeded sign matrix above
 *        (stream `seed`).
 *  scores: device float32 [n].  Asynchronous.
 */
SKLS_API int32_t skls_leverage_from_r_workspace(const skls_matrix* A, int32_t k, size_t* bytes);
SKLS_API int32_t skls_leverage_scores_from_r(const skls_matrix* A, const double* R, int32_t k, const double* Pi2,
                                             uint64_t seed, float* scores, void* ws, size_t ws_bytes,
                                             void* stream);

/*
 * Gram matrix C = A^T A (float32 output, float32 accumulation), used as the
 * target of the learned-value distortion loss.  A dense or CSR.
 *  C: device float32 d x d row-major.  Asynchronous.
 */
SKLS_API int32_t skls_gram_workspace(const skls_matrix* A, size_t* bytes);
SKLS_API int32_t skls_gram(const skls_matrix* A, float* C, void* ws, size_t ws_bytes, void* stream);

/*
 * Learned sketch values (an extension of Section 2: the signs of D become
 * trainable values w while h stays hashed).  With Y = S_w A and
 * E = Y^T Y - C (C = A^T A from skls_gram):
 *   loss = ||E||_F^2,   dloss/dw[i] = < (4 Y E)[h(i), :], A[i, :] >.
 *  A:          dense float32 input, d <= 4096.
 *  C:          device float32 d x d.
 *  w:          device float32 [n].
 *  grad_scale: the gradient is multiplied by this factor.
 *  accumulate: 0 -> grad_w = grad_scale * dloss/dw; 1 -> grad_w += it.
 *  loss:       device float32 scalar (always overwritten with the raw loss).
 *  grad_w:     device float32 [n], or NULL to evaluate the loss only.
 *  Asynchronous.
 */
SKLS_API int32_t skls_learned_workspace(const skls_matrix* A, int64_t t, size_t* bytes);
SKLS_API int32_t skls_learned_grad(const skls_matrix* A, const float* C, int64_t t, uint64_t seed, const float* w,
                                   float grad_scale, int32_t accumulate, float* loss, float* grad_w, void* ws,
                                   size_t ws_bytes, void* stream);

/*
 * The same loss and gradient with the forward sketch run from a reusable plan
 * (skls_sketch_plan of a dense matrix of this shape, float32 output,
 * row_start 0; t and seed come from desc).  Matrices of one shape share one
 * plan, since the plan depends only on (seed, n, t).  The workspace of
 * skls_learned_workspace suffices.  Asynchronous.
 */
SKLS_API int32_t skls_learned_grad_planned(const skls_matrix* A, const float* C, const skls_sketch_plan_desc* desc,
                                           const void* plan, size_t plan_bytes, const float* w, float grad_scale,
                                           int32_t accumulate, float* loss, float* grad_w, void* ws,
                                           size_t ws_bytes, void* stream);

/*
 * The weighted sum of the gradients of a batch of count matrices of one
 * shape (n, d), the forward sketches run from one reusable plan as in
 * skls_learned_grad_planned:
 *   loss[j] = ||E_j||_F^2 of matrix j (raw, unweighted),
 *   grad_w  = sum_j scale[j] * dloss_j/dw   (accumulate = 0), or += it.
 * At d <= 64 and t <= 4096 with a dense SORTED plan each step is one launch
 * over up to 16 matrices at a time (sketches, Gram, losses, the gradient of
 * each matrix into a slot of its own, the sum of the slots in matrix order).
 * Otherwise the matrices' chains of launches run on up to four streams at
 * once (the caller's and three of the library's, default priority), forked
 * from and joined back to `stream`; matrix j adds its weighted gradient into
 * the slot of lane j mod 4, and the slots are summed in lane order at the
 * end.  Either way the result is the same from run to run; it may differ in
 * the last bits from a sequence of skls_learned_grad_planned calls, which add
 * in matrix order.
 *  count:  number of matrices, >= 1.
 *  A:      host array of count dense float32 matrix descriptors of the
 *          plan's shape (each with its own ld).
 *  C:      host array of count device pointers to float32 d x d targets.
 *  scale:  host array of count weights, or NULL for weights 1.
 *  loss:   device float32 [count].
 *  grad_w: device float32 [n], or NULL to evaluate the losses only.
 *  ws:     skls_learned_batch_workspace bytes (A: any matrix of the shape).
 * Overlapping calls must use distinct workspaces.  Asynchronous.
 */
SKLS_API int32_t skls_learned_batch_workspace(const skls_matrix* A, int64_t t, size_t* bytes);
SKLS_API int32_t skls_learned_grad_batch(int32_t count, const skls_matrix* A, const float* const* C,
                                         const float* scale, const skls_sketch_plan_desc* desc, const void* plan,
                                         size_t plan_bytes, const float* w, int32_t accumulate, float* loss,
                                         float* grad_w, void* ws, size_t ws_bytes, void* stream);

/*
 * One Adam step (Kingma & Ba 2015) on w [n] (device float32) with gradient g,
 * moments m, v (device float32, caller-initialised to 0), step >= 1.
 * Asynchronous.
 */
SKLS_API int32_t skls_adam_step(int64_t n, float* w, const float* g, float* m, float* v, int32_t step, float lr,
                       float beta1, float beta2, float eps, void* stream);

/*
 * Kernel-phase timing (tracing).  While enabled, every kernel phase the library
 * launches ("sketch_plan", "sketch_apply", "gram", "cholesky", "trinv",
 * "lsqr_pass", "leverage", ...) is bracketed by HIP events recorded on the
 * stream of the call, so the times are those of the kernels on that stream.
 *  skls_profile_enable(on): clears all counters and turns timing on or off.
 *  skls_profile_count():    number of phase names recorded so far.
 *  skls_profile_get(i, ...): name (static until the next enable), number of
 *      timed launches and their total milliseconds for phase i; waits for the
 *      phase's pending events.  Process-wide; not meant for concurrent use.
 */
SKLS_API int32_t skls_profile_enable(int32_t on);
SKLS_API int32_t skls_profile_count(void);
SKLS_API int32_t skls_profile_get(int32_t index, const char** name, int64_t* launches, double* total_ms);

/*
 * Multiple-response regression min_Y ||A Y - B||_F by leverage-score sampling
 * (Section 7, theorem on the generalized-regression algorithm):
 *  1. leverage scores of A to constant relative error (Section 6 theorem):
 *     R1 from the float64 Gram of S1 A for the sparse embedding S1 with t rows
 *     (stream `seed`, as skls_sketch), scores = squared row norms of
 *     A R1^{-1} Pi2 with Pi2 the d x k_g sign matrix / sqrt(k_g) of
 *     skls_low_rank (stream seed ^ 0x6C65766572616765), float64 throughout;
 *  2. t_s draws with replacement with probabilities proportional to the
 *     scores (uniforms and the rule of skls_low_rank, stream
 *     seed ^ 0x73616D706C696E67); a row drawn c times enters once with weight
 *     sqrt(c / (t_s p)) -- the coreset;
 *  3. Y = R^{-1} Q^T (S B) for S A = Q R.
 * Synchronous.
 */
typedef struct {
  int64_t t;          /* rows of S1 (d <= t < 2^31) */
  int64_t t_s;        /* draws of the sampling (d <= t_s < 2^31) */
  uint64_t seed;
  int32_t k_g;        /* columns of Pi2 (0: 32; at most 64) */
  int32_t reserved[5];
} skls_multi_opts;

typedef struct {
  int64_t rows_sampled;  /* distinct rows in the coreset */
  double resid_fro;      /* ||A Y - B||_F (float64 accumulation) */
  double b_fro;          /* ||B||_F */
  float ms_scores, ms_solve;
  int32_t reserved[4];
} skls_multi_info;

SKLS_API int32_t skls_multi_lstsq_workspace(const skls_matrix* A, int64_t dp, const skls_multi_opts* opts,
                                            size_t* bytes);
/*
 *  A:       dense (F64, F32, BF16) or CSR, n x d, d <= 8192.
 *  B:       device float64 n x dp row-major, 1 <= dp <= 64.
 *  Y:       device float64 d x dp row-major.
 *  rows:    device int32 [min(n, t_s)] or NULL: the coreset's rows in
 *           increasing order (the first info->rows_sampled entries).
 *  weights: device float64 [min(n, t_s)] or NULL: their weights.
 * Errors: SKLS_ERR_RANK when S1 A or S A is numerically rank deficient.
 */
SKLS_API int32_t skls_multi_lstsq(const skls_matrix* A, const double* B, int64_t dp, const skls_multi_opts* opts,
                                  double* Y, int32_t* rows, double* weights, skls_multi_info* info, void* ws,
                                  size_t ws_bytes, void* stream);

/*
 * l_p regression min_x ||A x - b||_p for 1 <= p < inf (Section 9: the
 * conditioning step on generalized sparse embeddings, then two-stage row
 * sampling as in the l_p coreset algorithm of Dasgupta, Drineas, Harb, Kumar
 * and Mahoney that the section builds on):
 *  1. F A for F block-diagonal: the rows of A in blocks of w, every block
 *     embedded by the same generalized sparse embedding of skls_sketch_general
 *     (q groups of v buckets, a copies, stream `seed`; rows hashed by their
 *     index inside the block; t = a q v rows per block), float64;
 *  2. R from the float64 Gram of F A (Cholesky); A R^{-1} is the conditioned
 *     basis (the l_2 basis: the section leaves the general-p construction to
 *     its reference, and an l_2 basis is well conditioned for every p up to
 *     factors polynomial in the dimensions, which only the sample sizes feel);
 *  3. lam_i = (squared row norm of A R^{-1} Pi2)^{p/2}, Pi2 the d x k_g sign
 *     matrix / sqrt(k_g) of skls_low_rank (stream seed ^ 0x6C65766572616765):
 *     the l_p row norms of the basis estimated through l_2 norms;
 *  4. stage 1: row i kept iff u_i < pi_i = min(1, s1 lam_i / sum(lam)), u_i =
 *     (z_i >> 11) 2^-53 for output i of the stream seed ^ 0x73616D706C696E67,
 *     with weight pi_i^{-1/p}; x_c = the weighted l_p fit of the kept rows;
 *  5. stage 2: rho = A x_c - b; row i kept iff u'_i < min(1, s2 max(lam_i /
 *     sum(lam), |rho_i|^p / sum |rho|^p)) (u' from the stream
 *     seed ^ 0x726573616D706C65; the residual share is left out when rho = 0),
 *     with weight q_i^{-1/p}; x = the weighted l_p fit of those rows.
 * The weighted fits (min sum_i w_i^p |A_i x - b_i|^p over the kept rows) run
 * on the float64 coreset: p = 2 through the normal equations, p = 1 by a
 * primal-dual interior-point method on the dual linear program (stops when
 * the duality gap is at most tol * max(1, objective)), other p by iteratively
 * reweighted least squares (weights max(|r_i|, eta)^(p-2), with eta starting
 * at the mean |r| and shrinking 4x per step to 1e-9 of it; Newton steps
 * 1/(p-1) long with halving for p > 2; stops once eta is at its floor and the
 * objective changes by at most tol relative).  Every
 * fit starts from the least-squares solution of the kept rows and stops there
 * when its residuals are at rounding level (sum |r| <= 16 d 2^-53 sum |b| over
 * the kept rows): that solves a consistent system, which is optimal for every p.
 * Synchronous.
 */
typedef struct {
  double p;           /* 1 <= p < inf */
  int64_t q, v;       /* embedding groups and buckets per group (0: v = 8, q = max(16, ceil(2 d^2 / v))) */
  int32_t a;          /* copies of the embedding (0: 1; at most 256) */
  int32_t k_g;        /* columns of Pi2 (0: 32; at most 64) */
  int64_t w;          /* rows per block of F (0 or >= n: one block) */
  double s1, s2;      /* expected sample sizes of the two stages (0: 32 d each) */
  uint64_t seed;
  int32_t max_iter;   /* iterations of each weighted fit (0: 100) */
  int32_t reserved0;
  double tol;         /* stopping tolerance of the weighted fits (0: 1e-12) */
  int64_t reserved[4];
} skls_lp_opts;

typedef struct {
  int64_t rows_stage1, rows_stage2;  /* rows kept by the two draws */
  int32_t iters_stage1, iters_stage2;  /* weighted solves (factorizations) of each fit, the start included */
  int32_t converged;     /* 1 if both fits met their stopping rule */
  int32_t reserved0;
  double obj_stage1;     /* ||A x_c - b||_p^p (float64 accumulation) */
  double obj;            /* ||A x - b||_p^p */
  double coreset_obj;    /* stage-2 weighted objective at x */
  float ms_condition, ms_stage1, ms_stage2;
  int32_t reserved1;
  int64_t reserved[4];
} skls_lp_info;

SKLS_API int32_t skls_lp_regression_workspace(const skls_matrix* A, const skls_lp_opts* opts, size_t* bytes);
/*
 *  A:      dense (F64, F32, BF16) or CSR, n x d, d <= n < 2^31, d <= 4096
 *          (the residual passes further limit dense d to 512, or to 1024 /
 *          2048 / 4096 for F64 / F32 / BF16 rows whose length and start are
 *          multiples of 16 bytes).
 *  b:      device float64 [n].
 *  x:      device float64 [d], the result.
 *  x_c:    device float64 [d] or NULL: the stage-1 solution.
 *  rows1, w1, rows2, w2: device int32 / float64 arrays of at least n entries,
 *          or NULL: the kept rows of each stage in increasing order and their
 *          weights (the first info->rows_stage1 / rows_stage2 entries).
 * Errors: SKLS_ERR_ARG for p outside [1, inf); SKLS_ERR_RANK when F A is
 * numerically rank deficient or a stage keeps fewer than d rows or a rank
 * deficient set; SKLS_ERR_SHAPE when a stage keeps more rows than its
 * capacity (s + 8 sqrt(s) + 64, with s = s1 and 2 s2; not reached in
 * practice).
 */
SKLS_API int32_t skls_lp_regression(const skls_matrix* A, const double* b, const skls_lp_opts* opts, double* x,
                                    double* x_c, int32_t* rows1, double* w1, int32_t* rows2, double* w2,
                                    skls_lp_info* info, void* ws, size_t ws_bytes, void* stream);

/*
 * Rank-k approximation A ~ L diag(D) W^T (Section 8, theorem on low-rank
 * approximation), in the simplified form of the Section 10 experiments:
 *  1. Y = A R^T for R^ a t_r x m sparse embedding of the columns of A (h and
 *     the signs from the SplitMix64 stream `seed`, as for the rows in
 *     skls_sketch); U = an orthonormal basis of the column space of Y;
 *  2. S: t_s rows of the n drawn independently with replacement with
 *     probabilities proportional to the leverage scores of Y (Section 6: the
 *     squared row norms of Y R_Y^{-1} Pi2, R_Y the triangular factor of Y and
 *     Pi2 a t_r x k_g matrix of signs / sqrt(k_g), bit 0 of outputs
 *     r * k_g + c of the stream seed ^ 0x6C65766572616765), each drawn row
 *     scaled by 1 / sqrt(t_s p); draw j takes u_j = (z_j >> 11) * 2^-53 from
 *     output j of the stream seed ^ 0x73616D706C696E67 and picks the first
 *     row whose running score sum exceeds u_j times the total;
 *  3. S U = U~ S~ V~^T;  4. the best rank-k approximation [U~^T S A]_k and
 *     the SVD U^ D W^T of V~ S~^{-1} [U~^T S A]_k;  5. L = U U^.
 * The library evaluates these through equivalent QR-based factorisations and
 * finds [U~^T S A]_k by block subspace iteration with k + oversample columns,
 * stopped when the top-k Ritz values change by at most tol relative.
 * Synchronous (returns after the stream has finished the call).
 */
typedef struct {
  int64_t k;           /* target rank, 1 <= k <= 48 and k <= min(n, m) */
  int64_t t_r;         /* columns of R^; 0: ceil(k / eps), then at least k + oversample, at most min(m, 2048) */
  int64_t t_s;         /* draws of the sampling; 0: 64 * t_r */
  uint64_t seed;
  double eps;          /* accuracy parameter that sets the default t_r (0 < eps <= 1) */
  int32_t k_g;         /* columns of Pi2 (0: 32; at most 64) */
  int32_t oversample;  /* extra columns of the subspace iteration (0: 16); k + oversample <= 64 */
  int32_t max_iter;    /* subspace iterations (0: 60) */
  double tol;          /* relative change of the top-k Ritz values that ends the iteration (0: 1e-13) */
  int32_t reserved[4];
} skls_low_rank_opts;

typedef struct {
  int64_t t_r, t_s;       /* sizes used */
  int64_t rows_sampled;   /* distinct rows of A drawn by S */
  int64_t nnz_sampled;    /* their nonzeros (CSR) */
  int32_t iterations;     /* subspace iterations run */
  int32_t converged;      /* 1 when the Ritz values settled within max_iter */
  double resid_fro;       /* ||A - L diag(D) W^T||_F (float64 accumulation) */
  double fro_norm;        /* ||A||_F */
  float ms_sketch, ms_sample, ms_topk, ms_factors;
  int32_t reserved[4];
} skls_low_rank_info;

/*
 * Workspace of skls_low_rank for this matrix and these options (bytes).
 * Returns SKLS_ERR_ARG / SKLS_ERR_SHAPE for options the call would reject.
 */
SKLS_API int32_t skls_low_rank_workspace(const skls_matrix* A, const skls_low_rank_opts* opts, size_t* bytes);

/*
 *  A:      dense (F64, F32 or BF16) or CSR, n x m, n >= 1, m >= 1.
 *  L:      device float64 n x k row-major, orthonormal columns.
 *  D:      device float64 [k], decreasing, >= 0.
 *  W:      device float64 m x k row-major, orthonormal columns.
 *  info:   host, or NULL.
 * Errors: SKLS_ERR_RANK when Y or S U is numerically rank deficient (lower
 * t_r or raise t_s); SKLS_ERR_WORKSPACE when ws_bytes is below the query.
 * Columns of L and W that belong to zero values of D are zero.
 */
SKLS_API int32_t skls_low_rank(const skls_matrix* A, const skls_low_rank_opts* opts, double* L, double* D, double* W,
                               skls_low_rank_info* info, void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SKLS_H */
