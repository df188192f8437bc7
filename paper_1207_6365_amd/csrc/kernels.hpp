// Internal launchers shared by the C ABI (api.cpp) and the kernel sources.
#pragma once

#include "common.hpp"

namespace skls {

// ---------------------------------------------------------------- sketch.hip
int32_t launch_hash(int64_t n, uint32_t t, uint64_t seed, int64_t start, int32_t* bucket, int8_t* sign,
                    hipStream_t s);
int32_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
// p[i] *= alpha for count elements of type dtype (F64 or F32).
int32_t launch_scale(void* p, size_t count, int32_t dtype, double alpha, hipStream_t s);

// Sketch variant the library runs for this input (SKLS_SKETCH_AUTO resolved).
int32_t choose_sketch_variant(const skls_matrix& A, int64_t t, int32_t variant, int32_t out_dtype);
size_t sketch_ws_bytes(const skls_matrix& A, int64_t t, int32_t variant);
int32_t run_sketch(const skls_matrix& A, const void* b, int32_t b_dtype, int64_t t, uint64_t seed,
                   const float* w, int32_t variant, void* SA, void* Sb, int32_t out_dtype, void* ws,
                   size_t ws_bytes, hipStream_t s);
// The same with the hash given by a key (plain or one copy of a generalized
// sparse embedding).
int32_t run_sketch_key(const skls_matrix& A, const void* b, int32_t b_dtype, int64_t t, HashKey key,
                       const float* w, int32_t variant, void* SA, void* Sb, int32_t out_dtype, void* ws,
                       size_t ws_bytes, hipStream_t s);
int32_t launch_hash_key(int64_t n, uint32_t t, HashKey key, int64_t start, int32_t* bucket, int8_t* sign,
                        hipStream_t s);
// Reusable bucket plans: bytes of the device buffer, building it (without b
// and w), and the reduce with it.  `resolved` is the variant that ran
// (AUTO resolved); the apply needs the same A shape, t, key, variant and
// output type.
size_t sketch_plan_bytes(const skls_matrix& A, int64_t t, int32_t variant, int32_t out_dtype);
int32_t build_sketch_plan(const skls_matrix& A, int64_t t, HashKey key, int32_t variant, int32_t out_dtype,
                          void* plan, size_t plan_bytes, int32_t* resolved, hipStream_t s);
int32_t apply_sketch_plan(const skls_matrix& A, const void* b, int32_t b_dtype, int64_t t, HashKey key,
                          const float* w, int32_t resolved, void* SA, void* Sb, int32_t out_dtype, const void* plan,
                          size_t plan_bytes, hipStream_t s);
// The bucket order of a dense SORTED plan: off[t + 1] (bucket offsets into
// perm) and perm[n] (row ids in bucket order).  Both NULL when the plan is of
// another variant or layout.
int32_t sorted_plan_order(const skls_matrix& A, int64_t t, int32_t resolved, int32_t out_dtype, const void* plan,
                          size_t plan_bytes, const int32_t** off, const int32_t** perm);
// The apply of a dense SORTED plan (float32 output, no b) to up to
// kSortedMany dense float32 matrices of one shape in one launch: matrix j's
// sketch goes to SA + j * sa_stride.
constexpr int kSortedMany = 16;
int32_t apply_sorted_many(const skls_matrix* A, int count, int64_t t, HashKey key, const float* w, const void* plan,
                          size_t plan_bytes, float* SA, int64_t sa_stride, hipStream_t s);
// Argument checks shared by the sketch entry points (api.cpp).
int32_t check_sketch_args(const skls_matrix* A, const void* b, int32_t b_dtype, int64_t t, int32_t variant,
                          const void* SA, const void* Sb, int32_t out_dtype);

// ---------------------------------------------------------------- dense.hip
// Gram of the augmented matrix [M | v] (m x dd, dd = d or d+1), float64.
size_t gram_ws_bytes(int64_t m, int64_t dd);
int32_t run_gram(const void* M, int32_t dtype, int64_t ld, const void* v, int32_t v_dtype, int64_t m, int64_t d,
                 double* G /* dd x dd */, void* ws, size_t ws_bytes, hipStream_t s);
// The row splits of M^T M for d <= 64 (no v), at most max_splits (<= 256) of
// whole 64-row chunks, without their sum: split k at partial + k * pitch *
// pitch, entry (i, j), i <= j < d, at i * pitch + j.  ws as for run_gram
// (gram_ws_bytes(m, d) bytes); *splits = their number.
int32_t run_gram_small_partials(const void* M, int32_t dtype, int64_t ld, int64_t m, int64_t d, int max_splits,
                                void* ws, size_t ws_bytes, int* splits, int* pitch, hipStream_t s);
// The same for `count` float32 matrices of one shape (m x d, leading dimension
// d) at M + j * mstride, their splits at partial + j * pstride (at least
// max_splits * gram_small_split_doubles() doubles apart), in one launch.
int64_t gram_small_split_doubles();
int32_t run_gram_small_partials_many(const float* M, int count, int64_t mstride, int64_t m, int64_t d,
                                     int max_splits, double* partial, int64_t pstride, int* splits, int* pitch,
                                     hipStream_t s);
// Cholesky of the leading d x d block of G (leading dimension ldg): R upper,
// status[0] = 0 ok / 1 rank deficient.  With Rinv and RinvT (d x d each, or
// both NULL) it also forms R^{-1} and R^{-T} within the same launches.
int32_t run_cholesky(const double* G, int64_t ldg, int64_t d, double* R, double* Rinv, double* RinvT,
                     int32_t* status, double* scratch, hipStream_t s);
size_t cholesky_scratch_doubles(int64_t d);
// The inverses of R's diagonal 64 x 64 blocks that run_cholesky leaves in its
// scratch (block J at J * 64^2, ld 64), valid until the scratch is reused.
const double* cholesky_block_inverses(const double* scratch, int64_t d);
// R^{-1} (and its transpose); diag_inv: the block inverses of this R kept by
// run_cholesky, or NULL to compute them.
int32_t run_trinv(const double* R, int64_t d, double* Rinv, double* RinvT, hipStream_t s,
                  const double* diag_inv = nullptr);
// y = op(M) x for a d x d row-major float64 M (op = identity).
int32_t run_gemv(const double* M, int64_t d, const double* x, double* y, hipStream_t s);
// x = Rinv (RinvT c): sketch-and-solve from the Gram column c = M^T v.
// T = Rinv P (d x k), float32 result.
int32_t run_rinv_times(const double* Rinv, int64_t d, const double* P, int32_t k, float* T, hipStream_t s);
// Pi2 (rows x kg, row-major) = signs / sqrt(kg), sign of entry e from bit 0
// of output e of the stream seed ^ "leverage" (the projection of the
// Section 6 estimates used by every sampling path).
int32_t run_sign_projection(int64_t rows, int32_t kg, uint64_t seed, double* Pi2, hipStream_t s);
int32_t run_solve_from_gram(const double* Rinv, const double* RinvT, const double* c, int64_t d, double* x,
                            double* tmp, hipStream_t s);

// ---------------------------------------------------------------- stage2.hip
// FSA = F SA, FSb = F Sb (Sb may be NULL) for the m x t sign matrix F of the
// second sketch stage; scratch holds second_stage_scratch_floats floats.
size_t second_stage_scratch_floats(int64_t m, int64_t d, int64_t t);
int32_t run_second_stage(const void* SA, const void* Sb, int32_t dtype, int64_t t, int64_t d, int64_t m,
                         uint64_t seed, double* FSA, double* FSb, float* scratch, hipStream_t s);

// ---------------------------------------------------------------- lsqr.hip
// One pass over A: U_new[i] = A[i,:] p + coef * Z[i]; partial sums of
// ||U_new||^2 and A^T U_new per block.  Precision: TA = float or double.
struct PassArgs {
  const skls_matrix* A;
  const double* p;      // [d] (float64, converted on load)
  const double* coef;   // device scalar
  const void* Z;        // [n]: U (same type as U) or b (float64)
  int32_t z_is_b;       // 1: Z is float64 b, 0: Z is U
  void* U;              // [n], float64 or float32 (u_f64)
  int32_t u_f64;
  int32_t acc_f64;      // accumulate in float64
  double* partial;      // [nblk][d+1]
  int32_t nblk;
};
int32_t pass_blocks(const skls_matrix& A);
int32_t run_pass(const PassArgs& a, hipStream_t s);
// Sum partial[nblk][d+1] into out[d+1].
int32_t run_reduce_partials(const double* partial, int32_t nblk, int64_t d, double* out, double* tmp,
                            hipStream_t s);

// Device LSQR state (float64 slots).
enum {
  LSQR_ALPHA = 0,
  LSQR_BETA,
  LSQR_RHOBAR,
  LSQR_PHIBAR,
  LSQR_COEF,
  LSQR_RNORM,
  LSQR_ARNORM,
  LSQR_EST_R,
  LSQR_EST_AR,
  LSQR_ONE,
  LSQR_DONE,
  LSQR_STOP,   // 1 once a step met the inner target (later steps leave the state alone)
  LSQR_COUNT,  // steps taken since the last init
  LSQR_NSTATE
};
// The init and the steps also copy the state into `mirror` (device address
// of pinned host memory from lsqr_mirror, or NULL); the init adds *flag and
// *extra after it (mirror[LSQR_NSTATE], mirror[LSQR_NSTATE + 1]; 0 for NULL).
int32_t run_lsqr_init(const double* gsum, const double* vp, int64_t d, double* v, double* w, double* y, double* st,
                      hipStream_t s, double* mirror = nullptr, const int32_t* flag = nullptr,
                      const double* extra = nullptr);
// One step; it is skipped (state unchanged) once st[LSQR_STOP] is set, and
// sets it when the recurrence ends or est_ar <= target * est_r.
int32_t run_lsqr_step(const double* gsum, const double* vp, int64_t d, double* v, double* w, double* y, double* st,
                      double target, hipStream_t s, double* mirror = nullptr);
// LSQR_NSTATE + 2 doubles of pinned, coherent host memory per host thread
// (allocated on first use): its host and device addresses.
int32_t lsqr_mirror(double** host, double** dev);
// y = a * x (d-vectors), and *one = 1 when one is not NULL; x += t.
int32_t run_scale(const double* x, int64_t d, double a, double* y, hipStream_t s, double* one = nullptr);
int32_t run_add(double* x, const double* t, int64_t d, hipStream_t s);

// ---------------------------------------------------------------- leverage.hip
int32_t run_leverage(const skls_matrix& A, const float* T, int32_t k, float* scores, hipStream_t s);

// ---------------------------------------------------------------- learned.hip
int32_t run_learned_E(const double* P, int64_t ldp, const float* C, int64_t d, float* E, float* loss,
                      hipStream_t s);
int32_t run_learned_G(const float* Y, const float* E, int64_t t, int64_t d, float* G, hipStream_t s);
int32_t run_learned_gather(const skls_matrix& A, const float* G, uint32_t t, uint64_t seed, float scale,
                           bool accumulate, float* grad, hipStream_t s);
// Loss and E from the small-Gram splits (run_gram_small_partials), one block.
int32_t run_learned_PE(const double* partial, int S, int pitch, const float* C, int64_t d, float* E, float* loss,
                       hipStream_t s);
// G = 4 Y E and the gradient gather in one launch, from the bucket order of a
// dense SORTED plan (sorted_plan_order); d <= 64.
int32_t run_learned_G_gather(const float* Y, const float* E, int64_t t, const int32_t* off, const int32_t* perm,
                             const skls_matrix& A, float scale, bool accumulate, float* grad, hipStream_t s);
// Per-matrix arguments of the learned kernels that take several matrices of
// one shape at once (up to kSortedMany).
struct LearnedMany {
  const float* A[kSortedMany];
  int64_t ld[kSortedMany];
  const float* C[kSortedMany];
  float scale[kSortedMany];
};
// Loss and E of each of `count` matrices from its small-Gram splits (block j:
// splits at partial + j * pstride, E + j d^2, loss[j]).
int32_t run_learned_PE_many(const double* partial, int64_t pstride, int S, int pitch, const LearnedMany& args,
                            int count, int64_t d, float* E, float* loss, hipStream_t s);
// 4 Y E and the gather for each of `count` matrices (sketch at Y + j * ystride,
// E + j d^2), matrix j's weighted gradient written to grad + j * gstride;
// vec: every A is 16-byte aligned with ld and d multiples of 4.
int32_t run_learned_G_gather_many(const float* Y, int64_t ystride, const float* E, int64_t t, int64_t d,
                                  const int32_t* off, const int32_t* perm, const LearnedMany& args, int count,
                                  bool vec, float* grad, int64_t gstride, hipStream_t s);
int32_t run_sum_slots(int64_t n, const float* slots, int64_t stride, int k, float scale, bool accumulate,
                      float* grad, hipStream_t s);
int32_t run_adam(int64_t n, float* w, const float* g, float* m, float* v, int32_t step, float lr, float b1,
                 float b2, float eps, hipStream_t s);
int32_t run_convert_f64_to_f32(const double* in, float* out, int64_t count, hipStream_t s);

// ---------------------------------------------------------------- lowrank.hip
// Resolved sizes of a rank-k approximation (options checked and defaulted).
struct LowRankPlan {
  int64_t n, m, k, tr, ts, nsmax, nnzmax;
  int p, kg, max_iter;
  double tol;
  bool csr;
};
int32_t low_rank_plan(const skls_matrix& A, const skls_low_rank_opts& o, LowRankPlan& P);
size_t low_rank_ws_bytes(const LowRankPlan& P);
int32_t run_low_rank(const skls_matrix& A, const LowRankPlan& P, uint64_t seed, double* L, double* D, double* W,
                     skls_low_rank_info* info, void* ws, size_t ws_bytes, hipStream_t s);

// ---------------------------------------------------------------- regress.hip
struct MultiPlan {
  int64_t n, d, dp, t, ts, nsmax;
  int kg;
  size_t sk_bytes;
};
int32_t multi_plan(const skls_matrix& A, int64_t dp, const skls_multi_opts& o, MultiPlan& P);
size_t multi_ws_bytes(const MultiPlan& P);
int32_t run_multi_lstsq(const skls_matrix& A, const double* B, const MultiPlan& P, uint64_t seed, double* Y,
                        int32_t* rows_out, double* weights_out, skls_multi_info* info, void* ws, size_t ws_bytes,
                        hipStream_t s);

// ---------------------------------------------------------------- lp.hip
// Resolved sizes of an l_p regression (options checked and defaulted).
struct LpPlan {
  const skls_matrix* A;
  int64_t n, d, q, v, w, nb, t, cap;
  int32_t a, kg, max_iter;
  double p, s1, s2, tol;
  uint64_t seed;
  size_t sk_bytes;
};
int32_t lp_plan(const skls_matrix& A, const skls_lp_opts& o, LpPlan& P);
size_t lp_ws_bytes(const LpPlan& P);
int32_t run_lp(const skls_matrix& A, const double* b, const LpPlan& P, double* x, double* x_c, int32_t* rows1,
               double* w1, int32_t* rows2, double* w2, skls_lp_info* info, void* ws, size_t ws_bytes,
               hipStream_t s);
}  // namespace skls
