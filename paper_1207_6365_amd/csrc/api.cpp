// C ABI of libskls: argument validation, workspace layout and the order of
// kernel launches for each entry point.  Declarations and contracts are in
// include/skls.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "kernels.hpp"

namespace skls {

namespace {
thread_local char g_err[768] = "";
}

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}
void clear_error() { g_err[0] = '\0'; }
const char* last_error() { return g_err; }

int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

size_t dtype_size(int32_t dt) {
  switch (dt) {
    case SKLS_F64: return 8;
    case SKLS_F32: return 4;
    case SKLS_BF16: return 2;
    default: return 0;
  }
}

int32_t validate_matrix(const skls_matrix* A, bool allow_bf16) {
  if (A == nullptr) {
    set_error("matrix descriptor is NULL");
    return SKLS_ERR_ARG;
  }
  if (A->layout != SKLS_DENSE && A->layout != SKLS_CSR) {
    set_error("unknown layout %d", A->layout);
    return SKLS_ERR_ARG;
  }
  if (dtype_size(A->dtype) == 0 || (!allow_bf16 && A->dtype == SKLS_BF16)) {
    set_error("unsupported matrix dtype %d", A->dtype);
    return SKLS_ERR_DTYPE;
  }
  if (A->n < 0 || A->d < 1 || A->n >= (int64_t(1) << 31) || A->d >= (int64_t(1) << 31)) {
    set_error("matrix shape n=%lld d=%lld out of range (need 0 <= n < 2^31, 1 <= d < 2^31)",
              static_cast<long long>(A->n), static_cast<long long>(A->d));
    return SKLS_ERR_SHAPE;
  }
  if (A->layout == SKLS_DENSE) {
    if (A->ld < A->d) {
      set_error("dense leading dimension %lld < d %lld", static_cast<long long>(A->ld), static_cast<long long>(A->d));
      return SKLS_ERR_SHAPE;
    }
    if (A->n > 0 && A->val == nullptr) {
      set_error("dense values pointer is NULL");
      return SKLS_ERR_ARG;
    }
  } else {
    if (A->row_ptr == nullptr) {
      set_error("CSR row_ptr is NULL");
      return SKLS_ERR_ARG;
    }
    if (A->nnz < 0 || (!A->row_ptr_64 && A->nnz >= (int64_t(1) << 31))) {
      set_error("CSR nnz %lld out of range for the row pointer type", static_cast<long long>(A->nnz));
      return SKLS_ERR_SHAPE;
    }
    if (A->nnz > 0 && (A->col_idx == nullptr || A->val == nullptr)) {
      set_error("CSR col_idx or val is NULL");
      return SKLS_ERR_ARG;
    }
  }
  return SKLS_OK;
}

namespace {

int32_t check_t(int64_t t) {
  if (t < 1 || t >= (int64_t(1) << 31)) {
    set_error("t=%lld out of range [1, 2^31)", static_cast<long long>(t));
    return SKLS_ERR_SHAPE;
  }
  return SKLS_OK;
}

int32_t need_ws(const Arena& ar, const void* ws, size_t ws_bytes) {
  if (ar.used > 0 && (ws == nullptr || ws_bytes < ar.used)) {
    set_error("workspace too small: need %zu bytes, have %zu", ar.used, ws == nullptr ? size_t(0) : ws_bytes);
    return SKLS_ERR_WORKSPACE;
  }
  return SKLS_OK;
}

int32_t read_status(const int32_t* dstatus, hipStream_t s, int32_t* out) {
  SKLS_TRY_HIP(hipMemcpyAsync(out, dstatus, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  SKLS_TRY_HIP(hipStreamSynchronize(s));
  return SKLS_OK;
}

// ---------------------------------------------------------------- R of a tall matrix
struct QrWs {
  double* gram;
  size_t gram_bytes;
  double* G;
  double* W;
  int32_t* status;
  double* RinvT;
};

QrWs carve_qr(Arena& ar, int64_t m, int64_t d, int64_t dd) {
  QrWs q;
  q.gram_bytes = gram_ws_bytes(m, dd);
  q.gram = ar.take<double>(q.gram_bytes / sizeof(double) + 1);
  q.G = ar.take<double>(static_cast<size_t>(dd * dd));
  q.W = ar.take<double>(cholesky_scratch_doubles(d));
  q.status = ar.take<int32_t>(4);
  q.RinvT = ar.take<double>(static_cast<size_t>(d * d));
  return q;
}

// Gram -> Cholesky -> inverse.  G holds (M | v)^T (M | v) afterwards.
int32_t qr_from(const void* M, int32_t dtype, const void* v, int32_t v_dtype, int64_t m, int64_t d, const QrWs& q,
                double* R, double* Rinv, double* RinvT, hipStream_t s) {
  const int64_t dd = d + (v ? 1 : 0);
  SKLS_TRY(run_gram(M, dtype, d, v, v_dtype, m, d, q.G, q.gram, q.gram_bytes, s));
  SKLS_TRY(run_cholesky(q.G, dd, d, R, Rinv, Rinv ? RinvT : nullptr, q.status, q.W, s));
  return SKLS_OK;
}

// ---------------------------------------------------------------- lstsq workspace
struct LsWs {
  void* SA;
  void* Sb;
  void* sk;
  size_t sk_bytes;
  QrWs q;
  double* R;
  double* Rinv;
  double* tmp;
  double* vp;
  double* v;
  double* w;
  double* y;
  double* p;
  double* gsum;
  double* st;
  void* U;
  double* partial;
  double* red;
  int32_t nblk;
  double* FSA;   // second stage: F S A [m x d], F S b [m], split partials
  double* FSb;
  float* fpart;
};

LsWs carve_ls(Arena& ar, const skls_matrix& A, const skls_lstsq_opts& o) {
  LsWs L;
  const bool plain = o.precision == 0;
  const size_t es = plain ? 8 : 4;
  const int64_t t = o.t, d = A.d, dd = d + 1;
  L.SA = ar.take<char>(static_cast<size_t>(t * d) * es);
  L.Sb = ar.take<char>(static_cast<size_t>(t) * es);
  L.sk_bytes = sketch_ws_bytes(A, t, o.variant);
  L.sk = ar.take<char>(L.sk_bytes);
  const int64_t m = o.second_stage;
  L.q = carve_qr(ar, m > 0 ? m : t, d, dd);
  L.FSA = L.FSb = nullptr;
  L.fpart = nullptr;
  if (m > 0) {
    L.FSA = ar.take<double>(static_cast<size_t>(m * d));
    L.FSb = ar.take<double>(static_cast<size_t>(m));
    L.fpart = ar.take<float>(second_stage_scratch_floats(m, d, t));
  }
  L.R = ar.take<double>(static_cast<size_t>(d * d));
  L.Rinv = ar.take<double>(static_cast<size_t>(d * d));
  L.tmp = ar.take<double>(static_cast<size_t>(d));
  L.vp = ar.take<double>(static_cast<size_t>(d));
  L.v = ar.take<double>(static_cast<size_t>(d));
  L.w = ar.take<double>(static_cast<size_t>(d));
  L.y = ar.take<double>(static_cast<size_t>(d));
  L.p = ar.take<double>(static_cast<size_t>(d));
  L.gsum = ar.take<double>(static_cast<size_t>(dd));
  L.st = ar.take<double>(LSQR_NSTATE);
  L.U = ar.take<char>(static_cast<size_t>(A.n) * es);
  L.nblk = pass_blocks(A);
  L.partial = ar.take<double>(static_cast<size_t>(L.nblk) * dd);
  L.red = ar.take<double>(static_cast<size_t>(div_up(L.nblk, 32)) * dd);
  return L;
}

// ---------------------------------------------------------------- leverage workspace
struct LevWs {
  int32_t sk_dtype;
  void* SA;
  void* sk;
  size_t sk_bytes;
  QrWs q;
  double* R;
  double* Rinv;
  double* Pi2;  // generated projection (used when the caller passes none)
  float* T;
};

LevWs carve_lev(Arena& ar, const skls_matrix& A, int64_t t, int32_t k) {
  LevWs L;
  const int64_t d = A.d;
  L.sk_dtype = A.dtype == SKLS_F64 ? SKLS_F64 : SKLS_F32;
  const size_t es = L.sk_dtype == SKLS_F64 ? 8 : 4;
  L.SA = ar.take<char>(static_cast<size_t>(t * d) * es);
  L.sk_bytes = sketch_ws_bytes(A, t, SKLS_SKETCH_AUTO);
  L.sk = ar.take<char>(L.sk_bytes);
  L.q = carve_qr(ar, t, d, d);
  L.R = ar.take<double>(static_cast<size_t>(d * d));
  L.Rinv = ar.take<double>(static_cast<size_t>(d * d));
  L.Pi2 = ar.take<double>(static_cast<size_t>(d) * k);
  L.T = ar.take<float>(static_cast<size_t>(d) * k);
  return L;
}

// Workspace of the leverage scores from a given R: R^{-1}, its transpose
// (product scratch of the inverse), the projection and T = R^{-1} Pi2.
struct LevRWs {
  double* Rinv;
  double* RinvT;
  double* Pi2;
  float* T;
};

LevRWs carve_lev_r(Arena& ar, int64_t d, int32_t k) {
  LevRWs L;
  L.Rinv = ar.take<double>(static_cast<size_t>(d * d));
  L.RinvT = ar.take<double>(static_cast<size_t>(d * d));
  L.Pi2 = ar.take<double>(static_cast<size_t>(d) * k);
  L.T = ar.take<float>(static_cast<size_t>(d) * k);
  return L;
}

constexpr int32_t kMaxStageRows = 65536;

void fill_opts(skls_lstsq_opts& o) {
  if (o.delta <= 0.0) o.delta = 1e-6;
  if (o.sigma_lb <= 0.0) o.sigma_lb = 0.5;
  if (o.max_iter <= 0) o.max_iter = 100;
}

int32_t check_lstsq(const skls_matrix* A, const skls_lstsq_opts* opts) {
  SKLS_TRY(validate_matrix(A, true));
  if (opts == nullptr) {
    set_error("options pointer is NULL");
    return SKLS_ERR_ARG;
  }
  SKLS_TRY(check_t(opts->t));
  if (opts->t < A->d) {
    set_error("sketch rows t=%lld must be at least d=%lld", static_cast<long long>(opts->t),
              static_cast<long long>(A->d));
    return SKLS_ERR_SHAPE;
  }
  if (A->n < A->d) {
    set_error("least squares needs n >= d");
    return SKLS_ERR_SHAPE;
  }
  if (opts->precision != 0 && opts->precision != 1) {
    set_error("precision must be 0 (plain) or 1 (mixed)");
    return SKLS_ERR_ARG;
  }
  if (opts->sigma_lb > 1.0 || opts->delta < 0.0) {
    set_error("need 0 < sigma_lb <= 1 and delta >= 0");
    return SKLS_ERR_ARG;
  }
  if (opts->max_retries < 0 || opts->max_retries > 64) {
    set_error("max_retries must lie in [0, 64]");
    return SKLS_ERR_ARG;
  }
  if (opts->second_stage != 0 &&
      (opts->second_stage < A->d || opts->second_stage > opts->t || opts->second_stage > kMaxStageRows)) {
    set_error("second_stage m=%d must be 0 or satisfy d <= m <= t and m <= %d", opts->second_stage, kMaxStageRows);
    return SKLS_ERR_ARG;
  }
  return SKLS_OK;
}

int32_t check_stage(int64_t t, int64_t d, int64_t m) {
  SKLS_TRY(check_t(t));
  if (d < 1 || d > 8192 || m < 1 || m > kMaxStageRows) {
    set_error("second stage needs 1 <= d <= 8192 and 1 <= m <= %d", kMaxStageRows);
    return SKLS_ERR_SHAPE;
  }
  return SKLS_OK;
}

}  // namespace

int32_t check_sketch_args(const skls_matrix* A, const void* b, int32_t b_dtype, int64_t t, int32_t variant,
                          const void* SA, const void* Sb, int32_t out_dtype) {
  SKLS_TRY(validate_matrix(A, true));
  SKLS_TRY(check_t(t));
  if (variant < SKLS_SKETCH_AUTO || variant > SKLS_SKETCH_BINNED) {
    set_error("unknown sketch variant %d", variant);
    return SKLS_ERR_ARG;
  }
  if (SA == nullptr) {
    set_error("SA is NULL");
    return SKLS_ERR_ARG;
  }
  if ((b == nullptr) != (Sb == nullptr)) {
    set_error("b and Sb must be given together");
    return SKLS_ERR_ARG;
  }
  if (b != nullptr && b_dtype != SKLS_F64 && b_dtype != SKLS_F32) {
    set_error("b must be F64 or F32");
    return SKLS_ERR_DTYPE;
  }
  if (out_dtype != SKLS_F64 && out_dtype != SKLS_F32) {
    set_error("out_dtype must be F64 or F32");
    return SKLS_ERR_DTYPE;
  }
  return SKLS_OK;
}

}  // namespace skls

using namespace skls;

extern "C" {

const char* skls_status_str(int32_t status) {
  switch (status) {
    case SKLS_OK: return "SKLS_OK";
    case SKLS_ERR_ARG: return "SKLS_ERR_ARG";
    case SKLS_ERR_SHAPE: return "SKLS_ERR_SHAPE";
    case SKLS_ERR_DTYPE: return "SKLS_ERR_DTYPE";
    case SKLS_ERR_RANK: return "SKLS_ERR_RANK";
    case SKLS_ERR_NOCONV: return "SKLS_ERR_NOCONV";
    case SKLS_ERR_WORKSPACE: return "SKLS_ERR_WORKSPACE";
    case SKLS_ERR_DEVICE: return "SKLS_ERR_DEVICE";
    case SKLS_ERR_NOTIMPL: return "SKLS_ERR_NOTIMPL";
    default: return "SKLS_ERR_UNKNOWN";
  }
}

const char* skls_last_error(void) { return skls::last_error(); }

const char* skls_version(void) { return "skls 0.1.0 gfx950"; }

int32_t skls_hash(int64_t n, int64_t t, uint64_t seed, int64_t start, int32_t* bucket, int8_t* sign, void* stream) {
  clear_error();
  SKLS_TRY(check_t(t));
  if (n < 0 || start < 0) {
    set_error("n and start must be non-negative");
    return SKLS_ERR_SHAPE;
  }
  return launch_hash(n, static_cast<uint32_t>(t), seed, start, bucket, sign, as_stream(stream));
}

int32_t skls_sketch_workspace(const skls_matrix* A, int64_t t, int32_t variant, size_t* bytes) {
  clear_error();
  SKLS_TRY(validate_matrix(A, true));
  SKLS_TRY(check_t(t));
  if (bytes == nullptr) {
    set_error("bytes pointer is NULL");
    return SKLS_ERR_ARG;
  }
  if (variant < SKLS_SKETCH_AUTO || variant > SKLS_SKETCH_BINNED) {
    set_error("unknown sketch variant %d", variant);
    return SKLS_ERR_ARG;
  }
  *bytes = sketch_ws_bytes(*A, t, variant);
  return SKLS_OK;
}

int32_t skls_sketch(const skls_matrix* A, const void* b, int32_t b_dtype, int64_t t, uint64_t seed, const float* w,
                    int32_t variant, void* SA, void* Sb, int32_t out_dtype, void* ws, size_t ws_bytes, void* stream) {
  return skls_sketch_rows(A, 0, b, b_dtype, t, seed, w, variant, SA, Sb, out_dtype, ws, ws_bytes, stream);
}

int32_t skls_sketch_rows(const skls_matrix* A, int64_t row_start, const void* b, int32_t b_dtype, int64_t t,
                         uint64_t seed, const float* w, int32_t variant, void* SA, void* Sb, int32_t out_dtype,
                         void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  SKLS_TRY(check_sketch_args(A, b, b_dtype, t, variant, SA, Sb, out_dtype));
  if (row_start < 0) {
    set_error("row_start must be non-negative");
    return SKLS_ERR_SHAPE;
  }
  const size_t need = sketch_ws_bytes(*A, t, variant);
  if (need > 0 && (ws == nullptr || ws_bytes < need)) {
    set_error("sketch workspace too small: need %zu bytes", need);
    return SKLS_ERR_WORKSPACE;
  }
  return run_sketch_key(*A, b, b_dtype, t, plain_key(seed, static_cast<uint64_t>(row_start)), w, variant, SA, Sb,
                        out_dtype, ws, ws_bytes, as_stream(stream));
}

int32_t skls_sketch_plan_workspace(const skls_matrix* A, int64_t t, int32_t variant, int32_t out_dtype,
                                   size_t* bytes) {
  clear_error();
  SKLS_TRY(validate_matrix(A, true));
  SKLS_TRY(check_t(t));
  if (bytes == nullptr || variant < SKLS_SKETCH_AUTO || variant > SKLS_SKETCH_BINNED) {
    set_error("need bytes != NULL and a known variant");
    return SKLS_ERR_ARG;
  }
  if (out_dtype != SKLS_F64 && out_dtype != SKLS_F32) {
    set_error("out_dtype must be F64 or F32");
    return SKLS_ERR_DTYPE;
  }
  *bytes = sketch_plan_bytes(*A, t, variant, out_dtype);
  return SKLS_OK;
}

int32_t skls_sketch_plan(const skls_matrix* A, int64_t row_start, int64_t t, uint64_t seed, int32_t variant,
                         int32_t out_dtype, void* plan, size_t plan_bytes, skls_sketch_plan_desc* desc,
                         void* stream) {
  clear_error();
  SKLS_TRY(validate_matrix(A, true));
  SKLS_TRY(check_t(t));
  if (desc == nullptr || variant < SKLS_SKETCH_AUTO || variant > SKLS_SKETCH_BINNED) {
    set_error("need desc != NULL and a known variant");
    return SKLS_ERR_ARG;
  }
  if (row_start < 0) {
    set_error("row_start must be non-negative");
    return SKLS_ERR_SHAPE;
  }
  if (out_dtype != SKLS_F64 && out_dtype != SKLS_F32) {
    set_error("out_dtype must be F64 or F32");
    return SKLS_ERR_DTYPE;
  }
  const size_t need = sketch_plan_bytes(*A, t, variant, out_dtype);
  if (need > 0 && (plan == nullptr || plan_bytes < need)) {
    set_error("sketch plan buffer too small: need %zu bytes", need);
    return SKLS_ERR_WORKSPACE;
  }
  int32_t resolved = 0;
  SKLS_TRY(build_sketch_plan(*A, t, plain_key(seed, static_cast<uint64_t>(row_start)), variant, out_dtype, plan,
                             plan_bytes, &resolved, as_stream(stream)));
  *desc = skls_sketch_plan_desc{};
  desc->n = A->n;
  desc->d = A->d;
  desc->t = t;
  desc->row_start = row_start;
  desc->seed = seed;
  desc->layout = A->layout;
  desc->row_ptr_64 = A->layout == SKLS_CSR ? A->row_ptr_64 : 0;
  desc->variant = resolved;
  desc->out_dtype = out_dtype;
  desc->bytes = static_cast<int64_t>(need);
  return SKLS_OK;
}

int32_t skls_sketch_planned(const skls_matrix* A, const void* b, int32_t b_dtype, const float* w, void* SA, void* Sb,
                            const skls_sketch_plan_desc* desc, const void* plan, size_t plan_bytes, void* stream) {
  clear_error();
  if (desc == nullptr) {
    set_error("desc is NULL");
    return SKLS_ERR_ARG;
  }
  SKLS_TRY(check_sketch_args(A, b, b_dtype, desc->t, desc->variant, SA, Sb, desc->out_dtype));
  if (A->n != desc->n || A->d != desc->d || A->layout != desc->layout ||
      (A->layout == SKLS_CSR && A->row_ptr_64 != desc->row_ptr_64)) {
    set_error("the matrix does not match the plan (n, d, layout or row pointer width)");
    return SKLS_ERR_SHAPE;
  }
  if (desc->bytes > 0 && (plan == nullptr || plan_bytes < static_cast<size_t>(desc->bytes))) {
    set_error("sketch plan buffer too small: need %lld bytes", static_cast<long long>(desc->bytes));
    return SKLS_ERR_WORKSPACE;
  }
  return apply_sketch_plan(*A, b, b_dtype, desc->t, plain_key(desc->seed, static_cast<uint64_t>(desc->row_start)),
                           w, desc->variant, SA, Sb, desc->out_dtype, plan, plan_bytes, as_stream(stream));
}

int32_t skls_sketch_general_workspace(const skls_matrix* A, int64_t q, int64_t v, int32_t variant, size_t* bytes) {
  clear_error();
  SKLS_TRY(validate_matrix(A, true));
  if (bytes == nullptr || q < 1 || v < 1 || q * v >= (int64_t(1) << 31)) {
    set_error("need bytes != NULL, q >= 1, v >= 1 and q v < 2^31");
    return SKLS_ERR_ARG;
  }
  if (variant < SKLS_SKETCH_AUTO || variant > SKLS_SKETCH_BINNED) {
    set_error("unknown sketch variant %d", variant);
    return SKLS_ERR_ARG;
  }
  *bytes = sketch_ws_bytes(*A, q * v, variant);
  return SKLS_OK;
}

int32_t skls_sketch_general(const skls_matrix* A, const void* b, int32_t b_dtype, int64_t q, int64_t v, int32_t a,
                            uint64_t seed, int32_t variant, void* SA, void* Sb, int32_t out_dtype, void* ws,
                            size_t ws_bytes, void* stream) {
  clear_error();
  size_t need = 0;
  SKLS_TRY(skls_sketch_general_workspace(A, q, v, variant, &need));
  if (a < 1 || a > 256 || SA == nullptr || (b == nullptr) != (Sb == nullptr)) {
    set_error("need 1 <= a <= 256, SA != NULL, and b and Sb given together");
    return SKLS_ERR_ARG;
  }
  if (b != nullptr && b_dtype != SKLS_F64 && b_dtype != SKLS_F32) {
    set_error("b must be F64 or F32");
    return SKLS_ERR_DTYPE;
  }
  if (out_dtype != SKLS_F64 && out_dtype != SKLS_F32) {
    set_error("out_dtype must be F64 or F32");
    return SKLS_ERR_DTYPE;
  }
  if (need > 0 && (ws == nullptr || ws_bytes < need)) {
    set_error("sketch workspace too small: need %zu bytes", need);
    return SKLS_ERR_WORKSPACE;
  }
  hipStream_t s = as_stream(stream);
  const int64_t tc = q * v;
  const size_t ob = out_dtype == SKLS_F64 ? 8 : 4;
  for (int32_t j = 0; j < a; ++j) {
    HashKey key;
    key.seed = seed + static_cast<uint64_t>(j + 1) * 0xD1B54A32D192ED03ull;
    key.outer = seed;
    key.q = static_cast<uint32_t>(q);
    key.v = static_cast<uint32_t>(v);
    char* sa = static_cast<char*>(SA) + static_cast<size_t>(j) * tc * A->d * ob;
    char* sb = Sb ? static_cast<char*>(Sb) + static_cast<size_t>(j) * tc * ob : nullptr;
    SKLS_TRY(run_sketch_key(*A, b, b_dtype, tc, key, nullptr, variant, sa, sb, out_dtype, ws, ws_bytes, s));
  }
  if (a > 1) {
    const double sc = 1.0 / std::sqrt(static_cast<double>(a));
    SKLS_TRY(launch_scale(SA, static_cast<size_t>(a) * tc * A->d, out_dtype, sc, s));
    if (Sb) SKLS_TRY(launch_scale(Sb, static_cast<size_t>(a) * tc, out_dtype, sc, s));
  }
  return SKLS_OK;
}

int32_t skls_qr_r_workspace(int64_t m, int64_t d, size_t* bytes) {
  clear_error();
  if (bytes == nullptr || d < 1 || m < d) {
    set_error("need bytes != NULL and m >= d >= 1");
    return SKLS_ERR_SHAPE;
  }
  Arena ar(nullptr, 0);
  carve_qr(ar, m, d, d);
  *bytes = ar.used;
  return SKLS_OK;
}

int32_t skls_qr_r(const void* M, int32_t dtype, int64_t m, int64_t d, double* R, double* Rinv, void* ws,
                  size_t ws_bytes, void* stream) {
  clear_error();
  if (M == nullptr || R == nullptr) {
    set_error("M and R must be non-NULL");
    return SKLS_ERR_ARG;
  }
  if (dtype != SKLS_F64 && dtype != SKLS_F32) {
    set_error("M must be F64 or F32");
    return SKLS_ERR_DTYPE;
  }
  if (d < 1 || m < d || d > 8192 || m >= (int64_t(1) << 31)) {
    set_error("need 1 <= d <= 8192 and d <= m < 2^31");
    return SKLS_ERR_SHAPE;
  }
  hipStream_t s = as_stream(stream);
  Arena ar(ws, ws_bytes);
  QrWs q = carve_qr(ar, m, d, d);
  SKLS_TRY(need_ws(ar, ws, ws_bytes));
  SKLS_TRY(qr_from(M, dtype, nullptr, SKLS_F64, m, d, q, R, Rinv, q.RinvT, s));
  int32_t st = 0;
  SKLS_TRY(read_status(q.status, s, &st));
  if (st) {
    set_error("matrix is numerically rank deficient");
    return SKLS_ERR_RANK;
  }
  return SKLS_OK;
}

int32_t skls_lstsq_workspace(const skls_matrix* A, const skls_lstsq_opts* opts, size_t* bytes) {
  clear_error();
  SKLS_TRY(check_lstsq(A, opts));
  if (bytes == nullptr) {
    set_error("bytes pointer is NULL");
    return SKLS_ERR_ARG;
  }
  skls_lstsq_opts o = *opts;
  fill_opts(o);
  Arena ar(nullptr, 0);
  carve_ls(ar, *A, o);
  *bytes = ar.used;
  return SKLS_OK;
}

namespace {

// LSQR steps enqueued between reads of the device state: about 32 MB of A
// per batch, at most 8 steps.
int lsqr_batch(const skls_matrix& A, bool plain) {
  const int64_t es = A.dtype == SKLS_F64 ? 8 : (A.dtype == SKLS_F32 ? 4 : 2);
  const int64_t bytes = A.layout == SKLS_CSR ? A.nnz * (es + 4) + A.n * 8 : A.n * A.d * es;
  const int64_t per = bytes + A.n * (plain ? 16 : 8);  // plus U read and written
  const int64_t b = per > 0 ? (int64_t(32) << 20) / per : 8;
  return static_cast<int>(b < 1 ? 1 : (b > 8 ? 8 : b));
}

// One attempt of skls_lstsq with the seed in o (options filled, workspace
// carved); inf is reset and filled.
int32_t lstsq_once(const skls_matrix* A, const double* b, const skls_lstsq_opts& o, double* x, LsWs& L,
                   skls_lstsq_info& inf, hipStream_t s) {
  const bool plain = o.precision == 0;
  const int64_t d = A->d, dd = d + 1;
  std::memset(&inf, 0, sizeof inf);
  inf.resid_norm = inf.grad_norm = inf.ratio_bound = -1.0;

  hipEvent_t ev[4];
  for (auto& e : ev) SKLS_TRY_HIP(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int k = 0; k < 4; ++k) (void)hipEventDestroy(e[k]);
    }
  } guard{ev};

  // --- sketch-and-solve (Section 7): S [A | b], R of S A, x~ = R^{-1} R^{-T} (S A)^T S b
  const int32_t sk_dtype = plain ? SKLS_F64 : SKLS_F32;
  SKLS_TRY_HIP(hipEventRecord(ev[0], s));
  SKLS_TRY(run_sketch(*A, b, SKLS_F64, o.t, o.seed, o.w, o.variant, L.SA, L.Sb, sk_dtype, L.sk, L.sk_bytes, s));
  SKLS_TRY_HIP(hipEventRecord(ev[1], s));
  if (o.second_stage > 0) {
    // Pi1 = F S (Section 6): factor F S A, x~ from F S b
    SKLS_TRY(run_second_stage(L.SA, L.Sb, sk_dtype, o.t, d, o.second_stage, o.seed, L.FSA, L.FSb, L.fpart, s));
    SKLS_TRY(qr_from(L.FSA, SKLS_F64, L.FSb, SKLS_F64, o.second_stage, d, L.q, L.R, L.Rinv, L.q.RinvT, s));
  } else {
    SKLS_TRY(qr_from(L.SA, sk_dtype, L.Sb, sk_dtype, o.t, d, L.q, L.R, L.Rinv, L.q.RinvT, s));
  }
  if (o.x0 != nullptr) {
    SKLS_TRY_HIP(hipMemcpyAsync(x, o.x0, sizeof(double) * d, hipMemcpyDeviceToDevice, s));
  } else {
    SKLS_TRY(run_solve_from_gram(L.Rinv, L.q.RinvT, L.q.G + d * dd, d, x, L.tmp, s));
  }
  SKLS_TRY_HIP(hipEventRecord(ev[2], s));
  float ms = 0.0f;
  auto qr_times = [&]() -> int32_t {
    SKLS_TRY_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
    inf.ms_sketch = ms;
    SKLS_TRY_HIP(hipEventElapsedTime(&ms, ev[1], ev[2]));
    inf.ms_qr = ms;
    return SKLS_OK;
  };
  if (o.sketch_only) {
    int32_t rank_bad = 0;
    SKLS_TRY(read_status(L.q.status, s, &rank_bad));
    SKLS_TRY(qr_times());
    if (rank_bad) {
      set_error("the sketch S A is numerically rank deficient");
      return SKLS_ERR_RANK;
    }
    return SKLS_OK;
  }
  // The rank test of R and ||S b||^2 (close to ||b||^2 for an embedding) are
  // read with the first LSQR state, one host round trip later: the work
  // enqueued meanwhile on a rank-deficient R is discarded.
  double sb_norm2 = 0.0;
  double *hm = nullptr, *dm = nullptr;  // the state mirror: host and device addresses
  SKLS_TRY(lsqr_mirror(&hm, &dm));

  // --- R-preconditioned LSQR on M = A R^{-1} (Section 7.7), with float64
  //     residual refinement.  Plain: every pass in float64.  Mixed: inner
  //     passes in float32, each outer step restarts from the float64 residual.
  const double D = (1.0 + o.delta) * (1.0 + o.delta) - 1.0;
  const double thr = o.sigma_lb * std::sqrt(D / (1.0 + D));
  double hs[LSQR_NSTATE];
  int32_t status = SKLS_ERR_NOCONV;
  PassArgs pa;
  pa.A = A;
  pa.partial = L.partial;
  pa.nblk = L.nblk;
  pa.U = L.U;
  pa.u_f64 = plain ? 1 : 0;
  int outer = 0;
  for (;;) {
    // explicit residual r = b - A x and g = R^{-T} A^T r, float64 accumulation
    // (the first pass also sets the coefficient 1 it reads; init keeps it)
    SKLS_TRY(run_scale(x, d, -1.0, L.p, s, outer == 0 ? L.st + LSQR_ONE : nullptr));
    pa.p = L.p;
    pa.coef = L.st + LSQR_ONE;
    pa.Z = b;
    pa.z_is_b = 1;
    pa.acc_f64 = 1;
    SKLS_TRY(run_pass(pa, s));
    SKLS_TRY(run_reduce_partials(L.partial, L.nblk, d, L.gsum, L.red, s));
    SKLS_TRY(run_gemv(L.q.RinvT, d, L.gsum, L.vp, s));
    SKLS_TRY(run_lsqr_init(L.gsum, L.vp, d, L.v, L.w, L.y, L.st, s, dm, outer == 0 ? L.q.status : nullptr,
                           outer == 0 ? L.q.G + d * dd + d : nullptr));
    SKLS_TRY_HIP(hipStreamSynchronize(s));
    std::memcpy(hs, hm, sizeof hs);
    if (outer == 0) {
      sb_norm2 = hm[LSQR_NSTATE + 1];
      SKLS_TRY(qr_times());
      if (hm[LSQR_NSTATE] != 0.0) {
        set_error("the sketch S A is numerically rank deficient");
        return SKLS_ERR_RANK;
      }
    }
    const double rn = hs[LSQR_RNORM], gn = hs[LSQR_ARNORM];
    inf.resid_norm = rn;
    inf.grad_norm = gn;
    if (!(std::isfinite(rn) && std::isfinite(gn))) {
      set_error("non-finite residual (check A and b for NaN/Inf)");
      status = SKLS_ERR_ARG;
      break;
    }
    if (gn <= thr * rn || hs[LSQR_DONE] != 0.0) {
      inf.certified = (gn <= thr * rn) ? 1 : 0;
      status = SKLS_OK;
      break;
    }
    // A consistent system (b in the range of A) has min ||Ax - b|| = 0, where
    // no ratio can be certified: stop once the residual is at rounding level.
    if (rn <= 1e-13 * std::sqrt(sb_norm2)) {
      status = SKLS_OK;
      break;
    }
    if (inf.iterations >= o.max_iter) break;
    // inner LSQR on min || M y - r ||, y = 0 start
    const double ratio0 = gn / rn;
    const double target = plain ? 0.5 * thr : std::fmax(0.5 * thr, 1e-4 * ratio0);
    pa.acc_f64 = plain ? 1 : 0;
    pa.Z = L.U;
    pa.z_is_b = 0;
    pa.coef = L.st + LSQR_COEF;
    SKLS_TRY(run_gemv(L.Rinv, d, L.v, L.p, s));
    // Steps are enqueued in batches and the state is read once per batch:
    // the step kernel applies the stopping test itself and leaves the state
    // alone after it holds, so steps past the stop only repeat the same
    // pass.  The first batch is one step; later ones are one fewer than the
    // steps that the observed rate of decrease of est_ar / est_r predicts
    // are still needed, at most `cap` (several for a small A, where a host
    // round trip costs as much as a step; one for a large A).
    const int cap = lsqr_batch(*A, plain);
    int64_t taken = 0;  // steps of this inner solve already counted
    double ratio = ratio0;
    int nb_next = 1;
    while (inf.iterations < o.max_iter) {
      const int nb = std::min(nb_next, o.max_iter - inf.iterations);
      for (int b = 0; b < nb; ++b) {
        SKLS_TRY(run_pass(pa, s));
        SKLS_TRY(run_reduce_partials(L.partial, L.nblk, d, L.gsum, L.red, s));
        SKLS_TRY(run_gemv(L.q.RinvT, d, L.gsum, L.vp, s));
        SKLS_TRY(run_lsqr_step(L.gsum, L.vp, d, L.v, L.w, L.y, L.st, target, s, dm));
        SKLS_TRY(run_gemv(L.Rinv, d, L.v, L.p, s));
      }
      SKLS_TRY_HIP(hipStreamSynchronize(s));
      std::memcpy(hs, hm, sizeof hs);
      const int64_t count = static_cast<int64_t>(hs[LSQR_COUNT]);
      const int64_t did = count - taken;
      inf.iterations += static_cast<int32_t>(did);
      taken = count;
      if (hs[LSQR_STOP] != 0.0) break;
      const double now = hs[LSQR_EST_R] > 0.0 ? hs[LSQR_EST_AR] / hs[LSQR_EST_R] : 0.0;
      nb_next = 1;
      if (did > 0 && now > 0.0 && ratio > 0.0 && now < ratio) {
        const double rate = std::pow(now / ratio, 1.0 / static_cast<double>(did));
        // one step short of the prediction: a step is wasted only if the
        // decrease speeds up, and a wrong guess costs one more read
        const double need = std::ceil(std::log(target / now) / std::log(rate)) - 1.0;
        if (need > 1.0) nb_next = need >= cap ? cap : static_cast<int>(need);
      }
      ratio = now;
    }
    // x += R^{-1} y
    SKLS_TRY(run_gemv(L.Rinv, d, L.y, L.tmp, s));
    SKLS_TRY(run_add(x, L.tmp, d, s));
    ++outer;
  }
  inf.refinements = outer;
  SKLS_TRY_HIP(hipEventRecord(ev[3], s));
  SKLS_TRY_HIP(hipEventSynchronize(ev[3]));
  SKLS_TRY_HIP(hipEventElapsedTime(&ms, ev[2], ev[3]));
  inf.ms_iter = ms;
  {
    const double e = inf.grad_norm / o.sigma_lb;
    const double r2 = inf.resid_norm * inf.resid_norm - e * e;
    inf.ratio_bound = (r2 > 0.0) ? std::sqrt(1.0 + e * e / r2) : INFINITY;
  }
  if (status == SKLS_ERR_NOCONV) set_error("LSQR did not certify the target within max_iter=%d", o.max_iter);
  return status;
}

}  // namespace

int32_t skls_lstsq(const skls_matrix* A, const double* b, const skls_lstsq_opts* opts, double* x,
                   skls_lstsq_info* info, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  SKLS_TRY(check_lstsq(A, opts));
  if (b == nullptr || x == nullptr) {
    set_error("b and x must be non-NULL");
    return SKLS_ERR_ARG;
  }
  if (A->d > 8192) {
    set_error("lstsq supports d <= 8192");
    return SKLS_ERR_SHAPE;
  }
  skls_lstsq_opts o = *opts;
  fill_opts(o);
  hipStream_t s = as_stream(stream);
  Arena ar(ws, ws_bytes);
  LsWs L = carve_ls(ar, *A, o);
  SKLS_TRY(need_ws(ar, ws, ws_bytes));
  // attempt r sketches with seed + r * golden gamma: a fresh, independent S
  int32_t st = SKLS_OK;
  skls_lstsq_info inf;
  for (int32_t r = 0;; ++r) {
    skls_lstsq_opts a = o;
    a.seed = o.seed + static_cast<uint64_t>(r) * 0x9E3779B97F4A7C15ull;
    clear_error();
    st = lstsq_once(A, b, a, x, L, inf, s);
    inf.retries = r;
    if ((st != SKLS_ERR_RANK && st != SKLS_ERR_NOCONV) || r >= o.max_retries) break;
  }
  if (info) *info = inf;
  return st;
}

int32_t skls_second_stage_workspace(int64_t t, int64_t d, int64_t m, size_t* bytes) {
  clear_error();
  if (bytes == nullptr) {
    set_error("bytes pointer is NULL");
    return SKLS_ERR_ARG;
  }
  SKLS_TRY(check_stage(t, d, m));
  Arena ar(nullptr, 0);
  ar.take<float>(second_stage_scratch_floats(m, d, t));
  *bytes = ar.used;
  return SKLS_OK;
}

int32_t skls_second_stage(const void* SA, const void* Sb, int32_t dtype, int64_t t, int64_t d, int64_t m,
                          uint64_t seed, double* FSA, double* FSb, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  SKLS_TRY(check_stage(t, d, m));
  if (SA == nullptr || FSA == nullptr || (Sb != nullptr && FSb == nullptr)) {
    set_error("SA and FSA must be non-NULL, and FSb too when Sb is given");
    return SKLS_ERR_ARG;
  }
  if (dtype != SKLS_F64 && dtype != SKLS_F32) {
    set_error("SA must be F64 or F32");
    return SKLS_ERR_DTYPE;
  }
  Arena ar(ws, ws_bytes);
  float* part = ar.take<float>(second_stage_scratch_floats(m, d, t));
  SKLS_TRY(need_ws(ar, ws, ws_bytes));
  return run_second_stage(SA, Sb, dtype, t, d, m, seed, FSA, FSb, part, as_stream(stream));
}

int32_t skls_leverage_workspace(const skls_matrix* A, int64_t t, int32_t k, size_t* bytes) {
  clear_error();
  SKLS_TRY(validate_matrix(A, true));
  SKLS_TRY(check_t(t));
  if (bytes == nullptr || k < 1 || k > 64 || t < A->d) {
    set_error("need bytes != NULL, 1 <= k <= 64, t >= d");
    return SKLS_ERR_ARG;
  }
  Arena ar(nullptr, 0);
  carve_lev(ar, *A, t, k);
  *bytes = ar.used;
  return SKLS_OK;
}

int32_t skls_leverage_scores(const skls_matrix* A, int64_t t, uint64_t seed, int32_t k, const double* Pi2,
                             float* scores, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  SKLS_TRY(validate_matrix(A, true));
  SKLS_TRY(check_t(t));
  if (k < 1 || k > 64 || scores == nullptr) {
    set_error("need 1 <= k <= 64 and non-NULL scores");
    return SKLS_ERR_ARG;
  }
  if (t < A->d || A->d > 8192) {
    set_error("need d <= t and d <= 8192");
    return SKLS_ERR_SHAPE;
  }
  hipStream_t s = as_stream(stream);
  const int64_t d = A->d;
  Arena ar(ws, ws_bytes);
  LevWs L = carve_lev(ar, *A, t, k);
  SKLS_TRY(need_ws(ar, ws, ws_bytes));
  SKLS_TRY(run_sketch(*A, nullptr, SKLS_F64, t, seed, nullptr, SKLS_SKETCH_AUTO, L.SA, nullptr, L.sk_dtype, L.sk,
                      L.sk_bytes, s));
  SKLS_TRY(qr_from(L.SA, L.sk_dtype, nullptr, SKLS_F64, t, d, L.q, L.R, L.Rinv, L.q.RinvT, s));
  if (Pi2 == nullptr) {
    SKLS_TRY(run_sign_projection(d, k, seed, L.Pi2, s));
    Pi2 = L.Pi2;
  }
  SKLS_TRY(run_rinv_times(L.Rinv, d, Pi2, k, L.T, s));
  SKLS_TRY(run_leverage(*A, L.T, k, scores, s));
  int32_t st = 0;
  SKLS_TRY(read_status(L.q.status, s, &st));
  if (st) {
    set_error("the sketch S A is numerically rank deficient");
    return SKLS_ERR_RANK;
  }
  return SKLS_OK;
}

int32_t skls_leverage_from_r_workspace(const skls_matrix* A, int32_t k, size_t* bytes) {
  clear_error();
  SKLS_TRY(validate_matrix(A, true));
  if (bytes == nullptr || k < 1 || k > 64) {
    set_error("need bytes != NULL and 1 <= k <= 64");
    return SKLS_ERR_ARG;
  }
  Arena ar(nullptr, 0);
  carve_lev_r(ar, A->d, k);
  *bytes = ar.used;
  return SKLS_OK;
}

int32_t skls_leverage_scores_from_r(const skls_matrix* A, const double* R, int32_t k, const double* Pi2,
                                    uint64_t seed, float* scores, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  SKLS_TRY(validate_matrix(A, true));
  if (k < 1 || k > 64 || R == nullptr || scores == nullptr) {
    set_error("need 1 <= k <= 64 and non-NULL R, scores");
    return SKLS_ERR_ARG;
  }
  if (A->d > 8192) {
    set_error("need d <= 8192");
    return SKLS_ERR_SHAPE;
  }
  hipStream_t s = as_stream(stream);
  const int64_t d = A->d;
  Arena ar(ws, ws_bytes);
  LevRWs L = carve_lev_r(ar, d, k);
  SKLS_TRY(need_ws(ar, ws, ws_bytes));
  SKLS_TRY(run_trinv(R, d, L.Rinv, L.RinvT, s, nullptr));
  if (Pi2 == nullptr) {
    SKLS_TRY(run_sign_projection(d, k, seed, L.Pi2, s));
    Pi2 = L.Pi2;
  }
  SKLS_TRY(run_rinv_times(L.Rinv, d, Pi2, k, L.T, s));
  return run_leverage(*A, L.T, k, scores, s);
}

int32_t skls_gram_workspace(const skls_matrix* A, size_t* bytes) {
  clear_error();
  SKLS_TRY(validate_matrix(A, true));
  if (bytes == nullptr) {
    set_error("bytes pointer is NULL");
    return SKLS_ERR_ARG;
  }
  Arena ar(nullptr, 0);
  const size_t gb = gram_ws_bytes(A->n > 0 ? A->n : 1, A->d);
  ar.take<char>(gb);
  ar.take<double>(static_cast<size_t>(A->d * A->d));
  *bytes = ar.used;
  return SKLS_OK;
}

int32_t skls_gram(const skls_matrix* A, float* C, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  SKLS_TRY(validate_matrix(A, true));
  if (A->layout != SKLS_DENSE) {
    set_error("skls_gram supports dense A only");
    return SKLS_ERR_NOTIMPL;
  }
  if (C == nullptr) {
    set_error("C is NULL");
    return SKLS_ERR_ARG;
  }
  hipStream_t s = as_stream(stream);
  Arena ar(ws, ws_bytes);
  const int64_t m = A->n > 0 ? A->n : 1;
  const size_t gb = gram_ws_bytes(m, A->d);
  double* gw = reinterpret_cast<double*>(ar.take<char>(gb));
  double* G = ar.take<double>(static_cast<size_t>(A->d * A->d));
  SKLS_TRY(need_ws(ar, ws, ws_bytes));
  if (A->n == 0) return launch_fill_zero(C, static_cast<size_t>(A->d * A->d) * sizeof(float), s);
  SKLS_TRY(run_gram(A->val, A->dtype, A->ld, nullptr, SKLS_F64, A->n, A->d, G, gw, gb, s));
  return run_convert_f64_to_f32(G, C, A->d * A->d, s);
}

int32_t skls_learned_workspace(const skls_matrix* A, int64_t t, size_t* bytes) {
  clear_error();
  SKLS_TRY(validate_matrix(A, false));
  SKLS_TRY(check_t(t));
  if (bytes == nullptr) {
    set_error("bytes pointer is NULL");
    return SKLS_ERR_ARG;
  }
  const int64_t d = A->d;
  Arena ar(nullptr, 0);
  ar.take<float>(static_cast<size_t>(t * d));
  ar.take<char>(sketch_ws_bytes(*A, t, SKLS_SKETCH_SORTED));
  ar.take<char>(gram_ws_bytes(t, d));
  ar.take<double>(static_cast<size_t>(d * d));
  ar.take<float>(static_cast<size_t>(d * d));
  ar.take<float>(static_cast<size_t>(t * d));
  *bytes = ar.used;
  return SKLS_OK;
}

namespace {

int32_t check_learned(const skls_matrix* A, const float* C, const float* w, const float* loss) {
  SKLS_TRY(validate_matrix(A, false));
  if (A->layout != SKLS_DENSE || A->dtype != SKLS_F32) {
    set_error("learned values need a dense float32 A");
    return SKLS_ERR_DTYPE;
  }
  if (C == nullptr || w == nullptr || loss == nullptr) {
    set_error("C, w and loss must be non-NULL");
    return SKLS_ERR_ARG;
  }
  if (A->d > 4096) {
    set_error("learned values support d <= 4096");
    return SKLS_ERR_SHAPE;
  }
  return SKLS_OK;
}

// Scratch of the loss and gradient after the forward sketch: Gram partials,
// Y^T Y, E and G.
struct LearnedRest {
  size_t gb;
  double* gw;
  double* P;
  float* E;
  float* G;
};

LearnedRest carve_learned_rest(Arena& ar, int64_t t, int64_t d) {
  LearnedRest r;
  r.gb = gram_ws_bytes(t, d);
  r.gw = reinterpret_cast<double*>(ar.take<char>(r.gb));
  r.P = ar.take<double>(static_cast<size_t>(d * d));
  r.E = ar.take<float>(static_cast<size_t>(d * d));
  r.G = ar.take<float>(static_cast<size_t>(t * d));
  return r;
}

// The Gram of Y goes straight into the loss for t <= kPEMaxRows, in
// kPESplits row splits: k_learned_PE sums them in one block, whose reads of
// the splits bound it, so few long splits beat many short ones there.
constexpr int64_t kPEMaxRows = 4096;
constexpr int kPESplits = 4;

// Loss and gradient once the forward sketch Y = S_w A is formed.  At d <= 64
// (and t <= kPEMaxRows) the Gram's splits go straight into the loss and E;
// with the bucket order of the sketch's plan (off, perm) the product 4 Y E
// and the gather run as one launch as well.
int32_t learned_rest(const skls_matrix& A, const float* C, int64_t t, uint64_t seed, float grad_scale,
                     int32_t accumulate, float* loss, float* grad_w, const LearnedRest& r, const float* Y,
                     hipStream_t s, const int32_t* off = nullptr, const int32_t* perm = nullptr) {
  const int64_t d = A.d;
  double* P = r.P;
  float* E = r.E;
  float* G = r.G;
  if (d <= 64 && t <= kPEMaxRows) {
    int S = 0, pitch = 0;
    SKLS_TRY(run_gram_small_partials(Y, SKLS_F32, d, t, d, kPESplits, r.gw, r.gb, &S, &pitch, s));
    SKLS_TRY(run_learned_PE(r.gw, S, pitch, C, d, E, loss, s));
  } else {
    SKLS_TRY(run_gram(Y, SKLS_F32, d, nullptr, SKLS_F64, t, d, P, r.gw, r.gb, s));
    SKLS_TRY(run_learned_E(P, d, C, d, E, loss, s));
  }
  if (grad_w == nullptr) return SKLS_OK;
  if (d <= 64 && off != nullptr && perm != nullptr)
    return run_learned_G_gather(Y, E, t, off, perm, A, grad_scale, accumulate != 0, grad_w, s);
  SKLS_TRY(run_learned_G(Y, E, t, d, G, s));
  return run_learned_gather(A, G, static_cast<uint32_t>(t), seed, grad_scale, accumulate != 0, grad_w, s);
}

}  // namespace

int32_t skls_learned_grad(const skls_matrix* A, const float* C, int64_t t, uint64_t seed, const float* w,
                          float grad_scale, int32_t accumulate, float* loss, float* grad_w, void* ws, size_t ws_bytes,
                          void* stream) {
  clear_error();
  SKLS_TRY(check_learned(A, C, w, loss));
  SKLS_TRY(check_t(t));
  hipStream_t s = as_stream(stream);
  const int64_t d = A->d;
  Arena ar(ws, ws_bytes);
  float* Y = ar.take<float>(static_cast<size_t>(t * d));
  const size_t skb = sketch_ws_bytes(*A, t, SKLS_SKETCH_SORTED);
  void* sk = ar.take<char>(skb);
  const LearnedRest r = carve_learned_rest(ar, t, d);
  SKLS_TRY(need_ws(ar, ws, ws_bytes));
  SKLS_TRY(run_sketch(*A, nullptr, SKLS_F64, t, seed, w, SKLS_SKETCH_SORTED, Y, nullptr, SKLS_F32, sk, skb, s));
  return learned_rest(*A, C, t, seed, grad_scale, accumulate, loss, grad_w, r, Y, s);
}

int32_t skls_learned_grad_planned(const skls_matrix* A, const float* C, const skls_sketch_plan_desc* desc,
                                  const void* plan, size_t plan_bytes, const float* w, float grad_scale,
                                  int32_t accumulate, float* loss, float* grad_w, void* ws, size_t ws_bytes,
                                  void* stream) {
  clear_error();
  SKLS_TRY(check_learned(A, C, w, loss));
  if (desc == nullptr) {
    set_error("desc is NULL");
    return SKLS_ERR_ARG;
  }
  if (desc->n != A->n || desc->d != A->d || desc->layout != SKLS_DENSE || desc->out_dtype != SKLS_F32 ||
      desc->row_start != 0) {
    set_error("the plan must come from a dense float32-output sketch of a matrix of this shape, row_start 0");
    return SKLS_ERR_SHAPE;
  }
  if (desc->bytes > 0 && (plan == nullptr || plan_bytes < static_cast<size_t>(desc->bytes))) {
    set_error("sketch plan buffer too small: need %lld bytes", static_cast<long long>(desc->bytes));
    return SKLS_ERR_WORKSPACE;
  }
  const int64_t t = desc->t, d = A->d;
  hipStream_t s = as_stream(stream);
  Arena ar(ws, ws_bytes);
  float* Y = ar.take<float>(static_cast<size_t>(t * d));
  const LearnedRest r = carve_learned_rest(ar, t, d);
  SKLS_TRY(need_ws(ar, ws, ws_bytes));
  const int32_t *off = nullptr, *perm = nullptr;
  SKLS_TRY(sorted_plan_order(*A, t, desc->variant, SKLS_F32, plan, plan_bytes, &off, &perm));
  SKLS_TRY(apply_sketch_plan(*A, nullptr, SKLS_F64, t, plain_key(desc->seed), w, desc->variant, Y, nullptr, SKLS_F32,
                             plan, plan_bytes, s));
  return learned_rest(*A, C, t, desc->seed, grad_scale, accumulate, loss, grad_w, r, Y, s, off, perm);
}

namespace {

// Concurrent chains of the batched learned gradient: the caller's stream and
// kLanes - 1 more.
constexpr int kLanes = 4;

// Streams beside a caller's stream on the current device: non-blocking, of
// default priority, each with an event that joins it back; plus one event
// that forks work onto them.  Created once per host thread and device.
struct LanePool {
  hipStream_t s[kLanes - 1] = {};
  hipEvent_t done[kLanes - 1] = {};
  hipEvent_t fork = nullptr;
  bool ready = false;
};

int32_t lane_pool(LanePool** out) {
  thread_local LanePool pools[16];
  int dev = 0;
  SKLS_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 16) {
    set_error("device index %d out of range", dev);
    return SKLS_ERR_DEVICE;
  }
  LanePool& p = pools[dev];
  if (!p.ready) {
    LanePool q;
    bool ok = hipEventCreateWithFlags(&q.fork, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; ok && k < kLanes - 1; ++k)
      ok = hipStreamCreateWithFlags(&q.s[k], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&q.done[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      for (int k = 0; k < kLanes - 1; ++k) {
        if (q.s[k] != nullptr) (void)hipStreamDestroy(q.s[k]);
        if (q.done[k] != nullptr) (void)hipEventDestroy(q.done[k]);
      }
      if (q.fork != nullptr) (void)hipEventDestroy(q.fork);
      set_error("creating the streams of the batched gradient failed");
      return SKLS_ERR_DEVICE;
    }
    q.ready = true;
    p = q;
  }
  *out = &p;
  return SKLS_OK;
}

struct BatchLanes {
  float* Y[kLanes];
  LearnedRest r[kLanes];
  float* slots;  // kLanes gradient slots of n floats, one after another
};

// The other use of the batch workspace, when every step has a one-launch
// form (d <= 64, t <= kPEMaxRows, a dense sorted plan): up to kSortedMany
// matrices at a time, each with its sketch, Gram splits, E and gradient slot.
struct BatchMany {
  float* Y;
  int64_t ystride;
  double* partial;
  int64_t pstride;
  float* E;
  float* slots;
  int64_t gstride;
};

bool many_applies(int64_t d, int64_t t) { return d <= 64 && t <= kPEMaxRows; }

BatchMany carve_many(Arena& ar, int64_t n, int64_t t, int64_t d) {
  BatchMany b;
  b.ystride = div_up(t * d, 64) * 64;
  b.pstride = static_cast<int64_t>(kPESplits) * gram_small_split_doubles();
  b.gstride = div_up(n, 64) * 64;
  b.Y = ar.take<float>(static_cast<size_t>(kSortedMany * b.ystride));
  b.partial = ar.take<double>(static_cast<size_t>(kSortedMany * b.pstride));
  b.E = ar.take<float>(static_cast<size_t>(kSortedMany * d * d));
  b.slots = ar.take<float>(static_cast<size_t>(kSortedMany * b.gstride));
  return b;
}

BatchLanes carve_batch(Arena& ar, int64_t n, int64_t t, int64_t d) {
  BatchLanes b;
  for (int k = 0; k < kLanes; ++k) {
    b.Y[k] = ar.take<float>(static_cast<size_t>(t * d));
    b.r[k] = carve_learned_rest(ar, t, d);
  }
  b.slots = ar.take<float>(static_cast<size_t>(kLanes * n));
  return b;
}

}  // namespace

int32_t skls_learned_batch_workspace(const skls_matrix* A, int64_t t, size_t* bytes) {
  clear_error();
  SKLS_TRY(validate_matrix(A, false));
  SKLS_TRY(check_t(t));
  if (bytes == nullptr) {
    set_error("bytes pointer is NULL");
    return SKLS_ERR_ARG;
  }
  Arena ar(nullptr, 0);
  carve_batch(ar, A->n, t, A->d);
  size_t need = ar.used;
  if (many_applies(A->d, t)) {
    Arena am(nullptr, 0);
    carve_many(am, A->n, t, A->d);
    need = am.used > need ? am.used : need;
  }
  *bytes = need;
  return SKLS_OK;
}

int32_t skls_learned_grad_batch(int32_t count, const skls_matrix* A, const float* const* C, const float* scale,
                                const skls_sketch_plan_desc* desc, const void* plan, size_t plan_bytes,
                                const float* w, int32_t accumulate, float* loss, float* grad_w, void* ws,
                                size_t ws_bytes, void* stream) {
  clear_error();
  if (count < 1 || A == nullptr || C == nullptr || desc == nullptr) {
    set_error("need count >= 1 and non-NULL A, C and desc");
    return SKLS_ERR_ARG;
  }
  for (int32_t j = 0; j < count; ++j) {
    SKLS_TRY(check_learned(&A[j], C[j], w, loss));
    if (A[j].n != desc->n || A[j].d != desc->d || desc->layout != SKLS_DENSE || desc->out_dtype != SKLS_F32 ||
        desc->row_start != 0) {
      set_error("matrix %d: the plan must come from a dense float32-output sketch of a matrix of this shape, "
                "row_start 0", j);
      return SKLS_ERR_SHAPE;
    }
  }
  if (desc->bytes > 0 && (plan == nullptr || plan_bytes < static_cast<size_t>(desc->bytes))) {
    set_error("sketch plan buffer too small: need %lld bytes", static_cast<long long>(desc->bytes));
    return SKLS_ERR_WORKSPACE;
  }
  const int64_t t = desc->t, d = A[0].d, n = A[0].n;
  hipStream_t s = as_stream(stream);
  const int32_t *off = nullptr, *perm = nullptr;
  SKLS_TRY(sorted_plan_order(A[0], t, desc->variant, SKLS_F32, plan, plan_bytes, &off, &perm));
  if (off != nullptr && many_applies(d, t)) {
    // every step as one launch over up to kSortedMany matrices: the sketches,
    // the Gram splits, E and the losses, 4 Y E with the gather into one slot
    // per matrix, and the sum of the slots
    Arena am(ws, ws_bytes);
    const BatchMany b = carve_many(am, n, t, d);
    SKLS_TRY(need_ws(am, ws, ws_bytes));
    for (int32_t g0 = 0; g0 < count; g0 += kSortedMany) {
      const int cnt = count - g0 < kSortedMany ? count - g0 : kSortedMany;
      LearnedMany args{};
      bool vec = true;
      for (int j = 0; j < cnt; ++j) {
        const skls_matrix& M = A[g0 + j];
        args.A[j] = static_cast<const float*>(M.val);
        args.ld[j] = M.ld;
        args.C[j] = C[g0 + j];
        args.scale[j] = scale != nullptr ? scale[g0 + j] : 1.0f;
        vec = vec && reinterpret_cast<uintptr_t>(M.val) % 16 == 0 && M.ld % 4 == 0 && M.d % 4 == 0;
      }
      SKLS_TRY(apply_sorted_many(A + g0, cnt, t, plain_key(desc->seed), w, plan, plan_bytes, b.Y, b.ystride, s));
      int S = 0, pitch = 0;
      SKLS_TRY(run_gram_small_partials_many(b.Y, cnt, b.ystride, t, d, kPESplits, b.partial, b.pstride, &S, &pitch,
                                            s));
      SKLS_TRY(run_learned_PE_many(b.partial, b.pstride, S, pitch, args, cnt, d, b.E, loss + g0, s));
      if (grad_w != nullptr) {
        SKLS_TRY(run_learned_G_gather_many(b.Y, b.ystride, b.E, t, d, off, perm, args, cnt, vec, b.slots, b.gstride,
                                           s));
        SKLS_TRY(run_sum_slots(n, b.slots, b.gstride, cnt, 1.0f, accumulate != 0 || g0 > 0, grad_w, s));
      }
    }
    return SKLS_OK;
  }
  Arena ar(ws, ws_bytes);
  const BatchLanes b = carve_batch(ar, n, t, d);
  SKLS_TRY(need_ws(ar, ws, ws_bytes));
  const int lanes = count < kLanes ? count : kLanes;
  LanePool* pool = nullptr;
  hipStream_t st[kLanes] = {s, s, s, s};
  if (lanes > 1) {
    SKLS_TRY(lane_pool(&pool));
    SKLS_TRY_HIP(hipEventRecord(pool->fork, s));
    for (int k = 1; k < lanes; ++k) {
      SKLS_TRY_HIP(hipStreamWaitEvent(pool->s[k - 1], pool->fork, 0));
      st[k] = pool->s[k - 1];
    }
  }
  // matrix j runs on lane j mod lanes, adding its weighted gradient into
  // that lane's slot; the lanes' slots are summed on the caller's stream at
  // the end
  int32_t status = SKLS_OK;
  for (int32_t j = 0; j < count && status == SKLS_OK; ++j) {
    const int k = j % lanes;
    status = apply_sketch_plan(A[j], nullptr, SKLS_F64, t, plain_key(desc->seed), w, desc->variant, b.Y[k], nullptr,
                               SKLS_F32, plan, plan_bytes, st[k]);
    if (status == SKLS_OK)
      status = learned_rest(A[j], C[j], t, desc->seed, scale != nullptr ? scale[j] : 1.0f, j >= lanes ? 1 : 0,
                            loss + j, grad_w != nullptr ? b.slots + k * n : nullptr, b.r[k], b.Y[k], st[k], off,
                            perm);
  }
  // join even after a failure, so that no lane runs past the caller's stream
  for (int k = 1; k < lanes; ++k) {
    const hipError_t e1 = hipEventRecord(pool->done[k - 1], st[k]);
    const hipError_t e2 = hipStreamWaitEvent(s, pool->done[k - 1], 0);
    if (status == SKLS_OK && (e1 != hipSuccess || e2 != hipSuccess)) {
      set_error("joining the streams of the batched gradient failed");
      status = SKLS_ERR_DEVICE;
    }
  }
  if (status != SKLS_OK || grad_w == nullptr) return status;
  return run_sum_slots(n, b.slots, n, lanes, 1.0f, accumulate != 0, grad_w, s);
}

int32_t skls_adam_step(int64_t n, float* w, const float* g, float* m, float* v, int32_t step, float lr, float beta1,
                       float beta2, float eps, void* stream) {
  clear_error();
  if (n < 0 || step < 1 || (n > 0 && (w == nullptr || g == nullptr || m == nullptr || v == nullptr))) {
    set_error("need n >= 0, step >= 1 and non-NULL buffers");
    return SKLS_ERR_ARG;
  }
  if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f)) {
    set_error("bad Adam hyper-parameters");
    return SKLS_ERR_ARG;
  }
  return run_adam(n, w, g, m, v, step, lr, beta1, beta2, eps, as_stream(stream));
}

int32_t skls_multi_lstsq_workspace(const skls_matrix* A, int64_t dp, const skls_multi_opts* opts, size_t* bytes) {
  clear_error();
  SKLS_TRY(validate_matrix(A, true));
  if (opts == nullptr || bytes == nullptr) {
    set_error("opts and bytes must be non-NULL");
    return SKLS_ERR_ARG;
  }
  MultiPlan P;
  SKLS_TRY(multi_plan(*A, dp, *opts, P));
  *bytes = multi_ws_bytes(P);
  return SKLS_OK;
}

int32_t skls_multi_lstsq(const skls_matrix* A, const double* B, int64_t dp, const skls_multi_opts* opts, double* Y,
                         int32_t* rows, double* weights, skls_multi_info* info, void* ws, size_t ws_bytes,
                         void* stream) {
  clear_error();
  SKLS_TRY(validate_matrix(A, true));
  if (opts == nullptr || B == nullptr || Y == nullptr) {
    set_error("opts, B and Y must be non-NULL");
    return SKLS_ERR_ARG;
  }
  MultiPlan P;
  SKLS_TRY(multi_plan(*A, dp, *opts, P));
  return run_multi_lstsq(*A, B, P, opts->seed, Y, rows, weights, info, ws, ws_bytes, as_stream(stream));
}

int32_t skls_lp_regression_workspace(const skls_matrix* A, const skls_lp_opts* opts, size_t* bytes) {
  clear_error();
  SKLS_TRY(validate_matrix(A, true));
  if (opts == nullptr || bytes == nullptr) {
    set_error("opts and bytes must be non-NULL");
    return SKLS_ERR_ARG;
  }
  LpPlan P;
  SKLS_TRY(lp_plan(*A, *opts, P));
  *bytes = lp_ws_bytes(P);
  return SKLS_OK;
}

int32_t skls_lp_regression(const skls_matrix* A, const double* b, const skls_lp_opts* opts, double* x, double* x_c,
                           int32_t* rows1, double* w1, int32_t* rows2, double* w2, skls_lp_info* info, void* ws,
                           size_t ws_bytes, void* stream) {
  clear_error();
  SKLS_TRY(validate_matrix(A, true));
  if (opts == nullptr || b == nullptr || x == nullptr) {
    set_error("opts, b and x must be non-NULL");
    return SKLS_ERR_ARG;
  }
  LpPlan P;
  SKLS_TRY(lp_plan(*A, *opts, P));
  return run_lp(*A, b, P, x, x_c, rows1, w1, rows2, w2, info, ws, ws_bytes, as_stream(stream));
}

int32_t skls_low_rank_workspace(const skls_matrix* A, const skls_low_rank_opts* opts, size_t* bytes) {
  clear_error();
  SKLS_TRY(validate_matrix(A, true));
  if (opts == nullptr || bytes == nullptr) {
    set_error("opts and bytes must be non-NULL");
    return SKLS_ERR_ARG;
  }
  LowRankPlan P;
  SKLS_TRY(low_rank_plan(*A, *opts, P));
  *bytes = low_rank_ws_bytes(P);
  return SKLS_OK;
}

int32_t skls_low_rank(const skls_matrix* A, const skls_low_rank_opts* opts, double* L, double* D, double* W,
                      skls_low_rank_info* info, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  SKLS_TRY(validate_matrix(A, true));
  if (opts == nullptr || L == nullptr || D == nullptr || W == nullptr) {
    set_error("opts, L, D and W must be non-NULL");
    return SKLS_ERR_ARG;
  }
  LowRankPlan P;
  SKLS_TRY(low_rank_plan(*A, *opts, P));
  return run_low_rank(*A, P, opts->seed, L, D, W, info, ws, ws_bytes, as_stream(stream));
}

}  // extern "C"
