// Multiple-response regression min_Y ||A Y - B||_F by leverage-score sampling
// (Section 7, theorem on the generalized-regression algorithm):
//   1. leverage scores of A to constant relative error by the Section 6
//      theorem: R1 of a sparse-embedding sketch S1 A (t rows), T = R1^{-1} Pi2
//      (Pi2 the d x k_G sign matrix / sqrt(k_G) of the stream seed ^
//      "leverage"), scores = squared row norms of A T, all in float64;
//   2. t_S draws with replacement, probabilities proportional to the scores
//      (uniforms from the stream seed ^ "sampling"), a row drawn c times kept
//      once with weight sqrt(c / (t_S p)): the coreset;
//   3. Y~ = R^{-1} Q^T (S B) for S A = Q R, evaluated as
//      R^{-1} R^{-T} (S A)^T (S B) with R from the float64 Gram of S A.

#include "kernels.hpp"
#include "profile.hpp"
#include "sampling.hpp"

namespace skls {
namespace {

// partial[b] = sum over the block's entries of (AY - B)^2, slot nblk + b the
// sum of B^2 (n x dp, packed rows).
__global__ __launch_bounds__(kT) void k_resid_parts(int64_t count, const double* __restrict__ AY,
                                                    const double* __restrict__ B, double* __restrict__ partial) {
  __shared__ double sh[kT / kWave];
  double s = 0.0, q = 0.0;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x; e < count;
       e += static_cast<int64_t>(gridDim.x) * kT) {
    const double r = AY[e] - B[e];
    s += r * r;
    q += B[e] * B[e];
  }
  s = block_sum(s, sh);
  q = block_sum(q, sh);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = s;
    partial[gridDim.x + blockIdx.x] = q;
  }
}

__global__ void k_sum_two(const double* __restrict__ partial, int nblk, double* __restrict__ out) {
  if (threadIdx.x >= 2) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[threadIdx.x * nblk + b];
  out[threadIdx.x] = s;
}

constexpr int kResidBlocks = 256;

struct MrWs {
  void* sk;
  size_t sk_bytes;
  double* SA1;
  void* gram;
  size_t gram_bytes;
  double *G, *cholw, *R, *Rinv, *RinvT;
  int32_t* status;
  double *Pi2, *T, *Z, *score, *cum, *dtiles;
  int32_t *counts, *flag, *pos, *itiles, *last, *list;
  double *wts, *SAc, *SBc, *C, *Yt, *AY, *part, *sums;
  GemmScratch gs;
};

MrWs carve_mr(Arena& ar, const MultiPlan& P) {
  MrWs w;
  const int64_t n = P.n, d = P.d, dp = P.dp, ns = P.nsmax;
  w.sk_bytes = P.sk_bytes;
  w.sk = ar.take<char>(P.sk_bytes + 1);
  w.SA1 = ar.take<double>(static_cast<size_t>(P.t) * d);
  size_t gb = gram_ws_bytes(P.t, d);
  const size_t g2 = gram_ws_bytes(ns, d);
  w.gram_bytes = gb > g2 ? gb : g2;
  w.gram = ar.take<double>(w.gram_bytes / sizeof(double) + 1);
  w.G = ar.take<double>(static_cast<size_t>(d) * d);
  w.cholw = ar.take<double>(cholesky_scratch_doubles(d));
  w.R = ar.take<double>(static_cast<size_t>(d) * d);
  w.Rinv = ar.take<double>(static_cast<size_t>(d) * d);
  w.RinvT = ar.take<double>(static_cast<size_t>(d) * d);
  w.status = ar.take<int32_t>(4);
  w.Pi2 = ar.take<double>(static_cast<size_t>(d) * P.kg);
  w.T = ar.take<double>(static_cast<size_t>(d) * P.kg);
  w.Z = ar.take<double>(static_cast<size_t>(n) * P.kg);
  w.score = ar.take<double>(n);
  w.cum = ar.take<double>(n);
  w.dtiles = ar.take<double>(tiles_for(n));
  w.counts = ar.take<int32_t>(n);
  w.flag = ar.take<int32_t>(n);
  w.pos = ar.take<int32_t>(n);
  w.itiles = ar.take<int32_t>(tiles_for(n));
  w.last = ar.take<int32_t>(4);
  w.list = ar.take<int32_t>(ns);
  w.wts = ar.take<double>(ns);
  w.SAc = ar.take<double>(static_cast<size_t>(ns) * d);
  w.SBc = ar.take<double>(static_cast<size_t>(ns) * dp);
  w.C = ar.take<double>(static_cast<size_t>(d) * dp);
  w.Yt = ar.take<double>(static_cast<size_t>(d) * dp);
  w.AY = ar.take<double>(static_cast<size_t>(n) * dp);
  w.part = ar.take<double>(2 * kResidBlocks);
  w.sums = ar.take<double>(2);
  w.gs.doubles = size_t(1) << 21;
  w.gs.part = ar.take<double>(w.gs.doubles);
  return w;
}

}  // namespace

int32_t run_sign_projection(int64_t rows, int32_t kg, uint64_t seed, double* Pi2, hipStream_t s) {
  if (rows * kg == 0) return SKLS_OK;
  hipLaunchKernelGGL(k_sign_projection, dim3(grid_for(rows * kg, kT, 1 << 20)), dim3(kT), 0, s,
                     static_cast<int>(rows), kg, seed, Pi2);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t multi_plan(const skls_matrix& A, int64_t dp, const skls_multi_opts& o, MultiPlan& P) {
  P.n = A.n;
  P.d = A.d;
  P.dp = dp;
  P.t = o.t;
  P.ts = o.t_s;
  P.kg = o.k_g > 0 ? o.k_g : 32;
  if (dp < 1 || dp > 64 || P.kg > 64 || o.k_g < 0) {
    set_error("multi_lstsq: need 1 <= d' <= 64 and 0 <= k_g <= 64");
    return SKLS_ERR_ARG;
  }
  if (o.t < A.d || o.t >= (int64_t(1) << 31) || o.t_s < A.d || o.t_s >= (int64_t(1) << 31)) {
    set_error("multi_lstsq: need d <= t < 2^31 and d <= t_s < 2^31");
    return SKLS_ERR_SHAPE;
  }
  if (A.n >= (int64_t(1) << 31) || A.d > 8192) {
    set_error("multi_lstsq: need n < 2^31 and d <= 8192");
    return SKLS_ERR_SHAPE;
  }
  P.nsmax = std::min(P.n, P.ts);
  P.sk_bytes = sketch_ws_bytes(A, o.t, SKLS_SKETCH_AUTO);
  return SKLS_OK;
}

size_t multi_ws_bytes(const MultiPlan& P) {
  Arena ar(nullptr, 0);
  carve_mr(ar, P);
  return ar.used;
}

int32_t run_multi_lstsq(const skls_matrix& A, const double* B, const MultiPlan& P, uint64_t seed, double* Y,
                        int32_t* rows_out, double* weights_out, skls_multi_info* info, void* ws, size_t ws_bytes,
                        hipStream_t s) {
  Arena ar(ws, ws_bytes);
  MrWs w = carve_mr(ar, P);
  if (!ar.fits() || ws == nullptr) {
    set_error("multi_lstsq: workspace too small (%zu bytes needed)", ar.used);
    return SKLS_ERR_WORKSPACE;
  }
  const int64_t n = P.n, d = P.d, dp = P.dp;
  const int kg = P.kg, dpi = static_cast<int>(dp);
  skls_multi_info inf{};
  hipEvent_t ev[3];
  for (auto& e : ev) SKLS_TRY_HIP(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 3; ++i) (void)hipEventDestroy(e[i]);
    }
  } guard{ev};
  SKLS_TRY_HIP(hipEventRecord(ev[0], s));
  int32_t st_h = 0;

  // ---- step 1: scores from R1 of S1 A
  SKLS_TRY(run_sketch(A, nullptr, SKLS_F64, P.t, seed, nullptr, SKLS_SKETCH_AUTO, w.SA1, nullptr, SKLS_F64, w.sk,
                      w.sk_bytes, s));
  SKLS_TRY(run_gram(w.SA1, SKLS_F64, d, nullptr, SKLS_F64, P.t, d, w.G, w.gram, w.gram_bytes, s));
  SKLS_TRY(run_cholesky(w.G, d, d, w.R, w.Rinv, w.RinvT, w.status, w.cholw, s));
  SKLS_TRY(to_host(&st_h, w.status, sizeof st_h, s));
  if (st_h) {
    set_error("multi_lstsq: the sketch S1 A is numerically rank deficient");
    return SKLS_ERR_RANK;
  }
  int64_t ns = 0;
  {
    PhaseTimer pt("multi_scores", s);
    SKLS_TRY(row_norm_estimates(A, w.Rinv, kg, seed, w.Pi2, w.T, w.Z, w.score, w.last, w.gs, s));

    // ---- step 2: draws, the coreset
    SKLS_TRY(scan<double>(w.score, n, w.dtiles, w.cum, false, s));
    SKLS_TRY(launch_fill_zero(w.counts, static_cast<size_t>((n + 3) / 4) * 16, s));
    hipLaunchKernelGGL(k_sample, dim3(grid_for(P.ts, kT, 4096)), dim3(kT), 0, s, P.ts, n, seed, w.cum, w.score,
                       w.last, w.counts);
    SKLS_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_flags, dim3(grid_for(n, kT, 4096)), dim3(kT), 0, s, n, w.counts, w.flag);
    SKLS_CHECK_LAUNCH();
    SKLS_TRY(scan<int32_t>(w.flag, n, w.itiles, w.pos, true, s));
    int32_t hv[2];
    double total = 0.0;
    SKLS_TRY_HIP(hipMemcpyAsync(&hv[0], w.pos + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SKLS_TRY_HIP(hipMemcpyAsync(&hv[1], w.flag + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SKLS_TRY(to_host(&total, w.cum + (n - 1), sizeof total, s));
    if (!(total > 0.0) || !std::isfinite(total)) {
      set_error("multi_lstsq: the leverage scores are not positive and finite");
      return SKLS_ERR_RANK;
    }
    ns = static_cast<int64_t>(hv[0]) + hv[1];
    if (ns < d) {
      set_error("multi_lstsq: %lld distinct rows drawn, fewer than d = %lld (raise t_s)", static_cast<long long>(ns),
                static_cast<long long>(d));
      return SKLS_ERR_RANK;
    }
    hipLaunchKernelGGL(k_compact<int32_t>, dim3(grid_for(n, kT, 4096)), dim3(kT), 0, s, n, P.ts, w.counts, w.pos,
                       w.score, w.cum, nullptr, w.list, w.wts, nullptr);
    SKLS_CHECK_LAUNCH();
  }
  inf.rows_sampled = ns;
  SKLS_TRY_HIP(hipEventRecord(ev[1], s));

  // ---- step 3: S A, S B, R of S A, Y = R^{-1} R^{-T} (S A)^T (S B)
  {
    PhaseTimer pt("multi_solve", s);
    const unsigned gr = grid_for(ns, kT / kWave, 8192);
    int32_t st = with_value(A.dtype, [&](auto tv) -> int32_t {
      using TV = decltype(tv);
      if (A.layout != SKLS_CSR) {
        hipLaunchKernelGGL(k_gather_rows<TV>, dim3(gr), dim3(kT), 0, s, ns, d, A.ld, static_cast<const TV*>(A.val),
                           w.list, w.wts, w.SAc);
        SKLS_CHECK_LAUNCH();
        return SKLS_OK;
      }
      SKLS_TRY(launch_fill_zero(w.SAc, static_cast<size_t>(ns) * d * sizeof(double), s));
      return with_rowptr(A, [&](auto trt) -> int32_t {
        using TR = decltype(trt);
        hipLaunchKernelGGL((k_gather_csr_dense<TV, TR>), dim3(gr), dim3(kT), 0, s, ns, d,
                           static_cast<const TR*>(A.row_ptr), A.col_idx, static_cast<const TV*>(A.val), w.list,
                           w.wts, w.SAc);
        SKLS_CHECK_LAUNCH();
        return SKLS_OK;
      });
    });
    SKLS_TRY(st);
    hipLaunchKernelGGL(k_gather_rows<double>, dim3(gr), dim3(kT), 0, s, ns, dp, dp, B, w.list, w.wts, w.SBc);
    SKLS_CHECK_LAUNCH();
    SKLS_TRY(run_gram(w.SAc, SKLS_F64, d, nullptr, SKLS_F64, ns, d, w.G, w.gram, w.gram_bytes, s));
    SKLS_TRY(run_cholesky(w.G, d, d, w.R, w.Rinv, w.RinvT, w.status, w.cholw, s));
    SKLS_TRY(to_host(&st_h, w.status, sizeof st_h, s));
    if (st_h) {
      set_error("multi_lstsq: S A is numerically rank deficient (raise t_s)");
      return SKLS_ERR_RANK;
    }
    SKLS_TRY(gemm(true, d, dp, ns, 1.0, w.SAc, d, w.SBc, dp, w.C, dp, w.gs, s));
    SKLS_TRY(gemm(false, d, dp, d, 1.0, w.RinvT, d, w.C, dp, w.Yt, dp, w.gs, s));
    SKLS_TRY(gemm(false, d, dp, d, 1.0, w.Rinv, d, w.Yt, dp, Y, dp, w.gs, s));
    if (rows_out) SKLS_TRY_HIP(hipMemcpyAsync(rows_out, w.list, sizeof(int32_t) * ns, hipMemcpyDeviceToDevice, s));
    if (weights_out)
      SKLS_TRY_HIP(hipMemcpyAsync(weights_out, w.wts, sizeof(double) * ns, hipMemcpyDeviceToDevice, s));
    // ||A Y - B||_F and ||B||_F
    st = with_value(A.dtype, [&](auto tv) -> int32_t {
      using TV = decltype(tv);
      if (A.layout != SKLS_CSR) {
        return dense_times<TV>(n, d, static_cast<const TV*>(A.val), A.ld, Y, dp, w.AY, w.gs, s);
      }
      return with_rowptr(A, [&](auto trt) -> int32_t {
        using TR = decltype(trt);
        return spmm<TV, TR>(A, dpi, Y, w.AY, s);
      });
    });
    SKLS_TRY(st);
    hipLaunchKernelGGL(k_resid_parts, dim3(kResidBlocks), dim3(kT), 0, s, n * dp, w.AY, B, w.part);
    SKLS_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_sum_two, dim3(1), dim3(64), 0, s, w.part, kResidBlocks, w.sums);
    SKLS_CHECK_LAUNCH();
  }
  SKLS_TRY_HIP(hipEventRecord(ev[2], s));
  double sums[2];
  SKLS_TRY(to_host(sums, w.sums, sizeof sums, s));
  inf.resid_fro = std::sqrt(sums[0]);
  inf.b_fro = std::sqrt(sums[1]);
  float ms = 0.0f;
  SKLS_TRY_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
  inf.ms_scores = ms;
  SKLS_TRY_HIP(hipEventElapsedTime(&ms, ev[1], ev[2]));
  inf.ms_solve = ms;
  if (info) *info = inf;
  return SKLS_OK;
}

}  // namespace skls
