// Passes over A for the R-preconditioned Krylov iteration (Section 7.7: a
// conjugate-gradient type method on A R^{-1}, each step costing O(nnz(A) + d^2)).
//
// One streaming pass reads every row of A once and computes, for that row,
//   U_new[i] = A[i, :] p + coef * Z[i]
// and, from the same registers, the partial sums of ||U_new||^2 and of
// A^T U_new.  With p = R^{-1} v, Z = U and coef = -alpha/beta this is the
// bidiagonalisation step of LSQR (Paige & Saunders 1982) with u kept
// unnormalised (A^T (u / beta) = (A^T u) / beta is applied afterwards); with
// p = -x, Z = b and coef = 1 it is the residual r = b - A x together with
// A^T r.  The small float64 d-vector recurrences live in lsqr_step.
#include <type_traits>

#include "kernels.hpp"
#include "profile.hpp"

namespace skls {
namespace {

constexpr int kPassThreads = 256;
constexpr int kPassWaves = kPassThreads / kWave;
constexpr int kRows = 4;  // rows in flight per wavefront

template <typename TV, typename TA, int V>
struct Ld {
  __device__ __forceinline__ static void get(const TV* __restrict__ p, TA (&o)[V]) {
#pragma unroll
    for (int k = 0; k < V; ++k) o[k] = load_as<TA>(p, k);
  }
};
template <typename TA>
struct Ld<float, TA, 4> {
  __device__ __forceinline__ static void get(const float* __restrict__ p, TA (&o)[4]) {
    const nt_f4 x = stream_load<nt_f4>(p);
    o[0] = x[0];
    o[1] = x[1];
    o[2] = x[2];
    o[3] = x[3];
  }
};
template <typename TA>
struct Ld<double, TA, 2> {
  __device__ __forceinline__ static void get(const double* __restrict__ p, TA (&o)[2]) {
    const nt_d2 x = stream_load<nt_d2>(p);
    o[0] = static_cast<TA>(x[0]);
    o[1] = static_cast<TA>(x[1]);
  }
};
template <typename TA>
struct Ld<bf16_t, TA, 8> {
  __device__ __forceinline__ static void get(const bf16_t* __restrict__ p, TA (&o)[8]) {
    const nt_u4 x = stream_load<nt_u4>(p);
    o[0] = bf16_lo(x[0]);
    o[1] = bf16_hi(x[0]);
    o[2] = bf16_lo(x[1]);
    o[3] = bf16_hi(x[1]);
    o[4] = bf16_lo(x[2]);
    o[5] = bf16_hi(x[2]);
    o[6] = bf16_lo(x[3]);
    o[7] = bf16_hi(x[3]);
  }
};

template <typename TA, typename TU, bool ZB>
__device__ __forceinline__ TA load_z(const void* Z, int64_t r) {
  if (ZB) return static_cast<TA>(static_cast<const double*>(Z)[r]);
  return static_cast<TA>(static_cast<const TU*>(Z)[r]);
}

// Dense row-major A.  Lane `lane` owns columns q*64*V + lane*V + [0, V) for
// q < NC; each wavefront streams a contiguous range of rows, kRows at a time.
// Lanes past column d load column 0 instead (their p is 0 and their A^T U is
// never stored), so every load of a step is unconditional and in flight
// together.  ZB: Z is the float64 b (else U).
template <typename TV, typename TA, typename TU, int V, int NC, bool ZB>
__global__ __launch_bounds__(kPassThreads) void k_pass_dense(int64_t n, int d, int64_t ld, const TV* __restrict__ A,
                                                             const double* __restrict__ p,
                                                             const double* __restrict__ coefp, const void* Z,
                                                             TU* U, double* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char smem[];
  TA* red = reinterpret_cast<TA*>(smem);  // [kPassWaves][d]
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const TA coef = static_cast<TA>(coefp[0]);
  TA pv[NC][V], g[NC][V];
  bool live[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int c0 = q * kWave * V + lane * V;
    live[q] = c0 < d;
#pragma unroll
    for (int k = 0; k < V; ++k) {
      pv[q][k] = live[q] ? static_cast<TA>(p[c0 + k]) : TA(0);
      g[q][k] = TA(0);
    }
  }
  TA un = TA(0);
  const int64_t gw = static_cast<int64_t>(blockIdx.x) * kPassWaves + wid;
  const int64_t nw = static_cast<int64_t>(gridDim.x) * kPassWaves;
  const int64_t r0 = gw * n / nw, r1 = (gw + 1) * n / nw;
  int64_t r = r0;
  int cl[NC];  // this lane's first column of each slice (0 past d)
#pragma unroll
  for (int q = 0; q < NC; ++q) cl[q] = live[q] ? q * kWave * V + lane * V : 0;
  for (; r + kRows <= r1; r += kRows) {
    TA x[kRows][NC][V];
    TA z[kRows];
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
#pragma unroll
      for (int q = 0; q < NC; ++q) Ld<TV, TA, V>::get(A + static_cast<size_t>(r + j) * ld + cl[q], x[j][q]);
      z[j] = load_z<TA, TU, ZB>(Z, r + j);
    }
    TA dot[kRows];
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      TA s = TA(0);
#pragma unroll
      for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int k = 0; k < V; ++k) s += pv[q][k] * x[j][q][k];
      dot[j] = s;
    }
#pragma unroll
    for (int j = 0; j < kRows; ++j) dot[j] = wave_total(dot[j]);
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      const TA u = dot[j] + coef * z[j];
      if (lane == 0) U[r + j] = static_cast<TU>(u);
      un += u * u;
#pragma unroll
      for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int k = 0; k < V; ++k) g[q][k] += u * x[j][q][k];
    }
  }
  for (; r < r1; ++r) {
    TA x[NC][V];
    TA s = TA(0);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      Ld<TV, TA, V>::get(A + static_cast<size_t>(r) * ld + cl[q], x[q]);
#pragma unroll
      for (int k = 0; k < V; ++k) s += pv[q][k] * x[q][k];
    }
    s = wave_total(s);
    const TA u = s + coef * load_z<TA, TU, ZB>(Z, r);
    if (lane == 0) U[r] = static_cast<TU>(u);
    un += u * u;
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
      for (int k = 0; k < V; ++k) g[q][k] += u * x[q][k];
  }
  // block reduction of g (fixed order) and of ||U_new||^2
#pragma unroll
  for (int q = 0; q < NC; ++q)
    if (live[q])
#pragma unroll
      for (int k = 0; k < V; ++k) red[wid * d + q * kWave * V + lane * V + k] = g[q][k];
  TA* unr = red + kPassWaves * d;
  if (lane == 0) unr[wid] = un;
  __syncthreads();
  double* out = partial + static_cast<size_t>(blockIdx.x) * (d + 1);
  for (int c = threadIdx.x; c < d; c += kPassThreads) {
    double s = 0.0;
    for (int w = 0; w < kPassWaves; ++w) s += static_cast<double>(red[w * d + c]);
    out[c] = s;
  }
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kPassWaves; ++w) s += static_cast<double>(unr[w]);
    out[d] = s;
  }
}

// CSR A: a group of L lanes per row; A^T U_new accumulated in LDS with
// compare-and-swap adds.  ZB: Z is the float64 b (else U).
template <typename TV, typename TR, typename TA, typename TU, int L, bool ZB>
__global__ __launch_bounds__(kPassThreads) void k_pass_csr(int64_t n, int d, const TR* __restrict__ row_ptr,
                                                           const int32_t* __restrict__ col, const TV* __restrict__ val,
                                                           const double* __restrict__ p,
                                                           const double* __restrict__ coefp, const void* Z, TU* U,
                                                           double* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char smem[];
  TA* sp = reinterpret_cast<TA*>(smem);
  TA* gacc = sp + d;
  TA* scratch = gacc + d;
  for (int c = threadIdx.x; c < d; c += kPassThreads) {
    sp[c] = static_cast<TA>(p[c]);
    gacc[c] = TA(0);
  }
  __syncthreads();
  const TA coef = static_cast<TA>(coefp[0]);
  const int sub = threadIdx.x % L;
  const int64_t grp = (blockIdx.x * static_cast<int64_t>(kPassThreads) + threadIdx.x) / L;
  const int64_t ngrp = static_cast<int64_t>(gridDim.x) * kPassThreads / L;
  TA un = TA(0);
  for (int64_t r = grp; r < n; r += ngrp) {
    const TR a = row_ptr[r], e = row_ptr[r + 1];
    TA s = TA(0);
    for (TR k = a + sub; k < e; k += L) s += load_as<TA>(val, static_cast<size_t>(k)) * sp[col[k]];
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
    const TA u = s + coef * load_z<TA, TU, ZB>(Z, r);
    if (sub == 0) {
      U[r] = static_cast<TU>(u);
      un += u * u;
    }
    for (TR k = a + sub; k < e; k += L) lds_add1(gacc, col[k], u * load_as<TA>(val, static_cast<size_t>(k)));
  }
  const TA tot = block_sum(un, scratch);
  __syncthreads();
  double* out = partial + static_cast<size_t>(blockIdx.x) * (d + 1);
  for (int c = threadIdx.x; c < d; c += kPassThreads) out[c] = static_cast<double>(gacc[c]);
  if (threadIdx.x == 0) out[d] = static_cast<double>(tot);
}

// partial[nblk][cols] -> tmp[S2][cols] -> out[cols]
__global__ __launch_bounds__(256) void k_reduce_cols(const double* __restrict__ partial, int nblk, int cols,
                                                     int rows_per, double* __restrict__ tmp) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  const int b0 = blockIdx.y * rows_per;
  int b1 = b0 + rows_per;
  if (b1 > nblk) b1 = nblk;
  double s = 0.0;
  for (int b = b0; b < b1; ++b) s += partial[static_cast<size_t>(b) * cols + c];
  tmp[static_cast<size_t>(blockIdx.y) * cols + c] = s;
}

__global__ __launch_bounds__(256) void k_reduce_final(const double* __restrict__ tmp, int S2, int cols,
                                                      double* __restrict__ out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int b = 0; b < S2; ++b) s += tmp[static_cast<size_t>(b) * cols + c];
  out[c] = s;
}

template <typename F>
int32_t with_val(int32_t dt, F&& f) {
  switch (dt) {
    case SKLS_F64: return f(double{});
    case SKLS_F32: return f(float{});
    case SKLS_BF16: return f(bf16_t{});
    default: set_error("unsupported value dtype %d", dt); return SKLS_ERR_DTYPE;
  }
}

template <typename F>
int32_t with_nc(int nc, F&& f) {
  switch (nc) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 3:
    case 4: return f(std::integral_constant<int, 4>{});
    default: return f(std::integral_constant<int, 8>{});
  }
}

template <typename TV, typename TA, typename TU>
int32_t launch_pass_dense(const PassArgs& a, hipStream_t s) {
  const skls_matrix& A = *a.A;
  const int d = static_cast<int>(A.d);
  constexpr int VV = sizeof(TV) == 8 ? 2 : (sizeof(TV) == 4 ? 4 : 8);
  const bool vec = (reinterpret_cast<uintptr_t>(A.val) % 16 == 0) && ((A.ld * sizeof(TV)) % 16 == 0) && (d % VV == 0);
  const size_t lds = (static_cast<size_t>(kPassWaves) * d + kPassWaves) * sizeof(TA);
  auto go = [&](auto vc) -> int32_t {
    constexpr int V = decltype(vc)::value;
    const int nc = static_cast<int>(div_up(d, kWave * V));
    if (nc > 8) {
      set_error("dense pass supports d <= %d for this dtype", 8 * kWave * V);
      return SKLS_ERR_SHAPE;
    }
    return with_nc(nc, [&](auto ncc) -> int32_t {
      constexpr int NC = decltype(ncc)::value;
      if (a.z_is_b) {
        hipLaunchKernelGGL((k_pass_dense<TV, TA, TU, V, NC, true>), dim3(a.nblk), dim3(kPassThreads), lds, s, A.n, d,
                           A.ld, static_cast<const TV*>(A.val), a.p, a.coef, a.Z, static_cast<TU*>(a.U), a.partial);
      } else {
        hipLaunchKernelGGL((k_pass_dense<TV, TA, TU, V, NC, false>), dim3(a.nblk), dim3(kPassThreads), lds, s, A.n,
                           d, A.ld, static_cast<const TV*>(A.val), a.p, a.coef, a.Z, static_cast<TU*>(a.U),
                           a.partial);
      }
      SKLS_CHECK_LAUNCH();
      return SKLS_OK;
    });
  };
  if (vec) return go(std::integral_constant<int, VV>{});
  return go(std::integral_constant<int, 1>{});
}

template <typename TV, typename TA, typename TU>
int32_t launch_pass_csr(const PassArgs& a, hipStream_t s) {
  const skls_matrix& A = *a.A;
  const int d = static_cast<int>(A.d);
  const size_t lds = (2 * static_cast<size_t>(d) + kPassWaves) * sizeof(TA);
  if (lds > 65536) {
    set_error("CSR pass supports d <= %zu for this precision", (65536 / sizeof(TA) - kPassWaves) / 2);
    return SKLS_ERR_SHAPE;
  }
  const double avg = A.n > 0 ? static_cast<double>(A.nnz) / static_cast<double>(A.n) : 1.0;
  auto go = [&](auto tr, auto lc) -> int32_t {
    using TR = decltype(tr);
    constexpr int L = decltype(lc)::value;
    if (a.z_is_b) {
      hipLaunchKernelGGL((k_pass_csr<TV, TR, TA, TU, L, true>), dim3(a.nblk), dim3(kPassThreads), lds, s, A.n, d,
                         static_cast<const TR*>(A.row_ptr), A.col_idx, static_cast<const TV*>(A.val), a.p, a.coef,
                         a.Z, static_cast<TU*>(a.U), a.partial);
    } else {
      hipLaunchKernelGGL((k_pass_csr<TV, TR, TA, TU, L, false>), dim3(a.nblk), dim3(kPassThreads), lds, s, A.n, d,
                         static_cast<const TR*>(A.row_ptr), A.col_idx, static_cast<const TV*>(A.val), a.p, a.coef,
                         a.Z, static_cast<TU*>(a.U), a.partial);
    }
    SKLS_CHECK_LAUNCH();
    return SKLS_OK;
  };
  auto pick_l = [&](auto tr) -> int32_t {
    if (avg <= 6.0) return go(tr, std::integral_constant<int, 4>{});
    if (avg <= 24.0) return go(tr, std::integral_constant<int, 16>{});
    return go(tr, std::integral_constant<int, 64>{});
  };
  if (A.row_ptr_64) return pick_l(int64_t{});
  return pick_l(int32_t{});
}

}  // namespace

int32_t pass_blocks(const skls_matrix& A) {
  // enough blocks to cover the 256 compute units several times over while
  // keeping the partial sums small
  int64_t rows_per_wave = A.layout == SKLS_DENSE ? 64 : 256;
  int64_t b = div_up(A.n, rows_per_wave * kPassWaves);
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return static_cast<int32_t>(b);
}

int32_t run_pass(const PassArgs& a, hipStream_t s) {
  const skls_matrix& A = *a.A;
  PhaseTimer pt(a.acc_f64 ? "lsqr_pass_f64" : "lsqr_pass_f32", s);
  return with_val(A.dtype, [&](auto tv) -> int32_t {
    using TV = decltype(tv);
    if (a.acc_f64 && a.u_f64)
      return A.layout == SKLS_DENSE ? launch_pass_dense<TV, double, double>(a, s)
                                    : launch_pass_csr<TV, double, double>(a, s);
    if (a.acc_f64 && !a.u_f64)
      return A.layout == SKLS_DENSE ? launch_pass_dense<TV, double, float>(a, s)
                                    : launch_pass_csr<TV, double, float>(a, s);
    if (!a.acc_f64 && !a.u_f64)
      return A.layout == SKLS_DENSE ? launch_pass_dense<TV, float, float>(a, s)
                                    : launch_pass_csr<TV, float, float>(a, s);
    set_error("internal: float32 accumulation with a float64 U is not used");
    return SKLS_ERR_ARG;
  });
}

int32_t run_reduce_partials(const double* partial, int32_t nblk, int64_t d, double* out, double* tmp,
                            hipStream_t s) {
  const int cols = static_cast<int>(d + 1);
  const int rows_per = 32;
  const int S2 = static_cast<int>(div_up(nblk, rows_per));
  hipLaunchKernelGGL(k_reduce_cols, dim3(static_cast<unsigned>(div_up(cols, 256)), S2), dim3(256), 0, s, partial,
                     nblk, cols, rows_per, tmp);
  SKLS_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_reduce_final, dim3(static_cast<unsigned>(div_up(cols, 256))), dim3(256), 0, s, tmp, S2, cols,
                     out);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

}  // namespace skls

// ================================================================ LSQR recurrences
// Float64 scalars of the Paige-Saunders recurrence, kept on the device so
// that the host only reads them to decide when to stop.
namespace skls {
namespace {

// Thread 0 copies the state into the host mirror (when given) after writing
// it, so a host that waits for the stream reads it without a copy.
__device__ __forceinline__ void mirror_state(const double* __restrict__ st, double* __restrict__ mir) {
  if (mir == nullptr) return;
#pragma unroll
  for (int k = 0; k < LSQR_NSTATE; ++k) mir[k] = st[k];
}

__global__ __launch_bounds__(256) void k_lsqr_init(const double* __restrict__ gsum, const double* __restrict__ vp,
                                                   int d, double* __restrict__ v, double* __restrict__ w,
                                                   double* __restrict__ y, double* __restrict__ st,
                                                   double* __restrict__ mir, const int32_t* __restrict__ flag,
                                                   const double* __restrict__ extra) {
  __shared__ double scratch[4];
  const double beta = sqrt(gsum[d]);
  const double ib = beta > 0.0 ? 1.0 / beta : 0.0;
  double ss = 0.0;
  for (int c = threadIdx.x; c < d; c += 256) {
    const double t = vp[c] * ib;
    v[c] = t;
    ss += t * t;
  }
  const double alpha = sqrt(block_sum(ss, scratch));
  const double ia = alpha > 0.0 ? 1.0 / alpha : 0.0;
  for (int c = threadIdx.x; c < d; c += 256) {
    v[c] *= ia;
    w[c] = v[c];
    y[c] = 0.0;
  }
  if (threadIdx.x == 0) {
    st[LSQR_ALPHA] = alpha;
    st[LSQR_BETA] = beta;
    st[LSQR_RHOBAR] = alpha;
    st[LSQR_PHIBAR] = beta;
    st[LSQR_COEF] = beta > 0.0 ? -alpha / beta : 0.0;
    st[LSQR_RNORM] = beta;
    st[LSQR_ARNORM] = alpha * beta;
    st[LSQR_EST_R] = beta;
    st[LSQR_EST_AR] = alpha * beta;
    st[LSQR_ONE] = 1.0;
    st[LSQR_DONE] = (alpha > 0.0 && beta > 0.0) ? 0.0 : 1.0;
    st[LSQR_STOP] = 0.0;
    st[LSQR_COUNT] = 0.0;
    mirror_state(st, mir);
    if (mir != nullptr) {
      mir[LSQR_NSTATE] = flag != nullptr ? static_cast<double>(*flag) : 0.0;
      mir[LSQR_NSTATE + 1] = extra != nullptr ? *extra : 0.0;
    }
  }
}

__global__ __launch_bounds__(256) void k_lsqr_step(const double* __restrict__ gsum, const double* __restrict__ vp,
                                                   int d, double* __restrict__ v, double* __restrict__ w,
                                                   double* __restrict__ y, double* __restrict__ st, double target,
                                                   double* __restrict__ mir) {
  __shared__ double scratch[4];
  // read by every thread before thread 0 writes it below (after a barrier)
  if (st[LSQR_STOP] != 0.0) return;
  const double beta = sqrt(gsum[d]);
  const double ib = beta > 0.0 ? 1.0 / beta : 0.0;
  double ss = 0.0;
  for (int c = threadIdx.x; c < d; c += 256) {
    const double t = vp[c] * ib - beta * v[c];
    v[c] = t;
    ss += t * t;
  }
  const double alpha = sqrt(block_sum(ss, scratch));
  const double ia = alpha > 0.0 ? 1.0 / alpha : 0.0;
  const double rhobar = st[LSQR_RHOBAR], phibar = st[LSQR_PHIBAR];
  const double rho = hypot(rhobar, beta);
  const double c = rho > 0.0 ? rhobar / rho : 1.0;
  const double s = rho > 0.0 ? beta / rho : 0.0;
  const double theta = s * alpha;
  const double phi = c * phibar;
  const double t1 = rho > 0.0 ? phi / rho : 0.0;
  const double t2 = rho > 0.0 ? -theta / rho : 0.0;
  for (int k = threadIdx.x; k < d; k += 256) {
    const double vn = v[k] * ia;
    const double wk = w[k];
    y[k] += t1 * wk;
    w[k] = vn + t2 * wk;
    v[k] = vn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double phibar_new = s * phibar;
    st[LSQR_ALPHA] = alpha;
    st[LSQR_BETA] = beta;
    st[LSQR_RHOBAR] = -c * alpha;
    st[LSQR_PHIBAR] = phibar_new;
    st[LSQR_COEF] = beta > 0.0 ? -alpha / beta : 0.0;
    const double est_ar = phibar_new * alpha * fabs(c);
    const bool done = !(alpha > 0.0 && beta > 0.0);
    st[LSQR_EST_R] = phibar_new;
    st[LSQR_EST_AR] = est_ar;
    st[LSQR_DONE] = done ? 1.0 : 0.0;
    st[LSQR_COUNT] += 1.0;
    st[LSQR_STOP] = (done || est_ar <= target * phibar_new) ? 1.0 : 0.0;
    mirror_state(st, mir);
  }
}

__global__ void k_axpy_neg(const double* __restrict__ x, int d, double a, double* __restrict__ y,
                           double* __restrict__ one) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < d; c += gridDim.x * blockDim.x) y[c] = a * x[c];
  if (one != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *one = 1.0;
}

__global__ void k_add(double* __restrict__ x, const double* __restrict__ t, int d) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < d; c += gridDim.x * blockDim.x) x[c] += t[c];
}

}  // namespace

int32_t run_lsqr_init(const double* gsum, const double* vp, int64_t d, double* v, double* w, double* y, double* st,
                      hipStream_t s, double* mirror, const int32_t* flag, const double* extra) {
  hipLaunchKernelGGL(k_lsqr_init, dim3(1), dim3(256), 0, s, gsum, vp, static_cast<int>(d), v, w, y, st, mirror, flag,
                     extra);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t run_lsqr_step(const double* gsum, const double* vp, int64_t d, double* v, double* w, double* y, double* st,
                      double target, hipStream_t s, double* mirror) {
  hipLaunchKernelGGL(k_lsqr_step, dim3(1), dim3(256), 0, s, gsum, vp, static_cast<int>(d), v, w, y, st, target,
                     mirror);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t lsqr_mirror(double** host, double** dev) {
  thread_local double* h = nullptr;
  if (h == nullptr) {
    void* q = nullptr;
    SKLS_TRY_HIP(hipHostMalloc(&q, sizeof(double) * (LSQR_NSTATE + 2), hipHostMallocCoherent));
    h = static_cast<double*>(q);
  }
  *host = h;
  SKLS_TRY_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(dev), h, 0));
  return SKLS_OK;
}

int32_t run_scale(const double* x, int64_t d, double a, double* y, hipStream_t s, double* one) {
  hipLaunchKernelGGL(k_axpy_neg, dim3(static_cast<unsigned>(div_up(d, 256))), dim3(256), 0, s, x, static_cast<int>(d),
                     a, y, one);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t run_add(double* x, const double* t, int64_t d, hipStream_t s) {
  hipLaunchKernelGGL(k_add, dim3(static_cast<unsigned>(div_up(d, 256))), dim3(256), 0, s, x, t, static_cast<int>(d));
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

}  // namespace skls
