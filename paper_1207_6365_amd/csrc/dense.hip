// Dense float64 linear algebra on the sketch (Section 7: the sketched
// regression is solved through a QR factorisation of S A and R^{-1} Q^T S b).
//
// R is obtained as the Cholesky factor of the Gram matrix (S A)^T (S A)
// (CholeskyQR): the Gram of the augmented matrix [S A | S b] is a dense
// contraction over the t sketch rows and runs on the float64 matrix cores
// (v_mfma_f64_16x16x4f64) with split-K partial tiles; the Cholesky of the
// small d x d Gram, the triangular inverse and the d x d products run on
// vector units.  In exact arithmetic this R equals the R of a QR
// factorisation of S A with positive diagonal, and Q^T S b = R^{-T} (S A)^T S b.
#include <cmath>
#include <type_traits>

#include "kernels.hpp"
#include "profile.hpp"

namespace skls {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int kGT = 64;          // Gram output tile (kGT x kGT per block)
constexpr int kGK = 16;          // sketch rows staged in LDS per step
constexpr int kGThreads = 256;   // 4 waves, each 32 x 32 of the tile

template <typename TI>
__device__ __forceinline__ double gram_elem(const TI* __restrict__ M, int64_t ld, const void* __restrict__ v,
                                            int v_f64, int64_t k, int c, int d) {
  if (c < d) return load_as<double>(M, static_cast<size_t>(k) * ld + c);
  if (c == d && v != nullptr)
    return v_f64 ? static_cast<const double*>(v)[k] : static_cast<double>(static_cast<const float*>(v)[k]);
  return 0.0;
}

__device__ __forceinline__ void tile_of(int p, int T, int& ti, int& tj) {
  ti = 0;
  while (p >= T - ti) {
    p -= T - ti;
    ++ti;
  }
  tj = ti + p;
}

// Partial Gram tile over the rows of one split: partial[split][pair][64][64].
template <typename TI>
__global__ __launch_bounds__(kGThreads) void k_gram_partial(const TI* __restrict__ M, int64_t ld,
                                                            const void* __restrict__ v, int v_f64, int64_t m, int d,
                                                            int T, int64_t rows_per_split,
                                                            double* __restrict__ partial) {
  __shared__ double As[kGK][kGT];
  __shared__ double Bs[kGK][kGT];
  int ti, tj;
  tile_of(blockIdx.x, T, ti, tj);
  const int I0 = ti * kGT, J0 = tj * kGT;
  const int64_t k0 = static_cast<int64_t>(blockIdx.y) * rows_per_split;
  const int64_t k1 = (k0 + rows_per_split < m) ? k0 + rows_per_split : m;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int wi = wv >> 1, wj = wv & 1;
  const int lr = lane >> 4, lc = lane & 15;
  d4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};
  for (int64_t kb = k0; kb < k1; kb += kGK) {
    __syncthreads();
    for (int e = threadIdx.x; e < kGK * kGT; e += kGThreads) {
      const int r = e / kGT, c = e % kGT;
      const int64_t k = kb + r;
      const bool in = k < k1;
      As[r][c] = in ? gram_elem(M, ld, v, v_f64, k, I0 + c, d) : 0.0;
      Bs[r][c] = in ? gram_elem(M, ld, v, v_f64, k, J0 + c, d) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 4) {
      const double a0 = As[kk + lr][wi * 32 + lc];
      const double a1 = As[kk + lr][wi * 32 + 16 + lc];
      const double b0 = Bs[kk + lr][wj * 32 + lc];
      const double b1 = Bs[kk + lr][wj * 32 + 16 + lc];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
  // Output layout of v_mfma_f64_16x16x4f64: element e of lane l holds row
  // (l / 16) + 4 e, column l % 16 of the 16 x 16 block (checked on gfx950).
  double* out = partial + (static_cast<size_t>(blockIdx.y) * gridDim.x + blockIdx.x) * (kGT * kGT);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = wi * 32 + a * 16 + lr + 4 * e;
        const int colx = wj * 32 + b * 16 + lc;
        out[row * kGT + colx] = acc[a][b][e];
      }
}

__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ partial, int P, int S, int T, int dd,
                                                     double* __restrict__ G) {
  const int p = blockIdx.x;
  const int idx = blockIdx.y * 256 + threadIdx.x;
  double s = 0.0;
  for (int sp = 0; sp < S; ++sp) s += partial[(static_cast<size_t>(sp) * P + p) * (kGT * kGT) + idx];
  int ti, tj;
  tile_of(p, T, ti, tj);
  const int i = ti * kGT + idx / kGT, j = tj * kGT + idx % kGT;
  // diagonal tiles hold both (i, j) and (j, i): write each pair once
  if (i < dd && j < dd && (ti != tj || i <= j)) {
    G[static_cast<size_t>(i) * dd + j] = s;
    G[static_cast<size_t>(j) * dd + i] = s;
  }
}

// ---------------------------------------------------------------- blocked Cholesky
// Upper Cholesky G = R^T R in place on a d x d row-major copy W, by blocks of
// kCB rows: factor the diagonal block in LDS (and invert it), solve for the
// block row to its right, then update the trailing upper triangle.
constexpr int kCB = 64;

// W[K:K+kb, K:K+kb] -> R_KK (in place) and Kinv = R_KK^{-1} (kb x kb, ld kCB).
// LDS holds R_KK in the upper triangle of `a`; the inverse is built column by
// column (one thread per column) in the strict lower triangle, transposed,
// with its diagonal in the spare column kCB.
__global__ __launch_bounds__(256) void k_chol_diag(double* __restrict__ W, int d, int K, double* __restrict__ Kinv,
                                                   int32_t* __restrict__ bad) {
  __shared__ double a[kCB][kCB + 1];
  const int kb = (d - K) < kCB ? (d - K) : kCB;
  const int tid = threadIdx.x;
  for (int e = tid; e < kCB * (kCB + 1); e += 256) {
    const int i = e / (kCB + 1), j = e % (kCB + 1);
    a[i][j] = (i < kb && j < kb && j >= i) ? W[static_cast<size_t>(K + i) * d + K + j] : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < kb; ++k) {
    if (tid == 0) {
      double piv = a[k][k];
      if (!(piv > 0.0)) {
        bad[0] = 1;
        piv = 1.0;
      }
      a[k][k] = sqrt(piv);
    }
    __syncthreads();
    const double r = a[k][k];
    for (int j = k + 1 + tid; j < kb; j += 256) a[k][j] /= r;
    __syncthreads();
    const int nrem = kb - k - 1;
    for (int e = tid; e < nrem * nrem; e += 256) {
      const int i = k + 1 + e / nrem, j = k + 1 + e % nrem;
      if (j >= i) a[i][j] -= a[k][i] * a[k][j];
    }
    __syncthreads();
  }
  if (tid < kb) {
    const int j = tid;  // column j of the inverse: inv[i][j] kept at a[j][i] (i < j), inv[j][j] at a[j][kCB]
    a[j][kCB] = 1.0 / a[j][j];
    for (int i = j - 1; i >= 0; --i) {
      double s = a[i][j] * a[j][kCB];
      for (int l = i + 1; l < j; ++l) s += a[i][l] * a[j][l];
      a[j][i] = -s / a[i][i];
    }
  }
  __syncthreads();
  for (int e = tid; e < kb * kb; e += 256) {
    const int i = e / kb, j = e % kb;
    if (j >= i) W[static_cast<size_t>(K + i) * d + K + j] = a[i][j];
    Kinv[i * kCB + j] = (i == j) ? a[j][kCB] : (i < j ? a[j][i] : 0.0);
  }
}

constexpr int kCL = 32;  // rows of the panels staged per step

// Block row solve: W[K:K+kb, J0:J0+64] <- R_KK^{-T} W[K:K+kb, J0:J0+64].
__global__ __launch_bounds__(256) void k_chol_trsm(double* __restrict__ W, int d, int K,
                                                   const double* __restrict__ Kinv) {
  __shared__ double ki[kCL][kCB + 1];
  __shared__ double p[kCL][kCB + 1];
  const int kb = (d - K) < kCB ? (d - K) : kCB;
  const int J0 = K + kb + blockIdx.x * kCB;
  const int tid = threadIdx.x;
  const int j = tid % kCB, i0 = tid / kCB;  // this thread: rows i0, i0+4, ..., column j
  double acc[kCB / 4];
#pragma unroll
  for (int q = 0; q < kCB / 4; ++q) acc[q] = 0.0;
  for (int l0 = 0; l0 < kb; l0 += kCL) {
    __syncthreads();
    for (int e = tid; e < kCL * kCB; e += 256) {
      const int l = e / kCB, c = e % kCB;
      ki[l][c] = (l0 + l < kb && c < kb) ? Kinv[(l0 + l) * kCB + c] : 0.0;
      p[l][c] = (l0 + l < kb && J0 + c < d) ? W[static_cast<size_t>(K + l0 + l) * d + J0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kCB / 4; ++q) {
      const int i = i0 + 4 * q;
      double s = 0.0;
      for (int l = 0; l < kCL; ++l) s += ki[l][i] * p[l][j];  // Kinv is upper: ki[l][i] = 0 for l > i
      acc[q] += s;
    }
  }
  __syncthreads();  // every panel row is read before any is overwritten
  if (J0 + j < d) {
#pragma unroll
    for (int q = 0; q < kCB / 4; ++q) {
      const int i = i0 + 4 * q;
      if (i < kb) W[static_cast<size_t>(K + i) * d + J0 + j] = acc[q];
    }
  }
}

// Trailing update of the upper tile (I0, J0): W[I, J] -= R_KI^T R_KJ.
__global__ __launch_bounds__(256) void k_chol_syrk(double* __restrict__ W, int d, int K) {
  __shared__ double pi[kCL][kCB + 1];
  __shared__ double pj[kCL][kCB + 1];
  const int kb = (d - K) < kCB ? (d - K) : kCB;
  const int T0 = K + kb;
  const int nt = (d - T0 + kCB - 1) / kCB;
  int p = blockIdx.x, ti = 0;
  while (p >= nt - ti) {
    p -= nt - ti;
    ++ti;
  }
  const int I0 = T0 + ti * kCB, J0 = T0 + (ti + p) * kCB;
  const int tid = threadIdx.x;
  const int j = tid % kCB, i0 = tid / kCB;
  double acc[kCB / 4];
#pragma unroll
  for (int q = 0; q < kCB / 4; ++q) acc[q] = 0.0;
  for (int l0 = 0; l0 < kb; l0 += kCL) {
    __syncthreads();
    for (int e = tid; e < kCL * kCB; e += 256) {
      const int l = e / kCB, c = e % kCB;
      const bool in = l0 + l < kb;
      pi[l][c] = (in && I0 + c < d) ? W[static_cast<size_t>(K + l0 + l) * d + I0 + c] : 0.0;
      pj[l][c] = (in && J0 + c < d) ? W[static_cast<size_t>(K + l0 + l) * d + J0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kCB / 4; ++q) {
      const int i = i0 + 4 * q;
      double s = 0.0;
      for (int l = 0; l < kCL; ++l) s += pi[l][i] * pj[l][j];
      acc[q] += s;
    }
  }
#pragma unroll
  for (int q = 0; q < kCB / 4; ++q) {
    const int i = i0 + 4 * q;
    if (I0 + i < d && J0 + j < d && J0 + j >= I0 + i) W[static_cast<size_t>(I0 + i) * d + J0 + j] -= acc[q];
  }
}

// R = upper triangle of W; status = rank test on the diagonal.
__global__ __launch_bounds__(256) void k_chol_finish(const double* __restrict__ W, int d, double* __restrict__ R,
                                                     const int32_t* __restrict__ bad, int32_t* __restrict__ status,
                                                     double rtol) {
  for (int64_t idx = blockIdx.x * 256 + threadIdx.x; idx < static_cast<int64_t>(d) * d;
       idx += static_cast<int64_t>(gridDim.x) * 256) {
    const int i = static_cast<int>(idx / d), j = static_cast<int>(idx % d);
    R[idx] = j >= i ? W[idx] : 0.0;
  }
  if (blockIdx.x == 0) {
    __shared__ double smx[256], smn[256];
    double mx = 0.0, mn = INFINITY;
    for (int k = threadIdx.x; k < d; k += 256) {
      const double r = W[static_cast<size_t>(k) * d + k];
      mx = r > mx ? r : mx;
      mn = r < mn ? r : mn;
    }
    smx[threadIdx.x] = mx;
    smn[threadIdx.x] = mn;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int k = 1; k < 256; ++k) {
        mx = smx[k] > mx ? smx[k] : mx;
        mn = smn[k] < mn ? smn[k] : mn;
      }
      status[0] = (bad[0] || !(mn > rtol * mx)) ? 1 : 0;
    }
  }
}

__global__ void k_copy_upper(const double* __restrict__ G, int64_t ldg, int d, double* __restrict__ W,
                             int32_t* __restrict__ bad) {
  for (int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; idx < static_cast<int64_t>(d) * d;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int i = static_cast<int>(idx / d), j = static_cast<int>(idx % d);
    W[idx] = j >= i ? G[static_cast<size_t>(i) * ldg + j] : 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) bad[0] = 0;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Column j of R^{-1} by back substitution, one wavefront per column.
__global__ __launch_bounds__(kWave) void k_trinv(const double* __restrict__ R, int d, double* __restrict__ Rinv,
                                                 double* __restrict__ RinvT) {
  extern __shared__ double x[];
  const int lane = threadIdx.x;
  const int j = blockIdx.x;
  if (lane == 0) x[j] = 1.0 / R[static_cast<size_t>(j) * d + j];
  wave_sync();
  for (int i = j - 1; i >= 0; --i) {
    double s = 0.0;
    const double* row = R + static_cast<size_t>(i) * d;
    for (int k = i + 1 + lane; k <= j; k += kWave) s += row[k] * x[k];
    s = wave_sum(s);
    if (lane == 0) x[i] = -s / row[i];
    wave_sync();
  }
  for (int i = lane; i < d; i += kWave) {
    const double v = i <= j ? x[i] : 0.0;
    Rinv[static_cast<size_t>(i) * d + j] = v;
    RinvT[static_cast<size_t>(j) * d + i] = v;
  }
}

// y = M x, one wavefront per row of the d x d row-major M.
__global__ __launch_bounds__(256) void k_gemv(const double* __restrict__ M, int d, const double* __restrict__ x,
                                              double* __restrict__ y) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int row = blockIdx.x * 4 + wid;
  if (row >= d) return;
  const double* m = M + static_cast<size_t>(row) * d;
  double s = 0.0;
  for (int k = lane; k < d; k += kWave) s += m[k] * x[k];
  s = wave_sum(s);
  if (lane == 0) y[row] = s;
}

// T = R^{-1} P (d x d upper times d x k), float64 sums rounded to float32.
__global__ void k_rinv_times(const double* __restrict__ Rinv, int d, const double* __restrict__ P, int k,
                             float* __restrict__ T) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= static_cast<int64_t>(d) * k) return;
  const int i = static_cast<int>(idx / k), q = static_cast<int>(idx % k);
  double s = 0.0;
  for (int j = i; j < d; ++j) s += Rinv[static_cast<size_t>(i) * d + j] * P[static_cast<size_t>(j) * k + q];
  T[idx] = static_cast<float>(s);
}

__global__ void k_f64_to_f32(const double* __restrict__ in, float* __restrict__ out, int64_t count) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[i] = static_cast<float>(in[i]);
}

struct GramShape {
  int T, P, S;
  int64_t rps;
};

GramShape gram_shape(int64_t m, int64_t dd) {
  GramShape g;
  g.T = static_cast<int>(div_up(dd, kGT));
  g.P = g.T * (g.T + 1) / 2;
  int64_t S = div_up(2048, g.P);
  const int64_t max_split = div_up(m, 256);
  if (S > max_split) S = max_split;
  if (S < 1) S = 1;
  g.rps = div_up(div_up(m, S), kGK) * kGK;
  g.S = static_cast<int>(div_up(m, g.rps));
  if (g.S < 1) g.S = 1;
  return g;
}

}  // namespace

size_t gram_ws_bytes(int64_t m, int64_t dd) {
  const GramShape g = gram_shape(m, dd);
  return static_cast<size_t>(g.S) * g.P * kGT * kGT * sizeof(double) + 256;
}

int32_t run_gram(const void* M, int32_t dtype, int64_t ld, const void* v, int32_t v_dtype, int64_t m, int64_t d,
                 double* G, void* ws, size_t ws_bytes, hipStream_t s) {
  const int64_t dd = d + (v ? 1 : 0);
  const GramShape g = gram_shape(m, dd);
  if (ws_bytes < gram_ws_bytes(m, dd) || ws == nullptr) {
    set_error("gram workspace too small");
    return SKLS_ERR_WORKSPACE;
  }
  double* partial = static_cast<double*>(ws);
  const int v_f64 = v_dtype == SKLS_F64 ? 1 : 0;
  PhaseTimer pt("gram", s);
  auto launch = [&](auto tag) -> int32_t {
    using TI = decltype(tag);
    hipLaunchKernelGGL((k_gram_partial<TI>), dim3(g.P, g.S), dim3(kGThreads), 0, s, static_cast<const TI*>(M), ld,
                       v, v_f64, m, static_cast<int>(d), g.T, g.rps, partial);
    SKLS_CHECK_LAUNCH();
    return SKLS_OK;
  };
  int32_t st;
  switch (dtype) {
    case SKLS_F64: st = launch(double{}); break;
    case SKLS_F32: st = launch(float{}); break;
    case SKLS_BF16: st = launch(bf16_t{}); break;
    default: set_error("gram: bad dtype"); return SKLS_ERR_DTYPE;
  }
  if (st != SKLS_OK) return st;
  hipLaunchKernelGGL(k_gram_reduce, dim3(g.P, kGT * kGT / 256), dim3(256), 0, s, partial, g.P, g.S, g.T,
                     static_cast<int>(dd), G);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

size_t cholesky_scratch_doubles(int64_t d) { return static_cast<size_t>(d * d) + kCB * kCB + 8; }

int32_t run_cholesky(const double* G, int64_t ldg, int64_t d, double* R, int32_t* status, double* scratch,
                     hipStream_t s) {
  // Threshold: a Gram-based factor cannot resolve |R_kk| below about
  // sqrt(d * eps) * max |R_jj|; treat that as numerical rank deficiency.
  const double rtol = 4.0 * std::sqrt(static_cast<double>(d) * 2.220446049250313e-16);
  PhaseTimer pt("cholesky", s);
  // scratch: W [d*d] | Kinv [kCB*kCB] | bad flag
  double* W = scratch;
  double* Kinv = scratch + d * d;
  int32_t* bad = reinterpret_cast<int32_t*>(Kinv + kCB * kCB);
  const int di = static_cast<int>(d);
  const unsigned g = static_cast<unsigned>(div_up(d * d, 256) < 4096 ? div_up(d * d, 256) : 4096);
  hipLaunchKernelGGL(k_copy_upper, dim3(g), dim3(256), 0, s, G, ldg, di, W, bad);
  SKLS_CHECK_LAUNCH();
  for (int K = 0; K < di; K += kCB) {
    const int kb = (di - K) < kCB ? (di - K) : kCB;
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, s, W, di, K, Kinv, bad);
    SKLS_CHECK_LAUNCH();
    const int rest = di - K - kb;
    if (rest <= 0) break;
    const int nt = (rest + kCB - 1) / kCB;
    hipLaunchKernelGGL(k_chol_trsm, dim3(nt), dim3(256), 0, s, W, di, K, Kinv);
    SKLS_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_chol_syrk, dim3(nt * (nt + 1) / 2), dim3(256), 0, s, W, di, K);
    SKLS_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_chol_finish, dim3(g), dim3(256), 0, s, W, di, R, bad, status, rtol);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t run_trinv(const double* R, int64_t d, double* Rinv, double* RinvT, hipStream_t s) {
  PhaseTimer pt("trinv", s);
  hipLaunchKernelGGL(k_trinv, dim3(static_cast<unsigned>(d)), dim3(kWave), static_cast<size_t>(d) * sizeof(double), s,
                     R, static_cast<int>(d), Rinv, RinvT);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t run_gemv(const double* M, int64_t d, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_gemv, dim3(static_cast<unsigned>(div_up(d, 4))), dim3(256), 0, s, M, static_cast<int>(d), x,
                     y);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t run_solve_from_gram(const double* Rinv, const double* RinvT, const double* c, int64_t d, double* x,
                            double* tmp, hipStream_t s) {
  SKLS_TRY(run_gemv(RinvT, d, c, tmp, s));
  return run_gemv(Rinv, d, tmp, x, s);
}

int32_t run_rinv_times(const double* Rinv, int64_t d, const double* P, int32_t k, float* T, hipStream_t s) {
  hipLaunchKernelGGL(k_rinv_times, dim3(static_cast<unsigned>(div_up(d * k, 256))), dim3(256), 0, s, Rinv,
                     static_cast<int>(d), P, k, T);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t run_convert_f64_to_f32(const double* in, float* out, int64_t count, hipStream_t s) {
  if (count == 0) return SKLS_OK;
  int64_t g = div_up(count, 256);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_f64_to_f32, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, in, out, count);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

}  // namespace skls
