// Approximate leverage scores (Section 6): row norms of A T with
// T = R^{-1} Pi2 (d x k, float32), the squared norm of row i of A R^{-1}
// compressed by the Johnson-Lindenstrauss matrix Pi2.
//
// T sits in LDS.  Dense rows are staged through LDS in 256-row x 16-column
// tiles (coalesced reads of A) and each thread accumulates the k products of
// one row; CSR rows use one thread per row.  Accumulation is float32.
#include <type_traits>

#include "kernels.hpp"
#include "profile.hpp"

namespace skls {
namespace {

constexpr int kLevThreads = 256;
constexpr int kTileCols = 16;
constexpr int kTilePitch = kTileCols + 1;

template <typename TV, int K>
__global__ __launch_bounds__(kLevThreads) void k_leverage_dense(int64_t n, int d, int64_t ld,
                                                                const TV* __restrict__ A, const float* __restrict__ T,
                                                                int k, float* __restrict__ scores) {
  extern __shared__ __align__(16) float sm[];
  float* sT = sm;                                   // [d][K], zero-padded beyond k
  float* tile = sm + static_cast<size_t>(d) * K;    // [256][kTilePitch]
  for (int e = threadIdx.x; e < d * K; e += kLevThreads) {
    const int r = e / K, q = e % K;
    sT[e] = q < k ? T[static_cast<size_t>(r) * k + q] : 0.0f;
  }
  const int tid = threadIdx.x;
  for (int64_t rb = static_cast<int64_t>(blockIdx.x) * kLevThreads; rb < n;
       rb += static_cast<int64_t>(gridDim.x) * kLevThreads) {
    float acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = 0.0f;
    for (int c0 = 0; c0 < d; c0 += kTileCols) {
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kTileCols; ++j) {
        const int e = tid + kLevThreads * j;
        const int row = e / kTileCols, cc = e % kTileCols;
        const int64_t gr = rb + row;
        const int gc = c0 + cc;
        tile[row * kTilePitch + cc] = (gr < n && gc < d) ? load_as<float>(A, static_cast<size_t>(gr) * ld + gc) : 0.0f;
      }
      __syncthreads();
      const int cmax = (d - c0) < kTileCols ? (d - c0) : kTileCols;
      for (int cc = 0; cc < cmax; ++cc) {
        const float a = tile[tid * kTilePitch + cc];
        const float* trow = sT + static_cast<size_t>(c0 + cc) * K;
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] += a * trow[q];
      }
    }
    if (rb + tid < n) {
      float s = 0.0f;
#pragma unroll
      for (int q = 0; q < K; ++q) s += acc[q] * acc[q];
      scores[rb + tid] = s;
    }
  }
}

template <typename TV, typename TR, int K>
__global__ __launch_bounds__(kLevThreads) void k_leverage_csr(int64_t n, int d, const TR* __restrict__ row_ptr,
                                                              const int32_t* __restrict__ col,
                                                              const TV* __restrict__ val, const float* __restrict__ T,
                                                              int k, float* __restrict__ scores) {
  extern __shared__ __align__(16) float sm[];
  for (int e = threadIdx.x; e < d * K; e += kLevThreads) {
    const int r = e / K, q = e % K;
    sm[e] = q < k ? T[static_cast<size_t>(r) * k + q] : 0.0f;
  }
  __syncthreads();
  for (int64_t r = blockIdx.x * static_cast<int64_t>(kLevThreads) + threadIdx.x; r < n;
       r += static_cast<int64_t>(gridDim.x) * kLevThreads) {
    float acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = 0.0f;
    const TR e = row_ptr[r + 1];
    for (TR j = row_ptr[r]; j < e; ++j) {
      const float a = load_as<float>(val, static_cast<size_t>(j));
      const float* trow = sm + static_cast<size_t>(col[j]) * K;
#pragma unroll
      for (int q = 0; q < K; ++q) acc[q] += a * trow[q];
    }
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < K; ++q) s += acc[q] * acc[q];
    scores[r] = s;
  }
}

template <typename F>
int32_t with_k(int k, F&& f) {
  if (k <= 8) return f(std::integral_constant<int, 8>{});
  if (k <= 16) return f(std::integral_constant<int, 16>{});
  if (k <= 32) return f(std::integral_constant<int, 32>{});
  return f(std::integral_constant<int, 64>{});
}

template <typename Kern>
int32_t allow_lds(Kern kern, size_t lds) {
  if (lds > 65536) {
    SKLS_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(lds)));
  }
  return SKLS_OK;
}

}  // namespace

int32_t run_leverage(const skls_matrix& A, const float* T, int32_t k, float* scores, hipStream_t s) {
  if (k < 1 || k > 64) {
    set_error("leverage: k must lie in [1, 64]");
    return SKLS_ERR_ARG;
  }
  if (A.n == 0) return SKLS_OK;
  const int d = static_cast<int>(A.d);
  PhaseTimer pt("leverage", s);
  return with_k(k, [&](auto kc) -> int32_t {
    constexpr int K = decltype(kc)::value;
    auto per_dtype = [&](auto tv) -> int32_t {
      using TV = decltype(tv);
      int64_t blocks = div_up(A.n, kLevThreads);
      if (blocks > 4096) blocks = 4096;
      if (A.layout == SKLS_DENSE) {
        const size_t lds = (static_cast<size_t>(d) * K + kLevThreads * kTilePitch) * sizeof(float);
        if (lds > 160 * 1024) {
          set_error("leverage: d * k too large for LDS");
          return SKLS_ERR_SHAPE;
        }
        SKLS_TRY(allow_lds(k_leverage_dense<TV, K>, lds));
        hipLaunchKernelGGL((k_leverage_dense<TV, K>), dim3(static_cast<unsigned>(blocks)), dim3(kLevThreads), lds, s,
                           A.n, d, A.ld, static_cast<const TV*>(A.val), T, k, scores);
        SKLS_CHECK_LAUNCH();
        return SKLS_OK;
      }
      const size_t lds = static_cast<size_t>(d) * K * sizeof(float);
      if (lds > 160 * 1024) {
        set_error("leverage: d * k too large for LDS");
        return SKLS_ERR_SHAPE;
      }
      if (A.row_ptr_64) {
        SKLS_TRY(allow_lds(k_leverage_csr<TV, int64_t, K>, lds));
        hipLaunchKernelGGL((k_leverage_csr<TV, int64_t, K>), dim3(static_cast<unsigned>(blocks)), dim3(kLevThreads),
                           lds, s, A.n, d, static_cast<const int64_t*>(A.row_ptr), A.col_idx,
                           static_cast<const TV*>(A.val), T, k, scores);
      } else {
        SKLS_TRY(allow_lds(k_leverage_csr<TV, int32_t, K>, lds));
        hipLaunchKernelGGL((k_leverage_csr<TV, int32_t, K>), dim3(static_cast<unsigned>(blocks)), dim3(kLevThreads),
                           lds, s, A.n, d, static_cast<const int32_t*>(A.row_ptr), A.col_idx,
                           static_cast<const TV*>(A.val), T, k, scores);
      }
      SKLS_CHECK_LAUNCH();
      return SKLS_OK;
    };
    switch (A.dtype) {
      case SKLS_F64: return per_dtype(double{});
      case SKLS_F32: return per_dtype(float{});
      case SKLS_BF16: return per_dtype(bf16_t{});
      default: set_error("leverage: bad dtype"); return SKLS_ERR_DTYPE;
    }
  });
}

}  // namespace skls
