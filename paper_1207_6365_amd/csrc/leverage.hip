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

// Dense A on the float32 matrix cores (v_mfma_f32_16x16x4f32).  Each
// wavefront takes 16 rows at a time and walks the columns 4 at a time: lane l
// loads A[row0 + l % 16][c + l / 16] straight into the A operand (the 16 rows
// of a 64-column chunk are 4 KiB that stay in the L1 while the chunk is
// consumed), and the next chunk's loads are issued before the current one is
// multiplied.  T (zero-padded to d64 x 16 NB, float32) is in LDS and feeds the
// B operands.  Output element e of lane l is row 4 (l / 16) + e, column
// l % 16 of the 16 x 16 block; the squares of a row's NB blocks are summed
// over the 16 lanes of a DPP row.
typedef float f4_t __attribute__((ext_vector_type(4)));
constexpr int kLevChunk = 64;  // columns per chunk

// Wide-load form for rows whose length is a multiple of 4 and 16-byte aligned:
// each wavefront stages its 16 rows x 32 columns through a private LDS tile
// filled by 16-byte loads (8 lanes cover 128 contiguous bytes of a row), and
// reads the A operand back as 16-byte rows.  The contraction index is taken
// in a permuted order -- step (m, e) pairs lane (row, kk)'s element
// A[row][c0 + 16 m + 4 kk + e] with B row c0 + 16 m + 4 kk + e -- so that
// each lane's operands are one contiguous float4.  The next chunk is loaded
// before the current one is multiplied.  One block of 16 wavefronts per
// compute unit shares T.
constexpr int kWideCols = 32;
constexpr int kWidePitch = kWideCols + 4;  // floats; rows stay 16-byte aligned

template <typename TV>
__device__ __forceinline__ f4_t load4f(const TV* p) {
  if constexpr (std::is_same<TV, float>::value) {
    const nt_f4 x = stream_load<nt_f4>(p);
    return f4_t{x[0], x[1], x[2], x[3]};
  } else if constexpr (std::is_same<TV, double>::value) {
    const nt_d2 a = stream_load<nt_d2>(p);
    const nt_d2 b = stream_load<nt_d2>(p + 2);
    return f4_t{static_cast<float>(a[0]), static_cast<float>(a[1]), static_cast<float>(b[0]), static_cast<float>(b[1])};
  } else {
    const nt_u2 u = stream_load<nt_u2>(p);
    return f4_t{bf16_lo(u[0]), bf16_hi(u[0]), bf16_lo(u[1]), bf16_hi(u[1])};
  }
}

template <typename TV, int NB>
__global__ __launch_bounds__(1024) void k_leverage_wide(int64_t n, int d, int64_t ld, const TV* __restrict__ A,
                                                        const float* __restrict__ T, int k, int dpad,
                                                        float* __restrict__ scores) {
  extern __shared__ __align__(16) float smem[];
  constexpr int KW = 16 * NB;
  float* sT = smem;                                    // [dpad][KW]
  const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  float* tile = smem + static_cast<size_t>(dpad) * KW + static_cast<size_t>(wid) * 16 * kWidePitch;
  for (int e = threadIdx.x; e < dpad * KW; e += blockDim.x) {
    const int r = e / KW, q = e % KW;
    sT[e] = (r < d && q < k) ? T[static_cast<size_t>(r) * k + q] : 0.0f;
  }
  __syncthreads();
  const int li = lane & 15, lk = lane >> 4;
  // loads: lane -> row (lane >> 3) + 8 it, columns 4 (lane & 7) .. + 3
  const int lrow = lane >> 3, lcol = 4 * (lane & 7);
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwave = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  const int nchunk = dpad / kWideCols;
  for (int64_t r0 = wave * 16; r0 < n; r0 += nwave * 16) {
    const TV* rowp[2];
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int64_t r = r0 + lrow + 8 * it;
      rowp[it] = A + static_cast<size_t>(r < n ? r : n - 1) * ld;  // rows past n: computed, not stored
    }
    f4_t nxt[2];
#pragma unroll
    for (int it = 0; it < 2; ++it) nxt[it] = lcol < d ? load4f<TV>(rowp[it] + lcol) : f4_t{0.f, 0.f, 0.f, 0.f};
    f4_t acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = f4_t{0.f, 0.f, 0.f, 0.f};
    for (int ch = 0; ch < nchunk; ++ch) {
      const int c0 = ch * kWideCols;
#pragma unroll
      for (int it = 0; it < 2; ++it)
        *reinterpret_cast<f4_t*>(tile + (lrow + 8 * it) * kWidePitch + lcol) = nxt[it];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (ch + 1 < nchunk) {
        const int c = c0 + kWideCols + lcol;
#pragma unroll
        for (int it = 0; it < 2; ++it) nxt[it] = c < d ? load4f<TV>(rowp[it] + c) : f4_t{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int m = 0; m < kWideCols / 16; ++m) {
        const f4_t a = *reinterpret_cast<const f4_t*>(tile + li * kWidePitch + 16 * m + 4 * lk);
        const float* tb = sT + static_cast<size_t>(c0 + 16 * m + 4 * lk) * KW + li;
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int b = 0; b < NB; ++b)
            acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], tb[e * KW + 16 * b], acc[b], 0, 0, 0);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // row 4 lk + e: sum of squares over the NB blocks and the 16 lanes of the DPP row
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float v = 0.0f;
#pragma unroll
      for (int b = 0; b < NB; ++b) v += acc[b][e] * acc[b][e];
      v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, false));  // row_shr:1
      v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xf, 0xf, false));  // row_shr:2
      v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xf, 0xf, false));  // row_shr:4
      v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xf, 0xf, false));  // row_shr:8
      const int64_t r = r0 + 4 * lk + e;
      if (li == 15 && r < n) scores[r] = v;
    }
  }
}

template <typename TV, int NB>
__global__ __launch_bounds__(512) void k_leverage_mfma(int64_t n, int d, int64_t ld, const TV* __restrict__ A,
                                                       const float* __restrict__ T, int k, int d64,
                                                       float* __restrict__ scores) {
  extern __shared__ __align__(16) float sT[];  // [d64][16 NB]
  constexpr int KW = 16 * NB;
  for (int e = threadIdx.x; e < d64 * KW; e += blockDim.x) {
    const int r = e / KW, q = e % KW;
    sT[e] = (r < d && q < k) ? T[static_cast<size_t>(r) * k + q] : 0.0f;
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int li = lane & 15, lk = lane >> 4;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwave = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  const int nchunk = d64 / kLevChunk;
  for (int64_t r0 = wave * 16; r0 < n; r0 += nwave * 16) {
    const int64_t row = r0 + li < n ? r0 + li : n - 1;  // clamped: rows past n are computed, not stored
    const TV* arow = A + static_cast<size_t>(row) * ld;
    f4_t acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = f4_t{0.f, 0.f, 0.f, 0.f};
    // a[s] = A[row][c0 + 4 s + lk]: columns past d read column 0 (T is zero there)
    float cur[kLevChunk / 4], nxt[kLevChunk / 4];
#pragma unroll
    for (int q = 0; q < kLevChunk / 4; ++q) {
      const int c = 4 * q + lk;
      cur[q] = load_as<float>(arow, static_cast<size_t>(c < d ? c : 0));
    }
    for (int ch = 0; ch < nchunk; ++ch) {
      const int c0 = ch * kLevChunk;
      if (ch + 1 < nchunk) {
#pragma unroll
        for (int q = 0; q < kLevChunk / 4; ++q) {
          const int c = c0 + kLevChunk + 4 * q + lk;
          nxt[q] = load_as<float>(arow, static_cast<size_t>(c < d ? c : 0));
        }
      }
#pragma unroll
      for (int q = 0; q < kLevChunk / 4; ++q) {
        const float* trow = sT + static_cast<size_t>(c0 + 4 * q + lk) * KW + li;
#pragma unroll
        for (int b = 0; b < NB; ++b)
          acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(cur[q], trow[16 * b], acc[b], 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < kLevChunk / 4; ++q) cur[q] = nxt[q];
    }
    // row 4 lk + e: sum of squares over the NB blocks and the 16 lanes of the DPP row
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float v = 0.0f;
#pragma unroll
      for (int b = 0; b < NB; ++b) v += acc[b][e] * acc[b][e];
      v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, false));  // row_shr:1
      v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xf, 0xf, false));  // row_shr:2
      v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xf, 0xf, false));  // row_shr:4
      v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xf, 0xf, false));  // row_shr:8
      const int64_t r = r0 + 4 * lk + e;
      if (li == 15 && r < n) scores[r] = v;
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
        // matrix-core kernel while T fits LDS (d64 x 16 NB floats, two blocks per compute unit)
        constexpr int NB = K <= 16 ? 1 : (K <= 32 ? 2 : 4);
        const int d64 = static_cast<int>(div_up(d, kLevChunk) * kLevChunk);
        const size_t tl = static_cast<size_t>(d64) * 16 * NB * sizeof(float);
        constexpr int VB = sizeof(TV) == 2 ? 8 : 16;  // bytes of a 4-element load
        const bool wide = d % 4 == 0 && (A.ld * static_cast<int64_t>(sizeof(TV))) % VB == 0 &&
                          reinterpret_cast<uintptr_t>(A.val) % VB == 0;
        const int dpad = static_cast<int>(div_up(d, kWideCols) * kWideCols);
        const size_t wl = (static_cast<size_t>(dpad) * 16 * NB + 16 * kWidePitch * 16) * sizeof(float);
        if (wide && wl <= 150 * 1024) {
          SKLS_TRY(allow_lds(k_leverage_wide<TV, NB>, wl));
          int cus = 256;
          int dev = 0;
          if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
          int64_t g = div_up(A.n, 16 * 16);
          if (g > cus) g = cus;
          hipLaunchKernelGGL((k_leverage_wide<TV, NB>), dim3(static_cast<unsigned>(g)), dim3(1024), wl, s, A.n, d,
                             A.ld, static_cast<const TV*>(A.val), T, k, dpad, scores);
          SKLS_CHECK_LAUNCH();
          return SKLS_OK;
        }
        if (tl <= 72 * 1024) {
          SKLS_TRY(allow_lds(k_leverage_mfma<TV, NB>, tl));
          int64_t g = div_up(A.n, 16 * 8);
          if (g > 512) g = 512;
          hipLaunchKernelGGL((k_leverage_mfma<TV, NB>), dim3(static_cast<unsigned>(g)), dim3(512), tl, s, A.n, d, A.ld,
                             static_cast<const TV*>(A.val), T, k, d64, scores);
          SKLS_CHECK_LAUNCH();
          return SKLS_OK;
        }
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
