// Learned sketch values: the random signs of D (Section 2) become trainable
// per-row values w while the bucket map h stays hashed.  Forward Y = S_w A is
// the sketch kernel with w in place of the signs; with E = Y^T Y - A^T A the
// distortion loss is ||E||_F^2, dL/dY = 4 Y E, and the backward pass to the
// values is a gather: dL/dw_i = < (4 Y E)[h(i), :], A[i, :] >, one read of A.
#include "kernels.hpp"
#include "profile.hpp"

namespace skls {
namespace {

__global__ __launch_bounds__(1024) void k_learned_E(const double* __restrict__ P, int64_t ldp,
                                                    const float* __restrict__ C, int d, float* __restrict__ E,
                                                    float* __restrict__ loss) {
  __shared__ double scratch[16];
  double s = 0.0;
  for (int idx = threadIdx.x; idx < d * d; idx += blockDim.x) {
    const int i = idx / d, j = idx % d;
    const double e = P[static_cast<size_t>(i) * ldp + j] - static_cast<double>(C[idx]);
    E[idx] = static_cast<float>(e);
    s += e * e;
  }
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) *loss = static_cast<float>(s);
}

// G = 4 Y E (t x d times d x d).  A block forms a kGR x kGC tile of G; the
// inner index runs in chunks of kGKc staged in LDS (the Y rows and the E
// block), so every thread keeps four independent sums and the loads of a
// chunk are in flight together.  Entries outside t x d are staged as zeros
// from clamped, always valid addresses.
constexpr int kGR = 16, kGC = 64, kGKc = 64;

__global__ __launch_bounds__(256) void k_learned_G(const float* __restrict__ Y, const float* __restrict__ E,
                                                   int64_t t, int d, float* __restrict__ G) {
  __shared__ __align__(16) float Es[kGKc][kGC];
  __shared__ float Ys[kGR][kGKc + 1];
  const int tid = threadIdx.x;
  const int r = tid / 16, c4 = (tid % 16) * 4;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kGR;
  const int cb = blockIdx.y * kGC;
  float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < d; k0 += kGKc) {
    float e[kGKc * kGC / 256], y[kGR * kGKc / 256];
#pragma unroll
    for (int u = 0; u < kGKc * kGC / 256; ++u) {
      const int q = u * 256 + tid, kk = q / kGC, cc = q % kGC;
      const bool in = k0 + kk < d && cb + cc < d;
      const float x = E[in ? static_cast<size_t>(k0 + kk) * d + cb + cc : 0];
      e[u] = in ? x : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kGR * kGKc / 256; ++u) {
      const int q = u * 256 + tid, rr = q / kGKc, kk = q % kGKc;
      const bool in = r0 + rr < t && k0 + kk < d;
      const float x = Y[in ? static_cast<size_t>(r0 + rr) * d + k0 + kk : 0];
      y[u] = in ? x : 0.0f;
    }
    __syncthreads();  // the previous chunk's reads are done
#pragma unroll
    for (int u = 0; u < kGKc * kGC / 256; ++u) {
      const int q = u * 256 + tid;
      Es[q / kGC][q % kGC] = e[u];
    }
#pragma unroll
    for (int u = 0; u < kGR * kGKc / 256; ++u) {
      const int q = u * 256 + tid;
      Ys[q / kGKc][q % kGKc] = y[u];
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < kGKc; ++kk) {
      const float yv = Ys[r][kk];
      const float4 ev = *reinterpret_cast<const float4*>(&Es[kk][c4]);
      acc[0] += yv * ev.x;
      acc[1] += yv * ev.y;
      acc[2] += yv * ev.z;
      acc[3] += yv * ev.w;
    }
  }
  if (r0 + r >= t) return;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (cb + c4 + k < d) G[static_cast<size_t>(r0 + r) * d + cb + c4 + k] = 4.0f * acc[k];
}

// grad[i] = < G[h(i), :], A[i, :] > with 16 lanes per row; VEC (16-byte
// aligned rows, d a multiple of 4): each lane reads four consecutive entries
// of both rows at once.
template <bool VEC>
__global__ __launch_bounds__(256) void k_learned_gather(int64_t n, int d, int64_t ld, const float* __restrict__ A,
                                                        const float* __restrict__ G, uint32_t t, uint64_t seed,
                                                        float scale, int accumulate, float* __restrict__ grad) {
  constexpr int L = 16;
  const int sub = threadIdx.x % L;
  const int64_t grp = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / L;
  const int64_t ngrp = static_cast<int64_t>(gridDim.x) * blockDim.x / L;
  for (int64_t r = grp; r < n; r += ngrp) {
    const uint32_t h = bucket_of(splitmix64(seed, static_cast<uint64_t>(r)), t);
    const float* a = A + static_cast<size_t>(r) * ld;
    const float* g = G + static_cast<size_t>(h) * d;
    float s = 0.0f;
    if (VEC) {
      for (int c = sub * 4; c < d; c += L * 4) {
        const nt_f4 x = stream_load<nt_f4>(a + c);
        const float4 y = *reinterpret_cast<const float4*>(g + c);
        s += x[0] * y.x + x[1] * y.y + x[2] * y.z + x[3] * y.w;
      }
    } else {
      for (int c = sub; c < d; c += L) s += a[c] * g[c];
    }
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
    if (sub == 0) grad[r] = accumulate ? grad[r] + scale * s : scale * s;
  }
}

// grad = (accumulate ? grad : 0) + scale * (slot 0 + ... + slot k-1), the
// slots summed in index order.
__global__ void k_sum_slots(int64_t n, const float* __restrict__ slots, int64_t stride, int k, float scale,
                            int accumulate, float* __restrict__ grad) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    float s = slots[i];
    for (int j = 1; j < k; ++j) s += slots[j * stride + i];
    grad[i] = accumulate ? grad[i] + scale * s : scale * s;
  }
}

__global__ void k_adam(int64_t n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

}  // namespace

int32_t run_learned_E(const double* P, int64_t ldp, const float* C, int64_t d, float* E, float* loss,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_learned_E, dim3(1), dim3(1024), 0, s, P, ldp, C, static_cast<int>(d), E, loss);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t run_learned_G(const float* Y, const float* E, int64_t t, int64_t d, float* G, hipStream_t s) {
  hipLaunchKernelGGL(k_learned_G, dim3(static_cast<unsigned>(div_up(t, kGR)), static_cast<unsigned>(div_up(d, kGC))),
                     dim3(256), 0, s, Y, E, t, static_cast<int>(d), G);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t run_learned_gather(const skls_matrix& A, const float* G, uint32_t t, uint64_t seed, float scale,
                           bool accumulate, float* grad, hipStream_t s) {
  if (A.n == 0) return SKLS_OK;
  PhaseTimer pt("learned_gather", s);
  int64_t blocks = div_up(A.n * 16, 256);
  if (blocks > 8192) blocks = 8192;
  const bool vec = reinterpret_cast<uintptr_t>(A.val) % 16 == 0 && A.ld % 4 == 0 && A.d % 4 == 0 &&
                   reinterpret_cast<uintptr_t>(G) % 16 == 0;
  const auto kern = vec ? k_learned_gather<true> : k_learned_gather<false>;
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, A.n, static_cast<int>(A.d), A.ld,
                     static_cast<const float*>(A.val), G, t, seed, scale, accumulate ? 1 : 0, grad);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t run_sum_slots(int64_t n, const float* slots, int64_t stride, int k, float scale, bool accumulate,
                      float* grad, hipStream_t s) {
  if (n == 0) return SKLS_OK;
  int64_t blocks = div_up(n, 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_sum_slots, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, n, slots, stride, k, scale,
                     accumulate ? 1 : 0, grad);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t run_adam(int64_t n, float* w, const float* g, float* m, float* v, int32_t step, float lr, float b1,
                 float b2, float eps, hipStream_t s) {
  if (n == 0) return SKLS_OK;
  const float c1 = 1.0f - powf(b1, static_cast<float>(step));
  const float c2 = 1.0f - powf(b2, static_cast<float>(step));
  int64_t blocks = div_up(n, 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_adam, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, n, w, g, m, v, lr, b1, b2, eps, c1,
                     c2);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

}  // namespace skls
