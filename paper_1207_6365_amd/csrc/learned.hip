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

// P = the sum of the S row splits of Y^T Y (entries i <= j of split k at
// partial + k * pitch^2 + i * pitch + j), E = P - C in both triangles
// (float32) and loss = ||E||_F^2, in one block of 1024 threads (d <= 64, so
// at most four entries per thread).  Only entries i <= j read the splits,
// along the rows of the partial tile (the lower entries would read it down
// its columns, one cache line per lane); each writes E[i][j] and E[j][i].  A
// thread's entries read their splits together, eight splits at a time.
__device__ __forceinline__ void learned_pe_body(const double* __restrict__ partial, int S, int pitch,
                                                const float* __restrict__ C, int d, float* __restrict__ E,
                                                float* __restrict__ loss) {
  constexpr int kU = 4, kK = 8;
  __shared__ double scratch[16];
  const size_t stride = static_cast<size_t>(pitch) * pitch;
  const int n = d * d;
  const double* src[kU];
  int ii[kU], jj[kU];
  bool act[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int idx = static_cast<int>(threadIdx.x) + u * 1024;
    ii[u] = idx / d;
    jj[u] = idx % d;
    act[u] = idx < n && ii[u] <= jj[u];
    // idle lanes read entry (0, 0), one line for all of them
    src[u] = partial + (act[u] ? static_cast<size_t>(ii[u]) * pitch + jj[u] : 0);
  }
  double a[kU] = {0.0, 0.0, 0.0, 0.0};
  int k = 0;
  for (; k + kK <= S; k += kK) {
    double x[kK][kU];
#pragma unroll
    for (int kk = 0; kk < kK; ++kk)
#pragma unroll
      for (int u = 0; u < kU; ++u) x[kk][u] = src[u][(k + kk) * stride];
#pragma unroll
    for (int kk = 0; kk < kK; ++kk)
#pragma unroll
      for (int u = 0; u < kU; ++u) a[u] += x[kk][u];
  }
  for (; k < S; ++k)
#pragma unroll
    for (int u = 0; u < kU; ++u) a[u] += src[u][k * stride];
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < kU; ++u)
    if (act[u]) {
      const int i = ii[u], j = jj[u];
      const double e = a[u] - static_cast<double>(C[i * d + j]);
      E[i * d + j] = static_cast<float>(e);
      s += e * e;
      if (i != j) {
        const double f = a[u] - static_cast<double>(C[j * d + i]);
        E[j * d + i] = static_cast<float>(f);
        s += f * f;
      }
    }
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) *loss = static_cast<float>(s);
}

__global__ __launch_bounds__(1024) void k_learned_PE(const double* __restrict__ partial, int S, int pitch,
                                                     const float* __restrict__ C, int d, float* __restrict__ E,
                                                     float* __restrict__ loss) {
  learned_pe_body(partial, S, pitch, C, d, E, loss);
}

// Several matrices of one shape in one launch: block j takes matrix j, whose
// splits start at partial + j * pstride, E at E + j d^2 and loss at loss[j].
__global__ __launch_bounds__(1024) void k_learned_PE_many(const double* __restrict__ partial, int64_t pstride, int S,
                                                          int pitch, LearnedMany args, int d, float* __restrict__ E,
                                                          float* __restrict__ loss) {
  const int j = blockIdx.x;
  learned_pe_body(partial + j * pstride, S, pitch, args.C[j], d, E + static_cast<int64_t>(j) * d * d, loss + j);
}

// G = 4 Y E for the kFB buckets b0 .. b0 + kFB - 1 of this block, held in
// LDS, then the gradient of every row of those buckets:
//   grad[r] = scale * < G[h(r)], A[r] >   (d <= 64).
// The rows come from the bucket order of the sketch's plan, where the rows of
// the block's buckets are one contiguous run of perm; groups of 16 lanes take
// every 16th of them, kFU at a time, so their loads are in flight together.
// Loads are unconditional (clamped indices, values masked afterwards).
constexpr int kFB = 4, kFU = 4;

template <bool VEC>
__device__ __forceinline__ void learned_g_gather_body(const float* __restrict__ Y, const float* __restrict__ E,
                                                      int64_t t, int d, const int32_t* __restrict__ off,
                                                      const int32_t* __restrict__ perm, int64_t ld,
                                                      const float* __restrict__ A, float scale, int accumulate,
                                                      float* __restrict__ grad) {
  __shared__ float Es[64][64];
  __shared__ __align__(16) float Gs[kFB][64];
  __shared__ float Ys[kFB][64];
  const int tid = threadIdx.x;
  const int64_t b0 = static_cast<int64_t>(blockIdx.x) * kFB;
  float e[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int q = u * 256 + tid, k = q / 64, c = q % 64;
    const bool in = k < d && c < d;
    const float x = E[in ? k * d + c : 0];
    e[u] = in ? x : 0.0f;
  }
  const int r = tid / 64, c = tid % 64;  // kFB x 64 = 256 threads
  {
    const bool in = b0 + r < t && c < d;
    const float x = Y[in ? static_cast<size_t>(b0 + r) * d + c : 0];
    Ys[r][c] = in ? x : 0.0f;
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int q = u * 256 + tid;
    Es[q / 64][q % 64] = e[u];
  }
  __syncthreads();
  float acc = 0.0f;
#pragma unroll 8
  for (int k = 0; k < 64; ++k) acc += Ys[r][k] * Es[k][c];
  Gs[r][c] = 4.0f * acc;
  __syncthreads();
  if (b0 >= t) return;
  const int64_t bl = (b0 + kFB < t) ? b0 + kFB : t;
  const int32_t P0 = off[b0], P1 = off[bl];
  int32_t ob[kFB - 1];
#pragma unroll
  for (int u = 0; u < kFB - 1; ++u) ob[u] = off[(b0 + 1 + u < bl) ? b0 + 1 + u : bl];
  const int grp = tid / 16, sub = tid % 16;
  for (int32_t p = P0 + grp; p < P1; p += 16 * kFU) {
    int32_t row[kFU], kb[kFU];
    bool ok[kFU];
#pragma unroll
    for (int u = 0; u < kFU; ++u) {
      const int32_t pu = p + 16 * u;
      ok[u] = pu < P1;
      const int32_t pc = ok[u] ? pu : P0;
      row[u] = perm[pc];
      kb[u] = 0;
#pragma unroll
      for (int v = 0; v < kFB - 1; ++v) kb[u] += pc >= ob[v] ? 1 : 0;
    }
    float sum[kFU];
    if (VEC) {
      const bool live = sub * 4 < d;
      const int cc = live ? sub * 4 : 0;
      nt_f4 x[kFU];
#pragma unroll
      for (int u = 0; u < kFU; ++u) x[u] = stream_load<nt_f4>(A + static_cast<size_t>(row[u]) * ld + cc);
#pragma unroll
      for (int u = 0; u < kFU; ++u) {
        const float4 g = *reinterpret_cast<const float4*>(&Gs[kb[u]][cc]);
        const float v = x[u][0] * g.x + x[u][1] * g.y + x[u][2] * g.z + x[u][3] * g.w;
        sum[u] = live ? v : 0.0f;
      }
    } else {
#pragma unroll
      for (int u = 0; u < kFU; ++u) {
        sum[u] = 0.0f;
        for (int cc = sub; cc < d; cc += 16) sum[u] += A[static_cast<size_t>(row[u]) * ld + cc] * Gs[kb[u]][cc];
      }
    }
#pragma unroll
    for (int u = 0; u < kFU; ++u)
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) sum[u] += __shfl_xor(sum[u], o, kWave);
    if (sub == 0)
#pragma unroll
      for (int u = 0; u < kFU; ++u)
        if (ok[u]) grad[row[u]] = accumulate ? grad[row[u]] + scale * sum[u] : scale * sum[u];
  }
}

template <bool VEC>
__global__ __launch_bounds__(256) void k_learned_G_gather(const float* __restrict__ Y, const float* __restrict__ E,
                                                          int64_t t, int d, const int32_t* __restrict__ off,
                                                          const int32_t* __restrict__ perm, int64_t ld,
                                                          const float* __restrict__ A, float scale, int accumulate,
                                                          float* __restrict__ grad) {
  learned_g_gather_body<VEC>(Y, E, t, d, off, perm, ld, A, scale, accumulate, grad);
}

// Several matrices of one shape in one launch: matrix blockIdx.y has its
// sketch at Y + y * ystride, E at E + y d^2, and writes its weighted gradient
// to its own slot, grad + y * gstride.
template <bool VEC>
__global__ __launch_bounds__(256) void k_learned_G_gather_many(const float* __restrict__ Y, int64_t ystride,
                                                               const float* __restrict__ E, int64_t t, int d,
                                                               const int32_t* __restrict__ off,
                                                               const int32_t* __restrict__ perm, LearnedMany args,
                                                               float* __restrict__ grad, int64_t gstride) {
  const int j = blockIdx.y;
  learned_g_gather_body<VEC>(Y + j * ystride, E + static_cast<int64_t>(j) * d * d, t, d, off, perm, args.ld[j],
                             args.A[j], args.scale[j], 0, grad + j * gstride);
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

int32_t run_learned_PE(const double* partial, int S, int pitch, const float* C, int64_t d, float* E, float* loss,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_learned_PE, dim3(1), dim3(1024), 0, s, partial, S, pitch, C, static_cast<int>(d), E, loss);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t run_learned_G_gather(const float* Y, const float* E, int64_t t, const int32_t* off, const int32_t* perm,
                             const skls_matrix& A, float scale, bool accumulate, float* grad, hipStream_t s) {
  if (A.d > 64) {
    set_error("the fused gradient needs d <= 64");
    return SKLS_ERR_SHAPE;
  }
  PhaseTimer pt("learned_gather", s);
  const bool vec = reinterpret_cast<uintptr_t>(A.val) % 16 == 0 && A.ld % 4 == 0 && A.d % 4 == 0;
  const auto kern = vec ? k_learned_G_gather<true> : k_learned_G_gather<false>;
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(div_up(t, kFB))), dim3(256), 0, s, Y, E, t,
                     static_cast<int>(A.d), off, perm, A.ld, static_cast<const float*>(A.val), scale,
                     accumulate ? 1 : 0, grad);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t run_learned_PE_many(const double* partial, int64_t pstride, int S, int pitch, const LearnedMany& args,
                            int count, int64_t d, float* E, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_learned_PE_many, dim3(count), dim3(1024), 0, s, partial, pstride, S, pitch, args,
                     static_cast<int>(d), E, loss);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t run_learned_G_gather_many(const float* Y, int64_t ystride, const float* E, int64_t t, int64_t d,
                                  const int32_t* off, const int32_t* perm, const LearnedMany& args, int count,
                                  bool vec, float* grad, int64_t gstride, hipStream_t s) {
  if (d > 64) {
    set_error("the fused gradient needs d <= 64");
    return SKLS_ERR_SHAPE;
  }
  PhaseTimer pt("learned_gather", s);
  const dim3 grid(static_cast<unsigned>(div_up(t, kFB)), static_cast<unsigned>(count));
  const auto kern = vec ? k_learned_G_gather_many<true> : k_learned_G_gather_many<false>;
  hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, Y, ystride, E, t, static_cast<int>(d), off, perm, args, grad,
                     gstride);
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
