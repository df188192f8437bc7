// Shared device helpers and host error plumbing for libskls (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "skls.h"

namespace skls {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);
void clear_error();

#define SKLS_TRY_HIP(call)                                                                 \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) {                                                                \
      ::skls::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                         \
      return SKLS_ERR_DEVICE;                                                              \
    }                                                                                      \
  } while (0)

#define SKLS_TRY(expr)            \
  do {                            \
    int32_t s_ = (expr);          \
    if (s_ != SKLS_OK) return s_; \
  } while (0)

#define SKLS_CHECK_LAUNCH() SKLS_TRY_HIP(hipGetLastError())

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// ------------------------------------------------------------------ workspace
// Carves aligned sub-buffers out of one caller-provided workspace.  With a
// null base it only measures.
struct Arena {
  char* base;
  size_t cap;
  size_t used = 0;
  Arena(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
  template <typename T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + count * sizeof(T);
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
  bool fits() const { return used <= cap; }
};

// ------------------------------------------------------------------ hashing
// SplitMix64 output `i` of the stream with state `seed` (Steele, Lea & Flood,
// OOPSLA 2014): finaliser applied to seed + (i + 1) * golden gamma.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Bucket h(i) in [0, t) by multiply-high reduction of the upper 32 bits, and
// the sign of D from bit 0.
__device__ __forceinline__ uint32_t bucket_of(uint64_t z, uint32_t t) {
  return static_cast<uint32_t>(((z >> 32) * static_cast<uint64_t>(t)) >> 32);
}
__device__ __forceinline__ bool negative_of(uint64_t z) { return (z & 1ull) != 0; }

// ------------------------------------------------------------------ values
// bfloat16 storage: the upper 16 bits of a binary32.
struct bf16_t {
  uint16_t bits;
};

template <typename TA, typename TV>
__device__ __forceinline__ TA load_as(const TV* p, size_t i) {
  return static_cast<TA>(p[i]);
}
template <>
__device__ __forceinline__ float load_as<float, bf16_t>(const bf16_t* p, size_t i) {
  return __uint_as_float(static_cast<uint32_t>(p[i].bits) << 16);
}
template <>
__device__ __forceinline__ double load_as<double, bf16_t>(const bf16_t* p, size_t i) {
  return static_cast<double>(__uint_as_float(static_cast<uint32_t>(p[i].bits) << 16));
}

__device__ __forceinline__ float bf16_lo(uint32_t pair) { return __uint_as_float(pair << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t pair) { return __uint_as_float(pair & 0xFFFF0000u); }

// ------------------------------------------------------------------ wave ops
constexpr int kWave = 64;

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Block-wide sum for blockDim.x a multiple of 64 (<= 1024); `scratch` holds
// at least blockDim.x / 64 values.  Every thread receives the total.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* scratch) {
  v = wave_sum(v);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  T s = 0;
  const int nw = blockDim.x / kWave;
  for (int k = 0; k < nw; ++k) s += scratch[k];
  return s;
}

// ------------------------------------------------------------------ host helpers
int64_t div_up(int64_t a, int64_t b);
size_t dtype_size(int32_t dt);
// Validates a matrix descriptor; returns SKLS_OK or an error (with message).
int32_t validate_matrix(const skls_matrix* A, bool allow_bf16);

}  // namespace skls
