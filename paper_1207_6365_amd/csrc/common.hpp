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
// 16- and 8-byte loads of data that is read once (a stream over A): the
// non-temporal hint keeps it from displacing reusable lines in the caches.
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef unsigned nt_u4 __attribute__((ext_vector_type(4)));
typedef unsigned nt_u2 __attribute__((ext_vector_type(2)));
typedef int nt_i4 __attribute__((ext_vector_type(4)));
template <typename V>
__device__ __forceinline__ V stream_load(const void* p) {
  return __builtin_nontemporal_load(static_cast<const V*>(p));
}

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

// Which hash a sketch uses.  Plain sparse embedding (Section 2; v = 0): z =
// output r of the stream `seed`, bucket h(r) = bucket_of(z, t), sign from z.
// Generalized sparse embedding (Section 5), one of its stacked copies:
// bucket = h(r) v + h_j(r) with the outer h(r) = bucket_of(output r of the
// stream `outer`, q) shared by all copies and h_j(r) = bucket_of(z, v), z =
// output r of the copy's stream `seed` (which also gives the sign); t = q v.
// The kernels pass local row indices; `base` is added to them, so a block of
// rows that starts at global row `base` hashes its rows by their global index
// (S A = sum over row blocks g of S A_g, the linearity of Phi D).
struct HashKey {
  uint64_t seed;
  uint64_t outer;
  uint32_t q, v;
  uint64_t base = 0;
};
inline HashKey plain_key(uint64_t s, uint64_t base = 0) {
  HashKey k{s, 0, 0, 0};
  k.base = base;
  return k;
}
__device__ __forceinline__ uint64_t hk_z(const HashKey& k, uint64_t r) { return splitmix64(k.seed, r + k.base); }
__device__ __forceinline__ uint32_t hk_bucket(const HashKey& k, uint64_t z, uint64_t r, uint32_t t) {
  return k.v == 0 ? bucket_of(z, t) : bucket_of(splitmix64(k.outer, r + k.base), k.q) * k.v + bucket_of(z, k.v);
}
__device__ __forceinline__ uint32_t hk_bucket_r(const HashKey& k, uint64_t r, uint32_t t) {
  return hk_bucket(k, hk_z(k, r), r, t);
}

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

// Sum over the 64 lanes with DPP row shifts and row broadcasts (an inclusive
// scan whose last lane holds the total), returned to every lane; no LDS
// round trips.  All 64 lanes must be active.
__device__ __forceinline__ int32_t dpp_shift(int32_t x, int ctrl_sel) {
  switch (ctrl_sel) {
    case 0: return __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
    case 1: return __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
    case 2: return __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
    case 3: return __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
    case 4: return __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
    default: return __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false); // row_bcast:31 into rows 2, 3
  }
}

__device__ __forceinline__ float wave_total(float v) {
#pragma unroll
  for (int c = 0; c < 6; ++c) v += __int_as_float(dpp_shift(__float_as_int(v), c));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), kWave - 1));
}

__device__ __forceinline__ double wave_total(double v) {
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const long long b = __double_as_longlong(v);
    const int32_t lo = dpp_shift(static_cast<int32_t>(b & 0xffffffffll), c);
    const int32_t hi = dpp_shift(static_cast<int32_t>(b >> 32), c);
    v += __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<uint32_t>(lo));
  }
  const long long b = __double_as_longlong(v);
  const int32_t lo = __builtin_amdgcn_readlane(static_cast<int32_t>(b & 0xffffffffll), kWave - 1);
  const int32_t hi = __builtin_amdgcn_readlane(static_cast<int32_t>(b >> 32), kWave - 1);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<uint32_t>(lo));
}

// Floating-point adds into LDS as compare-and-swap loops.  gfx950 executes
// ds_add_f32 / ds_add_f64 at a small fraction of the rate of its integer LDS
// atomics (about 190 cycles per wave64 instruction per compute unit against
// 7 for ds_add_u32, measured), while ds_cmpst runs at integer speed; a lane
// whose swap lost to another lane or wave retries with the value it saw.
template <typename T>
struct FBits;
template <>
struct FBits<float> {
  using U = uint32_t;
  __device__ __forceinline__ static U to(float x) { return __float_as_uint(x); }
  __device__ __forceinline__ static float from(U u) { return __uint_as_float(u); }
};
template <>
struct FBits<double> {
  using U = unsigned long long;
  __device__ __forceinline__ static U to(double x) { return static_cast<U>(__double_as_longlong(x)); }
  __device__ __forceinline__ static double from(U u) { return __longlong_as_double(static_cast<long long>(u)); }
};

// acc[a[k]] += v[k] for the k < N whose bit is set in `mask` (elements of
// one lane may alias: their swaps are ordered and a stale one retries).
template <typename TO, int N>
__device__ __forceinline__ void lds_add(TO* acc, const int32_t (&a)[N], const TO (&v)[N],
                                        uint32_t mask = 0xffffffffu) {
  static_assert(N <= 32, "pending mask is 32 bits");
  using B = FBits<TO>;
  using U = typename B::U;
  U* q = reinterpret_cast<U*>(acc);
  U old[N];
#pragma unroll
  for (int k = 0; k < N; ++k) old[k] = q[a[k]];
  uint32_t pend = mask & (N == 32 ? 0xffffffffu : ((1u << N) - 1u));
  while (pend != 0) {
    U got[N];
#pragma unroll
    for (int k = 0; k < N; ++k)
      got[k] = ((pend >> k) & 1u) ? atomicCAS(q + a[k], old[k], B::to(B::from(old[k]) + v[k])) : old[k];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      if (got[k] == old[k]) pend &= ~(1u << k);
      old[k] = got[k];
    }
  }
}

template <typename TO>
__device__ __forceinline__ void lds_add1(TO* acc, int32_t a, TO v) {
  const int32_t aa[1] = {a};
  const TO vv[1] = {v};
  lds_add<TO, 1>(acc, aa, vv);
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
