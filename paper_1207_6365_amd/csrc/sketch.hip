// Sparse embedding S = Phi D applied to A and b (Section 2 of Clarkson &
// Woodruff; the O(nnz(A)) product behind the main theorem of Section 3 and the
// regression theorem of Section 7).
//
// Two schedules of the same sum SA[h(i), :] += sign(i) * A[i, :]:
//  * ATOMIC: rows are streamed in storage order (fully coalesced reads of A)
//    and every entry is added into SA with a device-wide float atomic.
//  * SORTED: a counting sort groups the rows by bucket (count -> scan ->
//    scatter); then one wavefront owns one bucket, sorts its row ids, reduces
//    its rows in increasing row order (registers for dense rows, a per-wave LDS
//    accumulator for CSR rows) and writes its row of SA exactly once.  No
//    zero-fill of SA, no global atomics on SA, bit-reproducible results.
#include <climits>
#include <type_traits>

#include "kernels.hpp"
#include "profile.hpp"

namespace skls {
namespace {

constexpr int kThreads = 256;
constexpr int kBucketWaves = kThreads / kWave;  // buckets per block in the sorted kernels
constexpr int kSortCap = 256;                    // largest bucket sorted in LDS
constexpr int kAccBudget = 4096;                 // bytes of LDS accumulators per wave (CSR)
constexpr int kAccMax = 12288;                   // largest single accumulator row (CSR)

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename TS>
__device__ __forceinline__ TS row_scale(uint64_t seed, int64_t r, const float* __restrict__ w) {
  if (w) return static_cast<TS>(w[r]);
  return negative_of(splitmix64(seed, static_cast<uint64_t>(r))) ? TS(-1) : TS(1);
}

template <typename TS>
__device__ __forceinline__ TS load_b(const void* __restrict__ b, int b_f64, int64_t r) {
  return b_f64 ? static_cast<TS>(static_cast<const double*>(b)[r]) : static_cast<TS>(static_cast<const float*>(b)[r]);
}

// ---------------------------------------------------------------- a1: hash
__global__ void k_hash(int64_t n, uint32_t t, uint64_t seed, int64_t start, int32_t* __restrict__ bucket,
                       int8_t* __restrict__ sign) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint64_t z = splitmix64(seed, static_cast<uint64_t>(start + i));
    if (bucket) bucket[i] = static_cast<int32_t>(bucket_of(z, t));
    if (sign) sign[i] = negative_of(z) ? int8_t(-1) : int8_t(1);
  }
}

__global__ void k_fill_zero(uint32_t* __restrict__ p, size_t words) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  const size_t vec = words / 4;
  uint4* p4 = reinterpret_cast<uint4*>(p);
  for (size_t k = i; k < vec; k += stride) p4[k] = make_uint4(0, 0, 0, 0);
  for (size_t k = vec * 4 + i; k < words; k += stride) p[k] = 0;
}

// ---------------------------------------------------------------- counting sort
__global__ void k_count(int64_t n, uint32_t t, uint64_t seed, int32_t* __restrict__ count, int32_t* __restrict__ rank) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint32_t h = bucket_of(splitmix64(seed, static_cast<uint64_t>(i)), t);
    rank[i] = atomicAdd(&count[h], 1);
  }
}

__global__ void k_scatter(int64_t n, uint32_t t, uint64_t seed, const int32_t* __restrict__ off,
                          const int32_t* __restrict__ rank, int32_t* __restrict__ perm) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint32_t h = bucket_of(splitmix64(seed, static_cast<uint64_t>(i)), t);
    perm[off[h] + rank[i]] = static_cast<int32_t>(i);
  }
}

// Exclusive scan of int32 counts: tiles of kScanTile items per block.
constexpr int kScanItems = 16;
constexpr int kScanTile = kThreads * kScanItems;

__device__ int32_t block_exclusive_scan(int32_t v, int32_t* wsum, int32_t* total) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  int32_t x = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int32_t y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  if (lane == kWave - 1) wsum[wid] = x;
  __syncthreads();
  int32_t base = 0, tot = 0;
  for (int k = 0; k < static_cast<int>(blockDim.x / kWave); ++k) {
    if (k < wid) base += wsum[k];
    tot += wsum[k];
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

__global__ __launch_bounds__(kThreads) void k_scan_reduce(const int32_t* __restrict__ in, int64_t count,
                                                          int32_t* __restrict__ bsum) {
  __shared__ int32_t scratch[kThreads / kWave];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + static_cast<int64_t>(threadIdx.x) * kScanItems;
  int32_t s = 0;
  for (int j = 0; j < kScanItems; ++j)
    if (base + j < count) s += in[base + j];
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) bsum[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_scan_top(int32_t* __restrict__ bsum, int64_t nb,
                                                       int32_t* __restrict__ total_out) {
  __shared__ int32_t wsum[kThreads / kWave];
  int32_t carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += kThreads) {
    const int64_t idx = c0 + threadIdx.x;
    const int32_t v = idx < nb ? bsum[idx] : 0;
    int32_t tot;
    const int32_t ex = block_exclusive_scan(v, wsum, &tot);
    if (idx < nb) bsum[idx] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *total_out = carry;
}

__global__ __launch_bounds__(kThreads) void k_scan_down(const int32_t* __restrict__ in, int64_t count,
                                                        const int32_t* __restrict__ bsum, int32_t* __restrict__ out) {
  __shared__ int32_t wsum[kThreads / kWave];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + static_cast<int64_t>(threadIdx.x) * kScanItems;
  int32_t v[kScanItems];
  int32_t s = 0;
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = base + j < count ? in[base + j] : 0;
    s += v[j];
  }
  int32_t tot;
  int32_t run = bsum[blockIdx.x] + block_exclusive_scan(s, wsum, &tot);
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < count) out[base + j] = run;
    run += v[j];
  }
}

// ---------------------------------------------------------------- bucket rows
// Loads the row ids of one bucket, sorted ascending, with their scales, into
// per-wave LDS.  Buckets larger than kSortCap are left unsorted (false).
template <typename TS>
__device__ __forceinline__ bool load_bucket(const int32_t* __restrict__ perm, int beg, int m, uint64_t seed,
                                            const float* __restrict__ w, int32_t* src, int32_t* dst, TS* scale,
                                            int lane) {
  if (m <= kWave) {
    const int32_t r = lane < m ? perm[beg + lane] : INT_MAX;
    int rank = 0;
    for (int k = 0; k < m; ++k) rank += (__builtin_amdgcn_readlane(r, k) < r) ? 1 : 0;
    if (lane < m) {
      dst[rank] = r;
      scale[rank] = row_scale<TS>(seed, r, w);
    }
    wave_sync();
    return true;
  }
  if (m <= kSortCap) {
    for (int j = lane; j < m; j += kWave) src[j] = perm[beg + j];
    wave_sync();
    for (int j = lane; j < m; j += kWave) {
      const int32_t r = src[j];
      int rank = 0;
      for (int k = 0; k < m; ++k) rank += (src[k] < r) ? 1 : 0;
      dst[rank] = r;
      scale[rank] = row_scale<TS>(seed, r, w);
    }
    wave_sync();
    return true;
  }
  return false;
}

template <typename TO>
constexpr size_t bucket_rows_bytes() {
  return kSortCap * (sizeof(TO) + 2 * sizeof(int32_t));
}

// ---------------------------------------------------------------- a2: CSR, sorted
template <typename TV, typename TR, typename TO, int L>
__global__ __launch_bounds__(kThreads) void k_sketch_csr_sorted(
    int d, uint32_t t, uint64_t seed, const TR* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const TV* __restrict__ val, const void* __restrict__ b, int b_f64, const float* __restrict__ w,
    const int32_t* __restrict__ off, const int32_t* __restrict__ perm, TO* __restrict__ SA, TO* __restrict__ Sb,
    int ncopy, int per_wave) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const uint32_t bkt = blockIdx.x * kBucketWaves + wid;
  if (bkt >= t) return;
  unsigned char* base = smem + static_cast<size_t>(wid) * per_wave;
  TO* scale = reinterpret_cast<TO*>(base);
  int32_t* src = reinterpret_cast<int32_t*>(base + kSortCap * sizeof(TO));
  int32_t* dst = src + kSortCap;
  TO* acc = reinterpret_cast<TO*>(base + bucket_rows_bytes<TO>());
  for (int k = lane; k < ncopy * d; k += kWave) acc[k] = TO(0);
  const int beg = off[bkt], m = off[bkt + 1] - beg;
  const bool sorted = load_bucket<TO>(perm, beg, m, seed, w, src, dst, scale, lane);
  constexpr int G = kWave / L;
  const int g = lane / L, sub = lane % L;
  TO* myacc = acc + (g % ncopy) * d;
  TO sb = TO(0);
  for (int j0 = 0; j0 < m; j0 += G) {
    const int j = j0 + g;
    if (j < m) {
      int32_t r;
      TO s;
      if (sorted) {
        r = dst[j];
        s = scale[j];
      } else {
        r = perm[beg + j];
        s = row_scale<TO>(seed, r, w);
      }
      const TR a = row_ptr[r], e = row_ptr[r + 1];
      for (TR k = a + sub; k < e; k += L) atomicAdd(&myacc[col[k]], s * load_as<TO>(val, static_cast<size_t>(k)));
      if (b != nullptr && sub == 0) sb += s * load_b<TO>(b, b_f64, r);
    }
  }
  wave_sync();
  sb = wave_sum(sb);
  TO* out = SA + static_cast<size_t>(bkt) * d;
  for (int c = lane; c < d; c += kWave) {
    TO v = acc[c];
    for (int q = 1; q < ncopy; ++q) v += acc[q * d + c];
    out[c] = v;
  }
  if (Sb != nullptr && lane == 0) Sb[bkt] = sb;
}

// ---------------------------------------------------------------- a2: dense, sorted
template <typename TV, typename TO, int V>
struct RowLoad {
  __device__ __forceinline__ static void load(const TV* __restrict__ p, TO (&out)[V]) {
#pragma unroll
    for (int k = 0; k < V; ++k) out[k] = load_as<TO>(p, k);
  }
};
template <typename TO>
struct RowLoad<float, TO, 4> {
  __device__ __forceinline__ static void load(const float* __restrict__ p, TO (&out)[4]) {
    const float4 x = *reinterpret_cast<const float4*>(p);
    out[0] = x.x;
    out[1] = x.y;
    out[2] = x.z;
    out[3] = x.w;
  }
};
template <typename TO>
struct RowLoad<double, TO, 2> {
  __device__ __forceinline__ static void load(const double* __restrict__ p, TO (&out)[2]) {
    const double2 x = *reinterpret_cast<const double2*>(p);
    out[0] = static_cast<TO>(x.x);
    out[1] = static_cast<TO>(x.y);
  }
};
template <typename TO>
struct RowLoad<bf16_t, TO, 8> {
  __device__ __forceinline__ static void load(const bf16_t* __restrict__ p, TO (&out)[8]) {
    const uint4 x = *reinterpret_cast<const uint4*>(p);
    out[0] = bf16_lo(x.x);
    out[1] = bf16_hi(x.x);
    out[2] = bf16_lo(x.y);
    out[3] = bf16_hi(x.y);
    out[4] = bf16_lo(x.z);
    out[5] = bf16_hi(x.z);
    out[6] = bf16_lo(x.w);
    out[7] = bf16_hi(x.w);
  }
};

template <typename TV, typename TO, int V>
__global__ __launch_bounds__(kThreads) void k_sketch_dense_sorted(
    int d, int64_t ld, uint32_t t, uint64_t seed, const TV* __restrict__ A, const void* __restrict__ b, int b_f64,
    const float* __restrict__ w, const int32_t* __restrict__ off, const int32_t* __restrict__ perm,
    TO* __restrict__ SA, TO* __restrict__ Sb) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const uint32_t bkt = blockIdx.x * kBucketWaves + wid;
  if (bkt >= t) return;
  unsigned char* base = smem + static_cast<size_t>(wid) * bucket_rows_bytes<TO>();
  TO* scale = reinterpret_cast<TO*>(base);
  int32_t* src = reinterpret_cast<int32_t*>(base + kSortCap * sizeof(TO));
  int32_t* dst = src + kSortCap;
  const int beg = off[bkt], m = off[bkt + 1] - beg;
  const bool sorted = load_bucket<TO>(perm, beg, m, seed, w, src, dst, scale, lane);
  auto row_at = [&](int j) -> int32_t { return sorted ? dst[j] : perm[beg + j]; };
  auto scale_at = [&](int j, int32_t r) -> TO { return sorted ? scale[j] : row_scale<TO>(seed, r, w); };
  if (Sb != nullptr) {
    TO sb = TO(0);
    for (int j = lane; j < m; j += kWave) {
      const int32_t r = row_at(j);
      sb += scale_at(j, r) * load_b<TO>(b, b_f64, r);
    }
    sb = wave_sum(sb);
    if (lane == 0) Sb[bkt] = sb;
  }
  TO* out = SA + static_cast<size_t>(bkt) * d;
  for (int c0 = lane * V; c0 < d; c0 += kWave * V) {
    TO acc[V];
#pragma unroll
    for (int k = 0; k < V; ++k) acc[k] = TO(0);
    int j = 0;
    for (; j + 4 <= m; j += 4) {
      int32_t r[4];
      TO s[4], x[4][V];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        r[q] = row_at(j + q);
        s[q] = scale_at(j + q, r[q]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) RowLoad<TV, TO, V>::load(A + static_cast<size_t>(r[q]) * ld + c0, x[q]);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < V; ++k) acc[k] += s[q] * x[q][k];
    }
    for (; j < m; ++j) {
      const int32_t r = row_at(j);
      const TO s = scale_at(j, r);
      TO x[V];
      RowLoad<TV, TO, V>::load(A + static_cast<size_t>(r) * ld + c0, x);
#pragma unroll
      for (int k = 0; k < V; ++k) acc[k] += s * x[k];
    }
#pragma unroll
    for (int k = 0; k < V; ++k) out[c0 + k] = acc[k];
  }
}

// ---------------------------------------------------------------- a2: atomic
template <typename TV, typename TR, typename TO, int L>
__global__ __launch_bounds__(kThreads) void k_sketch_csr_atomic(
    int64_t n, int d, uint32_t t, uint64_t seed, const TR* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const TV* __restrict__ val, const void* __restrict__ b, int b_f64, const float* __restrict__ w,
    TO* __restrict__ SA, TO* __restrict__ Sb) {
  const int64_t gid = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / L;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x / L;
  const int sub = threadIdx.x % L;
  for (int64_t r = gid; r < n; r += stride) {
    const uint64_t z = splitmix64(seed, static_cast<uint64_t>(r));
    const uint32_t h = bucket_of(z, t);
    const TO s = w ? static_cast<TO>(w[r]) : (negative_of(z) ? TO(-1) : TO(1));
    TO* dstrow = SA + static_cast<size_t>(h) * d;
    const TR e = row_ptr[r + 1];
    for (TR k = row_ptr[r] + sub; k < e; k += L)
      unsafeAtomicAdd(dstrow + col[k], s * load_as<TO>(val, static_cast<size_t>(k)));
    if (Sb != nullptr && sub == 0) unsafeAtomicAdd(Sb + h, s * load_b<TO>(b, b_f64, r));
  }
}

template <typename TV, typename TO>
__global__ __launch_bounds__(kThreads) void k_sketch_dense_atomic(
    int64_t n, int d, int64_t ld, uint32_t t, uint64_t seed, const TV* __restrict__ A, const void* __restrict__ b,
    int b_f64, const float* __restrict__ w, TO* __restrict__ SA, TO* __restrict__ Sb) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  for (int64_t r = wave; r < n; r += nwaves) {
    const uint64_t z = splitmix64(seed, static_cast<uint64_t>(r));
    const uint32_t h = bucket_of(z, t);
    const TO s = w ? static_cast<TO>(w[r]) : (negative_of(z) ? TO(-1) : TO(1));
    TO* dstrow = SA + static_cast<size_t>(h) * d;
    const TV* row = A + static_cast<size_t>(r) * ld;
    for (int c = lane; c < d; c += kWave) unsafeAtomicAdd(dstrow + c, s * load_as<TO>(row, c));
    if (Sb != nullptr && lane == 0) unsafeAtomicAdd(Sb + h, s * load_b<TO>(b, b_f64, r));
  }
}

// ---------------------------------------------------------------- dispatch
template <typename F>
int32_t with_value(int32_t dt, F&& f) {
  switch (dt) {
    case SKLS_F64: return f(double{});
    case SKLS_F32: return f(float{});
    case SKLS_BF16: return f(bf16_t{});
    default: set_error("unsupported value dtype %d", dt); return SKLS_ERR_DTYPE;
  }
}
template <typename F>
int32_t with_out(int32_t dt, F&& f) {
  switch (dt) {
    case SKLS_F64: return f(double{});
    case SKLS_F32: return f(float{});
    default: set_error("output dtype must be F64 or F32 (got %d)", dt); return SKLS_ERR_DTYPE;
  }
}
template <typename F>
int32_t with_rowptr(const skls_matrix& A, F&& f) {
  if (A.row_ptr_64) return f(int64_t{});
  return f(int32_t{});
}
template <typename F>
int32_t with_lanes(int L, F&& f) {
  if (L <= 4) return f(std::integral_constant<int, 4>{});
  if (L <= 16) return f(std::integral_constant<int, 16>{});
  return f(std::integral_constant<int, 64>{});
}

int lanes_per_row(const skls_matrix& A) {
  const double avg = A.n > 0 ? static_cast<double>(A.nnz) / static_cast<double>(A.n) : 1.0;
  if (avg <= 6.0) return 4;
  if (avg <= 24.0) return 16;
  return 64;
}

unsigned grid_for(int64_t work, int per_block, unsigned cap) {
  int64_t g = div_up(work, per_block);
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return static_cast<unsigned>(g);
}

template <typename TV>
bool vec_ok(const void* p, int64_t ld, int64_t d, int V) {
  const size_t es = sizeof(TV);
  return V > 1 && (reinterpret_cast<uintptr_t>(p) % 16 == 0) && ((static_cast<size_t>(ld) * es) % 16 == 0) &&
         (d % V == 0);
}

}  // namespace

// ================================================================ host
int32_t launch_hash(int64_t n, uint32_t t, uint64_t seed, int64_t start, int32_t* bucket, int8_t* sign,
                    hipStream_t s) {
  if (n == 0) return SKLS_OK;
  hipLaunchKernelGGL(k_hash, dim3(grid_for(n, kThreads, 16384)), dim3(kThreads), 0, s, n, t, seed, start, bucket,
                     sign);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return SKLS_OK;
  if (bytes % 4 != 0 || reinterpret_cast<uintptr_t>(p) % 16 != 0) {
    set_error("internal: zero fill needs 16-byte aligned, 4-byte multiple buffers");
    return SKLS_ERR_ARG;
  }
  const size_t words = bytes / 4;
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(static_cast<int64_t>(words / 4 + 1), kThreads, 8192)),
                     dim3(kThreads), 0, s, static_cast<uint32_t*>(p), words);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

size_t plan_bytes(int64_t n, int64_t t) {
  Arena ar(nullptr, 0);
  carve_plan(ar, n, t);
  return ar.used;
}

BucketPlan carve_plan(Arena& ar, int64_t n, int64_t t) {
  BucketPlan P;
  P.count = ar.take<int32_t>(static_cast<size_t>(t));
  P.off = ar.take<int32_t>(static_cast<size_t>(t) + 1);
  P.rank = ar.take<int32_t>(static_cast<size_t>(n));
  P.perm = ar.take<int32_t>(static_cast<size_t>(n));
  P.bsum = ar.take<int32_t>(static_cast<size_t>(div_up(t, kScanTile)) + 1);
  return P;
}

int32_t build_plan(int64_t n, uint32_t t, uint64_t seed, const BucketPlan& P, hipStream_t s) {
  SKLS_TRY(launch_fill_zero(P.count, static_cast<size_t>(t) * sizeof(int32_t), s));
  const unsigned g = grid_for(n, kThreads, 16384);
  if (n > 0) {
    hipLaunchKernelGGL(k_count, dim3(g), dim3(kThreads), 0, s, n, t, seed, P.count, P.rank);
    SKLS_CHECK_LAUNCH();
  }
  const int64_t nb = div_up(t, kScanTile);
  hipLaunchKernelGGL(k_scan_reduce, dim3(static_cast<unsigned>(nb)), dim3(kThreads), 0, s, P.count,
                     static_cast<int64_t>(t), P.bsum);
  SKLS_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kThreads), 0, s, P.bsum, nb, P.off + t);
  SKLS_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_scan_down, dim3(static_cast<unsigned>(nb)), dim3(kThreads), 0, s, P.count,
                     static_cast<int64_t>(t), P.bsum, P.off);
  SKLS_CHECK_LAUNCH();
  if (n > 0) {
    hipLaunchKernelGGL(k_scatter, dim3(g), dim3(kThreads), 0, s, n, t, seed, P.off, P.rank, P.perm);
    SKLS_CHECK_LAUNCH();
  }
  return SKLS_OK;
}

int32_t choose_sketch_variant(const skls_matrix& A, int64_t t, int32_t variant) {
  if (variant != SKLS_SKETCH_AUTO) return variant;
  // One wavefront per bucket needs many buckets with modest loads.
  if (A.n > 256 * t) return SKLS_SKETCH_ATOMIC;
  if (A.layout == SKLS_CSR && A.d * 8 > kAccMax) return SKLS_SKETCH_ATOMIC;
  return SKLS_SKETCH_SORTED;
}

size_t sketch_ws_bytes(const skls_matrix& A, int64_t t, int32_t variant) {
  const int32_t v = choose_sketch_variant(A, t, variant);
  if (v == SKLS_SKETCH_SORTED) return plan_bytes(A.n, t);
  return 0;
}

int32_t run_sketch(const skls_matrix& A, const void* b, int32_t b_dtype, int64_t t, uint64_t seed,
                   const float* w, int32_t variant, void* SA, void* Sb, int32_t out_dtype, void* ws,
                   size_t ws_bytes, hipStream_t s) {
  const int32_t v = choose_sketch_variant(A, t, variant);
  if (v != SKLS_SKETCH_ATOMIC && v != SKLS_SKETCH_SORTED) {
    set_error("unknown sketch variant %d", variant);
    return SKLS_ERR_ARG;
  }
  const int b_f64 = (b_dtype == SKLS_F64) ? 1 : 0;
  const uint32_t tt = static_cast<uint32_t>(t);
  const int d = static_cast<int>(A.d);
  const int64_t n = A.n;
  if (v == SKLS_SKETCH_ATOMIC) {
    return with_out(out_dtype, [&](auto to) -> int32_t {
      using TO = decltype(to);
      {
        PhaseTimer pt("sketch_zero", s);
        SKLS_TRY(launch_fill_zero(SA, static_cast<size_t>(t) * A.d * sizeof(TO), s));
        if (Sb) SKLS_TRY(launch_fill_zero(Sb, static_cast<size_t>(t) * sizeof(TO), s));
      }
      if (n == 0) return SKLS_OK;
      PhaseTimer pt("sketch_apply", s);
      return with_value(A.dtype, [&](auto tv) -> int32_t {
        using TV = decltype(tv);
        if (A.layout == SKLS_DENSE) {
          hipLaunchKernelGGL((k_sketch_dense_atomic<TV, TO>), dim3(grid_for(n * kWave, kThreads, 32768)),
                             dim3(kThreads), 0, s, n, d, A.ld, tt, seed, static_cast<const TV*>(A.val), b, b_f64, w,
                             static_cast<TO*>(SA), static_cast<TO*>(Sb));
          SKLS_CHECK_LAUNCH();
          return SKLS_OK;
        }
        return with_rowptr(A, [&](auto tr) -> int32_t {
          using TR = decltype(tr);
          return with_lanes(lanes_per_row(A), [&](auto lc) -> int32_t {
            constexpr int L = decltype(lc)::value;
            hipLaunchKernelGGL((k_sketch_csr_atomic<TV, TR, TO, L>), dim3(grid_for(n * L, kThreads, 32768)),
                               dim3(kThreads), 0, s, n, d, tt, seed, static_cast<const TR*>(A.row_ptr), A.col_idx,
                               static_cast<const TV*>(A.val), b, b_f64, w, static_cast<TO*>(SA),
                               static_cast<TO*>(Sb));
            SKLS_CHECK_LAUNCH();
            return SKLS_OK;
          });
        });
      });
    });
  }
  // SORTED
  Arena ar(ws, ws_bytes);
  BucketPlan P = carve_plan(ar, n, t);
  if (!ws || !ar.fits()) {
    set_error("sketch workspace too small: need %zu bytes, have %zu", ar.used, ws_bytes);
    return SKLS_ERR_WORKSPACE;
  }
  {
    PhaseTimer pt("sketch_plan", s);
    SKLS_TRY(build_plan(n, tt, seed, P, s));
  }
  const unsigned grid = static_cast<unsigned>(div_up(t, kBucketWaves));
  PhaseTimer pt("sketch_apply", s);
  return with_out(out_dtype, [&](auto to) -> int32_t {
    using TO = decltype(to);
    return with_value(A.dtype, [&](auto tv) -> int32_t {
      using TV = decltype(tv);
      if (A.layout == SKLS_DENSE) {
        const size_t lds = kBucketWaves * bucket_rows_bytes<TO>();
        constexpr int VV = sizeof(TV) == 8 ? 2 : (sizeof(TV) == 4 ? 4 : 8);
        if (vec_ok<TV>(A.val, A.ld, A.d, VV)) {
          hipLaunchKernelGGL((k_sketch_dense_sorted<TV, TO, VV>), dim3(grid), dim3(kThreads), lds, s, d, A.ld, tt,
                             seed, static_cast<const TV*>(A.val), b, b_f64, w, P.off, P.perm, static_cast<TO*>(SA),
                             static_cast<TO*>(Sb));
        } else {
          hipLaunchKernelGGL((k_sketch_dense_sorted<TV, TO, 1>), dim3(grid), dim3(kThreads), lds, s, d, A.ld, tt,
                             seed, static_cast<const TV*>(A.val), b, b_f64, w, P.off, P.perm, static_cast<TO*>(SA),
                             static_cast<TO*>(Sb));
        }
        SKLS_CHECK_LAUNCH();
        return SKLS_OK;
      }
      const size_t row_bytes = static_cast<size_t>(d) * sizeof(TO);
      if (row_bytes > static_cast<size_t>(kAccMax)) {
        set_error("sorted CSR sketch supports d * sizeof(out) <= %d bytes; use the atomic variant", kAccMax);
        return SKLS_ERR_SHAPE;
      }
      return with_rowptr(A, [&](auto tr) -> int32_t {
        using TR = decltype(tr);
        return with_lanes(lanes_per_row(A), [&](auto lc) -> int32_t {
          constexpr int L = decltype(lc)::value;
          constexpr int G = kWave / L;
          int ncopy = row_bytes > 0 ? static_cast<int>(kAccBudget / row_bytes) : G;
          if (ncopy < 1) ncopy = 1;
          if (ncopy > G) ncopy = G;
          const int per_wave = static_cast<int>((bucket_rows_bytes<TO>() + ncopy * row_bytes + 15) / 16 * 16);
          hipLaunchKernelGGL((k_sketch_csr_sorted<TV, TR, TO, L>), dim3(grid), dim3(kThreads),
                             static_cast<size_t>(per_wave) * kBucketWaves, s, d, tt, seed,
                             static_cast<const TR*>(A.row_ptr), A.col_idx, static_cast<const TV*>(A.val), b, b_f64,
                             w, P.off, P.perm, static_cast<TO*>(SA), static_cast<TO*>(Sb), ncopy, per_wave);
          SKLS_CHECK_LAUNCH();
          return SKLS_OK;
        });
      });
    });
  });
}

}  // namespace skls
