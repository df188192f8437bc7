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
constexpr int kAccMax = 12288;                   // largest accumulator row of S A in LDS (CSR)

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

__global__ __launch_bounds__(kThreads) void k_scan_down(const int32_t* in, int64_t count,
                                                        const int32_t* __restrict__ bsum, int32_t* out) {
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

// ---------------------------------------------------------------- two-level plan
// Counting sort of the rows by bucket without global atomics.  Buckets are
// grouped into coarse bins of `fine` consecutive buckets (a power of two).
//  1. coarse count: each block counts its chunk of rows per coarse bin in LDS
//     and writes the counts bin-major, so an exclusive scan of the whole array
//     gives every (bin, block) its output offset;
//  2. coarse scatter: each block writes its row ids to those offsets (LDS
//     atomics hand out the slots);
//  3. fine pass: one block per coarse bin counts, scans and scatters the bin's
//     rows by bucket with LDS counters, and writes the bucket offsets.
constexpr int kPlanItems = 16;
constexpr int kPlanChunk = kThreads * kPlanItems;  // rows per block in passes 1-2

__global__ __launch_bounds__(kThreads) void k_plan_coarse_count(int64_t n, uint32_t t, uint64_t seed, int sh, int C,
                                                                int nblk, int32_t* __restrict__ cnt) {
  extern __shared__ int32_t hist[];  // [C]
  for (int c = threadIdx.x; c < C; c += kThreads) hist[c] = 0;
  __syncthreads();
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kPlanChunk;
  for (int k = 0; k < kPlanItems; ++k) {
    const int64_t i = r0 + static_cast<int64_t>(k) * kThreads + threadIdx.x;
    if (i < n) atomicAdd(&hist[bucket_of(splitmix64(seed, static_cast<uint64_t>(i)), t) >> sh], 1);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += kThreads) cnt[static_cast<size_t>(c) * nblk + blockIdx.x] = hist[c];
}

__global__ __launch_bounds__(kThreads) void k_plan_coarse_scatter(int64_t n, uint32_t t, uint64_t seed, int sh, int C,
                                                                  int nblk, const int32_t* __restrict__ coff,
                                                                  int32_t* __restrict__ coarse) {
  extern __shared__ int32_t pos[];  // [C]
  for (int c = threadIdx.x; c < C; c += kThreads) pos[c] = coff[static_cast<size_t>(c) * nblk + blockIdx.x];
  __syncthreads();
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kPlanChunk;
  for (int k = 0; k < kPlanItems; ++k) {
    const int64_t i = r0 + static_cast<int64_t>(k) * kThreads + threadIdx.x;
    if (i < n) {
      const int c = static_cast<int>(bucket_of(splitmix64(seed, static_cast<uint64_t>(i)), t) >> sh);
      coarse[atomicAdd(&pos[c], 1)] = static_cast<int32_t>(i);
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_plan_fine(int64_t n, uint32_t t, uint64_t seed, int sh, int C, int nblk,
                                                        const int32_t* __restrict__ coff,
                                                        const int32_t* __restrict__ coarse,
                                                        int32_t* __restrict__ perm, int32_t* __restrict__ off) {
  extern __shared__ int32_t fcnt[];  // [fine]
  __shared__ int32_t wsum[kThreads / kWave];
  const int fine = 1 << sh;
  const int c = blockIdx.x;
  const int64_t beg = coff[static_cast<size_t>(c) * nblk];
  const int64_t end = (c + 1 < C) ? coff[static_cast<size_t>(c + 1) * nblk] : n;
  for (int f = threadIdx.x; f < fine; f += kThreads) fcnt[f] = 0;
  __syncthreads();
  const uint32_t base_bucket = static_cast<uint32_t>(c) << sh;
  for (int64_t p = beg + threadIdx.x; p < end; p += kThreads) {
    const int32_t r = coarse[p];
    atomicAdd(&fcnt[bucket_of(splitmix64(seed, static_cast<uint64_t>(r)), t) - base_bucket], 1);
  }
  __syncthreads();
  // exclusive scan of the fine counters: each thread owns a run of them
  const int per = (fine + kThreads - 1) / kThreads;
  const int f0 = threadIdx.x * per;
  int32_t run = 0;
  for (int q = 0; q < per; ++q)
    if (f0 + q < fine) run += fcnt[f0 + q];
  int32_t tot;
  int32_t pre = block_exclusive_scan(run, wsum, &tot);
  for (int q = 0; q < per; ++q) {
    const int f = f0 + q;
    if (f < fine) {
      const int32_t v = fcnt[f];
      fcnt[f] = pre;
      if (base_bucket + static_cast<uint32_t>(f) < t) off[base_bucket + f] = static_cast<int32_t>(beg) + pre;
      pre += v;
    }
  }
  if (c == C - 1 && threadIdx.x == 0) off[t] = static_cast<int32_t>(n);
  __syncthreads();
  for (int64_t p = beg + threadIdx.x; p < end; p += kThreads) {
    const int32_t r = coarse[p];
    const uint32_t f = bucket_of(splitmix64(seed, static_cast<uint64_t>(r)), t) - base_bucket;
    perm[beg + atomicAdd(&fcnt[f], 1)] = r;
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
// One wavefront per bucket.  Rows are taken 64 at a time: one lane per row
// loads the row's extent, a wave-wide scan turns the lengths into offsets, and
// the chunk's nonzeros are then walked as one flat list (a 6-step binary
// search in LDS maps each position to its row), so the loads of col/val are
// independent of each other and many are in flight.  Products accumulate into
// a per-wave LDS row of S A, written once at the end.
template <typename TR, typename TO>
struct FlatLds {
  TO scale[kSortCap];
  int32_t src[kSortCap];
  int32_t dst[kSortCap];
  TR rstart[kWave];
  int32_t pfx[kWave];
  TO rscale[kWave];
};

constexpr int kFlatUnroll = 4;

template <typename TV, typename TR, typename TO>
__global__ __launch_bounds__(kThreads) void k_sketch_csr_sorted(
    int d, uint32_t t, uint64_t seed, const TR* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const TV* __restrict__ val, const void* __restrict__ b, int b_f64, const float* __restrict__ w,
    const int32_t* __restrict__ off, const int32_t* __restrict__ perm, TO* __restrict__ SA, TO* __restrict__ Sb,
    int per_wave) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const uint32_t bkt = blockIdx.x * kBucketWaves + wid;
  if (bkt >= t) return;
  unsigned char* base = smem + static_cast<size_t>(wid) * per_wave;
  FlatLds<TR, TO>& L = *reinterpret_cast<FlatLds<TR, TO>*>(base);
  TO* acc = reinterpret_cast<TO*>(base + sizeof(FlatLds<TR, TO>));
  for (int k = lane; k < d; k += kWave) acc[k] = TO(0);
  const int beg = off[bkt], m = off[bkt + 1] - beg;
  const bool sorted = load_bucket<TO>(perm, beg, m, seed, w, L.src, L.dst, L.scale, lane);
  TO sb = TO(0);
  for (int j0 = 0; j0 < m; j0 += kWave) {
    const int j = j0 + lane;
    TR rs = 0;
    int32_t len = 0;
    TO sc = TO(0);
    if (j < m) {
      const int32_t r = sorted ? L.dst[j] : perm[beg + j];
      sc = sorted ? L.scale[j] : row_scale<TO>(seed, r, w);
      rs = row_ptr[r];
      len = static_cast<int32_t>(row_ptr[r + 1] - rs);
      if (b != nullptr) sb += sc * load_b<TO>(b, b_f64, r);
    }
    int32_t incl = len;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int32_t y = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += y;
    }
    const int32_t total = __builtin_amdgcn_readlane(incl, kWave - 1);
    L.pfx[lane] = incl - len;
    L.rstart[lane] = rs;
    L.rscale[lane] = sc;
    wave_sync();
    for (int p0 = 0; p0 < total; p0 += kWave * kFlatUnroll) {
      int32_t cidx[kFlatUnroll];
      TO v[kFlatUnroll];
#pragma unroll
      for (int u = 0; u < kFlatUnroll; ++u) {
        const int p = p0 + u * kWave + lane;
        cidx[u] = -1;
        if (p < total) {
          int q = 0;  // largest q with pfx[q] <= p (empty rows share the next row's offset)
#pragma unroll
          for (int step = kWave / 2; step > 0; step >>= 1)
            if (L.pfx[q + step] <= p) q += step;
          const TR k = L.rstart[q] + static_cast<TR>(p - L.pfx[q]);
          cidx[u] = col[k];
          v[u] = L.rscale[q] * load_as<TO>(val, static_cast<size_t>(k));
        }
      }
#pragma unroll
      for (int u = 0; u < kFlatUnroll; ++u)
        if (cidx[u] >= 0) atomicAdd(&acc[cidx[u]], v[u]);
    }
    wave_sync();
  }
  sb = wave_sum(sb);
  TO* out = SA + static_cast<size_t>(bkt) * d;
  for (int c = lane; c < d; c += kWave) out[c] = acc[c];
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
  // coarse bins of 2^sh buckets holding about 4096 rows each on average
  int sh = 0;
  while (sh < 12 && (n << (sh + 1)) <= int64_t(4096) * t) ++sh;
  const int64_t C = (t + (int64_t(1) << sh) - 1) >> sh;
  P.sh = sh;
  P.C = C <= 4096 ? static_cast<int>(C) : 0;  // 0: counting with global atomics
  P.nblk = static_cast<int>(div_up(n > 0 ? n : 1, kPlanChunk));
  const int64_t ncnt = P.C ? static_cast<int64_t>(P.C) * P.nblk : t;
  P.off = ar.take<int32_t>(static_cast<size_t>(t) + 1);
  P.perm = ar.take<int32_t>(static_cast<size_t>(n));
  P.rank = ar.take<int32_t>(static_cast<size_t>(n));
  P.count = ar.take<int32_t>(static_cast<size_t>(ncnt) + 1);
  P.bsum = ar.take<int32_t>(static_cast<size_t>(div_up(ncnt, kScanTile)) + 1);
  return P;
}

// Exclusive scan of count[0..ncnt) into out[0..ncnt) with out[ncnt] = total.
int32_t scan_counts(const int32_t* count, int64_t ncnt, int32_t* bsum, int32_t* out, hipStream_t s) {
  const int64_t nb = div_up(ncnt, kScanTile);
  hipLaunchKernelGGL(k_scan_reduce, dim3(static_cast<unsigned>(nb)), dim3(kThreads), 0, s, count, ncnt, bsum);
  SKLS_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kThreads), 0, s, bsum, nb, out + ncnt);
  SKLS_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_scan_down, dim3(static_cast<unsigned>(nb)), dim3(kThreads), 0, s, count, ncnt, bsum, out);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t build_plan(int64_t n, uint32_t t, uint64_t seed, const BucketPlan& P, hipStream_t s) {
  if (P.C > 0) {
    const size_t lds = static_cast<size_t>(P.C) * sizeof(int32_t);
    const int64_t ncnt = static_cast<int64_t>(P.C) * P.nblk;
    hipLaunchKernelGGL(k_plan_coarse_count, dim3(P.nblk), dim3(kThreads), lds, s, n, t, seed, P.sh, P.C, P.nblk,
                       P.count);
    SKLS_CHECK_LAUNCH();
    // the scanned (bin, block) offsets overwrite the counts in place (each
    // scan block reads its tile before writing it)
    SKLS_TRY(scan_counts(P.count, ncnt, P.bsum, P.count, s));
    hipLaunchKernelGGL(k_plan_coarse_scatter, dim3(P.nblk), dim3(kThreads), lds, s, n, t, seed, P.sh, P.C, P.nblk,
                       P.count, P.rank);
    SKLS_CHECK_LAUNCH();
    const size_t flds = (size_t(1) << P.sh) * sizeof(int32_t);
    hipLaunchKernelGGL(k_plan_fine, dim3(P.C), dim3(kThreads), flds, s, n, t, seed, P.sh, P.C, P.nblk, P.count,
                       P.rank, P.perm, P.off);
    SKLS_CHECK_LAUNCH();
    return SKLS_OK;
  }
  SKLS_TRY(launch_fill_zero(P.count, static_cast<size_t>(t) * sizeof(int32_t), s));
  const unsigned g = grid_for(n, kThreads, 16384);
  if (n > 0) {
    hipLaunchKernelGGL(k_count, dim3(g), dim3(kThreads), 0, s, n, t, seed, P.count, P.rank);
    SKLS_CHECK_LAUNCH();
  }
  SKLS_TRY(scan_counts(P.count, static_cast<int64_t>(t), P.bsum, P.off, s));
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
        const int per_wave = static_cast<int>((sizeof(FlatLds<TR, TO>) + row_bytes + 15) / 16 * 16);
        hipLaunchKernelGGL((k_sketch_csr_sorted<TV, TR, TO>), dim3(grid), dim3(kThreads),
                           static_cast<size_t>(per_wave) * kBucketWaves, s, d, tt, seed,
                           static_cast<const TR*>(A.row_ptr), A.col_idx, static_cast<const TV*>(A.val), b, b_f64, w,
                           P.off, P.perm, static_cast<TO*>(SA), static_cast<TO*>(Sb), per_wave);
        SKLS_CHECK_LAUNCH();
        return SKLS_OK;
      });
    });
  });
}

}  // namespace skls
