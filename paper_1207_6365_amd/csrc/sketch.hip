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
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "kernels.hpp"
#include "profile.hpp"

namespace skls {
namespace {

constexpr int kThreads = 256;
constexpr int kBucketWaves = kThreads / kWave;  // buckets per block in the sorted kernels
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

template <typename TR, bool EXT>
__global__ void k_scatter(int64_t n, uint32_t t, uint64_t seed, const int32_t* __restrict__ off,
                          const int32_t* __restrict__ rank, int32_t* __restrict__ perm, const TR* __restrict__ row_ptr,
                          TR* __restrict__ pstart, int32_t* __restrict__ plen) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint32_t h = bucket_of(splitmix64(seed, static_cast<uint64_t>(i)), t);
    const int64_t p = off[h] + rank[i];
    perm[p] = static_cast<int32_t>(i);
    if (EXT) {
      const TR s0 = row_ptr[i];
      pstart[p] = s0;
      plen[p] = static_cast<int32_t>(row_ptr[i + 1] - s0);
    }
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

// With EXT, each row also carries its CSR extent (start, length), read here
// in storage order, so the reduce kernels never gather row pointers.
template <typename TR, bool EXT>
__global__ __launch_bounds__(kThreads) void k_plan_coarse_scatter(int64_t n, uint32_t t, uint64_t seed, int sh, int C,
                                                                  int nblk, const int32_t* __restrict__ coff,
                                                                  int32_t* __restrict__ coarse,
                                                                  const TR* __restrict__ row_ptr,
                                                                  TR* __restrict__ cstart, int32_t* __restrict__ clen) {
  extern __shared__ int32_t pos[];  // [C]
  for (int c = threadIdx.x; c < C; c += kThreads) pos[c] = coff[static_cast<size_t>(c) * nblk + blockIdx.x];
  __syncthreads();
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kPlanChunk;
  for (int k = 0; k < kPlanItems; ++k) {
    const int64_t i = r0 + static_cast<int64_t>(k) * kThreads + threadIdx.x;
    if (i < n) {
      const int c = static_cast<int>(bucket_of(splitmix64(seed, static_cast<uint64_t>(i)), t) >> sh);
      const int32_t slot = atomicAdd(&pos[c], 1);
      coarse[slot] = static_cast<int32_t>(i);
      if (EXT) {
        const TR s0 = row_ptr[i];
        cstart[slot] = s0;
        clen[slot] = static_cast<int32_t>(row_ptr[i + 1] - s0);
      }
    }
  }
}

template <typename TR, bool EXT>
__global__ __launch_bounds__(kThreads) void k_plan_fine(int64_t n, uint32_t t, uint64_t seed, int sh, int C, int nblk,
                                                        const int32_t* __restrict__ coff,
                                                        const int32_t* __restrict__ coarse,
                                                        int32_t* __restrict__ perm, int32_t* __restrict__ off,
                                                        const TR* __restrict__ cstart,
                                                        const int32_t* __restrict__ clen, TR* __restrict__ pstart,
                                                        int32_t* __restrict__ plen) {
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
    const int64_t dstp = beg + atomicAdd(&fcnt[f], 1);
    perm[dstp] = r;
    if (EXT) {
      pstart[dstp] = cstart[p];
      plen[dstp] = clen[p];
    }
  }
}

// ---------------------------------------------------------------- a2: CSR, sorted
// A wavefront reduces one bucket at a time.  The plan already carries each row's extent
// (start, length), so the bucket's rows are loaded with coalesced reads and
// sorted by row id (up to kCsrSortCap rows, two per lane).  Rows are then
// taken 64 at a time: a wave-wide scan of the lengths gives each row its
// offset in the chunk's flat list of nonzeros, a byte table in LDS maps every
// position of that list to its row, and the column/value loads of up to
// 64 * kBurst positions are issued back to back before their products are
// added into the per-wave LDS row of S A (written once at the end).
constexpr int kCsrSortCap = 2 * kWave;
constexpr int kPosCap = 2048;
constexpr int kBurst = 16;

template <typename TR, typename TO>
struct CsrLds {
  TO dscale[kCsrSortCap];
  TR dstart[kCsrSortCap];
  int32_t dlen[kCsrSortCap];
  int32_t drow[kCsrSortCap];
  TR base[kWave];      // row start minus its offset in the flat list
  TO rscale[kWave];
  int32_t pfx[kWave];  // offsets (binary search when the table does not fit)
  uint8_t pos2row[kPosCap];
};

template <typename TV, typename TR, typename TO, bool TABLE>
__device__ __forceinline__ void csr_burst(const CsrLds<TR, TO>& L, const int32_t* __restrict__ col,
                                          const TV* __restrict__ val, TO* acc, int p0, int total, int lane) {
  int32_t c[kBurst];
  TO v[kBurst];
  bool ok[kBurst];
#pragma unroll
  for (int u = 0; u < kBurst; ++u) {
    const int p = p0 + u * kWave + lane;
    ok[u] = p < total;
    const int pp = ok[u] ? p : 0;
    int q;
    if (TABLE) {
      q = L.pos2row[pp];
    } else {
      q = 0;  // largest q with pfx[q] <= pp (empty rows share the next offset)
#pragma unroll
      for (int step = kWave / 2; step > 0; step >>= 1)
        if (L.pfx[q + step] <= pp) q += step;
    }
    const TR k = L.base[q] + static_cast<TR>(pp);
    c[u] = col[k];
    v[u] = L.rscale[q] * load_as<TO>(val, static_cast<size_t>(k));
  }
#pragma unroll
  for (int u = 0; u < kBurst; ++u)
    if (ok[u]) atomicAdd(&acc[c[u]], v[u]);
}

// Four consecutive values of a row (16-byte aligned group of nonzeros).
template <typename TV, typename TO>
struct Quad {
  __device__ __forceinline__ static void load(const TV* __restrict__ p, TO (&o)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = load_as<TO>(p, k);
  }
};
template <typename TO>
struct Quad<float, TO> {
  __device__ __forceinline__ static void load(const float* __restrict__ p, TO (&o)[4]) {
    const float4 x = *reinterpret_cast<const float4*>(p);
    o[0] = x.x;
    o[1] = x.y;
    o[2] = x.z;
    o[3] = x.w;
  }
};
template <typename TO>
struct Quad<double, TO> {
  __device__ __forceinline__ static void load(const double* __restrict__ p, TO (&o)[4]) {
    const double2 x = *reinterpret_cast<const double2*>(p);
    const double2 y = *reinterpret_cast<const double2*>(p + 2);
    o[0] = static_cast<TO>(x.x);
    o[1] = static_cast<TO>(x.y);
    o[2] = static_cast<TO>(y.x);
    o[3] = static_cast<TO>(y.y);
  }
};
template <typename TO>
struct Quad<bf16_t, TO> {
  __device__ __forceinline__ static void load(const bf16_t* __restrict__ p, TO (&o)[4]) {
    const uint2 x = *reinterpret_cast<const uint2*>(p);
    o[0] = bf16_lo(x.x);
    o[1] = bf16_hi(x.x);
    o[2] = bf16_lo(x.y);
    o[3] = bf16_hi(x.y);
  }
};

// Burst over groups of four nonzeros (rows whose start and length are
// multiples of four): one 16-byte load of columns and one of values per
// lane, so a load instruction covers sixteen rows of sixteen nonzeros.
constexpr int kBurstQ = 4;

template <typename TV, typename TR, typename TO, bool TABLE>
__device__ __forceinline__ void csr_burst_quad(const CsrLds<TR, TO>& L, const int32_t* __restrict__ col,
                                               const TV* __restrict__ val, TO* acc, int p0, int total, int lane) {
  int4 c[kBurstQ];
  TO v[kBurstQ][4];
  TO sc[kBurstQ];
  bool ok[kBurstQ];
#pragma unroll
  for (int u = 0; u < kBurstQ; ++u) {
    const int p = p0 + u * kWave + lane;
    ok[u] = p < total;
    const int pp = ok[u] ? p : 0;
    int q;
    if (TABLE) {
      q = L.pos2row[pp];
    } else {
      q = 0;
#pragma unroll
      for (int step = kWave / 2; step > 0; step >>= 1)
        if (L.pfx[q + step] <= pp) q += step;
    }
    const TR k = L.base[q] + static_cast<TR>(4 * pp);
    c[u] = *reinterpret_cast<const int4*>(col + k);
    Quad<TV, TO>::load(val + k, v[u]);
    sc[u] = L.rscale[q];
  }
#pragma unroll
  for (int u = 0; u < kBurstQ; ++u)
    if (ok[u]) {
      atomicAdd(&acc[c[u].x], sc[u] * v[u][0]);
      atomicAdd(&acc[c[u].y], sc[u] * v[u][1]);
      atomicAdd(&acc[c[u].z], sc[u] * v[u][2]);
      atomicAdd(&acc[c[u].w], sc[u] * v[u][3]);
    }
}

// Prefetched description of one bucket: its range in the plan and, for up
// to two rows per lane, the row id, extent and length.
template <typename TR>
struct CsrMeta {
  int beg, m;
  int32_t r0, r1, l0, l1;
  TR s0, s1;
};

template <typename TR>
__device__ __forceinline__ CsrMeta<TR> csr_meta(const int32_t* __restrict__ perm, const TR* __restrict__ pstart,
                                                const int32_t* __restrict__ plen, int beg, int m, int lane) {
  CsrMeta<TR> q;
  q.beg = beg;
  q.m = m;
  const bool h0 = lane < m && m <= kCsrSortCap, h1 = lane + kWave < m && m <= kCsrSortCap;
  q.r0 = h0 ? perm[beg + lane] : INT_MAX;
  q.r1 = h1 ? perm[beg + kWave + lane] : INT_MAX;
  q.s0 = h0 ? pstart[beg + lane] : TR(0);
  q.s1 = h1 ? pstart[beg + kWave + lane] : TR(0);
  q.l0 = h0 ? plen[beg + lane] : 0;
  q.l1 = h1 ? plen[beg + kWave + lane] : 0;
  return q;
}

// Each wavefront owns `bpw` consecutive buckets and walks them in order,
// loading the next bucket's rows while it reduces the current one.
template <typename TV, typename TR, typename TO>
__global__ __launch_bounds__(kThreads) void k_sketch_csr_sorted(
    int d, uint32_t t, int bpw, uint64_t seed, const int32_t* __restrict__ col, const TV* __restrict__ val,
    const void* __restrict__ b, int b_f64, const float* __restrict__ w, const int32_t* __restrict__ off,
    const int32_t* __restrict__ perm, const TR* __restrict__ pstart, const int32_t* __restrict__ plen,
    TO* __restrict__ SA, TO* __restrict__ Sb, int per_wave, int quad_ok) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int64_t b0 = (static_cast<int64_t>(blockIdx.x) * kBucketWaves + wid) * bpw;
  if (b0 >= t) return;
  const int nb = static_cast<int>((t - b0) < bpw ? (t - b0) : bpw);
  unsigned char* base = smem + static_cast<size_t>(wid) * per_wave;
  CsrLds<TR, TO>& L = *reinterpret_cast<CsrLds<TR, TO>*>(base);
  TO* acc = reinterpret_cast<TO*>(base + sizeof(CsrLds<TR, TO>));
  // bucket offsets of this wave's range (bpw < 64): lane k holds off[b0 + k]
  const int32_t myoff = lane <= nb ? off[b0 + lane] : 0;
  auto off_at = [&](int k) -> int32_t { return __builtin_amdgcn_readlane(myoff, k); };
  CsrMeta<TR> cur = csr_meta<TR>(perm, pstart, plen, off_at(0), off_at(1) - off_at(0), lane);
  for (int kb = 0; kb < nb; ++kb) {
    const uint32_t bkt = static_cast<uint32_t>(b0 + kb);
    CsrMeta<TR> nxt = cur;
    if (kb + 1 < nb) {
      const int nbeg = off_at(kb + 1);
      nxt = csr_meta<TR>(perm, pstart, plen, nbeg, off_at(kb + 2) - nbeg, lane);
    }
    for (int k = lane; k < d; k += kWave) acc[k] = TO(0);
    const int beg = cur.beg, m = cur.m;
    const bool sorted = m <= kCsrSortCap;
    if (sorted) {
      int rk0 = 0, rk1 = 0;
      const int m0 = m < kWave ? m : kWave;
      for (int k = 0; k < m0; ++k) {
        const int32_t x = __builtin_amdgcn_readlane(cur.r0, k);
        rk0 += x < cur.r0 ? 1 : 0;
        rk1 += x < cur.r1 ? 1 : 0;
      }
      for (int k = kWave; k < m; ++k) {
        const int32_t x = __builtin_amdgcn_readlane(cur.r1, k - kWave);
        rk0 += x < cur.r0 ? 1 : 0;
        rk1 += x < cur.r1 ? 1 : 0;
      }
      if (lane < m) {
        L.drow[rk0] = cur.r0;
        L.dstart[rk0] = cur.s0;
        L.dlen[rk0] = cur.l0;
        L.dscale[rk0] = row_scale<TO>(seed, cur.r0, w);
      }
      if (lane + kWave < m) {
        L.drow[rk1] = cur.r1;
        L.dstart[rk1] = cur.s1;
        L.dlen[rk1] = cur.l1;
        L.dscale[rk1] = row_scale<TO>(seed, cur.r1, w);
      }
    }
    wave_sync();
    TO sb = TO(0);
    for (int j0 = 0; j0 < m; j0 += kWave) {
      const int j = j0 + lane;
      int32_t len = 0;
      TR st = 0;
      TO sc = TO(0);
      if (j < m) {
        int32_t r;
        if (sorted) {
          r = L.drow[j];
          st = L.dstart[j];
          len = L.dlen[j];
          sc = L.dscale[j];
        } else {
          r = perm[beg + j];
          st = pstart[beg + j];
          len = plen[beg + j];
          sc = row_scale<TO>(seed, r, w);
        }
        if (b != nullptr) sb += sc * load_b<TO>(b, b_f64, r);
      }
      // groups of four nonzeros when every row of the chunk allows it
      const bool quad = quad_ok && __all(((static_cast<int64_t>(st) | len) & 3) == 0);
      const int32_t units = quad ? (len >> 2) : len;
      int32_t incl = units, mx = units;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int32_t y = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += y;
        const int32_t z = __shfl_xor(mx, o, kWave);
        mx = z > mx ? z : mx;
      }
      const int32_t total = __builtin_amdgcn_readlane(incl, kWave - 1);
      const int32_t pf = incl - units;
      L.base[lane] = st - static_cast<TR>(quad ? 4 * pf : pf);
      L.rscale[lane] = sc;
      L.pfx[lane] = pf;
      const bool table = total <= kPosCap && mx <= kWave;
      if (table)
        for (int e = 0; e < mx; ++e)
          if (e < units) L.pos2row[pf + e] = static_cast<uint8_t>(lane);
      wave_sync();
      // Branch-free bursts: positions past the end read position 0 (always
      // valid when total > 0) and are masked afterwards, so every load of
      // the burst is issued before the first wait.
      if (quad) {
        if (table) {
          for (int p0 = 0; p0 < total; p0 += kWave * kBurstQ)
            csr_burst_quad<TV, TR, TO, true>(L, col, val, acc, p0, total, lane);
        } else {
          for (int p0 = 0; p0 < total; p0 += kWave * kBurstQ)
            csr_burst_quad<TV, TR, TO, false>(L, col, val, acc, p0, total, lane);
        }
      } else if (table) {
        for (int p0 = 0; p0 < total; p0 += kWave * kBurst)
          csr_burst<TV, TR, TO, true>(L, col, val, acc, p0, total, lane);
      } else {
        for (int p0 = 0; p0 < total; p0 += kWave * kBurst)
          csr_burst<TV, TR, TO, false>(L, col, val, acc, p0, total, lane);
      }
      wave_sync();
    }
    sb = wave_sum(sb);
    TO* out = SA + static_cast<size_t>(bkt) * d;
    for (int c = lane; c < d; c += kWave) out[c] = acc[c];
    if (Sb != nullptr && lane == 0) Sb[bkt] = sb;
    wave_sync();
    cur = nxt;
  }
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

// Each wavefront owns `bpw` consecutive buckets; the next bucket's row ids are
// loaded while the current bucket's rows are summed in registers (lanes own
// column slices, 8 rows in flight).
template <typename TO>
struct DenseLds {
  TO dscale[kCsrSortCap];
  int32_t drow[kCsrSortCap];
};

// Sum of the bucket's rows for this lane's column slices.  Batches of RB rows
// are loaded unconditionally (rows past the end repeat row 0 and are skipped
// when summing), so all loads of a batch are in flight together; rows are
// added in bucket order.
template <typename TV, typename TO, int V, bool SORTED>
__device__ __forceinline__ void dense_rows(const DenseLds<TO>& L, const int32_t* __restrict__ perm, int beg, int m,
                                           uint64_t seed, const float* __restrict__ w, const TV* __restrict__ A,
                                           int64_t ld, int d, TO* __restrict__ out, int lane) {
  constexpr int RB = 8;
  for (int c0 = lane * V; c0 < d; c0 += kWave * V) {
    TO acc[V];
#pragma unroll
    for (int k = 0; k < V; ++k) acc[k] = TO(0);
    for (int j = 0; j < m; j += RB) {
      TO sc[RB], x[RB][V];
      bool ok[RB];
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        ok[q] = j + q < m;
        const int jc = ok[q] ? j + q : 0;
        const int32_t r = SORTED ? L.drow[jc] : perm[beg + jc];
        sc[q] = SORTED ? L.dscale[jc] : row_scale<TO>(seed, r, w);
        RowLoad<TV, TO, V>::load(A + static_cast<size_t>(r) * ld + c0, x[q]);
      }
#pragma unroll
      for (int q = 0; q < RB; ++q)
        if (ok[q])
#pragma unroll
          for (int k = 0; k < V; ++k) acc[k] += sc[q] * x[q][k];
    }
#pragma unroll
    for (int k = 0; k < V; ++k) out[c0 + k] = acc[k];
  }
}

template <typename TV, typename TO, int V>
__global__ __launch_bounds__(kThreads) void k_sketch_dense_sorted(
    int d, int64_t ld, uint32_t t, int bpw, uint64_t seed, const TV* __restrict__ A, const void* __restrict__ b,
    int b_f64, const float* __restrict__ w, const int32_t* __restrict__ off, const int32_t* __restrict__ perm,
    TO* __restrict__ SA, TO* __restrict__ Sb) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int64_t b0 = (static_cast<int64_t>(blockIdx.x) * kBucketWaves + wid) * bpw;
  if (b0 >= t) return;
  const int nb = static_cast<int>((t - b0) < bpw ? (t - b0) : bpw);
  DenseLds<TO>& L = *reinterpret_cast<DenseLds<TO>*>(smem + static_cast<size_t>(wid) * sizeof(DenseLds<TO>));
  const int32_t myoff = lane <= nb ? off[b0 + lane] : 0;
  auto off_at = [&](int k) -> int32_t { return __builtin_amdgcn_readlane(myoff, k); };
  auto fetch = [&](int beg, int m, int32_t& r0, int32_t& r1) {
    const bool ok = m <= kCsrSortCap;
    r0 = (ok && lane < m) ? perm[beg + lane] : INT_MAX;
    r1 = (ok && lane + kWave < m) ? perm[beg + kWave + lane] : INT_MAX;
  };
  int beg = off_at(0), m = off_at(1) - beg;
  int32_t r0, r1;
  fetch(beg, m, r0, r1);
  for (int kb = 0; kb < nb; ++kb) {
    const uint32_t bkt = static_cast<uint32_t>(b0 + kb);
    int nbeg = beg, nm = m;
    int32_t n0 = r0, n1 = r1;
    if (kb + 1 < nb) {
      nbeg = off_at(kb + 1);
      nm = off_at(kb + 2) - nbeg;
      fetch(nbeg, nm, n0, n1);
    }
    const bool sorted = m <= kCsrSortCap;
    if (sorted) {
      int rk0 = 0, rk1 = 0;
      const int m0 = m < kWave ? m : kWave;
      for (int k = 0; k < m0; ++k) {
        const int32_t x = __builtin_amdgcn_readlane(r0, k);
        rk0 += x < r0 ? 1 : 0;
        rk1 += x < r1 ? 1 : 0;
      }
      for (int k = kWave; k < m; ++k) {
        const int32_t x = __builtin_amdgcn_readlane(r1, k - kWave);
        rk0 += x < r0 ? 1 : 0;
        rk1 += x < r1 ? 1 : 0;
      }
      if (lane < m) {
        L.drow[rk0] = r0;
        L.dscale[rk0] = row_scale<TO>(seed, r0, w);
      }
      if (lane + kWave < m) {
        L.drow[rk1] = r1;
        L.dscale[rk1] = row_scale<TO>(seed, r1, w);
      }
    }
    wave_sync();
    if (Sb != nullptr) {
      TO sb = TO(0);
      for (int j = lane; j < m; j += kWave) {
        const int32_t r = sorted ? L.drow[j] : perm[beg + j];
        sb += (sorted ? L.dscale[j] : row_scale<TO>(seed, r, w)) * load_b<TO>(b, b_f64, r);
      }
      sb = wave_sum(sb);
      if (lane == 0) Sb[bkt] = sb;
    }
    TO* out = SA + static_cast<size_t>(bkt) * d;
    if (sorted)
      dense_rows<TV, TO, V, true>(L, perm, beg, m, seed, w, A, ld, d, out, lane);
    else
      dense_rows<TV, TO, V, false>(L, perm, beg, m, seed, w, A, ld, d, out, lane);
    wave_sync();
    beg = nbeg;
    m = nm;
    r0 = n0;
    r1 = n1;
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

size_t plan_bytes(int64_t n, int64_t t, int ext) {
  Arena ar(nullptr, 0);
  carve_plan(ar, n, t, ext);
  return ar.used;
}

BucketPlan carve_plan(Arena& ar, int64_t n, int64_t t, int ext) {
  BucketPlan P;
  // coarse bins of 2^sh buckets holding about 4096 rows each on average
  int sh = 0;
  while (sh < 12 && (n << (sh + 1)) <= int64_t(4096) * t) ++sh;
  const int64_t C = (t + (int64_t(1) << sh) - 1) >> sh;
  P.sh = sh;
  P.C = C <= 4096 ? static_cast<int>(C) : 0;  // 0: counting with global atomics
  P.nblk = static_cast<int>(div_up(n > 0 ? n : 1, kPlanChunk));
  P.ext = ext;
  const int64_t ncnt = P.C ? static_cast<int64_t>(P.C) * P.nblk : t;
  P.off = ar.take<int32_t>(static_cast<size_t>(t) + 1);
  P.perm = ar.take<int32_t>(static_cast<size_t>(n));
  P.rank = ar.take<int32_t>(static_cast<size_t>(n));
  P.count = ar.take<int32_t>(static_cast<size_t>(ncnt) + 1);
  P.bsum = ar.take<int32_t>(static_cast<size_t>(div_up(ncnt, kScanTile)) + 1);
  if (ext) {
    P.pstart = ar.take<char>(static_cast<size_t>(n) * ext);
    P.plen = ar.take<int32_t>(static_cast<size_t>(n));
    P.cstart = ar.take<char>(static_cast<size_t>(n) * ext);
    P.clen = ar.take<int32_t>(static_cast<size_t>(n));
  }
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

template <typename TR, bool EXT>
int32_t build_plan_t(int64_t n, uint32_t t, uint64_t seed, const BucketPlan& P, const TR* row_ptr, hipStream_t s) {
  TR* cstart = static_cast<TR*>(P.cstart);
  TR* pstart = static_cast<TR*>(P.pstart);
  if (P.C > 0) {
    const size_t lds = static_cast<size_t>(P.C) * sizeof(int32_t);
    const int64_t ncnt = static_cast<int64_t>(P.C) * P.nblk;
    hipLaunchKernelGGL(k_plan_coarse_count, dim3(P.nblk), dim3(kThreads), lds, s, n, t, seed, P.sh, P.C, P.nblk,
                       P.count);
    SKLS_CHECK_LAUNCH();
    // the scanned (bin, block) offsets overwrite the counts in place (each
    // scan block reads its tile before writing it)
    SKLS_TRY(scan_counts(P.count, ncnt, P.bsum, P.count, s));
    hipLaunchKernelGGL((k_plan_coarse_scatter<TR, EXT>), dim3(P.nblk), dim3(kThreads), lds, s, n, t, seed, P.sh, P.C,
                       P.nblk, P.count, P.rank, row_ptr, cstart, P.clen);
    SKLS_CHECK_LAUNCH();
    const size_t flds = (size_t(1) << P.sh) * sizeof(int32_t);
    hipLaunchKernelGGL((k_plan_fine<TR, EXT>), dim3(P.C), dim3(kThreads), flds, s, n, t, seed, P.sh, P.C, P.nblk,
                       P.count, P.rank, P.perm, P.off, cstart, P.clen, pstart, P.plen);
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
    hipLaunchKernelGGL((k_scatter<TR, EXT>), dim3(g), dim3(kThreads), 0, s, n, t, seed, P.off, P.rank, P.perm,
                       row_ptr, pstart, P.plen);
    SKLS_CHECK_LAUNCH();
  }
  return SKLS_OK;
}

int32_t build_plan(int64_t n, uint32_t t, uint64_t seed, const BucketPlan& P, const void* row_ptr, hipStream_t s) {
  if (P.ext == 8) return build_plan_t<int64_t, true>(n, t, seed, P, static_cast<const int64_t*>(row_ptr), s);
  if (P.ext == 4) return build_plan_t<int32_t, true>(n, t, seed, P, static_cast<const int32_t*>(row_ptr), s);
  return build_plan_t<int32_t, false>(n, t, seed, P, nullptr, s);
}

// Bytes per carried row start in the plan (0 for dense inputs).
int plan_ext(const skls_matrix& A) {
  if (A.layout != SKLS_CSR) return 0;
  return A.row_ptr_64 ? 8 : 4;
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
  if (v == SKLS_SKETCH_SORTED) return plan_bytes(A.n, t, plan_ext(A));
  return 0;
}

// Wavefronts of a kBucketWaves-wave block kernel that the device holds at
// once (occupancy from registers and LDS), cached per kernel, LDS size and
// device.
static int64_t resident_waves(const void* kernel, size_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, size_t, int>, int64_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  const auto key = std::make_tuple(kernel, lds, dev);
  std::lock_guard<std::mutex> lock(mu);
  const auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
  const int64_t r = static_cast<int64_t>(per_cu) * cus * kBucketWaves;
  cache.emplace(key, r);
  return r;
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
  BucketPlan P = carve_plan(ar, n, t, plan_ext(A));
  if (!ws || !ar.fits()) {
    set_error("sketch workspace too small: need %zu bytes, have %zu", ar.used, ws_bytes);
    return SKLS_ERR_WORKSPACE;
  }
  {
    PhaseTimer pt("sketch_plan", s);
    SKLS_TRY(build_plan(n, tt, seed, P, A.layout == SKLS_CSR ? A.row_ptr : nullptr, s));
  }
  PhaseTimer pt("sketch_apply", s);
  return with_out(out_dtype, [&](auto to) -> int32_t {
    using TO = decltype(to);
    return with_value(A.dtype, [&](auto tv) -> int32_t {
      using TV = decltype(tv);
      if (A.layout == SKLS_DENSE) {
        const size_t lds = kBucketWaves * sizeof(DenseLds<TO>);
        constexpr int VV = sizeof(TV) == 8 ? 2 : (sizeof(TV) == 4 ? 4 : 8);
        const bool vec = vec_ok<TV>(A.val, A.ld, A.d, VV);
        const void* kern = vec ? reinterpret_cast<const void*>(&k_sketch_dense_sorted<TV, TO, VV>)
                               : reinterpret_cast<const void*>(&k_sketch_dense_sorted<TV, TO, 1>);
        int bpw = static_cast<int>(div_up(t, resident_waves(kern, lds)));
        bpw = bpw < 1 ? 1 : (bpw > 63 ? 63 : bpw);
        const unsigned dgrid = static_cast<unsigned>(div_up(div_up(t, bpw), kBucketWaves));
        if (vec) {
          hipLaunchKernelGGL((k_sketch_dense_sorted<TV, TO, VV>), dim3(dgrid), dim3(kThreads), lds, s, d, A.ld, tt,
                             bpw, seed, static_cast<const TV*>(A.val), b, b_f64, w, P.off, P.perm,
                             static_cast<TO*>(SA), static_cast<TO*>(Sb));
        } else {
          hipLaunchKernelGGL((k_sketch_dense_sorted<TV, TO, 1>), dim3(dgrid), dim3(kThreads), lds, s, d, A.ld, tt,
                             bpw, seed, static_cast<const TV*>(A.val), b, b_f64, w, P.off, P.perm,
                             static_cast<TO*>(SA), static_cast<TO*>(Sb));
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
        const int per_wave = static_cast<int>((sizeof(CsrLds<TR, TO>) + row_bytes + 15) / 16 * 16);
        // one round of resident wavefronts, each walking consecutive buckets
        const size_t lds = static_cast<size_t>(per_wave) * kBucketWaves;
        int cbpw = static_cast<int>(div_up(t, resident_waves(
                                                  reinterpret_cast<const void*>(&k_sketch_csr_sorted<TV, TR, TO>), lds)));
        cbpw = cbpw < 1 ? 1 : (cbpw > 63 ? 63 : cbpw);
        const unsigned cgrid = static_cast<unsigned>(div_up(div_up(t, cbpw), kBucketWaves));
        const int quad_ok = (reinterpret_cast<uintptr_t>(A.col_idx) % 16 == 0) &&
                            (reinterpret_cast<uintptr_t>(A.val) % (4 * sizeof(TV)) == 0);
        hipLaunchKernelGGL((k_sketch_csr_sorted<TV, TR, TO>), dim3(cgrid), dim3(kThreads), lds, s, d, tt, cbpw,
                           seed, A.col_idx,
                           static_cast<const TV*>(A.val), b, b_f64, w, P.off, P.perm,
                           static_cast<const TR*>(P.pstart), P.plen, static_cast<TO*>(SA), static_cast<TO*>(Sb),
                           per_wave, quad_ok);
        SKLS_CHECK_LAUNCH();
        return SKLS_OK;
      });
    });
  });
}

}  // namespace skls
