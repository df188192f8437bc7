// Sparse embedding S = Phi D applied to A and b (Section 2 of Clarkson &
// Woodruff; the O(nnz(A)) product behind the main theorem of Section 3 and the
// regression theorem of Section 7).
//
// Three schedules of the same sum SA[h(i), :] += sign(i) * A[i, :]:
//  * ATOMIC: rows are streamed in storage order (fully coalesced reads of A)
//    and every entry is added into SA with a device-wide float atomic.
//  * BINNED: a counting sort groups the rows into coarse bins of consecutive
//    buckets; one block holds a bin's rows of SA in LDS, streams the bin's
//    rows and adds them with LDS atomics, then writes its rows of SA once.
//  * SORTED: a second counting pass orders each bin by bucket; one wavefront
//    owns one bucket, sorts its row ids, reduces its rows in increasing row
//    order (registers for dense rows, a per-wave LDS accumulator for CSR rows)
//    and writes its row of SA exactly once: bit-reproducible results.
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
__device__ __forceinline__ TS row_scale(HashKey seed, int64_t r, const float* __restrict__ w) {
  if (w) return static_cast<TS>(w[r]);
  return negative_of(hk_z(seed, static_cast<uint64_t>(r))) ? TS(-1) : TS(1);
}

template <typename TS>
__device__ __forceinline__ TS load_b(const void* __restrict__ b, int b_f64, int64_t r) {
  return b_f64 ? static_cast<TS>(static_cast<const double*>(b)[r]) : static_cast<TS>(static_cast<const float*>(b)[r]);
}

// ---------------------------------------------------------------- a1: hash
__global__ void k_hash(int64_t n, uint32_t t, HashKey seed, int64_t start, int32_t* __restrict__ bucket,
                       int8_t* __restrict__ sign) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint64_t z = hk_z(seed, static_cast<uint64_t>(start + i));
    if (bucket) bucket[i] = static_cast<int32_t>(hk_bucket(seed, z, static_cast<uint64_t>(start + i), t));
    if (sign) sign[i] = negative_of(z) ? int8_t(-1) : int8_t(1);
  }
}

template <typename T>
__global__ void k_scale(T* __restrict__ p, size_t count, T alpha) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[i] *= alpha;
}

__global__ void k_fill_zero(uint32_t* __restrict__ p, size_t words) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  const size_t vec = words / 4;
  uint4* p4 = reinterpret_cast<uint4*>(p);
  for (size_t k = i; k < vec; k += stride) p4[k] = make_uint4(0, 0, 0, 0);
  for (size_t k = vec * 4 + i; k < words; k += stride) p[k] = 0;
}

// ---------------------------------------------------------------- plan entries
// What the bucket plan carries per row.  Dense inputs: the row index.  CSR
// inputs: a record with the row's extent, its index and its share of S b, so
// the reduce kernels read row pointers and b only in storage order (here,
// while the plan is built) and never gather them.
template <typename TR, typename TO>
struct alignas(sizeof(TR) + sizeof(TO) == 8 ? 16 : 8) CsrRec {
  TR start;     // first nonzero of the row
  int32_t len;  // nonzeros in the row
  int32_t row;  // row index
  TO sbv;       // scale(row) * b[row], 0 without b
};
static_assert(sizeof(CsrRec<int32_t, float>) == 16, "record layout");
static_assert(sizeof(CsrRec<int64_t, float>) == 24, "record layout");
static_assert(sizeof(CsrRec<int32_t, double>) == 24, "record layout");
static_assert(sizeof(CsrRec<int64_t, double>) == 24, "record layout");

// Inputs the plan reads in storage order.
struct RowSrc {
  const void* row_ptr;  // CSR only
  const void* b;
  int b_f64;
  const float* w;
};

template <typename R>
struct Entry;
template <>
struct Entry<int32_t> {
  static constexpr bool kSb = false;
  using TO = float;
  __device__ __forceinline__ static int32_t make(const RowSrc&, int64_t i, uint64_t) {
    return static_cast<int32_t>(i);
  }
  __device__ __forceinline__ static int32_t extent(const RowSrc&, int64_t i) { return static_cast<int32_t>(i); }
  __device__ __forceinline__ static void set_sb(int32_t&, float) {}
  __device__ __forceinline__ static int32_t row(const int32_t& e) { return e; }
};
template <typename TR, typename TO_>
struct Entry<CsrRec<TR, TO_>> {
  static constexpr bool kSb = true;
  using TO = TO_;
  // the record without its share of S b
  __device__ __forceinline__ static CsrRec<TR, TO> extent(const RowSrc& src, int64_t i) {
    const TR* rp = static_cast<const TR*>(src.row_ptr);
    CsrRec<TR, TO> e;
    e.start = rp[i];
    e.len = static_cast<int32_t>(rp[i + 1] - e.start);
    e.row = static_cast<int32_t>(i);
    e.sbv = TO(0);
    return e;
  }
  __device__ __forceinline__ static CsrRec<TR, TO> make(const RowSrc& src, int64_t i, uint64_t z) {
    CsrRec<TR, TO> e = extent(src, i);
    if (src.b != nullptr) {
      const TO sc = src.w ? static_cast<TO>(src.w[i]) : (negative_of(z) ? TO(-1) : TO(1));
      e.sbv = sc * load_b<TO>(src.b, src.b_f64, i);
    }
    return e;
  }
  __device__ __forceinline__ static void set_sb(CsrRec<TR, TO>& e, TO v) { e.sbv = v; }
  __device__ __forceinline__ static int32_t row(const CsrRec<TR, TO>& e) { return e.row; }
};

// ---------------------------------------------------------------- counting sort
// One-level counting sort with global atomics, for plans with too many coarse
// bins for the LDS counters of the two-level plan.
__global__ void k_count(int64_t n, uint32_t t, HashKey seed, int32_t* __restrict__ count, int32_t* __restrict__ rank) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint32_t h = hk_bucket_r(seed, static_cast<uint64_t>(i), t);
    rank[i] = atomicAdd(&count[h], 1);
  }
}

template <typename R>
__global__ void k_scatter(int64_t n, uint32_t t, HashKey seed, const int32_t* __restrict__ off,
                          const int32_t* __restrict__ rank, RowSrc src, R* __restrict__ out) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint64_t z = hk_z(seed, static_cast<uint64_t>(i));
    out[off[hk_bucket(seed, z, static_cast<uint64_t>(i), t)] + rank[i]] = Entry<R>::make(src, i, z);
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
// grouped into coarse bins of 2^sh consecutive buckets.
//  1. coarse count: each block counts its chunk of rows per coarse bin in LDS
//     and writes the counts bin-major, so an exclusive scan of the whole array
//     gives every (bin, block) its output offset;
//  2. coarse scatter: each block writes its rows' plan entries to those
//     offsets (LDS atomics hand out the slots);
//  3. fine pass (bucket order only): one block per coarse bin counts, scans
//     and scatters the bin's entries by bucket and writes the bucket offsets.
// Large row chunks per block keep each (block, bin) run of entries long, so
// the scattered writes of pass 2 stay close to whole cache lines.
constexpr int kPlanThreads = 1024;
constexpr int kPlanItems = 16;
constexpr int kPlanChunk = kPlanThreads * kPlanItems;  // rows per block in passes 1-2
constexpr int kMaxBins = 8192;                         // LDS counters of passes 1-2

__global__ __launch_bounds__(kPlanThreads) void k_plan_coarse_count(int64_t n, uint32_t t, HashKey seed, int sh,
                                                                    int C, int nblk, int32_t* __restrict__ cnt) {
  extern __shared__ int32_t hist[];  // [C]
  for (int c = threadIdx.x; c < C; c += kPlanThreads) hist[c] = 0;
  __syncthreads();
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kPlanChunk;
#pragma unroll 4
  for (int k = 0; k < kPlanItems; ++k) {
    const int64_t i = r0 + static_cast<int64_t>(k) * kPlanThreads + threadIdx.x;
    if (i < n) atomicAdd(&hist[hk_bucket_r(seed, static_cast<uint64_t>(i), t) >> sh], 1);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += kPlanThreads) cnt[static_cast<size_t>(c) * nblk + blockIdx.x] = hist[c];
}

template <typename R>
__global__ __launch_bounds__(kPlanThreads) void k_plan_coarse_scatter(int64_t n, uint32_t t, HashKey seed, int sh,
                                                                      int C, int nblk,
                                                                      const int32_t* __restrict__ coff, RowSrc src,
                                                                      R* __restrict__ coarse) {
  extern __shared__ int32_t pos[];  // [C]
  for (int c = threadIdx.x; c < C; c += kPlanThreads) pos[c] = coff[static_cast<size_t>(c) * nblk + blockIdx.x];
  __syncthreads();
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kPlanChunk;
  if (r0 >= n) return;
  // eight rows per thread at a time: their loads (clamped to the last row so
  // none sits behind a branch) are in flight together, then the slots, then
  // the stores
  // (the optional inputs b and w are read in batches of their own under
  // uniform branches)
  constexpr int kU = 8;
  using TO = typename Entry<R>::TO;
  for (int k0 = 0; k0 < kPlanItems; k0 += kU) {
    R e[kU];
    int32_t bin[kU];
    bool ok[kU];
    int64_t ii[kU];
    uint64_t z[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = r0 + static_cast<int64_t>(k0 + u) * kPlanThreads + threadIdx.x;
      ok[u] = i < n;
      ii[u] = ok[u] ? i : n - 1;
      z[u] = hk_z(seed, static_cast<uint64_t>(ii[u]));
      e[u] = Entry<R>::extent(src, ii[u]);
      bin[u] = static_cast<int32_t>(hk_bucket(seed, z[u], static_cast<uint64_t>(ii[u]), t) >> sh);
    }
    if (Entry<R>::kSb && src.b != nullptr) {
      TO bv[kU], sc[kU];
      if (src.b_f64) {
#pragma unroll
        for (int u = 0; u < kU; ++u) bv[u] = static_cast<TO>(static_cast<const double*>(src.b)[ii[u]]);
      } else {
#pragma unroll
        for (int u = 0; u < kU; ++u) bv[u] = static_cast<TO>(static_cast<const float*>(src.b)[ii[u]]);
      }
      if (src.w != nullptr) {
#pragma unroll
        for (int u = 0; u < kU; ++u) sc[u] = static_cast<TO>(src.w[ii[u]]);
      } else {
#pragma unroll
        for (int u = 0; u < kU; ++u) sc[u] = negative_of(z[u]) ? TO(-1) : TO(1);
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) Entry<R>::set_sb(e[u], sc[u] * bv[u]);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (ok[u]) coarse[atomicAdd(&pos[bin[u]], 1)] = e[u];
  }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_plan_fine(int64_t n, uint32_t t, HashKey seed, int sh, int C, int nblk,
                                                        const int32_t* __restrict__ coff, const R* __restrict__ coarse,
                                                        R* __restrict__ fine_out, int32_t* __restrict__ off) {
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
    const int32_t r = Entry<R>::row(coarse[p]);
    atomicAdd(&fcnt[hk_bucket_r(seed, static_cast<uint64_t>(r), t) - base_bucket], 1);
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
    const R e = coarse[p];
    const uint32_t f = hk_bucket_r(seed, static_cast<uint64_t>(Entry<R>::row(e)), t) - base_bucket;
    fine_out[beg + atomicAdd(&fcnt[f], 1)] = e;
  }
}

// ---------------------------------------------------------------- one-pass local plan
// Rows grouped by coarse bin within fixed chunks of PER * kPlanThreads rows,
// in one kernel: each block counts its chunk's rows per bin in LDS, scans the
// counts, builds every row's plan entry from row pointers read in storage
// order, places it at its slot in an LDS copy of the chunk (LDS atomics hand
// out the slots) and writes the chunk out in bin order, so every global read
// and write is coalesced.  The per-chunk bin offsets go to
// offT[nseg x (C + 1)] (row q holds chunk q's exclusive offsets, then its
// size): bin c of chunk q is out[q * chunk + offT[q][c] ..
// q * chunk + offT[q][c + 1]).
template <typename R, int PER>
__global__ __launch_bounds__(kPlanThreads) void k_plan_local(int64_t n, uint32_t t, HashKey seed, int sh, int C,
                                                             RowSrc src, R* __restrict__ out,
                                                             int32_t* __restrict__ offT, int nseg) {
  constexpr int CH = PER * kPlanThreads;
  extern __shared__ __align__(16) unsigned char smem[];
  R* stage = reinterpret_cast<R*>(smem);                       // [CH]
  int32_t* cnt = reinterpret_cast<int32_t*>(smem + sizeof(R) * CH);  // [C + 1]
  __shared__ int32_t wsum[kPlanThreads / kWave];
  const int q = blockIdx.x;
  const int64_t r0 = static_cast<int64_t>(q) * CH;
  const int m = static_cast<int>(n - r0 < CH ? (n - r0 > 0 ? n - r0 : 0) : CH);
  for (int c = threadIdx.x; c <= C; c += kPlanThreads) cnt[c] = 0;
  __syncthreads();
  int32_t bin[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int p = u * kPlanThreads + threadIdx.x;
    bin[u] = static_cast<int32_t>(hk_bucket_r(seed, static_cast<uint64_t>(r0 + p), t) >> sh);
    if (p < m) atomicAdd(&cnt[bin[u]], 1);
  }
  __syncthreads();
  // exclusive scan of cnt[0..C): each thread owns a run of counters
  const int per = (C + kPlanThreads - 1) / kPlanThreads;
  const int c0 = threadIdx.x * per;
  int32_t run = 0;
  for (int k = 0; k < per; ++k)
    if (c0 + k < C) run += cnt[c0 + k];
  int32_t tot;
  int32_t pre = block_exclusive_scan(run, wsum, &tot);
  for (int k = 0; k < per; ++k)
    if (c0 + k < C) {
      const int32_t v = cnt[c0 + k];
      cnt[c0 + k] = pre;
      pre += v;
    }
  if (threadIdx.x == 0) cnt[C] = m;
  __syncthreads();
  for (int c = threadIdx.x; c <= C; c += kPlanThreads) offT[static_cast<size_t>(q) * (C + 1) + c] = cnt[c];
  __syncthreads();
  if (m > 0) {
    // entries of this thread's rows, read in storage order with loads clamped
    // to the chunk's last row so that all of them are in flight together
    // (the optional b and w under uniform branches of their own)
    using TO = typename Entry<R>::TO;
    R e[PER];
    int64_t ii[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int p = u * kPlanThreads + threadIdx.x;
      ii[u] = r0 + (p < m ? p : m - 1);
      e[u] = Entry<R>::extent(src, ii[u]);
    }
    if (Entry<R>::kSb && src.b != nullptr) {
      TO bv[PER], sc[PER];
      if (src.b_f64) {
#pragma unroll
        for (int u = 0; u < PER; ++u) bv[u] = static_cast<TO>(static_cast<const double*>(src.b)[ii[u]]);
      } else {
#pragma unroll
        for (int u = 0; u < PER; ++u) bv[u] = static_cast<TO>(static_cast<const float*>(src.b)[ii[u]]);
      }
      if (src.w != nullptr) {
#pragma unroll
        for (int u = 0; u < PER; ++u) sc[u] = static_cast<TO>(src.w[ii[u]]);
      } else {
#pragma unroll
        for (int u = 0; u < PER; ++u)
          sc[u] = negative_of(hk_z(seed, static_cast<uint64_t>(ii[u]))) ? TO(-1) : TO(1);
      }
#pragma unroll
      for (int u = 0; u < PER; ++u) Entry<R>::set_sb(e[u], sc[u] * bv[u]);
    }
#pragma unroll
    for (int u = 0; u < PER; ++u)
      if (u * kPlanThreads + static_cast<int>(threadIdx.x) < m) stage[atomicAdd(&cnt[bin[u]], 1)] = e[u];
  }
  __syncthreads();
  for (int k = threadIdx.x; k < m; k += kPlanThreads) out[r0 + k] = stage[k];
}

// Blocks are dispatched to the eight XCDs of the chip in turn; this maps the
// dispatch index to a work index so that each XCD takes one contiguous range
// of the work (neighbouring bins then share their L2 lines: segment tables,
// rows of S A).
__device__ __forceinline__ int xcd_major(int g, int G) {
  constexpr int kXcd = 8;
  if (G % kXcd != 0) return g;
  return (g % kXcd) * (G / kXcd) + g / kXcd;
}

// ---------------------------------------------------------------- bin segments
// Where a coarse bin's plan entries are: one contiguous range (two-level
// plan) or one range per chunk (one-pass local plan).
struct BinSegs {
  const int32_t* off;  // coarse offsets [C * nblk + 1] or local offsets [nseg x (C + 1)]
  int nseg;            // chunks (local) or row chunks of the coarse passes
  int local;
  int chunk;           // rows per chunk of the local plan
  int C;
  int64_t n;
};

constexpr int kMaxSeg = 1024;  // chunks a local plan may have (LDS table of the reduce)
constexpr int kMapCap = 2048;  // entries of a bin mapped at once

// LDS of a binned block besides the rows of S A: the bin's segment starts and
// prefix lengths, and the map from the bin's row index to its plan entry.
struct SegLds {
  int32_t start[kMaxSeg];
  int32_t pfx[kMaxSeg + 1];
  int32_t map[kMapCap];
};

// Fill L.start / L.pfx for bin c and return the bin's row count.
__device__ __forceinline__ int32_t load_segments(const BinSegs& S, int c, SegLds& L, int32_t* wsum) {
  const int ns = S.local ? S.nseg : 1;
  const int per = (ns + static_cast<int>(blockDim.x) - 1) / static_cast<int>(blockDim.x);
  const int q0 = threadIdx.x * per;
  int32_t len[4];  // ns <= kMaxSeg and blockDim.x >= 256: at most 4 per thread
  int32_t run = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int q = q0 + k;
    len[k] = 0;
    if (k < per && q < ns) {
      int64_t st, en;
      if (S.local) {
        const int32_t* o = S.off + static_cast<size_t>(q) * (S.C + 1) + c;
        st = static_cast<int64_t>(q) * S.chunk + o[0];
        en = static_cast<int64_t>(q) * S.chunk + o[1];
      } else {
        st = S.off[static_cast<size_t>(c) * S.nseg];
        en = (c + 1 < S.C) ? S.off[static_cast<size_t>(c + 1) * S.nseg] : S.n;
      }
      L.start[q] = static_cast<int32_t>(st);
      len[k] = static_cast<int32_t>(en - st);
      run += len[k];
    }
  }
  int32_t tot;
  int32_t pre = block_exclusive_scan(run, wsum, &tot);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int q = q0 + k;
    if (k < per && q < ns) {
      L.pfx[q] = pre;
      pre += len[k];
    }
  }
  if (threadIdx.x == 0) L.pfx[ns] = tot;
  __syncthreads();
  return tot;
}

// L.map[k] = plan entry of the bin's row p0 + k, for p0 + k < pe: one
// thread per segment writes the segment's part of [p0, pe), or, for a single
// segment, one thread per row.
__device__ __forceinline__ void map_rows(const BinSegs& S, SegLds& L, int32_t p0, int32_t pe) {
  if (!S.local) {
    for (int32_t k = threadIdx.x; k < pe - p0; k += blockDim.x) L.map[k] = L.start[0] + p0 + k;
    return;
  }
  for (int q = threadIdx.x; q < S.nseg; q += blockDim.x) {
    const int32_t lo = L.pfx[q] > p0 ? L.pfx[q] : p0;
    const int32_t hi = L.pfx[q + 1] < pe ? L.pfx[q + 1] : pe;
    for (int32_t j = lo; j < hi; ++j) L.map[j - p0] = L.start[q] + (j - L.pfx[q]);
  }
}

// ---------------------------------------------------------------- CSR row gather
// A wavefront reduces up to 128 CSR rows at a time (two per lane: rows lane
// and lane + 64 of the chunk) into an LDS accumulator.  Wave-wide scans of
// the row lengths give each row its offset in the chunk's flat list of
// nonzeros; a byte table in LDS maps every position of that list to its row
// (a binary search over the offsets when the table does not fit), and the
// column/value loads of 64 * K positions are issued back to back before their
// products are added into the accumulator.  When every row of the chunk
// starts and ends on a multiple of four nonzeros (and the arrays are 16-byte
// aligned), positions are groups of four: one 16-byte load of column indices
// and one of values per lane.
constexpr int kChunkRows = 2 * kWave;
constexpr int kPosCap = 1024;
constexpr int kBurst = 16;
constexpr int kBurstQ = 8;

template <typename TR, typename TO>
struct alignas(16) RowRef {
  TR base;      // row start minus its offset in the flat list
  int32_t off;  // row of the accumulator (element offset)
  TO scale;     // sign or learned value of the row
};

template <typename TR, typename TO>
struct GatherLds {
  RowRef<TR, TO> ref[kChunkRows];
  int32_t pfx[kChunkRows];
  uint8_t pos2row[kPosCap];
};

// Inclusive prefix sum over the 64 lanes with DPP row shifts and row
// broadcasts (no LDS round trips).
__device__ __forceinline__ int32_t wave_incl_scan(int32_t x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
  return x;
}

// Column indices and values of E consecutive nonzeros.
template <typename TV, typename TO, int E>
struct Group {
  __device__ __forceinline__ static void load(const int32_t* __restrict__ c, const TV* __restrict__ v,
                                              int32_t (&ci)[E], TO (&vo)[E]) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      ci[e] = c[e];
      vo[e] = load_as<TO>(v, e);
    }
  }
};
template <typename TV, typename TO>
struct Group<TV, TO, 4> {
  __device__ __forceinline__ static void load(const int32_t* __restrict__ c, const TV* __restrict__ v,
                                              int32_t (&ci)[4], TO (&vo)[4]) {
    const int4 x = *reinterpret_cast<const int4*>(c);
    ci[0] = x.x;
    ci[1] = x.y;
    ci[2] = x.z;
    ci[3] = x.w;
    if constexpr (std::is_same<TV, float>::value) {
      const float4 y = *reinterpret_cast<const float4*>(v);
      vo[0] = y.x;
      vo[1] = y.y;
      vo[2] = y.z;
      vo[3] = y.w;
    } else if constexpr (std::is_same<TV, double>::value) {
      const double2 y0 = *reinterpret_cast<const double2*>(v);
      const double2 y1 = *reinterpret_cast<const double2*>(v + 2);
      vo[0] = static_cast<TO>(y0.x);
      vo[1] = static_cast<TO>(y0.y);
      vo[2] = static_cast<TO>(y1.x);
      vo[3] = static_cast<TO>(y1.y);
    } else {
      const uint2 y = *reinterpret_cast<const uint2*>(v);
      vo[0] = bf16_lo(y.x);
      vo[1] = bf16_hi(y.x);
      vo[2] = bf16_lo(y.y);
      vo[3] = bf16_hi(y.y);
    }
  }
};

template <bool TABLE, typename TR, typename TO>
__device__ __forceinline__ int row_at(const GatherLds<TR, TO>& G, int pp) {
  if (TABLE) return G.pos2row[pp];
  int q = 0;  // largest q with pfx[q] <= pp (empty rows share the next offset)
#pragma unroll
  for (int step = kChunkRows / 2; step > 0; step >>= 1)
    if (G.pfx[q + step] <= pp) q += step;
  return q;
}

// One burst: positions p0 + u * 64 + lane.  Positions past the end repeat
// position 0 (valid whenever total > 0) so that every load of the burst is
// unconditional and in flight together, and add nothing.
template <typename TV, typename TR, typename TO, bool TABLE, int E>
__device__ __forceinline__ void gather_burst(const GatherLds<TR, TO>& G, const int32_t* __restrict__ col,
                                             const TV* __restrict__ val, TO* acc, int p0, int total,
                                             int lane) {
  constexpr int K = E == 4 ? kBurstQ : kBurst;
  int pp[K], q[K];
  bool ok[K];
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const int p = p0 + u * kWave + lane;
    ok[u] = p < total;
    pp[u] = ok[u] ? p : 0;
  }
#pragma unroll
  for (int u = 0; u < K; ++u) q[u] = row_at<TABLE>(G, pp[u]);
  RowRef<TR, TO> ref[K];
#pragma unroll
  for (int u = 0; u < K; ++u) ref[u] = G.ref[q[u]];
  int32_t c[K][E];
  TO v[K][E];
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const TR k = ref[u].base + static_cast<TR>(E * pp[u]);
    Group<TV, TO, E>::load(col + k, val + k, c[u], v[u]);
  }
  // adds in groups of eight elements
  constexpr int NG = E * K >= 8 ? 8 : E * K;
  static_assert((E * K) % NG == 0, "group size");
#pragma unroll
  for (int g0 = 0; g0 < E * K; g0 += NG) {
    int32_t a[NG];
    TO x[NG];
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < NG; ++k) {
      const int u = (g0 + k) / E, e = (g0 + k) % E;
      a[k] = ref[u].off + c[u][e];
      x[k] = ref[u].scale * v[u][e];
      m |= ok[u] ? (1u << k) : 0u;
    }
    lds_add<TO, NG>(acc, a, x, m);
  }
}

// This lane's two rows of the chunk: start, length (0: no row), scale and
// accumulator row.
template <typename TR, typename TO>
struct RowPair {
  TR st[2];
  int32_t len[2];
  TO sc[2];
  int32_t off[2];
};

// Reduce the chunk's rows into acc.
template <typename TV, typename TR, typename TO>
__device__ __forceinline__ void gather_chunk(GatherLds<TR, TO>& G, const RowPair<TR, TO>& R, int quad_ok,
                                             const int32_t* __restrict__ col, const TV* __restrict__ val, TO* acc,
                                             int lane) {
  const bool quad = quad_ok && __all((((static_cast<int64_t>(R.st[0]) | R.len[0]) & 3) == 0) &&
                                     (((static_cast<int64_t>(R.st[1]) | R.len[1]) & 3) == 0));
  const int32_t u0 = quad ? (R.len[0] >> 2) : R.len[0];
  const int32_t u1 = quad ? (R.len[1] >> 2) : R.len[1];
  const int32_t i0 = wave_incl_scan(u0), i1 = wave_incl_scan(u1);
  const int32_t t0 = __builtin_amdgcn_readlane(i0, kWave - 1);
  const int32_t total = t0 + __builtin_amdgcn_readlane(i1, kWave - 1);
  if (total == 0) return;
  const int32_t pf0 = i0 - u0, pf1 = t0 + i1 - u1;
  const int E = quad ? 4 : 1;
  RowRef<TR, TO> r0, r1;
  r0.base = R.st[0] - static_cast<TR>(E * pf0);
  r0.off = R.off[0];
  r0.scale = R.sc[0];
  r1.base = R.st[1] - static_cast<TR>(E * pf1);
  r1.off = R.off[1];
  r1.scale = R.sc[1];
  G.ref[lane] = r0;
  G.ref[lane + kWave] = r1;
  G.pfx[lane] = pf0;
  G.pfx[lane + kWave] = pf1;
  const bool table = total <= kPosCap && !__any(u0 > kWave || u1 > kWave);
  if (table)
    for (int e = 0; __any(e < u0 || e < u1); ++e) {
      if (e < u0) G.pos2row[pf0 + e] = static_cast<uint8_t>(lane);
      if (e < u1) G.pos2row[pf1 + e] = static_cast<uint8_t>(lane + kWave);
    }
  wave_sync();
  if (quad) {
    if (table) {
      for (int p0 = 0; p0 < total; p0 += kWave * kBurstQ)
        gather_burst<TV, TR, TO, true, 4>(G, col, val, acc, p0, total, lane);
    } else {
      for (int p0 = 0; p0 < total; p0 += kWave * kBurstQ)
        gather_burst<TV, TR, TO, false, 4>(G, col, val, acc, p0, total, lane);
    }
  } else if (table) {
    for (int p0 = 0; p0 < total; p0 += kWave * kBurst)
      gather_burst<TV, TR, TO, true, 1>(G, col, val, acc, p0, total, lane);
  } else {
    for (int p0 = 0; p0 < total; p0 += kWave * kBurst)
      gather_burst<TV, TR, TO, false, 1>(G, col, val, acc, p0, total, lane);
  }
  wave_sync();
}

// ---------------------------------------------------------------- a2: CSR, binned
// LDS-privatised scatter-add.  One block per (coarse bin, split) holds the
// bin's 2^sh rows of S A in LDS, its waves stream the bin's plan records in
// coarse order (128 rows per wave step) and add every product into the LDS
// copy with LDS atomics; the block then writes the rows once (one split) or
// adds them into S A with global atomics (several splits of a crowded bin,
// S A zeroed first).  The order of the additions is not fixed, so float
// results are not bit-reproducible (integer-valued inputs are exact).
constexpr int kBinThreads = 512;
constexpr int kBinWaves = kBinThreads / kWave;

template <typename TR, typename TO>
__device__ __forceinline__ CsrRec<TR, TO> load_rec(const CsrRec<TR, TO>* __restrict__ recs, int64_t j, bool has) {
  CsrRec<TR, TO> e;
  if (has) {
    e = recs[j];
  } else {
    e.start = TR(0);
    e.len = 0;
    e.row = 0;
    e.sbv = TO(0);
  }
  return e;
}

template <typename TV, typename TR, typename TO>
__global__ __launch_bounds__(kBinThreads) void k_sketch_csr_binned(
    int d, uint32_t t, int sh, int splits, HashKey seed, const int32_t* __restrict__ col,
    const TV* __restrict__ val, const float* __restrict__ w, BinSegs S, const CsrRec<TR, TO>* __restrict__ recs,
    TO* __restrict__ SA, TO* __restrict__ Sb, const void* __restrict__ bg, int bg_f64, int acc_bytes, int sb_bytes,
    int quad_ok) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t wsum[kBinWaves];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int gb = xcd_major(blockIdx.x, gridDim.x);
  const int c = gb / splits, sp = gb % splits;
  const uint32_t bk0 = static_cast<uint32_t>(c) << sh;
  const int fine = 1 << sh;
  const int nbk = (t - bk0) < static_cast<uint32_t>(fine) ? static_cast<int>(t - bk0) : fine;
  TO* acc = reinterpret_cast<TO*>(smem);
  TO* sbacc = reinterpret_cast<TO*>(smem + acc_bytes);
  SegLds& L = *reinterpret_cast<SegLds*>(smem + acc_bytes + sb_bytes);
  GatherLds<TR, TO>& G = *reinterpret_cast<GatherLds<TR, TO>*>(smem + acc_bytes + sb_bytes + sizeof(SegLds) +
                                                              wid * sizeof(GatherLds<TR, TO>));
  const int nacc = nbk * d;
  for (int e = threadIdx.x; e < nacc; e += kBinThreads) acc[e] = TO(0);
  for (int e = threadIdx.x; e < nbk; e += kBinThreads) sbacc[e] = TO(0);
  const int32_t total = load_segments(S, c, L, wsum);
  const int32_t beg = static_cast<int32_t>(static_cast<int64_t>(total) * sp / splits);
  const int32_t end = static_cast<int32_t>(static_cast<int64_t>(total) * (sp + 1) / splits);
  constexpr int32_t kStep = kBinWaves * kChunkRows;
  for (int32_t p0 = beg; p0 < end; p0 += kMapCap) {
    const int32_t pe = end - p0 < kMapCap ? end : p0 + kMapCap;
    map_rows(S, L, p0, pe);
    __syncthreads();
    // Record loads are unconditional: rows past the end read the piece's last
    // record (and count as empty), so no load sits behind a branch whose join
    // makes the compiler wait for it.
    auto rec_at = [&](int32_t j) -> CsrRec<TR, TO> { return recs[L.map[(j < pe ? j : pe - 1) - p0]]; };
    int32_t j0 = p0 + wid * kChunkRows;
    CsrRec<TR, TO> cur[2];
    if (j0 < pe) {
#pragma unroll
      for (int h = 0; h < 2; ++h) cur[h] = rec_at(j0 + h * kWave + lane);
    }
    for (; j0 < pe; j0 += kStep) {
      RowPair<TR, TO> R;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const bool has = j0 + h * kWave + lane < pe;
        const uint64_t z = hk_z(seed, static_cast<uint64_t>(cur[h].row));
        const int lb = static_cast<int>(hk_bucket(seed, z, static_cast<uint64_t>(cur[h].row), t) - bk0);
        R.st[h] = cur[h].start;
        R.len[h] = has ? cur[h].len : 0;
        R.sc[h] = w ? static_cast<TO>(w[cur[h].row]) : (negative_of(z) ? TO(-1) : TO(1));
        R.off[h] = lb * d;
        if (Sb != nullptr && has)
          lds_add1(sbacc, lb, bg ? R.sc[h] * load_b<TO>(bg, bg_f64, cur[h].row) : cur[h].sbv);
      }
      // next step's records are requested after this step's rows are set up
      // (so no wait there covers them) and before this step's gathers
      CsrRec<TR, TO> nxt[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) nxt[h] = rec_at(j0 + kStep + h * kWave + lane);
      gather_chunk<TV, TR, TO>(G, R, quad_ok, col, val, acc, lane);
      cur[0] = nxt[0];
      cur[1] = nxt[1];
    }
    __syncthreads();
  }
  TO* out = SA + static_cast<size_t>(bk0) * d;
  if (splits == 1) {
    for (int e = threadIdx.x; e < nacc; e += kBinThreads) out[e] = acc[e];
    if (Sb != nullptr)
      for (int e = threadIdx.x; e < nbk; e += kBinThreads) Sb[bk0 + e] = sbacc[e];
  } else {
    for (int e = threadIdx.x; e < nacc; e += kBinThreads) unsafeAtomicAdd(out + e, acc[e]);
    if (Sb != nullptr)
      for (int e = threadIdx.x; e < nbk; e += kBinThreads) unsafeAtomicAdd(Sb + bk0 + e, sbacc[e]);
  }
}

// ---------------------------------------------------------------- a2: CSR, sorted
// One wavefront reduces one bucket at a time from the plan's records in
// bucket order: it sorts the bucket's rows by row id (up to kCsrSortCap rows,
// two per lane), gathers them 128 at a time into its LDS row of S A and writes
// that row once.  Row order is fixed, so results are bit-reproducible for
// buckets of up to kCsrSortCap rows.
constexpr int kCsrSortCap = 2 * kWave;

template <typename TR, typename TO>
struct CsrLds {
  TO dscale[kCsrSortCap];
  TO dsbv[kCsrSortCap];
  TR dstart[kCsrSortCap];
  int32_t dlen[kCsrSortCap];
  GatherLds<TR, TO> g;
};

template <typename TR, typename TO>
struct CsrMeta {
  int beg, m;
  CsrRec<TR, TO> a, b;  // rows lane and lane + 64 of the bucket (row INT_MAX: none)
};

template <typename TR, typename TO>
__device__ __forceinline__ CsrMeta<TR, TO> csr_meta(const CsrRec<TR, TO>* __restrict__ recs, int beg, int m,
                                                    int lane) {
  CsrMeta<TR, TO> q;
  q.beg = beg;
  q.m = m;
  const bool h0 = lane < m && m <= kCsrSortCap, h1 = lane + kWave < m && m <= kCsrSortCap;
  q.a = load_rec(recs, beg + lane, h0);
  q.b = load_rec(recs, beg + kWave + lane, h1);
  if (!h0) q.a.row = INT_MAX;
  if (!h1) q.b.row = INT_MAX;
  return q;
}

// Each wavefront owns `bpw` consecutive buckets and walks them in order,
// loading the next bucket's records while it reduces the current one.
template <typename TV, typename TR, typename TO>
__global__ __launch_bounds__(kThreads) void k_sketch_csr_sorted(
    int d, uint32_t t, int bpw, HashKey seed, const int32_t* __restrict__ col, const TV* __restrict__ val,
    const float* __restrict__ w, const int32_t* __restrict__ off, const CsrRec<TR, TO>* __restrict__ recs,
    TO* __restrict__ SA, TO* __restrict__ Sb, const void* __restrict__ bg, int bg_f64, int per_wave, int quad_ok) {
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
  CsrMeta<TR, TO> cur = csr_meta<TR, TO>(recs, off_at(0), off_at(1) - off_at(0), lane);
  for (int kb = 0; kb < nb; ++kb) {
    const uint32_t bkt = static_cast<uint32_t>(b0 + kb);
    CsrMeta<TR, TO> nxt = cur;
    if (kb + 1 < nb) {
      const int nbeg = off_at(kb + 1);
      nxt = csr_meta<TR, TO>(recs, nbeg, off_at(kb + 2) - nbeg, lane);
    }
    for (int k = lane; k < d; k += kWave) acc[k] = TO(0);
    const int beg = cur.beg, m = cur.m;
    const bool sorted = m <= kCsrSortCap;
    if (sorted) {
      const int32_t r0 = cur.a.row, r1 = cur.b.row;
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
        L.dstart[rk0] = cur.a.start;
        L.dlen[rk0] = cur.a.len;
        L.dscale[rk0] = row_scale<TO>(seed, r0, w);
        L.dsbv[rk0] = bg ? L.dscale[rk0] * load_b<TO>(bg, bg_f64, r0) : cur.a.sbv;
      }
      if (lane + kWave < m) {
        L.dstart[rk1] = cur.b.start;
        L.dlen[rk1] = cur.b.len;
        L.dscale[rk1] = row_scale<TO>(seed, r1, w);
        L.dsbv[rk1] = bg ? L.dscale[rk1] * load_b<TO>(bg, bg_f64, r1) : cur.b.sbv;
      }
    }
    wave_sync();
    TO sb = TO(0);
    for (int j0 = 0; j0 < m; j0 += kChunkRows) {
      RowPair<TR, TO> R;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int j = j0 + h * kWave + lane;
        R.st[h] = TR(0);
        R.len[h] = 0;
        R.sc[h] = TO(0);
        R.off[h] = 0;
        if (j < m) {
          if (sorted) {
            R.st[h] = L.dstart[j];
            R.len[h] = L.dlen[j];
            R.sc[h] = L.dscale[j];
            sb += L.dsbv[j];
          } else {
            const CsrRec<TR, TO> e = recs[beg + j];
            R.st[h] = e.start;
            R.len[h] = e.len;
            R.sc[h] = row_scale<TO>(seed, e.row, w);
            sb += bg ? R.sc[h] * load_b<TO>(bg, bg_f64, e.row) : e.sbv;
          }
        }
      }
      gather_chunk<TV, TR, TO>(L.g, R, quad_ok, col, val, acc, lane);
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
    const nt_f4 x = stream_load<nt_f4>(p);
    out[0] = x[0];
    out[1] = x[1];
    out[2] = x[2];
    out[3] = x[3];
  }
};
template <typename TO>
struct RowLoad<double, TO, 2> {
  __device__ __forceinline__ static void load(const double* __restrict__ p, TO (&out)[2]) {
    const nt_d2 x = stream_load<nt_d2>(p);
    out[0] = static_cast<TO>(x[0]);
    out[1] = static_cast<TO>(x[1]);
  }
};
template <typename TO>
struct RowLoad<bf16_t, TO, 8> {
  __device__ __forceinline__ static void load(const bf16_t* __restrict__ p, TO (&out)[8]) {
    const nt_u4 x = stream_load<nt_u4>(p);
    out[0] = bf16_lo(x[0]);
    out[1] = bf16_hi(x[0]);
    out[2] = bf16_lo(x[1]);
    out[3] = bf16_hi(x[1]);
    out[4] = bf16_lo(x[2]);
    out[5] = bf16_hi(x[2]);
    out[6] = bf16_lo(x[3]);
    out[7] = bf16_hi(x[3]);
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

// Sum of the bucket's rows for this lane's column slices.  A row takes
// ceil(d / V) lanes; when that is at most 16 (32) the wave splits into 4 (2)
// groups of lanes, group g taking rows g, g + 4 (g + 2), ... of the bucket,
// and the groups' sums meet by lane exchanges at the end, so that narrow rows
// do not leave most of the wave idle.  Batches of RB rows per group are loaded
// unconditionally (rows past the end repeat row 0 and are skipped when
// summing), so all loads of a batch are in flight together.
template <typename TV, typename TO, int V, bool SORTED>
__device__ __forceinline__ void dense_rows(const DenseLds<TO>& L, const int32_t* __restrict__ perm, int beg, int m,
                                           HashKey seed, const float* __restrict__ w, const TV* __restrict__ A,
                                           int64_t ld, int d, TO* __restrict__ out, int lane) {
  constexpr int RB = 8;
  const int chunks = (d + V - 1) / V;
  const int LG = chunks <= 16 ? 16 : (chunks <= 32 ? 32 : kWave);  // lanes per group
  const int NG = kWave / LG, g = lane / LG, sub = lane % LG;
  for (int c0 = sub * V; c0 < d; c0 += LG * V) {
    TO acc[V];
#pragma unroll
    for (int k = 0; k < V; ++k) acc[k] = TO(0);
    for (int j = g; j < m; j += RB * NG) {
      TO sc[RB], x[RB][V];
      bool ok[RB];
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const int jq = j + q * NG;
        ok[q] = jq < m;
        const int jc = ok[q] ? jq : 0;
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
    // lanes of one column slice in the other groups hold the same trip
    // counts, so the exchanges run with every partner active
    for (int off = LG; off < kWave; off <<= 1)
#pragma unroll
      for (int k = 0; k < V; ++k) acc[k] += __shfl_xor(acc[k], off, kWave);
    if (g == 0)
#pragma unroll
      for (int k = 0; k < V; ++k) out[c0 + k] = acc[k];
  }
}

template <typename TV, typename TO, int V>
__device__ __forceinline__ void sketch_dense_sorted_body(int d, int64_t ld, uint32_t t, int bpw, HashKey seed,
                                                         const TV* __restrict__ A, const void* __restrict__ b,
                                                         int b_f64, const float* __restrict__ w,
                                                         const int32_t* __restrict__ off,
                                                         const int32_t* __restrict__ perm, TO* __restrict__ SA,
                                                         TO* __restrict__ Sb) {
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

template <typename TV, typename TO, int V>
__global__ __launch_bounds__(kThreads) void k_sketch_dense_sorted(
    int d, int64_t ld, uint32_t t, int bpw, HashKey seed, const TV* __restrict__ A, const void* __restrict__ b,
    int b_f64, const float* __restrict__ w, const int32_t* __restrict__ off, const int32_t* __restrict__ perm,
    TO* __restrict__ SA, TO* __restrict__ Sb) {
  sketch_dense_sorted_body<TV, TO, V>(d, ld, t, bpw, seed, A, b, b_f64, w, off, perm, SA, Sb);
}

// The same for up to kSortedMany dense float32 matrices of one shape sharing
// the plan (float32 output, no b): matrix blockIdx.y is args.A[y] (leading
// dimension args.ld[y]) and its sketch goes to SA + y * sa_stride.
struct SortedMany {
  const float* A[kSortedMany];
  int64_t ld[kSortedMany];
};

template <int V>
__global__ __launch_bounds__(kThreads) void k_sketch_dense_sorted_many(int d, uint32_t t, int bpw, HashKey seed,
                                                                       SortedMany args, const float* __restrict__ w,
                                                                       const int32_t* __restrict__ off,
                                                                       const int32_t* __restrict__ perm,
                                                                       float* __restrict__ SA, int64_t sa_stride) {
  const int y = blockIdx.y;
  sketch_dense_sorted_body<float, float, V>(d, args.ld[y], t, bpw, seed, args.A[y], nullptr, 0, w, off, perm,
                                            SA + static_cast<int64_t>(y) * sa_stride, nullptr);
}

// ---------------------------------------------------------------- a2: dense, binned
// The same LDS-privatised schedule for dense rows: each wave takes rows of
// the bin (RB at a time, all loads in flight together) and adds them, column
// slices per lane, into the bin's LDS rows of S A.
template <typename TV, typename TO, int V>
__global__ __launch_bounds__(kBinThreads) void k_sketch_dense_binned(
    int d, int64_t ld, uint32_t t, int sh, int splits, HashKey seed, const TV* __restrict__ A,
    const void* __restrict__ b, int b_f64, const float* __restrict__ w, BinSegs S,
    const int32_t* __restrict__ rows, TO* __restrict__ SA, TO* __restrict__ Sb, int acc_bytes, int sb_bytes) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t wsum[kBinWaves];
  constexpr int RB = 4;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int gb = xcd_major(blockIdx.x, gridDim.x);
  const int c = gb / splits, sp = gb % splits;
  const uint32_t bk0 = static_cast<uint32_t>(c) << sh;
  const int fine = 1 << sh;
  const int nbk = (t - bk0) < static_cast<uint32_t>(fine) ? static_cast<int>(t - bk0) : fine;
  TO* acc = reinterpret_cast<TO*>(smem);
  TO* sbacc = reinterpret_cast<TO*>(smem + acc_bytes);
  SegLds& L = *reinterpret_cast<SegLds*>(smem + acc_bytes + sb_bytes);
  const int nacc = nbk * d;
  for (int e = threadIdx.x; e < nacc; e += kBinThreads) acc[e] = TO(0);
  for (int e = threadIdx.x; e < nbk; e += kBinThreads) sbacc[e] = TO(0);
  const int32_t total = load_segments(S, c, L, wsum);
  const int32_t beg = static_cast<int32_t>(static_cast<int64_t>(total) * sp / splits);
  const int32_t end = static_cast<int32_t>(static_cast<int64_t>(total) * (sp + 1) / splits);
  for (int32_t p0 = beg; p0 < end; p0 += kMapCap) {
    const int32_t pe = end - p0 < kMapCap ? end : p0 + kMapCap;
    map_rows(S, L, p0, pe);
    __syncthreads();
    for (int32_t j0 = p0 + wid * RB; j0 < pe; j0 += kBinWaves * RB) {
      int32_t r[RB], o[RB];
      bool okq[RB];
      TO sc[RB];
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const bool ok = j0 + q < pe;
        r[q] = rows[L.map[(ok ? j0 + q : j0) - p0]];
        const uint64_t z = hk_z(seed, static_cast<uint64_t>(r[q]));
        const int lb = static_cast<int>(hk_bucket(seed, z, static_cast<uint64_t>(r[q]), t) - bk0);
        o[q] = lb * d;
        okq[q] = ok;
        sc[q] = w ? static_cast<TO>(w[r[q]]) : (negative_of(z) ? TO(-1) : TO(1));
        if (Sb != nullptr && ok && lane == 0) lds_add1(sbacc, lb, sc[q] * load_b<TO>(b, b_f64, r[q]));
      }
      for (int c0 = lane * V; c0 < d; c0 += kWave * V) {
        TO x[RB][V];
#pragma unroll
        for (int q = 0; q < RB; ++q) RowLoad<TV, TO, V>::load(A + static_cast<size_t>(r[q]) * ld + c0, x[q]);
#pragma unroll
        for (int q = 0; q < RB; ++q) {
          int32_t a[V];
          TO y[V];
#pragma unroll
          for (int k = 0; k < V; ++k) {
            a[k] = o[q] + c0 + k;
            y[k] = sc[q] * x[q][k];
          }
          lds_add<TO, V>(acc, a, y, okq[q] ? 0xffffffffu : 0u);
        }
      }
    }
    __syncthreads();
  }
  TO* out = SA + static_cast<size_t>(bk0) * d;
  if (splits == 1) {
    for (int e = threadIdx.x; e < nacc; e += kBinThreads) out[e] = acc[e];
    if (Sb != nullptr)
      for (int e = threadIdx.x; e < nbk; e += kBinThreads) Sb[bk0 + e] = sbacc[e];
  } else {
    for (int e = threadIdx.x; e < nacc; e += kBinThreads) unsafeAtomicAdd(out + e, acc[e]);
    if (Sb != nullptr)
      for (int e = threadIdx.x; e < nbk; e += kBinThreads) unsafeAtomicAdd(Sb + bk0 + e, sbacc[e]);
  }
}

// ---------------------------------------------------------------- a2: atomic
template <typename TV, typename TR, typename TO, int L>
__global__ __launch_bounds__(kThreads) void k_sketch_csr_atomic(
    int64_t n, int d, uint32_t t, HashKey seed, const TR* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const TV* __restrict__ val, const void* __restrict__ b, int b_f64, const float* __restrict__ w,
    TO* __restrict__ SA, TO* __restrict__ Sb) {
  const int64_t gid = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / L;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x / L;
  const int sub = threadIdx.x % L;
  for (int64_t r = gid; r < n; r += stride) {
    const uint64_t z = hk_z(seed, static_cast<uint64_t>(r));
    const uint32_t h = hk_bucket(seed, z, static_cast<uint64_t>(r), t);
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
    int64_t n, int d, int64_t ld, uint32_t t, HashKey seed, const TV* __restrict__ A, const void* __restrict__ b,
    int b_f64, const float* __restrict__ w, TO* __restrict__ SA, TO* __restrict__ Sb) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  for (int64_t r = wave; r < n; r += nwaves) {
    const uint64_t z = hk_z(seed, static_cast<uint64_t>(r));
    const uint32_t h = hk_bucket(seed, z, static_cast<uint64_t>(r), t);
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
int32_t launch_hash_key(int64_t n, uint32_t t, HashKey seed, int64_t start, int32_t* bucket, int8_t* sign,
                        hipStream_t s) {
  if (n == 0) return SKLS_OK;
  hipLaunchKernelGGL(k_hash, dim3(grid_for(n, kThreads, 16384)), dim3(kThreads), 0, s, n, t, seed, start, bucket,
                     sign);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t launch_hash(int64_t n, uint32_t t, uint64_t seed, int64_t start, int32_t* bucket, int8_t* sign,
                    hipStream_t s) {
  return launch_hash_key(n, t, plain_key(seed), start, bucket, sign, s);
}

int32_t launch_scale(void* p, size_t count, int32_t dtype, double alpha, hipStream_t s) {
  if (count == 0) return SKLS_OK;
  const unsigned g = grid_for(static_cast<int64_t>(count), kThreads, 8192);
  if (dtype == SKLS_F64)
    hipLaunchKernelGGL(k_scale<double>, dim3(g), dim3(kThreads), 0, s, static_cast<double*>(p), count, alpha);
  else
    hipLaunchKernelGGL(k_scale<float>, dim3(g), dim3(kThreads), 0, s, static_cast<float*>(p), count,
                       static_cast<float>(alpha));
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

namespace {

constexpr size_t kBinAcc = 32768;  // LDS bytes of S A rows held by one binned block

size_t round16(size_t x) { return (x + 15) / 16 * 16; }

// Shape of the bucket plan for one input, variant and output precision.
struct PlanShape {
  int32_t variant = SKLS_SKETCH_SORTED;
  int sh = 0;         // log2 of buckets per coarse bin
  int C = 0;          // coarse bins; 0 selects one global counting pass (sorted only)
  int nblk = 1;       // row chunks of the coarse passes
  size_t entry = 4;   // bytes per plan entry (row index or CSR record)
  int splits = 1;     // binned: blocks sharing one bin
  int local = 0;      // binned: one-pass plan by chunks of `per` * kPlanThreads rows
  int per = 0;        // rows per thread of the one-pass plan (4, 8 or 16)
  int nseg = 0;       // chunks of the one-pass plan
};

size_t entry_bytes(const skls_matrix& A, int out_bytes) {
  if (A.layout != SKLS_CSR) return sizeof(int32_t);
  return (!A.row_ptr_64 && out_bytes == 4) ? 16 : 24;
}

// Buckets per binned block: the largest power of two whose rows of S A fit
// kBinAcc bytes (at most 4096, and no more than t needs); 0 if one row does
// not fit.
int64_t binned_fine(const skls_matrix& A, int64_t t, int out_bytes) {
  const int64_t row = A.d * out_bytes;
  // LDS left for the rows of S A next to the per-wave gather tables (CSR)
  // and the bin's share of S b, within the 160 KiB of a compute unit
  int64_t budget = static_cast<int64_t>(kBinAcc);
  int64_t tables = static_cast<int64_t>(sizeof(SegLds));
  if (A.layout == SKLS_CSR) {
    const int64_t ref = (A.row_ptr_64 && out_bytes == 8) ? 32 : 16;
    tables += kBinWaves * (kChunkRows * (ref + 4) + kPosCap);
  }
  const int64_t left = 160 * 1024 - tables - 4096 * out_bytes;
  budget = left < budget ? left : budget;
  if (row > budget) return 0;
  int64_t fine = 1;
  while (fine < 4096 && fine < t && 2 * fine * row <= budget) fine *= 2;
  return fine;
}

bool binned_ok(const skls_matrix& A, int64_t t, int out_bytes) {
  const int64_t fine = binned_fine(A, t, out_bytes);
  return fine > 0 && div_up(t, fine) <= kMaxBins;
}

bool sorted_ok(const skls_matrix& A, int out_bytes) {
  return A.layout != SKLS_CSR || A.d * out_bytes <= kAccMax;
}

int32_t pick_variant(const skls_matrix& A, int64_t t, int32_t variant, int out_bytes) {
  if (variant != SKLS_SKETCH_AUTO) return variant;
  if (A.layout == SKLS_CSR) {
    // LDS-privatised accumulation when the bin rows fit in LDS
    if (binned_ok(A, t, out_bytes)) return SKLS_SKETCH_BINNED;
    if (A.n <= 256 * t && sorted_ok(A, out_bytes)) return SKLS_SKETCH_SORTED;
    return SKLS_SKETCH_ATOMIC;
  }
  // dense rows: one wavefront per bucket sums whole rows in registers
  if (A.n > 256 * t) return binned_ok(A, t, out_bytes) ? SKLS_SKETCH_BINNED : SKLS_SKETCH_ATOMIC;
  return SKLS_SKETCH_SORTED;
}

// LDS of the one-pass plan kernel: the chunk's entries and the bin counters.
size_t local_lds(int per, size_t entry, int C) {
  return entry * static_cast<size_t>(per) * kPlanThreads + static_cast<size_t>(C + 1) * sizeof(int32_t) + 256;
}

PlanShape plan_shape(const skls_matrix& A, int64_t t, int32_t v, int out_bytes) {
  PlanShape S;
  const int64_t n = A.n;
  S.variant = v;
  S.entry = entry_bytes(A, out_bytes);
  S.nblk = static_cast<int>(div_up(n > 0 ? n : 1, kPlanChunk));
  if (v == SKLS_SKETCH_BINNED) {
    const int64_t fine = binned_fine(A, t, out_bytes);
    while ((int64_t(1) << S.sh) < fine) ++S.sh;
    S.C = static_cast<int>(div_up(t, fine));
    // spread crowded bins over several blocks: about 1024 blocks in all,
    // each with at least 2048 rows
    const int64_t want = div_up(1024, S.C), rows = n / (static_cast<int64_t>(S.C) * 2048);
    int64_t sp = want < rows ? want : rows;
    S.splits = static_cast<int>(sp < 1 ? 1 : (sp > 64 ? 64 : sp));
    // one-pass plan: the largest chunk whose LDS copy and counters fit, used
    // while the per-bin segment table fits the reduce's LDS
    S.per = 16;
    while (S.per > 4 && local_lds(S.per, S.entry, S.C) > 160 * 1024) S.per >>= 1;
    S.nseg = static_cast<int>(div_up(n > 0 ? n : 1, static_cast<int64_t>(S.per) * kPlanThreads));
    S.local = (S.nseg <= kMaxSeg && local_lds(S.per, S.entry, S.C) <= 160 * 1024) ? 1 : 0;
    return S;
  }
  // bucket order: coarse bins of about 4096 rows for the fine pass
  int sh = 0;
  while (sh < 12 && (n << (sh + 1)) <= int64_t(4096) * t) ++sh;
  const int64_t C = (t + (int64_t(1) << sh) - 1) >> sh;
  S.sh = sh;
  S.C = C <= kMaxBins ? static_cast<int>(C) : 0;
  return S;
}

// Workspace of the plan: bin or bucket counts, scan partials, entries in
// coarse-bin order, and (bucket order) entries by bucket and bucket offsets.
struct BucketPlan {
  PlanShape S;
  int32_t* count = nullptr;  // [C * nblk + 1] (two-level) or [t + 1] (global)
  int32_t* bsum = nullptr;
  int32_t* rank = nullptr;   // [n] global counting only
  void* coarse = nullptr;    // [n] entries in coarse-bin order (two-level)
  void* fine = nullptr;      // [n] entries in bucket order (sorted)
  int32_t* off = nullptr;    // [t + 1] bucket offsets (sorted)
  int32_t* offT = nullptr;   // [nseg x (C + 1)] per-chunk bin offsets (one-pass plan)
};

BucketPlan carve_plan(Arena& ar, const PlanShape& S, int64_t n, int64_t t) {
  BucketPlan P;
  P.S = S;
  if (S.local) {
    P.offT = ar.take<int32_t>(static_cast<size_t>(S.C + 1) * S.nseg);
    P.coarse = ar.take<char>(static_cast<size_t>(n) * S.entry);
    return P;
  }
  const int64_t ncnt = S.C ? static_cast<int64_t>(S.C) * S.nblk : t;
  P.count = ar.take<int32_t>(static_cast<size_t>(ncnt) + 1);
  P.bsum = ar.take<int32_t>(static_cast<size_t>(div_up(ncnt, kScanTile)) + 1);
  if (S.C) {
    P.coarse = ar.take<char>(static_cast<size_t>(n) * S.entry);
  } else {
    P.rank = ar.take<int32_t>(static_cast<size_t>(n));
  }
  if (S.variant == SKLS_SKETCH_SORTED) {
    P.fine = ar.take<char>(static_cast<size_t>(n) * S.entry);
    P.off = ar.take<int32_t>(static_cast<size_t>(t) + 1);
  }
  return P;
}

size_t plan_bytes(const PlanShape& S, int64_t n, int64_t t) {
  Arena ar(nullptr, 0);
  carve_plan(ar, S, n, t);
  return ar.used;
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

int32_t allow_lds(const void* kernel, size_t lds);

template <typename R>
int32_t build_plan(int64_t n, uint32_t t, HashKey seed, const BucketPlan& P, const RowSrc& src, hipStream_t s) {
  const PlanShape& S = P.S;
  if (S.local) {
    const size_t lds = sizeof(R) * static_cast<size_t>(S.per) * kPlanThreads + static_cast<size_t>(S.C + 1) * 4;
    auto launch = [&](auto kern) -> int32_t {
      SKLS_TRY(allow_lds(reinterpret_cast<const void*>(kern), lds));
      hipLaunchKernelGGL(kern, dim3(S.nseg), dim3(kPlanThreads), lds, s, n, t, seed, S.sh, S.C, src,
                         static_cast<R*>(P.coarse), P.offT, S.nseg);
      SKLS_CHECK_LAUNCH();
      return SKLS_OK;
    };
    if (S.per == 16) return launch(&k_plan_local<R, 16>);
    if (S.per == 8) return launch(&k_plan_local<R, 8>);
    return launch(&k_plan_local<R, 4>);
  }
  if (S.C > 0) {
    const size_t lds = static_cast<size_t>(S.C) * sizeof(int32_t);
    const int64_t ncnt = static_cast<int64_t>(S.C) * S.nblk;
    hipLaunchKernelGGL(k_plan_coarse_count, dim3(S.nblk), dim3(kPlanThreads), lds, s, n, t, seed, S.sh, S.C, S.nblk,
                       P.count);
    SKLS_CHECK_LAUNCH();
    // the scanned (bin, block) offsets overwrite the counts in place (each
    // scan block reads its tile before writing it)
    SKLS_TRY(scan_counts(P.count, ncnt, P.bsum, P.count, s));
    hipLaunchKernelGGL((k_plan_coarse_scatter<R>), dim3(S.nblk), dim3(kPlanThreads), lds, s, n, t, seed, S.sh, S.C,
                       S.nblk, P.count, src, static_cast<R*>(P.coarse));
    SKLS_CHECK_LAUNCH();
    if (S.variant == SKLS_SKETCH_SORTED) {
      const size_t flds = (size_t(1) << S.sh) * sizeof(int32_t);
      hipLaunchKernelGGL((k_plan_fine<R>), dim3(S.C), dim3(kThreads), flds, s, n, t, seed, S.sh, S.C, S.nblk, P.count,
                         static_cast<const R*>(P.coarse), static_cast<R*>(P.fine), P.off);
      SKLS_CHECK_LAUNCH();
    }
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
    hipLaunchKernelGGL((k_scatter<R>), dim3(g), dim3(kThreads), 0, s, n, t, seed, P.off, P.rank, src,
                       static_cast<R*>(P.fine));
    SKLS_CHECK_LAUNCH();
  }
  return SKLS_OK;
}

// Wavefronts of a kBucketWaves-wave block kernel that the device holds at
// once (occupancy from registers and LDS), cached per kernel, LDS size and
// device.
int64_t resident_waves(const void* kernel, size_t lds) {
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

int buckets_per_wave(int64_t t, int64_t resident) {
  int64_t b = div_up(t, resident > 0 ? resident : 1);
  return static_cast<int>(b < 1 ? 1 : (b > 63 ? 63 : b));
}

int32_t allow_lds(const void* kernel, size_t lds) {
  if (lds > 65536) SKLS_TRY_HIP(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                    static_cast<int>(lds)));
  return SKLS_OK;
}

BinSegs bin_segs(const BucketPlan& P, int64_t n) {
  BinSegs g;
  g.off = P.S.local ? P.offT : P.count;
  g.nseg = P.S.local ? P.S.nseg : P.S.nblk;
  g.local = P.S.local;
  g.chunk = P.S.per * kPlanThreads;
  g.C = P.S.C;
  g.n = n;
  return g;
}

// Apply of the SORTED and BINNED variants once the plan is built.
// CSR records carry scale(row) * b[row] when the plan was built with b; a
// plan built without it (a reusable plan) takes b here instead (bg), and the
// reduce kernels gather b[row] for each record.
template <typename TO>
int32_t apply_planned(const skls_matrix& A, const BucketPlan& P, const void* b, int b_f64, uint32_t t, HashKey seed,
                      const float* w, TO* SA, TO* Sb, const void* bg, hipStream_t s) {
  const PlanShape& S = P.S;
  const int d = static_cast<int>(A.d);
  const int64_t n = A.n;
  return with_value(A.dtype, [&](auto tv) -> int32_t {
    using TV = decltype(tv);
    if (A.layout == SKLS_DENSE) {
      constexpr int VV = sizeof(TV) == 8 ? 2 : (sizeof(TV) == 4 ? 4 : 8);
      const bool vec = vec_ok<TV>(A.val, A.ld, A.d, VV);
      if (S.variant == SKLS_SKETCH_BINNED) {
        const int acc_bytes = static_cast<int>(round16((size_t(1) << S.sh) * d * sizeof(TO)));
        const int sb_bytes = static_cast<int>(round16((size_t(1) << S.sh) * sizeof(TO)));
        const size_t lds = acc_bytes + sb_bytes + sizeof(SegLds);
        const unsigned grid = static_cast<unsigned>(S.C) * S.splits;
        const int32_t* rows = static_cast<const int32_t*>(P.coarse);
        const BinSegs segs = bin_segs(P, n);
        if (vec) {
          SKLS_TRY(allow_lds(reinterpret_cast<const void*>(&k_sketch_dense_binned<TV, TO, VV>), lds));
          hipLaunchKernelGGL((k_sketch_dense_binned<TV, TO, VV>), dim3(grid), dim3(kBinThreads), lds, s, d, A.ld, t,
                             S.sh, S.splits, seed, static_cast<const TV*>(A.val), b, b_f64, w, segs, rows, SA, Sb,
                             acc_bytes, sb_bytes);
        } else {
          SKLS_TRY(allow_lds(reinterpret_cast<const void*>(&k_sketch_dense_binned<TV, TO, 1>), lds));
          hipLaunchKernelGGL((k_sketch_dense_binned<TV, TO, 1>), dim3(grid), dim3(kBinThreads), lds, s, d, A.ld, t,
                             S.sh, S.splits, seed, static_cast<const TV*>(A.val), b, b_f64, w, segs, rows, SA, Sb,
                             acc_bytes, sb_bytes);
        }
        SKLS_CHECK_LAUNCH();
        return SKLS_OK;
      }
      const size_t lds = kBucketWaves * sizeof(DenseLds<TO>);
      const void* kern = vec ? reinterpret_cast<const void*>(&k_sketch_dense_sorted<TV, TO, VV>)
                             : reinterpret_cast<const void*>(&k_sketch_dense_sorted<TV, TO, 1>);
      const int bpw = buckets_per_wave(t, resident_waves(kern, lds));
      const unsigned grid = static_cast<unsigned>(div_up(div_up(t, bpw), kBucketWaves));
      const int32_t* perm = static_cast<const int32_t*>(P.fine);
      if (vec) {
        hipLaunchKernelGGL((k_sketch_dense_sorted<TV, TO, VV>), dim3(grid), dim3(kThreads), lds, s, d, A.ld, t, bpw,
                           seed, static_cast<const TV*>(A.val), b, b_f64, w, P.off, perm, SA, Sb);
      } else {
        hipLaunchKernelGGL((k_sketch_dense_sorted<TV, TO, 1>), dim3(grid), dim3(kThreads), lds, s, d, A.ld, t, bpw,
                           seed, static_cast<const TV*>(A.val), b, b_f64, w, P.off, perm, SA, Sb);
      }
      SKLS_CHECK_LAUNCH();
      return SKLS_OK;
    }
    return with_rowptr(A, [&](auto tr) -> int32_t {
      using TR = decltype(tr);
      using Rec = CsrRec<TR, TO>;
      const int quad_ok = (reinterpret_cast<uintptr_t>(A.col_idx) % 16 == 0) &&
                          (reinterpret_cast<uintptr_t>(A.val) % (4 * sizeof(TV)) == 0);
      if (S.variant == SKLS_SKETCH_BINNED) {
        const int acc_bytes = static_cast<int>(round16((size_t(1) << S.sh) * d * sizeof(TO)));
        const int sb_bytes = static_cast<int>(round16((size_t(1) << S.sh) * sizeof(TO)));
        const size_t lds = acc_bytes + sb_bytes + sizeof(SegLds) + kBinWaves * sizeof(GatherLds<TR, TO>);
        const void* kern = reinterpret_cast<const void*>(&k_sketch_csr_binned<TV, TR, TO>);
        SKLS_TRY(allow_lds(kern, lds));
        hipLaunchKernelGGL((k_sketch_csr_binned<TV, TR, TO>), dim3(static_cast<unsigned>(S.C) * S.splits),
                           dim3(kBinThreads), lds, s, d, t, S.sh, S.splits, seed, A.col_idx,
                           static_cast<const TV*>(A.val), w, bin_segs(P, n), static_cast<const Rec*>(P.coarse), SA,
                           Sb, bg, b_f64, acc_bytes, sb_bytes, quad_ok);
        SKLS_CHECK_LAUNCH();
        return SKLS_OK;
      }
      // per wave: sort and gather tables and the bucket's row of S A
      const size_t row_bytes = static_cast<size_t>(d) * sizeof(TO);
      const int per_wave = static_cast<int>(round16(sizeof(CsrLds<TR, TO>) + row_bytes));
      const size_t lds = static_cast<size_t>(per_wave) * kBucketWaves;
      const void* kern = reinterpret_cast<const void*>(&k_sketch_csr_sorted<TV, TR, TO>);
      SKLS_TRY(allow_lds(kern, lds));
      // one round of resident wavefronts, each walking consecutive buckets
      const int bpw = buckets_per_wave(t, resident_waves(kern, lds));
      const unsigned grid = static_cast<unsigned>(div_up(div_up(t, bpw), kBucketWaves));
      hipLaunchKernelGGL((k_sketch_csr_sorted<TV, TR, TO>), dim3(grid), dim3(kThreads), lds, s, d, t, bpw, seed,
                         A.col_idx, static_cast<const TV*>(A.val), w, P.off, static_cast<const Rec*>(P.fine), SA,
                         Sb, bg, b_f64, per_wave, quad_ok);
      SKLS_CHECK_LAUNCH();
      return SKLS_OK;
    });
  });
}

int out_bytes_of(int32_t out_dtype) { return out_dtype == SKLS_F64 ? 8 : 4; }

}  // namespace

int32_t choose_sketch_variant(const skls_matrix& A, int64_t t, int32_t variant, int32_t out_dtype) {
  return pick_variant(A, t, variant, out_bytes_of(out_dtype));
}

// Workspace for either output precision (the query does not name one).
size_t sketch_ws_bytes(const skls_matrix& A, int64_t t, int32_t variant) {
  size_t need = 0;
  for (int ob : {4, 8}) {
    const int32_t v = pick_variant(A, t, variant, ob);
    if (v != SKLS_SKETCH_SORTED && v != SKLS_SKETCH_BINNED) continue;
    const size_t b = plan_bytes(plan_shape(A, t, v, ob), A.n, t);
    need = b > need ? b : need;
  }
  return need;
}

namespace {

int32_t check_variant(const skls_matrix& A, int64_t t, int32_t v, int ob, int32_t requested) {
  if (v != SKLS_SKETCH_ATOMIC && v != SKLS_SKETCH_SORTED && v != SKLS_SKETCH_BINNED) {
    set_error("unknown sketch variant %d", requested);
    return SKLS_ERR_ARG;
  }
  if (v == SKLS_SKETCH_BINNED && !binned_ok(A, t, ob)) {
    set_error("binned sketch needs d * sizeof(out) <= %zu bytes and t / buckets-per-bin <= %d", kBinAcc, kMaxBins);
    return SKLS_ERR_SHAPE;
  }
  if (v == SKLS_SKETCH_SORTED && !sorted_ok(A, ob)) {
    set_error("sorted CSR sketch supports d * sizeof(out) <= %d bytes; use the binned or atomic variant", kAccMax);
    return SKLS_ERR_SHAPE;
  }
  return SKLS_OK;
}

// ATOMIC: S A zeroed, then every entry added with a device-wide atomic.
int32_t run_atomic(const skls_matrix& A, const void* b, int b_f64, uint32_t tt, HashKey seed, const float* w, void* SA,
                   void* Sb, int32_t out_dtype, hipStream_t s) {
  const int d = static_cast<int>(A.d);
  const int64_t n = A.n;
  return with_out(out_dtype, [&](auto to) -> int32_t {
    using TO = decltype(to);
    {
      PhaseTimer pt("sketch_zero", s);
      SKLS_TRY(launch_fill_zero(SA, static_cast<size_t>(tt) * A.d * sizeof(TO), s));
      if (Sb) SKLS_TRY(launch_fill_zero(Sb, static_cast<size_t>(tt) * sizeof(TO), s));
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

// Build the bucket plan of a SORTED or BINNED sketch into P (b and w enter
// CSR records only when given).
int32_t plan_into(const skls_matrix& A, const BucketPlan& P, const void* b, int b_f64, uint32_t tt, HashKey seed,
                  const float* w, int32_t out_dtype, hipStream_t s) {
  const RowSrc src{A.layout == SKLS_CSR ? A.row_ptr : nullptr, b, b_f64, w};
  const int64_t n = A.n;
  PhaseTimer pt("sketch_plan", s);
  if (A.layout != SKLS_CSR) return build_plan<int32_t>(n, tt, seed, P, src, s);
  return with_out(out_dtype, [&](auto to) -> int32_t {
    using TO = decltype(to);
    return A.row_ptr_64 ? build_plan<CsrRec<int64_t, TO>>(n, tt, seed, P, src, s)
                        : build_plan<CsrRec<int32_t, TO>>(n, tt, seed, P, src, s);
  });
}

// Reduce with a built plan (S A zeroed first when several blocks share a bin).
int32_t apply_with(const skls_matrix& A, const BucketPlan& P, const void* b, int b_f64, uint32_t tt, HashKey seed,
                   const float* w, void* SA, void* Sb, int32_t out_dtype, const void* bg, hipStream_t s) {
  return with_out(out_dtype, [&](auto to) -> int32_t {
    using TO = decltype(to);
    if (P.S.splits > 1) {
      PhaseTimer pt("sketch_zero", s);
      SKLS_TRY(launch_fill_zero(SA, static_cast<size_t>(tt) * A.d * sizeof(TO), s));
      if (Sb) SKLS_TRY(launch_fill_zero(Sb, static_cast<size_t>(tt) * sizeof(TO), s));
    }
    PhaseTimer pt("sketch_apply", s);
    return apply_planned<TO>(A, P, b, b_f64, tt, seed, w, static_cast<TO*>(SA), static_cast<TO*>(Sb), bg, s);
  });
}

}  // namespace

int32_t run_sketch_key(const skls_matrix& A, const void* b, int32_t b_dtype, int64_t t, HashKey seed,
                       const float* w, int32_t variant, void* SA, void* Sb, int32_t out_dtype, void* ws,
                       size_t ws_bytes, hipStream_t s) {
  const int ob = out_bytes_of(out_dtype);
  const int32_t v = pick_variant(A, t, variant, ob);
  SKLS_TRY(check_variant(A, t, v, ob, variant));
  const int b_f64 = (b_dtype == SKLS_F64) ? 1 : 0;
  const uint32_t tt = static_cast<uint32_t>(t);
  if (v == SKLS_SKETCH_ATOMIC) return run_atomic(A, b, b_f64, tt, seed, w, SA, Sb, out_dtype, s);
  const PlanShape S = plan_shape(A, t, v, ob);
  Arena ar(ws, ws_bytes);
  const BucketPlan P = carve_plan(ar, S, A.n, t);
  if (!ws || !ar.fits()) {
    set_error("sketch workspace too small: need %zu bytes, have %zu", ar.used, ws_bytes);
    return SKLS_ERR_WORKSPACE;
  }
  SKLS_TRY(plan_into(A, P, b, b_f64, tt, seed, w, out_dtype, s));
  return apply_with(A, P, b, b_f64, tt, seed, w, SA, Sb, out_dtype, nullptr, s);
}

// ---------------------------------------------------------------- reusable plans
size_t sketch_plan_bytes(const skls_matrix& A, int64_t t, int32_t variant, int32_t out_dtype) {
  const int ob = out_bytes_of(out_dtype);
  const int32_t v = pick_variant(A, t, variant, ob);
  if (v != SKLS_SKETCH_SORTED && v != SKLS_SKETCH_BINNED) return 0;
  return plan_bytes(plan_shape(A, t, v, ob), A.n, t);
}

int32_t build_sketch_plan(const skls_matrix& A, int64_t t, HashKey seed, int32_t variant, int32_t out_dtype,
                          void* plan, size_t plan_bytes_, int32_t* resolved, hipStream_t s) {
  const int ob = out_bytes_of(out_dtype);
  const int32_t v = pick_variant(A, t, variant, ob);
  SKLS_TRY(check_variant(A, t, v, ob, variant));
  *resolved = v;
  if (v == SKLS_SKETCH_ATOMIC) return SKLS_OK;
  Arena ar(plan, plan_bytes_);
  const BucketPlan P = carve_plan(ar, plan_shape(A, t, v, ob), A.n, t);
  if (!plan || !ar.fits()) {
    set_error("sketch plan buffer too small: need %zu bytes, have %zu", ar.used, plan_bytes_);
    return SKLS_ERR_WORKSPACE;
  }
  return plan_into(A, P, nullptr, 0, static_cast<uint32_t>(t), seed, nullptr, out_dtype, s);
}

int32_t apply_sketch_plan(const skls_matrix& A, const void* b, int32_t b_dtype, int64_t t, HashKey seed,
                          const float* w, int32_t resolved, void* SA, void* Sb, int32_t out_dtype, const void* plan,
                          size_t plan_bytes_, hipStream_t s) {
  const int ob = out_bytes_of(out_dtype);
  SKLS_TRY(check_variant(A, t, resolved, ob, resolved));
  const int b_f64 = (b_dtype == SKLS_F64) ? 1 : 0;
  const uint32_t tt = static_cast<uint32_t>(t);
  if (resolved == SKLS_SKETCH_ATOMIC) return run_atomic(A, b, b_f64, tt, seed, w, SA, Sb, out_dtype, s);
  Arena ar(const_cast<void*>(plan), plan_bytes_);
  const BucketPlan P = carve_plan(ar, plan_shape(A, t, resolved, ob), A.n, t);
  if (!plan || !ar.fits()) {
    set_error("sketch plan buffer too small: need %zu bytes, have %zu", ar.used, plan_bytes_);
    return SKLS_ERR_WORKSPACE;
  }
  // CSR records of a reusable plan carry no share of S b: the reduce gathers b
  return apply_with(A, P, b, b_f64, tt, seed, w, SA, Sb, out_dtype, A.layout == SKLS_CSR ? b : nullptr, s);
}

int32_t sorted_plan_order(const skls_matrix& A, int64_t t, int32_t resolved, int32_t out_dtype, const void* plan,
                          size_t plan_bytes_, const int32_t** off, const int32_t** perm) {
  *off = nullptr;
  *perm = nullptr;
  if (A.layout != SKLS_DENSE || resolved != SKLS_SKETCH_SORTED) return SKLS_OK;
  Arena ar(const_cast<void*>(plan), plan_bytes_);
  const BucketPlan P = carve_plan(ar, plan_shape(A, t, resolved, out_bytes_of(out_dtype)), A.n, t);
  if (!plan || !ar.fits()) {
    set_error("sketch plan buffer too small: need %zu bytes, have %zu", ar.used, plan_bytes_);
    return SKLS_ERR_WORKSPACE;
  }
  *off = P.off;
  *perm = static_cast<const int32_t*>(P.fine);
  return SKLS_OK;
}

int32_t apply_sorted_many(const skls_matrix* A, int count, int64_t t, HashKey key, const float* w, const void* plan,
                          size_t plan_bytes, float* SA, int64_t sa_stride, hipStream_t s) {
  if (count < 1 || count > kSortedMany) {
    set_error("sorted sketch of several matrices: need 1 <= count <= %d", kSortedMany);
    return SKLS_ERR_ARG;
  }
  const int32_t *off = nullptr, *perm = nullptr;
  SKLS_TRY(sorted_plan_order(A[0], t, SKLS_SKETCH_SORTED, SKLS_F32, plan, plan_bytes, &off, &perm));
  if (off == nullptr) {
    set_error("sorted sketch of several matrices: the plan is not a dense sorted one");
    return SKLS_ERR_ARG;
  }
  SortedMany args{};
  bool vec = (sa_stride % 4) == 0;
  for (int j = 0; j < count; ++j) {
    if (A[j].layout != SKLS_DENSE || A[j].dtype != SKLS_F32 || A[j].n != A[0].n || A[j].d != A[0].d) {
      set_error("sorted sketch of several matrices: matrix %d is not a dense float32 matrix of the first's shape", j);
      return SKLS_ERR_SHAPE;
    }
    args.A[j] = static_cast<const float*>(A[j].val);
    args.ld[j] = A[j].ld;
    vec = vec && vec_ok<float>(A[j].val, A[j].ld, A[j].d, 4);
  }
  const uint32_t tt = static_cast<uint32_t>(t);
  const int d = static_cast<int>(A[0].d);
  const size_t lds = kBucketWaves * sizeof(DenseLds<float>);
  const void* kern = vec ? reinterpret_cast<const void*>(&k_sketch_dense_sorted_many<4>)
                         : reinterpret_cast<const void*>(&k_sketch_dense_sorted_many<1>);
  // each matrix as it would run alone (small sketches are bound by latency,
  // so the matrices' blocks together fill the chip better)
  const int bpw = buckets_per_wave(t, resident_waves(kern, lds));
  const dim3 grid(static_cast<unsigned>(div_up(div_up(t, bpw), kBucketWaves)), static_cast<unsigned>(count));
  const HashKey seed = key;
  if (vec)
    hipLaunchKernelGGL(k_sketch_dense_sorted_many<4>, grid, dim3(kThreads), lds, s, d, tt, bpw, seed, args, w, off,
                       perm, SA, sa_stride);
  else
    hipLaunchKernelGGL(k_sketch_dense_sorted_many<1>, grid, dim3(kThreads), lds, s, d, tt, bpw, seed, args, w, off,
                       perm, SA, sa_stride);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t run_sketch(const skls_matrix& A, const void* b, int32_t b_dtype, int64_t t, uint64_t seed,
                   const float* w, int32_t variant, void* SA, void* Sb, int32_t out_dtype, void* ws,
                   size_t ws_bytes, hipStream_t s) {
  return run_sketch_key(A, b, b_dtype, t, plain_key(seed), w, variant, SA, Sb, out_dtype, ws, ws_bytes, s);
}

}  // namespace skls
