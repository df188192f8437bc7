// Kernels and host helpers shared by the paths that sample rows by leverage
// scores (the rank-k approximation, Section 8 theorem in the Section 10 form,
// and multiple-response regression, Section 7 generalized regression):
// float64 GEMM on the matrix cores, fixed-order prefix sums, draws by binary
// search, compaction and gathers of the drawn rows, and sparse-times-dense
// products.  Everything sits in an unnamed namespace: each source file that
// includes this gets its own copy.
#pragma once

#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels.hpp"

namespace skls {
namespace {

constexpr uint64_t kPi2Salt = 0x6C65766572616765ull;     // "leverage"
constexpr uint64_t kSampleSalt = 0x73616D706C696E67ull;  // "sampling"
constexpr int kT = 256;

typedef double d4_t __attribute__((ext_vector_type(4)));

unsigned grid_for(int64_t work, int per_block, int64_t cap) {
  int64_t g = div_up(work > 0 ? work : 1, per_block);
  if (g > cap) g = cap;
  return static_cast<unsigned>(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------- float64 GEMM
// C (M x N) = alpha op(A) B on the float64 matrix cores, one tile per block
// of four wavefronts (32 x 32 outputs each; 64 x 64 tiles, or 128 x 32 for
// outputs at most 32 wide), the inner dimension staged through
// LDS 16 at a time.  op(A) = A (M x K, row-major, lda) or, with TA, A^T for A
// stored K x M; A may hold float64, float32 or bfloat16 values (widened on
// load).  B is K x N (ldb).  With several splits of the inner
// dimension (blockIdx.z), split z writes its partial product to
// C + z * split_stride.
template <bool TA, typename TAV, int WI>
__global__ __launch_bounds__(kT) void k_gemm(int64_t M, int64_t N, int64_t K, int64_t kc, double alpha,
                                             const TAV* __restrict__ A, int64_t lda,
                                             const double* __restrict__ B, int64_t ldb, double* __restrict__ C,
                                             int64_t ldc, int64_t split_stride) {
  constexpr int WJ = 4 / WI;           // wavefronts: WI x WJ, 32 x 32 outputs each
  constexpr int TM = 32 * WI, TN = 32 * WJ;
  __shared__ double As[16][TM + 1];
  __shared__ double Bs[16][TN + 1];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wv = tid / kWave;
  const int wi = wv / WJ, wj = wv % WJ;
  const int lr = lane >> 4, lc = lane & 15;
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * TM, j0 = static_cast<int64_t>(blockIdx.y) * TN;
  const int64_t kb = static_cast<int64_t>(blockIdx.z) * kc;
  const int64_t ke = (kb + kc) < K ? kb + kc : K;
  C += static_cast<int64_t>(blockIdx.z) * split_stride;
  d4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};
  // Each chunk of 16 inner indices is fetched into registers while the
  // previous one is multiplied.  Loads are unconditional (an index outside
  // the matrix reads element 0 and the value is masked afterwards), so all
  // loads of a chunk are in flight together.
  constexpr int RA = 16 * TM / kT, RB = 16 * TN / kT;
  double ra[RA], rb[RB];
  auto a_at = [&](int r, int& kk, int& c) {
    const int e = tid + r * kT;
    if (TA) {
      c = e % TM;
      kk = e / TM;
    } else {
      kk = e & 15;
      c = e >> 4;
    }
  };
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      int kk, c;
      a_at(r, kk, c);
      const int64_t gi = i0 + c, gk = k0 + kk;
      const bool in = gi < M && gk < ke;
      const size_t idx = in ? static_cast<size_t>(TA ? gk * lda + gi : gi * lda + gk) : 0;
      const double x = load_as<double>(A, idx);
      ra[r] = in ? x : 0.0;
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int e = tid + r * kT;
      const int c = e % TN, kk = e / TN;
      const int64_t gj = j0 + c, gk = k0 + kk;
      const bool in = gj < N && gk < ke;
      const double x = B[in ? gk * ldb + gj : 0];
      rb[r] = in ? x : 0.0;
    }
  };
  if (kb < ke) fetch(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += 16) {
    __syncthreads();  // the previous chunk's products are done with the tiles
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      int kk, c;
      a_at(r, kk, c);
      As[kk][c] = ra[r];
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int e = tid + r * kT;
      Bs[e / TN][e % TN] = rb[r];
    }
    __syncthreads();
    if (k0 + 16 < ke) fetch(k0 + 16);
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const double a0 = As[kk + lr][wi * 32 + lc], a1 = As[kk + lr][wi * 32 + 16 + lc];
      const double b0 = Bs[kk + lr][wj * 32 + lc], b1 = Bs[kk + lr][wj * 32 + 16 + lc];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
  // element e of lane l: row l / 16 + 4 e, column l % 16 of each 16 x 16 block
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = i0 + wi * 32 + a * 16 + lr + 4 * e, col = j0 + wj * 32 + b * 16 + lc;
        if (row < M && col < N) C[row * ldc + col] = alpha * acc[a][b][e];
      }
}

// C[i, j] = sum over splits of P[z][i, j] (M x N, leading dimension N).
__global__ void k_sum_splits(const double* __restrict__ P, int splits, int64_t MN, double* __restrict__ C) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < MN;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double s = 0.0;
    for (int z = 0; z < splits; ++z) s += P[static_cast<int64_t>(z) * MN + e];
    C[e] = s;
  }
}

// Pi2 [r][c] = +-1 / sqrt(k_G), sign from bit 0 of output r * k_G + c.
__global__ void k_sign_projection(int rows, int kg, uint64_t seed, double* __restrict__ Pi2) {
  const int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (e >= static_cast<int64_t>(rows) * kg) return;
  const uint64_t z = splitmix64(seed ^ kPi2Salt, static_cast<uint64_t>(e));
  const double v = 1.0 / sqrt(static_cast<double>(kg));
  Pi2[e] = negative_of(z) ? -v : v;
}

// out[i] = sum_c Z[i][c]^2 (one wavefront per row); last[0] = largest i with out[i] > 0.
__global__ __launch_bounds__(kT) void k_row_sqnorm(int64_t n, int cols, const double* __restrict__ Z,
                                                   double* __restrict__ out, int32_t* __restrict__ last) {
  __shared__ int32_t wlast[kT / kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t nw = static_cast<int64_t>(gridDim.x) * (kT / kWave);
  int32_t mine = -1;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kT / kWave) + threadIdx.x / kWave; i < n; i += nw) {
    double s = 0.0;
    for (int c = lane; c < cols; c += kWave) {
      const double z = Z[static_cast<size_t>(i) * cols + c];
      s += z * z;
    }
    s = wave_total(s);
    if (lane == 0) out[i] = s;
    if (s > 0.0) mine = static_cast<int32_t>(i);  // rows only grow along the loop
  }
  if (lane == 0) wlast[threadIdx.x / kWave] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t m = -1;
    for (int k = 0; k < kT / kWave; ++k) m = wlast[k] > m ? wlast[k] : m;
    if (m >= 0) atomicMax(last, m);
  }
}

// Inclusive prefix sums in three passes: per-block sums of kScanTile
// elements, a single-block scan of those sums, then the block scans with
// their offsets.  The order of additions is fixed (deterministic).
constexpr int kScanTile = 2048;  // 256 threads x 8

template <typename T>
__device__ T block_incl_scan(T v, T* sh) {
  // inclusive scan of one value per thread over the block (256 threads)
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < kT; off <<= 1) {
    const T add = tid >= off ? sh[tid - off] : T(0);
    __syncthreads();
    sh[tid] += add;
    __syncthreads();
  }
  const T r = sh[tid];
  __syncthreads();
  return r;
}

template <typename T>
__global__ __launch_bounds__(kT) void k_scan_tiles(const T* __restrict__ in, int64_t n, T* __restrict__ tile_sum) {
  __shared__ T sh[kT];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * 8;
  T s = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) s += (base + q < n) ? in[base + q] : T(0);
  const T tot = block_incl_scan(s, sh);
  if (threadIdx.x == kT - 1) tile_sum[blockIdx.x] = tot;
}

template <typename T>
__global__ __launch_bounds__(kT) void k_scan_top(T* __restrict__ tile_sum, int64_t ntiles) {
  // exclusive scan of the tile sums in place, one block, 256 at a time
  __shared__ T sh[kT];
  __shared__ T tot;
  T carry = 0;
  for (int64_t c0 = 0; c0 < ntiles; c0 += kT) {
    const int64_t i = c0 + threadIdx.x;
    const T v = i < ntiles ? tile_sum[i] : T(0);
    const T inc = block_incl_scan(v, sh);
    if (i < ntiles) tile_sum[i] = carry + inc - v;
    if (threadIdx.x == kT - 1) tot = inc;
    __syncthreads();
    carry += tot;
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(kT) void k_scan_apply(const T* __restrict__ in, int64_t n,
                                                   const T* __restrict__ tile_off, T* __restrict__ out,
                                                   int exclusive) {
  __shared__ T sh[kT];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * 8;
  T v[8];
  T s = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    v[q] = (base + q < n) ? in[base + q] : T(0);
    s += v[q];
  }
  const T inc = block_incl_scan(s, sh);
  T run = tile_off[blockIdx.x] + inc - s;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const T before = run;
    run += v[q];
    if (base + q < n) out[base + q] = exclusive ? before : run;
  }
}

// Draw j: u = (z >> 11) 2^-53 from the sampling stream, x = u * total; the row
// is the first i with cum[i] > x, at most `last` (the last positive score).
__global__ void k_sample(int64_t ts, int64_t n, uint64_t seed, const double* __restrict__ cum,
                         const double* __restrict__ score, const int32_t* __restrict__ last,
                         int32_t* __restrict__ counts) {
  const double total = cum[n - 1];
  const int64_t hi_row = static_cast<int64_t>(last[0]);
  for (int64_t j = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; j < ts;
       j += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint64_t z = splitmix64(seed ^ kSampleSalt, static_cast<uint64_t>(j));
    const double x = static_cast<double>(z >> 11) * 0x1.0p-53 * total;
    int64_t lo = 0, hi = n;  // first index with cum > x lies in [lo, hi]
    while (lo < hi) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      if (cum[mid] > x)
        hi = mid;
      else
        lo = mid + 1;
    }
    int64_t r = lo < hi_row ? lo : hi_row;
    // the running sums are rounded per tile; never land on a row without score
    while (r < hi_row && !(score[r] > 0.0)) ++r;
    atomicAdd(&counts[r], 1);
  }
}

__global__ void k_flags(int64_t n, const int32_t* __restrict__ counts, int32_t* __restrict__ flag) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    flag[i] = counts[i] > 0 ? 1 : 0;
}

// Sampled rows in increasing order: list[pos[i]] = i with weight
// sqrt(count_i total / (t_S score_i)); len[pos[i]] = nonzeros of row i (CSR).
template <typename TR>
__global__ void k_compact(int64_t n, int64_t ts, const int32_t* __restrict__ counts, const int32_t* __restrict__ pos,
                          const double* __restrict__ score, const double* __restrict__ cum,
                          const TR* __restrict__ row_ptr, int32_t* __restrict__ list, double* __restrict__ wts,
                          int64_t* __restrict__ len) {
  const double total = cum[n - 1];
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t c = counts[i];
    if (c == 0) continue;
    const int32_t p = pos[i];
    list[p] = static_cast<int32_t>(i);
    wts[p] = sqrt(static_cast<double>(c) * total / (static_cast<double>(ts) * score[i]));
    if (len) len[p] = static_cast<int64_t>(row_ptr[i + 1]) - static_cast<int64_t>(row_ptr[i]);
  }
}

// out[r][:] = w[r] * X[list[r]][:] (rows of width `cols`, float64 out)
template <typename TV>
__global__ __launch_bounds__(kT) void k_gather_rows(int64_t ns, int64_t cols, int64_t ldx, const TV* __restrict__ X,
                                                    const int32_t* __restrict__ list,
                                                    const double* __restrict__ w, double* __restrict__ out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t nw = static_cast<int64_t>(gridDim.x) * (kT / kWave);
  for (int64_t r = blockIdx.x * static_cast<int64_t>(kT / kWave) + threadIdx.x / kWave; r < ns; r += nw) {
    const size_t src = static_cast<size_t>(list[r]) * ldx;
    const double s = w[r];
    for (int64_t c = lane; c < cols; c += kWave)
      out[static_cast<size_t>(r) * cols + c] = s * load_as<double>(X, src + c);
  }
}

// Sampled CSR rows written densely: out[r][:] = w[r] * A[list[r]][:] (out
// zeroed first; repeated columns within a row are summed).
template <typename TV, typename TR>
__global__ __launch_bounds__(kT) void k_gather_csr_dense(int64_t ns, int64_t d, const TR* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col, const TV* __restrict__ val,
                                                         const int32_t* __restrict__ list,
                                                         const double* __restrict__ w, double* __restrict__ out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t nw = static_cast<int64_t>(gridDim.x) * (kT / kWave);
  for (int64_t r = blockIdx.x * static_cast<int64_t>(kT / kWave) + threadIdx.x / kWave; r < ns; r += nw) {
    const int32_t i = list[r];
    const int64_t b = static_cast<int64_t>(row_ptr[i]), e = static_cast<int64_t>(row_ptr[i + 1]);
    const double s = w[r];
    for (int64_t k = b + lane; k < e; k += kWave)
      unsafeAtomicAdd(out + static_cast<size_t>(r) * d + col[k], s * load_as<double>(val, static_cast<size_t>(k)));
  }
}

// Sampled CSR rows: columns copied, values scaled by the row weight (float64).
template <typename TV, typename TR>
__global__ __launch_bounds__(kT) void k_gather_csr(int64_t ns, const TR* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col, const TV* __restrict__ val,
                                                   const int32_t* __restrict__ list, const double* __restrict__ w,
                                                   const int64_t* __restrict__ rp, int32_t* __restrict__ col_out,
                                                   double* __restrict__ val_out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t nw = static_cast<int64_t>(gridDim.x) * (kT / kWave);
  for (int64_t r = blockIdx.x * static_cast<int64_t>(kT / kWave) + threadIdx.x / kWave; r < ns; r += nw) {
    const int32_t i = list[r];
    const int64_t b = static_cast<int64_t>(row_ptr[i]), e = static_cast<int64_t>(row_ptr[i + 1]);
    const int64_t o = rp[r];
    const double s = w[r];
    for (int64_t k = lane; k < e - b; k += kWave) {
      col_out[o + k] = col[b + k];
      val_out[o + k] = s * load_as<double>(val, static_cast<size_t>(b + k));
    }
  }
}

// ---------------------------------------------------------------- sparse products
__device__ __forceinline__ int32_t lane_i(int32_t v, int q) { return __builtin_amdgcn_readlane(v, q); }
__device__ __forceinline__ double lane_d(double v, int q) {
  const long long b = __double_as_longlong(v);
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int32_t>(b & 0xffffffffll), q));
  const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int32_t>(b >> 32), q));
  return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
}

// out (rows x p) = S X for S in CSR (any value and row-pointer type) and X
// (cols x p, float64); one wavefront per row.  The row's entries are loaded
// 64 at a time and read back lane by lane as scalars (uniform index), eight
// independent loads of X in flight.  HALF: p <= 32, the two half-waves take
// alternate entries and are summed at the end.
template <typename TV, typename TR, bool HALF>
__global__ __launch_bounds__(kT) void k_spmm(int64_t rows, int p, const TR* __restrict__ rp,
                                             const int32_t* __restrict__ col, const TV* __restrict__ val,
                                             const double* __restrict__ X, double* __restrict__ out) {
  constexpr int NB = 8;  // gathers in flight per lane
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t nw = static_cast<int64_t>(gridDim.x) * (kT / kWave);
  const int c = HALF ? (lane & 31) : lane;
  const int h = HALF ? (lane >> 5) : 0;
  const bool live = c < p;
  const int lc = live ? c : 0;
  constexpr int STEP = HALF ? 2 : 1;
  for (int64_t r = blockIdx.x * static_cast<int64_t>(kT / kWave) + threadIdx.x / kWave; r < rows; r += nw) {
    const int64_t b = static_cast<int64_t>(rp[r]), e = static_cast<int64_t>(rp[r + 1]);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t k0 = b; k0 < e; k0 += kWave) {
      const int64_t k = k0 + lane;
      const int32_t cj = k < e ? col[k] : 0;
      const double vj = k < e ? load_as<double>(val, static_cast<size_t>(k)) : 0.0;  // 0 beyond the row
      const int cnt = (e - k0) < kWave ? static_cast<int>(e - k0) : kWave;
      const int cnt_up = (cnt + NB * STEP - 1) / (NB * STEP) * (NB * STEP);  // zero values pad the tail
      for (int q = 0; q < cnt_up; q += NB * STEP) {
        int32_t j[NB];
        double v[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
          const int qa = q + u * STEP;
          if (HALF) {
            const int32_t ja = lane_i(cj, qa), jb = lane_i(cj, qa + 1);
            const double va = lane_d(vj, qa), vb = lane_d(vj, qa + 1);
            j[u] = h ? jb : ja;
            v[u] = h ? vb : va;
          } else {
            j[u] = lane_i(cj, qa);
            v[u] = lane_d(vj, qa);
          }
        }
        double x[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) x[u] = X[static_cast<size_t>(j[u]) * p + lc];
#pragma unroll
        for (int u = 0; u < NB; ++u) acc[u & 3] += v[u] * x[u];
      }
    }
    double a = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    if (HALF) a += __shfl_xor(a, 32);
    if (live && h == 0) out[static_cast<size_t>(r) * p + c] = a;
  }
}

// score[i] = || A[i, :] T ||^2 for CSR A and T (d x kg, kg <= 32, float64)
// with T staged in LDS (rows padded to 32 values), so the gathers of T's
// rows are LDS reads.  A wavefront takes eight consecutive rows at a time,
// eight lanes per row, four columns of T per lane; each lane loads its
// row's entries sixteen at a time (all loads in flight) and the squares are
// summed over the row's lanes.  last[0] = the largest row with a positive
// score.  Float64 throughout, no n x kg intermediate.
constexpr int kProjThreads = 512;
template <typename TV, typename TR>
__global__ __launch_bounds__(kProjThreads) void k_csr_proj_sqnorm(int64_t n, int d, int kg,
                                                                 const TR* __restrict__ rp,
                                                                 const int32_t* __restrict__ col,
                                                                 const TV* __restrict__ val,
                                                                 const double* __restrict__ T,
                                                                 double* __restrict__ score,
                                                                 int32_t* __restrict__ last) {
  extern __shared__ double Ts[];  // [d][32]
  __shared__ int32_t wlast[kProjThreads / kWave];
  for (int e = threadIdx.x; e < d * 32; e += kProjThreads) {
    const int r = e >> 5, c = e & 31;
    Ts[e] = c < kg ? T[static_cast<size_t>(r) * kg + c] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int slot = lane >> 3, cg = lane & 7;
  constexpr int kWaves = kProjThreads / kWave;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kWaves * 8;
  int32_t mine = -1;
  for (int64_t r0 = (static_cast<int64_t>(blockIdx.x) * kWaves + wid) * 8; r0 < n; r0 += stride) {
    const int64_t r = r0 + slot;
    const bool live = r < n;
    const int64_t b = live ? static_cast<int64_t>(rp[r]) : 0, e = live ? static_cast<int64_t>(rp[r + 1]) : 0;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int64_t k0 = b; __any(k0 < e); k0 += 16) {
      int32_t j[16];
      double v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int64_t k = k0 + q;
        const bool ok = k < e;
        j[q] = ok ? col[k] : 0;
        v[q] = ok ? load_as<double>(val, static_cast<size_t>(k)) : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const double* t = Ts + j[q] * 32 + cg * 4;
        const double2 t01 = *reinterpret_cast<const double2*>(t);
        const double2 t23 = *reinterpret_cast<const double2*>(t + 2);
        a0 += v[q] * t01.x;
        a1 += v[q] * t01.y;
        a2 += v[q] * t23.x;
        a3 += v[q] * t23.y;
      }
    }
    double sq = a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3;
    sq += __shfl_xor(sq, 1);
    sq += __shfl_xor(sq, 2);
    sq += __shfl_xor(sq, 4);
    if (live && cg == 0) {
      score[r] = sq;
      if (sq > 0.0) mine = static_cast<int32_t>(r) > mine ? static_cast<int32_t>(r) : mine;
    }
  }
  // largest row with a positive score: over the wave, the block, the grid
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t o = __shfl_xor(mine, off);
    mine = o > mine ? o : mine;
  }
  if (lane == 0) wlast[wid] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t m = -1;
    for (int k = 0; k < kWaves; ++k) m = wlast[k] > m ? wlast[k] : m;
    if (m >= 0) atomicMax(last, m);
  }
}

// out (rows x p) = A X for dense A (rows x cols, leading dimension ld, any
// value type) and X (cols x p); one wavefront per row as in k_spmm.
template <typename TV>
__global__ __launch_bounds__(kT) void k_dense_times(int64_t rows, int64_t cols, int64_t ld, int p,
                                                    const TV* __restrict__ A, const double* __restrict__ X,
                                                    double* __restrict__ out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t nw = static_cast<int64_t>(gridDim.x) * (kT / kWave);
  const int lc = lane < p ? lane : 0;
  for (int64_t r = blockIdx.x * static_cast<int64_t>(kT / kWave) + threadIdx.x / kWave; r < rows; r += nw) {
    double acc = 0.0;
    for (int64_t j0 = 0; j0 < cols; j0 += kWave) {
      const int64_t j = j0 + lane;
      const double aj = j < cols ? load_as<double>(A, static_cast<size_t>(r) * ld + j) : 0.0;
      const int cnt = (cols - j0) < kWave ? static_cast<int>(cols - j0) : kWave;
      for (int q = 0; q < cnt; ++q) acc += lane_d(aj, q) * X[static_cast<size_t>(j0 + q) * p + lc];
    }
    if (lane < p) out[static_cast<size_t>(r) * p + lane] = acc;
  }
}

}  // namespace

// ---------------------------------------------------------------- host side
namespace {

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
int32_t with_rowptr(const skls_matrix& A, F&& f) {
  if (A.row_ptr_64) return f(int64_t{});
  return f(int32_t{});
}

struct GemmScratch {
  double* part;
  size_t doubles;
};

// C = alpha op(A) B with the inner dimension split when the output has few
// tiles and the inner dimension is long.
template <typename TAV = double>
int32_t gemm(bool ta, int64_t M, int64_t N, int64_t K, double alpha, const TAV* A, int64_t lda, const double* B,
             int64_t ldb, double* C, int64_t ldc, const GemmScratch& sc, hipStream_t s) {
  if (M == 0 || N == 0) return SKLS_OK;
  const bool narrow = N <= 32;
  const int64_t TM = narrow ? 128 : 64, TN = narrow ? 32 : 64;
  const int64_t tiles = div_up(M, TM) * div_up(N, TN);
  int64_t splits = 1;
  if (tiles < 256 && K > 1024) {
    splits = div_up(512, tiles);
    const int64_t by_k = div_up(K, 256);
    if (splits > by_k) splits = by_k;
    if (splits > 256) splits = 256;
    while (splits > 1 && static_cast<size_t>(splits) * M * N > sc.doubles) --splits;
  }
  const int64_t kc = div_up(div_up(K > 0 ? K : 1, splits), 16) * 16;
  splits = div_up(K > 0 ? K : 1, kc);
  const dim3 grid(static_cast<unsigned>(div_up(M, TM)), static_cast<unsigned>(div_up(N, TN)),
                  static_cast<unsigned>(splits));
  double* out = splits > 1 ? sc.part : C;
  const int64_t ldo = splits > 1 ? N : ldc;
  if (splits > 1 && ldc != N) {
    set_error("internal: split GEMM needs a packed output");
    return SKLS_ERR_ARG;
  }
  auto launch = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(kT), 0, s, M, N, K, kc, alpha, A, lda, B, ldb, out, ldo, M * N);
  };
  if (ta)
    narrow ? launch(k_gemm<true, TAV, 4>) : launch(k_gemm<true, TAV, 2>);
  else
    narrow ? launch(k_gemm<false, TAV, 4>) : launch(k_gemm<false, TAV, 2>);
  SKLS_CHECK_LAUNCH();
  if (splits > 1) {
    hipLaunchKernelGGL(k_sum_splits, dim3(grid_for(M * N, kT, 4096)), dim3(kT), 0, s, sc.part,
                       static_cast<int>(splits), M * N, C);
    SKLS_CHECK_LAUNCH();
  }
  return SKLS_OK;
}

// out (n x k, float64) = A (n x d, float32 or bfloat16 rows) X (d x k,
// float64), k <= 16 NB, on float64 MFMA (v_mfma_f64_16x16x4f64).  X sits in
// LDS for the whole launch; each wavefront takes 16 rows at a time and
// stages a 16 x 32 slab of them in its own LDS tile (16-byte loads, 8 lanes
// per row, the next slab loaded while the current one is consumed), so that
// A is read once, in 128-byte row pieces.  Lane (li, lk) supplies row li of
// the slab at contraction indices 16 m + 4 lk + e, and row 16 m + 4 lk + e
// of X: any bijection of the contraction index over the lanes gives the
// same product.  Rows past n are computed from row n-1 and not stored.
constexpr int kDtCols = 32;
constexpr int kDtPitch = kDtCols + 4;  // floats; rows stay 16-byte aligned
typedef float dt_f4 __attribute__((ext_vector_type(4)));

template <typename TV>
__device__ __forceinline__ dt_f4 dt_load4(const TV* p) {
  if constexpr (std::is_same<TV, float>::value) {
    return stream_load<nt_f4>(p);
  } else {
    const nt_u2 u = stream_load<nt_u2>(p);
    return dt_f4{bf16_lo(u[0]), bf16_hi(u[0]), bf16_lo(u[1]), bf16_hi(u[1])};
  }
}

template <typename TV, int NB, int WAVES>
__global__ __launch_bounds__(WAVES * kWave) void k_dense_times_wide(int64_t n, int d, int64_t ld,
                                                                      const TV* __restrict__ A,
                                                                      const double* __restrict__ X, int k, int dpad,
                                                                      double* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char dt_smem[];
  constexpr int KW = 16 * NB;
  double* sX = reinterpret_cast<double*>(dt_smem);  // [dpad][KW]
  const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  float* tile = reinterpret_cast<float*>(dt_smem + static_cast<size_t>(dpad) * KW * sizeof(double)) +
                static_cast<size_t>(wid) * 16 * kDtPitch;
  for (int e = threadIdx.x; e < dpad * KW; e += blockDim.x) {
    const int r = e / KW, q = e % KW;
    sX[e] = (r < d && q < k) ? X[static_cast<size_t>(r) * k + q] : 0.0;
  }
  __syncthreads();
  const int li = lane & 15, lk = lane >> 4;
  const int lrow = lane >> 3, lcol = 4 * (lane & 7);  // loads: rows lrow, lrow + 8; columns lcol .. + 3
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwave = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  const int nchunk = dpad / kDtCols;
  for (int64_t r0 = wave * 16; r0 < n; r0 += nwave * 16) {
    const TV* rowp[2];
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int64_t r = r0 + lrow + 8 * it;
      rowp[it] = A + static_cast<size_t>(r < n ? r : n - 1) * ld;
    }
    dt_f4 nxt[2];
#pragma unroll
    for (int it = 0; it < 2; ++it) nxt[it] = lcol < d ? dt_load4<TV>(rowp[it] + lcol) : dt_f4{0.f, 0.f, 0.f, 0.f};
    d4_t acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = d4_t{0.0, 0.0, 0.0, 0.0};
    for (int ch = 0; ch < nchunk; ++ch) {
      const int c0 = ch * kDtCols;
#pragma unroll
      for (int it = 0; it < 2; ++it) *reinterpret_cast<dt_f4*>(tile + (lrow + 8 * it) * kDtPitch + lcol) = nxt[it];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (ch + 1 < nchunk) {
        const int c = c0 + kDtCols + lcol;
#pragma unroll
        for (int it = 0; it < 2; ++it) nxt[it] = c < d ? dt_load4<TV>(rowp[it] + c) : dt_f4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int m = 0; m < kDtCols / 16; ++m) {
        const dt_f4 a = *reinterpret_cast<const dt_f4*>(tile + li * kDtPitch + 16 * m + 4 * lk);
        const double* xb = sX + static_cast<size_t>(c0 + 16 * m + 4 * lk) * KW + li;
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int b = 0; b < NB; ++b)
            acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(static_cast<double>(a[e]), xb[e * KW + 16 * b], acc[b], 0,
                                                          0, 0);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // element e of lane (li, lk): row lk + 4 e, column 16 b + li
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t r = r0 + lk + 4 * e;
        const int c = 16 * b + li;
        if (r < n && c < k) out[static_cast<size_t>(r) * k + c] = acc[b][e];
      }
  }
}

// out (n x k, packed) = A X for dense A of value type TV: the slab kernel
// when the rows are float32 or bfloat16 with d a multiple of 4, 16-byte
// (bfloat16: 8-byte) aligned rows, k <= 32 and X fitting LDS; otherwise the
// tiled GEMM.
template <typename TV>
int32_t dense_times(int64_t n, int64_t d, const TV* A, int64_t ld, const double* X, int64_t k, double* out,
                    const GemmScratch& sc, hipStream_t s) {
  if constexpr (!std::is_same<TV, double>::value) {
    constexpr int VB = sizeof(TV) == 2 ? 8 : 16;
    const int64_t dpad = div_up(d, kDtCols) * kDtCols;
    // 16 wavefronts per block while X leaves room (16 columns), else 8
    const int NB = k <= 16 ? 1 : 2;
    const int waves = NB == 1 ? 16 : 8;
    const size_t lds = static_cast<size_t>(dpad) * 16 * NB * sizeof(double) +
                       static_cast<size_t>(waves) * 16 * kDtPitch * sizeof(float);
    const bool fits = d % 4 == 0 && (ld * static_cast<int64_t>(sizeof(TV))) % VB == 0 &&
                      reinterpret_cast<uintptr_t>(A) % VB == 0 && k >= 1 && k <= 32 && lds <= 150 * 1024 && n > 0;
    if (fits) {
      int cus = 256;
      int dev = 0;
      if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      int64_t g = div_up(n, 16 * waves);
      if (g > cus) g = cus;
      auto go = [&](auto kern) -> int32_t {
        if (lds > 65536)
          SKLS_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
        hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(g)), dim3(waves * kWave), lds, s, n,
                           static_cast<int>(d), ld, A, X, static_cast<int>(k), static_cast<int>(dpad), out);
        SKLS_CHECK_LAUNCH();
        return SKLS_OK;
      };
      return NB == 1 ? go(k_dense_times_wide<TV, 1, 16>) : go(k_dense_times_wide<TV, 2, 8>);
    }
  }
  return gemm<TV>(false, n, k, d, 1.0, A, ld, X, k, out, k, sc, s);
}

// out (n x p) = A X for CSR A (n x cols) and X (cols x p, float64), p <= 64.
template <typename TV, typename TR>
int32_t spmm(const skls_matrix& A, int p, const double* X, double* out, hipStream_t s) {
  const int64_t n = A.n;
  if (n == 0) return SKLS_OK;
  const auto* rp = static_cast<const TR*>(A.row_ptr);
  const auto* val = static_cast<const TV*>(A.val);
  const unsigned g = grid_for(n, kT / kWave, 8192);
  if (p <= 32)
    hipLaunchKernelGGL((k_spmm<TV, TR, true>), dim3(g), dim3(kT), 0, s, n, p, rp, A.col_idx, val, X, out);
  else
    hipLaunchKernelGGL((k_spmm<TV, TR, false>), dim3(g), dim3(kT), 0, s, n, p, rp, A.col_idx, val, X, out);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

// Section 6 row-norm estimates in float64: score_i = ||(A R^{-1} Pi2)_i||^2
// with Pi2 the d x kg sign matrix / sqrt(kg) of the stream seed ^
// "leverage".  Pi2, T (d x kg) and Z (n x kg) are scratch; last[0] receives
// the largest row with a positive score.
int32_t row_norm_estimates(const skls_matrix& A, const double* Rinv, int kg, uint64_t seed, double* Pi2, double* T,
                           double* Z, double* score, int32_t* last, const GemmScratch& gs, hipStream_t s) {
  const int64_t n = A.n, d = A.d;
  hipLaunchKernelGGL(k_sign_projection, dim3(grid_for(d * kg, kT, 1 << 20)), dim3(kT), 0, s, static_cast<int>(d), kg,
                     seed, Pi2);
  SKLS_CHECK_LAUNCH();
  SKLS_TRY(gemm(false, d, kg, d, 1.0, Rinv, d, Pi2, kg, T, kg, gs, s));
  SKLS_TRY(launch_fill_zero(last, 16, s));
  const size_t proj_lds = static_cast<size_t>(d) * 32 * sizeof(double);
  if (A.layout == SKLS_CSR && kg <= 32 && proj_lds <= 96 * 1024) {
    // CSR rows against T in LDS: the scores directly, no n x kg product
    if (n == 0) return SKLS_OK;
    return with_value(A.dtype, [&](auto tv) -> int32_t {
      using TV = decltype(tv);
      return with_rowptr(A, [&](auto trt) -> int32_t {
        using TR = decltype(trt);
        const void* kern = reinterpret_cast<const void*>(&k_csr_proj_sqnorm<TV, TR>);
        SKLS_TRY_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(proj_lds)));
        int cus = 256, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                     hipSuccess || cus < 1)
          cus = 256;
        const int64_t per_block = (kProjThreads / kWave) * 8;
        int64_t g = div_up(n, per_block);
        if (g > 2 * cus) g = 2 * cus;
        hipLaunchKernelGGL((k_csr_proj_sqnorm<TV, TR>), dim3(static_cast<unsigned>(g)), dim3(kProjThreads), proj_lds,
                           s, n, static_cast<int>(d), kg, static_cast<const TR*>(A.row_ptr), A.col_idx,
                           static_cast<const TV*>(A.val), T, score, last);
        SKLS_CHECK_LAUNCH();
        return SKLS_OK;
      });
    });
  }
  int32_t st = with_value(A.dtype, [&](auto tv) -> int32_t {
    using TV = decltype(tv);
    if (A.layout != SKLS_CSR) return dense_times<TV>(n, d, static_cast<const TV*>(A.val), A.ld, T, kg, Z, gs, s);
    return with_rowptr(A, [&](auto trt) -> int32_t {
      using TR = decltype(trt);
      return spmm<TV, TR>(A, kg, T, Z, s);
    });
  });
  SKLS_TRY(st);
  hipLaunchKernelGGL(k_row_sqnorm, dim3(grid_for(n, kT / kWave, 8192)), dim3(kT), 0, s, n, kg, Z, score, last);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

template <typename T>
int32_t scan(const T* in, int64_t n, T* tiles, T* out, bool exclusive, hipStream_t s) {
  if (n == 0) return SKLS_OK;
  const int64_t nt = div_up(n, kScanTile);
  hipLaunchKernelGGL(k_scan_tiles<T>, dim3(static_cast<unsigned>(nt)), dim3(kT), 0, s, in, n, tiles);
  SKLS_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_scan_top<T>, dim3(1), dim3(kT), 0, s, tiles, nt);
  SKLS_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_scan_apply<T>, dim3(static_cast<unsigned>(nt)), dim3(kT), 0, s, in, n, tiles, out,
                     exclusive ? 1 : 0);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}


int64_t tiles_for(int64_t n) { return div_up(n > 0 ? n : 1, kScanTile) + 1; }

int32_t to_host(void* dst, const void* src, size_t bytes, hipStream_t s) {
  SKLS_TRY_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
  SKLS_TRY_HIP(hipStreamSynchronize(s));
  return SKLS_OK;
}

}  // namespace
}  // namespace skls
