// Dense float64 linear algebra on the sketch (Section 7: the sketched
// regression is solved through a QR factorisation of S A and R^{-1} Q^T S b).
//
// R is obtained as the Cholesky factor of the Gram matrix (S A)^T (S A)
// (CholeskyQR): the Gram of the augmented matrix [S A | S b] is a dense
// contraction over the t sketch rows and runs on the float64 matrix cores
// (v_mfma_f64_16x16x4f64) with split-K partial tiles; the Cholesky of the
// small d x d Gram, the triangular inverse and the d x d products run on
// vector units.  In exact arithmetic this R equals the R of a QR
// factorisation of S A with positive diagonal, and Q^T S b = R^{-T} (S A)^T S b.
#include <cmath>
#include <type_traits>

#include "kernels.hpp"
#include "profile.hpp"

namespace skls {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int kGT = 128;         // Gram output tile (kGT x kGT per block)
constexpr int kGK = 32;          // sketch rows staged in LDS per step
constexpr int kGThreads = 256;   // 4 waves, each 64 x 64 of the tile
constexpr int kGLoads = kGK * kGT / 4 / kGThreads;  // 4-wide loads per thread per strip and step

__device__ __forceinline__ void tile_of(int p, int T, int& ti, int& tj) {
  ti = 0;
  while (p >= T - ti) {
    p -= T - ti;
    ++ti;
  }
  tj = ti + p;
}

// Staging type in LDS: float64 inputs stay float64, float32 and bfloat16
// inputs are staged as float32 (exact) and widened when fed to the matrix
// cores.
template <typename TI>
using GStage = typename std::conditional<std::is_same<TI, double>::value, double, float>::type;

// Four consecutive elements of row k, columns c .. c + 3; `in` tells whether
// they lie inside the matrix (rows before k1, columns before d).  VEC
// (16-byte aligned rows, d a multiple of 4): one vector load from a clamped,
// always valid address, so that all loads of a strip are in flight together
// (the zeroing of elements outside happens when they are stored to LDS).
// Otherwise element-wise guarded loads, already zeroed.
template <typename TI, bool VEC>
__device__ __forceinline__ void gload4(const TI* __restrict__ M, int64_t ld, int64_t k, int64_t k1, int c, int d,
                                       GStage<TI> (&o)[4], bool& in) {
  using TS = GStage<TI>;
  if (VEC) {
    in = k < k1 && c < d;
    const TI* p = M + static_cast<size_t>(in ? k : k1 - 1) * ld + (in ? c : 0);
    if constexpr (std::is_same<TI, float>::value) {
      const float4 y = *reinterpret_cast<const float4*>(p);
      o[0] = y.x;
      o[1] = y.y;
      o[2] = y.z;
      o[3] = y.w;
    } else if constexpr (std::is_same<TI, double>::value) {
      const double2 y0 = *reinterpret_cast<const double2*>(p);
      const double2 y1 = *reinterpret_cast<const double2*>(p + 2);
      o[0] = y0.x;
      o[1] = y0.y;
      o[2] = y1.x;
      o[3] = y1.y;
    } else {
      const uint2 y = *reinterpret_cast<const uint2*>(p);
      o[0] = bf16_lo(y.x);
      o[1] = bf16_hi(y.x);
      o[2] = bf16_lo(y.y);
      o[3] = bf16_hi(y.y);
    }
    return;
  }
  in = true;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    o[e] = (k < k1 && c + e < d) ? load_as<TS>(M, static_cast<size_t>(k) * ld + c + e) : TS(0);
}

template <typename TI, bool VEC, bool DIAG>
__device__ __forceinline__ void gram_fetch(const TI* __restrict__ M, int64_t ld, int64_t kb, int64_t k1, int I0,
                                           int J0, int d, GStage<TI> (&ra)[kGLoads][4],
                                           GStage<TI> (&rb)[kGLoads][4], bool (&ia)[kGLoads],
                                           bool (&ib)[kGLoads]) {
#pragma unroll
  for (int u = 0; u < kGLoads; ++u) {
    const int e = (u * kGThreads + static_cast<int>(threadIdx.x)) * 4;
    const int r = e / kGT, c = e % kGT;
    gload4<TI, VEC>(M, ld, kb + r, k1, I0 + c, d, ra[u], ia[u]);
    if (!DIAG) gload4<TI, VEC>(M, ld, kb + r, k1, J0 + c, d, rb[u], ib[u]);
  }
}

template <typename TS, bool DIAG>
__device__ __forceinline__ void gram_stash(TS (*As)[kGT], TS (*Bs)[kGT], const TS (&ra)[kGLoads][4],
                                           const TS (&rb)[kGLoads][4], const bool (&ia)[kGLoads],
                                           const bool (&ib)[kGLoads]) {
#pragma unroll
  for (int u = 0; u < kGLoads; ++u) {
    const int e = (u * kGThreads + static_cast<int>(threadIdx.x)) * 4;
    const int r = e / kGT, c = e % kGT;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      As[r][c + q] = ia[u] ? ra[u][q] : TS(0);
      if (!DIAG) Bs[r][c + q] = ib[u] ? rb[u][q] : TS(0);
    }
  }
}

// Partial Gram tile (ti, tj) over the rows [k0, k1) of one split, on the
// float64 matrix cores: partial[split][pair][kGT][kGT].  Strips of kGK rows
// are staged in LDS, the next strip's loads in flight while the current one
// is multiplied.  DIAG: the diagonal tiles (ti = tj = blockIdx.x; one strip
// serves both operands), which with WITHV also form their columns' share of
// M^T v; otherwise the off-diagonal tile pairs ti < tj.
template <typename TI, bool VEC, bool DIAG, bool WITHV>
__global__ __launch_bounds__(kGThreads) void k_gram_partial(const TI* __restrict__ M, int64_t ld,
                                                            const void* __restrict__ v, int v_f64, int64_t m, int d,
                                                            int T, int P, int64_t rows_per_split,
                                                            double* __restrict__ partial,
                                                            double* __restrict__ partial_v) {
  using TS = GStage<TI>;
  __shared__ TS As[2][kGK][kGT];
  __shared__ TS Bs[DIAG ? 1 : 2][DIAG ? 1 : kGK][kGT];
  __shared__ double vs[2][kGK];
  __shared__ double vred[kGT];
  int ti, tj, pair;
  if (DIAG) {
    ti = tj = blockIdx.x;
    pair = 0;
    for (int q = 0; q < ti; ++q) pair += T - q;  // index of (ti, ti) in the upper-triangle order
  } else {
    // off-diagonal pairs in order, skipping the diagonal ones
    int p = blockIdx.x;
    ti = 0;
    while (p >= T - ti - 1) {
      p -= T - ti - 1;
      ++ti;
    }
    tj = ti + 1 + p;
    pair = 0;
    for (int q = 0; q < ti; ++q) pair += T - q;
    pair += tj - ti;
  }
  const int I0 = ti * kGT, J0 = tj * kGT;
  const int64_t k0 = static_cast<int64_t>(blockIdx.y) * rows_per_split;
  const int64_t k1 = (k0 + rows_per_split < m) ? k0 + rows_per_split : m;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int wi = wv >> 1, wj = wv & 1;
  const int lr = lane >> 4, lc = lane & 15;
  d4_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};
  double vacc = 0.0;  // WITHV: column (tid % kGT) of M^T v over half of each strip's rows
  double vv = 0.0;    // WITHV, first tile: v^T v over row (tid % kGK) of each strip
  TS ra[kGLoads][4], rb[kGLoads][4];
  bool ia[kGLoads], ib[kGLoads];
  double rv = 0.0;
  // every thread loads one entry of v (clamped to a valid row) so that the
  // load is unconditional; the first kGK threads keep theirs
  auto vload = [&](int64_t kb) {
    if (WITHV) {
      const int64_t k = kb + (threadIdx.x % kGK);
      const int64_t kc = k < k1 ? k : k1 - 1;
      const double x =
          v_f64 ? static_cast<const double*>(v)[kc] : static_cast<double>(static_cast<const float*>(v)[kc]);
      rv = k < k1 ? x : 0.0;
    }
  };
  const bool full = I0 + kGT <= d && J0 + kGT <= d;  // the whole tile lies inside d x d
  int buf = 0;
  if (k0 < k1) {
    gram_fetch<TI, VEC, DIAG>(M, ld, k0, k1, I0, J0, d, ra, rb, ia, ib);
    vload(k0);
    gram_stash<TS, DIAG>(As[0], Bs[0], ra, rb, ia, ib);
    if (WITHV && threadIdx.x < kGK) vs[0][threadIdx.x] = rv;
  }
  __syncthreads();
  for (int64_t kb = k0; kb < k1; kb += kGK) {
    const bool more = kb + kGK < k1;
    if (more) {
      gram_fetch<TI, VEC, DIAG>(M, ld, kb + kGK, k1, I0, J0, d, ra, rb, ia, ib);
      vload(kb + kGK);
    }
    const TS(*Ab)[kGT] = As[buf];
    const TS(*Bb)[kGT] = DIAG ? As[buf] : Bs[DIAG ? 0 : buf];
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 4) {
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = static_cast<double>(Ab[kk + lr][wi * 64 + q * 16 + lc]);
        b[q] = static_cast<double>(Bb[kk + lr][wj * 64 + q * 16 + lc]);
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
    if (WITHV) {
      const int c = threadIdx.x % kGT, h = threadIdx.x / kGT;
#pragma unroll 4
      for (int r = h; r < kGK; r += kGThreads / kGT) vacc += static_cast<double>(Ab[r][c]) * vs[buf][r];
      if (threadIdx.x < kGK) vv += vs[buf][threadIdx.x] * vs[buf][threadIdx.x];
    }
    if (more) {
      gram_stash<TS, DIAG>(As[buf ^ 1], Bs[DIAG ? 0 : (buf ^ 1)], ra, rb, ia, ib);
      if (WITHV && threadIdx.x < kGK) vs[buf ^ 1][threadIdx.x] = rv;
    }
    __syncthreads();
    buf ^= 1;
  }
  // Output layout of v_mfma_f64_16x16x4f64: element e of lane l holds row
  // (l / 16) + 4 e, column l % 16 of the 16 x 16 block (checked on gfx950).
  double* out = partial + (static_cast<size_t>(blockIdx.y) * P + pair) * (kGT * kGT);
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = wi * 64 + x * 16 + lr + 4 * e;
        const int colx = wj * 64 + y * 16 + lc;
        if (full || (I0 + row < d && J0 + colx < d)) out[row * kGT + colx] = acc[x][y][e];
      }
  if (WITHV) {
    const int c = threadIdx.x % kGT, h = threadIdx.x / kGT;
    if (h == 1) vred[c] = vacc;
    __syncthreads();
    if (h == 0) partial_v[(static_cast<size_t>(blockIdx.y) * T + ti) * kGT + c] = vacc + vred[c];
    if (ti == 0 && threadIdx.x < kWave) {  // the first wave holds the kGK row sums of v^T v
      vv = wave_sum(vv);
      if (threadIdx.x == 0) partial_v[static_cast<size_t>(gridDim.y) * T * kGT + blockIdx.y] = vv;
    }
  }
}

// Gram of a matrix of at most 64 columns (with v: [M | v], at most 64 in
// all).  k_gram_partial gives each wave a 64 x 64 quadrant of a 128 x 128
// tile, so at d <= 64 one wave would take every row alone while three
// multiply zeros.  Here the four waves split each staged chunk of kSK rows by
// rows (16 each) and form only the 16 x 16 blocks on and above the diagonal
// of the one 64 x 64 tile (the reduction reads the upper triangle of diagonal
// tiles); their sums meet in LDS at the end.  Block b writes split b of the
// partial layout of k_gram_partial (pair 0), entries inside d x d, so
// k_gram_reduce finishes the Gram.
constexpr int kSK = 64;  // rows per staged chunk
constexpr int kSB = 10;  // 16 x 16 blocks (x <= y) of a 64 x 64 upper triangle
constexpr int kSL = kSK * 64 / 4 / kGThreads;  // 4-wide loads per thread per chunk

template <typename TI, bool VEC, bool WITHV>
__global__ __launch_bounds__(kGThreads) void k_gram_small(const TI* __restrict__ M, int64_t ld,
                                                          const void* __restrict__ v, int v_f64, int64_t m, int d,
                                                          int64_t rows_per_split, double* __restrict__ partial,
                                                          int64_t mstride, int64_t pstride) {
  // WITHV: the product is [M | v] with v as column dm = d - 1 (v in the
  // staging precision: float64 with float64 M, float32 otherwise).  Several
  // matrices of one shape: matrix blockIdx.y at M + y * mstride, its splits
  // at partial + y * pstride.
  M += static_cast<int64_t>(blockIdx.y) * mstride;
  partial += static_cast<int64_t>(blockIdx.y) * pstride;
  const int dm = WITHV ? d - 1 : d;
  using TS = GStage<TI>;
  constexpr size_t kStage = 2 * kSK * 64 * sizeof(TS);
  constexpr size_t kRed = 3 * kSB * 4 * kWave * sizeof(double);
  __shared__ __align__(16) unsigned char lds[kStage > kRed ? kStage : kRed];
  TS(*As)[kSK][64] = reinterpret_cast<TS(*)[kSK][64]>(lds);
  const int64_t k0 = static_cast<int64_t>(blockIdx.x) * rows_per_split;
  const int64_t k1 = (k0 + rows_per_split < m) ? k0 + rows_per_split : m;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int lr = lane >> 4, lc = lane & 15;
  d4_t acc[kSB];
#pragma unroll
  for (int n = 0; n < kSB; ++n) acc[n] = d4_t{0.0, 0.0, 0.0, 0.0};
  TS ra[kSL][4];
  bool ia[kSL];
  auto fetch = [&](int64_t kb) {
#pragma unroll
    for (int u = 0; u < kSL; ++u) {
      const int e = (u * kGThreads + static_cast<int>(threadIdx.x)) * 4;
      gload4<TI, VEC>(M, ld, kb + e / 64, k1, e % 64, dm, ra[u], ia[u]);
      if (WITHV) {
        const int c = e % 64;
        if (c <= dm && dm < c + 4) {  // this group of four holds column dm
          const int64_t k = kb + e / 64;
          const int64_t kc = k < k1 ? k : k1 - 1;
          const TS x = v_f64 ? static_cast<TS>(static_cast<const double*>(v)[kc])
                             : static_cast<TS>(static_cast<const float*>(v)[kc]);
          // VEC zeroes the whole group through ia; fill it explicitly
          if (VEC) {
#pragma unroll
            for (int q = 0; q < 4; ++q) ra[u][q] = TS(0);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (c + q == dm) ra[u][q] = k < k1 ? x : TS(0);
          ia[u] = true;
        }
      }
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < kSL; ++u) {
      const int e = (u * kGThreads + static_cast<int>(threadIdx.x)) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) As[buf][e / 64][e % 64 + q] = ia[u] ? ra[u][q] : TS(0);
    }
  };
  int buf = 0;
  if (k0 < k1) {
    fetch(k0);
    stash(0);
  }
  __syncthreads();
  for (int64_t kb = k0; kb < k1; kb += kSK) {
    const bool more = kb + kSK < k1;
    if (more) fetch(kb + kSK);
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      // the two operands of a diagonal tile are the same staged rows
      double a[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = static_cast<double>(As[buf][wv * 16 + kk + lr][q * 16 + lc]);
      int n = 0;
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = x; y < 4; ++y, ++n) acc[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], a[y], acc[n], 0, 0, 0);
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // the staging buffers are free (the loop ended on a barrier): waves 1..3
  // leave their sums in LDS, wave 0 adds them and stores the split
  double* red = reinterpret_cast<double*>(lds);
  if (wv > 0) {
#pragma unroll
    for (int n = 0; n < kSB; ++n)
#pragma unroll
      for (int e = 0; e < 4; ++e) red[((wv - 1) * kSB * 4 + n * 4 + e) * kWave + lane] = acc[n][e];
  }
  __syncthreads();
  if (wv != 0) return;
  double* out = partial + static_cast<size_t>(blockIdx.x) * (kGT * kGT);
  int n = 0;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = x; y < 4; ++y, ++n)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        double sum = acc[n][e];
#pragma unroll
        for (int w = 0; w < 3; ++w) sum += red[(w * kSB * 4 + n * 4 + e) * kWave + lane];
        // element e of lane l: row l / 16 + 4 e, column l % 16 of the block
        const int row = x * 16 + lr + 4 * e, col = y * 16 + lc;
        if (row < d && col < d) out[row * kGT + col] = sum;
      }
}

// G[i][j] (both triangles) from the partial tiles (diagonal tiles summed over
// Sd splits, the others over So); column d from the partial M^T v when v was
// given.
__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ partial,
                                                     const double* __restrict__ partial_v, int P, int Sd, int So,
                                                     int T, int d, int with_v, double* __restrict__ G) {
  const int dd = d + with_v;
  const int p = blockIdx.x;
  if (p == P) {  // the M^T v column and v^T v
    if (!with_v) return;
    for (int i = blockIdx.y * 256 + threadIdx.x; i < T * kGT; i += gridDim.y * 256) {
      if (i >= d) continue;
      double s = 0.0;
      for (int sp = 0; sp < Sd; ++sp) s += partial_v[static_cast<size_t>(sp) * T * kGT + i];
      G[static_cast<size_t>(i) * dd + d] = s;
      G[static_cast<size_t>(d) * dd + i] = s;
    }
    if (blockIdx.y == 0 && threadIdx.x == 0) {
      double s = 0.0;
      for (int sp = 0; sp < Sd; ++sp) s += partial_v[static_cast<size_t>(Sd) * T * kGT + sp];
      G[static_cast<size_t>(d) * dd + d] = s;
    }
    return;
  }
  int ti, tj;
  tile_of(p, T, ti, tj);
  const int S = ti == tj ? Sd : So;
  const int idx = blockIdx.y * 256 + threadIdx.x;
  const int i = ti * kGT + idx / kGT, j = tj * kGT + idx % kGT;
  // diagonal tiles hold both (i, j) and (j, i): write each pair once; the
  // partial tiles hold only entries inside the d x d matrix
  if (!(i < d && j < d && (ti != tj || i <= j))) return;
  // eight running sums so that eight loads are in flight
  const double* src = partial + static_cast<size_t>(p) * (kGT * kGT) + idx;
  const size_t stride = static_cast<size_t>(P) * (kGT * kGT);
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int sp = 0;
  for (; sp + 8 <= S; sp += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] += src[static_cast<size_t>(sp + u) * stride];
  }
  for (int u = 0; sp < S; ++sp, ++u) acc[u] += src[static_cast<size_t>(sp) * stride];
  const double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  G[static_cast<size_t>(i) * dd + j] = s;
  G[static_cast<size_t>(j) * dd + i] = s;
}

// ---------------------------------------------------------------- blocked Cholesky
// Upper Cholesky G = R^T R in place on a d x d row-major copy W, by blocks of
// kCB rows: factor the diagonal block in LDS (and invert it), solve for the
// block row to its right, then update the trailing upper triangle.
constexpr int kCB = 64;
constexpr int kCP = kCB + 1;  // LDS pitch of a 64 x 64 tile of doubles

// C (the 32 x 32 quadrant (wi, wj) of a 64 x 64 product, as 2 x 2 MFMA
// tiles of 16 x 16) += A^T B for A, B held in LDS by inner index:
// A[k][m], B[k][n], k in [0, 64).  Four wavefronts, one quadrant each.
// Accumulator element e of lane l: row wi * 32 + a * 16 + l / 16 + 4 e,
// column wj * 32 + b * 16 + l % 16.
__device__ __forceinline__ void mfma_atb64(const double (*A)[kCP], const double (*B)[kCP], d4_t (&acc)[2][2]) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int wi = wv >> 1, wj = wv & 1;
  const int lr = lane >> 4, lc = lane & 15;
#pragma unroll 4
  for (int kk = 0; kk < kCB; kk += 4) {
    const double a0 = A[kk + lr][wi * 32 + lc], a1 = A[kk + lr][wi * 32 + 16 + lc];
    const double b0 = B[kk + lr][wj * 32 + lc], b1 = B[kk + lr][wj * 32 + 16 + lc];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

template <typename F>
__device__ __forceinline__ void for_acc(F&& f) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int wi = wv >> 1, wj = wv & 1;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) f(a, b, e, wi * 32 + a * 16 + (lane >> 4) + 4 * e, wj * 32 + b * 16 + (lane & 15));
}

__device__ __forceinline__ void zero_acc(d4_t (&acc)[2][2]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};
}

// dst = the 64 x 64 tile at src (leading dimension ld), rows < nr and
// columns < nc, zero elsewhere; TRANS stores it transposed.  Every thread's
// sixteen loads are in flight before its LDS stores (the tiles sit in L2,
// so the latency of one load would otherwise be paid sixteen times).
template <bool TRANS>
__device__ __forceinline__ void tile_to_lds(double (*dst)[kCP], const double* __restrict__ src, int64_t ld, int nr,
                                            int nc) {
  double v[kCB * kCB / 256];
#pragma unroll
  for (int u = 0; u < kCB * kCB / 256; ++u) {
    const int e = static_cast<int>(threadIdx.x) + 256 * u;
    const int r = e >> 6, c = e & (kCB - 1);
    v[u] = (r < nr && c < nc) ? src[static_cast<int64_t>(r) * ld + c] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kCB * kCB / 256; ++u) {
    const int e = static_cast<int>(threadIdx.x) + 256 * u;
    const int r = e >> 6, c = e & (kCB - 1);
    if (TRANS)
      dst[c][r] = v[u];
    else
      dst[r][c] = v[u];
  }
}

// One level b in {16, 32} of the doubling inverse on the matrix cores:
// for each merge of two b x b diagonal blocks at o1 = 2 m b, o2 = o1 + b,
// T = r[o1:o2, o2:o2+b] x[o2.., o2..], then x[o1:o2, o2:o2+b] = -x[o1:o2, o1:o2] T.
// Entries past the tile's size are zero in r and x, so the full 64 x 64 is
// processed.  Wavefront w takes the 16 x 16 output tile w of the level.
template <int B>
__device__ __forceinline__ void inv_level_mfma(const double (*r)[kCP], double (*x)[kCP], double* t) {
  constexpr int kTiles = (B / 16) * (B / 16);  // output tiles per merge
  constexpr int kMerges = kCB / (2 * B);
  static_assert(kTiles * kMerges <= 4, "at most one tile per wavefront");
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int lr = lane >> 4, lc = lane & 15;
  const bool busy = wv < kTiles * kMerges;
  const int m = wv / kTiles, tile = wv % kTiles;
  const int ti = tile / (B / 16), tj = tile % (B / 16);
  const int o1 = 2 * m * B, o2 = o1 + B;
  double* tm = t + m * B * B;  // T of this merge, B x B row-major
  if (busy) {
    d4_t acc = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < B; kk += 4) {
      const double a = r[o1 + ti * 16 + lc][o2 + kk + lr];
      const double b = x[o2 + kk + lr][o2 + tj * 16 + lc];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) tm[(ti * 16 + lr + 4 * e) * B + tj * 16 + lc] = acc[e];
  }
  __syncthreads();
  if (busy) {
    d4_t acc = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < B; kk += 4) {
      const double a = x[o1 + ti * 16 + lc][o1 + kk + lr];
      const double b = tm[(kk + lr) * B + tj * 16 + lc];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) x[o1 + ti * 16 + lr + 4 * e][o2 + tj * 16 + lc] = -acc[e];
  }
  __syncthreads();
}

// x = r^{-1} for the kb x kb upper triangle r (kb <= kCB, r zero elsewhere),
// in LDS, by doubling: with the inverses of two neighbouring diagonal blocks
// known, the block above the diagonal between them is -X11 (R12 X22).  The
// levels of 1 to 8 columns run on vector units, those of 16 and 32 on the
// matrix cores.  `t` holds at least kCB * kCB / 4 values.  The whole block of
// 256 threads takes part; x is zero below the diagonal and past kb.
__device__ void tri_inv_lds(const double (*r)[kCP], double (*x)[kCP], double* t, int kb) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < kCB * kCB; e += nt) {
    const int i = e / kCB, j = e % kCB;
    x[i][j] = (i == j && i < kb) ? 1.0 / r[i][i] : 0.0;
  }
  __syncthreads();
  for (int sb = 0; sb < 4 && (1 << sb) < kb; ++sb) {
    const int b = 1 << sb, mb = b - 1;
    const int nm = (kb + 2 * b - 1) >> (sb + 1);  // merges (the last may lack a right block)
    // t_m[i][j] = sum_l r[o1 + i][o2 + l] x[o2 + l][o2 + j], l <= j
    for (int e = tid; e < (nm << (2 * sb)); e += nt) {
      const int m = e >> (2 * sb), i = (e >> sb) & mb, j = e & mb;
      const int o1 = (2 * m) << sb, o2 = o1 + b;
      if (o2 + j >= kb) continue;
      double s0 = 0.0;
      for (int l = 0; l <= j; ++l) s0 += r[o1 + i][o2 + l] * x[o2 + l][o2 + j];
      t[e] = s0;
    }
    __syncthreads();
    // x[o1 + i][o2 + j] = -sum_l x[o1 + i][o1 + l] t_m[l][j], l >= i
    for (int e = tid; e < (nm << (2 * sb)); e += nt) {
      const int m = e >> (2 * sb), i = (e >> sb) & mb, j = e & mb;
      const int o1 = (2 * m) << sb, o2 = o1 + b;
      if (o2 + j >= kb) continue;
      const double* tm = t + (m << (2 * sb));
      double s0 = 0.0;
      for (int l = i; l < b; ++l) s0 += x[o1 + i][o1 + l] * tm[(l << sb) + j];
      x[o1 + i][o2 + j] = -s0;
    }
    __syncthreads();
  }
  if (kb > 16) inv_level_mfma<16>(r, x, t);
  if (kb > 32) inv_level_mfma<32>(r, x, t);
}

// 1 / x to double precision: the hardware reciprocal estimate refined by two
// Newton steps (each roughly doubles the correct bits).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// Lane `src`'s value of v, in every lane (two 32-bit reads of one lane).
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(bits & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(bits >> 32), src);
  return __hiloint2double(hi, lo);
}

constexpr int kPW = 16;           // panel width of the tile factor
constexpr int kSP = kCP;          // LDS pitch of the scaled panel rows

// Factor the kb x kb tile whose upper triangle thread (g, j) (g = wave,
// j = lane) holds in c[q] = element (4 q + g, j) into rr = R_KK (upper, zero
// elsewhere), in panels of 16 rows.  The unscaled elimination
// a_ij -= a_ki (a_kj / a_kk) runs inside a panel on wavefront 0 alone, with
// lane j holding column j of the panel's rows in registers: the pivot of
// step k comes from the lane that holds it (readlane), the multipliers from
// an LDS copy of row k (one write, broadcast reads), so the chain from one
// column to the next has no block barrier.  The rows of a finished panel,
// scaled by 1 / sqrt(pivot), then update the trailing triangle on the
// matrix cores (rank 16, all four wavefronts).  R's rows are scaled by
// 1 / sqrt(pivot) at the end.  Each column still costs about 650 cycles: the
// LDS round trip, the reciprocal of the pivot and the update that yields the
// next pivot are a chain.
// Elements below the diagonal are updated too and cleared at the end.  `t`
// holds the scaled panel rows (at least kPW * kSP values).  Returns 1 if a
// pivot was not positive (it then counts as 1 and the factorisation goes on).
__device__ int factor_tile_panels(double (&c)[kCB / 4], double (*rr)[kCP], double* t, int kb) {
  __shared__ double piv_of[kCB];
  __shared__ int32_t any_bad;
  __shared__ __align__(16) double rowk[kCB];
  const int tid = threadIdx.x;
  const int j = tid & (kCB - 1), g = __builtin_amdgcn_readfirstlane(tid >> 6);
#pragma unroll
  for (int q = 0; q < kCB / 4; ++q) rr[4 * q + g][j] = c[q];
  if (tid == 0) any_bad = 0;
  __syncthreads();
  for (int p0 = 0; p0 < kb; p0 += kPW) {
    const int np = (kb - p0) < kPW ? kb - p0 : kPW;
    if (g == 0) {
      double a[kPW];
#pragma unroll
      for (int i = 0; i < kPW; ++i) a[i] = rr[p0 + i][j];
      int bad = 0;
      double pv[kPW];
#pragma unroll
      for (int k = 0; k < kPW; ++k) {
        pv[k] = 1.0;
        if (k < np) {
          double piv = lane_bcast(a[k], p0 + k);
          if (!(piv > 0.0)) {
            bad = 1;
            piv = 1.0;
          }
          pv[k] = piv;
          const double rp = recip(piv);
          if (j == 0) piv_of[p0 + k] = piv;
          // row k once to LDS; the panel's multipliers come back as
          // broadcast reads (fewer instructions than one readlane pair each)
          rowk[j] = a[k];
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          double f[kPW];
#pragma unroll
          for (int i = 0; i < kPW; i += 2) {
            const double2 pr = *reinterpret_cast<const double2*>(&rowk[p0 + i]);
            f[i] = pr.x;
            f[i + 1] = pr.y;
          }
#pragma unroll
          for (int i = k + 1; i < kPW; ++i)
            if (i < np) a[i] -= (f[i] * rp) * a[k];
          __builtin_amdgcn_wave_barrier();  // the reads of rowk are done before the next write
        }
      }
      // the panel's rows back, unscaled, and scaled by 1 / sqrt(pivot) for
      // the trailing update
#pragma unroll
      for (int i = 0; i < kPW; ++i)
        if (i < np) {
          rr[p0 + i][j] = a[i];
          t[i * kSP + j] = a[i] * recip(sqrt(pv[i]));
        }
      if (bad && j == 0) any_bad = 1;
    }
    __syncthreads();
    // trailing triangle [p0 + np, kb): a_rc -= sum_i t[i][r] t[i][c], 16 x 16
    // tiles (ti <= tj) on v_mfma_f64_16x16x4f64, one tile per wavefront at a time
    const int pe = p0 + np;
    const int nt = (kb - pe + 15) / 16;
    const int ntiles = nt * (nt + 1) / 2;
    const int lr = j >> 4, lc = j & 15;
    for (int tt = g; tt < ntiles; tt += 4) {
      int ti = 0, rem = tt;
      while (rem >= nt - ti) {
        rem -= nt - ti;
        ++ti;
      }
      const int r0 = pe + 16 * ti, c0 = pe + 16 * (ti + rem);
      d4_t acc = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < kPW; kk += 4) {
        const double av = t[(kk + lr) * kSP + r0 + lc];  // A[m][k] = t[k][r0 + m]
        const double bv = t[(kk + lr) * kSP + c0 + lc];  // B[k][n] = t[k][c0 + n]
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) rr[r0 + lr + 4 * e][c0 + lc] -= acc[e];
    }
    __syncthreads();
  }
  // R_kj = a_kj / sqrt(pivot_k) with a_kj the values at step k; zero below
  // the diagonal and past kb
  for (int e = tid; e < kCB * kCB; e += 256) {
    const int k = e / kCB, jj = e % kCB;
    double v = 0.0;
    if (k < kb && jj < kb && jj >= k) {
      const double rk = sqrt(piv_of[k]);
      v = jj == k ? rk : rr[k][jj] / rk;
    }
    rr[k][jj] = v;
  }
  __syncthreads();
  return any_bad;
}

// Where the factorisation writes R^{-1} (and its transpose), or nulls.
struct InvOut {
  double* X;   // d x d, R^{-1}
  double* XT;  // d x d, R^{-T}
};

// Factor + invert a diagonal tile held in c[] (see factor_tile_panels): writes
// R_KK into R (rows / columns K .. K + kb), its inverse into Kinv (ld kCB)
// and, when asked, into the diagonal block of R^{-1} and R^{-T}.
__device__ void finish_tile(double (&c)[kCB / 4], double* __restrict__ R, int d, int K, double* __restrict__ Kinv,
                            int32_t* __restrict__ bad, double (*rr)[kCP], double (*x)[kCP], double* t, InvOut inv) {
  const int kb = (d - K) < kCB ? (d - K) : kCB;
  const int tid = threadIdx.x;
  const int j = tid & (kCB - 1), g = tid >> 6;
  const int badk = factor_tile_panels(c, rr, t, kb);
  if (badk) atomicOr(bad, 1);
  for (int i = g; i < kb; i += 4)
    if (j >= i && j < kb) R[static_cast<size_t>(K + i) * d + K + j] = rr[i][j];
  tri_inv_lds(rr, x, t, kb);
  for (int i = g; i < kb; i += 4)
    if (j < kb) {
      Kinv[i * kCB + j] = x[i][j];
      if (inv.X != nullptr && j >= i) {
        inv.X[static_cast<size_t>(K + i) * d + K + j] = x[i][j];
        inv.XT[static_cast<size_t>(K + j) * d + K + i] = x[i][j];
      }
    }
}

// Block column K of X = R^{-1} above the diagonal, from X R = I:
//   X[J, K] = -(sum_{M = J .. K-1} X[J, M] R[M, K]) Kinv_K,   J < K,
// which needs only the columns of X before K, the rows of R above block row
// K in column K, and Kinv_K: all known once tile K is factored.  One block
// of 256 threads per J; a, b are 64 x 64 LDS tiles.  Writes X[J, K] and its
// transpose.
__device__ __forceinline__ void inv_column_tile(const double* __restrict__ R, int d, int J, int K, const double* __restrict__ Kinv,
                                InvOut inv, double (*a)[kCP], double (*b)[kCP]) {
  const int J0 = J * kCB, K0 = K * kCB;
  const int kbj = (d - J0) < kCB ? (d - J0) : kCB, kbk = (d - K0) < kCB ? (d - K0) : kCB;
  d4_t acc[2][2];
  zero_acc(acc);
  for (int M = J; M < K; ++M) {
    const int M0 = M * kCB;
    const int kbm = (d - M0) < kCB ? (d - M0) : kCB;
    __syncthreads();
    // a[k][m] = X[J0 + m][M0 + k] (transposed for the A^T B product), b = R[M, K]
    tile_to_lds<true>(a, inv.X + static_cast<size_t>(J0) * d + M0, d, kbj, kbm);
    tile_to_lds<false>(b, R + static_cast<size_t>(M0) * d + K0, d, kbm, kbk);
    __syncthreads();
    mfma_atb64(a, b, acc);
  }
  __syncthreads();
  // a[k][m] = acc[m][k], b = Kinv_K
  for_acc([&](int i, int j, int e, int row, int col) { a[col][row] = acc[i][j][e]; });
  tile_to_lds<false>(b, Kinv + static_cast<size_t>(K) * kCB * kCB, kCB, kbk, kbk);
  __syncthreads();
  zero_acc(acc);
  mfma_atb64(a, b, acc);
  for_acc([&](int i, int j, int e, int row, int col) {
    if (row < kbj && col < kbk) {
      inv.X[static_cast<size_t>(J0 + row) * d + K0 + col] = -acc[i][j][e];
      inv.XT[static_cast<size_t>(K0 + col) * d + J0 + row] = -acc[i][j][e];
    }
  });
}

// First diagonal tile: W[0:kb, 0:kb] -> R_00 and its inverse.
__global__ __launch_bounds__(256) void k_chol_first(const double* __restrict__ W, double* __restrict__ R, int d,
                                                    double* __restrict__ Kinv, int32_t* __restrict__ bad,
                                                    InvOut inv) {
  __shared__ double rr[kCB][kCP];
  __shared__ double x[kCB][kCP];
  __shared__ double t[kPW * kSP > kCB * kCB / 4 ? kPW * kSP : kCB * kCB / 4];
  const int kb = d < kCB ? d : kCB;
  const int tid = threadIdx.x;
  const int j = tid & (kCB - 1), g = tid >> 6;
  double c[kCB / 4];
#pragma unroll
  for (int q = 0; q < kCB / 4; ++q) {
    const int i = 4 * q + g;
    c[q] = (j < kb && i <= j) ? W[static_cast<size_t>(i) * d + j] : 0.0;
  }
  finish_tile(c, R, d, 0, Kinv, bad, rr, x, t, inv);
}

// d <= kCB: the whole factorisation in one block.  The upper triangle of G
// goes straight into the factor's registers, the tile is factored and
// inverted as in k_chol_first, the parts of R, R^{-1} and R^{-T} it leaves
// unwritten are zeroed, and the rank test of k_chol_finish runs on the
// factored diagonal (against G's own diagonal).
__global__ __launch_bounds__(256) void k_chol_small(const double* __restrict__ G, int64_t ldg, int d,
                                                    double* __restrict__ R, double* __restrict__ Kinv, InvOut inv,
                                                    int32_t* __restrict__ status, double rtol) {
  __shared__ double rr[kCB][kCP];
  __shared__ double x[kCB][kCP];
  __shared__ double t[kPW * kSP > kCB * kCB / 4 ? kPW * kSP : kCB * kCB / 4];
  __shared__ int32_t sbad;
  const int tid = threadIdx.x;
  const int j = tid & (kCB - 1), g = tid >> 6;
  if (tid == 0) sbad = 0;
  for (int e = tid; e < d * d; e += 256) {
    const int r = e / d, c = e % d;
    if (c < r) {
      R[e] = 0.0;
      if (inv.X != nullptr) inv.X[e] = 0.0;
    } else if (c > r && inv.X != nullptr) {
      inv.XT[e] = 0.0;
    }
  }
  double c[kCB / 4];
#pragma unroll
  for (int q = 0; q < kCB / 4; ++q) {
    const int i = 4 * q + g;
    c[q] = (j < d && i <= j) ? G[static_cast<size_t>(i) * ldg + j] : 0.0;
  }
  __syncthreads();  // sbad is set before finish_tile may raise it
  finish_tile(c, R, d, 0, Kinv, &sbad, rr, x, t, inv);
  __syncthreads();
  int32_t mine = 0;
  for (int k = tid; k < d; k += 256)
    if (!(rr[k][k] > rtol * sqrt(G[static_cast<size_t>(k) * ldg + k]))) mine = 1;
  if (mine) atomicOr(&sbad, 1);
  __syncthreads();
  if (tid == 0) status[0] = sbad ? 1 : 0;
}

// One step of the blocked Cholesky after block column K is factored (R_KK
// and Kinv_K = R_KK^{-1} known).  Block (ti, tj), ti <= tj, of the trailing
// block triangle, I = K + 1 + ti, J = K + 1 + tj (64-column blocks):
//   P_I = Kinv_K^T W[K, I], P_J = Kinv_K^T W[K, J]     (the rows R[K, I], R[K, J])
//   W[I, J] -= P_I^T P_J                                (on the matrix cores)
// The block of the diagonal tile (I, I) writes R[K, I] = P_I; the block of
// (K + 1, K + 1) then factors the updated tile and inverts it, so the next
// step finds R_{K+1,K+1} and Kinv_{K+1} ready.  W's block row K is only
// read (the solved rows go to R), so blocks may recompute the same P_I.
__global__ __launch_bounds__(256) void k_chol_step(double* __restrict__ W, double* __restrict__ R, int d, int K,
                                                   double* __restrict__ Kinv, int32_t* __restrict__ bad,
                                                   InvOut inv) {
  __shared__ double ki[kCB][kCP];
  __shared__ double pI[kCB][kCP];
  __shared__ double pJ[kCB][kCP];
  __shared__ double t[kPW * kSP > kCB * kCB / 4 ? kPW * kSP : kCB * kCB / 4];
  const int nb = (d + kCB - 1) / kCB;
  const int T = nb - K - 1;
  const int ntrail = T * (T + 1) / 2;
  if (static_cast<int>(blockIdx.x) >= ntrail) {
    // the blocks past the trailing update form block column K of R^{-1}
    inv_column_tile(R, d, static_cast<int>(blockIdx.x) - ntrail, K, Kinv, inv, pI, pJ);
    return;
  }
  int p = blockIdx.x, ti = 0;
  while (p >= T - ti) {
    p -= T - ti;
    ++ti;
  }
  const int tj = ti + p;
  const int r0 = K * kCB, kb = (d - r0) < kCB ? (d - r0) : kCB;
  const int I0 = (K + 1 + ti) * kCB, J0 = (K + 1 + tj) * kCB;
  const bool diag = ti == tj;
  const int tid = threadIdx.x;
  // Kinv_K and the unsolved rows W[K, I], W[K, J] (zero past kb and d)
  tile_to_lds<false>(ki, Kinv + static_cast<size_t>(K) * kCB * kCB, kCB, kb, kb);
  tile_to_lds<false>(pI, W + static_cast<size_t>(r0) * d + I0, d, kb, d - I0);
  if (!diag) tile_to_lds<false>(pJ, W + static_cast<size_t>(r0) * d + J0, d, kb, d - J0);
  __syncthreads();
  d4_t aI[2][2], aJ[2][2];
  zero_acc(aI);
  mfma_atb64(ki, pI, aI);
  if (!diag) {
    zero_acc(aJ);
    mfma_atb64(ki, pJ, aJ);
  }
  __syncthreads();  // every read of the unsolved rows is done
  for_acc([&](int a, int b, int e, int row, int col) { pI[row][col] = aI[a][b][e]; });
  if (!diag) for_acc([&](int a, int b, int e, int row, int col) { pJ[row][col] = aJ[a][b][e]; });
  __syncthreads();
  if (diag) {
    // this block owns column block I: the solved rows R[K, I]
    for (int e = tid; e < kb * kCB; e += 256) {
      const int l = e / kCB, c = e % kCB;
      if (I0 + c < d) R[static_cast<size_t>(r0 + l) * d + I0 + c] = pI[l][c];
    }
  }
  d4_t u[2][2];
  zero_acc(u);
  mfma_atb64(pI, diag ? pI : pJ, u);
  const bool next = diag && ti == 0;
  if (!next) {
    for_acc([&](int a, int b, int e, int row, int col) {
      if (I0 + row < d && J0 + col < d) {
        double* w = W + static_cast<size_t>(I0 + row) * d + J0 + col;
        *w = *w - u[a][b][e];
      }
    });
    return;
  }
  // (K + 1, K + 1): the updated tile goes through LDS (pJ is free) into the
  // factorisation's register layout
  __syncthreads();  // pI is read by every wavefront's update before reuse
  for_acc([&](int a, int b, int e, int row, int col) {
    const double w = (I0 + row < d && I0 + col < d) ? W[static_cast<size_t>(I0 + row) * d + I0 + col] : 0.0;
    pJ[row][col] = w - u[a][b][e];
  });
  __syncthreads();
  const int kb1 = (d - I0) < kCB ? (d - I0) : kCB;
  const int j = tid & (kCB - 1), g = tid >> 6;
  double c[kCB / 4];
#pragma unroll
  for (int q = 0; q < kCB / 4; ++q) {
    const int i = 4 * q + g;
    c[q] = (j < kb1 && i <= j) ? pJ[i][j] : 0.0;
  }
  __syncthreads();
  finish_tile(c, R, d, I0, Kinv + static_cast<size_t>(K + 1) * kCB * kCB, bad, pI, ki, t, inv);
}

// The last block column of R^{-1} (the steps form the others): block J < K.
__global__ __launch_bounds__(256) void k_inv_column(const double* __restrict__ R, int d, int K,
                                                    const double* __restrict__ Kinv, InvOut inv) {
  __shared__ double a[kCB][kCP];
  __shared__ double b[kCB][kCP];
  inv_column_tile(R, d, static_cast<int>(blockIdx.x), K, Kinv, inv, a, b);
}

// status = rank test on the diagonal of R, column by column: R_kk /
// sqrt(G_kk) is the sine of the angle between column k of the factored
// matrix and the span of the columns before it, which does not change when a
// column is scaled.  One block.
__global__ __launch_bounds__(256) void k_chol_finish(const double* __restrict__ R, int d,
                                                     const double* __restrict__ gdiag, const int32_t* __restrict__ bad,
                                                     int32_t* __restrict__ status, double rtol) {
  __shared__ int32_t sbad;
  if (threadIdx.x == 0) sbad = 0;
  __syncthreads();
  int32_t mine = 0;
  for (int k = threadIdx.x; k < d; k += 256) {
    const double r = R[static_cast<size_t>(k) * d + k];
    if (!(r > rtol * sqrt(gdiag[k]))) mine = 1;
  }
  if (mine) atomicOr(&sbad, 1);
  __syncthreads();
  if (threadIdx.x == 0) status[0] = (bad[0] || sbad) ? 1 : 0;
}

// W = upper triangle of G (zero below), R = 0, R^{-1} = R^{-T} = 0 (when
// asked), gdiag = diagonal of G, bad = 0.
__global__ void k_copy_upper(const double* __restrict__ G, int64_t ldg, int d, double* __restrict__ W,
                             double* __restrict__ R, InvOut inv, double* __restrict__ gdiag,
                             int32_t* __restrict__ bad) {
  for (int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; idx < static_cast<int64_t>(d) * d;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int i = static_cast<int>(idx / d), j = static_cast<int>(idx % d);
    const double g = G[static_cast<size_t>(i) * ldg + j];
    W[idx] = j >= i ? g : 0.0;
    R[idx] = 0.0;
    if (inv.X != nullptr) {
      inv.X[idx] = 0.0;
      inv.XT[idx] = 0.0;
    }
    if (i == j) gdiag[i] = g;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) bad[0] = 0;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inverses of the diagonal kCB x kCB blocks of R, one block of threads per
// diagonal block, written into Rinv; the rest of Rinv is zeroed here.
__global__ __launch_bounds__(256) void k_trinv_diag(const double* __restrict__ R, int d, double* __restrict__ Rinv) {
  __shared__ double rr[kCB][kCB + 1];
  __shared__ double x[kCB][kCB + 1];
  __shared__ double t[kCB * kCB / 4];
  const int K = blockIdx.x * kCB;
  const int kb = (d - K) < kCB ? (d - K) : kCB;
  for (int e = threadIdx.x; e < kCB * (kCB + 1); e += 256) {
    const int i = e / (kCB + 1), j = e % (kCB + 1);
    rr[i][j] = (i < kb && j < kb && j >= i) ? R[static_cast<size_t>(K + i) * d + K + j] : 0.0;
  }
  __syncthreads();
  tri_inv_lds(rr, x, t, kb);
  // this block writes rows K .. K + kb of Rinv: x on the diagonal block, zero elsewhere
  for (int64_t e = threadIdx.x; e < static_cast<int64_t>(kb) * d; e += 256) {
    const int i = static_cast<int>(e / d), j = static_cast<int>(e % d);
    Rinv[static_cast<size_t>(K + i) * d + j] = (j >= K && j < K + kb) ? x[i][j - K] : 0.0;
  }
}

// The same first level from inverses already at hand (those run_cholesky
// keeps, computed by tri_inv_lds from the same block of R): block K of
// Rinv's rows gets Kinv_K on the diagonal and zero elsewhere.
__global__ __launch_bounds__(256) void k_trinv_place(const double* __restrict__ Kinv, int d,
                                                     double* __restrict__ Rinv) {
  const int K = blockIdx.x * kCB;
  const int kb = (d - K) < kCB ? (d - K) : kCB;
  const double* KK = Kinv + static_cast<size_t>(blockIdx.x) * kCB * kCB;
  // the kb x kb block: a fixed count of loads per thread, all in flight
  double v[kCB * kCB / 256];
#pragma unroll
  for (int u = 0; u < kCB * kCB / 256; ++u) {
    const int e = u * 256 + threadIdx.x, i = e / kCB, j = e % kCB;
    v[u] = (i < kb && j < kb) ? KK[e] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kCB * kCB / 256; ++u) {
    const int e = u * 256 + threadIdx.x, i = e / kCB, j = e % kCB;
    if (i < kb && j < kb) Rinv[static_cast<size_t>(K + i) * d + K + j] = v[u];
  }
  // zeros elsewhere in these rows
  for (int i = 0; i < kb; ++i) {
    double* row = Rinv + static_cast<size_t>(K + i) * d;
    for (int j = threadIdx.x; j < d; j += 256)
      if (j < K || j >= K + kb) row[j] = 0.0;
  }
}

// One 64 x 64 tile of C = alpha A B (row-major, M x N, inner dimension K) on
// the float64 matrix cores; A, B, C point at the sub-blocks.
__device__ void gemm_tile64(const double* __restrict__ A, int lda, const double* __restrict__ B, int ldb,
                            double* __restrict__ C, int ldc, int M, int N, int K, int i0, int j0, double alpha,
                            double (*As)[64], double (*Bs)[64]) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int wi = wv >> 1, wj = wv & 1;
  const int lr = lane >> 4, lc = lane & 15;
  d4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 16) {
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int kk = e / 64, c = e % 64;
      As[kk][c] = (i0 + c < M && k0 + kk < K) ? A[static_cast<size_t>(i0 + c) * lda + k0 + kk] : 0.0;
      Bs[kk][c] = (k0 + kk < K && j0 + c < N) ? B[static_cast<size_t>(k0 + kk) * ldb + j0 + c] : 0.0;
    }
    __syncthreads();
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
  // element e of lane l: row (l / 16) + 4 e, column l % 16 of each 16 x 16 block
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = i0 + wi * 32 + a * 16 + lr + 4 * e, col = j0 + wj * 32 + b * 16 + lc;
        if (row < M && col < N) C[static_cast<size_t>(row) * ldc + col] = alpha * acc[a][b][e];
      }
}

// One level of the doubling for R^{-1}: for merge z of blocks of size b,
// o1 = 2 z b, o2 = o1 + b, o3 = min(o2 + b, d):
//   STEP 0: T[o1:o2, o2:o3] = R[o1:o2, o2:o3] Rinv[o2:o3, o2:o3]
//   STEP 1: Rinv[o1:o2, o2:o3] = -Rinv[o1:o2, o1:o2] T[o1:o2, o2:o3]
// (T is a d x d scratch used at the same positions).  Tiles of 64 x 64 over
// blockIdx.x, merges over blockIdx.y.
template <int STEP>
__global__ __launch_bounds__(256) void k_trinv_merge(const double* __restrict__ R, double* __restrict__ Rinv,
                                                     double* __restrict__ T, int d, int b) {
  __shared__ double As[16][64], Bs[16][64];
  const int o1 = 2 * blockIdx.y * b, o2 = o1 + b;
  if (o2 >= d) return;
  const int o3 = (o2 + b) < d ? o2 + b : d;
  const int b2 = o3 - o2;
  const int tn = (b2 + 63) / 64;
  const int i0 = (blockIdx.x / tn) * 64, j0 = (blockIdx.x % tn) * 64;
  if (i0 >= b) return;
  const size_t off12 = static_cast<size_t>(o1) * d + o2;
  if (STEP == 0) {
    gemm_tile64(R + off12, d, Rinv + static_cast<size_t>(o2) * d + o2, d, T + off12, d, b, b2, b2, i0, j0, 1.0, As,
                Bs);
  } else {
    gemm_tile64(Rinv + static_cast<size_t>(o1) * d + o1, d, T + off12, d, Rinv + off12, d, b, b2, b, i0, j0, -1.0,
                As, Bs);
  }
}

__global__ void k_transpose(const double* __restrict__ X, int d, double* __restrict__ Y) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int i = by + k, j = bx + threadIdx.x;
    tile[k][threadIdx.x] = (i < d && j < d) ? X[static_cast<size_t>(i) * d + j] : 0.0;
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int i = bx + k, j = by + threadIdx.x;
    if (i < d && j < d) Y[static_cast<size_t>(i) * d + j] = tile[threadIdx.x][k];
  }
}

// y = M x, one wavefront per row of the d x d row-major M.
__global__ __launch_bounds__(256) void k_gemv(const double* __restrict__ M, int d, const double* __restrict__ x,
                                              double* __restrict__ y) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int row = blockIdx.x * 4 + wid;
  if (row >= d) return;
  const double* m = M + static_cast<size_t>(row) * d;
  double s = 0.0;
  for (int k = lane; k < d; k += kWave) s += m[k] * x[k];
  s = wave_sum(s);
  if (lane == 0) y[row] = s;
}

// T = R^{-1} P (d x d upper times d x k), float64 sums rounded to float32.
__global__ void k_rinv_times(const double* __restrict__ Rinv, int d, const double* __restrict__ P, int k,
                             float* __restrict__ T) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= static_cast<int64_t>(d) * k) return;
  const int i = static_cast<int>(idx / k), q = static_cast<int>(idx % k);
  double s = 0.0;
  for (int j = i; j < d; ++j) s += Rinv[static_cast<size_t>(i) * d + j] * P[static_cast<size_t>(j) * k + q];
  T[idx] = static_cast<float>(s);
}

__global__ void k_f64_to_f32(const double* __restrict__ in, float* __restrict__ out, int64_t count) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[i] = static_cast<float>(in[i]);
}

struct GramShape {
  int T, P;
  int Sd, So;            // row splits of the diagonal / off-diagonal tiles
  int64_t rpd, rpo;      // rows per split
};

// Tiles of the d x d Gram (upper triangle of tile pairs) and row splits: each
// of the two launches (diagonal tiles, off-diagonal pairs) has about one block
// per compute unit, each taking a run of whole kGK-row strips.
GramShape gram_shape(int64_t m, int64_t d) {
  GramShape g;
  g.T = static_cast<int>(div_up(d > 0 ? d : 1, kGT));
  g.P = g.T * (g.T + 1) / 2;
  const int64_t max_split = div_up(m > 0 ? m : 1, 4 * kGK);
  auto split = [&](int tiles, int& S, int64_t& rps) {
    int64_t x = tiles > 0 ? 256 / tiles : 1;
    if (x > max_split) x = max_split;
    if (x < 1) x = 1;
    rps = div_up(div_up(m > 0 ? m : 1, x), kGK) * kGK;
    S = static_cast<int>(div_up(m > 0 ? m : 1, rps));
  };
  split(g.T, g.Sd, g.rpd);
  split(g.P - g.T, g.So, g.rpo);
  if (g.P == g.T) g.So = 0;
  return g;
}

// Splits of the small-Gram kernel: whole chunks of kSK rows, at most cap
// (<= 256).
int small_splits(int64_t m, int64_t& rps, int cap = 256) {
  const int64_t mm = m > 0 ? m : 1;
  int64_t x = div_up(mm, kSK);
  if (x > cap) x = cap;
  rps = div_up(div_up(mm, x), kSK) * kSK;
  return static_cast<int>(div_up(mm, rps));
}

size_t gram_bytes(const GramShape& g, int64_t m, int64_t d) {
  int S = g.Sd > g.So ? g.Sd : g.So;
  if (d <= 64) {
    // room for the small-Gram kernel's splits as well; their count is at
    // most min(256, ceil(m / kSK)), which grows with m, so a workspace sized
    // for m rows also serves every shorter matrix
    const int64_t x = div_up(m > 0 ? m : 1, kSK);
    const int Ss = static_cast<int>(x < 256 ? x : 256);
    S = Ss > S ? Ss : S;
  }
  return (static_cast<size_t>(S) * g.P * kGT * kGT + static_cast<size_t>(g.Sd) * (g.T * kGT + 1)) * sizeof(double) +
         512;
}

}  // namespace

size_t gram_ws_bytes(int64_t m, int64_t dd) {
  // dd = d (no v) or d + 1 (with v): size for either reading of dd
  size_t need = 0;
  for (int64_t d : {dd, dd - 1}) {
    if (d < 1) continue;
    const size_t b = gram_bytes(gram_shape(m, d), m, d);
    need = b > need ? b : need;
  }
  return need;
}

namespace {

// A second stream on the current device (default priority, created once per
// host thread and device) with the two events that fork work onto it from a
// caller's stream and join it back.
struct SideStream {
  int device = -1;
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

SideStream* side_stream() {
  thread_local SideStream side[16];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) return nullptr;
  SideStream& x = side[dev];
  if (x.s == nullptr) {
    if (hipStreamCreateWithFlags(&x.s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&x.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&x.join, hipEventDisableTiming) != hipSuccess) {
      x.s = nullptr;
      return nullptr;
    }
    x.device = dev;
  }
  return &x;
}

}  // namespace

namespace {

// The small-Gram launch (d columns of M, d + 1 <= 64 with v, d <= 64
// without): its splits go to partial.
int32_t launch_gram_small(const void* M, int32_t dtype, int64_t ld, const void* v, int v_f64, int64_t m, int64_t d,
                          double* partial, int* splits, hipStream_t s, int cap = 256, int count = 1,
                          int64_t mstride = 0, int64_t pstride = 0) {
  int64_t rps;
  const int S = small_splits(m, rps, cap);
  const int dp = static_cast<int>(v != nullptr ? d + 1 : d);  // columns of the product
  auto launch = [&](auto tag) -> int32_t {
    using TI = decltype(tag);
    const TI* Mt = static_cast<const TI*>(M);
    const bool vec = (reinterpret_cast<uintptr_t>(M) % 16 == 0) && ((ld * sizeof(TI)) % 16 == 0) && (d % 4 == 0) &&
                     ((mstride * static_cast<int64_t>(sizeof(TI))) % 16 == 0);
    const dim3 g(S, count), b(kGThreads);
    if (v != nullptr) {
      if (vec)
        hipLaunchKernelGGL((k_gram_small<TI, true, true>), g, b, 0, s, Mt, ld, v, v_f64, m, dp, rps, partial,
                           mstride, pstride);
      else
        hipLaunchKernelGGL((k_gram_small<TI, false, true>), g, b, 0, s, Mt, ld, v, v_f64, m, dp, rps, partial,
                           mstride, pstride);
    } else {
      if (vec)
        hipLaunchKernelGGL((k_gram_small<TI, true, false>), g, b, 0, s, Mt, ld, v, v_f64, m, dp, rps, partial,
                           mstride, pstride);
      else
        hipLaunchKernelGGL((k_gram_small<TI, false, false>), g, b, 0, s, Mt, ld, v, v_f64, m, dp, rps, partial,
                           mstride, pstride);
    }
    SKLS_CHECK_LAUNCH();
    return SKLS_OK;
  };
  *splits = S;
  switch (dtype) {
    case SKLS_F64: return launch(double{});
    case SKLS_F32: return launch(float{});
    case SKLS_BF16: return launch(bf16_t{});
    default: set_error("gram: bad dtype"); return SKLS_ERR_DTYPE;
  }
}

}  // namespace

int32_t run_gram_small_partials(const void* M, int32_t dtype, int64_t ld, int64_t m, int64_t d, int max_splits,
                                void* ws, size_t ws_bytes, int* splits, int* pitch, hipStream_t s) {
  if (d < 1 || d > 64 || max_splits < 1 || max_splits > 256) {
    set_error("small Gram: need 1 <= d <= 64 and 1 <= max_splits <= 256");
    return SKLS_ERR_SHAPE;
  }
  if (ws == nullptr || ws_bytes < gram_bytes(gram_shape(m, d), m, d)) {
    set_error("gram workspace too small");
    return SKLS_ERR_WORKSPACE;
  }
  *pitch = kGT;
  PhaseTimer pt("gram", s);
  return launch_gram_small(M, dtype, ld, nullptr, 0, m, d, static_cast<double*>(ws), splits, s, max_splits);
}

int64_t gram_small_split_doubles() { return static_cast<int64_t>(kGT) * kGT; }

int32_t run_gram_small_partials_many(const float* M, int count, int64_t mstride, int64_t m, int64_t d,
                                     int max_splits, double* partial, int64_t pstride, int* splits, int* pitch,
                                     hipStream_t s) {
  int64_t rps;
  if (d < 1 || d > 64 || count < 1 || max_splits < 1 || max_splits > 256 ||
      pstride < static_cast<int64_t>(small_splits(m, rps, max_splits)) * kGT * kGT) {
    set_error("small Gram of several matrices: bad shape or split room");
    return SKLS_ERR_SHAPE;
  }
  *pitch = kGT;
  PhaseTimer pt("gram", s);
  return launch_gram_small(M, SKLS_F32, d, nullptr, 0, m, d, partial, splits, s, max_splits, count, mstride,
                           pstride);
}

int32_t run_gram(const void* M, int32_t dtype, int64_t ld, const void* v, int32_t v_dtype, int64_t m, int64_t d,
                 double* G, void* ws, size_t ws_bytes, hipStream_t s) {
  const GramShape g = gram_shape(m, d);
  if (ws_bytes < gram_bytes(g, m, d) || ws == nullptr) {
    set_error("gram workspace too small");
    return SKLS_ERR_WORKSPACE;
  }
  Arena ar(ws, ws_bytes);
  // v rides along as column d when it is in the staging precision of M
  const bool small_v = v != nullptr && d + 1 <= 64 &&
                       (dtype == SKLS_F64 ? v_dtype == SKLS_F64 : v_dtype == SKLS_F32);
  if ((v == nullptr && d <= 64) || small_v) {
    PhaseTimer pt("gram", s);
    int S = 0;
    SKLS_TRY(launch_gram_small(M, dtype, ld, v, v_dtype == SKLS_F64 ? 1 : 0, m, d, static_cast<double*>(ws), &S, s));
    const int dp = static_cast<int>(v != nullptr ? d + 1 : d);
    hipLaunchKernelGGL(k_gram_reduce, dim3(2, kGT * kGT / 256), dim3(256), 0, s, static_cast<const double*>(ws),
                       static_cast<const double*>(ws), 1, S, 0, 1, dp, 0, G);
    SKLS_CHECK_LAUNCH();
    return SKLS_OK;
  }
  const int S = g.Sd > g.So ? g.Sd : g.So;
  double* partial = ar.take<double>(static_cast<size_t>(S) * g.P * kGT * kGT);
  double* partial_v = ar.take<double>(static_cast<size_t>(g.Sd) * (g.T * kGT + 1));  // M^T v parts, then v^T v parts
  const int v_f64 = v_dtype == SKLS_F64 ? 1 : 0;
  const int di = static_cast<int>(d);
  PhaseTimer pt("gram", s);
  // On large inputs the off-diagonal tiles run on a side stream beside the
  // diagonal ones (the two launches are independent), joined before the
  // reduction; on small ones the fork and join across queues cost more than
  // the overlap gains.
  SideStream* side = (g.So > 0 && m * d >= (int64_t(1) << 24)) ? side_stream() : nullptr;
  hipStream_t so = s;
  if (side != nullptr) {
    SKLS_TRY_HIP(hipEventRecord(side->fork, s));
    SKLS_TRY_HIP(hipStreamWaitEvent(side->s, side->fork, 0));
    so = side->s;
  }
  auto launch = [&](auto tag, auto vec) -> int32_t {
    using TI = decltype(tag);
    constexpr bool VEC = decltype(vec)::value;
    const TI* Mt = static_cast<const TI*>(M);
    if (v != nullptr) {
      hipLaunchKernelGGL((k_gram_partial<TI, VEC, true, true>), dim3(g.T, g.Sd), dim3(kGThreads), 0, s, Mt, ld, v,
                         v_f64, m, di, g.T, g.P, g.rpd, partial, partial_v);
    } else {
      hipLaunchKernelGGL((k_gram_partial<TI, VEC, true, false>), dim3(g.T, g.Sd), dim3(kGThreads), 0, s, Mt, ld, v,
                         v_f64, m, di, g.T, g.P, g.rpd, partial, partial_v);
    }
    SKLS_CHECK_LAUNCH();
    if (g.So > 0) {
      hipLaunchKernelGGL((k_gram_partial<TI, VEC, false, false>), dim3(g.P - g.T, g.So), dim3(kGThreads), 0, so, Mt,
                         ld, v, v_f64, m, di, g.T, g.P, g.rpo, partial, partial_v);
      SKLS_CHECK_LAUNCH();
    }
    return SKLS_OK;
  };
  auto with_vec = [&](auto tag) -> int32_t {
    using TI = decltype(tag);
    const bool vec = (reinterpret_cast<uintptr_t>(M) % 16 == 0) && ((ld * sizeof(TI)) % 16 == 0) && (d % 4 == 0);
    return vec ? launch(tag, std::true_type{}) : launch(tag, std::false_type{});
  };
  int32_t st;
  switch (dtype) {
    case SKLS_F64: st = with_vec(double{}); break;
    case SKLS_F32: st = with_vec(float{}); break;
    case SKLS_BF16: st = with_vec(bf16_t{}); break;
    default: set_error("gram: bad dtype"); return SKLS_ERR_DTYPE;
  }
  if (side != nullptr) {
    // join even after a failed launch, so that the side stream never runs
    // past the caller's stream
    const hipError_t e1 = hipEventRecord(side->join, side->s);
    const hipError_t e2 = hipStreamWaitEvent(s, side->join, 0);
    if (st == SKLS_OK && (e1 != hipSuccess || e2 != hipSuccess)) {
      set_error("gram: joining the side stream failed");
      return SKLS_ERR_DEVICE;
    }
  }
  if (st != SKLS_OK) return st;
  hipLaunchKernelGGL(k_gram_reduce, dim3(g.P + 1, kGT * kGT / 256), dim3(256), 0, s, partial, partial_v, g.P, g.Sd,
                     g.So, g.T, di, v ? 1 : 0, G);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

size_t cholesky_scratch_doubles(int64_t d) {
  return static_cast<size_t>(d * d) + static_cast<size_t>(div_up(d, kCB)) * kCB * kCB + static_cast<size_t>(d) + 8;
}

const double* cholesky_block_inverses(const double* scratch, int64_t d) { return scratch + d * d; }

int32_t run_cholesky(const double* G, int64_t ldg, int64_t d, double* R, double* Rinv, double* RinvT,
                     int32_t* status, double* scratch, hipStream_t s) {
  // Threshold: R_kk^2 = G_kk - sum_i R_ik^2 is formed with an error of
  // about d * eps * G_kk, so a Gram-based factor cannot resolve R_kk below
  // about sqrt(d * eps) * sqrt(G_kk); treat that as numerical rank
  // deficiency (a per-column test: scaling a column scales both sides).
  const double rtol = 4.0 * std::sqrt(static_cast<double>(d) * 2.220446049250313e-16);
  PhaseTimer pt("cholesky", s);
  // scratch: W [d*d] | inverses of the diagonal blocks [nb * kCB*kCB] |
  // diagonal of G [d] | bad flag
  double* W = scratch;
  double* Kinv = scratch + d * d;
  double* gdiag = Kinv + div_up(d, kCB) * kCB * kCB;
  int32_t* bad = reinterpret_cast<int32_t*>(gdiag + d);
  const InvOut inv{Rinv, Rinv != nullptr ? RinvT : nullptr};
  const int di = static_cast<int>(d);
  if (d <= kCB) {
    hipLaunchKernelGGL(k_chol_small, dim3(1), dim3(256), 0, s, G, ldg, di, R, Kinv, inv, status, rtol);
    SKLS_CHECK_LAUNCH();
    return SKLS_OK;
  }
  const unsigned g = static_cast<unsigned>(div_up(d * d, 256) < 4096 ? div_up(d * d, 256) : 4096);
  hipLaunchKernelGGL(k_copy_upper, dim3(g), dim3(256), 0, s, G, ldg, di, W, R, inv, gdiag, bad);
  SKLS_CHECK_LAUNCH();
  // block column 0, then one launch per step: the trailing update of step K,
  // the factorisation of diagonal tile K + 1 and (when asked) block column K
  // of R^{-1}; the last column of R^{-1} after the steps
  hipLaunchKernelGGL(k_chol_first, dim3(1), dim3(256), 0, s, W, R, di, Kinv, bad, inv);
  SKLS_CHECK_LAUNCH();
  const int nb = static_cast<int>(div_up(d, kCB));
  for (int K = 0; K + 1 < nb; ++K) {
    const int T = nb - K - 1;
    const int extra = inv.X != nullptr ? K : 0;
    hipLaunchKernelGGL(k_chol_step, dim3(T * (T + 1) / 2 + extra), dim3(256), 0, s, W, R, di, K, Kinv, bad, inv);
    SKLS_CHECK_LAUNCH();
  }
  if (inv.X != nullptr && nb > 1) {
    hipLaunchKernelGGL(k_inv_column, dim3(nb - 1), dim3(256), 0, s, R, di, nb - 1, Kinv, inv);
    SKLS_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_chol_finish, dim3(1), dim3(256), 0, s, R, di, gdiag, bad, status, rtol);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

// R^{-1} by doubling over diagonal blocks: inverses of the kCB-blocks (or
// diag_inv, the ones run_cholesky kept for this R), then
// levels b = kCB, 2 kCB, ... each merging neighbouring blocks with two
// products on the matrix cores.  RinvT (d x d) serves as the product scratch
// before it receives the transpose.
int32_t run_trinv(const double* R, int64_t d, double* Rinv, double* RinvT, hipStream_t s, const double* diag_inv) {
  PhaseTimer pt("trinv", s);
  const int di = static_cast<int>(d);
  const int nb = static_cast<int>(div_up(d, kCB));
  if (diag_inv != nullptr) {
    hipLaunchKernelGGL(k_trinv_place, dim3(nb), dim3(256), 0, s, diag_inv, di, Rinv);
  } else {
    hipLaunchKernelGGL(k_trinv_diag, dim3(nb), dim3(256), 0, s, R, di, Rinv);
  }
  SKLS_CHECK_LAUNCH();
  for (int b = kCB; b < di; b *= 2) {
    const unsigned merges = static_cast<unsigned>(div_up(d, 2 * static_cast<int64_t>(b)));
    const unsigned tiles = static_cast<unsigned>(div_up(b, 64) * div_up(b, 64));
    hipLaunchKernelGGL(k_trinv_merge<0>, dim3(tiles, merges), dim3(256), 0, s, R, Rinv, RinvT, di, b);
    SKLS_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_trinv_merge<1>, dim3(tiles, merges), dim3(256), 0, s, R, Rinv, RinvT, di, b);
    SKLS_CHECK_LAUNCH();
  }
  const unsigned g = static_cast<unsigned>(div_up(d, 32));
  hipLaunchKernelGGL(k_transpose, dim3(g, g), dim3(32, 8), 0, s, Rinv, di, RinvT);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t run_gemv(const double* M, int64_t d, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_gemv, dim3(static_cast<unsigned>(div_up(d, 4))), dim3(256), 0, s, M, static_cast<int>(d), x,
                     y);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t run_solve_from_gram(const double* Rinv, const double* RinvT, const double* c, int64_t d, double* x,
                            double* tmp, hipStream_t s) {
  SKLS_TRY(run_gemv(RinvT, d, c, tmp, s));
  return run_gemv(Rinv, d, tmp, x, s);
}

int32_t run_rinv_times(const double* Rinv, int64_t d, const double* P, int32_t k, float* T, hipStream_t s) {
  hipLaunchKernelGGL(k_rinv_times, dim3(static_cast<unsigned>(div_up(d * k, 256))), dim3(256), 0, s, Rinv,
                     static_cast<int>(d), P, k, T);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

int32_t run_convert_f64_to_f32(const double* in, float* out, int64_t count, hipStream_t s) {
  if (count == 0) return SKLS_OK;
  int64_t g = div_up(count, 256);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_f64_to_f32, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, in, out, count);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

}  // namespace skls
