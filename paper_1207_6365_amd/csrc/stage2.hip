// Optional second sketch stage: Pi1 = F S with F an m x t matrix of random
// signs / sqrt(m) (a dense Johnson-Lindenstrauss map), applied to the sparse
// embedding's output so that the factorisation works on m x d rows instead
// of t x d.  Section 6 (the leverage-score algorithm) composes the sparse
// embedding with a fast Johnson-Lindenstrauss transform in the same way, and
// the composition facts of Section 8 say the product keeps the embedding
// property.  Random signs stand in for the fast transform: they are exact in
// bf16, so the product runs on the matrix cores.
//
// F's entries are never stored.  Entry (i, r) is -1 / sqrt(m) when bit
// b(r mod 64) of SplitMix64 output i * W + floor(r / 64) of the stream
// seed ^ "stage2si" is set (W = ceil(t / 64)), else +1 / sqrt(m), where
// b(c) = 32 floor(c / 32) + 16 (c mod 2) + 15 - floor((c mod 32) / 2): a
// fixed order of the word's 64 bits that puts the signs of two neighbouring
// rows r, r + 1 at bits 15 and 31 of one 32-bit half shifted left, which are
// the sign bits of a pair of bf16 values.
//
// F (S A) runs on the bf16 matrix cores (v_mfma_f32_32x32x16_bf16): the
// signs are exact in bf16; S A is rounded to float32 and then to bf16 (round
// to nearest even each) on its way into LDS; the products accumulate in
// float32 per split of the t rows and the splits are summed in float64.
// F (S b) is formed in float64 from S b as given.
#include <cmath>

#include "kernels.hpp"
#include "profile.hpp"

namespace skls {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr uint64_t kStageSalt = 0x7374616765327369ull;  // "stage2si"
constexpr int kFM = 256;     // block tile: rows of F
constexpr int kFN = 128;     // block tile: columns of S A
constexpr int kFK = 64;      // rows of S A staged per step (one sign word per row of F)
constexpr int kFP = kFK + 8;  // LDS pitch (bf16) of a staged column

// Work index of dispatch index g of G: blocks go to the eight XCDs in turn,
// so consecutive work indices (the row tiles of F that read the same rows
// and columns of S A) are placed on one XCD and share its L2.
__device__ __forceinline__ int stage_xcd_major(int g, int G) {
  constexpr int kXcd = 8;
  if (G % kXcd != 0) return g;
  return (g % kXcd) * (G / kXcd) + g / kXcd;
}

__device__ __forceinline__ __bf16 to_bf16(float x) { return static_cast<__bf16>(x); }

// Sign pair j (0..3) of the 8-element fragment for rows c, c + 1 of a sign
// word: bits 15 and 31 of the word's 32-bit half `piece` shifted left by the
// pair's position, inserted into the bf16 pair (1.0, 1.0).
__device__ __forceinline__ uint32_t sign_pair(uint32_t shifted) {
  return (shifted & 0x80008000u) | 0x3F803F80u;
}

// part[z] (m x d, float32) = F'[:, rows of split z] (S A)[rows of split z, :]
// with F' = sqrt(m) F (entries +-1).  Block: a 256 x 128 output tile and
// one split of the t rows; wave (wi, wj) owns rows 128 wi .. + 127 and
// columns 64 wj .. + 63 as 4 x 2 MFMA tiles of 32 x 32.  MFMA lane layout
// (32x32x16 bf16): lane l holds A[l % 32][8 (l / 32) + u] and
// B[8 (l / 32) + u][l % 32], u = 0..7; accumulator element e is row
// 8 (e / 4) + 4 (l / 32) + e % 4, column l % 32.  Staging: thread
// (n = tid % 128, h = tid / 128) reads rows k0 + 32 h .. + 31 of column
// j0 + n (each load instruction reads 64 consecutive columns of one row)
// and writes them as four 8-element vectors of column n into one of two
// LDS buffers, so one barrier per 64-row step suffices.
template <typename TS>
__global__ __launch_bounds__(256) void k_fsa(int m, int d, int64_t t, int64_t W, int64_t kc, int tiles_m,
                                             int tiles_n, uint64_t seed, const TS* __restrict__ SA,
                                             float* __restrict__ part) {
  __shared__ __align__(16) __bf16 Bs[2][kFN][kFP];  // [buffer][column][row k]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, wi = wv >> 1, wj = wv & 1;
  const int lr = lane & 31, lh = lane >> 5;
  const int g = stage_xcd_major(blockIdx.x, gridDim.x);
  const int tm = g % tiles_m, tn = (g / tiles_m) % tiles_n, z = g / (tiles_m * tiles_n);
  const int i0 = tm * kFM, j0 = tn * kFN;
  const int64_t kb = static_cast<int64_t>(z) * kc;
  const int64_t ke = (kb + kc) < t ? kb + kc : t;
  const uint64_t sseed = seed ^ kStageSalt;

  // staging role: column j0 + sn, rows 32 sh .. 32 sh + 31 of each step (sh
  // is the same for the whole wavefront)
  const int sn = threadIdx.x & (kFN - 1);
  const int sh = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 7);
  const bool col_ok = j0 + sn < d;
  const int scol = col_ok ? j0 + sn : d - 1;  // a valid column for every lane
  float v[32];
  // Row r0 + u for u <= last, zero beyond it; the row base is uniform over
  // the wavefront, so each load is a scalar address plus the lane's column.
  auto load_step = [&](int64_t k0) {
    const int64_t r0 = k0 + 32 * sh;
    const int64_t lim = ke - 1 - r0;
    const int last = lim < 31 ? static_cast<int>(lim) : 31;
    // every load is issued (its address is valid); rows past the split and
    // clamped columns are cleared with a bit mask afterwards, so the loads
    // stay unconditional and all 32 are in flight together
    const uint32_t colmask = col_ok ? 0xFFFFFFFFu : 0u;
    if (last == 31) {  // a full step (every step but the last of a ragged split)
      const TS* row = SA + r0 * d;
#pragma unroll
      for (int u = 0; u < 32; ++u, row += d)
        v[u] = __uint_as_float(__float_as_uint(static_cast<float>(row[scol])) & colmask);
    } else {
#pragma unroll
      for (int u = 0; u < 32; ++u) {
        const TS* row = SA + (r0 + (u < last ? u : last)) * d;
        const float x = static_cast<float>(row[scol]);
        v[u] = __uint_as_float(__float_as_uint(x) & (u <= last ? colmask : 0u));
      }
    }
  };

  f32x16 acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[a][b][e] = 0.0f;

  if (kb < ke) load_step(kb);
  int buf = 0;
  for (int64_t k0 = kb; k0 < ke; k0 += kFK, buf ^= 1) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      bf16x8 w;
#pragma unroll
      for (int u = 0; u < 8; ++u) w[u] = to_bf16(v[8 * q + u]);
      *reinterpret_cast<bf16x8*>(&Bs[buf][sn][32 * sh + 8 * q]) = w;
    }
    // Bs[buf] is complete; every wave is also past its reads of Bs[buf ^ 1]
    // from the previous step, which the next step overwrites
    __syncthreads();
    if (k0 + kFK < ke) load_step(k0 + kFK);  // in flight during the products below
    // this lane's sign words, pre-shifted by its half's position (4 pairs)
    uint32_t pc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int row = i0 + wi * 128 + a * 32 + lr;
      const uint64_t zw =
          row < m ? splitmix64(sseed, static_cast<uint64_t>(row) * W + static_cast<uint64_t>(k0 >> 6)) : 0;
      pc[a][0] = static_cast<uint32_t>(zw) << (4 * lh);
      pc[a][1] = static_cast<uint32_t>(zw >> 32) << (4 * lh);
    }
#pragma unroll
    for (int s = 0; s < kFK / 16; ++s) {
      bf16x8 bf[2];
#pragma unroll
      for (int b = 0; b < 2; ++b)
        bf[b] = *reinterpret_cast<const bf16x8*>(&Bs[buf][wj * 64 + b * 32 + lr][16 * s + 8 * lh]);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        u32x4 f;
#pragma unroll
        for (int j = 0; j < 4; ++j) f[j] = sign_pair(pc[a][s >> 1] << (8 * (s & 1) + j));
        const bf16x8 af = __builtin_bit_cast(bf16x8, f);
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, bf[b], acc[a][b], 0, 0, 0);
      }
    }
  }
  float* out = part + static_cast<size_t>(z) * m * d;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = i0 + wi * 128 + a * 32 + 8 * (e / 4) + 4 * lh + (e % 4);
        const int col = j0 + wj * 64 + b * 32 + lr;
        if (row < m && col < d) out[static_cast<size_t>(row) * d + col] = acc[a][b][e];
      }
}

// FSA = scale * (sum over the splits of part), in float64.
__global__ void k_fsa_reduce(int64_t count, int splits, const float* __restrict__ part, double scale,
                             double* __restrict__ FSA) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < count;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double s = 0.0;
    for (int z = 0; z < splits; ++z) s += static_cast<double>(part[static_cast<size_t>(z) * count + e]);
    FSA[e] = scale * s;
  }
}

// F' (S b) partial sums: block (g, c) covers rows 64 g .. 64 g + 63 of F and
// sign words 64 c .. 64 c + 63 (rows 4096 c .. of S b).  The block stages
// that piece of S b in LDS as float64 (word w at w * kWP doubles); lane l
// of every wavefront owns word 64 c + l and wavefront wv rows
// 64 g + 16 wv .. + 15.  The sign of element e of a word sits at bit b(e);
// shifting the word's 32-bit half left by 31 - (b(e) mod 32) puts it at the
// sign bit of the element's high dword, where an xor applies it.
// part[c * m + i] = sum over the block's words of F'[i][r] Sb[r].
constexpr int kWP = 66;  // LDS pitch (doubles) of one word's 64 values
template <typename TS>
__global__ __launch_bounds__(256) void k_fsb(int m, int64_t t, int64_t W, uint64_t seed, const TS* __restrict__ Sb,
                                             double* __restrict__ part) {
  __shared__ __align__(16) double xs[64 * kWP];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t c = blockIdx.y;
  const int64_t r0 = c * 4096;
  for (int e = threadIdx.x; e < 4096; e += 256) {
    const int64_t r = r0 + e;
    xs[(e >> 6) * kWP + (e & 63)] = r < t ? static_cast<double>(Sb[r]) : 0.0;
  }
  __syncthreads();
  const int64_t w = c * 64 + lane;
  const int ib = blockIdx.x * 64 + wv * 16;
  const uint64_t sseed = seed ^ kStageSalt;
  uint64_t zr[16];
#pragma unroll
  for (int k = 0; k < 16; ++k)
    zr[k] = (ib + k < m && w < W) ? splitmix64(sseed, static_cast<uint64_t>(ib + k) * W + static_cast<uint64_t>(w)) : 0;
  double acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0.0;
  const double* xw = xs + lane * kWP;
#pragma unroll
  for (int q4 = 0; q4 < 4; ++q4) {  // 16 elements of the word at a time
    double x[16];
#pragma unroll
    for (int e = 0; e < 16; e += 2) {
      const double2 pr = *reinterpret_cast<const double2*>(xw + 16 * q4 + e);
      x[e] = pr.x;
      x[e + 1] = pr.y;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const uint32_t half = static_cast<uint32_t>(zr[k] >> (32 * (q4 >> 1)));
      double s = acc[k];
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int el = 16 * q4 + e;                                 // element of the word
        const int pos = 16 * (el & 1) + 15 - ((el & 31) >> 1);     // b(el) mod 32
        const uint32_t sgn = (half << (31 - pos)) & 0x80000000u;
        const uint64_t bits = static_cast<uint64_t>(__double_as_longlong(x[e])) ^ (static_cast<uint64_t>(sgn) << 32);
        s += __longlong_as_double(static_cast<long long>(bits));
      }
      acc[k] = s;
    }
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const double tot = wave_sum(acc[k]);
    if (lane == 0 && ib + k < m) part[c * m + ib + k] = tot;
  }
}

// FSb[i] = scale * sum over the word blocks of part[c * m + i].
__global__ void k_fsb_reduce(int m, int chunks, const double* __restrict__ part, double scale,
                             double* __restrict__ FSb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double s = 0.0;
  for (int c = 0; c < chunks; ++c) s += part[static_cast<size_t>(c) * m + i];
  FSb[i] = scale * s;
}

struct StageShape {
  int tiles_m, tiles_n, splits;
  int64_t kc;
};

// Splits of the t rows so that the grid holds about 1024 blocks (four per
// CU), each with at least 16 staging steps.
StageShape stage_shape(int64_t m, int64_t d, int64_t t) {
  StageShape S;
  S.tiles_m = static_cast<int>(div_up(m, kFM));
  S.tiles_n = static_cast<int>(div_up(d, kFN));
  const int64_t tiles = static_cast<int64_t>(S.tiles_m) * S.tiles_n;
  int64_t sp = 1024 / tiles;
  const int64_t most = div_up(t, 16 * kFK);
  if (sp > most) sp = most;
  if (sp < 1) sp = 1;
  S.kc = div_up(div_up(t, sp), kFK) * kFK;
  S.splits = static_cast<int>(div_up(t, S.kc));
  return S;
}

}  // namespace

size_t second_stage_scratch_floats(int64_t m, int64_t d, int64_t t) {
  const StageShape S = stage_shape(m, d, t);
  const size_t fsb = 2 * static_cast<size_t>(div_up(t, 4096)) * static_cast<size_t>(m);  // doubles
  return static_cast<size_t>(S.splits) * static_cast<size_t>(m) * static_cast<size_t>(d) + fsb + 4;
}

int32_t run_second_stage(const void* SA, const void* Sb, int32_t dtype, int64_t t, int64_t d, int64_t m,
                         uint64_t seed, double* FSA, double* FSb, float* scratch, hipStream_t s) {
  PhaseTimer pt("second_stage", s);
  const StageShape S = stage_shape(m, d, t);
  const int64_t W = div_up(t, 64);
  const double scale = 1.0 / std::sqrt(static_cast<double>(m));
  const int mi = static_cast<int>(m), di = static_cast<int>(d);
  const unsigned blocks = static_cast<unsigned>(S.tiles_m) * S.tiles_n * S.splits;
  if (dtype == SKLS_F64) {
    hipLaunchKernelGGL(k_fsa<double>, dim3(blocks), dim3(256), 0, s, mi, di, t, W, S.kc, S.tiles_m, S.tiles_n,
                       seed, static_cast<const double*>(SA), scratch);
  } else {
    hipLaunchKernelGGL(k_fsa<float>, dim3(blocks), dim3(256), 0, s, mi, di, t, W, S.kc, S.tiles_m, S.tiles_n,
                       seed, static_cast<const float*>(SA), scratch);
  }
  SKLS_CHECK_LAUNCH();
  const int64_t count = m * d;
  int64_t g = div_up(count, 256);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_fsa_reduce, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, count, S.splits, scratch, scale,
                     FSA);
  SKLS_CHECK_LAUNCH();
  if (Sb != nullptr) {
    // the float64 partials of F' (S b) follow the float32 ones, 8-byte aligned
    size_t off = static_cast<size_t>(S.splits) * static_cast<size_t>(m) * static_cast<size_t>(d);
    off = (off + 3) & ~static_cast<size_t>(3);
    double* pb = reinterpret_cast<double*>(scratch + off);
    const int chunks = static_cast<int>(div_up(t, 4096));
    const dim3 grid(static_cast<unsigned>(div_up(m, 64)), static_cast<unsigned>(chunks));
    if (dtype == SKLS_F64)
      hipLaunchKernelGGL(k_fsb<double>, grid, dim3(256), 0, s, mi, t, W, seed, static_cast<const double*>(Sb), pb);
    else
      hipLaunchKernelGGL(k_fsb<float>, grid, dim3(256), 0, s, mi, t, W, seed, static_cast<const float*>(Sb), pb);
    SKLS_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_fsb_reduce, dim3(static_cast<unsigned>(div_up(m, 256))), dim3(256), 0, s, mi, chunks, pb,
                       scale, FSb);
    SKLS_CHECK_LAUNCH();
  }
  return SKLS_OK;
}

}  // namespace skls
