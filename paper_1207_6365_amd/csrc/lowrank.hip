// Rank-k approximation A ~ L D W^T (Section 8, theorem on low-rank
// approximation) in the simplified form of the Section 10 experiments: a
// sparse embedding R^ of the columns, leverage-score sampling for S, and no
// randomized Hadamard transform.
//
// The steps of the theorem are evaluated through equivalent factorisations
// that keep every large product tall and thin:
//   1. Y = A R^T (n x t_R) by hashing columns; R_Y, the triangular factor of Y
//      (Gram on the float64 matrix cores, Cholesky).  U = Y R_Y^{-1} is the
//      orthonormal basis of the theorem and is never formed.
//   2. Scores of Section 6 for Y (squared row norms of Y R_Y^{-1} Pi2, Pi2 a
//      t_R x k_G sign matrix / sqrt(k_G)); t_S draws with replacement.  A row
//      drawn c times enters once with weight sqrt(c / (t_S p)), which leaves
//      S^T S, and so every quantity below, unchanged.
//   3. The QR factor R' of the weighted sampled rows of Y gives S U = Q' (R'
//      R_Y^{-1}) with Q' = (S Y) R'^{-1}; for an SVD S U = U~ S~ V~^T,
//      V~ S~^{-1} [U~^T S A]_k = R_Y R'^{-1} [Q'^T S A]_k.
//   4. [Q'^T S A]_k = P_k C_k by block subspace iteration on M = Q'^T S A
//      (t_R x m) with p = k + oversample columns, each side orthonormalised
//      through the eigendecomposition of its p x p Gram (Jacobi rotations),
//      stopped when the top-k Ritz values settle; then the Rayleigh-Ritz
//      rotation.
//   5. U X~ = (Y R'^{-1} P_k) C_k = B C_k; with B = Q_B G_B and C_k^T = Q_C G_C
//      (orthonormal Q), the SVD U^ D V^^T of G_B G_C^T gives L = Q_B U^,
//      W = Q_C V^.
// Randomness: R^ from the SplitMix64 stream `seed`, the signs of Pi2 from
// the stream seed ^ "leverage", the sampling uniforms u_j = (z_j >> 11) 2^-53
// from the stream seed ^ "sampling" (a draw takes the first row whose running
// score exceeds u_j times the total).

#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels.hpp"
#include "profile.hpp"
#include "sampling.hpp"

namespace skls {
namespace {

constexpr uint64_t kStartSalt = 0x7374617274626C6Bull;   // "startblk": subspace start
constexpr int kMaxTr = 2048;  // columns of Y a wave can hold in LDS
constexpr int kMaxP = 64;     // columns of the subspace iteration (Jacobi size)
// ---------------------------------------------------------------- step 1: Y = A R^T
// One wavefront per row; the row of Y is summed in LDS (compare-and-swap
// float64 adds) and written once.  Column j goes to bucket h(j) with sign
// sigma(j), read from the hashed column tables.
template <typename TV, typename TR>
__global__ __launch_bounds__(kT) void k_colsketch_csr(int64_t n, int tr, const TR* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col, const TV* __restrict__ val,
                                                      const int32_t* __restrict__ hb, const int8_t* __restrict__ hs,
                                                      double* __restrict__ Y) {
  extern __shared__ double ylds[];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  double* acc = ylds + static_cast<size_t>(wid) * tr;
  const int64_t nw = static_cast<int64_t>(gridDim.x) * (kT / kWave);
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kT / kWave) + wid; i < n; i += nw) {
    for (int c = lane; c < tr; c += kWave) acc[c] = 0.0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int64_t b = static_cast<int64_t>(row_ptr[i]), e = static_cast<int64_t>(row_ptr[i + 1]);
    for (int64_t k = b + lane; k < e; k += kWave) {
      const int32_t j = col[k];
      const double x = load_as<double>(val, static_cast<size_t>(k));
      lds_add1<double>(acc, hb[j], hs[j] < 0 ? -x : x);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double* yr = Y + static_cast<size_t>(i) * tr;
    for (int c = lane; c < tr; c += kWave) yr[c] = acc[c];
  }
}

template <typename TV>
__global__ __launch_bounds__(kT) void k_colsketch_dense(int64_t n, int64_t m, int64_t ld, int tr,
                                                        const TV* __restrict__ A, const int32_t* __restrict__ hb,
                                                        const int8_t* __restrict__ hs, double* __restrict__ Y) {
  extern __shared__ double ylds[];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  double* acc = ylds + static_cast<size_t>(wid) * tr;
  const int64_t nw = static_cast<int64_t>(gridDim.x) * (kT / kWave);
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kT / kWave) + wid; i < n; i += nw) {
    for (int c = lane; c < tr; c += kWave) acc[c] = 0.0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const size_t base = static_cast<size_t>(i) * ld;
    for (int64_t j = lane; j < m; j += kWave) {
      const double x = load_as<double>(A, base + j);
      if (x != 0.0) lds_add1<double>(acc, hb[j], hs[j] < 0 ? -x : x);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double* yr = Y + static_cast<size_t>(i) * tr;
    for (int c = lane; c < tr; c += kWave) yr[c] = acc[c];
  }
}

// ---------------------------------------------------------------- step 2: scores, sampling
// Omega [j][c] = +-1 (start of the subspace iteration).
__global__ void k_sign_block(int64_t rows, int cols, uint64_t seed, double* __restrict__ X) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < rows * cols;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint64_t z = splitmix64(seed ^ kStartSalt, static_cast<uint64_t>(e));
    X[e] = negative_of(z) ? -1.0 : 1.0;
  }
}

// Column counts of a CSR matrix (one atomic per entry).
// ---------------------------------------------------------------- transpose
// CSR -> CSC of the sampled rows by a counting sort whose counters live in
// LDS: the entries are cut into chunks of `chunk` entries and the columns
// into ranges of kTrCols; block (c, g) counts, then places, the entries of
// chunk c that fall in range g.  No device-scope atomics.
constexpr int kTrCols = 16384;  // columns per range (64 KiB of LDS counters)
constexpr int kTrChunks = 64;   // most chunks of entries
constexpr int kTrBatch = 8;     // entries per thread with loads in flight together

// rowid[e] = the row of entry e; one wavefront per row.
__global__ __launch_bounds__(kT) void k_entry_rows(int64_t rows, const int64_t* __restrict__ rp,
                                                   int32_t* __restrict__ rowid) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t nw = static_cast<int64_t>(gridDim.x) * (kT / kWave);
  for (int64_t r = blockIdx.x * static_cast<int64_t>(kT / kWave) + threadIdx.x / kWave; r < rows; r += nw)
    for (int64_t k = rp[r] + lane; k < rp[r + 1]; k += kWave) rowid[k] = static_cast<int32_t>(r);
}

// cnt[c * m + j] = entries of column j in chunk c, for the block's range.
__global__ __launch_bounds__(kT) void k_chunk_col_count(int64_t nnz, int64_t chunk, int m,
                                                        const int32_t* __restrict__ col, int32_t* __restrict__ cnt) {
  __shared__ int32_t h[kTrCols];
  const int64_t c = blockIdx.x;
  const int g0 = blockIdx.y * kTrCols;
  const int w = (m - g0) < kTrCols ? m - g0 : kTrCols;
  for (int i = threadIdx.x; i < w; i += kT) h[i] = 0;
  __syncthreads();
  const int64_t e0 = c * chunk;
  const int64_t e1 = (e0 + chunk) < nnz ? e0 + chunk : nnz;
  // kTrBatch independent column loads in flight per thread, then the adds
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kTrBatch * kT) {
    int j[kTrBatch];
#pragma unroll
    for (int u = 0; u < kTrBatch; ++u) {
      const int64_t x = e + static_cast<int64_t>(u) * kT;
      const int jj = col[x < e1 ? x : e1 - 1] - g0;  // an unconditional load (clamped index)
      j[u] = x < e1 ? jj : -1;
    }
#pragma unroll
    for (int u = 0; u < kTrBatch; ++u)
      if (static_cast<unsigned>(j[u]) < static_cast<unsigned>(w)) atomicAdd(&h[j[u]], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < w; i += kT) cnt[c * m + g0 + i] = h[i];
}

// Per column: the counts become exclusive prefixes over the chunks (in
// place) and tot[j] the column's total; tot[m] = 0 closes the scan input.
__global__ void k_chunk_prefix(int m, int chunks, int32_t* __restrict__ cnt, int32_t* __restrict__ tot) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > m) return;
  if (j == m) {
    tot[m] = 0;
    return;
  }
  int32_t sacc = 0;
  for (int c = 0; c < chunks; ++c) {
    const size_t e = static_cast<size_t>(c) * m + j;
    const int32_t v = cnt[e];
    cnt[e] = sacc;
    sacc += v;
  }
  tot[j] = sacc;
}

// Entry (r, j, v) of chunk c goes to slot cp[j] + cnt[c][j] + (its rank
// among the chunk's entries of column j, taken from an LDS cursor); rows
// within a column come in no fixed order.
__global__ __launch_bounds__(kT) void k_chunk_fill(int64_t nnz, int64_t chunk, int m, const int32_t* __restrict__ col,
                                                   const double* __restrict__ val, const int32_t* __restrict__ rowid,
                                                   const int32_t* __restrict__ cp, const int32_t* __restrict__ cnt,
                                                   int32_t* __restrict__ row_out, double* __restrict__ val_out) {
  __shared__ int32_t cur[kTrCols];
  const int64_t c = blockIdx.x;
  const int g0 = blockIdx.y * kTrCols;
  const int w = (m - g0) < kTrCols ? m - g0 : kTrCols;
  for (int i = threadIdx.x; i < w; i += kT) cur[i] = cp[g0 + i] + cnt[c * m + g0 + i];
  __syncthreads();
  const int64_t e0 = c * chunk;
  const int64_t e1 = (e0 + chunk) < nnz ? e0 + chunk : nnz;
  // kTrBatch entries per thread at a time: their loads are all issued
  // before the LDS cursor updates and the scattered stores
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kTrBatch * kT) {
    int j[kTrBatch];
    int32_t r[kTrBatch];
    double v[kTrBatch];
#pragma unroll
    for (int u = 0; u < kTrBatch; ++u) {
      const int64_t x = e + static_cast<int64_t>(u) * kT;
      const int64_t xc = x < e1 ? x : e1 - 1;  // unconditional loads (clamped index)
      const int jj = col[xc] - g0;
      j[u] = x < e1 ? jj : -1;
      r[u] = rowid[xc];
      v[u] = val[xc];
    }
#pragma unroll
    for (int u = 0; u < kTrBatch; ++u) {
      if (static_cast<unsigned>(j[u]) < static_cast<unsigned>(w)) {
        const int32_t slot = atomicAdd(&cur[j[u]], 1);
        row_out[slot] = r[u];
        val_out[slot] = v[u];
      }
    }
  }
}

// C = A B^T for k x k row-major A, B (k <= 64).
__global__ void k_small_abt(int k, const double* __restrict__ A, const double* __restrict__ B,
                            double* __restrict__ C) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= k * k) return;
  const int i = e / k, j = e % k;
  double s = 0.0;
  for (int l = 0; l < k; ++l) s += A[i * k + l] * B[j * k + l];
  C[e] = s;
}

// ---------------------------------------------------------------- one-sided Jacobi
// SVD of a small r x c matrix G (r, c <= 64, row-major, leading dimension c)
// by one-sided Jacobi rotations of its columns (Hestenes): G V = W with
// orthogonal columns; sig[j] = ||W_j|| sorted in decreasing order, V (c x c)
// and W (r x c, columns divided by sig where it is positive) permuted alike.
// For a symmetric positive semidefinite G, sig are its eigenvalues and V its
// eigenvectors.  Sweeps of a round-robin ordering (c - 1 rounds of disjoint
// pairs, one wavefront per pair, lane = row) until every pair is orthogonal
// to 1e-15 relative, at most 60 sweeps.
__global__ __launch_bounds__(1024) void k_jacobi(int r, int c, const double* __restrict__ G, double* __restrict__ sig,
                                                 double* __restrict__ V, double* __restrict__ Wout) {
  __shared__ double a[kMaxP][kMaxP + 1];  // a[column][row]
  __shared__ double v[kMaxP][kMaxP + 1];  // v[column][row]
  __shared__ double nrm[kMaxP];
  __shared__ int perm[kMaxP];
  __shared__ int pos[kMaxP];
  __shared__ int rotated;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int nwaves = blockDim.x / kWave;
  const int cc = c + (c & 1);  // even count (a zero column pads odd c)
  // pairs count as orthogonal once |<a_p, a_q>| is within twice the rounding
  // error of an r-term dot product
  const double tol = 2.0 * (r > 1 ? r : 1) * 0x1.0p-52;
  for (int e = tid; e < kMaxP * kMaxP; e += blockDim.x) {
    const int j = e / kMaxP, i = e % kMaxP;
    a[j][i] = (j < c && i < r) ? G[i * c + j] : 0.0;
    v[j][i] = (i == j) ? 1.0 : 0.0;
  }
  for (int e = tid; e < cc; e += blockDim.x) pos[e] = e;
  for (int e = tid; e < kMaxP; e += blockDim.x) perm[e] = e < c ? e : 0;
  __syncthreads();
  // rounding leaves |<a_p, a_q>| of order r u ||G||_F^2 at best
  double fro2 = 0.0;
  for (int j = 0; j < c; ++j)
    for (int i = 0; i < r; ++i) fro2 += a[j][i] * a[j][i];
  const double floor_abs = tol * fro2;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < cc - 1; ++round) {
      for (int pr = wid; pr < cc / 2; pr += nwaves) {
        // round-robin pairing: position 0 fixed, the others rotate
        const int x0 = pr == 0 ? 0 : 1 + (pr - 1 + round) % (cc - 1);
        const int x1 = 1 + (cc - 2 - pr + round) % (cc - 1);
        const int p = pos[x0], q = pos[x1];
        const double ap = a[p][lane], aq = a[q][lane];
        const double al = wave_total(ap * ap), be = wave_total(aq * aq), ga = wave_total(ap * aq);
        if (fabs(ga) > floor_abs && fabs(ga) > tol * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
          a[p][lane] = cs * ap - sn * aq;
          a[q][lane] = sn * ap + cs * aq;
          const double vp = v[p][lane], vq = v[q][lane];
          v[p][lane] = cs * vp - sn * vq;
          v[q][lane] = sn * vp + cs * vq;
          if (lane == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) break;
  }
  for (int j = wid; j < c; j += nwaves) {
    const double x = a[j][lane];
    const double s = wave_total(x * x);
    if (lane == 0) nrm[j] = sqrt(s);
  }
  __syncthreads();
  if (tid < c) {
    int rank = 0;
    for (int i = 0; i < c; ++i) rank += (nrm[i] > nrm[tid] || (nrm[i] == nrm[tid] && i < tid)) ? 1 : 0;
    perm[rank] = tid;
  }
  __syncthreads();
  for (int e = tid; e < c * c; e += blockDim.x) {
    const int i = e / c, k = e % c;
    V[e] = v[perm[k]][i];
  }
  for (int e = tid; e < r * c; e += blockDim.x) {
    const int i = e / c, k = e % c;
    const double s = nrm[perm[k]];
    Wout[e] = s > 0.0 ? a[perm[k]][i] / s : 0.0;
  }
  if (tid < c) sig[tid] = nrm[perm[tid]];
}

// Eigendecomposition of a symmetric c x c matrix (c <= 64) held in LDS, by
// the cyclic two-sided Jacobi method with a round-robin ordering.  Each
// round rotates the c/2 disjoint pairs of its schedule: one thread per pair
// computes the rotation from the current matrix, then each thread applies
// G <- J^T G J to one 2 x 2 block (row pair x column pair) and V <- V J to
// rows of one column pair.  Sweeps end when no pair has |g_pq| above twice
// the rounding level of a c-term sum, relative to sqrt(|g_pp g_qq|) and to
// max |g_ii| (below the latter rounding alone can keep it), at most 60; all
// pairs are tested together before each sweep, so no sweep is spent only to
// find that nothing rotates.
// All 1024 threads of the block call it; g and v are c padded to even cc.
struct JacLds {
  double g[kMaxP][kMaxP + 1];
  double v[kMaxP][kMaxP + 1];
  uint8_t tp[kMaxP][kMaxP / 2], tq[kMaxP][kMaxP / 2];  // schedule: round x pair
  double rc[kMaxP / 2], rs[kMaxP / 2];
  int rotated;
};

__device__ void jacobi_sym_lds(int c, JacLds& L) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int cc = c + (c & 1);
  const int np = cc / 2;
  const double tol = 2.0 * (c > 1 ? c : 1) * 0x1.0p-52;
  for (int e = tid; e < (cc - 1) * np; e += nt) {
    const int round = e / np, pr = e % np;
    L.tp[round][pr] = static_cast<uint8_t>(pr == 0 ? 0 : 1 + (pr - 1 + round) % (cc - 1));
    L.tq[round][pr] = static_cast<uint8_t>(1 + (cc - 2 - pr + round) % (cc - 1));
  }
  double dmax = 0.0;
  for (int i = 0; i < c; ++i) dmax = fmax(dmax, fabs(L.g[i][i]));
  const double floor_abs = tol * dmax;
  __syncthreads();
  // block (a, b) of this thread for the G update; (row, pair) items for V
  const int ba = tid / np, bb = tid % np;
  const bool gblk = tid < np * np;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) L.rotated = 0;
    __syncthreads();
    // any pair still above the tolerance?
    for (int e = tid; e < c * c; e += nt) {
      const int i = e / c, j = e % c;
      if (i < j) {
        const double ga = L.g[i][j];
        if (fabs(ga) > floor_abs && fabs(ga) > tol * sqrt(fabs(L.g[i][i] * L.g[j][j]))) L.rotated = 1;
      }
    }
    __syncthreads();
    const int open = L.rotated;
    __syncthreads();
    if (!open) break;
    for (int round = 0; round < cc - 1; ++round) {
      if (tid < np) {
        const int p = L.tp[round][tid], q = L.tq[round][tid];
        const double al = L.g[p][p], be = L.g[q][q], ga = L.g[p][q];
        double cs = 1.0, sn = 0.0;
        if (fabs(ga) > floor_abs && fabs(ga) > tol * sqrt(fabs(al * be))) {
          const double zeta = (be - al) / (2.0 * ga);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          cs = rsqrt(1.0 + t * t);
          sn = cs * t;
          L.rotated = 1;
        }
        L.rc[tid] = cs;
        L.rs[tid] = sn;
      }
      __syncthreads();
      if (gblk) {
        const int pa = L.tp[round][ba], qa = L.tq[round][ba], pb = L.tp[round][bb], qb = L.tq[round][bb];
        const double ca = L.rc[ba], sa = L.rs[ba], cb = L.rc[bb], sb = L.rs[bb];
        // columns: (x_pb, x_qb) -> (cb x_pb - sb x_qb, sb x_pb + cb x_qb)
        const double g00 = L.g[pa][pb], g01 = L.g[pa][qb], g10 = L.g[qa][pb], g11 = L.g[qa][qb];
        const double h00 = cb * g00 - sb * g01, h01 = sb * g00 + cb * g01;
        const double h10 = cb * g10 - sb * g11, h11 = sb * g10 + cb * g11;
        // rows: (y_pa, y_qa) -> (ca y_pa - sa y_qa, sa y_pa + ca y_qa)
        L.g[pa][pb] = ca * h00 - sa * h10;
        L.g[qa][pb] = sa * h00 + ca * h10;
        L.g[pa][qb] = ca * h01 - sa * h11;
        L.g[qa][qb] = sa * h01 + ca * h11;
      }
      for (int e = tid; e < cc * 32; e += nt) {
        const int i = e >> 5, pr = e & 31;
        if (pr < np) {
          const int p = L.tp[round][pr], q = L.tq[round][pr];
          const double cs = L.rc[pr], sn = L.rs[pr];
          const double vp = L.v[i][p], vq = L.v[i][q];
          L.v[i][p] = cs * vp - sn * vq;
          L.v[i][q] = sn * vp + cs * vq;
        }
      }
      __syncthreads();
    }
    const int any = L.rotated;
    __syncthreads();
    if (!any) break;
  }
}

__device__ void jacobi_load(int c, const double* __restrict__ G, JacLds& L) {
  for (int e = threadIdx.x; e < kMaxP * kMaxP; e += blockDim.x) {
    const int i = e / kMaxP, j = e % kMaxP;
    L.g[i][j] = (i < c && j < c) ? G[i * c + j] : 0.0;
    L.v[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
}

// Rank of diagonal entry tid among the first c (decreasing, ties by index).
__device__ int diag_rank(int c, const JacLds& L, int tid) {
  int rank = 0;
  const double d = L.g[tid][tid];
  for (int i = 0; i < c; ++i) rank += (L.g[i][i] > d || (L.g[i][i] == d && i < tid)) ? 1 : 0;
  return rank;
}

// G = V diag(lam) V^T for a symmetric c x c G; lam decreasing, V's columns
// permuted alike.
__global__ __launch_bounds__(1024) void k_jacobi_sym(int c, const double* __restrict__ G, double* __restrict__ lam,
                                                     double* __restrict__ V) {
  __shared__ JacLds L;
  __shared__ int perm[kMaxP];
  jacobi_load(c, G, L);
  jacobi_sym_lds(c, L);
  if (threadIdx.x < c) perm[diag_rank(c, L, threadIdx.x)] = threadIdx.x;
  __syncthreads();
  for (int e = threadIdx.x; e < c * c; e += blockDim.x) V[e] = L.v[e / c][perm[e % c]];
  if (threadIdx.x < c) lam[threadIdx.x] = L.g[perm[threadIdx.x]][perm[threadIdx.x]];
}

// Orthonormalising maps from the c x c Gram G = X^T X: Mx with X Mx having
// orthonormal columns and F with X = (X Mx) F on the span kept.  With
// only_if set, the kernel runs only when *only_if is nonzero (the Cholesky
// factor before it found X numerically rank deficient).  Near the
// identity (||G - I||_inf <= 1e-5) by the series G^{-1/2} = I - E/2 + 3E^2/8
// and G^{1/2} = I + E/2 - E^2/8 (E = G - I; the rest is O(||E||^3));
// otherwise from the eigendecomposition G = V diag(lam) V^T:
// Mx = V diag(lam^{-1/2}), F = diag(lam^{1/2}) V^T, with directions of
// eigenvalue <= floor_rel * lam_max dropped (zero columns).
__global__ __launch_bounds__(1024) void k_orth_maps(int c, const double* __restrict__ G, double floor_rel,
                                                    double* __restrict__ Mx, double* __restrict__ F,
                                                    const int32_t* __restrict__ only_if) {
  __shared__ JacLds L;
  __shared__ double rowsum[kMaxP];
  __shared__ double lam[kMaxP];
  if (only_if != nullptr && *only_if == 0) return;
  const int tid = threadIdx.x;
  jacobi_load(c, G, L);
  if (tid < c) {
    double sacc = 0.0;
    for (int j = 0; j < c; ++j) sacc += fabs(L.g[tid][j] - (tid == j ? 1.0 : 0.0));
    rowsum[tid] = sacc;
  }
  __syncthreads();
  double enorm = 0.0;
  for (int i = 0; i < c; ++i) enorm = fmax(enorm, rowsum[i]);
  if (enorm <= 1e-5) {
    for (int e = tid; e < c * c; e += blockDim.x) {
      const int i = e / c, j = e % c;
      double e2 = 0.0;
      for (int l = 0; l < c; ++l)
        e2 += (L.g[i][l] - (i == l ? 1.0 : 0.0)) * (L.g[l][j] - (l == j ? 1.0 : 0.0));
      const double eij = L.g[i][j] - (i == j ? 1.0 : 0.0);
      const double id = i == j ? 1.0 : 0.0;
      Mx[e] = id - 0.5 * eij + 0.375 * e2;
      F[e] = id + 0.5 * eij - 0.125 * e2;
    }
    return;
  }
  jacobi_sym_lds(c, L);
  if (tid < c) lam[tid] = L.g[tid][tid];
  __syncthreads();
  double lmax = 0.0;
  for (int i = 0; i < c; ++i) lmax = fmax(lmax, lam[i]);
  for (int e = tid; e < c * c; e += blockDim.x) {
    const int i = e / c, j = e % c;
    const double lj = lam[j], li = lam[i];
    const bool keepj = lj > floor_rel * lmax && lj > 0.0;
    const bool keepi = li > floor_rel * lmax && li > 0.0;
    Mx[e] = keepj ? L.v[i][j] / sqrt(lj) : 0.0;          // V[i][j] lam_j^{-1/2}
    F[e] = keepi ? sqrt(li) * L.v[j][i] : 0.0;           // lam_i^{1/2} V[j][i]
  }
}

// F' = F V lam^{-1/2} map (columns of eigenvalue <= floor_rel * lam_max
// dropped) from an eigendecomposition already at hand.
__global__ void k_svqb_maps(int p, const double* __restrict__ lam, const double* __restrict__ V, double floor_rel,
                            double* __restrict__ Mx) {
  const int e = threadIdx.x + blockIdx.x * blockDim.x;
  if (e >= p * p) return;
  const int j = e % p;
  const double lj = lam[j];
  const bool keep = lj > floor_rel * lam[0] && lj > 0.0;
  Mx[e] = keep ? V[e] / sqrt(lj) : 0.0;
}

// ---------------------------------------------------------------- residual
// partial[b][c] = sum over the block's rows of L[i, c] * AW[i, c]; slot k
// (c = k) of the block holds its share of sum A_ij^2 (CSR values or dense rows).
__global__ __launch_bounds__(kT) void k_col_dots(int64_t n, int k, const double* __restrict__ L,
                                                 const double* __restrict__ AW, double* __restrict__ partial) {
  __shared__ double sh[kT / kWave];
  for (int c = 0; c < k; ++c) {
    double s = 0.0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kT)
      s += L[static_cast<size_t>(i) * k + c] * AW[static_cast<size_t>(i) * k + c];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) partial[static_cast<size_t>(blockIdx.x) * (k + 1) + c] = s;
  }
}

template <typename TV>
__global__ __launch_bounds__(kT) void k_sumsq(int64_t count, const TV* __restrict__ x, int64_t rows, int64_t cols,
                                              int64_t ld, int k, double* __restrict__ partial) {
  __shared__ double sh[kT / kWave];
  double s = 0.0;
  if (rows < 0) {
    for (int64_t e = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x; e < count;
         e += static_cast<int64_t>(gridDim.x) * kT) {
      const double v = load_as<double>(x, static_cast<size_t>(e));
      s += v * v;
    }
  } else {
    for (int64_t e = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x; e < rows * cols;
         e += static_cast<int64_t>(gridDim.x) * kT) {
      const double v = load_as<double>(x, static_cast<size_t>((e / cols) * ld + e % cols));
      s += v * v;
    }
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) partial[static_cast<size_t>(blockIdx.x) * (k + 1) + k] = s;
}

__global__ void k_sum_cols(const double* __restrict__ partial, int nblk, int w, double* __restrict__ out) {
  const int c = threadIdx.x;
  if (c >= w) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[static_cast<size_t>(b) * w + c];
  out[c] = s;
}

}  // namespace

// ---------------------------------------------------------------- host side
namespace {

constexpr double kDropRel = 1e-24;  // Gram eigenvalues below this (relative) count as zero

struct LrWs {
  int32_t* hb;
  int8_t* hs;
  double* Y;
  void* gram;
  size_t gram_bytes;
  double *G, *cholw, *R, *Rinv, *RinvT;
  int32_t* status;
  double *Pi2, *T, *Z, *score, *cum, *dtiles;
  int32_t *counts, *flag, *pos, *itiles, *last;
  int32_t* list;
  double* wts;
  int64_t *len, *rp, *ltiles;
  int32_t* colc;
  double* valc;
  int32_t* rowT;
  double* valT;
  int32_t *cp, *ccnt, *ctiles, *rowid, *chunkcnt;
  double *SY, *Q, *F, *Ft, *G1, *X1, *P, *Pt;
  GemmScratch part;
  double *Gp, *V, *Wj, *lam, *Mx, *F1, *F2, *Fac;
  double *Pk, *T2, *Bq, *Bt, *Cq, *Ct, *FacB, *FacC, *K, *Uh, *Vh, *AW, *dots, *dsum;
  int nblk;
};

LrWs carve_lr(Arena& ar, const LowRankPlan& P) {
  LrWs w;
  const int64_t n = P.n, m = P.m, tr = P.tr, ns = P.nsmax, p = P.p, k = P.k;
  w.hb = ar.take<int32_t>(m);
  w.hs = ar.take<int8_t>(m);
  w.Y = ar.take<double>(static_cast<size_t>(n) * tr);
  size_t gb = 0;
  const int64_t rows_d[][2] = {{n, tr}, {ns, tr}, {tr, p}, {m, p}, {n, k}, {m, k}};
  for (const auto& rd : rows_d) {
    const size_t b = gram_ws_bytes(rd[0], rd[1]);
    gb = b > gb ? b : gb;
  }
  w.gram_bytes = gb;
  w.gram = ar.take<double>(gb / sizeof(double) + 1);
  w.G = ar.take<double>(static_cast<size_t>(tr) * tr);
  w.cholw = ar.take<double>(cholesky_scratch_doubles(tr));
  w.R = ar.take<double>(static_cast<size_t>(tr) * tr);
  w.Rinv = ar.take<double>(static_cast<size_t>(tr) * tr);
  w.RinvT = ar.take<double>(static_cast<size_t>(tr) * tr);
  w.status = ar.take<int32_t>(4);
  w.Pi2 = ar.take<double>(static_cast<size_t>(tr) * P.kg);
  w.T = ar.take<double>(static_cast<size_t>(tr) * P.kg);
  w.Z = ar.take<double>(static_cast<size_t>(n) * P.kg);
  w.score = ar.take<double>(n);
  w.cum = ar.take<double>(n);
  w.dtiles = ar.take<double>(tiles_for(n));
  w.counts = ar.take<int32_t>(n);
  w.flag = ar.take<int32_t>(n);
  w.pos = ar.take<int32_t>(n);
  w.itiles = ar.take<int32_t>(tiles_for(n));
  w.last = ar.take<int32_t>(4);
  w.list = ar.take<int32_t>(ns);
  w.wts = ar.take<double>(ns);
  w.len = ar.take<int64_t>(ns);
  w.rp = ar.take<int64_t>(ns + 1);
  w.ltiles = ar.take<int64_t>(tiles_for(ns));
  w.colc = P.csr ? ar.take<int32_t>(P.nnzmax) : nullptr;
  w.valc = ar.take<double>(P.nnzmax);
  w.rowT = P.csr ? ar.take<int32_t>(P.nnzmax) : nullptr;
  w.valT = P.csr ? ar.take<double>(P.nnzmax) : nullptr;
  w.cp = P.csr ? ar.take<int32_t>(m + 1) : nullptr;
  w.ccnt = P.csr ? ar.take<int32_t>(m + 1) : nullptr;
  w.ctiles = P.csr ? ar.take<int32_t>(tiles_for(m + 1)) : nullptr;
  w.rowid = P.csr ? ar.take<int32_t>(P.nnzmax) : nullptr;
  w.chunkcnt = P.csr ? ar.take<int32_t>(static_cast<size_t>(kTrChunks) * m) : nullptr;
  w.SY = ar.take<double>(static_cast<size_t>(ns) * tr);
  w.Q = ar.take<double>(static_cast<size_t>(ns) * tr);
  w.F = ar.take<double>(static_cast<size_t>(m) * p);
  w.Ft = ar.take<double>(static_cast<size_t>(m) * p);
  w.G1 = ar.take<double>(static_cast<size_t>(ns) * p);
  w.X1 = ar.take<double>(static_cast<size_t>(ns) * p);
  w.P = ar.take<double>(static_cast<size_t>(tr) * p);
  w.Pt = ar.take<double>(static_cast<size_t>(tr) * p);
  w.part.doubles = size_t(1) << 23;  // split-K partial products (64 MiB)
  w.part.part = ar.take<double>(w.part.doubles);
  const size_t pp = static_cast<size_t>(kMaxP) * kMaxP;
  w.Gp = ar.take<double>(pp);
  w.V = ar.take<double>(pp);
  w.Wj = ar.take<double>(pp);
  w.lam = ar.take<double>(kMaxP);
  w.Mx = ar.take<double>(pp);
  w.F1 = ar.take<double>(pp);
  w.F2 = ar.take<double>(pp);
  w.Fac = ar.take<double>(pp);
  w.Pk = ar.take<double>(static_cast<size_t>(tr) * k);
  w.T2 = ar.take<double>(static_cast<size_t>(tr) * k);
  w.Bq = ar.take<double>(static_cast<size_t>(n) * k);
  w.Bt = ar.take<double>(static_cast<size_t>(n) * k);
  w.Cq = ar.take<double>(static_cast<size_t>(m) * k);
  w.Ct = ar.take<double>(static_cast<size_t>(m) * k);
  w.FacB = ar.take<double>(pp);
  w.FacC = ar.take<double>(pp);
  w.K = ar.take<double>(pp);
  w.Uh = ar.take<double>(pp);
  w.Vh = ar.take<double>(pp);
  w.AW = ar.take<double>(static_cast<size_t>(n) * k);
  w.nblk = 256;
  w.dots = ar.take<double>(static_cast<size_t>(w.nblk) * (k + 1));
  w.dsum = ar.take<double>(k + 1);
  return w;
}

// X (rows x c, packed) -> X with orthonormal columns by two passes of
// Gram-based orthonormalisation (CholeskyQR2); fac (c x c) with
// X_in = X_out fac.  Pass 1 maps X by R^{-1} for the Cholesky factor R of
// its Gram; where that factor reports numerical rank deficiency, the
// eigendecomposition maps (which drop the null directions) replace it on
// the device, with no host round trip.  Pass 2 starts from a Gram within
// about kappa(X)^2 u of the identity and takes the series maps of
// k_orth_maps (or its eigen route when further away).
int32_t svqb2(double* X, double* tmp, int64_t rows, int c, double* fac, LrWs& w, hipStream_t s) {
  double* cur = X;
  double* nxt = tmp;
  int32_t* chol_bad = w.status + 2;
  for (int pass = 0; pass < 2; ++pass) {
    SKLS_TRY(run_gram(cur, SKLS_F64, c, nullptr, SKLS_F64, rows, c, w.Gp, w.gram, w.gram_bytes, s));
    if (pass == 0) {
      SKLS_TRY(run_cholesky(w.Gp, c, c, w.F1, w.Mx, w.Wj, chol_bad, w.cholw, s));
      hipLaunchKernelGGL(k_orth_maps, dim3(1), dim3(1024), 0, s, c, w.Gp, kDropRel, w.Mx, w.F1, chol_bad);
    } else {
      hipLaunchKernelGGL(k_orth_maps, dim3(1), dim3(1024), 0, s, c, w.Gp, kDropRel, w.Mx, w.F2,
                         static_cast<const int32_t*>(nullptr));
    }
    SKLS_CHECK_LAUNCH();
    SKLS_TRY(gemm(false, rows, c, c, 1.0, cur, c, w.Mx, c, nxt, c, w.part, s));
    std::swap(cur, nxt);
  }
  // after two passes the result is back in X
  if (fac) SKLS_TRY(gemm(false, c, c, c, 1.0, w.F2, c, w.F1, c, fac, c, w.part, s));
  return SKLS_OK;
}

}  // namespace

int32_t low_rank_plan(const skls_matrix& A, const skls_low_rank_opts& o, LowRankPlan& P) {
  P.n = A.n;
  P.m = A.d;
  P.csr = A.layout == SKLS_CSR;
  P.k = o.k;
  if (P.n >= (int64_t(1) << 31) || P.m >= (int64_t(1) << 31)) {
    set_error("low_rank: n and m must be below 2^31");
    return SKLS_ERR_SHAPE;
  }
  if (o.k < 1 || o.k > 48 || o.k > P.n || o.k > P.m) {
    set_error("low_rank: need 1 <= k <= 48 and k <= min(n, m)");
    return SKLS_ERR_ARG;
  }
  const int over = o.oversample > 0 ? o.oversample : 16;
  P.kg = o.k_g > 0 ? o.k_g : 32;
  if (P.kg > 64 || o.k_g < 0 || o.oversample < 0) {
    set_error("low_rank: need 0 <= k_g <= 64 and oversample >= 0");
    return SKLS_ERR_ARG;
  }
  const int64_t cap = std::min<int64_t>(std::min<int64_t>(P.m, P.n), kMaxTr);
  int64_t tr = o.t_r;
  if (tr == 0) {
    if (!(o.eps > 0.0 && o.eps <= 1.0)) {
      set_error("low_rank: give t_r or 0 < eps <= 1");
      return SKLS_ERR_ARG;
    }
    tr = static_cast<int64_t>(std::ceil(static_cast<double>(o.k) / o.eps));
    tr = std::max<int64_t>(tr, std::min<int64_t>(o.k + over, kMaxP));
    tr = std::min(tr, cap);
  }
  if (tr < o.k || tr > cap) {
    set_error("low_rank: need k <= t_r <= min(n, m, 2048)");
    return SKLS_ERR_ARG;
  }
  P.tr = tr;
  P.p = static_cast<int>(std::min<int64_t>(std::min<int64_t>(o.k + over, kMaxP), tr));
  P.ts = o.t_s > 0 ? o.t_s : 64 * tr;
  if (P.ts < tr || P.ts >= (int64_t(1) << 31) || o.t_s < 0) {
    set_error("low_rank: need t_r <= t_s < 2^31");
    return SKLS_ERR_ARG;
  }
  P.nsmax = std::min(P.n, P.ts);
  P.nnzmax = P.csr ? std::max<int64_t>(A.nnz, 1) : P.nsmax * P.m;
  P.max_iter = o.max_iter > 0 ? o.max_iter : 60;
  P.tol = o.tol > 0.0 ? o.tol : 1e-13;
  return SKLS_OK;
}

size_t low_rank_ws_bytes(const LowRankPlan& P) {
  Arena ar(nullptr, 0);
  carve_lr(ar, P);
  return ar.used;
}

int32_t run_low_rank(const skls_matrix& A, const LowRankPlan& P, uint64_t seed, double* Lout, double* Dout,
                     double* Wout, skls_low_rank_info* info, void* ws, size_t ws_bytes, hipStream_t s) {
  Arena ar(ws, ws_bytes);
  LrWs w = carve_lr(ar, P);
  if (!ar.fits() || ws == nullptr) {
    set_error("low_rank: workspace too small (%zu bytes needed)", ar.used);
    return SKLS_ERR_WORKSPACE;
  }
  const int64_t n = P.n, m = P.m, tr = P.tr, k = P.k;
  const int p = P.p, kg = P.kg, tri = static_cast<int>(tr);
  skls_low_rank_info inf{};
  inf.t_r = tr;
  inf.t_s = P.ts;
  hipEvent_t ev[5];
  for (auto& e : ev) SKLS_TRY_HIP(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 5; ++i) (void)hipEventDestroy(e[i]);
    }
  } guard{ev};
  SKLS_TRY_HIP(hipEventRecord(ev[0], s));

  // ---- step 1: Y = A R^T, and R_Y
  {
    PhaseTimer pt("lowrank_sketch", s);
    SKLS_TRY(launch_hash(m, static_cast<uint32_t>(tr), seed, 0, w.hb, w.hs, s));
    const size_t lds = static_cast<size_t>(kT / kWave) * tr * sizeof(double);
    const unsigned g = grid_for(n, kT / kWave, 8192);
    int32_t st = with_value(A.dtype, [&](auto tv) -> int32_t {
      using TV = decltype(tv);
      if (!P.csr) {
        if (lds > 65536)
          SKLS_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_colsketch_dense<TV>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
        hipLaunchKernelGGL(k_colsketch_dense<TV>, dim3(g), dim3(kT), lds, s, n, m, A.ld, tri,
                           static_cast<const TV*>(A.val), w.hb, w.hs, w.Y);
        SKLS_CHECK_LAUNCH();
        return SKLS_OK;
      }
      return with_rowptr(A, [&](auto trt) -> int32_t {
        using TR = decltype(trt);
        if (lds > 65536)
          SKLS_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_colsketch_csr<TV, TR>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
        hipLaunchKernelGGL((k_colsketch_csr<TV, TR>), dim3(g), dim3(kT), lds, s, n, tri,
                           static_cast<const TR*>(A.row_ptr), A.col_idx, static_cast<const TV*>(A.val), w.hb, w.hs,
                           w.Y);
        SKLS_CHECK_LAUNCH();
        return SKLS_OK;
      });
    });
    SKLS_TRY(st);
  }
  SKLS_TRY(run_gram(w.Y, SKLS_F64, tr, nullptr, SKLS_F64, n, tr, w.G, w.gram, w.gram_bytes, s));
  SKLS_TRY(run_cholesky(w.G, tr, tr, w.R, w.Rinv, w.RinvT, w.status, w.cholw, s));
  int32_t st_h = 0;
  SKLS_TRY(to_host(&st_h, w.status, sizeof st_h, s));
  if (st_h) {
    set_error("low_rank: A R^T is numerically rank deficient (lower t_r)");
    return SKLS_ERR_RANK;
  }
  SKLS_TRY_HIP(hipEventRecord(ev[1], s));

  // ---- step 2: scores of Y, sampling, sampled rows
  int64_t ns = 0, nnz_s = 0;
  {
    PhaseTimer pt("lowrank_sample", s);
    hipLaunchKernelGGL(k_sign_projection, dim3(grid_for(tr * kg, kT, 1 << 20)), dim3(kT), 0, s, tri, kg, seed,
                       w.Pi2);
    SKLS_CHECK_LAUNCH();
    SKLS_TRY(gemm(false, tr, kg, tr, 1.0, w.Rinv, tr, w.Pi2, kg, w.T, kg, w.part, s));
    SKLS_TRY(gemm(false, n, kg, tr, 1.0, w.Y, tr, w.T, kg, w.Z, kg, w.part, s));
    SKLS_TRY(launch_fill_zero(w.last, 16, s));
    hipLaunchKernelGGL(k_row_sqnorm, dim3(grid_for(n, kT / kWave, 8192)), dim3(kT), 0, s, n, kg, w.Z, w.score,
                       w.last);
    SKLS_CHECK_LAUNCH();
    SKLS_TRY(scan<double>(w.score, n, w.dtiles, w.cum, false, s));
    SKLS_TRY(launch_fill_zero(w.counts, static_cast<size_t>((n + 3) / 4) * 16, s));
    hipLaunchKernelGGL(k_sample, dim3(grid_for(P.ts, kT, 4096)), dim3(kT), 0, s, P.ts, n, seed, w.cum, w.score,
                       w.last, w.counts);
    SKLS_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_flags, dim3(grid_for(n, kT, 4096)), dim3(kT), 0, s, n, w.counts, w.flag);
    SKLS_CHECK_LAUNCH();
    SKLS_TRY(scan<int32_t>(w.flag, n, w.itiles, w.pos, true, s));
    int32_t hv[2];
    double total = 0.0;
    SKLS_TRY_HIP(hipMemcpyAsync(&hv[0], w.pos + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SKLS_TRY_HIP(hipMemcpyAsync(&hv[1], w.flag + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SKLS_TRY(to_host(&total, w.cum + (n - 1), sizeof total, s));
    if (!(total > 0.0) || !std::isfinite(total)) {
      set_error("low_rank: the leverage scores of A R^T are not positive and finite");
      return SKLS_ERR_RANK;
    }
    ns = static_cast<int64_t>(hv[0]) + hv[1];
    if (ns < tr) {
      set_error("low_rank: %lld distinct rows drawn, fewer than t_r = %lld (raise t_s)", static_cast<long long>(ns),
                static_cast<long long>(tr));
      return SKLS_ERR_RANK;
    }
    int32_t st = with_value(A.dtype, [&](auto tv) -> int32_t {
      using TV = decltype(tv);
      if (!P.csr) {
        hipLaunchKernelGGL(k_compact<int32_t>, dim3(grid_for(n, kT, 4096)), dim3(kT), 0, s, n, P.ts, w.counts,
                           w.pos, w.score, w.cum, nullptr, w.list, w.wts, nullptr);
        SKLS_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_gather_rows<TV>, dim3(grid_for(ns, kT / kWave, 8192)), dim3(kT), 0, s, ns, m, A.ld,
                           static_cast<const TV*>(A.val), w.list, w.wts, w.valc);
        SKLS_CHECK_LAUNCH();
        nnz_s = ns * m;
        return SKLS_OK;
      }
      return with_rowptr(A, [&](auto trt) -> int32_t {
        using TR = decltype(trt);
        const TR* rpA = static_cast<const TR*>(A.row_ptr);
        hipLaunchKernelGGL(k_compact<TR>, dim3(grid_for(n, kT, 4096)), dim3(kT), 0, s, n, P.ts, w.counts, w.pos,
                           w.score, w.cum, rpA, w.list, w.wts, w.len);
        SKLS_CHECK_LAUNCH();
        SKLS_TRY(scan<int64_t>(w.len, ns, w.ltiles, w.rp, true, s));
        int64_t hl[2];
        SKLS_TRY_HIP(hipMemcpyAsync(&hl[0], w.rp + (ns - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
        SKLS_TRY(to_host(&hl[1], w.len + (ns - 1), sizeof(int64_t), s));
        nnz_s = hl[0] + hl[1];
        SKLS_TRY_HIP(hipMemcpyAsync(w.rp + ns, &nnz_s, sizeof(int64_t), hipMemcpyHostToDevice, s));
        SKLS_TRY_HIP(hipStreamSynchronize(s));
        hipLaunchKernelGGL((k_gather_csr<TV, TR>), dim3(grid_for(ns, kT / kWave, 8192)), dim3(kT), 0, s, ns, rpA,
                           A.col_idx, static_cast<const TV*>(A.val), w.list, w.wts, w.rp, w.colc, w.valc);
        SKLS_CHECK_LAUNCH();
        // the transpose of the sampled rows, for the products with (S A)^T
        if (nnz_s >= (int64_t(1) << 31)) {
          set_error("low_rank: the sampled rows hold 2^31 or more nonzeros");
          return SKLS_ERR_SHAPE;
        }
        const int64_t chunk = std::max<int64_t>(16384, div_up(nnz_s, kTrChunks));
        const int chunks = static_cast<int>(std::max<int64_t>(div_up(nnz_s, chunk), 1));
        const dim3 tg(static_cast<unsigned>(chunks), static_cast<unsigned>(div_up(m, kTrCols)));
        hipLaunchKernelGGL(k_entry_rows, dim3(grid_for(ns, kT / kWave, 8192)), dim3(kT), 0, s, ns, w.rp, w.rowid);
        SKLS_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_chunk_col_count, tg, dim3(kT), 0, s, nnz_s, chunk, static_cast<int>(m), w.colc,
                           w.chunkcnt);
        SKLS_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_chunk_prefix, dim3(static_cast<unsigned>(div_up(m + 1, kT))), dim3(kT), 0, s,
                           static_cast<int>(m), chunks, w.chunkcnt, w.ccnt);
        SKLS_CHECK_LAUNCH();
        SKLS_TRY(scan<int32_t>(w.ccnt, m + 1, w.ctiles, w.cp, true, s));  // cp[m] = nnz_s
        hipLaunchKernelGGL(k_chunk_fill, tg, dim3(kT), 0, s, nnz_s, chunk, static_cast<int>(m), w.colc, w.valc,
                           w.rowid, w.cp, w.chunkcnt, w.rowT, w.valT);
        SKLS_CHECK_LAUNCH();
        return SKLS_OK;
      });
    });
    SKLS_TRY(st);
    hipLaunchKernelGGL(k_gather_rows<double>, dim3(grid_for(ns, kT / kWave, 8192)), dim3(kT), 0, s, ns, tr, tr,
                       w.Y, w.list, w.wts, w.SY);
    SKLS_CHECK_LAUNCH();
  }
  inf.rows_sampled = ns;
  inf.nnz_sampled = P.csr ? nnz_s : 0;
  SKLS_TRY_HIP(hipEventRecord(ev[2], s));

  // ---- steps 3 and 4: R' of S Y, Q' = S Y R'^{-1}, top-k of M = Q'^T S A
  {
    PhaseTimer pt("lowrank_topk", s);
    SKLS_TRY(run_gram(w.SY, SKLS_F64, tr, nullptr, SKLS_F64, ns, tr, w.G, w.gram, w.gram_bytes, s));
    SKLS_TRY(run_cholesky(w.G, tr, tr, w.R, w.Rinv, w.RinvT, w.status, w.cholw, s));
    SKLS_TRY(to_host(&st_h, w.status, sizeof st_h, s));
    if (st_h) {
      set_error("low_rank: S U is numerically rank deficient (raise t_s)");
      return SKLS_ERR_RANK;
    }
    SKLS_TRY(gemm(false, ns, tr, tr, 1.0, w.SY, tr, w.Rinv, tr, w.Q, tr, w.part, s));
    hipLaunchKernelGGL(k_sign_block, dim3(grid_for(m * p, kT, 8192)), dim3(kT), 0, s, m, p, seed, w.F);
    SKLS_CHECK_LAUNCH();
    const unsigned gr = grid_for(ns, kT / kWave, 8192);
    auto times_SA = [&](const double* X, double* out) -> int32_t {  // out (ns x p) = S A X
      if (P.csr) {
        if (p <= 32)
          hipLaunchKernelGGL((k_spmm<double, int64_t, true>), dim3(gr), dim3(kT), 0, s, ns, p, w.rp, w.colc, w.valc,
                             X, out);
        else
          hipLaunchKernelGGL((k_spmm<double, int64_t, false>), dim3(gr), dim3(kT), 0, s, ns, p, w.rp, w.colc, w.valc,
                             X, out);
        SKLS_CHECK_LAUNCH();
        return SKLS_OK;
      }
      return gemm(false, ns, p, m, 1.0, w.valc, m, X, p, out, p, w.part, s);
    };
    auto times_SAt = [&](const double* X, double* out) -> int32_t {  // out (m x p) = (S A)^T X
      if (P.csr) {
        const unsigned gm = grid_for(m, kT / kWave, 8192);
        if (p <= 32)
          hipLaunchKernelGGL((k_spmm<double, int32_t, true>), dim3(gm), dim3(kT), 0, s, m, p, w.cp, w.rowT, w.valT,
                             X, out);
        else
          hipLaunchKernelGGL((k_spmm<double, int32_t, false>), dim3(gm), dim3(kT), 0, s, m, p, w.cp, w.rowT, w.valT,
                             X, out);
        SKLS_CHECK_LAUNCH();
        return SKLS_OK;
      }
      return gemm(true, m, p, ns, 1.0, w.valc, m, X, p, out, p, w.part, s);
    };
    std::vector<double> prev(p, 0.0), cur(p, 0.0);
    int it = 0;
    bool conv = false;
    for (;;) {
      SKLS_TRY(times_SA(w.F, w.G1));
      SKLS_TRY(gemm(true, tr, p, ns, 1.0, w.Q, tr, w.G1, p, w.P, p, w.part, s));  // P = Q'^T (S A F)
      SKLS_TRY(svqb2(w.P, w.Pt, tr, p, nullptr, w, s));
      SKLS_TRY(gemm(false, ns, p, tr, 1.0, w.Q, tr, w.P, p, w.X1, p, w.part, s));
      SKLS_TRY(times_SAt(w.X1, w.F));  // F = M^T P
      SKLS_TRY(run_gram(w.F, SKLS_F64, p, nullptr, SKLS_F64, m, p, w.Gp, w.gram, w.gram_bytes, s));
      hipLaunchKernelGGL(k_jacobi_sym, dim3(1), dim3(1024), 0, s, p, w.Gp, w.lam, w.V);
      SKLS_CHECK_LAUNCH();
      SKLS_TRY(to_host(cur.data(), w.lam, sizeof(double) * p, s));
      ++it;
      if (it > 1) {
        double worst = 0.0;
        for (int64_t i = 0; i < k; ++i) {
          const double d = std::fabs(cur[i] - prev[i]) / (cur[0] > 0.0 ? cur[0] : 1.0);
          worst = d > worst ? d : worst;
        }
        if (worst <= P.tol) conv = true;
      }
      if (conv || it >= P.max_iter) break;
      prev = cur;
      // keep F well conditioned for the next product: F <- F V lam^{-1/2}
      hipLaunchKernelGGL(k_svqb_maps, dim3(grid_for(p * p, kT, 64)), dim3(kT), 0, s, p, w.lam, w.V, kDropRel,
                         w.Mx);
      SKLS_CHECK_LAUNCH();
      SKLS_TRY(gemm(false, m, p, p, 1.0, w.F, p, w.Mx, p, w.Ft, p, w.part, s));
      std::swap(w.F, w.Ft);
    }
    inf.iterations = it;
    inf.converged = conv ? 1 : 0;
    // Rayleigh-Ritz: P_k = P V[:, :k], C_k^T = M^T P_k = F V[:, :k]
    SKLS_TRY(gemm(false, tr, k, p, 1.0, w.P, p, w.V, p, w.Pk, k, w.part, s));
    SKLS_TRY(gemm(false, m, k, p, 1.0, w.F, p, w.V, p, w.Cq, k, w.part, s));
  }
  SKLS_TRY_HIP(hipEventRecord(ev[3], s));

  // ---- step 5: B = Y R'^{-1} P_k, orthonormal factors, k x k SVD
  {
    PhaseTimer pt("lowrank_factors", s);
    SKLS_TRY(gemm(false, tr, k, tr, 1.0, w.Rinv, tr, w.Pk, k, w.T2, k, w.part, s));
    SKLS_TRY(gemm(false, n, k, tr, 1.0, w.Y, tr, w.T2, k, w.Bq, k, w.part, s));
    const int ki = static_cast<int>(k);
    SKLS_TRY(svqb2(w.Bq, w.Bt, n, ki, w.FacB, w, s));
    SKLS_TRY(svqb2(w.Cq, w.Ct, m, ki, w.FacC, w, s));
    hipLaunchKernelGGL(k_small_abt, dim3(grid_for(k * k, kT, 64)), dim3(kT), 0, s, ki, w.FacB, w.FacC, w.K);
    SKLS_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(1024), 0, s, ki, ki, w.K, Dout, w.Vh, w.Uh);
    SKLS_CHECK_LAUNCH();
    SKLS_TRY(gemm(false, n, k, k, 1.0, w.Bq, k, w.Uh, k, Lout, k, w.part, s));
    SKLS_TRY(gemm(false, m, k, k, 1.0, w.Cq, k, w.Vh, k, Wout, k, w.part, s));
    // ||A - L D W^T||_F^2 = ||A||_F^2 - 2 sum_c D_c <L_c, (A W)_c> + sum_c D_c^2
    int32_t st = with_value(A.dtype, [&](auto tv) -> int32_t {
      using TV = decltype(tv);
      const unsigned g = grid_for(n, kT / kWave, 8192);
      if (!P.csr) {
        SKLS_TRY(dense_times<TV>(n, m, static_cast<const TV*>(A.val), A.ld, Wout, k, w.AW, w.part, s));
        hipLaunchKernelGGL(k_sumsq<TV>, dim3(w.nblk), dim3(kT), 0, s, int64_t(0), static_cast<const TV*>(A.val), n,
                           m, A.ld, ki, w.dots);
        SKLS_CHECK_LAUNCH();
        return SKLS_OK;
      }
      return with_rowptr(A, [&](auto trt) -> int32_t {
        using TR = decltype(trt);
        if (ki <= 32)
          hipLaunchKernelGGL((k_spmm<TV, TR, true>), dim3(g), dim3(kT), 0, s, n, ki,
                             static_cast<const TR*>(A.row_ptr), A.col_idx, static_cast<const TV*>(A.val), Wout, w.AW);
        else
          hipLaunchKernelGGL((k_spmm<TV, TR, false>), dim3(g), dim3(kT), 0, s, n, ki,
                             static_cast<const TR*>(A.row_ptr), A.col_idx, static_cast<const TV*>(A.val), Wout, w.AW);
        SKLS_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_sumsq<TV>, dim3(w.nblk), dim3(kT), 0, s, A.nnz, static_cast<const TV*>(A.val),
                           int64_t(-1), int64_t(0), int64_t(0), ki, w.dots);
        SKLS_CHECK_LAUNCH();
        return SKLS_OK;
      });
    });
    SKLS_TRY(st);
    hipLaunchKernelGGL(k_col_dots, dim3(w.nblk), dim3(kT), 0, s, n, ki, Lout, w.AW, w.dots);
    SKLS_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_sum_cols, dim3(1), dim3(kT), 0, s, w.dots, w.nblk, ki + 1, w.dsum);
    SKLS_CHECK_LAUNCH();
  }
  SKLS_TRY_HIP(hipEventRecord(ev[4], s));
  std::vector<double> hs(k + 1), hd(k);
  SKLS_TRY_HIP(hipMemcpyAsync(hd.data(), Dout, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  SKLS_TRY(to_host(hs.data(), w.dsum, sizeof(double) * (k + 1), s));
  double r2 = hs[k];
  for (int64_t c = 0; c < k; ++c) r2 += hd[c] * hd[c] - 2.0 * hd[c] * hs[c];
  inf.fro_norm = std::sqrt(hs[k]);
  inf.resid_fro = std::sqrt(r2 > 0.0 ? r2 : 0.0);
  float ms = 0.0f;
  SKLS_TRY_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
  inf.ms_sketch = ms;
  SKLS_TRY_HIP(hipEventElapsedTime(&ms, ev[1], ev[2]));
  inf.ms_sample = ms;
  SKLS_TRY_HIP(hipEventElapsedTime(&ms, ev[2], ev[3]));
  inf.ms_topk = ms;
  SKLS_TRY_HIP(hipEventElapsedTime(&ms, ev[3], ev[4]));
  inf.ms_factors = ms;
  if (info) *info = inf;
  return SKLS_OK;
}

}  // namespace skls
