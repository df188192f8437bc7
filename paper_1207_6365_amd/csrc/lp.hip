// l_p regression min_x ||A x - b||_p, 1 <= p < inf (Section 9):
//   1. F A for F block-diagonal, every block of w rows embedded by the same
//      generalized sparse embedding (Section 5; rows hashed by their index
//      inside the block), float64;
//   2. R of F A (float64 Gram, Cholesky): U = R^{-1} is the change of basis
//      that makes F A U well conditioned (the l_2 basis, see the header);
//   3. squared row norms of A R^{-1} Pi2 (Pi2 the d x k_G sign matrix /
//      sqrt(k_G) of the stream seed ^ "leverage"), raised to p/2: the
//      sampling weights lam_i;
//   4. stage 1: row i kept iff u_i < pi_i = min(1, s1 lam_i / sum lam)
//      (u_i from the stream seed ^ "sampling"), weight pi_i^{-1/p}; x_c the
//      weighted l_p fit of the kept rows;
//   5. stage 2: rho = A x_c - b; row i kept iff u'_i < min(1, s2 max(lam_i /
//      sum lam, |rho_i|^p / sum |rho|^p)) (stream seed ^ "resample"), x the
//      weighted fit of those rows.
// The weighted fits run on the gathered float64 coreset: p = 2 by the normal
// equations, p = 1 by a primal-dual interior-point method on the dual of the
// l_1 fit (Mehrotra predictor-corrector), other p by iteratively reweighted
// least squares (a floor on |r| in the weights that shrinks to 1e-9 of the
// starting mean; Newton steps of length 1/(p-1) with halving for p > 2).
// Every step solves a weighted normal system through the float64 Gram,
// Cholesky and the inverse factor.

#include <cmath>

#include "kernels.hpp"
#include "profile.hpp"
#include "sampling.hpp"

namespace skls {
namespace {

constexpr uint64_t kStage2Salt = 0x726573616D706C65ull;  // "resample"
constexpr int kRed = 256;                                 // blocks of the reductions over rows
constexpr int kResBlocks = 1024;                          // blocks of the coreset residual

__device__ __forceinline__ double uniform_at(uint64_t seed, uint64_t salt, int64_t i) {
  return static_cast<double>(splitmix64(seed ^ salt, static_cast<uint64_t>(i)) >> 11) * 0x1.0p-53;
}

// Block sums of the kT threads' values (fixed order), written by thread 0.
__device__ __forceinline__ void block_partial(double v, double* sh, double* out) {
  v = block_sum(v, sh);
  if (threadIdx.x == 0) *out = v;
}

// out[i] = x_i^e (x >= 0); partial[b] = block sums.
__global__ __launch_bounds__(kT) void k_pow_rows(int64_t n, const double* __restrict__ x, double e,
                                                 double* __restrict__ out, double* __restrict__ partial) {
  __shared__ double sh[kT / kWave];
  double s = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kT) {
    const double v = pow(x[i], e);
    out[i] = v;
    s += v;
  }
  block_partial(s, sh, partial + blockIdx.x);
}

// |U_i|^p for the residual U = b - A x of a pass; partial[b] = block sums.
__global__ __launch_bounds__(kT) void k_abs_pow_rows(int64_t n, const double* __restrict__ U, double p,
                                                     double* __restrict__ out, double* __restrict__ partial) {
  __shared__ double sh[kT / kWave];
  double s = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kT) {
    const double v = pow(fabs(U[i]), p);
    if (out) out[i] = v;
    s += v;
  }
  block_partial(s, sh, partial + blockIdx.x);
}

// out[j] = sum_b partial[j * nb + b], j < m: one block of kT threads, thread
// t summing b = t, t + kT, ... before the block sum (fixed order).
__global__ __launch_bounds__(kT) void k_sum_partials(const double* __restrict__ partial, int nb, int m,
                                                     double* __restrict__ out) {
  __shared__ double sh[kT / kWave];
  for (int j = 0; j < m; ++j) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kT) s += partial[j * nb + b];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[j] = s;
    __syncthreads();
  }
}

// k_sum_partials for the two interior-point sums (gap, objective), which it
// also writes with the factor status straight to pinned host memory.
__global__ __launch_bounds__(kT) void k_gap_publish(const double* __restrict__ partial, int nb,
                                                    double* __restrict__ out, const int32_t* __restrict__ status,
                                                    double* host_g, int32_t* host_st) {
  __shared__ double sh[kT / kWave];
  for (int j = 0; j < 2; ++j) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kT) s += partial[j * nb + b];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) {
      out[j] = s;
      host_g[j] = s;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) host_st[0] = status[0];
}

__device__ __forceinline__ double block_min(double v, double* sh) {
  for (int off = kWave / 2; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, kWave));
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double m = sh[0];
  for (int k = 1; k < kT / kWave; ++k) m = fmin(m, sh[k]);
  return m;
}

// Bernoulli draws: prob_i = min(1, s * share_i), share_i = lam_i / L, or
// max(lam_i / L, rp_i / Rt) when rp is given and Rt > 0 (sums = {L, Rt}).
__global__ __launch_bounds__(kT) void k_bernoulli(int64_t n, const double* __restrict__ lam,
                                                  const double* __restrict__ rp, const double* __restrict__ sums,
                                                  double s, uint64_t seed, uint64_t salt, int32_t* __restrict__ flag,
                                                  double* __restrict__ prob) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x;
  if (i >= n) return;
  double share = lam[i] / sums[0];
  if (rp != nullptr && sums[1] > 0.0) share = fmax(share, rp[i] / sums[1]);
  const double pr = fmin(1.0, s * share);
  prob[i] = pr;
  flag[i] = uniform_at(seed, salt, i) < pr ? 1 : 0;
}

// Kept rows in row order with weights prob^{-1/p}; pos = exclusive scan of
// flag; rows past the capacity are not written (the host rejects the draw).
__global__ __launch_bounds__(kT) void k_take(int64_t n, const int32_t* __restrict__ flag,
                                             const int32_t* __restrict__ pos, const double* __restrict__ prob,
                                             double p, int64_t cap, int32_t* __restrict__ list,
                                             double* __restrict__ wts) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x;
  if (i >= n || !flag[i] || pos[i] >= cap) return;
  list[pos[i]] = static_cast<int32_t>(i);
  wts[pos[i]] = pow(prob[i], -1.0 / p);
}

// out_i = M_i x - y_i (y may be NULL), one wavefront per row; with partial
// (grid of kResBlocks): partial[b] = block sum of |out_i|^p,
// partial[kResBlocks + b] = of |out_i|, partial[2 kResBlocks + b] = of |y_i|.
__global__ __launch_bounds__(kT) void k_resid_rows(int64_t ns, int64_t d, const double* __restrict__ M,
                                                   const double* __restrict__ x, const double* __restrict__ y,
                                                   double* __restrict__ out, double p,
                                                   double* __restrict__ partial) {
  __shared__ double sh[kT / kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t nw = static_cast<int64_t>(gridDim.x) * (kT / kWave);
  double sp = 0.0, s1 = 0.0, sy = 0.0;
  for (int64_t r = blockIdx.x * static_cast<int64_t>(kT / kWave) + threadIdx.x / kWave; r < ns; r += nw) {
    const double* row = M + static_cast<size_t>(r) * d;
    double s = 0.0;
    for (int64_t c = lane; c < d; c += kWave) s += row[c] * x[c];
    s = wave_total(s);
    const double yr = y ? y[r] : 0.0;
    const double v = s - yr;
    if (lane == 0) {
      out[r] = v;
      sp += pow(fabs(v), p);
      s1 += fabs(v);
      sy += fabs(yr);
    }
  }
  if (partial == nullptr) return;
  block_partial(sp, sh, partial + blockIdx.x);
  __syncthreads();
  block_partial(s1, sh, partial + kResBlocks + blockIdx.x);
  __syncthreads();
  block_partial(sy, sh, partial + 2 * kResBlocks + blockIdx.x);
}

// out[i][:] = c_i M[i][:] (c_i = sqrt(cw_i) when SQ), vout_i = c_i y_i.
template <bool SQ>
__global__ __launch_bounds__(kT) void k_scale_rows(int64_t ns, int64_t d, const double* __restrict__ M,
                                                   const double* __restrict__ y, const double* __restrict__ cw,
                                                   double* __restrict__ out, double* __restrict__ vout) {
  const int64_t total = ns * d;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * kT) {
    const int64_t r = e / d;
    const double c = SQ ? sqrt(cw[r]) : cw[r];
    out[e] = c * M[e];
    if (vout != nullptr && e - r * d == 0) vout[r] = c * y[r];
  }
}

// IRLS row weights: c_i = max(|r_i|, eta)^e.
__global__ __launch_bounds__(kT) void k_irls_weights(int64_t ns, const double* __restrict__ r, double eta, double e,
                                                     double* __restrict__ c) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x;
  if (i < ns) c[i] = pow(fmax(fabs(r[i]), eta), e);
}

// d-vectors: out = a - b; x = x + t (y - x); x += (*alpha) v.
__global__ void k_vlerp(int64_t d, const double* __restrict__ x, const double* __restrict__ y, double t,
                        double* __restrict__ out) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x;
  if (i < d) out[i] = x[i] + t * (y[i] - x[i]);
}

// ---------------------------------------------------------------- l_1 fit
// Dual of min ||M x - y||_1: max y^T a s.t. M^T a = c (= M^T 1/2), 0 <= a <= 1,
// slack sl = 1 - a, multipliers z (a >= 0) and w (a <= 1), with
// M x - z + w = y.  r = M x - y below.
__global__ __launch_bounds__(kT) void k_ipm_init(int64_t ns, const double* __restrict__ r, double delta,
                                                 double* __restrict__ a, double* __restrict__ sl,
                                                 double* __restrict__ z, double* __restrict__ w) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x;
  if (i >= ns) return;
  const double rr = -r[i];  // y - M x
  a[i] = 0.5;
  sl[i] = 0.5;
  w[i] = fmax(rr, 0.0) + delta;
  z[i] = fmax(-rr, 0.0) + delta;
}

// Duality gap sum(a z + sl w) -> partial[b]; sum |r| -> partial[kRed + b].
__global__ __launch_bounds__(kT) void k_ipm_gap(int64_t ns, const double* __restrict__ a,
                                                const double* __restrict__ sl, const double* __restrict__ z,
                                                const double* __restrict__ w, const double* __restrict__ r,
                                                double* __restrict__ partial) {
  __shared__ double sh[kT / kWave];
  double g = 0.0, f = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x; i < ns;
       i += static_cast<int64_t>(gridDim.x) * kT) {
    g += a[i] * z[i] + sl[i] * w[i];
    f += fabs(r[i]);
  }
  block_partial(g, sh, partial + blockIdx.x);
  __syncthreads();
  block_partial(f, sh, partial + kRed + blockIdx.x);
}

// Right-hand side of the reduced Newton system.  Predictor (CORR false):
// complementarity targets 0; corrector: sigma mu minus the predictor's
// second-order terms.  qi = 1 / (z/a + w/sl), qrho = qi rho.
template <bool CORR>
__global__ __launch_bounds__(kT) void k_ipm_rhs(int64_t ns, const double* __restrict__ r,
                                                const double* __restrict__ a, const double* __restrict__ sl,
                                                const double* __restrict__ z, const double* __restrict__ w,
                                                const double* __restrict__ da, const double* __restrict__ dz,
                                                const double* __restrict__ dw, const double* __restrict__ smu,
                                                double* __restrict__ qi, double* __restrict__ rho,
                                                double* __restrict__ qrho, double* __restrict__ r4,
                                                double* __restrict__ r5) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x;
  if (i >= ns) return;
  const double ai = a[i], si = sl[i], zi = z[i], wi = w[i];
  const double r3 = -r[i] + zi - wi;
  const double q = 1.0 / (zi / ai + wi / si);
  double t4 = -ai * zi, t5 = -si * wi;
  if (CORR) {
    const double ds = -da[i];
    t4 = smu[0] - ai * zi - da[i] * dz[i];
    t5 = smu[0] - si * wi - ds * dw[i];
  }
  const double rh = r3 + t4 / ai - t5 / si;
  qi[i] = q;
  rho[i] = rh;
  qrho[i] = q * rh;
  r4[i] = t4;
  r5[i] = t5;
}

// Directions from dx (Mdx = M dx) and the largest feasible step in [0, 1]
// for (a, sl) and for (z, w): partial[b], partial[kRed + b] (block minima).
__global__ __launch_bounds__(kT) void k_ipm_dirs(int64_t ns, const double* __restrict__ qi,
                                                 const double* __restrict__ rho, const double* __restrict__ Mdx,
                                                 const double* __restrict__ a, const double* __restrict__ sl,
                                                 const double* __restrict__ z, const double* __restrict__ w,
                                                 const double* __restrict__ r4, const double* __restrict__ r5,
                                                 double* __restrict__ da, double* __restrict__ dz,
                                                 double* __restrict__ dw, double* __restrict__ partial) {
  __shared__ double sh[2][kT];
  double mp = 1.0, md = 1.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x; i < ns;
       i += static_cast<int64_t>(gridDim.x) * kT) {
    const double dai = qi[i] * (rho[i] - Mdx[i]);
    const double dsi = -dai;
    const double dzi = (r4[i] - z[i] * dai) / a[i];
    const double dwi = (r5[i] - w[i] * dsi) / sl[i];
    da[i] = dai;
    dz[i] = dzi;
    dw[i] = dwi;
    if (dai < 0.0) mp = fmin(mp, -a[i] / dai);
    if (dsi < 0.0) mp = fmin(mp, -sl[i] / dsi);
    if (dzi < 0.0) md = fmin(md, -z[i] / dzi);
    if (dwi < 0.0) md = fmin(md, -w[i] / dwi);
  }
  sh[0][threadIdx.x] = mp;
  sh[1][threadIdx.x] = md;
  __syncthreads();
  for (int off = kT / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      sh[0][threadIdx.x] = fmin(sh[0][threadIdx.x], sh[0][threadIdx.x + off]);
      sh[1][threadIdx.x] = fmin(sh[1][threadIdx.x], sh[1][threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = sh[0][0];
    partial[kRed + blockIdx.x] = sh[1][0];
  }
}

// steps = {factor * min(1, primal ratio), factor * min(1, dual ratio)}.
__global__ __launch_bounds__(kT) void k_ipm_steps(const double* __restrict__ partial, int nb, double factor,
                                                  double* __restrict__ steps) {
  __shared__ double sh[kT / kWave];
  for (int j = 0; j < 2; ++j) {
    double m = 1.0;
    for (int b = threadIdx.x; b < nb; b += kT) m = fmin(m, partial[j * nb + b]);
    m = block_min(m, sh);
    if (threadIdx.x == 0) steps[j] = factor * m;
    __syncthreads();
  }
}

// Gap after the predictor step -> partial[b].
__global__ __launch_bounds__(kT) void k_ipm_gaff(int64_t ns, const double* __restrict__ a,
                                                 const double* __restrict__ sl, const double* __restrict__ z,
                                                 const double* __restrict__ w, const double* __restrict__ da,
                                                 const double* __restrict__ dz, const double* __restrict__ dw,
                                                 const double* __restrict__ steps, double* __restrict__ partial) {
  __shared__ double sh[kT / kWave];
  const double ap = steps[0], ad = steps[1];
  double g = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x; i < ns;
       i += static_cast<int64_t>(gridDim.x) * kT) {
    const double ds = -da[i];
    g += (a[i] + ap * da[i]) * (z[i] + ad * dz[i]) + (sl[i] + ap * ds) * (w[i] + ad * dw[i]);
  }
  block_partial(g, sh, partial + blockIdx.x);
}

// smu = (gap_aff / gap)^3 * gap / (2 ns).
__global__ __launch_bounds__(kT) void k_ipm_sigma(const double* __restrict__ partial, int nb,
                                                  const double* __restrict__ gap, int64_t ns,
                                                  double* __restrict__ smu) {
  __shared__ double sh[kT / kWave];
  double g = 0.0;
  for (int b = threadIdx.x; b < nb; b += kT) g += partial[b];
  g = block_sum(g, sh);
  if (threadIdx.x != 0) return;
  const double ratio = g / gap[0];
  smu[0] = ratio * ratio * ratio * (gap[0] / (2.0 * static_cast<double>(ns)));
}

// M^T v for the ns x d coreset: block b sums its slice of rows into
// part[b][:] (threads over columns), then k_col_sum adds the slices in
// block order.
constexpr int kRmvBlocks = 256;
__global__ __launch_bounds__(kT) void k_rmatvec_part(int64_t ns, int64_t d, const double* __restrict__ M,
                                                     const double* __restrict__ v, double* __restrict__ part) {
  const int64_t r0 = blockIdx.x * ns / gridDim.x, r1 = (blockIdx.x + 1) * ns / gridDim.x;
  for (int64_t c = threadIdx.x; c < d; c += kT) {
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) s += M[static_cast<size_t>(r) * d + c] * v[r];
    part[static_cast<size_t>(blockIdx.x) * d + c] = s;
  }
}
// 8 columns per block, 32 threads per column: thread t sums slices t,
// t + 32, ..., then thread 0 of each column adds the 32 sums in order.
// out[c] = s_sum * (sum of the slices) + s_other * other[c] (other may be NULL).
__global__ __launch_bounds__(kT) void k_col_sum(int nb, int64_t d, const double* __restrict__ part,
                                                double* __restrict__ out, double s_sum,
                                                const double* __restrict__ other, double s_other) {
  __shared__ double sh[kT / 8][8];
  const int cc = threadIdx.x & 7, t = threadIdx.x >> 3;
  const int64_t c = blockIdx.x * static_cast<int64_t>(8) + cc;
  double s = 0.0;
  if (c < d)
    for (int b = t; b < nb; b += kT / 8) s += part[static_cast<size_t>(b) * d + c];
  sh[t][cc] = s;
  __syncthreads();
  if (t == 0 && c < d) {
    double tot = 0.0;
    for (int k = 0; k < kT / 8; ++k) tot += sh[k][cc];
    out[c] = other != nullptr ? s_sum * tot + s_other * other[c] : s_sum * tot;
  }
}

// The step on the duals and slacks; x (d entries) is first copied to save
// and then moved by the dual step length along dx.
__global__ __launch_bounds__(kT) void k_ipm_update(int64_t ns, const double* __restrict__ steps,
                                                   double* __restrict__ a, double* __restrict__ sl,
                                                   double* __restrict__ z, double* __restrict__ w,
                                                   const double* __restrict__ da, const double* __restrict__ dz,
                                                   const double* __restrict__ dw, int64_t d,
                                                   const double* __restrict__ dx, double* __restrict__ x,
                                                   double* __restrict__ save) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x;
  for (int64_t j = i; j < d; j += static_cast<int64_t>(gridDim.x) * kT) {
    save[j] = x[j];
    x[j] += steps[1] * dx[j];
  }
  if (i >= ns) return;
  const double ap = steps[0], ad = steps[1];
  a[i] += ap * da[i];
  sl[i] -= ap * da[i];
  z[i] += ad * dz[i];
  w[i] += ad * dw[i];
}

// ---------------------------------------------------------------- workspace
struct LpWs {
  void* sk;
  size_t sk_bytes;
  double* FA;
  void* gram;
  size_t gram_bytes;
  double *G, *cholw, *R, *Rinv, *RinvT;
  int32_t* status;
  double *Pi2, *T, *Z, *score, *lam, *rp, *prob, *part, *rmv, *sums, *resid, *negx, *one, *ppart;
  int32_t *flag, *pos, *itiles, *last, *list;
  double* wts;
  // coreset
  double *Ms, *ys, *Mw, *yw, *r, *rt, *cw;
  double *a, *sl, *z, *w, *qi, *rho, *qrho, *r4, *r5, *da, *dz, *dw, *Mdx;
  double *x, *xn, *xt, *c, *r1, *rhs, *tmpd, *dx, *dev;
  GemmScratch gs;
};

LpWs carve_lp(Arena& ar, const LpPlan& P) {
  LpWs w;
  const int64_t n = P.n, d = P.d, cap = P.cap;
  w.sk_bytes = P.sk_bytes;
  w.sk = ar.take<char>(P.sk_bytes + 1);
  w.FA = ar.take<double>(static_cast<size_t>(P.nb) * P.t * d);
  size_t gb = gram_ws_bytes(static_cast<int64_t>(P.nb) * P.t, d);
  const size_t g2 = gram_ws_bytes(cap, d + 1);
  w.gram_bytes = gb > g2 ? gb : g2;
  w.gram = ar.take<double>(w.gram_bytes / sizeof(double) + 1);
  w.G = ar.take<double>(static_cast<size_t>(d + 1) * (d + 1));
  w.cholw = ar.take<double>(cholesky_scratch_doubles(d));
  w.R = ar.take<double>(static_cast<size_t>(d) * d);
  w.Rinv = ar.take<double>(static_cast<size_t>(d) * d);
  w.RinvT = ar.take<double>(static_cast<size_t>(d) * d);
  w.status = ar.take<int32_t>(4);
  w.Pi2 = ar.take<double>(static_cast<size_t>(d) * P.kg);
  w.T = ar.take<double>(static_cast<size_t>(d) * P.kg);
  w.Z = ar.take<double>(static_cast<size_t>(n) * P.kg);
  w.score = ar.take<double>(n);
  w.lam = ar.take<double>(n);
  w.rp = ar.take<double>(n);
  w.prob = ar.take<double>(n);
  w.resid = ar.take<double>(n);
  w.part = ar.take<double>(3 * kResBlocks + 2 * kRed);
  w.rmv = ar.take<double>(static_cast<size_t>(kRmvBlocks) * d);
  w.sums = ar.take<double>(8);
  w.negx = ar.take<double>(d);
  w.one = ar.take<double>(2);
  w.ppart = ar.take<double>(static_cast<size_t>(pass_blocks(*P.A)) * (d + 1));
  w.flag = ar.take<int32_t>(n);
  w.pos = ar.take<int32_t>(n);
  w.itiles = ar.take<int32_t>(tiles_for(n));
  w.last = ar.take<int32_t>(4);
  w.list = ar.take<int32_t>(cap);
  w.wts = ar.take<double>(cap);
  w.Ms = ar.take<double>(static_cast<size_t>(cap) * d);
  w.Mw = ar.take<double>(static_cast<size_t>(cap) * d);
  w.ys = ar.take<double>(cap);
  w.yw = ar.take<double>(cap);
  double** vecs[] = {&w.r, &w.rt, &w.cw, &w.a, &w.sl, &w.z, &w.w, &w.qi, &w.rho, &w.qrho, &w.r4, &w.r5,
                     &w.da, &w.dz, &w.dw, &w.Mdx};
  for (double** v : vecs) *v = ar.take<double>(cap);
  double** dvecs[] = {&w.x, &w.xn, &w.xt, &w.c, &w.r1, &w.rhs, &w.tmpd, &w.dx};
  for (double** v : dvecs) *v = ar.take<double>(d);
  w.dev = ar.take<double>(16);  // gap, pobj, steps[2], smu, -, -, -, coreset sums[3]
  w.gs.doubles = size_t(1) << 21;
  w.gs.part = ar.take<double>(w.gs.doubles);
  return w;
}

unsigned g_rows(int64_t n) { return grid_for(n, kT, 1u << 24); }

// out = M^T v for the coreset rows (ns x d, row-major).
int32_t rmatvec(const LpWs& w, int64_t ns, int64_t d, const double* v, double* out, hipStream_t s,
                double s_sum = 1.0, const double* other = nullptr, double s_other = 0.0) {
  hipLaunchKernelGGL(k_rmatvec_part, dim3(kRmvBlocks), dim3(kT), 0, s, ns, d, w.Ms, v, w.rmv);
  SKLS_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_col_sum, dim3(static_cast<unsigned>(div_up(d, 8))), dim3(kT), 0, s, kRmvBlocks, d, w.rmv,
                     out, s_sum, other, s_other);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

// ---------------------------------------------------------------- fits
struct Fit {
  int iters = 0;
  bool converged = false;
  double obj = 0.0;  // weighted objective sum |M x - y|^p at the result
};

// Weighted normal equations of the coreset rows scaled by cw (sqrt of cw
// when SQ): G = Mw^T Mw (with Mw^T yw appended when with_y), Cholesky, and
// the inverse factor.  With bad given, the Cholesky status is read back now
// (*bad = 1, and no inverse, when the factor broke down); without it the
// status stays on the device for the caller's next read.
template <bool SQ>
int32_t factor_weighted(const LpWs& w, int64_t ns, int64_t d, const double* cw, bool with_y, int32_t* bad,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_scale_rows<SQ>, dim3(grid_for(ns * d, kT, 8192)), dim3(kT), 0, s, ns, d, w.Ms, w.ys, cw,
                     w.Mw, with_y ? w.yw : nullptr);
  SKLS_CHECK_LAUNCH();
  const int64_t dd = with_y ? d + 1 : d;
  SKLS_TRY(run_gram(w.Mw, SKLS_F64, d, with_y ? w.yw : nullptr, SKLS_F64, ns, d, w.G, w.gram, w.gram_bytes, s));
  SKLS_TRY(run_cholesky(w.G, dd, d, w.R, w.Rinv, w.RinvT, w.status, w.cholw, s));
  if (bad != nullptr) {
    int32_t st = 0;
    SKLS_TRY(to_host(&st, w.status, sizeof st, s));
    *bad = st;
  }
  return SKLS_OK;
}

// r = M x - y on the coreset; f = sum |r|^p, f1 = sum |r|, fy = sum |y|;
// chol_bad (if given) receives the status of the last factorization.
int32_t resid(const LpWs& w, int64_t ns, int64_t d, const double* x, double* r, double p, double* f, double* f1,
              double* fy, hipStream_t s, int32_t* chol_bad = nullptr) {
  hipLaunchKernelGGL(k_resid_rows, dim3(kResBlocks), dim3(kT), 0, s, ns, d, w.Ms, x, w.ys, r, p, w.part);
  SKLS_CHECK_LAUNCH();
  // dev[8..10]: sums[0..1] hold the sampling totals for the whole call
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kT), 0, s, w.part, kResBlocks, 3, w.dev + 8);
  SKLS_CHECK_LAUNCH();
  if (chol_bad) SKLS_TRY_HIP(hipMemcpyAsync(chol_bad, w.status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  double h[3];
  SKLS_TRY(to_host(h, w.dev + 8, sizeof h, s));
  *f = h[0];
  if (f1) *f1 = h[1];
  if (fy) *fy = h[2];
  return SKLS_OK;
}

// The least-squares start fits every kept row to rounding: it solves the
// consistent system, which is optimal for every p.
bool exact_start(double f1, double fy, int64_t d) { return f1 <= 16.0 * static_cast<double>(d) * 0x1.0p-53 * fy; }

__global__ void k_fill(int64_t n, double v, double* __restrict__ p) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x;
  if (i < n) p[i] = v;
}

int32_t fill_value(double* p, int64_t n, double v, hipStream_t s) {
  if (n == 0) return SKLS_OK;
  hipLaunchKernelGGL(k_fill, dim3(g_rows(n)), dim3(kT), 0, s, n, v, p);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

// Least squares on the coreset rows scaled by cw; bad as for
// factor_weighted (NULL: the status is left on the device).
int32_t weighted_ls(const LpWs& w, int64_t ns, int64_t d, const double* cw, double* x, int32_t* bad,
                    hipStream_t s) {
  SKLS_TRY(factor_weighted<false>(w, ns, d, cw, true, bad, s));
  if (bad != nullptr && *bad) return SKLS_OK;
  return run_solve_from_gram(w.Rinv, w.RinvT, w.G + d * (d + 1), d, x, w.tmpd, s);
}

int32_t irls_ahead(const LpWs& w, int64_t ns, int64_t d, double p, int max_iter, double tol, double f0, double eta0,
                   double emin, Fit& out, hipStream_t s);

int32_t fit_irls(const LpWs& w, int64_t ns, int64_t d, double p, int max_iter, double tol, Fit& out,
                 hipStream_t s) {
  int32_t bad = 0;
  SKLS_TRY(fill_value(w.cw, ns, 1.0, s));
  SKLS_TRY(weighted_ls(w, ns, d, w.cw, w.x, &bad, s));
  if (bad) {
    set_error("lp_regression: the sampled rows are numerically rank deficient (raise s1 or s2)");
    return SKLS_ERR_RANK;
  }
  double f = 0.0, f1 = 0.0, fy = 0.0;
  SKLS_TRY(resid(w, ns, d, w.x, w.r, p, &f, &f1, &fy, s));
  out.iters = 1;
  if (p == 2.0 || exact_start(f1, fy, d)) {
    out.converged = true;
    out.obj = f;
    return SKLS_OK;
  }
  double eta = f1 / static_cast<double>(ns);
  const double emin = 1e-9 * eta;
  if (p < 2.0) return irls_ahead(w, ns, d, p, max_iter, tol, f, eta, emin, out, s);
  double* r = w.r;
  double* rt = w.rt;
  for (int it = 0; it < max_iter; ++it) {
    hipLaunchKernelGGL(k_irls_weights, dim3(g_rows(ns)), dim3(kT), 0, s, ns, r, eta, (p - 2.0) / 2.0, w.cw);
    SKLS_CHECK_LAUNCH();
    SKLS_TRY(weighted_ls(w, ns, d, w.cw, w.xn, nullptr, s));  // status read with the residual below
    double th = p <= 2.0 ? 1.0 : 1.0 / (p - 1.0);
    double ft = 0.0;
    for (;;) {
      hipLaunchKernelGGL(k_vlerp, dim3(g_rows(d)), dim3(kT), 0, s, d, w.x, w.xn, th, w.xt);
      SKLS_CHECK_LAUNCH();
      SKLS_TRY(resid(w, ns, d, w.xt, rt, p, &ft, nullptr, nullptr, s, &bad));
      if (bad || ft <= f || th < 1e-6 || p < 2.0) break;
      th *= 0.5;
    }
    if (bad) break;  // the factor broke down: keep the last iterate
    const bool done = eta <= emin && std::fabs(f - ft) <= tol * f;
    SKLS_TRY_HIP(hipMemcpyAsync(w.x, w.xt, sizeof(double) * d, hipMemcpyDeviceToDevice, s));
    std::swap(r, rt);
    f = ft;
    eta = std::max(emin, eta * 0.25);
    out.iters = it + 2;
    if (done) {
      out.converged = true;
      break;
    }
  }
  out.obj = f;
  return SKLS_OK;
}

// One reduced Newton solve: rhs = M^T qrho - r1, dx = (M^T Q M)^{-1} rhs,
// Mdx = M dx, then the directions and step bounds.
int32_t ipm_direction(const LpWs& w, int64_t ns, int64_t d, double factor, hipStream_t s) {
  SKLS_TRY(rmatvec(w, ns, d, w.qrho, w.rhs, s, 1.0, w.r1, -1.0));  // rhs = M^T qrho - r1
  SKLS_TRY(run_solve_from_gram(w.Rinv, w.RinvT, w.rhs, d, w.dx, w.tmpd, s));
  hipLaunchKernelGGL(k_resid_rows, dim3(kResBlocks), dim3(kT), 0, s, ns, d, w.Ms, w.dx, nullptr, w.Mdx, 1.0,
                     nullptr);
  SKLS_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_ipm_dirs, dim3(kRed), dim3(kT), 0, s, ns, w.qi, w.rho, w.Mdx, w.a, w.sl, w.z, w.w, w.r4,
                     w.r5, w.da, w.dz, w.dw, w.part);
  SKLS_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_ipm_steps, dim3(1), dim3(kT), 0, s, w.part, kRed, factor, w.dev + 2);
  SKLS_CHECK_LAUNCH();
  return SKLS_OK;
}

// Pinned host memory for reads that must not wait for later work on the
// stream: two slots of (gap, objective) and the factor status.  One small
// buffer per host thread, allocated on first use and kept.
// Coherent, so that a kernel's stores reach it without a copy.
struct GapSlots {
  double g[2][2];
  int32_t st[2];
};
GapSlots* gap_slots() {
  thread_local GapSlots* p = nullptr;
  if (p == nullptr) {
    void* q = nullptr;
    if (hipHostMalloc(&q, sizeof(GapSlots), hipHostMallocCoherent) == hipSuccess) p = static_cast<GapSlots*>(q);
  }
  return p;
}

int32_t fit_l1(const LpWs& w, int64_t ns, int64_t d, int max_iter, double tol, Fit& out, hipStream_t s) {
  int32_t bad = 0;
  SKLS_TRY(fill_value(w.cw, ns, 1.0, s));
  SKLS_TRY(weighted_ls(w, ns, d, w.cw, w.x, &bad, s));
  if (bad) {
    set_error("lp_regression: the sampled rows are numerically rank deficient (raise s1 or s2)");
    return SKLS_ERR_RANK;
  }
  double f = 0.0, f1 = 0.0, fy = 0.0;
  SKLS_TRY(resid(w, ns, d, w.x, w.r, 1.0, &f, &f1, &fy, s));
  out.iters = 1;
  out.obj = f;
  if (exact_start(f1, fy, d)) {
    out.converged = true;
    return SKLS_OK;
  }
  GapSlots* hs = gap_slots();
  if (hs == nullptr) {
    set_error("lp_regression: no pinned host memory for the gap reads");
    return SKLS_ERR_DEVICE;
  }
  GapSlots* dg = nullptr;  // the same memory as the device addresses it
  SKLS_TRY_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&dg), hs, 0));
  hipEvent_t ev[2];
  SKLS_TRY_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  if (hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    set_error("lp_regression: hipEventCreate failed");
    return SKLS_ERR_DEVICE;
  }
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      (void)hipEventDestroy(e[0]);
      (void)hipEventDestroy(e[1]);
    }
  } guard{ev};
  const unsigned g = g_rows(ns);
  hipLaunchKernelGGL(k_ipm_init, dim3(g), dim3(kT), 0, s, ns, w.r, f1 / static_cast<double>(ns), w.a, w.sl, w.z,
                     w.w);
  SKLS_CHECK_LAUNCH();
  // c = M^T a at the start (a = 1/2): the dual equality M^T a = c holds there
  SKLS_TRY(rmatvec(w, ns, d, w.a, w.c, s));
  // x before step it is kept in save[it & 1] (two slots: a step taken ahead
  // of its decision may have to be undone, and so may the one before it)
  double* save[2] = {w.xt, w.xn};
  // the duality gap and objective at the current iterate, and the status of
  // the factor of the step that led to it, into pinned slot k
  auto gap = [&](int k) -> int32_t {
    hipLaunchKernelGGL(k_resid_rows, dim3(kResBlocks), dim3(kT), 0, s, ns, d, w.Ms, w.x, w.ys, w.r, 1.0, nullptr);
    SKLS_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_ipm_gap, dim3(kRed), dim3(kT), 0, s, ns, w.a, w.sl, w.z, w.w, w.r, w.part);
    SKLS_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_gap_publish, dim3(1), dim3(kT), 0, s, w.part, kRed, w.dev, w.status, dg->g[k],
                       &dg->st[k]);
    SKLS_CHECK_LAUNCH();
    SKLS_TRY_HIP(hipEventRecord(ev[k], s));
    return SKLS_OK;
  };
  // one predictor-corrector step from the current iterate
  auto step = [&](int it) -> int32_t {
    // r1 = c - M^T a
    SKLS_TRY(rmatvec(w, ns, d, w.a, w.r1, s, -1.0, w.c, 1.0));
    // predictor
    hipLaunchKernelGGL(k_ipm_rhs<false>, dim3(g), dim3(kT), 0, s, ns, w.r, w.a, w.sl, w.z, w.w, w.da, w.dz, w.dw,
                       w.dev + 4, w.qi, w.rho, w.qrho, w.r4, w.r5);
    SKLS_CHECK_LAUNCH();
    SKLS_TRY(factor_weighted<true>(w, ns, d, w.qi, false, nullptr, s));  // status read with the next gap
    SKLS_TRY(ipm_direction(w, ns, d, 1.0, s));
    hipLaunchKernelGGL(k_ipm_gaff, dim3(kRed), dim3(kT), 0, s, ns, w.a, w.sl, w.z, w.w, w.da, w.dz, w.dw,
                       w.dev + 2, w.part);
    SKLS_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_ipm_sigma, dim3(1), dim3(kT), 0, s, w.part, kRed, w.dev, ns, w.dev + 4);
    SKLS_CHECK_LAUNCH();
    // corrector
    hipLaunchKernelGGL(k_ipm_rhs<true>, dim3(g), dim3(kT), 0, s, ns, w.r, w.a, w.sl, w.z, w.w, w.da, w.dz, w.dw,
                       w.dev + 4, w.qi, w.rho, w.qrho, w.r4, w.r5);
    SKLS_CHECK_LAUNCH();
    SKLS_TRY(ipm_direction(w, ns, d, 0.99995, s));
    // the duals and slacks, and x (saved first) by the dual step along dx
    hipLaunchKernelGGL(k_ipm_update, dim3(g), dim3(kT), 0, s, ns, w.dev + 2, w.a, w.sl, w.z, w.w, w.da, w.dz,
                       w.dw, d, w.dx, w.x, save[it & 1]);
    SKLS_CHECK_LAUNCH();
    return SKLS_OK;
  };
  auto restore = [&](int from) -> int32_t {
    SKLS_TRY_HIP(hipMemcpyAsync(w.x, save[from & 1], sizeof(double) * d, hipMemcpyDeviceToDevice, s));
    return SKLS_OK;
  };
  // Iteration it reads gap(it) while step(it), enqueued ahead of the
  // decision, already runs: the host's round trip is hidden behind the
  // step.  The iterates accepted are those of the plain loop (read the gap,
  // then step); a step taken ahead and not wanted is undone.
  SKLS_TRY(gap(0));
  if (max_iter > 0) SKLS_TRY(step(0));
  for (int it = 0; it <= max_iter; ++it) {
    const int k = it & 1;
    SKLS_TRY_HIP(hipEventSynchronize(ev[k]));
    const double hgap = hs->g[k][0], hobj = hs->g[k][1];
    const int32_t st = it > 0 ? hs->st[k] : 0;
    const bool ahead = it < max_iter;  // step(it) was enqueued
    if (st) {  // the factor of step(it - 1) broke down: back to the iterate before it
      SKLS_TRY(restore(it - 1));
      out.iters = it;
      break;
    }
    out.obj = hobj;
    if (hgap <= tol * std::max(1.0, hobj)) {
      if (ahead) SKLS_TRY(restore(it));
      out.converged = true;
      break;
    }
    if (!ahead) break;
    out.iters = it + 2;  // the least-squares start and it + 1 interior-point steps
    SKLS_TRY(gap(k ^ 1));
    if (it + 1 < max_iter) SKLS_TRY(step(it + 1));
  }
  SKLS_TRY_HIP(hipStreamSynchronize(s));
  return SKLS_OK;
}

// IRLS for 1 < p < 2 from the least-squares start (x_0 = w.x, r_0 = w.r,
// objective f0), with each iteration's objective and factor status read one
// iteration late.  Below p = 2 the step is taken in full, and the weights of
// the next iteration need only the residual on the device and eta, whose
// schedule is fixed.  So iteration k + 1 is enqueued before iteration k's
// result is read, and the host's round trip hides behind it.  Iterates live
// in a ring of three: x_{k+1} may already be enqueued when a broken factor in
// step k makes x_{k-1} the answer.  Residuals live in a ring of two.  The
// iterates, decisions and result are those of the plain loop in fit_irls.
int32_t irls_ahead(const LpWs& w, int64_t ns, int64_t d, double p, int max_iter, double tol, double f0, double eta0,
                   double emin, Fit& out, hipStream_t s) {
  GapSlots* hs = gap_slots();
  if (hs == nullptr) {
    set_error("lp_regression: no pinned host memory for the objective reads");
    return SKLS_ERR_DEVICE;
  }
  GapSlots* dg = nullptr;  // the same memory as the device addresses it
  SKLS_TRY_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&dg), hs, 0));
  hipEvent_t ev[2];
  SKLS_TRY_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  if (hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    set_error("lp_regression: hipEventCreate failed");
    return SKLS_ERR_DEVICE;
  }
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      (void)hipEventDestroy(e[0]);
      (void)hipEventDestroy(e[1]);
    }
  } guard{ev};
  double* X[3] = {w.x, w.xt, w.dx};  // x_k in X[k % 3] (dx is free outside the interior point)
  double* Rr[2] = {w.r, w.rt};        // r_k in Rr[k % 2]
  // eta of iteration k >= 1: eta0, then a quarter of the last, floored at emin
  auto eta_of = [&](int k) {
    double e = eta0;
    for (int i = 1; i < k; ++i) e = std::max(emin, e * 0.25);
    return e;
  };
  // iteration k from x_{k-1} and r_{k-1}: its objective and factor status go
  // to pinned slot k % 2
  auto iter = [&](int k) -> int32_t {
    hipLaunchKernelGGL(k_irls_weights, dim3(g_rows(ns)), dim3(kT), 0, s, ns, Rr[(k - 1) & 1], eta_of(k),
                       (p - 2.0) / 2.0, w.cw);
    SKLS_CHECK_LAUNCH();
    SKLS_TRY(weighted_ls(w, ns, d, w.cw, w.xn, nullptr, s));
    hipLaunchKernelGGL(k_vlerp, dim3(g_rows(d)), dim3(kT), 0, s, d, X[(k - 1) % 3], w.xn, 1.0, X[k % 3]);
    SKLS_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_resid_rows, dim3(kResBlocks), dim3(kT), 0, s, ns, d, w.Ms, X[k % 3], w.ys, Rr[k & 1], p,
                       w.part);
    SKLS_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_gap_publish, dim3(1), dim3(kT), 0, s, w.part, kResBlocks, w.dev + 8, w.status,
                       dg->g[k & 1], &dg->st[k & 1]);
    SKLS_CHECK_LAUNCH();
    SKLS_TRY_HIP(hipEventRecord(ev[k & 1], s));
    return SKLS_OK;
  };
  double f = f0;
  int result = 0;
  if (max_iter > 0) SKLS_TRY(iter(1));
  for (int k = 1; k <= max_iter; ++k) {
    if (k + 1 <= max_iter) SKLS_TRY(iter(k + 1));  // ahead of the decision on k
    SKLS_TRY_HIP(hipEventSynchronize(ev[k & 1]));
    const double fk = hs->g[k & 1][0];
    if (hs->st[k & 1]) break;  // the factor of step k broke down: keep x_{k-1}
    const bool done = eta_of(k) <= emin && std::fabs(f - fk) <= tol * f;
    f = fk;
    result = k;
    out.iters = k + 1;
    if (done) {
      out.converged = true;
      break;
    }
  }
  // x_result is intact: the iterations enqueued after it wrote the other slots
  if (result % 3 != 0)
    SKLS_TRY_HIP(hipMemcpyAsync(w.x, X[result % 3], sizeof(double) * d, hipMemcpyDeviceToDevice, s));
  out.obj = f;
  SKLS_TRY_HIP(hipStreamSynchronize(s));
  return SKLS_OK;
}

int32_t fit(const LpWs& w, int64_t ns, int64_t d, double p, int max_iter, double tol, Fit& out, hipStream_t s) {
  if (p == 1.0) return fit_l1(w, ns, d, max_iter, tol, out, s);
  return fit_irls(w, ns, d, p, max_iter, tol, out, s);
}

// Rows [r0, r1) of A as a matrix of its own (CSR keeps absolute offsets).
skls_matrix row_view(const skls_matrix& A, int64_t r0, int64_t r1) {
  skls_matrix V = A;
  V.n = r1 - r0;
  if (A.layout == SKLS_CSR) {
    const size_t es = A.row_ptr_64 ? 8 : 4;
    V.row_ptr = static_cast<const char*>(A.row_ptr) + static_cast<size_t>(r0) * es;
    // the entry count only steers the lanes per row
    V.nnz = A.n > 0 ? static_cast<int64_t>(static_cast<double>(A.nnz) * V.n / A.n) : 0;
  } else {
    V.val = static_cast<const char*>(A.val) + static_cast<size_t>(r0) * A.ld * dtype_size(A.dtype);
  }
  return V;
}

// ||A x - b||_p^p over all rows by one pass (U = b - A x); |U_i|^p kept in
// rp when given.
int32_t full_objective(const skls_matrix& A, const double* b, const LpWs& w, const double* x, double p, double* rp,
                       double* obj, hipStream_t s) {
  const int64_t n = A.n, d = A.d;
  SKLS_TRY_HIP(hipMemcpyAsync(w.negx, x, sizeof(double) * d, hipMemcpyDeviceToDevice, s));
  SKLS_TRY(launch_scale(w.negx, static_cast<size_t>(d), SKLS_F64, -1.0, s));
  PassArgs pa{};
  pa.A = &A;
  pa.p = w.negx;
  pa.coef = w.one;
  pa.Z = b;
  pa.z_is_b = 1;
  pa.U = w.resid;
  pa.u_f64 = 1;
  pa.acc_f64 = 1;
  pa.partial = w.ppart;
  pa.nblk = pass_blocks(A);
  SKLS_TRY(run_pass(pa, s));
  hipLaunchKernelGGL(k_abs_pow_rows, dim3(kRed), dim3(kT), 0, s, n, w.resid, p, rp, w.part);
  SKLS_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kT), 0, s, w.part, kRed, 1, w.sums + 1);
  SKLS_CHECK_LAUNCH();
  return to_host(obj, w.sums + 1, sizeof(double), s);
}

// Bernoulli draw, compaction and gather of the coreset; returns its size.
int32_t draw_coreset(const skls_matrix& A, const double* b, const LpWs& w, const LpPlan& P, double sz, bool stage2,
                     int64_t* ns_out, hipStream_t s) {
  const int64_t n = A.n, d = A.d;
  hipLaunchKernelGGL(k_bernoulli, dim3(g_rows(n)), dim3(kT), 0, s, n, w.lam, stage2 ? w.rp : nullptr, w.sums, sz,
                     P.seed, stage2 ? kStage2Salt : kSampleSalt, w.flag, w.prob);
  SKLS_CHECK_LAUNCH();
  SKLS_TRY(scan<int32_t>(w.flag, n, w.itiles, w.pos, true, s));
  int32_t hv[2];
  SKLS_TRY_HIP(hipMemcpyAsync(&hv[0], w.pos + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
  SKLS_TRY(to_host(&hv[1], w.flag + (n - 1), sizeof(int32_t), s));
  const int64_t ns = static_cast<int64_t>(hv[0]) + hv[1];
  if (ns > P.cap) {
    set_error("lp_regression: %lld rows kept, more than the capacity %lld", static_cast<long long>(ns),
              static_cast<long long>(P.cap));
    return SKLS_ERR_SHAPE;
  }
  if (ns < d) {
    set_error("lp_regression: stage %d kept %lld rows, fewer than d = %lld (raise s%d)", stage2 ? 2 : 1,
              static_cast<long long>(ns), static_cast<long long>(d), stage2 ? 2 : 1);
    return SKLS_ERR_RANK;
  }
  hipLaunchKernelGGL(k_take, dim3(g_rows(n)), dim3(kT), 0, s, n, w.flag, w.pos, w.prob, P.p, P.cap, w.list, w.wts);
  SKLS_CHECK_LAUNCH();
  const unsigned gr = grid_for(ns, kT / kWave, 8192);
  int32_t st = with_value(A.dtype, [&](auto tv) -> int32_t {
    using TV = decltype(tv);
    if (A.layout != SKLS_CSR) {
      hipLaunchKernelGGL(k_gather_rows<TV>, dim3(gr), dim3(kT), 0, s, ns, d, A.ld, static_cast<const TV*>(A.val),
                         w.list, w.wts, w.Ms);
      SKLS_CHECK_LAUNCH();
      return SKLS_OK;
    }
    SKLS_TRY(launch_fill_zero(w.Ms, static_cast<size_t>(ns) * d * sizeof(double), s));
    return with_rowptr(A, [&](auto trt) -> int32_t {
      using TR = decltype(trt);
      hipLaunchKernelGGL((k_gather_csr_dense<TV, TR>), dim3(gr), dim3(kT), 0, s, ns, d,
                         static_cast<const TR*>(A.row_ptr), A.col_idx, static_cast<const TV*>(A.val), w.list, w.wts,
                         w.Ms);
      SKLS_CHECK_LAUNCH();
      return SKLS_OK;
    });
  });
  SKLS_TRY(st);
  hipLaunchKernelGGL(k_gather_rows<double>, dim3(gr), dim3(kT), 0, s, ns, 1, 1, b, w.list, w.wts, w.ys);
  SKLS_CHECK_LAUNCH();
  *ns_out = ns;
  return SKLS_OK;
}

}  // namespace

int32_t lp_plan(const skls_matrix& A, const skls_lp_opts& o, LpPlan& P) {
  P.A = &A;
  P.n = A.n;
  P.d = A.d;
  P.p = o.p;
  if (!(o.p >= 1.0) || !std::isfinite(o.p)) {
    set_error("lp_regression: need 1 <= p < inf");
    return SKLS_ERR_ARG;
  }
  if (A.n < A.d || A.n >= (int64_t(1) << 31) || A.d > 4096) {
    set_error("lp_regression: need d <= n < 2^31 and d <= 4096");
    return SKLS_ERR_SHAPE;
  }
  P.v = o.v > 0 ? o.v : 8;
  P.a = o.a > 0 ? o.a : 1;
  P.q = o.q > 0 ? o.q : std::max<int64_t>(16, div_up(2 * A.d * A.d, P.v));
  P.kg = o.k_g > 0 ? o.k_g : 32;
  P.w = (o.w > 0 && o.w < A.n) ? o.w : A.n;
  P.s1 = o.s1 > 0 ? o.s1 : 32.0 * static_cast<double>(A.d);
  P.s2 = o.s2 > 0 ? o.s2 : 32.0 * static_cast<double>(A.d);
  P.max_iter = o.max_iter > 0 ? o.max_iter : 100;
  P.tol = o.tol > 0 ? o.tol : 1e-12;
  P.seed = o.seed;
  if (o.a < 0 || o.a > 256 || o.k_g < 0 || P.kg > 64 || o.q < 0 || o.v < 0 || o.w < 0 || o.s1 < 0 || o.s2 < 0 ||
      o.max_iter < 0 || !(o.tol >= 0)) {
    set_error("lp_regression: need 0 <= a <= 256, 0 <= k_g <= 64 and non-negative sizes");
    return SKLS_ERR_ARG;
  }
  if (P.q * P.v >= (int64_t(1) << 31)) {
    set_error("lp_regression: need q v < 2^31");
    return SKLS_ERR_SHAPE;
  }
  P.t = P.q * P.v * P.a;
  P.nb = div_up(A.n, P.w);
  if (P.nb * P.t < A.d || P.nb * P.t >= (int64_t(1) << 31)) {
    set_error("lp_regression: need d <= (blocks) a q v < 2^31");
    return SKLS_ERR_SHAPE;
  }
  auto cap_of = [&](double s) {
    const double c = s + 8.0 * std::sqrt(s) + 64.0;
    return c >= static_cast<double>(A.n) ? A.n : static_cast<int64_t>(c);
  };
  P.cap = std::max(cap_of(P.s1), cap_of(2.0 * P.s2));
  const skls_matrix full = row_view(A, 0, P.w);
  const skls_matrix last = row_view(A, (P.nb - 1) * P.w, A.n);
  P.sk_bytes = std::max(sketch_ws_bytes(full, P.q * P.v, SKLS_SKETCH_AUTO),
                        sketch_ws_bytes(last, P.q * P.v, SKLS_SKETCH_AUTO));
  return SKLS_OK;
}

size_t lp_ws_bytes(const LpPlan& P) {
  Arena ar(nullptr, 0);
  carve_lp(ar, P);
  return ar.used;
}

int32_t run_lp(const skls_matrix& A, const double* b, const LpPlan& P, double* x, double* x_c, int32_t* rows1,
               double* w1, int32_t* rows2, double* w2, skls_lp_info* info, void* ws, size_t ws_bytes,
               hipStream_t s) {
  Arena ar(ws, ws_bytes);
  LpWs w = carve_lp(ar, P);
  if (!ar.fits() || ws == nullptr) {
    set_error("lp_regression: workspace too small (%zu bytes needed)", ar.used);
    return SKLS_ERR_WORKSPACE;
  }
  const int64_t n = P.n, d = P.d;
  const int kg = P.kg;
  skls_lp_info inf{};
  hipEvent_t ev[4];
  for (auto& e : ev) SKLS_TRY_HIP(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 4; ++i) (void)hipEventDestroy(e[i]);
    }
  } guard{ev};
  SKLS_TRY_HIP(hipEventRecord(ev[0], s));
  SKLS_TRY(fill_value(w.one, 1, 1.0, s));

  // ---- conditioning: F A, R, and the sampling weights lam = (row norms^2)^{p/2}
  {
    PhaseTimer pt("lp_condition", s);
    const int64_t tc = P.q * P.v;
    for (int64_t j = 0; j < P.nb; ++j) {
      const skls_matrix V = row_view(A, j * P.w, std::min(n, (j + 1) * P.w));
      for (int32_t c = 0; c < P.a; ++c) {
        HashKey key;
        key.seed = P.seed + static_cast<uint64_t>(c + 1) * 0xD1B54A32D192ED03ull;
        key.outer = P.seed;
        key.q = static_cast<uint32_t>(P.q);
        key.v = static_cast<uint32_t>(P.v);
        double* out = w.FA + (static_cast<size_t>(j) * P.t + static_cast<size_t>(c) * tc) * d;
        SKLS_TRY(run_sketch_key(V, nullptr, SKLS_F64, tc, key, nullptr, SKLS_SKETCH_AUTO, out, nullptr, SKLS_F64,
                                w.sk, w.sk_bytes, s));
      }
    }
    const int64_t m = P.nb * P.t;
    if (P.a > 1) SKLS_TRY(launch_scale(w.FA, static_cast<size_t>(m) * d, SKLS_F64, 1.0 / std::sqrt(double(P.a)), s));
    SKLS_TRY(run_gram(w.FA, SKLS_F64, d, nullptr, SKLS_F64, m, d, w.G, w.gram, w.gram_bytes, s));
    SKLS_TRY(run_cholesky(w.G, d, d, w.R, w.Rinv, w.RinvT, w.status, w.cholw, s));
    int32_t st_h = 0;
    SKLS_TRY(to_host(&st_h, w.status, sizeof st_h, s));
    if (st_h) {
      set_error("lp_regression: F A is numerically rank deficient");
      return SKLS_ERR_RANK;
    }
    SKLS_TRY(row_norm_estimates(A, w.Rinv, kg, P.seed, w.Pi2, w.T, w.Z, w.score, w.last, w.gs, s));
    hipLaunchKernelGGL(k_pow_rows, dim3(kRed), dim3(kT), 0, s, n, w.score, P.p / 2.0, w.lam, w.part);
    SKLS_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kT), 0, s, w.part, kRed, 1, w.sums);
    SKLS_CHECK_LAUNCH();
    double L = 0.0;
    SKLS_TRY(to_host(&L, w.sums, sizeof L, s));
    if (!(L > 0.0) || !std::isfinite(L)) {
      set_error("lp_regression: the row-norm estimates are not positive and finite");
      return SKLS_ERR_RANK;
    }
  }
  SKLS_TRY_HIP(hipEventRecord(ev[1], s));

  // ---- stage 1: constant-factor fit on rows drawn by the basis norms
  int64_t ns = 0;
  Fit f1;
  {
    PhaseTimer pt("lp_stage1", s);
    SKLS_TRY(draw_coreset(A, b, w, P, P.s1, false, &ns, s));
    inf.rows_stage1 = ns;
    if (rows1) SKLS_TRY_HIP(hipMemcpyAsync(rows1, w.list, sizeof(int32_t) * ns, hipMemcpyDeviceToDevice, s));
    if (w1) SKLS_TRY_HIP(hipMemcpyAsync(w1, w.wts, sizeof(double) * ns, hipMemcpyDeviceToDevice, s));
    SKLS_TRY(fit(w, ns, d, P.p, P.max_iter, P.tol, f1, s));
    if (x_c) SKLS_TRY_HIP(hipMemcpyAsync(x_c, w.x, sizeof(double) * d, hipMemcpyDeviceToDevice, s));
    SKLS_TRY(full_objective(A, b, w, w.x, P.p, w.rp, &inf.obj_stage1, s));
  }
  SKLS_TRY_HIP(hipEventRecord(ev[2], s));

  // ---- stage 2: rows drawn by max(basis share, residual share)
  Fit f2;
  {
    PhaseTimer pt("lp_stage2", s);
    SKLS_TRY(draw_coreset(A, b, w, P, P.s2, true, &ns, s));
    inf.rows_stage2 = ns;
    if (rows2) SKLS_TRY_HIP(hipMemcpyAsync(rows2, w.list, sizeof(int32_t) * ns, hipMemcpyDeviceToDevice, s));
    if (w2) SKLS_TRY_HIP(hipMemcpyAsync(w2, w.wts, sizeof(double) * ns, hipMemcpyDeviceToDevice, s));
    SKLS_TRY(fit(w, ns, d, P.p, P.max_iter, P.tol, f2, s));
    SKLS_TRY_HIP(hipMemcpyAsync(x, w.x, sizeof(double) * d, hipMemcpyDeviceToDevice, s));
    SKLS_TRY(full_objective(A, b, w, w.x, P.p, nullptr, &inf.obj, s));
  }
  SKLS_TRY_HIP(hipEventRecord(ev[3], s));
  SKLS_TRY_HIP(hipStreamSynchronize(s));
  inf.iters_stage1 = f1.iters;
  inf.iters_stage2 = f2.iters;
  inf.converged = (f1.converged && f2.converged) ? 1 : 0;
  inf.coreset_obj = f2.obj;
  float ms = 0.0f;
  SKLS_TRY_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
  inf.ms_condition = ms;
  SKLS_TRY_HIP(hipEventElapsedTime(&ms, ev[1], ev[2]));
  inf.ms_stage1 = ms;
  SKLS_TRY_HIP(hipEventElapsedTime(&ms, ev[2], ev[3]));
  inf.ms_stage2 = ms;
  if (info) *info = inf;
  return SKLS_OK;
}

}  // namespace skls
