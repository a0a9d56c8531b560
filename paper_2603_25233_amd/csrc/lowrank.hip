// Low-rank SI of the paper (Sec. 3.1-3.4, Alg. 1, Alg. 2) on gfx950.
//
// One outer iteration n (source s = Sigma_s phi^{n-1} + G fixed):
//   1. sweep the p sampled angles (eq. (sampled-sweep));
//   2. MGS2-A (Alg. 2): per snapshot two projections (dc = X^T psi, psi -= X dc),
//      normalisation, up to m_max clean-up projections while |X(:,1)^T psi^| > eps_mgs;
//   3. incremental projected operators (Sec. 3.4): X^T Sigma_t X, X^T D_x^- X and
//      X^T D_y^- X grow by border blocks; X^T D^+ X = -(X^T D^- X)^T because the
//      upwind operator satisfies D(Omega)^T = D(-Omega); projected right-hand sides
//      X^T s and X^T g_side grow likewise;
//   4. q random unsampled candidates, Galerkin solves (eq. (galerkin-projection)),
//      residual norms ||s + g_j - (D_j + Sigma_t) X c_j||_2, greedy top p;
//   5. inner stop (Sec. 3.3): if the largest candidate residual is < eps_res, the
//      Galerkin coefficients of every unsampled angle give phi = X (C w) and the
//      loop ends when ||phi - phi_old||_2 <= eps_diff (else phi_old = phi);
//   6. after the last outer iteration, the truncated SVD of C and X U (Sec. 3.3).
// Angles are the classes of ordinates with equal (Omega_x, Omega_y): in X-Y geometry
// the SI equation depends on Omega only through them, so one sweep serves a class.
//
// MI355X layout.  The Galerkin matrices of every unsampled class are kept as LU
// factors (no pivoting: the symmetric part of X^T (D_j + Sigma_t) X is positive
// definite, so every leading minor is positive) and bordered by the p new rows and
// columns in each inner iteration, one wavefront per class; a candidate or a full
// projection is then one back substitution.  This gives the same coefficients as
// factorising the q candidate matrices from scratch, with O(K r^2 p) parallel work
// per iteration instead of q serial O(r^3) factorisations.  X is column-major in HBM
// ([r][ndof]); projections are row-chunked with per-block partial sums reduced in a
// fixed order, so results are bitwise repeatable.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <type_traits>

#include "lowrank.h"

namespace rte {

namespace {

constexpr double kR3 = 1.7320508075688772935;
constexpr int kTB = 256;          // threads per block of the row-chunked kernels
constexpr int kMaxP = 8;          // largest batch of new columns handled per bordering

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum NV per-thread values over a 256-thread block; results in red[0..NV).
template <int NV>
__device__ __forceinline__ void block_sum_vec(const double* v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) red[wave * NV + k] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < NV) {
    double s = 0.0;
    for (int w = 0; w < (kTB >> 6); ++w) s += red[w * NV + threadIdx.x];
    red[(kTB >> 6) * NV + threadIdx.x] = s;
  }
  __syncthreads();
}

// ------------------------------------------------------------------ projections
// Batched projection of NV vectors W[l] (stride nd) against columns of the basis.  A
// wavefront covers PjCfg<NV>::rows consecutive rows, rpt rows per lane, lane-interleaved
// (every column read is one contiguous 512-byte run per wavefront); a block holds
// kPjWaves wavefronts.
//   If r_upd > 0: W[l] -= sum_{c < r_upd} Xu[c] C[c NV + l] (written back).
//   Then, per wavefront wf: part[wf][c NV + l] = Xd[c]^T W[l] over its rows (c < r_dot),
//   part[wf][r_dot NV + l] = W[l].W[l] after the update and part[wf][r_dot NV + NV + l]
//   before it.
// The lane sums are reduced over the wavefront 16 values at a time by a transpose
// through the wavefront's own LDS rows and a fixed-order sum, so nothing but the C
// staging waits on a block-wide barrier; the columns of the next round are fetched
// before the current round is reduced.
constexpr int kPjWaves = 4;
constexpr int kPjVals = 16;          // values reduced per round
constexpr int kPjLd = kPjVals + 1;   // LDS row stride (doubles) of the transpose
constexpr int kPjRed = 64 * kPjLd;   // LDS doubles per wavefront

template <int NV>
struct PjCfg {
  static constexpr int rpt = NV == 3 || NV == 4 ? 4 : 2;  // rows per lane (NV rpt <= 16)
  static constexpr int rows = 64 * rpt;                   // rows per wavefront
  static constexpr int g = kPjVals / NV < 8 ? kPjVals / NV : 8;  // dot columns per round
  static constexpr int u = 16 / rpt;                      // update columns per round
};

__device__ __forceinline__ void lds_fence_wave() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
}

// Sum of 16 values over the 64 lanes of a wavefront; lane j < 16 returns the sum of value
// j (fixed order: four 16-lane segments summed in lane order, then two xor shuffles).
// rw: 64 * kPjLd doubles of LDS owned by this wavefront.
__device__ __forceinline__ double wave_colsum16(const double (&p)[kPjVals], double* rw) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < kPjVals; ++j) rw[lane * kPjLd + j] = p[j];
  lds_fence_wave();
  const int col = lane & 15, seg = lane >> 4;
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) s += rw[(seg * 16 + u) * kPjLd + col];
  lds_fence_wave();
  s += __shfl_xor(s, 16, 64);
  s += __shfl_xor(s, 32, 64);
  return s;
}

// out[c] = sum_b part[b][c] for c < n (and acc_into[c] += out[c] for c < n_acc).  A block of
// 256 threads handles 8 columns (cblk selects them): 32 lanes per column take every 32nd
// partial (eight running sums, fixed assignment), then fixed pairwise trees combine the
// sums and the lanes, so the result is the same on every run.  red: 256 doubles of LDS.
__device__ void reduce_cols_block(const double* part, int nblk, int stride, int n,
                                  double* __restrict__ out, double* __restrict__ acc_into,
                                  int n_acc, int cblk, double* red) {
  constexpr int NS = 8;
  const int c = cblk * 8 + (threadIdx.x >> 5);
  const int l = threadIdx.x & 31;
  double sv[NS];
#pragma unroll
  for (int u = 0; u < NS; ++u) sv[u] = 0.0;
  if (c < n) {
    // Every load is issued from a row clamped into range and masked at the add, so that
    // none waits behind a branch.
    for (int b0 = l; b0 - l < nblk; b0 += 32 * NS) {
      double v[NS];
#pragma unroll
      for (int u = 0; u < NS; ++u) v[u] = part[(long)min(b0 + 32 * u, nblk - 1) * stride + c];
#pragma unroll
      for (int u = 0; u < NS; ++u) sv[u] += b0 + 32 * u < nblk ? v[u] : 0.0;
    }
  }
#pragma unroll
  for (int h = NS / 2; h > 0; h >>= 1)
#pragma unroll
    for (int u = 0; u < h; ++u) sv[u] += sv[u + h];
  red[threadIdx.x] = sv[0];
  __syncthreads();
  for (int h = 16; h > 0; h >>= 1) {
    if (l < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (l == 0 && c < n) {
    const double v = red[threadIdx.x];
    out[c] = v;
    if (acc_into && c < n_acc) acc_into[c] += v;
  }
}

__global__ __launch_bounds__(256) void reduce_cols_kernel(const double* __restrict__ part, int nblk,
                                                          int stride, int n, double* __restrict__ out,
                                                          double* __restrict__ acc_into, int n_acc) {
  __shared__ double red[256];
  reduce_cols_block(part, nblk, stride, n, out, acc_into, n_acc, blockIdx.x, red);
}

template <typename TX, typename TW, int NV>
__global__ __launch_bounds__(64 * kPjWaves, 2) void bproj_kernel(
    const TX* __restrict__ Xu, int r_upd, const double* __restrict__ C, const TX* __restrict__ Xd,
    int r_dot, TW* __restrict__ W, long nd, double* __restrict__ part) {
  using Cfg = PjCfg<NV>;
  constexpr int RPT = Cfg::rpt, G = Cfg::g, U = Cfg::u;
  extern __shared__ double sm[];
  double* sC = sm;  // [r_upd NV]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* rw = sm + r_upd * NV + wave * kPjRed;
  const long wf = (long)blockIdx.x * kPjWaves + wave;
  const long i0 = wf * Cfg::rows + lane;
  for (int c = threadIdx.x; c < r_upd * NV; c += 64 * kPjWaves) sC[c] = C[c];
  __syncthreads();
  // Rows past nd read row 0 of their column (every load is unconditional, so none of them
  // waits inside a branch) and are zeroed in w; the basis values of such rows then only
  // ever meet w = 0 or results that are discarded.
  bool ok[RPT];
  long ix[RPT];
  double w[NV][RPT], before[NV], after[NV];
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    ok[t] = i0 + 64 * t < nd;
    ix[t] = ok[t] ? i0 + 64 * t : 0;
  }
  {
    TW wr[NV][RPT];
#pragma unroll
    for (int l = 0; l < NV; ++l)
#pragma unroll
      for (int t = 0; t < RPT; ++t) wr[l][t] = W[(long)l * nd + ix[t]];
#pragma unroll
    for (int l = 0; l < NV; ++l) {
      before[l] = 0.0;
#pragma unroll
      for (int t = 0; t < RPT; ++t) {
        w[l][t] = ok[t] ? (double)wr[l][t] : 0.0;
        before[l] += w[l][t] * w[l][t];
      }
    }
  }
  if (r_upd > 0) {
    double s[NV][RPT];
#pragma unroll
    for (int l = 0; l < NV; ++l)
#pragma unroll
      for (int t = 0; t < RPT; ++t) s[l][t] = 0.0;
    // U columns per round: all loads of a round are issued before its products
    int c = 0;
    for (; c + U <= r_upd; c += U) {
      TX xv[U][RPT];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int t = 0; t < RPT; ++t) xv[u][t] = Xu[(long)(c + u) * nd + ix[t]];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int l = 0; l < NV; ++l) {
          const double d = sC[(c + u) * NV + l];
#pragma unroll
          for (int t = 0; t < RPT; ++t) s[l][t] += (double)xv[u][t] * d;
        }
    }
    for (; c < r_upd; ++c) {
      TX xv[RPT];
#pragma unroll
      for (int t = 0; t < RPT; ++t) xv[t] = Xu[(long)c * nd + ix[t]];
#pragma unroll
      for (int l = 0; l < NV; ++l) {
        const double d = sC[c * NV + l];
#pragma unroll
        for (int t = 0; t < RPT; ++t) s[l][t] += (double)xv[t] * d;
      }
    }
#pragma unroll
    for (int l = 0; l < NV; ++l)
#pragma unroll
      for (int t = 0; t < RPT; ++t) {
        const TW nv = (TW)(w[l][t] - s[l][t]);
        w[l][t] = ok[t] ? (double)nv : 0.0;  // the stored (possibly rounded) value
        if (ok[t]) W[(long)l * nd + i0 + 64 * t] = nv;
      }
  }
#pragma unroll
  for (int l = 0; l < NV; ++l) {
    after[l] = 0.0;
#pragma unroll
    for (int t = 0; t < RPT; ++t) after[l] += w[l][t] * w[l][t];
  }
  const int stride = r_dot * NV + 2 * NV;
  double* out = part + wf * stride;
  if (r_dot > 0) {
    // columns past r_dot read column r_dot - 1; their sums are not stored
    TX xc[G][RPT], xn[G][RPT];
    auto fetch = [&](TX (&x)[G][RPT], int c0) {
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const long col = c0 + g < r_dot ? c0 + g : r_dot - 1;
#pragma unroll
        for (int t = 0; t < RPT; ++t) x[g][t] = Xd[col * nd + ix[t]];
      }
    };
    fetch(xc, 0);
    for (int c0 = 0; c0 < r_dot; c0 += G) {
      if (c0 + G < r_dot) fetch(xn, c0 + G);
      double p[kPjVals];
#pragma unroll
      for (int j = 0; j < kPjVals; ++j) p[j] = 0.0;
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int l = 0; l < NV; ++l)
#pragma unroll
          for (int t = 0; t < RPT; ++t) p[g * NV + l] += (double)xc[g][t] * w[l][t];
      const double tot = wave_colsum16(p, rw);
      if (lane < G * NV && c0 + lane / NV < r_dot) out[c0 * NV + lane] = tot;
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int t = 0; t < RPT; ++t) xc[g][t] = xn[g][t];
    }
  }
  double p[kPjVals];
#pragma unroll
  for (int j = 0; j < kPjVals; ++j) p[j] = 0.0;
#pragma unroll
  for (int l = 0; l < NV; ++l) {
    p[l] = after[l];
    p[NV + l] = before[l];
  }
  const double tot = wave_colsum16(p, rw);
  if (lane < 2 * NV) out[r_dot * NV + lane] = tot;
}

// Per-snapshot statistics of a batch, mstat[l] = (|psi|^2 now, |psi|^2 at the start,
// X(:,1)^T psi): from the batch projections (d1: pass 1, d3: pass 3 or the norms-only
// pass when the basis is empty); snapshot_done_kernel updates them after the projections
// against the columns appended earlier in the batch.
__global__ void mstat_init_kernel(int pn, int r0, const double* __restrict__ d1,
                                  const double* __restrict__ d3, double* __restrict__ mstat) {
  const int l = threadIdx.x;
  if (l >= pn) return;
  double* m = mstat + 4 * l;
  if (r0 > 0) {
    m[0] = d3[pn + l];
    m[1] = d1[(long)r0 * pn + pn + l];
    m[2] = d3[l];
  } else {
    m[0] = d3[l];
    m[1] = d3[pn + l];
    m[2] = 0.0;
  }
}

// The end of one snapshot of the device-side MGS2-A, in one launch: with |v|^2 = d3[1]
// (after projections against columns appended earlier in the batch; then also
// m[0] = d3[1], m[2] = d3[0]) or m[0] (the first snapshot), col = v (1 / |v|) (rounded as
// append_kernel with the host's 1 / |v|; a vanishing v gives a zero column, discarded by
// the host), and block 0 stores dst = (cvec[0 .. r), |v|, 0 ...).
template <typename TV, typename TC>
__global__ void snapshot_done_kernel(const TV* __restrict__ v, long nd, TC* __restrict__ col,
                                     const double* __restrict__ d3, double* __restrict__ m,
                                     const double* __restrict__ cvec, int r,
                                     double* __restrict__ dst, int rcap) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const double a = sqrt(d3 ? d3[1] : m[0]);
  const double ia = a > 0.0 ? 1.0 / a : 0.0;
  if (i < nd) col[i] = (TC)((double)v[i] * ia);
  if (blockIdx.x == 0) {
    if (d3 && threadIdx.x == 0) {
      m[0] = d3[1];
      m[2] = d3[0];
    }
    for (int k = threadIdx.x; k < rcap; k += blockDim.x) dst[k] = k < r ? cvec[k] : (k == r ? a : 0.0);
  }
}

// cvecs[l][i] = cb[i pn + l] for i < r0, 0 for r0 <= i < n (every snapshot l < pn of a batch)
__global__ void coef_cols_kernel(const double* __restrict__ cb, int pn, int r0,
                                 double* __restrict__ cvecs, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int l = blockIdx.y;
  if (i < n) cvecs[(long)l * n + i] = i < r0 ? cb[(long)i * pn + l] : 0.0;
}

// cvec[i] = cb[i pn + l] for i < r0, 0 for r0 <= i < n
__global__ void coef_col_kernel(const double* __restrict__ cb, int pn, int l, int r0,
                                double* __restrict__ cvec, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cvec[i] = i < r0 ? cb[(long)i * pn + l] : 0.0;
}
static void reduce_cols(const double* part, int nblk, int stride, int n, double* out,
                        double* acc_into, hipStream_t st, int n_acc = 0) {
  hipLaunchKernelGGL(reduce_cols_kernel, dim3((n + 7) / 8), dim3(256), 0, st, part, nblk, stride, n,
                     out, acc_into, n_acc);
}

template <typename TV, typename TC>
__global__ void append_kernel(const TV* __restrict__ v, double inv_alpha, TC* __restrict__ col,
                              long nd) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nd) col[i] = (TC)((double)v[i] * inv_alpha);
}

__global__ void store_coef_kernel(const double* __restrict__ cvec, int r, double alpha,
                                  int with_alpha, double* __restrict__ dst, int rcap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rcap) return;
  double x = 0.0;
  if (i < r) x = cvec[i];
  else if (i == r && with_alpha) x = alpha;
  dst[i] = x;
}

// ------------------------------------------------------------------ stencils
// Per cell u (4 values, k = 2q + p):  (I (x) L) u, (I (x) C) u etc. with
// L = [[1, s3], [-s3, 3]], C = (1, -s3)^T (1, s3); transposes likewise.
struct Q4 {
  double v[4];
};
__device__ __forceinline__ Q4 ld4(const double* p) { return Q4{{p[0], p[1], p[2], p[3]}}; }
__device__ __forceinline__ Q4 ld4(const float* p) { return Q4{{p[0], p[1], p[2], p[3]}}; }

// x-part of D_x^- at cell (a, b): (1/hx) [(I(x)L) u_c - (I(x)C) u_{c-1}]
template <typename T>
__device__ __forceinline__ Q4 dxm(const T* u, long c, int a, double ihx) {
  Q4 x = ld4(u + 4 * c), r;
  for (int q = 0; q < 2; ++q) {
    const double u0 = x.v[2 * q], u1 = x.v[2 * q + 1];
    r.v[2 * q] = u0 + kR3 * u1;
    r.v[2 * q + 1] = -kR3 * u0 + 3.0 * u1;
  }
  if (a > 0) {
    Q4 w = ld4(u + 4 * (c - 1));
    for (int q = 0; q < 2; ++q) {
      const double t = w.v[2 * q] + kR3 * w.v[2 * q + 1];
      r.v[2 * q] -= t;
      r.v[2 * q + 1] += kR3 * t;
    }
  }
  for (int k = 0; k < 4; ++k) r.v[k] *= ihx;
  return r;
}
// (D_x^-)^T: (1/hx) [(I(x)L^T) u_c - (I(x)C^T) u_{c+1}],  C^T = (1, s3)^T (1, -s3)
template <typename T>
__device__ __forceinline__ Q4 dxmT(const T* u, long c, int a, int nx, double ihx) {
  Q4 x = ld4(u + 4 * c), r;
  for (int q = 0; q < 2; ++q) {
    const double u0 = x.v[2 * q], u1 = x.v[2 * q + 1];
    r.v[2 * q] = u0 - kR3 * u1;
    r.v[2 * q + 1] = kR3 * u0 + 3.0 * u1;
  }
  if (a + 1 < nx) {
    Q4 w = ld4(u + 4 * (c + 1));
    for (int q = 0; q < 2; ++q) {
      const double t = w.v[2 * q] - kR3 * w.v[2 * q + 1];
      r.v[2 * q] -= t;
      r.v[2 * q + 1] -= kR3 * t;
    }
  }
  for (int k = 0; k < 4; ++k) r.v[k] *= ihx;
  return r;
}
// y versions act on q with p fixed
template <typename T>
__device__ __forceinline__ Q4 dym(const T* u, long c, int b, int nx, double ihy) {
  Q4 x = ld4(u + 4 * c), r;
  for (int p = 0; p < 2; ++p) {
    const double u0 = x.v[p], u1 = x.v[2 + p];
    r.v[p] = u0 + kR3 * u1;
    r.v[2 + p] = -kR3 * u0 + 3.0 * u1;
  }
  if (b > 0) {
    Q4 w = ld4(u + 4 * (c - nx));
    for (int p = 0; p < 2; ++p) {
      const double t = w.v[p] + kR3 * w.v[2 + p];
      r.v[p] -= t;
      r.v[2 + p] += kR3 * t;
    }
  }
  for (int k = 0; k < 4; ++k) r.v[k] *= ihy;
  return r;
}
template <typename T>
__device__ __forceinline__ Q4 dymT(const T* u, long c, int b, int nx, int ny, double ihy) {
  Q4 x = ld4(u + 4 * c), r;
  for (int p = 0; p < 2; ++p) {
    const double u0 = x.v[p], u1 = x.v[2 + p];
    r.v[p] = u0 - kR3 * u1;
    r.v[2 + p] = kR3 * u0 + 3.0 * u1;
  }
  if (b + 1 < ny) {
    Q4 w = ld4(u + 4 * (c + nx));
    for (int p = 0; p < 2; ++p) {
      const double t = w.v[p] - kR3 * w.v[2 + p];
      r.v[p] -= t;
      r.v[2 + p] -= kR3 * t;
    }
  }
  for (int k = 0; k < 4; ++k) r.v[k] *= ihy;
  return r;
}

// Y[(op * pn + m)][.] = op(P_m), op in {Sigma_t, D_x^-, D_y^-, (D_x^-)^T, (D_y^-)^T}
template <typename T>
__global__ void border_stencil_kernel(int nx, int ny, double ihx, double ihy,
                                      const double* __restrict__ sig, const T* __restrict__ P,
                                      int pn, long nd, T* __restrict__ Y) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long ncell = (long)nx * ny;
  if (c >= ncell) return;
  const int a = (int)(c % nx), b = (int)(c / nx);
  for (int m = 0; m < pn; ++m) {
    const T* u = P + (long)m * nd;
    Q4 r[5];
    Q4 x = ld4(u + 4 * c);
    for (int k = 0; k < 4; ++k) r[0].v[k] = sig[c] * x.v[k];
    r[1] = dxm(u, c, a, ihx);
    r[2] = dym(u, c, b, nx, ihy);
    r[3] = dxmT(u, c, a, nx, ihx);
    r[4] = dymT(u, c, b, nx, ny, ihy);
    for (int op = 0; op < 5; ++op)
      for (int k = 0; k < 4; ++k) Y[(long)(op * pn + m) * nd + 4 * c + k] = (T)r[op].v[k];
  }
}

// unit-flux boundary vectors: E[1 + s][.] = int_face g eta_k on side s (0 elsewhere)
__global__ void gunit_kernel(int nx, int ny, int mb, double hx, double hy,
                             const double* __restrict__ bc, double* __restrict__ E, long nd) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (long)nx * ny) return;
  const int a = (int)(c % nx), b = (int)(c / nx);
  const double sx = 1.0 / std::sqrt(hx), sy = 1.0 / std::sqrt(hy);
  for (int s = 0; s < 4; ++s) {
    double* o = E + (long)(1 + s) * nd + 4 * c;
    double v[4] = {0, 0, 0, 0};
    if (bc) {
      if (s == 0 && a == 0) {            // left face: l_p(-1) g_q
        for (int q = 0; q < 2; ++q) {
          const double gq = bc[((long)0 * mb + b) * 2 + q];
          v[2 * q] = sx * gq;
          v[2 * q + 1] = -kR3 * sx * gq;
        }
      } else if (s == 1 && a == nx - 1) { // right face: l_p(+1) g_q
        for (int q = 0; q < 2; ++q) {
          const double gq = bc[((long)1 * mb + b) * 2 + q];
          v[2 * q] = sx * gq;
          v[2 * q + 1] = kR3 * sx * gq;
        }
      } else if (s == 2 && b == 0) {      // bottom face: l_q(-1) g_p
        for (int p = 0; p < 2; ++p) {
          const double gp = bc[((long)2 * mb + a) * 2 + p];
          v[p] = sy * gp;
          v[2 + p] = -kR3 * sy * gp;
        }
      } else if (s == 3 && b == ny - 1) { // top face: l_q(+1) g_p
        for (int p = 0; p < 2; ++p) {
          const double gp = bc[((long)3 * mb + a) * 2 + p];
          v[p] = sy * gp;
          v[2 + p] = kR3 * sy * gp;
        }
      }
    }
    for (int k = 0; k < 4; ++k) o[k] = v[k];
  }
}

template <typename T>
__global__ void to_double_kernel(const T* __restrict__ a, double* __restrict__ b, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

// ------------------------------------------------------------------ E^T P
// part[blk][e PN + m] = sum over the block's rows of E[e][k] P[m][k]  (e < 5, m < PN): the
// projections of the source and boundary vectors on the new columns.  Threads stride
// over the rows; one block reduction at the end.
template <typename T, int PN>
__global__ __launch_bounds__(256) void edot_kernel(const double* __restrict__ E,
                                                  const T* __restrict__ P, long nd,
                                                  double* __restrict__ part) {
  constexpr int NV = 5 * PN;
  __shared__ double red[(kTB / 64 + 1) * NV];
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < nd; k += (long)gridDim.x * blockDim.x) {
    double pm[PN];
#pragma unroll
    for (int m = 0; m < PN; ++m) pm[m] = (double)P[(long)m * nd + k];
#pragma unroll
    for (int e = 0; e < 5; ++e) {
      const double ev = E[(long)e * nd + k];
#pragma unroll
      for (int m = 0; m < PN; ++m) acc[e * PN + m] += ev * pm[m];
    }
  }
  block_sum_vec<NV>(acc, red);
  if ((int)threadIdx.x < NV) part[(long)blockIdx.x * NV + threadIdx.x] = red[(kTB / 64) * NV + threadIdx.x];
}

// ------------------------------------------------------------------ X^T W, lanes over columns
// part[blk][c NV + l] = sum over the block's rows k of X[c][k] W[l][k]  (c < r, l < NV).
// Each lane owns one column of X, so the sums need no cross-lane reduction.  A wavefront
// covers 64 columns and reads them in sub-tiles of 128 bytes per column (8 columns per
// load instruction, whole cache lines), transposes each sub-tile through its own LDS
// rows, and then every lane walks down its column.  The NV vectors of W are staged per
// kXwRows-row chunk in LDS as [row][vector] (double-buffered: the next chunk is fetched
// into registers while the current one is used) and read as broadcasts.  A block of 256
// threads covers 256 columns (blockIdx.y selects the tile) and `nch` consecutive chunks;
// with fewer columns than 256, the wavefronts of a block split the sub-tiles of each chunk
// between them (row groups) and add their sums in a fixed order at the end.
constexpr int kXwRows = 128;

template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int n = 2;
  __device__ static double at(const double2& v, int i) { return i == 0 ? v.x : v.y; }
};
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int n = 4;
  __device__ static double at(const float4& v, int i) {
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
  }
};

template <typename T, int NV>
__global__ __launch_bounds__(256) void xtw_kernel(const T* __restrict__ X, int r,
                                                 const T* __restrict__ W, long nd, int nch,
                                                 double* __restrict__ part) {
  constexpr int NVP = (NV + 1) & ~1;                // even row stride: 16-byte pairs
  constexpr int PT = (NV * kXwRows + 255) / 256;     // staged values per thread
  constexpr int E = Vec16<T>::n;                     // elements per 16-byte load
  constexpr int SUB = 128 / (int)sizeof(T);          // rows of a sub-tile (128 B per column)
  constexpr int NSUB = kXwRows / SUB;                // sub-tiles per chunk
  constexpr int LDX = SUB + 1;                       // LDS row stride of the transpose
  using V = typename Vec16<T>::type;
  __shared__ __align__(16) double Ws[2][kXwRows * NVP];
  __shared__ T Xs[4][64 * LDX];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // column tiles of 64 in this block (1, 2 or 4) and row groups (4, 2 or 1)
  const int ncol = min(256, r - (int)blockIdx.y * 256);
  const int ntile = ncol <= 64 ? 1 : (ncol <= 128 ? 2 : 4);
  const int ngrp = 4 / ntile, tile = wave % ntile, grp = wave / ntile;
  const int c = blockIdx.y * 256 + tile * 64 + lane;
  const bool on = c < r;
  // load lane roles: column cw + 8 i + (lane >> 3), elements (lane & 7) E .. of the sub-tile
  const int cw = blockIdx.y * 256 + tile * 64;
  const bool won = cw < r;  // wavefronts past the last column only help with the staging
  const V* xcol[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int col = min(cw + 8 * i + (lane >> 3), r - 1);  // columns past r: any valid one
    xcol[i] = reinterpret_cast<const V*>(X + (long)col * nd);
  }
  const int eoff = (lane & 7) * E;
  T* xs = Xs[wave];
  const long kb = (long)blockIdx.x * nch * kXwRows;
  const int nq = (int)std::min<long>(nch, (nd - kb + kXwRows - 1) / kXwRows);
  // W staging: raw values are fetched a chunk ahead (unconditional loads from a clamped
  // address) and converted, with rows past nd zeroed, when they are stashed in LDS
  T wpf[PT];
  auto wfetch = [&](long k0) {
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int e = threadIdx.x + 256 * i, l = e / kXwRows, k = e % kXwRows;
      const bool in = e < NV * kXwRows && k0 + k < nd;
      wpf[i] = W[in ? (long)l * nd + k0 + k : 0];
    }
  };
  auto wstash = [&](double* ws, long k0) {
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int e = threadIdx.x + 256 * i, l = e / kXwRows, k = e % kXwRows;
      if (e < NV * kXwRows) ws[k * NVP + l] = k0 + k < nd ? (double)wpf[i] : 0.0;
    }
  };
  // rows past nd (last chunk only) read a clamped in-range address; their staged W is 0
  auto xload = [&](V (&xv)[8], long k0) {
    const long k = std::min<long>(k0 + eoff, nd - E) / E;
#pragma unroll
    for (int i = 0; i < 8; ++i) xv[i] = xcol[i][k];
  };
  double acc[NV];
#pragma unroll
  for (int l = 0; l < NV; ++l) acc[l] = 0.0;
  wfetch(kb);
  wstash(Ws[0], kb);
  V xv[8];
  if (won) xload(xv, kb + grp * SUB);
  __syncthreads();
  for (int q = 0; q < nq; ++q) {
    const long k0 = kb + (long)q * kXwRows;
    if (q + 1 < nq) wfetch(k0 + kXwRows);
    const double* ws = Ws[q & 1];
#pragma unroll 1
    for (int sb = grp; won && sb < NSUB; sb += ngrp) {
      // transpose the sub-tile: column 8 i + (lane >> 3), rows eoff .. eoff + E - 1
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int e = 0; e < E; ++e)
          xs[(8 * i + (lane >> 3)) * LDX + eoff + e] = (T)Vec16<T>::at(xv[i], e);
      lds_fence_wave();
      // next sub-tile (or the first of the next chunk) in flight during the products
      if (sb + ngrp < NSUB) xload(xv, k0 + (sb + ngrp) * SUB);
      else if (q + 1 < nq) xload(xv, k0 + kXwRows + grp * SUB);
      const T* xr = xs + lane * LDX;
      const double* wr = ws + sb * SUB * NVP;
#pragma unroll 4
      for (int kk = 0; kk < SUB; ++kk) {
        const double x = (double)xr[kk];
#pragma unroll
        for (int l = 0; l < NV; ++l) acc[l] += x * wr[kk * NVP + l];
      }
      lds_fence_wave();
    }
    if (q + 1 < nq) wstash(Ws[(q + 1) & 1], k0 + kXwRows);
    __syncthreads();
  }
  // row groups 1 .. ngrp-1 hand their sums to group 0 through LDS (reusing Ws)
  if (ngrp > 1) {
    double* red = &Ws[0][0];  // [ngrp - 1][64 ntile][NV] <= 3 * 64 * NV doubles
    if (grp > 0)
#pragma unroll
      for (int l = 0; l < NV; ++l) red[(((grp - 1) * ntile + tile) * 64 + lane) * NV + l] = acc[l];
    __syncthreads();
    if (grp == 0)
      for (int g = 1; g < ngrp; ++g)
#pragma unroll
        for (int l = 0; l < NV; ++l) acc[l] += red[(((g - 1) * ntile + tile) * 64 + lane) * NV + l];
  }
  if (on && grp == 0)
#pragma unroll
    for (int l = 0; l < NV; ++l) part[((long)blockIdx.x * r + c) * NV + l] = acc[l];
}

// ------------------------------------------------------------------ X C products
// out[m][i] = sum_c X[c][i] C[c*ldc + m] for m < nm (<= NM), rows i; C staged in LDS.
// Four columns of X are loaded per round before their products are summed.
template <typename T, typename TO, int NM>
__global__ __launch_bounds__(256) void xc_kernel(const T* __restrict__ X, int r, long nd,
                                                 const double* __restrict__ C, int ldc, int nm,
                                                 TO* __restrict__ out) {
  __shared__ double Cs[64][NM];
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = i < nd;
  const long il = ok ? i : 0;  // rows past nd read row 0 (unconditional loads); not stored
  double acc[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) acc[m] = 0.0;
  for (int c0 = 0; c0 < r; c0 += 64) {
    const int cn = min(64, r - c0);
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * NM; e += 256) {
      const int c = e / NM, m = e % NM;
      Cs[c][m] = (c < cn && m < nm) ? C[(long)(c0 + c) * ldc + m] : 0.0;
    }
    __syncthreads();
    int c = 0;
    for (; c + 4 <= cn; c += 4) {
      T x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = X[(long)(c0 + c + u) * nd + il];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int m = 0; m < NM; ++m) acc[m] += (double)x[u] * Cs[c + u][m];
    }
    for (; c < cn; ++c) {
      const double x = (double)X[(long)(c0 + c) * nd + il];
#pragma unroll
      for (int m = 0; m < NM; ++m) acc[m] += x * Cs[c][m];
    }
  }
  if (ok)
#pragma unroll
    for (int m = 0; m < NM; ++m)
      if (m < nm) out[(long)m * nd + i] = (TO)acc[m];
}

// Cm[i][m] = Cg[list[m]][i] for i < r, m < nm
__global__ void gather_cg_kernel(const double* __restrict__ Cg, int rcap, const int* __restrict__ list,
                                 int nm, int r, double* __restrict__ Cm) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= r * nm) return;
  const int i = t / nm, m = t % nm;
  Cm[t] = Cg[(size_t)rcap * list[m] + i];
}

// ------------------------------------------------------------------ residual norms
struct ClassDev {
  double ax, ay;  // |Omega_x|, |Omega_y|
  int sx, sy;
};

// part[blk][m] = ||s + g_j - (D_j + Sigma_t) V_m||^2 over the block's cells
template <typename T>
__global__ __launch_bounds__(256) void residual_kernel(
    int nx, int ny, double ihx, double ihy, const double* __restrict__ sig,
    const double* __restrict__ src, const double* __restrict__ E, long nd,
    const T* __restrict__ V, int nm, const int* __restrict__ cls,
    const ClassDev* __restrict__ cd, const double* __restrict__ ex, double* __restrict__ part) {
  __shared__ double red[8];
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  const ClassDev k = cd[cls[m]];
  const T* u = V + (long)m * nd;
  const double* exm = ex ? ex + (long)m * nd : nullptr;  // angular source of the candidate
  double s2 = 0.0;
  if (c < (long)nx * ny) {
    const int a = (int)(c % nx), b = (int)(c / nx);
    Q4 dx = k.sx > 0 ? dxm(u, c, a, ihx) : dxmT(u, c, a, nx, ihx);
    Q4 dy = k.sy > 0 ? dym(u, c, b, nx, ihy) : dymT(u, c, b, nx, ny, ihy);
    Q4 x = ld4(u + 4 * c);
    const double* gx = E + (long)(1 + (k.sx > 0 ? 0 : 1)) * nd + 4 * c;
    const double* gy = E + (long)(1 + (k.sy > 0 ? 2 : 3)) * nd + 4 * c;
    for (int q = 0; q < 4; ++q) {
      double rr = src[4 * c + q] + k.ax * gx[q] + k.ay * gy[q] - k.ax * dx.v[q] -
                  k.ay * dy.v[q] - sig[c] * x.v[q];
      if (exm) rr += exm[4 * c + q];
      s2 += rr * rr;
    }
  }
  const double w = wave_sum(s2);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
    part[(long)blockIdx.x * nm + m] = t;
  }
}

// ------------------------------------------------------------------ projected operators
// Scatter the border blocks into the projected matrices.
//   colY [r1][3 pn]: X^T [Sigma_t P, D_x^- P, D_y^- P]
//   rowY [r0][2 pn]: X_old^T [(D_x^-)^T P, (D_y^-)^T P]
//   ext  [5][pn]   : [s, g_L, g_R, g_B, g_T]^T P
__global__ void scatter_border_kernel(int r0, int pn, int rcap, const double* __restrict__ colY,
                                      const double* __restrict__ ext, double* __restrict__ Tm,
                                      double* __restrict__ Dx, double* __restrict__ Dy,
                                      double* __restrict__ bsrc, double* __restrict__ bside) {
  const int r1 = r0 + pn;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < r1 * pn) {
    const int i = t / pn, m = t % pn, j = r0 + m;
    const double* row = colY + (long)i * 5 * pn;
    Tm[(long)i * rcap + j] = row[m];
    Dx[(long)i * rcap + j] = row[pn + m];
    Dy[(long)i * rcap + j] = row[2 * pn + m];
    if (i < r0) {  // Sigma_t symmetric; D rows from the transposed products
      Tm[(long)j * rcap + i] = row[m];
      const double* rw = row + 3 * pn;
      Dx[(long)j * rcap + i] = rw[m];
      Dy[(long)j * rcap + i] = rw[pn + m];
    }
  }
  if (t < pn) {
    bsrc[r0 + t] = ext[0 * pn + t];
    for (int s = 0; s < 4; ++s) bside[(long)s * rcap + r0 + t] = ext[(1 + s) * pn + t];
  }
}

__device__ __forceinline__ double amat(const double* Tm, const double* Dx, const double* Dy,
                                       int rcap, const ClassDev& k, int i, int j) {
  const double dx = k.sx > 0 ? Dx[(long)i * rcap + j] : Dx[(long)j * rcap + i];
  const double dy = k.sy > 0 ? Dy[(long)i * rcap + j] : Dy[(long)j * rcap + i];
  return Tm[(long)i * rcap + j] + k.ax * dx + k.ay * dy;
}

__device__ __forceinline__ double bvec(const double* bsrc, const double* bside, int rcap,
                                       const ClassDev& k, int i) {
  return bsrc[i] + k.ax * bside[(long)(k.sx > 0 ? 0 : 1) * rcap + i] +
         k.ay * bside[(long)(k.sy > 0 ? 2 : 3) * rcap + i];
}

// ------------------------------------------------------------------ bordered LU
// One 256-thread workgroup per class in cls[].  Factor storage per class:
//   Lt[rcap][rcap]: Lt[i][j] = L(j, i) (column i of the unit lower factor, j > i)
//   U [rcap][rcap]: row-major upper factor;  y[rcap]: L^{-1} b.
// Extends the factorisation of the leading r0 x r0 block by pn rows/columns.
// The triangular solves are blocked by 64 rows: the 64 x 64 diagonal block is staged
// in LDS and solved by one wavefront with the unknowns in registers (one row per
// lane, values broadcast with readlane); the rows below are then updated by the whole
// workgroup, reading the factor columns with coalesced loads.
constexpr int kLuThreads = 256;
constexpr int kLuB = 64;           // block of the triangular solves
constexpr int kLuLd = kLuB + 1;    // LDS row stride of a staged diagonal block

__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// X[m][0..n) <- T^{-1} X[m][0..n) for m < pn (X in LDS, row stride n), T lower
// triangular with column i stored contiguously: T(j, i) = M[i rcap + j] for j >= i;
// unit diagonal if `unit`, else T(i, i) = M[i rcap + i].  Dg: kLuB * kLuLd doubles of LDS.
__device__ void lu_lower_solve(const double* __restrict__ M, int rcap, bool unit, int n, double* X,
                               int pn, double* Dg) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int b0 = 0; b0 < n; b0 += kLuB) {
    const int nb = min(kLuB, n - b0);
    // Dg[i][j] = T(b0 + j, b0 + i)  (column i of the block); all loads issued first
    {
      constexpr int NE = kLuB * kLuB / kLuThreads;
      double t[NE];
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        const int e = tid + kLuThreads * u, i = e / kLuB, j = e % kLuB;
        t[u] = (i < nb && j < nb) ? M[(long)(b0 + i) * rcap + b0 + j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        const int e = tid + kLuThreads * u;
        Dg[(e / kLuB) * kLuLd + e % kLuB] = t[u];
      }
    }
    __syncthreads();
    if (wave == 0) {
      double v[kMaxP];
#pragma unroll
      for (int m = 0; m < kMaxP; ++m) v[m] = (m < pn && lane < nb) ? X[m * n + b0 + lane] : 0.0;
      const double rd = (!unit && lane < nb) ? 1.0 / Dg[lane * kLuLd + lane] : 1.0;
      for (int i = 0; i < nb; ++i) {
        const double t = lane > i ? Dg[i * kLuLd + lane] : 0.0;
        const double ri = unit ? 1.0 : readlane_d(rd, i);
#pragma unroll
        for (int m = 0; m < kMaxP; ++m) {
          if (m >= pn) break;
          const double zi = readlane_d(v[m], i) * ri;
          v[m] = lane == i ? zi : v[m] - t * zi;
        }
      }
#pragma unroll
      for (int m = 0; m < kMaxP; ++m)
        if (m < pn && lane < nb) X[m * n + b0 + lane] = v[m];
    }
    __syncthreads();
    // rows below the block (16 factor entries in flight per thread)
    for (int j = b0 + nb + tid; j < n; j += kLuThreads) {
      double acc[kMaxP];
#pragma unroll
      for (int m = 0; m < kMaxP; ++m) acc[m] = 0.0;
      for (int i0 = 0; i0 < nb; i0 += 16) {
        double t[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          t[u] = i0 + u < nb ? M[(long)(b0 + i0 + u) * rcap + j] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u)
#pragma unroll
          for (int m = 0; m < kMaxP; ++m)
            if (m < pn && i0 + u < nb) acc[m] += t[u] * X[m * n + b0 + i0 + u];
      }
#pragma unroll
      for (int m = 0; m < kMaxP; ++m)
        if (m < pn) X[m * n + j] -= acc[m];
    }
    __syncthreads();
  }
}

// Two workgroups per class (blockIdx.y): 0 solves U_12 = L_11^{-1} A_12 into the new
// columns of U, 1 solves L_21 = A_21 U_11^{-1} (U_11^T L_21^T = A_21^T) into the new
// columns of L^T.  The two touch disjoint parts of the factors.
__global__ __launch_bounds__(kLuThreads, 2) void lu_border_kernel(
    int r0, int pn, int rcap, const int* __restrict__ cls, const ClassDev* __restrict__ cd,
    const double* __restrict__ Tm, const double* __restrict__ Dx, const double* __restrict__ Dy,
    double* __restrict__ Lt_all, double* __restrict__ U_all) {
  extern __shared__ double sm[];
  double* vec = sm;                       // [pn][r0]
  double* Dg = sm + (long)pn * r0;        // [kLuB][kLuLd]
  const int cl = cls[blockIdx.x];
  const bool lower = blockIdx.y == 1;
  const ClassDev k = cd[cl];
  const size_t fsz = (size_t)rcap * rcap;
  double* Lt = Lt_all + fsz * cl;
  double* U = U_all + fsz * cl;
  const int tid = threadIdx.x;
  for (int e = tid; e < pn * r0; e += kLuThreads) {
    const int m = e / r0, i = e % r0;
    vec[e] = lower ? amat(Tm, Dx, Dy, rcap, k, r0 + m, i) : amat(Tm, Dx, Dy, rcap, k, i, r0 + m);
  }
  __syncthreads();
  if (lower) lu_lower_solve(U, rcap, false, r0, vec, pn, Dg);
  else lu_lower_solve(Lt, rcap, true, r0, vec, pn, Dg);
  double* dst = lower ? Lt : U;
  for (int e = tid; e < pn * r0; e += kLuThreads) {
    const int m = e / r0, i = e % r0;
    dst[(size_t)i * rcap + r0 + m] = vec[e];
  }
}

// The corner of the bordered factorisation, one workgroup per class:
// S = A_22 - L_21 U_12 (no pivoting, as for the leading block), its LU, and the new
// entries of y = L^{-1} b.
__global__ __launch_bounds__(kLuThreads) void lu_corner_kernel(
    int r0, int pn, int rcap, const int* __restrict__ cls, const ClassDev* __restrict__ cd,
    const double* __restrict__ Tm, const double* __restrict__ Dx, const double* __restrict__ Dy,
    const double* __restrict__ bsrc, const double* __restrict__ bside,
    const double* __restrict__ btime, double* __restrict__ Lt_all, double* __restrict__ U_all,
    double* __restrict__ y_all) {
  __shared__ double S[kMaxP][kMaxP], yn[kMaxP];
  const int cl = cls[blockIdx.x];
  const ClassDev k = cd[cl];
  const size_t fsz = (size_t)rcap * rcap;
  double* Lt = Lt_all + fsz * cl;
  double* U = U_all + fsz * cl;
  double* y = y_all + (size_t)rcap * cl;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // one wavefront per dot product
  for (int d = wave; d < pn * pn + pn; d += kLuThreads / 64) {
    const bool isy = d >= pn * pn;
    const int m = isy ? d - pn * pn : d / pn, mm = d % pn;
    double s = 0.0;
    for (int i = lane; i < r0; i += 64)
      s += Lt[(size_t)i * rcap + r0 + m] * (isy ? y[i] : U[(size_t)i * rcap + r0 + mm]);
    s = wave_sum(s);
    if (lane == 0) {
      if (isy) {
        double b = bvec(bsrc, bside, rcap, k, r0 + m);
        if (btime) b += btime[(size_t)rcap * cl + r0 + m];
        yn[m] = b - s;
      }
      else S[m][mm] = amat(Tm, Dx, Dy, rcap, k, r0 + m, r0 + mm) - s;
    }
  }
  __syncthreads();
  if (tid == 0) {
    // LU of S without pivoting (in place), then finish y
    for (int c = 0; c < pn; ++c)
      for (int i = c + 1; i < pn; ++i) {
        const double f = S[i][c] / S[c][c];
        S[i][c] = f;
        for (int j = c + 1; j < pn; ++j) S[i][j] -= f * S[c][j];
      }
    for (int m = 0; m < pn; ++m) {
      double v = yn[m];
      for (int mm = 0; mm < m; ++mm) v -= S[m][mm] * yn[mm];
      yn[m] = v;
      y[r0 + m] = v;
    }
    for (int m = 0; m < pn; ++m)
      for (int mm = 0; mm < pn; ++mm) {
        if (mm >= m) U[(size_t)(r0 + m) * rcap + r0 + mm] = S[m][mm];
        else Lt[(size_t)(r0 + mm) * rcap + r0 + m] = S[m][mm];
      }
  }
}

// c = U^{-1} y for each class in cls[] -> Cg[cl][.], blocked by 64 rows from the bottom:
// the contributions of the solved rows (one wavefront per row dot product), then the
// diagonal block by one wavefront with the unknowns in registers.
__global__ __launch_bounds__(kLuThreads) void backsub_kernel(int r, int rcap,
                                                             const int* __restrict__ cls,
                                                             const double* __restrict__ U_all,
                                                             const double* __restrict__ y_all,
                                                             double* __restrict__ Cg) {
  extern __shared__ double sm[];
  double* x = sm;            // [r]
  double* Dg = sm + r;       // [kLuB][kLuLd]: Dg[k][i] = U(b0 + k, b0 + i)
  const int cl = cls[blockIdx.x];
  const double* U = U_all + (size_t)rcap * rcap * cl;
  const double* y = y_all + (size_t)rcap * cl;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < r; i += kLuThreads) x[i] = y[i];
  const int nblk = (r + kLuB - 1) / kLuB;
  for (int bb = nblk - 1; bb >= 0; --bb) {
    const int b0 = bb * kLuB, nb = min(kLuB, r - b0), e0 = b0 + nb;
    {
      constexpr int NE = kLuB * kLuB / kLuThreads;
      double t[NE];
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        const int e = tid + kLuThreads * u, kk = e / kLuB, i = e % kLuB;
        t[u] = (kk < nb && i < nb) ? U[(long)(b0 + kk) * rcap + b0 + i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        const int e = tid + kLuThreads * u;
        Dg[(e / kLuB) * kLuLd + e % kLuB] = t[u];
      }
    }
    // x[b0 + kk] -= U(b0 + kk, e0 ..) x[e0 ..]: each wavefront takes 4 rows at a time
    for (int k0 = 4 * wave; k0 < nb; k0 += 4 * (kLuThreads / 64)) {
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
      for (int j = e0 + lane; j < r; j += 64) {
        const double xj = x[j];
        double u4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) u4[q] = k0 + q < nb ? U[(long)(b0 + k0 + q) * rcap + j] : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) s4[q] += u4[q] * xj;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double sq = wave_sum(s4[q]);
        if (lane == 0 && k0 + q < nb) x[b0 + k0 + q] -= sq;
      }
    }
    __syncthreads();
    if (wave == 0) {
      double v = lane < nb ? x[b0 + lane] : 0.0;
      const double rd = lane < nb ? 1.0 / Dg[lane * kLuLd + lane] : 1.0;
      for (int i = nb - 1; i >= 0; --i) {
        const double t = lane < i ? Dg[lane * kLuLd + i] : 0.0;
        const double ci = readlane_d(v, i) * readlane_d(rd, i);
        v = lane == i ? ci : v - t * ci;
      }
      if (lane < nb) x[b0 + lane] = v;
    }
    __syncthreads();
  }
  double* out = Cg + (size_t)rcap * cl;
  for (int i = tid; i < rcap; i += kLuThreads) out[i] = i < r ? x[i] : 0.0;
}

// cw[i] = sum_c wc[c] C(i, c), C(:, c) = R column if sampled else Galerkin; also
// writes the r x K matrix Cc (column c scaled by sqrt(mult[c])) for the SVD when Cc != null.
__global__ void cw_kernel(int r, int rcap, int K, const int* __restrict__ sampled,
                          const double* __restrict__ Rst, const double* __restrict__ Cg,
                          const double* __restrict__ wc, const double* __restrict__ mult,
                          double* __restrict__ cw, double* __restrict__ Bsvd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= r) return;
  double s = 0.0;
  for (int c = 0; c < K; ++c) {
    const double v = sampled[c] ? Rst[(size_t)rcap * c + i] : Cg[(size_t)rcap * c + i];
    s += wc[c] * v;
    if (Bsvd) Bsvd[(size_t)i * K + c] = v * std::sqrt(mult[c]);
  }
  cw[i] = s;
}

// part[blk] = sum (a - b)^2 over the block
__global__ void diff2_kernel(const double* __restrict__ a, const double* __restrict__ b, long n,
                             double* __restrict__ part) {
  __shared__ double red[8];
  double s = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double d = a[i] - b[i];
    s += d * d;
  }
  const double w = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += red[k];
    part[blockIdx.x] = t;
  }
}

// ------------------------------------------------------------------ backward Euler source
// Rows r0 .. r0 + pn - 1 of the projected angular source of every class:
// btime[k][r0 + l] = sum_i (Xp_i^T x_{r0+l}) ct[i][k], with xtp[i pn + l] = Xp_i^T x_{r0+l}.
__global__ void time_rows_kernel(int K, int rp, int pn, int r0, int rcap,
                                 const double* __restrict__ xtp, const double* __restrict__ ct,
                                 double* __restrict__ btime) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= K * pn) return;
  const int k = t / pn, l = t % pn;
  double s = 0.0;
  for (int i = 0; i < rp; ++i) s += xtp[(size_t)i * pn + l] * ct[(size_t)i * K + k];
  btime[(size_t)k * rcap + r0 + l] = s;
}

// Ctm[i][m] = ct[i][cls[m]]: the source coefficients of nm classes
__global__ void gather_ct_kernel(const double* __restrict__ ct, int rp, int K,
                                 const int* __restrict__ cls, int nm, double* __restrict__ Ctm) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rp * nm) return;
  const int i = t / nm, m = t % nm;
  Ctm[t] = ct[(size_t)i * K + cls[m]];
}

// out[m] += src for the nm vectors of out
__global__ void add_src_kernel(long nd, int nm, const double* __restrict__ src,
                               double* __restrict__ out) {
  const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nd) return;
  const double v = src[j];
  for (int m = 0; m < nm; ++m) out[(size_t)m * nd + j] += v;
}

// ------------------------------------------------------------------ one-sided Jacobi SVD
// B [r][K] rows rotated pairwise (Hestenes on B^T); Qt [r][r] accumulates the rotations
// (row i of Qt is column i of U).  pairs: [npairs][2] for this round.
__global__ __launch_bounds__(64) void jacobi_round_kernel(double* __restrict__ B, int K,
                                                          double* __restrict__ Qt, int r,
                                                          const int* __restrict__ pairs,
                                                          double* __restrict__ off) {
  const int i = pairs[2 * blockIdx.x], j = pairs[2 * blockIdx.x + 1];
  const int lane = threadIdx.x;
  if (i < 0 || j < 0) {
    if (lane == 0) off[blockIdx.x] = 0.0;
    return;
  }
  double* bi = B + (size_t)i * K;
  double* bj = B + (size_t)j * K;
  double a = 0.0, b = 0.0, g = 0.0;
  for (int t = lane; t < K; t += 64) {
    const double x = bi[t], y = bj[t];
    a += x * x;
    b += y * y;
    g += x * y;
  }
  a = wave_sum(a);
  b = wave_sum(b);
  g = wave_sum(g);
  double o = 0.0;
  if (a > 0.0 && b > 0.0) o = std::fabs(g) / std::sqrt(a * b);
  if (lane == 0) off[blockIdx.x] = o;
  if (o <= 1e-15 || g == 0.0) return;
  const double zeta = (b - a) / (2.0 * g);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
  const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
  for (int u = lane; u < K; u += 64) {
    const double x = bi[u], y = bj[u];
    bi[u] = cs * x - sn * y;
    bj[u] = sn * x + cs * y;
  }
  double* qi = Qt + (size_t)i * r;
  double* qj = Qt + (size_t)j * r;
  for (int u = lane; u < r; u += 64) {
    const double x = qi[u], y = qj[u];
    qi[u] = cs * x - sn * y;
    qj[u] = sn * x + cs * y;
  }
}

__global__ void row_norms_kernel(const double* __restrict__ B, int r, int K, double* __restrict__ s) {
  const int i = blockIdx.x;
  double a = 0.0;
  for (int t = threadIdx.x; t < K; t += 64) a += B[(size_t)i * K + t] * B[(size_t)i * K + t];
  a = wave_sum(a);
  if (threadIdx.x == 0) s[i] = std::sqrt(a);
}

__global__ void identity_kernel(double* Q, int r) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (long)r * r) Q[t] = (t / r == t % r) ? 1.0 : 0.0;
}

// Csel[c][m] = Qt[order[m]][c]  (c < r, m < rp): the kept columns of U
__global__ void gather_u_kernel(const double* __restrict__ Qt, int r, const int* __restrict__ order,
                                int rp, double* __restrict__ Csel) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)r * rp) return;
  const int c = (int)(t / rp), m = (int)(t % rp);
  Csel[t] = Qt[(size_t)order[m] * r + c];
}

// V[m][j] = B[order[m]][cls[j]] / (s_m sqrt(mult[cls[j]]))
__global__ void build_v_kernel(const double* __restrict__ B, int K, const int* __restrict__ order,
                               const double* __restrict__ sv, int rp, const int* __restrict__ cls,
                               const double* __restrict__ mult, int n_dirs, double* __restrict__ V) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)rp * n_dirs) return;
  const int m = (int)(t / n_dirs), j = (int)(t % n_dirs);
  const double s = sv[m];
  const int c = cls[j];
  V[t] = s > 0.0 ? B[(size_t)order[m] * K + c] / (s * std::sqrt(mult[c])) : 0.0;
}

// ------------------------------------------------------------------ DEIM point selection
// Greedy DEIM interpolation points (Chaturantabut-Sorensen) of the leading rp right
// singular vectors of the class coefficient matrix (the alternative sampling of the
// Remark in Sec. 3.2).  The DEIM residual of column l (column l minus its interpolant at
// the points of the previous columns) is column l of the Schur complement after l steps
// of Gaussian elimination, so the points are the row pivots of partial pivoting; one
// workgroup eliminates in place.  W [K][rp] work array, V(c, l) = B[order[l]][c] /
// (s_l sqrt(mult[c])) (B holds S V^T of the multiplicity-weighted classes after the
// one-sided Jacobi rotations).  Pivot: the largest |W(c, l)| over unpicked rows by the
// 30-bit ordering key of the residual norms, the lower class on ties.  Stops once `need`
// unsampled classes are picked or the remaining column is zero; piv gets the points in
// order, npiv[0] their number.  used [K] work flags.
constexpr int kDeimThreads = 256;

__device__ __forceinline__ unsigned long long deim_key(double v) {
  if (!(v > 0.0)) return 0ull;
  int e = 0;
  const double m = frexp(v, &e);
  long long q = (long long)floor(ldexp(m, 30) + 0.5);
  if (q == (1ll << 30)) {
    ++e;
    q = 1ll << 29;
  }
  return ((unsigned long long)(e + 4096) << 32) | (unsigned long long)q;
}

__global__ __launch_bounds__(kDeimThreads) void deim_kernel(
    const double* __restrict__ B, int K, const int* __restrict__ order,
    const double* __restrict__ sv, int rp, const double* __restrict__ mult,
    const int* __restrict__ sampled, int need, double* __restrict__ W, int* __restrict__ used,
    int* __restrict__ piv, int* __restrict__ npiv) {
  __shared__ unsigned long long skey[kDeimThreads];
  __shared__ int sidx[kDeimThreads];
  __shared__ int spiv;
  const int tid = threadIdx.x;
  for (long t = tid; t < (long)K * rp; t += kDeimThreads) {
    const int c = (int)(t / rp), l = (int)(t % rp);
    W[t] = B[(size_t)order[l] * K + c] / (sv[l] * sqrt(mult[c]));
  }
  for (int c = tid; c < K; c += kDeimThreads) used[c] = 0;
  __syncthreads();
  int np = 0, found = 0;
  for (int l = 0; l < rp && found < need; ++l) {
    unsigned long long bk = 0ull;
    int bi = K;
    for (int c = tid; c < K; c += kDeimThreads) {
      if (used[c]) continue;
      const unsigned long long k = deim_key(fabs(W[(size_t)c * rp + l]));
      if (k > bk || (k == bk && c < bi)) {
        bk = k;
        bi = c;
      }
    }
    skey[tid] = bk;
    sidx[tid] = bi;
    __syncthreads();
    for (int h = kDeimThreads / 2; h > 0; h >>= 1) {
      if (tid < h) {
        const unsigned long long ko = skey[tid + h];
        const int io = sidx[tid + h];
        if (ko > skey[tid] || (ko == skey[tid] && io < sidx[tid])) {
          skey[tid] = ko;
          sidx[tid] = io;
        }
      }
      __syncthreads();
    }
    if (skey[0] == 0ull) break;  // the rest of column l is zero: no more points
    if (tid == 0) {
      spiv = sidx[0];
      used[spiv] = 1;
      piv[np] = spiv;
    }
    __syncthreads();
    const int pv = spiv;
    ++np;
    if (!sampled[pv]) ++found;
    // eliminate column l from the unpicked rows (columns l + 1 .. rp - 1)
    const int nr = rp - l - 1;
    const double d = W[(size_t)pv * rp + l];
    if (nr > 0)
      for (long t = tid; t < (long)K * nr; t += kDeimThreads) {
        const int c = (int)(t / nr), k = l + 1 + (int)(t % nr);
        if (used[c]) continue;
        W[(size_t)c * rp + k] -= W[(size_t)c * rp + l] / d * W[(size_t)pv * rp + k];
      }
    __syncthreads();
  }
  if (tid == 0) npiv[0] = np;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Random draws: partial Fisher-Yates over the ascending pool with swap index
// i + floor(u (n - i) / 2^64).
struct Stream {
  const uint64_t* v;
  int64_t n, i = 0;
  uint64_t next() {
    if (i >= n) {
      set_error("random stream exhausted after %lld values", (long long)n);
      throw Error{RTE_ERAND};
    }
    return v[i++];
  }
};

// candidates whose residuals are evaluated together (X C for at most 32 columns)
constexpr int kCandChunk = 32;

std::vector<int> draw(Stream& s, std::vector<int> pool, int k) {
  std::sort(pool.begin(), pool.end());
  const int n = (int)pool.size();
  k = std::min(k, n);
  for (int i = 0; i < k; ++i) {
    const unsigned __int128 prod = (unsigned __int128)s.next() * (unsigned __int128)(n - i);
    const int j = i + (int)(uint64_t)(prod >> 64);
    std::swap(pool[i], pool[j]);
  }
  pool.resize(k);
  return pool;
}

// Ordering key of a residual norm: (binary exponent, mantissa rounded to 30 bits).
// Angles related by a symmetry of the medium have residuals equal in exact arithmetic;
// comparing rounded keys lets the class index break those ties deterministically.
std::pair<int, long long> order_key(double v) {
  if (!(v > 0.0)) return {-100000, 0};
  int e = 0;
  const double m = std::frexp(v, &e);  // v = m 2^e, 0.5 <= m < 1
  long long q = (long long)std::floor(std::ldexp(m, 30) + 0.5);
  if (q == (1LL << 30)) return {e + 1, 1LL << 29};
  return {e, q};
}

// l1 tail rule: smallest l with sum_{i>l} s_i <= eps * sum_i s_i (s descending)
int tail_rank(const std::vector<double>& s, double eps) {
  double tot = 0.0;
  for (double x : s) tot += x;
  if (tot == 0.0) return 0;
  for (size_t l = 0; l <= s.size(); ++l) {
    double tail = 0.0;
    for (size_t i = l; i < s.size(); ++i) tail += s[i];
    if (tail <= eps * tot) return (int)l;
  }
  return (int)s.size();
}

}  // namespace

// The per-class sources of a backward Euler sweep: out[m] = src + Xp ct[:, cls[m]], the
// product as X C in chunks of 32 classes (one pass over Xp per chunk).
void time_class_sources(const TimeSrc& ts, const int* cls_dev, int nm, long nd, const double* src,
                        double* out, double* ctm, hipStream_t st) {
  const unsigned nb = (unsigned)((nd + 255) / 256);
  if (cls_dev)
    hipLaunchKernelGGL(gather_ct_kernel, dim3((ts.rp * nm + 255) / 256), dim3(256), 0, st, ts.ct, ts.rp,
                       ts.K, cls_dev, nm, ctm);
  const double* C = cls_dev ? ctm : ts.ct;
  const int ldc = cls_dev ? nm : ts.K;
  for (int m0 = 0; m0 < nm; m0 += 32)
    hipLaunchKernelGGL((xc_kernel<double, double, 32>), dim3(nb), dim3(256), 0, st, ts.Xp, ts.rp, nd,
                       C + m0, ldc, std::min(32, nm - m0), out + (size_t)m0 * nd);
  hipLaunchKernelGGL(add_src_kernel, dim3(nb), dim3(256), 0, st, nd, nm, src, out);
  RTE_CHECK_HIP(hipGetLastError());
}

// ================================================================== the solver
template <typename T>
struct LowRank {
  const rte_problem* prob;
  const rte_solve_params* prm;
  hipStream_t st;
  Geom g;
  long nd;
  int K = 0, rcap = 0;
  double eps_mgs = 0.0, tol_break = 0.0;
  // classes
  std::vector<int> cls_of, reps;
  std::vector<double> wc, mult;
  std::vector<ClassDev> cd;
  DevBuf<ClassDev> d_cd;
  DevBuf<int> d_cls_of, d_sampled, d_list[4];
  DevBuf<double> d_wc, d_mult;
  // fields
  DevBuf<T> X, Y, V;
  // Snapshots are swept and projected in FP64 in both precisions: their coefficients
  // (the R columns of the sampled classes) enter phi directly, and a rounding bias of
  // the FP32 sweep would be amplified by the DSA step in scattering-dominated cells.
  DevBuf<double> psi, swork;
  DevBuf<double> src, E, phi_k, phi_old, part, cvec, cw, dpart, cb, d1, d2, d3, mstat;
  DevBuf<double> cvecs;  // [kMaxP][rcap + 2]: the device-side MGS2-A's per-snapshot cvec
  DevBuf<double> psi_save;     // snapshots after the batch projections (roll-back copy)
  // basis-update variants of Sec. 4.2: the snapshots of the outer iteration in sampling
  // order (their classes in snap_cls), from which a full QR rebuilds the basis
  DevBuf<double> snaps;
  std::vector<int> snap_cls;
  int full_qrs = 0;
  double* h_mstat = nullptr;   // pinned copy of mstat
  // projected operators and factors
  DevBuf<double> Tm, Dx, Dy, bsrc, bside, Lt, U, yv, Cg, Rst, tsd, tsd2, tsd3, xwp;
  DevBuf<SweepDir> d_dirs;
  DevBuf<double> Cm, rpart, rsums;
  SweepDir* h_dirs = nullptr;  // pinned staging
  int* h_list[4] = {nullptr, nullptr, nullptr, nullptr};  // pinned staging for class lists
  int* h_flags = nullptr;      // pinned staging for the sampled flags
  int rblk = 0;
  // bookkeeping
  std::vector<int> sampled;
  int r = 0;
  int mgs_failures = 0, breakdowns = 0, swept = 0, swept_total = 0;
  Stream rs{nullptr, 0};
  const int32_t* replay = nullptr;
  int64_t n_replay = 0, replay_pos = 0;
  rte_solve_result* res;
  double ms_sweep = 0.0, ms_lr = 0.0;
  hipEvent_t e0, e1;
  // backward Euler step: the angular source psi^m / dt (FP64 only) and its projections
  const TimeSrc* ts = nullptr;
  DevBuf<double> tsrc, twork, btime, tex, tctm, txp;

  bool sweep_pending = false;
  // waits for the stream; adds the time of a sweep enqueued since the last wait
  void sync() {
    RTE_CHECK_HIP(hipStreamSynchronize(st));
    if (sweep_pending) {
      float ms = 0.f;
      RTE_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
      ms_sweep += ms;
      sweep_pending = false;
    }
  }

  void setup() {
    g = make_geom(prob);
    nd = g.ndof;
    // classes of equal (Omega_x, Omega_y), numbered by their smallest ordinate
    const int N = prob->n_dirs;
    cls_of.assign(N, -1);
    for (int j = 0; j < N; ++j) {
      if (cls_of[j] >= 0) continue;
      const int c = (int)reps.size();
      cls_of[j] = c;
      for (int i = j + 1; i < N; ++i)
        if (cls_of[i] < 0 && std::fabs(prob->dirs[3 * i] - prob->dirs[3 * j]) <= 1e-12 &&
            std::fabs(prob->dirs[3 * i + 1] - prob->dirs[3 * j + 1]) <= 1e-12)
          cls_of[i] = c;
      reps.push_back(j);
    }
    K = (int)reps.size();
    wc.assign(K, 0.0);
    mult.assign(K, 0.0);
    for (int j = 0; j < N; ++j) {
      wc[cls_of[j]] += prob->wts[j];
      mult[cls_of[j]] += 1.0;
    }
    cd.resize(K);
    for (int c = 0; c < K; ++c) {
      const double ox = prob->dirs[3 * reps[c]], oy = prob->dirs[3 * reps[c] + 1];
      cd[c] = ClassDev{std::fabs(ox), std::fabs(oy), ox >= 0.0 ? 1 : -1, oy >= 0.0 ? 1 : -1};
    }
    rcap = prm->max_rank > 0 ? std::min(prm->max_rank, K) : K;
    const int p = prm->p;
    RTE_REQUIRE(p <= kMaxP, "p = %d exceeds the supported maximum %d", p, kMaxP);
    RTE_REQUIRE((size_t)2 * p * rcap * sizeof(double) <= 65536,
                "p * max_rank = %d too large for the bordered factorisation", p * rcap);
    RTE_REQUIRE(prm->q <= K, "q = %d exceeds the number of ordinate classes %d", prm->q, K);
    const bool mixed = sizeof(T) == sizeof(float);
    eps_mgs = mixed ? std::max(prm->eps_mgs, 1e-6) : prm->eps_mgs;
    tol_break = mixed ? 1e-6 : 1e-12;
    // device buffers
    d_cd.alloc(K);
    RTE_CHECK_HIP(hipMemcpy(d_cd.get(), cd.data(), K * sizeof(ClassDev), hipMemcpyHostToDevice));
    d_cls_of.alloc(N);
    RTE_CHECK_HIP(hipMemcpy(d_cls_of.get(), cls_of.data(), N * sizeof(int), hipMemcpyHostToDevice));
    d_wc.alloc(K);
    RTE_CHECK_HIP(hipMemcpy(d_wc.get(), wc.data(), K * sizeof(double), hipMemcpyHostToDevice));
    d_mult.alloc(K);
    RTE_CHECK_HIP(hipMemcpy(d_mult.get(), mult.data(), K * sizeof(double), hipMemcpyHostToDevice));
    d_sampled.alloc(K);
    for (int i = 0; i < 4; ++i) d_list[i].alloc(K);
    X.alloc((size_t)rcap * nd);
    psi.alloc((size_t)p * nd);
    swork.alloc(sweep_input_elems(g));  // sweep workspace without the scalar flux
    Y.alloc((size_t)5 * p * nd);
    V.alloc((size_t)32 * nd);
    src.alloc(nd);
    E.alloc((size_t)5 * nd);
    phi_k.alloc(nd);
    phi_old.alloc(nd);
    // projection partials: one row per wavefront (at least 128 rows each), rcap kMaxP dot
    // products and 2 kMaxP norms per row
    const int rdot_cap = std::max(rcap, ts ? ts->rp : 0);  // widest projection basis
    part.alloc((size_t)((nd + 127) / 128 + kPjWaves) * ((size_t)rdot_cap * kMaxP + 2 * kMaxP));
    cb.alloc((size_t)rcap * kMaxP);
    mstat.alloc(4 * kMaxP);
    psi_save.alloc((size_t)p * nd);
    if (prm->basis_update != 0) snaps.alloc((size_t)K * nd);
    RTE_CHECK_HIP(hipHostMalloc((void**)&h_mstat, 4 * kMaxP * sizeof(double), hipHostMallocDefault));
    d1.alloc((size_t)rcap * kMaxP + 2 * kMaxP);
    d2.alloc((size_t)rcap * kMaxP + 2 * kMaxP);
    d3.alloc((size_t)rcap * kMaxP + 2 * kMaxP);
    cvec.alloc(rcap + 2);
    cvecs.alloc((size_t)kMaxP * (rcap + 2));
    cw.alloc(rcap);
    dpart.alloc(4096);
    Tm.alloc((size_t)rcap * rcap); Dx.alloc((size_t)rcap * rcap); Dy.alloc((size_t)rcap * rcap);
    bsrc.alloc(rcap); bside.alloc((size_t)4 * rcap);
    Lt.alloc((size_t)K * rcap * rcap); U.alloc((size_t)K * rcap * rcap);
    yv.alloc((size_t)K * rcap); Cg.alloc((size_t)K * rcap); Rst.alloc((size_t)K * rcap);
    // a p-class plan, or (backward Euler) p one-class plans of up to two entries each
    d_dirs.alloc(2 * kMaxP);
    RTE_CHECK_HIP(hipHostMalloc((void**)&h_dirs, 2 * kMaxP * sizeof(SweepDir), hipHostMallocDefault));
    if (ts && ts->rp > 0) {
      RTE_REQUIRE((std::is_same<T, double>::value), "the backward Euler step is FP64 only");
      tsrc.alloc((size_t)p * nd);
      twork.alloc(sweep_input_elems(g) + (size_t)p * nd);
      btime.alloc((size_t)K * rcap);
      tex.alloc((size_t)kCandChunk * nd);
      tctm.alloc((size_t)ts->rp * kCandChunk);
      txp.alloc((size_t)ts->rp * kMaxP + 2 * kMaxP);
    }
    for (int i = 0; i < 4; ++i)
      RTE_CHECK_HIP(hipHostMalloc((void**)&h_list[i], (size_t)K * sizeof(int), hipHostMallocDefault));
    RTE_CHECK_HIP(hipHostMalloc((void**)&h_flags, (size_t)K * sizeof(int), hipHostMallocDefault));
    rblk = (int)((g.ncell + 255) / 256);
    Cm.alloc((size_t)rcap * 32);
    rpart.alloc((size_t)rblk * 32);
    rsums.alloc(32);
    tsd.alloc((size_t)512 * 5 * kMaxP);
    tsd2.alloc((size_t)rcap * 5 * kMaxP);
    {
      const long nchunk = (nd + kXwRows - 1) / kXwRows;
      const long nch = std::max<long>(1, nchunk / 512);
      xwp.alloc((size_t)((nchunk + nch - 1) / nch) * rcap * 5 * kMaxP);
    }
    tsd3.alloc((size_t)rcap * 2 * kMaxP + 5 * kMaxP);
    RTE_CHECK_HIP(hipEventCreate(&e0));
    RTE_CHECK_HIP(hipEventCreate(&e1));
    // boundary unit vectors (rows 1..4 of E); row 0 holds the source of the outer step
    hipLaunchKernelGGL(gunit_kernel, dim3((g.ncell + 255) / 256), dim3(256), 0, st, g.nx, g.ny,
                       g.mb, g.hx, g.hy, prob->bc, E.get(), nd);
    RTE_CHECK_HIP(hipGetLastError());
    rs.v = prm->rand;
    rs.n = prm->rand ? prm->n_rand : 0;
    replay = prm->replay;
    n_replay = prm->replay ? prm->n_replay : 0;
  }

  ~LowRank() {
    if (h_dirs) (void)hipHostFree(h_dirs);
    for (int i = 0; i < 4; ++i)
      if (h_list[i]) (void)hipHostFree(h_list[i]);
    if (h_mstat) (void)hipHostFree(h_mstat);
    if (h_flags) (void)hipHostFree(h_flags);
  }

  // ------------------------------------------------------------ sweeps
  void sweep_classes(const std::vector<int>& cl) {
    if (ts && ts->rp > 0) {
      sweep_classes_time(cl);
      return;
    }
    RTE_CHECK_HIP(hipEventRecord(e0, st));
    std::vector<SweepDir> dirs;
    for (size_t i = 0; i < cl.size(); ++i) {
      const ClassDev& k = cd[cl[i]];
      SweepDir d;
      d.a = k.ax / g.hx;
      d.b = k.ay / g.hy;
      d.w = 0.0;
      d.sx = k.sx;
      d.sy = k.sy;
      d.slot = (int)i;
      d.pad = 0;
      dirs.push_back(d);
    }
    SweepPlan pl = make_sweep_plan(g, dirs, false, true, sizeof(double));
    std::memcpy(h_dirs, pl.groups.data(), pl.groups.size() * sizeof(SweepDir));
    RTE_CHECK_HIP(hipMemcpyAsync(d_dirs.get(), h_dirs, pl.groups.size() * sizeof(SweepDir),
                                 hipMemcpyHostToDevice, st));
    sweep_enqueue<double>(g, pl, d_dirs.get(), prob->sigma_t, src.get(), prob->bc, psi.get(),
                          nullptr, swork.get(), st);
    RTE_CHECK_HIP(hipEventRecord(e1, st));
    sweep_pending = true;  // timed at the next synchronisation (see sync)
    swept += (int)cl.size();
    swept_total += (int)cl.size();
  }

  // Backward Euler: the classes differ in their angular source; one sweep with a source
  // per class (row i of tsrc for slot i).
  void sweep_classes_time(const std::vector<int>& cl) {
    RTE_CHECK_HIP(hipEventRecord(e0, st));
    std::vector<SweepDir> dirs;
    for (size_t i = 0; i < cl.size(); ++i) {
      const ClassDev& k = cd[cl[i]];
      SweepDir d;
      d.a = k.ax / g.hx;
      d.b = k.ay / g.hy;
      d.w = 0.0;
      d.sx = k.sx;
      d.sy = k.sy;
      d.slot = (int)i;
      d.pad = 0;
      dirs.push_back(d);
    }
    SweepPlan pl = make_sweep_plan(g, dirs, false, true, sizeof(double), true);
    RTE_REQUIRE(pl.groups.size() <= 2 * (size_t)kMaxP, "internal: sweep staging too small");
    RTE_REQUIRE(sweep_work_elems(g, pl, false) <= twork.n, "internal: sweep workspace too small");
    std::memcpy(h_dirs, pl.groups.data(), pl.groups.size() * sizeof(SweepDir));
    RTE_CHECK_HIP(hipMemcpyAsync(d_dirs.get(), h_dirs, pl.groups.size() * sizeof(SweepDir),
                                 hipMemcpyHostToDevice, st));
    const int* dl = upload_list(3, cl);
    time_class_sources(*ts, dl, (int)cl.size(), nd, src.get(), tsrc.get(), tctm.get(), st);
    sweep_enqueue<double>(g, pl, d_dirs.get(), prob->sigma_t, tsrc.get(), prob->bc, psi.get(),
                          nullptr, twork.get(), st);
    RTE_CHECK_HIP(hipEventRecord(e1, st));
    sweep_pending = true;
    swept += (int)cl.size();
    swept_total += (int)cl.size();
  }

  // ------------------------------------------------------------ projections
  template <int NV>
  void bproj_n(double* W, const T* Xu, int r_upd, const double* C, const T* Xd, int r_dot,
               double* out, double* acc_into) {
    const long nwf = (nd + PjCfg<NV>::rows - 1) / PjCfg<NV>::rows;
    const int nb = (int)((nwf + kPjWaves - 1) / kPjWaves);
    const size_t sm = (size_t)(r_upd * NV + kPjWaves * kPjRed) * sizeof(double);
    const int n = r_dot * NV + 2 * NV;
    RTE_REQUIRE(part.n >= (size_t)nb * kPjWaves * n, "internal: projection scratch too small");
    hipLaunchKernelGGL((bproj_kernel<T, double, NV>), dim3(nb), dim3(64 * kPjWaves), sm, st, Xu, r_upd, C,
                       Xd, r_dot, W, nd, part.get());
    reduce_cols(part.get(), nb * kPjWaves, n, n, out, acc_into, st, acc_into ? r_dot * NV : 0);
    RTE_CHECK_HIP(hipGetLastError());
  }
  // W: nv vectors (stride nd).  If r_upd > 0, W -= Xu C (C: [r_upd][nv]); then
  // out[c nv + l] = Xd[c]^T W[l] for c < r_dot, out[r_dot nv + l] = ||W[l]||^2 after the
  // update, out[r_dot nv + nv + l] = ||W[l]||^2 before it; acc_into[j] += out[j] for the
  // dot products when acc_into is given.
  void bproj(double* W, int nv, const T* Xu, int r_upd, const double* C, const T* Xd, int r_dot,
             double* out, double* acc_into) {
    switch (nv) {
      case 1: bproj_n<1>(W, Xu, r_upd, C, Xd, r_dot, out, acc_into); break;
      case 2: bproj_n<2>(W, Xu, r_upd, C, Xd, r_dot, out, acc_into); break;
      case 3: bproj_n<3>(W, Xu, r_upd, C, Xd, r_dot, out, acc_into); break;
      case 4: bproj_n<4>(W, Xu, r_upd, C, Xd, r_dot, out, acc_into); break;
      case 5: bproj_n<5>(W, Xu, r_upd, C, Xd, r_dot, out, acc_into); break;
      case 6: bproj_n<6>(W, Xu, r_upd, C, Xd, r_dot, out, acc_into); break;
      case 7: bproj_n<7>(W, Xu, r_upd, C, Xd, r_dot, out, acc_into); break;
      case 8: bproj_n<8>(W, Xu, r_upd, C, Xd, r_dot, out, acc_into); break;
      default: RTE_REQUIRE(false, "internal: projection batch of %d vectors", nv);
    }
  }

  void to_host(double* h, const double* d, int n) {
    RTE_CHECK_HIP(hipMemcpyAsync(h, d, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, st));
  }

  // MGS2-A (Alg. 2) for the sampled snapshots psi[0 .. pn) of classes cls[0 .. pn).
  // Alg. 2 takes the snapshots one after the other, each against the basis including the
  // columns appended before it in the same batch.  Here the two projections against the
  // basis as it stood before the batch are made for all snapshots together (one pass over
  // X serves the whole batch); then, snapshot by snapshot in batch order, two projections
  // against the columns appended earlier in the batch, the normalisation, the clean-up
  // projections and the append.  The appended columns are orthogonal to the old basis,
  // so both orders give the same snapshots and coefficients in exact arithmetic.
  //
  // The per-snapshot steps first run on the device without waiting for the host, on the
  // assumption that no snapshot breaks down and none needs a clean-up projection (the
  // usual case); the host then checks the statistics of every snapshot in order and, from
  // the first one that fails, rolls back (basis size, snapshots restored from a copy taken
  // after the batch projections) and takes the decisions one snapshot at a time.
  void mgs_batch(const std::vector<int>& cls) {
    const int pn = (int)cls.size();
    const int r0 = r;
    if (r0 > 0) {
      device_fill(cb.get(), 0.0, (long)r0 * pn, st);
      const T* X0 = X.get();
      // pass 1: C1 = X^T psi;  pass 2: psi -= X C1, C2 = X^T psi;  pass 3: psi -= X C2
      bproj(psi.get(), pn, nullptr, 0, nullptr, X0, r0, d1.get(), cb.get());
      bproj(psi.get(), pn, X0, r0, d1.get(), X0, r0, d2.get(), cb.get());
      bproj(psi.get(), pn, X0, r0, d2.get(), X0, 1, d3.get(), nullptr);
    } else {
      bproj(psi.get(), pn, nullptr, 0, nullptr, nullptr, 0, d3.get(), nullptr);
    }
    hipLaunchKernelGGL(mstat_init_kernel, dim3(1), dim3(64), 0, st, pn, r0, d1.get(), d3.get(),
                       mstat.get());
    RTE_CHECK_HIP(hipGetLastError());
    int lseq = 0;  // first snapshot taken with host decisions
    if (r0 + pn <= rcap) {
      RTE_CHECK_HIP(hipMemcpyAsync(psi_save.get(), psi.get(), (size_t)pn * nd * sizeof(double),
                                   hipMemcpyDeviceToDevice, st));
      // every snapshot's coefficients against the old basis at once (one slice each)
      const int nc = rcap + 2;
      hipLaunchKernelGGL(coef_cols_kernel, dim3((nc + 127) / 128, pn), dim3(128), 0, st, cb.get(),
                         pn, r0, cvecs.get(), nc);
      for (int l = 0; l < pn; ++l) {
        double* v = psi.get() + (size_t)l * nd;
        double* cv = cvecs.get() + (size_t)l * nc;
        if (l > 0) intra_passes(v, r0, l, cv);
        hipLaunchKernelGGL((snapshot_done_kernel<double, T>), dim3((nd + 255) / 256), dim3(256), 0,
                           st, v, nd, X.get() + (size_t)(r0 + l) * nd, l > 0 ? d3.get() : nullptr,
                           mstat.get() + 4 * l, cv, r0 + l, Rst.get() + (size_t)rcap * cls[l], rcap);
        RTE_CHECK_HIP(hipGetLastError());
      }
      to_host(h_mstat, mstat.get(), 4 * pn);
      sync();
      lseq = pn;
      for (int l = 0; l < pn && lseq == pn; ++l) {
        const double* m = h_mstat + 4 * l;
        const double alpha = std::sqrt(m[0]);
        if (alpha <= tol_break * std::sqrt(m[1]) || alpha == 0.0 ||
            (r0 + l > 0 && std::fabs(m[2]) / alpha > eps_mgs))
          lseq = l;
      }
      r = r0 + lseq;
      if (lseq == pn) return;
      RTE_CHECK_HIP(hipMemcpyAsync(psi.get() + (size_t)lseq * nd, psi_save.get() + (size_t)lseq * nd,
                                   (size_t)(pn - lseq) * nd * sizeof(double), hipMemcpyDeviceToDevice, st));
    } else {
      to_host(h_mstat, mstat.get(), 4 * pn);
      sync();
    }
    for (int l = lseq; l < pn; ++l) {
      double* v = psi.get() + (size_t)l * nd;
      coef_col(l, pn, r0);
      double nrm2 = h_mstat[4 * l], x1dot = h_mstat[4 * l + 2];
      const int nnew = r - r0;
      if (nnew > 0) {
        double tail[2];
        intra_passes(v, r0, nnew);
        to_host(tail, d3.get(), 2);
        sync();
        x1dot = tail[0];
        nrm2 = tail[1];
      }
      finish(v, cls[l], nrm2, h_mstat[4 * l + 1], x1dot);
    }
  }

  // cvec = (coefficients of snapshot l against the old basis, zeros)
  void coef_col(int l, int pn, int r0) {
    hipLaunchKernelGGL(coef_col_kernel, dim3((rcap + 2 + 127) / 128), dim3(128), 0, st, cb.get(),
                       pn, l, r0, cvec.get(), rcap + 2);
    RTE_CHECK_HIP(hipGetLastError());
  }

  // two projections of v against the nnew columns appended after r0 (coefficients into
  // cv[r0 ..], cv = cvec by default); the last pass leaves X(:,1)^T v and |v|^2 in d3[0],
  // d3[1]
  void intra_passes(double* v, int r0, int nnew, double* cv = nullptr) {
    const T* Xn = X.get() + (size_t)r0 * nd;
    if (!cv) cv = cvec.get();
    bproj(v, 1, nullptr, 0, nullptr, Xn, nnew, d1.get(), cv + r0);
    bproj(v, 1, Xn, nnew, d1.get(), Xn, nnew, d2.get(), cv + r0);
    bproj(v, 1, Xn, nnew, d2.get(), X.get(), 1, d3.get(), nullptr);
  }

  // Normalisation, clean-up projections and append of one snapshot whose coefficients
  // against the current basis are in cvec (Alg. 2); a snapshot that vanishes against
  // the basis (breakdown) keeps its coefficients and adds no column.
  bool finish(double* v, int cl, double nrm2, double orig2, double x1dot) {
    double alpha = std::sqrt(nrm2);
    if (alpha <= tol_break * std::sqrt(orig2) || alpha == 0.0) {
      ++breakdowns;
      hipLaunchKernelGGL(store_coef_kernel, dim3((rcap + 127) / 128), dim3(128), 0, st, cvec.get(),
                         r, 0.0, 0, Rst.get() + (size_t)rcap * cl, rcap);
      RTE_CHECK_HIP(hipGetLastError());
      return false;
    }
    if (r > 0) {
      double t = std::fabs(x1dot) / alpha;
      for (int m = 0; m < prm->m_max && t > eps_mgs; ++m) {
        double tail[2];
        bproj(v, 1, nullptr, 0, nullptr, X.get(), r, d1.get(), cvec.get());
        bproj(v, 1, X.get(), r, d1.get(), X.get(), 1, d3.get(), nullptr);
        to_host(tail, d3.get(), 2);
        sync();
        alpha = std::sqrt(tail[1]);
        t = std::fabs(tail[0]) / alpha;
      }
      if (t > eps_mgs) ++mgs_failures;
    }
    RTE_REQUIRE(r < rcap, "the basis reached max_rank = %d", rcap);
    hipLaunchKernelGGL((append_kernel<double, T>), dim3((nd + 255) / 256), dim3(256), 0, st, v,
                       1.0 / alpha, X.get() + (size_t)r * nd, nd);
    hipLaunchKernelGGL(store_coef_kernel, dim3((rcap + 127) / 128), dim3(128), 0, st, cvec.get(), r,
                       alpha, 1, Rst.get() + (size_t)rcap * cl, rcap);
    RTE_CHECK_HIP(hipGetLastError());
    ++r;
    return true;
  }

  // ------------------------------------------------------------ basis-update variants
  // (Sec. 4.2).  A full QR factorises the matrix of all snapshots of the outer iteration
  // again: Gram-Schmidt with two projections per snapshot (and the clean-up passes of
  // Alg. 2), in sampling order, from an empty basis, so the sampled classes get the
  // columns of R as coefficients.  The projected operators and the Galerkin factors of
  // the unsampled classes are then rebuilt from the new basis (rebuild_operators): the
  // incremental bordering needs the nested basis that a full QR does not keep.

  // copies the pn snapshots of the batch behind the stored ones (not yet counted)
  void stash_batch(int pn) {
    RTE_CHECK_HIP(hipMemcpyAsync(snaps.get() + snap_cls.size() * (size_t)nd, psi.get(),
                                 (size_t)pn * nd * sizeof(double), hipMemcpyDeviceToDevice, st));
  }

  // the basis from scratch over the first snap_cls.size() stored snapshots
  void rebuild_basis() {
    ++full_qrs;
    const int mf = mgs_failures, bd = breakdowns;
    r = 0;
    const int ns = (int)snap_cls.size(), p = prm->p;
    for (int c0 = 0; c0 < ns; c0 += p) {
      const int pn = std::min(p, ns - c0);
      RTE_CHECK_HIP(hipMemcpyAsync(psi.get(), snaps.get() + (size_t)c0 * nd,
                                   (size_t)pn * nd * sizeof(double), hipMemcpyDeviceToDevice, st));
      mgs_batch(std::vector<int>(snap_cls.begin() + c0, snap_cls.begin() + c0 + pn));
    }
    mgs_failures = mf;  // the rebuild's own clean-up decisions are not Alg. 2 failures
    breakdowns = bd;
  }

  // projected operators and Galerkin factors of `uns` for the whole current basis
  void rebuild_operators(const std::vector<int>& uns) {
    for (int c0 = 0; c0 < r; c0 += prm->p) {
      const int pn = std::min(prm->p, r - c0);
      border(c0, pn);
      lu_border(c0, pn, uns);
    }
  }

  // MGS-QR: per snapshot one block projection against the basis, normalisation and the
  // orthogonality test against X(:,1); a failure replaces the basis by a full QR of the
  // snapshots so far.  Returns true if the basis was replaced (the operators must then
  // be rebuilt, not bordered).
  bool mgs_qr_batch(const std::vector<int>& cls) {
    const int pn = (int)cls.size();
    const int ns0 = (int)snap_cls.size();
    stash_batch(pn);
    bool fresh = false;
    for (int l = 0; l < pn; ++l) {
      double* v = psi.get() + (size_t)l * nd;
      RTE_CHECK_HIP(hipMemcpyAsync(v, snaps.get() + (size_t)(ns0 + l) * nd, nd * sizeof(double),
                                   hipMemcpyDeviceToDevice, st));
      snap_cls.push_back(cls[l]);
      device_fill(cvec.get(), 0.0, rcap + 2, st);
      double tail[3] = {0.0, 0.0, 0.0};  // X(:,1)^T v, |v|^2 after, |v|^2 before
      if (r > 0) {
        bproj(v, 1, nullptr, 0, nullptr, X.get(), r, d1.get(), cvec.get());
        bproj(v, 1, X.get(), r, d1.get(), X.get(), 1, d3.get(), nullptr);
        to_host(tail, d3.get(), 3);
      } else {
        bproj(v, 1, nullptr, 0, nullptr, nullptr, 0, d3.get(), nullptr);
        to_host(tail + 1, d3.get(), 2);
      }
      sync();
      const double alpha = std::sqrt(tail[1]);
      if (alpha <= tol_break * std::sqrt(tail[2]) || alpha == 0.0) {
        ++breakdowns;
        hipLaunchKernelGGL(store_coef_kernel, dim3((rcap + 127) / 128), dim3(128), 0, st,
                           cvec.get(), r, 0.0, 0, Rst.get() + (size_t)rcap * cls[l], rcap);
        RTE_CHECK_HIP(hipGetLastError());
        continue;
      }
      if (r > 0 && std::fabs(tail[0]) / alpha > eps_mgs) {
        rebuild_basis();
        fresh = true;
        continue;
      }
      RTE_REQUIRE(r < rcap, "the basis reached max_rank = %d", rcap);
      hipLaunchKernelGGL((append_kernel<double, T>), dim3((nd + 255) / 256), dim3(256), 0, st, v,
                         1.0 / alpha, X.get() + (size_t)r * nd, nd);
      hipLaunchKernelGGL(store_coef_kernel, dim3((rcap + 127) / 128), dim3(128), 0, st,
                         cvec.get(), r, alpha, 1, Rst.get() + (size_t)rcap * cls[l], rcap);
      RTE_CHECK_HIP(hipGetLastError());
      ++r;
    }
    return fresh;
  }

  // ------------------------------------------------------------ bordering
  // out[e pn + m] = E[e]^T P[m] for the 5 vectors of E and the pn new columns P
  template <int PN>
  void edot_n(const T* P, int nbk) {
    hipLaunchKernelGGL((edot_kernel<T, PN>), dim3(nbk), dim3(kTB), 0, st, E.get(), P, nd, tsd.get());
  }
  void edot(const T* P, int pn, double* out) {
    const int nbk = 512;
    switch (pn) {
      case 1: edot_n<1>(P, nbk); break;
      case 2: edot_n<2>(P, nbk); break;
      case 3: edot_n<3>(P, nbk); break;
      case 4: edot_n<4>(P, nbk); break;
      case 5: edot_n<5>(P, nbk); break;
      case 6: edot_n<6>(P, nbk); break;
      case 7: edot_n<7>(P, nbk); break;
      case 8: edot_n<8>(P, nbk); break;
      default: RTE_REQUIRE(false, "internal: %d new columns", pn);
    }
    reduce_cols(tsd.get(), nbk, 5 * pn, 5 * pn, out, nullptr, st);
    RTE_CHECK_HIP(hipGetLastError());
  }

  template <int NV>
  void xtw_n(const T* A, int na, const T* B, dim3 grid, int nch) {
    hipLaunchKernelGGL((xtw_kernel<T, NV>), grid, dim3(256), 0, st, A, na, B, nd, nch, xwp.get());
  }
  // out[a nb + b] = A[a]^T B[b] for a < na columns of A, b < nb = 5 pn vectors of B
  void xtw(const T* A, int na, const T* B, int nb, double* out) {
    const long nchunk = (nd + kXwRows - 1) / kXwRows;
    const int nch = (int)std::max<long>(1, nchunk / 512);
    const int nbk = (int)((nchunk + nch - 1) / nch);
    RTE_REQUIRE(xwp.n >= (size_t)nbk * na * nb, "internal: X^T W scratch too small");
    const dim3 grid(nbk, (na + 255) / 256);
    switch (nb) {
      case 5: xtw_n<5>(A, na, B, grid, nch); break;
      case 10: xtw_n<10>(A, na, B, grid, nch); break;
      case 15: xtw_n<15>(A, na, B, grid, nch); break;
      case 20: xtw_n<20>(A, na, B, grid, nch); break;
      case 25: xtw_n<25>(A, na, B, grid, nch); break;
      case 30: xtw_n<30>(A, na, B, grid, nch); break;
      case 35: xtw_n<35>(A, na, B, grid, nch); break;
      case 40: xtw_n<40>(A, na, B, grid, nch); break;
      default: RTE_REQUIRE(false, "internal: X^T W with %d vectors", nb);
    }
    reduce_cols(xwp.get(), nbk, na * nb, na * nb, out, nullptr, st);
    RTE_CHECK_HIP(hipGetLastError());
  }

  void border(int r0, int pn) {
    const T* P = X.get() + (size_t)r0 * nd;
    hipLaunchKernelGGL((border_stencil_kernel<T>), dim3((g.ncell + 255) / 256), dim3(256), 0, st,
                       g.nx, g.ny, 1.0 / g.hx, 1.0 / g.hy, prob->sigma_t, P, pn, nd, Y.get());
    RTE_CHECK_HIP(hipGetLastError());
    const int r1 = r0 + pn;
    // X^T [Sigma_t P, D_x^- P, D_y^- P, (D_x^-)^T P, (D_y^-)^T P] in one pass over X
    // (the last two blocks are used for the old rows only)
    xtw(X.get(), r1, Y.get(), 5 * pn, tsd2.get());
    double* ext = tsd3.get();
    edot(P, pn, ext);
    const int nt = std::max(r1 * pn, 5);
    hipLaunchKernelGGL(scatter_border_kernel, dim3((nt + 127) / 128), dim3(128), 0, st, r0, pn,
                       rcap, tsd2.get(), ext, Tm.get(), Dx.get(), Dy.get(), bsrc.get(),
                       bside.get());
    RTE_CHECK_HIP(hipGetLastError());
    if constexpr (std::is_same<T, double>::value) {
      if (ts && ts->rp > 0) {
        // X_new^T psi^m_k / dt = (Xp^T X_new)^T ct[k]: the new rows of every class's
        // right-hand side
        bproj(const_cast<double*>(P), pn, nullptr, 0, nullptr, ts->Xp, ts->rp, txp.get(), nullptr);
        hipLaunchKernelGGL(time_rows_kernel, dim3((K * pn + 127) / 128), dim3(128), 0, st, K, ts->rp,
                           pn, r0, rcap, txp.get(), ts->ct, btime.get());
        RTE_CHECK_HIP(hipGetLastError());
      }
    }
  }

  // Class lists: 0 for the bordered factorisations, 1 for the candidates, 2 for the
  // unsampled classes at a convergence check or the truncation, 3 for the sampled classes
  // of a backward Euler sweep.  Each kind is uploaded
  // at most once between two synchronisations of the inner loop, so its staging buffer
  // is free again when it is next written.
  const int* upload_list(int kind, const std::vector<int>& l) {
    std::memcpy(h_list[kind], l.data(), l.size() * sizeof(int));
    RTE_CHECK_HIP(hipMemcpyAsync(d_list[kind].get(), h_list[kind], l.size() * sizeof(int),
                                 hipMemcpyHostToDevice, st));
    return d_list[kind].get();
  }

  void lu_border(int r0, int pn, const std::vector<int>& classes) {
    if (classes.empty() || pn == 0) return;
    const int* dl = upload_list(0, classes);
    const size_t sm = ((size_t)pn * r0 + (size_t)kLuB * kLuLd) * sizeof(double);
    if (r0 > 0)
      hipLaunchKernelGGL(lu_border_kernel, dim3((unsigned)classes.size(), 2), dim3(kLuThreads), sm,
                         st, r0, pn, rcap, dl, d_cd.get(), Tm.get(), Dx.get(), Dy.get(), Lt.get(),
                         U.get());
    hipLaunchKernelGGL(lu_corner_kernel, dim3((unsigned)classes.size()), dim3(kLuThreads), 0, st,
                       r0, pn, rcap, dl, d_cd.get(), Tm.get(), Dx.get(), Dy.get(), bsrc.get(),
                       bside.get(), btime.get(), Lt.get(), U.get(), yv.get());
    RTE_CHECK_HIP(hipGetLastError());
  }

  // Galerkin coefficients of the classes (list kind `kind`, see upload_list)
  void galerkin(const std::vector<int>& classes, int kind) {
    if (classes.empty() || r == 0) return;
    const int* dl = upload_list(kind, classes);
    hipLaunchKernelGGL(backsub_kernel, dim3((unsigned)classes.size()), dim3(kLuThreads),
                       ((size_t)r + (size_t)kLuB * kLuLd) * sizeof(double), st, r, rcap, dl,
                       U.get(), yv.get(), Cg.get());
    RTE_CHECK_HIP(hipGetLastError());
  }

  // Galerkin solves and residual norms of the candidates (host values in draw order)
  // Residual norms of the candidates, evaluated kCandChunk at a time (q may exceed it:
  // with q >= the number of unsampled ordinates every one of them is a candidate, the
  // fully greedy selection).
  std::vector<double> residuals(const std::vector<int>& cand) {
    const int ntot = (int)cand.size();
    std::vector<double> out(ntot, 0.0);
    for (int c0 = 0; c0 < ntot; c0 += kCandChunk) {
      const int nm = std::min(kCandChunk, ntot - c0);
      residual_chunk(std::vector<int>(cand.begin() + c0, cand.begin() + c0 + nm), out.data() + c0);
    }
    for (auto& x : out) x = std::sqrt(x);
    return out;
  }

  // squared residual norms of nm <= kCandChunk candidates into out (synchronous)
  void residual_chunk(const std::vector<int>& cand, double* out) {
    const int nm = (int)cand.size();
    const int* dl = upload_list(1, cand);
    if (r > 0) {
      hipLaunchKernelGGL(backsub_kernel, dim3((unsigned)nm), dim3(kLuThreads),
                         ((size_t)r + (size_t)kLuB * kLuLd) * sizeof(double), st, r, rcap, dl,
                         U.get(), yv.get(), Cg.get());
      hipLaunchKernelGGL(gather_cg_kernel, dim3((r * nm + 255) / 256), dim3(256), 0, st, Cg.get(),
                         rcap, dl, nm, r, Cm.get());
      hipLaunchKernelGGL((xc_kernel<T, T, 32>), dim3((nd + 255) / 256), dim3(256), 0, st, X.get(), r,
                         nd, Cm.get(), nm, nm, V.get());
    } else {
      RTE_CHECK_HIP(hipMemsetAsync(V.get(), 0, (size_t)nm * nd * sizeof(T), st));
    }
    double* exv = nullptr;  // backward Euler: psi^m / dt of each candidate
    if constexpr (std::is_same<T, double>::value) {
      if (ts && ts->rp > 0) {
        hipLaunchKernelGGL(gather_ct_kernel, dim3((ts->rp * nm + 255) / 256), dim3(256), 0, st, ts->ct,
                           ts->rp, ts->K, dl, nm, tctm.get());
        hipLaunchKernelGGL((xc_kernel<double, double, 32>), dim3((nd + 255) / 256), dim3(256), 0, st,
                           ts->Xp, ts->rp, nd, tctm.get(), nm, nm, tex.get());
        exv = tex.get();
      }
    }
    hipLaunchKernelGGL((residual_kernel<T>), dim3(rblk, nm), dim3(256), 0, st, g.nx, g.ny,
                       1.0 / g.hx, 1.0 / g.hy, prob->sigma_t, src.get(), E.get(), nd, V.get(), nm,
                       dl, d_cd.get(), exv, rpart.get());
    reduce_cols(rpart.get(), rblk, nm, nm, rsums.get(), nullptr, st);
    RTE_CHECK_HIP(hipGetLastError());
    RTE_CHECK_HIP(hipMemcpyAsync(out, rsums.get(), nm * sizeof(double), hipMemcpyDeviceToHost, st));
    sync();
  }

  // phi_k = X (C w) with the current coefficients; Bsvd optional
  void scalar_flux(double* Bsvd) {
    std::memcpy(h_flags, sampled.data(), K * sizeof(int));
    RTE_CHECK_HIP(hipMemcpyAsync(d_sampled.get(), h_flags, K * sizeof(int),
                                 hipMemcpyHostToDevice, st));
    if (r == 0) {
      device_fill(phi_k.get(), 0.0, nd, st);
      return;
    }
    hipLaunchKernelGGL(cw_kernel, dim3((r + 63) / 64), dim3(64), 0, st, r, rcap, K, d_sampled.get(),
                       Rst.get(), Cg.get(), d_wc.get(), d_mult.get(), cw.get(), Bsvd);
    hipLaunchKernelGGL((xc_kernel<T, double, 1>), dim3((nd + 255) / 256), dim3(256), 0, st, X.get(), r,
                       nd, cw.get(), 1, 1, phi_k.get());
    RTE_CHECK_HIP(hipGetLastError());
  }

  double diff_norm(const double* a, const double* b) {
    const int nb = 1024;
    hipLaunchKernelGGL(diff2_kernel, dim3(nb), dim3(256), 0, st, a, b, nd, dpart.get());
    double* out = dpart.get() + 2048;
    reduce_cols(dpart.get(), nb, 1, 1, out, nullptr, st);
    RTE_CHECK_HIP(hipGetLastError());
    double h = 0.0;
    RTE_CHECK_HIP(hipMemcpyAsync(&h, out, sizeof(double), hipMemcpyDeviceToHost, st));
    sync();
    return std::sqrt(h);
  }

  // Replay list: per outer iteration, groups "count, id, ..." ended by a 0 count.
  // Returns the next group of this outer iteration, or an empty vector when the
  // outer iteration's groups are used up (the greedy choice then takes over).
  std::vector<int> next_replay() {
    if (!replay || replay_pos >= n_replay) return {};
    const int cnt = replay[replay_pos];
    if (cnt == 0) return {};
    RTE_REQUIRE(cnt >= 1 && cnt <= prm->p && replay_pos + 1 + cnt <= n_replay, "bad replay group");
    std::vector<int> v(replay + replay_pos + 1, replay + replay_pos + 1 + cnt);
    replay_pos += 1 + cnt;
    for (int c : v)
      RTE_REQUIRE(c >= 0 && c < K && !sampled[c], "replay class %d invalid or already sampled", c);
    return v;
  }
  // skip to the start of the next outer iteration's groups
  void end_replay_outer() {
    if (!replay) return;
    while (replay_pos < n_replay && replay[replay_pos] != 0) replay_pos += 1 + replay[replay_pos];
    if (replay_pos < n_replay) ++replay_pos;
  }

  void log_sample(int c) {
    if (res && res->sample_log && res->sample_log_len < res->sample_log_cap)
      res->sample_log[res->sample_log_len++] = c;
  }
  void log_resid(double v) {
    if (res && res->resid_log && res->resid_log_len < res->resid_log_cap)
      res->resid_log[res->resid_log_len++] = v;
  }

  // ------------------------------------------------------------ one low-rank SI
  // On entry src holds Sigma_s phi_prev + G; phi_old = phi_prev.
  void inner(const double* phi_prev) {
    const auto t0 = std::chrono::steady_clock::now();
    const double ms_sw0 = ms_sweep;
    r = 0;
    sampled.assign(K, 0);
    RTE_CHECK_HIP(hipMemcpyAsync(phi_old.get(), phi_prev, nd * sizeof(double), hipMemcpyDeviceToDevice, st));
    std::vector<int> samples = next_replay();
    if (samples.empty()) {
      std::vector<int> all(K);
      std::iota(all.begin(), all.end(), 0);
      samples = draw(rs, all, prm->p);
    }
    snap_cls.clear();
    while (true) {
      sweep_classes(samples);
      const int r0 = r;
      bool fresh = false;  // basis replaced by a full QR: rebuild, do not border
      if (prm->basis_update == 0) {
        mgs_batch(samples);
      } else if (prm->basis_update == 1) {
        fresh = mgs_qr_batch(samples);
      } else {
        stash_batch((int)samples.size());
        snap_cls.insert(snap_cls.end(), samples.begin(), samples.end());
        rebuild_basis();
        fresh = true;
      }
      for (int c : samples) {
        sampled[c] = 1;
        log_sample(c);
      }
      const int pn = r - r0;
      std::vector<int> uns;
      for (int c = 0; c < K; ++c)
        if (!sampled[c]) uns.push_back(c);
      if (fresh) {
        rebuild_operators(uns);
      } else if (pn > 0) {
        border(r0, pn);
        lu_border(r0, pn, uns);
      }
      if (uns.empty()) {
        scalar_flux(nullptr);
        break;
      }
      std::vector<int> cand = draw(rs, uns, prm->q);
      std::vector<double> rn = residuals(cand);
      for (double v : rn) log_resid(v);
      double mx = 0.0;
      for (double v : rn) mx = std::max(mx, v);
      bool stop = false;
      if (mx < prm->eps_res) {
        galerkin(uns, 2);
        scalar_flux(nullptr);
        const double d = diff_norm(phi_k.get(), phi_old.get());
        if (d <= prm->eps_diff) stop = true;
        else
          RTE_CHECK_HIP(hipMemcpyAsync(phi_old.get(), phi_k.get(), nd * sizeof(double),
                                       hipMemcpyDeviceToDevice, st));
      }
      if (stop) break;
      samples = next_replay();
      if (samples.empty()) {
        std::vector<int> order(cand.size());
        std::iota(order.begin(), order.end(), 0);
        std::vector<std::pair<int, long long>> key(cand.size());
        for (size_t i = 0; i < cand.size(); ++i) key[i] = order_key(rn[i]);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
          if (key[a] != key[b]) return key[a] > key[b];
          return cand[a] < cand[b];
        });
        samples.clear();
        for (int i = 0; i < (int)order.size() && (int)samples.size() < prm->p; ++i)
          samples.push_back(cand[order[i]]);
        if (prm->sampling == 1) {
          std::vector<int> greedy;
          for (int i : order) greedy.push_back(cand[i]);
          samples = deim_samples(greedy);
        }
      }
    }
    end_replay_outer();
    ms_lr += ms_since(t0) - (ms_sweep - ms_sw0);
  }

  // ------------------------------------------------------------ truncation (Sec. 3.3)
  // One-sided Jacobi SVD of the r x K class matrix B (columns weighted by the square roots
  // of the class multiplicities, so that its singular values are those of the r x N_Omega
  // coefficient matrix): on return the rows of B are s_i v_i^T, the rows of Qt the
  // columns of U, order the rows by descending singular value and sorted the values.
  void svd_rows(double* Bp, double* Qtp, std::vector<int>& order, std::vector<double>& sorted) {
    DevBuf<double> sv(r);
    hipLaunchKernelGGL(identity_kernel, dim3((r * r + 255) / 256), dim3(256), 0, st, Qtp, r);
    // round-robin pairs
    const int m = r + (r & 1);
    const int npairs = m / 2;
    std::vector<int> pairs((size_t)(m - 1) * npairs * 2);
    std::vector<int> ring(m);
    std::iota(ring.begin(), ring.end(), 0);
    for (int rd = 0; rd < m - 1; ++rd) {
      for (int k = 0; k < npairs; ++k) {
        int a = ring[k], b = ring[m - 1 - k];
        if (a >= r || b >= r) a = b = -1;
        pairs[((size_t)rd * npairs + k) * 2] = a;
        pairs[((size_t)rd * npairs + k) * 2 + 1] = b;
      }
      // rotate all but the first
      const int last = ring[m - 1];
      for (int k = m - 1; k > 1; --k) ring[k] = ring[k - 1];
      ring[1] = last;
    }
    DevBuf<int> dpairs(pairs.size());
    RTE_CHECK_HIP(hipMemcpy(dpairs.get(), pairs.data(), pairs.size() * sizeof(int), hipMemcpyHostToDevice));
    DevBuf<double> off((size_t)(m - 1) * npairs);
    std::vector<double> hoff((size_t)(m - 1) * npairs);
    for (int sweep = 0; sweep < 60 && m > 1; ++sweep) {
      for (int rd = 0; rd < m - 1; ++rd)
        hipLaunchKernelGGL(jacobi_round_kernel, dim3(npairs), dim3(64), 0, st, Bp, K, Qtp, r,
                           dpairs.get() + (size_t)rd * npairs * 2, off.get() + (size_t)rd * npairs);
      RTE_CHECK_HIP(hipGetLastError());
      RTE_CHECK_HIP(hipMemcpyAsync(hoff.data(), off.get(), hoff.size() * sizeof(double),
                                   hipMemcpyDeviceToHost, st));
      sync();
      double mx = 0.0;
      for (double v : hoff) mx = std::max(mx, v);
      if (mx <= 1e-15) break;
    }
    hipLaunchKernelGGL(row_norms_kernel, dim3(r), dim3(64), 0, st, Bp, r, K, sv.get());
    std::vector<double> hs(r);
    RTE_CHECK_HIP(hipMemcpyAsync(hs.data(), sv.get(), r * sizeof(double), hipMemcpyDeviceToHost, st));
    sync();
    order.resize(r);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hs[a] > hs[b]; });
    sorted.resize(r);
    for (int i = 0; i < r; ++i) sorted[i] = hs[order[i]];
  }

  // the r x K class matrix (multiplicity-weighted columns, Galerkin coefficients for the
  // unsampled classes) into Bp
  void class_matrix(double* Bp) {
    std::vector<int> uns;
    for (int c = 0; c < K; ++c)
      if (!sampled[c]) uns.push_back(c);
    galerkin(uns, 2);
    std::memcpy(h_flags, sampled.data(), K * sizeof(int));
    RTE_CHECK_HIP(hipMemcpyAsync(d_sampled.get(), h_flags, K * sizeof(int),
                                 hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(cw_kernel, dim3((r + 63) / 64), dim3(64), 0, st, r, rcap, K, d_sampled.get(),
                       Rst.get(), Cg.get(), d_wc.get(), d_mult.get(), cw.get(), Bp);
    RTE_CHECK_HIP(hipGetLastError());
  }

  // DEIM sampling (Remark in Sec. 3.2): the first p unsampled classes among the DEIM points
  // of the leading r' right singular vectors of C (r' by the eps_svd rule); fewer are
  // completed from `greedy` (the candidates in residual order).
  std::vector<int> deim_samples(const std::vector<int>& greedy) {
    std::vector<int> out;
    if (r > 0) {
      DevBuf<double> B((size_t)r * K), Qt((size_t)r * r);
      class_matrix(B.get());
      std::vector<int> order;
      std::vector<double> sorted;
      svd_rows(B.get(), Qt.get(), order, sorted);
      const int rp = tail_rank(sorted, prm->eps_svd);
      if (rp > 0) {
        DevBuf<int> dord(rp), used(K), piv(rp + 1);
        DevBuf<double> dsv(rp), Wk((size_t)K * rp);
        RTE_CHECK_HIP(hipMemcpyAsync(dord.get(), order.data(), rp * sizeof(int), hipMemcpyHostToDevice, st));
        RTE_CHECK_HIP(hipMemcpyAsync(dsv.get(), sorted.data(), rp * sizeof(double), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(deim_kernel, dim3(1), dim3(kDeimThreads), 0, st, B.get(), K, dord.get(),
                           dsv.get(), rp, d_mult.get(), d_sampled.get(), prm->p, Wk.get(), used.get(),
                           piv.get(), piv.get() + rp);
        RTE_CHECK_HIP(hipGetLastError());
        std::vector<int> hp(rp + 1);
        RTE_CHECK_HIP(hipMemcpyAsync(hp.data(), piv.get(), (rp + 1) * sizeof(int), hipMemcpyDeviceToHost, st));
        sync();
        for (int i = 0; i < hp[rp]; ++i)
          if (!sampled[hp[i]] && (int)out.size() < prm->p) out.push_back(hp[i]);
      }
    }
    for (int c : greedy) {
      if ((int)out.size() >= prm->p) break;
      if (std::find(out.begin(), out.end(), c) == out.end()) out.push_back(c);
    }
    return out;
  }

  int truncate(double* Xo, double* So, double* Vo) {
    if (r == 0) return 0;
    DevBuf<double> B((size_t)r * K), Qt((size_t)r * r);
    // coefficients of every class (Galerkin for the unsampled ones)
    class_matrix(B.get());
    std::vector<int> order;
    std::vector<double> sorted;
    svd_rows(B.get(), Qt.get(), order, sorted);
    const int rp = tail_rank(sorted, prm->eps_svd);
    if (rp > 0 && (Xo || So || Vo)) {
      DevBuf<int> dord(rp);
      RTE_CHECK_HIP(hipMemcpy(dord.get(), order.data(), rp * sizeof(int), hipMemcpyHostToDevice));
      if (So) RTE_CHECK_HIP(hipMemcpyAsync(So, sorted.data(), rp * sizeof(double), hipMemcpyHostToDevice, st));
      if (Xo) {
        DevBuf<double> Csel((size_t)r * rp);
        hipLaunchKernelGGL(gather_u_kernel, dim3((r * rp + 255) / 256), dim3(256), 0, st, Qt.get(), r,
                           dord.get(), rp, Csel.get());
        for (int m0 = 0; m0 < rp; m0 += 32)
          hipLaunchKernelGGL((xc_kernel<T, double, 32>), dim3((nd + 255) / 256), dim3(256), 0, st, X.get(),
                             r, nd, Csel.get() + m0, rp, std::min(32, rp - m0), Xo + (size_t)m0 * nd);
        RTE_CHECK_HIP(hipGetLastError());
        sync();
      }
      if (Vo) {
        DevBuf<double> dsv(rp);
        RTE_CHECK_HIP(hipMemcpy(dsv.get(), sorted.data(), rp * sizeof(double), hipMemcpyHostToDevice));
        const long tot = (long)rp * prob->n_dirs;
        hipLaunchKernelGGL(build_v_kernel, dim3((tot + 255) / 256), dim3(256), 0, st, B.get(), K,
                           dord.get(), dsv.get(), rp, d_cls_of.get(), d_mult.get(), prob->n_dirs, Vo);
        RTE_CHECK_HIP(hipGetLastError());
      }
      sync();
    }
    return rp;
  }
};

template <typename T>
static rte_status run_lowrank(const rte_problem* prob, const rte_solve_params* prm,
                              const double* phi0, double* phi_out, double* Xo, double* So,
                              double* Vo, rte_solve_result* res, hipStream_t st,
                              const TimeSrc* ts) {
  const auto t_start = std::chrono::steady_clock::now();
  LowRank<T> lr;
  lr.prob = prob;
  lr.prm = prm;
  lr.st = st;
  lr.res = res;
  lr.ts = ts;
  lr.setup();
  const long nd = lr.nd;
  const Geom& g = lr.g;
  DevBuf<double> phi_prev(nd);
  if (phi0)
    RTE_CHECK_HIP(hipMemcpyAsync(phi_prev.get(), phi0, nd * sizeof(double), hipMemcpyDeviceToDevice, st));
  else
    device_fill(phi_prev.get(), 0.0, nd, st);
  std::unique_ptr<DSA, void (*)(DSA*)> dsa(nullptr, dsa_destroy);
  if (prm->use_dsa) dsa.reset(dsa_create(g, prob->sigma_t, prob->sigma_s, st));
  double ms_dsa = 0.0;
  int dsa_iters = 0, n = 0, rank = 0;
  bool conv = false;
  for (n = 1; n <= prm->max_outer; ++n) {
    make_source<double>(g, prob->sigma_s, phi_prev.get(), prob->G, lr.src.get(), st);
    RTE_CHECK_HIP(hipMemcpyAsync(lr.E.get(), lr.src.get(), nd * sizeof(double),
                                 hipMemcpyDeviceToDevice, st));
    lr.inner(phi_prev.get());
    const double d = max_abs_diff(lr.phi_k.get(), phi_prev.get(), nd, st);
    if (res && res->history) res->history[n - 1] = d;
    if (res && res->ranks) res->ranks[n - 1] = lr.r;
    if (res && res->swept) res->swept[n - 1] = lr.swept;
    if (prm->phi_checkpoints)
      RTE_CHECK_HIP(hipMemcpyAsync(prm->phi_checkpoints + (long)(n - 1) * nd, lr.phi_k.get(),
                                   nd * sizeof(double), hipMemcpyDeviceToDevice, st));
    conv = d <= prm->eps_si;
    const bool last = conv || n == prm->max_outer;
    // the truncation of Sec. 3.3 after every inner loop when its rank is asked for (the
    // oversampling metric of Sec. 4); X U, S and V are formed for the last one only
    if (last || (res && res->trunc_ranks)) {
      const int rp = last ? lr.truncate(Xo, So, Vo) : lr.truncate(nullptr, nullptr, nullptr);
      if (res && res->trunc_ranks) res->trunc_ranks[n - 1] = rp;
      if (last) rank = rp;
    }
    if (progress_enabled())
      std::fprintf(stderr, "[rte] low rank: outer %d, |phi* - phi|_inf %.3e, basis %d, swept %d, %.0f ms\n",
                   n, d, lr.r, lr.swept, ms_since(t_start));
    if (last) break;
    const auto t0 = std::chrono::steady_clock::now();
    if (dsa) {
      dsa_iters += dsa_apply(dsa.get(), lr.phi_k.get(), phi_prev.get(), phi_prev.get(), prm->eps_dsa, st);
      RTE_CHECK_HIP(hipStreamSynchronize(st));
    } else {
      RTE_CHECK_HIP(hipMemcpyAsync(phi_prev.get(), lr.phi_k.get(), nd * sizeof(double),
                                   hipMemcpyDeviceToDevice, st));
    }
    ms_dsa += ms_since(t0);
    lr.swept = 0;
  }
  if (n > prm->max_outer) n = prm->max_outer;
  RTE_CHECK_HIP(hipMemcpyAsync(phi_out, lr.phi_k.get(), nd * sizeof(double), hipMemcpyDeviceToDevice, st));
  RTE_CHECK_HIP(hipStreamSynchronize(st));
  if (res) {
    res->outer_iters = n;
    res->converged = conv ? 1 : 0;
    res->rank = rank;
    res->n_swept = lr.swept_total;
    res->mgs_failures = lr.mgs_failures;
    res->breakdowns = lr.breakdowns;
    res->full_qrs = lr.full_qrs;
    res->dsa_iters = dsa_iters;
    res->ms_sweep = lr.ms_sweep;
    res->ms_lowrank = lr.ms_lr;
    res->ms_dsa = ms_dsa;
    res->ms_total = ms_since(t_start);
  }
  (void)hipEventDestroy(lr.e0);
  (void)hipEventDestroy(lr.e1);
  return conv ? RTE_OK : RTE_ENOCONV;
}

rte_status lowrank_solve(const rte_problem* prob, const rte_solve_params* prm, const double* phi0,
                         double* phi_out, double* X, double* S, double* V, rte_solve_result* res,
                         hipStream_t st, const TimeSrc* ts) {
  if (prm->prec == RTE_FP64) return run_lowrank<double>(prob, prm, phi0, phi_out, X, S, V, res, st, ts);
  RTE_REQUIRE(!ts || ts->rp == 0, "the backward Euler step is FP64 only");
  return run_lowrank<float>(prob, prm, phi0, phi_out, X, S, V, res, st, ts);
}

}  // namespace rte
