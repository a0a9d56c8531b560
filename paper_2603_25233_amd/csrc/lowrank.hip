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
// A block of kProjWaves wavefronts covers kProjRows consecutive rows; each lane owns
// kProjRpt rows (lane-interleaved, so every column read is one contiguous run per
// wavefront).
//   If r_upd > 0: v -= sum_{c<r_upd} X[c] dc[c] (written back), one sum per row.
//   Then part[blk][c] = X[c]^T v over the block's rows for c < r_dot, 16 columns at a
//   time: each lane sums its rows, the 64 x 16 lane partials of a wavefront are
//   transposed through LDS and summed in a fixed order, then the wavefronts' sums are
//   added in wavefront order.
//   part[blk][r_dot] = v.v after the update, part[blk][r_dot + 1] = v.v before.
constexpr int kProjRpt = 2;
constexpr int kProjWaves = 4;
constexpr int kProjRows = 64 * kProjRpt * kProjWaves;
constexpr int kProjCols = 16;
constexpr int kProjRed = 64 * (kProjCols + 1) + 4 * kProjCols;  // LDS doubles per wavefront

// Column sums over the block: every lane contributes kProjCols values; lane c <
// kProjCols of wavefront 0 returns the block sum of column c.  red: kProjWaves *
// kProjRed + kProjWaves * kProjCols doubles of LDS.
__device__ __forceinline__ double block_colsum(const double (&p)[kProjCols], double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int LD = kProjCols + 1;
  double* rw = red + wave * kProjRed;
#pragma unroll
  for (int j = 0; j < kProjCols; ++j) rw[lane * LD + j] = p[j];
  __syncthreads();
  const int col = lane % kProjCols, seg = lane / kProjCols;  // 4 segments of 16 lanes
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) s += rw[(seg * 16 + u) * LD + col];
  double* r2 = rw + 64 * LD;
  r2[seg * kProjCols + col] = s;
  __syncthreads();
  double* wsum = red + kProjWaves * kProjRed;
  if (lane < kProjCols) {
    double t = 0.0;
#pragma unroll
    for (int g = 0; g < 4; ++g) t += r2[g * kProjCols + lane];
    wsum[wave * kProjCols + lane] = t;
  }
  __syncthreads();
  double t = 0.0;
  if (wave == 0 && lane < kProjCols)
#pragma unroll
    for (int w = 0; w < kProjWaves; ++w) t += wsum[w * kProjCols + lane];
  __syncthreads();
  return t;
}

template <typename T>
__global__ __launch_bounds__(64 * kProjWaves) void proj_kernel(
    const T* __restrict__ X, long nd, int r_upd, int r_dot, T* __restrict__ v,
    const double* __restrict__ dc, double* __restrict__ part) {
  extern __shared__ double sm[];
  double* sdc = sm;            // [r_upd]
  double* red = sm + r_upd;    // reduction buffers
  const int tid = threadIdx.x;
  const long i0 = (long)blockIdx.x * kProjRows + (tid >> 6) * (64 * kProjRpt) + (tid & 63);
  for (int c = tid; c < r_upd; c += 64 * kProjWaves) sdc[c] = dc[c];
  __syncthreads();
  double x[kProjRpt];
  bool ok[kProjRpt];
  double before = 0.0, after = 0.0;
#pragma unroll
  for (int t = 0; t < kProjRpt; ++t) {
    const long i = i0 + 64 * t;
    ok[t] = i < nd;
    x[t] = ok[t] ? (double)v[i] : 0.0;
    before += x[t] * x[t];
  }
  if (r_upd > 0) {
    double s[kProjRpt];
#pragma unroll
    for (int t = 0; t < kProjRpt; ++t) s[t] = 0.0;
    // 8 columns per round: all loads of a round are issued before its sums
    int c = 0;
    for (; c + 8 <= r_upd; c += 8) {
      double xv[8][kProjRpt];
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int t = 0; t < kProjRpt; ++t)
          xv[u][t] = ok[t] ? (double)X[(long)(c + u) * nd + i0 + 64 * t] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double d = sdc[c + u];
#pragma unroll
        for (int t = 0; t < kProjRpt; ++t) s[t] += xv[u][t] * d;
      }
    }
    for (; c < r_upd; ++c) {
      const double d = sdc[c];
#pragma unroll
      for (int t = 0; t < kProjRpt; ++t)
        if (ok[t]) s[t] += (double)X[(long)c * nd + i0 + 64 * t] * d;
    }
#pragma unroll
    for (int t = 0; t < kProjRpt; ++t)
      if (ok[t]) {
        v[i0 + 64 * t] = (T)(x[t] - s[t]);
        x[t] = (double)v[i0 + 64 * t];  // the stored (possibly rounded) value
      }
  }
#pragma unroll
  for (int t = 0; t < kProjRpt; ++t) after += x[t] * x[t];
  const int stride = r_dot + 2;
  double* out = part + (long)blockIdx.x * stride;
  for (int c0 = 0; c0 < r_dot; c0 += kProjCols) {
    double p[kProjCols];
#pragma unroll
    for (int j = 0; j < kProjCols; ++j) {
      p[j] = 0.0;
      if (c0 + j < r_dot) {
        const T* xc = X + (long)(c0 + j) * nd;
#pragma unroll
        for (int t = 0; t < kProjRpt; ++t)
          if (ok[t]) p[j] += (double)xc[i0 + 64 * t] * x[t];
      }
    }
    const double tot = block_colsum(p, red);
    if (tid < kProjCols && c0 + tid < r_dot) out[c0 + tid] = tot;
  }
  double p[kProjCols];
#pragma unroll
  for (int j = 0; j < kProjCols; ++j) p[j] = j == 0 ? after : (j == 1 ? before : 0.0);
  const double tot = block_colsum(p, red);
  if (tid < 2) out[r_dot + tid] = tot;
}

// out[c] = sum_b part[b][c] for c < n (and acc_into[c] += out[c] for c < n_acc).  A block of
// 256 threads handles 8 columns: 32 lanes per column take every 32nd partial (four
// running sums, fixed assignment), then a fixed pairwise tree combines the lanes, so
// the sum is the same on every run.
__global__ __launch_bounds__(256) void reduce_cols_kernel(const double* __restrict__ part, int nblk,
                                                          int stride, int n, double* __restrict__ out,
                                                          double* __restrict__ acc_into, int n_acc) {
  __shared__ double red[256];
  const int c = blockIdx.x * 8 + (threadIdx.x >> 5);
  const int l = threadIdx.x & 31;
  double s4[4] = {0.0, 0.0, 0.0, 0.0};
  if (c < n) {
    int b = l;
    for (; b + 96 < nblk; b += 128)
#pragma unroll
      for (int u = 0; u < 4; ++u) s4[u] += part[(long)(b + 32 * u) * stride + c];
    if (b < nblk) s4[0] += part[(long)b * stride + c];
    if (b + 32 < nblk) s4[1] += part[(long)(b + 32) * stride + c];
    if (b + 64 < nblk) s4[2] += part[(long)(b + 64) * stride + c];
  }
  red[threadIdx.x] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
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

static void reduce_cols(const double* part, int nblk, int stride, int n, double* out,
                        double* acc_into, hipStream_t st, int n_acc = 0) {
  hipLaunchKernelGGL(reduce_cols_kernel, dim3((n + 7) / 8), dim3(256), 0, st, part, nblk, stride, n,
                     out, acc_into, n_acc);
}

template <typename T>
__global__ void append_kernel(const T* __restrict__ v, double inv_alpha, T* __restrict__ col,
                              long nd) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nd) col[i] = (T)((double)v[i] * inv_alpha);
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

// ------------------------------------------------------------------ tall-skinny A^T B
// part[chunk][a][b] = sum over the chunk rows of A[a][.] B[b][.]  (a < na, b < nb)
// Block tile: 64 vectors of A (blockIdx.x) x 32 of B (blockIdx.z) over 32 rows at a
// time, staged in LDS; the next 32 rows are fetched into registers while the current
// ones are used.
template <typename TA, typename TB>
__global__ __launch_bounds__(256) void tsdot_kernel(const TA* __restrict__ A, int na,
                                                    const TB* __restrict__ B, int nb, long nd,
                                                    long kchunk, double* __restrict__ part) {
  __shared__ double As[32][65];
  __shared__ double Bs[32][33];
  const int a0 = blockIdx.x * 64, b0 = blockIdx.z * 32;
  const long k0 = (long)blockIdx.y * kchunk, k1 = min(nd, k0 + kchunk);
  const int ta = threadIdx.x & 31, tb = threadIdx.x >> 5;  // tb in 0..7
  // element e = threadIdx.x + 256 u of a tile: column e >> 5, row e & 31
  double ra[8], rb[4];
  auto fetch = [&](long kk) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = threadIdx.x + 256 * u, col = e >> 5;
      const long k = kk + (e & 31);
      ra[u] = (a0 + col < na && k < k1) ? (double)A[(long)(a0 + col) * nd + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = threadIdx.x + 256 * u, col = e >> 5;
      const long k = kk + (e & 31);
      rb[u] = (b0 + col < nb && k < k1) ? (double)B[(long)(b0 + col) * nd + k] : 0.0;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = threadIdx.x + 256 * u;
      As[e & 31][e >> 5] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = threadIdx.x + 256 * u;
      Bs[e & 31][e >> 5] = rb[u];
    }
  };
  double acc[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
  fetch(k0);
  stash();
  __syncthreads();
  for (long kk = k0; kk < k1; kk += 32) {
    const bool more = kk + 32 < k1;
    if (more) fetch(kk + 32);
#pragma unroll 8
    for (int k = 0; k < 32; ++k) {
      const double x0 = As[k][ta], x1 = As[k][ta + 32];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double y = Bs[k][tb + 8 * j];
        acc[0][j] += x0 * y;
        acc[1][j] += x1 * y;
      }
    }
    __syncthreads();
    if (more) stash();
    __syncthreads();
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 4; ++j) {
      const int a = a0 + ta + 32 * i, b = b0 + tb + 8 * j;
      if (a < na && b < nb) part[((long)blockIdx.y * na + a) * nb + b] = acc[i][j];
    }
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
      double x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = ok ? (double)X[(long)(c0 + c + u) * nd + i] : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int m = 0; m < NM; ++m) acc[m] += x[u] * Cs[c + u][m];
    }
    for (; c < cn; ++c) {
      const double x = ok ? (double)X[(long)(c0 + c) * nd + i] : 0.0;
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
    const ClassDev* __restrict__ cd, double* __restrict__ part) {
  __shared__ double red[8];
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  const ClassDev k = cd[cls[m]];
  const T* u = V + (long)m * nd;
  double s2 = 0.0;
  if (c < (long)nx * ny) {
    const int a = (int)(c % nx), b = (int)(c / nx);
    Q4 dx = k.sx > 0 ? dxm(u, c, a, ihx) : dxmT(u, c, a, nx, ihx);
    Q4 dy = k.sy > 0 ? dym(u, c, b, nx, ihy) : dymT(u, c, b, nx, ny, ihy);
    Q4 x = ld4(u + 4 * c);
    const double* gx = E + (long)(1 + (k.sx > 0 ? 0 : 1)) * nd + 4 * c;
    const double* gy = E + (long)(1 + (k.sy > 0 ? 2 : 3)) * nd + 4 * c;
    for (int q = 0; q < 4; ++q) {
      const double rr = src[4 * c + q] + k.ax * gx[q] + k.ay * gy[q] - k.ax * dx.v[q] -
                        k.ay * dy.v[q] - sig[c] * x.v[q];
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
// Scatter the border blocks computed by tsdot into the projected matrices.
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
// One 64-thread workgroup per class in cls[].  Factor storage per class:
//   Lt[rcap][rcap]: Lt[i][j] = L(j, i) (column i of the unit lower factor, j > i)
//   U [rcap][rcap]: row-major upper factor;  y[rcap]: L^{-1} b.
// Extends the factorisation of the leading r0 x r0 block by pn rows/columns.
constexpr int kLuRows = 8;  // factor rows staged per round in lu_border_kernel

__global__ __launch_bounds__(64) void lu_border_kernel(
    int r0, int pn, int rcap, const int* __restrict__ cls, const ClassDev* __restrict__ cd,
    const double* __restrict__ Tm, const double* __restrict__ Dx, const double* __restrict__ Dy,
    const double* __restrict__ bsrc, const double* __restrict__ bside, double* __restrict__ Lt_all,
    double* __restrict__ U_all, double* __restrict__ y_all) {
  extern __shared__ double sm[];
  double* col = sm;                       // [pn][r0]: A_12 -> U_12
  double* row = sm + (long)pn * r0;       // [pn][r0]: A_21 -> L_21
  __shared__ double S[kMaxP][kMaxP], yn[kMaxP];
  const int cl = cls[blockIdx.x];
  const ClassDev k = cd[cl];
  const size_t fsz = (size_t)rcap * rcap;
  double* Lt = Lt_all + fsz * cl;
  double* U = U_all + fsz * cl;
  double* y = y_all + (size_t)rcap * cl;
  const int lane = threadIdx.x;
  for (int m = 0; m < pn; ++m)
    for (int i = lane; i < r0; i += 64) {
      col[m * r0 + i] = amat(Tm, Dx, Dy, rcap, k, i, r0 + m);
      row[m * r0 + i] = amat(Tm, Dx, Dy, rcap, k, r0 + m, i);
    }
  __syncthreads();
  // Rows of L^T and U are staged in LDS kLuRows at a time (columns from the block's
  // first row on), so the sequential sweeps below wait for global memory once per
  // kLuRows rows.
  double* stg = sm + (size_t)2 * pn * r0;  // [kLuRows][r0]
  // U_12 = L_11^{-1} A_12 (unit lower, column sweeps)
  for (int i0 = 0; i0 < r0; i0 += kLuRows) {
    const int nb = min(kLuRows, r0 - i0), w = r0 - i0;
    __syncthreads();
    for (int ii = 0; ii < nb; ++ii)
      for (int j = lane; j < w; j += 64) stg[ii * w + j] = Lt[(size_t)(i0 + ii) * rcap + i0 + j];
    __syncthreads();
    for (int ii = 0; ii < nb; ++ii) {
      const int i = i0 + ii;
      const int lb = ii * w - i0;  // stg[lb + j] = L^T(i, j)
      for (int j = i + 1 + lane; j < r0; j += 64) {
        const double l = stg[lb + j];
        for (int m = 0; m < pn; ++m) col[m * r0 + j] -= l * col[m * r0 + i];
      }
      __syncthreads();
    }
  }
  // L_21 = A_21 U_11^{-1}: x U = a, row sweeps of U
  for (int i0 = 0; i0 < r0; i0 += kLuRows) {
    const int nb = min(kLuRows, r0 - i0), w = r0 - i0;
    __syncthreads();
    for (int ii = 0; ii < nb; ++ii)
      for (int j = lane; j < w; j += 64) stg[ii * w + j] = U[(size_t)(i0 + ii) * rcap + i0 + j];
    __syncthreads();
    for (int ii = 0; ii < nb; ++ii) {
      const int i = i0 + ii;
      const int ub = ii * w - i0;  // stg[ub + j] = U(i, j)
      const double piv = stg[ub + i];
      for (int m = 0; m < pn; ++m) {
        // every lane reads the current a_i before lane 0 rescales it
        const double xi = row[m * r0 + i] / piv;
        for (int j = i + 1 + lane; j < r0; j += 64) row[m * r0 + j] -= xi * stg[ub + j];
        __syncthreads();
        if (lane == 0) row[m * r0 + i] = xi;
      }
      __syncthreads();
    }
  }
  // S = A_22 - L_21 U_12 and the new entries of y
  for (int m = 0; m < pn; ++m)
    for (int mm = 0; mm < pn; ++mm) {
      double s = 0.0;
      for (int i = lane; i < r0; i += 64) s += row[m * r0 + i] * col[mm * r0 + i];
      s = wave_sum(s);
      if (lane == 0) S[m][mm] = amat(Tm, Dx, Dy, rcap, k, r0 + m, r0 + mm) - s;
    }
  for (int m = 0; m < pn; ++m) {
    double s = 0.0;
    for (int i = lane; i < r0; i += 64) s += row[m * r0 + i] * y[i];
    s = wave_sum(s);
    if (lane == 0) yn[m] = bvec(bsrc, bside, rcap, k, r0 + m) - s;
  }
  __syncthreads();
  if (lane == 0) {
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
  for (int m = 0; m < pn; ++m)
    for (int i = lane; i < r0; i += 64) {
      U[(size_t)i * rcap + r0 + m] = col[m * r0 + i];
      Lt[(size_t)i * rcap + r0 + m] = row[m * r0 + i];
    }
}

// c = U^{-1} y for each class in cls[] (row-oriented back substitution) -> Cg[cl][.]
__global__ __launch_bounds__(64) void backsub_kernel(int r, int rcap, const int* __restrict__ cls,
                                                     const double* __restrict__ U_all,
                                                     const double* __restrict__ y_all,
                                                     double* __restrict__ Cg) {
  extern __shared__ double x[];
  const int cl = cls[blockIdx.x];
  const double* U = U_all + (size_t)rcap * rcap * cl;
  const double* y = y_all + (size_t)rcap * cl;
  const int lane = threadIdx.x;
  for (int i = r - 1; i >= 0; --i) {
    const double* ui = U + (size_t)i * rcap;
    double s = 0.0;
    for (int j = i + 1 + lane; j < r; j += 64) s += ui[j] * x[j];
    s = wave_sum(s);
    if (lane == 0) x[i] = (y[i] - s) / ui[i];
    __syncthreads();
  }
  double* out = Cg + (size_t)rcap * cl;
  for (int i = lane; i < rcap; i += 64) out[i] = i < r ? x[i] : 0.0;
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

// ================================================================== the solver
template <typename T>
struct LowRank {
  const rte_problem* prob;
  const rte_solve_params* prm;
  hipStream_t st;
  Geom g;
  long nd;
  int K = 0, rcap = 0, nblk = 0;
  long chunk = 0;
  double eps_mgs = 0.0, tol_break = 0.0;
  // classes
  std::vector<int> cls_of, reps;
  std::vector<double> wc, mult;
  std::vector<ClassDev> cd;
  DevBuf<ClassDev> d_cd;
  DevBuf<int> d_cls_of, d_sampled, d_list;
  DevBuf<double> d_wc, d_mult;
  // fields
  DevBuf<T> X, psi, srcT, Y, V, swork;
  DevBuf<double> src, E, phi_k, phi_old, part, dvec, cvec, cw, dpart;
  // projected operators and factors
  DevBuf<double> Tm, Dx, Dy, bsrc, bside, Lt, U, yv, Cg, Rst, tsd, tsd2, tsd3;
  DevBuf<SweepDir> d_dirs;
  DevBuf<double> Cm, rpart, rsums;
  SweepDir* h_dirs = nullptr;  // pinned staging
  int* h_list = nullptr;       // pinned staging for class lists
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

  void sync() { RTE_CHECK_HIP(hipStreamSynchronize(st)); }

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
    RTE_REQUIRE(prm->q <= 32, "q = %d exceeds the supported maximum 32", prm->q);
    const bool mixed = sizeof(T) == sizeof(float);
    eps_mgs = mixed ? std::max(prm->eps_mgs, 1e-6) : prm->eps_mgs;
    tol_break = mixed ? 1e-6 : 1e-12;
    chunk = kProjRows;
    nblk = (int)((nd + chunk - 1) / chunk);
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
    d_list.alloc(K);
    X.alloc((size_t)rcap * nd);
    psi.alloc((size_t)p * nd);
    srcT.alloc(nd);
    swork.alloc(sweep_input_elems(g));  // sweep workspace without the scalar flux
    Y.alloc((size_t)5 * p * nd);
    V.alloc((size_t)32 * nd);
    src.alloc(nd);
    E.alloc((size_t)5 * nd);
    phi_k.alloc(nd);
    phi_old.alloc(nd);
    part.alloc((size_t)nblk * (rcap + 2) + 64);
    dvec.alloc(rcap + 2);
    cvec.alloc(rcap + 2);
    cw.alloc(rcap);
    dpart.alloc(4096);
    Tm.alloc((size_t)rcap * rcap); Dx.alloc((size_t)rcap * rcap); Dy.alloc((size_t)rcap * rcap);
    bsrc.alloc(rcap); bside.alloc((size_t)4 * rcap);
    Lt.alloc((size_t)K * rcap * rcap); U.alloc((size_t)K * rcap * rcap);
    yv.alloc((size_t)K * rcap); Cg.alloc((size_t)K * rcap); Rst.alloc((size_t)K * rcap);
    d_dirs.alloc(kMaxP);
    RTE_CHECK_HIP(hipHostMalloc((void**)&h_dirs, kMaxP * sizeof(SweepDir), hipHostMallocDefault));
    RTE_CHECK_HIP(hipHostMalloc((void**)&h_list, (size_t)K * sizeof(int), hipHostMallocDefault));
    RTE_CHECK_HIP(hipHostMalloc((void**)&h_flags, (size_t)K * sizeof(int), hipHostMallocDefault));
    rblk = (int)((g.ncell + 255) / 256);
    Cm.alloc((size_t)rcap * 32);
    rpart.alloc((size_t)rblk * 32);
    rsums.alloc(32);
    tsd.alloc((size_t)65536 * 5 * kMaxP);  // nch * na <= 65536 (see tsdot), nb <= 5 kMaxP
    tsd2.alloc((size_t)rcap * 5 * kMaxP);
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
    if (h_list) (void)hipHostFree(h_list);
    if (h_flags) (void)hipHostFree(h_flags);
  }

  // ------------------------------------------------------------ sweeps
  void sweep_classes(const std::vector<int>& cl) {
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
    SweepPlan pl = make_sweep_plan(g, dirs, false, true, sizeof(T));
    std::memcpy(h_dirs, pl.groups.data(), pl.groups.size() * sizeof(SweepDir));
    RTE_CHECK_HIP(hipMemcpyAsync(d_dirs.get(), h_dirs, pl.groups.size() * sizeof(SweepDir),
                                 hipMemcpyHostToDevice, st));
    sweep_enqueue<T>(g, pl, d_dirs.get(), prob->sigma_t, srcT.get(), prob->bc, psi.get(), nullptr,
                     swork.get(), st);
    RTE_CHECK_HIP(hipEventRecord(e1, st));
    sync();
    float ms = 0.f;
    RTE_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
    ms_sweep += ms;
    swept += (int)cl.size();
    swept_total += (int)cl.size();
  }

  // ------------------------------------------------------------ projections
  // part <- proj_kernel(...); then dvec[0..r_dot+2) = column sums; if acc, cvec += dots
  void proj(T* v, int r_upd, const double* dc, int r_dot, bool acc) {
    const size_t sm = (size_t)(r_upd + kProjWaves * (kProjRed + kProjCols)) * sizeof(double);
    hipLaunchKernelGGL((proj_kernel<T>), dim3(nblk), dim3(64 * kProjWaves), sm, st, X.get(), nd,
                       r_upd, r_dot, v, dc, part.get());
    const int n = r_dot + 2;
    // the column sums, and c += the dot products when accumulating
    reduce_cols(part.get(), nblk, n, n, dvec.get(), acc ? cvec.get() : nullptr, st, acc ? r_dot : 0);
    RTE_CHECK_HIP(hipGetLastError());
  }

  void read_tail(int r_dot, double out[2]) {
    RTE_CHECK_HIP(hipMemcpyAsync(out, dvec.get() + r_dot, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    sync();
  }

  // MGS2-A (Alg. 2) for snapshot v of class cl; returns true if appended.
  bool mgs2a(T* v, int cl) {
    RTE_CHECK_HIP(hipMemsetAsync(cvec.get(), 0, (rcap + 2) * sizeof(double), st));
    double tail[2];
    double x1dot = 0.0, nrm2 = 0.0, orig2 = 0.0;
    if (r == 0) {
      proj(v, 0, nullptr, 0, false);
      read_tail(0, tail);
      nrm2 = tail[0];
      orig2 = tail[1];
    } else {
      // projection 1: dc = X^T v   (also ||v_orig||^2)
      proj(v, 0, nullptr, r, true);
      RTE_CHECK_HIP(hipMemcpyAsync(&orig2, dvec.get() + r + 1, sizeof(double), hipMemcpyDeviceToHost, st));
      // v -= X dc ; projection 2: dc = X^T v  (the update reads a copy of dc)
      copy_dc();
      proj(v, r, dcsave.get(), r, true);
      // v -= X dc ; ||v||^2, X(:,1)^T v
      copy_dc();
      proj(v, r, dcsave.get(), 1, false);
      read_tail(1, tail);
      RTE_CHECK_HIP(hipMemcpyAsync(&x1dot, dvec.get(), sizeof(double), hipMemcpyDeviceToHost, st));
      sync();
      nrm2 = tail[0];
    }
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
        proj(v, 0, nullptr, r, true);
        copy_dc();
        proj(v, r, dcsave.get(), 1, false);
        read_tail(1, tail);
        RTE_CHECK_HIP(hipMemcpyAsync(&x1dot, dvec.get(), sizeof(double), hipMemcpyDeviceToHost, st));
        sync();
        alpha = std::sqrt(tail[0]);
        t = std::fabs(x1dot) / alpha;
      }
      if (t > eps_mgs) ++mgs_failures;
    }
    RTE_REQUIRE(r < rcap, "the basis reached max_rank = %d", rcap);
    hipLaunchKernelGGL((append_kernel<T>), dim3((nd + 255) / 256), dim3(256), 0, st, v,
                       1.0 / alpha, X.get() + (size_t)r * nd, nd);
    hipLaunchKernelGGL(store_coef_kernel, dim3((rcap + 127) / 128), dim3(128), 0, st, cvec.get(), r,
                       alpha, 1, Rst.get() + (size_t)rcap * cl, rcap);
    RTE_CHECK_HIP(hipGetLastError());
    ++r;
    return true;
  }
  DevBuf<double> dcsave;
  void copy_dc() {
    RTE_CHECK_HIP(hipMemcpyAsync(dcsave.get(), dvec.get(), (size_t)r * sizeof(double),
                                 hipMemcpyDeviceToDevice, st));
  }

  // ------------------------------------------------------------ bordering
  void tsdot(const void* A, bool a_double, int na, const void* B, bool b_double, int nb,
             double* out) {
    const int gx = (na + 63) / 64;
    long nch = std::max<long>(1, std::min<long>((nd + 2047) / 2048, std::max(1, 1024 / gx)));
    const long kchunk = ((nd + nch - 1) / nch + 31) / 32 * 32;
    nch = (nd + kchunk - 1) / kchunk;
    DevBuf<double>& buf = tsd;
    RTE_REQUIRE(buf.n >= (size_t)nch * na * nb, "internal: tsdot scratch too small");
    dim3 grid(gx, (unsigned)nch, (unsigned)((nb + 31) / 32));
    if (a_double && b_double)
      hipLaunchKernelGGL((tsdot_kernel<double, double>), grid, dim3(256), 0, st, (const double*)A, na,
                         (const double*)B, nb, nd, kchunk, buf.get());
    else if (!a_double && !b_double)
      hipLaunchKernelGGL((tsdot_kernel<T, T>), grid, dim3(256), 0, st, (const T*)A, na,
                         (const T*)B, nb, nd, kchunk, buf.get());
    else if (a_double)
      hipLaunchKernelGGL((tsdot_kernel<double, T>), grid, dim3(256), 0, st, (const double*)A, na,
                         (const T*)B, nb, nd, kchunk, buf.get());
    else
      hipLaunchKernelGGL((tsdot_kernel<T, double>), grid, dim3(256), 0, st, (const T*)A, na,
                         (const double*)B, nb, nd, kchunk, buf.get());
    const int n = na * nb;
    reduce_cols(buf.get(), (int)nch, n, n, out, nullptr, st);
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
    tsdot(X.get(), sizeof(T) == 8, r1, Y.get(), sizeof(T) == 8, 5 * pn, tsd2.get());
    double* ext = tsd3.get();
    tsdot(E.get(), true, 5, P, sizeof(T) == 8, pn, ext);
    const int nt = std::max(r1 * pn, 5);
    hipLaunchKernelGGL(scatter_border_kernel, dim3((nt + 127) / 128), dim3(128), 0, st, r0, pn,
                       rcap, tsd2.get(), ext, Tm.get(), Dx.get(), Dy.get(), bsrc.get(),
                       bside.get());
    RTE_CHECK_HIP(hipGetLastError());
  }

  // every caller synchronises before the staging buffer is reused
  void upload_list(const std::vector<int>& l) {
    std::memcpy(h_list, l.data(), l.size() * sizeof(int));
    RTE_CHECK_HIP(hipMemcpyAsync(d_list.get(), h_list, l.size() * sizeof(int),
                                 hipMemcpyHostToDevice, st));
  }

  void lu_border(int r0, int pn, const std::vector<int>& classes) {
    if (classes.empty() || pn == 0) return;
    upload_list(classes);
    const size_t sm = ((size_t)2 * pn * r0 + (size_t)kLuRows * r0) * sizeof(double);
    hipLaunchKernelGGL(lu_border_kernel, dim3((unsigned)classes.size()), dim3(64), sm, st, r0, pn,
                       rcap, d_list.get(), d_cd.get(), Tm.get(), Dx.get(), Dy.get(), bsrc.get(),
                       bside.get(), Lt.get(), U.get(), yv.get());
    RTE_CHECK_HIP(hipGetLastError());
    sync();  // the class list is reused by the next call
  }

  void galerkin(const std::vector<int>& classes) {
    if (classes.empty() || r == 0) return;
    upload_list(classes);
    hipLaunchKernelGGL(backsub_kernel, dim3((unsigned)classes.size()), dim3(64),
                       (size_t)rcap * sizeof(double), st, r, rcap, d_list.get(), U.get(), yv.get(),
                       Cg.get());
    RTE_CHECK_HIP(hipGetLastError());
    sync();
  }

  // candidate residual norms (host values in draw order)
  std::vector<double> residuals(const std::vector<int>& cand) {
    const int nm = (int)cand.size();
    std::vector<double> out(nm, 0.0);
    upload_list(cand);
    if (r > 0) {
      hipLaunchKernelGGL(gather_cg_kernel, dim3((r * nm + 255) / 256), dim3(256), 0, st, Cg.get(),
                         rcap, d_list.get(), nm, r, Cm.get());
      hipLaunchKernelGGL((xc_kernel<T, T, 32>), dim3((nd + 255) / 256), dim3(256), 0, st, X.get(), r,
                         nd, Cm.get(), nm, nm, V.get());
    } else {
      RTE_CHECK_HIP(hipMemsetAsync(V.get(), 0, (size_t)nm * nd * sizeof(T), st));
    }
    hipLaunchKernelGGL((residual_kernel<T>), dim3(rblk, nm), dim3(256), 0, st, g.nx, g.ny,
                       1.0 / g.hx, 1.0 / g.hy, prob->sigma_t, src.get(), E.get(), nd, V.get(), nm,
                       d_list.get(), d_cd.get(), rpart.get());
    reduce_cols(rpart.get(), rblk, nm, nm, rsums.get(), nullptr, st);
    RTE_CHECK_HIP(hipGetLastError());
    RTE_CHECK_HIP(hipMemcpyAsync(out.data(), rsums.get(), nm * sizeof(double), hipMemcpyDeviceToHost, st));
    sync();
    for (auto& x : out) x = std::sqrt(x);
    return out;
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
  // On entry src (double) and srcT hold Sigma_s phi_prev + G; phi_old = phi_prev.
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
    while (true) {
      sweep_classes(samples);
      const int r0 = r;
      for (size_t l = 0; l < samples.size(); ++l) {
        mgs2a(psi.get() + (size_t)l * nd, samples[l]);
        sampled[samples[l]] = 1;
        log_sample(samples[l]);
      }
      const int pn = r - r0;
      std::vector<int> uns;
      for (int c = 0; c < K; ++c)
        if (!sampled[c]) uns.push_back(c);
      if (pn > 0) {
        border(r0, pn);
        lu_border(r0, pn, uns);
      }
      if (uns.empty()) {
        scalar_flux(nullptr);
        break;
      }
      std::vector<int> cand = draw(rs, uns, prm->q);
      galerkin(cand);
      std::vector<double> rn = residuals(cand);
      for (double v : rn) log_resid(v);
      double mx = 0.0;
      for (double v : rn) mx = std::max(mx, v);
      bool stop = false;
      if (mx < prm->eps_res) {
        galerkin(uns);
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
      }
    }
    end_replay_outer();
    ms_lr += ms_since(t0) - (ms_sweep - ms_sw0);
  }

  // ------------------------------------------------------------ truncation (Sec. 3.3)
  int truncate(double* Xo, double* So, double* Vo) {
    if (r == 0) return 0;
    DevBuf<double> B((size_t)r * K), Qt((size_t)r * r), sv(r);
    // coefficients of every class (Galerkin for the unsampled ones)
    std::vector<int> uns;
    for (int c = 0; c < K; ++c)
      if (!sampled[c]) uns.push_back(c);
    galerkin(uns);
    scalar_flux(B.get());
    hipLaunchKernelGGL(identity_kernel, dim3((r * r + 255) / 256), dim3(256), 0, st, Qt.get(), r);
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
        hipLaunchKernelGGL(jacobi_round_kernel, dim3(npairs), dim3(64), 0, st, B.get(), K, Qt.get(), r,
                           dpairs.get() + (size_t)rd * npairs * 2, off.get() + (size_t)rd * npairs);
      RTE_CHECK_HIP(hipGetLastError());
      RTE_CHECK_HIP(hipMemcpyAsync(hoff.data(), off.get(), hoff.size() * sizeof(double),
                                   hipMemcpyDeviceToHost, st));
      sync();
      double mx = 0.0;
      for (double v : hoff) mx = std::max(mx, v);
      if (mx <= 1e-15) break;
    }
    hipLaunchKernelGGL(row_norms_kernel, dim3(r), dim3(64), 0, st, B.get(), r, K, sv.get());
    std::vector<double> hs(r);
    RTE_CHECK_HIP(hipMemcpyAsync(hs.data(), sv.get(), r * sizeof(double), hipMemcpyDeviceToHost, st));
    sync();
    std::vector<int> order(r);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hs[a] > hs[b]; });
    std::vector<double> sorted(r);
    for (int i = 0; i < r; ++i) sorted[i] = hs[order[i]];
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
                              double* Vo, rte_solve_result* res, hipStream_t st) {
  const auto t_start = std::chrono::steady_clock::now();
  LowRank<T> lr;
  lr.prob = prob;
  lr.prm = prm;
  lr.st = st;
  lr.res = res;
  lr.setup();
  lr.dcsave.alloc(lr.rcap + 2);
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
    make_source<T>(g, prob->sigma_s, phi_prev.get(), prob->G, lr.srcT.get(), st);
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
    if (conv || n == prm->max_outer) {
      rank = lr.truncate(Xo, So, Vo);
      break;
    }
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
                         hipStream_t st) {
  if (prm->prec == RTE_FP64) return run_lowrank<double>(prob, prm, phi0, phi_out, X, S, V, res, st);
  return run_lowrank<float>(prob, prm, phi0, phi_out, X, S, V, res, st);
}

}  // namespace rte
