// Diffusion synthetic acceleration (paper Sec. 2.2, eqs. (DSA), (diffusion-correction)).
//
// The correction solves, on the transport's DG-Q1 space, the modified interior
// penalty (MIP) form of  -div(D grad dphi) + sigma_a dphi = sigma_s (phi* - phi_prev)
// with D = 1/(3 sigma_t):
//   b(u,v) = sum_K (D grad u, grad v)_K + (sigma_a u, v)_K
//          + sum_interior k_e [[u]][[v]] + {{D d_n u}}[[v]] + [[u]]{{D d_n v}}
//          + sum_boundary k_e u v - 1/2 (D d_n u) v - 1/2 u (D d_n v),
//   k_e = max(1/4, (C/2)(D-/h- + D+/h+)) inside, max(1/4, C D/h) on the boundary, C = 8.
// ([[u]] = u+ - u- with n from the "-" to the "+" cell.)  With the orthonormal tensor
// Legendre basis every face integral factorises: a vertical face couples the
// x-degrees p through a 2x2 matrix and leaves the y-degree q alone (and vice
// versa), with traces l_p(+-1) = (1, +-sqrt3)/sqrt(h) and d/dx l_p = (0, 2 sqrt3/h^1.5).
// The 4x4 blocks are built on the device in closed form (one thread per cell); the SPD
// system is solved by conjugate gradients, all scalars kept on the device and every
// reduction done in a fixed order.  Preconditioner (symmetric two-level, symmetric
// positive definite):
//   z1 = S r,  z2 = z1 + P V P^T (r - A z1),  M^{-1} r = z2 + S (r - A z2),
// S = w B^{-1} with B the 4x4 diagonal blocks and w = 0.7 (B^{-1} A has its spectrum in
// (0, 2), so 2 S^{-1} - A is positive definite), P the embedding of continuous bilinear
// functions (nodal values at the cell corners) in the DG-Q1 space, V one V-cycle of
// geometric multigrid on the Galerkin operator P^T A P (9-point stencils; bilinear
// interpolation, full weighting, Galerkin coarse operators, l1-Jacobi smoothing, exact
// solve on the coarsest grid).  The continuous coarse space carries the smooth error
// that block Jacobi alone removes only in O(1/h) iterations.  Against the additive form
// B^{-1} + P V P^T the CG needs about 40 % fewer iterations for two more block products
// per iteration.
// Layout for the bandwidth-bound CG iteration: the blocks are Kronecker sums (an x-face
// couples only the x-degrees, a y-face only the y-degrees, the volume term is diagonal),
// so a cell's row of A is 14 numbers (the diagonal block's 4 diagonal entries and its two
// off-diagonal couplings, a 2 x 2 x-coupling and a 2 x 2 y-coupling), and these follow in
// closed form from D of the cell and its four neighbours and sigma_a of the cell: the
// matrix products read those two numbers per cell and form the row in registers instead
// of reading stored blocks.  The preconditioner's inverse diagonal blocks and the
// V-cycle's stencils are read in FP32 (built in FP64 and rounded once, so the
// preconditioner stays a fixed symmetric operator, as CG needs; every sum is FP64).
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <tuple>
#include <vector>

#include "common.h"

namespace rte {

static constexpr double kCip = 8.0;
// damping of the block Jacobi smoother in the two-level preconditioner
static constexpr double kSmoothW = 0.7;

// one grid of the multigrid hierarchy on the continuous Q1 space (mx x my nodes)
struct MgLevel {
  int mx = 0, my = 0;
  DevBuf<double> A9;    // [node][9] stencil, entry (dj + 1) 3 + (di + 1)
  DevBuf<float> A9c;    // the same rounded to FP32: the stencils the cycle reads
  DevBuf<double> dinv;  // l1-Jacobi: 1 / (a_ii + sum_{j != i} |a_ij|)
  DevBuf<double> x, b, t;
};

// device view of a level (for the single-workgroup V-cycle of the small grids)
struct MgDev {
  int mx, my;
  const float* A9;
  const double* dinv;
  double *x, *b, *t;
};

struct DSA {
  Geom g;
  DevBuf<double> diag, ax, ay, minv, sig_s;  // [ncell][16] blocks, [ncell]
  DevBuf<double> dcoef, sa;                    // [ncell] D = 1/(3 sigma_t), sigma_a
  DevBuf<float> mc;                            // [10][ncell] upper triangle of B^{-1} (FP32)
  DevBuf<double> r, r2, z, p0, p1, q, b;         // r, r2: the residual, alternating
  DevBuf<double> z1, t;                        // the preconditioner's smoothing passes
  DevBuf<double> part1, part2, part3, part4;   // per-block partial sums
  // The CG solution of the current solve and of the two before (xs[xc], xs[x1], xs[x2]),
  // and the right-hand sides of the two before plus the current one's copy (bs[b1],
  // bs[b2], bs[bsv]); roles rotate after each solve.  nprev: previous solves held (<= 2).
  DevBuf<double> xs[3], bs[3];
  int xc = 0, x1 = 1, x2 = 2, bsv = 0, b1 = 1, b2 = 2, nprev = 0;
  int last_iters = 0;  // CG iterations of the previous solve
  DevBuf<double> scal;                         // device scalars (see Sc below)
  int nblk = 0;                                // blocks of the cell kernels
  int ntile = 0;                               // tiles of the smoothing passes
  std::vector<std::unique_ptr<MgLevel>> mg;    // mg[0]: the nodes of the DG mesh
  DevBuf<double> cinv;                         // dense inverse on the coarsest grid
  int ncoarse = 0;                             // its size (0: smoothing only)
  int lsmall = 0;                              // first level of the one-workgroup V-cycle
  int tile_blocks = 0;                         // levels below this many large-tile blocks
                                               // take the small tiles
  DevBuf<MgDev> mgdev;                         // device views of every level
  std::vector<int> small_off;                  // LDS offsets of the one-workgroup cycle
  size_t small_lds = 0;                        // its LDS bytes (0: it runs on global memory)
};

// layout of the device scalar block
// S_BB = b.b of the current solve; S_B1B1, S_B2B2, S_B1B2 = dot products of the previous two
// right-hand sides b1 (the last), b2; S_BB1, S_BB2 = b.b1, b.b2; S_C1, S_C2 the guess weights
enum Sc {
  S_RHO = 0, S_ALPHA, S_BETA, S_RR, S_TOL2, S_DONE, S_ITERS, S_PQ,
  S_BB, S_B1B1, S_B2B2, S_B1B2, S_BB1, S_BB2, S_C1, S_C2, S_N
};

namespace {

// ------------------------------------------------------------ host assembly
using M4 = double[16];

// Kronecker placement of a 2x2 matrix P acting on the x-degree (k = 2q + p)
__host__ __device__ void put_p(double* B, const double P[2][2], double scale) {
  for (int q = 0; q < 2; ++q)
    for (int p = 0; p < 2; ++p)
      for (int pp = 0; pp < 2; ++pp) B[(2 * q + p) * 4 + (2 * q + pp)] += scale * P[p][pp];
}
// ... acting on the y-degree
__host__ __device__ void put_q(double* B, const double Q[2][2], double scale) {
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 2; ++q)
      for (int qq = 0; qq < 2; ++qq) B[(2 * q + p) * 4 + (2 * qq + p)] += scale * Q[q][qq];
}

// P = k jX jY^T + jX aY^T + aX jY^T
__host__ __device__ void face2(double P[2][2], double k, const double jX[2], const double jY[2], const double aX[2],
           const double aY[2]) {
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) P[i][j] = k * jX[i] * jY[j] + jX[i] * aY[j] + aX[i] * jY[j];
}

__host__ __device__ bool inv4(const double* A, double* out) {
  double m[4][8];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 8; ++j) m[i][j] = j < 4 ? A[4 * i + j] : (j - 4 == i ? 1.0 : 0.0);
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int i = c + 1; i < 4; ++i)
      if (fabs(m[i][c]) > fabs(m[piv][c])) piv = i;
    if (m[piv][c] == 0.0) return false;
    if (piv != c)
      for (int j = 0; j < 8; ++j) {
        const double t = m[c][j];
        m[c][j] = m[piv][j];
        m[piv][j] = t;
      }
    const double iv = 1.0 / m[c][c];
    for (int j = 0; j < 8; ++j) m[c][j] *= iv;
    for (int i = 0; i < 4; ++i)
      if (i != c) {
        const double f = m[i][c];
        for (int j = 0; j < 8; ++j) m[i][j] -= f * m[c][j];
      }
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) out[4 * i + j] = m[i][j + 4];
  return true;
}

// ------------------------------------------------------------ device kernels
__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// Constants of the orthonormal Legendre basis across cells of width h: 1/h, the traces
// l_0 = 1/sqrt(h) and |l_1| = sqrt(3)/sqrt(h) at the faces, the derivative
// l_1' = 2 sqrt(3)/h^1.5, and the volume term 12/h^2 of the degree-1 function.
struct Axis {
  double ih, t0, t1, d1, vol;
};
Axis axis_of(double h) {
  const double r3 = std::sqrt(3.0), sh = std::sqrt(h);
  return Axis{1.0 / h, 1.0 / sh, r3 / sh, 2.0 * r3 / (h * sh), 12.0 / (h * h)};
}

// The 2 x 2 blocks of one interior face between a "-" cell (diffusion Dm) and a "+" cell
// (Dp) in the basis of the direction across the face: Pm adds to the "-" cell's diagonal
// block, Pp to the "+" cell's, C couples the "-" cell's test functions to the "+" cell's
// trial functions (the terms of the assembly in dsa_blocks_kernel).
__device__ __forceinline__ void face_blocks(double Dm, double Dp, const Axis& h, double Pm[2][2],
                                            double Pp[2][2], double C[2][2]) {
  const double eR[2] = {h.t0, h.t1}, eL[2] = {h.t0, -h.t1};
  const double dd[2] = {0.0, h.d1};
  const double kap = fmax(0.25, 0.5 * kCip * (Dm * h.ih + Dp * h.ih));
  double jm[2], am[2], jp[2], ap[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    jm[i] = -eR[i];  // jump and average seen from the "-" cell
    am[i] = 0.5 * Dm * dd[i];
    jp[i] = eL[i];   // ... from the "+" cell
    ap[i] = 0.5 * Dp * dd[i];
  }
  face2(Pm, kap, jm, jm, am, am);
  face2(C, kap, jm, jp, am, ap);
  face2(Pp, kap, jp, jp, ap, ap);
}

// The diagonal-block contribution of a boundary face (the "+" side if hi, else "-")
__device__ __forceinline__ void boundary_block(double D, const Axis& h, bool hi, double P[2][2]) {
  const double e[2] = {h.t0, hi ? h.t1 : -h.t1};
  const double dd[2] = {0.0, h.d1};
  const double kap = fmax(0.25, kCip * D * h.ih);
  double dn[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) dn[i] = (hi ? 1.0 : -1.0) * D * dd[i];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) P[i][j] = kap * e[i] * e[j] - 0.5 * e[i] * dn[j] - 0.5 * dn[i] * e[j];
}

// The diffusion operator as the kernels see it: per-cell D = 1/(3 sigma_t) and
// sigma_a = sigma_t - sigma_s; every block of a cell's row of A is formed from these.
struct OpA {
  int nx, ny;
  Axis x, y;
  const double* __restrict__ D;
  const double* __restrict__ sa;
};

// Cell (a, b)'s row of A in compact form from D of the cell and its four neighbours
// (dn[0..3] = left, right, bottom, top; unused where the neighbour is missing):
// m[0..13] = (B_00, B_11, B_22, B_33, B_01, B_02, X_00, X_01, X_10, X_11, Y_00, Y_01, Y_10,
// Y_11), with B the diagonal block (it couples DOF k = 2 q + p with k ^ 1 through B_01 and
// with k ^ 2 through B_02), X (x) I the coupling to the right neighbour and Y (x) I to the
// top one; xl and yb are the left and bottom neighbours' X and Y (the cell's couplings to
// them are their transposes).  The diagonal entries sum the volume term and the faces
// left, right, bottom, top in that order.
__device__ __forceinline__ void cell_row(const OpA& op, int a, int b, double Dc, const double* dn,
                                         double sa, double* m, double* xl, double* yb) {
  double Pl[2][2], Pr[2][2], Qb[2][2], Qt[2][2], T[2][2], C[2][2];
  double X[2][2] = {{0.0, 0.0}, {0.0, 0.0}}, Y[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  if (a > 0) {
    face_blocks(dn[0], Dc, op.x, T, Pl, C);
    xl[0] = C[0][0], xl[1] = C[0][1], xl[2] = C[1][0], xl[3] = C[1][1];
  } else {
    boundary_block(Dc, op.x, false, Pl);
  }
  if (a + 1 < op.nx) face_blocks(Dc, dn[1], op.x, Pr, T, X);
  else boundary_block(Dc, op.x, true, Pr);
  if (b > 0) {
    face_blocks(dn[2], Dc, op.y, T, Qb, C);
    yb[0] = C[0][0], yb[1] = C[0][1], yb[2] = C[1][0], yb[3] = C[1][1];
  } else {
    boundary_block(Dc, op.y, false, Qb);
  }
  if (b + 1 < op.ny) face_blocks(Dc, dn[3], op.y, Qt, T, Y);
  else boundary_block(Dc, op.y, true, Qt);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int p = k & 1, q = k >> 1;
    double v = sa + Dc * (p ? op.x.vol : 0.0) + Dc * (q ? op.y.vol : 0.0);
    v += Pl[p][p];
    v += Pr[p][p];
    v += Qb[q][q];
    v += Qt[q][q];
    m[k] = v;
  }
  m[4] = Pl[0][1] + Pr[0][1];
  m[5] = Qb[0][1] + Qt[0][1];
  m[6] = X[0][0]; m[7] = X[0][1]; m[8] = X[1][0]; m[9] = X[1][1];
  m[10] = Y[0][0]; m[11] = Y[0][1]; m[12] = Y[1][0]; m[13] = Y[1][1];
}

// acc = (A u)_c for cell c = (a, b) from its row (cell_row); fetch(cell, v) gives u on a
// neighbouring cell.
template <class F>
__device__ __forceinline__ void block_apply(const double* m, const double* xl, const double* yb,
                                            int nx, int ny, long c, int a, int b, const double* u,
                                            F fetch, double* acc) {
  double nb[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = m[k] * u[k] + m[4] * u[k ^ 1] + m[5] * u[k ^ 2];
  if (a + 1 < nx) {  // X (x) I: acc[2q + p] += X[p][.] nb[2q + .]
    fetch(c + 1, nb);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int p = k & 1, qb = k & 2;
      acc[k] += m[6 + 2 * p] * nb[qb] + m[7 + 2 * p] * nb[qb + 1];
    }
  }
  if (a > 0) {  // the left neighbour's X^T
    fetch(c - 1, nb);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int p = k & 1, qb = k & 2;
      acc[k] += xl[p] * nb[qb] + xl[2 + p] * nb[qb + 1];
    }
  }
  if (b + 1 < ny) {  // Y (x) I: acc[2q + p] += Y[q][.] nb[2 . + p]
    fetch(c + nx, nb);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int p = k & 1, qq = k >> 1;
      acc[k] += m[10 + 2 * qq] * nb[p] + m[11 + 2 * qq] * nb[2 + p];
    }
  }
  if (b > 0) {  // the bottom neighbour's Y^T
    fetch(c - nx, nb);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int p = k & 1, qq = k >> 1;
      acc[k] += yb[qq] * nb[p] + yb[2 + qq] * nb[2 + p];
    }
  }
}

// out = B_c^{-1} v from the upper triangle of the symmetric inverse block
// (mc[k][c], row-major 00 01 02 03 11 12 13 22 23 33), stored in FP32: the smoother is
// w B^{-1} rounded once, still a fixed symmetric operator (the sums are FP64)
__device__ __forceinline__ void binv_apply(const float* __restrict__ mc, long ncell, long c,
                                           const double* v, double* out) {
  double m[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) m[k] = (double)mc[(long)k * ncell + c];
  out[0] = m[0] * v[0] + m[1] * v[1] + m[2] * v[2] + m[3] * v[3];
  out[1] = m[1] * v[0] + m[4] * v[1] + m[5] * v[2] + m[6] * v[3];
  out[2] = m[2] * v[0] + m[5] * v[1] + m[7] * v[2] + m[8] * v[3];
  out[3] = m[3] * v[0] + m[6] * v[1] + m[8] * v[2] + m[9] * v[3];
}

// The symmetric inverse diagonal blocks as their upper triangles (one FP32 array per
// entry), and the per-cell D and sigma_a the operator's rows are formed from.
__global__ __launch_bounds__(256) void dsa_compact_kernel(long ncell, const double* __restrict__ minv,
                                                         const double* __restrict__ sigma_t,
                                                         const double* __restrict__ sigma_s,
                                                         float* __restrict__ mc,
                                                         double* __restrict__ D,
                                                         double* __restrict__ sa) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const double* M = minv + 16 * c;
  const double w[10] = {M[0], M[1], M[2], M[3], M[5], M[6], M[7], M[10], M[11], M[15]};
#pragma unroll
  for (int k = 0; k < 10; ++k) mc[(long)k * ncell + c] = (float)w[k];
  D[c] = 1.0 / (3.0 * sigma_t[c]);
  sa[c] = sigma_t[c] - sigma_s[c];
}

// sums nblk partials in a fixed order into sc[slot]
__global__ __launch_bounds__(1024) void reduce_kernel(const double* __restrict__ part, int nblk,
                                                      double* __restrict__ out) {
  __shared__ double red[1024];
  double v = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) v += part[i];
  const double s = block_sum(v, red);
  if (threadIdx.x == 0) *out = s;
}

// reduce_kernel into sc[S_PQ], then alpha = rho / (p.q) (one launch)
__global__ __launch_bounds__(1024) void reduce_alpha_kernel(const double* __restrict__ part, int nblk,
                                                            double* __restrict__ sc) {
  __shared__ double red[1024];
  double v = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) v += part[i];
  const double s = block_sum(v, red);
  if (threadIdx.x == 0) {
    sc[S_PQ] = s;
    if (sc[S_DONE] == 0.0) sc[S_ALPHA] = sc[S_RHO] / s;
  }
}

// the reductions of r.r (part2) into sc[S_RR] and of r.z (part1) into sc[S_PQ], then the
// convergence test and beta (one launch)
__global__ __launch_bounds__(1024) void reduce_beta_kernel(const double* __restrict__ part,
                                                           int n1, const double* __restrict__ part2,
                                                           int n2, double* __restrict__ sc) {
  __shared__ double red[1024];
  double v = 0.0, v2 = 0.0;
  for (int i = threadIdx.x; i < n1; i += blockDim.x) v += part[i];
  for (int i = threadIdx.x; i < n2; i += blockDim.x) v2 += part2[i];
  const double s2 = block_sum(v2, red);
  const double s = block_sum(v, red);
  if (threadIdx.x == 0) {
    sc[S_PQ] = s;
    if (sc[S_DONE] == 0.0) sc[S_RR] = s2;
    if (sc[S_DONE] == 0.0) {
      sc[S_ITERS] += 1.0;
      if (sc[S_RR] <= sc[S_TOL2]) {
        sc[S_DONE] = 1.0;
      } else {
        sc[S_BETA] = s / sc[S_RHO];
        sc[S_RHO] = s;
      }
    }
  }
}

// tol2 = tol^2 |b|^2 (the tolerance is relative to the right-hand side, whatever the
// initial guess), beta = alpha = 0, done when the initial residual already meets it; the
// right-hand side's dot products move down the history for the next solve's guess
__global__ void start_kernel(double* sc, double tol) {
  sc[S_TOL2] = tol * tol * sc[S_BB];
  sc[S_B2B2] = sc[S_B1B1];
  sc[S_B1B2] = sc[S_BB1];
  sc[S_B1B1] = sc[S_BB];
  sc[S_BETA] = 0.0;
  sc[S_ALPHA] = 0.0;
  sc[S_ITERS] = 0.0;
  sc[S_DONE] = (sc[S_RR] <= sc[S_TOL2]) ? 1.0 : 0.0;
}

// The guess weights (c1, c2) minimise |b - c1 b1 - c2 b2| (nprev = 2; the normal equations
// of the 2 x 2 Gram matrix, or the one-term fit c1 = b.b1 / b1.b1 when that matrix is
// nearly singular) or |b - c1 b1| (nprev = 1); b.b1 and b.b2 from per-block partials.
__global__ __launch_bounds__(1024) void guess_weights_kernel(const double* __restrict__ p1,
                                                            const double* __restrict__ p2, int n,
                                                            int nprev, double* __restrict__ sc) {
  __shared__ double red[1024];
  double v1 = 0.0, v2 = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    v1 += p1[i];
    if (nprev > 1) v2 += p2[i];
  }
  const double bb1 = block_sum(v1, red);
  const double bb2 = nprev > 1 ? block_sum(v2, red) : 0.0;
  if (threadIdx.x == 0) {
    sc[S_BB1] = bb1;
    sc[S_BB2] = bb2;
    const double g11 = sc[S_B1B1], g22 = sc[S_B2B2], g12 = sc[S_B1B2];
    double c1 = g11 > 0.0 ? bb1 / g11 : 0.0, c2 = 0.0;
    const double det = g11 * g22 - g12 * g12;
    if (nprev > 1 && det > 1e-10 * g11 * g22) {
      c1 = (bb1 * g22 - bb2 * g12) / det;
      c2 = (bb2 * g11 - bb1 * g12) / det;
    }
    sc[S_C1] = c1;
    sc[S_C2] = c2;
  }
}

// x = c1 x1 + c2 x2 (x2 ignored when nprev = 1)
__global__ void guess_combine_kernel(long n, const double* __restrict__ x1,
                                     const double* __restrict__ x2, int nprev,
                                     double* __restrict__ x, const double* __restrict__ sc) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double c1 = sc[S_C1], c2 = sc[S_C2];
  x[i] = nprev > 1 ? c1 * x1[i] + c2 * x2[i] : c1 * x1[i];
}

// x += alpha p_k, out = a + x: the last iteration's update of x, which the iterations
// leave to the next matrix product (k = the iteration count; iteration k's direction is in
// p1 when k is odd, p0 when even; alpha = 0 and p0 = 0 when no iteration ran).  x keeps
// the solution for the next solve's initial guess.
__global__ void axpy_out_kernel(long n, const double* __restrict__ a, double* __restrict__ x,
                                const double* __restrict__ p0, const double* __restrict__ p1,
                                const double* __restrict__ sc, double* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* p = ((long)sc[S_ITERS] & 1) ? p1 : p0;
  const double xi = x[i] + sc[S_ALPHA] * p[i];
  x[i] = xi;
  out[i] = a[i] + xi;
}

// ------------------------------------------------------------ two-level preconditioner
// Bilinear nodal function -> DG-Q1 coefficients on a cell: coefficient k = 2q + p of the
// nodal basis function of corner (i, j) is ap(p, i) aq(q, j) with
//   ap(0, i) = sqrt(hx)/2,  ap(1, i) = (2i - 1) sqrt(hx) / (2 sqrt3)   (same in y).
struct Emb {
  double x0, x1, y0, y1;  // ap(0,.), |ap(1,.)|, aq(0,.), |aq(1,.)|
  __host__ __device__ double w(int k, int i, int j) const {
    const int p = k & 1, q = k >> 1;
    const double wx = p ? (i ? x1 : -x1) : x0;
    const double wy = q ? (j ? y1 : -y1) : y0;
    return wx * wy;
  }
};

__device__ __forceinline__ double stencil9(const float* __restrict__ A9,
                                           const double* __restrict__ x, int mx, int my, int i,
                                           int j) {
  const float* a = A9 + 9L * ((long)j * mx + i);
  double s = 0.0;
#pragma unroll
  for (int dj = -1; dj <= 1; ++dj) {
    const int jj = j + dj;
    if (jj < 0 || jj >= my) continue;
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
      const int ii = i + di;
      if (ii < 0 || ii >= mx) continue;
      s += (double)a[(dj + 1) * 3 + di + 1] * x[(long)jj * mx + ii];
    }
  }
  return s;
}

// The multi-kernel levels of the cycle run as two kernels per level.  Down: the two
// pre-smoothing sweeps from x = 0, the residual and its full-weighting restriction; up: the
// prolongation with the first post-smoothing sweep, then the second sweep.  Each block owns
// a tile and forms the intermediate vectors on the tile and the rings its later steps need
// (the neighbours' share recomputed, 0 outside the grid, where the stencil's entries are 0
// too) in LDS, so a level costs two launches instead of five.  Every node's value is the
// same sum in the same order as with one kernel per step (stencil rows dj = -1..1, in each
// di = -1..1).

// The phases below run over a thread's entries e = threadIdx.x + 256 k < N of an LDS
// region (256-thread blocks) in two unrolled passes: first every global load of all its
// entries (unconditional, from a node clamped into the grid; entries outside use 0), then
// the arithmetic, so that a phase waits for memory once rather than once per entry.
template <int N>
constexpr int per_thread() { return (N + 255) / 256; }

// a node's stencil row, smoother weight and right-hand side
struct NodeIn {
  float a[9];
  double dinv, b;
};
__device__ __forceinline__ NodeIn load_node(const float* __restrict__ A9,
                                           const double* __restrict__ dinv,
                                           const double* __restrict__ b, long n) {
  NodeIn v;
#pragma unroll
  for (int k = 0; k < 9; ++k) v.a[k] = A9[9 * n + k];
  v.dinv = dinv[n];
  v.b = b[n];
  return v;
}

// sum of the node's stencil times the LDS array v of row width w around entry e
__device__ __forceinline__ double lds_stencil(const float* a, const double* v, int w, int e) {
  double s = 0.0;
#pragma unroll
  for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
    for (int di = -1; di <= 1; ++di) s += (double)a[(dj + 1) * 3 + di + 1] * v[e + dj * w + di];
  return s;
}

// Down, for the coarse nodes [I0, I0 + CX) x [J0, J0 + CY): with y = dinv b,
// x = y + dinv (b - A y) (stored on the fine nodes [2 I0, 2 I0 + 2 CX) x [2 J0, 2 J0 + 2 CY)),
// t = b - A x, and bc = R t.  y lives on the fine nodes 2 I0 - 3 .. 2 I0 + 2 CX + 1 (x one
// node in, t two), so that the restriction of the block's coarse nodes finds t on all
// their fine neighbours.
// The tile is CX x CY coarse nodes: 32 x 8 (fine tile 64 x 16) on the large grids, 8 x 8 on
// the others (kSmallTileBlocks), which then run more, shorter blocks: a block's time is
// mostly the latency of its three dependent load phases, not its arithmetic.
constexpr int kDX = 32, kDY = 8, kDXs = 8, kDYs = 8;
template <int CX, int CY>
__global__ __launch_bounds__(256) void mg_down_kernel(int mx, int my, const float* __restrict__ A9,
                                                     const double* __restrict__ dinv,
                                                     const double* __restrict__ b,
                                                     double* __restrict__ x, int mxc, int myc,
                                                     double* __restrict__ bc,
                                                     const double* __restrict__ sc) {
  constexpr int WY = 2 * CX + 5, HY = 2 * CY + 5, WX = WY - 2, HX = HY - 2, WT = WY - 4,
                HT = HY - 4;
  __shared__ double Y[HY * WY], X[HX * WX], T[HT * WT];
  if (sc[S_DONE] != 0.0) return;
  const int I0 = (int)blockIdx.x * CX, J0 = (int)blockIdx.y * CY;
  const int fi = 2 * I0 - 3, fj = 2 * J0 - 3;  // fine node of Y[0]
  auto inside = [&](int i, int j) { return i >= 0 && i < mx && j >= 0 && j < my; };
  auto node = [&](int i, int j) {  // clamped into the grid
    return (long)min(max(j, 0), my - 1) * mx + min(max(i, 0), mx - 1);
  };
  constexpr int K1 = per_thread<HY * WY>(), K2 = per_thread<HX * WX>(), K3 = per_thread<HT * WT>();
  double dv[K1], bv[K1];
  NodeIn in2[K2], in3[K3];
  auto load2 = [&] {
#pragma unroll
    for (int k = 0; k < K2; ++k) {
      const int e = (int)threadIdx.x + 256 * k;
      in2[k] = load_node(A9, dinv, b, node(fi + 1 + e % WX, fj + 1 + e / WX));
    }
  };
  auto load3 = [&] {
#pragma unroll
    for (int k = 0; k < K3; ++k) {
      const int e = (int)threadIdx.x + 256 * k;
      in3[k] = load_node(A9, dinv, b, node(fi + 2 + e % WT, fj + 2 + e / WT));
    }
  };
#pragma unroll
  for (int k = 0; k < K1; ++k) {
    const int e = (int)threadIdx.x + 256 * k;
    const long n = node(fi + e % WY, fj + e / WY);
    dv[k] = dinv[n];
    bv[k] = b[n];
  }
#pragma unroll
  for (int k = 0; k < K1; ++k) {
    const int e = (int)threadIdx.x + 256 * k;
    if (e < HY * WY) Y[e] = inside(fi + e % WY, fj + e / WY) ? dv[k] * bv[k] : 0.0;
  }
  __syncthreads();
  load2();
#pragma unroll
  for (int k = 0; k < K2; ++k) {
    const int e = (int)threadIdx.x + 256 * k;
    if (e >= HX * WX) continue;
    const int ex = e % WX, ey = e / WX, i = fi + 1 + ex, j = fj + 1 + ey;
    double v = 0.0;
    if (inside(i, j)) {
      const int ey0 = (ey + 1) * WY + ex + 1;
      v = Y[ey0] + in2[k].dinv * (in2[k].b - lds_stencil(in2[k].a, Y, WY, ey0));
      if (i >= 2 * I0 && i < 2 * I0 + 2 * CX && j >= 2 * J0 && j < 2 * J0 + 2 * CY)
        x[(long)j * mx + i] = v;
    }
    X[e] = v;
  }
  __syncthreads();
  load3();
#pragma unroll
  for (int k = 0; k < K3; ++k) {
    const int e = (int)threadIdx.x + 256 * k;
    if (e >= HT * WT) continue;
    const int ex = e % WT, ey = e / WT;
    T[e] = inside(fi + 2 + ex, fj + 2 + ey)
               ? in3[k].b - lds_stencil(in3[k].a, X, WX, (ey + 1) * WX + ex + 1)
               : 0.0;
  }
  __syncthreads();
  // full weighting (transpose of bilinear interpolation): fine node (2I + di, 2J + dj) has
  // weight (1 - |di|/2)(1 - |dj|/2) in coarse node (I, J)
  for (int e = threadIdx.x; e < CX * CY; e += blockDim.x) {
    const int I = I0 + e % CX, J = J0 + e / CX;
    if (I >= mxc || J >= myc) continue;
    double s = 0.0;
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj) {
      const int j = 2 * J + dj;
      if (j < 0 || j >= my) continue;
#pragma unroll
      for (int di = -1; di <= 1; ++di) {
        const int i = 2 * I + di;
        if (i < 0 || i >= mx) continue;
        s += (di ? 0.5 : 1.0) * (dj ? 0.5 : 1.0) * T[(j - fj - 2) * WT + i - fi - 2];
      }
    }
    bc[(long)J * mxc + I] = s;
  }
}

// Up, for the fine nodes [i0, i0 + kUX) x [j0, j0 + kUY): with y = x + P xc (bilinear
// prolongation), t = y + dinv (b - A y), xout = t + dinv (b - A t).  y lives two nodes
// around the tile, t one.
// The tile is UX x UY fine nodes: 64 x 16 on the large grids, 16 x 16 on the small ones.
constexpr int kUX = 64, kUY = 16, kUXs = 16, kUYs = 16;
template <int UX, int UY>
__global__ __launch_bounds__(256) void mg_up_kernel(int mx, int my, const float* __restrict__ A9,
                                                   const double* __restrict__ dinv,
                                                   const double* __restrict__ b,
                                                   const double* __restrict__ x, int mxc,
                                                   const double* __restrict__ xc,
                                                   double* __restrict__ xout,
                                                   const double* __restrict__ sc) {
  constexpr int WY = UX + 4, HY = UY + 4, WT = UX + 2, HT = UY + 2;
  __shared__ double Y[HY * WY], T[HT * WT];
  if (sc[S_DONE] != 0.0) return;
  const int i0 = (int)blockIdx.x * UX, j0 = (int)blockIdx.y * UY;
  const int fi = i0 - 2, fj = j0 - 2;  // fine node of Y[0]
  auto inside = [&](int i, int j) { return i >= 0 && i < mx && j >= 0 && j < my; };
  auto node = [&](int i, int j) {  // clamped into the grid
    return (long)min(max(j, 0), my - 1) * mx + min(max(i, 0), mx - 1);
  };
  const int myc = (my + 1) / 2;
  auto cnode = [&](int I, int J) { return (long)min(J, myc - 1) * mxc + min(I, mxc - 1); };
  constexpr int K1 = per_thread<HY * WY>(), K2 = per_thread<HT * WT>(), K3 = per_thread<UX * UY>();
  double xv[K1], c[K1][4];
  NodeIn in2[K2], in3[K3];
  auto load2 = [&] {
#pragma unroll
    for (int k = 0; k < K2; ++k) {
      const int e = (int)threadIdx.x + 256 * k;
      in2[k] = load_node(A9, dinv, b, node(fi + 1 + e % WT, fj + 1 + e / WT));
    }
  };
  auto load3 = [&] {
#pragma unroll
    for (int k = 0; k < K3; ++k) {
      const int e = (int)threadIdx.x + 256 * k;
      in3[k] = load_node(A9, dinv, b, node(i0 + e % UX, j0 + e / UX));
    }
  };
#pragma unroll
  for (int k = 0; k < K1; ++k) {
    const int e = (int)threadIdx.x + 256 * k;
    const int i = min(max(fi + e % WY, 0), mx - 1), j = min(max(fj + e / WY, 0), my - 1);
    xv[k] = x[node(i, j)];
    const int c0 = i >> 1, c1 = (i + 1) >> 1, r0 = j >> 1, r1 = (j + 1) >> 1;
    c[k][0] = xc[cnode(c0, r0)];
    c[k][1] = xc[cnode(c1, r0)];
    c[k][2] = xc[cnode(c0, r1)];
    c[k][3] = xc[cnode(c1, r1)];
  }
#pragma unroll
  for (int k = 0; k < K1; ++k) {
    const int e = (int)threadIdx.x + 256 * k;
    if (e < HY * WY)
      Y[e] = inside(fi + e % WY, fj + e / WY)
                 ? xv[k] + 0.25 * (c[k][0] + c[k][1] + c[k][2] + c[k][3])
                 : 0.0;
  }
  __syncthreads();
  load2();
#pragma unroll
  for (int k = 0; k < K2; ++k) {
    const int e = (int)threadIdx.x + 256 * k;
    if (e >= HT * WT) continue;
    const int ex = e % WT, ey = e / WT;
    const int ey0 = (ey + 1) * WY + ex + 1;
    T[e] = inside(fi + 1 + ex, fj + 1 + ey)
               ? Y[ey0] + in2[k].dinv * (in2[k].b - lds_stencil(in2[k].a, Y, WY, ey0))
               : 0.0;
  }
  __syncthreads();
  load3();
#pragma unroll
  for (int k = 0; k < K3; ++k) {
    const int e = (int)threadIdx.x + 256 * k;
    const int ex = e % UX, ey = e / UX, i = i0 + ex, j = j0 + ey;
    if (!inside(i, j)) continue;
    const int ey0 = (ey + 1) * WT + ex + 1;
    xout[(long)j * mx + i] = T[ey0] + in3[k].dinv * (in3[k].b - lds_stencil(in3[k].a, T, WT, ey0));
  }
}

// V-cycle of the levels l0 .. nlev-1 by one workgroup (the small grids): the same steps
// as the multi-kernel cycle, separated by workgroup barriers.  Where the levels fit, the
// workgroup first copies their stencils, smoothers and the right-hand side of level l0 into
// LDS (with the coarsest grid's dense inverse if there is room), runs every step on LDS
// and writes only level l0's solution back; otherwise the steps read and write the levels
// in global memory.  Both forms do the same arithmetic in the same order.
constexpr int kSmallThreads = 1024;
constexpr long kSmallNodes = 1100;  // grids this small run inside the one workgroup
constexpr int kMaxSmallLevels = 8;
constexpr int kCoarseDense = 100;   // largest grid solved by its dense inverse
constexpr int kCoarseSweeps = 20;   // l1-Jacobi sweeps on a coarsest grid that is larger

// LDS byte offsets of one level's arrays (-1: not held; the dense coarsest grid needs only
// b and x)
struct SmallLevel {
  int mx, my, oA, od, ob, ox, ot;
};
struct SmallPlan {
  int nl;     // levels l0 .. l0 + nl - 1
  int ocinv;  // dense inverse in LDS at this offset, or -1
  SmallLevel lv[kMaxSmallLevels];
};

__device__ __forceinline__ void sm_jacobi(const MgDev& L, const double* x, double* out) {
  const long n = (long)L.mx * L.my;
  for (long k = threadIdx.x; k < n; k += blockDim.x) {
    const int i = (int)(k % L.mx), j = (int)(k / L.mx);
    out[k] = x ? x[k] + L.dinv[k] * (L.b[k] - stencil9(L.A9, x, L.mx, L.my, i, j))
               : L.dinv[k] * L.b[k];
  }
  __syncthreads();
}

// n elements of 4 bytes (float) or 8 (double) into LDS, 16 bytes per load where aligned
template <class T>
__device__ __forceinline__ void copy_to_lds(T* __restrict__ dst, const T* __restrict__ src, long n) {
  constexpr int kv = 16 / sizeof(T);
  const long nv = ((reinterpret_cast<uintptr_t>(src) & 15) == 0) ? n / kv : 0;
  const float4* s4 = reinterpret_cast<const float4*>(src);
  float4* d4 = reinterpret_cast<float4*>(dst);
#pragma unroll 4
  for (long k = threadIdx.x; k < nv; k += blockDim.x) d4[k] = s4[k];
  for (long k = nv * kv + threadIdx.x; k < n; k += blockDim.x) dst[k] = src[k];
}

// red[8 i + u] = sum over j = u (mod 8) of the whole blocks of eight of ci[j][i] b[j], the
// tail j >= 8 floor(nc / 8) added to u = 0 (the dense inverse is symmetric: column i is
// read as row i)
__device__ __forceinline__ void coarse_terms(const double* __restrict__ ci,
                                             const double* __restrict__ b, int nc,
                                             double* __restrict__ red) {
  const int nb8 = nc / 8 * 8;
  for (int e = threadIdx.x; e < 8 * nc; e += blockDim.x) {
    const int i = e >> 3, u = e & 7;
    double s = 0.0;
    for (int j = u; j < nb8; j += 8) s += ci[(long)j * nc + i] * b[j];
    if (u == 0)
      for (int j = nb8; j < nc; ++j) s += ci[(long)j * nc + i] * b[j];
    red[e] = s;
  }
}

template <bool kLds>
__global__ __launch_bounds__(kSmallThreads) void mg_small_kernel(const MgDev* __restrict__ lv,
                                                                 int l0, int nlev,
                                                                 const double* __restrict__ cinv,
                                                                 int nc, int coarse_sweeps,
                                                                 SmallPlan plan,
                                                                 const double* __restrict__ sc) {
  extern __shared__ __align__(16) unsigned char sm_small[];
  __shared__ double red[8 * kCoarseDense];
  if (sc[S_DONE] != 0.0) return;
  // the view of level l the steps work on
  auto level = [&](int l) {
    MgDev v = lv[l];
    if constexpr (kLds) {
      const SmallLevel& P = plan.lv[l - l0];
      v.A9 = P.oA >= 0 ? reinterpret_cast<const float*>(sm_small + P.oA) : nullptr;
      v.dinv = P.od >= 0 ? reinterpret_cast<const double*>(sm_small + P.od) : nullptr;
      v.b = reinterpret_cast<double*>(sm_small + P.ob);
      v.x = reinterpret_cast<double*>(sm_small + P.ox);
      v.t = P.ot >= 0 ? reinterpret_cast<double*>(sm_small + P.ot) : nullptr;
    }
    return v;
  };
  if constexpr (kLds) {
    for (int l = l0; l < nlev; ++l) {
      const MgDev G = lv[l];
      const SmallLevel& P = plan.lv[l - l0];
      const long n = (long)G.mx * G.my;
      if (P.oA >= 0) copy_to_lds(reinterpret_cast<float*>(sm_small + P.oA), G.A9, 9 * n);
      if (P.od >= 0) copy_to_lds(reinterpret_cast<double*>(sm_small + P.od), G.dinv, n);
      if (l == l0) copy_to_lds(reinterpret_cast<double*>(sm_small + P.ob), G.b, n);
    }
    if (plan.ocinv >= 0)
      copy_to_lds(reinterpret_cast<double*>(sm_small + plan.ocinv), cinv, (long)nc * nc);
    __syncthreads();
  }
  // down: pre-smoothing, residual, restriction
  for (int l = l0; l + 1 < nlev; ++l) {
    const MgDev L = level(l), C = level(l + 1);
    sm_jacobi(L, nullptr, L.t);
    sm_jacobi(L, L.t, L.x);
    const long n = (long)L.mx * L.my;
    for (long k = threadIdx.x; k < n; k += blockDim.x) {
      const int i = (int)(k % L.mx), j = (int)(k / L.mx);
      L.t[k] = L.b[k] - stencil9(L.A9, L.x, L.mx, L.my, i, j);
    }
    __syncthreads();
    const long nc2 = (long)C.mx * C.my;
    for (long k = threadIdx.x; k < nc2; k += blockDim.x) {
      const int I = (int)(k % C.mx), J = (int)(k / C.mx);
      double s = 0.0;
      for (int dj = -1; dj <= 1; ++dj) {
        const int j = 2 * J + dj;
        if (j < 0 || j >= L.my) continue;
        for (int di = -1; di <= 1; ++di) {
          const int i = 2 * I + di;
          if (i < 0 || i >= L.mx) continue;
          s += (di ? 0.5 : 1.0) * (dj ? 0.5 : 1.0) * L.t[(long)j * L.mx + i];
        }
      }
      C.b[k] = s;
    }
    __syncthreads();
  }
  // coarsest grid: x = A^{-1} b by the dense inverse (eight lanes per node, then the eight
  // sums paired), or l1-Jacobi sweeps
  {
    const MgDev C = level(nlev - 1);
    if (nc > 0) {
      if (kLds && plan.ocinv >= 0)
        coarse_terms(reinterpret_cast<const double*>(sm_small + plan.ocinv), C.b, nc, red);
      else
        coarse_terms(cinv, C.b, nc, red);
      __syncthreads();
      for (int i = threadIdx.x; i < nc; i += blockDim.x) {
        const double* s = red + 8 * i;
        C.x[i] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
      }
      __syncthreads();
    } else {
      sm_jacobi(C, nullptr, C.t);
      for (int s = 1; s < coarse_sweeps; s += 2) {
        sm_jacobi(C, C.t, C.x);
        if (s + 1 < coarse_sweeps) sm_jacobi(C, C.x, C.t);
      }
    }
  }
  // up: prolongation, post-smoothing
  for (int l = nlev - 2; l >= l0; --l) {
    const MgDev L = level(l), C = level(l + 1);
    const long n = (long)L.mx * L.my;
    for (long k = threadIdx.x; k < n; k += blockDim.x) {
      const int i = (int)(k % L.mx), j = (int)(k / L.mx);
      const int i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1;
      L.x[k] += 0.25 * (C.x[(long)j0 * C.mx + i0] + C.x[(long)j0 * C.mx + i1] +
                        C.x[(long)j1 * C.mx + i0] + C.x[(long)j1 * C.mx + i1]);
    }
    __syncthreads();
    sm_jacobi(L, L.x, L.t);
    sm_jacobi(L, L.t, L.x);
  }
  if constexpr (kLds) {  // level l0's solution for the next finer level's prolongation
    const MgDev L = level(l0), G = lv[l0];
    const long n = (long)L.mx * L.my;
    for (long k = threadIdx.x; k < n; k += blockDim.x) G.x[k] = L.x[k];
  }
}

// b0 = P^T r at node (i, j): the corner (i - a, j - b) of each adjacent cell (a, b), the
// cells' rows in increasing order, then their columns; tval(a, b, k) is r's entry k in cell
// (a, b).  Every caller sums in this one order.
template <class F>
__device__ __forceinline__ double node_restrict(const Emb& em, int nx, int ny, int i, int j,
                                                F tval) {
  double s = 0.0;
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int b = j - 1 + cb;
    if (b < 0 || b >= ny) continue;
#pragma unroll
    for (int ca = 0; ca < 2; ++ca) {
      const int a = i - 1 + ca;
      if (a < 0 || a >= nx) continue;
#pragma unroll
      for (int k = 0; k < 4; ++k) s += em.w(k, i - a, j - b) * tval(a, b, k);
    }
  }
  return s;
}

// The preconditioner's two smoothing passes (symmetric two-level, damped block Jacobi
// S = w B^{-1} before and after the coarse correction; see precondition).  Both work on
// tiles of kCX x kCY cells, one cell per thread: the vector the block product needs is
// formed once per cell of the tile and its ring in LDS (zero outside the grid), so the
// neighbours' blocks are not recomputed per cell.  The partial dot products are per tile.
constexpr int kCX = 64, kCY = 8, kCW = kCX + 2, kCH = kCY + 2;

dim3 cell_tiles(int nx, int ny) {
  return dim3((unsigned)((nx + kCX - 1) / kCX), (unsigned)((ny + kCY - 1) / kCY));
}

// fills tile[(kCH)(kCW)][4] with f(cell, out) and dtile[(kCH)(kCW)] with D on the block's
// cells and their ring
template <class F>
__device__ __forceinline__ void fill_cell_tile(double* tile, double* dtile, const double* D,
                                               int nx, int ny, F f) {
  const int a0 = (int)blockIdx.x * kCX - 1, b0 = (int)blockIdx.y * kCY - 1;
  for (int e = threadIdx.x; e < kCW * kCH; e += blockDim.x) {
    const int a = a0 + e % kCW, b = b0 + e / kCW;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    double dv = 0.0;
    if (a >= 0 && a < nx && b >= 0 && b < ny) {
      f((long)b * nx + a, v);
      dv = D[(long)b * nx + a];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) tile[4 * e + k] = v[k];
    dtile[e] = dv;
  }
  __syncthreads();
}

// (A u)_c of tile cell e0 (cell c = (a, b)) from the tile of u and of D
__device__ __forceinline__ void tile_apply(const OpA& op, const double* tile, const double* dtile,
                                           int e0, long c, int a, int b, double* u, double* acc) {
  auto fetch = [&](long c2, double* o) {  // the tile entry of a neighbour of c
    const long d = c2 - c;
    const int e = d == op.nx ? e0 + kCW : d == -op.nx ? e0 - kCW : d == 1 ? e0 + 1 : e0 - 1;
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = tile[4 * e + k];
  };
  const double dn[4] = {dtile[e0 - 1], dtile[e0 + 1], dtile[e0 - kCW], dtile[e0 + kCW]};
  double m[14], xl[4], yb[4];
  cell_row(op, a, b, dtile[e0], dn, op.sa[c], m, xl, yb);
#pragma unroll
  for (int k = 0; k < 4; ++k) u[k] = tile[4 * e0 + k];
  block_apply(m, xl, yb, op.nx, op.ny, c, a, b, u, fetch, acc);
}

// The conjugate-gradient product on the same tiles: p_new = z + beta p_old (formed on the
// tile and its ring), q = A p_new, part = p_new.q per tile; also the previous iteration's
// x += alpha p_old (alpha still holds that iteration's step: this launch precedes the new
// step's reduction; alpha = 0 and p_old = 0 before the first).
__global__ __launch_bounds__(kCX * kCY) void spmv_kernel(OpA op, const double* __restrict__ z,
                                                        const double* __restrict__ pold,
                                                        double* __restrict__ pnew,
                                                        double* __restrict__ q,
                                                        double* __restrict__ x,
                                                        double* __restrict__ part,
                                                        const double* __restrict__ sc) {
  __shared__ double tile[4 * kCW * kCH];
  __shared__ double dtile[kCW * kCH];
  __shared__ double red[kCX * kCY];
  if (sc[S_DONE] != 0.0) return;
  const double beta = sc[S_BETA], alpha = sc[S_ALPHA];
  const int nx = op.nx, ny = op.ny;
  fill_cell_tile(tile, dtile, op.D, nx, ny, [&](long c2, double* o) {
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = z[4 * c2 + k] + beta * pold[4 * c2 + k];
  });
  const int lx = (int)threadIdx.x % kCX, ly = (int)threadIdx.x / kCX;
  const int a = (int)blockIdx.x * kCX + lx, b = (int)blockIdx.y * kCY + ly;
  double dot = 0.0;
  if (a < nx && b < ny) {
    const long c = (long)b * nx + a;
    double u[4], acc[4];
    tile_apply(op, tile, dtile, (ly + 1) * kCW + lx + 1, c, a, b, u, acc);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      x[4 * c + k] += alpha * pold[4 * c + k];
      pnew[4 * c + k] = u[k];
      q[4 * c + k] = acc[k];
      dot += u[k] * acc[k];
    }
  }
  const double s = block_sum(dot, red);
  if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// The initial residual of a guess x: r = b - A x (r holds b on entry; each block reads and
// writes only its own cells of r), bprev = b (saved for the next solve's guess), part2 =
// r.r per tile.
__global__ __launch_bounds__(kCX * kCY) void guess_residual_kernel(OpA op,
                                                                  const double* __restrict__ x,
                                                                  double* __restrict__ r,
                                                                  double* __restrict__ bprev,
                                                                  double* __restrict__ part2) {
  __shared__ double tile[4 * kCW * kCH];
  __shared__ double dtile[kCW * kCH];
  __shared__ double red[kCX * kCY];
  const int nx = op.nx, ny = op.ny;
  fill_cell_tile(tile, dtile, op.D, nx, ny, [&](long c2, double* o) {
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = x[4 * c2 + k];
  });
  const int lx = (int)threadIdx.x % kCX, ly = (int)threadIdx.x / kCX;
  const int a = (int)blockIdx.x * kCX + lx, b = (int)blockIdx.y * kCY + ly;
  double rr = 0.0;
  if (a < nx && b < ny) {
    const long c = (long)b * nx + a;
    double u[4], acc[4];
    tile_apply(op, tile, dtile, (ly + 1) * kCW + lx + 1, c, a, b, u, acc);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double bk = r[4 * c + k];
      const double rk = bk - acc[k];
      bprev[4 * c + k] = bk;
      r[4 * c + k] = rk;
      rr += rk * rk;
    }
  }
  const double s = block_sum(rr, red);
  if (threadIdx.x == 0) part2[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// First: z1 = S r, t = r - A z1.  With kUpd, r is first updated from the conjugate-
// gradient step: r = rin - alpha q (formed on the tile and its ring, stored to rout on the
// tile: rin stays intact for the neighbouring tiles' rings), part2 = r.r per tile.
template <bool kUpd>
__global__ __launch_bounds__(kCX * kCY) void dg_smooth1_kernel(OpA op,
                                                              const float* __restrict__ mc,
                                                              const double* __restrict__ rin,
                                                              const double* __restrict__ q,
                                                              double* __restrict__ rout, double w,
                                                              double* __restrict__ z1,
                                                              Emb em, double* __restrict__ t,
                                                              double* __restrict__ b0,
                                                              double* __restrict__ part2,
                                                              const double* __restrict__ sc) {
  __shared__ double tile[4 * kCW * kCH];
  __shared__ double dtile[kCW * kCH];
  __shared__ double red[kCX * kCY];
  if (sc[S_DONE] != 0.0) return;
  const double alpha = kUpd ? sc[S_ALPHA] : 0.0;
  const int nx = op.nx, ny = op.ny;
  const long ncell = (long)nx * ny;
  auto rv = [&](long c2, double* v) {
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = kUpd ? rin[4 * c2 + k] - alpha * q[4 * c2 + k] : rin[4 * c2 + k];
  };
  fill_cell_tile(tile, dtile, op.D, nx, ny, [&](long c2, double* o) {
    double v[4];
    rv(c2, v);
    binv_apply(mc, ncell, c2, v, o);
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] *= w;
  });
  const int lx = (int)threadIdx.x % kCX, ly = (int)threadIdx.x / kCX;
  const int a = (int)blockIdx.x * kCX + lx, b = (int)blockIdx.y * kCY + ly;
  double rr = 0.0, tv[4];
  const bool in = a < nx && b < ny;
  if (in) {
    const long c = (long)b * nx + a;
    double u[4], acc[4], r[4];
    tile_apply(op, tile, dtile, (ly + 1) * kCW + lx + 1, c, a, b, u, acc);
    rv(c, r);
    const bool edge = lx == 0 || lx == kCX - 1 || ly == 0 || ly == kCY - 1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (kUpd) rout[4 * c + k] = r[k];
      rr += r[k] * r[k];
      z1[4 * c + k] = u[k];
      tv[k] = r[k] - acc[k];
      if (edge) t[4 * c + k] = tv[k];
    }
  }
  // b0 = P^T t on the nodes whose cells all lie in this tile, from t in LDS (the tile's
  // array is free once every thread has applied the block product)
  __syncthreads();
  if (in) {
#pragma unroll
    for (int k = 0; k < 4; ++k) tile[4 * (ly * kCX + lx) + k] = tv[k];
  }
  __syncthreads();
  {
    const int a0 = (int)blockIdx.x * kCX, c0 = (int)blockIdx.y * kCY;
    const int aend = min(a0 + kCX, nx), cend = min(c0 + kCY, ny);
    const int ilo = a0 == 0 ? 0 : a0 + 1, ihi = aend == nx ? nx : aend - 1;
    const int jlo = c0 == 0 ? 0 : c0 + 1, jhi = cend == ny ? ny : cend - 1;
    const int wn = ihi - ilo + 1, hn = jhi - jlo + 1;
    for (int e = (int)threadIdx.x; e < wn * hn; e += kCX * kCY) {
      const int i = ilo + e % wn, j = jlo + e / wn;
      b0[(long)j * (nx + 1) + i] = node_restrict(em, nx, ny, i, j, [&](int ca, int cb, int k) {
        return tile[4 * ((cb - c0) * kCX + ca - a0) + k];
      });
    }
  }
  if (kUpd) {
    const double s = block_sum(rr, red);
    if (threadIdx.x == 0) part2[blockIdx.y * gridDim.x + blockIdx.x] = s;
  }
}

// b0 on the nodes that cell tiles share (node columns i = kCX m and rows j = kCY m strictly
// inside the grid): dg_smooth1_kernel restricts every other node from its tile in LDS and
// stores t on its edge cells for this kernel.  Nodes on the shared rows come first (nrow of
// them), then those on the shared columns that are not on a shared row.
__global__ __launch_bounds__(256) void dg_restrict_edges_kernel(int nx, int ny, Emb em,
                                                               const double* __restrict__ t,
                                                               double* __restrict__ b0,
                                                               const double* __restrict__ sc) {
  if (sc[S_DONE] != 0.0) return;
  const int mx = nx + 1;
  const int nxe = (nx - 1) / kCX, nye = (ny - 1) / kCY;  // shared columns, shared rows
  const long nrow = (long)nye * mx;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j;
  if (e < nrow) {
    j = kCY * (int)(e / mx + 1);
    i = (int)(e % mx);
  } else {
    const long f = e - nrow;
    if (f >= (long)nxe * (ny + 1)) return;
    i = kCX * (int)(f / (ny + 1) + 1);
    j = (int)(f % (ny + 1));
    if (j > 0 && j < ny && j % kCY == 0) return;  // on a shared row
  }
  b0[(long)j * mx + i] = node_restrict(em, nx, ny, i, j, [&](int a, int b, int k) {
    return t[4 * ((long)b * nx + a) + k];
  });
}

// number of nodes dg_restrict_edges_kernel handles (one thread each)
long restrict_edge_threads(int nx, int ny) {
  return (long)((ny - 1) / kCY) * (nx + 1) + (long)((nx - 1) / kCX) * (ny + 1);
}

// Second: z2 = z1 + P x0 (the prolonged coarse correction), z = z2 + S (r - A z2);
// part1 = r.z per tile.
__global__ __launch_bounds__(kCX * kCY) void dg_smooth2_kernel(OpA op, Emb em,
                                                              const float* __restrict__ mc,
                                                              const double* __restrict__ r,
                                                              const double* __restrict__ z1,
                                                              const double* __restrict__ x0, double w,
                                                              double* __restrict__ z,
                                                              double* __restrict__ part1,
                                                              const double* __restrict__ sc) {
  __shared__ double tile[4 * kCW * kCH];
  __shared__ double dtile[kCW * kCH];
  __shared__ double red[kCX * kCY];
  if (sc[S_DONE] != 0.0) return;
  const int nx = op.nx, ny = op.ny;
  const long ncell = (long)nx * ny;
  const int mx = nx + 1;
  fill_cell_tile(tile, dtile, op.D, nx, ny, [&](long c2, double* o) {
    const int a2 = (int)(c2 % nx), b2 = (int)(c2 / nx);
    double u[4];
#pragma unroll
    for (int cj = 0; cj < 2; ++cj)
#pragma unroll
      for (int ci = 0; ci < 2; ++ci) u[2 * cj + ci] = x0[(long)(b2 + cj) * mx + a2 + ci];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double v = z1[4 * c2 + k];
#pragma unroll
      for (int m = 0; m < 4; ++m) v += em.w(k, m & 1, m >> 1) * u[m];
      o[k] = v;
    }
  });
  const int lx = (int)threadIdx.x % kCX, ly = (int)threadIdx.x / kCX;
  const int a = (int)blockIdx.x * kCX + lx, b = (int)blockIdx.y * kCY + ly;
  double rz = 0.0;
  if (a < nx && b < ny) {
    const long c = (long)b * nx + a;
    double u[4], acc[4], tv[4], st[4];
    tile_apply(op, tile, dtile, (ly + 1) * kCW + lx + 1, c, a, b, u, acc);
#pragma unroll
    for (int k = 0; k < 4; ++k) tv[k] = r[4 * c + k] - acc[k];
    binv_apply(mc, ncell, c, tv, st);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double zk = u[k] + w * st[k];
      z[4 * c + k] = zk;
      rz += r[4 * c + k] * zk;
    }
  }
  const double s = block_sum(rz, red);
  if (threadIdx.x == 0) part1[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// r = b = sigma_s (phi* - phi_prev); p_old = 0; part2 = b.b.  Without a previous solve
// (kPrev false): x = 0 and bsave = b.  With one: part3 = b.b1 and, when there are two,
// part4 = b.b2 (the guess is then formed and its residual by guess_residual_kernel, which
// also stores bsave = b).  One degree of freedom per thread, so that every load and store
// is one contiguous run per wavefront; a block of kInitThreads covers kInitThreads / 4
// cells, one partial sum each.
constexpr int kInitThreads = 1024;
template <bool kPrev>
__global__ __launch_bounds__(kInitThreads) void init_r_kernel(
    long ncell, const double* __restrict__ sig_s, const double* __restrict__ phis,
    const double* __restrict__ phip, double* __restrict__ x, double* __restrict__ r,
    double* __restrict__ pold, double* __restrict__ bsave, const double* __restrict__ b1,
    const double* __restrict__ b2, double* __restrict__ part2, double* __restrict__ part3,
    double* __restrict__ part4) {
  __shared__ double red[kInitThreads];
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double rr = 0.0, r1 = 0.0, r2 = 0.0;
  if (i < 4 * ncell) {
    const double rv = sig_s[i >> 2] * (phis[i] - phip[i]);
    r[i] = rv;
    pold[i] = 0.0;
    rr = rv * rv;
    if (kPrev) {
      r1 = rv * b1[i];
      if (b2) r2 = rv * b2[i];
    } else {
      x[i] = 0.0;
      bsave[i] = rv;
    }
  }
  const double s = block_sum(rr, red);
  if (threadIdx.x == 0) part2[blockIdx.x] = s;
  if (kPrev) {
    const double t1 = block_sum(r1, red);
    if (threadIdx.x == 0) part3[blockIdx.x] = t1;
    if (b2) {
      const double t2 = block_sum(r2, red);
      if (threadIdx.x == 0) part4[blockIdx.x] = t2;
    }
  }
}

// clears the done flag before the first application of the preconditioner
__global__ void clear_done_kernel(double* sc) { sc[S_DONE] = 0.0; }

// One thread per cell: the diagonal block, the couplings to the right and top neighbours
// (zero on the boundary) and the inverse diagonal block, in closed form.  bad[0] = 1 if
// a diagonal block is singular.
__global__ __launch_bounds__(256) void dsa_blocks_kernel(int nx, int ny, double hx, double hy,
                                                        const double* __restrict__ sigma_t,
                                                        const double* __restrict__ sigma_s,
                                                        double* __restrict__ diag,
                                                        double* __restrict__ ax,
                                                        double* __restrict__ ay,
                                                        double* __restrict__ minv,
                                                        int* __restrict__ bad) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (long)nx * ny) return;
  const int a = (int)(c % nx), b = (int)(c / nx);
  const double r3 = sqrt(3.0);
  const double eRx[2] = {1 / sqrt(hx), r3 / sqrt(hx)};
  const double eLx[2] = {1 / sqrt(hx), -r3 / sqrt(hx)};
  const double dx[2] = {0.0, 2.0 * r3 / (hx * sqrt(hx))};
  const double eRy[2] = {1 / sqrt(hy), r3 / sqrt(hy)};
  const double eLy[2] = {1 / sqrt(hy), -r3 / sqrt(hy)};
  const double dy[2] = {0.0, 2.0 * r3 / (hy * sqrt(hy))};
  auto Dc = [&](long cc) { return 1.0 / (3.0 * sigma_t[cc]); };
  double B[16], AX[16], AY[16];
  for (int k = 0; k < 16; ++k) B[k] = AX[k] = AY[k] = 0.0;
  const double D = Dc(c), sa = sigma_t[c] - sigma_s[c];
  // volume: D (12/hx^2 on p = 1, 12/hy^2 on q = 1) + sigma_a I
  for (int k = 0; k < 4; ++k) {
    const int p = k & 1, q = k >> 1;
    B[5 * k] += sa + D * (p ? 12.0 / (hx * hx) : 0.0) + D * (q ? 12.0 / (hy * hy) : 0.0);
  }
  double P[2][2];
  // x faces: this cell is "-" of its right face and "+" of its left face
  for (int side = 0; side < 2; ++side) {
    const bool right = side == 1;
    const int an = right ? a + 1 : a - 1;
    const double* e = right ? eRx : eLx;
    if (an >= 0 && an < nx) {
      const long cn = (long)b * nx + an;
      const double Dn = Dc(cn);
      const double kap = fmax(0.25, 0.5 * kCip * (D / hx + Dn / hx));
      // jump and average seen from this cell
      double j[2], av[2];
      for (int i = 0; i < 2; ++i) {
        j[i] = right ? -e[i] : e[i];
        av[i] = 0.5 * D * dx[i];
      }
      face2(P, kap, j, j, av, av);
      put_p(B, P, 1.0);
      if (right) {  // coupling (test here, trial in the right neighbour)
        double jn[2], an2[2];
        for (int i = 0; i < 2; ++i) {
          jn[i] = eLx[i];
          an2[i] = 0.5 * Dn * dx[i];
        }
        face2(P, kap, j, jn, av, an2);
        put_p(AX, P, 1.0);
      }
    } else {
      const double kap = fmax(0.25, kCip * D / hx);
      double dn[2];
      for (int i = 0; i < 2; ++i) dn[i] = (right ? 1.0 : -1.0) * D * dx[i];
      for (int i = 0; i < 2; ++i)
        for (int jj = 0; jj < 2; ++jj)
          P[i][jj] = kap * e[i] * e[jj] - 0.5 * e[i] * dn[jj] - 0.5 * dn[i] * e[jj];
      put_p(B, P, 1.0);
    }
  }
  // y faces
  for (int side = 0; side < 2; ++side) {
    const bool top = side == 1;
    const int bn = top ? b + 1 : b - 1;
    const double* e = top ? eRy : eLy;
    if (bn >= 0 && bn < ny) {
      const long cn = (long)bn * nx + a;
      const double Dn = Dc(cn);
      const double kap = fmax(0.25, 0.5 * kCip * (D / hy + Dn / hy));
      double j[2], av[2];
      for (int i = 0; i < 2; ++i) {
        j[i] = top ? -e[i] : e[i];
        av[i] = 0.5 * D * dy[i];
      }
      face2(P, kap, j, j, av, av);
      put_q(B, P, 1.0);
      if (top) {
        double jn[2], an2[2];
        for (int i = 0; i < 2; ++i) {
          jn[i] = eLy[i];
          an2[i] = 0.5 * Dn * dy[i];
        }
        face2(P, kap, j, jn, av, an2);
        put_q(AY, P, 1.0);
      }
    } else {
      const double kap = fmax(0.25, kCip * D / hy);
      double dn[2];
      for (int i = 0; i < 2; ++i) dn[i] = (top ? 1.0 : -1.0) * D * dy[i];
      for (int i = 0; i < 2; ++i)
        for (int jj = 0; jj < 2; ++jj)
          P[i][jj] = kap * e[i] * e[jj] - 0.5 * e[i] * dn[jj] - 0.5 * dn[i] * e[jj];
      put_q(B, P, 1.0);
    }
  }
  double Mi[16];
  if (!inv4(B, Mi)) atomicOr(bad, 1);
  for (int k = 0; k < 16; ++k) {
    diag[16 * c + k] = B[k];
    ax[16 * c + k] = AX[k];
    ay[16 * c + k] = AY[k];
    minv[16 * c + k] = Mi[k];
  }
}

// Row of P^T A P at node (i, j) of the (nx + 1) x (ny + 1) nodal grid: the blocks whose
// test cell has the node as a corner (the diagonal blocks of the up to four cells around
// it and their couplings to the left / right / lower / upper neighbours), each projected
// on the bilinear corner functions.  Couplings of nodes two apart vanish for continuous
// functions and are not stored.  Fixed summation order.
__global__ __launch_bounds__(256) void mg_fine_kernel(int nx, int ny, Emb em,
                                                     const double* __restrict__ diag,
                                                     const double* __restrict__ ax,
                                                     const double* __restrict__ ay,
                                                     double* __restrict__ A9) {
  const int mx = nx + 1, my = ny + 1;
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= (long)mx * my) return;
  const int i = (int)(n % mx), j = (int)(n / mx);
  double row[9];
  for (int k = 0; k < 9; ++k) row[k] = 0.0;
  // block B (or B^T) between test cell (a, b), corner (mi, mj) = node, and trial cell (a2, b2)
  auto add = [&](const double* B, bool tr, int mi, int mj, int a2, int b2) {
    for (int mm = 0; mm < 4; ++mm) {
      const int di = a2 + (mm & 1) - i, dj = b2 + (mm >> 1) - j;
      if (di < -1 || di > 1 || dj < -1 || dj > 1) continue;
      double v = 0.0;
      for (int k = 0; k < 4; ++k) {
        const double wk = em.w(k, mi, mj);
        for (int kk = 0; kk < 4; ++kk)
          v += wk * (tr ? B[4 * kk + k] : B[4 * k + kk]) * em.w(kk, mm & 1, mm >> 1);
      }
      row[(dj + 1) * 3 + di + 1] += v;
    }
  };
  for (int cb = 0; cb < 2; ++cb) {
    const int b = j - 1 + cb;
    if (b < 0 || b >= ny) continue;
    for (int ca = 0; ca < 2; ++ca) {
      const int a = i - 1 + ca;
      if (a < 0 || a >= nx) continue;
      const long c = (long)b * nx + a;
      const int mi = i - a, mj = j - b;
      add(diag + 16 * c, false, mi, mj, a, b);
      if (a + 1 < nx) add(ax + 16 * c, false, mi, mj, a + 1, b);
      if (a > 0) add(ax + 16 * (c - 1), true, mi, mj, a - 1, b);
      if (b + 1 < ny) add(ay + 16 * c, false, mi, mj, a, b + 1);
      if (b > 0) add(ay + 16 * (c - nx), true, mi, mj, a, b - 1);
    }
  }
  for (int k = 0; k < 9; ++k) A9[9 * n + k] = row[k];
}

// Galerkin coarse operator R A P at coarse node (I, J): bilinear interpolation (fine
// node 2I <-> coarse I, weight 1/2 to the two coarse neighbours of an odd fine node),
// gathered over the 3 x 3 fine nodes that interpolate from (I, J).
__global__ __launch_bounds__(256) void mg_rap_kernel(int mx, int my,
                                                    const double* __restrict__ Af, int mxc,
                                                    int myc, double* __restrict__ Ac) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= (long)mxc * myc) return;
  const int I = (int)(n % mxc), J = (int)(n / mxc);
  double row[9];
  for (int k = 0; k < 9; ++k) row[k] = 0.0;
  for (int fj = -1; fj <= 1; ++fj) {
    const int j = 2 * J + fj;
    if (j < 0 || j >= my) continue;
    for (int fi = -1; fi <= 1; ++fi) {
      const int i = 2 * I + fi;
      if (i < 0 || i >= mx) continue;
      const double wi = (fi ? 0.5 : 1.0) * (fj ? 0.5 : 1.0);  // P[(i, j)][(I, J)]
      const double* a = Af + 9 * ((long)j * mx + i);
      for (int dj = -1; dj <= 1; ++dj) {
        const int j2 = j + dj;
        if (j2 < 0 || j2 >= my) continue;
        for (int di = -1; di <= 1; ++di) {
          const int i2 = i + di;
          if (i2 < 0 || i2 >= mx) continue;
          const double v = wi * a[(dj + 1) * 3 + di + 1];
          // coarse parents of (i2, j2)
          const int i0 = i2 >> 1, i1 = (i2 + 1) >> 1, j0 = j2 >> 1, j1 = (j2 + 1) >> 1;
          const double wx = i0 == i1 ? 1.0 : 0.5, wy = j0 == j1 ? 1.0 : 0.5;
          for (int pj = 0; pj < (j0 == j1 ? 1 : 2); ++pj)
            for (int pi = 0; pi < (i0 == i1 ? 1 : 2); ++pi) {
              const int oi = (pi ? i1 : i0) - I, oj = (pj ? j1 : j0) - J;
              row[(oj + 1) * 3 + oi + 1] += v * wx * wy;
            }
        }
      }
    }
  }
  for (int k = 0; k < 9; ++k) Ac[9 * n + k] = row[k];
}

// l1-Jacobi: dinv = 1 / (a_ii + sum_{j != i} |a_ij|); bad |= 2 for a non-positive diagonal
__global__ __launch_bounds__(256) void mg_dinv_kernel(long n, const double* __restrict__ A9,
                                                     double* __restrict__ dinv,
                                                     int* __restrict__ bad) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < 9; ++k) s += k == 4 ? A9[9 * i + k] : fabs(A9[9 * i + k]);
  if (!(A9[9 * i + 4] > 0.0) || !(s > 0.0)) atomicOr(bad, 2);
  dinv[i] = s > 0.0 ? 1.0 / s : 0.0;
}

__global__ void to_float_kernel(long n, const double* __restrict__ a, float* __restrict__ b) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// ------------------------------------------------------------ set-up

Emb embedding(const Geom& g) {
  const double r3 = std::sqrt(3.0);
  return Emb{std::sqrt(g.hx) / 2, std::sqrt(g.hx) / (2 * r3), std::sqrt(g.hy) / 2,
             std::sqrt(g.hy) / (2 * r3)};
}

unsigned nblocks(long n) { return (unsigned)((n + 255) / 256); }

// Dense inverse of the coarsest operator (Cholesky, then the inverse column by column),
// symmetrised so that the device can read columns as rows.
std::vector<double> coarse_inverse(const std::vector<double>& A, int mx, int my) {
  const int nc = mx * my;
  std::vector<double> M((size_t)nc * nc, 0.0);
  for (int j = 0; j < my; ++j)
    for (int i = 0; i < mx; ++i)
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
          const int i2 = i + di, j2 = j + dj;
          if (i2 < 0 || i2 >= mx || j2 < 0 || j2 >= my) continue;
          M[(size_t)(j * mx + i) * nc + j2 * mx + i2] = A[9 * ((size_t)j * mx + i) + (dj + 1) * 3 + di + 1];
        }
  for (int i = 0; i < nc; ++i)  // the assembled entries agree to rounding
    for (int j = 0; j < i; ++j) {
      const double v = 0.5 * (M[(size_t)i * nc + j] + M[(size_t)j * nc + i]);
      M[(size_t)i * nc + j] = M[(size_t)j * nc + i] = v;
    }
  std::vector<double> L((size_t)nc * nc, 0.0);
  for (int j = 0; j < nc; ++j) {
    double sjj = M[(size_t)j * nc + j];
    for (int k = 0; k < j; ++k) sjj -= L[(size_t)j * nc + k] * L[(size_t)j * nc + k];
    RTE_REQUIRE(sjj > 0.0, "DSA: coarse operator not positive definite");
    const double ljj = std::sqrt(sjj);
    L[(size_t)j * nc + j] = ljj;
    for (int i = j + 1; i < nc; ++i) {
      double t = M[(size_t)i * nc + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * nc + k] * L[(size_t)j * nc + k];
      L[(size_t)i * nc + j] = t / ljj;
    }
  }
  std::vector<double> inv((size_t)nc * nc), y(nc);
  for (int e = 0; e < nc; ++e) {
    for (int i = 0; i < nc; ++i) {  // L y = e_e
      double t = i == e ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) t -= L[(size_t)i * nc + k] * y[k];
      y[i] = t / L[(size_t)i * nc + i];
    }
    for (int i = nc - 1; i >= 0; --i) {  // L^T x = y
      double t = y[i];
      for (int k = i + 1; k < nc; ++k) t -= L[(size_t)k * nc + i] * inv[(size_t)k * nc + e];
      inv[(size_t)i * nc + e] = t / L[(size_t)i * nc + i];
    }
  }
  for (int i = 0; i < nc; ++i)
    for (int j = 0; j < i; ++j) {
      const double v = 0.5 * (inv[(size_t)i * nc + j] + inv[(size_t)j * nc + i]);
      inv[(size_t)i * nc + j] = inv[(size_t)j * nc + i] = v;
    }
  return inv;
}

}  // namespace

// LDS bytes one workgroup may use on the current device
size_t max_lds_bytes() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
    return 65536;
  return (size_t)v;
}

// LDS layout of the one-workgroup cycle (levels lsmall .. end): b and x of every level,
// stencil, smoother and scratch vector of every level but a dense-solved coarsest, then
// the dense inverse if it still fits.  small_lds stays 0 when the levels do not fit.
void plan_small_cycle(DSA* d, size_t budget) {
  const int nl = (int)d->mg.size() - d->lsmall;
  d->small_off.assign(7 * kMaxSmallLevels + 1, -1);
  d->small_lds = 0;
  if (nl > kMaxSmallLevels) return;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 15) & ~(size_t)15;
    return (int)o;
  };
  for (int i = 0; i < nl; ++i) {
    const MgLevel& L = *d->mg[d->lsmall + i];
    const size_t n = (size_t)L.mx * L.my;
    int* o = &d->small_off[7 * i];
    o[0] = L.mx;
    o[1] = L.my;
    o[4] = take(8 * n);  // b
    o[5] = take(8 * n);  // x
    if (!(i == nl - 1 && d->ncoarse > 0)) {
      o[2] = take(4 * 9 * n);  // stencils (FP32)
      o[3] = take(8 * n);      // l1-Jacobi weights
      o[6] = take(8 * n);      // scratch vector
    }
  }
  if (off > budget) return;
  const size_t nci = (size_t)d->ncoarse * d->ncoarse * 8;
  if (d->ncoarse > 0 && off + nci <= budget) d->small_off[7 * kMaxSmallLevels] = take(nci);
  d->small_lds = off;
}

// The blocks, the nodal hierarchy and its smoothers are assembled on the device; only
// the coarsest grid (at most kCoarseDense nodes) is inverted on the host.
// grids whose large-tile launch has fewer blocks than this (four per compute unit) take the
// small tiles: at 1024 x 1024 cells, the 513^2 .. 65^2 grids.  RTE_MG_TILE_BLOCKS overrides
// it (0: large tiles on every level); both tile shapes give bitwise the same cycle.
constexpr int kSmallTileBlocks = 1024;

static int tile_blocks_setting() {
  const char* v = std::getenv("RTE_MG_TILE_BLOCKS");
  return v && v[0] ? std::max(0, std::atoi(v)) : kSmallTileBlocks;
}

DSA* dsa_create(const Geom& g, const double* sigma_t_dev, const double* sigma_s_dev,
                hipStream_t st) {
  DSA* d = new DSA();
  try {
    d->g = g;
    d->tile_blocks = tile_blocks_setting();
    const long n = g.ncell;
    DevBuf<int> bad(1);
    RTE_CHECK_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int), st));
    d->diag.alloc(16 * n); d->ax.alloc(16 * n); d->ay.alloc(16 * n); d->minv.alloc(16 * n);
    hipLaunchKernelGGL(dsa_blocks_kernel, dim3(nblocks(n)), dim3(256), 0, st, g.nx, g.ny, g.hx,
                       g.hy, sigma_t_dev, sigma_s_dev, d->diag.get(), d->ax.get(), d->ay.get(),
                       d->minv.get(), bad.get());
    d->mc.alloc(10 * n);
    d->dcoef.alloc(n);
    d->sa.alloc(n);
    hipLaunchKernelGGL(dsa_compact_kernel, dim3(nblocks(n)), dim3(256), 0, st, n, d->minv.get(),
                       sigma_t_dev, sigma_s_dev, d->mc.get(), d->dcoef.get(), d->sa.get());
    // grid hierarchy: vertex-centred halving while both node counts allow it
    std::vector<std::pair<int, int>> dims{{g.nx + 1, g.ny + 1}};
    while (true) {
      const int mx = dims.back().first, my = dims.back().second;
      if ((long)mx * my <= kCoarseDense) break;
      if ((mx - 1) % 2 || (my - 1) % 2 || mx < 5 || my < 5) break;
      dims.push_back({(mx + 1) / 2, (my + 1) / 2});
    }
    for (size_t l = 0; l < dims.size(); ++l) {
      d->mg.push_back(std::make_unique<MgLevel>());
      MgLevel& L = *d->mg[l];
      L.mx = dims[l].first;
      L.my = dims[l].second;
      const long nn = (long)L.mx * L.my;
      L.A9.alloc(9 * nn);
      L.dinv.alloc(nn);
      L.x.alloc(nn);
      L.b.alloc(nn);
      L.t.alloc(nn);
      if (l == 0)
        hipLaunchKernelGGL(mg_fine_kernel, dim3(nblocks(nn)), dim3(256), 0, st, g.nx, g.ny,
                           embedding(g), d->diag.get(), d->ax.get(), d->ay.get(), L.A9.get());
      else {
        const MgLevel& F = *d->mg[l - 1];
        hipLaunchKernelGGL(mg_rap_kernel, dim3(nblocks(nn)), dim3(256), 0, st, F.mx, F.my,
                           F.A9.get(), L.mx, L.my, L.A9.get());
      }
      hipLaunchKernelGGL(mg_dinv_kernel, dim3(nblocks(nn)), dim3(256), 0, st, nn, L.A9.get(),
                         L.dinv.get(), bad.get());
      L.A9c.alloc(9 * nn);
      hipLaunchKernelGGL(to_float_kernel, dim3(nblocks(9 * nn)), dim3(256), 0, st, 9 * nn, L.A9.get(),
                         L.A9c.get());
      RTE_CHECK_HIP(hipGetLastError());
    }
    const MgLevel& Lc = *d->mg.back();
    const int nc = Lc.mx * Lc.my;
    std::vector<double> Ac;
    if (nc <= kCoarseDense) {
      Ac.resize((size_t)9 * nc);
      RTE_CHECK_HIP(hipMemcpyAsync(Ac.data(), Lc.A9.get(), Ac.size() * sizeof(double),
                                   hipMemcpyDeviceToHost, st));
    }
    int hbad = 0;
    RTE_CHECK_HIP(hipMemcpyAsync(&hbad, bad.get(), sizeof(int), hipMemcpyDeviceToHost, st));
    RTE_CHECK_HIP(hipStreamSynchronize(st));
    RTE_REQUIRE(!(hbad & 1), "DSA: singular diagonal block");
    RTE_REQUIRE(!(hbad & 2), "DSA: non-positive diagonal in the multigrid hierarchy");
    d->ncoarse = 0;
    if (nc <= kCoarseDense) {
      const std::vector<double> inv = coarse_inverse(Ac, Lc.mx, Lc.my);
      d->cinv.alloc(inv.size());
      RTE_CHECK_HIP(hipMemcpy(d->cinv.get(), inv.data(), inv.size() * sizeof(double),
                              hipMemcpyHostToDevice));
      d->ncoarse = nc;
    }
    // the one-workgroup cycle takes over from the first level that is small enough
    d->lsmall = (int)d->mg.size() - 1;
    while (d->lsmall > 0 && (long)d->mg[d->lsmall - 1]->mx * d->mg[d->lsmall - 1]->my <= kSmallNodes)
      --d->lsmall;
    plan_small_cycle(d, max_lds_bytes() - sizeof(double) * 8 * kCoarseDense);
    std::vector<MgDev> views;
    for (auto& L : d->mg)
      views.push_back(MgDev{L->mx, L->my, L->A9c.get(), L->dinv.get(), L->x.get(), L->b.get(), L->t.get()});
    d->mgdev.alloc(views.size());
    RTE_CHECK_HIP(hipMemcpy(d->mgdev.get(), views.data(), views.size() * sizeof(MgDev),
                            hipMemcpyHostToDevice));
    d->sig_s.alloc(n);
    RTE_CHECK_HIP(hipMemcpyAsync(d->sig_s.get(), sigma_s_dev, n * sizeof(double),
                                 hipMemcpyDeviceToDevice, st));
    const long nd = g.ndof;
    for (int i = 0; i < 3; ++i) d->xs[i].alloc(nd), d->bs[i].alloc(nd);
    d->r.alloc(nd); d->r2.alloc(nd); d->z.alloc(nd); d->p0.alloc(nd); d->p1.alloc(nd);
    d->q.alloc(nd);
    d->z1.alloc(nd); d->t.alloc(nd);
    d->nblk = (int)((n + 255) / 256);
    {
      const dim3 tg = cell_tiles(g.nx, g.ny);
      d->ntile = (int)(tg.x * tg.y);
    }
    d->part1.alloc(std::max(d->nblk, d->ntile)); d->part2.alloc(std::max(d->nblk, d->ntile));
    d->part3.alloc(d->nblk);
    d->part4.alloc(d->nblk);
    d->scal.alloc(S_N);
    RTE_CHECK_HIP(hipMemsetAsync(d->scal.get(), 0, S_N * sizeof(double), st));
    return d;
  } catch (...) {
    delete d;
    throw;
  }
}

void dsa_destroy(DSA* d) { delete d; }

namespace {

OpA op_of(const DSA* d) {
  return OpA{d->g.nx, d->g.ny, axis_of(d->g.hx), axis_of(d->g.hy), d->dcoef.get(), d->sa.get()};
}

// where level l's V-cycle leaves its solution: x for the one-workgroup cycle, t for a
// level of the two-kernel cycle (its up kernel cannot overwrite x, which neighbouring
// blocks still read)
const double* level_solution(const DSA* d, int l) {
  return l == d->lsmall ? d->mg[l]->x.get() : d->mg[l]->t.get();
}

// one V-cycle on level l (x = V b), two l1-Jacobi sweeps before and after
void vcycle(DSA* d, int l, hipStream_t st) {
  MgLevel& L = *d->mg[l];
  const double* sc = d->scal.get();
  if (l == d->lsmall) {
    SmallPlan P{};
    P.nl = (int)d->mg.size() - l;
    P.ocinv = d->small_off[7 * kMaxSmallLevels];
    for (int i = 0; i < P.nl && i < kMaxSmallLevels; ++i) {
      const int* o = &d->small_off[7 * i];
      P.lv[i] = SmallLevel{o[0], o[1], o[2], o[3], o[4], o[5], o[6]};
    }
    if (d->small_lds > 0)
      hipLaunchKernelGGL(mg_small_kernel<true>, dim3(1), dim3(kSmallThreads), d->small_lds, st,
                         d->mgdev.get(), l, (int)d->mg.size(), d->cinv.get(), d->ncoarse,
                         kCoarseSweeps, P, sc);
    else
      hipLaunchKernelGGL(mg_small_kernel<false>, dim3(1), dim3(kSmallThreads), 0, st,
                         d->mgdev.get(), l, (int)d->mg.size(), d->cinv.get(), d->ncoarse,
                         kCoarseSweeps, P, sc);
    return;
  }
  MgLevel& C = *d->mg[l + 1];
  auto grid = [](int mx, int my, int tx, int ty) {
    return dim3((unsigned)((mx + tx - 1) / tx), (unsigned)((my + ty - 1) / ty));
  };
  const dim3 down = grid(C.mx, C.my, kDX, kDY);
  if (down.x * down.y >= (unsigned)d->tile_blocks)
    hipLaunchKernelGGL((mg_down_kernel<kDX, kDY>), down, dim3(256), 0, st, L.mx, L.my,
                       L.A9c.get(), L.dinv.get(), L.b.get(), L.x.get(), C.mx, C.my, C.b.get(), sc);
  else
    hipLaunchKernelGGL((mg_down_kernel<kDXs, kDYs>), grid(C.mx, C.my, kDXs, kDYs), dim3(256), 0, st,
                       L.mx, L.my, L.A9c.get(), L.dinv.get(), L.b.get(), L.x.get(), C.mx, C.my,
                       C.b.get(), sc);
  vcycle(d, l + 1, st);
  const dim3 up = grid(L.mx, L.my, kUX, kUY);
  if (up.x * up.y >= (unsigned)d->tile_blocks)
    hipLaunchKernelGGL((mg_up_kernel<kUX, kUY>), up, dim3(256), 0, st, L.mx, L.my, L.A9c.get(),
                       L.dinv.get(), L.b.get(), L.x.get(), C.mx, level_solution(d, l + 1),
                       L.t.get(), sc);
  else
    hipLaunchKernelGGL((mg_up_kernel<kUXs, kUYs>), grid(L.mx, L.my, kUXs, kUYs), dim3(256), 0, st,
                       L.mx, L.my, L.A9c.get(), L.dinv.get(), L.b.get(), L.x.get(), C.mx,
                       level_solution(d, l + 1), L.t.get(), sc);
}

// z = M^{-1} r, part1 = r.z per tile.  M^{-1} is the symmetric two-level preconditioner
//   z1 = S r,  z2 = z1 + P V P^T (r - A z1),  z = z2 + S (r - A z2),
// S = w B^{-1} the damped block Jacobi smoother (w = kSmoothW), V one V-cycle.  It is
// symmetric positive definite since 2 S^{-1} - A is (w < 1: B^{-1} A has its spectrum in
// (0, 2)).
// With q != nullptr, r = rin - alpha q first (into rout, part2 = r.r per tile); else
// r = rin (rout unused).
void precondition(DSA* d, const double* rin, const double* q, double* rout, double* z,
                  hipStream_t st) {
  const Geom& g = d->g;
  const Emb em = embedding(g);
  const double* sc = d->scal.get();
  MgLevel& L0 = *d->mg[0];
  const OpA op = op_of(d);
  const double* r = q ? rout : rin;
  if (q)
    hipLaunchKernelGGL(dg_smooth1_kernel<true>, cell_tiles(g.nx, g.ny), dim3(kCX * kCY), 0, st, op,
                       d->mc.get(), rin, q, rout, kSmoothW, d->z1.get(), em, d->t.get(),
                       L0.b.get(), d->part2.get(), sc);
  else
    hipLaunchKernelGGL(dg_smooth1_kernel<false>, cell_tiles(g.nx, g.ny), dim3(kCX * kCY), 0, st,
                       op, d->mc.get(), rin, nullptr, nullptr, kSmoothW, d->z1.get(), em,
                       d->t.get(), L0.b.get(), nullptr, sc);
  const long ne = restrict_edge_threads(g.nx, g.ny);
  if (ne > 0)
    hipLaunchKernelGGL(dg_restrict_edges_kernel, dim3(nblocks(ne)), dim3(256), 0, st, g.nx, g.ny,
                       em, d->t.get(), L0.b.get(), sc);
  vcycle(d, 0, st);
  hipLaunchKernelGGL(dg_smooth2_kernel, cell_tiles(g.nx, g.ny), dim3(kCX * kCY), 0, st, op, em,
                     d->mc.get(), r, d->z1.get(), level_solution(d, 0), kSmoothW, z, d->part1.get(), sc);
}

}  // namespace

int dsa_apply(DSA* d, const double* phi_star, const double* phi_prev, double* phi_next,
              double rel_tol, hipStream_t st) {
  const Geom& g = d->g;
  const long n = g.ncell;
  const int nb = d->nblk;
  double* sc = d->scal.get();
  // The initial guess: zero for the first solve; afterwards the combination of the last
  // two solutions whose right-hand sides best fit this one (least squares; one term after
  // the first solve): successive right-hand sides of SI-DSA are nearly dependent once the
  // iteration settles.  Its residual is formed exactly.
  double* x = d->xs[d->xc].get();
  double* bsave = d->bs[d->bsv].get();
  if (d->nprev == 0) {
    hipLaunchKernelGGL(init_r_kernel<false>, dim3(nb), dim3(kInitThreads), 0, st, n, d->sig_s.get(),
                       phi_star, phi_prev, x, d->r.get(), d->p0.get(), bsave, nullptr, nullptr,
                       d->part2.get(), nullptr, nullptr);
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, st, d->part2.get(), nb, sc + S_BB);
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, st, d->part2.get(), nb, sc + S_RR);
  } else {
    const double* bp2 = d->nprev > 1 ? d->bs[d->b2].get() : nullptr;
    hipLaunchKernelGGL(init_r_kernel<true>, dim3(nb), dim3(kInitThreads), 0, st, n, d->sig_s.get(),
                       phi_star, phi_prev, x, d->r.get(), d->p0.get(), nullptr,
                       d->bs[d->b1].get(), bp2, d->part2.get(), d->part3.get(), d->part4.get());
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, st, d->part2.get(), nb, sc + S_BB);
    hipLaunchKernelGGL(guess_weights_kernel, dim3(1), dim3(1024), 0, st, d->part3.get(),
                       d->part4.get(), nb, d->nprev, sc);
    hipLaunchKernelGGL(guess_combine_kernel, dim3((g.ndof + 255) / 256), dim3(256), 0, st, g.ndof,
                       d->xs[d->x1].get(), d->xs[d->x2].get(), d->nprev, x, sc);
    hipLaunchKernelGGL(guess_residual_kernel, cell_tiles(g.nx, g.ny), dim3(kCX * kCY), 0, st,
                       op_of(d), x, d->r.get(), bsave, d->part2.get());
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, st, d->part2.get(), d->ntile,
                       sc + S_RR);
  }
  hipLaunchKernelGGL(clear_done_kernel, dim3(1), dim3(1), 0, st, sc);
  precondition(d, d->r.get(), nullptr, nullptr, d->z.get(), st);
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, st, d->part1.get(), d->ntile, sc + S_RHO);
  hipLaunchKernelGGL(start_kernel, dim3(1), dim3(1), 0, st, sc, rel_tol);
  RTE_CHECK_HIP(hipGetLastError());
  // Iteration k writes p_k to pnew and r_k to rnext; both pairs alternate (p1 holds p_k for
  // odd k, which axpy_out_kernel relies on).
  double* pold = d->p0.get();
  double* pnew = d->p1.get();
  double* rcur = d->r.get();
  double* rnext = d->r2.get();
  const dim3 tiles = cell_tiles(g.nx, g.ny);
  // Iterations are enqueued in batches, the done flag read back after each: the first batch
  // is one fewer than the previous solve took (successive solves need about as many), the
  // later ones short, so that few iterations are enqueued after convergence (they return at
  // once) and the host waits on the stream only once or twice per solve.
  const int max_iter = 40000;
  int batch = std::max(d->last_iters - 1, 4);
  double hsc[S_N];
  for (int it = 0; it < max_iter; it += batch, batch = 2) {
    for (int k = 0; k < batch; ++k) {
      hipLaunchKernelGGL(spmv_kernel, tiles, dim3(kCX * kCY), 0, st, op_of(d), d->z.get(), pold,
                         pnew, d->q.get(), x, d->part1.get(), sc);
      hipLaunchKernelGGL(reduce_alpha_kernel, dim3(1), dim3(1024), 0, st, d->part1.get(), d->ntile,
                         sc);
      precondition(d, rcur, d->q.get(), rnext, d->z.get(), st);
      hipLaunchKernelGGL(reduce_beta_kernel, dim3(1), dim3(1024), 0, st, d->part1.get(), d->ntile,
                         d->part2.get(), d->ntile, sc);
      std::swap(pold, pnew);
      std::swap(rcur, rnext);
    }
    RTE_CHECK_HIP(hipGetLastError());
    RTE_CHECK_HIP(hipMemcpyAsync(hsc, sc, sizeof(hsc), hipMemcpyDeviceToHost, st));
    RTE_CHECK_HIP(hipStreamSynchronize(st));
    if (hsc[S_DONE] != 0.0) break;
  }
  hipLaunchKernelGGL(axpy_out_kernel, dim3((g.ndof + 255) / 256), dim3(256), 0, st, g.ndof,
                     phi_star, x, d->p0.get(), d->p1.get(), sc, phi_next);
  // this solve becomes the latest of the history
  std::tie(d->xc, d->x1, d->x2) = std::make_tuple(d->x2, d->xc, d->x1);
  std::tie(d->bsv, d->b1, d->b2) = std::make_tuple(d->b2, d->bsv, d->b1);
  d->nprev = std::min(d->nprev + 1, 2);
  d->last_iters = (int)hsc[S_ITERS];
  RTE_CHECK_HIP(hipGetLastError());
  return d->last_iters;
}

}  // namespace rte
