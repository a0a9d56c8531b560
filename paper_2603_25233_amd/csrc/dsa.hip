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
// The 4x4 blocks are built on the host in closed form; the SPD system is solved by
// conjugate gradients with the inverse 4x4 diagonal blocks as preconditioner, all
// scalars kept on the device and every reduction done in a fixed order.
#include <cmath>
#include <cstring>

#include "common.h"

namespace rte {

static constexpr double kCip = 8.0;

struct DSA {
  Geom g;
  DevBuf<double> diag, ax, ay, minv, sig_s;  // [ncell][16] blocks, [ncell]
  DevBuf<double> x, r, z, p0, p1, q, b;
  DevBuf<double> part1, part2;                 // per-block partial sums
  DevBuf<double> scal;                         // device scalars (see Sc below)
  int nblk = 0;
};

// layout of the device scalar block
enum Sc { S_RHO = 0, S_ALPHA, S_BETA, S_RR, S_TOL2, S_DONE, S_ITERS, S_PQ, S_N };

namespace {

// ------------------------------------------------------------ host assembly
using M4 = double[16];

// Kronecker placement of a 2x2 matrix P acting on the x-degree (k = 2q + p)
void put_p(double* B, const double P[2][2], double scale) {
  for (int q = 0; q < 2; ++q)
    for (int p = 0; p < 2; ++p)
      for (int pp = 0; pp < 2; ++pp) B[(2 * q + p) * 4 + (2 * q + pp)] += scale * P[p][pp];
}
// ... acting on the y-degree
void put_q(double* B, const double Q[2][2], double scale) {
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 2; ++q)
      for (int qq = 0; qq < 2; ++qq) B[(2 * q + p) * 4 + (2 * qq + p)] += scale * Q[q][qq];
}

// P = k jX jY^T + jX aY^T + aX jY^T
void face2(double P[2][2], double k, const double jX[2], const double jY[2], const double aX[2],
           const double aY[2]) {
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) P[i][j] = k * jX[i] * jY[j] + jX[i] * aY[j] + aX[i] * jY[j];
}

bool inv4(const double* A, double* out) {
  double m[4][8];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 8; ++j) m[i][j] = j < 4 ? A[4 * i + j] : (j - 4 == i ? 1.0 : 0.0);
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int i = c + 1; i < 4; ++i)
      if (std::fabs(m[i][c]) > std::fabs(m[piv][c])) piv = i;
    if (m[piv][c] == 0.0) return false;
    if (piv != c)
      for (int j = 0; j < 8; ++j) std::swap(m[c][j], m[piv][j]);
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
__device__ __forceinline__ void mv4(const double* __restrict__ B, const double* u, double* acc) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
    acc[i] += B[4 * i] * u[0] + B[4 * i + 1] * u[1] + B[4 * i + 2] * u[2] + B[4 * i + 3] * u[3];
}
__device__ __forceinline__ void mtv4(const double* __restrict__ B, const double* u, double* acc) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
    acc[i] += B[i] * u[0] + B[4 + i] * u[1] + B[8 + i] * u[2] + B[12 + i] * u[3];
}

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

// p_new = z + beta p_old (on the fly for the neighbours), q = A p_new, part = p.q
__global__ __launch_bounds__(256) void spmv_kernel(
    int nx, int ny, const double* __restrict__ diag, const double* __restrict__ ax,
    const double* __restrict__ ay, const double* __restrict__ z, const double* __restrict__ pold,
    double* __restrict__ pnew, double* __restrict__ q, double* __restrict__ part,
    const double* __restrict__ sc) {
  __shared__ double red[256];
  if (sc[S_DONE] != 0.0) return;
  const double beta = sc[S_BETA];
  const long ncell = (long)nx * ny;
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double dot = 0.0;
  if (c < ncell) {
    const int a = (int)(c % nx), b = (int)(c / nx);
    auto pv = [&](long cc, double* o) {
#pragma unroll
      for (int k = 0; k < 4; ++k) o[k] = z[4 * cc + k] + beta * pold[4 * cc + k];
    };
    double u[4], acc[4] = {0, 0, 0, 0}, nb[4];
    pv(c, u);
    mv4(diag + 16 * c, u, acc);
    if (a + 1 < nx) { pv(c + 1, nb); mv4(ax + 16 * c, nb, acc); }
    if (a > 0) { pv(c - 1, nb); mtv4(ax + 16 * (c - 1), nb, acc); }
    if (b + 1 < ny) { pv(c + nx, nb); mv4(ay + 16 * c, nb, acc); }
    if (b > 0) { pv(c - nx, nb); mtv4(ay + 16 * (c - nx), nb, acc); }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      pnew[4 * c + k] = u[k];
      q[4 * c + k] = acc[k];
      dot += u[k] * acc[k];
    }
  }
  const double s = block_sum(dot, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
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

__global__ void alpha_kernel(double* sc) {
  if (sc[S_DONE] != 0.0) return;
  sc[S_ALPHA] = sc[S_RHO] / sc[S_PQ];
}

// x += alpha p, r -= alpha q, z = Minv r, part1 = r.z, part2 = r.r
__global__ __launch_bounds__(256) void update_kernel(
    long ncell, const double* __restrict__ minv, const double* __restrict__ p,
    const double* __restrict__ q, double* __restrict__ x, double* __restrict__ r,
    double* __restrict__ z, double* __restrict__ part1, double* __restrict__ part2,
    const double* __restrict__ sc) {
  __shared__ double red[256];
  if (sc[S_DONE] != 0.0) return;
  const double alpha = sc[S_ALPHA];
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double rz = 0.0, rr = 0.0;
  if (c < ncell) {
    double rv[4], zv[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      x[4 * c + k] += alpha * p[4 * c + k];
      rv[k] = r[4 * c + k] - alpha * q[4 * c + k];
      r[4 * c + k] = rv[k];
    }
    mv4(minv + 16 * c, rv, zv);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      z[4 * c + k] = zv[k];
      rz += rv[k] * zv[k];
      rr += rv[k] * rv[k];
    }
  }
  const double s1 = block_sum(rz, red);
  const double s2 = block_sum(rr, red);
  if (threadIdx.x == 0) {
    part1[blockIdx.x] = s1;
    part2[blockIdx.x] = s2;
  }
}

// after reductions of r.z into sc[S_PQ] (reused as scratch) and r.r into sc[S_RR]
__global__ void beta_kernel(double* sc, double rz_new_unused) {
  if (sc[S_DONE] != 0.0) return;
  sc[S_ITERS] += 1.0;
  if (sc[S_RR] <= sc[S_TOL2]) {
    sc[S_DONE] = 1.0;
    return;
  }
  sc[S_BETA] = sc[S_PQ] / sc[S_RHO];
  sc[S_RHO] = sc[S_PQ];
}

// r = b = sigma_s (phi* - phi_prev); z = Minv r; x = 0; p_old = 0; part1 = r.z; part2 = r.r
__global__ __launch_bounds__(256) void init_kernel(
    long ncell, const double* __restrict__ sig_s, const double* __restrict__ phis,
    const double* __restrict__ phip, const double* __restrict__ minv, double* __restrict__ x,
    double* __restrict__ r, double* __restrict__ z, double* __restrict__ pold,
    double* __restrict__ part1, double* __restrict__ part2) {
  __shared__ double red[256];
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double rz = 0.0, rr = 0.0;
  if (c < ncell) {
    double rv[4], zv[4] = {0, 0, 0, 0};
    const double s = sig_s[c];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      rv[k] = s * (phis[4 * c + k] - phip[4 * c + k]);
      r[4 * c + k] = rv[k];
      x[4 * c + k] = 0.0;
      pold[4 * c + k] = 0.0;
    }
    mv4(minv + 16 * c, rv, zv);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      z[4 * c + k] = zv[k];
      rz += rv[k] * zv[k];
      rr += rv[k] * rv[k];
    }
  }
  const double s1 = block_sum(rz, red);
  const double s2 = block_sum(rr, red);
  if (threadIdx.x == 0) {
    part1[blockIdx.x] = s1;
    part2[blockIdx.x] = s2;
  }
}

// rho = r.z, rr = r.r, tol2 = tol^2 * rr, beta = 0
__global__ void start_kernel(double* sc, double tol) {
  sc[S_TOL2] = tol * tol * sc[S_RR];
  sc[S_BETA] = 0.0;
  sc[S_ITERS] = 0.0;
  sc[S_DONE] = (sc[S_RR] == 0.0) ? 1.0 : 0.0;
}

__global__ void axpy_out_kernel(long n, const double* __restrict__ a, const double* __restrict__ x,
                                double* __restrict__ out) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] + x[i];
}

}  // namespace

DSA* dsa_create(const Geom& g, const double* sigma_t_dev, const double* sigma_s_dev,
                hipStream_t st) {
  DSA* d = new DSA();
  try {
    d->g = g;
    const long n = g.ncell;
    std::vector<double> st_h(n), ss_h(n);
    RTE_CHECK_HIP(hipMemcpy(st_h.data(), sigma_t_dev, n * sizeof(double), hipMemcpyDeviceToHost));
    RTE_CHECK_HIP(hipMemcpy(ss_h.data(), sigma_s_dev, n * sizeof(double), hipMemcpyDeviceToHost));
    std::vector<double> diag(16 * n, 0.0), ax(16 * n, 0.0), ay(16 * n, 0.0), minv(16 * n, 0.0);
    const double hx = g.hx, hy = g.hy, r3 = std::sqrt(3.0);
    const double eRx[2] = {1 / std::sqrt(hx), r3 / std::sqrt(hx)};
    const double eLx[2] = {1 / std::sqrt(hx), -r3 / std::sqrt(hx)};
    const double dx[2] = {0.0, 2.0 * r3 / (hx * std::sqrt(hx))};
    const double eRy[2] = {1 / std::sqrt(hy), r3 / std::sqrt(hy)};
    const double eLy[2] = {1 / std::sqrt(hy), -r3 / std::sqrt(hy)};
    const double dy[2] = {0.0, 2.0 * r3 / (hy * std::sqrt(hy))};
    auto Dc = [&](long c) { return 1.0 / (3.0 * st_h[c]); };
    for (int b = 0; b < g.ny; ++b)
      for (int a = 0; a < g.nx; ++a) {
        const long c = (long)b * g.nx + a;
        double* B = &diag[16 * c];
        const double D = Dc(c), sa = st_h[c] - ss_h[c];
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
          if (an >= 0 && an < g.nx) {
            const long cn = (long)b * g.nx + an;
            const double Dn = Dc(cn);
            const double kap = std::max(0.25, 0.5 * kCip * (D / hx + Dn / hx));
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
              put_p(&ax[16 * c], P, 1.0);
            }
          } else {
            const double kap = std::max(0.25, kCip * D / hx);
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
          if (bn >= 0 && bn < g.ny) {
            const long cn = (long)bn * g.nx + a;
            const double Dn = Dc(cn);
            const double kap = std::max(0.25, 0.5 * kCip * (D / hy + Dn / hy));
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
              put_q(&ay[16 * c], P, 1.0);
            }
          } else {
            const double kap = std::max(0.25, kCip * D / hy);
            double dn[2];
            for (int i = 0; i < 2; ++i) dn[i] = (top ? 1.0 : -1.0) * D * dy[i];
            for (int i = 0; i < 2; ++i)
              for (int jj = 0; jj < 2; ++jj)
                P[i][jj] = kap * e[i] * e[jj] - 0.5 * e[i] * dn[jj] - 0.5 * dn[i] * e[jj];
            put_q(B, P, 1.0);
          }
        }
        RTE_REQUIRE(inv4(B, &minv[16 * c]), "DSA: singular diagonal block at cell %ld", c);
      }
    d->diag.alloc(16 * n); d->ax.alloc(16 * n); d->ay.alloc(16 * n); d->minv.alloc(16 * n);
    RTE_CHECK_HIP(hipMemcpy(d->diag.get(), diag.data(), 16 * n * sizeof(double), hipMemcpyHostToDevice));
    RTE_CHECK_HIP(hipMemcpy(d->ax.get(), ax.data(), 16 * n * sizeof(double), hipMemcpyHostToDevice));
    RTE_CHECK_HIP(hipMemcpy(d->ay.get(), ay.data(), 16 * n * sizeof(double), hipMemcpyHostToDevice));
    RTE_CHECK_HIP(hipMemcpy(d->minv.get(), minv.data(), 16 * n * sizeof(double), hipMemcpyHostToDevice));
    d->sig_s.alloc(n);
    RTE_CHECK_HIP(hipMemcpy(d->sig_s.get(), sigma_s_dev, n * sizeof(double), hipMemcpyDeviceToDevice));
    const long nd = g.ndof;
    d->x.alloc(nd); d->r.alloc(nd); d->z.alloc(nd); d->p0.alloc(nd); d->p1.alloc(nd); d->q.alloc(nd);
    d->nblk = (int)((n + 255) / 256);
    d->part1.alloc(d->nblk); d->part2.alloc(d->nblk);
    d->scal.alloc(S_N);
    RTE_CHECK_HIP(hipMemset(d->scal.get(), 0, S_N * sizeof(double)));
    (void)st;
    return d;
  } catch (...) {
    delete d;
    throw;
  }
}

void dsa_destroy(DSA* d) { delete d; }

int dsa_apply(DSA* d, const double* phi_star, const double* phi_prev, double* phi_next,
              double rel_tol, hipStream_t st) {
  const Geom& g = d->g;
  const long n = g.ncell;
  const int nb = d->nblk;
  double* sc = d->scal.get();
  hipLaunchKernelGGL(init_kernel, dim3(nb), dim3(256), 0, st, n, d->sig_s.get(), phi_star,
                     phi_prev, d->minv.get(), d->x.get(), d->r.get(), d->z.get(), d->p0.get(),
                     d->part1.get(), d->part2.get());
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, st, d->part1.get(), nb, sc + S_RHO);
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, st, d->part2.get(), nb, sc + S_RR);
  hipLaunchKernelGGL(start_kernel, dim3(1), dim3(1), 0, st, sc, rel_tol);
  RTE_CHECK_HIP(hipGetLastError());
  double* pold = d->p0.get();
  double* pnew = d->p1.get();
  const int chunk = 16, max_iter = 40000;
  double hsc[S_N];
  int it = 0;
  for (; it < max_iter; it += chunk) {
    for (int k = 0; k < chunk; ++k) {
      hipLaunchKernelGGL(spmv_kernel, dim3(nb), dim3(256), 0, st, g.nx, g.ny, d->diag.get(),
                         d->ax.get(), d->ay.get(), d->z.get(), pold, pnew, d->q.get(),
                         d->part1.get(), sc);
      hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, st, d->part1.get(), nb, sc + S_PQ);
      hipLaunchKernelGGL(alpha_kernel, dim3(1), dim3(1), 0, st, sc);
      hipLaunchKernelGGL(update_kernel, dim3(nb), dim3(256), 0, st, n, d->minv.get(), pnew,
                         d->q.get(), d->x.get(), d->r.get(), d->z.get(), d->part1.get(),
                         d->part2.get(), sc);
      hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, st, d->part1.get(), nb, sc + S_PQ);
      hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, st, d->part2.get(), nb, sc + S_RR);
      hipLaunchKernelGGL(beta_kernel, dim3(1), dim3(1), 0, st, sc, 0.0);
      std::swap(pold, pnew);
    }
    RTE_CHECK_HIP(hipGetLastError());
    RTE_CHECK_HIP(hipMemcpyAsync(hsc, sc, sizeof(hsc), hipMemcpyDeviceToHost, st));
    RTE_CHECK_HIP(hipStreamSynchronize(st));
    if (hsc[S_DONE] != 0.0) break;
  }
  hipLaunchKernelGGL(axpy_out_kernel, dim3((g.ndof + 255) / 256), dim3(256), 0, st, g.ndof,
                     phi_star, d->x.get(), phi_next);
  RTE_CHECK_HIP(hipGetLastError());
  return (int)hsc[S_ITERS];
}

}  // namespace rte
