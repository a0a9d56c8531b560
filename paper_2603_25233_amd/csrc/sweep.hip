// Upwind DG-Q1 transport sweep on gfx950 (paper Sec. 2.2, "Transport sweeps").
//
// For an ordinate with signs (sx, sy) the cells are taken in upwind order; with
// cells reflected so that the sweep always runs towards +x and +y ("canonical
// frame") the cell system of the upwind DG weak form (Sec. 2.1) is
//
//   (sigma I + a (I (x) L) + b (L (x) I)) psi' = s' + a c (x) u + b v (x) c,
//   L = [[1, sqrt3], [-sqrt3, 3]],  c = (1, -sqrt3),  a = |Omega_x|/hx, b = |Omega_y|/hy,
//
// with DOF index k = 2q + p (p: x-degree, q: y-degree), s' the source with the
// odd-in-x moments multiplied by sx and the odd-in-y ones by sy, u the inflow
// trace on the x face (u_q = psi_0q + sqrt3 psi_1q of the upwind cell, or
// sqrt(hx) times the face moments of g on the boundary) and v that on the y face.
// All blocks lie in the commutative algebra spanned by I and L (L^2 = 4L - 6I), so
// the 4x4 solve is a 2x2 block Cramer rule:
//   psi'_0 = Delta^{-1} [(A + 3b) R_0 - sqrt3 b R_1],  psi'_1 = Delta^{-1} [sqrt3 b R_0 + (A + b) R_1],
//   A = sigma + a L,  Delta = A^2 + 4bA + 6b^2 = d0 I + d1 L,
//   d0 = sigma^2 + 4 b sigma + 6 b^2 - 6 a^2,  d1 = 2a (sigma + 2a + 2b),
//   Delta^{-1} = ((d0 + 4 d1) I - d1 L) / (d0^2 + 4 d0 d1 + 6 d1^2).
//
// Parallel layout (diagonal wavefront, KBA-style, one direction batch per
// workgroup): thread r owns canonical row r and, at step t, the cell of column
// t - r, so all cells of one anti-diagonal are solved together.  The x-inflow trace
// stays in registers; the y-inflow trace of row r comes from row r-1 of the
// previous step through a double-buffered LDS slot, one barrier per step.  D
// directions of the same quadrant are solved per thread in lock step (ILP); their
// weighted sum is written once per cell when the scalar flux is requested.
#include <cmath>

#include "common.h"

namespace rte {

namespace {

constexpr double kSqrt3 = 1.7320508075688772935;

template <typename T>
struct Cell {
  T p[4];
  T uo[2];  // outflow trace on the downstream x face (index q)
  T vo[2];  // outflow trace on the downstream y face (index p)
};

template <typename T>
__device__ __forceinline__ void solve_cell(T sig, T a, T b, const T s[4], const T u[2],
                                           const T v[2], Cell<T>& out) {
  const T r3 = T(kSqrt3);
  const T R0 = s[0] + a * u[0] + b * v[0];
  const T R1 = s[1] - r3 * a * u[0] + b * v[1];
  const T R2 = s[2] + a * u[1] - r3 * b * v[0];
  const T R3 = s[3] - r3 * a * u[1] - r3 * b * v[1];
  // L applied to the two p-vectors (R0,R1) and (R2,R3)
  const T l00 = R0 + r3 * R1, l01 = T(3) * R1 - r3 * R0;
  const T l10 = R2 + r3 * R3, l11 = T(3) * R3 - r3 * R2;
  const T c3 = sig + T(3) * b, c1 = sig + b, rb = r3 * b;
  const T y00 = c3 * R0 + a * l00 - rb * R2;
  const T y01 = c3 * R1 + a * l01 - rb * R3;
  const T y10 = rb * R0 + c1 * R2 + a * l10;
  const T y11 = rb * R1 + c1 * R3 + a * l11;
  const T d0 = sig * sig + T(4) * b * sig + T(6) * (b * b - a * a);
  const T d1 = T(2) * a * (sig + T(2) * (a + b));
  const T det = d0 * d0 + T(4) * d0 * d1 + T(6) * d1 * d1;
  const T inv = T(1) / det;
  const T e0 = (d0 + T(4) * d1) * inv, e1 = -d1 * inv;
  const T m0 = y00 + r3 * y01, m1 = T(3) * y01 - r3 * y00;
  const T n0 = y10 + r3 * y11, n1 = T(3) * y11 - r3 * y10;
  out.p[0] = e0 * y00 + e1 * m0;
  out.p[1] = e0 * y01 + e1 * m1;
  out.p[2] = e0 * y10 + e1 * n0;
  out.p[3] = e0 * y11 + e1 * n1;
  out.uo[0] = out.p[0] + r3 * out.p[1];
  out.uo[1] = out.p[2] + r3 * out.p[3];
  out.vo[0] = out.p[0] + r3 * out.p[2];
  out.vo[1] = out.p[1] + r3 * out.p[3];
}

template <typename T>
struct Vec4 {
  T v[4];
};

template <typename T>
__device__ __forceinline__ Vec4<T> load4(const T* p) {
  Vec4<T> r;
  if constexpr (sizeof(T) == 8) {
    const double2* q = reinterpret_cast<const double2*>(p);
    double2 x = q[0], y = q[1];
    r.v[0] = x.x; r.v[1] = x.y; r.v[2] = y.x; r.v[3] = y.y;
  } else {
    float4 x = *reinterpret_cast<const float4*>(p);
    r.v[0] = x.x; r.v[1] = x.y; r.v[2] = x.z; r.v[3] = x.w;
  }
  return r;
}

template <typename T>
__device__ __forceinline__ void store4(T* p, const T v[4]) {
  if constexpr (sizeof(T) == 8) {
    double2* q = reinterpret_cast<double2*>(p);
    q[0] = make_double2(v[0], v[1]);
    q[1] = make_double2(v[2], v[3]);
  } else {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  }
}

// One workgroup sweeps D directions (dirs[blockIdx.x*D + d]) of one quadrant.
// psi: [slots][ndof] or null.  part: [gridDim.x][ndof] weighted partial sums or null.
template <typename T, int D>
__global__ __launch_bounds__(1024) void sweep_kernel(
    int nx, int ny, int mb, double shx, double shy, const SweepDir* __restrict__ dirs,
    const double* __restrict__ sigma_t, const T* __restrict__ src,
    const double* __restrict__ bc, T* __restrict__ psi, T* __restrict__ part, long ndof) {
  extern __shared__ unsigned char smem_raw[];
  T* vbuf = reinterpret_cast<T*>(smem_raw);  // [2][blockDim.x][D][2]
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const SweepDir* grp = dirs + (long)blockIdx.x * D;
  const int sx = grp[0].sx, sy = grp[0].sy;
  const T fx = T(sx), fy = T(sy), fxy = T(sx * sy);
  T a[D], b[D], w[D];
  long base[D];
  bool valid[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    a[d] = T(grp[d].a);
    b[d] = T(grp[d].b);
    w[d] = T(grp[d].w);
    valid[d] = grp[d].slot >= 0;
    base[d] = valid[d] ? (long)grp[d].slot * ndof : 0;
  }
  const bool row_ok = tid < ny;
  const int brow = sy > 0 ? tid : ny - 1 - tid;
  T u[D][2];
  {
    T g0 = T(0), g1 = T(0);
    if (row_ok && bc) {
      const int side = sx > 0 ? 0 : 1;
      g0 = T(bc[((long)side * mb + brow) * 2 + 0]);
      g1 = T(bc[((long)side * mb + brow) * 2 + 1]);
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
      u[d][0] = T(shx) * g0;
      u[d][1] = T(shx) * g1 * fy;
    }
  }
  const int nsteps = nx + ny - 1;
  for (int t = 0; t < nsteps; ++t) {
    const int ap = t - tid;
    if (row_ok && ap >= 0 && ap < nx) {
      const int acol = sx > 0 ? ap : nx - 1 - ap;
      const long c = (long)brow * nx + acol;
      T v[D][2];
      if (tid == 0) {
        T g0 = T(0), g1 = T(0);
        if (bc) {
          const int side = sy > 0 ? 2 : 3;
          g0 = T(bc[((long)side * mb + acol) * 2 + 0]);
          g1 = T(bc[((long)side * mb + acol) * 2 + 1]);
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
          v[d][0] = T(shy) * g0;
          v[d][1] = T(shy) * g1 * fx;
        }
      } else {
        const T* rd = vbuf + ((long)((t - 1) & 1) * nt + (tid - 1)) * D * 2;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          v[d][0] = rd[2 * d];
          v[d][1] = rd[2 * d + 1];
        }
      }
      const T sig = T(sigma_t[c]);
      const Vec4<T> s4 = load4(src + 4 * c);
      const T s[4] = {s4.v[0], fx * s4.v[1], fy * s4.v[2], fxy * s4.v[3]};
      T acc[4] = {T(0), T(0), T(0), T(0)};
      T* wr = vbuf + ((long)(t & 1) * nt + tid) * D * 2;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        Cell<T> cell;
        solve_cell<T>(sig, a[d], b[d], s, u[d], v[d], cell);
        u[d][0] = cell.uo[0];
        u[d][1] = cell.uo[1];
        wr[2 * d] = cell.vo[0];
        wr[2 * d + 1] = cell.vo[1];
        const T ph[4] = {cell.p[0], fx * cell.p[1], fy * cell.p[2], fxy * cell.p[3]};
        if (psi && valid[d]) store4(psi + base[d] + 4 * c, ph);
        if (part) {
#pragma unroll
          for (int k = 0; k < 4; ++k) acc[k] += w[d] * ph[k];
        }
      }
      if (part) store4(part + (long)blockIdx.x * ndof + 4 * c, acc);
    }
    __syncthreads();
  }
}

// phi[i] = sum_g part[g][i] in group order (deterministic).
template <typename T>
__global__ void reduce_parts_kernel(const T* __restrict__ part, int ngroups, long ndof,
                                    T* __restrict__ phi) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ndof) return;
  T s = T(0);
  for (int g = 0; g < ngroups; ++g) s += part[(long)g * ndof + i];
  phi[i] = s;
}

}  // namespace

// Groups directions by quadrant into padded groups of D (padding has slot = -1).
static std::vector<SweepDir> make_groups(const std::vector<SweepDir>& in, int D) {
  std::vector<SweepDir> out;
  for (int qx = 1; qx >= -1; qx -= 2)
    for (int qy = 1; qy >= -1; qy -= 2) {
      std::vector<SweepDir> q;
      for (const auto& d : in)
        if (d.sx == qx && d.sy == qy) q.push_back(d);
      for (size_t i = 0; i < q.size(); i += D)
        for (int d = 0; d < D; ++d) {
          if (i + d < q.size()) {
            out.push_back(q[i + d]);
          } else {
            SweepDir pad = q[i];
            pad.slot = -1;
            pad.w = 0.0;
            out.push_back(pad);
          }
        }
    }
  return out;
}

SweepPlan make_sweep_plan(const Geom& g, const std::vector<SweepDir>& dirs, bool want_phi,
                          size_t elem_bytes) {
  RTE_REQUIRE(g.ny >= 1 && g.ny <= 1024, "sweep: ny = %d outside [1, 1024]", g.ny);
  RTE_REQUIRE(!dirs.empty(), "sweep: no directions");
  SweepPlan pl;
  pl.nt = ((g.ny + 63) / 64) * 64;
  int D = 1;
  if (want_phi) {
    // enough workgroups to cover the chip first, then fewer partial sums
    const size_t lds_per_dir = 2ull * pl.nt * 2 * elem_bytes;
    while (D < 4 && dirs.size() / (2 * D) >= 256 && lds_per_dir * 2 * D <= 65536) D *= 2;
  }
  pl.D = D;
  pl.groups = make_groups(dirs, D);
  pl.ngroups = (int)(pl.groups.size() / D);
  return pl;
}

template <typename T>
void sweep_enqueue(const Geom& g, const SweepPlan& pl, const SweepDir* dirs_dev,
                   const double* sigma_t, const T* src, const double* bc, T* psi, T* phi,
                   T* part, hipStream_t st) {
  const size_t lds = 2ull * pl.nt * pl.D * 2 * sizeof(T);
  dim3 grid(pl.ngroups), block(pl.nt);
  const double shx = std::sqrt(g.hx), shy = std::sqrt(g.hy);
  T* pp = phi ? part : nullptr;
#define RTE_SWEEP_CASE(DD)                                                                \
  hipLaunchKernelGGL((sweep_kernel<T, DD>), grid, block, lds, st, g.nx, g.ny, g.mb, shx,  \
                     shy, dirs_dev, sigma_t, src, bc, psi, pp, g.ndof)
  if (pl.D == 1) RTE_SWEEP_CASE(1);
  else if (pl.D == 2) RTE_SWEEP_CASE(2);
  else RTE_SWEEP_CASE(4);
#undef RTE_SWEEP_CASE
  RTE_CHECK_HIP(hipGetLastError());
  if (phi) {
    const int tb = 256;
    hipLaunchKernelGGL((reduce_parts_kernel<T>), dim3((g.ndof + tb - 1) / tb), dim3(tb), 0, st,
                       part, pl.ngroups, g.ndof, phi);
    RTE_CHECK_HIP(hipGetLastError());
  }
}

template <typename T>
void launch_sweep(const Geom& g, const std::vector<SweepDir>& dirs, const double* sigma_t,
                  const T* src, const double* bc, T* psi, T* phi, hipStream_t st) {
  SweepPlan pl = make_sweep_plan(g, dirs, phi != nullptr, sizeof(T));
  DevBuf<SweepDir> ddirs(pl.groups.size());
  RTE_CHECK_HIP(hipMemcpy(ddirs.get(), pl.groups.data(), pl.groups.size() * sizeof(SweepDir),
                          hipMemcpyHostToDevice));
  DevBuf<T> part;
  if (phi) part.alloc((size_t)pl.ngroups * g.ndof);
  sweep_enqueue<T>(g, pl, ddirs.get(), sigma_t, src, bc, psi, phi, part.get(), st);
  // the temporaries are freed at scope exit: the kernels must be done with them
  RTE_CHECK_HIP(hipStreamSynchronize(st));
}

#define RTE_INST(T)                                                                            \
  template void sweep_enqueue<T>(const Geom&, const SweepPlan&, const SweepDir*,              \
                                 const double*, const T*, const double*, T*, T*, T*,           \
                                 hipStream_t);                                                 \
  template void launch_sweep<T>(const Geom&, const std::vector<SweepDir>&, const double*,     \
                                const T*, const double*, T*, T*, hipStream_t);
RTE_INST(double)
RTE_INST(float)
#undef RTE_INST

}  // namespace rte
