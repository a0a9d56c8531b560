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
// workgroup): a thread owns a canonical row and, at step t, the cell of column
// t - row, so all cells of one anti-diagonal are solved together.  The x-inflow
// trace stays in registers; the y-inflow trace of row r comes from row r-1 of the
// previous step through a double-buffered LDS slot, one barrier per step.  A small
// kernel first copies the source and cross section into anti-diagonal order per
// quadrant, so that the loads of one step are contiguous; the results leave through
// an LDS ring written back by a dedicated store wavefront in row chunks (see
// sweep_kernel).  D directions of the same quadrant are solved per thread in lock
// step (ILP); their weighted sum is written once per cell when only the scalar flux
// is requested.
#include <algorithm>
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

// Raw source moments and cross section of one cell, fetched a superstep ahead.
template <typename T>
struct Slot {
  T s[4];
  T sig;
};

// Diagonal-major cell numbering of one quadrant.  In the canonical frame (cell
// coordinates reflected so that the sweep runs towards +x, +y) the cell of row r and
// column ap lies on anti-diagonal t = r + ap; anti-diagonals are stored one after the
// other, each in increasing r.  diag_first(t) is the position of anti-diagonal t's
// first cell, whose row is max(0, t - nx + 1).
__host__ __device__ __forceinline__ long diag_first(int t, int nx, int ny) {
  const long tl = t;
  const long a = t <= ny ? tl * (tl + 1) / 2 : (long)ny * (ny + 1) / 2 + (tl - ny) * ny;
  const long u = t > nx ? tl - nx : 0;
  return a - u * (u + 1) / 2;
}

// Diagonal-major copies of the sweep inputs for the quadrants in qmask: the source
// moments (with the quadrant's reflections applied to the odd moments) and sigma_t,
// converted to T.  dsrc: [4][ncell][4], dsig: [4][ncell].
template <typename T>
__global__ void diag_layout_kernel(int nx, int ny, int qmask, const double* __restrict__ sigma_t,
                                   const T* __restrict__ src, T* __restrict__ dsrc,
                                   T* __restrict__ dsig) {
  const long ncell = (long)nx * ny;
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int acol = (int)(c % nx), brow = (int)(c / nx);
  const Vec4<T> s4 = load4(src + 4 * c);
  const T sg = T(sigma_t[c]);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (!((qmask >> q) & 1)) continue;
    const int sx = (q & 1) ? -1 : 1, sy = (q & 2) ? -1 : 1;
    const int r = sy > 0 ? brow : ny - 1 - brow;
    const int ap = sx > 0 ? acol : nx - 1 - acol;
    const int t = r + ap;
    const long k = q * ncell + diag_first(t, nx, ny) + r - (t >= nx ? t - nx + 1 : 0);
    const T v[4] = {s4.v[0], T(sx) * s4.v[1], T(sy) * s4.v[2], T(sx * sy) * s4.v[3]};
    store4(dsrc + 4 * k, v);
    dsig[k] = sg;
  }
}

// One workgroup sweeps D directions (dirs[blockIdx.x*D + d]) of one quadrant.
// psi: [slots][ndof] or null (D == 1 when psi is written).  part: [gridDim.x][ndof]
// weighted partial sums or null.  dsrc/dsig: the diagonal-major inputs.
//
// Roles.  The first nc = blockDim.x - 64 threads compute; compute thread j owns the
// canonical rows j + k nc, k < RPT (both on the current anti-diagonal, so they are
// independent work).  The last wavefront only stores.  At step t the compute threads
// solve the cells of canonical column t - r and leave one 4-vector per row in an LDS
// ring of 2 ch steps (psi, or sum_d w_d psi_d when only the scalar flux is wanted).
// While the compute threads fill one chunk of ch steps, the store wavefront writes the
// previous chunk, a 1/ch share of its rows per step, each row as ch consecutive cells
// (16 bytes per lane), so a store instruction touches few cache lines.  Compute
// wavefronts issue no global stores, so waiting for their prefetched loads never
// waits for store acknowledgements (one vector-memory counter covers both).
//
// Prefetch.  Time is cut into supersteps of SS steps; consecutive rows of a step are
// consecutive in the diagonal-major inputs.  The inputs of superstep K + 1 are
// requested at the start of superstep K and waited for at its end.
template <typename T, int D, int NTB, int RPT>
__global__ __launch_bounds__(NTB) void sweep_kernel(
    int nx, int ny, int mb, int ch, double shx, double shy, const SweepDir* __restrict__ dirs,
    const T* __restrict__ dsrc_all, const T* __restrict__ dsig_all,
    const double* __restrict__ bc, T* __restrict__ psi, T* __restrict__ part, long ndof) {
  constexpr int SS = RPT == 1 ? 4 : 2;
  extern __shared__ unsigned char smem_raw[];
  const int tid = threadIdx.x;
  const int nc = blockDim.x - 64;            // compute threads
  const int nr = nc * RPT;                   // padded rows
  const int nsm = 2 * ch - 1;                // ring slot mask (ch is a power of two)
  T* vbuf = reinterpret_cast<T*>(smem_raw);  // [2][nr][D][2] y-inflow traces by row
  T* vbnd = vbuf + 4L * nr * D;              // [nx][2] inflow of canonical row 0
  T* ring = vbnd + 2L * nx;                  // [2 ch][nr][4] outputs by step and row
  const SweepDir* grp = dirs + (long)blockIdx.x * D;
  const int sx = grp[0].sx, sy = grp[0].sy;
  const T fx = T(sx), fy = T(sy), fxy = T(sx * sy);
  const long ncell = (long)nx * ny;
  const int q = (sx < 0 ? 1 : 0) + (sy < 0 ? 2 : 0);
  {
    const int yside = sy > 0 ? 2 : 3;
    for (int i = tid; i < nx; i += blockDim.x) {
      T g0 = T(0), g1 = T(0);
      if (bc) {
        g0 = T(bc[((long)yside * mb + i) * 2 + 0]);
        g1 = T(bc[((long)yside * mb + i) * 2 + 1]);
      }
      vbnd[2 * i] = T(shy) * g0;
      vbnd[2 * i + 1] = T(shy) * g1 * fx;
    }
  }
  const int nsteps = nx + ny - 1;
  if (tid >= nc) {
    // ------------------------------------------------ store wavefront
    const int lane = tid - nc;
    constexpr int LPC = sizeof(T) * 4 / 16;  // lanes per cell (16 bytes per lane)
    const int lpr = LPC * ch;                // lanes per row chunk
    const int rpi = 64 / lpr;                // rows per store instruction
    const int jrow = lane / lpr, ci = (lane % lpr) / LPC, half = lane % LPC;
    const bool wpsi = psi && grp[0].slot >= 0;
    T* pdst = wpsi ? psi + (long)grp[0].slot * ndof : nullptr;
    const T w0 = T(grp[0].w);
    T* pp = part ? part + (long)blockIdx.x * ndof : nullptr;
    // rows j (mod rpi ch) = jrow + rpi * piece of the chunk starting at step t0
    auto flush = [&](int t0, int piece) {
      const int t = t0 + ci;  // the step of this lane's cell
      if (t >= nsteps) return;
      const T* slot = ring + (long)(t & nsm) * nr * 4;
      for (int r = jrow + rpi * piece; r < ny; r += rpi * ch) {
        const int ap = t - r;
        if (ap >= 0 && ap < nx) {
          const int brow = sy > 0 ? r : ny - 1 - r;
          const long c = (long)brow * nx + (sx > 0 ? ap : nx - 1 - ap);
          const T* e = slot + (long)r * 4 + half * (16 / sizeof(T));
          if constexpr (sizeof(T) == 8) {
            const double2 v = *reinterpret_cast<const double2*>(e);
            if (wpsi) *reinterpret_cast<double2*>(pdst + 4 * c + 2 * half) = v;
            if (pp) {
              const double2 wv = D == 1 ? make_double2(w0 * v.x, w0 * v.y) : v;
              *reinterpret_cast<double2*>(pp + 4 * c + 2 * half) = wv;
            }
          } else {
            const float4 v = *reinterpret_cast<const float4*>(e);
            if (wpsi) *reinterpret_cast<float4*>(pdst + 4 * c) = v;
            if (pp) {
              const float4 wv = D == 1 ? make_float4(w0 * v.x, w0 * v.y, w0 * v.z, w0 * v.w) : v;
              *reinterpret_cast<float4*>(pp + 4 * c) = wv;
            }
          }
        }
      }
    };
    __syncthreads();  // vbnd ready
    for (int t = 0; t < nsteps; ++t) {
      // steps t0 - ch .. t0 - 1 are complete: write one piece of them per step
      const int t0 = t & ~(ch - 1);
      if (t0 >= ch) flush(t0 - ch, t - t0);
      __syncthreads();
    }
    const int tl = (nsteps - 1) & ~(ch - 1);  // first step of the last chunk
    if (tl >= ch)
      for (int piece = nsteps - tl; piece < ch; ++piece) flush(tl - ch, piece);
    for (int piece = 0; piece < ch; ++piece) flush(tl, piece);
    return;
  }
  // -------------------------------------------------- compute wavefronts
  T a[D], b[D], w[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    a[d] = T(grp[d].a);
    b[d] = T(grp[d].b);
    w[d] = T(grp[d].w);
  }
  const T* dsrc = dsrc_all + 4 * q * ncell;
  const T* dsig = dsig_all + q * ncell;
  int row[RPT];
  bool row_ok[RPT];
  T u[RPT][D][2];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    row[k] = tid + k * nc;
    row_ok[k] = row[k] < ny;
    const int brow = sy > 0 ? row[k] : ny - 1 - row[k];
    T g0 = T(0), g1 = T(0);
    if (row_ok[k] && bc) {
      const int side = sx > 0 ? 0 : 1;
      g0 = T(bc[((long)side * mb + brow) * 2 + 0]);
      g1 = T(bc[((long)side * mb + brow) * 2 + 1]);
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
      u[k][d][0] = T(shx) * g0;
      u[k][d][1] = T(shx) * g1 * fy;
    }
  }
  auto fetch = [&](Slot<T> (&sl)[RPT][SS], int K) {
#pragma unroll
    for (int i = 0; i < SS; ++i) {
      const int t = SS * K + i;
      const long base = diag_first(t, nx, ny) - (t >= nx ? t - nx + 1 : 0);
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int ap = t - row[k];
        if (row_ok[k] && ap >= 0 && ap < nx) {
          const long idx = base + row[k];
          sl[k][i].sig = dsig[idx];
          const Vec4<T> s4 = load4(dsrc + 4 * idx);
#pragma unroll
          for (int m = 0; m < 4; ++m) sl[k][i].s[m] = s4.v[m];
        }
      }
    }
  };
  Slot<T> A[RPT][SS], B[RPT][SS];
  fetch(A, 0);
  __syncthreads();  // vbnd ready
  for (int K = 0; SS * K < nsteps; ++K) {
    fetch(B, K + 1);
#pragma unroll
    for (int i = 0; i < SS; ++i) {
      const int t = SS * K + i;
      if (t < nsteps) {
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          const int r = row[k];
          const int ap = t - r;
          if (row_ok[k] && ap >= 0 && ap < nx) {
            const T* rd = r == 0 ? vbnd + 2 * (sx > 0 ? ap : nx - 1 - ap)
                                 : vbuf + ((long)((t + 1) & 1) * nr + (r - 1)) * D * 2;
            const int rstride = r == 0 ? 0 : 2;
            T* wr = vbuf + ((long)(t & 1) * nr + r) * D * 2;
            const Slot<T>& in = A[k][i];
            T acc[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int d = 0; d < D; ++d) {
              const T v[2] = {rd[rstride * d], rd[rstride * d + 1]};
              Cell<T> cell;
              solve_cell<T>(in.sig, a[d], b[d], in.s, u[k][d], v, cell);
              u[k][d][0] = cell.uo[0];
              u[k][d][1] = cell.uo[1];
              wr[2 * d] = cell.vo[0];
              wr[2 * d + 1] = cell.vo[1];
              const T ph[4] = {cell.p[0], fx * cell.p[1], fy * cell.p[2], fxy * cell.p[3]};
              if (D == 1) {
#pragma unroll
                for (int m = 0; m < 4; ++m) acc[m] = ph[m];
              } else {
#pragma unroll
                for (int m = 0; m < 4; ++m) acc[m] += w[d] * ph[m];
              }
            }
            store4(ring + ((long)(t & nsm) * nr + r) * 4, acc);
          }
        }
        __syncthreads();
      }
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k)
#pragma unroll
      for (int i = 0; i < SS; ++i) A[k][i] = B[k][i];
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

// vbuf [2][nr][D][2] + vbnd [nx][2] + ring [2 ch][nr][4], nr = padded rows
static size_t sweep_lds_bytes(const Geom& g, int nr, int D, int ch, size_t eb) {
  return (4ull * nr * D + 2ull * g.nx + 8ull * ch * nr) * eb;
}

// LDS bytes one workgroup may use on the current device
static size_t max_lds_per_block() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
    return 65536;
  return (size_t)v;
}

// compute threads and rows per compute thread for ny rows (one wavefront is added
// for the stores; a workgroup holds at most 1024 threads)
static void sweep_threads(int ny, int& nc, int& rpt) {
  rpt = ny <= 960 ? 1 : 2;
  nc = ((ny + rpt - 1) / rpt + 63) / 64 * 64;
}

// LDS per workgroup that still lets two workgroups share a compute unit (160 KB)
constexpr size_t kLdsTwoPerCU = 80 * 1024;

SweepPlan make_sweep_plan(const Geom& g, const std::vector<SweepDir>& dirs, bool want_phi,
                          bool want_psi, size_t elem_bytes) {
  RTE_REQUIRE(g.ny >= 1 && g.ny <= 1024, "sweep: ny = %d outside [1, 1024]", g.ny);
  RTE_REQUIRE(g.nx >= 1 && g.nx <= 4096, "sweep: nx = %d outside [1, 4096]", g.nx);
  RTE_REQUIRE(!dirs.empty(), "sweep: no directions");
  SweepPlan pl;
  int nc, rpt;
  sweep_threads(g.ny, nc, rpt);  // one more wavefront stores
  pl.nt = nc + 64;
  pl.rpt = rpt;
  const int nr = nc * rpt;
  const size_t lmax = max_lds_per_block();
  const size_t lcap = std::min(lmax, kLdsTwoPerCU);
  int D = 1;
  if (want_phi && !want_psi) {
    // enough workgroups to cover the chip first, then fewer partial sums; D is bounded
    // by the register budget (FP64: 2, and 1 beyond 576 threads)
    const int dmax = elem_bytes == 8 ? (pl.nt <= 576 && rpt == 1 ? 2 : 1) : 4;
    while (D < dmax && dirs.size() / (2 * D) >= 256 && sweep_lds_bytes(g, nr, 2 * D, 1, elem_bytes) <= lcap)
      D *= 2;
  }
  // store chunk: up to 128 bytes of one row per chunk (16 bytes per lane)
  const int chmax = (int)(128 / (4 * elem_bytes));
  int ch = 1;
  while (ch < chmax && sweep_lds_bytes(g, nr, D, 2 * ch, elem_bytes) <= lcap) ch *= 2;
  RTE_REQUIRE(sweep_lds_bytes(g, nr, D, ch, elem_bytes) <= lmax,
              "sweep: %d x %d cells need %zu bytes of LDS per workgroup (device limit %zu)", g.nx,
              g.ny, sweep_lds_bytes(g, nr, D, ch, elem_bytes), lmax);
  pl.D = D;
  pl.ch = ch;
  pl.groups = make_groups(dirs, D);
  pl.ngroups = (int)(pl.groups.size() / D);
  for (const auto& d : pl.groups) pl.qmask |= 1 << ((d.sx < 0 ? 1 : 0) + (d.sy < 0 ? 2 : 0));
  return pl;
}

size_t sweep_work_elems(const Geom& g, const SweepPlan& pl, bool want_phi) {
  return 20ull * g.nx * g.ny + (want_phi ? (size_t)pl.ngroups * g.ndof : 0);
}

template <typename T>
void sweep_enqueue(const Geom& g, const SweepPlan& pl, const SweepDir* dirs_dev,
                   const double* sigma_t, const T* src, const double* bc, T* psi, T* phi,
                   T* work, hipStream_t st) {
  RTE_REQUIRE(!psi || pl.D == 1, "sweep: psi needs a plan with one direction per workgroup");
  const long ncell = (long)g.nx * g.ny;
  T* dsrc = work;
  T* dsig = work + 16 * ncell;
  T* part = work + 20 * ncell;
  {
    const int tb = 256;
    hipLaunchKernelGGL((diag_layout_kernel<T>), dim3((ncell + tb - 1) / tb), dim3(tb), 0, st, g.nx,
                       g.ny, pl.qmask, sigma_t, src, dsrc, dsig);
    RTE_CHECK_HIP(hipGetLastError());
  }
  const size_t lds = sweep_lds_bytes(g, (pl.nt - 64) * pl.rpt, pl.D, pl.ch, sizeof(T));
  dim3 grid(pl.ngroups), block(pl.nt);
  const double shx = std::sqrt(g.hx), shy = std::sqrt(g.hy);
  T* pp = phi ? part : nullptr;
#define RTE_SWEEP_CASE(DD, NTB, RP)                                                                \
  hipLaunchKernelGGL((sweep_kernel<T, DD, NTB, RP>), grid, block, lds, st, g.nx, g.ny, g.mb, pl.ch, \
                     shx, shy, dirs_dev, dsrc, dsig, bc, psi, pp, g.ndof)
  // FP64 plans use D = 2 only with at most 576 threads (register budget)
#define RTE_SWEEP_D(NTB, RP)                                         \
  if (pl.D == 1) RTE_SWEEP_CASE(1, NTB, RP);                         \
  else if constexpr (sizeof(T) == 8 && (NTB > 576 || RP > 1)) bad(); \
  else if (pl.D == 2) RTE_SWEEP_CASE(2, NTB, RP);                    \
  else if constexpr (sizeof(T) == 8) bad();                          \
  else RTE_SWEEP_CASE(4, NTB, RP);
  auto bad = [&] { RTE_REQUIRE(false, "sweep: no kernel for D = %d, %d threads", pl.D, pl.nt); };
  if (pl.rpt == 2) {
    RTE_SWEEP_D(576, 2)
  } else if (pl.nt <= 320) {
    RTE_SWEEP_D(320, 1)
  } else if (pl.nt <= 576) {
    RTE_SWEEP_D(576, 1)
  } else {
    RTE_SWEEP_D(1024, 1)
  }
#undef RTE_SWEEP_D
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
  SweepPlan pl = make_sweep_plan(g, dirs, phi != nullptr, psi != nullptr, sizeof(T));
  DevBuf<SweepDir> ddirs(pl.groups.size());
  RTE_CHECK_HIP(hipMemcpy(ddirs.get(), pl.groups.data(), pl.groups.size() * sizeof(SweepDir),
                          hipMemcpyHostToDevice));
  DevBuf<T> work(sweep_work_elems(g, pl, phi != nullptr));
  sweep_enqueue<T>(g, pl, ddirs.get(), sigma_t, src, bc, psi, phi, work.get(), st);
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
