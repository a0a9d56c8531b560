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
// quadrant; staging wavefronts of the sweep workgroup move each step's inputs from
// there into LDS two steps ahead, so the compute wavefronts issue no global loads
// and never wait for their own stores (see sweep_kernel).  D directions of the same
// quadrant are solved per thread in lock step (ILP); their weighted sum is written
// once per cell when only the scalar flux is requested.
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

// 1/x for a positive normal x: the hardware reciprocal refined by Newton steps
// (r <- r + r (1 - x r)), two in FP64 and one in FP32, to working precision.
template <typename T>
__device__ __forceinline__ T recip(T x) {
  if constexpr (sizeof(T) == 8) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
  } else {
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
  }
}

// FP64: the x-coupling a L is folded into the diagonal coefficients of the first factor
// and the second factor is expanded into three scalars (54 FP64 operations per cell).
// FP32 keeps the factored form: the mixed-precision solves amplify the rounding of the
// FP32 sweeps through the diffusion correction, and the factored form's rounding is the
// one their accuracy was measured with.
template <typename T>
__device__ __forceinline__ void solve_cell(T sig, T a, T b, const T s[4], const T u[2],
                                           const T v[2], Cell<T>& out) {
  const T r3 = T(kSqrt3);
  const T ar3 = r3 * a, rb = r3 * b;
  const T R0 = s[0] + a * u[0] + b * v[0];
  const T R1 = s[1] - ar3 * u[0] + b * v[1];
  const T R2 = s[2] + a * u[1] - rb * v[0];
  const T R3 = s[3] - ar3 * u[1] - rb * v[1];
  const T d0 = sig * sig + T(4) * b * sig + T(6) * (b * b - a * a);
  const T d1 = T(2) * a * (sig + T(2) * (a + b));
  const T det = d0 * d0 + T(4) * d0 * d1 + T(6) * d1 * d1;
  const T inv = recip(det);  // det >= sigma^4 > 0 (sigma_t in [1e-30, 1e30])
  if constexpr (sizeof(T) == 8) {
    // (A + 3b) R_0 - sqrt3 b R_1 and sqrt3 b R_0 + (A + b) R_1 with A = sigma + a L
    const T y00 = (sig + (T(3) * b + a)) * R0 + ar3 * R1 - rb * R2;
    const T y01 = (sig + T(3) * (a + b)) * R1 - ar3 * R0 - rb * R3;
    const T y10 = rb * R0 + (sig + (a + b)) * R2 + ar3 * R3;
    const T y11 = rb * R1 + (sig + (b + T(3) * a)) * R3 - ar3 * R2;
    // e0 I + e1 L with e0 = (d0 + 4 d1)/det, e1 = -d1/det, expanded: f1 = e0 + e1,
    // f3 = e0 + 3 e1, g = sqrt3 e1
    const T f1 = (d0 + T(3) * d1) * inv, f3 = (d0 + d1) * inv, g = -r3 * d1 * inv;
    out.p[0] = f1 * y00 + g * y01;
    out.p[1] = f3 * y01 - g * y00;
    out.p[2] = f1 * y10 + g * y11;
    out.p[3] = f3 * y11 - g * y10;
  } else {
    // L applied to the two p-vectors (R0,R1) and (R2,R3)
    const T l00 = R0 + r3 * R1, l01 = T(3) * R1 - r3 * R0;
    const T l10 = R2 + r3 * R3, l11 = T(3) * R3 - r3 * R2;
    const T c3 = sig + T(3) * b, c1 = sig + b;
    const T y00 = c3 * R0 + a * l00 - rb * R2;
    const T y01 = c3 * R1 + a * l01 - rb * R3;
    const T y10 = rb * R0 + c1 * R2 + a * l10;
    const T y11 = rb * R1 + c1 * R3 + a * l11;
    const T e0 = (d0 + T(4) * d1) * inv, e1 = -d1 * inv;
    const T m0 = y00 + r3 * y01, m1 = T(3) * y01 - r3 * y00;
    const T n0 = y10 + r3 * y11, n1 = T(3) * y11 - r3 * y10;
    out.p[0] = e0 * y00 + e1 * m0;
    out.p[1] = e0 * y01 + e1 * m1;
    out.p[2] = e0 * y10 + e1 * n0;
    out.p[3] = e0 * y11 + e1 * n1;
  }
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

// Sigma_t of anti-diagonal t starts at sig_first(t) in its quadrant's array: the
// diagonal-major position advanced by (CPS - 1) t and rounded up to a multiple of
// CPS = 16 / sizeof(T) cells, so every diagonal's block starts on a 16-byte boundary
// (and blocks never overlap).  sig_stride is the per-quadrant length.
template <typename T>
__host__ __device__ __forceinline__ long sig_first(int t, int nx, int ny) {
  constexpr long CPS = 16 / sizeof(T);
  return (diag_first(t, nx, ny) + (CPS - 1) * t + CPS - 1) / CPS * CPS;
}
template <typename T>
__host__ __device__ __forceinline__ long sig_stride(int nx, int ny) {
  constexpr long CPS = 16 / sizeof(T);
  return ((long)nx * ny + (CPS - 1) * (long)(nx + ny) + 2 * CPS) / CPS * CPS;
}

// Elements of T in one 16-byte piece.
template <typename T>
constexpr int kPiece = 16 / (int)sizeof(T);

// Diagonal-major copies of the sweep inputs for the quadrants in qmask: the source
// moments (with the quadrant's reflections applied to the odd moments) and sigma_t,
// converted to T, and per step t the y-inflow trace of canonical row 0 (the boundary
// data of column t, zero for t >= nx) in a 16-byte piece.
// dsrc: [4][ncell][4], dsig: [4][sig_stride], dbnd: [4][nx + ny - 1][kPiece].
template <typename T>
__global__ __launch_bounds__(256) void diag_layout_kernel(int nx, int ny, int qmask,
                                                         const double* __restrict__ sigma_t,
                                                         const T* __restrict__ src,
                                                         const double* __restrict__ bc, int mb,
                                                         double shy, T* __restrict__ dsrc,
                                                         T* __restrict__ dsig,
                                                         T* __restrict__ dbnd) {
  // One workgroup per anti-diagonal t of quadrant q = blockIdx.y: the diagonal's cells are
  // gathered from the row-major arrays and stored as one contiguous run (the XCD-contiguous
  // order of the diagonals lets neighbouring diagonals, which read the other cells of the
  // same lines, share an L2).
  const int q = blockIdx.y;
  if (!((qmask >> q) & 1)) return;
  const int nsteps = nx + ny - 1;
  const int t = (int)xcd_block(blockIdx.x, gridDim.x);
  const int sx = (q & 1) ? -1 : 1, sy = (q & 2) ? -1 : 1;
  const long ncell = (long)nx * ny;
  if (threadIdx.x == 0) {  // the y-inflow piece of canonical row 0
    T v[kPiece<T>];
#pragma unroll
    for (int i = 0; i < kPiece<T>; ++i) v[i] = T(0);
    if (bc && t < nx) {
      const int col = sx > 0 ? t : nx - 1 - t;
      const int yside = sy > 0 ? 2 : 3;
      v[0] = T(shy * bc[((long)yside * mb + col) * 2 + 0]);
      v[1] = T(shy * bc[((long)yside * mb + col) * 2 + 1] * sx);
    }
#pragma unroll
    for (int i = 0; i < kPiece<T>; ++i) dbnd[((long)q * nsteps + t) * kPiece<T> + i] = v[i];
  }
  const int lo = t >= nx ? t - nx + 1 : 0, hi = t < ny ? t : ny - 1;
  const long k0 = q * ncell + diag_first(t, nx, ny) - lo;
  const long s0 = q * sig_stride<T>(nx, ny) + sig_first<T>(t, nx, ny) - lo;
  for (int r = lo + (int)threadIdx.x; r <= hi; r += blockDim.x) {
    const int ap = t - r;
    const int acol = sx > 0 ? ap : nx - 1 - ap, brow = sy > 0 ? r : ny - 1 - r;
    const long c = (long)brow * nx + acol;
    if (src) {  // src == null: per-direction sources, laid out by diag_src_dirs_kernel
      const Vec4<T> s4 = load4(src + 4 * c);
      const T v[4] = {s4.v[0], T(sx) * s4.v[1], T(sy) * s4.v[2], T(sx * sy) * s4.v[3]};
      store4(dsrc + 4 * (k0 + r), v);
    }
    dsig[s0 + r] = T(sigma_t[c]);
  }
}

// Per-direction sources: slot s's source (row s of src, [ny][nx][4]) in the diagonal-major
// order of its own quadrant's canonical frame, with the odd moments' signs of that frame.
// The quadrant of each slot (q = (sx < 0) + 2 (sy < 0)) travels in the kernel arguments.
constexpr int kSlotsMax = 2048;
struct SlotQuads {
  int8_t q[kSlotsMax];
};

template <typename T>
__global__ void diag_src_dirs_kernel(int nx, int ny, int slot0, SlotQuads sq,
                                     const T* __restrict__ src, T* __restrict__ dsrc) {
  const long ncell = (long)nx * ny;
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int s = slot0 + (int)blockIdx.y;
  const int q = sq.q[blockIdx.y];
  if (q < 0) return;  // a slot no direction writes
  const int sx = (q & 1) ? -1 : 1, sy = (q & 2) ? -1 : 1;
  const int acol = (int)(c % nx), brow = (int)(c / nx);
  const int r = sy > 0 ? brow : ny - 1 - brow;
  const int ap = sx > 0 ? acol : nx - 1 - acol;
  const int t = r + ap;
  const int lo = t >= nx ? t - nx + 1 : 0;
  const long k = diag_first(t, nx, ny) + r - lo;
  const Vec4<T> s4 = load4(src + (long)s * 4 * ncell + 4 * c);
  const T v[4] = {s4.v[0], T(sx) * s4.v[1], T(sy) * s4.v[2], T(sx * sy) * s4.v[3]};
  store4(dsrc + (long)s * 4 * ncell + 4 * k, v);
}

// Rows of one step that a staging wavefront carries at most (plans may use fewer, with
// more staging wavefronts, when the issue of the copies bounds the step).
constexpr int kStageRows = 256;
// Input slots in LDS: the staging wavefronts fill step t + 2 while step t is solved.
// FP64 workgroups of two directions with two rows per thread (up to 1024 rows) have the
// LDS for two slots only: they fill step t + 1 while step t is solved and wait for it
// before the barrier that ends step t (such a step is long enough to cover the copy).
constexpr int kInSlots = 3;
__host__ __device__ constexpr int in_slots(size_t eb, int D, int RPT) {
  return eb == 8 && D == 2 && RPT == 2 ? 2 : kInSlots;
}

// s_waitcnt immediate for vmcnt(n), n <= 63 (the 6-bit counter: bits 3:0 and 15:14),
// with expcnt and lgkmcnt not waited for.
constexpr int vmcnt_imm(int n) { return 0xF70 | (n & 15) | ((n >> 4) << 14); }

// Output write-back geometry for element type T: a row's results leave in aligned
// chunks of 128 bytes (kChunkCells cells), 16 bytes per lane, 8 rows per store
// instruction; the LDS ring keeps the last kRingSlots steps.
template <typename T>
struct WriteBack {
  static constexpr int kCellBytes = 4 * sizeof(T);
  static constexpr int kChunkCells = 128 / kCellBytes;  // 4 (FP64) or 8 (FP32)
  static constexpr int kLanesPerCell = kCellBytes / 16;  // 2 or 1
  static constexpr int kRingSlots = kChunkCells + 1;
};
// Rows whose chunks one write-back wavefront stores.
constexpr int kWbRows = 64;

// Aligned groups of cells for direct stores.  A row is swept one cell per step (towards
// +x, or towards -x when sx < 0); the cells of the flat [ny][nx] numbering form aligned
// groups of GC = 128 bytes / cell size (4 cells in FP64, 8 in FP32: one cache line).  A
// row's cells of one group are kept in registers until the row leaves the group (at the
// group's end or the row's end) and then stored together, so that whole lines leave
// the cache instead of 16- or 32-byte pieces (which cost a full 64-byte memory write
// each).
template <typename T, int NC = 128 / (4 * (int)sizeof(T))>
struct RowGroup {
  static constexpr int GC = NC;  // cells per group (a power of two)
  T buf[GC - 1][4];  // the kept cells, newest last (a shift register: static indices only)
  int k = 0;         // how many are kept
};

// Takes the moments v of cell c (canonical column ap) of a row swept in direction sx;
// when base2 is given, the run is also stored there scaled by w2 (psi and its weighted
// scalar-flux share from one buffer).
template <typename T, int NC>
__device__ __forceinline__ void put_grouped(T* base, long c, int ap, int nx, int sx, const T v[4],
                                            RowGroup<T, NC>& g, T* base2 = nullptr, T w2 = T(0)) {
  constexpr int GC = NC;
  const int pos = (int)(c & (GC - 1));  // position in the group (base is 256-byte aligned)
  const bool last = ap == nx - 1 || (sx > 0 ? pos == GC - 1 : pos == 0);
  if (!last) {
#pragma unroll
    for (int i = 0; i + 1 < GC - 1; ++i)
#pragma unroll
      for (int m = 0; m < 4; ++m) g.buf[i][m] = g.buf[i + 1][m];
#pragma unroll
    for (int m = 0; m < 4; ++m) g.buf[GC - 2][m] = v[m];
    ++g.k;
    return;
  }
  // buf[i] (i >= GC - 1 - k) holds cell c - (GC - 1 - i) towards +x, c + (GC - 1 - i)
  // towards -x: with c itself one contiguous run of k + 1 cells
  const int k = g.k;
  auto put = [&](long cell, const T x[4]) {
    store4(base + 4 * cell, x);
    if (base2) {
      T wx[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) wx[m] = w2 * x[m];
      store4(base2 + 4 * cell, wx);
    }
  };
  put(c, v);
#pragma unroll
  for (int i = 0; i < GC - 1; ++i)
    if (i >= GC - 1 - k) put(c + (long)sx * (i - (GC - 1)), g.buf[i]);
  g.k = 0;
}

typedef __attribute__((address_space(3))) void lds_void;

// One workgroup sweeps D directions (dirs[blockIdx.x*D + d]) of one quadrant.
// psi: [slots][ndof] or null; part: [gridDim.x][ndof] weighted partial sums or null
// (not both).  dsrc/dsig: the diagonal-major inputs.
//
// Roles.  The first nc threads compute; compute thread j owns the canonical rows
// j + k nc, k < RPT (both on the current anti-diagonal, so they are independent
// work).  The next wavefronts stage inputs, SR rows each, with direct global-to-LDS
// loads.  With the LDS output ring, the last wavefronts (one per kWbRows rows) store
// the results from the ring.  Compute wavefronts read their inputs from LDS and issue
// only LDS writes with the ring, otherwise global stores, which they never wait for.
//
// Per step t: the compute threads solve the cells of canonical column t - r, taking
// the source and sigma_t of step t from LDS input slot t mod 3 and the y-inflow trace
// from row r - 1 of step t - 1 (double-buffered LDS, one barrier per step); the
// x-inflow trace stays in registers.  Meanwhile the staging wavefronts copy the cells
// of step t + 2 into slot (t + 2) mod 3 (last read in step t - 1) and, before the
// barrier that ends step t, wait only for the copies of step t + 1 (issued one step
// earlier): vector memory counts complete in issue order, so waiting until no more
// than this step's copies are outstanding suffices, and a copy has a whole step to land.
// A staging wavefront issues the same number of copies in every step in which it has
// cells (none in the others), so that the counts waited for are constants of the kernel
// and the staging loop keeps no per-step tallies.
//
// Output mode OUT (compile time; bit 4: one source per direction, from row `slot` of
// the per-direction layouts, for psi plans of one direction per workgroup): bit 0 the
// LDS ring, bit 1 psi, bit 2 the weighted
// partial sums of the scalar flux (psi and the partial sums together only for D = 1),
// bit 3 large plans without the ring: psi leaves in line-sized groups of a row's cells,
// partial sums without psi in the diagonal-major order of the canonical frame (one
// contiguous run per step); small plans store each cell, which keeps their
// latency-bound step short.
// With the ring, step t leaves its results in LDS ring slot t mod kRingSlots
// (per direction for psi, or the weighted sum over the group's directions for the
// scalar flux).  A row's cells are grouped into aligned chunks of kChunkCells
// physical columns; while step t is solved the write-back wavefronts store, from the
// ring, the chunks whose last cell was solved at step t - 1 (one row in kChunkCells,
// plus the short end chunk of one row when nx is not a multiple of kChunkCells and the
// sweep runs towards +x), so every store instruction writes whole 128-byte lines and
// the compute wavefronts' step does not wait for them.  Without the ring (LDS too
// small, or plans too small for the store bandwidth to matter) each thread stores its
// cell.
template <typename T, int D, int NTB, int RPT, int SR, int OUT>
__global__ __launch_bounds__(NTB) void sweep_kernel(
    int nx, int ny, int mb, int nc, double shx, double shy,
    const SweepDir* __restrict__ dirs, const T* __restrict__ dsrc_all,
    const T* __restrict__ dsig_all, const T* __restrict__ dbnd_all, const double* __restrict__ bc,
    T* __restrict__ psi, T* __restrict__ part, long ndof) {
  using WB = WriteBack<T>;
  constexpr bool RING = (OUT & 1) != 0, PSI = (OUT & 2) != 0, PP = (OUT & 4) != 0;
  constexpr bool GRP = (OUT & 8) != 0;  // direct stores in line-sized groups (put_grouped)
  constexpr bool DSRC = (OUT & 16) != 0;  // one source per direction (D == 1, psi only)
  static_assert(!DSRC || (D == 1 && !PP), "per-direction sources: one direction, psi only");
  static_assert(PSI || PP, "no output");
  static_assert(!(PSI && PP) || D == 1, "psi with the scalar flux needs one direction per workgroup");
  constexpr int CW = WB::kChunkCells, NS = WB::kRingSlots, LPC = WB::kLanesPerCell;
  constexpr int CPC = 4 * (int)sizeof(T) / 16;  // 16-byte pieces per source cell
  constexpr int CPS = 16 / (int)sizeof(T);      // sigma_t cells per 16-byte piece
  extern __shared__ unsigned char smem_raw[];
  const int tid = threadIdx.x;
  const int nr = nc * RPT;                    // padded rows
  const int nrs = nr + 2 * CPS;               // sigma_t slot length
  constexpr int RD = PSI ? D : 1;             // ring entries per row and step
  constexpr int BS = kPiece<T>;                // elements of a 16-byte piece
  T* vbuf = reinterpret_cast<T*>(smem_raw);   // [2][nr][D][2] y-inflow traces by row
  constexpr int S = in_slots(sizeof(T), D, RPT);
  T* in_src = vbuf + 4L * nr * D;             // [S][nr][4] source moments of the step
  T* in_sig = in_src + 4L * S * nr;           // [S][nrs] sigma_t of the step (shifted)
  T* in_bnd = in_sig + (long)S * nrs;         // [S][BS] y-inflow of canonical row 0
                                              // + [BS] pad (dummy copies)
  T* ring = in_bnd + (S + 1) * BS;            // [NS][nr][RD][4] outputs by step and row
  const SweepDir* grp = dirs + (long)blockIdx.x * D;
  const int sx = grp[0].sx, sy = grp[0].sy;
  const T fx = T(sx), fy = T(sy), fxy = T(sx * sy);
  const long ncell = (long)nx * ny;
  const int q = (sx < 0 ? 1 : 0) + (sy < 0 ? 2 : 0);
  const int nsteps = nx + ny - 1;
  const int nst = (nr + SR - 1) / SR;  // staging wavefronts
  if (RING && tid >= nc + 64 * nst) {
    // ---------------------------------------------- write-back wavefronts
    // The rows are taken in blocks of kWbRows; write-back wavefront k stores the chunks
    // of blocks per k .. per k + per - 1 (per = 1 unless the thread budget of the kernel
    // left fewer wavefronts than blocks): 8 lanes (16 bytes each) per row, 8 rows per
    // store instruction; instruction i of a block covers rows b + CW (jrow + 8 i) +
    // rho(t), rho(t) the residue (mod CW) of the rows whose last cell closed an aligned
    // chunk at step t - 1.  The flat cell index of a lane's cell is affine in its row and
    // the step, and the ring slot of the cell depends on the step and the lane's cell only.
    constexpr int NI = kWbRows / CW / 8;  // store instructions per block and step
    const int lane = tid & 63;
    const int nwb = (int)(blockDim.x >> 6) - ((nc >> 6) + nst);
    const int nblk = (nr + kWbRows - 1) / kWbRows;
    const int per = (nblk + nwb - 1) / nwb;
    const int wb0 = ((tid - nc - 64 * nst) >> 6) * per * kWbRows;
    const int wb1 = wb0 + per * kWbRows;  // rows wb0 .. wb1 - 1
    const int jrow = lane >> 3;
    const int cc = (lane & 7) / LPC, half = lane % LPC;  // cell within the chunk, piece
    T* pdst = PSI && psi && grp[0].slot >= 0 ? psi + (long)grp[0].slot * ndof : nullptr;
    T* pp = part ? part + (long)blockIdx.x * ndof : nullptr;
    const T w0 = T(grp[0].w);
    const long Cr = (long)sy * nx - sx;
    const long C0 = (sy > 0 ? 0 : (long)(ny - 1) * nx) + (sx > 0 ? -CW : nx);
    const int roff = sx > 0 ? 1 + cc : NS - 1 - cc;  // ring slot = (t + roff) mod NS
    const int eoff = half * (16 / (int)sizeof(T));
    // One ring entry per row and step: psi of the one direction (psi plans have D = 1),
    // or the weighted sum over the group's directions.
    static_assert(!RING || !PSI || D == 1, "psi write-back with one direction per workgroup");
    using V = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
    // the ring piece of row r in slot `slot`
    auto ring_piece = [&](int slot, int r) {
      return *reinterpret_cast<const V*>(ring + ((long)slot * nr + r) * 4 + eoff);
    };
    // The ring holds canonical-frame moments: the odd-in-x ones take the sign sx and the
    // odd-in-y ones sy here (FP64: a lane's piece is (p0, p1) or (p2, p3)).
    const T sg0 = LPC == 2 && half ? fy : T(1), sg1 = LPC == 2 && half ? fxy : fx;
    const T wg0 = D == 1 ? w0 * sg0 : sg0, wg1 = D == 1 ? w0 * sg1 : sg1;
    // psi (and, for one direction, the weighted partial sum) of the cell c
    auto put_piece = [&](long c, const V& v) {
      if constexpr (sizeof(T) == 8) {
        if (PSI && pdst)
          *reinterpret_cast<double2*>(pdst + 4 * c + eoff) = make_double2(sg0 * v.x, sg1 * v.y);
        if constexpr (PP)
          *reinterpret_cast<double2*>(pp + 4 * c + eoff) = make_double2(wg0 * v.x, wg1 * v.y);
      } else {
        if (PSI && pdst)
          *reinterpret_cast<float4*>(pdst + 4 * c) = make_float4(v.x, fx * v.y, fy * v.z, fxy * v.w);
        if constexpr (PP) {
          const float wgt = D == 1 ? w0 : 1.0f;
          *reinterpret_cast<float4*>(pp + 4 * c) =
              make_float4(wgt * v.x, wgt * fx * v.y, wgt * fy * v.z, wgt * fxy * v.w);
        }
      }
    };
    const int endc = nx % CW;  // cells in the short end chunk of a row (0: none)
    // Chunks closed by the cells solved at step t - 1 (st = t mod NS).
    auto write_back = [&](int t, int st) {
      const int rho = (sx > 0 ? t : t - nx) & (CW - 1);
      const long cu = Cr * rho + (long)sx * t;
      int slot = st + roff;
      slot = slot >= NS ? slot - NS : slot;
      for (int b = wb0; b < wb1; b += kWbRows) {
        // all ring reads of the block first (rows clamped into the ring), then the
        // stores, so that one LDS round trip serves them
        V v[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i) {
          const int r = b + CW * (jrow + 8 * i) + rho;
          v[i] = ring_piece(slot, r < nr ? r : nr - 1);
        }
#pragma unroll
        for (int i = 0; i < NI; ++i) {
          const int r = b + CW * (jrow + 8 * i) + rho;
          const int apl = t - 1 - r;  // canonical column solved at step t - 1
          const bool ok = r < ny && (unsigned)apl < (unsigned)nx &&
                          (sx > 0 || nx - 1 - apl + cc < nx);
          if (ok) put_piece(C0 + Cr * (r - rho) + cc + cu, v[i]);
        }
      }
      // the short end chunk of row t - nx (towards +x only)
      if (sx > 0 && endc != 0) {
        const int r = t - nx;
        if (r >= wb0 && r < wb1 && r < ny && jrow == 0 && cc < endc) {
          const int col = nx - endc + cc;
          const int brow = sy > 0 ? r : ny - 1 - r;
          put_piece((long)brow * nx + col, ring_piece((r + col) % NS, r));
        }
      }
    };
    // Step t's chunks close at step t - 1 and leave while step t is solved: the ring
    // slot written in step t is none of the CW read here, and the reads have landed
    // before this wavefront reaches the barrier that ends step t.
    __syncthreads();  // step 0 staged
    int ns = 0;       // t mod NS
    for (int t = 0; t < nsteps; ++t) {
      if (t > 0) write_back(t, ns);
      __syncthreads();
      ns = ns + 1 == NS ? 0 : ns + 1;
    }
    write_back(nsteps, ns);  // chunks closed by the last step
    return;
  }
  if (tid >= nc) {
    // ------------------------------------------------ staging wavefronts
    // Issue priority: staging wavefronts first, then compute, then write-back.  A copy
    // issued late lands late and holds up the barrier that waits for it; giving the
    // staging wavefronts the top priority took the full-angle sweep from 473 to 458 us
    // (FP64) and from 318 to 285 us (FP32).
    __builtin_amdgcn_s_setprio(3);
    // Step t's cells are rows lo..hi of anti-diagonal t, contiguous in the
    // diagonal-major arrays.  Staging wavefront sw copies rows lo + SR sw ..
    // lo + SR sw + SR - 1 (16 bytes per lane, lanes past the step masked off): the
    // source to in_src rows lo.., sigma_t to in_sig positions sh(t) + lo.., where
    // sh(t) = -lo mod CPS keeps the copy 16-byte aligned on both sides.
    const int lane = tid & 63;
    const int sw = (tid - nc) >> 6;
    const int c0 = sw * SR;  // first cell of this wavefront within a step
    // the quadrant's layout of the shared source, or this direction's own source
    const long src_row = DSRC ? (long)grp[0].slot : (long)q;
    const float4* src16 = reinterpret_cast<const float4*>(dsrc_all + 4 * src_row * ncell);
    const float4* sig16 = reinterpret_cast<const float4*>(dsig_all + q * sig_stride<T>(nx, ny));
    const float4* bnd16 = reinterpret_cast<const float4*>(dbnd_all) + (long)q * nsteps;
    float4* pad = reinterpret_cast<float4*>(in_bnd + S * BS);
    // A wavefront with cells in a step issues the same number of copies (K, and one
    // more, the y-inflow piece of row 0, in wavefront 0, which always has cells), so
    // that the waits are constants: a copy with no cells left for it moves one 16-byte
    // piece (lane 0, from a valid address) into the LDS pad, which nothing reads.  A
    // wavefront without cells in step t + 2 issues nothing and waits for all its copies.
    constexpr int NIS = SR * CPC / 64;         // source copies
    constexpr int NIG = (SR / CPS + 63) / 64;  // sigma_t copies
    constexpr int K = NIS + NIG;
    static_assert(K + 1 <= 63, "outstanding copies exceed the vmcnt range");
    const bool w0 = sw == 0;
    // after the copies of step t + 2 (any: whether it had cells for this wavefront), those
    // of step t + 1 have landed
    // (two slots: every copy issued so far has landed)
    auto wait_next = [&](bool any) {
      if (S == 2 || !any) __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
      else if (w0) __builtin_amdgcn_s_waitcnt(vmcnt_imm(K + 1));
      else __builtin_amdgcn_s_waitcnt(vmcnt_imm(K));
    };
    // copies of step t (first row lo, first diagonal-major position df) into slot sl;
    // false if the step has no cells for this wavefront (then nothing is issued)
    auto stage = [&](int t, int lo, long df, int sl) {
      const int hi = t < ny ? t : ny - 1;
      const int nce = hi - lo + 1 - c0;  // cells left for this wavefront
      if (nce <= 0) return false;
      const int ncw = nce < SR ? nce : SR;
      const float4* gs = src16 + (df + c0) * CPC;
      float4* ls = reinterpret_cast<float4*>(in_src) + ((long)sl * nr + lo + c0) * CPC;
#pragma unroll
      for (int i = 0; i < NIS; ++i) {
        const bool mine = 64 * i + lane < ncw * CPC;
        if (mine || lane == 0)
          __builtin_amdgcn_global_load_lds((const void*)(mine ? gs + 64 * i + lane : bnd16),
                                           (lds_void*)(64 * i < ncw * CPC ? ls + 64 * i : pad),
                                           16, 0, 0);
      }
      // sigma_t: ceil(ncw / CPS) pieces, at sig_first(t) (diagonal-major position
      // advanced by (CPS - 1) t, rounded up to a multiple of CPS)
      const long sf = (df + (CPS - 1) * (long)t + CPS - 1) / CPS * CPS;
      const int sh = (-lo) & (CPS - 1);
      const float4* gg = sig16 + (sf + c0) / CPS;
      float4* lg = reinterpret_cast<float4*>(in_sig + (long)sl * nrs + sh + lo + c0);
      const int npg = (ncw + CPS - 1) / CPS;
#pragma unroll
      for (int i = 0; i < NIG; ++i) {
        const bool mine = 64 * i + lane < npg;
        if (mine || lane == 0)
          __builtin_amdgcn_global_load_lds((const void*)(mine ? gg + 64 * i + lane : bnd16),
                                           (lds_void*)(64 * i < npg ? lg + 64 * i : pad), 16, 0,
                                           0);
      }
      if (w0 && lane == 0)  // the y-inflow piece of row 0
        __builtin_amdgcn_global_load_lds((const void*)(bnd16 + t),
                                         (lds_void*)(in_bnd + BS * sl), 16, 0, 0);
      return true;
    };
    // (lo, df) of the next step to stage, advanced one step at a time
    int lo = 0;
    long df = 0;
    auto advance = [&](int t) {
      df += (t < ny ? t : ny - 1) - lo + 1;
      lo += t + 1 >= nx ? 1 : 0;
    };
    // Plain barriers: the copies are waited for explicitly.  AHEAD = S - 1 steps are
    // staged before the loop; step t + AHEAD is staged during step t.
    constexpr int AHEAD = S - 1;
    stage(0, lo, df, 0);
    advance(0);
    bool any = false;
    if (AHEAD == 2 && nsteps > 1) {
      any = stage(1, lo, df, 1);
      advance(1);
    }
    wait_next(any);                // step 0 landed
    __builtin_amdgcn_s_barrier();  // step 0 staged
    int sla = AHEAD;               // (t + AHEAD) mod S
    for (int t = 0; t < nsteps; ++t) {
      any = false;
      if (t + AHEAD < nsteps) {
        any = stage(t + AHEAD, lo, df, sla);
        advance(t + AHEAD);
      }
      wait_next(any);                // copies of step t + 1 landed
      __builtin_amdgcn_s_barrier();  // end of step t
      sla = sla == S - 1 ? 0 : sla + 1;
    }
    __builtin_amdgcn_s_waitcnt(0);
    return;
  }
  // -------------------------------------------------- compute wavefronts
  __builtin_amdgcn_s_setprio(2);  // below the staging wavefronts, above the write-back
  T a[D], b[D], w[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    a[d] = T(grp[d].a);
    b[d] = T(grp[d].b);
    w[d] = T(grp[d].w);
  }
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
  // output bases per direction (null: padding direction or no psi); without the ring
  // each thread stores its cells
  T* pdst[D];
#pragma unroll
  for (int d = 0; d < D; ++d)
    pdst[d] = !RING && psi && grp[d].slot >= 0 ? psi + (long)grp[d].slot * ndof : nullptr;
  T* pp = !RING && part ? part + (long)blockIdx.x * ndof : nullptr;
  const T w0 = T(grp[0].w);
  // Direct stores leave in aligned line-sized groups of a row's cells (put_grouped).
  // With two psi directions per workgroup (FP64, two rows per thread) the register budget
  // holds groups of two cells (64 bytes, the memory's write granule) per row and direction.
  constexpr int QGC = D > 1 ? 64 / (4 * (int)sizeof(T)) : 128 / (4 * (int)sizeof(T));
  RowGroup<T, QGC> qgrp[RPT][RD];  // psi per direction ...
  RowGroup<T> pgrp[RPT];           // ... and the weighted scalar-flux sum
  (void)qgrp;
  (void)pgrp;
  __syncthreads();  // step 0 staged
  int ns = 0;       // t mod NS
  int si = 0;       // t mod S: input slot
  for (int t = 0; t < nsteps; ++t) {
    const int sl = t & 1;
    const int lo = t >= nx ? t - nx + 1 : 0;
    const T* sigs = in_sig + (long)si * nrs + ((-lo) & (CPS - 1));
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int r = row[k];
      const int ap = t - r;
      if (row_ok[k] && ap >= 0 && ap < nx) {
        const T* rd = r == 0 ? in_bnd + BS * si : vbuf + ((long)(sl ^ 1) * nr + (r - 1)) * D * 2;
        const int rstride = r == 0 ? 0 : 2;
        T* wr = vbuf + ((long)sl * nr + r) * D * 2;
        const Vec4<T> s4 = load4(in_src + ((long)si * nr + r) * 4);
        const T sig = sigs[r];
        T* rg = ring + ((long)ns * nr + r) * RD * 4;
        T acc[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const T v[2] = {rd[rstride * d], rd[rstride * d + 1]};
          Cell<T> cell;
          solve_cell<T>(sig, a[d], b[d], s4.v, u[k][d], v, cell);
          u[k][d][0] = cell.uo[0];
          u[k][d][1] = cell.uo[1];
          wr[2 * d] = cell.vo[0];
          wr[2 * d + 1] = cell.vo[1];
          // back to the physical frame's signs of the odd moments; with the ring the
          // write-back wavefronts apply them
          T ph[4] = {cell.p[0], cell.p[1], cell.p[2], cell.p[3]};
          if constexpr (!RING) {
            ph[1] *= fx;
            ph[2] *= fy;
            ph[3] *= fxy;
          }
          if constexpr (PSI) {
            if constexpr (RING) {
              store4(rg + 4 * d, ph);
            } else {
              const int brow = sy > 0 ? r : ny - 1 - r;
              const long c = (long)brow * nx + (sx > 0 ? ap : nx - 1 - ap);
              // with the partial sums (D == 1 here) both leave from the one psi buffer
              if constexpr (GRP) {
                if (pdst[d]) put_grouped(pdst[d], c, ap, nx, sx, ph, qgrp[k][d], PP ? pp : nullptr, w0);
              } else {
                if (pdst[d]) store4(pdst[d] + 4 * c, ph);
                if constexpr (PP) {  // D == 1 here
                  T wv[4];
#pragma unroll
                  for (int m = 0; m < 4; ++m) wv[m] = w0 * ph[m];
                  store4(pp + 4 * c, wv);
                }
              }
            }
          } else {
#pragma unroll
            for (int m = 0; m < 4; ++m) acc[m] = D == 1 ? ph[m] : acc[m] + w[d] * ph[m];
          }
        }
        if constexpr (!PSI) {
          if constexpr (RING) {
            store4(rg, acc);
          } else {
            const int brow = sy > 0 ? r : ny - 1 - r;
            T wv[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) wv[m] = D == 1 ? w0 * acc[m] : acc[m];
            const long c = (long)brow * nx + (sx > 0 ? ap : nx - 1 - ap);
            // large plans: the partial sums in diagonal-major order, so that each step's
            // cells leave as one contiguous run (reduce_quadrants_kernel reorders them)
            if constexpr (GRP) store4(pp + 4 * (diag_first(t, nx, ny) + r - lo), wv);
            else store4(pp + 4 * c, wv);
          }
        }
      }
    }
    __syncthreads();
    ns = ns + 1 == NS ? 0 : ns + 1;
    si = si + 1 == S ? 0 : si + 1;
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

// Diagonal-major partial sums (large phi-only plans): the groups of one quadrant, in group
// order, summed into the slot of its first group g[0] (in place: each element is read and
// written by one thread).  The list travels in the kernel arguments, up to kListMax groups
// per launch; acc = 1 continues the sum already in the first group's slot.
constexpr int kListMax = 1024;
struct GroupList {
  int n, acc;
  int16_t g[kListMax];
};

template <typename T>
__global__ void reduce_quadrant_kernel(T* __restrict__ part, long ndof, int g0, GroupList L) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ndof) return;
  T s = L.acc ? part[(long)g0 * ndof + i] : T(0);
  int k = 0;
  for (; k + 8 <= L.n; k += 8) {  // eight loads in flight, added in list order
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(long)L.g[k + u] * ndof + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; k < L.n; ++k) s += part[(long)L.g[k] * ndof + i];
  part[(long)g0 * ndof + i] = s;
}

// phi of cell (a, b) = sum over the swept quadrants q (in order) of the quadrant sum at the
// cell's diagonal-major position in q's canonical frame.
template <typename T>
__global__ void gather_quadrants_kernel(const T* __restrict__ part, long ndof, int nx, int ny,
                                        int g00, int g01, int g02, int g03, T* __restrict__ phi) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (long)nx * ny) return;
  const int a = (int)(c % nx), b = (int)(c / nx);
  T s[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int g0 = q == 0 ? g00 : q == 1 ? g01 : q == 2 ? g02 : g03;
    if (g0 < 0) continue;
    const int ap = (q & 1) ? nx - 1 - a : a, r = (q & 2) ? ny - 1 - b : b;
    const int t = ap + r;
    const int lo = t >= nx ? t - nx + 1 : 0;
    const Vec4<T> v = load4(part + (long)g0 * ndof + 4 * (diag_first(t, nx, ny) + r - lo));
#pragma unroll
    for (int m = 0; m < 4; ++m) s[m] += v.v[m];
  }
  store4(phi + 4 * c, s);
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

// vbuf [2][nr][D][2] + in_src [S][nr][4] + in_sig [S][nr + 2 CPS] + in_bnd [S + 1][CPS]
// + ring [kRingSlots][nr][RD][4] (with the ring; RD = D for psi, 1 for the scalar
// flux), nr = padded rows, S = in_slots(eb, D, rows per thread)
static size_t sweep_lds_bytes(int nr, int D, bool psi, bool ring, size_t eb, int rpt) {
  const size_t S = in_slots(eb, D, rpt);
  const size_t slots = ring ? (eb == 8 ? WriteBack<double>::kRingSlots : WriteBack<float>::kRingSlots) : 0;
  const size_t cps = 16 / eb;
  return (4ull * nr * D + 4ull * S * nr + S * (nr + 2 * cps) + (S + 1) * cps +
          4ull * slots * nr * (psi ? D : 1)) * eb;
}

// LDS bytes one workgroup may use on the current device
static size_t max_lds_per_block() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
    return 65536;
  return (size_t)v;
}

// compute threads, rows per compute thread and staging wavefronts for ny rows: a
// staging wavefront carries srows rows, at least `rows` (64 or 128 when requested: 64
// only while nc <= 256, 128 while nc <= 640) and otherwise 256, so that the workgroup
// fits the kernels' thread counts (960, or 768 with two rows per thread)
static void sweep_threads(int ny, int rows, int& nc, int& rpt, int& nst, int& srows) {
  rpt = ny <= 768 ? 1 : 2;
  nc = ((ny + rpt - 1) / rpt + 63) / 64 * 64;
  srows = kStageRows;
  if (rows < kStageRows && rpt == 1)
    srows = rows <= 64 && nc <= 256 ? 64 : (nc <= 640 ? 128 : kStageRows);
  nst = (nc * rpt + srows - 1) / srows;
}

// Accelerator complex dies (XCDs) of the device, each with its own L2
constexpr int kXcds = 8;

// LDS per workgroup that still lets two workgroups share a compute unit (160 KB)
constexpr size_t kLdsTwoPerCU = 80 * 1024;

SweepPlan make_sweep_plan(const Geom& g, const std::vector<SweepDir>& dirs, bool want_phi,
                          bool want_psi, size_t elem_bytes, bool per_dir_src) {
  RTE_REQUIRE(!per_dir_src || (want_psi && !want_phi),
              "sweep: per-direction sources are for psi plans without the scalar flux");
  RTE_REQUIRE(g.ny >= 1 && g.ny <= 1024, "sweep: ny = %d outside [1, 1024]", g.ny);
  RTE_REQUIRE(g.nx >= 1 && g.nx <= 1 << 20, "sweep: nx = %d outside [1, 2^20]", g.nx);
  RTE_REQUIRE(!dirs.empty(), "sweep: no directions");
  SweepPlan pl;
  // Staging wavefronts: the issue of a step's copies bounds the step when few workgroups
  // run (small plans: 64 rows per staging wavefront) and for psi (128 rows; at 256 rows
  // and 512 ordinates FP64 measured 3 % faster than 64 and 7 % faster than 256, FP32 1 %
  // faster than 256); else 256 rows.
  const bool small = dirs.size() < 64;
  int nc, rpt, nst, srows;
  sweep_threads(g.ny, small ? 64 : (want_psi ? 128 : kStageRows), nc, rpt,
                nst, srows);
  pl.nc = nc;
  pl.nt = nc + 64 * nst;  // write-back wavefronts are added below with the ring
  pl.rpt = rpt;
  pl.srows = srows;
  const int nr = nc * rpt;
  const size_t lmax = max_lds_per_block();
  const size_t lcap = std::min(lmax, kLdsTwoPerCU);
  // Directions per workgroup (scalar flux only): enough workgroups to cover the chip
  // first; then D > 1 shares the staged inputs and the partial sums among directions.
  // D is bounded by the register budget (FP64: 2, with one row per thread only up to
  // 576 threads; FP32: 4) and by LDS (FP64 with two rows per thread: two input slots).
  // With psi, one direction per workgroup (measured faster: two workgroups share a
  // compute unit), except FP64 with two rows per thread, where one workgroup fills a
  // compute unit's LDS and two directions halve the rounds.
  const int dmax = per_dir_src ? 1
                   : want_psi ? (elem_bytes == 8 && rpt == 2 && !want_phi ? 2 : 1)
                              : elem_bytes == 8 ? ((pl.nt <= 576 || rpt == 2) ? 2 : 1) : 4;
  int D = 1;
  while (D < dmax && dirs.size() / (2 * D) >= 256 &&
         sweep_lds_bytes(nr, 2 * D, want_psi, rpt == 1, elem_bytes, rpt) <= lmax)
    D *= 2;
  // the output ring if it fits and the plan is large enough for the store bandwidth to
  // matter (else each thread stores its cells directly, which is shorter per step)
  // Write-back wavefronts (with the ring): one per kWbRows rows, fewer (each storing
  // several blocks of rows) where the kernel's thread budget (two rows per thread: 768;
  // FP64 with D = 2: 576; else 960) would be exceeded.
  const int tcap = rpt == 2 ? 768 : elem_bytes == 8 && D > 1 ? 576 : 960;
  const int nwb = std::min((nr + kWbRows - 1) / kWbRows, (tcap - pl.nt) / 64);
  const bool ring = dirs.size() >= 64 && nwb >= 1 &&
                    sweep_lds_bytes(nr, D, want_psi, true, elem_bytes, rpt) <= lmax;
  RTE_REQUIRE(sweep_lds_bytes(nr, D, want_psi, ring, elem_bytes, rpt) <= lmax,
              "sweep: %d x %d cells need %zu bytes of LDS per workgroup (device limit %zu)", g.nx,
              g.ny, sweep_lds_bytes(nr, D, want_psi, ring, elem_bytes, rpt), lmax);
  pl.D = D;
  pl.ring = ring ? 1 : 0;
  // Large plans without the ring (two rows per thread) store in line-sized groups: their
  // direct stores would otherwise write each 32-byte piece as a 64-byte burst.  Small
  // plans (the low-rank loop's few ordinates) store each cell: their bytes are few and
  // the grouping's register moves lengthen their latency-bound step.
  pl.grouped = !ring && rpt == 2 && dirs.size() >= 64 ? 1 : 0;
  if (ring) pl.nt += 64 * nwb;
  pl.psi = want_psi ? 1 : 0;
  pl.dsrc = per_dir_src ? 1 : 0;
  for (const auto& d : dirs) pl.nslots = std::max(pl.nslots, d.slot + 1);
  pl.groups = make_groups(dirs, D);
  pl.ngroups = (int)(pl.groups.size() / D);
  // Workgroups are dealt to the XCDs in turn (workgroup b to XCD b mod kXcds), each with
  // its own L2.  Giving each XCD a contiguous run of the quadrant-ordered groups lets its
  // L2 hold the staged inputs of one or two quadrants instead of all four.
  if (pl.ngroups >= 2 * kXcds) {
    std::vector<SweepDir> perm(pl.groups.size());
    const int G = pl.ngroups;
    for (int x = 0, start = 0; x < kXcds; ++x) {
      const int nx_ = (G - x + kXcds - 1) / kXcds;  // workgroups b = x + kXcds j < G
      for (int j = 0; j < nx_; ++j)
        std::copy_n(pl.groups.begin() + (long)(start + j) * D, D,
                    perm.begin() + (long)(x + kXcds * j) * D);
      start += nx_;
    }
    pl.groups.swap(perm);
  }
  for (const auto& d : pl.groups) pl.qmask |= 1 << ((d.sx < 0 ? 1 : 0) + (d.sy < 0 ? 2 : 0));
  return pl;
}

size_t sweep_input_elems(const Geom& g) {
  // both precisions use the larger of the two sigma_t strides
  const size_t qs = std::max(sig_stride<double>(g.nx, g.ny), sig_stride<float>(g.nx, g.ny));
  return 16ull * g.nx * g.ny + 4 * qs + 4ull * kPiece<float> * (g.nx + g.ny - 1);
}

size_t sweep_work_elems(const Geom& g, const SweepPlan& pl, bool want_phi) {
  return sweep_input_elems(g) + (want_phi ? (size_t)pl.ngroups * g.ndof : 0) +
         (pl.dsrc ? (size_t)pl.nslots * g.ndof : 0);
}

template <typename T>
void sweep_enqueue(const Geom& g, const SweepPlan& pl, const SweepDir* dirs_dev,
                   const double* sigma_t, const T* src, const double* bc, T* psi, T* phi,
                   T* work, hipStream_t st) {
  const long ncell = (long)g.nx * g.ny;
  RTE_REQUIRE(!psi || pl.psi, "sweep: the plan was made for the scalar flux only");
  RTE_REQUIRE(!(psi && phi) || pl.D == 1, "sweep: psi with the scalar flux needs one direction per workgroup");
  T* dsrc = work;              // [4][ncell][4]
  T* dsig = work + 16 * ncell;  // [4][sig_stride]
  T* dbnd = dsig + 4 * sig_stride<T>(g.nx, g.ny);  // [4][nsteps][kPiece]
  T* part = work + sweep_input_elems(g);
  const double shx = std::sqrt(g.hx), shy = std::sqrt(g.hy);
  {
    hipLaunchKernelGGL((diag_layout_kernel<T>), dim3((unsigned)(g.nx + g.ny - 1), 4), dim3(256), 0,
                       st, g.nx, g.ny, pl.qmask, sigma_t, pl.dsrc ? nullptr : src, bc, g.mb, shy,
                       dsrc, dsig, dbnd);
    RTE_CHECK_HIP(hipGetLastError());
  }
  if (pl.dsrc) {  // each direction's own source, in its quadrant's diagonal-major order
    RTE_REQUIRE(!phi, "sweep: per-direction sources give psi only");
    dsrc = work + sweep_input_elems(g);
    std::vector<int8_t> quad(pl.nslots, (int8_t)-1);
    for (const auto& d : pl.groups)
      if (d.slot >= 0) quad[d.slot] = (int8_t)((d.sx < 0 ? 1 : 0) + (d.sy < 0 ? 2 : 0));
    const int tb = 256;
    for (int s0 = 0; s0 < pl.nslots; s0 += kSlotsMax) {
      const int ns = std::min(kSlotsMax, pl.nslots - s0);
      SlotQuads sq;
      for (int k = 0; k < ns; ++k) sq.q[k] = quad[s0 + k];
      hipLaunchKernelGGL((diag_src_dirs_kernel<T>), dim3((unsigned)((ncell + tb - 1) / tb), ns),
                         dim3(tb), 0, st, g.nx, g.ny, s0, sq, src, dsrc);
    }
    RTE_CHECK_HIP(hipGetLastError());
  }
  const size_t lds = sweep_lds_bytes(pl.nc * pl.rpt, pl.D, psi != nullptr, pl.ring != 0, sizeof(T),
                                     pl.rpt);
  dim3 grid(pl.ngroups), block(pl.nt);
  T* pp = phi ? part : nullptr;
  // output mode: bit 0 the LDS ring, bit 1 psi, bit 2 the scalar-flux partial sums
  const int mode = (pl.ring ? 1 : 0) | (psi ? 2 : 0) | (pp ? 4 : 0) | (pl.grouped ? 8 : 0) |
                   (pl.dsrc ? 16 : 0);
#define RTE_SWEEP_K(DD, NTB, RP, SR, M)                                                         \
  RTE_REQUIRE(pl.nt <= NTB, "internal: %d threads for a sweep kernel of %d", pl.nt, NTB);        \
  hipLaunchKernelGGL((sweep_kernel<T, DD, NTB, RP, SR, M>), grid, block, lds, st, g.nx, g.ny,    \
                     g.mb, pl.nc, shx, shy, dirs_dev, dsrc, dsig, dbnd, bc, psi, pp, g.ndof)
// grouped direct stores (mode bit 8) exist for two rows per thread only
#define RTE_SWEEP_GRP(DD, NTB, RP, SR, M)                      \
  do {                                                         \
    if constexpr (RP == 2) {                                   \
      RTE_SWEEP_K(DD, NTB, RP, SR, M);                         \
    } else {                                                   \
      bad();                                                   \
    }                                                          \
  } while (0)
#define RTE_SWEEP_CASE(DD, NTB, RP, SR)                        \
  do {                                                         \
    if constexpr (DD == 1) {                                   \
      switch (mode) {                                          \
        case 2: RTE_SWEEP_K(DD, NTB, RP, SR, 2); break;        \
        case 3: RTE_SWEEP_K(DD, NTB, RP, SR, 3); break;        \
        case 4: RTE_SWEEP_K(DD, NTB, RP, SR, 4); break;        \
        case 5: RTE_SWEEP_K(DD, NTB, RP, SR, 5); break;        \
        case 6: RTE_SWEEP_K(DD, NTB, RP, SR, 6); break;        \
        case 7: RTE_SWEEP_K(DD, NTB, RP, SR, 7); break;        \
        case 10: RTE_SWEEP_GRP(DD, NTB, RP, SR, 10); break;    \
        case 12: RTE_SWEEP_GRP(DD, NTB, RP, SR, 12); break;    \
        case 14: RTE_SWEEP_GRP(DD, NTB, RP, SR, 14); break;    \
        case 18: RTE_SWEEP_K(DD, NTB, RP, SR, 18); break;      \
        case 19: RTE_SWEEP_K(DD, NTB, RP, SR, 19); break;      \
        case 26: RTE_SWEEP_GRP(DD, NTB, RP, SR, 26); break;    \
        default: bad();                                        \
      }                                                        \
    } else if (mode == 4) {                                    \
      RTE_SWEEP_K(DD, NTB, RP, SR, 4);                         \
    } else if (mode == 5) {                                    \
      RTE_SWEEP_K(DD, NTB, RP, SR, 5);                         \
    } else if (mode == 12) {                                   \
      RTE_SWEEP_GRP(DD, NTB, RP, SR, 12);                      \
    } else if constexpr (RP == 2 && sizeof(T) == 8) {          \
      if (mode == 10) {                                        \
        RTE_SWEEP_K(DD, NTB, RP, SR, 10);                      \
      } else {                                                 \
        bad();                                                 \
      }                                                        \
    } else {                                                   \
      bad();                                                   \
    }                                                          \
  } while (0)
  // FP64 plans use D = 2 only with at most 576 threads or with two rows per thread
  // (register budget)
#define RTE_SWEEP_D(NTB, RP, SR)                                                  \
  if (pl.D == 1) RTE_SWEEP_CASE(1, NTB, RP, SR);                                  \
  else if constexpr (sizeof(T) == 8 && NTB > 576 && RP == 1) bad();               \
  else if (pl.D == 2) RTE_SWEEP_CASE(2, NTB, RP, SR);                \
  else if constexpr (sizeof(T) == 8) bad();                          \
  else RTE_SWEEP_CASE(4, NTB, RP, SR);
  auto bad = [&] { RTE_REQUIRE(false, "sweep: no kernel for D = %d, %d threads", pl.D, pl.nt); };
  RTE_REQUIRE(pl.nt <= 1024, "sweep: %d threads", pl.nt);
  if (pl.rpt == 2) {
    RTE_REQUIRE(pl.srows == 256, "internal: staging rows %d", pl.srows);
    RTE_SWEEP_D(768, 2, 256)
  } else if (pl.srows == 64) {
    if (pl.nt <= 320) {
      RTE_SWEEP_D(320, 1, 64)
    } else {
      RTE_SWEEP_D(576, 1, 64)
    }
  } else if (pl.srows == 128) {
    if (pl.nt <= 576) {
      RTE_SWEEP_D(576, 1, 128)
    } else {
      RTE_SWEEP_D(960, 1, 128)
    }
  } else if (pl.nt <= 320) {
    RTE_SWEEP_D(320, 1, 256)
  } else if (pl.nt <= 576) {
    RTE_SWEEP_D(576, 1, 256)
  } else {
    RTE_SWEEP_D(960, 1, 256)
  }
#undef RTE_SWEEP_D
#undef RTE_SWEEP_CASE
#undef RTE_SWEEP_GRP
#undef RTE_SWEEP_K
  RTE_CHECK_HIP(hipGetLastError());
  if (phi) {
    const int tb = 256;
    if (mode == 12) {  // diagonal-major partial sums: per quadrant, then gathered per cell
      std::vector<int> lists[4];
      RTE_REQUIRE(pl.ngroups <= 32767, "sweep: %d workgroups", pl.ngroups);
      for (int b = 0; b < pl.ngroups; ++b) {
        const SweepDir& d = pl.groups[(size_t)b * pl.D];
        lists[(d.sx < 0 ? 1 : 0) + (d.sy < 0 ? 2 : 0)].push_back(b);
      }
      int g0[4] = {-1, -1, -1, -1};
      for (int q = 0; q < 4; ++q) {
        const std::vector<int>& l = lists[q];
        if (l.empty()) continue;
        g0[q] = l[0];
        for (size_t k0 = 0; k0 < l.size(); k0 += kListMax) {
          GroupList L;
          L.n = (int)std::min(l.size() - k0, (size_t)kListMax);
          L.acc = k0 > 0 ? 1 : 0;
          for (int k = 0; k < L.n; ++k) L.g[k] = (int16_t)l[k0 + k];
          hipLaunchKernelGGL((reduce_quadrant_kernel<T>), dim3((unsigned)((g.ndof + tb - 1) / tb)),
                             dim3(tb), 0, st, part, g.ndof, g0[q], L);
        }
      }
      hipLaunchKernelGGL((gather_quadrants_kernel<T>), dim3((unsigned)((g.ncell + tb - 1) / tb)),
                         dim3(tb), 0, st, part, g.ndof, g.nx, g.ny, g0[0], g0[1], g0[2], g0[3], phi);
    } else {
      hipLaunchKernelGGL((reduce_parts_kernel<T>), dim3((g.ndof + tb - 1) / tb), dim3(tb), 0, st,
                         part, pl.ngroups, g.ndof, phi);
    }
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
