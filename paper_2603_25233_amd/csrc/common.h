// Internal declarations of the rte library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/rte.h"

namespace rte {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
const char* last_error();

struct Error {
  rte_status code;
};

#define RTE_CHECK_HIP(expr)                                                            \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::rte::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                      \
      throw ::rte::Error{e_ == hipErrorOutOfMemory ? RTE_ENOMEM : RTE_EHIP};           \
    }                                                                                  \
  } while (0)

#define RTE_REQUIRE(cond, ...)             \
  do {                                     \
    if (!(cond)) {                         \
      ::rte::set_error(__VA_ARGS__);       \
      throw ::rte::Error{RTE_EINVAL};      \
    }                                      \
  } while (0)

// ---------------------------------------------------------------- device memory
// Inside a StreamScope (one per entry point that takes a stream) buffers come from and go
// back to a cache of idle blocks; outside one, straight from hipMalloc / to hipFree.
// pool_alloc sets *pooled to whether the block belongs to the cache.
void* pool_alloc(size_t bytes, bool* pooled);
void pool_free(void* p, size_t bytes, bool pooled);
void pool_release_all();
// Marks the calls on `st` that allocate the library's temporaries; at the end of the
// outermost scope `st` is synchronised once and the buffers released in it become idle.
struct StreamScope {
  explicit StreamScope(hipStream_t st);
  ~StreamScope();
  StreamScope(const StreamScope&) = delete;
  StreamScope& operator=(const StreamScope&) = delete;
};

// Device buffer owned by one library call (released on scope exit, also on error).
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  bool pooled = false;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  void alloc(size_t count) {
    release();
    n = count;
    if (count) p = static_cast<T*>(pool_alloc(count * sizeof(T), &pooled));
  }
  void release() {
    if (p) pool_free(p, n * sizeof(T), pooled);
    p = nullptr;
    n = 0;
    pooled = false;
  }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  T* get() const { return p; }
};

// ---------------------------------------------------------------- problem on the host
struct Geom {
  int nx, ny, mb;          // cells; mb = max(nx, ny) (length of a boundary-data side)
  double x0, x1, y0, y1, hx, hy;
  long ncell, ndof;
};

Geom make_geom(const rte_problem* p);

// Per-outer-iteration progress lines on stderr when the environment variable
// RTE_PROGRESS is set to a non-empty value other than "0".
bool progress_enabled();
// Host checks of the problem; with need_materials the per-cell cross sections are also
// range-checked by a kernel on `st` (the caller's stream, so that it sees what earlier
// work on that stream wrote), followed by a synchronisation of `st`.
void validate_problem(const rte_problem* p, bool need_materials, hipStream_t st);

// Per-direction sweep parameters (canonical frame: the sweep always runs towards
// +x and +y after a reflection of the cell coordinates by the direction signs).
struct SweepDir {
  double a;      // |Omega_x| / hx
  double b;      // |Omega_y| / hy
  double w;      // weight used when accumulating phi
  int sx, sy;    // signs of the direction actually swept (+1 / -1)
  int slot;      // output slot in psi
  int pad;
};

// A sweep plan groups directions of one quadrant into workgroups of D directions
// (padding entries have slot = -1).  `groups` is uploaded to the device by the caller.
struct SweepPlan {
  std::vector<SweepDir> groups;
  int D = 1, ngroups = 0;
  int nt = 64;    // threads per workgroup: nc compute threads + staging wavefronts
  int nc = 64;
  int rpt = 1;    // rows per compute thread
  int ring = 1;   // results leave through the LDS ring (else direct stores)
  int grouped = 0;  // direct stores in line-sized groups of a row's cells
  int psi = 1;    // planned for psi output (else the scalar flux only)
  int qmask = 0;  // quadrants swept (bit q = (sx < 0) + 2 (sy < 0))
  int srows = 256;  // rows of a step that each staging wavefront copies
  int dsrc = 0;     // one source per direction: the source of psi slot s is row s of a
                    // [nslots][ndof] array (psi only, one direction per workgroup)
  int nslots = 0;   // 1 + the largest psi slot
};
// Plans for psi (want_psi) or for the scalar flux only; a psi plan also serves
// calls that request both.
SweepPlan make_sweep_plan(const Geom& g, const std::vector<SweepDir>& dirs, bool want_phi,
                          bool want_psi, size_t elem_bytes, bool per_dir_src = false);
// Elements of T the sweep needs as workspace: the diagonal-major copies of the
// source and cross section (about 5 ncell per quadrant) and, when phi is requested,
// the per-group partial sums ([ngroups][ndof]); with one source per direction, the
// diagonal-major copy of each ([nslots][ndof]).
size_t sweep_input_elems(const Geom& g);
size_t sweep_work_elems(const Geom& g, const SweepPlan& pl, bool want_phi);
// Enqueues the sweep (no synchronisation).  work: sweep_work_elems(g, pl, phi != null)
// elements.  psi != null needs a plan made with want_psi.  With a per-direction-source
// plan, src is [nslots][ndof] (the source of psi slot s in row s).
template <typename T>
void sweep_enqueue(const Geom& g, const SweepPlan& pl, const SweepDir* dirs_dev,
                   const double* sigma_t, const T* src, const double* bc, T* psi, T* phi,
                   T* work, hipStream_t st);
// One-shot sweep with its own temporaries; returns after completion on `st`.
template <typename T>
void launch_sweep(const Geom& g, const std::vector<SweepDir>& dirs, const double* sigma_t,
                  const T* src, const double* bc, T* psi, T* phi, hipStream_t st);

// ---------------------------------------------------------------- DSA (diffusion correction)
struct DSA;
DSA* dsa_create(const Geom& g, const double* sigma_t_dev, const double* sigma_s_dev,
                hipStream_t st);
void dsa_destroy(DSA* d);
// delta = A^{-1} Sigma_s (phi_star - phi_prev);  phi_next = phi_star + delta.
// Returns the number of CG iterations.
int dsa_apply(DSA* d, const double* phi_star, const double* phi_prev, double* phi_next,
              double rel_tol, hipStream_t st);

// ---------------------------------------------------------------- small device helpers
// Workgroups are dealt to the eight XCDs in turn (workgroup b to XCD b mod 8), each with
// its own L2.  This maps the n workgroups of a one-dimensional launch so that each XCD
// runs a contiguous range of them: neighbouring work items then belong to workgroups of
// the same XCD, and their loads of shared lines hit its L2.  (A bijection of [0, n).)
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned n) {
  const unsigned q = n / 8, r = n % 8, x = b % 8;
  return x * q + min(x, r) + b / 8;
}

void device_fill(double* p, double v, long n, hipStream_t st);
// out = sigma_s * phi + G (per cell), G may be null
template <typename T>
void make_source(const Geom& g, const double* sigma_s, const double* phi, const double* G,
                 T* out, hipStream_t st);
// host value of max |a - b| (synchronises)
double max_abs_diff(const double* a, const double* b, long n, hipStream_t st);

}  // namespace rte
