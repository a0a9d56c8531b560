// C ABI entry points of the rte library: validation, set-up helpers (Appendix A/B)
// and the sweep entry points.  The SI-DSA solver lives in solver.hip.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.h"

namespace rte {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

const char* last_error() { return g_err; }

Geom make_geom(const rte_problem* p) {
  Geom g;
  g.nx = p->nx;
  g.ny = p->ny;
  g.mb = p->nx > p->ny ? p->nx : p->ny;
  g.x0 = p->x0; g.x1 = p->x1; g.y0 = p->y0; g.y1 = p->y1;
  g.hx = (p->x1 - p->x0) / p->nx;
  g.hy = (p->y1 - p->y0) / p->ny;
  g.ncell = (long)p->nx * p->ny;
  g.ndof = 4 * g.ncell;
  return g;
}

namespace {
__global__ void check_sigma_kernel(const double* st, const double* ss, long n, int* bad) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double t = st[i];
  int b = 0;
  if (!(t >= 1e-30) || !(t <= 1e30)) b |= 1;
  if (ss) {
    const double s = ss[i];
    if (!(s >= 0.0) || !(s <= t)) b |= 2;
  }
  if (b) atomicOr(bad, b);
}

__global__ void fill_kernel(double* p, double v, long n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename T>
__global__ void source_kernel(const double* __restrict__ sigma_s, const double* __restrict__ phi,
                              const double* __restrict__ G, T* __restrict__ out, long ndof) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ndof) return;
  double v = sigma_s[i >> 2] * phi[i];
  if (G) v += G[i];
  out[i] = T(v);
}

// per-block max |a-b| -> out[block]
__global__ void maxdiff_kernel(const double* __restrict__ a, const double* __restrict__ b, long n,
                               double* __restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    m = fmax(m, fabs(a[i] - b[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}
}  // namespace

bool progress_enabled() {
  static const bool on = [] {
    const char* v = std::getenv("RTE_PROGRESS");
    return v && v[0] && std::strcmp(v, "0") != 0;
  }();
  return on;
}

void validate_problem(const rte_problem* p, bool need_materials, hipStream_t st) {
  RTE_REQUIRE(p != nullptr, "problem is NULL");
  RTE_REQUIRE(p->nx >= 1 && p->ny >= 1, "nx, ny must be >= 1 (got %d, %d)", p->nx, p->ny);
  RTE_REQUIRE(p->x1 > p->x0 && p->y1 > p->y0, "empty domain");
  RTE_REQUIRE(p->n_dirs >= 1, "n_dirs must be >= 1");
  RTE_REQUIRE(p->dirs && p->wts, "dirs and wts are required");
  RTE_REQUIRE(p->sigma_t, "sigma_t is required");
  double sw = 0.0;
  for (int j = 0; j < p->n_dirs; ++j) {
    const double* o = p->dirs + 3 * j;
    const double nrm = o[0] * o[0] + o[1] * o[1] + o[2] * o[2];
    RTE_REQUIRE(std::fabs(nrm - 1.0) < 1e-10, "direction %d is not a unit vector", j);
    RTE_REQUIRE(p->wts[j] >= 0.0, "weight %d is negative", j);
    sw += p->wts[j];
  }
  RTE_REQUIRE(std::fabs(sw - 1.0) <= 1e-12, "weights sum to %.17g, not 1", sw);
  if (need_materials) {
    RTE_REQUIRE(p->sigma_s, "sigma_s is required");
    const long n = (long)p->nx * p->ny;
    DevBuf<int> bad(1);
    RTE_CHECK_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int), st));
    hipLaunchKernelGGL(check_sigma_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p->sigma_t,
                       p->sigma_s, n, bad.get());
    RTE_CHECK_HIP(hipGetLastError());
    int hb = 0;
    RTE_CHECK_HIP(hipMemcpyAsync(&hb, bad.get(), sizeof(int), hipMemcpyDeviceToHost, st));
    RTE_CHECK_HIP(hipStreamSynchronize(st));
    RTE_REQUIRE(!(hb & 1), "sigma_t must lie in [1e-30, 1e30] in every cell");
    RTE_REQUIRE(!(hb & 2), "sigma_s must satisfy 0 <= sigma_s <= sigma_t in every cell");
  }
}

void device_fill(double* p, double v, long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
  RTE_CHECK_HIP(hipGetLastError());
}

template <typename T>
void make_source(const Geom& g, const double* sigma_s, const double* phi, const double* G,
                 T* out, hipStream_t st) {
  hipLaunchKernelGGL((source_kernel<T>), dim3((g.ndof + 255) / 256), dim3(256), 0, st, sigma_s,
                     phi, G, out, g.ndof);
  RTE_CHECK_HIP(hipGetLastError());
}
template void make_source<double>(const Geom&, const double*, const double*, const double*,
                                  double*, hipStream_t);
template void make_source<float>(const Geom&, const double*, const double*, const double*,
                                 float*, hipStream_t);

double max_abs_diff(const double* a, const double* b, long n, hipStream_t st) {
  const int nb = 512;
  DevBuf<double> part(nb);
  hipLaunchKernelGGL(maxdiff_kernel, dim3(nb), dim3(256), 0, st, a, b, n, part.get());
  RTE_CHECK_HIP(hipGetLastError());
  std::vector<double> h(nb);
  RTE_CHECK_HIP(hipMemcpyAsync(h.data(), part.get(), nb * sizeof(double), hipMemcpyDeviceToHost, st));
  RTE_CHECK_HIP(hipStreamSynchronize(st));
  double m = 0.0;
  for (double x : h) m = x > m ? x : m;
  return m;
}

static std::vector<SweepDir> sweep_dirs(const rte_problem* p, const Geom& g, const int32_t* idx,
                                        int n, bool adjoint) {
  std::vector<SweepDir> v(n);
  for (int i = 0; i < n; ++i) {
    const int j = idx[i];
    RTE_REQUIRE(j >= 0 && j < p->n_dirs, "dir_idx[%d] = %d out of range", i, j);
    const double ox = p->dirs[3 * j], oy = p->dirs[3 * j + 1];
    SweepDir d;
    d.a = std::fabs(ox) / g.hx;
    d.b = std::fabs(oy) / g.hy;
    d.w = p->wts[j];
    // (D_j + Sigma_t)^T = D_{-Omega_j} + Sigma_t: the adjoint sweeps the reversed ordinate
    d.sx = ((ox >= 0.0) != adjoint) ? 1 : -1;
    d.sy = ((oy >= 0.0) != adjoint) ? 1 : -1;
    d.slot = i;
    d.pad = 0;
    v[i] = d;
  }
  return v;
}

static rte_status sweep_common(const rte_problem* prob, const int32_t* dir_idx, int32_t n_sel,
                               const void* src, void* psi, void* phi, rte_precision prec,
                               void* stream, bool adjoint) {
  try {
    StreamScope scope((hipStream_t)stream);
    validate_problem(prob, false, (hipStream_t)stream);
    RTE_REQUIRE(dir_idx && n_sel >= 1, "dir_idx / n_sel");
    RTE_REQUIRE(src, "src is NULL");
    RTE_REQUIRE(psi || phi, "one of psi, phi is required");
    RTE_REQUIRE(prec == RTE_FP64 || prec == RTE_MIXED, "unknown precision %d", (int)prec);
    Geom g = make_geom(prob);
    std::vector<SweepDir> dirs = sweep_dirs(prob, g, dir_idx, n_sel, adjoint);
    hipStream_t st = (hipStream_t)stream;
    if (prec == RTE_FP64)
      launch_sweep<double>(g, dirs, prob->sigma_t, (const double*)src, prob->bc, (double*)psi,
                           (double*)phi, st);
    else
      launch_sweep<float>(g, dirs, prob->sigma_t, (const float*)src, prob->bc, (float*)psi,
                          (float*)phi, st);
    return RTE_OK;
  } catch (const Error& e) {
    return e.code;
  }
}

// Gauss-Legendre nodes/weights on [-1,1] by Newton's method on P_n; nodes mirrored so
// that x_{n-1-i} = -x_i exactly.
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute the derivative at the converged node
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = pk;
    }
    if (n == 1) { p1 = z; p0 = 1.0; }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    const double wi = 2.0 / ((1.0 - z * z) * dp * dp);
    // z is the i-th largest node
    x[n - 1 - i] = z;
    x[i] = -z;
    w[n - 1 - i] = wi;
    w[i] = wi;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

// ---------------------------------------------------------------- allocation-free sweep
// rte_sweep_noalloc takes its workspace (the direction table, the anti-diagonal copies
// of the inputs and the per-workgroup partial sums of the scalar flux) from this
// file-scope device array instead of hipMalloc.  Each device holds its own copy for the
// lifetime of the process.  In host code `scratch` only names a host-side stand-in:
// kernels and copies get the device address from hipGetSymbolAddress (scratch_address).
constexpr size_t kScratchBytes = size_t(256) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex scratch_mu;
std::vector<void*> scratch_dev;  // per device ordinal: device address of `scratch`

// Device address of the current device's `scratch`, looked up once per device with that
// device current (its first rte_sweep_noalloc call).
void* scratch_address() {
  int dev = 0;
  RTE_CHECK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(scratch_mu);
  if ((int)scratch_dev.size() <= dev) scratch_dev.resize(dev + 1, nullptr);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    RTE_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    RTE_REQUIRE(p != nullptr, "hipGetSymbolAddress gave no address for the scratch array");
    scratch_dev[dev] = p;
  }
  return scratch_dev[dev];
}
}  // namespace

// The sweep of launch_sweep with the workspace carved from `scratch`.  The workspace is
// fully written by the layout kernel and the sweep before it is read, so nothing needs
// clearing.  The call waits for its kernels (the direction table is copied from host
// memory that ends with the call), like rte_sweep.
template <typename T>
static void noalloc_sweep(const Geom& g, const std::vector<SweepDir>& dirs, const double* sigma_t,
                          const T* src, const double* bc, T* psi, T* phi, hipStream_t st) {
  SweepPlan pl = make_sweep_plan(g, dirs, phi != nullptr, psi != nullptr, sizeof(T));
  const size_t dir_bytes = (pl.groups.size() * sizeof(SweepDir) + 255) / 256 * 256;
  const size_t work_bytes = sweep_work_elems(g, pl, phi != nullptr) * sizeof(T);
  RTE_REQUIRE(dir_bytes + work_bytes <= kScratchBytes,
              "rte_sweep_noalloc: this sweep needs %zu bytes of workspace; the scratch array "
              "holds %zu (use rte_sweep or a sweep plan)", dir_bytes + work_bytes, kScratchBytes);
  unsigned char* base = static_cast<unsigned char*>(scratch_address());
  SweepDir* ddirs = reinterpret_cast<SweepDir*>(base);
  T* work = reinterpret_cast<T*>(base + dir_bytes);
  RTE_CHECK_HIP(hipMemcpyAsync(ddirs, pl.groups.data(), pl.groups.size() * sizeof(SweepDir),
                               hipMemcpyHostToDevice, st));
  sweep_enqueue<T>(g, pl, ddirs, sigma_t, src, bc, psi, phi, work, st);
  RTE_CHECK_HIP(hipStreamSynchronize(st));
}

}  // namespace rte

struct rte_sweep_plan_s {
  rte::Geom g;
  rte::SweepPlan pl;                      // psi only
  rte::SweepPlan plf;                     // scalar flux only
  rte::SweepPlan plb;                     // psi and the scalar flux
  rte::DevBuf<rte::SweepDir> dirs, dirsf, dirsb;
  rte::DevBuf<unsigned char> work;
  const double* sigma_t = nullptr;
  const double* bc = nullptr;
  rte_precision prec = RTE_FP64;
  bool want_phi = false;
};

using namespace rte;

extern "C" {

const char* rte_last_error(void) { return rte::last_error(); }

int32_t rte_abi_version(void) { return 4; }

rte_status rte_sweep(const rte_problem* prob, const int32_t* dir_idx, int32_t n_sel,
                     const void* src, void* psi, void* phi, rte_precision prec, void* stream) {
  return sweep_common(prob, dir_idx, n_sel, src, psi, phi, prec, stream, false);
}

rte_status rte_sweep_noalloc(const rte_problem* prob, const int32_t* dir_idx, int32_t n_sel,
                             const void* src, void* psi, void* phi, rte_precision prec,
                             void* stream) {
  try {
    validate_problem(prob, false, (hipStream_t)stream);
    RTE_REQUIRE(dir_idx && n_sel >= 1, "dir_idx / n_sel");
    RTE_REQUIRE(src, "src is NULL");
    RTE_REQUIRE(psi || phi, "one of psi, phi is required");
    RTE_REQUIRE(prec == RTE_FP64 || prec == RTE_MIXED, "unknown precision %d", (int)prec);
    Geom g = make_geom(prob);
    std::vector<SweepDir> dirs = sweep_dirs(prob, g, dir_idx, n_sel, false);
    hipStream_t st = (hipStream_t)stream;
    if (prec == RTE_FP64)
      noalloc_sweep<double>(g, dirs, prob->sigma_t, (const double*)src, prob->bc, (double*)psi,
                            (double*)phi, st);
    else
      noalloc_sweep<float>(g, dirs, prob->sigma_t, (const float*)src, prob->bc, (float*)psi,
                           (float*)phi, st);
    return RTE_OK;
  } catch (const Error& e) {
    return e.code;
  }
}

rte_status rte_adjoint_sweep(const rte_problem* prob, const int32_t* dir_idx, int32_t n_sel,
                             const void* src, void* psi, void* phi, rte_precision prec,
                             void* stream) {
  return sweep_common(prob, dir_idx, n_sel, src, psi, phi, prec, stream, true);
}

rte_status rte_sweep_plan_create(const rte_problem* prob, const int32_t* dir_idx, int32_t n_sel,
                                 rte_precision prec, int32_t want_phi, int32_t adjoint,
                                 rte_sweep_plan* plan) {
  rte_sweep_plan_s* h = nullptr;
  try {
    RTE_REQUIRE(plan, "plan is NULL");
    *plan = nullptr;
    validate_problem(prob, false, nullptr);
    RTE_REQUIRE(dir_idx && n_sel >= 1, "dir_idx / n_sel");
    RTE_REQUIRE(prec == RTE_FP64 || prec == RTE_MIXED, "unknown precision %d", (int)prec);
    h = new rte_sweep_plan_s();
    h->g = make_geom(prob);
    std::vector<SweepDir> dirs = sweep_dirs(prob, h->g, dir_idx, n_sel, adjoint != 0);
    const size_t eb = prec == RTE_FP64 ? sizeof(double) : sizeof(float);
    auto upload = [&](const SweepPlan& p, DevBuf<SweepDir>& d) {
      d.alloc(p.groups.size());
      RTE_CHECK_HIP(hipMemcpy(d.get(), p.groups.data(), p.groups.size() * sizeof(SweepDir),
                              hipMemcpyHostToDevice));
    };
    h->pl = make_sweep_plan(h->g, dirs, false, true, eb);
    upload(h->pl, h->dirs);
    size_t work = sweep_work_elems(h->g, h->pl, false);
    if (want_phi) {
      h->plf = make_sweep_plan(h->g, dirs, true, false, eb);
      upload(h->plf, h->dirsf);
      h->plb = make_sweep_plan(h->g, dirs, true, true, eb);
      upload(h->plb, h->dirsb);
      work = std::max(work, sweep_work_elems(h->g, h->plf, true));
      work = std::max(work, sweep_work_elems(h->g, h->plb, true));
    }
    h->work.alloc(work * eb);
    h->sigma_t = prob->sigma_t;
    h->bc = prob->bc;
    h->prec = prec;
    h->want_phi = want_phi != 0;
    *plan = h;
    return RTE_OK;
  } catch (const Error& e) {
    delete h;
    return e.code;
  }
}

rte_status rte_sweep_execute(rte_sweep_plan h, const void* src, void* psi, void* phi,
                             void* stream) {
  try {
    RTE_REQUIRE(h, "plan is NULL");
    RTE_REQUIRE(src, "src is NULL");
    RTE_REQUIRE(psi || phi, "one of psi, phi is required");
    RTE_REQUIRE(!phi || h->want_phi, "the plan was created without the scalar-flux workspace");
    hipStream_t st = (hipStream_t)stream;
    const SweepPlan& pl = !phi ? h->pl : !psi ? h->plf : h->plb;
    const SweepDir* dd = !phi ? h->dirs.get() : !psi ? h->dirsf.get() : h->dirsb.get();
    if (h->prec == RTE_FP64)
      sweep_enqueue<double>(h->g, pl, dd, h->sigma_t, (const double*)src, h->bc,
                            (double*)psi, (double*)phi, (double*)h->work.get(), st);
    else
      sweep_enqueue<float>(h->g, pl, dd, h->sigma_t, (const float*)src, h->bc,
                           (float*)psi, (float*)phi, (float*)h->work.get(), st);
    return RTE_OK;
  } catch (const Error& e) {
    return e.code;
  }
}

rte_status rte_sweep_plan_destroy(rte_sweep_plan h) {
  if (h) {
    (void)hipDeviceSynchronize();
    delete h;
  }
  return RTE_OK;
}

rte_status rte_cl_quadrature(int32_t n_theta, int32_t n_z, double* dirs, double* wts) {
  try {
    RTE_REQUIRE(n_theta >= 1 && n_z >= 1, "CL rule needs n_theta, n_z >= 1");
    RTE_REQUIRE(dirs && wts, "output arrays are NULL");
    std::vector<double> mu, wz;
    gauss_legendre(n_z, mu, wz);
    for (int a = 0; a < n_z; ++a) {
      const double s = std::sqrt(1.0 - mu[a] * mu[a]);
      for (int b = 0; b < n_theta; ++b) {
        const double th = (2.0 * b + 1.0) * M_PI / n_theta;
        const int j = a * n_theta + b;
        dirs[3 * j] = std::cos(th) * s;
        dirs[3 * j + 1] = std::sin(th) * s;
        dirs[3 * j + 2] = mu[a];
        wts[j] = 0.5 * wz[a] / n_theta;
      }
    }
    return RTE_OK;
  } catch (const Error& e) {
    return e.code;
  }
}

rte_status rte_box_source_moments(int32_t nx, int32_t ny, double x0, double x1, double y0,
                                  double y1, double value, double bx0, double bx1, double by0,
                                  double by1, double* G) {
  try {
    RTE_REQUIRE(nx >= 1 && ny >= 1 && x1 > x0 && y1 > y0, "bad mesh");
    RTE_REQUIRE(G, "G is NULL");
    const double hx = (x1 - x0) / nx, hy = (y1 - y0) / ny;
    const double r3 = std::sqrt(3.0);
    // int over [lo,hi] of l_0, l_1 on a cell of centre c and width h
    auto moments = [&](double lo, double hi, double c, double h, double m[2]) {
      const double xl = 2.0 * (lo - c) / h, xh = 2.0 * (hi - c) / h;
      m[0] = (hi - lo) / std::sqrt(h);
      m[1] = r3 * std::sqrt(h) * 0.25 * (xh * xh - xl * xl);
    };
    for (int b = 0; b < ny; ++b) {
      const double ya = y0 + b * hy, yb = ya + hy;
      const double lo_y = std::max(ya, by0), hi_y = std::min(yb, by1);
      if (hi_y <= lo_y) continue;
      double my[2];
      moments(lo_y, hi_y, ya + 0.5 * hy, hy, my);
      for (int a = 0; a < nx; ++a) {
        const double xa = x0 + a * hx, xb = xa + hx;
        const double lo_x = std::max(xa, bx0), hi_x = std::min(xb, bx1);
        if (hi_x <= lo_x) continue;
        double mx[2];
        moments(lo_x, hi_x, xa + 0.5 * hx, hx, mx);
        double* c = G + 4 * ((long)b * nx + a);
        for (int q = 0; q < 2; ++q)
          for (int p = 0; p < 2; ++p) c[2 * q + p] += value * mx[p] * my[q];
      }
    }
    return RTE_OK;
  } catch (const Error& e) {
    return e.code;
  }
}

rte_status rte_inflow_face_moments(int32_t nx, int32_t ny, double x0, double x1, double y0,
                                  double y1, int32_t side, int32_t index, double value,
                                  double* bc) {
  try {
    RTE_REQUIRE(nx >= 1 && ny >= 1 && x1 > x0 && y1 > y0, "bad mesh");
    RTE_REQUIRE(bc, "bc is NULL");
    RTE_REQUIRE(side >= 0 && side < 4, "side must be 0..3 (L, R, B, T), got %d", side);
    const int count = side < 2 ? ny : nx;
    RTE_REQUIRE(index >= 0 && index < count, "face index %d out of range [0, %d)", index, count);
    // a constant g on a face of length h: int g l_0 = g sqrt(h), int g l_1 = 0
    const double h = side < 2 ? (y1 - y0) / ny : (x1 - x0) / nx;
    const int mb = nx > ny ? nx : ny;
    bc[2 * ((long)side * mb + index)] += value * std::sqrt(h);
    return RTE_OK;
  } catch (const Error& e) {
    return e.code;
  }
}

rte_status rte_gaussian_source_moments(int32_t nx, int32_t ny, double x0, double x1, double y0,
                                       double y1, double amp, double alpha, double cx, double cy,
                                       double* G) {
  try {
    RTE_REQUIRE(nx >= 1 && ny >= 1 && x1 > x0 && y1 > y0, "bad mesh");
    RTE_REQUIRE(alpha > 0.0 && std::isfinite(alpha), "alpha must be positive and finite");
    RTE_REQUIRE(std::isfinite(amp) && std::isfinite(cx) && std::isfinite(cy), "non-finite input");
    RTE_REQUIRE(G, "G is NULL");
    const double hx = (x1 - x0) / nx, hy = (y1 - y0) / ny;
    const double r3 = std::sqrt(3.0), sa = std::sqrt(alpha);
    const double k0 = 0.5 * std::sqrt(M_PI / alpha);
    // erf(b) - erf(a) for a <= b, through erfc on the side away from 0 (no cancellation
    // of two values close to +-1)
    auto derf = [](double a, double b) {
      if (a >= 0.0) return std::erfc(a) - std::erfc(b);
      if (b <= 0.0) return std::erfc(-b) - std::erfc(-a);
      return std::erf(b) - std::erf(a);
    };
    // moments of g(t) = exp(-alpha (t - t0)^2) on the cells of one axis against
    // l_0 = 1/sqrt(h) and l_1 = sqrt3 xi / sqrt(h), xi = 2 (t - c) / h:
    //   int g = k0 [erf(sa u)]_ua^ub,  int (t - c) g = [-g / (2 alpha)]_ua^ub + (t0 - c) int g,
    // with u = t - t0
    auto axis = [&](int n, double lo, double h, double t0, std::vector<double>& m) {
      m.assign(2 * (size_t)n, 0.0);
      for (int i = 0; i < n; ++i) {
        const double a = lo + i * h, b = a + h, c = a + 0.5 * h;
        const double ua = a - t0, ub = b - t0;
        const double i0 = k0 * derf(sa * ua, sa * ub);
        const double i1 = (std::exp(-alpha * ua * ua) - std::exp(-alpha * ub * ub)) / (2.0 * alpha) +
                          (t0 - c) * i0;
        m[2 * i] = i0 / std::sqrt(h);
        m[2 * i + 1] = r3 * 2.0 * i1 / (h * std::sqrt(h));
      }
    };
    std::vector<double> mx, my;
    axis(nx, x0, hx, cx, mx);
    axis(ny, y0, hy, cy, my);
    for (int b = 0; b < ny; ++b)
      for (int a = 0; a < nx; ++a) {
        double* c = G + 4 * ((long)b * nx + a);
        for (int q = 0; q < 2; ++q)
          for (int p = 0; p < 2; ++p) c[2 * q + p] += amp * mx[2 * a + p] * my[2 * b + q];
      }
    return RTE_OK;
  } catch (const Error& e) {
    return e.code;
  }
}

}  // extern "C"
