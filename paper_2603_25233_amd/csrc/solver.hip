// SI-DSA driver (paper Alg. 1): full-rank SI (Sec. 2.2) and the low-rank SI of Sec. 3
// (lowrank.hip), outer stopping test, DSA step; exit currents and cross-section
// gradients for the adjoint (project addition).
//
// Readings shared with the oracle:
//   * the outer test ||phi^{n,*} - phi^{n-1}||_inf <= eps_si (coefficient vector) is
//     taken before the DSA step (Alg. 1), and phi^{n,*} of the last step is returned;
//   * the DSA right-hand side is Sigma_s (phi^{n,*} - phi^{n-1}).
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>

#include "common.h"
#include "lowrank.h"

namespace rte {

namespace {

__global__ void to_double_kernel(const float* __restrict__ a, double* __restrict__ b, long n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

// out = Sigma_s (a - b) in float: the change of the isotropic scattering source
__global__ void incr_source_kernel(const double* __restrict__ sigma_s, const double* __restrict__ a,
                                   const double* __restrict__ b, float* __restrict__ out, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)(sigma_s[i >> 2] * (a[i] - b[i]));
}

// acc += (double) d
__global__ void accumulate_kernel(double* __restrict__ acc, const float* __restrict__ d, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) acc[i] += (double)d[i];
}

// J[side][i] for boundary faces from psi [n_dirs][ndof]; one thread per face,
// ordinates summed in index order.
__global__ void exit_current_kernel(int nx, int ny, int mb, double hx, double hy, int n_dirs,
                                    const double* __restrict__ ox, const double* __restrict__ oy,
                                    const double* __restrict__ w, const double* __restrict__ psi,
                                    long ndof, double* __restrict__ J) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= 4 * mb) return;
  const int side = f / mb, i = f % mb;
  const int count = side < 2 ? ny : nx;
  if (i >= count) {
    J[f] = 0.0;
    return;
  }
  const double r3 = 1.7320508075688772935;
  long c;
  double tr0, tr1, scale;  // trace integral = scale * (psi_0 + tr1 * psi_k)
  int k;
  if (side == 0) { c = (long)i * nx; k = 1; tr1 = -r3; scale = std::sqrt(hy / hx) / hy; }
  else if (side == 1) { c = (long)i * nx + nx - 1; k = 1; tr1 = r3; scale = std::sqrt(hy / hx) / hy; }
  else if (side == 2) { c = i; k = 2; tr1 = -r3; scale = std::sqrt(hx / hy) / hx; }
  else { c = (long)(ny - 1) * nx + i; k = 2; tr1 = r3; scale = std::sqrt(hx / hy) / hx; }
  tr0 = 1.0;
  double acc = 0.0;
  for (int j = 0; j < n_dirs; ++j) {
    const double on = side == 0 ? -ox[j] : side == 1 ? ox[j] : side == 2 ? -oy[j] : oy[j];
    if (on <= 0.0) continue;
    const double* pc = psi + (long)j * ndof + 4 * c;
    acc += w[j] * on * (tr0 * pc[0] + tr1 * pc[k]);
  }
  J[f] = acc * scale;
}

// Detector misfit L = 1/2 sum_e (J_e - J_obs,e)^2 over the boundary faces and the
// adjoint inflow it induces: on face e the isotropic inflow (J_e - J_obs,e)/|e|, whose
// face moments are ((J_e - J_obs,e)/sqrt|e|, 0).  One block; part of L per thread
// summed in a fixed order.
__global__ __launch_bounds__(256) void misfit_kernel(int nx, int ny, int mb, double hx, double hy,
                                                     const double* __restrict__ J,
                                                     const double* __restrict__ J_obs,
                                                     double* __restrict__ bc_adj,
                                                     double* __restrict__ loss) {
  __shared__ double red[256];
  double s = 0.0;
  for (int f = threadIdx.x; f < 4 * mb; f += 256) {
    const int side = f / mb, i = f % mb;
    const bool valid = i < (side < 2 ? ny : nx);
    const double len = side < 2 ? hy : hx;
    const double d = valid ? J[f] - J_obs[f] : 0.0;
    s += 0.5 * d * d;
    bc_adj[2 * f] = valid ? d / sqrt(len) : 0.0;
    bc_adj[2 * f + 1] = 0.0;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0];
}

// grad_a[c] = -sum_j w_j <mu_j, psi_j>_c ; grad_s[c] = grad_a[c] + <phi_adj, phi>_c
__global__ void gradient_kernel(long ncell, int n_dirs, const double* __restrict__ w,
                                const double* __restrict__ psi, const double* __restrict__ mu,
                                long ndof, const double* __restrict__ phi,
                                const double* __restrict__ phia, double* __restrict__ ga,
                                double* __restrict__ gs) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  double acc = 0.0;
  for (int j = 0; j < n_dirs; ++j) {
    const double* a = psi + (long)j * ndof + 4 * c;
    const double* b = mu + (long)j * ndof + 4 * c;
    acc += w[j] * (a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3]);
  }
  const double g = -acc;
  ga[c] = g;
  const double* p = phi + 4 * c;
  const double* q = phia + 4 * c;
  gs[c] = g + (p[0] * q[0] + p[1] * q[1] + p[2] * q[2] + p[3] * q[3]);
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

std::vector<SweepDir> all_dirs(const rte_problem* p, const Geom& g, bool adjoint) {
  std::vector<SweepDir> v(p->n_dirs);
  for (int j = 0; j < p->n_dirs; ++j) {
    const double ox = p->dirs[3 * j], oy = p->dirs[3 * j + 1];
    SweepDir d;
    d.a = std::fabs(ox) / g.hx;
    d.b = std::fabs(oy) / g.hy;
    d.w = p->wts[j];
    d.sx = ((ox >= 0.0) != adjoint) ? 1 : -1;
    d.sy = ((oy >= 0.0) != adjoint) ? 1 : -1;
    d.slot = j;
    d.pad = 0;
    v[j] = d;
  }
  return v;
}

// One direction per class of equal (Omega_x, Omega_y), in order of the smallest member,
// carrying the class's summed weight (added in ordinate order).  In X-Y geometry the
// sweep of an ordinate depends on Omega only through (Omega_x, Omega_y), so the Omega_z
// twins of a class have identical psi and sum_j w_j psi_j is unchanged.
std::vector<SweepDir> fold_classes(const rte_problem* p, std::vector<SweepDir> v) {
  std::vector<SweepDir> out;
  std::vector<int> rep;  // ordinate index of each class's first member
  for (int j = 0; j < p->n_dirs; ++j) {
    int c = -1;
    for (int k = 0; k < (int)rep.size(); ++k) {
      const int i = rep[k];
      if (std::fabs(p->dirs[3 * i] - p->dirs[3 * j]) <= 1e-12 &&
          std::fabs(p->dirs[3 * i + 1] - p->dirs[3 * j + 1]) <= 1e-12) {
        c = k;
        break;
      }
    }
    if (c < 0) {
      rep.push_back(j);
      SweepDir d = v[j];
      d.slot = (int)out.size();
      out.push_back(d);
    } else {
      out[c].w += v[j].w;
    }
  }
  return out;
}

std::vector<SweepDir> class_dirs(const rte_problem* p, const Geom& g) {
  return fold_classes(p, all_dirs(p, g, false));
}

// Full-rank SI-DSA in precision T (sweeps and the swept scalar flux in T).
template <typename T>
static rte_status fr_solve(const rte_problem* prob, const rte_solve_params* prm,
                           const double* phi0, double* phi_out, rte_solve_result* res,
                           hipStream_t st) {
  const auto t_start = std::chrono::steady_clock::now();
  const Geom g = make_geom(prob);
  const long nd = g.ndof;
  std::vector<SweepDir> dirs = all_dirs(prob, g, prm->adjoint != 0);
  if (prm->fold_classes) dirs = fold_classes(prob, std::move(dirs));
  const int n_swept_dirs = (int)dirs.size();
  SweepPlan plan = make_sweep_plan(g, dirs, true, false, sizeof(T));
  DevBuf<SweepDir> ddirs(plan.groups.size());
  RTE_CHECK_HIP(hipMemcpy(ddirs.get(), plan.groups.data(), plan.groups.size() * sizeof(SweepDir),
                          hipMemcpyHostToDevice));
  DevBuf<T> work(sweep_work_elems(g, plan, true)), src(nd), phiT;
  DevBuf<double> phi_prev(nd), phi_star(nd);
  if (sizeof(T) != sizeof(double)) phiT.alloc(nd);
  if (phi0)
    RTE_CHECK_HIP(hipMemcpyAsync(phi_prev.get(), phi0, nd * sizeof(double), hipMemcpyDeviceToDevice, st));
  else
    device_fill(phi_prev.get(), 0.0, nd, st);
  std::unique_ptr<DSA, void (*)(DSA*)> dsa(nullptr, dsa_destroy);
  if (prm->use_dsa) dsa.reset(dsa_create(g, prob->sigma_t, prob->sigma_s, st));
  hipEvent_t e0, e1;
  RTE_CHECK_HIP(hipEventCreate(&e0));
  RTE_CHECK_HIP(hipEventCreate(&e1));
  double ms_sweep = 0.0, ms_dsa = 0.0;
  int dsa_iters = 0, n = 0;
  bool conv = false;
  const double* G = prm->adjoint ? nullptr : prob->G;
  for (n = 1; n <= prm->max_outer; ++n) {
    RTE_CHECK_HIP(hipEventRecord(e0, st));
    make_source<T>(g, prob->sigma_s, phi_prev.get(), G, src.get(), st);
    T* phi_sw = sizeof(T) == sizeof(double) ? (T*)phi_star.get() : phiT.get();
    sweep_enqueue<T>(g, plan, ddirs.get(), prob->sigma_t, src.get(), prob->bc, nullptr, phi_sw,
                     work.get(), st);
    if (sizeof(T) != sizeof(double))
      hipLaunchKernelGGL(to_double_kernel, dim3((nd + 255) / 256), dim3(256), 0, st,
                         (const float*)phiT.get(), phi_star.get(), nd);
    RTE_CHECK_HIP(hipEventRecord(e1, st));
    const double d = max_abs_diff(phi_star.get(), phi_prev.get(), nd, st);
    float ms = 0.f;
    RTE_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
    ms_sweep += ms;
    if (res && res->history) res->history[n - 1] = d;
    if (prm->phi_checkpoints)
      RTE_CHECK_HIP(hipMemcpyAsync(prm->phi_checkpoints + (long)(n - 1) * nd, phi_star.get(),
                                   nd * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (progress_enabled())
      std::fprintf(stderr, "[rte] full rank: outer %d, |phi* - phi|_inf %.3e, %.0f ms\n", n, d,
                   ms_since(t_start));
    if (d <= prm->eps_si) {
      conv = true;
      break;
    }
    if (n == prm->max_outer) break;
    const auto t0 = std::chrono::steady_clock::now();
    if (dsa) {
      dsa_iters += dsa_apply(dsa.get(), phi_star.get(), phi_prev.get(), phi_prev.get(),
                             prm->eps_dsa, st);
      RTE_CHECK_HIP(hipStreamSynchronize(st));
    } else {
      RTE_CHECK_HIP(hipMemcpyAsync(phi_prev.get(), phi_star.get(), nd * sizeof(double),
                                   hipMemcpyDeviceToDevice, st));
    }
    ms_dsa += ms_since(t0);
  }
  if (n > prm->max_outer) n = prm->max_outer;
  RTE_CHECK_HIP(hipMemcpyAsync(phi_out, phi_star.get(), nd * sizeof(double),
                               hipMemcpyDeviceToDevice, st));
  RTE_CHECK_HIP(hipStreamSynchronize(st));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (res) {
    res->outer_iters = n;
    res->converged = conv ? 1 : 0;
    res->rank = 0;
    res->n_swept = n * n_swept_dirs;
    res->dsa_iters = dsa_iters;
    res->ms_sweep = ms_sweep;
    res->ms_dsa = ms_dsa;
    res->ms_lowrank = 0.0;
    res->ms_total = ms_since(t_start);
  }
  return conv ? RTE_OK : RTE_ENOCONV;
}

// Mixed-precision full-rank SI-DSA.  The SI map is affine in phi with the inflow in
// its constant part, so phi^{n,*} - phi^{n-1,*} = W T^{-1} Sigma_s (phi^{n-1} - phi^{n-2})
// with vacuum inflow.  Outer iterations sweep the whole source in FP64 until the SI
// change d_n = |phi^{n,*} - phi^{n-1}|_inf falls to kMixedSwitch |phi^{n,*}|_inf; after that
// they sweep only the change of the scattering source, in FP32, and add the swept change
// to phi^{n-1,*} in FP64.  FP32 rounding then enters only relative to the (small, and
// shrinking) increments: the diffusion correction, which amplifies the smooth part of
// any error of phi^{n,*} by up to sigma_s / sigma_a, no longer sees FP32 rounding of the
// flux itself.  With kMixedSwitch = 1e-3 the rounding that reaches phi is about
// 6e-8 * 1e-3 times that amplification.
constexpr double kMixedSwitch = 1e-3;

static rte_status fr_solve_mixed(const rte_problem* prob, const rte_solve_params* prm,
                                 const double* phi0, double* phi_out, rte_solve_result* res,
                                 hipStream_t st) {
  const auto t_start = std::chrono::steady_clock::now();
  const Geom g = make_geom(prob);
  const long nd = g.ndof;
  std::vector<SweepDir> dirs = all_dirs(prob, g, prm->adjoint != 0);
  if (prm->fold_classes) dirs = fold_classes(prob, std::move(dirs));
  const int n_swept_dirs = (int)dirs.size();
  SweepPlan p64 = make_sweep_plan(g, dirs, true, false, sizeof(double));
  SweepPlan p32 = make_sweep_plan(g, dirs, true, false, sizeof(float));
  DevBuf<SweepDir> d64(p64.groups.size()), d32(p32.groups.size());
  RTE_CHECK_HIP(hipMemcpy(d64.get(), p64.groups.data(), p64.groups.size() * sizeof(SweepDir),
                          hipMemcpyHostToDevice));
  RTE_CHECK_HIP(hipMemcpy(d32.get(), p32.groups.data(), p32.groups.size() * sizeof(SweepDir),
                          hipMemcpyHostToDevice));
  DevBuf<double> work64(sweep_work_elems(g, p64, true)), src64(nd), phi_prev(nd), phi_pp(nd),
      phi_star(nd), zero(nd);
  DevBuf<float> work32(sweep_work_elems(g, p32, true)), src32(nd), dphi(nd);
  if (phi0)
    RTE_CHECK_HIP(hipMemcpyAsync(phi_prev.get(), phi0, nd * sizeof(double), hipMemcpyDeviceToDevice, st));
  else
    device_fill(phi_prev.get(), 0.0, nd, st);
  device_fill(zero.get(), 0.0, nd, st);
  std::unique_ptr<DSA, void (*)(DSA*)> dsa(nullptr, dsa_destroy);
  if (prm->use_dsa) dsa.reset(dsa_create(g, prob->sigma_t, prob->sigma_s, st));
  hipEvent_t e0, e1;
  RTE_CHECK_HIP(hipEventCreate(&e0));
  RTE_CHECK_HIP(hipEventCreate(&e1));
  double ms_sweep = 0.0, ms_dsa = 0.0;
  int dsa_iters = 0, n = 0, n64 = 0;
  bool conv = false, full64 = true;
  const double* G = prm->adjoint ? nullptr : prob->G;
  const unsigned nb = (unsigned)((nd + 255) / 256);
  for (n = 1; n <= prm->max_outer; ++n) {
    RTE_CHECK_HIP(hipEventRecord(e0, st));
    if (full64) {
      make_source<double>(g, prob->sigma_s, phi_prev.get(), G, src64.get(), st);
      sweep_enqueue<double>(g, p64, d64.get(), prob->sigma_t, src64.get(), prob->bc, nullptr,
                            phi_star.get(), work64.get(), st);
      ++n64;
    } else {
      hipLaunchKernelGGL(incr_source_kernel, dim3(nb), dim3(256), 0, st, prob->sigma_s,
                         phi_prev.get(), phi_pp.get(), src32.get(), nd);
      sweep_enqueue<float>(g, p32, d32.get(), prob->sigma_t, src32.get(), nullptr, nullptr,
                           dphi.get(), work32.get(), st);
      hipLaunchKernelGGL(accumulate_kernel, dim3(nb), dim3(256), 0, st, phi_star.get(),
                         dphi.get(), nd);
    }
    RTE_CHECK_HIP(hipGetLastError());
    RTE_CHECK_HIP(hipEventRecord(e1, st));
    const double d = max_abs_diff(phi_star.get(), phi_prev.get(), nd, st);
    float ms = 0.f;
    RTE_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
    ms_sweep += ms;
    if (res && res->history) res->history[n - 1] = d;
    if (prm->phi_checkpoints)
      RTE_CHECK_HIP(hipMemcpyAsync(prm->phi_checkpoints + (long)(n - 1) * nd, phi_star.get(),
                                   nd * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (progress_enabled())
      std::fprintf(stderr, "[rte] full rank (mixed, %s sweep): outer %d, |phi* - phi|_inf %.3e, %.0f ms\n",
                   full64 ? "FP64" : "FP32 increment", n, d, ms_since(t_start));
    if (d <= prm->eps_si) {
      conv = true;
      break;
    }
    if (n == prm->max_outer) break;
    if (full64 && d <= kMixedSwitch * max_abs_diff(phi_star.get(), zero.get(), nd, st))
      full64 = false;
    RTE_CHECK_HIP(hipMemcpyAsync(phi_pp.get(), phi_prev.get(), nd * sizeof(double),
                                 hipMemcpyDeviceToDevice, st));
    const auto t0 = std::chrono::steady_clock::now();
    if (dsa) {
      dsa_iters += dsa_apply(dsa.get(), phi_star.get(), phi_prev.get(), phi_prev.get(),
                             prm->eps_dsa, st);
      RTE_CHECK_HIP(hipStreamSynchronize(st));
    } else {
      RTE_CHECK_HIP(hipMemcpyAsync(phi_prev.get(), phi_star.get(), nd * sizeof(double),
                                   hipMemcpyDeviceToDevice, st));
    }
    ms_dsa += ms_since(t0);
  }
  if (n > prm->max_outer) n = prm->max_outer;
  RTE_CHECK_HIP(hipMemcpyAsync(phi_out, phi_star.get(), nd * sizeof(double),
                               hipMemcpyDeviceToDevice, st));
  RTE_CHECK_HIP(hipStreamSynchronize(st));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (res) {
    res->outer_iters = n;
    res->converged = conv ? 1 : 0;
    res->rank = 0;
    res->n_swept = n * n_swept_dirs;
    res->dsa_iters = dsa_iters;
    res->ms_sweep = ms_sweep;
    res->ms_dsa = ms_dsa;
    res->ms_lowrank = 0.0;
    res->ms_total = ms_since(t_start);
    res->fp64_sweeps = n64;
  }
  return conv ? RTE_OK : RTE_ENOCONV;
}

static void validate_params(const rte_problem* prob, const rte_solve_params* p) {
  RTE_REQUIRE(p, "params is NULL");
  RTE_REQUIRE(p->max_outer >= 1, "max_outer must be >= 1");
  RTE_REQUIRE(p->eps_si >= 0.0, "eps_si must be >= 0");
  RTE_REQUIRE(p->eps_dsa > 0.0 && p->eps_dsa < 1.0, "eps_dsa must be in (0, 1)");
  RTE_REQUIRE(p->prec == RTE_FP64 || p->prec == RTE_MIXED, "unknown precision");
  if (p->adjoint) {
    RTE_REQUIRE(p->full_rank, "the adjoint solve is full rank only");
  }
  RTE_REQUIRE(p->fold_classes == 0 || p->fold_classes == 1, "fold_classes must be 0 or 1");
  RTE_REQUIRE(p->basis_update >= 0 && p->basis_update <= 2, "basis_update must be 0, 1 or 2");
  RTE_REQUIRE(p->sampling == 0 || p->sampling == 1, "sampling must be 0 (greedy) or 1 (DEIM)");
  if (!p->full_rank) {
    RTE_REQUIRE(p->p >= 1 && p->q >= p->p, "need 1 <= p <= q (p = %d, q = %d)", p->p, p->q);
    RTE_REQUIRE(p->m_max >= 0, "m_max must be >= 0");
    RTE_REQUIRE(p->eps_res >= 0 && p->eps_diff >= 0 && p->eps_svd >= 0 && p->eps_mgs >= 0,
                "thresholds must be >= 0");
    RTE_REQUIRE(p->replay || (p->rand && p->n_rand > 0),
                "the low-rank solver needs a random stream (rand, n_rand) or a replay list");
    RTE_REQUIRE(p->max_rank >= 0, "max_rank must be >= 0");
  }
  (void)prob;
}

void validate_solve_params(const rte_problem* prob, const rte_solve_params* p) {
  validate_params(prob, p);
}

}  // namespace rte

using namespace rte;

extern "C" {

rte_status rte_lowrank_si_dsa_solve(const rte_problem* prob, const rte_solve_params* params,
                                    const double* phi0, double* phi_out, double* X, double* S,
                                    double* V, rte_solve_result* res, void* stream) {
  try {
    StreamScope scope((hipStream_t)stream);
    validate_problem(prob, true, (hipStream_t)stream);
    validate_params(prob, params);
    RTE_REQUIRE(phi_out, "phi_out is NULL");
    hipStream_t st = (hipStream_t)stream;
    if (res) {
      res->outer_iters = res->converged = res->rank = res->n_swept = 0;
      res->mgs_failures = res->breakdowns = res->dsa_iters = res->full_qrs = 0;
      res->fp64_sweeps = 0;
      res->sample_log_len = res->resid_log_len = 0;
      res->ms_sweep = res->ms_lowrank = res->ms_dsa = res->ms_total = 0.0;
    }
    if (params->full_rank) {
      if (params->prec == RTE_FP64) return fr_solve<double>(prob, params, phi0, phi_out, res, st);
      return fr_solve_mixed(prob, params, phi0, phi_out, res, st);
    }
    return lowrank_solve(prob, params, phi0, phi_out, X, S, V, res, st);
  } catch (const Error& e) {
    return e.code;
  }
}

rte_status rte_exit_currents(const rte_problem* prob, const double* phi, double* J, void* stream) {
  try {
    StreamScope scope((hipStream_t)stream);
    validate_problem(prob, true, (hipStream_t)stream);
    RTE_REQUIRE(phi && J, "phi and J are required");
    hipStream_t st = (hipStream_t)stream;
    const Geom g = make_geom(prob);
    DevBuf<double> src(g.ndof), psi((size_t)prob->n_dirs * g.ndof);
    make_source<double>(g, prob->sigma_s, phi, prob->G, src.get(), st);
    launch_sweep<double>(g, all_dirs(prob, g, false), prob->sigma_t, src.get(), prob->bc,
                         psi.get(), nullptr, st);
    std::vector<double> ox(prob->n_dirs), oy(prob->n_dirs);
    for (int j = 0; j < prob->n_dirs; ++j) {
      ox[j] = prob->dirs[3 * j];
      oy[j] = prob->dirs[3 * j + 1];
    }
    DevBuf<double> dox(prob->n_dirs), doy(prob->n_dirs), dw(prob->n_dirs);
    RTE_CHECK_HIP(hipMemcpy(dox.get(), ox.data(), ox.size() * 8, hipMemcpyHostToDevice));
    RTE_CHECK_HIP(hipMemcpy(doy.get(), oy.data(), oy.size() * 8, hipMemcpyHostToDevice));
    RTE_CHECK_HIP(hipMemcpy(dw.get(), prob->wts, ox.size() * 8, hipMemcpyHostToDevice));
    const int nf = 4 * g.mb;
    hipLaunchKernelGGL(exit_current_kernel, dim3((nf + 127) / 128), dim3(128), 0, st, g.nx, g.ny,
                       g.mb, g.hx, g.hy, prob->n_dirs, dox.get(), doy.get(), dw.get(), psi.get(),
                       g.ndof, J);
    RTE_CHECK_HIP(hipGetLastError());
    RTE_CHECK_HIP(hipStreamSynchronize(st));
    return RTE_OK;
  } catch (const Error& e) {
    return e.code;
  }
}

rte_status rte_detector_misfit(const rte_problem* prob, const double* J, const double* J_obs,
                               double* bc_adj, double* loss, void* stream) {
  try {
    StreamScope scope((hipStream_t)stream);
    validate_problem(prob, true, (hipStream_t)stream);
    RTE_REQUIRE(J && J_obs && bc_adj && loss, "missing array");
    hipStream_t st = (hipStream_t)stream;
    const Geom g = make_geom(prob);
    DevBuf<double> dl(1);
    hipLaunchKernelGGL(misfit_kernel, dim3(1), dim3(256), 0, st, g.nx, g.ny, g.mb, g.hx, g.hy, J,
                       J_obs, bc_adj, dl.get());
    RTE_CHECK_HIP(hipGetLastError());
    RTE_CHECK_HIP(hipMemcpyAsync(loss, dl.get(), sizeof(double), hipMemcpyDeviceToHost, st));
    RTE_CHECK_HIP(hipStreamSynchronize(st));
    return RTE_OK;
  } catch (const Error& e) {
    return e.code;
  }
}

rte_status rte_cross_section_gradient(const rte_problem* prob, const double* phi,
                                      const double* phi_adj, const double* bc_adj,
                                      double* grad_sigma_a, double* grad_sigma_s, void* stream) {
  try {
    StreamScope scope((hipStream_t)stream);
    validate_problem(prob, true, (hipStream_t)stream);
    RTE_REQUIRE(phi && phi_adj && grad_sigma_a && grad_sigma_s, "missing array");
    hipStream_t st = (hipStream_t)stream;
    const Geom g = make_geom(prob);
    const size_t tot = (size_t)prob->n_dirs * g.ndof;
    DevBuf<double> src(g.ndof), psi(tot), mu(tot);
    make_source<double>(g, prob->sigma_s, phi, prob->G, src.get(), st);
    launch_sweep<double>(g, all_dirs(prob, g, false), prob->sigma_t, src.get(), prob->bc,
                         psi.get(), nullptr, st);
    make_source<double>(g, prob->sigma_s, phi_adj, nullptr, src.get(), st);
    launch_sweep<double>(g, all_dirs(prob, g, true), prob->sigma_t, src.get(), bc_adj, mu.get(),
                         nullptr, st);
    DevBuf<double> dw(prob->n_dirs);
    RTE_CHECK_HIP(hipMemcpy(dw.get(), prob->wts, prob->n_dirs * 8, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(gradient_kernel, dim3((g.ncell + 255) / 256), dim3(256), 0, st, g.ncell,
                       prob->n_dirs, dw.get(), psi.get(), mu.get(), g.ndof, phi, phi_adj,
                       grad_sigma_a, grad_sigma_s);
    RTE_CHECK_HIP(hipGetLastError());
    RTE_CHECK_HIP(hipStreamSynchronize(st));
    return RTE_OK;
  } catch (const Error& e) {
    return e.code;
  }
}

}  // extern "C"
