// Implicit time marching: one backward Euler step (the extension outlined in Sec. 3.7).
//
// With unit particle speed, a step of size dt of
//   d psi/dt + Omega . grad psi + sigma_t psi = sigma_s phi + Q
// is, in the S_N-DG discretisation of Sec. 2.1 (eq. (mat-vec-a)), the steady system with
// the total cross section Sigma_t + M/dt and the extra right-hand side M psi_j^m / dt of
// ordinate j.  The mass matrix M of the orthonormal Legendre basis is the identity, so the
// step is the steady problem with sigma_t + 1/dt per cell plus the angular source
// psi_j^m / dt, and the SI-DSA of Sec. 2.2 or the low-rank SI-DSA of Sec. 3 solves it (the
// DSA on the step's cross sections).
//
// psi^m enters in factor form, psi^m = X_prev diag(S_prev) V_prev^T, the form the
// low-rank step returns, and is the same on the Omega_z twins of a class of equal
// (Omega_x, Omega_y).  Per class c the source is sum_i Xp_i ct[i][c] with
// ct[i][c] = S_prev[i] V_prev[i][rep(c)] / dt.
//   full rank: one sweep of the classes, each with its own source (a per-direction-source
//     sweep plan), psi written, and
//     phi^{n,*} = sum_c w_c psi_c in class order; psi^{m+1} is the psi of the last SI
//     sweep, returned as X = [psi_c], S = 1, V = the class indicator;
//   low rank: the low-rank solver with the angular source in its sweeps, its Galerkin
//     right-hand sides and its candidate residuals; psi^{m+1} = X S V^T of the truncation
//     after the last outer iteration.
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "common.h"
#include "lowrank.h"

namespace rte {
namespace {

__global__ void sigma_step_kernel(long n, const double* __restrict__ sig, double inv_dt,
                                  double* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = sig[i] + inv_dt;
}

// ct[i][c] = S[i] V[i][rep[c]] / dt
__global__ void time_coef_kernel(int rp, int K, const int* __restrict__ rep,
                                 const double* __restrict__ S, const double* __restrict__ V,
                                 int n_dirs, double inv_dt, double* __restrict__ ct) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= K * rp) return;
  const int i = t / K, c = t % K;
  ct[t] = S[i] * V[(size_t)i * n_dirs + rep[c]] * inv_dt;
}

// phi = sum_c w[c] psi[c], in class order
__global__ void class_sum_kernel(long nd, int K, const double* __restrict__ psi,
                                 const double* __restrict__ w, double* __restrict__ phi) {
  const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nd) return;
  double s = 0.0;
  for (int c = 0; c < K; ++c) s += w[c] * psi[(size_t)c * nd + j];
  phi[j] = s;
}

// S = 1, V[c][j] = 1 if ordinate j is in class c
__global__ void class_factors_kernel(int K, int n_dirs, const int* __restrict__ cls_of,
                                     double* __restrict__ S, double* __restrict__ V) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < K) S[t] = 1.0;
  if (t >= K * n_dirs) return;
  const int c = t / n_dirs, j = t % n_dirs;
  V[t] = cls_of[j] == c ? 1.0 : 0.0;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Full-rank SI-DSA of the step problem (sigma_t already shifted by 1/dt in prob).
rte_status fr_time_step(const rte_problem* prob, const rte_solve_params* prm, const TimeSrc& ts,
                        const std::vector<SweepDir>& dirs, const std::vector<int>& cls_of,
                        const double* phi0, double* phi_out, double* X, double* S, double* V,
                        rte_solve_result* res, hipStream_t st) {
  const auto t_start = std::chrono::steady_clock::now();
  const Geom g = make_geom(prob);
  const long nd = g.ndof;
  const int K = (int)dirs.size();
  // one plan over the classes (psi of class c to slot c of X); with psi^m each class has
  // its own source (row c of csrc)
  std::vector<SweepDir> cdirs(dirs);
  for (int c = 0; c < K; ++c) cdirs[c].slot = c;
  const SweepPlan plan = make_sweep_plan(g, cdirs, false, true, sizeof(double), ts.rp > 0);
  DevBuf<SweepDir> ddirs(plan.groups.size());
  RTE_CHECK_HIP(hipMemcpy(ddirs.get(), plan.groups.data(), plan.groups.size() * sizeof(SweepDir),
                          hipMemcpyHostToDevice));
  std::vector<double> hw(K);
  for (int c = 0; c < K; ++c) hw[c] = dirs[c].w;
  DevBuf<double> dw(K), work(sweep_work_elems(g, plan, false)), src(nd), phi_prev(nd), phi_star(nd);
  DevBuf<double> csrc(ts.rp > 0 ? (size_t)K * nd : 0);
  RTE_CHECK_HIP(hipMemcpy(dw.get(), hw.data(), K * sizeof(double), hipMemcpyHostToDevice));
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
  const unsigned nb = (unsigned)((nd + 255) / 256);
  for (n = 1; n <= prm->max_outer; ++n) {
    RTE_CHECK_HIP(hipEventRecord(e0, st));
    make_source<double>(g, prob->sigma_s, phi_prev.get(), prob->G, src.get(), st);
    if (ts.rp > 0) time_class_sources(ts, nullptr, K, nd, src.get(), csrc.get(), nullptr, st);
    sweep_enqueue<double>(g, plan, ddirs.get(), prob->sigma_t, ts.rp > 0 ? csrc.get() : src.get(),
                          prob->bc, X, nullptr, work.get(), st);
    hipLaunchKernelGGL(class_sum_kernel, dim3(nb), dim3(256), 0, st, nd, K, X, dw.get(), phi_star.get());
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
      std::fprintf(stderr, "[rte] backward Euler, full rank: outer %d, |phi* - phi|_inf %.3e, %.0f ms\n",
                   n, d, ms_since(t_start));
    if (d <= prm->eps_si) {
      conv = true;
      break;
    }
    if (n == prm->max_outer) break;
    const auto t0 = std::chrono::steady_clock::now();
    if (dsa) {
      dsa_iters += dsa_apply(dsa.get(), phi_star.get(), phi_prev.get(), phi_prev.get(), prm->eps_dsa, st);
      RTE_CHECK_HIP(hipStreamSynchronize(st));
    } else {
      RTE_CHECK_HIP(hipMemcpyAsync(phi_prev.get(), phi_star.get(), nd * sizeof(double),
                                   hipMemcpyDeviceToDevice, st));
    }
    ms_dsa += ms_since(t0);
  }
  if (n > prm->max_outer) n = prm->max_outer;
  RTE_CHECK_HIP(hipMemcpyAsync(phi_out, phi_star.get(), nd * sizeof(double), hipMemcpyDeviceToDevice, st));
  DevBuf<int> dcls(cls_of.size());
  RTE_CHECK_HIP(hipMemcpyAsync(dcls.get(), cls_of.data(), cls_of.size() * sizeof(int),
                               hipMemcpyHostToDevice, st));
  const long tot = (long)K * prob->n_dirs;
  hipLaunchKernelGGL(class_factors_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, K,
                     prob->n_dirs, dcls.get(), S, V);
  RTE_CHECK_HIP(hipGetLastError());
  RTE_CHECK_HIP(hipStreamSynchronize(st));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (res) {
    res->outer_iters = n;
    res->converged = conv ? 1 : 0;
    res->rank = K;
    res->n_swept = n * K;
    res->dsa_iters = dsa_iters;
    res->ms_sweep = ms_sweep;
    res->ms_dsa = ms_dsa;
    res->ms_lowrank = 0.0;
    res->ms_total = ms_since(t_start);
  }
  return conv ? RTE_OK : RTE_ENOCONV;
}

}  // namespace

void validate_solve_params(const rte_problem* prob, const rte_solve_params* p);

}  // namespace rte

using namespace rte;

extern "C" {

rte_status rte_backward_euler_step(const rte_problem* prob, const rte_solve_params* params,
                                   double dt, int32_t r_prev, const double* X_prev,
                                   const double* S_prev, const double* V_prev, const double* phi0,
                                   double* phi_out, double* X, double* S, double* V,
                                   rte_solve_result* res, void* stream) {
  try {
    hipStream_t st = (hipStream_t)stream;
    StreamScope scope(st);
    validate_problem(prob, true, st);
    validate_solve_params(prob, params);
    RTE_REQUIRE(params->prec == RTE_FP64, "the backward Euler step is FP64 only");
    RTE_REQUIRE(!params->adjoint, "the backward Euler step is a forward solve");
    RTE_REQUIRE(std::isfinite(dt) && dt > 0.0, "dt must be positive and finite");
    RTE_REQUIRE(phi_out && X && S && V, "phi_out, X, S and V must be given");
    RTE_REQUIRE(r_prev >= 0, "r_prev must be >= 0");
    RTE_REQUIRE(r_prev == 0 || (X_prev && S_prev && V_prev), "X_prev, S_prev, V_prev are NULL");
    const Geom g = make_geom(prob);
    const long nd = g.ndof;
    const int N = prob->n_dirs;
    // classes of equal (Omega_x, Omega_y) and their representatives
    std::vector<int> cls_of(N, -1), rep;
    for (int j = 0; j < N; ++j) {
      if (cls_of[j] >= 0) continue;
      cls_of[j] = (int)rep.size();
      for (int i = j + 1; i < N; ++i)
        if (cls_of[i] < 0 && std::fabs(prob->dirs[3 * i] - prob->dirs[3 * j]) <= 1e-12 &&
            std::fabs(prob->dirs[3 * i + 1] - prob->dirs[3 * j + 1]) <= 1e-12)
          cls_of[i] = (int)rep.size();
      rep.push_back(j);
    }
    const int K = (int)rep.size();
    const int cap = params->max_rank > 0 ? params->max_rank : K;
    if (params->full_rank)
      RTE_REQUIRE(cap >= K, "the full-rank step returns psi as %d class columns: max_rank = %d", K,
                  params->max_rank);
    // X must not overlap X_prev (the full-rank step writes psi into X while reading psi^m)
    if (r_prev > 0) {
      const char* a = (const char*)X;
      const char* b = (const char*)X_prev;
      const size_t la = (size_t)cap * nd * sizeof(double), lb = (size_t)r_prev * nd * sizeof(double);
      RTE_REQUIRE(a + la <= b || b + lb <= a, "X must not overlap X_prev");
    }
    // psi^m must be equal on the ordinates of a class (as every psi the library returns)
    if (r_prev > 0) {
      std::vector<double> hv((size_t)r_prev * N);
      RTE_CHECK_HIP(hipMemcpyAsync(hv.data(), V_prev, hv.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      RTE_CHECK_HIP(hipStreamSynchronize(st));
      for (int i = 0; i < r_prev; ++i)
        for (int j = 0; j < N; ++j) {
          const double v = hv[(size_t)i * N + j], vr = hv[(size_t)i * N + rep[cls_of[j]]];
          RTE_REQUIRE(std::isfinite(v), "V_prev is not finite");
          RTE_REQUIRE(v == vr, "V_prev differs between ordinates %d and %d of equal (Omega_x, Omega_y)",
                      j, rep[cls_of[j]]);
        }
    }
    if (res) {
      res->outer_iters = res->converged = res->rank = res->n_swept = 0;
      res->mgs_failures = res->breakdowns = res->dsa_iters = res->full_qrs = 0;
      res->fp64_sweeps = 0;
      res->sample_log_len = res->resid_log_len = 0;
      res->ms_sweep = res->ms_lowrank = res->ms_dsa = res->ms_total = 0.0;
    }
    // the step problem: sigma_t + 1/dt
    DevBuf<double> sig(g.ncell);
    hipLaunchKernelGGL(sigma_step_kernel, dim3((unsigned)((g.ncell + 255) / 256)), dim3(256), 0, st,
                       g.ncell, prob->sigma_t, 1.0 / dt, sig.get());
    RTE_CHECK_HIP(hipGetLastError());
    rte_problem p2 = *prob;
    p2.sigma_t = sig.get();
    validate_problem(&p2, true, st);
    // the angular source per class
    TimeSrc ts;
    DevBuf<double> ct;
    if (r_prev > 0) {
      DevBuf<int> drep(K);
      RTE_CHECK_HIP(hipMemcpyAsync(drep.get(), rep.data(), K * sizeof(int), hipMemcpyHostToDevice, st));
      ct.alloc((size_t)K * r_prev);
      hipLaunchKernelGGL(time_coef_kernel, dim3((unsigned)(((long)K * r_prev + 255) / 256)), dim3(256), 0,
                         st, r_prev, K, drep.get(), S_prev, V_prev, N, 1.0 / dt, ct.get());
      RTE_CHECK_HIP(hipGetLastError());
      RTE_CHECK_HIP(hipStreamSynchronize(st));
      ts.rp = r_prev;
      ts.K = K;
      ts.Xp = X_prev;
      ts.ct = ct.get();
    }
    if (params->full_rank) {
      std::vector<SweepDir> dirs = class_dirs(&p2, g);
      return fr_time_step(&p2, params, ts, dirs, cls_of, phi0, phi_out, X, S, V, res, st);
    }
    return lowrank_solve(&p2, params, phi0, phi_out, X, S, V, res, st, &ts);
  } catch (const Error& e) {
    return e.code;
  }
}

}  // extern "C"
