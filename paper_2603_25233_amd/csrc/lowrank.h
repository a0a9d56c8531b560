// Low-rank SI-DSA (paper Sec. 3, Alg. 1 and Alg. 2) -- internal interface.
#pragma once

#include "common.h"

namespace rte {

std::vector<SweepDir> all_dirs(const rte_problem* p, const Geom& g, bool adjoint);

// One direction per class of equal (Omega_x, Omega_y), numbered by the smallest member,
// with the class's summed weight; slot = class index.
std::vector<SweepDir> class_dirs(const rte_problem* p, const Geom& g);

// The angular source psi^m / dt of a backward Euler step (FP64), per class c of equal
// (Omega_x, Omega_y): psi^m_c / dt = Xp ct[c], Xp [rp][ndof] (column i contiguous),
// ct [K][rp] (DEV).  rp = 0: no source.
struct TimeSrc {
  int rp = 0;
  const double* Xp = nullptr;
  const double* ct = nullptr;
};
// out = src + Xp ct[c] (fixed summation order)
void time_class_source(const TimeSrc& ts, int c, long nd, const double* src, double* out,
                       hipStream_t st);

rte_status lowrank_solve(const rte_problem* prob, const rte_solve_params* prm, const double* phi0,
                         double* phi_out, double* X, double* S, double* V, rte_solve_result* res,
                         hipStream_t st, const TimeSrc* ts = nullptr);

}  // namespace rte
