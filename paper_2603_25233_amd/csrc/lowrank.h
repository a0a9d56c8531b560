// Low-rank SI-DSA (paper Sec. 3, Alg. 1 and Alg. 2) -- internal interface.
#pragma once

#include "common.h"

namespace rte {

std::vector<SweepDir> all_dirs(const rte_problem* p, const Geom& g, bool adjoint);

// One direction per class of equal (Omega_x, Omega_y), numbered by the smallest member,
// with the class's summed weight; slot = class index.
std::vector<SweepDir> class_dirs(const rte_problem* p, const Geom& g);

// The angular source psi^m / dt of a backward Euler step (FP64), per class c of equal
// (Omega_x, Omega_y): psi^m_c / dt = sum_i Xp_i ct[i][c], Xp [rp][ndof] (column i
// contiguous), ct [rp][K] (DEV).  rp = 0: no source.
struct TimeSrc {
  int rp = 0, K = 0;
  const double* Xp = nullptr;
  const double* ct = nullptr;
};
// out[m] = src + psi^m_{cls[m]} / dt for m < nm (fixed summation order; cls: DEV class
// list with ctm a DEV workspace of rp nm doubles, or null for classes 0 .. nm - 1)
void time_class_sources(const TimeSrc& ts, const int* cls_dev, int nm, long nd, const double* src,
                        double* out, double* ctm, hipStream_t st);

rte_status lowrank_solve(const rte_problem* prob, const rte_solve_params* prm, const double* phi0,
                         double* phi_out, double* X, double* S, double* V, rte_solve_result* res,
                         hipStream_t st, const TimeSrc* ts = nullptr);

}  // namespace rte
