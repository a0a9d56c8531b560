// Low-rank SI-DSA (paper Sec. 3, Alg. 1 and Alg. 2) -- internal interface.
#pragma once

#include "common.h"

namespace rte {

std::vector<SweepDir> all_dirs(const rte_problem* p, const Geom& g, bool adjoint);

rte_status lowrank_solve(const rte_problem* prob, const rte_solve_params* prm, const double* phi0,
                         double* phi_out, double* X, double* S, double* V, rte_solve_result* res,
                         hipStream_t st);

}  // namespace rte
