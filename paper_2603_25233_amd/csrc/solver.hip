// SI-DSA solver entry points (full-rank and low-rank, Alg. 1).
#include "common.h"

using namespace rte;

extern "C" {

rte_status rte_lowrank_si_dsa_solve(const rte_problem*, const rte_solve_params*, const double*,
                                    double*, double*, double*, double*, rte_solve_result*,
                                    void*) {
  set_error("rte_lowrank_si_dsa_solve: not available yet");
  return RTE_EINVAL;
}

rte_status rte_exit_currents(const rte_problem*, const double*, double*, void*) {
  set_error("rte_exit_currents: not available yet");
  return RTE_EINVAL;
}

rte_status rte_cross_section_gradient(const rte_problem*, const double*, const double*,
                                      const double*, double*, double*, void*) {
  set_error("rte_cross_section_gradient: not available yet");
  return RTE_EINVAL;
}

}  // extern "C"
