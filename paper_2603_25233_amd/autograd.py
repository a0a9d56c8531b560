"""torch.autograd binding of the boundary-detector misfit and its adjoint gradient.

forward: full-rank SI-DSA forward solve, exit currents J and
    L = 1/2 sum_e (J_e - J_obs,e)^2 (rte_lowrank_si_dsa_solve, rte_exit_currents,
    rte_detector_misfit);
backward: adjoint SI-DSA solve with the adjoint boundary data and
    dL/dsigma_a, dL/dsigma_s per cell (rte_lowrank_si_dsa_solve with adjoint = 1,
    rte_cross_section_gradient).
The gradient is that of the discrete fixed point (implicit differentiation); every
step runs in librte.so.
"""
import torch

from . import rte


class DetectorMisfit(torch.autograd.Function):
    """L(sigma_a, sigma_s) for a problem template (geometry, ordinates, source, inflow)."""

    @staticmethod
    def forward(ctx, sigma_a, sigma_s, base, J_obs, solve_kw):
        prob = rte.Problem(base.nx, base.ny, base.domain, base.dirs, base.wts,
                           sigma_a.detach() + sigma_s.detach(), sigma_s, G=base.G, bc=base.bc,
                           device=base.device)
        fw = rte.solve(prob, full_rank=1, **solve_kw)
        J = rte.exit_currents(prob, fw["phi"])
        loss, bc_adj = rte.detector_misfit(prob, J, J_obs)
        ctx.prob, ctx.solve_kw = prob, solve_kw
        ctx.save_for_backward(fw["phi"], bc_adj)
        ctx.mark_non_differentiable(J)
        return torch.tensor(loss, dtype=torch.float64, device=sigma_a.device), J

    @staticmethod
    def backward(ctx, g_loss, g_J):
        phi, bc_adj = ctx.saved_tensors
        ad = rte.solve(ctx.prob, full_rank=1, adjoint=1, G_override=None, bc_override=bc_adj,
                       **ctx.solve_kw)
        ga, gs = rte.cross_section_gradient(ctx.prob, phi, ad["phi"], bc_adj)
        return g_loss * ga, g_loss * gs, None, None, None


def detector_misfit(sigma_a, sigma_s, base, J_obs, **solve_kw):
    """(L, J) with L differentiable in sigma_a and sigma_s ([ny][nx] float64 tensors)."""
    kw = dict(eps_si=1e-12, max_outer=2000, eps_dsa=1e-13)
    kw.update(solve_kw)
    return DetectorMisfit.apply(sigma_a, sigma_s, base, J_obs, kw)
