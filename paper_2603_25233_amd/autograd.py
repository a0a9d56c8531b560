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


class DetectorMisfitBatch(torch.autograd.Function):
    """Sum over source configurations s of the misfits L_s of DetectorMisfit: each
    configuration has its own inflow data bc[s] (the sources of an optical-tomography
    experiment) and observations J_obs[s].  forward: one forward solve, exit currents
    and misfit per configuration; backward: one adjoint solve and gradient each, summed."""

    @staticmethod
    def forward(ctx, sigma_a, sigma_s, base, bcs, J_obs, solve_kw):
        sig_t = sigma_a.detach() + sigma_s.detach()
        total = 0.0
        Js, saved = [], []
        for s in range(bcs.shape[0]):
            prob = rte.Problem(base.nx, base.ny, base.domain, base.dirs, base.wts, sig_t,
                               sigma_s.detach(), G=base.G, bc=bcs[s], device=base.device)
            fw = rte.solve(prob, full_rank=1, **solve_kw)
            J = rte.exit_currents(prob, fw["phi"])
            loss, bc_adj = rte.detector_misfit(prob, J, J_obs[s])
            total += loss
            Js.append(J)
            saved.append((prob, fw["phi"], bc_adj))
        ctx.saved, ctx.solve_kw = saved, solve_kw
        J = torch.stack(Js)
        ctx.mark_non_differentiable(J)
        return torch.tensor(total, dtype=torch.float64, device=sigma_a.device), J

    @staticmethod
    def backward(ctx, g_loss, g_J):
        ga_sum = gs_sum = None
        for prob, phi, bc_adj in ctx.saved:
            ad = rte.solve(prob, full_rank=1, adjoint=1, G_override=None, bc_override=bc_adj,
                           **ctx.solve_kw)
            ga, gs = rte.cross_section_gradient(prob, phi, ad["phi"], bc_adj)
            ga_sum = ga if ga_sum is None else ga_sum + ga
            gs_sum = gs if gs_sum is None else gs_sum + gs
        ctx.saved = None
        return g_loss * ga_sum, g_loss * gs_sum, None, None, None, None


def detector_misfit_batch(sigma_a, sigma_s, base, bcs, J_obs, **solve_kw):
    """(sum_s L_s, J [S][4][max(nx,ny)]) for inflow data bcs [S][4][max(nx,ny)][2] and
    observations J_obs [S][4][max(nx,ny)]; differentiable in sigma_a and sigma_s."""
    kw = dict(eps_si=1e-12, max_outer=2000, eps_dsa=1e-13)
    kw.update(solve_kw)
    bcs = torch.as_tensor(bcs, dtype=torch.float64, device=base.device).contiguous()
    J_obs = torch.as_tensor(J_obs, dtype=torch.float64, device=base.device).contiguous()
    return DetectorMisfitBatch.apply(sigma_a, sigma_s, base, bcs, J_obs, kw)


def detector_misfit(sigma_a, sigma_s, base, J_obs, **solve_kw):
    """(L, J) with L differentiable in sigma_a and sigma_s ([ny][nx] float64 tensors)."""
    kw = dict(eps_si=1e-12, max_outer=2000, eps_dsa=1e-13)
    kw.update(solve_kw)
    return DetectorMisfit.apply(sigma_a, sigma_s, base, J_obs, kw)
