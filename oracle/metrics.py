"""Reporting metrics of Sec. 4 (speedup, compression ratio, oversampling, effective rank)."""
import numpy as np

from .lowrank import truncation_rank


def compression_ratio(rank, n_x, n_omega):
    """DOFs of X S V^T over DOFs of Psi: r (N_x + N_Omega + 1) / (N_x N_Omega), Sec. 4.

    X has N_x r entries, V has N_Omega r, the diagonal core S has r.
    """
    return rank * (n_x + n_omega + 1) / (n_x * n_omega)


def oversampling(n_sampled, rank):
    """(number of sampled angles - solution rank) / solution rank, Sec. 4."""
    return (n_sampled - rank) / rank


def effective_rank(psi_matrix, eps_svd):
    """Rank of the full-rank Psi (N_x x N_Omega) under the same truncation rule (Sec. 4.3)."""
    s = np.linalg.svd(np.asarray(psi_matrix, dtype=np.float64), compute_uv=False)
    return truncation_rank(s, eps_svd)
