"""Earth Mover's Distance between vector sets, exact and entropic -- TEST INFRASTRUCTURE ONLY.

Restates from the paper (GEM, arXiv 2603.20336, Sec. 4.2):
  * EMD(P1, P2) = min over transport plans T of sum_ij t_ij d(p_i, p'_j),
    subject to sum_j t_ij = 1 / m1, sum_i t_ij = 1 / m2, t_ij >= 0 (Eq. EMD);
  * qEMD: the same with d(NN(p_i), NN(p'_j)) for the nearest centroids of
    C_quant (Eq. qEMD) -- here the sets are handed over as their centroid rows;
  * the bound CH <= EMD, with the Chamfer distance averaged over the first
    set: (1 / m1) sum_i min_j d(p_i, p'_j).

Readings (listed in the design notes): d is the Euclidean distance (a metric,
as the triangle-inequality argument of Sec. 4.2 needs). The GPU computes the
entropic approximation of Cuturi ("Sinkhorn Distances", NIPS 2013) in the
log domain: from g = 0, n_iter rounds of
    f_i <- log(1 / m1) - logsumexp_j (g_j - C_ij / eps)
    g_j <- log(1 / m2) - logsumexp_i (f_i - C_ij / eps)
and the cost sum_ij exp(f_i + g_j - C_ij / eps) C_ij of the resulting plan.
"""
from __future__ import annotations

import numpy as np


def _f64(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64)


def cost_matrix(A, B) -> np.ndarray:
    """Euclidean distances d(a_i, b_j), each summed term by term in float64."""
    A, B = _f64(A), _f64(B)
    diff = A[:, None, :] - B[None, :, :]
    return np.sqrt((diff * diff).sum(axis=2))


def emd_exact(A, B) -> float:
    """The transport problem of Sec. 4.2 solved as a linear program (SciPy's HiGHS)."""
    from scipy.optimize import linprog
    C = cost_matrix(A, B)
    m1, m2 = C.shape
    rows = np.zeros((m1, m1 * m2))
    cols = np.zeros((m2, m1 * m2))
    for i in range(m1):
        rows[i, i * m2:(i + 1) * m2] = 1.0
    for j in range(m2):
        cols[j, j::m2] = 1.0
    A_eq = np.vstack([rows, cols])
    b_eq = np.concatenate([np.full(m1, 1.0 / m1), np.full(m2, 1.0 / m2)])
    res = linprog(C.reshape(-1), A_eq=A_eq, b_eq=b_eq, bounds=(0, None), method="highs")
    if not res.success:
        raise RuntimeError(res.message)
    return float(res.fun)


def _lse(x, axis):
    m = x.max(axis=axis, keepdims=True)
    return (m + np.log(np.exp(x - m).sum(axis=axis, keepdims=True))).squeeze(axis)


def sinkhorn(A, B, eps: float, n_iter: int, return_plan: bool = False):
    """Entropic EMD after n_iter log-domain Sinkhorn rounds (Cuturi 2013), float64."""
    C = cost_matrix(A, B)
    m1, m2 = C.shape
    K = -C / eps
    f = np.zeros(m1)
    g = np.zeros(m2)
    for _ in range(n_iter):
        f = np.log(1.0 / m1) - _lse(g[None, :] + K, axis=1)
        g = np.log(1.0 / m2) - _lse(f[:, None] + K, axis=0)
    T = np.exp(f[:, None] + g[None, :] + K)
    cost = float((T * C).sum())
    return (cost, T) if return_plan else cost


def chamfer_distance(A, B) -> float:
    """(1 / m1) sum_i min_j d(a_i, b_j): the Chamfer distance that EMD bounds from above."""
    return float(cost_matrix(A, B).min(axis=1).mean())
