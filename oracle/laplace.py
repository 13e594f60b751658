"""CPU oracle for the Laplace cascade around the J/K build (test
infrastructure only: the tests, the smoke check and the benchmark's CPU
leg may import it).

Plain FP64 numpy, written from the paper and sharing nothing with the GPU
library:

* ``minimax_grid`` -- the best uniform approximation of 1/x on
  [xmin, xmax] by an n-term exponential sum (Sect. 2, Eq. (laplace) and the
  minimax-grid paragraph), found here by a different method from the
  library's exchange: for fixed nodes the best weights are a linear
  program over a dense sample (the epigraph form of the max-error
  minimization), and the nodes minimize that LP optimum (Nelder-Mead in log
  t).  Practical for a few nodes only.
* ``alternation`` -- the extrema of an error curve, for the characterization
  of the best approximation (2n + 1 alternating extrema of equal size).
* ``scaled_coefficients`` -- Eq. (scaledcoeff).
* ``level_density`` -- Eq. (aodensk) (Eq. (aodens) with R the amplitudes).
* ``laplace_fock`` -- Eq. (laplacefock).
* ``cascade_step`` -- one forward edge of the level-k loop of Algorithm
  ltao: J/K build (the J/K oracle), back-transform, occupied-virtual block,
  next-level densities on the grid.
"""
from __future__ import annotations

import numpy as np


def error_curve(tau, w, x):
    """1/x - sum_k w_k exp(-x tau_k)."""
    return 1.0 / x - np.exp(-np.outer(x, tau)) @ w


def _best_weights(tau, x):
    """min over w of max_j |1/x_j - sum_k w_k exp(-x_j tau_k)| as an LP in
    (w, E): minimize E subject to -E <= error_j <= E."""
    from scipy.optimize import linprog
    n = len(tau)
    A = np.exp(-np.outer(x, tau))
    b = 1.0 / x
    # error_j = b_j - A_j w;  b - A w <= E  ->  -A w - E <= -b ;  A w - b <= E -> A w - E <= b
    ones = np.ones((len(x), 1))
    A_ub = np.vstack([np.hstack([-A, -ones]), np.hstack([A, -ones])])
    b_ub = np.concatenate([-b, b])
    c = np.zeros(n + 1)
    c[-1] = 1.0
    res = linprog(c, A_ub=A_ub, b_ub=b_ub, bounds=[(None, None)] * n + [(0, None)], method="highs")
    if not res.success:
        return np.full(n, np.nan), np.inf
    return res.x[:n], res.x[-1]


def minimax_grid(n: int, xmin: float, xmax: float, nsample: int = 400, start=None, polish: int = 1):
    """(tau, w, err): the n-term minimax grid for 1/x on [xmin, xmax]
    (scaled to [1, R] internally).  ``start`` optionally gives initial nodes
    on [xmin, xmax]."""
    from scipy.optimize import minimize
    R = xmax / xmin
    x = np.exp(np.linspace(0.0, np.log(R), nsample))
    if start is None:
        lt0 = np.linspace(-np.log(R) - 0.5, 1.0, n) if n > 1 else np.array([-0.5 * np.log(R) - 0.5])
    else:
        lt0 = np.log(np.asarray(start) * xmin)

    def f(lt):
        return _best_weights(np.exp(lt), x)[1]

    lt = lt0
    for _ in range(1 + polish):   # a restart polishes the simplex
        fa = 1e-9 * f(lt)
        best = minimize(f, lt, method="Nelder-Mead", options=dict(xatol=1e-8, fatol=fa, maxfev=800 * n))
        lt = best.x
    tau = np.sort(np.exp(lt))
    w, _ = _best_weights(tau, x)
    xs = np.exp(np.linspace(0.0, np.log(R), 20 * nsample))
    err = float(np.max(np.abs(error_curve(tau, w, xs))))
    return tau / xmin, w / xmin, err / xmin


def alternation(tau, w, xmin: float, xmax: float, nsample: int = 200000):
    """Values of the error curve at its local extrema (both ends included),
    merged so that neighbours alternate in sign (the larger kept)."""
    x = np.exp(np.linspace(np.log(xmin), np.log(xmax), nsample))
    e = error_curve(np.asarray(tau), np.asarray(w), x)
    # slope signs, a zero difference (flat to rounding) taking the sign before it
    sg = np.sign(np.diff(e))
    for j in range(1, len(sg)):
        if sg[j] == 0:
            sg[j] = sg[j - 1]
    idx = [0] + [j for j in range(1, len(sg)) if sg[j] != sg[j - 1] and sg[j - 1] != 0] + [len(e) - 1]
    vals = []
    for j in idx:
        v = e[j]
        if vals and np.sign(vals[-1]) == np.sign(v):
            if abs(v) > abs(vals[-1]):
                vals[-1] = v
        else:
            vals.append(v)
    return np.array(vals)


def scaled_coefficients(C, eps, nocc: int, tau: float):
    """Eq. (scaledcoeff): U = C_occ diag(exp(+eps_i tau)), V = C_vir diag(exp(-eps_a tau))."""
    U = C[:, :nocc] * np.exp(eps[:nocc] * tau)[None, :]
    V = C[:, nocc:] * np.exp(-eps[nocc:] * tau)[None, :]
    return U, V


def level_density(C, eps, nocc: int, tau: float, R):
    """Eq. (aodensk): sum_ia U_{mu i} R_{ia} V_{nu a}."""
    U, V = scaled_coefficients(C, eps, nocc, tau)
    return U @ R @ V.T


def laplace_fock(C, J, K):
    """Eq. (laplacefock): C^T (2J - K) C."""
    return C.T @ (2.0 * J - K) @ C


def cascade_step(basis, D, C, eps, nocc: int, tau, tol: float = 1e-12):
    """(J, K, Rov, Dnext) of one forward edge for densities D[nd, n, n]."""
    import oracle
    J, K = oracle.jk(basis, D, tol)
    Rov = np.stack([laplace_fock(C, J[x], K[x])[:nocc, nocc:] for x in range(D.shape[0])])
    Dn = np.stack([np.stack([level_density(C, eps, nocc, t, Rov[x]) for t in tau]) for x in range(D.shape[0])])
    return J, K, Rov, Dn
