"""CPU oracle for the Cholesky-factor (CD) J/K build (test infrastructure
only: the tests, the smoke check and the benchmark's CPU leg may import it).

Plain FP64 numpy on top of the J/K oracle's integrals, sharing nothing with
the GPU library:

* ``cd_matrix`` -- the two-electron operator as a matrix over the basis
  function pairs m >= n, (mn|ls) with the pairs' shell quartets kept by the
  column-fill Schwarz screen Q_ab Q_cd >= screen_tol (the decoupled screen of
  the passage on positive semidefiniteness of the CD operator) and zero
  elsewhere.
* ``pivoted_cholesky`` -- the factor of Eq. (cdfact): textbook pivoted
  Cholesky, one vector per step, pivot = the largest remaining diagonal,
  stop once it is at most the threshold delta.  Near-equal diagonals (within
  a relative 1e-10, e.g. the exactly equal (p_x p_x|p_x p_x) and
  (p_y p_y|p_y p_y) of one atom) go to the lowest pair index, so that two
  implementations whose sums round differently still take the same pivots.
* ``unpack`` -- the factor as symmetric n x n matrices B_Q.
* ``cd_jk`` -- Eq. (cdj) for J and Eq. (cdknonsym) for K of the factored
  densities D = U V^T (Eq. (cdk) is the case U = V).
"""
from __future__ import annotations

import numpy as np

import oracle

# relative window within which remaining diagonals count as equal for the pivot choice
PIVOT_TIE = 1e-10


def function_shells(basis) -> np.ndarray:
    """Shell index of every basis function (functions in shell order)."""
    b = basis.as_arrays() if hasattr(basis, "as_arrays") else basis
    l = np.asarray(b["shell_l"], dtype=np.int64)
    nfunc = 2 * l + 1 if int(b["spherical"]) else (l + 1) * (l + 2) // 2
    return np.repeat(np.arange(l.shape[0]), nfunc)


def pair_index(n: int):
    """Function pairs m >= n in the order m (m + 1) / 2 + n: arrays (m, n)."""
    m, k = np.tril_indices(n)
    return m, k


def cd_matrix(basis, screen_tol: float) -> np.ndarray:
    """V[P][Q] = (mn|ls) for P = (m, n), Q = (l, s), m >= n, l >= s, kept where
    the Schwarz factors of the shell pairs satisfy Q_ab Q_cd >= screen_tol."""
    E = oracle.eri_full(basis)
    n = E.shape[0]
    m, k = pair_index(n)
    V = E[m, k][:, m, k]
    sh = function_shells(basis)
    Qs = oracle.schwarz(basis)
    qp = Qs[sh[m], sh[k]]
    keep = np.outer(qp, qp) >= screen_tol
    return np.where(keep, V, 0.0)


def pivoted_cholesky(V: np.ndarray, delta: float, max_vectors: int | None = None):
    """Rows B[Q] of the factor with V ~ B^T B, and the pivots taken, in order.

    Each step: the pivot p is the (first near-)largest remaining diagonal
    d_p; if d_p <= delta the factor is complete.  The new vector is the
    residual column, (V[:, p] - sum over earlier vectors of B_j B_j[p]),
    divided by sqrt(d_p); the remaining diagonal drops by its square, and
    d_p itself becomes zero."""
    npair = V.shape[0]
    d = np.diag(V).astype(np.float64).copy()
    rows, piv = [], []
    while npair:
        dmax = d.max()
        if not dmax > delta:
            break
        if max_vectors is not None and len(rows) == max_vectors:
            raise ValueError("pivoted_cholesky: more vectors needed than allowed")
        p = int(np.flatnonzero(d >= (1.0 - PIVOT_TIE) * dmax)[0])
        col = V[:, p].copy()
        for r in rows:
            col -= r * r[p]
        b = col / np.sqrt(d[p])
        d -= b * b
        d[p] = 0.0
        rows.append(b)
        piv.append(p)
    B = np.array(rows).reshape(len(rows), npair)
    return B, np.array(piv, dtype=np.int64)


def unpack(B: np.ndarray, n: int) -> np.ndarray:
    """Packed rows [nvec][n (n + 1) / 2] -> symmetric matrices [nvec][n][n]."""
    m, k = pair_index(n)
    out = np.zeros((B.shape[0], n, n))
    out[:, m, k] = B
    out[:, k, m] = B
    return out


def cd_jk(Bf: np.ndarray, U: np.ndarray, V: np.ndarray):
    """J and K of the densities D[x] = U[x] V[x]^T from the factor Bf [nvec][n][n].

    J[x] = sum_Q B_Q gamma_Q[x], gamma_Q[x] = sum_ls B_Q[l][s] D[x][l][s]   (Eq. (cdj))
    K[x] = sum_Q (B_Q U[x]) (B_Q V[x])^T                                   (Eq. (cdknonsym))
    U, V: [nd][n][r]."""
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    nd, n, _r = U.shape
    J = np.zeros((nd, n, n))
    K = np.zeros((nd, n, n))
    for x in range(nd):
        D = U[x] @ V[x].T
        gamma = np.einsum("qls,ls->q", Bf, D, optimize=True)
        J[x] = np.einsum("q,qmn->mn", gamma, Bf, optimize=True)
        BU = Bf @ U[x]      # [nvec][n][r]
        BV = Bf @ V[x]
        K[x] = np.einsum("qmi,qni->mn", BU, BV, optimize=True)
    return J, K
