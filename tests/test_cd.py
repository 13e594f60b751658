"""Pins of the CD (Cholesky-factor) J/K oracle, Eqs. (cdfact)-(cdknonsym):
checked against the direct J/K oracle, LAPACK's Cholesky and the bounds a
pivoted Cholesky factor of a positive semidefinite matrix obeys."""
import numpy as np
import pytest
from scipy.linalg import solve_triangular

import oracle
from oracle import cd
from paper_2607_05622_amd import synth


@pytest.fixture(scope="module")
def small():
    b = synth.random_basis(5151, 3, 2)
    return b, cd.cd_matrix(b, 0.0)


def test_screen_off_is_the_full_operator(small):
    b, V = small
    E = oracle.eri_full(b)
    n = E.shape[0]
    # pair (m, n) at m (m + 1) / 2 + n; spot entries by hand
    for (m, k, l, s) in [(0, 0, 0, 0), (5, 2, 7, 7), (n - 1, 0, n - 2, n - 3), (9, 9, 4, 1)]:
        P, Q = m * (m + 1) // 2 + k, l * (l + 1) // 2 + s
        assert V[P, Q] == E[m, k, l, s]
        assert abs(E[k, m, s, l] - E[m, k, l, s]) <= 1e-14 * abs(E[m, k, l, s]) + 1e-16
    assert np.abs(V - V.T).max() <= 1e-13 * np.abs(V).max()
    assert np.linalg.eigvalsh(V).min() > -1e-12      # an ERI metric is positive semidefinite


def test_column_fill_screen_zeroes_exactly_the_screened_quartets():
    # Cartesian functions: the Schwarz factors bound their integrals
    b = synth.random_basis(5152, 4, 2, spherical=0)
    tol = 1e-4
    V0, V = cd.cd_matrix(b, 0.0), cd.cd_matrix(b, tol)
    sh = cd.function_shells(b)
    Q = oracle.schwarz(b)
    m, k = cd.pair_index(sh.shape[0])
    q = Q[sh[m], sh[k]]
    kept = np.outer(q, q) >= tol
    assert 0 < kept.sum() < kept.size
    assert np.array_equal(V[kept], V0[kept]) and not V[~kept].any()
    # every dropped entry obeys its Schwarz bound |(mn|ls)| <= Q_ab Q_cd < tol
    assert np.abs(V0[~kept]).max() < tol


@pytest.mark.parametrize("delta", [1e-2, 1e-4, 1e-7])
def test_residual_is_bounded_by_delta(small, delta):
    _b, V = small
    B, piv = cd.pivoted_cholesky(V, delta)
    R = V - B.T @ B
    # the residual of a pivoted Cholesky factor is positive semidefinite with
    # diagonal <= delta, so every entry is at most delta in size
    assert np.diag(R).max() <= delta * (1 + 1e-9)
    assert np.abs(R).max() <= delta * (1 + 1e-9) + 1e-13
    assert np.linalg.eigvalsh(R).min() > -1e-11
    assert len(set(piv.tolist())) == len(piv)


def test_rank_grows_as_delta_shrinks(small):
    _b, V = small
    ns = [cd.pivoted_cholesky(V, d)[0].shape[0] for d in (1e-1, 1e-3, 1e-5, 1e-8)]
    assert ns == sorted(ns) and ns[0] < ns[-1] <= V.shape[0]
    assert cd.pivoted_cholesky(V, 10 * np.diag(V).max())[0].shape[0] == 0


def test_factor_is_lapack_cholesky_of_the_pivoted_block(small):
    """On its pivots S the factor is the lower Cholesky factor of V[S, S]
    (LAPACK), and elsewhere the triangular solve of V[S, :] against it."""
    _b, V = small
    B, piv = cd.pivoted_cholesky(V, 1e-6)
    L = np.linalg.cholesky(V[np.ix_(piv, piv)])
    assert np.allclose(B[:, piv], L.T, rtol=0, atol=1e-11)
    X = solve_triangular(L, V[piv, :], lower=True)
    assert np.allclose(B, X, rtol=0, atol=1e-9)


def test_pivots_are_the_largest_remaining_diagonals(small):
    _b, V = small
    B, piv = cd.pivoted_cholesky(V, 1e-5)
    d = np.diag(V).copy()
    for k, p in enumerate(piv):
        assert d[p] >= d.max() * (1 - cd.PIVOT_TIE)
        d = np.diag(V) - (B[: k + 1] ** 2).sum(0)
        assert abs(d[p]) < 1e-12


def test_max_vectors_is_enforced(small):
    _b, V = small
    with pytest.raises(ValueError):
        cd.pivoted_cholesky(V, 1e-8, max_vectors=3)


@pytest.mark.parametrize("spherical", [1, 0])
def test_cd_jk_of_a_full_factor_is_the_direct_build(spherical):
    """With delta far below the operator's scale the CD J and K equal the
    direct build of Eq. (jkbuild) for D = U V^T (catches a transposed K)."""
    b = synth.random_basis(5153 + spherical, 3, 2, spherical=spherical)
    n = b.nbf()
    V = cd.cd_matrix(b, 0.0)
    B, _ = cd.pivoted_cholesky(V, 1e-13)
    U, W = synth.random_factors(77, 2, n, 4)
    J, K = cd.cd_jk(cd.unpack(B, n), U, W)
    D = np.einsum("xmi,xni->xmn", U, W)
    Jd, Kd = oracle.jk(b, D, tol=0.0)
    for x in range(2):
        assert np.abs(J[x] - Jd[x]).max() <= 1e-9 * np.abs(Jd[x]).max()
        assert np.abs(K[x] - Kd[x]).max() <= 1e-9 * np.abs(Kd[x]).max()
    assert not np.allclose(K[0], K[0].T, atol=1e-6)   # non-symmetric D: K is not symmetric


def test_cd_jk_error_follows_the_residual(small):
    """|J_cd - J| <= delta sum |D| entrywise (|R| <= delta), and the symmetric
    case U = V of Eq. (cdk) gives a symmetric K."""
    b, V = small
    n = b.nbf()
    delta = 1e-4
    B, _ = cd.pivoted_cholesky(V, delta)
    U, W = synth.random_factors(78, 1, n, 3)
    J, K = cd.cd_jk(cd.unpack(B, n), U, W)
    D = U[0] @ W[0].T
    Jd, Kd = oracle.jk(b, D[None], tol=0.0)
    assert np.abs(J[0] - Jd[0]).max() <= delta * np.abs(D).sum()
    assert np.abs(K[0] - Kd[0]).max() <= delta * np.abs(D).sum()
    _J, Ks = cd.cd_jk(cd.unpack(B, n), U, U)
    assert np.allclose(Ks[0], Ks[0].T, rtol=0, atol=1e-13)


def test_unpack_layout():
    B = np.arange(6.0)[None]
    F = cd.unpack(B, 3)
    assert np.array_equal(F[0], np.array([[0, 1, 3], [1, 2, 4], [3, 4, 5]], dtype=float))
