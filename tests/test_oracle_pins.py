"""Pins for the CPU oracle: closed forms, textbook values, derivative
identities, symmetries and invariants that a plausible mistake in the oracle
(a dropped term, a wrong sign or index, a transposed operand) would break.

None of these compares the oracle with itself: each expected value comes from
scipy, numpy, an independent closed form, a textbook table, or a property of
the exact mathematics.
"""
import itertools
import math
import os

import numpy as np
import pytest
from scipy.special import erf

import oracle
from jets import boys_ref, prim_norm, primitive_eri
from paper_2607_05622_amd import synth
from paper_2607_05622_amd.synth import CART, Basis

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Boys ----

@pytest.mark.parametrize("T", [0.0, 1e-6, 0.05, 0.73, 2.5, 9.1, 17.0, 29.999, 30.0, 30.001, 41.0, 120.0])
def test_boys_matches_confluent_hypergeometric(T):
    F = oracle.boys(10, T)
    ref = np.array([boys_ref(m, T) for m in range(11)])
    assert np.max(np.abs(F / ref - 1)) < 2e-14


def test_boys_at_zero_and_asymptote():
    F = oracle.boys(10, 0.0)
    assert np.allclose(F, [1.0 / (2 * m + 1) for m in range(11)], rtol=1e-15, atol=0)
    T = 200.0
    F = oracle.boys(8, T)
    for m in range(9):
        dfm = math.prod(range(2 * m - 1, 0, -2)) if m > 0 else 1.0
        asym = dfm / 2 ** (m + 1) * math.sqrt(math.pi / T ** (2 * m + 1))
        assert abs(F[m] / asym - 1) < 1e-14


def test_boys_erf_closed_form_and_quadrature():
    x, w = np.polynomial.legendre.leggauss(200)
    t = 0.5 * (x + 1)
    w = 0.5 * w
    for T in [0.3, 4.0, 12.0, 25.0, 33.0]:
        F = oracle.boys(6, T)
        assert abs(F[0] - 0.5 * math.sqrt(math.pi / T) * erf(math.sqrt(T))) < 1e-15
        for m in range(7):
            quad = float(np.sum(w * t ** (2 * m) * np.exp(-T * t * t)))
            assert abs(F[m] / quad - 1) < 1e-13


def test_boys_branch_continuity():
    # the two branches meet at T = 30: step across it and remove the
    # first-order change dF_m/dT = -F_{m+1}
    h = 1e-7
    lo = oracle.boys(9, 30.0 - h)
    hi = oracle.boys(9, 30.0 + h)
    pred = hi[:9] + 2 * h * hi[1:10]
    assert np.max(np.abs(lo[:9] / pred - 1)) < 1e-13


# ---------------------------------------------------- textbook (ss|ss) ----

def _read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, *v = line.split()
            vals[k] = [float(x) for x in v]
    return vals


def test_h2_sto3g_textbook_integrals():
    g = _read_golden("h2_sto3g_szabo_ostlund.txt")
    R = g["R"][0]
    b = Basis(np.array([[0, 0, 0], [0, 0, R]], float), np.ones(2), np.array([0, 1], np.int32),
              np.array([0, 0], np.int32), np.array([3, 3], np.int32),
              np.array(g["exps"] * 2), np.array(g["coefs"] * 2), 1)
    S = oracle.overlap(b)
    G = oracle.eri_full(b)
    assert abs(S[0, 1] - g["S12"][0]) < 6e-5
    assert abs(G[0, 0, 0, 0] - g["(11|11)"][0]) < 6e-5
    assert abs(G[0, 0, 1, 1] - g["(11|22)"][0]) < 6e-5
    assert abs(G[1, 0, 0, 0] - g["(21|11)"][0]) < 6e-5
    assert abs(G[1, 0, 1, 0] - g["(21|21)"][0]) < 6e-5


def _ssss_closed_form(centres, ea, ca, eb, cb, ec, cc, ed, cd):
    """Contracted (ss|ss) from the closed form, normalized primitives."""
    A, B, C, D = centres
    tot = 0.0
    for a, wa in zip(ea, ca):
        for b, wb in zip(eb, cb):
            for c, wc in zip(ec, cc):
                for d, wd in zip(ed, cd):
                    p, q = a + b, c + d
                    P = (a * A + b * B) / p
                    Q = (c * C + d * D) / q
                    rho = p * q / (p + q)
                    T = rho * np.sum((P - Q) ** 2)
                    F0 = 1.0 if T == 0 else 0.5 * math.sqrt(math.pi / T) * erf(math.sqrt(T))
                    v = 2 * math.pi ** 2.5 / (p * q * math.sqrt(p + q)) * F0
                    v *= math.exp(-a * b / p * np.sum((A - B) ** 2)) * math.exp(-c * d / q * np.sum((C - D) ** 2))
                    tot += wa * wb * wc * wd * prim_norm(a, 0) * prim_norm(b, 0) * prim_norm(c, 0) * prim_norm(d, 0) * v
    return tot


def _contraction_scale(ex, c, l):
    s = np.array([[(2 * math.sqrt(x * y) / (x + y)) ** (l + 1.5) for y in ex] for x in ex])
    return 1.0 / math.sqrt(c @ s @ c)


def test_contracted_ssss_closed_form():
    rng = np.random.default_rng(11)
    cent = rng.normal(size=(4, 3)) * 1.5
    exps = [np.exp(rng.uniform(np.log(0.15), np.log(50), 3)) for _ in range(4)]
    cofs = [rng.normal(size=3) for _ in range(4)]
    b = Basis(cent, np.ones(4), np.arange(4, dtype=np.int32), np.zeros(4, np.int32),
              np.full(4, 3, np.int32), np.concatenate(exps), np.concatenate(cofs), 1)
    tile = oracle.eri_shell_quartet(b, 0, 1, 2, 3, lambda s: 1)
    w = [c * _contraction_scale(e, c, 0) for e, c in zip(exps, cofs)]
    ref = _ssss_closed_form(cent, exps[0], w[0], exps[1], w[1], exps[2], w[2], exps[3], w[3])
    assert abs(tile[0, 0, 0, 0] / ref - 1) < 1e-13


def test_far_apart_s_shells_coulomb_limit():
    # normalized charge distributions 60 bohr apart interact as 1/R
    R = 60.0
    b = Basis(np.array([[0, 0, 0], [R, 0, 0]], float), np.ones(2), np.array([0, 1], np.int32),
              np.zeros(2, np.int32), np.array([2, 2], np.int32),
              np.array([0.8, 2.3, 1.1, 0.4]), np.array([0.7, 0.4, -0.3, 1.0]), 1)
    t = oracle.eri_shell_quartet(b, 0, 0, 1, 1, lambda s: 1)
    assert abs(t[0, 0, 0, 0] * R - 1) < 1e-14


# ------------------------------------------- p/d via derivative identity ----

CLASSES = [(la, lb, lc, ld) for la in range(3) for lb in range(la + 1)
           for lc in range(3) for ld in range(lc + 1)
           if (la * (la + 1) // 2 + lb) >= (lc * (lc + 1) // 2 + ld)]


@pytest.mark.parametrize("cls", CLASSES)
def test_primitive_eri_equals_derivatives_of_closed_form(cls):
    assert len(CLASSES) == 21
    rng = np.random.default_rng(100 + sum(l * 3 ** i for i, l in enumerate(cls)))
    cent = rng.normal(size=(4, 3)) * 0.9
    ex = list(np.exp(rng.uniform(np.log(0.3), np.log(3.0), 4)))
    ls = list(cls)
    b = Basis(cent, np.ones(4), np.arange(4, dtype=np.int32), np.array(ls, np.int32),
              np.ones(4, np.int32), np.array(ex), np.ones(4), 0)
    tile = oracle.eri_shell_quartet(b, 0, 1, 2, 3, lambda s: len(CART[ls[s]]))
    comps = [range(len(CART[l])) for l in ls]
    allidx = list(itertools.product(*comps))
    pick = [allidx[0], allidx[-1]] + [allidx[i] for i in rng.choice(len(allidx), size=min(4, len(allidx)), replace=False)]
    nrm = math.prod(prim_norm(ex[i], ls[i]) for i in range(4))
    for idx in pick:
        pw = [CART[ls[i]][idx[i]] for i in range(4)]
        ref = primitive_eri(cent, ex, pw) * nrm
        assert abs(tile[idx] - ref) <= 1e-12 * max(abs(ref), 1e-3 * np.max(np.abs(tile)))


# ----------------------------------------------- ERI tensor structure ----

@pytest.fixture(scope="module")
def small_spd():
    b = synth.random_basis(7, 3, 2)   # 3 atoms, s/p/d, pure d
    return b, oracle.eri_full(b)


def test_eight_fold_symmetry(small_spd):
    _, G = small_spd
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)]:
        assert np.max(np.abs(G - G.transpose(perm))) < 1e-13


def test_schwarz_inequality_and_psd(small_spd):
    _, G = small_spd
    n = G.shape[0]
    M = G.reshape(n * n, n * n)
    diag = np.sqrt(np.abs(np.diag(M)))
    assert np.all(np.abs(M) <= np.outer(diag, diag) * (1 + 1e-12) + 1e-14)
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    assert ev.min() >= -1e-12 * ev.max()


# ---------------------------------------------- overlap / normalization ----

def test_overlap_unit_diagonal_and_independent_agreement():
    for sph in (0, 1):
        b = synth.random_basis(21, 4, 2, spherical=sph)
        S = oracle.overlap(b)
        S2 = synth.overlap_matrix(b)      # independent Obara-Saika code
        if sph:
            assert np.max(np.abs(np.diag(S) - 1)) < 1e-13
        else:
            l = np.repeat(b.shell_l, (b.shell_l + 1) * (b.shell_l + 2) // 2)
            # x^l-normalized Cartesians: diag is (2lx-1)!!(2ly-1)!!(2lz-1)!!/(2l-1)!!
            d = []
            for lv in b.shell_l:
                for (x, y, z) in CART[int(lv)]:
                    df = lambda k: math.prod(range(2 * k - 1, 0, -2)) if k > 0 else 1
                    d.append(df(x) * df(y) * df(z) / df(int(lv)))
            assert np.max(np.abs(np.diag(S) - np.array(d))) < 1e-13
            del l
        assert np.max(np.abs(S - S2)) < 1e-13
        assert np.linalg.eigvalsh(S).min() > 0


def test_loewdin_orthonormal():
    w = synth.config0()
    orb = w.meta["orbitals"]
    S = oracle.overlap(w.basis)
    assert np.max(np.abs(orb.C.T @ S @ orb.C - np.eye(S.shape[0]))) < 1e-11


def test_spherical_transform_matches_textbook_constants():
    b = synth.random_basis(5, 2, 1)
    T = oracle.cart_to_basis(b)
    Tref = synth.cart_to_basis_matrix(b)
    assert np.max(np.abs(T - Tref)) < 1e-13


# ------------------------------------------------------ J/K structure ----

@pytest.fixture(scope="module")
def jk_small():
    b = synth.random_basis(9, 3, 2)
    D = synth.random_densities(3, 3, b.nbf())
    J, K = oracle.jk(b, D, 0.0)
    return b, D, J, K


def test_jk_brute_equals_screened_scatter(jk_small):
    b, D, J, K = jk_small
    Jb, Kb = oracle.jk_brute(b, D)
    assert np.max(np.abs(J - Jb)) < 1e-12
    assert np.max(np.abs(K - Kb)) < 1e-12


def test_jk_against_einsum_definition(small_spd):
    b, G = small_spd
    D = synth.random_densities(4, 2, b.nbf())
    J, K = oracle.jk(b, D, 0.0)
    assert np.max(np.abs(J - np.einsum("mnls,xls->xmn", G, D))) < 1e-12
    assert np.max(np.abs(K - np.einsum("mlns,xls->xmn", G, D))) < 1e-12


def test_jk_symmetry_relations(jk_small):
    b, D, J, K = jk_small
    Dt = D.transpose(0, 2, 1).copy()
    Ds = 0.5 * (D + Dt)
    Jt, Kt = oracle.jk(b, Dt, 0.0)
    Js, Ks = oracle.jk(b, Ds, 0.0)
    sc = np.max(np.abs(K))
    assert np.max(np.abs(J - Js)) < 1e-12 * sc          # J depends only on sym(D)
    assert np.max(np.abs(J - J.transpose(0, 2, 1))) < 1e-12 * sc
    assert np.max(np.abs(Kt - K.transpose(0, 2, 1))) < 1e-12 * sc   # K(D^T) = K(D)^T
    assert np.max(np.abs(Ks - Ks.transpose(0, 2, 1))) < 1e-12 * sc
    # the antisymmetric part of D gives an antisymmetric, non-zero K
    Ka = K - Ks
    assert np.max(np.abs(Ka + Ka.transpose(0, 2, 1))) < 1e-12 * sc
    assert np.max(np.abs(Ka)) > 1e-3 * sc


def test_jk_linearity_and_reciprocity(jk_small):
    b, D, J, K = jk_small
    J1, K1 = oracle.jk(b, D[:1], 0.0)
    J2, K2 = oracle.jk(b, D[1:2], 0.0)
    J12, K12 = oracle.jk(b, 2.0 * D[:1] - 0.5 * D[1:2], 0.0)
    assert np.max(np.abs(J12 - (2 * J1 - 0.5 * J2))) < 1e-12
    assert np.max(np.abs(K12 - (2 * K1 - 0.5 * K2))) < 1e-12
    assert abs(np.sum(D[0] * J2[0]) - np.sum(D[1] * J1[0])) < 1e-11
    assert abs(np.sum(D[0] * K2[0]) - np.sum(D[1] * K1[0])) < 1e-11
    Ds = 0.5 * (D[0] + D[0].T)
    Js, _ = oracle.jk(b, Ds, 0.0)
    assert np.sum(Ds * Js[0]) > 0


def test_adversarial_tiny_bases_brute_force():
    # one atom; repeated identical shells (a = b, c = d, ab = cd cases)
    cases = []
    cases.append(synth.random_basis(31, 1, 1))
    b = synth.random_basis(32, 2, 1)
    rep = b.subset([0, 0, 3, 3, 5, 5])
    cases.append(rep)
    cases.append(synth.random_basis(33, 1, 1).subset([5]))       # one d shell
    for bb in cases:
        D = synth.random_densities(7, 2, bb.nbf())
        J, K = oracle.jk(bb, D, 0.0)
        Jb, Kb = oracle.jk_brute(bb, D)
        assert np.max(np.abs(J - Jb)) < 1e-12
        assert np.max(np.abs(K - Kb)) < 1e-12


def test_translation_invariance(jk_small):
    b, D, J, K = jk_small
    J2, K2 = oracle.jk(b.translated([3.1, -1.7, 0.45]), D, 0.0)
    assert np.max(np.abs(J - J2)) < 1e-12
    assert np.max(np.abs(K - K2)) < 1e-12


def test_axis_permutation_covariance():
    # Cartesian basis: (x,y,z) -> (y,z,x) maps each Cartesian component onto
    # another one of the same shell; J and K follow by the same permutation.
    b = synth.random_basis(41, 3, 2, spherical=0)
    D = synth.random_densities(8, 2, b.nbf())
    J, K = oracle.jk(b, D, 0.0)
    b2 = b.translated([0, 0, 0])
    b2.xyz = b.xyz[:, [2, 0, 1]]          # new (x,y,z) = old (z,x,y)
    # old function with powers (lx,ly,lz) becomes new powers (ly,lz,lx)
    perm = []
    off = 0
    for l in b.shell_l:
        comps = CART[int(l)]
        for (lx, ly, lz) in comps:
            perm.append(off + comps.index((lz, lx, ly)))
        off += len(comps)
    perm = np.array(perm)
    # new function perm[i] equals old function i
    D2 = np.zeros_like(D)
    D2[:, perm[:, None], perm[None, :]] = D
    J2, K2 = oracle.jk(b2, D2, 0.0)
    assert np.max(np.abs(J2[:, perm[:, None], perm[None, :]] - J)) < 1e-12
    assert np.max(np.abs(K2[:, perm[:, None], perm[None, :]] - K)) < 1e-12


def test_spherical_route_equals_transformed_integrals():
    b = synth.random_basis(51, 2, 2)
    G = oracle.eri_full(b)               # four-index transform of Cartesian ERIs
    D = synth.random_densities(9, 2, b.nbf())
    J, K = oracle.jk(b, D, 0.0)          # matrix-level T D T^T route
    assert np.max(np.abs(J - np.einsum("mnls,xls->xmn", G, D))) < 1e-12
    assert np.max(np.abs(K - np.einsum("mlns,xls->xmn", G, D))) < 1e-12


# ------------------------------------------------------------- Laplace ----

def test_laplace_identity_is_exact_through_jk():
    w = synth.config0()
    orb = w.meta["orbitals"]
    t = w.meta["t"]
    rng = np.random.default_rng(5)
    T = rng.normal(scale=0.05, size=(orb.n_occ, orb.C.shape[1] - orb.n_occ))
    lo, hi = orb.gap_range()
    wts = synth.laplace_weights(t, lo, hi)
    Dk = np.stack([synth.laplace_density(orb, T, tk) for tk in t])
    delta = orb.e_vir[None, :] - orb.e_occ[:, None]
    E = sum(wk * np.exp(-delta * tk) for wk, tk in zip(wts, t)) - 1.0 / delta
    D_exact = orb.C_occ @ (T / delta) @ orb.C_vir.T
    D_err = orb.C_occ @ (T * E) @ orb.C_vir.T
    Jk, Kk = oracle.jk(w.basis, Dk, 0.0)
    Je, Ke = oracle.jk(w.basis, np.stack([D_exact, D_err]), 0.0)
    lhsJ = np.tensordot(wts, Jk, 1) - Je[0]
    lhsK = np.tensordot(wts, Kk, 1) - Ke[0]
    sc = max(np.max(np.abs(Je[0])), 1e-30)
    assert np.max(np.abs(lhsJ - Je[1])) < 1e-12 * sc + 1e-15
    assert np.max(np.abs(lhsK - Ke[1])) < 1e-12 * max(np.max(np.abs(Ke[0])), 1e-30) + 1e-15
    # and the quadrature's own relative error matches the fitted report
    err = synth.laplace_max_rel_error(t, wts, lo, hi)
    x = delta.ravel()
    fit = np.max(np.abs(x * (np.exp(-np.outer(x, t)) @ wts) - 1))
    assert fit <= err * (1 + 1e-9)


# ----------------------------------------------------------- screening ----

def test_screening_error_within_dropped_bound():
    w = synth.config0()
    b, D = w.basis, w.D
    J0, K0 = oracle.jk(b, D, 0.0)
    tol = 1e-6                          # loose enough that quartets are dropped
    J1, K1 = oracle.jk(b, D, tol)
    n_all = oracle.count_quartets(b, D, 0.0)
    n_kept = oracle.count_quartets(b, D, tol)
    assert n_kept < n_all
    # each dropped quartet contributes at most Q_ab Q_cd Dmax < tol per
    # element for each of its (at most 8) orderings and each function
    # quartet of the tile (<= 3^4 for s/p)
    bound = (n_all - n_kept) * 8 * 81 * tol
    assert np.max(np.abs(J1 - J0)) <= bound
    assert np.max(np.abs(K1 - K0)) <= bound
    J2, K2 = oracle.jk(b, D, 1e-12)
    assert np.max(np.abs(J2 - J0)) < 1e-10
    assert np.max(np.abs(K2 - K0)) < 1e-10


def test_blocks_equal_full_build():
    b = synth.random_basis(61, 3, 2)
    D = synth.random_densities(10, 2, b.nbf())
    J, K = oracle.jk(b, D, 1e-12)
    fo = b.func_offsets()
    pairs = [(0, 0), (4, 1), (5, 12), (13, 5)]
    for (a, c), (Jb, Kb) in zip(pairs, oracle.jk_blocks(b, D, pairs, 1e-12)):
        assert np.max(np.abs(Jb - J[:, fo[a]:fo[a + 1], fo[c]:fo[c + 1]])) < 1e-12
        assert np.max(np.abs(Kb - K[:, fo[a]:fo[a + 1], fo[c]:fo[c + 1]])) < 1e-12


def test_quartet_count_matches_workload_table():
    w = synth.config0()
    assert oracle.count_quartets(w.basis, w.D, 0.0) == 9316


# ------------------------------------------------- screening quantities ----

def _shell_slices(b, cart=True):
    l = np.asarray(b.shell_l)
    n = (l + 1) * (l + 2) // 2 if cart else b.shell_nfunc()
    off = np.concatenate([[0], np.cumsum(n)])
    return [slice(int(off[s]), int(off[s + 1])) for s in range(len(l))]


@pytest.mark.parametrize("seed,atoms,heavy", [(41, 3, 2), (42, 4, 1)])
def test_schwarz_equals_full_tensor_diagonal(seed, atoms, heavy):
    """Q_ab = sqrt(max over m in a, n in b of (mn|mn)), read off the full
    Cartesian ERI tensor (a Cartesian basis, so the tensor's functions are
    the ones the factors are defined over)."""
    b = synth.random_basis(seed, atoms, heavy, spherical=0)
    G = oracle.eri_full(b)
    n = G.shape[0]
    diag = np.einsum("mnmn->mn", G)
    sl = _shell_slices(b)
    ns = len(sl)
    ref = np.array([[math.sqrt(diag[sl[a], sl[c]].max()) for c in range(ns)] for a in range(ns)])
    Q = oracle.schwarz(b)
    assert n == sum(s.stop - s.start for s in sl)
    assert np.max(np.abs(Q - ref) / ref) <= 1e-14
    assert np.all(Q == Q.T)


def _pair_dmax(b, D):
    """Per shell pair, max |D_cart| over the batch and both orientations,
    with D_cart = T D T^T from the input generator's own T."""
    T = synth.cart_to_basis_matrix(b)
    Dc = T[None] @ np.asarray(D).reshape(-1, *np.shape(D)[-2:]) @ T.T[None]
    A = np.max(np.abs(Dc), axis=0)
    A = np.maximum(A, A.T)
    sl = _shell_slices(b)
    return np.array([[A[sa, sb].max() for sb in sl] for sa in sl]), Dc


def _keep(Q, M, a, b_, c, d, tol):
    qq = Q[a, b_] * Q[c, d]
    if qq < tol:
        return False
    m = max(M[a, b_], M[c, d], M[a, c], M[a, d], M[b_, c], M[b_, d])
    return qq * m >= tol


@pytest.mark.parametrize("tol", [0.0, 1e-12, 1e-7, 1e-4])
def test_quartet_count_brute_force(tol):
    """The oracle's count of kept canonical quartets equals a direct
    enumeration of a >= b, c >= d, (ab) >= (cd) with the screening rule
    applied to Schwarz factors read off the full tensor and density maxima
    from the input generator's basis change."""
    for seed, atoms, heavy in [(43, 3, 2), (44, 5, 2)]:
        b = synth.random_basis(seed, atoms, heavy, spherical=0)
        D = synth.random_densities(seed, 3, b.nbf())
        G = oracle.eri_full(b)
        diag = np.einsum("mnmn->mn", G)
        sl = _shell_slices(b)
        ns = len(sl)
        Q = np.array([[math.sqrt(diag[sl[a], sl[c]].max()) for c in range(ns)] for a in range(ns)])
        M, _ = _pair_dmax(b, D)
        pairs = [(a, bb) for a in range(ns) for bb in range(a + 1)]
        n = 0
        for i, (a, bb) in enumerate(pairs):
            for c, d in pairs[:i + 1]:
                n += _keep(Q, M, a, bb, c, d, tol)
        assert oracle.count_quartets(b, D, tol) == n, (seed, tol)


def _dropped_bounds(b, D, blocks, tol):
    """Per element of each requested block (A, B), a bound on what the
    screen drops from J and K (user basis): every dropped (ij|kl) obeys
    |(ij|kl)| <= Q_ab Q_cd (Schwarz), so a dropped quartet moves J_ij by at
    most Q_AB Q_CD sum_{k in C, l in D} |D_kl|, and K_ij likewise through
    the quartet (A C | B D); the spherical transform multiplies by |T|."""
    Q = oracle.schwarz(b)
    M, Dc = _pair_dmax(b, D)
    T = np.abs(synth.cart_to_basis_matrix(b))
    sl, slf = _shell_slices(b), _shell_slices(b, cart=False)
    ns = len(sl)
    absD = np.abs(Dc)
    blk = np.array([[absD[:, sl[c], sl[d]].sum(axis=(1, 2)) for d in range(ns)] for c in range(ns)])  # [C][D][x]
    out = []
    for A, B in blocks:
        bj = np.zeros(Dc.shape[0])
        bk = np.zeros(Dc.shape[0])
        for c in range(ns):
            for d in range(ns):
                if not _keep(Q, M, A, B, c, d, tol):
                    bj += Q[A, B] * Q[c, d] * blk[c, d]
                if not _keep(Q, M, A, c, B, d, tol):
                    bk += Q[A, c] * Q[B, d] * blk[c, d]
        # the bound holds for every Cartesian element of the block; map it
        # through |T| to the basis functions of the block
        ta, tb = T[sl[A], slf[A]], T[sl[B], slf[B]]
        ones = np.ones((sl[A].stop - sl[A].start, sl[B].stop - sl[B].start))
        shape = ta.T @ ones @ tb
        out.append((bj[:, None, None] * shape[None], bk[:, None, None] * shape[None]))
    return out


def test_screening_within_per_element_bound_tiny_workload():
    """Tiny workload, whole matrices: screened minus unscreened J and K,
    element by element, within the dropped-quartet Schwarz bound, at the
    production threshold and at a loose one that drops many quartets."""
    w = synth.config0()
    b, D = w.basis, w.D
    J0, K0 = oracle.jk(b, D, 0.0)
    ns = b.nshells
    blocks = [(a, c) for a in range(ns) for c in range(ns)]
    fo = b.func_offsets()
    for tol in (1e-12, 1e-5):
        J1, K1 = oracle.jk(b, D, tol)
        assert oracle.count_quartets(b, D, tol) < oracle.count_quartets(b, D, 0.0) or tol == 1e-12
        for (a, c), (bj, bk) in zip(blocks, _dropped_bounds(b, D, blocks, tol)):
            s = (slice(None), slice(fo[a], fo[a + 1]), slice(fo[c], fo[c + 1]))
            assert np.all(np.abs(J1[s] - J0[s]) <= bj + 1e-14), (tol, a, c)
            assert np.all(np.abs(K1[s] - K0[s]) <= bk + 1e-14), (tol, a, c)


def test_screening_within_per_element_bound_medium_workload():
    """312-AO workload (16 Laplace pseudo-densities): on sampled shell-pair
    blocks of every pair class, the screened minus unscreened oracle
    blocks lie within the per-element dropped-quartet bound, at the
    production threshold 1e-12 and at a loose 1e-7."""
    w = synth.config1()
    b, D = w.basis, w.D
    l = b.shell_l
    rng = np.random.default_rng(11)
    blocks = []
    for la, lb in [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (0, 2)]:
        A = np.nonzero(l == la)[0]
        B = np.nonzero(l == lb)[0]
        blocks.append((int(A[rng.integers(len(A))]), int(B[rng.integers(len(B))])))
    ref = oracle.jk_blocks(b, D, blocks, 0.0)
    for tol in (1e-12, 1e-7):
        scr = oracle.jk_blocks(b, D, blocks, tol)
        bounds = _dropped_bounds(b, D, blocks, tol)
        for (A, B), (Jr, Kr), (Js, Ks), (bj, bk) in zip(blocks, ref, scr, bounds):
            assert np.all(np.abs(Js - Jr) <= bj + 1e-14), (tol, A, B)
            assert np.all(np.abs(Ks - Kr) <= bk + 1e-14), (tol, A, B)
        if tol == 1e-7:
            # the loose threshold really drops work from these blocks
            assert any(np.max(np.abs(Js - Jr)) > 0 for (Jr, _), (Js, _) in zip(ref, scr))
