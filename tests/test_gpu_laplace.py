"""GPU parity of the Laplace cascade around the J/K build (Sect. 2): the
level-k densities, the Laplace-Fock back-transform and one forward edge of
the cascade through the C-ABI, against the CPU oracle (oracle/laplace.py and
the J/K oracle).  Bars: the dense steps are FP64 products, checked at 1e-12
of the largest element; a forward edge inherits the J/K bar (1e-10
absolute) and is checked at 1e-9 of the largest element."""
import numpy as np
import pytest

import oracle
from oracle import laplace as L
from paper_2607_05622_amd import jk, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def _t(a, dev):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def _relmax(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("n,nocc,nr,ntau", [(28, 9, 3, 5), (150, 21, 2, 3), (129, 64, 1, 7)])
def test_level_densities(dev, n, nocc, nr, ntau):
    rng = np.random.default_rng(n + nocc)
    C = rng.normal(size=(n, n)) / np.sqrt(n)
    eps = np.concatenate([np.sort(rng.uniform(-1.5, -0.3, nocc)), np.sort(rng.uniform(0.1, 3.0, n - nocc))])
    R = rng.normal(size=(nr, nocc, n - nocc))
    tau, _, _ = jk.jk_laplace_grid(ntau, 0.4, 4.5)
    D = jk.jk_laplace_densities(_t(C, dev), _t(eps, dev), nocc, tau, _t(R, dev)).cpu().numpy()
    for r in range(nr):
        for k, t in enumerate(tau):
            ref = L.level_density(C, eps, nocc, t, R[r])
            assert _relmax(D[r, k], ref) <= 1e-12, (r, k)


@pytest.mark.parametrize("n,nocc,nd", [(28, 9, 2), (150, 21, 3), (200, 65, 70)])
def test_back_transform(dev, n, nocc, nd):
    rng = np.random.default_rng(7 * n + nd)
    C = rng.normal(size=(n, n)) / np.sqrt(n)
    J = rng.normal(size=(nd, n, n))
    K = rng.normal(size=(nd, n, n))
    F, Rov = jk.jk_laplace_fock(_t(C, dev), nocc, _t(J, dev), _t(K, dev))
    F, Rov = F.cpu().numpy(), Rov.cpu().numpy()
    for x in range(nd):
        ref = L.laplace_fock(C, J[x], K[x])
        assert _relmax(F[x], ref) <= 1e-12, x
        assert _relmax(Rov[x], ref[:nocc, nocc:]) <= 1e-12, x
    # either output alone
    _, R2 = jk.jk_laplace_fock(_t(C, dev), nocc, _t(J, dev), _t(K, dev), want_f=False)
    assert np.array_equal(R2.cpu().numpy(), Rov)


def test_forward_edge_tiny(dev):
    """One forward edge on the 28-AO workload's four Laplace pseudo-densities
    against the oracle's J/K, back-transform and next-level densities."""
    w0 = synth.config0()
    b, orb = w0.basis, w0.meta["orbitals"]
    D = w0.meta["laplace_D"]
    tau, _, _ = jk.jk_laplace_grid(4, *orb.gap_range())
    Jr, Kr, Rr, Dr = L.cascade_step(b, D, orb.C, orb.eps, orb.n_occ, tau)
    h = jk.JKBasis(b)
    try:
        J, K, Rov, Dn = jk.jk_laplace_step(h.h, _t(D, dev), _t(orb.C, dev), _t(orb.eps, dev), orb.n_occ, tau)
        J, K, Rov, Dn = (x.cpu().numpy() for x in (J, K, Rov, Dn))
    finally:
        h.close()
    assert np.max(np.abs(J - Jr)) <= 1e-10 and np.max(np.abs(K - Kr)) <= 1e-10
    assert _relmax(Rov, Rr) <= 1e-9 and _relmax(Dn, Dr) <= 1e-9


def test_forward_edge_medium_on_its_own_builds(dev):
    """At 312 AO and 16 densities: the edge's back-transform and densities
    equal the oracle's dense steps applied to the edge's own J and K (the J/K
    build itself is checked against the oracle at this size elsewhere)."""
    w1 = synth.config1()
    orb = w1.meta["orbitals"]
    tau, _, _ = jk.jk_laplace_grid(6, *orb.gap_range())
    h = jk.JKBasis(w1.basis)
    try:
        J, K, Rov, Dn = jk.jk_laplace_step(h.h, _t(w1.D, dev), _t(orb.C, dev), _t(orb.eps, dev), orb.n_occ, tau)
        J, K, Rov, Dn = (x.cpu().numpy() for x in (J, K, Rov, Dn))
    finally:
        h.close()
    for x in (0, 7, 15):
        ref = L.laplace_fock(orb.C, J[x], K[x])[:orb.n_occ, orb.n_occ:]
        assert _relmax(Rov[x], ref) <= 1e-12, x
        for k in (0, 5):
            assert _relmax(Dn[x, k], L.level_density(orb.C, orb.eps, orb.n_occ, tau[k], ref)) <= 1e-12, (x, k)


def test_invalid_cascade_arguments(dev):
    import torch
    C = torch.zeros((10, 10), dtype=torch.float64, device=dev)
    eps = torch.zeros(10, dtype=torch.float64, device=dev)
    R = torch.zeros((1, 4, 6), dtype=torch.float64, device=dev)
    with pytest.raises(jk.JKError):
        jk.jk_laplace_densities(C, eps, 4, np.zeros(65), R)      # too many grid points
    with pytest.raises(jk.JKError):
        jk.jk_laplace_densities(C, eps, 4, np.array([np.nan]), R)
