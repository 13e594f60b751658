"""The seeded input generator: reproducible bytes and the workload recipes."""
import numpy as np
import pytest

from paper_2607_05622_amd import synth


def test_same_seed_same_bytes():
    a = synth.config0()
    b = synth.config0()
    assert a.D.tobytes() == b.D.tobytes()
    assert a.basis.exps.tobytes() == b.basis.exps.tobytes()
    assert a.basis.xyz.tobytes() == b.basis.xyz.tobytes()


@pytest.mark.parametrize("n", [4, 30, 52])
def test_geometry_nearest_neighbours(n):
    rng = np.random.Generator(np.random.PCG64(n))
    x = synth.random_geometry(rng, n)
    d = np.linalg.norm(x[:, None] - x[None], axis=-1) + np.eye(n) * 1e9
    nn = d.min(axis=1)
    assert nn.min() >= 2.2 - 1e-12 and nn.max() <= 3.0 + 1e-12
    assert np.all(np.linalg.norm(x, axis=1) <= 2.6 * n ** (1 / 3) + 1e-12)


def test_workload_sizes():
    w0 = synth.config0()
    assert w0.basis.nbf() == 28 and w0.D.shape == (2, 28, 28)
    assert np.allclose(w0.D[0], w0.D[0].T) and not np.allclose(w0.D[1], w0.D[1].T)
    assert w0.meta["laplace_D"].shape == (4, 28, 28)
    rng = np.random.Generator(np.random.PCG64(1))
    b1 = synth.make_basis(rng, 30, 18)
    assert (b1.nbf(), b1.ncart(), b1.nshells) == (312, 330, 144)
    b2 = synth.make_basis(rng, 52, 40)
    assert (b2.nbf(), b2.ncart(), b2.nshells) == (620, 660, 276)
    assert set(np.unique(b2.shell_nprim)) == {3}
    assert b2.exps.min() >= 0.15 and b2.exps.max() <= 50.0


def test_loewdin_and_laplace_fit():
    w = synth.config0()
    orb = w.meta["orbitals"]
    S = synth.overlap_matrix(w.basis)
    assert np.max(np.abs(orb.C.T @ S @ orb.C - np.eye(28))) < 1e-11
    lo, hi = orb.gap_range()
    errs = []
    for n in (4, 8, 10):
        t = synth.laplace_nodes(n)
        errs.append(synth.laplace_max_rel_error(t, synth.laplace_weights(t, lo, hi), lo, hi))
    assert errs[0] > errs[1] > errs[2]


def test_request_stream():
    reqs = synth.request_stream(500, 10.0)
    nd = np.array([r["nd"] for r in reqs])
    assert nd.min() >= 1 and nd.max() <= 64
    t = np.array([r["arrival"] for r in reqs])
    assert np.all(np.diff(t) > 0)
    assert abs(np.mean(np.diff(t)) - 0.1) < 0.02
