"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

FP64 path bar: max |dJ|, |dK| <= 1e-10 per element (absolute), the bar the
build states for its FP64 path.  Mixed path bar: per density
||dJ||_F/||J||_F and ||dK||_F/||K||_F <= 1e-8 against the FP64 oracle.
Integrals are checked class by class; whole builds on small bases span
several tiles and ragged density counts; the 312-AO workload is checked at
full size, every element, against the whole oracle build; the 620-AO
workload on sampled shell-pair blocks of every pair class the oracle
computes one by one.
"""
import itertools
import time

import numpy as np
import pytest

import oracle
from paper_2607_05622_amd import jk, synth
from paper_2607_05622_amd.synth import CART

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def gpu_jk(basis, D, dev, **opts):
    import torch
    b = jk.JKBasis(basis)
    try:
        Dt = torch.tensor(np.asarray(D), dtype=torch.float64, device=dev)
        if Dt.dim() == 2:
            Dt = Dt.unsqueeze(0)
        J, K = b.build(Dt, **opts)
        torch.cuda.synchronize()
        return (J.cpu().numpy() if J is not None else None), (K.cpu().numpy() if K is not None else None)
    finally:
        b.close()


def maxabs(a, b):
    return float(np.max(np.abs(a - b)))


def test_eri_tiles_every_class(dev):
    # one atom of each kind per centre so every (la lb | lc ld) occurs
    b = synth.random_basis(77, 4, 4, spherical=0)
    h = jk.JKBasis(b)
    l = b.shell_l
    by_l = {k: [int(s) for s in np.nonzero(l == k)[0]] for k in range(3)}
    rng = np.random.default_rng(0)
    quartets = []
    for cls in itertools.product(range(3), repeat=4):
        q = [by_l[c][int(rng.integers(len(by_l[c])))] for c in cls]
        quartets.append(tuple(q))
    # plus coincident-shell quartets
    quartets += [(0, 0, 0, 0), (by_l[2][0], by_l[2][0], by_l[1][0], by_l[1][0]),
                 (by_l[2][1], by_l[1][1], by_l[2][1], by_l[1][1])]
    tiles = h.eri_tiles(quartets)
    h.close()
    nc = lambda s: len(CART[int(l[s])])
    worst = 0.0
    for q, t in zip(quartets, tiles):
        ref = oracle.eri_shell_quartet(b, *q, nc)
        scale = max(1.0, float(np.max(np.abs(ref))))
        err = maxabs(t, ref) / scale
        worst = max(worst, err)
        assert err <= 1e-12, (q, err)
    print("worst relative tile error", worst)


def test_config0_fp64(dev):
    w = synth.config0()
    for D in (w.D, w.meta["laplace_D"]):
        Jr, Kr = oracle.jk(w.basis, D, 1e-12)
        J, K = gpu_jk(w.basis, D, dev)
        assert maxabs(J, Jr) <= TOL and maxabs(K, Kr) <= TOL


@pytest.mark.parametrize("nd", [1, 3, 17, 40])
def test_spd_molecule_ragged_nd(dev, nd):
    b = synth.random_basis(101 + nd, 5, 3)
    D = synth.random_densities(nd, nd, b.nbf())
    Jr, Kr = oracle.jk(b, D, 1e-12)
    J, K = gpu_jk(b, D, dev)
    assert maxabs(J, Jr) <= TOL and maxabs(K, Kr) <= TOL


@pytest.mark.parametrize("dig_kernel", [1, 2, 3])
def test_every_digestion_kernel(dev, dig_kernel):
    """Each digestion kernel the tunables select (1: one workgroup per
    task; 2: wave-private tasks; 3: one pass, K_ad and K_bd per quartet),
    with 16- and 8-density groups, FP64 and mixed, against the oracle on a
    5-atom s/p/d molecule with 17 densities (a ragged last group), short
    pieces so every bra pair spans several."""
    b = synth.random_basis(731, 5, 3)
    D = synth.random_densities(732, 17, b.nbf())
    Jr, Kr = oracle.jk(b, D, 1e-12)
    old = [jk.jk_tune_get(c) for c in range(21)]
    try:
        for g in (16, 8):
            for c in range(21):
                jk.jk_tune_set(c, seg_max=16, g_max=g, dig_kernel=dig_kernel, eri_block=256)
            J, K = gpu_jk(b, D, dev)
            assert maxabs(J, Jr) <= TOL and maxabs(K, Kr) <= TOL, g
            J, K = gpu_jk(b, D, dev, precision=jk.JK_MIXED)
            assert np.all(rel_frob(J, Jr) <= 1e-8) and np.all(rel_frob(K, Kr) <= 1e-8), g
    finally:
        for c, t in enumerate(old):
            jk.jk_tune_set(c, **t)


def test_cartesian_basis(dev):
    b = synth.random_basis(202, 4, 3, spherical=0)
    D = synth.random_densities(5, 4, b.nbf())
    Jr, Kr = oracle.jk(b, D, 1e-12)
    J, K = gpu_jk(b, D, dev)
    assert maxabs(J, Jr) <= TOL and maxabs(K, Kr) <= TOL


def test_degenerate_bases(dev):
    one_atom = synth.random_basis(31, 1, 1)
    rep = synth.random_basis(32, 2, 1).subset([0, 0, 3, 3, 5, 5])
    one_shell = synth.random_basis(33, 1, 1).subset([5])
    s_only = synth.random_basis(34, 3, 0, heavy=(0,), light=(0, 0))
    for bb in (one_atom, rep, one_shell, s_only):
        D = synth.random_densities(7, 2, bb.nbf())
        Jr, Kr = oracle.jk(bb, D, 0.0)
        J, K = gpu_jk(bb, D, dev, schwarz_tol=0.0)
        assert maxabs(J, Jr) <= TOL and maxabs(K, Kr) <= TOL


def test_want_flags_and_zero_density(dev):
    b = synth.random_basis(303, 3, 2)
    D = synth.random_densities(3, 2, b.nbf())
    Jr, Kr = oracle.jk(b, D, 1e-12)
    J, K = gpu_jk(b, D, dev, want_k=0)
    assert K is None and maxabs(J, Jr) <= TOL
    J, K = gpu_jk(b, D, dev, want_j=0)
    assert J is None and maxabs(K, Kr) <= TOL
    J, K = gpu_jk(b, np.zeros_like(D), dev)
    assert np.all(J == 0) and np.all(K == 0)


def test_unwanted_output_pointer_is_never_touched(dev):
    """want_j = 0 (or want_k = 0) with a non-NULL output pointer, through the
    raw C-ABI: the unwanted buffer keeps its sentinel values and the wanted
    matrix matches the oracle."""
    import ctypes
    import torch
    b = synth.random_basis(304, 3, 2)
    D = synth.random_densities(5, 3, b.nbf())
    Jr, Kr = oracle.jk(b, D, 1e-12)
    h = jk.JKBasis(b)
    lib = jk.load()
    Dt = torch.tensor(D, device=dev)
    for want_j, want_k in ((0, 1), (1, 0)):
        o = jk.jk_default_opts(want_j=want_j, want_k=want_k)
        J = torch.full_like(Dt, 12345.0)
        K = torch.full_like(Dt, -6789.0)
        rc = lib.jk_build(h.h, Dt.shape[0], Dt.data_ptr(), J.data_ptr(), K.data_ptr(), ctypes.byref(o))
        assert rc == jk.JK_OK, jk.jk_last_error()
        torch.cuda.synchronize()
        J, K = J.cpu().numpy(), K.cpu().numpy()
        if want_j:
            assert maxabs(J, Jr) <= TOL and np.all(K == -6789.0)
        else:
            assert maxabs(K, Kr) <= TOL and np.all(J == 12345.0)
    h.close()


def test_structure_of_gpu_results(dev):
    b = synth.random_basis(404, 4, 2)
    D = synth.random_densities(4, 2, b.nbf())
    Dt = D.transpose(0, 2, 1).copy()
    J, K = gpu_jk(b, np.concatenate([D, Dt, 0.5 * (D + Dt)]), dev)
    sc = np.max(np.abs(K))
    assert maxabs(J[0], J[0].T) <= 1e-12 * sc
    assert maxabs(J[0], J[4]) <= 1e-12 * sc            # J(D) = J(sym D)
    assert maxabs(K[2], K[0].T) <= 1e-12 * sc          # K(D^T) = K(D)^T


def test_symmetric_hint_skips_transposed_exchange(dev):
    """Symmetric densities with symmetric_hint = 1 (the D^T exchange
    contractions skipped, K = Kc + Kc^T): the same J and K as without the
    hint, and the oracle's, for more than 8 densities (where it applies) and
    for fewer (where it is ignored)."""
    b = synth.random_basis(410, 4, 3)
    for nd in (12, 5):
        D = synth.random_densities(411 + nd, nd, b.nbf(), symmetric=True)
        Jr, Kr = oracle.jk(b, D, 1e-12)
        J0, K0 = gpu_jk(b, D, dev)
        J1, K1 = gpu_jk(b, D, dev, symmetric_hint=1)
        assert maxabs(J1, J0) <= 1e-12 and maxabs(K1, K0) <= 1e-12, nd
        assert maxabs(J1, Jr) <= TOL and maxabs(K1, Kr) <= TOL, nd


def test_repeat_determinism(dev):
    b = synth.random_basis(505, 5, 3)
    D = synth.random_densities(5, 8, b.nbf())
    runs = [gpu_jk(b, D, dev) for _ in range(4)]
    for J, K in runs[1:]:
        assert maxabs(J, runs[0][0]) <= 1e-13 and maxabs(K, runs[0][1]) <= 1e-13


def test_user_workspace_and_stream(dev):
    import torch
    b = synth.random_basis(606, 4, 2)
    D = synth.random_densities(6, 5, b.nbf())
    Jr, Kr = oracle.jk(b, D, 1e-12)
    h = jk.JKBasis(b)
    o = jk.jk_default_opts()
    nbytes = jk.jk_workspace_bytes(h.h, 5, o)
    assert nbytes > 0
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    o.workspace = ws.data_ptr()
    o.workspace_bytes = nbytes
    s = torch.cuda.Stream(device=dev)
    Dt = torch.tensor(D, device=dev)
    torch.cuda.synchronize()
    J, K = jk.jk_build(h.h, Dt, opts=o, stream=s)
    s.synchronize()
    assert maxabs(J.cpu().numpy(), Jr) <= TOL and maxabs(K.cpu().numpy(), Kr) <= TOL
    o.workspace_bytes = nbytes - 1
    with pytest.raises(jk.JKError):
        jk.jk_build(h.h, Dt, opts=o, stream=s)
    h.close()


def test_invalid_build_arguments(dev):
    import torch
    b = jk.JKBasis(synth.random_basis(707, 2, 1))
    lib = jk.load()
    o = jk.jk_default_opts()
    D = torch.zeros(1, b.nbf, b.nbf, dtype=torch.float64, device=dev)
    assert lib.jk_build(b.h, 0, D.data_ptr(), D.data_ptr(), D.data_ptr(), None) == jk.JK_EINVAL
    assert lib.jk_build(b.h, 1, None, D.data_ptr(), D.data_ptr(), None) == jk.JK_EINVAL
    o.schwarz_tol = -1.0
    assert lib.jk_build(b.h, 1, D.data_ptr(), D.data_ptr(), D.data_ptr(), o) == jk.JK_EINVAL
    o = jk.jk_default_opts(precision=7)
    assert lib.jk_build(b.h, 1, D.data_ptr(), D.data_ptr(), D.data_ptr(), o) == jk.JK_EINVAL
    b.close()


@pytest.fixture(scope="module")
def medium_ref():
    """The 312-AO workload (16 Laplace pseudo-densities) and the oracle's
    whole screened build of it (about two minutes on 16 host threads)."""
    w = synth.config1()
    t0 = time.perf_counter()
    Jr, Kr = oracle.jk(w.basis, w.D, 1e-12)
    print(f"medium oracle: {time.perf_counter() - t0:.1f} s on {oracle.threads()} threads", flush=True)
    return w, Jr, Kr


def test_medium_workload_full_fp64(dev, medium_ref):
    """312 AO, 16 non-symmetric densities, the benchmark's launch
    configuration: every element of J and K against the oracle."""
    w, Jr, Kr = medium_ref
    J, K = gpu_jk(w.basis, w.D, dev)
    ej, ek = maxabs(J, Jr), maxabs(K, Kr)
    print(f"medium fp64: max|dJ| {ej:.2e} max|dK| {ek:.2e} (max|J| {np.max(np.abs(Jr)):.2f}, "
          f"max|K| {np.max(np.abs(Kr)):.2f})")
    assert ej <= TOL and ek <= TOL


# ------------------------------------------------------------ mixed tier ----

def rel_frob(a, b):
    """Per-density ||a - b||_F / ||b||_F."""
    return np.sqrt(np.sum((a - b) ** 2, axis=(1, 2)) / np.maximum(np.sum(b ** 2, axis=(1, 2)), 1e-300))


def fp32_tier_count(b, tol, bound):
    """Canonical shell quartets kept by Q_ab Q_cd >= tol, and of those the
    ones with Q_ab Q_cd < bound and la + lb + lc + ld <= 4, from the oracle's
    Schwarz factors."""
    Q = oracle.schwarz(b)
    l = np.asarray(b.shell_l)
    ns = len(l)
    pa, pb = np.tril_indices(ns)
    q = Q[pa, pb]
    lp = l[pa] + l[pb]
    n_all = n32 = 0
    for i in range(len(q)):
        qq = q[i] * q[:i + 1]
        keep = qq >= tol
        n_all += int(keep.sum())
        n32 += int((keep & (qq < bound) & (lp[i] + lp[:i + 1] <= 4)).sum())
    return n_all, n32


def test_mixed_precision_against_oracle(dev):
    b = synth.random_basis(808, 8, 5)
    D = synth.random_densities(8, 6, b.nbf())
    Jr, Kr = oracle.jk(b, D, 1e-12)
    h = jk.JKBasis(b)
    import torch
    Dt = torch.tensor(D, device=dev)
    J, K = h.build(Dt, precision=jk.JK_MIXED)
    torch.cuda.synchronize()
    st = h.stats()
    h.close()
    J, K = J.cpu().numpy(), K.cpu().numpy()
    # the FP32 tier holds exactly the Schwarz-kept quartets with Q_ab Q_cd
    # below the bound and total angular momentum <= 4, counted here from the
    # oracle's Schwarz factors; on this basis that is about a quarter
    n_all, n32 = fp32_tier_count(b, 1e-12, 1e-6)
    print(f"mixed: {st['quartets_fp32']:.0f} of {st['quartets']:.0f} quartets in FP32 "
          f"(oracle count {n32} of {n_all})")
    assert st["quartets"] == n_all and st["quartets_fp32"] == n32
    assert n32 > 0.2 * n_all                                   # the FP32 tier is exercised
    assert np.all(rel_frob(J, Jr) <= 1e-8) and np.all(rel_frob(K, Kr) <= 1e-8)
    print("mixed: max rel-Frobenius J %.2e K %.2e, max-abs J %.2e K %.2e" % (
        rel_frob(J, Jr).max(), rel_frob(K, Kr).max(), maxabs(J, Jr), maxabs(K, Kr)))


def test_mixed_bound_zero_is_fp64(dev):
    b = synth.random_basis(809, 5, 3)
    D = synth.random_densities(9, 3, b.nbf())
    J1, K1 = gpu_jk(b, D, dev)
    J2, K2 = gpu_jk(b, D, dev, precision=jk.JK_MIXED, fp32_bound=0.0)
    assert maxabs(J1, J2) <= 1e-13 and maxabs(K1, K2) <= 1e-13


def test_medium_workload_full_mixed(dev, medium_ref):
    """312 AO, 16 densities, mixed precision: per density relative
    Frobenius error of J and K against the whole oracle build."""
    w, Jr, Kr = medium_ref
    Jm, Km = gpu_jk(w.basis, w.D, dev, precision=jk.JK_MIXED)
    ej, ek = rel_frob(Jm, Jr), rel_frob(Km, Kr)
    print(f"medium mixed vs oracle per density: max rel-Frobenius J {ej.max():.2e} K {ek.max():.2e}, "
          f"max-abs J {maxabs(Jm, Jr):.2e} K {maxabs(Km, Kr):.2e}")
    assert np.all(ej <= 1e-8) and np.all(ek <= 1e-8)


def sample_blocks(basis, seed, per_class=3,
                  classes=((0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (0, 2))):
    """per_class shell-pair blocks (A, B) of every (l_A, l_B), drawn with a
    seeded generator."""
    l = basis.shell_l
    rng = np.random.default_rng(seed)
    out = []
    for la, lb in classes:
        A = [int(s) for s in np.nonzero(l == la)[0]]
        B = [int(s) for s in np.nonzero(l == lb)[0]]
        for _ in range(per_class):
            out.append((A[int(rng.integers(len(A)))], B[int(rng.integers(len(B)))]))
    return out


def block_errors(J, K, basis, blocks, refs):
    """Max-abs over the blocks, and per density the relative Frobenius
    error restricted to the blocks."""
    fo = basis.func_offsets()
    ej = ek = 0.0
    nd = J.shape[0]
    dj2, dk2, rj2, rk2 = np.zeros(nd), np.zeros(nd), np.zeros(nd), np.zeros(nd)
    for (a, c), (Jb, Kb) in zip(blocks, refs):
        sl = (slice(None), slice(fo[a], fo[a + 1]), slice(fo[c], fo[c + 1]))
        ej = max(ej, maxabs(J[sl], Jb))
        ek = max(ek, maxabs(K[sl], Kb))
        dj2 += np.sum((J[sl] - Jb) ** 2, axis=(1, 2))
        dk2 += np.sum((K[sl] - Kb) ** 2, axis=(1, 2))
        rj2 += np.sum(Jb ** 2, axis=(1, 2))
        rk2 += np.sum(Kb ** 2, axis=(1, 2))
    return ej, ek, np.sqrt(dj2 / rj2), np.sqrt(dk2 / rk2)


@pytest.fixture(scope="module")
def large_run(dev):
    """The 620-AO workload (40 densities): FP64 and mixed GPU builds in the
    benchmark's launch configuration, and 21 oracle blocks, three of every
    shell-pair class."""
    w = synth.config2()
    print(f"large workload: {w.basis.nbf()} AO, {w.D.shape[0]} densities", flush=True)
    t0 = time.perf_counter()
    J64, K64 = gpu_jk(w.basis, w.D, dev)
    Jm, Km = gpu_jk(w.basis, w.D, dev, precision=jk.JK_MIXED)
    print(f"large: two GPU builds with set-up {time.perf_counter() - t0:.1f} s", flush=True)
    blocks = sample_blocks(w.basis, 2)
    t0 = time.perf_counter()
    refs = oracle.jk_blocks(w.basis, w.D, blocks, 1e-12)
    print(f"large: {len(blocks)} oracle blocks {time.perf_counter() - t0:.1f} s", flush=True)
    return w, J64, K64, Jm, Km, blocks, refs


def test_large_workload_fp64_blocks(dev, large_run):
    """620 AO, 40 non-symmetric densities (the memory-ceiling molecule), FP64:
    three sampled shell-pair blocks of every pair class against the oracle,
    element by element; J symmetric at any size."""
    w, J64, K64, _, _, blocks, refs = large_run
    ej, ek, _, _ = block_errors(J64, K64, w.basis, blocks, refs)
    print(f"large fp64 on {len(blocks)} blocks: max|dJ| {ej:.2e} max|dK| {ek:.2e}")
    assert ej <= TOL and ek <= TOL
    assert maxabs(J64, J64.transpose(0, 2, 1)) <= 1e-12 * np.max(np.abs(J64))


def test_large_workload_mixed(dev, large_run):
    """620 AO, 40 densities, mixed precision: against the oracle on the
    sampled blocks (per density relative Frobenius over the blocks, and
    max-abs), and against the GPU's FP64 build over whole matrices."""
    w, J64, K64, Jm, Km, blocks, refs = large_run
    ej, ek, fj, fk = block_errors(Jm, Km, w.basis, blocks, refs)
    gj, gk = rel_frob(Jm, J64), rel_frob(Km, K64)
    print(f"large mixed vs oracle on blocks: max-abs J {ej:.2e} K {ek:.2e}, per density rel-Frobenius "
          f"J {fj.max():.2e} K {fk.max():.2e}; vs GPU FP64 whole matrices J {gj.max():.2e} K {gk.max():.2e}")
    assert np.all(fj <= 1e-8) and np.all(fk <= 1e-8)
    assert np.all(gj <= 1e-8) and np.all(gk <= 1e-8)


def test_mixed_contraction_lengths(dev):
    """Shells of 1, 2, 7 and 16 primitives in one basis (the interleaved
    primitive-pair records pad each group of 64 pairs to its longest list),
    FP64 and mixed, against the oracle."""
    b = synth.random_basis(1700, 3, 1, nprims=(1, 2, 7, 16))
    D = synth.random_densities(1701, 3, b.nbf())
    Jr, Kr = oracle.jk(b, D, 1e-12)
    J, K = gpu_jk(b, D, dev)
    assert maxabs(J, Jr) <= TOL and maxabs(K, Kr) <= TOL
    Jm, Km = gpu_jk(b, D, dev, precision=jk.JK_MIXED)
    assert np.all(rel_frob(Jm, Jr) <= 1e-8) and np.all(rel_frob(Km, Kr) <= 1e-8)


# ------------------------------------------------------- batched launch ----

def _batch(bases, Ds, dev, **opts):
    import torch
    hs = [jk.JKBasis(b) for b in bases]
    try:
        Dt = [torch.tensor(D, device=dev) for D in Ds]
        o = jk.jk_default_opts(**opts)
        Js, Ks = jk.jk_build_batch([h.h for h in hs], Dt, opts=o)
        torch.cuda.synchronize()
        return [J.cpu().numpy() for J in Js], [K.cpu().numpy() for K in Ks]
    finally:
        for h in hs:
            h.close()


def test_batch_uneven_molecules(dev):
    specs = [(1, 1, 3), (3, 2, 1), (5, 3, 8), (2, 2, 17), (4, 1, 5), (6, 4, 2)]
    bases = [synth.random_basis(900 + i, na, nh) for i, (na, nh, _) in enumerate(specs)]
    Ds = [synth.random_densities(950 + i, nd, b.nbf()) for i, (b, (_, _, nd)) in enumerate(zip(bases, specs))]
    Jb, Kb = _batch(bases, Ds, dev)
    for b, D, J, K in zip(bases, Ds, Jb, Kb):
        Jr, Kr = oracle.jk(b, D, 1e-12)
        assert maxabs(J, Jr) <= TOL and maxabs(K, Kr) <= TOL
        Js, Ks = gpu_jk(b, D, dev)
        assert maxabs(J, Js) <= 1e-13 and maxabs(K, Ks) <= 1e-13


def test_batch_mixed_precision(dev):
    bases = [synth.random_basis(970 + i, 4 + 2 * i, 3 + i) for i in range(3)]
    Ds = [synth.random_densities(980 + i, 4 + 3 * i, b.nbf()) for i, b in enumerate(bases)]
    Jb, Kb = _batch(bases, Ds, dev, precision=jk.JK_MIXED)
    for b, D, J, K in zip(bases, Ds, Jb, Kb):
        Jr, Kr = oracle.jk(b, D, 1e-12)
        assert np.all(rel_frob(J, Jr) <= 1e-8) and np.all(rel_frob(K, Kr) <= 1e-8)


def test_batch_workload_64_molecules(dev, capsys, tmp_path):
    """The 64-molecule uneven workload in one batched build, with schedules
    from the autotuner (run on the batch's largest molecule, cached as JSON
    and loaded): every molecule equals its own build; the eight smallest
    against the whole oracle build, the four largest on sampled shell-pair
    blocks.  Reports progress on the terminal even when output is captured."""
    import torch

    def note(msg):
        with capsys.disabled():
            print(f"[batch-64] {msg}", flush=True)

    ws = synth.config3()
    note("64-molecule workload generated")
    bases = [w.basis for w in ws]
    Ds = [w.D for w in ws]
    hs = []
    for i, b in enumerate(bases):
        hs.append(jk.JKBasis(b))
        if i % 8 == 7:
            note(f"{i + 1} handles created")
    old_tune = [jk.jk_tune_get(c) for c in range(21)]
    try:
        Dt = [torch.tensor(D, device=dev) for D in Ds]
        big = int(np.argmax([b.nbf() for b in bases]))
        cache = str(tmp_path / "tune_batch.json")
        jk.jk_autotune(hs[big].h, Dt[big], torch.empty_like(Dt[big]), torch.empty_like(Dt[big]), cache_path=cache)
        for c in range(21):
            jk.jk_tune_set(c)
        jk.jk_tune_load(cache)
        note(f"schedules tuned on molecule {big} ({bases[big].nbf()} AO) and loaded from {cache}")
        Jt, Kt = jk.jk_build_batch([h.h for h in hs], Dt)
        torch.cuda.synchronize()
        Jb = [J.cpu().numpy() for J in Jt]
        Kb = [K.cpu().numpy() for K in Kt]
        note("batched build done")
        for i in range(len(ws)):
            Js, Ks = hs[i].build(Dt[i])
            torch.cuda.synchronize()
            assert maxabs(Jb[i], Js.cpu().numpy()) <= 1e-12 and maxabs(Kb[i], Ks.cpu().numpy()) <= 1e-12, i
    finally:
        for h in hs:
            h.close()
        for c, t in enumerate(old_tune):
            jk.jk_tune_set(c, **t)
    note("each molecule equals its own build")
    order = np.argsort([b.nbf() for b in bases])
    for i in order[:8]:
        Jr, Kr = oracle.jk(bases[i], Ds[i], 1e-12)
        assert maxabs(Jb[i], Jr) <= TOL and maxabs(Kb[i], Kr) <= TOL, i
        note(f"molecule {i} ({bases[i].nbf()} AO) matches the oracle")
    for i in order[-4:]:
        blocks = sample_blocks(bases[i], 30 + int(i), per_class=1)
        refs = oracle.jk_blocks(bases[i], Ds[i], blocks, 1e-12)
        ej, ek, _, _ = block_errors(Jb[i], Kb[i], bases[i], blocks, refs)
        assert ej <= TOL and ek <= TOL, (i, ej, ek)
        note(f"molecule {i} ({bases[i].nbf()} AO, {Ds[i].shape[0]} densities) matches the oracle "
             f"on {len(blocks)} blocks")


# ------------------------------------------------------------ HIP graphs ----

def test_graph_replays_match_eager_builds(dev):
    import torch
    b = synth.random_basis(1111, 5, 3)
    h = jk.JKBasis(b)
    nd = 6
    n = b.nbf()
    o = jk.jk_default_opts()
    nbytes = jk.jk_workspace_bytes(h.h, nd, o)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    o.workspace = ws.data_ptr()
    o.workspace_bytes = nbytes
    D = torch.zeros(nd, n, n, dtype=torch.float64, device=dev)
    J = torch.empty_like(D)
    K = torch.empty_like(D)
    g = jk.jk_graph_create(h.h, D, J, K, o)
    s = torch.cuda.Stream(device=dev)
    for rep in range(4):
        Dn = torch.tensor(synth.random_densities(1200 + rep, nd, n), device=dev)
        D.copy_(Dn)
        torch.cuda.synchronize()
        jk.jk_graph_launch(g, s)
        s.synchronize()
        Jg, Kg = J.clone(), K.clone()
        Je, Ke = h.build(Dn.clone())          # eager build between replays
        torch.cuda.synchronize()
        assert float((Jg - Je).abs().max()) <= 1e-13 and float((Kg - Ke).abs().max()) <= 1e-13, rep
    jk.jk_graph_destroy(g)
    h.close()


# --------------------------------------------------------------- serving ----

def _requests(bases, dev, n, rate, seed):
    import torch
    from paper_2607_05622_amd.serve import Request
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    out = []
    for i in range(n):
        m = int(rng.integers(len(bases)))
        nd = int(np.floor(np.exp(rng.uniform(0, np.log(17)))))
        D = torch.tensor(synth.random_densities(seed * 1000 + i, nd, bases[m].nbf()), device=dev)
        out.append(Request(i, float(t[i]), m, D))
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_served_results_equal_alone(dev, precision):
    """Requests served in the mix (batched launches, graphs, overlapping
    slots) equal the same requests built alone."""
    from paper_2607_05622_amd.serve import JKServer
    bases = [synth.random_basis(1300 + i, 2 + 2 * i, 1 + i) for i in range(4)]
    srv = JKServer(bases, n_slots=3, mem_budget=3 * (256 << 20), precision=precision, max_batch=6)
    srv.warm_graphs(max_nd=16)
    reqs = _requests(bases, dev, 40, rate=400.0, seed=7)
    stats = srv.run(reqs)
    assert stats["requests"] == 40 and stats["mean_batch"] > 1.0
    assert srv.peak_admitted <= srv.slot_bytes
    for r in reqs:
        Ja, Ka = gpu_jk(bases[r.mol], r.D.cpu().numpy(), dev, precision=precision)
        J, K = r.J.cpu().numpy(), r.K.cpu().numpy()
        if precision == 0:
            assert maxabs(J, Ja) <= 1e-12 and maxabs(K, Ka) <= 1e-12, r.index
        else:
            assert np.all(rel_frob(J, Ja) <= 1e-8) and np.all(rel_frob(K, Ka) <= 1e-8), r.index
    srv.close()


def test_served_stream_resident_molecules_against_oracle(dev, capsys):
    """The served stream over the 16 resident molecules (50-730 AO) in mixed
    precision: a burst that the server folds into multi-request launches on
    several slots, then a lone late request that replays a HIP graph.  Every
    request equals the same request built alone; one request per molecule is
    checked against the oracle: on molecules of at most 210 AO over whole
    matrices (per density relative Frobenius), on the larger ones on sampled
    blocks, whose error must stay within 1e-8 of the whole matrix's norm per
    density (a necessary condition of the whole-matrix bar)."""
    import torch
    from paper_2607_05622_amd.serve import JKServer, Request

    def note(msg):
        with capsys.disabled():
            print(f"[served] {msg}", flush=True)

    mols = synth.config4_molecules()
    bases = [m.basis for m in mols]
    stream = synth.request_stream(24, 1.0)
    reqs = []
    for i, r in enumerate(stream):
        mol = i % 16 if i < 16 else r["mol"]
        nd = min(r["nd"], 16)
        D = torch.tensor(synth.request_densities(mols[mol].meta["orbitals"], nd, r["seed"]), device=dev)
        reqs.append(Request(i, 0.002 * i, mol, D))
    # a lone request long after the burst: served by a graph replay
    D = torch.tensor(synth.request_densities(mols[3].meta["orbitals"], 5, 4_100_000), device=dev)
    reqs.append(Request(len(reqs), 8.0, 3, D))
    t0 = time.perf_counter()
    srv = JKServer(bases, n_slots=3, precision=jk.JK_MIXED, max_batch=6)
    note(f"16 molecules resident ({min(b.nbf() for b in bases)}-{max(b.nbf() for b in bases)} AO) "
         f"in {time.perf_counter() - t0:.1f} s")
    launches = []
    stats = srv.run(reqs, on_launch=lambda si, b: launches.append((si, len(b))))
    note(f"{stats['requests']} requests served: mean batch {stats['mean_batch']:.2f}, "
         f"graph fraction {stats['graph_fraction']:.2f}, slots used {sorted(set(s for s, _ in launches))}")
    assert stats["requests"] == len(reqs)
    assert max(n for _, n in launches) > 1 and len(set(s for s, _ in launches)) > 1
    assert reqs[-1].graph
    checked = set()
    for r in reqs:
        Ja, Ka = gpu_jk(bases[r.mol], r.D.cpu().numpy(), dev, precision=jk.JK_MIXED)
        J, K = r.J.cpu().numpy(), r.K.cpu().numpy()
        assert np.all(rel_frob(J, Ja) <= 1e-8) and np.all(rel_frob(K, Ka) <= 1e-8), r.index
        if r.mol in checked and r.index != len(reqs) - 1:
            continue
        checked.add(r.mol)
        if bases[r.mol].nbf() <= 210:
            Jr, Kr = oracle.jk(bases[r.mol], r.D.cpu().numpy(), 1e-12)
            fj, fk = rel_frob(J, Jr), rel_frob(K, Kr)
        else:
            blocks = sample_blocks(bases[r.mol], 40 + r.index, per_class=1, classes=((0, 0), (2, 1), (1, 2)))
            refs = oracle.jk_blocks(bases[r.mol], r.D.cpu().numpy(), blocks, 1e-12)
            fo = bases[r.mol].func_offsets()
            dj2, dk2 = np.zeros(r.nd), np.zeros(r.nd)
            for (a, c), (Jb, Kb) in zip(blocks, refs):
                sl = (slice(None), slice(fo[a], fo[a + 1]), slice(fo[c], fo[c + 1]))
                dj2 += np.sum((J[sl] - Jb) ** 2, axis=(1, 2))
                dk2 += np.sum((K[sl] - Kb) ** 2, axis=(1, 2))
            fj = np.sqrt(dj2 / np.sum(J ** 2, axis=(1, 2)))
            fk = np.sqrt(dk2 / np.sum(K ** 2, axis=(1, 2)))
        assert np.all(fj <= 1e-8) and np.all(fk <= 1e-8), (r.index, fj.max(), fk.max())
    note(f"every request equals its own build; {len(checked)} molecules match the oracle on sampled blocks")
    assert len(checked) == 16
    srv.close()


def test_served_low_budget_waits_but_completes(dev):
    from paper_2607_05622_amd.serve import JKServer
    bases = [synth.random_basis(1400 + i, 3 + i, 2) for i in range(2)]
    reqs = _requests(bases, dev, 12, rate=1000.0, seed=9)
    srv = JKServer(bases, n_slots=1, mem_budget=64 << 20, precision=0, max_batch=8, use_graphs=False)
    alone = max(srv.workspace_bytes([r]) for r in reqs)
    srv.close()
    # a budget that holds one request at a time
    srv = JKServer(bases, n_slots=1, mem_budget=alone + 4096, precision=0, max_batch=8, use_graphs=False)
    stats = srv.run(reqs)
    assert stats["requests"] == 12 and srv.peak_admitted <= srv.slot_bytes
    for r in reqs:
        Jr, Kr = oracle.jk(bases[r.mol], r.D.cpu().numpy(), 1e-12)
        assert maxabs(r.J.cpu().numpy(), Jr) <= TOL and maxabs(r.K.cpu().numpy(), Kr) <= TOL
    srv.close()


def test_autotune_keeps_results(dev, tmp_path):
    import torch
    b = synth.random_basis(1500, 6, 4)
    D = synth.random_densities(1501, 9, b.nbf())
    Jr, Kr = oracle.jk(b, D, 1e-12)
    old = [jk.jk_tune_get(c) for c in range(21)]
    h = jk.JKBasis(b)
    try:
        Dt = torch.tensor(D, device=dev)
        J = torch.empty_like(Dt)
        K = torch.empty_like(Dt)
        path = str(tmp_path / "tune.json")
        jk.jk_autotune(h.h, Dt, J, K, cache_path=path)
        assert '"arch": "gfx950"' in open(path).read()
        J, K = h.build(Dt)
        torch.cuda.synchronize()
        assert maxabs(J.cpu().numpy(), Jr) <= TOL and maxabs(K.cpu().numpy(), Kr) <= TOL
        jk.jk_tune_load(path)
    finally:
        h.close()
        for c, t in enumerate(old):
            jk.jk_tune_set(c, **t)
