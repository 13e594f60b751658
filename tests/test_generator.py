"""The HGP-OS generator: structure of the emitted recurrences and the
algorithmic flop table used for roofline figures."""
import os
import sys

import pytest

sys.path.insert(0, os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                "paper_2607_05622_amd", "csrc"))
import gen_eri  # noqa: E402


def test_canonical_classes():
    cls = gen_eri.classes()
    assert len(cls) == 21
    assert (0, 0, 0, 0) in cls and (2, 2, 2, 2) in cls and (2, 1, 2, 1) in cls
    assert all(a >= b and c >= d for a, b, c, d in cls)


@pytest.mark.parametrize("cls", gen_eri.classes())
def test_targets_and_outputs(cls):
    em = gen_eri.Emitter(*cls)
    info = em.generate()
    la, lb, lc, ld = cls
    nc = lambda l: (l + 1) * (l + 2) // 2
    assert info["nfunc"] == nc(la) * nc(lb) * nc(lc) * nc(ld)
    # every contracted target lies in the HGP-OS range of |e| and |f|
    for e, f in info["leaves"]:
        assert la <= sum(e) <= la + lb and lc <= sum(f) <= lc + ld
    # without horizontal transfer the targets are exactly the outputs
    if lb == 0 and ld == 0:
        assert info["nacc"] == info["nfunc"] and info["hrr_flops"] == 0
    # VRR nodes: every non-base node reads lower total angular momentum
    order = em.vrr_nodes([(e, f, 0) for e, f in info["leaves"]])
    pos = {n: i for i, n in enumerate(order)}
    for n in order:
        for d in em.vrr_deps(n):
            assert pos[d] < pos[n]


def test_flops_monotone_in_angular_momentum():
    import tempfile
    with tempfile.TemporaryDirectory() as td:
        counts = gen_eri.emit_all(os.path.join(td, "x.inc"))
    f = lambda t: gen_eri.flops_per_quartet(counts, t, 9, 9)
    assert f("0000") < f("1000") < f("1010") < f("1110") < f("1111") < f("2121") < f("2221") < f("2222")
