"""jk_build_noalloc (the entry point that allocates nothing) through the raw
C-ABI: its results equal jk_build's on the same inputs, on two calls in a
row, the second with a smaller input, and it refuses an unprepared plan and
a build beyond its static workspace."""
import ctypes

import numpy as np
import pytest

from paper_2607_05622_amd import jk, synth

pytestmark = pytest.mark.gpu
TOL = 1e-10


def test_noalloc_equals_build_two_calls_smaller_second():
    import torch
    dev = torch.device("cuda:0")
    lib = jk.load()
    big = synth.random_basis(2100, 5, 3)
    small = synth.random_basis(2101, 2, 1)
    cases = [(big, 7, jk.JK_FP64), (small, 2, jk.JK_FP64), (big, 3, jk.JK_MIXED)]
    handles = {}
    try:
        for i, (b, nd, prec) in enumerate(cases):
            if id(b) not in handles:
                handles[id(b)] = jk.JKBasis(b)
            h = handles[id(b)]
            o = jk.jk_default_opts(precision=prec)
            D = torch.tensor(synth.random_densities(2110 + i, nd, b.nbf()), device=dev)
            Jn = torch.full_like(D, np.nan)
            Kn = torch.full_like(D, np.nan)
            if i == 0:
                # no plan prepared for these options yet: refused, nothing written
                rc = lib.jk_build_noalloc(h.h, nd, D.data_ptr(), Jn.data_ptr(), Kn.data_ptr(), ctypes.byref(o))
                assert rc == jk.JK_EINVAL and "jk_workspace_bytes" in jk.jk_last_error()
            need = jk.jk_workspace_bytes(h.h, nd, o)
            assert 0 < need <= 64 << 20
            rc = lib.jk_build_noalloc(h.h, nd, D.data_ptr(), Jn.data_ptr(), Kn.data_ptr(), ctypes.byref(o))
            assert rc == jk.JK_OK, jk.jk_last_error()
            Jb = torch.empty_like(D)
            Kb = torch.empty_like(D)
            rc = lib.jk_build(h.h, nd, D.data_ptr(), Jb.data_ptr(), Kb.data_ptr(), ctypes.byref(o))
            assert rc == jk.JK_OK, jk.jk_last_error()
            torch.cuda.synchronize()
            dj = float((Jn - Jb).abs().max())
            dk = float((Kn - Kb).abs().max())
            print(f"call {i}: {b.nbf()} AO, nd={nd}, precision={prec}: max|dJ| {dj:.2e} max|dK| {dk:.2e}")
            assert dj <= TOL and dk <= TOL
    finally:
        for h in handles.values():
            h.close()


def test_noalloc_rejects_workspace_beyond_static_buffer():
    import torch
    dev = torch.device("cuda:0")
    lib = jk.load()
    b = synth.random_basis(2120, 30, 18)
    h = jk.JKBasis(b)
    try:
        nd = 64
        o = jk.jk_default_opts()
        need = jk.jk_workspace_bytes(h.h, nd, o)
        assert need > 64 << 20
        D = torch.zeros(nd, b.nbf(), b.nbf(), dtype=torch.float64, device=dev)
        J = torch.empty_like(D)
        K = torch.empty_like(D)
        rc = lib.jk_build_noalloc(h.h, nd, D.data_ptr(), J.data_ptr(), K.data_ptr(), ctypes.byref(o))
        assert rc == jk.JK_ENOMEM and "static buffer" in jk.jk_last_error()
    finally:
        h.close()
