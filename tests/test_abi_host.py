"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/jk.h declares, and rejects invalid arguments with the
documented codes before touching the device."""
import ctypes
import math

import numpy as np
import pytest

from paper_2607_05622_amd import jk, synth


@pytest.fixture(scope="module")
def lib():
    return jk.load()


def test_exports_every_declared_function(lib):
    names = jk.declared_functions()
    assert len(names) >= 10
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []


def test_default_opts(lib):
    o = jk.jk_default_opts()
    assert (o.precision, o.schwarz_tol, o.fp32_bound, o.want_j, o.want_k) == (jk.JK_FP64, 1e-12, 1e-6, 1, 1)
    assert o.stream is None and o.workspace is None


def _create(lib, arrays):
    d, keep = jk._desc(arrays)
    h = ctypes.c_void_p()
    rc = lib.jk_create_basis(ctypes.byref(d), ctypes.byref(h))
    return rc, h


def _mutate(**kw):
    a = synth.random_basis(3, 2, 1).as_arrays()
    for k, v in kw.items():
        a[k] = v(a) if callable(v) else v
    return a


@pytest.mark.parametrize("bad", [
    dict(shell_l=lambda a: np.where(np.arange(len(a["shell_l"])) == 0, 3, a["shell_l"]).astype(np.int32)),
    dict(shell_l=lambda a: np.where(np.arange(len(a["shell_l"])) == 1, -1, a["shell_l"]).astype(np.int32)),
    dict(shell_nprim=lambda a: np.where(np.arange(len(a["shell_nprim"])) == 0, 0, a["shell_nprim"]).astype(np.int32)),
    dict(exps=lambda a: np.where(np.arange(len(a["exps"])) == 2, -0.5, a["exps"])),
    dict(exps=lambda a: np.where(np.arange(len(a["exps"])) == 2, 0.0, a["exps"])),
    dict(exps=lambda a: np.where(np.arange(len(a["exps"])) == 2, np.nan, a["exps"])),
    dict(coefs=lambda a: np.where(np.arange(len(a["coefs"])) == 1, np.inf, a["coefs"])),
    dict(shell_atom=lambda a: np.where(np.arange(len(a["shell_atom"])) == 0, 99, a["shell_atom"]).astype(np.int32)),
    dict(spherical=2),
    dict(natoms=0),
])
def test_invalid_descriptor_rejected(lib, bad):
    rc, h = _create(lib, _mutate(**bad))
    assert rc == jk.JK_EINVAL
    assert h.value is None
    assert len(jk.jk_last_error()) > 10


def test_null_arguments(lib):
    h = ctypes.c_void_p()
    assert lib.jk_create_basis(None, ctypes.byref(h)) == jk.JK_EINVAL
    d, keep = jk._desc(synth.random_basis(3, 2, 1).as_arrays())
    d.exps = None
    assert lib.jk_create_basis(ctypes.byref(d), ctypes.byref(h)) == jk.JK_EINVAL
    assert lib.jk_create_basis(ctypes.byref(d), None) == jk.JK_EINVAL
    lib.jk_destroy(None)                                  # NULL-safe
    assert lib.jk_nbf(None) == jk.JK_EINVAL
    assert lib.jk_build(None, 1, None, None, None, None) == jk.JK_EINVAL
    assert lib.jk_workspace_bytes(None, 4, None) == 0
    assert lib.jk_quartet_count(None, 1e-12) == jk.JK_EINVAL
    out = (ctypes.c_double * 6)()
    assert lib.jk_last_stats(None, out) == jk.JK_EINVAL
    assert lib.jk_eri_tiles(None, 1, None, None) == jk.JK_EINVAL


def test_last_error_is_per_thread(lib):
    import threading
    lib.jk_nbf(None)
    msg = jk.jk_last_error()
    seen = []

    def other():
        seen.append(jk.jk_last_error())

    t = threading.Thread(target=other)
    t.start()
    t.join()
    assert msg and seen == [""]


def test_header_constants_match_binding():
    txt = open(jk.HEADER).read()
    for name, val in [("JK_OK", 0), ("JK_EINVAL", -1), ("JK_ENOMEM", -2), ("JK_EDEVICE", -3),
                      ("JK_EUNSUPPORTED", -4), ("JK_FP64", 0), ("JK_MIXED", 1)]:
        assert f"#define {name} " in txt
        assert getattr(jk, name) == val


def test_tune_table_and_cache(tmp_path, lib):
    old = [jk.jk_tune_get(c) for c in range(21)]
    try:
        jk.jk_tune_set(3, 512, 8, 2, 64)
        assert jk.jk_tune_get(3) == dict(seg_max=512, g_max=8, dig_kernel=2, eri_block=64)
        for bad in [(-1, 256, 4), (21, 256, 4), (0, 0, 4), (0, 256, 3), (0, 256, 32), (0, 256, 16, 4),
                    (0, 256, 16, 1, 32), (0, 256, 16, 1, 512)]:
            with pytest.raises(jk.JKError):
                jk.jk_tune_set(*bad)
        p = tmp_path / "tune.json"
        p.write_text('{"arch": "gfx950", "entries": [\n'
                     '  {"class": 0, "seg_max": 2048, "g_max": 16, "dig_kernel": 2, "eri_block": 128,'
                     ' "ms_per_build": 0.1},\n'
                     '  {"class": 20, "seg_max": 128, "g_max": 4, "ms_per_build": 0.2}\n]}\n')
        jk.jk_tune_load(str(p))
        assert jk.jk_tune_get(0) == dict(seg_max=2048, g_max=16, dig_kernel=2, eri_block=128)
        # fields absent from an entry take their defaults
        assert jk.jk_tune_get(20) == dict(seg_max=128, g_max=4, dig_kernel=1, eri_block=256)
        q = tmp_path / "other.json"
        q.write_text('{"arch": "gfx942", "entries": [{"class": 0, "seg_max": 64, "g_max": 4}]}')
        with pytest.raises(jk.JKError):
            jk.jk_tune_load(str(q))
        assert jk.jk_tune_get(0)["seg_max"] == 2048
    finally:
        for c, t in enumerate(old):
            jk.jk_tune_set(c, **t)


def test_cd_entry_points_reject_bad_arguments_on_the_host():
    """Argument checks of the CD entry points run before any device work."""
    lib = jk.load()
    n = ctypes.c_int32(0)
    assert lib.jk_cd_factor(None, 1e-4, 1e-6, 10, None, None, ctypes.byref(n), None) == jk.JK_EINVAL
    assert lib.jk_cd_jk(0, 1, None, 1, 1, None, None, None, None, None) == jk.JK_EINVAL
    assert lib.jk_cd_jk(4, 1, None, 1, 0, None, None, None, None, None) == jk.JK_EINVAL
    # neither J nor K wanted
    assert lib.jk_cd_jk(4, 1, None, 1, 1, None, None, None, None, None) == jk.JK_EINVAL
    assert "both NULL" in jk.jk_last_error()
