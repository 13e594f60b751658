"""CPU oracle for the AO-direct J/K build (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``jk_oracle.c`` (plain C, FP64, OpenMP),
which shares no code with the GPU library; see that file's header for what
is computed and which passages of the paper each part follows.

Functions take a basis as the dict produced by ``Basis.as_arrays()`` from
the seeded input generator, or anything with the same keys.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jk_oracle.c")
_LIB = os.path.join(_HERE, "_liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no hand-written SIMD)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
        _lib.oracle_count_quartets.restype = ctypes.c_longlong
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _basis_args(b):
    if hasattr(b, "as_arrays"):
        b = b.as_arrays()
    keep = [b["xyz"], b["shell_atom"], b["shell_l"], b["shell_nprim"], b["exps"], b["coefs"]]
    args = [ctypes.c_int(int(b["natoms"])), _dp(b["xyz"]), ctypes.c_int(int(b["nshells"])),
            _ip(b["shell_atom"]), _ip(b["shell_l"]), _ip(b["shell_nprim"]), _dp(b["exps"]),
            _dp(b["coefs"]), ctypes.c_int(int(b["spherical"]))]
    return args, keep


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle: {what} rejected its arguments (rc={rc})")


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def threads() -> int:
    return int(_load().oracle_get_threads())


def boys(mmax: int, T: float) -> np.ndarray:
    F = np.zeros(mmax + 1)
    _load().oracle_boys(ctypes.c_int(mmax), ctypes.c_double(T), _dp(F))
    return F


def nbf(basis) -> int:
    args, _k = _basis_args(basis)
    return int(_load().oracle_nbf(*args))


def ncart(basis) -> int:
    args, _k = _basis_args(basis)
    return int(_load().oracle_ncart(*args))


def cart_to_basis(basis) -> np.ndarray:
    args, _k = _basis_args(basis)
    nc, nf = ncart(basis), nbf(basis)
    T = np.zeros((nc, nf))
    _check(_load().oracle_cart_to_basis(*args, _dp(T)), "cart_to_basis")
    return T


def eri_shell_quartet(basis, a, b, c, d, ncart_of) -> np.ndarray:
    """Cartesian tile (ab|cd); ``ncart_of`` gives the Cartesian size of a shell."""
    args, _k = _basis_args(basis)
    out = np.zeros((ncart_of(a), ncart_of(b), ncart_of(c), ncart_of(d)))
    _check(_load().oracle_eri_shell_quartet(*args, a, b, c, d, _dp(out)), "eri_shell_quartet")
    return out


def eri_full(basis) -> np.ndarray:
    args, _k = _basis_args(basis)
    n = nbf(basis)
    out = np.zeros((n, n, n, n))
    _check(_load().oracle_eri_full(*args, _dp(out)), "eri_full")
    return out


def overlap(basis) -> np.ndarray:
    args, _k = _basis_args(basis)
    n = nbf(basis)
    S = np.zeros((n, n))
    _check(_load().oracle_overlap(*args, _dp(S)), "overlap")
    return S


def schwarz(basis) -> np.ndarray:
    args, _k = _basis_args(basis)
    b = basis.as_arrays() if hasattr(basis, "as_arrays") else basis
    ns = int(b["nshells"])
    Q = np.zeros((ns, ns))
    _check(_load().oracle_schwarz(*args, _dp(Q)), "schwarz")
    return Q


def _dens(D, n):
    D = np.ascontiguousarray(D, dtype=np.float64)
    if D.ndim == 2:
        D = D[None]
    if D.shape[1:] != (n, n):
        raise ValueError(f"density shape {D.shape} does not match nbf={n}")
    return D


def jk_brute(basis, D):
    """J and K literally from the full ERI tensor (tiny bases only)."""
    args, _k = _basis_args(basis)
    n = nbf(basis)
    D = _dens(D, n)
    J = np.zeros_like(D)
    K = np.zeros_like(D)
    _check(_load().oracle_jk_brute(*args, D.shape[0], _dp(D), _dp(J), _dp(K)), "jk_brute")
    return J, K


def jk(basis, D, tol: float = 1e-12):
    """Screened J and K over canonical shell quartets (tol=0: unscreened)."""
    args, _k = _basis_args(basis)
    n = nbf(basis)
    D = _dens(D, n)
    J = np.zeros_like(D)
    K = np.zeros_like(D)
    _check(_load().oracle_jk_screened(*args, D.shape[0], _dp(D), _dp(J), _dp(K),
                                      ctypes.c_double(tol)), "jk_screened")
    return J, K


def jk_sample(basis, D, stride: int, offset: int = 0, tol: float = 1e-12):
    """Partial screened build over bra pairs with index % stride == offset.
    Returns (J_part, K_part, kept quartets visited, kept quartets total)."""
    args, _k = _basis_args(basis)
    n = nbf(basis)
    D = _dens(D, n)
    J = np.zeros_like(D)
    K = np.zeros_like(D)
    done = ctypes.c_longlong()
    total = ctypes.c_longlong()
    _check(_load().oracle_jk_screened_sample(*args, D.shape[0], _dp(D), _dp(J), _dp(K), ctypes.c_double(tol),
                                             int(stride), int(offset), ctypes.byref(done), ctypes.byref(total)),
           "jk_screened_sample")
    return J, K, int(done.value), int(total.value)


def count_quartets(basis, D, tol: float = 1e-12) -> int:
    args, _k = _basis_args(basis)
    n = nbf(basis)
    D = _dens(D, n)
    return int(_load().oracle_count_quartets(*args, D.shape[0], _dp(D), ctypes.c_double(tol)))


def jk_blocks(basis, D, pairs, tol: float = 1e-12):
    """User-basis blocks J[x][A][B], K[x][A][B] for shell pairs (A, B)."""
    args, _k = _basis_args(basis)
    b = basis.as_arrays() if hasattr(basis, "as_arrays") else basis
    n = nbf(basis)
    D = _dens(D, n)
    nd = D.shape[0]
    l = np.asarray(b["shell_l"])
    nf = np.where((l == 2) & (int(b["spherical"]) == 1), 5, (l + 1) * (l + 2) // 2)
    A = np.array([p[0] for p in pairs], dtype=np.int32)
    B = np.array([p[1] for p in pairs], dtype=np.int32)
    sizes = [nd * int(nf[a]) * int(nf[bb]) for a, bb in zip(A, B)]
    Jo = np.zeros(sum(sizes))
    Ko = np.zeros(sum(sizes))
    _check(_load().oracle_jk_blocks(*args, nd, _dp(D), ctypes.c_double(tol), len(pairs),
                                    _ip(A), _ip(B), _dp(Jo), _dp(Ko)), "jk_blocks")
    out = []
    off = 0
    for (a, bb), s in zip(zip(A, B), sizes):
        shp = (nd, int(nf[a]), int(nf[bb]))
        out.append((Jo[off:off + s].reshape(shp), Ko[off:off + s].reshape(shp)))
        off += s
    return out
