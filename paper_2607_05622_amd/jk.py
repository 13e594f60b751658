"""Python binding of the J/K C-ABI (include/jk.h): argument marshalling only.

Every step of a build runs in the HIP library ``libjk.so`` built next to this
file; there is no fallback.  If the library is missing this module raises on
first use.  Functions keep the C names; ``JKBasis`` is a small owner of a
handle.  Device arrays are torch tensors (``cuda``, float64, contiguous),
used only as memory and stream carriers.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjk.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "jk.h")

JK_OK, JK_EINVAL, JK_ENOMEM, JK_EDEVICE, JK_EUNSUPPORTED = 0, -1, -2, -3, -4
JK_FP64, JK_MIXED = 0, 1
JK_CD_MAX_VECTORS = 65535


class JKError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"jk error {code}: {msg}")
        self.code = code


class jk_basis_desc(ctypes.Structure):
    _fields_ = [("natoms", ctypes.c_int32), ("xyz", ctypes.POINTER(ctypes.c_double)),
                ("nshells", ctypes.c_int32), ("shell_atom", ctypes.POINTER(ctypes.c_int32)),
                ("shell_l", ctypes.POINTER(ctypes.c_int32)), ("shell_nprim", ctypes.POINTER(ctypes.c_int32)),
                ("exps", ctypes.POINTER(ctypes.c_double)), ("coefs", ctypes.POINTER(ctypes.c_double)),
                ("spherical", ctypes.c_int32)]


class jk_tune_t(ctypes.Structure):
    _fields_ = [("seg_max", ctypes.c_int32), ("g_max", ctypes.c_int32), ("dig_kernel", ctypes.c_int32),
                ("eri_block", ctypes.c_int32)]


class jk_build_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("schwarz_tol", ctypes.c_double),
                ("fp32_bound", ctypes.c_double), ("want_j", ctypes.c_int32), ("want_k", ctypes.c_int32),
                ("symmetric_hint", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libjk.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library {path} is missing: run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    vp, c_int, c_i64, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
    lib.jk_default_opts.argtypes = [ctypes.POINTER(jk_build_opts)]
    lib.jk_default_opts.restype = None
    lib.jk_create_basis.argtypes = [ctypes.POINTER(jk_basis_desc), ctypes.POINTER(vp)]
    lib.jk_create_basis.restype = c_int
    lib.jk_nbf.argtypes = [vp]
    lib.jk_nbf.restype = c_int
    lib.jk_build.argtypes = [vp, ctypes.c_int32, dp, dp, dp, ctypes.POINTER(jk_build_opts)]
    lib.jk_build.restype = c_int
    lib.jk_build_noalloc.argtypes = [vp, ctypes.c_int32, dp, dp, dp, ctypes.POINTER(jk_build_opts)]
    lib.jk_build_noalloc.restype = c_int
    lib.jk_workspace_bytes.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(jk_build_opts)]
    lib.jk_workspace_bytes.restype = ctypes.c_size_t
    lib.jk_destroy.argtypes = [vp]
    lib.jk_destroy.restype = None
    lib.jk_last_error.argtypes = []
    lib.jk_last_error.restype = ctypes.c_char_p
    lib.jk_quartet_count.argtypes = [vp, ctypes.c_double]
    lib.jk_quartet_count.restype = c_i64
    lib.jk_last_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.jk_last_stats.restype = c_int
    lib.jk_eri_tiles.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_double)]
    lib.jk_eri_tiles.restype = c_int
    pp = ctypes.POINTER(ctypes.c_void_p)
    lib.jk_build_batch.argtypes = [ctypes.c_int32, pp, ctypes.POINTER(ctypes.c_int32), pp, pp, pp,
                                   ctypes.POINTER(jk_build_opts)]
    lib.jk_build_batch.restype = c_int
    lib.jk_batch_workspace_bytes.argtypes = [ctypes.c_int32, pp, ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(jk_build_opts)]
    lib.jk_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.jk_autotune.argtypes = [vp, ctypes.c_int32, dp, dp, dp, ctypes.POINTER(jk_build_opts), ctypes.c_char_p]
    lib.jk_autotune.restype = c_int
    lib.jk_tune_load.argtypes = [ctypes.c_char_p]
    lib.jk_tune_load.restype = c_int
    lib.jk_tune_set.argtypes = [ctypes.c_int32, ctypes.POINTER(jk_tune_t)]
    lib.jk_tune_set.restype = c_int
    lib.jk_tune_get.argtypes = [ctypes.c_int32, ctypes.POINTER(jk_tune_t)]
    lib.jk_tune_get.restype = c_int
    lib.jk_graph_create.argtypes = [vp, ctypes.c_int32, dp, dp, dp, ctypes.POINTER(jk_build_opts),
                                    ctypes.POINTER(ctypes.c_void_p)]
    lib.jk_graph_create.restype = c_int
    lib.jk_graph_launch.argtypes = [vp, vp]
    lib.jk_graph_launch.restype = c_int
    lib.jk_graph_destroy.argtypes = [vp]
    lib.jk_graph_destroy.restype = None
    lib.jk_profile_enable.argtypes = [vp, ctypes.c_int32]
    lib.jk_profile_enable.restype = c_int
    lib.jk_profile_read.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
    lib.jk_profile_read.restype = c_int
    hd = ctypes.POINTER(ctypes.c_double)
    i32, f64 = ctypes.c_int32, ctypes.c_double
    lib.jk_laplace_grid.argtypes = [i32, f64, f64, hd, hd, hd]
    lib.jk_laplace_grid.restype = c_int
    lib.jk_laplace_shift.argtypes = [i32, hd, hd, f64, f64, hd]
    lib.jk_laplace_shift.restype = c_int
    lib.jk_laplace_densities.argtypes = [i32, i32, i32, dp, dp, i32, hd, i32, dp, dp, vp]
    lib.jk_laplace_densities.restype = c_int
    lib.jk_laplace_fock.argtypes = [i32, i32, i32, dp, i32, dp, dp, dp, dp, vp]
    lib.jk_laplace_fock.restype = c_int
    lib.jk_laplace_step.argtypes = [vp, i32, dp, dp, dp, i32, i32, dp, dp, i32, hd, dp, dp,
                                    ctypes.POINTER(jk_build_opts)]
    lib.jk_laplace_step.restype = c_int
    lib.jk_cd_factor.argtypes = [vp, f64, f64, i32, dp, dp, ctypes.POINTER(ctypes.c_int32), vp]
    lib.jk_cd_factor.restype = c_int
    lib.jk_cd_jk.argtypes = [i32, i32, dp, i32, i32, dp, dp, dp, dp, vp]
    lib.jk_cd_jk.restype = c_int
    _lib = lib
    return lib


def declared_functions(header: str = HEADER) -> list[str]:
    """Names of the functions include/jk.h declares."""
    txt = open(header).read()
    return sorted(set(re.findall(r"\b(jk_[a-z_]+)\s*\(", txt)))


def jk_last_error() -> str:
    return load().jk_last_error().decode()


def _check(rc):
    if rc != JK_OK:
        raise JKError(rc, jk_last_error())


def jk_default_opts(**kw) -> jk_build_opts:
    o = jk_build_opts()
    load().jk_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _desc(arrays: dict):
    keep = dict(
        xyz=np.ascontiguousarray(arrays["xyz"], dtype=np.float64).reshape(-1),
        shell_atom=np.ascontiguousarray(arrays["shell_atom"], dtype=np.int32),
        shell_l=np.ascontiguousarray(arrays["shell_l"], dtype=np.int32),
        shell_nprim=np.ascontiguousarray(arrays["shell_nprim"], dtype=np.int32),
        exps=np.ascontiguousarray(arrays["exps"], dtype=np.float64),
        coefs=np.ascontiguousarray(arrays["coefs"], dtype=np.float64))
    d = jk_basis_desc()
    d.natoms = int(arrays["natoms"])
    d.nshells = int(arrays["nshells"])
    d.spherical = int(arrays["spherical"])
    for k in ("xyz", "exps", "coefs"):
        setattr(d, k, keep[k].ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    for k in ("shell_atom", "shell_l", "shell_nprim"):
        setattr(d, k, keep[k].ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return d, keep


def jk_create_basis(basis) -> int:
    """Returns the opaque handle as an integer; ``basis`` is a synth.Basis or
    a dict with the descriptor's arrays."""
    arrays = basis.as_arrays() if hasattr(basis, "as_arrays") else basis
    d, keep = _desc(arrays)
    h = ctypes.c_void_p()
    _check(load().jk_create_basis(ctypes.byref(d), ctypes.byref(h)))
    del keep
    return h.value


def jk_nbf(h) -> int:
    n = load().jk_nbf(h)
    if n < 0:
        _check(n)
    return n


def jk_destroy(h) -> None:
    load().jk_destroy(h)


def jk_quartet_count(h, tol: float = 1e-12) -> int:
    n = load().jk_quartet_count(h, tol)
    if n < 0:
        _check(int(n))
    return int(n)


def jk_last_stats(h) -> dict:
    out = (ctypes.c_double * 6)()
    _check(load().jk_last_stats(h, out))
    keys = ["quartets", "quartets_fp32", "function_quartets", "primitive_quartets", "eri_flops", "digest_flops"]
    return dict(zip(keys, list(out)))


def jk_workspace_bytes(h, nd: int, opts: jk_build_opts | None = None) -> int:
    return int(load().jk_workspace_bytes(h, nd, ctypes.byref(opts) if opts is not None else None))


def _dev_ptr(t, n, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 cuda tensor")
    if t.dim() != 3 or t.shape[1] != n or t.shape[2] != n:
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected [nd, {n}, {n}]")
    return t.data_ptr()


def jk_build(h, D, J=None, K=None, opts: jk_build_opts | None = None, stream=None):
    """J and K of the densities D[nd, n, n] (torch cuda float64).  Output
    tensors are allocated when not given.  Runs on ``stream`` (a
    torch.cuda.Stream) or torch's current stream."""
    import torch
    n = jk_nbf(h)
    if D.dim() == 2:
        D = D.unsqueeze(0)
    nd = D.shape[0]
    o = opts if opts is not None else jk_default_opts()
    if J is None and o.want_j:
        J = torch.empty_like(D)
    if K is None and o.want_k:
        K = torch.empty_like(D)
    s = stream if stream is not None else torch.cuda.current_stream(D.device)
    o.stream = ctypes.c_void_p(s.cuda_stream)
    dp = _dev_ptr(D, n, "D")
    jp = _dev_ptr(J, n, "J") if o.want_j else None
    kp = _dev_ptr(K, n, "K") if o.want_k else None
    _check(load().jk_build(h, nd, dp, jp, kp, ctypes.byref(o)))
    return J, K


def _ptr_array(vals):
    arr = (ctypes.c_void_p * len(vals))()
    for i, v in enumerate(vals):
        arr[i] = v
    return arr


def jk_batch_workspace_bytes(hs, nds, opts: jk_build_opts | None = None) -> int:
    nd = (ctypes.c_int32 * len(nds))(*nds)
    return int(load().jk_batch_workspace_bytes(len(hs), _ptr_array(hs), nd,
                                               ctypes.byref(opts) if opts is not None else None))


def jk_build_batch(hs, Ds, Js=None, Ks=None, opts: jk_build_opts | None = None, stream=None):
    """One batched build over several molecules: hs handles, Ds list of
    [nd_i, n_i, n_i] cuda float64 tensors.  Returns lists Js, Ks."""
    import torch
    o = opts if opts is not None else jk_default_opts()
    nmol = len(hs)
    if len(Ds) != nmol:
        raise ValueError("one density tensor per handle")
    ns = [jk_nbf(h) for h in hs]
    Js = Js if Js is not None else ([torch.empty_like(D) for D in Ds] if o.want_j else [None] * nmol)
    Ks = Ks if Ks is not None else ([torch.empty_like(D) for D in Ds] if o.want_k else [None] * nmol)
    dps = [_dev_ptr(D, n, "D") for D, n in zip(Ds, ns)]
    jps = [_dev_ptr(J, n, "J") if o.want_j else None for J, n in zip(Js, ns)]
    kps = [_dev_ptr(K, n, "K") if o.want_k else None for K, n in zip(Ks, ns)]
    s = stream if stream is not None else torch.cuda.current_stream(Ds[0].device)
    o.stream = ctypes.c_void_p(s.cuda_stream)
    nd = (ctypes.c_int32 * nmol)(*[int(D.shape[0]) for D in Ds])
    _check(load().jk_build_batch(nmol, _ptr_array(hs), nd, _ptr_array(dps), _ptr_array(jps), _ptr_array(kps),
                                 ctypes.byref(o)))
    return Js, Ks


def jk_autotune(h, D, J, K, opts: jk_build_opts | None = None, cache_path: str | None = None, stream=None):
    import torch
    n = jk_nbf(h)
    o = opts if opts is not None else jk_default_opts()
    s = stream if stream is not None else torch.cuda.current_stream(D.device)
    o.stream = ctypes.c_void_p(s.cuda_stream)
    _check(load().jk_autotune(h, int(D.shape[0]), _dev_ptr(D, n, "D"), _dev_ptr(J, n, "J"), _dev_ptr(K, n, "K"),
                              ctypes.byref(o), cache_path.encode() if cache_path else None))


def jk_tune_load(path: str) -> None:
    _check(load().jk_tune_load(path.encode()))


def jk_tune_set(cls: int, seg_max: int = 128, g_max: int = 16, dig_kernel: int = 1, eri_block: int = 256) -> None:
    t = jk_tune_t(seg_max, g_max, dig_kernel, eri_block)
    _check(load().jk_tune_set(cls, ctypes.byref(t)))


def jk_tune_get(cls: int) -> dict:
    t = jk_tune_t()
    _check(load().jk_tune_get(cls, ctypes.byref(t)))
    return dict(seg_max=t.seg_max, g_max=t.g_max, dig_kernel=t.dig_kernel, eri_block=t.eri_block)


def jk_graph_create(h, D, J, K, opts: jk_build_opts) -> int:
    """Capture one build into a HIP graph (opts.workspace required)."""
    n = jk_nbf(h)
    g = ctypes.c_void_p()
    _check(load().jk_graph_create(h, int(D.shape[0]), _dev_ptr(D, n, "D"), _dev_ptr(J, n, "J") if opts.want_j else None,
                                  _dev_ptr(K, n, "K") if opts.want_k else None, ctypes.byref(opts), ctypes.byref(g)))
    return g.value


def jk_graph_launch(g, stream=None) -> None:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(load().jk_graph_launch(g, ctypes.c_void_p(s.cuda_stream)))


def jk_graph_destroy(g) -> None:
    load().jk_graph_destroy(g)


def jk_profile_enable(h, on: bool) -> None:
    _check(load().jk_profile_enable(h, 1 if on else 0))


def jk_profile_read(h, kind: int, cls: int) -> dict:
    out = (ctypes.c_double * 5)()
    _check(load().jk_profile_read(h, kind, cls, out))
    return dict(zip(["ms", "launches", "flops", "quartets", "bytes"], list(out)))


def jk_eri_tiles(h, shells, shell_l) -> list:
    """Cartesian ERI tiles for user shell quartets [(a, b, c, d), ...];
    ``shell_l`` gives each user shell's angular momentum (tile sizes)."""
    sh = np.ascontiguousarray(np.asarray(shells, dtype=np.int32).reshape(-1, 4))
    l = np.asarray(shell_l)
    nc = (l + 1) * (l + 2) // 2
    sizes = [int(np.prod([nc[s] for s in q])) for q in sh]
    out = np.zeros(max(sum(sizes), 1))
    _check(load().jk_eri_tiles(h, len(sh), sh.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    res, off = [], 0
    for q, s in zip(sh, sizes):
        res.append(out[off:off + s].reshape([int(nc[x]) for x in q]))
        off += s
    return res


class JKBasis:
    """Owner of one library handle."""

    def __init__(self, basis):
        self.basis = basis
        self.h = jk_create_basis(basis)
        self.nbf = jk_nbf(self.h)

    def build(self, D, J=None, K=None, stream=None, **opts):
        o = jk_default_opts(**opts) if opts else None
        return jk_build(self.h, D, J, K, o, stream)

    def eri_tiles(self, shells):
        arrays = self.basis.as_arrays() if hasattr(self.basis, "as_arrays") else self.basis
        return jk_eri_tiles(self.h, shells, arrays["shell_l"])

    def quartet_count(self, tol=1e-12):
        return jk_quartet_count(self.h, tol)

    def stats(self):
        return jk_last_stats(self.h)

    def close(self):
        if self.h:
            jk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------ Laplace grids and cascade --

def _hd(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def jk_laplace_grid(n: int, xmin: float, xmax: float):
    """Minimax grid (tau, w, max_err) for 1/x on [xmin, xmax] (host arrays)."""
    tau, w, err = np.zeros(n), np.zeros(n), ctypes.c_double()
    _check(load().jk_laplace_grid(n, xmin, xmax, _hd(tau), _hd(w), ctypes.byref(err)))
    return tau, w, err.value


def jk_laplace_shift(tau, w, omega: float, dmin: float):
    """Weights reweighted for 1/(D - omega)."""
    tau, w = np.ascontiguousarray(tau, dtype=np.float64), np.ascontiguousarray(w, dtype=np.float64)
    out = np.zeros_like(w)
    _check(load().jk_laplace_shift(len(tau), _hd(tau), _hd(w), omega, dmin, _hd(out)))
    return out


def _dev_mat(t, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 cuda tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


def _stream(s, dev):
    import torch
    s = s if s is not None else torch.cuda.current_stream(dev)
    return ctypes.c_void_p(s.cuda_stream)


def jk_laplace_densities(C, eps, nocc: int, tau, R, D=None, stream=None):
    """D[r, k] = U^k R[r] (V^k)^T for residuals R[nr, nocc, nvir] on the grid
    tau (host); C[n, nmo] and eps[nmo] on the device."""
    import torch
    n, nmo = C.shape
    nvir = nmo - nocc
    nr = R.shape[0]
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    if D is None:
        D = torch.empty((nr, len(tau), n, n), dtype=torch.float64, device=C.device)
    _check(load().jk_laplace_densities(n, nocc, nvir, _dev_mat(C, (n, nmo), "C"), _dev_mat(eps, (nmo,), "eps"),
                                       len(tau), _hd(tau), nr, _dev_mat(R, (nr, nocc, nvir), "R"),
                                       _dev_mat(D, (nr, len(tau), n, n), "D"), _stream(stream, C.device)))
    return D


def jk_laplace_fock(C, nocc: int, J, K, F=None, Rov=None, want_f=True, want_r=True, stream=None):
    """F = C^T (2J - K) C per density and its occupied-virtual block."""
    import torch
    n, nmo = C.shape
    nvir = nmo - nocc
    nd = J.shape[0]
    if want_f and F is None:
        F = torch.empty((nd, nmo, nmo), dtype=torch.float64, device=C.device)
    if want_r and Rov is None:
        Rov = torch.empty((nd, nocc, nvir), dtype=torch.float64, device=C.device)
    _check(load().jk_laplace_fock(n, nocc, nvir, _dev_mat(C, (n, nmo), "C"), nd, _dev_mat(J, (nd, n, n), "J"),
                                  _dev_mat(K, (nd, n, n), "K"),
                                  _dev_mat(F, (nd, nmo, nmo), "F") if want_f else None,
                                  _dev_mat(Rov, (nd, nocc, nvir), "Rov") if want_r else None,
                                  _stream(stream, C.device)))
    return F, Rov


def jk_laplace_step(h, D, C, eps, nocc: int, tau, opts: jk_build_opts | None = None, stream=None):
    """One forward edge of the cascade: returns (J, K, Rov, Dnext)."""
    import torch
    n = jk_nbf(h)
    nd = D.shape[0]
    nmo = C.shape[1]
    nvir = nmo - nocc
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    J, K = torch.empty_like(D), torch.empty_like(D)
    Rov = torch.empty((nd, nocc, nvir), dtype=torch.float64, device=D.device)
    Dn = torch.empty((nd, len(tau), n, n), dtype=torch.float64, device=D.device)
    o = opts if opts is not None else jk_default_opts()
    o.stream = _stream(stream, D.device)
    _check(load().jk_laplace_step(h, nd, _dev_ptr(D, n, "D"), _dev_ptr(J, n, "J"), _dev_ptr(K, n, "K"), nocc, nvir,
                                  _dev_mat(C, (n, nmo), "C"), _dev_mat(eps, (nmo,), "eps"), len(tau), _hd(tau),
                                  _dev_mat(Rov, (nd, nocc, nvir), "Rov"), _dev_mat(Dn, (nd, len(tau), n, n), "Dnext"),
                                  ctypes.byref(o)))
    return J, K, Rov, Dn


def jk_cd_factor(h, delta: float, screen_tol: float | None = None, max_vectors: int | None = None,
                 device=None, stream=None):
    """The factor of Eq. (cdfact): returns (B [nvec, n, n], pivots [nvec]) as
    torch cuda tensors.  screen_tol defaults to 0.01 delta; max_vectors to
    min(8 n, n (n + 1) / 2) (the call fails if more are needed)."""
    import torch
    n = jk_nbf(h)
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    if screen_tol is None:
        screen_tol = 0.01 * delta
    if max_vectors is None:
        max_vectors = min(8 * n, n * (n + 1) // 2, JK_CD_MAX_VECTORS)
    B = torch.empty((max(max_vectors, 1), n, n), dtype=torch.float64, device=dev)
    piv = torch.empty((max(max_vectors, 1),), dtype=torch.int32, device=dev)
    nvec = ctypes.c_int32(0)
    _check(load().jk_cd_factor(h, float(delta), float(screen_tol), int(max_vectors), B.data_ptr(), piv.data_ptr(),
                               ctypes.byref(nvec), _stream(stream, dev)))
    k = nvec.value
    return B[:k], piv[:k]


def jk_cd_jk(B, U, V, want_j: bool = True, want_k: bool = True, stream=None):
    """J and K of D[x] = U[x] V[x]^T (U, V [nd, n, r]) from the factor B
    [nvec, n, n]: Eqs. (cdj) and (cdknonsym)."""
    import torch
    nvec, n = B.shape[0], U.shape[1]
    nd, r = U.shape[0], U.shape[2]
    J = torch.empty((nd, n, n), dtype=torch.float64, device=U.device) if want_j else None
    K = torch.empty((nd, n, n), dtype=torch.float64, device=U.device) if want_k else None
    if nvec == 0:
        B = torch.empty((1, n, n), dtype=torch.float64, device=U.device)
    _check(load().jk_cd_jk(n, nvec, _dev_mat(B, (max(nvec, 1), n, n), "B"), nd, r, _dev_mat(U, (nd, n, r), "U"),
                           _dev_mat(V, (nd, n, r), "V"), J.data_ptr() if want_j else None,
                           K.data_ptr() if want_k else None, _stream(stream, U.device)))
    return J, K
