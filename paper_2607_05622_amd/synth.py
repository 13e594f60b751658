"""Seeded synthetic workloads for the AO-direct J/K build.

This module only draws inputs: molecules, contracted s/p/d Gaussian shells and
the (generally non-symmetric) densities that are fed to a J/K build.  It holds
none of the build's arithmetic (no two-electron integrals, no J/K contraction)
and imports nothing else from this package, so that both the GPU path and the
CPU oracle can be driven from the same bytes.

Shapes follow the paper's workloads (Sect. "Performance on the RTX 4060": 28 to
730 AO, up to the memory ceiling) and its density definitions:

* Laplace-scaled coefficients and the level-1 AO pseudo-density, Eqs.
  (scaledcoeff) and (aodens): U = C_occ e^{+eps_i t}, V = C_vir e^{-eps_a t},
  D = U T V^T, with T a random occupied-virtual amplitude block standing in for
  the residual of Eq. (aodensk).
* The Laplace identity of Eq. (laplace), 1/x ~ sum_k w_k exp(-x t_k), with
  least-squares weights on fixed log-spaced nodes (the paper uses minimax
  grids; fixed nodes are what the workloads prescribe).

The one integral that is computed here is the overlap matrix, needed to
Loewdin-orthonormalize random MO coefficients.  It is written out on its own
(Obara-Saika one-dimensional overlaps) and is used for nothing else.

Conventions shared with every consumer of a basis (they define the basis, not
the method):

* a primitive of angular momentum l is normalized on its x^l component;
  each Cartesian component keeps that constant (d_xy then has self-overlap
  1/3);
* a contraction is rescaled so that its x^l component has unit self-overlap;
* Cartesian order within a shell is lexicographic (xx, xy, xz, yy, yz, zz),
  p is (x, y, z);
* pure d functions are ordered m = -2..2 as (xy, yz, 3z^2-r^2, xz, x^2-y^2),
  each of unit self-overlap.

All randomness uses numpy's PCG64 with the seeds documented per workload.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Cartesian exponent triples in lexicographic order, per l.
CART = {
    0: [(0, 0, 0)],
    1: [(1, 0, 0), (0, 1, 0), (0, 0, 1)],
    2: [(2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)],
}

# Pure-d coefficients over x^2-normalized Cartesian d components
# (rows: xy, yz, z2, xz, x2-y2; columns: xx, xy, xz, yy, yz, zz).
_S3 = math.sqrt(3.0)
SPH_D = np.array([
    [0.0, _S3, 0.0, 0.0, 0.0, 0.0],
    [0.0, 0.0, 0.0, 0.0, _S3, 0.0],
    [-0.5, 0.0, 0.0, -0.5, 0.0, 1.0],
    [0.0, 0.0, _S3, 0.0, 0.0, 0.0],
    [_S3 / 2, 0.0, 0.0, -_S3 / 2, 0.0, 0.0],
])

HEAVY_SP = (0, 0, 0, 1, 1)          # 3 s + 2 p
HEAVY_SPD = (0, 0, 0, 1, 1, 2)      # 3 s + 2 p + 1 d
LIGHT = (0, 0, 1)                   # 2 s + 1 p
NPRIM = 3
EXP_RANGE = (0.15, 50.0)


def _dfact(n: int) -> float:
    r = 1.0
    while n > 1:
        r *= n
        n -= 2
    return r


@dataclass
class Basis:
    """A molecule and its contracted shells, laid out as the C-ABI takes them."""

    xyz: np.ndarray            # [natoms, 3] bohr
    charges: np.ndarray        # [natoms] labels only (8 heavy, 1 light)
    shell_atom: np.ndarray     # [nshell] int32
    shell_l: np.ndarray        # [nshell] int32
    shell_nprim: np.ndarray    # [nshell] int32
    exps: np.ndarray           # concatenated primitive exponents
    coefs: np.ndarray          # concatenated coefficients of unit-normalized primitives
    spherical: int = 1

    @property
    def natoms(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def nshells(self) -> int:
        return int(self.shell_l.shape[0])

    def shell_nfunc(self) -> np.ndarray:
        l = self.shell_l
        if self.spherical:
            return 2 * l + 1
        return (l + 1) * (l + 2) // 2

    def nbf(self) -> int:
        return int(self.shell_nfunc().sum())

    def ncart(self) -> int:
        l = self.shell_l
        return int(((l + 1) * (l + 2) // 2).sum())

    def prim_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.shell_nprim)]).astype(np.int64)

    def func_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.shell_nfunc())]).astype(np.int64)

    def as_arrays(self) -> dict:
        """Contiguous arrays with the dtypes of the C-ABI descriptor."""
        return dict(
            xyz=np.ascontiguousarray(self.xyz, dtype=np.float64).reshape(-1),
            shell_atom=np.ascontiguousarray(self.shell_atom, dtype=np.int32),
            shell_l=np.ascontiguousarray(self.shell_l, dtype=np.int32),
            shell_nprim=np.ascontiguousarray(self.shell_nprim, dtype=np.int32),
            exps=np.ascontiguousarray(self.exps, dtype=np.float64),
            coefs=np.ascontiguousarray(self.coefs, dtype=np.float64),
            spherical=int(self.spherical),
            natoms=self.natoms,
            nshells=self.nshells,
        )

    def translated(self, shift) -> "Basis":
        b = Basis(**{k: getattr(self, k).copy() if isinstance(getattr(self, k), np.ndarray)
                     else getattr(self, k) for k in self.__dataclass_fields__})
        b.xyz = b.xyz + np.asarray(shift, dtype=np.float64)[None, :]
        return b

    def subset(self, shells) -> "Basis":
        """The same molecule restricted to the listed shells (in that order)."""
        shells = list(shells)
        po = self.prim_offsets()
        ex = np.concatenate([self.exps[po[s]:po[s + 1]] for s in shells]) if shells else np.zeros(0)
        co = np.concatenate([self.coefs[po[s]:po[s + 1]] for s in shells]) if shells else np.zeros(0)
        return Basis(self.xyz.copy(), self.charges.copy(),
                     self.shell_atom[shells].copy(), self.shell_l[shells].copy(),
                     self.shell_nprim[shells].copy(), ex, co, self.spherical)


# --------------------------------------------------------------------------
# geometry and shells
# --------------------------------------------------------------------------

def random_geometry(rng: np.random.Generator, n_atoms: int,
                    dmin: float = 2.2, dmax: float = 3.0) -> np.ndarray:
    """Random sequential addition inside a sphere.

    The first atom sits at the origin.  Each further atom is placed at
    dmin..dmax bohr (uniform) from a randomly chosen existing atom along a
    random direction, and is accepted when it is at least dmin from every
    other atom and inside a sphere of radius 2.6 n^(1/3) bohr.  Every atom's
    nearest neighbour therefore lies in [dmin, dmax].
    """
    radius = 2.6 * max(n_atoms, 1) ** (1.0 / 3.0)
    pos = [np.zeros(3)]
    tries = 0
    while len(pos) < n_atoms:
        tries += 1
        if tries > 200000:
            raise RuntimeError("geometry generation did not converge")
        parent = pos[int(rng.integers(len(pos)))]
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        cand = parent + v * rng.uniform(dmin, dmax)
        if np.linalg.norm(cand) > radius:
            continue
        d = np.linalg.norm(np.asarray(pos) - cand[None, :], axis=1)
        if d.min() < dmin:
            continue
        pos.append(cand)
    return np.asarray(pos, dtype=np.float64)


def _same_centre_overlap(a, b, l):
    """<x^l e^{-a r^2} | x^l e^{-b r^2}> for unit-normalized primitives."""
    return (2.0 * np.sqrt(a * b) / (a + b)) ** (l + 1.5)


def random_shell(rng: np.random.Generator, l: int, nprim: int = NPRIM):
    """Exponents log-uniform on [0.15, 50]; N(0,1) coefficients of
    unit-normalized primitives, redrawn when the contraction nearly cancels
    (norm below 1e-3 of sqrt(sum c^2))."""
    lo, hi = np.log(EXP_RANGE[0]), np.log(EXP_RANGE[1])
    while True:
        ex = np.exp(rng.uniform(lo, hi, size=nprim))
        c = rng.normal(size=nprim)
        s = _same_centre_overlap(ex[:, None], ex[None, :], l)
        norm2 = float(c @ s @ c)
        if norm2 > (1e-3) ** 2 * float(c @ c):
            return ex, c


def make_basis(rng: np.random.Generator, n_atoms: int, n_heavy: int,
               heavy=HEAVY_SPD, light=LIGHT, spherical: int = 1, nprims=(NPRIM,)) -> Basis:
    """Shell k of the molecule (in order) gets nprims[k % len(nprims)]
    primitives."""
    xyz = random_geometry(rng, n_atoms)
    charges = np.array([8.0] * n_heavy + [1.0] * (n_atoms - n_heavy))
    sa, sl, sn, ex, co = [], [], [], [], []
    for ia in range(n_atoms):
        for l in (heavy if ia < n_heavy else light):
            e, c = random_shell(rng, l, int(nprims[len(sl) % len(nprims)]))
            sa.append(ia)
            sl.append(l)
            sn.append(len(e))
            ex.append(e)
            co.append(c)
    return Basis(xyz, charges, np.array(sa, np.int32), np.array(sl, np.int32),
                 np.array(sn, np.int32), np.concatenate(ex), np.concatenate(co),
                 spherical)


# --------------------------------------------------------------------------
# overlap (for Loewdin orthonormalization only)
# --------------------------------------------------------------------------

def _os_overlap_1d(la, lb, PA, PB, p):
    """1-D Obara-Saika overlap table s[i, j] / s[0, 0] for i<=la, j<=lb."""
    s = np.zeros((la + 1, lb + 1) + np.shape(p))
    s[0, 0] = 1.0
    for i in range(la + 1):
        for j in range(lb + 1):
            if i == 0 and j == 0:
                continue
            if i > 0:
                v = PA * s[i - 1, j]
                if i > 1:
                    v = v + (i - 1) / (2 * p) * s[i - 2, j]
                if j > 0:
                    v = v + j / (2 * p) * s[i - 1, j - 1]
            else:
                v = PB * s[i, j - 1]
                if j > 1:
                    v = v + (j - 1) / (2 * p) * s[i, j - 2]
            s[i, j] = v
    return s


def _contraction_scale(ex, c, l):
    """Factor that makes the contraction's x^l component unit-normalized."""
    s = _same_centre_overlap(ex[:, None], ex[None, :], l)
    return 1.0 / math.sqrt(float(c @ s @ c))


def _prim_norm(a, l):
    return np.sqrt((2 * a / np.pi) ** 1.5 * (4 * a) ** l / _dfact(2 * l - 1))


def overlap_matrix(basis: Basis) -> np.ndarray:
    """Overlap matrix in the basis' own functions (pure d if spherical).

    Vectorized over all shell pairs of one (l_a, l_b) combination and their
    primitive pairs."""
    po = basis.prim_offsets()
    ns = basis.nshells
    npmax = int(basis.shell_nprim.max())
    ls = np.asarray(basis.shell_l)
    # padded primitive tables: exponents (1.0 where absent) and weights (0)
    ex = np.ones((ns, npmax))
    wt = np.zeros((ns, npmax))
    for s in range(ns):
        l = int(ls[s])
        e = basis.exps[po[s]:po[s + 1]]
        c = basis.coefs[po[s]:po[s + 1]]
        ex[s, :len(e)] = e
        wt[s, :len(e)] = c * _prim_norm(e, l) * _contraction_scale(e, c, l)
    cen = basis.xyz[basis.shell_atom]
    ncart = np.array([len(CART[int(l)]) for l in ls])
    co = np.concatenate([[0], np.cumsum(ncart)])
    S = np.zeros((co[-1], co[-1]))
    for li in range(int(ls.max()) + 1):
        for lj in range(li + 1):
            I = np.nonzero(ls == li)[0]
            Jn = np.nonzero(ls == lj)[0]
            ii, jj = np.meshgrid(I, Jn, indexing="ij")
            ii, jj = ii.ravel(), jj.ravel()
            if li == lj:
                keep = ii >= jj
                ii, jj = ii[keep], jj[keep]
            if len(ii) == 0:
                continue
            a = ex[ii][:, :, None]          # [npair, npa, 1]
            b = ex[jj][:, None, :]          # [npair, 1, npb]
            p = a + b
            A = cen[ii]
            B = cen[jj]
            ab2 = np.sum((A - B) ** 2, axis=1)[:, None, None]
            pref = (np.pi / p) ** 1.5 * np.exp(-a * b / p * ab2)
            w = wt[ii][:, :, None] * wt[jj][:, None, :] * pref
            tabs = []
            for k in range(3):
                P = (a * A[:, k, None, None] + b * B[:, k, None, None]) / p
                tabs.append(_os_overlap_1d(li, lj, P - A[:, k, None, None], P - B[:, k, None, None], p))
            blk = np.zeros((len(ii), len(CART[li]), len(CART[lj])))
            for u, (ax, ay, az) in enumerate(CART[li]):
                for v, (bx, by, bz) in enumerate(CART[lj]):
                    blk[:, u, v] = np.sum(w * tabs[0][ax, bx] * tabs[1][ay, by] * tabs[2][az, bz], axis=(1, 2))
            for t in range(len(ii)):
                i, j = ii[t], jj[t]
                S[co[i]:co[i + 1], co[j]:co[j + 1]] = blk[t]
                S[co[j]:co[j + 1], co[i]:co[i + 1]] = blk[t].T
    T = cart_to_basis_matrix(basis)
    return T.T @ S @ T


def cart_to_basis_matrix(basis: Basis) -> np.ndarray:
    """T with phi_basis = sum_cart T[cart, basis] phi_cart (identity for
    Cartesian bases and for s/p shells)."""
    nc = [len(CART[int(l)]) for l in basis.shell_l]
    nf = basis.shell_nfunc()
    T = np.zeros((sum(nc), int(nf.sum())))
    ci = fi = 0
    for s, l in enumerate(basis.shell_l):
        if l == 2 and basis.spherical:
            T[ci:ci + 6, fi:fi + 5] = SPH_D.T
        else:
            T[ci:ci + nc[s], fi:fi + nc[s]] = np.eye(nc[s])
        ci += nc[s]
        fi += int(nf[s])
    return T


def loewdin(C: np.ndarray, S: np.ndarray) -> np.ndarray:
    """C (C^T S C)^{-1/2}: columns orthonormal under S."""
    M = C.T @ S @ C
    w, V = np.linalg.eigh(M)
    return C @ (V * (1.0 / np.sqrt(w))) @ V.T


# --------------------------------------------------------------------------
# Laplace grid and densities
# --------------------------------------------------------------------------

def laplace_nodes(n: int, lo: float = 0.05, hi: float = 20.0) -> np.ndarray:
    return np.exp(np.linspace(np.log(lo), np.log(hi), n))


def laplace_weights(t: np.ndarray, xmin: float, xmax: float, nsample: int = 4000) -> np.ndarray:
    """Least-squares weights for 1/x ~ sum_k w_k exp(-x t_k) on [xmin, xmax],
    minimizing the relative error x*sum - 1 on a log-dense sample."""
    x = np.exp(np.linspace(np.log(xmin), np.log(xmax), nsample))
    A = x[:, None] * np.exp(-x[:, None] * t[None, :])
    w, *_ = np.linalg.lstsq(A, np.ones_like(x), rcond=None)
    return w


def laplace_max_rel_error(t, w, xmin, xmax, nsample: int = 20000) -> float:
    x = np.exp(np.linspace(np.log(xmin), np.log(xmax), nsample))
    return float(np.max(np.abs(x * (np.exp(-np.outer(x, t)) @ w) - 1.0)))


@dataclass
class Orbitals:
    C: np.ndarray          # [nbf, nbf], columns orthonormal under S
    eps: np.ndarray        # [nbf]
    n_occ: int

    @property
    def C_occ(self):
        return self.C[:, :self.n_occ]

    @property
    def C_vir(self):
        return self.C[:, self.n_occ:]

    @property
    def e_occ(self):
        return self.eps[:self.n_occ]

    @property
    def e_vir(self):
        return self.eps[self.n_occ:]

    def gap_range(self):
        d = self.e_vir[None, :] - self.e_occ[:, None]
        return float(d.min()), float(d.max())


def random_orbitals(rng: np.random.Generator, basis: Basis, n_occ: int) -> Orbitals:
    n = basis.nbf()
    S = overlap_matrix(basis)
    C = loewdin(rng.normal(size=(n, n)), S)
    eps = np.concatenate([rng.uniform(-1.5, -0.3, size=n_occ),
                          rng.uniform(0.1, 3.0, size=n - n_occ)])
    return Orbitals(C, eps, n_occ)


def laplace_density(orb: Orbitals, T: np.ndarray, t: float) -> np.ndarray:
    """Level-1 pseudo-density C_occ diag(e^{eps_i t}) T diag(e^{-eps_a t}) C_vir^T."""
    U = orb.C_occ * np.exp(orb.e_occ * t)[None, :]
    V = orb.C_vir * np.exp(-orb.e_vir * t)[None, :]
    return U @ T @ V.T


def laplace_densities(rng: np.random.Generator, orb: Orbitals, t: np.ndarray,
                      n_states: int, amp_sd: float = 0.05):
    """Densities ordered [state][node]; amplitudes T_ia ~ N(0, amp_sd)."""
    nv = orb.C.shape[1] - orb.n_occ
    Ts = [rng.normal(scale=amp_sd, size=(orb.n_occ, nv)) for _ in range(n_states)]
    D = np.stack([laplace_density(orb, Ts[s], tk) for s in range(n_states) for tk in t])
    return D, Ts


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    basis: Basis
    D: np.ndarray                       # [nd, nbf, nbf]
    meta: dict = field(default_factory=dict)


def config0(seed: int = 0) -> Workload:
    """28 AO: 2 heavy (3s2p) + 2 light (2s1p), two random densities (one
    symmetric, one not) and four Laplace pseudo-densities (n_occ 9)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    basis = make_basis(rng, 4, 2, heavy=HEAVY_SP, light=LIGHT, spherical=1)
    n = basis.nbf()
    u = rng.normal(size=(n, n)) * 0.1
    dsym = np.triu(u) + np.triu(u, 1).T
    dns = rng.normal(size=(n, n)) * 0.1
    orb = random_orbitals(rng, basis, 9)
    t = laplace_nodes(4)
    DL, _ = laplace_densities(rng, orb, t, 1)
    return Workload("tiny-28ao", basis, np.stack([dsym, dns]),
                    dict(laplace_D=DL, t=t, orbitals=orb))


def laplace_workload(name: str, seed: int, n_atoms: int, n_heavy: int, n_occ: int,
                     n_t: int, n_states: int) -> Workload:
    rng = np.random.Generator(np.random.PCG64(seed))
    basis = make_basis(rng, n_atoms, n_heavy)
    orb = random_orbitals(rng, basis, min(n_occ, basis.nbf() - 1))
    t = laplace_nodes(n_t)
    D, Ts = laplace_densities(rng, orb, t, n_states)
    lo, hi = orb.gap_range()
    w = laplace_weights(t, lo, hi)
    return Workload(name, basis, D, dict(t=t, w=w, orbitals=orb, amplitudes=Ts))


def config1() -> Workload:
    """~312 AO (18 heavy 3s2p1d, 12 light 2s1p), 8 nodes x 2 states."""
    return laplace_workload("medium-312ao", 1000, 30, 18, 40, 8, 2)


def config2() -> Workload:
    """~620 AO (40 heavy, 12 light), 10 nodes x 4 states."""
    return laplace_workload("large-620ao", 2000, 52, 40, 40, 10, 4)


def config3(n_mol: int = 64) -> list[Workload]:
    """64 uneven molecules: atoms U{3..40}, heavy fraction U[0.4, 0.8],
    1..32 densities each."""
    out = []
    for i in range(n_mol):
        rng = np.random.Generator(np.random.PCG64(3000 + i))
        n_atoms = int(rng.integers(3, 41))
        frac = rng.uniform(0.4, 0.8)
        n_heavy = max(1, int(round(frac * n_atoms)))
        nd = int(rng.integers(1, 33))
        basis = make_basis(rng, n_atoms, n_heavy)
        n_occ = max(1, min(40, basis.nbf() // 8))
        orb = random_orbitals(rng, basis, n_occ)
        t = laplace_nodes(8)
        n_states = (nd + 7) // 8
        D, _ = laplace_densities(rng, orb, t, n_states)
        out.append(Workload(f"batch-{i}", basis, D[:nd], dict(t=t, orbitals=orb)))
    return out


def config4_molecules(n_mol: int = 16, lo_ao: float = 50, hi_ao: float = 730) -> list[Workload]:
    """16 resident molecules with AO counts log-spaced over 50..730
    (heavy fraction 0.6); each carries orbitals to draw request densities."""
    out = []
    targets = np.exp(np.linspace(np.log(lo_ao), np.log(hi_ao), n_mol))
    for i, tgt in enumerate(targets):
        rng = np.random.Generator(np.random.PCG64(4000 + i))
        n_atoms = max(2, int(round(tgt / 10.4)))
        n_heavy = max(1, int(round(0.6 * n_atoms)))
        basis = make_basis(rng, n_atoms, n_heavy)
        n_occ = max(1, min(40, basis.nbf() // 8))
        orb = random_orbitals(rng, basis, n_occ)
        out.append(Workload(f"served-{i}", basis, np.zeros((0, basis.nbf(), basis.nbf())),
                            dict(orbitals=orb, t=laplace_nodes(8))))
    return out


def request_stream(n_req: int, rate_hz: float, n_mol: int = 16, seed: int = 4_000_000):
    """Poisson arrivals; each request names a molecule and a density count
    nd = floor(exp(U[0, ln 65))) in [1, 64]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_hz, size=n_req)
    t = np.cumsum(gaps)
    mol = rng.integers(0, n_mol, size=n_req)
    nd = np.floor(np.exp(rng.uniform(0.0, np.log(65.0), size=n_req))).astype(int)
    nd = np.clip(nd, 1, 64)
    return [dict(index=i, arrival=float(t[i]), mol=int(mol[i]), nd=int(nd[i]),
                 seed=seed + i) for i in range(n_req)]


def request_densities(orb: Orbitals, nd: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    t = laplace_nodes(8)
    n_states = (nd + 7) // 8
    D, _ = laplace_densities(rng, orb, t, n_states)
    return D[:nd]


def random_basis(seed: int, n_atoms: int, n_heavy: int, spherical: int = 1,
                 heavy=HEAVY_SPD, light=LIGHT, nprims=(NPRIM,)) -> Basis:
    """A small seeded basis for tests (same recipe as the workloads; nprims
    cycles the contraction lengths over the shells)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return make_basis(rng, n_atoms, n_heavy, heavy=heavy, light=light, spherical=spherical, nprims=nprims)


def random_densities(seed: int, nd: int, n: int, scale: float = 0.1,
                     symmetric: bool = False) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    D = rng.normal(size=(nd, n, n)) * scale
    if symmetric:
        D = 0.5 * (D + D.transpose(0, 2, 1))
    return D


def random_factors(seed: int, nd: int, n: int, r: int, scale: float = 0.3):
    """Seeded left and right factors U, V [nd][n][r] of densities D = U V^T
    (transition-density-like: rank r, not symmetric)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    U = rng.normal(size=(nd, n, r)) * scale
    V = rng.normal(size=(nd, n, r)) * scale
    return U, V


def random_symmetric_stack(seed: int, nvec: int, n: int, scale: float = 0.2) -> np.ndarray:
    """Seeded symmetric matrices [nvec][n][n] (stand-ins for a factor's rows)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    B = rng.normal(size=(nvec, n, n)) * scale
    return 0.5 * (B + B.transpose(0, 2, 1))
