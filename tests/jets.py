"""Truncated multivariate Taylor polynomials ("jets") for pinning integrals.

A Cartesian Gaussian with powers up to 2 is a derivative of an s Gaussian
with respect to its centre:

    x_A   e^{-a r_A^2} = (1/2a)            d/dA_x        e^{-a r_A^2}
    x_A^2 e^{-a r_A^2} = (1/4a^2) (d^2/dA_x^2 + 2a)     e^{-a r_A^2}

so every s/p/d primitive two-electron integral is a combination of centre
derivatives of the closed-form (ss|ss) integral

    (ss|ss) = 2 pi^{5/2} / (p q sqrt(p+q)) exp(-ab/p |AB|^2)
              exp(-cd/q |CD|^2) F_0(rho |PQ|^2),

with dF_m/dT = -F_{m+1}.  This module evaluates those derivatives exactly
(up to rounding) by propagating Taylor coefficients, so the check shares
nothing with either recurrence family under test.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy.special import hyp1f1


def boys_ref(m: int, T: float) -> float:
    """F_m(T) = 1F1(m+1/2; m+3/2; -T) / (2m+1) (scipy)."""
    return float(hyp1f1(m + 0.5, m + 1.5, -T) / (2 * m + 1))


class Jet:
    """Polynomial in nv variables, coefficient array c[k1,...,knv] for
    prod d_i^{k_i}, truncated at per-variable orders ``orders``."""

    def __init__(self, c: np.ndarray):
        self.c = c

    @staticmethod
    def const(v, orders):
        c = np.zeros(tuple(o + 1 for o in orders))
        c[(0,) * len(orders)] = v
        return Jet(c)

    @staticmethod
    def var(v, i, orders):
        j = Jet.const(v, orders)
        if orders[i] >= 1:
            idx = [0] * len(orders)
            idx[i] = 1
            j.c[tuple(idx)] = 1.0
        return j

    @property
    def value(self):
        return float(self.c.flat[0])

    def _coerce(self, o):
        return o if isinstance(o, Jet) else Jet.const(float(o), [s - 1 for s in self.c.shape])

    def __add__(self, o):
        o = self._coerce(o)
        return Jet(self.c + o.c)

    __radd__ = __add__

    def __neg__(self):
        return Jet(-self.c)

    def __sub__(self, o):
        return self + (-self._coerce(o))

    def __rsub__(self, o):
        return self._coerce(o) - self

    def __mul__(self, o):
        if not isinstance(o, Jet):
            return Jet(self.c * float(o))
        a, b = self.c, o.c
        out = np.zeros_like(a)
        shape = a.shape
        for idx in zip(*np.nonzero(a)):
            src = tuple(slice(0, s - i) for s, i in zip(shape, idx))
            dst = tuple(slice(i, s) for s, i in zip(shape, idx))
            out[dst] += a[idx] * b[src]
        return Jet(out)

    __rmul__ = __mul__

    def total_order(self):
        return sum(s - 1 for s in self.c.shape)

    def compose(self, derivs):
        """f(self) given derivs[k] = f^{(k)}(value), k = 0..total order."""
        u0 = self.value
        du = self - u0
        res = Jet.const(derivs[0], [s - 1 for s in self.c.shape])
        p = Jet.const(1.0, [s - 1 for s in self.c.shape])
        for k in range(1, self.total_order() + 1):
            p = p * du
            res = res + p * (derivs[k] / math.factorial(k))
        return res

    def exp(self):
        e = math.exp(self.value)
        return self.compose([e] * (self.total_order() + 1))

    def boys0(self):
        T = self.value
        n = self.total_order()
        return self.compose([(-1) ** k * boys_ref(k, T) for k in range(n + 1)])

    def deriv(self, ks):
        """d^{k1..kn} f at the expansion point."""
        return float(self.c[tuple(ks)]) * math.prod(math.factorial(k) for k in ks)


def prim_norm(a: float, l: int) -> float:
    df = 1.0
    for n in range(2 * l - 1, 0, -2):
        df *= n
    return math.sqrt((2 * a / math.pi) ** 1.5 * (4 * a) ** l / df)


def primitive_eri(centres, exps, powers) -> float:
    """Unnormalized primitive integral (g_A g_B | g_C g_D) with Cartesian
    powers ``powers[i] = (lx, ly, lz)`` via derivatives of (ss|ss)."""
    # one jet variable per (centre, axis) with a non-zero power
    vars_ = [(i, ax) for i in range(4) for ax in range(3) if powers[i][ax] > 0]
    orders = [powers[i][ax] for i, ax in vars_]
    if not vars_:
        orders = [0]
    X = [[None] * 3 for _ in range(4)]
    for i in range(4):
        for ax in range(3):
            if (i, ax) in vars_:
                X[i][ax] = Jet.var(float(centres[i][ax]), vars_.index((i, ax)), orders)
            else:
                X[i][ax] = Jet.const(float(centres[i][ax]), orders)
    a, b, c, d = exps
    p, q = a + b, c + d
    rho = p * q / (p + q)
    ab2 = sum((X[0][k] - X[1][k]) * (X[0][k] - X[1][k]) for k in range(3))
    cd2 = sum((X[2][k] - X[3][k]) * (X[2][k] - X[3][k]) for k in range(3))
    P = [(X[0][k] * a + X[1][k] * b) * (1.0 / p) for k in range(3)]
    Q = [(X[2][k] * c + X[3][k] * d) * (1.0 / q) for k in range(3)]
    pq2 = sum((P[k] - Q[k]) * (P[k] - Q[k]) for k in range(3))
    f = (ab2 * (-a * b / p)).exp() * (cd2 * (-c * d / q)).exp() * (pq2 * rho).boys0()
    f = f * (2 * math.pi ** 2.5 / (p * q * math.sqrt(p + q)))
    # apply the derivative operators
    total = 0.0
    choices = []
    for (i, ax) in vars_:
        n = powers[i][ax]
        al = exps[i]
        if n == 1:
            choices.append([(1, 1.0 / (2 * al))])
        else:  # n == 2: (d^2 + 2a) / 4a^2
            choices.append([(2, 1.0 / (4 * al * al)), (0, 2 * al / (4 * al * al))])
    if not vars_:
        return f.value
    for combo in itertools.product(*choices):
        ks = [k for k, _ in combo]
        w = math.prod(wt for _, wt in combo)
        total += w * f.deriv(ks)
    return total
