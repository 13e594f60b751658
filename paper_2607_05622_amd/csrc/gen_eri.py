"""Generate straight-line HIP for the Head-Gordon-Pople / Obara-Saika ERI
recurrence of every canonical s/p/d shell-quartet class, and count its flops.

The recurrence family is the one the paper's kernels use (Sect. 3,
"DAG-driven, spill-bounded GPU chunking": a vertical-recurrence tower feeding
horizontal raises, VRR-A -> VRR-C -> HRR-AB -> HRR-CD).  Per primitive
quartet the vertical recurrence builds [e0|f0]^(m) from the Boys values
[00|00]^(m) = pref * F_m(T):

  VRR-A  [e+1_i,0|00]^(m) = PA_i [e|0]^(m) + WP_i [e|0]^(m+1)
                            + e_i/(2p) ([e-1_i|0]^(m) - rho/p [e-1_i|0]^(m+1))
  VRR-C  [e|f+1_i]^(m)    = QC_i [e|f]^(m) + WQ_i [e|f]^(m+1)
                            + f_i/(2q) ([e|f-1_i]^(m) - rho/q [e|f-1_i]^(m+1))
                            + e_i/(2(p+q)) [e-1_i|f]^(m+1)

The targets [e|f]^(0), la <= |e| <= la+lb and lc <= |f| <= lc+ld, are summed
over primitive quartets; the horizontal recurrences then act on contracted
values:

  HRR-AB (a, b+1_i| = (a+1_i, b| + AB_i (a, b|
  HRR-CD |c, d+1_i) = |c+1_i, d) + CD_i |c, d)

Each class is emitted as a DAG with dead nodes removed (only what the final
Cartesian tile needs).  The same walk yields the algorithmic flop count per
shell quartet used for every roofline figure: an FMA counts 2, a multiply or
add 1.

Usage: python gen_eri.py OUT.inc [--counts COUNTS.json]
"""
from __future__ import annotations

import json
import sys
from functools import lru_cache

LMAX = 2


def cart(l):
    return [(x, y, l - x - y) for x in range(l, -1, -1) for y in range(l - x, -1, -1)]


# lexicographic order xx, xy, xz, yy, yz, zz (matches the rest of the library)
def cart_lex(l):
    out = []
    for x in range(l, -1, -1):
        for y in range(l - x, -1, -1):
            out.append((x, y, l - x - y))
    return out


def classes():
    """Canonical classes (la lb | lc ld): la >= lb, lc >= ld, bra pair class
    index >= ket pair class index, pair class index = la(la+1)/2 + lb."""
    out = []
    for la in range(LMAX + 1):
        for lb in range(la + 1):
            for lc in range(LMAX + 1):
                for ld in range(lc + 1):
                    if la * (la + 1) // 2 + lb >= lc * (lc + 1) // 2 + ld:
                        out.append((la, lb, lc, ld))
    return out


def add(v, i, d=1):
    w = list(v)
    w[i] += d
    return tuple(w)


def pick_dir(v):
    """Direction to lower: the largest component (ties -> x, y, z)."""
    m = max(v)
    return v.index(m)


class Emitter:
    def __init__(self, la, lb, lc, ld):
        self.la, self.lb, self.lc, self.ld = la, lb, lc, ld
        self.L = la + lb + lc + ld
        self.lines = []
        self.flops = 0
        self.names = {}

    # ---------------- VRR -------------
    def vrr_deps(self, node):
        e, f, m = node
        if sum(f) > 0:
            i = pick_dir(f)
            f1 = add(f, i, -1)
            deps = [(e, f1, m), (e, f1, m + 1)]
            if f1[i] > 0:
                f2 = add(f1, i, -1)
                deps += [(e, f2, m), (e, f2, m + 1)]
            if e[i] > 0:
                deps += [(add(e, i, -1), f1, m + 1)]
            return deps
        if sum(e) > 0:
            i = pick_dir(e)
            e1 = add(e, i, -1)
            deps = [(e1, f, m), (e1, f, m + 1)]
            if e1[i] > 0:
                e2 = add(e1, i, -1)
                deps += [(e2, f, m), (e2, f, m + 1)]
            return deps
        return []

    def vrr_nodes(self, targets):
        need = set()
        stack = list(targets)
        while stack:
            n = stack.pop()
            if n in need:
                continue
            need.add(n)
            stack.extend(self.vrr_deps(n))
        # topological order: by total angular momentum, then by m descending
        return sorted(need, key=lambda n: (sum(n[0]) + sum(n[1]), sum(n[1]), -n[2], n))

    def vname(self, n):
        e, f, m = n
        return "v_%d%d%d_%d%d%d_%d" % (e + f + (m,))

    def emit_vrr(self, targets):
        """Emit the per-primitive VRR; returns the target variable names."""
        order = self.vrr_nodes(targets)
        out = []
        flops = 0
        for n in order:
            e, f, m = n
            nm = self.vname(n)
            if sum(e) == 0 and sum(f) == 0:
                out.append("const R %s = F[%d];" % (nm, m))
                continue
            X = "xyz"
            if sum(f) > 0:
                i = pick_dir(f)
                f1 = add(f, i, -1)
                terms = ["QC%s * %s" % (X[i], self.vname((e, f1, m))),
                         "WQ%s * %s" % (X[i], self.vname((e, f1, m + 1)))]
                flops += 3  # mul + fma
                if f1[i] > 0:
                    f2 = add(f1, i, -1)
                    k = f1[i]
                    terms.append("o2q_%d * (%s - rq * %s)" % (k, self.vname((e, f2, m)), self.vname((e, f2, m + 1))))
                    flops += 4  # fma + fma
                if e[i] > 0:
                    terms.append("o2pq_%d * %s" % (e[i], self.vname((add(e, i, -1), f1, m + 1))))
                    flops += 2
            else:
                i = pick_dir(e)
                e1 = add(e, i, -1)
                terms = ["PA%s * %s" % (X[i], self.vname((e1, f, m))),
                         "WP%s * %s" % (X[i], self.vname((e1, f, m + 1)))]
                flops += 3
                if e1[i] > 0:
                    e2 = add(e1, i, -1)
                    k = e1[i]
                    terms.append("o2p_%d * (%s - rp * %s)" % (k, self.vname((e2, f, m)), self.vname((e2, f, m + 1))))
                    flops += 4
            out.append("const R %s = %s;" % (nm, " + ".join(terms)))
        return out, flops, len(order)

    # ---------------- HRR -------------
    def hrr_plan(self):
        la, lb, lc, ld = self.la, self.lb, self.lc, self.ld
        finals = [(a, b, c, d) for a in cart_lex(la) for b in cart_lex(lb)
                  for c in cart_lex(lc) for d in cart_lex(ld)]
        need = {}
        order = []

        def visit(node):
            if node in need:
                return
            a, b, c, d = node
            if sum(b) > 0:
                i = pick_dir(b)
                deps = [(add(a, i), add(b, i, -1), c, d), (a, add(b, i, -1), c, d)]
                kind = ("AB", i)
            elif sum(d) > 0:
                i = pick_dir(d)
                deps = [(a, b, add(c, i), add(d, i, -1)), (a, b, c, add(d, i, -1))]
                kind = ("CD", i)
            else:
                deps = []
                kind = ("ACC", None)
            for dp in deps:
                visit(dp)
            need[node] = (kind, deps)
            order.append(node)

        for fn in finals:
            visit(fn)
        return finals, order, need

    def hname(self, n):
        a, b, c, d = n
        return "h_%d%d%d_%d%d%d_%d%d%d_%d%d%d" % (a + b + c + d)

    def generate(self):
        la, lb, lc, ld = self.la, self.lb, self.lc, self.ld
        finals, order, need = self.hrr_plan()
        # contracted VRR targets = HRR leaves
        leaves = sorted({(n[0], n[2]) for n in order if need[n][0][0] == "ACC"})
        targets = [(e, f, 0) for (e, f) in leaves]
        vrr_code, vrr_flops, vrr_nodes = self.emit_vrr(targets)
        # HRR code
        hrr_code = []
        hrr_flops = 0
        X = "xyz"
        leaf_index = {lf: i for i, lf in enumerate(leaves)}
        for n in order:
            kind, deps = need[n]
            if kind[0] == "ACC":
                hrr_code.append("const R %s = acc[%d];" % (self.hname(n), leaf_index[(n[0], n[2])]))
            else:
                vec = "AB" if kind[0] == "AB" else "CD"
                hrr_code.append("const R %s = %s + %s%s * %s;" % (
                    self.hname(n), self.hname(deps[0]), vec, X[kind[1]], self.hname(deps[1])))
                hrr_flops += 2
        outputs = [self.hname(f) for f in finals]
        return dict(
            cls=(la, lb, lc, ld), L=self.L, nacc=len(leaves),
            leaves=leaves, vrr_code=vrr_code, hrr_code=hrr_code, outputs=outputs,
            vrr_flops=vrr_flops, vrr_nodes=vrr_nodes, hrr_flops=hrr_flops,
            nfunc=len(finals),
        )


# Classes with more contracted targets than SPLIT_NACC are evaluated in
# passes over groups of bra components e (about TARGET_BUDGET accumulators
# per group), so that no pass keeps more than a few dozen accumulators live:
# each pass runs the primitive loop over its own recurrence cone, applies
# HRR-CD to its e's and stores (e0|cd) to scratch; HRR-AB then assembles the
# tile one ket function pair at a time.
SPLIT_NACC = 40
TARGET_BUDGET = 32
# per-class budgets where timing on MI355X preferred fewer, larger passes
# (fewer repeats of the primitive set-up and Boys evaluation)
CLASS_BUDGET = {(1, 1, 1, 1): 96, (2, 0, 1, 1): 64, (2, 1, 1, 0): 64, (2, 1, 1, 1): 96, (2, 2, 1, 0): 96,
                (2, 2, 1, 1): 64, (2, 2, 2, 0): 64, (2, 2, 2, 1): 64, (2, 2, 2, 2): 64}


def split_plan(em, info):
    """Groups of e (in the sorted e order) and the derived index sets."""
    leaves = info["leaves"]
    es = sorted({e for e, f in leaves}, key=lambda e: (sum(e), e))
    fs = sorted({f for e, f in leaves}, key=lambda f: (sum(f), f))
    budget = CLASS_BUDGET.get((em.la, em.lb, em.lc, em.ld), TARGET_BUDGET)
    per = max(1, budget // len(fs))
    groups = [es[i:i + per] for i in range(0, len(es), per)]
    return es, fs, groups


def emit_split(em, info, R="R"):
    """Code for the split evaluation of one class: per-group VRR and HRR-CD,
    and the HRR-AB applied per ket function pair."""
    la, lb, lc, ld = em.la, em.lb, em.lc, em.ld
    es, fs, groups = split_plan(em, info)
    eidx = {e: i for i, e in enumerate(es)}
    fidx = {f: i for i, f in enumerate(fs)}
    cds = [(c, d) for c in cart_lex(lc) for d in cart_lex(ld)]
    abs_ = [(a, b) for a in cart_lex(la) for b in cart_lex(lb)]
    X = "xyz"
    out = {"groups": [], "NE": len(es), "NCD": len(cds), "NAB": len(abs_), "NFT": len(fs)}
    vrr_flops_total = 0
    hrr_flops = 0
    for gi, grp in enumerate(groups):
        targets = [(e, f, 0) for e in grp for f in fs]
        code, fl, nn = em.emit_vrr(targets)
        vrr_flops_total += fl
        acc_lines = ["acc[%d] += %s;" % (i, em.vname(t)) for i, t in enumerate(targets)]
        # HRR-CD on this group's e's: (e|c, d+1_i) = (e|c+1_i, d) + CD_i (e|c, d)
        hc = []
        memo = {}

        def node(e, c, d):
            key = (e, c, d)
            if key in memo:
                return memo[key]
            if sum(d) == 0:
                nm = "acc[%d]" % (grp.index(e) * len(fs) + fidx[c])
                memo[key] = nm
                return nm
            i = pick_dir(d)
            n1 = node(e, add(c, i), add(d, i, -1))
            n2 = node(e, c, add(d, i, -1))
            nm = "u_%d%d%d_%d%d%d_%d%d%d" % (e + c + d)
            hc.append("const R %s = %s + CD%s * %s;" % (nm, n1, X[i], n2))
            memo[key] = nm
            return nm
        sinks = []
        for e in grp:
            for ci, (c, d) in enumerate(cds):
                nm = node(e, c, d)
                sinks.append("sink(%d, %s);" % (eidx[e] * len(cds) + ci, nm))
        hrr_flops += 2 * len(hc)
        out["groups"].append(dict(n=len(targets), vrr=code, acc=acc_lines, hrrcd=hc, sinks=sinks))
    # HRR-AB: (a, b+1_i| = (a+1_i, b| + AB_i (a, b|, leaves (e, 0|
    memo = {}
    hab = []
    loads = []

    def nodeab(a, b):
        key = (a, b)
        if key in memo:
            return memo[key]
        if sum(b) == 0:
            nm = "w_%d%d%d" % a
            loads.append("const R %s = load(%d);" % (nm, eidx[a]))
            memo[key] = nm
            return nm
        i = pick_dir(b)
        n1 = nodeab(add(a, i), add(b, i, -1))
        n2 = nodeab(a, add(b, i, -1))
        nm = "v_%d%d%d_%d%d%d" % (a + b)
        hab.append("const R %s = %s + AB%s * %s;" % (nm, n1, X[i], n2))
        memo[key] = nm
        return nm
    ab_sinks = []
    for ai, (a, b) in enumerate(abs_):
        ab_sinks.append("sink(%d, %s);" % (ai, nodeab(a, b)))
    hrr_flops += 2 * len(hab) * len(cds)
    out["hab"] = loads + hab
    out["ab_sinks"] = ab_sinks
    out["vrr_flops_total"] = vrr_flops_total
    out["hrr_flops"] = hrr_flops
    return out


# Per-primitive-quartet set-up and Boys cost (flops), counted from the kernel
# source: the quartet geometry (~34), the prefactor (3), Taylor + exp +
# downward recursion of the Boys function (2*7 + 2*8 + 3L), folding the
# prefactor into F (L+1), and the contraction adds (one per target).
def prim_setup_flops(L, nacc):
    return 34 + 3 + (14 + 16 + 3 * L) + (L + 1) + nacc


def class_tag(c):
    return "%d%d%d%d" % c


def emit_all(path, counts_path=None):
    infos = []
    src = []
    src.append("// Generated by gen_eri.py -- do not edit.\n")
    src.append("// Straight-line HGP-OS recurrences for the 21 canonical s/p/d classes.\n")
    for c in classes():
        em = Emitter(*c)
        info = em.generate()
        infos.append(info)
        tag = class_tag(c)
        la, lb, lc, ld = c
        L = info["L"]
        src.append("template <typename R> struct Eri%s {" % tag)
        src.append("  static constexpr int L = %d, NACC = %d, NF = %d;" % (L, info["nacc"], info["nfunc"]))
        src.append("  template <typename T> using With = Eri%s<T>;   // the same class in precision T" % tag)
        src.append("  static constexpr int LA = %d, LB = %d, LC = %d, LD = %d;" % c)
        # VRR: needs F[0..L], PA, WP, QC, WQ, o2p_k, o2q_k, o2pq_k, rp, rq
        src.append("  // vertical recurrence in precision R, contracted into accumulators of type A")
        src.append("  template <typename A>")
        src.append("  __device__ static __forceinline__ void vrr(const R* __restrict__ F, const VrrCoef<R>& k, A* __restrict__ acc) {")
        src.append("    const R PAx = k.PA[0], PAy = k.PA[1], PAz = k.PA[2];")
        src.append("    const R WPx = k.WP[0], WPy = k.WP[1], WPz = k.WP[2];")
        src.append("    const R QCx = k.QC[0], QCy = k.QC[1], QCz = k.QC[2];")
        src.append("    const R WQx = k.WQ[0], WQy = k.WQ[1], WQz = k.WQ[2];")
        src.append("    const R rp = k.rp, rq = k.rq;")
        src.append("    const R o2p_1 = k.o2p, o2p_2 = R(2) * k.o2p, o2p_3 = R(3) * k.o2p;")
        src.append("    const R o2q_1 = k.o2q, o2q_2 = R(2) * k.o2q, o2q_3 = R(3) * k.o2q;")
        src.append("    const R o2pq_1 = k.o2pq, o2pq_2 = R(2) * k.o2pq, o2pq_3 = R(3) * k.o2pq, o2pq_4 = R(4) * k.o2pq;")
        src.append("    (void)PAx; (void)PAy; (void)PAz; (void)WPx; (void)WPy; (void)WPz;")
        src.append("    (void)QCx; (void)QCy; (void)QCz; (void)WQx; (void)WQy; (void)WQz; (void)rp; (void)rq;")
        src.append("    (void)o2p_1; (void)o2p_2; (void)o2p_3; (void)o2q_1; (void)o2q_2; (void)o2q_3;")
        src.append("    (void)o2pq_1; (void)o2pq_2; (void)o2pq_3; (void)o2pq_4;")
        for line in info["vrr_code"]:
            src.append("    " + line)
        vnames = [Emitter(*c).vname((e, f, 0)) for (e, f) in info["leaves"]]
        for i, v in enumerate(vnames):
            src.append("    acc[%d] += %s;" % (i, v))
        src.append("  }")
        # HRR: acc -> out via a functor sink(index, value)
        split = info["nacc"] > SPLIT_NACC
        src.append("  static constexpr bool kSplit = %s;" % ("true" if split else "false"))
        if split:
            sp = emit_split(em, info)
            info["split"] = sp
            gn = [g["n"] for g in sp["groups"]]
            src.append("  static constexpr int NE = %d, NCD = %d, NAB = %d, NG = %d, GMAX = %d;" % (
                sp["NE"], sp["NCD"], sp["NAB"], len(gn), max(gn)))
            src.append("  template <int G, typename A> __device__ static __forceinline__ void vrr_group(const R* __restrict__ F, const VrrCoef<R>& k, A* __restrict__ acc) {")
            src.append("    const R PAx = k.PA[0], PAy = k.PA[1], PAz = k.PA[2];")
            src.append("    const R WPx = k.WP[0], WPy = k.WP[1], WPz = k.WP[2];")
            src.append("    const R QCx = k.QC[0], QCy = k.QC[1], QCz = k.QC[2];")
            src.append("    const R WQx = k.WQ[0], WQy = k.WQ[1], WQz = k.WQ[2];")
            src.append("    const R rp = k.rp, rq = k.rq;")
            src.append("    const R o2p_1 = k.o2p, o2p_2 = R(2) * k.o2p, o2p_3 = R(3) * k.o2p;")
            src.append("    const R o2q_1 = k.o2q, o2q_2 = R(2) * k.o2q, o2q_3 = R(3) * k.o2q;")
            src.append("    const R o2pq_1 = k.o2pq, o2pq_2 = R(2) * k.o2pq, o2pq_3 = R(3) * k.o2pq, o2pq_4 = R(4) * k.o2pq;")
            src.append("    (void)PAx; (void)PAy; (void)PAz; (void)WPx; (void)WPy; (void)WPz;")
            src.append("    (void)QCx; (void)QCy; (void)QCz; (void)WQx; (void)WQy; (void)WQz; (void)rp; (void)rq;")
            src.append("    (void)o2p_1; (void)o2p_2; (void)o2p_3; (void)o2q_1; (void)o2q_2; (void)o2q_3;")
            src.append("    (void)o2pq_1; (void)o2pq_2; (void)o2pq_3; (void)o2pq_4;")
            for gi, g in enumerate(sp["groups"]):
                src.append("    %sif constexpr (G == %d) {" % ("" if gi == 0 else "else ", gi))
                for line in g["vrr"] + g["acc"]:
                    src.append("      " + line)
                src.append("    }")
            src.append("  }")
            src.append("  template <int G, class Sink>")
            src.append("  __device__ static __forceinline__ void hrrcd_group(const R* __restrict__ acc, const R CD[3], Sink&& sink) {")
            src.append("    const R CDx = CD[0], CDy = CD[1], CDz = CD[2];")
            src.append("    (void)CDx; (void)CDy; (void)CDz;")
            for gi, g in enumerate(sp["groups"]):
                src.append("    %sif constexpr (G == %d) {" % ("" if gi == 0 else "else ", gi))
                for line in g["hrrcd"] + g["sinks"]:
                    src.append("      " + line)
                src.append("    }")
            src.append("  }")
            src.append("  template <class Load, class Sink>")
            src.append("  __device__ static __forceinline__ void hrrab(Load&& load, const R AB[3], Sink&& sink) {")
            src.append("    const R ABx = AB[0], ABy = AB[1], ABz = AB[2];")
            src.append("    (void)ABx; (void)ABy; (void)ABz;")
            for line in sp["hab"] + sp["ab_sinks"]:
                src.append("    " + line)
            src.append("  }")
            src.append("  static constexpr int GN[NG] = {%s};" % ", ".join(str(x) for x in gn))
        src.append("  template <class Sink>")
        src.append("  __device__ static __forceinline__ void hrr(const R* __restrict__ acc, const R AB[3], const R CD[3], Sink&& sink) {")
        src.append("    const R ABx = AB[0], ABy = AB[1], ABz = AB[2];")
        src.append("    const R CDx = CD[0], CDy = CD[1], CDz = CD[2];")
        src.append("    (void)ABx; (void)ABy; (void)ABz; (void)CDx; (void)CDy; (void)CDz;")
        for line in info["hrr_code"]:
            src.append("    " + line)
        for i, o in enumerate(info["outputs"]):
            src.append("    sink(%d, %s);" % (i, o))
        src.append("  }")
        src.append("};\n")
    # dispatch list: X(class index, tag, la, lb, lc, ld)
    ent = []
    for c in classes():
        la, lb, lc, ld = c
        X = la * (la + 1) // 2 + lb
        Y = lc * (lc + 1) // 2 + ld
        ent.append("X(%d, %s, %d, %d, %d, %d)" % (X * (X + 1) // 2 + Y, class_tag(c), la, lb, lc, ld))
    src.append("#define JK_CLASS_LIST(X) \\\n  " + " \\\n  ".join(ent) + "\n")
    with open(path, "w") as fh:
        fh.write("\n".join(src))
    counts = {}
    for info in infos:
        L = info["L"]
        sp = info.get("split")
        counts[class_tag(info["cls"])] = dict(
            L=L, nfunc=info["nfunc"], nacc=info["nacc"], vrr_nodes=info["vrr_nodes"],
            vrr_flops=info["vrr_flops"], hrr_flops=info["hrr_flops"],
            prim_flops=prim_setup_flops(L, info["nacc"]),
            split_groups=len(sp["groups"]) if sp else 1,
            split_vrr_flops=sp["vrr_flops_total"] if sp else info["vrr_flops"],
            split_hrr_flops=sp["hrr_flops"] if sp else info["hrr_flops"])
    if counts_path:
        with open(counts_path, "w") as fh:
            json.dump(counts, fh, indent=1, sort_keys=True)
    return counts


def emit_cost(path, counts):
    """C++ table kClassCost[class index] of the per-class flop counts."""
    lines = ["// Generated by gen_eri.py -- do not edit.",
             "// Algorithmic flops of the HGP-OS path per class: per primitive quartet",
             "// (set-up + Boys + contraction, and vertical recurrence) and per",
             "// contracted quartet (horizontal recurrences); FMA = 2 flops.",
             "struct ClassCost { int nfunc, nacc, prim_flops, vrr_flops, hrr_flops; };",
             "constexpr ClassCost kClassCost[21] = {"]
    rows = {}
    for c in classes():
        la, lb, lc, ld = c
        X = la * (la + 1) // 2 + lb
        Y = lc * (lc + 1) // 2 + ld
        k = counts[class_tag(c)]
        rows[X * (X + 1) // 2 + Y] = "    {%d, %d, %d, %d, %d},  // (%d%d|%d%d)" % (
            k["nfunc"], k["nacc"], k["prim_flops"], k["vrr_flops"], k["hrr_flops"], la, lb, lc, ld)
    lines += [rows[i] for i in range(21)]
    lines.append("};\n")
    with open(path, "w") as fh:
        fh.write("\n".join(lines))


def flops_per_quartet(counts, tag, nprim_bra, nprim_ket):
    c = counts[tag]
    npq = nprim_bra * nprim_ket
    return npq * (c["prim_flops"] + c["vrr_flops"]) + c["hrr_flops"]


if __name__ == "__main__":
    out = sys.argv[1]
    cp = None
    if "--counts" in sys.argv:
        cp = sys.argv[sys.argv.index("--counts") + 1]
    counts = emit_all(out, cp)
    if "--cost" in sys.argv:
        emit_cost(sys.argv[sys.argv.index("--cost") + 1], counts)
    for k, v in sorted(counts.items()):
        print(k, v, "flops/quartet(9x9 prims)=", flops_per_quartet(counts, k, 9, 9))
