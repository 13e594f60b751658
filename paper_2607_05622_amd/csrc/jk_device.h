// Device-side building blocks of the J/K build: FP64 Boys function,
// primitive-quartet set-up, the screening decision, and the per-class ERI tile
// kernel (instantiated once per class in jk_class.hip; digestion is in
// jk_digest.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "jk_internal.h"
#include "jk_launch.h"

namespace jk {

#include "eri_gen.inc"

// Pointers into device memory reached through descriptors are generic to
// the compiler; naming them global makes their accesses global (not flat)
// instructions, whose completion is counted apart from LDS and scalar
// traffic, so loads stay in flight across other work.
template <typename T>
using gptr = T __attribute__((address_space(1)))*;
template <typename T>
__device__ __forceinline__ gptr<T> glob(T* p) {
    return (gptr<T>)p;
}

// The descriptor of molecule i of a batch (or mol0 for a single build),
// copied into registers.  Read through a reference, its fields would be
// reloaded after every store or atomic the kernel issues (the compiler
// cannot rule out that they alias it), and each reload waits for those to
// complete.
__device__ __forceinline__ MolDesc load_mol(const MolDesc* mols, const MolDesc& mol0, int i) {
    if (!mols) return mol0;
    const gptr<const unsigned long long> w = (gptr<const unsigned long long>)(mols + i);
    const gptr<const int> n = (gptr<const int>)(w + 13);
    MolDesc m;
    m.pairs = reinterpret_cast<const PairInfo*>(w[0]);
    m.prims = reinterpret_cast<const double*>(w[1]);
    m.dmax = reinterpret_cast<const double*>(w[2]);
    m.D = reinterpret_cast<const double*>(w[3]);
    m.J = reinterpret_cast<double*>(w[4]);
    m.K = reinterpret_cast<double*>(w[5]);
    m.KT = reinterpret_cast<double*>(w[6]);
    m.DS = reinterpret_cast<const double*>(w[7]);
    m.ds_off = reinterpret_cast<const int*>(w[8]);
    m.Df = reinterpret_cast<const float*>(w[9]);
    m.DSf = reinterpret_cast<const float*>(w[10]);
    m.DT = reinterpret_cast<const double*>(w[11]);
    m.DTf = reinterpret_cast<const float*>(w[12]);
    m.ns = n[0];
    m.nc = n[1];
    m.nd = n[2];
    m.ndp = n[3];
    m.pslots = n[4];
    m.pad = 0;
    return m;
}

// ---------------------------------------------------------------- Boys ---

// 1/sqrt(x) for normal positive x: the hardware estimate (about 23 correct
// bits) refined by two Newton steps y <- y + y (1/2 - x y^2 / 2), each of
// which doubles the correct bits.
__device__ __forceinline__ double rsqrt_f64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = fma(y, fma(-h * y, y, 0.5), y);
    y = fma(y, fma(-h * y, y, 0.5), y);
    return y;
}


// F_m(T), m = 0..L, multiplied by pref.  T < kBoysTMax: seven-term Taylor
// expansion of F_L about the nearest grid point (dF_m/dT = -F_{m+1}), exp(-T)
// from the tabulated exp(-T0) and an eight-term series, then the downward
// recursion F_m = (2T F_{m+1} + e^{-T}) / (2m+1).  Beyond: the asymptotic
// form F_0 = sqrt(pi/T)/2, F_{m+1} = F_m (2m+1)/(2T); the dropped e^{-T}
// terms are below 2e-22.
template <int L>
__device__ __forceinline__ void boys_f64(double T, double pref, gptr<const double> tab, double* __restrict__ F) {
    constexpr double inv_odd[16] = {1.0,       1.0 / 3,  1.0 / 5,  1.0 / 7,  1.0 / 9,  1.0 / 11,
                                    1.0 / 13,  1.0 / 15, 1.0 / 17, 1.0 / 19, 1.0 / 21, 1.0 / 23,
                                    1.0 / 25,  1.0 / 27, 1.0 / 29, 1.0 / 31};
    if (T < kBoysTMax) {
        const int i = static_cast<int>(T * kBoysInvStep + 0.5);
        const double x = static_cast<double>(i) * (1.0 / kBoysInvStep) - T;   // -(T - T0)
        const gptr<const double> r = tab + i * kBoysCols;
        double f = r[L + 6];
        f = fma(f, x * (1.0 / 6), r[L + 5]);
        f = fma(f, x * (1.0 / 5), r[L + 4]);
        f = fma(f, x * 0.25, r[L + 3]);
        f = fma(f, x * (1.0 / 3), r[L + 2]);
        f = fma(f, x * 0.5, r[L + 1]);
        f = fma(f, x, r[L]);
        F[L] = f;
        if constexpr (L > 0) {
            double e = 1.0 / 5040;
            e = fma(e, x, 1.0 / 720);
            e = fma(e, x, 1.0 / 120);
            e = fma(e, x, 1.0 / 24);
            e = fma(e, x, 1.0 / 6);
            e = fma(e, x, 0.5);
            e = fma(e, x, 1.0);
            e = fma(e, x, 1.0);
            e *= r[kBoysCols - 1];
            const double t2 = T + T;
#pragma unroll
            for (int m = L - 1; m >= 0; --m) F[m] = fma(t2, F[m + 1], e) * inv_odd[m];
        }
    } else {
        const double rt = rsqrt_f64(T);
        double f = 0.88622692545275801365 * rt;   // sqrt(pi)/2 / sqrt(T)
        F[0] = f;
        const double h = 0.5 * rt * rt;
#pragma unroll
        for (int m = 0; m < L; ++m) {
            f *= static_cast<double>(2 * m + 1) * h;
            F[m + 1] = f;
        }
    }
#pragma unroll
    for (int m = 0; m <= L; ++m) F[m] *= pref;
}

// FP32 tier: F_m(T) in FP32 inside the table range (five-term Taylor
// expansion about the nearest grid point, exp(-T) likewise, downward
// recursion), the FP64 asymptotic form beyond it; the FP64 prefactor is
// applied in FP64 before rounding to FP32.
template <int L>
__device__ __forceinline__ void boys_f32(double T, double pref, gptr<const float> tab, float* __restrict__ F) {
    if (T < kBoysTMax) {
        const int i = static_cast<int>(T * kBoysInvStep + 0.5);
        const float x = static_cast<float>(static_cast<double>(i) * (1.0 / kBoysInvStep) - T);
        const gptr<const float> r = tab + i * kBoysCols;
        float f = r[L + 4];
        f = fmaf(f, x * 0.25f, r[L + 3]);
        f = fmaf(f, x * (1.0f / 3), r[L + 2]);
        f = fmaf(f, x * 0.5f, r[L + 1]);
        f = fmaf(f, x, r[L]);
        F[L] = f;
        if constexpr (L > 0) {
            float e = 1.0f / 120;
            e = fmaf(e, x, 1.0f / 24);
            e = fmaf(e, x, 1.0f / 6);
            e = fmaf(e, x, 0.5f);
            e = fmaf(e, x, 1.0f);
            e = fmaf(e, x, 1.0f);
            e *= r[kBoysCols - 1];
            const float t2 = static_cast<float>(T + T);
#pragma unroll
            for (int m = L - 1; m >= 0; --m) F[m] = fmaf(t2, F[m + 1], e) * (1.0f / static_cast<float>(2 * m + 1));
        }
#pragma unroll
        for (int m = 0; m <= L; ++m) F[m] = static_cast<float>(static_cast<double>(F[m]) * pref);
    } else {
        double Fd[L + 1];
        const double rt = rsqrt_f64(T);
        double f = 0.88622692545275801365 * rt;
        Fd[0] = f;
        const double h = 0.5 * rt * rt;
#pragma unroll
        for (int m = 0; m < L; ++m) {
            f *= static_cast<double>(2 * m + 1) * h;
            Fd[m + 1] = f;
        }
#pragma unroll
        for (int m = 0; m <= L; ++m) F[m] = static_cast<float>(Fd[m] * pref);
    }
}

// Boys values of the working precision R.
template <int L, typename R>
__device__ __forceinline__ void boys_r(double T, double pref, const EriTileArgs& a, R* F) {
    if constexpr (sizeof(R) == 8) boys_f64<L>(T, pref, glob(a.boys), F);
    else boys_f32<L>(T, pref, glob(a.boys32), F);
}

template <typename R>
__device__ __forceinline__ void coef_to(const VrrCoef<double>& k, VrrCoef<R>& o) {
    for (int i = 0; i < 3; ++i) {
        o.PA[i] = static_cast<R>(k.PA[i]);
        o.WP[i] = static_cast<R>(k.WP[i]);
        o.QC[i] = static_cast<R>(k.QC[i]);
        o.WQ[i] = static_cast<R>(k.WQ[i]);
    }
    o.rp = static_cast<R>(k.rp);
    o.rq = static_cast<R>(k.rq);
    o.o2p = static_cast<R>(k.o2p);
    o.o2q = static_cast<R>(k.o2q);
    o.o2pq = static_cast<R>(k.o2pq);
}

// Per-primitive-quartet quantities of the vertical recurrence.
__device__ __forceinline__ void prim_setup(const PrimPair& P, const PrimPair& Q, const double* A,
                                           const double* C, VrrCoef<double>& k, double& T,
                                           double& pref) {
    const double p = P.p, q = Q.p;
    const double rs = rsqrt_f64(p + q);
    const double ipq = rs * rs;
    const double rho = p * q * ipq;
    const double PQx = P.P[0] - Q.P[0], PQy = P.P[1] - Q.P[1], PQz = P.P[2] - Q.P[2];
    T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);
    pref = P.E * Q.E * rs;
    const double qf = q * ipq, pf = p * ipq;
    k.WP[0] = -qf * PQx;
    k.WP[1] = -qf * PQy;
    k.WP[2] = -qf * PQz;
    k.WQ[0] = pf * PQx;
    k.WQ[1] = pf * PQy;
    k.WQ[2] = pf * PQz;
    k.PA[0] = P.P[0] - A[0];
    k.PA[1] = P.P[1] - A[1];
    k.PA[2] = P.P[2] - A[2];
    k.QC[0] = Q.P[0] - C[0];
    k.QC[1] = Q.P[1] - C[1];
    k.QC[2] = Q.P[2] - C[2];
    k.rp = qf;
    k.rq = pf;
    k.o2p = P.o2p;
    k.o2q = Q.o2p;
    k.o2pq = 0.5 * ipq;
}

// Identical decision in every kernel: keep (ab|cd) iff Q_ab Q_cd >= tol and
// Q_ab Q_cd * max(Dmax over ab, cd, ac, ad, bc, bd) >= tol.
__device__ __forceinline__ bool keep_quartet(const PairInfo& P, const PairInfo& Q, const double* dmax_p, int ns,
                                             double tol) {
    const double qq = P.q * Q.q;
    if (qq < tol) return false;
    if (dmax_p == nullptr) return true;
    const gptr<const double> dmax = glob(dmax_p);
    const int a = P.sa, b = P.sb, c = Q.sa, d = Q.sb;
    double m = dmax[a * ns + b];
    m = fmax(m, dmax[c * ns + d]);
    m = fmax(m, dmax[a * ns + c]);
    m = fmax(m, dmax[a * ns + d]);
    m = fmax(m, dmax[b * ns + c]);
    m = fmax(m, dmax[b * ns + d]);
    return qq * m >= tol;
}

// ------------------------------------------------------------ ERI tile ---

// Block blk of a launch belongs to the last item whose first block is <= blk.
__device__ __forceinline__ int find_item(const EriItem* __restrict__ items, int n, long long blk) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].blk0 <= blk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The primitive-pair record in slot `slot` of the planes at pl (pslots
// entries each), in three 16-byte loads.
typedef double v2d __attribute__((ext_vector_type(2)));
__device__ __forceinline__ PrimPair load_prim(gptr<const v2d> pl, long long pslots, int slot) {
    const v2d a = pl[slot], b = pl[pslots + slot], c = pl[2 * pslots + slot];
    PrimPair r;
    r.p = a.x;
    r.E = a.y;
    r.P[0] = b.x;
    r.P[1] = b.y;
    r.P[2] = c.x;
    r.o2p = c.y;
    r.pad0 = r.pad1 = 0.0;
    return r;
}

// Calls body(bra primitive pair, ket primitive pair) for every primitive
// quartet, ket-major; a pair's records start in slot b0 (bra) or k0 (ket),
// kPrimLane apart.  The lanes of a wavefront hold different ket pairs of
// (mostly) one bra pair, so each ket record is loaded once per quartet and
// the bra records, at one address across the wavefront, inside.  (Loading
// the next quartet's records ahead of the body stopped paying once the ket
// records were laid out for coalesced loads.)
template <class Body>
__device__ __forceinline__ void prim_loop(const MolDesc& m, int b0, int nb, int k0, int nk, Body body) {
    const gptr<const v2d> pl = glob(reinterpret_cast<const v2d*>(m.prims));
    const long long ps = m.pslots;
#pragma unroll 1
    for (int j = 0; j < nk; ++j) {
        const PrimPair qq = load_prim(pl, ps, k0 + kPrimLane * j);
#pragma unroll 1
        for (int i = 0; i < nb; ++i) body(load_prim(pl, ps, b0 + kPrimLane * i), qq);
    }
}

// A shell pair record, read field by field through a global pointer.
__device__ __forceinline__ PairInfo load_pair(gptr<const PairInfo> p) {
    const gptr<const double> d = (gptr<const double>)p;
    const gptr<const int> n = (gptr<const int>)(d + 7);
    PairInfo r;
    r.A[0] = d[0];
    r.A[1] = d[1];
    r.A[2] = d[2];
    r.AB[0] = d[3];
    r.AB[1] = d[4];
    r.AB[2] = d[5];
    r.q = d[6];
    r.prim_off = n[0];
    r.nprim = n[1];
    r.sa = n[2];
    r.sb = n[3];
    r.fa = n[4];
    r.fb = n[5];
    return r;
}

// One contracted quartet, one lane.  R = double (FP64 tier) or float (FP32
// tier: the vertical recurrence per primitive quartet runs in FP32; the
// contraction over primitives and both horizontal recurrences run in FP64,
// since the horizontal steps multiply by the pair separations, which are
// large for exactly the small, distant quartets of this tier; the tile is
// stored as float).
template <class C, typename R>
__device__ __forceinline__ bool eri_one(const EriTileArgs& a, const MolDesc& m, const EriItem& it, long long q) {
    const long long bkw = glob(reinterpret_cast<const long long*>(it.quartets))[q];   // (bra, ket) pair ids
    const PairInfo P = load_pair(glob(m.pairs) + static_cast<int>(bkw & 0xffffffff));
    const PairInfo Q = load_pair(glob(m.pairs) + static_cast<int>(bkw >> 32));
    const long long nq = it.n;
    const gptr<R> out = glob(static_cast<R*>(a.tiles)) + it.tile_off + q;
    if (!keep_quartet(P, Q, m.dmax, m.ns, a.tol)) {
#pragma unroll 1
        for (int f = 0; f < C::NF; ++f) out[static_cast<long long>(f) * nq] = R(0);
        return false;
    }
    using C64 = typename C::template With<double>;
    double acc[C::NACC];
#pragma unroll
    for (int i = 0; i < C::NACC; ++i) acc[i] = 0.0;
    prim_loop(m, P.prim_off, P.nprim, Q.prim_off, Q.nprim,
              [&](const PrimPair& pp, const PrimPair& qq) {
                  VrrCoef<double> kd;
                  double T, pref;
                  prim_setup(pp, qq, P.A, Q.A, kd, T, pref);
                  R F[C::L + 1];
                  boys_r<C::L, R>(T, pref, a, F);
                  if constexpr (sizeof(R) == 8) {
                      C::vrr(F, kd, acc);
                  } else {
                      VrrCoef<R> k;
                      coef_to(kd, k);
                      C::vrr(F, k, acc);
                  }
              });
    C64::hrr(acc, P.AB, Q.AB, [&](int f, double v) { out[static_cast<long long>(f) * nq] = static_cast<R>(v); });
    return true;
}

// High angular momentum: passes over groups of bra components.  Each pass
// runs the primitive loop for its own part of the vertical recurrence, keeps
// only its group's accumulators live, applies HRR-CD and parks (e0|cd) in
// scratch; HRR-AB then assembles the tile one ket function pair at a time.
template <class C, typename R, int G>
__device__ __forceinline__ void eri_split_pass(const EriTileArgs& a, const MolDesc& m, const PairInfo& P,
                                               const PairInfo& Q, gptr<double> scr, long long nq) {
    if constexpr (G < C::NG) {
        using C64 = typename C::template With<double>;
        double acc[C::GMAX];
#pragma unroll
        for (int i = 0; i < C::GN[G]; ++i) acc[i] = 0.0;
        prim_loop(m, P.prim_off, P.nprim, Q.prim_off, Q.nprim,
                  [&](const PrimPair& pp, const PrimPair& qq) {
                      VrrCoef<double> kd;
                      double T, pref;
                      prim_setup(pp, qq, P.A, Q.A, kd, T, pref);
                      R F[C::L + 1];
                      boys_r<C::L, R>(T, pref, a, F);
                      if constexpr (sizeof(R) == 8) {
                          C::template vrr_group<G>(F, kd, acc);
                      } else {
                          VrrCoef<R> k;
                          coef_to(kd, k);
                          C::template vrr_group<G>(F, k, acc);
                      }
                  });
        C64::template hrrcd_group<G>(acc, Q.AB, [&](int idx, double v) { scr[static_cast<long long>(idx) * nq] = v; });
        eri_split_pass<C, R, G + 1>(a, m, P, Q, scr, nq);
    }
}

template <class C, typename R>
__device__ __forceinline__ bool eri_one_split(const EriTileArgs& a, const MolDesc& m, const EriItem& it,
                                              long long q) {
    const long long bkw = glob(reinterpret_cast<const long long*>(it.quartets))[q];   // (bra, ket) pair ids
    const PairInfo P = load_pair(glob(m.pairs) + static_cast<int>(bkw & 0xffffffff));
    const PairInfo Q = load_pair(glob(m.pairs) + static_cast<int>(bkw >> 32));
    const long long nq = it.n;
    const gptr<R> out = glob(static_cast<R*>(a.tiles)) + it.tile_off + q;
    if (!keep_quartet(P, Q, m.dmax, m.ns, a.tol)) {
#pragma unroll 1
        for (int f = 0; f < C::NF; ++f) out[static_cast<long long>(f) * nq] = R(0);
        return false;
    }
    // (e0|cd) in FP64 in both tiers: the item's scratch region holds NF x n doubles
    const gptr<double> scr = glob(static_cast<double*>(a.scratch)) + it.tile_off + q;
    eri_split_pass<C, R, 0>(a, m, P, Q, scr, nq);
    using C64 = typename C::template With<double>;
#pragma unroll 1
    for (int cd = 0; cd < C::NCD; ++cd) {
        C64::hrrab([&](int e) -> double { return scr[static_cast<long long>(e * C::NCD + cd) * nq]; }, P.AB,
                   [&](int ab, double v) { out[static_cast<long long>(ab * C::NCD + cd) * nq] = static_cast<R>(v); });
    }
    return true;
}

// Minimum waves per SIMD an integral kernel is compiled for: 2 where timing
// the classes at 1 to 8 showed a gain ((ds|ds) and (dp|ds)); elsewhere the
// register allocation the compiler picks is fastest.
template <class C>
constexpr int eri_waves() {
    return (C::LA == 2 && C::LB == 0 && C::LC == 2 && C::LD == 0) ||
                   (C::LA == 2 && C::LB == 1 && C::LC == 2 && C::LD == 0)
               ? 2
               : 1;
}

// Grid-stride over the blocks of every item of the launch (all molecules of
// a batch for one class and tier).
template <class C, typename R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(eri_waves<C>()))) void k_eri_tile(EriTileArgs a) {
    for (long long blk = blockIdx.x; blk < a.nblocks; blk += gridDim.x) {
        const EriItem it = a.items[find_item(a.items, a.nitems, blk)];
        const long long q = (blk - it.blk0) * blockDim.x + threadIdx.x;
        bool kept = false;
        if (q < it.n) {
            const MolDesc m = load_mol(a.mols, a.mol0, it.mol);
            if constexpr (C::kSplit) kept = eri_one_split<C, R>(a, m, it, q);
            else kept = eri_one<C, R>(a, m, it, q);
        }
        if (a.kept) {
            // measurement: quartets the whole screen kept, one atomic per wavefront
            const unsigned long long mask = __ballot(kept);
            if ((threadIdx.x & 63) == 0 && mask) atomicAdd(a.kept, static_cast<unsigned long long>(__popcll(mask)));
        }
    }
}

}  // namespace jk
