// Device-side building blocks of the J/K build: FP64 Boys function,
// primitive-quartet set-up, the screening decision, and the per-class ERI tile
// and digestion kernels (instantiated once per class in jk_class.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "jk_internal.h"
#include "jk_launch.h"

namespace jk {

#include "eri_gen.inc"

// ---------------------------------------------------------------- Boys ---

// F_m(T), m = 0..L, multiplied by pref.  T < kBoysTMax: seven-term Taylor
// expansion of F_L about the nearest grid point (dF_m/dT = -F_{m+1}), exp(-T)
// from the tabulated exp(-T0) and an eight-term series, then the downward
// recursion F_m = (2T F_{m+1} + e^{-T}) / (2m+1).  Beyond: the asymptotic
// form F_0 = sqrt(pi/T)/2, F_{m+1} = F_m (2m+1)/(2T); the dropped e^{-T}
// terms are below 2e-22.
template <int L>
__device__ __forceinline__ void boys_f64(double T, double pref, const double* __restrict__ tab,
                                         double* __restrict__ F) {
    constexpr double inv_odd[16] = {1.0,       1.0 / 3,  1.0 / 5,  1.0 / 7,  1.0 / 9,  1.0 / 11,
                                    1.0 / 13,  1.0 / 15, 1.0 / 17, 1.0 / 19, 1.0 / 21, 1.0 / 23,
                                    1.0 / 25,  1.0 / 27, 1.0 / 29, 1.0 / 31};
    if (T < kBoysTMax) {
        const int i = static_cast<int>(T * kBoysInvStep + 0.5);
        const double x = static_cast<double>(i) * (1.0 / kBoysInvStep) - T;   // -(T - T0)
        const double* __restrict__ r = tab + i * kBoysCols;
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
        const double it = 1.0 / T;
        double f = sqrt(0.78539816339744830962 * it);   // sqrt(pi/4 / T)
        F[0] = f;
        const double h = 0.5 * it;
#pragma unroll
        for (int m = 0; m < L; ++m) {
            f *= static_cast<double>(2 * m + 1) * h;
            F[m + 1] = f;
        }
    }
#pragma unroll
    for (int m = 0; m <= L; ++m) F[m] *= pref;
}

// Per-primitive-quartet quantities of the vertical recurrence.
__device__ __forceinline__ void prim_setup(const PrimPair& P, const PrimPair& Q, const double* A,
                                           const double* C, VrrCoef<double>& k, double& T,
                                           double& pref) {
    const double p = P.p, q = Q.p;
    const double ipq = 1.0 / (p + q);
    const double rho = p * q * ipq;
    const double PQx = P.P[0] - Q.P[0], PQy = P.P[1] - Q.P[1], PQz = P.P[2] - Q.P[2];
    T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);
    pref = P.E * Q.E * sqrt(ipq);
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
__device__ __forceinline__ bool keep_quartet(const PairInfo& P, const PairInfo& Q,
                                             const double* __restrict__ dmax, int ns, double tol) {
    const double qq = P.q * Q.q;
    if (qq < tol) return false;
    if (dmax == nullptr) return true;
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

template <class C>
__global__ __launch_bounds__(256) void k_eri_tile(EriTileArgs a) {
    const long long q = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= a.nq) return;
    const int2 bk = a.quartets[q];
    const PairInfo& P = a.pairs[bk.x];
    const PairInfo& Q = a.pairs[bk.y];
    double* __restrict__ out = a.out + q;
    if (!keep_quartet(P, Q, a.dmax, a.ns, a.tol)) {
#pragma unroll 1
        for (int f = 0; f < C::NF; ++f) out[static_cast<long long>(f) * a.nq] = 0.0;
        return;
    }
    double acc[C::NACC];
#pragma unroll
    for (int i = 0; i < C::NACC; ++i) acc[i] = 0.0;
    const PrimPair* __restrict__ pb = a.prims + P.prim_off;
    const PrimPair* __restrict__ pk = a.prims + Q.prim_off;
    const int nb = P.nprim, nk = Q.nprim;
#pragma unroll 1
    for (int i = 0; i < nb; ++i) {
        const PrimPair pp = pb[i];
#pragma unroll 1
        for (int j = 0; j < nk; ++j) {
            const PrimPair qq = pk[j];
            VrrCoef<double> k;
            double T, pref;
            prim_setup(pp, qq, P.A, Q.A, k, T, pref);
            double F[C::L + 1];
            boys_f64<C::L>(T, pref, a.boys, F);
            C::vrr(F, k, acc);
        }
    }
    const long long nq = a.nq;
    C::hrr(acc, P.AB, Q.AB, [&](int f, double v) { out[static_cast<long long>(f) * nq] = v; });
}

// High angular momentum: passes over groups of bra components.  Each pass
// runs the primitive loop for its own part of the vertical recurrence, keeps
// only its group's accumulators live, applies HRR-CD and parks (e0|cd) in
// scratch; HRR-AB then assembles the tile one ket function pair at a time.
template <class C, int G>
__device__ __forceinline__ void eri_split_pass(const EriTileArgs& a, const PairInfo& P, const PairInfo& Q,
                                               double* __restrict__ scr, long long nq) {
    if constexpr (G < C::NG) {
        double acc[C::GMAX];
#pragma unroll
        for (int i = 0; i < C::GN[G]; ++i) acc[i] = 0.0;
        const PrimPair* __restrict__ pb = a.prims + P.prim_off;
        const PrimPair* __restrict__ pk = a.prims + Q.prim_off;
        const int nb = P.nprim, nk = Q.nprim;
#pragma unroll 1
        for (int i = 0; i < nb; ++i) {
            const PrimPair pp = pb[i];
#pragma unroll 1
            for (int j = 0; j < nk; ++j) {
                const PrimPair qq = pk[j];
                VrrCoef<double> k;
                double T, pref;
                prim_setup(pp, qq, P.A, Q.A, k, T, pref);
                double F[C::L + 1];
                boys_f64<C::L>(T, pref, a.boys, F);
                C::template vrr_group<G>(F, k, acc);
            }
        }
        C::template hrrcd_group<G>(acc, Q.AB, [&](int idx, double v) { scr[static_cast<long long>(idx) * nq] = v; });
        eri_split_pass<C, G + 1>(a, P, Q, scr, nq);
    }
}

template <class C>
__global__ __launch_bounds__(256) void k_eri_tile_split(EriTileArgs a) {
    const long long q = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= a.nq) return;
    const int2 bk = a.quartets[q];
    const PairInfo& P = a.pairs[bk.x];
    const PairInfo& Q = a.pairs[bk.y];
    double* __restrict__ out = a.out + q;
    const long long nq = a.nq;
    if (!keep_quartet(P, Q, a.dmax, a.ns, a.tol)) {
#pragma unroll 1
        for (int f = 0; f < C::NF; ++f) out[static_cast<long long>(f) * nq] = 0.0;
        return;
    }
    double* __restrict__ scr = a.scratch + q;
    eri_split_pass<C, 0>(a, P, Q, scr, nq);
#pragma unroll 1
    for (int cd = 0; cd < C::NCD; ++cd) {
        C::hrrab([&](int e) -> double { return scr[static_cast<long long>(e * C::NCD + cd) * nq]; }, P.AB,
                 [&](int ab, double v) { out[static_cast<long long>(ab * C::NCD + cd) * nq] = v; });
    }
}

// -------------------------------------------------------------- digest ---

// One workgroup per (segment, density group).  A segment is a run of
// quartets of one class sharing the bra pair (a b); its contributions to K
// fall in four strips -- rows of a and b (K_ac, K_ad, K_bc, K_bd) and columns
// of a and b (K_ca, K_da, K_cb, K_db) -- restricted to the function windows of
// the ket shells' angular momenta.  The strips accumulate in LDS and are
// flushed once with coalesced FP64 atomics: rows into K [x][i][j], columns
// into KT [x][i][j] (K_{row,col} gets KT[col][row]).  J_ab is reduced over
// the segment in registers and LDS; J_cd goes straight to J [i][j][x],
// coalesced over the density lanes.  Scatter of every distinct index
// permutation with the canonical-fold multiplicity w (Sect. 3, Eq.
// (quartet_scatter)).
//
// Thread t handles density x0 + (t % G) for quartets slot, slot + S, ...
// (S = blockDim / G); lanes that share a quartet read the same tile words.
// Digestion of one quartet for one density; OUTER is the unroll pragma of
// the loops over output elements (full unroll keeps a register tile in
// registers, no unroll keeps large tiles streaming from memory).
#define JK_DIGEST_QUARTET(OUTER) \
            if (a.want_j) { \
                /* J_ab += w sum_kl I (D_kl + D_lk); J_cd += w sum_ij I (D_ij + D_ji) */ \
OUTER \
                for (int k = 0; k < NC; ++k) \
OUTER \
                    for (int l = 0; l < ND; ++l) { \
                        const double s2 = w * (Dv(fc + k, fd + l) + Dv(fd + l, fc + k)); \
                        double t = 0.0; \
_Pragma("unroll") \
                        for (int i = 0; i < NA; ++i) \
_Pragma("unroll") \
                            for (int j = 0; j < NB; ++j) { \
                                const double v = I(i, j, k, l); \
                                jacc[i * NB + j] = fma(v, s2, jacc[i * NB + j]); \
                                t = fma(v, Dv(fa + i, fb + j) + Dv(fb + j, fa + i), t); \
                            } \
                        unsafeAtomicAdd(Jm + ((fc + k) * nc + fd + l) * ndp, w * t); \
                    } \
            } \
            if (a.want_k) { \
                /* rows of a: K_ac[i][k] += sum_jl I D_bd[j][l]; K_ad[i][l] += sum_jk I D_bc[j][k] */ \
                /* cols of a: K_ca[k][i] += sum_jl I D_db[l][j]; K_da[l][i] += sum_jk I D_cb[k][j] */ \
OUTER \
                for (int i = 0; i < NA; ++i) { \
OUTER \
                    for (int k = 0; k < NC; ++k) { \
                        double s1 = 0.0, s2 = 0.0; \
_Pragma("unroll") \
                        for (int j = 0; j < NB; ++j) \
_Pragma("unroll") \
                            for (int l = 0; l < ND; ++l) { \
                                const double v = I(i, j, k, l); \
                                s1 = fma(v, Dv(fb + j, fd + l), s1); \
                                s2 = fma(v, Dv(fd + l, fb + j), s2); \
                            } \
                        atomicAdd(S(i, cc + k), w * s1); \
                        atomicAdd(S(NA + NB + i, cc + k), w * s2); \
                    } \
OUTER \
                    for (int l = 0; l < ND; ++l) { \
                        double s1 = 0.0, s2 = 0.0; \
_Pragma("unroll") \
                        for (int j = 0; j < NB; ++j) \
_Pragma("unroll") \
                            for (int k = 0; k < NC; ++k) { \
                                const double v = I(i, j, k, l); \
                                s1 = fma(v, Dv(fb + j, fc + k), s1); \
                                s2 = fma(v, Dv(fc + k, fb + j), s2); \
                            } \
                        atomicAdd(S(i, cd + l), w * s1); \
                        atomicAdd(S(NA + NB + i, cd + l), w * s2); \
                    } \
                } \
                /* rows of b: K_bc[j][k] += sum_il I D_ad[i][l]; K_bd[j][l] += sum_ik I D_ac[i][k] */ \
                /* cols of b: K_cb[k][j] += sum_il I D_da[l][i]; K_db[l][j] += sum_ik I D_ca[k][i] */ \
OUTER \
                for (int j = 0; j < NB; ++j) { \
OUTER \
                    for (int k = 0; k < NC; ++k) { \
                        double s1 = 0.0, s2 = 0.0; \
_Pragma("unroll") \
                        for (int i = 0; i < NA; ++i) \
_Pragma("unroll") \
                            for (int l = 0; l < ND; ++l) { \
                                const double v = I(i, j, k, l); \
                                s1 = fma(v, Dv(fa + i, fd + l), s1); \
                                s2 = fma(v, Dv(fd + l, fa + i), s2); \
                            } \
                        atomicAdd(S(NA + j, cc + k), w * s1); \
                        atomicAdd(S(2 * NA + NB + j, cc + k), w * s2); \
                    } \
OUTER \
                    for (int l = 0; l < ND; ++l) { \
                        double s1 = 0.0, s2 = 0.0; \
_Pragma("unroll") \
                        for (int i = 0; i < NA; ++i) \
_Pragma("unroll") \
                            for (int k = 0; k < NC; ++k) { \
                                const double v = I(i, j, k, l); \
                                s1 = fma(v, Dv(fa + i, fc + k), s1); \
                                s2 = fma(v, Dv(fc + k, fa + i), s2); \
                            } \
                        atomicAdd(S(NA + j, cd + l), w * s1); \
                        atomicAdd(S(2 * NA + NB + j, cd + l), w * s2); \
                    } \
                } \
            } \
        

template <int LA, int LB, int LC, int LD>
__global__ __launch_bounds__(256) void k_digest(DigestArgs a) {
    extern __shared__ double lds[];
    constexpr int NA = (LA + 1) * (LA + 2) / 2, NB = (LB + 1) * (LB + 2) / 2;
    constexpr int NC = (LC + 1) * (LC + 2) / 2, ND = (LD + 1) * (LD + 2) / 2;
    constexpr int NF = NA * NB * NC * ND;
    constexpr int R = 2 * (NA + NB);
    constexpr bool kRegTile = NF <= 36;
    const int G = a.G;
    // blocks of one segment share an XCD (block b runs on XCD b % 8)
    const int b = blockIdx.x;
    const int xcd = b & 7, kk = b >> 3;
    const int seg = (kk / a.ngroups) * 8 + xcd;
    const int grp = kk - (kk / a.ngroups) * a.ngroups;
    if (seg >= a.nseg) return;
    const int x0 = grp * G;
    const int gn = min(G, a.nd - x0);
    const int W = a.colAw + a.colBw;
    const int nstrip = a.want_k ? R * G * W : 0;
    double* __restrict__ strips = lds;            // [R][G][W]
    double* __restrict__ jab = lds + nstrip;      // [NA*NB][G]
    const int nlds = nstrip + (a.want_j ? NA * NB * G : 0);
    for (int i = threadIdx.x; i < nlds; i += blockDim.x) lds[i] = 0.0;
    __syncthreads();

    const int2 sg = a.segs[seg];
    const long long q0 = sg.x - a.qbase;
    const int slots = blockDim.x / G;
    const int slot = threadIdx.x / G, g = threadIdx.x - slot * G;
    const bool active = slot < slots && g < gn;
    const PairInfo& P = a.pairs[a.quartets[q0].x];
    const int fa = P.fa, fb = P.fb;
    const long long nc = a.nc, ndp = a.ndp, nq = a.nq;
    auto lcol = [&](int col) { return (col >= a.colA0 && col < a.colA0 + a.colAw) ? col - a.colA0 : a.colAw + (col - a.colB0); };
    double jacc[NA * NB];
#pragma unroll
    for (int e = 0; e < NA * NB; ++e) jacc[e] = 0.0;
    if (active) {
        const int x = x0 + g;
        const double* __restrict__ Dm = a.D + x;
        auto Dv = [&](int r, int c) -> double { return Dm[(r * nc + c) * ndp]; };
        double* __restrict__ Jm = a.J + x;
        double* __restrict__ sA = strips + static_cast<long long>(g) * W;   // row block 0, density g
        auto S = [&](int row, int col) -> double* { return sA + static_cast<long long>(row) * G * W + col; };
#pragma unroll 1
        for (int qi = slot; qi < sg.y; qi += slots) {
            const long long q = q0 + qi;
            const int2 bk = a.quartets[q];
            const PairInfo& Q = a.pairs[bk.y];
            if (!keep_quartet(P, Q, a.dmax, a.ns, a.tol)) continue;
            double w = 1.0;
            if (P.sa == P.sb) w *= 0.5;
            if (Q.sa == Q.sb) w *= 0.5;
            if (bk.x == bk.y) w *= 0.5;
            const double* __restrict__ tg = a.tiles + q;
            double treg[kRegTile ? NF : 1];
            if constexpr (kRegTile) {
#pragma unroll
                for (int f = 0; f < NF; ++f) treg[f] = tg[f * nq];
            }
            auto I = [&](int i, int j, int k, int l) -> double {
                const int f = ((i * NB + j) * NC + k) * ND + l;
                if constexpr (kRegTile) return treg[f];
                else return tg[static_cast<long long>(f) * nq];
            };
            const int fc = Q.fa, fd = Q.fb;
            const int cc = lcol(fc), cd = lcol(fd);
            if constexpr (kRegTile) {
                JK_DIGEST_QUARTET(_Pragma("unroll"))
            } else {
                JK_DIGEST_QUARTET(_Pragma("unroll 1"))
            }
}
        if (a.want_j) {
#pragma unroll
            for (int e = 0; e < NA * NB; ++e) atomicAdd(jab + e * G + g, jacc[e]);
        }
    }
    __syncthreads();
    // flush: column index fastest, so lanes write consecutive addresses
    if (a.want_k) {
        const long long mat = nc * nc;
        for (int idx = threadIdx.x; idx < R * G * W; idx += blockDim.x) {
            const int c = idx % W;
            const int rg = idx / W;
            const int gg = rg % G, r = rg / G;
            if (gg >= gn) continue;
            const double v = strips[idx];
            if (v == 0.0) continue;
            const int col = c < a.colAw ? a.colA0 + c : a.colB0 + (c - a.colAw);
            const long long x = x0 + gg;
            if (r < NA) unsafeAtomicAdd(a.K + x * mat + (fa + r) * nc + col, v);
            else if (r < NA + NB) unsafeAtomicAdd(a.K + x * mat + (fb + r - NA) * nc + col, v);
            else if (r < 2 * NA + NB) unsafeAtomicAdd(a.KT + x * mat + (fa + r - NA - NB) * nc + col, v);
            else unsafeAtomicAdd(a.KT + x * mat + (fb + r - 2 * NA - NB) * nc + col, v);
        }
    }
    if (a.want_j) {
        for (int idx = threadIdx.x; idx < NA * NB * G; idx += blockDim.x) {
            const int e = idx / G, gg = idx - e * G;
            if (gg >= gn) continue;
            const int i = e / NB, j = e - i * NB;
            unsafeAtomicAdd(a.J + ((fa + i) * nc + fb + j) * ndp + x0 + gg, jab[idx]);
        }
    }
}

}  // namespace jk
