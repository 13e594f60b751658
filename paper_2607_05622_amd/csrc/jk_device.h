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

// -------------------------------------------------------------- digest ---

// Lane (slot, x): slot picks the quartet, x the density (strided by dg).
// Tile element (i j | k l) of quartet q sits at tiles[f * nq + q],
// f = ((i NB + j) NC + k) ND + l.  Densities and accumulators are
// [row][col][x] with x innermost (ndp entries per matrix element).
template <int LA, int LB, int LC, int LD>
__global__ __launch_bounds__(256) void k_digest(DigestArgs a) {
    constexpr int NA = (LA + 1) * (LA + 2) / 2, NB = (LB + 1) * (LB + 2) / 2;
    constexpr int NC = (LC + 1) * (LC + 2) / 2, ND = (LD + 1) * (LD + 2) / 2;
    constexpr int NF = NA * NB * NC * ND;
    constexpr bool kRegTile = NF <= 108;
    const int dg = a.dg;
    const int slot = threadIdx.x / dg;
    const int x0 = threadIdx.x - slot * dg;
    const long long q = static_cast<long long>(blockIdx.x) * (blockDim.x / dg) + slot;
    if (q >= a.nq || x0 >= a.ndp) return;
    const int2 bk = a.quartets[q];
    const PairInfo& P = a.pairs[bk.x];
    const PairInfo& Q = a.pairs[bk.y];
    if (!keep_quartet(P, Q, a.dmax, a.ns, a.tol)) return;
    double w = 1.0;
    if (P.sa == P.sb) w *= 0.5;
    if (Q.sa == Q.sb) w *= 0.5;
    if (bk.x == bk.y) w *= 0.5;
    const long long nq = a.nq;
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
    const int fa = P.fa, fb = P.fb, fc = Q.fa, fd = Q.fb;
    const long long nc = a.nc, ndp = a.ndp;
    for (int x = x0; x < a.ndp; x += dg) {
        const double* __restrict__ Dm = a.D + x;
        auto Dv = [&](int r, int c) -> double { return Dm[(r * nc + c) * ndp]; };
        double* __restrict__ Jm = a.J + x;
        double* __restrict__ Km = a.K + x;
        if (a.want_j) {
            // J_ab += sum_kl (ij|kl) (D_kl + D_lk), J_cd += sum_ij (ij|kl) (D_ij + D_ji)
            double s2cd[NC * ND];
#pragma unroll
            for (int k = 0; k < NC; ++k)
#pragma unroll
                for (int l = 0; l < ND; ++l) s2cd[k * ND + l] = Dv(fc + k, fd + l) + Dv(fd + l, fc + k);
            double s2ab[NA * NB];
#pragma unroll
            for (int i = 0; i < NA; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j) s2ab[i * NB + j] = Dv(fa + i, fb + j) + Dv(fb + j, fa + i);
#pragma unroll
            for (int i = 0; i < NA; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    double s = 0.0;
#pragma unroll
                    for (int k = 0; k < NC; ++k)
#pragma unroll
                        for (int l = 0; l < ND; ++l) s = fma(I(i, j, k, l), s2cd[k * ND + l], s);
                    unsafeAtomicAdd(Jm + ((fa + i) * nc + fb + j) * ndp, w * s);
                }
#pragma unroll
            for (int k = 0; k < NC; ++k)
#pragma unroll
                for (int l = 0; l < ND; ++l) {
                    double s = 0.0;
#pragma unroll
                    for (int i = 0; i < NA; ++i)
#pragma unroll
                        for (int j = 0; j < NB; ++j) s = fma(I(i, j, k, l), s2ab[i * NB + j], s);
                    unsafeAtomicAdd(Jm + ((fc + k) * nc + fd + l) * ndp, w * s);
                }
        }
        if (a.want_k) {
            // K_ac[i][k] += sum_jl I D_bd[j][l];  K_ca[k][i] += sum_jl I D_db[l][j]
#pragma unroll
            for (int i = 0; i < NA; ++i)
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    double s1 = 0.0, s2 = 0.0;
#pragma unroll
                    for (int j = 0; j < NB; ++j)
#pragma unroll
                        for (int l = 0; l < ND; ++l) {
                            const double v = I(i, j, k, l);
                            s1 = fma(v, Dv(fb + j, fd + l), s1);
                            s2 = fma(v, Dv(fd + l, fb + j), s2);
                        }
                    unsafeAtomicAdd(Km + ((fa + i) * nc + fc + k) * ndp, w * s1);
                    unsafeAtomicAdd(Km + ((fc + k) * nc + fa + i) * ndp, w * s2);
                }
            // K_bc[j][k] += sum_il I D_ad[i][l];  K_cb[k][j] += sum_il I D_da[l][i]
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    double s1 = 0.0, s2 = 0.0;
#pragma unroll
                    for (int i = 0; i < NA; ++i)
#pragma unroll
                        for (int l = 0; l < ND; ++l) {
                            const double v = I(i, j, k, l);
                            s1 = fma(v, Dv(fa + i, fd + l), s1);
                            s2 = fma(v, Dv(fd + l, fa + i), s2);
                        }
                    unsafeAtomicAdd(Km + ((fb + j) * nc + fc + k) * ndp, w * s1);
                    unsafeAtomicAdd(Km + ((fc + k) * nc + fb + j) * ndp, w * s2);
                }
            // K_ad[i][l] += sum_jk I D_bc[j][k];  K_da[l][i] += sum_jk I D_cb[k][j]
#pragma unroll
            for (int i = 0; i < NA; ++i)
#pragma unroll
                for (int l = 0; l < ND; ++l) {
                    double s1 = 0.0, s2 = 0.0;
#pragma unroll
                    for (int j = 0; j < NB; ++j)
#pragma unroll
                        for (int k = 0; k < NC; ++k) {
                            const double v = I(i, j, k, l);
                            s1 = fma(v, Dv(fb + j, fc + k), s1);
                            s2 = fma(v, Dv(fc + k, fb + j), s2);
                        }
                    unsafeAtomicAdd(Km + ((fa + i) * nc + fd + l) * ndp, w * s1);
                    unsafeAtomicAdd(Km + ((fd + l) * nc + fa + i) * ndp, w * s2);
                }
            // K_bd[j][l] += sum_ik I D_ac[i][k];  K_db[l][j] += sum_ik I D_ca[k][i]
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int l = 0; l < ND; ++l) {
                    double s1 = 0.0, s2 = 0.0;
#pragma unroll
                    for (int i = 0; i < NA; ++i)
#pragma unroll
                        for (int k = 0; k < NC; ++k) {
                            const double v = I(i, j, k, l);
                            s1 = fma(v, Dv(fa + i, fc + k), s1);
                            s2 = fma(v, Dv(fc + k, fa + i), s2);
                        }
                    unsafeAtomicAdd(Km + ((fb + j) * nc + fd + l) * ndp, w * s1);
                    unsafeAtomicAdd(Km + ((fd + l) * nc + fb + j) * ndp, w * s2);
                }
        }
    }
}

}  // namespace jk
