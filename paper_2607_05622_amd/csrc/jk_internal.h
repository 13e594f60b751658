// Internal data layout shared by the host side and the kernels of the J/K
// library.  Nothing here is part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jk {

constexpr int kMaxL = 2;
constexpr int kNumPairClass = 6;    // ss ps pp ds dp dd
constexpr int kNumClass = 21;       // canonical (la lb | lc ld)

// Boys table: F_m(T0) for m = 0..kBoysCols-2 and exp(-T0) in the last
// column, at T0 = i / kBoysInvStep for T0 < kBoysTMax.
constexpr int kBoysCols = 16;
constexpr double kBoysInvStep = 32.0;
constexpr double kBoysTMax = 50.0;
constexpr int kBoysPoints = 1601;   // 0 .. 50 inclusive at 1/32

// One shell pair (a >= b in internal shell order, so la >= lb).
struct PairInfo {
    double A[3];      // centre of a
    double AB[3];     // A - B
    double q;         // Schwarz factor sqrt(max (mn|mn))
    int32_t prim_off; // slot of the first primitive-pair record (record j in slot prim_off + kPrimLane j)
    int32_t nprim;    // number of primitive-pair records
    int32_t sa, sb;   // internal shells
    int32_t fa, fb;   // first internal Cartesian function of a, b
};

// One primitive pair of a shell pair: p = alpha + beta, P = (alpha A +
// beta B)/p, E = sqrt(2) pi^(5/4) c_a c_b exp(-alpha beta/p |AB|^2) / p (so
// that the primitive-quartet prefactor 2 pi^(5/2) K_ab K_cd / (p q
// sqrt(p+q)) is E_ab E_cd / sqrt(p+q)), o2p = 1/(2p).
struct PrimPair {
    double p, P[3], E, o2p, pad0, pad1;
};

// Device layout of the primitive-pair records: three planes of pslots
// (2 x double) entries, (p, E), (P_x, P_y), (P_z, 1/2p).  The pairs are
// taken in groups of kPrimLane consecutive pair ids; record j of pair i sits
// in slot base(i / kPrimLane) + kPrimLane j + i % kPrimLane, so the lanes of
// a wavefront reading record j of consecutive ket pairs read consecutive
// entries.
constexpr int kPrimLane = 64;

// Per-primitive-quartet coefficients of the vertical recurrence.
template <typename R>
struct VrrCoef {
    R PA[3], WP[3], QC[3], WQ[3];
    R rp, rq;          // rho/p, rho/q
    R o2p, o2q, o2pq;  // 1/2p, 1/2q, 1/2(p+q)
};

// Canonical class index of (la lb | lc ld) with la >= lb, lc >= ld and
// pair class(la,lb) >= pair class(lc,ld).
__host__ __device__ inline int pair_class(int la, int lb) { return la * (la + 1) / 2 + lb; }
__host__ __device__ inline int quartet_class(int X, int Y) { return X * (X + 1) / 2 + Y; }

__host__ __device__ constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }

// Quartets a digestion workgroup stages in LDS per chunk for class
// (la lb | lc ld) with nf Cartesian functions per quartet, in pass C
// (dig_qb_c) and pass D (dig_qb_d): a multiple of the MFMA k-depth 4 and at
// most ~47 KB of LDS (52 KB for (dd|dd)); chosen by timing each class on
// the 312-AO workload at 4 to 32.
__host__ __device__ constexpr int dig_qb_default(int nf) {
    return nf <= 27 ? 16 : (nf <= 90 ? 32 : (nf <= 170 ? 16 : (nf <= 324 ? 8 : 4)));
}
__host__ __device__ constexpr int dig_qb_c(int la, int lb, int lc, int ld, int nf) {
    const int t = la * 1000 + lb * 100 + lc * 10 + ld;
    return (t == 1110 || t == 2221) ? 8
           : (t == 2011 || t == 1111 || t == 2211) ? 16
           : (t == 1000 || t == 2000 || t == 2120) ? 32
           : dig_qb_default(nf);
}
__host__ __device__ constexpr int dig_qb_d(int la, int lb, int lc, int ld, int nf) {
    const int t = la * 1000 + lb * 100 + lc * 10 + ld;
    return (t == 1110 || t == 2111) ? 8 : (t == 2011 || t == 1111) ? 16 : dig_qb_default(nf);
}

// Minimum waves per SIMD the digestion kernels of class (la lb | lc ld) are
// compiled for (pass C; pass D uses 3): the register budget that trades
// spills against latency hiding, chosen by timing each class of pass C on
// the 620-AO workload (40 densities) at 1 to 4 (e.g. (dd|dp): 54.7 ms at 1,
// 29.4 ms at 3 per build).
__host__ __device__ constexpr int dig_waves_c(int la, int lb, int lc, int ld) {
    const int t = la * 1000 + lb * 100 + lc * 10 + ld;
    return (t == 2100) ? 1
           : (t == 2120 || t == 2121 || t == 2211 || t == 2221 || t == 2222) ? 3
           : (t == 1000 || t == 1110 || t == 2020) ? 4
           : 2;
}

// Pass D of the FP64 tier on 4 x 4 matrix-core blocks (k_digest_d4) for
// class (la lb | lc ld), instead of 16 x 16 tiles: timed per class on the
// 620-AO workload (0.76-0.83 of the 16 x 16 time where it is used; the six
// classes left out ran 3-33% slower on it).
__host__ __device__ constexpr bool dig_d4(int la, int lb, int lc, int ld) {
    const int t = la * 1000 + lb * 100 + lc * 10 + ld;
    return !(t == 1111 || t == 2111 || t == 2121 || t == 2210 || t == 2211 || t == 2222);
}

// The K waves of pass C (FP64 tier) on 4 x 4 matrix-core blocks for class
// (la lb | lc ld): timed per class on the 620-AO workload, where pass C took
// 0.71-0.95 of its 16 x 16 time for these seven classes; the others ran at
// 0.97-1.42 of it (their longer K rows fill 16-row tiles, and the extra
// accumulators cost registers).
__host__ __device__ constexpr bool dig_c4(int la, int lb, int lc, int ld) {
    const int t = la * 1000 + lb * 100 + lc * 10 + ld;
    return t == 0 || t == 1000 || t == 1010 || t == 1100 || t == 2000 || t == 2010 || t == 2011;
}

}  // namespace jk
