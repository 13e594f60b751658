// Digestion of ERI tiles against stacked densities on the FP64 matrix cores.
//
// For a canonical quartet (ab|cd) with fold weight w (Sect. 3, Eq.
// (quartet_scatter)) and every density x of the batch, digestion adds
//   J_ab += w I D^S_cd,  J_cd += w I D^S_ab          (D^S = D + D^T)
//   K_ac += w I D_bd,  K_bc += w I D_ad,  K_ad += w I D_bc,  K_bd += w I D_ac
// and the same four with D^T into KT (the transposed contributions), so that
// J = Jc + Jc^T and K = Kc + KTc^T hold for non-symmetric D (Eq. (jkbuild)).
//
// J reads D^S from records packed per shell pair (built once per call), so
// the ket pairs of a bra block, visited in pair order, read neighbouring
// records; the K updates read D itself.
//
// The FP32 tier of mixed builds is digested in FP32: FP32 tiles against
// FP32 copies of D and D^S on the FP32 matrix cores, each chunk's sums added
// into FP64 accumulators, which are flushed into the FP64 J and K (the
// paper's FP32 evaluation with FP64 accumulation, Sect. 3 mixed-precision
// paragraph).
//
// Each update is a contraction of the tile with a gather of the densities,
// stacked along the MFMA N dimension: 16 densities (the D and D^T
// contractions then run on separate waves), or 8 densities in columns 0-7
// and the same 8 with D^T in columns 8-15.  One workgroup owns one task: a
// piece of the quartets of one bra pair and one density group.  It stages
// the tiles of a chunk (up to QB quartets of one run) in LDS once; its waves
// then take one role each (J; K with D; K with D^T), so a wave holds only
// its own accumulators.  The quartets of a bra pair sit in the class list in
// (c, d) order, so the updates whose output is indexed by c (J_ab, K_ac,
// K_bc) keep their sums in the MFMA accumulators until the run of equal c
// ends; J_cd is written per quartet.  Pass C walks that order and also
// writes each tile, quartet-major, at its position in the (d, c) order;
// pass D walks that copy in runs of equal d for K_ad and K_bd, for most
// classes of the FP64 tier on 4 x 4 matrix-core blocks (k_digest_d4), whose
// 4-row output tiles fit pass D's short outputs.
#pragma once

#include "jk_device.h"

namespace jk {

typedef double v4d __attribute__((ext_vector_type(4)));

// C(16x16) += A(16x4) B(4x16) in FP64 on the matrix cores.  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and holds C[4 r + l / 16][l % 16]
// in element r.
__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void gadd(double* p, double v) { (void)__builtin_amdgcn_global_atomic_fadd_f64(glob(p), v); }

typedef float v4f __attribute__((ext_vector_type(4)));

// Matrix-core step of the digestion in compute type R.  FP64: element e of
// lane l holds output row 4 e + l / 16; FP32 (v_mfma_f32_16x16x4f32): row
// 4 (l / 16) + e; both hold column l % 16 and take A[l % 16][l / 16],
// B[l / 16][l % 16] (probed).
template <typename R>
struct DigMma;
template <>
struct DigMma<double> {
    using V = v4d;
    static __device__ __forceinline__ V step(double a, double b, V c) { return mfma_f64(a, b, c); }
    static __device__ __forceinline__ int row(int e, int r4) { return 4 * e + r4; }
    static __device__ __forceinline__ const double* dens(const MolDesc& m) { return m.D; }
    static __device__ __forceinline__ const double* dtrans(const MolDesc& m) { return m.DT; }
    static __device__ __forceinline__ const double* dsym(const MolDesc& m) { return m.DS; }
};
template <>
struct DigMma<float> {
    using V = v4f;
    static __device__ __forceinline__ V step(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int e, int r4) { return 4 * r4 + e; }
    static __device__ __forceinline__ const float* dens(const MolDesc& m) { return m.Df; }
    static __device__ __forceinline__ const float* dtrans(const MolDesc& m) { return m.DTf; }
    static __device__ __forceinline__ const float* dsym(const MolDesc& m) { return m.DSf; }
};

// Accumulator tile of a sum that spans chunks: FP64 runs accumulate in the
// matrix-core registers directly; FP32 runs keep each chunk's sum in FP32
// and add it into an FP64 copy at the end of the chunk (fold).
template <typename R>
struct DigAcc {
    typename DigMma<R>::V a;
    v4d s;   // FP64 sum of the folded chunks (unused for R = double)
    __device__ __forceinline__ void zero() {
        a = typename DigMma<R>::V{0, 0, 0, 0};
        if constexpr (sizeof(R) == 4) s = v4d{0.0, 0.0, 0.0, 0.0};
    }
    __device__ __forceinline__ void fold() {
        if constexpr (sizeof(R) == 4) {
#pragma unroll
            for (int e = 0; e < 4; ++e) s[e] += static_cast<double>(a[e]);
            a = typename DigMma<R>::V{0, 0, 0, 0};
        }
    }
    // the FP64 value of element e (after fold for R = float)
    __device__ __forceinline__ double get(int e) const {
        if constexpr (sizeof(R) == 4) return s[e];
        else return a[e];
    }
};

// Workgroup barrier that orders LDS only: the waves' atomics and stores to
// device memory stay in flight across it (nothing in the workgroup reads
// them back), where __syncthreads would wait for every one of them.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The task of the calling workgroup: its block item, part and density
// group.  Workgroup b runs on XCD b % 8 and takes task b / 8 of that XCD,
// found by bisection over the XCD's items.  Returns nullptr when idle.
__device__ __forceinline__ const DigItem* dig_task(const DigestArgs& a, int& p0, int& plen, int& grp) {
    const int b = blockIdx.x, xcd = b & 7, task = b >> 3;
    int lo = 0, hi = a.nitems / 8 - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.items[xcd + 8 * mid].kstart <= task) lo = mid;
        else hi = mid - 1;
    }
    const DigItem* it = a.items + xcd + 8 * lo;
    if (it->kstart > task) return nullptr;
    const int local = task - it->kstart;
    const int pc = local / it->ngroups;
    if (pc >= it->nparts) return nullptr;
    grp = local - pc * it->ngroups;
    const gptr<const int> parts = glob(it->parts);
    p0 = parts[pc];
    plen = (pc + 1 < it->nparts ? parts[pc + 1] : it->len) - p0;
    return it;
}

template <int LA, int LB, int LC, int LD>
struct DigShape {
    static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    static constexpr int NF = NA * NB * NC * ND, NAB = NA * NB, NCD = NC * ND;
    static constexpr int QB = dig_qb_c(LA, LB, LC, LD, NF), QBP = QB + 1;       // pass C
    static constexpr int QB_D = dig_qb_d(LA, LB, LC, LD, NF), QBP_D = QB_D + 1;  // pass D
    static constexpr int WAVES_C = dig_waves_c(LA, LB, LC, LD), WAVES_D = 3;
    // accumulator tiles (16 output rows each) per update
    static constexpr int MJ = (NAB + 15) / 16;          // J_ab rows (i, j)
    static constexpr int M2 = (QB * NCD + 15) / 16;     // J_cd rows (quartet, k, l)
    static constexpr int KJ2 = (NAB + 3) / 4;           // J_cd k-steps over (i, j)
    static constexpr int M3 = (NA * NC + 15) / 16;      // K_ac rows (i, k)
    static constexpr int M4 = (NB * NC + 15) / 16;      // K_bc rows (j, k)
    static constexpr int M5 = (NA * ND + 15) / 16;      // K_ad rows (i, l)
    static constexpr int M6 = (NB * ND + 15) / 16;      // K_bd rows (j, l)
    static constexpr int NACC_C = MJ > M3 + M4 ? MJ : M3 + M4;
    static constexpr int NACC_D = M5 + M6;
};

// Density access of one lane.  The lane's MFMA column is density x; its K
// contractions read D[F][V] (tr = false) or D[V][F] (tr = true) for a fixed
// bra-side function F and a ket-side function V.  D[V][F] is read as
// DT[F][V] from the transposed copy, so both forms walk the bra rows F.
template <typename R = double>
struct DigLane {
    int x;
    bool tr;
    long long sRow, ndp;
    gptr<const R> Dx, DTx, Kx;
    __device__ DigLane(const MolDesc& m, int x_, bool tr_) : x(x_), tr(tr_) {
        ndp = m.ndp;
        sRow = static_cast<long long>(m.nc) * ndp;
        Dx = glob(DigMma<R>::dens(m)) + x;
        DTx = glob(DigMma<R>::dtrans(m)) + x;
        Kx = tr ? DTx : Dx;
    }
    __device__ __forceinline__ R d(long long r, long long c) const { return Dx[r * sRow + c * ndp]; }
    __device__ __forceinline__ R dt(long long r, long long c) const { return DTx[r * sRow + c * ndp]; }
    __device__ __forceinline__ R dk(long long F, long long V) const { return Kx[F * sRow + V * ndp]; }
};

// Fold weight of a canonical quartet from its shells: 1/2 for a = b, for
// c = d and for (ab) = (cd).
__device__ __forceinline__ double fold_weight(int sa, int sb, int sc, int sd) {
    return (sa == sb ? 0.5 : 1.0) * (sc == sd ? 0.5 : 1.0) * (sa == sc && sb == sd ? 0.5 : 1.0);
}

// Adds a finished K accumulator tile into K (D contraction) or KT (D^T
// contraction) and clears it; rowmap turns an output row into its (row,
// column) function.
template <int NROW, typename R, class RowMap>
__device__ __forceinline__ void dig_flush_k(const MolDesc& m, const DigLane<R>& L, int r4, DigAcc<R>& acc, int mt,
                                            RowMap rowmap) {
    acc.fold();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int mo = mt * 16 + DigMma<R>::row(r, r4);
        if (mo < NROW && L.x < m.nd) {
            long long row, col;
            rowmap(mo, row, col);
            gadd((L.tr ? m.KT : m.K) + (row * m.nc + col) * L.ndp + L.x, acc.get(r));
        }
    }
    acc.zero();
}

// Scan of the next chunk, done identically by every wave: up to QB
// positions from p on whose ket shell (field `shift` of kin.x) equals that of
// position p.  Returns n >= 1; `more` tells whether the run goes on after it.
template <int QB>
__device__ __forceinline__ int dig_chunk(gptr<const long long> kin, int p, int pend, int lane, int shift, int2& kv,
                                         bool& more) {
    int sh = -1;
    kv = make_int2(0, 0);
    if (lane <= QB && p + lane < pend) {
        const long long raw = kin[p + lane];   // the int2 (x, y) as one 8-byte word
        kv = make_int2(static_cast<int>(raw & 0xffffffff), static_cast<int>(raw >> 32));
        sh = (kv.x >> shift) & 0xffff;
    }
    const int s0 = __shfl(sh, 0);
    const unsigned long long same = __ballot(sh == s0);
    const int n = __builtin_ctzll(~same);
    more = n > QB;
    return more ? QB : n;
}

// v_mfma_f64_4x4x4f64: four independent 4 x 4 products with k-depth 4; it
// issues every 16 cycles, a quarter of the 16 x 16 x 4 form, at the same
// FP64 rate.  Lane l = 16 q + 4 b + r works on block b: it supplies A[r][q]
// and B[q][r] and holds C[q][r] (probed).  Below, u = 4 q + r.
struct Mfma4 {
    static __device__ __forceinline__ int block(int lane) { return (lane >> 2) & 3; }
    static __device__ __forceinline__ int u(int lane) { return ((lane >> 4) << 2) | (lane & 3); }
    static __device__ __forceinline__ double step(double a, double b, double c) {
        return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int arow(int u) { return u & 3; }
    static __device__ __forceinline__ int ak(int u) { return u >> 2; }
    static __device__ __forceinline__ int bk(int u) { return u >> 2; }
    static __device__ __forceinline__ int bcol(int u) { return u & 3; }
    static __device__ __forceinline__ int crow(int u) { return u >> 2; }
    static __device__ __forceinline__ int ccol(int u) { return u & 3; }
};

// K_ad += I D_bc and K_bd += I D_ac for the n quartets of a staged chunk
// whose ket shell c (first function fc) is shared and whose d functions
// start at sV[q]: output rows (q, i, l) and (q, j, l), contraction over
// (j, k) and (i, k) against density operands fixed for the chunk.  Adds
// each finished row into K (or KT for the D^T contraction).
template <int LA, int LB, int LC, int LD, int QB, typename R>
__device__ __forceinline__ void dig_kd_rows(const MolDesc& m, const DigLane<R>& L, int r4, int c16, const R* sT,
                                            const int* sV, int n, int fa, int fb, int fc) {
    using MM = DigMma<R>;
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    constexpr int NCD = NC * ND, QBP = QB + 1;
    constexpr int RAD = NA * ND, RBD = NB * ND;                 // output rows per quartet
    constexpr int KAD = (NB * NC + 3) / 4, KBD = (NA * NC + 3) / 4;   // k-steps
    constexpr int MAD = (QB * RAD + 15) / 16, MBD = (QB * RBD + 15) / 16;
    const long long nc = m.nc;
    double* const out = L.tr ? m.KT : m.K;
    // the density operands of the chunk: D_bc at k-row (j, k), D_ac at (i, k)
    R bad[KAD], bbd[KBD];
#pragma unroll
    for (int t = 0; t < KAD; ++t) {
        const int kk = 4 * t + r4;
        bad[t] = kk < NB * NC ? L.dk(fb + kk / NC, fc + kk % NC) : R(0);
    }
#pragma unroll
    for (int t = 0; t < KBD; ++t) {
        const int kk = 4 * t + r4;
        bbd[t] = kk < NA * NC ? L.dk(fa + kk / NC, fc + kk % NC) : R(0);
    }
    // K_ad: row (q, i, l), k-row (j, k) of tile function ((i NB + j) NC + k) ND + l
#pragma unroll 1
    for (int mt = 0; mt < MAD; ++mt) {
        if (mt * 16 >= n * RAD) break;
        const int r = mt * 16 + c16;
        const int q = r < n * RAD ? r / RAD : 0, u = r < n * RAD ? r - (r / RAD) * RAD : 0;
        const int i = u / ND, l = u - (u / ND) * ND;
        typename MM::V v = {0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < KAD; ++t) {
            const int kk = 4 * t + r4 < NB * NC ? 4 * t + r4 : NB * NC - 1;
            const int j = kk / NC, k = kk - (kk / NC) * NC;
            v = MM::step(sT[(((i * NB + j) * NC + k) * ND + l) * QBP + q], bad[t], v);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int mo = mt * 16 + MM::row(e, r4);
            const int qo = mo / RAD, uo = mo - (mo / RAD) * RAD;
            if (qo < n && L.x < m.nd) {
                const int io = uo / ND, lo = uo - (uo / ND) * ND;
                gadd(out + ((fa + io) * nc + sV[qo] + lo) * L.ndp + L.x, static_cast<double>(v[e]));
            }
        }
    }
    // K_bd: row (q, j, l), k-row (i, k)
#pragma unroll 1
    for (int mt = 0; mt < MBD; ++mt) {
        if (mt * 16 >= n * RBD) break;
        const int r = mt * 16 + c16;
        const int q = r < n * RBD ? r / RBD : 0, u = r < n * RBD ? r - (r / RBD) * RBD : 0;
        const int j = u / ND, l = u - (u / ND) * ND;
        typename MM::V v = {0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < KBD; ++t) {
            const int kk = 4 * t + r4 < NA * NC ? 4 * t + r4 : NA * NC - 1;
            const int i = kk / NC, k = kk - (kk / NC) * NC;
            v = MM::step(sT[(((i * NB + j) * NC + k) * ND + l) * QBP + q], bbd[t], v);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int mo = mt * 16 + MM::row(e, r4);
            const int qo = mo / RBD, uo = mo - (mo / RBD) * RBD;
            if (qo < n && L.x < m.nd) {
                const int jo = uo / ND, lo = uo - (uo / ND) * ND;
                gadd(out + ((fb + jo) * nc + sV[qo] + lo) * L.ndp + L.x, static_cast<double>(v[e]));
            }
        }
    }
}

// Pass C: J_ab, J_cd (wave 0), K_ac, K_bc (the other waves) over runs of
// equal ket shell c, and the D-order copy of the tiles for pass D.
//
// One-pass form (OP): the K waves also take K_ad and K_bd, so there is no
// pass D and no copy.  Over a run of equal c their density operands D_bc
// and D_ac are fixed (loaded once per chunk) while the output block moves
// with d; so, like J_cd, they are contracted with one output row per
// (quartet, bra function, d function), which fills the matrix-core rows,
// and each row is added to K as it is finished.
template <int LA, int LB, int LC, int LD, typename TT, bool G16, bool OP = false>
__global__ __launch_bounds__(192) __attribute__((amdgpu_waves_per_eu(DigShape<LA, LB, LC, LD>::WAVES_C)))
void k_digest_c(DigestArgs a) {
    using S = DigShape<LA, LB, LC, LD>;
    constexpr int NA = S::NA, NB = S::NB, NC = S::NC, ND = S::ND, NF = S::NF, NAB = S::NAB, NCD = S::NCD;
    constexpr int QB = S::QB, QBP = S::QBP;
    constexpr int MJ = S::MJ, M2 = S::M2, KJ2 = S::KJ2, M3 = S::M3, M4 = S::M4, NACC = S::NACC_C;
    using R = TT;               // compute type: FP64 tier in FP64, FP32 tier in FP32
    using MM = DigMma<R>;
    __shared__ R sT[NF * QBP];
    __shared__ int sV[QB];
    __shared__ int sP[QB];
    __shared__ int sO[QB];

    int p0 = 0, plen = 0, grp = 0;
    const DigItem* itp = dig_task(a, p0, plen, grp);
    if (!itp) return;
    const DigItem it = *itp;
    const int wave = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
    const int c16 = lane & 15, r4 = lane >> 4;
    const MolDesc m = load_mol(a.mols, a.mol0, it.mol);
    const DigLane<R> L(m, G16 ? grp * 16 + c16 : grp * 8 + (c16 & 7), G16 ? wave == 2 : c16 >= 8);
    const long long nc = m.nc;
    // FP64 tier: the K waves on 4 x 4 blocks (4-row tiles of K_ac and K_bc),
    // with their own lane map: four densities per block, or with 8-density
    // groups the D contraction on blocks 0, 1 and the D^T one on 2, 3
    constexpr bool K4 = !OP && sizeof(TT) == 8 && dig_c4(LA, LB, LC, LD);
    constexpr int T3 = (NA * NC + 3) / 4, T4 = (NB * NC + 3) / 4, NT4 = K4 ? T3 + T4 : 1;
    const int blk4 = Mfma4::block(lane), u4 = Mfma4::u(lane);
    const int xb4 = G16 ? grp * 16 + 4 * blk4 + Mfma4::bcol(u4) : grp * 8 + 4 * (blk4 & 1) + Mfma4::bcol(u4);
    const int xc4 = G16 ? grp * 16 + 4 * blk4 + Mfma4::ccol(u4) : grp * 8 + 4 * (blk4 & 1) + Mfma4::ccol(u4);
    const bool tr4 = G16 ? wave == 2 : blk4 >= 2;
    const DigLane<R> L4(m, K4 ? xb4 : 0, K4 && tr4);
    int frow4[NT4];
    double acc4[NT4];
#pragma unroll
    for (int t = 0; t < NT4; ++t) {
        frow4[t] = 0;
        acc4[t] = 0.0;
        if (K4 && wave != 0) {
            const int r = 4 * (t < T3 ? t : t - T3) + Mfma4::arow(u4);
            if (t < T3 && r < NA * NC) frow4[t] = (r / NC) * NB * NCD + (r % NC) * ND;
            if (t >= T3 && r < NB * NC) frow4[t] = (r / NC) * NCD + (r % NC) * ND;
        }
    }
    const PairInfo& P = m.pairs[it.bra];
    const int fa = P.fa, fb = P.fb, sa = P.sa, sb = P.sb;
    const gptr<const TT> tile = glob(static_cast<const TT*>(a.tiles)) + it.tile_off;
    const long long nq = it.chunk_n, qrel = it.blk0 - it.chunk_q0;
    const gptr<const long long> kin = glob(reinterpret_cast<const long long*>(it.kin)) + it.blk0;
    const gptr<const int> posl = glob(it.pos) + it.blk0;
    const bool jrole = wave == 0;

    // symmetrized densities of the lane's column (8-density groups: columns 0-7 only)
    const bool jcol = G16 || c16 < 8;
    const gptr<const R> dsx = glob(MM::dsym(m)) + L.x;
    // J_cd's B operand, fixed for the task: D^S_ab at k-row ij = 4 t + r4
    R sab[KJ2];
    {
        const long long u0 = m.ds_off[sa * m.ns + sb];
#pragma unroll
        for (int t = 0; t < KJ2; ++t) {
            const int ij = 4 * t + r4;
            sab[t] = (jrole && a.want_j && ij < NAB && jcol) ? dsx[(u0 + ij) * L.ndp] : R(0);
        }
    }
    // tile row of this lane's A operand in each accumulator tile of its role
    int frow[NACC];
#pragma unroll
    for (int t = 0; t < NACC; ++t) {
        frow[t] = 0;
        if (jrole) {
            const int r = t * 16 + c16;
            if (t < MJ && r < NAB) frow[t] = r * NCD;
        } else if (t < M3) {
            const int r = t * 16 + c16;
            if (r < NA * NC) frow[t] = (r / NC) * NB * NCD + (r % NC) * ND;
        } else if (t < M3 + M4) {
            const int r = (t - M3) * 16 + c16;
            if (r < NB * NC) frow[t] = (r / NC) * NCD + (r % NC) * ND;
        }
    }
    DigAcc<R> acc[NACC];
#pragma unroll
    for (int t = 0; t < NACC; ++t) acc[t].zero();

    const int pend = p0 + plen;
    for (int p = p0; p < pend;) {
        int2 kv;
        bool more;
        const int n = dig_chunk<QB>(kin, p, pend, lane, 0, kv, more);
        const int fc = __shfl(kv.y & 0xffff, 0);
        // fold weight of the lane's quartet (0 past the chunk), applied to the staged tile
        const R wl = lane < n ? static_cast<R>(fold_weight(sa, sb, kv.x & 0xffff, kv.x >> 16)) : R(0);
        if (wave == 0 && lane < QB) {
            sV[lane] = lane < n ? kv.y >> 16 : fc;
            sP[lane] = lane < n ? posl[p + lane] : 0;
            // first packed D^S unit of the quartet's ket pair (c, d)
            sO[lane] = lane < n && a.want_j ? m.ds_off[(kv.x & 0xffff) * m.ns + (kv.x >> 16)] : 0;
        }
        // tile loads do not wait for the scan: positions past the run get weight 0
        for (int base = 0; base < NF * QB; base += static_cast<int>(blockDim.x)) {
            const int idx = base + static_cast<int>(threadIdx.x);
            const int f = idx / QB, qb = idx - (idx / QB) * QB;
            R t = R(0);
            if (idx < NF * QB && p + qb < pend) t = tile[f * nq + qrel + p + qb];
            const R w = __shfl(wl, qb);
            if (idx < NF * QB) sT[f * QBP + qb] = w * t;
        }
        lds_barrier();
        if (!OP && a.want_k && grp == 0) {
            const gptr<TT> cp = glob(static_cast<TT*>(a.dcopy)) + it.tile_off;
            for (int idx = static_cast<int>(threadIdx.x); idx < n * NF; idx += static_cast<int>(blockDim.x)) {
                const int qb = idx / NF, f = idx - (idx / NF) * NF;
                cp[(qrel + sP[qb]) * NF + f] = static_cast<TT>(sT[f * QBP + qb]);
            }
        }
        const int nquad = (n + 3) >> 2;
        if (jrole) {
            if (a.want_j) {
                // J_ab: contraction over (d in run, k, l)
                for (int s = 0; s < nquad; ++s) {
                    const int qb = 4 * s + r4;
                    const long long u = sO[qb];
                    // the quad's B operands first, so their loads are in flight together:
                    // the packed D^S record of the ket pair
                    R bv[NCD];
#pragma unroll
                    for (int v = 0; v < NCD; ++v) bv[v] = jcol ? dsx[(u + v) * L.ndp] : R(0);
#pragma unroll
                    for (int v = 0; v < NCD; ++v)
#pragma unroll
                        for (int t = 0; t < MJ; ++t)
                            acc[t].a = MM::step(sT[(frow[t] + v) * QBP + qb], bv[v], acc[t].a);
                }
#pragma unroll
                for (int t = 0; t < MJ; ++t) acc[t].fold();
                // J_cd: one output row per (quartet, k, l), contraction over (i, j)
                for (int mt = 0; mt < M2; ++mt) {
                    if (mt * 16 >= n * NCD) break;
                    const int r = mt * 16 + c16;
                    const int qa = r < QB * NCD ? r / NCD : 0, va = r < QB * NCD ? r - (r / NCD) * NCD : 0;
                    typename MM::V cd = {0, 0, 0, 0};
#pragma unroll
                    for (int t = 0; t < KJ2; ++t) {
                        const int ij = 4 * t + r4 < NAB ? 4 * t + r4 : NAB - 1;
                        cd = MM::step(sT[(ij * NCD + va) * QBP + qa], sab[t], cd);
                    }
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        double v = static_cast<double>(cd[e]);
                        if constexpr (!G16) v += __shfl_xor(v, 8);
                        const int mo = mt * 16 + MM::row(e, r4);
                        const int qo = mo / NCD, vo = mo - (mo / NCD) * NCD;
                        if (qo < n && L.x < m.nd && !L.tr) {
                            const int k = vo / ND, l = vo - (vo / ND) * ND;
                            gadd(m.J + ((fc + k) * nc + sV[qo] + l) * L.ndp + L.x, v);
                        }
                    }
                }
            }
        } else if (K4 && a.want_k) {
            const int ak = Mfma4::ak(u4), bk = Mfma4::bk(u4), crow = Mfma4::crow(u4);
            for (int s = 0; s < nquad; ++s) {
                const int qa = 4 * s + ak;                  // A's quartet (k index)
                const long long V0 = sV[4 * s + bk];        // B's quartet: its d functions
                R b3[NB * ND], b4[NA * ND];
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int l = 0; l < ND; ++l) b3[j * ND + l] = L4.dk(fb + j, V0 + l);
#pragma unroll
                for (int i = 0; i < NA; ++i)
#pragma unroll
                    for (int l = 0; l < ND; ++l) b4[i * ND + l] = L4.dk(fa + i, V0 + l);
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int l = 0; l < ND; ++l)
#pragma unroll
                        for (int t = 0; t < T3; ++t)
                            acc4[t] = Mfma4::step(sT[(frow4[t] + j * NCD + l) * QBP + qa], b3[j * ND + l], acc4[t]);
#pragma unroll
                for (int i = 0; i < NA; ++i)
#pragma unroll
                    for (int l = 0; l < ND; ++l)
#pragma unroll
                        for (int t = T3; t < NT4; ++t)
                            acc4[t] = Mfma4::step(sT[(frow4[t] + i * NB * NCD + l) * QBP + qa], b4[i * ND + l], acc4[t]);
            }
            if (!more) {
                double* const out = tr4 ? m.KT : m.K;
#pragma unroll
                for (int t = 0; t < NT4; ++t) {
                    const bool ac = t < T3;
                    const int r = 4 * (ac ? t : t - T3) + crow;
                    if (r < (ac ? NA * NC : NB * NC) && xc4 < m.nd) {
                        const long long row = (ac ? fa : fb) + r / NC, col = fc + r % NC;
                        gadd(out + (row * nc + col) * L4.ndp + xc4, acc4[t]);
                    }
                    acc4[t] = 0.0;
                }
            }
        } else if (a.want_k) {
            for (int s = 0; s < nquad; ++s) {
                const int qb = 4 * s + r4;
                const long long V0 = sV[qb];
                // the quad's B operands first: D_bd for K_ac, D_ad for K_bc
                R b3[NB * ND], b4[NA * ND];
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int l = 0; l < ND; ++l) b3[j * ND + l] = L.dk(fb + j, V0 + l);
#pragma unroll
                for (int i = 0; i < NA; ++i)
#pragma unroll
                    for (int l = 0; l < ND; ++l) b4[i * ND + l] = L.dk(fa + i, V0 + l);
                // K_ac: contraction over (j, l)
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int l = 0; l < ND; ++l)
#pragma unroll
                        for (int t = 0; t < M3; ++t)
                            acc[t].a = MM::step(sT[(frow[t] + j * NCD + l) * QBP + qb], b3[j * ND + l], acc[t].a);
                // K_bc: contraction over (i, l)
#pragma unroll
                for (int i = 0; i < NA; ++i)
#pragma unroll
                    for (int l = 0; l < ND; ++l)
#pragma unroll
                        for (int t = M3; t < M3 + M4; ++t)
                            acc[t].a = MM::step(sT[(frow[t] + i * NB * NCD + l) * QBP + qb], b4[i * ND + l], acc[t].a);
            }
#pragma unroll
            for (int t = 0; t < M3 + M4; ++t) acc[t].fold();
            if constexpr (OP) dig_kd_rows<LA, LB, LC, LD, QB, R>(m, L, r4, c16, sT, sV, n, fa, fb, fc);
            if (!more) {
#pragma unroll
                for (int t = 0; t < M3; ++t)
                    dig_flush_k<NA * NC>(m, L, r4, acc[t], t, [&](int mo, long long& row, long long& col) {
                        row = fa + mo / NC;
                        col = fc + mo % NC;
                    });
#pragma unroll
                for (int t = M3; t < M3 + M4; ++t)
                    dig_flush_k<NB * NC>(m, L, r4, acc[t], t - M3, [&](int mo, long long& row, long long& col) {
                        row = fb + mo / NC;
                        col = fc + mo % NC;
                    });
            }
        }
        p += n;
        lds_barrier();
    }
    if (jrole && a.want_j) {
#pragma unroll
        for (int t = 0; t < MJ; ++t)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                double v = acc[t].get(e);
                if constexpr (!G16) v += __shfl_xor(v, 8);
                const int mo = t * 16 + MM::row(e, r4);
                if (mo < NAB && L.x < m.nd && !L.tr) {
                    const int i = mo / NB, j = mo - (mo / NB) * NB;
                    gadd(m.J + ((fa + i) * nc + fb + j) * L.ndp + L.x, v);
                }
            }
    }
}

// Pass D: K_ad and K_bd over runs of equal ket shell d, from the D-order
// copy; one wave per K contraction (D, and D^T when 16 densities).
template <int LA, int LB, int LC, int LD, typename TT, bool G16>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(DigShape<LA, LB, LC, LD>::WAVES_D)))
void k_digest_d(DigestArgs a) {
    using S = DigShape<LA, LB, LC, LD>;
    constexpr int NA = S::NA, NB = S::NB, NC = S::NC, ND = S::ND, NF = S::NF, NCD = S::NCD;
    constexpr int QB = S::QB_D, QBP = S::QBP_D;
    constexpr int M5 = S::M5, M6 = S::M6, NACC = S::NACC_D;
    using R = TT;
    using MM = DigMma<R>;
    __shared__ R sT[NF * QBP];
    __shared__ int sV[QB];

    int p0 = 0, plen = 0, grp = 0;
    const DigItem* itp = dig_task(a, p0, plen, grp);
    if (!itp) return;
    const DigItem it = *itp;
    const int wave = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
    const int c16 = lane & 15, r4 = lane >> 4;
    const MolDesc m = load_mol(a.mols, a.mol0, it.mol);
    const DigLane<R> L(m, G16 ? grp * 16 + c16 : grp * 8 + (c16 & 7), G16 ? wave == 1 : c16 >= 8);
    const PairInfo& P = m.pairs[it.bra];
    const int fa = P.fa, fb = P.fb;
    const gptr<const TT> cp = glob(static_cast<const TT*>(a.dcopy)) + it.tile_off;
    const long long qrel = it.blk0 - it.chunk_q0;
    const gptr<const long long> kin = glob(reinterpret_cast<const long long*>(it.kin)) + it.blk0;

    int frow[NACC];
#pragma unroll
    for (int t = 0; t < NACC; ++t) {
        frow[t] = 0;
        if (t < M5) {
            const int r = t * 16 + c16;
            if (r < NA * ND) frow[t] = (r / ND) * NB * NCD + r % ND;
        } else {
            const int r = (t - M5) * 16 + c16;
            if (r < NB * ND) frow[t] = (r / ND) * NCD + r % ND;
        }
    }
    DigAcc<R> acc[NACC];
#pragma unroll
    for (int t = 0; t < NACC; ++t) acc[t].zero();

    const int pend = p0 + plen;
    for (int p = p0; p < pend;) {
        int2 kv;
        bool more;
        const int n = dig_chunk<QB>(kin, p, pend, lane, 16, kv, more);
        const int fd = __shfl(kv.y >> 16, 0), fc0 = __shfl(kv.y & 0xffff, 0);
        if (wave == 0 && lane < QB) sV[lane] = lane < n ? kv.y & 0xffff : fc0;
        for (int base = 0; base < NF * QB; base += static_cast<int>(blockDim.x)) {
            const int idx = base + static_cast<int>(threadIdx.x);
            const int qb = idx / NF, f = idx - (idx / NF) * NF;
            R t = R(0);
            if (idx < NF * QB && p + qb < pend) t = cp[(qrel + p + qb) * NF + f];
            if (idx < NF * QB) sT[f * QBP + qb] = qb < n ? t : R(0);
        }
        lds_barrier();
        const int nquad = (n + 3) >> 2;
        for (int s = 0; s < nquad; ++s) {
            const int qb = 4 * s + r4;
            const long long V0 = sV[qb];
            // the quad's B operands first: D_bc for K_ad, D_ac for K_bd
            R b5[NB * NC], b6[NA * NC];
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int k = 0; k < NC; ++k) b5[j * NC + k] = L.dk(fb + j, V0 + k);
#pragma unroll
            for (int i = 0; i < NA; ++i)
#pragma unroll
                for (int k = 0; k < NC; ++k) b6[i * NC + k] = L.dk(fa + i, V0 + k);
            // K_ad: contraction over (j, k)
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int k = 0; k < NC; ++k)
#pragma unroll
                    for (int t = 0; t < M5; ++t)
                        acc[t].a = MM::step(sT[(frow[t] + j * NCD + k * ND) * QBP + qb], b5[j * NC + k], acc[t].a);
            // K_bd: contraction over (i, k)
#pragma unroll
            for (int i = 0; i < NA; ++i)
#pragma unroll
                for (int k = 0; k < NC; ++k)
#pragma unroll
                    for (int t = M5; t < M5 + M6; ++t)
                        acc[t].a = MM::step(sT[(frow[t] + i * NB * NCD + k * ND) * QBP + qb], b6[i * NC + k], acc[t].a);
        }
#pragma unroll
        for (int t = 0; t < NACC; ++t) acc[t].fold();
        if (!more) {
#pragma unroll
            for (int t = 0; t < M5; ++t)
                dig_flush_k<NA * ND>(m, L, r4, acc[t], t, [&](int mo, long long& row, long long& col) {
                    row = fa + mo / ND;
                    col = fd + mo % ND;
                });
#pragma unroll
            for (int t = M5; t < M5 + M6; ++t)
                dig_flush_k<NB * ND>(m, L, r4, acc[t], t - M5, [&](int mo, long long& row, long long& col) {
                    row = fb + mo / ND;
                    col = fd + mo % ND;
                });
        }
        p += n;
        lds_barrier();
    }
}

// Pass D on 4 x 4 blocks (FP64 tier): the same contractions as k_digest_d,
// with output tiles of 4 rows instead of 16.  The outputs of pass D (K_ad:
// NA ND rows, K_bd: NB ND rows) are short for most classes, so 16-row tiles
// leave most of each matrix-core operation idle; 4-row tiles waste at most
// three rows.  The four blocks of a wave take four densities each (16-density
// groups) or, with 8-density groups, the D contraction (blocks 0, 1) and the
// D^T one (blocks 2, 3).
template <int LA, int LB, int LC, int LD, bool G16>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(DigShape<LA, LB, LC, LD>::WAVES_D)))
void k_digest_d4(DigestArgs a) {
    using S = DigShape<LA, LB, LC, LD>;
    constexpr int NA = S::NA, NB = S::NB, NC = S::NC, ND = S::ND, NF = S::NF, NCD = S::NCD;
    constexpr int QB = S::QB_D, QBP = S::QBP_D;
    constexpr int T5 = (NA * ND + 3) / 4, T6 = (NB * ND + 3) / 4, NT = T5 + T6;   // 4-row output tiles
    __shared__ double sT[NF * QBP];
    __shared__ int sV[QB];

    int p0 = 0, plen = 0, grp = 0;
    const DigItem* itp = dig_task(a, p0, plen, grp);
    if (!itp) return;
    const DigItem it = *itp;
    const int wave = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
    const int blk = Mfma4::block(lane), u = Mfma4::u(lane);
    const int arow = Mfma4::arow(u), ak = Mfma4::ak(u), bk = Mfma4::bk(u);
    const int crow = Mfma4::crow(u);
    // density of the lane's B column and of its output column, and the form
    const int xb = G16 ? grp * 16 + 4 * blk + Mfma4::bcol(u) : grp * 8 + 4 * (blk & 1) + Mfma4::bcol(u);
    const int xc = G16 ? grp * 16 + 4 * blk + Mfma4::ccol(u) : grp * 8 + 4 * (blk & 1) + Mfma4::ccol(u);
    const bool tr = G16 ? wave == 1 : blk >= 2;
    const MolDesc m = load_mol(a.mols, a.mol0, it.mol);
    const DigLane<double> L(m, xb, tr);
    double* const out = tr ? m.KT : m.K;
    const PairInfo& P = m.pairs[it.bra];
    const int fa = P.fa, fb = P.fb;
    const gptr<const double> cp = glob(static_cast<const double*>(a.dcopy)) + it.tile_off;
    const long long qrel = it.blk0 - it.chunk_q0;
    const gptr<const long long> kin = glob(reinterpret_cast<const long long*>(it.kin)) + it.blk0;

    // tile row of this lane's A operand: K_ad rows (i, l), K_bd rows (j, l)
    int frow[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        frow[t] = 0;
        if (t < T5) {
            const int r = 4 * t + arow;
            if (r < NA * ND) frow[t] = (r / ND) * NB * NCD + r % ND;
        } else {
            const int r = 4 * (t - T5) + arow;
            if (r < NB * ND) frow[t] = (r / ND) * NCD + r % ND;
        }
    }
    double acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = 0.0;

    const int pend = p0 + plen;
    for (int p = p0; p < pend;) {
        int2 kv;
        bool more;
        const int n = dig_chunk<QB>(kin, p, pend, lane, 16, kv, more);
        const int fd = __shfl(kv.y >> 16, 0), fc0 = __shfl(kv.y & 0xffff, 0);
        if (wave == 0 && lane < QB) sV[lane] = lane < n ? kv.y & 0xffff : fc0;
        for (int base = 0; base < NF * QB; base += static_cast<int>(blockDim.x)) {
            const int idx = base + static_cast<int>(threadIdx.x);
            const int qb = idx / NF, f = idx - (idx / NF) * NF;
            double t = 0.0;
            if (idx < NF * QB && p + qb < pend) t = cp[(qrel + p + qb) * NF + f];
            if (idx < NF * QB) sT[f * QBP + qb] = qb < n ? t : 0.0;
        }
        lds_barrier();
        const int nquad = (n + 3) >> 2;
        for (int s = 0; s < nquad; ++s) {
            const int qa = 4 * s + ak;                  // A's quartet (k index)
            const long long V0 = sV[4 * s + bk];        // B's quartet: its c functions
            double b5[NB * NC], b6[NA * NC];
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int k = 0; k < NC; ++k) b5[j * NC + k] = L.dk(fb + j, V0 + k);
#pragma unroll
            for (int i = 0; i < NA; ++i)
#pragma unroll
                for (int k = 0; k < NC; ++k) b6[i * NC + k] = L.dk(fa + i, V0 + k);
            // K_ad: contraction over (j, k)
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int k = 0; k < NC; ++k)
#pragma unroll
                    for (int t = 0; t < T5; ++t)
                        acc[t] = Mfma4::step(sT[(frow[t] + j * NCD + k * ND) * QBP + qa], b5[j * NC + k], acc[t]);
            // K_bd: contraction over (i, k)
#pragma unroll
            for (int i = 0; i < NA; ++i)
#pragma unroll
                for (int k = 0; k < NC; ++k)
#pragma unroll
                    for (int t = T5; t < NT; ++t)
                        acc[t] = Mfma4::step(sT[(frow[t] + i * NB * NCD + k * ND) * QBP + qa], b6[i * NC + k], acc[t]);
        }
        if (!more) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const bool ad = t < T5;
                const int r = 4 * (ad ? t : t - T5) + crow;
                if (r < (ad ? NA * ND : NB * ND) && xc < m.nd) {
                    const long long row = (ad ? fa : fb) + r / ND, col = fd + r % ND;
                    gadd(out + (row * m.nc + col) * L.ndp + xc, acc[t]);
                }
                acc[t] = 0.0;
            }
        }
        p += n;
        lds_barrier();
    }
}

}  // namespace jk
