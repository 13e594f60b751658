// Digestion of ERI tiles against stacked densities on the FP64 matrix cores.
//
// For a canonical quartet (ab|cd) with fold weight w (Sect. 3, Eq.
// (quartet_scatter)) and every density x of the batch, digestion adds
//   J_ab += w I D^S_cd,  J_cd += w I D^S_ab          (D^S = D + D^T)
//   K_ac += w I D_bd,  K_bc += w I D_ad,  K_ad += w I D_bc,  K_bd += w I D_ac
// and the same four with D^T into KT (the transposed contributions), so that
// J = Jc + Jc^T and K = Kc + KTc^T hold for non-symmetric D (Eq. (jkbuild)).
//
// Each update is a contraction of the tile with a gather of the densities,
// stacked along the MFMA N dimension (16 densities, or 8 densities and their
// transposes).  One wave owns one task: a piece of the quartets of one bra
// pair and one density group.  The quartets of a bra pair sit in the class
// list in (c, d) order, so the updates whose output is indexed by c (J_ab,
// K_ac, K_bc) run over runs of equal c and keep their sums in the MFMA
// accumulators until the run ends; J_cd is written per quartet.  Pass C
// walks that order and also writes each tile, quartet-major, at its position
// in the (d, c) order; pass D walks the copy in runs of equal d for K_ad and
// K_bd.  Tiles are staged in LDS per chunk of QB quartets of one run.
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

// Completes a wave's LDS writes before its lanes read each other's values.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <int LA, int LB, int LC, int LD>
struct DigShape {
    static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    static constexpr int NF = NA * NB * NC * ND, NAB = NA * NB, NCD = NC * ND;
    static constexpr int QB = dig_qb(NF), QBP = QB + 1, WPB = dig_wpb(NF);
};

// The task of the calling wave.  Items are dealt to the XCDs round-robin
// (item i on XCD i % 8, workgroup b runs on XCD b % 8), so the density groups
// of one item share an L2; on its XCD an item owns tasks [kstart, kstart +
// ngroups).
__device__ __forceinline__ const DigItem* dig_task(const DigestArgs& a, int wpb, int& grp) {
    const int b = blockIdx.x, xcd = b & 7;
    const int task = (b >> 3) * wpb + static_cast<int>(threadIdx.x >> 6);
    if (xcd >= a.nitems) return nullptr;
    int lo = 0, hi = (a.nitems - 1 - xcd) >> 3;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.items[xcd + 8 * mid].kstart <= task) lo = mid;
        else hi = mid - 1;
    }
    const DigItem* it = a.items + xcd + 8 * lo;
    grp = task - it->kstart;
    if (grp < 0 || grp >= it->ngroups) return nullptr;
    return it;
}

// Lane geometry of a density group.  G16: column c of the MFMA output is
// density 16 g + c; the D and D^T contractions use separate accumulators.
// Otherwise columns 0-7 are densities 8 g + c with D and columns 8-15 the
// same densities with D^T.
template <bool G16>
struct DigLane {
    int x;              // density of this lane's column
    bool tr;            // column takes D^T (8-density form)
    long long sRow;     // stride of a density row, nc * ndp
    long long sF, sV;   // strides of (F, V) in the lane's element D[F][V] or D[V][F]
    long long ndp;
    const double* Dx;   // D + x
    __device__ DigLane(const MolDesc& m, int grp, int c16) {
        ndp = m.ndp;
        sRow = static_cast<long long>(m.nc) * ndp;
        x = G16 ? grp * 16 + c16 : grp * 8 + (c16 & 7);
        tr = !G16 && c16 >= 8;
        sF = tr ? ndp : sRow;
        sV = tr ? sRow : ndp;
        Dx = m.D + x;
    }
    __device__ __forceinline__ double d(long long r, long long c) const { return Dx[r * sRow + c * ndp]; }
    // 8-density form: D[F][V] in columns 0-7, D[V][F] in columns 8-15
    __device__ __forceinline__ double dh(long long F, long long V) const { return Dx[F * sF + V * sV]; }
};

// Fold weight of a canonical quartet: 1/2 for a = b, for c = d and for
// (ab) = (cd).
__device__ __forceinline__ double fold_weight(const PairInfo& P, int bra, const PairInfo& Q, int ket) {
    return (P.sa == P.sb ? 0.5 : 1.0) * (Q.sa == Q.sb ? 0.5 : 1.0) * (bra == ket ? 0.5 : 1.0);
}

// Adds a finished K accumulator tile into K (D contraction) and KT (D^T
// contraction); rowmap turns an output row into its (row, column) function.
template <bool G16, int NT, int NROW, class RowMap>
__device__ __forceinline__ void dig_flush_k(const MolDesc& m, const DigLane<G16>& L, int r4, v4d (&acc)[NT],
                                            int mt, RowMap rowmap) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int mo = mt * 16 + 4 * r + r4;
        if (mo < NROW && L.x < m.nd) {
            long long row, col;
            rowmap(mo, row, col);
            const long long off = (row * m.nc + col) * L.ndp + L.x;
            if constexpr (G16) {
                unsafeAtomicAdd(m.K + off, acc[0][r]);
                unsafeAtomicAdd(m.KT + off, acc[1][r]);
            } else {
                unsafeAtomicAdd((L.tr ? m.KT : m.K) + off, acc[0][r]);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
}

// Pass C: J_ab, J_cd, K_ac, K_bc over runs of equal ket shell c, and the
// D-order copy of the tiles for pass D.
template <int LA, int LB, int LC, int LD, typename TT, bool G16>
__global__ __launch_bounds__((64 * DigShape<LA, LB, LC, LD>::WPB)) void k_digest_c(DigestArgs a) {
    using S = DigShape<LA, LB, LC, LD>;
    constexpr int NA = S::NA, NB = S::NB, NC = S::NC, ND = S::ND, NF = S::NF, NAB = S::NAB, NCD = S::NCD;
    constexpr int QB = S::QB, QBP = S::QBP, WPB = S::WPB;
    constexpr int NT = G16 ? 2 : 1;
    constexpr int MJ = (NAB + 15) / 16, M3 = (NA * NC + 15) / 16, M4 = (NB * NC + 15) / 16;
    constexpr int KJ2 = (NAB + 3) / 4, M2 = (QB * NCD + 15) / 16;
    __shared__ double sT_all[WPB][NF * QBP];
    __shared__ double sW_all[WPB][QB];
    __shared__ int sV_all[WPB][QB];
    __shared__ int sP_all[WPB][QB];

    int grp = 0;
    const DigItem* itp = dig_task(a, WPB, grp);
    if (!itp) return;
    const DigItem it = *itp;
    const int wave = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
    const int c16 = lane & 15, r4 = lane >> 4;
    double* __restrict__ sT = sT_all[wave];
    double* __restrict__ sW = sW_all[wave];
    int* __restrict__ sV = sV_all[wave];
    int* __restrict__ sP = sP_all[wave];
    const MolDesc& m = a.mols ? a.mols[it.mol] : a.mol0;
    const DigLane<G16> L(m, grp, c16);
    const long long nc = m.nc;
    const int2* __restrict__ ql = it.quartets + it.blk0;
    const int bra = ql[0].x;
    const PairInfo& P = m.pairs[bra];
    const int fa = P.fa, fb = P.fb;
    const TT* __restrict__ tile = static_cast<const TT*>(a.tiles) + it.tile_off;
    const long long nq = it.chunk_n, qrel = it.blk0 - it.chunk_q0;

    // J_cd's B operand, fixed for the block: D^S_ab at k-row ij = 4 t + r4
    double sab[KJ2];
#pragma unroll
    for (int t = 0; t < KJ2; ++t) {
        const int ij = 4 * t + r4;
        sab[t] = 0.0;
        if (a.want_j && ij < NAB) {
            const int i = ij / NB, j = ij - (ij / NB) * NB;
            if constexpr (G16) sab[t] = L.d(fa + i, fb + j) + L.d(fb + j, fa + i);
            else sab[t] = L.dh(fa + i, fb + j);
        }
    }
    // tile row of this lane's A operand in each M tile
    int fJ[MJ], f3[M3], f4[M4];
#pragma unroll
    for (int mt = 0; mt < MJ; ++mt) {
        const int r = mt * 16 + c16;
        fJ[mt] = (r < NAB ? r : 0) * NCD;
    }
#pragma unroll
    for (int mt = 0; mt < M3; ++mt) {
        const int r = mt * 16 + c16;
        f3[mt] = r < NA * NC ? (r / NC) * NB * NCD + (r % NC) * ND : 0;
    }
#pragma unroll
    for (int mt = 0; mt < M4; ++mt) {
        const int r = mt * 16 + c16;
        f4[mt] = r < NB * NC ? (r / NC) * NCD + (r % NC) * ND : 0;
    }
    v4d accJ[MJ], acc3[M3][NT], acc4[M4][NT];
#pragma unroll
    for (int mt = 0; mt < MJ; ++mt) accJ[mt] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int mt = 0; mt < M3; ++mt)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc3[mt][t] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int mt = 0; mt < M4; ++mt)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc4[mt][t] = v4d{0.0, 0.0, 0.0, 0.0};

    const int pend = it.p0 + it.plen;
    for (int p = it.p0; p < pend;) {
        // chunk: up to QB quartets from p on with the ket shell c of quartet p
        const bool in = lane < QB && p + lane < pend;
        int ket = 0, csh = -1;
        if (in) {
            ket = ql[p + lane].y;
            csh = m.pairs[ket].sa;
        }
        const int c0 = __shfl(csh, 0);
        const unsigned long long same = __ballot(in && csh == c0);
        const int n = __builtin_ctzll(~same);
        bool more = false;
        if (n == QB && p + n < pend) more = m.pairs[ql[p + n].y].sa == c0;
        const int fc = m.pairs[__shfl(ket, 0)].fa;
        if (lane < QB) {
            double w = 0.0;
            int fd = fc, pos = 0;
            if (lane < n) {
                const PairInfo& Q = m.pairs[ket];
                w = fold_weight(P, bra, Q, ket);
                fd = Q.fb;
                pos = it.order[it.blk0 + p + lane];
            }
            sW[lane] = w;
            sV[lane] = fd;
            sP[lane] = pos;
        }
        for (int idx = lane; idx < NF * QB; idx += 64) {
            const int f = idx / QB, qb = idx - (idx / QB) * QB;
            sT[f * QBP + qb] = qb < n ? static_cast<double>(tile[f * nq + qrel + p + qb]) : 0.0;
        }
        wave_lds_sync();
        if (a.want_k && grp == 0) {
            TT* __restrict__ cp = static_cast<TT*>(a.dcopy) + it.tile_off;
            for (int idx = lane; idx < n * NF; idx += 64) {
                const int qb = idx / NF, f = idx - (idx / NF) * NF;
                cp[(qrel + sP[qb]) * NF + f] = static_cast<TT>(sT[f * QBP + qb]);
            }
        }
        const int nquad = (n + 3) >> 2;
        if (a.want_j) {
            // J_ab: contraction over (d in run, k, l)
            for (int s = 0; s < nquad; ++s) {
                const int qb = 4 * s + r4;
                const double w = sW[qb];
                const long long V0 = sV[qb];
#pragma unroll
                for (int k = 0; k < NC; ++k)
#pragma unroll
                    for (int l = 0; l < ND; ++l) {
                        double bv;
                        if constexpr (G16) bv = w * (L.d(fc + k, V0 + l) + L.d(V0 + l, fc + k));
                        else bv = w * L.dh(fc + k, V0 + l);
#pragma unroll
                        for (int mt = 0; mt < MJ; ++mt)
                            accJ[mt] = mfma_f64(sT[(fJ[mt] + k * ND + l) * QBP + qb], bv, accJ[mt]);
                    }
            }
            // J_cd: one output row per (quartet, k, l), contraction over (i, j)
            for (int mt = 0; mt < M2; ++mt) {
                if (mt * 16 >= n * NCD) break;
                const int r = mt * 16 + c16;
                const int qa = r < QB * NCD ? r / NCD : 0, va = r < QB * NCD ? r - (r / NCD) * NCD : 0;
                v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int t = 0; t < KJ2; ++t) {
                    const int ij = 4 * t + r4 < NAB ? 4 * t + r4 : NAB - 1;
                    acc = mfma_f64(sT[(ij * NCD + va) * QBP + qa], sab[t], acc);
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    double v = acc[e];
                    if constexpr (!G16) v += __shfl_xor(v, 8);
                    const int mo = mt * 16 + 4 * e + r4;
                    const int qo = mo / NCD, vo = mo - (mo / NCD) * NCD;
                    if (qo < n && L.x < m.nd && !L.tr) {
                        const int k = vo / ND, l = vo - (vo / ND) * ND;
                        unsafeAtomicAdd(m.J + ((fc + k) * nc + sV[qo] + l) * L.ndp + L.x, sW[qo] * v);
                    }
                }
            }
        }
        if (a.want_k) {
            for (int s = 0; s < nquad; ++s) {
                const int qb = 4 * s + r4;
                const double w = sW[qb];
                const long long V0 = sV[qb];
                // K_ac (+ KT): contraction over (j, l) with D_bd
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int l = 0; l < ND; ++l) {
                        double b0, b1 = 0.0;
                        if constexpr (G16) {
                            b0 = w * L.d(fb + j, V0 + l);
                            b1 = w * L.d(V0 + l, fb + j);
                        } else {
                            b0 = w * L.dh(fb + j, V0 + l);
                        }
#pragma unroll
                        for (int mt = 0; mt < M3; ++mt) {
                            const double av = sT[(f3[mt] + j * NCD + l) * QBP + qb];
                            acc3[mt][0] = mfma_f64(av, b0, acc3[mt][0]);
                            if constexpr (G16) acc3[mt][NT - 1] = mfma_f64(av, b1, acc3[mt][NT - 1]);
                        }
                    }
                // K_bc (+ KT): contraction over (i, l) with D_ad
#pragma unroll
                for (int i = 0; i < NA; ++i)
#pragma unroll
                    for (int l = 0; l < ND; ++l) {
                        double b0, b1 = 0.0;
                        if constexpr (G16) {
                            b0 = w * L.d(fa + i, V0 + l);
                            b1 = w * L.d(V0 + l, fa + i);
                        } else {
                            b0 = w * L.dh(fa + i, V0 + l);
                        }
#pragma unroll
                        for (int mt = 0; mt < M4; ++mt) {
                            const double av = sT[(f4[mt] + i * NB * NCD + l) * QBP + qb];
                            acc4[mt][0] = mfma_f64(av, b0, acc4[mt][0]);
                            if constexpr (G16) acc4[mt][NT - 1] = mfma_f64(av, b1, acc4[mt][NT - 1]);
                        }
                    }
            }
            if (!more) {
#pragma unroll
                for (int mt = 0; mt < M3; ++mt)
                    dig_flush_k<G16, NT, NA * NC>(m, L, r4, acc3[mt], mt, [&](int mo, long long& row, long long& col) {
                        row = fa + mo / NC;
                        col = fc + mo % NC;
                    });
#pragma unroll
                for (int mt = 0; mt < M4; ++mt)
                    dig_flush_k<G16, NT, NB * NC>(m, L, r4, acc4[mt], mt, [&](int mo, long long& row, long long& col) {
                        row = fb + mo / NC;
                        col = fc + mo % NC;
                    });
            }
        }
        p += n;
        wave_lds_sync();
    }
    if (a.want_j) {
#pragma unroll
        for (int mt = 0; mt < MJ; ++mt)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                double v = accJ[mt][e];
                if constexpr (!G16) v += __shfl_xor(v, 8);
                const int mo = mt * 16 + 4 * e + r4;
                if (mo < NAB && L.x < m.nd && !L.tr) {
                    const int i = mo / NB, j = mo - (mo / NB) * NB;
                    unsafeAtomicAdd(m.J + ((fa + i) * nc + fb + j) * L.ndp + L.x, v);
                }
            }
    }
}

// Pass D: K_ad and K_bd over runs of equal ket shell d, from the D-order copy.
template <int LA, int LB, int LC, int LD, typename TT, bool G16>
__global__ __launch_bounds__((64 * DigShape<LA, LB, LC, LD>::WPB)) void k_digest_d(DigestArgs a) {
    using S = DigShape<LA, LB, LC, LD>;
    constexpr int NA = S::NA, NB = S::NB, NC = S::NC, ND = S::ND, NF = S::NF, NCD = S::NCD;
    constexpr int QB = S::QB, QBP = S::QBP, WPB = S::WPB;
    constexpr int NT = G16 ? 2 : 1;
    constexpr int M5 = (NA * ND + 15) / 16, M6 = (NB * ND + 15) / 16;
    __shared__ double sT_all[WPB][NF * QBP];
    __shared__ double sW_all[WPB][QB];
    __shared__ int sV_all[WPB][QB];

    int grp = 0;
    const DigItem* itp = dig_task(a, WPB, grp);
    if (!itp) return;
    const DigItem it = *itp;
    const int wave = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
    const int c16 = lane & 15, r4 = lane >> 4;
    double* __restrict__ sT = sT_all[wave];
    double* __restrict__ sW = sW_all[wave];
    int* __restrict__ sV = sV_all[wave];
    const MolDesc& m = a.mols ? a.mols[it.mol] : a.mol0;
    const DigLane<G16> L(m, grp, c16);
    const int2* __restrict__ ql = it.quartets + it.blk0;
    const int* __restrict__ dord = it.order + it.blk0;
    const int bra = ql[0].x;
    const PairInfo& P = m.pairs[bra];
    const int fa = P.fa, fb = P.fb;
    const TT* __restrict__ cp = static_cast<const TT*>(a.dcopy) + it.tile_off;
    const long long qrel = it.blk0 - it.chunk_q0;

    int f5[M5], f6[M6];
#pragma unroll
    for (int mt = 0; mt < M5; ++mt) {
        const int r = mt * 16 + c16;
        f5[mt] = r < NA * ND ? (r / ND) * NB * NCD + r % ND : 0;
    }
#pragma unroll
    for (int mt = 0; mt < M6; ++mt) {
        const int r = mt * 16 + c16;
        f6[mt] = r < NB * ND ? (r / ND) * NCD + r % ND : 0;
    }
    v4d acc5[M5][NT], acc6[M6][NT];
#pragma unroll
    for (int mt = 0; mt < M5; ++mt)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc5[mt][t] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int mt = 0; mt < M6; ++mt)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc6[mt][t] = v4d{0.0, 0.0, 0.0, 0.0};

    const int pend = it.p0 + it.plen;
    for (int p = it.p0; p < pend;) {
        const bool in = lane < QB && p + lane < pend;
        int ket = 0, dsh = -1;
        if (in) {
            ket = ql[dord[p + lane]].y;
            dsh = m.pairs[ket].sb;
        }
        const int d0 = __shfl(dsh, 0);
        const unsigned long long same = __ballot(in && dsh == d0);
        const int n = __builtin_ctzll(~same);
        bool more = false;
        if (n == QB && p + n < pend) more = m.pairs[ql[dord[p + n]].y].sb == d0;
        const PairInfo& Q0 = m.pairs[__shfl(ket, 0)];
        const int fd = Q0.fb, fc0 = Q0.fa;
        if (lane < QB) {
            double w = 0.0;
            int fc = fc0;
            if (lane < n) {
                const PairInfo& Q = m.pairs[ket];
                w = fold_weight(P, bra, Q, ket);
                fc = Q.fa;
            }
            sW[lane] = w;
            sV[lane] = fc;
        }
        for (int idx = lane; idx < NF * QB; idx += 64) {
            const int qb = idx / NF, f = idx - (idx / NF) * NF;
            sT[f * QBP + qb] = qb < n ? static_cast<double>(cp[(qrel + p + qb) * NF + f]) : 0.0;
        }
        wave_lds_sync();
        const int nquad = (n + 3) >> 2;
        for (int s = 0; s < nquad; ++s) {
            const int qb = 4 * s + r4;
            const double w = sW[qb];
            const long long V0 = sV[qb];
            // K_ad (+ KT): contraction over (j, k) with D_bc
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    double b0, b1 = 0.0;
                    if constexpr (G16) {
                        b0 = w * L.d(fb + j, V0 + k);
                        b1 = w * L.d(V0 + k, fb + j);
                    } else {
                        b0 = w * L.dh(fb + j, V0 + k);
                    }
#pragma unroll
                    for (int mt = 0; mt < M5; ++mt) {
                        const double av = sT[(f5[mt] + j * NCD + k * ND) * QBP + qb];
                        acc5[mt][0] = mfma_f64(av, b0, acc5[mt][0]);
                        if constexpr (G16) acc5[mt][NT - 1] = mfma_f64(av, b1, acc5[mt][NT - 1]);
                    }
                }
            // K_bd (+ KT): contraction over (i, k) with D_ac
#pragma unroll
            for (int i = 0; i < NA; ++i)
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    double b0, b1 = 0.0;
                    if constexpr (G16) {
                        b0 = w * L.d(fa + i, V0 + k);
                        b1 = w * L.d(V0 + k, fa + i);
                    } else {
                        b0 = w * L.dh(fa + i, V0 + k);
                    }
#pragma unroll
                    for (int mt = 0; mt < M6; ++mt) {
                        const double av = sT[(f6[mt] + i * NB * NCD + k * ND) * QBP + qb];
                        acc6[mt][0] = mfma_f64(av, b0, acc6[mt][0]);
                        if constexpr (G16) acc6[mt][NT - 1] = mfma_f64(av, b1, acc6[mt][NT - 1]);
                    }
                }
        }
        if (!more) {
#pragma unroll
            for (int mt = 0; mt < M5; ++mt)
                dig_flush_k<G16, NT, NA * ND>(m, L, r4, acc5[mt], mt, [&](int mo, long long& row, long long& col) {
                    row = fa + mo / ND;
                    col = fd + mo % ND;
                });
#pragma unroll
            for (int mt = 0; mt < M6; ++mt)
                dig_flush_k<G16, NT, NB * ND>(m, L, r4, acc6[mt], mt, [&](int mo, long long& row, long long& col) {
                    row = fb + mo / ND;
                    col = fd + mo % ND;
                });
        }
        p += n;
        wave_lds_sync();
    }
}

}  // namespace jk
