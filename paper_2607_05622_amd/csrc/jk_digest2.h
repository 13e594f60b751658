// Digestion with wave-private tasks.
//
// The same contractions as jk_digest.h (passes C and D over the same work
// items, the same fold weights and flushes), but every wavefront owns one
// task -- a piece of one bra pair's quartets and one density group -- and
// performs every update of its pass itself: J_ab, J_cd and K_ac, K_bc with D
// and with D^T in pass C; K_ad, K_bd with D and with D^T in pass D.  A wave
// stages its own chunks in its own part of the workgroup's LDS, so waves
// never wait for one another: there are no workgroup barriers, and a wave
// stalled on its density gathers leaves the matrix cores to the other waves
// of its SIMD.  Four waves (four tasks) per workgroup, or two where a chunk
// needs more LDS.
#pragma once

#include "jk_digest.h"

namespace jk {

// Four waves (tasks) per workgroup.  A wave's chunk holds dig2_qb(NF)
// quartets, so that the four chunks fit in 64 KB of LDS and two workgroups
// (eight waves) share a CU; classes of more than 408 functions per quartet
// are not digested this way (their chunks would be too short).
constexpr int kDig2Waves = 4;

// Classes the wave-private kernels are compiled for.
__host__ __device__ constexpr bool dig2_class(int la, int lb, int lc, int ld, int nf) { return nf <= 408; }
__host__ __device__ constexpr int dig2_qb(int nf) {
    return nf <= 62 ? 32 : (nf <= 120 ? 16 : (nf <= 226 ? 8 : (nf <= 408 ? 4 : 0)));
}

// Orders the wave's LDS traffic: its stores before its later loads and its
// loads before later stores (no other wave touches this part of LDS).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// The task of wave `wave` of the calling workgroup: workgroup b runs on XCD
// b % 8 and its waves take tasks WPB (b / 8) .. WPB (b / 8) + WPB - 1 of
// that XCD.  Returns nullptr when idle.
template <int WPB>
__device__ __forceinline__ const DigItem* dig2_task(const DigestArgs& a, int wave, int& p0, int& plen, int& grp) {
    const int b = blockIdx.x, xcd = b & 7, task = (b >> 3) * WPB + wave;
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

// Adds a finished accumulator tile into dst[(row, col)] at density column x
// and clears it (rowmap: output row -> function pair).
template <int NROW, class RowMap>
__device__ __forceinline__ void dig2_flush(double* dst, long long nc, long long ndp, int x, bool live, int r4,
                                           v4d& acc, int mt, RowMap rowmap) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int mo = mt * 16 + 4 * r + r4;
        if (mo < NROW && live) {
            long long row, col;
            rowmap(mo, row, col);
            gadd(dst + (row * nc + col) * ndp + x, acc[r]);
        }
    }
    acc = v4d{0.0, 0.0, 0.0, 0.0};
}

// Pass C, one task per wave.  G16: the lane's column is density x of a
// group of 16; the wave keeps K_ac, K_bc accumulators for D (into K) and for
// D^T (into KT), and J from D + D^T.  G16 = false: columns 0-7 are 8
// densities with D, columns 8-15 the same 8 with D^T, in one accumulator set.
template <int LA, int LB, int LC, int LD, typename TT, bool G16>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_digest2_c(DigestArgs a) {
    using S = DigShape<LA, LB, LC, LD>;
    constexpr int NA = S::NA, NB = S::NB, NC = S::NC, ND = S::ND, NF = S::NF, NAB = S::NAB, NCD = S::NCD;
    constexpr int QB = dig2_qb(NF), QBP = QB + 1;
    static_assert(QB > 0, "class too large for wave-private digestion");
    constexpr int MJ = S::MJ, M2 = (QB * NCD + 15) / 16, KJ2 = S::KJ2, M3 = S::M3, M4 = S::M4;
    constexpr int NK = M3 + M4;                 // K tiles per density form
    constexpr int WPB = kDig2Waves;
    __shared__ double sTall[WPB][NF * QBP];
    __shared__ int sVall[WPB][QB];
    __shared__ int sPall[WPB][QB];
    __shared__ int sOall[WPB][QB];

    const int wave = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
    if (wave >= WPB) return;
    int p0 = 0, plen = 0, grp = 0;
    const DigItem* itp = dig2_task<WPB>(a, wave, p0, plen, grp);
    if (!itp) return;
    double* sT = sTall[wave];
    int* sV = sVall[wave];
    int* sP = sPall[wave];
    int* sO = sOall[wave];
    const DigItem it = *itp;
    const int c16 = lane & 15, r4 = lane >> 4;
    const MolDesc m = load_mol(a.mols, a.mol0, it.mol);
    // the lane's density column; tr: its column holds D^T (8-density groups only)
    const DigLane<double> L(m, G16 ? grp * 16 + c16 : grp * 8 + (c16 & 7), G16 ? false : c16 >= 8);
    const bool live = L.x < m.nd;
    const long long nc = m.nc;
    const PairInfo& P = m.pairs[it.bra];
    const int fa = P.fa, fb = P.fb, sa = P.sa, sb = P.sb;
    const gptr<const TT> tile = glob(static_cast<const TT*>(a.tiles)) + it.tile_off;
    const long long nq = it.chunk_n, qrel = it.blk0 - it.chunk_q0;
    const gptr<const long long> kin = glob(reinterpret_cast<const long long*>(it.kin)) + it.blk0;
    const gptr<const int> posl = glob(it.pos) + it.blk0;
    const bool wj = a.want_j, wk = a.want_k, skipT = a.skip_t != 0;

    // symmetrized densities of the lane's column (8-density groups: columns 0-7 only)
    const bool jcol = G16 || c16 < 8;
    const gptr<const double> dsx = glob(m.DS) + L.x;
    // J_cd's B operand, fixed for the task: D^S_ab at k-row ij = 4 t + r4
    double sab[KJ2];
    {
        const long long u0 = wj ? m.ds_off[sa * m.ns + sb] : 0;
#pragma unroll
        for (int t = 0; t < KJ2; ++t) {
            const int ij = 4 * t + r4;
            sab[t] = (wj && ij < NAB && jcol) ? dsx[(u0 + ij) * L.ndp] : 0.0;
        }
    }
    // tile row of the lane's A operand in each accumulator tile
    int fj[MJ], fk[NK];
#pragma unroll
    for (int t = 0; t < MJ; ++t) {
        const int r = t * 16 + c16;
        fj[t] = r < NAB ? r * NCD : 0;
    }
#pragma unroll
    for (int t = 0; t < NK; ++t) {
        fk[t] = 0;
        if (t < M3) {
            const int r = t * 16 + c16;
            if (r < NA * NC) fk[t] = (r / NC) * NB * NCD + (r % NC) * ND;
        } else {
            const int r = (t - M3) * 16 + c16;
            if (r < NB * NC) fk[t] = (r / NC) * NCD + (r % NC) * ND;
        }
    }
    v4d accJ[MJ], accK[NK], accT[G16 ? NK : 1];
#pragma unroll
    for (int t = 0; t < MJ; ++t) accJ[t] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < NK; ++t) accK[t] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < (G16 ? NK : 1); ++t) accT[t] = v4d{0.0, 0.0, 0.0, 0.0};

    const int pend = p0 + plen;
    for (int p = p0; p < pend;) {
        int2 kv;
        bool more;
        const int n = dig_chunk<QB>(kin, p, pend, lane, 0, kv, more);
        const int fc = __shfl(kv.y & 0xffff, 0);
        const double wl = lane < n ? fold_weight(sa, sb, kv.x & 0xffff, kv.x >> 16) : 0.0;
        if (lane < QB) {
            sV[lane] = lane < n ? kv.y >> 16 : fc;
            sP[lane] = lane < n && wk && grp == 0 ? posl[p + lane] : 0;
            // first packed D^S unit of the quartet's ket pair (c, d)
            sO[lane] = lane < n && wj ? m.ds_off[(kv.x & 0xffff) * m.ns + (kv.x >> 16)] : 0;
        }
#pragma unroll 4
        for (int base = 0; base < NF * QB; base += 64) {
            const int idx = base + lane;
            const int f = idx / QB, qb = idx - (idx / QB) * QB;
            double t = 0.0;
            if (idx < NF * QB && p + qb < pend) t = static_cast<double>(tile[f * nq + qrel + p + qb]);
            const double w = __shfl(wl, qb);
            if (idx < NF * QB) sT[f * QBP + qb] = w * t;
        }
        wave_lds_sync();
        if (wk && grp == 0) {
            const gptr<TT> cp = glob(static_cast<TT*>(a.dcopy)) + it.tile_off;
            for (int idx = lane; idx < n * NF; idx += 64) {
                const int qb = idx / NF, f = idx - (idx / NF) * NF;
                cp[(qrel + sP[qb]) * NF + f] = static_cast<TT>(sT[f * QBP + qb]);
            }
        }
        const int nquad = (n + 3) >> 2;
        if (wj) {
            // J_ab: contraction over (d in run, k, l)
            #pragma unroll 1
            for (int s = 0; s < nquad; ++s) {
                const int qb = 4 * s + r4;
                const long long u = sO[qb];
                // the packed D^S record of the ket pair
                double bv[NCD];
#pragma unroll
                for (int v = 0; v < NCD; ++v) bv[v] = jcol ? dsx[(u + v) * L.ndp] : 0.0;
#pragma unroll
                for (int v = 0; v < NCD; ++v)
#pragma unroll
                    for (int t = 0; t < MJ; ++t) accJ[t] = mfma_f64(sT[(fj[t] + v) * QBP + qb], bv[v], accJ[t]);
            }
            // J_cd: one output row per (quartet, k, l), contraction over (i, j)
            #pragma unroll 1
            for (int mt = 0; mt < M2; ++mt) {
                if (mt * 16 >= n * NCD) break;
                const int r = mt * 16 + c16;
                const int qa = r < QB * NCD ? r / NCD : 0, va = r < QB * NCD ? r - (r / NCD) * NCD : 0;
                v4d cd = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int t = 0; t < KJ2; ++t) {
                    const int ij = 4 * t + r4 < NAB ? 4 * t + r4 : NAB - 1;
                    cd = mfma_f64(sT[(ij * NCD + va) * QBP + qa], sab[t], cd);
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    double v = cd[e];
                    if constexpr (!G16) v += __shfl_xor(v, 8);
                    const int mo = mt * 16 + 4 * e + r4;
                    const int qo = mo / NCD, vo = mo - (mo / NCD) * NCD;
                    if (qo < n && live && !L.tr) {
                        const int k = vo / ND, l = vo - (vo / ND) * ND;
                        gadd(m.J + ((fc + k) * nc + sV[qo] + l) * L.ndp + L.x, v);
                    }
                }
            }
        }
        if (wk) {
            #pragma unroll 1
            for (int s = 0; s < nquad; ++s) {
                const int qb = 4 * s + r4;
                const long long V0 = sV[qb];
                // K_ac: contraction over (j, l) with D_bd; K_bc: over (i, l) with D_ad
                // (one l at a time: its gathers, then its matrix instructions)
#pragma unroll 1
                for (int l = 0; l < ND; ++l) {
                    double b3[NB], b4[NA], t3[G16 ? NB : 1], t4[G16 ? NA : 1];
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        b3[j] = L.dk(fb + j, V0 + l);
                        if constexpr (G16) t3[j] = L.dt(fb + j, V0 + l);
                    }
#pragma unroll
                    for (int i = 0; i < NA; ++i) {
                        b4[i] = L.dk(fa + i, V0 + l);
                        if constexpr (G16) t4[i] = L.dt(fa + i, V0 + l);
                    }
#pragma unroll
                    for (int j = 0; j < NB; ++j)
#pragma unroll
                        for (int t = 0; t < M3; ++t) {
                            const double av = sT[(fk[t] + j * NCD + l) * QBP + qb];
                            accK[t] = mfma_f64(av, b3[j], accK[t]);
                            if (G16 && !skipT) accT[t] = mfma_f64(av, t3[j], accT[t]);
                        }
#pragma unroll
                    for (int i = 0; i < NA; ++i)
#pragma unroll
                        for (int t = M3; t < NK; ++t) {
                            const double av = sT[(fk[t] + i * NB * NCD + l) * QBP + qb];
                            accK[t] = mfma_f64(av, b4[i], accK[t]);
                            if (G16 && !skipT) accT[t] = mfma_f64(av, t4[i], accT[t]);
                        }
                }
            }
            if (!more) {
                auto mac = [&](int mo, long long& row, long long& col) {
                    row = fa + mo / NC;
                    col = fc + mo % NC;
                };
                auto mbc = [&](int mo, long long& row, long long& col) {
                    row = fb + mo / NC;
                    col = fc + mo % NC;
                };
                double* const kd = L.tr ? m.KT : m.K;
#pragma unroll
                for (int t = 0; t < M3; ++t) dig2_flush<NA * NC>(kd, nc, L.ndp, L.x, live, r4, accK[t], t, mac);
#pragma unroll
                for (int t = M3; t < NK; ++t) dig2_flush<NB * NC>(kd, nc, L.ndp, L.x, live, r4, accK[t], t - M3, mbc);
                if (G16 && !skipT) {
#pragma unroll
                    for (int t = 0; t < M3; ++t) dig2_flush<NA * NC>(m.KT, nc, L.ndp, L.x, live, r4, accT[t], t, mac);
#pragma unroll
                    for (int t = M3; t < NK; ++t)
                        dig2_flush<NB * NC>(m.KT, nc, L.ndp, L.x, live, r4, accT[t], t - M3, mbc);
                }
            }
        }
        p += n;
        wave_lds_sync();
    }
    if (wj) {
#pragma unroll
        for (int t = 0; t < MJ; ++t)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                double v = accJ[t][e];
                if constexpr (!G16) v += __shfl_xor(v, 8);
                const int mo = t * 16 + 4 * e + r4;
                if (mo < NAB && live && !L.tr) {
                    const int i = mo / NB, j = mo - (mo / NB) * NB;
                    gadd(m.J + ((fa + i) * nc + fb + j) * L.ndp + L.x, v);
                }
            }
    }
}

// Pass D, one task per wave: K_ad and K_bd over runs of equal ket shell d,
// from the D-order copy, with D and D^T (as in pass C).
template <int LA, int LB, int LC, int LD, typename TT, bool G16>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_digest2_d(DigestArgs a) {
    using S = DigShape<LA, LB, LC, LD>;
    constexpr int NA = S::NA, NB = S::NB, NC = S::NC, ND = S::ND, NF = S::NF, NCD = S::NCD;
    constexpr int QB = dig2_qb(NF), QBP = QB + 1;
    static_assert(QB > 0, "class too large for wave-private digestion");
    constexpr int M5 = S::M5, M6 = S::M6, NK = M5 + M6;
    constexpr int WPB = kDig2Waves;
    __shared__ double sTall[WPB][NF * QBP];
    __shared__ int sVall[WPB][QB];

    const int wave = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
    if (wave >= WPB) return;
    int p0 = 0, plen = 0, grp = 0;
    const DigItem* itp = dig2_task<WPB>(a, wave, p0, plen, grp);
    if (!itp) return;
    double* sT = sTall[wave];
    int* sV = sVall[wave];
    const DigItem it = *itp;
    const int c16 = lane & 15, r4 = lane >> 4;
    const MolDesc m = load_mol(a.mols, a.mol0, it.mol);
    const DigLane<double> L(m, G16 ? grp * 16 + c16 : grp * 8 + (c16 & 7), G16 ? false : c16 >= 8);
    const bool live = L.x < m.nd;
    const long long nc = m.nc;
    const PairInfo& P = m.pairs[it.bra];
    const int fa = P.fa, fb = P.fb;
    const gptr<const TT> cp = glob(static_cast<const TT*>(a.dcopy)) + it.tile_off;
    const long long qrel = it.blk0 - it.chunk_q0;
    const gptr<const long long> kin = glob(reinterpret_cast<const long long*>(it.kin)) + it.blk0;
    const bool skipT = a.skip_t != 0;

    int fk[NK];
#pragma unroll
    for (int t = 0; t < NK; ++t) {
        fk[t] = 0;
        if (t < M5) {
            const int r = t * 16 + c16;
            if (r < NA * ND) fk[t] = (r / ND) * NB * NCD + r % ND;
        } else {
            const int r = (t - M5) * 16 + c16;
            if (r < NB * ND) fk[t] = (r / ND) * NCD + r % ND;
        }
    }
    v4d accK[NK], accT[G16 ? NK : 1];
#pragma unroll
    for (int t = 0; t < NK; ++t) accK[t] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < (G16 ? NK : 1); ++t) accT[t] = v4d{0.0, 0.0, 0.0, 0.0};

    const int pend = p0 + plen;
    for (int p = p0; p < pend;) {
        int2 kv;
        bool more;
        const int n = dig_chunk<QB>(kin, p, pend, lane, 16, kv, more);
        const int fd = __shfl(kv.y >> 16, 0), fc0 = __shfl(kv.y & 0xffff, 0);
        if (lane < QB) sV[lane] = lane < n ? kv.y & 0xffff : fc0;
#pragma unroll 4
        for (int base = 0; base < NF * QB; base += 64) {
            const int idx = base + lane;
            const int qb = idx / NF, f = idx - (idx / NF) * NF;
            double t = 0.0;
            if (idx < NF * QB && p + qb < pend) t = static_cast<double>(cp[(qrel + p + qb) * NF + f]);
            if (idx < NF * QB) sT[f * QBP + qb] = qb < n ? t : 0.0;
        }
        wave_lds_sync();
        const int nquad = (n + 3) >> 2;
        #pragma unroll 1
        for (int s = 0; s < nquad; ++s) {
            const int qb = 4 * s + r4;
            const long long V0 = sV[qb];
            // K_ad: contraction over (j, k) with D_bc; K_bd: over (i, k) with D_ac
#pragma unroll 1
            for (int k = 0; k < NC; ++k) {
                double b5[NB], b6[NA], t5[G16 ? NB : 1], t6[G16 ? NA : 1];
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    b5[j] = L.dk(fb + j, V0 + k);
                    if constexpr (G16) t5[j] = L.dt(fb + j, V0 + k);
                }
#pragma unroll
                for (int i = 0; i < NA; ++i) {
                    b6[i] = L.dk(fa + i, V0 + k);
                    if constexpr (G16) t6[i] = L.dt(fa + i, V0 + k);
                }
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int t = 0; t < M5; ++t) {
                        const double av = sT[(fk[t] + j * NCD + k * ND) * QBP + qb];
                        accK[t] = mfma_f64(av, b5[j], accK[t]);
                        if (G16 && !skipT) accT[t] = mfma_f64(av, t5[j], accT[t]);
                    }
#pragma unroll
                for (int i = 0; i < NA; ++i)
#pragma unroll
                    for (int t = M5; t < NK; ++t) {
                        const double av = sT[(fk[t] + i * NB * NCD + k * ND) * QBP + qb];
                        accK[t] = mfma_f64(av, b6[i], accK[t]);
                        if (G16 && !skipT) accT[t] = mfma_f64(av, t6[i], accT[t]);
                    }
            }
        }
        if (!more) {
            auto mad = [&](int mo, long long& row, long long& col) {
                row = fa + mo / ND;
                col = fd + mo % ND;
            };
            auto mbd = [&](int mo, long long& row, long long& col) {
                row = fb + mo / ND;
                col = fd + mo % ND;
            };
            double* const kd = L.tr ? m.KT : m.K;
#pragma unroll
            for (int t = 0; t < M5; ++t) dig2_flush<NA * ND>(kd, nc, L.ndp, L.x, live, r4, accK[t], t, mad);
#pragma unroll
            for (int t = M5; t < NK; ++t) dig2_flush<NB * ND>(kd, nc, L.ndp, L.x, live, r4, accK[t], t - M5, mbd);
            if (G16 && !skipT) {
#pragma unroll
                for (int t = 0; t < M5; ++t) dig2_flush<NA * ND>(m.KT, nc, L.ndp, L.x, live, r4, accT[t], t, mad);
#pragma unroll
                for (int t = M5; t < NK; ++t) dig2_flush<NB * ND>(m.KT, nc, L.ndp, L.x, live, r4, accT[t], t - M5, mbd);
            }
        }
        p += n;
        wave_lds_sync();
    }
}

}  // namespace jk
