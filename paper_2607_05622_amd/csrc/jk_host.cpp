// Host side of the J/K C-ABI: basis ingest, resident shell-pair data, Schwarz
// factors, screened quartet lists, workspace and the launch sequence of one
// build.  See include/jk.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "jk.h"
#include "jk_cd.h"
#include "jk_internal.h"
#include "jk_launch.h"

namespace jk {
#include "eri_cost.inc"   // kClassCost[21]: generated flop counts per class
}

using namespace jk;

static_assert(kNoAllocScratchBytes == JK_NOALLOC_MAX_BYTES, "static workspace size");

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPC(expr)                                                                       \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) return fail(JK_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr double kPi = 3.14159265358979323846;
// Primitive-pair screen: a primitive pair (alpha, beta) of shells a, b is
// kept iff |E_ab| max(1, |AB|)^(la+lb) >= kPrimPairTol, E_ab the prefactor
// of PrimPair (its Gaussian product factor exp(-alpha beta/p |AB|^2) times
// the contraction weights), the power bounding the separations the
// recurrences multiply in.  1e-6 of the default quartet threshold: what is
// dropped stays far below FP64 rounding of the contracted integrals.
constexpr double kPrimPairTol = 1e-18;
// Integral work buffer cap (elements): 2 GB of FP64 tiles, so a launch of a
// high angular momentum class holds a few hundred thousand quartets, many
// waves per SIMD at its one-wave occupancy.
constexpr long long kTileCapElems = 256ll << 20;
// Launch lanes of a build: consecutive class/tier launches alternate between
// the caller's stream and a helper stream of the handle, each lane with its
// own integral work and scratch buffers, so one class's integrals overlap
// another's digestion and the launches' ramp-ups and tails overlap.
constexpr int kLanes = 2;

double dfact(int n) {
    double r = 1.0;
    for (; n > 1; n -= 2) r *= n;
    return r;
}

// Boys table: F_m(T0), m = 0..kBoysCols-2, and exp(-T0) at T0 = i/32.  F at the
// top order comes from its power series exp(-T) sum_k (2T)^k / prod_{j<=k}
// (2m+2j+1), summed in long double; lower orders by downward recursion.
std::vector<double> make_boys_table() {
    std::vector<double> t(static_cast<size_t>(kBoysPoints) * kBoysCols);
    const int mtop = kBoysCols - 2 + 8;
    for (int i = 0; i < kBoysPoints; ++i) {
        const long double T = static_cast<long double>(i) / kBoysInvStep;
        long double term = 1.0L / (2 * mtop + 1), sum = term;
        for (int k = 1; k < 4000; ++k) {
            term *= 2.0L * T / (2 * mtop + 2 * k + 1);
            sum += term;
            if (term < sum * 1e-22L) break;
        }
        const long double e = expl(-T);
        long double f = e * sum;
        std::vector<long double> F(mtop + 1);
        F[mtop] = f;
        for (int m = mtop - 1; m >= 0; --m) F[m] = (2.0L * T * F[m + 1] + e) / (2 * m + 1);
        for (int m = 0; m < kBoysCols - 1; ++m) t[static_cast<size_t>(i) * kBoysCols + m] = static_cast<double>(F[m]);
        t[static_cast<size_t>(i) * kBoysCols + kBoysCols - 1] = static_cast<double>(e);
    }
    return t;
}

const std::vector<double>& boys_table() {
    static std::vector<double> t = make_boys_table();
    return t;
}

// Pure-d coefficients over x^2-normalized Cartesian d components, user order
// (xy, yz, 3z^2-r^2, xz, x^2-y^2) x Cartesian (xx, xy, xz, yy, yz, zz).
const double kSphD[5][6] = {
    {0, 1.7320508075688772935, 0, 0, 0, 0},
    {0, 0, 0, 0, 1.7320508075688772935, 0},
    {-0.5, 0, 0, -0.5, 0, 1.0},
    {0, 0, 1.7320508075688772935, 0, 0, 0},
    {0.86602540378443864676, 0, 0, -0.86602540378443864676, 0, 0},
};

int class_nf(int cls) { return kClassCost[cls].nfunc; }

// Schedule tunables per class (process-wide; chosen by jk_autotune): the
// length cap of a digestion part (a run of one bra pair's quartets with one
// ket shell, digested by one task; longer runs are cut), the densities a
// digestion task takes at once (16, or 8 when g_max < 16 or the batch has at
// most 8 densities), the digestion kernel (1: workgroup-shared chunks, 2:
// wave-private tasks) and the quartets per integral workgroup.
struct Tune {
    int seg_max = 256;
    int g_max = 16;
    int dig_kernel = 1;
    int eri_block = 256;
};
std::mutex g_tune_mu;
Tune g_tune[kNumClass];
int g_tune_gen = 0;

Tune tune_of(int cls) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    return g_tune[cls];
}


// A class list holds its FP64-tier quartets (Q_ab Q_cd >= fp32 bound) first
// and its FP32-tier quartets after them.  Within a tier the quartets of one
// bra pair are consecutive (a block) with ket pairs in (c, d) order.
struct ClassList {
    long long count = 0;
    long long n64 = 0;               // quartets of the FP64 tier (list prefix)
    int nblk64 = 0;                  // blocks of the FP64 tier (prefix of blocks)
    double prim_quartets[2] = {0, 0};   // sum of nprim_bra * nprim_ket per tier
    int2* dev = nullptr;
    std::vector<int2> blocks;        // (first quartet, count)
    std::vector<int> block_bra;      // bra shell pair of each block
    // digestion parts per pass (0: runs of equal c in list order, 1: runs of
    // equal d in (d, c) order, packed whole up to the tunable cap, longer
    // runs cut at it): block k's parts start
    // at positions parts[ps][part_off[ps][k] ..] of the block
    std::vector<int> part_off[2];
    int* dev_parts[2] = {nullptr, nullptr};
    int* dev_pos = nullptr;          // per quartet: its position in the block's (d, c) order
    int2* dev_kin = nullptr;         // per quartet, list order: (c | d << 16, fc | fd << 16) of the ket
    int2* dev_kind = nullptr;        // the same per position of the blocks' (d, c) orders
};

// pair class X -> (la, lb)
const int kPairL[6][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}};

// Highest total angular momentum la + lb + lc + ld whose quartets may take
// the FP32 tier.  Beyond it the terms of the FP32 vertical recurrence for
// distant pairs exceed the integral by more than the FP32 precision buys
// (measured: d-d classes of the 620-AO workload in FP32 give relative J/K
// errors of ~5e-6 at a Schwarz bound of 1e-6).
constexpr int kFp32MaxL = 4;

}  // namespace

// Error recording for the other translation units of the library.
int record_error(int code, const char* msg) { return fail(code, "%s", msg); }


namespace {
struct CachedPlan;
void free_plan(CachedPlan* cp);
}

struct jk_basis_s {
    int device = 0;
    int natoms = 0, ns = 0, nf = 0, nc = 0, spherical = 1;
    // internal shells are the user shells sorted by l (stable)
    std::vector<int> user_of_int, int_of_user, l_int, f0_int, ncart_int, nprim_int;
    std::vector<int> user_f0;   // user function offset per user shell
    std::vector<double> centre_int;   // [ns][3]
    std::vector<std::vector<double>> exps_int, w_int;   // normalized contraction weights
    std::vector<PairInfo> pairs;
    std::vector<PrimPair> prims;          // set-up only: records, pair-major
    std::vector<double> prim_planes;      // set-up only: their device layout (kPrimLane)
    int pslots = 0;
    std::vector<int> pair_id;   // [ns][ns] -> pair index for a >= b, else -1
    std::vector<int> pairs_of_class[kNumPairClass];
    // device
    PairInfo* d_pairs = nullptr;
    double* d_prims = nullptr;
    double* d_boys = nullptr;
    CartMap* d_cmap = nullptr;
    UserMap* d_umap = nullptr;
    int* d_shell_f0 = nullptr;
    int* d_shell_nf = nullptr;
    int* d_ds_off = nullptr;          // [ns][ns]: first packed unit of shell pair (c, d), c >= d
    hipStream_t aux = nullptr;        // helper stream of the second launch lane (default priority)
    long long ds_units = 0;           // packed units over all shell pairs (sum of nc nd)
    // quartet lists for the current tolerance (older lists are retired, not
    // freed, because builds on other streams may still read them)
    std::mutex mu;
    double list_tol = -1.0;
    double list_bound = 1e-6;          // FP32-tier bound the lists are partitioned with
    float* d_boys32 = nullptr;
    ClassList lists[kNumClass];
    std::vector<void*> retired;
    int list_gen = 0;                  // bumped whenever the lists are rebuilt
    int tune_gen = -1;                 // tunables the lists' digestion parts were cut with
    std::vector<CachedPlan*> plans;    // single-molecule plans (freed by jk_destroy)
    double stats[6] = {0, 0, 0, 0, 0, 0};
    // measurement: event pairs around integral / digestion launches
    struct ProfRec {
        int kind, cls;
        hipEvent_t e0, e1;
        double flops, quartets, bytes;
    };
    bool profiling = false;
    std::vector<ProfRec> prof;
    double prof_acc[6][kNumClass][5] = {};
    // per tier and class: quartets the whole screen kept in profiled builds
    // (device counters, folded and cleared by jk_profile_read)
    unsigned long long* d_kept = nullptr;

    ~jk_basis_s() {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(device);
        (void)hipFree(d_pairs);
        (void)hipFree(d_prims);
        (void)hipFree(d_boys);
        (void)hipFree(d_boys32);
        (void)hipFree(d_cmap);
        (void)hipFree(d_umap);
        (void)hipFree(d_shell_f0);
        (void)hipFree(d_shell_nf);
        (void)hipFree(d_ds_off);
        if (aux) (void)hipStreamDestroy(aux);
        for (auto& l : lists) {
            (void)hipFree(l.dev);
            (void)hipFree(l.dev_pos);
            (void)hipFree(l.dev_kin);
            (void)hipFree(l.dev_kind);
            (void)hipFree(l.dev_parts[0]);
            (void)hipFree(l.dev_parts[1]);
        }
        for (auto* p : retired) (void)hipFree(p);
        (void)hipFree(d_kept);
        for (auto& r : prof) {
            (void)hipEventDestroy(r.e0);
            (void)hipEventDestroy(r.e1);
        }
        (void)hipSetDevice(cur);
    }
};

namespace jk {
int basis_view(jk_basis_t h, BasisView* v) {
    if (!h || !v) return fail(JK_EINVAL, "basis_view: NULL argument");
    v->device = h->device;
    v->ns = h->ns;
    v->nf = h->nf;
    v->spherical = h->spherical;
    v->pairs = h->pairs;
    for (int X = 0; X < kNumPairClass; ++X) v->pairs_of_class[X] = h->pairs_of_class[X];
    v->uf0.assign(h->ns, 0);
    v->nuf.assign(h->ns, 0);
    for (int s = 0; s < h->ns; ++s) {
        const int su = h->user_of_int[s];
        v->uf0[s] = h->user_f0[su];
        v->nuf[s] = h->user_f0[su + 1] - h->user_f0[su];
    }
    v->d_pairs = h->d_pairs;
    v->d_prims = h->d_prims;
    v->d_boys = h->d_boys;
    v->d_boys32 = h->d_boys32;
    v->d_umap = h->d_umap;
    v->pslots = h->pslots;
    return JK_OK;
}
}  // namespace jk

namespace {

template <class T>
int upload(T** dst, const std::vector<T>& src) {
    const size_t n = std::max<size_t>(src.size(), 1);
    HIPC(hipMalloc(reinterpret_cast<void**>(dst), n * sizeof(T)));
    if (!src.empty()) HIPC(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return JK_OK;
}

// Evaluate Cartesian tiles for a host list of canonical (bra pair, ket pair)
// quartets of one class; tiles come back [nq][NF].
int eval_tiles(jk_basis_s* h, int cls, const std::vector<int2>& quartets, std::vector<double>& tiles) {
    const long long nq = static_cast<long long>(quartets.size());
    const int NF = class_nf(cls);
    tiles.assign(static_cast<size_t>(nq) * NF, 0.0);
    if (nq == 0) return JK_OK;
    int2* dq = nullptr;
    double* dout = nullptr;
    double* dscr = nullptr;
    EriItem* ditem = nullptr;
    HIPC(hipMalloc(&dq, nq * sizeof(int2)));
    HIPC(hipMalloc(&dout, nq * NF * sizeof(double)));
    HIPC(hipMalloc(&dscr, nq * NF * sizeof(double)));
    HIPC(hipMalloc(&ditem, sizeof(EriItem)));
    int rc = JK_OK;
    do {
        EriItem it{};
        it.quartets = dq;
        it.n = nq;
        it.tile_off = 0;
        it.blk0 = 0;
        it.mol = 0;
        if (hipMemcpy(dq, quartets.data(), nq * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(ditem, &it, sizeof(it), hipMemcpyHostToDevice) != hipSuccess) {
            rc = fail(JK_EDEVICE, "eval_tiles: copy in failed");
            break;
        }
        EriTileArgs a{};
        a.items = ditem;
        a.nitems = 1;
        a.nblocks = (nq + 255) / 256;
        a.block = 256;
        a.mol0.pairs = h->d_pairs;
        a.mol0.prims = h->d_prims;
        a.mol0.pslots = h->pslots;
        a.mol0.dmax = nullptr;
        a.mol0.ns = h->ns;
        a.mols = nullptr;
        a.boys = h->d_boys;
        a.boys32 = h->d_boys32;
        a.tol = 0.0;
        a.tiles = dout;
        a.scratch = dscr;
        hipError_t e = launch_eri_tile(cls, a, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            rc = fail(JK_EDEVICE, "eri tile kernel: %s", hipGetErrorString(e));
            break;
        }
        std::vector<double> fm(static_cast<size_t>(nq) * NF);
        if (hipMemcpy(fm.data(), dout, fm.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
            rc = fail(JK_EDEVICE, "eval_tiles: copy out failed");
            break;
        }
        for (long long q = 0; q < nq; ++q)
            for (int f = 0; f < NF; ++f) tiles[q * NF + f] = fm[static_cast<size_t>(f) * nq + q];
    } while (0);
    (void)hipFree(dq);
    (void)hipFree(dout);
    (void)hipFree(dscr);
    (void)hipFree(ditem);
    return rc;
}

int compute_schwarz(jk_basis_s* h) {
    for (int X = 0; X < kNumPairClass; ++X) {
        const auto& ps = h->pairs_of_class[X];
        if (ps.empty()) continue;
        std::vector<int2> qs(ps.size());
        for (size_t i = 0; i < ps.size(); ++i) qs[i] = make_int2(ps[i], ps[i]);
        std::vector<double> tiles;
        const int cls = quartet_class(X, X);
        int rc = eval_tiles(h, cls, qs, tiles);
        if (rc) return rc;
        const int NF = class_nf(cls);
        for (size_t i = 0; i < ps.size(); ++i) {
            PairInfo& P = h->pairs[ps[i]];
            const int na = h->ncart_int[P.sa], nb = h->ncart_int[P.sb];
            double mx = 0.0;
            for (int u = 0; u < na; ++u)
                for (int v = 0; v < nb; ++v) {
                    const double d = tiles[i * NF + ((u * nb + v) * na + u) * nb + v];
                    mx = std::max(mx, d);
                }
            P.q = std::sqrt(mx);
        }
    }
    return JK_OK;
}

// Runs body(i) for i in [0, n) on up to hardware_concurrency() host threads
// (at most 16), in contiguous chunks handed out dynamically.
template <class Body>
void parallel_for(long long n, Body body) {
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const long long nt = std::min<long long>(hw, n);
    if (nt <= 1) {
        for (long long i = 0; i < n; ++i) body(i);
        return;
    }
    const long long chunk = std::max<long long>(1, n / (nt * 8));
    std::atomic<long long> next{0};
    auto worker = [&]() {
        for (;;) {
            const long long i0 = next.fetch_add(chunk);
            if (i0 >= n) return;
            const long long i1 = std::min(n, i0 + chunk);
            for (long long i = i0; i < i1; ++i) body(i);
        }
    };
    std::vector<std::thread> ts;
    for (long long t = 1; t < nt; ++t) ts.emplace_back(worker);
    worker();
    for (auto& t : ts) t.join();
}

// One bra pair's share of a class list: its kept ket pairs per tier (ket
// index order) and the digestion parts of each of its two blocks per pass
// (start positions within the block).
struct BraLists {
    std::vector<int> keep[2];
    std::vector<int> parts[2][2];   // [tier][pass]
    double primq[2] = {0, 0};
};

// Build the class-bucketed quartet lists kept by Q_ab Q_cd >= tol.  Within a
// class: bra pair outer, ket pairs in index order.  The bra pairs of a class
// are independent: their keep lists, (d, c) orders and digestion parts are
// made on host threads, then written at offsets from a prefix sum.
int build_lists(jk_basis_s* h, double tol, double bound) {
    ClassList fresh[kNumClass];
    for (int X = 0; X < kNumPairClass; ++X) {
        for (int Y = 0; Y <= X; ++Y) {
            const int cls = quartet_class(X, Y);
            // FP32 tier only for classes of total angular momentum <= kFp32MaxL:
            // higher classes cancel too strongly in the vertical recurrence
            const bool fp32_ok = kPairL[X][0] + kPairL[X][1] + kPairL[Y][0] + kPairL[Y][1] <= kFp32MaxL;
            const auto& bra = h->pairs_of_class[X];
            const auto& ket = h->pairs_of_class[Y];
            // ket pairs sorted by Q, descending, to stop early
            std::vector<int> ks(ket);
            std::sort(ks.begin(), ks.end(), [&](int u, int v) { return h->pairs[u].q > h->pairs[v].q; });
            const int cap = std::max(4, tune_of(cls).seg_max);
            const bool pack = kClassCost[cls].nfunc <= 18;
            const size_t nbra = bra.size();
            std::vector<BraLists> bl(nbra);
            // phase 1: per bra pair, its kept kets per tier and the parts of its blocks
            parallel_for(static_cast<long long>(nbra), [&](long long bi) {
                const int b = bra[bi];
                BraLists& B = bl[bi];
                const double qb = h->pairs[b].q;
                std::vector<int> keep;
                for (int k : ks) {
                    if (qb * h->pairs[k].q < tol) break;
                    if (X == Y && k > b) continue;
                    keep.push_back(k);
                }
                std::sort(keep.begin(), keep.end());
                for (int k : keep) {
                    const int t = fp32_ok && qb * h->pairs[k].q < bound ? 1 : 0;
                    B.keep[t].push_back(k);
                    B.primq[t] += static_cast<double>(h->pairs[b].nprim) * h->pairs[k].nprim;
                }
                std::vector<int> idx, sv[2];
                for (int t = 0; t < 2; ++t) {
                    const std::vector<int>& kp = B.keep[t];
                    const size_t n = kp.size();
                    if (n == 0) continue;
                    // ket shell c (pass C, list order) and d (pass D, (d, c) order) per position
                    idx.resize(n);
                    for (size_t i = 0; i < n; ++i) idx[i] = static_cast<int>(i);
                    std::stable_sort(idx.begin(), idx.end(), [&](int u, int v) {
                        const PairInfo& U = h->pairs[kp[u]];
                        const PairInfo& V = h->pairs[kp[v]];
                        return U.sb != V.sb ? U.sb < V.sb : U.sa < V.sa;
                    });
                    sv[0].resize(n);
                    sv[1].resize(n);
                    for (size_t i = 0; i < n; ++i) {
                        sv[0][i] = h->pairs[kp[i]].sa;
                        sv[1][i] = h->pairs[kp[idx[i]]].sb;
                    }
                    // parts: runs of equal c (pass C) or d (pass D), a run
                    // longer than cap cut into pieces of cap.  Classes of at
                    // most 18 functions per quartet pack consecutive whole
                    // runs into one part up to cap positions: their runs are
                    // short and a workgroup's set-up outweighs its work.
                    for (int ps = 0; ps < 2; ++ps) {
                        const std::vector<int>& kv = sv[ps];
                        std::vector<int>& out = B.parts[t][ps];
                        const size_t ucap = static_cast<size_t>(cap), none = ~size_t(0);
                        size_t open = none;   // first position of the part being filled
                        for (size_t p = 0; p < n;) {
                            size_t r = p + 1;
                            while (r < n && kv[r] == kv[p]) ++r;
                            if (r - p > ucap) {
                                if (open != none) out.push_back(static_cast<int>(open));
                                open = none;
                                for (size_t c = p; c < r; c += ucap) out.push_back(static_cast<int>(c));
                            } else {
                                if (open != none && (!pack || r - open > ucap)) {
                                    out.push_back(static_cast<int>(open));
                                    open = none;
                                }
                                if (open == none) open = p;
                            }
                            p = r;
                        }
                        if (open != none) out.push_back(static_cast<int>(open));
                    }
                }
            });
            // phase 2: offsets of every bra pair's blocks (FP64 tier, then FP32 tier)
            ClassList& F = fresh[cls];
            std::vector<long long> qoff[2];
            std::vector<int> boff[2];
            long long nq[2] = {0, 0};
            for (int t = 0; t < 2; ++t) {
                qoff[t].resize(nbra);
                boff[t].resize(nbra);
                for (size_t bi = 0; bi < nbra; ++bi) {
                    qoff[t][bi] = nq[t];
                    nq[t] += static_cast<long long>(bl[bi].keep[t].size());
                }
                F.prim_quartets[t] = 0.0;
                for (size_t bi = 0; bi < nbra; ++bi) F.prim_quartets[t] += bl[bi].primq[t];
            }
            const long long total = nq[0] + nq[1];
            F.count = total;
            F.n64 = nq[0];
            for (int t = 0; t < 2; ++t) {
                for (size_t bi = 0; bi < nbra; ++bi) {
                    if (bl[bi].keep[t].empty()) continue;
                    const long long q0 = (t ? nq[0] : 0) + qoff[t][bi];
                    F.blocks.push_back(make_int2(static_cast<int>(q0), static_cast<int>(bl[bi].keep[t].size())));
                    F.block_bra.push_back(bra[bi]);
                    boff[t][bi] = static_cast<int>(F.blocks.size()) - 1;
                }
                if (t == 0) F.nblk64 = static_cast<int>(F.blocks.size());
            }
            // part_off[ps][k] is the first part of block k; fill it from the part counts
            const int nblk = static_cast<int>(F.blocks.size());
            std::vector<int> parts[2];
            for (int ps = 0; ps < 2; ++ps) {
                F.part_off[ps].assign(nblk + 1, 0);
                for (int t = 0; t < 2; ++t)
                    for (size_t bi = 0; bi < nbra; ++bi)
                        if (!bl[bi].keep[t].empty())
                            F.part_off[ps][boff[t][bi] + 1] = static_cast<int>(bl[bi].parts[t][ps].size());
                for (int k = 0; k < nblk; ++k) F.part_off[ps][k + 1] += F.part_off[ps][k];
                parts[ps].resize(F.part_off[ps][nblk]);
            }
            // phase 3: every bra pair writes its quartets, ket records, (d, c)
            // positions and parts at its offsets
            std::vector<int2> out(total), kin(total), kind(total);
            std::vector<int> pos(total);
            parallel_for(static_cast<long long>(nbra), [&](long long bi) {
                const int b = bra[bi];
                std::vector<int> idx;
                for (int t = 0; t < 2; ++t) {
                    const std::vector<int>& kp = bl[bi].keep[t];
                    const size_t n = kp.size();
                    if (n == 0) continue;
                    const long long q0 = (t ? nq[0] : 0) + qoff[t][bi];
                    for (size_t i = 0; i < n; ++i) {
                        const PairInfo& Q = h->pairs[kp[i]];
                        out[q0 + i] = make_int2(b, kp[i]);
                        kin[q0 + i] = make_int2(Q.sa | (Q.sb << 16), Q.fa | (Q.fb << 16));
                    }
                    idx.resize(n);
                    for (size_t i = 0; i < n; ++i) idx[i] = static_cast<int>(i);
                    std::stable_sort(idx.begin(), idx.end(), [&](int u, int v) {
                        const PairInfo& U = h->pairs[kp[u]];
                        const PairInfo& V = h->pairs[kp[v]];
                        return U.sb != V.sb ? U.sb < V.sb : U.sa < V.sa;
                    });
                    for (size_t p = 0; p < n; ++p) {
                        kind[q0 + p] = kin[q0 + idx[p]];
                        pos[q0 + idx[p]] = static_cast<int>(p);
                    }
                    const int k = boff[t][bi];
                    for (int ps = 0; ps < 2; ++ps)
                        std::copy(bl[bi].parts[t][ps].begin(), bl[bi].parts[t][ps].end(),
                                  parts[ps].begin() + F.part_off[ps][k]);
                }
            });
            std::vector<BraLists>().swap(bl);
            if (!out.empty()) {
                int rc = upload(&F.dev, out);
                if (!rc) rc = upload(&F.dev_pos, pos);
                if (!rc) rc = upload(&F.dev_kin, kin);
                if (!rc) rc = upload(&F.dev_kind, kind);
                if (!rc) rc = upload(&F.dev_parts[0], parts[0]);
                if (!rc) rc = upload(&F.dev_parts[1], parts[1]);
                if (rc) {
                    for (auto& f : fresh) {
                        (void)hipFree(f.dev);
                        (void)hipFree(f.dev_pos);
                        (void)hipFree(f.dev_kin);
                        (void)hipFree(f.dev_kind);
                        (void)hipFree(f.dev_parts[0]);
                        (void)hipFree(f.dev_parts[1]);
                    }
                    return rc;
                }
            }
        }
    }
    for (int c = 0; c < kNumClass; ++c) {
        if (h->lists[c].dev) h->retired.push_back(h->lists[c].dev);
        if (h->lists[c].dev_pos) h->retired.push_back(h->lists[c].dev_pos);
        if (h->lists[c].dev_kin) h->retired.push_back(h->lists[c].dev_kin);
        if (h->lists[c].dev_kind) h->retired.push_back(h->lists[c].dev_kind);
        for (int ps = 0; ps < 2; ++ps)
            if (h->lists[c].dev_parts[ps]) h->retired.push_back(h->lists[c].dev_parts[ps]);
        h->lists[c] = fresh[c];
    }
    h->list_tol = tol;
    h->list_bound = bound;
    h->list_gen++;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        h->tune_gen = g_tune_gen;
    }
    return JK_OK;
}

// Lists usable for a build with tolerance tol and, in mixed mode, FP32 bound
// `bound` (bound < 0: any partition will do).
int ensure_lists(jk_basis_s* h, double tol, double bound) {
    std::lock_guard<std::mutex> g(h->mu);
    const bool tol_ok = h->list_tol >= 0 && h->list_tol <= tol;
    const bool bound_ok = bound < 0 || h->list_bound == bound;
    int tg;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        tg = g_tune_gen;
    }
    if (tol_ok && bound_ok && h->tune_gen == tg) return JK_OK;
    return build_lists(h, tol_ok ? h->list_tol : tol, bound < 0 ? h->list_bound : bound);
}

// ----------------------------------------------------------- work plans ---

// One class and tier of a build: an integral launch over eri items and two
// digestion launches (pass C, pass D) over dig items, all molecules together.
struct LaunchRec {
    int cls = 0, fp32 = 0, g16 = 1, dig_kernel = 1, eri_block = 256;
    int eri0 = 0, neri = 0;
    long long eri_blocks = 0;
    int dig0[2] = {0, 0}, ndig[2] = {0, 0};
    unsigned dig_blocks[2] = {0, 0};
    double eri_flops = 0, dig_flops[2] = {0, 0}, quartets = 0, tile_bytes = 0;
};

struct MolRun {
    jk_basis_s* h;
    int nd;
};

struct WorkPlan {
    bool skip_t = false;             // symmetric densities: KT contractions skipped (K = Kc + Kc^T)
    std::vector<EriItem> eri;
    std::vector<DigItem> dig[2];
    std::vector<LaunchRec> launches;
    long long tile_elems = 1296;
    double stats[6] = {0, 0, 0, 0, 0, 0};
};

// Density stride of a molecule with nd densities: a multiple of the
// digestion group, 16 beyond 8 densities and 8 up to there.
int dens_stride(int nd) { return nd > 8 ? (nd + 15) / 16 * 16 : 8; }

// Split every class list (per tier) of every molecule into tile items of
// whole blocks and digestion pieces (pass C in list order, pass D in (d, c)
// order), packing items into launches whose tiles fit a buffer of cap
// elements.
int plan_work(const std::vector<MolRun>& mols, const jk_build_opts* o, long long cap, WorkPlan& wp) {
    const bool mixed = o->precision == JK_MIXED;
    bool all16 = true;
    for (const MolRun& r : mols) all16 = all16 && dens_stride(r.nd) % 16 == 0;
    // symmetric densities: with 16-density groups the D^T contractions give
    // the same sums as the D ones, so they are skipped and K = Kc + Kc^T
    wp.skip_t = o->symmetric_hint && o->want_k && all16;
    for (int c = 0; c < kNumClass; ++c) {
        const int NF = class_nf(c);
        const Tune tn = tune_of(c);
        const int g16 = all16 && (wp.skip_t || tn.g_max >= 16);
        const int G = g16 ? 16 : 8;
        for (int tier = 0; tier < (mixed ? 2 : 1); ++tier) {
            const int fp32 = mixed && tier == 1;
            LaunchRec L;
            long long used = 0;
            // digestion items (blocks) per pass and XCD; workgroup 8 k + x of a
            // launch runs on XCD x and takes task k of that XCD.  A bra pair's
            // pieces and density groups all run on one XCD, consecutively, so
            // the tasks an XCD runs together read the same density rows
            // through its L2; blocks go to the XCD with the least work so far.
            std::vector<DigItem> xq[2][8];
            int xtasks[2][8] = {};
            // the launch's blocks in list order: their items per pass, and work
            std::vector<std::array<DigItem, 2>> pend;
            std::vector<double> pwork;
            int npass = 1;
            auto flush = [&]() {
                if (L.neri > 0) {
                    double xwork[8] = {};
                    for (size_t k = 0; k < pend.size(); ++k) {
                        const int x = static_cast<int>(std::min_element(xwork, xwork + 8) - xwork);
                        xwork[x] += pwork[k];
                        for (int ps = 0; ps < npass; ++ps) {
                            DigItem d = pend[k][ps];
                            d.kstart = xtasks[ps][x];
                            xtasks[ps][x] += d.nparts * d.ngroups;
                            xq[ps][x].push_back(d);
                        }
                    }
                    for (int ps = 0; ps < 2; ++ps) {
                        size_t kmax = 0;
                        int tmax = 0;
                        for (int x = 0; x < 8; ++x) {
                            kmax = std::max(kmax, xq[ps][x].size());
                            tmax = std::max(tmax, xtasks[ps][x]);
                        }
                        DigItem idle{};
                        idle.kstart = std::numeric_limits<int>::max();
                        idle.ngroups = 1;
                        for (size_t k = 0; k < kmax; ++k)
                            for (int x = 0; x < 8; ++x) wp.dig[ps].push_back(k < xq[ps][x].size() ? xq[ps][x][k] : idle);
                        L.ndig[ps] = static_cast<int>(8 * kmax);
                        L.dig_blocks[ps] = static_cast<unsigned>(8 * tmax);
                    }
                    wp.launches.push_back(L);
                }
                for (auto& v : xq)
                    for (auto& w : v) w.clear();
                for (auto& v : xtasks)
                    for (int& t : v) t = 0;
                pend.clear();
                pwork.clear();
                LaunchRec fresh;
                fresh.cls = c;
                fresh.fp32 = fp32;
                fresh.g16 = g16;
                fresh.dig_kernel = tn.dig_kernel;
                fresh.eri_block = tn.eri_block;
                fresh.eri0 = static_cast<int>(wp.eri.size());
                fresh.dig0[0] = static_cast<int>(wp.dig[0].size());
                fresh.dig0[1] = static_cast<int>(wp.dig[1].size());
                L = fresh;
                used = 0;
            };
            flush();
            for (size_t mi = 0; mi < mols.size(); ++mi) {
                jk_basis_s* h = mols[mi].h;
                const int nd = mols[mi].nd;
                const ClassList& CL = h->lists[c];
                if (CL.count == 0) continue;
                const int nblk = static_cast<int>(CL.blocks.size());
                const int bbeg = tier ? CL.nblk64 : 0, bend = (tier || !mixed) ? nblk : CL.nblk64;
                if (bbeg >= bend) continue;
                const long long nq_tier = mixed ? (tier ? CL.count - CL.n64 : CL.n64) : CL.count;
                const double prim_tier = mixed ? CL.prim_quartets[tier] : CL.prim_quartets[0] + CL.prim_quartets[1];
                const double prim_avg = prim_tier / static_cast<double>(std::max<long long>(nq_tier, 1));
                // density groups holding at least one of the nd densities (the
                // padding of the density stride beyond them is never digested)
                const int ngroups = (nd + G - 1) / G;
                for (int b0 = bbeg; b0 < bend;) {
                    const long long q0 = CL.blocks[b0].x;
                    int b1 = b0;
                    while (b1 < bend && (CL.blocks[b1].x + CL.blocks[b1].y - q0) * NF <= cap - used) ++b1;
                    if (b1 == b0) {
                        if (used > 0) {
                            flush();
                            continue;
                        }
                        return fail(JK_EDEVICE, "internal: a bra-pair block exceeds the work buffer");
                    }
                    const long long n = CL.blocks[b1 - 1].x + CL.blocks[b1 - 1].y - q0;
                    EriItem e{};
                    e.quartets = CL.dev + q0;
                    e.n = n;
                    e.tile_off = used;
                    e.blk0 = L.eri_blocks;
                    e.mol = static_cast<int>(mi);
                    wp.eri.push_back(e);
                    L.neri++;
                    L.eri_blocks += (n + tn.eri_block - 1) / tn.eri_block;
                    // one-pass digestion (kernel 3) has no pass D
                    npass = o->want_k && tn.dig_kernel != 3 ? 2 : 1;
                    for (int k = b0; k < b1; ++k) {
                        pend.emplace_back();
                        pwork.push_back(static_cast<double>(CL.blocks[k].y) * ngroups);
                        for (int ps = 0; ps < npass; ++ps) {
                            DigItem& d = pend.back()[ps];
                            d = DigItem{};
                            d.kin = ps ? CL.dev_kind : CL.dev_kin;
                            d.pos = CL.dev_pos;
                            d.bra = CL.block_bra[k];
                            d.blk0 = CL.blocks[k].x;
                            d.chunk_q0 = q0;
                            d.chunk_n = n;
                            d.tile_off = used;
                            d.len = CL.blocks[k].y;
                            d.parts = CL.dev_parts[ps] + CL.part_off[ps][k];
                            d.nparts = CL.part_off[ps][k + 1] - CL.part_off[ps][k];
                            d.ngroups = ngroups;
                            d.mol = static_cast<int>(mi);
                        }
                    }
                    const double ef = n * (prim_avg * (kClassCost[c].prim_flops + kClassCost[c].vrr_flops) +
                                           kClassCost[c].hrr_flops);
                    // pass C: J_ab and J_cd (2 FMA), K_ac and K_bc with D and D^T (4 FMA);
                    // pass D: K_ad and K_bd with D and D^T (4 FMA) per function quartet and density
                    const double fq = static_cast<double>(n) * NF * nd;
                    const bool one = tn.dig_kernel == 3;
                    const double dfc = fq * 2.0 * ((o->want_j ? 2 : 0) + (o->want_k ? (one ? 8 : 4) : 0));
                    const double dfd = one ? 0.0 : fq * 2.0 * (o->want_k ? 4 : 0);
                    const double df = dfc + dfd;
                    L.eri_flops += ef;
                    L.dig_flops[0] += dfc;
                    L.dig_flops[1] += dfd;
                    L.quartets += n;
                    L.tile_bytes += static_cast<double>(n) * NF * (fp32 ? sizeof(float) : sizeof(double));
                    wp.stats[0] += n;
                    if (fp32) wp.stats[1] += n;
                    wp.stats[2] += static_cast<double>(n) * NF;
                    wp.stats[3] += n * prim_avg;
                    wp.stats[4] += ef;
                    wp.stats[5] += df;
                    used += n * NF;
                    wp.tile_elems = std::max(wp.tile_elems, used);
                    b0 = b1;
                }
            }
            flush();
        }
    }
    return JK_OK;
}

// Per-molecule workspace: densities and accumulators.
struct MolSpace {
    size_t off_D, off_J, off_K, off_KT, off_dmax, off_DS, off_Df, off_DSf, off_DT, off_DTf, bytes;
};

inline size_t al256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

MolSpace mol_space(const jk_basis_s* h, int nd, const jk_build_opts* o) {
    MolSpace m{};
    const size_t mat = static_cast<size_t>(h->nc) * h->nc * dens_stride(nd) * sizeof(double);
    size_t off = 0;
    m.off_D = off;
    off += al256(mat);
    m.off_J = off;
    if (o->want_j) off += al256(mat);
    m.off_K = off;
    if (o->want_k) off += al256(mat);
    m.off_KT = off;
    if (o->want_k) off += al256(mat);
    m.off_dmax = off;
    off += al256(static_cast<size_t>(h->ns) * h->ns * sizeof(double));
    m.off_DS = off;
    const size_t ds = static_cast<size_t>(h->ds_units) * dens_stride(nd);
    if (o->want_j) off += al256(ds * sizeof(double));
    // FP32 copies for the FP32 tier of mixed builds
    const bool mixed = o->precision == JK_MIXED;
    m.off_Df = off;
    if (mixed && o->want_k) off += al256(mat / 2);
    m.off_DSf = off;
    if (mixed && o->want_j) off += al256(ds * sizeof(float));
    // transposed densities for the D^T exchange contractions (D itself when
    // the caller promises symmetric densities)
    const bool dt = o->want_k && !o->symmetric_hint;
    m.off_DT = off;
    if (dt) off += al256(mat);
    m.off_DTf = off;
    if (dt && mixed) off += al256(mat / 2);
    m.bytes = off;
    return m;
}

// A cached plan of a single-molecule build, with its items on the device.
struct CachedPlan {
    int nd, mixed, want_j, want_k, sym, gen, tgen;
    WorkPlan wp;
    EriItem* d_eri = nullptr;
    DigItem* d_dig[2] = {nullptr, nullptr};
};

bool valid_opts(const jk_build_opts* o) {
    return o && (o->precision == JK_FP64 || o->precision == JK_MIXED) && std::isfinite(o->schwarz_tol) &&
           o->schwarz_tol >= 0 && (o->symmetric_hint == 0 || o->symmetric_hint == 1) &&
           (o->want_j == 0 || o->want_j == 1) && (o->want_k == 0 || o->want_k == 1);
}

}  // namespace

extern "C" {

void jk_default_opts(jk_build_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = JK_FP64;
    o->schwarz_tol = 1e-12;
    o->fp32_bound = 1e-6;
    o->want_j = 1;
    o->want_k = 1;
}

const char* jk_last_error(void) { return g_err.c_str(); }

int jk_create_basis(const jk_basis_desc* d, jk_basis_t* out) {
    if (!out) return fail(JK_EINVAL, "jk_create_basis: out is NULL");
    *out = nullptr;
    if (!d) return fail(JK_EINVAL, "jk_create_basis: descriptor is NULL");
    if (d->natoms < 1 || d->nshells < 1) return fail(JK_EINVAL, "jk_create_basis: natoms and nshells must be >= 1");
    if (!d->xyz || !d->shell_atom || !d->shell_l || !d->shell_nprim || !d->exps || !d->coefs)
        return fail(JK_EINVAL, "jk_create_basis: NULL array in descriptor");
    if (d->spherical != 0 && d->spherical != 1) return fail(JK_EINVAL, "jk_create_basis: spherical must be 0 or 1");
    for (int i = 0; i < 3 * d->natoms; ++i)
        if (!std::isfinite(d->xyz[i])) return fail(JK_EINVAL, "jk_create_basis: non-finite coordinate");
    long long po = 0;
    for (int s = 0; s < d->nshells; ++s) {
        if (d->shell_l[s] < 0 || d->shell_l[s] > JK_MAX_L)
            return fail(JK_EINVAL, "jk_create_basis: shell %d has l=%d outside 0..%d", s, d->shell_l[s], JK_MAX_L);
        if (d->shell_nprim[s] < 1 || d->shell_nprim[s] > JK_MAX_PRIM)
            return fail(JK_EINVAL, "jk_create_basis: shell %d has nprim=%d outside 1..%d", s, d->shell_nprim[s],
                        JK_MAX_PRIM);
        if (d->shell_atom[s] < 0 || d->shell_atom[s] >= d->natoms)
            return fail(JK_EINVAL, "jk_create_basis: shell %d on atom %d outside 0..%d", s, d->shell_atom[s],
                        d->natoms - 1);
        for (int k = 0; k < d->shell_nprim[s]; ++k) {
            const double a = d->exps[po + k], c = d->coefs[po + k];
            if (!(a > 0.0) || !std::isfinite(a))
                return fail(JK_EINVAL, "jk_create_basis: shell %d exponent %d is %g (must be > 0 and finite)", s, k, a);
            if (!std::isfinite(c)) return fail(JK_EINVAL, "jk_create_basis: shell %d coefficient %d not finite", s, k);
        }
        po += d->shell_nprim[s];
    }

    std::unique_ptr<jk_basis_s> h(new jk_basis_s());
    HIPC(hipGetDevice(&h->device));
    // device address of the no-alloc entry point's static workspace (once per device)
    HIPC(static_scratch_init());
    HIPC(hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking));
    const int ns = d->nshells;
    h->natoms = d->natoms;
    h->ns = ns;
    h->spherical = d->spherical;
    // user layout
    std::vector<long long> prim0(ns + 1, 0);
    h->user_f0.assign(ns + 1, 0);
    for (int s = 0; s < ns; ++s) {
        prim0[s + 1] = prim0[s] + d->shell_nprim[s];
        const int l = d->shell_l[s];
        const int nfn = (d->spherical && l == 2) ? 5 : ncart(l);
        h->user_f0[s + 1] = h->user_f0[s] + nfn;
    }
    h->nf = h->user_f0[ns];
    // internal order: by l, stable
    h->user_of_int.resize(ns);
    for (int s = 0; s < ns; ++s) h->user_of_int[s] = s;
    std::stable_sort(h->user_of_int.begin(), h->user_of_int.end(),
                     [&](int u, int v) { return d->shell_l[u] < d->shell_l[v]; });
    h->int_of_user.resize(ns);
    h->l_int.resize(ns);
    h->f0_int.resize(ns + 1);
    h->ncart_int.resize(ns);
    h->nprim_int.resize(ns);
    h->centre_int.resize(3 * ns);
    h->exps_int.resize(ns);
    h->w_int.resize(ns);
    int fc = 0;
    for (int si = 0; si < ns; ++si) {
        const int su = h->user_of_int[si];
        h->int_of_user[su] = si;
        const int l = d->shell_l[su];
        h->l_int[si] = l;
        h->f0_int[si] = fc;
        h->ncart_int[si] = ncart(l);
        fc += ncart(l);
        const int np = d->shell_nprim[su];
        h->nprim_int[si] = np;
        for (int k = 0; k < 3; ++k) h->centre_int[3 * si + k] = d->xyz[3 * d->shell_atom[su] + k];
        // contraction weights: coefficient x primitive norm, rescaled so the
        // x^l component has unit self-overlap; same-centre overlap of two
        // normalized primitives is (2 sqrt(ab)/(a+b))^(l+3/2)
        std::vector<double> ex(np), w(np);
        for (int k = 0; k < np; ++k) {
            ex[k] = d->exps[prim0[su] + k];
            w[k] = d->coefs[prim0[su] + k];
        }
        double s2 = 0.0;
        for (int i = 0; i < np; ++i)
            for (int j = 0; j < np; ++j)
                s2 += w[i] * w[j] * std::pow(2.0 * std::sqrt(ex[i] * ex[j]) / (ex[i] + ex[j]), l + 1.5);
        if (!(s2 > 0.0) || !std::isfinite(s2))
            return fail(JK_EINVAL, "jk_create_basis: shell %d contraction has zero norm", su);
        const double sc = 1.0 / std::sqrt(s2);
        for (int k = 0; k < np; ++k) {
            const double a = ex[k];
            w[k] *= sc * std::sqrt(std::pow(2.0 * a / kPi, 1.5) * std::pow(4.0 * a, l) / dfact(2 * l - 1));
        }
        h->exps_int[si] = ex;
        h->w_int[si] = w;
    }
    h->f0_int[ns] = fc;
    h->nc = fc;
    if (fc > 0xffff)
        return fail(JK_EUNSUPPORTED, "jk_create_basis: %d Cartesian functions (at most 65535)", fc);

    // shell pairs (a >= b internal, la >= lb) and primitive pairs
    h->pair_id.assign(static_cast<size_t>(ns) * ns, -1);
    const double E0 = std::sqrt(2.0) * std::pow(kPi, 1.25);
    for (int a = 0; a < ns; ++a) {
        for (int b = 0; b <= a; ++b) {
            PairInfo P{};
            const double* A = &h->centre_int[3 * a];
            const double* B = &h->centre_int[3 * b];
            double ab2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                P.A[k] = A[k];
                P.AB[k] = A[k] - B[k];
                ab2 += P.AB[k] * P.AB[k];
            }
            P.sa = a;
            P.sb = b;
            P.fa = h->f0_int[a];
            P.fb = h->f0_int[b];
            P.prim_off = static_cast<int>(h->prims.size());
            // primitive pairs whose prefactor, times the largest power of the
            // pair separation the recurrences can apply, is below
            // kPrimPairTol are left out
            const double ang = std::pow(std::max(1.0, std::sqrt(ab2)), h->l_int[a] + h->l_int[b]);
            for (int i = 0; i < h->nprim_int[a]; ++i)
                for (int j = 0; j < h->nprim_int[b]; ++j) {
                    const double al = h->exps_int[a][i], be = h->exps_int[b][j];
                    const double p = al + be;
                    PrimPair pp{};
                    pp.p = p;
                    for (int k = 0; k < 3; ++k) pp.P[k] = (al * A[k] + be * B[k]) / p;
                    pp.E = E0 * h->w_int[a][i] * h->w_int[b][j] * std::exp(-al * be / p * ab2) / p;
                    pp.o2p = 0.5 / p;
                    if (std::fabs(pp.E) * ang >= kPrimPairTol) h->prims.push_back(pp);
                }
            P.nprim = static_cast<int>(h->prims.size()) - P.prim_off;
            const int id = static_cast<int>(h->pairs.size());
            h->pair_id[static_cast<size_t>(a) * ns + b] = id;
            h->pairs.push_back(P);
            h->pairs_of_class[pair_class(h->l_int[a], h->l_int[b])].push_back(id);
        }
    }
    // device layout of the primitive-pair records: groups of kPrimLane
    // consecutive pair ids, record j of every pair of a group side by side
    {
        const int npair = static_cast<int>(h->pairs.size());
        std::vector<long long> slot0(npair);
        long long nslot = 0;
        for (int g0 = 0; g0 < npair; g0 += kPrimLane) {
            const int g1 = std::min(npair, g0 + kPrimLane);
            int mx = 0;
            for (int i = g0; i < g1; ++i) {
                mx = std::max(mx, h->pairs[i].nprim);
                slot0[i] = nslot + (i - g0);
            }
            nslot += static_cast<long long>(kPrimLane) * mx;
        }
        if (nslot > (1ll << 30))
            return fail(JK_EUNSUPPORTED, "jk_create_basis: %lld primitive-pair slots (at most 2^30)", nslot);
        h->pslots = static_cast<int>(nslot);
        h->prim_planes.assign(static_cast<size_t>(6 * nslot), 0.0);
        double* pl = h->prim_planes.data();
        for (int i = 0; i < npair; ++i) {
            PairInfo& P = h->pairs[i];
            for (int j = 0; j < P.nprim; ++j) {
                const PrimPair& r = h->prims[static_cast<size_t>(P.prim_off) + j];
                const long long sl = slot0[i] + static_cast<long long>(kPrimLane) * j;
                pl[2 * sl] = r.p;
                pl[2 * sl + 1] = r.E;
                pl[2 * (nslot + sl)] = r.P[0];
                pl[2 * (nslot + sl) + 1] = r.P[1];
                pl[2 * (2 * nslot + sl)] = r.P[2];
                pl[2 * (2 * nslot + sl) + 1] = r.o2p;
            }
            P.prim_off = static_cast<int>(slot0[i]);
        }
        std::vector<PrimPair>().swap(h->prims);
    }

    // basis-change maps
    std::vector<CartMap> cmap(h->nc);
    std::vector<UserMap> umap(h->nf);
    for (int si = 0; si < ns; ++si) {
        const int su = h->user_of_int[si];
        const int l = h->l_int[si];
        const int cf = h->f0_int[si], uf = h->user_f0[su];
        if (l == 2 && h->spherical) {
            for (int i = 0; i < 6; ++i) cmap[cf + i] = CartMap{};
            for (int m = 0; m < 5; ++m) {
                UserMap um{};
                for (int i = 0; i < 6; ++i) {
                    const double c = kSphD[m][i];
                    if (c == 0.0) continue;
                    um.idx[um.n] = cf + i;
                    um.c[um.n] = c;
                    ++um.n;
                    CartMap& cm = cmap[cf + i];
                    cm.idx[cm.n] = uf + m;
                    cm.c[cm.n] = c;
                    ++cm.n;
                }
                umap[uf + m] = um;
            }
        } else {
            for (int i = 0; i < ncart(l); ++i) {
                CartMap cm{};
                cm.idx[0] = uf + i;
                cm.c[0] = 1.0;
                cm.n = 1;
                cmap[cf + i] = cm;
                UserMap um{};
                um.idx[0] = cf + i;
                um.c[0] = 1.0;
                um.n = 1;
                umap[uf + i] = um;
            }
        }
    }
    std::vector<int> sf0(h->f0_int.begin(), h->f0_int.begin() + ns);
    int rc;
    if ((rc = upload(&h->d_pairs, h->pairs))) return rc;
    if ((rc = upload(&h->d_prims, h->prim_planes))) return rc;
    std::vector<double>().swap(h->prim_planes);
    if ((rc = upload(&h->d_boys, boys_table()))) return rc;
    {
        std::vector<float> t32(boys_table().begin(), boys_table().end());
        if ((rc = upload(&h->d_boys32, t32))) return rc;
    }
    if ((rc = upload(&h->d_cmap, cmap))) return rc;
    if ((rc = upload(&h->d_umap, umap))) return rc;
    if ((rc = upload(&h->d_shell_f0, sf0))) return rc;
    if ((rc = upload(&h->d_shell_nf, h->ncart_int))) return rc;
    {
        // packed symmetrized-density records: shell pair (c, d), c >= d, in pair order
        std::vector<int> off(static_cast<size_t>(ns) * ns, -1);
        long long u = 0;
        for (const PairInfo& P : h->pairs) {
            off[static_cast<size_t>(P.sa) * ns + P.sb] = static_cast<int>(u);
            u += static_cast<long long>(h->ncart_int[P.sa]) * h->ncart_int[P.sb];
        }
        h->ds_units = u;
        if ((rc = upload(&h->d_ds_off, off))) return rc;
    }
    if ((rc = compute_schwarz(h.get()))) return rc;
    HIPC(hipMemcpy(h->d_pairs, h->pairs.data(), h->pairs.size() * sizeof(PairInfo), hipMemcpyHostToDevice));
    if ((rc = ensure_lists(h.get(), 1e-12, 1e-6))) return rc;
    *out = h.release();
    return JK_OK;
}

int jk_nbf(jk_basis_t h) { return h ? h->nf : fail(JK_EINVAL, "jk_nbf: NULL handle"); }

void jk_destroy(jk_basis_t h) {
    if (!h) return;
    for (CachedPlan* cp : h->plans) free_plan(cp);
    h->plans.clear();
    delete h;
}

int64_t jk_quartet_count(jk_basis_t h, double tol) {
    if (!h || !(tol >= 0)) return fail(JK_EINVAL, "jk_quartet_count: bad arguments");
    long long n = 0;
    for (int X = 0; X < kNumPairClass; ++X)
        for (int Y = 0; Y <= X; ++Y)
            for (int b : h->pairs_of_class[X])
                for (int k : h->pairs_of_class[Y]) {
                    if (X == Y && k > b) continue;
                    if (h->pairs[b].q * h->pairs[k].q >= tol) ++n;
                }
    return n;
}

int jk_last_stats(jk_basis_t h, double out[6]) {
    if (!h || !out) return fail(JK_EINVAL, "jk_last_stats: bad arguments");
    std::lock_guard<std::mutex> g(h->mu);
    for (int i = 0; i < 6; ++i) out[i] = h->stats[i];
    return JK_OK;
}

}  // extern "C"

namespace {

// Launch every class/tier of a plan on stream s.  prof: handle that records
// per-kernel events when profiling is on (single-molecule builds).
// Launch every class/tier of a plan: launch i runs on lane i % kLanes (lane 0
// the caller's stream s, lane 1 the helper stream aux, forked from and joined
// back into s) with that lane's integral work buffer and scratch, each tb
// bytes at work + 2 lane tb and work + (2 lane + 1) tb.
hipError_t run_plan(const WorkPlan& wp, const EriItem* d_eri, DigItem* const d_dig[2], const MolDesc& mol0,
                    const MolDesc* d_mols, char* work, size_t tb, const jk_build_opts* o, const double* boys,
                    const float* boys32, hipStream_t s, hipStream_t aux, jk_basis_s* prof) {
    hipError_t e = hipSuccess;
    // while profiling, one lane: every kernel's event time is then its own
    const int lanes = (aux && wp.launches.size() > 1 && !(prof && prof->profiling)) ? kLanes : 1;
    hipEvent_t fork = nullptr, join = nullptr;
    if (lanes > 1) {
        e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(aux, fork, 0);
        if (e != hipSuccess) {
            if (fork) (void)hipEventDestroy(fork);
            if (join) (void)hipEventDestroy(join);
            return e;
        }
    }
    for (size_t li = 0; li < wp.launches.size() && e == hipSuccess; ++li) {
        const LaunchRec& L = wp.launches[li];
        const int lane = static_cast<int>(li % lanes);
        const hipStream_t ls = lane ? aux : s;
        void* const tiles = work + 2 * lane * tb;
        void* const scratch = work + (2 * lane + 1) * tb;
        EriTileArgs ea{};
        ea.items = d_eri + L.eri0;
        ea.nitems = L.neri;
        ea.nblocks = L.eri_blocks;
        ea.mol0 = mol0;
        ea.mols = d_mols;
        ea.boys = boys;
        ea.boys32 = boys32;
        ea.tol = o->schwarz_tol;
        ea.tiles = tiles;
        ea.scratch = scratch;
        ea.kept = (prof && prof->profiling && prof->d_kept) ? prof->d_kept + L.fp32 * kNumClass + L.cls : nullptr;
        ea.block = L.eri_block;
        DigestArgs da[2]{};
        for (int ps = 0; ps < 2; ++ps) {
            da[ps].items = d_dig[ps] + L.dig0[ps];
            da[ps].nitems = L.ndig[ps];
            da[ps].mol0 = mol0;
            da[ps].mols = d_mols;
            da[ps].tiles = tiles;
            da[ps].dcopy = scratch;
            da[ps].want_j = o->want_j;
            da[ps].want_k = o->want_k;
            da[ps].skip_t = wp.skip_t ? 1 : 0;
            da[ps].nblocks = L.ndig[ps] > 0 ? L.dig_blocks[ps] : 0;
        }
        const bool timed = prof && prof->profiling;
        hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
        if (timed) {
            for (auto& x : ev)
                if (e == hipSuccess) e = hipEventCreate(&x);
            if (e == hipSuccess) e = hipEventRecord(ev[0], ls);
            if (e != hipSuccess) break;
        }
        e = launch_eri_tile(L.cls, ea, ls, L.fp32);
        if (e == hipSuccess && timed) e = hipEventRecord(ev[1], ls);
        if (e == hipSuccess) e = launch_digest(L.cls, da[0], ls, L.fp32, 0, L.g16, L.dig_kernel);
        if (e == hipSuccess && timed) e = hipEventRecord(ev[2], ls);
        if (e == hipSuccess) e = launch_digest(L.cls, da[1], ls, L.fp32, 1, L.g16, L.dig_kernel);
        if (e == hipSuccess && timed) e = hipEventRecord(ev[3], ls);
        if (e != hipSuccess) break;
        if (timed) {
            std::lock_guard<std::mutex> g(prof->mu);
            prof->prof.push_back({0 + 2 * L.fp32, L.cls, ev[0], ev[1], L.eri_flops, L.quartets, L.tile_bytes});
            prof->prof.push_back({1 + 2 * L.fp32, L.cls, ev[1], ev[2], L.dig_flops[0], L.quartets, L.tile_bytes});
            if (L.ndig[1] > 0)
                prof->prof.push_back({4 + L.fp32, L.cls, ev[2], ev[3], L.dig_flops[1], L.quartets, L.tile_bytes});
            else
                (void)hipEventDestroy(ev[3]);
        }
    }
    if (lanes > 1) {
        // join lane 1 back into s whatever happened, so nothing after the
        // build on s (the back-transform, a workspace free) runs before it
        hipError_t e2 = hipEventRecord(join, aux);
        if (e2 == hipSuccess) e2 = hipStreamWaitEvent(s, join, 0);
        if (e == hipSuccess) e = e2;
        (void)hipEventDestroy(fork);
        (void)hipEventDestroy(join);
    }
    return e;
}

void free_plan(CachedPlan* cp) {
    if (!cp) return;
    (void)hipFree(cp->d_eri);
    (void)hipFree(cp->d_dig[0]);
    (void)hipFree(cp->d_dig[1]);
    delete cp;
}

// The cached plan of a single-molecule build (created on first use).
int get_plan(jk_basis_s* h, int nd, const jk_build_opts* o, CachedPlan** out) {
    const int mixed = o->precision == JK_MIXED;
    int tgen;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        tgen = g_tune_gen;
    }
    std::lock_guard<std::mutex> g(h->mu);
    for (CachedPlan* cp : h->plans)
        if (cp->nd == nd && cp->mixed == mixed && cp->want_j == o->want_j && cp->want_k == o->want_k &&
            cp->sym == o->symmetric_hint && cp->gen == h->list_gen && cp->tgen == tgen) {
            *out = cp;
            return JK_OK;
        }
    CachedPlan* cp = new CachedPlan();
    cp->nd = nd;
    cp->mixed = mixed;
    cp->want_j = o->want_j;
    cp->want_k = o->want_k;
    cp->sym = o->symmetric_hint;
    cp->gen = h->list_gen;
    cp->tgen = tgen;
    int rc = plan_work({MolRun{h, nd}}, o, kTileCapElems, cp->wp);
    if (!rc) rc = upload(&cp->d_eri, cp->wp.eri);
    if (!rc) rc = upload(&cp->d_dig[0], cp->wp.dig[0]);
    if (!rc) rc = upload(&cp->d_dig[1], cp->wp.dig[1]);
    if (rc) {
        free_plan(cp);
        return rc;
    }
    h->plans.push_back(cp);
    *out = cp;
    return JK_OK;
}

// The cached plan of a single-molecule build, or nullptr if none was made
// yet for these options (never creates one).
CachedPlan* find_plan(jk_basis_s* h, int nd, const jk_build_opts* o) {
    const int mixed = o->precision == JK_MIXED;
    int tgen;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        tgen = g_tune_gen;
    }
    std::lock_guard<std::mutex> g(h->mu);
    for (CachedPlan* cp : h->plans)
        if (cp->nd == nd && cp->mixed == mixed && cp->want_j == o->want_j && cp->want_k == o->want_k &&
            cp->sym == o->symmetric_hint && cp->gen == h->list_gen && cp->tgen == tgen)
            return cp;
    return nullptr;
}

// Whether the resident lists serve a build with tolerance tol and FP32
// bound `bound` (bound < 0: any) without being rebuilt.
bool lists_ready(jk_basis_s* h, double tol, double bound) {
    std::lock_guard<std::mutex> g(h->mu);
    int tg;
    {
        std::lock_guard<std::mutex> g2(g_tune_mu);
        tg = g_tune_gen;
    }
    return h->list_tol >= 0 && h->list_tol <= tol && (bound < 0 || h->list_bound == bound) && h->tune_gen == tg;
}

// Pre- and post-stages of one molecule: D_cart, density screen, zeroed
// accumulators; back-transform of J and K.
hipError_t mol_pre(const jk_basis_s* h, int nd, const double* D, const jk_build_opts* o, char* base,
                   const MolSpace& ms, MolDesc& md, hipStream_t s) {
    double* Dc = reinterpret_cast<double*>(base + ms.off_D);
    double* Jc = o->want_j ? reinterpret_cast<double*>(base + ms.off_J) : nullptr;
    double* Kc = o->want_k ? reinterpret_cast<double*>(base + ms.off_K) : nullptr;
    double* KTc = o->want_k ? reinterpret_cast<double*>(base + ms.off_KT) : nullptr;
    double* dmax = reinterpret_cast<double*>(base + ms.off_dmax);
    const int ndp = dens_stride(nd);
    const long long mat = static_cast<long long>(h->nc) * h->nc * ndp;
    double* DS = o->want_j ? reinterpret_cast<double*>(base + ms.off_DS) : nullptr;
    const bool mixed = o->precision == JK_MIXED;
    float* Df = mixed && o->want_k ? reinterpret_cast<float*>(base + ms.off_Df) : nullptr;
    float* DSf = mixed && o->want_j ? reinterpret_cast<float*>(base + ms.off_DSf) : nullptr;
    const bool dt = o->want_k && !o->symmetric_hint;
    double* DT = dt ? reinterpret_cast<double*>(base + ms.off_DT) : nullptr;
    float* DTf = dt && mixed ? reinterpret_cast<float*>(base + ms.off_DTf) : nullptr;
    hipError_t e = launch_sph2cart(D, nd, h->nf, h->d_cmap, h->nc, ndp, Dc, s);
    if (e == hipSuccess) e = launch_pair_dmax(Dc, h->nc, ndp, nd, h->d_shell_f0, h->d_shell_nf, h->ns, dmax, s);
    if (e == hipSuccess && DS)
        e = launch_pair_ds(Dc, h->nc, ndp, nd, h->d_pairs, static_cast<int>(h->pairs.size()), h->d_shell_nf,
                           h->d_ds_off, h->ns, DS, s);
    if (e == hipSuccess && Df) e = launch_to_f32(Dc, Df, mat, s);
    if (e == hipSuccess && DT) e = launch_transpose(Dc, h->nc, ndp, DT, s);
    if (e == hipSuccess && DTf) e = launch_to_f32(DT, DTf, mat, s);
    if (e == hipSuccess && DSf) e = launch_to_f32(DS, DSf, static_cast<long long>(h->ds_units) * ndp, s);
    if (e == hipSuccess && Jc) e = launch_zero(Jc, mat, s);
    if (e == hipSuccess && Kc) e = launch_zero(Kc, mat, s);
    if (e == hipSuccess && KTc) e = launch_zero(KTc, mat, s);
    md.pairs = h->d_pairs;
    md.prims = h->d_prims;
    md.pslots = h->pslots;
    md.dmax = dmax;
    md.D = Dc;
    md.J = Jc;
    md.K = Kc;
    md.KT = KTc;
    md.DS = DS;
    md.ds_off = h->d_ds_off;
    md.Df = Df;
    md.DSf = DSf;
    md.DT = DT ? DT : Dc;      // symmetric_hint: D^T = D
    md.DTf = DTf ? DTf : Df;
    md.ns = h->ns;
    md.nc = h->nc;
    md.nd = nd;
    md.ndp = ndp;
    return e;
}

// Outputs the build does not produce are never touched: their pointers are
// dropped here (the caller may pass any value for them).
hipError_t mol_post(const jk_basis_s* h, int nd, const MolDesc& md, double* J, double* K, bool skip_t,
                    hipStream_t s) {
    return launch_cart2sph(md.J, md.K, skip_t ? md.K : md.KT, nd, h->nf, h->d_umap, h->nc, md.ndp,
                           md.J ? J : nullptr, md.K ? K : nullptr, s);
}

int check_opts(const char* who, const jk_build_opts* o) {
    if (!valid_opts(o)) return fail(JK_EINVAL, "%s: invalid options", who);
    if (o->precision == JK_MIXED && !(o->fp32_bound >= 0 && std::isfinite(o->fp32_bound)))
        return fail(JK_EINVAL, "%s: fp32_bound must be finite and >= 0", who);
    return JK_OK;
}

size_t tile_bytes_of(const WorkPlan& wp) { return al256(static_cast<size_t>(wp.tile_elems) * sizeof(double)); }

struct DeviceGuard {
    int prev = -1;
    int ok(int dev) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) return fail(JK_EDEVICE, "hipGetDevice failed");
        if (cur != dev) {
            if (hipSetDevice(dev) != hipSuccess) return fail(JK_EDEVICE, "hipSetDevice(%d) failed", dev);
            prev = cur;
        }
        return JK_OK;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

extern "C" {

size_t jk_workspace_bytes(jk_basis_t h, int32_t nd, const jk_build_opts* o) {
    jk_build_opts def;
    if (!o) {
        jk_default_opts(&def);
        o = &def;
    }
    if (!h || nd < 1 || check_opts("jk_workspace_bytes", o)) return 0;
    DeviceGuard dg;
    if (dg.ok(h->device)) return 0;
    if (ensure_lists(h, o->schwarz_tol, o->precision == JK_MIXED ? o->fp32_bound : -1.0)) return 0;
    CachedPlan* cp = nullptr;
    if (get_plan(h, nd, o, &cp)) return 0;
    return mol_space(h, nd, o).bytes + 2 * kLanes * tile_bytes_of(cp->wp);
}

int jk_build(jk_basis_t h, int32_t nd, const double* D, double* J, double* K, const jk_build_opts* o) {
    jk_build_opts def;
    if (!o) {
        jk_default_opts(&def);
        o = &def;
    }
    if (!h) return fail(JK_EINVAL, "jk_build: NULL handle");
    if (nd < 1) return fail(JK_EINVAL, "jk_build: nd=%d must be >= 1", nd);
    int rc = check_opts("jk_build", o);
    if (rc) return rc;
    if (!D) return fail(JK_EINVAL, "jk_build: D is NULL");
    if (o->want_j && !J) return fail(JK_EINVAL, "jk_build: J is NULL but want_j is set");
    if (o->want_k && !K) return fail(JK_EINVAL, "jk_build: K is NULL but want_k is set");
    DeviceGuard dg;
    if ((rc = dg.ok(h->device))) return rc;
    const int mixed = o->precision == JK_MIXED;
    if ((rc = ensure_lists(h, o->schwarz_tol, mixed ? o->fp32_bound : -1.0))) return rc;
    CachedPlan* cp = nullptr;
    if ((rc = get_plan(h, nd, o, &cp))) return rc;
    hipStream_t s = static_cast<hipStream_t>(o->stream);
    const MolSpace ms = mol_space(h, nd, o);
    const size_t tb = tile_bytes_of(cp->wp);
    const size_t total = ms.bytes + 2 * kLanes * tb;
    char* ws = static_cast<char*>(o->workspace);
    bool own = false;
    if (ws) {
        if (o->workspace_bytes < total)
            return fail(JK_EINVAL, "jk_build: workspace of %zu bytes is below the %zu required", o->workspace_bytes,
                        total);
    } else {
        hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&ws), total, s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(JK_ENOMEM, "jk_build: cannot allocate %zu bytes of workspace (%s)", total,
                        hipGetErrorString(e));
        }
        own = true;
    }
    MolDesc md{};
    hipError_t e = mol_pre(h, nd, D, o, ws, ms, md, s);
    if (e == hipSuccess)
        e = run_plan(cp->wp, cp->d_eri, cp->d_dig, md, nullptr, ws + ms.bytes, tb, o, h->d_boys, h->d_boys32, s,
                     h->aux, h);
    if (e == hipSuccess) e = mol_post(h, nd, md, J, K, cp->wp.skip_t, s);
    if (own) {
        hipError_t e2 = hipFreeAsync(ws, s);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return fail(JK_EDEVICE, "jk_build: %s", hipGetErrorString(e));
    {
        std::lock_guard<std::mutex> g(h->mu);
        for (int i = 0; i < 6; ++i) h->stats[i] = cp->wp.stats[i];
    }
    return JK_OK;
}

int jk_build_noalloc(jk_basis_t h, int32_t nd, const double* D, double* J, double* K, const jk_build_opts* o) {
    jk_build_opts def;
    if (!o) {
        jk_default_opts(&def);
        o = &def;
    }
    if (!h) return fail(JK_EINVAL, "jk_build_noalloc: NULL handle");
    if (nd < 1) return fail(JK_EINVAL, "jk_build_noalloc: nd=%d must be >= 1", nd);
    int rc = check_opts("jk_build_noalloc", o);
    if (rc) return rc;
    if (!D) return fail(JK_EINVAL, "jk_build_noalloc: D is NULL");
    if (o->want_j && !J) return fail(JK_EINVAL, "jk_build_noalloc: J is NULL but want_j is set");
    if (o->want_k && !K) return fail(JK_EINVAL, "jk_build_noalloc: K is NULL but want_k is set");
    DeviceGuard dg;
    if ((rc = dg.ok(h->device))) return rc;
    const int mixed = o->precision == JK_MIXED;
    CachedPlan* cp = lists_ready(h, o->schwarz_tol, mixed ? o->fp32_bound : -1.0) ? find_plan(h, nd, o) : nullptr;
    if (!cp)
        return fail(JK_EINVAL,
                    "jk_build_noalloc: no launch plan for nd=%d and these options; prepare it once with "
                    "jk_workspace_bytes(h, nd, o), which may allocate",
                    nd);
    const MolSpace ms = mol_space(h, nd, o);
    const size_t tb = tile_bytes_of(cp->wp);
    const size_t total = ms.bytes + 2 * kLanes * tb;
    if (total > kNoAllocScratchBytes)
        return fail(JK_ENOMEM,
                    "jk_build_noalloc: the build needs %zu bytes of workspace, above the %zu of the static buffer",
                    total, kNoAllocScratchBytes);
    char* ws = static_cast<char*>(static_scratch(h->device));
    if (!ws) return fail(JK_EDEVICE, "jk_build_noalloc: static workspace not set up on device %d", h->device);
    hipStream_t s = static_cast<hipStream_t>(o->stream);
    MolDesc md{};
    hipError_t e = mol_pre(h, nd, D, o, ws, ms, md, s);
    if (e == hipSuccess)
        e = run_plan(cp->wp, cp->d_eri, cp->d_dig, md, nullptr, ws + ms.bytes, tb, o, h->d_boys, h->d_boys32, s,
                     nullptr, nullptr);   // one launch lane: no events or helper-stream work
    if (e == hipSuccess) e = mol_post(h, nd, md, J, K, cp->wp.skip_t, s);
    if (e != hipSuccess) return fail(JK_EDEVICE, "jk_build_noalloc: %s", hipGetErrorString(e));
    {
        std::lock_guard<std::mutex> g(h->mu);
        for (int i = 0; i < 6; ++i) h->stats[i] = cp->wp.stats[i];
    }
    return JK_OK;
}

}  // extern "C"

namespace {

// Host memory released by the stream once the work before it has run.
void free_host_cb(void* p) { std::free(p); }

struct BatchSetup {
    std::vector<MolRun> runs;
    WorkPlan wp;
    std::vector<MolSpace> ms;
    std::vector<size_t> mol_off;
    size_t off_tiles = 0, tb = 0, off_items = 0, total = 0;
    size_t eri_bytes = 0, dig_bytes[2] = {0, 0}, mol_bytes = 0;
};

int batch_setup(int32_t nmol, const jk_basis_t* hs, const int32_t* nd, const jk_build_opts* o, BatchSetup& b) {
    if (nmol < 1 || !hs || !nd) return fail(JK_EINVAL, "jk_build_batch: nmol >= 1 and non-NULL arrays required");
    const int mixed = o->precision == JK_MIXED;
    for (int i = 0; i < nmol; ++i) {
        if (!hs[i]) return fail(JK_EINVAL, "jk_build_batch: handle %d is NULL", i);
        if (nd[i] < 1) return fail(JK_EINVAL, "jk_build_batch: nd[%d]=%d must be >= 1", i, nd[i]);
        if (hs[i]->device != hs[0]->device) return fail(JK_EINVAL, "jk_build_batch: handles on different devices");
        int rc = ensure_lists(hs[i], o->schwarz_tol, mixed ? o->fp32_bound : -1.0);
        if (rc) return rc;
        b.runs.push_back(MolRun{hs[i], nd[i]});
    }
    int rc = plan_work(b.runs, o, kTileCapElems, b.wp);
    if (rc) return rc;
    size_t off = 0;
    for (int i = 0; i < nmol; ++i) {
        b.ms.push_back(mol_space(hs[i], nd[i], o));
        b.mol_off.push_back(off);
        off += b.ms.back().bytes;
    }
    const size_t tb = tile_bytes_of(b.wp);
    b.tb = tb;
    b.off_tiles = off;             // kLanes pairs of (integral work buffer, scratch)
    off += 2 * kLanes * tb;
    b.off_items = off;
    b.eri_bytes = al256(std::max<size_t>(1, b.wp.eri.size()) * sizeof(EriItem));
    b.dig_bytes[0] = al256(std::max<size_t>(1, b.wp.dig[0].size()) * sizeof(DigItem));
    b.dig_bytes[1] = al256(std::max<size_t>(1, b.wp.dig[1].size()) * sizeof(DigItem));
    b.mol_bytes = al256(nmol * sizeof(MolDesc));
    off += b.eri_bytes + b.dig_bytes[0] + b.dig_bytes[1] + b.mol_bytes;
    b.total = off;
    return JK_OK;
}

}  // namespace

extern "C" {

size_t jk_batch_workspace_bytes(int32_t nmol, const jk_basis_t* h, const int32_t* nd, const jk_build_opts* o) {
    jk_build_opts def;
    if (!o) {
        jk_default_opts(&def);
        o = &def;
    }
    if (check_opts("jk_batch_workspace_bytes", o) || nmol < 1 || !h || !h[0]) return 0;
    DeviceGuard dg;
    if (dg.ok(h[0]->device)) return 0;
    BatchSetup b;
    if (batch_setup(nmol, h, nd, o, b)) return 0;
    return b.total;
}

int jk_build_batch(int32_t nmol, const jk_basis_t* hs, const int32_t* nd, const double* const* D,
                   double* const* J, double* const* K, const jk_build_opts* o) {
    jk_build_opts def;
    if (!o) {
        jk_default_opts(&def);
        o = &def;
    }
    int rc = check_opts("jk_build_batch", o);
    if (rc) return rc;
    if (nmol < 1 || !hs || !nd || !D || (o->want_j && !J) || (o->want_k && !K))
        return fail(JK_EINVAL, "jk_build_batch: NULL arrays");
    for (int i = 0; i < nmol; ++i)
        if (!D[i] || (o->want_j && !J[i]) || (o->want_k && !K[i]))
            return fail(JK_EINVAL, "jk_build_batch: NULL matrix pointer for molecule %d", i);
    if (!hs[0]) return fail(JK_EINVAL, "jk_build_batch: handle 0 is NULL");
    DeviceGuard dg;
    if ((rc = dg.ok(hs[0]->device))) return rc;
    BatchSetup b;
    if ((rc = batch_setup(nmol, hs, nd, o, b))) return rc;
    hipStream_t s = static_cast<hipStream_t>(o->stream);
    char* ws = static_cast<char*>(o->workspace);
    bool own = false;
    if (ws) {
        if (o->workspace_bytes < b.total)
            return fail(JK_EINVAL, "jk_build_batch: workspace of %zu bytes is below the %zu required",
                        o->workspace_bytes, b.total);
    } else {
        hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&ws), b.total, s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(JK_ENOMEM, "jk_build_batch: cannot allocate %zu bytes of workspace (%s)", b.total,
                        hipGetErrorString(e));
        }
        own = true;
    }
    std::vector<MolDesc> mds(nmol);
    hipError_t e = hipSuccess;
    for (int i = 0; i < nmol && e == hipSuccess; ++i)
        e = mol_pre(hs[i], nd[i], D[i], o, ws + b.mol_off[i], b.ms[i], mds[i], s);
    // work items and molecule table, staged through host memory the stream frees
    EriItem* d_eri = reinterpret_cast<EriItem*>(ws + b.off_items);
    DigItem* const d_dig[2] = {reinterpret_cast<DigItem*>(ws + b.off_items + b.eri_bytes),
                               reinterpret_cast<DigItem*>(ws + b.off_items + b.eri_bytes + b.dig_bytes[0])};
    const size_t mol_at = b.eri_bytes + b.dig_bytes[0] + b.dig_bytes[1];
    MolDesc* d_mols = reinterpret_cast<MolDesc*>(ws + b.off_items + mol_at);
    const size_t host_bytes = mol_at + b.mol_bytes;
    char* stage = static_cast<char*>(std::malloc(host_bytes));
    if (!stage) e = hipErrorOutOfMemory;
    if (e == hipSuccess) {
        std::memcpy(stage, b.wp.eri.data(), b.wp.eri.size() * sizeof(EriItem));
        std::memcpy(stage + b.eri_bytes, b.wp.dig[0].data(), b.wp.dig[0].size() * sizeof(DigItem));
        std::memcpy(stage + b.eri_bytes + b.dig_bytes[0], b.wp.dig[1].data(), b.wp.dig[1].size() * sizeof(DigItem));
        std::memcpy(stage + mol_at, mds.data(), nmol * sizeof(MolDesc));
        e = hipMemcpyAsync(ws + b.off_items, stage, host_bytes, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipLaunchHostFunc(s, free_host_cb, stage);
        else std::free(stage);
    }
    if (e == hipSuccess)
        e = run_plan(b.wp, d_eri, d_dig, mds[0], d_mols, ws + b.off_tiles, b.tb, o, hs[0]->d_boys,
                     hs[0]->d_boys32, s, hs[0]->aux, nullptr);
    for (int i = 0; i < nmol && e == hipSuccess; ++i)
        e = mol_post(hs[i], nd[i], mds[i], o->want_j ? J[i] : nullptr, o->want_k ? K[i] : nullptr, b.wp.skip_t, s);
    if (own) {
        hipError_t e2 = hipFreeAsync(ws, s);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return fail(JK_EDEVICE, "jk_build_batch: %s", hipGetErrorString(e));
    for (int i = 0; i < nmol; ++i) {
        std::lock_guard<std::mutex> g(hs[i]->mu);
        hs[i]->stats[0] = -1;   // per-molecule statistics are not kept for batches
    }
    return JK_OK;
}

int jk_tune_set(int32_t cls, const jk_tune_t* t) {
    if (cls < 0 || cls >= kNumClass || !t || t->seg_max < 4 || t->seg_max > (1 << 20) ||
        !(t->g_max == 1 || t->g_max == 2 || t->g_max == 4 || t->g_max == 8 || t->g_max == 16) ||
        !(t->dig_kernel >= 1 && t->dig_kernel <= 3) ||
        !(t->eri_block == 64 || t->eri_block == 128 || t->eri_block == 256))
        return fail(JK_EINVAL, "jk_tune_set: bad arguments");
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[cls].seg_max = t->seg_max;
    g_tune[cls].g_max = t->g_max;
    g_tune[cls].dig_kernel = t->dig_kernel;
    g_tune[cls].eri_block = t->eri_block;
    ++g_tune_gen;
    return JK_OK;
}

int jk_tune_get(int32_t cls, jk_tune_t* t) {
    if (cls < 0 || cls >= kNumClass || !t) return fail(JK_EINVAL, "jk_tune_get: bad arguments");
    std::lock_guard<std::mutex> g(g_tune_mu);
    t->seg_max = g_tune[cls].seg_max;
    t->g_max = g_tune[cls].g_max;
    t->dig_kernel = g_tune[cls].dig_kernel;
    t->eri_block = g_tune[cls].eri_block;
    return JK_OK;
}

static const char* kArch = "gfx950";

int jk_tune_load(const char* path) {
    if (!path) return fail(JK_EINVAL, "jk_tune_load: NULL path");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(JK_EINVAL, "jk_tune_load: cannot open %s", path);
    std::string txt;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, n);
    std::fclose(f);
    if (txt.find(std::string("\"arch\": \"") + kArch + "\"") == std::string::npos)
        return fail(JK_EUNSUPPORTED, "jk_tune_load: %s holds no entries for %s", path, kArch);
    int applied = 0;
    size_t pos = 0;
    while ((pos = txt.find("\"class\":", pos)) != std::string::npos) {
        int cls = -1;
        const size_t end = txt.find('}', pos);
        const std::string ent = txt.substr(pos, end - pos);
        if (std::sscanf(ent.c_str(), "\"class\": %d", &cls) == 1) {
            // every field optional but the class; absent ones keep their defaults
            jk_tune_t t{128, 16, 1, 256};
            auto field = [&](const char* key, int32_t& v) {
                const size_t q = ent.find(key);
                int x;
                if (q != std::string::npos && std::sscanf(ent.c_str() + q + std::strlen(key), " %d", &x) == 1) v = x;
            };
            field("\"seg_max\":", t.seg_max);
            field("\"g_max\":", t.g_max);
            field("\"dig_kernel\":", t.dig_kernel);
            field("\"eri_block\":", t.eri_block);
            if (cls >= 0 && cls < kNumClass && jk_tune_set(cls, &t) == JK_OK) ++applied;
        }
        pos = end == std::string::npos ? txt.size() : end;
    }
    return applied > 0 ? JK_OK : fail(JK_EINVAL, "jk_tune_load: no valid entries in %s", path);
}

int jk_autotune(jk_basis_t h, int32_t nd, const double* D, double* J, double* K, const jk_build_opts* o,
                const char* cache_path) {
    if (!h || !o || nd < 1 || !D || !J || !K) return fail(JK_EINVAL, "jk_autotune: bad arguments");
    jk_build_opts oo = *o;
    hipStream_t s = static_cast<hipStream_t>(o->stream);
    jk_tune_t best[kNumClass];
    double best_ms[kNumClass];
    for (int c = 0; c < kNumClass; ++c) {
        int rc = jk_tune_get(c, &best[c]);
        if (rc) return rc;
        best_ms[c] = 1e300;
    }
    // times one candidate per class (every class set at once: the classes'
    // launches are separate, so each class's time is its own); keeps the best
    auto trial = [&](auto&& make) -> int {
        jk_tune_t cand[kNumClass];
        for (int c = 0; c < kNumClass; ++c) {
            cand[c] = best[c];
            make(c, cand[c]);
            int rc = jk_tune_set(c, &cand[c]);
            if (rc) return rc;
        }
        int rc = jk_build(h, nd, D, J, K, &oo);   // warm-up: lists, plans
        if (rc) return rc;
        if (hipStreamSynchronize(s) != hipSuccess) return fail(JK_EDEVICE, "jk_autotune: sync failed");
        if ((rc = jk_profile_enable(h, 1))) return rc;
        for (int r = 0; r < 2 && !rc; ++r) rc = jk_build(h, nd, D, J, K, &oo);
        jk_profile_enable(h, 0);
        if (rc) return rc;
        for (int c = 0; c < kNumClass; ++c) {
            double tot = 0, v[5];
            for (int kind = 0; kind < 6; ++kind) {
                if ((rc = jk_profile_read(h, kind, c, v))) return rc;
                tot += v[0];
            }
            if (tot > 0 && tot < best_ms[c]) {
                best_ms[c] = tot;
                best[c] = cand[c];
            }
        }
        return JK_OK;
    };
    // coordinate search: digestion kernel x density group, then piece
    // length, then integral workgroup size, each around the best so far
    int rc;
    for (int k : {1, 2, 3})
        for (int g : {16, 8})
            if ((rc = trial([&](int, jk_tune_t& t) { t.dig_kernel = k; t.g_max = g; }))) return rc;
    for (int seg : {32, 64, 128, 256})
        if ((rc = trial([&](int, jk_tune_t& t) { t.seg_max = seg; }))) return rc;
    for (int blk : {64, 128, 256})
        if ((rc = trial([&](int, jk_tune_t& t) { t.eri_block = blk; }))) return rc;
    for (int c = 0; c < kNumClass; ++c)
        if ((rc = jk_tune_set(c, &best[c]))) return rc;
    if (cache_path) {
        FILE* f = std::fopen(cache_path, "w");
        if (!f) return fail(JK_EINVAL, "jk_autotune: cannot write %s", cache_path);
        std::fprintf(f, "{\"arch\": \"%s\", \"nd\": %d, \"nbf\": %d, \"entries\": [\n", kArch, nd, h->nf);
        for (int c = 0; c < kNumClass; ++c)
            std::fprintf(f,
                         "  {\"class\": %d, \"seg_max\": %d, \"g_max\": %d, \"dig_kernel\": %d, \"eri_block\": %d, "
                         "\"ms_per_build\": %.5f}%s\n",
                         c, best[c].seg_max, best[c].g_max, best[c].dig_kernel, best[c].eri_block,
                         best_ms[c] < 1e299 ? best_ms[c] / 2 : -1.0, c + 1 < kNumClass ? "," : "");
        std::fprintf(f, "]}\n");
        std::fclose(f);
    }
    return JK_OK;
}

struct jk_graph_s {
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

int jk_graph_create(jk_basis_t h, int32_t nd, const double* D, double* J, double* K, const jk_build_opts* o,
                    jk_graph_t* out) {
    if (!out) return fail(JK_EINVAL, "jk_graph_create: out is NULL");
    *out = nullptr;
    if (!h || !o) return fail(JK_EINVAL, "jk_graph_create: NULL handle or options");
    if (!o->workspace) return fail(JK_EINVAL, "jk_graph_create: a workspace is required");
    if (h->profiling) return fail(JK_EINVAL, "jk_graph_create: profiling must be off");
    DeviceGuard dg;
    int rc = dg.ok(h->device);
    if (rc) return rc;
    // plan and kernel attributes outside the capture
    if (jk_workspace_bytes(h, nd, o) == 0) return fail(JK_EINVAL, "jk_graph_create: invalid build arguments");
    {
        CachedPlan* cp = nullptr;
        if ((rc = get_plan(h, nd, o, &cp))) return rc;
    }
    hipStream_t cs = nullptr;
    HIPC(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    jk_build_opts oc = *o;
    oc.stream = cs;
    std::unique_ptr<jk_graph_s> g(new jk_graph_s());
    g->device = h->device;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = jk_build(h, nd, D, J, K, &oc);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &graph);
        g->graph = graph;
        if (rc == JK_OK && e2 != hipSuccess) rc = fail(JK_EDEVICE, "jk_graph_create: capture failed (%s)", hipGetErrorString(e2));
        if (rc == JK_OK) {
            e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) rc = fail(JK_EDEVICE, "jk_graph_create: instantiate failed (%s)", hipGetErrorString(e));
        }
    } else {
        rc = fail(JK_EDEVICE, "jk_graph_create: begin capture failed (%s)", hipGetErrorString(e));
    }
    (void)hipStreamDestroy(cs);
    if (rc != JK_OK) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        return rc;
    }
    *out = g.release();
    return JK_OK;
}

int jk_graph_launch(jk_graph_t g, void* stream) {
    if (!g) return fail(JK_EINVAL, "jk_graph_launch: NULL graph");
    DeviceGuard dg;
    int rc = dg.ok(g->device);
    if (rc) return rc;
    HIPC(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
    return JK_OK;
}

void jk_graph_destroy(jk_graph_t g) {
    if (!g) return;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
}

int jk_profile_enable(jk_basis_t h, int32_t on) {
    if (!h || (on != 0 && on != 1)) return fail(JK_EINVAL, "jk_profile_enable: bad arguments");
    DeviceGuard dg;
    int rc = dg.ok(h->device);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(h->mu);
    if (on && !h->d_kept) {
        HIPC(hipMalloc(&h->d_kept, 2 * kNumClass * sizeof(unsigned long long)));
        HIPC(hipMemset(h->d_kept, 0, 2 * kNumClass * sizeof(unsigned long long)));
    }
    h->profiling = on != 0;
    return JK_OK;
}

int jk_profile_read(jk_basis_t h, int32_t kind, int32_t cls, double out[5]) {
    if (!h || !out || kind < 0 || kind > 5 || cls < 0 || cls >= kNumClass)
        return fail(JK_EINVAL, "jk_profile_read: bad arguments");
    std::lock_guard<std::mutex> g(h->mu);
    // fold every pending record into the accumulators; the start event of a
    // digestion record is the end event of its integral record, so events
    // are destroyed only once both uses are folded
    std::vector<hipEvent_t> dead;
    for (auto& r : h->prof) HIPC(hipEventSynchronize(r.e1));
    // the kept counters cover exactly the pending records: scale their
    // quartet and flop counts (list quartets) to the quartets the whole
    // screen kept, per tier and class
    double ratio[2][kNumClass];
    for (auto& v : ratio)
        for (double& x : v) x = 1.0;
    if (h->d_kept && !h->prof.empty()) {
        DeviceGuard dg;
        int rc = dg.ok(h->device);
        if (rc) return rc;
        unsigned long long kept[2 * kNumClass];
        HIPC(hipMemcpy(kept, h->d_kept, sizeof(kept), hipMemcpyDeviceToHost));
        HIPC(hipMemset(h->d_kept, 0, sizeof(kept)));
        double listed[2][kNumClass] = {};
        for (auto& r : h->prof)
            if (r.kind == 0 || r.kind == 2) listed[r.kind / 2][r.cls] += r.quartets;
        for (int t = 0; t < 2; ++t)
            for (int c = 0; c < kNumClass; ++c)
                if (listed[t][c] > 0) ratio[t][c] = static_cast<double>(kept[t * kNumClass + c]) / listed[t][c];
    }
    for (auto& r : h->prof) {
        float ms = 0.0f;
        HIPC(hipEventElapsedTime(&ms, r.e0, r.e1));
        const int tier = (r.kind == 2 || r.kind == 3 || r.kind == 5) ? 1 : 0;
        const double f = ratio[tier][r.cls];
        double* a = h->prof_acc[r.kind][r.cls];
        a[0] += ms;
        a[1] += 1;
        a[2] += r.flops * f;
        a[3] += r.quartets * f;
        a[4] += r.bytes;
        dead.push_back(r.e0);
        dead.push_back(r.e1);
    }
    h->prof.clear();
    std::sort(dead.begin(), dead.end());
    dead.erase(std::unique(dead.begin(), dead.end()), dead.end());
    for (auto ev : dead) (void)hipEventDestroy(ev);
    for (int i = 0; i < 5; ++i) {
        out[i] = h->prof_acc[kind][cls][i];
        h->prof_acc[kind][cls][i] = 0.0;
    }
    return JK_OK;
}

int jk_eri_tiles(jk_basis_t h, int32_t nq, const int32_t* shells, double* out) {
    if (!h || nq < 0 || (nq > 0 && (!shells || !out))) return fail(JK_EINVAL, "jk_eri_tiles: bad arguments");
    const int ns = h->ns;
    struct Req {
        int cls;
        int2 pq;
        int map[4];     // requested position -> canonical position
        int nreq[4];    // Cartesian sizes in requested order
        size_t off;
    };
    std::vector<Req> reqs(nq);
    size_t off = 0;
    for (int r = 0; r < nq; ++r) {
        int s[4];
        for (int k = 0; k < 4; ++k) {
            const int u = shells[4 * r + k];
            if (u < 0 || u >= ns) return fail(JK_EINVAL, "jk_eri_tiles: shell index %d out of range", u);
            s[k] = h->int_of_user[u];
        }
        // canonical orientation: a >= b, c >= d (internal), bra class >= ket class
        int pos[4] = {0, 1, 2, 3};   // canonical slot -> requested position
        if (s[pos[0]] < s[pos[1]]) std::swap(pos[0], pos[1]);
        if (s[pos[2]] < s[pos[3]]) std::swap(pos[2], pos[3]);
        const int X = pair_class(h->l_int[s[pos[0]]], h->l_int[s[pos[1]]]);
        const int Y = pair_class(h->l_int[s[pos[2]]], h->l_int[s[pos[3]]]);
        if (X < Y) {
            std::swap(pos[0], pos[2]);
            std::swap(pos[1], pos[3]);
        }
        Req& q = reqs[r];
        q.cls = quartet_class(std::max(X, Y), std::min(X, Y));
        const int bra = h->pair_id[static_cast<size_t>(s[pos[0]]) * ns + s[pos[1]]];
        const int ket = h->pair_id[static_cast<size_t>(s[pos[2]]) * ns + s[pos[3]]];
        q.pq = make_int2(bra, ket);
        for (int k = 0; k < 4; ++k) q.map[pos[k]] = k;
        size_t sz = 1;
        for (int k = 0; k < 4; ++k) {
            q.nreq[k] = h->ncart_int[s[k]];
            sz *= q.nreq[k];
        }
        q.off = off;
        off += sz;
    }
    for (int c = 0; c < kNumClass; ++c) {
        std::vector<int2> qs;
        std::vector<int> who;
        for (int r = 0; r < nq; ++r)
            if (reqs[r].cls == c) {
                qs.push_back(reqs[r].pq);
                who.push_back(r);
            }
        if (qs.empty()) continue;
        std::vector<double> tiles;
        int rc = eval_tiles(h, c, qs, tiles);
        if (rc) return rc;
        const int NF = class_nf(c);
        for (size_t t = 0; t < who.size(); ++t) {
            const Req& q = reqs[who[t]];
            int ncan[4];
            for (int k = 0; k < 4; ++k) ncan[q.map[k]] = q.nreq[k];
            int idx[4];
            for (idx[0] = 0; idx[0] < q.nreq[0]; ++idx[0])
                for (idx[1] = 0; idx[1] < q.nreq[1]; ++idx[1])
                    for (idx[2] = 0; idx[2] < q.nreq[2]; ++idx[2])
                        for (idx[3] = 0; idx[3] < q.nreq[3]; ++idx[3]) {
                            int ci[4];
                            for (int k = 0; k < 4; ++k) ci[q.map[k]] = idx[k];
                            const int f = ((ci[0] * ncan[1] + ci[1]) * ncan[2] + ci[2]) * ncan[3] + ci[3];
                            const size_t o = q.off + ((static_cast<size_t>(idx[0]) * q.nreq[1] + idx[1]) * q.nreq[2] + idx[2]) * q.nreq[3] + idx[3];
                            out[o] = tiles[t * NF + f];
                        }
        }
    }
    return JK_OK;
}

}  // extern "C"
