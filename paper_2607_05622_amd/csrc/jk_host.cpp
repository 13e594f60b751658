// Host side of the J/K C-ABI: basis ingest, resident shell-pair data, Schwarz
// factors, screened quartet lists, workspace and the launch sequence of one
// build.  See include/jk.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "jk.h"
#include "jk_internal.h"
#include "jk_launch.h"

namespace jk {
#include "eri_cost.inc"   // kClassCost[21]: generated flop counts per class
}

using namespace jk;

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
constexpr long long kTileCapElems = 32ll << 20;   // 256 MB FP64 work buffer cap

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

// Runs of quartets sharing a bra pair, capped in length: the unit of work of
// the digestion kernel.
constexpr int kSegMax = 1024;

struct Chunk {
    int s0, s1;          // segments [s0, s1)
    long long q0, q1;    // quartets [q0, q1) of the class list
};

struct ClassList {
    long long count = 0;
    double prim_quartets = 0;   // sum of nprim_bra * nprim_ket
    int2* dev = nullptr;
    std::vector<int2> segs;     // (first quartet, count)
    int2* dev_segs = nullptr;
};

// pair class X -> (la, lb)
const int kPairL[6][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}};

}  // namespace

struct jk_basis_s {
    int device = 0;
    int natoms = 0, ns = 0, nf = 0, nc = 0, spherical = 1;
    // internal shells are the user shells sorted by l (stable)
    std::vector<int> user_of_int, int_of_user, l_int, f0_int, ncart_int, nprim_int;
    std::vector<int> user_f0;   // user function offset per user shell
    std::vector<double> centre_int;   // [ns][3]
    std::vector<std::vector<double>> exps_int, w_int;   // normalized contraction weights
    std::vector<PairInfo> pairs;
    std::vector<PrimPair> prims;
    std::vector<int> pair_id;   // [ns][ns] -> pair index for a >= b, else -1
    std::vector<int> pairs_of_class[kNumPairClass];
    // device
    PairInfo* d_pairs = nullptr;
    PrimPair* d_prims = nullptr;
    double* d_boys = nullptr;
    CartMap* d_cmap = nullptr;
    UserMap* d_umap = nullptr;
    int* d_shell_f0 = nullptr;
    int* d_shell_nf = nullptr;
    // quartet lists for the current tolerance (older lists are retired, not
    // freed, because builds on other streams may still read them)
    std::mutex mu;
    double list_tol = -1.0;
    ClassList lists[kNumClass];
    std::vector<int2*> retired;
    int lds_cap = 65536;               // dynamic LDS bytes per workgroup
    int lw_off[kMaxL + 1] = {}, lw_len[kMaxL + 1] = {};   // Cartesian function window per l
    size_t prepared[kNumClass] = {};   // LDS attribute already granted per class
    double stats[6] = {0, 0, 0, 0, 0, 0};
    // measurement: event pairs around integral / digestion launches
    struct ProfRec {
        int kind, cls;
        hipEvent_t e0, e1;
        double flops, quartets, bytes;
    };
    bool profiling = false;
    std::vector<ProfRec> prof;
    double prof_acc[2][kNumClass][5] = {};

    ~jk_basis_s() {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(device);
        (void)hipFree(d_pairs);
        (void)hipFree(d_prims);
        (void)hipFree(d_boys);
        (void)hipFree(d_cmap);
        (void)hipFree(d_umap);
        (void)hipFree(d_shell_f0);
        (void)hipFree(d_shell_nf);
        for (auto& l : lists) {
            (void)hipFree(l.dev);
            (void)hipFree(l.dev_segs);
        }
        for (auto* p : retired) (void)hipFree(p);
        for (auto& r : prof) {
            (void)hipEventDestroy(r.e0);
            (void)hipEventDestroy(r.e1);
        }
        (void)hipSetDevice(cur);
    }
};

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
    HIPC(hipMalloc(&dq, nq * sizeof(int2)));
    HIPC(hipMalloc(&dout, nq * NF * sizeof(double)));
    HIPC(hipMalloc(&dscr, nq * NF * sizeof(double)));
    int rc = JK_OK;
    do {
        if (hipMemcpy(dq, quartets.data(), nq * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess) {
            rc = fail(JK_EDEVICE, "eval_tiles: copy in failed");
            break;
        }
        EriTileArgs a{};
        a.quartets = dq;
        a.nq = nq;
        a.pairs = h->d_pairs;
        a.prims = h->d_prims;
        a.boys = h->d_boys;
        a.dmax = nullptr;
        a.ns = h->ns;
        a.tol = 0.0;
        a.out = dout;
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

// Build the class-bucketed quartet lists kept by Q_ab Q_cd >= tol.  Within a
// class: bra pair outer, ket pairs in index order.
int build_lists(jk_basis_s* h, double tol) {
    ClassList fresh[kNumClass];
    for (int X = 0; X < kNumPairClass; ++X) {
        for (int Y = 0; Y <= X; ++Y) {
            const int cls = quartet_class(X, Y);
            const auto& bra = h->pairs_of_class[X];
            const auto& ket = h->pairs_of_class[Y];
            // ket pairs sorted by Q, descending, to stop early
            std::vector<int> ks(ket);
            std::sort(ks.begin(), ks.end(), [&](int u, int v) { return h->pairs[u].q > h->pairs[v].q; });
            std::vector<int2> out;
            std::vector<int> keep;
            double primq = 0;
            for (int b : bra) {
                const double qb = h->pairs[b].q;
                keep.clear();
                for (int k : ks) {
                    if (qb * h->pairs[k].q < tol) break;
                    if (X == Y && k > b) continue;
                    keep.push_back(k);
                }
                std::sort(keep.begin(), keep.end());
                for (int k : keep) {
                    out.push_back(make_int2(b, k));
                    primq += static_cast<double>(h->pairs[b].nprim) * h->pairs[k].nprim;
                }
            }
            fresh[cls].count = static_cast<long long>(out.size());
            fresh[cls].prim_quartets = primq;
            // segments: bra-pair runs of at most kSegMax quartets
            auto& segs = fresh[cls].segs;
            for (size_t q = 0; q < out.size();) {
                size_t e = q + 1;
                while (e < out.size() && out[e].x == out[q].x && static_cast<int>(e - q) < kSegMax) ++e;
                segs.push_back(make_int2(static_cast<int>(q), static_cast<int>(e - q)));
                q = e;
            }
            if (!out.empty()) {
                int rc = upload(&fresh[cls].dev, out);
                if (!rc) rc = upload(&fresh[cls].dev_segs, segs);
                if (rc) {
                    for (auto& f : fresh) {
                        (void)hipFree(f.dev);
                        (void)hipFree(f.dev_segs);
                    }
                    return rc;
                }
            }
        }
    }
    for (int c = 0; c < kNumClass; ++c) {
        if (h->lists[c].dev) h->retired.push_back(h->lists[c].dev);
        if (h->lists[c].dev_segs) h->retired.push_back(h->lists[c].dev_segs);
        h->lists[c] = fresh[c];
    }
    h->list_tol = tol;
    return JK_OK;
}

int ensure_lists(jk_basis_s* h, double tol) {
    std::lock_guard<std::mutex> g(h->mu);
    if (h->list_tol >= 0 && h->list_tol <= tol) return JK_OK;
    return build_lists(h, tol);
}

struct Plan {
    int ndp, dg;
    size_t off_D, off_J, off_K, off_KT, off_dmax, off_tile, off_scr, total;
    long long tile_elems;
};

Plan make_plan(const jk_basis_s* h, int nd, const jk_build_opts* o) {
    Plan p{};
    p.dg = 1;
    p.ndp = nd;
    const size_t mat = static_cast<size_t>(h->nc) * h->nc * p.ndp * sizeof(double);
    auto al = [](size_t v) { return (v + 255) & ~static_cast<size_t>(255); };
    size_t off = 0;
    p.off_D = off;
    off += al(mat);
    p.off_J = off;
    if (o->want_j) off += al(mat);
    const size_t kmat = static_cast<size_t>(h->nc) * h->nc * nd * sizeof(double);
    p.off_K = off;
    if (o->want_k) off += al(kmat);
    p.off_KT = off;
    if (o->want_k) off += al(kmat);
    p.off_dmax = off;
    off += al(static_cast<size_t>(h->ns) * h->ns * sizeof(double));
    // tile buffer: the largest class volume, capped
    long long need = 1296;
    for (int c = 0; c < kNumClass; ++c) {
        const long long v = h->lists[c].count * class_nf(c);
        need = std::max(need, std::min(v, kTileCapElems));
    }
    if (h->list_tol < 0) need = kTileCapElems;
    p.tile_elems = need;
    p.off_tile = off;
    off += al(static_cast<size_t>(need) * sizeof(double));
    p.off_scr = off;   // (e0|cd) of pass-evaluated classes: never larger than the tile
    off += al(static_cast<size_t>(need) * sizeof(double));
    p.total = off;
    return p;
}

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
    for (int l = kMaxL; l >= 0; --l) {
        h->lw_off[l] = fc;
        h->lw_len[l] = 0;
    }
    for (int si = ns - 1; si >= 0; --si) {
        const int l = h->l_int[si];
        h->lw_off[l] = h->f0_int[si];
        h->lw_len[l] += ncart(l);
    }
    {
        int cap = 0;
        HIPC(hipDeviceGetAttribute(&cap, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
        h->lds_cap = cap > 0 ? cap : 65536;
    }

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
            for (int i = 0; i < h->nprim_int[a]; ++i)
                for (int j = 0; j < h->nprim_int[b]; ++j) {
                    const double al = h->exps_int[a][i], be = h->exps_int[b][j];
                    const double p = al + be;
                    PrimPair pp{};
                    pp.p = p;
                    for (int k = 0; k < 3; ++k) pp.P[k] = (al * A[k] + be * B[k]) / p;
                    pp.E = E0 * h->w_int[a][i] * h->w_int[b][j] * std::exp(-al * be / p * ab2) / p;
                    pp.o2p = 0.5 / p;
                    h->prims.push_back(pp);
                }
            P.nprim = h->nprim_int[a] * h->nprim_int[b];
            const int id = static_cast<int>(h->pairs.size());
            h->pair_id[static_cast<size_t>(a) * ns + b] = id;
            h->pairs.push_back(P);
            h->pairs_of_class[pair_class(h->l_int[a], h->l_int[b])].push_back(id);
        }
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
    if ((rc = upload(&h->d_prims, h->prims))) return rc;
    if ((rc = upload(&h->d_boys, boys_table()))) return rc;
    if ((rc = upload(&h->d_cmap, cmap))) return rc;
    if ((rc = upload(&h->d_umap, umap))) return rc;
    if ((rc = upload(&h->d_shell_f0, sf0))) return rc;
    if ((rc = upload(&h->d_shell_nf, h->ncart_int))) return rc;
    if ((rc = compute_schwarz(h.get()))) return rc;
    HIPC(hipMemcpy(h->d_pairs, h->pairs.data(), h->pairs.size() * sizeof(PairInfo), hipMemcpyHostToDevice));
    if ((rc = ensure_lists(h.get(), 1e-12))) return rc;
    *out = h.release();
    return JK_OK;
}

int jk_nbf(jk_basis_t h) { return h ? h->nf : fail(JK_EINVAL, "jk_nbf: NULL handle"); }

void jk_destroy(jk_basis_t h) { delete h; }

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

size_t jk_workspace_bytes(jk_basis_t h, int32_t nd, const jk_build_opts* o) {
    jk_build_opts def;
    if (!o) {
        jk_default_opts(&def);
        o = &def;
    }
    if (!h || nd < 1 || !valid_opts(o)) return 0;
    if (ensure_lists(h, o->schwarz_tol)) return 0;
    return make_plan(h, nd, o).total;
}

int jk_last_stats(jk_basis_t h, double out[6]) {
    if (!h || !out) return fail(JK_EINVAL, "jk_last_stats: bad arguments");
    std::lock_guard<std::mutex> g(h->mu);
    for (int i = 0; i < 6; ++i) out[i] = h->stats[i];
    return JK_OK;
}

int jk_build(jk_basis_t h, int32_t nd, const double* D, double* J, double* K, const jk_build_opts* o) {
    jk_build_opts def;
    if (!o) {
        jk_default_opts(&def);
        o = &def;
    }
    if (!h) return fail(JK_EINVAL, "jk_build: NULL handle");
    if (nd < 1) return fail(JK_EINVAL, "jk_build: nd=%d must be >= 1", nd);
    if (!valid_opts(o)) return fail(JK_EINVAL, "jk_build: invalid options");
    if (!D) return fail(JK_EINVAL, "jk_build: D is NULL");
    if (o->want_j && !J) return fail(JK_EINVAL, "jk_build: J is NULL but want_j is set");
    if (o->want_k && !K) return fail(JK_EINVAL, "jk_build: K is NULL but want_k is set");
    if (o->precision != JK_FP64) return fail(JK_EUNSUPPORTED, "jk_build: only JK_FP64 is available in this build");
    int cur = 0;
    HIPC(hipGetDevice(&cur));
    if (cur != h->device) HIPC(hipSetDevice(h->device));
    int rc = ensure_lists(h, o->schwarz_tol);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(o->stream);
    const Plan p = make_plan(h, nd, o);
    char* ws = static_cast<char*>(o->workspace);
    bool own = false;
    if (ws) {
        if (o->workspace_bytes < p.total)
            return fail(JK_EINVAL, "jk_build: workspace of %zu bytes is below the %zu required", o->workspace_bytes,
                        p.total);
    } else {
        hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&ws), p.total, s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(JK_ENOMEM, "jk_build: cannot allocate %zu bytes of workspace (%s)", p.total,
                        hipGetErrorString(e));
        }
        own = true;
    }
    double* Dc = reinterpret_cast<double*>(ws + p.off_D);
    double* Jc = o->want_j ? reinterpret_cast<double*>(ws + p.off_J) : nullptr;
    double* Kc = o->want_k ? reinterpret_cast<double*>(ws + p.off_K) : nullptr;
    double* KTc = o->want_k ? reinterpret_cast<double*>(ws + p.off_KT) : nullptr;
    double* dmax = reinterpret_cast<double*>(ws + p.off_dmax);
    double* tiles = reinterpret_cast<double*>(ws + p.off_tile);
    double* scratch = reinterpret_cast<double*>(ws + p.off_scr);
    const long long mat = static_cast<long long>(h->nc) * h->nc * p.ndp;
    const long long kmat = static_cast<long long>(h->nc) * h->nc * nd;
    hipError_t e = launch_sph2cart(D, nd, h->nf, h->d_cmap, h->nc, p.ndp, Dc, s);
    if (e == hipSuccess) e = launch_pair_dmax(Dc, h->nc, p.ndp, nd, h->d_shell_f0, h->d_shell_nf, h->ns, dmax, s);
    if (e == hipSuccess && Jc) e = launch_zero(Jc, mat, s);
    if (e == hipSuccess && Kc) e = launch_zero(Kc, kmat, s);
    if (e == hipSuccess && KTc) e = launch_zero(KTc, kmat, s);
    double nq_tot = 0, nfq = 0, npq = 0, eri_flops = 0, dig_flops = 0;
    for (int c = 0; c < kNumClass && e == hipSuccess; ++c) {
        const ClassList& L = h->lists[c];
        if (L.count == 0) continue;
        const int NF = class_nf(c);
        int X = 0;
        while (quartet_class(X + 1, 0) <= c && X + 1 < kNumPairClass) ++X;
        const int Y = c - quartet_class(X, 0);
        const int la = kPairL[X][0], lb = kPairL[X][1], lc = kPairL[Y][0], ld = kPairL[Y][1];
        const int NA = ncart(la), NB = ncart(lb);
        // LDS windows: Cartesian functions of the ket shells' angular momenta
        const int colA0 = h->lw_off[lc], colAw = h->lw_len[lc];
        const int colB0 = ld != lc ? h->lw_off[ld] : 0, colBw = ld != lc ? h->lw_len[ld] : 0;
        const size_t per_density = sizeof(double) * ((o->want_k ? 2 * (NA + NB) * (colAw + colBw) : 0) +
                                                     (o->want_j ? NA * NB : 0));
        int G = 16;
        while (G > 1 && (G / 2 >= nd || G * per_density > static_cast<size_t>(h->lds_cap))) G /= 2;
        if (per_density > static_cast<size_t>(h->lds_cap)) {
            if (own) (void)hipFreeAsync(ws, s);
            return fail(JK_EUNSUPPORTED, "jk_build: class %d needs %zu bytes of LDS per density (limit %d)", c,
                        per_density, h->lds_cap);
        }
        const size_t lds_bytes = G * per_density;
        {
            std::lock_guard<std::mutex> g(h->mu);
            if (h->prepared[c] < lds_bytes) {
                e = digest_prepare(c, lds_bytes);
                if (e == hipSuccess) h->prepared[c] = lds_bytes;
            }
        }
        if (e != hipSuccess) break;
        const long long cap = p.tile_elems / NF;
        const int nseg = static_cast<int>(L.segs.size());
        for (int s0 = 0; s0 < nseg && e == hipSuccess;) {
            // chunk: whole segments whose quartets fit the tile buffer
            const long long q0 = L.segs[s0].x;
            int s1 = s0;
            while (s1 < nseg && L.segs[s1].x + L.segs[s1].y - q0 <= cap) ++s1;
            if (s1 == s0) {
                e = hipErrorInvalidValue;   // a segment larger than the work buffer: never by construction
                break;
            }
            const long long q1 = L.segs[s1 - 1].x + L.segs[s1 - 1].y;
            const long long n = q1 - q0;
            EriTileArgs ea{};
            ea.quartets = L.dev + q0;
            ea.nq = n;
            ea.pairs = h->d_pairs;
            ea.prims = h->d_prims;
            ea.boys = h->d_boys;
            ea.dmax = dmax;
            ea.ns = h->ns;
            ea.tol = o->schwarz_tol;
            ea.out = tiles;
            ea.scratch = scratch;
            const double cost_q = L.prim_quartets / static_cast<double>(L.count);
            hipEvent_t ev[2] = {nullptr, nullptr};
            if (h->profiling) {
                for (auto& x : ev)
                    if (e == hipSuccess) e = hipEventCreate(&x);
                if (e == hipSuccess) e = hipEventRecord(ev[0], s);
                if (e != hipSuccess) break;
            }
            e = launch_eri_tile(c, ea, s);
            if (e != hipSuccess) break;
            if (h->profiling) {
                e = hipEventRecord(ev[1], s);
                if (e != hipSuccess) break;
                std::lock_guard<std::mutex> g(h->mu);
                h->prof.push_back({0, c, ev[0], ev[1],
                                   n * (cost_q * (kClassCost[c].prim_flops + kClassCost[c].vrr_flops) +
                                        kClassCost[c].hrr_flops),
                                   static_cast<double>(n), static_cast<double>(n) * NF * sizeof(double)});
            }
            DigestArgs da{};
            da.quartets = L.dev + q0;
            da.nq = n;
            da.segs = L.dev_segs + s0;
            da.qbase = q0;
            da.nseg = s1 - s0;
            da.G = G;
            da.ngroups = (nd + G - 1) / G;
            da.nd = nd;
            da.pairs = h->d_pairs;
            da.dmax = dmax;
            da.ns = h->ns;
            da.tol = o->schwarz_tol;
            da.tiles = tiles;
            da.D = Dc;
            da.J = Jc;
            da.K = Kc;
            da.KT = KTc;
            da.nc = h->nc;
            da.ndp = p.ndp;
            da.colA0 = colA0;
            da.colAw = colAw;
            da.colB0 = colB0;
            da.colBw = colBw;
            da.want_j = o->want_j;
            da.want_k = o->want_k;
            e = launch_digest(c, da, s);
            if (h->profiling && e == hipSuccess) {
                hipEvent_t e2 = nullptr;
                e = hipEventCreate(&e2);
                if (e == hipSuccess) e = hipEventRecord(e2, s);
                if (e == hipSuccess) {
                    std::lock_guard<std::mutex> g(h->mu);
                    h->prof.push_back({1, c, ev[1], e2,
                                       static_cast<double>(n) * NF * nd *
                                           (2.0 * (o->want_j ? 2 : 0) + 2.0 * (o->want_k ? 8 : 0)),
                                       static_cast<double>(n),
                                       static_cast<double>(n) * NF * sizeof(double) * da.ngroups});
                }
            }
            s0 = s1;
        }
        nq_tot += L.count;
        nfq += static_cast<double>(L.count) * NF;
        npq += L.prim_quartets;
        eri_flops += L.prim_quartets * (kClassCost[c].prim_flops + kClassCost[c].vrr_flops) +
                     static_cast<double>(L.count) * kClassCost[c].hrr_flops;
        dig_flops += static_cast<double>(L.count) * NF * nd * (2.0 * (o->want_j ? 2 : 0) + 2.0 * (o->want_k ? 8 : 0));
    }
    if (e == hipSuccess) e = launch_cart2sph(Jc, Kc, KTc, nd, h->nf, h->d_umap, h->nc, p.ndp, J, K, s);
    if (own) {
        hipError_t e2 = hipFreeAsync(ws, s);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return fail(JK_EDEVICE, "jk_build: %s", hipGetErrorString(e));
    {
        std::lock_guard<std::mutex> g(h->mu);
        h->stats[0] = nq_tot;
        h->stats[1] = 0;
        h->stats[2] = nfq;
        h->stats[3] = npq;
        h->stats[4] = eri_flops;
        h->stats[5] = dig_flops;
    }
    if (cur != h->device) (void)hipSetDevice(cur);
    return JK_OK;
}

int jk_profile_enable(jk_basis_t h, int32_t on) {
    if (!h || (on != 0 && on != 1)) return fail(JK_EINVAL, "jk_profile_enable: bad arguments");
    std::lock_guard<std::mutex> g(h->mu);
    h->profiling = on != 0;
    return JK_OK;
}

int jk_profile_read(jk_basis_t h, int32_t kind, int32_t cls, double out[5]) {
    if (!h || !out || kind < 0 || kind > 1 || cls < 0 || cls >= kNumClass)
        return fail(JK_EINVAL, "jk_profile_read: bad arguments");
    std::lock_guard<std::mutex> g(h->mu);
    // fold every pending record into the accumulators; the start event of a
    // digestion record is the end event of its integral record, so events
    // are destroyed only once both uses are folded
    std::vector<hipEvent_t> dead;
    for (auto& r : h->prof) {
        HIPC(hipEventSynchronize(r.e1));
        float ms = 0.0f;
        HIPC(hipEventElapsedTime(&ms, r.e0, r.e1));
        double* a = h->prof_acc[r.kind][r.cls];
        a[0] += ms;
        a[1] += 1;
        a[2] += r.flops;
        a[3] += r.quartets;
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
