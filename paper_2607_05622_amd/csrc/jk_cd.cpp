// Cholesky-factor (CD) J/K (Eqs. (cdfact)-(cdknonsym)): host entry points.
//
// jk_cd_factor  the factor B of Eq. (cdfact) by pivoted Cholesky over the
//               screened two-electron operator, built as a pool of integrals
//               over the significant function pairs that is released again
// jk_cd_jk      J of Eq. (cdj) and K of Eq. (cdknonsym) from B for densities
//               given as factors D = U V^T
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <thread>
#include <vector>

#include "jk.h"
#include "jk_cd.h"
#include "jk_gemm.h"
#include "jk_internal.h"
#include "jk_launch.h"

// records the thread's error message (jk_host.cpp)
int record_error(int code, const char* msg);

namespace {

using namespace jk;

int cfail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return record_error(code, buf);
}

int hip_fail(const char* who, hipError_t e) {
    (void)hipGetLastError();
    return cfail(JK_EDEVICE, "%s: %s", who, hipGetErrorString(e));
}

#define CDC(expr)                                                \
    do {                                                         \
        hipError_t e_ = (expr);                                  \
        if (e_ != hipSuccess) return hip_fail(#expr, e_);        \
    } while (0)

// Device buffers of one call, released at its end (after the stream has
// drained: the factorization synchronizes before it returns).
struct Buffers {
    std::vector<void*> ps;
    template <class T>
    hipError_t get(T** p, size_t count) {
        void* q = nullptr;
        const hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
        if (e == hipSuccess) ps.push_back(q);
        *p = static_cast<T*>(q);
        return e;
    }
    ~Buffers() {
        for (void* p : ps) (void)hipFree(p);
    }
};

// Async scratch of jk_cd_jk, released on the call's stream.
struct Scratch {
    hipStream_t s;
    void* p = nullptr;
    explicit Scratch(hipStream_t st) : s(st) {}
    hipError_t get(size_t bytes) { return hipMallocAsync(&p, bytes, s); }
    ~Scratch() {
        if (p) (void)hipFreeAsync(p, s);
    }
};

struct DevGuard {
    int prev = -1;
    hipError_t set(int dev) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess || cur == dev) return e;
        prev = cur;
        return hipSetDevice(dev);
    }
    ~DevGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

int ncart_of(int l) { return (l + 1) * (l + 2) / 2; }
const int kPairLs[kNumPairClass][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}};

// Tile elements per integral launch (256 MB of FP64 tiles).
constexpr long long kCdTileElems = 32ll << 20;
// Budget of one density group's half-transforms B U and B V in jk_cd_jk
// (elements: 16 GB).
constexpr long long kCdGroupElems = 2ll << 30;
// Steps between two reads of the loop state at the start (doubling up to 256).
constexpr int kCdPollFirst = 16, kCdPollMax = 256;

}  // namespace

extern "C" {

int jk_cd_factor(jk_basis_t h, double delta, double screen_tol, int32_t max_vectors, double* B, int32_t* pivots,
                 int32_t* nvec_out, void* stream) {
    if (!h || !nvec_out) return cfail(JK_EINVAL, "jk_cd_factor: NULL handle or nvec_out");
    *nvec_out = 0;
    if (!(delta > 0.0) || !std::isfinite(delta))
        return cfail(JK_EINVAL, "jk_cd_factor: delta must be finite and > 0 (got %g)", delta);
    if (!(screen_tol >= 0.0) || !std::isfinite(screen_tol))
        return cfail(JK_EINVAL, "jk_cd_factor: screen_tol must be finite and >= 0 (got %g)", screen_tol);
    if (max_vectors < 0 || max_vectors > JK_CD_MAX_VECTORS)
        return cfail(JK_EINVAL, "jk_cd_factor: max_vectors=%d outside 0..%d", max_vectors, JK_CD_MAX_VECTORS);
    if (max_vectors > 0 && !B) return cfail(JK_EINVAL, "jk_cd_factor: NULL B");
    BasisView v;
    int rc = basis_view(h, &v);
    if (rc) return rc;
    DevGuard dg;
    CDC(dg.set(v.device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nf = v.nf;
    const long long npair = static_cast<long long>(nf) * (nf + 1) / 2;

    // significant shell pairs: Q_ab max_cd Q_cd >= screen_tol (a pair below
    // it has no kept entry); their function pairs are the operator's rows,
    // in the order m (m + 1) / 2 + n
    double qmax = 0.0;
    for (const PairInfo& P : v.pairs) qmax = std::max(qmax, P.q);
    std::vector<int> cidx(static_cast<size_t>(npair), -1);
    for (const PairInfo& P : v.pairs) {
        if (!(P.q * qmax >= screen_tol)) continue;
        for (int i = 0; i < v.nuf[P.sa]; ++i)
            for (int j = 0; j < v.nuf[P.sb]; ++j) {
                const long long m = v.uf0[P.sa] + i, n = v.uf0[P.sb] + j;
                cidx[m >= n ? m * (m + 1) / 2 + n : n * (n + 1) / 2 + m] = 0;
            }
    }
    std::vector<long long> sig;
    std::vector<int> pm, pn;
    for (long long m = 0, t = 0; m < nf; ++m)
        for (long long n = 0; n <= m; ++n, ++t)
            if (cidx[t] == 0) {
                cidx[t] = static_cast<int>(sig.size());
                sig.push_back(t);
                pm.push_back(static_cast<int>(m));
                pn.push_back(static_cast<int>(n));
            }
    const long long nsig = static_cast<long long>(sig.size());
    if (nsig == 0) return JK_OK;   // nothing significant: the factor is empty

    // kept quartets per class (canonical: bra pair class >= ket pair class,
    // ket <= bra within one class), Q_ab Q_cd >= screen_tol: per bra pair
    // the kets in descending Q up to the first that fails, bra pairs spread
    // over host threads (the order of a class's quartets does not matter:
    // every operator entry has one writer)
    std::vector<int> ksorted[kNumPairClass];
    for (int Y = 0; Y < kNumPairClass; ++Y) {
        ksorted[Y] = v.pairs_of_class[Y];
        std::sort(ksorted[Y].begin(), ksorted[Y].end(),
                  [&](int a, int b) { return v.pairs[a].q > v.pairs[b].q; });
    }
    const int nthr = static_cast<int>(std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
    std::vector<int2> qs[kNumClass];
    long long maxq = 0;
    for (int X = 0; X < kNumPairClass; ++X)
        for (int Y = 0; Y <= X; ++Y) {
            const std::vector<int>& bra = v.pairs_of_class[X];
            const std::vector<int>& ket = ksorted[Y];
            std::vector<std::vector<int2>> part(nthr);
            std::vector<std::thread> pool;
            for (int t = 0; t < nthr; ++t)
                pool.emplace_back([&, t]() {
                    for (size_t i = t; i < bra.size(); i += nthr) {
                        const int b = bra[i];
                        const double qb = v.pairs[b].q;
                        for (int k : ket) {
                            if (qb * v.pairs[k].q < screen_tol) break;
                            if (X == Y && k > b) continue;
                            part[t].push_back(make_int2(b, k));
                        }
                    }
                });
            for (auto& th : pool) th.join();
            std::vector<int2>& out = qs[quartet_class(X, Y)];
            for (auto& pv : part) out.insert(out.end(), pv.begin(), pv.end());
            maxq = std::max<long long>(maxq, static_cast<long long>(out.size()));
        }

    size_t free_b = 0, total_b = 0;
    CDC(hipMemGetInfo(&free_b, &total_b));
    const double need = 8.0 * (static_cast<double>(nsig) * nsig + static_cast<double>(max_vectors + 1) * nsig) +
                        16.0 * kCdTileElems + 8.0 * maxq;
    if (need > 0.9 * static_cast<double>(free_b))
        return cfail(JK_ENOMEM, "jk_cd_factor: the operator over %lld function pairs and %d vectors need %.1f GB, %.1f GB free",
                     nsig, max_vectors, need / 1e9, free_b / 1e9);

    Buffers buf;
    double *V = nullptr, *Bc = nullptr, *d = nullptr, *bmax = nullptr, *tiles = nullptr, *scr = nullptr;
    int *dcidx = nullptr, *dpm = nullptr, *dpn = nullptr, *duf0 = nullptr, *piv = nullptr;
    long long* dsig = nullptr;
    int2* dq = nullptr;
    EriItem* ditem = nullptr;
    CdState* st = nullptr;
    CDC(buf.get(&V, static_cast<size_t>(nsig) * nsig));
    CDC(buf.get(&Bc, static_cast<size_t>(max_vectors) * nsig));
    CDC(buf.get(&d, nsig));
    CDC(buf.get(&bmax, (nsig + 255) / 256));
    CDC(buf.get(&tiles, kCdTileElems));
    CDC(buf.get(&scr, kCdTileElems));
    CDC(buf.get(&dcidx, cidx.size()));
    CDC(buf.get(&dpm, pm.size()));
    CDC(buf.get(&dpn, pn.size()));
    CDC(buf.get(&dsig, sig.size()));
    CDC(buf.get(&duf0, v.uf0.size()));
    CDC(buf.get(&piv, static_cast<size_t>(max_vectors) + 1));
    CDC(buf.get(&dq, maxq));
    CDC(buf.get(&ditem, 1));
    CDC(buf.get(&st, 1));
    CDC(hipMemcpyAsync(dcidx, cidx.data(), cidx.size() * sizeof(int), hipMemcpyHostToDevice, s));
    CDC(hipMemcpyAsync(dpm, pm.data(), pm.size() * sizeof(int), hipMemcpyHostToDevice, s));
    CDC(hipMemcpyAsync(dpn, pn.data(), pn.size() * sizeof(int), hipMemcpyHostToDevice, s));
    CDC(hipMemcpyAsync(dsig, sig.data(), sig.size() * sizeof(long long), hipMemcpyHostToDevice, s));
    CDC(hipMemcpyAsync(duf0, v.uf0.data(), v.uf0.size() * sizeof(int), hipMemcpyHostToDevice, s));
    const CdState st0{0, 0, 0.0};
    CDC(hipMemcpyAsync(st, &st0, sizeof st0, hipMemcpyHostToDevice, s));
    CDC(launch_zero(V, nsig * nsig, s));
    CDC(hipStreamSynchronize(s));

    // the operator pool: integral tiles of every kept quartet, scattered into V
    for (int X = 0; X < kNumPairClass; ++X)
        for (int Y = 0; Y <= X; ++Y) {
            const int cls = quartet_class(X, Y);
            const std::vector<int2>& list = qs[cls];
            if (list.empty()) continue;
            const int la = kPairLs[X][0], lb = kPairLs[X][1], lc = kPairLs[Y][0], ld = kPairLs[Y][1];
            const int NF = ncart_of(la) * ncart_of(lb) * ncart_of(lc) * ncart_of(ld);
            const long long chunk = kCdTileElems / NF;
            CDC(hipStreamSynchronize(s));   // the previous class's launches no longer read dq
            CDC(hipMemcpy(dq, list.data(), list.size() * sizeof(int2), hipMemcpyHostToDevice));
            for (long long q0 = 0; q0 < static_cast<long long>(list.size()); q0 += chunk) {
                const long long n = std::min<long long>(chunk, static_cast<long long>(list.size()) - q0);
                EriItem it{};
                it.quartets = dq + q0;
                it.n = n;
                CDC(hipStreamSynchronize(s));   // the previous chunk's launch has read ditem
                CDC(hipMemcpy(ditem, &it, sizeof it, hipMemcpyHostToDevice));
                EriTileArgs a{};
                a.items = ditem;
                a.nitems = 1;
                a.nblocks = (n + 255) / 256;
                a.block = 256;
                a.mol0.pairs = v.d_pairs;
                a.mol0.prims = v.d_prims;
                a.mol0.pslots = v.pslots;
                a.mol0.ns = v.ns;
                a.boys = v.d_boys;
                a.boys32 = v.d_boys32;
                a.tol = 0.0;
                a.tiles = tiles;
                a.scratch = scr;
                CDC(launch_eri_tile(cls, a, s, 0));
                CdScatterArgs c{};
                c.tiles = tiles;
                c.n = n;
                c.quartets = dq + q0;
                c.pairs = v.d_pairs;
                c.uf0 = duf0;
                c.umap = v.d_umap;
                c.cidx = dcidx;
                c.nsig = nsig;
                c.V = V;
                const int ls[4] = {la, lb, lc, ld};
                for (int i = 0; i < 4; ++i) {
                    c.nc[i] = ncart_of(ls[i]);
                    c.nu[i] = v.spherical ? 2 * ls[i] + 1 : ncart_of(ls[i]);
                }
                CDC(launch_cd_scatter(c, s));
            }
        }

    // pivoted Cholesky: device-side steps, the host reading the loop state
    // after every few of them
    CDC(launch_cd_diag(V, nsig, d, bmax, s));
    CdState hs{0, 0, 0.0};
    int poll = kCdPollFirst;
    for (int k = 0; k <= max_vectors;) {
        const int kend = std::min(k + poll, max_vectors + 1);
        for (; k < kend; ++k) CDC(launch_cd_step(V, nsig, Bc, d, bmax, piv, delta, k, max_vectors, st, s));
        CDC(hipMemcpyAsync(&hs, st, sizeof hs, hipMemcpyDeviceToHost, s));
        CDC(hipStreamSynchronize(s));
        if (hs.done) break;
        poll = std::min(2 * poll, kCdPollMax);
    }
    if (hs.done != 1) {
        *nvec_out = max_vectors;
        return cfail(JK_ENOMEM, "jk_cd_factor: more than max_vectors=%d vectors are needed at delta=%g", max_vectors,
                     delta);
    }
    const int nvec = hs.nvec;
    if (nvec > 0) {
        CDC(launch_zero(B, static_cast<long long>(nvec) * nf * nf, s));
        CDC(launch_cd_expand(Bc, nsig, nvec, dpm, dpn, nf, B, piv, dsig, pivots, s));
    }
    CDC(hipStreamSynchronize(s));
    *nvec_out = nvec;
    return JK_OK;
}

int jk_cd_jk(int32_t nf, int32_t nvec, const double* B, int32_t nd, int32_t r, const double* U, const double* V,
             double* J, double* K, void* stream) {
    if (nf < 1 || nvec < 0 || nd < 0 || r < 1)
        return cfail(JK_EINVAL, "jk_cd_jk: bad sizes nf=%d nvec=%d nd=%d r=%d", nf, nvec, nd, r);
    if (!J && !K) return cfail(JK_EINVAL, "jk_cd_jk: J and K both NULL");
    if (nd == 0) return JK_OK;
    if ((nvec > 0 && !B) || !U || !V) return cfail(JK_EINVAL, "jk_cd_jk: NULL input");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const long long nn = static_cast<long long>(nf) * nf;
    if (nvec == 0) {
        if (J) CDC(launch_zero(J, nd * nn, s));
        if (K) CDC(launch_zero(K, nd * nn, s));
        return JK_OK;
    }
    const long long vr = static_cast<long long>(nvec) * r;
    // split-K chunks of the two long contractions (gamma over nf^2, K over nvec r)
    const long long kg = 4096, kk = 1024;
    const int ng = static_cast<int>((nn + kg - 1) / kg), nk = static_cast<int>((vr + kk - 1) / kk);
    const long long gparts = static_cast<long long>(ng) * nvec * nd;
    const long long kparts = static_cast<long long>(nk) * nn;
    // K runs over groups of xg densities whose half-transforms B U, B V fit
    // the group budget together
    const long long per = 2 * static_cast<long long>(nf) * vr;
    const int xg = static_cast<int>(std::max<long long>(1, std::min<long long>(nd, kCdGroupElems / per)));
    // scratch: D [nd][nf][nf], gamma parts and gamma (J); BU, BV [xg][nf][nvec r],
    // the group's factors [nf][xg r] twice and the K parts (K)
    const long long wj = J ? nd * nn + gparts + static_cast<long long>(nvec) * nd : 0;
    const long long wk = K ? xg * per + 2 * static_cast<long long>(nf) * xg * r + kparts : 0;
    Scratch sc(s);
    if (sc.get(static_cast<size_t>(wj + wk) * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return cfail(JK_ENOMEM, "jk_cd_jk: %.1f GB of scratch could not be allocated", 8.0 * (wj + wk) / 1e9);
    }
    double* w = static_cast<double*>(sc.p);
    if (J) {
        double* D = w;
        double* gp = D + nd * nn;
        double* gamma = gp + gparts;
        // D[x] = U[x] V[x]^T
        GemmArgs g{U, V, D, nf, nf, r, 0, 1, r, r, nf, static_cast<long long>(nf) * r,
                   static_cast<long long>(nf) * r, nn, 1.0, 0.0};
        CDC(launch_gemm(g, nd, s));
        // gamma[Q][x] = sum_P B[Q][P] D[x][P]: split over P in ng chunks of kg
        // (the last one shorter), then summed
        GemmArgs a{B, D, gp, nvec, nd, static_cast<int>(kg), 0, 1, static_cast<int>(nn), static_cast<int>(nn), nd,
                   kg, kg, static_cast<long long>(nvec) * nd, 1.0, 0.0};
        a.klast = static_cast<int>(nn - (ng - 1) * kg);
        CDC(launch_gemm(a, ng, s));
        CDC(launch_cd_sum(gp, ng, static_cast<long long>(nvec) * nd, static_cast<long long>(nvec) * nd, gamma, s));
        // J[x][P] = sum_Q gamma[Q][x] B[Q][P]
        GemmArgs jj{gamma, B, J, nd, static_cast<int>(nn), nvec, 1, 0, nd, static_cast<int>(nn), static_cast<int>(nn),
                    0, 0, 0, 1.0, 0.0};
        CDC(launch_gemm(jj, 1, s));
    }
    if (K) {
        double* BU = w + wj;
        double* BV = BU + xg * (per / 2);
        double* UG = BV + xg * (per / 2);
        double* VG = UG + static_cast<long long>(nf) * xg * r;
        double* kp = VG + static_cast<long long>(nf) * xg * r;
        for (int x0 = 0; x0 < nd; x0 += xg) {
            const int nx = std::min(xg, nd - x0);
            const int wcol = nx * r;
            CDC(launch_cd_gather(U, nf, r, x0, nx, UG, s));
            CDC(launch_cd_gather(V, nf, r, x0, nx, VG, s));
            // BU_x[mu][(Q, m)] = sum_k B[Q][mu][k] U[x][k][m] for the whole group at
            // once: one product per Q against the group's factors side by side,
            // its column groups of r stored density-major
            GemmArgs bu{B, UG, BU, nf, wcol, nf, 0, 0, nf, wcol, static_cast<int>(vr), nn, 0, r, 1.0, 0.0,
                        r, static_cast<long long>(nf) * vr};
            CDC(launch_gemm(bu, nvec, s));
            GemmArgs bv{B, VG, BV, nf, wcol, nf, 0, 0, nf, wcol, static_cast<int>(vr), nn, 0, r, 1.0, 0.0,
                        r, static_cast<long long>(nf) * vr};
            CDC(launch_gemm(bv, nvec, s));
            for (int xl = 0; xl < nx; ++xl) {
                const double* BUx = BU + static_cast<long long>(xl) * nf * vr;
                const double* BVx = BV + static_cast<long long>(xl) * nf * vr;
                // K[mu][nu] = sum_(Q,m) BU_x[mu][(Q,m)] BV_x[nu][(Q,m)], split over (Q, m)
                // in nk chunks of kk (the last one shorter)
                double* Kx = K + static_cast<long long>(x0 + xl) * nn;
                GemmArgs a{BUx, BVx, kp, nf, nf, static_cast<int>(kk), 0, 1, static_cast<int>(vr),
                           static_cast<int>(vr), nf, kk, kk, nn, 1.0, 0.0};
                a.klast = static_cast<int>(vr - (nk - 1) * kk);
                CDC(launch_gemm(a, nk, s));
                const int nb = nk;
                CDC(launch_cd_sum(kp, nb, nn, nn, Kx, s));
            }
        }
    }
    return JK_OK;
}

}  // extern "C"
