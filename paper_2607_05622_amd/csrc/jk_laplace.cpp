// Laplace grids and the forward Laplace cascade (Sect. 2): host entry points.
//
// jk_laplace_grid      minimax grid of Eq. (laplace) (Remez exchange, jk_remez.h)
// jk_laplace_shift     omega-shifted weights of Eq. (eomshift)
// jk_laplace_densities level-k AO densities of Eqs. (scaledcoeff), (aodensk)
// jk_laplace_fock      Laplace-Fock back-transform of Eq. (laplacefock) and
//                      its occupied-virtual block, the next level's residual
// jk_laplace_step      one forward edge of the cascade: J/K build of the
//                      level-(k-1) densities, back-transform, level-k densities
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "jk.h"
#include "jk_gemm.h"
#include "jk_remez.h"

// records the thread's error message (jk_host.cpp)
int record_error(int code, const char* msg);

namespace {

int lfail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return record_error(code, buf);
}

int hip_fail(const char* who, hipError_t e) {
    (void)hipGetLastError();
    return lfail(JK_EDEVICE, "%s: %s", who, hipGetErrorString(e));
}

// Device scratch for one call, released on the call's stream.
struct Scratch {
    hipStream_t s;
    void* p = nullptr;
    explicit Scratch(hipStream_t st) : s(st) {}
    hipError_t get(size_t bytes) { return hipMallocAsync(&p, bytes, s); }
    ~Scratch() {
        if (p) (void)hipFreeAsync(p, s);
    }
};

}  // namespace

extern "C" {

int jk_laplace_grid(int32_t n, double xmin, double xmax, double* tau, double* w, double* max_err) {
    if (n < 1 || n > JK_LAPLACE_MAX_POINTS)
        return lfail(JK_EINVAL, "jk_laplace_grid: n=%d outside 1..%d", n, JK_LAPLACE_MAX_POINTS);
    if (!(xmin > 0.0) || !(xmax > xmin) || !std::isfinite(xmax))
        return lfail(JK_EINVAL, "jk_laplace_grid: need 0 < xmin < xmax < inf (got %g, %g)", xmin, xmax);
    if (!tau || !w) return lfail(JK_EINVAL, "jk_laplace_grid: NULL output");
    const jk::RemezResult r = jk::remez_inverse(n, xmax / xmin);
    if (!r.ok)
        return lfail(JK_EUNSUPPORTED,
                     r.precision_limited
                         ? "jk_laplace_grid: fewer than %d points already reach the FP64 rounding floor on a range ratio %g"
                         : "jk_laplace_grid: the exchange did not converge for %d points on a range ratio %g; use fewer",
                     n, xmax / xmin);
    for (int k = 0; k < n; ++k) {
        tau[k] = r.t[k] / xmin;
        w[k] = r.w[k] / xmin;
    }
    if (max_err) *max_err = r.err / xmin;
    return JK_OK;
}

int jk_laplace_shift(int32_t n, const double* tau, const double* w, double omega, double dmin, double* w_out) {
    if (n < 1 || !tau || !w || !w_out) return lfail(JK_EINVAL, "jk_laplace_shift: bad arguments");
    if (!std::isfinite(omega) || !(omega < dmin))
        return lfail(JK_EINVAL, "jk_laplace_shift: omega=%g must lie below the smallest denominator %g", omega, dmin);
    for (int k = 0; k < n; ++k) w_out[k] = w[k] * std::exp(omega * tau[k]);
    return JK_OK;
}

int jk_laplace_densities(int32_t n, int32_t nocc, int32_t nvir, const double* C, const double* eps, int32_t ntau,
                         const double* tau, int32_t nr, const double* R, double* D, void* stream) {
    if (n < 1 || nocc < 1 || nvir < 1 || nr < 1 || ntau < 1 || ntau > JK_LAPLACE_MAX_POINTS || !C || !eps || !tau ||
        !R || !D)
        return lfail(JK_EINVAL, "jk_laplace_densities: bad arguments");
    const int nmo = nocc + nvir;
    hipStream_t s = static_cast<hipStream_t>(stream);
    jk::ScaleTaus taus{};
    taus.n = ntau;
    for (int k = 0; k < ntau; ++k) {
        if (!std::isfinite(tau[k])) return lfail(JK_EINVAL, "jk_laplace_densities: tau[%d] not finite", k);
        taus.t[k] = tau[k];
    }
    const size_t nU = static_cast<size_t>(ntau) * n * nocc, nV = static_cast<size_t>(ntau) * n * nvir,
                 nY = static_cast<size_t>(nr) * n * nvir;
    Scratch ws(s);
    hipError_t e = ws.get((nU + nV + nY) * sizeof(double));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return lfail(JK_ENOMEM, "jk_laplace_densities: cannot allocate %zu bytes", (nU + nV + nY) * sizeof(double));
    }
    double* const U = static_cast<double*>(ws.p);
    double* const V = U + nU;
    double* const Y = V + nV;
    // U^k = C_occ exp(+eps_i tau_k), V^k = C_vir exp(-eps_a tau_k)
    e = jk::launch_scale_cols(C, n, nmo, 0, nocc, eps, taus, 1.0, U, s);
    if (e == hipSuccess) e = jk::launch_scale_cols(C, n, nmo, nocc, nvir, eps, taus, -1.0, V, s);
    for (int k = 0; k < ntau && e == hipSuccess; ++k) {
        // Y[r] = U^k R[r]  (n x nvir)
        jk::GemmArgs g1{U + static_cast<size_t>(k) * n * nocc, R, Y, n, nvir, nocc, 0, 0, nocc, nvir, nvir,
                        0, static_cast<long long>(nocc) * nvir, static_cast<long long>(n) * nvir, 1.0, 0.0};
        e = jk::launch_gemm(g1, nr, s);
        // D[r][k] = Y[r] (V^k)^T  (n x n)
        jk::GemmArgs g2{Y, V + static_cast<size_t>(k) * n * nvir, D + static_cast<size_t>(k) * n * n, n, n, nvir, 0, 1,
                        nvir, nvir, n, static_cast<long long>(n) * nvir, 0, static_cast<long long>(ntau) * n * n, 1.0,
                        0.0};
        if (e == hipSuccess) e = jk::launch_gemm(g2, nr, s);
    }
    if (e != hipSuccess) return hip_fail("jk_laplace_densities", e);
    return JK_OK;
}

int jk_laplace_fock(int32_t n, int32_t nocc, int32_t nvir, const double* C, int32_t nd, const double* J,
                    const double* K, double* F, double* Rov, void* stream) {
    if (n < 1 || nocc < 1 || nvir < 1 || nd < 1 || !C || !J || !K || (!F && !Rov))
        return lfail(JK_EINVAL, "jk_laplace_fock: bad arguments");
    const int nmo = nocc + nvir;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // densities in chunks, so the scratch (2J - K and (2J - K) C) stays bounded
    const int chunk = nd < 64 ? nd : 64;
    const size_t nT = static_cast<size_t>(chunk) * n * n, nZ = static_cast<size_t>(chunk) * n * nmo;
    Scratch ws(s);
    hipError_t e = ws.get((nT + nZ) * sizeof(double));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return lfail(JK_ENOMEM, "jk_laplace_fock: cannot allocate %zu bytes", (nT + nZ) * sizeof(double));
    }
    double* const T = static_cast<double*>(ws.p);
    double* const Z = T + nT;
    const long long nn = static_cast<long long>(n) * n;
    for (int x0 = 0; x0 < nd && e == hipSuccess; x0 += chunk) {
        const int b = nd - x0 < chunk ? nd - x0 : chunk;
        e = jk::launch_axpby(b * nn, 2.0, J + x0 * nn, -1.0, K + x0 * nn, T, s);
        // Z = (2J - K) C  (n x nmo)
        jk::GemmArgs gz{T, C, Z, n, nmo, n, 0, 0, n, nmo, nmo, nn, 0, static_cast<long long>(n) * nmo, 1.0, 0.0};
        if (e == hipSuccess) e = jk::launch_gemm(gz, b, s);
        if (F && e == hipSuccess) {   // F = C^T Z  (nmo x nmo)
            jk::GemmArgs gf{C, Z, F + static_cast<size_t>(x0) * nmo * nmo, nmo, nmo, n, 1, 0, nmo, nmo, nmo, 0,
                            static_cast<long long>(n) * nmo, static_cast<long long>(nmo) * nmo, 1.0, 0.0};
            e = jk::launch_gemm(gf, b, s);
        }
        if (Rov && e == hipSuccess) {   // R = C_occ^T Z_vir  (nocc x nvir)
            jk::GemmArgs gr{C, Z + nocc, Rov + static_cast<size_t>(x0) * nocc * nvir, nocc, nvir, n, 1, 0, nmo, nmo,
                            nvir, 0, static_cast<long long>(n) * nmo, static_cast<long long>(nocc) * nvir, 1.0, 0.0};
            e = jk::launch_gemm(gr, b, s);
        }
    }
    if (e != hipSuccess) return hip_fail("jk_laplace_fock", e);
    return JK_OK;
}

int jk_laplace_step(jk_basis_t h, int32_t nd, const double* D, double* J, double* K, int32_t nocc, int32_t nvir,
                    const double* C, const double* eps, int32_t ntau, const double* tau, double* Rov, double* Dnext,
                    const jk_build_opts* o) {
    jk_build_opts def;
    if (!o) {
        jk_default_opts(&def);
        o = &def;
    }
    if (!h) return lfail(JK_EINVAL, "jk_laplace_step: NULL handle");
    if (!o->want_j || !o->want_k) return lfail(JK_EINVAL, "jk_laplace_step: the back-transform needs both J and K");
    const int n = jk_nbf(h);
    if (nocc < 1 || nvir < 1 || nocc + nvir > n)
        return lfail(JK_EINVAL, "jk_laplace_step: nocc=%d, nvir=%d for %d basis functions", nocc, nvir, n);
    if (!Rov || !Dnext) return lfail(JK_EINVAL, "jk_laplace_step: NULL output");
    int rc = jk_build(h, nd, D, J, K, o);
    if (rc) return rc;
    if ((rc = jk_laplace_fock(n, nocc, nvir, C, nd, J, K, nullptr, Rov, o->stream))) return rc;
    return jk_laplace_densities(n, nocc, nvir, C, eps, ntau, tau, nd, Rov, Dnext, o->stream);
}

}  // extern "C"
