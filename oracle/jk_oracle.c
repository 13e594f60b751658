/*
 * jk_oracle.c -- plain, slow, FP64 CPU oracle for the AO-direct J/K build.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it exists so that the tests, the smoke check and the CPU
 * baseline of the benchmark have an independent reference.  It shares no
 * code, header, table or constant generator with the GPU library.
 *
 * What it computes (the plain definitions, written out):
 *
 *   J(D)_{mn} = sum_{ls} (mn|ls) D_{ls},   K(D)_{mn} = sum_{ls} (ml|ns) D_{ls}
 *
 * for every density of a batch (paper Sect. 2.2, Eq. (jkbuild)); the
 * per-quartet scatter form over unique shell quartets (Sect. 3, Eq.
 * (quartet_scatter)) is the same sum regrouped.  Builds are bare: no 1/2,
 * no spin factor, no 2J-K (Sect. 2, "Notation and conventions").  D may be
 * any real matrix and is never symmetrized for K (Sect. 2.4).  Pure d
 * functions enter at matrix level, D_cart = T D T^T and J = T^T J_cart T
 * (Sect. 3, screening-robustness paragraph).
 *
 * Two-electron integrals over contracted Cartesian Gaussians are evaluated
 * with the McMurchie-Davidson scheme (Hermite expansion coefficients E and
 * Hermite Coulomb integrals R; Helgaker, Joergensen and Olsen, "Molecular
 * Electronic-Structure Theory", ch. 9).  This is deliberately a different
 * recurrence family from the Head-Gordon-Pople / Obara-Saika scheme that
 * the GPU path follows (Sect. 3, "DAG-driven, spill-bounded GPU chunking").
 *
 * The Boys function F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt is evaluated by
 * its power series (one series per m, long double) for T < 30 and by
 * F_0 = sqrt(pi/T) erf(sqrt T)/2 with upward recursion above.
 *
 * Screening: the same deterministic rule as the GPU path, restated here:
 * a shell quartet (ab|cd) is kept iff Q_ab Q_cd >= tol and
 * Q_ab Q_cd * Dmax >= tol, where Q_ab = sqrt(max_{m in a, n in b} (mn|mn))
 * (Cartesian functions) and Dmax is the largest |D_cart| over all densities
 * in the six shell-pair blocks ab, cd, ac, ad, bc, bd (both orientations).
 * tol = 0 keeps everything.  The rule is invariant under the eight index
 * permutations, so every ordered shell quartet inherits its canonical
 * representative's decision.
 *
 * Conventions of a basis (shared definition, not shared code): primitives
 * are normalized on their x^l component, a contraction is rescaled to unit
 * x^l self-overlap, Cartesian order is lexicographic, pure d is ordered
 * (xy, yz, 3z^2-r^2, xz, x^2-y^2) with each function normalized numerically.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXL 2
#define OR_MAXPRIM 16
#define OR_MAXM 12           /* Boys orders available: 0..OR_MAXM */
#define OR_MAXCART 6

typedef struct {
    int l, nprim, ncart, nfunc;
    double c[3];
    double a[OR_MAXPRIM];
    double w[OR_MAXPRIM];    /* coefficient x primitive norm x contraction scale */
    int cart_off, func_off;  /* offsets in the Cartesian / user function lists */
} or_shell;

typedef struct {
    int nshell, ncart, nfunc, spherical;
    or_shell* sh;
    double* T;               /* [ncart][nfunc]: phi_user = sum T[cart][user] phi_cart */
} or_basis;

static const int CARTX[3][6][3] = {
    {{0, 0, 0}},
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
    {{2, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}},
};

static int g_threads = 0;
void oracle_set_threads(int n) { g_threads = n; }
int oracle_get_threads(void) {
#ifdef _OPENMP
    return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Boys function                                                       */
/* ------------------------------------------------------------------ */

/* F_m(T) = exp(-T) sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1)) */
static double boys_series(int m, double T) {
    long double term = 1.0L / (2 * m + 1), sum = term;
    long double x2 = 2.0L * T;
    for (int k = 1; k < 2000; k++) {
        term *= x2 / (long double)(2 * m + 2 * k + 1);
        sum += term;
        if (term < 1e-21L * sum) break;
    }
    return (double)(expl(-(long double)T) * sum);
}

void oracle_boys(int mmax, double T, double* F) {
    if (T < 30.0) {
        for (int m = 0; m <= mmax; m++) F[m] = boys_series(m, T);
        return;
    }
    long double e = expl(-(long double)T);
    long double f = 0.5L * sqrtl(3.14159265358979323846264338327950288L / T) * erfl(sqrtl((long double)T));
    F[0] = (double)f;
    for (int m = 0; m < mmax; m++) {
        f = ((2 * m + 1) * f - e) / (2.0L * T);
        F[m + 1] = (double)f;
    }
}

/* ------------------------------------------------------------------ */
/* McMurchie-Davidson pieces                                           */
/* ------------------------------------------------------------------ */

/* Hermite expansion coefficients E[i][j][t] of x_A^i x_B^j on one axis
 * (the Gaussian-product exponential is kept outside). */
static void md_E(int la, int lb, double p, double PA, double PB, double E[3][3][5]) {
    memset(E, 0, sizeof(double) * 3 * 3 * 5);
    double o2p = 0.5 / p;
    E[0][0][0] = 1.0;
    for (int i = 0; i <= la; i++) {
        for (int j = 0; j <= lb; j++) {
            if (i == 0 && j == 0) continue;
            for (int t = 0; t <= i + j; t++) {
                double v;
                if (i > 0) {
                    v = PA * E[i - 1][j][t];
                    if (t > 0) v += o2p * E[i - 1][j][t - 1];
                    if (t + 1 <= i - 1 + j) v += (t + 1) * E[i - 1][j][t + 1];
                } else {
                    v = PB * E[i][j - 1][t];
                    if (t > 0) v += o2p * E[i][j - 1][t - 1];
                    if (t + 1 <= i + j - 1) v += (t + 1) * E[i][j - 1][t + 1];
                }
                E[i][j][t] = v;
            }
        }
    }
}

#define RDIM 9   /* t,u,v <= 8 */
/* Hermite Coulomb integrals R^0_{tuv}(rho, PQ) for t+u+v <= L. */
static void md_R(int L, double rho, const double PQ[3], double* R0 /* [RDIM^3] */) {
    static const int S = RDIM;
    double T = rho * (PQ[0] * PQ[0] + PQ[1] * PQ[1] + PQ[2] * PQ[2]);
    double F[OR_MAXM + 1];
    oracle_boys(L, T, F);
    /* Rn[n][t][u][v] */
    double Rn[RDIM][RDIM][RDIM][RDIM];
    double f = 1.0;
    for (int n = 0; n <= L; n++) {
        Rn[n][0][0][0] = f * F[n];
        f *= -2.0 * rho;
    }
    /* build by total order: R^n_{tuv} needs R^{n+1} at lower total order */
    for (int tot = 1; tot <= L; tot++) {
        for (int n = 0; n + tot <= L; n++) {
            for (int t = 0; t <= tot; t++) {
                for (int u = 0; u + t <= tot; u++) {
                    int v = tot - t - u;
                    double val;
                    if (t > 0) {
                        val = PQ[0] * Rn[n + 1][t - 1][u][v];
                        if (t > 1) val += (t - 1) * Rn[n + 1][t - 2][u][v];
                    } else if (u > 0) {
                        val = PQ[1] * Rn[n + 1][t][u - 1][v];
                        if (u > 1) val += (u - 1) * Rn[n + 1][t][u - 2][v];
                    } else {
                        val = PQ[2] * Rn[n + 1][t][u][v - 1];
                        if (v > 1) val += (v - 1) * Rn[n + 1][t][u][v - 2];
                    }
                    Rn[n][t][u][v] = val;
                }
            }
        }
    }
    for (int t = 0; t <= L; t++)
        for (int u = 0; u + t <= L; u++)
            for (int v = 0; v + t + u <= L; v++) R0[(t * S + u) * S + v] = Rn[0][t][u][v];
}

/* Contracted Cartesian ERI tile (ab|cd), out[ia][ib][ic][id]. */
static void eri_quartet(const or_shell* A, const or_shell* B, const or_shell* C,
                        const or_shell* D, double* out) {
    const int na = A->ncart, nb = B->ncart, nc = C->ncart, nd = D->ncart;
    const int L = A->l + B->l + C->l + D->l;
    const int Lab = A->l + B->l, Lcd = C->l + D->l;
    const double pi = 3.14159265358979323846;
    memset(out, 0, sizeof(double) * na * nb * nc * nd);
    double AB2 = 0, CD2 = 0;
    for (int k = 0; k < 3; k++) {
        AB2 += (A->c[k] - B->c[k]) * (A->c[k] - B->c[k]);
        CD2 += (C->c[k] - D->c[k]) * (C->c[k] - D->c[k]);
    }
    static const int S = RDIM;
    double R0[RDIM * RDIM * RDIM];
    double Eab[3][3][3][5], Ecd[3][3][3][5];
    /* W[tuv][ic][id] = sum_{tau nu phi} (-1)^{tau+nu+phi} E^{cd}_{tau nu phi} R_{t+tau,u+nu,v+phi} */
    double W[RDIM * RDIM * RDIM][OR_MAXCART * OR_MAXCART];
    for (int i = 0; i < A->nprim; i++)
    for (int j = 0; j < B->nprim; j++) {
        double a = A->a[i], b = B->a[j], p = a + b;
        double P[3];
        for (int k = 0; k < 3; k++) {
            P[k] = (a * A->c[k] + b * B->c[k]) / p;
            md_E(A->l, B->l, p, P[k] - A->c[k], P[k] - B->c[k], Eab[k]);
        }
        double Kab = exp(-a * b / p * AB2) * A->w[i] * B->w[j];
        for (int k2 = 0; k2 < C->nprim; k2++)
        for (int l2 = 0; l2 < D->nprim; l2++) {
            double c = C->a[k2], d = D->a[l2], q = c + d;
            double Q[3], PQ[3];
            for (int k = 0; k < 3; k++) {
                Q[k] = (c * C->c[k] + d * D->c[k]) / q;
                md_E(C->l, D->l, q, Q[k] - C->c[k], Q[k] - D->c[k], Ecd[k]);
                PQ[k] = P[k] - Q[k];
            }
            double rho = p * q / (p + q);
            md_R(L, rho, PQ, R0);
            double pref = 2.0 * pow(pi, 2.5) / (p * q * sqrt(p + q)) * Kab *
                          exp(-c * d / q * CD2) * C->w[k2] * D->w[l2];
            /* ket side first */
            for (int t = 0; t <= Lab; t++)
            for (int u = 0; u + t <= Lab; u++)
            for (int v = 0; v + t + u <= Lab; v++) {
                double* w = W[(t * S + u) * S + v];
                for (int ic = 0; ic < nc; ic++)
                for (int id = 0; id < nd; id++) {
                    const int* cx = CARTX[C->l][ic];
                    const int* dx = CARTX[D->l][id];
                    double s = 0.0;
                    for (int tt = 0; tt <= cx[0] + dx[0]; tt++)
                    for (int uu = 0; uu <= cx[1] + dx[1]; uu++)
                    for (int vv = 0; vv <= cx[2] + dx[2]; vv++) {
                        double e = Ecd[0][cx[0]][dx[0]][tt] * Ecd[1][cx[1]][dx[1]][uu] *
                                   Ecd[2][cx[2]][dx[2]][vv];
                        if ((tt + uu + vv) & 1) e = -e;
                        s += e * R0[((t + tt) * S + (u + uu)) * S + (v + vv)];
                    }
                    w[ic * nd + id] = s;
                }
            }
            (void)Lcd;
            /* bra side */
            for (int ia = 0; ia < na; ia++)
            for (int ib = 0; ib < nb; ib++) {
                const int* ax = CARTX[A->l][ia];
                const int* bx = CARTX[B->l][ib];
                double* o = out + (ia * nb + ib) * nc * nd;
                for (int t = 0; t <= ax[0] + bx[0]; t++)
                for (int u = 0; u <= ax[1] + bx[1]; u++)
                for (int v = 0; v <= ax[2] + bx[2]; v++) {
                    double e = pref * Eab[0][ax[0]][bx[0]][t] * Eab[1][ax[1]][bx[1]][u] *
                               Eab[2][ax[2]][bx[2]][v];
                    const double* w = W[(t * S + u) * S + v];
                    for (int k = 0; k < nc * nd; k++) o[k] += e * w[k];
                }
            }
        }
    }
}

/* Overlap tile <a|b>, out[ia][ib], Cartesian. */
static void overlap_pair(const or_shell* A, const or_shell* B, double* out) {
    const double pi = 3.14159265358979323846;
    memset(out, 0, sizeof(double) * A->ncart * B->ncart);
    double AB2 = 0;
    for (int k = 0; k < 3; k++) AB2 += (A->c[k] - B->c[k]) * (A->c[k] - B->c[k]);
    double E[3][3][3][5];
    for (int i = 0; i < A->nprim; i++)
    for (int j = 0; j < B->nprim; j++) {
        double a = A->a[i], b = B->a[j], p = a + b;
        for (int k = 0; k < 3; k++) {
            double P = (a * A->c[k] + b * B->c[k]) / p;
            md_E(A->l, B->l, p, P - A->c[k], P - B->c[k], E[k]);
        }
        double pref = pow(pi / p, 1.5) * exp(-a * b / p * AB2) * A->w[i] * B->w[j];
        for (int ia = 0; ia < A->ncart; ia++)
        for (int ib = 0; ib < B->ncart; ib++) {
            const int* ax = CARTX[A->l][ia];
            const int* bx = CARTX[B->l][ib];
            out[ia * B->ncart + ib] += pref * E[0][ax[0]][bx[0]][0] * E[1][ax[1]][bx[1]][0] *
                                       E[2][ax[2]][bx[2]][0];
        }
    }
}

/* ------------------------------------------------------------------ */
/* basis set-up                                                        */
/* ------------------------------------------------------------------ */

static double dfact(int n) {
    double r = 1;
    while (n > 1) { r *= n; n -= 2; }
    return r;
}

static void free_basis(or_basis* b) {
    free(b->sh);
    free(b->T);
    b->sh = NULL;
    b->T = NULL;
}

/* Returns 0 on success, -1 on an invalid descriptor. */
static int make_basis(or_basis* b, int natoms, const double* xyz, int nshells, const int* shell_atom,
                      const int* shell_l, const int* shell_nprim, const double* exps,
                      const double* coefs, int spherical) {
    const double pi = 3.14159265358979323846;
    memset(b, 0, sizeof(*b));
    if (nshells < 0 || natoms < 1) return -1;
    b->nshell = nshells;
    b->spherical = spherical;
    b->sh = (or_shell*)calloc(nshells > 0 ? nshells : 1, sizeof(or_shell));
    int po = 0, co = 0, fo = 0;
    for (int s = 0; s < nshells; s++) {
        or_shell* S = &b->sh[s];
        int l = shell_l[s], np = shell_nprim[s], at = shell_atom[s];
        if (l < 0 || l > OR_MAXL || np < 1 || np > OR_MAXPRIM || at < 0 || at >= natoms) {
            free_basis(b);
            return -1;
        }
        S->l = l;
        S->nprim = np;
        S->ncart = (l + 1) * (l + 2) / 2;
        S->nfunc = (spherical && l == 2) ? 5 : S->ncart;
        for (int k = 0; k < 3; k++) S->c[k] = xyz[3 * at + k];
        for (int i = 0; i < np; i++) {
            double a = exps[po + i];
            if (!(a > 0) || !isfinite(a) || !isfinite(coefs[po + i])) { free_basis(b); return -1; }
            S->a[i] = a;
            S->w[i] = coefs[po + i] * sqrt(pow(2 * a / pi, 1.5) * pow(4 * a, l) / dfact(2 * l - 1));
        }
        /* rescale the contraction to unit self-overlap of its x^l component */
        double ov[36];
        overlap_pair(S, S, ov);
        double sc = 1.0 / sqrt(ov[0]);
        for (int i = 0; i < np; i++) S->w[i] *= sc;
        S->cart_off = co;
        S->func_off = fo;
        po += np;
        co += S->ncart;
        fo += S->nfunc;
    }
    b->ncart = co;
    b->nfunc = fo;
    b->T = (double*)calloc((size_t)(co > 0 ? co : 1) * (fo > 0 ? fo : 1), sizeof(double));
    for (int s = 0; s < nshells; s++) {
        or_shell* S = &b->sh[s];
        if (S->nfunc == S->ncart) {
            for (int i = 0; i < S->ncart; i++) b->T[(size_t)(S->cart_off + i) * fo + S->func_off + i] = 1.0;
            continue;
        }
        /* pure d: polynomial coefficients over (xx, xy, xz, yy, yz, zz),
         * normalized with this shell's own Cartesian overlap */
        static const double poly[5][6] = {
            {0, 1, 0, 0, 0, 0},      /* xy */
            {0, 0, 0, 0, 1, 0},      /* yz */
            {-1, 0, 0, -1, 0, 2},    /* 2zz - xx - yy */
            {0, 0, 1, 0, 0, 0},      /* xz */
            {1, 0, 0, -1, 0, 0},     /* xx - yy */
        };
        double ov[36];
        overlap_pair(S, S, ov);
        for (int m = 0; m < 5; m++) {
            double n2 = 0;
            for (int i = 0; i < 6; i++)
                for (int j = 0; j < 6; j++) n2 += poly[m][i] * ov[i * 6 + j] * poly[m][j];
            double sc = 1.0 / sqrt(n2);
            for (int i = 0; i < 6; i++)
                b->T[(size_t)(S->cart_off + i) * fo + S->func_off + m] = poly[m][i] * sc;
        }
    }
    return 0;
}

#define BASIS_ARGS int natoms, const double *xyz, int nshells, const int *shell_atom, \
    const int *shell_l, const int *shell_nprim, const double *exps, const double *coefs, int spherical
#define BASIS_PASS natoms, xyz, nshells, shell_atom, shell_l, shell_nprim, exps, coefs, spherical

int oracle_nbf(BASIS_ARGS) {
    or_basis b;
    if (make_basis(&b, BASIS_PASS)) return -1;
    int n = b.nfunc;
    free_basis(&b);
    return n;
}

int oracle_ncart(BASIS_ARGS) {
    or_basis b;
    if (make_basis(&b, BASIS_PASS)) return -1;
    int n = b.ncart;
    free_basis(&b);
    return n;
}

/* T matrix [ncart][nfunc]. */
int oracle_cart_to_basis(BASIS_ARGS, double* T) {
    or_basis b;
    if (make_basis(&b, BASIS_PASS)) return -1;
    memcpy(T, b.T, sizeof(double) * b.ncart * b.nfunc);
    free_basis(&b);
    return 0;
}

/* Contracted, normalized Cartesian ERI tile of shells (a b | c d). */
int oracle_eri_shell_quartet(BASIS_ARGS, int a, int bb, int c, int d, double* out) {
    or_basis b;
    if (make_basis(&b, BASIS_PASS)) return -1;
    if (a < 0 || bb < 0 || c < 0 || d < 0 || a >= b.nshell || bb >= b.nshell || c >= b.nshell ||
        d >= b.nshell) {
        free_basis(&b);
        return -1;
    }
    eri_quartet(&b.sh[a], &b.sh[bb], &b.sh[c], &b.sh[d], out);
    free_basis(&b);
    return 0;
}

/* Full Cartesian ERI tensor [nc^4] (no symmetry used). */
static double* full_cart_eri(const or_basis* b) {
    size_t n = b->ncart;
    double* G = (double*)calloc(n * n * n * n, sizeof(double));
    int ns = b->nshell;
#pragma omp parallel for schedule(dynamic) collapse(2) num_threads(oracle_get_threads())
    for (int sa = 0; sa < ns; sa++)
    for (int sb = 0; sb < ns; sb++) {
        double tile[1296];
        const or_shell *A = &b->sh[sa], *B = &b->sh[sb];
        for (int sc = 0; sc < ns; sc++)
        for (int sd = 0; sd < ns; sd++) {
            const or_shell *C = &b->sh[sc], *D = &b->sh[sd];
            eri_quartet(A, B, C, D, tile);
            for (int i = 0; i < A->ncart; i++)
            for (int j = 0; j < B->ncart; j++)
            for (int k = 0; k < C->ncart; k++)
            for (int l = 0; l < D->ncart; l++)
                G[(((size_t)(A->cart_off + i) * n + B->cart_off + j) * n + C->cart_off + k) * n +
                  D->cart_off + l] = tile[((i * B->ncart + j) * C->ncart + k) * D->ncart + l];
        }
    }
    return G;
}

/* Full ERI tensor in the basis' own functions, [nf^4] (brute force). */
int oracle_eri_full(BASIS_ARGS, double* out) {
    or_basis b;
    if (make_basis(&b, BASIS_PASS)) return -1;
    size_t nc = b.ncart, nf = b.nfunc;
    double* G = full_cart_eri(&b);
    /* transform one index at a time: out = T^T x T^T x T^T x T^T applied to G */
    double* X = (double*)calloc(nc * nc * nc * nf, sizeof(double));
    double* Y = (double*)calloc(nc * nc * nf * nf, sizeof(double));
    double* Z = (double*)calloc(nc * nf * nf * nf, sizeof(double));
    for (size_t i = 0; i < nc * nc * nc; i++)
        for (size_t l = 0; l < nc; l++)
            for (size_t m = 0; m < nf; m++) X[i * nf + m] += G[i * nc + l] * b.T[l * nf + m];
    for (size_t i = 0; i < nc * nc; i++)
        for (size_t k = 0; k < nc; k++)
            for (size_t m = 0; m < nf; m++)
                for (size_t q = 0; q < nf; q++)
                    Y[(i * nf + m) * nf + q] += X[(i * nc + k) * nf + q] * b.T[k * nf + m];
    for (size_t i = 0; i < nc; i++)
        for (size_t j = 0; j < nc; j++)
            for (size_t m = 0; m < nf; m++)
                for (size_t r = 0; r < nf * nf; r++)
                    Z[(i * nf + m) * nf * nf + r] += Y[(i * nc + j) * nf * nf + r] * b.T[j * nf + m];
    memset(out, 0, sizeof(double) * nf * nf * nf * nf);
    for (size_t i = 0; i < nc; i++)
        for (size_t m = 0; m < nf; m++)
            for (size_t r = 0; r < nf * nf * nf; r++)
                out[m * nf * nf * nf + r] += Z[i * nf * nf * nf + r] * b.T[i * nf + m];
    free(G);
    free(X);
    free(Y);
    free(Z);
    free_basis(&b);
    return 0;
}

/* Overlap matrix in the basis' own functions, [nf][nf]. */
int oracle_overlap(BASIS_ARGS, double* S) {
    or_basis b;
    if (make_basis(&b, BASIS_PASS)) return -1;
    size_t nc = b.ncart, nf = b.nfunc;
    double* Sc = (double*)calloc(nc * nc, sizeof(double));
    double tile[36];
    for (int i = 0; i < b.nshell; i++)
        for (int j = 0; j < b.nshell; j++) {
            overlap_pair(&b.sh[i], &b.sh[j], tile);
            for (int u = 0; u < b.sh[i].ncart; u++)
                for (int v = 0; v < b.sh[j].ncart; v++)
                    Sc[(b.sh[i].cart_off + u) * nc + b.sh[j].cart_off + v] = tile[u * b.sh[j].ncart + v];
        }
    for (size_t m = 0; m < nf; m++)
        for (size_t n = 0; n < nf; n++) {
            double s = 0;
            for (size_t i = 0; i < nc; i++)
                for (size_t j = 0; j < nc; j++) s += b.T[i * nf + m] * Sc[i * nc + j] * b.T[j * nf + n];
            S[m * nf + n] = s;
        }
    free(Sc);
    free_basis(&b);
    return 0;
}

/* ------------------------------------------------------------------ */
/* matrix-level basis change                                           */
/* ------------------------------------------------------------------ */

/* Dc[x] = T D[x] T^T */
static double* to_cart(const or_basis* b, int nd, const double* D) {
    size_t nc = b->ncart, nf = b->nfunc;
    double* Dc = (double*)calloc((size_t)nd * nc * nc, sizeof(double));
    double* tmp = (double*)calloc(nc * nf, sizeof(double));
    for (int x = 0; x < nd; x++) {
        const double* Dx = D + (size_t)x * nf * nf;
        memset(tmp, 0, sizeof(double) * nc * nf);
        for (size_t i = 0; i < nc; i++)
            for (size_t m = 0; m < nf; m++) {
                double t = b->T[i * nf + m];
                if (t == 0) continue;
                for (size_t n = 0; n < nf; n++) tmp[i * nf + n] += t * Dx[m * nf + n];
            }
        double* o = Dc + (size_t)x * nc * nc;
        for (size_t i = 0; i < nc; i++)
            for (size_t j = 0; j < nc; j++) {
                double s = 0;
                for (size_t n = 0; n < nf; n++) s += tmp[i * nf + n] * b->T[j * nf + n];
                o[i * nc + j] = s;
            }
    }
    free(tmp);
    return Dc;
}

/* out[x] = T^T M[x] T */
static void from_cart(const or_basis* b, int nd, const double* M, double* out) {
    size_t nc = b->ncart, nf = b->nfunc;
    double* tmp = (double*)calloc(nf * nc, sizeof(double));
    for (int x = 0; x < nd; x++) {
        const double* Mx = M + (size_t)x * nc * nc;
        memset(tmp, 0, sizeof(double) * nf * nc);
        for (size_t i = 0; i < nc; i++)
            for (size_t m = 0; m < nf; m++) {
                double t = b->T[i * nf + m];
                if (t == 0) continue;
                for (size_t j = 0; j < nc; j++) tmp[m * nc + j] += t * Mx[i * nc + j];
            }
        double* o = out + (size_t)x * nf * nf;
        for (size_t m = 0; m < nf; m++)
            for (size_t n = 0; n < nf; n++) {
                double s = 0;
                for (size_t j = 0; j < nc; j++) s += tmp[m * nc + j] * b->T[j * nf + n];
                o[m * nf + n] = s;
            }
    }
    free(tmp);
}

/* ------------------------------------------------------------------ */
/* J/K                                                                 */
/* ------------------------------------------------------------------ */

/* J and K straight from the full tensor, literally as defined. */
int oracle_jk_brute(BASIS_ARGS, int nd, const double* D, double* J, double* K) {
    or_basis b;
    if (make_basis(&b, BASIS_PASS)) return -1;
    size_t n = b.ncart;
    double* G = full_cart_eri(&b);
    double* Dc = to_cart(&b, nd, D);
    double* Jc = (double*)calloc((size_t)nd * n * n, sizeof(double));
    double* Kc = (double*)calloc((size_t)nd * n * n, sizeof(double));
    for (int x = 0; x < nd; x++) {
        const double* d = Dc + (size_t)x * n * n;
        double* j = Jc + (size_t)x * n * n;
        double* k = Kc + (size_t)x * n * n;
        for (size_t m = 0; m < n; m++)
            for (size_t nn = 0; nn < n; nn++) {
                double sj = 0, sk = 0;
                for (size_t l = 0; l < n; l++)
                    for (size_t s = 0; s < n; s++) {
                        sj += G[((m * n + nn) * n + l) * n + s] * d[l * n + s];   /* (mn|ls) D_ls */
                        sk += G[((m * n + l) * n + nn) * n + s] * d[l * n + s];   /* (ml|ns) D_ls */
                    }
                j[m * n + nn] = sj;
                k[m * n + nn] = sk;
            }
    }
    from_cart(&b, nd, Jc, J);
    from_cart(&b, nd, Kc, K);
    free(G);
    free(Dc);
    free(Jc);
    free(Kc);
    free_basis(&b);
    return 0;
}

/* Schwarz factors Q[a][b] = sqrt(max (mn|mn)), full nshell x nshell. */
static double* schwarz(const or_basis* b) {
    int ns = b->nshell;
    double* Q = (double*)calloc((size_t)ns * ns + 1, sizeof(double));
#pragma omp parallel for schedule(dynamic) num_threads(oracle_get_threads())
    for (int a = 0; a < ns; a++) {
        double tile[1296];
        for (int c = 0; c <= a; c++) {
            const or_shell *A = &b->sh[a], *C = &b->sh[c];
            eri_quartet(A, C, A, C, tile);
            double mx = 0;
            int n1 = A->ncart, n2 = C->ncart;
            for (int i = 0; i < n1; i++)
                for (int j = 0; j < n2; j++) {
                    double v = tile[((i * n2 + j) * n1 + i) * n2 + j];
                    if (v > mx) mx = v;
                }
            Q[a * ns + c] = Q[c * ns + a] = sqrt(mx);
        }
    }
    return Q;
}

int oracle_schwarz(BASIS_ARGS, double* Qout) {
    or_basis b;
    if (make_basis(&b, BASIS_PASS)) return -1;
    double* Q = schwarz(&b);
    memcpy(Qout, Q, sizeof(double) * b.nshell * b.nshell);
    free(Q);
    free_basis(&b);
    return 0;
}

/* Dmax over densities and both orientations, per shell pair. */
static double* pair_dmax(const or_basis* b, int nd, const double* Dc) {
    int ns = b->nshell;
    size_t n = b->ncart;
    double* M = (double*)calloc((size_t)ns * ns + 1, sizeof(double));
    for (int a = 0; a < ns; a++)
        for (int c = 0; c < ns; c++) {
            double mx = 0;
            for (int x = 0; x < nd; x++)
                for (int i = 0; i < b->sh[a].ncart; i++)
                    for (int j = 0; j < b->sh[c].ncart; j++) {
                        double v = fabs(Dc[(size_t)x * n * n + (b->sh[a].cart_off + i) * n + b->sh[c].cart_off + j]);
                        double w = fabs(Dc[(size_t)x * n * n + (b->sh[c].cart_off + j) * n + b->sh[a].cart_off + i]);
                        if (v > mx) mx = v;
                        if (w > mx) mx = w;
                    }
            M[a * ns + c] = mx;
        }
    return M;
}

static int keep_quartet(int ns, const double* Q, const double* M, int a, int b, int c, int d, double tol) {
    if (tol <= 0) return 1;
    double qq = Q[a * ns + b] * Q[c * ns + d];
    if (qq < tol) return 0;
    double m = M[a * ns + b];
    double v;
    v = M[c * ns + d]; if (v > m) m = v;
    v = M[a * ns + c]; if (v > m) m = v;
    v = M[a * ns + d]; if (v > m) m = v;
    v = M[b * ns + c]; if (v > m) m = v;
    v = M[b * ns + d]; if (v > m) m = v;
    return qq * m >= tol;
}

/* Number of canonical shell quartets kept by the screening rule
 * (a >= b, c >= d, ab >= cd). */
long long oracle_count_quartets(BASIS_ARGS, int nd, const double* D, double tol) {
    or_basis b;
    if (make_basis(&b, BASIS_PASS)) return -1;
    int ns = b.nshell;
    double* Dc = to_cart(&b, nd, D);
    double* Q = schwarz(&b);
    double* M = pair_dmax(&b, nd, Dc);
    long long cnt = 0;
    for (int a = 0; a < ns; a++)
        for (int bb = 0; bb <= a; bb++)
            for (int c = 0; c <= a; c++)
                for (int d = 0; d <= (c == a ? bb : c); d++)
                    cnt += keep_quartet(ns, Q, M, a, bb, c, d, tol);
    free(Dc);
    free(Q);
    free(M);
    free_basis(&b);
    return cnt;
}

/* Screened build over canonical shell quartets; every *distinct* index
 * permutation of a kept quartet is scattered exactly once.  Only bra pairs
 * with index % stride == offset are visited (stride 1: the whole build);
 * *done receives the number of kept quartets visited, *total the number
 * kept over all bra pairs. */
static int jk_screened_strided(BASIS_ARGS, int nd, const double* D, double* J, double* K, double tol,
                               int stride, int offset, long long* done, long long* total);

int oracle_jk_screened(BASIS_ARGS, int nd, const double* D, double* J, double* K, double tol) {
    return jk_screened_strided(BASIS_PASS, nd, D, J, K, tol, 1, 0, NULL, NULL);
}

/* A bounded sample of the screened build (for timing the CPU baseline). */
int oracle_jk_screened_sample(BASIS_ARGS, int nd, const double* D, double* J, double* K, double tol,
                              int stride, int offset, long long* done, long long* total) {
    if (stride < 1 || offset < 0 || offset >= stride) return -1;
    return jk_screened_strided(BASIS_PASS, nd, D, J, K, tol, stride, offset, done, total);
}

static int jk_screened_strided(BASIS_ARGS, int nd, const double* D, double* J, double* K, double tol,
                               int stride, int offset, long long* done, long long* total) {
    or_basis b;
    if (make_basis(&b, BASIS_PASS)) return -1;
    int ns = b.nshell;
    size_t n = b.ncart;
    double* Dc = to_cart(&b, nd, D);
    double* Q = schwarz(&b);
    double* M = pair_dmax(&b, nd, Dc);
    size_t mat = (size_t)nd * n * n;
    double* Jc = (double*)calloc(mat, sizeof(double));
    double* Kc = (double*)calloc(mat, sizeof(double));
    int npair = ns * (ns + 1) / 2;
    int* pa = (int*)malloc(sizeof(int) * (npair + 1));
    int* pb = (int*)malloc(sizeof(int) * (npair + 1));
    for (int a = 0, k = 0; a < ns; a++)
        for (int bb = 0; bb <= a; bb++, k++) { pa[k] = a; pb[k] = bb; }
    long long n_done = 0, n_total = 0;
    if (total) {
        for (int pab = 0; pab < npair; pab++)
            for (int pcd = 0; pcd <= pab; pcd++)
                n_total += keep_quartet(ns, Q, M, pa[pab], pb[pab], pa[pcd], pb[pcd], tol);
    }
#pragma omp parallel num_threads(oracle_get_threads()) reduction(+ : n_done)
    {
        double* Jt = (double*)calloc(mat, sizeof(double));
        double* Kt = (double*)calloc(mat, sizeof(double));
        double tile[1296];
#pragma omp for schedule(dynamic)
        for (int pab = 0; pab < npair; pab++) {
            if (pab % stride != offset) continue;
            int a = pa[pab], bb = pb[pab];
            for (int pcd = 0; pcd <= pab; pcd++) {
                int c = pa[pcd], d = pb[pcd];
                if (!keep_quartet(ns, Q, M, a, bb, c, d, tol)) continue;
                n_done++;
                const or_shell *A = &b.sh[a], *B = &b.sh[bb], *C = &b.sh[c], *Dd = &b.sh[d];
                eri_quartet(A, B, C, Dd, tile);
                int nA = A->ncart, nB = B->ncart, nC = C->ncart, nD = Dd->ncart;
                /* the eight orderings (p q | r s) as positions into (a b c d) */
                static const int perm[8][4] = {{0, 1, 2, 3}, {1, 0, 2, 3}, {0, 1, 3, 2}, {1, 0, 3, 2},
                                               {2, 3, 0, 1}, {3, 2, 0, 1}, {2, 3, 1, 0}, {3, 2, 1, 0}};
                int sh[4] = {a, bb, c, d};
                int seen[8][4];
                int nseen = 0;
                for (int P = 0; P < 8; P++) {
                    int t[4] = {sh[perm[P][0]], sh[perm[P][1]], sh[perm[P][2]], sh[perm[P][3]]};
                    int dup = 0;
                    for (int s = 0; s < nseen; s++)
                        if (seen[s][0] == t[0] && seen[s][1] == t[1] && seen[s][2] == t[2] && seen[s][3] == t[3]) dup = 1;
                    if (dup) continue;
                    memcpy(seen[nseen++], t, sizeof(t));
                    const or_shell* S4[4] = {A, B, C, Dd};
                    const or_shell *Sp = S4[perm[P][0]], *Sq = S4[perm[P][1]], *Sr = S4[perm[P][2]], *Ss = S4[perm[P][3]];
                    int idx[4];
                    int nn[4] = {nA, nB, nC, nD};
                    (void)nn;
                    /* loop over all function quartets of the tile; position i of the
                     * permuted quartet is original position perm[P][i] */
                    for (int i0 = 0; i0 < nA; i0++)
                    for (int i1 = 0; i1 < nB; i1++)
                    for (int i2 = 0; i2 < nC; i2++)
                    for (int i3 = 0; i3 < nD; i3++) {
                        double v = tile[((i0 * nB + i1) * nC + i2) * nD + i3];
                        if (v == 0.0) continue;
                        idx[0] = i0; idx[1] = i1; idx[2] = i2; idx[3] = i3;
                        size_t mu = Sp->cart_off + idx[perm[P][0]];
                        size_t nu = Sq->cart_off + idx[perm[P][1]];
                        size_t ka = Sr->cart_off + idx[perm[P][2]];
                        size_t la = Ss->cart_off + idx[perm[P][3]];
                        /* (mu nu | ka la): J_{mu nu} += v D_{ka la}; K_{mu ka} += v D_{nu la} */
                        for (int x = 0; x < nd; x++) {
                            const double* dx = Dc + (size_t)x * n * n;
                            Jt[(size_t)x * n * n + mu * n + nu] += v * dx[ka * n + la];
                            Kt[(size_t)x * n * n + mu * n + ka] += v * dx[nu * n + la];
                        }
                    }
                }
            }
        }
#pragma omp critical
        {
            for (size_t i = 0; i < mat; i++) {
                Jc[i] += Jt[i];
                Kc[i] += Kt[i];
            }
        }
        free(Jt);
        free(Kt);
    }
    from_cart(&b, nd, Jc, J);
    from_cart(&b, nd, Kc, K);
    if (done) *done = n_done;
    if (total) *total = n_total;
    free(pa);
    free(pb);
    free(Dc);
    free(Q);
    free(M);
    free(Jc);
    free(Kc);
    free_basis(&b);
    return 0;
}

/* Selected blocks of J and K: for each requested ordered shell pair (A, B),
 * the user-basis blocks J[x][A][B] and K[x][A][B], summed over every ordered
 * shell pair (C, D) with the screening rule.  Output layout per request r:
 * [nd][nfA][nfB] at offset off[r] (caller sizes buffers with
 * oracle_block_sizes). */
int oracle_jk_blocks(BASIS_ARGS, int nd, const double* D, double tol, int nreq, const int* reqA,
                     const int* reqB, double* Jout, double* Kout) {
    or_basis b;
    if (make_basis(&b, BASIS_PASS)) return -1;
    int ns = b.nshell;
    size_t n = b.ncart, nf = b.nfunc;
    double* Dc = to_cart(&b, nd, D);
    double* Q = schwarz(&b);
    double* M = pair_dmax(&b, nd, Dc);
    size_t off = 0;
    for (int r = 0; r < nreq; r++) {
        int a = reqA[r], bb = reqB[r];
        if (a < 0 || bb < 0 || a >= ns || bb >= ns) { off = (size_t)-1; break; }
        const or_shell *A = &b.sh[a], *B = &b.sh[bb];
        int nA = A->ncart, nB = B->ncart;
        double* Jb = (double*)calloc((size_t)nd * nA * nB, sizeof(double));
        double* Kb = (double*)calloc((size_t)nd * nA * nB, sizeof(double));
#pragma omp parallel num_threads(oracle_get_threads())
        {
            double* Jt = (double*)calloc((size_t)nd * nA * nB, sizeof(double));
            double* Kt = (double*)calloc((size_t)nd * nA * nB, sizeof(double));
            double tile[1296];
#pragma omp for schedule(dynamic) collapse(2)
            for (int c = 0; c < ns; c++)
                for (int d = 0; d < ns; d++) {
                    const or_shell *C = &b.sh[c], *Dd = &b.sh[d];
                    int nC = C->ncart, nD = Dd->ncart;
                    if (keep_quartet(ns, Q, M, a, bb, c, d, tol)) {   /* (AB|CD) D_CD */
                        eri_quartet(A, B, C, Dd, tile);
                        for (int x = 0; x < nd; x++) {
                            const double* dx = Dc + (size_t)x * n * n;
                            for (int i = 0; i < nA; i++)
                                for (int j = 0; j < nB; j++) {
                                    double s = 0;
                                    for (int k = 0; k < nC; k++)
                                        for (int l = 0; l < nD; l++)
                                            s += tile[((i * nB + j) * nC + k) * nD + l] *
                                                 dx[(C->cart_off + k) * n + Dd->cart_off + l];
                                    Jt[((size_t)x * nA + i) * nB + j] += s;
                                }
                        }
                    }
                    if (keep_quartet(ns, Q, M, a, c, bb, d, tol)) {   /* (AC|BD) D_CD */
                        eri_quartet(A, C, B, Dd, tile);
                        for (int x = 0; x < nd; x++) {
                            const double* dx = Dc + (size_t)x * n * n;
                            for (int i = 0; i < nA; i++)
                                for (int j = 0; j < nB; j++) {
                                    double s = 0;
                                    for (int k = 0; k < nC; k++)
                                        for (int l = 0; l < nD; l++)
                                            s += tile[((i * nC + k) * nB + j) * nD + l] *
                                                 dx[(C->cart_off + k) * n + Dd->cart_off + l];
                                    Kt[((size_t)x * nA + i) * nB + j] += s;
                                }
                        }
                    }
                }
#pragma omp critical
            {
                for (size_t i = 0; i < (size_t)nd * nA * nB; i++) {
                    Jb[i] += Jt[i];
                    Kb[i] += Kt[i];
                }
            }
            free(Jt);
            free(Kt);
        }
        /* user basis: T_A^T X T_B */
        int fA = A->nfunc, fB = B->nfunc;
        for (int x = 0; x < nd; x++)
            for (int m = 0; m < fA; m++)
                for (int q = 0; q < fB; q++) {
                    double sj = 0, sk = 0;
                    for (int i = 0; i < nA; i++)
                        for (int j = 0; j < nB; j++) {
                            double t = b.T[(A->cart_off + i) * nf + A->func_off + m] *
                                       b.T[(B->cart_off + j) * nf + B->func_off + q];
                            sj += t * Jb[((size_t)x * nA + i) * nB + j];
                            sk += t * Kb[((size_t)x * nA + i) * nB + j];
                        }
                    Jout[off + ((size_t)x * fA + m) * fB + q] = sj;
                    Kout[off + ((size_t)x * fA + m) * fB + q] = sk;
                }
        off += (size_t)nd * fA * fB;
        free(Jb);
        free(Kb);
    }
    free(Dc);
    free(Q);
    free(M);
    free_basis(&b);
    return off == (size_t)-1 ? -1 : 0;
}
