/*
 * jk.h -- C-ABI of the AO-direct J/K build for AMD MI355X (gfx950).
 *
 * The library computes, for a batch of nd real (generally non-symmetric)
 * densities D^x over a basis of contracted s/p/d Gaussian shells,
 *
 *   J^x_{mn} = sum_{ls} (mn|ls) D^x_{ls},    K^x_{mn} = sum_{ls} (ml|ns) D^x_{ls}
 *
 * (paper Sect. 2.2, Eq. (jkbuild)).  Two-electron integrals are generated on
 * the fly on the GPU and never stored beyond a bounded work buffer; no
 * four-index tensor is allocated.  Builds are bare: no factor 1/2, no spin
 * factor, no 2J-K (Sect. 2, "Notation and conventions").  K uses the whole D:
 * its antisymmetric part is never dropped (Sect. 2.4); J depends only on
 * (D + D^T)/2, which follows from (mn|ls) = (mn|sl).  Pure d functions enter at
 * matrix level, D_cart = T D T^T and J = T^T J_cart T (Sect. 3,
 * screening-robustness paragraph), so the kernels stay Cartesian.
 *
 * Screening (Sect. 2.2, "Cost": O(N^2) once Schwarz screening is applied): a
 * canonical shell quartet (ab|cd) is evaluated iff Q_ab Q_cd >= tol and
 * Q_ab Q_cd * Dmax >= tol, with Q_ab = sqrt(max_{m in a, n in b} (mn|mn)) over
 * Cartesian functions and Dmax the largest |D_cart| over the batch in the six
 * shell-pair blocks ab, cd, ac, ad, bc, bd.
 *
 * Conventions of a basis.  Coefficients multiply primitives normalized on
 * their x^l component; the library rescales each contraction to unit x^l
 * self-overlap.  Function order within a shell: p = (x, y, z); Cartesian d =
 * (xx, xy, xz, yy, yz, zz); pure d = (xy, yz, 3z^2-r^2, xz, x^2-y^2), each
 * of unit self-overlap.  Matrices are row-major, D[x][l][s] = D^x_{ls}.
 *
 * Errors.  Every entry point returns JK_OK or a negative code and never
 * throws; jk_last_error() gives a message for the calling thread.  Kernel
 * faults are asynchronous: they surface at the next synchronizing call on
 * the stream.
 */
#ifndef JK_H
#define JK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define JK_OK 0
#define JK_EINVAL (-1)       /* bad descriptor or argument */
#define JK_ENOMEM (-2)       /* device memory for the request can never fit */
#define JK_EDEVICE (-3)      /* HIP runtime error; message has the detail */
#define JK_EUNSUPPORTED (-4) /* valid request outside what this build supports */

#define JK_MAX_L 2           /* s, p, d */
#define JK_MAX_PRIM 16       /* primitives per shell */

#define JK_FP64 0            /* every quartet in FP64 */
#define JK_MIXED 1           /* quartets with Q_ab Q_cd < fp32_bound in FP32, FP64 accumulation */

typedef struct jk_basis_s* jk_basis_t; /* opaque; owned by the library */

/* Basis descriptor.  All pointers are host memory, read during
 * jk_create_basis only. */
typedef struct {
    int32_t natoms;
    const double* xyz;          /* [natoms*3], bohr */
    int32_t nshells;
    const int32_t* shell_atom;  /* [nshells], 0..natoms-1 */
    const int32_t* shell_l;     /* [nshells], 0..JK_MAX_L */
    const int32_t* shell_nprim; /* [nshells], 1..JK_MAX_PRIM */
    const double* exps;         /* concatenated per shell, > 0 and finite */
    const double* coefs;        /* concatenated per shell, finite */
    int32_t spherical;          /* 1: pure d (5 functions); 0: Cartesian d (6) */
} jk_basis_desc;

/* Build options; jk_default_opts() fills the defaults. */
typedef struct {
    int32_t precision;      /* JK_FP64 (default) or JK_MIXED */
    double schwarz_tol;     /* screening threshold tol, default 1e-12; >= 0 */
    double fp32_bound;      /* JK_MIXED: Q_ab Q_cd below this -> FP32, default 1e-6 */
    int32_t want_j;         /* default 1 */
    int32_t want_k;         /* default 1 */
    int32_t symmetric_hint; /* 0 (default) or 1: the caller promises D == D^T for every density;
                               with more than 8 densities the exchange contractions with D^T
                               (equal to those with D) are then skipped and K = Kc + Kc^T.
                               For a non-symmetric D the K so built is that of (D + D^T)/2's
                               D-half only: do not set it then.  J never depends on it. */
    void* stream;           /* hipStream_t for all work of the call; NULL = default stream */
    void* workspace;        /* optional device buffer of >= jk_workspace_bytes();
                               NULL: the library allocates stream-ordered memory */
    size_t workspace_bytes; /* size of `workspace` */
} jk_build_opts;

void jk_default_opts(jk_build_opts* o);

/* Ingest a basis on the current HIP device: validates the descriptor,
 * normalizes contractions, builds the resident shell-pair data, Schwarz
 * factors and screened quartet lists.  Synchronous.  On success *out owns
 * device memory until jk_destroy.  JK_EINVAL for an invalid descriptor
 * (l > JK_MAX_L, nprim outside 1..JK_MAX_PRIM, exponent <= 0 or non-finite,
 * NULL arrays, shell_atom out of range); JK_EUNSUPPORTED for more than
 * 65535 Cartesian functions. */
int jk_create_basis(const jk_basis_desc* d, jk_basis_t* out);

/* Number of basis functions n of the D/J/K matrices (pure or Cartesian). */
int jk_nbf(jk_basis_t h);

/* J and K for nd densities (Eq. (jkbuild), Sect. 2.2):
 *   J[x][m][n] = sum_{l,s} (mn|ls) D[x][l][s],  K[x][m][n] = sum_{l,s} (ml|ns) D[x][l][s],
 * bare builds (no 1/2, no 2J - K; the notation paragraph of Sect. 2) for
 * generally non-symmetric D, which is used whole for K (Sect. 2.4).  The
 * only approximation is the Schwarz and density screen at o->schwarz_tol
 * (and, for JK_MIXED, the FP32 tier below o->fp32_bound; Sect. 3).  D, J, K
 * are device pointers to row-major [nd][n][n] FP64 arrays (n = jk_nbf); J and
 * K are overwritten.  The caller
 * owns D, J, K and the stream; D must stay valid, and J/K untouched, until
 * the stream has passed the call.  Asynchronous on o->stream.  Either output
 * may be NULL when the matching want_ flag is 0.  Re-entrant: one handle may
 * be used concurrently on several streams, each call with its own workspace.
 * JK_EINVAL for nd < 1, NULL pointers, tol < 0 or an unknown precision;
 * JK_ENOMEM when the workspace cannot be obtained. */
int jk_build(jk_basis_t h, int32_t nd, const double* D, double* J, double* K,
             const jk_build_opts* o);

/* Device bytes one jk_build call with nd densities needs as workspace. */
size_t jk_workspace_bytes(jk_basis_t h, int32_t nd, const jk_build_opts* o);

/* jk_build for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  The
 * same computation and arguments as jk_build (o->workspace and
 * o->workspace_bytes are ignored), but the workspace is a static device
 * buffer of the library of JK_NOALLOC_MAX_BYTES per device, held until the
 * process ends; the call allocates nothing.  Its launch plan must exist:
 * call jk_workspace_bytes(h, nd, o) once beforehand with the same nd and
 * options (that call may allocate).  All calls on one device share the one
 * buffer, so calls that overlap on a device (other streams, other threads)
 * race and must not be issued; the buffer keeps the last call's contents,
 * and each call clears what it accumulates into.  JK_EINVAL as jk_build and
 * when no plan was prepared; JK_ENOMEM when jk_workspace_bytes(h, nd, o)
 * exceeds JK_NOALLOC_MAX_BYTES. */
#define JK_NOALLOC_MAX_BYTES ((size_t)64 << 20)
int jk_build_noalloc(jk_basis_t h, int32_t nd, const double* D, double* J, double* K,
                     const jk_build_opts* o);

/* Builds for several molecules at once (Eq. (jkbuild) per molecule; the
 * paper launches only the realized class buckets, Sect. 3, "DAG-driven,
 * spill-bounded GPU chunking"): nmol handles (same device), density counts
 * nd[i] and device pointers D[i], J[i], K[i] (host arrays of nmol entries;
 * matrices as in jk_build).  For every shell-quartet class and precision
 * tier, an integral launch and the two digestion launches (passes over runs
 * of equal ket shell c and d) each walk a work list of (molecule, tile)
 * items of all molecules, so uneven molecules share the GPU; a class whose
 * tiles exceed the 2 GB work buffer is split into several such launches.
 * There is no single persistent launch over all classes.  Results are those
 * of nmol separate jk_build calls.  Asynchronous on o->stream; workspace from
 * jk_batch_workspace_bytes or stream-ordered allocation. */
int jk_build_batch(int32_t nmol, const jk_basis_t* h, const int32_t* nd, const double* const* D,
                   double* const* J, double* const* K, const jk_build_opts* o);
size_t jk_batch_workspace_bytes(int32_t nmol, const jk_basis_t* h, const int32_t* nd,
                                const jk_build_opts* o);

/* Schedule tunables and autotuning.  Per canonical class (index 0..20) the
 * library keeps four launch parameters, process-wide:
 *   seg_max    length cap of a digestion piece (quartets of one bra pair
 *              digested by one task: a run of equal ket shell, cut at the
 *              cap; classes of at most 18 functions per quartet pack
 *              consecutive runs up to the cap), 4..2^20, default 128;
 *   g_max      densities a digestion task takes at once: 16 (default), or
 *              any of 1, 2, 4, 8 for 8 (also used when a build has at most 8);
 *   dig_kernel 1 (default): a workgroup stages each chunk of tiles once for
 *              waves of different roles; 2: every wave owns a task and all
 *              its roles (classes of at most 408 functions per quartet;
 *              others use 1); 3: as 1 in one pass over runs of equal ket
 *              shell c, the two K blocks indexed by d added per quartet;
 *   eri_block  quartets (threads) per integral workgroup: 64, 128 or 256
 *              (default).
 * The paper launches integral work per realized bucket and notes that the
 * best mapping depends on the bucket (Sect. 3, "DAG-driven, spill-bounded GPU
 * chunking"); jk_autotune picks these per class by timing: with the event
 * profiler it times candidates on the given build (digestion kernel x
 * density group, then piece length, then integral workgroup size, each around
 * the best so far), keeps the fastest per class, applies it process-wide and,
 * if cache_path is not NULL, writes it as JSON keyed by GPU architecture and
 * class; jk_tune_load applies such a file (absent fields keep defaults).
 * Synchronizes o->stream.  Changing the tunables makes later builds
 * regenerate their cached work plans.  JK_EINVAL for values outside the
 * ranges above. */
typedef struct {
    int32_t seg_max;
    int32_t g_max;
    int32_t dig_kernel;
    int32_t eri_block;
} jk_tune_t;
int jk_autotune(jk_basis_t h, int32_t nd, const double* D, double* J, double* K,
                const jk_build_opts* o, const char* cache_path);
int jk_tune_load(const char* path);
int jk_tune_set(int32_t cls, const jk_tune_t* t);
int jk_tune_get(int32_t cls, jk_tune_t* t);

/* HIP graph of one build, for callers that replay the same build shape
 * (serving loops with fixed per-slot buffers).  jk_graph_create captures
 * jk_build(h, nd, D, J, K, o) into an executable graph; the pointers D, J, K
 * and o->workspace (required: nothing is allocated inside the graph) are
 * baked in, so each replay reads the current contents of D and overwrites J
 * and K.  o->stream is ignored; profiling must be off.  jk_graph_launch
 * replays it on `stream` (hipStream_t, NULL = default). */
typedef struct jk_graph_s* jk_graph_t;
int jk_graph_create(jk_basis_t h, int32_t nd, const double* D, double* J, double* K,
                    const jk_build_opts* o, jk_graph_t* out);
int jk_graph_launch(jk_graph_t g, void* stream);
void jk_graph_destroy(jk_graph_t g);

/* Release everything the handle owns.  NULL-safe.  The caller must have
 * synchronized every stream that used the handle. */
void jk_destroy(jk_basis_t h);

/* Message of the last failure on the calling thread ("" if none). */
const char* jk_last_error(void);

/* Canonical shell quartets kept by the Schwarz part of the screen at
 * tolerance tol (the density part is applied per call). */
int64_t jk_quartet_count(jk_basis_t h, double tol);

/* Statistics of the most recent jk_build on this handle (host values):
 * out[0] shell quartets in the Schwarz-screened lists (the density part of
 * the screen may skip more at run time), out[1] of them in FP32, out[2]
 * Cartesian function quartets, out[3] primitive quartets, out[4] algorithmic
 * ERI flops, out[5] algorithmic digestion flops. */
int jk_last_stats(jk_basis_t h, double out[6]);

/* Contracted, normalized Cartesian ERI tiles (ab|cd) for nq shell quartets
 * given as user shell indices shells[4*i .. 4*i+3] (host memory).  out
 * (host) receives the tiles back to back, each [na][nb][nc][nd] in Cartesian
 * component order.  For tests of the integral kernels.  Synchronous. */
int jk_eri_tiles(jk_basis_t h, int32_t nq, const int32_t* shells, double* out);

/* Kernel timing for measurement.  jk_profile_enable(h, 1) makes every later
 * jk_build on h record a HIP event pair around each integral and digestion
 * launch, on the build's stream, and run the build's launches one after
 * another on that stream (unprofiled builds alternate them between the
 * caller's stream and a helper stream), so each kernel's time is its own;
 * jk_profile_read synchronizes those events
 * and returns, per kernel, totals since the last read, then clears them.
 * kind 0 = integral (ERI tile) kernel, 1 = digestion pass C (J, and K
 * over runs of equal ket shell c), 4 = digestion pass D (K over runs of
 * equal d); 2, 3 and 5 the same for the FP32 tier of JK_MIXED builds;
 * cls = canonical class index 0..20.  out[0] total milliseconds, out[1] launches,
 * out[2] algorithmic flops of the quartets the whole screen kept (Schwarz and
 * density parts), out[3] those quartets (counted on the device by the integral
 * kernels), out[4] bytes written (integral tiles) or read (tiles, digestion).
 * Not for concurrent builds. */
int jk_profile_enable(jk_basis_t h, int32_t on);
int jk_profile_read(jk_basis_t h, int32_t kind, int32_t cls, double out[5]);

/* ---- Laplace grids and the forward Laplace cascade (Sect. 2) ----------- */

#define JK_LAPLACE_MAX_POINTS 64

/* Minimax grid of Eq. (laplace): n nodes tau[k] and weights w[k] (host
 * arrays of n) such that max |1/x - sum_k w[k] exp(-x tau[k])| over
 * x in [xmin, xmax] is smallest (the best uniform approximation by an
 * exponential sum; the paper's minimax grid paragraph of Sect. 2).  Found by
 * the Remez exchange on [1, xmax/xmin] and scaled; *max_err (may be NULL)
 * receives that largest error.  Host only, synchronous.  JK_EINVAL for n
 * outside 1..JK_LAPLACE_MAX_POINTS or not 0 < xmin < xmax < inf;
 * JK_EUNSUPPORTED when the exchange does not converge for that many points
 * on that range ratio (fewer points do; the message says which case). */
int jk_laplace_grid(int32_t n, double xmin, double xmax, double* tau, double* w, double* max_err);

/* Omega-shifted weights of Eq. (eomshift): w_out[k] = w[k] exp(omega tau[k]),
 * so that sum_k w_out[k] exp(-D tau[k]) approximates 1/(D - omega) wherever
 * the grid approximates 1/(D - omega) (the grid must cover the shifted range
 * [dmin - omega, dmax - omega]).  JK_EINVAL unless omega < dmin, the
 * smallest denominator (the paper's validity condition). */
int jk_laplace_shift(int32_t n, const double* tau, const double* w, double omega, double dmin, double* w_out);

/* Level-k AO densities of Eqs. (scaledcoeff) and (aodensk): for every
 * residual r < nr and grid point k < ntau,
 *   D[r][k] = U^k R[r] (V^k)^T,  U^k = C_occ diag(exp(+eps_i tau_k)),
 *                                V^k = C_vir diag(exp(-eps_a tau_k)).
 * Device pointers: C [n][nocc + nvir] row-major (AO rows, MO columns, the
 * nocc occupied first), eps [nocc + nvir], R [nr][nocc][nvir],
 * D [nr][ntau][n][n] (overwritten); tau is a host array of ntau
 * (1..JK_LAPLACE_MAX_POINTS).  Asynchronous on stream (a hipStream_t, NULL
 * = default); scratch of ntau n (nocc + nvir) + nr n nvir doubles is taken
 * and released on that stream.  JK_EINVAL for bad sizes or NULL pointers,
 * JK_ENOMEM when the scratch cannot be allocated. */
int jk_laplace_densities(int32_t n, int32_t nocc, int32_t nvir, const double* C, const double* eps, int32_t ntau,
                         const double* tau, int32_t nr, const double* R, double* D, void* stream);

/* Laplace-Fock back-transform of Eq. (laplacefock) for nd densities:
 * F[x] = C^T (2 J[x] - K[x]) C ([nd][nocc + nvir][nocc + nvir]) and/or its
 * occupied-virtual block Rov[x] = F[x][occ][vir] ([nd][nocc][nvir]), the
 * residual that seeds the next level of the cascade (reading of the
 * "occupied-virtual projection" of Eq. (aodensk)).  Device pointers, C as
 * for jk_laplace_densities, J and K [nd][n][n] as jk_build writes them; F or
 * Rov may be NULL (not both).  Asynchronous on stream; scratch of at most
 * 64 n (n + nocc + nvir) doubles.  JK_EINVAL, JK_ENOMEM as above. */
int jk_laplace_fock(int32_t n, int32_t nocc, int32_t nvir, const double* C, int32_t nd, const double* J,
                    const double* K, double* F, double* Rov, void* stream);

/* One forward edge of the level-k cascade (Algorithm ltao, the level-k
 * loop): J and K of the nd level-(k-1) densities D (jk_build, into the
 * caller's J and K), their back-transform's occupied-virtual blocks Rov
 * ([nd][nocc][nvir]) and the level-k densities Dnext ([nd][ntau][n][n]) on
 * the grid tau (host, ntau points), all on o->stream.  n = jk_nbf(h);
 * o->want_j and o->want_k must be set.  Errors as jk_build and the two
 * calls above. */
int jk_laplace_step(jk_basis_t h, int32_t nd, const double* D, double* J, double* K, int32_t nocc, int32_t nvir,
                    const double* C, const double* eps, int32_t ntau, const double* tau, double* Rov, double* Dnext,
                    const jk_build_opts* o);

/* ---------------------------------------------------------------------
 * Cholesky-factor (CD) J/K (Eqs. (cdfact), (cdj), (cdk), (cdknonsym),
 * Sect. 3): the two-electron operator as (mn|ls) ~ sum_Q B_Q[m][n] B_Q[l][s],
 * and J and K read off the factor by dense products.
 * ------------------------------------------------------------------- */

#define JK_CD_MAX_VECTORS 65535

/* The factor of Eq. (cdfact) by pivoted Cholesky.  The operator is the
 * matrix of (mn|ls) over the basis function pairs m >= n (user basis), with
 * the entries of shell quartets whose Schwarz factors give
 * Q_ab Q_cd < screen_tol set to zero: the column-fill screen of the passage
 * on the positive semidefiniteness of the CD operator, which recommends
 * screen_tol = 0.01 delta.  Each step takes as pivot the largest remaining
 * diagonal (among diagonals within a relative 1e-10 of it, the lowest pair
 * index m (m + 1) / 2 + n) and adds one vector; the factor is complete when
 * the largest remaining diagonal is <= delta, so every entry of the
 * operator minus B^T B is at most delta in size.  The operator is held as
 * a pool of (number of significant pairs)^2 doubles during the call and
 * released before it returns.
 *
 * B: device, [max_vectors][n][n] (n = jk_nbf(h)); its first *nvec_out
 * matrices are overwritten with the symmetric B_Q, the rest untouched.
 * pivots: device int32 [max_vectors] or NULL: the pair index of each
 * vector's pivot.  Runs on stream (a hipStream_t, NULL = default) and
 * returns when the factor is complete.  JK_EINVAL for bad arguments
 * (delta <= 0, screen_tol < 0, max_vectors outside 0..JK_CD_MAX_VECTORS);
 * JK_ENOMEM when the pool does not fit in free device memory or more than
 * max_vectors vectors are needed (then *nvec_out = max_vectors and B is
 * not written). */
int jk_cd_factor(jk_basis_t h, double delta, double screen_tol, int32_t max_vectors, double* B, int32_t* pivots,
                 int32_t* nvec_out, void* stream);

/* J and K of nd densities D[x] = U[x] V[x]^T from a factor B (Eq. (cdj) for
 * J; Eq. (cdknonsym) for K, Eq. (cdk) being the case U = V):
 *   J[x] = sum_Q B_Q gamma_Q[x],  gamma_Q[x] = sum_ls B_Q[l][s] D[x][l][s]
 *   K[x] = sum_Q (B_Q U[x]) (B_Q V[x])^T
 * Device pointers: B [nvec][nf][nf] symmetric (as jk_cd_factor writes it),
 * U and V [nd][nf][r] row-major, J and K [nd][nf][nf] (overwritten; either
 * may be NULL, not both).  Asynchronous on stream; scratch is taken and
 * released on it: for J, nd nf^2 + (ceil(nf^2 / 4096) + 1) nvec nd
 * doubles; for K, 2 g nf (nvec + 1) r + ceil(nvec r / 1024) nf^2 doubles,
 * g the densities whose half-transforms B_Q U, B_Q V share 16 GB.  JK_EINVAL for bad sizes or NULL inputs, JK_ENOMEM when the
 * scratch cannot be allocated. */
int jk_cd_jk(int32_t nf, int32_t nvec, const double* B, int32_t nd, int32_t r, const double* U, const double* V,
             double* J, double* K, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* JK_H */
