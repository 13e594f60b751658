// Cholesky-factor (CD) J/K of Eqs. (cdfact)-(cdknonsym): internal view of a
// basis and the launchers of the CD kernels (jk_cd.hip).  Not part of the
// C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "jk.h"
#include "jk_launch.h"

namespace jk {

// What the CD factorization reads of a basis handle (copied host data,
// borrowed device pointers).  Internal shells are the user shells sorted by
// l; user functions are in user shell order.
struct BasisView {
    int device = 0, ns = 0, nf = 0, spherical = 1;
    std::vector<PairInfo> pairs;                 // shell pairs a >= b (internal), with Schwarz factors
    std::vector<int> pairs_of_class[kNumPairClass];
    std::vector<int> uf0, nuf;                   // per internal shell: first user function, user functions
    const PairInfo* d_pairs = nullptr;
    const double* d_prims = nullptr;
    const double* d_boys = nullptr;
    const float* d_boys32 = nullptr;
    const UserMap* d_umap = nullptr;
    int pslots = 0;
};
int basis_view(jk_basis_t h, BasisView* v);

// Shared state of the factorization loop on the device.
struct CdState {
    int done;        // set once the largest remaining diagonal is <= delta
    int nvec;        // vectors made (valid once done)
    double dp;       // remaining diagonal of the current pivot
};

// Scatter of one chunk of integral tiles (layout [NF][n]) of class (la lb |
// lc ld) into the pair operator V [nsig][nsig]: element (mn|ls) in user
// functions (Cartesian tiles contracted with the user maps) goes to
// V[cidx[mn]][cidx[ls]] and its mirror.
struct CdScatterArgs {
    const double* tiles;
    long long n;                 // quartets of the chunk
    const int2* quartets;        // (bra pair, ket pair) per quartet
    const PairInfo* pairs;
    const int* uf0;              // per internal shell
    const UserMap* umap;
    const int* cidx;             // user pair m (m + 1) / 2 + n (m >= n) -> operator row, -1 if absent
    long long nsig;
    double* V;
    int nc[4];                   // Cartesian functions of the four shells of the class
    int nu[4];                   // user functions of the four shells
};
hipError_t launch_cd_scatter(const CdScatterArgs& a, hipStream_t s);
// d[i] = V[i][i]; bmax[b] = the largest of d over block b of 256 (n > 0)
hipError_t launch_cd_diag(const double* V, long long n, double* d, double* bmax, hipStream_t s);
// step k (n > 0): pivot choice (one workgroup, from the block maxima bmax),
// then the new row Bc[k], the diagonal update and its new block maxima;
// both do nothing once st->done is set.  At k = kcap only the pivot choice
// runs, to tell a complete factor (done = 1) from one that needs more than
// kcap vectors (done = 2).
hipError_t launch_cd_step(const double* V, long long n, double* Bc, double* d, double* bmax, int* piv, double delta,
                          int k, int kcap, CdState* st, hipStream_t s);
// B[q][m][n] = B[q][n][m] = Bc[q][i] for (m, n) = (pm[i], pn[i]), q < nvec
// (B zeroed beforehand); pivots_out[q] = the user pair index of piv[q]
hipError_t launch_cd_expand(const double* Bc, long long nsig, int nvec, const int* pm, const int* pn, int nf,
                            double* B, const int* piv, const long long* sig_pair, int* pivots_out,
                            hipStream_t s);
// out[k][xl r + m] = in[x0 + xl][k][m] (in: [nd][nf][r]), xl < xg
hipError_t launch_cd_gather(const double* in, int nf, int r, int x0, int xg, double* out, hipStream_t s);
// out[i] = sum over b < nb of parts[b * stride + i], i < n
hipError_t launch_cd_sum(const double* parts, int nb, long long stride, long long n, double* out, hipStream_t s);

}  // namespace jk
