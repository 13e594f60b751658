// Kernel argument blocks and launchers of the J/K library (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "jk_internal.h"

namespace jk {

// Internal Cartesian function i in terms of user functions: i contributes
// c[u] * (user function idx[u]) to D_cart = T D T^T (at most two entries).
struct CartMap {
    int32_t idx[2];
    double c[2];
    int32_t n, pad;
};

// User function m as a combination of internal Cartesian functions
// (at most three entries, for 3z^2 - r^2).
struct UserMap {
    int32_t idx[3];
    int32_t n;
    double c[3];
};

struct EriTileArgs {
    const int2* quartets;   // this chunk's (bra pair, ket pair) indices
    long long nq;
    const PairInfo* pairs;
    const PrimPair* prims;
    const double* boys;
    const double* dmax;     // [ns][ns] or nullptr (no density screen)
    int ns;
    double tol;
    double* out;            // [NF][nq]
    double* scratch;        // [NE*NCD][nq], classes evaluated in passes
};

struct DigestArgs {
    const int2* quartets;   // this chunk's quartets
    long long nq;           // quartets in the chunk (tile stride)
    const int2* segs;       // this chunk's segments (first quartet in the class list, count)
    long long qbase;        // class-list index of the chunk's first quartet
    int nseg;
    int G;                  // densities per workgroup (power of two)
    int ngroups;            // ceil(nd / G)
    int nd;
    const PairInfo* pairs;
    const double* dmax;
    int ns;
    double tol;
    const double* tiles;    // [NF][nq]
    const double* D;        // [nc][nc][ndp]
    double* J;              // [nc][nc][ndp]
    double* K;              // [nd][nc][nc], row-strip contributions
    double* KT;             // [nd][nc][nc], column-strip contributions, transposed
    int nc, ndp;
    int colA0, colAw, colB0, colBw;   // LDS column windows (ket shells' functions)
    int want_j, want_k;
};

// Allow the digestion kernel of class cls up to lds_bytes of dynamic LDS.
hipError_t digest_prepare(int cls, size_t lds_bytes);

// one launcher pair per canonical class index, defined in jk_class.hip
#define JK_FOR_CLASS_INDEX(X) \
    X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) X(20)
#define JK_DECLARE(n)                                                       \
    hipError_t launch_eri_tile_c##n(const EriTileArgs& a, hipStream_t s); \
    hipError_t launch_digest_c##n(const DigestArgs& a, hipStream_t s);    \
    hipError_t digest_prepare_c##n(size_t lds_bytes);
JK_FOR_CLASS_INDEX(JK_DECLARE)
#undef JK_DECLARE

hipError_t launch_eri_tile(int cls, const EriTileArgs& a, hipStream_t s);
hipError_t launch_digest(int cls, const DigestArgs& a, hipStream_t s);
hipError_t launch_sph2cart(const double* D, int nd, int nf, const CartMap* cmap, int nc, int ndp, double* Dc,
                           hipStream_t s);
hipError_t launch_cart2sph(const double* Jc, const double* Kc, const double* KTc, int nd, int nf,
                           const UserMap* umap, int nc, int ndp, double* J, double* K, hipStream_t s);
hipError_t launch_pair_dmax(const double* Dc, int nc, int ndp, int nd, const int* shell_f0, const int* shell_nf,
                            int ns, double* dmax, hipStream_t s);
hipError_t launch_zero(double* p, long long n, hipStream_t s);

}  // namespace jk
