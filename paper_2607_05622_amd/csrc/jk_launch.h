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

// Everything a kernel needs to know about one molecule of a launch.
struct MolDesc {
    const PairInfo* pairs;
    const PrimPair* prims;
    const double* dmax;     // [ns][ns] or nullptr (no density screen)
    const double* D;        // [nc][nc][nd]
    double* J;              // [nc][nc][nd]
    double* K;              // [nd][nc][nc], row-strip contributions
    double* KT;             // [nd][nc][nc], column-strip contributions, transposed
    int ns, nc, nd, pad;
};

// A contiguous run of one molecule's class list whose tiles occupy
// [tile_off, tile_off + NF * n) of the work buffer, layout [NF][n].
struct EriItem {
    const int2* quartets;   // first quartet of the item
    long long n;            // quartets (tile stride)
    long long tile_off;     // element offset in the work buffer
    long long blk0;         // first block (256 quartets per block) of the item
    int mol, pad;
};

struct EriTileArgs {
    const EriItem* items;
    int nitems;
    long long nblocks;
    MolDesc mol0;           // used when mols == nullptr (one molecule)
    const MolDesc* mols;
    const double* boys;
    const float* boys32;    // the same table in FP32 (FP32 tier)
    double tol;
    void* tiles;            // double (FP64 tier) or float (FP32 tier)
    void* scratch;          // (e0|cd) of pass-evaluated classes, same offsets as tiles
};

// One digestion unit: a run of quartets sharing the bra pair, digested by
// ngroups workgroups of G densities each.
struct DigItem {
    const int2* quartets;   // the molecule's class list
    int2 seg;               // (first quartet in the class list, count)
    long long chunk_q0;     // class-list index of the first quartet of the seg's tile item
    long long chunk_n;      // tile stride of that item
    long long tile_off;     // element offset of that item's tiles
    int mol, G, ngroups, kstart;   // kstart: first block index within this item's XCD
    int colA0, colAw, colB0, colBw;   // LDS column windows (ket shells' functions)
    int dstrip, pad;                  // 1: density strips staged in LDS too
};

struct DigestArgs {
    const DigItem* items;
    int nitems;
    MolDesc mol0;
    const MolDesc* mols;
    double tol;
    const void* tiles;
    int want_j, want_k;
    size_t lds_bytes;       // dynamic LDS of the launch (largest item)
    unsigned nblocks;       // 8 x the largest per-XCD block count
};

// one launcher pair per canonical class index, defined in jk_class.hip
#define JK_FOR_CLASS_INDEX(X) \
    X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) X(20)
#define JK_DECLARE(n)                                                                 \
    hipError_t launch_eri_tile_c##n(const EriTileArgs& a, hipStream_t s, int fp32); \
    hipError_t launch_digest_c##n(const DigestArgs& a, hipStream_t s, int fp32);    \
    hipError_t digest_prepare_c##n(size_t lds_bytes);
JK_FOR_CLASS_INDEX(JK_DECLARE)
#undef JK_DECLARE

// fp32 = 1: the FP32 tier (float recurrences and tiles)
hipError_t launch_eri_tile(int cls, const EriTileArgs& a, hipStream_t s, int fp32 = 0);
hipError_t launch_digest(int cls, const DigestArgs& a, hipStream_t s, int fp32 = 0);
// Allow the digestion kernels of class cls up to lds_bytes of dynamic LDS.
hipError_t digest_prepare(int cls, size_t lds_bytes);
hipError_t launch_sph2cart(const double* D, int nd, int nf, const CartMap* cmap, int nc, int ndp, double* Dc,
                           hipStream_t s);
hipError_t launch_cart2sph(const double* Jc, const double* Kc, const double* KTc, int nd, int nf,
                           const UserMap* umap, int nc, int ndp, double* J, double* K, hipStream_t s);
hipError_t launch_pair_dmax(const double* Dc, int nc, int ndp, int nd, const int* shell_f0, const int* shell_nf,
                            int ns, double* dmax, hipStream_t s);
hipError_t launch_zero(double* p, long long n, hipStream_t s);

}  // namespace jk
