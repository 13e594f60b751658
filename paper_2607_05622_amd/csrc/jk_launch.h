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

// Everything a kernel needs to know about one molecule of a launch.  The
// density-indexed matrices are density-innermost, [nc][nc][ndp], with ndp
// the density count rounded up to the digestion group (zero beyond nd).
struct MolDesc {
    const PairInfo* pairs;
    const double* prims;    // primitive-pair planes (layout at kPrimLane)
    const double* dmax;     // [ns][ns] or nullptr (no density screen)
    const double* D;        // Cartesian densities
    double* J;              // Coulomb accumulator (J = Jc + Jc^T at the end)
    double* K;              // exchange, row contributions K[a][c]
    double* KT;             // exchange, transposed contributions (K += KT^T at the end)
    const double* DS;       // D + D^T per shell pair (c >= d): [unit][ndp], unit = ds_off[c][d] + k ND + l
    const int* ds_off;      // [ns][ns]: first unit of shell pair (c, d), c >= d in internal order
    const float* Df;        // FP32 copies of D and DS (mixed builds; FP32-tier digestion)
    const float* DSf;
    const double* DT;       // transposed densities DT[i][j][x] = D[j][i][x] (the D^T exchange contractions)
    const float* DTf;       // its FP32 copy (mixed builds)
    int ns, nc, nd, ndp;
    int pslots, pad;        // entries per primitive-pair plane
};
// load_mol reads the fields at these offsets
static_assert(__builtin_offsetof(MolDesc, KT) == 48 && __builtin_offsetof(MolDesc, ds_off) == 64 &&
                  __builtin_offsetof(MolDesc, DSf) == 80 && __builtin_offsetof(MolDesc, DTf) == 96 &&
                  __builtin_offsetof(MolDesc, ns) == 104 && __builtin_offsetof(MolDesc, pslots) == 120 &&
                  sizeof(MolDesc) == 128,
              "MolDesc layout");

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
    unsigned long long* kept;  // when not null: += quartets kept by the whole screen (measurement)
    int block;              // threads (quartets) per workgroup: 64, 128 or 256; blocks of the items count these
};

// Digestion work of one bra pair (a "block": the bra pair's quartets of one
// class and tier, consecutive in the class list with ket pairs in (c, d)
// order).  Its tasks, one workgroup each, are its parts times the density
// groups of 8 or 16: task kstart + pc * ngroups + g digests part pc for
// group g.  Pass C walks the block in list order and its parts are runs of
// equal ket shell c; pass D walks the order sorted by (d, c) and its parts
// are runs of equal d (runs longer than a cap are cut; classes with few
// functions per quartet pack consecutive runs up to the cap).  Blocks are dealt to the XCDs: item i of a launch belongs to XCD
// i % 8, whose tasks are numbered from 0 in item order (idle padding items
// have kstart = INT_MAX).
struct DigItem {
    const int2* kin;        // per position of this pass's order: ket shells (c | d << 16) and
                            // their first Cartesian functions (fc | fd << 16)
    const int* pos;         // pass C: (d, c)-order position of each list quartet within its block
    long long blk0;         // class-list index of the block's first quartet
    long long chunk_q0;     // class-list index of the first quartet of the block's tile item
    long long chunk_n;      // tile stride of that item
    long long tile_off;     // element offset of that item's tiles (and of its D-order copy)
    const int* parts;       // start position of each part within the block
    int len, nparts;        // quartets and parts of the block
    int ngroups, kstart;    // density groups; first task on its XCD
    int mol, bra;           // molecule, bra shell pair
};

struct DigestArgs {
    const DigItem* items;
    int nitems;             // a multiple of 8
    MolDesc mol0;
    const MolDesc* mols;
    const void* tiles;      // [NF][n] per tile item, double or float
    void* dcopy;            // D-order copy [n][NF] per tile item, written by pass C
    int want_j, want_k;
    int skip_t;             // D == D^T promised: the D^T contractions (KT) are not digested
    unsigned nblocks;       // 8 x the largest per-XCD task count
};

// one launcher pair per canonical class index, defined in jk_class.hip
#define JK_FOR_CLASS_INDEX(X) \
    X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) X(20)
#define JK_DECLARE(n)                                                                 \
    hipError_t launch_eri_tile_c##n(const EriTileArgs& a, hipStream_t s, int fp32); \
    hipError_t launch_digest_c##n(const DigestArgs& a, hipStream_t s, int fp32, int pass, int g16, int kernel);
JK_FOR_CLASS_INDEX(JK_DECLARE)
#undef JK_DECLARE

// fp32 = 1: the FP32 tier (float recurrences and tiles)
hipError_t launch_eri_tile(int cls, const EriTileArgs& a, hipStream_t s, int fp32 = 0);
// pass 0: C-order digestion (J, K rows/columns of c), pass 1: D-order (K of d);
// g16 = 1: 16 densities per wave task, 0: 8; kernel 1: workgroup-shared
// chunks (jk_digest.h), 2: wave-private tasks (jk_digest2.h) where compiled
// for the class, else 1
hipError_t launch_digest(int cls, const DigestArgs& a, hipStream_t s, int fp32, int pass, int g16, int kernel);
hipError_t launch_sph2cart(const double* D, int nd, int nf, const CartMap* cmap, int nc, int ndp, double* Dc,
                           hipStream_t s);
hipError_t launch_cart2sph(const double* Jc, const double* Kc, const double* KTc, int nd, int nf,
                           const UserMap* umap, int nc, int ndp, double* J, double* K, hipStream_t s);
// DS[ds_off[c][d] + k ND + l][x] = Dc[fc + k][fd + l][x] + Dc[fd + l][fc + k][x] for every shell
// pair c >= d (x < nd; zero up to ndp)
hipError_t launch_pair_ds(const double* Dc, int nc, int ndp, int nd, const PairInfo* pairs, int npair,
                          const int* shell_nf, const int* ds_off, int ns, double* DS, hipStream_t s);
hipError_t launch_pair_dmax(const double* Dc, int nc, int ndp, int nd, const int* shell_f0, const int* shell_nf,
                            int ns, double* dmax, hipStream_t s);
hipError_t launch_zero(double* p, long long n, hipStream_t s);
// DT[i][j][x] = D[j][i][x] for an nc x nc matrix of ndp-vectors
hipError_t launch_transpose(const double* D, int nc, int ndp, double* DT, hipStream_t s);
// dst[i] = (float) src[i], i < n
hipError_t launch_to_f32(const double* src, float* dst, long long n, hipStream_t s);

// Static workspace of jk_build_noalloc (bytes per device).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
// Looks up and keeps the device address of the static workspace on the
// current device (once per device; later calls return at once).
hipError_t static_scratch_init();
// The kept address on device dev, or nullptr before static_scratch_init ran there.
void* static_scratch(int dev);

}  // namespace jk
