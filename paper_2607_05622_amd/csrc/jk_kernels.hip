// HIP kernels of the AO-direct J/K build for gfx950.
//
// Stages of one build (each a kernel here, launched by jk_host.cpp):
//   sph2cart   D_cart = T D T^T, density-innermost layout [i][j][x]
//   pair_dmax  per shell pair, max |D_cart| over the batch (density screen)
//   eri_tile   one lane per canonical shell quartet of one class: primitive
//              loop -> Boys -> HGP-OS vertical recurrence -> contraction ->
//              horizontal recurrences -> Cartesian tile to a work buffer
//   digest     tiles against stacked densities on the FP64 matrix cores
//              (jk_digest.h), two passes, FP64 atomics into [i][j][x]
//              accumulators
//   cart2sph   J = T^T (Jc + Jc^T) T, K = T^T (Kc + KTc^T) T back to [x][m][n]
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "jk_internal.h"
#include "jk_launch.h"

namespace jk {

// ------------------------------------------------------ basis changes ---

// Dc[i][j][x] = sum_{m,n} T[i][m] D[x][m][n] T[j][n]; zero for nd <= x < ndp.
__global__ void k_sph2cart(const double* __restrict__ D, int nd, int nf, const CartMap* __restrict__ cmap,
                           int nc, int ndp, double* __restrict__ Dc) {
    const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<long long>(nc) * nc) return;
    const int i = static_cast<int>(t / nc), j = static_cast<int>(t - static_cast<long long>(i) * nc);
    const CartMap mi = cmap[i], mj = cmap[j];
    double* __restrict__ o = Dc + t * ndp;
    for (int x = 0; x < ndp; ++x) {
        double s = 0.0;
        if (x < nd) {
            const double* __restrict__ Dx = D + static_cast<long long>(x) * nf * nf;
            for (int u = 0; u < mi.n; ++u)
                for (int v = 0; v < mj.n; ++v)
                    s = fma(mi.c[u] * mj.c[v], Dx[static_cast<long long>(mi.idx[u]) * nf + mj.idx[v]], s);
        }
        o[x] = s;
    }
}

// J[x][m][n] = sum T[i][m] (Jc[i][j][x] + Jc[j][i][x]) T[j][n] and
// K[x][m][n] = sum T[i][m] (Kc[i][j][x] + KTc[j][i][x]) T[j][n], accumulators
// density-innermost with stride ndp.  A matrix is written only when both its
// accumulator and its output are given (a build without J or K has no
// accumulator for it, whatever output pointer the caller passed).
__global__ void k_cart2sph(const double* __restrict__ Jc, const double* __restrict__ Kc,
                           const double* __restrict__ KTc, int nd, int nf, const UserMap* __restrict__ umap,
                           int nc, int ndp, double* __restrict__ J, double* __restrict__ K) {
    const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<long long>(nf) * nf) return;
    const int m = static_cast<int>(t / nf), n = static_cast<int>(t - static_cast<long long>(m) * nf);
    const UserMap um = umap[m], un = umap[n];
    const bool doj = Jc && J, dok = Kc && KTc && K;
    for (int x = 0; x < nd; ++x) {
        double sj = 0.0, sk = 0.0;
        for (int u = 0; u < um.n; ++u)
            for (int v = 0; v < un.n; ++v) {
                const double c = um.c[u] * un.c[v];
                const long long ij = (static_cast<long long>(um.idx[u]) * nc + un.idx[v]) * ndp + x;
                const long long ji = (static_cast<long long>(un.idx[v]) * nc + um.idx[u]) * ndp + x;
                if (doj) sj = fma(c, Jc[ij] + Jc[ji], sj);
                if (dok) sk = fma(c, Kc[ij] + KTc[ji], sk);
            }
        if (doj) J[static_cast<long long>(x) * nf * nf + t] = sj;
        if (dok) K[static_cast<long long>(x) * nf * nf + t] = sk;
    }
}

// The symmetrized densities the Coulomb digestion reads, packed per shell
// pair so that the ket pairs of a bra block, visited in pair order, read
// neighbouring records: one thread per (pair, k, l), all densities.
__global__ void k_pair_ds(const double* __restrict__ Dc, int nc, int ndp, int nd, const PairInfo* __restrict__ pairs,
                          int npair, const int* __restrict__ shell_nf, const int* __restrict__ ds_off, int ns,
                          double* __restrict__ DS) {
    const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int p = static_cast<int>(t / 36), kl = static_cast<int>(t - static_cast<long long>(p) * 36);
    if (p >= npair) return;
    const PairInfo P = pairs[p];
    const int nb = shell_nf[P.sb];
    if (kl >= shell_nf[P.sa] * nb) return;
    const int k = kl / nb, l = kl - (kl / nb) * nb;
    const double* a = Dc + (static_cast<long long>(P.fa + k) * nc + P.fb + l) * ndp;
    const double* b = Dc + (static_cast<long long>(P.fb + l) * nc + P.fa + k) * ndp;
    double* o = DS + (static_cast<long long>(ds_off[P.sa * ns + P.sb]) + kl) * ndp;
    for (int x = 0; x < ndp; ++x) o[x] = x < nd ? a[x] + b[x] : 0.0;
}

// dmax[s][t] = max over the batch and both orientations of |Dc| in block (s, t).
__global__ void k_pair_dmax(const double* __restrict__ Dc, int nc, int ndp, int nd, const int* __restrict__ shell_f0,
                            const int* __restrict__ shell_nf, int ns, double* __restrict__ dmax) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns * ns) return;
    const int s = t / ns, u = t - s * ns;
    double m = 0.0;
    for (int i = 0; i < shell_nf[s]; ++i)
        for (int j = 0; j < shell_nf[u]; ++j) {
            const double* a = Dc + (static_cast<long long>(shell_f0[s] + i) * nc + shell_f0[u] + j) * ndp;
            const double* b = Dc + (static_cast<long long>(shell_f0[u] + j) * nc + shell_f0[s] + i) * ndp;
            for (int x = 0; x < nd; ++x) m = fmax(m, fmax(fabs(a[x]), fabs(b[x])));
        }
    dmax[t] = m;
}

__global__ void k_transpose(const double* __restrict__ D, int nc, int ndp, double* __restrict__ DT) {
    const long long n = static_cast<long long>(nc) * nc * ndp;
    for (long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += static_cast<long long>(gridDim.x) * blockDim.x) {
        const long long ij = e / ndp;
        const int x = static_cast<int>(e - ij * ndp);
        const int i = static_cast<int>(ij / nc), j = static_cast<int>(ij - static_cast<long long>(i) * nc);
        DT[e] = D[(static_cast<long long>(j) * nc + i) * ndp + x];
    }
}

__global__ void k_to_f32(const double* __restrict__ src, float* __restrict__ dst, long long n) {
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<long long>(gridDim.x) * blockDim.x)
        dst[i] = static_cast<float>(src[i]);
}

__global__ void k_zero(double* __restrict__ p, long long n) {
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<long long>(gridDim.x) * blockDim.x)
        p[i] = 0.0;
}

// ------------------------------------------------------------ launchers ---

static inline unsigned blocks_for(long long n, int per) { return static_cast<unsigned>((n + per - 1) / per); }

hipError_t launch_eri_tile(int cls, const EriTileArgs& a, hipStream_t s, int fp32) {
    if (a.nblocks <= 0) return hipSuccess;
    switch (cls) {
#define JK_CASE(n) \
    case n: return launch_eri_tile_c##n(a, s, fp32);
        JK_FOR_CLASS_INDEX(JK_CASE)
#undef JK_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_digest(int cls, const DigestArgs& a, hipStream_t s, int fp32, int pass, int g16, int kernel) {
    if (a.nblocks == 0) return hipSuccess;
    switch (cls) {
#define JK_CASE(n) \
    case n: return launch_digest_c##n(a, s, fp32, pass, g16, kernel);
        JK_FOR_CLASS_INDEX(JK_CASE)
#undef JK_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sph2cart(const double* D, int nd, int nf, const CartMap* cmap, int nc, int ndp, double* Dc,
                           hipStream_t s) {
    const long long n = static_cast<long long>(nc) * nc;
    hipLaunchKernelGGL(k_sph2cart, dim3(blocks_for(n, 256)), dim3(256), 0, s, D, nd, nf, cmap, nc, ndp, Dc);
    return hipGetLastError();
}

hipError_t launch_cart2sph(const double* Jc, const double* Kc, const double* KTc, int nd, int nf,
                           const UserMap* umap, int nc, int ndp, double* J, double* K, hipStream_t s) {
    const long long n = static_cast<long long>(nf) * nf;
    hipLaunchKernelGGL(k_cart2sph, dim3(blocks_for(n, 256)), dim3(256), 0, s, Jc, Kc, KTc, nd, nf, umap, nc, ndp,
                       J, K);
    return hipGetLastError();
}

hipError_t launch_pair_ds(const double* Dc, int nc, int ndp, int nd, const PairInfo* pairs, int npair,
                          const int* shell_nf, const int* ds_off, int ns, double* DS, hipStream_t s) {
    hipLaunchKernelGGL(k_pair_ds, dim3(blocks_for(static_cast<long long>(npair) * 36, 256)), dim3(256), 0, s, Dc, nc,
                       ndp, nd, pairs, npair, shell_nf, ds_off, ns, DS);
    return hipGetLastError();
}

hipError_t launch_pair_dmax(const double* Dc, int nc, int ndp, int nd, const int* shell_f0, const int* shell_nf,
                            int ns, double* dmax, hipStream_t s) {
    hipLaunchKernelGGL(k_pair_dmax, dim3(blocks_for(static_cast<long long>(ns) * ns, 256)), dim3(256), 0, s, Dc,
                       nc, ndp, nd, shell_f0, shell_nf, ns, dmax);
    return hipGetLastError();
}

// ------------------------------------------- static workspace (no-alloc) ---

// The workspace of jk_build_noalloc: a file-scope device array, one copy per
// device, held until the process ends.  Host code never passes its name to a
// kernel (on the host it is only a stand-in symbol); it uses the device
// address hipGetSymbolAddress returns, looked up once per device with that
// device current and kept here.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_init() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_addr[dev]) return hipSuccess;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_addr[dev] = ptr;
    return hipSuccess;
}

void* static_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    return g_scratch_addr[dev];
}

hipError_t launch_transpose(const double* D, int nc, int ndp, double* DT, hipStream_t s) {
    const long long n = static_cast<long long>(nc) * nc * ndp;
    long long g = (n + 255) / 256;
    if (g > 16384) g = 16384;
    hipLaunchKernelGGL(k_transpose, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, D, nc, ndp, DT);
    return hipGetLastError();
}

hipError_t launch_to_f32(const double* src, float* dst, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    long long g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_to_f32, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_zero(double* p, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    long long g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_zero, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace jk
