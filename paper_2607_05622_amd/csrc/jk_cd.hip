// Kernels of the Cholesky-factor (CD) J/K path (Eqs. (cdfact)-(cdknonsym)):
// the scatter of integral tiles into the pair operator, the steps of the
// pivoted Cholesky factorization over it, the expansion of the factor into
// symmetric matrices and a reduction of split-K partial products.  The dense
// products of the J/K contractions run in the batched FP64 matrix-core GEMM
// (jk_gemm.hip).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "jk_cd.h"

namespace jk {

namespace {

__device__ inline long long tri(long long m, long long n) { return m * (m + 1) / 2 + n; }

// One thread per (quartet, user-function element): the element is the
// Cartesian tile contracted with the user maps of its four functions
// (identity for Cartesian shells, at most three terms per spherical d).  Of
// the elements that land on one operator entry, only one writes it: within a
// shell pair a = b the one with m >= n, within a quartet of equal bra and ket
// pairs the one whose bra pair index is the larger; it also writes the
// mirror entry, so the operator is exactly symmetric.
__global__ __launch_bounds__(256) void k_cd_scatter(CdScatterArgs a) {
    const long long q = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
    if (q >= a.n) return;
    int e = static_cast<int>(blockIdx.y);
    const int i3 = e % a.nu[3];
    e /= a.nu[3];
    const int i2 = e % a.nu[2];
    e /= a.nu[2];
    const int i1 = e % a.nu[1];
    const int i0 = e / a.nu[1];
    const int2 qt = a.quartets[q];
    const PairInfo P = a.pairs[qt.x];
    const PairInfo Q = a.pairs[qt.y];
    if (P.sa == P.sb && i0 < i1) return;
    if (Q.sa == Q.sb && i2 < i3) return;
    const int m = a.uf0[P.sa] + i0, n = a.uf0[P.sb] + i1;
    const int l = a.uf0[Q.sa] + i2, s = a.uf0[Q.sb] + i3;
    const long long pmn = m >= n ? tri(m, n) : tri(n, m);
    const long long pls = l >= s ? tri(l, s) : tri(s, l);
    if (qt.x == qt.y && pmn < pls) return;
    const int cp = a.cidx[pmn], cq = a.cidx[pls];
    if (cp < 0 || cq < 0) return;
    const UserMap u0 = a.umap[m], u1 = a.umap[n], u2 = a.umap[l], u3 = a.umap[s];
    double v = 0.0;
    for (int t0 = 0; t0 < u0.n; ++t0)
        for (int t1 = 0; t1 < u1.n; ++t1)
            for (int t2 = 0; t2 < u2.n; ++t2)
                for (int t3 = 0; t3 < u3.n; ++t3) {
                    const int f = (((u0.idx[t0] - P.fa) * a.nc[1] + (u1.idx[t1] - P.fb)) * a.nc[2] +
                                   (u2.idx[t2] - Q.fa)) * a.nc[3] + (u3.idx[t3] - Q.fb);
                    v = fma(u0.c[t0] * u1.c[t1] * u2.c[t2] * u3.c[t3], a.tiles[static_cast<long long>(f) * a.n + q], v);
                }
    a.V[static_cast<long long>(cp) * a.nsig + cq] = v;
    a.V[static_cast<long long>(cq) * a.nsig + cp] = v;
}

// Largest value over a workgroup of 256 (every thread gets it).
__device__ inline double block_max256(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    v = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    return v;
}

// d[i] = V[i][i], and per block of 256 diagonals their largest (bmax)
__global__ __launch_bounds__(256) void k_cd_diag(const double* __restrict__ V, long long n, double* __restrict__ d,
                                                 double* __restrict__ bmax) {
    __shared__ double red[4];
    const long long i = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
    double v = -__DBL_MAX__;
    if (i < n) {
        v = V[i * n + i];
        d[i] = v;
    }
    v = block_max256(v, red);
    if (threadIdx.x == 0) bmax[blockIdx.x] = v;
}

// Pivot of step k (one workgroup of 1024): the largest remaining diagonal,
// and among the diagonals within a relative 1e-10 of it the one of lowest
// index.  It reads only the per-block maxima of the remaining diagonals
// (bmax, nb blocks of 256) and then one block: the first block whose
// maximum reaches the threshold holds the first diagonal that does.  If the
// largest is <= delta the factor is complete (done = 1, nvec = k); if k has
// reached the caller's capacity the factor does not fit (done = 2).
constexpr double kPivotTie = 1e-10;

__global__ __launch_bounds__(1024) void k_cd_pivot(const double* __restrict__ d, const double* __restrict__ bmax,
                                                   long long n, double delta, int k, int kcap, int* __restrict__ piv,
                                                   CdState* __restrict__ st) {
    if (st->done) return;
    __shared__ double smax[16];
    __shared__ int sidx[16];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nb = static_cast<int>((n + 255) / 256);
    double mx = -__DBL_MAX__;
    for (int b = tid; b < nb; b += 1024) mx = fmax(mx, bmax[b]);
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    if (lane == 0) smax[w] = mx;
    __syncthreads();
    mx = smax[0];
    for (int i = 1; i < 16; ++i) mx = fmax(mx, smax[i]);
    if (!(mx > delta) || k >= kcap) {
        if (tid == 0) {
            st->done = mx > delta ? 2 : 1;
            st->nvec = k;
        }
        return;
    }
    const double thr = (1.0 - kPivotTie) * mx;
    // first block whose maximum reaches thr
    int fb = 0x7fffffff;
    for (int b = tid; b < nb; b += 1024)
        if (bmax[b] >= thr) {
            fb = b;
            break;
        }
    for (int o = 32; o > 0; o >>= 1) fb = min(fb, __shfl_xor(fb, o));
    if (lane == 0) sidx[w] = fb;
    __syncthreads();
    fb = sidx[0];
    for (int i = 1; i < 16; ++i) fb = min(fb, sidx[i]);
    __syncthreads();
    // first diagonal of that block that reaches thr (the first 256 threads)
    int best = 0x7fffffff;
    if (tid < 256) {
        const long long i = static_cast<long long>(fb) * 256 + tid;
        if (i < n && d[i] >= thr) best = tid;
    }
    for (int o = 32; o > 0; o >>= 1) best = min(best, __shfl_xor(best, o));
    if (lane == 0) sidx[w] = best;
    __syncthreads();
    if (tid == 0) {
        for (int i = 1; i < 4; ++i) best = min(best, sidx[i]);
        best = min(best, sidx[0]);
        const int p = fb * 256 + best;
        piv[k] = p;
        st->dp = d[p];
    }
}

// Row k of the factor: Bc[k][i] = (V[p][i] - sum_j<k Bc[j][i] Bc[j][p]) /
// sqrt(d_p) (V is symmetric, so row p is read, coalesced), and the diagonal
// update d[i] -= Bc[k][i]^2 with d[p] = 0.  The earlier rows' pivot entries
// are staged in LDS 256 at a time.
__global__ __launch_bounds__(256) void k_cd_column(const double* __restrict__ V, long long n, double* __restrict__ Bc,
                                                   double* __restrict__ d, double* __restrict__ bmax,
                                                   const int* __restrict__ piv, int k, const CdState* __restrict__ st) {
    if (st->done) return;
    __shared__ double bp[256];
    __shared__ double red[4];
    const int p = piv[k];
    const double dp = st->dp;
    const long long i = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
    const bool in = i < n;
    double s = in ? V[static_cast<long long>(p) * n + i] : 0.0;
    for (int j0 = 0; j0 < k; j0 += 256) {
        const int j = j0 + static_cast<int>(threadIdx.x);
        bp[threadIdx.x] = j < k ? Bc[static_cast<long long>(j) * n + p] : 0.0;
        __syncthreads();
        const int jn = min(256, k - j0);
        if (in) {
            const double* row = Bc + static_cast<long long>(j0) * n + i;
#pragma unroll 8
            for (int jj = 0; jj < jn; ++jj) s = fma(-row[static_cast<long long>(jj) * n], bp[jj], s);
        }
        __syncthreads();
    }
    double dn = -__DBL_MAX__;
    if (in) {
        const double b = s / sqrt(dp);
        Bc[static_cast<long long>(k) * n + i] = b;
        dn = i == p ? 0.0 : d[i] - b * b;
        d[i] = dn;
    }
    dn = block_max256(dn, red);
    if (threadIdx.x == 0) bmax[blockIdx.x] = dn;
}

__global__ void k_cd_expand(const double* __restrict__ Bc, long long nsig, const int* __restrict__ pm,
                            const int* __restrict__ pn, int nf, double* __restrict__ B, const int* __restrict__ piv,
                            const long long* __restrict__ sig_pair, int* __restrict__ pivots_out) {
    const long long t = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
    const long long q = blockIdx.y;
    if (t < nsig) {
        const double v = Bc[q * nsig + t];
        const long long base = q * nf * static_cast<long long>(nf);
        B[base + static_cast<long long>(pm[t]) * nf + pn[t]] = v;
        B[base + static_cast<long long>(pn[t]) * nf + pm[t]] = v;
    }
    if (pivots_out && t == 0) pivots_out[q] = static_cast<int>(sig_pair[piv[q]]);
}

__global__ void k_cd_sum(const double* __restrict__ parts, int nb, long long stride, long long n,
                         double* __restrict__ out) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += parts[b * stride + i];
    out[i] = s;
}

// out[k][xl r + m] = in[x0 + xl][k][m] for xl < xg: the density group's
// factors side by side, as one nf x (xg r) operand
__global__ void k_cd_gather(const double* __restrict__ in, int nf, int r, int x0, int xg, double* __restrict__ out) {
    const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const long long w = static_cast<long long>(xg) * r;
    if (t >= w * nf) return;
    const long long k = t / w, c = t - k * w;
    const long long xl = c / r, m = c - xl * r;
    out[t] = in[((x0 + xl) * nf + k) * r + m];
}

unsigned blocks_of(long long n, int per) { return static_cast<unsigned>((n + per - 1) / per); }

}  // namespace

hipError_t launch_cd_scatter(const CdScatterArgs& a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    const dim3 grid(blocks_of(a.n, 256), a.nu[0] * a.nu[1] * a.nu[2] * a.nu[3]);
    hipLaunchKernelGGL(k_cd_scatter, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cd_diag(const double* V, long long n, double* d, double* bmax, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cd_diag, dim3(blocks_of(n, 256)), dim3(256), 0, s, V, n, d, bmax);
    return hipGetLastError();
}

hipError_t launch_cd_step(const double* V, long long n, double* Bc, double* d, double* bmax, int* piv, double delta,
                          int k, int kcap, CdState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_cd_pivot, dim3(1), dim3(1024), 0, s, d, bmax, n, delta, k, kcap, piv, st);
    if (k >= kcap) return hipGetLastError();
    hipLaunchKernelGGL(k_cd_column, dim3(blocks_of(n, 256)), dim3(256), 0, s, V, n, Bc, d, bmax, piv, k, st);
    return hipGetLastError();
}

hipError_t launch_cd_expand(const double* Bc, long long nsig, int nvec, const int* pm, const int* pn, int nf,
                            double* B, const int* piv, const long long* sig_pair, int* pivots_out, hipStream_t s) {
    if (nvec == 0) return hipSuccess;
    const dim3 grid(blocks_of(nsig > 0 ? nsig : 1, 256), nvec);
    hipLaunchKernelGGL(k_cd_expand, grid, dim3(256), 0, s, Bc, nsig, pm, pn, nf, B, piv, sig_pair, pivots_out);
    return hipGetLastError();
}

hipError_t launch_cd_gather(const double* in, int nf, int r, int x0, int xg, double* out, hipStream_t s) {
    const long long n = static_cast<long long>(nf) * xg * r;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cd_gather, dim3(blocks_of(n, 256)), dim3(256), 0, s, in, nf, r, x0, xg, out);
    return hipGetLastError();
}

hipError_t launch_cd_sum(const double* parts, int nb, long long stride, long long n, double* out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cd_sum, dim3(blocks_of(n, 256)), dim3(256), 0, s, parts, nb, stride, n, out);
    return hipGetLastError();
}

}  // namespace jk
