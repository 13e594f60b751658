// Dense steps of the Laplace cascade on gfx950 (Sect. 2): the Laplace-
// scaled coefficients of Eq. (scaledcoeff), the level-k AO densities of
// Eq. (aodensk) and the Laplace-Fock back-transform of Eq. (laplacefock).
// All are batched products of dense FP64 matrices, run on the FP64 matrix
// cores, plus two elementwise kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "jk_gemm.h"

namespace jk {

typedef double v4d __attribute__((ext_vector_type(4)));

// C[b] = alpha op(A[b]) op(B[b]) + beta C[b], row-major.  A workgroup of four
// waves computes a 64 x 64 tile of C, each wave a 32 x 32 quarter as 2 x 2
// tiles of v_mfma_f64_16x16x4f64 (lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and holds C[4 r + l / 16][l % 16] in element r), over K
// in chunks of 16 staged in LDS as [k][m] and [k][n].  The next chunk's
// global loads are issued into registers before the current chunk's
// products, so their latency overlaps the matrix-core work.
constexpr int kTile = 64, kChunk = 16, kPer = kTile * kChunk / 256;

struct ChunkRegs {
    double a[kPer], b[kPer];
};

__device__ inline void load_chunk(const GemmArgs& g, const double* __restrict__ A, const double* __restrict__ B,
                                  int m0, int n0, int k0, int K, int tid, ChunkRegs& r) {
    // the element order follows the memory order so loads coalesce
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = tid + 256 * u;
        int mm, kk;
        if (g.ta) {   // op(A)[m][k] = A[k][m]
            kk = e / kTile;
            mm = e - kk * kTile;
        } else {
            mm = e / kChunk;
            kk = e - mm * kChunk;
        }
        const int gm = m0 + mm, gk = k0 + kk;
        r.a[u] = (gm < g.M && gk < K)
                     ? (g.ta ? A[static_cast<long long>(gk) * g.lda + gm] : A[static_cast<long long>(gm) * g.lda + gk])
                     : 0.0;
        int nn;
        if (g.tb) {   // op(B)[k][n] = B[n][k]
            nn = e / kChunk;
            kk = e - nn * kChunk;
        } else {
            kk = e / kTile;
            nn = e - kk * kTile;
        }
        const int gn = n0 + nn, gk2 = k0 + kk;
        r.b[u] = (gn < g.N && gk2 < K)
                     ? (g.tb ? B[static_cast<long long>(gn) * g.ldb + gk2] : B[static_cast<long long>(gk2) * g.ldb + gn])
                     : 0.0;
    }
}

__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    __shared__ double sA[kChunk][kTile + 1];
    __shared__ double sB[kChunk][kTile + 1];
    const long long b = blockIdx.z;
    const double* __restrict__ A = g.A + b * g.sa;
    const double* __restrict__ B = g.B + b * g.sb;
    double* __restrict__ C = g.C + b * g.sc;
    const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int c16 = lane & 15, r4 = lane >> 4;
    v4d acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    const int K = g.klast > 0 && blockIdx.z == gridDim.z - 1 ? g.klast : g.K;
    ChunkRegs r;
    load_chunk(g, A, B, m0, n0, 0, K, tid, r);
    for (int k0 = 0; k0 < K; k0 += kChunk) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + 256 * u;
            if (g.ta) sA[e / kTile][e % kTile] = r.a[u];
            else sA[e % kChunk][e / kChunk] = r.a[u];
            if (g.tb) sB[e % kChunk][e / kChunk] = r.b[u];
            else sB[e / kTile][e % kTile] = r.b[u];
        }
        __syncthreads();
        if (k0 + kChunk < K) load_chunk(g, A, B, m0, n0, k0 + kChunk, K, tid, r);
#pragma unroll
        for (int ks = 0; ks < kChunk; ks += 4) {
            double a[2], bb[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = sA[ks + r4][wm + 16 * i + c16];
#pragma unroll
            for (int j = 0; j < 2; ++j) bb[j] = sB[ks + r4][wn + 16 * j + c16];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int gm = m0 + wm + 16 * i + 4 * rr + r4, gn = n0 + wn + 16 * j + c16;
                if (gm < g.M && gn < g.N) {
                    const long long col = g.gcols > 0 ? (gn / g.gcols) * g.gstride + gn % g.gcols : gn;
                    double* const p = C + static_cast<long long>(gm) * g.ldc + col;
                    *p = g.beta == 0.0 ? g.alpha * acc[i][j][rr] : fma(g.alpha, acc[i][j][rr], g.beta * *p);
                }
            }
}

hipError_t launch_gemm(const GemmArgs& g, int batch, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0 || batch <= 0) return hipSuccess;
    const dim3 grid((g.N + kTile - 1) / kTile, (g.M + kTile - 1) / kTile, batch);
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

// out[k][i][c] = C[i][c0 + c] exp(sign eps[c0 + c] tau[k]) for c < ncols
// (Eq. (scaledcoeff): sign +1 on occupied, -1 on virtual columns).
__global__ void k_scale_cols(const double* __restrict__ Cm, int n, int nmo, int c0, int ncols,
                             const double* __restrict__ eps, ScaleTaus taus, double sign, double* __restrict__ out) {
    const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const long long per = static_cast<long long>(n) * ncols;
    if (t >= per * taus.n) return;
    const int k = static_cast<int>(t / per);
    const long long r = t - k * per;
    const int i = static_cast<int>(r / ncols), c = static_cast<int>(r - static_cast<long long>(i) * ncols);
    out[t] = Cm[static_cast<long long>(i) * nmo + c0 + c] * exp(sign * eps[c0 + c] * taus.t[k]);
}

hipError_t launch_scale_cols(const double* Cm, int n, int nmo, int c0, int ncols, const double* eps,
                             const ScaleTaus& taus, double sign, double* out, hipStream_t s) {
    const long long tot = static_cast<long long>(n) * ncols * taus.n;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_cols, dim3(static_cast<unsigned>((tot + 255) / 256)), dim3(256), 0, s, Cm, n, nmo, c0,
                       ncols, eps, taus, sign, out);
    return hipGetLastError();
}

// out = a x + b y over n elements (the 2J - K of the back-transform)
__global__ void k_axpby(long long n, double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                        double* __restrict__ out) {
    const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < n) out[t] = fma(a, x[t], b * y[t]);
}

hipError_t launch_axpby(long long n, double a, const double* x, double b, const double* y, double* out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpby, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, n, a, x, b, y, out);
    return hipGetLastError();
}

}  // namespace jk
