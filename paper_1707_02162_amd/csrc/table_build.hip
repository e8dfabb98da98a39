// Process 1 of REDO (Sec. II, Eq. redoform): the one-time FP64 build of the
// discrete-operator table and of the drift propagators.  The table is built
// outside every iteration loop (Sec. III), so these kernels favour plain,
// bounds-checked code over speed: an LDS-tiled FP64 complex GEMM, identity
// fills and the single rounding of each FP64 entry to FP32 storage.
#include "redo_internal.h"

namespace redo {
namespace {

constexpr int ZK = 16;   // k-slice

// C[b] = alpha * A[b] B[b] + beta * I for n x n row-major c128 matrices, ZT x ZT
// output tiles (64, or 32 for launches of few tiles).  256 threads, each owns an
// R x R strided sub-block (rows ty + 16 r, cols tx + 16 c), R = ZT / 16; every
// element is one FMA chain over k = 0 .. n - 1 in order, whatever the tile edge.
template <int ZT>
__global__ __launch_bounds__(256) void zgemm_kernel(int n, const double2* __restrict__ A, long long sA,
                                                     const double2* __restrict__ B, long long sB,
                                                     double2* __restrict__ C, long long sC, double2 alpha,
                                                     double beta) {
    constexpr int RR = ZT / 16;
    constexpr int LOADS = ZK * ZT / 256;
    __shared__ double2 As[ZK][ZT + 1];
    __shared__ double2 Bs[ZK][ZT + 1];
    const int bz = blockIdx.z;
    A += sA * bz;
    B += sB * bz;
    C += sC * bz;
    const int i0 = blockIdx.y * ZT, j0 = blockIdx.x * ZT;
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    double2 acc[RR][RR];
#pragma unroll
    for (int r = 0; r < RR; ++r)
#pragma unroll
        for (int c = 0; c < RR; ++c) acc[r][c] = make_double2(0.0, 0.0);
    for (int k0 = 0; k0 < n; k0 += ZK) {
#pragma unroll
        for (int m = 0; m < LOADS; ++m) {
            const int e = tid + 256 * m;
            const int ai = e / ZK, ak = e % ZK;
            const int gi = i0 + ai, gk = k0 + ak;
            As[ak][ai] = (gi < n && gk < n) ? A[(long long)gi * n + gk] : make_double2(0.0, 0.0);
            const int bk = e / ZT, bj = e % ZT;
            const int hk = k0 + bk, hj = j0 + bj;
            Bs[bk][bj] = (hk < n && hj < n) ? B[(long long)hk * n + hj] : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < ZK; ++k) {
            double2 a[RR], b[RR];
#pragma unroll
            for (int r = 0; r < RR; ++r) a[r] = As[k][ty + 16 * r];
#pragma unroll
            for (int c = 0; c < RR; ++c) b[c] = Bs[k][tx + 16 * c];
#pragma unroll
            for (int r = 0; r < RR; ++r)
#pragma unroll
                for (int c = 0; c < RR; ++c) {
                    acc[r][c].x = fma(a[r].x, b[c].x, acc[r][c].x);
                    acc[r][c].x = fma(-a[r].y, b[c].y, acc[r][c].x);
                    acc[r][c].y = fma(a[r].x, b[c].y, acc[r][c].y);
                    acc[r][c].y = fma(a[r].y, b[c].x, acc[r][c].y);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < RR; ++r)
#pragma unroll
        for (int c = 0; c < RR; ++c) {
            const int i = i0 + ty + 16 * r, j = j0 + tx + 16 * c;
            if (i < n && j < n) {
                double2 v = zmul(alpha, acc[r][c]);
                if (i == j) v.x += beta;
                C[(long long)i * n + j] = v;
            }
        }
}

__global__ void fill_identity_kernel(int n, double2* C, long long sC, long long total) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const long long nn = (long long)n * n;
    const long long b = e / nn, r = e % nn;
    const int i = (int)(r / n), j = (int)(r % n);
    C[b * sC + r] = make_double2(i == j ? 1.0 : 0.0, 0.0);
}

// dst + b * dst_batch_stride <- (float) src[b]   (round to nearest even, once)
__global__ void round_entries_kernel(long long nn, int batch, const double2* __restrict__ src,
                                     float2* __restrict__ dst, long long dst_batch_stride) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nn * batch) return;
    const long long b = e / nn, r = e % nn;
    const double2 v = src[e];
    dst[b * dst_batch_stride + r] = make_float2((float)v.x, (float)v.y);
}

__global__ void round_z_kernel(long long count, const double2* __restrict__ src, float2* __restrict__ dst) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) dst[e] = make_float2((float)src[e].x, (float)src[e].y);
}

// V[r][a] = exp(-i dt h[r][a]) evaluated in FP64, rounded once
__global__ void drift_diag_kernel(long long count, const double* __restrict__ h, double dt, float2* __restrict__ V) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const double2 v = expmi(dt * h[e]);
    V[e] = make_float2((float)v.x, (float)v.y);
}

// A <- (A + A^T) / 2: the thread of element (i, j), i < j, writes the same value to both places
__global__ void symmetrize_kernel(int n, double2* __restrict__ A, long long sA) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nn = (long long)n * n;
    if (e >= nn) return;
    const long long i = e / n, j = e % n;
    if (i >= j) return;
    double2* a = A + sA * blockIdx.y;
    const double2 x = a[i * n + j], y = a[j * n + i];
    const double2 v = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y + y.y));
    a[i * n + j] = v;
    a[j * n + i] = v;
}

inline unsigned blocks_for(long long n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t zgemm_batched(int n, int batch, const double2* A, long long sA, const double2* B, long long sB,
                         double2* C, long long sC, double2 alpha, double beta, hipStream_t st) {
    if (batch < 1) return hipSuccess;
    if (batch > 65535) return hipErrorInvalidValue;
    const long long t64 = (long long)((n + 63) / 64) * ((n + 63) / 64) * batch;
    if (t64 >= 1024 || n <= 32) {
        dim3 grid((n + 63) / 64, (n + 63) / 64, batch);
        hipLaunchKernelGGL(zgemm_kernel<64>, grid, dim3(256), 0, st, n, A, sA, B, sB, C, sC, alpha, beta);
    } else {
        // few tiles (single products, small batches): 32 x 32 tiles, four times the workgroups
        dim3 grid((n + 31) / 32, (n + 31) / 32, batch);
        hipLaunchKernelGGL(zgemm_kernel<32>, grid, dim3(256), 0, st, n, A, sA, B, sB, C, sC, alpha, beta);
    }
    return hipGetLastError();
}

hipError_t fill_identity_z(int n, int batch, double2* C, long long sC, hipStream_t st) {
    const long long total = (long long)n * n * batch;
    hipLaunchKernelGGL(fill_identity_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, st, n, C, sC, total);
    return hipGetLastError();
}

hipError_t round_table_entries(int n, int batch, const double2* src, float2* dst, long long dst_batch_stride,
                               hipStream_t st) {
    const long long nn = (long long)n * n;
    hipLaunchKernelGGL(round_entries_kernel, dim3(blocks_for(nn * batch, 256)), dim3(256), 0, st, nn, batch, src,
                       dst, dst_batch_stride);
    return hipGetLastError();
}

hipError_t round_z_to_c(long long count, const double2* src, float2* dst, hipStream_t st) {
    hipLaunchKernelGGL(round_z_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, st, count, src, dst);
    return hipGetLastError();
}

hipError_t drift_diag_phases(int d, int n_drift, const double* h, double dt, float2* V, hipStream_t st) {
    const long long count = (long long)d * n_drift;
    hipLaunchKernelGGL(drift_diag_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, st, count, h, dt, V);
    return hipGetLastError();
}

hipError_t symmetrize_z(int n, int batch, double2* A, long long sA, hipStream_t st) {
    if (n < 2 || batch < 1) return hipSuccess;
    if (batch > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(symmetrize_kernel, dim3(blocks_for((long long)n * n, 256), batch), dim3(256), 0, st, n, A, sA);
    return hipGetLastError();
}

}  // namespace redo
