// Coarse graining of whole amplitude arrays (Sec. II, Eq. cgrain) and the
// FP64 unitary-fidelity reduction (Sec. III: F_U = |Tr(U_f^dag U) / Tr(U_f^dag U_f)|^2).
#include "redo_internal.h"

namespace redo {
namespace {

__global__ void quantise_kernel(long long count, int phased, double eps, double qmax, const float* __restrict__ u,
                                int* __restrict__ codes, double* __restrict__ phi, DeviceFlags* flags) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    double p;
    const int q = quantise_one(u + (phased ? 2 * e : e), phased, eps, qmax, &p, flags);
    codes[e] = q;
    if (phi) phi[e] = p;
}

// one workgroup per instance; FP64 accumulation of Tr(U_f^dag U) and Tr(U_f^dag U_f)
__global__ __launch_bounds__(256) void fidelity_kernel(long long nn, const float2* __restrict__ Uf, long long sf,
                                                       const float2* __restrict__ U, long long su, double2* overlap,
                                                       double* fidelity) {
    __shared__ double sr[256], si[256], sn[256];
    const long long b = blockIdx.x;
    const float2* f = Uf + b * sf;
    const float2* x = U + b * su;
    double ar = 0.0, ai = 0.0, an = 0.0;
    for (long long e = threadIdx.x; e < nn; e += 256) {
        const float2 a = f[e], c = x[e];
        ar += (double)a.x * c.x + (double)a.y * c.y;
        ai += (double)a.x * c.y - (double)a.y * c.x;
        an += (double)a.x * a.x + (double)a.y * a.y;
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    sn[threadIdx.x] = an;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sr[threadIdx.x] += sr[threadIdx.x + s];
            si[threadIdx.x] += si[threadIdx.x + s];
            sn[threadIdx.x] += sn[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double gr = sr[0] / sn[0], gi = si[0] / sn[0];
        if (overlap) overlap[b] = make_double2(gr, gi);
        if (fidelity) fidelity[b] = gr * gr + gi * gi;
    }
}

// the same sums over a slice of one instance (grid: slices x instances); partials [B][S][3]
__global__ __launch_bounds__(256) void fidelity_slice_kernel(long long nn, int S, const float2* __restrict__ Uf,
                                                             long long sf, const float2* __restrict__ U, long long su,
                                                             double* __restrict__ part) {
    __shared__ double sr[256], si[256], sn[256];
    const int s = blockIdx.x;
    const long long b = blockIdx.y;
    const long long len = (nn + S - 1) / S;
    const long long lo = s * len, hi = lo + len < nn ? lo + len : nn;
    const float2* f = Uf + b * sf;
    const float2* x = U + b * su;
    double ar = 0.0, ai = 0.0, an = 0.0;
#pragma unroll 4
    for (long long e = lo + threadIdx.x; e < hi; e += 256) {
        const float2 a = f[e], c = x[e];
        ar += (double)a.x * c.x + (double)a.y * c.y;
        ai += (double)a.x * c.y - (double)a.y * c.x;
        an += (double)a.x * a.x + (double)a.y * a.y;
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    sn[threadIdx.x] = an;
    __syncthreads();
    for (int t = 128; t > 0; t >>= 1) {
        if ((int)threadIdx.x < t) {
            sr[threadIdx.x] += sr[threadIdx.x + t];
            si[threadIdx.x] += si[threadIdx.x + t];
            sn[threadIdx.x] += sn[threadIdx.x + t];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* o = part + (b * S + s) * 3;
        o[0] = sr[0];
        o[1] = si[0];
        o[2] = sn[0];
    }
}

// slices summed in order (deterministic): overlap g = Tr(U_f^dag U)/nu, F = |g|^2, nu = Tr(U_f^dag U_f)
__global__ void fidelity_final_kernel(int B, int S, const double* __restrict__ part, double2* overlap,
                                      double* fidelity, double* nu) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double r = 0.0, i = 0.0, n = 0.0;
    for (int s = 0; s < S; ++s) {
        const double* o = part + ((long long)b * S + s) * 3;
        r += o[0];
        i += o[1];
        n += o[2];
    }
    const double gr = r / n, gi = i / n;
    if (overlap) overlap[b] = make_double2(gr, gi);
    if (fidelity) fidelity[b] = gr * gr + gi * gi;
    if (nu) nu[b] = n;
}

int fidelity_slices(int B) { return B >= 1024 ? 1 : (1024 / B < 64 ? 1024 / B : 64); }

}  // namespace

size_t fidelity_partial_doubles(int B) { return (size_t)3 * B * fidelity_slices(B); }

hipError_t unitary_fidelity_sliced(int d, int B, const float2* Uf, long long sf, const float2* U, long long su,
                                   double2* overlap, double* fidelity, double* nu, double* part, hipStream_t st) {
    const int S = fidelity_slices(B);
    hipLaunchKernelGGL(fidelity_slice_kernel, dim3(S, B), dim3(256), 0, st, (long long)d * d, S, Uf, sf, U, su, part);
    hipLaunchKernelGGL(fidelity_final_kernel, dim3((B + 63) / 64), dim3(64), 0, st, B, S, part, overlap, fidelity, nu);
    return hipGetLastError();
}

hipError_t quantise_all(const redo_table_s* t, const float* u, int B, int N, int* codes, double* phi,
                        hipStream_t st) {
    const long long count = (long long)B * N * t->desc.K;
    const unsigned grid = (unsigned)((count + 255) / 256);
    hipLaunchKernelGGL(quantise_kernel, dim3(grid), dim3(256), 0, st, count, t->desc.phased, t->desc.eps, t->qmax,
                       u, codes, t->desc.phased ? phi : nullptr, t->flags);
    return hipGetLastError();
}

hipError_t unitary_fidelity(int d, int B, const float2* Uf, const float2* U, double2* overlap, double* fidelity,
                            hipStream_t st) {
    const long long nn = (long long)d * d;
    hipLaunchKernelGGL(fidelity_kernel, dim3(B), dim3(256), 0, st, nn, Uf, nn, U, nn, overlap, fidelity);
    return hipGetLastError();
}

}  // namespace redo
