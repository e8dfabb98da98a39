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

}  // namespace

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

hipError_t unitary_fidelity_strided(int d, int B, const float2* Uf, long long sf, const float2* U, long long su,
                                    double2* overlap, double* fidelity, hipStream_t st) {
    hipLaunchKernelGGL(fidelity_kernel, dim3(B), dim3(256), 0, st, (long long)d * d, Uf, sf, U, su, overlap, fidelity);
    return hipGetLastError();
}

}  // namespace redo
