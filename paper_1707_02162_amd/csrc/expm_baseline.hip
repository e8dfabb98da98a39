// Plain per-step exponential, the comparison point of the method: every step
// propagator U_n = exp[-i dt (H0 + H_n)] (Sec. III, Eq. propUn) evaluated
// directly by scaling and squaring of a Taylor polynomial in Paterson-
// Stockmeyer form, on the same batched MFMA GEMM as the REDO path, so that a
// speed ratio measures the algorithm and not kernel quality.
#include "large_path.h"

namespace redo {
namespace {

struct Norms {
    double s[16];
};

// max over (b, n) of sum_k |amplitude_k| ||S_k||_1 (phased: (|u_x| + |u_y|) ||S_k||_1)
__global__ void amp_bound_kernel(long long count, int K, int phased, const float* __restrict__ u, Norms nrm,
                                 unsigned long long* out) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const int kk = phased ? 2 : 1;
    double w = 0.0;
    for (int k = 0; k < K; ++k) {
        const float* up = u + (e * K + k) * kk;
        const double a = phased ? fabs((double)up[0]) + fabs((double)up[1]) : fabs((double)up[0]);
        w += a * nrm.s[k];
    }
    if (!(w <= 1.7976931348623157e308)) w = 1.7976931348623157e308;
    atomicMax(out, (unsigned long long)__double_as_longlong(w));  // non-negative doubles order as integers
}

// A_b = -i scale (H0 + sum_k H_k(u_bk)) for the pairs of a chunk; pair i reads
// its amplitudes at u + (pair0 + i) * ustride and its drift ((pair0 + i) / drift_div) % n_drift
// split = 1 (signed channels): A_b = -i scale sum_k (sign q eps)_bk S_k, the control term alone
// at the coarse-grained amplitude of Eq. cgrain, for the split step exp(A) V
__global__ __launch_bounds__(256) void build_A_kernel(int d, int K, int phased, int dense, int n_drift, int count,
                                                      long long pair0, int drift_div, const float* __restrict__ u,
                                                      long long ustride, const float2* __restrict__ S,
                                                      const float2* __restrict__ Sy, const double* __restrict__ h,
                                                      const float2* __restrict__ H, double scale, float2* A, int split,
                                                      double eps, double qmax) {
    const long long nn = (long long)d * d;
    const int i = blockIdx.y;
    if (i >= count) return;
    const long long pair = pair0 + i;
    const int drift = (int)((pair / drift_div) % n_drift);
    const float* up = u + pair * ustride;
    const int kk = phased ? 2 : 1;
    float uq[16];
    if (split)
        for (int k = 0; k < K && k < 16; ++k) {
            double phi;
            uq[k] = (float)((double)quantise_one(up + k, 0, eps, qmax, &phi, nullptr) * eps);
        }
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long long)gridDim.x * blockDim.x) {
        const int a = (int)(e / d), c = (int)(e % d);
        float2 hv;
        if (split) {
            hv = make_float2(0.f, 0.f);
        } else if (dense) {
            hv = H[(long long)drift * nn + e];
        } else {
            hv = make_float2(a == c ? (float)h[(long long)drift * d + a] : 0.f, 0.f);
        }
        for (int k = 0; k < K; ++k) {
            const float2 sv = S[(long long)k * nn + e];
            const float ux = split ? uq[k < 16 ? k : 15] : up[k * kk];
            hv.x = fmaf(ux, sv.x, hv.x);
            hv.y = fmaf(ux, sv.y, hv.y);
            if (phased) {
                const float2 yv = Sy[(long long)k * nn + e];
                const float uy = up[k * kk + 1];
                hv.x = fmaf(uy, yv.x, hv.x);
                hv.y = fmaf(uy, yv.y, hv.y);
            }
        }
        // -i scale hv
        A[(long long)i * nn + e] = make_float2((float)(scale * hv.y), (float)(-scale * hv.x));
    }
}

struct Coefs {
    float c[8];
};

// out_i = c_0 I + sum_{j=1}^{r-1} c_j A^j_i, powers at pw + ((j - 1) * count + i) * nn
__global__ void lincomb_kernel(int d, int count, int r, Coefs cf, const float2* __restrict__ pw, float2* out) {
    const long long nn = (long long)d * d;
    const int i = blockIdx.y;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long long)gridDim.x * blockDim.x) {
        float2 v = make_float2((e / d) == (e % d) ? cf.c[0] : 0.f, 0.f);
        for (int j = 1; j < r; ++j) {
            const float2 p = pw[((long long)(j - 1) * count + i) * nn + e];
            v.x = fmaf(cf.c[j], p.x, v.x);
            v.y = fmaf(cf.c[j], p.y, v.y);
        }
        out[(long long)i * nn + e] = v;
    }
}

__global__ void expm_descs_kernel(GemmDesc* descs, int count, const float2* A, long long sA, const float2* B, long long sB,
                                  float2* C, long long sC, const float2* add, long long sAdd) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    GemmDesc g{};
    g.active = 1;
    g.alpha = 1.f;
    g.A = A + i * sA;
    g.B = B + i * sB;
    g.C = C + i * sC;
    g.addend = add ? add + i * sAdd : nullptr;
    descs[i] = g;
}

int grid_x(long long nn, int count) { return (int)std::max<long long>(1, std::min<long long>((nn + 255) / 256, (1LL << 22) / count)); }

}  // namespace

hipError_t expm_amp_bound(int B, int N, int K, int phased, const float* u, const double* snorm, unsigned long long* out,
                          hipStream_t st) {
    Norms n{};
    for (int k = 0; k < K && k < 16; ++k) n.s[k] = snorm[k];
    const long long count = (long long)B * N;
    hipLaunchKernelGGL(amp_bound_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, K, phased, u, n, out);
    return hipGetLastError();
}

hipError_t expm_build_A(const redo_table_s* t, int count, long long pair0, int drift_div, const float* u, long long ustride,
                        double scale, float2* A, hipStream_t st, int split) {
    const int d = t->desc.d;
    hipLaunchKernelGGL(build_A_kernel, dim3(grid_x((long long)d * d, count), count), dim3(256), 0, st, d, t->desc.K,
                       t->desc.phased, t->desc.drift_is_diag ? 0 : 1, t->desc.n_drift, count, pair0, drift_div, u,
                       ustride, t->S32, t->Sy32, t->h64, t->H32, scale, A, split, t->desc.eps, t->qmax);
    return hipGetLastError();
}

hipError_t expm_lincomb(int d, int count, int r, const float* c, const float2* pw, float2* out, hipStream_t st) {
    Coefs cf{};
    for (int j = 0; j < r && j < 8; ++j) cf.c[j] = c[j];
    hipLaunchKernelGGL(lincomb_kernel, dim3(grid_x((long long)d * d, count), count), dim3(256), 0, st, d, count, r, cf, pw, out);
    return hipGetLastError();
}

hipError_t expm_descs(GemmDesc* descs, int count, const float2* A, long long sA, const float2* B, long long sB, float2* C,
                      long long sC, const float2* add, long long sAdd, hipStream_t st) {
    hipLaunchKernelGGL(expm_descs_kernel, dim3((count + 63) / 64), dim3(64), 0, st, descs, count, A, sA, B, sB, C, sC,
                       add, sAdd);
    return hipGetLastError();
}

}  // namespace redo

namespace redo {
namespace {
// chain descriptors from tracked locations: X[loc^1]_b = U_i X[loc]_b for b = b0 + i, inactive skipped
// kscale (nullable): diagonal of the right factor, per drift ([n_drift][d]): X' = U diag(v) X
__global__ void chain_descs_kernel(GemmDesc* descs, int count, int b0, const float2* U, long long sU, float2* X0,
                                   float2* X1, long long xstride, int* loc, const int* n_steps, int step,
                                   const float2* kscale, int d, int n_drift) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int b = b0 + i;
    const bool active = n_steps ? step < n_steps[b] : true;
    float2* X[2] = {X0, X1};
    const int l = loc[b];
    GemmDesc g{};
    g.active = active ? 1 : 0;
    g.alpha = 1.f;
    g.A = U + i * sU;
    g.B = X[l] + (long long)b * xstride;
    g.C = X[l ^ 1] + (long long)b * xstride;
    if (kscale) g.kscale = kscale + (long long)(b % n_drift) * d;
    descs[i] = g;
    if (active) loc[b] = l ^ 1;
}
}  // namespace

hipError_t chain_descs(GemmDesc* descs, int count, int b0, const float2* U, long long sU, float2* X0, float2* X1,
                       long long xstride, int* loc, const int* n_steps, int step, hipStream_t st, const float2* kscale,
                       int d, int n_drift) {
    hipLaunchKernelGGL(chain_descs_kernel, dim3((count + 63) / 64), dim3(64), 0, st, descs, count, b0, U, sU, X0, X1,
                       xstride, loc, n_steps, step, kscale, d, n_drift);
    return hipGetLastError();
}
}  // namespace redo
