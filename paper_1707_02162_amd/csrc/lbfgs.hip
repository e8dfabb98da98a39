// Batched limited-memory BFGS for GRAPE-type ascent (an optimiser beside the paper's
// gradient steps): every instance b keeps its own history of at most m pairs
// (s = x_{k+1} - x_k, y = g_k - g_{k+1} for the ascent gradient g of its objective) in ring
// buffers, and its direction is d = H g with H the L-BFGS inverse-curvature estimate of -F
// (two-loop recursion, initial scale s.y / y.y of the newest pair).  Vectors are FP32,
// every dot product is accumulated in FP64.  One workgroup per instance for the recursion
// and the history update; the trial point is elementwise.
#include <algorithm>

#include "redo_internal.h"

namespace redo {
namespace {

constexpr int LB_NT = 256;
constexpr int LB_MMAX = 32;

// workgroup sum of one double per thread, returned to every thread
__device__ inline double lb_sum(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();   // red is free (the previous sum was read)
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < LB_NT / 64; ++w) s += red[w];
    return s;
}

// workgroup maximum of one double per thread, returned to every thread
__device__ inline double lb_max(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int w = 1; w < LB_NT / 64; ++w) s = fmax(s, red[w]);
    return s;
}

// slot of the i-th newest pair (i = 0: newest)
__device__ inline int lb_slot(int head, int i, int m) { return ((head - 1 - i) % m + m) % m; }

__global__ __launch_bounds__(LB_NT) void lbfgs_direction_kernel(int B, long long P, int m, const float* __restrict__ g,
                                                                const float* __restrict__ S,
                                                                const float* __restrict__ Y,
                                                                const double* __restrict__ rho,
                                                                const int* __restrict__ count,
                                                                const int* __restrict__ head, double gamma0,
                                                                float* __restrict__ dir, double* __restrict__ gd) {
    __shared__ double red[LB_NT / 64];
    __shared__ double al[LB_MMAX];
    const int b = blockIdx.x, t = threadIdx.x;
    const float* gb = g + (long long)b * P;
    float* q = dir + (long long)b * P;
    const int cnt = min(count[b], m), hd = head[b];
    double gm = 0.0;
    for (long long e = t; e < P; e += LB_NT) {
        q[e] = gb[e];
        gm = fmax(gm, fabs((double)gb[e]));
    }
    gm = lb_max(gm, red);
    // without curvature information: the gradient scaled so that its largest entry moves by gamma0
    const double g0 = gm > 0.0 ? gamma0 / gm : 0.0;
    // newest to oldest: a_i = rho_i s_i.q, q -= a_i y_i
    for (int i = 0; i < cnt; ++i) {
        const int sl = lb_slot(hd, i, m);
        const float* s = S + ((long long)sl * B + b) * P;
        const float* y = Y + ((long long)sl * B + b) * P;
        double acc = 0.0;
        for (long long e = t; e < P; e += LB_NT) acc += (double)s[e] * q[e];
        const double a = rho[(long long)sl * B + b] * lb_sum(acc, red);
        if (t == 0) al[i] = a;
        for (long long e = t; e < P; e += LB_NT) q[e] = (float)((double)q[e] - a * y[e]);
        __syncthreads();
    }
    double gamma = g0;
    if (cnt > 0) {
        const int sl = lb_slot(hd, 0, m);
        const float* y = Y + ((long long)sl * B + b) * P;
        double yy = 0.0;
        for (long long e = t; e < P; e += LB_NT) yy += (double)y[e] * y[e];
        yy = lb_sum(yy, red);
        gamma = yy > 0.0 ? 1.0 / (rho[(long long)sl * B + b] * yy) : g0;   // s.y / y.y
    }
    for (long long e = t; e < P; e += LB_NT) q[e] = (float)(gamma * q[e]);
    __syncthreads();
    // oldest to newest: beta = rho_i y_i.r, r += s_i (a_i - beta)
    for (int i = cnt - 1; i >= 0; --i) {
        const int sl = lb_slot(hd, i, m);
        const float* s = S + ((long long)sl * B + b) * P;
        const float* y = Y + ((long long)sl * B + b) * P;
        double acc = 0.0;
        for (long long e = t; e < P; e += LB_NT) acc += (double)y[e] * q[e];
        const double beta = rho[(long long)sl * B + b] * lb_sum(acc, red);
        const double c = al[i] - beta;
        for (long long e = t; e < P; e += LB_NT) q[e] = (float)((double)q[e] + c * s[e]);
        __syncthreads();
    }
    double acc = 0.0;
    for (long long e = t; e < P; e += LB_NT) acc += (double)gb[e] * q[e];
    double dot = lb_sum(acc, red);
    if (!(dot > 0.0)) {
        // not an ascent direction (or no curvature yet): the scaled gradient
        for (long long e = t; e < P; e += LB_NT) q[e] = (float)(g0 * gb[e]);
        __syncthreads();
        acc = 0.0;
        for (long long e = t; e < P; e += LB_NT) acc += (double)gb[e] * q[e];
        dot = lb_sum(acc, red);
    }
    if (t == 0) gd[b] = dot;
}

__global__ void lbfgs_trial_kernel(long long n, long long P, const float* __restrict__ x, const float* __restrict__ dir,
                                   const double* __restrict__ alpha, float* __restrict__ xt) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    xt[e] = (float)((double)x[e] + alpha[e / P] * dir[e]);
}

// the pair of an accepted step into the ring (curvature y.s > 0 only); a rejected step
// clears the instance's history
__global__ __launch_bounds__(LB_NT) void lbfgs_push_kernel(int B, long long P, int m, const float* __restrict__ x,
                                                           const float* __restrict__ xn, const float* __restrict__ g,
                                                           const float* __restrict__ gn,
                                                           const int* __restrict__ accept, float* __restrict__ S,
                                                           float* __restrict__ Y, double* __restrict__ rho,
                                                           int* __restrict__ count, int* __restrict__ head) {
    __shared__ double red[LB_NT / 64];
    const int b = blockIdx.x, t = threadIdx.x;
    if (!accept[b]) {
        if (t == 0) count[b] = 0;
        return;
    }
    const int sl = head[b] % m;
    float* s = S + ((long long)sl * B + b) * P;
    float* y = Y + ((long long)sl * B + b) * P;
    double ys = 0.0, ss = 0.0, yy = 0.0;
    for (long long e = t; e < P; e += LB_NT) {
        const long long i = (long long)b * P + e;
        const float se = xn[i] - x[i], ye = g[i] - gn[i];
        s[e] = se;
        y[e] = ye;
        ys += (double)ye * se;
        ss += (double)se * se;
        yy += (double)ye * ye;
    }
    ys = lb_sum(ys, red);
    ss = lb_sum(ss, red);
    yy = lb_sum(yy, red);
    if (t == 0 && ys > 1e-12 * sqrt(ss * yy)) {
        rho[(long long)sl * B + b] = 1.0 / ys;
        head[b] = (sl + 1) % m;
        count[b] = min(count[b] + 1, m);
    }
}

inline unsigned lb_blocks(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace
}  // namespace redo

using namespace redo;

extern "C" {

redo_status redo_lbfgs_direction(int32_t B, int64_t P, int32_t m, const float* g, const float* S, const float* Y,
                                 const double* rho, const int32_t* count, const int32_t* head, double gamma0,
                                 float* dir, double* gd, void* stream) {
    if (B < 1 || B > 65535 || P < 1 || m < 1 || m > LB_MMAX || !g || !S || !Y || !rho || !count || !head || !dir ||
        !gd || !(gamma0 > 0.0))
        return fail(REDO_ERR_ARG, "bad L-BFGS direction arguments");
    hipLaunchKernelGGL(lbfgs_direction_kernel, dim3(B), dim3(LB_NT), 0, static_cast<hipStream_t>(stream), B,
                       (long long)P, m, g, S, Y, rho, count, head, gamma0, dir, gd);
    REDO_HIP(hipGetLastError());
    return REDO_OK;
}

redo_status redo_lbfgs_trial(int32_t B, int64_t P, const float* x, const float* dir, const double* alpha, float* xt,
                             void* stream) {
    if (B < 1 || P < 1 || !x || !dir || !alpha || !xt) return fail(REDO_ERR_ARG, "bad L-BFGS trial arguments");
    const long long n = (long long)B * P;
    hipLaunchKernelGGL(lbfgs_trial_kernel, dim3(lb_blocks(n)), dim3(256), 0, static_cast<hipStream_t>(stream), n,
                       (long long)P, x, dir, alpha, xt);
    REDO_HIP(hipGetLastError());
    return REDO_OK;
}

redo_status redo_lbfgs_push(int32_t B, int64_t P, int32_t m, const float* x, const float* xn, const float* g,
                            const float* gn, const int32_t* accept, float* S, float* Y, double* rho, int32_t* count,
                            int32_t* head, void* stream) {
    if (B < 1 || B > 65535 || P < 1 || m < 1 || m > LB_MMAX || !x || !xn || !g || !gn || !accept || !S || !Y ||
        !rho || !count || !head)
        return fail(REDO_ERR_ARG, "bad L-BFGS history arguments");
    hipLaunchKernelGGL(lbfgs_push_kernel, dim3(B), dim3(LB_NT), 0, static_cast<hipStream_t>(stream), B, (long long)P,
                       m, x, xn, g, gn, accept, S, Y, rho, count, head);
    REDO_HIP(hipGetLastError());
    return REDO_OK;
}

}  // extern "C"
