// Learned warm start (not part of the paper's method): a three-layer
// perceptron, tanh activations, BF16 weights and activations on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation, trained with Adam by the
// kernels below; the same Adam kernel drives REDO-GRAPE amplitude ascent.
#include <algorithm>

#include "redo_internal.h"

namespace redo {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ inline unsigned short to_bf16(float x) {
    unsigned u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float from_bf16(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

// one operand: FP32 or BF16 storage, element (r, k) at p[r * sr + k * sk]
struct Opnd {
    const float* f;
    const unsigned short* h;
    long long sr, sk;
    __device__ inline unsigned short get(int r, int k) const {
        const long long e = (long long)r * sr + (long long)k * sk;
        return f ? to_bf16(f[e]) : h[e];
    }
};

constexpr int MT = 64, KS = 16, LDK = KS + 8;

// C[m][n] = sum_k A(m, k) B(n, k)  (B given by rows n), then epilogue:
//   mode 0: C = acc;  mode 1: C = tanh(acc + bias[n]);  mode 2: C = acc + beta * C (accumulate)
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K, Opnd A, Opnd Bo, float* C, long long ldc,
                                                        const float* bias, int mode) {
    __shared__ __attribute__((aligned(16))) unsigned short As[MT * LDK];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[MT * LDK];
    const int m0 = blockIdx.y * MT, n0 = blockIdx.x * MT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    for (int k0 = 0; k0 < K; k0 += KS) {
        for (int e = threadIdx.x; e < MT * KS; e += 256) {
            const int r = e / KS, k = e % KS;
            const int gm = m0 + r, gn = n0 + r, gk = k0 + k;
            As[r * LDK + k] = (gm < M && gk < K) ? A.get(gm, gk) : (unsigned short)0;
            Bs[r * LDK + k] = (gn < N && gk < K) ? Bo.get(gn, gk) : (unsigned short)0;
        }
        __syncthreads();
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(As + (wm + (lane & 31)) * LDK + 8 * (lane >> 5));
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(Bs + (wn + (lane & 31)) * LDK + 8 * (lane >> 5));
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        const int n = n0 + wn + (lane & 31);
        if (m < M && n < N) {
            float v = acc[r];
            float* c = C + (long long)m * ldc + n;
            if (mode == 1) v = tanhf(v + bias[n]);
            if (mode == 2) v += *c;
            *c = v;
        }
    }
}

// delta = g * (1 - y^2)
__global__ void tanh_back_kernel(long long n, const float* g, const float* y, float* out) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = g[e] * (1.f - y[e] * y[e]);
}

// dy = 2 (y - t) / n, loss partial sums in FP64
__global__ void mse_kernel(long long n, const float* y, const float* t, float* dy, double* loss) {
    __shared__ double red[256];
    double s = 0.0;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const double r = (double)y[e] - (double)t[e];
        s += r * r;
        dy[e] = (float)(2.0 * r / (double)n);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(loss, red[0] / (double)n);
}

// column sums: out[j] = sum_r in[r][j]
__global__ void colsum_kernel(int rows, int cols, const float* in, float* out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += in[(long long)r * cols + j];
    out[j] = (float)s;
}

// Adam on p (descent when sign = 1, ascent when sign = -1), clamped to [lo, hi];
// optional BF16 copy of the updated parameters
__global__ void adam_kernel(long long n, float* p, unsigned short* pb, const float* g, float* m, float* v, float lr,
                            float b1, float b2, float eps, float c1, float c2, float sign, float lo, float hi) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gg = sign * g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    float x = p[e] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    x = fminf(fmaxf(x, lo), hi);
    p[e] = x;
    if (pb) pb[e] = to_bf16(x);
}

// projected gradient ascent: p <- clamp(p + alpha g, lo, hi)
__global__ void ascent_kernel(long long n, float* p, const float* g, float alpha, float lo, float hi) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    p[e] = fminf(fmaxf(fmaf(alpha, g[e], p[e]), lo), hi);
}

// out[r] = mean of row r of in[rows][cols], FP64, one workgroup per row (fixed summation order)
__global__ __launch_bounds__(256) void row_mean_kernel(int cols, const double* in, double* out) {
    const double* x = in + (long long)blockIdx.x * cols;
    double s = 0.0;
    for (int c = threadIdx.x; c < cols; c += 256) s += x[c];
    __shared__ double part[256];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = part[0] / cols;
}

__global__ void to_bf16_kernel(long long n, const float* in, unsigned short* out) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = to_bf16(in[e]);
}

// 2 d^2 features of U with its global phase removed (trace made real, >= 0): [Re | Im]
__global__ void features_kernel(int d, const float2* U, float* out) {
    const int b = blockIdx.x;
    const long long nn = (long long)d * d;
    const float2* u = U + b * nn;
    __shared__ double tr[256], ti[256];
    double sr = 0, si = 0;
    for (int a = threadIdx.x; a < d; a += 256) {
        sr += u[(long long)a * d + a].x;
        si += u[(long long)a * d + a].y;
    }
    tr[threadIdx.x] = sr;
    ti[threadIdx.x] = si;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            tr[threadIdx.x] += tr[threadIdx.x + k];
            ti[threadIdx.x] += ti[threadIdx.x + k];
        }
        __syncthreads();
    }
    const double mag = sqrt(tr[0] * tr[0] + ti[0] * ti[0]);
    double cr = 1.0, ci = 0.0;  // conj(phase)
    if (mag > 1e-12) {
        cr = tr[0] / mag;
        ci = -ti[0] / mag;
    }
    for (long long e = threadIdx.x; e < nn; e += 256) {
        const double xr = u[e].x, xi = u[e].y;
        out[b * 2 * nn + e] = (float)(xr * cr - xi * ci);
        out[b * 2 * nn + nn + e] = (float)(xr * ci + xi * cr);
    }
}

inline unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }

hipError_t gemm(int M, int N, int K, Opnd A, Opnd B, float* C, long long ldc, const float* bias, int mode,
                hipStream_t st) {
    dim3 grid((N + MT - 1) / MT, (M + MT - 1) / MT);
    hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, st, M, N, K, A, B, C, ldc, bias, mode);
    return hipGetLastError();
}

}  // namespace
}  // namespace redo

using namespace redo;

extern "C" {

redo_status redo_mlp_target_features(int32_t d, int32_t B, const float* U, float* features, void* stream) {
    if (d < 1 || B < 1 || !U || !features) return fail(REDO_ERR_ARG, "bad feature arguments");
    hipLaunchKernelGGL(features_kernel, dim3(B), dim3(256), 0, static_cast<hipStream_t>(stream), d,
                       reinterpret_cast<const float2*>(U), features);
    REDO_HIP(hipGetLastError());
    return REDO_OK;
}

redo_status redo_mlp_forward(const redo_mlp* net, int32_t batch, const float* x, float* acts, void* stream) {
    if (!net || batch < 1 || !x || !acts) return fail(REDO_ERR_ARG, "bad forward arguments");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const float* in = x;
    float* out = acts;
    for (int l = 0; l < 3; ++l) {
        const int ni = net->sizes[l], no = net->sizes[l + 1];
        if (ni < 1 || no < 1 || !net->W[l] || !net->b[l]) return fail(REDO_ERR_ARG, "bad layer");
        Opnd A{in, nullptr, ni, 1};
        Opnd Bw{nullptr, net->W[l], ni, 1};   // row n of W^T is row n of W: element (n, k) = W[n][k]
        REDO_HIP(gemm(batch, no, ni, A, Bw, out, no, net->b[l], 1, st));
        in = out;
        out += (size_t)batch * no;
    }
    return REDO_OK;
}

redo_status redo_mlp_loss_grad(const redo_mlp* net, int32_t batch, const float* x, const float* target, float* acts,
                               float* scratch, const redo_mlp_grads* grads, double* loss, void* stream) {
    if (!net || !grads || batch < 1 || !x || !target || !acts || !scratch || !loss)
        return fail(REDO_ERR_ARG, "bad loss/gradient arguments");
    hipStream_t st = static_cast<hipStream_t>(stream);
    redo_status s = redo_mlp_forward(net, batch, x, acts, stream);
    if (s != REDO_OK) return s;
    const int* S = net->sizes;
    const float* act[4] = {x, acts, acts + (size_t)batch * S[1], acts + (size_t)batch * (S[1] + S[2])};
    // scratch: two buffers of batch * max width
    int wmax = 0;
    for (int l = 1; l < 4; ++l) wmax = std::max(wmax, S[l]);
    float* g0 = scratch;
    float* g1 = scratch + (size_t)batch * wmax;
    REDO_HIP(hipMemsetAsync(loss, 0, sizeof(double), st));
    const long long ny = (long long)batch * S[3];
    hipLaunchKernelGGL(mse_kernel, dim3((unsigned)std::min<long long>(nblk(ny), 1024)), dim3(256), 0, st, ny, act[3],
                       target, g0, loss);
    REDO_HIP(hipGetLastError());
    for (int l = 2; l >= 0; --l) {
        const int ni = S[l], no = S[l + 1];
        const long long n = (long long)batch * no;
        // delta = g * (1 - a^2) through the tanh of layer l
        hipLaunchKernelGGL(tanh_back_kernel, dim3(nblk(n)), dim3(256), 0, st, n, g0, act[l + 1], g1);
        REDO_HIP(hipGetLastError());
        // dW[o][i] = sum_b delta[b][o] a_in[b][i]: rows o of delta^T, rows i of a_in^T
        Opnd Dt{g1, nullptr, 1, no};
        Opnd Ait{act[l], nullptr, 1, ni};
        REDO_HIP(gemm(no, ni, batch, Dt, Ait, grads->W[l], ni, nullptr, 0, st));
        hipLaunchKernelGGL(colsum_kernel, dim3((no + 255) / 256), dim3(256), 0, st, batch, no, g1, grads->b[l]);
        REDO_HIP(hipGetLastError());
        if (l > 0) {
            // g_in[b][i] = sum_o delta[b][o] W[o][i]: rows b of delta, rows i of W^T
            Opnd Dl{g1, nullptr, no, 1};
            Opnd Wt{nullptr, net->W[l], 1, ni};
            REDO_HIP(gemm(batch, ni, no, Dl, Wt, g0, ni, nullptr, 0, st));
        }
    }
    return REDO_OK;
}

redo_status redo_adam_update(int64_t n, float* param, uint16_t* param_bf16, const float* grad, float* m, float* v,
                             float lr, float beta1, float beta2, float eps, int32_t step, float sign, float lo, float hi,
                             void* stream) {
    if (n < 1 || !param || !grad || !m || !v || step < 1) return fail(REDO_ERR_ARG, "bad Adam arguments");
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3(nblk(n)), dim3(256), 0, static_cast<hipStream_t>(stream), (long long)n, param,
                       param_bf16, grad, m, v, lr, beta1, beta2, eps, c1, c2, sign, lo, hi);
    REDO_HIP(hipGetLastError());
    return REDO_OK;
}

redo_status redo_ascent_step(int64_t n, float* param, const float* grad, float alpha, float lo, float hi,
                             void* stream) {
    if (n < 1 || !param || !grad || !(lo <= hi)) return fail(REDO_ERR_ARG, "bad ascent-step arguments");
    hipLaunchKernelGGL(ascent_kernel, dim3(nblk(n)), dim3(256), 0, static_cast<hipStream_t>(stream), (long long)n, param,
                       grad, alpha, lo, hi);
    REDO_HIP(hipGetLastError());
    return REDO_OK;
}

redo_status redo_time_average(int32_t rows, int32_t cols, const double* in, double* out, void* stream) {
    if (rows < 1 || cols < 1 || !in || !out) return fail(REDO_ERR_ARG, "bad time-average arguments");
    hipLaunchKernelGGL(row_mean_kernel, dim3(rows), dim3(256), 0, static_cast<hipStream_t>(stream), cols, in, out);
    REDO_HIP(hipGetLastError());
    return REDO_OK;
}

redo_status redo_to_bf16(int64_t n, const float* in, uint16_t* out, void* stream) {
    if (n < 1 || !in || !out) return fail(REDO_ERR_ARG, "bad conversion arguments");
    hipLaunchKernelGGL(to_bf16_kernel, dim3(nblk(n)), dim3(256), 0, static_cast<hipStream_t>(stream), (long long)n, in, out);
    REDO_HIP(hipGetLastError());
    return REDO_OK;
}

}  // extern "C"
