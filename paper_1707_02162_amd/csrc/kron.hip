// Structure-aware chain (a competitor of the dense REDO factors, not the paper's
// method): when d = 2^n and every control generator is a sum of single-spin
// terms, S_k = sum_q s_kq, the factors of one step factorise over the spins,
//     exp(-i theta S_k) = (x)_q exp(-i theta s_kq),
// and the step of Sec. III (Eq. propUn, split form U_n = Z (prod_k R_k) Z^dag V)
// becomes a row scaling, one 2 x 2 unitary per spin, and a row scaling:
//     U_n X = post (.) [ (x)_q g_q ] (pre (.) X),   g_q = prod_k exp(-i theta_k s_kq),
// with pre = Z^dag V and post = Z (Strang: pre = Z^dag V(dt/2), post = V(dt/2) Z).
// theta_k = dt times the REDO-quantised amplitude (Sec. II, Eq. cgrain) or the
// amplitude as given.  Cost per step and instance O(n d^2) instead of O(d^3).
#include "large_path.h"
#include "redo_internal.h"

namespace redo {
namespace {

constexpr int KRON_NT = 512;
constexpr int KRON_VB = 4;                  // row bits held in registers per round
constexpr int KRON_VALS = 1 << KRON_VB;     // values per thread

// per instance and step: the spins' 2 x 2 factors in FP64 (rounded once to FP32) and
// the two diagonal row scalings
struct KronPlanArgs {
    const double2* s;     // [K][n][4] single-spin generators
    const double* h;      // [n_drift][d] diagonal drifts
    const double* g;      // [K][d] phase generators (phased) or null
    const int* codes;     // [B][N][K] (quantised) or null
    const double* phi;    // [B][N][K] (quantised, phased) or null
    const float* u;       // amplitudes (unquantised) or null
    const int* n_steps;
    float2* gates;        // [B][n][4]
    float2* pre;          // [B][d]
    float2* post;         // [B][d]
    double eps, dt;
    int n, d, K, N, n_drift, phased, strang, step;
};

// exp(-i theta s) for a Hermitian 2 x 2 s = a0 I + ax X + ay Y + az Z:
// e^{-i theta a0} (cos(theta r) I - i sin(theta r) (a . sigma) / r), r = |a|
__device__ inline void exp2x2(const double2* s, double theta, double2 (&e)[4]) {
    const double a0 = 0.5 * (s[0].x + s[3].x), az = 0.5 * (s[0].x - s[3].x);
    const double ax = s[1].x, ay = -s[1].y;
    const double r = sqrt(ax * ax + ay * ay + az * az);
    double c, sn;
    sincos(theta * r, &sn, &c);
    const double f = r > 0.0 ? sn / r : theta;   // sin(theta r) / r
    const double2 ph = expmi(theta * a0);
    // M = c I - i f (a . sigma);  a . sigma = [[az, ax - i ay], [ax + i ay, -az]]
    const double2 m00 = make_double2(c, -f * az), m11 = make_double2(c, f * az);
    const double2 m01 = make_double2(-f * ay, -f * ax), m10 = make_double2(f * ay, -f * ax);
    e[0] = zmul(ph, m00);
    e[1] = zmul(ph, m01);
    e[2] = zmul(ph, m10);
    e[3] = zmul(ph, m11);
}

__global__ __launch_bounds__(256) void kron_plan_kernel(KronPlanArgs a) {
    const int b = blockIdx.x;
    if (a.n_steps && a.step >= a.n_steps[b]) return;
    const long long ci = ((long long)b * a.N + a.step) * a.K;
    // channel amplitudes: theta_k = dt Omega_k (signed for unphased channels), phases phi_k
    __shared__ double th[16], ph[16];
    if ((int)threadIdx.x < a.K) {
        const int k = threadIdx.x;
        double om, p = 0.0;
        if (a.codes) {
            om = a.codes[ci + k] * a.eps;   // negative codes carry the sign (unphased)
            if (a.phased) p = a.phi[ci + k];
        } else if (a.phased) {
            const double ux = a.u[(ci + k) * 2], uy = a.u[(ci + k) * 2 + 1];
            om = sqrt(ux * ux + uy * uy);
            p = atan2(uy, ux);
        } else {
            om = a.u[ci + k];
        }
        th[k] = om * a.dt;
        ph[k] = p;
    }
    __syncthreads();
    if ((int)threadIdx.x < a.n) {
        const int q = threadIdx.x;
        double2 acc[4] = {make_double2(1, 0), make_double2(0, 0), make_double2(0, 0), make_double2(1, 0)};
        for (int k = 0; k < a.K; ++k) {
            double2 e[4];
            exp2x2(a.s + ((long long)k * a.n + q) * 4, th[k], e);
            // acc <- e acc (channel 0 acts first)
            const double2 n00 = zadd(zmul(e[0], acc[0]), zmul(e[1], acc[2]));
            const double2 n01 = zadd(zmul(e[0], acc[1]), zmul(e[1], acc[3]));
            const double2 n10 = zadd(zmul(e[2], acc[0]), zmul(e[3], acc[2]));
            const double2 n11 = zadd(zmul(e[2], acc[1]), zmul(e[3], acc[3]));
            acc[0] = n00, acc[1] = n01, acc[2] = n10, acc[3] = n11;
        }
        float2* o = a.gates + ((long long)b * a.n + q) * 4;
        for (int e = 0; e < 4; ++e) o[e] = make_float2((float)acc[e].x, (float)acc[e].y);
    }
    const double* hb = a.h + (long long)(b % a.n_drift) * a.d;
    for (int r = threadIdx.x; r < a.d; r += blockDim.x) {
        double tz = 0.0;   // Z = diag(e^{-i tz})
        if (a.phased)
            for (int k = 0; k < a.K; ++k) tz += ph[k] * a.g[(long long)k * a.d + r];
        const double hd = a.dt * hb[r];
        double2 p, q;
        if (a.strang) {
            p = expmi(0.5 * hd - tz);
            q = expmi(0.5 * hd + tz);
        } else {
            p = expmi(hd - tz);
            q = expmi(tz);
        }
        a.pre[(long long)b * a.d + r] = make_float2((float)p.x, (float)p.y);
        a.post[(long long)b * a.d + r] = make_float2((float)q.x, (float)q.y);
    }
}

__device__ inline long long kron_xcd(long long bid, long long nb) {
    return (nb % 8 == 0) ? (bid % 8) * (nb / 8) + bid / 8 : bid;
}

// LDS row swizzle: the low KRON_VB row bits XOR the next KRON_VB (a bijection), so that
// the rows one instruction touches in any round fall into different banks
__device__ inline int kron_lds(int a, int c, int sw) { return (a ^ ((a >> KRON_VB) & (KRON_VALS - 1))) * sw + c; }

template <int D>
struct KronShape {
    static constexpr int n = D == 128 ? 7 : D == 256 ? 8 : D == 512 ? 9 : D == 1024 ? 10 : D == 2048 ? 11 : 12;
    static constexpr int SW = KRON_NT * KRON_VALS / D;   // columns per workgroup (8192 values in LDS)
    static constexpr int rounds = (n + KRON_VB - 1) / KRON_VB;
    static_assert(rounds >= 2 && rounds <= 3, "two or three register rounds");
};

// row of register value i and thread part `rest` in a round whose register bits start at lo
__device__ inline int kron_row(int rest, int i, int lo) {
    return (rest & ((1 << lo) - 1)) | (i << lo) | ((rest >> lo) << (lo + KRON_VB));
}

template <int J>
__device__ inline void kron_gate_bit(float2 (&v)[KRON_VALS], const float2* gq) {
    const float2 g00 = gq[0], g01 = gq[1], g10 = gq[2], g11 = gq[3];
#pragma unroll
    for (int i = 0; i < KRON_VALS; ++i) {
        if (i & (1 << J)) continue;
        const int i1 = i | (1 << J);
        const float2 x = v[i], y = v[i1];
        float2 r0 = make_float2(0.f, 0.f), r1 = make_float2(0.f, 0.f);
        cfma(r0, g00, x);
        cfma(r0, g01, y);
        cfma(r1, g10, x);
        cfma(r1, g11, y);
        v[i] = r0;
        v[i1] = r1;
    }
}

// register bits of round R start at row bit lo(R); round R applies spins VB R .. VB R + VB - 1
template <int D, int R>
struct KronRound {
    static constexpr int n = KronShape<D>::n, VB = KRON_VB;
    static constexpr int lo = VB * R < n - VB ? VB * R : n - VB;
    static constexpr int q0 = VB * R, q1 = VB * R + VB < n ? VB * R + VB : n;
};

template <int D, int R, int Q>
__device__ inline void kron_round_gate(float2 (&v)[KRON_VALS], const float2* gl) {
    using RR = KronRound<D, R>;
    if constexpr (RR::q0 + Q < RR::q1) kron_gate_bit<RR::q0 + Q - RR::lo>(v, gl + (RR::q0 + Q) * 4);
}

template <int D, int R>
__device__ inline void kron_round_gates(float2 (&v)[KRON_VALS], const float2* gl) {
    static_assert(KRON_VB == 4, "one call per register bit");
    kron_round_gate<D, R, 0>(v, gl);
    kron_round_gate<D, R, 1>(v, gl);
    kron_round_gate<D, R, 2>(v, gl);
    kron_round_gate<D, R, 3>(v, gl);
}

// hand the strip from the register layout of round R - 1 to that of round R through LDS
template <int D, int R>
__device__ inline void kron_exchange(float2 (&v)[KRON_VALS], float2* buf, int rest, int c) {
    constexpr int SW = KronShape<D>::SW;
#pragma unroll
    for (int i = 0; i < KRON_VALS; ++i) buf[kron_lds(kron_row(rest, i, KronRound<D, R - 1>::lo), c, SW)] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < KRON_VALS; ++i) v[i] = buf[kron_lds(kron_row(rest, i, KronRound<D, R>::lo), c, SW)];
    __syncthreads();
}

// One step for every instance: workgroup = (instance, strip of SW columns).  Pass 0
// reads the strip from HBM with register bits = row bits 0..VB-1, applies the pre
// scaling and spins 0..VB-1, and parks the strip in LDS; pass r takes row bits
// lo_r .. lo_r + VB - 1 (lo_r = min(VB r, n - VB)) and applies spins VB r .. VB r + VB - 1;
// the last pass applies the post scaling and writes the strip back in place.
// 64 KiB of LDS per workgroup: two workgroups (four waves per SIMD) per CU.
template <int D>
__global__ __launch_bounds__(KRON_NT, 4) void kron_step_kernel(float2* X0, float2* X1, const int* loc,
                                                               long long xstride, const float2* __restrict__ gates,
                                                               const float2* __restrict__ pre,
                                                               const float2* __restrict__ post, const int* n_steps,
                                                               int step) {
    using S = KronShape<D>;
    constexpr int n = S::n, SW = S::SW, NSTRIP = D / SW;
    __shared__ float2 buf[KRON_NT * KRON_VALS];
    __shared__ float2 gl[n * 4];
    const long long bid = kron_xcd(blockIdx.x, gridDim.x);
    const int b = (int)(bid / NSTRIP), strip = (int)(bid % NSTRIP);
    if (n_steps && step >= n_steps[b]) return;   // uniform over the workgroup
    float2* X = ((loc && loc[b]) ? X1 : X0) + (long long)b * xstride + strip * SW;
    const int t = threadIdx.x, c = t % SW, rest = t / SW;
    if (t < n * 4) gl[t] = gates[(long long)b * n * 4 + t];
    const float2* pb = pre + (long long)b * D;
    const float2* qb = post + (long long)b * D;
    float2 v[KRON_VALS];
#pragma unroll
    for (int i = 0; i < KRON_VALS; ++i) {
        const int a = kron_row(rest, i, 0);
        v[i] = cmul(pb[a], X[(long long)a * D + c]);
    }
    __syncthreads();   // gates in LDS
    kron_round_gates<D, 0>(v, gl);
    kron_exchange<D, 1>(v, buf, rest, c);
    kron_round_gates<D, 1>(v, gl);
    if constexpr (S::rounds > 2) {
        kron_exchange<D, 2>(v, buf, rest, c);
        kron_round_gates<D, 2>(v, gl);
    }
    constexpr int flo = KronRound<D, S::rounds - 1>::lo;
#pragma unroll
    for (int i = 0; i < KRON_VALS; ++i) {
        const int a = kron_row(rest, i, flo);
        X[(long long)a * D + c] = cmul(qb[a], v[i]);
    }
}

// kron_step_kernel<1024> followed, in the same workgroup, by the observable in the right
// Walsh frame on the strip it has just written, while the strip is still in registers: the
// strip goes to the exchange buffer in the layout of the one-pass observable (16-byte
// chunks swizzled by row, mx8_off), each pair of lanes forms (M W)_aj for a row and four
// columns from the packed lists and adds D_j Re(conj(W_aj) (M W)_aj) (FP32 within a row,
// FP64 across rows); the workgroup's sum goes to partial[b][strip].  The observable's own
// read of every state disappears.
template <int WP>
__global__ __launch_bounds__(KRON_NT, 4) void kron_step_obs_kernel(float2* X0, float2* X1, const int* loc,
                                                                   long long xstride,
                                                                   const float2* __restrict__ gates,
                                                                   const float2* __restrict__ pre,
                                                                   const float2* __restrict__ post,
                                                                   const int* n_steps, int step,
                                                                   const int* __restrict__ cols,
                                                                   const float2* __restrict__ vals,
                                                                   const double* __restrict__ spec,
                                                                   double* __restrict__ partial) {
    constexpr int D = 1024;
    using S = KronShape<D>;
    constexpr int n = S::n, SW = S::SW, NSTRIP = D / SW;
    static_assert(SW == 8 && S::rounds > 2, "8-column strips, the buffer free after the last exchange");
    __shared__ float2 buf[KRON_NT * KRON_VALS];
    __shared__ float2 gl[n * 4];
    __shared__ double red[KRON_NT / 64];
    const long long bid = kron_xcd(blockIdx.x, gridDim.x);
    const int b = (int)(bid / NSTRIP), strip = (int)(bid % NSTRIP);
    if (n_steps && step >= n_steps[b]) return;   // uniform over the workgroup
    float2* X = ((loc && loc[b]) ? X1 : X0) + (long long)b * xstride + strip * SW;
    const int t = threadIdx.x, c = t % SW, rest = t / SW;
    if (t < n * 4) gl[t] = gates[(long long)b * n * 4 + t];
    const float2* pb = pre + (long long)b * D;
    const float2* qb = post + (long long)b * D;
    float2 v[KRON_VALS];
#pragma unroll
    for (int i = 0; i < KRON_VALS; ++i) {
        const int a = kron_row(rest, i, 0);
        v[i] = cmul(pb[a], X[(long long)a * D + c]);
    }
    __syncthreads();   // gates in LDS
    kron_round_gates<D, 0>(v, gl);
    kron_exchange<D, 1>(v, buf, rest, c);
    kron_round_gates<D, 1>(v, gl);
    kron_exchange<D, 2>(v, buf, rest, c);
    kron_round_gates<D, 2>(v, gl);
    constexpr int flo = KronRound<D, S::rounds - 1>::lo;
    // the last exchange ended with a barrier after its reads: the buffer is free
#pragma unroll
    for (int i = 0; i < KRON_VALS; ++i) {
        const int a = kron_row(rest, i, flo);
        const float2 y = cmul(qb[a], v[i]);
        X[(long long)a * D + c] = y;
        buf[mx8_off(a, c)] = y;
    }
    __syncthreads();
    asm volatile("" ::: "memory");   // the observable's mask loads stay below the step (register pressure)
    constexpr int LPR = 2, CPL = SW / LPR, NCH = CPL / 2, RPP = KRON_NT / LPR;
    const float4* strip4 = reinterpret_cast<const float4*>(buf);
    const int lr = t % LPR;
    float dj[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) dj[u] = (float)spec[strip * SW + lr * CPL + u];
    // M_ac = f(a XOR c) (the frame needs it): row a's list is row 0's with every column XORed
    // by a, so the masks and values are read once (one address for every lane), zeros skipped
    int mk[WP];
    float2 fv[WP];
    obs_list<WP>(cols, vals, 0, mk, fv);
    double sum = 0.0;
    for (int a = t / LPR; a < D; a += RPP) {
        float2 acc[CPL];
#pragma unroll
        for (int u = 0; u < CPL; ++u) acc[u] = make_float2(0.f, 0.f);
#pragma unroll
        for (int e = 0; e < WP; ++e) {
            if (fv[e].x == 0.f && fv[e].y == 0.f) continue;   // the same for every lane
            const int c = a ^ mk[e];
#pragma unroll
            for (int j = 0; j < NCH; ++j) {
                const int ch = lr * NCH + j;
                const float4 x = strip4[c * 4 + ((ch ^ (c >> 2)) & 3)];
                cfma(acc[2 * j], fv[e], make_float2(x.x, x.y));
                cfma(acc[2 * j + 1], fv[e], make_float2(x.z, x.w));
            }
            asm volatile("" ::: "memory");   // one mask's gathers at a time (register pressure)
        }
        float row = 0.f;
#pragma unroll
        for (int j = 0; j < NCH; ++j) {
            const int ch = lr * NCH + j;
            const float4 wv = strip4[a * 4 + ((ch ^ (a >> 2)) & 3)];
            row += dj[2 * j] * (wv.x * acc[2 * j].x + wv.y * acc[2 * j].y) +
                   dj[2 * j + 1] * (wv.z * acc[2 * j + 1].x + wv.w * acc[2 * j + 1].y);
        }
        sum += (double)row;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
    if ((t & 63) == 0) red[t >> 6] = sum;
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < KRON_NT / 64; ++w) s += red[w];
        partial[(long long)b * NSTRIP + strip] = s;
    }
}

template <int WP>
hipError_t launch_kron_step_obs(int B, float2* X0, float2* X1, const int* loc, long long xstride, const float2* gates,
                                const float2* pre, const float2* post, const int* n_steps, int step, const int* pc,
                                const float2* pv, const double* spec, double* partial, hipStream_t st) {
    constexpr int NSTRIP = 1024 / KronShape<1024>::SW;
    void* tok = nullptr;
    const bool prof = profiling_on();
    if (prof) profile_begin(st, &tok, 1);
    hipLaunchKernelGGL(kron_step_obs_kernel<WP>, dim3((unsigned)((long long)B * NSTRIP)), dim3(KRON_NT), 0, st, X0, X1,
                       loc, xstride, gates, pre, post, n_steps, step, pc, pv, spec, partial);
    if (prof) profile_end(st, tok);
    return hipGetLastError();
}

// the step and the Walsh-frame observable in one launch (d = 1024), then the per-instance sums
hipError_t kron_step_observable(int B, float2* X0, float2* X1, const int* loc, long long xstride,
                                const float2* gates, const float2* pre, const float2* post, const int* n_steps,
                                int step, int w, const int* pc, const float2* pv, const float2* vals,
                                const double* spec, double* partial, double* out, long long out_stride,
                                hipStream_t st) {
    hipError_t e;
    switch ((w + 3) / 4 * 4) {
        case 4: e = launch_kron_step_obs<4>(B, X0, X1, loc, xstride, gates, pre, post, n_steps, step, pc, pv, spec, partial, st); break;
        case 8: e = launch_kron_step_obs<8>(B, X0, X1, loc, xstride, gates, pre, post, n_steps, step, pc, pv, spec, partial, st); break;
        case 12: e = launch_kron_step_obs<12>(B, X0, X1, loc, xstride, gates, pre, post, n_steps, step, pc, pv, spec, partial, st); break;
        default: e = launch_kron_step_obs<16>(B, X0, X1, loc, xstride, gates, pre, post, n_steps, step, pc, pv, spec, partial, st);
    }
    if (e != hipSuccess) return e;
    return observable_final(1024 / KronShape<1024>::SW, B, partial, vals, 1024 * w, n_steps, step, out, out_stride, st);
}

template <int D>
hipError_t launch_kron_step(int B, float2* X0, float2* X1, const int* loc, long long xstride, const float2* gates,
                            const float2* pre, const float2* post, const int* n_steps, int step, hipStream_t st) {
    constexpr int NSTRIP = D / KronShape<D>::SW;
    void* tok = nullptr;
    const bool prof = profiling_on();
    if (prof) profile_begin(st, &tok, 1);
    hipLaunchKernelGGL(kron_step_kernel<D>, dim3((unsigned)((long long)B * NSTRIP)), dim3(KRON_NT), 0, st, X0, X1, loc,
                       xstride, gates, pre, post, n_steps, step);
    if (prof) profile_end(st, tok);
    return hipGetLastError();
}

hipError_t kron_step(int d, int B, float2* X0, float2* X1, const int* loc, long long xstride, const float2* gates,
                     const float2* pre, const float2* post, const int* n_steps, int step, hipStream_t st) {
    switch (d) {
        case 128: return launch_kron_step<128>(B, X0, X1, loc, xstride, gates, pre, post, n_steps, step, st);
        case 256: return launch_kron_step<256>(B, X0, X1, loc, xstride, gates, pre, post, n_steps, step, st);
        case 512: return launch_kron_step<512>(B, X0, X1, loc, xstride, gates, pre, post, n_steps, step, st);
        case 1024: return launch_kron_step<1024>(B, X0, X1, loc, xstride, gates, pre, post, n_steps, step, st);
        case 2048: return launch_kron_step<2048>(B, X0, X1, loc, xstride, gates, pre, post, n_steps, step, st);
        case 4096: return launch_kron_step<4096>(B, X0, X1, loc, xstride, gates, pre, post, n_steps, step, st);
        default: return hipErrorInvalidValue;
    }
}

struct KronWS {
    int* codes;
    double* phi;
    float2* W1;
    float2* gates;
    float2 *pre, *post;
    GemmDesc* descs;
    float2* E;   // re-projection scratch: E = (I - X^dag X) / 2 of a chunk
    double* obs_partial;
    int* loc;
    float2* obsT;
    size_t bytes;
    KronWS(const redo_table_s* t, int B, int N, void* base) {
        const int d = t->desc.d, K = t->desc.K;
        const size_t mat = (size_t)d * d;
        Carve c(base);
        codes = c.take<int>((size_t)B * N * K);
        phi = c.take<double>((size_t)B * N * K);
        W1 = c.take<float2>(mat * B);
        gates = c.take<float2>((size_t)B * 16 * 4);
        pre = c.take<float2>((size_t)B * d);
        post = c.take<float2>((size_t)B * d);
        descs = c.take<GemmDesc>((size_t)2 * B);
        E = c.take<float2>(mat * std::min(B, REPROJECT_CHUNK));
        obs_partial = c.take<double>(observable_partial_doubles(d, B));
        loc = c.take<int>(B);
        obsT = c.take<float2>(mat * std::min(B, OBS_CHUNK));
        bytes = c.used;
    }
};

}  // namespace

bool kron_supported(const redo_table_s* t) {
    const int d = t->desc.d;
    return t->kron_n > 0 && t->desc.drift_is_diag && d >= 128 && d <= 4096 && (d & (d - 1)) == 0;
}

size_t kron_workspace_bytes(const redo_table_s* t, int B, int N) { return KronWS(t, B, N, nullptr).bytes; }

redo_status kron_chain(redo_table_s* t, int quantised, const float* u, const int* n_steps, int B, int N,
                       int step_offset, int reproject_every, const float* X0, float* U_total, const int* obs_cols,
                       const float* obs_vals, int obs_width, double* obs_out, void* workspace, size_t workspace_bytes,
                       hipStream_t st, bool walsh_frame, const double* walsh) {
    KronWS need(t, B, N, nullptr);
    if (!workspace || workspace_bytes < need.bytes)
        return fail(REDO_ERR_WORKSPACE, "structure-aware chain workspace needs " + std::to_string(need.bytes) + " bytes");
    KronWS w(t, B, N, workspace);
    const int d = t->desc.d;
    const long long mat = (long long)d * d;
    float2* X[2] = {reinterpret_cast<float2*>(U_total), w.W1};
    if (quantised) REDO_HIP(quantise_all(t, u, B, N, w.codes, w.phi, st));
    if (!X0)
        REDO_HIP(walsh_frame ? walsh_fill(d, B, X[0], mat, st) : fill_identity(d, B, X[0], mat, st));
    else if (X0 != U_total)
        REDO_HIP(hipMemcpyAsync(X[0], X0, sizeof(float2) * mat * B, hipMemcpyDeviceToDevice, st));
    REDO_HIP(fill_int(w.loc, B, 0, st));
    KronPlanArgs pa{};
    pa.s = t->kron_s;
    pa.h = t->h64;
    pa.g = t->desc.phased ? t->g64 : nullptr;
    pa.n_steps = n_steps;
    pa.gates = w.gates;
    pa.pre = w.pre;
    pa.post = w.post;
    pa.eps = t->desc.eps;
    pa.dt = t->desc.dt;
    pa.n = t->kron_n;
    pa.d = d;
    pa.K = t->desc.K;
    pa.N = N;
    pa.n_drift = t->desc.n_drift;
    pa.phased = t->desc.phased;
    pa.strang = t->desc.splitting;
    if (quantised) {
        pa.codes = w.codes;
        pa.phi = t->desc.phased ? w.phi : nullptr;
    } else {
        pa.u = u;
    }
    // in the Walsh frame at d = 1024 the observable rides on the step kernel (steps without
    // a re-projection: there it must see the re-projected state)
    const bool fuse = walsh_frame && obs_out && d == 1024;
    int* pc = nullptr;
    float2* pv = nullptr;
    if (fuse) {
        REDO_HIP(obs_pack_lists(d, B, obs_width, obs_cols, reinterpret_cast<const float2*>(obs_vals), w.obs_partial, st));
        obs_packed_lists(d, B, w.obs_partial, &pc, &pv);
    }
    for (int n = 0; n < N; ++n) {
        pa.step = n;
        hipLaunchKernelGGL(kron_plan_kernel, dim3(B), dim3(256), 0, st, pa);
        REDO_HIP(hipGetLastError());
        const bool reproj = reproject_every > 0 && ((long long)step_offset + n + 1) % reproject_every == 0;
        if (fuse && !reproj) {
            REDO_HIP(kron_step_observable(B, X[0], X[1], w.loc, mat, w.gates, w.pre, w.post, n_steps, n, obs_width, pc,
                                          pv, reinterpret_cast<const float2*>(obs_vals), walsh, w.obs_partial,
                                          obs_out + n, N, st));
            continue;
        }
        REDO_HIP(kron_step(d, B, X[0], X[1], w.loc, mat, w.gates, w.pre, w.post, n_steps, n, st));
        if (reproj)   // X <- X (3I - X^dag X) / 2 into the other buffer, Gram product in 3M FP32
            REDO_HIP(reproject_states(d, B, X[0], X[1], mat, w.E, w.descs, w.loc, n_steps, n, 1, t->flags, st));
        if (obs_out)
            REDO_HIP(walsh_frame ? observable_walsh(d, B, X[0], X[1], w.loc, mat, obs_cols,
                                             reinterpret_cast<const float2*>(obs_vals), obs_width, walsh, n_steps,
                                             n, w.obs_partial, obs_out + n, N, st)
                           : observable(d, B, X[0], X[1], w.loc, mat, obs_cols,
                                        reinterpret_cast<const float2*>(obs_vals), obs_width, n_steps, n,
                                        w.obs_partial, obs_out + n, N, w.obsT, OBS_CHUNK, st));
    }
    REDO_HIP(gather_back(d, B, X[0], X[1], mat, w.loc, st));
    return REDO_OK;
}

}  // namespace redo
