// State-transfer GRAPE (Sec. III, the state fidelity F_S = |<psi_f|psi(T)>|^2):
// the forward chain psi_n = U_n psi_{n-1} and the backward scan
// chi_{n-1} = U_n^dag chi_n (chi_N = psi_f) on vectors, with every step
// applied as its REDO factors (process 2, or the composed levels of process
// 3) between the drift and phase scalings of the split step (Sec. III, Eqs.
// vn and vnd).  The gradient uses the same trace identities as the unitary
// adjoint with the rank-one Y_n = psi_n chi_n^dag:
//     dg/dOmega_kn = -i dt chi_n^dag Z S_k Z^dag psi_n,
//     dg/dphi_kn   = -i (chi_n^dag G_k psi_n - chi_{n-1}^dag G_k psi_{n-1}),
// g = <psi_f|psi_N>, dF_S = 2 Re(conj(g) dg).  Every product is a batched
// matrix-vector product over the instances: the factors are the FP32 table
// entries, the vectors psi_n and chi_n, the phase scalings and the products'
// sums are FP64, so each factor application adds only the rounding of its
// stored factor; traces accumulate in FP64.
#include <algorithm>
#include <cstring>
#include <string>

#include "large_path.h"

namespace redo {
namespace {

struct MvDesc {
    const float2* F;      // d x d factor (FP32), or null (identity)
    const double2* pre;   // scaling of the input vector, or null
    const double2* post;  // scaling of the output vector, or null
    const double2* x;
    double2* y;
    int adj;              // 1: y = post . F^dag (pre . x)
    int conj_scales;      // 1: conj(pre), conj(post)
};

// y = post . op(F) (pre . x), one workgroup of 16 waves per 16 rows of y reading those
// rows of op(F) whole (16 d complex entries, 128 KiB at d = 1024) in blocks of 16
// independent loads per thread, the scaled input in LDS (FP64, 16 d bytes), FP64
// products and sums of the FP32 factor entries: nothing leaves the workgroup
// before the result, so one factor application is one launch and the summation order
// is fixed.  blockIdx.y runs over the instances of up to two independent chains, the
// forward chain and the backward scan: y < B takes descs0[y], y >= B descs1[y - B].
constexpr int MV_R = 16;
constexpr int MV_NT = 1024;
static_assert(MV_NT / 64 == MV_R && 64 % MV_R == 0, "one wave per row, column groups of the adjoint");
constexpr int MV_U = 16;    // loads per thread in flight

// the factors come through descriptors, which the compiler cannot place in an address
// space: mark them global so the loads are global (vector-memory counter only), not flat
typedef float mv_v2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const mv_v2 mv_gv2;

__device__ inline float2 mv_load(const float2* p, long long i) {
    const mv_v2 v = ((mv_gv2*)p)[i];
    return make_float2(v.x, v.y);
}

__device__ inline double2 mv_scale(const MvDesc& m, const double2* s, int i) {
    const double2 p = s[i];
    return m.conj_scales ? zconj(p) : p;
}

__device__ inline double2 mv_input(const MvDesc& m, int c) {
    const double2 v = m.x[c];
    return m.pre ? zmul(mv_scale(m, m.pre, c), v) : v;
}

// a += f x and a += conj(f) x in FP64, f an FP32 factor entry
__device__ inline void zfma_f(double2& a, float2 f, double2 x) {
    a.x += (double)f.x * x.x - (double)f.y * x.y;
    a.y += (double)f.x * x.y + (double)f.y * x.x;
}
__device__ inline void zfma_fc(double2& a, float2 f, double2 x) {
    a.x += (double)f.x * x.x + (double)f.y * x.y;
    a.y += (double)f.x * x.y - (double)f.y * x.x;
}

__global__ __launch_bounds__(MV_NT) void matvec_kernel(int d, const MvDesc* __restrict__ descs0,
                                                       const MvDesc* __restrict__ descs1, int B) {
    extern __shared__ double2 xs[];   // [d]: pre . x
    __shared__ double2 red[MV_NT / 64][MV_R];
    const int z = blockIdx.y;
    const MvDesc m = z < B ? descs0[z] : descs1[z - B];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int r0 = blockIdx.x * MV_R;
    if (!m.F) {   // identity factor: copy with the scalings
        const int r = r0 + t;
        if (t < MV_R && r < d) {
            double2 v = mv_input(m, r);
            if (m.post) v = zmul(mv_scale(m, m.post, r), v);
            m.y[r] = v;
        }
        return;
    }
    for (int c = t; c < d; c += MV_NT) xs[c] = mv_input(m, c);
    __syncthreads();
    double2 acc = make_double2(0.0, 0.0);
    if (m.adj) {
        // y_r = sum_c conj(F[c][r]) x_c: lanes over the MV_R rows (one segment of row c of F)
        // and 64 / MV_R column groups, waves over the others (64 in all); column c = 64 j + group
        const int rl = lane % MV_R, cg = lane / MV_R + (64 / MV_R) * wv, r = r0 + rl;
        const bool ok = r < d;
        for (int cb = 0; cb < d; cb += 64 * MV_U) {
            float2 f[MV_U];
#pragma unroll
            for (int j = 0; j < MV_U; ++j) {
                const int c = cb + cg + 64 * j;
                f[j] = (ok && c < d) ? mv_load(m.F, (long long)c * d + r) : make_float2(0.f, 0.f);
            }
#pragma unroll
            for (int j = 0; j < MV_U; ++j) {
                const int c = cb + cg + 64 * j;
                if (c < d) zfma_fc(acc, f[j], xs[c]);
            }
        }
#pragma unroll
        for (int o = MV_R; o < 64; o <<= 1) {
            acc.x += __shfl_xor(acc.x, o);
            acc.y += __shfl_xor(acc.y, o);
        }
        if (lane < MV_R) red[wv][lane] = acc;
    } else {
        // y_r = sum_c F[r][c] x_c: wave w takes row r0 + w, lanes over columns c = lane + 64 j
        // (512 contiguous bytes of the row per load), then a wave sum
        const int r = r0 + wv;
        const bool ok = r < d;
        for (int cb = 0; cb < d; cb += 64 * MV_U) {
            float2 f[MV_U];
#pragma unroll
            for (int j = 0; j < MV_U; ++j) {
                const int c = cb + lane + 64 * j;
                f[j] = (ok && c < d) ? mv_load(m.F, (long long)r * d + c) : make_float2(0.f, 0.f);
            }
#pragma unroll
            for (int j = 0; j < MV_U; ++j) {
                const int c = cb + lane + 64 * j;
                if (c < d) zfma_f(acc, f[j], xs[c]);
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            acc.x += __shfl_xor(acc.x, o);
            acc.y += __shfl_xor(acc.y, o);
        }
        if (lane == 0) red[0][wv] = acc;
    }
    __syncthreads();
    const int r = r0 + t;
    if (t < MV_R && r < d) {
        double2 v = red[0][t];
        if (m.adj) {
#pragma unroll
            for (int w = 1; w < MV_NT / 64; ++w) v = make_double2(v.x + red[w][t].x, v.y + red[w][t].y);
        }
        if (m.post) v = zmul(mv_scale(m, m.post, r), v);
        m.y[r] = v;
    }
}

struct StatePlan {
    const float2* T;
    const float2* V;        // dense drifts or null
    const double* h;        // diagonal drifts or null
    const double* g;
    const float2* cache;
    const int* codes;       // [B][N][K] (this step at + step * K)
    const double* phi;
    const int* n_steps;
    long long ent;
    int d, K, P, base, n_drift, phased, dense, strang, cache_levels, all_cached, slots, N, step, backward;
    int all;                // 1: grid (B, N), every step and both directions in one launch
    double dt;
    double2* Psi;           // forward vectors [B][N + 1][d] (FP64)
    double2* Chi;           // backward vectors [B][N + 1][d] (FP64)
    long long vs;           // per-instance stride of Psi and Chi
    double2* tmp0;          // [2][B][d] ping-pong for the slots in between, per direction
    double2* tmp1;
    double2 *pre, *post, *pstar;  // [B][d] per planned step (FP64 phases)
    MvDesc* descs;          // [slots][B] per planned step and direction
    int B;
};

// per instance and step: the step's scale vectors and one descriptor per slot.  Forward
// (psi <- U psi): pre on slot 0 (with the dense drift as slot 0 and Z^dag after it),
// post on the last slot.  Backward (chi <- U^dag chi): the slots in reverse order,
// adjoint factors, conjugated scalings.  With a.all the launch covers every step
// (blockIdx.y) and writes the descriptors of both directions.
__global__ void state_plan_kernel(StatePlan a) {
    const int b = blockIdx.x, d = a.d;
    const int step = a.all ? (int)blockIdx.y : a.step;
    const long long so = a.all ? (long long)step * a.B * d : 0;
    double2* pre = a.pre + so;
    double2* post = a.post + so;
    double2* pstar = a.pstar + so;
    const bool active = a.n_steps ? step < a.n_steps[b] : true;
    const int* cb = a.codes + ((long long)b * a.N + step) * a.K;
    const double* pb = a.phi ? a.phi + ((long long)b * a.N + step) * a.K : nullptr;
    const int drift = b % a.n_drift;
    for (int r = threadIdx.x; r < d; r += blockDim.x) {
        double th = 0.0;
        if (a.phased)
            for (int k = 0; k < a.K; ++k) th += pb[k] * a.g[(long long)k * d + r];
        const double hd = (!a.dense && a.strang) ? 0.5 * a.dt * a.h[(long long)drift * d + r] : 0.0;
        const double2 po = expmi(th + hd);
        post[(long long)b * d + r] = po;
        pstar[(long long)b * d + r] = zconj(po);
        if (!a.dense) {
            const double hdt = a.strang ? 0.5 * a.dt : a.dt;
            pre[(long long)b * d + r] = expmi(hdt * a.h[(long long)drift * d + r] - th);
        }
    }
    if (threadIdx.x != 0) return;
    const int S = a.slots;
    for (int dir = a.all ? 0 : a.backward; dir <= (a.all ? 1 : a.backward); ++dir) {
        const double2* src = dir ? a.Chi + (long long)(step + 1) * d : a.Psi + (long long)step * d;
        double2* dst = dir ? a.Chi + (long long)step * d : a.Psi + (long long)(step + 1) * d;
        MvDesc* out = a.all ? a.descs + (long long)(dir * a.N + step) * S * a.B : a.descs;
        for (int i = 0; i < S; ++i) {
            // forward slot index of the i-th application
            const int s = dir ? S - 1 - i : i;
            MvDesc m{};
            const long long tb = (long long)(dir * a.B + b) * d;
            m.x = i == 0 ? src + (long long)b * a.vs : ((i - 1) % 2 == 0 ? a.tmp0 : a.tmp1) + tb;
            m.y = i == S - 1 ? dst + (long long)b * a.vs : (i % 2 == 0 ? a.tmp0 : a.tmp1) + tb;
            if (active) {
                int fadj = 0;
                if (a.dense && s == 0) {
                    m.F = a.V + (long long)drift * a.ent;
                } else {
                    const int slot = s - a.dense;
                    const int k = a.all_cached ? slot : slot / a.P;
                    const int j = a.all_cached ? 0 : slot % a.P;
                    const int q = cb[k];
                    const int aq = q < 0 ? -q : q;
                    fadj = q < 0 ? 1 : 0;
                    if (a.all_cached) {
                        if (aq != 0) m.F = a.cache + ((long long)k * a.cache_levels + aq) * a.ent;
                    } else {
                        const int c = digit_of(q, j, a.base);
                        if (c) m.F = a.T + ((long long)(k * a.P + j) * (a.base - 1) + (c - 1)) * a.ent;
                    }
                }
                m.adj = dir ? 1 - fadj : fadj;
                // the scalings of the forward step: pre before slot 0 (diagonal drift), Z^dag after
                // the dense drift (slot 0), Z (times the second half drift, Strang) after the last slot
                const double2* fpre = (!a.dense && s == 0) ? pre + (long long)b * d : nullptr;
                const double2* fpost = nullptr;
                if (a.dense && s == 0 && a.phased) fpost = pstar + (long long)b * d;
                if (s == S - 1 && (a.phased || a.strang) && !(a.dense && s == 0)) fpost = post + (long long)b * d;
                if (!dir) {
                    m.pre = fpre;
                    m.post = fpost;
                } else {
                    m.pre = fpost;
                    m.post = fpre;
                    m.conj_scales = 1;
                }
            }
            out[(long long)i * a.B + b] = m;
        }
    }
}

// Traces of Y = psi chi^dag for step s (psi = psi_{s+1}, chi = chi_{s+1}) and every channel:
//   T1 = chi^dag S^psi psi, T2 = chi^dag S^{pi/2} psi (phased, q = 0), D = chi^dag G psi,
// with S^psi_aj = exp(-i psi (g_a - g_j)) S_aj (times exp(-i dt/2 (h_a - h_j)), Strang).
// One workgroup per (instance, step); the column phases ride on psi (rounded to FP32 in
// LDS: these traces enter only the gradient), the row phases on chi; sums in FP64.
__global__ __launch_bounds__(256) void state_trace_kernel(int d, int N, int K, int phased, int strang, double dt,
                                                          int n_drift, const double2* __restrict__ Psi,
                                                          const double2* __restrict__ Chi, long long vs,
                                                          const float2* __restrict__ S32, const int* spc,
                                                          const double2* spv, int sw, const double* g,
                                                          const double* h, const int* codes, const double* phi,
                                                          const int* n_steps, double* tr) {
    extern __shared__ float2 pv[];   // [2][d]: psi with the column phases of T1 and of T2
    __shared__ double red[6][256];
    const int s = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
    const bool active = n_steps ? s < n_steps[b] : true;
    const double2* psi = Psi + (long long)b * vs + (long long)(s + 1) * d;
    const double2* chi = Chi + (long long)b * vs + (long long)(s + 1) * d;
    const long long hb = (long long)(b % n_drift) * d;
    for (int k = 0; k < K; ++k) {
        const long long ci = ((long long)b * N + s) * K + k;
        const int q = active ? codes[ci] : 1;
        const bool origin = phased && q == 0;
        const double ps = (phased && !origin && active) ? phi[ci] : 0.0;
        const double hdt = strang ? 0.5 * dt : 0.0;
        __syncthreads();
        for (int j = tid; j < d; j += 256) {
            const double gj = phased ? g[(long long)k * d + j] : 0.0;
            const double hj = strang ? h[hb + j] : 0.0;
            const double2 x = psi[j];
            const double2 e1 = zconj(expmi(ps * gj + hdt * hj));
            pv[j] = make_float2((float)(e1.x * x.x - e1.y * x.y), (float)(e1.x * x.y + e1.y * x.x));
            if (origin) {
                const double2 e2 = zconj(expmi(1.5707963267948966 * gj + hdt * hj));
                pv[d + j] = make_float2((float)(e2.x * x.x - e2.y * x.y), (float)(e2.x * x.y + e2.y * x.x));
            }
        }
        __syncthreads();
        double v[6] = {0, 0, 0, 0, 0, 0};
        if (active)
            for (int a = tid; a < d; a += 256) {
                const double ga = phased ? g[(long long)k * d + a] : 0.0;
                const double ha = strang ? h[hb + a] : 0.0;
                const double2 c = chi[a];
                // row factor conj(chi_a) exp(-i (psi g_a + dt/2 h_a))
                const double2 ra = zmul(make_double2(c.x, -c.y), expmi(ps * ga + hdt * ha));
                double s1r = 0, s1i = 0, s2r = 0, s2i = 0;
                if (sw > 0) {
                    for (int t = 0; t < sw; ++t) {
                        const int j = spc[(long long)a * sw + t];
                        const double2 sv = spv[((long long)k * d + a) * sw + t];
                        const float2 x = pv[j];
                        s1r += sv.x * x.x - sv.y * x.y;
                        s1i += sv.x * x.y + sv.y * x.x;
                        if (origin) {
                            const float2 x2 = pv[d + j];
                            s2r += sv.x * x2.x - sv.y * x2.y;
                            s2i += sv.x * x2.y + sv.y * x2.x;
                        }
                    }
                } else {
                    const float2* Sr = S32 + (long long)k * d * d + (long long)a * d;
                    for (int j = 0; j < d; ++j) {
                        const float2 sv = Sr[j];
                        const float2 x = pv[j];
                        s1r += (double)sv.x * x.x - (double)sv.y * x.y;
                        s1i += (double)sv.x * x.y + (double)sv.y * x.x;
                        if (origin) {
                            const float2 x2 = pv[d + j];
                            s2r += (double)sv.x * x2.x - (double)sv.y * x2.y;
                            s2i += (double)sv.x * x2.y + (double)sv.y * x2.x;
                        }
                    }
                }
                v[0] += ra.x * s1r - ra.y * s1i;
                v[1] += ra.x * s1i + ra.y * s1r;
                if (origin) {
                    const double2 ra2 = zmul(make_double2(c.x, -c.y), expmi(1.5707963267948966 * ga + hdt * ha));
                    v[2] += ra2.x * s2r - ra2.y * s2i;
                    v[3] += ra2.x * s2i + ra2.y * s2r;
                }
                if (phased) {
                    const double2 x = psi[a];
                    // conj(chi_a) g_a psi_a
                    v[4] += ga * (c.x * x.x + c.y * x.y);
                    v[5] += ga * (c.x * x.y - c.y * x.x);
                }
            }
#pragma unroll
        for (int c = 0; c < 6; ++c) red[c][tid] = v[c];
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (tid < st)
#pragma unroll
                for (int c = 0; c < 6; ++c) red[c][tid] += red[c][tid + st];
            __syncthreads();
        }
        if (tid < 6) tr[(((long long)b * N + s) * K + k) * 6 + tid] = red[tid][0];
    }
}

// overlap g = <psi_f|psi_N> (FP64), F_S = |g|^2; D_0 = chi_0^dag G psi_0; nu = 1
__global__ void state_final_kernel(int d, int K, int phased, const float2* psif, const double2* Psi,
                                   const double2* Chi, long long vs, int N, const int* n_steps, const double* g,
                                   double2* ov, double* fidelity, double* d0, double* nu) {
    const int b = blockIdx.x, tid = threadIdx.x;
    __shared__ double red[2][256];
    const double2* pn = Psi + (long long)b * vs + (long long)N * d;
    double gr = 0, gi = 0;
    for (int a = tid; a < d; a += 256) {
        const float2 f = psif[(long long)b * d + a];
        const double2 x = pn[a];
        gr += (double)f.x * x.x + (double)f.y * x.y;
        gi += (double)f.x * x.y - (double)f.y * x.x;
    }
    red[0][tid] = gr;
    red[1][tid] = gi;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) {
            red[0][tid] += red[0][tid + st];
            red[1][tid] += red[1][tid + st];
        }
        __syncthreads();
    }
    if (tid == 0) {
        ov[b] = make_double2(red[0][0], red[1][0]);
        if (fidelity) fidelity[b] = red[0][0] * red[0][0] + red[1][0] * red[1][0];
        nu[b] = 1.0;
    }
    const double2* p0 = Psi + (long long)b * vs;
    const double2* c0 = Chi + (long long)b * vs;
    for (int k = 0; k < K; ++k) {
        __syncthreads();
        double dr = 0, di = 0;
        if (phased)
            for (int a = tid; a < d; a += 256) {
                const double ga = g[(long long)k * d + a];
                const double2 c = c0[a], x = p0[a];
                dr += ga * (c.x * x.x + c.y * x.y);
                di += ga * (c.x * x.y - c.y * x.x);
            }
        red[0][tid] = dr;
        red[1][tid] = di;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (tid < st) {
                red[0][tid] += red[0][tid + st];
                red[1][tid] += red[1][tid + st];
            }
            __syncthreads();
        }
        if (tid == 0) {
            d0[((long long)b * K + k) * 2] = red[0][0];
            d0[((long long)b * K + k) * 2 + 1] = red[1][0];
        }
    }
}

// widens the caller's c64 vectors [B][d] into the FP64 chain arrays (instance stride vs)
__global__ void widen_kernel(int d, const float2* __restrict__ in, double2* __restrict__ out, long long vs) {
    const int b = blockIdx.y;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= d) return;
    const float2 v = in[(long long)b * d + a];
    out[(long long)b * vs + a] = make_double2(v.x, v.y);
}

struct StateWS {
    int* codes;
    double* phi;
    double2 *Psi, *Chi, *tmp0, *tmp1, *pre, *post, *pstar;
    MvDesc* descs;
    double *tr, *d0, *nu;
    double2* ov;
    size_t bytes;
    StateWS(const redo_table_s* t, int B, int N, int slots, void* base, int plan_steps = 1) {
        const int d = t->desc.d, K = t->desc.K;
        char* p = static_cast<char*>(base);
        size_t used = 0;
        auto take = [&](size_t n) {
            char* q = p ? p + used : nullptr;
            used += align_up(n);
            return q;
        };
        codes = reinterpret_cast<int*>(take(sizeof(int) * (size_t)B * N * K));
        phi = reinterpret_cast<double*>(take(sizeof(double) * (size_t)B * N * K));
        Psi = reinterpret_cast<double2*>(take(sizeof(double2) * (size_t)B * (N + 1) * d));
        Chi = reinterpret_cast<double2*>(take(sizeof(double2) * (size_t)B * (N + 1) * d));
        tmp0 = reinterpret_cast<double2*>(take(sizeof(double2) * 2 * (size_t)B * d));
        tmp1 = reinterpret_cast<double2*>(take(sizeof(double2) * 2 * (size_t)B * d));
        pre = reinterpret_cast<double2*>(take(sizeof(double2) * (size_t)plan_steps * B * d));
        post = reinterpret_cast<double2*>(take(sizeof(double2) * (size_t)plan_steps * B * d));
        pstar = reinterpret_cast<double2*>(take(sizeof(double2) * (size_t)plan_steps * B * d));
        descs = reinterpret_cast<MvDesc*>(take(sizeof(MvDesc) * (size_t)(plan_steps > 1 ? 2 : 1) * plan_steps * B * slots));
        tr = reinterpret_cast<double*>(take(sizeof(double) * (size_t)B * N * K * 6));
        d0 = reinterpret_cast<double*>(take(sizeof(double) * (size_t)B * K * 2));
        nu = reinterpret_cast<double*>(take(sizeof(double) * (size_t)B));
        ov = reinterpret_cast<double2*>(take(sizeof(double2) * (size_t)B));
        bytes = used;
    }
};

bool cached_all(const redo_table_s* t) {
    return t->cache && t->cache_lo == 0 && (double)t->cache_hi >= t->qmax;
}

int state_slots(const redo_table_s* t) {
    return (t->desc.drift_is_diag ? 0 : 1) + (cached_all(t) ? t->desc.K : t->desc.K * t->desc.digits);
}

// every step planned in one launch when its scale vectors and descriptors take at most this much
constexpr size_t STATE_PLAN_ALL_BYTES = size_t(256) << 20;
// the matrix-vector kernel keeps the FP64 input vector in LDS (16 d bytes)
constexpr int STATE_MAX_D = 8192;

int state_plan_steps(const redo_table_s* t, int B, int N) {
    const size_t per_step = (size_t)B * (3 * sizeof(double2) * t->desc.d + 2 * sizeof(MvDesc) * state_slots(t));
    return (N <= 65535 && per_step * N <= STATE_PLAN_ALL_BYTES) ? N : 1;   // grid.y bounds N
}

}  // namespace

size_t state_grape_workspace_bytes(const redo_table_s* t, int B, int N) {
    return StateWS(t, B, N, state_slots(t), nullptr, state_plan_steps(t, B, N)).bytes;
}

redo_status state_grape(redo_table_s* t, const float* u, const int* n_steps, int B, int N, const float* psi0,
                        const float* psif, double* fidelity, double* overlap, float* grad, void* workspace,
                        size_t workspace_bytes, hipStream_t st) {
    if (B > 32767) return fail(REDO_ERR_UNSUPPORTED, "state GRAPE takes at most 32767 instances per call");
    if (t->desc.d > STATE_MAX_D)
        return fail(REDO_ERR_UNSUPPORTED, "state GRAPE keeps its FP64 input vector in LDS: d <= 8192");
    const int S = state_slots(t);
    const int PS = state_plan_steps(t, B, N);
    StateWS need(t, B, N, S, nullptr, PS);
    if (!workspace || workspace_bytes < need.bytes)
        return fail(REDO_ERR_WORKSPACE, "state GRAPE workspace needs " + std::to_string(need.bytes) + " bytes");
    StateWS w(t, B, N, S, workspace, PS);
    const int d = t->desc.d, K = t->desc.K;
    const long long vs = (long long)(N + 1) * d;
    REDO_HIP(quantise_all(t, u, B, N, w.codes, w.phi, st));
    // psi_0 and chi_N, widened to FP64
    hipLaunchKernelGGL(widen_kernel, dim3((d + 255) / 256, B), dim3(256), 0, st, d,
                       reinterpret_cast<const float2*>(psi0), w.Psi, vs);
    hipLaunchKernelGGL(widen_kernel, dim3((d + 255) / 256, B), dim3(256), 0, st, d,
                       reinterpret_cast<const float2*>(psif), w.Chi + (size_t)N * d, vs);
    REDO_HIP(hipGetLastError());
    StatePlan p{};
    p.T = t->T32;
    p.V = t->desc.drift_is_diag ? nullptr : t->V32;
    p.h = t->h64;
    p.g = t->g64;
    p.cache = t->cache;
    p.codes = w.codes;
    p.phi = t->desc.phased ? w.phi : nullptr;
    p.n_steps = n_steps;
    p.ent = t->entry_elems;
    p.d = d;
    p.K = K;
    p.P = t->desc.digits;
    p.base = t->desc.base;
    p.n_drift = t->desc.n_drift;
    p.phased = t->desc.phased;
    p.dense = t->desc.drift_is_diag ? 0 : 1;
    p.strang = t->desc.splitting;
    p.cache_levels = t->cache ? t->cache_hi - t->cache_lo + 1 : 0;
    p.all_cached = cached_all(t) ? 1 : 0;
    p.slots = S;
    p.N = N;
    p.dt = t->desc.dt;
    p.tmp0 = w.tmp0;
    p.tmp1 = w.tmp1;
    p.pre = w.pre;
    p.post = w.post;
    p.pstar = w.pstar;
    p.descs = w.descs;
    p.B = B;
    p.vs = vs;
    p.Psi = w.Psi;
    p.Chi = w.Chi;
    p.all = PS > 1 ? 1 : 0;
    const int nrt = (d + MV_R - 1) / MV_R;
    if (S == 0) return fail(REDO_ERR_UNSUPPORTED, "no factor slots");
    const size_t mv_lds = sizeof(double2) * (size_t)d;
    REDO_HIP(hipFuncSetAttribute((const void*)matvec_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)mv_lds));
    if (p.all) {
        // every step planned at once: step n of the forward chain and step N - 1 - n of the
        // backward scan (independent chains) share each launch
        hipLaunchKernelGGL(state_plan_kernel, dim3(B, N), dim3(256), 0, st, p);
        REDO_HIP(hipGetLastError());
        for (int n = 0; n < N; ++n) {
            const MvDesc* fw = w.descs + (size_t)n * S * B;
            const MvDesc* bw = w.descs + (size_t)(N + N - 1 - n) * S * B;
            for (int i = 0; i < S; ++i)
                hipLaunchKernelGGL(matvec_kernel, dim3(nrt, 2 * B), dim3(MV_NT), mv_lds, st, d, fw + (size_t)i * B,
                                   bw + (size_t)i * B, B);
            REDO_HIP(hipGetLastError());
        }
    } else {
        auto run_step = [&](int n, int backward) -> hipError_t {
            p.step = n;
            p.backward = backward;
            hipLaunchKernelGGL(state_plan_kernel, dim3(B), dim3(256), 0, st, p);
            for (int i = 0; i < S; ++i)
                hipLaunchKernelGGL(matvec_kernel, dim3(nrt, B), dim3(MV_NT), mv_lds, st, d, w.descs + (size_t)i * B,
                                   (const MvDesc*)nullptr, B);
            return hipGetLastError();
        };
        for (int n = 0; n < N; ++n) REDO_HIP(run_step(n, 0));
        for (int n = N - 1; n >= 0; --n) REDO_HIP(run_step(n, 1));
    }
    hipLaunchKernelGGL(state_final_kernel, dim3(B), dim3(256), 0, st, d, K, t->desc.phased,
                       reinterpret_cast<const float2*>(psif), w.Psi, w.Chi, vs, N, n_steps, t->g64, w.ov, fidelity,
                       w.d0, w.nu);
    REDO_HIP(hipGetLastError());
    if (overlap) REDO_HIP(hipMemcpyAsync(overlap, w.ov, sizeof(double2) * B, hipMemcpyDeviceToDevice, st));
    const size_t tr_lds = sizeof(float2) * 2 * (size_t)d;
    REDO_HIP(hipFuncSetAttribute((const void*)state_trace_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)tr_lds));
    hipLaunchKernelGGL(state_trace_kernel, dim3(N, B), dim3(256), tr_lds, st, d, N, K, t->desc.phased,
                       t->desc.splitting, t->desc.dt, t->desc.n_drift, w.Psi, w.Chi, vs, t->S32, t->spat_cols,
                       t->spat_vals, t->spat_w, t->g64, t->h64, w.codes, t->desc.phased ? w.phi : nullptr, n_steps,
                       w.tr);
    REDO_HIP(hipGetLastError());
    REDO_HIP(grad_assemble(B, N, K, t->desc.phased, t->desc.eps, t->desc.dt, w.codes,
                           t->desc.phased ? w.phi : nullptr, w.tr, w.d0, w.ov, w.nu, n_steps, grad, 0, st));
    return REDO_OK;
}

}  // namespace redo
