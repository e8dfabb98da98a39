// Small kernels around the batched GEMMs of the large-d REDO path: per-step
// planning (which table entries a step's digits select, Sec. II, processes 2
// and 3; the drift and phase scalings of the split step, Sec. III), the
// observable of Sec. IV, and the traces and gradient assembly of the GRAPE
// adjoint (Sec. III).  All traces accumulate in FP64.
#include <algorithm>
#include <cmath>

#include "large_path.h"

namespace redo {
namespace {

struct PlanArgs {
    const float2* T;        // table [K][P][b-1][d][d]
    const float2* V;        // dense drifts [n_drift][d][d] (dense) or null
    const double* h;        // diagonal drifts [n_drift][d] (diag) or null
    const double* g;        // phase generators [K][d] or null
    const float2* cache;    // composed levels [K][levels][d][d] or null
    const int* codes;       // codes of this step, instance b at codes + b * code_stride
    const double* phi;      // same layout, or null
    const int* n_steps;     // [B] or null
    long long ent;          // d*d
    long long code_stride;
    int d, K, P, base, n_drift, phased, dense;
    int cache_lo, cache_hi, cache_levels;
    int step;               // step index n (for the activity test)
    int drift_div;          // drift of instance b: ((drift_offset + b) / drift_div) % n_drift
    long long drift_offset;
    double dt;
    float2* X[2];           // state buffers (per instance stride xstride)
    long long xstride;
    int* loc;               // [B]: which buffer holds the state of instance b (updated here)
    int compose;            // 1: the state starts as the identity (no B operand)
    int slots;              // launched slots: dense + K (all levels cached) or dense + K * P
    int all_cached;
    const uint16_t* cache_bf;   // pre-split BF16 panels of the cache, or null
    int bf_conj;            // negative levels may use the conjugated panel of |q|
    int strang;             // U_n = V(dt/2) C_n V(dt/2): half drift in pre, half in post (diagonal drift)
    float2* pre;            // [B][d] scale vectors of this step
    float2* post;
    float2* pstar;
    GemmDesc* descs;        // [slots][B]
    int B;
};

// One workgroup per instance: the step's scale vectors and one descriptor per
// launched slot.  A slot whose factor is the identity is switched off (no
// copy); the state's buffer is tracked per instance in loc[b].  The drift and
// Z^dag scaling rides on the first active factor, Z on the last one; a step
// with no active factor becomes one scaled copy.
__global__ __launch_bounds__(256) void plan_step_kernel(PlanArgs a) {
    const int b = blockIdx.x;
    const int d = a.d;
    const bool active = a.n_steps ? a.step < a.n_steps[b] : true;
    const int* cb = a.codes + (long long)b * a.code_stride;
    const double* pb = a.phi ? a.phi + (long long)b * a.code_stride : nullptr;
    const int drift = (int)(((a.drift_offset + b) / a.drift_div) % a.n_drift);
    if (active)
        for (int r = threadIdx.x; r < d; r += blockDim.x) {
            double th = 0.0;
            if (a.phased)
                for (int k = 0; k < a.K; ++k) th += pb[k] * a.g[(long long)k * d + r];
            const double hd = (!a.dense && a.strang) ? 0.5 * a.dt * a.h[(long long)drift * d + r] : 0.0;
            const double2 po = expmi(th + hd);                   // e^{-i theta} (times v^{1/2}, Strang)
            a.post[(long long)b * d + r] = make_float2((float)po.x, (float)po.y);
            a.pstar[(long long)b * d + r] = make_float2((float)po.x, (float)-po.y);
            if (!a.dense) {
                const double hdt = a.strang ? 0.5 * a.dt : a.dt;
                const double2 pr = expmi(hdt * a.h[(long long)drift * d + r] - th);   // v e^{+i theta}
                a.pre[(long long)b * d + r] = make_float2((float)pr.x, (float)pr.y);
            }
        }
    if (threadIdx.x != 0) return;
    const int S = a.slots;
    int loc = a.loc[b];
    // factors of every slot (null = identity)
    const float2* fa[64];
    const uint16_t* fb[64];   // the factor's pre-split panel, if any
    int fo[64];
    int last = -1, first_table = -1;
    for (int s = 0; s < S; ++s) {
        fa[s] = nullptr;
        fb[s] = nullptr;
        fo[s] = 0;
        if (!active) continue;
        if (a.dense && s == 0) {
            fa[s] = a.V + (long long)drift * a.ent;
        } else {
            const int slot = s - a.dense;
            const int k = a.all_cached ? slot : slot / a.P;
            const int j = a.all_cached ? 0 : slot % a.P;
            const int q = cb[k];
            const int aq = q < 0 ? -q : q;
            fo[s] = q < 0 ? 1 : 0;
            if (a.cache && aq >= a.cache_lo && aq <= a.cache_hi) {
                if (j == 0 && aq != 0) {
                    const long long ce = (long long)k * a.cache_levels + (aq - a.cache_lo);
                    fa[s] = a.cache + ce * a.ent;
                    if (a.cache_bf && (q > 0 || a.bf_conj)) fb[s] = a.cache_bf + ce * 4 * a.ent;
                }
            } else {
                const int c = digit_of(q, j, a.base);
                if (c) fa[s] = a.T + ((long long)(k * a.P + j) * (a.base - 1) + (c - 1)) * a.ent;
            }
            if (fa[s] && first_table < 0) first_table = s;
        }
        if (fa[s]) last = s;
    }
    const bool any_table = first_table >= 0;
    // a step with no factor at all: one scaled copy on the last slot
    const int copy_slot = (active && last < 0) ? S - 1 : -1;
    bool first_op = true;
    for (int s = 0; s < S; ++s) {
        GemmDesc g{};
        g.alpha = 1.f;
        const bool use = fa[s] != nullptr || s == copy_slot;
        g.active = use ? 1 : 0;
        if (use) {
            g.A = fa[s];
            g.opA = fo[s];
            g.Abf = fb[s];
            g.conjA = fo[s];
            g.B = (a.compose && first_op) ? nullptr : a.X[loc] + (long long)b * a.xstride;
            g.C = a.X[loc ^ 1] + (long long)b * a.xstride;
            if (a.dense) {
                if (s == 0 && a.phased && any_table) g.rscale = a.pstar + (long long)b * d;
            } else if (s == first_table || s == copy_slot) {
                g.kscale = a.pre + (long long)b * d;
            }
            if ((a.phased || a.strang) && (s == last || s == copy_slot) && (s != 0 || !a.dense))
                g.rscale = a.post + (long long)b * d;
            loc ^= 1;
            first_op = false;
        }
        a.descs[(long long)s * a.B + b] = g;
    }
    a.loc[b] = loc;
}

// re-projection descriptors from the tracked locations:
// phase 0: E_b = (I - X^dag X) / 2 (a Gram product);  phase 1: X'_b = X_b + X_b E_b into the
// other buffer (and flip loc)
__global__ void reproject_descs_kernel(GemmDesc* descs, int count, int b0, float2* X0, float2* X1, long long xstride,
                                       float2* E, long long estride, int* loc, const int* n_steps, int step, int phase) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int b = b0 + i;
    const bool active = n_steps ? step < n_steps[b] : true;
    GemmDesc g{};
    g.active = active ? 1 : 0;
    float2* X[2] = {X0, X1};
    const int l = loc[b];
    float2* xb = X[l] + (long long)b * xstride;
    if (phase == 0) {
        g.A = xb;
        g.opA = 1;
        g.B = xb;
        g.C = E + (long long)i * estride;
        g.alpha = -0.5f;
        g.beta_identity = 0.5f;
    } else {
        g.A = xb;
        g.B = E + (long long)i * estride;
        g.C = X[l ^ 1] + (long long)b * xstride;
        g.alpha = 1.f;
        g.addend = xb;
        if (active) loc[b] = l ^ 1;
    }
    descs[i] = g;
}

// unitarity watchdog of a re-projection step: E_b = (I - X^dag X) / 2 holds the Gram
// matrix, so ||X^dag X - I||_F = 2 ||E_b||_F; one workgroup per active instance, FP64 sum
__global__ __launch_bounds__(256) void unitarity_check_kernel(int d, const float2* __restrict__ E, long long estride,
                                                              const int* n_steps, int b0, int step, DeviceFlags* flags) {
    const int i = blockIdx.x;
    const int b = b0 + i;
    if (n_steps && step >= n_steps[b]) return;
    const float2* eb = E + (long long)i * estride;
    const long long nn = (long long)d * d;
    double s = 0.0;
    for (long long e = threadIdx.x; e < nn; e += 256) {
        const float2 v = eb[e];
        s += (double)v.x * v.x + (double)v.y * v.y;
    }
    __shared__ double part[256];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) report_drift(flags, 2.0 * sqrt(part[0] / d));
}

// copies the states that ended in buffer 1 back to buffer 0
__global__ void gather_back_kernel(long long nn, float2* X0, const float2* X1, long long xstride, const int* loc) {
    const int b = blockIdx.y;
    if (loc[b] == 0) return;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long long)gridDim.x * blockDim.x)
        X0[(long long)b * xstride + e] = X1[(long long)b * xstride + e];
}

__global__ void fill_int_kernel(int* p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// generic descriptors for a batch: C_b = op(A_b) op(B_b), inactive -> copy of op(B_b) (or skip)
__global__ void fill_descs_kernel(GemmDesc* descs, int count, const float2* A, long long sA, int opA, const float2* Bm,
                                  long long sB, int opB, float2* C, long long sC, const int* n_steps, int step,
                                  int inactive_mode, float alpha, float beta) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    GemmDesc g{};
    g.active = 1;
    g.alpha = alpha;
    g.beta_identity = beta;
    g.A = A ? A + b * sA : nullptr;
    g.B = Bm ? Bm + b * sB : nullptr;
    g.C = C + b * sC;
    g.opA = opA;
    g.opB = opB;
    const bool active = n_steps ? step < n_steps[b] : true;
    if (!active) {
        if (inactive_mode == 0) g.active = 0;
        if (inactive_mode == 2) {
            g.B = nullptr;
        } else {
            g.A = nullptr;
        }
        g.alpha = 1.f;
        g.beta_identity = 0.f;
    }
    descs[b] = g;
}

// GRAPE with every state kept: descriptors of all paired launches in one pass
__global__ void grape_pair_descs_kernel(GemmDesc* descs, int N, int B, const float2* U, long long sU, float2* X,
                                        long long sX, float2* LH, long long sL, long long mat, const int* n_steps) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)2 * N * B) return;
    const int b = (int)(e % B);
    const int which = (int)((e / B) % 2);
    const int i = (int)(e / (2LL * B));
    const int len = n_steps ? n_steps[b] : N;
    GemmDesc g{};
    g.active = 1;
    g.alpha = 1.f;
    if (which == 0) {
        // X_{i+1} = U_i X_i (X_0 = I: the identity right operand is a copy)
        g.A = i < len ? U + b * sU + (long long)i * mat : nullptr;
        g.B = i == 0 ? nullptr : X + b * sX + (long long)(i - 1) * mat;
        g.C = X + b * sX + (long long)i * mat;
    } else {
        // LH_m = U_m^H LH_{m+1}; past the length a copy of LH_{m+1}
        const int m = N - 1 - i;
        g.A = m < len ? U + b * sU + (long long)m * mat : nullptr;
        g.opA = 1;
        g.B = LH + b * sL + (long long)(m + 1) * mat;
        g.C = LH + b * sL + (long long)m * mat;
    }
    descs[e] = g;
}

// Observable in two passes over the instance (each pass reads X once):
//   pass 1: T = M X from column strips of X held in LDS (every row index available),
//   pass 2: (X M)_ac = sum_t X_a,cols[c][t] conj(vals[c][t]) from row blocks in LDS,
//           partial sums of Re((X M)_ac conj(T_ac)).
// Both passes stage their LDS fill through registers (several loads in flight
// per lane) and keep at most 64 KiB (pass 1) / 32 KiB (pass 2) of LDS per
// workgroup, so that workgroups share a CU and one's fill overlaps another's
// arithmetic.  Row lists are read two passes ahead (pass 1); column lists and
// the entries of T one column ahead (pass 2).  The list width is padded to WP
// (a multiple of 4) with zero-valued entries; padded entries load a valid
// index and contribute nothing.  Workgroups of one instance are kept on one
// XCD (round-robin dispatch over 8 XCDs).  Measured at d = 1024 (4096
// instances) this pair beat a single pass that gathers the rows of M X from
// L2 instead of writing T (26 vs 16 ms per step of 1024 instances).
constexpr int OBS_WMAX = 16;
constexpr int WALSH_DMAX = 2048;   // the strip of 8 columns in LDS: 128 KiB
inline int pow2_floor(int x) {
    int p = 1;
    while (p * 2 <= x) p *= 2;
    return p;
}
// strip width and row-block height: at most 64 KiB (8 x 1024 complex) and 32 KiB
// (4 x 1024 complex) of LDS, powers of two so that they divide d
inline int obs_strip(int d) { return pow2_floor(std::max(1, std::min(8, 8 * 1024 / d))); }
inline int obs_rows(int d) { return pow2_floor(std::max(1, std::min(4, 4 * 1024 / d))); }

__device__ inline long long xcd_local(long long bid, long long nb) {
    return (nb % 8 == 0) ? (bid % 8) * (nb / 8) + bid / 8 : bid;
}

// caller's row lists [d][w] -> packed [d][WP]
__global__ void obs_pack_kernel(int d, int w, int wp, const int* __restrict__ cols, const float2* __restrict__ vals,
                                int* __restrict__ pc, float2* __restrict__ pv) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= d * wp) return;
    const int a = e / wp, t = e % wp;
    pc[e] = t < w ? cols[(long long)a * w + t] : a;
    pv[e] = t < w ? vals[(long long)a * w + t] : make_float2(0.f, 0.f);
}

// Pass 1.  SW columns per strip; CPL complex entries per lane, LPR lanes per
// row; row lists are read two passes ahead.
template <int SW, int WP, int NT>
__global__ __launch_bounds__(NT, NT / 128) void observable_mx_kernel(int d, int b0, const float2* __restrict__ X0,
                                                           const float2* __restrict__ X1, const int* loc,
                                                           long long xstride, const int* __restrict__ cols,
                                                           const float2* __restrict__ vals, int w,
                                                           const int* n_steps, int step, float2* T) {
    constexpr int CPL = SW >= 2 ? 2 : 1;
    constexpr int LPR = SW / CPL;
    constexpr int RPP = NT / LPR;                   // rows per pass of the workgroup
    extern __shared__ float2 strip[];               // [d][SW]
    const int nstrip = d / SW;
    const long long bid = xcd_local(blockIdx.x, gridDim.x);
    const int i = (int)(bid / nstrip), sidx = (int)(bid % nstrip);
    const int b = b0 + i;
    if (n_steps && step >= n_steps[b]) return;      // uniform over the workgroup
    const float2* Xb = ((loc && loc[b]) ? X1 : X0) + (long long)b * xstride;
    const int c0 = sidx * SW;
    const int tid = threadIdx.x;
    const int cp = (tid % LPR) * CPL;
    int a = tid / LPR;
    int cc0[WP], cc1[WP];
    float2 cv0[WP], cv1[WP];
    obs_list<WP>(cols, vals, min(a, d - 1), cc0, cv0);
    obs_list<WP>(cols, vals, min(a + RPP, d - 1), cc1, cv1);
    const int n = d * SW;
    if (n % (NT * 16) == 0) {
        for (int base = 0; base < n; base += NT * 16) {
            float2 r[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = base + u * NT + tid;
                r[u] = Xb[(long long)(e / SW) * d + c0 + e % SW];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) strip[base + u * NT + tid] = r[u];
        }
    } else {
        for (int e = tid; e < n; e += NT) strip[e] = Xb[(long long)(e / SW) * d + c0 + e % SW];
    }
    __syncthreads();
    float2* Tb = T + (long long)i * d * d;
    for (; a < d; a += RPP) {
        int cc2[WP];
        float2 cv2[WP];
        const int a2 = a + 2 * RPP;
        if (a2 < d) obs_list<WP>(cols, vals, a2, cc2, cv2);
        float2 acc[CPL];
#pragma unroll
        for (int u = 0; u < CPL; ++u) acc[u] = make_float2(0.f, 0.f);
#pragma unroll
        for (int t = 0; t < WP; ++t) {
            const float2* src = strip + (long long)cc0[t] * SW + cp;
            if constexpr (CPL == 2) {
                const float4 x = *reinterpret_cast<const float4*>(src);
                cfma(acc[0], cv0[t], make_float2(x.x, x.y));
                cfma(acc[1], cv0[t], make_float2(x.z, x.w));
            } else {
                cfma(acc[0], cv0[t], src[0]);
            }
        }
        float2* dst = Tb + (long long)a * d + c0 + cp;
        if constexpr (CPL == 2)
            *reinterpret_cast<float4*>(dst) = make_float4(acc[0].x, acc[0].y, acc[1].x, acc[1].y);
        else
            dst[0] = acc[0];
#pragma unroll
        for (int t = 0; t < WP; ++t) {
            cc0[t] = cc1[t];
            cv0[t] = cv1[t];
            cc1[t] = cc2[t];
            cv1[t] = cv2[t];
        }
    }
}

// Pass 1 for 8-column strips: LPR lanes per row (1 when the strip has at least NT
// rows), each lane CPL = 8 / LPR columns, so one load instruction of a wave fetches
// the lists of 64 / LPR rows.  The strip's 16-byte chunks (two columns) are swizzled
// by row, chunk c of row a at position c ^ ((a >> 2) & 3) (mx8_off), so that the
// chunks 16 lanes of 16 neighbouring rows read fall into distinct banks.
template <int WP, int NT, int LPR>
__global__ __launch_bounds__(NT, NT / 128) void observable_mx8_kernel(int d, int b0, const float2* __restrict__ X0,
                                                                      const float2* __restrict__ X1, const int* loc,
                                                                      long long xstride, const int* __restrict__ cols,
                                                                      const float2* __restrict__ vals,
                                                                      const int* n_steps, int step, float2* T) {
    constexpr int SW = 8, CPL = SW / LPR, NCH = CPL / 2, RPP = NT / LPR;
    extern __shared__ float2 strip[];   // [d][8], 16-byte chunks swizzled (mx8_off)
    const int nstrip = d / SW;
    const long long bid = xcd_local(blockIdx.x, gridDim.x);
    const int i = (int)(bid / nstrip), sidx = (int)(bid % nstrip);
    const int b = b0 + i;
    if (n_steps && step >= n_steps[b]) return;      // uniform over the workgroup
    const float2* Xb = ((loc && loc[b]) ? X1 : X0) + (long long)b * xstride;
    const int c0 = sidx * SW;
    const int tid = threadIdx.x;
    const int n = d * SW;
    for (int base = 0; base < n; base += NT * 16) {
        float2 r[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = min(base + u * NT + tid, n - 1);
            r[u] = Xb[(long long)(e / SW) * d + c0 + e % SW];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = base + u * NT + tid;
            if (e < n) strip[mx8_off(e / SW, e % SW)] = r[u];
        }
    }
    __syncthreads();
    const float4* strip4 = reinterpret_cast<const float4*>(strip);
    const int lr = tid % LPR;
    int a = tid / LPR;
    float2* Tb = T + (long long)i * d * d;
    int cc[WP];
    float2 cv[WP];
    obs_list<WP>(cols, vals, min(a, d - 1), cc, cv);
    for (; a < d; a += RPP) {
        int nc[WP];
        float2 nv[WP];
        const int an = a + RPP;
        if (an < d) obs_list<WP>(cols, vals, an, nc, nv);
        float2 acc[CPL];
#pragma unroll
        for (int u = 0; u < CPL; ++u) acc[u] = make_float2(0.f, 0.f);
#pragma unroll
        for (int t = 0; t < WP; ++t) {
#pragma unroll
            for (int j = 0; j < NCH; ++j) {
                const int ch = lr * NCH + j;
                const float4 x = strip4[cc[t] * 4 + ((ch ^ (cc[t] >> 2)) & 3)];
                cfma(acc[2 * j], cv[t], make_float2(x.x, x.y));
                cfma(acc[2 * j + 1], cv[t], make_float2(x.z, x.w));
            }
        }
        float2* dst = Tb + (long long)a * d + c0 + lr * CPL;
#pragma unroll
        for (int j = 0; j < NCH; ++j)
            *reinterpret_cast<float4*>(dst + 2 * j) = make_float4(acc[2 * j].x, acc[2 * j].y, acc[2 * j + 1].x, acc[2 * j + 1].y);
        if (an < d) {
#pragma unroll
            for (int t = 0; t < WP; ++t) {
                cc[t] = nc[t];
                cv[t] = nv[t];
            }
        }
    }
}

// Pass 2.  R rows of X per workgroup, held column-major in LDS ([d][R]: the R
// entries of a column are one contiguous run, read as R/2 16-byte words);
// each lane takes columns c, c + NT, ...; the R entries of T and the row list
// of the next column are read while the current column is summed.
template <int R, int WP, int NT>
__global__ __launch_bounds__(NT, NT / 128) void observable_dot_kernel(int d, int b0, const float2* __restrict__ X0,
                                                            const float2* __restrict__ X1, const int* loc,
                                                            long long xstride, const int* __restrict__ cols,
                                                            const float2* __restrict__ vals, int w,
                                                            const int* n_steps, int step, const float2* __restrict__ T,
                                                            double* partial) {
    extern __shared__ float2 rowsT[];   // [d][R]
    __shared__ double red[NT];
    const int nrb = d / R;
    const long long bid = xcd_local(blockIdx.x, gridDim.x);
    const int i = (int)(bid / nrb), rb = (int)(bid % nrb);
    const int b = b0 + i;
    const int tid = threadIdx.x;
    const bool active = n_steps ? step < n_steps[b] : true;
    const float2* Xb = ((loc && loc[b]) ? X1 : X0) + (long long)b * xstride + (long long)rb * R * d;
    const float2* Tb = T + (long long)i * d * d + (long long)rb * R * d;
    double acc = 0.0;
    int c = tid;
    int cc[WP];
    float2 cv[WP], mx[R];
    if (active) {
        const int c_ = min(c, d - 1);
        obs_list<WP>(cols, vals, c_, cc, cv);
#pragma unroll
        for (int r = 0; r < R; ++r) mx[r] = Tb[(long long)r * d + c_];
        // rows rb R .. rb R + R - 1, R 16-byte loads in flight per lane and pass
        const float4* src = reinterpret_cast<const float4*>(Xb);
        const int half = d / 2;
        for (int cp = tid; cp < half; cp += NT) {
            float4 v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = src[(long long)r * half + cp];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                rowsT[(2 * cp) * R + r] = make_float2(v[r].x, v[r].y);
                rowsT[(2 * cp + 1) * R + r] = make_float2(v[r].z, v[r].w);
            }
        }
    }
    __syncthreads();
    if (active) {
        for (; c < d; c += NT) {
            const int cn = c + NT;
            int nc[WP];
            float2 nv[WP], nm[R];
            if (cn < d) {
                obs_list<WP>(cols, vals, cn, nc, nv);
#pragma unroll
                for (int r = 0; r < R; ++r) nm[r] = Tb[(long long)r * d + cn];
            }
            float2 xm[R];
#pragma unroll
            for (int r = 0; r < R; ++r) xm[r] = make_float2(0.f, 0.f);
#pragma unroll
            for (int t = 0; t < WP; ++t) {
                const float2 m = cconj(cv[t]);
                const float2* col = rowsT + (long long)cc[t] * R;
                if constexpr (R >= 2) {
#pragma unroll
                    for (int r = 0; r < R; r += 2) {
                        const float4 x = *reinterpret_cast<const float4*>(col + r);
                        cfma(xm[r], make_float2(x.x, x.y), m);
                        cfma(xm[r + 1], make_float2(x.z, x.w), m);
                    }
                } else {
                    cfma(xm[0], col[0], m);
                }
                asm volatile("" ::: "memory");   // one list entry's gathers at a time (register pressure)
            }
#pragma unroll
            for (int r = 0; r < R; ++r) acc += (double)xm[r].x * mx[r].x + (double)xm[r].y * mx[r].y;
            if (cn < d) {
#pragma unroll
                for (int t = 0; t < WP; ++t) {
                    cc[t] = nc[t];
                    cv[t] = nv[t];
                }
#pragma unroll
                for (int r = 0; r < R; ++r) mx[r] = nm[r];
            }
        }
    }
    red[tid] = acc;
    __syncthreads();
    for (int st = NT / 2; st > 0; st >>= 1) {
        if (tid < st) red[tid] += red[tid + st];
        __syncthreads();
    }
    if (tid == 0) partial[(long long)b * nrb + rb] = red[0];
}

// The right Walsh frame (observables M with M_ij = f(i XOR j)): with H the d x d
// Sylvester-Hadamard matrix, H_ij = (-1)^popcount(i & j), and Hn = H / sqrt(d) (orthogonal,
// Hn Hn = I), such an M is Hn D Hn with D = H f real and diagonal.  A state X is carried as
// W = X Hn: the chain's products act from the left and the Newton-Schulz re-projection
// commutes with the rotation, so both run on W unchanged, and
//     Tr(X M X^dag M) = Tr(W D W^dag M) = sum_j D_j w_j^dag M w_j
// over the columns w_j of W: one pass over W with no intermediate M X.

// W_0 = Hn: the identity in the right Walsh frame
__global__ void walsh_fill_kernel(long long nn, int d, int B, float2* X, long long stride, float s) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn * B;
         e += (long long)gridDim.x * blockDim.x) {
        const long long b = e / nn, ij = e % nn;
        const int i = (int)(ij / d), j = (int)(ij % d);
        X[b * stride + ij] = make_float2((__popc(i & j) & 1) ? -s : s, 0.f);
    }
}

// In place X <- X Hn for a batch of d x d matrices (its own inverse), one wave per row:
// lane l holds the E = d / 64 consecutive entries l E .. l E + E - 1; the butterflies of
// the low log2(E) index bits run in registers, those of the six lane bits through xor
// shuffles.  rows = B d.
template <int E>
__global__ __launch_bounds__(256) void walsh_right_kernel(int d, long long rows, float2* X, long long stride,
                                                          float s) {
    const long long row = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= rows) return;   // a whole wave
    const int lane = threadIdx.x & 63;
    const long long b = row / d, i = row % d;
    float4* p = reinterpret_cast<float4*>(X + b * stride + i * d + (long long)lane * E);
    float2 v[E];
#pragma unroll
    for (int u = 0; u < E / 2; ++u) {
        const float4 q = p[u];
        v[2 * u] = make_float2(q.x, q.y);
        v[2 * u + 1] = make_float2(q.z, q.w);
    }
#pragma unroll
    for (int h = 1; h < E; h <<= 1)
#pragma unroll
        for (int k = 0; k < E; ++k)
            if (!(k & h)) {
                const float2 a = v[k], c = v[k + h];
                v[k] = make_float2(a.x + c.x, a.y + c.y);
                v[k + h] = make_float2(a.x - c.x, a.y - c.y);
            }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const bool upper = (lane & m) != 0;
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const float ox = __shfl_xor(v[k].x, m), oy = __shfl_xor(v[k].y, m);
            v[k] = upper ? make_float2(ox - v[k].x, oy - v[k].y) : make_float2(v[k].x + ox, v[k].y + oy);
        }
    }
#pragma unroll
    for (int u = 0; u < E / 2; ++u)
        p[u] = make_float4(s * v[2 * u].x, s * v[2 * u].y, s * v[2 * u + 1].x, s * v[2 * u + 1].y);
}

// row of element e of an 8-column strip (column e % 8).  With whole-row lanes (LPR = 1) the
// 80-byte rows of 8 consecutive e go to rows r and r + 4 by turns within each block of 8 rows:
// an 8-byte store serves 16 lanes per pass over 32 banks, and rows 4 apart start 16 banks
// apart, so each pass writes 32 distinct banks (neighbouring rows would share 4)
template <int LPR>
__device__ inline int strip_row(int e) {
    if constexpr (LPR == 1) {
        const int s = (e >> 3) & 7;
        return ((e >> 6) << 3) | ((s & 1) << 2) | (s >> 1);
    } else {
        return e >> 3;
    }
}

// The observable in the right Walsh frame, one pass: the 8-column strip of W in LDS (as
// observable_mx8_kernel).  The frame needs M_ac = f(a XOR c) with f real, so row a's list is
// row 0's with every column XORed by a: the masks m and values f(m) are read once from row 0
// (one address for every lane; zero entries, the padding among them, skipped) and
//     w_j^dag M w_j = f(0) sum_a |W_aj|^2 + sum_{m != 0} 2 f(m) sum_{a < a^m} Re(conj(W_aj) W_{a^m, j}),
// each unordered pair once: the rows with a zero at the top bit of m, a = the pair index with
// that zero inserted.  LPR lanes share a pair (8 / LPR columns each); a lane's column sums
// stay in FP32 over its pairs and masks, then D_j weights them and the workgroup sum runs in
// FP64 to partial[b][strip].
template <int WP, int NT, int LPR>
__global__ __launch_bounds__(NT, NT / 128) void observable_walsh_kernel(int d, int b0, const float2* __restrict__ X0,
                                                                        const float2* __restrict__ X1, const int* loc,
                                                                        long long xstride,
                                                                        const int* __restrict__ cols,
                                                                        const float2* __restrict__ vals,
                                                                        const double* __restrict__ spec,
                                                                        const int* n_steps, int step,
                                                                        double* partial) {
    constexpr int SW = 8, CPL = SW / LPR, NCH = CPL / 2, RPP = NT / LPR;
    // LPR = 1: rows of 10 float2 (80 bytes: the 16 rows that one pass of 16-byte reads covers
    // start 20 banks apart, all distinct, so lanes read the same chunk position of their rows
    // without conflicts, at fixed offsets); else [d][8] with swizzled 16-byte chunks (mx8_off)
    constexpr int RS = LPR == 1 ? 10 : 8;
    extern __shared__ float2 strip[];   // then, LPR > 1, NT doubles for the reduction
    const int nstrip = d / SW;
    const long long bid = xcd_local(blockIdx.x, gridDim.x);
    const int i = (int)(bid / nstrip), sidx = (int)(bid % nstrip);
    const int b = b0 + i;
    if (n_steps && step >= n_steps[b]) return;      // uniform over the workgroup
    const float2* Xb = ((loc && loc[b]) ? X1 : X0) + (long long)b * xstride;
    const int c0 = sidx * SW;
    const int tid = threadIdx.x;
    const int n = d * SW;
    for (int base = 0; base < n; base += NT * 16) {
        float2 r[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = min(base + u * NT + tid, n - 1);
            r[u] = Xb[(long long)strip_row<LPR>(e) * d + c0 + e % SW];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = base + u * NT + tid;
            if (e < n) {
                if constexpr (LPR == 1)
                    strip[strip_row<LPR>(e) * RS + e % SW] = r[u];
                else
                    strip[mx8_off(e / SW, e % SW)] = r[u];
            }
        }
    }
    __syncthreads();
    const float4* strip4 = reinterpret_cast<const float4*>(strip);
    const int lr = tid % LPR;
    float dj[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) dj[u] = (float)spec[c0 + lr * CPL + u];
    int mk[WP];
    float2 fv[WP];
    obs_list<WP>(cols, vals, 0, mk, fv);
    // the lane's NCH 16-byte chunks of row a: columns lr * CPL .. lr * CPL + CPL - 1
    auto chunk = [&](int a, int j) { return strip4[a * 4 + (((lr * NCH + j) ^ (a >> 2)) & 3)]; };
    float acc[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) acc[u] = 0.f;
#pragma unroll
    for (int t = 0; t < WP; ++t) {
        if (fv[t].x == 0.f && fv[t].y == 0.f) continue;   // the same for every lane
        const int m = mk[t];
        float sm[CPL];
#pragma unroll
        for (int u = 0; u < CPL; ++u) sm[u] = 0.f;
        if constexpr (LPR == 1) {
            // a lane owns whole rows: chunk j of row a at fixed offset j of its 80-byte row
            if (m == 0) {
                for (int a = tid; a < d; a += NT) {
                    const float4* xa = strip4 + a * (RS / 2);
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float4 x = xa[j];
                        sm[2 * j] = fmaf(x.x, x.x, fmaf(x.y, x.y, sm[2 * j]));
                        sm[2 * j + 1] = fmaf(x.z, x.z, fmaf(x.w, x.w, sm[2 * j + 1]));
                    }
                }
#pragma unroll
                for (int u = 0; u < CPL; ++u) acc[u] = fmaf(fv[t].x, sm[u], acc[u]);
            } else {
                const int top = 31 - __clz(m);
                const int low = (1 << top) - 1;
                // a 16-byte read serves 16 lanes per pass over 64 banks, and row a starts at
                // bank 20 a mod 64, a function of a mod 16: 16 lanes of consecutive pairs take
                // 16 residues when top >= 4, but only the 8 with bit top clear when top < 4;
                // lanes 8..15 of each 16 then start from the partner row a ^ m (the pair's
                // product is symmetric in its rows, so the sums are the same bit for bit)
                const int flip = (top < 4 && (tid & 8)) ? m : 0;
                for (int pr = tid; pr < d / 2; pr += NT) {
                    const int a = (((pr & ~low) << 1) | (pr & low)) ^ flip;
                    const float4* xa = strip4 + a * (RS / 2);
                    const float4* yc = strip4 + (a ^ m) * (RS / 2);
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float4 x = xa[j], y = yc[j];
                        sm[2 * j] = fmaf(x.x, y.x, fmaf(x.y, y.y, sm[2 * j]));
                        sm[2 * j + 1] = fmaf(x.z, y.z, fmaf(x.w, y.w, sm[2 * j + 1]));
                    }
                }
#pragma unroll
                for (int u = 0; u < CPL; ++u) acc[u] = fmaf(2.f * fv[t].x, sm[u], acc[u]);
            }
        } else if (m == 0) {
            for (int a = tid / LPR; a < d; a += RPP) {
#pragma unroll
                for (int j = 0; j < NCH; ++j) {
                    const float4 x = chunk(a, j);
                    sm[2 * j] = fmaf(x.x, x.x, fmaf(x.y, x.y, sm[2 * j]));
                    sm[2 * j + 1] = fmaf(x.z, x.z, fmaf(x.w, x.w, sm[2 * j + 1]));
                }
            }
#pragma unroll
            for (int u = 0; u < CPL; ++u) acc[u] = fmaf(fv[t].x, sm[u], acc[u]);
        } else {
            const int top = 31 - __clz(m);
            const int low = (1 << top) - 1;
            for (int pr = tid / LPR; pr < d / 2; pr += RPP) {
                const int a = ((pr & ~low) << 1) | (pr & low);
                const int c = a ^ m;
#pragma unroll
                for (int j = 0; j < NCH; ++j) {
                    const float4 x = chunk(a, j), y = chunk(c, j);
                    sm[2 * j] = fmaf(x.x, y.x, fmaf(x.y, y.y, sm[2 * j]));
                    sm[2 * j + 1] = fmaf(x.z, y.z, fmaf(x.w, y.w, sm[2 * j + 1]));
                }
            }
#pragma unroll
            for (int u = 0; u < CPL; ++u) acc[u] = fmaf(2.f * fv[t].x, sm[u], acc[u]);
        }
    }
    double sum = 0.0;
#pragma unroll
    for (int u = 0; u < CPL; ++u) sum += (double)dj[u] * (double)acc[u];
    // the reduction after the strip (LPR > 1), or in the strip's own memory once every lane is
    // done with it (LPR = 1: two 80 KiB workgroups per CU leave no room beside it)
    double* red = reinterpret_cast<double*>(strip + (LPR == 1 ? 0 : RS * d));
    if constexpr (LPR == 1) __syncthreads();
    red[tid] = sum;
    __syncthreads();
    for (int st = NT / 2; st > 0; st >>= 1) {
        if (tid < st) red[tid] += red[tid + st];
        __syncthreads();
    }
    if (tid == 0) partial[(long long)b * nstrip + sidx] = red[0];
}

__global__ void observable_final_kernel(int nparts, const double* partial, const float2* vals, int nvals,
                                        const int* n_steps, int step, double* out, long long out_stride) {
    const int b = blockIdx.x;
    __shared__ double red[256];
    double s = 0.0, m2 = 0.0;
    for (int e = threadIdx.x; e < nparts; e += 256) s += partial[(long long)b * nparts + e];
    for (int e = threadIdx.x; e < nvals; e += 256) m2 += (double)vals[e].x * vals[e].x + (double)vals[e].y * vals[e].y;
    red[threadIdx.x] = s;
    __syncthreads();
    for (int t = 128; t > 0; t >>= 1) {
        if ((int)threadIdx.x < t) red[threadIdx.x] += red[threadIdx.x + t];
        __syncthreads();
    }
    const double tot = red[0];
    __syncthreads();
    red[threadIdx.x] = m2;
    __syncthreads();
    for (int t = 128; t > 0; t >>= 1) {
        if ((int)threadIdx.x < t) red[threadIdx.x] += red[threadIdx.x + t];
        __syncthreads();
    }
    const bool active = n_steps ? step < n_steps[b] : true;
    if (threadIdx.x == 0 && active) out[(long long)b * out_stride] = tot / red[0];
}

// GRAPE traces of Y = X_{s+1} L_{s+1} for every channel k:
//   T1 = Tr(S^psi Y) with psi = phi (q != 0) or 0 (q == 0), S^psi_ab = e^{-i psi (g_a - g_b)} S_ab
//   T2 = Tr(S^{pi/2} Y) (phased, q == 0 only), Dg = Tr(G Y)
// Tile (32 x 32 of (a, b)) partial sums; block (tile, k, b).
constexpr int TT = 32;
__global__ __launch_bounds__(256) void trace_partial_kernel(int d, int K, int phased, const float2* __restrict__ Y,
                                                            long long ystride, const float2* __restrict__ S,
                                                            const double* __restrict__ g,
                                                            const int* __restrict__ codes,
                                                            const double* __restrict__ phi, long long code_stride,
                                                            const int* n_steps, int step, double* partial,
                                                            int cartesian, const double* h, int n_drift,
                                                            double hdt) {
    const int ntile = (d / TT) * (d / TT);
    const int tile = blockIdx.x, k = blockIdx.y, b = blockIdx.z;
    const int a0 = (tile / (d / TT)) * TT, b0 = (tile % (d / TT)) * TT;
    __shared__ float2 Ys[TT][TT + 1];  // Ys[bb][aa] = Y[b0 + bb][a0 + aa]
    __shared__ double2 pa[TT], pb[TT], qa[TT], qb[TT];
    __shared__ double red[6][256];
    const bool active = n_steps ? step < n_steps[b] : true;
    const float2* Yb = Y + (long long)b * ystride;
    int q = 0;
    double ph = 0.0;
    if (active) {
        q = codes[(long long)b * code_stride + k];
        if (phased) ph = phi[(long long)b * code_stride + k];
    }
    const bool origin = phased && (q == 0 || cartesian);
    const double psi = phased && !origin ? ph : 0.0;
    for (int e = threadIdx.x; e < TT * TT; e += 256) {
        const int bb = e / TT, aa = e % TT;
        Ys[bb][aa] = active ? Yb[(long long)(b0 + bb) * d + a0 + aa] : make_float2(0.f, 0.f);
    }
    if (threadIdx.x < TT) {
        const int r = threadIdx.x;
        const double ga = phased ? g[(long long)k * d + a0 + r] : 0.0, gb = phased ? g[(long long)k * d + b0 + r] : 0.0;
        pa[r] = expmi(psi * ga);                    // e^{-i psi g_a}
        pb[r] = zconj(expmi(psi * gb));             // e^{+i psi g_b}
        qa[r] = expmi(1.5707963267948966 * ga);
        qb[r] = zconj(expmi(1.5707963267948966 * gb));
        if (hdt != 0.0) {
            // Strang: the generator seen by the trace is V(dt/2) S V(dt/2)^dag
            const long long hb_ = (long long)(b % n_drift) * d;
            const double2 ea = expmi(hdt * h[hb_ + a0 + r]), eb = zconj(expmi(hdt * h[hb_ + b0 + r]));
            pa[r] = zmul(pa[r], ea);
            pb[r] = zmul(pb[r], eb);
            qa[r] = zmul(qa[r], ea);
            qb[r] = zmul(qb[r], eb);
        }
    }
    __syncthreads();
    double t1r = 0, t1i = 0, t2r = 0, t2i = 0, dr = 0, di = 0;
    for (int e = threadIdx.x; e < TT * TT; e += 256) {
        const int aa = e / TT, bb = e % TT;  // S[a][b] coalesced along b
        const float2 sv = S[(long long)k * d * d + (long long)(a0 + aa) * d + b0 + bb];
        const float2 y = Ys[bb][aa];
        const double yr = y.x, yi = y.y;
        double sr = sv.x, si = sv.y;
        if (phased || hdt != 0.0) {
            const double2 p = zmul(pa[aa], pb[bb]);
            const double r_ = p.x * sr - p.y * si, i_ = p.x * si + p.y * sr;
            sr = r_;
            si = i_;
        }
        t1r += sr * yr - si * yi;
        t1i += sr * yi + si * yr;
        if (origin) {
            const double2 p = zmul(qa[aa], qb[bb]);
            const double r_ = p.x * sv.x - p.y * sv.y, i_ = p.x * sv.y + p.y * sv.x;
            t2r += r_ * yr - i_ * yi;
            t2i += r_ * yi + i_ * yr;
        }
        if (phased && a0 + aa == b0 + bb) {
            const double ga = g[(long long)k * d + a0 + aa];
            dr += ga * yr;
            di += ga * yi;
        }
    }
    double v[6] = {t1r, t1i, t2r, t2i, dr, di};
#pragma unroll
    for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int c = 0; c < 6; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 6) partial[(((long long)b * K + k) * ntile + tile) * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// sums the tile partials: out[b][k][0..5] (T1 re/im, T2 re/im, D re/im)
__global__ void trace_final_kernel(int ntile, int K, const double* partial, double* out, long long out_bstride) {
    const int k = blockIdx.y, b = blockIdx.x;
    __shared__ double red[6][64];
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int t = threadIdx.x; t < ntile; t += 64)
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] += partial[(((long long)b * K + k) * ntile + t) * 6 + c];
#pragma unroll
    for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int s = 32; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int c = 0; c < 6; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 6) out[(long long)b * out_bstride + k * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// Contribution of one pattern entry to the traces of channel k: entry (a, j) of S_k
// (is_diag false, slot e of row a) or the diagonal (is_diag, for D), with
// y = Y[j][a]: T1 += S^psi_aj y, T2 += S^{pi/2}_aj y (origin), D += g_a y, where
// S^psi_aj = exp(-i psi (g_a - g_j)) S_aj, times exp(-i dt/2 (h_a - h_j)) with the
// Strang splitting (hdt != 0).
struct SptChannel {
    bool origin;     // phased with q = 0, or Cartesian: also T2
    double psi;      // phase of the step (0 unless phased and not at the origin)
};

__device__ inline SptChannel spt_channel(int phased, int cartesian, const int* codes, const double* phi, long long ci) {
    SptChannel c;
    const int q = codes[ci];
    c.origin = phased && (q == 0 || cartesian);
    c.psi = phased && !c.origin ? phi[ci] : 0.0;
    return c;
}

__device__ inline void spt_contrib(double v[6], bool is_diag, int phased, const SptChannel& ch, int d, int k, int a,
                                   int j, int e, int sw, double yr, double yi, const double2* __restrict__ spv,
                                   const double* __restrict__ g, const double* __restrict__ h, long long hb,
                                   double hdt) {
    if (!is_diag) {
        double2 sv = spv[((long long)k * d + a) * sw + e];
        if (hdt != 0.0) sv = zmul(expmi(hdt * (h[hb + a] - h[hb + j])), sv);   // V(dt/2) S V(dt/2)^dag
        double cr = sv.x, cim = sv.y;
        if (phased && ch.psi != 0.0) {
            const double2 p = expmi(ch.psi * (g[(long long)k * d + a] - g[(long long)k * d + j]));
            cr = p.x * sv.x - p.y * sv.y;
            cim = p.x * sv.y + p.y * sv.x;
        }
        v[0] += cr * yr - cim * yi;
        v[1] += cr * yi + cim * yr;
        if (ch.origin) {
            const double2 p = expmi(1.5707963267948966 * (g[(long long)k * d + a] - g[(long long)k * d + j]));
            const double r_ = p.x * sv.x - p.y * sv.y, i_ = p.x * sv.y + p.y * sv.x;
            v[2] += r_ * yr - i_ * yi;
            v[3] += r_ * yi + i_ * yr;
        }
    } else if (phased) {
        const double ga = g[(long long)k * d + a];
        v[4] += ga * yr;
        v[5] += ga * yi;
    }
}

// GRAPE traces from stored factors, for generators with a sparse pattern:
// Y = X_{s+1} L_{s+1} is needed only where S_k^T (and the diagonal) is
// nonzero, and L = LH^H is stored conjugate-transposed so that both operands
// of Y[j][a] = sum_c X[j][c] conj(LH[a][c]) are contiguous rows.  One wave per
// row a (SPT_RPB rows per workgroup); the dot products accumulate in FP64.
// For every channel k the row's share of T1 = Tr(S^psi Y), T2 = Tr(S^{pi/2} Y)
// (phased, q = 0 or Cartesian) and D = Tr(G Y) goes to partial[(b N + s)][k][blk][6]
// (s counted from step0).
// Workgroups are dealt to the 8 XCDs, each with its own L2, in turn by linear index; the
// index is remapped so that every row block of one step runs on the same XCD (step = XCD
// mod 8), whose L2 then serves the rows of X_s that the step's row blocks share, instead
// of every XCD pulling the whole state.  grid.x = (d / SPT_RPB) * (steps rounded up to a
// multiple of 8), grid.y = B.
constexpr int SPT_RPB = 4;
constexpr int SPT_XCD = 8;
template <int WP>
__global__ __launch_bounds__(256) void sparse_trace_kernel(int d, int N, int step0, int nsl, int K, int phased,
                                                           int cartesian,
                                                           int sw, const float2* __restrict__ X, long long xsb,
                                                           const float2* __restrict__ LH, long long lsb,
                                                           const int* __restrict__ spc,
                                                           const double2* __restrict__ spv,
                                                           const double* __restrict__ g,
                                                           const int* __restrict__ codes,
                                                           const double* __restrict__ phi, const int* n_steps,
                                                           double* partial, const double* __restrict__ h,
                                                           int n_drift, double hdt) {
    constexpr int NE = WP + 1;                      // pattern entries + the diagonal
    __shared__ double red[SPT_RPB][NE][6];
    const int nblk = d / SPT_RPB;
    const int xcd = (int)blockIdx.x % SPT_XCD, on_xcd = (int)blockIdx.x / SPT_XCD;
    const int blk = on_xcd % nblk, sl = (on_xcd / nblk) * SPT_XCD + xcd, b = blockIdx.y;
    if (sl >= nsl) return;   // padding of the step count to a multiple of 8
    const int s = step0 + sl;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int a = blk * SPT_RPB + wave;
    const long long mat = (long long)d * d;
    const bool active = (!n_steps || s < n_steps[b]) && s < N;
    double yr[NE], yi[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) yr[e] = yi[e] = 0.0;
    int jt[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) jt[e] = e < sw ? spc[(long long)a * sw + e] : a;
    if (active) {
        const float2* Xs = X + (long long)b * xsb + (long long)s * mat;
        const float2* Lr = LH + (long long)b * lsb + (long long)(s + 1) * mat + (long long)a * d;
        for (int c0 = 0; c0 < d; c0 += 64 * 8) {
            float2 l[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int c = c0 + lane + 64 * u;
                l[u] = c < d ? Lr[c] : make_float2(0.f, 0.f);
            }
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                if (e < sw || e == WP) {
                    const float2* xr = Xs + (long long)jt[e] * d;
                    float2 x[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int c = c0 + lane + 64 * u;
                        x[u] = c < d ? xr[c] : make_float2(0.f, 0.f);
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        // x conj(l)
                        yr[e] += (double)x[u].x * l[u].x + (double)x[u].y * l[u].y;
                        yi[e] += (double)x[u].y * l[u].x - (double)x[u].x * l[u].y;
                    }
                }
                asm volatile("" ::: "memory");   // one row's loads in flight at a time (register pressure)
            }
        }
#pragma unroll
        for (int e = 0; e < NE; ++e)
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                yr[e] += __shfl_xor(yr[e], o);
                yi[e] += __shfl_xor(yi[e], o);
            }
    }
    // lane e (< sw) owns pattern entry e, lane WP the diagonal
    double my_r = 0.0, my_i = 0.0;
    int my_j = a;
#pragma unroll
    for (int e = 0; e < NE; ++e)
        if (lane == e) {
            my_r = yr[e];
            my_i = yi[e];
            my_j = jt[e];
        }
    const bool mine = active && (lane < sw || lane == WP);
    for (int k = 0; k < K; ++k) {
        double v[6] = {0, 0, 0, 0, 0, 0};
        if (mine)
            spt_contrib(v, lane == WP, phased, spt_channel(phased, cartesian, codes, phi, ((long long)b * N + s) * K + k),
                        d, k, a, my_j, lane, sw, my_r, my_i, spv, g, h, (long long)(b % n_drift) * d, hdt);
        if (lane < NE)
#pragma unroll
            for (int c = 0; c < 6; ++c) red[wave][lane][c] = v[c];
        __syncthreads();
        if (threadIdx.x < 6) {
            double acc = 0.0;
            for (int w2 = 0; w2 < SPT_RPB; ++w2)
                for (int e = 0; e < NE; ++e) acc += red[w2][e][threadIdx.x];
            partial[((((long long)b * nsl + sl) * K + k) * nblk + blk) * 6 + threadIdx.x] = acc;
        }
        __syncthreads();
    }
}

// The same traces for d <= 1024 in two kernels.  sparse_y_kernel: one workgroup per
// (instance, step), each thread owning SPS_RPT rows a (a0 and a0 + d / 2); X_s passes
// through LDS in chunks of SPS_C columns, stored [c][row] so that the lanes of a wave,
// which read rows of the pattern of consecutive rows, hit consecutive addresses; the
// thread's rows of LH_(s+1) come straight to its registers, and each thread accumulates
// its rows' entries Y[j][a] = sum_c X[j][c] conj(LH[a][c]) in FP64 with no partial sums
// across lanes, then stores them to ybuf[b][s][a][slot].  Every element of X_s and
// LH_(s+1) is read from memory once.  sparse_ysum_kernel weighs the entries per channel
// (the FP64 phase factors, which would crowd the accumulators out of registers) and sums
// the workgroup into tr[b][s][k][6].
constexpr int SPS_C = 8;
constexpr int SPS_RPT = 2;
constexpr int SPS_DMAX = 1024;
constexpr int SPS_NT = SPS_DMAX / SPS_RPT;
constexpr int SPS_NE = SPAT_WMAX + 1;   // slots per row in ybuf
template <int WP>
__global__ __launch_bounds__(SPS_NT) void sparse_y_kernel(int d, int N, int step0, int steps, int sw,
                                                          const float2* __restrict__ X, long long xsb,
                                                          const float2* __restrict__ LH, long long lsb,
                                                          const int* __restrict__ spc, const int* n_steps,
                                                          double2* __restrict__ ybuf) {
    constexpr int NE = WP + 1;                      // pattern slots + the diagonal
    // [SPS_C][SPS_DMAX]: a fixed row stride, so that each column's offset is an immediate of
    // the LDS reads (with d as the stride their addresses would have to sit in registers)
    __shared__ float2 xs[SPS_C * SPS_DMAX];
    const int sl = blockIdx.x, b = blockIdx.y, s = step0 + sl;
    const int t = threadIdx.x, nt = d / SPS_RPT;
    if (!((!n_steps || s < n_steps[b]) && s < N)) return;   // the same for the whole workgroup
    const long long mat = (long long)d * d;
    double yr[SPS_RPT][NE], yi[SPS_RPT][NE];
    int jt[SPS_RPT][NE];
#pragma unroll
    for (int r = 0; r < SPS_RPT; ++r) {
        const int a = t + r * nt;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            yr[r][e] = yi[r][e] = 0.0;
            // slots past the pattern width (and the diagonal slot WP): row a
            jt[r][e] = e < sw ? spc[(long long)a * sw + e] : a;
        }
    }
    const float2* Xs = X + (long long)b * xsb + (long long)s * mat;
    const float2* L0 = LH + (long long)b * lsb + (long long)(s + 1) * mat;
    for (int c0 = 0; c0 < d; c0 += SPS_C) {
        __syncthreads();   // the previous chunk is consumed
        // each thread stages the chunk of its own rows of X_s and keeps that of LH_(s+1): all
        // loads in flight at once
        float4 v[SPS_RPT][SPS_C / 2], l[SPS_RPT][SPS_C / 2];
#pragma unroll
        for (int r = 0; r < SPS_RPT; ++r)
#pragma unroll
            for (int u = 0; u < SPS_C / 2; ++u) {
                v[r][u] = *reinterpret_cast<const float4*>(Xs + (long long)(t + r * nt) * d + c0 + 2 * u);
                l[r][u] = *reinterpret_cast<const float4*>(L0 + (long long)(t + r * nt) * d + c0 + 2 * u);
            }
#pragma unroll
        for (int r = 0; r < SPS_RPT; ++r)
#pragma unroll
            for (int u = 0; u < SPS_C / 2; ++u) {
                xs[(2 * u) * SPS_DMAX + t + r * nt] = make_float2(v[r][u].x, v[r][u].y);
                xs[(2 * u + 1) * SPS_DMAX + t + r * nt] = make_float2(v[r][u].z, v[r][u].w);
            }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < SPS_C; ++c) {
#pragma unroll
            for (int r = 0; r < SPS_RPT; ++r) {
                const double lr = (c & 1) ? l[r][c / 2].z : l[r][c / 2].x;
                const double li = (c & 1) ? l[r][c / 2].w : l[r][c / 2].y;
                // every slot, the padding ones included: no branches in the loop
#pragma unroll
                for (int e = 0; e < NE; ++e) {
                    const float2 x = xs[c * SPS_DMAX + jt[r][e]];
                    const double xr = x.x, xi = x.y;
                    // x conj(l) as four FP64 FMAs
                    yr[r][e] = fma(xr, lr, fma(xi, li, yr[r][e]));
                    yi[r][e] = fma(xi, lr, fma(-xr, li, yi[r][e]));
                }
            }
            asm volatile("" ::: "memory");   // one column's LDS reads in flight at a time (register pressure)
        }
    }
    double2* yo = ybuf + ((long long)b * steps + sl) * d * SPS_NE;
#pragma unroll
    for (int r = 0; r < SPS_RPT; ++r)
#pragma unroll
        for (int e = 0; e < NE; ++e)
            if (e < sw || e == WP) yo[(long long)(t + r * nt) * SPS_NE + (e == WP ? SPAT_WMAX : e)] =
                                       make_double2(yr[r][e], yi[r][e]);
}

// one workgroup of 256 per (instance, step): weights of the entries in ybuf (slot e < sw
// of row a: entry (a, spc[a][e]); slot SPAT_WMAX: the diagonal) per channel, summed
__global__ __launch_bounds__(256) void sparse_ysum_kernel(int d, int N, int step0, int steps, int K, int phased,
                                                          int cartesian, int sw, const double2* __restrict__ ybuf,
                                                          const int* __restrict__ spc,
                                                          const double2* __restrict__ spv,
                                                          const double* __restrict__ g,
                                                          const int* __restrict__ codes,
                                                          const double* __restrict__ phi, const int* n_steps,
                                                          double* __restrict__ tr, const double* __restrict__ h,
                                                          int n_drift, double hdt) {
    __shared__ double red[4][6];
    const int sl = blockIdx.x, b = blockIdx.y, s = step0 + sl;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    double* out = tr + ((long long)b * N + s) * K * 6;
    if (!((!n_steps || s < n_steps[b]) && s < N)) {
        for (int i = t; i < K * 6; i += 256) out[i] = 0.0;
        return;
    }
    const double2* yb = ybuf + ((long long)b * steps + sl) * d * SPS_NE;
    const long long hb = (long long)(b % n_drift) * d;
    for (int k = 0; k < K; ++k) {
        const SptChannel ch = spt_channel(phased, cartesian, codes, phi, ((long long)b * N + s) * K + k);
        double v[6] = {0, 0, 0, 0, 0, 0};
        for (int a = t; a < d; a += 256) {
            for (int e = 0; e < sw; ++e) {
                const double2 y = yb[(long long)a * SPS_NE + e];
                spt_contrib(v, false, phased, ch, d, k, a, spc[(long long)a * sw + e], e, sw, y.x, y.y, spv, g, h,
                            hb, hdt);
            }
            if (phased) {
                const double2 y = yb[(long long)a * SPS_NE + SPAT_WMAX];
                spt_contrib(v, true, phased, ch, d, k, a, a, 0, sw, y.x, y.y, spv, g, h, hb, hdt);
            }
        }
#pragma unroll
        for (int c = 0; c < 6; ++c)
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v[c] += __shfl_xor(v[c], o);
        if (lane == 0)
#pragma unroll
            for (int c = 0; c < 6; ++c) red[wave][c] = v[c];
        __syncthreads();
        if (t < 6) out[k * 6 + t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
        __syncthreads();
    }
}

// gradient assembly for every (b, s, k):
//   tr[b][s][k][6]: traces of Y_{s+1}; dm[b][m][k][2]: Tr(G Y_m) for m = 0 .. N (from tr and D_0)
__global__ void grad_kernel(int B, int N, int K, int phased, double eps, double dt, const int* codes,
                            const double* phi, const double* tr, const double* d0, const double2* overlap,
                            const double* nu, const int* n_steps, float* grad, int cartesian) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)B * N * K) return;
    const int k = (int)(e % K);
    const int s = (int)((e / K) % N);
    const int b = (int)(e / ((long long)K * N));
    const int len = n_steps ? n_steps[b] : N;
    const int KK = phased ? 2 : 1;
    float* gp = grad + e * KK;
    if (s >= len) {
        gp[0] = 0.f;
        if (phased) gp[1] = 0.f;
        return;
    }
    const double gr = overlap[b].x, gi = overlap[b].y;
    const double scale = 2.0 / nu[b];
    auto im_gc = [&](double zr, double zi) { return gr * zi - gi * zr; };
    const double* t = tr + e * 6;
    const int q = codes[e];
    if (!phased) {
        gp[0] = (float)(scale * dt * im_gc(t[0], t[1]));
        return;
    }
    if (q == 0 || cartesian) {
        gp[0] = (float)(scale * dt * im_gc(t[0], t[1]));
        gp[1] = (float)(scale * dt * im_gc(t[2], t[3]));
        return;
    }
    // D of Y_s: from the traces of step s-1 (its D is of Y_s), or D_0
    double Dr, Di;
    if (s == 0) {
        Dr = d0[((long long)b * K + k) * 2];
        Di = d0[((long long)b * K + k) * 2 + 1];
    } else {
        const double* tp = tr + (e - K) * 6;
        Dr = tp[4];
        Di = tp[5];
    }
    const double om = q * eps;
    const double dFo = scale * dt * im_gc(t[0], t[1]);
    const double dFp = scale * im_gc(t[4] - Dr, t[5] - Di);
    const double p = phi[e];
    const double cp = cos(p), sp = sin(p);
    gp[0] = (float)(cp * dFo - sp * dFp / om);
    gp[1] = (float)(sp * dFo + cp * dFp / om);
}

// D_0 = Tr(G_k L_0) per instance and channel, plus nu = Tr(U_f^dag U_f)
__global__ void d0_kernel(int d, int K, int phased, const float2* L, long long lstride, const double* g, double* d0,
                          int conj_l) {
    const int b = blockIdx.x, k = blockIdx.y;
    __shared__ double rr[256], ri[256];
    double sr = 0, si = 0;
    if (phased)
        for (int a = threadIdx.x; a < d; a += 256) {
            const float2 v = L[(long long)b * lstride + (long long)a * d + a];
            sr += g[(long long)k * d + a] * v.x;
            si += g[(long long)k * d + a] * (conj_l ? -v.y : v.y);
        }
    rr[threadIdx.x] = sr;
    ri[threadIdx.x] = si;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            rr[threadIdx.x] += rr[threadIdx.x + s];
            ri[threadIdx.x] += ri[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        d0[((long long)b * K + k) * 2] = rr[0];
        d0[((long long)b * K + k) * 2 + 1] = ri[0];
    }
}

__global__ void identity_kernel(long long nn, int d, int B, float2* X, long long stride) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn * B;
         e += (long long)gridDim.x * blockDim.x) {
        const long long b = e / nn, r = e % nn;
        X[b * stride + r] = make_float2((r / d) == (r % d) ? 1.f : 0.f, 0.f);
    }
}

}  // namespace

hipError_t plan_step(const PlanLaunch& p, hipStream_t st) {
    PlanArgs a;
    a.T = p.T;
    a.V = p.V;
    a.h = p.h;
    a.g = p.g;
    a.cache = p.cache;
    a.codes = p.codes;
    a.phi = p.phi;
    a.n_steps = p.n_steps;
    a.ent = p.ent;
    a.code_stride = p.code_stride;
    a.d = p.d;
    a.K = p.K;
    a.P = p.P;
    a.base = p.base;
    a.n_drift = p.n_drift;
    a.phased = p.phased;
    a.dense = p.dense;
    a.strang = p.strang;
    a.cache_lo = p.cache_lo;
    a.cache_hi = p.cache_hi;
    a.cache_levels = p.cache_hi - p.cache_lo + 1;
    a.step = p.step;
    a.drift_div = p.drift_div;
    a.drift_offset = p.drift_offset;
    a.dt = p.dt;
    a.X[0] = p.X0;
    a.X[1] = p.X1;
    a.xstride = p.xstride;
    a.loc = p.loc;
    a.compose = p.compose;
    a.slots = p.slots;
    a.all_cached = p.all_cached;
    a.cache_bf = p.cache_bf;
    a.bf_conj = p.bf_conj;
    a.pre = p.pre;
    a.post = p.post;
    a.pstar = p.pstar;
    a.descs = p.descs;
    a.B = p.B;
    if (a.slots > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(plan_step_kernel, dim3(p.B), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t reproject_descs(GemmDesc* descs, int count, int b0, float2* X0, float2* X1, long long xstride, float2* E,
                           long long estride, int* loc, const int* n_steps, int step, int phase, hipStream_t st) {
    hipLaunchKernelGGL(reproject_descs_kernel, dim3((count + 63) / 64), dim3(64), 0, st, descs, count, b0, X0, X1,
                       xstride, E, estride, loc, n_steps, step, phase);
    return hipGetLastError();
}

hipError_t unitarity_check(int d, int count, int b0, const float2* E, long long estride, const int* n_steps, int step,
                           DeviceFlags* flags, hipStream_t st) {
    hipLaunchKernelGGL(unitarity_check_kernel, dim3(count), dim3(256), 0, st, d, E, estride, n_steps, b0, step, flags);
    return hipGetLastError();
}

hipError_t reproject_states(int d, int B, float2* X0, float2* X1, long long xstride, float2* E, GemmDesc* descs,
                            int* loc, const int* n_steps, int step, int precision, DeviceFlags* flags, hipStream_t st) {
    for (int b0 = 0; b0 < B; b0 += REPROJECT_CHUNK) {
        const int ch = std::min(REPROJECT_CHUNK, B - b0);
        hipError_t e = reproject_descs(descs, ch, b0, X0, X1, xstride, E, xstride, loc, n_steps, step, 0, st);
        if (e == hipSuccess) e = cgemm_batched(d, ch, descs, precision, st, GEMM_ROLE_GRAM);
        if (e == hipSuccess) e = unitarity_check(d, ch, b0, E, xstride, n_steps, step, flags, st);
        if (e == hipSuccess) e = reproject_descs(descs, ch, b0, X0, X1, xstride, E, xstride, loc, n_steps, step, 1, st);
        if (e == hipSuccess) e = cgemm_batched(d, ch, descs, 2, st, GEMM_ROLE_REPROJECT);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t gather_back(int d, int B, float2* X0, const float2* X1, long long xstride, const int* loc, hipStream_t st) {
    const long long nn = (long long)d * d;
    const int bx = (int)std::max<long long>(1, std::min<long long>((nn + 255) / 256, (1LL << 22) / B));
    hipLaunchKernelGGL(gather_back_kernel, dim3(bx, B), dim3(256), 0, st, nn, X0, X1, xstride, loc);
    return hipGetLastError();
}

hipError_t fill_int(int* p, int n, int v, hipStream_t st) {
    hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t fill_descs(GemmDesc* descs, int count, const float2* A, long long sA, int opA, const float2* B, long long sB,
                      int opB, float2* C, long long sC, const int* n_steps, int step, int inactive_mode, float alpha,
                      float beta, hipStream_t st) {
    hipLaunchKernelGGL(fill_descs_kernel, dim3((count + 63) / 64), dim3(64), 0, st, descs, count, A, sA, opA, B, sB,
                       opB, C, sC, n_steps, step, inactive_mode, alpha, beta);
    return hipGetLastError();
}

hipError_t grape_pair_descs(GemmDesc* descs, int N, int B, const float2* U, long long sU, float2* X, long long sX,
                            float2* LH, long long sL, long long mat, const int* n_steps, hipStream_t st) {
    const long long n = (long long)2 * N * B;
    hipLaunchKernelGGL(grape_pair_descs_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, descs, N, B, U, sU,
                       X, sX, LH, sL, mat, n_steps);
    return hipGetLastError();
}

// partial sums of every instance, then the packed row lists ([d][OBS_WMAX] ints and complex)
size_t observable_partial_doubles(int d, int B) {
    return (size_t)B * (d / obs_rows(d)) + (size_t)d * OBS_WMAX * 3 / 2 + 2;
}

template <int SW, int WP, int NT>
static hipError_t launch_mx(int d, int cnt, int b0, const float2* X0, const float2* X1, const int* loc,
                            long long xstride, const int* cols, const float2* vals, int w, const int* n_steps,
                            int step, float2* T, hipStream_t st) {
    const void* k = (const void*)observable_mx_kernel<SW, WP, NT>;
    const size_t lds = sizeof(float2) * (size_t)SW * d;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((observable_mx_kernel<SW, WP, NT>), dim3((unsigned)((long long)(d / SW) * cnt)), dim3(NT), lds,
                       st, d, b0, X0, X1, loc, xstride, cols, vals, w, n_steps, step, T);
    return hipGetLastError();
}

template <int WP, int NT, int LPR>
static hipError_t launch_mx8(int d, int cnt, int b0, const float2* X0, const float2* X1, const int* loc,
                             long long xstride, const int* cols, const float2* vals, int w, const int* n_steps,
                             int step, float2* T, hipStream_t st) {
    const void* k = (const void*)observable_mx8_kernel<WP, NT, LPR>;
    const size_t lds = sizeof(float2) * (size_t)8 * d;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((observable_mx8_kernel<WP, NT, LPR>), dim3((unsigned)((long long)(d / 8) * cnt)), dim3(NT), lds,
                       st, d, b0, X0, X1, loc, xstride, cols, vals, n_steps, step, T);
    return hipGetLastError();
}

template <int R, int WP, int NT>
static hipError_t launch_dot(int d, int cnt, int b0, const float2* X0, const float2* X1, const int* loc,
                             long long xstride, const int* cols, const float2* vals, int w, const int* n_steps,
                             int step, const float2* T, double* partial, hipStream_t st) {
    const void* k = (const void*)observable_dot_kernel<R, WP, NT>;
    const size_t lds = sizeof(float2) * (size_t)R * d;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((observable_dot_kernel<R, WP, NT>), dim3((unsigned)((long long)(d / R) * cnt)), dim3(NT), lds,
                       st, d, b0, X0, X1, loc, xstride, cols, vals, w, n_steps, step, T, partial);
    return hipGetLastError();
}

template <int WP>
static hipError_t obs_chunk(int d, int cnt, int b0, const float2* X0, const float2* X1, const int* loc,
                            long long xstride, const int* cols, const float2* vals, int w, const int* n_steps,
                            int step, float2* T, double* partial, hipStream_t st) {
    const int SW = obs_strip(d), R = obs_rows(d);
    hipError_t e;
#define MXA d, cnt, b0, X0, X1, loc, xstride, cols, vals, w, n_steps, step, T, st
#define DTA d, cnt, b0, X0, X1, loc, xstride, cols, vals, w, n_steps, step, T, partial, st
    switch (SW) {
        case 8:
            e = d >= 256 ? launch_mx8<WP, 256, 1>(MXA) : d >= 128 ? launch_mx8<WP, 256, 2>(MXA) : launch_mx8<WP, 256, 4>(MXA);
            break;
        case 4: e = launch_mx<4, WP, 256>(MXA); break;
        case 2: e = launch_mx<2, WP, 256>(MXA); break;
        default: e = launch_mx<1, WP, 256>(MXA);
    }
    if (e != hipSuccess) return e;
    switch (R) {
        case 4: return launch_dot<4, WP, 256>(DTA);
        case 2: return launch_dot<2, WP, 256>(DTA);
        default: return launch_dot<1, WP, 256>(DTA);
    }
#undef MXA
#undef DTA
}

hipError_t observable(int d, int B, const float2* X0, const float2* X1, const int* loc, long long xstride,
                      const int* cols, const float2* vals, int w, const int* n_steps, int step, double* partial,
                      double* out, long long out_stride, float2* T, int chunk, hipStream_t st) {
    if (w < 1 || w > OBS_WMAX) return hipErrorInvalidValue;
    const int wp = (w + 3) / 4 * 4;
    // packed lists after the partial sums, 16-byte aligned
    const size_t np = (size_t)B * (d / obs_rows(d));
    int* pc = reinterpret_cast<int*>(partial + np + (np & 1));
    float2* pv = reinterpret_cast<float2*>(pc + (size_t)d * OBS_WMAX);
    hipLaunchKernelGGL(obs_pack_kernel, dim3((d * wp + 255) / 256), dim3(256), 0, st, d, w, wp, cols, vals, pc, pv);
    hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
    for (int b0 = 0; b0 < B; b0 += chunk) {
        const int cnt = std::min(chunk, B - b0);
        hipError_t e;
        switch (wp) {
            case 4: e = obs_chunk<4>(d, cnt, b0, X0, X1, loc, xstride, pc, pv, wp, n_steps, step, T, partial, st); break;
            case 8: e = obs_chunk<8>(d, cnt, b0, X0, X1, loc, xstride, pc, pv, wp, n_steps, step, T, partial, st); break;
            case 12: e = obs_chunk<12>(d, cnt, b0, X0, X1, loc, xstride, pc, pv, wp, n_steps, step, T, partial, st); break;
            default: e = obs_chunk<16>(d, cnt, b0, X0, X1, loc, xstride, pc, pv, wp, n_steps, step, T, partial, st);
        }
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(observable_final_kernel, dim3(B), dim3(256), 0, st, d / obs_rows(d), partial, vals, d * w,
                       n_steps, step, out, out_stride);
    return hipGetLastError();
}

bool walsh_dim(int d) { return d >= 128 && d <= WALSH_DMAX && (d & (d - 1)) == 0; }

hipError_t walsh_fill(int d, int B, float2* X, long long stride, hipStream_t st) {
    const long long nn = (long long)d * d;
    const long long blocks = std::min<long long>((nn * B + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(walsh_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st, nn, d, B, X, stride,
                       (float)(1.0 / std::sqrt((double)d)));
    return hipGetLastError();
}

hipError_t walsh_right(int d, int B, float2* X, long long stride, hipStream_t st) {
    if (d < 128 || d > 4096 || (d & (d - 1)) != 0) return hipErrorInvalidValue;
    const long long rows = (long long)B * d;
    const dim3 grid((unsigned)((rows + 3) / 4));
    const float s = (float)(1.0 / std::sqrt((double)d));
    switch (d / 64) {
        case 2: hipLaunchKernelGGL(walsh_right_kernel<2>, grid, dim3(256), 0, st, d, rows, X, stride, s); break;
        case 4: hipLaunchKernelGGL(walsh_right_kernel<4>, grid, dim3(256), 0, st, d, rows, X, stride, s); break;
        case 8: hipLaunchKernelGGL(walsh_right_kernel<8>, grid, dim3(256), 0, st, d, rows, X, stride, s); break;
        case 16: hipLaunchKernelGGL(walsh_right_kernel<16>, grid, dim3(256), 0, st, d, rows, X, stride, s); break;
        case 32: hipLaunchKernelGGL(walsh_right_kernel<32>, grid, dim3(256), 0, st, d, rows, X, stride, s); break;
        default: hipLaunchKernelGGL(walsh_right_kernel<64>, grid, dim3(256), 0, st, d, rows, X, stride, s);
    }
    return hipGetLastError();
}

template <int WP, int LPR>
static hipError_t launch_walsh_obs(int d, int B, const float2* X0, const float2* X1, const int* loc,
                                   long long xstride, const int* cols, const float2* vals, const double* spec,
                                   const int* n_steps, int step, double* partial, hipStream_t st) {
    const void* k = (const void*)observable_walsh_kernel<WP, 256, LPR>;
    // LPR = 1: 80-byte rows, the reduction in the strip's memory; else 64-byte rows and NT doubles
    const size_t lds = LPR == 1 ? sizeof(float2) * (size_t)10 * d : sizeof(float2) * (size_t)8 * d + 256 * sizeof(double);
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((observable_walsh_kernel<WP, 256, LPR>), dim3((unsigned)((long long)(d / 8) * B)), dim3(256),
                       lds, st, d, 0, X0, X1, loc, xstride, cols, vals, spec, n_steps, step, partial);
    return hipGetLastError();
}

template <int WP>
static hipError_t walsh_obs(int d, int B, const float2* X0, const float2* X1, const int* loc, long long xstride,
                            const int* cols, const float2* vals, const double* spec, const int* n_steps, int step,
                            double* partial, hipStream_t st) {
    // enough lanes per pair that the d / 2 pairs of a mask cover the 256 threads
    if (d >= 512) return launch_walsh_obs<WP, 1>(d, B, X0, X1, loc, xstride, cols, vals, spec, n_steps, step, partial, st);
    if (d == 256) return launch_walsh_obs<WP, 2>(d, B, X0, X1, loc, xstride, cols, vals, spec, n_steps, step, partial, st);
    return launch_walsh_obs<WP, 4>(d, B, X0, X1, loc, xstride, cols, vals, spec, n_steps, step, partial, st);
}

hipError_t observable_walsh(int d, int B, const float2* X0, const float2* X1, const int* loc, long long xstride,
                            const int* cols, const float2* vals, int w, const double* spec, const int* n_steps,
                            int step, double* partial, double* out, long long out_stride, hipStream_t st) {
    if (w < 1 || w > OBS_WMAX || !walsh_dim(d) || (long long)(d / 8) * B > 0x7fffffffLL) return hipErrorInvalidValue;
    const int wp = (w + 3) / 4 * 4;
    // packed lists after the partial sums, as observable()
    const size_t np = (size_t)B * (d / obs_rows(d));
    int* pc = reinterpret_cast<int*>(partial + np + (np & 1));
    float2* pv = reinterpret_cast<float2*>(pc + (size_t)d * OBS_WMAX);
    hipLaunchKernelGGL(obs_pack_kernel, dim3((d * wp + 255) / 256), dim3(256), 0, st, d, w, wp, cols, vals, pc, pv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (wp) {
        case 4: e = walsh_obs<4>(d, B, X0, X1, loc, xstride, pc, pv, spec, n_steps, step, partial, st); break;
        case 8: e = walsh_obs<8>(d, B, X0, X1, loc, xstride, pc, pv, spec, n_steps, step, partial, st); break;
        case 12: e = walsh_obs<12>(d, B, X0, X1, loc, xstride, pc, pv, spec, n_steps, step, partial, st); break;
        default: e = walsh_obs<16>(d, B, X0, X1, loc, xstride, pc, pv, spec, n_steps, step, partial, st);
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(observable_final_kernel, dim3(B), dim3(256), 0, st, d / 8, partial, vals, d * w, n_steps, step,
                       out, out_stride);
    return hipGetLastError();
}

void obs_packed_lists(int d, int B, double* partial, int** pc, float2** pv) {
    const size_t np = (size_t)B * (d / obs_rows(d));
    *pc = reinterpret_cast<int*>(partial + np + (np & 1));
    *pv = reinterpret_cast<float2*>(*pc + (size_t)d * OBS_WMAX);
}

hipError_t obs_pack_lists(int d, int B, int w, const int* cols, const float2* vals, double* partial, hipStream_t st) {
    if (w < 1 || w > OBS_WMAX) return hipErrorInvalidValue;
    const int wp = (w + 3) / 4 * 4;
    int* pc;
    float2* pv;
    obs_packed_lists(d, B, partial, &pc, &pv);
    hipLaunchKernelGGL(obs_pack_kernel, dim3((d * wp + 255) / 256), dim3(256), 0, st, d, w, wp, cols, vals, pc, pv);
    return hipGetLastError();
}

hipError_t observable_final(int nparts, int B, const double* partial, const float2* vals, int nvals,
                            const int* n_steps, int step, double* out, long long out_stride, hipStream_t st) {
    hipLaunchKernelGGL(observable_final_kernel, dim3(B), dim3(256), 0, st, nparts, partial, vals, nvals, n_steps, step,
                       out, out_stride);
    return hipGetLastError();
}

size_t trace_partial_doubles(int d, int B, int K) { return (size_t)B * K * (d / TT) * (d / TT) * 6; }

hipError_t traces(int d, int B, int K, int phased, const float2* Y, long long ystride, const float2* S,
                  const double* g, const int* codes, const double* phi, long long code_stride, const int* n_steps,
                  int step, double* partial, double* out, long long out_bstride, int cartesian, hipStream_t st,
                  const double* h, int n_drift, double hdt) {
    const int ntile = (d / TT) * (d / TT);
    hipLaunchKernelGGL(trace_partial_kernel, dim3(ntile, K, B), dim3(256), 0, st, d, K, phased, Y, ystride, S, g, codes,
                       phi, code_stride, n_steps, step, partial, cartesian, h, n_drift, hdt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(trace_final_kernel, dim3(B, K), dim3(64), 0, st, ntile, K, partial, out, out_bstride);
    return hipGetLastError();
}

hipError_t grad_assemble(int B, int N, int K, int phased, double eps, double dt, const int* codes, const double* phi,
                         const double* tr, const double* d0, const double2* overlap, const double* nu,
                         const int* n_steps, float* grad, int cartesian, hipStream_t st) {
    const long long n = (long long)B * N * K;
    hipLaunchKernelGGL(grad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, B, N, K, phased, eps, dt, codes,
                       phi, tr, d0, overlap, nu, n_steps, grad, cartesian);
    return hipGetLastError();
}

hipError_t d0_traces(int d, int B, int K, int phased, const float2* L, long long lstride, const double* g, double* d0,
                     hipStream_t st, int conj_l) {
    hipLaunchKernelGGL(d0_kernel, dim3(B, K), dim3(256), 0, st, d, K, phased, L, lstride, g, d0, conj_l);
    return hipGetLastError();
}

size_t sparse_trace_partial_doubles(int d, int B, int steps, int K) {
    const size_t rows = (size_t)B * steps * K * (d / SPT_RPB) * 6;
    // d <= 1024: the per-step kernels keep every entry of Y at the pattern instead
    return d <= 1024 ? std::max(rows, (size_t)B * steps * d * (SPAT_WMAX + 1) * 2) : rows;
}

template <int WP>
static void launch_spt(dim3 grid, hipStream_t st, int d, int N, int step0, int nsl, int K, int phased, int cartesian,
                       int sw,
                       const float2* X, long long xsb, const float2* LH, long long lsb, const int* spc,
                       const double2* spv, const double* g, const int* codes, const double* phi, const int* n_steps,
                       double* partial, const double* h, int n_drift, double hdt) {
    hipLaunchKernelGGL(sparse_trace_kernel<WP>, grid, dim3(256), 0, st, d, N, step0, nsl, K, phased, cartesian, sw, X,
                       xsb, LH, lsb, spc, spv, g, codes, phi, n_steps, partial, h, n_drift, hdt);
}

hipError_t sparse_traces(int d, int B, int N, int step0, int steps, int K, int phased, int cartesian, int sw,
                         const float2* X, long long xsb, const float2* LH, long long lsb, const int* spc,
                         const double2* spv, const double* g, const int* codes, const double* phi,
                         const int* n_steps, double* partial, double* tr, hipStream_t st, const double* h,
                         int n_drift, double hdt) {
    if (sw < 1 || sw > SPAT_WMAX || d % SPT_RPB != 0) return hipErrorInvalidValue;
    const int wp = (sw + 3) / 4 * 4;
    if (d <= SPS_DMAX && d % (64 * SPS_RPT) == 0 && wp <= 12 && B <= 65535) {
        // partial holds ybuf: [B][steps][d][SPS_NE] complex FP64
        double2* ybuf = reinterpret_cast<double2*>(partial);
        const dim3 sgrid(steps, B);
#define REDO_SPS(W)                                                                                                   \
    hipLaunchKernelGGL(sparse_y_kernel<W>, sgrid, dim3(d / SPS_RPT), 0, st, d, N, step0, steps, sw, X, xsb, LH, lsb, \
                       spc, n_steps, ybuf)
        switch (wp) {   // 16 slots would not fit the registers: the row-block kernel below
            case 4: REDO_SPS(4); break;
            case 8: REDO_SPS(8); break;
            default: REDO_SPS(12);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(sparse_ysum_kernel, sgrid, dim3(256), 0, st, d, N, step0, steps, K, phased, cartesian, sw,
                           ybuf, spc, spv, g, codes, phi, n_steps, tr, h, n_drift, hdt);
#undef REDO_SPS
        return hipGetLastError();
    }
    const long long padded = (long long)(d / SPT_RPB) * ((steps + SPT_XCD - 1) / SPT_XCD * SPT_XCD);
    if (padded > 0x7fffffffLL || B > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)padded, B);
    switch (wp) {
        case 4: launch_spt<4>(grid, st, d, N, step0, steps, K, phased, cartesian, sw, X, xsb, LH, lsb, spc, spv, g, codes, phi, n_steps, partial, h, n_drift, hdt); break;
        case 8: launch_spt<8>(grid, st, d, N, step0, steps, K, phased, cartesian, sw, X, xsb, LH, lsb, spc, spv, g, codes, phi, n_steps, partial, h, n_drift, hdt); break;
        case 12: launch_spt<12>(grid, st, d, N, step0, steps, K, phased, cartesian, sw, X, xsb, LH, lsb, spc, spv, g, codes, phi, n_steps, partial, h, n_drift, hdt); break;
        default: launch_spt<16>(grid, st, d, N, step0, steps, K, phased, cartesian, sw, X, xsb, LH, lsb, spc, spv, g, codes, phi, n_steps, partial, h, n_drift, hdt);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // sum the row blocks: instance (b, s) of this chunk writes tr[b][step0 + s][k][6]
    for (int b = 0; b < B; ++b) {
        hipLaunchKernelGGL(trace_final_kernel, dim3(steps, K), dim3(64), 0, st, d / SPT_RPB, K,
                           partial + (size_t)b * steps * K * (d / SPT_RPB) * 6,
                           tr + ((size_t)b * N + step0) * K * 6, (long long)K * 6);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t fill_identity(int d, int B, float2* X, long long stride, hipStream_t st) {
    const long long nn = (long long)d * d;
    const long long blocks = std::min<long long>((nn * B + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(identity_kernel, dim3((unsigned)blocks), dim3(256), 0, st, nn, d, B, X, stride);
    return hipGetLastError();
}

}  // namespace redo
