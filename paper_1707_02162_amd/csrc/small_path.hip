// Small-dimension REDO path (d = 2 .. 64): one fused kernel runs a whole
// chain per instance.  Each step quantises its amplitudes (Sec. II, Eq.
// cgrain), multiplies the state by the table factors that the digits select
// (processes 1 and 2, Eqs. redoform and exp2prod) between the drift and
// phase scalings of the split step (Sec. III, Eqs. vn and vnd), and chains
// the result (Sec. III, Eq. propUn).  Products are staged in LDS; every
// thread owns a TB x TB strided sub-block of one instance's d x d state
// (TB = 2 up to d = 32, 4 at d = 64), so an instance is (d/TB)^2 threads and a
// 256-thread workgroup hosts several.
// The GRAPE kernel adds a checkpointed backward scan for the gradient.  When
// the table's level cache holds every level (process 3), each channel takes
// one composed factor per step instead of one per non-zero digit.
#include "redo_internal.h"

namespace redo {
namespace {

constexpr int KMAX = 16;

struct TView {
    const float2* T;
    const float2* cache;   // every level composed (process 3): [K][levels][d][d], or null
    const float2* V;
    const double* h;
    const double* g;
    const signed char* g2;   // 2 g as integers (every g a half-integer), or null
    const float2* S;
    DeviceFlags* flags;
    long long ent;   // d*d
    int d, K, P, base, phased, diag, n_drift;
    int levels;            // cache levels (q = 0 .. levels - 1)
    int strang;            // 1: U_n = V(dt/2) C_n V(dt/2) (diagonal drift)
    double eps, qmax, dt;
};

TView view_of(const redo_table_s* t) {
    TView v;
    v.T = t->T32;
    // the fused kernels use the level cache only when it holds every level
    const bool all = t->cache && t->cache_lo == 0 && (double)t->cache_hi >= t->qmax;
    v.cache = all ? t->cache : nullptr;
    v.levels = all ? t->cache_hi + 1 : 0;
    v.V = t->V32;
    v.h = t->h64;
    v.g = t->g64;
    v.g2 = t->g2;
    v.S = t->S32;
    v.flags = t->flags;
    v.ent = t->entry_elems;
    v.d = t->desc.d;
    v.K = t->desc.K;
    v.P = t->desc.digits;
    v.base = t->desc.base;
    v.phased = t->desc.phased;
    v.diag = t->desc.drift_is_diag;
    v.n_drift = t->desc.n_drift;
    v.eps = t->desc.eps;
    v.qmax = t->qmax;
    v.dt = t->desc.dt;
    v.strang = t->desc.splitting;
    return v;
}

// d <= 32: 2 x 2 sub-blocks (d^2/4 threads per instance: more waves per CU to
// hide the latency of the per-step barriers and table loads); d = 64: 4 x 4
// (one instance per 256-thread workgroup).
template <int D>
struct Cfg {
    static constexpr int TB = D >= 64 ? 4 : 2;  // sub-block edge per thread
    static constexpr int NT = D / TB;          // threads along a row of sub-blocks
    static constexpr int TPI = NT * NT;        // threads per instance
    static constexpr int IPB = 256 / TPI;      // instances per workgroup
    // float2 of padding after each instance's LDS buffers: their sizes (2 or 3 d^2 float2) are
    // multiples of 256 bytes at d = 4, 8, so that without it the lanes of the instances sharing a
    // wave would meet in the same banks at every access (measured: 70-75 % of the LDS cycles of the
    // d = 4 kernels were bank conflicts)
    static constexpr int PAD = 4;
    // instances of at least one wave take each step's codes and control pairs from a per-step
    // header in LDS (ChanHdr); so do phased channels at every d (HD below)
    static constexpr bool HDR = TPI >= 64;
    // the products run on the matrix cores (one output quadrant per wave, the result handed to the
    // owning threads through one more LDS buffer): chains at d = 32, 64, GRAPE at d = 32 (at d = 64
    // its accumulators would push the GRAPE kernel's live state out of registers)
    static constexpr bool MF = D == 32 || D == 64, MFG = D == 32;
    static constexpr int NBUF_CHAIN = MF ? 3 : 2, NBUF_GRAPE = MFG ? 4 : 3;   // d x d LDS buffers per instance
};

// LDS word of element (r, c) of an instance's d x d buffer.  d = 32, 64: the column index is XORed
// with a function of the row, so that the matrix-core operand reads (lanes down a column of the
// left factor, or along a row of the right one) fall in distinct banks; smaller d: row-major.
template <int D>
__device__ inline int lidx(int r, int c) {
    if constexpr (D == 32)
        return r * D + (c ^ (((r << 1) ^ ((r & 1) << 4)) & 31));
    else if constexpr (D == 64)
        return r * D + (c ^ (r & 31));
    else
        return r * D + c;
}

// Barrier among the threads of one instance around its LDS buffers.  At d <= 16
// an instance's threads are lanes of one wave, whose LDS accesses execute in
// program order: a compiler fence suffices and the waves of a workgroup run
// independently.  At d >= 32 an instance spans the workgroup's four waves.
template <int D>
__device__ inline void inst_sync() {
    if constexpr (Cfg<D>::TPI > 64) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Drift phases exp(-i hdt h_a) of the rows (or columns) idx + NT r the thread owns
// (hdt = dt, or dt/2 for the Strang halves), in FP64 (ph64, combined with the phase
// rotations of phased channels before the single rounding) and rounded once to FP32
// (ph): constant along the chain, so computed once per instance.
template <int D>
__device__ inline void drift_phases(const TView& tv, int drift, int idx, float2 (&ph)[Cfg<D>::TB],
                                    double2 (&ph64)[Cfg<D>::TB]) {
    constexpr int TB = Cfg<D>::TB, NT = Cfg<D>::NT;
    const double hdt = tv.strang ? 0.5 * tv.dt : tv.dt;
#pragma unroll
    for (int r = 0; r < TB; ++r) {
        if (tv.diag) {
            ph64[r] = expmi(hdt * tv.h[(long long)drift * D + idx + NT * r]);
            ph[r] = make_float2((float)ph64[r].x, (float)ph64[r].y);
        } else {
            ph64[r] = make_double2(1.0, 0.0);
            ph[r] = make_float2(1.f, 0.f);
        }
    }
}

// ---------------------------------------------------------------- LDS helpers
// element (r, c) of the thread's sub-block is (ti + NT r, tj + NT c)
template <int D>
__device__ inline void store_block(float2* Ms, const float2 (&x)[Cfg<D>::TB][Cfg<D>::TB], int ti, int tj) {
    constexpr int TB = Cfg<D>::TB, NT = Cfg<D>::NT;
#pragma unroll
    for (int r = 0; r < TB; ++r)
#pragma unroll
        for (int c = 0; c < TB; ++c) Ms[lidx<D>(ti + NT * r, tj + NT * c)] = x[r][c];
}

// Ms <- src (d x d from global), or src^dag when adj
template <int D>
__device__ inline void stage(float2* Ms, const float2* __restrict__ src, bool adj, int lt) {
    constexpr int TPI = Cfg<D>::TPI;
    for (int e = lt; e < D * D; e += TPI) {
        const float2 v = src[e];
        if (adj)
            Ms[lidx<D>(e % D, e / D)] = cconj(v);
        else
            Ms[lidx<D>(e / D, e % D)] = v;
    }
}

// A table entry travels global -> registers -> LDS: each thread holds TB^2 of
// its D^2 elements (element lt + TPI i), so the next factor's loads are in
// flight while the current product runs.
template <int D>
struct FactorRegs {
    float2 v[Cfg<D>::TB * Cfg<D>::TB];
};
template <int D>
__device__ inline void fetch_factor(FactorRegs<D>& f, const float2* __restrict__ src, int lt) {
    constexpr int TPI = Cfg<D>::TPI, NR = Cfg<D>::TB * Cfg<D>::TB;
#pragma unroll
    for (int i = 0; i < NR; ++i) f.v[i] = src[lt + TPI * i];
}
template <int D>
__device__ inline void put_factor(float2* Ms, const FactorRegs<D>& f, bool adj, int lt) {
    constexpr int TPI = Cfg<D>::TPI, NR = Cfg<D>::TB * Cfg<D>::TB;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int e = lt + TPI * i;
        if (adj)
            Ms[lidx<D>(e % D, e / D)] = cconj(f.v[i]);
        else
            Ms[lidx<D>(e / D, e % D)] = f.v[i];
    }
}

// x <- (A B) on the thread's block, A and B d x d in LDS.  Matrix cores (MM; d = 32, 64): wave w forms
// output quadrant (w / 2, w % 2) with four real products per k-block (v_mfma_f32_16x16x4_f32 at
// d = 32, v_mfma_f32_32x32x2_f32 at d = 64; FP32 accumulation), writes it to Rs and, after a barrier,
// every thread reads its own block back; the caller's next barrier precedes the next write of Rs.
// Vector FMAs on the thread's block otherwise.
template <int D, bool MM>
__device__ inline void mul_left(float2 (&x)[Cfg<D>::TB][Cfg<D>::TB], const float2* A, const float2* B, float2* Rs,
                                int ti, int tj) {
    constexpr int TB = Cfg<D>::TB, NT = Cfg<D>::NT;
    if constexpr (MM) {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, qi = w >> 1, qj = w & 1;
        if constexpr (D == 32) {
            typedef float fx4 __attribute__((ext_vector_type(4)));
            const int i = 16 * qi + (lane & 15), j = 16 * qj + (lane & 15), kq = lane >> 4;
            fx4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k0 = 0; k0 < D; k0 += 4) {
                const float2 a = A[lidx<D>(i, k0 + kq)], b = B[lidx<D>(k0 + kq, j)];
                cr = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, cr, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.y, ci, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, b.y, cr, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.x, ci, 0, 0, 0);
            }
            // element (4 (lane / 16) + r, lane % 16) of the quadrant in register r
#pragma unroll
            for (int r = 0; r < 4; ++r) Rs[lidx<D>(16 * qi + 4 * kq + r, j)] = make_float2(cr[r], ci[r]);
        } else {
            typedef float fx16 __attribute__((ext_vector_type(16)));
            const int i = 32 * qi + (lane & 31), j = 32 * qj + (lane & 31), kq = lane >> 5;
            fx16 cr, ci;
#pragma unroll
            for (int r = 0; r < 16; ++r) cr[r] = ci[r] = 0.f;
#pragma unroll 4
            for (int k0 = 0; k0 < D; k0 += 2) {
                const float2 a = A[lidx<D>(i, k0 + kq)], b = B[lidx<D>(k0 + kq, j)];
                cr = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, cr, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.y, ci, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_32x32x2f32(-a.y, b.y, cr, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.x, ci, 0, 0, 0);
            }
            // element (8 (r / 4) + 4 (lane / 32) + r % 4, lane % 32) of the quadrant in register r
#pragma unroll
            for (int r = 0; r < 16; ++r)
                Rs[lidx<D>(32 * qi + 8 * (r >> 2) + 4 * kq + (r & 3), j)] = make_float2(cr[r], ci[r]);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < TB; ++r)
#pragma unroll
            for (int c = 0; c < TB; ++c) x[r][c] = Rs[lidx<D>(ti + NT * r, tj + NT * c)];
        return;
    }
    float2 acc[TB][TB];
#pragma unroll
    for (int r = 0; r < TB; ++r)
#pragma unroll
        for (int c = 0; c < TB; ++c) acc[r][c] = make_float2(0.f, 0.f);
#pragma unroll 8
    for (int m = 0; m < D; ++m) {
        float2 f[TB], y[TB];
#pragma unroll
        for (int r = 0; r < TB; ++r) f[r] = A[lidx<D>(ti + NT * r, m)];
#pragma unroll
        for (int c = 0; c < TB; ++c) y[c] = B[lidx<D>(m, tj + NT * c)];
#pragma unroll
        for (int r = 0; r < TB; ++r)
#pragma unroll
            for (int c = 0; c < TB; ++c) cfma(acc[r][c], f[r], y[c]);
    }
#pragma unroll
    for (int r = 0; r < TB; ++r)
#pragma unroll
        for (int c = 0; c < TB; ++c) x[r][c] = acc[r][c];
}

// reduce over the TPI threads of one instance (consecutive lanes); all get the sum
template <int D>
__device__ inline double inst_sum(double v, double* scratch) {
    constexpr int TPI = Cfg<D>::TPI;
    constexpr int W = TPI < 64 ? TPI : 64;
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if constexpr (TPI > 64) {
        __syncthreads();
        if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
        __syncthreads();
        v = scratch[0] + scratch[1] + scratch[2] + scratch[3];
    }
    return v;
}

// the six trace sums over the instance's lanes within each wave (the first half of inst_sum)
template <int D>
__device__ inline void wave_sums(double (&v)[6]) {
    constexpr int TPI = Cfg<D>::TPI;
    constexpr int W = TPI < 64 ? TPI : 64;
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1)
#pragma unroll
        for (int j = 0; j < 6; ++j) v[j] += __shfl_xor(v[j], off, 64);
}

// ---------------------------------------------------------------- one step
// The channels of one step, for instances of at least one wave: one thread per channel quantises
// its control (Sec. II, Eq. cgrain) and, for a phased channel, forms the rotation angle's half-angle
// phase (or the angle), and every thread of the instance reads them from LDS; without it every
// thread walks each channel's chain of dependent loads and FP64 arithmetic itself, once per slot.
struct ChanHdr {
    int q;          // the code
    float ux, uy;   // the control as given (uy: phased channels)
    double2 rot;    // phased: half_phase(ux, uy) with half-integer generators, else (phi, 0)
};
static_assert(sizeof(ChanHdr) == 32, "four float2 of LDS per channel");

// thread lt < K writes channel lt's entry; report: this pass reports non-finite and clamped controls
template <int D>
__device__ inline void make_header(const TView& tv, const float* us, bool active, bool report, int lt,
                                   ChanHdr* hd) {
    if (lt >= tv.K) return;
    const int KK = tv.phased ? 2 : 1;
    ChanHdr c;
    c.ux = active ? us[KK * lt] : 0.f;
    c.uy = (active && tv.phased) ? us[KK * lt + 1] : 0.f;
    double phi = 0.0;
    DeviceFlags* fl = report ? tv.flags : nullptr;
    c.q = 0;
    if (active) {
        // two calls with fixed pointer arguments: a conditional &phi would put phi in scratch memory
        if (tv.phased && !tv.g2)
            c.q = quantise_one(us + KK * lt, tv.phased, tv.eps, tv.qmax, &phi, fl);
        else
            c.q = quantise_one(us + KK * lt, tv.phased, tv.eps, tv.qmax, nullptr, fl);
    }
    c.rot = (active && tv.phased && tv.g2) ? half_phase((double)c.ux, (double)c.uy) : make_double2(phi, 0.0);
    hd[lt] = c;
}

// Phase rotations exp(+i theta_a), theta_a = sum_k phi_k g_k[a], of the rows (or
// columns) idx + NT r the thread owns (phased channels, Sec. III: Z = exp(-i theta G),
// so Z^dag scales index a by exp(+i theta_a)).  Phase generators of spins (every g a
// half-integer) give exp(i phi_k g) = (exp(i phi_k / 2))^(2g) from the control pair
// itself, with no transcendental function; others one FP64 sincos of the summed angle.
template <int D>
__device__ inline void step_rotations(const TView& tv, const float* us, bool active, int idx,
                                      double2 (&P)[Cfg<D>::TB]) {
    constexpr int TB = Cfg<D>::TB, NT = Cfg<D>::NT;
#pragma unroll
    for (int r = 0; r < TB; ++r) P[r] = make_double2(1.0, 0.0);
    if (!active || !tv.phased) return;
    if (tv.g2) {
        for (int k = 0; k < tv.K; ++k) {
            const double2 hp = half_phase((double)us[2 * k], (double)us[2 * k + 1]);
#pragma unroll
            for (int r = 0; r < TB; ++r) P[r] = zmul(P[r], zpow(hp, tv.g2[(long long)k * D + idx + NT * r]));
        }
    } else {
        double th[TB];
#pragma unroll
        for (int r = 0; r < TB; ++r) th[r] = 0.0;
        for (int k = 0; k < tv.K; ++k) {
            double phi;
            quantise_one(us + 2 * k, 1, tv.eps, tv.qmax, &phi, nullptr);
#pragma unroll
            for (int r = 0; r < TB; ++r) th[r] += phi * tv.g[(long long)k * D + idx + NT * r];
        }
#pragma unroll
        for (int r = 0; r < TB; ++r) P[r] = zconj(expmi(th[r]));
    }
}

// step_rotations from the step's header: the same arithmetic in the same order
template <int D>
__device__ inline void header_rotations(const TView& tv, const ChanHdr* hd, const signed char* g2l, const double* gl,
                                        bool active, int idx, double2 (&P)[Cfg<D>::TB]) {
    constexpr int TB = Cfg<D>::TB, NT = Cfg<D>::NT;
#pragma unroll
    for (int r = 0; r < TB; ++r) P[r] = make_double2(1.0, 0.0);
    if (!active || !tv.phased) return;
    if (tv.g2) {
        for (int k = 0; k < tv.K; ++k) {
            const double2 hp = hd[k].rot;
#pragma unroll
            for (int r = 0; r < TB; ++r) P[r] = zmul(P[r], zpow(hp, g2l[k * D + idx + NT * r]));
        }
    } else {
        double th[TB];
#pragma unroll
        for (int r = 0; r < TB; ++r) th[r] = 0.0;
        for (int k = 0; k < tv.K; ++k) {
            const double phi = hd[k].rot.x;
#pragma unroll
            for (int r = 0; r < TB; ++r) th[r] += phi * gl[k * D + idx + NT * r];
        }
#pragma unroll
        for (int r = 0; r < TB; ++r) P[r] = zconj(expmi(th[r]));
    }
}

__device__ inline float2 to_f2(double2 e) { return make_float2((float)e.x, (float)e.y); }

// x <- U_n x with U_n = Z [prod_k R_k] Z^dag V
// dph: the drift phases of the thread's rows (drift_phases), used when the channels are unphased
// report: non-finite and clamped controls are reported (by the header's channel threads with HD,
// else by the thread that passes it); hd: the instance's step header (HD); MM: matrix-core products
template <int D, bool MM, bool HD>
__device__ void step_left(const TView& tv, float2 (&x)[Cfg<D>::TB][Cfg<D>::TB], float2* Xs, float2* Fs, float2* Rs,
                          const float* us, int drift, bool active, bool report, int lt, int ti, int tj,
                          const float2 (&dph)[Cfg<D>::TB], const double2 (&dph64)[Cfg<D>::TB], ChanHdr* hd,
                          const signed char* g2l, const double* gl) {
    constexpr int TB = Cfg<D>::TB;
    const int KK = tv.phased ? 2 : 1;
    double2 P[TB];
    if constexpr (HD) {
        // the previous step's header was last read before the barriers of its last slot
        make_header<D>(tv, us, active, report, lt, hd);
        inst_sync<D>();
        header_rotations<D>(tv, hd, g2l, gl, active, ti, P);
    } else {
        step_rotations<D>(tv, us, active, ti, P);
    }
    // drift (or its first half, Strang), then Z^dag (diagonal scalings of rows)
    if (tv.diag) {
        if (active) {
#pragma unroll
            for (int r = 0; r < TB; ++r) {
                const float2 s = tv.phased ? to_f2(zmul(dph64[r], P[r])) : dph[r];
#pragma unroll
                for (int c = 0; c < TB; ++c) x[r][c] = cmul(s, x[r][c]);
            }
        }
    } else {
        inst_sync<D>();
        if (active) {
            stage<D>(Fs, tv.V + (long long)drift * tv.ent, false, lt);
            store_block<D>(Xs, x, ti, tj);
        }
        inst_sync<D>();
        if (active) {
            mul_left<D, MM>(x, Fs, Xs, Rs, ti, tj);
            if (tv.phased) {
#pragma unroll
                for (int r = 0; r < TB; ++r) {
                    const float2 s = to_f2(P[r]);
#pragma unroll
                    for (int c = 0; c < TB; ++c) x[r][c] = cmul(s, x[r][c]);
                }
            }
        }
    }
    // table factors: channel 0 first (rightmost), digits ascending; slot s = k P + j,
    // or one slot per channel (its composed level) when every level is cached.
    // The entry of the next slot is fetched while the current product runs.
    const int PE = tv.cache ? 1 : tv.P;
    const int nslot = tv.K * PE;
    auto slot_code = [&](int sl, bool rep) -> int {
        if constexpr (HD) return hd[sl / PE].q;
        return active ? quantise_one(us + KK * (sl / PE), tv.phased, tv.eps, tv.qmax, nullptr,
                                     rep ? tv.flags : nullptr)
                      : 0;
    };
    // the factor of slot sl for code q: nonzero digit c (or level |q|), else null
    auto entry_of = [&](int sl, int q) -> const float2* {
        if (tv.cache) {
            const int aq = q < 0 ? -q : q;
            return aq == 0 ? nullptr : tv.cache + ((long long)(sl / PE) * tv.levels + aq) * tv.ent;
        }
        const int c = digit_of(q, sl % PE, tv.base);
        return c == 0 ? nullptr : tv.T + ((long long)sl * (tv.base - 1) + (c - 1)) * tv.ent;
    };
    FactorRegs<D> fr;
    int q = slot_code(0, report);
    const float2* f = entry_of(0, q);
    if (f) fetch_factor<D>(fr, f, lt);
    for (int sl = 0; sl < nslot; ++sl) {
        inst_sync<D>();
        if (f) {
            put_factor<D>(Fs, fr, q < 0, lt);
            store_block<D>(Xs, x, ti, tj);
        }
        inst_sync<D>();
        const bool mult = f != nullptr;
        if (sl + 1 < nslot) {
            const int sn = sl + 1;
            if (sn % PE == 0) q = slot_code(sn, report);
            f = entry_of(sn, q);
            if (f) fetch_factor<D>(fr, f, lt);
        }
        if (mult) mul_left<D, MM>(x, Fs, Xs, Rs, ti, tj);
    }
    // Z, then the second half of the drift (Strang)
    if (active && (tv.phased || tv.strang)) {
#pragma unroll
        for (int r = 0; r < TB; ++r) {
            float2 s = dph[r];
            if (tv.phased) s = to_f2(tv.strang ? zmul(zconj(P[r]), dph64[r]) : zconj(P[r]));
#pragma unroll
            for (int c = 0; c < TB; ++c) x[r][c] = cmul(s, x[r][c]);
        }
    }
}

// l <- l U_n  (the backward scan), U_n = Z [prod_k R_k] Z^dag V
// dpc: the drift phases of the thread's columns (drift_phases), used when the channels are unphased
// hd: the step's header, published by the caller (HD); MM: matrix-core products
template <int D, bool MM, bool HD>
__device__ void step_right(const TView& tv, float2 (&l)[Cfg<D>::TB][Cfg<D>::TB], float2* Ls, float2* Fs, float2* Rs,
                           const float* us, int drift, bool active, int lt, int ti, int tj,
                           const float2 (&dpc)[Cfg<D>::TB], const double2 (&dpc64)[Cfg<D>::TB], const ChanHdr* hd,
                           const signed char* g2l, const double* gl) {
    constexpr int TB = Cfg<D>::TB;
    const int KK = tv.phased ? 2 : 1;
    // phase rotations exp(i theta_c) of the columns the thread owns
    double2 Pc[TB];
    if constexpr (HD)
        header_rotations<D>(tv, hd, g2l, gl, active, tj, Pc);
    else
        step_rotations<D>(tv, us, active, tj, Pc);
    // columns: the second half of the drift (Strang), then Z
    if (active && (tv.phased || tv.strang)) {
#pragma unroll
        for (int c = 0; c < TB; ++c) {
            float2 s = dpc[c];
            if (tv.phased) s = to_f2(tv.strang ? zmul(zconj(Pc[c]), dpc64[c]) : zconj(Pc[c]));
#pragma unroll
            for (int r = 0; r < TB; ++r) l[r][c] = cmul(l[r][c], s);
        }
    }
    // slots in reverse order (last channel, highest digit first); next entry prefetched
    {
        const int PE = tv.cache ? 1 : tv.P;
        const int nslot = tv.K * PE;
        auto slot_code = [&](int sl) -> int {
            if constexpr (HD) return hd[sl / PE].q;
            return active ? quantise_one(us + KK * (sl / PE), tv.phased, tv.eps, tv.qmax, nullptr, nullptr) : 0;
        };
        auto entry_of = [&](int sl, int q) -> const float2* {
            if (tv.cache) {
                const int aq = q < 0 ? -q : q;
                return aq == 0 ? nullptr : tv.cache + ((long long)(sl / PE) * tv.levels + aq) * tv.ent;
            }
            const int c = digit_of(q, sl % PE, tv.base);
            return c == 0 ? nullptr : tv.T + ((long long)sl * (tv.base - 1) + (c - 1)) * tv.ent;
        };
        FactorRegs<D> fr;
        int sl = nslot - 1;
        int q = slot_code(sl);
        const float2* f = entry_of(sl, q);
        if (f) fetch_factor<D>(fr, f, lt);
        for (; sl >= 0; --sl) {
            inst_sync<D>();
            if (f) {
                put_factor<D>(Fs, fr, q < 0, lt);
                store_block<D>(Ls, l, ti, tj);
            }
            inst_sync<D>();
            const bool mult = f != nullptr;
            if (sl > 0) {
                const int sn = sl - 1;
                if (sn % PE == PE - 1) q = slot_code(sn);
                f = entry_of(sn, q);
                if (f) fetch_factor<D>(fr, f, lt);
            }
            if (mult) mul_left<D, MM>(l, Ls, Fs, Rs, ti, tj);  // (Ls Fs) restricted to own block
        }
    }
    if (tv.diag) {
        if (active) {
#pragma unroll
            for (int c = 0; c < TB; ++c) {
                const float2 s = tv.phased ? to_f2(zmul(dpc64[c], Pc[c])) : dpc[c];
#pragma unroll
                for (int r = 0; r < TB; ++r) l[r][c] = cmul(l[r][c], s);
            }
        }
    } else {
        if (active && tv.phased) {
#pragma unroll
            for (int c = 0; c < TB; ++c) {
                const float2 s = to_f2(Pc[c]);
#pragma unroll
                for (int r = 0; r < TB; ++r) l[r][c] = cmul(l[r][c], s);
            }
        }
        inst_sync<D>();
        if (active) {
            stage<D>(Fs, tv.V + (long long)drift * tv.ent, false, lt);
            store_block<D>(Ls, l, ti, tj);
        }
        inst_sync<D>();
        if (active) mul_left<D, MM>(l, Ls, Fs, Rs, ti, tj);
    }
}

// Newton-Schulz polar step x <- x (3I - x^dag x) / 2  (uniform barriers); the
// watchdog counts an instance whose ||x^dag x - I||_F / sqrt(D) exceeds UNITARITY_WARN
template <int D>
__device__ void reproject(float2 (&x)[Cfg<D>::TB][Cfg<D>::TB], float2* Xs, float2* Fs, float2* Rs, bool active, int ti, int tj,
                          double* red, DeviceFlags* flags, bool leader) {
    constexpr int TB = Cfg<D>::TB, NT = Cfg<D>::NT;
    double dev2 = 0.0;
    inst_sync<D>();
    if (active) store_block<D>(Xs, x, ti, tj);
    inst_sync<D>();
    float2 z[TB][TB];
    if (active) {
        // z = x^dag x on the thread's block
#pragma unroll
        for (int r = 0; r < TB; ++r)
#pragma unroll
            for (int c = 0; c < TB; ++c) z[r][c] = make_float2(0.f, 0.f);
        for (int m = 0; m < D; ++m) {
            float2 a[TB], b[TB];
#pragma unroll
            for (int r = 0; r < TB; ++r) a[r] = cconj(Xs[lidx<D>(m, ti + NT * r)]);
#pragma unroll
            for (int c = 0; c < TB; ++c) b[c] = Xs[lidx<D>(m, tj + NT * c)];
#pragma unroll
            for (int r = 0; r < TB; ++r)
#pragma unroll
                for (int c = 0; c < TB; ++c) cfma(z[r][c], a[r], b[c]);
        }
#pragma unroll
        for (int r = 0; r < TB; ++r)
#pragma unroll
            for (int c = 0; c < TB; ++c) {
                const double er = (double)z[r][c].x - (ti + NT * r == tj + NT * c ? 1.0 : 0.0), ei = z[r][c].y;
                dev2 += er * er + ei * ei;
                z[r][c] = make_float2(-0.5f * z[r][c].x, -0.5f * z[r][c].y);
                if (ti + NT * r == tj + NT * c) z[r][c].x += 1.5f;
            }
        store_block<D>(Fs, z, ti, tj);
    }
    dev2 = inst_sum<D>(dev2, red);
    if (active && leader) report_drift(flags, sqrt(dev2 / D));
    inst_sync<D>();
    if (active) mul_left<D, Cfg<D>::MF>(x, Xs, Fs, Rs, ti, tj);
}

// The phase generators' diagonals (g, and 2g as integers) into LDS for the header kernels: every
// thread reads them at every step (through these arrays, which the compiler then knows to be LDS).
template <int D, bool HD>
__device__ inline void stage_generators(const TView& tv, signed char* g2s, double* gs) {
    if constexpr (HD) {
        if (tv.phased) {
            for (int e = threadIdx.x; e < tv.K * D; e += 256) {
                gs[e] = tv.g[e];
                if (tv.g2) g2s[e] = tv.g2[e];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- chain kernel
// PH: the table's phased flag as a compile-time constant (the signed-channel instance carries
// no phase arithmetic: no atan2 or sincos per step, far fewer registers).  That instance at
// d <= 16 fits 128 registers without spills, four waves per SIMD.
template <int D, int PH>
__global__ __launch_bounds__(256, (PH == 0 && D <= 16) ? 4 : 1) void small_chain_kernel(TView tv_in, SmallChainArgs a,
                                                                                        int ninst) {
    TView tv = tv_in;
    tv.phased = PH;
    constexpr int TB = Cfg<D>::TB, NT = Cfg<D>::NT, TPI = Cfg<D>::TPI, IPB = Cfg<D>::IPB;
    extern __shared__ float2 lds[];
    __shared__ double red[4];
    __shared__ int nblk;
    const int tid = threadIdx.x, slot = tid / TPI, lt = tid % TPI;
    const int ti = lt / NT, tj = lt % NT;
    const int inst = blockIdx.x * IPB + slot;
    const bool valid = inst < ninst;
    constexpr bool HDR = Cfg<D>::HDR || PH == 1;
    __shared__ signed char g2s[HDR ? KMAX * D : 1];
    __shared__ double gs[HDR ? KMAX * D : 1];
    stage_generators<D, HDR>(tv, g2s, gs);
    // step headers (K per instance) after the instances' buffers, then the observable's row lists
    ChanHdr* hdr = reinterpret_cast<ChanHdr*>(lds + (long long)IPB * (Cfg<D>::NBUF_CHAIN * D * D + Cfg<D>::PAD));
    ChanHdr* hd = hdr + (HDR ? slot * tv.K : 0);
    float2* Xs = lds + (long long)slot * (Cfg<D>::NBUF_CHAIN * D * D + Cfg<D>::PAD);
    float2* Fs = Xs + D * D;
    float2* Rs = Fs + D * D;   // product results (matrix-core products)
    int b = 0, n0 = 0, len = 0;
    if (valid) {
        if (a.compose) {
            b = inst / a.N_max;
            n0 = inst % a.N_max;
            len = (a.n_steps && n0 >= a.n_steps[b]) ? 0 : 1;   // steps past a ragged length: none
        } else {
            b = inst;
            len = a.n_steps ? a.n_steps[b] : a.N_max;
        }
    }
    if (tid == 0) nblk = 0;
    __syncthreads();
    if (lt == 0 && len > 0) atomicMax(&nblk, len);
    __syncthreads();
    const int N = nblk;
    const int drift = b % tv.n_drift;
    const int KK = tv.phased ? 2 : 1;
    const float* ub = a.u + ((long long)b * a.N_max + n0) * tv.K * KK;

    float2 x[TB][TB];
#pragma unroll
    for (int r = 0; r < TB; ++r)
#pragma unroll
        for (int c = 0; c < TB; ++c) {
            const int row = ti + NT * r, col = tj + NT * c;
            if (valid && a.X0 && !a.compose)
                x[r][c] = a.X0[(long long)b * D * D + row * D + col];
            else
                x[r][c] = make_float2(row == col ? 1.f : 0.f, 0.f);
        }

    double obs_norm = 1.0;
    // the observable's row lists, once per workgroup, after the instances' buffers
    float2* ovs = reinterpret_cast<float2*>(hdr + (HDR ? IPB * tv.K : 0));
    int* ocs = reinterpret_cast<int*>(ovs + (a.obs_out ? D * a.obs_width : 0));
    if (a.obs_out) {
        for (int e = tid; e < D * a.obs_width; e += 256) {
            ovs[e] = a.obs_vals[e];
            ocs[e] = a.obs_cols[e];
        }
        __syncthreads();
        // Tr(M M) = sum of |M_ab|^2 over the row lists (M Hermitian)
        double s = 0.0;
        for (int e = lt; e < D * a.obs_width; e += TPI) {
            const float2 v = ovs[e];
            s += (double)v.x * v.x + (double)v.y * v.y;
        }
        obs_norm = inst_sum<D>(s, red);
    }
    // An observable with M_ac = f(a XOR c) (the collective transverse magnetisation of
    // Sec. IV is one), checked here on the device: every row's list is row 0's with its
    // columns XORed by the row index, no duplicate columns, at most XMAX terms.  Then
    // (X M)_ab = sum_t conj(f_t) X_{a, b^m_t} and (M X)_ab = sum_t f_t X_{a^m_t, b} need
    // no list: for an instance inside one wave (d <= 16) the partner entries are lane
    // shuffles (low bits of the mask) and the thread's own other sub-block entry (the
    // high bit).
    constexpr int XMAX = 8;
    int nmask = 0;
    int mk[XMAX];
    float2 fv[XMAX];
    if constexpr (TPI <= 64) {
        __shared__ int xor_ok;
        if (a.obs_out) {
            if (tid == 0) xor_ok = 1;
            __syncthreads();
            const int w = a.obs_width;
            for (int ra = tid; ra < D; ra += 256) {
                int cnt = 0, cnt0 = 0;
                bool ok = true;
                for (int e = 0; e < w; ++e) {
                    const float2 v0 = ovs[e];
                    if (v0.x != 0.f || v0.y != 0.f) ++cnt0;
                    const float2 v = ovs[ra * w + e];
                    if (v.x == 0.f && v.y == 0.f) continue;
                    ++cnt;
                    const int c = ocs[ra * w + e];
                    bool found = false;
                    for (int e0 = 0; e0 < w; ++e0) {
                        const float2 u0 = ovs[e0];
                        if ((u0.x != 0.f || u0.y != 0.f) && ocs[e0] == (c ^ ra) && u0.x == v.x && u0.y == v.y)
                            found = true;
                    }
                    for (int e2 = 0; e2 < e; ++e2) {
                        const float2 u2 = ovs[ra * w + e2];
                        if ((u2.x != 0.f || u2.y != 0.f) && ocs[ra * w + e2] == c) ok = false;   // duplicate
                    }
                    ok = ok && found;
                }
                if (!ok || cnt != cnt0 || cnt0 > XMAX) atomicAnd(&xor_ok, 0);
            }
            __syncthreads();
#pragma unroll
            for (int t = 0; t < XMAX; ++t) {
                mk[t] = 0;
                fv[t] = make_float2(0.f, 0.f);
            }
            if (xor_ok) {
                for (int e = 0; e < w; ++e) {
                    const float2 v = ovs[e];
                    if (v.x == 0.f && v.y == 0.f) continue;
                    // compile-time register indices (a runtime index would put the arrays in scratch)
#pragma unroll
                    for (int t = 0; t < XMAX; ++t)
                        if (t == nmask) {
                            mk[t] = ocs[e];
                            fv[t] = v;
                        }
                    ++nmask;
                }
            }
        }
    }
    float2 dph[TB];
    double2 dph64[TB];
    drift_phases<D>(tv, drift, ti, dph, dph64);
    for (int n = 0; n < N; ++n) {
        const bool active = valid && n < len;
        step_left<D, Cfg<D>::MF, HDR>(tv, x, Xs, Fs, Rs, ub + (long long)n * tv.K * KK, drift, active, HDR || lt == 0, lt, ti, tj, dph, dph64, hd, g2s, gs);
        if (a.reproject_every > 0 && !a.compose && ((a.step_offset + n + 1) % a.reproject_every) == 0)
            reproject<D>(x, Xs, Fs, Rs, active, ti, tj, red, tv.flags, lt == 0);
        if (a.X_prefix && active) {
            float2* dst = a.X_prefix + ((long long)b * a.N_max + n) * D * D;
#pragma unroll
            for (int r = 0; r < TB; ++r)
#pragma unroll
                for (int c = 0; c < TB; ++c) dst[(ti + NT * r) * D + tj + NT * c] = x[r][c];
        }
        if (a.obs_out && nmask > 0) {
            // m_n = sum_ab (X M)_ab conj((M X)_ab) / Tr(M M) with the XOR masks (lane shuffles)
            float2 xm[TB][TB], mx[TB][TB];
#pragma unroll
            for (int r = 0; r < TB; ++r)
#pragma unroll
                for (int c = 0; c < TB; ++c) xm[r][c] = mx[r][c] = make_float2(0.f, 0.f);
#pragma unroll
            for (int t = 0; t < XMAX; ++t) {
                if (t >= nmask) break;                        // the same for every lane
                const int ml = mk[t] % NT, mh = mk[t] / NT;   // mh is 0 or 1 (TB = 2)
                const float2 f = fv[t];
#pragma unroll
                for (int r = 0; r < TB; ++r)
#pragma unroll
                    for (int c = 0; c < TB; ++c) {
                        // X_{a, b^m}: lane tj ^ ml, own column c ^ mh;  X_{a^m, b}: lane ti ^ ml, row r ^ mh
                        const float2 sc = mh ? x[r][c ^ 1] : x[r][c];
                        const float2 sr = mh ? x[r ^ 1][c] : x[r][c];
                        float2 vc = sc, vr = sr;
                        if (ml) {
                            vc = make_float2(__shfl_xor(sc.x, ml, 64), __shfl_xor(sc.y, ml, 64));
                            vr = make_float2(__shfl_xor(sr.x, ml * NT, 64), __shfl_xor(sr.y, ml * NT, 64));
                        }
                        cfma(xm[r][c], vc, cconj(f));
                        cfma(mx[r][c], f, vr);
                    }
            }
            double acc = 0.0;
            if (active) {
#pragma unroll
                for (int r = 0; r < TB; ++r)
#pragma unroll
                    for (int c = 0; c < TB; ++c) acc += (double)xm[r][c].x * mx[r][c].x + (double)xm[r][c].y * mx[r][c].y;
            }
            acc = inst_sum<D>(acc, red);
            if (active && lt == 0) a.obs_out[(long long)b * a.N_max + n] = acc / obs_norm;
        } else if (a.obs_out) {
            // m_n = sum_ab (X M)_ab conj((M X)_ab) / Tr(M M)
            inst_sync<D>();
            if (active) store_block<D>(Xs, x, ti, tj);
            inst_sync<D>();
            double acc = 0.0;
            if (active) {
#pragma unroll
                for (int r = 0; r < TB; ++r)
#pragma unroll
                    for (int c = 0; c < TB; ++c) {
                        const int ra = ti + NT * r, cb = tj + NT * c;
                        float2 xm = make_float2(0.f, 0.f), mx = make_float2(0.f, 0.f);
                        for (int t = 0; t < a.obs_width; ++t) {
                            const int colb = ocs[cb * a.obs_width + t];
                            cfma(xm, Xs[lidx<D>(ra, colb)], cconj(ovs[cb * a.obs_width + t]));
                            const int cola = ocs[ra * a.obs_width + t];
                            cfma(mx, ovs[ra * a.obs_width + t], Xs[lidx<D>(cola, cb)]);
                        }
                        acc += (double)xm.x * mx.x + (double)xm.y * mx.y;
                    }
            }
            acc = inst_sum<D>(acc, red);
            if (active && lt == 0) a.obs_out[(long long)b * a.N_max + n] = acc / obs_norm;
        }
    }
    if (valid) {
        float2* dst = a.X_out + (long long)inst * D * D;
#pragma unroll
        for (int r = 0; r < TB; ++r)
#pragma unroll
            for (int c = 0; c < TB; ++c) dst[(ti + NT * r) * D + tj + NT * c] = x[r][c];
    }
}

// ---------------------------------------------------------------- GRAPE kernel
// With the step propagators composed beforehand (one chain launch in compose mode, every
// (instance, step) in parallel), a scan step is one product with the stored U_n:
// x <- U_n x (forward and recompute) or l <- l U_n (backward).
template <int D, bool MM>
__device__ inline void pre_left(float2 (&x)[Cfg<D>::TB][Cfg<D>::TB], float2* Xs, float2* Fs, float2* Rs,
                                const float2* Un, bool active, int lt, int ti, int tj) {
    FactorRegs<D> fr;
    if (active) fetch_factor<D>(fr, Un, lt);
    inst_sync<D>();
    if (active) {
        put_factor<D>(Fs, fr, false, lt);
        store_block<D>(Xs, x, ti, tj);
    }
    inst_sync<D>();
    if (active) mul_left<D, MM>(x, Fs, Xs, Rs, ti, tj);
}
template <int D, bool MM>
__device__ inline void pre_right(float2 (&l)[Cfg<D>::TB][Cfg<D>::TB], float2* Ls, float2* Fs, float2* Rs,
                                 const float2* Un, bool active, int lt, int ti, int tj) {
    FactorRegs<D> fr;
    if (active) fetch_factor<D>(fr, Un, lt);
    inst_sync<D>();
    if (active) {
        put_factor<D>(Fs, fr, false, lt);
        store_block<D>(Ls, l, ti, tj);
    }
    inst_sync<D>();
    if (active) mul_left<D, MM>(l, Ls, Fs, Rs, ti, tj);
}

// Per instance: forward chain with checkpoints, overlap g, then for every
// checkpoint segment from the last: recompute its states, and walk it
// backwards with L_N = U_f^dag, Y_n = X_n L_n, L_{n-1} = L_n U_n.
template <int D>
__device__ inline void load_block(float2 (&x)[Cfg<D>::TB][Cfg<D>::TB], const float2* src, int ti, int tj) {
    constexpr int TB = Cfg<D>::TB, NT = Cfg<D>::NT;
#pragma unroll
    for (int r = 0; r < TB; ++r)
#pragma unroll
        for (int c = 0; c < TB; ++c) x[r][c] = src[(ti + NT * r) * D + tj + NT * c];
}
template <int D>
__device__ inline void save_block(const float2 (&x)[Cfg<D>::TB][Cfg<D>::TB], float2* dst, int ti, int tj) {
    constexpr int TB = Cfg<D>::TB, NT = Cfg<D>::NT;
#pragma unroll
    for (int r = 0; r < TB; ++r)
#pragma unroll
        for (int c = 0; c < TB; ++c) dst[(ti + NT * r) * D + tj + NT * c] = x[r][c];
}

// PRE: the step propagators are in a.Up (pre_left / pre_right), else built from the factors
template <int D, int PH, bool PRE>
__global__ __launch_bounds__(256) void small_grape_kernel(TView tv_in, SmallGrapeArgs a) {
    TView tv = tv_in;
    tv.phased = PH;
    constexpr int TB = Cfg<D>::TB, NT = Cfg<D>::NT, TPI = Cfg<D>::TPI, IPB = Cfg<D>::IPB;
    constexpr int NW = TPI > 64 ? TPI / 64 : 1;   // waves per instance
    extern __shared__ float2 lds[];
    __shared__ double red[4];
    __shared__ double tred[NW > 1 ? KMAX * 6 * NW : 1];   // per-wave partial traces [k][6][wave]
    __shared__ int nblk;
    const int tid = threadIdx.x, slot = tid / TPI, lt = tid % TPI;
    const int ti = lt / NT, tj = lt % NT;
    const int b = blockIdx.x * IPB + slot;
    const bool valid = b < a.B;
    constexpr bool HDR = Cfg<D>::HDR || PH == 1;
    __shared__ signed char g2s[HDR ? KMAX * D : 1];
    __shared__ double gs[HDR ? KMAX * D : 1];
    stage_generators<D, HDR>(tv, g2s, gs);
    // step headers per instance, after the instances' buffers: [0] the forward and recompute scans,
    // [1 + (s & 1)] backward step s, K channels each
    ChanHdr* hdr = reinterpret_cast<ChanHdr*>(lds + (long long)IPB * (Cfg<D>::NBUF_GRAPE * D * D + Cfg<D>::PAD));
    ChanHdr* hF = hdr + (HDR ? slot * 3 * tv.K : 0);
    ChanHdr* hB = hF + (HDR ? tv.K : 0);
    float2* Xs = lds + (long long)slot * (Cfg<D>::NBUF_GRAPE * D * D + Cfg<D>::PAD);
    float2* Fs = Xs + D * D;
    float2* Ls = Fs + D * D;
    float2* Rs = Ls + D * D;   // product results (matrix-core products)
    const int len = valid ? (a.n_steps ? a.n_steps[b] : a.N_max) : 0;
    if (tid == 0) nblk = 0;
    __syncthreads();
    if (lt == 0 && len > 0) atomicMax(&nblk, len);
    __syncthreads();
    const int N = nblk;
    const int C = a.checkpoint_every;
    // one segment covers the chain: the forward pass keeps every state in the segment buffer
    // and the backward pass needs no recompute (the same states, bit for bit); uniform per
    // workgroup, as C and N are
    const bool whole = C >= N;
    const int drift = valid ? b % tv.n_drift : 0;
    const int KK = tv.phased ? 2 : 1;
    const long long ustride = (long long)tv.K * KK;
    const float* ub = a.u + (long long)b * a.N_max * ustride;
    float2* ck = a.ckpt + (long long)b * a.n_ckpt * D * D;
    float2* sg = a.seg + (long long)b * C * D * D;

    // ---- forward with checkpoints X_0, X_C, X_2C, ...
    float2 x[TB][TB];
#pragma unroll
    for (int r = 0; r < TB; ++r)
#pragma unroll
        for (int c = 0; c < TB; ++c) x[r][c] = make_float2((ti + NT * r) == (tj + NT * c) ? 1.f : 0.f, 0.f);
    float2 dph[TB], dpc[TB];
    double2 dph64[TB], dpc64[TB];
    drift_phases<D>(tv, drift, ti, dph, dph64);
    drift_phases<D>(tv, drift, tj, dpc, dpc64);
    for (int n = 0; n < N; ++n) {
        const bool active = valid && n < len;
        if (active && n % C == 0) save_block<D>(x, ck + (long long)(n / C) * D * D, ti, tj);
        if constexpr (PRE)
            pre_left<D, Cfg<D>::MFG>(x, Xs, Fs, Rs, a.Up + ((long long)b * a.N_max + n) * D * D, active, lt, ti, tj);
        else
            step_left<D, Cfg<D>::MFG, HDR>(tv, x, Xs, Fs, Rs, ub + n * ustride, drift, active, HDR || lt == 0, lt, ti, tj, dph, dph64, hF, g2s, gs);
        if (whole && active) save_block<D>(x, sg + (long long)n * D * D, ti, tj);
    }
    // ---- overlap g = Tr(U_f^dag X_N) / Tr(U_f^dag U_f)
    const float2* Uf = a.U_target + (long long)(valid ? b : 0) * D * D;
    double gr = 0.0, gi = 0.0, nu = 0.0;
    if (valid) {
#pragma unroll
        for (int r = 0; r < TB; ++r)
#pragma unroll
            for (int c = 0; c < TB; ++c) {
                const float2 f = Uf[(ti + NT * r) * D + tj + NT * c];
                gr += (double)f.x * x[r][c].x + (double)f.y * x[r][c].y;
                gi += (double)f.x * x[r][c].y - (double)f.y * x[r][c].x;
                nu += (double)f.x * f.x + (double)f.y * f.y;
            }
    }
    gr = inst_sum<D>(gr, red);
    gi = inst_sum<D>(gi, red);
    nu = inst_sum<D>(nu, red);
    gr /= nu;
    gi /= nu;
    if (valid && lt == 0) {
        a.fidelity[b] = gr * gr + gi * gi;
        if (a.overlap) a.overlap[b] = make_double2(gr, gi);
    }
    // ---- backward: L_N = U_f^dag
    float2 l[TB][TB];
#pragma unroll
    for (int r = 0; r < TB; ++r)
#pragma unroll
        for (int c = 0; c < TB; ++c) l[r][c] = cconj(Uf[(tj + NT * c) * D + ti + NT * r]);
    bool has_pend = false;
    int pend_step = -1;
    const double scale = 2.0 / nu;   // dF = 2 Re(conj(g) dg) with the 1/nu of g folded in
    float* gb = a.grad + (long long)b * a.N_max * ustride;
    double* pb_ = a.pend + (long long)(valid ? b : 0) * tv.K * 6;   // [K][6]: T1 re/im, T2 re/im, D re/im
    // zero the gradient of steps past this instance's length
    if (valid)
        for (long long e = (long long)len * ustride + lt; e < (long long)a.N_max * ustride; e += TPI) gb[e] = 0.f;

    // gradient of channel k of step s from its traces (pb_[k]) and D of the earlier state
    auto finalize = [&](int s, int k, double Dr, double Di) {
        const float* us = ub + (long long)s * ustride;
        const double* pk = pb_ + k * 6;
        const ChanHdr* hs = hB + (s & 1) * tv.K;   // step s's header (HDR), intact until step s - 2
        const int q = HDR ? hs[k].q : quantise_one(us + KK * k, tv.phased, tv.eps, tv.qmax, nullptr, nullptr);
        auto im_gc = [&](double zr, double zi) { return gr * zi - gi * zr; };   // Im(conj(g) z)
        if (!tv.phased) {
            gb[(long long)s * ustride + k] = (float)(scale * tv.dt * im_gc(pk[0], pk[1]));
        } else if (q == 0) {
            gb[(long long)s * ustride + 2 * k] = (float)(scale * tv.dt * im_gc(pk[0], pk[1]));
            gb[(long long)s * ustride + 2 * k + 1] = (float)(scale * tv.dt * im_gc(pk[2], pk[3]));
        } else {
            const double om = (double)q * tv.eps;
            const double dFo = scale * tv.dt * im_gc(pk[0], pk[1]);
            const double dFp = scale * im_gc(pk[4] - Dr, pk[5] - Di);
            // cos and sin of phi = atan2(u_y, u_x): the pair over its modulus (q != 0: finite, nonzero)
            const double ux = HDR ? hs[k].ux : us[2 * k], uy = HDR ? hs[k].uy : us[2 * k + 1];
            const double mu = sqrt(ux * ux + uy * uy);
            const double cp = ux / mu, sp = uy / mu;
            gb[(long long)s * ustride + 2 * k] = (float)(cp * dFo - sp * dFp / om);
            gb[(long long)s * ustride + 2 * k + 1] = (float)(sp * dFo + cp * dFp / om);
        }
    };

    // the traces of channel k of the current step: complete the pending (later) step's
    // gradient with this step's D, then keep them as pending
    auto commit = [&](int k, const double (&v6)[6]) {
        if (has_pend) finalize(pend_step, k, v6[4], v6[5]);
        double* pk = pb_ + k * 6;
#pragma unroll
        for (int j = 0; j < 6; ++j) pk[j] = v6[j];
    };

    const int nseg = (N + C - 1) / C;
    for (int sgi = nseg - 1; sgi >= 0; --sgi) {
        const int s0 = sgi * C, s1 = min(N, s0 + C);
        // recompute X_{s0+1} .. X_{s1} into the segment buffer (kept by the forward pass when
        // one segment covers the chain)
        const bool seg_active = valid && s0 < len && !whole;
        if (seg_active) load_block<D>(x, ck + (long long)sgi * D * D, ti, tj);
        for (int n = s0; n < (whole ? s0 : s1); ++n) {
            const bool active = valid && n < len;
            if constexpr (PRE)
                pre_left<D, Cfg<D>::MFG>(x, Xs, Fs, Rs, a.Up + ((long long)b * a.N_max + n) * D * D, active, lt, ti, tj);
            else
                step_left<D, Cfg<D>::MFG, HDR>(tv, x, Xs, Fs, Rs, ub + n * ustride, drift, active, false, lt, ti, tj, dph, dph64, hF, g2s, gs);
            if (active) save_block<D>(x, sg + (long long)(n - s0) * D * D, ti, tj);
        }
        for (int s = s1 - 1; s >= s0; --s) {
            const bool active = valid && s < len;
            // step s's header: its buffer last served step s + 2, whose readers are all past the
            // barriers of step s + 1; the barriers below publish it
            ChanHdr* hs = hB + (s & 1) * tv.K;
            if constexpr (HDR) make_header<D>(tv, ub + (long long)s * ustride, active, false, lt, hs);
            // Y_{s+1} = X_{s+1} L_{s+1}
            inst_sync<D>();
            if (active) {
                float2 xs[TB][TB];
                load_block<D>(xs, sg + (long long)(s - s0) * D * D, ti, tj);
                store_block<D>(Xs, xs, ti, tj);
                store_block<D>(Ls, l, ti, tj);
            }
            inst_sync<D>();
            float2 y[TB][TB];
            if (active) mul_left<D, Cfg<D>::MFG>(y, Xs, Ls, Rs, ti, tj);
            // traces per channel; lane 0 completes the gradient of the pending (later) step
            const float* us = ub + (long long)s * ustride;
            for (int k = 0; k < tv.K; ++k) {
                double phi = 0.0;
                int q = 0;
                if (active) {
                    if constexpr (HDR) {
                        q = hs[k].q;
                        if (!tv.g2) phi = hs[k].rot.x;
                    } else if (tv.g2) {
                        q = quantise_one(us + KK * k, tv.phased, tv.eps, tv.qmax, nullptr, nullptr);
                    } else {
                        q = quantise_one(us + KK * k, tv.phased, tv.eps, tv.qmax, &phi, nullptr);
                    }
                }
                const bool origin = tv.phased && q == 0;
                const double psi = tv.phased ? (origin ? 0.0 : phi) : 0.0;
                // half-integer generators: exp(i psi / 2) from the pair, and exp(i pi / 4) at the origin
                double2 hp = make_double2(1.0, 0.0);
                if (tv.g2 && tv.phased && !origin && active)
                    hp = HDR ? hs[k].rot : half_phase((double)us[2 * k], (double)us[2 * k + 1]);
                const double2 hq = make_double2(0.70710678118654752, 0.70710678118654752);
                double tr = 0.0, tim = 0.0, ur = 0.0, ui = 0.0, dr = 0.0, di = 0.0;
                if (active) {
                    const double* gk = tv.phased ? (HDR ? (const double*)gs : tv.g) + (long long)k * D : nullptr;
                    const float2* Sk = tv.S + (long long)k * D * D;
                    // exp(-i psi (g_aa - g_bb)) = pa[c] pb[r] (aa = column index of the block, bb = row);
                    // Strang: the generator seen by the trace is V(dt/2) S V(dt/2)^dag, one more phase
                    // exp(-i dt/2 (h_aa - h_bb)) in both products
                    double2 pa[TB], pb[TB], qa[TB], qb[TB];
#pragma unroll
                    for (int t2 = 0; t2 < TB; ++t2) {
                        pa[t2] = make_double2(1.0, 0.0);
                        pb[t2] = make_double2(1.0, 0.0);
                        if (tv.strang) {
                            pa[t2] = expmi(0.5 * tv.dt * tv.h[(long long)drift * D + tj + NT * t2]);
                            pb[t2] = zconj(expmi(0.5 * tv.dt * tv.h[(long long)drift * D + ti + NT * t2]));
                        }
                        qa[t2] = pa[t2];
                        qb[t2] = pb[t2];
                        if (gk && tv.g2) {
                            const signed char* g2k = (HDR ? (const signed char*)g2s : tv.g2) + (long long)k * D;
                            if (!origin) {
                                pa[t2] = zmul(pa[t2], zconj(zpow(hp, g2k[tj + NT * t2])));
                                pb[t2] = zmul(pb[t2], zpow(hp, g2k[ti + NT * t2]));
                            } else {
                                qa[t2] = zmul(qa[t2], zconj(zpow(hq, g2k[tj + NT * t2])));
                                qb[t2] = zmul(qb[t2], zpow(hq, g2k[ti + NT * t2]));
                            }
                        } else {
                            if (gk && psi != 0.0) {
                                pa[t2] = zmul(pa[t2], expmi(psi * gk[tj + NT * t2]));
                                pb[t2] = zmul(pb[t2], zconj(expmi(psi * gk[ti + NT * t2])));
                            }
                            if (origin) {
                                qa[t2] = zmul(qa[t2], expmi(1.5707963267948966 * gk[tj + NT * t2]));
                                qb[t2] = zmul(qb[t2], zconj(expmi(1.5707963267948966 * gk[ti + NT * t2])));
                            }
                        }
                    }
#pragma unroll
                    for (int r = 0; r < TB; ++r)
#pragma unroll
                        for (int c = 0; c < TB; ++c) {
                            // y[r][c] = Y[bb][aa], contributes S^psi[aa][bb] Y[bb][aa]
                            const int bb = ti + NT * r, aa = tj + NT * c;
                            const float2 sv = Sk[aa * D + bb];
                            const double yr = y[r][c].x, yi = y[r][c].y;
                            const double2 p = zmul(pa[c], pb[r]);
                            const double s_r = p.x * sv.x - p.y * sv.y, s_i = p.x * sv.y + p.y * sv.x;
                            tr += s_r * yr - s_i * yi;
                            tim += s_r * yi + s_i * yr;
                            if (origin) {
                                const double2 e = zmul(qa[c], qb[r]);
                                const double t_r = e.x * sv.x - e.y * sv.y, t_i = e.x * sv.y + e.y * sv.x;
                                ur += t_r * yr - t_i * yi;
                                ui += t_r * yi + t_i * yr;
                            }
                            if (gk && aa == bb) {
                                dr += gk[aa] * yr;
                                di += gk[aa] * yi;
                            }
                        }
                }
                double v6[6] = {tr, tim, ur, ui, dr, di};
                const int nv = tv.phased ? 6 : 2;
                wave_sums<D>(v6);
                if constexpr (NW > 1) {
                    // the wave's partial sums wait in LDS for the one barrier after the last channel
                    if ((lt & 63) == 0)
                        for (int j = 0; j < nv; ++j) tred[(k * 6 + j) * NW + (lt >> 6)] = v6[j];
                } else if (active && lt == 0) {
                    commit(k, v6);
                }
            }
            if constexpr (NW > 1) {
                // one barrier for every channel's traces (instead of two per trace); thread 0 adds
                // the waves' partials in wave order.  The next writes to tred follow the barriers
                // of step_right.
                __syncthreads();
                if (active && lt == 0) {
                    const int nv = tv.phased ? 6 : 2;
                    for (int k = 0; k < tv.K; ++k) {
                        double v6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                        for (int j = 0; j < nv; ++j) {
                            double t = tred[(k * 6 + j) * NW];
#pragma unroll
                            for (int w = 1; w < NW; ++w) t += tred[(k * 6 + j) * NW + w];
                            v6[j] = t;
                        }
                        commit(k, v6);
                    }
                }
            }
            if (active) {
                has_pend = true;
                pend_step = s;
            }
            // L_s = L_{s+1} U_s
            if constexpr (PRE)
                pre_right<D, Cfg<D>::MFG>(l, Ls, Fs, Rs, a.Up + ((long long)b * a.N_max + s) * D * D, active, lt, ti, tj);
            else
                step_right<D, Cfg<D>::MFG, HDR>(tv, l, Ls, Fs, Rs, us, drift, active, lt, ti, tj, dpc, dpc64, hs, g2s, gs);
        }
    }
    // D_0 = Tr(G Y_0), Y_0 = X_0 L_0 = L_0
    for (int k = 0; k < tv.K; ++k) {
        double dr = 0.0, di = 0.0;
        if (valid && tv.phased) {
            const double* gk = tv.g + (long long)k * D;
#pragma unroll
            for (int r = 0; r < TB; ++r)
#pragma unroll
                for (int c = 0; c < TB; ++c)
                    if (ti + NT * r == tj + NT * c) {
                        dr += gk[ti + NT * r] * l[r][c].x;
                        di += gk[ti + NT * r] * l[r][c].y;
                    }
        }
        if (tv.phased) {
            dr = inst_sum<D>(dr, red);
            di = inst_sum<D>(di, red);
        }
        if (valid && lt == 0 && has_pend) finalize(pend_step, k, dr, di);
    }
}

template <int D>
hipError_t launch_chain(const TView& tv, const SmallChainArgs& a, int ninst, hipStream_t st) {
    constexpr int IPB = Cfg<D>::IPB;
    const bool hdr = Cfg<D>::HDR || tv.phased;
    const size_t lds = (size_t)IPB * (Cfg<D>::NBUF_CHAIN * D * D + Cfg<D>::PAD) * sizeof(float2) +
                       (hdr ? (size_t)IPB * tv.K * sizeof(ChanHdr) : 0) +
                       (a.obs_out ? (size_t)D * a.obs_width * (sizeof(float2) + sizeof(int)) : 0);
    const void* k = tv.phased ? (const void*)small_chain_kernel<D, 1> : (const void*)small_chain_kernel<D, 0>;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int grid = (ninst + IPB - 1) / IPB;
    if (tv.phased)
        hipLaunchKernelGGL((small_chain_kernel<D, 1>), dim3(grid), dim3(256), lds, st, tv, a, ninst);
    else
        hipLaunchKernelGGL((small_chain_kernel<D, 0>), dim3(grid), dim3(256), lds, st, tv, a, ninst);
    return hipGetLastError();
}

template <int D>
hipError_t launch_grape(const TView& tv, const SmallGrapeArgs& a, hipStream_t st) {
    constexpr int IPB = Cfg<D>::IPB;
    const bool hdr = Cfg<D>::HDR || tv.phased;
    const size_t lds = (size_t)IPB * (Cfg<D>::NBUF_GRAPE * D * D + Cfg<D>::PAD) * sizeof(float2) +
                       (hdr ? (size_t)IPB * 3 * tv.K * sizeof(ChanHdr) : 0);
    const bool pre = a.Up != nullptr;
    if (pre) {
        // every step's propagator U_n, all (instance, step) pairs in parallel
        SmallChainArgs c{};
        c.u = a.u;
        c.n_steps = a.n_steps;
        c.B = a.B;
        c.N_max = a.N_max;
        c.compose = 1;
        c.X_out = a.Up;
        hipError_t e = launch_chain<D>(tv, c, a.B * a.N_max, st);
        if (e != hipSuccess) return e;
    }
    const void* k = tv.phased ? (pre ? (const void*)small_grape_kernel<D, 1, true> : (const void*)small_grape_kernel<D, 1, false>)
                              : (pre ? (const void*)small_grape_kernel<D, 0, true> : (const void*)small_grape_kernel<D, 0, false>);
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int grid = (a.B + IPB - 1) / IPB;
    if (tv.phased) {
        if (pre)
            hipLaunchKernelGGL((small_grape_kernel<D, 1, true>), dim3(grid), dim3(256), lds, st, tv, a);
        else
            hipLaunchKernelGGL((small_grape_kernel<D, 1, false>), dim3(grid), dim3(256), lds, st, tv, a);
    } else {
        if (pre)
            hipLaunchKernelGGL((small_grape_kernel<D, 0, true>), dim3(grid), dim3(256), lds, st, tv, a);
        else
            hipLaunchKernelGGL((small_grape_kernel<D, 0, false>), dim3(grid), dim3(256), lds, st, tv, a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t small_chain(const redo_table_s* t, const SmallChainArgs& a, hipStream_t st) {
    const TView tv = view_of(t);
    const int ninst = a.compose ? a.B * a.N_max : a.B;
    switch (tv.d) {
        case 2: return launch_chain<2>(tv, a, ninst, st);
        case 4: return launch_chain<4>(tv, a, ninst, st);
        case 8: return launch_chain<8>(tv, a, ninst, st);
        case 16: return launch_chain<16>(tv, a, ninst, st);
        case 32: return launch_chain<32>(tv, a, ninst, st);
        case 64: return launch_chain<64>(tv, a, ninst, st);
        default: return hipErrorInvalidValue;
    }
}

size_t small_grape_workspace_bytes(int d, int K, long long B, long long N_max, long long C) {
    const long long nck = (N_max + C - 1) / C;
    const size_t mats = sizeof(float2) * (size_t)d * d * (size_t)B * (size_t)(nck + C);
    return ((mats + 255) & ~size_t(255)) + sizeof(double) * (size_t)B * K * 6;
}

size_t small_grape_precomposed_bytes(int d, long long B, long long N_max) {
    // only where the fused kernel leaves the chip mostly idle (at most one wave per SIMD across
    // the instances): there its sequence of dependent per-factor products is the time, and the
    // composition, parallel over steps, removes it; a batch that fills the chip gains nothing
    // from the extra pass and the stored propagators' memory traffic
    int tpi = 0;
    switch (d) {
        case 2: tpi = Cfg<2>::TPI; break;
        case 4: tpi = Cfg<4>::TPI; break;
        case 8: tpi = Cfg<8>::TPI; break;
        case 16: tpi = Cfg<16>::TPI; break;
        case 32: tpi = Cfg<32>::TPI; break;
        case 64: tpi = Cfg<64>::TPI; break;
        default: return 0;
    }
    if ((double)B * tpi > (double)SMALL_PRECOMPOSED_MAX_THREADS) return 0;
    const double bytes = (double)sizeof(float2) * d * d * (double)B * (double)N_max;
    return bytes <= (double)SMALL_PRECOMPOSED_MAX ? 256 + (size_t)bytes : 0;
}

hipError_t small_grape(const redo_table_s* t, const SmallGrapeArgs& a, hipStream_t st) {
    const TView tv = view_of(t);
    switch (tv.d) {
        case 2: return launch_grape<2>(tv, a, st);
        case 4: return launch_grape<4>(tv, a, st);
        case 8: return launch_grape<8>(tv, a, st);
        case 16: return launch_grape<16>(tv, a, st);
        case 32: return launch_grape<32>(tv, a, st);
        case 64: return launch_grape<64>(tv, a, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace redo
