// Split-BF16 batched complex GEMM on CDNA4 matrix cores (precision 2 of the
// large-d path): the GemmDesc contract of cgemm.hip, each FP32 operand carried as
// BF16 hi + lo and every real product formed as hi*hi + hi*lo + lo*hi on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation; the cached levels can be read
// as pre-split panels (split_panels).
#include <cstdlib>
#include <string>

#include "cgemm_common.h"

namespace redo {
namespace {

// ---------------------------------------------------------------------------
// Split-BF16 products: each FP32 operand x is carried as hi = RNE_bf16(x) and
// lo = RNE_bf16(x - hi); a real product is hi*hi + hi*lo + lo*hi on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation (the lo*lo term, ~2^-16
// relative, is dropped).  LDS holds four bf16 planes (re hi, re lo, im hi,
// im lo) per operand, k contiguous, so a lane reads its 8 k-values of one
// row in one 16-byte access.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// round to nearest even in hardware (v_cvt_pk_bf16_f32 on gfx950)
__device__ inline void split_bf16(float x, unsigned short& h, unsigned short& l) {
    const __bf16 hb = (__bf16)x;
    h = __builtin_bit_cast(unsigned short, hb);
    l = __builtin_bit_cast(unsigned short, (__bf16)(x - (float)hb));
}
// two values at once: hp = (hi(b) << 16) | hi(a), lp likewise for the remainders
__device__ inline void split_bf16x2(float a, float b, unsigned& hp, unsigned& lp) {
    unsigned short ha, la, hb, lb;
    split_bf16(a, ha, la);
    split_bf16(b, hb, lb);
    hp = ha | ((unsigned)hb << 16);
    lp = la | ((unsigned)lb << 16);
}

template <int BM, int BN>
struct BCfg {
    static constexpr int THREADS = 256;
    static constexpr int WM = BM / 2, WN = BN / 2;
    static constexpr int FM = WM / 32, FN = WN / 32;
    static constexpr int AV = BM * KT / 2 / THREADS;
    static constexpr int BV = BN * KT / 2 / THREADS;
    // bf16 per plane: 32-byte rows (KT values); the A planes 32 bytes apart beyond their size
    static constexpr int APLANE = BM * KT + 16, BPLANE = BN * KT;
    static constexpr int ASZ = 4 * APLANE, BSZ = 4 * BPLANE;   // bf16 per stage buffer
};

// LDS offset (bf16 units) of element (row, k) of plane p: planes PLANE apart, 32-byte rows whose
// two 16-byte halves swap when bit 2 and bit 3 of the row differ.  With the A planes 32 bytes
// beyond a multiple of 128 bytes apart, every access pattern of the kernel is free of bank
// conflicts: the 16-byte fragment reads of 16 consecutive rows (64 banks per pass), the
// 16-byte stores of 8 lanes (one row, four planes, two halves; or 8 rows of one plane) and the
// 8-byte stores of 16 lanes (8 rows, both quarters of one half) (32 banks per pass on stores).
// Each pattern was checked with the LDS bank-conflict counter; the swap on bit 3 alone left
// every store two-way conflicted.
template <int PLANE>
__device__ inline int pl_off(int row, int p, int k) {
    return p * PLANE + row * KT + ((((k >> 3) ^ (row >> 2) ^ (row >> 3)) & 1) << 3) + (k & 7);
}

// plane p of element e: 0 re hi, 1 re lo, 2 im hi, 3 im lo
template <int BM, int BN, bool KSL>
__device__ inline void store_stage_bf(const GemmDesc& g, int k0, const float4 (&ra)[GCfg<BM, BN>::AV],
                                      const float4 (&rb)[GCfg<BM, BN>::BV], const float2* ks, unsigned short* As,
                                      unsigned short* Bs) {
    using C = BCfg<BM, BN>;
    const int t = threadIdx.x;
#pragma unroll
    for (int m = 0; m < C::AV; ++m) {
        const int e = t + C::THREADS * m;
        const float4 v = ra[m];
        unsigned short h[4], l[4];
        if (g.opA == 0) {
            // elements (row, 2kq) and (row, 2kq + 1): pack pairs along k
            const int row = e / (KT / 2), kq = e % (KT / 2);
            split_bf16(v.x, h[0], l[0]);
            split_bf16(v.y, h[1], l[1]);
            split_bf16(v.z, h[2], l[2]);
            split_bf16(v.w, h[3], l[3]);
            *reinterpret_cast<unsigned*>(As + pl_off<C::APLANE>(row, 0, 2 * kq)) = h[0] | ((unsigned)h[2] << 16);
            *reinterpret_cast<unsigned*>(As + pl_off<C::APLANE>(row, 1, 2 * kq)) = l[0] | ((unsigned)l[2] << 16);
            *reinterpret_cast<unsigned*>(As + pl_off<C::APLANE>(row, 2, 2 * kq)) = h[1] | ((unsigned)h[3] << 16);
            *reinterpret_cast<unsigned*>(As + pl_off<C::APLANE>(row, 3, 2 * kq)) = l[1] | ((unsigned)l[3] << 16);
        } else {
            // A^H: elements (2iq, kr) and (2iq + 1, kr), conjugated
            const int kr = e / (BM / 2), iq = e % (BM / 2);
            split_bf16(v.x, h[0], l[0]);
            split_bf16(-v.y, h[1], l[1]);
            split_bf16(v.z, h[2], l[2]);
            split_bf16(-v.w, h[3], l[3]);
            const int r0 = 2 * iq, r1 = 2 * iq + 1;
            As[pl_off<C::APLANE>(r0, 0, kr)] = h[0];
            As[pl_off<C::APLANE>(r0, 1, kr)] = l[0];
            As[pl_off<C::APLANE>(r0, 2, kr)] = h[1];
            As[pl_off<C::APLANE>(r0, 3, kr)] = l[1];
            As[pl_off<C::APLANE>(r1, 0, kr)] = h[2];
            As[pl_off<C::APLANE>(r1, 1, kr)] = l[2];
            As[pl_off<C::APLANE>(r1, 2, kr)] = h[3];
            As[pl_off<C::APLANE>(r1, 3, kr)] = l[3];
        }
    }
#pragma unroll
    for (int m = 0; m < C::BV; ++m) {
        const int e = t + C::THREADS * m;
        const float4 v = rb[m];
        unsigned short h[4], l[4];
        if (g.opB == 0) {
            // elements (k = kr, j = 2jq) and (kr, 2jq + 1), stored at [j][k]
            const int kr = e / (BN / 2), jq = e % (BN / 2);
            float2 a = f2(v.x, v.y), b = f2(v.z, v.w);
            if (g.kscale) {
                const float2 sc = KSL ? ks[kr] : ldg2(g.kscale + k0 + kr);
                a = cmul(sc, a);
                b = cmul(sc, b);
            }
            split_bf16(a.x, h[0], l[0]);
            split_bf16(a.y, h[1], l[1]);
            split_bf16(b.x, h[2], l[2]);
            split_bf16(b.y, h[3], l[3]);
            const int c0 = 2 * jq, c1 = 2 * jq + 1;
            Bs[pl_off<C::BPLANE>(c0, 0, kr)] = h[0];
            Bs[pl_off<C::BPLANE>(c0, 1, kr)] = l[0];
            Bs[pl_off<C::BPLANE>(c0, 2, kr)] = h[1];
            Bs[pl_off<C::BPLANE>(c0, 3, kr)] = l[1];
            Bs[pl_off<C::BPLANE>(c1, 0, kr)] = h[2];
            Bs[pl_off<C::BPLANE>(c1, 1, kr)] = l[2];
            Bs[pl_off<C::BPLANE>(c1, 2, kr)] = h[3];
            Bs[pl_off<C::BPLANE>(c1, 3, kr)] = l[3];
        } else {
            // B^H: elements (k = 2kq, j = row) and (2kq + 1, row), conjugated: pack along k
            const int row = e / (KT / 2), kq = e % (KT / 2);
            float2 a = f2(v.x, -v.y), b = f2(v.z, -v.w);
            if (g.kscale) {
                a = cmul(KSL ? ks[2 * kq] : ldg2(g.kscale + k0 + 2 * kq), a);
                b = cmul(KSL ? ks[2 * kq + 1] : ldg2(g.kscale + k0 + 2 * kq + 1), b);
            }
            split_bf16(a.x, h[0], l[0]);
            split_bf16(a.y, h[1], l[1]);
            split_bf16(b.x, h[2], l[2]);
            split_bf16(b.y, h[3], l[3]);
            *reinterpret_cast<unsigned*>(Bs + pl_off<C::BPLANE>(row, 0, 2 * kq)) = h[0] | ((unsigned)h[2] << 16);
            *reinterpret_cast<unsigned*>(Bs + pl_off<C::BPLANE>(row, 1, 2 * kq)) = l[0] | ((unsigned)l[2] << 16);
            *reinterpret_cast<unsigned*>(Bs + pl_off<C::BPLANE>(row, 2, 2 * kq)) = h[1] | ((unsigned)h[3] << 16);
            *reinterpret_cast<unsigned*>(Bs + pl_off<C::BPLANE>(row, 3, 2 * kq)) = l[1] | ((unsigned)l[3] << 16);
        }
    }
}

// Split-BF16 staging of op(A) = A and op(B) = B on 128 x 64 tiles: every thread
// takes a run of consecutive k (8 of one row of A as four 16-byte loads; 4 of one
// column of B as four 8-byte loads) and writes each bf16 plane as one 16-byte (A)
// or 8-byte (B) word.  A thread's row is (t & 15) + 16 (t >> 5) with k-half
// (t >> 4) & 1; its B column is (t >> 1) & 63 with k-quarter (t & 1) + 2 (t >> 7),
// so that the words of one store pass fall into distinct LDS banks (pl_off).
template <int BM, int BN>
__device__ constexpr bool bf_fast_tiles() { return BM == 128 && BN == 64; }

// Staging modes of the split-BF16 product, uniform per workgroup: 0 any op(A), op(B)
// (generic loads and splits); 1 A and B as given (A split as loaded); 2 A from its
// pre-split panels (no split), B as given; 3 as 2 with op(A) the conjugate of the
// panel matrix.  Modes 1 to 3 need 128 x 64 tiles.
//
// Mode 2 reads the 128 x 16 tile of op(A) as the 16 KiB of contiguous panel memory
// that hold it: lane l of wave w takes 16 bytes at 4096 w + 1024 m + 16 l (m = 0..3),
// that is row 32 w + 8 m + l / 8, plane (l / 2) % 4, k-half l % 2.
template <int BM, int BN, int MODE>
__device__ inline void load_stage_bf(const GemmDesc& g, int d, int i0, int j0, int k0, float4 (&ra)[GCfg<BM, BN>::AV],
                                     float4 (&rb)[GCfg<BM, BN>::BV]) {
    if constexpr (MODE != 0) {
        static_assert(bf_fast_tiles<BM, BN>(), "staging modes 1 and 2 need 128 x 64 tiles");
        {
            const int t = threadIdx.x;
            if constexpr (MODE >= 2) {
                const float2* sp = reinterpret_cast<const float2*>(g.Abf + ((long long)(k0 / KT) * d + i0) * 64) +
                                   512 * (t >> 6) + 2 * (t & 63);
#pragma unroll
                for (int m = 0; m < 4; ++m) ra[m] = ldg4(sp + 128 * m);
            } else {
                const int row = (t & 15) + 16 * (t >> 5), kh = (t >> 4) & 1;
                const float2* sa = g.A + (long long)(i0 + row) * d + k0 + 8 * kh;
#pragma unroll
                for (int m = 0; m < 4; ++m) ra[m] = ldg4(sa + 2 * m);
            }
            const int j = (t >> 1) & 63, kg = (t & 1) + 2 * (t >> 7);
            const float2* sb = g.B + (long long)(k0 + 4 * kg) * d + j0 + j;
            const float2 v0 = ldg2(sb), v1 = ldg2(sb + d), v2 = ldg2(sb + 2 * (long long)d),
                         v3 = ldg2(sb + 3 * (long long)d);
            rb[0] = make_float4(v0.x, v0.y, v1.x, v1.y);
            rb[1] = make_float4(v2.x, v2.y, v3.x, v3.y);
            return;
        }
    }
    load_stage<BM, BN>(g, d, i0, j0, k0, ra, rb);
}

__device__ inline unsigned pack_bf(unsigned short lo16, unsigned short hi16) { return lo16 | ((unsigned)hi16 << 16); }

template <int BM, int BN, int MODE>
__device__ inline void store_stage_bf_fast(const GemmDesc& g, const float4 (&ra)[GCfg<BM, BN>::AV],
                                           const float4 (&rb)[GCfg<BM, BN>::BV], const float2* ks,
                                           unsigned short* As, unsigned short* Bs) {
    using C = BCfg<BM, BN>;
    const int t = threadIdx.x;
    if constexpr (MODE >= 2) {
        // A from panels: each 16 bytes are 8 k of one plane of one row, stored as loaded
        // (the conjugation of MODE 3 is taken in the products)
        const int lane = t & 63, pl = (lane >> 1) & 3, kh = lane & 1;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int row = 32 * (t >> 6) + 8 * m + (lane >> 3);
            *reinterpret_cast<uint4*>(As + pl_off<C::APLANE>(row, pl, 8 * kh)) = __builtin_bit_cast(uint4, ra[m]);
        }
    } else {
        // A: 8 complex at k = 8 kh .. 8 kh + 7 of one row -> one uint4 per plane
        const int row = (t & 15) + 16 * (t >> 5), kh = (t >> 4) & 1;
        unsigned w[4][4];   // [plane][k pair]
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            split_bf16x2(ra[m].x, ra[m].z, w[0][m], w[1][m]);
            split_bf16x2(ra[m].y, ra[m].w, w[2][m], w[3][m]);
        }
#pragma unroll
        for (int pl = 0; pl < 4; ++pl)
            *reinterpret_cast<uint4*>(As + pl_off<C::APLANE>(row, pl, 8 * kh)) = make_uint4(w[pl][0], w[pl][1], w[pl][2], w[pl][3]);
    }
    {
        // B: 4 complex at k = 4 kg .. 4 kg + 3 of one column -> one uint2 per plane; the
        // two quarters of a half-row are neighbouring lanes (16 lanes: 8 columns x 2)
        const int j = (t >> 1) & 63, kg = (t & 1) + 2 * (t >> 7);
        float2 v[4] = {f2(rb[0].x, rb[0].y), f2(rb[0].z, rb[0].w), f2(rb[1].x, rb[1].y), f2(rb[1].z, rb[1].w)};
        if (g.kscale) {
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) v[kk] = cmul(ks[4 * kg + kk], v[kk]);
        }
        unsigned w[4][2];   // [plane][k pair]
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            split_bf16x2(v[2 * q].x, v[2 * q + 1].x, w[0][q], w[1][q]);
            split_bf16x2(v[2 * q].y, v[2 * q + 1].y, w[2][q], w[3][q]);
        }
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) *reinterpret_cast<uint2*>(Bs + pl_off<C::BPLANE>(j, pl, 4 * kg)) = make_uint2(w[pl][0], w[pl][1]);
    }
}

// Pre-split panels (layout in split_panels): one thread per (matrix, 16-column
// block, row) turns 16 FP32 complex entries into the 128 bytes of four planes,
// with the rounding of split_bf16
__global__ __launch_bounds__(256) void split_panels_kernel(int d, long long count, const float2* __restrict__ src,
                                                           uint16_t* __restrict__ dst) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per = (long long)d * (d / KT);
    if (e >= count * per) return;
    const long long mtx = e / per, r = e % per;
    const int kb = (int)(r / d), i = (int)(r % d);
    const float2* s = src + mtx * d * d + (long long)i * d + kb * KT;
    uint16_t* o = dst + mtx * 4 * d * d + ((long long)kb * d + i) * 64;
    unsigned w[4][8];   // [plane][k pair]
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const float4 v = ldg4(s + 2 * q);
        split_bf16x2(v.x, v.z, w[0][q], w[1][q]);
        split_bf16x2(v.y, v.w, w[2][q], w[3][q]);
    }
    uint4* o4 = reinterpret_cast<uint4*>(o);
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) {
        o4[2 * pl] = make_uint4(w[pl][0], w[pl][1], w[pl][2], w[pl][3]);
        o4[2 * pl + 1] = make_uint4(w[pl][4], w[pl][5], w[pl][6], w[pl][7]);
    }
}

__device__ inline bf16x8 neg8(bf16x8 x) {
    uint4 u = __builtin_bit_cast(uint4, x);
    u.x ^= 0x80008000u;
    u.y ^= 0x80008000u;
    u.z ^= 0x80008000u;
    u.w ^= 0x80008000u;
    return __builtin_bit_cast(bf16x8, u);
}

#define MF16(a, b, c) __builtin_amdgcn_mfma_f32_32x32x16_bf16((a), (b), (c), 0, 0, 0)

// One 128 x 64 (or 64 x 64) output tile; MODE is the staging mode of load_stage_bf, GRAM
// the store of the Gram role (store_c)
template <int BM, int BN, int MODE, bool GRAM>
__device__ __forceinline__ void bf16x3_tile(const GemmDesc& g, int d, int i0, int j0,
                                            unsigned short (*As)[BCfg<BM, BN>::ASZ],
                                            unsigned short (*Bs)[BCfg<BM, BN>::BSZ], float2 (*Ks)[KT]) {
    using C = BCfg<BM, BN>;
    const int nk = d / KT;
    // k-scaling through LDS, prefetched two stages ahead as in cgemm_kernel (128 x 64 tiles)
    constexpr bool KSL = BM == 128;
    if constexpr (KSL) {
        ks_fetch(g, 0, Ks);
        if (nk > 1) ks_fetch(g, 1, Ks);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wi0 = (wave >> 1) * C::WM, wj0 = (wave & 1) * C::WN;
    floatx16 accR[C::FM][C::FN], accI[C::FM][C::FN];
#pragma unroll
    for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
        for (int jb = 0; jb < C::FN; ++jb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                accR[ib][jb][r] = 0.f;
                accI[ib][jb][r] = 0.f;
            }
    float4 ra[C::AV], rb[C::BV];
    load_stage_bf<BM, BN, MODE>(g, d, i0, j0, 0, ra, rb);
    if (KSL && g.kscale != nullptr) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // Ks[0], Ks[1] landed
        __syncthreads();
    }
    if constexpr (MODE != 0)
        store_stage_bf_fast<BM, BN, MODE>(g, ra, rb, Ks[0], As[0], Bs[0]);
    else
        store_stage_bf<BM, BN, KSL>(g, 0, ra, rb, Ks[0], As[0], Bs[0]);
    __syncthreads();
    const int koff = 8 * (lane >> 5);
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) load_stage_bf<BM, BN, MODE>(g, d, i0, j0, (kt + 1) * KT, ra, rb);
        // slot (kt + 2) % 3 was last read by the store of stage kt - 1, before the previous barrier
        if (KSL && kt + 2 < nk) ks_fetch(g, kt + 2, Ks);
        bf16x8 a[C::FM][4], b[C::FN][4], na[C::FM][2];
#pragma unroll
        for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
            for (int pl = 0; pl < 4; ++pl)
                a[ib][pl] = *reinterpret_cast<const bf16x8*>(As[buf] + pl_off<C::APLANE>(wi0 + ib * 32 + (lane & 31), pl, koff));
#pragma unroll
        for (int jb = 0; jb < C::FN; ++jb)
#pragma unroll
            for (int pl = 0; pl < 4; ++pl)
                b[jb][pl] = *reinterpret_cast<const bf16x8*>(Bs[buf] + pl_off<C::BPLANE>(wj0 + jb * 32 + (lane & 31), pl, koff));
        // pi: the imaginary planes that enter Ci, mi: their negatives that enter Cr; MODE 3
        // takes conj(A) by exchanging the two (Ai -> -Ai), at no cost
        bf16x8 pi[C::FM][2], mi[C::FM][2];
#pragma unroll
        for (int ib = 0; ib < C::FM; ++ib) {
            na[ib][0] = neg8(a[ib][2]);
            na[ib][1] = neg8(a[ib][3]);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                pi[ib][h] = MODE == 3 ? na[ib][h] : a[ib][2 + h];
                mi[ib][h] = MODE == 3 ? a[ib][2 + h] : na[ib][h];
            }
        }
        // Cr += Ar Br - Ai Bi,  Ci += Ar Bi + Ai Br; each real product hi*hi + hi*lo + lo*hi
#pragma unroll
        for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
            for (int jb = 0; jb < C::FN; ++jb) accR[ib][jb] = MF16(a[ib][0], b[jb][0], accR[ib][jb]);
#pragma unroll
        for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
            for (int jb = 0; jb < C::FN; ++jb) accI[ib][jb] = MF16(a[ib][0], b[jb][2], accI[ib][jb]);
#pragma unroll
        for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
            for (int jb = 0; jb < C::FN; ++jb) accR[ib][jb] = MF16(a[ib][0], b[jb][1], accR[ib][jb]);
#pragma unroll
        for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
            for (int jb = 0; jb < C::FN; ++jb) accI[ib][jb] = MF16(a[ib][0], b[jb][3], accI[ib][jb]);
#pragma unroll
        for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
            for (int jb = 0; jb < C::FN; ++jb) accR[ib][jb] = MF16(a[ib][1], b[jb][0], accR[ib][jb]);
#pragma unroll
        for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
            for (int jb = 0; jb < C::FN; ++jb) accI[ib][jb] = MF16(a[ib][1], b[jb][2], accI[ib][jb]);
#pragma unroll
        for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
            for (int jb = 0; jb < C::FN; ++jb) accR[ib][jb] = MF16(mi[ib][0], b[jb][2], accR[ib][jb]);
#pragma unroll
        for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
            for (int jb = 0; jb < C::FN; ++jb) accI[ib][jb] = MF16(pi[ib][0], b[jb][0], accI[ib][jb]);
#pragma unroll
        for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
            for (int jb = 0; jb < C::FN; ++jb) accR[ib][jb] = MF16(mi[ib][0], b[jb][3], accR[ib][jb]);
#pragma unroll
        for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
            for (int jb = 0; jb < C::FN; ++jb) accI[ib][jb] = MF16(pi[ib][0], b[jb][1], accI[ib][jb]);
#pragma unroll
        for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
            for (int jb = 0; jb < C::FN; ++jb) accR[ib][jb] = MF16(mi[ib][1], b[jb][2], accR[ib][jb]);
#pragma unroll
        for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
            for (int jb = 0; jb < C::FN; ++jb) accI[ib][jb] = MF16(pi[ib][1], b[jb][0], accI[ib][jb]);
        if (kt + 1 < nk) {
            if constexpr (MODE != 0)
                store_stage_bf_fast<BM, BN, MODE>(g, ra, rb, Ks[(kt + 1) % 3], As[buf ^ 1], Bs[buf ^ 1]);
            else
                store_stage_bf<BM, BN, KSL>(g, (kt + 1) * KT, ra, rb, Ks[(kt + 1) % 3], As[buf ^ 1], Bs[buf ^ 1]);
        }
        if (KSL && g.kscale != nullptr) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this stage's ks_fetch landed
        __syncthreads();
    }
#pragma unroll
    for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
        for (int jb = 0; jb < C::FN; ++jb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = i0 + wi0 + ib * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
                const int j = j0 + wj0 + jb * 32 + (lane & 31);
                float2 v = f2(accR[ib][jb][r], accI[ib][jb][r]);
                if (g.rscale) v = cmul(ldg2(g.rscale + i), v);
                if (g.cscale) v = cmul(v, ldg2(g.cscale + j));
                v.x *= g.alpha;
                v.y *= g.alpha;
                if (g.addend) v = cadd(v, ldg2(g.addend + (long long)i * d + j));
                if (i == j) v.x += g.beta_identity;
                store_c<GRAM>(g, d, i, j, v);
            }
}

template <int BM, int BN, int ROLE>
// ROLE separates instantiations for profiles, and the Gram role (4) runs the upper tiles
// only, as in cgemm_kernel.  At least three waves per SIMD (a 24-byte spill; 211 -> 192 ms
// for 4096 products at d = 1024): the splits keep the vector ALU busy, and a third wave
// hides more of it behind the MFMAs
__global__ __launch_bounds__(256, 3) void cgemm_bf16x3_kernel(int d, int batch, const GemmDesc* __restrict__ descs) {
    using C = BCfg<BM, BN>;
    __shared__ __attribute__((aligned(16))) unsigned short As[2][C::ASZ];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[2][C::BSZ];
    __shared__ float2 Ks[3][KT];   // k-scaling of stages kt, kt + 1, kt + 2
    constexpr bool GRAM = ROLE == GEMM_ROLE_GRAM;
    const int tiles_n = d / BN;
    const int ntile = GRAM ? (int)gram_tile_count<BM, BN>(d) : (d / BM) * tiles_n;
    int bid = blockIdx.x;
    const int nb = gridDim.x;
    if (nb % NXCD == 0) bid = (bid % NXCD) * (nb / NXCD) + bid / NXCD;
    const int be = bid / ntile, tile = bid % ntile;
    const GemmDesc g = descs[be];
    if (!g.active) return;
    int i0, j0;
    if constexpr (GRAM) {
        gram_tile<BM, BN>(d, tile, i0, j0);
    } else {
        i0 = (tile / tiles_n) * BM;
        j0 = (tile % tiles_n) * BN;
    }
    if (g.A == nullptr || g.B == nullptr) {
        copy_tile(g, d, i0, j0, BM, BN);
        return;
    }
    // the staging mode is uniform per workgroup: one inlined copy of the tile per mode
    if constexpr (bf_fast_tiles<BM, BN>()) {
        if (g.opB == 0 && g.Abf) {
            if (g.conjA)
                bf16x3_tile<BM, BN, 3, GRAM>(g, d, i0, j0, As, Bs, Ks);
            else
                bf16x3_tile<BM, BN, 2, GRAM>(g, d, i0, j0, As, Bs, Ks);
            return;
        }
        if (g.opB == 0 && g.opA == 0) {
            bf16x3_tile<BM, BN, 1, GRAM>(g, d, i0, j0, As, Bs, Ks);
            return;
        }
    }
    bf16x3_tile<BM, BN, 0, GRAM>(g, d, i0, j0, As, Bs, Ks);
}

#undef MF16

template <int BM, int BN>
hipError_t launch_bf(int d, int batch, const GemmDesc* descs, hipStream_t st, int role) {
    const long long tiles = role == GEMM_ROLE_GRAM ? gram_tile_count<BM, BN>(d) : (long long)(d / BM) * (d / BN);
    const long long blocks = tiles * batch;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    if (role == GEMM_ROLE_GRAM)
        hipLaunchKernelGGL((cgemm_bf16x3_kernel<BM, BN, GEMM_ROLE_GRAM>), dim3((unsigned)blocks), dim3(256), 0, st, d,
                           batch, descs);
    else if (role == GEMM_ROLE_REPROJECT)
        hipLaunchKernelGGL((cgemm_bf16x3_kernel<BM, BN, 2>), dim3((unsigned)blocks), dim3(256), 0, st, d, batch, descs);
    else if (role == GEMM_ROLE_COMPOSE)
        hipLaunchKernelGGL((cgemm_bf16x3_kernel<BM, BN, 3>), dim3((unsigned)blocks), dim3(256), 0, st, d, batch, descs);
    else if (role == GEMM_ROLE_EXPM)
        hipLaunchKernelGGL((cgemm_bf16x3_kernel<BM, BN, 1>), dim3((unsigned)blocks), dim3(256), 0, st, d, batch, descs);
    else
        hipLaunchKernelGGL((cgemm_bf16x3_kernel<BM, BN, 0>), dim3((unsigned)blocks), dim3(256), 0, st, d, batch, descs);
    return hipGetLastError();
}

}  // namespace

hipError_t split_panels(int d, long long count, const float2* src, uint16_t* dst, hipStream_t st) {
    if (d % KT != 0 || count < 0) return hipErrorInvalidValue;
    const long long threads = count * d * (d / KT);
    if (threads == 0) return hipSuccess;
    const long long blocks = (threads + 255) / 256;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(split_panels_kernel, dim3((unsigned)blocks), dim3(256), 0, st, d, count, src, dst);
    return hipGetLastError();
}

// the split-BF16 launch of cgemm_batched: 128 x 64 tiles when big, else 64 x 64
hipError_t cgemm_bf16_launch(int d, int batch, const GemmDesc* descs, hipStream_t st, int role, bool big) {
    return big ? launch_bf<128, 64>(d, batch, descs, st, role) : launch_bf<64, 64>(d, batch, descs, st, role);
}

}  // namespace redo
