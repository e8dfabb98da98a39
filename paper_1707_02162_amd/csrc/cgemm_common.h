// Shared pieces of the batched complex GEMM kernels (cgemm.hip: FP32 4M / 3M;
// cgemm_bf16.hip: split BF16): operand accessors, the generic register staging of a
// stage, the k-scaling prefetch into LDS and the identity-operand tiles.
#pragma once

#include "redo_internal.h"

namespace redo {
namespace {


typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int KT = 16;     // complex k per LDS stage
constexpr int NXCD = 8;    // MI355X: 8 XCDs, workgroups dispatched round-robin

template <int BM, int BN>
struct GCfg {
    static constexpr int THREADS = 256;                 // 4 waves, 2 x 2
    static constexpr int WM = BM / 2, WN = BN / 2;      // wave tile
    static constexpr int FM = WM / 32, FN = WN / 32;    // 32x32 MFMA blocks per wave
    static constexpr int LDA = BM + 4, LDB = BN + 4;    // padded LDS rows (complex)
    static constexpr int AV = BM * KT / 2 / THREADS;    // float4 loads of A per thread per stage
    static constexpr int BV = BN * KT / 2 / THREADS;
};

__device__ inline float2 f2(float a, float b) { return make_float2(a, b); }

// The operands come through descriptor pointers, which the compiler cannot
// place in an address space: these accessors mark them as global memory so
// that loads and stores are global (vector-memory counter only) instead of
// flat ones, which would also hold up every LDS wait in the MFMA loop.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const v4f gcv4;
typedef __attribute__((address_space(1))) const v2f gcv2;
typedef __attribute__((address_space(1))) v2f gv2;
__device__ inline float4 ldg4(const float2* p) {
    const v4f v = *(gcv4*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ inline float2 ldg2(const float2* p) {
    const v2f v = *(gcv2*)p;
    return make_float2(v.x, v.y);
}
__device__ inline void stg2(float2* p, float2 v) { *(gv2*)p = v2f{v.x, v.y}; }

// global -> registers for one stage
template <int BM, int BN>
__device__ inline void load_stage(const GemmDesc& g, int d, int i0, int j0, int k0, float4 (&ra)[GCfg<BM, BN>::AV],
                                  float4 (&rb)[GCfg<BM, BN>::BV]) {
    using C = GCfg<BM, BN>;
    const int t = threadIdx.x;
#pragma unroll
    for (int m = 0; m < C::AV; ++m) {
        const int e = t + C::THREADS * m;
        if (g.opA == 0) {
            const int row = e / (KT / 2), kq = e % (KT / 2);
            ra[m] = ldg4(g.A + (long long)(i0 + row) * d + k0 + 2 * kq);
        } else {
            const int kr = e / (BM / 2), iq = e % (BM / 2);
            ra[m] = ldg4(g.A + (long long)(k0 + kr) * d + i0 + 2 * iq);
        }
    }
#pragma unroll
    for (int m = 0; m < C::BV; ++m) {
        const int e = t + C::THREADS * m;
        if (g.opB == 0) {
            const int kr = e / (BN / 2), jq = e % (BN / 2);
            rb[m] = ldg4(g.B + (long long)(k0 + kr) * d + j0 + 2 * jq);
        } else {
            const int row = e / (KT / 2), kq = e % (KT / 2);
            rb[m] = ldg4(g.B + (long long)(j0 + row) * d + k0 + 2 * kq);
        }
    }
}

// The KT k-scaling factors of stage s into LDS (ring slot s % 3) by the first 2 KT lanes, one
// float each, global -> LDS without registers (a register prefetch would cost the 3M form its
// third wave per SIMD; loading them in store_stage stalled every stage on a global load).  Lane l
// writes LDS byte M0 + 4 l.  Issued from asm so that the compiler, which cannot tell the slot from
// the operand tiles, does not wait for it (and for the tile prefetch) before every LDS read: the
// caller waits on the vector-memory counter before the barrier that publishes the slot.  Loads the
// compiler does not know about only make its own vector-memory waits stricter (in-order counter).
__device__ inline void ks_fetch(const GemmDesc& g, int s, float2 (*Ks)[KT]) {
    if (g.kscale != nullptr && threadIdx.x < 2 * KT) {
        const float* src = reinterpret_cast<const float*>(g.kscale + s * KT) + threadIdx.x;
        const unsigned lds = (unsigned)(size_t)(__attribute__((address_space(3))) float2*)Ks[s % 3];
        // no memory clobber: the slot is read only after two barriers
        asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dword %1, off" ::"s"(lds), "v"(src) : "m0");
    }
}

// An entry with an identity operand: this tile of C = alpha rs o op(X) o (ks or cs) + beta I, no products.
// Gram role: the tiles (ti, tj) that meet the upper triangle j >= i are those with
// tj >= ti BM / BN; they are numbered row-tile by row-tile
template <int BM, int BN>
__host__ __device__ constexpr long long gram_tile_count(int d) {
    static_assert(BM % BN == 0, "row tiles are whole multiples of column tiles");
    return (long long)(d / BM) * (d / BN) - (long long)(BM / BN) * (d / BM) * (d / BM - 1) / 2;
}

template <int BM, int BN>
__device__ inline void gram_tile(int d, int u, int& i0, int& j0) {
    constexpr int q = BM / BN;
    const int cn = d / BN;
    int ti = 0;
    while (u >= cn - q * ti) {   // row-tile ti holds cn - q ti tiles (at least q)
        u -= cn - q * ti;
        ++ti;
    }
    i0 = ti * BM;
    j0 = (q * ti + u) * BN;
}

// the store of element (i, j); in the Gram role only j >= i is stored, the strictly upper
// elements also as their conjugates at (j, i), so each element of C is written once
template <bool GRAM>
__device__ inline void store_c(const GemmDesc& g, int d, int i, int j, float2 v) {
    if constexpr (GRAM) {
        if (j < i) return;
        if (j > i) stg2(g.C + (long long)j * d + i, cconj(v));
    }
    stg2(g.C + (long long)i * d + j, v);
}

__device__ inline void copy_tile(const GemmDesc& g, int d, int i0, int j0, int BM, int BN) {
    for (int e = threadIdx.x; e < BM * BN; e += blockDim.x) {
        const int i = i0 + e / BN, j = j0 + e % BN;
        const long long ij = (long long)i * d + j, ji = (long long)j * d + i;
        float2 v;
        if (g.A == nullptr && g.B == nullptr) {
            v = f2(i == j ? 1.f : 0.f, 0.f);
            if (g.kscale && i == j) v = ldg2(g.kscale + i);
        } else if (g.A == nullptr) {
            v = g.opB == 0 ? ldg2(g.B + ij) : cconj(ldg2(g.B + ji));   // diag(ks) op(B)
            if (g.kscale) v = cmul(ldg2(g.kscale + i), v);
        } else {
            v = g.opA == 0 ? ldg2(g.A + ij) : cconj(ldg2(g.A + ji));   // op(A) diag(ks)
            if (g.kscale) v = cmul(v, ldg2(g.kscale + j));
        }
        if (g.rscale) v = cmul(ldg2(g.rscale + i), v);
        if (g.cscale) v = cmul(v, ldg2(g.cscale + j));
        v.x *= g.alpha;
        v.y *= g.alpha;
        if (g.addend) v = cadd(v, ldg2(g.addend + ij));
        if (i == j) v.x += g.beta_identity;
        stg2(g.C + ij, v);
    }
}

}  // namespace
}  // namespace redo
