// Batched complex GEMM on CDNA4 matrix cores for the large-d REDO path.
//
// Every product the method performs at d >= 128 is a dense d x d complex
// contraction: a table factor applied to the chain state (Sec. II, process 2;
// Sec. III, chain of Eq. propUn), a Newton-Schulz re-projection, or a
// backward-scan product of the adjoint.  One launch runs a batch of
// independent products, each described by a GemmDesc:
//
//     C = alpha * diag(rs) op(A) diag(ks) op(B) diag(cs) + beta I
//
// with op in {N, H}; A = NULL means the identity, as does B = NULL: such an
// entry's tiles are scaled copies, done by the same launch.  FP32 complex
// products use v_mfma_f32_32x32x2_f32 either as four real products (4M) or three
// (Gauss, 3M); FP32 accumulation throughout (this file); split-BF16 products are
// in cgemm_bf16.hip.
// Tiles are staged through double-buffered LDS; tiles of one batch entry
// are mapped to one XCD so its operands are shared in that XCD's L2.
#include <cstdlib>
#include <string>

#include "cgemm_common.h"

namespace redo {
namespace {

// registers -> LDS (k-major tiles As[k][i], Bs[k][j]); conjugation, transposition and the k-scaling
// here, the stage's KT scaling factors read from LDS (KSL: ks, prefetched) or from global memory
template <int BM, int BN, bool KSL>
__device__ inline void store_stage(const GemmDesc& g, int k0, const float4 (&ra)[GCfg<BM, BN>::AV],
                                   const float4 (&rb)[GCfg<BM, BN>::BV], const float2* ks, float2* As, float2* Bs) {
    using C = GCfg<BM, BN>;
    const int t = threadIdx.x;
#pragma unroll
    for (int m = 0; m < C::AV; ++m) {
        const int e = t + C::THREADS * m;
        const float4 v = ra[m];
        if (g.opA == 0) {
            const int row = e / (KT / 2), kq = e % (KT / 2);
            As[(2 * kq) * C::LDA + row] = f2(v.x, v.y);
            As[(2 * kq + 1) * C::LDA + row] = f2(v.z, v.w);
        } else {
            const int kr = e / (BM / 2), iq = e % (BM / 2);
            *reinterpret_cast<float4*>(As + kr * C::LDA + 2 * iq) = make_float4(v.x, -v.y, v.z, -v.w);
        }
    }
#pragma unroll
    for (int m = 0; m < C::BV; ++m) {
        const int e = t + C::THREADS * m;
        const float4 v = rb[m];
        if (g.opB == 0) {
            const int kr = e / (BN / 2), jq = e % (BN / 2);
            float2 a = f2(v.x, v.y), b = f2(v.z, v.w);
            if (g.kscale) {
                const float2 s = KSL ? ks[kr] : ldg2(g.kscale + k0 + kr);
                a = cmul(s, a);
                b = cmul(s, b);
            }
            *reinterpret_cast<float4*>(Bs + kr * C::LDB + 2 * jq) = make_float4(a.x, a.y, b.x, b.y);
        } else {
            const int row = e / (KT / 2), kq = e % (KT / 2);
            float2 a = f2(v.x, -v.y), b = f2(v.z, -v.w);
            if (g.kscale) {
                a = cmul(KSL ? ks[2 * kq] : ldg2(g.kscale + k0 + 2 * kq), a);
                b = cmul(KSL ? ks[2 * kq + 1] : ldg2(g.kscale + k0 + 2 * kq + 1), b);
            }
            Bs[(2 * kq) * C::LDB + row] = a;
            Bs[(2 * kq + 1) * C::LDB + row] = b;
        }
    }
}

// MODE 0: 4M, MODE 1: 3M (Gauss).  ROLE separates the instantiations that the
// method's chain step products (0), the plain-exponential comparison point (1), the
// Newton-Schulz re-projections (2) and the composition of single step propagators (3)
// launch, so that profiles attribute their time apart; the code is the same.  The Gram
// role (4, a re-projection's A^H A) runs only the tiles that meet the upper triangle and
// mirrors them (gram_tile, store_c).
template <int BM, int BN, int MODE, int ROLE>
// at least three waves per SIMD: the 3M form then keeps its 96 accumulators in VGPRs
// (167 registers, no spills) instead of two waves with AGPRs, 240 -> 218 ms for 4096
// products at d = 1024; the LDS already bounds every form at three workgroups per CU
__global__ __launch_bounds__(256, 3) void cgemm_kernel(int d, int batch, const GemmDesc* __restrict__ descs) {
    using C = GCfg<BM, BN>;
    __shared__ float2 As[2][KT * C::LDA];
    __shared__ float2 Bs[2][KT * C::LDB];
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
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wi0 = (wave >> 1) * C::WM, wj0 = (wave & 1) * C::WN;
    const int nk = d / KT;
    // k-scaling through LDS for the large tile (big batches: 1.1 % faster at d = 1024); the 64 x 64
    // tile of small batches, latency-bound at two waves per SIMD, was 2 % slower with it
    constexpr bool KSL = BM == 128;
    if constexpr (KSL) {
        ks_fetch(g, 0, Ks);
        if (nk > 1) ks_fetch(g, 1, Ks);
    }
    constexpr int NACC = MODE == 0 ? 2 : 3;
    floatx16 acc[NACC][C::FM][C::FN];
#pragma unroll
    for (int a = 0; a < NACC; ++a)
#pragma unroll
        for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
            for (int jb = 0; jb < C::FN; ++jb)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[a][ib][jb][r] = 0.f;

    float4 ra[C::AV], rb[C::BV];
    load_stage<BM, BN>(g, d, i0, j0, 0, ra, rb);
    if (KSL && g.kscale != nullptr) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // Ks[0], Ks[1] landed
        __syncthreads();
    }
    store_stage<BM, BN, KSL>(g, 0, ra, rb, Ks[0], As[0], Bs[0]);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) load_stage<BM, BN>(g, d, i0, j0, (kt + 1) * KT, ra, rb);
        // slot (kt + 2) % 3 was last read by the store of stage kt - 1, before the previous barrier
        if (KSL && kt + 2 < nk) ks_fetch(g, kt + 2, Ks);
        const float2* Ab = As[buf];
        const float2* Bb = Bs[buf];
#pragma unroll
        for (int kk = 0; kk < KT; kk += 2) {
            const int kr = kk + (lane >> 5);
            float2 a[C::FM], b[C::FN];
#pragma unroll
            for (int ib = 0; ib < C::FM; ++ib) a[ib] = Ab[kr * C::LDA + wi0 + ib * 32 + (lane & 31)];
#pragma unroll
            for (int jb = 0; jb < C::FN; ++jb) b[jb] = Bb[kr * C::LDB + wj0 + jb * 32 + (lane & 31)];
            if constexpr (MODE == 0) {
#pragma unroll
                for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
                    for (int jb = 0; jb < C::FN; ++jb)
                        acc[0][ib][jb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[ib].x, b[jb].x, acc[0][ib][jb], 0, 0, 0);
#pragma unroll
                for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
                    for (int jb = 0; jb < C::FN; ++jb)
                        acc[1][ib][jb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[ib].x, b[jb].y, acc[1][ib][jb], 0, 0, 0);
#pragma unroll
                for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
                    for (int jb = 0; jb < C::FN; ++jb)
                        acc[0][ib][jb] = __builtin_amdgcn_mfma_f32_32x32x2f32(-a[ib].y, b[jb].y, acc[0][ib][jb], 0, 0, 0);
#pragma unroll
                for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
                    for (int jb = 0; jb < C::FN; ++jb)
                        acc[1][ib][jb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[ib].y, b[jb].x, acc[1][ib][jb], 0, 0, 0);
            } else {
#pragma unroll
                for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
                    for (int jb = 0; jb < C::FN; ++jb)
                        acc[0][ib][jb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[ib].x, b[jb].x, acc[0][ib][jb], 0, 0, 0);
#pragma unroll
                for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
                    for (int jb = 0; jb < C::FN; ++jb)
                        acc[1][ib][jb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[ib].y, b[jb].y, acc[1][ib][jb], 0, 0, 0);
#pragma unroll
                for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
                    for (int jb = 0; jb < C::FN; ++jb)
                        acc[2][ib][jb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[ib].x + a[ib].y, b[jb].x + b[jb].y,
                                                                              acc[2][ib][jb], 0, 0, 0);
            }
        }
        if (kt + 1 < nk) store_stage<BM, BN, KSL>(g, (kt + 1) * KT, ra, rb, Ks[(kt + 1) % 3], As[buf ^ 1], Bs[buf ^ 1]);
        if (KSL && g.kscale != nullptr) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this stage's ks_fetch landed
        __syncthreads();
    }
    // epilogue: element (i, j) of a 32x32 block lives in lane j + 32 * ((i / 4) % 2), register 4 * (i / 8) + i % 4
#pragma unroll
    for (int ib = 0; ib < C::FM; ++ib)
#pragma unroll
        for (int jb = 0; jb < C::FN; ++jb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = i0 + wi0 + ib * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
                const int j = j0 + wj0 + jb * 32 + (lane & 31);
                float2 v;
                if constexpr (MODE == 0) {
                    v = f2(acc[0][ib][jb][r], acc[1][ib][jb][r]);
                } else {
                    const float t1 = acc[0][ib][jb][r], t2 = acc[1][ib][jb][r], t3 = acc[2][ib][jb][r];
                    v = f2(t1 - t2, t3 - t1 - t2);
                }
                if (g.rscale) v = cmul(ldg2(g.rscale + i), v);
                if (g.cscale) v = cmul(v, ldg2(g.cscale + j));
                v.x *= g.alpha;
                v.y *= g.alpha;
                if (g.addend) v = cadd(v, ldg2(g.addend + (long long)i * d + j));
                if (i == j) v.x += g.beta_identity;
                store_c<GRAM>(g, d, i, j, v);
            }
}

template <int BM, int BN, int MODE>
hipError_t launch(int d, int batch, const GemmDesc* descs, hipStream_t st, int role) {
    const long long tiles = role == GEMM_ROLE_GRAM ? gram_tile_count<BM, BN>(d) : (long long)(d / BM) * (d / BN);
    const long long blocks = tiles * batch;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    if (role == GEMM_ROLE_GRAM)
        hipLaunchKernelGGL((cgemm_kernel<BM, BN, MODE, GEMM_ROLE_GRAM>), dim3((unsigned)blocks), dim3(256), 0, st, d,
                           batch, descs);
    else if (role == GEMM_ROLE_REPROJECT)
        hipLaunchKernelGGL((cgemm_kernel<BM, BN, MODE, 2>), dim3((unsigned)blocks), dim3(256), 0, st, d, batch, descs);
    else if (role == GEMM_ROLE_COMPOSE)
        hipLaunchKernelGGL((cgemm_kernel<BM, BN, MODE, 3>), dim3((unsigned)blocks), dim3(256), 0, st, d, batch, descs);
    else if (role == GEMM_ROLE_EXPM)
        hipLaunchKernelGGL((cgemm_kernel<BM, BN, MODE, 1>), dim3((unsigned)blocks), dim3(256), 0, st, d, batch, descs);
    else
        hipLaunchKernelGGL((cgemm_kernel<BM, BN, MODE, 0>), dim3((unsigned)blocks), dim3(256), 0, st, d, batch, descs);
    return hipGetLastError();
}

}  // namespace

// precision: 0 = 4M FP32, 1 = 3M FP32, 2 = split BF16 (hi*hi + hi*lo + lo*hi)
hipError_t cgemm_batched(int d, int batch, const GemmDesc* descs, int precision, hipStream_t st, int role) {
    if (d % 64 != 0 || batch < 1) return hipErrorInvalidValue;
    hipError_t e = hipSuccess;
    const bool big = d % 128 == 0 && (long long)(d / 128) * (d / 64) * batch >= 512;
    void* tok = nullptr;
    const bool prof = profiling_on();
    if (prof) profile_begin(st, &tok, role == GEMM_ROLE_REPROJECT || role == GEMM_ROLE_GRAM ? 2 : 0);
    // 128x64 tiles: three workgroups per CU for 4M (64 accumulator registers per lane); 3M (96)
    // is also faster there than on 128x128 tiles (240 vs 280 ms for 4096 products at d = 1024)
    if (precision == 2)
        e = cgemm_bf16_launch(d, batch, descs, st, role, big);
    else if (precision == 1)
        e = big ? launch<128, 64, 1>(d, batch, descs, st, role) : launch<64, 64, 1>(d, batch, descs, st, role);
    else
        e = big ? launch<128, 64, 0>(d, batch, descs, st, role) : launch<64, 64, 0>(d, batch, descs, st, role);
    if (prof) profile_end(st, tok);
    return e;
}

}  // namespace redo
