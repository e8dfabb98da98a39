// Internal declarations of the REDO library (host and device).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/redo.h"

namespace redo {

// ---------------------------------------------------------------------------
// complex helpers on float2 / double2 (interleaved re, im)
// ---------------------------------------------------------------------------
__host__ __device__ inline float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__host__ __device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 zmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
// a += b * c  (complex)
__device__ inline void cfma(float2& a, float2 b, float2 c) {
    a.x = fmaf(b.x, c.x, a.x);
    a.x = fmaf(-b.y, c.y, a.x);
    a.y = fmaf(b.x, c.y, a.y);
    a.y = fmaf(b.y, c.x, a.y);
}
// exp(-i x) in FP64
__device__ inline double2 expmi(double x) {
    double s, c;
    sincos(x, &s, &c);
    return make_double2(c, -s);
}

// exp(+i phi / 2) for the phase phi = atan2(uy, ux) in (-pi, pi] of a Cartesian
// control pair (signed zeros as atan2; a non-finite pair has phi = 0, as in
// quantise_one), from the half-angle formulas on (ux, uy) / |u|: no
// transcendental function.  The branch keeps both components well conditioned:
// cos(phi/2) >= 1/sqrt(2) when cos(phi) >= 0, else |sin(phi/2)| >= 1/sqrt(2).
__device__ inline double2 half_phase(double ux, double uy) {
    const double om = sqrt(ux * ux + uy * uy);
    if (!(om <= 1.7976931348623157e308)) return make_double2(1.0, 0.0);
    if (om == 0.0) return signbit(ux) ? make_double2(0.0, copysign(1.0, uy)) : make_double2(1.0, copysign(0.0, uy));
    const double c = ux / om, s = uy / om;
    if (c >= 0.0) {
        const double ch = sqrt(0.5 * (1.0 + c));
        return make_double2(ch, s / (2.0 * ch));
    }
    const double sh = sqrt(0.5 * (1.0 - c));
    return make_double2(fabs(s) / (2.0 * sh), copysign(sh, uy));
}

// z^m for an integer m (conj(z)^|m| for m < 0) by repeated products
__device__ inline double2 zpow(double2 z, int m) {
    if (m < 0) {
        z.y = -z.y;
        m = -m;
    }
    double2 r = make_double2(1.0, 0.0);
    for (int i = 0; i < m; ++i) r = make_double2(r.x * z.x - r.y * z.y, r.x * z.y + r.y * z.x);
    return r;
}

// Device-side latched conditions (one per table).
struct DeviceFlags {
    unsigned long long clamped;
    unsigned int nonfinite;
    unsigned int unitarity;           // re-projection steps whose state drifted off unitarity
    unsigned long long max_drift;     // bits of the largest ||X^dag X - I||_F / sqrt(d) seen (a non-negative double)
};

// the unitarity watchdog: a state whose ||X^dag X - I||_F / sqrt(d) exceeds this at a
// re-projection step is counted (the Newton-Schulz step still runs)
constexpr double UNITARITY_WARN = 1e-3;

__device__ inline void report_drift(DeviceFlags* f, double drift) {
    if (!f) return;
    atomicMax(&f->max_drift, (unsigned long long)__double_as_longlong(drift));
    if (!(drift <= UNITARITY_WARN)) atomicAdd(&f->unitarity, 1u);   // NaN counts too
}

// ---------------------------------------------------------------------------
// Coarse graining (Sec. II, Eq. cgrain): the one place where floating point
// decides an integer code.  IEEE FP64 from the FP32 inputs: the squares of
// FP32 values are exact in FP64, so a contracted fma gives the same sum.
// Returns q (negated for a negative signed amplitude); *phi gets atan2.
// ---------------------------------------------------------------------------
__device__ inline int quantise_one(const float* up, int phased, double eps, double qmax,
                                   double* phi, DeviceFlags* flags) {
    double om;
    bool neg = false;
    if (phased) {
        const double ux = up[0], uy = up[1];
        om = sqrt(ux * ux + uy * uy);
        if (phi) *phi = atan2(uy, ux);
    } else {
        const double x = up[0];
        om = fabs(x);
        neg = x < 0.0;
        if (phi) *phi = 0.0;
    }
    if (!(om <= 1.7976931348623157e308)) {  // NaN or Inf
        if (flags) atomicOr(&flags->nonfinite, 1u);
        if (phi) *phi = 0.0;
        return 0;
    }
    double qf = floor(om / eps + 0.5);
    if (qf > qmax) {
        if (flags) atomicAdd(&flags->clamped, 1ull);
        qf = qmax;
    }
    const int q = (int)qf;
    return neg ? -q : q;
}

// digit j of code |q| in base b
__device__ inline int digit_of(int q, int j, int base) {
    int a = q < 0 ? -q : q;
    for (int t = 0; t < j; ++t) a /= base;
    return a % base;
}

}  // namespace redo

// ---------------------------------------------------------------------------
// the opaque table
// ---------------------------------------------------------------------------
struct redo_table_s {
    redo_table_desc desc;
    double qmax;            // b^P - 1
    int64_t entry_elems;    // d*d
    // device buffers owned by the table
    float2* T32 = nullptr;  // [K][P][b-1][d][d]
    double* h64 = nullptr;  // diagonal drifts [n_drift][d] (drift_is_diag)
    float2* V32 = nullptr;  // drift propagators: diag [n_drift][d] or dense [n_drift][d][d]
    double* g64 = nullptr;  // phase generators [K][d] (phased)
    signed char* g2 = nullptr;  // 2 g64 as integers [K][d] when every entry is a half-integer with |2g| <= 64, else null
    float2* S32 = nullptr;  // generators rounded to FP32, [K][d][d]
    float2* Sy32 = nullptr; // y-partners exp(-i pi/2 G) S exp(i pi/2 G) of phased generators, FP32 [K][d][d]
    float2* H32 = nullptr;  // dense drifts rounded to FP32 [n_drift][d][d] (dense drift only)
    std::vector<double> h_norm;  // ||H0_r||_1
    double2* S64 = nullptr; // generators as given (FP64), [K][d][d]: source of every FP64 rebuild
    std::vector<double> s_norm;  // ||S_k||_1
    redo::DeviceFlags* flags = nullptr;
    size_t bytes = 0;
    double drift_max = 0.0;       // unitarity watchdog as read by the last redo_get_device_status
    long long drift_count = 0;
    bool grad_ok = false;   // channels commute with each other, phases with drift
    std::string grad_why;
    // composed level cache (process 3): R(q) for q in [cache_lo, cache_hi]
    float2* cache = nullptr;
    int cache_lo = 0, cache_hi = -1;
    // the same levels as pre-split BF16 panels (hi/lo of re and im) for the split-BF16
    // products, or null; cache_bf_conj: every channel's generator is real, so each cached
    // level is an exactly symmetric matrix and R(-q) = R(q)^H = conj(R(q))
    uint16_t* cache_bf = nullptr;
    bool cache_bf_conj = false;
    std::vector<char> s_real;   // per channel: the generator has no imaginary part
    // sparsity pattern of the generators (union over channels), when every row has at
    // most SPAT_WMAX nonzeros: column lists [d][spat_w] (padded with the row index) and
    // the FP64 values of every channel at those positions [K][d][spat_w] (0 where absent)
    int spat_w = 0;
    int* spat_cols = nullptr;
    double2* spat_vals = nullptr;
    // d = 2^n and every generator a sum of single-spin terms, S_k = sum_q s_kq on spin q
    // (bit q of the basis index): n, and the 2 x 2 terms [K][n][2][2] in FP64; else 0
    int kron_n = 0;
    double2* kron_s = nullptr;
};

constexpr int SPAT_WMAX = 16;

namespace redo {

// error reporting (thread-local string)
redo_status fail(redo_status st, const std::string& msg);
void clear_last_error();
redo_status hip_fail(hipError_t e, const char* what);

#define REDO_HIP(call)                                          \
    do {                                                        \
        hipError_t _e = (call);                                 \
        if (_e != hipSuccess) return ::redo::hip_fail(_e, #call); \
    } while (0)

// ---------------------------------------------------------------------------
// launchers implemented in the .hip files
// ---------------------------------------------------------------------------
// FP64 complex GEMM, batched with strides: C = alpha*A*B + beta*I  (n x n)
hipError_t zgemm_batched(int n, int batch, const double2* A, long long sA, const double2* B,
                         long long sB, double2* C, long long sC, double2 alpha, double beta,
                         hipStream_t st);
hipError_t fill_identity_z(int n, int batch, double2* C, long long sC, hipStream_t st);
hipError_t round_table_entries(int n, int batch, const double2* src, float2* dst, long long dst_batch_stride,
                               hipStream_t st);
hipError_t drift_diag_phases(int d, int n_drift, const double* h, double dt, float2* V, hipStream_t st);
hipError_t round_z_to_c(long long count, const double2* src, float2* dst, hipStream_t st);
// A[b] <- (A[b] + A[b]^T) / 2 in place (n x n c128): the exact symmetry of a level
// whose generator is real, restored after the FP64 products
hipError_t symmetrize_z(int n, int batch, double2* A, long long sA, hipStream_t st);
// pre-split BF16 panels of count d x d FP32 complex matrices (cgemm.hip): entry (i, k) of
// plane p (0 re hi, 1 re lo, 2 im hi, 3 im lo; hi = RNE(x), lo = RNE(x - hi)) at bf16
// offset ((k / 16) d + i) 64 + 16 p + k % 16 of its matrix (8 d^2 bytes per matrix)
hipError_t split_panels(int d, long long count, const float2* src, uint16_t* dst, hipStream_t st);

hipError_t quantise_all(const redo_table_s* t, const float* u, int B, int N, int* codes, double* phi,
                        hipStream_t st);

// small-d fused chain / compose (d <= 64)
struct SmallChainArgs {
    const float* u;          // amplitudes
    const int* n_steps;      // [B] or null
    int B, N_max;            // instance layout of u
    int compose;             // 1: instance = (b, n), one step from identity, output U_out
    int step_offset, reproject_every;
    const float2* X0;        // [B][d][d] or null
    float2* X_out;           // [B][d][d] (chain) or [B][N][d][d] (compose)
    float2* X_prefix;        // [B][N_max][d][d] or null
    const int* obs_cols;
    const float2* obs_vals;
    int obs_width;
    double* obs_out;         // [B][N_max]
};
hipError_t small_chain(const redo_table_s* t, const SmallChainArgs& a, hipStream_t st);

struct SmallGrapeArgs {
    const float* u;
    const int* n_steps;
    int B, N_max;
    const float2* U_target;
    int checkpoint_every;    // > 0
    double* fidelity;
    double2* overlap;
    float* grad;
    float2* ckpt;            // workspace [B][n_ckpt][d][d]
    float2* seg;             // workspace [B][checkpoint_every][d][d]
    double* pend;            // workspace [B][K][6]: traces of the step whose gradient waits for the next D
    int n_ckpt;
    float2* Up;              // workspace [B][N_max][d][d]: the step propagators composed beforehand, or null
};
hipError_t small_grape(const redo_table_s* t, const SmallGrapeArgs& a, hipStream_t st);
// workspace of the fused d <= 64 GRAPE kernel (checkpoints, one segment, pending traces)
size_t small_grape_workspace_bytes(int d, int K, long long B, long long N_max, long long C);
// the further workspace of the precomposed form (every step's U_n, 256-byte aligned start), 0 when
// it would exceed SMALL_PRECOMPOSED_MAX, or when the batch's threads exceed
// SMALL_PRECOMPOSED_MAX_THREADS (one wave per SIMD on 256 CUs); the fused form then builds
// each step from its factors
constexpr size_t SMALL_PRECOMPOSED_MAX = size_t(4) << 30;
// the fused GRAPE (d <= 64) keeps every state of the forward pass (one checkpoint segment, no
// recompute) when the checkpoint interval is left to the library and its workspace stays
// within this; else it checkpoints every ceil(sqrt(N_max)) steps
constexpr size_t SMALL_FULL_STORAGE_MAX = size_t(8) << 30;
constexpr long long SMALL_PRECOMPOSED_MAX_THREADS = 256LL * 4 * 64;
size_t small_grape_precomposed_bytes(int d, long long B, long long N_max);

// fidelity reduction, FP64
hipError_t unitary_fidelity(int d, int B, const float2* Uf, const float2* U, double2* overlap,
                            double* fidelity, hipStream_t st);
// the same over many workgroups per instance (slices), FP64 partials in part
// (fidelity_partial_doubles(B) doubles); also writes nu = Tr(U_f^dag U_f) when nu is not null
size_t fidelity_partial_doubles(int B);
hipError_t unitary_fidelity_sliced(int d, int B, const float2* Uf, long long sf, const float2* U, long long su,
                                   double2* overlap, double* fidelity, double* nu, double* part, hipStream_t st);

// ---------------------------------------------------------------------------
// large-d path (d >= 128, d % 64 == 0): batched complex GEMM on MFMA
// ---------------------------------------------------------------------------
struct GemmDesc {
    const float2* A;     // d x d, or null for A = I
    const float2* B;     // d x d
    float2* C;           // d x d (must not alias A or B)
    const float2* kscale;  // scales row k of B (diag on the right of op(A)), or null
    const float2* rscale;  // scales row i of C, or null
    const float2* cscale;  // scales column j of C, or null
    int opA;             // 0: A, 1: A^H
    int opB;             // 0: B, 1: B^H
    int active;          // 0: skip this entry entirely
    float beta_identity; // C += beta * I after scaling (Newton-Schulz), usually 0
    float alpha;         // C = alpha * (...)
    int conjA;           // with Abf: op(A) = conj(panel matrix), which equals its adjoint (symmetric)
    const float2* addend;  // C += addend (d x d) after alpha, or null
    const uint16_t* Abf;   // op(A) as pre-split BF16 panels (split_panels layout), or null;
                           // read by the split-BF16 product in place of A, which stays valid
};
static_assert(sizeof(GemmDesc) % 8 == 0, "desc alignment");

// role: 0 a REDO chain step product, 1 the plain-exponential comparison point, 2 a
// Newton-Schulz re-projection product, 3 the composition of single step propagators
// (redo_compose_steps, the step factors of GRAPE); each role is a separate kernel
// instantiation (same code), so that profiles attribute time apart.  Role 4 is the Gram
// product of a re-projection, C = alpha A^H A + beta I with alpha, beta real and no
// scaling, addend or null operand: C is Hermitian, so only the tiles that meet the upper
// triangle run and each writes the conjugate of its strictly upper elements below the
// diagonal.  Re-projection launches (roles 2 and 4) are timed as profile kind 2
constexpr int GEMM_ROLE_STEP = 0, GEMM_ROLE_EXPM = 1, GEMM_ROLE_REPROJECT = 2, GEMM_ROLE_COMPOSE = 3,
              GEMM_ROLE_GRAM = 4;
hipError_t cgemm_batched(int d, int batch, const GemmDesc* descs, int precision, hipStream_t st, int role = 0);
// the split-BF16 launch behind cgemm_batched (cgemm_bf16.hip): 128 x 64 tiles when big, else 64 x 64
hipError_t cgemm_bf16_launch(int d, int batch, const GemmDesc* descs, hipStream_t st, int role, bool big);

// launch timing (profile.cpp)
bool profiling_on();
constexpr int PROFILE_KINDS = 3;   // 0: batched GEMM, 1: structure-aware step, 2: re-projection GEMM
void profile_begin(hipStream_t st, void** token, int kind = 0);
void profile_end(hipStream_t st, void* token);

}  // namespace redo
