// Large-dimension REDO path (d >= 128, d % 64 == 0): batched complex GEMMs on MFMA.
#pragma once
#include "redo_internal.h"

namespace redo {

size_t large_workspace_bytes(const redo_table_s* t, int op, int B, int N_max);
size_t large_grape_workspace_bytes(const redo_table_s* t, int B, int N_max, int checkpoint_every);

redo_status large_compose(redo_table_s* t, int precision, const float* u, int B, int N, float* U_out,
                          void* workspace, size_t workspace_bytes, hipStream_t st);

redo_status large_chain(redo_table_s* t, int precision, const float* u, const int* n_steps, int B, int N_max,
                        int step_offset, int reproject_every, const float* X0, float* U_total, const int* obs_cols,
                        const float* obs_vals, int obs_width, double* obs_out, void* workspace,
                        size_t workspace_bytes, hipStream_t st, bool walsh_frame = false, const double* walsh = nullptr);

// expm = 1: the plain per-step exponential with the first-order GRAPE gradient (the comparison point)
redo_status large_grape(redo_table_s* t, int precision, const float* u, const int* n_steps, int B, int N_max,
                        const float* U_target, int checkpoint_every, double* fidelity, double* overlap, float* grad,
                        void* workspace, size_t workspace_bytes, hipStream_t st, int expm);
size_t large_grape_workspace_bytes_mode(const redo_table_s* t, int B, int N_max, int checkpoint_every, int expm);

// plain per-step exponential (expm_path.cpp)
size_t expm_chain_workspace_bytes(const redo_table_s* t, int B, int N);
size_t expm_compose_workspace_bytes(const redo_table_s* t);
redo_status expm_compose_pairs(const redo_table_s* t, int precision, long long I, int N, const float* u, float2* U_out,
                               void* ws, hipStream_t st, int* gemms_per_step);
redo_status expm_chain(redo_table_s* t, int precision, const float* u, const int* n_steps, int B, int N, int step_offset,
                       int reproject_every, const float* X0, float* U_total, const int* obs_cols, const float* obs_vals,
                       int obs_width, double* obs_out, void* workspace, size_t workspace_bytes, hipStream_t st,
                       bool walsh_frame = false, const double* walsh = nullptr, int split = 0);

// ---- kernels of large_kernels.hip
struct PlanLaunch {
    const float2* T;
    const float2* V;
    const double* h;
    const double* g;
    const float2* cache;
    const int* codes;
    const double* phi;
    const int* n_steps;
    long long ent, code_stride;
    int d, K, P, base, n_drift, phased, dense, cache_lo, cache_hi, step, drift_div;
    long long drift_offset;  // instance b of the launch is global index drift_offset + b
    double dt;
    float2* X0;
    float2* X1;
    long long xstride;
    int* loc;
    int compose, slots, all_cached;
    const uint16_t* cache_bf;   // pre-split BF16 panels of the cache (split-BF16 products), or null
    int bf_conj;             // negative levels take the conjugated panel of |q|
    int strang;              // 1: half the drift before the controls, half after
    float2* pre;
    float2* post;
    float2* pstar;
    GemmDesc* descs;
    int B;
};
hipError_t plan_step(const PlanLaunch& p, hipStream_t st);

// inactive_mode: 0 skip the entry, 1 copy op(B) into C, 2 copy op(A) into C
hipError_t fill_descs(GemmDesc* descs, int count, const float2* A, long long sA, int opA, const float2* B,
                      long long sB, int opB, float2* C, long long sC, const int* n_steps, int step,
                      int inactive_mode, float alpha, float beta, hipStream_t st);
size_t observable_partial_doubles(int d, int B);
// T: scratch of `chunk` d x d matrices (instances processed `chunk` at a time)
constexpr int OBS_CHUNK = 256;
constexpr int REPROJECT_CHUNK = 256;   // instances re-projected per launch (scratch bound)

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// bump allocator over the caller's workspace (with base == nullptr it only measures)
struct Carve {
    char* base;
    size_t used = 0;
    explicit Carve(void* p) : base(static_cast<char*>(p)) {}
    template <class T>
    T* take(size_t count) {
        T* p = reinterpret_cast<T*>(base ? base + used : nullptr);
        used += align_up(sizeof(T) * count);
        return p;
    }
};

// structure-aware chain (spin-factorised control blocks), d = 2^n, 128 <= d <= 4096
bool kron_supported(const redo_table_s* t);
size_t kron_workspace_bytes(const redo_table_s* t, int B, int N);
redo_status kron_chain(redo_table_s* t, int quantised, const float* u, const int* n_steps, int B, int N,
                       int step_offset, int reproject_every, const float* X0, float* U_total, const int* obs_cols,
                       const float* obs_vals, int obs_width, double* obs_out, void* workspace, size_t workspace_bytes,
                       hipStream_t st, bool walsh_frame = false, const double* walsh = nullptr);
// walsh_frame: the state is carried in the right Walsh frame, W = X H / sqrt(d) (X0 and U_total
// too; X0 = NULL starts from H / sqrt(d)), and the observable, M = Hn diag(walsh) Hn with walsh
// its spectrum (device, d doubles), is evaluated there in one pass
// GRAPE keeps every forward state and backward factor (no recomputation) when
// that needs at most this much workspace and no checkpoint interval is given
constexpr size_t GRAPE_FULL_STORAGE_BYTES = size_t(48) << 30;
// checkpoint interval used for a requested one (0: automatic)
// descriptors of the paired GRAPE launches of every step i (forward X_{i+1} = U_i X_i, backward
// LH_m = U_m^H LH_{m+1}, m = N - 1 - i): descs[(2 i + which) B + b]
hipError_t grape_pair_descs(GemmDesc* descs, int N, int B, const float2* U, long long sU, float2* X, long long sX,
                            float2* LH, long long sL, long long mat, const int* n_steps, hipStream_t st);
// state-transfer GRAPE on vectors (every d)
size_t state_grape_workspace_bytes(const redo_table_s* t, int B, int N);
redo_status state_grape(redo_table_s* t, const float* u, const int* n_steps, int B, int N, const float* psi0,
                        const float* psif, double* fidelity, double* overlap, float* grad, void* workspace,
                        size_t workspace_bytes, hipStream_t st);
int large_grape_checkpoint(const redo_table_s* t, int B, int N, int requested, int expm);
hipError_t observable(int d, int B, const float2* X0, const float2* X1, const int* loc, long long xstride,
                      const int* cols, const float2* vals, int w, const int* n_steps, int step, double* partial,
                      double* out, long long out_stride, float2* T, int chunk, hipStream_t st);
// observable row lists: the strip layout of the LDS passes and the packed lists
__device__ inline int mx8_off(int a, int col) { return a * 8 + ((((col >> 1) ^ (a >> 2)) & 3) << 1) + (col & 1); }

// the row list of row a from the packed layout [d][WP] (padded entries: column a,
// value 0), as WP/4 + WP/2 16-byte loads
template <int WP>
__device__ inline void obs_list(const int* __restrict__ cols, const float2* __restrict__ vals, int a,
                                int (&cc)[WP], float2 (&cv)[WP]) {
    const int4* c4 = reinterpret_cast<const int4*>(cols + (long long)a * WP);
    const float4* v4 = reinterpret_cast<const float4*>(vals + (long long)a * WP);
#pragma unroll
    for (int q = 0; q < WP / 4; ++q) {
        const int4 x = c4[q];
        cc[4 * q] = x.x;
        cc[4 * q + 1] = x.y;
        cc[4 * q + 2] = x.z;
        cc[4 * q + 3] = x.w;
    }
#pragma unroll
    for (int q = 0; q < WP / 2; ++q) {
        const float4 y = v4[q];
        cv[2 * q] = make_float2(y.x, y.y);
        cv[2 * q + 1] = make_float2(y.z, y.w);
    }
}

// the packed lists live after the partial sums of observable(); obs_pack_lists fills them
void obs_packed_lists(int d, int B, double* partial, int** pc, float2** pv);
hipError_t obs_pack_lists(int d, int B, int w, const int* cols, const float2* vals, double* partial, hipStream_t st);
hipError_t observable_final(int nparts, int B, const double* partial, const float2* vals, int nvals,
                            const int* n_steps, int step, double* out, long long out_stride, hipStream_t st);

// the right Walsh frame W = X H / sqrt(d) (observables with M_ij = f(i XOR j))
bool walsh_dim(int d);   // d = 128 .. 2048, a power of two
hipError_t walsh_fill(int d, int B, float2* X, long long stride, hipStream_t st);
hipError_t walsh_right(int d, int B, float2* X, long long stride, hipStream_t st);   // d = 128 .. 4096
hipError_t observable_walsh(int d, int B, const float2* X0, const float2* X1, const int* loc, long long xstride,
                            const int* cols, const float2* vals, int w, const double* spec, const int* n_steps,
                            int step, double* partial, double* out, long long out_stride, hipStream_t st);
// after phase 0 of a re-projection (E = (I - X^dag X) / 2 for instances b0 .. b0 + count - 1):
// counts every active instance with ||X^dag X - I||_F / sqrt(d) > UNITARITY_WARN in flags
hipError_t unitarity_check(int d, int count, int b0, const float2* E, long long estride, const int* n_steps, int step,
                           DeviceFlags* flags, hipStream_t st);
hipError_t reproject_descs(GemmDesc* descs, int count, int b0, float2* X0, float2* X1, long long xstride, float2* E,
                           long long estride, int* loc, const int* n_steps, int step, int phase, hipStream_t st);
// Newton-Schulz re-projection of every active instance at a re-projection step,
// X <- X (3I - X^dag X) / 2 written as X + X E with E = (I - X^dag X) / 2, REPROJECT_CHUNK
// instances at a time through the scratch E (xstride apart) and descs (REPROJECT_CHUNK
// entries): the Gram product X^dag X at the given GEMM precision (Hermitian: the upper tiles
// only), the unitarity watchdog on E, then X E as a split-BF16 product with X added in FP32
// into the other buffer (loc flips).  E is of the order of the drift, so the split's relative
// error of about 2^-16 in X E stays far below the FP32 rounding of X itself.
hipError_t reproject_states(int d, int B, float2* X0, float2* X1, long long xstride, float2* E, GemmDesc* descs,
                            int* loc, const int* n_steps, int step, int precision, DeviceFlags* flags, hipStream_t st);
hipError_t gather_back(int d, int B, float2* X0, const float2* X1, long long xstride, const int* loc, hipStream_t st);
hipError_t fill_int(int* p, int n, int v, hipStream_t st);
size_t trace_partial_doubles(int d, int B, int K);
// cartesian = 1: every step takes the traces of the x and y generators (first-order GRAPE gradient)
hipError_t traces(int d, int B, int K, int phased, const float2* Y, long long ystride, const float2* S,
                  const double* g, const int* codes, const double* phi, long long code_stride, const int* n_steps,
                  int step, double* partial, double* out, long long out_bstride, int cartesian, hipStream_t st,
                  const double* h = nullptr, int n_drift = 1, double hdt = 0.0);
hipError_t grad_assemble(int B, int N, int K, int phased, double eps, double dt, const int* codes, const double* phi,
                         const double* tr, const double* d0, const double2* overlap, const double* nu,
                         const int* n_steps, float* grad, int cartesian, hipStream_t st);
hipError_t d0_traces(int d, int B, int K, int phased, const float2* L, long long lstride, const double* g, double* d0,
                     hipStream_t st, int conj_l = 0);
size_t sparse_trace_partial_doubles(int d, int B, int steps, int K);
hipError_t sparse_traces(int d, int B, int N, int step0, int steps, int K, int phased, int cartesian, int sw,
                         const float2* X, long long xsb, const float2* LH, long long lsb, const int* spc,
                         const double2* spv, const double* g, const int* codes, const double* phi,
                         const int* n_steps, double* partial, double* tr, hipStream_t st, const double* h,
                         int n_drift, double hdt);
hipError_t fill_identity(int d, int B, float2* X, long long stride, hipStream_t st);

}  // namespace redo
