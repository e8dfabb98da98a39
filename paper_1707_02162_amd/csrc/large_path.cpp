// Host orchestration of the large-d REDO path (d >= 128): every product of
// the method is a batched MFMA complex GEMM over the instances of a call.
//
// Chain (Sec. III, Eq. propUn with the split step of Eqs. vn, vnd): per step
// one planning kernel maps the digits of every instance to table entries
// (Sec. II, process 2) and then one batched GEMM per factor slot multiplies
// the states, with the drift and phase scalings fused into the first and last
// slot.  GRAPE (Sec. III): every step propagator is composed once per call,
// the forward chain keeps checkpoints, and the backward scan recomputes each
// segment and runs the products Y = X L and L U_n as one batched launch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "large_path.h"

namespace redo {
namespace {

constexpr int COMPOSE_CHUNK = 64;      // (instance, step) pairs composed per launch

int slots_of(const redo_table_s* t) { return (t->desc.drift_is_diag ? 0 : 1) + t->desc.K * t->desc.digits; }

// every level 0 .. b^P - 1 is in the composed cache: one factor slot per channel
bool all_cached(const redo_table_s* t) { return t->cache && t->cache_lo == 0 && (double)t->cache_hi >= t->qmax; }

int launch_slots(const redo_table_s* t) {
    return (t->desc.drift_is_diag ? 0 : 1) + (all_cached(t) ? t->desc.K : t->desc.K * t->desc.digits);
}

// layout of every workspace; with base == nullptr it only measures
struct ChainWS {
    int* codes;
    double* phi;
    float2* W1;
    float2 *pre, *post, *pstar;
    GemmDesc* descs;
    float2* E;   // re-projection scratch: E = (I - X^dag X) / 2 of a chunk
    double* obs_partial;
    int* loc;
    float2* obsT;
    size_t bytes;
    ChainWS(const redo_table_s* t, int B, int N, void* base) {
        const int d = t->desc.d, K = t->desc.K;
        const size_t mat = (size_t)d * d;
        Carve c(base);
        codes = c.take<int>((size_t)B * N * K);
        phi = c.take<double>((size_t)B * N * K);
        W1 = c.take<float2>(mat * B);
        pre = c.take<float2>((size_t)B * d);
        post = c.take<float2>((size_t)B * d);
        pstar = c.take<float2>((size_t)B * d);
        descs = c.take<GemmDesc>((size_t)std::max(slots_of(t), 2) * B);
        E = c.take<float2>(mat * std::min(B, REPROJECT_CHUNK));
        obs_partial = c.take<double>(observable_partial_doubles(d, B));
        loc = c.take<int>(B);
        obsT = c.take<float2>(mat * std::min(B, OBS_CHUNK));
        bytes = c.used;
    }
};

struct ComposeWS {
    int* codes;
    double* phi;
    float2* tmp;
    float2 *pre, *post, *pstar;
    GemmDesc* descs;
    int* loc;
    size_t bytes;
    ComposeWS(const redo_table_s* t, long long I, void* base) {
        const int d = t->desc.d, K = t->desc.K;
        const size_t mat = (size_t)d * d;
        const int ch = (int)std::min<long long>(I, COMPOSE_CHUNK);
        Carve c(base);
        codes = c.take<int>((size_t)I * K);
        phi = c.take<double>((size_t)I * K);
        tmp = c.take<float2>(mat * ch);
        pre = c.take<float2>((size_t)ch * d);
        post = c.take<float2>((size_t)ch * d);
        pstar = c.take<float2>((size_t)ch * d);
        descs = c.take<GemmDesc>((size_t)slots_of(t) * ch);
        loc = c.take<int>(ch);
        bytes = c.used;
    }
};

struct GrapeWS {
    ComposeWS* comp = nullptr;
    void* comp_base;
    float2* Ustore;
    float2* ckpt;
    float2* seg;
    float2 *Xa, *Xb, *La, *Lb, *Y;
    double* tr;
    double* tpart;
    double* d0;
    double* nu;
    double2* ov;
    double* fpart;
    GemmDesc* descs;
    size_t bytes;
    GrapeWS(const redo_table_s* t, int B, int N, int C, void* base, int expm = 0) {
        const int d = t->desc.d, K = t->desc.K;
        const size_t mat = (size_t)d * d;
        const int nck = (N + C - 1) / C;
        Carve c(base);
        Ustore = c.take<float2>(mat * B * N);
        ckpt = c.take<float2>(mat * B * nck);
        seg = c.take<float2>(mat * B * C * 2);
        Xa = c.take<float2>(mat * B);
        Xb = c.take<float2>(mat * B);
        La = c.take<float2>(mat * B);
        Lb = c.take<float2>(mat * B);
        Y = c.take<float2>(mat * B);
        tr = c.take<double>((size_t)B * N * K * 6);
        tpart = c.take<double>(trace_partial_doubles(d, B, K));
        d0 = c.take<double>((size_t)B * K * 2);
        nu = c.take<double>(B);
        ov = c.take<double2>(B);
        fpart = c.take<double>(fidelity_partial_doubles(B));
        descs = c.take<GemmDesc>((size_t)3 * B);
        comp_base = base ? c.base + c.used : nullptr;
        ComposeWS cw(t, (long long)B * N, nullptr);
        c.used += expm ? std::max(cw.bytes, align_up(sizeof(int) * (size_t)B * N * t->desc.K) +
                                                align_up(sizeof(double) * (size_t)B * N * t->desc.K) +
                                                expm_compose_workspace_bytes(t))
                       : cw.bytes;
        bytes = c.used;
    }
};

// GRAPE with every state stored (checkpoint interval 1): the forward states
// X_1 .. X_N and the conjugate-transposed backward factors LH_0 .. LH_N
// (LH_n = L_n^H, L_n = U_f^dag U_{N-1} ... U_n) are kept, so the two chains run
// side by side in one batched launch per step and nothing is recomputed.
constexpr int SPT_STEPS = 2048;   // (instance, step) pairs per sparse-trace launch
struct FullGrapeWS {
    void* comp_base;
    float2* Ustore;
    float2* Xs;
    float2* LHs;
    float2* Y;
    double* tr;
    double* tpart;
    double* d0;
    double* nu;
    double2* ov;
    double* fpart;
    GemmDesc* descs;
    int sch;
    size_t bytes;
    FullGrapeWS(const redo_table_s* t, int B, int N, void* base, int expm) {
        const int d = t->desc.d, K = t->desc.K;
        const size_t mat = (size_t)d * d;
        Carve c(base);
        Ustore = c.take<float2>(mat * B * N);
        Xs = c.take<float2>(mat * B * N);
        LHs = c.take<float2>(mat * B * (N + 1));
        const bool sparse = t->spat_w > 0;
        Y = c.take<float2>(sparse ? 0 : mat * B);
        tr = c.take<double>((size_t)B * N * K * 6);
        sch = std::max(1, std::min(N, SPT_STEPS / B));
        tpart = c.take<double>(sparse ? sparse_trace_partial_doubles(d, B, sch, K) : trace_partial_doubles(d, B, K));
        d0 = c.take<double>((size_t)B * K * 2);
        nu = c.take<double>(B);
        ov = c.take<double2>(B);
        fpart = c.take<double>(fidelity_partial_doubles(B));
        descs = c.take<GemmDesc>((size_t)2 * B * N);   // the paired launches of every step
        comp_base = base ? c.base + c.used : nullptr;
        ComposeWS cw(t, (long long)B * N, nullptr);
        c.used += expm ? std::max(cw.bytes, align_up(sizeof(int) * (size_t)B * N * t->desc.K) +
                                                align_up(sizeof(double) * (size_t)B * N * t->desc.K) +
                                                expm_compose_workspace_bytes(t))
                       : cw.bytes;
        bytes = c.used;
    }
};

long long ceil_sqrt_ll(long long n) {
    long long c = (long long)std::ceil(std::sqrt((double)n));
    while (c * c < n) ++c;
    while (c > 1 && (c - 1) * (c - 1) >= n) --c;
    return std::max(1LL, c);
}

// half step of the Strang splitting seen by the adjoint's traces (0: drift-first split, or the
// plain exponential, which is not split)
double strang_hdt(const redo_table_s* t, int expm) { return (t->desc.splitting && !expm) ? 0.5 * t->desc.dt : 0.0; }

int gemm_prec(int precision) { return precision == REDO_PREC_F32_3M ? 1 : precision == REDO_PREC_BF16X3 ? 2 : 0; }

redo_status check_precision(int) { return REDO_OK; }

PlanLaunch plan_base(const redo_table_s* t) {
    PlanLaunch p{};
    p.T = t->T32;
    p.V = t->desc.drift_is_diag ? nullptr : t->V32;
    p.h = t->h64;
    p.g = t->g64;
    p.ent = t->entry_elems;
    p.d = t->desc.d;
    p.K = t->desc.K;
    p.P = t->desc.digits;
    p.base = t->desc.base;
    p.n_drift = t->desc.n_drift;
    p.phased = t->desc.phased;
    p.dense = t->desc.drift_is_diag ? 0 : 1;
    p.dt = t->desc.dt;
    p.xstride = t->entry_elems;
    p.drift_div = 1;
    p.cache = t->cache;
    p.cache_lo = t->cache_lo;
    p.cache_hi = t->cache_hi;
    p.slots = launch_slots(t);
    p.all_cached = all_cached(t) ? 1 : 0;
    p.cache_bf = t->cache_bf;
    p.bf_conj = t->cache_bf_conj ? 1 : 0;
    p.strang = t->desc.splitting;
    return p;
}

// compose U_i for I flattened (instance, step) pairs whose codes are already quantised
redo_status compose_pairs(redo_table_s* t, int precision, long long I, int N, const ComposeWS& w, float2* U_out,
                          hipStream_t st) {
    const int S = launch_slots(t);
    const long long mat = t->entry_elems;
    for (long long i0 = 0; i0 < I; i0 += COMPOSE_CHUNK) {
        const int ch = (int)std::min<long long>(COMPOSE_CHUNK, I - i0);
        PlanLaunch p = plan_base(t);
        p.codes = w.codes + i0 * t->desc.K;
        p.phi = t->desc.phased ? w.phi + i0 * t->desc.K : nullptr;
        p.code_stride = t->desc.K;
        p.step = 0;
        // pair i of this chunk is global pair i0 + i, whose drift follows its instance (i0 + i) / N
        p.drift_div = N;
        p.drift_offset = i0;
        p.X0 = U_out + i0 * mat;
        p.X1 = w.tmp;
        p.loc = w.loc;
        p.compose = 1;
        p.pre = w.pre;
        p.post = w.post;
        p.pstar = w.pstar;
        p.descs = w.descs;
        p.B = ch;
        REDO_HIP(fill_int(w.loc, ch, 0, st));
        REDO_HIP(plan_step(p, st));
        for (int s = 0; s < S; ++s)
            REDO_HIP(cgemm_batched(t->desc.d, ch, w.descs + (size_t)s * ch, gemm_prec(precision), st, GEMM_ROLE_COMPOSE));
        REDO_HIP(gather_back(t->desc.d, ch, p.X0, w.tmp, mat, w.loc, st));
    }
    return REDO_OK;
}

}  // namespace

size_t large_workspace_bytes(const redo_table_s* t, int op, int B, int N) {
    switch (op) {
        case REDO_OP_COMPOSE: return ComposeWS(t, (long long)B * N, nullptr).bytes;
        case REDO_OP_CHAIN: return ChainWS(t, B, N, nullptr).bytes;
        case REDO_OP_GRAPE: return large_grape_workspace_bytes_mode(t, B, N, 0, 0);
        case REDO_OP_EXPM_CHAIN: return expm_chain_workspace_bytes(t, B, N);
        case REDO_OP_EXPM_GRAPE: return large_grape_workspace_bytes_mode(t, B, N, 0, 1);
        default: return 0;
    }
}

int large_grape_checkpoint(const redo_table_s* t, int B, int N, int requested, int expm) {
    if (requested > 0) return requested;
    if (FullGrapeWS(t, B, N, nullptr, expm).bytes <= GRAPE_FULL_STORAGE_BYTES) return 1;
    return (int)ceil_sqrt_ll(N);
}

size_t large_grape_workspace_bytes(const redo_table_s* t, int B, int N, int C) {
    return large_grape_workspace_bytes_mode(t, B, N, C, 0);
}

size_t large_grape_workspace_bytes_mode(const redo_table_s* t, int B, int N, int C, int expm) {
    C = large_grape_checkpoint(t, B, N, C, expm);
    if (C == 1) return FullGrapeWS(t, B, N, nullptr, expm).bytes;
    return GrapeWS(t, B, N, C, nullptr, expm).bytes;
}

redo_status large_compose(redo_table_s* t, int precision, const float* u, int B, int N, float* U_out, void* workspace,
                          size_t workspace_bytes, hipStream_t st) {
    redo_status s = check_precision(precision);
    if (s != REDO_OK) return s;
    const long long I = (long long)B * N;
    ComposeWS need(t, I, nullptr);
    if (!workspace || workspace_bytes < need.bytes)
        return fail(REDO_ERR_WORKSPACE, "compose workspace needs " + std::to_string(need.bytes) + " bytes");
    ComposeWS w(t, I, workspace);
    REDO_HIP(quantise_all(t, u, B, N, w.codes, w.phi, st));
    return compose_pairs(t, precision, I, N, w, reinterpret_cast<float2*>(U_out), st);
}

redo_status large_chain(redo_table_s* t, int precision, const float* u, const int* n_steps, int B, int N,
                        int step_offset, int reproject_every, const float* X0, float* U_total, const int* obs_cols,
                        const float* obs_vals, int obs_width, double* obs_out, void* workspace, size_t workspace_bytes,
                        hipStream_t st, bool walsh_frame, const double* walsh) {
    redo_status s = check_precision(precision);
    if (s != REDO_OK) return s;
    ChainWS need(t, B, N, nullptr);
    if (!workspace || workspace_bytes < need.bytes)
        return fail(REDO_ERR_WORKSPACE, "chain workspace needs " + std::to_string(need.bytes) + " bytes");
    ChainWS w(t, B, N, workspace);
    const int d = t->desc.d;
    const long long mat = t->entry_elems;
    float2* X[2] = {reinterpret_cast<float2*>(U_total), w.W1};
    REDO_HIP(quantise_all(t, u, B, N, w.codes, w.phi, st));
    if (!X0)
        REDO_HIP(walsh_frame ? walsh_fill(d, B, X[0], mat, st) : fill_identity(d, B, X[0], mat, st));
    else if (X0 != U_total)
        REDO_HIP(hipMemcpyAsync(X[0], X0, sizeof(float2) * mat * B, hipMemcpyDeviceToDevice, st));
    REDO_HIP(fill_int(w.loc, B, 0, st));
    const int S = launch_slots(t);
    const int prec = gemm_prec(precision);
    for (int n = 0; n < N; ++n) {
        PlanLaunch p = plan_base(t);
        p.codes = w.codes + (size_t)n * t->desc.K;
        p.phi = t->desc.phased ? w.phi + (size_t)n * t->desc.K : nullptr;
        p.code_stride = (long long)N * t->desc.K;
        p.n_steps = n_steps;
        p.step = n;
        p.X0 = X[0];
        p.X1 = X[1];
        p.loc = w.loc;
        p.pre = w.pre;
        p.post = w.post;
        p.pstar = w.pstar;
        p.descs = w.descs;
        p.B = B;
        REDO_HIP(plan_step(p, st));
        for (int sl = 0; sl < S; ++sl) REDO_HIP(cgemm_batched(d, B, w.descs + (size_t)sl * B, prec, st));
        if (reproject_every > 0 && ((long long)step_offset + n + 1) % reproject_every == 0)
            REDO_HIP(reproject_states(d, B, X[0], X[1], mat, w.E, w.descs, w.loc, n_steps, n, prec, t->flags, st));
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

namespace {

redo_status large_grape_full(redo_table_s* t, int precision, const float* u, const int* n_steps, int B, int N,
                             const float* U_target, double* fidelity, double* overlap, float* grad, void* workspace,
                             size_t workspace_bytes, hipStream_t st, int expm) {
    FullGrapeWS need(t, B, N, nullptr, expm);
    if (!workspace || workspace_bytes < need.bytes)
        return fail(REDO_ERR_WORKSPACE, "GRAPE workspace needs " + std::to_string(need.bytes) + " bytes");
    FullGrapeWS w(t, B, N, workspace, expm);
    ComposeWS cw(t, (long long)B * N, w.comp_base);
    const int d = t->desc.d, K = t->desc.K;
    const long long mat = t->entry_elems;
    const int prec = gemm_prec(precision);
    const float2* Uf = reinterpret_cast<const float2*>(U_target);
    redo_status s;
    REDO_HIP(quantise_all(t, u, B, N, cw.codes, cw.phi, st));
    if (expm) {
        char* ex = static_cast<char*>(w.comp_base) + align_up(sizeof(int) * (size_t)B * N * K) +
                   align_up(sizeof(double) * (size_t)B * N * K);
        s = expm_compose_pairs(t, precision, (long long)B * N, N, u, w.Ustore, ex, st, nullptr);
    } else {
        s = compose_pairs(t, precision, (long long)B * N, N, cw, w.Ustore, st);
    }
    if (s != REDO_OK) return s;
    const long long sU = mat * N, sX = mat * N, sL = mat * (N + 1);
    // LH_N = U_f (identity left operand: a copy)
    REDO_HIP(fill_descs(w.descs, B, nullptr, 0, 0, Uf, mat, 0, w.LHs + (size_t)N * mat, sL, nullptr, 0, 1, 1.f, 0.f, st));
    REDO_HIP(cgemm_batched(d, B, w.descs, prec, st, expm));
    // step i: X_{i+1} = U_i X_i (X_0 = I) and LH_m = U_m^H LH_{m+1} with m = N - 1 - i;
    // past an instance's length both copy their right operand
    // the descriptors of every paired launch at once, then one batched GEMM per step
    REDO_HIP(grape_pair_descs(w.descs, N, B, w.Ustore, sU, w.Xs, sX, w.LHs, sL, mat, n_steps, st));
    for (int i = 0; i < N; ++i) REDO_HIP(cgemm_batched(d, 2 * B, w.descs + (size_t)i * 2 * B, prec, st, expm));
    REDO_HIP(unitary_fidelity_sliced(d, B, Uf, mat, w.Xs + (size_t)(N - 1) * mat, sX, w.ov, fidelity, w.nu, w.fpart, st));
    if (overlap) REDO_HIP(hipMemcpyAsync(overlap, w.ov, sizeof(double2) * B, hipMemcpyDeviceToDevice, st));
    const long long code_stride = (long long)N * K;
    if (t->spat_w > 0) {
        for (int s0 = 0; s0 < N; s0 += w.sch) {
            const int ns = std::min(w.sch, N - s0);
            REDO_HIP(sparse_traces(d, B, N, s0, ns, K, t->desc.phased, expm, t->spat_w, w.Xs, sX, w.LHs, sL,
                                   t->spat_cols, t->spat_vals, t->g64, cw.codes, t->desc.phased ? cw.phi : nullptr,
                                   n_steps, w.tpart, w.tr, st, t->h64, t->desc.n_drift, strang_hdt(t, expm)));
        }
    } else {
        for (int sidx = 0; sidx < N; ++sidx) {
            // Y = X_{s+1} L_{s+1} = X_{s+1} LH_{s+1}^H
            REDO_HIP(fill_descs(w.descs, B, w.Xs + (size_t)sidx * mat, sX, 0, w.LHs + (size_t)(sidx + 1) * mat, sL, 1,
                                w.Y, mat, n_steps, sidx, 0, 1.f, 0.f, st));
            REDO_HIP(cgemm_batched(d, B, w.descs, prec, st, expm));
            REDO_HIP(traces(d, B, K, t->desc.phased, w.Y, mat, t->S32, t->g64, cw.codes + (size_t)sidx * K,
                            t->desc.phased ? cw.phi + (size_t)sidx * K : nullptr, code_stride, n_steps, sidx, w.tpart,
                            w.tr + (size_t)sidx * K * 6, code_stride * 6, expm, st, t->h64, t->desc.n_drift,
                            strang_hdt(t, expm)));
        }
    }
    REDO_HIP(d0_traces(d, B, K, t->desc.phased, w.LHs, sL, t->g64, w.d0, st, 1));
    REDO_HIP(grad_assemble(B, N, K, t->desc.phased, t->desc.eps, t->desc.dt, cw.codes,
                           t->desc.phased ? cw.phi : nullptr, w.tr, w.d0, w.ov, w.nu, n_steps, grad, expm, st));
    return REDO_OK;
}

}  // namespace

redo_status large_grape(redo_table_s* t, int precision, const float* u, const int* n_steps, int B, int N,
                        const float* U_target, int C, double* fidelity, double* overlap, float* grad, void* workspace,
                        size_t workspace_bytes, hipStream_t st, int expm) {
    redo_status s = check_precision(precision);
    if (s != REDO_OK) return s;
    C = large_grape_checkpoint(t, B, N, C, expm);
    if (C == 1)
        return large_grape_full(t, precision, u, n_steps, B, N, U_target, fidelity, overlap, grad, workspace,
                                workspace_bytes, st, expm);
    GrapeWS need(t, B, N, C, nullptr, expm);
    if (!workspace || workspace_bytes < need.bytes)
        return fail(REDO_ERR_WORKSPACE, "GRAPE workspace needs " + std::to_string(need.bytes) + " bytes");
    GrapeWS w(t, B, N, C, workspace, expm);
    ComposeWS cw(t, (long long)B * N, w.comp_base);
    const int d = t->desc.d, K = t->desc.K;
    const long long mat = t->entry_elems;
    const int prec = gemm_prec(precision);
    const float2* Uf = reinterpret_cast<const float2*>(U_target);
    // every step propagator once
    REDO_HIP(quantise_all(t, u, B, N, cw.codes, cw.phi, st));
    if (expm) {
        // the codes and phases stay at the front of the compose area; the exponential scratch follows them
        char* ex = static_cast<char*>(w.comp_base) + align_up(sizeof(int) * (size_t)B * N * K) +
                   align_up(sizeof(double) * (size_t)B * N * K);
        s = expm_compose_pairs(t, precision, (long long)B * N, N, u, w.Ustore, ex, st, nullptr);
    } else {
        s = compose_pairs(t, precision, (long long)B * N, N, cw, w.Ustore, st);
    }
    if (s != REDO_OK) return s;
    // forward chain with checkpoints X_0, X_C, ...; the states of the last segment go
    // straight into a segment buffer so that segment needs no recomputation
    const int nck = (N + C - 1) / C;
    const int last0 = (nck - 1) * C;
    float2* segbuf[2] = {w.seg, w.seg + (size_t)B * C * mat};
    int cur_seg = 0;
    REDO_HIP(fill_identity(d, B, w.Xa, mat, st));
    const float2* xin = w.Xa;
    long long xin_stride = mat;
    float2* pp[2] = {w.Xa, w.Xb};
    int pp_i = 0;
    for (int n = 0; n < N; ++n) {
        if (n % C == 0) {
            REDO_HIP(fill_descs(w.descs, B, nullptr, 0, 0, xin, xin_stride, 0, w.ckpt + (size_t)(n / C) * mat, mat * nck,
                                n_steps, n, 0, 1.f, 0.f, st));
            REDO_HIP(cgemm_batched(d, B, w.descs, prec, st, expm));
        }
        float2* out;
        long long out_stride;
        if (n >= last0) {
            out = segbuf[cur_seg] + (size_t)(n - last0) * mat;
            out_stride = mat * C;
        } else {
            pp_i ^= 1;
            out = pp[pp_i];
            out_stride = mat;
        }
        // inactive steps copy the state forward
        REDO_HIP(fill_descs(w.descs, B, w.Ustore + (size_t)n * mat, mat * N, 0, xin, xin_stride, 0, out, out_stride,
                            n_steps, n, 1, 1.f, 0.f, st));
        REDO_HIP(cgemm_batched(d, B, w.descs, prec, st, expm));
        xin = out;
        xin_stride = out_stride;
    }
    REDO_HIP(unitary_fidelity_sliced(d, B, Uf, mat, xin, xin_stride, w.ov, fidelity, w.nu, w.fpart, st));
    if (overlap) REDO_HIP(hipMemcpyAsync(overlap, w.ov, sizeof(double2) * B, hipMemcpyDeviceToDevice, st));
    // backward: L_N = U_f^dag
    float2* L = w.La;
    float2* Ln = w.Lb;
    REDO_HIP(fill_descs(w.descs, B, nullptr, 0, 0, Uf, mat, 1, L, mat, nullptr, 0, 1, 1.f, 0.f, st));
    REDO_HIP(cgemm_batched(d, B, w.descs, prec, st, expm));
    const long long code_stride = (long long)N * K;
    for (int sg = nck - 1; sg >= 0; --sg) {
        const int s0 = sg * C, s1 = std::min(N, s0 + C);
        const int p0 = (sg - 1) * C;               // the previous segment [p0, s0), full length C
        float2* nseg = segbuf[cur_seg ^ 1];
        int rec = 0;                                // recompute steps of the previous segment issued so far
        auto rec_descs = [&](GemmDesc* dst) -> hipError_t {
            const int n = p0 + rec;
            const float2* src = rec == 0 ? w.ckpt + (size_t)(sg - 1) * mat : nseg + (size_t)(rec - 1) * mat;
            const long long src_stride = rec == 0 ? mat * nck : mat * C;
            return fill_descs(dst, B, w.Ustore + (size_t)n * mat, mat * N, 0, src, src_stride, 0,
                              nseg + (size_t)rec * mat, mat * C, n_steps, n, 0, 1.f, 0.f, st);
        };
        for (int sidx = s1 - 1; sidx >= s0; --sidx) {
            // Y = X_{s+1} L, L' = L U_s, and one recompute step of the previous segment, in one launch
            REDO_HIP(fill_descs(w.descs, B, segbuf[cur_seg] + (size_t)(sidx - s0) * mat, mat * C, 0, L, mat, 0, w.Y, mat,
                                n_steps, sidx, 0, 1.f, 0.f, st));
            REDO_HIP(fill_descs(w.descs + B, B, L, mat, 0, w.Ustore + (size_t)sidx * mat, mat * N, 0, Ln, mat, n_steps,
                                sidx, 2, 1.f, 0.f, st));
            int batch = 2 * B;
            if (sg > 0 && rec < C) {
                REDO_HIP(rec_descs(w.descs + 2 * B));
                ++rec;
                batch = 3 * B;
            }
            REDO_HIP(cgemm_batched(d, batch, w.descs, prec, st, expm));
            REDO_HIP(traces(d, B, K, t->desc.phased, w.Y, mat, t->S32, t->g64, cw.codes + (size_t)sidx * K,
                            t->desc.phased ? cw.phi + (size_t)sidx * K : nullptr, code_stride, n_steps, sidx, w.tpart,
                            w.tr + (size_t)sidx * K * 6, code_stride * 6, expm, st, t->h64, t->desc.n_drift,
                            strang_hdt(t, expm)));
            std::swap(L, Ln);
        }
        // the rest of the previous segment when this one was shorter
        while (sg > 0 && rec < C) {
            REDO_HIP(rec_descs(w.descs));
            REDO_HIP(cgemm_batched(d, B, w.descs, prec, st, expm));
            ++rec;
        }
        cur_seg ^= 1;
    }
    REDO_HIP(d0_traces(d, B, K, t->desc.phased, L, mat, t->g64, w.d0, st));
    REDO_HIP(grad_assemble(B, N, K, t->desc.phased, t->desc.eps, t->desc.dt, cw.codes,
                           t->desc.phased ? cw.phi : nullptr, w.tr, w.d0, w.ov, w.nu, n_steps, grad, expm, st));
    return REDO_OK;
}

}  // namespace redo
