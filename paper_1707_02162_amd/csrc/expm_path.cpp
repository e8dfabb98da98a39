// Host orchestration of the plain per-step exponential (the comparison point
// of the method): U_n = exp[-i dt (H0 + H_n)] (Sec. III, Eq. propUn) by
// scaling and squaring of a Taylor polynomial evaluated in Paterson-Stockmeyer
// form, on the batched MFMA GEMM of the REDO path.  The degree and the number
// of squarings come from a bound on ||dt (H0 + H_n)||_1 over the call so that
// the truncation error stays below the FP32 unit roundoff.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "large_path.h"

namespace redo {

hipError_t expm_amp_bound(int B, int N, int K, int phased, const float* u, const double* snorm, unsigned long long* out,
                          hipStream_t st);
hipError_t expm_build_A(const redo_table_s* t, int count, long long pair0, int drift_div, const float* u,
                        long long ustride, double scale, float2* A, hipStream_t st, int split = 0);
hipError_t expm_lincomb(int d, int count, int r, const float* c, const float2* pw, float2* out, hipStream_t st);
hipError_t expm_descs(GemmDesc* descs, int count, const float2* A, long long sA, const float2* B, long long sB, float2* C,
                      long long sC, const float2* add, long long sAdd, hipStream_t st);
hipError_t chain_descs(GemmDesc* descs, int count, int b0, const float2* U, long long sU, float2* X0, float2* X1,
                       long long xstride, int* loc, const int* n_steps, int step, hipStream_t st,
                       const float2* kscale = nullptr, int d = 0, int n_drift = 1);

namespace {

constexpr int EXPM_CHUNK = 128;


struct PSPlan {
    int m = 0, r = 1, q = 0, s = 0;
    double theta = 0.0;
    int gemms() const { return (r - 1) + q + s; }
};

// cheapest (degree, squarings) whose Taylor tail at theta / 2^s is below u/2, u = 2^-24
PSPlan choose_plan(double theta) {
    const double tol = 0.5 * std::ldexp(1.0, -24);
    PSPlan best;
    int best_cost = 1 << 30;
    for (int m = 2; m <= 20; ++m) {
        int r = 1, qq = m;
        for (int rr = 1; rr <= m; ++rr) {
            const int cost = (rr - 1) + m / rr;
            if (cost < (r - 1) + qq) {
                r = rr;
                qq = m / rr;
            }
        }
        for (int s = 0; s < 60; ++s) {
            const double x = theta / std::ldexp(1.0, s);
            double term = 1.0, tail = 0.0;
            for (int i = 1; i <= m + 40; ++i) {
                term *= x / i;
                if (i > m) tail += term;
            }
            if (tail <= tol) {
                const int cost = (r - 1) + qq + s;
                if (cost < best_cost) {
                    best_cost = cost;
                    best.m = m;
                    best.r = r;
                    best.q = qq;
                    best.s = s;
                }
                break;
            }
        }
    }
    best.theta = theta;
    return best;
}

struct ExpmChunkWS {
    float2 *pw, *P, *P2, *Bi;
    GemmDesc* descs;
    static size_t bytes(int d, int r) {
        const size_t mat = sizeof(float2) * (size_t)d * d * EXPM_CHUNK;
        return align_up(mat * r) + 3 * align_up(mat) + align_up(sizeof(GemmDesc) * EXPM_CHUNK);
    }
    ExpmChunkWS(int d, int r, char* base) {
        const size_t mat = sizeof(float2) * (size_t)d * d * EXPM_CHUNK;
        size_t off = 0;
        pw = reinterpret_cast<float2*>(base + off);
        off += align_up(mat * r);
        P = reinterpret_cast<float2*>(base + off);
        off += align_up(mat);
        P2 = reinterpret_cast<float2*>(base + off);
        off += align_up(mat);
        Bi = reinterpret_cast<float2*>(base + off);
        off += align_up(mat);
        descs = reinterpret_cast<GemmDesc*>(base + off);
    }
};

// exp(A_i) for `cnt` pairs starting at pair0; result left in w.P (stride d*d)
redo_status expm_chunk(const redo_table_s* t, const PSPlan& pl, int prec, int cnt, long long pair0, int drift_div,
                       const float* u, long long ustride, ExpmChunkWS& w, hipStream_t st, int split = 0) {
    const int d = t->desc.d;
    const long long nn = (long long)d * d;
    REDO_HIP(expm_build_A(t, cnt, pair0, drift_div, u, ustride, t->desc.dt / std::ldexp(1.0, pl.s), w.pw, st, split));
    for (int j = 2; j <= pl.r; ++j) {
        REDO_HIP(expm_descs(w.descs, cnt, w.pw + (size_t)(j - 2) * cnt * nn, nn, w.pw, nn,
                            w.pw + (size_t)(j - 1) * cnt * nn, nn, nullptr, 0, st));
        REDO_HIP(cgemm_batched(d, cnt, w.descs, prec, st, 1));
    }
    // Taylor coefficients 1/i!, block i holds c_{i r} .. c_{i r + r - 1}
    auto coef = [&](int i) { return i > pl.m ? 0.0 : 1.0 / std::tgamma(i + 1.0); };
    auto block = [&](int i, float* c) {
        for (int j = 0; j < pl.r; ++j) c[j] = (float)coef(i * pl.r + j);
    };
    float c[8];
    if (pl.r > 8) return fail(REDO_ERR_UNSUPPORTED, "Paterson-Stockmeyer block too wide");
    // P = B_q, where B_q also takes c_{q r + r} .. c_m when r does not divide m + 1
    block(pl.q, c);
    REDO_HIP(expm_lincomb(d, cnt, pl.r, c, w.pw, w.P, st));
    float2* P = w.P;
    float2* P2 = w.P2;
    // degree beyond q r + r - 1 is not needed: q = floor(m / r) so q r + r - 1 >= m
    for (int i = pl.q - 1; i >= 0; --i) {
        block(i, c);
        REDO_HIP(expm_lincomb(d, cnt, pl.r, c, w.pw, w.Bi, st));
        REDO_HIP(expm_descs(w.descs, cnt, P, nn, w.pw + (size_t)(pl.r - 1) * cnt * nn, nn, P2, nn, w.Bi, nn, st));
        REDO_HIP(cgemm_batched(d, cnt, w.descs, prec, st, 1));
        std::swap(P, P2);
    }
    for (int s = 0; s < pl.s; ++s) {
        REDO_HIP(expm_descs(w.descs, cnt, P, nn, P, nn, P2, nn, nullptr, 0, st));
        REDO_HIP(cgemm_batched(d, cnt, w.descs, prec, st, 1));
        std::swap(P, P2);
    }
    if (P != w.P) REDO_HIP(hipMemcpyAsync(w.P, P, sizeof(float2) * nn * cnt, hipMemcpyDeviceToDevice, st));
    return REDO_OK;
}

redo_status plan_for_call(const redo_table_s* t, int B, int N, const float* u, unsigned long long* dbound, PSPlan* out,
                          hipStream_t st, int split = 0) {
    REDO_HIP(hipMemsetAsync(dbound, 0, sizeof(unsigned long long), st));
    REDO_HIP(expm_amp_bound(B, N, t->desc.K, t->desc.phased, u, t->s_norm.data(), dbound, st));
    unsigned long long bits = 0;
    REDO_HIP(hipMemcpyAsync(&bits, dbound, sizeof(bits), hipMemcpyDeviceToHost, st));
    REDO_HIP(hipStreamSynchronize(st));
    double amp;
    std::memcpy(&amp, &bits, sizeof(amp));
    double hmax = 0.0;
    if (!split)
        for (double v : t->h_norm) hmax = std::max(hmax, v);
    // split: the coarse-grained amplitude exceeds the given one by at most eps / 2 per channel
    if (split)
        for (int k = 0; k < t->desc.K; ++k) amp += 0.5 * t->desc.eps * t->s_norm[k];
    *out = choose_plan(t->desc.dt * (hmax + amp));
    return REDO_OK;
}

int ps_r_max(int d) { return 5; }

}  // namespace

size_t expm_chain_workspace_bytes(const redo_table_s* t, int B, int N) {
    const int d = t->desc.d;
    const size_t mat = sizeof(float2) * (size_t)d * d;
    return align_up(mat * B) + align_up(mat * std::min(B, REPROJECT_CHUNK)) + align_up(mat * std::min(B, OBS_CHUNK)) +
           align_up(sizeof(double) * observable_partial_doubles(d, B)) +
           align_up(sizeof(int) * B) + align_up(sizeof(GemmDesc) * std::max(B, REPROJECT_CHUNK)) + align_up(8) +
           ExpmChunkWS::bytes(d, ps_r_max(d));
}

size_t expm_compose_workspace_bytes(const redo_table_s* t) { return ExpmChunkWS::bytes(t->desc.d, ps_r_max(t->desc.d)) + align_up(8); }

// U_out[i] = exp(-i dt H) for I pairs with amplitudes at u + i * ustride
redo_status expm_compose_pairs(const redo_table_s* t, int precision, long long I, int N, const float* u, float2* U_out,
                               void* ws, hipStream_t st, int* gemms_per_step) {
    const int d = t->desc.d;
    const long long nn = (long long)d * d;
    char* base = static_cast<char*>(ws);
    unsigned long long* dbound = reinterpret_cast<unsigned long long*>(base);
    ExpmChunkWS w(d, ps_r_max(d), base + align_up(8));
    PSPlan pl;
    redo_status s = plan_for_call(t, (int)std::min<long long>(I, 1LL << 30), 1, u, dbound, &pl, st);
    if (s != REDO_OK) return s;
    if (pl.r > ps_r_max(d)) return fail(REDO_ERR_UNSUPPORTED, "exponential norm too large for the baseline plan");
    if (gemms_per_step) *gemms_per_step = pl.gemms();
    const int prec = precision == REDO_PREC_F32_3M ? 1 : 0;
    const long long ustride = (long long)t->desc.K * (t->desc.phased ? 2 : 1);
    for (long long i0 = 0; i0 < I; i0 += EXPM_CHUNK) {
        const int cnt = (int)std::min<long long>(EXPM_CHUNK, I - i0);
        s = expm_chunk(t, pl, prec, cnt, i0, N, u, ustride, w, st);
        if (s != REDO_OK) return s;
        REDO_HIP(hipMemcpyAsync(U_out + i0 * nn, w.P, sizeof(float2) * nn * cnt, hipMemcpyDeviceToDevice, st));
    }
    return REDO_OK;
}

redo_status expm_chain(redo_table_s* t, int precision, const float* u, const int* n_steps, int B, int N, int step_offset,
                       int reproject_every, const float* X0, float* U_total, const int* obs_cols, const float* obs_vals,
                       int obs_width, double* obs_out, void* workspace, size_t workspace_bytes, hipStream_t st,
                       bool walsh_frame, const double* walsh, int split) {
    if (precision == REDO_PREC_BF16X3) return fail(REDO_ERR_UNSUPPORTED, "the exponential baseline runs in FP32");
    if (split && (t->desc.phased || t->desc.K != 1 || !t->desc.drift_is_diag || t->desc.splitting))
        return fail(REDO_ERR_UNSUPPORTED,
                    "the split exponential chain takes one signed channel, a diagonal drift and the Lie split");
    const size_t need = expm_chain_workspace_bytes(t, B, N);
    if (!workspace || workspace_bytes < need)
        return fail(REDO_ERR_WORKSPACE, "exponential chain workspace needs " + std::to_string(need) + " bytes");
    const int d = t->desc.d;
    const long long nn = (long long)d * d;
    const size_t mat = sizeof(float2) * (size_t)nn;
    char* base = static_cast<char*>(workspace);
    size_t off = 0;
    float2* W1 = reinterpret_cast<float2*>(base + off);
    off += align_up(mat * B);
    float2* E = reinterpret_cast<float2*>(base + off);   // re-projection scratch
    off += align_up(mat * std::min(B, REPROJECT_CHUNK));
    float2* obsT = reinterpret_cast<float2*>(base + off);
    off += align_up(mat * std::min(B, OBS_CHUNK));
    double* obs_partial = reinterpret_cast<double*>(base + off);
    off += align_up(sizeof(double) * observable_partial_doubles(d, B));
    int* loc = reinterpret_cast<int*>(base + off);
    off += align_up(sizeof(int) * B);
    GemmDesc* descs = reinterpret_cast<GemmDesc*>(base + off);
    off += align_up(sizeof(GemmDesc) * std::max(B, REPROJECT_CHUNK));
    unsigned long long* dbound = reinterpret_cast<unsigned long long*>(base + off);
    off += align_up(8);
    ExpmChunkWS w(d, ps_r_max(d), base + off);
    PSPlan pl;
    redo_status s = plan_for_call(t, B, N, u, dbound, &pl, st, split);
    if (s != REDO_OK) return s;
    if (pl.r > ps_r_max(d)) return fail(REDO_ERR_UNSUPPORTED, "exponential norm too large for the baseline plan");
    const int prec = precision == REDO_PREC_F32_3M ? 1 : 0;
    float2* X[2] = {reinterpret_cast<float2*>(U_total), W1};
    if (!X0)
        REDO_HIP(walsh_frame ? walsh_fill(d, B, X[0], nn, st) : fill_identity(d, B, X[0], nn, st));
    else if (X0 != U_total)
        REDO_HIP(hipMemcpyAsync(X[0], X0, mat * B, hipMemcpyDeviceToDevice, st));
    REDO_HIP(fill_int(loc, B, 0, st));
    const long long ustride_pair = (long long)t->desc.K * (t->desc.phased ? 2 : 1);
    for (int n = 0; n < N; ++n) {
        for (int b0 = 0; b0 < B; b0 += EXPM_CHUNK) {
            const int cnt = std::min(EXPM_CHUNK, B - b0);
            // entry i is instance b = b0 + i: amplitudes at u + (b N + n) K(2), drift b % n_drift
            s = expm_chunk(t, pl, prec, cnt, b0, 1, u + (long long)n * ustride_pair, ustride_pair * N, w, st, split);
            if (s != REDO_OK) return s;
            // split: X' = exp(A) V X with the drift phases V on the right (diagonal drift)
            REDO_HIP(chain_descs(descs, cnt, b0, w.P, nn, X[0], X[1], nn, loc, n_steps, n, st,
                                 split ? t->V32 : nullptr, d, t->desc.n_drift));
            REDO_HIP(cgemm_batched(d, cnt, descs, prec, st, 1));
        }
        if (reproject_every > 0 && ((long long)step_offset + n + 1) % reproject_every == 0)
            REDO_HIP(reproject_states(d, B, X[0], X[1], nn, E, descs, loc, n_steps, n, prec, t->flags, st));
        if (obs_out)
            REDO_HIP(walsh_frame ? observable_walsh(d, B, X[0], X[1], loc, nn, obs_cols,
                                                    reinterpret_cast<const float2*>(obs_vals), obs_width, walsh,
                                                    n_steps, n, obs_partial, obs_out + n, N, st)
                                 : observable(d, B, X[0], X[1], loc, nn, obs_cols,
                                              reinterpret_cast<const float2*>(obs_vals), obs_width, n_steps, n,
                                              obs_partial, obs_out + n, N, obsT, OBS_CHUNK, st));
    }
    REDO_HIP(gather_back(d, B, X[0], X[1], nn, loc, st));
    return REDO_OK;
}

}  // namespace redo
