// Host side of the C ABI declared in include/redo.h: argument validation,
// the one-time FP64 table build (Sec. II, process 1), workspace sizing and
// dispatch to the small-d fused kernels or the large-d MFMA path.
#include <algorithm>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <string>
#include <vector>

#include "large_path.h"
#include "redo_internal.h"

// an observable M_ij = f(i XOR j) bound to its Walsh spectrum (host analysis, device copies)
struct redo_walsh_obs_s {
    int d = 0, w = 0;
    int* cols = nullptr;          // device [d][w]
    float2* vals = nullptr;       // device [d][w]
    double* spec = nullptr;       // device [d]
    std::vector<double> spectrum; // host copy
};

namespace redo {

static thread_local std::string g_last_error;

redo_status fail(redo_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

void clear_last_error() { g_last_error.clear(); }

redo_status hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? REDO_ERR_ALLOC : REDO_ERR_HIP;
}

namespace {

bool small_dim(int d) { return d == 2 || d == 4 || d == 8 || d == 16 || d == 32 || d == 64; }
bool large_dim(int d) { return d >= 128 && d % 64 == 0 && d <= 16384; }

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    template <class T>
    T* as() const {
        return static_cast<T*>(p);
    }
};

hipError_t dev_alloc(DevBuf& b, size_t bytes) { return hipMalloc(&b.p, std::max<size_t>(bytes, 16)); }

// relative anti-Hermitian part of an interleaved complex d x d matrix
double antiherm_rel(const double* m, int d) {
    double num = 0.0, den = 0.0;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            const double ar = m[2 * ((size_t)i * d + j)], ai = m[2 * ((size_t)i * d + j) + 1];
            const double br = m[2 * ((size_t)j * d + i)], bi = -m[2 * ((size_t)j * d + i) + 1];
            num += (ar - br) * (ar - br) + (ai - bi) * (ai - bi);
            den += ar * ar + ai * ai;
        }
    return den > 0 ? std::sqrt(num / den) : 0.0;
}

double norm1(const double* m, int d) {
    double best = 0.0;
    for (int j = 0; j < d; ++j) {
        double s = 0.0;
        for (int i = 0; i < d; ++i) s += std::hypot(m[2 * ((size_t)i * d + j)], m[2 * ((size_t)i * d + j) + 1]);
        best = std::max(best, s);
    }
    return best;
}

// exp(-i theta H) in FP64 on the GPU by scaling and squaring of a degree-16
// Taylor polynomial (Horner form): P <- I + (A_s / i) P, A_s = -i theta H / 2^s,
// then P <- P^2 s times; s makes ||A_s||_1 <= 1/2, where the truncation
// error is below 1e-19.  H, out: c128 d x d device; scratch: 1 matrix.
redo_status expm_fp64(int d, const double2* H, double theta, double h_norm1, double2* out, double2* scratch,
                      hipStream_t st) {
    const double a = std::fabs(theta) * h_norm1;
    int s = 0;
    while (a / std::ldexp(1.0, s) > 0.5) ++s;
    const int m = 16;
    REDO_HIP(fill_identity_z(d, 1, out, 0, st));
    double2* cur = out;
    double2* nxt = scratch;
    for (int i = m; i >= 1; --i) {
        const double2 alpha = make_double2(0.0, -theta / (std::ldexp(1.0, s) * i));
        REDO_HIP(zgemm_batched(d, 1, H, 0, cur, 0, nxt, 0, alpha, 1.0, st));
        std::swap(cur, nxt);
    }
    for (int r = 0; r < s; ++r) {
        REDO_HIP(zgemm_batched(d, 1, cur, 0, cur, 0, nxt, 0, make_double2(1.0, 0.0), 0.0, st));
        std::swap(cur, nxt);
    }
    if (cur != out) REDO_HIP(hipMemcpyAsync(out, cur, sizeof(double2) * d * d, hipMemcpyDeviceToDevice, st));
    return REDO_OK;
}

redo_status check_desc(const redo_table_desc* d) {
    if (!d) return fail(REDO_ERR_ARG, "desc is NULL");
    if (!small_dim(d->d) && !large_dim(d->d))
        return fail(REDO_ERR_ARG, "d must be a power of two in [2, 64] or a multiple of 64 in [128, 16384]");
    if (d->K < 1 || d->K > 16) return fail(REDO_ERR_ARG, "K must be in [1, 16]");
    if (d->base < 2) return fail(REDO_ERR_ARG, "base must be >= 2");
    if (d->digits < 1) return fail(REDO_ERR_ARG, "digits must be >= 1");
    double levels = 1.0;
    for (int j = 0; j < d->digits; ++j) levels *= d->base;
    if (levels - 1.0 > 2147483647.0) return fail(REDO_ERR_ARG, "base^digits - 1 exceeds 2^31 - 1");
    if (!(d->dt > 0.0) || !std::isfinite(d->dt)) return fail(REDO_ERR_ARG, "dt must be finite and > 0");
    if (!(d->eps > 0.0) || !std::isfinite(d->eps)) return fail(REDO_ERR_ARG, "eps must be finite and > 0");
    if (d->phased != 0 && d->phased != 1) return fail(REDO_ERR_ARG, "phased must be 0 or 1");
    if (d->drift_is_diag != 0 && d->drift_is_diag != 1) return fail(REDO_ERR_ARG, "drift_is_diag must be 0 or 1");
    if (d->n_drift < 1) return fail(REDO_ERR_ARG, "n_drift must be >= 1");
    if (d->splitting != 0 && d->splitting != 1) return fail(REDO_ERR_ARG, "splitting must be 0 or 1");
    if (d->splitting == 1 && !d->drift_is_diag)
        return fail(REDO_ERR_UNSUPPORTED, "the Strang splitting is provided for diagonal drifts");
    return REDO_OK;
}

// the observable of a Walsh-frame chain: present when obs_out is, of the table's dimension,
// at most 16 entries per row
redo_status check_walsh_obs(const redo_table_s* t, const redo_walsh_obs_s* obs, const double* obs_out) {
    if (!obs_out) return REDO_OK;
    if (!obs) return fail(REDO_ERR_ARG, "obs_out needs a Walsh observable");
    if (obs->d != t->desc.d) return fail(REDO_ERR_ARG, "the Walsh observable is of another dimension than the table");
    if (obs->w > 16) return fail(REDO_ERR_UNSUPPORTED, "observables with more than 16 entries per row");
    return REDO_OK;
}

// Powers of one digit operator, Tj[c] = E^c for c = 2 .. b - 1, from Tj[1] = E: by
// doubling, E^(h + i) = E^i E^h for h = 1, 2, 4, ... and i = 1 .. min(h, b - 1 - h),
// one batched product per h (log2(b) sequential launches instead of b - 2, and a
// product depth of log2(c) for E^c).  Every table build and check uses this order.
redo_status digit_powers(int d, int b, double2* Tj, hipStream_t hs) {
    const size_t nn = (size_t)d * d;
    for (int h = 1; h < b - 1; h *= 2) {
        const int cnt = std::min(h, b - 1 - h);
        REDO_HIP(zgemm_batched(d, cnt, Tj + nn, (long long)nn, Tj + nn * h, 0, Tj + nn * (h + 1), (long long)nn,
                               make_double2(1.0, 0.0), 0.0, hs));
    }
    return REDO_OK;
}

long long ceil_sqrt(long long n) {
    long long c = (long long)std::ceil(std::sqrt((double)n));
    while (c * c < n) ++c;
    while (c > 1 && (c - 1) * (c - 1) >= n) --c;
    return std::max(1LL, c);
}

// checkpoint interval of the fused GRAPE (d <= 64): the requested one, else every state kept
// (one segment) when that workspace fits SMALL_FULL_STORAGE_MAX, else ceil(sqrt(N_max))
long long small_grape_interval(const redo_table_s* t, long long B, long long N_max, long long requested) {
    if (requested > 0) return requested;
    if (small_grape_workspace_bytes(t->desc.d, t->desc.K, B, N_max, N_max) <= SMALL_FULL_STORAGE_MAX) return N_max;
    return ceil_sqrt(N_max);
}

// the pre-split BF16 copy of the level cache, if any
redo_status free_cache_bf(redo_table_s* t) {
    if (!t->cache_bf) return REDO_OK;
    REDO_HIP(hipFree(t->cache_bf));
    t->bytes -= sizeof(float2) * (size_t)t->entry_elems * t->desc.K * (size_t)(t->cache_hi - t->cache_lo + 1);
    t->cache_bf = nullptr;
    t->cache_bf_conj = false;
    return REDO_OK;
}

}  // namespace
}  // namespace redo

using namespace redo;

extern "C" {

const char* redo_last_error(void) { return g_last_error.c_str(); }

const char* redo_status_string(redo_status s) {
    switch (s) {
        case REDO_OK: return "ok";
        case REDO_ERR_ARG: return "invalid argument";
        case REDO_ERR_ALLOC: return "device allocation failed";
        case REDO_ERR_HIP: return "HIP runtime error";
        case REDO_ERR_NOT_HERMITIAN: return "operator is not Hermitian";
        case REDO_ERR_NONFINITE: return "non-finite amplitude";
        case REDO_ERR_UNSUPPORTED: return "unsupported";
        case REDO_ERR_WORKSPACE: return "workspace too small";
        case REDO_WARN_CLAMPED: return "amplitudes clamped";
        case REDO_WARN_UNITARITY: return "state drifted off unitarity";
        default: return "unknown status";
    }
}

redo_status redo_build_table(const redo_table_desc* desc, const double* H0, const double* S, const double* g,
                             void* stream, redo_table* out) {
    g_last_error.clear();
    if (!out) return fail(REDO_ERR_ARG, "out is NULL");
    *out = nullptr;
    redo_status st = check_desc(desc);
    if (st != REDO_OK) return st;
    if (!H0 || !S) return fail(REDO_ERR_ARG, "H0 and S must not be NULL");
    if (desc->phased && !g) return fail(REDO_ERR_ARG, "g must be given for phased channels");
    const int d = desc->d, K = desc->K, P = desc->digits, b = desc->base, R = desc->n_drift;
    const size_t nn = (size_t)d * d;
    hipStream_t hs = static_cast<hipStream_t>(stream);

    // ---- host copies for validation
    std::vector<double> hS(2 * nn * K), hH, hg;
    REDO_HIP(hipMemcpyAsync(hS.data(), S, sizeof(double) * hS.size(), hipMemcpyDeviceToHost, hs));
    if (desc->drift_is_diag)
        hH.resize((size_t)R * d);
    else
        hH.resize(2 * nn * R);
    REDO_HIP(hipMemcpyAsync(hH.data(), H0, sizeof(double) * hH.size(), hipMemcpyDeviceToHost, hs));
    if (desc->phased) {
        hg.resize((size_t)K * d);
        REDO_HIP(hipMemcpyAsync(hg.data(), g, sizeof(double) * hg.size(), hipMemcpyDeviceToHost, hs));
    }
    REDO_HIP(hipStreamSynchronize(hs));
    for (double v : hS)
        if (!std::isfinite(v)) return fail(REDO_ERR_ARG, "S has non-finite entries");
    for (double v : hH)
        if (!std::isfinite(v)) return fail(REDO_ERR_ARG, "H0 has non-finite entries");
    for (double v : hg)
        if (!std::isfinite(v)) return fail(REDO_ERR_ARG, "g has non-finite entries");
    std::vector<double> s_norm(K);
    for (int k = 0; k < K; ++k) {
        const double* m = hS.data() + 2 * nn * k;
        if (antiherm_rel(m, d) > 1e-10) return fail(REDO_ERR_NOT_HERMITIAN, "S_" + std::to_string(k) + " is not Hermitian");
        s_norm[k] = norm1(m, d);
    }
    std::vector<double> h_norm(R, 0.0);
    if (!desc->drift_is_diag)
        for (int r = 0; r < R; ++r) {
            const double* m = hH.data() + 2 * nn * r;
            if (antiherm_rel(m, d) > 1e-10) return fail(REDO_ERR_NOT_HERMITIAN, "H0 is not Hermitian");
            h_norm[r] = norm1(m, d);
        }

    auto t = std::make_unique<redo_table_s>();
    t->desc = *desc;
    double levels = 1.0;
    for (int j = 0; j < P; ++j) levels *= b;
    t->qmax = levels - 1.0;
    t->entry_elems = (long long)nn;

    // ---- conditions of the adjoint formulas
    {
        bool ok = true;
        std::string why;
        const double tol = 1e-9;
        if (desc->phased) {
            for (int k = 0; k < K && ok; ++k) {
                const double* gk = hg.data() + (size_t)k * d;
                for (int kk = 0; kk < K && ok; ++kk) {
                    if (kk == k) continue;
                    const double* m = hS.data() + 2 * nn * kk;
                    for (size_t e = 0; e < nn && ok; ++e) {
                        const size_t i = e / d, j = e % d;
                        if (std::fabs(gk[i] - gk[j]) * std::hypot(m[2 * e], m[2 * e + 1]) > tol * (1 + s_norm[kk])) {
                            ok = false;
                            why = "phase generator g_" + std::to_string(k) + " does not commute with S_" + std::to_string(kk);
                        }
                    }
                }
                if (!desc->drift_is_diag)
                    for (int r = 0; r < R && ok; ++r) {
                        const double* m = hH.data() + 2 * nn * r;
                        for (size_t e = 0; e < nn && ok; ++e) {
                            const size_t i = e / d, j = e % d;
                            if (std::fabs(gk[i] - gk[j]) * std::hypot(m[2 * e], m[2 * e + 1]) > tol * (1 + h_norm[r])) {
                                ok = false;
                                why = "phase generator g_" + std::to_string(k) + " does not commute with the drift";
                            }
                        }
                    }
            }
        }
        if (ok && K > 1) {
            // [S_k, S_kk] = 0 for every pair, from FP64 products on the GPU
            DevBuf w;
            REDO_HIP(dev_alloc(w, sizeof(double2) * nn * 2));
            std::vector<double> c1(2 * nn), c2(2 * nn);
            const double2* Sd = reinterpret_cast<const double2*>(S);
            for (int k = 0; k < K && ok; ++k)
                for (int kk = k + 1; kk < K && ok; ++kk) {
                    REDO_HIP(zgemm_batched(d, 1, Sd + nn * k, 0, Sd + nn * kk, 0, w.as<double2>(), 0,
                                           make_double2(1.0, 0.0), 0.0, hs));
                    REDO_HIP(zgemm_batched(d, 1, Sd + nn * kk, 0, Sd + nn * k, 0, w.as<double2>() + nn, 0,
                                           make_double2(1.0, 0.0), 0.0, hs));
                    REDO_HIP(hipMemcpyAsync(c1.data(), w.p, sizeof(double2) * nn, hipMemcpyDeviceToHost, hs));
                    REDO_HIP(hipMemcpyAsync(c2.data(), w.as<double2>() + nn, sizeof(double2) * nn,
                                            hipMemcpyDeviceToHost, hs));
                    REDO_HIP(hipStreamSynchronize(hs));
                    double diff = 0.0;
                    for (size_t e = 0; e < 2 * nn; ++e) diff = std::max(diff, std::fabs(c1[e] - c2[e]));
                    if (diff > tol * (1 + s_norm[k] * s_norm[kk])) {
                        ok = false;
                        why = "S_" + std::to_string(k) + " and S_" + std::to_string(kk) + " do not commute";
                    }
                }
        }
        t->grad_ok = ok;
        t->grad_why = why;
    }

    // ---- device allocations owned by the table
    auto alloc = [&](void** p, size_t bytes) -> hipError_t {
        t->bytes += bytes;
        return hipMalloc(p, std::max<size_t>(bytes, 16));
    };
    struct Guard {
        redo_table_s* t;
        bool armed = true;
        ~Guard() {
            if (armed && t) redo_table_destroy(t);
        }
    } guard{t.get()};
    REDO_HIP(alloc((void**)&t->T32, sizeof(float2) * nn * (size_t)K * P * (b - 1)));
    REDO_HIP(alloc((void**)&t->S32, sizeof(float2) * nn * K));
    REDO_HIP(alloc((void**)&t->S64, sizeof(double2) * nn * K));
    REDO_HIP(hipMemcpyAsync(t->S64, S, sizeof(double2) * nn * K, hipMemcpyDeviceToDevice, hs));
    t->s_norm = s_norm;
    t->s_real.assign(K, 1);
    for (int k = 0; k < K; ++k)
        for (size_t e = 0; e < nn; ++e)
            if (hS[2 * (nn * k + e) + 1] != 0.0) {
                t->s_real[k] = 0;
                break;
            }
    REDO_HIP(alloc((void**)&t->flags, sizeof(DeviceFlags)));
    REDO_HIP(hipMemsetAsync(t->flags, 0, sizeof(DeviceFlags), hs));
    if (desc->drift_is_diag) {
        REDO_HIP(alloc((void**)&t->h64, sizeof(double) * d * R));
        REDO_HIP(alloc((void**)&t->V32, sizeof(float2) * d * R));
    } else {
        REDO_HIP(alloc((void**)&t->V32, sizeof(float2) * nn * R));
    }
    if (desc->phased) REDO_HIP(alloc((void**)&t->g64, sizeof(double) * d * K));
    // sparsity pattern of the generators (the adjoint's traces then need only these entries)
    {
        std::vector<std::vector<int>> rows(d);
        size_t wmax = 0;
        for (int a = 0; a < d && wmax <= (size_t)SPAT_WMAX; ++a) {
            for (int j = 0; j < d; ++j) {
                bool nz = false;
                for (int k = 0; k < K && !nz; ++k) {
                    const size_t e = nn * k + (size_t)a * d + j;
                    nz = hS[2 * e] != 0.0 || hS[2 * e + 1] != 0.0;
                }
                if (nz) rows[a].push_back(j);
            }
            wmax = std::max(wmax, rows[a].size());
        }
        if (wmax >= 1 && wmax <= (size_t)SPAT_WMAX) {
            const int w = (int)wmax;
            std::vector<int> hc((size_t)d * w);
            std::vector<double> hv(2 * (size_t)K * d * w, 0.0);
            for (int a = 0; a < d; ++a)
                for (int t2 = 0; t2 < w; ++t2) {
                    const bool real = t2 < (int)rows[a].size();
                    const int j = real ? rows[a][t2] : a;
                    hc[(size_t)a * w + t2] = j;
                    if (real)
                        for (int k = 0; k < K; ++k) {
                            const size_t e = nn * k + (size_t)a * d + j, o = ((size_t)k * d + a) * w + t2;
                            hv[2 * o] = hS[2 * e];
                            hv[2 * o + 1] = hS[2 * e + 1];
                        }
                }
            REDO_HIP(alloc((void**)&t->spat_cols, sizeof(int) * hc.size()));
            REDO_HIP(alloc((void**)&t->spat_vals, sizeof(double) * hv.size()));
            REDO_HIP(hipMemcpyAsync(t->spat_cols, hc.data(), sizeof(int) * hc.size(), hipMemcpyHostToDevice, hs));
            REDO_HIP(hipMemcpyAsync(t->spat_vals, hv.data(), sizeof(double) * hv.size(), hipMemcpyHostToDevice, hs));
            REDO_HIP(hipStreamSynchronize(hs));
            t->spat_w = w;
        }
    }

    // single-spin structure of the generators: S_k = sum_q s_kq, s_kq acting on bit q of the
    // basis index.  The off-diagonal entries of s_kq are S_k[0][2^q] and S_k[2^q][0]; the
    // diagonal of S_k must be c + sum_q D_q bit_q(a), split as c/n + D_q bit_q(a) over the
    // spins.  Accepted when the sum reproduces S_k entry by entry to 1e-12 relative.
    {
        int n = 0;
        while ((1 << n) < d) ++n;
        if ((1 << n) == d && n >= 1) {
            std::vector<double> ks((size_t)K * n * 8, 0.0);
            bool ok = true;
            for (int k = 0; k < K && ok; ++k) {
                const double* m = hS.data() + 2 * nn * k;
                auto at = [&](size_t i, size_t j, int c) { return m[2 * (i * d + j) + c]; };
                double scale = 0.0;
                for (size_t e = 0; e < nn; ++e) scale = std::max(scale, std::hypot(m[2 * e], m[2 * e + 1]));
                const double tol = 1e-12 * std::max(scale, 1e-300);
                const double c0 = at(0, 0, 0);
                for (int q = 0; q < n; ++q) {
                    double* o = ks.data() + ((size_t)k * n + q) * 8;
                    const size_t p = (size_t)1 << q;
                    o[0] = c0 / n;                                   // s[0][0]
                    o[2] = at(0, p, 0), o[3] = at(0, p, 1);          // s[0][1]
                    o[4] = at(p, 0, 0), o[5] = at(p, 0, 1);          // s[1][0]
                    o[6] = c0 / n + (at(p, p, 0) - c0);              // s[1][1]
                }
                for (size_t a = 0; a < (size_t)d && ok; ++a)
                    for (size_t j = 0; j < (size_t)d && ok; ++j) {
                        double er = 0.0, ei = 0.0;
                        const size_t x = a ^ j;
                        if (x == 0) {
                            for (int q = 0; q < n; ++q) er += ks[((size_t)k * n + q) * 8 + (((a >> q) & 1) ? 6 : 0)];
                        } else if ((x & (x - 1)) == 0) {
                            int q = 0;
                            while (((size_t)1 << q) != x) ++q;
                            const double* o = ks.data() + ((size_t)k * n + q) * 8 + (((a >> q) & 1) ? 4 : 2);
                            er = o[0];
                            ei = o[1];
                        }
                        if (std::fabs(at(a, j, 0) - er) > tol || std::fabs(at(a, j, 1) - ei) > tol) ok = false;
                    }
            }
            if (ok) {
                REDO_HIP(alloc((void**)&t->kron_s, sizeof(double) * ks.size()));
                REDO_HIP(hipMemcpyAsync(t->kron_s, ks.data(), sizeof(double) * ks.size(), hipMemcpyHostToDevice, hs));
                REDO_HIP(hipStreamSynchronize(hs));
                t->kron_n = n;
            }
        }
    }

    // ---- FP64 build: E_kj = exp(-i b^j eps dt S_k), T_kj[c] = E_kj^c (powers by doubling)
    {
        DevBuf E, Tj, scratch;
        REDO_HIP(dev_alloc(E, sizeof(double2) * nn));
        REDO_HIP(dev_alloc(Tj, sizeof(double2) * nn * b));
        REDO_HIP(dev_alloc(scratch, sizeof(double2) * nn));
        const double2* Sd = reinterpret_cast<const double2*>(S);
        for (int k = 0; k < K; ++k)
            for (int j = 0; j < P; ++j) {
                const double theta = std::pow((double)b, j) * desc->eps * desc->dt;
                double2* T = Tj.as<double2>();
                st = expm_fp64(d, Sd + nn * k, theta, s_norm[k], T + nn, scratch.as<double2>(), hs);
                if (st != REDO_OK) return st;
                st = digit_powers(d, b, T, hs);
                if (st != REDO_OK) return st;
                REDO_HIP(round_table_entries(d, b - 1, T + nn, t->T32 + (long long)nn * (b - 1) * (k * P + j),
                                             (long long)nn, hs));
            }
        // drift propagators V = exp(-i dt H0)
        if (desc->drift_is_diag) {
            REDO_HIP(hipMemcpyAsync(t->h64, H0, sizeof(double) * d * R, hipMemcpyDeviceToDevice, hs));
            REDO_HIP(drift_diag_phases(d, R, t->h64, desc->dt, t->V32, hs));
        } else {
            const double2* Hd = reinterpret_cast<const double2*>(H0);
            for (int r = 0; r < R; ++r) {
                st = expm_fp64(d, Hd + nn * r, desc->dt, h_norm[r], E.as<double2>(), scratch.as<double2>(), hs);
                if (st != REDO_OK) return st;
                REDO_HIP(round_z_to_c((long long)nn, E.as<double2>(), t->V32 + nn * r, hs));
            }
        }
        REDO_HIP(round_z_to_c((long long)nn * K, Sd, t->S32, hs));
        // plain-exponential baseline inputs: y-partners of phased generators, FP32 dense drifts
        if (desc->phased) {
            std::vector<float> hy(2 * nn * K);
            for (int k = 0; k < K; ++k) {
                const double* gk = hg.data() + (size_t)k * d;
                for (size_t e = 0; e < nn; ++e) {
                    const size_t i = e / d, j = e % d;
                    // exp(-i pi/2 (g_i - g_j)) S_ij
                    const double ang = -0.5 * M_PI * (gk[i] - gk[j]);
                    const double c = std::cos(ang), sn = std::sin(ang);
                    const double sr = hS[2 * (nn * k + e)], si = hS[2 * (nn * k + e) + 1];
                    hy[2 * (nn * k + e)] = (float)(c * sr - sn * si);
                    hy[2 * (nn * k + e) + 1] = (float)(c * si + sn * sr);
                }
            }
            REDO_HIP(alloc((void**)&t->Sy32, sizeof(float2) * nn * K));
            REDO_HIP(hipMemcpyAsync(t->Sy32, hy.data(), sizeof(float2) * nn * K, hipMemcpyHostToDevice, hs));
            REDO_HIP(hipStreamSynchronize(hs));
        }
        if (!desc->drift_is_diag) {
            REDO_HIP(alloc((void**)&t->H32, sizeof(float2) * nn * R));
            REDO_HIP(round_z_to_c((long long)nn * R, reinterpret_cast<const double2*>(H0), t->H32, hs));
        }
        t->h_norm.assign(R, 0.0);
        for (int r = 0; r < R; ++r) {
            if (desc->drift_is_diag) {
                for (int a = 0; a < d; ++a) t->h_norm[r] = std::max(t->h_norm[r], std::fabs(hH[(size_t)r * d + a]));
            } else {
                t->h_norm[r] = h_norm[r];
            }
        }
        if (desc->phased) REDO_HIP(hipMemcpyAsync(t->g64, g, sizeof(double) * d * K, hipMemcpyDeviceToDevice, hs));
        // phase generators of spins (every entry a half-integer): the fused small-d kernels then form
        // exp(i phi g) as a power of exp(i phi / 2), with no transcendental function per step
        if (desc->phased) {
            std::vector<signed char> g2((size_t)K * d);
            bool half = true;
            for (size_t e = 0; e < g2.size() && half; ++e) {
                const double v = 2.0 * hg[e];
                if (!(std::fabs(v) <= 64.0) || v != std::nearbyint(v)) half = false;
                else g2[e] = (signed char)std::lround(v);
            }
            if (half) {
                REDO_HIP(alloc((void**)&t->g2, g2.size()));
                REDO_HIP(hipMemcpyAsync(t->g2, g2.data(), g2.size(), hipMemcpyHostToDevice, hs));
                REDO_HIP(hipStreamSynchronize(hs));
            }
        }
        REDO_HIP(hipStreamSynchronize(hs));
    }
    guard.armed = false;
    *out = t.release();
    return REDO_OK;
}

redo_status redo_table_destroy(redo_table t) {
    if (!t) return REDO_OK;
    (void)hipDeviceSynchronize();
    void* bufs[] = {t->T32,   t->h64,    t->V32,       t->g64,       t->g2,     t->S32,    t->S64,   t->Sy32,
                    t->H32,   t->flags,  t->cache,     t->cache_bf,  t->spat_cols, t->spat_vals, t->kron_s};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    delete t;
    return REDO_OK;
}

redo_status redo_cache_split_bf16(redo_table t, int32_t keep, void* stream) {
    clear_last_error();
    if (!t) return fail(REDO_ERR_ARG, "table is NULL");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    REDO_HIP(hipStreamSynchronize(hs));
    {
        const redo_status fs = free_cache_bf(t);
        if (fs != REDO_OK) return fs;
    }
    if (!keep) return REDO_OK;
    if (!t->cache) return fail(REDO_ERR_ARG, "no level cache to split (call redo_cache_levels first)");
    if (t->desc.d < 128 || t->desc.d % 64 != 0)
        return fail(REDO_ERR_UNSUPPORTED, "pre-split levels serve the d >= 128 (d % 64 == 0) products only");
    const long long count = (long long)t->desc.K * (t->cache_hi - t->cache_lo + 1);
    const size_t bytes = sizeof(float2) * (size_t)t->entry_elems * (size_t)count;
    void* p = nullptr;
    REDO_HIP(hipMalloc(&p, bytes));
    const hipError_t e = split_panels(t->desc.d, count, t->cache, static_cast<uint16_t*>(p), hs);
    const hipError_t e2 = e == hipSuccess ? hipStreamSynchronize(hs) : e;
    if (e2 != hipSuccess) {
        (void)hipFree(p);
        return hip_fail(e2, "split_panels");
    }
    t->cache_bf = static_cast<uint16_t*>(p);
    bool conj = true;
    for (int k = 0; k < t->desc.K; ++k) conj = conj && t->s_real[k];
    t->cache_bf_conj = conj;
    t->bytes += bytes;
    return REDO_OK;
}

redo_status redo_cache_levels(redo_table t, int32_t q_lo, int32_t q_hi, void* stream) {
    g_last_error.clear();
    if (!t) return fail(REDO_ERR_ARG, "table is NULL");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    REDO_HIP(hipStreamSynchronize(hs));
    {
        const redo_status fs = free_cache_bf(t);
        if (fs != REDO_OK) return fs;
    }
    if (t->cache) {
        REDO_HIP(hipFree(t->cache));
        t->bytes -= sizeof(float2) * (size_t)t->entry_elems * t->desc.K * (size_t)(t->cache_hi - t->cache_lo + 1);
        t->cache = nullptr;
        t->cache_lo = 0;
        t->cache_hi = -1;
    }
    if (q_hi < 0) return REDO_OK;  // clear only
    if (q_lo < 0 || q_lo > q_hi || (double)q_hi > t->qmax) return fail(REDO_ERR_ARG, "need 0 <= q_lo <= q_hi <= b^P - 1");
    const int d = t->desc.d, K = t->desc.K, P = t->desc.digits, b = t->desc.base;
    const size_t nn = (size_t)d * d;
    const long long L = (long long)q_hi - q_lo + 1;
    void* cache = nullptr;
    REDO_HIP(hipMalloc(&cache, sizeof(float2) * nn * K * (size_t)L));
    struct Free {
        void* p;
        ~Free() {
            if (p) (void)hipFree(p);
        }
    } guard{cache};
    // FP64 digit tables T64[j][c] = E_j^c, c = 0 .. b-1, rebuilt exactly as in the table build
    DevBuf T64, E, tmp, Rh, Rn, scratch;
    REDO_HIP(dev_alloc(T64, sizeof(double2) * nn * P * b));
    REDO_HIP(dev_alloc(E, sizeof(double2) * nn));
    REDO_HIP(dev_alloc(tmp, sizeof(double2) * nn * b));
    REDO_HIP(dev_alloc(Rh, sizeof(double2) * nn));
    REDO_HIP(dev_alloc(Rn, sizeof(double2) * nn));
    REDO_HIP(dev_alloc(scratch, sizeof(double2) * nn));
    double2* T = T64.as<double2>();
    for (int k = 0; k < K; ++k) {
        for (int j = 0; j < P; ++j) {
            const double theta = std::pow((double)b, j) * t->desc.eps * t->desc.dt;
            redo_status st = expm_fp64(d, t->S64 + nn * k, theta, t->s_norm[k], E.as<double2>(), scratch.as<double2>(), hs);
            if (st != REDO_OK) return st;
            double2* Tj = T + nn * (size_t)j * b;
            REDO_HIP(fill_identity_z(d, 1, Tj, 0, hs));
            REDO_HIP(hipMemcpyAsync(Tj + nn, E.p, sizeof(double2) * nn, hipMemcpyDeviceToDevice, hs));
            st = digit_powers(d, b, Tj, hs);
            if (st != REDO_OK) return st;
        }
        // R(q) = T[0][c_0] (T[1][c_1] T[2][c_2] ...), grouped by the high part h = q / b
        for (long long h = q_lo / b; h <= q_hi / b; ++h) {
            double2* R = nullptr;  // product of the digits j >= 1 (null = identity)
            long long rest = h;
            for (int j = 1; j < P; ++j) {
                const int c = (int)(rest % b);
                rest /= b;
                if (c == 0) continue;
                const double2* f = T + nn * ((size_t)j * b + c);
                if (!R) {
                    REDO_HIP(hipMemcpyAsync(Rh.p, f, sizeof(double2) * nn, hipMemcpyDeviceToDevice, hs));
                    R = Rh.as<double2>();
                } else {
                    REDO_HIP(zgemm_batched(d, 1, R, 0, f, 0, Rn.as<double2>(), 0, make_double2(1.0, 0.0), 0.0, hs));
                    REDO_HIP(hipMemcpyAsync(Rh.p, Rn.p, sizeof(double2) * nn, hipMemcpyDeviceToDevice, hs));
                }
            }
            const long long c_lo = std::max<long long>(0, q_lo - h * b);
            const long long c_hi = std::min<long long>(b - 1, q_hi - h * b);
            const int cnt = (int)(c_hi - c_lo + 1);
            float2* dst = static_cast<float2*>(cache) + nn * ((size_t)k * L + (size_t)(h * b + c_lo - q_lo));
            if (R) {
                REDO_HIP(zgemm_batched(d, cnt, T + nn * (size_t)c_lo, nn, R, 0, tmp.as<double2>(), nn,
                                       make_double2(1.0, 0.0), 0.0, hs));
            } else {
                REDO_HIP(hipMemcpyAsync(tmp.p, T + nn * (size_t)c_lo, sizeof(double2) * nn * cnt,
                                        hipMemcpyDeviceToDevice, hs));
            }
            // a real generator gives symmetric levels: make the FP64 products exactly so
            if (t->s_real[k]) REDO_HIP(symmetrize_z(d, cnt, tmp.as<double2>(), nn, hs));
            REDO_HIP(round_table_entries(d, cnt, tmp.as<double2>(), dst, nn, hs));
        }
    }
    REDO_HIP(hipStreamSynchronize(hs));
    guard.p = nullptr;
    t->cache = static_cast<float2*>(cache);
    t->cache_lo = q_lo;
    t->cache_hi = q_hi;
    t->bytes += sizeof(float2) * nn * K * (size_t)L;
    return REDO_OK;
}

redo_status redo_level_f64(redo_table t, int32_t k, int32_t q, double* out, void* stream) {
    g_last_error.clear();
    if (!t || !out) return fail(REDO_ERR_ARG, "table and out must not be NULL");
    if (k < 0 || k >= t->desc.K) return fail(REDO_ERR_ARG, "channel out of range");
    if (q < 0 || (double)q > t->qmax) return fail(REDO_ERR_ARG, "need 0 <= q <= b^P - 1");
    const int d = t->desc.d, P = t->desc.digits, b = t->desc.base;
    const size_t nn = (size_t)d * d;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    double2* R = reinterpret_cast<double2*>(out);
    DevBuf Tb, Rh, Rn, scratch;
    REDO_HIP(dev_alloc(Tb, sizeof(double2) * nn * b));
    REDO_HIP(dev_alloc(Rh, sizeof(double2) * nn));
    REDO_HIP(dev_alloc(Rn, sizeof(double2) * nn));
    REDO_HIP(dev_alloc(scratch, sizeof(double2) * nn));
    // T[j][c] = E_j^c with E_j from the scaling-and-squaring Taylor exponential and the
    // powers by doubling, then R = T[0][c_0] (T[1][c_1] T[2][c_2] ...): the operations
    // and their order of redo_build_table and redo_cache_levels
    auto digit_op = [&](int j, int c, double2* dst) -> redo_status {
        const double theta = std::pow((double)b, j) * t->desc.eps * t->desc.dt;
        double2* T = Tb.as<double2>();
        redo_status st = expm_fp64(d, t->S64 + nn * k, theta, t->s_norm[k], T + nn, scratch.as<double2>(), hs);
        if (st != REDO_OK) return st;
        st = digit_powers(d, b, T, hs);
        if (st != REDO_OK) return st;
        REDO_HIP(hipMemcpyAsync(dst, T + nn * c, sizeof(double2) * nn, hipMemcpyDeviceToDevice, hs));
        return REDO_OK;
    };
    bool have_high = false;
    long long rest = q / b;
    for (int j = 1; j < P; ++j) {
        const int c = (int)(rest % b);
        rest /= b;
        if (c == 0) continue;
        redo_status st = digit_op(j, c, have_high ? Rn.as<double2>() : Rh.as<double2>());
        if (st != REDO_OK) return st;
        if (have_high) {
            REDO_HIP(zgemm_batched(d, 1, Rh.as<double2>(), 0, Rn.as<double2>(), 0, scratch.as<double2>(), 0,
                                   make_double2(1.0, 0.0), 0.0, hs));
            REDO_HIP(hipMemcpyAsync(Rh.p, scratch.p, sizeof(double2) * nn, hipMemcpyDeviceToDevice, hs));
        }
        have_high = true;
    }
    const int c0 = q % b;
    if (c0 == 0) {
        if (have_high) {
            REDO_HIP(hipMemcpyAsync(R, Rh.p, sizeof(double2) * nn, hipMemcpyDeviceToDevice, hs));
        } else {
            REDO_HIP(fill_identity_z(d, 1, R, 0, hs));
        }
    } else {
        redo_status st = digit_op(0, c0, have_high ? Rn.as<double2>() : R);
        if (st != REDO_OK) return st;
        if (have_high)
            REDO_HIP(zgemm_batched(d, 1, Rn.as<double2>(), 0, Rh.as<double2>(), 0, R, 0, make_double2(1.0, 0.0), 0.0,
                                   hs));
    }
    if (t->s_real[k]) REDO_HIP(symmetrize_z(d, 1, R, 0, hs));
    REDO_HIP(hipStreamSynchronize(hs));
    return REDO_OK;
}

redo_status redo_table_query(redo_table t, redo_table_desc* desc, size_t* bytes) {
    if (!t) return fail(REDO_ERR_ARG, "table is NULL");
    if (desc) *desc = t->desc;
    if (bytes) *bytes = t->bytes;
    return REDO_OK;
}

size_t redo_workspace_bytes(redo_table t, int32_t op, int32_t B, int32_t N_max) {
    if (!t || B < 1 || N_max < 1) return 0;
    const int d = t->desc.d;
    const size_t mat = sizeof(float2) * (size_t)d * d;
    if ((op == REDO_OP_EXPM_CHAIN || op == REDO_OP_EXPM_GRAPE) && d % 64 == 0) return large_workspace_bytes(t, op, B, N_max);
    if (op == REDO_OP_STATE_GRAPE) return state_grape_workspace_bytes(t, B, N_max);
    if (op == REDO_OP_KRON_CHAIN) return kron_supported(t) ? kron_workspace_bytes(t, B, N_max) : 0;
    if (small_dim(d)) {
        switch (op) {
            case REDO_OP_COMPOSE:
            case REDO_OP_CHAIN: return 0;
            case REDO_OP_GRAPE:
                return small_grape_workspace_bytes(d, t->desc.K, B, N_max, small_grape_interval(t, B, N_max, 0)) +
                       small_grape_precomposed_bytes(d, B, N_max);
            default: return 0;
        }
    }
    return large_workspace_bytes(t, op, B, N_max);
}

size_t redo_grape_workspace_bytes(redo_table t, int32_t B, int32_t N_max, int32_t checkpoint_every) {
    if (!t || B < 1 || N_max < 1 || checkpoint_every < 0) return 0;
    const int d = t->desc.d;
    if (small_dim(d)) {
        const long long C = small_grape_interval(t, B, N_max, checkpoint_every);
        return small_grape_workspace_bytes(d, t->desc.K, B, N_max, C) + small_grape_precomposed_bytes(d, B, N_max);
    }
    return large_grape_workspace_bytes(t, B, N_max, checkpoint_every);
}

size_t redo_grape_workspace_min_bytes(redo_table t, int32_t B, int32_t N_max, int32_t checkpoint_every) {
    if (!t || B < 1 || N_max < 1 || checkpoint_every < 0) return 0;
    const int d = t->desc.d;
    if (small_dim(d)) {
        const long long C = small_grape_interval(t, B, N_max, checkpoint_every);
        return small_grape_workspace_bytes(d, t->desc.K, B, N_max, C);
    }
    return large_grape_workspace_bytes(t, B, N_max, checkpoint_every);
}

redo_status redo_quantise(redo_table t, const float* u, int32_t B, int32_t N_max, int32_t* codes, double* phi,
                          void* stream) {
    g_last_error.clear();
    if (!t) return fail(REDO_ERR_ARG, "table is NULL");
    if (B < 1 || N_max < 1) return fail(REDO_ERR_ARG, "B and N_max must be >= 1");
    if (!u || !codes) return fail(REDO_ERR_ARG, "u and codes must not be NULL");
    if (t->desc.phased && !phi) return fail(REDO_ERR_ARG, "phi must be given for phased channels");
    REDO_HIP(quantise_all(t, u, B, N_max, codes, phi, static_cast<hipStream_t>(stream)));
    return REDO_OK;
}

redo_status redo_compose_steps(redo_table t, int32_t precision, const float* u, int32_t B, int32_t N, float* U_out,
                               void* workspace, size_t workspace_bytes, void* stream) {
    g_last_error.clear();
    if (!t) return fail(REDO_ERR_ARG, "table is NULL");
    if (B < 1 || N < 1) return fail(REDO_ERR_ARG, "B and N must be >= 1");
    if ((long long)B * N > 2147483647LL) return fail(REDO_ERR_ARG, "B*N too large");
    if (!u || !U_out) return fail(REDO_ERR_ARG, "u and U_out must not be NULL");
    if (precision < REDO_PREC_F32 || precision > REDO_PREC_BF16X3) return fail(REDO_ERR_ARG, "unknown precision");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (small_dim(t->desc.d)) {
        if (precision != REDO_PREC_F32) return fail(REDO_ERR_UNSUPPORTED, "d <= 64 runs in FP32 only");
        SmallChainArgs a{};
        a.u = u;
        a.B = B;
        a.N_max = N;
        a.compose = 1;
        a.X_out = reinterpret_cast<float2*>(U_out);
        REDO_HIP(small_chain(t, a, hs));
        return REDO_OK;
    }
    return large_compose(t, precision, u, B, N, U_out, workspace, workspace_bytes, hs);
}

redo_status redo_chain_propagator(redo_table t, int32_t precision, const float* u, const int32_t* n_steps, int32_t B,
                                  int32_t N_max, int32_t step_offset, int32_t reproject_every, const float* X0,
                                  float* U_total, float* X_prefix, const int32_t* obs_cols, const float* obs_vals,
                                  int32_t obs_width, double* obs_out, void* workspace, size_t workspace_bytes,
                                  void* stream) {
    g_last_error.clear();
    if (!t) return fail(REDO_ERR_ARG, "table is NULL");
    if (B < 1 || N_max < 1) return fail(REDO_ERR_ARG, "B and N_max must be >= 1");
    if (!u || !U_total) return fail(REDO_ERR_ARG, "u and U_total must not be NULL");
    if (step_offset < 0 || reproject_every < 0) return fail(REDO_ERR_ARG, "step_offset, reproject_every must be >= 0");
    if (precision < REDO_PREC_F32 || precision > REDO_PREC_BF16X3) return fail(REDO_ERR_ARG, "unknown precision");
    if (obs_out && (!obs_cols || !obs_vals || obs_width < 1))
        return fail(REDO_ERR_ARG, "obs_out needs obs_cols, obs_vals and obs_width >= 1");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (small_dim(t->desc.d)) {
        if (precision != REDO_PREC_F32) return fail(REDO_ERR_UNSUPPORTED, "d <= 64 runs in FP32 only");
        SmallChainArgs a{};
        a.u = u;
        a.n_steps = n_steps;
        a.B = B;
        a.N_max = N_max;
        a.compose = 0;
        a.step_offset = step_offset;
        a.reproject_every = reproject_every;
        a.X0 = reinterpret_cast<const float2*>(X0);
        a.X_out = reinterpret_cast<float2*>(U_total);
        a.X_prefix = reinterpret_cast<float2*>(X_prefix);
        a.obs_cols = obs_cols;
        a.obs_vals = reinterpret_cast<const float2*>(obs_vals);
        a.obs_width = obs_width;
        a.obs_out = obs_out;
        REDO_HIP(small_chain(t, a, hs));
        return REDO_OK;
    }
    if (X_prefix) return fail(REDO_ERR_UNSUPPORTED, "X_prefix is provided for d <= 64 only");
    if (obs_out && obs_width > 16) return fail(REDO_ERR_UNSUPPORTED, "observables with more than 16 entries per row");
    return large_chain(t, precision, u, n_steps, B, N_max, step_offset, reproject_every, X0, U_total, obs_cols,
                       obs_vals, obs_width, obs_out, workspace, workspace_bytes, hs);
}

redo_status redo_table_spins(redo_table t, int32_t* n_spins) {
    g_last_error.clear();
    if (!t || !n_spins) return fail(REDO_ERR_ARG, "table and n_spins must not be NULL");
    *n_spins = t->kron_n;
    return REDO_OK;
}

redo_status redo_kron_chain(redo_table t, int32_t quantised, const float* u, const int32_t* n_steps, int32_t B,
                            int32_t N_max, int32_t step_offset, int32_t reproject_every, const float* X0,
                            float* U_total, const int32_t* obs_cols, const float* obs_vals, int32_t obs_width,
                            double* obs_out, void* workspace, size_t workspace_bytes, void* stream) {
    g_last_error.clear();
    if (!t) return fail(REDO_ERR_ARG, "table is NULL");
    if (B < 1 || N_max < 1) return fail(REDO_ERR_ARG, "B and N_max must be >= 1");
    if (!u || !U_total) return fail(REDO_ERR_ARG, "u and U_total must not be NULL");
    if (quantised != 0 && quantised != 1) return fail(REDO_ERR_ARG, "quantised must be 0 or 1");
    if (step_offset < 0 || reproject_every < 0) return fail(REDO_ERR_ARG, "step_offset, reproject_every must be >= 0");
    if (obs_out && (!obs_cols || !obs_vals || obs_width < 1))
        return fail(REDO_ERR_ARG, "obs_out needs obs_cols, obs_vals and obs_width >= 1");
    if (t->kron_n == 0) return fail(REDO_ERR_UNSUPPORTED, "the generators are not sums of single-spin terms");
    if (!kron_supported(t))
        return fail(REDO_ERR_UNSUPPORTED, "the structure-aware chain needs a diagonal drift and d = 128 .. 4096");
    if (obs_out && obs_width > 16) return fail(REDO_ERR_UNSUPPORTED, "observables with more than 16 entries per row");
    return kron_chain(t, quantised, u, n_steps, B, N_max, step_offset, reproject_every, X0, U_total, obs_cols,
                      obs_vals, obs_width, obs_out, workspace, workspace_bytes, static_cast<hipStream_t>(stream));
}

redo_status redo_observable_walsh(int32_t d, const int32_t* cols, const float* vals, int32_t width,
                                  double* spectrum) {
    g_last_error.clear();
    if (d < 2 || (d & (d - 1)) != 0) return fail(REDO_ERR_ARG, "d must be a power of two >= 2");
    if (!cols || !vals || !spectrum || width < 1)
        return fail(REDO_ERR_ARG, "cols, vals and spectrum must not be NULL, width >= 1");
    // the nonzeros of each row, duplicates summed, sorted by column
    struct Entry {
        int col;
        double re, im;
    };
    auto row_entries = [&](int i, std::vector<Entry>& out) -> bool {
        out.clear();
        for (int e = 0; e < width; ++e) {
            const int c = cols[(size_t)i * width + e];
            if (c < 0 || c >= d) return false;
            out.push_back({c, (double)vals[2 * ((size_t)i * width + e)], (double)vals[2 * ((size_t)i * width + e) + 1]});
        }
        std::sort(out.begin(), out.end(), [](const Entry& x, const Entry& y) { return x.col < y.col; });
        std::vector<Entry> m;
        for (const Entry& x : out) {
            if (!m.empty() && m.back().col == x.col) {
                m.back().re += x.re;
                m.back().im += x.im;
            } else {
                m.push_back(x);
            }
        }
        out.clear();
        for (const Entry& x : m)
            if (x.re != 0.0 || x.im != 0.0) out.push_back(x);
        return true;
    };
    std::vector<Entry> f0, ri;
    if (!row_entries(0, f0)) return fail(REDO_ERR_ARG, "a column index is outside 0 .. d-1");
    for (const Entry& x : f0)
        if (x.im != 0.0) return fail(REDO_ERR_UNSUPPORTED, "the observable is not a real function of i XOR j");
    std::vector<double> fv(d, 0.0);
    for (const Entry& x : f0) fv[x.col] = x.re;
    for (int i = 1; i < d; ++i) {
        if (!row_entries(i, ri)) return fail(REDO_ERR_ARG, "a column index is outside 0 .. d-1");
        if (ri.size() != f0.size())
            return fail(REDO_ERR_UNSUPPORTED, "the observable is not a real function of i XOR j");
        for (const Entry& x : ri)
            if (x.im != 0.0 || x.re != fv[x.col ^ i] || fv[x.col ^ i] == 0.0)
                return fail(REDO_ERR_UNSUPPORTED, "the observable is not a real function of i XOR j");
    }
    // spectrum = H f (Sylvester order), butterflies in FP64
    for (int h = 1; h < d; h <<= 1)
        for (int i = 0; i < d; i += 2 * h)
            for (int j = i; j < i + h; ++j) {
                const double a = fv[j], b = fv[j + h];
                fv[j] = a + b;
                fv[j + h] = a - b;
            }
    std::copy(fv.begin(), fv.end(), spectrum);
    return REDO_OK;
}

redo_status redo_walsh_observable_create(int32_t d, const int32_t* cols, const float* vals, int32_t width,
                                         redo_walsh_obs* out) {
    g_last_error.clear();
    if (!out) return fail(REDO_ERR_ARG, "out is NULL");
    *out = nullptr;
    std::vector<double> spec(d > 0 ? (size_t)d : 1);
    redo_status st = redo_observable_walsh(d, cols, vals, width, spec.data());
    if (st != REDO_OK) return st;
    auto h = std::make_unique<redo_walsh_obs_s>();
    h->d = d;
    h->w = width;
    h->spectrum = spec;
    const size_t ne = (size_t)d * width;
    hipError_t e = hipMalloc((void**)&h->cols, sizeof(int) * ne);
    if (e == hipSuccess) e = hipMalloc((void**)&h->vals, sizeof(float2) * ne);
    if (e == hipSuccess) e = hipMalloc((void**)&h->spec, sizeof(double) * d);
    if (e == hipSuccess) e = hipMemcpy(h->cols, cols, sizeof(int) * ne, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->vals, vals, sizeof(float2) * ne, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->spec, spec.data(), sizeof(double) * d, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        redo_walsh_observable_destroy(h.release());
        return hip_fail(e, "Walsh observable upload");
    }
    *out = h.release();
    return REDO_OK;
}

redo_status redo_walsh_observable_spectrum(redo_walsh_obs obs, double* spectrum) {
    g_last_error.clear();
    if (!obs || !spectrum) return fail(REDO_ERR_ARG, "obs and spectrum must not be NULL");
    std::copy(obs->spectrum.begin(), obs->spectrum.end(), spectrum);
    return REDO_OK;
}

redo_status redo_walsh_observable_destroy(redo_walsh_obs obs) {
    if (!obs) return REDO_OK;
    (void)hipDeviceSynchronize();
    if (obs->cols) (void)hipFree(obs->cols);
    if (obs->vals) (void)hipFree(obs->vals);
    if (obs->spec) (void)hipFree(obs->spec);
    delete obs;
    return REDO_OK;
}

redo_status redo_walsh_right(int32_t d, int32_t B, float* X, int64_t stride, void* stream) {
    g_last_error.clear();
    if (d < 128 || d > 4096 || (d & (d - 1)) != 0) return fail(REDO_ERR_ARG, "d must be a power of two in 128 .. 4096");
    if (B < 1 || !X || stride < (int64_t)d * d) return fail(REDO_ERR_ARG, "B >= 1, X not NULL, stride >= d*d");
    REDO_HIP(walsh_right(d, B, reinterpret_cast<float2*>(X), (long long)stride, static_cast<hipStream_t>(stream)));
    return REDO_OK;
}

redo_status redo_chain_propagator_walsh(redo_table t, int32_t precision, const float* u, const int32_t* n_steps,
                                        int32_t B, int32_t N_max, int32_t step_offset, int32_t reproject_every,
                                        const float* W0, float* W_total, redo_walsh_obs obs, double* obs_out,
                                        void* workspace, size_t workspace_bytes, void* stream) {
    g_last_error.clear();
    if (!t) return fail(REDO_ERR_ARG, "table is NULL");
    if (B < 1 || N_max < 1) return fail(REDO_ERR_ARG, "B and N_max must be >= 1");
    if (!u || !W_total) return fail(REDO_ERR_ARG, "u and W_total must not be NULL");
    if (step_offset < 0 || reproject_every < 0) return fail(REDO_ERR_ARG, "step_offset, reproject_every must be >= 0");
    if (precision < REDO_PREC_F32 || precision > REDO_PREC_BF16X3) return fail(REDO_ERR_ARG, "unknown precision");
    redo_status st = check_walsh_obs(t, obs, obs_out);
    if (st != REDO_OK) return st;
    if (!walsh_dim(t->desc.d)) return fail(REDO_ERR_UNSUPPORTED, "the Walsh frame needs d = 2^n, 128 .. 2048");
    return large_chain(t, precision, u, n_steps, B, N_max, step_offset, reproject_every, W0, W_total,
                       obs_out ? obs->cols : nullptr, obs_out ? reinterpret_cast<const float*>(obs->vals) : nullptr,
                       obs_out ? obs->w : 0, obs_out, workspace, workspace_bytes, static_cast<hipStream_t>(stream),
                       true, obs_out ? obs->spec : nullptr);
}

redo_status redo_kron_chain_walsh(redo_table t, int32_t quantised, const float* u, const int32_t* n_steps, int32_t B,
                                  int32_t N_max, int32_t step_offset, int32_t reproject_every, const float* W0,
                                  float* W_total, redo_walsh_obs obs, double* obs_out, void* workspace,
                                  size_t workspace_bytes, void* stream) {
    g_last_error.clear();
    if (!t) return fail(REDO_ERR_ARG, "table is NULL");
    if (B < 1 || N_max < 1) return fail(REDO_ERR_ARG, "B and N_max must be >= 1");
    if (!u || !W_total) return fail(REDO_ERR_ARG, "u and W_total must not be NULL");
    if (quantised != 0 && quantised != 1) return fail(REDO_ERR_ARG, "quantised must be 0 or 1");
    if (step_offset < 0 || reproject_every < 0) return fail(REDO_ERR_ARG, "step_offset, reproject_every must be >= 0");
    redo_status st = check_walsh_obs(t, obs, obs_out);
    if (st != REDO_OK) return st;
    if (t->kron_n == 0) return fail(REDO_ERR_UNSUPPORTED, "the generators are not sums of single-spin terms");
    if (!kron_supported(t))
        return fail(REDO_ERR_UNSUPPORTED, "the structure-aware chain needs a diagonal drift and d = 128 .. 4096");
    if (!walsh_dim(t->desc.d)) return fail(REDO_ERR_UNSUPPORTED, "the Walsh frame needs d = 2^n, 128 .. 2048");
    return kron_chain(t, quantised, u, n_steps, B, N_max, step_offset, reproject_every, W0, W_total,
                      obs_out ? obs->cols : nullptr, obs_out ? reinterpret_cast<const float*>(obs->vals) : nullptr,
                      obs_out ? obs->w : 0, obs_out, workspace, workspace_bytes, static_cast<hipStream_t>(stream), true,
                      obs_out ? obs->spec : nullptr);
}

redo_status redo_unitary_fidelity(int32_t d, int32_t B, const float* U_target, const float* U, double* overlap,
                                  double* fidelity, void* stream) {
    g_last_error.clear();
    if (d < 1 || B < 1) return fail(REDO_ERR_ARG, "d and B must be >= 1");
    if (!U_target || !U) return fail(REDO_ERR_ARG, "U_target and U must not be NULL");
    REDO_HIP(unitary_fidelity(d, B, reinterpret_cast<const float2*>(U_target), reinterpret_cast<const float2*>(U),
                              reinterpret_cast<double2*>(overlap), fidelity, static_cast<hipStream_t>(stream)));
    return REDO_OK;
}

redo_status redo_grape_fidelity_grad(redo_table t, int32_t precision, const float* u, const int32_t* n_steps,
                                     int32_t B, int32_t N_max, const float* U_target, int32_t checkpoint_every,
                                     double* fidelity, double* overlap, float* grad, void* workspace,
                                     size_t workspace_bytes, void* stream) {
    g_last_error.clear();
    if (!t) return fail(REDO_ERR_ARG, "table is NULL");
    if (B < 1 || N_max < 1) return fail(REDO_ERR_ARG, "B and N_max must be >= 1");
    if (!u || !U_target || !fidelity || !grad) return fail(REDO_ERR_ARG, "u, U_target, fidelity, grad must not be NULL");
    if (checkpoint_every < 0) return fail(REDO_ERR_ARG, "checkpoint_every must be >= 0");
    if (precision < REDO_PREC_F32 || precision > REDO_PREC_BF16X3) return fail(REDO_ERR_ARG, "unknown precision");
    if (!t->grad_ok) return fail(REDO_ERR_UNSUPPORTED, "adjoint needs commuting channels: " + t->grad_why);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (small_dim(t->desc.d)) {
        const long long C = small_grape_interval(t, B, N_max, checkpoint_every);
        if (precision != REDO_PREC_F32) return fail(REDO_ERR_UNSUPPORTED, "d <= 64 runs in FP32 only");
        const long long nck = (N_max + C - 1) / C;
        const size_t need = small_grape_workspace_bytes(t->desc.d, t->desc.K, B, N_max, C);
        if (!workspace || workspace_bytes < need)
            return fail(REDO_ERR_WORKSPACE, "GRAPE workspace needs " + std::to_string(need) + " bytes");
        SmallGrapeArgs a{};
        a.u = u;
        a.n_steps = n_steps;
        a.B = B;
        a.N_max = N_max;
        a.U_target = reinterpret_cast<const float2*>(U_target);
        a.checkpoint_every = (int)C;
        a.fidelity = fidelity;
        a.overlap = reinterpret_cast<double2*>(overlap);
        a.grad = grad;
        a.n_ckpt = (int)nck;
        a.ckpt = static_cast<float2*>(workspace);
        a.seg = a.ckpt + (size_t)B * nck * t->desc.d * t->desc.d;
        {
            const size_t mats = sizeof(float2) * (size_t)t->desc.d * t->desc.d * (size_t)B * (size_t)(nck + C);
            a.pend = reinterpret_cast<double*>(static_cast<char*>(workspace) + ((mats + 255) & ~size_t(255)));
        }
        // with room for every step's propagator, they are composed first (in parallel over steps) and
        // each scan step is one product; with the minimum workspace each step is built from its factors
        const size_t pre = small_grape_precomposed_bytes(t->desc.d, B, N_max);
        if (pre > 0 && workspace_bytes >= need + pre)
            a.Up = reinterpret_cast<float2*>(static_cast<char*>(workspace) + ((need + 255) & ~size_t(255)));
        REDO_HIP(small_grape(t, a, hs));
        return REDO_OK;
    }
    return large_grape(t, precision, u, n_steps, B, N_max, U_target, checkpoint_every, fidelity, overlap, grad,
                       workspace, workspace_bytes, hs, 0);
}

redo_status redo_grape_state_fidelity_grad(redo_table t, int32_t precision, const float* u, const int32_t* n_steps,
                                           int32_t B, int32_t N_max, const float* psi0, const float* psi_f,
                                           double* fidelity, double* overlap, float* grad, void* workspace,
                                           size_t workspace_bytes, void* stream) {
    g_last_error.clear();
    if (!t) return fail(REDO_ERR_ARG, "table is NULL");
    if (B < 1 || N_max < 1) return fail(REDO_ERR_ARG, "B and N_max must be >= 1");
    if (!u || !psi0 || !psi_f || !fidelity || !grad)
        return fail(REDO_ERR_ARG, "u, psi0, psi_f, fidelity, grad must not be NULL");
    if (precision != REDO_PREC_F32) return fail(REDO_ERR_UNSUPPORTED, "state GRAPE runs in FP32");
    if (!t->grad_ok) return fail(REDO_ERR_UNSUPPORTED, "adjoint needs commuting channels: " + t->grad_why);
    return state_grape(t, u, n_steps, B, N_max, psi0, psi_f, fidelity, overlap, grad, workspace, workspace_bytes,
                       static_cast<hipStream_t>(stream));
}

redo_status redo_expm_chain(redo_table t, int32_t precision, const float* u, const int32_t* n_steps, int32_t B,
                            int32_t N_max, int32_t step_offset, int32_t reproject_every, const float* X0,
                            float* U_total, const int32_t* obs_cols, const float* obs_vals, int32_t obs_width,
                            double* obs_out, void* workspace, size_t workspace_bytes, void* stream) {
    g_last_error.clear();
    if (!t) return fail(REDO_ERR_ARG, "table is NULL");
    if (B < 1 || N_max < 1) return fail(REDO_ERR_ARG, "B and N_max must be >= 1");
    if (!u || !U_total) return fail(REDO_ERR_ARG, "u and U_total must not be NULL");
    if (step_offset < 0 || reproject_every < 0) return fail(REDO_ERR_ARG, "step_offset, reproject_every must be >= 0");
    if (precision < REDO_PREC_F32 || precision > REDO_PREC_BF16X3) return fail(REDO_ERR_ARG, "unknown precision");
    if (obs_out && (!obs_cols || !obs_vals || obs_width < 1))
        return fail(REDO_ERR_ARG, "obs_out needs obs_cols, obs_vals and obs_width >= 1");
    if (t->desc.d % 64 != 0) return fail(REDO_ERR_UNSUPPORTED, "the exponential baseline needs d a multiple of 64");
    if (obs_out && obs_width > 16) return fail(REDO_ERR_UNSUPPORTED, "observables with more than 16 entries per row");
    return expm_chain(t, precision, u, n_steps, B, N_max, step_offset, reproject_every, X0, U_total, obs_cols, obs_vals,
                      obs_width, obs_out, workspace, workspace_bytes, static_cast<hipStream_t>(stream));
}

redo_status redo_expm_chain_walsh(redo_table t, int32_t precision, const float* u, const int32_t* n_steps, int32_t B,
                                  int32_t N_max, int32_t step_offset, int32_t reproject_every, const float* W0,
                                  float* W_total, redo_walsh_obs obs, double* obs_out, void* workspace,
                                  size_t workspace_bytes, void* stream) {
    g_last_error.clear();
    if (!t) return fail(REDO_ERR_ARG, "table is NULL");
    if (B < 1 || N_max < 1) return fail(REDO_ERR_ARG, "B and N_max must be >= 1");
    if (!u || !W_total) return fail(REDO_ERR_ARG, "u and W_total must not be NULL");
    if (step_offset < 0 || reproject_every < 0) return fail(REDO_ERR_ARG, "step_offset, reproject_every must be >= 0");
    if (precision < REDO_PREC_F32 || precision > REDO_PREC_BF16X3) return fail(REDO_ERR_ARG, "unknown precision");
    redo_status st = check_walsh_obs(t, obs, obs_out);
    if (st != REDO_OK) return st;
    if (!walsh_dim(t->desc.d)) return fail(REDO_ERR_UNSUPPORTED, "the Walsh frame needs d = 2^n, 128 .. 2048");
    return expm_chain(t, precision, u, n_steps, B, N_max, step_offset, reproject_every, W0, W_total,
                      obs_out ? obs->cols : nullptr, obs_out ? reinterpret_cast<const float*>(obs->vals) : nullptr,
                      obs_out ? obs->w : 0, obs_out, workspace, workspace_bytes, static_cast<hipStream_t>(stream), true,
                      obs_out ? obs->spec : nullptr);
}

redo_status redo_expm_split_chain(redo_table t, int32_t precision, const float* u, const int32_t* n_steps, int32_t B,
                                  int32_t N_max, int32_t step_offset, int32_t reproject_every, const float* X0,
                                  float* U_total, int32_t walsh_frame, redo_walsh_obs obs, double* obs_out,
                                  void* workspace, size_t workspace_bytes, void* stream) {
    g_last_error.clear();
    if (!t) return fail(REDO_ERR_ARG, "table is NULL");
    if (B < 1 || N_max < 1) return fail(REDO_ERR_ARG, "B and N_max must be >= 1");
    if (!u || !U_total) return fail(REDO_ERR_ARG, "u and U_total must not be NULL");
    if (step_offset < 0 || reproject_every < 0) return fail(REDO_ERR_ARG, "step_offset, reproject_every must be >= 0");
    if (precision < REDO_PREC_F32 || precision > REDO_PREC_BF16X3) return fail(REDO_ERR_ARG, "unknown precision");
    if (walsh_frame != 0 && walsh_frame != 1) return fail(REDO_ERR_ARG, "walsh_frame must be 0 or 1");
    if (!walsh_frame && obs_out) return fail(REDO_ERR_ARG, "the observable is evaluated in the Walsh frame only");
    redo_status st = check_walsh_obs(t, obs, obs_out);
    if (st != REDO_OK) return st;
    if (t->desc.d % 64 != 0) return fail(REDO_ERR_UNSUPPORTED, "the exponential baseline needs d a multiple of 64");
    if (walsh_frame && !walsh_dim(t->desc.d))
        return fail(REDO_ERR_UNSUPPORTED, "the Walsh frame needs d = 2^n, 128 .. 2048");
    return expm_chain(t, precision, u, n_steps, B, N_max, step_offset, reproject_every, X0, U_total,
                      obs_out ? obs->cols : nullptr, obs_out ? reinterpret_cast<const float*>(obs->vals) : nullptr,
                      obs_out ? obs->w : 0, obs_out, workspace, workspace_bytes, static_cast<hipStream_t>(stream),
                      walsh_frame != 0, obs_out ? obs->spec : nullptr, 1);
}

redo_status redo_expm_grape_fidelity_grad(redo_table t, int32_t precision, const float* u, const int32_t* n_steps,
                                          int32_t B, int32_t N_max, const float* U_target, int32_t checkpoint_every,
                                          double* fidelity, double* overlap, float* grad, void* workspace,
                                          size_t workspace_bytes, void* stream) {
    g_last_error.clear();
    if (!t) return fail(REDO_ERR_ARG, "table is NULL");
    if (B < 1 || N_max < 1) return fail(REDO_ERR_ARG, "B and N_max must be >= 1");
    if (!u || !U_target || !fidelity || !grad) return fail(REDO_ERR_ARG, "u, U_target, fidelity, grad must not be NULL");
    if (checkpoint_every < 0) return fail(REDO_ERR_ARG, "checkpoint_every must be >= 0");
    if (precision < REDO_PREC_F32 || precision > REDO_PREC_BF16X3) return fail(REDO_ERR_ARG, "unknown precision");
    if (t->desc.d % 64 != 0) return fail(REDO_ERR_UNSUPPORTED, "the exponential baseline needs d a multiple of 64");
    if (precision == REDO_PREC_BF16X3) return fail(REDO_ERR_UNSUPPORTED, "the exponential baseline runs in FP32");
    return large_grape(t, precision, u, n_steps, B, N_max, U_target, checkpoint_every, fidelity, overlap, grad,
                       workspace, workspace_bytes, static_cast<hipStream_t>(stream), 1);
}

redo_status redo_get_device_status(redo_table t, void* stream, int64_t* n_clamped) {
    g_last_error.clear();
    if (!t) return fail(REDO_ERR_ARG, "table is NULL");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    REDO_HIP(hipStreamSynchronize(hs));
    DeviceFlags f{};
    REDO_HIP(hipMemcpy(&f, t->flags, sizeof(f), hipMemcpyDeviceToHost));
    REDO_HIP(hipMemset(t->flags, 0, sizeof(DeviceFlags)));
    if (n_clamped) *n_clamped = (int64_t)f.clamped;
    double drift = 0.0;
    static_assert(sizeof(drift) == sizeof(f.max_drift), "drift bits");
    std::memcpy(&drift, &f.max_drift, sizeof(drift));
    t->drift_max = drift;
    t->drift_count = (long long)f.unitarity;
    if (f.nonfinite) return fail(REDO_ERR_NONFINITE, "a non-finite amplitude was seen");
    if (f.unitarity) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "%u re-projection step(s) found ||X^dag X - I||_F / sqrt(d) above %g (largest %.3e)",
                      f.unitarity, UNITARITY_WARN, drift);
        return fail(REDO_WARN_UNITARITY, msg);
    }
    if (f.clamped) return REDO_WARN_CLAMPED;
    return REDO_OK;
}

redo_status redo_unitarity_report(redo_table t, double* max_drift, int64_t* count) {
    g_last_error.clear();
    if (!t) return fail(REDO_ERR_ARG, "table is NULL");
    if (max_drift) *max_drift = t->drift_max;
    if (count) *count = (int64_t)t->drift_count;
    return REDO_OK;
}

}  // extern "C"
