// GRAPE objective and gradient at d <= 64 without any device allocation: the
// fused small-d kernel of redo_grape_fidelity_grad with its workspace
// (checkpoints, one recomputed segment, pending traces) taken from a
// file-scope device array instead of a caller buffer.
#include <mutex>
#include <string>

#include "redo_internal.h"

namespace redo {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;

// One copy per GPU, held until the process ends.  Host code never uses this
// name as an address: it takes the device address from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of this GPU's scratch, looked up once per device with that device current
redo_status scratch_address(void** out) {
    int dev = -1;
    REDO_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(REDO_ERR_UNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e == hipSuccess ? hipErrorInvalidSymbol : e, "hipGetSymbolAddress");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return REDO_OK;
}

long long ceil_sqrt_ll(long long n) {
    long long c = 1;
    while (c * c < n) ++c;
    return c;
}

bool small_d(int d) { return d == 2 || d == 4 || d == 8 || d == 16 || d == 32 || d == 64; }

}  // namespace
}  // namespace redo

using namespace redo;

extern "C" {

size_t redo_grape_noalloc_max_bytes(void) { return kScratchBytes; }

redo_status redo_grape_fidelity_grad_noalloc(redo_table t, int32_t precision, const float* u, const int32_t* n_steps,
                                             int32_t B, int32_t N_max, const float* U_target,
                                             int32_t checkpoint_every, double* fidelity, double* overlap,
                                             float* grad, void* stream) {
    clear_last_error();
    if (!t) return fail(REDO_ERR_ARG, "table is NULL");
    if (B < 1 || N_max < 1) return fail(REDO_ERR_ARG, "B and N_max must be >= 1");
    if (!u || !U_target || !fidelity || !grad) return fail(REDO_ERR_ARG, "u, U_target, fidelity, grad must not be NULL");
    if (checkpoint_every < 0) return fail(REDO_ERR_ARG, "checkpoint_every must be >= 0");
    if (precision < REDO_PREC_F32 || precision > REDO_PREC_BF16X3) return fail(REDO_ERR_ARG, "unknown precision");
    const int d = t->desc.d;
    if (!small_d(d)) return fail(REDO_ERR_UNSUPPORTED, "the allocation-free GRAPE entry covers d <= 64");
    if (precision != REDO_PREC_F32) return fail(REDO_ERR_UNSUPPORTED, "d <= 64 runs in FP32 only");
    if (!t->grad_ok) return fail(REDO_ERR_UNSUPPORTED, "adjoint needs commuting channels: " + t->grad_why);
    const long long C = checkpoint_every > 0 ? checkpoint_every : ceil_sqrt_ll(N_max);
    const long long nck = (N_max + C - 1) / C;
    const size_t need = small_grape_workspace_bytes(d, t->desc.K, B, N_max, C);
    if (need > kScratchBytes)
        return fail(REDO_ERR_UNSUPPORTED, "this GRAPE call needs " + std::to_string(need) +
                                              " bytes of scratch; the allocation-free entry holds " +
                                              std::to_string(kScratchBytes));
    void* ws = nullptr;
    redo_status st = scratch_address(&ws);
    if (st != REDO_OK) return st;
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
    a.ckpt = static_cast<float2*>(ws);
    a.seg = a.ckpt + (size_t)B * nck * d * d;
    const size_t mats = sizeof(float2) * (size_t)d * d * (size_t)B * (size_t)(nck + C);
    a.pend = reinterpret_cast<double*>(static_cast<char*>(ws) + ((mats + 255) & ~size_t(255)));
    REDO_HIP(small_grape(t, a, static_cast<hipStream_t>(stream)));
    return REDO_OK;
}

}  // extern "C"
