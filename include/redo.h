/*
 * redo.h — C ABI of the REDO propagator library for AMD Instinct MI355X (gfx950).
 *
 * REDO (Rapid Exponentiation using Discrete Operators, Bhole & Mahesh,
 * arXiv 1707.02162) evaluates long sequences of piecewise-constant
 * propagators U_n = exp[-i dt (H0 + H_n)] without a matrix exponential per
 * step: every control amplitude is coarse-grained into base-b digits
 * (Sec. II, Eq. cgrain), every single-operator exponential becomes a product
 * of precomputed discrete operators (Sec. II, processes 1 and 2, Eqs.
 * redoform and exp2prod), and the drift is split off per step
 * (Sec. III, Eqs. vn and vnd).
 *
 * Conventions shared by every entry point
 *   - Every data pointer is a DEVICE pointer (HIP, the caller's allocation)
 *     unless marked "host".  The library never keeps a caller pointer past
 *     the call that received it.
 *   - Matrices are dense, row-major, contiguous.  Complex numbers are
 *     interleaved (re, im): "c64" = 2 x float, "c128" = 2 x double
 *     (the layouts of torch.complex64 / torch.complex128).
 *   - `stream` is a hipStream_t (NULL = the null stream).  All work is
 *     enqueued on it; calls return before the GPU finishes, except those
 *     documented as synchronising.  Device-side conditions (non-finite or
 *     clamped amplitudes) are latched in the table handle and read with
 *     redo_get_device_status.
 *   - Errors are status codes; no exception or abort crosses the ABI.
 *     Arguments are validated on the host before anything is launched; on
 *     error nothing is written and redo_last_error() (thread-local) says why.
 *   - A table handle may be used from several streams after it is built,
 *     except for redo_cache_levels / redo_get_device_status, which must not
 *     overlap other calls on the same handle.
 *
 * Data layouts of the per-call arrays (B instances, N_max steps, K channels):
 *   u        float [B][N_max][K]     signed amplitudes (table built with phased = 0)
 *            float [B][N_max][K][2]  Cartesian pairs (u_x, u_y) (phased = 1)
 *            in rad/s; the stride between instances is N_max*K (x2) floats.
 *   n_steps  int32 [B] per-instance lengths (1..N_max), or NULL for all N_max;
 *            steps n >= n_steps[b] are ignored.
 */
#ifndef REDO_H
#define REDO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct redo_table_s* redo_table;

typedef enum {
    REDO_OK = 0,
    REDO_ERR_ARG = 1,            /* invalid argument (size, NULL, range) */
    REDO_ERR_ALLOC = 2,          /* device allocation failed */
    REDO_ERR_HIP = 3,            /* a HIP runtime call failed */
    REDO_ERR_NOT_HERMITIAN = 4,  /* a generator or drift is not Hermitian */
    REDO_ERR_NONFINITE = 5,      /* a non-finite amplitude was seen on the device */
    REDO_ERR_UNSUPPORTED = 6,    /* valid, but not provided by this build */
    REDO_ERR_WORKSPACE = 7,      /* workspace smaller than redo_workspace_bytes */
    REDO_WARN_CLAMPED = 100,     /* some amplitude exceeded (b^P - 1) eps and was clamped */
    REDO_WARN_UNITARITY = 101    /* at a re-projection step a state had ||X^dag X - I||_F / sqrt(d) > 1e-3 */
} redo_status;

typedef enum {
    REDO_PREC_F32 = 0,     /* FP32 complex products, four real products per complex one */
    REDO_PREC_F32_3M = 1,  /* FP32, three real products (Gauss) per complex one; d >= 128 */
    REDO_PREC_BF16X3 = 2   /* split BF16: hi*hi + hi*lo + lo*hi, FP32 accumulate; d >= 128 */
} redo_precision;

typedef enum {
    REDO_OP_COMPOSE = 0,
    REDO_OP_CHAIN = 1,
    REDO_OP_GRAPE = 2,
    REDO_OP_EXPM_CHAIN = 3,
    REDO_OP_EXPM_GRAPE = 4,
    REDO_OP_STATE_GRAPE = 5,
    REDO_OP_KRON_CHAIN = 6
} redo_op;

/* Problem description of one table (Sec. II coarse graining; Sec. III model). */
typedef struct {
    int32_t d;             /* Hilbert-space dimension: a power of two 2..64, or a multiple of 64 >= 128 */
    int32_t K;             /* control channels, 1..16 */
    int32_t base;          /* b >= 2 */
    int32_t digits;        /* P >= 1, with b^P - 1 <= 2^31 - 1 */
    double dt;             /* segment length Delta t (s), > 0 */
    double eps;            /* amplitude quantum (rad/s), > 0: the paper's b^l */
    int32_t phased;        /* 1: channel k takes a Cartesian pair and its x-generator S_k is rotated by the
                                 diagonal phase generator g_k, H_kn = Z_n (Omega_kn S_k) Z_n^dag (Sec. III, Eq. vn);
                              0: channel k takes a signed amplitude, H_kn = u_kn S_k */
    int32_t drift_is_diag; /* 1: H0 is real diagonal, double [n_drift][d]; 0: c128 [n_drift][d][d] */
    int32_t n_drift;       /* number of drift Hamiltonians (>= 1); instance b uses drift b % n_drift */
    int32_t splitting;     /* 0: U_n = C_n V, the drift split off before the controls (Sec. III, the paper's
                                 split); 1: the symmetric Strang form U_n = V(dt/2) C_n V(dt/2), second
                                 order in dt (diagonal drifts only) */
} redo_table_desc;

/*
 * Process 1 of Sec. II (Eq. redoform, read as exp(-i c b^j eps dt S_k), digit
 * j = 0..P-1, coefficient c = 1..b-1): builds the table of discrete operators
 *     T_k[j][c] = exp(-i c b^j eps dt S_k)
 * in FP64 on the GPU (scaling-and-squaring Taylor for c = 1, then powers),
 * rounded once to FP32 for storage, plus the drift propagators
 * V = exp(-i dt H0) (Sec. III: the drift is split off each step).
 *   H0  double [n_drift][d] (diagonal) or c128 [n_drift][d][d]; Hermitian
 *   S   c128 [K][d][d]      Hermitian control generators (x-generators when phased)
 *   g   double [K][d]       diagonal phase generators (phased), else NULL
 * Inputs are read during the call only.  Synchronises `stream`.
 * Errors: REDO_ERR_ARG, REDO_ERR_NOT_HERMITIAN (relative anti-Hermitian part
 * > 1e-10), REDO_ERR_ALLOC, REDO_ERR_HIP.  On success *out owns the table
 * (device memory: K*P*(b-1)*d*d*8 bytes + drifts) until redo_table_destroy.
 */
redo_status redo_build_table(const redo_table_desc* desc, const double* H0, const double* S,
                             const double* g, void* stream, redo_table* out);

/* Frees the table and everything it owns.  NULL is accepted.  Synchronises the device. */
redo_status redo_table_destroy(redo_table table);

/*
 * Process 3 of Sec. II: a repeated coarse-grained value is evaluated once.
 * Composes, for every channel k and every level q_lo <= q <= q_hi, the REDO
 * factor R_k(q) = T_k[0][c_0] T_k[1][c_1] ... in FP64 (from the FP64 digit
 * operators, rebuilt as in redo_build_table) and keeps it, rounded once to
 * FP32, in the table (K*(q_hi-q_lo+1)*d*d*8 bytes of device memory).  Later
 * calls apply one product per channel and step for every amplitude whose
 * level is cached, instead of one per non-zero digit (at d <= 64 only when
 * the cache holds every level 0 .. b^P - 1); results then agree with the
 * uncached path to FP32 rounding.  A channel whose generator is real (every
 * imaginary part zero) has symmetric levels; their FP64 products are made
 * exactly symmetric, (R + R^T)/2, before the rounding.  Replaces any earlier
 * cache (and frees its pre-split copy); q_hi < 0 only frees it.  Synchronises
 * `stream`.  Must not overlap other calls on the same table.  Errors:
 * REDO_ERR_ARG, REDO_ERR_ALLOC.
 */
redo_status redo_cache_levels(redo_table table, int32_t q_lo, int32_t q_hi, void* stream);

/*
 * The cached levels of process 3 (Sec. II) a second time, as the operands of
 * the split-BF16 products (precision REDO_PREC_BF16X3) read them: every FP32
 * entry x held as hi = RNE_bf16(x) and lo = RNE_bf16(x - hi) for its real and
 * imaginary parts, in panels of 16 columns (8 bytes per entry, the size of the
 * FP32 cache).  Split-BF16 products at d >= 128 then load a cached level
 * without splitting it; the state is still split as it is loaded.  A negative
 * level q uses the panel of |q| conjugated, which is R(|q|)^H only when every
 * channel's generator is real (levels exactly symmetric); otherwise negative
 * levels keep the in-kernel split.  Results are identical (as values) to those
 * without the copy.  keep = 1 builds the copy (replacing an earlier one), 0
 * frees it; it is also freed with the cache.  Synchronises `stream`.  Errors:
 * REDO_ERR_ARG (no cache), REDO_ERR_UNSUPPORTED (d < 128 or d % 64 != 0),
 * REDO_ERR_ALLOC, REDO_ERR_HIP.
 */
redo_status redo_cache_split_bf16(redo_table table, int32_t keep, void* stream);

/*
 * Check of process 1 in FP64 (not part of the method's hot path): the level
 * R_k(q) = T_k[0][c_0] T_k[1][c_1] ... of channel k, code q (0 <= q <= b^P - 1),
 * composed in FP64 on the device by the operations, in the order, that
 * redo_build_table and redo_cache_levels use before their single rounding to
 * FP32 (scaling-and-squaring Taylor exponential of each digit's generator
 * exp(-i b^j eps dt S_k), powers by repeated products, then the product over
 * the digits, made exactly symmetric when S_k is real).  out: c128 [d][d],
 * device, caller-owned.  Allocates scratch;
 * synchronises `stream`.  REDO_ERR_ARG for k or q out of range.
 */
redo_status redo_level_f64(redo_table table, int32_t k, int32_t q, double* out, void* stream);

/* Host copy of the descriptor and the table's device footprint in bytes. */
redo_status redo_table_query(redo_table table, redo_table_desc* desc, size_t* device_bytes);

/* Bytes of workspace that `op` needs for B instances of up to N_max steps
 * (0 on invalid arguments).  Workspace is caller-owned device memory.  For
 * REDO_OP_GRAPE and REDO_OP_EXPM_GRAPE this assumes the automatic checkpoint
 * interval (checkpoint_every = 0, see redo_grape_fidelity_grad). */
size_t redo_workspace_bytes(redo_table table, int32_t op, int32_t B, int32_t N_max);

/* Workspace of redo_grape_fidelity_grad for a checkpoint interval
 * (0 = automatic). */
size_t redo_grape_workspace_bytes(redo_table table, int32_t B, int32_t N_max, int32_t checkpoint_every);

/* The smallest workspace redo_grape_fidelity_grad accepts for the same call
 * (Sec. III, GRAPE through REDO): at d <= 64 the checkpoints, one recomputed
 * segment and the pending traces, without the precomposed step propagators
 * (each scan step is then built from its factors); at d >= 128 the same as
 * redo_grape_workspace_bytes.  The interval is part of the call: with 0 it is
 * the automatic one, at d <= 64 every state kept when that fits 8 GiB, so a
 * caller short of memory passes an explicit interval (ceil(sqrt(N_max)) gives
 * the checkpointed scan).  0 on invalid arguments. */
size_t redo_grape_workspace_min_bytes(redo_table table, int32_t B, int32_t N_max, int32_t checkpoint_every);

/*
 * Coarse graining alone (Sec. II, Eq. cgrain): for every (b, n, k) with
 * n < N_max, the code q = min(floor(Omega/eps + 1/2), b^P - 1) with
 * Omega = |u| (signed tables) or sqrt(u_x^2 + u_y^2) (phased), evaluated in
 * FP64 from the FP32 inputs with IEEE rounding.
 *   codes  int32 [B][N_max][K]: q, negated for a negative signed amplitude
 *   phi    double [B][N_max][K]: atan2(u_y, u_x) (phased), or NULL
 * Non-finite amplitudes give q = 0 and latch REDO_ERR_NONFINITE; clamps are counted.
 */
redo_status redo_quantise(redo_table table, const float* u, int32_t B, int32_t N_max,
                          int32_t* codes, double* phi, void* stream);

/*
 * Process 2 of Sec. II (Eq. exp2prod) with the drift split of Sec. III:
 * every step propagator
 *     U_n = Z_n [prod_k R_k(q_kn)] Z_n^dag V,    R_k = T_k[0][c_0] T_k[1][c_1] ... (c_j = 0 skipped)
 * (channel 1 rightmost; Z_n = diag exp(-i sum_k phi_kn g_k) when phased; for
 * a negative signed amplitude R_k is replaced by its adjoint).
 *   U_out  c64 [B][N][d][d]
 * Workspace: redo_workspace_bytes(table, REDO_OP_COMPOSE, B, N).
 */
redo_status redo_compose_steps(redo_table table, int32_t precision, const float* u, int32_t B,
                               int32_t N, float* U_out, void* workspace, size_t workspace_bytes,
                               void* stream);

/*
 * The chain U = U_N ... U_1 (Sec. III, Eq. propUn) of REDO steps, per instance:
 *     X_0 = X0[b] (identity when X0 is NULL),  X_n = U_n X_{n-1},  n = 1 .. n_steps[b].
 *   X0        c64 [B][d][d] or NULL
 *   U_total   c64 [B][d][d]  receives X_{n_steps[b]} (may equal X0)
 *   X_prefix  c64 [B][N_max][d][d] receives X_1 .. X_N, or NULL (d <= 64 only)
 *   reproject_every  R > 0: after every step whose global index
 *             (step_offset + n) is a multiple of R, replace X by its
 *             Newton-Schulz polar step X (3I - X^dag X) / 2; 0 = never.
 *             At d >= 128 it is computed as X + X E with
 *             E = (I - X^dag X) / 2: X^dag X at the call's precision, X E
 *             as a split-BF16 product (E is of the order of the drift, so
 *             its relative error of about 2^-16 stays far below the FP32
 *             rounding of X), X added in FP32
 *   obs_cols, obs_vals, obs_width  an optional Hermitian observable M in
 *             row-list form: int32 [d][w] column indices and c64 [d][w] values
 *             of row a (pad with value 0); NULL/0 for none
 *   obs_out   double [B][N_max]: Tr(X_n M X_n^dag M) / Tr(M M) after step n
 *             (Sec. IV: <M>(t) for rho(0) = M), or NULL; at d >= 128 at most
 *             16 entries per row (REDO_ERR_UNSUPPORTED otherwise)
 * Workspace: redo_workspace_bytes(table, REDO_OP_CHAIN, B, N_max).
 */
redo_status redo_chain_propagator(redo_table table, int32_t precision, const float* u,
                                  const int32_t* n_steps, int32_t B, int32_t N_max,
                                  int32_t step_offset, int32_t reproject_every, const float* X0,
                                  float* U_total, float* X_prefix, const int32_t* obs_cols,
                                  const float* obs_vals, int32_t obs_width, double* obs_out,
                                  void* workspace, size_t workspace_bytes, void* stream);

/*
 * Spin structure of the table's generators: *n_spins = n when d = 2^n and every
 * S_k is a sum of single-spin terms, S_k = sum_q s_kq with s_kq a 2 x 2
 * Hermitian acting on bit q of the basis index (checked when the table is
 * built, entry by entry in FP64 to 1e-12 relative), else 0.
 */
redo_status redo_table_spins(redo_table table, int32_t* n_spins);

/*
 * Structure-aware chain: a competitor of the dense REDO factors, not the
 * paper's method.  With spin-structured generators (redo_table_spins > 0) the
 * control factors of one step factorise over the spins,
 *     exp(-i theta S_k) = (x)_q exp(-i theta s_kq),
 * so the split step of Sec. III (Eq. propUn: U_n = Z_n (prod_k R_k) Z_n^dag V,
 * or the Strang form) acts on the rows of X as a diagonal scaling, one 2 x 2
 * unitary per spin g_q = prod_k exp(-i theta_k s_kq) (FP64, rounded once to
 * FP32), and a diagonal scaling: O(n d^2) work per step instead of O(d^3).
 *   quantised  1: theta_k = dt x the REDO-quantised amplitude (Sec. II, Eq.
 *                 cgrain), the same U_n as redo_chain_propagator up to
 *                 rounding; 0: the amplitudes as given (the exact split step)
 * Other arguments, layouts, the observable and the re-projection as
 * redo_chain_propagator (FP32; the re-projection's two dense products per
 * realisation in the three-product form).  Needs d = 128 .. 4096 and a diagonal drift;
 * REDO_ERR_UNSUPPORTED otherwise.
 * Workspace: redo_workspace_bytes(table, REDO_OP_KRON_CHAIN, B, N_max).
 */
redo_status redo_kron_chain(redo_table table, int32_t quantised, const float* u, const int32_t* n_steps,
                            int32_t B, int32_t N_max, int32_t step_offset, int32_t reproject_every,
                            const float* X0, float* U_total, const int32_t* obs_cols, const float* obs_vals,
                            int32_t obs_width, double* obs_out, void* workspace, size_t workspace_bytes,
                            void* stream);

/*
 * The right Walsh frame.  With H the d x d Sylvester-Hadamard matrix,
 * H_ij = (-1)^popcount(i & j), and Hn = H / sqrt(d) (orthogonal, Hn Hn = I), an
 * observable whose entries depend only on i XOR j, M_ij = f(i XOR j) with f real
 * (a collective transverse magnetisation sum_q I_x^(q), Sec. IV, is one), is
 * M = Hn diag(D) Hn with D = H f.  A chain state X carried as W = X Hn evolves by
 * the same left products, W_n = U_n W_{n-1}, the Newton-Schulz step commutes
 * with the rotation, and the observable of redo_chain_propagator becomes
 *     Tr(X M X^dag M) = sum_j D_j w_j^dag M w_j   (w_j: column j of W),
 * one pass over W with no intermediate product M X.
 *
 * redo_observable_walsh: host-side analysis of the row lists (host pointers,
 * layout as obs_cols/obs_vals of redo_chain_propagator, duplicates summed):
 * REDO_OK and spectrum[d] = D (host, FP64) when M_ij = f(i XOR j) holds for
 * every entry with f real; REDO_ERR_UNSUPPORTED when it does not;
 * REDO_ERR_ARG for d not a power of two, NULL pointers or columns out of range.
 * No GPU work.
 */
redo_status redo_observable_walsh(int32_t d, const int32_t* cols, const float* vals, int32_t width,
                                  double* spectrum);

/*
 * In place X_b <- X_b Hn for B matrices c64 [d][d] spaced stride complex
 * entries apart (stride >= d*d) on the device: into the right Walsh frame and,
 * applied again, back (Hn Hn = I).  d a power of two in 128 .. 4096
 * (REDO_ERR_ARG otherwise).  FP32, log2(d) butterfly levels per row.
 */
redo_status redo_walsh_right(int32_t d, int32_t B, float* X, int64_t stride, void* stream);

/*
 * An observable of the right Walsh frame bound to its spectrum.  Created from
 * row lists on the host (layout as obs_cols/obs_vals of redo_chain_propagator,
 * duplicates summed) by the analysis of redo_observable_walsh: REDO_OK when
 * M_ij = f(i XOR j) holds for every entry with f real, and then *out owns
 * device copies of the lists and of the spectrum D = H f; REDO_ERR_UNSUPPORTED
 * when M is not of that form; REDO_ERR_ARG for bad sizes or pointers;
 * REDO_ERR_ALLOC / REDO_ERR_HIP.  The handle is the only way an observable
 * reaches the Walsh-frame chains, so a spectrum always describes its lists.
 * Synchronous.  redo_walsh_observable_spectrum copies D to the host (double [d]);
 * redo_walsh_observable_destroy frees the handle (NULL accepted; synchronises
 * the device).
 */
typedef struct redo_walsh_obs_s* redo_walsh_obs;
redo_status redo_walsh_observable_create(int32_t d, const int32_t* cols, const float* vals, int32_t width,
                                         redo_walsh_obs* out);
redo_status redo_walsh_observable_spectrum(redo_walsh_obs obs, double* spectrum);
redo_status redo_walsh_observable_destroy(redo_walsh_obs obs);

/*
 * redo_chain_propagator, redo_kron_chain and redo_expm_chain (the comparison
 * point) with the state in the right Walsh frame: W0 (or H/sqrt(d) when NULL,
 * the identity in that frame) and W_total are W = X Hn (convert with
 * redo_walsh_right), and the observable comes as a handle from
 * redo_walsh_observable_create (of the table's dimension, at most 16 entries per
 * row) for the one-pass evaluation; obs_out as there (obs may be NULL when
 * obs_out is NULL).  Needs d a power of two in 128 .. 2048
 * (REDO_ERR_UNSUPPORTED otherwise); no X_prefix.  Same workspace as the
 * corresponding chain (REDO_OP_CHAIN, REDO_OP_KRON_CHAIN, REDO_OP_EXPM_CHAIN).
 */
redo_status redo_chain_propagator_walsh(redo_table table, int32_t precision, const float* u,
                                        const int32_t* n_steps, int32_t B, int32_t N_max,
                                        int32_t step_offset, int32_t reproject_every, const float* W0,
                                        float* W_total, redo_walsh_obs obs, double* obs_out,
                                        void* workspace, size_t workspace_bytes, void* stream);
redo_status redo_kron_chain_walsh(redo_table table, int32_t quantised, const float* u,
                                  const int32_t* n_steps, int32_t B, int32_t N_max, int32_t step_offset,
                                  int32_t reproject_every, const float* W0, float* W_total, redo_walsh_obs obs,
                                  double* obs_out, void* workspace, size_t workspace_bytes, void* stream);
redo_status redo_expm_chain_walsh(redo_table table, int32_t precision, const float* u,
                                  const int32_t* n_steps, int32_t B, int32_t N_max, int32_t step_offset,
                                  int32_t reproject_every, const float* W0, float* W_total, redo_walsh_obs obs,
                                  double* obs_out, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Unitary fidelity (Sec. III): g_b = Tr(U_f^dag U) / Tr(U_f^dag U_f),
 * F_b = |g_b|^2, accumulated in FP64.
 *   U_target, U  c64 [B][d][d];  overlap c128 [B] or NULL;  fidelity double [B] or NULL
 */
redo_status redo_unitary_fidelity(int32_t d, int32_t B, const float* U_target, const float* U,
                                  double* overlap, double* fidelity, void* stream);

/*
 * GRAPE objective and gradient through REDO (Sec. III; the table stays
 * outside the iteration loop): F_b = |Tr(U_f^dag X_N) / Tr(U_f^dag U_f)|^2
 * and dF_b/du at the quantised amplitudes, by a forward chain
 * X_n = U_n X_{n-1} and a backward scan
 *     L_N = U_f^dag,  L_{n-1} = L_n U_n,  Y_n = X_n L_n,
 *     dg/dOmega_kn = -i dt Tr(Z S_k Z^dag Y_n) / Tr(U_f^dag U_f),
 *     dg/dphi_kn   = -i (Tr(G_k Y_n) - Tr(G_k Y_{n-1})) / Tr(U_f^dag U_f),
 * then dF = 2 Re(conj(g) dg) and the Cartesian chain rule.  The quantised
 * step is differentiated as the continuous split step at the quantised
 * point (straight-through).  Needs channels whose generators commute with
 * each other and whose phase generators commute with the drift and with the
 * other channels (REDO_ERR_UNSUPPORTED otherwise).
 * Memory schedule: with checkpoint_every = 1 every forward state and every
 * backward factor is kept (3 B N_max d^2 complex entries of workspace at
 * d >= 128): the two scans run side by side in one batched launch per step
 * and nothing is recomputed; when the generators have at most 16 nonzeros per
 * row the traces read Y_n only at those entries, as FP64 dot products of rows
 * of X_n and L_n^dag.  With checkpoint_every = C > 1 only every C-th state is
 * kept and each segment is recomputed during the backward scan.  0 selects 1
 * when that workspace is at most 48 GiB (d >= 128), else ceil(sqrt(N_max)).
 * At d <= 64 the fused kernel keeps the forward states of C consecutive steps
 * (one segment) besides the checkpoints; a C of at least N_max makes that one
 * segment the whole chain, written by the forward pass, so nothing is
 * recomputed (the same states, bit for bit), and 0 selects N_max when that
 * workspace (B N_max d^2 complex entries and the pending traces) is at most
 * 8 GiB, else ceil(sqrt(N_max)).  At
 * d <= 64, with the workspace that redo_workspace_bytes / redo_grape_workspace_bytes
 * report, every step's propagator U_n (B N_max d^2 complex entries, when that
 * is at most 4 GiB and the batch's threads, B (d/2)^2 below d = 64 and 256 B at
 * d = 64, are at most 65,536: batches too small to fill the GPU) is composed
 * first, all (instance, step) pairs in parallel, and each scan step is then one
 * product; a workspace of only the checkpoints,
 * one segment and the pending traces (the allocation-free entry's scratch) is
 * also accepted, and each scan step is then built from its factors (the same
 * result up to FP32 rounding).
 *   U_target  c64 [B][d][d];  fidelity double [B];  overlap c128 [B] or NULL
 *   grad      float, same layout as u (entries of steps >= n_steps[b] are set to 0)
 * Workspace: redo_workspace_bytes(table, REDO_OP_GRAPE, B, N_max).
 */
redo_status redo_grape_fidelity_grad(redo_table table, int32_t precision, const float* u,
                                     const int32_t* n_steps, int32_t B, int32_t N_max,
                                     const float* U_target, int32_t checkpoint_every,
                                     double* fidelity, double* overlap, float* grad,
                                     void* workspace, size_t workspace_bytes, void* stream);

/*
 * State-transfer GRAPE through REDO (Sec. III, the state fidelity):
 *     F_S,b = |<psi_f,b| U_b |psi_0,b>|^2,  U_b = U_N ... U_1 (REDO steps, as in
 * redo_chain_propagator, the level cache used when it holds every level), and
 * dF_S/du at the quantised amplitudes, by the forward chain psi_n = U_n psi_{n-1}
 * and the backward scan chi_{n-1} = U_n^dag chi_n, chi_N = psi_f, with the trace
 * identities of redo_grape_fidelity_grad on the rank-one Y_n = psi_n chi_n^dag
 * (no normalisation: g = <psi_f|psi_N>).  Every product is a batched
 * matrix-vector product of an FP32 factor (REDO_PREC_F32 only) with an FP64
 * vector, summed in FP64 (psi_n, chi_n and the phase scalings are FP64, so
 * only the factors' FP32 rounding accumulates); d <= 8192
 * (REDO_ERR_UNSUPPORTED beyond); every state is kept, and
 * when every step's plan fits (N_max <= 65535) each launch applies one factor
 * of forward step n and one of backward step N_max - 1 - n together.
 * Same channel conditions as redo_grape_fidelity_grad.  B <= 32767
 * (REDO_ERR_UNSUPPORTED beyond).
 *   psi0, psi_f  c64 [B][d] (the caller normalises them)
 *   fidelity double [B];  overlap c128 [B] (g) or NULL;  grad float, same layout as u
 * Workspace: redo_workspace_bytes(table, REDO_OP_STATE_GRAPE, B, N_max).
 */
redo_status redo_grape_state_fidelity_grad(redo_table table, int32_t precision, const float* u,
                                           const int32_t* n_steps, int32_t B, int32_t N_max, const float* psi0,
                                           const float* psi_f, double* fidelity, double* overlap, float* grad,
                                           void* workspace, size_t workspace_bytes, void* stream);

/*
 * The comparison point of the method (not REDO): the same chain with every
 * step evaluated directly as U_n = exp[-i dt (H0 + H_n)] (Sec. III, Eq.
 * propUn; H_n = sum_k u_x S_k + u_y S_k^y for phased channels, with S_k^y the
 * x-generator rotated by exp(-i pi/2 G_k)), by scaling and squaring of a
 * Taylor polynomial in Paterson-Stockmeyer form whose degree and squarings
 * keep the truncation below the FP32 unit roundoff for a bound of
 * ||dt (H0 + H_n)||_1 over the call (one device-to-host read per call).  Same
 * arguments, layouts and batched GEMMs as redo_chain_propagator; d a multiple
 * of 64 (so also d = 64, on the batched GEMMs), FP32 (REDO_PREC_F32 or
 * REDO_PREC_F32_3M).  Amplitudes are used unquantised.
 * Workspace: redo_workspace_bytes(table, REDO_OP_EXPM_CHAIN, B, N_max).
 */
redo_status redo_expm_chain(redo_table table, int32_t precision, const float* u, const int32_t* n_steps,
                            int32_t B, int32_t N_max, int32_t step_offset, int32_t reproject_every,
                            const float* X0, float* U_total, const int32_t* obs_cols, const float* obs_vals,
                            int32_t obs_width, double* obs_out, void* workspace, size_t workspace_bytes,
                            void* stream);

/*
 * The equal-result comparison point: the chain of redo_chain_propagator's split
 * model with each control factor evaluated as an exponential instead of table
 * products, U_n = exp(-i dt (sign q eps)_n S) V (Sec. III, Eq. propUn split as in
 * Eq. vnd; the amplitude coarse-grained as in Eq. cgrain, Sec. II), by the
 * scaling-and-squaring Taylor polynomial of redo_expm_chain on the same GEMMs,
 * the drift phases V applied inside the chain product.  Its result is that of
 * the REDO chain up to FP32 rounding (the table product equals the exponential
 * at the quantised amplitude), so a speed ratio against the REDO chain compares
 * the two at equal accuracy.  One signed channel, a diagonal drift and the Lie
 * split (REDO_ERR_UNSUPPORTED otherwise); d a multiple of 64; FP32.
 *   walsh_frame  0: X0 / U_total in the computational basis, no observable
 *                   (obs_out must be NULL);
 *                1: the right Walsh frame as redo_expm_chain_walsh, with obs and
 *                   obs_out as there
 * Workspace: redo_workspace_bytes(table, REDO_OP_EXPM_CHAIN, B, N_max).
 */
redo_status redo_expm_split_chain(redo_table table, int32_t precision, const float* u, const int32_t* n_steps,
                                  int32_t B, int32_t N_max, int32_t step_offset, int32_t reproject_every,
                                  const float* X0, float* U_total, int32_t walsh_frame, redo_walsh_obs obs,
                                  double* obs_out, void* workspace, size_t workspace_bytes, void* stream);

/*
 * GRAPE with the plain per-step exponential (the comparison point): the
 * fidelity of the unquantised chain and the usual first-order gradient
 * dU_n/du ~ -i dt H_k U_n (the GRAPE approximation of Khaneja et al., cited in
 * Sec. III), through the same forward and backward scans (and the same
 * memory schedule) as redo_grape_fidelity_grad.  d a multiple of 64, FP32.
 * Workspace: redo_workspace_bytes(table, REDO_OP_EXPM_GRAPE, B, N_max)
 * (automatic checkpoint interval).
 */
redo_status redo_expm_grape_fidelity_grad(redo_table table, int32_t precision, const float* u,
                                          const int32_t* n_steps, int32_t B, int32_t N_max,
                                          const float* U_target, int32_t checkpoint_every, double* fidelity,
                                          double* overlap, float* grad, void* workspace,
                                          size_t workspace_bytes, void* stream);

/*
 * Waits for `stream`, then reports and clears the conditions latched by the
 * device since the last call: REDO_ERR_NONFINITE if a non-finite amplitude
 * was seen, else REDO_WARN_UNITARITY if the unitarity watchdog fired, else
 * REDO_WARN_CLAMPED if any amplitude was clamped, else REDO_OK.
 * *n_clamped (host, nullable) receives the number of clamped amplitudes.
 * The watchdog: at every re-projection step of a chain (reproject_every > 0;
 * the state is a product of unitary steps, Sec. III Eq. propUn, so FP32
 * rounding is the only way off the unitary group), the drift
 * ||X^dag X - I||_F / sqrt(d) of each instance's state is measured in FP64
 * before the Newton-Schulz step; instances above 1e-3 are counted, and the
 * largest drift seen is kept (redo_unitarity_report).
 */
redo_status redo_get_device_status(redo_table table, void* stream, int64_t* n_clamped);

/* The unitarity watchdog as read by the last redo_get_device_status on this
 * table: the largest drift ||X^dag X - I||_F / sqrt(d) seen at a re-projection
 * step and the number of (instance, step) pairs above 1e-3 (host outputs,
 * nullable).  No GPU work. */
redo_status redo_unitarity_report(redo_table table, double* max_drift, int64_t* count);

/*
 * redo_grape_fidelity_grad without any device allocation, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): d <= 64 only (REDO_ERR_UNSUPPORTED otherwise), same
 * arguments, results and errors as redo_grape_fidelity_grad minus the
 * workspace.  The fused kernel's scratch (checkpoints, one recomputed segment,
 * pending traces; each scan step built from its factors, no precomposed step
 * propagators) comes from a
 * file-scope device array of redo_grape_noalloc_max_bytes() = 64 MiB, one copy
 * per GPU held until the process ends; a call that needs more is refused with
 * REDO_ERR_UNSUPPORTED before anything is launched.  Nothing in the array needs
 * to start at zero (every entry is written before it is read).  All calls on one
 * GPU share that array: calls that overlap in time on one GPU (several streams
 * or threads) race and must be serialised by the caller.
 */
size_t redo_grape_noalloc_max_bytes(void);
redo_status redo_grape_fidelity_grad_noalloc(redo_table table, int32_t precision, const float* u,
                                             const int32_t* n_steps, int32_t B, int32_t N_max,
                                             const float* U_target, int32_t checkpoint_every, double* fidelity,
                                             double* overlap, float* grad, void* stream);

/*
 * ---- Learned warm start (not part of the paper's method) ----
 * A three-layer perceptron maps a target unitary to initial control amplitudes
 * for a REDO-GRAPE run (plain REDO-GRAPE remains the fallback and the arbiter of
 * its fidelity):  h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), y = tanh(W3 h2 + b3).
 * Weights and activations enter the products as BF16 (round to nearest even),
 * products accumulate in FP32 on the matrix cores.
 */
typedef struct {
    int32_t sizes[4];          /* n_in, h1, h2, n_out */
    const uint16_t* W[3];      /* BF16 weights of layer l, [sizes[l+1]][sizes[l]] row-major (device) */
    const float* b[3];         /* FP32 biases of layer l, [sizes[l+1]] (device) */
} redo_mlp;

typedef struct {
    float* W[3];               /* FP32 gradients, shaped like the weights (device) */
    float* b[3];
} redo_mlp_grads;

/* Network input of a target: its 2 d^2 real entries [Re | Im] after removing the
 * global phase (trace rotated onto the non-negative real axis).
 *   U c64 [B][d][d] -> features float [B][2 d d] */
redo_status redo_mlp_target_features(int32_t d, int32_t B, const float* U, float* features, void* stream);

/* Forward pass of `batch` rows x [batch][sizes[0]]; acts receives h1, h2, y
 * back to back: float [batch][sizes[1] + sizes[2] + sizes[3]]. */
redo_status redo_mlp_forward(const redo_mlp* net, int32_t batch, const float* x, float* acts, void* stream);

/* Mean squared error of y against target [batch][sizes[3]] (FP64, written to the
 * device double *loss) and its gradients with respect to every weight and bias
 * (forward included).  scratch: float [2][batch][max(sizes[1..3])]. */
redo_status redo_mlp_loss_grad(const redo_mlp* net, int32_t batch, const float* x, const float* target,
                               float* acts, float* scratch, const redo_mlp_grads* grads, double* loss,
                               void* stream);

/*
 * Batched L-BFGS ascent steps (an optimiser beside plain gradient ascent; for
 * REDO-GRAPE the objective is F_U and g its gradient).  B instances of P
 * FP32 parameters each; per instance a history of at most m <= 32 pairs in ring
 * buffers (device, caller-owned, zero count to start):
 *   S, Y   float [m][B][P]  s = x_{k+1} - x_k,  y = g_k - g_{k+1}
 *   rho    double [m][B]    1 / (y . s);  count, head  int32 [B]
 * redo_lbfgs_direction: dir_b = H_b g_b by the two-loop recursion (initial scale
 *   s.y / y.y of the newest pair), gd[b] = g_b . dir_b (double); with no pair,
 *   or when the result is not an ascent direction, dir_b = gamma0 g_b / max|g_b|
 *   (the largest entry moves by gamma0).  Dot products in FP64.
 * redo_lbfgs_trial: xt_b = x_b + alpha[b] dir_b (alpha double [B]).
 * redo_lbfgs_push: for accept[b] != 0 the pair (xn - x, g - gn) enters the
 *   ring when y.s > 0 (curvature condition); accept[b] == 0 clears instance b's
 *   history.
 * Errors: REDO_ERR_ARG (sizes, NULL, m out of range).
 */
redo_status redo_lbfgs_direction(int32_t B, int64_t P, int32_t m, const float* g, const float* S,
                                 const float* Y, const double* rho, const int32_t* count,
                                 const int32_t* head, double gamma0, float* dir, double* gd, void* stream);
redo_status redo_lbfgs_trial(int32_t B, int64_t P, const float* x, const float* dir, const double* alpha,
                             float* xt, void* stream);
redo_status redo_lbfgs_push(int32_t B, int64_t P, int32_t m, const float* x, const float* xn,
                            const float* g, const float* gn, const int32_t* accept, float* S, float* Y,
                            double* rho, int32_t* count, int32_t* head, void* stream);

/* One Adam step on n parameters (bias-corrected with step >= 1): descent when
 * sign = 1, ascent when sign = -1, result clamped to [lo, hi]; when param_bf16
 * is not NULL it receives the updated parameters rounded to BF16.  Also the
 * amplitude update of REDO-GRAPE. */
redo_status redo_adam_update(int64_t n, float* param, uint16_t* param_bf16, const float* grad, float* m,
                             float* v, float lr, float beta1, float beta2, float eps, int32_t step, float sign,
                             float lo, float hi, void* stream);

/* One projected gradient-ascent step of REDO-GRAPE (the update of Sec. III's
 * GRAPE loop with the amplitude constraint as a clamp): param <- clamp(param +
 * alpha grad, lo, hi) elementwise on n floats (device).  REDO_ERR_ARG for n < 1,
 * NULL pointers or lo > hi. */
redo_status redo_ascent_step(int64_t n, float* param, const float* grad, float alpha, float lo, float hi,
                             void* stream);

/* Time average of an observable series (Sec. IV: the order parameter Q is the
 * mean of the magnetisation response over the time points): out[r] = mean of
 * in[r][0 .. cols-1], FP64 (device arrays in double [rows][cols], out double
 * [rows]); the summation order is fixed.  REDO_ERR_ARG for empty sizes or NULL. */
redo_status redo_time_average(int32_t rows, int32_t cols, const double* in, double* out, void* stream);

/* Round n floats to BF16 (nearest even). */
redo_status redo_to_bf16(int64_t n, const float* in, uint16_t* out, void* stream);

/*
 * Launch timing (diagnostics, not part of the method).  While enabled, every
 * batched complex-GEMM launch of the large-d path (kind 0: the step products
 * and those of the comparison point), every step launch of redo_kron_chain
 * (kind 1) and every GEMM launch of a Newton-Schulz re-projection (kind 2) is
 * bracketed by HIP events recorded on the stream it runs on.  redo_profile_read_kind waits for those events and
 * returns the summed duration (ms) and the number of launches of one kind
 * since that kind's last reset; redo_profile_read is kind 0.  Process-wide;
 * may be called from any thread.
 */
redo_status redo_profile_enable(int32_t enable);
redo_status redo_profile_read(double* gemm_ms, int64_t* gemm_launches, int32_t reset);
redo_status redo_profile_read_kind(int32_t kind, double* ms, int64_t* launches, int32_t reset);

const char* redo_status_string(redo_status status);
const char* redo_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* REDO_H */
