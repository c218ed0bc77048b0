/*
 * nqsvmc.h - C ABI of libnqsvmc.so: the variational Monte Carlo hot path for
 * neural quantum states on AMD Instinct MI355X (gfx950).
 *
 * Method: Schmitt & Reh, "jVMC: Versatile and performant variational Monte
 * Carlo leveraging automated differentiation and GPU acceleration" (SciPost
 * Phys. Codebases).  One stochastic-reconfiguration / TDVP step (the paper's
 * Algorithm 1) is
 *     vmc_sample -> vmc_log_psi -> vmc_grad_log_psi -> vmc_local_energy
 *                -> vmc_sr_solve
 * and each call below names the passage that defines what it computes.
 *
 * Conventions (all calls)
 *  - Every data pointer is a caller-owned DEVICE pointer unless its name ends
 *    in _host.  The library never frees caller memory.  Opaque handles are
 *    created and destroyed by the library.
 *  - Calls are asynchronous on the context's HIP stream (the one passed to
 *    vmc_ctx_create, or the null stream).  Outputs are valid after
 *    vmc_ctx_sync() or an event recorded on that stream.  Calls that return
 *    results in _host arguments synchronise the stream themselves.
 *  - Every call returns a status: VMC_OK (0) or a negative VMC_ERR_* code; the
 *    message of the last failure on a context is vmc_last_error(ctx).  No C++
 *    exception crosses this boundary.  A handle that failed is left unchanged.
 *  - Sizes are int64_t.  One context per host thread; calls on one context
 *    must not overlap.
 *
 * Spin configurations (the paper's 0/1 basis of Sec. 4.2): N sites packed in
 * W = ceil(N/64) little-endian uint64 words per configuration, site i in word
 * i/64, bit i%64; a set bit is spin up (sigma = 2s - 1 = +1).  Bits >= N in
 * the last word must be zero.  A batch of B configurations is B*W words,
 * configuration-major.
 *
 * Complex numbers are interleaved (re, im): c128 = 2 doubles, c64 = 2 floats.
 */
#ifndef NQSVMC_H
#define NQSVMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
enum {
  VMC_OK = 0,
  VMC_ERR_INVALID_ARG = -1,  /* bad size, null pointer, inconsistent handles */
  VMC_ERR_OOM = -2,          /* device allocation failed                      */
  VMC_ERR_HIP = -3,          /* a HIP runtime call failed                     */
  VMC_ERR_NOT_PD = -4,       /* shifted S not positive definite (see info)    */
  VMC_ERR_NONFINITE = -5,    /* NaN/Inf in parameters or results              */
  VMC_ERR_UNSUPPORTED = -6,  /* valid request the library does not implement  */
  VMC_ERR_WORKSPACE = -7     /* request exceeds the workspace limit           */
};

/* compute precision of network evaluations (vmc_model_set_precision) */
enum vmc_prec { VMC_F64 = 0, VMC_F32 = 1, VMC_BF16 = 2 };

/* element types of parameter / gradient buffers */
enum vmc_dtype { VMC_DT_F64 = 0, VMC_DT_C128 = 1, VMC_DT_C64 = 2, VMC_DT_F32 = 3 };

/* Metropolis proposals */
enum { VMC_PROP_FLIP = 0, VMC_PROP_EXCHANGE = 1, VMC_PROP_MADE_MIX = 2 };

/* [[.]] of eq:tdvp_gen / eq:tdvp_util */
enum { VMC_SR_COMPLEX = 0, VMC_SR_REAL = 1, VMC_SR_IMAG = 2 };

typedef struct vmc_ctx vmc_ctx;
typedef struct vmc_model vmc_model;
typedef struct vmc_ham vmc_ham;
typedef struct vmc_sampler vmc_sampler;
typedef struct vmc_made vmc_made;

/* ---- context ------------------------------------------------------------ */
/* Binds a HIP device and stream (hip_stream may be NULL: the null stream).  */
int vmc_ctx_create(int hip_device, void* hip_stream, vmc_ctx** out);
/* Releases the caller's handle.  Every model, Hamiltonian, sampler and MADE
 * created from the context holds a reference of its own, so the handle may be
 * released before them (in any order); the context and its workspace are
 * freed when the last reference goes.  Each *_destroy synchronises the
 * context's stream first.  A sampler borrows its model and Hamiltonian: they
 * must outlive its last vmc_sampler_sample call, not its destroy.            */
int vmc_ctx_destroy(vmc_ctx* ctx);
int vmc_ctx_sync(vmc_ctx* ctx);
/* Message of the last failed call on ctx ("" if none).  Valid until the next call. */
const char* vmc_last_error(vmc_ctx* ctx);
/* Caps the library-owned device workspace (bytes; 0 = no cap).  Calls that
 * would need more return VMC_ERR_WORKSPACE. */
int vmc_ctx_set_workspace_limit(vmc_ctx* ctx, size_t bytes);
/* Library version string. */
const char* vmc_version(void);
/* Per-phase device timing: when enabled, the library brackets each phase of
 * its calls (e.g. "sample", "eloc", "grad", "sr.herk", "sr.chol") with HIP
 * events on the context's stream.  vmc_ctx_set_timing(ctx, 1) enables and
 * clears the accumulators, 0 disables.  vmc_ctx_get_timing synchronises the
 * stream and returns the summed milliseconds and the number of brackets of
 * `phase` (0 and 0 if it never ran). */
int vmc_ctx_set_timing(vmc_ctx* ctx, int enable);
int vmc_ctx_get_timing(vmc_ctx* ctx, const char* phase, double* total_ms_host, int64_t* count_host);

/* ---- models (the paper's NQS, Sec. 4.2 "Variational wave functions") ---- */
/* Restricted Boltzmann machine, eq:rbm_ex:
 *   log psi(s) = sum_i a_i sigma_i + sum_j log cosh(theta_j),
 *   theta_j = b_j + sum_i W_ji sigma_i.
 * Flat parameter order: [a (N), b (N_h), W (N_h x N, row-major)], K = N + N_h + N*N_h.
 * is_complex = 0 keeps all parameters real (imaginary parts forced to 0).  */
int vmc_model_create_rbm(vmc_ctx* ctx, int n_visible, int n_hidden, int is_complex, vmc_model** out);
/* Two-layer periodic CNN on an Lx x Ly torus (the paper's convolutional
 * NQS class, Sec. 4.2 "nets"):
 *   z1[c,y,x] = b1_c + sum_{dy,dx} W1[c,dy,dx] sigma[(y+dy)%Ly, (x+dx)%Lx]
 *   z2[c,y,x] = b2_c + sum_{c',dy,dx} W2[c,c',dy,dx] logcosh(z1[c',(y+dy)%Ly,(x+dx)%Lx])
 *   log psi   = sum_{c,y,x} logcosh(z2[c,y,x])
 * Flat order: [W1 (C*k*k), b1 (C), W2 (C*C*k*k, [c_out][c_in][dy][dx]), b2 (C)], complex. */
int vmc_model_create_cnn(vmc_ctx* ctx, int Lx, int Ly, int channels, int kernel, vmc_model** out);
/* Autoregressive state with direct sampling (Sec. 2.4 "Autoregressive neural
 * quantum states"): psi(s) = sqrt(q(s)), q(s) = prod_i p_i(s_i | s_<i) given by a
 * masked network with one ReLU hidden layer of n_hidden units (MADE; hidden
 * degree m(k) = k mod (N - 1) + 1, inputs and outputs have degree d + 1 for
 * site d):  a = (W1 * M1) s + b1,  l = (W2 * M2) relu(a) + b2,
 *   log psi(s) = (1/2) sum_i [s_i l_i - softplus(l_i)],  s_i in {0, 1} (bit i),
 * with M1[k, d] = [m(k) >= d + 1] and M2[i, k] = [i + 1 > m(k)].  Real and
 * normalised over all 2^N configurations.  Only the unmasked weights are
 * parameters, K = N n_hidden + n_hidden + N, in the order
 *   [W1 (k ascending, then d = 0 .. m(k)-1) | b1 (n_hidden) |
 *    W2 (i ascending, then k ascending with m(k) <= i) | b2 (N)];
 * imaginary parts passed to set_params are dropped.  Float64 only
 * (set_precision with F32/BF16 returns VMC_ERR_UNSUPPORTED), no vmc_log_psi_vjp.
 * A sampler on this model draws independent samples directly (the Philox
 * stream of the masked network's sampler with the sampler's seed and counter
 * = the number of earlier vmc_sample calls); its proposal must be
 * VMC_PROP_FLIP, sweep and thermalisation settings are ignored and the
 * reported acceptance is 1.  N in [2, 1024], n_hidden in [1, 1024].          */
int vmc_model_create_autoregressive(vmc_ctx* ctx, int n_sites, int n_hidden, vmc_model** out);
/* Translation-symmetric single-layer network with ELU activation on a ring of
 * L sites, the ground-state ansatz of the paper's example (Sec. 5.1,
 * eq:gs_nqs):
 *   theta_{a,w} = b_a + sum_l W_{a,l} sigma_{(l + w) mod L},  sigma = 2 s - 1,
 *   log psi(s)  = sum_{a=1..alpha} sum_{w=0..L-1} ELU(theta_{a,w}),
 *   ELU(x) = x (x > 0), e^x - 1 (x <= 0).
 * Real parameters [W (alpha x L, row-major), b (alpha)], K = alpha (L + 1).
 * Float64; O_k also as F64 / F32; samplers take single flips (VMC_PROP_FLIP);
 * no vmc_log_psi_vjp.  L in [2, 1024], alpha in [1, 64], and alpha L small
 * enough for the per-configuration LDS tile (else VMC_ERR_INVALID_ARG).      */
int vmc_model_create_symelu(vmc_ctx* ctx, int L, int alpha, vmc_model** out);
/* Tabulated wave function (test model): the K = 2^N parameters are the
 * complex log-amplitudes, theta_code = log psi(s), code = sum_i bit_i 2^i
 * (n_sites <= 24).  log psi is a lookup, O_k(s) = [k = code(s)] (one-hot rows
 * of length 2^N), local energies read the connected amplitudes from the table,
 * and a sampler runs Metropolis chains with the same Philox stream, proposals
 * (flip or exchange) and acceptance rule as for the networks.  A table holding
 * an eigenvector has E_loc = E_0 wherever psi != 0 (Sec. 5.1).
 * logpsi_table_c128: 2^N complex128 on the device (NULL: all zero, i.e. the
 * uniform state); must be finite (VMC_ERR_NONFINITE).  Float64 only; no
 * vmc_log_psi_vjp.                                                          */
int vmc_model_create_table(vmc_ctx* ctx, int n_sites, const void* logpsi_table_c128, vmc_model** out);
int vmc_model_num_params(const vmc_model* m, int64_t* K);
int vmc_model_num_sites(const vmc_model* m, int* N);
/* Copies K parameters from device memory (dtype C128, C64 or, for real RBMs, F64)
 * into the model; converted to the model's internal float64 master copy.
 * Returns VMC_ERR_NONFINITE if any parameter is NaN/Inf (model unchanged). */
int vmc_model_set_params(vmc_model* m, const void* params_dev, int dtype);
/* Writes the K parameters as complex128 (dtype C128) or complex64 (C64). */
int vmc_model_get_params(const vmc_model* m, void* params_dev, int dtype);
/* Precision of network evaluation in vmc_log_psi and vmc_local_energy:
 * VMC_F64 (default) or, for the RBM, VMC_F32 / VMC_BF16: theta = b + W sigma on
 * the matrix cores with float32 accumulation (bfloat16: every parameter
 * rounded to bfloat16 first), log cosh / tanh and the connected-configuration
 * ratios in float32, all sums over hidden units, sites and slots in float64.
 * For the CNN the setting applies to TFIM local energies only (log psi stays
 * float64): the layer-1 log-cosh changes of all flips form one matrix that
 * multiplies a fixed matrix built from W2 on the matrix cores (bfloat16
 * operands with VMC_BF16, float32 with VMC_F32; float32 accumulation), layer
 * activations and log cosh in float32, window and slot sums in float64; it
 * needs Lx, Ly >= 2 kernel - 1 (else VMC_ERR_UNSUPPORTED).
 * O_k (vmc_grad_log_psi), the sampler and the SR solve are unaffected. */
int vmc_model_set_precision(vmc_model* m, int prec);
int vmc_model_destroy(vmc_model* m);

/* ---- Hamiltonians (Sec. 4.2 "Operators", eq:operator_mapping) ---------- */
/* Bonds: for each site i = y*Lx + x in order, the bond to +x, then (Ly > 1)
 * the bond to +y; periodic wraps, open boundaries drop wrapping bonds.  A
 * periodic direction needs length >= 3.
 * TFIM (Sec. 5): H = -J sum_<ij> Z_i Z_j - h sum_i X_i.                       */
int vmc_ham_create_tfim(vmc_ctx* ctx, int Lx, int Ly, int periodic, double J, double h, vmc_ham** out);
/* Heisenberg in Pauli matrices: H = J sum_<ij> (X_i X_j + Y_i Y_j + Z_i Z_j). */
int vmc_ham_create_heisenberg(vmc_ctx* ctx, int Lx, int Ly, int periodic, double J, vmc_ham** out);
/* M_max = 1 + N (TFIM) or 1 + n_bonds (Heisenberg). */
int vmc_ham_max_connected(const vmc_ham* H, int* M_max);
int vmc_ham_num_bonds(const vmc_ham* H, int* n_bonds);
/* The paper's get_s_primes (Sec. 4.2): for each configuration the connected
 * configurations and matrix elements, in the canonical slot order: slot 0 is
 * the diagonal (always present, element -J*(n_al - n_anti) for TFIM,
 * +J*(n_al - n_anti) for Heisenberg, one float64 product); then the non-zero
 * off-diagonal terms in term order (X on sites 0..N-1 with element -h;
 * exchange on anti-aligned bonds in bond order with element 2J).  Slots at
 * and beyond count[b] repeat s with element 0.
 *   sp:  B*M_max*W words;  mel: B*M_max doubles;  count: B int32.
 * Test export: the hot path (vmc_local_energy) never writes s' to memory.  */
int vmc_ham_connected(vmc_ham* H, const uint64_t* s, int64_t B, uint64_t* sp, double* mel, int32_t* count);
int vmc_ham_destroy(vmc_ham* H);

/* ---- hot path ------------------------------------------------------------ */
/* log psi(s) (the NQS __call__, Sec. 4.2) for B configurations.
 *   s: B*W words; logpsi: B complex128.  Im log psi is defined modulo 2*pi. */
int vmc_log_psi(vmc_model* m, const uint64_t* s, int64_t B, double* logpsi);

/* Local energy, eq:Oloc with O = H:
 *   E_loc(s) = sum_j H_{s s'_j} exp(log psi(s'_j) - log psi(s))
 * over the connected configurations of vmc_ham_connected (s' never leave the
 * chip).  logpsi_s is ignored (may be NULL): the kernel evaluates both sides
 * itself.  eloc: B complex128.  The model's site count must equal the
 * Hamiltonian's.                                                              */
int vmc_local_energy(vmc_model* m, vmc_ham* H, const uint64_t* s, int64_t B,
                     const double* logpsi_s, double* eloc);

/* Log-derivatives O_k(s) = d log psi(s) / d theta_k (Sec. 2.2; the complex
 * derivative for holomorphic nets, Sec. 2.3), flat parameter order.
 *   O: B*K elements, sample-major (row n = sample n), dtype C128 or C64; the
 *   real-parameter networks (autoregressive state, symmetric ELU network)
 *   also write F64 or F32.                                                    */
int vmc_grad_log_psi(vmc_model* m, const uint64_t* s, int64_t B, void* O, int dtype);

/* Reverse-mode product with the log-derivatives (the backward of log psi for
 * automatic differentiation in the conjugate-Wirtinger convention of
 * holomorphic maps):  out_k = sum_n g_n conj(O_nk(s_n)).
 *   g: B complex128 (the incoming cotangent);  out: K complex128.
 * O is recomputed from the configurations; no activations are stored.        */
int vmc_log_psi_vjp(vmc_model* m, const uint64_t* s, int64_t B, const double* g, double* out);

/* vmc_log_psi_vjp for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, result and kernels, but the scratch is a fixed 32 MiB
 * device array of the library (one per GPU, held until the process ends)
 * instead of the context's workspace, and the call makes no allocation of any
 * kind and does not synchronise.  Samples are processed in chunks that fit
 * the array, so any B works; a model whose smallest chunk does not fit (RBM:
 * 512 (N_h + 1)(N + 1) bytes plus one sample's 32 N_h + 8 N + 24 bytes; CNN:
 * 16 K bytes) returns VMC_ERR_WORKSPACE.  RBM and CNN models only
 * (VMC_ERR_UNSUPPORTED otherwise).  All calls on one GPU share the array:
 * calls that overlap on one GPU (other streams, other contexts, other host
 * threads) race and give wrong results; serialise them.                     */
int vmc_log_psi_vjp_noalloc(vmc_model* m, const uint64_t* s, int64_t B, const double* g, double* out);

/* Metropolis sampler of p(s) = |psi(s)|^2/<psi|psi> (Sec. 2.1, Sec. 4.2
 * "Sampler"), all chains in sync.
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11), key = (seed & 0xffffffff,
 * seed >> 32).  Proposal t (counted from 0 over the sampler's life) of chain c
 * uses x = Philox((c, t & 0xffffffff, t >> 32, 0)):
 *   flip:      site l = (x0 * N) >> 32, s' = s with bit l flipped;
 *   exchange:  bond b = (x0 * n_bonds) >> 32, the two spins of bond b swapped
 *              (aligned pair: identity move, accepted);
 *   u = ((x1 << 21) | (x2 >> 11)) * 2^-53;
 *   r = 2 Re(log psi(s') - log psi(s)); accept iff r >= 0 or u < exp(r).
 * Initial state of chain c: flip - word w = (y0 | y1 << 32) for w even and
 * (y2 | y3 << 32) for w odd, y = Philox((c, w/2, 0, 2)), masked to N bits;
 * exchange - sites 0..N/2-1 up, then Fisher-Yates for i = N-1..1 swapping i
 * with j = (y0 * (i+1)) >> 32, y = Philox((c, i, 1, 2)) (needs N even).
 * A sweep is sweep_steps proposals (0 = N); therm_sweeps sweeps run before the
 * first recorded sample of the sampler's life.                                */
typedef struct {
  int proposal;      /* VMC_PROP_FLIP | VMC_PROP_EXCHANGE | VMC_PROP_MADE_MIX */
  int n_chains;      /* > 0 */
  int sweep_steps;   /* proposals per sweep; 0 means N */
  int therm_sweeps;  /* thermalisation sweeps before the first sample */
  int global_steps;  /* MADE_MIX: global proposals at the start of every sweep, in [0, 1024] */
  uint64_t seed;
} vmc_sampler_opts;
/* The sampler keeps a reference to m (and H for bonds); both must outlive it. */
int vmc_sampler_create(vmc_ctx* ctx, vmc_model* m, vmc_ham* H, const vmc_sampler_opts* opts, vmc_sampler** out);
/* Draws ceil(n_samples / n_chains) sweeps' worth of samples, one per chain per
 * sweep, sample-major: output index k*n_chains + c.  s_out: n_written*W
 * words; logpsi_out: n_written complex128 (may be NULL).  *n_written and
 * *accept_rate_host (acceptance of this call's proposals; may be NULL) are
 * host outputs; the call synchronises the stream.  The buffers must hold the
 * rounded-up count.                                                          */
int vmc_sample(vmc_sampler* S, int64_t n_samples, uint64_t* s_out, double* logpsi_out,
               int64_t* n_written, double* accept_rate_host);
/* Chain state (configurations, step counter, seed) as a host byte blob;
 * *bytes in: capacity of buf_host (buf_host NULL: query size), out: size.
 * VMC_ERR_INVALID_ARG before the first vmc_sample (no state yet).  After
 * set_state the chains continue exactly as the saved sampler would have.    */
int vmc_sampler_get_state(vmc_sampler* S, void* buf_host, size_t* bytes);
int vmc_sampler_set_state(vmc_sampler* S, const void* buf_host, size_t bytes);
/* Acceptance statistics of the last vmc_sample call: overall acceptance (flips
 * and global proposals), the acceptance of global (MADE) proposals and their
 * number (MADE_MIX only). */
int vmc_sampler_get_stats(vmc_sampler* S, double* accept_rate_host, double* global_accept_rate_host,
                          int64_t* n_global_host);
/* Frozen MADE proposal used by VMC_PROP_MADE_MIX (the sampler copies its
 * parameters; later training of md does not affect the sampler).            */
int vmc_sampler_set_proposal_made(vmc_sampler* S, const vmc_made* md);
int vmc_sampler_destroy(vmc_sampler* S);

/* Regularised SR / TDVP solve: eq:qfm, eq:force_vector, eq:tdvp_util and the
 * diagonal shift of Sec. 3.1:
 *   S_kk' = <O_k^* O_k'> - <O_k^*><O_k'>,  F_k = <O_k^* E> - <O_k^*><E>,
 *   S~ = [[S]] + nu_rel * diag([[S]]) + eps_abs * I,
 *   S~ x = -[[gamma F]]   (Cholesky S~ = L L^H, two triangular solves).
 * <.> is the sample mean (weights == NULL) or the weighted mean with weights
 * normalised to sum 1.  The factor 2 of the SR gradient (eq:energy_gradient)
 * is left to the caller's step size: theta <- theta + tau * x.
 *   O: N*K sample-major, dtype C64 or C128, or real F32 / F64 (real
 *   log-derivatives: S is then real whatever the mode);  eloc: N complex128;
 *   weights: N doubles or NULL;  x: K complex128 (written on success).
 * S is formed on the matrix cores from centred O in float32 (C64 / F32 input)
 * or float64 (C128 / F64 input); factorisation and solves are float64.  The
 * complex products of the float32 Gram and of the Cholesky's block updates use
 * three real products per term (Re = A + B, Im = C - A + B with A = sum Re Re',
 * B = sum Im Im', C = sum (Re - Im)(Re' + Im') for the Gram; the bound on the
 * rounding error of Im grows by at most a factor of about 2).  Real O is packed
 * two samples per complex row (Re of the Gram of the packed matrix is S), which
 * halves the Gram work.
 * Returns VMC_ERR_NOT_PD with info->fail_index = first failing column, or
 * VMC_ERR_UNSUPPORTED for VMC_SR_IMAG (Im S is antisymmetric, not PD: that
 * projection is solved by vmc_sr_solve_eig).
 * info_host (may be NULL) is written on return; the call synchronises.       */
typedef struct {
  double nu_rel;     /* relative diagonal shift (the paper's nu) */
  double eps_abs;    /* additive shift */
  int mode;          /* VMC_SR_COMPLEX | VMC_SR_REAL | VMC_SR_IMAG */
  double gamma_re, gamma_im;  /* gamma = 1: SR / imaginary time; gamma = i: real time */
  int gram;          /* S product: 0 = by O dtype (float32 matrix cores for C64 / F32,
                        float64 for C128 / F64); 1 = split-float16 matrix-core products
                        (C64 / F32 input only): each centred value is scaled per column
                        by a power of two and split into hi + lo float16 parts,
                        three products per term, float32 accumulation, relative
                        error ~2^-21 per product term */
} vmc_sr_opts;
typedef struct {
  double e_mean[2];  /* <E_loc> */
  double e_var;      /* <|E_loc - <E_loc>|^2> */
  double residual;   /* ||S~ x + [[gamma F]]|| / ||[[gamma F]]|| */
  double min_pivot;  /* smallest Cholesky pivot (before the square root) */
  int64_t fail_index;  /* -1, or the column where factorisation failed */
} vmc_sr_info;
int vmc_sr_solve(vmc_ctx* ctx, const void* O, int O_dtype, const double* eloc, const double* weights,
                 int64_t N, int64_t K, const vmc_sr_opts* opts, double* x, vmc_sr_info* info_host);

/* Test export of the first half of vmc_sr_solve (eq:qfm, eq:force_vector):
 * the shifted matrix and the force exactly as the solve forms them (same
 * kernels, same arguments), with no factorisation.
 *   S_out: K*K complex128 (device, row-major, both triangles) receives
 *          S~ = [[S]] + nu_rel diag([[S]]) + eps_abs I; for VMC_SR_IMAG it
 *          receives the Hermitian matrix i Im[S] (purely imaginary entries,
 *          zero diagonal) that the eigen solve decomposes;
 *   F_out: K complex128 (device) receives F (not projected, no gamma).
 * info_host (may be NULL): e_mean and e_var; residual and min_pivot NaN.
 * Same argument rules as vmc_sr_solve; the call synchronises.               */
int vmc_sr_fisher(vmc_ctx* ctx, const void* O, int O_dtype, const double* eloc, const double* weights,
                  int64_t N, int64_t K, const vmc_sr_opts* opts, double* S_out, double* F_out,
                  vmc_sr_info* info_host);

/* The shifted system regularised through the eigendecomposition of S~
 * (Sec. 3.3 "Pseudo-inverse" and "Eliminating noisy contributions"):
 *   S~ = V diag(lambda) V^dagger (device Jacobi, vmc_eigh),
 *   rho = V^dagger [[gamma F]],  x = -V diag(lambda^+) rho, where
 *   lambda_j^+ = 1/lambda_j (0 if lambda_j = 0)                  eps_pinv = 0
 *              = 0 if |lambda_j/lambda_1| < eps_pinv, else 1/lambda_j   hard
 *              = 1/(lambda_j (1 + (eps_pinv/|lambda_j/lambda_1|)^6))   soft
 * with lambda_1 the eigenvalue of largest modulus, times 1/(1 + (eps_snr /
 * SNR_j)^6) when eps_snr > 0.  SNR_j = |rho_j| / sqrt(var_j / N) estimates the
 * signal-to-noise ratio of the Monte Carlo mean rho_j: var_j is the weighted
 * variance over samples of the eigen-basis components of the per-sample terms
 * f_n = [[gamma (E_n - <E>) conj(O_n - <O>)]] whose weighted sum is [[gamma F]]
 * (formed as V^dagger H V with H = sum_n w_n f_n f_n^dagger on the matrix cores).
 * Same inputs, projection modes and shifts as vmc_sr_solve, plus the Im
 * projection (eq:tdvp_im, real parameters of a non-holomorphic network, where
 * it keeps the symplectic structure and conserves energy; Sec. 2.3):
 * VMC_SR_IMAG solves Im[S~] x = -Im[gamma F] with A = Im[S~] real and
 * antisymmetric.  A has no real eigendecomposition; the Hermitian i A does
 * (eigenvalues in +- pairs, lambda_1 and the cutoffs as above), and A x = b is
 * (i A) x = i b, so the formulas above apply to i A, i b and the per-sample
 * terms i Im[f_n]; x is real (imaginary parts written as 0).  IMAG needs
 * complex O (C64 or C128) and eps_abs = 0 (else VMC_ERR_INVALID_ARG; nu_rel
 * has no effect since diag Im S = 0); with eps_pinv = 0 a numerically zero
 * eigenvalue (odd K) is inverted, so set a cutoff.
 * info: residual = ||S~ x + [[gamma F]]|| / ||[[gamma F]]|| (not small when
 * components are cut), min_pivot = smallest eigenvalue of S~ (of i A for
 * IMAG), fail_index -1.
 * evals (K float64, device, may be NULL): the eigenvalues (unordered);
 * snr (K float64, device, may be NULL): SNR_j (computed whenever snr is given);
 * *sweeps_host (may be NULL): Jacobi sweeps used.  O(K^3) per sweep: meant for
 * K up to a few thousand (K <= 16384).                                       */
typedef struct {
  double eps_pinv;  /* cutoff relative to |lambda_1| (0: plain inverse of the non-zero eigenvalues) */
  int soft;         /* 0: hard cutoff, 1: soft cutoff */
  double eps_snr;   /* signal-to-noise cutoff (0: none) */
  double tol;       /* Jacobi stops at ||offdiag(A)||_F <= tol ||A||_F (0: 1e-14) */
  int max_sweeps;   /* Jacobi sweep limit (0: 50) */
} vmc_eig_opts;
int vmc_sr_solve_eig(vmc_ctx* ctx, const void* O, int O_dtype, const double* eloc, const double* weights,
                     int64_t N, int64_t K, const vmc_sr_opts* opts, const vmc_eig_opts* eig, double* x,
                     vmc_sr_info* info_host, double* evals, double* snr, int* sweeps_host);

/* Quadratic form of the (unshifted) quantum Fisher matrix, eq:qfm:
 *   *out_host = v^dagger S v = sum_n w_n |(O_n - <O>) . v|^2   (weights normalised;
 *   NULL = uniform), computed from the samples without forming S (the step-size
 * control of the adaptive integrator measures changes in this norm, Sec. 4.3
 * "Stepper").  O as in vmc_sr_solve; v: K complex128 (device).  Synchronises. */
int vmc_fisher_quad(vmc_ctx* ctx, const void* O, int O_dtype, const double* weights, int64_t N, int64_t K,
                    const double* v, double* out_host);

/* Eigendecomposition of a Hermitian K x K complex128 matrix (row-major, both
 * triangles, device) by parallel cyclic Jacobi rotations in float64:
 * A = V diag(evals) V^dagger, V unitary (K x K complex128, row-major, columns
 * are eigenvectors), evals K float64 (unordered).  A is not modified.  tol and
 * max_sweeps as in vmc_eig_opts (0: defaults).  Synchronises the stream.     */
int vmc_eigh(vmc_ctx* ctx, const double* A, int64_t K, double tol, int max_sweeps, double* evals, double* V,
             int* sweeps_host);

/* The same shifted system solved by conjugate gradient (the paper notes, with
 * the diagonal shift of Sec. 3.1, that the shifted equation may be solved by
 * an iterative solver such as conjugate gradient).  S is never formed: each
 * iteration applies S v = Obar^H (Obar v) as two passes over O itself, the
 * centring and weights applied in float64 ((Obar v)_n = sqrt(w_n)(O_n.v -
 * <O>.v), (Obar^H u)_k = sum_n conj(O_nk) sqrt(w_n) u_n - conj(<O_k>) sum_n
 * sqrt(w_n) u_n, w normalised), so the operator is exactly that of the given
 * O, plus the shift
 * nu_rel diag(S) + eps_abs; Jacobi preconditioner M = (1 + nu_rel) diag(S) +
 * eps_abs.  Stops when the recursive residual ||r|| / ||b|| <= tol (checked
 * every 8 iterations) or after max_iter iterations; info->residual is then
 * the true residual ||b - S~ x|| / ||b||, recomputed with one more product
 * (check it against tol: reaching max_iter is not an error).  info->min_pivot
 * is NaN and fail_index -1; opts->gram is ignored.  Workspace O((N + K) *
 * (1 + N / 256)) values: no K x K matrix and no copy of O, so K is not limited
 * to 65536.
 * VMC_ERR_UNSUPPORTED for VMC_SR_IMAG.  iterations_host (may be NULL)
 * receives the number of iterations.  The call synchronises.                 */
typedef struct {
  double tol;    /* relative residual target, > 0 */
  int max_iter;  /* >= 1 */
} vmc_cg_opts;
int vmc_sr_solve_cg(vmc_ctx* ctx, const void* O, int O_dtype, const double* eloc, const double* weights,
                    int64_t N, int64_t K, const vmc_sr_opts* opts, const vmc_cg_opts* cg, double* x,
                    vmc_sr_info* info_host, int* iterations_host);

/* ---- learned proposal: masked autoregressive network (MADE) ------------- */
/* q(s) = prod_d p_d^{s_d} (1-p_d)^{1-s_d},  p = sigmoid(W2m relu(W1m sigma' + b1) + b2)
 * with MADE masks (Germain et al. 2015; hidden degree m(k) = k mod (N-1) + 1,
 * M1[k,d] = [m(k) >= d+1], M2[d,k] = [d+1 > m(k)]) on input x = s (0/1).
 * Flat order: [W1 (H x N), b1 (H), W2 (N x H), b2 (N)], float64 on the host side. */
int vmc_made_create(vmc_ctx* ctx, int n_in, int n_hidden, vmc_made** out);
int vmc_made_num_params(const vmc_made* md, int64_t* P);
int vmc_made_set_params(vmc_made* md, const double* params_dev);
int vmc_made_get_params(const vmc_made* md, double* params_dev);
/* log q(s) for B configurations (float64 out). */
int vmc_made_log_q(vmc_made* md, const uint64_t* s, int64_t B, double* logq);
/* Mean negative log-likelihood gradient over B configurations, flat order. */
int vmc_made_nll_grad(vmc_made* md, const uint64_t* s, int64_t B, double* grad, double* nll_host);
/* Adam (Kingma & Ba 2015; beta1 0.9, beta2 0.999, eps 1e-8) on minibatches of
 * `batch` rows of s for `epochs` passes in order; *nll_host = mean NLL of the
 * last epoch.                                                                 */
int vmc_made_train(vmc_made* md, const uint64_t* s, int64_t B, int epochs, int batch, double lr, double* nll_host);
/* Autoregressive samples: row c uses Philox((c, counter_lo, counter_hi, 1 + 256*(d/4))),
 * site d up iff x_{d%4} * 2^-32 < p_d.  s_out: B*W words; logq: B doubles.
 * In VMC_PROP_MADE_MIX every sweep (thermalisation sweeps included) starts
 * with global_steps global proposals made by all chains together, then the
 * sweep's single-spin flips of VMC_PROP_FLIP (their counter t counts flips
 * only).  Global proposal g of chain c (g counted from 0 over the sampler's
 * life) is the sample of row c with counter g, accepted iff r >= 0 or
 * u < exp(r),  r = 2 Re(log psi(s') - log psi(s)) + log q(s) - log q(s'),
 * u = ((x1 << 21) | (x2 >> 11)) 2^-53 of x = Philox((c, g_lo, g_hi, 3)).
 * Each global step and each flip leaves |psi|^2 invariant.  The sampler
 * draws the proposals (with their log q and theta) blocked over 16 sites at
 * a time on the float64 matrix cores, one global step ahead, on a second
 * stream of default priority that it creates and owns; vmc_sample orders
 * later work on the context's stream after that stream's work.  log q of
 * the chain states comes from the plain masked forward pass: the same logits
 * up to rounding order (about 1e-14 relative, below the 2^-32 resolution of
 * the draws).  The MADE must fit the blocked pass: 16 (H + 1) + 1280
 * doubles, 16 W words and H + 32 ints of LDS (H <= 1024 with W <= 64 does). */
int vmc_made_sample(vmc_made* md, int64_t B, uint64_t seed, uint64_t counter, uint64_t* s_out, double* logq);
int vmc_made_destroy(vmc_made* md);

/* ---- measurement utilities (not part of the method) --------------------- */
/* Plain device copy of `bytes` (a positive multiple of 16; 16-byte aligned
 * device buffers, not overlapping) on the context's stream: the HBM bandwidth
 * reference, and the known transfer against which hardware traffic counters
 * are scaled.  Timed as phase "calib.copy" when timing is on.               */
int vmc_calib_copy(vmc_ctx* ctx, const void* src, void* dst, int64_t bytes);
/* Read-only stream over `bytes` (a positive multiple of 16, 16-byte aligned):
 * the bandwidth ceiling of read-dominated kernels.  out: device buffer of
 * 8192 x 16 bytes receiving one xor-folded word per work-group.  Phase
 * "calib.read".                                                              */
int vmc_calib_read(vmc_ctx* ctx, const void* src, int64_t bytes, void* out);
/* Matrix-core loop: n_groups work-groups of 4 waves, each wave `iters` rounds
 * of 8 independent chains of one MFMA type: kind VMC_DT_F64
 * (v_mfma_f64_16x16x4f64), VMC_DT_F32 (v_mfma_f32_16x16x4f32) or
 * VMC_CALIB_BF16 (v_mfma_f32_16x16x32_bf16).  out: device buffer of
 * n_groups*256 elements (double for F64, float otherwise) that receives the
 * accumulator sums.  *flops_host = the flops issued.  Phase "calib.mfma".    */
enum { VMC_CALIB_BF16 = 16 };
int vmc_calib_mfma(vmc_ctx* ctx, int kind, int n_groups, int iters, void* out, double* flops_host);

#ifdef __cplusplus
}
#endif
#endif /* NQSVMC_H */
