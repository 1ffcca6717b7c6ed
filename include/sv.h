/*
 * sv.h -- C ABI of libsv.so, a state-vector gate-application library for one
 * AMD MI355X (gfx950) GPU.
 *
 * What it computes (Sec. II-A of the paper, Eq. 1-4): an n-qubit state is a
 * vector of 2^n complex amplitudes; a k-qubit gate is a dense 2^k x 2^k
 * complex matrix U applied by matrix-vector product to each of the 2^(n-k)
 * groups of amplitudes that agree on every non-target bit and enumerate the
 * target bits.  Gates on disjoint qubits combine by tensor product (Eq. 3) and
 * gates on the same qubits by matrix product; the fusion pass (Sec. II-C,
 * Sec. IV-D) builds such combined gates so that each pass over the state does
 * more work per byte.
 *
 * Conventions used by every entry point:
 *   - qubit q is bit q of the amplitude index (0-based, little-endian);
 *   - a gate's matrix is row-major, 2^k x 2^k complex128 given as 2*4^k
 *     doubles with re/im interleaved; local bit j of its row/column index is
 *     state bit qubits[j]; the output is w = U v;
 *   - the device state is complex64 with re/im interleaved (8 bytes per
 *     amplitude), in a buffer the caller allocates and owns;
 *   - every call returns an int status (SV_OK or a negative code); nothing
 *     aborts or throws across the ABI; sv_last_error() describes the last
 *     failure on the calling thread.  Validation happens before any device
 *     work: a call that fails with SV_EINVAL leaves the state untouched.
 *   - a HIP runtime failure returns SV_EDEVICE and poisons the handle: every
 *     later call on it returns SV_ESTATE except sv_free.
 *   - calls on one handle are not thread-safe; distinct handles are.
 */
#ifndef SV_H
#define SV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define SV_OK 0
#define SV_EINVAL (-1)        /* bad argument: qubit range/duplicate, k, null, sizes */
#define SV_ENOMEM (-2)        /* buffer too small or an allocation failed */
#define SV_EDEVICE (-3)       /* a HIP runtime call failed */
#define SV_EUNSUPPORTED (-4)  /* valid request this build does not implement */
#define SV_ESTATE (-5)        /* handle poisoned by an earlier device failure */

/* ---- enumerations ------------------------------------------------------- */
#define SV_C64 0              /* state dtype: complex64 (the only one built) */

/* Arithmetic of a pass.  FP32_VALU: every pass on vector FP32 FMAs
 * (register passes with at most four targets besides bit 0 multiply in the
 * 3M form, three real products per complex multiply-accumulate, with the
 * matrix's ur + ui and ui - ur formed in FP64).
 * FP32_MFMA: passes with k >= 4 as a real GEMM in the 4M form
 * [Yr;Yi] = [[Ur,-Ui],[Ui,Ur]] [Xr;Xi] on FP32 matrix cores.
 * BF16X3 / FP16X3: the same GEMM with every operand split into hi + lo
 * halves of the narrow type and three products (hi*hi + hi*lo + lo*hi)
 * accumulated in FP32; FP16X3 scales amplitudes by 2^14 before the split,
 * so it needs |c| < ~4: sv_apply_circuit at FP16X3 rejects (SV_EINVAL) a
 * circuit with a gate that is not unitary, or a state whose sum |c|^2 may
 * exceed 15 (after sv_write_amplitudes or a non-unitary gate it measures the
 * sum once with one read sweep before deciding). */
#define SV_PREC_FP32_VALU 0
#define SV_PREC_FP32_MFMA 1
#define SV_PREC_BF16X3 2
#define SV_PREC_FP16X3 3

/* Fusion policy of sv_apply_circuit / sv_fuse.  NONE applies every gate as
 * its own pass; GREEDY builds blocks of at most max_k qubits (vertical fusion
 * by matrix product, horizontal by tensor product, per-qubit order kept);
 * BLOCK is greedy in passes: each pass takes the set of at most max_k qubits
 * that absorbs the most remaining gates (grown from every gate of the current
 * front), which needs far fewer passes than GREEDY on lattice circuits.
 * LEARNED scores candidate partitions (GREEDY for every k <= max_k,
 * cost-aware GREEDY variants, BLOCK, beam searches over BLOCK's passes,
 * PHASE) with the cost-model network loaded by sv_cost_model_load and keeps
 * the cheapest, unless it has more passes than the fewest-pass candidate and
 * is predicted less than 5 % cheaper; with no model loaded it keeps the
 * candidate with the fewest passes (every pass moves the same bytes).  For
 * states of 28 qubits and more at BF16X3, FP16X3 or FP32_MFMA, LEARNED also
 * lets a block take diagonal gates that reach up to 3 qubits outside its
 * targets (at bit 4 or above) as control bits: such a block is one gate per
 * control value on the same targets, and sv_apply_circuit runs all of them
 * as one matrix-core launch when the block has k >= 4 targets.  PHASE is
 * GREEDY in which pure-phase diagonal gates of at most two qubits (CZ, CP,
 * RZ, Z, S, T, ...) never block one another: those
 * that fit join dense blocks, the others are gathered into phase blocks of
 * any width.  sv_fuse returns a phase block as its canonical diagonal gates
 * (one CP-form gate per interacting pair, one diagonal per qubit); in
 * sv_apply_circuit every maximal run of such gates is one elementwise pass
 * that multiplies amplitude i by exp(i * theta(i)), theta a quadratic
 * polynomial in the bits of i. */
#define SV_FUSE_NONE 0
#define SV_FUSE_GREEDY 1
#define SV_FUSE_LEARNED 2
#define SV_FUSE_PHASE 3
#define SV_FUSE_BLOCK 4

/* Kernel variant of a pass (for tests and tuning; AUTO is the default).
 * REG: each lane owns whole groups in registers, gathered straight from HBM
 * (coalesced when no target sits in the low 7 bits).  LDS: a workgroup
 * stages a tile of 2^T amplitudes in LDS and scatters groups from there
 * (for low targets).  MFMA: matrix-core GEMM (k >= 4 and an MFMA precision). */
#define SV_VARIANT_AUTO 0
#define SV_VARIANT_REG 1
#define SV_VARIANT_LDS 2
#define SV_VARIANT_MFMA 3
#define SV_VARIANT_SHFL 4     /* all targets in bits 0..6 (two or three in 1..6: within 1..5), k <= 3: one coalesced
                                 16-byte element per lane, partners by cross-lane permutes */

#define SV_MAX_K 6            /* largest fused gate */
#define SV_MAX_QUBITS 40      /* largest state the index arithmetic supports */
#define SV_COST_FEATURES 40   /* k, n, 34-bit target mask, 4 precision one-hot */

/* ---- types -------------------------------------------------------------- */
typedef struct sv_state sv_state; /* opaque handle */

/* One gate: k target qubits (qubits[0..k-1], distinct, any order) and its
 * matrix (2*4^k doubles, borrowed for the duration of the call only).
 * Controls (Eq. 4's indicator 1_c): the gate acts only on the basis states
 * whose bits in cmask equal those of cval and leaves every other amplitude
 * untouched.  cmask = 0 (a zero-initialised struct) is an ordinary gate;
 * cmask must be disjoint from the targets and cval a subset of cmask. */
typedef struct {
  int32_t k;
  int32_t qubits[SV_MAX_K];
  const double* matrix;
  uint64_t cmask;
  uint64_t cval;
} sv_gate;

typedef struct {
  int32_t max_k;      /* fusion block size limit, 1..6 (ignored for NONE) */
  int32_t fusion;     /* SV_FUSE_* */
  int32_t precision;  /* SV_PREC_* */
  int32_t use_graph;  /* 1: launch the passes as one hipGraph on the handle's
                         stream (captured on a private stream of the handle,
                         so any stream works).  The handle keeps the last graph and
                         a device copy of its pass data.  A later call with the
                         same gates, matrix values and options (and no cost
                         model or tuned table loaded in between) relaunches it
                         without fusing or uploading; one whose passes encode to
                         the same bytes relaunches it after fusing.  A different
                         circuit replaces it (the stream is synchronised first). */
  int32_t variant;    /* SV_VARIANT_* (AUTO unless a test forces one) */
  int32_t timing;     /* 1: bracket every pass with HIP events on the handle's
                         stream and report per-variant device time in stats
                         (needs stats; passes are then launched without a graph) */
} sv_run_opts;

typedef struct {
  uint64_t gates_in;     /* gates given */
  uint64_t passes;       /* fused passes launched */
  uint64_t bytes;        /* algorithmic HBM bytes: 16 * 2^n per pass, 16 * 2^(n-c)
                            for a controlled pass with c controls; for sv_batch_run
                            16 * 2^n per LDS-resident circuit (one read, one write)
                            plus 16 * 2^n per pass of every other circuit */
  double useful_flops;   /* sum over passes of groups * 2^k (8*2^k - 2), groups =
                            2^(n-k) (2^(n-k-c) for a controlled pass) */
  double fuse_s;         /* host time in the fusion pass */
  double gpu_s;          /* device time of the passes (HIP events) */
  double variant_s[5];   /* with opts.timing: device time per kernel family: 1 register
                            (gather or wavefront shuffle, controlled passes included),
                            2 LDS, 3 matrix core, 4 phase-only (index 0 unused) */
  uint64_t variant_passes[5]; /* with opts.timing: passes per kernel family */
  uint64_t graph_relaunched;  /* 1 when opts.use_graph relaunched the handle's kept
                                 graph without capturing a new one */
  uint64_t variant_bytes[5];  /* with opts.timing: algorithmic bytes per kernel family */
  uint64_t launches;          /* kernel launches the call issued (inside its graph when it
                                 ran as one): one per pass for sv_apply_circuit; for
                                 sv_batch_run one LDS-resident launch plus one per level */
} sv_run_stats;

/* ---- state -------------------------------------------------------------- */

/* The state of Sec. II-A, Eq. 1: 2^n complex amplitudes, here complex64.
 * Wrap a caller-owned device buffer as an n-qubit complex64 state and write
 * |0...0> into it (asynchronously on `hip_stream`, a hipStream_t or NULL for
 * the default stream).  dev_buf must hold at least 8 * 2^n bytes and stay
 * valid until sv_free; it is never freed by the library.  1 <= n <= 40.
 * The library allocates only the handle and a small device arena for gate
 * matrices and reduction partials.  Errors: SV_EINVAL (n, dtype, null),
 * SV_ENOMEM (buf_bytes < 8 * 2^n or arena allocation). */
int sv_alloc(int n_qubits, int dtype, void* dev_buf, size_t buf_bytes, void* hip_stream,
             sv_state** out);

/* Release the handle and its arena (waits for the handle's stream first).
 * Never frees the borrowed state buffer.  NULL is accepted. */
int sv_free(sv_state* s);

/* Overwrite the state with the basis state |index> (Eq. 1 with the single
 * amplitude c_index = 1; the basis-state inputs of the Sec. VI circuits),
 * asynchronously.  SV_EINVAL if index >= 2^n. */
int sv_set_basis(sv_state* s, uint64_t index);

/* Number of qubits of a handle (or SV_EINVAL for NULL). */
int sv_num_qubits(const sv_state* s);

/* ---- gate application (Eq. 4) ------------------------------------------- */

/* Apply one k-qubit gate (1 <= k <= min(6, n)) in FP32 on the handle's
 * stream.  The matrix is rounded once to complex64 and copied before the
 * call returns, so the caller may reuse it immediately.  Asynchronous.
 * SV_EINVAL: qubit out of range or repeated, bad k, NULL matrix/qubits. */
int sv_apply_gate(sv_state* s, const int32_t* qubits, int k, const double* matrix);

/* Controlled gate (Eq. 4 with the indicator 1_c; the paper's controlled-gate
 * kernel, Sec. IV): apply the k-qubit matrix to the targets only on the
 * 2^(n-k-nc) groups whose control qubits controls[0..nc-1] hold
 * control_values[0..nc-1] (each 0 or 1; NULL means all 1), in FP32 on the
 * handle's stream, touching only those groups' amplitudes.  Controls and
 * targets are distinct; 0 <= nc and k + nc <= n.  Asynchronous; the matrix
 * is copied before the call returns.  SV_EINVAL on bad arguments. */
int sv_apply_controlled_gate(sv_state* s, const int32_t* qubits, int k, const double* matrix, int nc,
                             const int32_t* controls, const int32_t* control_values);

/* Apply a circuit: validate all gates, fuse them per opts (FP64 on the host),
 * round each fused matrix once to the pass precision, upload every matrix
 * with one host-to-device copy, then launch one in-place pass per fused gate
 * (as one hipGraph when opts->use_graph).  opts NULL means {max_k 4, GREEDY,
 * FP32_VALU, no graph, AUTO}.  FUSE_NONE + FP32_VALU is the plain unfused
 * FP32 baseline: same kernels, one pass per gate.  When stats is not NULL the
 * call waits for the passes and fills it; otherwise it returns once the work
 * is queued.  The result equals applying the gates one at a time in order,
 * up to FP32 (or split-precision) rounding.  A controlled gate whose targets
 * and controls together span at most max_k qubits is lifted to a dense gate
 * on those qubits and fused (not with FUSE_NONE); a wider one is applied as
 * a controlled pass of its own: on the matrix cores at an MFMA precision when
 * it has k >= 4 targets and at most 3 controls (none on bit 0), else in FP32.
 * Consecutive controlled gates on the same targets and controls covering
 * every control value (a fused block with controls) run as one launch. */
int sv_apply_circuit(sv_state* s, const sv_gate* gates, size_t n_gates, const sv_run_opts* opts,
                     sv_run_stats* stats);

/* ---- fusion (Sec. II-C, Sec. IV-D; Eq. 3) ------------------------------- */

/* Fuse a gate list on the host in FP64 without touching any device.  On
 * success *out is a library-allocated array of *n_out fused gates whose
 * qubits are ascending and whose matrices are the ordered products of the
 * absorbed gates lifted to the block's qubits; (*block_of_gate)[i] is the
 * index of the fused gate that absorbed input gate i (for a block with
 * control bits, which comes out as 2^c controlled gates, the first of them).
 * Applying *out in order equals applying `in` in order.  Free with sv_fused_free.  n_qubits bounds
 * the qubit indices.  block_of_gate may be NULL. */
int sv_fuse(const sv_gate* in, size_t n_in, int n_qubits, const sv_run_opts* opts, sv_gate** out,
            size_t* n_out, int32_t** block_of_gate);
int sv_fused_free(sv_gate* fused, size_t n, int32_t* block_of_gate);

/* ---- reductions and read-back ------------------------------------------- */

/* sum_i |c_i|^2 (Eq. 1), FP32 products accumulated in FP64 through a
 * two-level block reduction.  Synchronises the handle's stream. */
int sv_norm(sv_state* s, double* norm_sq);

/* sv_norm for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): no
 * handle, no allocation, no synchronisation.  Enqueues on hip_stream (a
 * hipStream_t, NULL for the default stream) the same two-level FP64
 * reduction sum_i |c_i|^2 as sv_norm over the complex64 state at dev_state
 * (re/im interleaved, 8 * 2^n_qubits bytes within buf_bytes, 16-byte
 * aligned, caller-owned) and writes the result to the device double at
 * dev_out (caller-owned, 8-byte aligned) when the stream reaches it.  Both
 * pointers must be device memory on the calling thread's current device.
 * The first-level partials live in a static per-device scratch of 2048
 * doubles (16 KiB, held by each device the library runs on until the
 * process ends); every call writes the partials it reads, so nothing has
 * to be cleared.  Every call on one device shares that scratch: calls whose
 * execution overlaps on one GPU (on different streams) race.  States of
 * 1..40 qubits (SV_MAX_QUBITS); anything else is SV_EINVAL.  Errors:
 * SV_EINVAL (NULL, bad alignment, n_qubits outside 1..40, buf_bytes <
 * 8 * 2^n, a pointer that is not device memory on the current device),
 * SV_EDEVICE (a launch failed). */
int sv_norm_noalloc(const void* dev_state, int n_qubits, size_t buf_bytes, void* hip_stream, double* dev_out);

/* Expectation values of Pauli strings (the paper's expectation-value kernel,
 * Sec. IV: a read of the state that writes nothing back).  Term t is the
 * string with X on the qubits of xmask[t] only, Z on zmask[t] only and Y on
 * both; out[t] = <psi|P_t|psi> (real: P_t is Hermitian), not divided by
 * <psi|psi>.  Products are formed in FP32 from the complex64 amplitudes and
 * accumulated in FP64.  Terms that share an X/Y part share one sweep of the
 * state (up to 8 terms per sweep).  Synchronises the handle's stream.
 * SV_EINVAL: a mask reaches past n, n_terms > 0 with NULL arrays. */
int sv_expect_pauli(sv_state* s, size_t n_terms, const uint64_t* xmask, const uint64_t* zmask, double* out);

/* Born probabilities of measuring m = n_meas qubits (1 <= m <= 12):
 * out[o] (2^m doubles) = sum of |c_i|^2 over the indices whose bit
 * qubits[j] is bit j of o.  Squares in FP32, sums in FP64.  Synchronises. */
int sv_marginal_probs(sv_state* s, int n_meas, const int32_t* qubits, double* out);

/* Sample basis states from p_i = |c_i|^2 by the inverse CDF: for each
 * uniforms[j] in [0, 1), out[j] = the smallest i with p_0 + ... + p_i >
 * uniforms[j] * sum(p) (FP64 prefix sums; a value past the end, from
 * rounding, takes the last index with p_i > 0).  The caller draws the
 * uniforms, so the result is reproducible.  The state is not changed.
 * Synchronises.  SV_EINVAL: a uniform outside [0, 1), NULL arrays, or a
 * zero state. */
int sv_sample(sv_state* s, size_t n_shots, const double* uniforms, uint64_t* out);

/* Read-back of the final state vector, which Sec. VI compares amplitude by
 * amplitude with a reference simulator.  Copy amplitudes [start, start +
 * count) to host memory as complex64 (2*count floats, re/im interleaved,
 * caller-owned), in chunks of 2^26 amplitudes.  Synchronous.  SV_EINVAL if
 * start + count > 2^n or host_out is NULL. */
int sv_read_amplitudes(sv_state* s, uint64_t start, uint64_t count, float* host_out);

/* Load amplitudes of a prepared state (any linear combination of Eq. 1; it
 * need not be normalised) or of a checkpoint: copy 2*count floats from host
 * (complex64, interleaved, caller-owned) into [start, start+count).
 * Synchronous.  SV_EINVAL if start + count > 2^n or host_in is NULL. */
int sv_write_amplitudes(sv_state* s, uint64_t start, uint64_t count, const float* host_in);

/* ---- batching ------------------------------------------------------------ */

/* Many independent circuits at once: the group parallelism of Sec. IV
 * (every group of every circuit's pass is independent) spread over a whole
 * batch, with each circuit fused as in Sec. II-C.  Runs n_circuits circuits,
 * circuit c on states[c] (each handle on the same device).  The work is
 * queued on the stream of states[0], after the work already queued on the
 * other handles' streams; the call returns once it has finished.  All
 * launches are captured in one hipGraph: circuits whose state fits in LDS
 * (n <= the autotuned limit: at most 14 qubits = 128 KiB, and no more than
 * the device's LDS per workgroup) run in one workgroup each, entirely on
 * chip, with one HBM read and one write;
 * larger ones advance one fused pass per launch of a level kernel that
 * covers that pass of every circuit that has one (the kernel boundary is
 * the barrier between a circuit's dependent passes).  On a device failure
 * every handle in the batch is poisoned.  Gates are fused first per opts (fusion mode and max_k; GREEDY
 * with max_k 4 when opts is NULL; the precision is always FP32), circuits on
 * host threads.  A controlled gate wider than max_k with its controls is
 * rejected (SV_EINVAL).  States of at most 30 qubits.  When stats is not NULL
 * the call waits and fills it.  Equivalent to sv_apply_circuit on each state
 * in turn. */
int sv_batch_run(sv_state* const* states, const sv_gate* const* circuits, const size_t* n_gates,
                 size_t n_circuits, const sv_run_opts* opts, sv_run_stats* stats);

/* ---- autotuner ----------------------------------------------------------- */

/* Time the candidate tile shapes of every kernel variant on a scratch state
 * of n qubits on the handle's device (the handle's state is overwritten) and
 * keep the fastest per (variant, k, lowest-target bucket, precision).
 * Results persist across calls in this process; sv_tune_save/sv_tune_load
 * write and read them as JSON. */
int sv_autotune(sv_state* s, int budget_ms);
int sv_tune_save(const char* path);
int sv_tune_load(const char* path);

/* ---- learned fusion cost model (3-layer MLP, FP32, trained on the GPU) --- */

typedef struct sv_mlp sv_mlp; /* opaque: parameters + Adam moments on the device */

/* Network SV_COST_FEATURES -> width -> width -> 1 with ReLU; parameters drawn
 * He-uniform from a SplitMix64 stream seeded by `seed`.  All device work on
 * hip_stream. */
int sv_mlp_create(int width, uint64_t seed, void* hip_stream, sv_mlp** out);
int sv_mlp_free(sv_mlp* m);
/* Number of parameters and their flat layout: W1 [width x F], b1 [width],
 * W2 [width x width], b2 [width], W3 [1 x width], b3 [1] (row-major). */
int sv_mlp_num_params(const sv_mlp* m, size_t* count);
int sv_mlp_get_params(sv_mlp* m, float* host_params);
int sv_mlp_set_params(sv_mlp* m, const float* host_params);
/* Forward pass on device arrays: x [batch x SV_COST_FEATURES] -> y [batch]. */
int sv_mlp_forward(sv_mlp* m, const float* x_dev, int batch, float* y_dev);
/* Mean squared error of forward(x) against y and its gradient with respect to
 * every parameter (same layout as the parameters), both copied to the host;
 * grad_host may be NULL. */
int sv_mlp_loss_grad(sv_mlp* m, const float* x_dev, const float* y_dev, int batch, float* loss_host,
                     float* grad_host);
/* One Adam update with the gradient of the last sv_mlp_loss_grad. */
int sv_mlp_adam_step(sv_mlp* m, float lr, float beta1, float beta2, float eps);
/* Full-batch training loop on the device (loss_grad + adam per epoch);
 * *final_loss receives the last loss. */
int sv_mlp_train(sv_mlp* m, const float* x_dev, const float* y_dev, int n, int epochs, float lr,
                 float* final_loss);
/* Install the network's current parameters as the cost model used by
 * SV_FUSE_LEARNED (host copy; the network may be freed afterwards), or load
 * / save them from / to a little-endian float32 file with a small header. */
int sv_cost_model_install(sv_mlp* m);
int sv_cost_model_save(const char* path);
int sv_cost_model_load(const char* path);
/* Remove the installed cost model: SV_FUSE_LEARNED then runs the same
 * candidate search and keeps the partition with the fewest passes (what the
 * method does without the network).  Always SV_OK. */
int sv_cost_model_clear(void);
/* Host-side prediction of log(pass seconds / 2^n) for a gate (k, qubits,
 * n, precision) under the installed model: what the partition search uses. */
int sv_cost_model_predict(int k, const int32_t* qubits, int n_qubits, int precision, double* out);
/* Feature vector of a pass as the model sees it (SV_COST_FEATURES floats). */
int sv_cost_features(int k, const int32_t* qubits, int n_qubits, int precision, float* out);

/* ---- diagnostics --------------------------------------------------------- */

/* Describe the last failure on this thread; valid until the next call. */
const char* sv_last_error(void);
/* Library version string. */
const char* sv_version(void);
/* sizeof of an ABI struct, for bindings to check their layout: which 0
 * sv_gate, 1 sv_run_opts, 2 sv_run_stats; 0 for any other value. */
size_t sv_struct_size(int which);

#ifdef __cplusplus
}
#endif
#endif /* SV_H */
