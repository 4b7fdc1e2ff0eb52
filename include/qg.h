/*
 * qg.h -- C ABI of the MI355X state-vector circuit simulator (libqg.so).
 *
 * The library simulates the method of Q-GEAR (arXiv 2504.03967): a circuit given
 * as gate-list tensors (Sec. 2.1 "Circuit encoding", App. B) is applied to a
 * 2^n-amplitude complex state (App. A, eq. (hilbert)), which is then reduced to
 * probabilities, seeded shot samples and Pauli-Z-string expectation values
 * (the "circuit in, state and counts out" statement of Sec. 2 and App. A).
 *
 * Conventions shared by every entry point:
 *  - Qubit q is bit q of the amplitude index (little-endian).  App. A's
 *    3-qubit CX example (control q0, target q2 exchanges |100>,|101> and
 *    |110>,|111>) is indices 1<->5 and 3<->7 under this reading.
 *  - Amplitudes are interleaved complex: {re, im} pairs of double (QG_C128,
 *    16 bytes) or float (QG_C64, 8 bytes), index-contiguous in device memory.
 *  - Every call returns a qg_status (0 = success, < 0 = error) and never
 *    throws.  On error, qg_last_error() returns a message for the calling
 *    thread.  Arguments are validated on the host before anything is launched:
 *    a failed validation leaves the state and all outputs untouched.
 *  - Host arrays passed in (gate tensors, index lists, masks, coefficients)
 *    are read before the call returns; the caller keeps ownership.
 *  - Output pointers are device pointers owned by the caller.  Work is
 *    enqueued on the HIP stream given to the call (or bound to the state) and
 *    is asynchronous: outputs are valid after that stream has been
 *    synchronised.  A kernel fault surfaces as QG_EDEVICE on a later call.
 *  - A qg_state handle may be used from one thread at a time.
 */
#ifndef QGEAR_MI355X_QG_H_
#define QGEAR_MI355X_QG_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QG_OK = 0,
    QG_EINVAL = -1,       /* an argument failed validation */
    QG_ENOMEM = -2,       /* a device or host allocation failed, or the state does not fit */
    QG_EDEVICE = -3,      /* a HIP runtime call or kernel launch failed */
    QG_EUNSUPPORTED = -4, /* valid request the library does not implement */
    QG_EINTERNAL = -5
} qg_status;

typedef enum { QG_C64 = 0, QG_C128 = 1 } qg_dtype;

/* Gate codes of the circuit encoding.  Matrices act on (alpha_{bit=0}, alpha_{bit=1})
 * of the target; c = cos(theta/2), s = sin(theta/2):
 *   H = [[1,1],[1,-1]]/sqrt2        X = [[0,1],[1,0]]
 *   RX = [[c,-is],[-is,c]]          RY = [[c,-s],[s,c]]
 *   RZ = diag(e^{-i theta/2}, e^{+i theta/2})
 *   U3(theta,phi,lambda) = [[c, -e^{i lambda} s], [e^{i phi} s, e^{i(phi+lambda)} c]]
 *   CX: X on q1 where bit q0 = 1 (App. A, eq. (cx))
 *   CZ: -1 where bits q0 and q1 are both 1
 *   CP(theta): e^{i theta} where bits q0 and q1 are both 1 (the CR1 of eq. (cr1))
 *   SWAP: exchange bits q0 and q1 */
typedef enum {
    QG_H = 0, QG_X = 1, QG_RX = 2, QG_RY = 3, QG_RZ = 4, QG_U3 = 5,
    QG_CX = 6, QG_CZ = 7, QG_CP = 8, QG_SWAP = 9
} qg_op;

/* Fusion modes of qg_apply_circuit. */
typedef enum {
    QG_FUSE_NONE = 0,    /* one device pass per gate */
    QG_FUSE_GREEDY = 1,  /* greedy fixed-width fusion: a pass holds gates whose non-diagonal
                            targets span at most 5 qubits outside the low, always-resident
                            tile qubits (the fusion width 5 of App. D.2); gates on
                            disjoint qubits commute, so each pass takes every pending gate
                            that fits and is not blocked by an earlier gate on its qubits */
    QG_FUSE_LEARNED = 2  /* cost-model planner (qg_mlp_*); falls back to greedy without a model */
} qg_fusion;

typedef struct qg_state qg_state; /* opaque */

/* One circuit in the encoding of Sec. 2.1 / App. B, padded as in Lemma 2:
 *   gate_type  [n_gates][3] = {code, q0, q1}: q0 = control or first qubit
 *              (-1 for single-qubit gates), q1 = target or second qubit;
 *   gate_param [n_gates][3] = {theta, phi, lambda}; single-parameter gates
 *              (RX, RY, RZ, CP) read theta only; unused entries are ignored;
 *   param_idx  [n_gates] trainable-parameter slot of the gate's theta, or -1;
 *              may be NULL (no trainable parameters).  Only RX, RY, RZ and CP
 *              may carry a slot. */
typedef struct {
    int32_t n_qubits;
    int32_t n_gates;
    const int32_t *gate_type;
    const double *gate_param;
    const int32_t *param_idx;
} qg_circuit;

/* Create a state of n_qubits qubits set to |0...0> (App. A, eq. (hilbert)).
 * dev_buf: NULL -> the library allocates (and later frees) 2^n amplitudes;
 * otherwise a caller-owned device buffer of at least buf_bytes >= 2^n * size
 * of an amplitude, borrowed for the handle's lifetime and never freed.
 * hip_stream: the hipStream_t (NULL = default stream) all work on this state
 * is enqueued on.  Limits: 1 <= n <= 33 (QG_C128) or 34 (QG_C64).
 * Errors: QG_EINVAL (n out of range, buffer too small, out NULL), QG_ENOMEM. */
qg_status qg_state_alloc(int n_qubits, qg_dtype dtype, void *dev_buf, size_t buf_bytes,
                         void *hip_stream, qg_state **out);

/* Release a handle (and the buffer, if the library allocated it).  Waits for
 * the state's stream.  NULL is accepted. */
qg_status qg_state_free(qg_state *s);

/* Reset the state to |0...0>. */
qg_status qg_state_reset(qg_state *s);

/* Re-bind the stream later calls on this state are enqueued on. */
qg_status qg_state_set_stream(qg_state *s, void *hip_stream);

/* Device pointer of the amplitudes, qubit count and dtype of a state. */
qg_status qg_state_info(const qg_state *s, void **dev_ptr, int *n_qubits, qg_dtype *dtype);

/* Apply the circuit's gates, in order, to the state (App. A: each gate is the
 * Kronecker-product operator of eq. (tp) / eq. (cx) / eq. (cr1) applied to the
 * whole vector).  The circuit must have the state's qubit count.
 * fusion_mode: a qg_fusion value.  Results agree with gate-by-gate
 * application up to floating-point rounding for every mode.
 * Errors: QG_EINVAL (qubit out of range, q0 == q1 on a two-qubit gate, unknown
 * code, non-finite parameter, n mismatch), QG_ENOMEM, QG_EDEVICE. */
qg_status qg_apply_circuit(qg_state *s, const qg_circuit *c, int fusion_mode);

/* Reset the state to |0...0> and apply the circuit (the paper's circuits all
 * start from |0...0>): the same result as qg_state_reset followed by
 * qg_apply_circuit, bit for bit.  Because the library wrote |0...0> itself, it
 * knows which amplitudes are still zero when each pass starts: a pass mixes
 * amplitudes only within its tiles, so an amplitude with a 1 on a qubit that no
 * earlier pass held in its tile is zero, and each tile pass visits only the
 * tiles that can hold a nonzero amplitude (up to the first pass that runs on
 * another kernel, after which every pass visits all of its tiles).  Arguments
 * and errors as for qg_apply_circuit. */
qg_status qg_apply_from_zero(qg_state *s, const qg_circuit *c, int fusion_mode);

/* Probabilities p_i = |alpha_i|^2 (eq. (hilbert)), computed in FP64 for both
 * dtypes.  idx == NULL: all 2^n values into out[2^n]; otherwise n_idx host
 * indices (each < 2^n) and out[n_idx].  out is a device pointer. */
qg_status qg_probs(qg_state *s, const uint64_t *idx, int64_t n_idx, double *out);

/* Draw `shots` samples of the basis-state index from p (the paper's "shots",
 * Sec. 3 / Table 1).  Shot k uses the uniform u_k = (x >> 11) 2^-53 of the
 * Philox4x32-10 block x = out1:out0 with key (seed lo, seed hi) and counter
 * (k lo, k hi, 0, 0), and returns the smallest index i whose cumulative
 * probability exceeds u_k * sum(p) (the GPU groups the cumulative sums in a
 * 64-ary tree, so an r within rounding of a boundary may pick the neighbour).
 * out_idx: device array of `shots` uint64, in shot order.  shots >= 0. */
qg_status qg_sample(qg_state *s, int64_t shots, uint64_t seed, uint64_t *out_idx);

/* Pauli-Z-string expectations <Z_m> = sum_i p_i (-1)^{popcount(i & zmask[m])}
 * for n_terms host masks (each < 2^n), accumulated in FP64.  Not an operation
 * of the paper, which reports shot counts only: it is the observable of the
 * workloads this library serves (sums of Z_i Z_j terms), evaluated from the
 * probabilities p_i = |alpha_i|^2 of App. A's state vector.  One read of the
 * state serves up to 64 masks.  out_terms: device
 * [n_terms] or NULL; out_sum: device scalar sum_m coeff[m] <Z_m> or NULL
 * (coeff may be NULL only when out_sum is NULL).  n_terms >= 0. */
qg_status qg_expval(qg_state *s, const uint64_t *zmask, const double *coeff, int n_terms,
                    double *out_terms, double *out_sum);

/* qg_expval without any allocation, for callers that cannot allocate memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as qg_expval, with these
 * differences:
 *  - n_terms <= 256; more is QG_EINVAL (nothing is launched);
 *  - masks and coefficients (host arrays, read before the call returns) reach
 *    the device as kernel arguments; every partial sum lives in one static
 *    device array of the library, about 2 MiB, held on each device that uses
 *    it until the process ends; the call allocates no device or pinned host
 *    memory and clears nothing with hipMemsetAsync;
 *  - that array is shared by every call on the device and keeps the last
 *    call's contents: calls that overlap on one device (concurrent streams,
 *    threads) race and must be ordered by the caller;
 *  - the state's device must be the current device. */
qg_status qg_expval_noalloc(qg_state *s, const uint64_t *zmask, const double *coeff, int n_terms,
                            double *out_terms, double *out_sum);

/* Value and gradient of f = sum_m coeff[m] <Z_{zmask[m]}> for the circuit applied
 * to |0...0>, by one adjoint reverse sweep (Jones & Gacon 2020; the paper's
 * adjoint GPU modes, Sec. 2): for each gate with param_idx >= 0, RX/RY/RZ add
 * Im<lambda|P|psi> and CP adds -2 Im<lambda|P11|psi> to grad[param_idx].
 * The library allocates the two working states and releases them before
 * returning.  out_value: device scalar; out_grad: device [n_params].
 * Errors: QG_EINVAL (also for a slot >= n_params or on a gate that is not RX,
 * RY, RZ or CP), QG_ENOMEM (two states do not fit). */
qg_status qg_adjoint_grad(const qg_circuit *c, qg_dtype dtype, const uint64_t *zmask,
                          const double *coeff, int n_terms, int n_params, void *hip_stream,
                          double *out_value, double *out_grad);

/* Batched form (the paper's parallel / multi-circuit mode, Sec. 2.4): n_circ
 * independent circuits of possibly different qubit counts (1..22), each from
 * |0...0>; out[c] = sum_{i<n_c-1} <Z_i Z_{i+1}> of circuit c (obs_kind
 * QG_OBS_ZZ_CHAIN), or sum over its CSR terms k in [obs_off[c], obs_off[c+1])
 * of coeff[k] <Z_{zmask[k]}> (QG_OBS_CSR; host arrays, obs_off has n_circ + 1
 * entries starting at 0).  Circuits whose state fits one tile (2^12 amplitudes
 * in complex128, 2^13 in complex64) run in one persistent launch and never
 * touch device memory; larger ones keep their states in device memory (at
 * most batch_group_mib MiB or half the free memory at a time, in groups) and
 * run pass by pass, one launch per pass index for all circuits of a group.
 * out: device
 * [n_circ] (written when the launch runs; each value is a fixed-order sum, the
 * same on every launch). */
typedef enum { QG_OBS_ZZ_CHAIN = 0, QG_OBS_CSR = 1 } qg_obs_kind;

/* One-shot: plan, upload, launch, release (the release waits for the stream). */
qg_status qg_batch_expval(const qg_circuit *circs, int n_circ, qg_dtype dtype, int obs_kind,
                          const int64_t *obs_off, const uint64_t *zmask, const double *coeff,
                          void *hip_stream, double *out);

/* Reusable batch: qg_batch_create plans and uploads every circuit, allocates
 * the device states of its multi-tile circuits and, when hip_stream is not the
 * NULL stream, captures the launches into a HIP graph; qg_batch_launch replays
 * it (or launches directly) on that stream.  qg_batch_set_params uploads new
 * angles for circuits with the same gate structure (codes and qubits;
 * QG_EINVAL otherwise), enqueued on the stream before the next launch.
 * qg_batch_free waits for the stream. */
typedef struct qg_batch qg_batch;
qg_status qg_batch_create(const qg_circuit *circs, int n_circ, qg_dtype dtype, int obs_kind,
                          const int64_t *obs_off, const uint64_t *zmask, const double *coeff,
                          void *hip_stream, double *out, qg_batch **handle);
qg_status qg_batch_set_params(qg_batch *b, const qg_circuit *circs);
qg_status qg_batch_launch(qg_batch *b);
qg_status qg_batch_free(qg_batch *b);

/* Plan inspection (host only, no device needed): the pass each gate of the
 * circuit is executed in under fusion_mode, written to pass_of_gate[n_gates]
 * (host, may be NULL), and the pass count to *n_passes.  Passes run in
 * increasing order and cover every gate exactly once; two gates that share a
 * qubit run in circuit order. */
qg_status qg_plan_passes(const qg_circuit *c, qg_dtype dtype, int fusion_mode,
                         int32_t *pass_of_gate, int32_t *n_passes);

/* Kernel family that runs each pass of qg_apply_circuit's plan (host only, no
 * device needed): kernel_of_pass[min(capacity, passes)] (host, may be NULL)
 * gets one qg_kernel code per pass, in execution order, and *n_passes the pass
 * count.  The choice follows the current tuning keys (lane_swap, lane_gate,
 * dense_min_gates). */
typedef enum {
    QG_KERNEL_TILE = 0,       /* tile pass: gates applied in registers, layouts exchanged through LDS */
    QG_KERNEL_DENSE = 1,      /* dense k-qubit block (fused unitary) */
    QG_KERNEL_SWAP_HALF = 2,  /* SWAP of two qubits above the cache-line bits: half the state moves */
    QG_KERNEL_SWAP_LANE = 3,  /* SWAP with its lower qubit inside a cache line: cross-lane exchange */
    QG_KERNEL_LANE_GATE = 4   /* one-qubit gate or CX with its target inside a cache line */
} qg_kernel;
qg_status qg_plan_kernels(const qg_circuit *c, qg_dtype dtype, int fusion_mode,
                          int32_t *kernel_of_pass, int32_t capacity, int32_t *n_passes);

/* HBM bytes a plan moves (host only, no device needed): *n_passes gets its pass
 * count and *hbm_bytes the bytes its passes read and write in device memory,
 * each pass counted as one read and one write of every tile it visits (the half
 * state of a SWAP or CX permutation pass, the tiles a pass conditioned on a
 * qubit outside its tile skips excluded).  form:
 *   QG_FORM_APPLY    qg_apply_circuit with fusion_mode;
 *   QG_FORM_FROM_ZERO qg_apply_from_zero with fusion_mode: the reset's write of
 *                    the state, then the passes over the tiles they visit;
 *   QG_FORM_ADJOINT  qg_adjoint_grad: the greedy forward sweep (from the zeroed
 *                    state, so its first passes skip the tiles still zero), the
 *                    observable (read psi twice, write lambda) and the reverse
 *                    sweep over both states (fusion_mode ignored);
 *   QG_FORM_BATCHED  one circuit of qg_batch_expval (fusion_mode ignored): 0 for
 *                    a circuit whose state fits one tile (registers and LDS
 *                    only), else its state in device memory streamed once per
 *                    pass (the first pass writes it without reading it, unless
 *                    the pass skips tiles and the state is filled first) and
 *                    read once by the observable (n_qubits <= 22).
 * Either output may be NULL.  Errors: QG_EINVAL for an invalid circuit, dtype,
 * form or fusion mode. */
typedef enum { QG_FORM_APPLY = 0, QG_FORM_ADJOINT = 1, QG_FORM_BATCHED = 2, QG_FORM_FROM_ZERO = 3 } qg_form;
qg_status qg_plan_bytes(const qg_circuit *c, qg_dtype dtype, int form, int fusion_mode, int32_t *n_passes,
                        double *hbm_bytes);

/* ---- Learned fusion: the cost model (not in the paper; its backend fixes the
 * fusion width at 5, App. D.2).  An MLP with three ReLU hidden layers of width
 * 64 and a linear scalar output, FP32, run by the library's own forward,
 * backward and Adam kernels.  Flat parameter layout: W1[n_in][64], b1[64],
 * W2[64][64], b2[64], W3[64][64], b3[64], W4[64], b4.  x, t, y, grad and
 * theta are host arrays; calls on a model are synchronous on its stream. */
typedef struct qg_mlp qg_mlp;
/* New model: He-uniform weights from SplitMix64(seed), zero biases.
 * hidden must be 64 (QG_EUNSUPPORTED otherwise); 1 <= n_in <= 256. */
qg_status qg_mlp_create(int n_in, int hidden, uint64_t seed, void *hip_stream, qg_mlp **out);
qg_status qg_mlp_n_params(const qg_mlp *m, int64_t *n);
/* Replace the parameters (and reset Adam's moments and step). */
qg_status qg_mlp_set_params(qg_mlp *m, const float *theta);
qg_status qg_mlp_get_params(qg_mlp *m, float *theta);
/* y[B] for x[B][n_in]. */
qg_status qg_mlp_forward(qg_mlp *m, const float *x, int B, float *y);
/* Mean-squared-error loss of the batch and its gradient grad[n_params]. */
qg_status qg_mlp_grad(qg_mlp *m, const float *x, const float *t, int B, double *loss, float *grad);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with the given gradient. */
qg_status qg_mlp_adam_step(qg_mlp *m, const float *grad, float lr);
/* Minibatch Adam on N samples for `epochs` epochs (a SplitMix64(seed)
 * Fisher-Yates shuffle per epoch, full batches only); loss_per_epoch[epochs]
 * (host, may be NULL) receives the mean batch loss of each epoch. */
qg_status qg_mlp_train(qg_mlp *m, const float *x, const float *t, int N, int epochs, int batch, float lr,
                       uint64_t seed, double *loss_per_epoch);
qg_status qg_mlp_free(qg_mlp *m);

/* Number of features of a candidate pass, and the candidate strategies:
 * config k < QG_PASS_DENSE is a tile pass allowing 4 + k required qubits
 * outside the low block (k = 1 is the greedy default, width 5); config
 * QG_PASS_DENSE is a dense block on the matrix cores. */
#define QG_PASS_FEATURES 24
#define QG_PASS_CONFIGS 5
#define QG_PASS_DENSE 4
/* Features of the whole circuit run as one pass under candidate config k
 * (features[QG_PASS_FEATURES], host); *n_passes (may be NULL) receives the
 * number of passes the greedy rule of that config would form (1 for the
 * dense strategy, which needs n >= 8 and at most 6 touched qubits). */
qg_status qg_pass_features(const qg_circuit *c, qg_dtype dtype, int config, float *features, int32_t *n_passes);
/* Installs the model QG_FUSE_LEARNED plans with (NULL: greedy fallback).  The
 * learned planner prices candidate passes (each start gate, each strategy)
 * with one batched forward of the model, predicting ln(pass time in
 * microseconds), and keeps the partition of least predicted total time (dynamic
 * programming); plans are cached per circuit structure.  The model must have
 * QG_PASS_FEATURES inputs and stay alive while installed. */
qg_status qg_set_cost_model(qg_mlp *m);

/* Process-wide planner tuning (not part of the paper's method; performance only,
 * results are identical up to rounding for every setting).  Keys:
 *   dense_min_gates                  a run of gates touching <= 6 qubits with at least
 *                                    this many gates runs as one dense MFMA block;
 *                                    0 (default): the break-even measured on MI355X
 *                                    per precision and block width (24 / 20 / 28 gates
 *                                    for 4 / 5 / 6 qubits in complex128, 16 / 16 / 24
 *                                    in complex64); 1 << 30: never
 *   batch_group_mib                  batched form: at most this many MiB of multi-tile
 *                                    circuit states at a time (and at most half the
 *                                    free device memory; default 32768)
 *   adjoint_tile_bits / adjoint_low_bits
 *                                    qg_adjoint_grad's reverse sweep in complex128: tile
 *                                    qubits (8..11, default 10) and low block (3..8,
 *                                    default 5); two states of 8 amplitudes per thread
 *   dense_tile_bits                  tile of a dense block: its k qubits and the
 *                                    (dense_tile_bits - k) lowest other qubits (10..13,
 *                                    default 11)
 *   tile_bits_c128 / tile_bits_c64   qubits per tile (amplitudes streamed per workgroup)
 *   reg_bits_c128 / reg_bits_c64     amplitudes per thread = 2^reg_bits
 *   low_bits_c128 / low_bits_c64     lowest qubits kept in every fused tile
 *   max_high_c128 / max_high_c64     fusion width: targets >= low_bits per pass
 *   nt                               non-temporal state loads/stores: 0 off, 1 when every
 *                                    wavefront access covers whole cache lines, 2 always
 *   swz_bits                         tile-order swizzle of the launch
 *   cls<k>_<tile|reg|swz>_<dt>       shape of pass class k (see qg_autotune)
 *   tgt<q>_<tile|reg|swz|xcd>_<dt>   shape of single-gate passes on target q (tile 0:
 *                                    use the class; see qg_autotune)
 *   xcd                              1: each of the 8 XCDs streams a contiguous eighth
 *                                    of a pass's tiles (blocks are dealt to XCDs in
 *                                    turn); 0: block b takes tile b
 *   pipe                             forward passes on persistent blocks that load
 *                                    their next tile while computing the current one:
 *                                    0 never, 1 passes with several register layouts
 *                                    or at least pipe_min_ops ops, 2 always
 *   pipe_min_ops                     see pipe
 *   diag_run_min                     runs of at least this many consecutive diagonal
 *                                    gates in a register layout become one factor per
 *                                    amplitude (0: never)
 *   lane_swap                        1: a standalone SWAP whose lower qubit lies inside
 *                                    a cache line runs as a cross-lane exchange kernel
 *   lane_gate                        1: a single one-qubit gate or CX whose target lies
 *                                    inside a cache line runs as a cross-lane exchange
 *   half_lds_c128, half_lds_c64      1 / 0: multi-phase passes move the tile between
 *                                    layouts through LDS as real parts, then imaginary
 *                                    parts (half the LDS per workgroup); the batched
 *                                    form always does so
 * Errors: QG_EINVAL for an unknown key or a value out of range.  Not
 * thread-safe against concurrent planning. */
qg_status qg_set_tuning(const char *key, int64_t value);
qg_status qg_get_tuning(const char *key, int64_t *value);

/* Autotuner (a measured search; not part of the paper).  Passes are classed by
 * the highest qubit they need in registers: 0 below the cache-line bits, 1 below
 * 12, 2 below 20, 3 from 20 up, 4 none (diagonal only).  For each class that the
 * state's qubit count can exercise, single-gate passes on up to three of the
 * class's targets are timed (HIP events, median of reps after one warm-up run,
 * summed over the targets) on the state for 8 candidate (tile bits, register
 * bits, swizzle) shapes; the fastest becomes the class's
 * entry for the state's dtype (tuning keys cls<k>_tile_<dt>, cls<k>_reg_<dt>,
 * cls<k>_swz_<dt>; fused passes use the class's swizzle).  The state's
 * amplitudes are overwritten and reset to |0...0> at the end; the call waits
 * for the state's stream.  table: host int32[5][3] (tile, reg, swz) or NULL.
 * Then, per target qubit, single-gate U3 passes are timed for 6 (tile bits,
 * register bits, swizzle, XCD order) candidates and the fastest becomes that
 * target's entry (tuning keys tgt<q>_tile_<dt>, tgt<q>_reg_<dt>,
 * tgt<q>_swz_<dt>, tgt<q>_xcd_<dt>; tile 0 means "use the class"), used by
 * single-gate passes of one-qubit mixing gates.  Targets whose single gates run
 * on the lane kernel (lane_gate) are not timed and keep tile 0. */
qg_status qg_autotune(qg_state *s, int reps, int32_t *table);

/* Message describing the calling thread's last failed call ("" if none). */
const char *qg_last_error(void);

/* Library version string. */
const char *qg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QGEAR_MI355X_QG_H_ */
