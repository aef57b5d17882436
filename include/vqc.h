/*
 * vqc.h -- C ABI of the MI355X (gfx950) variational-quantum-circuit hot path.
 *
 * The method is the state-vector simulator with memory-efficient reverse-mode
 * gradients of Liao et al., "JuliVQC: an Efficient Variational Quantum Circuit
 * Simulator for Near-Term Quantum Algorithms" (arXiv:2406.19212):
 * gate application (Sec. 3.1, Eqs. (3) and (twoqubitgate), Alg. 1), channels
 * as superoperators on the vectorised density matrix (Sec. 3.4,
 * Eq. (channel2)), Pauli-sum expectation values (Sec. 2.5) and the adjoint
 * gradient sweep (Sec. 3.3, Alg. 2; Sec. 3.5).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Qubits are 0-based.  Qubit k is bit k of the amplitude index: the paper's
 *   column-major storage with the first qubit fastest (Sec. 2.1).
 * - Amplitudes are complex128, interleaved (re, im), 16 bytes each; the layout
 *   of vqc_c128, std::complex<double> and torch.complex128.
 * - A pure n-qubit state holds 2^n amplitudes.  A mixed state is the
 *   vectorised density matrix (Sec. 3.4) with 4^n entries:
 *   v[x + 2^n y] = rho[x][y]; ket bits 0..n-1, bra bits n..2n-1 (Sec. 2.1).
 * - Gate and Kraus matrices follow the paper's QuantumGate convention
 *   (Sec. 2.2): column-major storage of the 2^m x 2^m matrix, element
 *   (out, in) at data[out + 2^m * in]; the local index of an m-qubit op is
 *   l = sum_t b_{qubits[t]} 2^t (first listed qubit = least significant).
 *   vqc_mat_from_external converts a textbook row-major matrix.
 * - Device buffers are caller-owned (e.g. torch tensors) and must stay alive
 *   while work that uses them is queued.  Host arrays passed in are copied
 *   before the call returns.
 * - Work is queued on the HIP stream bound to the state or batch and runs
 *   asynchronously; only calls with host outputs synchronise that stream.
 * - Every call returns vqc_status (0 = VQC_OK, negative = error) and never
 *   aborts.  Arguments are validated on the host before any launch; a call
 *   that returns an error has queued no work and left every buffer unchanged.
 * - Handles are not thread-safe; use one handle per stream.
 */
#ifndef VQC_ABI_INCLUDED
#define VQC_ABI_INCLUDED

#ifndef __HIPCC_RTC__
#include <stddef.h>
#include <stdint.h>
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VQC_OK = 0,
  VQC_ERR_ARG = -1,           /* null pointer, bad size or count */
  VQC_ERR_QUBIT = -2,         /* qubit out of range or repeated */
  VQC_ERR_UNSUPPORTED = -3,   /* op arity or combination not supported */
  VQC_ERR_KIND = -4,          /* pure/mixed mismatch */
  VQC_ERR_NOT_CPTP = -5,      /* Kraus set fails sum K^dagger K = I to 1e-12 */
  VQC_ERR_NONFINITE = -6,     /* NaN or Inf in a host-side input */
  VQC_ERR_OOM = -7,           /* device allocation failed */
  VQC_ERR_HIP = -8,           /* HIP runtime error */
  VQC_ERR_NOT_HERMITIAN = -9, /* gradient asked for a complex-coefficient H */
  VQC_ERR_NOT_UNITARY = -10,  /* backward through a non-unitary gate matrix */
  VQC_ERR_ILL_CONDITIONED = -11, /* a channel's inverse exceeds the condition bound */
  VQC_ERR_SCRATCH_LIMIT = -12,  /* input larger than the allocation-free call's fixed scratch */
  VQC_ERR_IN_USE = -13          /* circuit bound to a live batch (destroy, autotune) */
} vqc_status;

typedef enum { VQC_PURE = 0, VQC_MIXED = 1 } vqc_kind;

typedef struct { double re, im; } vqc_c128;

typedef struct vqc_state_s *vqc_state;     /* view of a caller-owned buffer */
typedef struct vqc_circuit_s *vqc_circuit; /* planned op table + device tables */
typedef struct vqc_batch_s *vqc_batch;     /* many circuits/parameter sets */

/* Op types (Sec. 2.2).  Rotations are exp(-i theta P / 2); Ry = [[c,-s],[s,c]];
 * sqrt(G) = ((1+i) I + (1-i) G)/2 for G in {X, Y, W}, W = (X+Y)/sqrt(2).
 * Two-qubit gates use the local index b_{q0} + 2 b_{q1}: CNOT/CONTROL/CR* have
 * the control on qubits[0] and the target on qubits[1]; FSIM takes
 * (theta, phi, Delta+, Delta-, Delta-off) as printed in Sec. 2.2. */
enum {
  VQC_X = 1, VQC_Y, VQC_Z, VQC_H, VQC_S, VQC_T, VQC_SX, VQC_SY, VQC_SW,
  VQC_RX, VQC_RY, VQC_RZ, VQC_ID,
  VQC_CZ = 20, VQC_CNOT, VQC_SWAP, VQC_ISWAP, VQC_FSIM, VQC_CRX, VQC_CRY, VQC_CRZ,
  VQC_CONTROL, /* CONTROLGate(i, j, U): data = 2x2 target matrix */
  VQC_MATRIX,  /* QuantumGate(positions, data): data = 2^m x 2^m, m <= 3 */
  /* three-qubit gates (Sec. 2.2), local index b_{q0} + 2 b_{q1} + 4 b_{q2}:
   * TOFFOLI flips qubits[2] when qubits[0] and qubits[1] are 1; FREDKIN swaps
   * qubits[1] and qubits[2] when qubits[0] is 1; CCONTROL is
   * CONTROLCONTROLGate(i, j, k, U): the 2x2 data U on qubits[2] when
   * qubits[0] and qubits[1] are 1.  In circuits they are expanded into exact
   * one- and two-qubit sequences: Toffoli as six CNOTs with H, T and T^dagger
   * (Nielsen and Chuang, Fig. 4.9), Fredkin as CNOT . Toffoli . CNOT, CCONTROL
   * as CV, CNOT, CV^dagger, CNOT, CV with V the principal square root of U
   * (Barenco et al. 1995, Lemma 6.1). */
  VQC_TOFFOLI, VQC_FREDKIN, VQC_CCONTROL,
  /* channels (Sec. 2.2); params[0] = gamma or p.  Depolarizing uses
   * K0 = sqrt(1-3p/4) I, K1..3 = sqrt(p/4) sigma (trace preserving);
   * DEPOLARIZING2 uses K0 = sqrt(1-15p/16) I, K_ab = sqrt(p/16) sigma_a(x)sigma_b. */
  VQC_AMPLITUDE_DAMPING = 40, VQC_PHASE_DAMPING, VQC_DEPOLARIZING, VQC_DEPOLARIZING2,
  VQC_KRAUS    /* QuantumMap(positions, kraus): data = n_kraus blocks of 2^m x 2^m */
};

/* One op of a circuit (Sec. 2.3).  param_index[k] >= 0 marks parameter k as
 * variational (the paper's isparas) and names its slot in the flat theta
 * vector (active_parameters order is the caller's choice of indices); -1
 * means params[k] is used as a fixed value.  Channels take no variational
 * parameters (Sec. 2.2). */
typedef struct {
  int type;
  int n_qubits;           /* 1, 2, or 3 */
  int qubits[4];
  double params[5];
  int param_index[5];
  int n_data;             /* complex entries at data (0 if none) */
  const vqc_c128 *data;   /* host memory, column-major blocks */
} vqc_op;

/* H = sum_t (coeff_re[t] + i coeff_im[t]) P_t with P_t|x> = i^{|Y|}
 * (-1)^{popcount(x & z_mask)} |x ^ x_mask>: X on bit k sets x_mask bit k,
 * Z sets z_mask bit k, Y sets both (Sec. 2.5).  Host arrays; coeff_im may be
 * NULL (all zero). */
typedef struct {
  int n_terms;
  const uint64_t *x_mask;
  const uint64_t *z_mask;
  const double *coeff_re;
  const double *coeff_im;
} vqc_pauli_sum;

/* Fusion and launch shape (chosen by vqc_circuit_autotune or by hand).
 * tile_bits: qubits per LDS tile (K); low_bits: contiguous low qubits every
 * tile includes (c); reg_bits: qubits held per thread (R, 3 or 4);
 * grid_blocks: persistent grid size (0 = one block per tile).  Zero fields
 * take the library default.
 * remap: passes may move qubits into the contiguous low block for the next
 * pass (the state ends in the standard layout; the circuit then holds a
 * second state buffer of the same size, two for the gradient plan, and a
 * batch one or two per item): 1 on, -1 off, 0 default (on from 12 qubits,
 * pure states; the gradient plan moves qubits up to 30 qubits).
 * jit: the forward and adjoint passes of a pure-state circuit run as kernels
 * compiled at circuit creation for this circuit's op sequence (hipRTC; the fused-pass
 * driver with every op's kind and register bits fixed at compile time, the
 * parameters still read from device memory, so one compile serves every
 * theta; code objects are cached on disk): 1 on (creation fails with
 * VQC_ERR_HIP if the compile fails), -1 off, 0 default (on from 20 qubits
 * with tiles of at most 11 qubits, silently off if the compile fails).  The
 * environment variable VQC_JIT=0 (or 1) turns them off (on) for every
 * eligible circuit.  Read at circuit creation, each 0/1: VQC_JIT_FWD_SPLIT
 * (forward tiles exchanged through LDS as real and imaginary halves; default
 * 1), VQC_JIT_HSQRT (phase-factored sqrt(X), sqrt(Y), sqrt(W) applied times
 * sqrt(2), the tile rescaled once per pass; default 1), VQC_JIT_RECFREE (ops
 * without a parameter record skip the program-entry chain; default 1),
 * VQC_JIT_ADJ_SPLIT (adjoint driver: 1, the default, reads lane slots from
 * the planner's table and moves the tile through LDS as real and imaginary
 * halves; 2 the same with whole amplitudes; 0 the older driver, where
 * VQC_JIT_ADJ_SHARED (Phi and Psi share one LDS tile; default 1) and
 * VQC_JIT_ADJ_SWZ (a searched swizzle instead of the fixed fold; default 0)
 * apply).  VQC_JIT_CACHE names the code-object cache directory. */
typedef struct {
  int tile_bits;
  int low_bits;
  int reg_bits;
  int grid_blocks;
  int remap;
  int jit;
} vqc_tune;

typedef struct {
  int n_ops;
  int n_elementary;   /* ops after lowering (mixed: ket/bra halves, superops) */
  int n_passes;       /* HBM passes of the forward plan */
  int n_stages;       /* register stages over all passes */
  int n_var;          /* derivative slots (variational parameters used) */
  int n_params;
  vqc_tune tune;
  double alg_bytes_per_amp; /* algorithmic HBM bytes per amplitude, unfused ops */
  int n_adj_passes;   /* HBM passes of the adjoint (gradient) plan */
  int n_fwd_moves;    /* forward passes that move qubits (run out of place) */
  int n_adj_moves;    /* adjoint passes that move qubits */
  int n_jit_passes;   /* forward passes running as circuit-specialised kernels */
  int jit_cached;     /* 1: their code object came from the on-disk cache */
  double jit_ms;      /* compile (or cache load) and module load time */
  int n_jit_adj_passes; /* adjoint (gradient) passes running as specialised kernels */
} vqc_circuit_stats;

/* ------------------------------------------------------------------ misc */
const char *vqc_status_string(int status);
int vqc_version(void);

/* Convert a textbook row-major 2^m x 2^m matrix whose qubits[0] is the MOST
 * significant bit of the row/column index into this library's column-major
 * matrix with qubits[0] as the least significant bit (the paper's
 * n_qubits_mat_from_external, Sec. 2.2).  m in 1..4; host arrays. */
vqc_status vqc_mat_from_external(int m, const vqc_c128 *row_major, vqc_c128 *out_col_major);

/* ---------------------------------------------------------------- states */

/* StateVector(n) / DensityMatrix(n) of Sec. 2.1.  dev_buf: caller-owned
 * device buffer of 2^n (PURE) or 4^n (MIXED) complex128.  host_init: NULL
 * writes |0..0> (resp. |0..0><0..0|), otherwise 2^n or 4^n host amplitudes
 * that are copied in.  stream: hipStream_t (NULL = default stream).
 * n_qubits: 1..33 (PURE), 1..16 (MIXED).  The handle does not own dev_buf. */
vqc_status vqc_state_init(vqc_state *out, vqc_kind kind, int n_qubits, void *dev_buf,
                          const vqc_c128 *host_init, void *stream);
/* Rewrite |0..0> (resp. |0..0><0..0|) into the state's buffer (async). */
vqc_status vqc_state_reset(vqc_state s);
/* Rebind a state handle to another buffer/stream without touching data. */
vqc_status vqc_state_rebind(vqc_state s, void *dev_buf, void *stream);
vqc_status vqc_state_destroy(vqc_state s);

/* Apply one m-qubit gate matrix (m = 1, 2, 3), Eqs. (3) / (twoqubitgate) and
 * Alg. 1 for m = 3 (one dense 8x8 product per group of eight amplitudes).
 * On a mixed state the gate acts as rho -> U rho U^dagger (Sec. 3.5: a gate
 * is a one-Kraus channel).  Diagonal and controlled matrices (m <= 2) are
 * detected and take the kernels that touch only the amplitudes that change.
 * m = 3 synchronises the stream (the matrix is copied from host memory). */
vqc_status vqc_apply_gate(vqc_state s, int m, const int *qubits, const vqc_c128 *matrix);

/* Apply one typed op (Sec. 2.2 predefined gates, parametric gates with the
 * values in op->params, or a channel on a mixed state).  Structured gates
 * (diagonal, CZ, CNOT, fSim) use dedicated kernels. */
vqc_status vqc_apply_op(vqc_state s, const vqc_op *op);

/* QuantumMap(positions, kraus) on a MIXED state (Sec. 2.2, Eq. (channel));
 * applied as the superoperator sum_s conj(K_s) (x) K_s on bits
 * (qubits, qubits + n) of vec(rho) (Eq. (channel2)).  m = 1, 2, 3; kraus:
 * n_kraus (1..64) column-major 2^m x 2^m blocks, qubits[0] = bit 0 of their
 * index, complete to 1e-12 (else VQC_ERR_NOT_CPTP).  m = 3 applies
 * sum_s K_s rho K_s^dagger term by term on each 8 x 8 block of rho and
 * synchronises the stream.  In circuits a three-qubit channel runs as an HBM
 * pass of its own (the same block kernel; the adjoint sweep applies the
 * adjoint Kraus set K_s^dagger to Psi and, in the inverse form, the inverse
 * of its 64 x 64 superoperator, computed on the host at circuit creation, to
 * Phi); batches refuse such circuits (VQC_ERR_UNSUPPORTED). */
vqc_status vqc_apply_channel(vqc_state s, int m, const int *qubits, int n_kraus,
                             const vqc_c128 *kraus);

/* expectation(op, state) of Sec. 2.5: <psi|H|psi> (PURE) or Tr(H rho) (MIXED),
 * written to *out_host (synchronises the stream).  Deterministic FP64 two-stage
 * reduction. */
vqc_status vqc_expectation(vqc_state s, const vqc_pauli_sum *H, vqc_c128 *out_host);

/* vqc_expectation for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same result, with every intermediate (first-stage
 * partial sums, the Pauli terms, the job record, the result) in one fixed
 * device array of the library, 1 MiB + 33 KiB, that each GPU holds until the
 * process ends.  No device or host heap allocation happens on this path; the
 * first call on a GPU looks up that GPU's copy of the array.  Limits: at most
 * 1024 terms and 2^28 summed amplitudes (PURE n <= 28; every MIXED size), else
 * VQC_ERR_SCRATCH_LIMIT with nothing queued.  Every call on one GPU shares the
 * array: calls that overlap on one GPU (several streams or host threads) race
 * and must be serialised by the caller.  Nothing in the array needs to start
 * at zero (every partial sum is written before it is read).  Synchronises the
 * state's stream; other errors as in vqc_expectation. */
vqc_status vqc_expectation_noalloc(vqc_state s, const vqc_pauli_sum *H, vqc_c128 *out_host);

/* sum |psi_x|^2 (PURE) or Tr(rho) (MIXED) into *out_host (synchronises). */
vqc_status vqc_norm(vqc_state s, double *out_host);

/* Read `count` amplitudes psi[idx[i]] (PURE) into out_host (synchronises).
 * idx_host: host int64 indices in [0, 2^n). */
vqc_status vqc_gather(vqc_state s, int count, const int64_t *idx_host, vqc_c128 *out_host);

/* measure!(state, i) of Sec. 2.4: measure qubit `qubit` (0-based) of a PURE or
 * MIXED state and collapse it in place.  The probability masses s0, s1 of
 * the qubit's two values are summed on the device (|psi_x|^2, resp. the
 * diagonal of rho, over basis states x); outcome_out = 0 when u < s0/(s0+s1),
 * else 1, with u a caller-supplied uniform number in [0,1); prob_out = the
 * outcome's exact probability s_o/(s0+s1).  The state becomes P psi / sqrt(s_o)
 * (PURE) or P rho P / s_o (MIXED), P the projector on the outcome, so it has
 * unit norm (resp. trace) afterwards.  Synchronises the stream once.  Errors:
 * VQC_ERR_QUBIT, VQC_ERR_ARG (u outside [0,1), a state of zero norm: then
 * the state is unchanged), VQC_ERR_NONFINITE. */
vqc_status vqc_measure(vqc_state s, int qubit, double u, int *outcome_out, double *prob_out);

/* Bitstring sampling (the random-circuit sampling use of Sec. 1): for each
 * of `count` caller-supplied uniform numbers u_host[k] in [0,1), out_host[k]
 * is the first basis state x (index order) whose cumulative probability
 * C(x) = sum_{y <= x} w(y) exceeds u_k C(2^n - 1), with w = |psi_y|^2 (PURE)
 * or rho[y][y] (MIXED).  Cumulative sums are taken per block of 4096 basis
 * states and then within a block, so an outcome can differ from a plain
 * left-to-right sum only where u_k C lies within rounding of a boundary; a
 * returned x has w(x) > 0.  The samples are grouped by block on the device,
 * so each block of the state is read once however many samples fall in it.
 * The state is not changed.  count < 2^31.  Host arrays; synchronises.
 * Errors: VQC_ERR_ARG (u outside [0,1), zero norm), VQC_ERR_NONFINITE. */
vqc_status vqc_sample(vqc_state s, int count, const double *u_host, int64_t *out_host);

/* fuse_gates(circ) of Sec. 2.3, for noiseless circuits, applied until no
 * one-qubit gate sits next to a two-qubit gate on its qubit: a run of
 * one-qubit gates on a qubit is absorbed into the two-qubit gate before it on
 * that qubit (U <- g U, in order), else into the two-qubit gate after it
 * (U <- U g_last ... g_first); one-qubit gates on a qubit that no two-qubit
 * gate touches stay.  Every
 * output op is a general VQC_MATRIX gate evaluated at theta_host (host
 * double[n_params]), so the result has no variational parameters.  The
 * output holds the ops in their order of first appearance; the state it
 * produces equals the input circuit's up to rounding.  out_ops: caller array
 * of n_ops entries; out_data: caller array of 16 * n_ops complex entries that
 * the output ops' data pointers refer to; *n_out receives the op count.
 * Builds the matrices on the device (default stream; synchronises).  Errors:
 * VQC_ERR_KIND for a channel, VQC_ERR_UNSUPPORTED for ops wider than two
 * qubits, and the op validation errors of vqc_circuit_create. */
vqc_status vqc_fuse_gates(int n_qubits, int n_ops, const vqc_op *ops, int n_params,
                          const double *theta_host, vqc_op *out_ops, vqc_c128 *out_data, int *n_out);

/* ---------------------------------------------------------------- circuits */

/* Build a circuit (QCircuit, Sec. 2.3) for states of `n_qubits` and `kind`,
 * plan its fused HBM passes and upload its tables.  theta has n_params
 * entries.  tune may be NULL (defaults).  ops and their data are copied. */
vqc_status vqc_circuit_create(vqc_circuit *out, int n_qubits, vqc_kind kind, int n_ops,
                              const vqc_op *ops, int n_params, const vqc_tune *tune);
/* VQC_ERR_IN_USE (and nothing freed) while a batch created with c is alive. */
vqc_status vqc_circuit_destroy(vqc_circuit c);
vqc_status vqc_circuit_stats_get(vqc_circuit c, vqc_circuit_stats *out);

/* apply!(circ, state) of Sec. 2.4: run the whole circuit in place, as fused
 * passes.  theta_dev: device double[n_params] (may be NULL when n_params = 0). */
vqc_status vqc_apply_circuit(vqc_state s, vqc_circuit c, const double *theta_dev);

/* apply(circ, state) / circ * state of Sec. 2.4: the circuit applied to a copy
 * of src written into dst (same kind and size; src is left unchanged).  Runs
 * on dst's stream: work queued on another stream for src must be complete. */
vqc_status vqc_apply_circuit_out(vqc_state dst, const vqc_state src, vqc_circuit c, const double *theta_dev);

/* vqc_apply_circuit with a HIP event recorded on the state's stream between
 * consecutive pass launches; pass_ms_host[p] receives the duration of pass p
 * (host float[n_passes], see vqc_circuit_stats).  Synchronises the stream. */
vqc_status vqc_apply_circuit_timed(vqc_state s, vqc_circuit c, const double *theta_dev, float *pass_ms_host);

/* gradient(loss, circ) with loss = Re<psi|H|psi> (PURE, Alg. 2) or Tr(H rho)
 * (MIXED, Sec. 3.5), H with real coefficients.  s holds the final state
 * produced by vqc_apply_circuit(c, theta) from |0..0> (or from init_dev).
 * PURE: s is uncomputed in place back to the initial state (Phi <- Q^dagger
 * Phi).  MIXED: s is left unchanged; the states before each op are recomputed
 * from checkpoints of a forward re-run from init_dev (NULL = |0..0><0..0|),
 * using at most checkpoint_budget_bytes of device memory (0 = library
 * default).  grad_dev: device double[n_params], overwritten (parameters
 * shared by several ops get the sum).  energy_host: optional loss value
 * (synchronises when non-NULL). */
vqc_status vqc_backward(vqc_circuit c, const double *theta_dev, vqc_state s,
                        const vqc_pauli_sum *H, double *grad_dev, double *energy_host,
                        const void *init_dev, size_t checkpoint_budget_bytes);

/* gradient(loss, circ) by Alg. 2 in its inverse form (Sec. 3.3: Q^{-1} in
 * place of Q^dagger, which extends the sweep to channels; Sec. 3.5):
 * walking the ops backwards, Phi <- M^{-1} Phi, g += Re<<Psi| dM |Phi>>,
 * Psi <- M^dagger Psi.  Only two states are kept (no checkpoints), at the
 * price of rounding amplified by the channels' condition numbers.  s holds
 * the final state of vqc_apply_circuit(c, theta) and is uncomputed in place
 * (back to the initial state up to that rounding).  max_cond bounds the
 * 1-norm condition number ||M|| ||M^{-1}|| of every non-unitary op (a
 * channel, or a fused run of one-qubit ops holding one), computed on the
 * device; a larger one (or a singular channel) returns
 * VQC_ERR_ILL_CONDITIONED before any state is touched.  max_cond <= 0 takes
 * 1e8.  PURE circuits run vqc_backward (Q^{-1} = Q^dagger).  MIXED circuits
 * with a non-unitary gate matrix return VQC_ERR_NOT_UNITARY.  grad_dev and
 * energy_host as in vqc_backward.  Synchronises the stream once (the
 * condition check). */
vqc_status vqc_backward_inverse(vqc_circuit c, const double *theta_dev, vqc_state s,
                                const vqc_pauli_sum *H, double *grad_dev, double *energy_host,
                                double max_cond);

/* Autotuner: time candidate tunes of c on the scratch state s (its contents
 * are destroyed), then re-plan c with the fastest and write that tune to
 * *out.  This replaces the fixed aggregation sizes of Sec. 3.2 (Fig. 3) by a
 * measured choice.  target VQC_TUNE_FORWARD times vqc_apply_circuit from
 * |0..0>; VQC_TUNE_GRADIENT times vqc_apply_circuit + vqc_backward with the
 * observable H (real coefficients).  Candidates: pure states, tile bits
 * 10..11 (fewer for small n) x low-block bits 3..5 x register bits 3..4 with
 * the circuit's qubit-move setting, and the current shape with qubit moves
 * switched (from 12 qubits); density matrices: low-block bits 3..6 and qubit
 * moves on/off (tiles of 11 bits).  Circuits with specialised passes compile
 * each candidate (code objects are cached on disk).  A candidate whose plan,
 * compile or timed runs fail is not chosen; VQC_ERR_HIP if none ran (c keeps
 * its previous tune).  VQC_ERR_IN_USE while a batch holds c (its tables would
 * be replaced).  Synchronises the stream. */
enum { VQC_TUNE_FORWARD = 0, VQC_TUNE_GRADIENT = 1 };
vqc_status vqc_circuit_autotune_ex(vqc_circuit c, vqc_state s, const double *theta_dev,
                                   const vqc_pauli_sum *H, int target, vqc_tune *out);
/* vqc_circuit_autotune_ex with target VQC_TUNE_FORWARD. */
vqc_status vqc_circuit_autotune(vqc_circuit c, vqc_state s, const double *theta_dev,
                                vqc_tune *out);

/* ---------------------------------------------------------------- batches */

/* A batch of B items run together: item b applies circuits[b] (circuits may
 * repeat and may have different widths) to states_dev[b] with parameters
 * theta_dev[b].  All device pointers are bound at creation so the batch can
 * be captured as a hipGraph.  Every circuit must share one tune.  stream:
 * hipStream_t for all work. */
vqc_status vqc_batch_create(vqc_batch *out, int B, const vqc_circuit *circuits,
                            void *const *states_dev, const double *const *theta_dev,
                            void *stream);
vqc_status vqc_batch_destroy(vqc_batch b);

/* Initialise every item to |0..0> (resp. |0..0><0..0|) and run the circuits:
 * one persistent-grid launch per fused pass step for the whole batch. */
vqc_status vqc_batch_forward(vqc_batch b);

/* energies_dev[b] = loss of item b for the same H (device doubles). */
vqc_status vqc_batch_expectation(vqc_batch b, const vqc_pauli_sum *H, double *energies_dev);

/* Backward of every item after vqc_batch_forward (see vqc_backward):
 * grads_dev[b] (device double[n_params of item b]), energies_dev (optional
 * device double[B]).  Mixed items recompute from |0..0><0..0|. */
vqc_status vqc_batch_backward(vqc_batch b, const vqc_pauli_sum *H, double *const *grads_dev,
                              double *energies_dev, size_t checkpoint_budget_bytes);

/* vqc_backward_inverse for every item of a MIXED batch after
 * vqc_batch_forward: one register-pass launch per step for all items (the
 * items' inverse superoperators and the largest condition number are computed
 * first; above max_cond, or for a singular channel, VQC_ERR_ILL_CONDITIONED
 * before any state changes).  Each item's state is uncomputed in place.
 * PURE batches run vqc_batch_backward.  Synchronises once. */
vqc_status vqc_batch_backward_inverse(vqc_batch b, const vqc_pauli_sum *H, double *const *grads_dev,
                                      double *energies_dev, double max_cond);

/* Capture forward + backward (H, grads, energies as above) into a hipGraph
 * once; vqc_batch_replay launches it on the batch stream.  Capture queues no
 * work.  Replays reuse the pointers bound at creation. */
vqc_status vqc_batch_capture(vqc_batch b, const vqc_pauli_sum *H, double *const *grads_dev,
                             double *energies_dev, size_t checkpoint_budget_bytes);
vqc_status vqc_batch_replay(vqc_batch b);

/* --------------------------------------------------- surrogate network
 * A small MLP model of the variational energy landscape (not part of the
 * paper): E_hat(theta) = w3 . gelu(W2 gelu(W1 theta + b1) + b2) + b3, with
 * gelu(x) = x Phi(x) (exact erf).  Parameters and activations are FP32;
 * every matrix product rounds its FP32 inputs to BF16 (nearest-even) and
 * accumulates in FP32 on MFMA.  Parameter buffer layout (FP32, device):
 * W1[h1][n_in], b1[h1], W2[h2][h1], b2[h2], w3[h2], b3[1].  Activations are
 * row-major [batch][features]. */
typedef struct vqc_mlp_s *vqc_mlp;

/* C[M x N] = alpha op(A) op(B) + beta C, FP32 in/out, BF16 products with FP32
 * accumulation.  op(A)[m][k] = A[m*lda + k] (ta = 0) or A[k*lda + m] (ta = 1);
 * op(B)[k][n] = B[k*ldb + n] (tb = 0) or B[n*ldb + k] (tb = 1).  Device
 * pointers; stream as in vqc_state_init. */
vqc_status vqc_gemm_bf16(int M, int N, int K, const float *A, int lda, int ta, const float *B, int ldb, int tb,
                         float *C, int ldc, float alpha, float beta, void *stream);

/* Network n_in -> h1 -> h2 -> 1 for batches up to max_batch; allocates the
 * parameters (uninitialised: write them through vqc_mlp_buffers), gradient,
 * Adam moments and activation workspace. */
vqc_status vqc_mlp_create(vqc_mlp *out, int n_in, int h1, int h2, int max_batch, void *stream);
vqc_status vqc_mlp_destroy(vqc_mlp m);
/* Device pointers to the parameter and gradient buffers and their length. */
vqc_status vqc_mlp_buffers(vqc_mlp m, float **params, float **grads, size_t *count);

/* y[b] = E_hat(x[b]) for x [batch][n_in]; when dydx is non-NULL also the
 * input gradient dE_hat/dx [batch][n_in] (backpropagation to the input). */
vqc_status vqc_mlp_forward(vqc_mlp m, int batch, const float *x, float *y, float *dydx);

/* Parameter gradient (into the gradient buffer) of the loss
 *   L = mean_b (E_hat(x_b) - e_b)^2 + lambda / (batch n_in) sum_b |dE_hat/dx(x_b) - g_b|^2
 * where g may be NULL (then lambda is ignored).  The gradient term needs the
 * second derivatives of the network (double backpropagation).  y and dydx
 * (optional, device) receive the forward outputs. */
vqc_status vqc_mlp_backward(vqc_mlp m, int batch, const float *x, const float *e, const float *g, float lambda,
                            float *y, float *dydx);

/* One Adam step on the parameters with the current gradient (step >= 1). */
vqc_status vqc_mlp_adam(vqc_mlp m, float lr, float beta1, float beta2, float eps, int step);

/* `steps` plain gradient-descent steps on the inputs: x <- x - lr dE_hat/dx
 * (the surrogate's proposal for each row of x). */
vqc_status vqc_mlp_descend_inputs(vqc_mlp m, int batch, float *x, float lr, int steps);

#ifdef __cplusplus
}
#endif
#endif /* VQC_ABI_INCLUDED */
