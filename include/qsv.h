/*
 * qsv.h -- C ABI of the cache-blocked state-vector library (one AMD MI355X, gfx950).
 *
 * What is computed (Doi & Horii, arXiv:2102.02957):
 *   A state of 2^n complex amplitudes (Sec. II-A), qubit k <-> bit k of the
 *   amplitude index, evolved by a circuit, i.e. a sequence of gates (Sec. II-A,
 *   Eq. (1) u3 and Eq. (2) CNOT).  The result is psi_out = U_G ... U_1 psi_in in
 *   the original qubit order.
 *
 *   Blocked mode follows the paper's cache blocking (Sec. IV): the circuit is
 *   transpiled into sections (begin_blocking ... end_blocking) each of which
 *   acts only on the 2^c amplitudes of a chunk (Sec. II-B, IV-C), with
 *   chunk_swap operations between sections choosing which qubits are local.
 *   On one GPU the chunk is staged in on-chip memory (registers + LDS) instead
 *   of GPU memory, so every section costs one read and one write of the state
 *   in HBM instead of one per gate.  Per-gate mode applies one kernel per gate
 *   (the baseline of Sec. V-A: every gate is one pass over the state).
 *
 * Conventions shared by every call:
 *   - A state is a caller-owned, contiguous device array of 2^n amplitudes,
 *     interleaved (re, im): float pairs for QSV_C64, double pairs for
 *     QSV_C128, 256-byte aligned.  The library never frees or reallocates it.
 *   - All device work is asynchronous on the caller's HIP stream `stream`
 *     (hipStream_t passed as void*; NULL = the default stream); no call
 *     synchronises the stream except qsv_timing_read.  Host arrays passed in
 *     (gates, terms, offsets) are read during the call only.  Device faults
 *     surface at the caller's next synchronisation.
 *   - A context may be used from several streams and threads.  Calls are
 *     serialised on the host; the context's device workspaces (parameter
 *     tables, reduction partials, observable tables) are ordered across streams
 *     with events, so the device work of two calls on different streams never
 *     shares them concurrently.  Under HIP graph capture no event is recorded:
 *     a context used inside a captured graph must not be used from another
 *     stream while that graph runs, and qsv_reserve must have sized its
 *     workspaces beforehand (a workspace that would have to grow during
 *     capture returns QSV_E_STATE).
 *   - Every call returns a qsv_status; nothing throws across the ABI.  A
 *     thread-local message for the last failure is returned by qsv_last_error().
 *   - Arguments are validated eagerly on the host; an invalid call leaves all
 *     buffers untouched and returns QSV_E_INVALID (or QSV_E_UNSUPPORTED).
 */
#ifndef QSV_INCLUDE_QSV_H_
#define QSV_INCLUDE_QSV_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QSV_OK = 0,
    QSV_E_INVALID = -1,     /* bad argument (qubit out of range, duplicate, size) */
    QSV_E_NOMEM = -2,       /* a library-owned workspace allocation failed */
    QSV_E_HIP = -3,         /* a HIP runtime call or kernel launch failed */
    QSV_E_UNSUPPORTED = -4, /* valid request this build does not handle */
    QSV_E_NUMERIC = -5,     /* non-finite angle, matrix entry or observable coefficient */
    QSV_E_STATE = -6        /* call out of order (e.g. destroyed object) */
} qsv_status;

typedef enum { QSV_C64 = 1, QSV_C128 = 2 } qsv_dtype;

/* Gate kinds.  Qubit order of q[]:
 *   one-qubit kinds: q[0]
 *   QSV_CX: q[0] = control, q[1] = target   (Eq. (2): swap of the x_c=1 pairs)
 *   QSV_CZ, QSV_CP, QSV_SWAP: q[0], q[1]
 *   QSV_UNITARY: q[0..nq-1], q[0] the least significant bit of the matrix's
 *                row/column index (local index = sum_j bit(q[j]) << j)
 * Angles p[]:
 *   QSV_U3: (theta, phi, lambda) of Eq. (1) (the paper's psi is OpenQASM's phi)
 *   QSV_RX/RY/RZ: theta, exp(-i theta P / 2);  QSV_P: diag(1, e^{i p[0]});
 *   QSV_CP: diag(1, 1, 1, e^{i p[0]}). */
enum {
    QSV_H = 1, QSV_X, QSV_Y, QSV_Z, QSV_S, QSV_SDG, QSV_T, QSV_TDG,
    QSV_RX, QSV_RY, QSV_RZ, QSV_P, QSV_U3,
    QSV_CX, QSV_CZ, QSV_CP, QSV_SWAP,
    QSV_UNITARY,
    /* Noise channels rho <- sum_m K_m rho K_m^dagger, accepted by qsv_plan_density only
     * (Sec. III-A: the simulator's noise model for noisy simulation and its density-matrix
     * and super-operator methods):
     *   QSV_AMP_DAMP   1 qubit, p[0] = gamma:  K0 = [[1, 0], [0, sqrt(1-gamma)]],
     *                                          K1 = [[0, sqrt(gamma)], [0, 0]]
     *   QSV_PHASE_DAMP 1 qubit, p[0] = lambda: K0 = [[1, 0], [0, sqrt(1-lambda)]],
     *                                          K1 = [[0, 0], [0, sqrt(lambda)]]
     *   QSV_DEPOLARIZE 1 qubit, p[0] = p:      sqrt(1-p) I, sqrt(p/3) X, sqrt(p/3) Y, sqrt(p/3) Z
     *   QSV_KRAUS      nq = 1 or 2, param = number of operators M in [1, 16]; m = M matrices
     *                  of 2^nq x 2^nq complex, row-major, back to back (local index as for
     *                  QSV_UNITARY).  Completeness sum K^dagger K = I is not required. */
    QSV_AMP_DAMP, QSV_PHASE_DAMP, QSV_DEPOLARIZE, QSV_KRAUS
};

#define QSV_MAX_QUBITS 34       /* 2^34 amplitudes: 128 GiB complex64, 256 GiB complex128 */
#define QSV_MAX_GATE_QUBITS 5
#define QSV_MAX_TERMS 4096      /* Z-strings per observable */

typedef struct {
    int32_t kind;
    int32_t nq;                  /* number of qubits; must match the kind */
    int32_t q[QSV_MAX_GATE_QUBITS];
    int32_t param;               /* >= 0: p[0] is taken from params[param] at run time
                                    (QSV_RX/RY/RZ/P only; qsv_adjoint_grad, qsv_apply_params) */
    double p[3];
    const double *m;             /* QSV_UNITARY: 2^nq x 2^nq complex, row-major, (re, im)
                                    pairs, host memory, read during qsv_plan_blocks only */
} qsv_gate;

enum { QSV_SWAP_REMAP = 0, QSV_SWAP_MATERIALIZE = 1 };
enum { QSV_MODE_BLOCKED = 0, QSV_MODE_PER_GATE = 1 };

typedef struct {
    int32_t chunk_bits;          /* c: qubits per chunk (Sec. II-B "nc"); 0 = default
                                    (12 for QSV_C128, 13 for QSV_C64) */
    int32_t pinned_low_bits;     /* L: physical bits 0..L-1 always local (coalescing); -1 = default */
    int32_t fusion_max_qubits;   /* f: fuse consecutive in-section gates up to f qubits; 0/1 = off */
    int32_t swap_mode;           /* QSV_SWAP_REMAP (chunk_swap = change of the chunk's bit set,
                                    no data moves) or QSV_SWAP_MATERIALIZE (chunk_swap moves
                                    amplitudes, Sec. IV-C Fig. "chunk_swap") */
    int32_t diag_free;           /* 1: diagonal gates and CX controls need not be local (Sec. V-A:
                                    QFT's diagonal gates need less exchange) */
    int32_t register_bits;       /* r: amplitudes per GPU thread = 2^r; 0 = default.  A chunk
                                    runs on 2^(c-r) threads: c - r <= 9 for r <= 4, <= 8 for r = 5 */
    int32_t io_phases;           /* 1: a section whose first (last) phase holds one of the six
                                    lowest local bits in registers gathers (scatters) through an
                                    extra op-free phase in which lanes sit on those bits: one more
                                    LDS transposition for coalesced HBM access (large states
                                    only); 0: gather and scatter in the phases' own maps */
    int32_t planner;             /* chunk choice (Sec. IV-A leaves it open; its heuristic is
                                    not claimed optimal): QSV_PLANNER_DEFAULT (greedy
                                    candidates scored by a greedy rollout of the rest, one
                                    section of lookahead above 1024 gates), _GREEDY (one
                                    section of lookahead), _BEAM (beam searches over
                                    section sequences (one beam ranked by remaining gates, one by a greedy
                                    rollout of the rest), never more sections than DEFAULT; remap
                                    mode), _EXACT (minimum number of sections by breadth-first
                                    search; remap mode, at most 64 gates and 24 qubits,
                                    QSV_E_UNSUPPORTED beyond or when the search is too large) */
    int32_t section_kernel;      /* QSV_KERNEL_REGISTERS: the chunk lives in registers (2^r
                                    amplitudes per thread) and moves between register phases
                                    through LDS; QSV_KERNEL_LDS: the chunk stays in LDS for the
                                    whole section (2^c amplitudes of LDS per workgroup, at most
                                    128 KiB) and every op reads and writes it there (one phase per
                                    section; register_bits is ignored; plans without bound
                                    parameters, not for qsv_batch_run); QSV_KERNEL_PAIRED: a
                                    section whose gates are all dense 2-qubit gates on chunk
                                    qubits runs phases of two fused gate pairs at fixed register
                                    positions (the amplitudes are updated in place, no run-time
                                    choice of registers); other sections use the register
                                    phases; the plan uses 4 register bits; QSV_KERNEL_MFMA:
                                    as QSV_KERNEL_LDS, with in-section gates fused into blocks
                                    of up to fusion_max_qubits (4 or 5) qubits (commuting gates
                                    gathered across the section, not only consecutive ones)
                                    and every dense op of 4 or 5 qubits applied as a complex
                                    matrix product on the matrix cores (chunk_bits >= 9; gates
                                    of up to 5 qubits) */
} qsv_options;

enum { QSV_KERNEL_REGISTERS = 0, QSV_KERNEL_LDS = 1, QSV_KERNEL_PAIRED = 2, QSV_KERNEL_MFMA = 3 };
enum { QSV_PLANNER_DEFAULT = 0, QSV_PLANNER_GREEDY = 1, QSV_PLANNER_BEAM = 2,
       QSV_PLANNER_EXACT = 3 };

/* Fill *opt with the defaults for dt. */
qsv_status qsv_default_options(qsv_dtype dt, qsv_options *opt);

/* ---- plans (host only; no GPU needed) ------------------------------------ */

typedef struct qsv_plan qsv_plan;

/* Cache-blocking transpile (Sec. IV-A, the transpiler listing): bit
 * reordering, chunk qubit choice, chunk_swap insertion, section scan, then
 * per-section register phases and gate fusion.  `g` is read during the call
 * only.  n in [1, QSV_MAX_QUBITS].  The plan is immutable and may be shared
 * between threads and contexts; destroy it only when no launch using it is in
 * flight.  Errors: QSV_E_INVALID on a bad gate (kind, nq, qubit range,
 * duplicates, missing matrix) or option; QSV_E_NUMERIC on a non-finite angle or
 * matrix entry; QSV_E_UNSUPPORTED when the launch grid of a section would exceed
 * the hardware limits (n - register_bits > 31 or n - chunk_bits > 30). */
qsv_status qsv_plan_blocks(const qsv_options *opt, qsv_dtype dt, int n,
                           const qsv_gate *g, size_t ng, qsv_plan **plan);
void qsv_plan_destroy(qsv_plan *plan);

/* Density-matrix plan (Sec. III-A: the density-matrix method of the simulator; the
 * cache blocking applies unchanged).  The n-qubit density matrix rho is held as a
 * state of 2n qubits: amplitude index i | (j << n) holds rho[i][j] (row i = qubits
 * 0..n-1, column j = qubits n..2n-1).  A gate U on qubits Q becomes U on Q and conj(U)
 * on Q + n, since (U rho U^dagger)[i][j] = sum U[i][i'] conj(U[j][j']) rho[i'][j']; a
 * channel with k-qubit Kraus operators K_m on Q becomes one dense 2k-qubit gate on
 * (Q, Q + n) with S[a | b << k][c | e << k] = sum_m K_m[a][c] conj(K_m[b][e]).  The
 * result is an ordinary plan of 2n qubits for qsv_apply_circuit / qsv_apply_sections;
 * qsv_init_basis with basis b | (b << n) prepares |b><b|, qsv_norm gives the purity
 * Tr(rho^2), qsv_dm_trace and qsv_dm_expval read the diagonal.  n in [1, 17]; gates
 * with bound parameters are refused (QSV_E_UNSUPPORTED). */
qsv_status qsv_plan_density(const qsv_options *opt, qsv_dtype dt, int n, const qsv_gate *g,
                            size_t ng, qsv_plan **plan);

typedef struct {
    int32_t n, dtype, chunk_bits, register_bits, pinned_low_bits;
    int32_t fusion_max_qubits;   /* fusion width applied: the requested one capped at
                                    register_bits and at 4 */
    int32_t swap_mode, diag_free;
    int64_t n_gates;             /* gates in the circuit */
    int64_t n_sections;          /* begin_blocking/end_blocking pairs */
    int64_t n_chunk_swaps;       /* qubits moved into the chunk over the whole plan */
    int64_t n_phases;            /* register phases over all sections */
    int64_t n_device_ops;        /* in-section ops after fusion */
    int64_t n_params;            /* 1 + largest gate param index (0 if none) */
    double  section_flops;       /* FP operations of the blocked path (FMA = 2) */
    int32_t final_perm[64];      /* logical qubit q sits at physical bit final_perm[q] after
                                    the last section (identity in remap mode) */
} qsv_plan_stats;
qsv_status qsv_plan_get_stats(const qsv_plan *plan, qsv_plan_stats *out);

/* Flat export of the transpiled circuit (Sec. IV-A output + Sec. IV-C ops):
 *   QSV_OP_BEGIN: begin_blocking; `mask` = physical bits of the chunk
 *   QSV_OP_END:   end_blocking
 *   QSV_OP_CHUNK_SWAP: swap physical bits q[0], q[1] (materialise mode only)
 *   QSV_OP_GATE:  circuit gate `gate` applied on physical qubits q[0..nq-1]
 * Writes at most `cap` ops; *n_ops receives the total needed. */
enum { QSV_OP_BEGIN = 1, QSV_OP_END = 2, QSV_OP_CHUNK_SWAP = 3, QSV_OP_GATE = 4 };
typedef struct {
    int32_t tag, gate, nq, q[QSV_MAX_GATE_QUBITS];
    uint64_t mask;
} qsv_op;
qsv_status qsv_plan_export(const qsv_plan *plan, qsv_op *ops, size_t cap, size_t *n_ops);

/* ---- device context ---------------------------------------------------- */

typedef struct qsv_ctx qsv_ctx;

/* Bind a context to HIP device `hip_device` for states of type dt: the
 * memory space that holds the state (Sec. II-B: one memory space per GPU;
 * Sec. IV-B: the state and its chunks live in the GPU's memory).  The context
 * owns small workspaces (uploaded plan tables, reduction partials, parameter
 * and observable tables), grown on demand or sized up front by qsv_reserve.
 * Options are per plan (qsv_plan_blocks), not per context.
 * Errors: QSV_E_HIP if no device is present, QSV_E_INVALID for a bad device
 * index or dtype. */
qsv_status qsv_create(qsv_ctx **ctx, int hip_device, qsv_dtype dt);
void qsv_destroy(qsv_ctx *ctx);
const char *qsv_last_error(void);

/* Size every context workspace that the calls below need for `plan` (or, with
 * plan == NULL, for reductions over states of n qubits) and `batch` states,
 * and upload the plan's device tables.  After it, qsv_apply_circuit,
 * qsv_apply_sections, qsv_apply_params, qsv_norm, qsv_overlap, qsv_expval,
 * qsv_normalize and qsv_adjoint_grad with that plan (n, batch at most the
 * reserved ones, at most QSV_MAX_TERMS terms) allocate nothing and only
 * enqueue kernels, so they may be captured into a HIP graph.  Must not be
 * called during capture (QSV_E_STATE). */
qsv_status qsv_reserve(qsv_ctx *ctx, const qsv_plan *plan, int n, int batch, void *stream);

/* state <- |basis> (Sec. IV-C: only one amplitude is 1, the rest 0). */
qsv_status qsv_init_basis(qsv_ctx *ctx, void *state, int n, uint64_t basis, void *stream);

/* state <- U_plan state, in place.  mode QSV_MODE_BLOCKED runs one kernel per
 * section (plus one permutation pass per chunk_swap group in materialise
 * mode, and a final reorder to the original qubit order); QSV_MODE_PER_GATE
 * runs one kernel per circuit gate.  The plan's dtype must match the
 * context's and plan n must equal n.  Plans with parameter-bound gates need
 * qsv_apply_params. */
qsv_status qsv_apply_circuit(qsv_ctx *ctx, const qsv_plan *plan, void *state, int n,
                             int mode, void *stream);

/* Checkpoint/resume: run sections [s0, s1) of a remap-mode blocked plan.  At
 * every section boundary the state is the circuit prefix's state in the
 * original order. */
qsv_status qsv_apply_sections(qsv_ctx *ctx, const qsv_plan *plan, void *state, int n,
                              int64_t s0, int64_t s1, void *stream);

/* Host-resident state: GPU memory as the cache of a state held in host memory (Sec.
 * IV-C: chunks stored in CPU memory are fetched to the GPU to run a section; Sec. V-B
 * runs 33-35 qubits on GPUs plus host memory; Sec. VI: slower storage fetched into
 * faster memory).  `host_state` is pinned host memory (hipHostMalloc) of 2^n
 * amplitudes, 256-byte aligned.  Sections [s0, s1) of a remap-mode plan run on slices:
 * for section s the state is cut along the o highest bits that are not local in s
 * (qsv_plan_stream_bits), o the smallest value for which three slice buffers of
 * 2^(n-o) amplitudes fit in `hbm_budget` bytes of device memory; each slice is copied
 * to the device (contiguous runs of 2^(lowest cut bit) amplitudes), runs the section
 * kernel there and is copied back, with the copies of neighbouring slices overlapping
 * the kernels on library streams.  All of a section's slices are back in host memory
 * before the next section reads any.  The call is asynchronous: the copies start after
 * the work already on `stream` and `stream` waits for the last one.  The result equals
 * qsv_apply_sections on a device-resident state bit for bit.  Plans that read
 * non-local qubits (diag_free gates on such qubits) are refused (plan with
 * diag_free = 0), as are budgets that need more cut bits than some section leaves
 * non-local (QSV_E_UNSUPPORTED). */
qsv_status qsv_apply_host(qsv_ctx *ctx, const qsv_plan *plan, void *host_state, int n,
                          size_t hbm_budget, int64_t s0, int64_t s1, void *stream);
/* The cut bits of every section for o slice bits: mask_out[s] (host array of
 * n_sections entries).  Host only.  QSV_E_UNSUPPORTED when a section has fewer than o
 * non-local bits or slices would hold less than one chunk. */
qsv_status qsv_plan_stream_bits(const qsv_plan *plan, int o, uint64_t *mask_out);

/* Blocked apply of a parameterised plan to `batch` states stored back to back
 * (state b at states + b * 2^n amplitudes), parameters params_dev[b * P + p]
 * (device, double), P = stats.n_params. */
qsv_status qsv_apply_params(qsv_ctx *ctx, const qsv_plan *plan, void *states, int n, int batch,
                            const double *params_dev, void *stream);

/* ---- FP64 reductions (deterministic; device outputs) ------------------- */

typedef struct { double coeff; uint64_t zmask; } qsv_zterm;  /* coeff * prod_{i in zmask} Z_i */

/* out_dev[0] = <psi|psi> */
qsv_status qsv_norm(qsv_ctx *ctx, const void *state, int n, double *out_dev, void *stream);
/* out_dev[0..3] = Re<a|b>, Im<a|b>, <a|a>, <b|b> */
qsv_status qsv_overlap(qsv_ctx *ctx, const void *a, const void *b, int n, double *out_dev,
                       void *stream);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): qsv_overlap with its reduction
 * partials in a fixed library array of QSV_NOALLOC_PARTIALS doubles per GPU (64 KiB,
 * enough for any n <= QSV_MAX_QUBITS; larger requests are refused with QSV_E_INVALID),
 * instead of a context workspace.  The call allocates nothing and only enqueues two
 * kernels; the array's address is looked up once per device in qsv_create.  All calls
 * on one GPU share that array and it keeps the last call's contents (every entry is
 * written before it is read): calls that overlap in time on one GPU, from any context or
 * stream, race, and the caller must order them. */
#define QSV_NOALLOC_PARTIALS 8192
qsv_status qsv_overlap_noalloc(qsv_ctx *ctx, const void *a, const void *b, int n,
                               double *out_dev, void *stream);
/* out_dev[0] = sum_x |a_x|^2 sum_t coeff_t (-1)^popcount(x & zmask_t).  terms: host
 * array of 1..QSV_MAX_TERMS entries, read during the call (it travels to the device in
 * kernel arguments; the call does not synchronise).  QSV_E_NUMERIC for a non-finite
 * coefficient. */
qsv_status qsv_expval(qsv_ctx *ctx, const void *state, int n, const qsv_zterm *terms,
                      size_t n_terms, double *out_dev, void *stream);
/* Density matrices of n qubits (2^(2n) amplitudes, see qsv_plan_density), FP64 sums of the
 * diagonal in a fixed order: out_dev[0] = Tr(rho) = sum_i Re rho[i][i];
 * qsv_dm_expval: out_dev[0] = Tr(rho H) = sum_i Re rho[i][i] sum_t coeff_t (-1)^popcount(i & zmask_t). */
qsv_status qsv_dm_trace(qsv_ctx *ctx, const void *rho, int n, double *out_dev, void *stream);
qsv_status qsv_dm_expval(qsv_ctx *ctx, const void *rho, int n, const qsv_zterm *terms,
                         size_t n_terms, double *out_dev, void *stream);

/* Divide the state by sqrt(<psi|psi>) (computed in FP64); norm_out_dev[0] = <psi|psi>
 * before scaling.  A zero or non-finite norm leaves the state unscaled and sets
 * norm_out_dev[0] to it; the caller checks it. */
qsv_status qsv_normalize(qsv_ctx *ctx, void *state, int n, double *norm_out_dev, void *stream);
/* dst <- src (2^n amplitudes): a plain streaming copy. */
qsv_status qsv_copy(qsv_ctx *ctx, void *dst, const void *src, int n, void *stream);

/* ---- adjoint gradient -------------------------------------------------- */

/* E_b = <psi_b|H|psi_b>, grad_b[p] = dE_b / dtheta_p for psi_b = U(theta_b)|0>, H = sum of
 * Z-strings (terms: host array), for `batch` parameter vectors params_dev[b * P + p]
 * (device, double; P = stats.n_params).  psi_dev and lambda_dev are caller workspaces of
 * batch * 2^n amplitudes each; their contents on return are unspecified (the reverse sweep
 * runs psi back towards |0>).  energy_dev[batch], grad_dev[batch * P] (device, double).
 * The forward pass is the blocked apply; the reverse sweep follows the blocked plan
 * backwards, one kernel per section holding the psi and lambda chunks, with per-chunk
 * FP64 partials reduced in a fixed order.  Needs a remap-mode plan with fusion of at most
 * 2 qubits (QSV_E_UNSUPPORTED otherwise). */
qsv_status qsv_adjoint_grad(qsv_ctx *ctx, const qsv_plan *plan, const qsv_zterm *terms,
                            size_t n_terms, const double *params_dev, int batch,
                            void *psi_dev, void *lambda_dev, double *energy_dev,
                            double *grad_dev, void *stream);

/* ---- batched trajectories ---------------------------------------------- */

/* Run `count` independent circuits (e.g. noisy trajectories with sampled Pauli
 * insertions: the noisy simulation and repeated shots of Sec. III-A, each run as its
 * own state), each on its own state of n_b qubits stored at states + offsets[b]
 * amplitudes (offsets: host array; states must not overlap and must start on 256-byte
 * boundaries), in one graph launch: every state is set to |0>; then, for each section
 * depth d, one kernel runs section d of every plan that has one, a workgroup per
 * (state, chunk); the last section of each plan writes per-chunk FP64 norms, reduced in
 * chunk order, and every state is rescaled by 1/sqrt(norm).  norms_dev[b] receives
 * <psi_b|psi_b> before the rescale.  The sequence is captured into a HIP graph on the
 * first call for a given (plans, offsets, states, norms_dev) and replayed afterwards.
 * Plans: same dtype as the context, remap mode, no bound parameters, equal
 * register_bits, chunk_bits - register_bits <= 8 (QSV_E_UNSUPPORTED otherwise). */
qsv_status qsv_batch_run(qsv_ctx *ctx, int count, const qsv_plan *const *plans,
                         const uint64_t *offsets, void *states, double *norms_dev,
                         void *stream);

/* ---- autotuning -------------------------------------------------------- */

/* Time `n_cands` option sets on the circuit (n, g, ng): for each, plan, run one
 * untimed blocked apply on `state` (a caller-owned scratch of 2^n amplitudes of the
 * context's dtype, overwritten), then `reps` timed applies between HIP events on
 * `stream`.  With max_sections > 0 a remap-mode candidate runs only its first
 * max_sections sections (qsv_apply_sections) and its time is scaled by
 * S / max_sections, S being that candidate's section count, so large circuits are
 * compared without running them whole; then (refine > 0) the `refine` best estimates
 * are timed again on whole applies and the winner is the fastest of those.
 * *best = index of the winner; ms_out[k] (host, may be NULL) = milliseconds per whole
 * apply (measured for refined candidates, else the estimate), +inf for candidates that
 * cannot be planned.  Chooses chunk_bits, pinned_low_bits,
 * fusion_max_qubits, register_bits and the schedule options (swap_mode, io_phases)
 * for the caller's own workload (the paper's chunk size nc, Sec. II-B, is a free
 * parameter). */
qsv_status qsv_autotune(qsv_ctx *ctx, qsv_dtype dt, int n, const qsv_gate *g, size_t ng,
                        const qsv_options *cands, int n_cands, void *state, int reps,
                        int max_sections, int refine, void *stream, int *best, double *ms_out);
/* The same for a batch of circuits run through qsv_batch_run (ns[b], gates[b], ngs[b],
 * offsets[b] as there; states / norms_dev are overwritten). */
qsv_status qsv_autotune_batch(qsv_ctx *ctx, qsv_dtype dt, int count, const int *ns,
                              const qsv_gate *const *gates, const size_t *ngs,
                              const uint64_t *offsets, const qsv_options *cands, int n_cands,
                              void *states, double *norms_dev, int reps, void *stream, int *best,
                              double *ms_out);

/* The same for qsv_adjoint_grad on a parameterised circuit: every candidate plan runs
 * the whole forward + reverse sweep (psi_dev, lambda_dev, energy_dev, grad_dev are
 * overwritten); candidates the adjoint sweep does not support get +inf. */
qsv_status qsv_autotune_adjoint(qsv_ctx *ctx, qsv_dtype dt, int n, const qsv_gate *g, size_t ng,
                                const qsv_zterm *terms, size_t n_terms, const double *params_dev,
                                int batch, void *psi_dev, void *lambda_dev, double *energy_dev,
                                double *grad_dev, const qsv_options *cands, int n_cands, int reps,
                                void *stream, int *best, double *ms_out);

/* ---- timing (in-library HIP events around each launch) ------------------ */

/* When enabled, every section / per-gate launch is bracketed by HIP events on the
 * launch stream; qsv_timing_read returns the summed kernel milliseconds and launch
 * counts since the last reset for kernel class `which`
 * (0 = section kernels, 1 = per-gate kernels).  Reading synchronises the stream. */
qsv_status qsv_timing_enable(qsv_ctx *ctx, int enable);
qsv_status qsv_timing_read(qsv_ctx *ctx, int which, double *total_ms, int64_t *launches,
                           int reset);

#ifdef __cplusplus
}
#endif
#endif /* QSV_INCLUDE_QSV_H_ */
