/*
 * qsim.h -- C ABI of libqsim, an MI355X (gfx950) implementation of the
 * unitary-matrix circuit simulation method of TornadoQSim (arXiv 2305.14398).
 *
 * The method (Section 5.3, stages 1-6; Algorithms 1 and 2):
 *   1-3  split the ordered gate list into steps and fetch each gate's matrix;
 *   4    expand each step into its dense 2^n x 2^n operator: the Kronecker
 *        product of the step's gates with identities on idle qubits (Eq. 9s1),
 *        two-qubit gates on non-adjacent qubits embedded over their span;
 *   5    multiply the step operators into the circuit unitary,
 *        result <- A . result from result = I;
 *   6    multiply the circuit unitary by the initial state vector.
 *
 * Conventions used by every call
 * ------------------------------
 * Qubit order: little-endian.  Qubit q is bit q of a basis-state index
 *   (qubit 0 is the least significant bit).
 * N = 2^n_qubits, 1 <= n_qubits <= QSIM_MAX_QUBITS.
 * Complex matrices ("planar complex64"): two N x N float32 planes, the real
 *   plane followed by the imaginary plane, 8*N*N bytes in total.  Row-major:
 *   entry (r, c) real part at [r*N + c], imaginary part at [N*N + r*N + c].
 *   Column-major (QSIM_LAYOUT_COL): entry (r, c) at [c*N + r] and
 *   [N*N + c*N + r].
 * Split 16-bit operands (QSIM_SPLIT_BF16 / QSIM_SPLIT_FP16): four N x N
 *   16-bit planes in the order re_hi, re_lo, im_hi, im_lo (8*N*N bytes),
 *   value = hi + lo * 2^-QSIM_LO_SCALE_LOG2 for fp16 (lo is stored
 *   pre-scaled) and hi + lo for bf16.  The three-product split precisions
 *   (QSIM_SPLIT_BF16_3M / QSIM_SPLIT_FP16_3M) add two planes sum_hi, sum_lo
 *   holding the split of the float32 sum re + im (12*N*N bytes, six planes);
 *   qsim_op_bytes gives the size of one operand in any precision.  From
 *   n_qubits = 6 on, three-product operands are fragment-blocked: with i the
 *   storage row and k the storage column (the contraction index), element
 *   (plane p, i, k) is at 16-bit index
 *     (((i/32) * (N/16) + k/16) * 6 + p) * 512 + ((i%32) + 32*((k/8)%2)) * 8 + k%8,
 *   i.e. 32 x 16 blocks in row-block-major order, each holding its six planes
 *   as contiguous 1 KiB MFMA fragments.  Below 6 qubits they are planar.
 * State vectors: planar complex64, N float32 real parts then N imaginary.
 * Device pointers are hipMalloc'd (or torch-allocated) memory on the
 *   context's device, 256-byte aligned, owned by the caller; the library does
 *   not keep them after a call returns (except qsim_submit, see there).
 * Streams: `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *   Device work is enqueued on it asynchronously; calls that return host
 *   values synchronise that stream first and say so.
 * Errors: every argument is checked before any device work is enqueued.  A
 *   call returns a qsim_status; on failure nothing was launched and
 *   qsim_last_error() describes the problem.  Errors the device reports
 *   later surface as QSIM_E_DEVICE from the next call on the context.
 */
#ifndef LIBQSIM_QSIM_H_
#define LIBQSIM_QSIM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QSIM_MAX_QUBITS 16
#define QSIM_MAX_GATES_PER_STEP 16
#define QSIM_LO_SCALE_LOG2 12

typedef enum qsim_status {
    QSIM_OK = 0,
    QSIM_PENDING = 1,        /* qsim_poll: request not finished yet */
    QSIM_E_INVALID = -1,     /* malformed argument (null, bad gate, overlap, alignment) */
    QSIM_E_RANGE = -2,       /* size out of range (qubits, workspace too small) */
    QSIM_E_OOM = -3,         /* arena / workspace cannot hold the request */
    QSIM_E_DEVICE = -4,      /* a HIP call failed */
    QSIM_E_FULL = -5,        /* qsim_submit: queue full (back-pressure) */
    QSIM_E_UNKNOWN_ID = -6,  /* qsim_poll: no such request */
    QSIM_E_CANCELLED = -7    /* request dropped because the engine stopped before admitting it */
} qsim_status;

/* Arithmetic of the chain product (stage 5). */
typedef enum qsim_precision {
    QSIM_FP32_4M = 0,     /* float32 MFMA, four real products per complex product */
    QSIM_FP32_3M = 1,     /* float32 MFMA, three real products (Gauss) */
    QSIM_SPLIT_BF16 = 2,  /* operands split into bf16 hi + lo, three bf16 MFMA passes, fp32 accumulate */
    QSIM_SPLIT_FP16 = 3,  /* operands split into fp16 hi + scaled lo, three passes, fp32 accumulate */
    QSIM_SPLIT_BF16_3M = 4, /* as QSIM_SPLIT_BF16 with three real products (Gauss): 9 MFMAs per k-block, not 12 */
    QSIM_SPLIT_FP16_3M = 5  /* as QSIM_SPLIT_FP16 with three real products (Gauss) */
} qsim_precision;

/* Gate kinds.  A gate with control >= 0 is the controlled version of its kind
 * (Section 2.3, Eq. 7): CNOT = {QSIM_X, control c, target t}, CZ = {QSIM_Z, ..},
 * CR_phi = {QSIM_R, .., theta = phi}.  Matrices (rows = output bit):
 *   H, X, Y, Z, R_phi = diag(1, e^{i phi}) as in Section 2.3, Table 1;
 *   S = diag(1, i), T = diag(1, e^{i pi/4}) (named in Section 5.2.2);
 *   RX, RY, RZ(theta) = exp(-i theta sigma_{x,y,z} / 2);
 *   U2 = the caller's 2x2 matrix in u[] (row-major (re, im) pairs);
 *   SWAP exchanges qubits `target` and `control` (the second qubit; not a
 *   controlled gate; used by the QFT figure of Section 2.5);
 *   CUSTOM = a registered unitary (qsim_register_unitary) of m qubits applied
 *   to the range target .. target+m-1 (Section 5.2.2: custom functions are
 *   registered with the operation data provider, then applied to a range of
 *   qubits); `op_id` names it, `control` must be -1. */
typedef enum qsim_kind {
    QSIM_H = 0, QSIM_X = 1, QSIM_Y = 2, QSIM_Z = 3, QSIM_S = 4, QSIM_T = 5,
    QSIM_R = 6, QSIM_RX = 7, QSIM_RY = 8, QSIM_RZ = 9, QSIM_U2 = 10, QSIM_SWAP = 11,
    QSIM_CUSTOM = 12
} qsim_kind;

typedef struct qsim_gate {
    int32_t kind;      /* qsim_kind */
    int32_t target;    /* qubit the 2x2 acts on; first qubit of a SWAP; lowest qubit of a CUSTOM range */
    int32_t control;   /* control qubit, -1 if none; second qubit of a SWAP */
    int32_t op_id;     /* QSIM_CUSTOM: id from qsim_register_unitary; 0 for every other kind */
    double theta;      /* angle of R, RX, RY, RZ; ignored otherwise */
    double u[8];       /* QSIM_U2 only: u00 re, u00 im, u01 re, u01 im, u10 .., u11 .. */
} qsim_gate;           /* 88 bytes */

/* ---- Operation data provider (Section 5.2.2) -------------------------------------------------
 * Registers a custom unitary of m = n_qubits qubits (1 <= m <= QSIM_CUSTOM_MAX_QUBITS) under a
 * unique name.  `matrix` is 2^m x 2^m, row-major, (re, im) float64 pairs (2 * 4^m doubles); row
 * and column index bit k is qubit target+k of the range the operation is applied to.  The
 * matrix is checked to be unitary (max |M^H M - I| <= 1e-9), copied, and uploaded to every
 * visible device; entries live until the process ends.  Process-wide and thread-safe; host
 * only when no device is visible.  QSIM_E_INVALID for a duplicate name, a non-finite entry or
 * a non-unitary matrix; QSIM_E_RANGE for m out of range or a full registry
 * (QSIM_CUSTOM_MAX_OPS entries).  *id_out receives the id (>= 1). */
#define QSIM_CUSTOM_MAX_QUBITS 6
#define QSIM_CUSTOM_MAX_OPS 4096
qsim_status qsim_register_unitary(const char* name, int n_qubits, const double* matrix, int32_t* id_out);
/* Looks up a registered operation by name: its id and qubit count (either out pointer may be
 * NULL).  QSIM_E_UNKNOWN_ID if no operation has that name. */
qsim_status qsim_find_unitary(const char* name, int32_t* id_out, int* n_qubits_out);

typedef enum qsim_layout { QSIM_LAYOUT_ROW = 0, QSIM_LAYOUT_COL = 1 } qsim_layout;

typedef struct qsim_ctx qsim_ctx;

/* Thread-local description of the last failure on this thread; valid until the
 * next qsim call on the same thread.  Never NULL. */
const char* qsim_last_error(void);

/* Library version string. */
const char* qsim_version(void);

/* Create a context on HIP device `device` (0-based).  Allocates about 9 MB of
 * device scratch for reductions.  *out receives the context. */
qsim_status qsim_ctx_create(int device, qsim_ctx** out);
/* Destroy a context (stops its serving engine, if started).  NULL is a no-op. */
qsim_status qsim_ctx_destroy(qsim_ctx* ctx);

/* Stages 1-2 (Section 5.2.1: steps are created as gates are added).  Host only.
 * A gate joins the most recent step if its qubit span [min q, max q] is
 * disjoint from the span of every gate already in that step; otherwise it
 * opens a new step.  Writes n_steps+1 offsets into step_offsets (capacity
 * n_gates+1 int32): step j holds gates [step_offsets[j], step_offsets[j+1]).
 * Validates every gate (qubits in range, control != target, kind known).
 * Also fails if a step would exceed QSIM_MAX_GATES_PER_STEP (cannot happen
 * for disjoint spans when n_qubits <= 16). */
qsim_status qsim_pack_steps(int n_qubits, const qsim_gate* gates, int n_gates,
                            int32_t* step_offsets, int* n_steps_out);

/* Workspace qsim_unitary_chain needs for (n_qubits, prec), in bytes
 * (scratch step operator + ping-pong chain buffers), or 0 if out of range. */
size_t qsim_chain_workspace_bytes(int n_qubits, int prec);

/* Bytes of one N x N operand in the format of `prec` (what qsim_build_step
 * writes and qsim_step_multiply reads): 8*N*N for the float32 precisions and
 * the four-plane split ones, 12*N*N for the six-plane three-product split
 * ones; 0 if out of range. */
size_t qsim_op_bytes(int n_qubits, int prec);

/* Stage 4 (Algorithm 2, Eq. 9s1): write the dense operator of ONE step.
 * gates[0..n_gates) must have pairwise disjoint spans (QSIM_E_INVALID
 * otherwise).  Each entry is the product over the step's gates of their
 * matrix entries (identity on idle qubits), computed in float64 and rounded
 * once to the output format.
 * prec QSIM_FP32_4M / QSIM_FP32_3M: planar complex64 in `layout`;
 * prec QSIM_SPLIT_BF16 / QSIM_SPLIT_FP16: four split 16-bit planes in `layout`;
 * prec QSIM_SPLIT_BF16_3M / QSIM_SPLIT_FP16_3M: six planes, the last two the
 *      split of the float32 sum of each entry's rounded real and imaginary parts.
 * d_op: qsim_op_bytes(n_qubits, prec) bytes, caller-owned. */
qsim_status qsim_build_step(qsim_ctx* ctx, int n_qubits, const qsim_gate* gates, int n_gates,
                            int prec, int layout, void* d_op, void* stream);

/* Stage 5, one product (Algorithm 1, result <- A . result): C = S . U for
 * N x N complex matrices.  Operand layouts follow what each MFMA shape reads
 * contiguously along the contraction index:
 *   QSIM_FP32_4M / QSIM_FP32_3M: d_S planar complex64 COLUMN-major, d_Uin
 *      planar complex64 row-major, d_Uout (required) planar complex64
 *      row-major; d_Uout_split must be NULL.
 *   QSIM_SPLIT_BF16 / QSIM_SPLIT_FP16 (four planes) and QSIM_SPLIT_BF16_3M /
 *      QSIM_SPLIT_FP16_3M (six planes, qsim_op_bytes): d_S split planes
 *      ROW-major, d_Uin split planes COLUMN-major.  d_Uout (optional): C as
 *      planar complex64 row-major; d_Uout_split (optional): C as split planes
 *      column-major, i.e. the d_Uin of the next product.  At least one output;
 *      each requested output costs one kernel launch.  The three-product forms
 *      take T1 = Sr Ur, T2 = Si Ui, T3 = (Sr + Si)(Ur + Ui), Re C = T1 - T2,
 *      Im C = T3 - T1 - T2 (9 MFMAs per 16-deep k-block instead of 12).
 * Outputs must not alias inputs or each other. */
qsim_status qsim_step_multiply(qsim_ctx* ctx, int n_qubits, int prec, const void* d_S,
                               const void* d_Uin, void* d_Uout, void* d_Uout_split, void* stream);

/* Stages 4-5 for a whole circuit: d_U = S_k ... S_1 (row-major planar
 * complex64).  The first step's operator is the first partial product
 * (multiplying by the initial identity is exact and is skipped), so a
 * k-step circuit costs k expansions and k-1 products.  With a split
 * precision the partial products are carried in split form (re-split from the
 * float32 accumulators after every product) and only the last is written as
 * float32.
 * step_offsets: NULL -> packed with the qsim_pack_steps rule; otherwise
 *      n_steps+1 monotone offsets with offsets[0] = 0 and offsets[n_steps] =
 *      n_gates, each step of pairwise disjoint spans and 1..16 gates.
 * d_ws: device workspace of ws_bytes >= qsim_chain_workspace_bytes(n, prec)
 *      (2 matrices for float32, 3 operands of qsim_op_bytes for split
 *      precisions), not overlapping d_U.
 * n_gates == 0 yields the identity. */
qsim_status qsim_unitary_chain(qsim_ctx* ctx, int n_qubits, const qsim_gate* gates, int n_gates,
                               const int32_t* step_offsets, int n_steps, int prec,
                               void* d_U, void* d_ws, size_t ws_bytes, void* stream);

/* Stages 4 and 5 fused.  Section 5.3 lets a backend change how stages 4-6
 * compute; here one product C = S . U takes the step operator S straight from
 * the step's gates, entry by entry inside the product kernel, and never
 * stores it.  S's entries are the ones qsim_build_step writes (float64
 * product of the gate factors, rounded once), so d_Uout is bit-identical to
 * qsim_build_step (column-major) followed by qsim_step_multiply with the same
 * precision and tile table.
 * prec: QSIM_FP32_4M or QSIM_FP32_3M (QSIM_E_INVALID otherwise).
 * gates[0..n_gates): one step, pairwise disjoint spans (n_gates 0 = identity).
 * d_Uin, d_Uout: planar complex64 row-major, 8*N*N bytes each, caller-owned,
 *      256-byte aligned, not aliasing (QSIM_E_INVALID otherwise). */
qsim_status qsim_step_multiply_fused(qsim_ctx* ctx, int n_qubits, int prec, const qsim_gate* gates,
                                     int n_gates, const void* d_Uin, void* d_Uout, void* stream);

/* Workspace of qsim_unitary_chain_fused: one matrix (8*N*N bytes) for the
 * float32 precisions; 0 for split precisions or out-of-range arguments. */
size_t qsim_chain_fused_workspace_bytes(int n_qubits, int prec);

/* qsim_unitary_chain with stages 4 and 5 fused: the first step is expanded
 * into the first partial product as before, and every later product computes
 * its step operator inside the product (qsim_step_multiply_fused).  No step
 * operator is stored, so d_ws holds only the second ping-pong matrix
 * (ws_bytes >= qsim_chain_fused_workspace_bytes).  Same arguments, checks and
 * bit-identical results as qsim_unitary_chain; float32 precisions only. */
qsim_status qsim_unitary_chain_fused(qsim_ctx* ctx, int n_qubits, const qsim_gate* gates, int n_gates,
                                     const int32_t* step_offsets, int n_steps, int prec,
                                     void* d_U, void* d_ws, size_t ws_bytes, void* stream);

/* Stage 6: d_psi = d_U . psi0 (complex64 matrix-vector product over the full
 * row-major U).  d_psi0: planar complex64 initial state, or NULL for |0...0>
 * (Eq. 9).  Then, in float64: norm2 = sum |psi_i|^2 and, if d_prob is not
 * NULL, d_prob[i] = |psi_i|^2 / norm2 (N doubles).  If h_norm2 is not NULL the
 * stream is synchronised and *h_norm2 receives norm2. */
qsim_status qsim_apply_state(qsim_ctx* ctx, int n_qubits, const void* d_U, const void* d_psi0,
                             void* d_psi, double* d_prob, double* h_norm2, void* stream);

/* Measurement (the paper's simulateAndCollapse, Section 5.2.3): draws `shots`
 * basis-state indices with probabilities d_prob (N float64 values, e.g. from
 * qsim_apply_state; they need not sum exactly to 1).  The caller supplies the
 * random numbers: d_uniform holds `shots` float64 values in [0, 1), and shot k
 * is the smallest index i with u_k * C[N-1] < C[i], where C is the cumulative
 * sum of d_prob in float64 (each of 1024 threads sums a contiguous chunk, chunk
 * totals are scanned in a fixed order).  d_out: `shots` int64.  Uses the
 * context's scratch, like the drift calls: calls on one context must not
 * overlap on different streams. */
qsim_status qsim_sample(qsim_ctx* ctx, int n_qubits, const double* d_prob, const double* d_uniform, int shots,
                        int64_t* d_out, void* stream);

/* Unitarity drift of a row-major planar complex64 U (Section 2.3: a gate
 * matrix is unitary iff U^H = U^-1): computes D = U^H U - I in float64 and
 * returns h_out[0] = max |D_ij| and h_out[1] = ||D||_F / sqrt(N).  No N x N
 * float64 matrix is stored; the upper triangle of U^H U is formed with three
 * real float64 products (3 N^3 flops).  Synchronises the stream. */
qsim_status qsim_unitarity_drift(qsim_ctx* ctx, int n_qubits, const void* d_U, double* h_out,
                                 void* stream);
/* The same check without waiting: d_out (device memory, 2 doubles, 8-byte
 * aligned) receives max |D_ij| and ||D||_F / sqrt(N) when the stream reaches
 * it.  Uses the context's scratch for partial sums: calls on one context must
 * not overlap on different streams. */
qsim_status qsim_unitarity_drift_async(qsim_ctx* ctx, int n_qubits, const void* d_U, double* d_out, void* stream);
/* The asynchronous drift check for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no context, no workspace argument, and no allocation on any call.
 * Runs on the current device and `stream` with the same kernels, grid and
 * fixed-order reduction as qsim_unitarity_drift_async, so d_out (device, 2
 * doubles, 8-byte aligned) receives the same max |D_ij| and ||D||_F / sqrt(N)
 * bit for bit.  The partial sums live in one static 32 KiB device array per
 * GPU (2 x 2048 doubles, the most the drift grid ever uses; held until the
 * process ends), so any 1 <= n_qubits <= 16 fits and larger n is rejected with
 * QSIM_E_RANGE.  Every call on a device shares that array: calls that overlap
 * on one device (different streams or threads) race and must be ordered by the
 * caller.  Errors: QSIM_E_RANGE for n_qubits, QSIM_E_INVALID for NULL or
 * unaligned pointers, QSIM_E_DEVICE if the array's address cannot be resolved
 * or the launch fails. */
qsim_status qsim_unitarity_drift_noalloc(int n_qubits, const void* d_U, double* d_out, void* stream);

/* Probe form of the drift check for serving: with the fixed unit vector
 * x_j = exp(2 pi i frac(j g)) / sqrt(N) (g = (sqrt 5 - 1) / 2), computes
 * d = U^H (U x) - x in float64 (two passes over U) and returns
 * h_out[0] = max |d_j|, h_out[1] = |d|_2.  Synchronises the stream. */
qsim_status qsim_unitarity_drift_probe(qsim_ctx* ctx, int n_qubits, const void* d_U, double* h_out, void* stream);

/* ---- Batches of circuits of mixed size (stages 4-5 for many circuits) ----
 * One iteration of a batch expands the current step of every circuit that has
 * one in a single grouped launch, then takes every such circuit's current
 * chain product in a single grouped launch (persistent grid over a device job
 * table; each circuit keeps its own size and tile configuration).  Results
 * are the same products as qsim_unitary_chain with the same precision and
 * tile configuration, circuit by circuit. */
typedef struct qsim_circuit_desc {
    int32_t n_qubits;
    int32_t n_gates;
    const qsim_gate* gates;       /* copied at plan creation */
    const int32_t* step_offsets;  /* NULL: the qsim_pack_steps rule; else n_steps+1 offsets */
    int32_t n_steps;
    int32_t reserved;             /* must be 0 */
    void* d_U;                    /* out: row-major planar complex64 U (8*N*N bytes, 256-byte aligned) */
} qsim_circuit_desc;

#define QSIM_BATCH_GRAPH 1  /* capture the plan's launches in a hipGraph at first launch and replay it */

typedef struct qsim_batch_plan qsim_batch_plan;

/* Workspace a batch needs (2 matrices per circuit for float32, 3 operands of qsim_op_bytes for split
 * precisions, each rounded up to 256 bytes). */
qsim_status qsim_batch_workspace_bytes(const qsim_circuit_desc* circuits, int count, int prec, size_t* out);
/* Validate the batch, build and upload the job tables of every iteration (this
 * allocates the tables on the device; launching allocates nothing).  The
 * workspace and every d_U must stay valid and untouched by others for the
 * plan's lifetime; d_U ranges must not overlap each other or the workspace. */
qsim_status qsim_batch_plan_create(qsim_ctx* ctx, const qsim_circuit_desc* circuits, int count, int prec, void* d_ws,
                                   size_t ws_bytes, int flags, qsim_batch_plan** out);
/* Enqueue the whole batch on `stream` (2 grouped kernels per iteration, or one graph launch with QSIM_BATCH_GRAPH). */
qsim_status qsim_batch_plan_launch(qsim_batch_plan* plan, void* stream);
/* Iterations, number of chain products and their flop count (8 N^3 each). */
qsim_status qsim_batch_plan_info(const qsim_batch_plan* plan, int* iterations, int* products, double* flops);
/* Wait for the device and free the plan's tables and graph.  NULL is a no-op. */
qsim_status qsim_batch_plan_destroy(qsim_batch_plan* plan);
/* One-shot batch: create, launch, synchronise the stream, destroy. */
qsim_status qsim_unitary_chain_batched(qsim_ctx* ctx, const qsim_circuit_desc* circuits, int count, int prec,
                                       void* d_ws, size_t ws_bytes, void* stream);

/* ---- Tile autotuner ----
 * For n in [max(n_lo, 7), n_hi] (n_hi <= 13; below 7 qubits a 128-wide tile
 * does not fit, so n = 6 always uses 64) times grouped launches of identical
 * products with 64x64 and 128x128 tiles and records the faster tile edge per
 * n in the context (used by every later product of that precision family:
 * float32, split bf16 or split fp16; split fp16 always uses 64).  ms_out
 * (nullable, 2 doubles per n from 7): milliseconds per product for tile 64 and
 * tile 128 (-1 if not applicable).
 * The timed operands are seeded pseudo-random values (not zeros: the chip's
 * clock follows the switching power, so all-zero operands would time faster
 * than any chain).  The 64 / 128 timings stay in the context (qsim_tune_ms,
 * qsim_tune_save).  Synchronises; allocates scratch for the timing runs. */
qsim_status qsim_autotune(qsim_ctx* ctx, int prec, int n_lo, int n_hi, double* ms_out);
/* Current tile edge per qubit count (17 ints, index n; 0 = whole-product path). */
qsim_status qsim_tune_get(qsim_ctx* ctx, int prec, int* tiles_out);
/* Override the tile edge (64 or 128; split fp16: 64 only) for n in 7..16. */
qsim_status qsim_tune_set(qsim_ctx* ctx, int prec, int n_qubits, int tile);
/* Milliseconds per product the autotuner measured for (prec, n): ms_out[2n]
 * with 64-wide tiles, ms_out[2n + 1] with 128-wide ones, -1 where not measured
 * (34 doubles, n = 0..16). */
qsim_status qsim_tune_ms(qsim_ctx* ctx, int prec, double* ms_out);
/* Tile cache: qsim_tune_save writes the context's tile table, its tuned flags
 * and the measured timings of every precision to a small JSON file, with the
 * device (name, architecture, compute units) and the library build
 * (qsim_build_id: a hash of the sources it was built from).  qsim_tune_load
 * reads such a file into the context; QSIM_E_INVALID (table unchanged) if it
 * cannot be read, is malformed, holds an invalid tile, or was written by
 * another build or for another device, so a stale choice is never applied. */
qsim_status qsim_tune_save(qsim_ctx* ctx, const char* path);
qsim_status qsim_tune_load(qsim_ctx* ctx, const char* path);
const char* qsim_build_id(void);

/* ---- Serving: continuous batching of submitted circuits ----
 * qsim_serve_start runs an engine thread for the context with its own HIP
 * stream.  A request is admitted in arrival order once the caller's device
 * arena has room for its footprint (chain workspace: 2 matrices of 8*N*N
 * bytes for float32, 3 operands of qsim_op_bytes for split precisions, plus U
 * (8*N*N) when d_U is NULL; each rounded up to 256) and fewer than max_active
 * requests are admitted.
 * QSIM_SERVE_CONTINUOUS: every engine iteration advances every admitted
 *   request by one step (stages 4-5) in one grouped expansion launch and one
 *   grouped product launch; a request whose chain is complete gets stage 6
 *   (psi = U psi0, float64 norm) and, if asked, the float64 probe drift.
 *   Requests that arrive while others are on the GPU join at the next
 *   iteration.  Each request's arithmetic does not depend on what else is in
 *   flight (same tiles, same order), so results are identical alone and in
 *   the mix.
 * QSIM_SERVE_FIFO: the plain baseline; one request at a time through the
 *   qsim_unitary_chain kernels.
 * The engine allocates its job tables and result slots at start; serving
 * allocates nothing.  Calls may come from any thread. */
#define QSIM_SERVE_CONTINUOUS 0
#define QSIM_SERVE_FIFO 1

/* Continuous-mode policies.
 * QSIM_POLICY_ARRIVAL: admit in arrival order; every iteration advances every
 *   admitted request by one step.
 * QSIM_POLICY_SHORTEST: admit the queued request with the least estimated work
 *   (8 N^3 per chain product) that fits the arena; every iteration advances the
 *   admitted requests in order of least remaining work until the iteration's
 *   work reaches iter_budget_tflop (at least one request per iteration), so
 *   short circuits are not held to the pace of large ones.
 * QSIM_POLICY_AGED: as QSIM_POLICY_SHORTEST, ordered by remaining work minus
 *   aging_tflop_per_s x seconds since submission, so a request that has waited
 *   long enough overtakes newer small ones (bounds the tail that least work
 *   first alone gives the largest requests). */
#define QSIM_POLICY_ARRIVAL 0
#define QSIM_POLICY_SHORTEST 1
#define QSIM_POLICY_AGED 2

typedef struct qsim_serve_config {
    int32_t prec;            /* qsim_precision of every served chain */
    int32_t mode;            /* QSIM_SERVE_CONTINUOUS or QSIM_SERVE_FIFO */
    int32_t max_active;      /* 1..4096 requests advanced together (forced to 1 in FIFO mode) */
    int32_t queue_capacity;  /* queued (not yet admitted) requests before qsim_submit returns QSIM_E_FULL */
    void* d_arena;           /* caller-owned device memory, 256-byte aligned, untouched by others while serving */
    size_t arena_bytes;
    int32_t policy;          /* QSIM_POLICY_ARRIVAL, _SHORTEST or _AGED (continuous mode) */
    int32_t reserved;        /* must be 0 */
    double iter_budget_tflop;/* QSIM_POLICY_SHORTEST / _AGED: product work per iteration (e.g. 2.0) */
    double aging_tflop_per_s;/* QSIM_POLICY_AGED: work credit per second of waiting (> 0); ignored otherwise */
} qsim_serve_config;

#define QSIM_REQ_DRIFT_PROBE 1u  /* also compute the probe drift (qsim_unitarity_drift_probe) */
#define QSIM_REQ_DRIFT_FULL 2u   /* instead, the full float64 check (qsim_unitarity_drift): 3 N^3 flops */

typedef struct qsim_request {
    int32_t n_qubits;
    int32_t n_gates;
    const qsim_gate* gates;  /* copied by qsim_submit */
    void* d_psi;             /* out: final state, planar complex64 (2N floats); required */
    const void* d_psi0;      /* initial state (planar complex64) or NULL for |0...0> */
    void* d_U;               /* out: circuit unitary, row-major planar complex64, or NULL (kept in the arena) */
    uint32_t flags;          /* QSIM_REQ_DRIFT_PROBE or QSIM_REQ_DRIFT_FULL (not both), or 0 */
    uint32_t reserved;       /* must be 0 */
} qsim_request;              /* d_psi, d_psi0 and d_U must stay valid until the request is polled done */

typedef struct qsim_result {
    int32_t status;          /* QSIM_PENDING, QSIM_OK, QSIM_E_DEVICE or QSIM_E_CANCELLED */
    int32_t n_steps;
    double norm2;            /* float64 sum |psi_i|^2 */
    double drift_max;        /* probe: max |d_j|; full: max |D_ij| (-1 if not requested) */
    double drift_l2;         /* probe: |d|_2; full: ||D||_F / sqrt(N) (-1 if not requested) */
    uint64_t t_submit_ns;    /* steady clock: submitted, admitted, results observed by the engine */
    uint64_t t_start_ns;
    uint64_t t_done_ns;
} qsim_result;

typedef struct qsim_serve_stats {
    int64_t iterations;        /* engine iterations (FIFO: requests served) */
    int64_t grouped_launches;  /* grouped expansion + product launches */
    int64_t admitted;
    int64_t completed;
    int64_t peak_active;
    uint64_t arena_high_water; /* bytes */
} qsim_serve_stats;

qsim_status qsim_serve_start(qsim_ctx* ctx, const qsim_serve_config* cfg);
/* Serve every admitted request to completion, cancel queued ones and stop the
 * thread.  Results not yet polled are dropped with the engine. */
qsim_status qsim_serve_stop(qsim_ctx* ctx);
/* Validate and copy the request, queue it; *id_out identifies it.
 * QSIM_E_FULL: queue at capacity (retry later); QSIM_E_OOM: the request can
 * never fit the arena. */
qsim_status qsim_submit(qsim_ctx* ctx, const qsim_request* req, uint64_t* id_out);
/* Non-blocking.  QSIM_PENDING while queued or running; QSIM_OK once finished,
 * with *out filled (out->status tells the request's own outcome) and the id
 * released; QSIM_E_UNKNOWN_ID for ids never issued or already collected. */
qsim_status qsim_poll(qsim_ctx* ctx, uint64_t id, qsim_result* out);
qsim_status qsim_serve_get_stats(qsim_ctx* ctx, qsim_serve_stats* out);

/* Kernel timing with HIP events (instrumentation, not part of the method).
 * While enabled, every launch the context makes is bracketed by two events
 * recorded on the launch stream; qsim_profile_read waits for the timed
 * launches and returns per-class launch counts and summed durations.
 * Classes: expansion (stage 4), chain product (stage 5), apply incl. the
 * float64 norm/probabilities (stage 6), unitarity drift, full-state passes.  Enabling resets the
 * totals; use from one host thread at a time. */
#define QSIM_PROFILE_EXPAND 0
#define QSIM_PROFILE_PRODUCT 1
#define QSIM_PROFILE_APPLY 2
#define QSIM_PROFILE_DRIFT 3
#define QSIM_PROFILE_FSV 4
#define QSIM_PROFILE_KINDS 5
typedef struct qsim_kernel_stats {
    int64_t count[QSIM_PROFILE_KINDS];
    double total_ms[QSIM_PROFILE_KINDS];
} qsim_kernel_stats;

qsim_status qsim_profile_enable(qsim_ctx* ctx, int enable);
qsim_status qsim_profile_read(qsim_ctx* ctx, qsim_kernel_stats* out);

/* ---- Full-state-vector simulation (Appendix A, Eq. 12) ------------------------------------
 * The gate-by-gate method that the paper names as the next backend to
 * accelerate (Section 7): each gate updates the pairs of amplitudes whose
 * indices differ in its target bit (only those whose control bit is 1 for a
 * controlled gate), in place, without any 2^n x 2^n operator.  States are
 * planar complex64: 2^n float re values then 2^n float im values (8 * 2^n
 * bytes, 256-byte aligned, caller-owned); up to QSIM_FSV_MAX_QUBITS qubits.
 *
 * The library groups consecutive gates into passes over the state.  A pass
 * names 12 local qubits: qubits 0..low_qubits-1 and n_high others; it holds
 * only gates whose target is local, or that are diagonal (Z, S, T, R, RZ and
 * their controlled forms, which need no local qubit); controls may be any
 * qubit; a SWAP needs both qubits local (it permutes amplitudes exactly); a
 * custom operation needs its whole range local (its matrix is rounded to
 * float32).  Each pass reads and
 * writes the whole state once (16 bytes per amplitude), whatever its gate
 * count.  For n <= 12 one pass holds every gate.  Gate matrices are the
 * float64 ones of the unitary path rounded once to float32; amplitude
 * arithmetic is float32. */
#define QSIM_FSV_MAX_QUBITS 34
#define QSIM_FSV_MAX_HIGH 6
typedef struct qsim_fsv_plan qsim_fsv_plan;
typedef struct qsim_fsv_pass_info {
    int32_t low_qubits;             /* qubits 0..low_qubits-1 are local (0 in a permutation pass) */
    int32_t n_high;                 /* further local qubits, ascending in high[] */
    int32_t high[QSIM_FSV_MAX_HIGH]; /* -1 past n_high */
    int32_t first_op;               /* the pass's gates: order[first_op .. first_op + n_ops) */
    int32_t n_ops;
    int32_t permutation;            /* 1: a pass of pairwise disjoint SWAPs on any qubits, applied as one
                                       permutation of the state (states of more than 12 qubits, when only
                                       SWAPs are ready); 0: a pass over 12 local qubits */
} qsim_fsv_pass_info;

/* Host only (no device, no context): the pass schedule of a gate list.
 * Writes min(capacity, passes) records and *n_passes; QSIM_E_RANGE if
 * capacity > 0 and the schedule needs more records (capacity 0 just counts).
 * A gate must run after every earlier gate that shares a qubit with it unless
 * both are diagonal; within that rule a pass may take gates from further on in
 * the circuit, so passes hold ranges of an execution order rather than of the
 * gate list.  order (NULL, or n_gates entries) receives that order: gate
 * indices, pass by pass, and within a pass in the order its launch applies
 * them (operations on disjoint qubits, and diagonal ones, commute, so the
 * pass is reordered to need fewer register-layout changes; a run of diagonal
 * operations is applied as multiplied-out tables, in any order equal; an
 * operation without a control may run in a scaled form whose scalar factor the
 * pass applies when it stores).  A pass with permutation = 1 applies its
 * SWAPs, pairwise disjoint, as one permutation of the state. */
qsim_status qsim_fsv_schedule(int n_qubits, const qsim_gate* gates, int n_gates, qsim_fsv_pass_info* passes,
                              int capacity, int* n_passes, int32_t* order);
/* Validates the gates, schedules them and uploads the operation table to the
 * context's device (a synchronous copy; the plan owns that memory).  The gate
 * array may be freed on return. */
qsim_status qsim_fsv_plan_create(qsim_ctx* ctx, int n_qubits, const qsim_gate* gates, int n_gates,
                                 qsim_fsv_plan** out);
qsim_status qsim_fsv_plan_info(const qsim_fsv_plan* plan, int* n_qubits, int* n_passes, int* n_ops);
/* Frees the plan; work already enqueued with it must have finished. */
qsim_status qsim_fsv_plan_destroy(qsim_fsv_plan* plan);
/* Applies the plan's circuit to d_psi in place: one launch per pass on
 * `stream`, asynchronous.  A plan may run any number of times, on any stream
 * of its device. */
qsim_status qsim_fsv_run(qsim_ctx* ctx, const qsim_fsv_plan* plan, void* d_psi, void* stream);
/* d_psi <- |basis> (asynchronous). */
qsim_status qsim_fsv_init_basis(qsim_ctx* ctx, int n_qubits, int64_t basis, void* d_psi, void* stream);
/* *h_norm2 <- sum |psi_i|^2 accumulated in float64 in a fixed order (waits
 * for the stream).  Uses the context's scratch: calls on one context must not
 * overlap on different streams. */
qsim_status qsim_fsv_norm2(qsim_ctx* ctx, int n_qubits, const void* d_psi, double* h_norm2, void* stream);
/* Measurement of a full state (the collapsing method, Section 5.2.3), with
 * the rule of qsim_sample: shot k is the smallest index i with
 * u_k * C[N-1] < C[i], C the float64 cumulative sum of |psi_i|^2 (it need
 * not be normalised).  The distribution is not materialised: d_ws
 * (qsim_fsv_sample_workspace_bytes(n) bytes, 256-byte aligned) holds the
 * float64 prefix of the probability mass of consecutive blocks of 1024
 * amplitudes; each shot searches that prefix, then its block.  d_uniform:
 * `shots` float64 values in [0, 1) from the caller; d_out: `shots` int64.
 * Asynchronous.  Within rounding of C (a different summation order than a
 * sequential sum), a shot next to a boundary may take the neighbouring
 * outcome. */
size_t qsim_fsv_sample_workspace_bytes(int n_qubits);
qsim_status qsim_fsv_sample(qsim_ctx* ctx, int n_qubits, const void* d_psi, const double* d_uniform, int shots,
                            int64_t* d_out, void* d_ws, size_t ws_bytes, void* stream);

/* ---- Device peaks (measurement) ----
 * The rooflines are quoted against vendor peaks; these probes measure what one
 * device sustains.  qsim_probe_mfma: the issue rate of one MFMA shape with
 * four independent accumulator chains per wave (no dependency stalls),
 * 2048 workgroups x 256 threads, in TFLOP/s (2 flops per multiply-add):
 *   kind 0 v_mfma_f32_32x32x2f32, 1 v_mfma_f32_32x32x16_bf16,
 *   2 v_mfma_f32_32x32x16_f16, 3 v_mfma_f64_16x16x4f64.
 * random_operands != 0: operands with pseudo-random mantissas (toggling bits,
 * as in dense products; the chip may lower its clock); 0: constant operands.
 * Writes one float per workgroup into the context's scratch; synchronous.
 * qsim_probe_copy: a streaming device copy of `bytes` (a multiple of 64 MiB)
 * from d_src to d_dst (non-overlapping, 256-byte aligned), 16-byte loads and
 * stores, four in flight per thread; *gbs_out = 2 * bytes / time (read +
 * write), mean of 10 copies after one warm-up; synchronous. */
qsim_status qsim_probe_mfma(qsim_ctx* ctx, int kind, int random_operands, double* tflops_out);
qsim_status qsim_probe_copy(qsim_ctx* ctx, const void* d_src, void* d_dst, size_t bytes, double* gbs_out);

#ifdef __cplusplus
}
#endif
#endif /* LIBQSIM_QSIM_H_ */
