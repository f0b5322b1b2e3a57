/*
 * diaq.h — C ABI of libdiaq_hip, an MI355X (gfx950) implementation of the
 * DiaQ state-vector hot path (Chundury, Li, Suh, Mueller: "DiaQ: Efficient
 * State-Vector Quantum Simulation", arXiv:2405.01250).
 *
 * What the library computes
 * -------------------------
 * A quantum gate acting on k <= 3 target qubits (plus up to 3 control
 * qubits) of an n-qubit register is expanded to the 2^n x 2^n time-step
 * unitary I_above (x) Gate (x) I_below (Sec. II-C) and stored in the DiaQ
 * format (Sec. IV): a set of diagonals, each identified by its index
 * dIndex = column - row, each stored compactly with exactly N - |dIndex|
 * entries (N = 2^n).  The state vector is advanced by the DiaQ sparse
 * matrix-vector product (Alg. 2).  Around that sit the DiaQ matrix product
 * used for gate fusion (Alg. 1, Sec. VI), the transpose-by-relabelling of
 * Sec. IV, expectation values, adjoint (reverse-sweep) gradients and
 * batched circuits.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Qubit order is little-endian: qubit q is bit q of an amplitude index,
 *    so a one-qubit gate on q has diagonals at 0 and +-2^q.  (The paper's
 *    "first qubit", H (x) I_8 in its Fig. 2, is qubit n-1 here.)
 *  - Complex numbers are interleaved (re, im).  DIAQ_C128 = two doubles,
 *    DIAQ_C64 = two floats (the float/double option of Sec. V).
 *  - State vectors, scratch vectors and DiaQ values live in device memory
 *    owned by the caller unless stated otherwise; pointers must be 16-byte
 *    aligned (256-byte alignment is recommended, the byte-alignment option
 *    of Sec. V).
 *  - Every call is asynchronous on the context's HIP stream, except the
 *    calls documented as returning host results, which synchronise it.
 *  - Every call returns a diaq_status_t; no C++ exception crosses the ABI.
 *    On error the outputs are left untouched and diaq_last_error() returns
 *    a thread-local message.
 *  - A context is not thread-safe; use one context per host thread/stream.
 */
#ifndef DIAQ_H
#define DIAQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ */
/* Status codes, dtypes, handles                                       */
/* ------------------------------------------------------------------ */

typedef enum diaq_status {
  DIAQ_OK = 0,
  DIAQ_ERR_INVALID_ARGUMENT = 1, /* bad qubit index, NULL pointer, aliasing */
  DIAQ_ERR_NOT_MULTIPLYABLE = 2, /* dimension mismatch (Alg. 1 / Alg. 2 guard) */
  DIAQ_ERR_OUT_OF_MEMORY = 3,    /* device or host allocation failed */
  DIAQ_ERR_DEVICE = 4,           /* a HIP runtime call failed */
  DIAQ_ERR_UNSUPPORTED = 5       /* valid request that the library does not support */
} diaq_status_t;

typedef enum diaq_dtype {
  DIAQ_C64 = 0,  /* complex float, 8 bytes per element */
  DIAQ_C128 = 1  /* complex double, 16 bytes per element */
} diaq_dtype_t;

typedef struct diaq_ctx* diaq_ctx_t; /* device, stream, workspace, tuning */
typedef struct diaq_dia* diaq_dia_t; /* one DiaQ matrix (Sec. IV) */

/* ------------------------------------------------------------------ */
/* Gates                                                               */
/* ------------------------------------------------------------------ */

/* Gate kinds.  c = cos(t/2), s = sin(t/2) for an angle t = params[0].
 * Multi-target matrices index their rows/columns with targets[0] as the
 * least-significant local bit.  Controlled kinds put the control qubits in
 * controls[] and the target(s) in targets[]. */
typedef enum diaq_gate_kind {
  DIAQ_GATE_I = 0,
  DIAQ_GATE_H = 1,      /* (1/sqrt2)[[1,1],[1,-1]] */
  DIAQ_GATE_X = 2,
  DIAQ_GATE_Y = 3,
  DIAQ_GATE_Z = 4,
  DIAQ_GATE_S = 5,      /* diag(1, i) */
  DIAQ_GATE_SDG = 6,    /* diag(1, -i) */
  DIAQ_GATE_T = 7,      /* diag(1, e^{i pi/4}) */
  DIAQ_GATE_TDG = 8,    /* diag(1, e^{-i pi/4}) */
  DIAQ_GATE_SX = 9,     /* (1/2)[[1+i, 1-i],[1-i, 1+i]] */
  DIAQ_GATE_RX = 10,    /* [[c, -is],[-is, c]]                 = exp(-i t X/2) */
  DIAQ_GATE_RY = 11,    /* [[c, -s],[s, c]]                     = exp(-i t Y/2) */
  DIAQ_GATE_RZ = 12,    /* diag(e^{-it/2}, e^{it/2})            = exp(-i t Z/2) */
  DIAQ_GATE_P = 13,     /* diag(1, e^{it}) */
  DIAQ_GATE_U3 = 14,    /* params (theta, phi, lambda):
                           [[c, -e^{i lambda} s],[e^{i phi} s, e^{i(phi+lambda)} c]] */
  DIAQ_GATE_SWAP = 15,  /* 2 targets: exchanges local states 01 and 10 */
  DIAQ_GATE_RXX = 16,   /* 2 targets: exp(-i t X(x)X/2) */
  DIAQ_GATE_RYY = 17,   /* 2 targets: exp(-i t Y(x)Y/2) */
  DIAQ_GATE_RZZ = 18,   /* 2 targets: diag(e^{-it/2}, e^{it/2}, e^{it/2}, e^{-it/2}) */
  DIAQ_GATE_MATRIX = 19 /* k targets: the 2^k x 2^k complex128 row-major
                           matrix at diaq_gate_t.matrix (host memory) */
} diaq_gate_kind_t;

#define DIAQ_MAX_TARGETS 3
#define DIAQ_MAX_CONTROLS 3

/* One gate.  Controlled gates (CX = X with one control, CZ, CP, CCX, CSWAP,
 * controlled rotations) are the base kind plus controls: where every
 * control bit of an amplitude index is 1 the local matrix acts on the
 * targets, elsewhere the identity does.
 *
 * Differentiation: a gate whose kind is a rotation (RX, RY, RZ, P, RXX,
 * RYY, RZZ, controlled or not) may name a gradient slot.  With
 * U = exp(-i a G / 2), a = params[0], the adjoint sweep adds
 * param_scale * dE/da to grad[param_index]; param_scale is the caller's
 * chain factor d a / d theta (for example 2 when a = 2 * gamma). */
typedef struct diaq_gate {
  int32_t kind;                        /* diaq_gate_kind_t */
  int32_t ntargets;                    /* 1..3, must match the kind */
  int32_t ncontrols;                   /* 0..3 */
  int32_t targets[DIAQ_MAX_TARGETS];   /* distinct qubits in [0, n) */
  int32_t controls[DIAQ_MAX_CONTROLS]; /* distinct, disjoint from targets */
  double params[3];                    /* angles in radians, per kind */
  int32_t param_index;                 /* -1: constant gate */
  double param_scale;                  /* chain factor, see above */
  const double* matrix;                /* DIAQ_GATE_MATRIX only, else NULL */
} diaq_gate_t;

/* ------------------------------------------------------------------ */
/* Context                                                             */
/* ------------------------------------------------------------------ */

/* Thread-local text of the last error raised on this host thread. */
const char* diaq_last_error(void);
const char* diaq_status_string(diaq_status_t status);

/* Create a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  The context owns a growing
 * device workspace for expanded diagonals and reduction partials. */
diaq_status_t diaq_create(int32_t device, void* hip_stream, diaq_ctx_t* out);
diaq_status_t diaq_set_stream(diaq_ctx_t ctx, void* hip_stream);
diaq_status_t diaq_synchronize(diaq_ctx_t ctx);
/* Frees the workspace; DiaQ matrices created on the context stay valid. */
diaq_status_t diaq_destroy(diaq_ctx_t ctx);

/* ------------------------------------------------------------------ */
/* DiaQ matrices (Sec. IV)                                              */
/* ------------------------------------------------------------------ */

/* Wrap or allocate a DiaQ matrix of dimension 2^nqubits with `ndiag`
 * diagonals at `offsets` (host, col - row, strictly ascending, each
 * |offset| < 2^nqubits).  The values of diagonal k are packed after those
 * of diagonals 0..k-1 and hold N - |offsets[k]| elements, element t being
 * A[t + max(0,-d), t + max(0,d)] (the compact layout of Sec. IV).
 * `values` is a caller-owned device buffer of that total size, or NULL to
 * let the library allocate one (zero-filled, freed by diaq_dia_free). */
diaq_status_t diaq_dia_create(diaq_ctx_t ctx, int32_t nqubits,
                              diaq_dtype_t dtype, int32_t ndiag,
                              const int64_t* offsets, void* values,
                              diaq_dia_t* out);
/* Shape query.  Any output pointer may be NULL. */
diaq_status_t diaq_dia_info(diaq_dia_t A, int32_t* nqubits, int32_t* ndiag,
                            int32_t* dtype, int64_t* nvalues, void** values);
/* Copy the offsets (ndiag entries) and packing starts (ndiag + 1 entries)
 * to host arrays; either may be NULL. */
diaq_status_t diaq_dia_offsets(diaq_dia_t A, int64_t* offsets,
                               int64_t* starts);
/* Transpose by relabelling (Sec. IV: the diagonal indices change sign and
 * the compact diagonals are reused unchanged).  `out` is a new handle that
 * shares A's values (A must outlive it); conjugate != 0 gives A^dagger. */
diaq_status_t diaq_dia_transpose(diaq_dia_t A, int32_t conjugate,
                                 diaq_dia_t* out);
/* Copy the stored values (diaq_dia_info's nvalues elements, packed in
 * stored order) to `dst`: device memory if dst_on_host == 0, else host
 * memory.  The numpy-to-DiaQ converters of Sec. V go the other way through
 * diaq_dia_create with caller-filled values.  Synchronises the stream. */
diaq_status_t diaq_dia_copy_values(diaq_ctx_t ctx, diaq_dia_t A, void* dst,
                                   int32_t dst_on_host);
/* Release a handle (and the values, if the library allocated them). */
diaq_status_t diaq_dia_free(diaq_dia_t A);

/* ------------------------------------------------------------------ */
/* Gate expansion: the time-step unitary of Sec. II-C in DiaQ form      */
/* ------------------------------------------------------------------ */

/* Host-only query: the diagonal indices the expanded gate occupies (sorted
 * ascending) and the number of stored elements.  The indices are the
 * differences scatter(c) - scatter(r) over the structurally non-zero
 * entries M[r][c] of the gate's local matrix, plus 0 for controlled gates;
 * scatter places local bit j at qubit targets[j] (Sec. II-C; for
 * I_a (x) M (x) I_b this is Alg. 3's dim_b * dIndex).  `offsets` may be
 * NULL; at most 27 entries are written. */
diaq_status_t diaq_from_gate_query(const diaq_gate_t* gate, int32_t nqubits,
                                   int32_t* ndiag, int64_t* offsets,
                                   int64_t* nvalues);
/* Expand `gate` on an n-qubit register into a new DiaQ matrix whose values
 * the library allocates (freed by diaq_dia_free).  Element (i, j) of the
 * expansion is M[loc(i)][loc(j)] when i and j agree outside the targets
 * and all controls of i are 1, the identity's delta(i,j) when a control is
 * 0, and 0 otherwise; loc gathers the target bits. */
diaq_status_t diaq_from_gate(diaq_ctx_t ctx, const diaq_gate_t* gate,
                             int32_t nqubits, diaq_dtype_t dtype,
                             diaq_dia_t* out);

/* Pauli-sum observable H = sum_t coef_t * P_t as a DiaQ matrix.  Term t is
 * X^x Z^z up to the phase i^{popcount(x & z)} (so x = z = bit q is Y_q):
 * xmask[t], zmask[t] are bit masks over qubits, coef[t] a real weight.  Each
 * term occupies the diagonals (i xor x) - i; equal indices are summed. */
diaq_status_t diaq_from_pauli_sum(diaq_ctx_t ctx, int32_t nqubits,
                                  diaq_dtype_t dtype, int32_t nterms,
                                  const uint64_t* xmask, const uint64_t* zmask,
                                  const double* coef, diaq_dia_t* out);

/* ------------------------------------------------------------------ */
/* Kernels                                                              */
/* ------------------------------------------------------------------ */

#define DIAQ_TRANSPOSE 1u /* apply A^T  (indices negated, Sec. IV) */
#define DIAQ_CONJUGATE 2u /* conjugate the stored values */
#define DIAQ_ADJOINT 3u   /* apply A^dagger */

/* DiaQ sparse matrix-vector product (Alg. 2): y <- op(A) x, where op is
 * selected by `flags`.  y is overwritten, not accumulated; x and y are
 * device vectors of 2^n elements of A's dtype and must not overlap
 * (DIAQ_ERR_INVALID_ARGUMENT), except that a matrix whose only diagonal is
 * the principal one may run in place (x == y). */
diaq_status_t diaq_spmv(diaq_ctx_t ctx, diaq_dia_t A, const void* x, void* y,
                        uint32_t flags);

/* DiaQ matrix product (Alg. 1): out <- second * first, i.e. the matrix that
 * applies `first` and then `second`.  Every pair of diagonals (a of first,
 * b of second) contributes to diagonal a + b; contributions to one index
 * are summed in ascending order of a.  Result diagonals whose elements all
 * have |value| <= drop_tol are dropped (drop_tol = 0 drops exact zeros
 * only).  Dimension or dtype mismatch: DIAQ_ERR_NOT_MULTIPLYABLE.  The
 * library allocates the result's values.  Synchronises the stream. */
diaq_status_t diaq_fuse(diaq_ctx_t ctx, diaq_dia_t first, diaq_dia_t second,
                        double drop_tol, diaq_dia_t* out);

/* ------------------------------------------------------------------ */
/* Circuits                                                             */
/* ------------------------------------------------------------------ */

/* Execution plan for diaq_apply_circuit.  A zero-filled plan (or NULL) is
 * the plain path: one expansion and one Alg. 2 product per gate. */
typedef struct diaq_plan {
  int32_t fuse;             /* 1: gate-level fusion (Alg. 1 on the local
                               matrices, diagonal gates absorbed) */
  int32_t max_fused_qubits; /* with fuse: cap on a fused group's qubits,
                               1..3 on the DiaQ plan (non-diagonal qubits),
                               1..5 with kron (groups of 4 or 5 qubits
                               become dense 2^k x 2^k operations); 0 = 2;
                               other values are INVALID_ARGUMENT */
  int32_t kron;             /* 1: Alg. 3 products, no expanded diagonals */
  int32_t rows_per_thread;  /* SpMV rows per lane (0 = tuned default) */
  int32_t block;            /* SpMV workgroup size: 0 or 256 (the kernels are
                               built for 256-lane workgroups; any other
                               value is INVALID_ARGUMENT) */
  int32_t reserved[3];
} diaq_plan_t;

/* state <- U_{end-1} ... U_{begin} state for gates[begin, end) with
 * 0 <= begin <= end <= ngates (a saved state plus a gate index resumes a
 * run).  `state` and `scratch` are distinct device vectors of 2^n
 * elements; scratch contents are clobbered.  Diagonals are expanded into
 * the context workspace, each starting on a 256-byte boundary. */
diaq_status_t diaq_apply_circuit(diaq_ctx_t ctx, const diaq_gate_t* gates,
                                 int64_t ngates, int64_t begin, int64_t end,
                                 int32_t nqubits, diaq_dtype_t dtype,
                                 void* state, void* scratch,
                                 const diaq_plan_t* plan);

/* Circuit graphs.  The launch sequence of one diaq_apply_circuit call over
 * all of `gates` (same plan, same state and scratch pointers, the gate
 * parameters as given now) recorded once into a HIP graph, then replayed
 * with one launch per call: for short circuits on small states, where the
 * host's planning and per-kernel launch cost exceed the kernels' run time.
 * The graph owns its expansion and table workspaces (other calls on the
 * context never touch them) and re-uploads its small tables from pinned
 * host memory on every replay, so replays are independent of whatever ran
 * in between.  Creating the graph runs nothing; each launch applies the
 * circuit once to `state` on the context's stream, like
 * diaq_apply_circuit.  state and scratch must stay allocated while the
 * graph lives.  Errors: INVALID_ARGUMENT as diaq_apply_circuit, or a graph
 * of another device; OUT_OF_MEMORY; DEVICE if recording fails. */
typedef struct diaq_graph* diaq_graph_t;
diaq_status_t diaq_circuit_graph_create(diaq_ctx_t ctx, const diaq_gate_t* gates,
                                        int64_t ngates, int32_t nqubits,
                                        diaq_dtype_t dtype, void* state,
                                        void* scratch, const diaq_plan_t* plan,
                                        diaq_graph_t* out);
diaq_status_t diaq_circuit_graph_launch(diaq_ctx_t ctx, diaq_graph_t graph);
/* Number of nodes (kernels and copies) in the recorded graph. */
diaq_status_t diaq_circuit_graph_nodes(diaq_graph_t graph, int64_t* nodes);
/* Waits for the device, then releases the graph and its workspaces. */
diaq_status_t diaq_circuit_graph_free(diaq_graph_t graph);

/* Device-to-device copy of `bytes` from src to dst (device pointers, both
 * 16-byte aligned, bytes a multiple of 16, no overlap) by a streaming
 * kernel on the context's stream: the drivers' own state copies, exported
 * as the plain-copy reference of bandwidth measurements.  Errors:
 * INVALID_ARGUMENT for NULL, misaligned or overlapping buffers. */
diaq_status_t diaq_copy(diaq_ctx_t ctx, const void* src, void* dst, size_t bytes);

/* Host-only: the number of expansion + product launches (operations)
 * diaq_apply_circuit issues for `gates` under `plan`, and the algorithmic
 * bytes they move (expansion writes plus product reads and writes, the
 * sum over operations of s * (2E + 2N)).  Either output may be NULL. */
diaq_status_t diaq_plan_count(const diaq_gate_t* gates, int64_t ngates,
                              int32_t nqubits, diaq_dtype_t dtype,
                              const diaq_plan_t* plan, int64_t* nops,
                              double* bytes);

/* Expectation value <psi|H|phi> (phi = NULL means phi = psi) written to
 * out[0] (real part) and out[1] (imaginary part), host memory.  The sum is
 * reduced in a fixed order, so repeated calls are bitwise equal.
 * Synchronises the stream. */
diaq_status_t diaq_expect(diaq_ctx_t ctx, diaq_dia_t H, const void* psi,
                          const void* phi, double* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * expectation value of diaq_expect, same kernels and summation order, with
 * no allocation, no free and no synchronisation.  The result (real part,
 * imaginary part) is written to dres, caller-owned device memory of two
 * doubles, asynchronously on the context's stream.  psi, phi (NULL: psi)
 * and dres are 16-byte aligned.  The per-workgroup partial sums live in a
 * static device array of 2^20 entries (16 MiB) that each device the
 * library runs on holds until the process ends; a matrix whose product
 * needs more partials than that (more than 2^28 rows at the default one row
 * per lane) returns DIAQ_ERR_UNSUPPORTED before anything is launched.
 * Every partial is written before it is read, so nothing carries over from
 * an earlier call, but all calls on one device share the array: calls that
 * overlap in time (other streams, other contexts, other host threads) race
 * and must be serialised by the caller. */
diaq_status_t diaq_expect_noalloc(diaq_ctx_t ctx, diaq_dia_t H, const void* psi,
                                  const void* phi, double* dres);

/* Adjoint gradient of E(theta) = <psi|H|psi>, psi = U_G...U_1 psi0.
 * Forward pass, lambda = H psi, then a reverse sweep that for g = G..1
 * adds param_scale * Im<lambda|G_g|psi> to grad[param_index] of every
 * differentiable gate and steps psi and lambda back through U_g^dagger (the
 * conjugate-transposed DiaQ matrix of the same expansion).  `work` holds
 * 3 * 2^n elements of device memory.  Writes *expval and grad[0..nparams)
 * (host, zeroed first).  plan == NULL (or kron == 0): every gate and every
 * U^dagger is expanded and applied by Alg. 2; plan->kron: the forward pass
 * runs fused Alg. 3 operations in place (max_fused_qubits, default 4) and
 * the reverse sweep is cut into segments of consecutive gates whose
 * non-diagonal targets fit in 3 qubits, each segment one pass over psi and
 * lambda replaying its gates per coset in exact reverse order (dots taken
 * before each gate is undone; n < 3 falls back to one pass per gate).
 * Synchronises the stream. */
diaq_status_t diaq_adjoint_grad(diaq_ctx_t ctx, const diaq_gate_t* gates,
                                int64_t ngates, int32_t nqubits,
                                diaq_dtype_t dtype, diaq_dia_t H,
                                const void* psi0, void* work,
                                int64_t nparams, double* expval,
                                double* grad, const diaq_plan_t* plan);

/* ------------------------------------------------------------------ */
/* Batched circuits: one persistent launch, optionally a captured graph  */
/* ------------------------------------------------------------------ */

/* One circuit of a batch.  It starts from |0...0>; every gate acts on at
 * most 2 targets plus at most 2 controls.  The observable is diagonal:
 * H = sum_t coef[t] * Z^{zmask[t]} (zmask = 0 is the identity term), as
 * for MaxCut-type cost functions.  A differentiable gate (param_index >= 0)
 * takes the angle param_scale * theta[param_index] when diaq_batch_run is
 * given theta, else params[0]; gradients are per circuit, nparams each. */
typedef struct diaq_circuit {
  int32_t nqubits;  /* 1..30 */
  int32_t nparams;
  int64_t ngates;
  const diaq_gate_t* gates; /* host */
  int32_t nterms;
  int32_t reserved;
  const uint64_t* zmask;    /* host, nterms */
  const double* coef;       /* host, nterms */
} diaq_circuit_t;

typedef struct diaq_batch* diaq_batch_t;

#define DIAQ_BATCH_GRAPH 1u /* capture upload + kernel + download in a
                               hipGraph once and replay it on every run */

/* Upload a batch: gate tables, observables and per-circuit state vectors
 * (two of 2^n elements per circuit, complex128) are placed in device memory
 * owned by the handle. */
diaq_status_t diaq_batch_create(diaq_ctx_t ctx, const diaq_circuit_t* circuits,
                                int32_t ncircuits, uint32_t flags,
                                diaq_batch_t* out);
/* Run every circuit of the batch in one persistent launch: forward pass,
 * E_c = <psi_c|H_c|psi_c>, and the adjoint reverse sweep for dE_c/dtheta.
 * theta (host, sum of nparams entries, circuit-major) may be NULL.
 * Writes expvals[ncircuits] and grads[sum nparams] (host).  Workgroups
 * take whole circuits from a device queue in decreasing order of work; a
 * circuit of at most 12 qubits keeps both of its vectors in LDS.
 * Synchronises the stream. */
diaq_status_t diaq_batch_run(diaq_batch_t batch, const double* theta,
                             double* expvals, double* grads);
diaq_status_t diaq_batch_free(diaq_batch_t batch);

/* ------------------------------------------------------------------ */
/* Tuning knobs of the product kernel (set by the autotuner)            */
/* ------------------------------------------------------------------ */

/* Zero in any field selects the built-in default. */
typedef struct diaq_tuning {
  int32_t spmv_rows;       /* rows per lane in one tile: 1, 2 or 4 */
  int32_t spmv_group_bits; /* how many high coupling qubits a workgroup
                              pairs its tiles over: 1..3, or -1 for none */
  int32_t spmv_chunk;      /* diagonals whose loads are issued together:
                              1 or 3 */
  int32_t spmv_nontemporal;/* 1: stream diagonal values and y with
                              non-temporal hints; -1: plain accesses */
  int32_t spmv_group_min_qubit; /* only qubits >= this are paired (their
                              partner rows are too far apart in launch
                              order to meet in the caches) */
  int32_t expand_nontemporal; /* 1: write expanded diagonals with
                              non-temporal hints; -1: plain stores;
                              0: hints for complex64 only (measured the
                              faster choice for each type) */
  int32_t diag_pad;        /* elements of padding between the expanded
                              diagonals in the circuit workspace (-1: none) */
  int32_t spmv_xcd_runs;   /* 0: XCD-aware tile order (each XCD has its own
                              L2): products whose diagonals couple tiles 1,
                              2 or 4 apart hand each XCD runs of consecutive
                              tiles, and unpaired products on one coupling
                              qubit whose partner rows lie >= 16 MiB apart
                              alternate partner tiles on each XCD;
                              -1: plain launch order */
  uint64_t spmv_group_qubits; /* when non-zero, bit q says whether tiles are
                              paired across coupling qubit q (a per-qubit
                              choice that replaces spmv_group_min_qubit) */
  /* Alg. 3 (plan.kron) kernels */
  int32_t kron_stage_qubit; /* an operation of at most four qubits whose lowest
                              qubit is below this is staged through LDS
                              (0: default 3; -1: never) */
  int32_t kron_split;      /* dense groups of four and five qubits: 0 default,
                              1 one lane per coset (2^k amplitudes in
                              registers), 2 the rows of 64 cosets split over
                              the waves of a block, 8 rows per wave (inputs
                              streamed from LDS), 3 the same with 4 rows per
                              wave, 4 fp64 matrix-core products of 16 cosets
                              at a time (groups whose qubits are all >= 4;
                              others take the default), the matrix re-read
                              from LDS for every tile, 5 the same with the
                              matrix held in registers, 6 rows split as in 2
                              with five-qubit products formed from three
                              real multiplications per complex one, 7
                              products of 16 cosets at a time on the matrix
                              cores with each wave's next inputs loaded
                              during its products, in the state's precision
                              (complex64: fp32 operands and sums; groups
                              whose qubits are all >= 4, others take the
                              default).  The default uses 7 for such groups
                              of five qubits, and of four in complex64. */
  int32_t kron_nontemporal;/* per-coset Alg. 3 kernel state streams: 0 default,
                              1 non-temporal hints, -1 plain accesses */
  int32_t kron_small_qubits; /* plan.kron on at most this many qubits runs
                              the whole circuit in LDS, one launch per run of
                              gates whose matrices fit the kernel arguments
                              (0: default, as many qubits as the state fits
                              in LDS, held as complex128 either way: 13 on
                              160 KiB; -1: never) */
  int32_t kron_order;      /* order in which the workgroups of the Alg. 3
                              kernels take their blocks of cosets: 0 default
                              (per-coset kernel: XCD eighths for operations
                              that rewrite every row, else launch order;
                              staged and row-split group kernels: halves
                              interleaved), 1 each XCD a contiguous eighth,
                              2 the two halves interleaved, 3 blocks
                              scattered by an odd multiplier */
  int32_t spmv_order;      /* tile order of the product kernel where neither
                              XCD runs nor partner alternation apply: 0 launch
                              order, 1 each XCD a contiguous eighth of the
                              tiles, 2 the two halves interleaved */
  int32_t spmv_pack;       /* complex64 amplitudes in pairs, 16-byte units:
                              DiaQ products whose offsets and diagonal starts
                              are all even (no coupling on qubit 0), and the
                              per-coset and diagonal Alg. 3 kernels of gates
                              that neither act on nor are controlled by
                              qubit 0 (two cosets per lane); 0 default (on),
                              -1 never */
} diaq_tuning_t;

diaq_status_t diaq_set_tuning(diaq_ctx_t ctx, const diaq_tuning_t* t);
diaq_status_t diaq_get_tuning(diaq_ctx_t ctx, diaq_tuning_t* t);

/* Launch shape of the Alg. 2 product kernel for one expanded gate, as
 * diaq_spmv and diaq_apply_circuit (plain plan) choose it under the knobs
 * *t (NULL: built-in defaults).  Host-only: no device call, no context.
 * Gates whose expansion holds only the principal diagonal run the in-place
 * kernel (in_place = 1, the other fields describe one row per lane).
 * Returns INVALID_ARGUMENT for an invalid gate or knob set. */
typedef struct diaq_spmv_shape {
  int32_t in_place;        /* 1: principal diagonal only, updated in place */
  int32_t rows_per_lane;   /* rows a lane owns in each tile: 1, 2 or 4 */
  int32_t group;           /* tiles one workgroup owns: 1, 2, 4 or 8 */
  int32_t chunk;           /* diagonals whose loads are issued together: 1 or 3 */
  int32_t nontemporal;     /* 1: value and y streams carry non-temporal hints */
  int32_t tile_log2;       /* log2(rows of one tile) */
  int32_t group_qubits[3]; /* coupling qubits the tiles of a workgroup differ
                              in, ascending; -1 where unused */
  int32_t xcd_run_log2;    /* > 0: each XCD takes runs of 2^xcd_run_log2
                              consecutive tiles */
  int32_t pair_bit;        /* > 0: each XCD alternates between tiles that
                              differ in this tile-index bit */
  int32_t tile_order;      /* otherwise: 0 launch order, 1 XCD-contiguous
                              eighths, 2 halves interleaved */
  int64_t blocks;          /* workgroups of the launch */
  int32_t packed;          /* 1: complex64 amplitudes taken in pairs (16-byte
                              units; rows_per_lane then counts units, and
                              tile_log2 and group_qubits are in amplitudes) */
  int32_t reserved;
} diaq_spmv_shape_t;
diaq_status_t diaq_spmv_shape(const diaq_gate_t* gate, int32_t nqubits, diaq_dtype_t dtype,
                              const diaq_tuning_t* t, diaq_spmv_shape_t* out);

/* ------------------------------------------------------------------ */
/* Autotuning                                                           */
/* ------------------------------------------------------------------ */

/* Pick the product kernel's knobs for 2^nqubits-element vectors: time the
 * DiaQ SpMV of expanded one-qubit gates on qubits spread over the register
 * (and a CX) under every candidate tuning, keep the fastest, then decide
 * tile pairing qubit by qubit (a U3 on each qubit from the tile size up,
 * timed paired and unpaired), install the result in the context and write
 * it to *out.  With cache_path (a JSON file) the
 * result is stored under a key naming the device, n and dtype, and a
 * later call with the same key reads it back without timing.  Allocates
 * and frees its own test vectors.  Synchronises the stream. */
diaq_status_t diaq_autotune(diaq_ctx_t ctx, int32_t nqubits, diaq_dtype_t dtype,
                            const char* cache_path, diaq_tuning_t* out);

/* Choose a plan (fusion depth 1..3 on expanded DiaQ products or, when
 * allow_kron != 0, also Alg. 3 in-place products with groups of 1..5
 * qubits) for one circuit: candidates are ranked by a byte model
 * (diaq_plan_count, weighted by nominal product rates) and skipped when
 * their largest expanded operation would not fit in free device memory;
 * the best `measure` candidates are then timed on the circuit's first
 * quarter (at least 64 gates, all of a shorter circuit) on scratch
 * vectors, and the fastest wins.  Synchronises the stream. */
diaq_status_t diaq_autotune_plan(diaq_ctx_t ctx, const diaq_gate_t* gates,
                                 int64_t ngates, int32_t nqubits,
                                 diaq_dtype_t dtype, int32_t allow_kron,
                                 int32_t measure, diaq_plan_t* out);

/* ------------------------------------------------------------------ */
/* Matrix-level simulation (Sec. II-A): unitary simulation and          */
/* density-matrix evolution, on DiaQ matrices through the Alg. 1 product */
/* ------------------------------------------------------------------ */

/* Per-gate record of a chained product, the quantities behind the
 * sparsity and diagonal-count curves of Sec. III-A. */
typedef struct diaq_chain_step {
  int32_t ndiag;    /* stored diagonals after this time step */
  int32_t reserved;
  int64_t nnz;      /* stored elements with |v| > drop_tol (v != 0 if 0) */
  int64_t nvalues;  /* stored elements: the DiaQ footprint in elements */
} diaq_chain_step_t;

/* Number of stored elements of A (its applied view's values) with
 * |v| > tol, or v != 0 when tol = 0 (Sec. III-A sparsity = 1 - nnz / 4^n).
 * Synchronises the stream.  tol < 0: DIAQ_ERR_INVALID_ARGUMENT. */
diaq_status_t diaq_dia_nnz(diaq_ctx_t ctx, diaq_dia_t A, double tol, int64_t* nnz);

/* out[0] + i out[1] = Tr(A B) = sum_d sum_i A[i, i+d] B[i+d, i], pairing A's
 * diagonal d with B's diagonal -d (either operand may be a transposed or
 * conjugated view).  Gives Tr(H rho) and the purity Tr(rho^2).  Summed per
 * workgroup, then in a fixed order: repeat calls are bitwise equal.
 * Dimension or dtype mismatch: DIAQ_ERR_NOT_MULTIPLYABLE.  Synchronises. */
diaq_status_t diaq_trace_product(diaq_ctx_t ctx, diaq_dia_t A, diaq_dia_t B, double* out);

/* Unitary simulation (Sec. II-A; Sec. III-A tracks its sparsity): the
 * circuit's 2^n x 2^n unitary U = G_{ngates-1} ... G_0 * start, each G_t
 * the expanded time-step matrix of gate t (Sec. II-C), multiplied in by
 * Alg. 1 (diaq_fuse) one gate at a time.  start = NULL starts from the
 * identity; start is not modified.  After each gate, diagonals whose values
 * all have |v| <= drop_tol are dropped and, if steps != NULL, steps[t]
 * receives the diagonal count and non-zeros.  The library allocates *out
 * (free with diaq_dia_free).  n outside [1, 15]: DIAQ_ERR_UNSUPPORTED (the
 * product can hold up to 2^(n+1) - 1 diagonals).  Invalid gate: the
 * diaq_from_gate error, with nothing allocated.  Synchronises. */
diaq_status_t diaq_unitary(diaq_ctx_t ctx, const diaq_gate_t* gates, int64_t ngates, int32_t nqubits,
                           diaq_dtype_t dtype, diaq_dia_t start, double drop_tol, diaq_chain_step_t* steps,
                           diaq_dia_t* out);

/* Density-matrix evolution (Sec. II-A): rho <- G_t rho G_t^dagger for each
 * gate in order, as two Alg. 1 products per gate, the right factor being
 * G_t's transposed, conjugated view (a relabelling, Sec. IV).  rho is any
 * DiaQ matrix of n <= 15 qubits (typically Hermitian, unit trace) and is
 * not modified; *out is allocated by the library.  drop_tol and steps as
 * for diaq_unitary.  Synchronises. */
diaq_status_t diaq_density_evolve(diaq_ctx_t ctx, const diaq_gate_t* gates, int64_t ngates, diaq_dia_t rho,
                                  double drop_tol, diaq_chain_step_t* steps, diaq_dia_t* out);

/* ------------------------------------------------------------------ */
/* Kernel timing (the counterpart of the simulator trace timer the paper
 * reads its times from, Sec. VII)                                      */
/* ------------------------------------------------------------------ */

/* Totals over the launches issued by diaq_apply_circuit between start and
 * stop, timed with HIP events recorded on the context's stream around each
 * kernel.  Bytes are algorithmic: an expansion writes E stored elements; a
 * product reads E stored elements and one vector and writes one vector
 * (E + 2N elements), whatever the caches do. */
typedef struct diaq_profile {
  int64_t expand_launches;
  double expand_ms;
  double expand_bytes;
  int64_t spmv_launches;
  double spmv_ms;
  double spmv_bytes;
} diaq_profile_t;

diaq_status_t diaq_profile_start(diaq_ctx_t ctx);
/* Synchronises the stream, fills *out, and stops recording. */
diaq_status_t diaq_profile_stop(diaq_ctx_t ctx, diaq_profile_t* out);

#ifdef __cplusplus
}
#endif

#endif /* DIAQ_H */
