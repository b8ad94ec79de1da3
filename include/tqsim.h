/*
 * tqsim.h -- C ABI of an MI355X (gfx950) library for tree-based noisy
 * quantum-circuit simulation by Monte Carlo Pauli trajectories, after
 * "Accelerating Simulation of Quantum Circuits under Noise via
 * Computational Reuse" (Wang, Tannu, Nair; arXiv 2203.13892).
 *
 * The problem statement follows the paper: a circuit and a noise model go in
 * (Sec. 2.4 and Sec. 4.3: noise operators are inserted into the circuit,
 * the depolarizing channel being the main model), together with the shot
 * count and the tree shape (Sec. 3.1: a tree (A_0, .., A_{k-1}) over k
 * consecutive subcircuits; Sec. 3.2: Dynamic Circuit Partition chooses it);
 * one measured outcome per leaf comes out (Sec. 2.2 and Sec. 3.1: the tree
 * yields prod A_j outcomes).
 *
 * Conventions used by every call:
 *   - Bit q of a basis index is qubit q (little-endian).
 *   - A gate on qubits (q_0, .., q_{a-1}), a in {1, 2}, carries a
 *     (2^a x 2^a) complex matrix, row-major, interleaved (re, im) doubles;
 *     local index bit j of the matrix is qubit q_j.
 *   - Pauli probabilities of a gate are 4^a doubles indexed by
 *     code = sum_j c_j 4^j with c_j in {0: I, 1: X, 2: Y, 3: Z} acting on
 *     q_j; entry 0 is the identity.  The drawn operator acts right after its
 *     gate, on that gate's qubits.
 *   - The tree has `levels` subcircuits; cut[0] = 0 < cut[1] < .. <
 *     cut[levels] = number of gates; subcircuit l is gates
 *     [cut[l], cut[l+1]).  Level l has I_l = A_0 * .. * A_l instances; node
 *     (l, m) is a child of (l-1, m / A_l); global node ids run level by
 *     level.  Leaf lambda is node (levels-1, lambda).  The per-shot form is
 *     levels = 1, arity = {N}.
 *   - Noise sampling: SplitMix64 (Steele, Lea, Flood 2014).  Node nu's
 *     stream under seed s is SplitMix64 started at state s + nu * 2^32 *
 *     0x9E3779B97F4A7C15; a draw z becomes (z >> 11) * 2^-53.  In gate order
 *     each gate takes one uniform u1; when u1 < p_g (p_g = sum of the
 *     non-identity probabilities in code order) a second uniform u2 selects
 *     the first code whose running probability sum exceeds u2 * p_g.  A leaf
 *     then takes one more uniform: its measurement uniform u.
 *   - Measurement: outcome = min { x : sum_{y <= x} |psi_y|^2 > u * T } with
 *     T = sum_x |psi_x|^2, accumulated in FP64 in index order (largest x with
 *     nonzero probability if rounding leaves no such x).
 *
 * Ownership: every input array is copied during the call.  Opaque objects
 * belong to the caller until their *_destroy (NULL is accepted).  Device
 * memory is never allocated by the library: the caller passes a device
 * workspace (for example a torch uint8 tensor) of at least the size that
 * tqs_workspace_bytes reports, and a HIP stream (NULL = the null stream).
 *
 * Threads: calls on different objects may run concurrently.  Runs that use
 * the same plan or batch must not overlap (a run keeps its timing events in
 * the plan or batch), and runs that share a workspace must be ordered on
 * the device (same stream, or synchronised) since each run owns the whole
 * workspace until it returns.
 *
 * Errors: every call returns a tqs_status; a negative value means failure,
 * and tqs_last_error() gives a message for the calling thread.  No call
 * aborts or throws across this boundary.
 */
#ifndef TQSIM_H
#define TQSIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TQS_OK = 0,
    TQS_E_ARG = -1,         /* bad argument (NULL, out of range, not unitary) */
    TQS_E_SHAPE = -2,       /* tree shape or cuts invalid */
    TQS_E_WORKSPACE = -3,   /* workspace too small or misaligned */
    TQS_E_HIP = -4,         /* HIP runtime error (message carries its text) */
    TQS_E_OOM = -5,         /* host allocation failed */
    TQS_E_UNSUPPORTED = -6  /* valid request outside what the library supports */
} tqs_status;

typedef enum { TQS_C64 = 0, TQS_C128 = 1 } tqs_precision;

typedef struct tqs_circuit tqs_circuit;
typedef struct tqs_noise tqs_noise;
typedef struct tqs_plan tqs_plan;

/* Tree shape (Sec. 3.1).  arity[levels], cut[levels + 1]. */
typedef struct {
    uint32_t levels;
    const uint64_t *arity;
    const uint32_t *cut;
} tqs_tree;

/* Planner and executor knobs; zero fields take the defaults. */
typedef struct {
    uint32_t tile_qubits;      /* qubits per one-wave tile: 6 lane + register qubits
                                  (10..12 at complex64, default 11; 10..11 at complex128,
                                  default 10) */
    uint32_t max_ops_per_pass; /* gates applied per HBM pass (default 1024) */
    uint32_t chunk_states;     /* live states per tree level (default: as many as fill
                                  8 GiB, between 1 and 1024) */
    uint32_t sample_block_log; /* log2 amplitudes per sampling block (default 12) */
    uint32_t pass_cost;        /* estimated lane instructions per amplitude allowed in one
                                  pass before a new pass starts (default 480) */
    uint32_t no_merge;         /* 1: compute every node's state.  Default 0: nodes of one
                                  chunk whose parents share a state and whose frames and
                                  noise events are equal share one state (Sec. 6,
                                  inter-shot redundancy; most often siblings without an
                                  event), each leaf still sampled with its own draw */
    uint32_t separate_sampling; /* 1: sampling reads the final states in kernels of its own.
                                  Default 0: the last pass of the leaf level also writes
                                  the FP64 sampling partial sums when its tile allows */
    uint32_t jit;              /* pass kernels specialised to the plan (its ops fixed at compile
                                  time, compiled with hipRTC on the plan's first run and kept
                                  with the plan): 1 on, 2 off.  Default 0: on for states of
                                  2^16 amplitudes or more.  Same results either way; nodes a
                                  specialised kernel does not take run in the generic one */
    uint32_t mfma_min_ops;     /* specialised complex64 kernels with full 11-qubit tiles: runs
                                  of at least this many consecutive dense ops on the five
                                  register qubits become one 32x32 unitary (FP64 product, cast
                                  once) applied on the matrix cores (MFMA).  0: the default
                                  (6: the block costs about as much as five two-qubit gates
                                  on the vector units); 1000 or more: off.  Nodes with a noise
                                  event between the ops of such a run go to the generic
                                  kernel */
    uint32_t lds_levels;       /* generic complex64 kernels (tiles of at most five register
                                  qubits), tree levels of two or more passes whose state fits
                                  one workgroup's LDS (up to 2^14 amplitudes, at most eight
                                  tiles): all passes of the level in one launch, one workgroup
                                  per state, the state kept in LDS between passes.  1 on, 2 off;
                                  default 0: off (such states stay in the device's caches between
                                  passes anyway, and the LDS cuts occupancy).  Amplitudes agree
                                  to rounding with the pass-by-pass form */
    uint32_t level_exchange;   /* lane exchanges at the end of a tree level: when the qubits
                                  the next level's gates change do not fit the lanes plus the
                                  register slots of one tile, the last pass of a level ends
                                  with exchanges that put them in reach, so the next level
                                  may need fewer passes, while the later levels' layout
                                  changes too, which can make their passes slower.  1 on,
                                  2 off; default 0: the tree is planned both ways and the
                                  exchanges are kept when they save at least a tenth of the
                                  passes weighted by their levels' node counts.  Same results
                                  either way */
} tqs_tuning;

/* Timing and traffic of one run. */
typedef struct {
    double ms_wall;            /* host wall time of the call */
    double ms_device;          /* device time from upload to outcomes (HIP events) */
    double ms_passes;          /* device time of the gate-apply passes */
    double ms_sample;          /* device time of the sampling kernels */
    uint64_t launches;         /* kernels launched */
    uint64_t pass_launches;    /* of which gate-apply passes */
    uint64_t pass_states;      /* sum over pass launches of states processed */
    uint64_t bytes_passes;     /* algorithmic HBM bytes of the passes (read + write, with the
                                  sampling partials the last leaf pass writes) */
    uint64_t bytes_sample;     /* algorithmic HBM bytes of sampling */
    uint64_t events;           /* noise events in the insertion list */
    uint64_t nodes_merged;     /* nodes whose state is an identical earlier node's */
    uint64_t jit_launches;     /* pass launches of plan-specialised kernels */
    uint64_t jit_states;       /* states those launches processed */
    uint64_t bytes_jit;        /* their algorithmic HBM bytes (as bytes_passes) */
    double ms_jit;             /* their device time (HIP events around each such launch) */
} tqs_run_stats;

/* ---------------------------------------------------------------- circuit */

/* New empty circuit on n_qubits (1..30). */
tqs_status tqs_circuit_create(uint32_t n_qubits, tqs_circuit **out);

/* Append a gate (Sec. 2.1: circuits are ordered gates).  `qubits` has
 * `arity` distinct entries < n; `mat` is (2^arity)^2 interleaved complex
 * doubles and must be unitary to 1e-9; `pauli` is NULL (noiseless) or 4^arity
 * non-negative probabilities summing to 1 within 1e-9 (Sec. 2.4: noise
 * operators drawn after the gate). */
tqs_status tqs_circuit_add_gate(tqs_circuit *c, uint32_t arity, const uint32_t *qubits,
                                const double *mat, const double *pauli);

/* Set the depolarizing channel on every gate (Sec. 4.3, depolarizing channel
 * built from X, Y, Z): total non-identity probability p1 for one-qubit and
 * p2 for two-qubit gates, spread evenly over the 3 or 15 non-identity
 * Paulis.  Replaces any per-gate probabilities. */
tqs_status tqs_circuit_set_depolarizing(tqs_circuit *c, double p1, double p2);

/* Read-out channel (Sec. 4.3, read-out: a measured bit flips with a given
 * probability): p_flip[n_qubits] in [0, 1], bit q of every outcome flips
 * independently with probability p_flip[q] after the measurement.  NULL
 * removes it.  The flips are drawn with the insertion list (tqs_noise_sample)
 * and do not change any state. */
tqs_status tqs_circuit_set_readout(tqs_circuit *c, const double *p_flip);

/* Number of qubits and gates. */
tqs_status tqs_circuit_info(const tqs_circuit *c, uint32_t *n_qubits, uint32_t *n_gates);

void tqs_circuit_destroy(tqs_circuit *c);

/* -------------------------------------------------------------- tree shape */

/* Dynamic Circuit Partition (Sec. 3.2).  The first subcircuit has
 * max(1, ceil(copy_cost)) gates (the shortest that amortises one state copy,
 * Sec. 3.2.2 and Sec. 3.6); its error rate is 1 - prod(1 - e_i) with e_i the
 * gates' non-identity probabilities (Sec. 3.2.3); A0_min is the ceiling of
 * the sample-size bound z^2 p(1-p)/eps^2 / (1 + z^2 p(1-p)/(eps^2 N)); k is
 * the most further subcircuits with A_r = floor((N/A0_min)^(1/k)) >= 2,
 * capped by floor((G - L0)/max(1, copy_cost)) and by max_levels - 1; A_0 is
 * raised to ceil(N / A_r^k) so that the tree has at least N leaves; the
 * remaining gates are split into k equal parts, larger parts first
 * (Sec. 3.2.4).  A result with *levels == 1 is the per-shot form.
 * arity and cut must hold max_levels and max_levels + 1 entries. */
tqs_status tqs_dcp(const tqs_circuit *c, uint64_t shots, double z, double eps,
                   double copy_cost, uint32_t max_levels, uint32_t *levels,
                   uint64_t *arity, uint32_t *cut);

/* ------------------------------------------------------------------- noise */

/* Sample the noise insertion list of every tree node plus one measurement
 * uniform per leaf (Sec. 2.4 and Sec. 3.1; generator in the header
 * comment).  With a read-out channel each leaf then takes n_qubits more
 * uniforms v_q and its flip mask has bit q set when v_q < p_flip[q].
 * Host only. */
tqs_status tqs_noise_sample(const tqs_circuit *c, const tqs_tree *tree, uint64_t seed,
                            tqs_noise **out);

/* Build an insertion list from explicit data: node_off[n_nodes + 1] (CSR
 * over global node ids), ev_gate / ev_code[node_off[n_nodes]] (gate index
 * inside the node's subcircuit range, non-zero Pauli code; sorted by gate
 * within a node, one event per gate at most), leaf_u[n_leaves] in [0, 1). */
tqs_status tqs_noise_import(const tqs_circuit *c, const tqs_tree *tree,
                            const uint64_t *node_off, const uint32_t *ev_gate,
                            const uint8_t *ev_code, const double *leaf_u, tqs_noise **out);

/* Borrowed views of an insertion list; valid until tqs_noise_destroy. */
tqs_status tqs_noise_view(const tqs_noise *nz, const uint64_t **node_off,
                          const uint32_t **ev_gate, const uint8_t **ev_code,
                          const double **leaf_u, uint64_t *n_nodes, uint64_t *n_leaves);

/* Set explicit read-out flip masks, leaf_flip[n_leaves] (copied; bit q
 * flips qubit q's measured bit), or remove them with NULL.  A run refuses
 * masks with bits at or above the plan's qubit count (TQS_E_ARG). */
tqs_status tqs_noise_set_flips(tqs_noise *nz, const uint32_t *leaf_flip);

/* Borrowed view of the flip masks: *leaf_flip = NULL when there are none. */
tqs_status tqs_noise_flips(const tqs_noise *nz, const uint32_t **leaf_flip);

void tqs_noise_destroy(tqs_noise *nz);

/* -------------------------------------------------------------------- plan */

/* Plan a circuit under a tree shape: gates are grouped into HBM passes
 * (tiles of staged qubits), matrices cast once to the run precision.
 * tuning may be NULL.  Host only. */
tqs_status tqs_plan_create(const tqs_circuit *c, const tqs_tree *tree, tqs_precision prec,
                           const tqs_tuning *tuning, tqs_plan **out);

/* Number of HBM passes of subcircuit `level` and in total. */
tqs_status tqs_plan_info(const tqs_plan *p, uint32_t level, uint32_t *passes_level,
                         uint32_t *passes_total, uint32_t *chunk_states);

/* Device workspace bytes that tqs_run needs for this plan and insertion
 * list, exactly (host work over the list's nodes and events); nz may be
 * NULL for a bound valid for any list of this tree with at most one event
 * per gate of each node. */
tqs_status tqs_workspace_bytes(const tqs_plan *p, const tqs_noise *nz, uint64_t *bytes);

/* Text description of the plan, for tests and analysis (no device work).
 * Writes at most cap bytes, NUL-terminated, into buf (may be NULL) and the
 * full size including the NUL into *len.  Lines:
 *   plan <n> <passes> <gates> <levels>
 *   layout <physical position of logical qubit 0> ... (after the last level)
 *   gate <g> <pass> <slot after it> <arity> <phys q0> <phys q1>   (positions
 *        when the gate runs; a noise event of gate g acts there)
 *   level <l> <first pass> <pass count>
 *   pass <p> <op count> regs <register positions...>
 *   dense <arity> <phys q0> <phys q1> <slot0> <slot1> | <row-major matrix, re im ...>
 *   diag <slot0> <slot1> | <arity> <phys q0> <phys q1> <diagonal, re im ...> | ...
 *   block <pass> <first op> <end op>   (global op indices fused into one 32x32 unitary
 *        that the specialised kernel applies on the matrix cores; tuning.mfma_min_ops)
 *   sampling <tiled> <pattern bits> <tile bits> <in-block tile bits> <summed bits> | <source
 *        of each block-index bit: 128 + pattern bit, or tile bit>  (tiled = 1: the last
 *        leaf pass writes per-tile partial masses, lane positions first, then registers)
 * Ops run in the listed order; gate slot s of a pass lies between ops whose
 * slot ranges end at s and begin at s.  A dense op with no circuit gate in
 * its slot is a lane exchange (a swap of two positions). */
tqs_status tqs_plan_describe(const tqs_plan *p, char *buf, uint64_t cap, uint64_t *len);

/* Compile the plan's specialised pass kernels now (tuning.jit; a no-op when
 * they are off).  Runs otherwise compile them on the plan's first run.  No
 * device is needed; the code is kept with the plan (and shared by identical
 * plans in the process).  TQS_E_HIP with the compiler's log on failure. */
tqs_status tqs_plan_compile(tqs_plan *p);

/* The HIP source of the plan's specialised pass kernels (for tests and
 * inspection): *len gets the size with the terminating NUL; buf may be
 * NULL; output is truncated to cap. */
tqs_status tqs_plan_jit_source(const tqs_plan *p, char *buf, uint64_t cap, uint64_t *len);

void tqs_plan_destroy(tqs_plan *p);

/* --------------------------------------------------------------------- run */

/* Simulate every leaf of the tree (Sec. 3.1: each node runs its subcircuit
 * instance with its own noise on a copy of its parent's state; each leaf
 * is sampled once).  d_workspace: device pointer, 256-byte aligned,
 * ws_bytes >= tqs_workspace_bytes.  stream: hipStream_t or NULL.  outcomes:
 * host array of n_leaves.  Stream-ordered; returns after the outcomes are on
 * the host.  stats may be NULL.
 * Errors: a run that fails after it enqueued device work waits for that work
 * on the stream before it returns, so the workspace may be freed or reused at
 * once and the plan stays valid (resume with tqs_run_range).  For tests of
 * these paths the environment variable TQS_FAULT injects a failure on the
 * host (no kernel is altered): "alloc" fails the run's host metadata
 * allocation (TQS_E_OOM, before any device call); "launch:K" fails its K-th
 * pass from 0 (TQS_E_HIP, after the passes before it were enqueued). */
tqs_status tqs_run(tqs_plan *p, const tqs_noise *nz, void *d_workspace, uint64_t ws_bytes,
                   void *stream, uint64_t *outcomes, tqs_run_stats *stats);

/* The same run in two halves, so that the host work of the next run (its
 * noise metadata, schedule and packing, about 2 ms for a 16384-leaf tree)
 * overlaps this run's device work.  tqs_run_start does everything up to the
 * outcome download, enqueued on `stream`, and returns without waiting;
 * tqs_run_finish waits for it, writes `outcomes` (host, n_leaves, owned by
 * the caller until then) and, with flags TQS_RUN_STATS, the statistics, and
 * frees the run.  At most two runs of one plan may be in flight (TQS_E_ARG
 * beyond), each with a workspace of its own; every started run must be
 * finished, and before its plan is destroyed.  Errors as tqs_run; a start
 * that fails leaves nothing to finish (*out NULL). */
typedef struct tqs_pending tqs_pending;
#define TQS_RUN_STATS 1u
tqs_status tqs_run_start(tqs_plan *p, const tqs_noise *nz, void *d_workspace, uint64_t ws_bytes,
                         void *stream, uint64_t *outcomes, uint32_t flags, tqs_pending **out);
tqs_status tqs_run_finish(tqs_pending *run, tqs_run_stats *stats);

/* As tqs_run, but only level-0 subtrees [first, last) are simulated; the
 * outcomes of their leaves go to outcomes[0 ..): resuming a failed run or
 * splitting one across devices gives the same outcomes as one whole run. */
tqs_status tqs_run_range(tqs_plan *p, const tqs_noise *nz, void *d_workspace,
                         uint64_t ws_bytes, void *stream, uint64_t first, uint64_t last,
                         uint64_t *outcomes, tqs_run_stats *stats);

/* As tqs_run, and also return the final (pre-measurement) amplitudes of the
 * listed leaves as complex128 (host, n * 2^n interleaved doubles), with the
 * noise frame applied (for tests and analysis; not a fast path). */
tqs_status tqs_run_capture(tqs_plan *p, const tqs_noise *nz, void *d_workspace,
                           uint64_t ws_bytes, void *stream, uint64_t *outcomes,
                           const uint64_t *leaves, uint64_t n, double *host_amps);

/* As tqs_run, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no workspace argument and no allocation.  The run uses a static device
 * array of the library, 64 MiB, one per GPU, held until the process ends;
 * a run that needs more (tqs_workspace_bytes) returns TQS_E_WORKSPACE.  The
 * stream (or NULL, the null stream) must belong to the current device.  All
 * calls on one GPU share its array and it keeps the last call's contents:
 * calls that overlap on one GPU (other threads, other streams) race, so
 * the caller orders them.  Outcomes as tqs_run; no statistics.  No HIP
 * allocation of any kind: the metadata goes up from pageable host memory
 * and the outcomes come straight down (no pinned staging), and the plan's
 * specialised kernels are used only when an earlier run already loaded them
 * on this device (else the generic kernels take every state; same
 * outcomes up to rounding). */
tqs_status tqs_run_noalloc(tqs_plan *p, const tqs_noise *nz, void *stream, uint64_t *outcomes);

/* --------------------------------------------------------------- batches
 * Several runs (each a plan with its insertion list; different circuits,
 * qubit counts and trees) advanced together: the k-th launch of every run
 * (a pass over a chunk of states, or the sampling of a leaf chunk) joins one
 * combined launch, so small circuits fill the device together (the runs'
 * trees follow Sec. 3.1 each, unchanged).  Every plan needs the same
 * precision and tile width.  The batch keeps pointers to the plans and
 * insertion lists, which must outlive it.  Outcomes of run i start at the
 * sum of the leaf counts of runs 0..i-1. */
typedef struct tqs_batch tqs_batch;
tqs_status tqs_batch_create(tqs_plan *const *plans, const tqs_noise *const *noises, uint32_t count,
                            tqs_batch **out);
/* Device workspace bytes, total leaves, combined launch steps (any pointer may be NULL). */
tqs_status tqs_batch_info(const tqs_batch *b, uint64_t *workspace_bytes, uint64_t *leaves, uint32_t *steps);
/* Runs the batch (stream-ordered; returns with the outcomes on the host).
 * stats (nullable) gets ms_device, ms_wall and launches. */
tqs_status tqs_batch_run(tqs_batch *b, void *d_workspace, uint64_t ws_bytes, void *stream,
                         uint64_t *outcomes, tqs_run_stats *stats);
/* Replay (on != 0) or plain launches (0, the default) for later runs: with
 * replay, the batch's kernel launches are recorded once into a HIP graph on
 * a private stream (for the workspace address of that run; a run with
 * another workspace records again) and each run launches the graph on its
 * stream after the usual metadata upload.  This removes the host's cost of
 * issuing the launches, which matters only when it is comparable to the
 * kernels' own time.  Outcomes are the same either way. */
tqs_status tqs_batch_use_graph(tqs_batch *b, uint32_t on);

void tqs_batch_destroy(tqs_batch *b);

/* ------------------------------------------------- learned tree shape ---
 * A two-hidden-layer perceptron (ReLU, FP32) that predicts, from circuit,
 * noise, shot-count and candidate-shape features, a tree shape's run time
 * and fidelity spread; it stands in for the partition heuristic (Sec. 3.2)
 * when its prediction is trusted.  All pointers are device pointers (caller
 * owned, 4-byte aligned); calls are stream-ordered and do not synchronise.
 * Parameters, one array of tqs_mlp_param_count floats, row-major with the
 * input index first: W1[d_in x h], b1[h], W2[h x h], b2[h], W3[h x d_out],
 * b3[d_out]; forward y = relu(relu(x W1 + b1) W2 + b2) W3 + b3.
 * Limits: d_in, h <= 4096, d_out <= 64, batch <= 2^20; violations return
 * TQS_E_ARG. */
uint64_t tqs_mlp_param_count(uint32_t d_in, uint32_t h, uint32_t d_out);
/* Floats of device scratch that forward / loss_grad need for `batch` rows. */
uint64_t tqs_mlp_scratch_floats(uint32_t d_in, uint32_t h, uint32_t d_out, uint32_t batch);
/* y[batch x d_out] from x[batch x d_in] (row-major). */
tqs_status tqs_mlp_forward(const float *params, uint32_t d_in, uint32_t h, uint32_t d_out,
                           const float *x, uint32_t batch, float *y, float *scratch, void *stream);
/* Weighted squared error L = (1/B) sum_b sum_o w_o (y_bo - t_bo)^2 into
 * *loss (device float) and dL/dparams into grad (param_count floats),
 * by back-propagation; ReLU'(0) is taken as 0. */
tqs_status tqs_mlp_loss_grad(const float *params, uint32_t d_in, uint32_t h, uint32_t d_out,
                             const float *x, const float *target, const float *out_weight,
                             uint32_t batch, float *grad, float *loss, float *scratch, void *stream);
/* One Adam step (step counts from 1) on params with moments m, v. */
tqs_status tqs_mlp_adam(float *params, const float *grad, float *m, float *v, uint64_t count,
                        float lr, float beta1, float beta2, float eps, uint32_t step, void *stream);

/* ------------------------------------------------------- results, errors */

/* Sorted unique outcomes and their counts; values/counts hold n entries. */
tqs_status tqs_histogram(const uint64_t *outcomes, uint64_t n, uint64_t *values,
                         uint64_t *counts, uint64_t *n_unique);

/* Device copy bandwidth probe: copies `bytes` within the workspace `reps`
 * times with the library's streaming kernel and reports GB/s (read + write).
 * The workspace must hold 2 * bytes. */
tqs_status tqs_probe_copy(void *d_workspace, uint64_t bytes, uint32_t reps, void *stream,
                          double *gbps);

/* Message of the last failed call on this thread (never NULL). */
const char *tqs_last_error(void);

/* Library version string. */
const char *tqs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TQSIM_H */
