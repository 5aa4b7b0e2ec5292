/*
 * jf.h -- C ABI of the Jamiolkowski-fidelity library (MI355X / gfx950).
 *
 * Computes F_J(E, U) = (1/d^2) * sum_k |tr(U^dagger E_k)|^2, d = 2^n, between an ideal circuit U
 * and its noisy implementation E = {E_k} (Hong, Ying, Feng, Zhou, Li, "Approximate Equivalence
 * Checking of Noisy Quantum Circuits", Section III, the closed form under "Ease of
 * calculation"), by tensor-network contraction:
 *   - Algorithm I (Section IV-A): one closed miter network tr(U^dagger E_k) per Kraus tuple k;
 *     all tuples of a circuit are contracted together (the Kraus index of every noise site is
 *     an open leg of one network, batched or sliced with prefix reuse);
 *   - Algorithm II (Section IV-B): the single doubled network tr((U^dagger (x) U^T) M_E).
 *
 * Conventions
 *   - Every call returns a jf_status; nothing is thrown across the ABI.  On error the outputs
 *     are left untouched and jf_last_error() returns a message (thread-local).
 *   - Inputs are copied at load: the caller may free every array it passed once a call returns.
 *   - Handles (jf_circuit, jf_plan) belong to the caller and are released with jf_free_*.
 *     A plan is immutable after jf_plan_contraction; use one stream per plan at a time.
 *   - Device memory: the caller passes a device workspace of at least the size reported by
 *     jf_plan_info (jf_batch_workspace for a batch), 256-byte aligned, and a hipStream_t (as
 *     void*; NULL = the null stream).  Fidelity calls enqueue on that stream, synchronise it
 *     and write results to caller host memory.  A workspace keeps the plan's device tables
 *     between calls, and a later call with the same plan and address does not upload them again:
 *     before memory that served as a workspace is freed or written for anything else, call
 *     jf_workspace_release on it.
 *   - Qubit 0 is the most significant bit of a basis index; a two-qubit matrix acts on
 *     (q0, q1) with q0 the more significant; CX/CZ/CS have their control on q0.
 *   - Matrices are row-major with interleaved (re, im) doubles.
 *   - Noise strengths are error probabilities (a depolarising channel of strength p keeps the
 *     state with probability 1-p; the paper's Example 2 writes the no-error probability).
 */
#ifndef JF_H
#define JF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  JF_OK = 0,
  JF_E_ARG = -1,          /* bad argument (NULL handle, bad size, bad enum, bad gate index) */
  JF_E_NOT_UNITARY = -2,  /* a gate matrix violates ||G^dagger G - I||_max <= tol */
  JF_E_NOT_TP = -3,       /* a Kraus set violates ||sum K^dagger K - I||_max <= tol (Section II-B) */
  JF_E_QUBIT = -4,        /* qubit index out of range, or a two-qubit gate on one qubit */
  JF_E_TOO_LARGE = -5,    /* no contraction order fits the intermediate-size cap, or Algorithm I's
                             per-Kraus-tuple output of a component exceeds 2^34 values */
  JF_E_OOM = -6,          /* workspace smaller than required */
  JF_E_HIP = -7,          /* a HIP runtime call failed (message in jf_last_error) */
  JF_E_UNSUPPORTED = -8   /* valid request this library does not provide */
} jf_status;

typedef enum {
  JF_C128 = 0,       /* complex128 storage, FP64 arithmetic */
  JF_C64 = 1,        /* complex64 storage, FP32 MFMA with FP32 accumulation */
  JF_C64_BF16X6 = 2  /* complex64 storage, split precision: every FP32 operand of a contraction step
                        is split exactly into three BF16 numbers (x = x0 + x1 + x2, "3 x BF16") and
                        each real product is formed from the six piece products x0 y0, x0 y1,
                        x1 y0, x0 y2, x1 y1, x2 y0 on the BF16 matrix cores with FP32 accumulation
                        (the three dropped ones are below 2^-24 of the product); noise-carrying
                        operators keep a fourth piece, the BF16 residual of the FP64 operator */
} jf_dtype;
/* In every dtype the closing contractions (the steps after which every intermediate stays within
 * 2^12 elements; a component whose whole program stays within that size runs the complex128
 * program), the traces t_k, sum_k |t_k|^2 (double-double over fixed reduction trees) and 1 - F_J
 * are evaluated in FP64 on the GPU. */

typedef enum {
  JF_GATE_H = 0, JF_GATE_S, JF_GATE_SDG, JF_GATE_T, JF_GATE_TDG, JF_GATE_X, JF_GATE_Y, JF_GATE_Z,
  JF_GATE_SX, JF_GATE_RZ, JF_GATE_RX, JF_GATE_RY,
  JF_GATE_SU2,   /* RZ(theta[0]) RY(theta[1]) RZ(theta[2]) */
  JF_GATE_CX, JF_GATE_CZ, JF_GATE_CS, JF_GATE_SWAP,
  JF_GATE_MAT1,  /* explicit 2x2 unitary in mat (8 doubles) */
  JF_GATE_MAT2   /* explicit 4x4 unitary in mat (32 doubles) on (q0, q1) */
} jf_gate_kind;
/* Gate matrices (Section II-A, Example 1): H = (X+Z)/sqrt2, S = diag(1,i), T = diag(1,e^{i pi/4}),
 * SX = ((1+i)I + (1-i)X)/2, RP(t) = exp(-i t P/2), CS = diag(1,1,1,i), SWAP as in Example 1. */

typedef struct {
  int kind;          /* jf_gate_kind */
  int q0, q1;        /* target qubit(s); q1 ignored for one-qubit gates */
  double theta[3];   /* angles of RZ/RX/RY (theta[0]) and SU2 (all three) */
  const double* mat; /* MAT1/MAT2 only: interleaved row-major matrix, copied at load */
} jf_gate;

typedef enum {
  JF_NOISE_KRAUS = 0,          /* explicit Kraus set: n_kraus matrices in kraus */
  JF_NOISE_DEPOLARIZING = 1,   /* {sqrt(1-p) I, sqrt(p/3) X, sqrt(p/3) Y, sqrt(p/3) Z} */
  JF_NOISE_BIT_FLIP = 2,       /* {sqrt(1-p) I, sqrt(p) X} */
  JF_NOISE_PHASE_FLIP = 3,     /* {sqrt(1-p) I, sqrt(p) Z} */
  JF_NOISE_BIT_PHASE_FLIP = 4, /* {sqrt(1-p) I, sqrt(p) Y} */
  JF_NOISE_AMPLITUDE_DAMPING = 5 /* {[[1,0],[0,sqrt(1-p)]], [[0,sqrt(p)],[0,0]]}, p = gamma */
} jf_noise_kind;

typedef struct {
  int after_op;        /* the site acts right after noisy gate after_op; -1 = before gate 0.
                          Several sites after the same gate act in array order. */
  int qubit;
  int channel;         /* jf_noise_kind */
  double p;            /* strength (named channels) */
  int n_kraus;         /* JF_NOISE_KRAUS: number of 2x2 Kraus operators (1..16) */
  const double* kraus; /* JF_NOISE_KRAUS: n_kraus x 8 doubles, copied at load */
} jf_noise;

typedef struct {
  double fj;              /* F_J */
  double one_minus_fj;    /* 1 - F_J.  Alg I: sum_k |t_k|^2 of each component is a double-double
                             (TwoSum, fixed reduction trees), the product over components a
                             double-double, and 1 - F_J = (1 - hi) - lo, where 1 - hi is exact for
                             hi in [0.5, 2] (Sterbenz).  Alg II: 1 - Re T/d^2, exact (Sterbenz) when
                             Re T/d^2 lies in [0.5, 2]; Re T itself is an FP64 sum. */
  double imag_residual;   /* Alg II: |Im T| / d^2 (mathematically 0); Alg I: 0 */
  long long kraus_terms;  /* prod_i n_i, the number of Kraus tuples the result covers, saturated at
                             2^63 - 1 (an Algorithm II network with 40 depolarising sites covers
                             4^40) */
  long long work_items;   /* slices (DFS leaves) executed */
  double max_log2_intermediate; /* largest intermediate of the executed program, log2 elements */
  double path_flops;      /* real flops of the executed contraction program (complex MAC = 8) */
  double path_bytes;      /* algorithmic HBM bytes of the program (each step reads its input
                             tensor and writes its output once) */
  double seconds;         /* device time of the last run (events around the enqueued work) */
} jf_result;

typedef struct jf_circuit jf_circuit;
typedef struct jf_plan jf_plan;

/* Plan flags */
#define JF_FLAG_NO_CANCEL 1u   /* keep every U^dagger U pair (skip the local optimisation of
                                  Section IV-C that cancels adjacent mutually inverse gates) */
#define JF_FLAG_NO_FUSE   2u   /* one contraction step per network tensor (no block fusion) */
#define JF_FLAG_NO_BATCH  4u   /* slice every Kraus index (one DFS leaf per Kraus tuple) */
#define JF_FLAG_GRAPH     8u   /* jf_fidelity_alg1 / alg2 capture the step program into a hipGraph
                                  and replay it (see there) */
#define JF_FLAG_NO_CHAIN 16u   /* run every step as its own launch: no chains of in-place complex64
                                  steps applied to one LDS tile per HBM pass (same results bit for
                                  bit; chains are the default) */
/* Search effort of the planner: JF_FLAG_EFFORT(e), e = 1..15, runs 2^(e+5) randomised greedy
 * restarts per component.  The default (e = 0 in the flags) sizes the search to the network:
 * min(2^17, max(2^12, 8e7 / tensors)) restarts, i.e. 2^17 up to ~600 tensors and 2^16 at ~1200,
 * and to the stakes: 512 when the first greedy paths already estimate under 200 us of device time.
 * More restarts find cheaper contraction orders; the plan is reproducible for a given effort. */
#define JF_FLAG_EFFORT(e) (((unsigned)(e) & 15u) << 8)

/*
 * jf_load_circuit -- ingest an ideal circuit, its noisy implementation and the noise sites
 * (Problem 1: the classical description of an ideal circuit and a noisy implementation).
 *   n_qubits     1..62
 *   ideal        n_ideal gates of U in application order
 *   noisy_gates  gates of the noisy implementation; NULL means the same as ideal
 *   noise        n_noise one-qubit noise sites placed between noisy gates (Section II-B)
 *   tol          unitarity / trace-preservation tolerance (<= 0 selects 1e-10)
 * Validates every gate (unitary) and Kraus set (sum K^dagger K = I).  Errors: JF_E_ARG,
 * JF_E_QUBIT, JF_E_NOT_UNITARY, JF_E_NOT_TP.
 */
jf_status jf_load_circuit(int n_qubits, const jf_gate* ideal, int n_ideal,
                          const jf_gate* noisy_gates, int n_noisy,
                          const jf_noise* noise, int n_noise, double tol, jf_circuit** out);

/*
 * jf_plan_contraction -- build the network of Algorithm I (alg = 1, Section IV-A: the miter of
 * E_k and U^dagger closed into a trace, Kraus index of each site an open leg) or Algorithm II
 * (alg = 2, Section IV-B: q and q' wires, V on q and V* on q', noise as M_N on (q, q')), apply
 * the exact local cancellation of adjacent U^dagger U pairs (Section IV-C), search a greedy
 * minimum-intermediate-size contraction order, slice Kraus indices while the largest
 * intermediate exceeds 2^max_log2_intermediate elements (<= 0 selects 30), fuse consecutive
 * steps into small-operator blocks and lower the order to a device step program.
 * alg = 0 plans both algorithms and keeps the one whose step program has the smaller estimated
 * device time (jf_plan_stats.alg tells which; call jf_fidelity_alg1 or _alg2 accordingly).
 * Algorithm I holds one FP64 complex value per Kraus tuple of each connected component, sliced
 * or not, so a component with more than 34 Kraus-index bits (256 GiB of values) is
 * JF_E_TOO_LARGE for alg = 1 (alg = 0 then keeps Algorithm II).
 * Host only (no GPU needed).  Errors: JF_E_ARG, JF_E_TOO_LARGE, JF_E_UNSUPPORTED.
 */
jf_status jf_plan_contraction(const jf_circuit* circuit, int alg, jf_dtype dtype,
                              int max_log2_intermediate, unsigned flags, jf_plan** out);

/* Workspace bytes a fidelity call on this plan needs, and the plan's static costs
 * (kraus_terms, work_items, max_log2_intermediate, path_flops, path_bytes). Host only. */
jf_status jf_plan_info(const jf_plan* plan, size_t* workspace_bytes, jf_result* static_costs);

/* Host-side description of the lowered program (for tests and reports): number of device
 * steps, fused blocks, components and sliced Kraus sites.  Host only. */
typedef struct {
  int n_steps, n_components, n_sliced_sites, n_open_bits;
  int n_tensors_before_cancel, n_tensors_after_cancel;
  double planner_seconds;
  double empty_loops;
  int alg;             /* 1 or 2: the algorithm of the plan */
  double est_seconds;  /* planner's cost-model estimate of one run's device time */
  int n_swaps_rewired; /* SWAP gates (after the cancellation) replaced by crossed wires */
  int n_sliced_wires;  /* wire legs sliced: each is fixed to 0 and 1 in turn and the partial results
                          of the depth-first leaves are added (plans over the cap) */
} jf_plan_stats;
jf_status jf_plan_stats_get(const jf_plan* plan, jf_plan_stats* stats);

/* Text description of the lowered program, one line per device step:
 * "comp step level kS kN L rA rC tiles in_prec out_prec compute nvar flops bytes rowsA rowsC sA nC
 *  chain", rowsA .. nC being comma-separated bit positions (A for tile rows and summed legs, C for
 * tile rows and new legs; "-" when empty).  compute is f64, f32, f32x2 (FP32 with the operator kept
 * as an FP32 pair), split or split4 (the split form; split4 with the fourth operator piece).  chain is the index (within the component) of the chain the step
 * belongs to, -1 if it runs as its own launch (see JF_FLAG_NO_CHAIN).
 * Writes at most len bytes (NUL-terminated) and returns the full length needed. Host only. */
long long jf_plan_describe(const jf_plan* plan, char* buf, long long len);

/*
 * jf_fidelity_alg1 -- run an Algorithm I plan on the GPU.
 *   dev_ws/ws_bytes  device workspace (>= jf_plan_info size), stream = hipStream_t or NULL
 *   term_traces      optional host array of 2*kraus_terms doubles: t_k/d = tr(U^dagger E_k)/d
 *                    as (re, im), tuples in lexicographic order of the site indices with the
 *                    first site (in time order) most significant.
 * Plans made with JF_FLAG_GRAPH capture the step program into a hipGraph on the first call for a
 * (workspace, stream, kernel choice) and replay it in later calls; with the NULL stream such a
 * plan uses a stream of its own, ordered after the work already on the NULL stream.  (On MI355X
 * replay gains a few percent on a non-default stream, since the cost per step is on the GPU side,
 * and the NULL-stream hand-off adds ~40 us.)  A plan with both LDS-resident and larger
 * components runs the former's persistent launch on a second stream of the plan's own, forked
 * from and joined back to the run's stream by events (inside the graph too).  The first call
 * allocates a small pinned host landing area per plan (held until jf_free_plan), into which the
 * device writes F_J; the call synchronises before returning.
 * Errors: JF_E_ARG (not an Alg I plan), JF_E_OOM (workspace too small), JF_E_HIP.
 */
jf_status jf_fidelity_alg1(jf_plan* plan, void* dev_ws, size_t ws_bytes, void* stream,
                           jf_result* out, double* term_traces);

/* jf_fidelity_alg2 -- run an Algorithm II plan: F_J = Re(T)/d^2, |Im T|/d^2 reported.  Graph
 * capture and streams as jf_fidelity_alg1. */
jf_status jf_fidelity_alg2(jf_plan* plan, void* dev_ws, size_t ws_bytes, void* stream,
                           jf_result* out);

/*
 * jf_fidelity_batch -- run n plans (Alg I or Alg II, any mix, one dtype per plan) as one
 * batched submission (the networks are independent, Section IV-A): small components execute
 * LDS-resident, one workgroup each, in a single persistent launch on a second stream (forked from
 * and joined back to the caller's stream by events) beside the larger ones' step programs, which
 * run back to back; the whole submission is captured once into a hipGraph (cached on
 * the first plan, keyed by the plans, the workspace and the stream) and replayed.  Each plan keeps
 * its tables, outputs and sums in a region of its own; since the programs run one after another,
 * their level buffers share one region sized for the largest, so the workspace is the sum of the
 * plans' small parts plus the largest buffer set.  out[i] receives plan i's result.  The workspace
 * must hold jf_batch_workspace bytes.
 */
jf_status jf_batch_workspace(jf_plan* const* plans, int n, size_t* workspace_bytes);
jf_status jf_fidelity_batch(jf_plan* const* plans, int n, void* dev_ws, size_t ws_bytes,
                            void* stream, jf_result* out);

/*
 * jf_fidelity_noalloc -- for callers that cannot allocate: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Runs an Algorithm I or II plan as
 * jf_fidelity_alg1 / jf_fidelity_alg2 do (the same kernels, launched eagerly: no hipGraph, also
 * for JF_FLAG_GRAPH plans) with the library's own static device scratch as the workspace:
 * JF_NOALLOC_BYTES per GPU, a file-scope device array that each GPU the library runs on holds
 * until the process ends.  The call makes no hipMalloc, hipFree, hipHostMalloc or other
 * allocating call; results are copied straight into the caller's host memory.
 *   stream       hipStream_t as void* (NULL = the null stream); the call synchronises it
 *   out          as jf_fidelity_alg1 / alg2, except out->seconds: host wall time of the call
 *   term_traces  optional, Algorithm I plans only, as in jf_fidelity_alg1
 * All calls on one GPU share its scratch and leave their contents in it (a plan's tables are
 * copied in again whenever another plan used the scratch last; the call clears its own outputs),
 * so calls that overlap in time on one GPU -- from several threads or streams -- race: the caller
 * serialises them.  Errors: JF_E_ARG, JF_E_OOM (the plan's workspace, jf_plan_info, exceeds
 * JF_NOALLOC_BYTES: run it through jf_fidelity_alg1 / alg2 with a caller workspace), JF_E_HIP.
 */
#define JF_NOALLOC_BYTES (128u << 20)
jf_status jf_fidelity_noalloc(jf_plan* plan, void* stream, jf_result* out, double* term_traces);

/*
 * jf_profile_run -- measurement aid: runs the plan's program once like jf_fidelity_alg1/alg2,
 * with a pair of HIP events attached to the dispatch of every contraction-step kernel
 * (hipExtLaunchKernelGGL: the events time the kernel itself, not the queue gaps around it), and
 * reports the summed kernel time together with the algorithmic bytes and flops of those
 * launches (each step reads its input tensor and writes its output once).  F_J is not returned.
 */
typedef struct {
  long long launches;   /* contraction-step kernel launches */
  double kernel_ms;     /* sum of their event-measured durations */
  double bytes;         /* algorithmic bytes of those launches */
  double flops;         /* real flops of those launches (complex MAC = 8) */
  double total_ms;      /* event time of the whole enqueued program */
  double max_launch_ms; /* longest single launch */
} jf_profile;
jf_status jf_profile_run(jf_plan* plan, void* dev_ws, size_t ws_bytes, void* stream, jf_profile* out);

/*
 * jf_profile_steps -- the same run, reported per launch: out[i] for the i-th contraction-step
 * launch in program order (i < cap), *n_launches = number of launches.  mode is the step's
 * arithmetic (0 FP64, 1 FP32, 2 FP32 in / FP64 out, 3 split form, 4 FP32 with a two-term operator,
 * 5 split form with a fourth operator piece);
 * variant the kernel that ran it (jf_kernel_variant, never AUTO); steps the number of program
 * steps the launch ran (1, or the length of a chain: variant JF_KV_CHAIN, kS = kN the largest
 * summed extent of its steps, L the log2 of its LDS tile, mode 4 if it holds a step with a
 * two-term operator, flops the chain's, bytes one read and one write of the intermediate);
 * threads the workgroup size of the launch (with variant and mode, it names the kernel).
 */
typedef struct {
  double ms;     /* event-measured duration */
  double flops;  /* real flops (complex MAC = 8) */
  double bytes;  /* algorithmic bytes: input tensor read once, output written once */
  int kS, kN, L; /* log2 of summed, new and per-tile row extents */
  int mode, variant, component;
  int steps;     /* program steps run by this launch */
  int threads;   /* workgroup size */
} jf_step_profile;
jf_status jf_profile_steps(jf_plan* plan, void* dev_ws, size_t ws_bytes, void* stream, jf_step_profile* out,
                           int cap, int* n_launches);

/*
 * jf_stream_copy -- measurement aid: copies bytes from src to dst (device buffers, 16-byte aligned;
 * bytes a multiple of bytes_per_lane = 8 or 16) with a plain streaming kernel -- nontemporal loads
 * and stores of bytes_per_lane per lane, a resident grid striding over the buffer -- and returns its
 * duration in *ms (HIP events attached to the dispatch).  2 bytes / ms is the HBM rate the step
 * kernels' access pattern can reach, the ceiling their per-launch rates are set against.
 * Synchronises the stream; bytes = 0 copies nothing and returns 0 ms.  Errors: JF_E_ARG (a NULL
 * pointer, a buffer not 16-byte aligned, bytes_per_lane other than 8 or 16, bytes not a multiple of
 * it: checked before anything is launched), JF_E_HIP.
 */
jf_status jf_stream_copy(const void* src, void* dst, size_t bytes, int bytes_per_lane, void* stream, double* ms);

/*
 * Kernels that can run a contraction step.  The staged kernels stage a tile of the input in LDS
 * and multiply it on the matrix cores; the direct kernels load every lane's matrix-core operands
 * straight into registers; FMA multiplies on the vector units; the Gauss kernels are direct
 * kernels that form each complex product from three real ones (Re.Re, Im.Im and (Re+Im).(Re+Im)),
 * a quarter fewer matrix-core products, with the imaginary part's rounding error relative to the
 * largest of the three (two-term FP32 blocks: the residual's products first).  AUTO is a fixed rule measured
 * on MI355X.  Not every kernel takes every shape: a step keeps the AUTO rule where its choice
 * does not apply.
 */
typedef enum {
  JF_KV_AUTO = 0,
  JF_KV_STAGED_256 = 1,
  JF_KV_STAGED_512 = 2,
  JF_KV_DIRECT_256 = 3,
  JF_KV_DIRECT_512 = 4,
  JF_KV_FMA = 5,
  JF_KV_GAUSS_256 = 6,
  JF_KV_GAUSS_512 = 7,
  JF_KV_CHAIN = 8   /* reported by jf_profile_steps only: a chain of in-place complex64 steps
                       applied to one LDS tile per HBM pass (not a choice for
                       jf_set_kernel_variant) */
} jf_kernel_variant;

/*
 * jf_autotune -- the autotuner of the tile / kernel choice.  Runs the plan once on the caller's
 * workspace and stream; on the first visit of each contraction step it times every kernel that
 * can run the step (a warm-up launch, then reps launches between HIP events, on the step's own
 * input and output buffers) and keeps the fastest for all later runs of this plan; a chain of
 * steps is timed as one launch against its steps run one launch each (with their tuned kernels)
 * and the faster is kept.  The
 * workspace contents are undefined afterwards (no result is produced).  Choices are cached for
 * the process by step shape (arithmetic, kS, kN, rows per tile, tile count, in place or not) and
 * by chain shape, so plans sharing shapes are tuned once.  A chain computes exactly what its steps
 * compute with the Gauss kernels (same products in the same order).  Kernels sum in different orders, so a tuned plan may
 * differ from an untuned one in the last bits; replays of a tuned plan are bitwise identical.
 * reps <= 0 means 3.  Synchronises the stream.  Errors: JF_E_ARG, JF_E_OOM (workspace too
 * small), JF_E_HIP.
 */
jf_status jf_autotune(jf_plan* plan, void* dev_ws, size_t ws_bytes, void* stream, int reps);

/*
 * jf_set_kernel_variant -- force one kernel (jf_kernel_variant) on every step it can run; the
 * other steps keep the AUTO rule.  Chains stay chains under JF_KV_GAUSS_256 / 512 (they compute
 * the Gauss form) and are split into their steps under the other kernels.  JF_KV_AUTO restores the
 * rule and the chains everywhere (and so undoes jf_autotune).  For testing each kernel against
 * the oracle.  Host only.  Errors: JF_E_ARG (JF_KV_CHAIN is not a per-step kernel).
 */
jf_status jf_set_kernel_variant(jf_plan* plan, int variant);

/* Definition 1: C1 and C2 are epsilon-equivalent iff F_J > 1 - eps (strict). Returns 1/0,
 * or -1 for a NULL result. */
int jf_is_equivalent(const jf_result* result, double eps);

/*
 * jf_decide_equivalence -- Definition 1 with early stopping (Algorithm I, Section IV-A: the terms
 * |tr(U^dagger E_k)|^2 / d^2 are nonnegative, so a partial sum above 1 - eps decides equivalence).
 * For an Algorithm I plan with sliced Kraus sites, every component but the one with the most
 * depth-first leaves runs in full and that one runs leaf by leaf; after each leaf the library
 * holds a two-sided bound on F_J:
 *   fj_lower = the terms computed so far (complete for the other components),
 *   fj_upper = fj_lower + (the mass of the leaves not yet run) x (the mass of every other site),
 * where the mass of a Kraus tuple is prod_i ||K_{k_i}||^2 (operator norms; w_k for Pauli
 * channels), an upper bound on its term.  It stops as soon as fj_lower - margin > 1 - eps
 * (decision 1: equivalent) or fj_upper + margin <= 1 - eps (decision 0: not equivalent), where
 * margin is the parity bar of the plan's form (1e-12 complex128, 1e-6 complex64 and split form).
 * Plans with one leaf (and Algorithm II plans) run once and decide from F_J; decision -1 means
 * F_J lies within the margin of 1 - eps.  Leaves run in depth-first order (Kraus operator 0 of
 * each sliced site first: the no-error operator for the built-in channels).  Synchronises the
 * stream after every leaf.  Errors: JF_E_ARG (eps outside (0, 1]), JF_E_OOM, JF_E_HIP.
 */
typedef struct {
  int decision;           /* 1 equivalent, 0 not equivalent, -1 within the margin of 1 - eps */
  double fj_lower, fj_upper;
  double margin;
  long long leaves_run, leaves_total;  /* depth-first leaves (work items) run / in the plan */
  double seconds;         /* device time, HIP events */
} jf_decision;
jf_status jf_decide_equivalence(jf_plan* plan, double eps, void* dev_ws, size_t ws_bytes, void* stream,
                                jf_decision* out);

/*
 * jf_workspace_release -- the caller is done with [dev_ws, dev_ws + ws_bytes) as a workspace (it
 * will free it or use it for something else).  The library forgets which plan tables it holds,
 * so every plan uploads its tables again the next time it is given memory in that range.  Host
 * only: touches no device memory, and needs no synchronisation beyond the caller's own (the
 * fidelity calls have synchronised their streams when they return).  ws_bytes = 0 releases the
 * one address.  Errors: JF_E_ARG (NULL dev_ws).
 */
jf_status jf_workspace_release(const void* dev_ws, size_t ws_bytes);

void jf_free_circuit(jf_circuit* circuit);
void jf_free_plan(jf_plan* plan);
const char* jf_last_error(void);

/*
 * jf_emulate_plan -- validation aid for the lowering, not a fidelity path: executes a plan's
 * device step program on the host in FP64 with exactly the offset tables the GPU kernels use
 * and writes the traces (Alg I, as term_traces above) or T/d^2 (Alg II, out[0..1]).  Lets the
 * CPU test suite check the planner, slicing and block fusion; no fidelity entry point calls it.
 */
jf_status jf_emulate_plan(const jf_plan* plan, double* out, long long out_len);

#ifdef __cplusplus
}
#endif
#endif /* JF_H */
