/*
 * met_bp.h -- C ABI of the MI355X (gfx950) syndrome belief-propagation decoder
 * for multi-edge-type (MET) LDPC codes.
 *
 * Method: Wang, Zhang, Yu, Guo, "High speed error correction for
 * continuous-variable quantum key distribution with multi-edge type LDPC code"
 * (arXiv:1711.01783).  The decoder is the flooding sum-product algorithm of the
 * Methods section (Steps 1-5, eq. (1)-(5)), run in log-likelihood ratios (last
 * Methods paragraph) on many codewords at once (Results, "High speed error
 * correction with MET-LDPC codes"), with degree-1 variable nodes left out of
 * the iterations (same passage; Discussion; Table 1 note 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Return value: 0 (MET_OK) or a negative MET_E* code; the text of the last
 *   error of the calling thread is available from met_last_error().  No entry
 *   point aborts the process.  Arguments are validated before any HIP call, so
 *   argument errors are reported identically on machines without a GPU.
 * Ownership: the caller owns every buffer it passes.  The library owns only a
 *   code handle (host adjacency plus one device copy per GPU it was used on)
 *   until met_code_free().  "dev" marks device pointers (HIP device memory of
 *   the current device), "host" marks host pointers.
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Device work
 *   is enqueued asynchronously on it; outputs are valid once it has drained.
 * LLR sign: L = ln p(x=0)/p(x=1), i.e. L = -ln q0 with the paper's ratio
 *   q0 = p(1)/p(0) of eq. (1).  A hard decision is 1 iff the posterior is < 0
 *   (Step 5: c = 1 iff q > 1); a posterior of exactly 0 gives 0.
 * Layouts: frame-major row arrays; llr and posterior are float32 [B][N] in the
 *   code's variable-node order, bits uint8 [B][N] (0/1), syndromes uint8 [B][M]
 *   (0/1) in the code's check order.
 * Concurrency: calls on different streams with different workspaces may run
 *   concurrently; a workspace must not be shared by overlapping calls.
 */
#ifndef MET_BP_H
#define MET_BP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MET_OK 0
#define MET_EINVAL (-1)   /* bad argument: null/misaligned pointer, size, profile */
#define MET_ENOMEM (-2)   /* host or device allocation failed */
#define MET_EHIP (-3)     /* a HIP runtime call failed; see met_last_error() */
#define MET_ESTATE (-4)   /* call not valid in the current state */

/* met_decode flags */
#define MET_EARLY_EXIT 0u   /* default: a frame stops at the first iteration whose
                               hard decision satisfies its syndrome (Step 5) */
#define MET_FIXED_ITERS 1u  /* every frame runs max_iter iterations; converged
                               reports the syndrome test after the last one */
#define MET_NO_COMPACT 2u   /* early exit without compaction: frames that are
                               still running stay in their groups of 64 (by
                               default, every 4 iterations, finished frames are
                               written out and running ones are packed into as
                               few groups as hold them, when that frees at least
                               a quarter of the occupied groups; results are
                               identical either way; no compaction when
                               posteriors are requested) */
#define MET_C2V_FP16 8u     /* check-to-variable messages stored as IEEE half
                               (rounded to nearest; all arithmetic in float):
                               half the message bytes.  Groups of 64 frames
                               only (B > 32), no compaction.  Results are not
                               those of the float decoder; its gate is the
                               frame error rate (within the 95 % interval of
                               the float decoder's on the same frames) */
#define MET_C2V_Q8 16u      /* check-to-variable messages stored in 8 bits:
                               sign and a 7-bit index into a log-uniform grid
                               of magnitudes (0, then 2^-14 to 2^5 in 126
                               steps, 5.4 % rounding at most), read back
                               through a 128-entry table; all arithmetic in
                               float.  A quarter of the message bytes.  Groups
                               of 64 frames only (B > 32), no compaction.
                               Gated like MET_C2V_FP16 by the frame error rate */
#define MET_CHECK_LUT 32u   /* with MET_C2V_Q8: table-driven check update (the
                               lookup-table form of the LLR update, last
                               paragraph of Methods): a message input's phi
                               is read from a 512-entry table at the index of
                               its magnitude on a grid 4x finer than the
                               storage grid, an output's 8-bit code from a
                               second table at the index of its phi-domain sum
                               (checks of a compiled shape; run-time-degree
                               checks keep the evaluated phi).  Degree-1
                               inputs and decisions stay in float.  Gated by
                               the frame error rate */
#define MET_NO_DEG1_SKIP 4u /* degree-1 variable nodes take part in every
                               iteration like the others (their check messages
                               are stored and their posteriors updated; the
                               Table 1 "all VNs" reference); by default they
                               never enter the iterations.  The results agree
                               with the default to FP32 rounding: a degree-1
                               node's message is re-formed as (L + c) - c
                               instead of L.  The first such call builds a
                               second layout of the code (host and device). */

#define MET_MAX_EDGE_TYPES 8
#define MET_MAX_CHECK_DEGREE 32
#define MET_MAX_VN_DEGREE 65536

typedef struct met_code met_code; /* opaque */

/* A MET degree profile (Methods: MET-LDPC codes generalise LDPC codes; the
 * paper's distributions are from its reference [WANGRA] and not reproduced).
 * Rows are node types; vn_deg / cn_deg are row-major [n_types][n_edge_types]
 * degree matrices; fractions are relative to N.  Variable-node counts follow
 * the fractions (floor, last type takes the remainder); check counts follow
 * from socket balance and cn_frac must agree with them within 1 % of N. */
typedef struct {
  int32_t n_edge_types;
  int32_t n_vn_types;
  const double *vn_frac;  /* host [n_vn_types] */
  const int32_t *vn_deg;  /* host [n_vn_types * n_edge_types] */
  int32_t n_cn_types;
  const double *cn_frac;  /* host [n_cn_types] */
  const int32_t *cn_deg;  /* host [n_cn_types * n_edge_types] */
} met_profile;

/* Bookkeeping in the terms of Table 1 of the paper. */
typedef struct {
  int64_t N, M, E;                   /* variable nodes, checks, edges */
  int64_t E_type[MET_MAX_EDGE_TYPES];
  int64_t n_deg1;                    /* degree-1 variable nodes ("ignored VNs") */
  int64_t edges_to_pass;             /* E - n_deg1 (Table 1 note 2) */
  int64_t n_msg_vn;                  /* variable nodes of degree != 1 */
  int64_t n_msg_edges;               /* edges to variable nodes of degree >= 2 */
  int64_t n_leaf_edges;              /* edges to degree-1 variable nodes */
  int32_t n_edge_types;
  int32_t n_check_classes;           /* runs of checks decoded by one kernel shape */
  int32_t max_check_degree;
  int32_t max_vn_degree;
} met_code_stats;

/* Builds a code from a degree profile: per edge type, a seeded random
 * permutation of check sockets (SplitMix64 + Fisher-Yates), repaired so that no
 * variable/check pair repeats, then sorted by (check, edge type, variable).
 * The paper uses progressive edge growth instead (Methods, first paragraph);
 * this construction is the project's substitute.  Host-only: needs no GPU.
 * p: host profile; 2 <= N <= 2^30; *out receives a new handle.
 * Errors: MET_EINVAL for an inconsistent profile (edge type in two check types,
 * unbalanceable sockets, check degree < 2 or > MET_MAX_CHECK_DEGREE, variable
 * degree above MET_MAX_VN_DEGREE, failed multi-edge repair) or more than
 * INT32_MAX edges (edge positions are int32), MET_ENOMEM when host memory runs
 * out.  No entry point lets a C++ exception escape: an unexpected one returns
 * MET_ESTATE with its message in met_last_error(). */
int met_code_build(const met_profile *p, int64_t N, uint64_t seed, met_code **out);

/* Builds a code from a degree profile by progressive edge growth, the
 * construction the paper uses (Methods, first paragraph).  Node counts and
 * per-check socket counts as in met_code_build; then edges are placed node by
 * node (v = 0..N-1), edge type by edge type, each to the check that is, among
 * those with a free socket of its type and not yet adjacent to v, outside the
 * deepest breadth-first layer of v's neighbourhood in the type-t graph built
 * so far (at most depth[t] check layers searched), among those the least
 * filled with type-t edges, and among ties a seeded uniform draw (SplitMix64
 * stream number n_edge_types, one draw per edge).  No cycle of length
 * <= 2 depth[t] enters the type-t graph wherever free sockets allow; no pair
 * repeats.
 * depth: host int32 [n_edge_types], each 1..16, or NULL for the default
 * (1 where a layer cannot grow, else the largest K with
 * (d_v - 1) ((d_v - 1)(d_c - 1))^(K-1) <= 1024 for the largest type-t degrees
 * d_v, d_c: the expected size of the last layer searched).
 * Cost grows with the searched layers: N = 10^6 at the default depths takes
 * seconds to tens of seconds on one host core.
 * Errors: as met_code_build, and MET_EINVAL for a depth outside 1..16 or an
 * edge that finds no free check. */
int met_code_build_peg(const met_profile *p, int64_t N, uint64_t seed, const int32_t *depth, met_code **out);

/* A code from an explicit edge list (E edges, host arrays, any order; etype may
 * be NULL for a single edge type).  Used for small hand-built codes in tests.
 * Errors: MET_EINVAL for out-of-range indices, repeated pairs, a check of
 * degree < 2 or > MET_MAX_CHECK_DEGREE. */
int met_code_from_edges(int64_t N, int64_t M, int64_t E, const int32_t *vn, const int32_t *cn,
                        const int8_t *etype, met_code **out);

/* Fills *out (host).  Errors: MET_EINVAL on NULL. */
int met_code_info(const met_code *c, met_code_stats *out);

/* A run of consecutive checks that one check kernel handles: n_msg edges to
 * variable nodes of degree >= 2 and n_leaf edges to degree-1 variable nodes per
 * check (-1 for runs of mixed shapes), and the number of distinct variable
 * nodes of degree >= 2 those checks reach.  first_check counts in the
 * decoder's check order: the code's order with the checks of each such run
 * sorted by their smallest (then largest) variable node of degree >= 2, so
 * that checks sharing a node are updated together.  Syndromes and all other
 * arguments stay in the code's own check order. */
typedef struct {
  int32_t n_msg, n_leaf;
  int64_t first_check, n_checks;
  int64_t n_msg_vn_touched;
} met_check_class;

/* Copies up to max_entries check classes of the code (host array) and their
 * count into *n.  Errors: MET_EINVAL on NULL. */
int met_code_classes(const met_code *c, met_check_class *out, int32_t max_entries, int32_t *n);

/* Copies the edge list in check order into host arrays of length E.  Any of
 * vn / cn / etype may be NULL.  Errors: MET_EINVAL on a NULL code. */
int met_code_export(const met_code *c, int32_t *vn, int32_t *cn, int8_t *etype);

/* Releases the handle and its device copies (NULL is ignored).  The caller
 * must ensure no queued work still uses the code. */
void met_code_free(met_code *c);

/* Syndrome S = H x mod 2 for B frames (Step 1: Bob's syndrome S_B = H U).
 * bits: dev uint8 [B][N] (0/1); syn: dev uint8 [B][M] output.
 * The first call on a device uploads the adjacency (allocates device memory).
 * Errors: MET_EINVAL (NULL pointer, B < 1), MET_EHIP. */
int met_syndrome(const met_code *c, const uint8_t *bits, int32_t B, uint8_t *syn, void *stream);

/* ---- Multidimensional reconciliation (the decoder's front end) ----------
 * Results, "Information reconciliation for CV-QKD system", and Methods Step 1:
 * the correlated Gaussian raw keys of Alice (x) and Bob (y = x + z, noise
 * variance sigma_z^2) become Bob's random bit string and, on Alice's side,
 * log-likelihood ratios of a virtual binary-input AWGN channel, which
 * met_decode takes together with Bob's syndrome (met_syndrome of his bits).
 * Both strings are cut into blocks of d in {1, 2, 4, 8} consecutive values of a
 * frame, read as elements of the Cayley-Dickson algebra of dimension d
 * (product (a, b)(c, e) = (a c - conj(e) b, e a + b conj(c)), conj((a, b)) =
 * (conj(a), -b): reals, complex numbers, quaternions, octonions).
 *
 * Bob: for each block, alpha = u conj(y / |y|) with u = (1 - 2 bits) / sqrt(d)
 * (y / |y| taken as e_0 when |y| = 0), so that alpha (y / |y|) = u.
 *   y:     dev float32 [B][N], 16-byte aligned
 *   bits:  dev uint8   [B][N] (0/1; only bit 0 is read), 8-byte aligned
 *   alpha: dev float32 [B][N] output (one unit element per block), 16-byte aligned
 *   ynorm: dev float32 [B][N/d] output, |y| of every block
 * Alice: llr = 2 |y| (alpha x) / (sqrt(d) sigma_z^2) per block, i.e.
 * 2 |x| |y| v / (sqrt(d) sigma_z^2) with v = alpha x / |x| her noisy copy of u;
 * L = ln p(bit 0) / p(bit 1), the decoder's convention.
 *   x, alpha: dev float32 [B][N], ynorm dev float32 [B][N/d]; llr dev float32
 *   [B][N] output; x, alpha, llr 16-byte aligned; sigma_z2 > 0.
 * N must be a multiple of d and B N <= 2^36.  The caller owns every buffer;
 * work is queued on the stream.  Errors: MET_EINVAL, MET_EHIP. */
int met_mdr_bob(const float *y, const uint8_t *bits, int64_t B, int64_t N, int32_t d, float *alpha, float *ynorm,
                void *stream);
int met_mdr_alice(const float *x, const float *alpha, const float *ynorm, float sigma_z2, int64_t B, int64_t N,
                  int32_t d, float *llr, void *stream);

/* Workspace size in bytes that met_decode needs for this code, B frames and
 * these flags (want_posterior != 0 when a posterior output will be passed).
 * Errors: MET_EINVAL. */
int met_decode_workspace_bytes(const met_code *c, int32_t B, uint32_t flags, int32_t want_posterior,
                               size_t *bytes);

/* Decodes B frames against their syndromes: flooding sum-product BP of the
 * Methods section -- Step 2 / eq. (1) initialisation from channel LLRs, Step 3 /
 * eq. (2)-(3) check update with the sign of the target syndrome bit, Step 4 /
 * eq. (4) variable update of variable nodes of degree >= 2 only, Step 5 /
 * eq. (5) posteriors, hard decision and syndrome test.  Degree-1 variable nodes
 * never enter the iterations; their posteriors are formed from their check's
 * message when needed (Results; Table 1 note 1).
 *   llr:       dev float32 [B][N], 4-byte aligned
 *   syn:       dev uint8   [B][M]
 *   max_iter:  >= 1
 *   flags:     MET_EARLY_EXIT or MET_FIXED_ITERS, optionally | MET_NO_COMPACT,
 *              | MET_NO_DEG1_SKIP and/or | MET_C2V_FP16 or | MET_C2V_Q8 (with
 *              | MET_CHECK_LUT)
 *   bits:      dev uint8 [B][N] output, hard decisions at each frame's stop
 *   iters:     dev int32 [B] output, iterations run (1..max_iter)
 *   converged: dev uint8 [B] output, 1 iff H bits = syn
 *   posterior: dev float32 [B][N] output, or NULL
 *   workspace: dev, 256-byte aligned, at least met_decode_workspace_bytes();
 *              its contents need not be initialised
 * The first call on a device uploads the adjacency (allocates); later calls
 * allocate nothing.  Errors: MET_EINVAL, MET_EHIP. */
int met_decode(const met_code *c, const float *llr, const uint8_t *syn, int32_t B, int32_t max_iter,
               uint32_t flags, uint8_t *bits, int32_t *iters, uint8_t *converged, float *posterior,
               void *workspace, size_t ws_bytes, void *stream);

/* met_decode for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * same decoder, arguments and results as met_decode without the workspace
 * arguments: the workspace is a fixed array of MET_NOALLOC_SCRATCH_BYTES bytes
 * inside the library, one per device, held from the library's first use of a
 * device until the process ends.  No call allocates, frees or uploads:
 *   - the code's adjacency must already be on the current device (an earlier
 *     met_decode or met_syndrome on that device uploads it); else MET_ESTATE;
 *   - decodes whose workspace (met_decode_workspace_bytes) exceeds the array
 *     fail with MET_EINVAL (without posteriors the array holds, at the three
 *     profiles' sizes, N = 65536 with up to 192 frames, N = 2^18 with 32,
 *     N = 10^6 with 4);
 *   - MET_NO_DEG1_SKIP (which builds a second layout) is MET_EINVAL;
 *   - per-launch timing must be off (it creates events); else MET_ESTATE.
 * Every call on a device shares that device's array and leaves its contents
 * behind (every decode initialises what it reads): calls that overlap in time
 * on one device, on any streams, race and give wrong results; order them on
 * one stream or synchronise in between.  Errors: MET_EINVAL, MET_ESTATE,
 * MET_EHIP. */
#define MET_NOALLOC_SCRATCH_BYTES (256u << 20)
int met_decode_noalloc(const met_code *c, const float *llr, const uint8_t *syn, int32_t B, int32_t max_iter,
                       uint32_t flags, uint8_t *bits, int32_t *iters, uint8_t *converged, float *posterior,
                       void *stream);

/* Measurement support (not part of decoding).  While enabled, every kernel
 * launched by met_decode in this process is bracketed by two HIP events
 * recorded on the caller's stream, the stream the kernel runs on.
 * met_timing_collect waits for the recorded events, writes up to max_entries
 * per-kernel records (launch count, summed duration) and clears the record.
 * Enabling allocates HIP events; decoding results are unaffected.
 * Errors: MET_EINVAL (NULL output), MET_EHIP. */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
} met_kernel_time;
int met_timing_enable(int32_t on);
int met_timing_collect(met_kernel_time *out, int32_t max_entries, int32_t *n_entries);

/* ---- Weighted BP (learnable message scales) ------------------------------
 * The decoder above run for a fixed number of iterations L, with the
 * check-to-variable message of every edge of type t produced in iteration l
 * multiplied by weights[t * L + (l - 1)] after the syndrome sign (Step 3) and
 * before the variable update (Step 4).  weights = 1 gives exactly met_decode's
 * fixed-iteration results.  The forward pass keeps the message state of every
 * ckpt_every-th iteration in the workspace; the backward pass recomputes the
 * iterations between checkpoints and runs hand-written adjoint kernels in
 * reverse.  Irregular (non-compiled) check shapes must have degree <= 16. */

/* Workspace bytes for forward + backward (B frames, L iterations, a checkpoint
 * every ckpt_every iterations).  Errors: MET_EINVAL. */
int met_wbp_workspace_bytes(const met_code *c, int32_t B, int32_t iterations, int32_t ckpt_every, size_t *bytes);

/* Forward pass.  llr dev f32 [B][N], syn dev u8 [B][M], weights dev f32
 * [n_edge_types][iterations]; outputs posterior dev f32 [B][N] (after the last
 * iteration, eq. (5)), and optionally bits dev u8 [B][N] and converged dev u8
 * [B] (may be NULL).  The workspace (256-byte aligned, uninitialised) must be
 * passed unchanged to met_wbp_backward.  Errors: MET_EINVAL, MET_EHIP. */
int met_wbp_forward(const met_code *c, const float *llr, const uint8_t *syn, int32_t B, int32_t iterations,
                    const float *weights, int32_t ckpt_every, float *posterior, uint8_t *bits,
                    uint8_t *converged, void *workspace, size_t ws_bytes, void *stream);

/* Backward pass: grad_posterior dev f32 [B][N] (dLoss/dposterior) ->
 * grad_weights dev f32 [n_edge_types][iterations] (overwritten).  Same code,
 * B, iterations, weights, ckpt_every and workspace as the forward call.
 * Deterministic (fixed reduction order).  Errors: MET_EINVAL, MET_EHIP. */
int met_wbp_backward(const met_code *c, const float *grad_posterior, int32_t B, int32_t iterations,
                     const float *weights, int32_t ckpt_every, float *grad_weights, void *workspace,
                     size_t ws_bytes, void *stream);

/* Launch-shape choices for met_decode_ex and met_decode_batched; 0 in a field
 * selects the default. */
#define MET_BATCH_NO_STAGGER 1u /* batched: all jobs start in the same phase */
#define MET_BATCH_NO_GRAPH 2u   /* batched: plain launches instead of a HIP graph */
#define MET_BATCH_PHASE_LAUNCHES 4u /* batched: one launch per phase instead of
                                   one persistent launch: every launch holds the
                                   tiles of every job in that phase (the kernel
                                   boundary is the barrier); captured in the
                                   same HIP graph.  Same results.  Launches of
                                   jobs whose frames have all stopped still run
                                   (their tiles return at once) */
#define MET_BATCH_KIND_STREAMS 8u /* batched, implies MET_BATCH_PHASE_LAUNCHES:
                                   the launches of one phase (checks of the
                                   (3,1) / (2,1) shapes, checks of the other
                                   shapes, variable updates) run on parallel
                                   streams (graph branches) and join at the
                                   end of the phase */
#define MET_BATCH_JOB_STREAMS 16u /* batched, implies MET_BATCH_PHASE_LAUNCHES:
                                   each job's launches form a chain of their
                                   own on one of up to 4 parallel streams,
                                   joined once after the last phase; excludes
                                   MET_BATCH_KIND_STREAMS.  The parallel modes
                                   use side streams the library creates per
                                   device (default priority) and keeps; calls
                                   that use them must not overlap on one
                                   device */
#define MET_BATCH_JOBS_IN_TURN 32u /* batched, implies MET_BATCH_PHASE_LAUNCHES:
                                   the same per-job chains one job after the
                                   other on the launching stream (each job's
                                   data stays in the caches between its
                                   launches); excludes the two above */

typedef struct {
  int32_t check_steps_per_wave; /* 1, 2 or 4: steps of 64/W checks each wave of
                                   the check kernel loads before computing
                                   (groups of 64 frames only); default 4 */
  int32_t variable_chunk;       /* 8, 16 or 32: message gathers the variable
                                   kernel keeps in flight; default 16 */
  int32_t blocks_per_cu;        /* batched: resident blocks per compute unit
                                   of the persistent launch (0 = as many as
                                   fit; unused by phase launches, where the
                                   autotuner reports 0) */
  uint32_t batch_flags;         /* batched: MET_BATCH_* */
  int32_t interleave;           /* batched: frames per group, 16, 32 or 64
                                   (one check step per wave below 64);
                                   default 64 */
  int32_t reserved[3];          /* must be 0 */
} met_tuning;

/* met_decode with explicit launch shapes (tuning may be NULL).  Results do not
 * depend on the tuning.  Errors: as met_decode, MET_EINVAL for bad tuning. */
int met_decode_ex(const met_code *c, const float *llr, const uint8_t *syn, int32_t B, int32_t max_iter,
                  uint32_t flags, uint8_t *bits, int32_t *iters, uint8_t *converged, float *posterior,
                  void *workspace, size_t ws_bytes, const met_tuning *tuning, void *stream);

/* ---- Batched decoding ------------------------------------------------------
 * Several decode jobs -- possibly different codes (rates), batch sizes and
 * iteration budgets -- in one HIP graph (set-up, iterations, outputs; cached
 * per configuration) whose iterations of all jobs are interleaved phase by
 * phase.  Each job's results are identical to met_decode's for the same
 * inputs (the same tile bodies decode them).  The iterations run as one
 * persistent launch (the default; its grid is sized to be resident at once
 * and steps through the phases of all jobs with a grid-wide barrier between
 * them) or as one launch per phase (MET_BATCH_PHASE_LAUNCHES and the stream
 * modes below); met_batched_autotune picks among them.  Where a job's (3,1) /
 * (2,1) check classes fill the GPU on their own, the phase schedules launch
 * them with the plain decoder's check kernel.  Batches holding codes with check degrees that have
 * no compiled shape run their check tiles with one step per wave, except the
 * (3,1) / (2,1) checks where the schedule gives them launches of their own
 * (phase launches without stagger, or on parallel streams). */
typedef struct {
  const met_code *code;
  const float *llr;     /* dev f32 [B][N] */
  const uint8_t *syn;   /* dev u8 [B][M] */
  int32_t B, max_iter;
  uint32_t flags;       /* MET_EARLY_EXIT or MET_FIXED_ITERS */
  uint8_t *bits;        /* dev u8 [B][N] out */
  int32_t *iters;       /* dev i32 [B] out */
  uint8_t *converged;   /* dev u8 [B] out */
  float *posterior;     /* must be NULL (posteriors: use met_decode) */
} met_job;

/* Workspace bytes for these jobs.  Errors: MET_EINVAL. */
int met_batched_workspace_bytes(const met_job *jobs, int32_t n_jobs, size_t *bytes);

/* Enqueues all jobs on `stream` (tuning may be NULL).  The workspace (256-byte
 * aligned) must not be shared with overlapping calls.  After the stream has
 * drained, met_batched_check tells whether the persistent launch's barrier
 * ever expired (which happens only if its blocks were not all resident, e.g.
 * another process held compute units); results are then invalid.
 * Errors: MET_EINVAL, MET_EHIP. */
int met_decode_batched(const met_job *jobs, int32_t n_jobs, void *workspace, size_t ws_bytes,
                       const met_tuning *tuning, void *stream);
int met_batched_check(const void *workspace, int32_t *barrier_expired);

/* Autotuner of the batched launch: times candidate launch shapes (check steps
 * per wave 4/2/1 x resident blocks per compute unit 6..2 with groups of 64
 * frames, and blocks per compute unit 6/4/2 with groups of 32 and of 16, then
 * the stagger of the fastest; then one launch per phase, MET_BATCH_PHASE_LAUNCHES,
 * for the same widths and steps, staggered or not) on the same jobs with every budget capped at probe_iters
 * iterations (0 selects 6), discards shapes whose barrier expired, and writes
 * the fastest to *best (its time per probe run to *best_ms if not NULL).
 * Synchronises `stream`; overwrites the jobs' outputs.  Results are cached per
 * device and job signature (code, sizes, budgets, flags) for the life of the
 * process.  Errors: MET_EINVAL, MET_EHIP. */
int met_batched_autotune(const met_job *jobs, int32_t n_jobs, void *workspace, size_t ws_bytes,
                         int32_t probe_iters, met_tuning *best, float *best_ms, void *stream);

/* Message of the last failing call on this thread ("" if none). */
const char *met_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MET_BP_H */
