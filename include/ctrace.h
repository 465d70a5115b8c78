/*
 * ctrace — CT-HYB local trace on one MI355X (gfx950), C ABI.
 *
 * What it computes (Sec. 2.2, the local weight w_loc, evaluated in the block
 * form of Sec. 3.3.1):
 *
 *   w_loc(C) = Tr[ P(beta - tau_n) O_n P(tau_n - tau_{n-1}) ... O_1 P(tau_1) ]
 *            = sum_{q0} Tr[ P(q0) F_n(q_{n-1}) ... P(q1) F_1(q0) P(q0) ],
 *
 * with P(x) = exp(-x H_loc) diagonal in the H_loc eigenbasis, O_j an
 * annihilator or creator, F_alpha(q) its dense block from sector q to sector
 * s_alpha(q), and the sum running over the start sectors q0 whose sector
 * string q0 -> q1 -> ... returns to q0 without entering the zero sector.
 * The time-ordering sign is not applied: the caller passes the operators
 * already in time order, as in the naive form of Sec. 3.3.1.
 *
 * Conventions used by every entry point
 *  - Operator code: op = 2*flavor + dagger (dagger = 1 for c+).  op[0] at
 *    tau[0] acts first (rightmost factor).  tau is non-decreasing in
 *    [0, beta); equal times are applied in array order.
 *  - Values: trace = (re + i*im) * exp(log_scale).  The split between
 *    mantissa and scale is not unique; compare values, not fields.
 *  - Streams: all device work is enqueued on the hipStream_t given to
 *    ctr_create.  Host-pointer entry points return after the result is on
 *    the host; *_device entry points only enqueue.
 *  - Memory: the library never allocates device memory.  Everything it
 *    keeps (operator blocks, tables, kernel buffers, per-call scratch) is carved out of the
 *    arena the caller passes to ctr_create (pre-allocated device pool, as in
 *    Sec. 3.3.2), except the per-call scratch of ctr_trace_batch_device_static,
 *    which lives in a fixed array of the library's code object on every
 *    device.  Running out of arena returns CTR_ERR_OOM and leaves the
 *    context usable.
 *  - Threads: a context is not thread safe; use one per host thread.
 *  - Errors: no exceptions cross the ABI; ctr_last_error gives detail.
 */
#ifndef CTRACE_H
#define CTRACE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CTR_ABI_VERSION 1

typedef enum {
  CTR_OK = 0,
  CTR_ERR_ARG = -1,         /* bad pointer, size or table content */
  CTR_ERR_OOM = -2,         /* arena too small for this call (context still usable) */
  CTR_ERR_DEVICE = -3,      /* a HIP runtime call failed */
  CTR_ERR_UNSORTED = -4,    /* tau not non-decreasing */
  CTR_ERR_RANGE = -5,       /* tau outside [0, beta) or operator code out of range */
  CTR_ERR_STATE = -6,       /* call needs ctr_set_impurity first */
  CTR_ERR_UNSUPPORTED = -7, /* impurity or option outside what the kernels handle */
  CTR_ERR_BUSY = -8         /* serving: the impurity's queue is full; submit again later */
} ctr_status;

/* ctr_opts.precision */
enum { CTR_FP64 = 0, CTR_FP32_SPLIT = 1 };

/* ctr_value.flags bits */
enum {
  CTR_FLAG_ZERO = 1,      /* no sector string survives: the trace is exactly 0 */
  CTR_FLAG_REJECTED = 2,  /* lazy call: bound below threshold, trace not evaluated */
  CTR_FLAG_INVALID = 4    /* device-input call: this configuration failed validation */
};

typedef struct ctr_ctx ctr_ctx;

typedef struct {
  double re, im;       /* mantissa of the trace (im = 0 for real impurities) */
  double log_scale;    /* trace = (re + i im) * exp(log_scale) */
  double log_bound;    /* log of the lazy upper bound on |trace| (same units);
                          -inf when no string survives */
  double log_abs;      /* log of the sum of the moduli of the evaluated contributions (per string
                          and column panel), same units: |trace| <= exp(log_abs), and
                          |trace| << exp(log_abs) marks a cancellation-dominated trace whose
                          rounding error scales with exp(log_abs); -inf when nothing was evaluated */
  int32_t n_strings;   /* number of surviving sector strings */
  int32_t flags;       /* CTR_FLAG_* */
} ctr_value;

/* ctr_opts.kernel: which chain kernel runs the block products */
enum {
  CTR_KERNEL_AUTO = 0,    /* the kernel ctr_tune picked, for non-lazy FP64 batches of at least a
                             quarter of its sample; otherwise FP64 with sectors <= 128 states: the
                             wavefront kernel; else the block-grouped rounds (lazy calls included)
                             for batches of >= 48 traces, and for any batch once a sector exceeds
                             384 states (their row-chunked items), while the arena holds their
                             scratch; else the LDS-resident workgroup kernel when the panel fits
                             LDS, else streaming.  FP32-split: the grouped split items for batches
                             of >= 48 or where the LDS kernel cannot run, else the LDS kernel */
  CTR_KERNEL_WAVE = 1,    /* one wavefront per 8-column panel; sectors <= 128 states, FP64 only */
  CTR_KERNEL_BLOCK = 2,   /* one workgroup per 16-column panel, X in LDS (<= 1024 real / 576 complex) */
  CTR_KERNEL_STREAM = 3,  /* one workgroup per 16-column panel, X in global memory; any size, FP64 only */
  CTR_KERNEL_GROUPED = 4, /* block-grouped rounds: all strings of the batch advance one operator per
                             round and the strings at the same block share one wide product; FP64;
                             sectors <= 384 states keep every row of a block in one work item, larger
                             ones take the row-chunked items of CTR_KERNEL_GROUPED_ROWS; lazy calls
                             reject by the string bounds before the rounds (no refinement while strings
                             run).  Synchronises the stream once per batch (to size its scratch from
                             the number of surviving strings) */
  CTR_KERNEL_GROUPED_ROWS = 5 /* the block-grouped rounds with work items of 32 columns x 256 rows of a
                             block (FP32-split: 16 x 128) for any sector size: the per-column power of
                             two is a device-wide maximum over the row chunks, applied when the next
                             round loads the column */
};

typedef struct {
  int32_t precision;   /* CTR_FP64 (default) or CTR_FP32_SPLIT */
  int32_t slices;      /* CTR_FP32_SPLIT: 8-bit slices per operand, 6 (also for 0) or 7; seven cut the
                          truncation error ~256-fold for a third more FP32 products (28 instead of 21) */
  int32_t kernel;      /* CTR_KERNEL_*; a kernel that cannot run this impurity/precision
                          gives CTR_ERR_UNSUPPORTED */
  int32_t flags;       /* CTR_OPT_* bits; 0 for the defaults */
} ctr_opts;

/* ctr_opts.flags */
enum {
  CTR_OPT_GRAPH = 1    /* grouped rounds: the rounds of every chunk are built into one HIP graph (one
                          kernel node per round, each depending on the one before) and launched as one,
                          instead of one launch per round; the graph is instantiated per chunk (the
                          rounds and their work items depend on the batch).  Same kernels, same values;
                          ignored by the per-string kernels */
};

/*
 * The impurity in sector form (Sec. 3.3.1): sector dimensions, the H_loc
 * eigenvalues of every sector, the sector map s_alpha(q) and the annihilator
 * blocks in the eigenbases.
 *
 *  beta          inverse temperature (> 0)
 *  n_flavors     number of flavors (1..32); operator codes run over 2*n_flavors
 *  n_sectors     number of sectors
 *  is_complex    0: blocks are float64; 1: blocks are complex128 (interleaved re, im)
 *  sector_dim    [n_sectors] sector dimensions (>= 1)
 *  energies      [sum(sector_dim)] eigenvalues, sector after sector, in the
 *                order of that sector's basis (any order); unshifted (the
 *                library subtracts the global minimum and folds it into
 *                log_scale)
 *  next          [n_sectors * 2*n_flavors] row-major, next[q*2nf + op] = sector
 *                reached from q by operator op, or -1 (zero sector).  Must be
 *                consistent: next[q][2f+1] = p  <=>  next[p][2f] = q.
 *  blocks        [n_sectors * n_flavors] pointers: blocks[q*nf + f] is the
 *                annihilator block of flavor f leaving sector q, row-major
 *                dim(next[q][2f]) x dim(q), element [m][n] = <m| c_f |n>
 *                (reading of the index order of Sec. 3.3.1: output row first).
 *                NULL iff next[q][2f] == -1.  Creator blocks are not passed:
 *                the block of c+_f leaving q is the conjugate transpose of the
 *                annihilator block leaving next[q][2f+1].
 *  block_norm    optional [n_sectors * n_flavors] spectral norms of the blocks
 *                (used by the lazy bound); NULL means 1, exact for every
 *                nonzero block of c_f in an orthonormal eigenbasis.
 */
typedef struct {
  double beta;
  int32_t n_flavors;
  int32_t n_sectors;
  int32_t is_complex;
  int32_t reserved;              /* must be 0 */
  const int32_t *sector_dim;
  const double *energies;
  const int32_t *next;
  const void *const *blocks;
  const double *block_norm;
} ctr_impurity;

/* Library version string. */
const char *ctr_version(void);

/* Human-readable name of a status code. */
const char *ctr_status_string(ctr_status s);

/* Last error message of a context (empty string if none); valid until the
 * next call on the context. */
const char *ctr_last_error(const ctr_ctx *ctx);

/*
 * Create a context on HIP device `device`, sub-allocating from the caller's
 * device arena [arena, arena + arena_bytes) (alignment 256 bytes; the caller
 * keeps ownership and must keep it alive until ctr_destroy), enqueueing all
 * work on `hip_stream` (a hipStream_t, or NULL for the null stream).
 * Errors: CTR_ERR_ARG (null out/arena, arena < 1 MiB), CTR_ERR_DEVICE.
 */
ctr_status ctr_create(int device, void *arena, size_t arena_bytes, void *hip_stream, ctr_ctx **out);

/* Destroy a context (NULL allowed).  Waits for the context's stream. */
void ctr_destroy(ctr_ctx *ctx);

/*
 * Load an impurity: validates the tables, copies energies, tables and
 * blocks to the arena in the kernels' layout (column-major, zero padded,
 * creator blocks materialised, complex split into planes).  Host buffers
 * are read during the call only.  Replaces any previous impurity and
 * resets the arena.  Errors: CTR_ERR_ARG (inconsistent tables, missing
 * block), CTR_ERR_OOM, CTR_ERR_UNSUPPORTED (more than 32767 sectors),
 * CTR_ERR_DEVICE.
 */
ctr_status ctr_set_impurity(ctr_ctx *ctx, const ctr_impurity *imp);

/* Bytes of the arena in use by the loaded impurity. */
size_t ctr_arena_resident_bytes(const ctr_ctx *ctx);

/*
 * One trace.  tau[n_ops], op[n_ops] are host arrays (0 <= n_ops <= 512; 0
 * gives the partition function Z = Tr exp(-beta H)).  opts may be NULL (FP64).
 * Errors: CTR_ERR_UNSORTED, CTR_ERR_RANGE, CTR_ERR_STATE, CTR_ERR_OOM,
 * CTR_ERR_DEVICE.  A configuration none of whose strings survives returns
 * CTR_OK with flags CTR_FLAG_ZERO and re = im = 0.
 */
ctr_status ctr_trace(ctr_ctx *ctx, int32_t n_ops, const double *tau, const int32_t *op,
                     const ctr_opts *opts, ctr_value *out);

/*
 * n_cfg traces in one pass.  Configuration c is tau[offsets[c] ..
 * offsets[c+1]), op[same]; offsets has n_cfg + 1 entries, offsets[0] = 0.
 * All host arrays; out[n_cfg] host.  Large batches are split internally
 * to fit the arena.  Errors as ctr_trace (the first invalid configuration
 * fails the whole call before any device work).
 */
ctr_status ctr_trace_batch(ctr_ctx *ctx, int32_t n_cfg, const int64_t *offsets, const double *tau,
                           const int32_t *op, const ctr_opts *opts, ctr_value *out);

/*
 * Same as ctr_trace_batch with every array already in device memory
 * (d_offsets[n_cfg+1], d_tau, d_op, d_out[n_cfg]); enqueues work on the
 * context's stream and returns without waiting, except that the
 * block-grouped kernel (CTR_KERNEL_GROUPED, or AUTO choosing it) waits once
 * per chunk for the number of surviving strings, which sizes its scratch.
 * Validation happens on the device: an invalid
 * configuration gets CTR_FLAG_INVALID and re = im = 0.  Errors:
 * CTR_ERR_OOM (per-call scratch does not fit; the call is split into
 * chunks first, so this means even one configuration does not fit),
 * CTR_ERR_STATE, CTR_ERR_DEVICE.
 */
ctr_status ctr_trace_batch_device(ctr_ctx *ctx, int32_t n_cfg, const int64_t *d_offsets,
                                  const double *d_tau, const int32_t *d_op, const ctr_opts *opts,
                                  ctr_value *d_out);

/*
 * For callers that cannot allocate device memory per call (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same traces as ctr_trace_batch_device, with the per-call scratch (string
 * records, panel results, per-configuration counters) taken from a fixed
 * array of CTR_STATIC_SCRATCH_BYTES that the library keeps on every device it
 * runs on until the process ends, instead of from the context's arena.  The
 * call allocates nothing (no hipMalloc, no events) and only enqueues work.
 * It runs the per-string chain kernels (AUTO never takes the grouped rounds
 * here; asking for CTR_KERNEL_GROUPED or CTR_KERNEL_GROUPED_ROWS gives
 * CTR_ERR_UNSUPPORTED).  A batch
 * whose scratch exceeds the array is rejected with CTR_ERR_OOM before any
 * device work (the message states the bytes it needs); it is not split.
 * Every call on one device shares that device's array: calls whose work
 * overlaps on the device (other streams, other contexts or threads) race and
 * must be serialised by the caller.  Other arguments and errors as
 * ctr_trace_batch_device.
 */
#define CTR_STATIC_SCRATCH_BYTES (64u << 20)
ctr_status ctr_trace_batch_device_static(ctr_ctx *ctx, int32_t n_cfg, const int64_t *d_offsets,
                                         const double *d_tau, const int32_t *d_op, const ctr_opts *opts,
                                         ctr_value *d_out);

/*
 * Lazy traces (Sec. 3.3.1, lazy-trace bounds): per configuration, the
 * upper bound B = sum_s rank_s * prod ||P|| * prod ||F|| (spectral norms,
 * exact for the diagonal propagators) is computed first; if
 * log(B) < log_threshold[c] the configuration is reported with
 * CTR_FLAG_REJECTED and not evaluated, otherwise the exact trace is
 * returned.  Host arrays as in ctr_trace_batch.
 */
ctr_status ctr_trace_lazy_batch(ctr_ctx *ctx, int32_t n_cfg, const int64_t *offsets, const double *tau,
                                const int32_t *op, const double *log_threshold, const ctr_opts *opts,
                                ctr_value *out);

/*
 * One lazy trace (Sec. 3.3.1): ctr_trace_lazy_batch of the single
 * configuration (tau[n_ops], op[n_ops], host arrays) against log_threshold;
 * *out as there.  Same arguments and errors as ctr_trace.
 */
ctr_status ctr_trace_lazy(ctr_ctx *ctx, int32_t n_ops, const double *tau, const int32_t *op, double log_threshold,
                          const ctr_opts *opts, ctr_value *out);

/*
 * Histogram of a conserved sector label (Sec. 2.3.2, the estimator of the
 * impurity density matrix, tau-integrated, summed over the states of every
 * label; Sec. 4.2, the valence histogram over N).  For configuration c and
 * label l,
 *
 *   h_l(C) = beta^-1 int_0^beta w_loc(C, P_l(tau)) dtau / w_loc(C),
 *
 * P_l = projector onto the sectors q with sector_label[q] == l.  Such a
 * projector commutes with H_loc, so the integral is the sum over the
 * surviving sector strings s of w_s * (time s spends in label-l sectors),
 * divided by beta * w_loc.
 *
 *  sector_label  host [n_sectors], values 0 .. n_labels-1 (CTR_ERR_RANGE otherwise)
 *  n_labels      1 .. CTR_MAX_LABELS
 *  out           host [n_cfg] traces, as ctr_trace_batch
 *  hist          host [n_cfg * n_labels * 2]: h_l(C) of configuration c at
 *                hist[2*(c*n_labels + l)] (real part) and [.. + 1] (imaginary
 *                part; zero for real impurities).  All zeros for a
 *                configuration whose trace is zero or invalid.
 * The labels of a nonzero configuration sum to 1 up to rounding.  Other
 * arguments and errors as ctr_trace_batch; any chain kernel and precision.
 */
#define CTR_MAX_LABELS 4096
ctr_status ctr_trace_histogram(ctr_ctx *ctx, int32_t n_cfg, const int64_t *offsets, const double *tau,
                               const int32_t *op, const int32_t *sector_label, int32_t n_labels,
                               const ctr_opts *opts, ctr_value *out, double *hist);

/*
 * The impurity density-matrix estimator (Sec. 2.3.2), tau-integrated, summed
 * over a batch with caller weights.  For configuration C with trace w(C) != 0
 *
 *   R(C) = (beta w(C))^-1 int_0^beta A(tau) dtau,
 *
 * where A(tau) is the time-ordered product cut at tau and closed the other
 * way round (the product that starts and ends at tau, Tr A(tau) = w(C)); it is
 * block diagonal in the sectors and Tr R(C) = 1.  The tau integral over every
 * interval between operators is done in closed form in the eigenbasis.
 *
 *  weight   host [n_cfg][2] complex weights (re, im) or NULL for 1 each
 *  out      host [n_cfg] traces of the configurations (as ctr_trace_batch)
 *  rho      host [sum_q dim_q^2][2]: sum_C weight_C R(C), sector after sector,
 *           each block row-major [u][v] over the sector's eigenbasis (the order
 *           of its energies), complex interleaved; overwritten.  Configurations
 *           whose trace is zero contribute nothing.
 * Host arrays as ctr_trace_batch; the batch is not split (CTR_ERR_OOM when it
 * does not fit the arena).  FP64.  Errors: CTR_ERR_UNSUPPORTED for sectors of
 * more than 1024 states, and those of ctr_trace_batch.
 */
ctr_status ctr_density_matrix(ctr_ctx *ctx, int32_t n_cfg, const int64_t *offsets, const double *tau,
                              const int32_t *op, const double *weight, ctr_value *out, double *rho);

/*
 * Markov chains around the trace (Sec. 2.3.1 sampling; App. C
 * Metropolis-Hastings; App. D Pauli-aware pair insertion and removal;
 * Sec. 2.2 w_hyb).  Each chain holds a configuration, its |w_loc| and the
 * inverse of every flavor's hybridisation block M_f[r][s] = Delta_f(tc_r -
 * ta_s) (creators r, annihilators s), with
 *
 *   Delta_f(x) = -sum_k V_fk^2 exp(-x eps_fk) / (1 + exp(-beta eps_fk)),  0 < x < beta,
 *   Delta_f(x - beta) = -Delta_f(x)            (a discrete bath per flavor).
 *
 * A step proposes one move per chain from six caller-drawn uniforms u[0..5]
 * in [0, 1) (u0 < 1/2 insert, else remove; u1 flavor = floor(u1 n_f); u2 the
 * operator after which to insert, or the first of the pair to remove, among
 * the flavor's N operators; u3, u5 the two times inside that interval (u2,
 * u3 scaled by beta for an empty flavor: creator at u2 beta, annihilator at
 * u3 beta); u4 the Metropolis uniform, drawn first).  Proposal ratios:
 * insertion N d^2 / (2 (N + 2)) (d = length of the interval), beta^2 into an
 * empty flavor; removal the inverse of the insertion that undoes it.  The
 * sampled weight is |w_loc w_hyb|: a move is accepted iff
 * q |w_hyb'/w_hyb| |w_loc'| >= u4 |w_loc|.  The hybridisation ratio comes
 * from a fast update of the inverse on the host (O(k^2)); the local traces
 * of all chains' proposals are one ctr_trace_lazy_batch call per step with
 * threshold log(u4 |w_loc| / (q |w_hyb'/w_hyb|)).
 *
 *  opts->n_chains      number of chains (>= 1); all start at order zero
 *  opts->n_bath        levels per flavor (>= 0), bath_eps / bath_v [n_flavors * n_bath]
 *  opts->rebuild_every accepted moves of a flavor between recomputations of its
 *                      inverse from scratch (0: 64)
 *  opts->full_traces   0 or 1 (see the struct); both take the same decisions
 * The context must stay alive and loaded while the chains exist.
 */
typedef struct ctr_mc ctr_mc;
typedef struct {
  int32_t n_chains;
  int32_t n_bath;
  const double *bath_eps;
  const double *bath_v;
  int32_t rebuild_every;
  int32_t full_traces;           /* 0: lazy batch (proposals stop at their bound); 1: full traces, the
                                    decision taken on the host from the exact values */
} ctr_mc_opts;

/* Errors: CTR_ERR_ARG, CTR_ERR_STATE (no impurity), trace errors. */
ctr_status ctr_mc_create(ctr_ctx *ctx, const ctr_mc_opts *opts, ctr_mc **out);
/* Replaces chain `chain`'s configuration (host arrays, strictly increasing
 * times, every flavor alternating between creators and annihilators).
 * CTR_ERR_ARG if a flavor is unbalanced or not alternating, or a weight is
 * zero; CTR_ERR_RANGE / CTR_ERR_UNSORTED as ctr_trace. */
ctr_status ctr_mc_set_config(ctr_mc *mc, int32_t chain, int32_t n_ops, const double *tau, const int32_t *op);
/* One move per chain.  u: host [n_chains * 6] uniforms in [0, 1)
 * (CTR_ERR_RANGE otherwise).  decision (host [n_chains], may be NULL): 1
 * accepted, 0 rejected, -1 no proposal (nothing to remove, coinciding times,
 * more than 512 operators).  Synchronous. */
ctr_status ctr_mc_step(ctr_mc *mc, const double *u, int32_t *decision);
/* Chain `chain`'s configuration into tau/op (capacity cap; *n_ops is set even
 * when it does not fit, then CTR_ERR_ARG) and, if log_w is not NULL,
 * log_w[0] = log|w_loc|, log_w[1] = log|w_hyb|. */
ctr_status ctr_mc_config(const ctr_mc *mc, int32_t chain, int32_t cap, double *tau, int32_t *op, int32_t *n_ops,
                         double *log_w);
/* Totals since creation: steps, proposals, proposals rejected by the lazy bound, accepted moves. */
ctr_status ctr_mc_stats(const ctr_mc *mc, int64_t *n_steps, int64_t *n_proposed, int64_t *n_lazy_rejected,
                        int64_t *n_accepted);
/* Wall time since creation spent in ctr_mc_step's host passes (proposals,
 * hybridisation updates, batch assembly) and inside its trace batches. */
ctr_status ctr_mc_timing(const ctr_mc *mc, double *host_ms, double *trace_ms);
void ctr_mc_destroy(ctr_mc *mc);

/* Log of the lazy upper bound on |trace| for one configuration (-inf if no
 * string survives).  Host arrays. */
ctr_status ctr_bound(ctr_ctx *ctx, int32_t n_ops, const double *tau, const int32_t *op, double *log_bound);

/*
 * Sector strings of one operator string (Sec. 3.3.1, the map s_alpha(q)):
 * writes the start sectors q0 whose string survives, ascending, into
 * q0_out[0 .. *n_out) (q0_out must hold n_sectors entries).  Computed by
 * the same device kernel the traces use.
 */
ctr_status ctr_strings(ctr_ctx *ctx, int32_t n_ops, const int32_t *op, int32_t *q0_out, int32_t *n_out);

/*
 * Autotuning of the chain kernel and its tile shape (8-column panels on
 * 4x4x4 MFMA, 16-column panels on 16x16x4, grouped items of 16/32/64
 * columns; the grouped rounds in each of their tile shapes for this
 * impurity).  Evaluates the sample batch (host arrays, as ctr_trace_batch)
 * once with every kernel and shape that can run it in FP64, timing each second
 * run with HIP events.  The grouped rounds keep their fastest shape (for
 * every later call that runs them), and the fastest kernel becomes the
 * choice of CTR_KERNEL_AUTO for FP64 batches of at least n_cfg / 4 traces
 * (smaller batches and lazy or
 * FP32-split calls keep the built-in choice) until the next
 * ctr_set_impurity.  *chosen (may be NULL) receives the CTR_KERNEL_* picked;
 * ms_per_kernel (may be NULL) receives 5 entries indexed by CTR_KERNEL_*,
 * the measured milliseconds (the best shape's for the grouped rounds) or -1
 * where a kernel did not run.
 */
ctr_status ctr_tune(ctr_ctx *ctx, int32_t n_cfg, const int64_t *offsets, const double *tau, const int32_t *op,
                    int32_t *chosen, double *ms_per_kernel);

/*
 * The chain kernel (CTR_KERNEL_WAVE .. CTR_KERNEL_GROUPED_ROWS, never AUTO;
 * 0 before any trace call) and the FP32-split slices (0 for FP64) of the last
 * trace call on the context, as AUTO resolved them (for reports that name the
 * kernel they time).  slices may be NULL.  Errors: CTR_ERR_ARG.
 */
ctr_status ctr_last_kernel(const ctr_ctx *ctx, int32_t *kernel, int32_t *slices);

/* Wait for all work enqueued by the context. */
ctr_status ctr_synchronize(ctr_ctx *ctx);

/*
 * Measured peaks of the matrix units on the context's device (the roofline
 * of the chain kernels, Sec. 3.3.2 names the matrix multiplication as the
 * critical kernel): register-only loops of independent MFMA instructions,
 * eight wavefronts per SIMD, timed with HIP events on the context's stream.
 * out (host, 5 doubles): [0] FP64 MFMA 16x16x4 TFLOP/s, [1] FP64 MFMA 4x4x4
 * (four blocks) TFLOP/s, [2] FP32 MFMA 16x16x4 TFLOP/s, [3] the device's
 * reported clock in MHz, [4] compute units.  Uses 2 KiB of arena scratch.
 * Synchronous.  Errors: CTR_ERR_ARG, CTR_ERR_OOM, CTR_ERR_DEVICE.
 */
ctr_status ctr_probe_peaks(ctr_ctx *ctx, double *out);

/*
 * Instrumentation for roofline reports: when enabled (on != 0), every launch
 * of the chain kernel (the block-product loop) is bracketed by HIP events
 * recorded on the context's stream.  ctr_kernel_timing_read waits for the
 * stream, returns the summed duration in milliseconds and the number of
 * launches since the last read, and clears the record.
 */
ctr_status ctr_kernel_timing(ctr_ctx *ctx, int32_t on);
ctr_status ctr_kernel_timing_read(ctr_ctx *ctx, double *total_ms, int32_t *n_launches);

/*
 * Serving: continuous batching of trace requests from many Markov chains
 * (Sec. 3.2: many chains share one GPU; the lazy trace of Sec. 3.3.1 decides
 * their moves).  A server drives one or more contexts (one per impurity),
 * each from a worker thread of its own on the context's stream, so the
 * impurities' work overlaps on the device.  Requests are queued per impurity;
 * whenever a worker's device pass ends it admits the requests that arrived
 * meanwhile, in arrival order, up to max_batch and up to hbm_budget bytes of
 * per-call scratch, and runs them as one batch (ctr_trace_batch, or
 * ctr_trace_lazy_batch when any admitted request has a finite threshold).
 * Every result is the value the same request gets alone, up to the rounding
 * of the kernel the batch size selects.
 *
 * While a server runs, its contexts belong to it: the caller must not use
 * them.  Destroy the server before destroying the contexts.
 */
typedef struct ctr_server ctr_server;

typedef struct {
  int32_t max_batch;    /* most requests per device pass and impurity (>= 1) */
  int32_t max_pending;  /* most queued, not yet admitted requests per impurity (>= 1);
                           ctr_server_submit returns CTR_ERR_BUSY beyond it */
  size_t hbm_budget;    /* arena bytes a batch may occupy in its context's arena (per-call scratch and,
                           where the grouped rounds can run, the carried matrices of every surviving
                           sector string of the admitted configurations, estimated by walking the
                           sector map on the host); at least one request is always admitted;
                           0 = all of the arena not held by the impurity */
  const double *grid_share; /* optional [n_ctx] fractions in (0, 1]: each context launches only that
                           share of the workgroups of its persistent kernels while the server holds
                           it (grouped rounds keep at least 64), so that a long pass of one impurity
                           leaves slots on the device for the others' kernels; the contexts get the
                           whole device back at ctr_server_destroy.  NULL: every context launches
                           full grids */
  double max_pass_flop;  /* cap on the estimated block-product flops of one pass (every surviving string
                           at its narrowest width, 2 flops per multiply-add, 8 complex; host walk of the
                           sector map): a pass stops admitting once the next request would exceed it, so
                           long passes of a heavy impurity do not hold back requests that arrive
                           meanwhile; at least one request is always admitted; 0 = no cap */
} ctr_server_opts;

typedef struct {
  uint64_t tag;         /* the caller's tag of the request */
  int32_t impurity;     /* index of its context in ctr_server_create's list */
  int32_t status;       /* CTR_OK, or the error of the device pass that evaluated it */
  ctr_value value;      /* as ctr_trace / ctr_trace_lazy_batch */
  double latency_ms;    /* from ctr_server_submit to completion */
  int32_t batch;        /* number of requests in the device pass that evaluated it */
  int32_t reserved;
} ctr_result;

/*
 * Starts one worker thread per context.  ctxs[n_ctx] must each have an
 * impurity loaded.  Errors: CTR_ERR_ARG (bad options or contexts, a grid
 * share outside (0, 1]), CTR_ERR_STATE (a context without impurity).
 */
ctr_status ctr_server_create(ctr_ctx *const *ctxs, int32_t n_ctx, const ctr_server_opts *opts,
                             ctr_server **out);

/*
 * Queues one trace of impurity `impurity` (the configuration is copied; the
 * arrays may be reused on return).  log_threshold = -INFINITY asks for the
 * plain trace; a finite value makes it a lazy request (CTR_FLAG_REJECTED when
 * the bound is below it).  The configuration is validated here: errors
 * CTR_ERR_ARG, CTR_ERR_RANGE, CTR_ERR_UNSORTED as ctr_trace; CTR_ERR_BUSY when
 * max_pending requests of that impurity are waiting; CTR_ERR_STATE after
 * ctr_server_destroy began.
 */
ctr_status ctr_server_submit(ctr_server *srv, int32_t impurity, uint64_t tag, int32_t n_ops, const double *tau,
                             const int32_t *op, double log_threshold);

/*
 * Moves up to max completed results into out[] (completion order) and sets
 * *n_out.  wait != 0 blocks until at least one result is available or no
 * request is outstanding.
 */
ctr_status ctr_server_poll(ctr_server *srv, ctr_result *out, int32_t max, int32_t *n_out, int32_t wait);

/* Blocks until every submitted request has completed (results stay queued for poll). */
ctr_status ctr_server_drain(ctr_server *srv);

/* Device passes run and requests evaluated so far, per server. */
ctr_status ctr_server_stats(const ctr_server *srv, int64_t *n_passes, int64_t *n_requests);

/* Stops the workers after the requests already admitted, drops the rest, frees the server. */
void ctr_server_destroy(ctr_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* CTRACE_H */
