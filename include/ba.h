/*
 * ba.h - C ABI of the MI355X (gfx950) Blahut-Arimoto engine for the
 * finite-length binary deletion channel BDC_d.
 *
 * The method (Pinto & Ribeiro, "Improved Capacity Upper Bounds for the Deletion
 * Channel using a Parallelized Blahut-Arimoto Algorithm"):
 *   inputs  x in {0,1}^n, outputs y in {0,1}^{<=n} (Section 2.2);
 *   W(y|x) = emb(y,x) d^(n-|y|) (1-d)^|y|, emb = number of embeddings of y in x
 *   as a subsequence (Section 2.2, numerator of P_{n,k});
 *   one BA iteration (Section 2.3, Algorithm 1):  q = W^T p,
 *   D(x) = sum_y W(y|x) log(W(y|x)/q(y)),  p <- p e^D / Z,
 *   with the Blahut bounds  L = log sum_x p(x) e^{D(x)} <= C_n(d) <= U = max_x D(x)
 *   and the stopping quantity max_x log(p_{t+1}(x)/p_t(x)) = U - L (Section 2.3).
 *
 * Conventions used by every entry point
 * -------------------------------------
 *  - String order: x = (x_0..x_{n-1}) is the index sum_i x_i 2^(n-1-i); an output
 *    y of length k has rank (2^k - 1) + sum_i y_i 2^(k-1-i).  Arrays over inputs
 *    have 2^n entries; arrays over outputs have 2^(n+1) - 1 entries.
 *  - Units: everything crossing this boundary is in bits (the paper's logarithm
 *    base, Section 2.1), except log-probability arrays (logp, theta), which are
 *    natural logarithms.
 *  - Memory: a context owns host state only.  All device memory the library
 *    uses is one caller-provided workspace (ba_workspace_bytes / ba_bind); the
 *    library never allocates device memory itself.  Pointers named *_dev are
 *    device pointers borrowed for the duration of the call; all other pointers
 *    are host pointers.  Work is queued on the bound HIP stream.
 *  - Errors: every int-returning call returns BA_OK (0) or a negative BA_E*
 *    code; nothing aborts, throws or exits.  Outputs are written only on BA_OK.
 *    ba_last_error() gives a message for the most recent failure on a context.
 *  - Threads: a context may be used by one host thread at a time.  Calls that
 *    overlap on one context race.
 */
#ifndef BA_H
#define BA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ba_ctx ba_ctx;

enum {
  BA_OK = 0,
  BA_EINVAL = -1,    /* an argument is out of range */
  BA_ENOMEM = -2,    /* host allocation failed, or the bound workspace is too small */
  BA_EDEVICE = -3,   /* a HIP call failed (message in ba_last_error) */
  BA_ESTATE = -4,    /* call not valid in the context's state (e.g. before ba_bind) */
  BA_ENUMERIC = -5   /* NaN or Inf found in a log-probability input or iterate */
};

/* Precision of the iteration.  Certification (ba_bounds, ba_run's checks,
 * ba_eval, ba_grad) is always FP64. */
enum {
  BA_PREC_FP64 = 0,     /* FP64 iterates, log domain */
  BA_PREC_FP32_LOG = 1  /* FP32 iterates in the log domain, FP64 certification */
};

/* How the two sweeps q = W^T p and W v are evaluated.  Both give the same
 * values (up to rounding order).
 *  BA_ENGINE_STREAM:   the paper's method (Sections 3-4): every nonzero W(y|x)
 *                      is generated on the fly by an exact integer embedding-count
 *                      DP over the subsequences of x and visited once per sweep
 *                      (scatter into q, gather for D).
 *  BA_ENGINE_FACTORED: the same two products evaluated position by position: the
 *                      deletion channel acts on each input bit independently, so
 *                      W^T p and W v factor into n sparse stages of width
 *                      2^(n+1); the nonzeros are never enumerated.
 *  BA_ENGINE_PULL:     q = W^T p in pull form (Section 5): every output y sums
 *                      over its length-n supersequences, enumerated by
 *                      Algorithms 5-6, with an embedding-count DP per pair; no
 *                      atomics and a fixed summation order (deterministic).  W v
 *                      as in BA_ENGINE_STREAM. */
enum {
  BA_ENGINE_STREAM = 0,
  BA_ENGINE_FACTORED = 1,
  BA_ENGINE_PULL = 2
};

/* ---- lifetime --------------------------------------------------------------- */

/* One instance: 1 <= n <= 20, 0 <= d <= 1.  FP64 iteration, FACTORED engine,
 * p_0 uniform (Section 2.3).  *out receives a new context (free with ba_free).
 * BA_EINVAL if n or d is out of range or out is NULL. */
int ba_init(int n, double d, ba_ctx **out);

/* A batch of `count` independent instances (1 <= count <= 4096), instance i with
 * length n[i] in [1, 20] and deletion probability d[i] in [0, 1].  Instances with
 * the same n share the embedding-count tables and are advanced by the same kernel
 * launches (Section 2.2: W depends on d only through the weights
 * d^(n-k) (1-d)^k).  prec is BA_PREC_*; cert_every >= 1 is the number of
 * iterations between FP64 certifications in ba_run.  Host arrays n and d are
 * copied. */
int ba_init_batch(int count, const int *n, const double *d, int prec, int cert_every,
                  ba_ctx **out);

/* A batch of exact deletion channels BDC_{n,k} (Section 2.2): on input x the
 * output is a uniformly random length-k subsequence position set, so
 * W(y|x) = emb(y,x)/C(n,k) for |y| = k and 0 otherwise; its capacity is C_{n,k}.
 * Bounds from ba_bounds/ba_run bracket C_{n,k}; combined over k they bound C_n(d)
 * by Lemma 2: C_n(d) <= sum_k C(n,k) d^(n-k) (1-d)^k C_{n,k}.  1 <= n[i] <= 20,
 * 0 <= k[i] <= n[i]; everything else as ba_init_batch.  ba_grad's dI/dd is
 * rejected (BA_EINVAL) for these instances. */
int ba_init_exact(int count, const int *n, const int *k, int prec, int cert_every, ba_ctx **out);

/* Select BA_ENGINE_*.  Allowed at any time after init; takes effect at the next
 * call that runs sweeps. */
int ba_set_engine(ba_ctx *c, int engine);

/* Stopping rule of ba_run.  BA_STOP_ITERATE (default): stop when the current
 * iterate's gap U - L is below the tolerance (the rule of Section 2.3).
 * BA_STOP_BEST: stop when the best certified bounds seen so far (max L, min U over
 * the iterates evaluated in FP64) are closer than the tolerance; the upper bound
 * is not monotone in the iteration count, so this can stop earlier.  Both report
 * valid bounds. */
enum { BA_STOP_ITERATE = 0, BA_STOP_BEST = 1 };
int ba_set_stop_rule(ba_ctx *c, int rule);

/* Symmetric iteration (Appendix A, Theorem 4: from the uniform law every BA iterate
 * of BDC_d and of BDC_{n,k} satisfies p(g x) = p(x) for g = complement and
 * reversal, and then q(g y) = q(y)).
 * enable = 1: complement.  The iterations of the factored engine evaluate only the
 * inputs x < 2^(n-1) and the stage entries whose first column bit is 0, reading the
 * other half from the complement (about half the memory traffic; same results up
 * to rounding).  Applies to groups with even n >= 4 and BA_TUNE_FACTORED_FUSE >= 1
 * (its kernels take two positions per launch).  At n = 20 with FP32 iterates, step
 * 1 and BA_TUNE_FACTORED_FUSE = 8 the iterations instead run the default plan's
 * kernels on half their rows and column tiles (the rows that start with 0, the
 * tiles whose first column bit is 0), writing log p at x and at cpl x.
 * enable = 2: complement and reversal.  As 1 for the factored engine; in addition
 * the iterations of the stream engine compute q = W^T p by Algorithm 7: only inputs
 * that are the smallest member of their orbit {x, cpl x, rev x, cpl rev x} are
 * visited, each nonzero adding (|O_x| / |O_y|) p(x) emb(y,x) to the output's orbit
 * representative, whose value the other members of the orbit then take.
 * Other groups, the pull engine, certification, ba_eval and ba_grad run the full
 * kernels.  Enabling it on a bound context checks that every iterate is invariant
 * (max |log p(x) - log p(g x)| <= 1e-9 nats for FP64, 1e-4 for FP32 iterates, over
 * the group's maps) and then makes it exactly so; BA_EINVAL (mode left off) if
 * not.  While enabled, ba_set_logp applies the same check after setting the law
 * and switches the mode off (BA_EINVAL) if it fails.  enable = 0 switches back to
 * the full kernels.  Off by default. */
int ba_set_symmetry(ba_ctx *c, int enable);

/* Update step of the iterations (ba_step, ba_run): log p <- log p + eta D - log
 * sum_x p e^{eta D}, i.e. p <- p e^{eta D} / Z, entropic mirror ascent on I(p) with
 * step eta; eta = 1 (default) is the BA update of Section 2.3 exactly.  The
 * reported and certified bounds L = log sum p e^D <= C <= max D stay valid for any
 * iterate; eta > 1 is not monotone in I and can oscillate for large eta (eta = 2
 * roughly halves the iterations the lower bound needs on the cases measured;
 * eta = 3 oscillated at n = 10, d = 0.67).  0 < eta <= 8, else BA_EINVAL. */
int ba_set_step(ba_ctx *c, double eta);

/* Floor of the iterates' log-probabilities (Section 2.3 leaves zero-probability
 * inputs untreated: at the BA optimum of BDC_d many inputs have p = 0, and their
 * log p falls without bound).  After every update and after ba_set_logp,
 * log p(x) >= max_x log p(x) - nats.  Defaults: 700 nats for BA_PREC_FP64 iterates,
 * 80 for BA_PREC_FP32_LOG (e^-80 is a normal float).  Allowed: 50 <= nats <= 700
 * (FP64) or <= 87 (FP32), else BA_EINVAL (below 50 nats the floored mass, up to
 * 2^n e^-nats, would no longer be negligible next to the iterate's own bounds).  A
 * lower floor lets an input whose D(x) rises above L again recover sooner; the
 * certified bounds hold for any full-support law, so they stay valid.  Certification (ba_bounds, ba_run's
 * checks, ba_eval, ba_grad) always floors at 700 nats. */
int ba_set_floor(ba_ctx *c, double nats);

/* Run ba_run's iteration chunks as one captured HIP graph (replayed until the
 * stopping rule holds) instead of individual launches.  Needs a non-null bound
 * stream (capture is not allowed on the legacy null stream): BA_ESTATE otherwise,
 * reported by ba_run.  The graph is rebuilt after ba_bind, ba_set_engine,
 * ba_set_tuning, ba_set_step, ba_set_symmetry or a change of chunk length. */
int ba_set_graphs(ba_ctx *c, int enable);

/* Tuning knobs (they never change results beyond rounding order).
 *  BA_TUNE_SCATTER_LDS_KB: LDS budget (1..160 KB, default 64) of the stream
 *  engine's scatter; outputs short enough for the budget are accumulated in LDS
 *  before going to device memory.  Capped by the device's per-block limit. */
enum {
  BA_TUNE_SCATTER_LDS_KB = 0,
  /* BA_TUNE_FACTORED_FUSE: positions per launch of the factored engine: 8 (default)
   * as 7, and at n >= 12 (FP32 iterates, step 1, full kernels) inside one ba_step
   * call from its second iteration on, the D launch of every iteration but the last
   * also makes the next iteration's update and first eight forward positions on the
   * same inputs (the new log p shifted by the previous iteration's max of log p + D
   * instead of the current one: iterates equal to FP32 rounding); 7
   * as 6, and at n = 20 (FP32 iterates) the forward sweep in two launches: its
   * first eight positions and its last twelve (one block per row of the eighth
   * stage of output length 8, which recomputes that row's ancestors; three
   * four-position steps through LDS), the same sums in the same order as four
   * positions per launch; 6 as 5, and at n >= 12 with FP32 iterates the backward
   * sweep's first eight positions in one launch with D and the block maxima of
   * log p + D, so that an update left to the next iteration's first launch shifts by
   * that max instead of normalising (no final-record launch; iterates equal to FP32
   * rounding), the launches before it stopping at position 8 (at n = 20 one launch
   * of the last twelve positions, three four-position steps through LDS; the same
   * sums in the same order as four positions per launch); 5
   * as 4, with the forward's first eight positions in one launch (two four-position
   * steps through LDS, the same sums in the same order; n >= 12); 4 as 3, with the
   * forward's last four positions in one launch whose outputs are staged in LDS
   * (n >= 12); 3 as 2, with the backward's four-position launches paired into
   * eight-position launches (the same sums in the same order) while four positions
   * remain for the last launch; 2 four (the forward's last 1-4 positions and the
   * backward's first n mod 4 two or one at a time), 1 two, 0 one.  The
   * complement-symmetric kernels take at most level 4 in the forward sweep and 3 in
   * the backward sweep. */
  BA_TUNE_FACTORED_FUSE = 1,
  /* BA_TUNE_CONCURRENT_GROUPS: 1 (default) gives every group of instances (one
   * length n) its own branch of the graph that ba_run captures (ba_set_graphs), so
   * the groups' launches run concurrently; 0 captures them one group after another
   * on the bound stream.  The iterates are the same either way (groups share no
   * arrays).  Eager launches (ba_step) always use the bound stream. */
  BA_TUNE_CONCURRENT_GROUPS = 2,
  /* BA_TUNE_PERSISTENT: all iterations of one ba_step call (or of one ba_run chunk)
   * of a group with n <= 13 (FP32 iterates) or n <= 12 (FP64) as one launch: one
   * block per instance iterates it with every intermediate array in LDS, one input
   * position per stage (factored engine, not with ba_set_symmetry; timed as
   * BA_K_SWEEP1 by ba_time_kernels).  0: never (the launch chain); 1 (default):
   * for n <= 11, and for any such group of a context with several groups (its
   * launch then overlaps the other groups' launches); 2: whenever the group fits.
   * Same iteration up to the order of additions. */
  BA_TUNE_PERSISTENT = 3,
  /* BA_TUNE_STAGE8_COLUMNS: log2 of the columns each block of the factored engine's
   * eight-position backward launches covers (with correspondingly more subtree
   * roots per block): 0 (default) as many as the rows hold up to 16 (FP32) or 8
   * (FP64), else 1 .. 4 (FP32) / 1 .. 3 (FP64), capped by the row width.  The same
   * sums in the same order (bitwise-equal iterates). */
  BA_TUNE_STAGE8_COLUMNS = 4,
  /* BA_TUNE_PERSIST_THREADS: threads per block of the persistent launch (256, 512
   * or 1024, the default). */
  BA_TUNE_PERSIST_THREADS = 5
};
int ba_set_tuning(ba_ctx *c, int key, int value);

/* Free the host state.  The workspace stays owned by the caller.  NULL is a no-op. */
void ba_free(ba_ctx *c);

/* ---- memory and stream -------------------------------------------------------- */

/* Bytes of device workspace the context needs (alignment 256). */
int ba_workspace_bytes(const ba_ctx *c, size_t *bytes);

/* Bind a caller-owned device workspace of at least ba_workspace_bytes bytes
 * (256-byte aligned) and a HIP stream (hipStream_t, may be NULL for the null
 * stream).  Builds the count tables and the per-instance constants on the
 * stream and resets every instance to p_0 = uniform.  Can be called again to
 * move the context to another workspace (state is reset).  BA_ENOMEM if bytes is
 * too small, BA_EINVAL if the pointer is NULL or misaligned. */
int ba_bind(ba_ctx *c, void *workspace_dev, size_t bytes, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): ba_bind without a
 * workspace.  The context is bound to a device array owned by the library, one
 * copy per GPU (32 MiB, held until the process ends), on the device current on the
 * calling thread; hip_stream must belong to that device (may be NULL).  Enough for
 * one FP64 instance up to n = 16 or a small batch: BA_ENOMEM, with the sizes in
 * ba_last_error, if ba_workspace_bytes exceeds 32 MiB.  Does what ba_bind does
 * (count tables, constants, H, uniform start; everything the iterations read is
 * written first, so the array's previous contents do not matter) and calls no
 * device allocation routine.  Every context bound this way on one GPU shares that
 * GPU's array: binding one takes it from the previous one, whose later calls
 * return BA_ESTATE until it is bound again, and calls that overlap on one GPU race.
 * ba_bind or ba_free releases the array. */
int ba_bind_static(ba_ctx *c, void *hip_stream);

/* ---- iteration ---------------------------------------------------------------- */

/* Queue `iters` >= 0 BA iterations (Section 2.3: output law, refined input law,
 * normalisation) for every instance that has not converged.  Asynchronous: no
 * host synchronisation.  An instance whose current-iterate gap U - L (in the
 * iteration precision) falls below its tolerance (see ba_run) stops updating.
 * FP32 iterates with eta = 1 at n = 20 (factored engine, default launch plan)
 * are scaled by a max shift instead of normalised between the iterations of one
 * call (the sweeps do not depend on the scale; the last update of the call
 * normalises): after the first iteration the shift is the max of log p + D, from
 * the third on that of the iteration before (the new log p then lies at most n ln 2
 * above 0), so their in-call L, U and I are not formed; the iterate a call leaves
 * is normalised.  BA_ESTATE before ba_bind. */
int ba_step(ba_ctx *c, int iters);

/* Iterate until the FP64-certified gap U - L is below gap_bits for every instance
 * or until max_iters further iterations, certifying every cert_every iterations
 * (FP32 iterates; FP64 iterates are tested every iteration on the device).
 * Synchronises once per chunk of iterations; while no instance is frozen the
 * chunk's sweep kernels skip the per-instance frozen-flag test (the kernels that
 * write the iterate always make it).  Instances that already meet gap_bits
 * stay frozen, so repeated calls continue a run.
 * *iters_done (host, may be NULL) receives the number of iterations performed by
 * the slowest instance.  The stopping rule is that of Section 2.3 with the
 * tolerance in bits. */
int ba_run(ba_ctx *c, double gap_bits, int max_iters, int *iters_done);

/* FP64 certification of the current iterate of every instance: lower and upper
 * bounds on C_n(d) in bits (lower <= C_n(d) <= upper).  The iterate is first
 * normalised and floored at (max log p - 700) so that every input keeps a
 * representable probability; the bounds are valid for that full-support law.
 * lower_bits/upper_bits are host arrays of length count.  Blocks. */
int ba_bounds(ba_ctx *c, double *lower_bits, double *upper_bits);

/* Best certified bounds seen so far (max lower, min upper) over the FP64 iterates
 * (BA_PREC_FP64: every iteration) and the certifications of ba_run/ba_bounds,
 * host arrays of length count; and completed iterations per instance (host int
 * array of length count, may be NULL).  Blocks. */
int ba_best_bounds(ba_ctx *c, double *lower_bits, double *upper_bits, int *iters);

/* ---- single-instance evaluation hooks (count == 1 contexts, or instance 0) -------- */

/* FP64 evaluation at an arbitrary log-probability vector logp_dev (2^n doubles,
 * not necessarily normalised; normalised and floored as in ba_bounds).  Optional
 * outputs (NULL to skip):
 *   r_dev[2^(n+1)-1]  r(y) e^{-M} = sum_x p(x) emb(y,x) e^{-M}, M = max of the
 *                     normalised floored log p (so q(y) = w_k r(y) e^M);
 *   D_dev[2^n]        D(x) in nats;
 *   out4 (host[4])    {L bits, U bits, I bits, M nats}.
 * Does not change the iterate.  Blocks. */
int ba_eval(ba_ctx *c, const double *logp_dev, double *r_dev, double *D_dev, double *out4);

/* Mutual information and its gradients for p = softmax(theta), theta_dev[2^n]
 * (FP64 device array): *I_bits = I(p; d); dI_dtheta_dev[2^n] (device, may be
 * NULL) = p (D - I) / ln 2;  *dI_dd_bits (host, may be NULL) =
 * sum_x p(x) sum_y s_k W(y|x) log(W(y|x)/q(y)) / ln 2 with
 * s_k = (n-k)/d - k/(1-d).  BA_EINVAL for d in {0, 1} when dI_dd_bits is
 * requested.  Does not change the iterate.  Blocks. */
int ba_grad(ba_ctx *c, const double *theta_dev, double *I_bits, double *dI_dtheta_dev,
            double *dI_dd_bits);

/* Entropic mirror ascent on I(softmax(theta)): `steps` times
 * theta <- theta + eta * D(theta), in place on theta_dev[2^n] (FP64).  eta = 1
 * reproduces the BA update.  Asynchronous. */
int ba_mirror_ascent(ba_ctx *c, double *theta_dev, double eta, int steps);

/* Copy the current iterate (natural log of p, normalised) of every instance into
 * logp_dev (device, FP64, instances concatenated in order, 2^n[i] each), or load
 * it from there (not necessarily normalised; resets convergence flags).
 * BA_ENUMERIC if the loaded values contain NaN or +Inf. */
int ba_get_logp(ba_ctx *c, double *logp_dev);
int ba_set_logp(ba_ctx *c, const double *logp_dev);

/* ---- embedding counts (parity hooks for the count generator) ---------------- */

/* Row x of the embedding-count matrix of instance 0's n, computed on the device
 * by the same count generator the sweeps use: rank_dev[i], emb_dev[i] (device
 * uint32 arrays of capacity cap) in increasing rank order, *nnz (host) = number
 * of distinct subsequences of x.  BA_EINVAL if x >= 2^n or cap < nnz (then
 * *nnz is still set and nothing is written).  Blocks. */
int ba_row_counts(ba_ctx *c, uint32_t x, uint32_t *rank_dev, uint32_t *emb_dev, int cap,
                  int *nnz);

/* Whole-matrix check of the count generator for instance 0's n, on the device:
 * stats (host uint64[6]) = {total nonzeros, rows whose length sums
 * sum_{|y|=k} emb(y,x) differ from C(n,k) for some k, 0 (reserved), minimum row
 * nnz, maximum row nnz, maximum emb}.  Expected: total = 2*3^n - 2^n, 0 failing
 * rows, min nnz = n+1, max emb = C(n, floor(n/2)).  Blocks. */
int ba_verify_counts(ba_ctx *c, uint64_t *stats);

/* ---- introspection ------------------------------------------------------------ */

int ba_instance_count(const ba_ctx *c);
/* Nonzeros of W for length n: 2*3^n - 2^n. */
uint64_t ba_nnz(int n);
const char *ba_strerror(int code);
const char *ba_last_error(const ba_ctx *c);

/* ---- measurement ---------------------------------------------------------------- */

/* Run `iters` iterations (like ba_step) with a HIP event pair around every kernel
 * launch, on the bound stream, and report the summed device time per kernel
 * class in ms (host double[BA_NKCLASS], indexed by BA_K_*) together with the
 * number of launches per class (host int[BA_NKCLASS], may be NULL).  Blocks. */
enum {
  BA_K_SWEEP1 = 0,   /* q = W^T p  (stream: scatter kernel; factored: forward stages) */
  BA_K_LOGR = 1,     /* v(y) = w_k log r(y) */
  BA_K_SWEEP2 = 2,   /* W v        (stream: gather kernel; factored: backward stages) */
  BA_K_REDUCE = 3,   /* D, partial maxima and log-sum-exp */
  BA_K_UPDATE = 4,   /* normalisation and log p update */
  BA_NKCLASS = 5
};
int ba_time_kernels(ba_ctx *c, int iters, double *ms, int *launches);

#ifdef __cplusplus
}
#endif

#endif /* BA_H */
