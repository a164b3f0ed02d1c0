// Internal declarations shared by the HIP sources of libba (not part of the ABI).
//
// Notation (paper, Sections 2.2-2.3): x in {0,1}^n is an input, y in {0,1}^{<=n}
// an output, emb(y,x) the number of embeddings of y in x, w_k = d^(n-k)(1-d)^k,
// W(y|x) = emb(y,x) w_|y|.  One BA iteration computes
//   r(y) = sum_x p(x) emb(y,x)          (so q(y) = w_k r(y)),
//   G(x) = sum_y emb(y,x) w_k log r(y),
//   D(x) = H(x) - G(x),  H(x) = sum_y emb(y,x) w_k log emb(y,x),
// because log(W/q) = log(emb/r): the weight w_k cancels.  Both sweeps work on
// r scaled by e^{-M} (M = max log p); the shift is undone in the D kernel
// (sum_y W(y|x) = 1).
//
// Instances that share n form a group; every per-instance array of a group is
// one allocation with a fixed stride per instance (instance b at b*stride).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ba {

constexpr int kNMax = 20;       // largest supported input length
constexpr int kHalfMax = 10;    // largest half length ceil(20/2)
constexpr int kWave = 64;       // CDNA wavefront
constexpr int kBlock = 256;     // threads per block
constexpr int kTile = 8;        // instances handled together by one stream-engine launch
constexpr double kLn2 = 0.69314718055994530942;
constexpr double kFloor64 = 700.0;  // floor on log p, nats below the max (FP64)
constexpr double kFloor32 = 80.0;   // floor on log p, nats below the max (FP32 iterates)
constexpr double kFloor32Max = 87.0;  // largest FP32 floor: e^-87 is still a normal float
// smallest floor: the floored mass, at most 2^20 e^-50 < 2.0e-16 of the total, stays
// below FP64 resolution, so the bounds the kernels form from an iterate without
// renormalising it after the floor are those of its normalised law
constexpr double kFloorMin = 50.0;
constexpr int kPartStride = 8;      // doubles per block record of a reduction
constexpr int kMaxRedBlocks = 1024; // blocks per instance of a reduction
// per-instance record buffer: block records [0, kMaxRedBlocks), a second set used
// by the normalisation passes, then the final (combined) record
constexpr int kFinalRec = 2 * kMaxRedBlocks * kPartStride;
constexpr int kPartDoubles = kFinalRec + kPartStride;

inline __host__ __device__ uint32_t out_count(int n) { return (2u << n) - 1u; }  // 2^(n+1)-1

// ---------------------------------------------------------------------------
// Count tables for one input length n, split as x = x1 x2 with |x1| = n1 =
// ceil(n/2) and |x2| = n2 = floor(n/2).
//
// Every distinct subsequence y of x factors uniquely as y = y1 y2 where y1 is
// the longest prefix of y that is a subsequence of x1 (the greedy, NextPos-based
// embedding of Section 4 uses x1 as far as it can) and y2 is a subsequence of x2;
// conversely a pair (y1 <= x1, y2 <= x2) arises this way iff y2 is empty or y1
// followed by the first bit of y2 is not a subsequence of x1.  The class of
// (x1, y1) records which bits can still extend y1 inside x1.
//
// T1 entry (16 bytes), one per (x1, y1 distinct subsequence of x1):
//   w.x = x1 | y1 << 10 | k1 << 20 | cls << 24
//   bytes 4..15: byte u = emb(y1[0:k1-u], x1), u = 0..k1   (<= C(10,5) = 252)
// classes, also the sort order of T1:
//   0: only bit 1 extends y1 in x1 -> compatible y2 start with 0 (or are empty)
//   1: no bit extends y1           -> every y2
//   2: only bit 0 extends y1       -> y2 start with 1 (or are empty)
//   3: both bits extend y1         -> only the empty y2
// So y2 starting with 0 pair with T1[cg[0], cg[2]) and y2 starting with 1 with
// T1[cg[1], cg[3]).  T1 is stored twice: sorted by (cls, x1, y1) for the scatter
// sweep (distinct targets across lanes) and by (cls, y1, x1) for the gather sweep
// (lanes sharing y1 read the same cache lines).
//
// T2 entry (16 bytes), one per (x2, y2 distinct subsequence of x2), grouped per
// x2 as [empty][y2 starting with 0, by rank][y2 starting with 1, by rank]:
//   w.x = y2 | k2 << 10 | jmax << 14
//   bytes 4..15: E2s[j] = emb(y2, x2[j:n2]), j = 0..n2; jmax = last j with E2s > 0
// ---------------------------------------------------------------------------
struct Tables {
  int n, n1, n2;
  uint32_t m1;          // number of T1 entries = 2*3^n1 - 2^n1
  uint32_t m2;          // number of T2 entries = 2*3^n2 - 2^n2
  uint32_t cg[5];       // class boundaries in T1
  const uint4* t1s;     // sorted (cls, x1, y1)
  const uint4* t1g;     // sorted (cls, y1, x1)
  const uint4* t2;      // grouped per x2
  const uint32_t* off2; // [2^n2 + 1] start of x2's group in t2
  const uint32_t* n0_2; // [2^n2] number of y2 starting with 0 for x2
};

// Per-instance constants, FP64: w[k] = d^(n-k)(1-d)^k, sw[k] = s_k w_k with
// s_k = (n-k)/d - k/(1-d) (zero when d is 0 or 1).
struct Consts {
  double w[kNMax + 1];
  double sw[kNMax + 1];
  double pad[2];
};

// Per-instance scalar state (device, FP64, nats).
struct State {
  double M;           // max log p of the current iterate
  double L, U, I;     // bounds and rate at the last evaluated iterate
  double certL, certU, certI, certM;  // last FP64 evaluation
  double bestL, bestU;                // best certified bounds
  double tol;         // freeze when U - L < tol (nats); < 0 disables
  double lse;         // scratch: log-sum-exp of the last normalisation
  int iters;          // completed updates
  int converged;      // 1: frozen (kernels skip the instance)
  int bad;            // non-finite value seen
  int stop_best;      // 1: the tolerance test uses the best bounds so far
};

// One group of nb instances with length n, arrays at fixed strides.
template <typename T>
struct Group {
  int n, nb;
  size_t xs, ys;      // strides: inputs (2^n) and outputs (2^(n+1)-1 rounded up)
  T* lp;              // log p
  T* p;               // p e^{-M}
  T* r;               // r(y) e^{-M}
  T* v;               // v(y) = w_k log(r(y) e^{-M})  (or s_k w_k log ... )
  T* v2;              // stream engine: v in split layout, stride v2s
  size_t v2s;
  T* g;               // G(x)
  T* gd;              // Gd(x) (gradient evaluations only)
  T* D;               // D(x)
  T* f0;              // factored engine ping-pong, stride fs
  T* f1;
  size_t fs;
  const double* h;    // H(x) (FP64 always)
  const double* hd;   // Hd(x)
  const T* hf;        // H(x) rounded to T (the same array as h when T is double)
  double* part;       // per-block partials, stride ps
  size_t ps;
  State* st;          // [nb]
  const Consts* cs;   // [nb]
  double eta;         // update step: log p <- log p + eta D - log sum p e^{eta D} (1 = BA)
  int frz;            // 0: no instance can be frozen by a gap tolerance (none is set); the
                      // sweep kernels of the default launch plan then skip reading the
                      // frozen flag, which the update kernels always test
  int s8lc;           // eight-position backward launches: log2 of the columns per block
                      // (0: as many as the rows hold, up to the value lanes of a node)
  int dsum;           // iterations with eta = 1: the D launch stores log p + D in D (the
                      // update then reads one array: log p <- (log p + D) - L, the same
                      // rounding as before); 0: D itself (certification, a step eta != 1)
  int half;           // complement-symmetric iterate, launch plan level 8 at n = 20 (FP32):
                      // the stages keep the rows that start with 0 (and the empty row),
                      // the D launches take the column tiles whose first bit is 0 and
                      // write log p (and log p + D) at x and at its complement
};

enum StreamOp { kOpScatter = 0, kOpGather = 1, kOpInit = 2, kOpRow = 3, kOpVerify = 4, kOpScatterOrbit = 5 };

// Orbits of Appendix A: the k-bit string v under complement and reversal (the group
// {id, cpl, rev, cpl rev}); rep = its smallest member (lexicographic order is
// numeric order), size = the number of distinct members (1, 2 or 4).
__device__ __forceinline__ void orbit_of(uint32_t v, int k, uint32_t& rep, uint32_t& size) {
  const uint32_t m = k ? (0xffffffffu >> (32 - k)) : 0u;
  const uint32_t a = v, b = v ^ m, c = k ? (__brev(v) >> (32 - k)) : 0u, d = c ^ m;
  rep = min(min(a, b), min(c, d));
  size = 1u + (b != a ? 1u : 0u) + ((c != a && c != b) ? 1u : 0u) + ((d != a && d != b && d != c) ? 1u : 0u);
}

// Extra arguments of the non-iteration stream ops.
struct StreamExtra {
  double* h;                  // init: H(x), stride xs
  double* hd;                 // init: Hd(x)
  unsigned long long* fix;    // init: fixed-point accumulators, 4 words per input, stride 4 xs
  uint32_t target_x;          // row
  uint32_t* row_dense;        // row: dense counts by rank
  uint32_t* bins;             // verify: [2^n][n+2] length sums and nonzero counts
  unsigned long long* stats;  // verify: [6]
};

// ---- order-independent sums of doubles ---------------------------------------
// A value v is split exactly into v = a 2^-40 + b 2^-80 + r with integers a, b
// (0 <= b < 2^40, 0 <= r < 2^-80) and the integer parts are added with 64-bit
// integer atomics, whose result does not depend on the order of the additions.
// Used for sums of at most a few thousand terms with |sum| < 2^22 (H and the
// scaled Hd of the init pass): no overflow, truncation below 2^-68 in total.
constexpr double kFixScale = 1099511627776.0;  // 2^40

__device__ __forceinline__ void fix_add(unsigned long long* w, double v) {
  const double s = v * kFixScale;
  const double a = floor(s);
  const double b = floor((s - a) * kFixScale);
  __hip_atomic_fetch_add(w, (unsigned long long)(long long)a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_fetch_add(w + 1, (unsigned long long)(long long)b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double fix_value(const unsigned long long* w) {
  return double((long long)w[0]) / kFixScale + double((long long)w[1]) / (kFixScale * kFixScale);
}

// Hd(x) = sum_y s_k w_k emb log emb is accumulated as Hd 2^-e with 2^e > max_k |s_k|,
// so that each scaled term is bounded like the terms of H.
__device__ __forceinline__ int hd_exponent(const Consts& c, int n) {
  double smax = 0.0;
  for (int k = 0; k <= n; ++k)
    if (c.w[k] > 0.0) smax = fmax(smax, fabs(c.sw[k] / c.w[k]));
  int e = 0;
  if (smax > 0.0) (void)frexp(smax, &e);
  return e > 0 ? e : 0;
}

// ---- launch wrappers (defined in the .hip files) ---------------------------

// ba_persist.hip: `iters` iterations of every instance of a small group in one launch
// (one block per instance, all arrays in LDS); n <= 13 (FP32) or 12 (FP64).
bool persist_supported(int n, size_t esz);
template <typename T>
hipError_t launch_persist(const Group<T>& g, int iters, double floor, int check_tol, int threads, hipStream_t s);

// ba_tables.hip
size_t table_bytes(int n);
hipError_t build_tables(int n, void* mem, hipStream_t s, Tables* out_host);

// ba_stream.hip
template <typename T>
hipError_t launch_stream(StreamOp op, const Tables& tb, const Group<T>& g, int k0,
                         const StreamExtra& ex, hipStream_t s);
// r(y) = r(rep(y)) for every output that is not its orbit's representative.
template <typename T>
hipError_t launch_orbit_expand(const Group<T>& g, hipStream_t s);
template <typename T>
hipError_t launch_combine_r(const Group<T>& g, int n1, int n2, int k0, hipStream_t s);
int stream_lds_limit();  // largest dynamic LDS a block may request on this device
hipError_t launch_row_compact(const uint32_t* dense, int n, uint32_t* rank_out,
                              uint32_t* emb_out, int cap, uint32_t* nnz_dev, hipStream_t s);

// ba_pull.hip: r in pull form over the supersequences of every output (Section 5),
// through a partial buffer of pull_partial_bytes (written, then summed per output
// in a fixed order).
size_t pull_partial_bytes(int n, int nb, size_t esz);
template <typename T>
hipError_t launch_pull(const Group<T>& g, T* partial, hipStream_t s);

// ba_factored.hip: the two products stage by stage.
// fuse = 1: two positions per launch (k_fwd_stage2 / k_bwd_stage2); fuse = 2: four
// positions per launch (k_fwd_stage4 / k_bwd_stage4) with the leftover positions
// two (or one) at a time: the last 1-4 in the forward, the first n mod 4 in the
// backward; fuse = 3: as 2 with eight positions per backward launch
// (k_bwd_stage8) while four remain for the last; fuse = 4: as 3 with the last four
// forward positions in one launch (k_fwd_last4, n >= 12); fuse = 5: as 4 with the
// first eight forward positions in one launch (k_fwd_first8); fuse = 6: as 5 with
// the backward sweep at n = 20 (FP32) in two launches (k_bwd_stage12, then
// k_bwd_stage8_p with D); fuse = 7: as 6 with the forward positions 8 .. 19 at
// n = 20 (FP32) in one launch (k_fwd_stage12); fuse = 8: as 7 with the D launch of
// an iteration inside a ba_step call fused with the next iteration's update and first
// eight forward positions (FusedNext).
// logv = 1: the last forward launch writes v = w_k log r instead of r.
// dpart = 1: the last backward launch also forms D = H - G - M and the block
// records of k_dpart, writing D instead of G; *dpart_blocks returns the number of
// records it wrote, or 0 if it could not fuse (smallest n), in which case the
// caller launches k_dpart itself.
//
// upd: the update of the previous iteration, fused into the forward sweep's first
// launch (which then reads log p and D instead of p, and writes log p but not p).
struct FusedUpdate {
  double floor;
  int check_tol;
  int nmax;  // > 0: shift by the max (see k_fwd_first8): the D launch left nmax block
             // maxima of log p + D and no final record; 0: the update from the final record
};
// Offset (doubles) of the block maxima of log p + D (floats) in an iterate group's
// record buffer: the second record set, which only ba_set_logp's passes use.
constexpr size_t kBlockMaxima = size_t(kMaxRedBlocks) * kPartStride;
// True when launch_forward's first launch is the four-position one at i = 0.
bool forward_update_fusable(int n, int fuse);
// True when launch_forward's first launch is the eight-position one (k_fwd_first8).
bool forward_first8(int n, int fuse);
// True when launch_backward's D launch (FP32) also writes the block maxima of log p + D.
bool backward_writes_maxima(int n, int fuse, int esz);
// The D launch of an iteration fused with the next iteration's update and first eight
// forward positions (fuse = 8: FP32 iterates, eta = 1, n >= 12, the iterate scaled by
// a max shift, i.e. not the first iteration of a ba_step call): it writes its block
// maxima of log p + D to set par of two sets in the record buffer's second set and
// shifts by the max of set 1 - par (the D launch before it); the next forward sweep
// then starts from its F_8 (launch_forward with first8_done).
struct FusedNext {
  double floor;
  int par;
  int nprev;  // block maxima the D launch before it wrote
};
// True when launch_backward can take a FusedNext (element bytes esz).
bool backward_fuses_next(int n, int fuse, int esz);
// True when a complement-symmetric FP32 iterate can run the full plan's kernels on half
// the rows and column tiles (Group::half: the twelve-position plan of n = 20).
bool half_plan_fits(int n, int fuse);
template <typename T>
hipError_t launch_forward(const Group<T>& g, hipStream_t s, int* launches, int fuse, int logv,
                          const FusedUpdate* upd = nullptr, int first8_done = 0);  // p -> r
template <typename T>
hipError_t launch_backward(const Group<T>& g, hipStream_t s, int* launches, int fuse, int dpart,
                           int* dpart_blocks, const FusedNext* next = nullptr);  // v -> G
int factored_launches(int n, int fuse);   // forward launches (two positions each when fuse != 0)
int backward_launches(int n, int fuse, int esz = 4);  // launches of launch_backward (esz: element bytes)
int forward_launches(int n, int fuse, int esz = 4);  // launches of launch_forward
// Complement-symmetric iteration (iterate invariant under complement): the two
// products on the canonical half, v and D fused as above; v is stored at compact
// indices (2^n entries) and D, G for x < 2^(n-1).  Supported for even n >= 4 with
// two positions per launch.
bool symmetric_supported(int n, int fuse);
template <typename T>
hipError_t launch_forward_sym(const Group<T>& g, hipStream_t s, int* launches, int fuse,
                              const FusedUpdate* upd = nullptr);
template <typename T>
hipError_t launch_backward_sym(const Group<T>& g, hipStream_t s, int* launches, int* dpart_blocks, int fuse);
// The first backward launch of the complement-symmetric iteration for n % 4 == 0,
// n >= 12: eight positions (n-8 .. n-1) from the compact v into dst.
template <typename T>
hipError_t launch_backward8_sym_v(const Group<T>& g, hipStream_t s, T* dst);

// ba_reduce.hip
template <typename T>
hipError_t launch_logr(const Group<T>& g, int use_sw, int want_v2, int n1, int n2, hipStream_t s);
template <typename T>
hipError_t launch_dpart(const Group<T>& g, int nblk, int use_hd, const T* gd, hipStream_t s);
// Combine the nblk block records of every instance into its final record.
template <typename T>
hipError_t launch_final_parts(const Group<T>& g, int nblk, hipStream_t s);
// sym: D holds x < 2^(n-1) only (complement-symmetric iteration); the update
// writes each value to x and cpl x.
template <typename T>
hipError_t launch_update(const Group<T>& g, int nblk, double floor, int check_tol, int sym, hipStream_t s);
// out[b] = max_x |log p(x) - log p(cpl x)| (device, one double per instance).
template <typename T>
hipError_t launch_sym_check(const Group<T>& g, double* out, int orbit, hipStream_t s);
template <typename T>
hipError_t launch_symmetrize(const Group<T>& g, int orbit, hipStream_t s);
int reduce_blocks(int n);

// Certification: FP64 evaluation of the current iterate of a group (any T).
// Step 1 (two partial passes) normalises, floors and renormalises log p into the
// FP64 group's lp/p; step 2 finishes after the FP64 sweeps and D.
template <typename T>
hipError_t launch_cert_prepare(const Group<T>& src, const Group<double>& dst, int nblk,
                               double floor, hipStream_t s);
hipError_t launch_cert_finish(const Group<double>& g, int nblk, State* out, int write_best,
                              hipStream_t s);
hipError_t launch_grad_finish(const Group<double>& g, int nblk, double* out4,
                              double* grad_theta, hipStream_t s);
hipError_t launch_mirror_update(int n, double* theta, const double* D, double eta,
                                hipStream_t s);
template <typename T>
hipError_t launch_get_logp(const Group<T>& g, double* dst, hipStream_t s);
template <typename T>
hipError_t launch_set_logp(const Group<T>& g, const double* src, int nblk, double floor,
                           hipStream_t s);
template <typename T>
hipError_t launch_reset(const Group<T>& g, hipStream_t s);
hipError_t launch_fill_zero(void* ptr, size_t bytes, hipStream_t s);
hipError_t launch_copy_f64(double* dst, const double* src, size_t count, hipStream_t s);
hipError_t launch_to_float(const double* src, float* dst, size_t count, hipStream_t s);

}  // namespace ba
