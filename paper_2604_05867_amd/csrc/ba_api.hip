// Host side of the C ABI declared in include/ba.h.
//
// A context holds host state only: instance parameters, the workspace layout
// and the bound stream.  All device memory comes from the caller's workspace.
// Every iteration step is a fixed sequence of kernel launches on the bound
// stream with no host synchronisation; host round trips happen only in the
// calls documented as blocking.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ba.h"
#include "ba_internal.h"

using namespace ba;

// Device memory owned by the library for ba_bind_static: one copy of this array
// per GPU, alive until the process ends.  In host code its name is only a
// stand-in; the device address is obtained with hipGetSymbolAddress per device.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

inline size_t al256(size_t b) { return (b + 255) & ~size_t(255); }
inline size_t pad64(size_t n) { return (n + 63) & ~size_t(63); }

// Offsets of one group's arrays inside the workspace.
struct GroupLayout {
  size_t tables;
  size_t lp, p, r, v, v2, g, gd, D, f0, f1;     // iteration arrays (precision T)
  size_t h, hd, hf, part, st, cs;
  size_t c_lp, c_p, c_r, c_v, c_v2, c_g, c_gd, c_D, c_f0, c_f1, c_part, c_st;  // FP64 cert
  size_t pull;                                  // pull-sweep partials (FP64-sized)
};

struct GroupHost {
  int n = 0;
  std::vector<int> inst;      // global instance ids, increasing
  GroupLayout L{};
  Tables tb{};
  Group<float> gf{};          // iteration group if FP32
  Group<double> gd{};         // iteration group if FP64
  Group<double> cert{};       // FP64 evaluation group
  size_t xs = 0, ys = 0, v2s = 0, fs = 0, ps = 0;
};

}  // namespace

struct ba_ctx {
  int count = 0;
  std::vector<int> n;
  std::vector<double> d;
  std::vector<int> kexact;  // >= 0: exact deletion channel BDC_{n,k} for that instance
  int prec = BA_PREC_FP64;
  int cert_every = 1;
  int engine = BA_ENGINE_FACTORED;
  std::vector<GroupHost> groups;
  std::vector<std::pair<int, int>> where;  // instance -> (group, slot)
  size_t need = 0;
  size_t misc = 0;       // misc area: stats[8] u64, nnz u32, out4 double, scratch State
  size_t symdev = 0;     // one double per instance: symmetry deviation
  size_t verify = 0;     // verify bins / dense row for group of instance 0
  size_t verify_bytes = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  bool bound = false;
  int static_dev = -1;   // device whose static scratch this context is bound to, else -1
  std::string err;
  // tuning
  int scatter_lds_kb = 64;
  int fuse = 8;  // factored engine: positions per launch (see BA_TUNE_FACTORED_FUSE)
  int stop_rule = BA_STOP_ITERATE;
  int sym = 0;   // complement-symmetric iteration requested
  double eta = 1.0;  // update step (1 = BA)
  double floor = 0.0;  // floor of the iterates' log p below their max (nats); 0 = precision default
  // graph replay of ba_run chunks
  bool use_graph = false;
  // set once a gap tolerance has been given (ba_run): instances may then be frozen
  bool armed = false;
  // frozen-flag test in the sweep kernels: -1 = decided by `armed` (ba_step), else
  // the value ba_run chose for the current chunk
  int frz_override = -1;
  // one graph per frozen-flag mode (index = frz)
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  // captured chunks: each group of instances (one n) on its own branch of the graph
  int concurrent = 1;
  // groups small enough for LDS iterate in one persistent launch per call/chunk
  // (0 never, 1 automatic, 2 whenever they fit), with this many threads per block
  int persistent = 1;
  int persist_threads = 1024;
  // eight-position backward launches: log2 of the columns per block (0: widest)
  int s8lc = 0;
  std::vector<hipStream_t> aux;      // one per group, default priority
  std::vector<hipEvent_t> join_ev;   // one per group
  hipEvent_t fork_ev = nullptr;
  int gchunk = -1;
  int gengine = -1;
  // timing hook
  bool timing = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_class;    // class of the bracket opened by the event, -1 for a close
  std::vector<int> ev_kernels;  // kernels launched inside the bracket
};

namespace {

int fail(ba_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                                    \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail((ctx), BA_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

uint64_t ipow3(int e) {
  uint64_t v = 1;
  while (e-- > 0) v *= 3;
  return v;
}

bool valid_d(double d) { return d >= 0.0 && d <= 1.0 && isfinite(d); }

// Exact deletion channel BDC_{n,k} (Section 2.2): W(y|x) = emb(y,x)/C(n,k) for
// |y| = k, so w_j = [j = k]/C(n,k); no deletion probability, no d-gradient.
void make_consts_exact(int n, int k, Consts* c) {
  memset(c, 0, sizeof(*c));
  double binom = 1.0;
  for (int i = 1; i <= k; ++i) binom = binom * double(n - k + i) / double(i);
  c->w[k] = 1.0 / binom;
}

void make_consts(int n, double d, Consts* c) {
  memset(c, 0, sizeof(*c));
  for (int k = 0; k <= n; ++k) {
    const double a = (n - k == 0) ? 1.0 : pow(d, double(n - k));
    const double b = (k == 0) ? 1.0 : pow(1.0 - d, double(k));
    c->w[k] = a * b;
    c->sw[k] = (d > 0.0 && d < 1.0) ? ((n - k) / d - k / (1.0 - d)) * c->w[k] : 0.0;
  }
}

size_t elem(const ba_ctx* c) { return c->prec == BA_PREC_FP32_LOG ? sizeof(float) : sizeof(double); }

// Floor of the iterates' log p below their maximum (ba_set_floor, else the default
// of the iteration precision).
double iterate_floor(const ba_ctx* c) {
  if (c->floor > 0.0) return c->floor;
  return c->prec == BA_PREC_FP32_LOG ? kFloor32 : kFloor64;
}

void plan(ba_ctx* c) {
  // group instances by n (order of first appearance)
  c->groups.clear();
  c->where.assign(c->count, {0, 0});
  for (int i = 0; i < c->count; ++i) {
    int gi = -1;
    for (size_t j = 0; j < c->groups.size(); ++j)
      if (c->groups[j].n == c->n[i]) gi = int(j);
    if (gi < 0) {
      GroupHost g;
      g.n = c->n[i];
      c->groups.push_back(g);
      gi = int(c->groups.size()) - 1;
    }
    c->where[i] = {gi, int(c->groups[gi].inst.size())};
    c->groups[gi].inst.push_back(i);
  }
  const size_t T = elem(c);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += al256(bytes); return r; };
  for (auto& g : c->groups) {
    const int n = g.n, n1 = (n + 1) / 2, n2 = n / 2;
    const size_t nb = g.inst.size();
    g.xs = pad64(size_t(1) << n);
    g.ys = pad64(out_count(n));
    g.v2s = pad64(size_t(out_count(n1)) * out_count(n2));
    g.fs = pad64(size_t(2) << n);
    g.ps = size_t(kPartDoubles);
    GroupLayout& L = g.L;
    L.tables = take(table_bytes(n));
    L.lp = take(nb * g.xs * T);
    L.p = take(nb * g.xs * T);
    L.r = take(nb * g.ys * T);
    L.v = take(nb * g.ys * T);
    L.v2 = take(nb * g.v2s * T);
    L.g = take(nb * g.xs * T);
    L.gd = take(nb * g.xs * T);
    L.D = take(nb * g.xs * T);
    L.f0 = take(nb * g.fs * T);
    L.f1 = take(nb * g.fs * T);
    L.h = take(nb * g.xs * 8);
    L.hd = take(nb * g.xs * 8);
    L.hf = take(nb * g.xs * T);
    L.part = take(nb * g.ps * 8);
    L.st = take(nb * sizeof(State));
    L.cs = take(nb * sizeof(Consts));
    L.c_lp = take(nb * g.xs * 8);
    L.c_p = take(nb * g.xs * 8);
    L.c_r = take(nb * g.ys * 8);
    L.c_v = take(nb * g.ys * 8);
    L.c_v2 = take(nb * g.v2s * 8);
    L.c_g = take(nb * g.xs * 8);
    L.c_gd = take(nb * g.xs * 8);
    L.c_D = take(nb * g.xs * 8);
    L.c_f0 = take(nb * g.fs * 8);
    L.c_f1 = take(nb * g.fs * 8);
    L.c_part = take(nb * g.ps * 8);
    L.c_st = take(nb * sizeof(State));
    L.pull = take(pull_partial_bytes(n, int(nb), 8));
  }
  // verify bins for instance 0's n (also the dense row buffer)
  const int n0 = c->n[0];
  c->verify_bytes = (size_t(1) << n0) * size_t(n0 + 2) * 4;
  if (c->verify_bytes < size_t(out_count(n0)) * 4) c->verify_bytes = size_t(out_count(n0)) * 4;
  c->verify = take(c->verify_bytes);
  c->misc = take(4096);
  c->symdev = take(size_t(c->count) * 8);
  c->need = o;
}

template <typename T>
Group<T> make_group(char* ws, const GroupHost& g, bool cert) {
  const GroupLayout& L = g.L;
  Group<T> G{};
  G.n = g.n;
  G.nb = int(g.inst.size());
  G.xs = g.xs;
  G.ys = g.ys;
  G.v2s = g.v2s;
  G.fs = g.fs;
  G.ps = g.ps;
  G.lp = reinterpret_cast<T*>(ws + (cert ? L.c_lp : L.lp));
  G.p = reinterpret_cast<T*>(ws + (cert ? L.c_p : L.p));
  G.r = reinterpret_cast<T*>(ws + (cert ? L.c_r : L.r));
  G.v = reinterpret_cast<T*>(ws + (cert ? L.c_v : L.v));
  G.v2 = reinterpret_cast<T*>(ws + (cert ? L.c_v2 : L.v2));
  G.g = reinterpret_cast<T*>(ws + (cert ? L.c_g : L.g));
  G.gd = reinterpret_cast<T*>(ws + (cert ? L.c_gd : L.gd));
  G.D = reinterpret_cast<T*>(ws + (cert ? L.c_D : L.D));
  G.f0 = reinterpret_cast<T*>(ws + (cert ? L.c_f0 : L.f0));
  G.f1 = reinterpret_cast<T*>(ws + (cert ? L.c_f1 : L.f1));
  G.h = reinterpret_cast<const double*>(ws + L.h);
  G.hd = reinterpret_cast<const double*>(ws + L.hd);
  // H in the iteration precision (a rounded copy for FP32, H itself for FP64)
  G.hf = (sizeof(T) == sizeof(double) || cert) ? reinterpret_cast<const T*>(ws + L.h)
                                               : reinterpret_cast<const T*>(ws + L.hf);
  G.part = reinterpret_cast<double*>(ws + (cert ? L.c_part : L.part));
  G.st = reinterpret_cast<State*>(ws + (cert ? L.c_st : L.st));
  G.cs = reinterpret_cast<const Consts*>(ws + L.cs);
  G.eta = 1.0;
  G.frz = 1;
  G.s8lc = 0;
  return G;
}

// Restrict a group view to one instance slot.
template <typename T>
Group<T> slot_view(Group<T> G, int j) {
  G.nb = 1;
  G.lp += size_t(j) * G.xs;
  G.p += size_t(j) * G.xs;
  G.r += size_t(j) * G.ys;
  G.v += size_t(j) * G.ys;
  G.v2 += size_t(j) * G.v2s;
  G.g += size_t(j) * G.xs;
  G.gd += size_t(j) * G.xs;
  G.D += size_t(j) * G.xs;
  G.f0 += size_t(j) * G.fs;
  G.f1 += size_t(j) * G.fs;
  G.h += size_t(j) * G.xs;
  G.hd += size_t(j) * G.xs;
  G.hf += size_t(j) * G.xs;
  G.part += size_t(j) * G.ps;
  G.st += j;
  G.cs += j;
  return G;
}

// Longest output length accumulated in LDS by the scatter, for an LDS budget.
int k0_for(int n, int nbt, size_t esz, size_t budget) {
  int k0 = 0;
  while (k0 + 1 <= n && size_t((2u << (k0 + 1)) - 1u) * nbt * esz <= budget) ++k0;
  return k0;
}

// ---- timing hook: events around kernel classes ------------------------------
struct Timer {
  ba_ctx* c;
  Timer(ba_ctx* c_, int cls, int kernels) : c(c_) { mark(cls, kernels); }
  ~Timer() { mark(-1, 0); }
  void mark(int cls, int kernels) {
    if (!c->timing) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, c->stream);
    c->ev.push_back(e);
    c->ev_class.push_back(cls);
    c->ev_kernels.push_back(kernels);
  }
};

// One sweep pair + reductions on group G (iteration or certification group).
// The complement-symmetric kernels run for this group's iterations: up to four
// positions per launch, the forward sweep with the last four positions in one
// launch from fuse level 4 on, the backward sweep with its first eight positions
// in one launch from level 3 on (n % 4 == 0, n >= 12).
int sym_fuse_fwd(const ba_ctx* c) { return c->fuse < 4 ? c->fuse : 4; }
int sym_fuse_bwd(const ba_ctx* c) { return c->fuse < 3 ? c->fuse : 3; }
int sym_backward_launches(int n, int fuse) {
  if (fuse >= 3 && n % 4 == 0 && n >= 12) return backward_launches(n, 2) - 1;
  return backward_launches(n, fuse < 2 ? fuse : 2);
}

bool sym_active(const ba_ctx* c, int n) {
  return c->sym && c->engine == BA_ENGINE_FACTORED && symmetric_supported(n, c->fuse);
}

// A complement-symmetric iterate at n = 20 with FP32 iterates, eta = 1 and launch plan
// level 8 runs the full plan's kernels on half the rows and column tiles
// (Group::half) instead of the complement-symmetric kernels.
bool half_plan(const ba_ctx* c, int n) {
  return sym_active(c, n) && c->prec == BA_PREC_FP32_LOG && c->eta == 1.0 && half_plan_fits(n, c->fuse);
}

// tail = 1 (factored engine, iteration only): the last forward launch writes v
// and the last backward launch forms D and its block records; *tail_done is the
// number of those records, 0 if the backward part was not fused (then the caller
// launches k_dpart).
template <typename T>
int sweeps(ba_ctx* c, const GroupHost& gh, const Group<T>& G, int use_sw_g, T* g_out, int tail = 0,
           int* tail_done = nullptr, const FusedUpdate* upd = nullptr, bool first8_done = false,
           const FusedNext* next = nullptr) {
  if (tail_done) *tail_done = 0;
  hipStream_t s = c->stream;
  const int n = gh.n, n1 = (n + 1) / 2, n2 = n / 2;
  const StreamExtra ex{};
  if (c->engine == BA_ENGINE_PULL) {
    {
      Timer t(c, BA_K_SWEEP1, 2 * ((G.nb + kTile - 1) / kTile));
      HIPCHK(c, launch_pull<T>(G, reinterpret_cast<T*>(c->ws + gh.L.pull), s));
    }
    {
      Timer t(c, BA_K_LOGR, 1);
      HIPCHK(c, launch_logr<T>(G, use_sw_g, 1, n1, n2, s));
    }
    {
      Timer t(c, BA_K_SWEEP2, 1);
      Group<T> G2 = G;
      G2.g = g_out;
      HIPCHK(c, launch_fill_zero(g_out, size_t(G.nb) * G.xs * sizeof(T), s));
      HIPCHK(c, launch_stream<T>(kOpGather, gh.tb, G2, 0, ex, s));
    }
  } else if (c->engine == BA_ENGINE_STREAM) {
    const int nbt = G.nb < kTile ? G.nb : kTile;
    const size_t budget = std::min<size_t>(size_t(c->scatter_lds_kb) * 1024, size_t(stream_lds_limit()));
    const int k0 = k0_for(n, nbt, sizeof(T), budget);
    // iterations under ba_set_symmetry(2): Algorithm 7 over complement/reversal orbits
    const bool orbit = tail && c->sym == 2;
    {
      Timer t(c, BA_K_SWEEP1, 1);
      HIPCHK(c, launch_fill_zero(G.r, size_t(G.nb) * G.ys * sizeof(T), s));
      HIPCHK(c, launch_fill_zero(G.v2, size_t(G.nb) * G.v2s * sizeof(T), s));
      HIPCHK(c, launch_stream<T>(orbit ? kOpScatterOrbit : kOpScatter, gh.tb, G, k0, ex, s));
      HIPCHK(c, launch_combine_r<T>(G, n1, n2, k0, s));
      if (orbit) HIPCHK(c, launch_orbit_expand<T>(G, s));
    }
    {
      Timer t(c, BA_K_LOGR, 1);
      HIPCHK(c, launch_logr<T>(G, use_sw_g, 1, n1, n2, s));
    }
    {
      Timer t(c, BA_K_SWEEP2, 1);
      Group<T> G2 = G;
      G2.g = g_out;
      HIPCHK(c, launch_fill_zero(g_out, size_t(G.nb) * G.xs * sizeof(T), s));
      HIPCHK(c, launch_stream<T>(kOpGather, gh.tb, G2, k0, ex, s));
    }
  } else if (tail && !use_sw_g && sym_active(c, n) && !G.half) {
    {
      Timer t(c, BA_K_SWEEP1, forward_launches(n, sym_fuse_fwd(c)));
      HIPCHK(c, launch_forward_sym<T>(G, s, nullptr, sym_fuse_fwd(c), upd));
    }
    {
      Timer t(c, BA_K_SWEEP2, sym_backward_launches(n, sym_fuse_bwd(c)));
      Group<T> G2 = G;
      G2.g = g_out;
      HIPCHK(c, launch_backward_sym<T>(G2, s, nullptr, tail_done, sym_fuse_bwd(c)));
    }
  } else {
    const int fuse_tail = (tail && !use_sw_g) ? 1 : 0;
    {
      Timer t(c, BA_K_SWEEP1, forward_launches(n, c->fuse, int(sizeof(T))) - (first8_done ? 1 : 0));
      HIPCHK(c, launch_forward<T>(G, s, nullptr, c->fuse, fuse_tail, upd, first8_done ? 1 : 0));
    }
    if (!fuse_tail) {
      Timer t(c, BA_K_LOGR, 1);
      HIPCHK(c, launch_logr<T>(G, use_sw_g, 0, n1, n2, s));
    }
    {
      Timer t(c, BA_K_SWEEP2, backward_launches(n, c->fuse, int(sizeof(T))));
      Group<T> G2 = G;
      G2.g = g_out;
      G2.s8lc = c->s8lc;
      HIPCHK(c, launch_backward<T>(G2, s, nullptr, c->fuse, fuse_tail, tail_done, next));
    }
  }
  return BA_OK;
}

// The update of an iteration can be left pending and fused into the next
// iteration's first forward launch (factored engine, full or complement-symmetric
// kernels with four positions per launch).
bool update_fusable(const ba_ctx* c, const GroupHost& gh) {
  if (c->engine != BA_ENGINE_FACTORED) return false;
  if (sym_active(c, gh.n) && !half_plan(c, gh.n)) return forward_update_fusable(gh.n, sym_fuse_fwd(c));
  return forward_update_fusable(gh.n, c->fuse);
}

// FP32 BA iterations at n >= 12 (launch plan levels 6-8): an update left pending to
// the next eight-position first launch can shift by the max of log p + D instead of
// normalising (k_fwd_first8), from the block maxima the D launch wrote, with no
// final-record launch.
bool update_by_max(const ba_ctx* c, const GroupHost& gh) {
  return c->engine == BA_ENGINE_FACTORED && c->prec == BA_PREC_FP32_LOG && c->eta == 1.0 &&
         (!sym_active(c, gh.n) || half_plan(c, gh.n)) && forward_first8(gh.n, c->fuse) &&
         backward_writes_maxima(gh.n, c->fuse, 4);
}

// One iteration.  fused_in: the previous iteration's update is pending and done by
// this iteration's first forward launch (by the max from nmax_in block maxima when
// nmax_in > 0); leave_pending: this iteration's update is left to the next
// iteration's first forward launch, and *nmax_out > 0 when that one shifts by the max.
// first8_done: the previous iteration's D launch made this iteration's update and
// first eight forward positions; next: this iteration's D launch makes the next one's
// (then no record, reduction or update launch follows here).
template <typename T>
int iterate_group(ba_ctx* c, const GroupHost& gh, const Group<T>& G0, bool fused_in, int nmax_in,
                  bool leave_pending, int* nmax_out, bool first8_done = false, const FusedNext* next = nullptr) {
  Group<T> G = G0;
  G.eta = c->eta;
  G.dsum = c->eta == 1.0 ? 1 : 0;  // the D array carries log p + D to the update
  G.half = half_plan(c, gh.n) ? 1 : 0;
  // The kernels that write log p, p and the state always test the frozen flag, so
  // a frozen instance's iterate and state stay untouched whether or not the sweeps
  // test it too; skipping the test there (frz = 0) only sweeps a frozen instance
  // again into its own scratch arrays.  ba_run chooses per chunk (0 while no
  // instance is frozen); otherwise the test is made once a tolerance has been set,
  // before which only a non-finite value can freeze an instance.
  G.frz = c->frz_override >= 0 ? c->frz_override : (c->armed ? 1 : 0);
  const double floor = iterate_floor(c);
  const int check_tol = c->prec == BA_PREC_FP64 ? 1 : 0;
  const FusedUpdate fu{floor, check_tol, nmax_in};
  int nblk = 0;  // block records written by the fused D launch, if any
  int rc = sweeps<T>(c, gh, G, 0, G.g, 1, &nblk, fused_in ? &fu : nullptr, first8_done, next);
  if (rc) return rc;
  if (next) {
    if (nmax_out) *nmax_out = nblk;  // the block maxima it wrote
    return BA_OK;
  }
  const bool by_max = leave_pending && nblk > 0 && update_by_max(c, gh);
  if (nmax_out) *nmax_out = by_max ? nblk : 0;
  if (!by_max) {
    Timer t(c, BA_K_REDUCE, nblk ? 1 : 2);
    if (!nblk) {
      nblk = reduce_blocks(gh.n);
      HIPCHK(c, launch_dpart<T>(G, nblk, 0, nullptr, c->stream));
    }
    HIPCHK(c, launch_final_parts<T>(G, nblk, c->stream));
  }
  if (!leave_pending) {
    Timer t(c, BA_K_UPDATE, 1);
    HIPCHK(c, launch_update<T>(G, reduce_blocks(gh.n), floor, check_tol, sym_active(c, gh.n) && !G.half ? 1 : 0,
                               c->stream));
  }
  return BA_OK;
}

// FP64 evaluation of `src` (any precision) through the certification group; the
// results land in cert.D / cert.r / cert.st and, via finish, in `out` states.
template <typename T>
int certify_group(ba_ctx* c, const GroupHost& gh, const Group<T>& src, const Group<double>& cert,
                  State* out, int write_best) {
  const int nblk = reduce_blocks(gh.n);
  HIPCHK(c, launch_cert_prepare<T>(src, cert, nblk, kFloor64, c->stream));
  int rc = sweeps<double>(c, gh, cert, 0, cert.g);
  if (rc) return rc;
  HIPCHK(c, launch_dpart<double>(cert, nblk, 0, nullptr, c->stream));
  HIPCHK(c, launch_cert_finish(cert, nblk, out, write_best, c->stream));
  return BA_OK;
}

int certify_all(ba_ctx* c, int write_best) {
  for (auto& gh : c->groups) {
    int rc;
    if (c->prec == BA_PREC_FP32_LOG) rc = certify_group<float>(c, gh, gh.gf, gh.cert, gh.gf.st, write_best);
    else rc = certify_group<double>(c, gh, gh.gd, gh.cert, gh.gd.st, write_best);
    if (rc) return rc;
  }
  return BA_OK;
}

int read_states(ba_ctx* c, std::vector<State>& out) {
  out.resize(c->count);
  for (auto& gh : c->groups) {
    std::vector<State> tmp(gh.inst.size());
    const State* src = (c->prec == BA_PREC_FP32_LOG) ? gh.gf.st : gh.gd.st;
    HIPCHK(c, hipMemcpyAsync(tmp.data(), src, tmp.size() * sizeof(State), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t j = 0; j < gh.inst.size(); ++j) out[gh.inst[j]] = tmp[j];
  }
  return BA_OK;
}

int write_states(ba_ctx* c, const std::vector<State>& in) {
  for (auto& gh : c->groups) {
    std::vector<State> tmp(gh.inst.size());
    for (size_t j = 0; j < gh.inst.size(); ++j) tmp[j] = in[gh.inst[j]];
    State* dst = (c->prec == BA_PREC_FP32_LOG) ? gh.gf.st : gh.gd.st;
    HIPCHK(c, hipMemcpyAsync(dst, tmp.data(), tmp.size() * sizeof(State), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return BA_OK;
}

void drop_graph(ba_ctx* c) {
  for (auto& g : c->gexec) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  c->gchunk = -1;
  c->gengine = -1;
}

// Per-device address of `scratch` (set once per device by hipGetSymbolAddress with
// that device current) and the context currently bound to it.
constexpr int kMaxDevices = 64;
struct StaticScratch {
  std::mutex mu;
  void* ptr[kMaxDevices] = {};
  const ba_ctx* owner[kMaxDevices] = {};
};
StaticScratch& static_scratch() {
  static StaticScratch s;
  return s;
}

// Give up this context's claim on a device's static scratch (if it holds one).
void release_static(ba_ctx* c) {
  if (c->static_dev < 0) return;
  StaticScratch& S = static_scratch();
  std::lock_guard<std::mutex> lock(S.mu);
  if (S.owner[c->static_dev] == c) S.owner[c->static_dev] = nullptr;
  c->static_dev = -1;
}

int check_ctx(ba_ctx* c) {
  if (!c) return BA_EINVAL;
  if (!c->bound) return fail(c, BA_ESTATE, "context is not bound to a workspace (call ba_bind)");
  if (c->static_dev >= 0) {
    StaticScratch& S = static_scratch();
    std::lock_guard<std::mutex> lock(S.mu);
    if (S.owner[c->static_dev] != c) {
      c->bound = false;
      return fail(c, BA_ESTATE, "the library's static workspace on device " + std::to_string(c->static_dev) +
                                    " was bound to another context since (bind this one again)");
    }
  }
  return BA_OK;
}

int new_ctx(int count, const int* n, const double* d, int prec, int cert_every, ba_ctx** out) {
  if (!out || count < 1 || count > 4096 || !n || !d || cert_every < 1 ||
      (prec != BA_PREC_FP64 && prec != BA_PREC_FP32_LOG))
    return BA_EINVAL;
  for (int i = 0; i < count; ++i)
    if (n[i] < 1 || n[i] > kNMax || !valid_d(d[i])) return BA_EINVAL;
  ba_ctx* c = new (std::nothrow) ba_ctx();
  if (!c) return BA_ENOMEM;
  c->count = count;
  c->n.assign(n, n + count);
  c->d.assign(d, d + count);
  c->kexact.assign(count, -1);
  c->prec = prec;
  c->cert_every = cert_every;
  plan(c);
  *out = c;
  return BA_OK;
}

}  // namespace

extern "C" {

int ba_init(int n, double d, ba_ctx** out) { return new_ctx(1, &n, &d, BA_PREC_FP64, 1, out); }

int ba_init_batch(int count, const int* n, const double* d, int prec, int cert_every, ba_ctx** out) {
  return new_ctx(count, n, d, prec, cert_every, out);
}

int ba_init_exact(int count, const int* n, const int* k, int prec, int cert_every, ba_ctx** out) {
  if (!k || !n || count < 1 || count > 4096) return BA_EINVAL;
  for (int i = 0; i < count; ++i)
    if (k[i] < 0 || k[i] > n[i]) return BA_EINVAL;
  std::vector<double> d(count, 0.5);
  int rc = new_ctx(count, n, d.data(), prec, cert_every, out);
  if (rc) return rc;
  (*out)->kexact.assign(k, k + count);
  return BA_OK;
}

int ba_set_engine(ba_ctx* c, int engine) {
  if (!c || (engine != BA_ENGINE_STREAM && engine != BA_ENGINE_FACTORED && engine != BA_ENGINE_PULL))
    return BA_EINVAL;
  if (engine != c->engine) drop_graph(c);
  c->engine = engine;
  return BA_OK;
}

int ba_set_tuning(ba_ctx* c, int key, int value) {
  if (!c) return BA_EINVAL;
  if (key == BA_TUNE_SCATTER_LDS_KB) {
    if (value < 1 || value > 160) return fail(c, BA_EINVAL, "scatter LDS budget must be 1..160 KB");
    c->scatter_lds_kb = value;
    drop_graph(c);
    return BA_OK;
  }
  if (key == BA_TUNE_STAGE8_COLUMNS) {
    if (value < 0 || value > 4) return fail(c, BA_EINVAL, "stage-8 columns must be 0 .. 4 (log2)");
    c->s8lc = value;
    drop_graph(c);
    return BA_OK;
  }
  if (key == BA_TUNE_PERSIST_THREADS) {
    if (value != 256 && value != 512 && value != 1024)
      return fail(c, BA_EINVAL, "persistent threads must be 256, 512 or 1024");
    c->persist_threads = value;
    drop_graph(c);
    return BA_OK;
  }
  if (key == BA_TUNE_PERSISTENT) {
    if (value < 0 || value > 2) return fail(c, BA_EINVAL, "persistent must be 0, 1 or 2");
    c->persistent = value;
    drop_graph(c);
    return BA_OK;
  }
  if (key == BA_TUNE_CONCURRENT_GROUPS) {
    if (value != 0 && value != 1) return fail(c, BA_EINVAL, "concurrent groups must be 0 or 1");
    c->concurrent = value;
    drop_graph(c);
    return BA_OK;
  }
  if (key == BA_TUNE_FACTORED_FUSE) {
    if (value < 0 || value > 8) return fail(c, BA_EINVAL, "fuse must be 0 .. 8");
    c->fuse = value;
    drop_graph(c);
    return BA_OK;
  }
  return fail(c, BA_EINVAL, "unknown tuning key");
}

int ba_set_stop_rule(ba_ctx* c, int rule) {
  if (!c || (rule != BA_STOP_ITERATE && rule != BA_STOP_BEST)) return BA_EINVAL;
  c->stop_rule = rule;
  return BA_OK;
}

int ba_set_graphs(ba_ctx* c, int enable) {
  if (!c) return BA_EINVAL;
  c->use_graph = enable != 0;
  if (!c->use_graph) drop_graph(c);
  return BA_OK;
}

void ba_free(ba_ctx* c) {
  if (!c) return;
  release_static(c);
  drop_graph(c);
  for (auto e : c->join_ev) (void)hipEventDestroy(e);
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  for (auto st : c->aux) (void)hipStreamDestroy(st);
  for (auto e : c->ev) (void)hipEventDestroy(e);
  delete c;
}

int ba_workspace_bytes(const ba_ctx* c, size_t* bytes) {
  if (!c || !bytes) return BA_EINVAL;
  *bytes = c->need;
  return BA_OK;
}

namespace {

// Lay the context out in `ws` and build its count tables, constants, H and start
// states on `stream` (every array the iterations read is written here first).
int bind_workspace(ba_ctx* c, void* ws, size_t bytes, void* stream) {
  drop_graph(c);
  c->ws = static_cast<char*>(ws);
  c->ws_bytes = bytes;
  c->stream = static_cast<hipStream_t>(stream);
  c->bound = false;
  hipStream_t s = c->stream;
  for (auto& gh : c->groups) {
    gh.gf = make_group<float>(c->ws, gh, false);
    gh.gd = make_group<double>(c->ws, gh, false);
    gh.cert = make_group<double>(c->ws, gh, true);
    HIPCHK(c, build_tables(gh.n, c->ws + gh.L.tables, s, &gh.tb));
    // per-instance constants
    std::vector<Consts> cs(gh.inst.size());
    for (size_t j = 0; j < gh.inst.size(); ++j) {
      const int i = gh.inst[j];
      if (c->kexact[i] >= 0) make_consts_exact(gh.n, c->kexact[i], &cs[j]);
      else make_consts(gh.n, c->d[i], &cs[j]);
    }
    HIPCHK(c, hipMemcpyAsync(c->ws + gh.L.cs, cs.data(), cs.size() * sizeof(Consts), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
    // H and Hd: one pass of the count generator over all nonzeros (init op)
    const size_t nb = gh.inst.size();
    HIPCHK(c, launch_fill_zero(c->ws + gh.L.h, nb * gh.xs * 8, s));
    HIPCHK(c, launch_fill_zero(c->ws + gh.L.hd, nb * gh.xs * 8, s));
    StreamExtra ex{};
    ex.h = reinterpret_cast<double*>(c->ws + gh.L.h);
    ex.hd = reinterpret_cast<double*>(c->ws + gh.L.hd);
    // the init pass's fixed-point words (4 per input and instance) live in the FP64
    // certification arrays c_lp .. c_v (at least 2 xs + 2 ys doubles per instance),
    // which hold nothing yet
    ex.fix = reinterpret_cast<unsigned long long*>(c->ws + gh.L.c_lp);
    HIPCHK(c, launch_stream<double>(kOpInit, gh.tb, gh.cert, 0, ex, s));
    if (c->prec == BA_PREC_FP32_LOG)
      HIPCHK(c, launch_to_float(reinterpret_cast<const double*>(c->ws + gh.L.h),
                                reinterpret_cast<float*>(c->ws + gh.L.hf), nb * gh.xs, s));
    // states
    HIPCHK(c, launch_fill_zero(c->ws + gh.L.c_st, nb * sizeof(State), s));
    if (c->prec == BA_PREC_FP32_LOG) HIPCHK(c, launch_reset<float>(gh.gf, s));
    else HIPCHK(c, launch_reset<double>(gh.gd, s));
  }
  HIPCHK(c, hipStreamSynchronize(s));
  c->bound = true;
  return BA_OK;
}

}  // namespace

int ba_bind(ba_ctx* c, void* ws, size_t bytes, void* stream) {
  if (!c || !ws || (reinterpret_cast<uintptr_t>(ws) & 255u)) return fail(c, BA_EINVAL, "workspace pointer NULL or not 256-byte aligned");
  if (bytes < c->need) return fail(c, BA_ENOMEM, "workspace smaller than ba_workspace_bytes");
  release_static(c);
  return bind_workspace(c, ws, bytes, stream);
}

int ba_bind_static(ba_ctx* c, void* stream) {
  if (!c) return BA_EINVAL;
  if (c->need > kStaticScratchBytes)
    return fail(c, BA_ENOMEM, "context needs " + std::to_string(c->need) + " bytes of workspace; the static workspace "
                              "holds " + std::to_string(kStaticScratchBytes) + " (use ba_bind)");
  int dev = -1;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(c, BA_EDEVICE, "device index out of range for the static workspace");
  void* ptr = nullptr;
  {
    StaticScratch& S = static_scratch();
    std::lock_guard<std::mutex> lock(S.mu);
    if (!S.ptr[dev]) {
      void* p = nullptr;
      HIPCHK(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
      if (!p || (reinterpret_cast<uintptr_t>(p) & 255u))
        return fail(c, BA_EDEVICE, "static workspace address missing or not 256-byte aligned");
      S.ptr[dev] = p;
    }
    ptr = S.ptr[dev];
    if (c->static_dev >= 0 && S.owner[c->static_dev] == c) S.owner[c->static_dev] = nullptr;
    S.owner[dev] = c;  // a context bound here before loses it (its next call: BA_ESTATE)
    c->static_dev = dev;
  }
  const int rc = bind_workspace(c, ptr, kStaticScratchBytes, stream);
  if (rc) release_static(c);
  return rc;
}

namespace {

// Whether a group's iterations run as one persistent launch (ba_persist.hip): the
// factored engine's products, without the complement-symmetric kernels, for groups
// whose arrays fit in LDS.  Automatic choice (measured on MI355X, per iteration): a
// block per instance beats the launch chain up to n = 11 on its own (n = 8: 11
// against 22 us); from n = 12 one CU per instance is slower than the chain over the
// whole GPU, unless other groups' launches fill the GPU meanwhile (several groups).
bool use_persist(const ba_ctx* c, const GroupHost& gh) {
  if (!c->persistent || c->engine != BA_ENGINE_FACTORED || sym_active(c, gh.n) ||
      !persist_supported(gh.n, elem(c)))
    return false;
  return c->persistent == 2 || gh.n <= 11 || c->groups.size() > 1;
}

// `iters` iterations of one group: one persistent launch, or the launch chain with
// each update but the last fused into the next iteration's first launch where
// possible.
int step_group(ba_ctx* c, GroupHost& gh, int iters) {
  if (iters > 0 && use_persist(c, gh)) {
    Timer t(c, BA_K_SWEEP1, 1);
    const double floor = iterate_floor(c);
    if (c->prec == BA_PREC_FP32_LOG) {
      Group<float> G = gh.gf;
      G.eta = c->eta;
      HIPCHK(c, launch_persist<float>(G, iters, floor, 0, c->persist_threads, c->stream));
    } else {
      Group<double> G = gh.gd;
      G.eta = c->eta;
      HIPCHK(c, launch_persist<double>(G, iters, floor, 1, c->persist_threads, c->stream));
    }
    return BA_OK;
  }
  const bool fu = update_fusable(c, gh);
  // launch plan level 8: from the second iteration of the call on (the iterate then
  // carries a max shift), every D launch but the last also makes the next iteration's
  // update and first eight forward positions
  const bool fnext = fu && update_by_max(c, gh) && backward_fuses_next(gh.n, c->fuse, 4);
  int nmax = 0;
  bool done8 = false;
  for (int it = 0; it < iters; ++it) {
    const bool in = fu && it > 0 && !done8, out = fu && it + 1 < iters;
    const int nin = in ? nmax : 0;
    const bool nx = fnext && it >= 1 && it + 1 < iters;
    const FusedNext fn{iterate_floor(c), it & 1, nmax};
    const int rc = (c->prec == BA_PREC_FP32_LOG)
                       ? iterate_group<float>(c, gh, gh.gf, in, nin, out, &nmax, done8, nx ? &fn : nullptr)
                       : iterate_group<double>(c, gh, gh.gd, in, nin, out, &nmax);
    if (rc) return rc;
    done8 = nx;
  }
  return BA_OK;
}

// Streams and events that give each group its own branch of a captured chunk
// (created once, outside any capture).
int ensure_branches(ba_ctx* c) {
  const size_t ng = c->groups.size();
  if (!c->fork_ev) HIPCHK(c, hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
  while (c->aux.size() < ng) {
    hipStream_t st = nullptr;
    HIPCHK(c, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    c->aux.push_back(st);
  }
  while (c->join_ev.size() < ng) {
    hipEvent_t e = nullptr;
    HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->join_ev.push_back(e);
  }
  return BA_OK;
}

// One chunk of ba_run inside a capture on c->stream: k iterations and, for FP32
// iterates, the FP64 certification.  With several groups and concurrency on, every
// group's work goes on its own stream forked from and joined back into c->stream,
// so the graph holds one independent branch per group and the short launches of
// the small groups overlap the long ones of the large groups.
int capture_chunk(ba_ctx* c, int k) {
  if (!(c->concurrent && c->groups.size() > 1)) {
    int rc = ba_step(c, k);
    if (!rc && c->prec == BA_PREC_FP32_LOG) rc = certify_all(c, 1);
    return rc;
  }
  hipStream_t main = c->stream;
  HIPCHK(c, hipEventRecord(c->fork_ev, main));
  int rc = BA_OK;
  for (size_t gi = 0; gi < c->groups.size() && !rc; ++gi) {
    GroupHost& gh = c->groups[gi];
    hipStream_t br = c->aux[gi];
    HIPCHK(c, hipStreamWaitEvent(br, c->fork_ev, 0));
    c->stream = br;
    rc = step_group(c, gh, k);
    if (!rc && c->prec == BA_PREC_FP32_LOG)
      rc = certify_group<float>(c, gh, gh.gf, gh.cert, gh.gf.st, 1);
    c->stream = main;
    if (rc) break;
    HIPCHK(c, hipEventRecord(c->join_ev[gi], br));
    HIPCHK(c, hipStreamWaitEvent(main, c->join_ev[gi], 0));
  }
  c->stream = main;
  return rc;
}

}  // namespace

int ba_step(ba_ctx* c, int iters) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (iters < 0) return fail(c, BA_EINVAL, "iters < 0");
  // group after group (they share no arrays); within one call, the update of every
  // iteration but the last is fused into the next iteration's first launch where
  // possible; the call ends with log p and p of the last iterate in place
  for (auto& gh : c->groups)
    if ((rc = step_group(c, gh, iters))) return rc;
  return BA_OK;
}

int ba_run(ba_ctx* c, double gap_bits, int max_iters, int* iters_done) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!(gap_bits > 0.0) || max_iters < 0) return fail(c, BA_EINVAL, "gap_bits must be > 0 and max_iters >= 0");
  std::vector<State> st;
  if ((rc = read_states(c, st))) return rc;
  std::vector<int> start(c->count);
  c->armed = true;
  for (int i = 0; i < c->count; ++i) {
    start[i] = st[i].iters;
    st[i].tol = gap_bits * kLn2;
    st[i].stop_best = (c->stop_rule == BA_STOP_BEST) ? 1 : 0;
    // an instance stays frozen only if it already meets this tolerance (so ba_run
    // can be called repeatedly to continue a run)
    const double last = (c->prec == BA_PREC_FP64) ? st[i].U - st[i].L : st[i].certU - st[i].certL;
    const double gap = st[i].stop_best ? st[i].bestU - st[i].bestL : last;
    if (!st[i].bad && !(st[i].converged && gap < st[i].tol)) st[i].converged = 0;
  }
  if ((rc = write_states(c, st))) return rc;
  // FP64 iterates: the update kernel tests the gap of every iterate and freezes the
  // instance at the first one below tol; FP32: certify every cert_every iterations.
  const int chunk = (c->prec == BA_PREC_FP64) ? 32 : c->cert_every;
  int done = 0;
  bool all = false;
  if (c->use_graph && !c->stream)
    return fail(c, BA_ESTATE, "graph capture needs a non-null stream (bind one)");
  if (c->use_graph && c->concurrent && c->groups.size() > 1 && (rc = ensure_branches(c))) return rc;
  // the sweeps skip the frozen-flag test while no instance is frozen (the host
  // knows from the states it reads after every chunk)
  auto any_frozen = [&]() {
    for (int i = 0; i < c->count; ++i)
      if (st[i].converged || st[i].bad) return true;
    return false;
  };
  struct FrzScope {
    ba_ctx* c;
    ~FrzScope() { c->frz_override = -1; }
  } frz_scope{c};
  while (done < max_iters) {
    const int k = std::min(chunk, max_iters - done);
    const int frz = any_frozen() ? 1 : 0;
    c->frz_override = frz;
    if (c->use_graph && k == chunk) {
      if (c->gchunk != chunk || c->gengine != c->engine) drop_graph(c);
      if (!c->gexec[frz]) {
        hipGraph_t graph = nullptr;
        HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        const int rc2 = capture_chunk(c, k);
        hipError_t ec = hipStreamEndCapture(c->stream, &graph);
        if (rc2) { if (graph) (void)hipGraphDestroy(graph); return rc2; }
        HIPCHK(c, ec);
        hipError_t ei = hipGraphInstantiate(&c->gexec[frz], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(c, ei);
        c->gchunk = chunk;
        c->gengine = c->engine;
      }
      HIPCHK(c, hipGraphLaunch(c->gexec[frz], c->stream));
    } else {
      if ((rc = ba_step(c, k))) return rc;
      if (c->prec == BA_PREC_FP32_LOG && (rc = certify_all(c, 1))) return rc;
    }
    done += k;
    if ((rc = read_states(c, st))) return rc;
    all = true;
    for (int i = 0; i < c->count; ++i) {
      if (st[i].bad) return fail(c, BA_ENUMERIC, "non-finite value in instance " + std::to_string(i));
      if (!st[i].converged) all = false;
    }
    if (all) break;
  }
  // certify the final iterates (records best bounds)
  if ((rc = certify_all(c, 1))) return rc;
  if ((rc = read_states(c, st))) return rc;
  int most = 0;
  for (int i = 0; i < c->count; ++i) {
    if (st[i].bad) return fail(c, BA_ENUMERIC, "non-finite value in instance " + std::to_string(i));
    most = std::max(most, st[i].iters - start[i]);
  }
  if (iters_done) *iters_done = most;
  return BA_OK;
}

int ba_bounds(ba_ctx* c, double* lower, double* upper) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!lower || !upper) return fail(c, BA_EINVAL, "NULL output");
  if ((rc = certify_all(c, 1))) return rc;
  std::vector<State> st;
  if ((rc = read_states(c, st))) return rc;
  for (int i = 0; i < c->count; ++i)
    if (st[i].bad) return fail(c, BA_ENUMERIC, "non-finite value in instance " + std::to_string(i));
  for (int i = 0; i < c->count; ++i) {
    lower[i] = st[i].certL / kLn2;
    upper[i] = st[i].certU / kLn2;
  }
  return BA_OK;
}

int ba_best_bounds(ba_ctx* c, double* lower, double* upper, int* iters) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!lower || !upper) return fail(c, BA_EINVAL, "NULL output");
  std::vector<State> st;
  if ((rc = read_states(c, st))) return rc;
  for (int i = 0; i < c->count; ++i) {
    lower[i] = st[i].bestL / kLn2;
    upper[i] = st[i].bestU / kLn2;
    if (iters) iters[i] = st[i].iters;
  }
  return BA_OK;
}

int ba_eval(ba_ctx* c, const double* logp_dev, double* r_dev, double* D_dev, double* out4) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!logp_dev) return fail(c, BA_EINVAL, "NULL logp");
  const auto [gi, slot] = c->where[0];
  GroupHost& gh = c->groups[gi];
  Group<double> src = slot_view(gh.gd, 0);
  src.lp = const_cast<double*>(logp_dev);
  src.xs = size_t(1) << gh.n;
  Group<double> cert = slot_view(gh.cert, slot);
  State* scratch = reinterpret_cast<State*>(c->ws + c->misc + 256);
  HIPCHK(c, launch_fill_zero(scratch, 256, c->stream));
  if ((rc = certify_group<double>(c, gh, src, cert, scratch, 0))) return rc;
  const size_t X = size_t(1) << gh.n;
  if (r_dev) HIPCHK(c, launch_copy_f64(r_dev, cert.r, out_count(gh.n), c->stream));
  if (D_dev) HIPCHK(c, launch_copy_f64(D_dev, cert.D, X, c->stream));
  State h;
  HIPCHK(c, hipMemcpyAsync(&h, scratch, sizeof(State), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (h.bad) return fail(c, BA_ENUMERIC, "non-finite value in logp");
  if (out4) {
    out4[0] = h.certL / kLn2;
    out4[1] = h.certU / kLn2;
    out4[2] = h.certI / kLn2;
    out4[3] = h.certM;
  }
  return BA_OK;
}

int ba_grad(ba_ctx* c, const double* theta_dev, double* I_bits, double* dI_dtheta_dev, double* dI_dd_bits) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!theta_dev || !I_bits) return fail(c, BA_EINVAL, "NULL theta or I");
  if (dI_dd_bits && (c->kexact[0] >= 0 || !(c->d[0] > 0.0 && c->d[0] < 1.0)))
    return fail(c, BA_EINVAL, "dI/dd is undefined at d = 0 or d = 1");
  const auto [gi, slot] = c->where[0];
  GroupHost& gh = c->groups[gi];
  hipStream_t s = c->stream;
  const int nblk = reduce_blocks(gh.n);
  Group<double> src = slot_view(gh.gd, 0);
  src.lp = const_cast<double*>(theta_dev);
  src.xs = size_t(1) << gh.n;
  Group<double> cert = slot_view(gh.cert, slot);
  HIPCHK(c, launch_cert_prepare<double>(src, cert, nblk, kFloor64, s));
  if ((rc = sweeps<double>(c, gh, cert, 0, cert.g))) return rc;
  // second gather with v = s_k w_k log r: Gd
  const int n1 = (gh.n + 1) / 2, n2 = gh.n / 2;
  {
    Group<double> Gd = cert;
    Gd.g = cert.gd;
    const bool split = c->engine != BA_ENGINE_FACTORED;  // stream gather for W v
    HIPCHK(c, launch_logr<double>(cert, 1, split, n1, n2, s));
    if (split) {
      const StreamExtra ex{};
      HIPCHK(c, launch_fill_zero(cert.gd, cert.xs * sizeof(double), s));
      HIPCHK(c, launch_stream<double>(kOpGather, gh.tb, Gd, 0, ex, s));
    } else {
      Gd.s8lc = c->s8lc;
      HIPCHK(c, launch_backward<double>(Gd, s, nullptr, c->fuse, 0, nullptr));
    }
  }
  HIPCHK(c, launch_dpart<double>(cert, nblk, 1, cert.gd, s));
  double* out4 = reinterpret_cast<double*>(c->ws + c->misc + 128);
  HIPCHK(c, launch_grad_finish(cert, nblk, out4, dI_dtheta_dev, s));
  double h[4];
  HIPCHK(c, hipMemcpyAsync(h, out4, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (!isfinite(h[0]) || !isfinite(h[1])) return fail(c, BA_ENUMERIC, "non-finite gradient");
  *I_bits = h[0];
  if (dI_dd_bits) *dI_dd_bits = h[1];
  return BA_OK;
}

int ba_mirror_ascent(ba_ctx* c, double* theta_dev, double eta, int steps) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!theta_dev || steps < 0 || !isfinite(eta)) return fail(c, BA_EINVAL, "bad mirror-ascent arguments");
  const auto [gi, slot] = c->where[0];
  GroupHost& gh = c->groups[gi];
  const int nblk = reduce_blocks(gh.n);
  Group<double> src = slot_view(gh.gd, 0);
  src.lp = theta_dev;
  src.xs = size_t(1) << gh.n;
  Group<double> cert = slot_view(gh.cert, slot);
  for (int t = 0; t < steps; ++t) {
    HIPCHK(c, launch_cert_prepare<double>(src, cert, nblk, kFloor64, c->stream));
    if ((rc = sweeps<double>(c, gh, cert, 0, cert.g))) return rc;
    HIPCHK(c, launch_dpart<double>(cert, nblk, 0, nullptr, c->stream));
    HIPCHK(c, launch_mirror_update(gh.n, theta_dev, cert.D, eta, c->stream));
  }
  return BA_OK;
}

int ba_get_logp(ba_ctx* c, double* logp_dev) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!logp_dev) return fail(c, BA_EINVAL, "NULL logp");
  size_t off = 0;
  for (int i = 0; i < c->count; ++i) {
    const auto [gi, slot] = c->where[i];
    GroupHost& gh = c->groups[gi];
    if (c->prec == BA_PREC_FP32_LOG) HIPCHK(c, launch_get_logp<float>(slot_view(gh.gf, slot), logp_dev + off, c->stream));
    else HIPCHK(c, launch_get_logp<double>(slot_view(gh.gd, slot), logp_dev + off, c->stream));
    off += size_t(1) << c->n[i];
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return BA_OK;
}

// Symmetric mode: check that every instance's iterate is invariant under
// complement (within a rounding tolerance of its precision), then make it exactly
// so by copying the half x < 2^(n-1) onto the complements.
int sym_check_and_fix(ba_ctx* c) {
  hipStream_t s = c->stream;
  double* dev = reinterpret_cast<double*>(c->ws + c->symdev);
  std::vector<double> host(c->count);
  size_t k = 0;
  std::vector<std::pair<size_t, size_t>> span;  // per group: first slot in dev, count
  for (auto& gh : c->groups) {
    const int orbit = c->sym == 2 ? 1 : 0;
    if (c->prec == BA_PREC_FP32_LOG) HIPCHK(c, launch_sym_check<float>(gh.gf, dev + k, orbit, s));
    else HIPCHK(c, launch_sym_check<double>(gh.gd, dev + k, orbit, s));
    span.push_back({k, gh.inst.size()});
    k += gh.inst.size();
  }
  HIPCHK(c, hipMemcpyAsync(host.data(), dev, k * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  const double tol = (c->prec == BA_PREC_FP32_LOG) ? 1e-4 : 1e-9;
  for (size_t gi = 0; gi < c->groups.size(); ++gi)
    for (size_t j = 0; j < span[gi].second; ++j) {
      const double dv = host[span[gi].first + j];
      if (!(dv <= tol))
        return fail(c, BA_EINVAL, "iterate of instance " + std::to_string(c->groups[gi].inst[j]) +
                                      (c->sym == 2 ? " is not invariant under complement and reversal"
                                                    : " is not complement-symmetric") +
                                      " (max |log p(x) - log p(g x)| = " +
                                      std::to_string(dv) + ")");
    }
  for (auto& gh : c->groups) {
    const int orbit = c->sym == 2 ? 1 : 0;
    if (c->prec == BA_PREC_FP32_LOG) HIPCHK(c, launch_symmetrize<float>(gh.gf, orbit, s));
    else HIPCHK(c, launch_symmetrize<double>(gh.gd, orbit, s));
  }
  return BA_OK;
}

int ba_set_logp(ba_ctx* c, const double* logp_dev) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!logp_dev) return fail(c, BA_EINVAL, "NULL logp");
  size_t off = 0;
  for (int i = 0; i < c->count; ++i) {
    const auto [gi, slot] = c->where[i];
    GroupHost& gh = c->groups[gi];
    const int nblk = reduce_blocks(gh.n);
    const double floor = iterate_floor(c);
    if (c->prec == BA_PREC_FP32_LOG) HIPCHK(c, launch_set_logp<float>(slot_view(gh.gf, slot), logp_dev + off, nblk, floor, c->stream));
    else HIPCHK(c, launch_set_logp<double>(slot_view(gh.gd, slot), logp_dev + off, nblk, floor, c->stream));
    off += size_t(1) << c->n[i];
  }
  std::vector<State> st;
  if ((rc = read_states(c, st))) return rc;
  for (int i = 0; i < c->count; ++i)
    if (st[i].bad) return fail(c, BA_ENUMERIC, "logp contains NaN or +Inf (instance " + std::to_string(i) + ")");
  if (c->sym && (rc = sym_check_and_fix(c))) {
    c->sym = 0;
    drop_graph(c);
    return rc;
  }
  return BA_OK;
}

int ba_set_step(ba_ctx* c, double eta) {
  if (!c) return BA_EINVAL;
  if (!(eta > 0.0 && eta <= 8.0)) return fail(c, BA_EINVAL, "step must be in (0, 8]");
  c->eta = eta;
  drop_graph(c);
  return BA_OK;
}

int ba_set_floor(ba_ctx* c, double nats) {
  if (!c) return BA_EINVAL;
  const double top = (c->prec == BA_PREC_FP32_LOG) ? kFloor32Max : kFloor64;
  if (!(nats >= kFloorMin && nats <= top))
    return fail(c, BA_EINVAL, "floor must be in [" + std::to_string(int(kFloorMin)) + ", " +
                                  std::to_string(int(top)) + "] nats for this precision");
  c->floor = nats;
  drop_graph(c);
  return BA_OK;
}

int ba_set_symmetry(ba_ctx* c, int enable) {
  if (!c || enable < 0 || enable > 2) return c ? fail(c, BA_EINVAL, "enable must be 0, 1 or 2") : BA_EINVAL;
  if (enable && c->bound) {
    c->sym = enable;
    const int rc = sym_check_and_fix(c);
    if (rc) {
      c->sym = 0;
      return rc;
    }
  }
  c->sym = enable;
  drop_graph(c);
  return BA_OK;
}

int ba_row_counts(ba_ctx* c, uint32_t x, uint32_t* rank_dev, uint32_t* emb_dev, int cap, int* nnz) {
  int rc = check_ctx(c);
  if (rc) return rc;
  const auto [gi, slot] = c->where[0];
  GroupHost& gh = c->groups[gi];
  if (!nnz || x >= (1u << gh.n) || cap < 0 || (cap > 0 && (!rank_dev || !emb_dev)))
    return fail(c, BA_EINVAL, "bad row arguments");
  hipStream_t s = c->stream;
  uint32_t* dense = reinterpret_cast<uint32_t*>(c->ws + c->verify);
  uint32_t* nnz_dev = reinterpret_cast<uint32_t*>(c->ws + c->misc + 64);
  HIPCHK(c, launch_fill_zero(dense, al256(size_t(out_count(gh.n)) * 4), s));
  StreamExtra ex{};
  ex.target_x = x;
  ex.row_dense = dense;
  HIPCHK(c, launch_stream<double>(kOpRow, gh.tb, slot_view(gh.cert, slot), 0, ex, s));
  HIPCHK(c, launch_row_compact(dense, gh.n, rank_dev, emb_dev, cap, nnz_dev, s));
  uint32_t h = 0;
  HIPCHK(c, hipMemcpyAsync(&h, nnz_dev, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  *nnz = int(h);
  if (int(h) > cap) return fail(c, BA_EINVAL, "cap smaller than the row's nonzero count");
  return BA_OK;
}

int ba_verify_counts(ba_ctx* c, uint64_t* stats) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!stats) return fail(c, BA_EINVAL, "NULL stats");
  const auto [gi, slot] = c->where[0];
  GroupHost& gh = c->groups[gi];
  hipStream_t s = c->stream;
  uint32_t* bins = reinterpret_cast<uint32_t*>(c->ws + c->verify);
  unsigned long long* st_dev = reinterpret_cast<unsigned long long*>(c->ws + c->misc);
  HIPCHK(c, launch_fill_zero(bins, al256(c->verify_bytes), s));
  unsigned long long init[8] = {0, 0, 0, ~0ull, 0, 0, 0, 0};
  HIPCHK(c, hipMemcpyAsync(st_dev, init, sizeof(init), hipMemcpyHostToDevice, s));
  StreamExtra ex{};
  ex.bins = bins;
  ex.stats = st_dev;
  HIPCHK(c, launch_stream<double>(kOpVerify, gh.tb, slot_view(gh.cert, slot), 0, ex, s));
  unsigned long long h[8];
  HIPCHK(c, hipMemcpyAsync(h, st_dev, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  for (int i = 0; i < 6; ++i) stats[i] = h[i];
  stats[2] = 0;
  return BA_OK;
}

int ba_time_kernels(ba_ctx* c, int iters, double* ms, int* launches) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!ms || iters < 0) return fail(c, BA_EINVAL, "bad timing arguments");
  for (auto e : c->ev) (void)hipEventDestroy(e);
  c->ev.clear();
  c->ev_class.clear();
  c->ev_kernels.clear();
  c->timing = true;
  rc = ba_step(c, iters);
  c->timing = false;
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < BA_NKCLASS; ++k) {
    ms[k] = 0.0;
    if (launches) launches[k] = 0;
  }
  for (size_t i = 0; i + 1 < c->ev.size(); i += 2) {
    float t = 0.f;
    HIPCHK(c, hipEventElapsedTime(&t, c->ev[i], c->ev[i + 1]));
    const int k = c->ev_class[i];
    if (k >= 0 && k < BA_NKCLASS) {
      ms[k] += t;
      if (launches) launches[k] += c->ev_kernels[i];
    }
  }
  for (auto e : c->ev) (void)hipEventDestroy(e);
  c->ev.clear();
  c->ev_class.clear();
  c->ev_kernels.clear();
  return BA_OK;
}

int ba_instance_count(const ba_ctx* c) { return c ? c->count : 0; }

uint64_t ba_nnz(int n) {
  if (n < 0 || n > 40) return 0;
  return 2 * ipow3(n) - (uint64_t(1) << n);
}

const char* ba_strerror(int code) {
  switch (code) {
    case BA_OK: return "ok";
    case BA_EINVAL: return "invalid argument";
    case BA_ENOMEM: return "out of memory or workspace too small";
    case BA_EDEVICE: return "HIP device error";
    case BA_ESTATE: return "invalid state";
    case BA_ENUMERIC: return "non-finite value";
  }
  return "unknown error";
}

const char* ba_last_error(const ba_ctx* c) { return c ? c->err.c_str() : ""; }

}  // extern "C"
