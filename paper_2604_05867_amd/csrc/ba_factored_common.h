// Device helpers shared by the factored-engine kernels (full and complement-
// symmetric variants): vector loads, the row visiting order of a launch, the
// fused D epilogue and the register part of the four-position forward step.
// Included by ba_factored.hip and ba_symmetric.hip only.
#pragma once

#include "ba_internal.h"
#include "ba_part.h"

namespace ba {
namespace fac {

// Vector of V consecutive elements (16-byte loads/stores when V*sizeof(T) is a
// multiple of 16 and the address is aligned to it).
template <typename T, int V>
struct Vec {
  T v[V];
};
template <typename T, int V>
__device__ __forceinline__ Vec<T, V> ld(const T* p) {
  Vec<T, V> r;
  if constexpr ((V * sizeof(T)) % 16 == 0) {
#pragma unroll
    for (int k = 0; k < int(V * sizeof(T) / 16); ++k)
      reinterpret_cast<uint4*>(r.v)[k] = reinterpret_cast<const uint4*>(p)[k];
  } else {
#pragma unroll
    for (int k = 0; k < V; ++k) r.v[k] = p[k];
  }
  return r;
}
template <typename T, int V>
__device__ __forceinline__ void stv(T* p, const Vec<T, V>& a) {
  if constexpr ((V * sizeof(T)) % 16 == 0) {
#pragma unroll
    for (int k = 0; k < int(V * sizeof(T) / 16); ++k)
      reinterpret_cast<uint4*>(p)[k] = reinterpret_cast<const uint4*>(a.v)[k];
  } else {
#pragma unroll
    for (int k = 0; k < V; ++k) p[k] = a.v[k];
  }
}

__device__ __forceinline__ int length_of_rank(uint32_t r) { return 31 - __clz(r + 1u); }

// Element idx of an array whose byte size is below 4 GiB, addressed as a 32-bit
// byte offset from the (wavefront-uniform) base, so that the access can take the
// base from scalar registers and one vector register for the offset.
template <typename T>
__device__ __forceinline__ T& at(T* base, uint32_t idx) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * uint32_t(sizeof(T)));
}
template <typename T>
__device__ __forceinline__ const T& at(const T* base, uint32_t idx) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * uint32_t(sizeof(T)));
}

// Rank of the complement of the string of rank R (same length).
__device__ __forceinline__ uint32_t mirror_rank(uint32_t R) {
  return 3u * (1u << length_of_rank(R)) - 3u - R;
}

// Compact index of the canonical member of {y, cpl y} (complement-symmetric
// iteration): the empty row at 0, a row 0z of length k at 2^(k-1) + bits(z).
__device__ __forceinline__ uint32_t compact_rank(uint32_t R) {
  if (R == 0u) return 0u;
  const int k = length_of_rank(R);
  const uint32_t a = R + 1u - (1u << k), half = 1u << (k - 1);
  return half + (a < half ? a : (2u * half - 1u - a));
}

template <typename T, int V>
__device__ __forceinline__ Vec<T, V> zero_vec() {
  Vec<T, V> z;
#pragma unroll
  for (int k = 0; k < V; ++k) z.v[k] = T(0);
  return z;
}

// v(y) = w_k log r(y) for the output of rank y (0 where w_k = 0).
template <typename T>
__device__ __forceinline__ T log_weighted(const Consts& cs, uint32_t y, T r) {
  return wlog_t<T>(T(cs.w[length_of_rank(y)]), r);
}

// ---------------------------------------------------------------------------
// Visiting order of the rows of a two-position launch.
//
// Output row c needs source rows c, its parent and its grandparent (forward), or
// its children and grandchildren (backward).  In plain rank order those are read
// again far apart in time (rank c vs 2c vs 4c), and most re-reads miss the
// per-XCD L2.  Instead, per column tile of 2^cw_log2 chunks, the rows above level
// lb are visited first in rank order, then the subtrees rooted at level lb one
// after another, each breadth-first (2^h - 1 rows in 2^h slots), so every re-read
// row was fetched a subtree (<= kTileBytes) earlier.  Logical blocks are spread
// over the XCDs in contiguous runs (hardware block b runs on XCD b mod 8), so one
// subtree stays on one L2.
// ---------------------------------------------------------------------------
struct Order {
  uint32_t nlog;  // logical row slots per column tile (per unit when kb > 0)
  uint32_t top;   // rows above level lb: 2^lb - 1
  uint32_t nct;   // column tiles
  int lb, h;      // level of the subtree roots, subtree height (levels)
  int cw_log2;    // log2 of the column-tile width in chunks
  uint32_t kb;    // 0, or blocks per XCD of the unit partition (make_order_xcd)
  uint32_t mir;   // unit partition: subtree t shares its XCD with 2^lb - 1 - t
};

constexpr size_t kTileBytes = size_t(1) << 19;

// levels: output levels of the launch (rows 0 .. 2^levels - 2); cols_log2: log2
// of the chunks per row; chunk_bytes: bytes one thread covers in a source row.
inline Order make_order(int levels, int cols_log2, size_t chunk_bytes) {
  Order o;
  o.cw_log2 = cols_log2 < 6 ? cols_log2 : 6;
  const size_t seg = (size_t(1) << o.cw_log2) * chunk_bytes;
  int h = 1;
  while (h < levels && (seg << (h + 1)) <= kTileBytes) ++h;
  o.h = h;
  o.lb = levels - h;
  o.top = (1u << o.lb) - 1u;
  o.nlog = (o.lb == 0) ? (1u << h) - 1u : o.top + (1u << (o.lb + h));
  o.nct = 1u << (cols_log2 - o.cw_log2);
  o.kb = 0;
  o.mir = 0;
  return o;
}

inline uint32_t order_threads(const Order& o) { return o.nct * o.nlog << o.cw_log2; }

// A partition of the launch into 8 m units that are each read from one XCD's L2
// only: a unit is one column tile of the whole tree (rows of >= 256 chunks, tiles
// of 32 or 64 chunks), or, for narrower rows, one of the 8 subtrees rooted at
// level 3 over all columns.  A row's ancestors then lie in its own unit (or among
// the 7 rows above level 3, visited by the trailing blocks), so a row read again
// by its descendants is an L2 hit instead of a fetch by a second XCD.  Each unit
// holds 2^h slots (the subtree's rows breadth-first and one padding slot) per
// chunk; XCD x runs units x m .. x m + m - 1 (hardware block 8 k + x, k < kb).
// mirror: a thread also reads the complement of its row (the complement-symmetric
// kernels), so the subtrees are rooted at level 4 and XCD x takes the complementary
// pair x, 15 - x.  False when a unit is not a whole number of blocks.
inline bool make_order_xcd(int levels, int cols_log2, uint32_t block, Order& o, bool mirror = false) {
  int cw, lb;
  if (cols_log2 >= 8) {
    cw = cols_log2 - 3 < 6 ? cols_log2 - 3 : 6;
    lb = 0;
  } else {
    cw = cols_log2;
    lb = mirror ? 4 : 3;
  }
  const int h = levels - lb;
  if (h < 1 || h + cw > 30 || ((uint32_t(1) << (h + cw)) % block) != 0u) return false;
  o.cw_log2 = cw;
  o.lb = lb;
  o.h = h;
  o.top = (1u << lb) - 1u;
  o.nct = 1u << (cols_log2 - cw);
  o.nlog = 1u << h;
  o.kb = ((o.nct << lb) >> 3) * ((uint32_t(1) << (h + cw)) / block);
  o.mir = lb == 4 ? 1u : 0u;
  return true;
}

// Blocks of an ordered launch with `block` threads per block.
inline uint32_t order_blocks(const Order& o, uint32_t block) {
  if (o.kb == 0u) {
    const uint32_t t = order_threads(o);
    const uint32_t g = t == 0 ? 1u : (t + block - 1) / block;
    return (g + 7u) & ~7u;
  }
  const uint32_t tb = ((o.top << o.cw_log2) + block - 1u) / block;  // the rows above level lb
  return 8u * (o.kb + (tb + 7u) / 8u);
}

__device__ __forceinline__ uint32_t logical_block() {
  const uint32_t G = gridDim.x, bx = blockIdx.x;
  return (G & 7u) ? bx : (bx & 7u) * (G >> 3) + (bx >> 3);
}

// (row, chunk) of logical slot q; false for a padding slot or past the end.
__device__ __forceinline__ bool order_slot_q(const Order& o, uint32_t q, uint32_t& row, uint32_t& chunk) {
  const uint32_t rest = q >> o.cw_log2;
  // one column tile (narrow rows): no division
  const uint32_t ct = (o.nct == 1u) ? (rest >= o.nlog ? 1u : 0u) : rest / o.nlog;
  if (ct >= o.nct) return false;
  uint32_t L = rest - ct * o.nlog;
  chunk = (ct << o.cw_log2) + (q & ((1u << o.cw_log2) - 1u));
  if (L < o.top) {
    row = L;
    return true;
  }
  L -= o.top;
  const uint32_t mask = (1u << o.h) - 1u;
  const uint32_t t = L >> o.h, j = L & mask;
  if (j == mask) return false;
  const int k = 31 - __clz(j + 1u);
  row = (1u << (o.lb + k)) - 1u + (t << k) + (j + 1u - (1u << k));
  return true;
}

// (row, chunk) of this thread in the unit partition of make_order_xcd.
__device__ __forceinline__ bool order_slot_xcd(const Order& o, uint32_t& row, uint32_t& chunk) {
  const uint32_t x = blockIdx.x & 7u, k = blockIdx.x >> 3;
  const uint32_t cmask = (1u << o.cw_log2) - 1u;
  if (k >= o.kb) {  // the rows above level lb (one column tile)
    const uint32_t q = (((k - o.kb) << 3) + x) * kBlock + threadIdx.x;
    row = q >> o.cw_log2;
    chunk = q & cmask;
    return row < o.top;
  }
  const uint32_t q = (x * o.kb + k) * kBlock + threadIdx.x;
  const int ul = o.h + o.cw_log2;
  const uint32_t unit = q >> ul, r = q & ((1u << ul) - 1u);
  const uint32_t j = r >> o.cw_log2;
  if (j == o.nlog - 1u) return false;
  const uint32_t ct = unit >> o.lb;
  uint32_t t = unit & o.top;
  if (o.mir) t = (t & 1u) ? o.top - (t >> 1) : (t >> 1);  // units 2x, 2x + 1: subtrees x, 15 - x
  const int lv = 31 - __clz(j + 1u);
  row = (1u << (o.lb + lv)) - 1u + (t << lv) + (j + 1u - (1u << lv));
  chunk = (ct << o.cw_log2) + (r & cmask);
  return true;
}

// This thread's (row, chunk), one slot per thread.  Every kernel that takes an
// Order runs kBlock threads per block; the block size is that constant rather than
// blockDim.x, which is read from the dispatch packet with a vector load that each
// wavefront would wait for before forming its first address.
__device__ __forceinline__ bool order_slot(const Order& o, uint32_t& row, uint32_t& chunk) {
  if (o.kb != 0u) return order_slot_xcd(o, row, chunk);
  return order_slot_q(o, logical_block() * kBlock + threadIdx.x, row, chunk);
}

// The loads of H and log p for d_records_pre (issued early by callers that hold
// them while other work runs).
template <typename T, int V, int N>
__device__ __forceinline__ void d_loads(const Group<T>& g, int b, const uint32_t (&x)[N], Vec<T, V> (&h)[N],
                                        Vec<T, V> (&l)[N]) {
  const T* hf = g.hf + (size_t)b * g.xs;
  const T* lp = g.lp + (size_t)b * g.xs;
#pragma unroll
  for (int u = 0; u < N; ++u) {
    h[u] = ld<T, V>(hf + x[u]);
    l[u] = ld<T, V>(lp + x[u]);
  }
}

// D(x) = H(x) - G(x) - M for N groups of V consecutive inputs (group u starts at
// input x[u]), with H (in d, replaced by D) and log p (l) already loaded: D (or log p
// + D, Group::dsum) is stored and the inputs' terms are added to the record p.  The maxima of log p + D
// (and of log p + eta D) and of D over the groups, then the sums of exponentials
// relative to those maxima and of p D, are formed in the iterate's precision T with
// no branch per input, and folded into p once.  wt: the number of inputs each value
// stands for (2 when only one of each complement pair is evaluated).
template <typename T, int V, int N>
__device__ __forceinline__ void d_records_pre(const Group<T>& g, int b, double M, const uint32_t (&x)[N],
                                              const Vec<T, V> (&G)[N], Vec<T, V> (&d)[N], const Vec<T, V> (&l)[N],
                                              Part& p, double wt = 1.0) {
  T* D = g.D + (size_t)b * g.xs;
  T am = T(-INFINITY), dm = T(-INFINITY);
  Vec<T, V> a[N];  // log p + D
#pragma unroll
  for (int u = 0; u < N; ++u)
#pragma unroll
    for (int k = 0; k < V; ++k) {
      d[u].v[k] = d[u].v[k] - G[u].v[k] - T(M);
      a[u].v[k] = l[u].v[k] + d[u].v[k];
      am = fmax(am, a[u].v[k]);
      dm = fmax(dm, d[u].v[k]);
    }
  if (g.dsum) {  // uniform: one store loop or the other (a selected struct would go to scratch)
#pragma unroll
    for (int u = 0; u < N; ++u) stv<T, V>(D + x[u], a[u]);
  } else {
#pragma unroll
    for (int u = 0; u < N; ++u) stv<T, V>(D + x[u], d[u]);
  }
  T s = T(0), i = T(0);
#pragma unroll
  for (int u = 0; u < N; ++u)
#pragma unroll
    for (int k = 0; k < V; ++k) {
      s += exp_t<T>((l[u].v[k] + d[u].v[k]) - am);
      i += exp_t<T>(l[u].v[k]) * d[u].v[k];
    }
  Part q{double(am), wt * double(s), double(dm), wt * double(i), 0.0, -INFINITY, 0.0};
  if (g.eta != 1.0) {
    const T eta = T(g.eta);
    T m2 = T(-INFINITY), s2 = T(0);
#pragma unroll
    for (int u = 0; u < N; ++u)
#pragma unroll
      for (int k = 0; k < V; ++k) m2 = fmax(m2, l[u].v[k] + eta * d[u].v[k]);
#pragma unroll
    for (int u = 0; u < N; ++u)
#pragma unroll
      for (int k = 0; k < V; ++k) s2 += exp_t<T>((l[u].v[k] + eta * d[u].v[k]) - m2);
    q.m2 = double(m2);
    q.s2 = wt * double(s2);
  }
  p = part_is_empty(p) ? q : combine(p, q);
}

// d_records_pre for FP32 iterates with the thread's record left in single precision
// (q, for store_block_part_f32); D is that of d_records_pre, the record's sums use
// the hardware exponential (2^(x log2 e), relative error below |x| 2^-23), which the
// single-precision record of an FP32 iterate does not need better than that.
// half: the inputs stand for themselves and their complements (complement-symmetric
// iterate): log p + D (or D) is written at x and at cpl x = 2^n - 1 - x, and the
// record's sums count every input twice.
__device__ __forceinline__ void d_records_pre_f(const Group<float>& g, int b, double M, const uint32_t (&x)[2],
                                                const Vec<float, 4> (&G)[2], Vec<float, 4> (&d)[2],
                                                const Vec<float, 4> (&l)[2], PartF& q, bool half = false) {
  using T = float;
  constexpr int N = 2, V = 4;
  T* D = g.D + (size_t)b * g.xs;
  T am = T(-INFINITY), dm = T(-INFINITY);
  Vec<T, V> a[N];  // log p + D
#pragma unroll
  for (int u = 0; u < N; ++u)
#pragma unroll
    for (int k = 0; k < V; ++k) {
      d[u].v[k] = d[u].v[k] - G[u].v[k] - T(M);
      a[u].v[k] = l[u].v[k] + d[u].v[k];
      am = fmax(am, a[u].v[k]);
      dm = fmax(dm, d[u].v[k]);
    }
  if (g.dsum) {  // uniform: one store loop or the other (a selected struct would go to scratch)
#pragma unroll
    for (int u = 0; u < N; ++u) stv<T, V>(D + x[u], a[u]);
  } else {
#pragma unroll
    for (int u = 0; u < N; ++u) stv<T, V>(D + x[u], d[u]);
  }
  if (half) {
    const uint32_t X = 1u << g.n;
#pragma unroll
    for (int u = 0; u < N; ++u) {
      Vec<T, V> r;
#pragma unroll
      for (int k = 0; k < V; ++k) r.v[k] = g.dsum ? a[u].v[V - 1 - k] : d[u].v[V - 1 - k];
      stv<T, V>(D + (X - uint32_t(V) - x[u]), r);
    }
  }
  T s = T(0), i = T(0);
#pragma unroll
  for (int u = 0; u < N; ++u)
#pragma unroll
    for (int k = 0; k < V; ++k) {
      s += __expf((l[u].v[k] + d[u].v[k]) - am);
      i += __expf(l[u].v[k]) * d[u].v[k];
    }
  if (half) {
    s += s;
    i += i;
  }
  q = PartF{am, s, dm, i, T(-INFINITY), T(0)};
  if (g.eta != 1.0) {
    const T eta = T(g.eta);
    T m2 = T(-INFINITY), s2 = T(0);
#pragma unroll
    for (int u = 0; u < N; ++u)
#pragma unroll
      for (int k = 0; k < V; ++k) m2 = fmax(m2, l[u].v[k] + eta * d[u].v[k]);
#pragma unroll
    for (int u = 0; u < N; ++u)
#pragma unroll
      for (int k = 0; k < V; ++k) s2 += __expf((l[u].v[k] + eta * d[u].v[k]) - m2);
    q.m2 = m2;
    q.s2 = half ? s2 + s2 : s2;
  }
}

// d_records_pre with its own loads.
template <typename T, int V, int N>
__device__ __forceinline__ void d_records(const Group<T>& g, int b, double M, const uint32_t (&x)[N],
                                          const Vec<T, V> (&G)[N], Part& p, double wt = 1.0) {
  // every load before the first store: D could alias H or log p as far as the
  // compiler knows, so a store between them would serialise each load behind it
  Vec<T, V> l[N], d[N];
  d_loads<T, V, N>(g, b, x, d, l);
  d_records_pre<T, V, N>(g, b, M, x, G, d, l, p, wt);
}

// Register parts of the four-position forward step for one (y, column).
//
// The 30 rows below a row y after four stages, from y's values at the first three
// of them (F1z = F_{i+1}[y], 8 column groups; F2z, F3z) and F1s, the two children of
// y at stage i+1 (the halves of F_i[y]): breadth-first, depth d index m at
// (1 << d) - 2 + m.
template <typename T>
__device__ __forceinline__ void fwd4_subtree(const T (&F1z)[8], const T (&F2z)[4], const T (&F3z)[2],
                                             const T (&F1s)[2][8], T (&F4)[30]) {
  // stage 2: subtree depth 1..2 (breadth-first 0..5)
  T F2s[6][4];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int g = 0; g < 4; ++g) F2s[c][g] = (F1s[c][g] + F1s[c][4 + g]) + F1z[c * 4 + g];
#pragma unroll
  for (int c = 0; c < 4; ++c)  // depth 2: child c/2 of y, then bit c&1
#pragma unroll
    for (int g = 0; g < 4; ++g) F2s[2 + c][g] = F1s[c >> 1][(c & 1) * 4 + g];
  // stage 3: subtree depth 1..3 (breadth-first 0..13)
  T F3s[14][2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int g = 0; g < 2; ++g) F3s[c][g] = (F2s[c][g] + F2s[c][2 + g]) + F2z[c * 2 + g];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int g = 0; g < 2; ++g) F3s[2 + c][g] = (F2s[2 + c][g] + F2s[2 + c][2 + g]) + F2s[c >> 1][(c & 1) * 2 + g];
#pragma unroll
  for (int c = 0; c < 8; ++c)
#pragma unroll
    for (int g = 0; g < 2; ++g) F3s[6 + c][g] = F2s[2 + (c >> 1)][(c & 1) * 2 + g];
  // stage 4: subtree depth 1..4
#pragma unroll
  for (int c = 0; c < 2; ++c) F4[c] = (F3s[c][0] + F3s[c][1]) + F3z[c];
#pragma unroll
  for (int c = 0; c < 4; ++c) F4[2 + c] = (F3s[2 + c][0] + F3s[2 + c][1]) + F3s[c >> 1][c & 1];
#pragma unroll
  for (int c = 0; c < 8; ++c) F4[6 + c] = (F3s[6 + c][0] + F3s[6 + c][1]) + F3s[2 + (c >> 1)][c & 1];
#pragma unroll
  for (int c = 0; c < 16; ++c) F4[14 + c] = F3s[6 + (c >> 1)][c & 1];
}

// first stage on: F1p holds F_{i+1} of the path P_0 = y .. P_3 (8 groups), F1s
// that of the two children of y; lastb[j] = last bit of P_j.  Returns F_{i+4}[y]
// and, in F4, the 30 rows below y (as fwd4_subtree).
template <typename T>
__device__ __forceinline__ T fwd4_after_stage1(const T (&F1p)[4][8], const T (&F1s)[2][8],
                                               const uint32_t (&lastb)[4], T (&F4)[30]) {
  // stage 2: path P_0..P_2 (4 groups)
  T F2p[3][4];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int g = 0; g < 4; ++g)
      F2p[j][g] = (F1p[j][g] + F1p[j][4 + g]) + (lastb[j] ? F1p[j + 1][4 + g] : F1p[j + 1][g]);
  // stage 3: path P_0..P_1 (2 groups)
  T F3p[2][2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int g = 0; g < 2; ++g)
      F3p[j][g] = (F2p[j][g] + F2p[j][2 + g]) + (lastb[j] ? F2p[j + 1][2 + g] : F2p[j + 1][g]);
  fwd4_subtree<T>(F1p[0], F2p[0], F3p[0], F1s, F4);
  // stage 4: y (1 group)
  return (F3p[0][0] + F3p[0][1]) + (lastb[0] ? F3p[1][1] : F3p[1][0]);
}

// Stage 1 from the loaded rows F0 (path P_0..P_3, 16 column groups) and H4 (the
// half of P_4 selected by the last bit of P_3), then stages 2-4.
template <typename T>
__device__ __forceinline__ T fwd4_registers(const T (&F0)[4][16], const T (&H4)[8], const uint32_t (&lastb)[4],
                                            T (&F4)[30]) {
  // stage 1: path P_0..P_3 (8 groups), children of y (parent halves chosen by
  // select, so every register index is static)
  T F1p[4][8], F1s[2][8];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int g = 0; g < 8; ++g)
      F1p[j][g] = (F0[j][g] + F0[j][8 + g]) + (lastb[j] ? F0[j + 1][8 + g] : F0[j + 1][g]);
#pragma unroll
  for (int g = 0; g < 8; ++g) F1p[3][g] = (F0[3][g] + F0[3][8 + g]) + H4[g];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int g = 0; g < 8; ++g) F1s[c][g] = F0[0][c * 8 + g];
  return fwd4_after_stage1<T>(F1p, F1s, lastb, F4);
}

// Path ranks of y and their last bits: P_{j+1} = parent(P_j) (garbage past the
// empty row; such rows are never loaded).
__device__ __forceinline__ void fwd4_path(uint32_t y, uint32_t (&P)[5], uint32_t (&lastb)[4]) {
  P[0] = y;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    lastb[j] = (P[j] - 1u) & 1u;
    P[j + 1] = (P[j] - 1u) >> 1;
  }
}

inline uint32_t grid_for(uint32_t total) {
  uint32_t g = (total + kBlock - 1) / kBlock;
  return g > 8192u ? 8192u : (g == 0 ? 1u : g);
}

// Blocks for an ordered launch, a multiple of 8 so that the XCD placement of
// logical_block applies (the extra blocks find no slot).
inline uint32_t blocks_for(uint32_t threads, uint32_t block = kBlock) {
  const uint32_t g = threads == 0 ? 1u : (threads + block - 1) / block;
  return (g + 7u) & ~7u;
}

// Threads per block of the four-position launches without records.
constexpr uint32_t kStage4Block = kBlock;

// The last four forward positions in one launch (k_fwd_last4, k_fwd_last4_sym): from
// this n on, with blocks of kLast4Threads and kLast4Stage values of LDS staging (the
// 2 + 4 + 8 + 16 rows below each of 64 leaves, padded to odd row strides).
constexpr int kLast4MinN = 12;
constexpr int kLast4Threads = 128;
constexpr int kLast4Stage = (3 + 5 + 9 + 17) * 64;

inline int ilog2(uint32_t v) { return 31 - __builtin_clz(v); }

}  // namespace fac
}  // namespace ba
