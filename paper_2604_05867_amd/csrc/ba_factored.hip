// Factored engine: r = E^T p and G = E v evaluated one input position at a time.
//
// The deletion channel deletes each input bit independently (Section 2.2), so the
// embedding-count matrix E[x][y] = emb(y,x) is a product of n sparse stages.
// After the first i positions of x have been processed, the state is indexed by
// (y', s): y' is the output produced so far (|y'| <= i, by rank) and s the
// n - i input bits still to come.
//
// Forward (output law, Section 2.3 step 1):
//   F_0[empty][x] = p(x),
//   F_{i+1}[y''][s'] = F_i[y''][0 s'] + F_i[y''][1 s']        (bit i deleted)
//                     + F_i[y''[:-1]][last(y'') s']            (bit i kept),
//   F_n[y][empty] = sum_x p(x) emb(y,x) = r(y).
// Backward (the transpose, for G(x) = sum_y emb(y,x) v(y)):
//   B_n[y][empty] = v(y),
//   B_i[y'][b s'] = B_{i+1}[y'][s'] + B_{i+1}[y' b][s'],   G(x) = B_0[empty][x].
// With ranks, y' b has rank 2 rank(y') + 1 + b and y''[:-1] rank (rank(y'')-1)/2.
// Stage i has (2^(i+1)-1) 2^(n-i) < 2^(n+1) entries, row-major (row = rank).
// Each stage is a streaming pass with unit-stride reads and writes; the default
// launches take two positions at a time.
//
// Two tails of an iteration are fused into these launches: the last forward
// launch can write v(y) = w_k log r(y) instead of r, and the last backward launch
// can form D(x) = H(x) - G(x) - M with the reduction records of the Blahut
// quantities (Section 2.3) instead of writing G.
#include "ba_internal.h"
#include "ba_part.h"

namespace ba {
namespace {

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

template <typename T, int V>
__device__ __forceinline__ Vec<T, V> zero_vec() {
  Vec<T, V> z;
#pragma unroll
  for (int k = 0; k < V; ++k) z.v[k] = T(0);
  return z;
}

template <typename T>
__device__ __forceinline__ T log_t(T v);
template <>
__device__ __forceinline__ float log_t<float>(float v) { return logf(v); }
template <>
__device__ __forceinline__ double log_t<double>(double v) { return log(v); }

// v(y) = w_k log r(y) for the output of rank y (0 where w_k = 0).
template <typename T>
__device__ __forceinline__ T log_weighted(const Consts& cs, uint32_t y, T r) {
  const T wk = T(cs.w[length_of_rank(y)]);
  return (wk == T(0)) ? T(0) : wk * log_t<T>(r);
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
  uint32_t nlog;  // logical row slots per column tile
  uint32_t top;   // rows above level lb: 2^lb - 1
  uint32_t nct;   // column tiles
  int lb, h;      // level of the subtree roots, subtree height (levels)
  int cw_log2;    // log2 of the column-tile width in chunks
};

constexpr size_t kTileBytes = size_t(1) << 19;

// levels: output levels of the launch (rows 0 .. 2^levels - 2); cols_log2: log2
// of the chunks per row; chunk_bytes: bytes one thread covers in a source row.
Order make_order(int levels, int cols_log2, size_t chunk_bytes) {
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
  return o;
}

uint32_t order_threads(const Order& o) { return o.nct * o.nlog << o.cw_log2; }

__device__ __forceinline__ uint32_t logical_block() {
  const uint32_t G = gridDim.x, bx = blockIdx.x;
  return (G & 7u) ? bx : (bx & 7u) * (G >> 3) + (bx >> 3);
}

// (row, chunk) of logical slot q; false for a padding slot or past the end.
__device__ __forceinline__ bool order_slot_q(const Order& o, uint32_t q, uint32_t& row, uint32_t& chunk) {
  const uint32_t rest = q >> o.cw_log2;
  const uint32_t ct = rest / o.nlog;
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

// This thread's (row, chunk), one slot per thread.
__device__ __forceinline__ bool order_slot(const Order& o, uint32_t& row, uint32_t& chunk) {
  return order_slot_q(o, logical_block() * kBlock + threadIdx.x, row, chunk);
}

// D(x) = H(x) - G(x) - M for V consecutive inputs, accumulated into the record.
template <typename T, int V>
__device__ __forceinline__ void d_epilogue(const Group<T>& g, int b, double M, uint32_t x, const Vec<T, V>& G,
                                           Part& p, double wt = 1.0) {
  const Vec<T, V> h = ld<T, V>(g.hf + (size_t)b * g.xs + x);
  const Vec<T, V> l = ld<T, V>(g.lp + (size_t)b * g.xs + x);
  Vec<T, V> d;
#pragma unroll
  for (int k = 0; k < V; ++k) {
    d.v[k] = h.v[k] - G.v[k] - T(M);
    const double lk = double(l.v[k]);
    part_add<T>(p, lk + double(d.v[k]), double(d.v[k]), exp_in(lk, T()), 0.0, wt, g.eta != 1.0,
                lk + g.eta * double(d.v[k]));
  }
  stv<T, V>(g.D + (size_t)b * g.xs + x, d);
}

// One forward stage; each thread produces V consecutive columns of one row
// (V divides the row width S = 2^(n-i-1)).  LOGV: last stage, write v.
template <typename T, int V, bool LOGV>
__global__ __launch_bounds__(kBlock) void k_fwd_stage(int n, int i, const T* __restrict__ src,
                                                      size_t sstride, T* __restrict__ dst,
                                                      size_t dstride, const State* st, const Consts* cs) {
  const int b = blockIdx.y;
  if (st[b].converged) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh = n - i - 1;                    // log2 of the output width
  const uint32_t S = 1u << sh;
  const uint32_t rows_in = (2u << i) - 1u;
  const uint32_t total = (((4u << i) - 1u) << sh) / V;
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
    const uint32_t idx = q * V;
    const uint32_t row = idx >> sh;
    const uint32_t s = idx & (S - 1u);
    Vec<T, V> acc;
#pragma unroll
    for (int k = 0; k < V; ++k) acc.v[k] = T(0);
    if (row < rows_in) {
      const uint32_t base = row << (sh + 1);
      const Vec<T, V> a = ld<T, V>(src + base + s), c = ld<T, V>(src + base + S + s);
#pragma unroll
      for (int k = 0; k < V; ++k) acc.v[k] = a.v[k] + c.v[k];
    }
    if (row >= 1u) {
      const uint32_t rp = (row - 1u) >> 1, bb = (row - 1u) & 1u;
      const Vec<T, V> a = ld<T, V>(src + (rp << (sh + 1)) + (bb << sh) + s);
#pragma unroll
      for (int k = 0; k < V; ++k) acc.v[k] += a.v[k];
    }
    if constexpr (LOGV) {
#pragma unroll
      for (int k = 0; k < V; ++k) acc.v[k] = log_weighted<T>(cs[b], idx + k, acc.v[k]);
    }
    stv<T, V>(dst + idx, acc);
  }
}


// Four forward stages at once (positions i .. i+3).  One thread per (source row y
// of F_i, column s of the output width S4): it loads F_i of y and of its 4
// ancestors P_1..P_4 (16 column groups u s each; absent rows are zero) and runs
// the single stage
//   F_{k+1}[z][g] = F_k[z][0g] + F_k[z][1g] (if z is a row of F_k) + F_k[parent z][last(z) g]
// in registers on the rows that reach the outputs: the path P_0 = y .. P_{4-k} and,
// when y has length i (a leaf of F_i), its subtree down to depth k.  It writes the
// output row y and, for a leaf, the 30 rows below it (all rows of F_{i+4} of
// length >= i are below exactly one leaf).  LOGV: last stage, write v = w_k log r.
// Register part of the four-position forward step for one (y, column): F0 holds
// F_i of the path P_0 = y .. P_3 (16 groups) and H4 the half of P_4 selected by
// last(P_3); lastb[j] = last bit of P_j.  Returns F_{i+4}[y] and, in F4, the 30
// rows below y (breadth-first: depth d, index m at (1 << d) - 2 + m).
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
  // stage 2: path P_0..P_2 (4 groups), subtree depth 1..2 (breadth-first 0..5)
  T F2p[3][4], F2s[6][4];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int g = 0; g < 4; ++g)
      F2p[j][g] = (F1p[j][g] + F1p[j][4 + g]) + (lastb[j] ? F1p[j + 1][4 + g] : F1p[j + 1][g]);
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int g = 0; g < 4; ++g) F2s[c][g] = (F1s[c][g] + F1s[c][4 + g]) + F1p[0][c * 4 + g];
#pragma unroll
  for (int c = 0; c < 4; ++c)  // depth 2: child c/2 of y, then bit c&1
#pragma unroll
    for (int g = 0; g < 4; ++g) F2s[2 + c][g] = F1s[c >> 1][(c & 1) * 4 + g];
  // stage 3: path P_0..P_1 (2 groups), subtree depth 1..3 (breadth-first 0..13)
  T F3p[2][2], F3s[14][2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int g = 0; g < 2; ++g)
      F3p[j][g] = (F2p[j][g] + F2p[j][2 + g]) + (lastb[j] ? F2p[j + 1][2 + g] : F2p[j + 1][g]);
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int g = 0; g < 2; ++g) F3s[c][g] = (F2s[c][g] + F2s[c][2 + g]) + F2p[0][c * 2 + g];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int g = 0; g < 2; ++g) F3s[2 + c][g] = (F2s[2 + c][g] + F2s[2 + c][2 + g]) + F2s[c >> 1][(c & 1) * 2 + g];
#pragma unroll
  for (int c = 0; c < 8; ++c)
#pragma unroll
    for (int g = 0; g < 2; ++g) F3s[6 + c][g] = F2s[2 + (c >> 1)][(c & 1) * 2 + g];
  // stage 4: y (1 group), subtree depth 1..4
#pragma unroll
  for (int c = 0; c < 2; ++c) F4[c] = (F3s[c][0] + F3s[c][1]) + F3p[0][c];
#pragma unroll
  for (int c = 0; c < 4; ++c) F4[2 + c] = (F3s[2 + c][0] + F3s[2 + c][1]) + F3s[c >> 1][c & 1];
#pragma unroll
  for (int c = 0; c < 8; ++c) F4[6 + c] = (F3s[6 + c][0] + F3s[6 + c][1]) + F3s[2 + (c >> 1)][c & 1];
#pragma unroll
  for (int c = 0; c < 16; ++c) F4[14 + c] = F3s[6 + (c >> 1)][c & 1];
  return (F3p[0][0] + F3p[0][1]) + (lastb[0] ? F3p[1][1] : F3p[1][0]);
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

// Four forward stages at once (positions i .. i+3).  One thread per (source row y
// of F_i, column s of the output width S4): it loads F_i of y and of its 4
// ancestors P_1..P_4 (16 column groups u s each; absent rows are zero) and runs
// the single stage
//   F_{k+1}[z][g] = F_k[z][0g] + F_k[z][1g] (if z is a row of F_k) + F_k[parent z][last(z) g]
// in registers on the rows that reach the outputs: the path P_0 = y .. P_{4-k} and,
// when y has length i (a leaf of F_i), its subtree down to depth k.  It writes the
// output row y and, for a leaf, the 30 rows below it (all rows of F_{i+4} of
// length >= i are below exactly one leaf).  LOGV: last stage, write v = w_k log r.
template <typename T, bool LOGV>
__global__ __launch_bounds__(kBlock) void k_fwd_stage4(int n, int i, const T* __restrict__ src, size_t sstride,
                                                       T* __restrict__ dst, size_t dstride, const State* st,
                                                       const Consts* cs, Order o) {
  const int b = blockIdx.y;
  if (st[b].converged) return;
  uint32_t y, s;
  if (!order_slot(o, y, s)) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh = n - i - 4;                  // log2 of the output width S4
  const int ly = length_of_rank(y);
  uint32_t P[5], lastb[4];
  fwd4_path(y, P, lastb);
  T F0[4][16], H4[8];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int u = 0; u < 16; ++u) F0[j][u] = T(0);
#pragma unroll
  for (int u = 0; u < 8; ++u) H4[u] = T(0);
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (j <= ly) {
      const T* row = src + ((size_t)P[j] << (sh + 4)) + s;
#pragma unroll
      for (int u = 0; u < 16; ++u) F0[j][u] = row[uint32_t(u) << sh];
    }
  if (4 <= ly) {
    const T* row = src + ((size_t)P[4] << (sh + 4)) + (lastb[3] << (sh + 3)) + s;
#pragma unroll
    for (int u = 0; u < 8; ++u) H4[u] = row[uint32_t(u) << sh];
  }
  T F4[30];
  T vy = fwd4_registers<T>(F0, H4, lastb, F4);
  if constexpr (LOGV) vy = log_weighted<T>(cs[b], y, vy);
  dst[((size_t)y << sh) + s] = vy;
  if (ly != i) return;
#pragma unroll
  for (int d = 1; d <= 4; ++d)
#pragma unroll
    for (int m = 0; m < (1 << d); ++m) {
      const uint32_t rk = ((y + 1u) << d) - 1u + uint32_t(m);
      T v = F4[(1 << d) - 2 + m];
      if constexpr (LOGV) v = log_weighted<T>(cs[b], rk, v);
      dst[((size_t)rk << sh) + s] = v;
    }
}

// One backward stage; each thread produces V consecutive columns of one row
// (V divides the source row width S = 2^(n-i-1)).  DP: stage 0, write D and the
// reduction records instead of G.
template <typename T, int V, bool DP>
__global__ __launch_bounds__(kBlock) void k_bwd_stage(int n, int i, const T* __restrict__ src,
                                                      size_t sstride, T* __restrict__ dst,
                                                      size_t dstride, Group<T> g) {
  const int b = blockIdx.y;
  if (g.st[b].converged) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh = n - i - 1;                    // log2 of the source width
  const uint32_t S = 1u << sh;
  const uint32_t total = (((2u << i) - 1u) << (sh + 1)) / V;
  const double M = g.st[b].M;
  Part p = part_empty();
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
    const uint32_t idx = q * V;
    const uint32_t row = idx >> (sh + 1);
    const uint32_t s = idx & ((2u * S) - 1u);
    const uint32_t bb = s >> sh, sp = s & (S - 1u);
    const Vec<T, V> a = ld<T, V>(src + (row << sh) + sp);
    const Vec<T, V> c = ld<T, V>(src + ((2u * row + 1u + bb) << sh) + sp);
    Vec<T, V> o;
#pragma unroll
    for (int k = 0; k < V; ++k) o.v[k] = a.v[k] + c.v[k];
    if constexpr (DP) d_epilogue<T, V>(g, b, M, idx, o, p);
    else stv<T, V>(dst + idx, o);
  }
  if constexpr (DP) {
    p = block_reduce(p);
    store_block_part(g.part + (size_t)b * g.ps, blockIdx.x, p);
  }
}

// Two forward stages at once (positions i and i+1); one thread per (output row c,
// V consecutive columns s'').  Columns of F_i are u s'' with u = 2 x_i + x_{i+1}.
// With r = (c-1)/2 the parent of c, b = last(c), and g the parent of r:
//   F_{i+2}[c] = sum_u F_i[c][u]                                 (both bits deleted)
//              + F_i[r][b0] + F_i[r][b1] + F_i[r][0b] + F_i[r][1b]  (one kept)
//              + F_i[g][last(r) b]                               (both kept),
// terms whose source row is longer than i being absent.
template <typename T, int V>
__global__ __launch_bounds__(kBlock) void k_fwd_stage2(int n, int i, const T* __restrict__ src,
                                                       size_t sstride, T* __restrict__ dst,
                                                       size_t dstride, const State* st, Order o) {
  const int b = blockIdx.y;
  if (st[b].converged) return;
  uint32_t c, chunk;
  if (!order_slot(o, c, chunk)) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh = n - i - 2;                  // log2 of the output width S
  const uint32_t S = 1u << sh;
  const uint32_t rows_in = (2u << i) - 1u;   // rows of F_i
  const uint32_t s = chunk * V;
  const uint32_t r = (c - 1u) >> 1, bb = (c - 1u) & 1u;
  const uint32_t gp = (r - 1u) >> 1, lb = (r - 1u) & 1u;
  const bool has_own = c < rows_in, has_par = c >= 1u && r < rows_in, has_gp = c >= 1u && r >= 1u;
  // all present terms are loaded before any is used (absent ones stay zero), so a
  // thread's loads are in flight together
  Vec<T, V> a0 = zero_vec<T, V>(), a1 = a0, a2 = a0, a3 = a0, e = a0, p01 = a0, p10 = a0, gv = a0;
  if (has_own) {
    const T* pc = src + (c << (sh + 2)) + s;
    a0 = ld<T, V>(pc); a1 = ld<T, V>(pc + S); a2 = ld<T, V>(pc + 2 * S); a3 = ld<T, V>(pc + 3 * S);
  }
  if (has_par) {
    const T* pr = src + (r << (sh + 2)) + s;
    e = ld<T, V>(pr + 3u * bb * S); p01 = ld<T, V>(pr + S); p10 = ld<T, V>(pr + 2 * S);
  }
  if (has_gp) gv = ld<T, V>(src + (gp << (sh + 2)) + ((2u * lb + bb) << sh) + s);
  Vec<T, V> acc;
#pragma unroll
  for (int k = 0; k < V; ++k)
    acc.v[k] = (((a0.v[k] + a1.v[k]) + (a2.v[k] + a3.v[k])) + ((e.v[k] + e.v[k]) + (p01.v[k] + p10.v[k]))) +
               gv.v[k];
  stv<T, V>(dst + (c << sh) + s, acc);
}

// The same for output rows of width 1 (the last two positions): one output row;
// a source row is 4 consecutive values.  LOGV: write v instead of r.
// Present terms are loaded (absent ones stay zero) before any is used, so the
// loads of a thread's rows overlap.
template <typename T>
struct W1Loads {
  Vec<T, 4> own, par;
  T gp;
};
template <typename T>
__device__ __forceinline__ W1Loads<T> fwd_w1_load(uint32_t c, bool ok, uint32_t rows_in,
                                                  const T* __restrict__ src) {
  const uint32_t r = (c - 1u) >> 1, bb = (c - 1u) & 1u;
  const uint32_t gp = (r - 1u) >> 1, lb = (r - 1u) & 1u;
  W1Loads<T> w;
  w.own = zero_vec<T, 4>();
  w.par = w.own;
  w.gp = T(0);
  if (ok && c < rows_in) w.own = ld<T, 4>(src + 4u * c);
  if (ok && c >= 1u && r < rows_in) w.par = ld<T, 4>(src + 4u * r);
  if (ok && c >= 1u && r >= 1u) w.gp = src[4u * gp + 2u * lb + bb];
  return w;
}
template <typename T, bool LOGV>
__device__ __forceinline__ void fwd_w1_finish(uint32_t c, const W1Loads<T>& w, T* __restrict__ dst,
                                              const Consts& cs) {
  const uint32_t bb = (c - 1u) & 1u;
  const T e = bb ? w.par.v[3] : w.par.v[0];
  T acc = (((w.own.v[0] + w.own.v[1]) + (w.own.v[2] + w.own.v[3])) + ((e + e) + (w.par.v[1] + w.par.v[2]))) +
          w.gp;
  if constexpr (LOGV) acc = log_weighted<T>(cs, c, acc);
  dst[c] = acc;
}

// Each thread takes 4 slots, 64 apart, of its wavefront's 256 consecutive slots
// (one output value per slot is too little work per thread).
template <typename T, bool LOGV>
__global__ __launch_bounds__(kBlock) void k_fwd_stage2_w1(int n, const T* __restrict__ src, size_t sstride,
                                                          T* __restrict__ dst, size_t dstride,
                                                          const State* st, const Consts* cs, Order o) {
  const int b = blockIdx.y;
  if (st[b].converged) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const uint32_t rows_in = (1u << (n - 1)) - 1u;   // rows of F_{n-2}
  const uint32_t q0 = logical_block() * (4u * kBlock) + (threadIdx.x & ~63u) * 4u + (threadIdx.x & 63u);
  uint32_t c[4];
  bool ok[4];
  W1Loads<T> w[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    uint32_t chunk;
    ok[m] = order_slot_q(o, q0 + 64u * m, c[m], chunk);
    w[m] = fwd_w1_load<T>(c[m], ok[m], rows_in, src);
  }
#pragma unroll
  for (int m = 0; m < 4; ++m)
    if (ok[m]) fwd_w1_finish<T, LOGV>(c[m], w[m], dst, cs[b]);
}

// Two backward stages at once (positions i and i+1): for a row r of B_i and
// columns (b, c, s''),
//   B_i[r][b c s''] = B_{i+2}[r] + B_{i+2}[r c] + B_{i+2}[r b] + B_{i+2}[r b c]
// (subsets of the two positions that are kept); one thread per (r, V columns s'')
// reads the 7 rows of r's depth-2 subtree once and writes its 4 columns.  DP:
// stage 0 (one row), write D and the reduction records instead of G.
template <typename T, int V, bool DP>
__global__ __launch_bounds__(kBlock) void k_bwd_stage2(int n, int i, const T* __restrict__ src,
                                                       size_t sstride, T* __restrict__ dst,
                                                       size_t dstride, Group<T> g, Order o) {
  const int b = blockIdx.y;
  if (g.st[b].converged) return;
  uint32_t r, chunk;
  const bool valid = order_slot(o, r, chunk);
  if (!DP && !valid) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh = n - i - 2;                  // log2 of the source width S''
  const uint32_t S = 1u << sh;
  const uint32_t s = chunk * V;
  Part p = part_empty();
  if (valid) {
    const Vec<T, V> e = ld<T, V>(src + (r << sh) + s);
    const Vec<T, V> k0 = ld<T, V>(src + ((2u * r + 1u) << sh) + s);
    const Vec<T, V> k1 = ld<T, V>(src + ((2u * r + 2u) << sh) + s);
    const Vec<T, V> g00 = ld<T, V>(src + ((4u * r + 3u) << sh) + s);
    const Vec<T, V> g01 = ld<T, V>(src + ((4u * r + 4u) << sh) + s);
    const Vec<T, V> g10 = ld<T, V>(src + ((4u * r + 5u) << sh) + s);
    const Vec<T, V> g11 = ld<T, V>(src + ((4u * r + 6u) << sh) + s);
    Vec<T, V> o00, o01, o10, o11;
#pragma unroll
    for (int k = 0; k < V; ++k) {
      o00.v[k] = e.v[k] + k0.v[k] + k0.v[k] + g00.v[k];
      o01.v[k] = e.v[k] + k1.v[k] + k0.v[k] + g01.v[k];
      o10.v[k] = e.v[k] + k0.v[k] + k1.v[k] + g10.v[k];
      o11.v[k] = e.v[k] + k1.v[k] + k1.v[k] + g11.v[k];
    }
    if constexpr (DP) {
      const double M = g.st[b].M;
      d_epilogue<T, V>(g, b, M, s, o00, p);
      d_epilogue<T, V>(g, b, M, S + s, o01, p);
      d_epilogue<T, V>(g, b, M, 2 * S + s, o10, p);
      d_epilogue<T, V>(g, b, M, 3 * S + s, o11, p);
    } else {
      T* op = dst + (r << (sh + 2)) + s;
      stv<T, V>(op, o00);
      stv<T, V>(op + S, o01);
      stv<T, V>(op + 2 * S, o10);
      stv<T, V>(op + 3 * S, o11);
    }
  }
  if constexpr (DP) {
    p = block_reduce(p);
    store_block_part(g.part + (size_t)b * g.ps, blockIdx.x, p);
  }
}


// Four backward stages at once (positions i .. i+3): for a row y of B_i and
// columns (u, s), u = 4 bits,
//   B_i[y][u s] = sum over the subsets K of the 4 positions of B_{i+4}[y u_K][s]
// (u_K = the bits of u at the kept positions).  One thread per (y, column s):
// it loads the 31 rows of y's depth-4 subtree (breadth-first index t, children
// 2t+1 and 2t+2, the same as ranks) and applies the 4 single stages
// B_k[z][b g] = B_{k+1}[z][g] + B_{k+1}[z b][g] in registers.  DP: stage 0 (one
// row), write D and the reduction records instead of G.
template <typename T, bool DP>
__global__ __launch_bounds__(kBlock) void k_bwd_stage4(int n, int i, const T* __restrict__ src, size_t sstride,
                                                       T* __restrict__ dst, size_t dstride, Group<T> g, Order o) {
  const int b = blockIdx.y;
  if (g.st[b].converged) return;
  uint32_t y, s;
  const bool valid = order_slot(o, y, s);
  if (!DP && !valid) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh = n - i - 4;                  // log2 of the source width S4
  Part p = part_empty();
  if (valid) {
    T S[31];
#pragma unroll
    for (int d = 0; d <= 4; ++d)
#pragma unroll
      for (int m = 0; m < (1 << d); ++m)
        S[(1 << d) - 1 + m] = src[((((y + 1u) << d) - 1u + uint32_t(m)) << sh) + s];
    T A[15][2];
#pragma unroll
    for (int t = 0; t < 15; ++t) {
      A[t][0] = S[t] + S[2 * t + 1];
      A[t][1] = S[t] + S[2 * t + 2];
    }
    T B[7][4];
#pragma unroll
    for (int t = 0; t < 7; ++t)
#pragma unroll
      for (int bb = 0; bb < 2; ++bb)
#pragma unroll
        for (int q = 0; q < 2; ++q) B[t][bb * 2 + q] = A[t][q] + A[2 * t + 1 + bb][q];
    T C[3][8];
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
      for (int bb = 0; bb < 2; ++bb)
#pragma unroll
        for (int q = 0; q < 4; ++q) C[t][bb * 4 + q] = B[t][q] + B[2 * t + 1 + bb][q];
    T Dv[16];
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int q = 0; q < 8; ++q) Dv[bb * 8 + q] = C[0][q] + C[1 + bb][q];
    const uint32_t S4 = 1u << sh;
    if constexpr (DP) {
      const double M = g.st[b].M;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        Vec<T, 1> gv;
        gv.v[0] = Dv[u];
        d_epilogue<T, 1>(g, b, M, uint32_t(u) * S4 + s, gv, p);
      }
    } else {
      T* op = dst + (y << (sh + 4)) + s;
      if (sh == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          Vec<T, 4> w;
#pragma unroll
          for (int k = 0; k < 4; ++k) w.v[k] = Dv[4 * q + k];
          stv<T, 4>(op + 4 * q, w);
        }
      } else {
#pragma unroll
        for (int u = 0; u < 16; ++u) op[uint32_t(u) * S4] = Dv[u];
      }
    }
  }
  if constexpr (DP) {
    p = block_reduce(p);
    store_block_part(g.part + (size_t)b * g.ps, blockIdx.x, p);
  }
}

// The same for source rows of width 1 (the first backward launch, from v): one
// thread per output row r, which is 4 consecutive values.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bwd_stage2_w1(const T* __restrict__ src, size_t sstride,
                                                          T* __restrict__ dst, size_t dstride,
                                                          const State* st, Order o) {
  const int b = blockIdx.y;
  if (st[b].converged) return;
  uint32_t r, chunk;
  if (!order_slot(o, r, chunk)) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const T e = src[r], k0 = src[2u * r + 1u], k1 = src[2u * r + 2u];
  const T* gg = src + 4u * r + 3u;
  Vec<T, 4> out;
  out.v[0] = e + k0 + k0 + gg[0];
  out.v[1] = e + k1 + k0 + gg[1];
  out.v[2] = e + k0 + k1 + gg[2];
  out.v[3] = e + k1 + k1 + gg[3];
  stv<T, 4>(dst + 4u * r, out);
}


// ---------------------------------------------------------------------------
// Complement-symmetric variant (Theorem 4 of Appendix A: from the uniform law,
// every BA iterate satisfies p(cpl x) = p(x)).  Then every stage is symmetric,
// F_i[cpl y][cpl s] = F_i[y][s] and B_i[cpl y][cpl s] = B_i[y][s], so only the
// columns whose first bit is 0 are computed and stored (row stride halved), and
// the other half is read from the mirrored row and column.  The output law is
// kept for outputs that are empty or start with 0, at the compact index
// cr(0z) = 2^|z| + bits(z), cr(empty) = 0; D for inputs x < 2^(n-1).
// ---------------------------------------------------------------------------

// Rank of the complement of the string of rank R (same length).
__device__ __forceinline__ uint32_t mirror_rank(uint32_t R) {
  return 3u * (1u << length_of_rank(R)) - 3u - R;
}

// Compact index of the canonical member of {y, cpl y}.
__device__ __forceinline__ uint32_t compact_rank(uint32_t R) {
  if (R == 0u) return 0u;
  const int k = length_of_rank(R);
  const uint32_t a = R + 1u - (1u << k), half = 1u << (k - 1);
  return half + (a < half ? a : (2u * half - 1u - a));
}

template <typename T, int V>
__device__ __forceinline__ Vec<T, V> rev(const Vec<T, V>& a) {
  Vec<T, V> r;
#pragma unroll
  for (int k = 0; k < V; ++k) r.v[k] = a.v[V - 1 - k];
  return r;
}

// Two forward stages, canonical half: output columns s'' < S/2 of every row c of
// F_{i+2} (stride S/2) from F_i stored as its columns u s'' with u in {00, 01}
// (stride 2S); F_i[y][1b s''] = F_i[cpl y][0 (1-b) cpl s''].
template <typename T, int V>
__global__ __launch_bounds__(kBlock) void k_fwd_stage2_sym(int n, int i, const T* __restrict__ src,
                                                           size_t sstride, T* __restrict__ dst,
                                                           size_t dstride, const State* st, Order o) {
  const int b = blockIdx.y;
  if (st[b].converged) return;
  uint32_t c, chunk;
  if (!order_slot(o, c, chunk)) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh = n - i - 2;                  // log2 of the full output width S
  const uint32_t S = 1u << sh;
  const uint32_t rows_in = (2u << i) - 1u;
  const uint32_t s = chunk * V, m = S - s - V;  // chunk and its mirror
  const uint32_t r = (c - 1u) >> 1, bb = (c - 1u) & 1u;
  const uint32_t gp = (r - 1u) >> 1, lb = (r - 1u) & 1u;
  const bool has_own = c < rows_in, has_par = c >= 1u && r < rows_in, has_gp = c >= 1u && r >= 1u;
  // row y, u in {0,1} (stored half), column chunk at col
  auto at = [&](uint32_t y, uint32_t u, uint32_t col) { return src + (y << (sh + 1)) + (u << sh) + col; };
  // present terms loaded before use, absent ones zero (as in k_fwd_stage2)
  Vec<T, V> o00 = zero_vec<T, V>(), o01 = o00, o10 = o00, o11 = o00, e = o00, p01 = o00, p10 = o00, gv = o00;
  if (has_own) {
    const uint32_t cm = mirror_rank(c);
    o00 = ld<T, V>(at(c, 0, s)); o01 = ld<T, V>(at(c, 1, s));
    o10 = ld<T, V>(at(cm, 1, m)); o11 = ld<T, V>(at(cm, 0, m));
  }
  if (has_par) {
    // u = bb bb: 00 direct, 11 = cpl(00) of the mirrored row
    e = bb ? ld<T, V>(at(mirror_rank(r), 0, m)) : ld<T, V>(at(r, 0, s));
    p01 = ld<T, V>(at(r, 1, s));
    p10 = ld<T, V>(at(mirror_rank(r), 1, m));
  }
  if (has_gp) gv = lb ? ld<T, V>(at(mirror_rank(gp), 1u - bb, m)) : ld<T, V>(at(gp, bb, s));
  // mirrored chunks are read in reverse column order
  o10 = rev(o10);
  o11 = rev(o11);
  p10 = rev(p10);
  if (has_par && bb) e = rev(e);
  if (has_gp && lb) gv = rev(gv);
  Vec<T, V> acc;
#pragma unroll
  for (int k = 0; k < V; ++k)
    acc.v[k] = (((o00.v[k] + o01.v[k]) + (o10.v[k] + o11.v[k])) + ((e.v[k] + e.v[k]) + (p01.v[k] + p10.v[k]))) +
               gv.v[k];
  stv<T, V>(dst + (c << (sh - 1)) + s, acc);
}

// Last two forward positions, canonical outputs (empty or starting with 0): v at
// the compact index.  F_{n-2} is stored as 2 values per row (u = 00, 01).  Slots
// run over the subtree of the string "0" (local rank rho, compact index rho + 1);
// the slot of rho = 0 also produces the empty output.
template <typename T>
struct W1SymLoads {
  Vec<T, 2> own, ownm, par, parm;
  T gp;
};
template <typename T>
__device__ __forceinline__ W1SymLoads<T> fwd_w1_sym_load(uint32_t c, bool ok, uint32_t rows_in,
                                                         const T* __restrict__ src) {
  const uint32_t r = (c - 1u) >> 1, bb = (c - 1u) & 1u;
  const uint32_t gp = (r - 1u) >> 1, lb = (r - 1u) & 1u;
  W1SymLoads<T> w;
  w.own = zero_vec<T, 2>();
  w.ownm = w.own;
  w.par = w.own;
  w.parm = w.own;
  w.gp = T(0);
  if (ok && c < rows_in) {
    w.own = ld<T, 2>(src + 2u * c);
    w.ownm = ld<T, 2>(src + 2u * mirror_rank(c));
  }
  if (ok && c >= 1u && r < rows_in) {
    w.par = ld<T, 2>(src + 2u * r);
    w.parm = ld<T, 2>(src + 2u * mirror_rank(r));
  }
  if (ok && c >= 1u && r >= 1u) w.gp = lb ? src[2u * mirror_rank(gp) + 1u - bb] : src[2u * gp + bb];
  return w;
}
template <typename T>
__device__ __forceinline__ T fwd_w1_sym_value(uint32_t c, const W1SymLoads<T>& w) {
  const uint32_t bb = (c - 1u) & 1u;
  const T e = bb ? w.parm.v[0] : w.par.v[0];
  return (((w.own.v[0] + w.own.v[1]) + (w.ownm.v[0] + w.ownm.v[1])) + ((e + e) + (w.par.v[1] + w.parm.v[1]))) +
         w.gp;
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fwd_stage2_w1_sym(int n, const T* __restrict__ src, size_t sstride,
                                                              T* __restrict__ dst, size_t dstride,
                                                              const State* st, const Consts* cs, Order o) {
  const int b = blockIdx.y;
  if (st[b].converged) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const uint32_t rows_in = (1u << (n - 1)) - 1u;   // rows of F_{n-2}
  const uint32_t q0 = logical_block() * (4u * kBlock) + (threadIdx.x & ~63u) * 4u + (threadIdx.x & 63u);
  uint32_t rho[4], c[4];
  bool ok[4];
  W1SymLoads<T> w[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint32_t chunk;
    ok[j] = order_slot_q(o, q0 + 64u * j, rho[j], chunk);
    if (!ok[j]) rho[j] = 0u;
    const int k = length_of_rank(rho[j]);
    c[j] = rho[j] + (1u << k);  // global rank of the local rank rho in the subtree of "0"
    w[j] = fwd_w1_sym_load<T>(c[j], ok[j], rows_in, src);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (ok[j]) dst[rho[j] + 1u] = log_weighted<T>(cs[b], c[j], fwd_w1_sym_value<T>(c[j], w[j]));
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (ok[j] && rho[j] == 0u) {
      const W1SymLoads<T> we = fwd_w1_sym_load<T>(0u, true, rows_in, src);
      dst[0] = log_weighted<T>(cs[b], 0u, fwd_w1_sym_value<T>(0u, we));
    }
}

// v of the output of rank R from the compact array.
template <typename T>
__device__ __forceinline__ T v_sym(const T* __restrict__ v, uint32_t R) { return v[compact_rank(R)]; }

// First backward launch, canonical half: B_{n-2}[r][0 c] for every row r (two
// values per row, stride 2) from the compact v.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bwd_stage2_w1_sym(const T* __restrict__ src, size_t sstride,
                                                              T* __restrict__ dst, size_t dstride,
                                                              const State* st, Order o) {
  const int b = blockIdx.y;
  if (st[b].converged) return;
  uint32_t r, chunk;
  if (!order_slot(o, r, chunk)) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const T e = v_sym(src, r), k0 = v_sym(src, 2u * r + 1u), k1 = v_sym(src, 2u * r + 2u);
  const T g00 = v_sym(src, 4u * r + 3u), g01 = v_sym(src, 4u * r + 4u);
  Vec<T, 2> out;
  out.v[0] = e + k0 + k0 + g00;
  out.v[1] = e + k1 + k0 + g01;
  stv<T, 2>(dst + 2u * r, out);
}

// Two backward stages, canonical half: B_i[r][0 c s''] for every row r and every
// s'' (stride 2S) from B_{i+2} stored as its columns s'' < S/2 (stride S/2);
// a chunk in the upper half reads the mirrored rows cpl(r ...) at the mirrored
// chunk.  DP: stage 0, D for x < 2^(n-1), each value standing for x and cpl x.
template <typename T, int V, bool DP>
__global__ __launch_bounds__(kBlock) void k_bwd_stage2_sym(int n, int i, const T* __restrict__ src,
                                                           size_t sstride, T* __restrict__ dst,
                                                           size_t dstride, Group<T> g, Order o) {
  const int b = blockIdx.y;
  if (g.st[b].converged) return;
  uint32_t r, chunk;
  const bool valid = order_slot(o, r, chunk);
  if (!DP && !valid) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh = n - i - 2;                  // log2 of the full source width S
  const uint32_t S = 1u << sh;
  const uint32_t s = chunk * V;
  Part p = part_empty();
  if (valid) {
    const bool up = s >= S / 2u;
    const uint32_t col = up ? S - s - V : s;
    const uint32_t rr = up ? mirror_rank(r) : r;
    // children and grandchildren of r, or of cpl r with the bits flipped
    const uint32_t c0 = up ? 2u * rr + 2u : 2u * r + 1u, c1 = up ? 2u * rr + 1u : 2u * r + 2u;
    const uint32_t q00 = up ? 4u * rr + 6u : 4u * r + 3u, q01 = up ? 4u * rr + 5u : 4u * r + 4u;
    const int hs = sh - 1;                   // log2 of the stored width S/2
    Vec<T, V> e = ld<T, V>(src + (rr << hs) + col);
    Vec<T, V> k0 = ld<T, V>(src + (c0 << hs) + col), k1 = ld<T, V>(src + (c1 << hs) + col);
    Vec<T, V> g00 = ld<T, V>(src + (q00 << hs) + col), g01 = ld<T, V>(src + (q01 << hs) + col);
    if (up) { e = rev(e); k0 = rev(k0); k1 = rev(k1); g00 = rev(g00); g01 = rev(g01); }
    Vec<T, V> o00, o01;
#pragma unroll
    for (int k = 0; k < V; ++k) {
      o00.v[k] = e.v[k] + k0.v[k] + k0.v[k] + g00.v[k];
      o01.v[k] = e.v[k] + k1.v[k] + k0.v[k] + g01.v[k];
    }
    if constexpr (DP) {
      const double M = g.st[b].M;
      d_epilogue<T, V>(g, b, M, s, o00, p, 2.0);
      d_epilogue<T, V>(g, b, M, S + s, o01, p, 2.0);
    } else {
      T* op = dst + (r << (sh + 1)) + s;
      stv<T, V>(op, o00);
      stv<T, V>(op + S, o01);
    }
  }
  if constexpr (DP) {
    p = block_reduce(p);
    store_block_part(g.part + (size_t)b * g.ps, blockIdx.x, p);
  }
}


// Four forward stages, canonical half: as k_fwd_stage4 for the output columns
// s < S4/2 (stride S4/2), with F_i stored as its groups u < 8 (first bit 0, stride
// 8 S4); group u >= 8 of row z is group 15 - u of cpl z at column S4 - 1 - s.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fwd_stage4_sym(int n, int i, const T* __restrict__ src,
                                                           size_t sstride, T* __restrict__ dst, size_t dstride,
                                                           const State* st, Order o) {
  const int b = blockIdx.y;
  if (st[b].converged) return;
  uint32_t y, s;
  if (!order_slot(o, y, s)) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh = n - i - 4;                  // log2 of the full output width S4 (>= 1)
  const uint32_t S4 = 1u << sh, sm = S4 - 1u - s;
  const int ly = length_of_rank(y);
  uint32_t P[5], lastb[4];
  fwd4_path(y, P, lastb);
  T F0[4][16], H4[8];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int u = 0; u < 16; ++u) F0[j][u] = T(0);
#pragma unroll
  for (int u = 0; u < 8; ++u) H4[u] = T(0);
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (j <= ly) {
      const T* row = src + ((size_t)P[j] << (sh + 3));
      const T* rowm = src + ((size_t)mirror_rank(P[j]) << (sh + 3));
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        F0[j][u] = row[(uint32_t(u) << sh) + s];
        F0[j][8 + u] = rowm[(uint32_t(7 - u) << sh) + sm];
      }
    }
  if (4 <= ly) {
    if (lastb[3]) {
      const T* rowm = src + ((size_t)mirror_rank(P[4]) << (sh + 3));
#pragma unroll
      for (int u = 0; u < 8; ++u) H4[u] = rowm[(uint32_t(7 - u) << sh) + sm];
    } else {
      const T* row = src + ((size_t)P[4] << (sh + 3));
#pragma unroll
      for (int u = 0; u < 8; ++u) H4[u] = row[(uint32_t(u) << sh) + s];
    }
  }
  T F4[30];
  const T vy = fwd4_registers<T>(F0, H4, lastb, F4);
  const int ho = sh - 1;                     // log2 of the stored output width
  dst[((size_t)y << ho) + s] = vy;
  if (ly != i) return;
#pragma unroll
  for (int d = 1; d <= 4; ++d)
#pragma unroll
    for (int m = 0; m < (1 << d); ++m) {
      const uint32_t rk = ((y + 1u) << d) - 1u + uint32_t(m);
      dst[((size_t)rk << ho) + s] = F4[(1 << d) - 2 + m];
    }
}

// Four backward stages, canonical half: B_i[y][u s] for u < 8 (stride 8 S4) and
// every s, from B_{i+4} stored as its columns s < S4/2 (stride S4/2), or, VC, from
// the compact v (i + 4 = n).  A column in the upper half reads the subtree of
// cpl y with complemented paths at the mirrored column.  DP: stage 0, D for
// x < 2^(n-1) with weight 2.
template <typename T, bool DP, bool VC>
__global__ __launch_bounds__(kBlock) void k_bwd_stage4_sym(int n, int i, const T* __restrict__ src,
                                                           size_t sstride, T* __restrict__ dst, size_t dstride,
                                                           Group<T> g, Order o) {
  const int b = blockIdx.y;
  if (g.st[b].converged) return;
  uint32_t y, s;
  const bool valid = order_slot(o, y, s);
  if (!DP && !valid) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh = n - i - 4;                  // log2 of the full source width S4
  const uint32_t S4 = 1u << sh;
  Part p = part_empty();
  if (valid) {
    T S[31];
    if constexpr (VC) {
#pragma unroll
      for (int d = 0; d <= 4; ++d)
#pragma unroll
        for (int m = 0; m < (1 << d); ++m)
          S[(1 << d) - 1 + m] = v_sym(src, ((y + 1u) << d) - 1u + uint32_t(m));
    } else {
      const bool up = s >= S4 / 2u;
      const uint32_t yy = up ? mirror_rank(y) : y, col = up ? S4 - 1u - s : s;
      const int hs = sh - 1;                 // log2 of the stored width
#pragma unroll
      for (int d = 0; d <= 4; ++d)
#pragma unroll
        for (int m = 0; m < (1 << d); ++m) {
          const uint32_t mm = up ? (1u << d) - 1u - uint32_t(m) : uint32_t(m);
          S[(1 << d) - 1 + m] = src[((((yy + 1u) << d) - 1u + mm) << hs) + col];
        }
    }
    T A[15][2];
#pragma unroll
    for (int t = 0; t < 15; ++t) {
      A[t][0] = S[t] + S[2 * t + 1];
      A[t][1] = S[t] + S[2 * t + 2];
    }
    T B[7][4];
#pragma unroll
    for (int t = 0; t < 7; ++t)
#pragma unroll
      for (int bb = 0; bb < 2; ++bb)
#pragma unroll
        for (int q = 0; q < 2; ++q) B[t][bb * 2 + q] = A[t][q] + A[2 * t + 1 + bb][q];
    T C[3][8];
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
      for (int bb = 0; bb < 2; ++bb)
#pragma unroll
        for (int q = 0; q < 4; ++q) C[t][bb * 4 + q] = B[t][q] + B[2 * t + 1 + bb][q];
    T Dv[8];  // first bit 0 only
#pragma unroll
    for (int q = 0; q < 8; ++q) Dv[q] = C[0][q] + C[1][q];
    if constexpr (DP) {
      const double M = g.st[b].M;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        Vec<T, 1> gv;
        gv.v[0] = Dv[u];
        d_epilogue<T, 1>(g, b, M, uint32_t(u) * S4 + s, gv, p, 2.0);
      }
    } else {
      T* op = dst + (y << (sh + 3)) + s;
#pragma unroll
      for (int u = 0; u < 8; ++u) op[uint32_t(u) * S4] = Dv[u];
    }
  }
  if constexpr (DP) {
    p = block_reduce(p);
    store_block_part(g.part + (size_t)b * g.ps, blockIdx.x, p);
  }
}

inline uint32_t grid_for(uint32_t total) {
  uint32_t g = (total + kBlock - 1) / kBlock;
  return g > 8192u ? 8192u : (g == 0 ? 1u : g);
}

// Blocks for an ordered launch, a multiple of 8 so that the XCD placement of
// logical_block applies (the extra blocks find no slot).
inline uint32_t blocks_for(uint32_t threads) {
  const uint32_t g = threads == 0 ? 1u : (threads + kBlock - 1) / kBlock;
  return (g + 7u) & ~7u;
}

inline int ilog2(uint32_t v) { return 31 - __builtin_clz(v); }

}  // namespace

template <typename T>
hipError_t launch_forward(const Group<T>& g, hipStream_t s, int* launches, int fuse, int logv) {
  const int n = g.n;
  constexpr int V = 16 / sizeof(T);
  const T* src = g.p;
  size_t ss = g.xs;
  int k = 0;
  for (int i = 0; i < n; k++) {
    // four positions per launch except the last four or fewer, whose outputs (one
    // value per row) are written by the width-1 two-position kernel
    if (fuse == 2 && i + 4 < n) {
      const bool last = (i + 4 == n);
      const bool lv = last && logv;
      T* dst = last ? (lv ? g.v : g.r) : ((k & 1) ? g.f1 : g.f0);
      const size_t ds = last ? g.ys : g.fs;
      const uint32_t S4 = 1u << (n - i - 4);
      const Order o = make_order(i + 1, ilog2(S4), sizeof(T));
      const dim3 grid(blocks_for(order_threads(o)), g.nb);
      if (lv)
        hipLaunchKernelGGL((k_fwd_stage4<T, true>), grid, dim3(kBlock), 0, s, n, i, src, ss, dst, ds, g.st, g.cs, o);
      else
        hipLaunchKernelGGL((k_fwd_stage4<T, false>), grid, dim3(kBlock), 0, s, n, i, src, ss, dst, ds, g.st, g.cs,
                           o);
      if (launches) ++*launches;
      src = dst;
      ss = ds;
      i += 4;
      continue;
    }
    const int step = (fuse && i + 2 <= n) ? 2 : 1;
    const bool last = (i + step == n);
    const bool lv = last && logv;
    T* dst;
    size_t ds;
    if (last) { dst = lv ? g.v : g.r; ds = g.ys; }
    else { dst = (k & 1) ? g.f1 : g.f0; ds = g.fs; }
    if (step == 2) {
      const uint32_t S = 1u << (n - i - 2);  // output row width
      if (S == 1u) {
        const Order o = make_order(n + 1, 0, 4 * sizeof(T));
        const dim3 grid(blocks_for((order_threads(o) + 3u) / 4u), g.nb);
        if (lv)
          hipLaunchKernelGGL((k_fwd_stage2_w1<T, true>), grid, dim3(kBlock), 0, s, n, src, ss, dst, ds, g.st,
                             g.cs, o);
        else
          hipLaunchKernelGGL((k_fwd_stage2_w1<T, false>), grid, dim3(kBlock), 0, s, n, src, ss, dst, ds, g.st,
                             g.cs, o);
      } else if (S >= uint32_t(V)) {
        const Order o = make_order(i + 3, ilog2(S / V), V * sizeof(T));
        hipLaunchKernelGGL((k_fwd_stage2<T, V>), dim3(blocks_for(order_threads(o)), g.nb), dim3(kBlock), 0, s,
                           n, i, src, ss, dst, ds, g.st, o);
      } else {  // S = 2 < V (single precision, odd n)
        const Order o = make_order(i + 3, 0, 2 * sizeof(T));
        hipLaunchKernelGGL((k_fwd_stage2<T, 2>), dim3(blocks_for(order_threads(o)), g.nb), dim3(kBlock), 0, s,
                           n, i, src, ss, dst, ds, g.st, o);
      }
    } else {
      const uint32_t w = 1u << (n - i - 1);  // output row width
      const uint32_t total = ((4u << i) - 1u) * w;
      if (w >= uint32_t(V))
        hipLaunchKernelGGL((k_fwd_stage<T, V, false>), dim3(grid_for(total / V), g.nb), dim3(kBlock), 0, s, n,
                           i, src, ss, dst, ds, g.st, g.cs);
      else if (lv)
        hipLaunchKernelGGL((k_fwd_stage<T, 1, true>), dim3(grid_for(total), g.nb), dim3(kBlock), 0, s, n, i,
                           src, ss, dst, ds, g.st, g.cs);
      else
        hipLaunchKernelGGL((k_fwd_stage<T, 1, false>), dim3(grid_for(total), g.nb), dim3(kBlock), 0, s, n, i,
                           src, ss, dst, ds, g.st, g.cs);
    }
    if (launches) ++*launches;
    src = dst;
    ss = ds;
    i += step;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_backward(const Group<T>& g, hipStream_t s, int* launches, int fuse, int dpart,
                           int* dpart_blocks) {
  const int n = g.n;
  constexpr int V = 16 / sizeof(T);
  const T* src = g.v;
  size_t ss = g.ys;
  int k = 0;
  if (dpart_blocks) *dpart_blocks = 0;
  // fuse = 2: four positions per launch, the n mod 4 leftover positions first
  const int lead = (fuse == 2 && n >= 4) ? n % 4 : -1;
  for (int top = n; top > 0; k++) {           // B_top -> B_{top-step}
    if (lead >= 0 && n - top >= lead) {
      const int i = top - 4;
      const bool last = (i == 0);
      T* dst = last ? g.g : ((k & 1) ? g.f1 : g.f0);
      const size_t ds = last ? g.xs : g.fs;
      const uint32_t S4 = 1u << (n - i - 4);
      const Order o = make_order(i + 1, ilog2(S4), sizeof(T));
      const uint32_t nbk = blocks_for(order_threads(o));
      const bool dp = last && dpart && nbk <= uint32_t(kMaxRedBlocks);
      if (dp) {
        hipLaunchKernelGGL((k_bwd_stage4<T, true>), dim3(nbk, g.nb), dim3(kBlock), 0, s, n, i, src, ss, dst, ds, g,
                           o);
        if (dpart_blocks) *dpart_blocks = int(nbk);
      } else {
        hipLaunchKernelGGL((k_bwd_stage4<T, false>), dim3(nbk, g.nb), dim3(kBlock), 0, s, n, i, src, ss, dst, ds,
                           g, o);
      }
      if (launches) ++*launches;
      src = dst;
      ss = ds;
      top = i;
      continue;
    }
    const int step = (fuse && top >= 2 && !(lead >= 0 && n - top + 2 > lead)) ? 2 : 1;
    const int i = top - step;
    const bool last = (i == 0);
    T* dst;
    size_t ds;
    if (last) { dst = g.g; ds = g.xs; }
    else { dst = (k & 1) ? g.f1 : g.f0; ds = g.fs; }
    if (step == 2) {
      const uint32_t S = 1u << (n - i - 2);  // source row width
      if (S == 1u) {
        const Order o = make_order(i + 1, 0, 4 * sizeof(T));
        hipLaunchKernelGGL((k_bwd_stage2_w1<T>), dim3(blocks_for(order_threads(o)), g.nb), dim3(kBlock), 0, s,
                           src, ss, dst, ds, g.st, o);
      } else {
        // the fused D launch (one row, FP64 record arithmetic per value) runs one
        // column per thread for more wavefronts, if its records fit
        const Order o1 = make_order(i + 1, ilog2(S), sizeof(T));
        const uint32_t nb1 = blocks_for(order_threads(o1));
        const bool dp = last && dpart && nb1 <= uint32_t(kMaxRedBlocks);
        if (dp) {
          hipLaunchKernelGGL((k_bwd_stage2<T, 1, true>), dim3(nb1, g.nb), dim3(kBlock), 0, s, n, i, src, ss, dst,
                             ds, g, o1);
          if (dpart_blocks) *dpart_blocks = int(nb1);
        } else {
          const int Vx = S >= uint32_t(V) ? V : 2;
          const Order o = make_order(i + 1, ilog2(S / Vx), Vx * sizeof(T));
          const dim3 grid(blocks_for(order_threads(o)), g.nb);
          if (Vx == V)
            hipLaunchKernelGGL((k_bwd_stage2<T, V, false>), grid, dim3(kBlock), 0, s, n, i, src, ss, dst, ds, g, o);
          else
            hipLaunchKernelGGL((k_bwd_stage2<T, 2, false>), grid, dim3(kBlock), 0, s, n, i, src, ss, dst, ds, g, o);
        }
      }
    } else {
      const uint32_t w = 1u << (n - i - 1);  // source row width
      const uint32_t total = ((2u << i) - 1u) << (n - i);
      if (w >= uint32_t(V)) {
        const bool dp = last && dpart;
        uint32_t grid = grid_for(total / V);
        if (dp) {
          if (grid > uint32_t(kMaxRedBlocks)) grid = kMaxRedBlocks;
          hipLaunchKernelGGL((k_bwd_stage<T, V, true>), dim3(grid, g.nb), dim3(kBlock), 0, s, n, i, src, ss, dst,
                             ds, g);
          if (dpart_blocks) *dpart_blocks = int(grid);
        } else {
          hipLaunchKernelGGL((k_bwd_stage<T, V, false>), dim3(grid, g.nb), dim3(kBlock), 0, s, n, i, src, ss, dst,
                             ds, g);
        }
      } else {
        hipLaunchKernelGGL((k_bwd_stage<T, 1, false>), dim3(grid_for(total), g.nb), dim3(kBlock), 0, s, n, i, src,
                           ss, dst, ds, g);
      }
    }
    if (launches) ++*launches;
    src = dst;
    ss = ds;
    top = i;
  }
  return hipGetLastError();
}


bool symmetric_supported(int n, int fuse) { return fuse && n >= 4 && (n % 2) == 0; }

template <typename T>
hipError_t launch_forward_sym(const Group<T>& g, hipStream_t s, int* launches, int fuse) {
  const int n = g.n;
  constexpr int V = 16 / sizeof(T);
  const T* src = g.p;
  size_t ss = g.xs;
  int k = 0;
  int i0 = 0;
  for (; fuse == 2 && i0 + 4 < n; i0 += 4, k++) {
    T* dst = (k & 1) ? g.f1 : g.f0;
    const uint32_t S4 = 1u << (n - i0 - 4);
    const Order o = make_order(i0 + 1, ilog2(S4 / 2u), sizeof(T));
    hipLaunchKernelGGL((k_fwd_stage4_sym<T>), dim3(blocks_for(order_threads(o)), g.nb), dim3(kBlock), 0, s, n, i0,
                       src, ss, dst, g.fs, g.st, o);
    if (launches) ++*launches;
    src = dst;
    ss = g.fs;
  }
  for (int i = i0; i < n; i += 2, k++) {
    const bool last = (i + 2 == n);
    T* dst = last ? g.v : ((k & 1) ? g.f1 : g.f0);
    const size_t ds = last ? g.ys : g.fs;
    const uint32_t S = 1u << (n - i - 2);
    if (S == 1u) {
      const Order o = make_order(n, 0, 4 * sizeof(T));
      hipLaunchKernelGGL((k_fwd_stage2_w1_sym<T>), dim3(blocks_for((order_threads(o) + 3u) / 4u), g.nb),
                         dim3(kBlock), 0, s, n, src, ss, dst, ds, g.st, g.cs, o);
    } else {
      const uint32_t half = S / 2u;
      if (half >= uint32_t(V)) {
        const Order o = make_order(i + 3, ilog2(half / V), V * sizeof(T));
        hipLaunchKernelGGL((k_fwd_stage2_sym<T, V>), dim3(blocks_for(order_threads(o)), g.nb), dim3(kBlock), 0,
                           s, n, i, src, ss, dst, ds, g.st, o);
      } else {  // S = 4: two columns per row
        const Order o = make_order(i + 3, 0, 2 * sizeof(T));
        hipLaunchKernelGGL((k_fwd_stage2_sym<T, 2>), dim3(blocks_for(order_threads(o)), g.nb), dim3(kBlock), 0,
                           s, n, i, src, ss, dst, ds, g.st, o);
      }
    }
    if (launches) ++*launches;
    src = dst;
    ss = ds;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_backward_sym(const Group<T>& g, hipStream_t s, int* launches, int* dpart_blocks, int fuse) {
  const int n = g.n;
  constexpr int V = 16 / sizeof(T);
  const T* src = g.v;
  size_t ss = g.ys;
  int k = 0;
  if (dpart_blocks) *dpart_blocks = 0;
  const int lead = (fuse == 2) ? n % 4 : -1;  // even n: 0 or 2
  for (int top = n; top > 0; k++) {
    if (lead >= 0 && n - top >= lead) {
      const int i = top - 4;
      const bool last = (i == 0), vc = (top == n);
      T* dst = last ? g.g : ((k & 1) ? g.f1 : g.f0);
      const size_t ds = last ? g.xs : g.fs;
      const uint32_t S4 = 1u << (n - i - 4);
      const Order o = make_order(i + 1, ilog2(S4), sizeof(T));
      const uint32_t nbk = blocks_for(order_threads(o));
      const dim3 grid(nbk, g.nb);
      if (last) {
        if (nbk > uint32_t(kMaxRedBlocks)) return hipErrorInvalidValue;
        if (vc)
          hipLaunchKernelGGL((k_bwd_stage4_sym<T, true, true>), grid, dim3(kBlock), 0, s, n, i, src, ss, dst, ds, g, o);
        else
          hipLaunchKernelGGL((k_bwd_stage4_sym<T, true, false>), grid, dim3(kBlock), 0, s, n, i, src, ss, dst, ds, g,
                             o);
        if (dpart_blocks) *dpart_blocks = int(nbk);
      } else if (vc) {
        hipLaunchKernelGGL((k_bwd_stage4_sym<T, false, true>), grid, dim3(kBlock), 0, s, n, i, src, ss, dst, ds, g, o);
      } else {
        hipLaunchKernelGGL((k_bwd_stage4_sym<T, false, false>), grid, dim3(kBlock), 0, s, n, i, src, ss, dst, ds, g,
                           o);
      }
      if (launches) ++*launches;
      src = dst;
      ss = ds;
      top = i;
      continue;
    }
    const int i = top - 2;
    const bool last = (i == 0);
    T* dst = last ? g.g : ((k & 1) ? g.f1 : g.f0);
    const size_t ds = last ? g.xs : g.fs;
    const uint32_t S = 1u << (n - i - 2);  // full source row width
    if (S == 1u) {
      const Order o = make_order(i + 1, 0, 2 * sizeof(T));
      hipLaunchKernelGGL((k_bwd_stage2_w1_sym<T>), dim3(blocks_for(order_threads(o)), g.nb), dim3(kBlock), 0, s,
                         src, ss, dst, ds, g.st, o);
    } else if (last) {
      // one row; one column per thread (n <= 20 keeps the records within kMaxRedBlocks)
      const Order o = make_order(1, ilog2(S), sizeof(T));
      const uint32_t nb1 = blocks_for(order_threads(o));
      if (nb1 > uint32_t(kMaxRedBlocks)) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_bwd_stage2_sym<T, 1, true>), dim3(nb1, g.nb), dim3(kBlock), 0, s, n, i, src, ss, dst,
                         ds, g, o);
      if (dpart_blocks) *dpart_blocks = int(nb1);
    } else {
      const uint32_t Vx = (S / 2u >= uint32_t(V)) ? uint32_t(V) : 2u;
      const Order o = make_order(i + 1, ilog2(S / Vx), Vx * sizeof(T));
      const dim3 grid(blocks_for(order_threads(o)), g.nb);
      if (Vx == uint32_t(V))
        hipLaunchKernelGGL((k_bwd_stage2_sym<T, V, false>), grid, dim3(kBlock), 0, s, n, i, src, ss, dst, ds, g, o);
      else
        hipLaunchKernelGGL((k_bwd_stage2_sym<T, 2, false>), grid, dim3(kBlock), 0, s, n, i, src, ss, dst, ds, g, o);
    }
    if (launches) ++*launches;
    src = dst;
    ss = ds;
    top = i;
  }
  return hipGetLastError();
}

int factored_launches(int n, int fuse) { return fuse ? (n + 1) / 2 : n; }

int backward_launches(int n, int fuse) {
  if (fuse == 2 && n >= 4) return n / 4 + (n % 4 + 1) / 2;
  return factored_launches(n, fuse);
}

int forward_launches(int n, int fuse) {
  if (fuse == 2 && n > 4) {
    const int four = (n - 1) / 4;  // launches of four positions; the rest two at a time
    return four + (n - 4 * four + 1) / 2;
  }
  return factored_launches(n, fuse);
}

template hipError_t launch_forward<float>(const Group<float>&, hipStream_t, int*, int, int);
template hipError_t launch_forward<double>(const Group<double>&, hipStream_t, int*, int, int);
template hipError_t launch_backward<float>(const Group<float>&, hipStream_t, int*, int, int, int*);
template hipError_t launch_backward<double>(const Group<double>&, hipStream_t, int*, int, int, int*);
template hipError_t launch_forward_sym<float>(const Group<float>&, hipStream_t, int*, int);
template hipError_t launch_forward_sym<double>(const Group<double>&, hipStream_t, int*, int);
template hipError_t launch_backward_sym<float>(const Group<float>&, hipStream_t, int*, int*, int);
template hipError_t launch_backward_sym<double>(const Group<double>&, hipStream_t, int*, int*, int);

}  // namespace ba
