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
  for (int top = n; top > 0; k++) {           // B_top -> B_{top-step}
    const int step = (fuse && top >= 2) ? 2 : 1;
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
hipError_t launch_forward_sym(const Group<T>& g, hipStream_t s, int* launches) {
  const int n = g.n;
  constexpr int V = 16 / sizeof(T);
  const T* src = g.p;
  size_t ss = g.xs;
  int k = 0;
  for (int i = 0; i < n; i += 2, k++) {
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
hipError_t launch_backward_sym(const Group<T>& g, hipStream_t s, int* launches, int* dpart_blocks) {
  const int n = g.n;
  constexpr int V = 16 / sizeof(T);
  const T* src = g.v;
  size_t ss = g.ys;
  int k = 0;
  if (dpart_blocks) *dpart_blocks = 0;
  for (int top = n; top > 0; top -= 2, k++) {
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
  }
  return hipGetLastError();
}

int factored_launches(int n, int fuse) { return fuse ? (n + 1) / 2 : n; }

template hipError_t launch_forward<float>(const Group<float>&, hipStream_t, int*, int, int);
template hipError_t launch_forward<double>(const Group<double>&, hipStream_t, int*, int, int);
template hipError_t launch_backward<float>(const Group<float>&, hipStream_t, int*, int, int, int*);
template hipError_t launch_backward<double>(const Group<double>&, hipStream_t, int*, int, int, int*);
template hipError_t launch_forward_sym<float>(const Group<float>&, hipStream_t, int*);
template hipError_t launch_forward_sym<double>(const Group<double>&, hipStream_t, int*);
template hipError_t launch_backward_sym<float>(const Group<float>&, hipStream_t, int*, int*);
template hipError_t launch_backward_sym<double>(const Group<double>&, hipStream_t, int*, int*);

}  // namespace ba
