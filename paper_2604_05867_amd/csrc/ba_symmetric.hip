// Complement-symmetric variant of the factored engine (Appendix A, Theorem 4:
// from the uniform law every BA iterate satisfies p(cpl x) = p(x)).
#include "ba_factored_common.h"

namespace ba {
namespace {

using namespace fac;

// ---------------------------------------------------------------------------
// Complement-symmetric variant (Theorem 4 of Appendix A: from the uniform law,
// every BA iterate satisfies p(cpl x) = p(x)).  Then every stage is symmetric,
// F_i[cpl y][cpl s] = F_i[y][s] and B_i[cpl y][cpl s] = B_i[y][s], so only the
// columns whose first bit is 0 are computed and stored (row stride halved), and
// the other half is read from the mirrored row and column.  The output law is
// kept for outputs that are empty or start with 0, at the compact index
// cr(0z) = 2^|z| + bits(z), cr(empty) = 0; D for inputs x < 2^(n-1).
// ---------------------------------------------------------------------------


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
  auto chunk_at = [&](uint32_t y, uint32_t u, uint32_t col) { return src + (y << (sh + 1)) + (u << sh) + col; };
  // present terms loaded before use, absent ones zero (as in k_fwd_stage2)
  Vec<T, V> o00 = zero_vec<T, V>(), o01 = o00, o10 = o00, o11 = o00, e = o00, p01 = o00, p10 = o00, gv = o00;
  if (has_own) {
    const uint32_t cm = mirror_rank(c);
    o00 = ld<T, V>(chunk_at(c, 0, s)); o01 = ld<T, V>(chunk_at(c, 1, s));
    o10 = ld<T, V>(chunk_at(cm, 1, m)); o11 = ld<T, V>(chunk_at(cm, 0, m));
  }
  if (has_par) {
    // u = bb bb: 00 direct, 11 = cpl(00) of the mirrored row
    e = bb ? ld<T, V>(chunk_at(mirror_rank(r), 0, m)) : ld<T, V>(chunk_at(r, 0, s));
    p01 = ld<T, V>(chunk_at(r, 1, s));
    p10 = ld<T, V>(chunk_at(mirror_rank(r), 1, m));
  }
  if (has_gp) gv = lb ? ld<T, V>(chunk_at(mirror_rank(gp), 1u - bb, m)) : ld<T, V>(chunk_at(gp, bb, s));
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
      const uint32_t xs[2] = {s, S + s};
      const Vec<T, V> gs[2] = {o00, o01};
      d_records<T, V, 2>(g, b, M, xs, gs, p, 2.0);
    } else {
      T* op = dst + (r << (sh + 1)) + s;
      stv<T, V>(op, o00);
      stv<T, V>(op + S, o01);
    }
  }
  if constexpr (DP) {
    store_block_part(g.part + (size_t)b * g.ps, blockIdx.x, p);
  }
}


// Four forward stages, canonical half: as k_fwd_stage4 for the output columns
// s < S4/2 (stride S4/2), with F_i stored as its groups u < 8 (first bit 0, stride
// 8 S4); group u >= 8 of row z is group 15 - u of cpl z at column S4 - 1 - s.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fwd_stage4_sym(int n, int i, const T* __restrict__ src,
                                                           size_t sstride, T* __restrict__ dst, size_t dstride,
                                                           const State* st, Order o, int frz) {
  const int b = blockIdx.y;
  if (frz && st[b].converged) return;
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

// The four backward single stages on the 31 values S of a depth-4 subtree
// (breadth-first index 2^d - 1 + m), first-bit-0 outputs only: Dv[u], u < 8.
template <typename T>
__device__ __forceinline__ void bwd4_half(const T (&S)[31], T (&Dv)[8]) {
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
#pragma unroll
  for (int q = 0; q < 8; ++q) Dv[q] = C[0][q] + C[1][q];
}

// The same subtree with every path complemented (index m -> 2^d - 1 - m).
template <typename T>
__device__ __forceinline__ void mirror_subtree(const T (&S)[31], T (&Sm)[31]) {
#pragma unroll
  for (int d = 0; d <= 4; ++d)
#pragma unroll
    for (int m = 0; m < (1 << d); ++m) Sm[(1 << d) - 1 + m] = S[(1 << d) - 1 + ((1 << d) - 1 - m)];
}

// Four backward stages, canonical half: B_i[y][u s] for u < 8 (stride 8 S4) and
// every s, from B_{i+4} stored as its columns s < S4/2 (stride S4/2), or, VC, from
// the compact v (i + 4 = n).  One thread per (row w, column s < S4/2) loads w's
// depth-4 subtree at column s once and writes both (w, s) and (cpl w, S4-1-s),
// whose subtree is the mirror of the same values.  VC: one thread per row w that
// is empty or starts with 0 (local rank of the subtree of "0"; the thread of local
// rank 0 also takes the empty row), writing w and cpl w.  DP: stage 0, D for
// x < 2^(n-1) with weight 2.
template <typename T, bool DP, bool VC>
__global__ __launch_bounds__(kBlock) void k_bwd_stage4_sym(int n, int i, const T* __restrict__ src,
                                                           size_t sstride, T* __restrict__ dst, size_t dstride,
                                                           Group<T> g, Order o) {
  const int b = blockIdx.y;
  if (g.frz && g.st[b].converged) return;
  uint32_t q, s;
  const bool valid = order_slot(o, q, s);
  if (!DP && !valid) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh = n - i - 4;                  // log2 of the full source width S4
  const uint32_t S4 = 1u << sh;
  Part p = part_empty();
  if (valid) {
    // row w: for VC with i > 0 the slot is a local rank of the subtree of "0"
    const uint32_t w = (VC && i > 0) ? q + (1u << length_of_rank(q)) : q;
    const int rounds = (VC && i > 0 && q == 0u) ? 2 : 1;  // the empty row as well
#pragma unroll 1
    for (int rd = 0; rd < rounds; ++rd) {
      const uint32_t wr = rd ? 0u : w;
      T S[31];
#pragma unroll
      for (int d = 0; d <= 4; ++d)
#pragma unroll
        for (int m = 0; m < (1 << d); ++m) {
          const uint32_t node = ((wr + 1u) << d) - 1u + uint32_t(m);
          if constexpr (VC) S[(1 << d) - 1 + m] = v_sym(src, node);
          else S[(1 << d) - 1 + m] = src[((size_t)node << (sh - 1)) + s];
        }
      T Dv[8], Dm[8], Sm[31];
      bwd4_half<T>(S, Dv);
      mirror_subtree<T>(S, Sm);
      bwd4_half<T>(Sm, Dm);
      const uint32_t wm = mirror_rank(wr);
      if constexpr (DP) {
        // i = 0: w is the empty row; columns s and S4 - 1 - s (the same column when S4 = 1)
        const double M = g.st[b].M;
        uint32_t xs[8], xm[8];
        Vec<T, 1> gs[8], gm[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          xs[u] = uint32_t(u) * S4 + s;
          xm[u] = uint32_t(u) * S4 + (S4 - 1u - s);
          gs[u].v[0] = Dv[u];
          gm[u].v[0] = Dm[u];
        }
        d_records<T, 1, 8>(g, b, M, xs, gs, p, 2.0);
        if (S4 > 1u) d_records<T, 1, 8>(g, b, M, xm, gm, p, 2.0);
      } else {
        T* op = dst + ((size_t)wr << (sh + 3));
        T* om = dst + ((size_t)wm << (sh + 3));
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          op[uint32_t(u) * S4 + s] = Dv[u];
          if (wm != wr || (!VC && S4 > 1u)) om[uint32_t(u) * S4 + (S4 - 1u - s)] = Dm[u];
        }
      }
    }
  }
  if constexpr (DP) {
    store_block_part(g.part + (size_t)b * g.ps, blockIdx.x, p);
  }
}

// The four-position forward step of k_fwd_stage4_sym for output rows of width 1
// (sh = 0: every stored source row is its 8 groups of first bit 0).
template <typename T>
__device__ __forceinline__ T fwd4_sym_w1(const T* __restrict__ src, uint32_t y, int ly, T (&F4)[30]) {
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
      const T* row = src + ((size_t)P[j] << 3);
      const T* rowm = src + ((size_t)mirror_rank(P[j]) << 3);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        F0[j][u] = row[u];
        F0[j][8 + u] = rowm[7 - u];
      }
    }
  if (4 <= ly) {
    if (lastb[3]) {
      const T* rowm = src + ((size_t)mirror_rank(P[4]) << 3);
#pragma unroll
      for (int u = 0; u < 8; ++u) H4[u] = rowm[7 - u];
    } else {
      const T* row = src + ((size_t)P[4] << 3);
#pragma unroll
      for (int u = 0; u < 8; ++u) H4[u] = row[u];
    }
  }
  return fwd4_registers<T>(F0, H4, lastb, F4);
}

// The last four positions, canonical half (n >= kLast4MinN, four positions left
// after the four-position launches): k_fwd_last4 for the outputs that are empty or
// start with 0, written to the compact v (row R of length k >= 1 starting with 0 at
// R - 2^(k-1) + 1, the empty row at 0).  Deep block: a node a of level L - 6 (L =
// n - 4) starting with 0, its 64 leaves of level L and the 30 rows below each (first
// wavefront, staged in LDS and written as one compact run per level), and the 63
// rows of a's subtree above level L (second wavefront); the other blocks take the
// empty row and the rows of level < L - 6 starting with 0, by compact index.
template <typename T, bool LOGV>
__global__ __launch_bounds__(kLast4Threads) void k_fwd_last4_sym(int n, const T* __restrict__ src, size_t sstride,
                                                                 T* __restrict__ dst, size_t dstride,
                                                                 const State* st, const Consts* cs, int frz) {
  const int b = blockIdx.y;
  if (frz && st[b].converged) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int L = n - 4, La = L - 6;
  const uint32_t ndeep = 1u << (La - 1);          // nodes of level La starting with 0
  const uint32_t t = threadIdx.x;
  T F4[30];
  auto outv = [&](uint32_t rank, T r) -> T {
    if constexpr (LOGV) return log_weighted<T>(cs[b], rank, r);
    else return r;
  };
  if (blockIdx.x >= ndeep) {
    // compact index q < 2^(La-1): the empty row (q = 0) or rank q + 2^floor(log2 q) - 1
    const uint32_t q = (blockIdx.x - ndeep) * kLast4Threads + t;
    if (q >= ndeep) return;
    const uint32_t y = q == 0u ? 0u : q + (1u << (31 - __clz(q))) - 1u;
    dst[q] = outv(y, fwd4_sym_w1<T>(src, y, length_of_rank(y), F4));
    return;
  }
  __shared__ T stage[kLast4Stage];
  // hardware block 8 k + x runs on XCD x: node k of XCD x's run of ndeep / 8
  const uint32_t da = (ndeep & 7u) ? blockIdx.x : (blockIdx.x & 7u) * (ndeep >> 3) + (blockIdx.x >> 3);
  const uint32_t a = (1u << La) - 1u + da;        // level La, first bit 0
  const uint32_t A0 = ((a + 1u) << 6) - 1u;       // its first leaf (level L)
  T* s1 = stage;
  T* s2 = s1 + 3 * 64;
  T* s3 = s2 + 5 * 64;
  T* s4 = s3 + 9 * 64;
  if (t < 64u) {
    const uint32_t y = A0 + t;
    const T va = fwd4_sym_w1<T>(src, y, L, F4);
    dst[y - (1u << (L - 1)) + 1u] = outv(y, va);
    // F4: depth d, index m at (1 << d) - 2 + m; every row of depth d has length L + d
    const uint32_t r1 = ((y + 1u) << 1) - 1u, r2 = ((y + 1u) << 2) - 1u, r3 = ((y + 1u) << 3) - 1u,
                   r4 = ((y + 1u) << 4) - 1u;
#pragma unroll
    for (int q = 0; q < 2; ++q) s1[3u * t + q] = outv(r1 + q, F4[q]);
#pragma unroll
    for (int q = 0; q < 4; ++q) s2[5u * t + q] = outv(r2 + q, F4[2 + q]);
#pragma unroll
    for (int q = 0; q < 8; ++q) s3[9u * t + q] = outv(r3 + q, F4[6 + q]);
#pragma unroll
    for (int q = 0; q < 16; ++q) s4[17u * t + q] = outv(r4 + q, F4[14 + q]);
  } else if (t < 127u) {
    // node q of a's subtree above level L: depth d = log2(q + 1), length La + d
    const uint32_t q = t - 64u;
    const int d = length_of_rank(q);
    const uint32_t y = ((a + 1u) << d) - 1u + (q + 1u - (1u << d));
    dst[y - (1u << (La + d - 1)) + 1u] = outv(y, fwd4_sym_w1<T>(src, y, La + d, F4));
  }
  __syncthreads();
#pragma unroll
  for (int j = 1; j <= 4; ++j) {
    const uint32_t wj = 1u << j, stride = wj + 1u;
    const T* sj = j == 1 ? s1 : j == 2 ? s2 : j == 3 ? s3 : s4;
    T* out = dst + (wj * (A0 + 1u) - 1u) - (1u << (L + j - 1)) + 1u;
#pragma unroll
    for (uint32_t k = 0; k < wj / 2u; ++k) {
      const uint32_t e = k * kLast4Threads + t;
      out[e] = sj[(e >> j) * stride + (e & (wj - 1u))];
    }
  }
}

// The first four positions (i = 0) of the canonical half fused with the pending
// update, as k_fwd_first4_upd for the full kernels: the thread of column s < S4/2
// covers the 16 stored inputs x = u S4 + s and u S4 + (S4 - 1 - s) (u < 8, first
// bit 0, where D is kept), forms their new log p from the final record as k_update
// does, writes it at x and at cpl x, and uses p = e^{log p - M'} in registers as the
// row of F_0 that k_fwd_stage4_sym reads (group u >= 8 at s being p(cpl x) of the
// input u' = 15 - u at column S4 - 1 - s).  The values equal those of k_update
// followed by k_fwd_stage4_sym.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fwd_first4_upd_sym(int n, T* __restrict__ dst, size_t dstride,
                                                               Group<T> g, Order o, double floor, int check_tol) {
  const int b = blockIdx.y;
  if (g.st[b].converged) return;
  const UpdateParams up = update_params<T>(g, b, check_tol, blockIdx.x == 0 && threadIdx.x == 0);
  if (up.stop) return;
  uint32_t y, s;
  if (!order_slot(o, y, s)) return;  // y = 0, the one row of F_0
  dst += (size_t)b * dstride;
  T* lp = g.lp + (size_t)b * g.xs;
  const T* D = g.D + (size_t)b * g.xs;
  const int sh = n - 4;
  const uint32_t S4 = 1u << sh, sm = S4 - 1u - s, X = 1u << n;
  const T lo = T(up.Mn - floor), eta = T(g.eta);
  uint32_t xs[16];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    xs[u] = (uint32_t(u) << sh) + s;
    xs[8 + u] = (uint32_t(7 - u) << sh) + sm;
  }
  T nl[16], dv[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    if (!g.dsum) nl[u] = lp[xs[u]];  // dsum: D holds log p + D
    dv[u] = D[xs[u]];
  }
  T F0[4][16], H4[8];
#pragma unroll
  for (int j = 1; j < 4; ++j)
#pragma unroll
    for (int u = 0; u < 16; ++u) F0[j][u] = T(0);
#pragma unroll
  for (int u = 0; u < 8; ++u) H4[u] = T(0);
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    nl[u] = g.dsum ? update_value_sum<T>(up, lo, dv[u]) : update_value<T>(up, eta, lo, nl[u], dv[u]);
    lp[xs[u]] = nl[u];
    lp[X - 1u - xs[u]] = nl[u];
    F0[0][u] = exp_t<T>(nl[u] - T(up.Mn));
  }
  uint32_t P[5], lastb[4];
  fwd4_path(0u, P, lastb);
  T F4[30];
  const T vy = fwd4_registers<T>(F0, H4, lastb, F4);
  const int ho = sh - 1;                     // log2 of the stored output width
  dst[s] = vy;
#pragma unroll
  for (int d = 1; d <= 4; ++d)
#pragma unroll
    for (int m = 0; m < (1 << d); ++m)
      dst[((size_t)((1u << d) - 1u + uint32_t(m)) << ho) + s] = F4[(1 << d) - 2 + m];
}

}  // namespace

using namespace fac;

bool symmetric_supported(int n, int fuse) { return fuse && n >= 4 && (n % 2) == 0; }

template <typename T>
hipError_t launch_forward_sym(const Group<T>& g, hipStream_t s, int* launches, int fuse, const FusedUpdate* upd) {
  const int n = g.n;
  constexpr int V = 16 / sizeof(T);
  const T* src = g.p;
  size_t ss = g.xs;
  int k = 0;
  int i0 = 0;
  if (upd && !forward_update_fusable(n, fuse)) return hipErrorInvalidValue;
  for (; fuse >= 2 && i0 + 4 < n; i0 += 4, k++) {
    T* dst = (k & 1) ? g.f1 : g.f0;
    const uint32_t S4 = 1u << (n - i0 - 4);
    Order o = make_order(i0 + 1, ilog2(S4 / 2u), sizeof(T));
    make_order_xcd(i0 + 1, ilog2(S4 / 2u), kBlock, o, true);  // o unchanged where infeasible
    if (i0 == 0 && upd)
      hipLaunchKernelGGL((k_fwd_first4_upd_sym<T>), dim3(order_blocks(o, kBlock), g.nb), dim3(kBlock), 0, s, n,
                         dst, g.fs, g, o, upd->floor, upd->check_tol);
    else
      hipLaunchKernelGGL((k_fwd_stage4_sym<T>), dim3(order_blocks(o, kBlock), g.nb), dim3(kBlock), 0, s, n, i0,
                         src, ss, dst, g.fs, g.st, o, g.frz);
    if (launches) ++*launches;
    src = dst;
    ss = g.fs;
  }
  // fuse >= 4: the last four positions in one launch (writes the compact v)
  if (fuse >= 4 && n >= kLast4MinN && n - i0 == 4) {
    const uint32_t ndeep = 1u << (n - 11), top = ndeep;  // deep blocks; compact rows above
    const dim3 grid(ndeep + (top + kLast4Threads - 1u) / kLast4Threads, g.nb);
    hipLaunchKernelGGL((k_fwd_last4_sym<T, true>), grid, dim3(kLast4Threads), 0, s, n, src, ss, g.v, g.ys, g.st,
                       g.cs, g.frz);
    if (launches) ++*launches;
    return hipGetLastError();
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
  const int lead = (fuse >= 2) ? n % 4 : -1;  // even n: 0 or 2
  for (int top = n; top > 0; k++) {
    // fuse >= 3: the first eight positions (from the compact v) in one launch
    if (fuse >= 3 && top == n && n % 4 == 0 && n >= 12) {
      const hipError_t e = launch_backward8_sym_v<T>(g, s, (k & 1) ? g.f1 : g.f0);
      if (e != hipSuccess) return e;
      if (launches) ++*launches;
      src = (k & 1) ? g.f1 : g.f0;
      ss = g.fs;
      top = n - 8;
      continue;
    }
    if (lead >= 0 && n - top >= lead) {
      const int i = top - 4;
      const bool last = (i == 0), vc = (top == n);
      T* dst = last ? g.g : ((k & 1) ? g.f1 : g.f0);
      const size_t ds = last ? g.xs : g.fs;
      const uint32_t S4 = 1u << (n - i - 4);
      // rows w x columns s < S4/2, or (from v) the rows of the subtree of "0"
      Order o = vc ? (i > 0 ? make_order(i, 0, sizeof(T)) : make_order(1, 0, sizeof(T)))
                   : make_order(i + 1, ilog2(S4 / 2u), sizeof(T));
      if (!vc && !last) make_order_xcd(i + 1, ilog2(S4 / 2u), kBlock, o);  // o unchanged where infeasible
      const uint32_t nbk = order_blocks(o, kBlock);
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

template hipError_t launch_forward_sym<float>(const Group<float>&, hipStream_t, int*, int, const FusedUpdate*);
template hipError_t launch_forward_sym<double>(const Group<double>&, hipStream_t, int*, int, const FusedUpdate*);
template hipError_t launch_backward_sym<float>(const Group<float>&, hipStream_t, int*, int*, int);
template hipError_t launch_backward_sym<double>(const Group<double>&, hipStream_t, int*, int*, int);

}  // namespace ba
