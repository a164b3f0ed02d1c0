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

#include "ba_factored_common.h"

namespace ba {
namespace {

using namespace fac;

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


// The four-position forward step of one (row y of length ly, column s of the output
// width 2^sh): loads F_i of y's path and returns F_{i+4}[y] (and, in F4, the 30 rows
// below y; meaningful when y is a leaf).  The first stage is formed row by row from
// the deepest ancestor up, so that only one loaded row and the half of the row below
// it are live at a time.
template <typename T>
__device__ __forceinline__ T fwd4_thread(const T* __restrict__ src, int sh, uint32_t y, int ly, uint32_t s,
                                         T (&F4)[30]) {
  uint32_t P[5], lastb[4];
  fwd4_path(y, P, lastb);
  T F1p[4][8], F1s[2][8], Hc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) Hc[u] = T(0);
  if (4 <= ly) {
    const uint32_t row = (P[4] << (sh + 4)) + (lastb[3] << (sh + 3)) + s;
#pragma unroll
    for (int u = 0; u < 8; ++u) Hc[u] = at(src, row + (uint32_t(u) << sh));
  }
#pragma unroll
  for (int j = 3; j >= 0; --j) {
    T R[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) R[u] = T(0);
    if (j <= ly) {
      const uint32_t row = (P[j] << (sh + 4)) + s;
#pragma unroll
      for (int u = 0; u < 16; ++u) R[u] = at(src, row + (uint32_t(u) << sh));
    }
#pragma unroll
    for (int g = 0; g < 8; ++g) F1p[j][g] = (R[g] + R[8 + g]) + Hc[g];
    if (j > 0) {
#pragma unroll
      for (int g = 0; g < 8; ++g) Hc[g] = lastb[j - 1] ? R[8 + g] : R[g];
    } else {
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int g = 0; g < 8; ++g) F1s[c][g] = R[c * 8 + g];
    }
  }
  return fwd4_after_stage1<T>(F1p, F1s, lastb, F4);
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
                                                       const Consts* cs, Order o, int frz) {
  const int b = blockIdx.y;
  if (frz && st[b].converged) return;
  uint32_t y, s;
  if (!order_slot(o, y, s)) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh = n - i - 4;                  // log2 of the output width S4
  const int ly = length_of_rank(y);
  T F4[30];
  T vy = fwd4_thread<T>(src, sh, y, ly, s, F4);
  if constexpr (LOGV) vy = log_weighted<T>(cs[b], y, vy);
  at(dst, (y << sh) + s) = vy;
  if (ly != i) return;
#pragma unroll
  for (int d = 1; d <= 4; ++d)
#pragma unroll
    for (int m = 0; m < (1 << d); ++m) {
      const uint32_t rk = ((y + 1u) << d) - 1u + uint32_t(m);
      T v = F4[(1 << d) - 2 + m];
      if constexpr (LOGV) v = log_weighted<T>(cs[b], rk, v);
      at(dst, (rk << sh) + s) = v;
    }
}

// The first four positions (i = 0) fused with the update that the previous
// iteration left pending: every thread forms the update from the final record
// (as k_update does), writes the new log p of its 16 inputs x = u 2^(n-4) + s and
// uses p = e^{log p - M'} in registers as F_0 (p itself is not stored), then runs
// the step of k_fwd_stage4 for the one row of F_0.  The values equal those of
// k_update followed by k_fwd_stage4.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fwd_first4_upd(int n, T* __restrict__ dst, size_t dstride, Group<T> g,
                                                           Order o, double floor, int check_tol) {
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
  const T lo = T(up.Mn - floor), eta = T(g.eta);
  T nl[16], dv[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    if (!g.dsum) nl[u] = lp[(uint32_t(u) << sh) + s];  // dsum: D holds log p + D
    dv[u] = D[(uint32_t(u) << sh) + s];
  }
  T R[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    nl[u] = g.dsum ? update_value_sum<T>(up, lo, dv[u]) : update_value<T>(up, eta, lo, nl[u], dv[u]);
    lp[(uint32_t(u) << sh) + s] = nl[u];
    R[u] = exp_t<T>(nl[u] - T(up.Mn));
  }
  // the first stage of fwd4_thread for a row without ancestors
  uint32_t P[5], lastb[4];
  fwd4_path(0u, P, lastb);
  T F1p[4][8], F1s[2][8];
#pragma unroll
  for (int j = 1; j < 4; ++j)
#pragma unroll
    for (int q = 0; q < 8; ++q) F1p[j][q] = (T(0) + T(0)) + T(0);
#pragma unroll
  for (int q = 0; q < 8; ++q) F1p[0][q] = (R[q] + R[8 + q]) + T(0);
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int q = 0; q < 8; ++q) F1s[c][q] = R[c * 8 + q];
  T F4[30];
  dst[s] = fwd4_after_stage1<T>(F1p, F1s, lastb, F4);
#pragma unroll
  for (int d = 1; d <= 4; ++d)
#pragma unroll
    for (int m = 0; m < (1 << d); ++m)
      dst[((size_t)((1u << d) - 1u + uint32_t(m)) << sh) + s] = F4[(1 << d) - 2 + m];
}

// The first eight positions (i = 0..7) in one launch, for n >= kFirst8MinN; UPD:
// also the update the previous iteration left pending (as k_fwd_first4_upd).  A
// block takes 16 consecutive columns s of F_8 (width S8 = 2^(n-8)).  Step 1: the 16
// inputs x = u1 2^(n-4) + u2 S8 + s (u1 = 0..15, s = s0 + c) of pair (u2, c) are loaded
// (p, or log p and D with the update made) by two threads, eight each; the first runs
// the four-position step of the one row of F_0, leaving F_4[z][u2 S8 + s] for the 31
// rows z in LDS.  Step 2: thread (z, c)
// runs the four-position step of row z of F_4 (k_fwd_stage4 at i = 4) on the LDS rows
// of its path and writes F_8 of row z and, for a leaf, of the 30 rows below it (16
// lanes per row: 64-byte runs).  Every value is the same sum, in
// the same order, as with k_fwd_first4_upd (or k_fwd_stage4) and k_fwd_stage4.
constexpr int kFirst8MinN = 12;
constexpr uint32_t kFirst8Threads = 512;

// Positions 0-7 of the forward sweep for the columns s0 .. s0+15 of F_8, from the
// inputs held in R by threads t < 256 (R[u1] = p(x) for x = u1 2^(n-4) + u2 2^(n-8) +
// s0 + c1, pair t = u2 16 + c1, u1 < 16; the block synchronised after R was formed,
// buf free): the four-position step of the one row of F_0 for each pair leaves F_4
// (31 rows x 16 u2 x 16 columns) in buf, then thread (z, c), z < 31, runs the
// four-position step of row z of F_4 on the LDS rows of its path and writes F_8 of
// row z and, for a leaf, of the 30 rows below it.
// HALF (complement-symmetric iterate, the column block's first bit 0): F_8 keeps the
// rows that start with 0 and the empty row at every column; a value of a row that
// starts with 1 goes to its complement's row at the complementary column, one of the
// empty row to both columns.
template <int C>
constexpr uint32_t f4_pitch() { return 16u * uint32_t(C) + 16u; }  // F_4 row in LDS: 16 u2 x C columns, padded

// C: the columns of the block (16, or 8 with 128 pairs and 248 step-2 threads).
template <typename T, bool HALF = false, int C = 16>
__device__ __forceinline__ void first8_steps(T* buf, const T (&R)[16], uint32_t t, T* __restrict__ dst, int n,
                                             uint32_t s0) {
  static_assert(C == 16 || C == 8, "16 or 8 columns");
  constexpr uint32_t PC = f4_pitch<C>();
  constexpr int LC = C == 16 ? 4 : 3;
  const int sh8 = n - 8;
  auto put = [&](uint32_t R, uint32_t col, T v) {
    if constexpr (HALF) {
      const int k = length_of_rank(R);
      const uint32_t cc = (1u << sh8) - 1u - col;
      if (R == 0u) {
        at(dst, col) = v;
        at(dst, cc) = v;
      } else if (R + 1u - (1u << k) >= (1u << (k - 1))) {
        at(dst, (mirror_rank(R) << sh8) + cc) = v;
      } else {
        at(dst, (R << sh8) + col) = v;
      }
    } else {
      at(dst, (R << sh8) + col) = v;
    }
  };
  // step 1b: the four-position step of the one row of F_0 for pair pr
  if (t < 16u * C) {
    const uint32_t u2 = t >> LC, c1 = t & uint32_t(C - 1);
    // the first stage of fwd4_thread for the row without ancestors
    uint32_t P[5], lastb[4];
    fwd4_path(0u, P, lastb);
    T F1p[4][8], F1s[2][8];
#pragma unroll
    for (int j = 1; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 8; ++q) F1p[j][q] = (T(0) + T(0)) + T(0);
#pragma unroll
    for (int q = 0; q < 8; ++q) F1p[0][q] = (R[q] + R[8 + q]) + T(0);
#pragma unroll
    for (int cc = 0; cc < 2; ++cc)
#pragma unroll
      for (int q = 0; q < 8; ++q) F1s[cc][q] = R[cc * 8 + q];
    T F4[30];
    const T v0 = fwd4_after_stage1<T>(F1p, F1s, lastb, F4);
    T* col = buf + u2 * uint32_t(C) + c1;
    col[0] = v0;
#pragma unroll
    for (int z = 1; z < 31; ++z) col[uint32_t(z) * PC] = F4[z - 1];
  }
  __syncthreads();
  // step 2: thread (z, c), z < 31: fwd4_thread on the LDS rows of z's path
  const uint32_t z = t >> LC, c = t & uint32_t(C - 1);
  const int lz = length_of_rank(z);
  if (z < 31u) {
    T F4[30];
    uint32_t P[5], lastb[4];
    fwd4_path(z, P, lastb);
    T F1p[4][8], F1s[2][8], Hc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) Hc[u] = T(0);
    if (4 <= lz) {
      const T* row = buf + P[4] * PC + (lastb[3] ? 8u * C : 0u) + c;
#pragma unroll
      for (int u = 0; u < 8; ++u) Hc[u] = row[uint32_t(u) * C];
    }
#pragma unroll
    for (int j = 3; j >= 0; --j) {
      T R[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) R[u] = T(0);
      if (j <= lz) {
        const T* row = buf + P[j] * PC + c;
#pragma unroll
        for (int u = 0; u < 16; ++u) R[u] = row[uint32_t(u) * C];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) F1p[j][q] = (R[q] + R[8 + q]) + Hc[q];
      if (j > 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) Hc[q] = lastb[j - 1] ? R[8 + q] : R[q];
      } else {
#pragma unroll
        for (int cc = 0; cc < 2; ++cc)
#pragma unroll
          for (int q = 0; q < 8; ++q) F1s[cc][q] = R[cc * 8 + q];
      }
    }
    const T vz = fwd4_after_stage1<T>(F1p, F1s, lastb, F4);
    // F_8 of row z and, for a leaf, of the 30 rows below it: 16 consecutive columns of
    // each row per 16 lanes
    put(z, s0 + c, vz);
    if (lz == 4) {
#pragma unroll
      for (int d = 1; d <= 4; ++d)
#pragma unroll
        for (int m = 0; m < (1 << d); ++m) put(((z + 1u) << d) - 1u + uint32_t(m), s0 + c, F4[(1 << d) - 2 + m]);
    }
  }
}

template <typename T, bool UPD>
__global__ __launch_bounds__(kFirst8Threads) void k_fwd_first8(int n, const T* __restrict__ src, size_t sstride,
                                                               T* __restrict__ dst, size_t dstride, Group<T> g,
                                                               double floor, int check_tol, int nmax) {
  const int b = blockIdx.y;
  if ((UPD || g.frz) && g.st[b].converged) return;
  UpdateParams up{};
  if constexpr (UPD) {
    if (nmax > 0) {
      // shift by the max (FP32 iterates between two normalisations, eta = 1, the D
      // array holding log p + D): log p <- max(a - m, -floor) with m = max a over the
      // instance, from the D launch's nmax block maxima (each wave takes their max
      // itself), i.e. the new iterate scaled so that its max is 1.  Its exact
      // normalisation is a constant shift of log p that the sweeps, the floor and the
      // next D launch do not depend on; the update that ends a ba_step call (or a
      // ba_run chunk) normalises with L as usual.  No L, U or I is formed here.
      const float* bm = reinterpret_cast<const float*>(g.part + (size_t)b * g.ps + kBlockMaxima);
      float mv = -INFINITY;
      for (int j = int(threadIdx.x & (kWave - 1)); j < nmax; j += kWave) mv = fmaxf(mv, bm[j]);
#pragma unroll
      for (int off = kWave / 2; off > 0; off >>= 1) mv = fmaxf(mv, __shfl_xor(mv, off));
      const bool finite = isfinite(mv);
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        State* st = g.st + b;
        if (!finite) {
          st->bad = 1;
          st->converged = 1;
        } else {
          st->M = 0.0;
          st->iters += 1;
        }
      }
      if (!finite) return;
      up = UpdateParams{double(mv), double(mv), 0.0, false, false};  // L <- m: the new max is 0
    } else {
      up = update_params<T>(g, b, check_tol, blockIdx.x == 0 && threadIdx.x == 0);
    }
    if (up.stop) return;
  }
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh8 = n - 8;                      // log2 of the F_8 width
  // neighbouring column blocks share 128-byte lines: consecutive logical blocks on one XCD
  const uint32_t s0 = logical_block() * 16u, t = threadIdx.x;
  __shared__ T buf[31u * f4_pitch<16>()];
  // step 1a: all threads load (and update) 8 of the 16 inputs of pair pr = (u2, c):
  // u1 = 8 h .. 8 h + 7; the upper halves pass through LDS (the start of buf)
  const uint32_t h = t >> 8, pr = t & 255u;
  const uint32_t u2 = pr >> 4, c1 = pr & 15u;
  const uint32_t x0 = (u2 << sh8) + s0 + c1;  // u1 = 0
  T R[16];
  if constexpr (UPD) {
    T* lp = g.lp + (size_t)b * g.xs;
    const T* D = g.D + (size_t)b * g.xs;
    const T lo = T(up.Mn - floor), eta = T(g.eta);
    T nl[8], dv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t x = ((8u * h + uint32_t(k)) << (n - 4)) + x0;
      if (!g.dsum) nl[k] = lp[x];  // dsum: D holds log p + D
      dv[k] = D[x];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      nl[k] = g.dsum ? update_value_sum<T>(up, lo, dv[k]) : update_value<T>(up, eta, lo, nl[k], dv[k]);
      lp[((8u * h + uint32_t(k)) << (n - 4)) + x0] = nl[k];
      R[k] = exp_t<T>(nl[k] - T(up.Mn));
    }
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) R[k] = src[((8u * h + uint32_t(k)) << (n - 4)) + x0];
  }
  if (h) {
#pragma unroll
    for (int k = 0; k < 8; ++k) buf[uint32_t(k) * 256u + pr] = R[k];
  }
  __syncthreads();
  if (!h) {
#pragma unroll
    for (int k = 0; k < 8; ++k) R[8 + k] = buf[uint32_t(k) * 256u + pr];
  }
  __syncthreads();
  first8_steps<T>(buf, R, t, dst, n, s0);
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
    if constexpr (DP) {
      const uint32_t xs[1] = {idx};
      const Vec<T, V> gs[1] = {o};
      d_records<T, V, 1>(g, b, M, xs, gs, p);
    }
    else stv<T, V>(dst + idx, o);
  }
  if constexpr (DP) {
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

// The last two positions for n >= kLast2MinN, in the same formula as
// k_fwd_stage2_w1 (source rows of width 4, output rows of width 1):
//   r(c) = sum_u F[c][u] + 2 F[p][3 last(c)] + F[p][1] + F[p][2] + F[g][2 last(p) + last(c)]
// (p the parent, g the grandparent of c; terms of rows longer than n-2 are zero).
// Deep blocks (blockIdx.x < 2^(n-4) / kBlock): thread t takes the row a of level
// L = n-4 of rank A0 + t and every output row of a's subtree down to level n (31
// rows): it loads F of a, its 2 children and 4 grandchildren (its whole source
// subtree), of a's parent and one value of its grandparent.  Each level of a
// block's outputs is a contiguous run of ranks (kLast2Threads * 2^j values at
// level L+j), so the values are staged in LDS (row stride 2^j + 1 against bank
// conflicts) and written back coalesced.  The other blocks take one output row of
// level < L per thread.  Each output is the same sum, in the same order, as in
// k_fwd_stage2_w1.  One wavefront per block: its load, sum and store phases then
// drift apart from those of the other blocks on the CU (256-thread blocks, whose
// phases coincide, took 21.4 us at n = 20 and three instances; 64-thread blocks
// 13.6 us; the per-row kernel 17.4 us).
constexpr int kLast2Threads = 64;   // threads per block
constexpr int kLast2MinN = 12;      // 2^(n-4) >= kLast2Threads
constexpr int kLast2Lds = 1 + 3 + 5 + 9 + 17;  // LDS values per thread (padded)

template <typename T>
__device__ __forceinline__ T last2_sum(const Vec<T, 4>& own, const Vec<T, 4>& par, uint32_t b, T gv) {
  const T e = b ? par.v[3] : par.v[0];
  return (((own.v[0] + own.v[1]) + (own.v[2] + own.v[3])) + ((e + e) + (par.v[1] + par.v[2]))) + gv;
}
// No own row (level n-1): the same sum with the own terms zero.
template <typename T>
__device__ __forceinline__ T last2_sum_noown(const Vec<T, 4>& par, uint32_t b, T gv) {
  const T e = b ? par.v[3] : par.v[0];
  return ((e + e) + (par.v[1] + par.v[2])) + gv;
}

template <typename T, bool LOGV>
__global__ __launch_bounds__(kLast2Threads) void k_fwd_last2(int n, const T* __restrict__ src, size_t sstride,
                                                      T* __restrict__ dst, size_t dstride, const State* st,
                                                      const Consts* cs) {
  const int b = blockIdx.y;
  if (st[b].converged) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int L = n - 4;
  const uint32_t ndeep = (1u << L) / kLast2Threads;
  const uint32_t t = threadIdx.x;
  // v = w_k log r at the five levels L .. L+4 (LOGV), else r
  const T w0 = T(cs[b].w[L]), w1 = T(cs[b].w[L + 1]), w2 = T(cs[b].w[L + 2]), w3 = T(cs[b].w[L + 3]),
          w4 = T(cs[b].w[L + 4]);
  auto outv = [](T w, T r) -> T {
    if constexpr (LOGV) return wlog_t<T>(w, r);
    else return r;
  };
  if (blockIdx.x >= ndeep) {
    // shallow rows: levels 0 .. L-1, ranks 0 .. 2^L - 2
    const uint32_t c = (blockIdx.x - ndeep) * kLast2Threads + t;
    if (c + 1u >= (1u << L)) return;
    const Vec<T, 4> own = ld<T, 4>(src + 4u * c);
    Vec<T, 4> par = zero_vec<T, 4>();
    T gv = T(0);
    const uint32_t pr = (c - 1u) >> 1, bb = (c - 1u) & 1u;
    if (c >= 1u) par = ld<T, 4>(src + 4u * pr);
    if (c >= 3u) gv = src[4u * ((pr - 1u) >> 1) + 2u * ((pr - 1u) & 1u) + bb];
    T r = last2_sum<T>(own, par, bb, gv);
    if constexpr (LOGV) r = log_weighted<T>(cs[b], c, r);
    dst[c] = r;
    return;
  }
  __shared__ T stage[kLast2Lds * kLast2Threads];
  const uint32_t A0 = (1u << L) - 1u + blockIdx.x * kLast2Threads;
  const uint32_t a = A0 + t;
  const uint32_t pa = (a - 1u) >> 1, ba = (a - 1u) & 1u;  // L >= 8: parent and grandparent exist
  const uint32_t ga = (pa - 1u) >> 1, bp = (pa - 1u) & 1u;
  const Vec<T, 4> A = ld<T, 4>(src + 4u * a);
  const Vec<T, 4> P = ld<T, 4>(src + 4u * pa);
  const T gA = src[4u * ga + 2u * bp + ba];
  Vec<T, 4> C[2], GC[4];
#pragma unroll
  for (int q = 0; q < 2; ++q) C[q] = ld<T, 4>(src + 4u * (2u * a + 1u + q));
#pragma unroll
  for (int q = 0; q < 4; ++q) GC[q] = ld<T, 4>(src + 4u * (4u * a + 3u + q));
  // the grandparent terms of a's children: P[2 last(a) + q], selected by value
  const T P0 = P.v[0], P1 = P.v[1], P2 = P.v[2], P3 = P.v[3];
  const T Pq[2] = {ba ? P2 : P0, ba ? P3 : P1};
  // level L (stride 1), L+1 (3), L+2 (5), L+3 (9), L+4 (17) regions of the stage
  T* s0 = stage;
  T* s1 = s0 + kLast2Threads;
  T* s2 = s1 + 3 * kLast2Threads;
  T* s3 = s2 + 5 * kLast2Threads;
  T* s4 = s3 + 9 * kLast2Threads;
  s0[t] = outv(w0, last2_sum<T>(A, P, ba, gA));
#pragma unroll
  for (int q = 0; q < 2; ++q) s1[3u * t + q] = outv(w1, last2_sum<T>(C[q], A, uint32_t(q), Pq[q]));
#pragma unroll
  for (int q = 0; q < 4; ++q)
    s2[5u * t + q] = outv(w2, last2_sum<T>(GC[q], C[q >> 1], uint32_t(q & 1), A.v[q]));
#pragma unroll
  for (int q = 0; q < 8; ++q)
    s3[9u * t + q] = outv(w3, last2_sum_noown<T>(GC[q >> 1], uint32_t(q & 1), C[q >> 2].v[q & 3]));
#pragma unroll
  for (int q = 0; q < 16; ++q) s4[17u * t + q] = outv(w4, GC[q >> 2].v[q & 3]);
  __syncthreads();
  // level L+j: kLast2Threads * 2^j consecutive ranks from 2^j (A0 + 1) - 1
  dst[A0 + t] = s0[t];
#pragma unroll
  for (int j = 1; j <= 4; ++j) {
    const uint32_t w2 = 1u << j, stride = w2 + 1u;
    const T* sj = j == 1 ? s1 : j == 2 ? s2 : j == 3 ? s3 : s4;
    T* out = dst + (w2 * (A0 + 1u) - 1u);
#pragma unroll
    for (uint32_t k = 0; k < w2; ++k) {
      const uint32_t e = k * kLast2Threads + t;
      out[e] = sj[(e >> j) * stride + (e & (w2 - 1u))];
    }
  }
}

// The last four positions (n-4 .. n-1) for n >= kLast4MinN: the four-position step
// of k_fwd_stage4 at i = n-4 (output rows of width 1), with the outputs staged in
// LDS.  Deep block: the node a of level L - 6 (L = n-4) of rank 2^(L-6) - 1 +
// blockIdx.x and its subtree down to level n.  Its first wavefront takes the 64
// leaves of level L below a and their 30 rows below (level L+j of the block's outputs
// is one run of 64 2^j consecutive ranks, staged in LDS with row stride 2^j + 1
// against bank conflicts and written back coalesced); its second wavefront takes the
// 63 rows of a's subtree above level L (their outputs only), whose source rows are the
// leaves' ancestors, read again from the same CU's caches.  The other blocks take one
// row of level < L - 6 per thread.  Neighbouring nodes a share the cache lines at
// the ends of their rank runs (and their ancestors above level L - 6), so the deep
// blocks are spread over the XCDs in contiguous runs of a.

template <typename T, bool LOGV>
__global__ __launch_bounds__(kLast4Threads) void k_fwd_last4(int n, const T* __restrict__ src, size_t sstride,
                                                             T* __restrict__ dst, size_t dstride,
                                                             const State* st, const Consts* cs, int frz) {
  const int b = blockIdx.y;
  if (frz && st[b].converged) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int L = n - 4, La = L - 6;
  const uint32_t ndeep = 1u << La;
  const uint32_t t = threadIdx.x;
  T F4[30];
  if (blockIdx.x >= ndeep) {
    const uint32_t c = (blockIdx.x - ndeep) * kLast4Threads + t;
    if (c + 1u >= (1u << La)) return;
    T r = fwd4_thread<T>(src, 0, c, length_of_rank(c), 0u, F4);
    if constexpr (LOGV) r = log_weighted<T>(cs[b], c, r);
    dst[c] = r;
    return;
  }
  __shared__ T stage[kLast4Stage];
  // hardware block 8 k + x runs on XCD x: node k of XCD x's run of ndeep / 8
  const uint32_t da = (ndeep & 7u) ? blockIdx.x : (blockIdx.x & 7u) * (ndeep >> 3) + (blockIdx.x >> 3);
  const uint32_t a = ndeep - 1u + da;               // level La
  const uint32_t A0 = ((a + 1u) << 6) - 1u;         // its first leaf (level L)
  T* s1 = stage;
  T* s2 = s1 + 3 * 64;
  T* s3 = s2 + 5 * 64;
  T* s4 = s3 + 9 * 64;
  if (t < 64u) {
    const uint32_t y = A0 + t;
    const T va = fwd4_thread<T>(src, 0, y, L, 0u, F4);
    const T w0 = T(cs[b].w[L]), w1 = T(cs[b].w[L + 1]), w2 = T(cs[b].w[L + 2]), w3 = T(cs[b].w[L + 3]),
            w4 = T(cs[b].w[L + 4]);
    auto outv = [](T w, T r) -> T {
      if constexpr (LOGV) return wlog_t<T>(w, r);
      else return r;
    };
    dst[y] = outv(w0, va);
    // F4: depth d, index m at (1 << d) - 2 + m
#pragma unroll
    for (int q = 0; q < 2; ++q) s1[3u * t + q] = outv(w1, F4[q]);
#pragma unroll
    for (int q = 0; q < 4; ++q) s2[5u * t + q] = outv(w2, F4[2 + q]);
#pragma unroll
    for (int q = 0; q < 8; ++q) s3[9u * t + q] = outv(w3, F4[6 + q]);
#pragma unroll
    for (int q = 0; q < 16; ++q) s4[17u * t + q] = outv(w4, F4[14 + q]);
  } else if (t < 127u) {
    // node q of a's subtree above level L: depth d = log2(q + 1)
    const uint32_t q = t - 64u;
    const int d = length_of_rank(q);
    const uint32_t y = ((a + 1u) << d) - 1u + (q + 1u - (1u << d));
    T r = fwd4_thread<T>(src, 0, y, La + d, 0u, F4);
    if constexpr (LOGV) r = log_weighted<T>(cs[b], y, r);
    dst[y] = r;
  }
  __syncthreads();
#pragma unroll
  for (int j = 1; j <= 4; ++j) {
    const uint32_t wj = 1u << j, stride = wj + 1u;
    const T* sj = j == 1 ? s1 : j == 2 ? s2 : j == 3 ? s3 : s4;
    T* out = dst + (wj * (A0 + 1u) - 1u);
#pragma unroll
    for (uint32_t k = 0; k < wj / 2u; ++k) {
      const uint32_t e = k * kLast4Threads + t;
      out[e] = sj[(e >> j) * stride + (e & (wj - 1u))];
    }
  }
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
      const uint32_t xs[4] = {s, S + s, 2 * S + s, 3 * S + s};
      const Vec<T, V> gs[4] = {o00, o01, o10, o11};
      d_records<T, V, 4>(g, b, M, xs, gs, p);
    } else {
      T* op = dst + (r << (sh + 2)) + s;
      stv<T, V>(op, o00);
      stv<T, V>(op + S, o01);
      stv<T, V>(op + 2 * S, o10);
      stv<T, V>(op + 3 * S, o11);
    }
  }
  if constexpr (DP) {
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
// Loads of one (y, column s) of the four-position backward step: the 31 rows of
// y's depth-4 subtree, breadth-first (index t, children 2t+1 and 2t+2, as ranks).
template <typename T, int V>
__device__ __forceinline__ void bwd4_load(const T* __restrict__ src, int sh, uint32_t y, uint32_t s,
                                          Vec<T, V> (&S)[31]) {
#pragma unroll
  for (int d = 0; d <= 4; ++d)
#pragma unroll
    for (int m = 0; m < (1 << d); ++m)
      S[(1 << d) - 1 + m] = ld<T, V>(src + ((((y + 1u) << d) - 1u + uint32_t(m)) << sh) + s);
}

// The 4 single stages B_k[z][b g] = B_{k+1}[z][g] + B_{k+1}[z b][g] in registers:
// Dv[u] = B_i[y][u s].
template <typename T, int V>
__device__ __forceinline__ void bwd4_tree(const Vec<T, V> (&S)[31], Vec<T, V> (&Dv)[16]) {
  Vec<T, V> A[15][2];
#pragma unroll
  for (int t = 0; t < 15; ++t)
#pragma unroll
    for (int k = 0; k < V; ++k) {
      A[t][0].v[k] = S[t].v[k] + S[2 * t + 1].v[k];
      A[t][1].v[k] = S[t].v[k] + S[2 * t + 2].v[k];
    }
  Vec<T, V> B[7][4];
#pragma unroll
  for (int t = 0; t < 7; ++t)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int k = 0; k < V; ++k) B[t][bb * 2 + q].v[k] = A[t][q].v[k] + A[2 * t + 1 + bb][q].v[k];
  Vec<T, V> C[3][8];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < V; ++k) C[t][bb * 4 + q].v[k] = B[t][q].v[k] + B[2 * t + 1 + bb][q].v[k];
#pragma unroll
  for (int bb = 0; bb < 2; ++bb)
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int k = 0; k < V; ++k) Dv[bb * 8 + q].v[k] = C[0][q].v[k] + C[1 + bb][q].v[k];
}

// Row y of B_i at columns u S4 + s (u = 0..15); 16 consecutive values when S4 = 1.
template <typename T, int V>
__device__ __forceinline__ void bwd4_store(T* __restrict__ dst, int sh, uint32_t y, uint32_t s,
                                           const Vec<T, V> (&Dv)[16]) {
  T* op = dst + (y << (sh + 4)) + s;
  if (V == 1 && sh == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      Vec<T, 4> w;
#pragma unroll
      for (int k = 0; k < 4; ++k) w.v[k] = Dv[4 * q + k].v[0];
      stv<T, 4>(op + 4 * q, w);
    }
  } else {
#pragma unroll
    for (int u = 0; u < 16; ++u) stv<T, V>(op + (uint32_t(u) << sh), Dv[u]);
  }
}

template <typename T, int V, bool DP>
__global__ __launch_bounds__(kBlock) void k_bwd_stage4(int n, int i, const T* __restrict__ src, size_t sstride,
                                                       T* __restrict__ dst, size_t dstride, Group<T> g, Order o) {
  const int b = blockIdx.y;
  if (g.frz && g.st[b].converged) return;
  uint32_t y, chunk;
  const bool valid = order_slot(o, y, chunk);
  if (!DP && !valid) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh = n - i - 4;                  // log2 of the source width S4
  const uint32_t s = chunk * V;
  Part p = part_empty();
  if (valid) {
    Vec<T, V> S[31], Dv[16];
    bwd4_load<T, V>(src, sh, y, s, S);
    bwd4_tree<T, V>(S, Dv);
    if constexpr (DP) {
      const double M = g.st[b].M;
      uint32_t xs[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) xs[u] = (uint32_t(u) << sh) + s;
      d_records<T, V, 16>(g, b, M, xs, Dv, p);
    } else {
      bwd4_store<T, V>(dst, sh, y, s, Dv);
    }
  }
  if constexpr (DP) {
    store_block_part(g.part + (size_t)b * g.ps, blockIdx.x, p);
  }
}

// Eight backward positions per launch (i .. i+7) as two four-position steps with
// the intermediate B_{i+4} kept in LDS.  A block takes NR roots y of one level
// (consecutive ranks) and C columns s of the source width S8 = 2^(n-i-8), with
// NR * C = P: it copies the depth-8 subtrees of its roots at its columns into LDS
// (depth k is one run of NR 2^k consecutive ranks), forms B_{i+4}[z][u2 S8 + s]
// for the 31 rows z of each root's depth-4 subtree (step 1: one thread per
// (root, z, column), as a four-position thread with y = z), then
// B_i[y][(16 u1 + u2) S8 + s] (step 2: one thread per (root, u2, column)), staged
// in LDS and written back.  Every value is the same sum, in the same order, as
// with two four-position launches.  k_bwd_stage8 takes the mixed shapes
// (1 < NR < P); the two extremes, one root or one column, which the widest and the
// narrowest rows use, are k_bwd_stage8_p with bank-conflict-free layouts.
template <typename T>
constexpr int stage8_tile() { return sizeof(T) == 4 ? 16 : 8; }

// Root groups of an eight-position launch at position i with 2^lr roots per group:
// the levels below lr hold one (partial) group each; the full groups form a binary
// tree (the group of roots g 2^lr .. of level lr + l is node g of level l, its
// children's roots are its roots' children's) that is visited as the top levels in
// rank order, then subtrees of up to kStage8TileH levels breadth-first (2^h slots
// each, one unused), so that groups whose subtrees overlap run close together.
constexpr int kStage8TileH = 5;

__host__ __device__ inline void stage8_tiling(int i, int lr, uint32_t& npart, int& levels, int& h, int& lb) {
  npart = uint32_t(lr < i + 1 ? lr : i + 1);
  levels = i + 1 - lr;  // levels of the group tree
  h = levels < kStage8TileH ? levels : kStage8TileH;
  lb = levels - h;
}

__host__ __device__ inline uint32_t stage8_slots(int i, int lr) {
  uint32_t npart;
  int levels, h, lb;
  stage8_tiling(i, lr, npart, levels, h, lb);
  return levels > 0 ? npart + ((1u << lb) - 1u) + ((1u << lb) << h) : npart;
}

__device__ __forceinline__ bool stage8_group(uint32_t q, int i, int lr, uint32_t& lev, uint32_t& g0) {
  uint32_t npart;
  int levels, h, lb;
  stage8_tiling(i, lr, npart, levels, h, lb);
  if (q < npart) {
    lev = q;
    g0 = 0;
    return true;
  }
  if (levels <= 0) return false;
  q -= npart;
  const uint32_t top = (1u << lb) - 1u;
  uint32_t l, g;
  if (q < top) {
    l = uint32_t(31 - __clz(q + 1u));
    g = q + 1u - (1u << l);
  } else {
    q -= top;
    const uint32_t t = q >> h, j = q & ((1u << h) - 1u);
    if (j == (1u << h) - 1u || t >= (1u << lb)) return false;
    const int k = 31 - __clz(j + 1u);
    l = uint32_t(lb + k);
    g = (t << k) + (j + 1u - (1u << k));
  }
  lev = l + uint32_t(lr);
  g0 = g << lr;
  return true;
}

template <typename T, int LC>
__global__ __launch_bounds__(32 * stage8_tile<T>()) void k_bwd_stage8(int n, int i, const T* __restrict__ src,
                                                                    size_t sstride, T* __restrict__ dst,
                                                                    size_t dstride, const State* st) {
  constexpr int P = stage8_tile<T>();
  constexpr int LP = P == 16 ? 4 : P == 8 ? 3 : 2;
  static_assert(LC >= 1 && LC < LP, "columns per block (one root or one column: k_bwd_stage8_p)");
  constexpr uint32_t C = 1u << LC;           // columns per block
  constexpr int LR = LP - LC;                // log2 of the roots per (full) block
  constexpr uint32_t kPitch = 16u * C + 1u;  // B_{i+4} values per (root, z), padded
  const int b = blockIdx.z;
  if (st[b].converged) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh = n - i - 8;                  // log2 of S8
  // logical block: (root group, column block), column blocks innermost, so that
  // neighbouring columns and subtree-related groups share an XCD's L2; with 8 or
  // more column blocks, XCD x (hardware block 8 k + x) takes its eighth of the
  // column blocks of every group, so that the overlapping subtrees of a root and
  // its descendants are all read through one L2
  const int lcb = sh - LC;
  uint32_t lin;
  if (lcb >= 3) {
    const uint32_t x = blockIdx.x & 7u, k = blockIdx.x >> 3;
    const int cl = lcb - 3;
    lin = ((k >> cl) << lcb) + (x << cl) + (k & ((1u << cl) - 1u));
  } else {
    lin = logical_block();
  }
  uint32_t lev, g0;
  if (!stage8_group(lin >> lcb, i, LR, lev, g0)) return;
  const int lnr = int(lev) < LR ? int(lev) : LR;  // log2 of the roots of this block
  const uint32_t nr = 1u << lnr;
  const uint32_t r0 = (1u << lev) - 1u + g0;     // rank of the first root
  const uint32_t s0 = (lin & ((1u << lcb) - 1u)) * C;
  const uint32_t t = threadIdx.x;
  // one LDS buffer, used three times: the input subtrees [root][node q][column]
  // (511 C per root), then B_{i+4} as [root][z][u2][column] (kPitch per (root, z)),
  // then the outputs [root][u][column].  Lanes take consecutive columns, then
  // consecutive roots (odd strides 511 C and 31 kPitch), so reads of the same node
  // across lanes fall on distinct banks.
  constexpr uint32_t kIn = uint32_t(P) * 511u, kMid = 31u * (uint32_t(P) >> LC) * kPitch;
  __shared__ __attribute__((aligned(16))) T buf[kIn > kMid ? kIn : kMid];
  // copy-in: depth k of the roots' subtrees is one run of nr 2^k consecutive ranks;
  // every load of a thread is issued before its LDS stores
  if (LC == 0 && nr == uint32_t(P)) {
    // P roots, one column: depth k is a run of P 2^k consecutive ranks; the runs of
    // depth 5..8 hold 32 P 2^(k-5) values, i.e. 2^(k-5) per thread, and depths 0..4
    // together 31 P values, one per thread for the first 31 P threads
    constexpr uint32_t NT = 32u * P;
    T v[16];
    uint32_t li[16];
    {
      const uint32_t f = t;  // depths 0..4: f = P (2^k - 1) + m
      const int k = 31 - __clz((f >> LP) + 1u);
      const uint32_t m = f - ((1u << k) - 1u) * uint32_t(P);
      li[0] = ~0u;
      if (f < 31u * P) {
        v[0] = src[((r0 + 1u) << k) - 1u + m];
        li[0] = (m >> k) * 511u + (1u << k) - 1u + (m & ((1u << k) - 1u));
      }
    }
#pragma unroll
    for (int k = 5; k <= 8; ++k) {
      const uint32_t base = ((r0 + 1u) << k) - 1u;
#pragma unroll
      for (int j = 0; j < (1 << (k - 5)); ++j) {
        const uint32_t m = t + uint32_t(j) * NT;
        const int sl = (1 << (k - 5)) + j;  // 1, 2-3, 4-7, 8-15
        v[sl] = src[base + m];
        li[sl] = (m >> k) * 511u + (1u << k) - 1u + (m & ((1u << k) - 1u));
      }
    }
#pragma unroll
    for (int j = 0; j < 16; ++j)
      if (li[j] != ~0u) buf[li[j]] = v[j];
  } else {
    constexpr int kPer = (P * 511 + 32 * P - 1) / (32 * P);
    const int lrc = lnr + LC;
    const uint32_t total = (nr * 511u) << LC;
    T v[kPer];
    uint32_t li[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const uint32_t f = t + uint32_t(j) * (32u * P);
      li[j] = ~0u;
      if (f < total) {
        const int k = 31 - __clz((f >> lrc) + 1u);
        const uint32_t w = f - (((1u << k) - 1u) << lrc);
        const uint32_t m = w >> LC, c = w & (C - 1u);
        const uint32_t rho = m >> k, q = (1u << k) - 1u + (m & ((1u << k) - 1u));
        v[j] = src[((size_t)(((r0 + 1u) << k) - 1u + m) << sh) + s0 + c];
        li[j] = ((rho * 511u + q) << LC) + c;
      }
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j)
      if (li[j] != ~0u) buf[li[j]] = v[j];
  }
  __syncthreads();
  // step 1: thread (z = node e1 of root rho1's depth-4 subtree, column c1)
  Vec<T, 1> Dv[16];
  const bool s1 = t < ((31u * nr) << LC);
  const uint32_t c1 = t & (C - 1u), rest1 = t >> LC;
  const uint32_t rho1 = rest1 & (nr - 1u), e1 = rest1 >> lnr;
  if (s1) {
    // node e1's descendant (depth d, index m) is node ((e1 + 1) << d) + m - 1
    Vec<T, 1> S[31];
#pragma unroll
    for (int d = 0; d <= 4; ++d) {
      const T* row = buf + ((rho1 * 511u + ((e1 + 1u) << d) - 1u) << LC) + c1;
#pragma unroll
      for (int m = 0; m < (1 << d); ++m) S[(1 << d) - 1 + m].v[0] = row[uint32_t(m) << LC];
    }
    bwd4_tree<T, 1>(S, Dv);
  }
  __syncthreads();
  if (s1) {
    T* mp = buf + (rho1 * 31u + e1) * kPitch + c1;
#pragma unroll
    for (int u = 0; u < 16; ++u) mp[uint32_t(u) << LC] = Dv[u].v[0];
  }
  __syncthreads();
  // step 2: thread (root rho2, u2, column c2)
  const bool s2 = t < ((16u * nr) << LC);
  const uint32_t c2 = t & (C - 1u), rest2 = t >> LC;
  const uint32_t u2 = rest2 & 15u, rho2 = rest2 >> 4;
  if (s2) {
    Vec<T, 1> S[31];
    const T* mp = buf + rho2 * 31u * kPitch + (u2 << LC) + c2;
#pragma unroll
    for (int e = 0; e < 31; ++e) S[e].v[0] = mp[uint32_t(e) * kPitch];
    bwd4_tree<T, 1>(S, Dv);
  }
  __syncthreads();
  if (s2) {
    T* op = buf + ((rho2 * 256u + u2) << LC) + c2;
#pragma unroll
    for (int u = 0; u < 16; ++u) op[(uint32_t(u) * 16u) << LC] = Dv[u].v[0];
  }
  __syncthreads();
  if (LC == 0 && nr == uint32_t(P)) {
    // the P output rows of 256 values are consecutive: one contiguous block
    constexpr int VW = 16 / int(sizeof(T));
    T* o = dst + ((size_t)r0 << 8);
#pragma unroll
    for (uint32_t j = 0; j < (P * 256u) / (VW * 32u * P); ++j) {
      const uint32_t e = (t + j * 32u * P) * VW;
      stv<T, VW>(o + e, ld<T, VW>(buf + e));
    }
    return;
  }
  const uint32_t cnt = (nr * 256u) << LC;
  for (uint32_t e = t; e < cnt; e += 32u * P) {
    const uint32_t c = e & (C - 1u), rest = e >> LC;
    const uint32_t u = rest & 255u, rho = rest >> 8;
    dst[((size_t)(r0 + rho) << (sh + 8)) + (u << sh) + s0 + c] = buf[e];
  }
}

// Eight backward positions with P independent lanes of values per subtree node:
// one root and P columns (ROOTS = false, rows at least 16 P wide), or P roots of
// one level (consecutive ranks) and one column (ROOTS = true, rows of width 1; fewer
// roots on the levels above log2 P, the other lanes idle).  The steps are those of
// k_bwd_stage8, with LDS layouts free of bank conflicts: every node keeps its P
// values as one 64-byte row.  Per step-1 load a wavefront reads one subtree node of
// 4 (FP32; 8 in two halves for FP64) consecutive nodes z, i.e. nodes a 2^d + m for
// an aligned quad of 1-based heap indices a; with node rows at slot q every such
// load would hit one group of 16 banks for d >= 2.  Node q (1-based heap index in
// the depth-8 subtree) is therefore kept at slot sigma(q), whose low two bits are the
// parities of q's bits and of its odd-position bits: for every d these differ across
// an aligned quad of a (and the first parity across an aligned pair), so the four
// rows fall on distinct bank groups.  B_{i+4} is kept as [z][u][lane] with the 16 u
// rows of node z (1-based) permuted by u ^ (z mod 4), so that both its writers (4
// consecutive z) and its readers (4 consecutive u) cover 4 bank groups.  With
// roots, the copy-in writes 64 consecutive nodes of one root per wavefront, so root
// rho of node q sits at lane position rho ^ (q / 4 mod P) of the row.  The outputs
// are [u][column] (columns), or [root][u] with a row pitch of 260 (roots: lanes of
// one u-quad and 16 roots on 64 distinct banks), and leave through 16-byte vectors.
// kS8SymRoots: the first backward launch of the complement-symmetric iteration
// (i = n - 8), from the compact v: the roots are the rows starting with 0 (the
// subtree of "0", grouped as for kS8Roots over its levels) and, in one extra block,
// the empty row; root w writes its columns u < 128 to row w and its columns
// u >= 128, reversed, to row cpl w of the canonical-half B_i (row width 128).
// kS8ColumnsD: kS8Columns at i = 0 (the one root is the empty row, B_0 = G) with
// D(x) = H(x) - G(x) - M and the block's record formed instead of writing G; the
// record index is the block's column block.
// kS8ColumnsDU (FP32, eta = 1): kS8ColumnsD without the record, the D launch of an
// iteration fused with the next iteration's update and first eight forward positions
// on the same inputs: a = log p + D, the new iterate log p <- max(a - m', -floor),
// p = e^{log p} into LDS at G's slots, the block's max of a (for the next such launch),
// then first8_steps from p to F_8 (dst).  m' is the max of a of the iteration before
// (the block maxima that launch left, each wave taking their max itself), or 0: a is
// the same for any scale of p (D falls by what log p gains), and for the law it
// represents a <= 0 (D(x) <= -log p(x)) with max a >= -n ln 2, so either shift leaves
// the new log p at most n ln 2 above 0.  The shift only moves the floor, by m' - max
// a, which vanishes as the iteration converges.
// kS8ColumnsDH, kS8ColumnsDUH: kS8ColumnsD and kS8ColumnsDU for a complement-symmetric
// iterate (Group::half): B_i keeps the rows that start with 0 and the empty row, so a
// row that starts with 1 is read from its complement's row at the complementary
// columns, reversed; only the column blocks whose first bit is 0 run (x and cpl x
// then cover every input once), each record counts its inputs twice, and log p + D,
// log p and F_8 are written at x and at cpl x (F_8 at the rows that start with 0).
enum Stage8Mode {
  kS8Columns = 0, kS8Roots = 1, kS8SymRoots = 2, kS8ColumnsD = 3, kS8ColumnsDU = 4, kS8ColumnsDH = 5,
  kS8ColumnsDUH = 6
};

// The fused update of kS8ColumnsDU: the maxima it reads (nprev of them; nullptr: shift
// 0) and writes, and the floor.
struct S8Update {
  const float* mprev;  // per instance, at stride ps doubles
  float* mout;
  float floor;
  int nprev;
};

__host__ __device__ constexpr uint32_t stage8_sigma_bits(uint32_t q) {
  return ((uint32_t(__builtin_popcount(q & 0xAAAAAAAAu)) & 1u) << 1) | (uint32_t(__builtin_popcount(q)) & 1u);
}

// PT: value lanes per node (columns per block in the column modes), 0 for the
// precision's default (stage8_tile); the fused update of the half plan takes 8.
template <typename T, int MODE, int PT = 0>
__global__ __launch_bounds__(32 * (PT ? PT : stage8_tile<T>())) void k_bwd_stage8_p(
    int n, int i, const T* __restrict__ src, size_t sstride, T* __restrict__ dst, size_t dstride, const State* st,
    int frz, Group<T> g, S8Update fu) {
  constexpr bool ROOTS = MODE == kS8Roots || MODE == kS8SymRoots, SYM = MODE == kS8SymRoots;
  constexpr bool DU = MODE == kS8ColumnsDU || MODE == kS8ColumnsDUH;
  constexpr bool HC = MODE == kS8ColumnsDH || MODE == kS8ColumnsDUH;  // complement half
  constexpr bool DP = MODE == kS8ColumnsD || MODE == kS8ColumnsDH || DU;
  static_assert(!(DU || HC) || sizeof(T) == 4, "the fused update and the half plan are for FP32 iterates");
  constexpr uint32_t P = uint32_t(PT ? PT : stage8_tile<T>());  // value lanes per node
  constexpr int LP = P == 16 ? 4 : 3;
  constexpr uint32_t NT = 32u * P;                     // threads
  constexpr int VW = int(P) / 4;                       // P / VW = 4 vectors per node row
  static_assert(PT == 0 || MODE == kS8ColumnsDUH, "other tiles only for the half plan's fused update");
  constexpr uint32_t kOutPitch = 260u;                 // ROOTS: output row pitch
  const int b = blockIdx.z;
  if ((DU || frz) && st[b].converged) return;  // DU writes log p: frozen instances always stay
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh = n - i - 8;                  // log2 of S8 (0 for ROOTS)
  // logical block (root group, column block), column blocks innermost; with 8 or
  // more column blocks XCD x takes its eighth of the column blocks of every root
  const int lcb = ROOTS ? 0 : sh - LP - (HC ? 1 : 0);
  uint32_t lin = 0;
  if constexpr (ROOTS) {
    lin = logical_block();
  } else if (lcb >= 3) {
    const uint32_t x = blockIdx.x & 7u, k = blockIdx.x >> 3;
    const int cl = lcb - 3;
    lin = ((k >> cl) << lcb) + (x << cl) + (k & ((1u << cl) - 1u));
  } else {
    lin = logical_block();
  }
  uint32_t lev, g0;
  int lnr;                                   // log2 of the roots
  if constexpr (SYM) {
    // groups of the subtree of "0" (its level l is level l + 1), then the empty row
    const uint32_t nslot = stage8_slots(i - 1, LP);
    if (lin == nslot) {
      lev = 0;
      g0 = 0;
      lnr = 0;
    } else {
      if (lin > nslot || !stage8_group(lin, i - 1, LP, lev, g0)) return;
      lnr = int(lev) < LP ? int(lev) : LP;
      ++lev;
    }
  } else {
    if (!stage8_group(lin >> lcb, i, ROOTS ? LP : 0, lev, g0)) return;
    lnr = ROOTS ? (int(lev) < LP ? int(lev) : LP) : 0;
  }
  const uint32_t nr = 1u << lnr;
  const uint32_t r0 = (1u << lev) - 1u + g0;  // rank of the first root
  const uint32_t s0 = (lin & ((1u << lcb) - 1u)) * P;
  const uint32_t t = threadIdx.x;
  // DU: the buffer also holds first8_steps' F_4
  __shared__ __attribute__((aligned(16))) T buf[DU ? 31u * f4_pitch<int(P)>() : 512u * P];
  if constexpr (ROOTS) {
    // copy-in: depth k of the roots' subtrees is one run of nr 2^k consecutive ranks;
    // value m of the run is root m >> k, node 2^k + (m mod 2^k).  Full groups: the
    // runs of depth 5..8 hold NT 2^(k-5) values (2^(k-5) per thread), depths 0..4
    // together 31 P (one per thread of the first 31 P)
    auto lds_index = [](int k, uint32_t m) -> uint32_t {
      const uint32_t q = (1u << k) + (m & ((1u << k) - 1u)), rho = m >> k;
      return (((q & ~3u) | stage8_sigma_bits(q)) << LP) + (rho ^ ((q >> 2) & (P - 1u)));
    };
    if (nr == P) {
      T v[16];
      uint32_t li[16];
      {
        const int k = 31 - __clz((t >> LP) + 1u);
        const uint32_t m = t - ((1u << k) - 1u) * P;
        li[0] = ~0u;
        if (t < 31u * P) {
          const uint32_t rank = ((r0 + 1u) << k) - 1u + m;
          v[0] = src[SYM ? compact_rank(rank) : rank];
          li[0] = lds_index(k, m);
        }
      }
#pragma unroll
      for (int k = 5; k <= 8; ++k) {
        // SYM: rows of length lev + k starting with 0 sit at rank - 2^(lev + k - 1) + 1
        const uint32_t base = SYM ? ((r0 + 1u) << k) - (1u << (int(lev) + k - 1)) : ((r0 + 1u) << k) - 1u;
#pragma unroll
        for (int j = 0; j < (1 << (k - 5)); ++j) {
          const uint32_t m = t + uint32_t(j) * NT;
          const int sl = (1 << (k - 5)) + j;  // 1, 2-3, 4-7, 8-15
          v[sl] = src[base + m];
          li[sl] = lds_index(k, m);
        }
      }
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (li[j] != ~0u) buf[li[j]] = v[j];
    } else {
      for (uint32_t f = t; f < nr * 511u; f += NT) {
        const int k = 31 - __clz((f >> lnr) + 1u);
        const uint32_t m = f - (((1u << k) - 1u) << lnr);
        const uint32_t rank = ((r0 + 1u) << k) - 1u + m;
        buf[lds_index(k, m)] = src[SYM ? compact_rank(rank) : rank];
      }
    }
  } else {
    // copy-in: vector j of node q = f / 4 + 1 for f = t + k NT
    constexpr int kPer = int((511u * 4u + NT - 1u) / NT);
    Vec<T, VW> v[kPer];
    uint32_t li[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t f = t + uint32_t(k) * NT;
      const uint32_t q = (f >> 2) + 1u, j = f & 3u;
      li[k] = ~0u;
      if (q < 512u) {
        const int dq = 31 - __clz(q);
        const uint32_t m = q - (1u << dq);
        const uint32_t rank = ((r0 + 1u) << dq) - 1u + m;
        if (HC && dq > 0 && m >= (1u << (dq - 1))) {
          // a row that starts with 1 (the root is the empty row): its complement's row
          // (mirrored within the level) at the complementary columns, reversed
          const uint32_t mr = (1u << dq) - 1u + ((1u << dq) - 1u - m);
          const Vec<T, VW> w = ld<T, VW>(src + ((size_t)mr << sh) + ((1u << sh) - uint32_t(VW) - s0 - j * uint32_t(VW)));
#pragma unroll
          for (int e = 0; e < VW; ++e) v[k].v[e] = w.v[VW - 1 - e];
        } else {
          v[k] = ld<T, VW>(src + ((size_t)rank << sh) + s0 + j * uint32_t(VW));
        }
        li[k] = (((q & ~3u) | stage8_sigma_bits(q)) << LP) + j * uint32_t(VW);
      }
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k)
      if (li[k] != ~0u) stv<T, VW>(buf + li[k], v[k]);
  }
  // DP: the inputs x = w S8 + s0 + (vector j) of output column group w = f / 4 of
  // 256, vector j = f mod 4; their H and log p are loaded now and held through the
  // two steps (DU without HC forms D from step 2's registers instead, below)
  constexpr int KD = int((256u * 4u) / NT);
  uint32_t xs[KD];
  Vec<T, VW> hd[KD], lq[KD];
  if constexpr (DP) {
#pragma unroll
    for (int k = 0; k < KD; ++k) {
      const uint32_t f = t + uint32_t(k) * NT;
      xs[k] = ((f >> 2) << sh) + s0 + (f & 3u) * uint32_t(VW);
    }
    if constexpr (!(DU && !HC)) d_loads<T, VW, KD>(g, b, xs, hd, lq);
  }
  // DU: the shift m' from the previous launch's block maxima (every wave reduces them)
  float mprev = 0.0f;
  if constexpr (DU) {
    if (fu.mprev) {
      const float* bm = fu.mprev + (size_t)b * g.ps * 2u;
      mprev = -INFINITY;
      for (uint32_t j = t & (kWave - 1u); j < uint32_t(fu.nprev); j += kWave) mprev = fmaxf(mprev, bm[j]);
#pragma unroll
      for (int off = kWave / 2; off > 0; off >>= 1) mprev = fmaxf(mprev, __shfl_xor(mprev, off));
      if (!isfinite(mprev)) {
        if (lin == 0u && t == 0u) {
          g.st[b].bad = 1;
          g.st[b].converged = 1;
        }
        return;  // the whole block (mprev is the same in every wave)
      }
    }
  }
  __syncthreads();
  // step 1: thread (z = 1-based node a of the depth-4 subtree, lane c1); a = 0 idles
  Vec<T, 1> Dv[16];
  const uint32_t c1 = t & (P - 1u), a = t >> LP;
  if (a != 0u) {
    // node a 2^d + m (disjoint bits) sits at slot (a 2^d & ~3) + (m & ~3) +
    // (sigma bits of a 2^d xor those of m): four base addresses per depth, the rest
    // immediate offsets
    // (roots: lane position c1 ^ (q / 4 mod P), q / 4 = a 2^d / 4 xor m / 4)
    Vec<T, 1> S[31];
#pragma unroll
    for (int d = 0; d <= 4; ++d) {
      const uint32_t ad = a << d, fa = stage8_sigma_bits(ad);
      uint32_t base[4];
#pragma unroll
      for (uint32_t k = 0; k < 4u; ++k) base[k] = ((ad & ~3u) + (fa ^ k)) << LP;
      const uint32_t cx = ROOTS ? c1 ^ ((ad >> 2) & (P - 1u)) : c1;
#pragma unroll
      for (int m = 0; m < (1 << d); ++m) {
        const uint32_t lane = ROOTS ? cx ^ ((uint32_t(m) >> 2) & (P - 1u)) : cx;
        S[(1 << d) - 1 + m].v[0] = buf[base[stage8_sigma_bits(uint32_t(m))] + ((uint32_t(m) & ~3u) << LP) + lane];
      }
    }
    bwd4_tree<T, 1>(S, Dv);
  }
  __syncthreads();
  if (a != 0u) {
    uint32_t base[4];
#pragma unroll
    for (uint32_t k = 0; k < 4u; ++k) base[k] = (a << (4 + LP)) + ((k ^ (a & 3u)) << LP) + c1;
#pragma unroll
    for (int u = 0; u < 16; ++u) buf[base[u & 3] + ((uint32_t(u) & ~3u) << LP)] = Dv[u].v[0];
  }
  __syncthreads();
  // step 2: thread (u2, lane c2), u2 < 16
  const uint32_t c2 = t & (P - 1u), u2 = t >> LP;
  if (u2 < 16u) {
    uint32_t base[4];
#pragma unroll
    for (uint32_t k = 0; k < 4u; ++k) base[k] = ((u2 ^ k) << LP) + c2;
    Vec<T, 1> S[31];
#pragma unroll
    for (int e = 1; e <= 31; ++e) S[e - 1].v[0] = buf[base[e & 3] + (uint32_t(e) << (4 + LP))];
    bwd4_tree<T, 1>(S, Dv);
  }
  __syncthreads();
  if constexpr (DU && !HC) {
    // thread (u2, c2) holds G at the inputs x = u1 2^(n-4) + u2 2^(n-8) + s0 + c2,
    // u1 < 16, which are the inputs first8_steps takes from thread u2 P + c2: a = log
    // p + D, the new log p = max(a - m', -floor) and p = e^{log p} stay in registers
    // (H and log p loaded eight inputs at a time; no pass of G and p through LDS),
    // and the block's max of a goes to its maxima set.  (The half plan's 8-column
    // tiles keep the vector mapping of the branch below, which spreads the D work
    // over twice the threads and measured faster there.)
    const double M = g.st[b].M;
    float* lp = g.lp + (size_t)b * g.xs;
    const float* hf = g.hf + (size_t)b * g.xs;
    const float lo = -fu.floor;
    float am = -INFINITY;
    float R[16];
    if (u2 < 16u) {
      const uint32_t x0 = (u2 << (n - 8)) + s0 + c2;
#pragma unroll
      for (int h = 0; h < 16; h += 8) {
        float hv[8], lv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          hv[u] = hf[x0 + (uint32_t(h + u) << (n - 4))];
          lv[u] = lp[x0 + (uint32_t(h + u) << (n - 4))];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const uint32_t x = x0 + (uint32_t(h + u) << (n - 4));
          const float d = hv[u] - Dv[h + u].v[0] - float(M);
          const float a = lv[u] + d;
          am = fmaxf(am, a);
          const float y = a - mprev;
          const float nl = y > lo ? y : lo;
          lp[x] = nl;
          R[h + u] = exp_t<float>(nl);
        }
      }
    }
    // the block's max of a: waves, then the first wave over their maxima
    __shared__ float wmax[NT / kWave];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) am = fmaxf(am, __shfl_xor(am, off));
    if ((t & (kWave - 1u)) == 0u) wmax[t / kWave] = am;
    __syncthreads();
    if (t == 0u) {
      float m = wmax[0];
#pragma unroll
      for (uint32_t w = 1; w < NT / kWave; ++w) m = fmaxf(m, wmax[w]);
      fu.mout[(size_t)b * g.ps * 2u + (lin & ((1u << lcb) - 1u))] = m;
      if (lin == 0u) g.st[b].iters += 1;
    }
    first8_steps<float, false, int(P)>(buf, R, t, dst, n, s0);
    return;
  }
  if (u2 < 16u) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      if constexpr (ROOTS) buf[c2 * kOutPitch + uint32_t(u) * 16u + u2] = Dv[u].v[0];
      else buf[((uint32_t(u) * 16u + u2) << LP) + c2] = Dv[u].v[0];
    }
  }
  __syncthreads();
  if constexpr (SYM) {
    // copy-out: row w = r0 + rho takes columns 0..127; row cpl w (rank m0 - rho,
    // m0 = mirror of r0) takes 255 - c for its column c, except for the empty row
    const uint32_t m0 = r0 == 0u ? 0u : mirror_rank(r0);
#pragma unroll
    for (uint32_t k = 0; k < (P * 64u) / NT; ++k) {
      const uint32_t f = t + k * NT;
      const uint32_t rho = f >> 6, j = f & 31u;
      if (rho >= nr) continue;
      if ((f & 32u) == 0u) {
        stv<T, 4>(dst + ((size_t)(r0 + rho) << 7) + 4u * j, ld<T, 4>(buf + rho * kOutPitch + 4u * j));
      } else if (r0 != 0u) {
        const Vec<T, 4> w = ld<T, 4>(buf + rho * kOutPitch + 252u - 4u * j);
        Vec<T, 4> rv;
#pragma unroll
        for (int e = 0; e < 4; ++e) rv.v[e] = w.v[3 - e];
        stv<T, 4>(dst + ((size_t)(m0 - rho) << 7) + 4u * j, rv);
      }
    }
  } else if constexpr (ROOTS) {
    // copy-out: the nr output rows of 256 values are consecutive
    T* o = dst + ((size_t)r0 << 8);
#pragma unroll
    for (uint32_t k = 0; k < (P * 64u) / NT; ++k) {
      const uint32_t f = t + k * NT;
      const uint32_t rho = f >> 6, j = f & 63u;
      if (rho < nr) stv<T, 4>(o + (rho << 8) + 4u * j, ld<T, 4>(buf + rho * kOutPitch + 4u * j));
    }
  } else if constexpr (DU && HC) {
    // a = log p + D at the inputs xs (G of column group w, vector j), the new log p and
    // p = e^{log p}, which replaces G at the same slots (each thread reads and writes
    // only its own); with w = u1 16 + u2 and the block's 16 columns, p(x) of input
    // u1 2^(n-4) + u2 2^(n-8) + s0 + c1 sits at u1 256 + u2 16 + c1 as first8_steps wants
    const double M = g.st[b].M;
    float* lp = g.lp + (size_t)b * g.xs;
    const float lo = -fu.floor;
    float am = -INFINITY;
#pragma unroll
    for (int k = 0; k < KD; ++k) {
      const uint32_t f = t + uint32_t(k) * NT;
      float* slot = buf + ((f >> 2) << LP) + (f & 3u) * uint32_t(VW);
      const Vec<float, VW> gv = ld<float, VW>(slot);
      Vec<float, VW> nl, pv;
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        const float d = hd[k].v[e] - gv.v[e] - float(M);
        const float a = lq[k].v[e] + d;
        am = fmaxf(am, a);
        const float x = a - mprev;
        nl.v[e] = x > lo ? x : lo;
        pv.v[e] = exp_t<float>(nl.v[e]);
      }
      stv<float, VW>(lp + xs[k], nl);
      if constexpr (HC) {  // cpl x = 2^n - 1 - x
        Vec<float, VW> rv;
#pragma unroll
        for (int e = 0; e < VW; ++e) rv.v[e] = nl.v[VW - 1 - e];
        stv<float, VW>(lp + ((1u << n) - uint32_t(VW) - xs[k]), rv);
      }
      stv<float, VW>(slot, pv);
    }
    // the block's max of a: waves, then the first wave over their maxima
    __shared__ float wmax[NT / kWave];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) am = fmaxf(am, __shfl_xor(am, off));
    if ((t & (kWave - 1u)) == 0u) wmax[t / kWave] = am;
    __syncthreads();
    if (t == 0u) {
      float m = wmax[0];
#pragma unroll
      for (uint32_t w = 1; w < NT / kWave; ++w) m = fmaxf(m, wmax[w]);
      fu.mout[(size_t)b * g.ps * 2u + (lin & ((1u << lcb) - 1u))] = m;
      if (lin == 0u) g.st[b].iters += 1;
    }
    float R[16];
    if (t < 16u * P) {
#pragma unroll
      for (int u1 = 0; u1 < 16; ++u1) R[u1] = buf[uint32_t(u1) * 16u * P + t];
    }
    __syncthreads();
    first8_steps<float, HC, int(P)>(buf, R, t, dst, n, s0);
  } else if constexpr (DP && !DU) {
    // D at the inputs xs from G of column group w, vector j, and the block's record
    const double M = g.st[b].M;
    Vec<T, VW> gv[KD];
#pragma unroll
    for (int k = 0; k < KD; ++k) {
      const uint32_t f = t + uint32_t(k) * NT;
      gv[k] = ld<T, VW>(buf + ((f >> 2) << LP) + (f & 3u) * uint32_t(VW));
    }
    const int rec = int(lin & ((1u << lcb) - 1u));
    if constexpr (sizeof(T) == 4) {
      // FP32 iterates: the lanes' records reduced in single precision within each wave
      PartF q;
      d_records_pre_f(g, b, M, xs, gv, hd, lq, q, HC);
      double* part = g.part + (size_t)b * g.ps;
      store_block_part_f32<int(NT)>(part, rec, q, g.eta != 1.0, reinterpret_cast<float*>(part + kBlockMaxima));
    } else {
      Part p = part_empty();
      d_records_pre<T, VW, KD>(g, b, M, xs, gv, hd, lq, p);
      store_block_part_nt<int(NT)>(g.part + (size_t)b * g.ps, rec, p);
    }
  } else if constexpr (!DU) {
    // copy-out: output column group w = f / 4 of 256, vector j = f mod 4
    T* o = dst + ((size_t)r0 << (sh + 8)) + s0;
#pragma unroll
    for (uint32_t k = 0; k < (256u * 4u) / NT; ++k) {
      const uint32_t f = t + k * NT;
      const uint32_t w = f >> 2, j = f & 3u;
      stv<T, VW>(o + ((size_t)w << sh) + j * uint32_t(VW), ld<T, VW>(buf + (w << LP) + j * uint32_t(VW)));
    }
  }
}

// Twelve backward positions from v in one launch (i = n - 12 .. n - 1, for n =
// kStage12N, FP32), one root row y of B_i per block.  The depth-12 subtree of y in v
// (depth k is one run of 2^k consecutive ranks) is copied to LDS; three
// four-position steps then form B_{i+8} at the 511 nodes of depth <= 8 (16 columns
// each), B_{i+4} at the 31 nodes of depth <= 4 (256 columns) and the row B_i[y]
// (4096 columns), every value as bwd4_tree on 31 values: the same sums in the same
// order as three four-position launches.  Column u3 2^8 + u2 2^4 + u1 of B_i: u3
// holds the input bits of positions i .. i+3, u2 of i+4 .. i+7, u1 of i+8 .. i+11
// (the first one highest).
// Root order: XCD x (blockIdx.x mod 8) takes the roots in the subtree of node x of
// level 3, deepest level first, then root x of the 7 above level 3 (x < 7).  The
// subtrees of the roots an XCD takes lie in that node's eighth of v, except for
// those 7.
// LDS, 32 banks of 4 bytes, one padding word per 32: node q (1-based heap index in
// y's subtree) at stage12_slot(q) = q + q / 32.  For 32 consecutive nodes a of one
// level (32-aligned) and any descendant offset (d <= 4, m < 2^d) the slots of
// a 2^d + m are distinct mod 32, and slot(a 2^d + m) = slot(a 2^d) + m, so a step
// reads its 31 values at five per-thread bases plus instruction offsets.  B_{i+8} as
// [column][node] with the same slots (column pitch kS12P1); B_{i+4} as [node z]
// [column] with the odd pitch kS12P2 (written by 32 nodes z at one column, read at
// consecutive columns of one node).  (A block taking two roots, with the second
// one's loads in flight through the first one's steps, ran at three blocks per CU
// instead of four and was slower: 16.6 against 15.6 us at n = 20, 3 x FP32.)
constexpr int kStage12N = 20;
constexpr uint32_t kStage12Threads = 512;
constexpr uint32_t kS12Words = 8192u + 256u;      // LDS words: 8192 slots and their padding
constexpr uint32_t kS12P1 = 512u + 16u, kS12P2 = 257u;

__device__ __forceinline__ uint32_t stage12_slot(uint32_t q) { return q + (q >> 5); }

// HALF (complement-symmetric iterate, the twelve-position plan): v holds the rows that
// start with 0 (and the empty row), B_i is formed for those roots only (256 blocks);
// the empty root reads a row that starts with 1 at its complement, whose rank mirrors
// it within its level (the run of a level reversed).
template <bool HALF>
__global__ __launch_bounds__(kStage12Threads) __attribute__((amdgpu_waves_per_eu(8))) void k_bwd_stage12(
    int n, const float* __restrict__ src, size_t sstride, float* __restrict__ dst, size_t dstride, const State* st,
    int frz) {
  using T = float;
  const int b = blockIdx.y;
  if (frz && st[b].converged) return;
  const int i = n - 12;
  const uint32_t x = blockIdx.x & 7u, k = blockIdx.x >> 3;
  uint32_t root;
  if constexpr (HALF) {
    // slot k of XCD x: the 2^(L+1) - 1 roots of the subtree of level-4 node 0x (x as
    // three bits; L = i - 4 levels below it), deepest level first, then top root x of
    // the 8 above level 4 that are empty or start with 0 (ranks 0, 1, 3, 4, 7 .. 10)
    const int L = i - 4;
    if (k + 1u == (2u << L)) {
      root = x < 2u ? x : (x < 4u ? x + 1u : x + 3u);
    } else {
      const uint32_t r = (2u << L) - 1u - k;  // 1 .. 2^(L+1) - 1
      const int l = 31 - __clz(r);            // level l below level 4
      root = ((16u + x) << l) - 1u + ((2u << l) - 1u - r);
    }
  } else {
    // slot k of XCD x: the 2^(L+1) - 1 roots of level-3 node x's subtree (L = i - 3
    // levels below it), deepest level first, then top root x
    const int L = i - 3;
    if (k + 1u == (2u << L)) {
      if (x >= 7u) return;
      root = x;
    } else {
      const uint32_t r = (2u << L) - 1u - k;  // 1 .. 2^(L+1) - 1
      const int l = 31 - __clz(r);            // level l below level 3
      root = ((8u + x) << l) - 1u + ((2u << l) - 1u - r);
    }
  }
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  __shared__ __attribute__((aligned(16))) T buf[kS12Words];
  const uint32_t t = threadIdx.x;
  {
    // copy-in, every load of a thread before its LDS stores: depths 0..8 one node
    // q = t + 1 per thread, depth k >= 9 2^(k-9) values t + 512 j, whose slots are
    // (1 << k) + (1 << (k - 5)) + 528 j + slot(t)
    T v[16];
    const uint32_t q = t + 1u;
    const int kq = 31 - __clz(q);
    if (HALF && root == 0u) {
      // element m of level k: m or, from 2^(k-1) on (a row starting with 1), 2^k - 1 - m
      if (q < 512u) {
        const uint32_t m = q - (1u << kq);
        const uint32_t mm = (kq > 0 && m >= (1u << (kq - 1))) ? (1u << kq) - 1u - m : m;
        v[0] = src[(1u << kq) - 1u + mm];
      }
#pragma unroll
      for (int kk = 9; kk <= 12; ++kk) {
        const T* base = src + ((1u << kk) - 1u);
#pragma unroll
        for (int j = 0; j < (1 << (kk - 9)); ++j) {
          const uint32_t m = t + uint32_t(j) * kStage12Threads;
          v[(1 << (kk - 9)) + j] = base[m >= (1u << (kk - 1)) ? (1u << kk) - 1u - m : m];
        }
      }
    } else {
      if (q < 512u) v[0] = src[((root + 1u) << kq) - 1u + (q - (1u << kq))];
#pragma unroll
      for (int kk = 9; kk <= 12; ++kk) {
        const T* base = src + (((root + 1u) << kk) - 1u);
#pragma unroll
        for (int j = 0; j < (1 << (kk - 9)); ++j) v[(1 << (kk - 9)) + j] = base[t + uint32_t(j) * kStage12Threads];
      }
    }
    if (q < 512u) buf[stage12_slot(q)] = v[0];
    const uint32_t st0 = stage12_slot(t);
#pragma unroll
    for (int kk = 9; kk <= 12; ++kk)
#pragma unroll
      for (int j = 0; j < (1 << (kk - 9)); ++j)
        buf[st0 + (1u << kk) + (1u << (kk - 5)) + uint32_t(j) * 528u] = v[(1 << (kk - 9)) + j];
  }
  __syncthreads();
  // step 1: thread a = node of depth <= 8 (a = 0 idles): B_{i+8}[a][u1]
  Vec<T, 1> Dv[16];
  const uint32_t a = t;
  if (a != 0u) {
    Vec<T, 1> S[31];
#pragma unroll
    for (int d = 0; d <= 4; ++d) {
      const T* row = buf + stage12_slot(a << d);
#pragma unroll
      for (int m = 0; m < (1 << d); ++m) S[(1 << d) - 1 + m].v[0] = row[m];
    }
    bwd4_tree<T, 1>(S, Dv);
  }
  __syncthreads();
  if (a != 0u) {
    T* col = buf + stage12_slot(a);
#pragma unroll
    for (int u = 0; u < 16; ++u) col[uint32_t(u) * kS12P1] = Dv[u].v[0];
  }
  __syncthreads();
  // step 2: thread (column c = u1, node z of depth <= 4; z = 0 idles): B_{i+4}[z][u2 16 + c]
  const uint32_t c = t >> 5, z = t & 31u;
  if (z != 0u) {
    Vec<T, 1> S[31];
    const T* col = buf + c * kS12P1;
#pragma unroll
    for (int d = 0; d <= 4; ++d) {
      const T* row = col + stage12_slot(z << d);
#pragma unroll
      for (int m = 0; m < (1 << d); ++m) S[(1 << d) - 1 + m].v[0] = row[m];
    }
    bwd4_tree<T, 1>(S, Dv);
  }
  __syncthreads();
  if (z != 0u) {
    T* row = buf + z * kS12P2 + c;
#pragma unroll
    for (int u = 0; u < 16; ++u) row[uint32_t(u) * 16u] = Dv[u].v[0];
  }
  __syncthreads();
  // step 3: thread c2 < 256 (column u2 16 + u1): B_i[root][u3 256 + c2], written out
  if (t < 256u) {
    Vec<T, 1> S[31];
#pragma unroll
    for (int qq = 1; qq < 32; ++qq) S[qq - 1].v[0] = buf[uint32_t(qq) * kS12P2 + t];
    bwd4_tree<T, 1>(S, Dv);
    T* o = dst + ((size_t)root << 12) + t;
#pragma unroll
    for (int u = 0; u < 16; ++u) o[uint32_t(u) * 256u] = Dv[u].v[0];
  }
}

// Twelve forward positions in one launch (i = n - 12 .. n - 1 for n = kStage12N,
// FP32): F_i to r (LOGV: v = w_k log r), one block per leaf z of F_i (level i).
// The outputs in z's subtree (levels i .. n) depend on F_i of z and of its i
// ancestors A_1 .. A_i (A_k = k levels up), so each block recomputes that chain:
//   step 1, thread c2 < 256 (column u2 2^4 + u1 of F_{i+4}): F_{i+4} of the chain
//     from the root down (each row's four stages take the half of its parent's
//     values at the same stages that its last bit selects) and of the 30 rows below
//     z, the 16 column groups u3 of every row loaded from HBM or L2;
//   step 2, from those 40 rows (one all-zero row stands for the rows above the root):
//     thread (node q2 of depth 4 below z, u1) the four-position step of q2 with its
//     30 rows below, and items (row, u1) F_{i+8} of the 15 nodes of depth <= 3 below
//     z and of the chain rows A_1 .. A_{c+4} (c below);
//   step 3, from F_{i+8}: thread q3 (depth 8 below z) the step of q3 and its 30 rows
//     below, and items for the 255 nodes of depth <= 7 below z and for the chain rows
//     A_1 .. A_c, where c is the number of trailing zero bits of z (8 for the
//     first leaf): z is the first leaf below A_k exactly for k <= c, so every row above
//     level i is written by one block.
// Every value is the same sum in the same order as in k_fwd_stage4 and k_fwd_last4
// (each stage of a row adds its own two halves, then its parent's half), so the
// outputs equal those of the three launches bit for bit.  The subtree's outputs are
// staged in LDS at stage12_slot of their heap index below z and written as one run
// of ranks per level, as k_bwd_stage12 reads them.  Leaf order: XCD x (blockIdx.x mod
// 8) takes the run of 2^(i-3) leaves below node x of level 3, whose chains share
// their rows down to level 3 in that XCD's L2.
// LDS (one array, each step's output overwriting the previous step's input after a
// barrier): F_{i+4} as [row][c2] with pitch kF12P1 = 16 mod 32 (rows 1..31: heap index
// below z, 31 + k: A_k, 0: zeros), so that the two nodes of a half-wavefront read
// disjoint banks; F_{i+8} as [u1][stage12_slot(q)] with the odd pitch kF12P2 (q < 512
// below z, 511 + k: A_k, 0: zeros).
constexpr uint32_t kF12P1 = 256u + 16u;
constexpr uint32_t kF12P2 = 537u;
constexpr uint32_t kF12Words = 40u * kF12P1;
static_assert(kF12Words >= 16u * kF12P2 && kF12Words >= kS12Words, "step buffers fit the array");

// The four-position step of a row from LDS rows of its path P_0 .. P_4 (16 column
// groups at stride CS from each row pointer; rows above the root point at zeros), in
// rolling form: P_4 gives its F_i half, P_3 its F_{i+1}, P_2 up to F_{i+2}, P_1 up to
// F_{i+3}, each row adding to its own halves the half of its parent's values that
// its last bit selects (the sums of fwd4_thread, with fewer values live).  Returns
// F_{i+4}[P_0] and leaves P_0's F_i row (R) and its F_{i+1} .. F_{i+3} for
// fwd4_subtree.
template <typename T, uint32_t CS>
__device__ __forceinline__ T fwd4_roll(const T* const (&row)[5], const uint32_t (&lastb)[4], T (&R)[16],
                                       T (&F1)[8], T (&F2)[4], T (&F3)[2]) {
  T H0[8], H1[4], H2[2], H3 = T(0);
  {
    const T* h = row[4] + (lastb[3] ? 8u * CS : 0u);
#pragma unroll
    for (int g = 0; g < 8; ++g) H0[g] = h[uint32_t(g) * CS];
  }
#pragma unroll
  for (int j = 3; j >= 0; --j) {
#pragma unroll
    for (int u = 0; u < 16; ++u) R[u] = row[j][uint32_t(u) * CS];
#pragma unroll
    for (int g = 0; g < 8; ++g) F1[g] = (R[g] + R[8 + g]) + H0[g];
    if (j <= 2) {
#pragma unroll
      for (int g = 0; g < 4; ++g) F2[g] = (F1[g] + F1[4 + g]) + H1[g];
    }
    if (j <= 1) {
#pragma unroll
      for (int g = 0; g < 2; ++g) F3[g] = (F2[g] + F2[2 + g]) + H2[g];
    }
    if (j == 0) return (F3[0] + F3[1]) + H3;
    const bool lb = lastb[j - 1];
#pragma unroll
    for (int g = 0; g < 8; ++g) H0[g] = lb ? R[8 + g] : R[g];
#pragma unroll
    for (int g = 0; g < 4; ++g) H1[g] = lb ? F1[4 + g] : F1[g];
    if (j <= 2) {
#pragma unroll
      for (int g = 0; g < 2; ++g) H2[g] = lb ? F2[2 + g] : F2[g];
    }
    if (j <= 1) H3 = lb ? F3[1] : F3[0];
  }
  return T(0);  // not reached
}

// fwd4_roll with the 30 rows below P_0 (as fwd4_subtree).
template <typename T, uint32_t CS>
__device__ __forceinline__ T fwd4_roll_tree(const T* const (&row)[5], const uint32_t (&lastb)[4], T (&F4)[30]) {
  T R[16], F1[8], F2[4], F3[2], F1s[2][8];
  const T v = fwd4_roll<T, CS>(row, lastb, R, F1, F2, F3);
#pragma unroll
  for (int cc = 0; cc < 2; ++cc)
#pragma unroll
    for (int g = 0; g < 8; ++g) F1s[cc][g] = R[cc * 8 + g];
  fwd4_subtree<T>(F1, F2, F3, F1s, F4);
  return v;
}

// fwd4_roll for the row alone.
template <typename T, uint32_t CS>
__device__ __forceinline__ T fwd4_roll_row(const T* const (&row)[5], const uint32_t (&lastb)[4]) {
  T R[16], F1[8], F2[4], F3[2];
  return fwd4_roll<T, CS>(row, lastb, R, F1, F2, F3);
}

// Path of an item of steps 2 and 3 that is not a leaf step: node q (1..) below z at
// depth dq, or chain row A_k (q = 0); row indices: nodes q >> j, then A_1, A_2, ...
// (chain index k, 0 past the root).  lastb: a node's last bit, z's (bit 0 of the
// leaf index l), or A_k's (bit k of l).
__device__ __forceinline__ void fwd12_path(uint32_t q, uint32_t k0, uint32_t l, uint32_t (&node)[5],
                                           uint32_t (&chain)[5], uint32_t (&lastb)[4]) {
  constexpr uint32_t I = kStage12N - 12;
  const int dq = q ? 31 - __clz(q) : -1;
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const uint32_t qq = q >> j;
    const uint32_t k = (j <= dq) ? 0u : (q ? uint32_t(j - dq) : k0 + uint32_t(j));
    node[j] = (j <= dq) ? qq : 0u;
    chain[j] = k <= I ? k : 0u;
    if (j < 4) lastb[j] = (j <= dq) ? (qq >= 2u ? (qq & 1u) : (l & 1u)) : ((l >> k) & 1u);
  }
}

// HALF (complement-symmetric iterate): the leaves that start with 0 only (128 blocks),
// which form v on the rows that start with 0 and the empty row.
template <bool LOGV, bool HALF>
__global__ __launch_bounds__(kStage12Threads) __attribute__((amdgpu_waves_per_eu(6))) void k_fwd_stage12(
    int n, const float* __restrict__ src, size_t sstride, float* __restrict__ dst, size_t dstride, const State* st,
    const Consts* cs, int frz) {
  using T = float;
  constexpr int I = kStage12N - 12;
  const int b = blockIdx.y;
  if (n != kStage12N || (frz && st[b].converged)) return;
  constexpr int LX = HALF ? I - 4 : I - 3;  // log2 of the leaves per XCD
  const uint32_t l = ((blockIdx.x & 7u) << LX) + (blockIdx.x >> 3);  // leaf index
  const uint32_t z1 = (1u << I) + l;                                        // rank of z, plus 1
  const uint32_t c = l ? uint32_t(__ffs(l) - 1) : uint32_t(I);              // chain rows written here
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  __shared__ __attribute__((aligned(16))) T buf[kF12Words];
  const uint32_t t = threadIdx.x;
  // waves 0-3 take the leaf steps, waves 4-7 the other items (a wave-uniform branch)
  const bool leafw = __builtin_amdgcn_readfirstlane(t) < 256u;
  // step 1: F_{i+4} of the chain and of z's subtree, column t
  if (leafw) {
    T H0[8], H1[4], H2[2], H3 = T(0);
#pragma unroll
    for (int g = 0; g < 8; ++g) H0[g] = T(0);
#pragma unroll
    for (int g = 0; g < 4; ++g) H1[g] = T(0);
#pragma unroll
    for (int g = 0; g < 2; ++g) H2[g] = T(0);
#pragma unroll
    for (int j = I; j >= 0; --j) {
      const T* row = src + ((size_t)((z1 >> j) - 1u) << (kStage12N - I)) + t;  // A_j (A_0 = z)
      T R[16], F1[8], F2[4], F3[2];
#pragma unroll
      for (int u = 0; u < 16; ++u) R[u] = row[uint32_t(u) << 8];
#pragma unroll
      for (int g = 0; g < 8; ++g) F1[g] = (R[g] + R[8 + g]) + H0[g];
#pragma unroll
      for (int g = 0; g < 4; ++g) F2[g] = (F1[g] + F1[4 + g]) + H1[g];
#pragma unroll
      for (int g = 0; g < 2; ++g) F3[g] = (F2[g] + F2[2 + g]) + H2[g];
      buf[(j ? 31u + uint32_t(j) : 1u) * kF12P1 + t] = (F3[0] + F3[1]) + H3;
      if (j > 0) {
        const bool lb = (l >> (j - 1)) & 1u;  // last bit of A_{j-1}
#pragma unroll
        for (int g = 0; g < 8; ++g) H0[g] = lb ? R[8 + g] : R[g];
#pragma unroll
        for (int g = 0; g < 4; ++g) H1[g] = lb ? F1[4 + g] : F1[g];
#pragma unroll
        for (int g = 0; g < 2; ++g) H2[g] = lb ? F2[2 + g] : F2[g];
        H3 = lb ? F3[1] : F3[0];
      } else {
        T F1s[2][8], F4[30];
#pragma unroll
        for (int cc = 0; cc < 2; ++cc)
#pragma unroll
          for (int g = 0; g < 8; ++g) F1s[cc][g] = R[cc * 8 + g];
        fwd4_subtree<T>(F1, F2, F3, F1s, F4);
#pragma unroll
        for (int q = 2; q < 32; ++q) buf[uint32_t(q) * kF12P1 + t] = F4[q - 2];
      }
    }
    buf[t] = T(0);
  }
  __syncthreads();
  // step 2: F_{i+8}
  T o[31];
  const uint32_t nch = c + 4u < uint32_t(I) ? c + 4u : uint32_t(I);
  const uint32_t items2 = (15u + nch) * 16u;
  if (leafw) {
    const uint32_t q2 = 16u + (t >> 4), u1 = t & 15u;
    const T* row[5];
    uint32_t lastb[4];
#pragma unroll
    for (int j = 0; j < 5; ++j) row[j] = buf + (q2 >> j) * kF12P1 + u1;
#pragma unroll
    for (int j = 0; j < 4; ++j) lastb[j] = (q2 >> j) & 1u;
    T F4[30];
    o[0] = fwd4_roll_tree<T, 16u>(row, lastb, F4);
#pragma unroll
    for (int q = 0; q < 30; ++q) o[1 + q] = F4[q];
  } else {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t e = t - 256u + uint32_t(h) * 256u;
      if (e < items2) {
        const uint32_t rb = e >> 4, u1 = e & 15u;
        const uint32_t q = rb < 15u ? rb + 1u : 0u, k0 = rb < 15u ? 0u : rb - 14u;
        uint32_t node[5], chain[5], lastb[4];
        fwd12_path(q, k0, l, node, chain, lastb);
        const T* row[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) row[j] = buf + (node[j] ? node[j] : (chain[j] ? 31u + chain[j] : 0u)) * kF12P1 + u1;
        o[h] = fwd4_roll_row<T, 16u>(row, lastb);
      }
    }
  }
  __syncthreads();
  if (leafw) {
    const uint32_t q2 = 16u + (t >> 4), u1 = t & 15u;
    T* col = buf + u1 * kF12P2;
    col[stage12_slot(q2)] = o[0];
#pragma unroll
    for (int d = 1; d <= 4; ++d) {
      T* r = col + stage12_slot(q2 << d);
#pragma unroll
      for (int m = 0; m < (1 << d); ++m) r[m] = o[(1 << d) - 1 + m];
    }
    if (t < 16u) buf[t * kF12P2] = T(0);
  } else {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t e = t - 256u + uint32_t(h) * 256u;
      if (e < items2) {
        const uint32_t rb = e >> 4, u1 = e & 15u;
        buf[u1 * kF12P2 + stage12_slot(rb < 15u ? rb + 1u : 511u + (rb - 14u))] = o[h];
      }
    }
  }
  __syncthreads();
  // step 3: F_n = r, staged at stage12_slot of the heap index below z
  const uint32_t items3 = 255u + c;
  T w[5];
  if (leafw) {
    const uint32_t q3 = 256u + t;
    const T* row[5];
    uint32_t lastb[4];
#pragma unroll
    for (int j = 0; j < 5; ++j) row[j] = buf + stage12_slot(q3 >> j);
#pragma unroll
    for (int j = 0; j < 4; ++j) lastb[j] = (q3 >> j) & 1u;
    T F4[30];
    o[0] = fwd4_roll_tree<T, kF12P2>(row, lastb, F4);
#pragma unroll
    for (int q = 0; q < 30; ++q) o[1 + q] = F4[q];
#pragma unroll
    for (int d = 0; d <= 4; ++d) w[d] = T(cs[b].w[2 * I + d]);
  } else {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t e = t - 256u + uint32_t(h) * 256u;
      if (e < items3) {
        const uint32_t q = e < 255u ? e + 1u : 0u, k0 = e < 255u ? 0u : e - 254u;
        uint32_t node[5], chain[5], lastb[4];
        fwd12_path(q, k0, l, node, chain, lastb);
        const T* row[5];
#pragma unroll
        for (int j = 0; j < 5; ++j)
          row[j] = buf + stage12_slot(node[j] ? node[j] : (chain[j] ? 511u + chain[j] : 0u));
        o[h] = fwd4_roll_row<T, kF12P2>(row, lastb);
        w[h] = T(cs[b].w[q ? I + 31 - __clz(q) : I - int(k0)]);
      }
    }
  }
  auto outv = [](T wk, T r) -> T {
    if constexpr (LOGV) return wlog_t<T>(wk, r);
    else return r;
  };
  __syncthreads();
  if (leafw) {
    const uint32_t q3 = 256u + t;
    buf[stage12_slot(q3)] = outv(w[0], o[0]);
#pragma unroll
    for (int d = 1; d <= 4; ++d) {
      T* r = buf + stage12_slot(q3 << d);
#pragma unroll
      for (int m = 0; m < (1 << d); ++m) r[m] = outv(w[d], o[(1 << d) - 1 + m]);
    }
  } else {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t e = t - 256u + uint32_t(h) * 256u;
      if (e < 255u) buf[stage12_slot(e + 1u)] = outv(w[h], o[h]);
      else if (e < items3) dst[(z1 >> (e - 254u)) - 1u] = outv(w[h], o[h]);  // A_k, k = e - 254
    }
  }
  __syncthreads();
  // copy-out: depth k of z's subtree is the run of ranks (z + 1) 2^k - 1 + m
  {
    const uint32_t q = t + 1u;
    const int kq = 31 - __clz(q);
    if (q < 512u) dst[(z1 << kq) - 1u + (q - (1u << kq))] = buf[stage12_slot(q)];
    const uint32_t st0 = stage12_slot(t);
#pragma unroll
    for (int kk = 9; kk <= 12; ++kk) {
      T* base = dst + ((z1 << kk) - 1u);
#pragma unroll
      for (int j = 0; j < (1 << (kk - 9)); ++j)
        base[t + uint32_t(j) * kStage12Threads] = buf[st0 + (1u << kk) + (1u << (kk - 5)) + uint32_t(j) * 528u];
    }
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


}  // namespace

using namespace fac;

// Launch plan levels 6-8 with FP32 iterates for n >= kD8MinN: the backward sweep
// ends with one eight-position launch from B_8 that forms D (with the block records
// and maxima, or fused with the next iteration's update and first eight forward
// positions at level 8).  At n = kStage12N one twelve-position launch reaches B_8;
// at other n two-, four- and eight-position launches stop at position 8.
constexpr int kD8MinN = 12;
bool d8_plan(int n, int fuse, int esz) { return fuse >= 6 && esz == 4 && n >= kD8MinN; }

template <typename T>
hipError_t launch_forward(const Group<T>& g, hipStream_t s, int* launches, int fuse, int logv,
                          const FusedUpdate* upd, int first8_done) {
  const int n = g.n;
  constexpr int V = 16 / sizeof(T);
  const T* src = g.p;
  size_t ss = g.xs;
  int k = 0;
  if (upd && !forward_update_fusable(n, fuse)) return hipErrorInvalidValue;
  int i = 0;
  if (first8_done) {
    // F_8 was formed by the previous iteration's fused D launch (into f1); the
    // launches of positions 8 .. n-1 follow (the next one writes f0)
    if (upd || !backward_fuses_next(n, fuse, int(sizeof(T)))) return hipErrorInvalidValue;
    src = g.f1;
    ss = g.fs;
    i = 8;
    k = 0;
  }
  // fuse >= 4: the last four positions in one launch with LDS-staged outputs;
  // fuse >= 5: the first eight positions in one launch
  const bool last4 = fuse >= 4 && n >= kLast4MinN;
  const bool first8 = fuse >= 5 && n >= kFirst8MinN;
  for (; i < n; k++) {
    if (first8 && i == 0) {
      T* dst = (k & 1) ? g.f1 : g.f0;
      const dim3 grid(1u << (n - 12), g.nb);  // 16 columns of F_8 per block
      if (upd)
        hipLaunchKernelGGL((k_fwd_first8<T, true>), grid, dim3(kFirst8Threads), 0, s, n, src, ss, dst, g.fs, g,
                           upd->floor, upd->check_tol, upd->nmax);
      else
        hipLaunchKernelGGL((k_fwd_first8<T, false>), grid, dim3(kFirst8Threads), 0, s, n, src, ss, dst, g.fs, g,
                           0.0, 0, 0);
      if (launches) ++*launches;
      src = dst;
      ss = g.fs;
      i = 8;
      continue;
    }
    if constexpr (sizeof(T) == 4) {
      // fuse >= 7 at n = kStage12N: positions 8 .. n-1 in one launch
      if (fuse >= 7 && n == kStage12N && i == n - 12) {
        T* dst = logv ? g.v : g.r;
        const dim3 grid((1u << (n - 12)) >> (g.half ? 1 : 0), g.nb);  // one block per leaf of F_8
        if (g.half) {
          if (logv)
            hipLaunchKernelGGL((k_fwd_stage12<true, true>), grid, dim3(kStage12Threads), 0, s, n, src, ss, dst, g.ys,
                               g.st, g.cs, g.frz);
          else
            hipLaunchKernelGGL((k_fwd_stage12<false, true>), grid, dim3(kStage12Threads), 0, s, n, src, ss, dst,
                               g.ys, g.st, g.cs, g.frz);
        } else if (logv) {
          hipLaunchKernelGGL((k_fwd_stage12<true, false>), grid, dim3(kStage12Threads), 0, s, n, src, ss, dst, g.ys,
                             g.st, g.cs, g.frz);
        } else {
          hipLaunchKernelGGL((k_fwd_stage12<false, false>), grid, dim3(kStage12Threads), 0, s, n, src, ss, dst,
                             g.ys, g.st, g.cs, g.frz);
        }
        if (launches) ++*launches;
        break;
      }
    }
    if (last4 && n - i == 4) {
      T* dst = logv ? g.v : g.r;
      const uint32_t top = (1u << (n - 10)) - 1u;  // rows above the deep blocks' subtrees
      const dim3 grid((1u << (n - 10)) + (top + kLast4Threads - 1u) / kLast4Threads, g.nb);
      if (logv)
        hipLaunchKernelGGL((k_fwd_last4<T, true>), grid, dim3(kLast4Threads), 0, s, n, src, ss, dst, g.ys, g.st,
                           g.cs, g.frz);
      else
        hipLaunchKernelGGL((k_fwd_last4<T, false>), grid, dim3(kLast4Threads), 0, s, n, src, ss, dst, g.ys, g.st,
                           g.cs, g.frz);
      if (launches) ++*launches;
      break;
    }
    // four positions per launch except the last four or fewer, whose outputs (one
    // value per row) are written by the width-1 two-position kernel (or, with
    // last4, down to exactly four positions left)
    if (fuse >= 2 && i + 4 < n && !(last4 && n - i < 8)) {
      const bool last = (i + 4 == n);
      const bool lv = last && logv;
      T* dst = last ? (lv ? g.v : g.r) : ((k & 1) ? g.f1 : g.f0);
      const size_t ds = last ? g.ys : g.fs;
      const uint32_t S4 = 1u << (n - i - 4);
      Order o = make_order(i + 1, ilog2(S4), sizeof(T));
      make_order_xcd(i + 1, ilog2(S4), kStage4Block, o);  // o unchanged where infeasible
      const dim3 grid(order_blocks(o, kStage4Block), g.nb);
      if (i == 0 && upd)
        hipLaunchKernelGGL((k_fwd_first4_upd<T>), grid, dim3(kStage4Block), 0, s, n, dst, ds, g, o, upd->floor,
                           upd->check_tol);
      else if (lv)
        hipLaunchKernelGGL((k_fwd_stage4<T, true>), grid, dim3(kStage4Block), 0, s, n, i, src, ss, dst, ds, g.st,
                           g.cs, o, g.frz);
      else
        hipLaunchKernelGGL((k_fwd_stage4<T, false>), grid, dim3(kStage4Block), 0, s, n, i, src, ss, dst, ds, g.st,
                           g.cs, o, g.frz);
      if (launches) ++*launches;
      src = dst;
      ss = ds;
      i += 4;
      continue;
    }
    const int step = (fuse && i + 2 <= n && !(last4 && n - i - 2 < 4)) ? 2 : 1;
    const bool last = (i + step == n);
    const bool lv = last && logv;
    T* dst;
    size_t ds;
    if (last) { dst = lv ? g.v : g.r; ds = g.ys; }
    else { dst = (k & 1) ? g.f1 : g.f0; ds = g.fs; }
    if (step == 2) {
      const uint32_t S = 1u << (n - i - 2);  // output row width
      if (S == 1u && n >= kLast2MinN) {
        const dim3 grid(2u * ((1u << (n - 4)) / kLast2Threads), g.nb);
        if (lv)
          hipLaunchKernelGGL((k_fwd_last2<T, true>), grid, dim3(kLast2Threads), 0, s, n, src, ss, dst, ds, g.st,
                             g.cs);
        else
          hipLaunchKernelGGL((k_fwd_last2<T, false>), grid, dim3(kLast2Threads), 0, s, n, src, ss, dst, ds, g.st,
                             g.cs);
      } else if (S == 1u) {
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
                           int* dpart_blocks, const FusedNext* next) {
  if (next && !backward_fuses_next(g.n, fuse, int(sizeof(T)))) return hipErrorInvalidValue;
  const int n = g.n;
  constexpr int V = 16 / sizeof(T);
  const T* src = g.v;
  size_t ss = g.ys;
  // levels 6-8 at n other than kStage12N: the launches stop at position 8, and the
  // first one takes the parity that leaves B_8 in f0 (the fused D launch writes F_8
  // to f1)
  const bool to8 = sizeof(T) == 4 && d8_plan(n, fuse, int(sizeof(T))) && n != kStage12N;
  int k = to8 ? (backward_launches(n, fuse, int(sizeof(T))) - 2) & 1 : 0;
  if (dpart_blocks) *dpart_blocks = 0;
  // fuse = 2: four positions per launch, the n mod 4 leftover positions first;
  // fuse = 3: the same with eight positions per launch while four remain after
  const int lead = (fuse >= 2 && n >= 4) ? n % 4 : -1;
  for (int top = n; top > 0; k++) {           // B_top -> B_{top-step}
    // fuse >= 6 at n = kStage12N, FP32: the last twelve positions in one launch, then
    // the first eight in one (with D and its records when dpart)
    if constexpr (sizeof(T) == 4) {
      if (fuse >= 6 && n == kStage12N && top == n) {
        const int i = n - 12;
        T* dst = (k & 1) ? g.f1 : g.f0;
        if (g.half)
          hipLaunchKernelGGL(k_bwd_stage12<true>, dim3(1u << i, g.nb), dim3(kStage12Threads), 0, s, n, src, ss, dst,
                             g.fs, g.st, g.frz);
        else
          hipLaunchKernelGGL(k_bwd_stage12<false>, dim3(2u << i, g.nb), dim3(kStage12Threads), 0, s, n, src, ss, dst,
                             g.fs, g.st, g.frz);
        if (launches) ++*launches;
        src = dst;
        ss = g.fs;
        top = i;
        continue;
      }
    }
    if (sizeof(T) == 4 && d8_plan(n, fuse, int(sizeof(T))) && top == 8) {
      constexpr int LP = stage8_tile<T>() == 16 ? 4 : 3;
      // column blocks of P columns (half: those whose first column bit is 0)
      const dim3 grid((1u << (n - 8 - LP)) >> (g.half ? 1 : 0), 1, g.nb);
      const dim3 block(32 * stage8_tile<T>());
      if (g.half && !(dpart || next)) return hipErrorInvalidValue;
      if (next) {
        // D with the next iteration's update and first eight forward positions: F_8 to f1
        if (src == g.f1) return hipErrorInvalidValue;
        if constexpr (sizeof(T) == 4) {
          // maxima set k of instance 0 at kBlockMaxima + k kMaxRedBlocks floats (set 0 is
          // also the D launch's with records)
          float* m0 = reinterpret_cast<float*>(g.part + kBlockMaxima);
          const uint32_t ks = uint32_t(kMaxRedBlocks);
          const S8Update u{m0 + (next->par ? 0u : ks), m0 + (next->par ? ks : 0u), float(next->floor), next->nprev};
          if (g.half) {
            // 8 columns per block: twice the blocks of half the work (the half plan's
            // 16-column launch runs fewer blocks than CUs)
            const dim3 grid8((1u << (n - 8 - 3)) >> 1, 1, g.nb);
            hipLaunchKernelGGL((k_bwd_stage8_p<T, kS8ColumnsDUH, 8>), grid8, dim3(32 * 8), 0, s, n, 0, src, ss, g.f1,
                               g.fs, g.st, g.frz, g, u);
            if (dpart_blocks) *dpart_blocks = int(grid8.x);
          } else {
            hipLaunchKernelGGL((k_bwd_stage8_p<T, kS8ColumnsDU>), grid, block, 0, s, n, 0, src, ss, g.f1, g.fs,
                               g.st, g.frz, g, u);
            if (dpart_blocks) *dpart_blocks = int(grid.x);
          }
        }
      } else if (dpart) {
        if constexpr (sizeof(T) == 4) {
          if (g.half)
            hipLaunchKernelGGL((k_bwd_stage8_p<T, kS8ColumnsDH>), grid, block, 0, s, n, 0, src, ss, g.g, g.xs, g.st,
                               g.frz, g, S8Update{});
          else
            hipLaunchKernelGGL((k_bwd_stage8_p<T, kS8ColumnsD>), grid, block, 0, s, n, 0, src, ss, g.g, g.xs, g.st,
                               g.frz, g, S8Update{});
        }
        if (dpart_blocks) *dpart_blocks = int(grid.x);
      } else {
        hipLaunchKernelGGL((k_bwd_stage8_p<T, kS8Columns>), grid, block, 0, s, n, 0, src, ss, g.g, g.xs, g.st,
                           g.frz, g, S8Update{});
      }
      if (launches) ++*launches;
      top = 0;
      continue;
    }
    if (fuse >= 3 && lead >= 0 && n - top >= lead && top - 8 >= (to8 ? 8 : 4)) {
      const int i = top - 8;
      T* dst = (k & 1) ? g.f1 : g.f0;
      constexpr int LP = stage8_tile<T>() == 16 ? 4 : stage8_tile<T>() == 8 ? 3 : 2;
      const int sh = n - i - 8;
      int lc = sh < LP ? sh : LP;
      if (g.s8lc > 0 && g.s8lc < lc) lc = g.s8lc;  // tuned: fewer columns, more roots per block
      const dim3 grid(((stage8_slots(i, LP - lc) << (sh - lc)) + 7u) & ~7u, 1, g.nb);
      const dim3 block(32 * stage8_tile<T>());
      if (lc == LP) {
        hipLaunchKernelGGL((k_bwd_stage8_p<T, kS8Columns>), grid, block, 0, s, n, i, src, ss, dst, g.fs, g.st,
                           g.frz, g, S8Update{});
      } else if (lc == 0) {
        hipLaunchKernelGGL((k_bwd_stage8_p<T, kS8Roots>), grid, block, 0, s, n, i, src, ss, dst, g.fs, g.st,
                           g.frz, g, S8Update{});
      } else switch (lc) {
        case 1: hipLaunchKernelGGL((k_bwd_stage8<T, 1>), grid, block, 0, s, n, i, src, ss, dst, g.fs, g.st); break;
        case 2: hipLaunchKernelGGL((k_bwd_stage8<T, 2>), grid, block, 0, s, n, i, src, ss, dst, g.fs, g.st); break;
        default:
          if constexpr (LP == 4)
            hipLaunchKernelGGL((k_bwd_stage8<T, 3>), grid, block, 0, s, n, i, src, ss, dst, g.fs, g.st);
          break;
      }
      if (launches) ++*launches;
      src = dst;
      ss = g.fs;
      top = i;
      continue;
    }
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
        hipLaunchKernelGGL((k_bwd_stage4<T, 1, true>), dim3(nbk, g.nb), dim3(kBlock), 0, s, n, i, src, ss, dst, ds,
                           g, o);
        if (dpart_blocks) *dpart_blocks = int(nbk);
      } else {
        // one column per thread (2 or 4 per thread measured no faster: 0.079 ms per
        // backward sweep at n = 20 for 1, 0.081 for 2 and 4)
        // (two items per thread with all loads issued first: 0.0774 ms per sweep;
        // four: 0.0865)
        hipLaunchKernelGGL((k_bwd_stage4<T, 1, false>), dim3(blocks_for(order_threads(o), kStage4Block), g.nb),
                           dim3(kStage4Block), 0, s, n, i, src, ss, dst, ds, g, o);
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


int factored_launches(int n, int fuse) { return fuse ? (n + 1) / 2 : n; }

template <typename T>
hipError_t launch_backward8_sym_v(const Group<T>& g, hipStream_t s, T* dst) {
  const int n = g.n, i = n - 8;
  constexpr int LP = stage8_tile<T>() == 16 ? 4 : 3;
  if (n % 4 != 0 || i < 4) return hipErrorInvalidValue;
  const uint32_t slots = stage8_slots(i - 1, LP) + 1u;  // + the empty row
  const dim3 grid((slots + 7u) & ~7u, 1, g.nb);
  hipLaunchKernelGGL((k_bwd_stage8_p<T, kS8SymRoots>), grid, dim3(32 * stage8_tile<T>()), 0, s, n, i, g.v, g.ys,
                     dst, g.fs, g.st, g.frz, g, S8Update{});
  return hipGetLastError();
}
template hipError_t launch_backward8_sym_v<float>(const Group<float>&, hipStream_t, float*);
template hipError_t launch_backward8_sym_v<double>(const Group<double>&, hipStream_t, double*);

int backward_launches(int n, int fuse, int esz) {
  if (fuse >= 6 && n == kStage12N && esz == 4) return 2;
  if (d8_plan(n, fuse, esz)) {
    // the n mod 4 leading positions two or one at a time, eight-position launches
    // while they end at 8 or above, a four-position one if four are left, the D launch
    const int lead = n % 4, m = (n - lead - 8) / 4;
    return (lead + 1) / 2 + m / 2 + m % 2 + 1;
  }
  if (fuse >= 3 && n >= 4) {
    const int four = n / 4, eight = (four - 1) / 2;  // the last launch keeps four positions
    return four - eight + (n % 4 + 1) / 2;
  }
  if (fuse == 2 && n >= 4) return n / 4 + (n % 4 + 1) / 2;
  return factored_launches(n, fuse);
}

int forward_launches(int n, int fuse, int esz) {
  if (fuse >= 7 && n == kStage12N && esz == 4) return 2;
  if (fuse >= 5 && n >= kFirst8MinN) return forward_launches(n, 4) - 1;
  if (fuse >= 4 && n >= kLast4MinN) {
    const int four = (n - 4) / 4, rest = (n - 4) % 4;  // then 0-3 positions two or one at a time
    return four + (rest + 1) / 2 + 1;
  }
  if (fuse >= 2 && n > 4) {
    const int four = (n - 1) / 4;  // launches of four positions; the rest two at a time
    return four + (n - 4 * four + 1) / 2;
  }
  return factored_launches(n, fuse);
}

bool forward_update_fusable(int n, int fuse) { return fuse >= 2 && n > 4; }
bool forward_first8(int n, int fuse) { return fuse >= 5 && n >= kFirst8MinN; }
bool backward_writes_maxima(int n, int fuse, int esz) { return d8_plan(n, fuse, esz); }
bool backward_fuses_next(int n, int fuse, int esz) { return fuse >= 8 && d8_plan(n, fuse, esz); }
bool half_plan_fits(int n, int fuse) { return fuse >= 8 && n == kStage12N; }

template hipError_t launch_forward<float>(const Group<float>&, hipStream_t, int*, int, int, const FusedUpdate*,
                                          int);
template hipError_t launch_forward<double>(const Group<double>&, hipStream_t, int*, int, int,
                                           const FusedUpdate*, int);
template hipError_t launch_backward<float>(const Group<float>&, hipStream_t, int*, int, int, int*,
                                           const FusedNext*);
template hipError_t launch_backward<double>(const Group<double>&, hipStream_t, int*, int, int, int*,
                                            const FusedNext*);

}  // namespace ba
