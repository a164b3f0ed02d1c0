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
// Each stage is a streaming pass with unit-stride reads and writes.
#include "ba_internal.h"

namespace ba {
namespace {

// Vector of V consecutive elements (16-byte loads/stores for V*sizeof(T) == 16).
template <typename T, int V>
struct Vec {
  T v[V];
};
template <typename T, int V>
__device__ __forceinline__ Vec<T, V> ld(const T* p) {
  Vec<T, V> r;
  if constexpr (V * sizeof(T) == 16) {
    const uint4 q = *reinterpret_cast<const uint4*>(p);
    *reinterpret_cast<uint4*>(r.v) = q;
  } else {
#pragma unroll
    for (int k = 0; k < V; ++k) r.v[k] = p[k];
  }
  return r;
}
template <typename T, int V>
__device__ __forceinline__ void stv(T* p, const Vec<T, V>& a) {
  if constexpr (V * sizeof(T) == 16) {
    *reinterpret_cast<uint4*>(p) = *reinterpret_cast<const uint4*>(a.v);
  } else {
#pragma unroll
    for (int k = 0; k < V; ++k) p[k] = a.v[k];
  }
}

// One forward stage; each thread produces V consecutive columns of one row
// (V divides the row width S = 2^(n-i-1)).
template <typename T, int V>
__global__ __launch_bounds__(kBlock) void k_fwd_stage(int n, int i, const T* __restrict__ src,
                                                      size_t sstride, T* __restrict__ dst,
                                                      size_t dstride, const State* st) {
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
    stv<T, V>(dst + idx, acc);
  }
}

// One backward stage; each thread produces V consecutive columns of one row
// (V divides the source row width S = 2^(n-i-1)).
template <typename T, int V>
__global__ __launch_bounds__(kBlock) void k_bwd_stage(int n, int i, const T* __restrict__ src,
                                                      size_t sstride, T* __restrict__ dst,
                                                      size_t dstride, const State* st) {
  const int b = blockIdx.y;
  if (st[b].converged) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh = n - i - 1;                    // log2 of the source width
  const uint32_t S = 1u << sh;
  const uint32_t total = (((2u << i) - 1u) << (sh + 1)) / V;
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
    stv<T, V>(dst + idx, o);
  }
}

// Two forward stages at once (positions i and i+1).  Columns of F_i are u s''
// with u = 2 x_i + x_{i+1}.  Every row of F_{i+2} except the empty string is a
// child c_b = 2r+1+b of a root r (|r| <= i+1); the thread of root r produces both
// children, V consecutive columns s'':
//   F_{i+2}[c_b] = sum_u F_i[c_b][u]                      (both bits deleted)
//               + F_i[r][b0] + F_i[r][b1] + F_i[r][0b] + F_i[r][1b]   (one kept)
//               + F_i[parent(r)][last(r) b]               (both kept)
// (terms whose source row has length > i are absent).  Thread "root -1" produces
// the empty row, sum_u F_i[empty][u].
template <typename T, int V>
__global__ __launch_bounds__(kBlock) void k_fwd_stage2(int n, int i, const T* __restrict__ src,
                                                       size_t sstride, T* __restrict__ dst,
                                                       size_t dstride, const State* st) {
  const int b = blockIdx.y;
  if (st[b].converged) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh = n - i - 2;                  // log2 of the output width S''
  const uint32_t S = 1u << sh;
  const uint32_t rows_in = (2u << i) - 1u;   // rows of F_i
  const uint32_t roots = (4u << i) - 1u;     // rows of F_{i+1}
  const uint32_t cols = S / V;
  const uint32_t total = (roots + 1u) * cols;
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
    const uint32_t rr = q / cols;            // root + 1
    const uint32_t s = (q - rr * cols) * V;
    if (rr == 0) {
      Vec<T, V> o;
#pragma unroll
      for (int k = 0; k < V; ++k) o.v[k] = T(0);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const Vec<T, V> a = ld<T, V>(src + (u << sh) + s);
#pragma unroll
        for (int k = 0; k < V; ++k) o.v[k] += a.v[k];
      }
      stv<T, V>(dst + s, o);
      continue;
    }
    const uint32_t r = rr - 1u;
    Vec<T, V> o0, o1;
#pragma unroll
    for (int k = 0; k < V; ++k) { o0.v[k] = T(0); o1.v[k] = T(0); }
    if (r < rows_in) {
      const T* pr = src + (r << (sh + 2)) + s;
      const Vec<T, V> a00 = ld<T, V>(pr), a01 = ld<T, V>(pr + S), a10 = ld<T, V>(pr + 2 * S),
                      a11 = ld<T, V>(pr + 3 * S);
#pragma unroll
      for (int k = 0; k < V; ++k) {
        o0.v[k] = a00.v[k] + a01.v[k] + a00.v[k] + a10.v[k];   // b = 0: u in {00, 01, 00, 10}
        o1.v[k] = a10.v[k] + a11.v[k] + a01.v[k] + a11.v[k];   // b = 1: u in {10, 11, 01, 11}
      }
    }
    if (r >= 1u) {
      const uint32_t pa = (r - 1u) >> 1, lb = (r - 1u) & 1u;
      const T* pp = src + (pa << (sh + 2)) + ((2u * lb) << sh) + s;
      const Vec<T, V> a = ld<T, V>(pp), c = ld<T, V>(pp + S);
#pragma unroll
      for (int k = 0; k < V; ++k) { o0.v[k] += a.v[k]; o1.v[k] += c.v[k]; }
    }
    const uint32_t c0 = 2u * r + 1u, c1 = c0 + 1u;
    if (c0 < rows_in) {
      const T* p0 = src + (c0 << (sh + 2)) + s;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const Vec<T, V> a = ld<T, V>(p0 + (u << sh));
#pragma unroll
        for (int k = 0; k < V; ++k) o0.v[k] += a.v[k];
      }
    }
    if (c1 < rows_in) {
      const T* p1 = src + (c1 << (sh + 2)) + s;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const Vec<T, V> a = ld<T, V>(p1 + (u << sh));
#pragma unroll
        for (int k = 0; k < V; ++k) o1.v[k] += a.v[k];
      }
    }
    stv<T, V>(dst + (c0 << sh) + s, o0);
    stv<T, V>(dst + (c1 << sh) + s, o1);
  }
}

// Two backward stages at once (positions i and i+1): for a row r of B_i and
// columns (b, c, s''),
//   B_i[r][b c s''] = B_{i+2}[r] + B_{i+2}[r c] + B_{i+2}[r b] + B_{i+2}[r b c]
// (subsets of the two positions that are kept); one thread per (r, V columns s'')
// reads the 7 rows of r's depth-2 subtree once and writes its 4 columns.
template <typename T, int V>
__global__ __launch_bounds__(kBlock) void k_bwd_stage2(int n, int i, const T* __restrict__ src,
                                                       size_t sstride, T* __restrict__ dst,
                                                       size_t dstride, const State* st) {
  const int b = blockIdx.y;
  if (st[b].converged) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh = n - i - 2;                  // log2 of the source width S''
  const uint32_t S = 1u << sh;
  const uint32_t rows = (2u << i) - 1u;      // rows of B_i
  const uint32_t cols = S / V;
  const uint32_t total = rows * cols;
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
    const uint32_t r = q / cols;
    const uint32_t s = (q - r * cols) * V;
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
    T* o = dst + (r << (sh + 2)) + s;
    stv<T, V>(o, o00);
    stv<T, V>(o + S, o01);
    stv<T, V>(o + 2 * S, o10);
    stv<T, V>(o + 3 * S, o11);
  }
}

inline uint32_t grid_for(uint32_t total) {
  uint32_t g = (total + kBlock - 1) / kBlock;
  return g > 8192u ? 8192u : (g == 0 ? 1u : g);
}

}  // namespace

template <typename T>
hipError_t launch_forward(const Group<T>& g, hipStream_t s, int* launches, int fuse) {
  const int n = g.n;
  constexpr int V = 16 / sizeof(T);
  const T* src = g.p;
  size_t ss = g.xs;
  int k = 0;
  for (int i = 0; i < n; k++) {
    const int step = (fuse && i + 2 <= n) ? 2 : 1;
    T* dst;
    size_t ds;
    if (i + step == n) { dst = g.r; ds = g.ys; }
    else { dst = (k & 1) ? g.f1 : g.f0; ds = g.fs; }
    const uint32_t w = 1u << (n - i - step);  // output row width
    if (step == 2) {
      const uint32_t work = ((4u << i) * w);
      if (w >= uint32_t(V))
        hipLaunchKernelGGL((k_fwd_stage2<T, V>), dim3(grid_for(work / V), g.nb), dim3(kBlock), 0, s, n, i,
                           src, ss, dst, ds, g.st);
      else
        hipLaunchKernelGGL((k_fwd_stage2<T, 1>), dim3(grid_for(work), g.nb), dim3(kBlock), 0, s, n, i, src,
                           ss, dst, ds, g.st);
    } else {
      const uint32_t total = ((4u << i) - 1u) * w;
      if (w >= uint32_t(V))
        hipLaunchKernelGGL((k_fwd_stage<T, V>), dim3(grid_for(total / V), g.nb), dim3(kBlock), 0, s, n, i,
                           src, ss, dst, ds, g.st);
      else
        hipLaunchKernelGGL((k_fwd_stage<T, 1>), dim3(grid_for(total), g.nb), dim3(kBlock), 0, s, n, i, src,
                           ss, dst, ds, g.st);
    }
    if (launches) ++*launches;
    src = dst;
    ss = ds;
    i += step;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_backward(const Group<T>& g, hipStream_t s, int* launches, int fuse) {
  const int n = g.n;
  constexpr int V = 16 / sizeof(T);
  const T* src = g.v;
  size_t ss = g.ys;
  int k = 0;
  for (int top = n; top > 0; k++) {           // B_top -> B_{top-step}
    const int step = (fuse && top >= 2) ? 2 : 1;
    const int i = top - step;
    T* dst;
    size_t ds;
    if (i == 0) { dst = g.g; ds = g.xs; }
    else { dst = (k & 1) ? g.f1 : g.f0; ds = g.fs; }
    const uint32_t w = 1u << (n - i - step);  // source row width
    if (step == 2) {
      const uint32_t work = ((2u << i) - 1u) * w;
      if (w >= uint32_t(V))
        hipLaunchKernelGGL((k_bwd_stage2<T, V>), dim3(grid_for(work / V), g.nb), dim3(kBlock), 0, s, n, i,
                           src, ss, dst, ds, g.st);
      else
        hipLaunchKernelGGL((k_bwd_stage2<T, 1>), dim3(grid_for(work), g.nb), dim3(kBlock), 0, s, n, i, src,
                           ss, dst, ds, g.st);
    } else {
      const uint32_t total = ((2u << i) - 1u) << (n - i);
      if (w >= uint32_t(V))
        hipLaunchKernelGGL((k_bwd_stage<T, V>), dim3(grid_for(total / V), g.nb), dim3(kBlock), 0, s, n, i,
                           src, ss, dst, ds, g.st);
      else
        hipLaunchKernelGGL((k_bwd_stage<T, 1>), dim3(grid_for(total), g.nb), dim3(kBlock), 0, s, n, i, src,
                           ss, dst, ds, g.st);
    }
    if (launches) ++*launches;
    src = dst;
    ss = ds;
    top = i;
  }
  return hipGetLastError();
}

int factored_launches(int n, int fuse) { return fuse ? (n + 1) / 2 : n; }

template hipError_t launch_forward<float>(const Group<float>&, hipStream_t, int*, int);
template hipError_t launch_forward<double>(const Group<double>&, hipStream_t, int*, int);
template hipError_t launch_backward<float>(const Group<float>&, hipStream_t, int*, int);
template hipError_t launch_backward<double>(const Group<double>&, hipStream_t, int*, int);

}  // namespace ba
