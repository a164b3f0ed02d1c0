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

template <typename T>
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
  const uint32_t total = ((4u << i) - 1u) << sh;
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += gridDim.x * blockDim.x) {
    const uint32_t row = idx >> sh;
    const uint32_t s = idx & (S - 1u);
    T acc = T(0);
    if (row < rows_in) {
      const uint32_t base = row << (sh + 1);
      acc = src[base + s] + src[base + S + s];
    }
    if (row >= 1u) {
      const uint32_t rp = (row - 1u) >> 1, bb = (row - 1u) & 1u;
      acc += src[(rp << (sh + 1)) + (bb << sh) + s];
    }
    dst[idx] = acc;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_bwd_stage(int n, int i, const T* __restrict__ src,
                                                      size_t sstride, T* __restrict__ dst,
                                                      size_t dstride, const State* st) {
  const int b = blockIdx.y;
  if (st[b].converged) return;
  src += (size_t)b * sstride;
  dst += (size_t)b * dstride;
  const int sh = n - i - 1;                    // log2 of the source width
  const uint32_t S = 1u << sh;
  const uint32_t total = ((2u << i) - 1u) << (sh + 1);
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += gridDim.x * blockDim.x) {
    const uint32_t row = idx >> (sh + 1);
    const uint32_t s = idx & ((2u * S) - 1u);
    const uint32_t bb = s >> sh, sp = s & (S - 1u);
    dst[idx] = src[(row << sh) + sp] + src[((2u * row + 1u + bb) << sh) + sp];
  }
}

inline uint32_t grid_for(uint32_t total) {
  uint32_t g = (total + kBlock - 1) / kBlock;
  return g > 8192u ? 8192u : (g == 0 ? 1u : g);
}

}  // namespace

template <typename T>
hipError_t launch_forward(const Group<T>& g, hipStream_t s, int* launches) {
  const int n = g.n;
  const T* src = g.p;
  size_t ss = g.xs;
  for (int i = 0; i < n; ++i) {
    T* dst;
    size_t ds;
    if (i == n - 1) { dst = g.r; ds = g.ys; }
    else { dst = (i & 1) ? g.f1 : g.f0; ds = g.fs; }
    const uint32_t total = ((4u << i) - 1u) << (n - i - 1);
    hipLaunchKernelGGL(k_fwd_stage<T>, dim3(grid_for(total), g.nb), dim3(kBlock), 0, s, n, i, src,
                       ss, dst, ds, g.st);
    if (launches) ++*launches;
    src = dst;
    ss = ds;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_backward(const Group<T>& g, hipStream_t s, int* launches) {
  const int n = g.n;
  const T* src = g.v;
  size_t ss = g.ys;
  int k = 0;
  for (int i = n - 1; i >= 0; --i, ++k) {
    T* dst;
    size_t ds;
    if (i == 0) { dst = g.g; ds = g.xs; }
    else { dst = (k & 1) ? g.f1 : g.f0; ds = g.fs; }
    const uint32_t total = ((2u << i) - 1u) << (n - i);
    hipLaunchKernelGGL(k_bwd_stage<T>, dim3(grid_for(total), g.nb), dim3(kBlock), 0, s, n, i, src,
                       ss, dst, ds, g.st);
    if (launches) ++*launches;
    src = dst;
    ss = ds;
  }
  return hipGetLastError();
}

template hipError_t launch_forward<float>(const Group<float>&, hipStream_t, int*);
template hipError_t launch_forward<double>(const Group<double>&, hipStream_t, int*);
template hipError_t launch_backward<float>(const Group<float>&, hipStream_t, int*);
template hipError_t launch_backward<double>(const Group<double>&, hipStream_t, int*);

}  // namespace ba
