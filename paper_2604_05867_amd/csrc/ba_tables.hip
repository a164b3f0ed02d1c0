// Count tables of the stream engine: the distinct subsequences of every half
// string with their embedding counts (see ba_internal.h for the layout).
//
// The half strings have at most 10 bits, so every table entry is produced by a
// direct check of each candidate subsequence (greedy matching, Section 4's
// NextPos walk) and an exact integer embedding-count DP.  Built once per input
// length at bind time.
#include "ba_internal.h"

namespace ba {
namespace {

__device__ __forceinline__ int bit_at(uint32_t s, int len, int i) { return (s >> (len - 1 - i)) & 1; }

// Greedy embedding of y (length k) in x (length n): returns the position after
// the last matched bit, or -1 if y is not a subsequence of x.
__device__ int greedy_end(uint32_t y, int k, uint32_t x, int n) {
  int pos = 0;
  for (int t = 0; t < k; ++t) {
    const int b = bit_at(y, k, t);
    while (pos < n && bit_at(x, n, pos) != b) ++pos;
    if (pos == n) return -1;
    ++pos;
  }
  return pos;
}

// Which bits occur in x[g:n]: bit0 -> 1, bit1 -> 2.
__device__ int bits_after(uint32_t x, int n, int g) {
  int m = 0;
  for (int i = g; i < n; ++i) m |= 1 << bit_at(x, n, i);
  return m;
}

// Class of (x1, y1) as in ba_internal.h.
__device__ int class_of(int ext) {
  const bool e0 = ext & 1, e1 = ext & 2;
  if (e1 && !e0) return 0;
  if (!e0 && !e1) return 1;
  if (e0 && !e1) return 2;
  return 3;
}

__device__ __forceinline__ void unrank(uint32_t r, uint32_t* bits, int* k) {
  int kk = 31 - __clz(r + 1u);
  *k = kk;
  *bits = r - ((1u << kk) - 1u);
}

__device__ void put_byte(uint4& e, int j, uint32_t v) {
  const int w = 1 + (j >> 2), sh = 8 * (j & 3);
  if (w == 1) e.y |= v << sh;
  else if (w == 2) e.z |= v << sh;
  else e.w |= v << sh;
}

// T2 entry for y2 (rank r) in x2: E2s[j] = emb(y2, x2[j:n2]) by the suffix DP
// s[t] = #embeddings of y2[t:] in the current suffix.
__device__ uint4 make_t2(uint32_t y2, int k2, uint32_t x2, int n2) {
  uint32_t s[kHalfMax + 2];
  for (int t = 0; t <= k2; ++t) s[t] = (t == k2) ? 1u : 0u;
  uint32_t e2s[kHalfMax + 1];
  e2s[n2] = s[0];
  for (int i = n2 - 1; i >= 0; --i) {
    const int b = bit_at(x2, n2, i);
    for (int t = 0; t < k2; ++t)
      if (bit_at(y2, k2, t) == b) s[t] += s[t + 1];
    e2s[i] = s[0];
  }
  int jmax = 0;
  for (int j = 0; j <= n2; ++j)
    if (e2s[j] > 0) jmax = j;
  uint4 e = make_uint4(y2 | (uint32_t(k2) << 10) | (uint32_t(jmax) << 14), 0u, 0u, 0u);
  for (int j = 0; j <= n2; ++j) put_byte(e, j, e2s[j]);
  return e;
}

// T1 entry for y1 in x1: byte u = emb(y1[0:k1-u], x1), u = 0..k1 (prefix counts
// stored from the longest prefix down, so that the sweep kernels index them
// statically), by the prefix DP over x1.
__device__ uint4 make_t1(uint32_t x1, int n1, uint32_t y1, int k1, int cls) {
  uint32_t c[kHalfMax + 1];
  c[0] = 1;
  for (int t = 1; t <= k1; ++t) c[t] = 0;
  for (int i = 0; i < n1; ++i) {
    const int b = bit_at(x1, n1, i);
    for (int t = k1; t >= 1; --t)
      if (bit_at(y1, k1, t - 1) == b) c[t] += c[t - 1];
  }
  uint4 e = make_uint4(x1 | (y1 << 10) | (uint32_t(k1) << 20) | (uint32_t(cls) << 24), 0u, 0u, 0u);
  for (int t = 0; t <= k1; ++t) put_byte(e, k1 - t, c[t]);
  return e;
}

__global__ void k_t2_count(int n2, uint32_t* cnt2, uint32_t* n0) {
  const uint32_t x2 = blockIdx.x * blockDim.x + threadIdx.x;
  if (x2 >= (1u << n2)) return;
  uint32_t c = 0, c0 = 0;
  for (uint32_t r = 0; r < out_count(n2); ++r) {
    uint32_t y; int k;
    unrank(r, &y, &k);
    if (greedy_end(y, k, x2, n2) >= 0) {
      ++c;
      if (k >= 1 && bit_at(y, k, 0) == 0) ++c0;
    }
  }
  cnt2[x2] = c;
  n0[x2] = c0;
}

__global__ void k_t2_fill(int n2, const uint32_t* off2, uint4* t2) {
  const uint32_t x2 = blockIdx.x * blockDim.x + threadIdx.x;
  if (x2 >= (1u << n2)) return;
  uint32_t o = off2[x2];
  t2[o++] = make_t2(0, 0, x2, n2);  // empty string first
  for (int first = 0; first <= 1; ++first)
    for (int k = 1; k <= n2; ++k) {
      const uint32_t lo = first ? (1u << (k - 1)) : 0u, hi = first ? (1u << k) : (1u << (k - 1));
      for (uint32_t y = lo; y < hi; ++y)
        if (greedy_end(y, k, x2, n2) >= 0) t2[o++] = make_t2(y, k, x2, n2);
    }
}

// key = cls * S1 + rank(y1), counts over x1.
__global__ void k_t1_count_g(int n1, uint32_t* cnt) {
  const uint32_t S1 = out_count(n1);
  const uint32_t key = blockIdx.x * blockDim.x + threadIdx.x;
  if (key >= 4 * S1) return;
  const int cls = key / S1;
  uint32_t y; int k;
  unrank(key % S1, &y, &k);
  uint32_t c = 0;
  for (uint32_t x1 = 0; x1 < (1u << n1); ++x1) {
    const int g = greedy_end(y, k, x1, n1);
    if (g >= 0 && class_of(bits_after(x1, n1, g)) == cls) ++c;
  }
  cnt[key] = c;
}

// key = cls * 2^n1 + x1, counts over y1.
__global__ void k_t1_count_s(int n1, uint32_t* cnt) {
  const uint32_t X1 = 1u << n1;
  const uint32_t key = blockIdx.x * blockDim.x + threadIdx.x;
  if (key >= 4 * X1) return;
  const int cls = key / X1;
  const uint32_t x1 = key % X1;
  uint32_t c = 0;
  for (uint32_t r = 0; r < out_count(n1); ++r) {
    uint32_t y; int k;
    unrank(r, &y, &k);
    const int g = greedy_end(y, k, x1, n1);
    if (g >= 0 && class_of(bits_after(x1, n1, g)) == cls) ++c;
  }
  cnt[key] = c;
}

// Serial exclusive scans (init only; at most a few thousand entries each).
__global__ void k_scans(int n1, int n2, const uint32_t* cnt2, uint32_t* off2, const uint32_t* cntg,
                        uint32_t* offg, const uint32_t* cnts, uint32_t* offs, uint32_t* cg) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint32_t acc = 0;
  for (uint32_t i = 0; i < (1u << n2); ++i) { off2[i] = acc; acc += cnt2[i]; }
  off2[1u << n2] = acc;
  const uint32_t S1 = out_count(n1);
  acc = 0;
  for (uint32_t i = 0; i < 4 * S1; ++i) {
    if (i % S1 == 0) cg[i / S1] = acc;
    offg[i] = acc;
    acc += cntg[i];
  }
  cg[4] = acc;
  acc = 0;
  for (uint32_t i = 0; i < 4 * (1u << n1); ++i) { offs[i] = acc; acc += cnts[i]; }
}

__global__ void k_t1_fill_g(int n1, const uint32_t* offg, uint4* t1g) {
  const uint32_t S1 = out_count(n1);
  const uint32_t key = blockIdx.x * blockDim.x + threadIdx.x;
  if (key >= 4 * S1) return;
  const int cls = key / S1;
  uint32_t y; int k;
  unrank(key % S1, &y, &k);
  uint32_t o = offg[key];
  for (uint32_t x1 = 0; x1 < (1u << n1); ++x1) {
    const int g = greedy_end(y, k, x1, n1);
    if (g >= 0 && class_of(bits_after(x1, n1, g)) == cls) t1g[o++] = make_t1(x1, n1, y, k, cls);
  }
}

__global__ void k_t1_fill_s(int n1, const uint32_t* offs, uint4* t1s) {
  const uint32_t X1 = 1u << n1;
  const uint32_t key = blockIdx.x * blockDim.x + threadIdx.x;
  if (key >= 4 * X1) return;
  const int cls = key / X1;
  const uint32_t x1 = key % X1;
  uint32_t o = offs[key];
  for (uint32_t r = 0; r < out_count(n1); ++r) {
    uint32_t y; int k;
    unrank(r, &y, &k);
    const int g = greedy_end(y, k, x1, n1);
    if (g >= 0 && class_of(bits_after(x1, n1, g)) == cls) t1s[o++] = make_t1(x1, n1, y, k, cls);
  }
}

inline size_t al(size_t b) { return (b + 255) & ~size_t(255); }
inline uint32_t pow3(int e) { uint32_t v = 1; while (e-- > 0) v *= 3; return v; }
inline uint32_t distinct_total(int m) { return 2u * pow3(m) - (1u << m); }

struct Layout {
  size_t t1s, t1g, t2, off2, n0, cnt2, cntg, offg, cnts, offs, cg, total;
};

Layout layout(int n) {
  const int n1 = (n + 1) / 2, n2 = n / 2;
  const size_t m1 = distinct_total(n1), m2 = distinct_total(n2);
  const size_t S1 = out_count(n1), X1 = size_t(1) << n1, X2 = size_t(1) << n2;
  Layout L;
  size_t o = 0;
  L.t1s = o; o += al(m1 * 16);
  L.t1g = o; o += al(m1 * 16);
  L.t2 = o; o += al(m2 * 16);
  L.off2 = o; o += al((X2 + 1) * 4);
  L.n0 = o; o += al(X2 * 4);
  L.cnt2 = o; o += al(X2 * 4);
  L.cntg = o; o += al(4 * S1 * 4);
  L.offg = o; o += al(4 * S1 * 4);
  L.cnts = o; o += al(4 * X1 * 4);
  L.offs = o; o += al(4 * X1 * 4);
  L.cg = o; o += al(8 * 4);
  L.total = o;
  return L;
}

}  // namespace

size_t table_bytes(int n) { return layout(n).total; }

hipError_t build_tables(int n, void* mem, hipStream_t s, Tables* out) {
  const int n1 = (n + 1) / 2, n2 = n / 2;
  const Layout L = layout(n);
  char* b = static_cast<char*>(mem);
  auto U32 = [&](size_t off) { return reinterpret_cast<uint32_t*>(b + off); };
  auto U4 = [&](size_t off) { return reinterpret_cast<uint4*>(b + off); };
  const uint32_t X1 = 1u << n1, X2 = 1u << n2, S1 = out_count(n1);
  const int tb = 128;
  hipLaunchKernelGGL(k_t2_count, dim3((X2 + tb - 1) / tb), dim3(tb), 0, s, n2, U32(L.cnt2), U32(L.n0));
  hipLaunchKernelGGL(k_t1_count_g, dim3((4 * S1 + tb - 1) / tb), dim3(tb), 0, s, n1, U32(L.cntg));
  hipLaunchKernelGGL(k_t1_count_s, dim3((4 * X1 + tb - 1) / tb), dim3(tb), 0, s, n1, U32(L.cnts));
  hipLaunchKernelGGL(k_scans, dim3(1), dim3(64), 0, s, n1, n2, U32(L.cnt2), U32(L.off2), U32(L.cntg),
                     U32(L.offg), U32(L.cnts), U32(L.offs), U32(L.cg));
  hipLaunchKernelGGL(k_t2_fill, dim3((X2 + tb - 1) / tb), dim3(tb), 0, s, n2, U32(L.off2), U4(L.t2));
  hipLaunchKernelGGL(k_t1_fill_g, dim3((4 * S1 + tb - 1) / tb), dim3(tb), 0, s, n1, U32(L.offg), U4(L.t1g));
  hipLaunchKernelGGL(k_t1_fill_s, dim3((4 * X1 + tb - 1) / tb), dim3(tb), 0, s, n1, U32(L.offs), U4(L.t1s));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  uint32_t cg[8];
  e = hipMemcpyAsync(cg, U32(L.cg), sizeof(cg), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  Tables t;
  t.n = n; t.n1 = n1; t.n2 = n2;
  t.m1 = distinct_total(n1);
  t.m2 = distinct_total(n2);
  for (int i = 0; i < 5; ++i) t.cg[i] = cg[i];
  t.t1s = U4(L.t1s); t.t1g = U4(L.t1g); t.t2 = U4(L.t2);
  t.off2 = U32(L.off2); t.n0_2 = U32(L.n0);
  if (t.cg[4] != t.m1) return hipErrorInvalidValue;  // table build inconsistent
  *out = t;
  return hipSuccess;
}

}  // namespace ba
