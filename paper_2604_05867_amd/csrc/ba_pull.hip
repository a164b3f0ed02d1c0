// Pull form of sweep 1 (Section 5): r(y) = sum over the length-n supersequences x
// of y of p(x) emb(y, x), without atomics.
//
// A length-k output has N_k = sum_{i <= n-k} C(n, i) supersequences (Lemma 7).
// Each supersequence x of y is named by a position set S with |S| <= n - k: the
// positions that the leftmost embedding of y skips before it completes, together
// with the positions after it whose symbol differs from y's last symbol.
// Index i in [0, N_k) names one: w = |S| is the smallest w with
// i < sum_{j <= w} C(n, j), and S is the (i - sum_{j < w} C(n, j))-th w-subset
// in lexicographic order (the order of Section 5.1's unranking).  Given S, the
// positions outside S carry y in order followed by copies of y's last symbol,
// and every position in S carries the complement of the symbol at the next
// position outside S (of y's last symbol if there is none), so the leftmost
// embedding skips exactly S.  (The construction of Section 5.2 as printed writes 0
// after the embedding instead of y's last symbol, which is not one-to-one.)
//
// Work decomposition: the supersequence indices of every output are cut into
// chunks of kPullChunk; one thread takes one (output, chunk) item, runs the
// embedding-count DP of y in x for every index of its chunk (registers, 21
// counters) and accumulates p(x) emb for up to kTile instances; it writes one
// partial per instance, and a second kernel adds the partials of every output in
// a fixed order.  The result is deterministic: no atomics, fixed summation order.
#include "ba_internal.h"

namespace ba {
namespace {

constexpr int kPullChunk = 512;

struct PullPlan {
  int n;
  uint32_t chunks[kNMax + 1];    // chunks per output of length k
  uint32_t item_off[kNMax + 2];  // first item of length k
  uint32_t cum[kNMax + 2];       // cum[w] = sum_{j < w} C(n, j)
};

struct Binom {
  uint32_t c[kNMax + 1][kNMax + 1];
};

constexpr Binom make_binom() {
  Binom b{};
  for (int a = 0; a <= kNMax; ++a) {
    b.c[a][0] = 1;
    for (int k = 1; k <= a; ++k) b.c[a][k] = b.c[a - 1][k - 1] + (k <= a - 1 ? b.c[a - 1][k] : 0u);
  }
  return b;
}

__constant__ Binom kBinom = make_binom();

// x (MSB = position 0) of supersequence index i of y (k bits, MSB first).
__device__ __forceinline__ uint32_t supersequence_of(const PullPlan& P, uint32_t i, uint32_t y, int k) {
  const int n = P.n;
  int w = 0;
  while (i >= P.cum[w + 1]) ++w;
  // S from its lexicographic rank j: the reflected set {n-1-s : s in S} has
  // colexicographic rank C(n,w) - 1 - j in the combinatorial number system, read
  // off greedily by the largest binomial C(c, t) that fits, t = w .. 1
  uint32_t N = kBinom.c[n][w] - 1u - (i - P.cum[w]);
  uint32_t smask = 0;
  int c = n - 1;
  for (int t = w; t >= 1; --t) {
    while (kBinom.c[c][t] > N) --c;  // stops at c = t - 1 at the latest: C(t-1, t) = 0
    N -= kBinom.c[c][t];
    smask |= 1u << (n - 1 - c);
    --c;
  }
  // right to left: `carry` is the symbol at the nearest position outside S seen so
  // far (y's last symbol before any); outside S the m-th position (from the left)
  // holds y_m, or y's last symbol for m >= k
  const uint32_t last = k > 0 ? (y & 1u) : 0u;
  uint32_t carry = last, x = 0;
  for (int pos = n - 1; pos >= 0; --pos) {
    uint32_t bit;
    if ((smask >> pos) & 1u) {
      bit = 1u - carry;
    } else {
      const int m = pos - __popc(smask & ((1u << pos) - 1u));
      bit = m < k ? (y >> (k - 1 - m)) & 1u : last;
      carry = bit;
    }
    x |= bit << (n - 1 - pos);
  }
  return x;
}

// Number of embeddings of y (k bits, MSB first) in x (n bits): c[j] counts the
// embeddings of y[0:j] in the prefix of x read so far.
__device__ __forceinline__ uint32_t emb_count(uint32_t x, int n, uint32_t y, int k) {
  // ybit(j) = y_j, j = 0..k-1, as bit j of yr
  uint32_t yr = 0;
  for (int q = 0; q < k; ++q) yr |= ((y >> (k - 1 - q)) & 1u) << q;
  uint32_t c[kNMax + 1];
  c[0] = 1;
#pragma unroll
  for (int j = 1; j <= kNMax; ++j) c[j] = 0;
  for (int pos = 0; pos < n; ++pos) {
    const uint32_t xb = (x >> (n - 1 - pos)) & 1u;
#pragma unroll
    for (int j = kNMax; j >= 1; --j) c[j] += (((yr >> (j - 1)) & 1u) == xb) ? c[j - 1] : 0u;
  }
  uint32_t out = c[0];
#pragma unroll
  for (int j = 1; j <= kNMax; ++j) out = (j == k) ? c[j] : out;
  return out;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_pull_items(PullPlan P, Group<T> g, int b0, int nbt, T* partial,
                                                       uint32_t items) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= items) return;
  int k = 0;
  while (q >= P.item_off[k + 1]) ++k;
  const uint32_t local = q - P.item_off[k];
  const uint32_t y = local / P.chunks[k], chunk = local - y * P.chunks[k];
  const uint32_t Nk = P.cum[P.n - k + 1];
  const uint32_t i0 = chunk * kPullChunk, i1 = min(Nk, i0 + kPullChunk);
  T acc[kTile];
#pragma unroll
  for (int t = 0; t < kTile; ++t) acc[t] = T(0);
  for (uint32_t i = i0; i < i1; ++i) {
    const uint32_t x = supersequence_of(P, i, y, k);
    const T e = T(emb_count(x, P.n, y, k));
#pragma unroll
    for (int t = 0; t < kTile; ++t)
      if (t < nbt && !g.st[b0 + t].converged) acc[t] += g.p[(size_t)(b0 + t) * g.xs + x] * e;
  }
#pragma unroll
  for (int t = 0; t < kTile; ++t)
    if (t < nbt) partial[(size_t)t * items + q] = acc[t];
}

// r(y) = sum of y's partials in chunk order.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pull_finish(PullPlan P, Group<T> g, int b0, int nbt,
                                                        const T* partial, uint32_t items) {
  const uint32_t R = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (t >= nbt || R >= out_count(P.n) || g.st[b0 + t].converged) return;
  const int k = 31 - __clz(R + 1u);
  const uint32_t y = R + 1u - (1u << k);
  const uint32_t base = P.item_off[k] + y * P.chunks[k];
  T s = T(0);
  for (uint32_t c = 0; c < P.chunks[k]; ++c) s += partial[(size_t)t * items + base + c];
  g.r[(size_t)(b0 + t) * g.ys + R] = s;
}

PullPlan make_plan(int n, uint32_t* items) {
  PullPlan P{};
  P.n = n;
  uint64_t c = 1, cum = 0;
  for (int w = 0; w <= n; ++w) {
    P.cum[w] = uint32_t(cum);
    cum += c;
    c = c * uint64_t(n - w) / uint64_t(w + 1);
  }
  P.cum[n + 1] = uint32_t(cum);
  uint64_t off = 0;
  for (int k = 0; k <= n; ++k) {
    const uint64_t Nk = P.cum[n - k + 1];
    P.chunks[k] = uint32_t((Nk + kPullChunk - 1) / kPullChunk);
    P.item_off[k] = uint32_t(off);
    off += (uint64_t(1) << k) * P.chunks[k];
  }
  P.item_off[n + 1] = uint32_t(off);
  *items = uint32_t(off);
  return P;
}

}  // namespace

size_t pull_partial_bytes(int n, int nb, size_t esz) {
  uint32_t items = 0;
  (void)make_plan(n, &items);
  const int nbt = nb < kTile ? nb : kTile;
  return size_t(items) * size_t(nbt) * esz;
}

template <typename T>
hipError_t launch_pull(const Group<T>& g, T* partial, hipStream_t s) {
  uint32_t items = 0;
  const PullPlan P = make_plan(g.n, &items);
  for (int b0 = 0; b0 < g.nb; b0 += kTile) {
    const int nbt = (g.nb - b0) < kTile ? (g.nb - b0) : kTile;
    hipLaunchKernelGGL(k_pull_items<T>, dim3((items + kBlock - 1) / kBlock), dim3(kBlock), 0, s, P, g, b0, nbt,
                       partial, items);
    hipLaunchKernelGGL(k_pull_finish<T>, dim3((out_count(g.n) + kBlock - 1) / kBlock, nbt), dim3(kBlock), 0, s,
                       P, g, b0, nbt, (const T*)partial, items);
  }
  return hipGetLastError();
}

template hipError_t launch_pull<float>(const Group<float>&, float*, hipStream_t);
template hipError_t launch_pull<double>(const Group<double>&, double*, hipStream_t);

}  // namespace ba
