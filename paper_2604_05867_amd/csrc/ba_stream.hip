// Stream engine: the per-nonzero sweeps of the paper's method (Sections 3-4).
//
// Every nonzero W(y|x) is generated on the fly with its exact integer embedding
// count and visited once per sweep.  Work decomposition (MI355X-specific, see
// ba_internal.h for the tables): a block owns one right half x2 and a range of
// 64-entry chunks of T1; each wavefront takes one chunk, so lane l owns the pair
// (x1, y1) of entry chunk*64+l, i.e. the input x = x1 x2 and the prefix y1 of
// its outputs.  The lane runs the embedding-count DP of y1 over the positions of
// x2 once per chunk (in registers):
//   c[u]  = number of embeddings of y1[0:k1-u] in x1 x2[0:j]   (u = 0..k1)
//   l[0]  = emb(y1, x1),  l[j+1] = embeddings of y1 in x1 x2[0:j+1] whose last
//           bit sits at position j of x2,
// and then the wavefront walks the compatible suffixes y2 of x2 in lockstep
// (scalar loads of T2); the embedding count of y = y1 y2 is
//   emb(y, x) = sum_j l[j] * emb(y2, x2[j:n2])      (at most 11 integer MACs),
// because y2's first bit cannot be matched in x1 after y1's embedding (class
// rule), so y2 lies entirely in x2 to the right of y1's last bit.
//
// Ops: scatter  r(y) += p(x) emb(y,x)   (outputs with |y| <= k0 in LDS first)
//      scatter over orbits (Appendix A, Algorithm 7; iterates invariant under
//               complement and reversal): only inputs x that represent their orbit
//               take part, r(rep y) += (|O_x| / |O_y|) p(x) emb(y,x) (the split
//               layout at rep y's split into the same lengths), and the other
//               outputs of each orbit are filled in after the combine
//      gather   G(x) += emb(y,x) v(y)    (v in split layout V2[rank(y2)][rank(y1)])
//      init     H(x) += w_k emb log emb, Hd(x) += s_k w_k emb log emb (fixed-point
//               integer atomics: the same bits in every run)
//      row      dense row of one x (parity hook)
//      verify   per-row length sums and nonzero counts
#include "ba_internal.h"

namespace ba {
namespace {

__device__ __forceinline__ uint32_t byte_of(const uint4& t, int j) {
  const uint32_t w = (j < 4) ? t.y : ((j < 8) ? t.z : t.w);
  return (w >> (8 * (j & 3))) & 0xffu;
}

template <typename T>
__device__ __forceinline__ void atomic_add(T* p, T v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void lds_add(T* p, T v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// DPP row shifts (within 16-lane rows; lanes without a source read 0).
template <int D>
__device__ __forceinline__ int dpp_row_shr(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x110 + D, 0xf, 0xf, true);
}
__device__ __forceinline__ int dpp_row_shl1(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x101, 0xf, 0xf, true);
}
template <int D>
__device__ __forceinline__ float shr_t(float v) {
  return __int_as_float(dpp_row_shr<D>(__float_as_int(v)));
}
template <int D>
__device__ __forceinline__ double shr_t(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_row_shr<D>(int(b & 0xffffffffll));
  const int hi = dpp_row_shr<D>(int(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// Segmented inclusive sum over lanes of a 16-lane row: m_d = 1 when lane-d is in
// the same segment.  Afterwards the last lane of each segment holds its sum.
template <typename T>
__device__ __forceinline__ T seg_row_sum(T v, T m1, T m2, T m4, T m8) {
  v = fma(shr_t<1>(v), m1, v);
  v = fma(shr_t<2>(v), m2, v);
  v = fma(shr_t<4>(v), m4, v);
  v = fma(shr_t<8>(v), m8, v);
  return v;
}

constexpr uint32_t binom_dev(int n, int k) {
  uint32_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * uint32_t(n - k + i) / uint32_t(i);
  return r;
}

template <typename T, int OP>
__global__ __launch_bounds__(kBlock) void k_stream(Tables tb, Group<T> g, int k0, int parts,
                                                   StreamExtra ex) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr bool ORB = OP == kOpScatterOrbit;         // Algorithm 7
  constexpr bool SCAT = OP == kOpScatter || ORB;
  const int n1 = tb.n1, n2 = tb.n2;
  const uint32_t x2 = blockIdx.x / parts;
  const uint32_t part = blockIdx.x % parts;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const uint32_t S1 = out_count(n1);
  const uint32_t X1 = 1u << n1;

  // Instances of this launch's tile and which of them are still iterating.
  int b0 = 0, nbt = 1;
  uint32_t live = 1;
  if (SCAT || OP == kOpGather || OP == kOpInit) {
    b0 = blockIdx.y * kTile;
    nbt = min(kTile, g.nb - b0);
    live = 0;
    for (int b = 0; b < nbt; ++b)
      if (OP == kOpInit || !g.st[b0 + b].converged) live |= 1u << b;
    if (live == 0) return;  // uniform across the block
  }
  if (OP == kOpRow && x2 != (ex.target_x & ((1u << n2) - 1u))) return;

  const uint32_t nshort = (2u << k0) - 1u;
  T* rs = reinterpret_cast<T*>(smem);  // scatter: [nbt][nshort]
  T* gs = reinterpret_cast<T*>(smem);  // gather:  [nbt][X1]
  if (SCAT) {
    for (uint32_t i = threadIdx.x; i < nshort * nbt; i += kBlock) rs[i] = T(0);
  } else if (OP == kOpGather) {
    for (uint32_t i = threadIdx.x; i < X1 * nbt; i += kBlock) gs[i] = T(0);
  }
  __syncthreads();

  const uint4* __restrict__ t1 = (OP == kOpGather || SCAT) ? tb.t1g : tb.t1s;
  const uint32_t o2 = tb.off2[x2];
  const uint32_t c2 = tb.off2[x2 + 1] - o2;
  const uint32_t z0 = tb.n0_2[x2];
  const uint32_t nchunk = (tb.m1 + kWave - 1) / kWave;
  const uint32_t cpp = (nchunk + parts - 1) / parts;
  const uint32_t cb = part * cpp;
  const uint32_t ce = min(nchunk, cb + cpp);

  double wk[kNMax + 1], swk[kNMax + 1];
  if (OP == kOpInit) {
    // only used for single-instance init launches (nbt == 1 enforced by the host);
    // s_k w_k is taken pre-scaled by 2^-e (see hd_exponent)
    const int e = hd_exponent(g.cs[b0], g.n);
    for (int k = 0; k <= kNMax; ++k) { wk[k] = g.cs[b0].w[k]; swk[k] = ldexp(g.cs[b0].sw[k], -e); }
  }

  for (uint32_t ch = cb + wave; ch < ce; ch += kBlock / kWave) {
    const uint32_t e = ch * kWave + lane;
    const bool valid = e < tb.m1;
    const uint4 ent = valid ? t1[e] : make_uint4(0u, 0u, 0u, 0u);
    const uint32_t x1 = ent.x & 1023u;
    const uint32_t y1 = (ent.x >> 10) & 1023u;
    const int k1 = (ent.x >> 20) & 15;
    const uint32_t x = (x1 << n2) | x2;
    if (OP == kOpRow) {
      if (__ballot(valid && x == ex.target_x) == 0) continue;
    }

    // Embedding-count DP of y1 across x2 (c[u] for prefix length k1-u).
    uint32_t c[kHalfMax + 1];
#pragma unroll
    for (int u = 0; u <= kHalfMax; ++u) c[u] = byte_of(ent, u);
    const uint32_t kmask = (1u << k1) - 1u;
    const uint32_t m1 = y1 & kmask, m0 = ~y1 & kmask;
    uint32_t l[kHalfMax + 1];
    l[0] = c[0];
#pragma unroll
    for (int j = 0; j < kHalfMax; ++j) {
      if (j < n2) {
        const uint32_t mb = ((x2 >> (n2 - 1 - j)) & 1u) ? m1 : m0;
        const uint32_t before = c[0];
#pragma unroll
        for (int u = 0; u < kHalfMax; ++u) c[u] += ((mb >> u) & 1u) * c[u + 1];
        l[j + 1] = c[0] - before;
      } else {
        l[j + 1] = 0u;
      }
    }

    // Per-lane state of the op.
    T pl[kTile];
    T acc[kTile];
    double ah = 0.0, ahd = 0.0;
    const uint32_t A1 = y1 | (1u << k1);
    const uint32_t R1 = A1 - 1u;  // rank of y1
    const uint32_t ry1 = (ORB && k1) ? (__brev(y1) >> (32 - k1)) : 0u;  // reversal of y1
    // Scatter: lanes are sorted by (class, y1, x1), so lanes with the same y1 form
    // contiguous runs that, for a given y2, add into the same output.  Per run and
    // 16-lane row a segmented Hillis-Steele scan over DPP row shifts leaves the run's
    // sum in its last lane (sm_d = 1 when lane-d is in the same run and row).
    T sm1 = T(0), sm2 = T(0), sm4 = T(0), sm8 = T(0);
    bool emit = false;
    if (SCAT) {
      // Algorithm 7: an input that is not its orbit's representative adds nothing;
      // a representative stands for its |O_x| orbit members
      T ox = T(1);
      if constexpr (ORB) {
        uint32_t xr, xs;
        orbit_of(x, n1 + n2, xr, xs);
        ox = (xr == x) ? T(xs) : T(0);
      }
#pragma unroll
      for (int b = 0; b < kTile; ++b)
        pl[b] = (b < nbt && valid) ? ox * g.p[(size_t)(b0 + b) * g.xs + x] : T(0);
      const int key = valid ? int(((ent.x >> 24) & 3u) << 12 | R1) : -1;
      const int rl = lane & 15;
      // The DPP reads run with every lane active (a disabled source lane reads 0).
      const int kd1 = dpp_row_shr<1>(key), kd2 = dpp_row_shr<2>(key);
      const int kd4 = dpp_row_shr<4>(key), kd8 = dpp_row_shr<8>(key);
      const int ku1 = dpp_row_shl1(key);
      sm1 = (rl >= 1 && kd1 == key) ? T(1) : T(0);
      sm2 = (rl >= 2 && kd2 == key) ? T(1) : T(0);
      sm4 = (rl >= 4 && kd4 == key) ? T(1) : T(0);
      sm8 = (rl >= 8 && kd8 == key) ? T(1) : T(0);
      emit = (rl == 15) || (ku1 != key);
    }
    if (OP == kOpGather) {
#pragma unroll
      for (int b = 0; b < kTile; ++b) acc[b] = T(0);
    }

    // Three groups of y2: empty (all lanes), starting with 0, starting with 1.
#pragma unroll 1
    for (int grp = 0; grp < 3; ++grp) {
      uint32_t qb, qe, lo, hi;
      if (grp == 0) { qb = o2; qe = o2 + 1; lo = 0; hi = tb.m1; }
      else if (grp == 1) { qb = o2 + 1; qe = o2 + 1 + z0; lo = tb.cg[0]; hi = tb.cg[2]; }
      else { qb = o2 + 1 + z0; qe = o2 + c2; lo = tb.cg[1]; hi = tb.cg[3]; }
      const uint32_t cs0 = ch * kWave, ce0 = cs0 + kWave;
      if (qb >= qe || ce0 <= lo || cs0 >= hi) continue;  // uniform
      const bool ok = valid && e >= lo && e < hi;
      // One compatible suffix y2 (T2 entry t, uniform across the wavefront).
      auto body = [&](const uint4& t) {
        const uint32_t y2 = t.x & 1023u;
        const int k2 = (t.x >> 10) & 15;
        const int jmax = (t.x >> 14) & 15;
        uint32_t emb = 0;
#pragma unroll
        for (int j = 0; j <= kHalfMax; ++j)
          if (j <= jmax) emb = __umul24(l[j], byte_of(t, j)) + emb;
        const int k = k1 + k2;
        if (SCAT) {
          // All lanes take part in the run reduction (inactive lanes add 0), then
          // the last lane of each run (per 16-lane row) issues one atomic.
          const T fe = ok ? T(emb) : T(0);
          uint32_t rank = (A1 << k2) + y2 - 1u;
          size_t i2 = size_t((1u << k2) - 1u + y2) * S1 + R1;
          T oy = T(1);  // orbit mode: 1 / |O_y|
          if constexpr (ORB) {
            // the run's output y (shared by its lanes) goes to its representative,
            // weighted 1 / |O_y|, at the representative's split into the same
            // lengths k1 + k2 (the combine sums every split of an output).  The
            // reversal of y1 y2 is rev(y2) rev(y1): rev(y1) is the lane's, rev(y2)
            // is uniform across the wavefront.
            const uint32_t yv = (y1 << k2) | y2, mk = (1u << k) - 1u;
            const uint32_t ry = ((k2 ? (__brev(y2) >> (32 - k2)) : 0u) << k1) | ry1;
            const uint32_t a = yv, bb = yv ^ mk, cc = ry, dd = ry ^ mk;
            const uint32_t yr = min(min(a, bb), min(cc, dd));
            const uint32_t ys = 1u + (bb != a ? 1u : 0u) + ((cc != a && cc != bb) ? 1u : 0u) +
                                ((dd != a && dd != bb && dd != cc) ? 1u : 0u);
            rank = mk + yr;
            i2 = size_t((1u << k2) - 1u + (yr & ((1u << k2) - 1u))) * S1 + ((1u << k1) - 1u + (yr >> k2));
            oy = ys == 4u ? T(0.25) : (ys == 2u ? T(0.5) : T(1));  // 1 / |O_y|, exact
          }
#pragma unroll
          for (int b = 0; b < kTile; ++b) {
            if (b >= nbt || !((live >> b) & 1u)) continue;  // uniform
            T cv = seg_row_sum(pl[b] * fe, sm1, sm2, sm4, sm8);
            if (emit && ok && cv != T(0)) {
              if constexpr (ORB) cv = cv * oy;
              if (k <= k0) lds_add(&rs[b * nshort + rank], cv);
              else atomic_add(&g.v2[(size_t)(b0 + b) * g.v2s + i2], cv);
            }
          }
          return;
        }
        if (!ok) return;
        if (OP == kOpGather) {
          const size_t idx = size_t((1u << k2) - 1u + y2) * S1 + R1;
          const T fe = T(emb);
#pragma unroll
          for (int b = 0; b < kTile; ++b)
            if (b < nbt && ((live >> b) & 1u)) acc[b] += fe * g.v2[(size_t)(b0 + b) * g.v2s + idx];
        } else if (OP == kOpInit) {
          const double le = log(double(emb));
          const double t0 = double(emb) * le;
          ah += wk[k] * t0;
          ahd += swk[k] * t0;
        } else if (OP == kOpRow) {
          if (x == ex.target_x) ex.row_dense[(A1 << k2) + y2 - 1u] = emb;
        } else if (OP == kOpVerify) {
          atomicAdd(&ex.bins[(size_t)x * (tb.n + 2) + k], emb);
          atomicAdd(&ex.bins[(size_t)x * (tb.n + 2) + tb.n + 1], 1u);
          atomicMax(&ex.stats[5], (unsigned long long)emb);
        }
      };
      // Four suffixes per trip: their scalar loads (and, in the gather, their
      // V2 loads) are in flight together.
      uint32_t q = qb;
#pragma unroll 1
      for (; q + 4u <= qe; q += 4u) {
        const uint4 ta = tb.t2[q], tbb = tb.t2[q + 1u], tc = tb.t2[q + 2u], td = tb.t2[q + 3u];
        body(ta);
        body(tbb);
        body(tc);
        body(td);
      }
#pragma unroll 1
      for (; q < qe; ++q) body(tb.t2[q]);
    }
    if (OP == kOpGather && valid) {
#pragma unroll
      for (int b = 0; b < kTile; ++b)
        if (b < nbt && ((live >> b) & 1u)) lds_add(&gs[b * X1 + x1], acc[b]);
    }
    if (OP == kOpInit && valid) {
      // order-independent: H and Hd are the same bits in every run
      fix_add(ex.fix + 2 * (size_t)x, ah);
      fix_add(ex.fix + 2 * (g.xs + (size_t)x), ahd);
    }
  }

  if (SCAT) {
    __syncthreads();
    for (int b = 0; b < nbt; ++b) {
      if (!((live >> b) & 1u)) continue;
      for (uint32_t i = threadIdx.x; i < nshort; i += kBlock) {
        const T v = rs[b * nshort + i];
        if (v != T(0)) atomic_add(&g.r[(size_t)(b0 + b) * g.ys + i], v);
      }
    }
  } else if (OP == kOpGather) {
    __syncthreads();
    for (int b = 0; b < nbt; ++b) {
      if (!((live >> b) & 1u)) continue;
      for (uint32_t i = threadIdx.x; i < X1; i += kBlock) {
        const T v = gs[b * X1 + i];
        if (v != T(0)) atomic_add(&g.g[(size_t)(b0 + b) * g.xs + ((i << n2) | x2)], v);
      }
    }
  }
}

// Verify finish: one thread per row checks sum_{|y|=k} emb = C(n,k) and records
// nnz statistics.  stats = {total nnz, rows failing, 0, min nnz, max nnz, max emb}.
__global__ void k_verify_finish(int n, const unsigned int* bins, unsigned long long* stats) {
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= (1u << n)) return;
  const unsigned int* b = bins + (size_t)x * (n + 2);
  bool ok = true;
  for (int k = 0; k <= n; ++k) ok = ok && (b[k] == binom_dev(n, k));
  const unsigned long long nnz = b[n + 1];
  atomicAdd(&stats[0], nnz);
  if (!ok) atomicAdd(&stats[1], 1ull);
  atomicMin(&stats[3], nnz);
  atomicMax(&stats[4], nnz);
}

// r(y) for |y| > k0 from the split layout of the scatter: the sum over the splits
// y = y1 y2 (|y1| <= n1, |y2| <= n2) of R2[rank(y2)][rank(y1)].  Outputs with
// |y| <= k0 already hold their LDS-accumulated values.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_combine_r(Group<T> g, int n1, int n2, int k0) {
  const int b = blockIdx.y;
  if (g.st[b].converged) return;
  const uint32_t Y = out_count(g.n);
  const uint32_t S1 = out_count(n1);
  const T* r2 = g.v2 + (size_t)b * g.v2s;
  T* r = g.r + (size_t)b * g.ys;
  for (uint32_t y = blockIdx.x * blockDim.x + threadIdx.x; y < Y; y += gridDim.x * blockDim.x) {
    const int k = 31 - __clz(y + 1u);
    if (k <= k0) continue;
    const uint32_t yb = y + 1u - (1u << k);
    T acc = T(0);
    const int lo = k > n2 ? k - n2 : 0, hi = k < n1 ? k : n1;
    for (int k1 = lo; k1 <= hi; ++k1) {
      const int k2 = k - k1;
      const uint32_t y1 = yb >> k2, y2 = yb & ((1u << k2) - 1u);
      acc += r2[size_t((1u << k2) - 1u + y2) * S1 + ((1u << k1) - 1u + y1)];
    }
    r[y] = acc;
  }
}

// Row compaction: dense counts by rank -> (rank, emb) in increasing rank.
// One block; ballot-free two-level scan per 1024-rank window.
__global__ __launch_bounds__(1024) void k_row_compact(const uint32_t* dense, uint32_t total,
                                                      uint32_t* rank_out, uint32_t* emb_out,
                                                      int cap, uint32_t* nnz_dev) {
  __shared__ uint32_t sc[1024];
  __shared__ uint32_t base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (uint32_t w0 = 0; w0 < total; w0 += 1024) {
    const uint32_t r = w0 + threadIdx.x;
    const uint32_t v = (r < total) ? dense[r] : 0u;
    const uint32_t f = v != 0u;
    sc[threadIdx.x] = f;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
      const uint32_t t = (threadIdx.x >= off) ? sc[threadIdx.x - off] : 0u;
      __syncthreads();
      sc[threadIdx.x] += t;
      __syncthreads();
    }
    const uint32_t pos = base + sc[threadIdx.x] - f;
    if (f && pos < (uint32_t)cap) {
      rank_out[pos] = r;
      emb_out[pos] = v;
    }
    __syncthreads();
    if (threadIdx.x == 1023) base += sc[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) *nnz_dev = base;
}

// H(x) and Hd(x) from the fixed-point words of the init pass (one thread per input).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fix_finish(Group<T> g, StreamExtra ex) {
  const int b = blockIdx.y;
  const uint32_t X = 1u << g.n;
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= X) return;
  const unsigned long long* w = ex.fix + (size_t)b * 4 * g.xs;
  const int e = hd_exponent(g.cs[b], g.n);
  ex.h[(size_t)b * g.xs + x] = fix_value(w + 2 * (size_t)x);
  ex.hd[(size_t)b * g.xs + x] = ldexp(fix_value(w + 2 * (g.xs + (size_t)x)), e);
}

template <typename T, int OP>
hipError_t launch_op(const Tables& tb, const Group<T>& g, int k0, const StreamExtra& ex, hipStream_t s) {
  const uint32_t X2 = 1u << tb.n2;
  const uint32_t nchunk = (tb.m1 + kWave - 1) / kWave;
  // Spread each x2 over several blocks so that the grid holds >= ~2048 blocks.
  int parts = 1;
  if (OP != kOpRow) {
    while ((uint64_t)X2 * parts < 2048 && (uint32_t)parts * 8 < nchunk) parts *= 2;
  }
  constexpr bool SCAT = OP == kOpScatter || OP == kOpScatterOrbit;
  const int tiles = (SCAT || OP == kOpGather) ? (g.nb + kTile - 1) / kTile : (OP == kOpInit ? g.nb : 1);
  const int nbt = (SCAT || OP == kOpGather) ? (g.nb < kTile ? g.nb : kTile) : 1;
  size_t lds = 0;
  if (SCAT) lds = size_t((2u << k0) - 1u) * nbt * sizeof(T);
  if (OP == kOpGather) lds = size_t(1u << tb.n1) * nbt * sizeof(T);
  if (OP == kOpInit) {
    // one launch per instance (its own weights); per-lane partial sums go to the
    // fixed-point words, which k_fix_finish turns into H and Hd
    hipError_t e = launch_fill_zero(ex.fix, (size_t)g.nb * g.xs * 32, s);
    if (e != hipSuccess) return e;
    for (int b = 0; b < g.nb; ++b) {
      Group<T> gb = g;
      gb.nb = 1;
      gb.st = g.st + b;
      gb.cs = g.cs + b;
      StreamExtra eb = ex;
      eb.fix = ex.fix + (size_t)b * 4 * g.xs;
      hipLaunchKernelGGL((k_stream<T, OP>), dim3(X2 * parts, 1), dim3(kBlock), 0, s, tb, gb, k0,
                         parts, eb);
    }
    const uint32_t X = 1u << g.n;
    hipLaunchKernelGGL(k_fix_finish<T>, dim3((X + kBlock - 1) / kBlock, g.nb), dim3(kBlock), 0, s, g, ex);
    return hipGetLastError();
  }
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stream<T, OP>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_stream<T, OP>), dim3(X2 * parts, tiles), dim3(kBlock), lds, s, tb, g, k0,
                     parts, ex);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_stream(StreamOp op, const Tables& tb, const Group<T>& g, int k0,
                         const StreamExtra& ex, hipStream_t s) {
  switch (op) {
    case kOpScatter: return launch_op<T, kOpScatter>(tb, g, k0, ex, s);
    case kOpScatterOrbit: return launch_op<T, kOpScatterOrbit>(tb, g, k0, ex, s);
    case kOpGather: return launch_op<T, kOpGather>(tb, g, k0, ex, s);
    case kOpInit: return launch_op<T, kOpInit>(tb, g, k0, ex, s);
    case kOpRow: return launch_op<T, kOpRow>(tb, g, k0, ex, s);
    case kOpVerify: {
      hipError_t e = launch_op<T, kOpVerify>(tb, g, k0, ex, s);
      if (e != hipSuccess) return e;
      const uint32_t X = 1u << tb.n;
      hipLaunchKernelGGL(k_verify_finish, dim3((X + 255) / 256), dim3(256), 0, s, tb.n, ex.bins,
                         ex.stats);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_stream<float>(StreamOp, const Tables&, const Group<float>&, int,
                                         const StreamExtra&, hipStream_t);
template hipError_t launch_stream<double>(StreamOp, const Tables&, const Group<double>&, int,
                                          const StreamExtra&, hipStream_t);

// After the orbit scatter: the outputs that do not represent their orbit take the
// representative's value (Theorem 4: r(g y) = r(y) for an invariant input law).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_orbit_expand(Group<T> g) {
  const int b = blockIdx.y;
  if (g.st[b].converged) return;
  const uint32_t Y = out_count(g.n);
  T* r = g.r + (size_t)b * g.ys;
  for (uint32_t y = blockIdx.x * blockDim.x + threadIdx.x; y < Y; y += gridDim.x * blockDim.x) {
    const int k = 31 - __clz(y + 1u);
    const uint32_t bits = y + 1u - (1u << k);
    uint32_t rep, size;
    orbit_of(bits, k, rep, size);
    if (rep != bits) r[y] = r[(1u << k) - 1u + rep];
  }
}

template <typename T>
hipError_t launch_orbit_expand(const Group<T>& g, hipStream_t s) {
  const uint32_t Y = out_count(g.n);
  uint32_t grid = (Y + kBlock - 1) / kBlock;
  if (grid > 8192u) grid = 8192u;
  hipLaunchKernelGGL(k_orbit_expand<T>, dim3(grid, g.nb), dim3(kBlock), 0, s, g);
  return hipGetLastError();
}

template hipError_t launch_orbit_expand<float>(const Group<float>&, hipStream_t);
template hipError_t launch_orbit_expand<double>(const Group<double>&, hipStream_t);

template <typename T>
hipError_t launch_combine_r(const Group<T>& g, int n1, int n2, int k0, hipStream_t s) {
  uint32_t grid = (out_count(g.n) + kBlock - 1) / kBlock;
  if (grid > 4096u) grid = 4096u;
  hipLaunchKernelGGL(k_combine_r<T>, dim3(grid, g.nb), dim3(kBlock), 0, s, g, n1, n2, k0);
  return hipGetLastError();
}
template hipError_t launch_combine_r<float>(const Group<float>&, int, int, int, hipStream_t);
template hipError_t launch_combine_r<double>(const Group<double>&, int, int, int, hipStream_t);

int stream_lds_limit() {
  static int cached = 0;
  if (cached) return cached;
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess && v > 0)
    cached = v;
  else if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
    cached = v;
  else
    cached = 65536;
  return cached;
}

hipError_t launch_row_compact(const uint32_t* dense, int n, uint32_t* rank_out, uint32_t* emb_out,
                              int cap, uint32_t* nnz_dev, hipStream_t s) {
  hipLaunchKernelGGL(k_row_compact, dim3(1), dim3(1024), 0, s, dense, out_count(n), rank_out,
                     emb_out, cap, nnz_dev);
  return hipGetLastError();
}

}  // namespace ba
