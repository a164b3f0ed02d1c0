// Persistent BA iterations for small instances: one block per instance runs a
// whole chunk of iterations (Section 2.3: output law, refined input law,
// normalisation, repeated) with every intermediate array in LDS, so a chunk of a
// batched group is one launch however many iterations it holds.
//
// The two products are the factored engine's position-by-position stages, one
// position per step (the deletion channel acts on each input bit independently,
// Section 2.2):
//   forward   F_0[eps][x] = p(x) e^{-M},
//             F_{i+1}[y][s] = F_i[y][0 s] + F_i[y][1 s] + F_i[y[:-1]][last(y) s],
//             F_n[y] = r(y) e^{-M};
//   backward  B_n[y] = v(y) = w_k log r(y),  B_i[y][b s] = B_{i+1}[y][s] + B_{i+1}[y b][s],
//             B_0[eps][x] = G(x) = sum_y emb(y,x) v(y);
// then D(x) = H(x) - G(x) - M (Section 3's partial sums), the Blahut record of the
// iterate (L = log sum p e^D, U = max D, I = sum p D) and the update
// log p <- log p + D - L (floored), exactly as the multi-launch path forms them
// (the same update_params_rec and update_value), up to the order of additions.
//
// Layout: F_i / B_i row-major by rank (row y of a stage with 2^w columns at y 2^w),
// ping-ponging between two LDS arrays of 2^(n+1) values.  FP32 fits n <= 13 and
// FP64 n <= 12 in the 160 KB of a CU; larger groups use the multi-launch path.
#include "ba_internal.h"
#include "ba_part.h"

namespace ba {
namespace {

// NT threads per block (tuned: 256, 512 or 1024); each thread holds up to 2^13 / NT
// inputs' D values in registers.
constexpr int kPersistMaxInputs = 1 << 13;

__device__ __forceinline__ int rank_length(uint32_t r) { return 31 - __clz(r + 1u); }

// Four consecutive LDS values (16-byte aligned for FP32; two 16-byte halves for FP64).
template <typename T>
struct V4 {
  T v[4];
};
template <typename T>
__device__ __forceinline__ V4<T> v4_ld(const T* p) {
  V4<T> r;
  if constexpr (sizeof(T) == 4) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    r.v[0] = a.x; r.v[1] = a.y; r.v[2] = a.z; r.v[3] = a.w;
  } else {
    const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
    r.v[0] = a.x; r.v[1] = a.y; r.v[2] = b.x; r.v[3] = b.y;
  }
  return r;
}
template <typename T>
__device__ __forceinline__ void v4_st(T* p, const V4<T>& a) {
  if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(a.v[0], a.v[1], a.v[2], a.v[3]);
  } else {
    reinterpret_cast<double2*>(p)[0] = make_double2(a.v[0], a.v[1]);
    reinterpret_cast<double2*>(p)[1] = make_double2(a.v[2], a.v[3]);
  }
}
template <typename T>
__device__ __forceinline__ V4<T> v4_add(const V4<T>& a, const V4<T>& b) {
  V4<T> r;
#pragma unroll
  for (int k = 0; k < 4; ++k) r.v[k] = a.v[k] + b.v[k];
  return r;
}
template <typename T>
__device__ __forceinline__ V4<T> v4_zero() {
  V4<T> r;
#pragma unroll
  for (int k = 0; k < 4; ++k) r.v[k] = T(0);
  return r;
}

// Block reduction over NT threads: each wave reduces its lanes, then the first wave
// reduces the per-wave records (lanes past NT / 64 empty); the result is valid in
// thread 0 only.
template <int NT>
__device__ __forceinline__ Part persist_reduce(Part p, Part* sp) {
  p = wave_reduce(p);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0) sp[wave] = p;
  __syncthreads();
  Part r = part_empty();
  if (wave == 0) r = wave_reduce(lane < NT / kWave ? sp[lane] : part_empty());
  return r;
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_persist(Group<T> g, int iters, double floor, int check_tol) {
  constexpr int kPersistThreads = NT;
  constexpr int kPersistMaxPer = kPersistMaxInputs / NT;
  const int b = blockIdx.x;
  State* st = g.st + b;
  if (st->converged) return;  // uniform: frozen instances are not iterated
  extern __shared__ __attribute__((aligned(16))) unsigned char persist_smem[];
  __shared__ Part sp[NT / kWave];
  __shared__ UpdateParams up_sh;
  const int n = g.n;
  const uint32_t X = 1u << n, Y = (2u << n) - 1u, t = threadIdx.x;
  T* bufA = reinterpret_cast<T*>(persist_smem);
  T* bufB = bufA + (2u << n);
  T* lp = g.lp + (size_t)b * g.xs;
  T* pg = g.p + (size_t)b * g.xs;
  T* Dg = g.D + (size_t)b * g.xs;
  const T* hf = g.hf + (size_t)b * g.xs;
  const Consts& cs = g.cs[b];
  const bool step = g.eta != 1.0;
  double M = st->M;  // max log p of the current iterate (written before this launch)
  for (int it = 0; it < iters; ++it) {
    // F_0 = p e^{-M}: input x is handled by thread x mod kPersistThreads throughout,
    // so the log p it reads is the one it wrote in the previous iteration
    for (uint32_t x = t; x < X; x += kPersistThreads) bufA[x] = exp_t<T>(lp[x] - T(M));
    __syncthreads();
    T* src = bufA;
    T* dst = bufB;
    // forward: F_{i+1} (2^(i+2) - 1 rows of 2^w columns, w = n - i - 1) from F_i;
    // four consecutive columns per thread while rows are at least four wide
    for (int i = 0; i < n; ++i) {
      const int w = n - i - 1;
      const uint32_t rows_in = (2u << i) - 1u, total = ((4u << i) - 1u) << w;
      if (w >= 2) {
        const uint32_t cm = (1u << (w - 2)) - 1u;
        for (uint32_t q = t; q < (total >> 2); q += kPersistThreads) {
          const uint32_t y = q >> (w - 2), s = (q & cm) << 2;
          V4<T> v = v4_zero<T>();
          if (y < rows_in) v = v4_add(v4_ld(src + (y << (w + 1)) + s), v4_ld(src + (y << (w + 1)) + (1u << w) + s));
          if (y > 0u) {
            const uint32_t par = (y - 1u) >> 1, last = (y - 1u) & 1u;
            v = v4_add(v, v4_ld(src + (par << (w + 1)) + (last << w) + s));
          }
          v4_st(dst + (q << 2), v);
        }
      } else {
        const uint32_t cm = (1u << w) - 1u;
        for (uint32_t e = t; e < total; e += kPersistThreads) {
          const uint32_t y = e >> w, s = e & cm;
          T v = T(0);
          if (y < rows_in) v = src[(y << (w + 1)) + s] + src[(y << (w + 1)) + (1u << w) + s];
          if (y > 0u) {
            const uint32_t par = (y - 1u) >> 1, last = (y - 1u) & 1u;
            v += src[(par << (w + 1)) + (last << w) + s];
          }
          dst[e] = v;
        }
      }
      __syncthreads();
      T* tmp = src;
      src = dst;
      dst = tmp;
    }
    // v(y) = w_k log r(y), in place (B_n)
    for (uint32_t y = t; y < Y; y += kPersistThreads) {
      const T wk = T(cs.w[rank_length(y)]);
      src[y] = wlog_t<T>(wk, src[y]);
    }
    __syncthreads();
    // backward: B_i (2^(i+1) - 1 rows of 2^w columns, w = n - i) from B_{i+1}: column
    // b s of row y adds column s of rows y and y b; four consecutive columns of one
    // half per thread while the halves are at least four wide
    for (int i = n - 1; i >= 0; --i) {
      const int w = n - i;
      const uint32_t total = ((2u << i) - 1u) << w;
      if (w >= 3) {
        const uint32_t cm = (1u << (w - 2)) - 1u;
        for (uint32_t q = t; q < (total >> 2); q += kPersistThreads) {
          const uint32_t y = q >> (w - 2), c = (q & cm) << 2;
          const uint32_t bit = c >> (w - 1), s = c & ((1u << (w - 1)) - 1u);
          v4_st(dst + (q << 2), v4_add(v4_ld(src + (y << (w - 1)) + s),
                                       v4_ld(src + ((2u * y + 1u + bit) << (w - 1)) + s)));
        }
      } else {
        const uint32_t cm = (1u << (w - 1)) - 1u;
        for (uint32_t e = t; e < total; e += kPersistThreads) {
          const uint32_t y = e >> w, bit = (e >> (w - 1)) & 1u, s = e & cm;
          dst[e] = src[(y << (w - 1)) + s] + src[((2u * y + 1u + bit) << (w - 1)) + s];
        }
      }
      __syncthreads();
      T* tmp = src;
      src = dst;
      dst = tmp;
    }
    // D(x) = H(x) - G(x) - M and the record of the iterate
    T dv[kPersistMaxPer];
    Part p = part_empty();
#pragma unroll
    for (int j = 0; j < kPersistMaxPer; ++j) {
      const uint32_t x = t + uint32_t(j) * kPersistThreads;
      if (x < X) {
        dv[j] = hf[x] - src[x] - T(M);
        Dg[x] = dv[j];
        const double l = double(lp[x]);
        part_add<T>(p, l + double(dv[j]), double(dv[j]), exp_in(l, T()), 0.0, 1.0, step, l + g.eta * double(dv[j]));
      }
    }
    const Part P = persist_reduce<NT>(p, sp);  // valid in thread 0
    if (t == 0) up_sh = update_params_rec<T>(g, b, P, check_tol, true);
    __syncthreads();
    const UpdateParams u = up_sh;
    if (u.stop) break;  // frozen at this iterate (the state says so)
    const T lo = T(u.Mn - floor), eta = T(g.eta);
#pragma unroll
    for (int j = 0; j < kPersistMaxPer; ++j) {
      const uint32_t x = t + uint32_t(j) * kPersistThreads;
      if (x < X) {
        const T nl = update_value<T>(u, eta, lo, lp[x], dv[j]);
        lp[x] = nl;
        pg[x] = exp_t<T>(nl - T(u.Mn));
      }
    }
    M = u.Mn;
    __syncthreads();  // the reduction slots and LDS arrays are reused
  }
}

}  // namespace

bool persist_supported(int n, size_t esz) {
  const int top = esz == 4 ? 13 : 12;
  return n >= 1 && n <= top;
}

template <typename T, int NT>
hipError_t launch_persist_nt(const Group<T>& g, int iters, double floor, int check_tol, size_t lds, hipStream_t s) {
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_persist<T, NT>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_persist<T, NT>), dim3(g.nb), dim3(NT), lds, s, g, iters, floor, check_tol);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_persist(const Group<T>& g, int iters, double floor, int check_tol, int threads, hipStream_t s) {
  const size_t lds = size_t(4u << g.n) * sizeof(T);
  switch (threads) {
    case 256: return launch_persist_nt<T, 256>(g, iters, floor, check_tol, lds, s);
    case 512: return launch_persist_nt<T, 512>(g, iters, floor, check_tol, lds, s);
    case 1024: return launch_persist_nt<T, 1024>(g, iters, floor, check_tol, lds, s);
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_persist<float>(const Group<float>&, int, double, int, int, hipStream_t);
template hipError_t launch_persist<double>(const Group<double>&, int, double, int, int, hipStream_t);

}  // namespace ba
