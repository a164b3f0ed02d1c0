// Per-input and per-output elementwise kernels and the reductions of one BA
// iteration (Section 2.3): v(y) = w_k log r(y); D(x) = H(x) - G(x) - M; the
// Blahut quantities L = log sum_x p(x) e^{D(x)}, U = max_x D(x), I = sum_x p D;
// and the update log p <- log p + D - L (normalisation of W^{(t)}).
//
// Reductions are two-level: a partial kernel writes one record per block
// (wavefront shuffles, then LDS across the 4 wavefronts), a one-block-per-instance
// kernel combines them into the final record, and the update kernel reads that
// one record; there is no host round trip.  Records are FP64 for both iteration
// precisions.
#include <math.h>

#include "ba_internal.h"
#include "ba_part.h"

namespace ba {
namespace {

__device__ __forceinline__ int length_of_rank(uint32_t r) { return 31 - __clz(r + 1u); }

// v(y) = w_k log r(y)  (or s_k w_k log r(y)); a zero weight gives 0.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_logr(Group<T> g, int use_sw) {
  const int b = blockIdx.y;
  if (g.st[b].converged) return;
  const uint32_t Y = out_count(g.n);
  const double* w = use_sw ? g.cs[b].sw : g.cs[b].w;
  const T* r = g.r + (size_t)b * g.ys;
  T* v = g.v + (size_t)b * g.ys;
  for (uint32_t y = blockIdx.x * blockDim.x + threadIdx.x; y < Y; y += gridDim.x * blockDim.x) {
    const T wk = T(w[length_of_rank(y)]);
    v[y] = wlog_t<T>(wk, r[y]);
  }
}

// Same values written in the split layout V2[rank(y2)][rank(y1)] = v(y1 y2) used by
// the stream engine's gather sweep.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_logr_split(Group<T> g, int use_sw, int n1, int n2) {
  const int b = blockIdx.y;
  if (g.st[b].converged) return;
  const uint32_t S1 = out_count(n1), S2 = out_count(n2);
  const uint32_t total = S1 * S2;
  const double* w = use_sw ? g.cs[b].sw : g.cs[b].w;
  const T* r = g.r + (size_t)b * g.ys;
  T* v2 = g.v2 + (size_t)b * g.v2s;
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += gridDim.x * blockDim.x) {
    const uint32_t R2 = idx / S1, R1 = idx % S1;
    const int k1 = length_of_rank(R1), k2 = length_of_rank(R2);
    const uint32_t y1 = R1 + 1u - (1u << k1), y2 = R2 + 1u - (1u << k2);
    const uint32_t rank = ((y1 | (1u << k1)) << k2) + y2 - 1u;
    const T wk = T(w[k1 + k2]);
    v2[idx] = wlog_t<T>(wk, r[rank]);
  }
}

// D(x) = H(x) - G(x) - M and the per-block partials of L, U, I (and of
// sum p Dd with Dd = Hd - Gd when use_hd).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dpart(Group<T> g, int nblk, int use_hd, const T* gd) {
  const int b = blockIdx.y;
  if (g.st[b].converged) return;
  const uint32_t X = 1u << g.n;
  const double M = g.st[b].M;
  const T* lp = g.lp + (size_t)b * g.xs;
  const T* gg = g.g + (size_t)b * g.xs;
  const T* h = g.hf + (size_t)b * g.xs;
  T* D = g.D + (size_t)b * g.xs;
  Part p = part_empty();
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < X; x += gridDim.x * blockDim.x) {
    const T lpx = lp[x];
    const T dv = h[x] - gg[x] - T(M);
    D[x] = g.dsum ? T(lpx + dv) : dv;  // log p + D for the update (eta = 1), else D
    const double l = double(lpx);
    const double px = exp_in(l, T());
    const double pdd = use_hd ? px * (g.hd[(size_t)b * g.xs + x] - double(gd[(size_t)b * g.xs + x])) : 0.0;
    part_add<T>(p, l + double(dv), double(dv), px, pdd, 1.0, g.eta != 1.0, l + g.eta * double(dv));
  }
  store_block_part(g.part + (size_t)b * g.ps, blockIdx.x, p);
}

// Final record of every instance from its nblk block records (one block per instance).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_final_parts(Group<T> g, int nblk) {
  const int b = blockIdx.x;
  if (g.frz && g.st[b].converged) return;
  double* part = g.part + (size_t)b * g.ps;
  const Part P = gather_parts(part, nblk);
  if (threadIdx.x == 0) store_part(part + kFinalRec, P);
}

// log p <- max(log p + D - L, M' - floor),  p <- e^{log p - M'}, M' = max(log p + D) - L,
// from the final record of the D kernel (with a step eta != 1: log p + eta D minus
// its log-sum-exp, entropic mirror ascent on the iterate).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update(Group<T> g, int nblk, double floor, int check_tol, int sym) {
  const int b = blockIdx.y;
  if (g.st[b].converged) return;
  const UpdateParams u = update_params<T>(g, b, check_tol, blockIdx.x == 0 && threadIdx.x == 0);
  if (u.stop) return;
  const uint32_t X = 1u << g.n;
  T* lp = g.lp + (size_t)b * g.xs;
  T* p = g.p + (size_t)b * g.xs;
  const T* D = g.D + (size_t)b * g.xs;
  const T lo = T(u.Mn - floor), eta = T(g.eta);
  // sym: D holds the inputs x < 2^(n-1) only; their complements get the same values
  const uint32_t count = sym ? X / 2u : X;
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < count; x += gridDim.x * blockDim.x) {
    const T nl = g.dsum ? update_value_sum<T>(u, lo, D[x]) : update_value<T>(u, eta, lo, lp[x], D[x]);
    const T px = exp_t<T>(nl - T(u.Mn));
    lp[x] = nl;
    p[x] = px;
    if (sym) {
      lp[X - 1u - x] = nl;
      p[X - 1u - x] = px;
    }
  }
}

// Largest |log p(x) - log p(cpl x)| of every instance (one block per instance),
// with orbit = 1 also |log p(x) - log p(rev x)|.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sym_check(Group<T> g, double* out, int orbit) {
  const int b = blockIdx.x;
  const int n = g.n;
  const uint32_t X = 1u << n;
  const T* lp = g.lp + (size_t)b * g.xs;
  double m = 0.0;
  for (uint32_t x = threadIdx.x; x < X; x += blockDim.x) {
    double dv = fabs(double(lp[x]) - double(lp[X - 1u - x]));
    if (orbit) dv = fmax(dv, fabs(double(lp[x]) - double(lp[__brev(x) >> (32 - n)])));
    m = (dv > m || dv != dv) ? dv : m;  // NaN propagates
  }
  __shared__ double sm[kBlock];
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      const double o = sm[threadIdx.x + off];
      if (o > sm[threadIdx.x] || o != o) sm[threadIdx.x] = o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b] = sm[0];
}

// Make the iterate exactly invariant: copy the half x < 2^(n-1) onto the
// complements (log p and p), or with orbit = 1 give every input the values of its
// orbit's representative under complement and reversal (representatives are only
// read, the other members only written).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_symmetrize(Group<T> g, int orbit) {
  const int b = blockIdx.y;
  const uint32_t X = 1u << g.n;
  T* lp = g.lp + (size_t)b * g.xs;
  T* p = g.p + (size_t)b * g.xs;
  if (orbit) {
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < X; x += gridDim.x * blockDim.x) {
      uint32_t rep, size;
      orbit_of(x, g.n, rep, size);
      if (rep != x) {
        lp[x] = lp[rep];
        p[x] = p[rep];
      }
    }
    return;
  }
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < X / 2u; x += gridDim.x * blockDim.x) {
    lp[X - 1u - x] = lp[x];
    p[X - 1u - x] = p[x];
  }
}

// Certification, pass A: per-block max and log-sum-exp of log p (source precision).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lse_a(const T* lp, size_t xs, int n, double* part, size_t ps) {
  const int b = blockIdx.y;
  const uint32_t X = 1u << n;
  lp += (size_t)b * xs;
  Part p = part_empty();
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < X; x += gridDim.x * blockDim.x) {
    const double a = double(lp[x]);
    if (a > -INFINITY) {  // a zero probability adds nothing to the sum
      if (a > p.m) { p.s = p.s * exp(p.m - a) + 1.0; p.m = a; } else { p.s += exp(a - p.m); }
    }
    p.dmax = fmax(p.dmax, a);
    if (!(a < INFINITY) && !(a == -INFINITY)) p.i += 1.0;  // NaN or +Inf counter
  }
  p = block_reduce(p);
  if (threadIdx.x == 0) store_part(part + (size_t)b * ps + (size_t)blockIdx.x * kPartStride, p);
}

// Pass B: partials of log-sum-exp of the floored log p, max(log p, max - floor).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lse_b(const T* lp, size_t xs, int n, const double* partA,
                                                  double* partB, size_t ps, int nblk, double floor) {
  const int b = blockIdx.y;
  const uint32_t X = 1u << n;
  lp += (size_t)b * xs;
  const Part A = gather_parts(partA + (size_t)b * ps, nblk);
  const double lo = A.dmax - floor;
  Part p = part_empty();
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < X; x += gridDim.x * blockDim.x) {
    const double a = fmax(double(lp[x]), lo);
    if (a > p.m) { p.s = p.s * exp(p.m - a) + 1.0; p.m = a; } else { p.s += exp(a - p.m); }
  }
  p = block_reduce(p);
  if (threadIdx.x == 0) store_part(partB + (size_t)b * ps + (size_t)blockIdx.x * kPartStride, p);
}

// Pass C: write the normalised floored FP64 law and its max into the FP64 group.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cert_write(const T* lp, size_t xs, Group<double> dst,
                                                       const double* partA, const double* partB,
                                                       size_t ps, int nblk, double floor) {
  const int b = blockIdx.y;
  const uint32_t X = 1u << dst.n;
  lp += (size_t)b * xs;
  const Part A = gather_parts(partA + (size_t)b * ps, nblk);
  const Part B = gather_parts(partB + (size_t)b * ps, nblk);
  const double lo = A.dmax - floor;
  const double lse = B.m + log(B.s);
  const double Mc = A.dmax - lse;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    dst.st[b].M = Mc;
    dst.st[b].converged = 0;
    dst.st[b].bad = (A.i > 0.0 || !isfinite(Mc)) ? 1 : 0;
    dst.st[b].lse = lse;
  }
  double* o = dst.lp + (size_t)b * dst.xs;
  double* pp = dst.p + (size_t)b * dst.xs;
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < X; x += gridDim.x * blockDim.x) {
    const double a = fmax(double(lp[x]), lo) - lse;
    o[x] = a;
    pp[x] = exp(a - Mc);
  }
}

// Finish a certification: combine the FP64 D partials into certL/U/I of the
// iteration states `out` (and the best bounds); freeze when the certified gap is
// below tol (when write_best).
__global__ __launch_bounds__(kBlock) void k_cert_finish(Group<double> g, int nblk, State* out, int write_best) {
  const int b = blockIdx.x;
  const Part P = gather_parts(g.part + (size_t)b * g.ps, nblk);
  if (threadIdx.x != 0) return;
  const double L = P.m + log(P.s), U = P.dmax;
  State* st = out + b;
  st->certL = L;
  st->certU = U;
  st->certI = P.i;
  st->certM = g.st[b].M;
  if (!isfinite(L) || !isfinite(U) || g.st[b].bad) st->bad = 1;
  if (write_best && isfinite(L) && isfinite(U)) {
    if (L > st->bestL) st->bestL = L;
    if (U < st->bestU) st->bestU = U;
    const double gap = st->stop_best ? (st->bestU - st->bestL) : (U - L);
    if (st->tol >= 0.0 && gap < st->tol) st->converged = 1;
  }
}

// Gradient finish: out3 = {I bits, dI/dd bits, L bits}; grad = p (D - I) / ln 2.
__global__ __launch_bounds__(kBlock) void k_grad_finish(Group<double> g, int nblk, double* out3, double* grad) {
  const Part P = gather_parts(g.part, nblk);
  const double I = P.i;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    out3[0] = I / kLn2;
    out3[1] = P.id / kLn2;
    out3[2] = (P.m + log(P.s)) / kLn2;
    out3[3] = P.dmax / kLn2;
  }
  if (!grad) return;
  const uint32_t X = 1u << g.n;
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < X; x += gridDim.x * blockDim.x)
    grad[x] = exp(g.lp[x]) * (g.D[x] - I) / kLn2;
}

__global__ __launch_bounds__(kBlock) void k_mirror(int n, double* theta, const double* D, double eta) {
  const uint32_t X = 1u << n;
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < X; x += gridDim.x * blockDim.x)
    theta[x] += eta * D[x];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_get_logp(Group<T> g, double* dst) {
  const int b = blockIdx.y;
  const uint32_t X = 1u << g.n;
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < X; x += gridDim.x * blockDim.x)
    dst[(size_t)b * X + x] = double(g.lp[(size_t)b * g.xs + x]);
}

// Set: log p = max(src, max - floor) - lse, p = e^{log p - M}; resets the state.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_set_write(Group<T> g, const double* src, const double* partA,
                                                      const double* partB, size_t ps, int nblk,
                                                      double floor) {
  const int b = blockIdx.y;
  const uint32_t X = 1u << g.n;
  src += (size_t)b * X;
  const Part A = gather_parts(partA + (size_t)b * ps, nblk);
  const Part B = gather_parts(partB + (size_t)b * ps, nblk);
  const double lo = A.dmax - floor;
  const double lse = B.m + log(B.s);
  const double M = A.dmax - lse;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    State* st = g.st + b;
    st->M = M;
    st->iters = 0;
    st->converged = 0;
    st->bad = (A.i > 0.0 || !isfinite(M)) ? 1 : 0;
    st->bestL = -INFINITY;
    st->bestU = INFINITY;
  }
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < X; x += gridDim.x * blockDim.x) {
    const double a = fmax(src[x], lo) - lse;
    g.lp[(size_t)b * g.xs + x] = T(a);
    g.p[(size_t)b * g.xs + x] = T(exp(a - M));
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_reset(Group<T> g) {
  const int b = blockIdx.y;
  const uint32_t X = 1u << g.n;
  const double l0 = -double(g.n) * kLn2;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    State* st = g.st + b;
    st->M = l0;
    st->L = st->U = st->I = 0.0;
    st->certL = st->certU = st->certI = st->certM = 0.0;
    st->bestL = -INFINITY;
    st->bestU = INFINITY;
    st->tol = -1.0;
    st->lse = 0.0;
    st->iters = 0;
    st->converged = 0;
    st->bad = 0;
    st->stop_best = 0;
  }
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < X; x += gridDim.x * blockDim.x) {
    g.lp[(size_t)b * g.xs + x] = T(l0);
    g.p[(size_t)b * g.xs + x] = T(1);
  }
}

__global__ void k_fill_zero(uint4* p, size_t n16) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void k_to_float(const double* src, float* dst, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = float(src[i]);
}

__global__ void k_copy_f64(double* dst, const double* src, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

inline uint32_t grid_for(uint64_t total) {
  uint64_t g = (total + kBlock - 1) / kBlock;
  return g > 4096u ? 4096u : (g == 0 ? 1u : uint32_t(g));
}

}  // namespace

int reduce_blocks(int n) {
  const uint32_t X = 1u << n;
  uint32_t nb = (X + 4 * kBlock - 1) / (4 * kBlock);  // >= 4 elements per thread
  if (nb > 1024u) nb = 1024u;
  return nb < 1 ? 1 : int(nb);
}

template <typename T>
hipError_t launch_logr(const Group<T>& g, int use_sw, int want_v2, int n1, int n2, hipStream_t s) {
  if (want_v2) {
    const uint64_t total = uint64_t(out_count(n1)) * out_count(n2);
    hipLaunchKernelGGL(k_logr_split<T>, dim3(grid_for(total), g.nb), dim3(kBlock), 0, s, g, use_sw, n1, n2);
  } else {
    hipLaunchKernelGGL(k_logr<T>, dim3(grid_for(out_count(g.n)), g.nb), dim3(kBlock), 0, s, g, use_sw);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dpart(const Group<T>& g, int nblk, int use_hd, const T* gd, hipStream_t s) {
  hipLaunchKernelGGL(k_dpart<T>, dim3(nblk, g.nb), dim3(kBlock), 0, s, g, nblk, use_hd, gd);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_final_parts(const Group<T>& g, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_final_parts<T>, dim3(g.nb), dim3(kBlock), 0, s, g, nblk);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_update(const Group<T>& g, int nblk, double floor, int check_tol, int sym, hipStream_t s) {
  hipLaunchKernelGGL(k_update<T>, dim3(nblk, g.nb), dim3(kBlock), 0, s, g, nblk, floor, check_tol, sym);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sym_check(const Group<T>& g, double* out, int orbit, hipStream_t s) {
  hipLaunchKernelGGL(k_sym_check<T>, dim3(g.nb), dim3(kBlock), 0, s, g, out, orbit);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_symmetrize(const Group<T>& g, int orbit, hipStream_t s) {
  hipLaunchKernelGGL(k_symmetrize<T>, dim3(grid_for(1u << g.n), g.nb), dim3(kBlock), 0, s, g, orbit);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cert_prepare(const Group<T>& src, const Group<double>& dst, int nblk, double floor,
                               hipStream_t s) {
  // partials live in the destination group's record buffer: A at +0, B after the first set
  double* partA = dst.part;
  double* partB = dst.part + size_t(kMaxRedBlocks) * kPartStride;
  hipLaunchKernelGGL(k_lse_a<T>, dim3(nblk, src.nb), dim3(kBlock), 0, s, src.lp, src.xs, src.n, partA, dst.ps);
  hipLaunchKernelGGL(k_lse_b<T>, dim3(nblk, src.nb), dim3(kBlock), 0, s, src.lp, src.xs, src.n, partA, partB,
                     dst.ps, nblk, floor);
  hipLaunchKernelGGL(k_cert_write<T>, dim3(nblk, src.nb), dim3(kBlock), 0, s, src.lp, src.xs, dst, partA,
                     partB, dst.ps, nblk, floor);
  return hipGetLastError();
}

hipError_t launch_cert_finish(const Group<double>& g, int nblk, State* out, int write_best, hipStream_t s) {
  hipLaunchKernelGGL(k_cert_finish, dim3(g.nb), dim3(kBlock), 0, s, g, nblk, out, write_best);
  return hipGetLastError();
}

hipError_t launch_grad_finish(const Group<double>& g, int nblk, double* out4, double* grad_theta,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_grad_finish, dim3(grid_for(1u << g.n)), dim3(kBlock), 0, s, g, nblk, out4, grad_theta);
  return hipGetLastError();
}

hipError_t launch_mirror_update(int n, double* theta, const double* D, double eta, hipStream_t s) {
  hipLaunchKernelGGL(k_mirror, dim3(grid_for(1u << n)), dim3(kBlock), 0, s, n, theta, D, eta);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_get_logp(const Group<T>& g, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_get_logp<T>, dim3(grid_for(1u << g.n), g.nb), dim3(kBlock), 0, s, g, dst);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_set_logp(const Group<T>& g, const double* src, int nblk, double floor, hipStream_t s) {
  double* partA = g.part;
  double* partB = g.part + size_t(kMaxRedBlocks) * kPartStride;
  const size_t X = size_t(1) << g.n;
  hipLaunchKernelGGL(k_lse_a<double>, dim3(nblk, g.nb), dim3(kBlock), 0, s, src, X, g.n, partA, g.ps);
  hipLaunchKernelGGL(k_lse_b<double>, dim3(nblk, g.nb), dim3(kBlock), 0, s, src, X, g.n, partA, partB, g.ps,
                     nblk, floor);
  hipLaunchKernelGGL(k_set_write<T>, dim3(nblk, g.nb), dim3(kBlock), 0, s, g, src, partA, partB, g.ps, nblk,
                     floor);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_reset(const Group<T>& g, hipStream_t s) {
  hipLaunchKernelGGL(k_reset<T>, dim3(grid_for(1u << g.n), g.nb), dim3(kBlock), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void* ptr, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(n16)), dim3(kBlock), 0, s, static_cast<uint4*>(ptr), n16);
  return hipGetLastError();
}

hipError_t launch_to_float(const double* src, float* dst, size_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_to_float, dim3(grid_for(count)), dim3(kBlock), 0, s, src, dst, count);
  return hipGetLastError();
}

hipError_t launch_copy_f64(double* dst, const double* src, size_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_f64, dim3(grid_for(count)), dim3(kBlock), 0, s, dst, src, count);
  return hipGetLastError();
}

#define BA_INST(T)                                                                               \
  template hipError_t launch_logr<T>(const Group<T>&, int, int, int, int, hipStream_t);          \
  template hipError_t launch_dpart<T>(const Group<T>&, int, int, const T*, hipStream_t);         \
  template hipError_t launch_update<T>(const Group<T>&, int, double, int, int, hipStream_t);     \
  template hipError_t launch_sym_check<T>(const Group<T>&, double*, int, hipStream_t);          \
  template hipError_t launch_symmetrize<T>(const Group<T>&, int, hipStream_t);                  \
  template hipError_t launch_final_parts<T>(const Group<T>&, int, hipStream_t);                 \
  template hipError_t launch_cert_prepare<T>(const Group<T>&, const Group<double>&, int, double, \
                                             hipStream_t);                                       \
  template hipError_t launch_get_logp<T>(const Group<T>&, double*, hipStream_t);                \
  template hipError_t launch_set_logp<T>(const Group<T>&, const double*, int, double, hipStream_t); \
  template hipError_t launch_reset<T>(const Group<T>&, hipStream_t);
BA_INST(float)
BA_INST(double)
#undef BA_INST

}  // namespace ba
