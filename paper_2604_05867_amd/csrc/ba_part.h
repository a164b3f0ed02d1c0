// Device-side reduction records of one BA iteration (Section 2.3): for the
// current iterate, U = max_x D(x), L = log sum_x p(x) e^{D(x)} (online
// log-sum-exp of a = log p + D), I = sum_x p(x) D(x), for the derivative in d
// sum_x p(x) Dd(x), and for a step eta != 1 the normaliser log sum_x p e^{eta D}.  A kernel accumulates one record per thread, reduces it
// per block and stores one record per block; a one-block-per-instance kernel
// combines them into the final record that the update kernel reads.  Included by
// the .hip sources only.
#pragma once

#include <math.h>

#include "ba_internal.h"

namespace ba {

// log and exp in the iterate's precision
template <typename T>
__device__ __forceinline__ T log_t(T v);
template <>
__device__ __forceinline__ float log_t<float>(float v) { return logf(v); }
template <>
__device__ __forceinline__ double log_t<double>(double v) { return log(v); }
// w log r for a value r of the output law (v = w_k log r), 0 where w = 0.  FP32: the
// hardware base-2 logarithm times w ln 2; r is a normal number here (every iterate
// value is at least e^-87, the largest FP32 floor, and r sums such values).
template <typename T>
__device__ __forceinline__ T wlog_t(T w, T r);
template <>
__device__ __forceinline__ float wlog_t<float>(float w, float r) {
  return (w == 0.0f) ? 0.0f : (w * 0.693147180559945309f) * __builtin_amdgcn_logf(r);
}
template <>
__device__ __forceinline__ double wlog_t<double>(double w, double r) {
  return (w == 0.0) ? 0.0 : w * log(r);
}
template <typename T>
__device__ __forceinline__ T exp_t(T v);
template <>
__device__ __forceinline__ float exp_t<float>(float v) { return expf(v); }
template <>
__device__ __forceinline__ double exp_t<double>(double v) { return exp(v); }

struct Part {
  double m;     // max of a = log p + D
  double s;     // sum exp(a - m)
  double dmax;  // max D
  double i;     // sum p D
  double id;    // sum p Dd
  double m2;    // max of a2 = log p + eta D (step eta != 1 only)
  double s2;    // sum exp(a2 - m2)
};

__device__ __forceinline__ Part part_empty() {
  return Part{-INFINITY, 0.0, -INFINITY, 0.0, 0.0, -INFINITY, 0.0};
}

__device__ __forceinline__ double lse_merge_s(double m1, double s1, double m2, double s2, double m) {
  double r = 0.0;
  if (s1 != 0.0) r += s1 * exp(m1 - m);
  if (s2 != 0.0) r += s2 * exp(m2 - m);
  return r;
}

__device__ __forceinline__ Part combine(const Part& a, const Part& b) {
  Part c;
  c.m = fmax(a.m, b.m);
  c.s = (c.m == -INFINITY) ? 0.0 : lse_merge_s(a.m, a.s, b.m, b.s, c.m);
  c.dmax = fmax(a.dmax, b.dmax);
  c.i = a.i + b.i;
  c.id = a.id + b.id;
  c.m2 = fmax(a.m2, b.m2);
  c.s2 = (c.m2 == -INFINITY) ? 0.0 : lse_merge_s(a.m2, a.s2, b.m2, b.s2, c.m2);
  return c;
}

// True for a record that no input has been added to.
__device__ __forceinline__ bool part_is_empty(const Part& p) { return p.s == 0.0 && p.dmax == -INFINITY; }

__device__ __forceinline__ double exp_in(double v, double) { return exp(v); }
__device__ __forceinline__ double exp_in(double v, float) { return double(expf(float(v))); }

// Add one input with a = log p + D, D, p and p*Dd to a thread's record; the
// exponential of the running log-sum-exp is taken in precision E (the iterate's).
// wt: the number of inputs this value stands for (2 when only one of each
// complement pair x, cpl(x) is evaluated).
__device__ __forceinline__ void lse_add(double& m, double& s, double a, double wt, double) {
  if (a > m) {
    s = s * exp(m - a) + wt;
    m = a;
  } else {
    s += wt * exp(a - m);
  }
}
__device__ __forceinline__ void lse_add(double& m, double& s, double a, double wt, float) {
  if (a > m) {
    s = s * double(expf(float(m - a))) + wt;
    m = a;
  } else {
    s += wt * double(expf(float(a - m)));
  }
}

// a = log p + D, a2 = log p + eta D (used when eta != 1).
template <typename E>
__device__ __forceinline__ void part_add(Part& p, double a, double dv, double px, double pdd, double wt = 1.0,
                                         bool step = false, double a2 = 0.0) {
  lse_add(p.m, p.s, a, wt, E());
  if (step) lse_add(p.m2, p.s2, a2, wt, E());
  p.dmax = fmax(p.dmax, dv);
  p.i += wt * px * dv;
  p.id += wt * pdd;
}

// Reduction of one record per lane: max first, then every lane rescales its sum
// to the common max (one exponential per lane) and the rest are plain sums/maxes.
__device__ __forceinline__ Part wave_reduce(Part p) {
  double m = p.m, dmax = p.dmax;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    m = fmax(m, __shfl_xor(m, off));
    dmax = fmax(dmax, __shfl_xor(dmax, off));
  }
  double s = (p.s != 0.0) ? p.s * exp(p.m - m) : 0.0;
  double i = p.i, id = p.id;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    s += __shfl_xor(s, off);
    i += __shfl_xor(i, off);
    id += __shfl_xor(id, off);
  }
  // second log-sum-exp only where some lane has one (eta != 1)
  double m2 = p.m2, s2 = 0.0;
  if (__any(p.s2 != 0.0)) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m2 = fmax(m2, __shfl_xor(m2, off));
    s2 = (p.s2 != 0.0) ? p.s2 * exp(p.m2 - m2) : 0.0;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) s2 += __shfl_xor(s2, off);
  } else {
    m2 = -INFINITY;
  }
  return Part{m, s, dmax, i, id, m2, s2};
}

// A thread's record in single precision (the D launch of FP32 iterates): max of
// a = log p + D, sum exp(a - m), max D, sum p D, and for a step eta != 1 the max and
// sum for log p + eta D.
struct PartF {
  float m, s, dmax, i, m2, s2;
};

// The wavefront's records of single-precision lanes reduced as wave_reduce does, in
// single precision (max first, one hardware exponential per lane, then plain sums),
// the result in every lane widened to a double record.
__device__ __forceinline__ Part wave_reduce_f(const PartF& p, bool step) {
  float m = p.m, dmax = p.dmax;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    m = fmaxf(m, __shfl_xor(m, off));
    dmax = fmaxf(dmax, __shfl_xor(dmax, off));
  }
  float s = (p.s != 0.0f) ? p.s * __expf(p.m - m) : 0.0f, i = p.i;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    s += __shfl_xor(s, off);
    i += __shfl_xor(i, off);
  }
  Part r{double(m), double(s), double(dmax), double(i), 0.0, -INFINITY, 0.0};
  if (step) {
    float m2 = p.m2;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m2 = fmaxf(m2, __shfl_xor(m2, off));
    float s2 = (p.s2 != 0.0f) ? p.s2 * __expf(p.m2 - m2) : 0.0f;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) s2 += __shfl_xor(s2, off);
    r.m2 = double(m2);
    r.s2 = double(s2);
  }
  return r;
}

// Block reduction (blockDim.x == NT): every wave reduces its lanes, then every wave
// reduces the per-wave records (one per lane, lanes past NT / kWave empty), so the
// result is valid in every thread.  Empty lanes leave every sum and maximum exactly
// as it is, so the result does not depend on NT beyond the waves that hold records.
template <int NT>
__device__ __forceinline__ Part block_reduce_nt(Part p) {
  __shared__ Part sp[NT / kWave];
  p = wave_reduce(p);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) sp[wave] = p;
  __syncthreads();
  return wave_reduce(lane < NT / kWave ? sp[lane] : part_empty());
}
__device__ __forceinline__ Part block_reduce(Part p) { return block_reduce_nt<kBlock>(p); }

// The update of one iteration from the final record of its D kernel (at kFinalRec):
// L = log sum p e^D, U = max D; with a step eta != 1 the normaliser Le of
// log p + eta D.  Every caller derives the same values; `writer` stores them in
// the instance state (a stop freezes the instance instead of updating it).
struct UpdateParams {
  double L, Le, Mn;  // Mn: the max of the new log p
  bool step, stop;
};

// From the instance's final record P (any caller that holds it).
template <typename T>
__device__ __forceinline__ UpdateParams update_params_rec(const Group<T>& g, int b, const Part& P, int check_tol,
                                                          bool writer) {
  State* st = g.st + b;
  const double m = P.m, s = P.s, dmax = P.dmax, pi = P.i, m2 = P.m2, s2 = P.s2;
  const double L = m + log(s);
  const double U = dmax;
  // normaliser of the step: L itself for eta = 1 (BA)
  const bool step = g.eta != 1.0;
  const double Le = step ? m2 + log(s2) : L;
  const double Mn = (step ? m2 : m) - Le;
  const bool finite = isfinite(L) && isfinite(U) && isfinite(pi) && isfinite(Le);
  // FP64 iterates (check_tol): these are the exact bounds of the current iterate,
  // so they also update the best bounds; FP32 iterates leave that to certification.
  const double bL = (check_tol && finite) ? fmax(st->bestL, L) : st->bestL;
  const double bU = (check_tol && finite) ? fmin(st->bestU, U) : st->bestU;
  const double gap = st->stop_best ? (bU - bL) : (U - L);
  const bool stop = !finite || (check_tol && st->tol >= 0.0 && gap < st->tol);
  if (writer) {
    st->L = L;
    st->U = U;
    st->I = pi;
    st->bestL = bL;
    st->bestU = bU;
    if (!finite) st->bad = 1;
    if (stop) {
      st->converged = 1;
    } else {
      st->M = Mn;
      st->iters += 1;
    }
  }
  return UpdateParams{L, Le, Mn, step, stop};
}

// From the final record that an earlier kernel stored at kFinalRec.
template <typename T>
__device__ __forceinline__ UpdateParams update_params(const Group<T>& g, int b, int check_tol, bool writer) {
  const double* q = g.part + (size_t)b * g.ps + kFinalRec;
  const Part P{q[0], q[1], q[2], q[3], q[4], q[5], q[6]};
  return update_params_rec<T>(g, b, P, check_tol, writer);
}

// New log p of one input: max(log p + D - L, lo), or log p + eta D - Le with a step.
template <typename T>
__device__ __forceinline__ T update_value(const UpdateParams& u, T eta, T lo, T lpx, T dx) {
  const T nl = u.step ? lpx + eta * dx - T(u.Le) : lpx + dx - T(u.L);
  return nl > lo ? nl : lo;
}

// The same from a = log p + D as the D launch stored it (Group::dsum, eta = 1): the
// sum and then the difference, rounded as update_value rounds them.
template <typename T>
__device__ __forceinline__ T update_value_sum(const UpdateParams& u, T lo, T a) {
  const T nl = a - T(u.L);
  return nl > lo ? nl : lo;
}

__device__ __forceinline__ void store_part(double* dst, const Part& p) {
  dst[0] = p.m; dst[1] = p.s; dst[2] = p.dmax; dst[3] = p.i; dst[4] = p.id; dst[5] = p.m2; dst[6] = p.s2;
}

// A record written by an earlier kernel on the stream.
__device__ __forceinline__ Part load_part(const double* q) {
  return Part{q[0], q[1], q[2], q[3], q[4], q[5], q[6]};
}

// Combine the nblk records at src (every block that calls this does it in full, with
// NT threads; the result, valid in every thread, is the same for every NT >= nblk).
template <int NT>
__device__ __forceinline__ Part gather_parts_nt(const double* src, int nblk) {
  Part p = part_empty();
  for (int j = threadIdx.x; j < nblk; j += NT) p = combine(p, load_part(src + (size_t)j * kPartStride));
  return block_reduce_nt<NT>(p);
}
__device__ __forceinline__ Part gather_parts(const double* src, int nblk) { return gather_parts_nt<kBlock>(src, nblk); }

// Reduce the block's records and store the result as record rec of an instance
// whose records start at `part`: the first wave combines the per-wave records as
// block_reduce_nt does and its lane 0 writes (blockDim.x == NT, kBlock for
// store_block_part).
template <int NT>
__device__ __forceinline__ void store_block_part_nt(double* part, int rec, Part p) {
  __shared__ Part sp[NT / kWave];
  p = wave_reduce(p);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0) sp[wave] = p;
  __syncthreads();
  if (wave == 0) {
    const Part r = wave_reduce(lane < NT / kWave ? sp[lane] : part_empty());
    if (lane == 0) store_part(part + (size_t)rec * kPartStride, r);
  }
}
__device__ __forceinline__ void store_block_part(double* part, int rec, Part p) {
  store_block_part_nt<kBlock>(part, rec, p);
}

// The same from single-precision lane records: within each wave in single precision
// (wave_reduce_f), across the waves in double.
// maxima (may be null): also store the block's max of log p + D there, as a float
// at index rec.
template <int NT>
__device__ __forceinline__ void store_block_part_f32(double* part, int rec, const PartF& p, bool step,
                                                     float* maxima) {
  __shared__ Part sp[NT / kWave];
  const Part w = wave_reduce_f(p, step);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0) sp[wave] = w;
  __syncthreads();
  if (wave == 0) {
    const Part r = wave_reduce(lane < NT / kWave ? sp[lane] : part_empty());
    if (lane == 0) {
      store_part(part + (size_t)rec * kPartStride, r);
      if (maxima) maxima[rec] = float(r.m);  // exact: the max of floats
    }
  }
}

}  // namespace ba
