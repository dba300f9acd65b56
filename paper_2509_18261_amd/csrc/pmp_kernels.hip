// HIP kernels for gfx950: the particle-mesh-particle step of He et al. (2025),
// Sec. 2.2 (Steps 1-5), Sec. 3.1.1 (sink kernel and limiter) and Sec. 3.2.1
// (uniform supernova injection, momentum limiter eq. "lambda").
//
// Floating-point expressions are written in one fixed order and the file is
// built with -ffp-contract=off, so that the fixed-point path reproduces the
// same integers on every run and every launch shape.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "pmp_internal.h"

namespace pmp {
namespace {

constexpr double kFix = 0x1p40;         // fixed-point scale (40 fractional bits)
constexpr double kFixInv = 0x1p-40;
constexpr double kFixLimit = 0x1p62;    // largest accepted magnitude of a scaled value
constexpr int kWave = 64;

// ----------------------------------------------------------------- helpers

// Round v * 2^40 to the nearest integer, ties to even.
__device__ __forceinline__ bool quantise(double v, long long& q) {
  double s = v * kFix;
  if (!(fabs(s) < kFixLimit)) return false;
  q = (long long)rint(s);
  return true;
}

// exp(x) for the sink kernel weights (Sec. 3.1.1, eq. "kernel"), written from
// the Cody-Waite method: x = k ln2 + r with ln2 carried as a head on the
// 2^-32 grid plus a tail (k * head is then exact), exp(r) from its Taylor
// series through r^13 evaluated by Horner's rule on |r| <= ln2/2, and the
// result scaled by 2^k with an exact ldexp.
__device__ double kernel_exp(double x) {
  if (x != x) return x;
  if (x > 709.0) return __builtin_huge_val();
  if (x < -745.0) return 0.0;
  const double inv_ln2 = 0x1.71547652b82fep+0;
  const double ln2_head = 0x1.62e42ffp-1;
  const double ln2_tail = -0x1.718432a1b0e26p-35;
  const double k = rint(x * inv_ln2);
  const double r = (x - k * ln2_head) - k * ln2_tail;
  double p = 1.0 / 6227020800.0;  // 1/13!
  p = p * r + 1.0 / 479001600.0;  // 1/12!
  p = p * r + 1.0 / 39916800.0;
  p = p * r + 1.0 / 3628800.0;
  p = p * r + 1.0 / 362880.0;
  p = p * r + 1.0 / 40320.0;
  p = p * r + 1.0 / 5040.0;
  p = p * r + 1.0 / 720.0;
  p = p * r + 1.0 / 120.0;
  p = p * r + 1.0 / 24.0;
  p = p * r + 1.0 / 6.0;
  p = p * r + 0.5;
  p = p * r + 1.0;
  p = p * r + 1.0;
  return ldexp(p, (int)k);
}

__device__ __forceinline__ void raise_flag(DevStatus* st, unsigned f) {
  atomicOr(&st->flags, f);
}

// Largest b with off[b] <= p (off[0] = 0 <= p < off[nbox]).
__device__ __forceinline__ int find_box(const long long* off, int nbox, long long p) {
  int lo = 0, hi = nbox;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= p) lo = mid; else hi = mid;
  }
  return lo;
}

// Host cell floor(x) of a particle; false for a position outside the box
// (or NaN), which the caller skips and flags.
__device__ __forceinline__ bool host_cell(const DevBox& B, double x, double y, double z,
                                          int h[3]) {
  const double p[3] = {x, y, z};
  for (int a = 0; a < 3; ++a) {
    const double lo = (double)B.lo[a];
    if (!(p[a] >= lo && p[a] < lo + (double)B.n[a])) return false;
    h[a] = (int)floor(p[a]);
  }
  return true;
}

// Padded local index of global cell (i,j,k) in box B, or false if it lies
// outside the ghost-zoned box.
__device__ __forceinline__ bool pad_index(const DevBox& B, int g, int i, int j, int k,
                                          long long& idx) {
  const int li = i - B.lo[0] + g, lj = j - B.lo[1] + g, lk = k - B.lo[2] + g;
  if ((unsigned)li >= (unsigned)B.p[0] || (unsigned)lj >= (unsigned)B.p[1] ||
      (unsigned)lk >= (unsigned)B.p[2])
    return false;
  idx = ((long long)lk * B.p[1] + lj) * B.p[0] + li;
  return true;
}

// Squared distance from (x,y,z) to the centre of cell (i,j,k), fixed order.
__device__ __forceinline__ double dist2(double x, double y, double z, int i, int j, int k) {
  const double ddx = ((double)i + 0.5) - x;
  const double ddy = ((double)j + 0.5) - y;
  const double ddz = ((double)k + 0.5) - z;
  return (ddx * ddx + ddy * ddy) + ddz * ddz;
}

// Candidate range along one axis for a sphere of radius r centred at p: a
// superset of the cells with |i + 1/2 - p| <= r (membership is decided by
// dist2 alone).
__device__ __forceinline__ void sphere_range(double p, double r, int& lo, int& hi) {
  lo = (int)floor(p - r - 0.5) - 1;
  hi = (int)floor(p + r - 0.5) + 1;
}

__device__ __forceinline__ int imod(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

// accumulator element types
template <int ACC> struct AccT;
template <> struct AccT<PMP_ACC_F32> { using T = float; };
template <> struct AccT<PMP_ACC_F64> { using T = double; };
template <> struct AccT<PMP_ACC_FIX64> { using T = long long; };

template <class T> __device__ __forceinline__ double to_f64(T v);
template <> __device__ __forceinline__ double to_f64<float>(float v) { return (double)v; }
template <> __device__ __forceinline__ double to_f64<double>(double v) { return v; }
template <> __device__ __forceinline__ double to_f64<long long>(long long v) {
  return (double)v * kFixInv;
}

// Atomic adds into the global buffer (hardware float atomics on gfx950).
__device__ __forceinline__ void gadd(float* p, double c) { unsafeAtomicAdd(p, (float)c); }
__device__ __forceinline__ void gadd(double* p, double c) { unsafeAtomicAdd(p, c); }
__device__ __forceinline__ void gadd_fix(long long* p, long long q) {
  atomicAdd((unsigned long long*)p, (unsigned long long)q);
}

// Reductions over groups of W lanes (W a power of two <= 64, groups aligned).
template <int W, class T> __device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}
template <int W> __device__ __forceinline__ int group_min(int v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, W));
  return v;
}
template <int W> __device__ __forceinline__ int group_max(int v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, W));
  return v;
}

// ---------------------------------------------------------- zero and copy

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(1024) void k_zero(u32x4* __restrict__ p, long long n16, unsigned* __restrict__ tail,
                       int ntail) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const u32x4 z = {0u, 0u, 0u, 0u};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    __builtin_nontemporal_store(z, p + i);
  if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0u;
}

__global__ void k_copy(uint4* __restrict__ d, const uint4* __restrict__ s, long long n16,
                       unsigned* __restrict__ dt, const unsigned* __restrict__ st, int ntail) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    d[i] = s[i];
  if (blockIdx.x == 0 && (int)threadIdx.x < ntail) dt[threadIdx.x] = st[threadIdx.x];
}

__global__ void k_clear_status(DevStatus* st) {
  if (threadIdx.x == 0) {
    st->flags = 0u;
    st->reserved = 0u;
    st->touched = st->bind = st->lam = st->fall = 0ull;
  }
}

// ------------------------------------------------------------ CIC deposit

// One CIC particle (cloud-in-cell, cell-centred: per axis t = x - 1/2,
// i0 = floor(t), weights (1 - f, f) on (i0, i0 + 1) with f = t - i0).  `add`
// receives (global i, j, k, value) with value a double (float types) or a
// quantised int64 (fixed point); in fixed point the particle's rounding
// residue goes to its host cell so that its total is exact.
template <bool FIXED, class Add>
__device__ __forceinline__ bool cic_one(double x, double y, double z, double m, double V,
                                        const int h[3], Add&& add) {
  const double t[3] = {x - 0.5, y - 0.5, z - 0.5};
  int i0[3];
  double w[3][2];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double fl = floor(t[a]);
    const double f = t[a] - fl;
    i0[a] = (int)fl;
    w[a][0] = 1.0 - f;
    w[a][1] = f;
  }
  bool ok = true;
  long long qsum = 0;
#pragma unroll
  for (int dk = 0; dk < 2; ++dk)
#pragma unroll
    for (int dj = 0; dj < 2; ++dj)
#pragma unroll
      for (int di = 0; di < 2; ++di) {
        const double wx = w[0][di], wy = w[1][dj], wz = w[2][dk];
        if (wx == 0.0 || wy == 0.0 || wz == 0.0) continue;
        const double c = ((m * wx) * wy) * wz / V;
        if constexpr (FIXED) {
          long long q;
          if (!quantise(c, q)) { ok = false; continue; }
          add(i0[0] + di, i0[1] + dj, i0[2] + dk, q);
          qsum += q;
        } else {
          add(i0[0] + di, i0[1] + dj, i0[2] + dk, c);
        }
      }
  if constexpr (FIXED) {
    long long Q;
    if (ok && quantise(m / V, Q)) add(h[0], h[1], h[2], Q - qsum);
    else ok = false;
  }
  return ok;
}

template <int ACC>
__global__ __launch_bounds__(1024) void k_cic_direct(Mesh M, Particles P,
                                                    typename AccT<ACC>::T* __restrict__ buf,
                                                    const int* __restrict__ key,
                                                    const int* __restrict__ tile_count,
                                                    int dense_min) {
  using T = typename AccT<ACC>::T;
  constexpr bool FIXED = (ACC == PMP_ACC_FIX64);
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < P.n; p += stride) {
    if (key) {
      const int kt = key[p];
      if (kt >= 0 && tile_count[kt] >= dense_min) continue;  // done in LDS
    }
    const int b = (M.nbox == 1) ? 0 : find_box(P.box_off, M.nbox, p);
    const DevBox B = M.boxes[b];
    const double x = P.x[p], y = P.y[p], z = P.z[p], m = P.a[p];
    int h[3];
    if (!host_cell(B, x, y, z, h)) { raise_flag(M.status, PMP_FLAG_OUTSIDE); continue; }
    if (!isfinite(m)) { raise_flag(M.status, PMP_FLAG_NAN); continue; }
    T* base = buf + B.boff;
    const int g = M.ghost;
    auto add = [&](int i, int j, int k, auto v) {
      long long idx;
      if (!pad_index(B, g, i, j, k, idx)) { raise_flag(M.status, PMP_FLAG_REACH); return; }
      if constexpr (FIXED) gadd_fix(base + idx, v); else gadd(base + idx, v);
    };
    if (!cic_one<FIXED>(x, y, z, m, M.V, h, add)) raise_flag(M.status, PMP_FLAG_OVERFLOW);
  }
}

// ------------------------------------------------------- supernova deposit

// Uniform-sphere injection (Sec. 3.2.1, eq. "du" with full coverage, no
// momentum term): the N cells whose centres lie within r get m/(N V) and
// e/(N V).  A group of L lanes handles one particle: first it counts the
// members, then it adds.  If no centre lies within r the host cell takes the
// whole deposit.  Fixed point: residue to the host cell if it is a member,
// else to the first member in (k, j, i) order.
template <int ACC, int L>
__global__ __launch_bounds__(256) void k_sn_direct(Mesh M, Particles P,
                                                   typename AccT<ACC>::T* __restrict__ buf) {
  constexpr bool FIXED = (ACC == PMP_ACC_FIX64);
  const int lane = threadIdx.x % L;
  const long long ngroups = ((long long)gridDim.x * blockDim.x) / L;
  const int g = M.ghost;
  for (long long p = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / L; p < P.n;
       p += ngroups) {
    const int b = (M.nbox == 1) ? 0 : find_box(P.box_off, M.nbox, p);
    const DevBox B = M.boxes[b];
    const double x = P.x[p], y = P.y[p], z = P.z[p];
    const double m = P.b[p], e = P.c[p], r = P.r[p];
    int h[3];
    if (!host_cell(B, x, y, z, h)) {
      if (lane == 0) raise_flag(M.status, PMP_FLAG_OUTSIDE);
      continue;
    }
    if (!isfinite(m) || !isfinite(e) || !isfinite(r) || !(r >= 0.0)) {
      if (lane == 0) raise_flag(M.status, PMP_FLAG_NAN);
      continue;
    }
    if (floor(r + 0.5) > (double)g) {  // reach beyond the ghost zone
      if (lane == 0) raise_flag(M.status, PMP_FLAG_REACH);
      continue;
    }
    const double r2 = r * r;
    int lo[3], hi[3];
    sphere_range(x, r, lo[0], hi[0]);
    sphere_range(y, r, lo[1], hi[1]);
    sphere_range(z, r, lo[2], hi[2]);
    const int cx = hi[0] - lo[0] + 1, cy = hi[1] - lo[1] + 1;
    const int cxy = cx * cy;
    const int total = cxy * (hi[2] - lo[2] + 1);
    int cnt = 0, first = 0x7fffffff, hostm = 0;
    for (int t = lane; t < total; t += L) {
      const int kk = t / cxy, rem = t - kk * cxy, jj = rem / cx, ii = rem - jj * cx;
      const int i = lo[0] + ii, j = lo[1] + jj, k = lo[2] + kk;
      if (dist2(x, y, z, i, j, k) <= r2) {
        ++cnt;
        first = min(first, t);
        hostm |= (i == h[0] && j == h[1] && k == h[2]);
      }
    }
    int N = group_sum<L>(cnt);
    first = group_min<L>(first);
    hostm = group_max<L>(hostm);
    const bool only_host = (N == 0);
    if (only_host) { N = 1; hostm = 1; }
    const double cr = m / ((double)N * M.V);
    const double ce = e / ((double)N * M.V);
    long long qr = 0, qe = 0;
    if constexpr (FIXED) {
      if (!quantise(cr, qr) || !quantise(ce, qe)) {
        if (lane == 0) raise_flag(M.status, PMP_FLAG_OVERFLOW);
        continue;
      }
    }
    using T = typename AccT<ACC>::T;
    T* f0 = buf + B.boff;
    T* f4 = buf + B.boff + 4 * B.npad;
    bool reach_bad = false;
    for (int t = lane; t < total; t += L) {
      const int kk = t / cxy, rem = t - kk * cxy, jj = rem / cx, ii = rem - jj * cx;
      const int i = lo[0] + ii, j = lo[1] + jj, k = lo[2] + kk;
      const bool in = only_host ? (i == h[0] && j == h[1] && k == h[2])
                                : (dist2(x, y, z, i, j, k) <= r2);
      if (!in) continue;
      long long idx;
      if (!pad_index(B, g, i, j, k, idx)) { reach_bad = true; continue; }
      if constexpr (FIXED) {
        gadd_fix(f0 + idx, qr);
        gadd_fix(f4 + idx, qe);
      } else {
        gadd(f0 + idx, cr);
        gadd(f4 + idx, ce);
      }
    }
    if (reach_bad) raise_flag(M.status, PMP_FLAG_REACH);
    if constexpr (FIXED) {
      if (lane == 0) {
        long long Qr, Qe;
        if (quantise(m / M.V, Qr) && quantise(e / M.V, Qe)) {
          int ti = h[0], tj = h[1], tk = h[2];
          if (!hostm) {
            const int kk = first / cxy, rem = first - kk * cxy, jj = rem / cx;
            ti = lo[0] + (rem - jj * cx); tj = lo[1] + jj; tk = lo[2] + kk;
          }
          long long idx;
          if (pad_index(B, g, ti, tj, tk, idx)) {
            gadd_fix(f0 + idx, Qr - (long long)N * qr);
            gadd_fix(f4 + idx, Qe - (long long)N * qe);
          }
        } else {
          raise_flag(M.status, PMP_FLAG_OVERFLOW);
        }
      }
    }
  }
}

// ------------------------------------------------------------------ sinks

template <class S>
__device__ __forceinline__ long long state_cell(const DevBox& B, int iw, int jw, int kw) {
  return ((long long)(kw - B.lo[2]) * B.n[1] + (jw - B.lo[1])) * B.n[0] + (iw - B.lo[0]);
}

// Sink removal request (Sec. 3.1.1).  One wavefront per sink.  Pass 1 sums
// the Gaussian weights w = exp(-d^2/r_g^2) (eq. "kernel") and the kernel gas
// mass sum rho V on the 2^-40 grid (exact, order-free); the request is the
// fraction a of that mass.  Pass 2 adds each cell's removal
// k = max(M_req w / (W V), rho - rho_Tr) (eqs. "kernel_wgt",
// "accretion_function") to field 5.  Single box covering the domain: state
// reads wrap periodically, deposits go to the ghost-zoned buffer unwrapped.
template <int ACC, class S>
__global__ __launch_bounds__(64) void k_sink_deposit(Mesh M, Particles P,
                                                     const S* __restrict__ state,
                                                     typename AccT<ACC>::T* __restrict__ buf,
                                                     double* __restrict__ scratch, double r_k,
                                                     double r_gauss, double rho_tr) {
  constexpr bool FIXED = (ACC == PMP_ACC_FIX64);
  const int lane = threadIdx.x;
  const DevBox B = M.boxes[0];
  const int g = M.ghost;
  const double r2 = r_k * r_k, g2 = r_gauss * r_gauss;
  for (long long s = blockIdx.x; s < P.n; s += gridDim.x) {
    const double x = P.x[s], y = P.y[s], z = P.z[s], a = P.a[s];
    int h[3];
    if (!host_cell(B, x, y, z, h)) {
      if (lane == 0) {
        raise_flag(M.status, PMP_FLAG_OUTSIDE);
        scratch[2 * s] = 0.0;
        scratch[2 * s + 1] = 0.0;
      }
      continue;
    }
    int lo[3], hi[3];
    sphere_range(x, r_k, lo[0], hi[0]);
    sphere_range(y, r_k, lo[1], hi[1]);
    sphere_range(z, r_k, lo[2], hi[2]);
    const int cx = hi[0] - lo[0] + 1, cy = hi[1] - lo[1] + 1;
    const int cxy = cx * cy;
    const int total = cxy * (hi[2] - lo[2] + 1);
    long long wq = 0, mq = 0;
    bool ok = true;
    for (int t = lane; t < total; t += kWave) {
      const int kk = t / cxy, rem = t - kk * cxy, jj = rem / cx, ii = rem - jj * cx;
      const int i = lo[0] + ii, j = lo[1] + jj, k = lo[2] + kk;
      const double d2 = dist2(x, y, z, i, j, k);
      if (!(d2 <= r2)) continue;
      const long long c = state_cell<S>(B, imod(i, M.domain[0]), imod(j, M.domain[1]),
                                        imod(k, M.domain[2]));
      const double rho = (double)state[B.soff + c];
      const double w = kernel_exp(-(d2 / g2));
      long long q1, q2;
      if (!quantise(w, q1) || !quantise(rho * M.V, q2)) { ok = false; continue; }
      wq += q1;
      mq += q2;
    }
    wq = group_sum<kWave>(wq);
    mq = group_sum<kWave>(mq);
    if (!ok) raise_flag(M.status, PMP_FLAG_OVERFLOW);
    if (wq <= 0) {
      if (lane == 0) { scratch[2 * s] = 0.0; scratch[2 * s + 1] = 0.0; }
      continue;
    }
    const double W = (double)wq * kFixInv;
    const double Mreq = a * ((double)mq * kFixInv);
    if (lane == 0) { scratch[2 * s] = W; scratch[2 * s + 1] = Mreq; }
    using T = typename AccT<ACC>::T;
    T* f5 = buf + B.boff + 5 * B.npad;
    long long qreq = 0;
    int first = 0x7fffffff, hostm = 0;
    bool reach_bad = false;
    for (int t = lane; t < total; t += kWave) {
      const int kk = t / cxy, rem = t - kk * cxy, jj = rem / cx, ii = rem - jj * cx;
      const int i = lo[0] + ii, j = lo[1] + jj, k = lo[2] + kk;
      const double d2 = dist2(x, y, z, i, j, k);
      if (!(d2 <= r2)) continue;
      first = min(first, t);
      hostm |= (i == h[0] && j == h[1] && k == h[2]);
      const long long c = state_cell<S>(B, imod(i, M.domain[0]), imod(j, M.domain[1]),
                                        imod(k, M.domain[2]));
      const double rho = (double)state[B.soff + c];
      const double w = kernel_exp(-(d2 / g2));
      const double kreq = (Mreq * w) / (W * M.V);
      const double tr = rho - rho_tr;
      const double kc = (tr > kreq) ? tr : kreq;
      long long idx;
      if (!pad_index(B, g, i, j, k, idx)) { reach_bad = true; continue; }
      if constexpr (FIXED) {
        long long q1, q2;
        if (!quantise(kc, q1) || !quantise(kreq, q2)) { ok = false; continue; }
        gadd_fix(f5 + idx, q1);
        qreq += q2;
      } else {
        gadd(f5 + idx, kc);
      }
    }
    if (reach_bad) raise_flag(M.status, PMP_FLAG_REACH);
    if constexpr (FIXED) {
      qreq = group_sum<kWave>(qreq);
      first = group_min<kWave>(first);
      hostm = group_max<kWave>(hostm);
      if (lane == 0) {
        long long Q;
        if (ok && quantise(Mreq / M.V, Q)) {
          int ti = h[0], tj = h[1], tk = h[2];
          if (!hostm) {
            const int kk = first / cxy, rem = first - kk * cxy, jj = rem / cx;
            ti = lo[0] + (rem - jj * cx); tj = lo[1] + jj; tk = lo[2] + kk;
          }
          long long idx;
          if (pad_index(B, g, ti, tj, tk, idx)) gadd_fix(f5 + idx, Q - qreq);
        } else {
          raise_flag(M.status, PMP_FLAG_OVERFLOW);
        }
      }
    }
  }
}

// Removal limiter of Sec. 3.1.1: at most cap * rho unless the Truelove
// condition asks for more, and never below rho_floor.
__device__ __forceinline__ double limited_removal(double K, double rho, const Limits& L) {
  if (!(K > 0.0)) return 0.0;
  const double capped = (K < L.cap * rho) ? K : L.cap * rho;
  const double tr = rho - L.rho_tr;
  const double lim = (capped > tr) ? capped : tr;
  double room = rho - L.rho_floor;
  if (room < 0.0) room = 0.0;
  return (lim < room) ? lim : room;
}

// Step 4 (Sec. 2.2): each sink re-evaluates its removal over its kernel and
// gains sum eta k V (mass) and sum eta k V p/rho (momentum), eta = Kl/K from
// the folded buffer and the state before Step 5.  One wavefront per sink;
// fixed point sums each term on the 2^-40 grid.
template <int ACC, class S>
__global__ __launch_bounds__(64) void k_sink_update(Mesh M, Particles P,
                                                    const S* __restrict__ state,
                                                    const typename AccT<ACC>::T* __restrict__ buf,
                                                    const double* __restrict__ scratch,
                                                    double r_k, double r_gauss, Limits L,
                                                    double* dm, double* dpx, double* dpy,
                                                    double* dpz) {
  constexpr bool FIXED = (ACC == PMP_ACC_FIX64);
  const int lane = threadIdx.x;
  const DevBox B = M.boxes[0];
  const int g = M.ghost;
  const double r2 = r_k * r_k, g2 = r_gauss * r_gauss;
  for (long long s = blockIdx.x; s < P.n; s += gridDim.x) {
    const double x = P.x[s], y = P.y[s], z = P.z[s];
    const double W = scratch[2 * s], Mreq = scratch[2 * s + 1];
    double sm = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    long long qm = 0, qx = 0, qy = 0, qz = 0;
    bool ok = true;
    int h[3];
    if (W > 0.0 && host_cell(B, x, y, z, h)) {
      int lo[3], hi[3];
      sphere_range(x, r_k, lo[0], hi[0]);
      sphere_range(y, r_k, lo[1], hi[1]);
      sphere_range(z, r_k, lo[2], hi[2]);
      const int cx = hi[0] - lo[0] + 1, cy = hi[1] - lo[1] + 1;
      const int cxy = cx * cy;
      const int total = cxy * (hi[2] - lo[2] + 1);
      for (int t = lane; t < total; t += kWave) {
        const int kk = t / cxy, rem = t - kk * cxy, jj = rem / cx, ii = rem - jj * cx;
        const int i = lo[0] + ii, j = lo[1] + jj, k = lo[2] + kk;
        const double d2 = dist2(x, y, z, i, j, k);
        if (!(d2 <= r2)) continue;
        const int iw = imod(i, M.domain[0]), jw = imod(j, M.domain[1]), kw = imod(k, M.domain[2]);
        const long long c = state_cell<S>(B, iw, jw, kw);
        const double rho = (double)state[B.soff + c];
        const double w = kernel_exp(-(d2 / g2));
        const double kreq = (Mreq * w) / (W * M.V);
        const double tr = rho - L.rho_tr;
        const double kc = (tr > kreq) ? tr : kreq;
        const long long bidx = ((long long)(kw - B.lo[2] + g) * B.p[1] + (jw - B.lo[1] + g)) *
                                   B.p[0] + (iw - B.lo[0] + g);
        const double K = to_f64(buf[B.boff + 5 * B.npad + bidx]);
        const double Kl = limited_removal(K, rho, L);
        const double eta = (K > 0.0) ? Kl / K : 1.0;
        const double term = (eta * kc) * M.V;
        const double vx = (double)state[B.soff + B.ncell + c] / rho;
        const double vy = (double)state[B.soff + 2 * B.ncell + c] / rho;
        const double vz = (double)state[B.soff + 3 * B.ncell + c] / rho;
        if constexpr (FIXED) {
          long long a0, a1, a2, a3;
          if (!quantise(term, a0) || !quantise(term * vx, a1) || !quantise(term * vy, a2) ||
              !quantise(term * vz, a3)) { ok = false; continue; }
          qm += a0; qx += a1; qy += a2; qz += a3;
        } else {
          sm += term;
          sx += term * vx;
          sy += term * vy;
          sz += term * vz;
        }
      }
    }
    if constexpr (FIXED) {
      qm = group_sum<kWave>(qm);
      qx = group_sum<kWave>(qx);
      qy = group_sum<kWave>(qy);
      qz = group_sum<kWave>(qz);
      sm = (double)qm * kFixInv;
      sx = (double)qx * kFixInv;
      sy = (double)qy * kFixInv;
      sz = (double)qz * kFixInv;
    } else {
      sm = group_sum<kWave>(sm);
      sx = group_sum<kWave>(sx);
      sy = group_sum<kWave>(sy);
      sz = group_sum<kWave>(sz);
    }
    if (!ok) raise_flag(M.status, PMP_FLAG_OVERFLOW);
    if (lane == 0) {
      dm[s] = sm;
      dpx[s] = sx;
      dpy[s] = sy;
      dpz[s] = sz;
    }
  }
}

// -------------------------------------------------------------- ghost fold

// Owned cell number t (0 <= t < shell count) of the shell of a box: the cells
// within g of a face.  Order: z bands (low then high) whole planes, then in
// the interior z layers the y bands whole rows, then in the interior rows the
// x bands.
__device__ __forceinline__ void shell_cell(const int n[3], int g, long long t, int& i, int& j,
                                           int& k) {
  const int glz = min(g, n[2]), hsz = max(glz, n[2] - g), nbz = glz + (n[2] - hsz);
  const long long plane = (long long)n[0] * n[1];
  const long long cz = (long long)nbz * plane;
  if (t < cz) {
    const int kk = (int)(t / plane);
    const long long r = t - (long long)kk * plane;
    k = kk < glz ? kk : hsz + (kk - glz);
    j = (int)(r / n[0]);
    i = (int)(r - (long long)j * n[0]);
    return;
  }
  t -= cz;
  const int gly = min(g, n[1]), hsy = max(gly, n[1] - g), nby = gly + (n[1] - hsy);
  const long long cyc = (long long)(hsz - glz) * nby * n[0];
  if (t < cyc) {
    const long long row = t / n[0];
    i = (int)(t - row * n[0]);
    const int jj = (int)(row % nby);
    k = glz + (int)(row / nby);
    j = jj < gly ? jj : hsy + (jj - gly);
    return;
  }
  t -= cyc;
  const int glx = min(g, n[0]), hsx = max(glx, n[0] - g), nbx = glx + (n[0] - hsx);
  const int ii = (int)(t % nbx);
  const long long r = t / nbx;
  const int midy = hsy - gly;
  j = gly + (int)(r % midy);
  k = glz + (int)(r / midy);
  i = ii < glx ? ii : hsx + (ii - glx);
}

// Step 2 (Sec. 2.2; App. A.2): each owned shell cell gathers every ghost cell
// whose periodic image it is, in the fixed order of the plan, and writes the
// sum once.  Float buffers sum in double and round once.
template <int ACC, int F>
__global__ __launch_bounds__(1024) void k_fold(Mesh M, typename AccT<ACC>::T* __restrict__ buf) {
  using T = typename AccT<ACC>::T;
  using Sum = typename std::conditional<ACC == PMP_ACC_FIX64, long long, double>::type;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const int g = M.ghost;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < M.shell_cells;
       t += stride) {
    const int b = (M.nbox == 1) ? 0 : find_box(M.shell_prefix, M.nbox, t);
    const DevBox B = M.boxes[b];
    int i, j, k;
    shell_cell(B.n, g, t - M.shell_prefix[b], i, j, k);
    const long long dst = B.boff + ((long long)(k + g) * B.p[1] + (j + g)) * B.p[0] + (i + g);
    Sum acc[F];
#pragma unroll
    for (int f = 0; f < F; ++f) acc[f] = (Sum)buf[dst + f * B.npad];
    bool any = false;
    const int s1 = M.seg_off[b + 1];
    for (int s = M.seg_off[b]; s < s1; ++s) {
      const DevSeg S = M.segs[s];
      if (i < S.lo[0] || i >= S.hi[0] || j < S.lo[1] || j >= S.hi[1] || k < S.lo[2] ||
          k >= S.hi[2])
        continue;
      const DevBox& Bs = M.boxes[S.src];
      const long long src = Bs.boff + ((long long)(k + S.off[2]) * Bs.p[1] + (j + S.off[1])) *
                                          Bs.p[0] + (i + S.off[0]);
#pragma unroll
      for (int f = 0; f < F; ++f) acc[f] += (Sum)buf[src + f * Bs.npad];
      any = true;
    }
    if (any) {
#pragma unroll
      for (int f = 0; f < F; ++f) buf[dst + f * B.npad] = (T)acc[f];
    }
  }
}

// ------------------------------------------------------------------ apply

// Steps 3 + 5 per owned cell, in double precision (see pmp_apply).
template <class S, int ACC, int F>
__global__ __launch_bounds__(1024) void k_apply(Mesh M, S* __restrict__ state,
                                               const typename AccT<ACC>::T* __restrict__ buf,
                                               Limits L, double* __restrict__ eta) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const int g = M.ghost;
  unsigned long long touched = 0, bind = 0, lamc = 0, fall = 0;
  bool bad = false;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < M.owned_cells;
       t += stride) {
    const int b = (M.nbox == 1) ? 0 : find_box(M.owned_prefix, M.nbox, t);
    const DevBox B = M.boxes[b];
    const long long c = t - M.owned_prefix[b];
    const long long row = c / B.n[0];
    const int i = (int)(c - row * B.n[0]);
    const int j = (int)(row % B.n[1]);
    const int k = (int)(row / B.n[1]);
    const long long bi = B.boff + ((long long)(k + g) * B.p[1] + (j + g)) * B.p[0] + (i + g);
    S* st = state + B.soff + c;
    const double rho = (double)st[0];
    const double px = (double)st[B.ncell];
    const double py = (double)st[2 * B.ncell];
    const double pz = (double)st[3 * B.ncell];
    const double E = (double)st[4 * B.ncell];
    const double Dr = to_f64(buf[bi]);
    const double qx = to_f64(buf[bi + B.npad]);
    const double qy = to_f64(buf[bi + 2 * B.npad]);
    const double qz = to_f64(buf[bi + 3 * B.npad]);
    const double DE = to_f64(buf[bi + 4 * B.npad]);
    const double K = (F == 6) ? to_f64(buf[bi + 5 * B.npad]) : 0.0;
    const double Kl = limited_removal(K, rho, L);
    if (K > 0.0) {
      ++touched;
      if (Kl < K) ++bind;
    }
    const double f = 1.0 - Kl / rho;
    const double rho1 = f * rho + Dr;
    double E1 = f * E + DE;
    const double p0x = f * px, p0y = f * py, p0z = f * pz;
    double emin = 0.0;
    if (L.eint_mode == 1) {
      const double eint0 = E - ((px * px + py * py) + pz * pz) / (2.0 * rho);
      emin = rho1 * (eint0 / rho);
    }
    const double Kc = (2.0 * rho1) * (E1 - emin);
    const double sx = p0x + qx, sy = p0y + qy, sz = p0z + qz;
    const double g1 = ((sx * sx + sy * sy) + sz * sz) - Kc;
    const double pp = (p0x * p0x + p0y * p0y) + p0z * p0z;
    const double g0 = pp - Kc;
    double lam;
    if (g1 <= 0.0) {
      lam = 1.0;
    } else if (g0 <= 0.0) {
      const double qq = (qx * qx + qy * qy) + qz * qz;
      const double pq = (p0x * qx + p0y * qy) + p0z * qz;
      const double disc = pq * pq - qq * g0;
      const double sq = sqrt(disc);
      lam = (pq > 0.0) ? (-g0) / (pq + sq) : (sq - pq) / qq;
      if (lam > 1.0) lam = 1.0;
      if (lam < 0.0) lam = 0.0;
    } else {
      lam = 0.0;
      E1 = emin + pp / (2.0 * rho1);
      ++fall;
    }
    if (lam < 1.0) ++lamc;
    if (!(rho > 0.0) || !isfinite(E1) || !isfinite(rho1)) bad = true;
    st[0] = (S)rho1;
    st[B.ncell] = (S)(p0x + lam * qx);
    st[2 * B.ncell] = (S)(p0y + lam * qy);
    st[3 * B.ncell] = (S)(p0z + lam * qz);
    st[4 * B.ncell] = (S)E1;
    if (eta) eta[M.owned_prefix[b] + c] = (K > 0.0) ? Kl / K : 1.0;
  }
  // one atomic per wavefront and counter
  touched = group_sum<kWave>(touched);
  bind = group_sum<kWave>(bind);
  lamc = group_sum<kWave>(lamc);
  fall = group_sum<kWave>(fall);
  const unsigned long long nbad = group_sum<kWave>((unsigned long long)bad);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    if (touched) atomicAdd(&M.status->touched, touched);
    if (bind) atomicAdd(&M.status->bind, bind);
    if (lamc) atomicAdd(&M.status->lam, lamc);
    if (fall) {
      atomicAdd(&M.status->fall, fall);
      atomicOr(&M.status->flags, PMP_FLAG_FLOOR);
    }
    if (nbad) atomicOr(&M.status->flags, PMP_FLAG_NAN);
  }
}

inline int grid_for(long long n, int block, int cap) {
  long long g = (n + block - 1) / block;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_zero(void* buf, long long bytes, int block, hipStream_t s) {
  const long long n16 = bytes / 16;
  const int ntail = (int)((bytes - n16 * 16) / 4);
  const int grid = grid_for(n16, block, 256 * 32);
  hipLaunchKernelGGL(k_zero, dim3(grid), dim3(block), 0, s, (u32x4*)buf, n16,
                     (unsigned*)((char*)buf + n16 * 16), ntail);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, long long bytes, hipStream_t s) {
  const long long n16 = bytes / 16;
  const int ntail = (int)((bytes - n16 * 16) / 4);
  const int grid = grid_for(n16, 256, 256 * 32);
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, s, (uint4*)dst, (const uint4*)src, n16,
                     (unsigned*)((char*)dst + n16 * 16),
                     (const unsigned*)((const char*)src + n16 * 16), ntail);
  return hipGetLastError();
}

hipError_t launch_clear_status(DevStatus* st, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_cic_direct(const Mesh& M, const Particles& P, void* buf, const BinWork* bw,
                             int dense_min, int block, hipStream_t s) {
  if (P.n <= 0) return hipSuccess;
  const int grid = grid_for(P.n, block, M.num_cu * 32);
  const int* key = bw ? bw->key : nullptr;
  const int* cnt = bw ? bw->count : nullptr;
  switch (M.acc) {
    case PMP_ACC_F32:
      hipLaunchKernelGGL(k_cic_direct<PMP_ACC_F32>, dim3(grid), dim3(block), 0, s, M, P,
                         (float*)buf, key, cnt, dense_min);
      break;
    case PMP_ACC_F64:
      hipLaunchKernelGGL(k_cic_direct<PMP_ACC_F64>, dim3(grid), dim3(block), 0, s, M, P,
                         (double*)buf, key, cnt, dense_min);
      break;
    default:
      hipLaunchKernelGGL(k_cic_direct<PMP_ACC_FIX64>, dim3(grid), dim3(block), 0, s, M, P,
                         (long long*)buf, key, cnt, dense_min);
  }
  return hipGetLastError();
}

template <int ACC>
static void sn_launch_lanes(const Mesh& M, const Particles& P, void* buf, int lanes,
                            hipStream_t s) {
  using T = typename AccT<ACC>::T;
  const int block = 256;
  const long long groups_needed = P.n;
  const int per_block = block / lanes;
  const int grid = grid_for(groups_needed * lanes, block, M.num_cu * 64);
  (void)per_block;
  if (lanes == 16)
    hipLaunchKernelGGL((k_sn_direct<ACC, 16>), dim3(grid), dim3(block), 0, s, M, P, (T*)buf);
  else if (lanes == 32)
    hipLaunchKernelGGL((k_sn_direct<ACC, 32>), dim3(grid), dim3(block), 0, s, M, P, (T*)buf);
  else
    hipLaunchKernelGGL((k_sn_direct<ACC, 64>), dim3(grid), dim3(block), 0, s, M, P, (T*)buf);
}

hipError_t launch_sn_direct(const Mesh& M, const Particles& P, void* buf, int lanes,
                            hipStream_t s) {
  if (P.n <= 0) return hipSuccess;
  switch (M.acc) {
    case PMP_ACC_F32: sn_launch_lanes<PMP_ACC_F32>(M, P, buf, lanes, s); break;
    case PMP_ACC_F64: sn_launch_lanes<PMP_ACC_F64>(M, P, buf, lanes, s); break;
    default: sn_launch_lanes<PMP_ACC_FIX64>(M, P, buf, lanes, s);
  }
  return hipGetLastError();
}

template <int ACC, class S>
static void sink_dep(const Mesh& M, const Particles& P, const void* state, void* buf,
                     double* scratch, double r_k, double r_g, double rho_tr, hipStream_t s) {
  const int grid = grid_for(P.n, 1, 65536);
  hipLaunchKernelGGL((k_sink_deposit<ACC, S>), dim3(grid), dim3(64), 0, s, M, P,
                     (const S*)state, (typename AccT<ACC>::T*)buf, scratch, r_k, r_g, rho_tr);
}

hipError_t launch_sink_deposit(const Mesh& M, const Particles& P, const void* state,
                               void* buf, double* scratch, double r_k, double r_gauss,
                               const Limits& L, hipStream_t s) {
  if (P.n <= 0) return hipSuccess;
  const bool f32 = (M.state == PMP_STATE_F32);
  switch (M.acc) {
    case PMP_ACC_F32:
      f32 ? sink_dep<PMP_ACC_F32, float>(M, P, state, buf, scratch, r_k, r_gauss, L.rho_tr, s)
          : sink_dep<PMP_ACC_F32, double>(M, P, state, buf, scratch, r_k, r_gauss, L.rho_tr, s);
      break;
    case PMP_ACC_F64:
      f32 ? sink_dep<PMP_ACC_F64, float>(M, P, state, buf, scratch, r_k, r_gauss, L.rho_tr, s)
          : sink_dep<PMP_ACC_F64, double>(M, P, state, buf, scratch, r_k, r_gauss, L.rho_tr, s);
      break;
    default:
      f32 ? sink_dep<PMP_ACC_FIX64, float>(M, P, state, buf, scratch, r_k, r_gauss, L.rho_tr, s)
          : sink_dep<PMP_ACC_FIX64, double>(M, P, state, buf, scratch, r_k, r_gauss, L.rho_tr,
                                            s);
  }
  return hipGetLastError();
}

template <int ACC, class S>
static void sink_upd(const Mesh& M, const Particles& P, const void* state, const void* buf,
                     const double* scratch, double r_k, double r_g, const Limits& L,
                     double* dm, double* dpx, double* dpy, double* dpz, hipStream_t s) {
  const int grid = grid_for(P.n, 1, 65536);
  hipLaunchKernelGGL((k_sink_update<ACC, S>), dim3(grid), dim3(64), 0, s, M, P,
                     (const S*)state, (const typename AccT<ACC>::T*)buf, scratch, r_k, r_g, L,
                     dm, dpx, dpy, dpz);
}

hipError_t launch_sink_update(const Mesh& M, const Particles& P, const void* state,
                              const void* buf, const double* scratch, double r_k,
                              double r_gauss, const Limits& L, double* dm, double* dpx,
                              double* dpy, double* dpz, hipStream_t s) {
  if (P.n <= 0) return hipSuccess;
  const bool f32 = (M.state == PMP_STATE_F32);
#define PMP_SU(ACC)                                                                         \
  (f32 ? sink_upd<ACC, float>(M, P, state, buf, scratch, r_k, r_gauss, L, dm, dpx, dpy, dpz, \
                              s)                                                            \
       : sink_upd<ACC, double>(M, P, state, buf, scratch, r_k, r_gauss, L, dm, dpx, dpy,     \
                               dpz, s))
  switch (M.acc) {
    case PMP_ACC_F32: PMP_SU(PMP_ACC_F32); break;
    case PMP_ACC_F64: PMP_SU(PMP_ACC_F64); break;
    default: PMP_SU(PMP_ACC_FIX64);
  }
#undef PMP_SU
  return hipGetLastError();
}

template <int ACC>
static void fold_launch(const Mesh& M, void* buf, int block, hipStream_t s) {
  using T = typename AccT<ACC>::T;
  const int grid = grid_for(M.shell_cells, block, M.num_cu * 32);
  if (M.nfield == 6)
    hipLaunchKernelGGL((k_fold<ACC, 6>), dim3(grid), dim3(block), 0, s, M, (T*)buf);
  else
    hipLaunchKernelGGL((k_fold<ACC, 5>), dim3(grid), dim3(block), 0, s, M, (T*)buf);
}

hipError_t launch_fold(const Mesh& M, void* buf, int block, hipStream_t s) {
  if (M.shell_cells <= 0) return hipSuccess;
  switch (M.acc) {
    case PMP_ACC_F32: fold_launch<PMP_ACC_F32>(M, buf, block, s); break;
    case PMP_ACC_F64: fold_launch<PMP_ACC_F64>(M, buf, block, s); break;
    default: fold_launch<PMP_ACC_FIX64>(M, buf, block, s);
  }
  return hipGetLastError();
}

template <class S, int ACC>
static void apply_launch(const Mesh& M, void* state, const void* buf, const Limits& L,
                         double* eta, int block, hipStream_t s) {
  using T = typename AccT<ACC>::T;
  const int grid = grid_for(M.owned_cells, block, M.num_cu * 32);
  if (M.nfield == 6)
    hipLaunchKernelGGL((k_apply<S, ACC, 6>), dim3(grid), dim3(block), 0, s, M, (S*)state,
                       (const T*)buf, L, eta);
  else
    hipLaunchKernelGGL((k_apply<S, ACC, 5>), dim3(grid), dim3(block), 0, s, M, (S*)state,
                       (const T*)buf, L, eta);
}

hipError_t launch_apply(const Mesh& M, void* state, const void* buf, const Limits& L,
                        double* eta, int block, hipStream_t s) {
  const bool f32 = (M.state == PMP_STATE_F32);
  switch (M.acc) {
    case PMP_ACC_F32:
      f32 ? apply_launch<float, PMP_ACC_F32>(M, state, buf, L, eta, block, s)
          : apply_launch<double, PMP_ACC_F32>(M, state, buf, L, eta, block, s);
      break;
    case PMP_ACC_F64:
      f32 ? apply_launch<float, PMP_ACC_F64>(M, state, buf, L, eta, block, s)
          : apply_launch<double, PMP_ACC_F64>(M, state, buf, L, eta, block, s);
      break;
    default:
      f32 ? apply_launch<float, PMP_ACC_FIX64>(M, state, buf, L, eta, block, s)
          : apply_launch<double, PMP_ACC_FIX64>(M, state, buf, L, eta, block, s);
  }
  return hipGetLastError();
}

hipError_t launch_cic_binned(const Mesh& M, const Particles& P, void* buf, BinWork& bw,
                             const pmp_tuning& t, hipStream_t s) {
  (void)M; (void)P; (void)buf; (void)bw; (void)t; (void)s;
  return hipErrorNotSupported;
}

}  // namespace pmp
