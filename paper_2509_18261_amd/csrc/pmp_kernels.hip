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

#include <algorithm>
#include <type_traits>

#include "pmp_internal.h"

namespace pmp {
namespace {

constexpr double kFix = 0x1p40;         // fixed-point scale (40 fractional bits)
constexpr double kFixInv = 0x1p-40;
constexpr double kFixLimit = 0x1p62;    // largest accepted magnitude of a scaled value
constexpr double kFourPi = 0x1.921fb54442d18p+3;  // 4 pi, rounded to double
constexpr double kPi = 0x1.921fb54442d18p+1;      // pi, rounded to double
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

// Natural logarithm for the power laws of the supernova-remnant deposit
// (Sec. 3.2.1: M_sf and P_snr), from the series ln m = 2 atanh(s) =
// 2 (s + s^3/3 + ... + s^23/23), s = (m - 1)/(m + 1), on m in [sqrt(1/2),
// sqrt(2)) after x = m 2^e (|s| <= 0.172, omitted terms below 2^-60
// relative), Horner's rule, plus e ln 2 with the head/tail split of
// kernel_exp (e * head exact).
__device__ double kernel_log(double x) {
  if (x != x || x < 0.0) return __builtin_nan("");
  if (x == 0.0) return -__builtin_huge_val();
  if (__builtin_isinf(x)) return x;
  int e;
  double m = frexp(x, &e);
  if (m < 0x1.6a09e667f3bcdp-1) {  // sqrt(1/2), rounded to double
    m = m * 2.0;
    e = e - 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double s2 = s * s;
  double t = 1.0 / 23.0;
  t = t * s2 + 1.0 / 21.0;
  t = t * s2 + 1.0 / 19.0;
  t = t * s2 + 1.0 / 17.0;
  t = t * s2 + 1.0 / 15.0;
  t = t * s2 + 1.0 / 13.0;
  t = t * s2 + 1.0 / 11.0;
  t = t * s2 + 1.0 / 9.0;
  t = t * s2 + 1.0 / 7.0;
  t = t * s2 + 1.0 / 5.0;
  t = t * s2 + 1.0 / 3.0;
  t = t * s2 + 1.0;
  const double lnm = (2.0 * s) * t;
  const double ln2_head = 0x1.62e42ffp-1;
  const double ln2_tail = -0x1.718432a1b0e26p-35;
  const double k = (double)e;
  return k * ln2_head + (k * ln2_tail + lnm);
}

// x^a = exp(a ln x), x > 0.
__device__ __forceinline__ double kernel_pow(double x, double a) {
  return kernel_exp(a * kernel_log(x));
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

// Box of particle p when it is known to lie in boxes [lo, hi].
__device__ __forceinline__ int find_box_in(const long long* off, int lo, int hi, long long p) {
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= p) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Boxes holding particles [p0, p1) of a block (shared by the block): two
// searches per block, after which each particle's search is over the few
// boxes in between.  Call from every thread of the block.
__device__ __forceinline__ void block_box_range(const long long* off, int nbox, long long p0,
                                                long long p1, int& b0, int& b1) {
  __shared__ int sb[2];
  if (nbox == 1) {
    b0 = b1 = 0;
    return;
  }
  if (threadIdx.x == 0) sb[0] = find_box(off, nbox, p0);
  if (threadIdx.x == 1 || (blockDim.x == 1 && threadIdx.x == 0))
    sb[1] = find_box(off, nbox, max(p0, p1 - 1));
  __syncthreads();
  b0 = sb[0];
  b1 = sb[1];
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

// Candidate range along one axis for a sphere of radius r >= 0 centred at p:
// a superset of the cells whose centre passes the test dist2 <= r^2, which
// alone decides membership.  A member i has |i + 1/2 - p| <= r (1 + 3 eps)
// (every rounding in the test is relative), so it lies in
// [p - r - 1/2, p + r - 1/2] up to far less than the 1e-6 margin, which also
// covers rounding of the bounds.  The range may be empty (hi = lo - 1).
__device__ __forceinline__ void sphere_range(double p, double r, int& lo, int& hi) {
  lo = (int)ceil(p - r - 0.5 - 1e-6);
  hi = (int)floor(p + r - 0.5 + 1e-6);
}


__device__ __forceinline__ int imod(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

// Exact t / d for 0 <= t < 2^22 and d >= 1, from the float reciprocal inv =
// 1/d: the estimate is within one of the quotient, and one correction step
// settles it (far cheaper than an integer division, which gfx950 lacks).
__device__ __forceinline__ int small_div(int t, int d, float inv) {
  int q = (int)((float)t * inv);
  const int r = t - q * d;
  q += (r >= d) ? 1 : 0;
  q -= (r < 0) ? 1 : 0;
  return q;
}

// Offsets (ii, jj, kk) of entry t of a cube walked in (k, j, i) order with i
// fastest, cx cells along x and cxy per z plane; t < 2^22.
__device__ __forceinline__ void cube_cell(int t, int cx, int cxy, int& ii, int& jj, int& kk) {
  kk = small_div(t, cxy, 1.0f / (float)cxy);
  const int rem = t - kk * cxy;
  jj = small_div(rem, cx, 1.0f / (float)cx);
  ii = rem - jj * cx;
}

// accumulator element types
template <int ACC> struct AccT;
template <> struct AccT<PMP_ACC_F32> { using T = float; };
template <> struct AccT<PMP_ACC_F64> { using T = double; };
template <> struct AccT<PMP_ACC_FIX64> { using T = long long; };
template <> struct AccT<PMP_ACC_F64R> { using T = double; };

// Reproducibility mode (App. A.1): machine epsilon of double, and a summed
// buffer element v with error bound e truncated: its lowest
// nb = 52 + M + ceil(log2(e / |v|)) mantissa bits cleared, nb clamped to
// [0, 52].  ceil(log2 r) comes from frexp (r = m 2^k, m in [1/2, 1): k - 1
// when m = 1/2, else k), so it is exact.  Zero and non-finite sums, and
// elements nothing was added to, are left as they are.
constexpr double kEps = 0x1p-52;
__device__ __forceinline__ double truncate_bound(double v, double e, int margin) {
  if (v == 0.0 || !isfinite(v) || !(e > 0.0)) return v;
  int k;
  const double m = frexp(e / fabs(v), &k);
  int nb = 52 + margin + ((m == 0.5) ? k - 1 : k);
  if (nb <= 0) return v;
  nb = min(nb, 52);
  const unsigned long long mask = ~((1ull << nb) - 1ull);
  return __longlong_as_double((long long)((unsigned long long)__double_as_longlong(v) & mask));
}

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

// Sphere rows.  Fix a row (j, k) of the candidate box: the rounded test value
// dist2(i) is non-increasing up to the row's nearest cell i = floor(x) and
// non-decreasing after it (the rounded offset ((double)i + 0.5) - x is
// monotone in i and rounding is monotone), so the cells passing
// dist2 <= r^2 form one run [a, b].  row_members finds it from the
// real-arithmetic half-width and settles both ends with the exact test, which
// yields exactly the cells that testing every candidate would.
struct Sphere {
  double x, y, z, r2;
  int lo[3], hi[3];  // candidate range (global cells), a superset of the members
  int cy;            // candidate rows along y
  int nrows;         // candidate rows (j, k), k-major
  float icy;         // 1 / cy
};

__device__ __forceinline__ void sphere_init(Sphere& S, double x, double y, double z, double r) {
  S.x = x;
  S.y = y;
  S.z = z;
  S.r2 = r * r;
  sphere_range(x, r, S.lo[0], S.hi[0]);
  sphere_range(y, r, S.lo[1], S.hi[1]);
  sphere_range(z, r, S.lo[2], S.hi[2]);
  S.cy = S.hi[1] - S.lo[1] + 1;
  S.nrows = S.cy * (S.hi[2] - S.lo[2] + 1);
  S.icy = 1.0f / (float)S.cy;
}

__device__ __forceinline__ int small_div(int t, int d, float inv);

__device__ __forceinline__ void sphere_row(const Sphere& S, int t, int& j, int& k) {
  const int kk = small_div(t, S.cy, S.icy);
  k = S.lo[2] + kk;
  j = S.lo[1] + (t - kk * S.cy);
}

// Members [a, b] of row (j, k); empty when a > b.

// Members [a, b] of the row with rounded squared offsets y2, z2 of a sphere
// centred at x along the row, with r2 = r^2 and candidate cells [lo, hi].
// The run's ends are estimated in single precision; the exact test at the
// nearest cell c, at both estimated ends and at their outer neighbours runs
// as five independent evaluations, and only an estimate that is off (rare)
// walks further.
__device__ __forceinline__ void row_run(double x, double r2, int lo, int hi, double y2,
                                        double z2, int& a, int& b) {
  // the test value of cell i: the same rounded operations, in the same
  // order, as dist2 with dy^2 = y2 and dz^2 = z2
  auto d2 = [&](int i) {
    const double ddx = ((double)i + 0.5) - x;
    return (ddx * ddx + y2) + z2;
  };
  const int c = (int)floor(x);
  const float w2 = (float)(r2 - (y2 + z2));
  const float w = w2 > 0.0f ? sqrtf(w2) : 0.0f;
  const float xc = (float)(x - 0.5);
  int aa = (int)ceilf(xc - w), bb = (int)floorf(xc + w);
  aa = min(max(aa, lo), c);
  bb = max(min(bb, hi), c);
  const bool in_c = d2(c) <= r2;
  const bool in_a = d2(aa) <= r2, out_a = !(aa > lo && d2(aa - 1) <= r2);
  const bool in_b = d2(bb) <= r2, out_b = !(bb < hi && d2(bb + 1) <= r2);
  if (!in_c) {
    a = 1;
    b = 0;
    return;
  }
  // c is a member, so aa < c when aa is not, and bb > c when bb is not
  if (!out_a) {
    --aa;
    while (aa > lo && d2(aa - 1) <= r2) --aa;
  } else if (!in_a) {
    ++aa;
    while (aa < c && !(d2(aa) <= r2)) ++aa;
  }
  if (!out_b) {
    ++bb;
    while (bb < hi && d2(bb + 1) <= r2) ++bb;
  } else if (!in_b) {
    --bb;
    while (bb > c && !(d2(bb) <= r2)) --bb;
  }
  a = aa;
  b = bb;
}

__device__ __forceinline__ void row_members_yz(const Sphere& S, double y2, double z2, int& a,
                                               int& b) {
  row_run(S.x, S.r2, S.lo[0], S.hi[0], y2, z2, a, b);
}

// Members [a, b] of row (j, k); empty when a > b.
__device__ __forceinline__ void row_members(const Sphere& S, int j, int k, int& a, int& b) {
  const double dy = ((double)j + 0.5) - S.y, dz = ((double)k + 0.5) - S.z;
  row_members_yz(S, dy * dy, dz * dz, a, b);
}

// Count of a sphere over a group of L lanes (lanes over rows): member count
// N, the first member in (k, j, i) order packed as (row << 12) | (i - lo_x),
// whether the host cell h is a member, and whether a member falls outside
// the padded box B.
template <int L>
__device__ __forceinline__ void sphere_count(const Sphere& S, const DevBox& B, int g,
                                             const int h[3], int lane, int& N, int& first,
                                             int& hostm, int& outside,
                                             unsigned short* rows = nullptr) {
  int cnt = 0, key = 0x7fffffff, hm = 0, out = 0;
  for (int t = lane; t < S.nrows; t += L) {
    int j, k, a, b;
    sphere_row(S, t, j, k);
    row_members(S, j, k, a, b);
    if (rows)
      rows[t] = (a > b) ? (unsigned short)0x00ff
                        : (unsigned short)((a - S.lo[0]) | ((b - S.lo[0]) << 8));
    if (a > b) continue;
    cnt += b - a + 1;
    key = min(key, (t << 12) | (a - S.lo[0]));
    hm |= (j == h[1] && k == h[2] && a <= h[0] && h[0] <= b);
    long long idx;
    out |= !pad_index(B, g, a, j, k, idx) || !pad_index(B, g, b, j, k, idx);
  }
  N = group_sum<L>(cnt);
  first = group_min<L>(key);
  hostm = group_max<L>(hm);
  outside = group_max<L>(out);
}

// Global cell of a packed first-member key.
__device__ __forceinline__ void sphere_key_cell(const Sphere& S, int key, int& i, int& j,
                                                int& k) {
  sphere_row(S, key >> 12, j, k);
  i = S.lo[0] + (key & 4095);
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

// A second copy variant for the bandwidth calibration: a workgroup of 256
// threads moves groups of 1024 16-byte vectors, each thread four of them at
// a stride of 256 vectors (every load instruction coalesced over the
// wavefront, all four loads issued before the stores), nontemporal stores,
// grid-stride over the groups.
__global__ __launch_bounds__(256) void k_copy4(u32x4* __restrict__ d, const u32x4* __restrict__ s,
                                               long long ngroups) {
  for (long long gq = blockIdx.x; gq < ngroups; gq += gridDim.x) {
    const u32x4* src = s + gq * 1024 + threadIdx.x;
    u32x4 v0 = src[0], v1 = src[256], v2 = src[512], v3 = src[768];
    u32x4* dst = d + gq * 1024 + threadIdx.x;
    __builtin_nontemporal_store(v0, dst);
    __builtin_nontemporal_store(v1, dst + 256);
    __builtin_nontemporal_store(v2, dst + 512);
    __builtin_nontemporal_store(v3, dst + 768);
  }
}

// Global-atomic throughput microbenchmark: n_ops adds of 1 into dst[slots]
// (slots a power of two, mask = slots - 1).  pattern 0: op i -> element
// i & mask (a wavefront's 64 ops on consecutive elements); 1: a
// multiplicative hash of i, masked (scattered, distinct until the slots
// wrap); 2: element (i >> 62) & mask, i.e. element 0 for every op (all
// contend), computed from the lane's own index so that the address is a
// per-lane vector value like the other patterns'.
template <class T>
__device__ __forceinline__ void bench_add(T* p);
template <>
__device__ __forceinline__ void bench_add<unsigned long long>(unsigned long long* p) {
  atomicAdd(p, 1ull);
}
template <>
__device__ __forceinline__ void bench_add<float>(float* p) { unsafeAtomicAdd(p, 1.0f); }
template <>
__device__ __forceinline__ void bench_add<double>(double* p) { unsafeAtomicAdd(p, 1.0); }

template <class T>
__global__ __launch_bounds__(256) void k_atomic_bench(T* __restrict__ dst, unsigned long long mask,
                                                      int pattern, long long n_ops) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_ops; i += stride) {
    const unsigned long long u = (unsigned long long)i;
    unsigned long long e;
    if (pattern == 0) e = u & mask;
    else if (pattern == 1) e = ((u * 0x9E3779B97F4A7C15ull) >> 20) & mask;
    else e = (u >> 62) & mask;
    bench_add(dst + e);
  }
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
                                                    typename AccT<ACC>::T* __restrict__ buf) {
  using T = typename AccT<ACC>::T;
  constexpr bool FIXED = (ACC == PMP_ACC_FIX64);
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < P.n; p += stride) {
    const int b = (M.nbox == 1) ? 0 : find_box(P.box_off, M.nbox, p);
    const DevBox B = M.boxes[b];
    const double x = P.x[p], y = P.y[p], z = P.z[p], m = P.a[p];
    int h[3];
    if (!host_cell(B, x, y, z, h)) { raise_flag(M.status, PMP_FLAG_OUTSIDE); continue; }
    if (!isfinite(m)) { raise_flag(M.status, PMP_FLAG_NAN); continue; }
    T* base = buf + B.boff + M.slot[0] * B.npad;
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
// e/(N V).  A group of L lanes handles one particle, lanes over the sphere's
// rows: first the members are counted, then added.  If no centre lies within
// r the host cell takes the whole deposit.  Fixed point: residue to the host
// cell if it is a member, else to the first member in (k, j, i) order.
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
    Sphere S;
    sphere_init(S, x, y, z, r);
    int N, first, hostm, outside;
    sphere_count<L>(S, B, g, h, lane, N, first, hostm, outside);
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
    T* f0 = buf + B.boff + M.slot[0] * B.npad;
    T* f4 = buf + B.boff + M.slot[4] * B.npad;
    auto put = [&](int i, int j, int k) {
      long long idx;
      if (!pad_index(B, g, i, j, k, idx)) return;
      if constexpr (FIXED) {
        gadd_fix(f0 + idx, qr);
        gadd_fix(f4 + idx, qe);
      } else {
        gadd(f0 + idx, cr);
        gadd(f4 + idx, ce);
      }
    };
    if (only_host) {
      if (lane == 0) put(h[0], h[1], h[2]);
    } else {
      // candidates in (k, j, i) order, i fastest, so that the atomics of
      // adjacent lanes land in adjacent cells
      const int cx = S.hi[0] - S.lo[0] + 1, cxy = cx * S.cy;
      const int total = cxy * (S.hi[2] - S.lo[2] + 1);
      const float icx = 1.0f / (float)cx, icxy = 1.0f / (float)cxy;
      for (int t = lane; t < total; t += L) {
        const int kk = small_div(t, cxy, icxy), rem = t - kk * cxy;
        const int jj = small_div(rem, cx, icx), ii = rem - jj * cx;
        const int i = S.lo[0] + ii, j = S.lo[1] + jj, k = S.lo[2] + kk;
        if (dist2(x, y, z, i, j, k) <= S.r2) put(i, j, k);
      }
    }
    if (lane == 0 && outside) raise_flag(M.status, PMP_FLAG_REACH);
    if constexpr (FIXED) {
      if (lane == 0) {
        long long Qr, Qe;
        if (quantise(m / M.V, Qr) && quantise(e / M.V, Qe)) {
          int ti = h[0], tj = h[1], tk = h[2];
          if (!hostm) sphere_key_cell(S, first, ti, tj, tk);
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

// Where global cell (i, j, k) lives: wrapped into the periodic domain, the
// box that owns it (through the owner index when one box does not cover the
// domain), its local owned coordinates and the state element of its field 0.
// False when no box owns the cell.
struct CellLoc {
  const DevBox* B;
  int l[3];
  long long s;
};

// locate for a cell already wrapped into the domain (0 <= w[a] < domain[a]).
__device__ __forceinline__ bool locate_wrapped(const Mesh& M, const int w[3], CellLoc& L) {
  if (M.own_start == nullptr) {
    L.B = M.all_boxes;
  } else {
    const int bin = ((w[2] / M.own_bin[2]) * M.own_dims[1] + w[1] / M.own_bin[1]) *
                        M.own_dims[0] + w[0] / M.own_bin[0];
    const DevBox* hit = nullptr;
    for (int q = M.own_start[bin]; q < M.own_start[bin + 1] && hit == nullptr; ++q) {
      const DevBox* B = M.all_boxes + M.own_box[q];
      if ((unsigned)(w[0] - B->lo[0]) < (unsigned)B->n[0] &&
          (unsigned)(w[1] - B->lo[1]) < (unsigned)B->n[1] &&
          (unsigned)(w[2] - B->lo[2]) < (unsigned)B->n[2])
        hit = B;
    }
    if (hit == nullptr) return false;
    L.B = hit;
  }
  for (int a = 0; a < 3; ++a) L.l[a] = w[a] - L.B->lo[a];
  L.s = L.B->soff + ((long long)L.l[2] * L.B->n[1] + L.l[1]) * L.B->n[0] + L.l[0];
  return true;
}

__device__ __forceinline__ bool locate(const Mesh& M, int i, int j, int k, CellLoc& L) {
  const int w[3] = {imod(i, M.domain[0]), imod(j, M.domain[1]), imod(k, M.domain[2])};
  return locate_wrapped(M, w, L);
}

// Element of channel ch (its buffer slot) of the located cell in its owning
// box's padded buffer.
template <class T>
__device__ __forceinline__ T* owner_elem(const Mesh& M, T* buf, const CellLoc& Lc, int ch) {
  const DevBox& Bo = *Lc.B;
  const int g = M.ghost;
  return buf + Bo.boff + M.slot[ch] * Bo.npad +
         ((long long)(Lc.l[2] + g) * Bo.p[1] + (Lc.l[1] + g)) * Bo.p[0] + (Lc.l[0] + g);
}

// Box of sink s: the b with off[b] <= s < off[b + 1] (empty boxes skipped).
__device__ __forceinline__ int particle_box(const long long* off, int nbox, long long s) {
  int lo = 0, hi = nbox - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= s) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// One workgroup of kSinkBlock threads per sink.  Reductions over the
// workgroup: each wavefront reduces its lanes, then the wavefront results are
// combined in wavefront order (a fixed order, also for floats).  Every thread
// of the workgroup must call them (they synchronise).
constexpr int kSinkBlock = 256;

template <class T>
__device__ __forceinline__ T block_sum(T v) {
  __shared__ T red[kSinkBlock / kWave];
  v = group_sum<kWave>(v);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  T t = red[0];
#pragma unroll
  for (int w = 1; w < kSinkBlock / kWave; ++w) t += red[w];
  return t;
}

__device__ __forceinline__ int block_min(int v) {
  __shared__ int red[kSinkBlock / kWave];
  v = group_min<kWave>(v);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  int t = red[0];
#pragma unroll
  for (int w = 1; w < kSinkBlock / kWave; ++w) t = min(t, red[w]);
  return t;
}

__device__ __forceinline__ int block_max(int v) {
  __shared__ int red[kSinkBlock / kWave];
  v = group_max<kWave>(v);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  int t = red[0];
#pragma unroll
  for (int w = 1; w < kSinkBlock / kWave; ++w) t = max(t, red[w]);
  return t;
}

// Truelove density of one cell (Sec. 3.1.1, eq. "truelove"): the constant
// rho_tr, or with truelove_J > 0 the cell's own J^2 pi c_s^2 / (G dx^2), with
// c_s^2 = gamma (gamma - 1) e_int / rho, e_int = E - |p|^2 / (2 rho) taken as
// 0 where negative, and c_s = 0 where rho <= 0.
__device__ __forceinline__ double truelove_rho(const Limits& L, double rho, double px,
                                               double py, double pz, double E) {
  if (!(L.truelove_J > 0.0)) return L.rho_tr;
  double c2 = 0.0;
  if (rho > 0.0) {
    double eint = E - ((px * px + py * py) + pz * pz) / (2.0 * rho);
    if (!(eint > 0.0)) eint = 0.0;
    c2 = ((L.gamma * (L.gamma - 1.0)) * eint) / rho;
  }
  return (((L.truelove_J * L.truelove_J) * kPi) * c2) / ((L.G * L.dx) * L.dx);
}

// The Truelove density of the cell whose rho is st[0] (the other state
// fields at multiples of stride); reads only rho's field for a constant.
template <class S>
__device__ __forceinline__ double truelove_at(const Limits& L, const S* st, long long stride) {
  if (!(L.truelove_J > 0.0)) return L.rho_tr;
  return truelove_rho(L, (double)st[0], (double)st[stride], (double)st[2 * stride],
                      (double)st[3 * stride], (double)st[4 * stride]);
}

// Bondi-Hoyle request of one sink (Sec. 3.1.1, eqs. "rbh" and "mdot", and the
// clamp of r_acc), computed by every thread of the sink's workgroup.  Over the
// kernel cells, on the 2^-40 grid: gas mass sum rho V, momentum sum p V and
// sum rho V c_s with c_s^2 = gamma (gamma - 1) e_int / rho (e_int = E -
// |p|^2/(2 rho), negative values as 0; c_s = 0 where rho <= 0), and the cell
// count.  v_inf = |sum p V / M - v_sink|, c_inf = sum rho V c_s / M, rho_inf =
// M / (N V); r_BH = G m / (v_inf^2 + c_inf^2), mdot = 4 pi rho_inf r_BH^2
// (lambda^2 c_inf^2 + v_inf^2)^(1/2).  The request mdot dt is capped at M (M
// also when v_inf = c_inf = 0), r_acc = r_BH / dx clamped to [1/4, r_k/2].
template <class S>
__device__ void bondi_request(const Mesh& M, const S* __restrict__ state, const SinkParams& K,
                              long long s, double x, double y, double z, const int lo[3], int cx,
                              int cxy, int total, bool& ok, bool& reach, double& req,
                              double& racc) {
  const double r2 = K.r_k * K.r_k;
  long long qn = 0, qm = 0, qx = 0, qy = 0, qz = 0, qc = 0;
  for (int t = threadIdx.x; t < total; t += kSinkBlock) {
    int ii, jj, kk;
    cube_cell(t, cx, cxy, ii, jj, kk);
    const int i = lo[0] + ii, j = lo[1] + jj, k = lo[2] + kk;
    const double d2 = dist2(x, y, z, i, j, k);
    if (!(d2 <= r2)) continue;
    CellLoc Lc;
    if (!locate(M, i, j, k, Lc)) {
      reach = true;
      continue;
    }
    const long long c = Lc.s, nc = Lc.B->ncell;
    const double rho = (double)state[c];
    const double px = (double)state[c + nc];
    const double py = (double)state[c + 2 * nc];
    const double pz = (double)state[c + 3 * nc];
    const double E = (double)state[c + 4 * nc];
    double cs = 0.0;
    if (rho > 0.0) {
      double eint = E - ((px * px + py * py) + pz * pz) / (2.0 * rho);
      if (!(eint > 0.0)) eint = 0.0;
      cs = sqrt(((K.gamma * (K.gamma - 1.0)) * eint) / rho);
    }
    const double m = rho * M.V;
    long long a0, a1, a2, a3, a4;
    if (!quantise(m, a0) || !quantise(px * M.V, a1) || !quantise(py * M.V, a2) ||
        !quantise(pz * M.V, a3) || !quantise(m * cs, a4)) {
      ok = false;
      continue;
    }
    qm += a0; qx += a1; qy += a2; qz += a3; qc += a4;
    ++qn;
  }
  qn = block_sum(qn);
  qm = block_sum(qm);
  qx = block_sum(qx);
  qy = block_sum(qy);
  qz = block_sum(qz);
  qc = block_sum(qc);
  const double half = 0.5 * K.r_k;
  const double Mk = (double)qm * kFixInv;
  req = 0.0;
  racc = half;
  if (!(Mk > 0.0)) return;
  const double ux = ((double)qx * kFixInv) / Mk - K.vx[s];
  const double uy = ((double)qy * kFixInv) / Mk - K.vy[s];
  const double uz = ((double)qz * kFixInv) / Mk - K.vz[s];
  const double v2 = (ux * ux + uy * uy) + uz * uz;
  const double cinf = ((double)qc * kFixInv) / Mk;
  const double c2 = cinf * cinf;
  const double den = v2 + c2;
  if (!(den > 0.0)) {
    req = Mk;
    return;
  }
  const double rho_inf = Mk / ((double)qn * M.V);
  const double rbh = (K.G * K.m[s]) / den;
  const double mdot = ((kFourPi * rho_inf) * (rbh * rbh)) * sqrt((K.lambda * K.lambda) * c2 + v2);
  const double want = mdot * K.dt;
  req = (want <= Mk) ? want : Mk;
  const double rc = rbh / K.dx;
  racc = (rc < 0.25) ? 0.25 : ((rc > half) ? half : rc);
}

// Sink removal request (Sec. 3.1.1).  One workgroup per sink.  The request is
// the fraction a of the kernel gas mass with the fixed width r_gauss, or the
// Bondi-Hoyle request of bondi_request with its own width r_acc.  Pass 1 sums
// the Gaussian weights w = exp(-d^2/r_acc^2) (eq. "kernel") and the kernel gas
// mass sum rho V on the 2^-40 grid (exact, order-free).  Pass 2 adds each
// cell's removal k = max(M_req w / (W V), rho - rho_Tr) (eqs. "kernel_wgt",
// "accretion_function") to field 5 of the sink's own box, in its ghost zone
// where the kernel leaves the box (the fold moves it to the owners).  State
// reads go to the box that owns each (periodically wrapped) cell.  scratch
// receives W, M_req and r_acc^2 per sink.
template <int ACC, class S>
__global__ __launch_bounds__(kSinkBlock) void k_sink_deposit(Mesh M, Particles P,
                                                     const S* __restrict__ state,
                                                     typename AccT<ACC>::T* __restrict__ buf,
                                                     double* __restrict__ scratch, SinkParams K,
                                                     Limits L, double* __restrict__ bound) {
  constexpr bool FIXED = (ACC == PMP_ACC_FIX64);
  const int lane = threadIdx.x;
  const int g = M.ghost;
  const double r2 = K.r_k * K.r_k;
  for (long long s = blockIdx.x; s < P.n; s += gridDim.x) {
    const DevBox B = M.all_boxes[particle_box(P.box_off, M.nbox, s)];
    const double x = P.x[s], y = P.y[s], z = P.z[s];
    double* out = scratch + kSinkScratch * s;
    int h[3];
    if (!host_cell(B, x, y, z, h)) {
      if (lane == 0) {
        raise_flag(M.status, PMP_FLAG_OUTSIDE);
        out[0] = 0.0;
        out[1] = 0.0;
        out[2] = 0.0;
      }
      continue;
    }
    int lo[3], hi[3];
    sphere_range(x, K.r_k, lo[0], hi[0]);
    sphere_range(y, K.r_k, lo[1], hi[1]);
    sphere_range(z, K.r_k, lo[2], hi[2]);
    const int cx = hi[0] - lo[0] + 1, cy = hi[1] - lo[1] + 1;
    const int cxy = cx * cy;
    const int total = cxy * (hi[2] - lo[2] + 1);
    bool ok = true, reach_bad = false;
    double racc = K.r_gauss, Mbondi = 0.0;
    if (K.rate == PMP_SINK_BONDI)
      bondi_request<S>(M, state, K, s, x, y, z, lo, cx, cxy, total, ok, reach_bad, Mbondi, racc);
    const double g2 = racc * racc;
    long long wq = 0, mq = 0;
    for (int t = lane; t < total; t += kSinkBlock) {
      int ii, jj, kk;
      cube_cell(t, cx, cxy, ii, jj, kk);
      const int i = lo[0] + ii, j = lo[1] + jj, k = lo[2] + kk;
      const double d2 = dist2(x, y, z, i, j, k);
      if (!(d2 <= r2)) continue;
      CellLoc Lc;
      if (!locate(M, i, j, k, Lc)) {
        reach_bad = true;
        continue;
      }
      const double rho = (double)state[Lc.s];
      const double w = kernel_exp(-(d2 / g2));
      long long q1, q2;
      if (!quantise(w, q1) || !quantise(rho * M.V, q2)) { ok = false; continue; }
      wq += q1;
      mq += q2;
    }
    wq = block_sum(wq);
    mq = block_sum(mq);
    if (!ok) raise_flag(M.status, PMP_FLAG_OVERFLOW);
    if (reach_bad) raise_flag(M.status, PMP_FLAG_REACH);
    if (wq <= 0) {
      if (lane == 0) { out[0] = 0.0; out[1] = 0.0; out[2] = g2; }
      continue;
    }
    const double W = (double)wq * kFixInv;
    const double Mreq =
        (K.rate == PMP_SINK_BONDI) ? Mbondi : P.a[s] * ((double)mq * kFixInv);
    if (lane == 0) { out[0] = W; out[1] = Mreq; out[2] = g2; }
    using T = typename AccT<ACC>::T;
    T* f5 = buf + B.boff + M.slot[5] * B.npad;
    long long qreq = 0;
    int first = 0x7fffffff, hostm = 0;
    for (int t = lane; t < total; t += kSinkBlock) {
      int ii, jj, kk;
      cube_cell(t, cx, cxy, ii, jj, kk);
      const int i = lo[0] + ii, j = lo[1] + jj, k = lo[2] + kk;
      const double d2 = dist2(x, y, z, i, j, k);
      if (!(d2 <= r2)) continue;
      first = min(first, t);
      hostm |= (i == h[0] && j == h[1] && k == h[2]);
      CellLoc Lc;
      if (!locate(M, i, j, k, Lc)) {
        reach_bad = true;
        continue;
      }
      const double rho = (double)state[Lc.s];
      const double w = kernel_exp(-(d2 / g2));
      const double kreq = (Mreq * w) / (W * M.V);
      const double tr = rho - truelove_at(L, state + Lc.s, Lc.B->ncell);
      const double kc = (tr > kreq) ? tr : kreq;
      long long idx;
      if (!pad_index(B, g, i, j, k, idx)) { reach_bad = true; continue; }
      // the cell's element: in the home box's padded buffer (the fold moves
      // ghost cells later), or, on owner tiles, in the owning box's (no fold
      // follows)
      T* dst = f5 + idx;
      if (K.owner) dst = owner_elem(M, buf, Lc, 5);
      if constexpr (FIXED) {
        long long q1, q2;
        if (!quantise(kc, q1) || !quantise(kreq, q2)) { ok = false; continue; }
        gadd_fix(dst, q1);
        qreq += q2;
      } else if constexpr (ACC == PMP_ACC_F64R) {
        // the element's error bound (same index as the buffer) grows by
        // eps |sum after the addition| (the atomic returns the sum before)
        const double old = atomicAdd(dst, kc);
        atomicAdd(bound + (dst - buf), kEps * fabs(old + kc));
      } else {
        gadd(dst, kc);
      }
    }
    if (reach_bad) raise_flag(M.status, PMP_FLAG_REACH);
    if constexpr (FIXED) {
      qreq = block_sum(qreq);
      first = block_min(first);
      hostm = block_max(hostm);
      if (lane == 0) {
        long long Q;
        if (ok && quantise(Mreq / M.V, Q)) {
          int ti = h[0], tj = h[1], tk = h[2];
          if (!hostm) {
            int ii, jj, kk;
            cube_cell(first, cx, cxy, ii, jj, kk);
            ti = lo[0] + ii; tj = lo[1] + jj; tk = lo[2] + kk;
          }
          long long idx;
          if (pad_index(B, g, ti, tj, tk, idx)) {
            CellLoc Lr;
            if (!K.owner) gadd_fix(f5 + idx, Q - qreq);
            else if (locate(M, ti, tj, tk, Lr)) gadd_fix(owner_elem(M, buf, Lr, 5), Q - qreq);
          }
        } else {
          raise_flag(M.status, PMP_FLAG_OVERFLOW);
        }
      }
    }
  }
}

// Removal limiter of Sec. 3.1.1: at most cap * rho unless the Truelove
// condition (the cell's Truelove density rho_tr) asks for more, and never
// below rho_floor.
__device__ __forceinline__ double limited_removal(double K, double rho, double rho_tr,
                                                  const Limits& L) {
  if (!(K > 0.0)) return 0.0;
  const double capped = (K < L.cap * rho) ? K : L.cap * rho;
  const double tr = rho - rho_tr;
  const double lim = (capped > tr) ? capped : tr;
  double room = rho - L.rho_floor;
  if (room < 0.0) room = 0.0;
  return (lim < room) ? lim : room;
}

// Reproducibility mode: buffer elements with a nonzero error bound (those a
// global-atomic deposit reached) truncated once their deposits are complete.
__global__ __launch_bounds__(256) void k_truncate_bounds(double* __restrict__ buf,
                                                        const double* __restrict__ bound,
                                                        long long n, int margin) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double e = bound[i];
    if (e > 0.0) buf[i] = truncate_bound(buf[i], e, margin);
  }
}

// Step 4 (Sec. 2.2): each sink re-evaluates its removal over its kernel and
// gains sum eta k V (mass) and sum eta k V p/rho (momentum), eta = Kl/K from
// the folded buffer and the state before Step 5; W, the request and r_acc^2
// come from Step 1's scratch.  One workgroup per sink; fixed point sums each
// term on the 2^-40 grid.
template <int ACC, class S>
__global__ __launch_bounds__(kSinkBlock) void k_sink_update(Mesh M, Particles P,
                                                    const S* __restrict__ state,
                                                    const typename AccT<ACC>::T* __restrict__ buf,
                                                    const double* __restrict__ scratch,
                                                    double r_k, Limits L, double* dm,
                                                    double* dpx, double* dpy, double* dpz) {
  constexpr bool FIXED = (ACC == PMP_ACC_FIX64);
  const int lane = threadIdx.x;
  const int g = M.ghost;
  const double r2 = r_k * r_k;
  for (long long s = blockIdx.x; s < P.n; s += gridDim.x) {
    const DevBox B = M.all_boxes[particle_box(P.box_off, M.nbox, s)];
    const double x = P.x[s], y = P.y[s], z = P.z[s];
    const double* in = scratch + kSinkScratch * s;
    const double W = in[0], Mreq = in[1], g2 = in[2];
    double sm = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    long long qm = 0, qx = 0, qy = 0, qz = 0;
    bool ok = true, reach_bad = false;
    int h[3];
    if (W > 0.0 && host_cell(B, x, y, z, h)) {
      int lo[3], hi[3];
      sphere_range(x, r_k, lo[0], hi[0]);
      sphere_range(y, r_k, lo[1], hi[1]);
      sphere_range(z, r_k, lo[2], hi[2]);
      const int cx = hi[0] - lo[0] + 1, cy = hi[1] - lo[1] + 1;
      const int cxy = cx * cy;
      const int total = cxy * (hi[2] - lo[2] + 1);
      for (int t = lane; t < total; t += kSinkBlock) {
        int ii, jj, kk;
        cube_cell(t, cx, cxy, ii, jj, kk);
        const int i = lo[0] + ii, j = lo[1] + jj, k = lo[2] + kk;
        const double d2 = dist2(x, y, z, i, j, k);
        if (!(d2 <= r2)) continue;
        CellLoc Lc;
        if (!locate(M, i, j, k, Lc)) {
          reach_bad = true;
          continue;
        }
        const DevBox& Bo = *Lc.B;  // owner: its state and its folded buffer
        const double rho = (double)state[Lc.s];
        const double w = kernel_exp(-(d2 / g2));
        const double kreq = (Mreq * w) / (W * M.V);
        const double rtr = truelove_at(L, state + Lc.s, Bo.ncell);
        const double tr = rho - rtr;
        const double kc = (tr > kreq) ? tr : kreq;
        const long long bidx =
            ((long long)(Lc.l[2] + g) * Bo.p[1] + (Lc.l[1] + g)) * Bo.p[0] + (Lc.l[0] + g);
        const double K = to_f64(buf[Bo.boff + M.slot[5] * Bo.npad + bidx]);
        const double Kl = limited_removal(K, rho, rtr, L);
        const double eta = (K > 0.0) ? Kl / K : 1.0;
        const double term = (eta * kc) * M.V;
        const double vx = (double)state[Lc.s + Bo.ncell] / rho;
        const double vy = (double)state[Lc.s + 2 * Bo.ncell] / rho;
        const double vz = (double)state[Lc.s + 3 * Bo.ncell] / rho;
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
      qm = block_sum(qm);
      qx = block_sum(qx);
      qy = block_sum(qy);
      qz = block_sum(qz);
      sm = (double)qm * kFixInv;
      sx = (double)qx * kFixInv;
      sy = (double)qy * kFixInv;
      sz = (double)qz * kFixInv;
    } else {
      sm = block_sum(sm);
      sx = block_sum(sx);
      sy = block_sum(sy);
      sz = block_sum(sz);
    }
    if (!ok) raise_flag(M.status, PMP_FLAG_OVERFLOW);
    if (reach_bad) raise_flag(M.status, PMP_FLAG_REACH);
    if (lane == 0) {
      dm[s] = sm;
      dpx[s] = sx;
      dpy[s] = sy;
      dpz[s] = sz;
    }
  }
}

// ----------------------------------------- supernova remnants (TIGRESS)

// Sample points of cell (i, j, k) within the sphere of squared radius r2
// around (x, y, z): the centres of its ns^3 sub-cells of edge 1/ns (ns a
// power of two, so every coordinate is exact), each tested as
// (dx^2 + dy^2) + dz^2 <= r2.
__device__ __forceinline__ int covered_samples(double x, double y, double z, double r2, int i,
                                               int j, int k, int ns) {
  int c = 0;
  const double inv = 1.0 / (double)ns;  // a power of two: exact
  for (int c3 = 0; c3 < ns; ++c3) {
    const double dz = ((double)k + ((double)c3 + 0.5) * inv) - z;
    const double dz2 = dz * dz;
    for (int c2 = 0; c2 < ns; ++c2) {
      const double dy = ((double)j + ((double)c2 + 0.5) * inv) - y;
      const double dy2 = dy * dy;
      for (int c1 = 0; c1 < ns; ++c1) {
        const double dx = ((double)i + ((double)c1 + 0.5) * inv) - x;
        c += ((dx * dx + dy2) + dz2 <= r2) ? 1 : 0;
      }
    }
  }
  return c;
}

// Supernova remnants with the variant of the TIGRESS prescription of
// Sec. 3.2.1 (eqs. "du", "dp", "psnr").  One workgroup per remnant; lanes
// over the candidate cells [floor(x - r_K) - 1, floor(x + r_K) + 1]^3.
//   kernel   cells with a covered fraction w = (sample points within r_K) /
//            sub^3 > 0, or the host cell alone (w = 1) if there are none;
//   sums     V_snr = sum w V, M_gas = sum w rho V, P_gas = sum w p V on the
//            2^-40 grid (exact and order-free), the state read in the box
//            that owns each (periodically wrapped) cell;
//   scalars  M_snr = M_gas + M_ej, n_H = (M_snr / V_snr) nh_per_rho,
//            R_M = M_snr / (msf_coef n_H^-0.26), |p_rad| = psnr_coef
//            n_H^-0.17 (R_M > 1), sqrt(2 M_ej eps_K E_sn) (0.027 < R_M <= 1)
//            or 0, v_COM = (P_gas + M_ej v_s) / M_snr, E_kin = M_ej |v_s|^2/2;
//   deposit  per cell, a = w / V_snr and rhat from the remnant to the cell
//            centre (0 at the remnant): d rho = a M_ej, d p = w ((rho + M_ej /
//            V_snr) v_COM - p) + a |p_rad| rhat, d E = a (E_sn + E_kin) +
//            v_COM . (a |p_rad| rhat), added to the remnant's own box (its
//            ghost zone where the kernel leaves the box).
// Fixed point rounds every term on the 2^-40 grid; the mass and the injected
// energy keep the remainder rule (the residues of rint(M_ej / V 2^40) and
// rint((E_sn + E_kin) / V 2^40) to the host cell if it is a kernel cell,
// else to the first in (k, j, i) order).  info (nullable) [4][n]: V_snr,
// M_snr, n_H, |p_rad|.
template <int ACC, class S>
__global__ __launch_bounds__(kSinkBlock) void k_snr_deposit(Mesh M, SnrArgs A,
                                                    const S* __restrict__ state,
                                                    typename AccT<ACC>::T* __restrict__ buf,
                                                    double* __restrict__ info) {
  constexpr bool FIXED = (ACC == PMP_ACC_FIX64);
  using T = typename AccT<ACC>::T;
  const int lane = threadIdx.x;
  const int g = M.ghost;
  const double r2 = A.r_k * A.r_k;
  const int ns = A.sub;
  const double nsamp = (double)ns * (double)ns * (double)ns;
  for (long long s = blockIdx.x; s < A.n; s += gridDim.x) {
    const DevBox B = M.all_boxes[particle_box(A.box_off, M.nbox, s)];
    const double x = A.x[s], y = A.y[s], z = A.z[s];
    int h[3];
    if (!host_cell(B, x, y, z, h)) {
      if (lane == 0) raise_flag(M.status, PMP_FLAG_OUTSIDE);
      continue;
    }
    const double Mej = A.m[s], Esn = A.e[s];
    const double vs[3] = {A.vx[s], A.vy[s], A.vz[s]};
    int lo[3];
    const double pos[3] = {x, y, z};
    for (int a = 0; a < 3; ++a) lo[a] = (int)floor(pos[a] - A.r_k) - 1;
    const int cx = (int)floor(x + A.r_k) + 1 - lo[0] + 1;
    const int cy = (int)floor(y + A.r_k) + 1 - lo[1] + 1;
    const int cz = (int)floor(z + A.r_k) + 1 - lo[2] + 1;
    const int cxy = cx * cy, total = cxy * cz;
    // the kernel: some sample point within r_K (the host cell's nearest one
    // is the usual witness), else the host cell alone
    int any = covered_samples(x, y, z, r2, h[0], h[1], h[2], ns) > 0;
    if (!any) {
      for (int t = lane; t < total && !any; t += kSinkBlock) {
        int ii, jj, kk;
        cube_cell(t, cx, cxy, ii, jj, kk);
        any = covered_samples(x, y, z, r2, lo[0] + ii, lo[1] + jj, lo[2] + kk, ns) > 0;
      }
      any = block_max(any);
    }
    const bool alone = !any;
    long long qV = 0, qM = 0, qx = 0, qy = 0, qz = 0;
    bool ok = true, reach_bad = false;
    int first = 0x7fffffff, hostm = 0;
    for (int t = lane; t < total; t += kSinkBlock) {
      int ii, jj, kk;
      cube_cell(t, cx, cxy, ii, jj, kk);
      const int i = lo[0] + ii, j = lo[1] + jj, k = lo[2] + kk;
      const bool is_host = (i == h[0] && j == h[1] && k == h[2]);
      double w;
      if (alone) {
        if (!is_host) continue;
        w = 1.0;
      } else {
        const int c = covered_samples(x, y, z, r2, i, j, k, ns);
        if (c == 0) continue;
        w = (double)c / nsamp;
      }
      first = min(first, t);
      hostm |= is_host ? 1 : 0;
      CellLoc Lc;
      if (!locate(M, i, j, k, Lc)) {
        reach_bad = true;
        continue;
      }
      const long long c0 = Lc.s, nc = Lc.B->ncell;
      long long a0, a1, a2, a3, a4;
      if (!quantise(w * M.V, a0) || !quantise((w * (double)state[c0]) * M.V, a1) ||
          !quantise((w * (double)state[c0 + nc]) * M.V, a2) ||
          !quantise((w * (double)state[c0 + 2 * nc]) * M.V, a3) ||
          !quantise((w * (double)state[c0 + 3 * nc]) * M.V, a4)) {
        ok = false;
        continue;
      }
      qV += a0; qM += a1; qx += a2; qy += a3; qz += a4;
    }
    qV = block_sum(qV);
    qM = block_sum(qM);
    qx = block_sum(qx);
    qy = block_sum(qy);
    qz = block_sum(qz);
    const double Vsnr = (double)qV * kFixInv;
    if (!(Vsnr > 0.0)) {
      if (lane == 0) raise_flag(M.status, PMP_FLAG_NAN);
      continue;
    }
    const double Msnr = (double)qM * kFixInv + Mej;
    const double nH = (Msnr / Vsnr) * A.nh_per_rho;
    const double Msf = A.msf_coef * kernel_pow(nH, -0.26);
    const double RM = Msnr / Msf;
    double P = 0.0;
    if (RM > 1.0) P = A.psnr_coef * kernel_pow(nH, -0.17);
    else if (RM > 0.027) P = sqrt(((2.0 * Mej) * A.eps_k) * Esn);
    const double vc[3] = {((double)qx * kFixInv + Mej * vs[0]) / Msnr,
                          ((double)qy * kFixInv + Mej * vs[1]) / Msnr,
                          ((double)qz * kFixInv + Mej * vs[2]) / Msnr};
    const double Ekin = (0.5 * Mej) * ((vs[0] * vs[0] + vs[1] * vs[1]) + vs[2] * vs[2]);
    const double Eall = Esn + Ekin;
    const double dens_ej = Mej / Vsnr;
    if (info != nullptr && lane == 0) {
      info[s] = Vsnr;
      info[A.n + s] = Msnr;
      info[2 * A.n + s] = nH;
      info[3 * A.n + s] = P;
    }
    T* f0 = buf + B.boff + M.slot[0] * B.npad;
    T* f1 = buf + B.boff + M.slot[1] * B.npad;
    T* f2 = buf + B.boff + M.slot[2] * B.npad;
    T* f3 = buf + B.boff + M.slot[3] * B.npad;
    T* f4 = buf + B.boff + M.slot[4] * B.npad;
    long long qr_sum = 0, qe_sum = 0;
    for (int t = lane; t < total; t += kSinkBlock) {
      int ii, jj, kk;
      cube_cell(t, cx, cxy, ii, jj, kk);
      const int i = lo[0] + ii, j = lo[1] + jj, k = lo[2] + kk;
      double w;
      if (alone) {
        if (!(i == h[0] && j == h[1] && k == h[2])) continue;
        w = 1.0;
      } else {
        const int c = covered_samples(x, y, z, r2, i, j, k, ns);
        if (c == 0) continue;
        w = (double)c / nsamp;
      }
      CellLoc Lc;
      long long idx;
      if (!locate(M, i, j, k, Lc) || !pad_index(B, g, i, j, k, idx)) {
        reach_bad = true;
        continue;
      }
      const long long c0 = Lc.s, nc = Lc.B->ncell;
      const double rho = (double)state[c0];
      const double pc[3] = {(double)state[c0 + nc], (double)state[c0 + 2 * nc],
                            (double)state[c0 + 3 * nc]};
      const double aw = w / Vsnr;
      const double dr = aw * Mej;
      const double d[3] = {((double)i + 0.5) - x, ((double)j + 0.5) - y,
                           ((double)k + 0.5) - z};
      const double len = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
      const double pr = aw * P;
      double prad[3], dp[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        prad[a] = (len > 0.0) ? pr * (d[a] / len) : 0.0;
        dp[a] = w * ((rho + dens_ej) * vc[a] - pc[a]) + prad[a];
      }
      const double einj = aw * Eall;
      const double ecross = (vc[0] * prad[0] + vc[1] * prad[1]) + vc[2] * prad[2];
      if constexpr (FIXED) {
        long long q0, q1, q2, q3, q4, q5;
        if (!quantise(dr, q0) || !quantise(dp[0], q1) || !quantise(dp[1], q2) ||
            !quantise(dp[2], q3) || !quantise(einj, q4) || !quantise(ecross, q5)) {
          ok = false;
          continue;
        }
        gadd_fix(f0 + idx, q0);
        gadd_fix(f1 + idx, q1);
        gadd_fix(f2 + idx, q2);
        gadd_fix(f3 + idx, q3);
        gadd_fix(f4 + idx, (long long)((unsigned long long)q4 + (unsigned long long)q5));
        qr_sum += q0;
        qe_sum += q4;
      } else {
        gadd(f0 + idx, dr);
        gadd(f1 + idx, dp[0]);
        gadd(f2 + idx, dp[1]);
        gadd(f3 + idx, dp[2]);
        gadd(f4 + idx, einj + ecross);
      }
    }
    if (reach_bad) raise_flag(M.status, PMP_FLAG_REACH);
    if constexpr (FIXED) {
      qr_sum = block_sum(qr_sum);
      qe_sum = block_sum(qe_sum);
      first = block_min(first);
      hostm = block_max(hostm);
      if (lane == 0) {
        long long Qr, Qe;
        if (ok && quantise(Mej / M.V, Qr) && quantise(Eall / M.V, Qe)) {
          int ti = h[0], tj = h[1], tk = h[2];
          if (!hostm) {
            int ii, jj, kk;
            cube_cell(first, cx, cxy, ii, jj, kk);
            ti = lo[0] + ii; tj = lo[1] + jj; tk = lo[2] + kk;
          }
          long long idx;
          if (pad_index(B, g, ti, tj, tk, idx)) {
            gadd_fix(f0 + idx, (long long)((unsigned long long)Qr - (unsigned long long)qr_sum));
            gadd_fix(f4 + idx, (long long)((unsigned long long)Qe - (unsigned long long)qe_sum));
          }
        } else {
          raise_flag(M.status, PMP_FLAG_OVERFLOW);
        }
      }
    } else {
      if (!ok) raise_flag(M.status, PMP_FLAG_OVERFLOW);
    }
  }
}

// -------------------------------------------------------------- ghost fold

// Owned cell number t (0 <= t < shell count) of the shell of a box: the cells
// within g of a face.  Order: z bands (low then high) whole planes, then in
// the interior z layers the y bands whole rows, then in the interior rows the
// x bands.
__device__ __forceinline__ void shell_cell(const int n[3], int g, unsigned t, int& i, int& j,
                                           int& k) {
  const int glz = min(g, n[2]), hsz = max(glz, n[2] - g), nbz = glz + (n[2] - hsz);
  const unsigned nx = (unsigned)n[0];
  const unsigned plane = nx * (unsigned)n[1];
  const unsigned cz = (unsigned)nbz * plane;
  if (t < cz) {
    const unsigned kk = t / plane;
    const unsigned r = t - kk * plane;
    k = (int)kk < glz ? (int)kk : hsz + ((int)kk - glz);
    const unsigned jj = r / nx;
    j = (int)jj;
    i = (int)(r - jj * nx);
    return;
  }
  t -= cz;
  const int gly = min(g, n[1]), hsy = max(gly, n[1] - g), nby = gly + (n[1] - hsy);
  const unsigned cyc = (unsigned)(hsz - glz) * (unsigned)nby * nx;
  if (t < cyc) {
    const unsigned row = t / nx;
    i = (int)(t - row * nx);
    const unsigned kq = row / (unsigned)nby;
    const int jj = (int)(row - kq * (unsigned)nby);
    k = glz + (int)kq;
    j = jj < gly ? jj : hsy + (jj - gly);
    return;
  }
  t -= cyc;
  const int glx = min(g, n[0]), hsx = max(glx, n[0] - g), nbx = glx + (n[0] - hsx);
  const unsigned r = t / (unsigned)nbx;
  const int ii = (int)(t - r * (unsigned)nbx);
  const unsigned midy = (unsigned)(hsy - gly);
  const unsigned kq = r / midy;
  j = gly + (int)(r - kq * midy);
  k = glz + (int)kq;
  i = ii < glx ? ii : hsx + (ii - glx);
}

// Adds to acc every ghost cell (of any box) whose periodic image is owned
// cell (i, j, k) of box b, in the fixed order of the plan (App. A.2).
template <int ACC, int F, class Sum>
__device__ __forceinline__ bool fold_gather(const Mesh& M, int b, int i, int j, int k,
                                            const typename AccT<ACC>::T* __restrict__ buf,
                                            Sum acc[F]) {
  bool any = false;
  const DevBox& Bd = M.all_boxes[b];
  const int g = M.ghost;
  auto zone = [&](int v, int a) {
    const int gl = min(g, Bd.n[a]), hs = max(gl, Bd.n[a] - g);
    return v < gl ? 0 : (v < hs ? 1 : 2);
  };
  const int z = zone(i, 0) + 3 * zone(j, 1) + 9 * zone(k, 2);
  const int* zo = M.zone_off + 28 * b;
  const int q1 = zo[z + 1];
  for (int q = zo[z]; q < q1; ++q) {
    const ZoneSeg& S = M.zone_seg[q];
    if (i < S.lo[0] || i >= S.hi[0] || j < S.lo[1] || j >= S.hi[1] || k < S.lo[2] ||
        k >= S.hi[2])
      continue;
    const long long src = S.base + ((long long)k * S.p1 + j) * S.p0 + i;
#pragma unroll
    for (int f = 0; f < F; ++f) acc[f] += (Sum)buf[src + f * S.npad];
    any = true;
  }
  return any;
}

template <int ACC>
using SumT = typename std::conditional<ACC == PMP_ACC_FIX64, long long, double>::type;

// Step 2 (Sec. 2.2; App. A.2): each owned shell cell gathers every ghost cell
// whose periodic image it is, in the fixed order of the plan, and writes the
// sum once.  Float buffers sum in double and round once.
template <int ACC, int F>
__global__ __launch_bounds__(kChunk) void k_fold(Mesh M, typename AccT<ACC>::T* __restrict__ buf) {
  using T = typename AccT<ACC>::T;
  using Sum = SumT<ACC>;
  const int g = M.ghost;
  for (long long ch = blockIdx.x; ch < M.n_fold_chunks; ch += gridDim.x) {
    const int2 C = M.fold_chunks[ch];
    const int b = C.x;
    const DevBox B = M.all_boxes[b];
    const int t = C.y + (int)threadIdx.x;
    if (t >= B.shell) continue;
    int i, j, k;
    shell_cell(B.n, g, (unsigned)t, i, j, k);
    const long long dst = B.boff + ((long long)(k + g) * B.p[1] + (j + g)) * B.p[0] + (i + g);
    Sum acc[F];
#pragma unroll
    for (int f = 0; f < F; ++f) acc[f] = (Sum)buf[dst + f * B.npad];
    if (fold_gather<ACC, F>(M, b, i, j, k, buf, acc)) {
#pragma unroll
      for (int f = 0; f < F; ++f) buf[dst + f * B.npad] = (T)acc[f];
    }
  }
}

// ------------------------------------------------------------------ apply

// Limiter counters of one thread, reduced per wavefront before the atomics.
struct ApplyCounts {
  unsigned long long touched = 0, bind = 0, lam = 0, fall = 0;
  bool bad = false;
};

// Steps 3 + 5 for one owned cell, in double precision: st points at the
// cell's rho, the other state fields follow at multiples of stride; (Dr, q,
// DE, K) is the folded buffer.  Returns eta = Kl / K (1 when K = 0).  Reads
// all five fields (the energy limiter needs |p|^2); writes rho and E, and
// the momentum only where it changes.  A cell whose update is zero in every
// channel is left alone: Step 5 adds nothing and the limiters act on
// updates (its state is neither read nor written).
template <class S>
__device__ __forceinline__ double apply_cell(S* st, long long stride, double Dr, double qx,
                                             double qy, double qz, double DE, double K,
                                             const Limits& L, ApplyCounts& cnt) {
  if (Dr == 0.0 && qx == 0.0 && qy == 0.0 && qz == 0.0 && DE == 0.0 && K == 0.0) return 1.0;
  const double rho = (double)st[0];
  const double px = (double)st[stride];
  const double py = (double)st[2 * stride];
  const double pz = (double)st[3 * stride];
  const double E = (double)st[4 * stride];
  const double Kl =
      (K > 0.0) ? limited_removal(K, rho, truelove_rho(L, rho, px, py, pz, E), L) : 0.0;
  if (K > 0.0) {
    ++cnt.touched;
    if (Kl < K) ++cnt.bind;
  }
  // no removal: f = 1 - 0 / rho is exactly 1 for any nonzero, non-NaN rho
  double f = 1.0;
  if (!(Kl == 0.0 && rho != 0.0 && rho == rho)) f = 1.0 - Kl / rho;
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
    ++cnt.fall;
  }
  if (lam < 1.0) ++cnt.lam;
  if (!(rho > 0.0) || !isfinite(E1) || !isfinite(rho1)) cnt.bad = true;
  st[0] = (S)rho1;
  // momentum changes only through the removal (f < 1) or a momentum deposit:
  // otherwise the new value equals the stored one and is not written again
  if (f != 1.0 || qx != 0.0 || qy != 0.0 || qz != 0.0) {
    st[stride] = (S)(p0x + lam * qx);
    st[2 * stride] = (S)(p0y + lam * qy);
    st[3 * stride] = (S)(p0z + lam * qz);
  }
  st[4 * stride] = (S)E1;
  return (K > 0.0) ? Kl / K : 1.0;
}

// apply_cell for a cell without removal (K = 0) or momentum deposit (q = 0),
// with the same rounded operations: f = 1 - 0 / rho is exactly 1 for any
// nonzero, non-NaN rho, so rho1 = rho + Dr, E1 = E + DE, the momentum is
// unchanged (p + 0 squares to p^2), and the energy test reduces to
// |p|^2 - 2 rho1 E1 (e_int >= 0 mode): lam = 1, or the floor.  A zero or
// NaN rho, and the specific-e_int mode, take apply_cell itself.
template <class S>
__device__ __forceinline__ void apply_cell_nosrc(S* st, long long stride, double Dr, double DE,
                                                 const Limits& L, ApplyCounts& cnt) {
  if (Dr == 0.0 && DE == 0.0) return;  // no update: the cell is left alone
  const double rho = (double)st[0];
  if (!(rho != 0.0 && rho == rho) || L.eint_mode != 0) {
    apply_cell(st, stride, Dr, 0.0, 0.0, 0.0, DE, 0.0, L, cnt);
    return;
  }
  const double px = (double)st[stride];
  const double py = (double)st[2 * stride];
  const double pz = (double)st[3 * stride];
  const double E = (double)st[4 * stride];
  const double rho1 = rho + Dr;
  double E1 = E + DE;
  const double Kc = (2.0 * rho1) * E1;
  const double pp = (px * px + py * py) + pz * pz;
  if (!(pp - Kc <= 0.0)) {
    // lam = 0: the kinetic part stays, e_int at its floor
    E1 = 0.0 + pp / (2.0 * rho1);
    ++cnt.fall;
    ++cnt.lam;
  }
  if (!(rho > 0.0) || !isfinite(E1) || !isfinite(rho1)) cnt.bad = true;
  st[0] = (S)rho1;
  st[4 * stride] = (S)E1;
}

// One atomic per wavefront and counter (call from every lane of the wave).
__device__ __forceinline__ void flush_counts(const Mesh& M, ApplyCounts& cnt) {
  const unsigned long long touched = group_sum<kWave>(cnt.touched);
  const unsigned long long bind = group_sum<kWave>(cnt.bind);
  const unsigned long long lamc = group_sum<kWave>(cnt.lam);
  const unsigned long long fall = group_sum<kWave>(cnt.fall);
  const unsigned long long nbad = group_sum<kWave>((unsigned long long)cnt.bad);
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

// Steps 2 + 3 + 5 for the shell cells of a fused step: each shell cell
// gathers its ghost images in the plan's order (as k_fold) and is applied
// at once; the interior cells were applied by the tile pass.  (Register
// budget for 7 waves per SIMD; the apply kernel below fits 8.)
template <int ACC, int F>
__global__ __launch_bounds__(kChunk) __attribute__((amdgpu_waves_per_eu(7))) void k_fold_apply(Mesh M, void* __restrict__ state,
                                                      const typename AccT<ACC>::T* __restrict__ buf,
                                                      Limits L) {
  using Sum = SumT<ACC>;
  using T = typename AccT<ACC>::T;
  const int g = M.ghost;
  ApplyCounts cnt;
  for (long long ch = blockIdx.x; ch < M.n_fold_chunks; ch += gridDim.x) {
    const int2 C = M.fold_chunks[ch];
    const int b = C.x;
    const DevBox B = M.all_boxes[b];
    const int t = C.y + (int)threadIdx.x;
    if (t >= B.shell) continue;
    int i, j, k;
    shell_cell(B.n, g, (unsigned)t, i, j, k);
    const long long dst = B.boff + ((long long)(k + g) * B.p[1] + (j + g)) * B.p[0] + (i + g);
    Sum acc[F];
#pragma unroll
    for (int f = 0; f < F; ++f) acc[f] = (Sum)buf[dst + f * B.npad];
    fold_gather<ACC, F>(M, b, i, j, k, buf, acc);
    // the folded values as the buffer would hold them
    double v[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) v[q] = M.slot[q] >= 0 ? to_f64((T)acc[M.slot[q]]) : 0.0;
    const long long si = B.soff + ((long long)k * B.n[1] + j) * B.n[0] + i;
    // without momentum or removal channels (uniform): the source-free apply
    const bool nosrc = M.slot[1] < 0 && M.slot[2] < 0 && M.slot[3] < 0 && M.slot[5] < 0;
    if (M.state == PMP_STATE_F32) {
      if (nosrc) apply_cell_nosrc((float*)state + si, B.ncell, v[0], v[4], L, cnt);
      else apply_cell((float*)state + si, B.ncell, v[0], v[1], v[2], v[3], v[4], v[5], L, cnt);
    } else {
      if (nosrc) apply_cell_nosrc((double*)state + si, B.ncell, v[0], v[4], L, cnt);
      else apply_cell((double*)state + si, B.ncell, v[0], v[1], v[2], v[3], v[4], v[5], L, cnt);
    }
  }
  flush_counts(M, cnt);
}

// Steps 3 + 5 per owned cell, in double precision (see pmp_apply).
template <class S, int ACC>
__global__ __launch_bounds__(kChunk) __attribute__((amdgpu_waves_per_eu(8))) void k_apply(Mesh M, S* __restrict__ state,
                                                 const typename AccT<ACC>::T* __restrict__ buf,
                                                 Limits L, double* __restrict__ eta) {
  const int g = M.ghost;
  ApplyCounts cnt;
  // absent channels are identically zero (uniform branches)
  const int s0 = M.slot[0], s1 = M.slot[1], s2 = M.slot[2], s3 = M.slot[3], s4 = M.slot[4],
            s5 = M.slot[5];
  for (long long ch = blockIdx.x; ch < M.n_apply_chunks; ch += gridDim.x) {
    const int2 C = M.apply_chunks[ch];
    const int b = C.x;
    const DevBox B = M.all_boxes[b];
    const long long c = (long long)C.y + threadIdx.x;
    if (c >= B.ncell) continue;
    // box cells < 2^31: 32-bit index arithmetic
    const unsigned cu = (unsigned)c, nx = (unsigned)B.n[0], ny = (unsigned)B.n[1];
    const unsigned row = cu / nx;
    const int i = (int)(cu - row * nx);
    const unsigned kq = row / ny;
    const int j = (int)(row - kq * ny);
    const int k = (int)kq;
    const long long bi = B.boff + ((long long)(k + g) * B.p[1] + (j + g)) * B.p[0] + (i + g);
    const long long np = B.npad;
    const double Dr = s0 >= 0 ? to_f64(buf[bi + s0 * np]) : 0.0;
    const double qx = s1 >= 0 ? to_f64(buf[bi + s1 * np]) : 0.0;
    const double qy = s2 >= 0 ? to_f64(buf[bi + s2 * np]) : 0.0;
    const double qz = s3 >= 0 ? to_f64(buf[bi + s3 * np]) : 0.0;
    const double DE = s4 >= 0 ? to_f64(buf[bi + s4 * np]) : 0.0;
    const double K = s5 >= 0 ? to_f64(buf[bi + s5 * np]) : 0.0;
    const double e = apply_cell(state + B.soff + c, B.ncell, Dr, qx, qy, qz, DE, K, L, cnt);
    if (eta) eta[M.owned_prefix[b] + c] = e;
  }
  flush_counts(M, cnt);
}


// ------------------------------------------------------------- binned path
//
// Particles are binned into tiles of the padded box their stencil touches
// (a counting sort: count, scan, fill).  One workgroup then owns one tile:
// it accumulates every contribution to its cells in LDS (FP64 for the float
// buffers, int64 for fixed point) and stores each field of each cell once.
// No global atomics, and no separate zero fill: cells nobody touches are
// stored as zero.

// Padded-local cell range [lo, hi] of the CIC stencil of a particle.
__device__ __forceinline__ void cic_box(const DevBox& B, int g, double x, double y, double z,
                                        int lo[3], int hi[3]) {
  const double p[3] = {x, y, z};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = (int)floor(p[a] - 0.5) - B.lo[a] + g;
    hi[a] = lo[a] + 1;
  }
}

// Padded-local cell range holding every cell whose centre can pass the
// sphere test: a member i has |i + 1/2 - p| <= r (1 + 3 eps) (each rounding
// in the test is relative), so i lies in [p - r - 1/2, p + r - 1/2] up to far
// less than the 1e-6 margin, which also covers rounding of the bounds.
__device__ __forceinline__ void sphere_box(const DevBox& B, int g, double x, double y, double z,
                                           double r, int lo[3], int hi[3]) {
  const double p[3] = {x, y, z};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = (int)ceil(p[a] - r - 0.5 - 1e-6) - B.lo[a] + g;
    hi[a] = (int)floor(p[a] + r - 0.5 + 1e-6) - B.lo[a] + g;
  }
}

// Tiles overlapped by padded-local cells [lo, hi] clipped to the padded box.
__device__ __forceinline__ bool tile_range(const DevBox& B, const TileGrid& T, const int lo[3],
                                           const int hi[3], int tlo[3], int thi[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int l = max(lo[a], 0), h = min(hi[a], B.p[a] - 1);
    if (l > h) return false;
    if (a == 0) {
      // x boundaries at gx + k TX; the first and last tiles take the ghosts
      const int ntx = (B.n[0] + T.t[0] - 1) >> T.ts[0];
      tlo[0] = min(max(l - T.gx, 0) >> T.ts[0], ntx - 1);
      thi[0] = min(max(h - T.gx, 0) >> T.ts[0], ntx - 1);
    } else {
      tlo[a] = l >> T.ts[a];
      thi[a] = h >> T.ts[a];
    }
  }
  return true;
}

__device__ __forceinline__ long long tile_id(const TileGrid& T, int b, int tx, int ty, int tz) {
  const int* ta = T.tiles_axis + 3 * b;
  return T.tile_prefix[b] + ((long long)tz * ta[1] + ty) * ta[0] + tx;
}

// Owner tiles: calls f(tile id) once for every owner tile holding a cell of
// the global cell range [lo, hi] of a particle's own frame (hi - lo < domain
// per axis, lo > -domain) after wrapping it periodically.  Per axis the range
// wraps into at most two pieces; for each combination of pieces the boxes
// that meet it come from the owner index, each taken once, by the bin that
// holds the lowest cell of its intersection with the piece.  Distinct pieces
// never share a tile (the owner-tile condition), so each tile comes once.
// (owner_tiles_of below does the same for one known box.)
template <class F>
__device__ __forceinline__ void owner_tiles(const Mesh& M, const TileGrid& T, const int lo[3],
                                            const int hi[3], F&& f) {
  // per axis: pieces (l0, h0) and, when the range wraps, (l1, h1)
  int l0[3], h0[3], l1[3], h1[3], np[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int D = M.domain[a], l = lo[a], h = hi[a];
    np[a] = 1;
    l1[a] = 0;
    h1[a] = -1;
    if (l < 0 && h < 0) {
      l0[a] = l + D; h0[a] = h + D;
    } else if (l < 0) {
      l0[a] = 0; h0[a] = h; l1[a] = l + D; h1[a] = D - 1; np[a] = 2;
    } else if (l >= D) {
      l0[a] = l - D; h0[a] = h - D;
    } else if (h >= D) {
      l0[a] = l; h0[a] = D - 1; l1[a] = 0; h1[a] = h - D; np[a] = 2;
    } else {
      l0[a] = l; h0[a] = h;
    }
  }
  auto box_tiles = [&](int b, const DevBox& B, const int il[3], const int ih[3]) {
    int tlo[3], thi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      tlo[a] = (il[a] - B.lo[a]) >> T.ts[a];
      thi[a] = (ih[a] - B.lo[a]) >> T.ts[a];
    }
    for (int tz = tlo[2]; tz <= thi[2]; ++tz)
      for (int ty = tlo[1]; ty <= thi[1]; ++ty)
        for (int tx = tlo[0]; tx <= thi[0]; ++tx) f((int)tile_id(T, b, tx, ty, tz));
  };
  const int ncomb = np[0] * np[1] * np[2];
#pragma unroll 1
  for (int c = 0; c < ncomb; ++c) {
    const int cx = c % np[0], cy = (c / np[0]) % np[1], cz = c / (np[0] * np[1]);
    const int rl[3] = {cx ? l1[0] : l0[0], cy ? l1[1] : l0[1], cz ? l1[2] : l0[2]};
    const int rh[3] = {cx ? h1[0] : h0[0], cy ? h1[1] : h0[1], cz ? h1[2] : h0[2]};
    if (M.own_start == nullptr) {
      // one box covers the domain
      const int b = 0;
      const DevBox& B = M.all_boxes[b];
      int il[3], ih[3];
      bool hit = true;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        il[a] = max(rl[a], B.lo[a]);
        ih[a] = min(rh[a], B.lo[a] + B.n[a] - 1);
        hit = hit && il[a] <= ih[a];
      }
      if (hit) box_tiles(b, B, il, ih);
      continue;
    }
    int bl[3], bh[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      bl[a] = rl[a] / M.own_bin[a];
      bh[a] = rh[a] / M.own_bin[a];
    }
    for (int bz = bl[2]; bz <= bh[2]; ++bz)
      for (int by = bl[1]; by <= bh[1]; ++by)
        for (int bx = bl[0]; bx <= bh[0]; ++bx) {
          const int bin = (bz * M.own_dims[1] + by) * M.own_dims[0] + bx;
          const int bb[3] = {bx, by, bz};
          for (int q = M.own_start[bin]; q < M.own_start[bin + 1]; ++q) {
            const int b = M.own_box[q];
            const DevBox& B = M.all_boxes[b];
            int il[3], ih[3];
            bool hit = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              il[a] = max(rl[a], B.lo[a]);
              ih[a] = min(rh[a], B.lo[a] + B.n[a] - 1);
              hit = hit && il[a] <= ih[a] && il[a] / M.own_bin[a] == bb[a];
            }
            if (hit) box_tiles(b, B, il, ih);
          }
        }
  }
}

// Owner tiles: calls f(tile id) once for every owner tile of box R holding a
// cell of the global range [lo, hi] (as owner_tiles) after wrapping it.
template <class F>
__device__ __forceinline__ void owner_tiles_of(const Mesh& M, const NbrBox& R, const TileGrid& T,
                                               const int lo[3], const int hi[3], F&& f) {
  int tl[3][2], th[3][2], np[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int D = M.domain[a];
    // the range's periodic images that meet the box: shifts -D, 0, +D
    np[a] = 0;
#pragma unroll
    for (int k = -1; k <= 1; ++k) {
      const int l = max(lo[a] + k * D, R.lo[a]), h = min(hi[a] + k * D, R.lo[a] + R.n[a] - 1);
      if (l <= h && np[a] < 2) {
        tl[a][np[a]] = (l - R.lo[a]) >> T.ts[a];
        th[a][np[a]] = (h - R.lo[a]) >> T.ts[a];
        ++np[a];
      }
    }
  }
  for (int cz = 0; cz < np[2]; ++cz)
    for (int cy = 0; cy < np[1]; ++cy)
      for (int cx = 0; cx < np[0]; ++cx) {
        const int x0 = cx ? tl[0][1] : tl[0][0], x1 = cx ? th[0][1] : th[0][0];
        const int y0 = cy ? tl[1][1] : tl[1][0], y1 = cy ? th[1][1] : th[1][0];
        const int z0 = cz ? tl[2][1] : tl[2][0], z1 = cz ? th[2][1] : th[2][0];
        for (int tz = z0; tz <= z1; ++tz)
          for (int ty = y0; ty <= y1; ++ty)
            for (int tx = x0; tx <= x1; ++tx) f(R.tprefix + (tz * R.tax[1] + ty) * R.tax[0] + tx);
      }
}

// Calls f(tile id) for every tile holding a cell of the padded-local range
// [lo, hi] of box B (clipped to the padded box): the tiles of B itself (OWN
// 0), or the owner tiles of whichever boxes own those cells (OWN 1; OWN 2
// when one box covers the domain, so that box owns every cell).
template <int OWN, class F>
__device__ __forceinline__ void particle_tiles(const Mesh& M, const TileGrid& T, int b,
                                               const DevBox& B, const int lo[3], const int hi[3],
                                               F&& f, const NbrBox* nbr = nullptr) {
  if constexpr (!OWN) {
    int tlo[3], thi[3];
    if (!tile_range(B, T, lo, hi, tlo, thi)) return;
    for (int tz = tlo[2]; tz <= thi[2]; ++tz)
      for (int ty = tlo[1]; ty <= thi[1]; ++ty)
        for (int tx = tlo[0]; tx <= thi[0]; ++tx) f((int)tile_id(T, b, tx, ty, tz));
    return;
  } else {
  const int g = M.ghost;
  int gl[3], gh[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int l = max(lo[a], 0), h = min(hi[a], B.p[a] - 1);
    if (l > h) return;
    gl[a] = l - g + B.lo[a];
    gh[a] = h - g + B.lo[a];
  }
  // inside its own box's owned cells: that box's tiles, directly
  bool home = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) home = home && gl[a] >= B.lo[a] && gh[a] < B.lo[a] + B.n[a];
  if (home) {
    int tlo[3], thi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      tlo[a] = (gl[a] - B.lo[a]) >> T.ts[a];
      thi[a] = (gh[a] - B.lo[a]) >> T.ts[a];
    }
    for (int tz = tlo[2]; tz <= thi[2]; ++tz)
      for (int ty = tlo[1]; ty <= thi[1]; ++ty)
        for (int tx = tlo[0]; tx <= thi[0]; ++tx) f((int)tile_id(T, b, tx, ty, tz));
    return;
  }
  if constexpr (OWN == 2) {
    // one box covers the domain: its tiles, through the range's images
    NbrBox R;
    R.id = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      R.lo[a] = B.lo[a];
      R.n[a] = B.n[a];
      R.tax[a] = T.tiles_axis[a];
    }
    R.tprefix = 0;
    owner_tiles_of(M, R, T, gl, gh, f);
    return;
  }
  // the boxes that can own its cells: per direction the range reaches
  // beyond the box's faces, edges and corners, the one box the neighbour
  // table names (with its owner tiles); each distinct box then takes the
  // whole range (its owned cells clip it), so a box meets the range once.
  // Where several boxes meet one direction, or more than four boxes are
  // found, the owner index takes the whole range.
  // (first the directions and their box ids, at most four distinct boxes
  // kept as scalars; then each box's record again, from the cache)
  // box b's 27 records (nbr: a copy staged in LDS by the caller)
  const NbrBox* nb = nbr ? nbr : T.nbr + 27 * b;
  int i0 = -1, i1 = -1, i2 = -1, i3 = -1, d0 = 0, d1 = 0, d2 = 0, d3 = 0, count = 0;
  bool general = false;
  // per axis the range meets a run of the parts below (0), inside (1) and
  // above (2) the box: only those directions are visited
  int plo[3], phi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int lo_in = B.lo[a], hi_in = B.lo[a] + B.n[a] - 1;
    plo[a] = gl[a] < lo_in ? 0 : (gl[a] <= hi_in ? 1 : 2);
    phi[a] = gh[a] > hi_in ? 2 : (gh[a] >= lo_in ? 1 : 0);
  }
#pragma unroll 1
  for (int pz = plo[2]; pz <= phi[2]; ++pz)
#pragma unroll 1
    for (int py = plo[1]; py <= phi[1]; ++py)
#pragma unroll 1
      for (int px = plo[0]; px <= phi[0]; ++px) {
        const int d = (pz * 3 + py) * 3 + px;
        const int id = nb[d].id;
        if (id == -1) continue;  // no box owns cells there
        if (id == -2 || count == 4) {
          general = general || id == -2 || (id != i0 && id != i1 && id != i2 && id != i3);
          continue;
        }
        if (id == i0 || id == i1 || id == i2 || id == i3) continue;
        if (count == 0) { i0 = id; d0 = d; }
        else if (count == 1) { i1 = id; d1 = d; }
        else if (count == 2) { i2 = id; d2 = d; }
        else { i3 = id; d3 = d; }
        ++count;
      }
  if (general) {
    owner_tiles(M, T, gl, gh, f);
    return;
  }
#pragma unroll 1
  for (int q = 0; q < count; ++q) {
    const int d = q == 0 ? d0 : (q == 1 ? d1 : (q == 2 ? d2 : d3));
    const NbrBox R = nb[d];
    owner_tiles_of(M, R, T, gl, gh, f);
  }
  }
}

// Exclusive scan of count[0, n) into offset[0, n] (offset[n] = total) in
// three launches; count is cleared on the way (it becomes the fill cursor).
constexpr int kScanBlock = 1024;

__device__ __forceinline__ int block_inclusive_scan(int v, int* sh) {
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid / kWave;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int u = __shfl_up(v, o, kWave);
    if (lane >= o) v += u;
  }
  if (lane == kWave - 1) sh[wave] = v;
  __syncthreads();
  if (wave == 0) {
    int w = (lane < (int)(blockDim.x / kWave)) ? sh[lane] : 0;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int u = __shfl_up(w, o, kWave);
      if (lane >= o) w += u;
    }
    sh[lane] = w;
  }
  __syncthreads();
  if (wave > 0) v += sh[wave - 1];
  __syncthreads();
  return v;
}

// Exclusive scan in two launches.  The length is n, or, when dcount is
// given, min(n, *dcount << dshift) (a length known only on the device).
__device__ __forceinline__ long long scan_len(long long n, const int* dcount, int dshift) {
  return dcount ? min(n, (long long)(*dcount) << dshift) : n;
}

// Each block scans its kScanBlock values and leaves its total.
__global__ __launch_bounds__(kScanBlock) void k_scan_local(int* __restrict__ count,
                                                            int* __restrict__ offset,
                                                            int* __restrict__ block_sums,
                                                            long long n,
                                                            const int* __restrict__ dcount,
                                                            int dshift) {
  __shared__ int sh[kWave];
  n = scan_len(n, dcount, dshift);
  if ((long long)blockIdx.x * kScanBlock >= n) return;
  const long long i = (long long)blockIdx.x * kScanBlock + threadIdx.x;
  const int v = (i < n) ? count[i] : 0;
  const int inc = block_inclusive_scan(v, sh);
  if (i < n) offset[i] = inc - v;
  if (threadIdx.x == kScanBlock - 1) block_sums[blockIdx.x] = inc;
}

// Each block adds the total of the blocks before it, summed here (there are
// few); the last block writes offset[n], the grand total.
__global__ __launch_bounds__(kScanBlock) void k_scan_finish(int* __restrict__ offset,
                                                             const int* __restrict__ block_sums,
                                                             long long n,
                                                             const int* __restrict__ dcount,
                                                             int dshift) {
  __shared__ int sh[kWave];
  n = scan_len(n, dcount, dshift);
  const int nbe = (int)((n + kScanBlock - 1) / kScanBlock);
  const int b = blockIdx.x;
  if (b >= max(nbe, 1)) return;
  int part = 0;
  for (int i = threadIdx.x; i < b; i += blockDim.x) part += block_sums[i];
  part = group_sum<kWave>(part);
  if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = part;
  __syncthreads();
  int pre = 0;
  for (int w = 0; w < (int)(blockDim.x / kWave); ++w) pre += sh[w];
  const long long i = (long long)b * kScanBlock + threadIdx.x;
  if (i < n) offset[i] += pre;
  if (b == max(nbe, 1) - 1 && threadIdx.x == 0) offset[n] = pre + (nbe > 0 ? block_sums[b] : 0);
}

// Level 1 of the bucket sort, CIC.  Block k handles particles
// [k * kBinChunkCic, (k + 1) * kBinChunkCic).  Histogram pass (SCATTER =
// false): LDS counts of (particle, tile) pairs per coarse bucket, written to
// hist[bucket * nblk + k].  Scatter pass: hist holds the scanned positions;
// LDS cursors hand out slots and each pair's record (x, y, z, m) and tile are
// written there, so a block writes runs of consecutive slots per bucket.
// Column of level-1 block blk in a bucket's row of the histogram: blocks
// grouped by XCD (block i runs on XCD i mod 8), so that the counts sharing a
// cache line come from one XCD and merge in its L2.  A bijection on
// [0, nblk); positions within a bucket follow this order.
__device__ __forceinline__ int hist_col(int blk, int nblk) {
  const int x = blk & 7, k = nblk >> 3, r = nblk & 7;
  return x * k + min(x, r) + (blk >> 3);
}

// Owner tiles on several boxes: a level-1 block stages the neighbour records
// of its first kNbrCache boxes in LDS, so that the lookups of stencils that
// leave their box read LDS instead of waiting on global loads.
constexpr int kNbrCache = 4;
__device__ __forceinline__ void stage_nbr(const TileGrid& T, int bb0, int bb1, NbrBox* s) {
  const int n = 27 * min(bb1 - bb0 + 1, kNbrCache);
  for (int i = threadIdx.x; i < n; i += blockDim.x) s[i] = T.nbr[27 * bb0 + i];
}
__device__ __forceinline__ const NbrBox* nbr_of(const TileGrid& T, const NbrBox* s, int bb0,
                                                int b) {
  return (b - bb0 < kNbrCache) ? s + 27 * (b - bb0) : T.nbr + 27 * b;
}

template <bool SCATTER, int OWN>
__device__ __forceinline__ void l1_cic(int blk, const Mesh& M, const TileGrid& T,
                                       const Particles& P, int shift, int nb,
                                       int* __restrict__ hist, int nblk,
                                       double4* __restrict__ tmp, int* __restrict__ tmp_tile,
                                       long long cap, NbrBox* s_nbr) {
  extern __shared__ int h[];
  const int g = M.ghost;
  const int col = hist_col(blk, nblk);
  // hist is this kind's segment of the scanned histograms: positions are
  // taken relative to its first entry
  for (int c = threadIdx.x; c < nb; c += blockDim.x)
    h[c] = SCATTER ? hist[(long long)c * nblk + col] - hist[0] : 0;
  __syncthreads();
  const long long p0 = (long long)blk * kBinChunkCic;
  const long long p1 = min(p0 + kBinChunkCic, P.n);
  int bb0, bb1;
  block_box_range(P.box_off, M.nbox, p0, p1, bb0, bb1);
  if constexpr (OWN == 1) stage_nbr(T, bb0, bb1, s_nbr);  // read after the barriers below
  bool outside = false, nan = false, full = false;
  constexpr int UNR = kBinChunkCic / 256;
  // the thread's particles are loaded together, then binned one by one
  double px[UNR], py[UNR], pz[UNR], pm[UNR];
#pragma unroll
  for (int u = 0; u < UNR; ++u) {
    const long long p = p0 + threadIdx.x + (long long)u * blockDim.x;
    if (p < p1) {
      px[u] = P.x[p];
      py[u] = P.y[p];
      pz[u] = P.z[p];
      pm[u] = P.a[p];
    }
  }
  unsigned slow = 0;  // owner tiles: particles whose stencil leaves their box
  int sbox[UNR] = {};  // and their boxes (offsets from bb0)
#pragma unroll
  for (int u = 0; u < UNR; ++u) {
    const long long p = p0 + threadIdx.x + (long long)u * blockDim.x;
    if (p >= p1) continue;
    const int b = (bb0 == bb1) ? bb0 : find_box_in(P.box_off, bb0, bb1, p);
    const DevBox B = M.boxes[b];
    const double x = px[u], y = py[u], z = pz[u], m = pm[u];
    int hc[3];
    if (!host_cell(B, x, y, z, hc)) { outside = true; continue; }
    if (!isfinite(m)) { nan = true; continue; }
    int lo[3], hi[3], tlo[3], thi[3];
    cic_box(B, g, x, y, z, lo, hi);
    if constexpr (OWN) {
      // inside its box's owned cells: that box's owner tiles; else later
      bool home = true;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        home = home && lo[a] >= g && hi[a] < B.n[a] + g;
        tlo[a] = (lo[a] - g) >> T.ts[a];  // used only when home (offsets >= 0)
        thi[a] = (hi[a] - g) >> T.ts[a];
      }
      if (!home) {
        slow |= 1u << u;
        sbox[u] = b - bb0;
        continue;
      }
    } else {
      if (!tile_range(B, T, lo, hi, tlo, thi)) continue;
    }
    for (int tz = tlo[2]; tz <= thi[2]; ++tz)
      for (int ty = tlo[1]; ty <= thi[1]; ++ty)
        for (int tx = tlo[0]; tx <= thi[0]; ++tx) {
          const int t = (int)tile_id(T, b, tx, ty, tz);
          const int pos = atomicAdd(h + (t >> shift), 1);
          if (SCATTER) {
            if (pos < cap) {
              tmp[pos] = make_double4(x, y, z, m);
              tmp_tile[pos] = t;
            } else {
              full = true;
            }
          }
        }
  }
  if constexpr (OWN) {
    // stencils that reach other boxes or wrap (long code, long load
    // chains): gathered into a block-wide list and taken one per thread
    __shared__ int s_slow[kBinChunkCic];
    __shared__ int s_nslow;
    if (threadIdx.x == 0) s_nslow = 0;
    __syncthreads();
    // the box offset rides in the high bits when the block's box range fits
    // them (block-uniform), else the box is searched again
    const bool packed = bb1 - bb0 < (1 << (31 - kChunkBits));
    if (slow) {
      int at = atomicAdd(&s_nslow, __popc(slow));
#pragma unroll
      for (int u = 0; u < UNR; ++u)
        if ((slow >> u) & 1u)
          s_slow[at++] =
              ((int)threadIdx.x + u * (int)blockDim.x) | (packed ? sbox[u] << kChunkBits : 0);
    }
    __syncthreads();
    const int nslow = s_nslow;
#pragma unroll 1
    for (int i = threadIdx.x; i < nslow; i += blockDim.x) {
      const int sv = s_slow[i];
      const long long p = p0 + (sv & (kBinChunkCic - 1));
      const int b = packed ? bb0 + (sv >> kChunkBits) : find_box_in(P.box_off, bb0, bb1, p);
      const DevBox B = M.boxes[b];
      const double x = P.x[p], y = P.y[p], z = P.z[p], m = P.a[p];
      int lo[3], hi[3];
      cic_box(B, g, x, y, z, lo, hi);
      particle_tiles<OWN>(M, T, b, B, lo, hi, [&](int t) {
        const int pos = atomicAdd(h + (t >> shift), 1);
        if (SCATTER) {
          if (pos < cap) {
            tmp[pos] = make_double4(x, y, z, m);
            tmp_tile[pos] = t;
          } else {
            full = true;
          }
        }
      }, OWN == 1 ? nbr_of(T, s_nbr, bb0, b) : nullptr);
    }
  }
  if (!SCATTER) {
    if (outside) raise_flag(M.status, PMP_FLAG_OUTSIDE);
    if (nan) raise_flag(M.status, PMP_FLAG_NAN);
    __syncthreads();
    for (int c = threadIdx.x; c < nb; c += blockDim.x)
      hist[(long long)c * nblk + col] = h[c];
  } else if (full) {
    raise_flag(M.status, PMP_FLAG_CAPACITY);
  }
}

// Calls f(tile id) for the tiles a supernova's deposit touches: those of its
// sphere's candidate box, or of the host cell alone when N < 0.
template <int OWN, class F>
__device__ __forceinline__ void sn_tiles(const Mesh& M, const TileGrid& T, int b,
                                         const DevBox& B, double x, double y, double z,
                                         double r, int N, F&& f, const NbrBox* nbr = nullptr) {
  const int g = M.ghost;
  int slo[3], shi[3];
  if (N < 0) {
    const double q[3] = {x, y, z};
    for (int a = 0; a < 3; ++a) slo[a] = shi[a] = (int)floor(q[a]) - B.lo[a] + g;
  } else {
    sphere_box(B, g, x, y, z, r, slo, shi);
  }
  particle_tiles<OWN>(M, T, b, B, slo, shi, f, nbr);
}

// Supernova members, before binning: L lanes per particle (256 / L particles
// per block).  The lanes walk the sphere's candidate rows in (k, j) order,
// row t on lane t mod L: they count the members N (-1
// when no centre lies within r and the host cell takes the deposit; 0 when
// the particle is skipped) and find the fixed-point remainder cell (host if a
// member, else the first member in (k, j, i) order); the first lane writes
// the particle's SnPk.
template <int L>
__global__ __launch_bounds__(256) void k_sn_count(Mesh M, Particles P, SnPk* __restrict__ pk,
                                                  int wrap) {
  const int g = M.ghost;
  const long long p0 = (long long)blockIdx.x * (256 / L);
  const long long p1 = min(p0 + 256 / L, P.n);
  int bb0, bb1;
  block_box_range(P.box_off, M.nbox, p0, p1, bb0, bb1);
  const int sub = threadIdx.x & (L - 1);
  const long long p = p0 + threadIdx.x / L;
  const bool live = p < p1;
  const int b = !live ? 0 : (bb0 == bb1) ? bb0 : find_box_in(P.box_off, bb0, bb1, p);
  const DevBox B = M.boxes[b];
  double x = 0.5, y = 0.5, z = 0.5, m = 0.0, e = 0.0, r = 0.0;
  if (live) {
    x = P.x[p];
    y = P.y[p];
    z = P.z[p];
    m = P.b[p];
    e = P.c[p];
    r = P.r[p];
  }
  SnPk R;
  R.x = x;
  R.y = y;
  R.z = z;
  R.r = r;
  R.n = 0;
  R.ti = R.tj = R.tk = -1;
  R.vr = R.ve = 0.0;
  R.remr = R.reme = 0;
  int hc[3] = {0, 0, 0};
  unsigned flag = 0;
  if (live) {
    if (!host_cell(B, x, y, z, hc)) flag = PMP_FLAG_OUTSIDE;
    else if (!isfinite(m) || !isfinite(e) || !isfinite(r) || !(r >= 0.0)) flag = PMP_FLAG_NAN;
    else if (floor(r + 0.5) > (double)g) flag = PMP_FLAG_REACH;
  }
  const bool ok = live && !flag;
  Sphere Sp;
  sphere_init(Sp, x, y, z, ok ? r : 0.0);
  const int nrows = ok ? Sp.nrows : 0;
  // a row whose rounded dy^2 + dz^2 exceeds r^2 holds no member: the
  // rounded test value of each of its cells is at least that sum (the terms
  // are non-negative and rounding is monotone)
  int cnt = 0, key = 0x7fffffff, hm = 0, out = 0;
  // padded box of B, global cells
  const int plo[3] = {B.lo[0] - g, B.lo[1] - g, B.lo[2] - g};
  const int phi[3] = {B.lo[0] + B.n[0] + g - 1, B.lo[1] + B.n[1] + g - 1,
                      B.lo[2] + B.n[2] + g - 1};
  int jj = sub, kk = 0;  // row t = jj + cy * kk (cy >= 1 when there are rows)
  for (int t = sub; t < nrows; t += L) {
    while (jj >= Sp.cy) {
      jj -= Sp.cy;
      ++kk;
    }
    const int j = Sp.lo[1] + jj, k = Sp.lo[2] + kk;
    const double dy = ((double)j + 0.5) - Sp.y, dz = ((double)k + 0.5) - Sp.z;
    const double y2 = dy * dy, z2 = dz * dz;
    if (y2 + z2 <= Sp.r2) {
      int a, bb;
      row_members_yz(Sp, y2, z2, a, bb);
      if (a <= bb) {
        cnt += bb - a + 1;
        if (key == 0x7fffffff) key = (t << 12) | (a - Sp.lo[0]);  // the lane's first
        hm |= (j == hc[1] && k == hc[2] && a <= hc[0] && hc[0] <= bb);
        // a member outside the padded box
        out |= a < plo[0] || bb > phi[0] || j < plo[1] || j > phi[1] || k < plo[2] ||
               k > phi[2];
      }
    }
    jj += L;
  }
  cnt = group_sum<L>(cnt);
  key = group_min<L>(key);
  hm = group_max<L>(hm);
  out = group_max<L>(out);
  int N = cnt;
  if (ok && N == 0) N = -1;
  bool okq = ok;
  if (ok) {
    // member share, and for fixed point the remainder that makes the
    // deposited total exactly Q(m / V)
    const int NN = N < 0 ? 1 : N;
    const double cr = m / ((double)NN * M.V), ce = e / ((double)NN * M.V);
    if (M.acc == PMP_ACC_FIX64) {
      long long qr = 0, qe = 0, Qr = 0, Qe = 0;
      okq = quantise(cr, qr) && quantise(ce, qe) && quantise(m / M.V, Qr) &&
            quantise(e / M.V, Qe);
      R.vr = __longlong_as_double(qr);
      R.ve = __longlong_as_double(qe);
      R.remr = Qr - (long long)NN * qr;
      R.reme = Qe - (long long)NN * qe;
    } else {
      R.vr = cr;
      R.ve = ce;
    }
    if (!okq) flag = PMP_FLAG_OVERFLOW;
  }
  if (okq) {
    R.n = N;
    int ti = hc[0], tj = hc[1], tk = hc[2];
    if (N > 0 && !hm) sphere_key_cell(Sp, key, ti, tj, tk);
    long long idx;
    if (pad_index(B, g, ti, tj, tk, idx)) {
      if (wrap) {
        // owner tiles: the cell's periodic image, global
        R.ti = imod(ti, M.domain[0]);
        R.tj = imod(tj, M.domain[1]);
        R.tk = imod(tk, M.domain[2]);
      } else {
        R.ti = ti - B.lo[0] + g;
        R.tj = tj - B.lo[1] + g;
        R.tk = tk - B.lo[2] + g;
      }
    }
    if (out && sub == 0) raise_flag(M.status, PMP_FLAG_REACH);
  }
  if (flag && sub == 0) raise_flag(M.status, flag);
  if (live && sub == 0) pk[p] = R;
}

// Level 1, supernovae, histogram pass: one thread per particle counts it
// into the buckets of every tile its sphere touches (kBinChunkSn particles
// per block; skipped particles have n = 0).
template <int OWN>
__device__ __forceinline__ void l1_sn_hist(int blk, const Mesh& M, const TileGrid& T,
                                           const Particles& P, int shift, int nb,
                                           int* __restrict__ hist, int nblk,
                                           const SnPk* __restrict__ pk, NbrBox* s_nbr) {
  extern __shared__ int h[];
  const int col = hist_col(blk, nblk);
  for (int c = threadIdx.x; c < nb; c += blockDim.x) h[c] = 0;
  const long long p0 = (long long)blk * kBinChunkSn;
  const long long p1 = min(p0 + kBinChunkSn, P.n);
  int bb0, bb1;
  block_box_range(P.box_off, M.nbox, p0, p1, bb0, bb1);
  if constexpr (OWN == 1) stage_nbr(T, bb0, bb1, s_nbr);
  __syncthreads();
  for (long long p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    const SnPk& R = pk[p];
    const int N = R.n;
    if (N == 0) continue;
    const int b = (bb0 == bb1) ? bb0 : find_box_in(P.box_off, bb0, bb1, p);
    const DevBox B = M.boxes[b];
    sn_tiles<OWN>(M, T, b, B, R.x, R.y, R.z, R.r, N,
                  [&](int t) { atomicAdd(h + (t >> shift), 1); },
                  OWN == 1 ? nbr_of(T, s_nbr, bb0, b) : nullptr);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < nb; c += blockDim.x) hist[(long long)c * nblk + col] = h[c];
}

// Level 1, supernovae, scatter pass: one thread per particle writes its
// (particle, tile) entries at the positions the scanned histograms give.
template <int OWN>
__device__ __forceinline__ void l1_sn_scatter(int blk, const Mesh& M, const TileGrid& T,
                                              const Particles& P, int shift, int nb,
                                              int* __restrict__ hist, int nblk,
                                              const SnPk* __restrict__ pk, int* __restrict__ tmp,
                                              int* __restrict__ tmp_tile, long long cap,
                                              NbrBox* s_nbr) {
  extern __shared__ int h[];
  const int col = hist_col(blk, nblk);
  for (int c = threadIdx.x; c < nb; c += blockDim.x)
    h[c] = hist[(long long)c * nblk + col] - hist[0];
  const long long p0 = (long long)blk * kBinChunkSn;
  const long long p1 = min(p0 + kBinChunkSn, P.n);
  int bb0, bb1;
  block_box_range(P.box_off, M.nbox, p0, p1, bb0, bb1);
  if constexpr (OWN == 1) stage_nbr(T, bb0, bb1, s_nbr);
  __syncthreads();
  bool full = false;
  for (long long p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    const SnPk& R = pk[p];
    const int N = R.n;
    if (N == 0) continue;
    const int b = (bb0 == bb1) ? bb0 : find_box_in(P.box_off, bb0, bb1, p);
    const DevBox B = M.boxes[b];
    sn_tiles<OWN>(M, T, b, B, R.x, R.y, R.z, R.r, N, [&](int id) {
      const int pos = atomicAdd(h + (id >> shift), 1);
      if (pos < cap) {
        tmp[pos] = (int)p;
        tmp_tile[pos] = id;
      } else {
        full = true;
      }
    }, OWN == 1 ? nbr_of(T, s_nbr, bb0, b) : nullptr);
  }
  if (full) raise_flag(M.status, PMP_FLAG_CAPACITY);
}

// Level 1 for both kinds in one launch: blocks [0, nbc) take CIC chunks,
// the rest supernova chunks.
// (register budgets: the owner-tile variants' neighbour lookups would
// otherwise cost a wave per SIMD; the padded variants fit them already)
template <int OWN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) void k_l1_hist(Mesh M, TileGrid T, Particles C, Particles Sn,
                                                int shift, int nb, int* __restrict__ hc, int nbc,
                                                int* __restrict__ hs, int nbs,
                                                const SnPk* __restrict__ pk) {
  __shared__ NbrBox s_nbr[OWN == 1 ? 27 * kNbrCache : 1];
  if ((int)blockIdx.x < nbc)
    l1_cic<false, OWN>(blockIdx.x, M, T, C, shift, nb, hc, nbc, nullptr, nullptr, 0, s_nbr);
  else
    l1_sn_hist<OWN>(blockIdx.x - nbc, M, T, Sn, shift, nb, hs, nbs, pk, s_nbr);
}

template <int OWN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_l1_scatter(Mesh M, TileGrid T, Particles C,
                                                   Particles Sn, int shift, int nb,
                                                   int* __restrict__ hc, int nbc,
                                                   int* __restrict__ hs, int nbs,
                                                   double4* __restrict__ ctmp,
                                                   int* __restrict__ ctmp_tile, long long ccap,
                                                   const SnPk* __restrict__ pk,
                                                   int* __restrict__ stmp,
                                                   int* __restrict__ stmp_tile, long long scap) {
  __shared__ NbrBox s_nbr[OWN == 1 ? 27 * kNbrCache : 1];
  if ((int)blockIdx.x < nbc)
    l1_cic<true, OWN>(blockIdx.x, M, T, C, shift, nb, hc, nbc, ctmp, ctmp_tile, ccap, s_nbr);
  else
    l1_sn_scatter<OWN>(blockIdx.x - nbc, M, T, Sn, shift, nb, hs, nbs, pk, stmp, stmp_tile, scap,
                       s_nbr);
}

// Level 2: one workgroup per coarse bucket sorts the bucket's records by
// tile (LDS histogram, scan, cursors), writes the final records grouped by
// tile and the tile offsets off[tile] (off[ntiles] = total).
// Level 2 works on slices of at most kSlice records of one coarse bucket,
// for both kinds at once (buckets cc = kind * nb + c).  hist1 holds the
// scanned level-1 histograms: kind 0 (CIC, nblk0 blocks) then kind 1
// (supernovae, nblk1 blocks), then the grand total.
struct L2Geom {
  const int* hist1;
  int nb, nblk0, nblk1, shift;
  long long ntiles;
  long long cap0, cap1;  // entry capacity of each kind (level 1 drops entries past it)
};

__device__ __forceinline__ void bucket_range(const L2Geom& G, int cc, long long& start,
                                             long long& end) {
  const int kind = cc >= G.nb;
  const int c = cc - kind * G.nb;
  const int* H = kind ? G.hist1 + (long long)G.nb * G.nblk0 : G.hist1;
  const int nblk = kind ? G.nblk1 : G.nblk0;
  const long long base = H[0];
  // level 1 wrote only the entries below the capacity (and flagged the
  // rest): the bucket holds the part of its range below it, so the slices,
  // the level-2 histogram and the tile offsets never count dropped entries
  const long long cap = kind ? G.cap1 : G.cap0;
  start = min((long long)H[(long long)c * nblk] - base, cap);
  end = min((long long)H[(long long)(c + 1) * nblk] - base, cap);
}

// One block: slices per bucket, their exclusive prefix (slice_base), and the
// tile offsets of empty buckets and the kinds' totals.
__global__ __launch_bounds__(1024) void k_l2_plan(L2Geom G, int* __restrict__ slice_base,
                                                  int* __restrict__ off0,
                                                  int* __restrict__ off1,
                                                  int* __restrict__ heavy_count) {
  __shared__ int sh[kWave];
  __shared__ int carry;
  const int n = 2 * G.nb;
  if (threadIdx.x == 0) {
    carry = 0;
    *heavy_count = 0;  // chunk slots are claimed afresh after the sort
  }
  __syncthreads();
  for (int base_c = 0; base_c < n; base_c += blockDim.x) {
    const int cc = base_c + threadIdx.x;
    int ns = 0;
    if (cc < n) {
      long long start, end;
      bucket_range(G, cc, start, end);
      ns = (int)((end - start + kSlice - 1) / kSlice);
      const int kind = cc >= G.nb, c = cc - kind * G.nb;
      int* off = kind ? off1 : off0;
      if (ns == 0) {
        const long long t0 = (long long)c << G.shift;
        const int nf = (int)min((long long)1 << G.shift, G.ntiles - t0);
        for (int f = 0; f < nf; ++f) off[t0 + f] = (int)start;
      }
      if (c == G.nb - 1) off[G.ntiles] = (int)end;
    }
    const int inc = block_inclusive_scan(ns, sh);
    const int cv = carry;
    if (cc < n) slice_base[cc] = cv + inc - ns;
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) carry = cv + inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) slice_base[n] = carry;
}

__device__ __forceinline__ int find_slice(const int* slice_base, int n, int q) {
  int lo = 0, hi = n;  // largest cc with slice_base[cc] <= q
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (slice_base[mid] <= q) lo = mid; else hi = mid;
  }
  return lo;
}

// Per slice: LDS histogram of the slice's records over its bucket's tiles,
// written to hist2[2^shift * slice_base[cc] + f * ns + q] (bucket, tile,
// slice order), so that one exclusive scan of hist2 gives final positions.
__global__ __launch_bounds__(256) void k_l2_hist(L2Geom G, const int* __restrict__ slice_base,
                                                const int* __restrict__ tile0,
                                                const int* __restrict__ tile1, long long cap0,
                                                long long cap1, int* __restrict__ hist2) {
  extern __shared__ int h[];
  const int nf_max = 1 << G.shift;
  const int total = slice_base[2 * G.nb];
  for (int qg = blockIdx.x; qg < total; qg += gridDim.x) {
    const int cc = find_slice(slice_base, 2 * G.nb, qg);
    const int q = qg - slice_base[cc], ns = slice_base[cc + 1] - slice_base[cc];
    const int kind = cc >= G.nb, c = cc - kind * G.nb;
    long long start, end;
    bucket_range(G, cc, start, end);
    // records past the capacity were never written (flagged by level 1)
    const long long e0 = start + (long long)q * kSlice;
    const long long e1 = min(min(e0 + kSlice, end), kind ? cap1 : cap0);
    const int* tt = kind ? tile1 : tile0;
    const int t0 = c << G.shift;
    for (int f = threadIdx.x; f < nf_max; f += blockDim.x) h[f] = 0;
    __syncthreads();
    for (long long e = e0 + threadIdx.x; e < e1; e += blockDim.x) atomicAdd(h + (tt[e] - t0), 1);
    __syncthreads();
    const long long o = (long long)nf_max * slice_base[cc];
    for (int f = threadIdx.x; f < nf_max; f += blockDim.x) hist2[o + (long long)f * ns + q] = h[f];
    __syncthreads();
  }
}

// Per slice of one kind: LDS cursors from the scanned hist2 place every
// record at its final position, grouped by tile; slice 0 of a bucket writes
// the offsets of the bucket's tiles.
template <class Rec>
__device__ __forceinline__ void l2_scatter_slice(int qg, int kind, const L2Geom& G,
                                                 const int* __restrict__ slice_base,
                                                 const int* __restrict__ hist2,
                                                 const Rec* __restrict__ tmp,
                                                 const int* __restrict__ tmp_tile,
                                                 Rec* __restrict__ rec, int* __restrict__ off,
                                                 long long cap) {
  extern __shared__ int h[];
  const int nf_max = 1 << G.shift;
  // first position of this kind
  const long long kbase = hist2[(long long)nf_max * slice_base[kind * G.nb]];
  const int cc = find_slice(slice_base, 2 * G.nb, qg);
  const int q = qg - slice_base[cc], ns = slice_base[cc + 1] - slice_base[cc];
  const int c = cc - kind * G.nb;
  long long start, end;
  bucket_range(G, cc, start, end);
  const long long e0 = start + (long long)q * kSlice, e1 = min(min(e0 + kSlice, end), cap);
  const int t0 = c << G.shift;
  const int nf = (int)min((long long)nf_max, G.ntiles - t0);
  const long long o = (long long)nf_max * slice_base[cc];
  for (int f = threadIdx.x; f < nf_max; f += blockDim.x) {
    const int v = (int)(hist2[o + (long long)f * ns + q] - kbase);
    h[f] = v;
    if (q == 0 && f < nf) off[t0 + f] = v;
  }
  __syncthreads();
  // four entries per thread in flight: their tiles and records are loaded
  // together, then ranked and stored
  // (records as plain scalars: arrays of vector-type records would live in
  // scratch)
  constexpr int U = 4;
  constexpr bool QUAD = std::is_same<Rec, double4>::value;
  const long long stride = blockDim.x;
  for (long long e = e0 + threadIdx.x; e < e1; e += U * stride) {
    int tl[U] = {0, 0, 0, 0};
    double rx[U] = {0.0, 0.0, 0.0, 0.0}, ry[U] = {0.0, 0.0, 0.0, 0.0},
           rz[U] = {0.0, 0.0, 0.0, 0.0}, rw[U] = {0.0, 0.0, 0.0, 0.0};
    int ri[U] = {0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long eu = e + u * stride;
      if (eu < e1) {
        tl[u] = tmp_tile[eu];
        if constexpr (QUAD) {
          const double4 v = tmp[eu];
          rx[u] = v.x;
          ry[u] = v.y;
          rz[u] = v.z;
          rw[u] = v.w;
        } else {
          ri[u] = tmp[eu];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (e + u * stride < e1) {
        const int pos = atomicAdd(h + (tl[u] - t0), 1);
        if (pos < cap) {
          if constexpr (QUAD) rec[pos] = make_double4(rx[u], ry[u], rz[u], rw[u]);
          else rec[pos] = ri[u];
        }
      }
    }
  }
  __syncthreads();
}

// Per slice (both kinds in one launch): LDS cursors from the scanned hist2
// place every entry at its final position, grouped by tile; slice 0 of a
// bucket writes the offsets of the bucket's tiles.
__global__ __launch_bounds__(256) void k_l2_scatter(L2Geom G, const int* __restrict__ slice_base,
                                                   const int* __restrict__ hist2,
                                                   const double4* __restrict__ ctmp,
                                                   const int* __restrict__ ctmp_tile,
                                                   double4* __restrict__ crec,
                                                   int* __restrict__ coff, long long ccap,
                                                   const int* __restrict__ stmp,
                                                   const int* __restrict__ stmp_tile,
                                                   int* __restrict__ srec,
                                                   int* __restrict__ soff, long long scap) {
  const int split = slice_base[G.nb], total = slice_base[2 * G.nb];
  for (int qg = blockIdx.x; qg < total; qg += gridDim.x) {
    if (qg < split)
      l2_scatter_slice<double4>(qg, 0, G, slice_base, hist2, ctmp, ctmp_tile, crec, coff, ccap);
    else
      l2_scatter_slice<int>(qg, 1, G, slice_base, hist2, stmp, stmp_tile, srec, soff, scap);
  }
}

// Chunks a tile's entries are split into: at most cc CIC and cs supernova
// entries per chunk.
__device__ __forceinline__ int tile_chunks(long long nc, long long ns, int cc, int cs) {
  const long long a = (nc + cc - 1) / cc, b = (ns + cs - 1) / cs;
  return (int)max(1ll, max(a, b));
}

// Entry range [e0, e1) of tile t in a sorted list (entries past the
// capacity were never written: the fill flagged them).
__device__ __forceinline__ void tile_entries(const int* off, long long cap, long long t,
                                             long long& e0, long long& e1) {
  e0 = 0;
  e1 = 0;
  if (off) {
    e0 = min((long long)off[t], cap);
    e1 = min((long long)off[t + 1], cap);
  }
}

// One thread per tile: tiles with more entries than a chunk holds claim
// consecutive chunk slots (when slots remain) and list their chunks.
__global__ __launch_bounds__(256) void k_units(TileGrid T, const int* __restrict__ coff,
                                              long long ccap, const int* __restrict__ soff,
                                              long long scap, int cc, int cs,
                                              int* __restrict__ heavy_base,
                                              int2* __restrict__ heavy_unit,
                                              int* __restrict__ heavy_count,
                                              int* __restrict__ arrive, long long slot_cap) {
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < T.ntiles;
       t += (long long)gridDim.x * blockDim.x) {
    long long c0, c1, s0, s1;
    tile_entries(coff, ccap, t, c0, c1);
    tile_entries(soff, scap, t, s0, s1);
    const int chunks = tile_chunks(c1 - c0, s1 - s0, cc, cs);
    int base = -1;
    if (chunks > 1) {
      const int b0 = atomicAdd(heavy_count, chunks);
      if ((long long)b0 + chunks <= slot_cap) {
        base = b0;
        for (int j = 0; j < chunks; ++j) heavy_unit[b0 + j] = make_int2((int)t, j);
        arrive[b0] = 0;
      } else {
        // out of slots: the tile stays whole; mark the slots it claimed unused
        for (long long j = b0; j < min((long long)b0 + chunks, slot_cap); ++j)
          heavy_unit[j] = make_int2(-1, 0);
      }
    }
    heavy_base[t] = base;
  }
}

template <bool FIXED> struct LdsT;
template <> struct LdsT<true> { using T = unsigned long long; };
template <> struct LdsT<false> { using T = double; };

__device__ __forceinline__ void lds_add(unsigned long long* p, long long q) {
  atomicAdd(p, (unsigned long long)q);
}
__device__ __forceinline__ void lds_add(double* p, double v) { unsafeAtomicAdd(p, v); }

template <class T> __device__ __forceinline__ T from_lds(unsigned long long v);
// Reproducibility mode: the addition, then the bound of the element grows by
// eps |sum after it| (the LDS atomic returns the sum before).
__device__ __forceinline__ void lds_add_b(double* p, double* e, double v) {
  const double old = unsafeAtomicAdd(p, v);
  unsafeAtomicAdd(e, kEps * fabs(old + v));
}

template <> __device__ __forceinline__ long long from_lds<long long>(unsigned long long v) {
  return (long long)v;
}
template <class T> __device__ __forceinline__ T from_lds(double v) { return (T)v; }

// Owner tiles: cell index i of a particle's frame (-domain <= i < 2 domain)
// wrapped into [0, domain).
__device__ __forceinline__ int wrap_once(int i, int D) {
  return i < 0 ? i + D : (i >= D ? i - D : i);
}

// Owner tiles: the origin, in a particle's frame, of the periodic image of
// a tile [glo, glo + ext) that meets the particle's candidate cells [lo, hi]
// along axis a, and its code (1: + D, 2: - D) in bits 1 + 2a of `code`.
__device__ __forceinline__ int image_origin(int lo, int hi, int glo, int ext, int D, int a,
                                            int& code) {
  if (hi < glo) {
    code |= 2 << (1 + 2 * a);
    return glo - D;
  }
  if (lo >= glo + ext) {
    code |= 1 << (1 + 2 * a);
    return glo + D;
  }
  return glo;
}

__device__ __forceinline__ int image_shift(int code, int a, int glo, int D) {
  const int c = (code >> (1 + 2 * a)) & 3;
  return c == 1 ? glo + D : (c == 2 ? glo - D : glo);
}

// One workgroup per work unit (a whole tile, or one chunk of a split tile):
// CIC entries one per thread; supernovae in batches of up to one wavefront:
// one lane per entry gathers its particle's record, clips the sphere's
// candidate rows to the tile and adds the fixed-point remainder; then one
// thread per (entry, tile row) finds the row's member run with the exact row
// test and adds it.  Every addition goes to the LDS accumulators.  Then every present channel of every cell of the
// tile is stored once (channels without sources as zero).  Membership,
// shares and fixed-point remainders are the same as in the direct kernels.
// (7 waves per SIMD: the register budget that keeps the LDS-limited
// occupancy of the common tile shapes without spilling)
template <int ACC, int TYZ, bool OWN>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(7))) void k_tile_deposit(Mesh M, TileGrid T,
                                                      const int* __restrict__ coff,
                                                      const double4* __restrict__ crec,
                                                      long long ccap,
                                                      const int* __restrict__ soff,
                                                      const int* __restrict__ sidx,
                                                      const SnPk* __restrict__ pk,
                                                      long long scap, int cc, int cs,
                                                      const int* __restrict__ heavy_base,
                                                      const int2* __restrict__ heavy_unit,
                                                      const int* __restrict__ heavy_count,
                                                      int* __restrict__ arrive,
                                                      void* __restrict__ partial_v,
                                                      long long slot_cap,
                                                      typename AccT<ACC>::T* __restrict__ buf,
                                                      void* __restrict__ state, Limits L,
                                                      const int* __restrict__ sink_flag) {
  using OutT = typename AccT<ACC>::T;
  constexpr bool FIXED = (ACC == PMP_ACC_FIX64);
  constexpr bool BOUNDS = (ACC == PMP_ACC_F64R);  // error bounds beside the sums
  using LT = typename LdsT<FIXED>::T;
  constexpr int TY = TYZ, TZ = TYZ, S = TYZ * TYZ;
  ApplyCounts cnt;
  const int g = M.ghost;
  constexpr int YSH = (TYZ == 2) ? 1 : (TYZ == 4) ? 2 : 3;
  constexpr int SSH = 2 * YSH;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_last;
  LT* partial = reinterpret_cast<LT*>(partial_v);
  const int TX = T.wx;  // widest tile along x (LDS rows); a tile's own width is G.ext[0]
  const int tcells = TX * TY * TZ;
  const float inv_tx = 1.0f / (float)TX;
  // LDS rows of TX + 1 elements: the rows of one x column fall in different
  // banks, so lanes working on neighbouring rows do not conflict
  const int TXP = TX + 1;
  const int lcells = TXP * TY * TZ;
  LT* a0 = reinterpret_cast<LT*>(smem);
  LT* a4 = a0 + lcells;
  // reproducibility mode: the error bounds of a0 and a4
  double* eb0 = reinterpret_cast<double*>(a4 + lcells);
  double* eb4 = eb0 + lcells;
  // the current batch of the tile's supernovae
  constexpr int NB = kTileSnBatch;
  static_assert(NB <= kWave && sizeof(SnTile) % 16 == 0, "one batch entry per lane of a wave");
  SnTile* bent = reinterpret_cast<SnTile*>(BOUNDS ? reinterpret_cast<LT*>(eb4 + lcells)
                                                   : a4 + lcells);
  // work units: the chunks of split tiles first (the longest units), then
  // every other tile whole, in tile order
  const long long nheavy = min((long long)*heavy_count, slot_cap);
  for (long long unit = blockIdx.x; unit < T.ntiles + nheavy; unit += gridDim.x) {
    int tile;
    int chunk = 0, base = -1;
    if (unit < nheavy) {
      const int2 hu = heavy_unit[unit];
      if (hu.x < 0) continue;
      tile = hu.x;
      chunk = hu.y;
      base = heavy_base[tile];
    } else {
      tile = (int)(unit - nheavy);
    }
    // the tile's metadata, loaded together; a tile split into chunks is
    // done by its chunk units
    const int hb = heavy_base[tile];
    const TileGeo G = T.geo[tile];
    long long e0, e1, s0, s1;
    tile_entries(coff, ccap, tile, e0, e1);
    tile_entries(soff, scap, tile, s0, s1);
    if (unit >= nheavy && hb >= 0) continue;
    for (int c = threadIdx.x; c < lcells; c += blockDim.x) {
      a0[c] = (LT)0;
      a4[c] = (LT)0;
      if constexpr (BOUNDS) {
        eb0[c] = 0.0;
        eb4[c] = 0.0;
      }
    }
    int chunks = 1;
    if (base >= 0) {
      // this chunk's share of the tile's entries
      chunks = tile_chunks(e1 - e0, s1 - s0, cc, cs);
      const long long nc = e1 - e0, ns = s1 - s0;
      e1 = e0 + nc * (chunk + 1) / chunks;
      e0 = e0 + nc * chunk / chunks;
      s1 = s0 + ns * (chunk + 1) / chunks;
      s0 = s0 + ns * chunk / chunks;
    }
    __syncthreads();
    bool ovf = false;
    long long spos = s0;
    bool first = true;
    while (first || spos < s1) {
      // the batch's supernovae, one lane of the first wavefront each
      const int nq = (int)min((long long)NB, s1 - spos);
      if (threadIdx.x < kWave) {
        const int q = threadIdx.x;
        if (q < nq) {
          const SnPk& R = pk[sidx[spos + q]];
          Sphere Sp;
          sphere_init(Sp, R.x, R.y, R.z, R.r);
          SnTile E;
          E.x = R.x;
          E.y = R.y;
          E.z = R.z;
          E.r2 = Sp.r2;
          E.vr = R.vr;
          E.ve = R.ve;
          E.lo = Sp.lo[0];
          E.hi = Sp.hi[0];
          const bool host = R.n < 0;
          int lo1 = Sp.lo[1], hi1 = Sp.hi[1], lo2 = Sp.lo[2], hi2 = Sp.hi[2];
          if (host) {
            // the host cell alone
            E.lo = E.hi = (int)floor(R.x);
            lo1 = hi1 = (int)floor(R.y);
            lo2 = hi2 = (int)floor(R.z);
          } else if (R.n == 0) {
            hi1 = lo1 - 1;
          }
          // the tile's origin in the supernova's frame: with owner tiles, the
          // periodic image of the tile that the candidate box meets (one at
          // most), kept as two bits per axis beside the host bit
          int gl1 = G.glo[1], gl2 = G.glo[2];
          E.host = host;
          if constexpr (OWN) {
            const int gl0 = image_origin(E.lo, E.hi, G.glo[0], G.ext[0], M.domain[0], 0, E.host);
            gl1 = image_origin(lo1, hi1, G.glo[1], G.ext[1], M.domain[1], 1, E.host);
            gl2 = image_origin(lo2, hi2, G.glo[2], G.ext[2], M.domain[2], 2, E.host);
            (void)gl0;
          }
          // candidate rows inside the tile: v in [vlo, vhi], w in [wlo, whi]
          const int vlo = max(lo1 - gl1, 0), vhi = min(hi1 - gl1, G.ext[1] - 1);
          const int wlo = max(lo2 - gl2, 0), whi = min(hi2 - gl2, G.ext[2] - 1);
          E.rows = (vlo <= vhi && wlo <= whi)
                       ? (unsigned)(vlo | (vhi << 8) | (wlo << 16) | (whi << 24))
                       : 0x000000ffu;
          bent[q] = E;
          if constexpr (FIXED) {
            // the remainder, at its cell when the cell is in this tile
            const int* ro = OWN ? G.glo : G.o;
            const int lu = R.ti - ro[0], lv = R.tj - ro[1], lw = R.tk - ro[2];
            if (R.ti >= 0 && (unsigned)lu < (unsigned)G.ext[0] &&
                (unsigned)lv < (unsigned)G.ext[1] && (unsigned)lw < (unsigned)G.ext[2]) {
              const int tgt = (lw * TY + lv) * TXP + lu;
              lds_add(a0 + tgt, R.remr);
              lds_add(a4 + tgt, R.reme);
            }
          }
        }
      }
      if (first) {
        // CIC entries
        for (long long e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
          const double4 CR = crec[e];
          const int h[3] = {(int)floor(CR.x), (int)floor(CR.y), (int)floor(CR.z)};
          auto add = [&](int i, int j, int k, auto v) {
            if constexpr (OWN) {
              // owner tiles: the cell's periodic image
              i = wrap_once(i, M.domain[0]);
              j = wrap_once(j, M.domain[1]);
              k = wrap_once(k, M.domain[2]);
            }
            const int u = i - G.glo[0], vv = j - G.glo[1], w = k - G.glo[2];
            if ((unsigned)u < (unsigned)G.ext[0] && (unsigned)vv < (unsigned)G.ext[1] &&
                (unsigned)w < (unsigned)G.ext[2]) {
              const int lc = (w * TY + vv) * TXP + u;
              if constexpr (BOUNDS) lds_add_b(a0 + lc, eb0 + lc, v);
              else lds_add(a0 + lc, v);
            }
          };
          if (!cic_one<FIXED>(CR.x, CR.y, CR.z, CR.w, M.V, h, add)) ovf = true;
        }
        first = false;
      }
      __syncthreads();
      // supernova rows: the member run of tile row (v, w), clipped to the tile
      for (int it = threadIdx.x; it < (nq << SSH); it += blockDim.x) {
        const SnTile& E = bent[it >> SSH];
        const int sl = it & (S - 1);
        const int v = sl & (TY - 1), w = sl >> YSH;
        const unsigned rr = E.rows;
        int a = 1, b = 0;
        int gl0 = G.glo[0], gl1 = G.glo[1], gl2 = G.glo[2];
        if constexpr (OWN) {
          gl0 = image_shift(E.host, 0, gl0, M.domain[0]);
          gl1 = image_shift(E.host, 1, gl1, M.domain[1]);
          gl2 = image_shift(E.host, 2, gl2, M.domain[2]);
        }
        if (v < (int)(rr & 255u) || v > (int)((rr >> 8) & 255u) || w < (int)((rr >> 16) & 255u) ||
            w > (int)(rr >> 24)) {
          // not a candidate row (an empty range is stored as vlo = 255 > vhi)
        } else if (E.host & 1) {
          a = b = E.lo;
        } else {
          // rows whose rounded dy^2 + dz^2 exceeds r^2 hold no member
          const double dy = ((double)(gl1 + v) + 0.5) - E.y;
          const double dz = ((double)(gl2 + w) + 0.5) - E.z;
          const double y2 = dy * dy, z2 = dz * dz;
          if (y2 + z2 <= E.r2) row_run(E.x, E.r2, E.lo, E.hi, y2, z2, a, b);
        }
        const int ua = max(a - gl0, 0), ub = min(b - gl0, G.ext[0] - 1);
        LT* r0 = a0 + (w * TY + v) * TXP;
        LT* r4 = a4 + (w * TY + v) * TXP;
        if constexpr (FIXED) {
          const long long qr = __double_as_longlong(E.vr), qe = __double_as_longlong(E.ve);
          for (int u = ua; u <= ub; ++u) {
            lds_add(r0 + u, qr);
            lds_add(r4 + u, qe);
          }
        } else if constexpr (BOUNDS) {
          const double cr = E.vr, ce = E.ve;
          double* q0 = eb0 + (w * TY + v) * TXP;
          double* q4 = eb4 + (w * TY + v) * TXP;
          for (int u = ua; u <= ub; ++u) {
            lds_add_b(r0 + u, q0 + u, cr);
            lds_add_b(r4 + u, q4 + u, ce);
          }
        } else {
          const double cr = E.vr, ce = E.ve;
          for (int u = ua; u <= ub; ++u) {
            lds_add(r0 + u, cr);
            lds_add(r4 + u, ce);
          }
        }
      }
      spos += nq;
      __syncthreads();
    }
    if (ovf) raise_flag(M.status, PMP_FLAG_OVERFLOW);
    __syncthreads();
    if (base >= 0) {
      // a chunk of a split tile: leave the partial tile, and the last chunk
      // to finish (device-scope fence + arrival count) sums the chunks'
      // partial tiles in chunk order back into the accumulators
      LT* part = partial + (long long)(base + chunk) * 2 * lcells;
      for (int c = threadIdx.x; c < lcells; c += blockDim.x) {
        part[c] = a0[c];
        part[lcells + c] = a4[c];
      }
      __threadfence();
      __syncthreads();
      if (threadIdx.x == 0) s_last = (atomicAdd(arrive + base, 1) == chunks - 1);
      __syncthreads();
      if (!s_last) continue;
      __threadfence();
      const LT* p0 = partial + (long long)base * 2 * lcells;
      for (int c = threadIdx.x; c < lcells; c += blockDim.x) {
        LT r0 = p0[c], r4 = p0[lcells + c];
        for (int q = 1; q < chunks; ++q) {
          r0 += p0[2ll * q * lcells + c];
          r4 += p0[2ll * q * lcells + lcells + c];
        }
        a0[c] = r0;
        a4[c] = r4;
      }
      __syncthreads();
    }
    // every present channel of every cell is stored once: rho and E from
    // the accumulators, the others (no source in this pass) as zero.  In a
    // fused step, owned cells at least g from every face are applied here
    // instead (their buffer value, rounded to the buffer type, is final: no
    // ghost image reaches them)
    OutT* f0 = buf + G.boff;
    const long long np = (long long)G.p[0] * G.p[1] * G.p[2];
    // owner tiles a sink kernel may reach keep their cells for the sink
    // passes: stored, applied after the sink update
    const bool apply_here = state && !(OWN && sink_flag && sink_flag[tile]);
    const int n0 = G.p[0] - 2 * g, n1 = G.p[1] - 2 * g, n2 = G.p[2] - 2 * g;
    const long long ncell = (long long)n0 * n1 * n2;
    const int sr = M.slot[0], se = M.slot[4];
    // owned-local origin of the tile and its state offset; a cell's offset
    // from it fits 32 bits (at most TZ planes of the box)
    const int ox0 = G.o[0] - g, oy0 = G.o[1] - g, oz0 = G.o[2] - g;
    const long long tso = G.soff + ((long long)oz0 * n1 + oy0) * n0 + ox0;
    const long long tbo = ((long long)G.o[2] * G.p[1] + G.o[1]) * G.p[0] + G.o[0];
    // cell c = u + TX row of the LDS tile, advanced by blockDim per step
    const int drow = small_div((int)blockDim.x, TX, inv_tx), du = (int)blockDim.x - drow * TX;
    int row = small_div((int)threadIdx.x, TX, inv_tx);
    int u = (int)threadIdx.x - row * TX;
    for (int c = threadIdx.x; c < tcells; c += blockDim.x) {
      const int v = row & (TY - 1), w = row >> YSH;
      if (u < G.ext[0] && v < G.ext[1] && w < G.ext[2]) {
        const int lc = (w * TY + v) * TXP + u;
        LT r0 = a0[lc], r4 = a4[lc];
        if constexpr (BOUNDS) {
          // the tile holds every contribution to its cells: the sums are complete
          r0 = truncate_bound(r0, eb0[lc], M.margin);
          r4 = truncate_bound(r4, eb4[lc], M.margin);
        }
        const OutT vr = sr >= 0 ? from_lds<OutT>(r0) : (OutT)0;
        const OutT ve = se >= 0 ? from_lds<OutT>(r4) : (OutT)0;
        // owned-local coordinates: interior when g <= . < n - g on every axis
        // (with owner tiles every cell is owned and its sum complete: applied,
        // or, in a step with sinks, stored for the sink passes and the apply)
        const int ox = ox0 + u, oy = oy0 + v, oz = oz0 + w;
        if (apply_here && (OWN || (ox >= g && ox < n0 - g && oy >= g && oy < n1 - g &&
                                   oz >= g && oz < n2 - g))) {
          const long long si = tso + ((w * n1 + v) * n0 + u);
          if (M.state == PMP_STATE_F32)
            apply_cell_nosrc((float*)state + si, ncell, to_f64(vr), to_f64(ve), L, cnt);
          else
            apply_cell_nosrc((double*)state + si, ncell, to_f64(vr), to_f64(ve), L, cnt);
        } else {
          const long long idx = tbo + ((w * G.p[1] + v) * G.p[0] + u);
          for (int f = 0; f < M.nfield; ++f) {
            OutT val = (OutT)0;
            if (f == sr) val = vr;
            else if (f == se) val = ve;
            f0[idx + f * np] = val;
          }
        }
      }
      u += du;
      row += drow;
      if (u >= TX) {
        u -= TX;
        ++row;
      }
    }
    __syncthreads();
  }
  if (state) flush_counts(M, cnt);
}

// Owner tiles in a step with sinks: every owner tile a sink's kernel may
// reach is flagged (the kernel's cells lie within floor(r_K) + 1 cells of the
// host cell; the cube is widened by one more, and a flag too many only moves
// a tile's apply after the sink update).  Sinks outside their box are left
// to the deposit kernel, which flags them.  kSinkPlaneLanes threads per
// sink, each taking every kSinkPlaneLanes-th z plane of the sink's cube (the
// planes' tiles together are the cube's), so that sinks whose cube meets
// several boxes are not walked by one thread each.
constexpr int kSinkPlaneLanes = 16;
__global__ __launch_bounds__(256) void k_sink_tiles(Mesh M, TileGrid T, Particles P, int reach,
                                                   int* __restrict__ flag) {
  const int g = M.ghost;
  const int side = 2 * reach + 3;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < P.n * kSinkPlaneLanes;
       q += (long long)gridDim.x * blockDim.x) {
    const long long s = q / kSinkPlaneLanes;
    const int lane = (int)(q % kSinkPlaneLanes);
    const int b = particle_box(P.box_off, M.nbox, s);
    const DevBox B = M.boxes[b];
    int h[3];
    if (!host_cell(B, P.x[s], P.y[s], P.z[s], h)) continue;
    int lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      lo[a] = h[a] - reach - 1 - B.lo[a] + g;
      hi[a] = h[a] + reach + 1 - B.lo[a] + g;
    }
    for (int dz = lane; dz < side; dz += kSinkPlaneLanes) {
      lo[2] = hi[2] = h[2] - reach - 1 + dz - B.lo[2] + g;
      particle_tiles<1>(M, T, b, B, lo, hi, [&](int t) { flag[t] = 1; });
    }
  }
}

// Steps 3 + 5 for the cells of the flagged owner tiles, after the sink
// update: one workgroup per tile (unflagged tiles return at once), each
// cell's buffer channels read from its owned place, the limiter and the
// update as in k_apply.
template <class S, int ACC>
__global__ __launch_bounds__(256) void k_apply_tiles(Mesh M, TileGrid T, S* __restrict__ state,
                                                     const typename AccT<ACC>::T* __restrict__ buf,
                                                     const int* __restrict__ flag, Limits L) {
  const int g = M.ghost;
  ApplyCounts cnt;
  const int s0 = M.slot[0], s1 = M.slot[1], s2 = M.slot[2], s3 = M.slot[3], s4 = M.slot[4],
            s5 = M.slot[5];
  for (long long t = blockIdx.x; t < T.ntiles; t += gridDim.x) {
    if (!flag[t]) continue;
    const TileGeo G = T.geo[t];
    const int n0 = G.p[0] - 2 * g, n1 = G.p[1] - 2 * g, n2 = G.p[2] - 2 * g;
    const long long ncell = (long long)n0 * n1 * n2;
    const long long np = (long long)G.p[0] * G.p[1] * G.p[2];
    const int e0 = G.ext[0], e01 = G.ext[0] * G.ext[1], total = e01 * G.ext[2];
    for (int c = threadIdx.x; c < total; c += blockDim.x) {
      int u, v, w;
      cube_cell(c, e0, e01, u, v, w);
      // owned-local cell, its padded buffer index and its state index
      const int ox = G.o[0] - g + u, oy = G.o[1] - g + v, oz = G.o[2] - g + w;
      const long long bi = G.boff + ((long long)(oz + g) * G.p[1] + (oy + g)) * G.p[0] + (ox + g);
      const long long si = G.soff + ((long long)oz * n1 + oy) * n0 + ox;
      const double Dr = s0 >= 0 ? to_f64(buf[bi + s0 * np]) : 0.0;
      const double qx = s1 >= 0 ? to_f64(buf[bi + s1 * np]) : 0.0;
      const double qy = s2 >= 0 ? to_f64(buf[bi + s2 * np]) : 0.0;
      const double qz = s3 >= 0 ? to_f64(buf[bi + s3 * np]) : 0.0;
      const double DE = s4 >= 0 ? to_f64(buf[bi + s4 * np]) : 0.0;
      const double K = s5 >= 0 ? to_f64(buf[bi + s5 * np]) : 0.0;
      (void)apply_cell(state + si, ncell, Dr, qx, qy, qz, DE, K, L, cnt);
    }
  }
  flush_counts(M, cnt);
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

hipError_t launch_copy4(void* dst, const void* src, long long bytes, hipStream_t s) {
  const long long ngroups = bytes / 16384;
  const int grid = grid_for(ngroups, 1, 256 * 16);
  hipLaunchKernelGGL(k_copy4, dim3(grid), dim3(256), 0, s, (u32x4*)dst, (const u32x4*)src,
                     ngroups);
  return hipGetLastError();
}

hipError_t launch_atomic_bench(void* dst, long long slots, int type, int pattern,
                               long long n_ops, hipStream_t s) {
  const int grid = grid_for(n_ops, 256, 256 * 64);
  const unsigned long long mask = (unsigned long long)slots - 1ull;
  if (type == 0)
    hipLaunchKernelGGL(k_atomic_bench<unsigned long long>, dim3(grid), dim3(256), 0, s,
                       (unsigned long long*)dst, mask, pattern, n_ops);
  else if (type == 1)
    hipLaunchKernelGGL(k_atomic_bench<float>, dim3(grid), dim3(256), 0, s, (float*)dst, mask,
                       pattern, n_ops);
  else
    hipLaunchKernelGGL(k_atomic_bench<double>, dim3(grid), dim3(256), 0, s, (double*)dst, mask,
                       pattern, n_ops);
  return hipGetLastError();
}

hipError_t launch_clear_status(DevStatus* st, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_cic_direct(const Mesh& M, const Particles& P, void* buf, int block,
                             hipStream_t s) {
  if (P.n <= 0) return hipSuccess;
  const int grid = grid_for(P.n, block, M.num_cu * 32);
  switch (M.acc) {
    case PMP_ACC_F32:
      hipLaunchKernelGGL(k_cic_direct<PMP_ACC_F32>, dim3(grid), dim3(block), 0, s, M, P,
                         (float*)buf);
      break;
    case PMP_ACC_F64R:
    case PMP_ACC_F64:
      hipLaunchKernelGGL(k_cic_direct<PMP_ACC_F64>, dim3(grid), dim3(block), 0, s, M, P,
                         (double*)buf);
      break;
    default:
      hipLaunchKernelGGL(k_cic_direct<PMP_ACC_FIX64>, dim3(grid), dim3(block), 0, s, M, P,
                         (long long*)buf);
  }
  return hipGetLastError();
}


hipError_t launch_bin(const Mesh& M, const TileGrid& T, const Particles* cic,
                      const Particles* sn, BinWork& bw, int count_lanes, hipStream_t s) {
  const int nb = bw.nbuckets, S = bw.shift;
  const bool has_c = cic && cic->n > 0, has_s = sn && sn->n > 0;
  const int nbc = has_c ? (int)((cic->n + kBinChunkCic - 1) / kBinChunkCic) : 0;
  const int nbs = has_s ? (int)((sn->n + kBinChunkSn - 1) / kBinChunkSn) : 0;
  int* hc = bw.hist;
  int* hs = bw.hist + (long long)nb * nbc;
  const long long n = (long long)nb * (nbc + nbs);
  const size_t lds1 = (size_t)nb * sizeof(int);
  if (has_s) {
    const unsigned grid = (unsigned)((sn->n * count_lanes + 255) / 256);
    switch (count_lanes) {
      case 1: hipLaunchKernelGGL(k_sn_count<1>, dim3(grid), dim3(256), 0, s, M, *sn, bw.sn_pk, T.owner); break;
      case 2: hipLaunchKernelGGL(k_sn_count<2>, dim3(grid), dim3(256), 0, s, M, *sn, bw.sn_pk, T.owner); break;
      case 8: hipLaunchKernelGGL(k_sn_count<8>, dim3(grid), dim3(256), 0, s, M, *sn, bw.sn_pk, T.owner); break;
      case 16: hipLaunchKernelGGL(k_sn_count<16>, dim3(grid), dim3(256), 0, s, M, *sn, bw.sn_pk, T.owner); break;
      default: hipLaunchKernelGGL(k_sn_count<4>, dim3(grid), dim3(256), 0, s, M, *sn, bw.sn_pk, T.owner);
    }
  }
  if (has_c || has_s) {
#define PMP_L1H(OWN)                                                                        \
  hipLaunchKernelGGL(k_l1_hist<OWN>, dim3(nbc + nbs), dim3(256), lds1, s, M, T,               \
                     has_c ? *cic : Particles{}, has_s ? *sn : Particles{}, S, nb, hc, nbc, hs, \
                     nbs, (const SnPk*)bw.sn_pk)
    if (!T.owner) PMP_L1H(0);
    else if (M.own_start == nullptr) PMP_L1H(2);  // one box covers the domain
    else PMP_L1H(1);
#undef PMP_L1H
  }
  // exclusive scan of both kinds' histograms, in place; hist[n] = total
  const int nblocks = (int)((n + kScanBlock - 1) / kScanBlock);
  hipLaunchKernelGGL(k_scan_local, dim3(nblocks), dim3(kScanBlock), 0, s, bw.hist, bw.hist,
                     bw.block_sums, n, (const int*)nullptr, 0);
  hipLaunchKernelGGL(k_scan_finish, dim3(nblocks), dim3(kScanBlock), 0, s, bw.hist,
                     (const int*)bw.block_sums, n, (const int*)nullptr, 0);
  if (has_c || has_s) {
#define PMP_L1S(OWN)                                                                        \
  hipLaunchKernelGGL(k_l1_scatter<OWN>, dim3(nbc + nbs), dim3(256), lds1, s, M, T,            \
                     has_c ? *cic : Particles{}, has_s ? *sn : Particles{}, S, nb, hc, nbc, hs, \
                     nbs, bw.cic_tmp, bw.cic_tmp_tile, bw.cic_cap, (const SnPk*)bw.sn_pk,       \
                     bw.sn_tmp, bw.sn_tmp_tile, bw.sn_cap)
    if (!T.owner) PMP_L1S(0);
    else if (M.own_start == nullptr) PMP_L1S(2);
    else PMP_L1S(1);
#undef PMP_L1S
  }
  // level 2: balanced slices of every bucket, both kinds
  L2Geom G;
  G.hist1 = bw.hist;
  G.nb = nb;
  G.nblk0 = nbc;
  G.nblk1 = nbs;
  G.shift = S;
  G.ntiles = T.ntiles;
  G.cap0 = bw.cic_cap;
  G.cap1 = bw.sn_cap;
  hipLaunchKernelGGL(k_l2_plan, dim3(1), dim3(1024), 0, s, G, bw.slice_base, bw.cic_off,
                     bw.sn_off, bw.heavy_count);
  // hist2 is written in full for the slices in use ((slices in use) << S
  // entries, known on the device), and only that much is scanned
  const long long n2 = ((long long)1 << S) * bw.max_slices;
  const int* used = bw.slice_base + 2 * nb;
  const size_t lds2 = ((size_t)1 << S) * sizeof(int);
  const int grid2 = (int)std::min<long long>(bw.max_slices, (long long)M.num_cu * 8);
  hipLaunchKernelGGL(k_l2_hist, dim3(grid2), dim3(256), lds2, s, G, (const int*)bw.slice_base,
                     (const int*)bw.cic_tmp_tile, (const int*)bw.sn_tmp_tile, bw.cic_cap,
                     bw.sn_cap, bw.hist2);
  const int nblocks2 = (int)((n2 + kScanBlock - 1) / kScanBlock);
  hipLaunchKernelGGL(k_scan_local, dim3(nblocks2), dim3(kScanBlock), 0, s, bw.hist2, bw.hist2,
                     bw.block_sums2, n2, used, S);
  hipLaunchKernelGGL(k_scan_finish, dim3(nblocks2), dim3(kScanBlock), 0, s, bw.hist2,
                     (const int*)bw.block_sums2, n2, used, S);
  hipLaunchKernelGGL(k_l2_scatter, dim3(grid2), dim3(256), lds2, s, G, (const int*)bw.slice_base,
                     (const int*)bw.hist2, (const double4*)bw.cic_tmp,
                     (const int*)bw.cic_tmp_tile, bw.cic_rec, bw.cic_off, bw.cic_cap,
                     (const int*)bw.sn_tmp, (const int*)bw.sn_tmp_tile, bw.sn_rec, bw.sn_off,
                     bw.sn_cap);
  return hipGetLastError();
}

hipError_t launch_tile_prep(const Mesh& M, const TileGrid& T, const Particles* cic,
                            const Particles* sn, const BinWork& bw, const pmp_tuning& t,
                            hipStream_t s) {
  const int* coff = (cic && cic->n > 0) ? bw.cic_off : nullptr;
  const int* soff = (sn && sn->n > 0) ? bw.sn_off : nullptr;
  hipLaunchKernelGGL(k_units, dim3(grid_for(T.ntiles, 256, M.num_cu * 16)), dim3(256), 0, s, T,
                     coff, bw.cic_cap, soff, bw.sn_cap,
                     // the reproducibility mode never splits a tile: each tile
                     // sums all of its cells' contributions (and their bounds)
                     M.acc == PMP_ACC_F64R ? 0x7fffffff : t.chunk_cic,
                     M.acc == PMP_ACC_F64R ? 0x7fffffff : t.chunk_sn, bw.heavy_base,
                     bw.heavy_unit, bw.heavy_count, bw.arrive, bw.slot_cap);
  return hipGetLastError();
}

hipError_t launch_sink_tiles(const Mesh& M, const TileGrid& T, const Particles& sinks, double r_k,
                             int* flag, hipStream_t s) {
  // clear with a kernel (the step may be captured into a graph)
  hipError_t e = launch_zero(flag, T.ntiles * (long long)sizeof(int), 256, s);
  if (e != hipSuccess || sinks.n <= 0) return e;
  const int reach = (int)floor(r_k) + 1;
  hipLaunchKernelGGL(k_sink_tiles, dim3(grid_for(sinks.n * kSinkPlaneLanes, 256, M.num_cu * 16)),
                     dim3(256), 0, s, M, T, sinks, reach, flag);
  return hipGetLastError();
}

hipError_t launch_apply_tiles(const Mesh& M, const TileGrid& T, void* state, const void* buf,
                              const int* flag, const Limits& L, hipStream_t s) {
  const int grid = grid_for(T.ntiles, 1, M.num_cu * 32);
#define PMP_AT(S, ACC, TT)                                                                    \
  hipLaunchKernelGGL((k_apply_tiles<S, ACC>), dim3(grid), dim3(256), 0, s, M, T, (S*)state,   \
                     (const TT*)buf, flag, L)
  const bool f32 = M.state == PMP_STATE_F32;
  switch (M.acc) {
    case PMP_ACC_F32:
      if (f32) PMP_AT(float, PMP_ACC_F32, float); else PMP_AT(double, PMP_ACC_F32, float);
      break;
    case PMP_ACC_F64:
      if (f32) PMP_AT(float, PMP_ACC_F64, double); else PMP_AT(double, PMP_ACC_F64, double);
      break;
    default:
      if (f32) PMP_AT(float, PMP_ACC_FIX64, long long);
      else PMP_AT(double, PMP_ACC_FIX64, long long);
  }
#undef PMP_AT
  return hipGetLastError();
}

hipError_t launch_tile_deposit(const Mesh& M, const TileGrid& T, const Particles* cic,
                               const Particles* sn, const BinWork& bw, void* buf,
                               const pmp_tuning& t, void* state, const Limits& L,
                               hipStream_t s, const int* sink_flag) {
  const int* coff = (cic && cic->n > 0) ? bw.cic_off : nullptr;
  const int* soff = (sn && sn->n > 0) ? bw.sn_off : nullptr;
  const int block = t.tile_block;
  const size_t lds = (size_t)tile_lds_bytes_wx(T.wx, T.t[1], M.acc == PMP_ACC_F64R);
  long long grid = T.ntiles;
  if (t.tile_grid_per_cu > 0)
    grid = std::min<long long>(grid, (long long)M.num_cu * t.tile_grid_per_cu);
  if (grid < 1) grid = 1;
  if (grid > 0x7fffffffll) grid = 0x7fffffffll;
#define PMP_TILE(ACC, TT, TYZ, OWN)                                                           \
  hipLaunchKernelGGL((k_tile_deposit<ACC, TYZ, OWN>), dim3((unsigned)grid), dim3(block), lds, \
                     s, M, T, coff, (const double4*)bw.cic_rec, bw.cic_cap, soff,             \
                     (const int*)bw.sn_rec, (const SnPk*)bw.sn_pk, bw.sn_cap, t.chunk_cic,    \
                     t.chunk_sn,                                                              \
                     (const int*)bw.heavy_base, (const int2*)bw.heavy_unit,                   \
                     (const int*)bw.heavy_count, bw.arrive, bw.partial, bw.slot_cap,          \
                     (TT*)buf, state, L, sink_flag)
  // owner tiles: no reproducibility-mode variant (its bounds need the fold's order)
#define PMP_TILE_ACC(TYZ)                                                       \
  if (T.owner) {                                                                \
    switch (M.acc) {                                                            \
      case PMP_ACC_F32: PMP_TILE(PMP_ACC_F32, float, TYZ, true); break;         \
      case PMP_ACC_F64: PMP_TILE(PMP_ACC_F64, double, TYZ, true); break;        \
      default: PMP_TILE(PMP_ACC_FIX64, long long, TYZ, true);                   \
    }                                                                           \
  } else {                                                                      \
    switch (M.acc) {                                                            \
      case PMP_ACC_F32: PMP_TILE(PMP_ACC_F32, float, TYZ, false); break;        \
      case PMP_ACC_F64: PMP_TILE(PMP_ACC_F64, double, TYZ, false); break;       \
      case PMP_ACC_F64R: PMP_TILE(PMP_ACC_F64R, double, TYZ, false); break;     \
      default: PMP_TILE(PMP_ACC_FIX64, long long, TYZ, false);                  \
    }                                                                           \
  }
  switch (T.t[1]) {
    case 2: PMP_TILE_ACC(2); break;
    case 4: PMP_TILE_ACC(4); break;
    default: PMP_TILE_ACC(8);
  }
#undef PMP_TILE_ACC
#undef PMP_TILE
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
    case PMP_ACC_F64R:  // double buffer; its deposits are checked for the binned path
    case PMP_ACC_F64: sn_launch_lanes<PMP_ACC_F64>(M, P, buf, lanes, s); break;
    default: sn_launch_lanes<PMP_ACC_FIX64>(M, P, buf, lanes, s);
  }
  return hipGetLastError();
}

template <int ACC, class S>
static void sink_dep(const Mesh& M, const Particles& P, const void* state, void* buf,
                     double* scratch, const SinkParams& K, const Limits& L, double* bound,
                     hipStream_t s) {
  const int grid = grid_for(P.n, 1, 65536);
  hipLaunchKernelGGL((k_sink_deposit<ACC, S>), dim3(grid), dim3(kSinkBlock), 0, s, M, P,
                     (const S*)state, (typename AccT<ACC>::T*)buf, scratch, K, L, bound);
}

hipError_t launch_sink_deposit(const Mesh& M, const Particles& P, const void* state,
                               void* buf, double* scratch, const SinkParams& K,
                               const Limits& L, double* bound, hipStream_t s) {
  if (P.n <= 0) return hipSuccess;
  const bool f32 = (M.state == PMP_STATE_F32);
  const Limits& tr = L;
  switch (M.acc) {
    case PMP_ACC_F32:
      f32 ? sink_dep<PMP_ACC_F32, float>(M, P, state, buf, scratch, K, tr, nullptr, s)
          : sink_dep<PMP_ACC_F32, double>(M, P, state, buf, scratch, K, tr, nullptr, s);
      break;
    case PMP_ACC_F64:
      f32 ? sink_dep<PMP_ACC_F64, float>(M, P, state, buf, scratch, K, tr, nullptr, s)
          : sink_dep<PMP_ACC_F64, double>(M, P, state, buf, scratch, K, tr, nullptr, s);
      break;
    case PMP_ACC_F64R: {
      // bounds of every buffer element zeroed, the removal channel summed with
      // its bounds, then the elements it reached truncated
      hipError_t e = launch_zero(bound, M.buffer_elems * 8, 256, s);
      if (e != hipSuccess) return e;
      f32 ? sink_dep<PMP_ACC_F64R, float>(M, P, state, buf, scratch, K, tr, bound, s)
          : sink_dep<PMP_ACC_F64R, double>(M, P, state, buf, scratch, K, tr, bound, s);
      const int grid = grid_for(M.buffer_elems, 256, M.num_cu * 16);
      hipLaunchKernelGGL(k_truncate_bounds, dim3(grid), dim3(256), 0, s, (double*)buf,
                         (const double*)bound, M.buffer_elems, M.margin);
      break;
    }
    default:
      f32 ? sink_dep<PMP_ACC_FIX64, float>(M, P, state, buf, scratch, K, tr, nullptr, s)
          : sink_dep<PMP_ACC_FIX64, double>(M, P, state, buf, scratch, K, tr, nullptr, s);
  }
  return hipGetLastError();
}

template <int ACC, class S>
static void snr_dep(const Mesh& M, const SnrArgs& A, const void* state, void* buf, double* info,
                    hipStream_t s) {
  const int grid = grid_for(A.n, 1, 65536);
  hipLaunchKernelGGL((k_snr_deposit<ACC, S>), dim3(grid), dim3(kSinkBlock), 0, s, M, A,
                     (const S*)state, (typename AccT<ACC>::T*)buf, info);
}

hipError_t launch_snr_deposit(const Mesh& M, const SnrArgs& A, const void* state, void* buf,
                              double* info, hipStream_t s) {
  if (A.n <= 0) return hipSuccess;
  const bool f32 = (M.state == PMP_STATE_F32);
#define PMP_SNR(ACC)                                                               \
  (f32 ? snr_dep<ACC, float>(M, A, state, buf, info, s)                            \
       : snr_dep<ACC, double>(M, A, state, buf, info, s))
  switch (M.acc) {
    case PMP_ACC_F32: PMP_SNR(PMP_ACC_F32); break;
    case PMP_ACC_F64: PMP_SNR(PMP_ACC_F64); break;
    default: PMP_SNR(PMP_ACC_FIX64);
  }
#undef PMP_SNR
  return hipGetLastError();
}

template <int ACC, class S>
static void sink_upd(const Mesh& M, const Particles& P, const void* state, const void* buf,
                     const double* scratch, double r_k, const Limits& L, double* dm,
                     double* dpx, double* dpy, double* dpz, hipStream_t s) {
  const int grid = grid_for(P.n, 1, 65536);
  hipLaunchKernelGGL((k_sink_update<ACC, S>), dim3(grid), dim3(kSinkBlock), 0, s, M, P,
                     (const S*)state, (const typename AccT<ACC>::T*)buf, scratch, r_k, L, dm,
                     dpx, dpy, dpz);
}

hipError_t launch_sink_update(const Mesh& M, const Particles& P, const void* state,
                              const void* buf, const double* scratch, const SinkParams& K,
                              const Limits& L, double* dm, double* dpx, double* dpy,
                              double* dpz, hipStream_t s) {
  if (P.n <= 0) return hipSuccess;
  const bool f32 = (M.state == PMP_STATE_F32);
  const double r_k = K.r_k;
#define PMP_SU(ACC)                                                                            \
  (f32 ? sink_upd<ACC, float>(M, P, state, buf, scratch, r_k, L, dm, dpx, dpy, dpz, s)         \
       : sink_upd<ACC, double>(M, P, state, buf, scratch, r_k, L, dm, dpx, dpy, dpz, s))
  switch (M.acc) {
    case PMP_ACC_F32: PMP_SU(PMP_ACC_F32); break;
    case PMP_ACC_F64R:  // double buffer; its deposits are checked for the binned path
    case PMP_ACC_F64: PMP_SU(PMP_ACC_F64); break;
    default: PMP_SU(PMP_ACC_FIX64);
  }
#undef PMP_SU
  return hipGetLastError();
}

// ------------------------------------------------------------ sink creation

// Squared distance along one axis from p to the centre of cell i or of its
// periodic images one domain length n away, the smallest of the three (each
// as the distance test of dist2 computes it).  The sum of the three axes'
// smallest terms is the smallest dist2 over the 27 images, since rounded
// sums and squares are monotone.
__device__ __forceinline__ double image_term(int i, int n, double p) {
  const double a = ((double)i + 0.5) - p;
  const double b = ((double)(i - n) + 0.5) - p;
  const double c = ((double)(i + n) + 0.5) - p;
  double m = a * a;
  if (b * b < m) m = b * b;
  if (c * c < m) m = c * c;
  return m;
}

// Sink creation (Sec. 3.1.2), pass 1.  The blocks walk the apply chunks
// (256 owned cells of one box); each wavefront takes 64 of them.  A cell is a
// candidate when rho > rho_Tr (its Truelove density) and the folded removal
// channel K of its box is zero there.  The whole wavefront then tests each
// candidate in turn: first the existing sinks (lanes over the sinks, any one
// within r_K of the cell centre or of a periodic image disqualifies), then
// the cells within r_K (lanes over the (dy, dx) columns of the r_K cube, a
// loop over dz; each neighbour wrapped into the domain and found in the box
// that owns it, cells no box owns left out): a denser one (equal densities
// ranked by the global linear cell index, the lower index counting as
// denser) disqualifies.  Only the state before any creation is read.
// Qualifying cells are counted in work[0] and, up to max_new of them, their
// global linear index appended in arrival order to work[1 ..];
// work[1 + max_new ..] (pass 2's rank accumulators) is zeroed.  R = floor(r_K)
// must not exceed any axis length of the domain (one wrap per axis).
template <class T, class S>
__global__ __launch_bounds__(256) void k_create_find(Mesh M, const S* __restrict__ state,
                                                     const T* __restrict__ buf, SinkPos E,
                                                     double r_k, Limits L, long long max_new,
                                                     long long* __restrict__ work) {
  const int g = M.ghost;
  const int nx = M.domain[0], ny = M.domain[1], nz = M.domain[2];
  const int R = (int)floor(r_k), side = 2 * R + 1, plane = side * side;
  const double r2 = r_k * r_k;
  const int lane = threadIdx.x & (kWave - 1);
  const bool has_k = buf != nullptr && M.slot[5] >= 0;
  // the rank accumulators of pass 2 start at zero
  for (long long z = (long long)blockIdx.x * blockDim.x + threadIdx.x; z < max_new;
       z += (long long)gridDim.x * blockDim.x)
    work[1 + max_new + z] = 0;
  // the chunk loop is uniform over the block, so every wavefront runs the
  // ballots below with all its lanes
  for (long long ch = blockIdx.x; ch < M.n_apply_chunks; ch += gridDim.x) {
    const int2 C = M.apply_chunks[ch];
    const DevBox B = M.all_boxes[C.x];
    const long long c = (long long)C.y + threadIdx.x;  // owned cell of box C.x
    bool cand = false;
    double rho = 0.0;
    int gi = 0, gj = 0, gk = 0;
    long long key = 0;
    if (c < B.ncell) {
      const S* st = state + B.soff + c;
      rho = (double)st[0];
      if (rho > truelove_at(L, st, B.ncell)) {
        // box cells < 2^31: 32-bit quotients
        const unsigned cu = (unsigned)c, bnx = (unsigned)B.n[0], bny = (unsigned)B.n[1];
        const unsigned row = cu / bnx;
        const int li = (int)(cu - row * bnx);
        const int lk = (int)(row / bny);
        const int lj = (int)(row - (unsigned)lk * bny);
        gi = B.lo[0] + li;
        gj = B.lo[1] + lj;
        gk = B.lo[2] + lk;
        key = ((long long)gk * ny + gj) * nx + gi;
        cand = true;
        if (has_k) {
          const T* K = buf + B.boff + M.slot[5] * B.npad;
          cand = to_f64(K[((long long)(lk + g) * B.p[1] + (lj + g)) * B.p[0] + (li + g)]) == 0.0;
        }
      }
    }
    unsigned long long mask = __ballot(cand);
    while (mask) {
      const int src = __ffsll((long long)mask) - 1;
      mask &= mask - 1;
      const long long ck = __shfl(key, src, kWave);
      const double rc = __shfl(rho, src, kWave);
      const int ci = __shfl(gi, src, kWave), cj = __shfl(gj, src, kWave),
                cz = __shfl(gk, src, kWave);
      bool beaten = false;
      for (long long q = lane; q < E.n; q += kWave) {
        const double d2 = (image_term(ci, nx, E.x[q]) + image_term(cj, ny, E.y[q])) +
                          image_term(cz, nz, E.z[q]);
        beaten |= (d2 <= r2);
      }
      if (__ballot(beaten) == 0) {
        for (int q = lane; q < plane; q += kWave) {
          const int dj = q / side - R, di = q - (dj + R) * side - R;
          const int dyx = di * di + dj * dj;
          // members of this (dy, dx) column: dz^2 <= r_K^2 - dy^2 - dx^2, the
          // same test as (double)(dy^2 + dx^2 + dz^2) <= r_K^2 on integers
          int kmax = -1;
          while (kmax < R && (double)(dyx + (kmax + 1) * (kmax + 1)) <= r2) ++kmax;
          int w[3] = {ci + di, cj + dj, 0};
          w[0] += (w[0] < 0) ? nx : ((w[0] >= nx) ? -nx : 0);
          w[1] += (w[1] < 0) ? ny : ((w[1] >= ny) ? -ny : 0);
          for (int dk = -kmax; dk <= kmax; ++dk) {
            w[2] = cz + dk;
            w[2] += (w[2] < 0) ? nz : ((w[2] >= nz) ? -nz : 0);
            CellLoc Lc;
            if (!locate_wrapped(M, w, Lc)) continue;
            const long long o = ((long long)w[2] * ny + w[1]) * nx + w[0];
            const double ro = (double)state[Lc.s];
            beaten |= (o != ck) && ((ro > rc) || (ro == rc && o < ck));
          }
        }
      }
      if (__ballot(beaten) == 0 && lane == src) {
        const long long slot = (long long)atomicAdd((unsigned long long*)work, 1ull);
        if (slot < max_new) work[1 + slot] = ck;
      }
    }
  }
}

// Pass 2: the rank of each appended cell index (distinct keys), rank = how
// many others are smaller, accumulated into work[1 + max_new ..] (zeroed
// before).  Block (x, y) compares 256 keys against one LDS chunk of
// kRankChunk keys.  Does nothing when more cells qualified than max_new.
constexpr int kRankChunk = 2048;
__global__ __launch_bounds__(256) void k_create_rank(long long max_new,
                                                     long long* __restrict__ work) {
  __shared__ long long chunk[kRankChunk];
  const long long n = work[0];
  const long long t0 = (long long)blockIdx.x * blockDim.x;
  const long long u0 = (long long)blockIdx.y * kRankChunk;
  if (n > max_new || t0 >= n || u0 >= n) return;
  const long long* keys = work + 1;
  const int m = (int)((n - u0 < kRankChunk) ? n - u0 : kRankChunk);
  for (int u = threadIdx.x; u < m; u += blockDim.x) chunk[u] = keys[u0 + u];
  __syncthreads();
  const long long t = t0 + threadIdx.x;
  if (t >= n) return;
  const long long key = keys[t];
  long long rank = 0;
#pragma unroll 8
  for (int u = 0; u < m; ++u) rank += (chunk[u] < key);
  if (rank) atomicAdd((unsigned long long*)(work + 1 + max_new + t), (unsigned long long)rank);
}

// Pass 3: one thread per new sink, written at its rank (global cell index
// order).  The cell is found in the box that owns it.  The sink sits at the
// cell centre with mass (rho - rho_Tr) V and momentum mass * p / rho; the cell
// keeps its velocity and specific energy (rho -> rho_Tr, p -> (p / rho)
// rho_Tr, E -> (E / rho) rho_Tr), rho_Tr the cell's Truelove density before
// the update.  out is [7][max_new]: x, y, z, m, px, py, pz.
template <class S>
__global__ __launch_bounds__(256) void k_create_apply(Mesh M, S* __restrict__ state, Limits L,
                                                      long long max_new,
                                                      const long long* __restrict__ work,
                                                      double* __restrict__ out) {
  const long long n = work[0];
  if (n > max_new) return;
  const long long nx = M.domain[0], ny = M.domain[1];
  const long long* keys = work + 1;
  const long long* ranks = work + 1 + max_new;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x) {
    const long long c = keys[t], r = ranks[t];
    const long long row = c / nx;
    const int w[3] = {(int)(c - row * nx), (int)(row % ny), (int)(row / ny)};
    CellLoc Lc;
    if (!locate_wrapped(M, w, Lc)) continue;  // every key came from an owned cell
    S* cell = state + Lc.s;
    const long long nc = Lc.B->ncell;
    const double rho = (double)cell[0];
    const double rtr = truelove_at(L, (const S*)cell, nc);
    const double m = (rho - rtr) * M.V;
    out[r] = (double)w[0] + 0.5;
    out[max_new + r] = (double)w[1] + 0.5;
    out[2 * max_new + r] = (double)w[2] + 0.5;
    out[3 * max_new + r] = m;
    for (int a = 1; a <= 3; ++a) {
      const double v = (double)cell[a * nc] / rho;
      out[(3 + a) * max_new + r] = m * v;
      cell[a * nc] = (S)(v * rtr);
    }
    cell[4 * nc] = (S)(((double)cell[4 * nc] / rho) * rtr);
    cell[0] = (S)rtr;
  }
}

template <class T, class S>
static void create_launch(const Mesh& M, void* state, const void* buf, const SinkPos& E,
                          double r_k, const Limits& L, long long max_new, double* out,
                          long long* work, hipStream_t s) {
  const int grid = grid_for(M.n_apply_chunks, 1, M.num_cu * 32);
  hipLaunchKernelGGL((k_create_find<T, S>), dim3(grid), dim3(256), 0, s, M, (const S*)state,
                     (const T*)buf, E, r_k, L, max_new, work);
  if (max_new <= 0) return;
  const int gx = grid_for(max_new, 256, 1 << 30);
  const int gy = grid_for(max_new, kRankChunk, 1 << 30);
  hipLaunchKernelGGL(k_create_rank, dim3(gx, gy), dim3(256), 0, s, max_new, work);
  hipLaunchKernelGGL((k_create_apply<S>), dim3(grid_for(max_new, 256, 1024)), dim3(256), 0, s,
                     M, (S*)state, L, max_new, (const long long*)work, out);
}

hipError_t launch_sink_create(const Mesh& M, void* state, const void* buf, const SinkPos& E,
                              double r_k, const Limits& L, long long max_new, double* out,
                              long long* work, hipStream_t s) {
  hipError_t e = launch_zero(work, 8, 256, s);  // the count (the find pass zeroes the ranks)
  if (e != hipSuccess) return e;
  const bool f32 = (M.state == PMP_STATE_F32);
#define PMP_CR(T)                                                                     \
  (f32 ? create_launch<T, float>(M, state, buf, E, r_k, L, max_new, out, work, s)     \
       : create_launch<T, double>(M, state, buf, E, r_k, L, max_new, out, work, s))
  switch (M.acc) {
    case PMP_ACC_F32: PMP_CR(float); break;
    case PMP_ACC_F64R:
    case PMP_ACC_F64: PMP_CR(double); break;
    default: PMP_CR(long long);
  }
#undef PMP_CR
  return hipGetLastError();
}

template <int ACC>
static void fold_launch(const Mesh& M, void* buf, int block, hipStream_t s) {
  using T = typename AccT<ACC>::T;
  (void)block;
  const int grid = grid_for(M.n_fold_chunks, 1, M.num_cu * 64);
#define PMP_FOLD(F) \
  hipLaunchKernelGGL((k_fold<ACC, F>), dim3(grid), dim3(kChunk), 0, s, M, (T*)buf)
  switch (M.nfield) {
    case 1: PMP_FOLD(1); break;
    case 2: PMP_FOLD(2); break;
    case 3: PMP_FOLD(3); break;
    case 4: PMP_FOLD(4); break;
    case 5: PMP_FOLD(5); break;
    default: PMP_FOLD(6);
  }
#undef PMP_FOLD
}

template <int ACC>
static void fold_apply_launch(const Mesh& M, void* state, const void* buf, const Limits& L,
                              hipStream_t s) {
  using T = typename AccT<ACC>::T;
  const int grid = grid_for(M.n_fold_chunks, 1, M.num_cu * 64);
#define PMP_FA(F)                                                                           \
  hipLaunchKernelGGL((k_fold_apply<ACC, F>), dim3(grid), dim3(kChunk), 0, s, M, state,      \
                     (const T*)buf, L)
  switch (M.nfield) {
    case 1: PMP_FA(1); break;
    case 2: PMP_FA(2); break;
    case 3: PMP_FA(3); break;
    case 4: PMP_FA(4); break;
    case 5: PMP_FA(5); break;
    default: PMP_FA(6);
  }
#undef PMP_FA
}

hipError_t launch_fold_apply(const Mesh& M, void* state, const void* buf, const Limits& L,
                             hipStream_t s) {
  switch (M.acc) {
    case PMP_ACC_F32: fold_apply_launch<PMP_ACC_F32>(M, state, buf, L, s); break;
    case PMP_ACC_F64R:  // double buffer; its deposits are checked for the binned path
    case PMP_ACC_F64: fold_apply_launch<PMP_ACC_F64>(M, state, buf, L, s); break;
    default: fold_apply_launch<PMP_ACC_FIX64>(M, state, buf, L, s);
  }
  return hipGetLastError();
}

hipError_t launch_fold(const Mesh& M, void* buf, int block, hipStream_t s) {
  if (M.n_fold_chunks <= 0) return hipSuccess;
  switch (M.acc) {
    case PMP_ACC_F32: fold_launch<PMP_ACC_F32>(M, buf, block, s); break;
    case PMP_ACC_F64R:  // double buffer; its deposits are checked for the binned path
    case PMP_ACC_F64: fold_launch<PMP_ACC_F64>(M, buf, block, s); break;
    default: fold_launch<PMP_ACC_FIX64>(M, buf, block, s);
  }
  return hipGetLastError();
}

template <class S, int ACC>
static void apply_launch(const Mesh& M, void* state, const void* buf, const Limits& L,
                         double* eta, hipStream_t s) {
  using T = typename AccT<ACC>::T;
  const int grid = grid_for(M.n_apply_chunks, 1, M.num_cu * 64);
  hipLaunchKernelGGL((k_apply<S, ACC>), dim3(grid), dim3(kChunk), 0, s, M, (S*)state,
                     (const T*)buf, L, eta);
}

hipError_t launch_apply(const Mesh& M, void* state, const void* buf, const Limits& L,
                        double* eta, int block, hipStream_t s) {
  (void)block;
  const bool f32 = (M.state == PMP_STATE_F32);
  switch (M.acc) {
    case PMP_ACC_F32:
      f32 ? apply_launch<float, PMP_ACC_F32>(M, state, buf, L, eta, s)
          : apply_launch<double, PMP_ACC_F32>(M, state, buf, L, eta, s);
      break;
    case PMP_ACC_F64R:
    case PMP_ACC_F64:
      f32 ? apply_launch<float, PMP_ACC_F64>(M, state, buf, L, eta, s)
          : apply_launch<double, PMP_ACC_F64>(M, state, buf, L, eta, s);
      break;
    default:
      f32 ? apply_launch<float, PMP_ACC_FIX64>(M, state, buf, L, eta, s)
          : apply_launch<double, PMP_ACC_FIX64>(M, state, buf, L, eta, s);
  }
  return hipGetLastError();
}


}  // namespace pmp
