// HIP kernels (gfx950) of the split Crank-Nicolson PE range march, Eq. (4).
//
// One range step is two passes over the field u[theta][z] (depth contiguous):
//
//  pass A (depth pass, Eqs. (5)/(7)): per azimuth column, R = [I + beta_+ X] w
//    with w = [I + s_j D_theta] u^j, then solve [I + beta_- X] v = R.
//    A 256-lane workgroup owns 256/L columns; each column is split into L
//    contiguous chunks of M <= 17 rows (M odd), one per lane (L up to 256
//    lanes, so a column may span several wavefronts).  The column is staged through
//    LDS so that global loads and stores are coalesced along depth.  The
//    solve is a twisted factorisation: rows above the water/bottom interface
//    are eliminated top-down with the shared pivots of the all-water column,
//    rows below bottom-up with the shared pivots of the all-bottom column,
//    and the two interface rows form a 2x2 block.  Every first-order
//    recurrence of that elimination is split over the lanes: a local sweep
//    with zero carry, a segmented wavefront scan of the chunk's affine maps
//    (cross-lane shuffles), and a fix-up with the exact carry; three sweeps
//    in all (RHS and elimination end value; elimination, which also sums the
//    back-substitution end value; back substitution).
//
//  pass B (azimuth pass, Eqs. (6)/(8)): per depth, solve [I - s_j D_theta] u = v.
//    The operator is circulant (periodic) or Toeplitz (sector) with constant
//    coefficients and factors exactly as c (1 - rho S)(1 - rho S^-1), S the
//    cyclic shift, s rho^2 - (1 + 2s) rho + s = 0, |rho| < 1, c = s / rho.
//    The kernel solves u = (rho/s) (1 - rho S^-1)^-1 (1 - rho S)^-1 v directly:
//    two constant-coefficient recurrences (forward, backward) split into
//    azimuth chunks, with the cross-chunk carries and the periodic wrap (a
//    Sherman-Morrison rank-one correction of each cyclic bidiagonal factor)
//    evaluated in FP64; a sector adds the rank-one correction of its first
//    row.  (Solving for the defect u - v instead, from s D_theta v, cancels
//    about log10(4 sigma) digits on fields rough in azimuth: there u is
//    |v| / (4 sigma) while the defect is as large as v.)  Lanes are consecutive
//    depths, so every load and store is coalesced along z.  The same kernel
//    also applies the next step's azimuth factor [I + s_{j+1} D_theta] before
//    storing, so pass A of the next step is column-local.
//
// Precision split: kernels are templated on the storage type S of the field
// (float: complex64, double: complex128) and on the maximum chunk length.
// Every arithmetic operation and every coefficient is FP64 in both modes; in
// complex64 mode only the values held between sweeps are rounded to FP32.  A
// coefficient rounded to FP32 would perturb the per-step propagator by the same
// amount on every step and the error would grow linearly with range; data
// roundings change from step to step and only accumulate as a random walk.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "pe3d_internal.h"

namespace pe3d {

template <typename R>
using C = cplx<R>;

template <typename R>
__device__ __forceinline__ C<R> mk(R a, R b) {
  C<R> z;
  z.re = a;
  z.im = b;
  return z;
}
template <typename R>
__device__ __forceinline__ C<R> add(C<R> a, C<R> b) { return mk<R>(a.re + b.re, a.im + b.im); }
template <typename R>
__device__ __forceinline__ C<R> sub(C<R> a, C<R> b) { return mk<R>(a.re - b.re, a.im - b.im); }
template <typename R>
__device__ __forceinline__ C<R> mul(C<R> a, C<R> b) {
  return mk<R>(::fma(a.re, b.re, -a.im * b.im), ::fma(a.re, b.im, a.im * b.re));
}
// a*b + c
template <typename R>
__device__ __forceinline__ C<R> fma(C<R> a, C<R> b, C<R> c) {
  return mk<R>(::fma(a.re, b.re, ::fma(-a.im, b.im, c.re)), ::fma(a.re, b.im, ::fma(a.im, b.re, c.im)));
}
template <typename R>
__device__ __forceinline__ C<R> scl(R a, C<R> b) { return mk<R>(a * b.re, a * b.im); }
template <typename R>
__device__ __forceinline__ C<R> zero() { return mk<R>(R(0), R(0)); }
template <typename R>
__device__ __forceinline__ C<R> one() { return mk<R>(R(1), R(0)); }

template <typename R>
__device__ __forceinline__ C<R> shfl_up(C<R> v, int d, int w) {
  return mk<R>(__shfl_up(v.re, d, w), __shfl_up(v.im, d, w));
}
template <typename R>
__device__ __forceinline__ C<R> shfl_down(C<R> v, int d, int w) {
  return mk<R>(__shfl_down(v.re, d, w), __shfl_down(v.im, d, w));
}

// Lane moves inside a wavefront through DPP (a VALU operand modifier, no LDS
// round trip).  CTRL is a DPP control: row_shr:n 0x110+n and row_shl:n
// 0x100+n (lane i reads lane i-n / i+n of its row of 16), row_bcast:15 0x142
// and row_bcast:31 0x143 (lane 15 of a row / lane 31 to the rows after it),
// wave_shr:1 0x138 and wave_shl:1 0x130 (lane i reads lane i-1 / i+1 of the
// wavefront).  Lanes whose source falls outside the pattern, or whose row is
// not in ROWMASK, read 0.
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ double dpp_f64(double x) {
  const unsigned long long v = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, int(unsigned(v)), CTRL, ROWMASK, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, int(unsigned(v >> 32)), CTRL, ROWMASK, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)unsigned(hi) << 32) | unsigned(lo)));
}
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ C<double> dpp(C<double> v) {
  return mk<double>(dpp_f64<CTRL, ROWMASK>(v.re), dpp_f64<CTRL, ROWMASK>(v.im));
}

template <typename R>
__device__ __forceinline__ C<R> from_d(C<double> z) { return mk<R>(R(z.re), R(z.im)); }
template <typename R>
__device__ __forceinline__ C<double> to_d(C<R> z) { return mk<double>(double(z.re), double(z.im)); }
using D = C<double>;

// ---------------------------------------------------------------- FP64 helpers
// Field loads and stores through a pointer in the global address space:
// a uniform (scalar) base plus a 32-bit per-lane element offset.
template <typename S>
struct Vec2;
template <>
struct Vec2<float> {
  typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec2<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};
// threadIdx.x; FRESH: read afresh at each use.  Inside the persistent
// kernel's task loop the compiler would otherwise hoist the lane arithmetic
// of every pass body out of the loop and keep all of it live across the
// whole loop (spilling registers).
template <bool FRESH>
__device__ __forceinline__ int lane_id() {
  int x = threadIdx.x;
  if (FRESH) asm volatile("" : "+v"(x));
  return x;
}

template <typename S>
__device__ __forceinline__ C<S> gload(const C<S>* base, unsigned off) {
  using V = typename Vec2<S>::type;
  const __attribute__((address_space(1))) V* p = (const __attribute__((address_space(1))) V*)base;
  const V v = p[off];
  return mk<S>(v.x, v.y);
}
// FP64 complex table entry at a 32-bit byte offset from a uniform base
__device__ __forceinline__ C<double> gload_b(const void* base, unsigned boff) {
  using V = Vec2<double>::type;
  const __attribute__((address_space(1))) char* p = (const __attribute__((address_space(1))) char*)base;
  const V v = *(const __attribute__((address_space(1))) V*)(p + boff);
  return mk<double>(v.x, v.y);
}
template <typename S>
__device__ __forceinline__ void gstore(C<S>* base, unsigned off, C<S> val) {
  using V = typename Vec2<S>::type;
  __attribute__((address_space(1))) V* p = (__attribute__((address_space(1))) V*)base;
  V v;
  v.x = val.re;
  v.y = val.im;
  p[off] = v;
}

// Registers that stage field values in pass A: the complex itself for
// complex64, a double2 vector for complex128 (a 16-byte struct assigned under
// a condition into a private array is not promoted to registers by the
// compiler: it would live in scratch memory, each load waiting for the last).
template <typename S>
struct Stage {
  using T = C<S>;
};
template <>
struct Stage<double> {
  using T = Vec2<double>::type;
};
// (global address space: the field pointers of a batched launch come from
// memory, and a generic access would be a FLAT one)
__device__ __forceinline__ C<float> stage_load(const C<float>* p, size_t e) {
  using V = Vec2<float>::type;
  const V v = ((const __attribute__((address_space(1))) V*)p)[e];
  return mk<float>(v.x, v.y);
}
__device__ __forceinline__ Vec2<double>::type stage_load(const C<double>* p, size_t e) {
  using V = Vec2<double>::type;
  return ((const __attribute__((address_space(1))) V*)p)[e];
}
__device__ __forceinline__ C<float> stage_val(C<float> v) { return v; }
__device__ __forceinline__ C<double> stage_val(Vec2<double>::type v) { return mk<double>(v.x, v.y); }

__device__ __forceinline__ C<double> cdiv(C<double> a, C<double> b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    double r = b.im / b.re, den = b.re + b.im * r;
    return mk<double>((a.re + a.im * r) / den, (a.im - a.re * r) / den);
  }
  double r = b.re / b.im, den = b.re * r + b.im;
  return mk<double>((a.re * r + a.im) / den, (a.im * r - a.re) / den);
}
// principal square root
__device__ __forceinline__ C<double> csqrt(C<double> z) {
  double m = hypot(z.re, z.im);
  if (z.re >= 0.0) {
    double t = sqrt(0.5 * (m + z.re));
    return mk<double>(t, t > 0.0 ? z.im / (2.0 * t) : 0.0);
  }
  double t = sqrt(0.5 * (m - z.re));
  return mk<double>(fabs(z.im) / (2.0 * t), z.im >= 0.0 ? t : -t);
}
__device__ __forceinline__ C<double> cpow(C<double> z, long long n) {
  C<double> r = one<double>();
  while (n > 0) {
    if (n & 1) r = mul(r, z);
    z = mul(z, z);
    n >>= 1;
  }
  return r;
}
// azimuth coefficient of the step j -> j+1: (delta/4) Y = s D_theta,
// s = i dr / (4 k0 r_{j+1}^2 dtheta^2)
__device__ __forceinline__ double sigma_of(const ProbDesc& d, long long j) {
  double r = d.r0 + double(j + 1) * d.dr;
  return d.dr / (4.0 * d.k0 * r * r * d.dth * d.dth);
}
// Water nodes of column m at range r_{j+1} when the depth has range rows
// (the per-step matrix update of Fig. 2; the medium update writes them for the
// depth pass): D(r) between the column's depths at
// the rows r_i = br0 + i bdr (slope * (r - r_i) + D_i inside an interval, D_i
// at a node, the end values outside), then #{l = 1..nz : l dz <= D}.  Every
// operation is a correctly rounded FP64 one with no contraction, as on the
// host and in a plain evaluation of the same formula, so the integer count is
// the same everywhere.  Uniform across the column's lanes.
__device__ __forceinline__ int water_nodes_at(const ProbDesc& d, int m, long long j) {
  const double r = __dadd_rn(d.r0, __dmul_rn(double(j + 1), d.dr));
  const double* dc = d.dcol + (size_t)m * d.nbr;
  const int nr = d.nbr;
  auto node = [&](int i) { return __dadd_rn(d.br0, __dmul_rn(double(i), d.bdr)); };
  double D;
  if (r <= node(0)) {
    D = dc[0];
  } else if (r >= node(nr - 1)) {
    D = dc[nr - 1];
  } else {
    // the interval node(i) <= r < node(i+1): a first guess, then exact steps
    int i = int(fmin(fmax(floor(__ddiv_rn(__dsub_rn(r, d.br0), d.bdr)), 0.0), double(nr - 2)));
    while (i > 0 && node(i) > r) --i;
    while (i < nr - 2 && node(i + 1) <= r) ++i;
    const double ra = node(i);
    if (r == ra) {
      D = dc[i];
    } else {
      const double slope = __ddiv_rn(__dsub_rn(dc[i + 1], dc[i]), __dsub_rn(node(i + 1), ra));
      D = __dadd_rn(__dmul_rn(slope, __dsub_rn(r, ra)), dc[i]);
    }
  }
  const int N = d.nz;
  int nw = int(fmin(fmax(floor(__ddiv_rn(D, d.dz)), 0.0), double(N)));
  while (nw < N && __dmul_rn(double(nw + 1), d.dz) <= D) ++nw;
  while (nw > 0 && __dmul_rn(double(nw), d.dz) > D) --nw;
  return nw;
}

// Water-profile row in force at r_{j+1}: the last row whose range
// sr0 + i sdr (correctly rounded, as in a plain evaluation) is <= r_{j+1},
// row 0 before the first; a first guess, then exact comparisons.
__device__ __forceinline__ int ssp_row_at(const ProbDesc& d, long long j) {
  const double r = __dadd_rn(d.r0, __dmul_rn(double(j + 1), d.dr));
  auto node = [&](int i) { return __dadd_rn(d.sr0, __dmul_rn(double(i), d.sdr)); };
  const int nr = d.nsr;
  int i = int(fmin(fmax(floor(__ddiv_rn(__dsub_rn(r, d.sr0), d.sdr)), 0.0), double(nr - 1)));
  while (i > 0 && node(i) > r) --i;
  while (i < nr - 1 && node(i + 1) <= r) ++i;
  return i;
}

// The medium of step j: the water nodes of column m (depth rows) and the
// table pointers of the water row (water rows, one thread).
__device__ __forceinline__ void medium_update_col(const ProbDesc& d, int m, long long j) {
  if (d.nbr && m < d.nth) d.nwcol[m] = water_nodes_at(d, m, j);
}
__device__ __forceinline__ void medium_update_row(const ProbDesc& d, long long j) {
  const long long off = (long long)ssp_row_at(d, j) * d.row_stride;
  TabPtrs t;
  t.tabG = (const char*)d.tabG + off;
  t.tabC = (const char*)d.tabC + off;
  t.tabP = (const char*)d.tabP + off;
  t.rec = (const char*)d.rec + off;
  *d.cur = t;
}
__device__ __forceinline__ void medium_update(const ProbDesc& d, int tile, int koff) {
  const long long j = *d.jdev + koff;
  medium_update_col(d, tile * 256 + threadIdx.x, j);
  if (d.nsr && tile == 0 && threadIdx.x == 0) medium_update_row(d, j);
}
// The medium of the next step, written at the end of an azimuth pass by the
// workgroup of depth tile 0 (the next depth pass starts only after every
// workgroup of this one has finished, and this pass no longer reads it).
__device__ __forceinline__ void medium_update_next(const ProbDesc& d, int tile, int koff) {
  if (!(d.nbr || d.nsr) || tile != 0 || koff + 1 >= d.nsteps) return;
  const long long j = *d.jdev + koff + 1;
  for (int m = threadIdx.x; m < d.nth; m += blockDim.x) medium_update_col(d, m, j);
  if (d.nsr && threadIdx.x == 0) medium_update_row(d, j);
}

// root of s rho^2 - (1+2s) rho + s = 0 inside the unit circle, s = i sigma:
// rho = 2s / (1 + 2s + sqrt(1 + 4s)), and rho / s = 2 / (1 + 2s + sqrt(1 + 4s))
// (no division by s, which vanishes far from the source)
__device__ __forceinline__ C<double> rho_den(double sigma) {
  C<double> q = csqrt(mk<double>(1.0, 4.0 * sigma));
  return mk<double>(1.0 + q.re, 2.0 * sigma + q.im);
}
__device__ __forceinline__ C<double> rho_of(double sigma) {
  return cdiv(mk<double>(0.0, 2.0 * sigma), rho_den(sigma));
}
__device__ __forceinline__ C<double> rho_over_s(double sigma) {
  return cdiv(mk<double>(2.0, 0.0), rho_den(sigma));
}


template <typename R>
__device__ __forceinline__ C<R> shfl_idx(C<R> v, int src, int w) {
  return mk<R>(__shfl(v.re, src, w), __shfl(v.im, src, w));
}

__device__ __forceinline__ int ncp_of(int nc) {
  int p = 1;
  while (p < nc) p <<= 1;
  return p;
}

// ============================================================== pass A
// Workgroup of 256 lanes; a depth column uses L lanes (a power of two,
// 4..256; columns wider than a wavefront combine per-wavefront scan totals
// through LDS), 256/L columns per workgroup.  M (odd, <= 17) rows per lane.
//
// Lane layout of a column with interface rows k, k+1 (twisted factorisation):
//   top chain    rows 0..k in natural order, preceded by s >= 1 zero slots
//                so that row k is the last slot of lane a-1;
//   bottom chain rows N-1..k+1 (reversed), preceded by sb >= 1 zero slots
//                so that row k+1 is the last slot of lane a+nbl-1;
//   idle lanes   after the bottom chain.
// Both chains are eliminated in increasing lane order and back-substituted
// in decreasing lane order, so every lane runs the same code; the two
// interface rows sit in the last slot of their chain's last lane (the
// "head" lanes).  The leading zero slots have zero table entries, so a
// chain's first lane has a zero transfer product and no carry crosses from
// one chain into the next.
//
// Recurrences (nbmh = -beta_- h is the off-diagonal of every non-interface
// row of [I + beta_- X] with the rigid floor row halved; right-hand sides are
// carried divided by nbmh, Rt = R / nbmh, and Gh = nbmh / pivot):
//   elimination        yh_j = Gh_j (Rt_j + yh_{j-1})
//   back substitution  x_j  = yh_j + Gh_j x_{j+1}
// Both have the per-slot multiplier Gh_j, so one table of lane transfer
// products serves the two scans.
constexpr int kPassAThreads = 256;

// Exclusive scan of the affine lane maps x -> A x + B within a column:
// UP: lane t receives the composition of lanes 0..t-1 applied to 0; DOWN:
// of lanes L-1..t+1.  Inside a wavefront: an inclusive scan within each row
// of 16 lanes by DPP row shifts (segments of w < 16 lanes lie inside one row),
// then across rows (UP: DPP row broadcasts of lane 15 and lane 31; DOWN: the
// first lane of the next row and lane 32 by shuffles), then a DPP shift by
// one lane.  Columns wider than a wavefront combine the wavefront totals
// through LDS.  tot: LDS scratch, 2 complex per wavefront.
template <bool UP, bool FRESH>
__device__ __forceinline__ D scan_excl(D A, D B, int t, int L, D* tot) {
  const int w = L < 64 ? L : 64;
  const int tw = t & (w - 1);
  const int h = lane_id<FRESH>() & 63;
  const int pr = h & 15;
  // the lane's map composed after the neighbour's (ap, bq)
  auto comb = [&](const D& ap, const D& bq, bool take) {
    if (take) {
      B = fma(A, bq, B);
      A = mul(A, ap);
    }
  };
  if (UP) {
    if (w > 1) comb(dpp<0x111>(A), dpp<0x111>(B), tw >= 1 && pr >= 1);
    if (w > 2) comb(dpp<0x112>(A), dpp<0x112>(B), tw >= 2 && pr >= 2);
    if (w > 4) comb(dpp<0x114>(A), dpp<0x114>(B), tw >= 4 && pr >= 4);
    if (w > 8) comb(dpp<0x118>(A), dpp<0x118>(B), tw >= 8 && pr >= 8);
    if (w > 16) comb(dpp<0x142, 0xA>(A), dpp<0x142, 0xA>(B), (h & 16) != 0);
    if (w > 32) comb(dpp<0x143, 0xC>(A), dpp<0x143, 0xC>(B), (h & 32) != 0);
  } else {
    if (w > 1) comb(dpp<0x101>(A), dpp<0x101>(B), tw + 1 < w && pr + 1 < 16);
    if (w > 2) comb(dpp<0x102>(A), dpp<0x102>(B), tw + 2 < w && pr + 2 < 16);
    if (w > 4) comb(dpp<0x104>(A), dpp<0x104>(B), tw + 4 < w && pr + 4 < 16);
    if (w > 8) comb(dpp<0x108>(A), dpp<0x108>(B), tw + 8 < w && pr + 8 < 16);
    if (w > 16) {
      const int src = (h | 15) + 1;  // first lane of the next row (used by even rows)
      comb(shfl_idx(A, src, 64), shfl_idx(B, src, 64), (h & 16) == 0);
    }
    if (w > 32) comb(shfl_idx(A, 32, 64), shfl_idx(B, 32, 64), (h & 32) == 0);
  }
  D ea = UP ? dpp<0x138>(A) : dpp<0x130>(A);
  D eb = UP ? dpp<0x138>(B) : dpp<0x130>(B);
  if (UP ? (tw == 0) : (tw == w - 1)) {
    ea = one<double>();
    eb = zero<double>();
  }
  D x = zero<double>();
  if (L > 64) {
    const int wave = lane_id<FRESH>() >> 6;
    if (UP ? (tw == 63) : (tw == 0)) {
      tot[2 * wave + 0] = A;
      tot[2 * wave + 1] = B;
    }
    __syncthreads();
    const int nwv = L >> 6;
    const int wc = t >> 6;
    const int w0 = wave - wc;
    if (UP) {
      for (int q = 0; q < wc; ++q) x = fma(tot[2 * (w0 + q)], x, tot[2 * (w0 + q) + 1]);
    } else {
      for (int q = nwv - 1; q > wc; --q) x = fma(tot[2 * (w0 + q)], x, tot[2 * (w0 + q) + 1]);
    }
    __syncthreads();
  }
  return fma(ea, x, eb);
}

__host__ __device__ constexpr int pass_a_align(int b) { return (b + 15) & ~15; }

// LDS of one workgroup: 256/L column buffers of N + 2(M+1) entries (rows
// -(M+1)..N+M, zero outside the column), the interface exchange (2 complex
// per column) and the scan totals (2 complex per wavefront).
__host__ __device__ constexpr int pass_a_lds_bytes(int esz, int L, int N, int M) {
  return pass_a_align((kPassAThreads / L) * (N + 2 * (M + 1)) * esz) + (kPassAThreads / L) * 2 * 16 +
         8 * 16;
}

// MULTI: the depth pass of an N x 2D problem over a fixed medium (no range
// rows) for every step of a call in one launch: without azimuth coupling a
// column depends on nothing but itself, so the workgroup's columns stay in
// LDS from step to step, read from the caller's field once (koff = 0) and
// written back once.  Otherwise one step, koff steps into the call.
// FRESH: see lane_id (the persistent kernel)
template <typename S, int M, bool MULTI = false, bool FRESH = false>
__device__ __forceinline__ void pass_a_body(const ProbDesc& d, int tile, int koff, unsigned char* smem) {
  const int lane = lane_id<FRESH>();
  const int L = d.lpc;
  const int lgL = 31 - __clz(L);
  const int cpw = kPassAThreads >> lgL;
  const int cw = lane >> lgL;
  const int t = lane & (L - 1);
  const int N = d.nz, NT = d.nth;
  const int m0 = tile * cpw;
  const int m = m0 + cw;
  const bool colok = m < NT;
  const int ncols = min(cpw, NT - m0);
  constexpr int GA = M + 1;
  const int CS = N + 2 * GA;
  C<S>* buf = reinterpret_cast<C<S>*>(smem);
  D* xch = reinterpret_cast<D*>(smem + pass_a_align(cpw * CS * int(sizeof(C<S>))));
  D* tot = xch + 2 * cpw;
  const bool first = (koff == 0);
  const bool ystage = first && !d.nx2d;  // first step of a 3D march: apply [I + s_0 D]
  const C<S>* __restrict__ src = (const C<S>*)(first ? d.u : d.scr);
  C<S>* __restrict__ dst = (C<S>*)((MULTI || (d.nx2d && koff == d.nsteps - 1)) ? d.u : d.scr);

  // ---- zero the guard rows of every column buffer, stage the columns.  The
  //      workgroup's columns are one contiguous span of ncols*N values;
  //      thread `lane` takes entries lane + 256 q, q < M (ncols*N < 256 M),
  //      all loads issued before the first LDS write.  On the first step
  //      apply [I + s_0 D_theta] from the neighbouring columns.
  // the column's water nodes (they set the lane roles) are read first, so
  // that their latency overlaps the staging
  const int nw_early = colok ? ((const __attribute__((address_space(1))) int*)d.nwcol)[m] : 0;
  // the tables of this step's water row (uniform scalar loads)
  const __attribute__((address_space(4))) TabPtrs* const tcur =
      (const __attribute__((address_space(4))) TabPtrs*)d.cur;
  const void* const tabG = tcur->tabG;
  const void* const tabC = tcur->tabC;
  const void* const tabP = tcur->tabP;
  const void* const trec = tcur->rec;
  for (int i = lane; i < cpw * 2 * GA; i += kPassAThreads) {
    const int c = i / (2 * GA);
    const int g = i - c * 2 * GA;
    buf[c * CS + (g < GA ? g : N + g)] = zero<S>();
  }
  const int span = ncols * N;
  const float invN = 1.0f / float(N);
  const C<S>* __restrict__ base = src + (size_t)m0 * N;
  // complex64 with an even column length: thread `lane` takes the pairs of
  // entries 2 (lane + 256 q), q < (M+1)/2, with one 16-byte load each (a pair
  // never crosses a column; the span and its base are 16-byte aligned)
  const bool pairs = sizeof(S) == 4 && (N & 1) == 0;
  if (!ystage && pairs) {
    using F4 = float __attribute__((ext_vector_type(4)));
    constexpr int MP = (M + 1) / 2;
    const __attribute__((address_space(1))) F4* b4 = (const __attribute__((address_space(1))) F4*)base;
    F4 v2[MP];
    __builtin_amdgcn_s_setprio(2);  // issue the staging loads at raised priority
    #pragma unroll
    for (int q = 0; q < MP; ++q) {
      const int e = 2 * (lane + q * kPassAThreads);
      if (e < span) v2[q] = b4[e >> 1];
    }
    __builtin_amdgcn_s_setprio(0);
    #pragma unroll
    for (int q = 0; q < MP; ++q) {
      const int e = 2 * (lane + q * kPassAThreads);
      if (e < span) {
        const int c = cpw == 1 ? 0 : int((float(e) + 0.5f) * invN);
        const int idx = c * CS + GA + (e - c * N);
        buf[idx] = mk<S>(S(v2[q].x), S(v2[q].y));
        buf[idx + 1] = mk<S>(S(v2[q].z), S(v2[q].w));
      }
    }
  } else if (!ystage) {
    typename Stage<S>::T v[M];
    #pragma unroll
    for (int q = 0; q < M; ++q) {
      const int e = lane + q * kPassAThreads;
      if (e < span) v[q] = stage_load(base, e);
    }
    // LDS index of span entry e (column c = e / N, row e - c N): c CS + GA + e - c N
    if (cpw == 1) {
      #pragma unroll
      for (int q = 0; q < M; ++q) {
        const int e = lane + q * kPassAThreads;
        if (e < span) buf[GA + e] = stage_val(v[q]);
      }
    } else if (N >= kPassAThreads) {
      // e advances by 256 <= N per entry: the column advances by at most one
      int r = lane, idx = GA + lane;
      #pragma unroll
      for (int q = 0; q < M; ++q) {
        if (lane + q * kPassAThreads < span) buf[idx] = stage_val(v[q]);
        r += kPassAThreads;
        idx += kPassAThreads;
        if (r >= N) {
          r -= N;
          idx += 2 * GA;
        }
      }
    } else {
      #pragma unroll
      for (int q = 0; q < M; ++q) {
        const int e = lane + q * kPassAThreads;
        if (e < span) {
          const int c = int((float(e) + 0.5f) * invN);
          buf[c * CS + GA + (e - c * N)] = stage_val(v[q]);
        }
      }
    }
  } else {
    // first step of a march call only: groups of 4 entries (a rolled loop), so
    // that its three loads per entry do not set the kernel's register count
    const long long j = *d.jdev + koff;
    const double s0 = sigma_of(d, j);  // s_0 = i * s0
    constexpr int QG = 4;
#pragma unroll 1
    for (int q0 = 0; q0 < M; q0 += QG) {
      typename Stage<S>::T vc[QG], vl[QG], vr[QG];
      #pragma unroll
      for (int qq = 0; qq < QG; ++qq) {
        const int e = lane + (q0 + qq) * kPassAThreads;
        if (q0 + qq < M && e < span) {
          const int c = int((float(e) + 0.5f) * invN);
          const int r = e - c * N;
          const int mm = m0 + c;
          int ml = mm - 1, mr = mm + 1;
          if (d.periodic) {
            if (ml < 0) ml = NT - 1;
            if (mr >= NT) mr = 0;
          }
          // sector edges: load an in-range column, zero it below
          vc[qq] = stage_load(base, e);
          vl[qq] = stage_load(src, (size_t)max(ml, 0) * N + r);
          vr[qq] = stage_load(src, (size_t)min(mr, NT - 1) * N + r);
        }
      }
      #pragma unroll
      for (int qq = 0; qq < QG; ++qq) {
        const int e = lane + (q0 + qq) * kPassAThreads;
        if (q0 + qq < M && e < span) {
          const int c = int((float(e) + 0.5f) * invN);
          const int mm = m0 + c;
          const bool hl = d.periodic || mm > 0, hr = d.periodic || mm < NT - 1;
          const D uc = to_d(stage_val(vc[qq]));
          const D ul = hl ? to_d(stage_val(vl[qq])) : zero<double>();
          const D ur = hr ? to_d(stage_val(vr[qq])) : zero<double>();
          const D dd = sub(add(ul, ur), scl(2.0, uc));
          buf[c * CS + GA + (e - c * N)] = from_d<S>(mk<double>(uc.re - s0 * dd.im, uc.im + s0 * dd.re));
        }
      }
    }
  }

  // ---- lane role: the column's water nodes nw (at r_{j+1}, written by
  //      the medium update before this launch, when the depth depends on range)
  //      set its interface row k and record
  const int nw = nw_early;
  const int k = min(max(nw - 1, 0), N - 2);
  const int a = (k + 1) / M + 1;
  const int s = a * M - (k + 1);
  const int nbl = (N - k - 1) / M + 1;
  const int sb = nbl * M - (N - k - 1);
  const bool top = colok && t < a;
  const bool bot = colok && !top && t < a + nbl;
  const bool head = colok && (t == a - 1 || t == a + nbl - 1);
  const int tc = top ? t : (bot ? t - a : 0);
  const int sc = top ? s : (bot ? sb : M);
  const int tb = bot ? 1 : 0;
  // (idle lanes read and write the outermost guard row, which no chain lane
  // reads or writes)
  const int row0 = top ? t * M - s : (bot ? N - 1 - (tc * M - sb) : -GA);
  const int dir = top ? 1 : (bot ? -1 : 0);

  // table byte offsets of the lane's slots (lane-major, padded by M zero rows)
  const int LT = d.lt;
  unsigned offb[M];
  {
    const int lo = tb * M * LT + (M - sc) * LT + tc;  // slot j < sc
    const int hi = tb * M * LT + tc + 1 - sc * LT;    // slot j >= sc
    #pragma unroll
    for (int j = 0; j < M; ++j) offb[j] = unsigned((j < sc ? lo : hi) + j * LT) * 16u;
  }
  // A prefetch is issued only after the current slot's value `after` exists:
  // its offset passes through an empty volatile asm that also reads that
  // value, so the compiler can neither hoist the load to the phase start nor
  // sink the slot's arithmetic below it.
  // Table reads.  A lane needs the tables only for its chain rows below the
  // chain's converged tail: slots j < jlo are the chain's leading zero rows
  // (only its first lane has them), slots j >= jhi tail rows (the chain's
  // constants); idle lanes need none.  A wavefront in which no lane needs
  // them (wtab false) runs the sweeps with the constants instead of reads
  // (the tables hold the same values, so both forms give the same numbers).
  const int jlo = (top || bot) ? max(sc - tc * M, 0) : M;
  const int jhi = (top || bot) ? min(max(d.bconv[tb] + sc - tc * M, jlo), M) : M;
  const bool wtab = __ballot(jlo < jhi) != 0;
  auto G_at = [&](auto tab, int j, const D& after) {
    if constexpr (decltype(tab)::value) {
      unsigned o = offb[j];
      asm volatile("" : "+v"(o) : "v"(after.re));
      return gload_b(tabG, o);
    } else {
      D v = j < jlo ? zero<double>() : mk<double>(d.gt_re[tb], d.gt_im[tb]);
      asm volatile("" : "+v"(v.re), "+v"(v.im) : "v"(after.re));  // same order as the reads
      return v;
    }
  };
  auto C_at = [&](auto tab, int j, const D& after) {
    if constexpr (decltype(tab)::value) {
      unsigned o = offb[j];
      asm volatile("" : "+v"(o) : "v"(after.re));
      return gload_b(tabC, o);
    } else {
      D v = j < jlo ? zero<double>() : mk<double>(d.ct_re[tb], d.ct_im[tb]);
      asm volatile("" : "+v"(v.re), "+v"(v.im) : "v"(after.re));
      return v;
    }
  };
  // the head lanes' interface coefficients: RHS diagonal, previous and next
  // coefficient, elimination multiplier, then the two inverse entries
  const unsigned hoff = unsigned(nw * 12 + (bot ? 6 : 0)) * 16u;  // byte offset in the records
  auto hrec = [&](int q) { return gload_b(trec, hoff + unsigned(q) * 16u); };

  const D cbs = mk<double>(d.cbs_re, d.cbs_im);
  D tp = zero<double>();
  if (top || bot) tp = gload_b(tabP, unsigned((tb * (M + 1) + sc) * L + tc) * 16u);
  __syncthreads();

  // Table values are prefetched PF slots ahead.
  constexpr int PF = 6;

  // one step on the columns in LDS
  auto step = [&]() __attribute__((always_inline)) {
    // ---- phase 1: Rt = [I + beta_+ X] w / nbmh along the chain (sliding
    //      window), local elimination with zero carry -> the lane's map
    //      yh_out = tp yh_in + E
    const C<S>* col = buf + cw * CS + GA;
    D Rv[M];
    // GREG: the lane's multipliers stay in registers from the RHS sweep to the
    // elimination and back substitution (no further table reads); otherwise
    // those sweeps read the table again (fewer registers: complex64 with
    // M >= 15 keeps 3 waves per SIMD that way)
    constexpr bool GREG = sizeof(S) == 8 || M <= 13;
    D Gv[GREG ? M : 1];
    D E = zero<double>();
    auto phase1 = [&](auto tab) {
      D gq[PF], cq[PF];
      #pragma unroll
      for (int j = 0; j < PF; ++j)
        if (j < M) {
          gq[j] = G_at(tab, j, E);
          cq[j] = C_at(tab, j, E);
        }
      const C<S>* p = col + row0;
      D wp = to_d(p[-dir]);
      D wc = to_d(p[0]);
      // row of the next window entry, advanced by dir per slot; the empty asm
      // orders the read after the previous slot's value and is applied to the
      // index, not to a pointer, so the read stays an LDS read
      int rn = row0;
      #pragma unroll
      for (int j = 0; j < M; ++j) {
        const D g = gq[j % PF];
        const D cdv = cq[j % PF];
        if constexpr (GREG) Gv[j] = g;
        rn += dir;
        asm volatile("" : "+v"(rn) : "v"(E.re));
        const D wn = to_d(col[rn]);
        D R;
        if (j == M - 1) {
          D c0 = cdv, cp = cbs, cn = cbs, cf = one<double>();
          if (head) {
            c0 = hrec(0);
            cp = hrec(1);
            cn = hrec(2);
            cf = hrec(3);
          }
          R = fma(c0, wc, fma(cp, wp, mul(cn, wn)));
          const D y = fma(cf, E, R);
          E = head ? y : mul(g, y);
        } else {
          R = fma(cdv, wc, mul(cbs, add(wp, wn)));
          E = mul(g, add(R, E));
        }
        if (j + PF < M) {
          gq[j % PF] = G_at(tab, j + PF, E);
          cq[j % PF] = C_at(tab, j + PF, E);
        }
        Rv[j] = R;
        wp = wc;
        wc = wn;
      }
    };
    if (wtab)
      phase1(std::true_type{});
    else
      phase1(std::false_type{});
    const D cin = scan_excl<true, FRESH>(tp, E, t, L, tot);

    // ---- phase 2: elimination with the exact carry; Rv <- yh (head slot: the
    //      reduced interface right-hand side, divided by nbmh).  The same sweep
    //      accumulates the lane's local back-substitution end value with zero
    //      carry, X = sum_j (Gh_0 ... Gh_{j-1}) yh_j (the back substitution
    //      x_j = yh_j + Gh_j x_{j+1} unrolled from the lane's first slot), so the
    //      back substitution needs one sweep only; a head lane adds its own
    //      slot's term once the interface value is known.
    D X = zero<double>();
    D pr = one<double>();  // Gh_0 ... Gh_{j-1}
    if constexpr (GREG) {
      {
        D yh = cin;
        #pragma unroll
        for (int j = 0; j < M; ++j) {
          const D g = Gv[j];
          if (j == M - 1) {
            D cf = one<double>();
            if (head) cf = hrec(3);
            const D y = fma(cf, yh, Rv[j]);
            Rv[j] = head ? y : mul(g, y);
            if (!head) X = fma(pr, Rv[j], X);
          } else {
            yh = mul(g, add(Rv[j], yh));
            Rv[j] = yh;
            X = fma(pr, yh, X);
            pr = mul(pr, g);
            // keep the accumulation in slot order (not batched up over the sweep)
            asm volatile("" : "+v"(X.re), "+v"(X.im), "+v"(pr.re), "+v"(pr.im) : "v"(yh.re));
          }
        }
      }
    } else {
      // The elimination sweep reads the table in every wavefront; a lane that
      // needs no entry reads the chain's tail row or a zero row instead (the same
      // address for many lanes, fewer cache lines per read).
      const unsigned toff = unsigned(tb * M * LT + ((N - 2 + M) % M) * LT + (N - 2 + M) / M) * 16u;
      auto G2_at = [&](int j, const D& after) {
        unsigned o = (j >= jlo && j < jhi) ? offb[j] : (j < jlo ? 0u : toff);
        asm volatile("" : "+v"(o) : "v"(after.re));
        return gload_b(tabG, o);
      };
      {
        D yh = cin;
        D gq[PF];
        #pragma unroll
        for (int j = 0; j < PF; ++j)
          if (j < M) gq[j] = G2_at(j, yh);
        #pragma unroll
        for (int j = 0; j < M; ++j) {
          const D g = gq[j % PF];
          if (j == M - 1) {
            D cf = one<double>();
            if (head) cf = hrec(3);
            const D y = fma(cf, yh, Rv[j]);
            Rv[j] = head ? y : mul(g, y);
            if (!head) X = fma(pr, Rv[j], X);
          } else {
            yh = mul(g, add(Rv[j], yh));
            Rv[j] = yh;
            X = fma(pr, yh, X);
            pr = mul(pr, g);
            // keep the accumulation in slot order (not batched up over the sweep)
            asm volatile("" : "+v"(X.re), "+v"(X.im), "+v"(pr.re), "+v"(pr.im) : "v"(yh.re));
          }
          if (j + PF < M) gq[j % PF] = G2_at(j + PF, yh);
        }
      }
    }
    // ---- 2x2 interface block: v_k = i00 r_k + i01 r_{k+1}, v_{k+1} = i10 r_k + i11 r_{k+1}
    //      (inverse entries times nbmh, r divided by nbmh)
    if (head) xch[2 * cw + (bot ? 1 : 0)] = Rv[M - 1];
    __syncthreads();
    if (head) {
      Rv[M - 1] = fma(hrec(4), Rv[M - 1], mul(hrec(5), xch[2 * cw + (bot ? 0 : 1)]));
      X = fma(pr, Rv[M - 1], X);
    }
    const D xin = scan_excl<false, FRESH>(head ? zero<double>() : tp, X, t, L, tot);

    // ---- phase 3: back substitution with the exact carry, written to the column
    //      buffer (the input was last read before the interface barrier; zero
    //      slots and idle lanes write guard rows only)
    if constexpr (GREG) {
      {
        D x = xin;
        C<S>* p = buf + cw * CS + GA + row0 + dir * (M - 1);
        #pragma unroll
        for (int jj = 0; jj < M; ++jj) {
          const int j = M - 1 - jj;
          if (j == M - 1 && head) x = Rv[j];
          else x = fma(Gv[j], x, Rv[j]);
          *p = from_d<S>(x);
          p -= dir;
        }
      }
    } else {
      auto phase3 = [&](auto tab) {
        D x = xin;
        D gq[PF];
        #pragma unroll
        for (int jj = 0; jj < PF; ++jj)
          if (jj < M) gq[jj] = G_at(tab, M - 1 - jj, x);
        C<S>* p = buf + cw * CS + GA + row0 + dir * (M - 1);
        #pragma unroll
        for (int jj = 0; jj < M; ++jj) {
          const int j = M - 1 - jj;
          const D g = gq[jj % PF];
          if (j == M - 1 && head) x = Rv[j];
          else x = fma(g, x, Rv[j]);
          *p = from_d<S>(x);
          p -= dir;
          if (jj + PF < M) gq[jj % PF] = G_at(tab, j - PF, x);
        }
      };
      if (wtab)
        phase3(std::true_type{});
      else
        phase3(std::false_type{});
    }
    __syncthreads();
  };
  // every step of the call (MULTI), else this one
  if constexpr (MULTI) {
    for (int kk = 0; kk < d.nsteps; ++kk) step();
  } else {
    step();
  }
  {
    // the staging addresses are recomputed here rather than kept live
    int lane_r = lane;
    asm volatile("" : "+v"(lane_r));
    C<S>* __restrict__ out = dst + (size_t)m0 * N;
    if (pairs) {
      using F4 = float __attribute__((ext_vector_type(4)));
      constexpr int MP = (M + 1) / 2;
      __attribute__((address_space(1))) F4* o4 = (__attribute__((address_space(1))) F4*)out;
      #pragma unroll
      for (int q = 0; q < MP; ++q) {
        const int e = 2 * (lane_r + q * kPassAThreads);
        if (e < span) {
          const int c = cpw == 1 ? 0 : int((float(e) + 0.5f) * invN);
          const int idx = c * CS + GA + (e - c * N);
          const C<S> x0 = buf[idx], x1 = buf[idx + 1];
          F4 w;
          w.x = float(x0.re);
          w.y = float(x0.im);
          w.z = float(x1.re);
          w.w = float(x1.im);
          o4[e >> 1] = w;
        }
      }
    } else if (cpw == 1) {
      #pragma unroll
      for (int q = 0; q < M; ++q) {
        const int e = lane_r + q * kPassAThreads;
        if (e < span) gstore(out, unsigned(e), buf[GA + e]);
      }
    } else if (N >= kPassAThreads) {
      int r = lane_r, idx = GA + lane_r;
      #pragma unroll
      for (int q = 0; q < M; ++q) {
        const int e = lane_r + q * kPassAThreads;
        if (e < span) gstore(out, unsigned(e), buf[idx]);
        r += kPassAThreads;
        idx += kPassAThreads;
        if (r >= N) {
          r -= N;
          idx += 2 * GA;
        }
      }
    } else {
      #pragma unroll
      for (int q = 0; q < M; ++q) {
        const int e = lane_r + q * kPassAThreads;
        if (e < span) {
          const int c = int((float(e) + 0.5f) * invN);
          gstore(out, unsigned(e), buf[c * CS + GA + (e - c * N)]);
        }
      }
    }
  }
}

#define PE3D_PASS_A_ATTR __launch_bounds__(kPassAThreads)

template <typename S, int M>
__global__ PE3D_PASS_A_ATTR void pass_a_single(ProbDesc d, int koff) {
  extern __shared__ __align__(16) unsigned char smem_a[];
  pass_a_body<S, M>(d, blockIdx.x, koff, smem_a);
}

template <typename S, int M>
__global__ PE3D_PASS_A_ATTR void pass_a_multi(ProbDesc d) {
  extern __shared__ __align__(16) unsigned char smem_a[];
  pass_a_body<S, M, true>(d, blockIdx.x, 0, smem_a);
}

// Batched launch over work items of problems with any M: each workgroup takes
// the body specialised for its problem's M (a uniform branch).
template <typename S>
__global__ PE3D_PASS_A_ATTR __attribute__((amdgpu_waves_per_eu(sizeof(S) == 8 ? 2 : 3))) void pass_a_batch(const ProbDesc* __restrict__ descs,
                                              const WorkItem* __restrict__ items, int koff) {
  extern __shared__ __align__(16) unsigned char smem_a[];
  const WorkItem it = items[blockIdx.x];
  const ProbDesc d = descs[it.prob];
  switch (d.ma) {
    case 3: pass_a_body<S, 3>(d, it.tile, koff, smem_a); break;
    case 5: pass_a_body<S, 5>(d, it.tile, koff, smem_a); break;
    case 7: pass_a_body<S, 7>(d, it.tile, koff, smem_a); break;
    case 9: pass_a_body<S, 9>(d, it.tile, koff, smem_a); break;
    case 11: pass_a_body<S, 11>(d, it.tile, koff, smem_a); break;
    case 13: pass_a_body<S, 13>(d, it.tile, koff, smem_a); break;
    case 15: pass_a_body<S, 15>(d, it.tile, koff, smem_a); break;
    default: pass_a_body<S, 17>(d, it.tile, koff, smem_a); break;
  }
}

// ============================================================== pass B
// A workgroup of 512 lanes owns TD = 512/W consecutive depths of one problem.
// Every depth line of NT azimuths is cut into NC <= W chunks of M nodes (the
// last one may be shorter); lane = depth * W + chunk, so the chunks of one
// line are W consecutive lanes of one wavefront and every chunk scan is a
// wavefront shuffle scan.  The tile is staged through LDS (global loads and
// stores coalesced along depth); in LDS a chunk of one depth is contiguous,
// at c * CST + dl * DS with odd strides DS >= M and CST = TD DS + 1, so the
// lanes of a line read distinct banks and slot offsets are immediates.
struct BConst {
  D rho;      // root of s rho^2 - (1+2s) rho + s = 0 inside the unit circle
  D cs;       // rho / s = 1 / c, the scale of the factored operator
  D rinv;     // 1 / rho (sector)
  D rL;       // rho^lastlen
  D winv;     // 1 / (1 - rho^NT)      (periodic closure)
  D sinv;     // 1 / (1 - rho^(2NT+2)) (sector first-row correction)
  D rM;       // rho^M, chunk multiplier of the scans
  double s1;  // sigma of the next step (its azimuth factor is applied on store)
};

constexpr int kPassBPow = 64;  // sPowC / sPowS entries: chunks <= 64

__host__ __device__ constexpr int pass_b_ds(int M) { return M | 1; }
__host__ __device__ constexpr int pass_b_tile_elems(int W, int M, int nthr = kPassBThreads) {
  return W * ((nthr / W) * pass_b_ds(M) + 1);
}
__host__ __device__ constexpr int pass_b_lds_bytes(int esz, int W, int M, int nthr = kPassBThreads) {
  return ((pass_b_tile_elems(W, M, nthr) * esz + 15) & ~15) + int(sizeof(BConst)) + 2 * kPassBPow * 16;
}

// EQ: every chunk holds exactly M nodes (NT = W*M, M = MM); otherwise M =
// d.mb <= MM at run time and the last chunk holds NT - (NC-1) M nodes.
// NTHR: lanes of the workgroup (512; 256 in the persistent batched kernel,
// whose tiles then hold half the depths).
template <typename S, int MM, bool EQ, int NTHR = kPassBThreads>
__device__ __forceinline__ void pass_b_body(const ProbDesc& d, int tile, int koff, unsigned char* smem) {
  static_assert(NTHR == 256 || NTHR == 512, "pass B workgroups hold 256 or 512 lanes");
  const int tid = lane_id<NTHR != kPassBThreads>();
  const int W = d.wb;
  const int lgW = 31 - __clz(W);
  const int TD = NTHR >> lgW;
  const int lgTD = (NTHR == 512 ? 9 : 8) - lgW;
  const int M = EQ ? MM : d.mb;
  const int DS = EQ ? pass_b_ds(MM) : pass_b_ds(M);
  const int N = d.nz, NT = d.nth;
  const int NC = EQ ? W : d.nc;
  const int CST = TD * DS + 1;
  const int z0 = tile * TD;
  C<S>* tl = reinterpret_cast<C<S>*>(smem);
  BConst* K = reinterpret_cast<BConst*>(smem + ((W * CST * int(sizeof(C<S>)) + 15) & ~15));
  D* sPowC = reinterpret_cast<D*>(K + 1);  // rho^(M c)
  D* sPowS = sPowC + kPassBPow;            // rho^(2 NT - M c) (sector)
  const long long j = *d.jdev + koff;
  const bool last = (koff == d.nsteps - 1);
  const bool periodic = d.periodic != 0;
  const C<S>* __restrict__ src = (const C<S>*)d.scr;
  C<S>* __restrict__ dst = (C<S>*)(last ? d.u : d.scr);
  const float invM = 1.0f / float(M);
  auto lidx = [&](int m, int dl) {  // LDS index of azimuth m, depth dl
    const int c = EQ ? m / MM : int((float(m) + 0.5f) * invM);
    return c * CST + dl * DS + (m - c * M);
  };

  // ---- stage the tile: thread tid loads chunk tid / TD of depth z0 + tid % TD
  //      (W chunks x TD depths = NTHR threads); all loads issued before the
  //      first LDS write
  const int sdl = tid & (TD - 1);
  const int sc0 = tid >> lgTD;
  const int szc = min(z0 + sdl, N - 1);
  const bool szok = z0 + sdl < N;
  const int slen = EQ ? MM : (sc0 < NC - 1 ? M : (sc0 == NC - 1 ? NT - (NC - 1) * M : 0));
  {
    const unsigned o0 = unsigned(sc0 * M * N + szc);
    C<S> v[MM];
    // the staging loads issue at raised wave priority, so that every
    // wavefront's loads are in flight before the arithmetic of others
    __builtin_amdgcn_s_setprio(2);
    #pragma unroll
    for (int i = 0; i < MM; ++i)
      if (EQ || i < slen) v[i] = gload(src, o0 + unsigned(i * N));
    __builtin_amdgcn_s_setprio(0);
    // the step constants are computed while the loads are in flight
    // ---- step constants (wavefront 0; read by all after the staging barrier)
    if (tid < 64) {
      const double sg = sigma_of(d, j);
      const D rho = rho_of(sg);
      const int lastlen = NT - (NC - 1) * M;
      const D rM = cpow(rho, M);
      sPowC[tid] = cpow(rM, tid);
      if (!periodic) sPowS[tid] = cpow(rho, 2 * (long long)NT - (long long)M * tid);
      if (tid == 0) {
        K->rho = rho;
        K->cs = rho_over_s(sg);
        K->rinv = cdiv(one<double>(), rho);
        K->rL = cpow(rho, lastlen);
        const D rN = cpow(rho, NT);
        K->winv = cdiv(one<double>(), mk<double>(1.0 - rN.re, -rN.im));
        const D r2 = cpow(rho, 2 * (long long)NT + 2);
        K->sinv = cdiv(one<double>(), mk<double>(1.0 - r2.re, -r2.im));
        K->rM = rM;
        K->s1 = sigma_of(d, j + 1);
      }
    }
    C<S>* Ts = tl + sc0 * CST + sdl * DS;
    #pragma unroll
    for (int i = 0; i < MM; ++i)
      if (EQ || i < slen) Ts[i] = szok ? v[i] : zero<S>();
  }
  __syncthreads();

  // ---- lane role
  const int c = tid & (W - 1);
  const int dl = tid >> lgW;
  const int seg = tid & ~(W - 1) & 63;  // first lane of this line within the wavefront
  const int len = EQ ? MM : (c < NC - 1 ? M : (c == NC - 1 ? NT - (NC - 1) * M : 0));
  const D rho = K->rho;
  C<S>* T = tl + c * CST + dl * DS;
  auto vat = [&](int i) { return to_d(T[i]); };

  // ---- forward recurrence y_m = v_m + rho y_{m-1}: end value with zero carry
  D xr[MM];
  D E = zero<double>();
  #pragma unroll
  for (int i = 0; i < MM; ++i) {
    if (EQ || i < len) {
      xr[i] = vat(i);
      E = fma(rho, E, xr[i]);
      __builtin_amdgcn_sched_barrier(0);  // keep each LDS read next to its use
    }
  }
  // ---- forward chunk carries: inclusive scan over chunks 0..NC-2 (length M)
  // (inside rows of 16 lanes by DPP row shifts, multipliers rho^(M dd); then
  // from lane 15 / lane 31 by DPP row broadcasts, multiplier rho^(M dist))
  const int h = tid & 63;
  const int pr = h & 15;
  {
    D Sv = (c < NC - 1) ? E : zero<double>();
    D lv = K->rM;  // rho^(M dd)
    if (W > 1) {
      const D up = dpp<0x111>(Sv);
      if (c >= 1 && pr >= 1) Sv = fma(lv, up, Sv);
      lv = mul(lv, lv);
    }
    if (W > 2) {
      const D up = dpp<0x112>(Sv);
      if (c >= 2 && pr >= 2) Sv = fma(lv, up, Sv);
      lv = mul(lv, lv);
    }
    if (W > 4) {
      const D up = dpp<0x114>(Sv);
      if (c >= 4 && pr >= 4) Sv = fma(lv, up, Sv);
      lv = mul(lv, lv);
    }
    if (W > 8) {
      const D up = dpp<0x118>(Sv);
      if (c >= 8 && pr >= 8) Sv = fma(lv, up, Sv);
    }
    if (W > 16) {
      const D up = dpp<0x142, 0xA>(Sv);
      if (h & 16) Sv = fma(sPowC[pr + 1], up, Sv);
    }
    if (W > 32) {
      const D up = dpp<0x143, 0xC>(Sv);
      if (h & 32) Sv = fma(sPowC[(h & 31) + 1], up, Sv);
    }
    D y0 = zero<double>();  // y_{-1} = y_{NT-1} (periodic)
    if (periodic) {
      const D Sl = (NC >= 2) ? shfl_idx(Sv, seg + NC - 2, 64) : zero<double>();
      const D El = shfl_idx(E, seg + NC - 1, 64);
      y0 = mul(fma(K->rL, Sl, El), K->winv);
    }
    D prev = dpp<0x138>(Sv);
    if (c == 0) prev = zero<double>();
    D y = fma(sPowC[c < kPassBPow ? c : 0], y0, prev);
    #pragma unroll
    for (int i = 0; i < MM; ++i)
      if (EQ || i < len) {
        y = fma(rho, y, xr[i]);
        xr[i] = y;
      }
  }
  // ---- backward recurrence x_m = y_m + rho x_{m+1}: end value with zero carry,
  //      carries scanned downward over the chunks
  {
    D X = zero<double>();
    #pragma unroll
    for (int i = MM - 1; i >= 0; --i)
      if (EQ || i < len) X = fma(rho, X, xr[i]);
    D Sv = (c < NC) ? X : zero<double>();
    D lv = K->rM;
    if (W > 1) {
      const D dn = dpp<0x101>(Sv);
      if (c + 1 < W && pr + 1 < 16) Sv = fma(lv, dn, Sv);
      lv = mul(lv, lv);
    }
    if (W > 2) {
      const D dn = dpp<0x102>(Sv);
      if (c + 2 < W && pr + 2 < 16) Sv = fma(lv, dn, Sv);
      lv = mul(lv, lv);
    }
    if (W > 4) {
      const D dn = dpp<0x104>(Sv);
      if (c + 4 < W && pr + 4 < 16) Sv = fma(lv, dn, Sv);
      lv = mul(lv, lv);
    }
    if (W > 8) {
      const D dn = dpp<0x108>(Sv);
      if (c + 8 < W && pr + 8 < 16) Sv = fma(lv, dn, Sv);
    }
    if (W > 16) {  // from the first lane of the next row
      const D dn = shfl_idx(Sv, (h | 15) + 1, 64);
      if ((h & 16) == 0) Sv = fma(sPowC[16 - pr], dn, Sv);
    }
    if (W > 32) {  // from lane 32
      const D dn = shfl_idx(Sv, 32, 64);
      if ((h & 32) == 0) Sv = fma(sPowC[32 - h], dn, Sv);
    }
    const D xN = periodic ? mul(shfl_idx(Sv, seg, 64), K->winv) : zero<double>();  // x_NT = x_0
    D nxt = dpp<0x130>(Sv);
    D x;
    if (c >= NC - 1) x = xN;
    else x = fma(mul(sPowC[NC - 2 - c], K->rL), xN, nxt);
    #pragma unroll
    for (int i = MM - 1; i >= 0; --i)
      if (EQ || i < len) {
        x = fma(rho, x, xr[i]);
        xr[i] = x;
      }
  }
  // ---- u = (rho/s) x, written to the tile rounded to S (the next step
  //      starts from u as stored, exactly as a new march call would); sector:
  //      rank-one correction of the first row,
  //      x_m -= Kc (rho^m - rho^{2NT-m}),  Kc = rho^2 x_0 / (1 - rho^{2NT+2})
  const D cs = K->cs;
  if (periodic) {
    #pragma unroll
    for (int i = 0; i < MM; ++i)
      if (EQ || i < len) {
        T[i] = from_d<S>(mul(cs, xr[i]));
        __builtin_amdgcn_sched_barrier(0);
      }
  } else {
    const D x0 = shfl_idx(xr[0], seg, 64);
    const D Kc = mul(mul(rho, rho), mul(x0, K->sinv));
    D pa = mul(Kc, sPowC[c < kPassBPow ? c : 0]);
    D pb = mul(Kc, sPowS[c < kPassBPow ? c : 0]);
    const D rinv = K->rinv;
    #pragma unroll
    for (int i = 0; i < MM; ++i)
      if (EQ || i < len) {
        const D x = sub(xr[i], sub(pa, pb));
        pa = mul(pa, rho);
        pb = mul(pb, rinv);
        T[i] = from_d<S>(mul(cs, x));
        __builtin_amdgcn_sched_barrier(0);
      }
  }
  // ---- next step's azimuth factor w = u + s_{j+1} D_theta u over the tile.
  //      All lanes of a line are in one wavefront: the chunk-edge neighbours
  //      are read before any lane of the line writes, and each lane then
  //      reads slot i+1 before writing slot i.
  if (!last) {
    D ul, ur;
    if (c > 0) ul = to_d(T[M - 1 - CST]);
    else if (periodic) ul = to_d(tl[lidx(NT - 1, dl)]);
    else ul = zero<double>();
    if (c < NC - 1) ur = to_d(T[CST]);
    else ur = periodic ? to_d(tl[dl * DS]) : zero<double>();
    const double s1 = K->s1;
    D a = ul, b = vat(0);
    #pragma unroll
    for (int i = 0; i < MM; ++i)
      if (EQ || i < len) {
        const D nx = (EQ ? (i + 1 < MM) : (i + 1 < len)) ? vat(i + 1 < MM ? i + 1 : i) : ur;
        const D dd = sub(add(a, nx), scl(2.0, b));
        T[i] = from_d<S>(mk<double>(b.re - s1 * dd.im, b.im + s1 * dd.re));
        a = b;
        b = nx;
        __builtin_amdgcn_sched_barrier(0);
      }
  }
  __syncthreads();
  // ---- store the tile (coalesced along depth)
  if (szok) {
    int sc0r = sc0;
    asm volatile("" : "+v"(sc0r));  // recomputed here rather than kept live through the solve
    const unsigned o0 = unsigned(sc0r * M * N + szc);
    const C<S>* Ts = tl + sc0r * CST + sdl * DS;
    #pragma unroll
    for (int i = 0; i < MM; ++i)
      if (EQ || i < slen) gstore(dst, o0 + unsigned(i * N), Ts[i]);
  }
}

// ============================================================== pass B by cyclic reduction
// Parallel cyclic reduction of [I - s D_theta] u = v, the alternative to the
// chunked recurrences above.  The equation at azimuth m is
//   b u_m + a (u_{m-d} + u_{m+d}) = v_m,   b = 1 + 2s, a = -s, d = 1;
// adding k = -a/b times the equations at m - d and m + d removes u_{m-d} and
// u_{m+d} and leaves the same form at distance 2d:
//   v_m <- v_m + k (v_{m-d} + v_{m+d}),  a <- k a,  b <- b + 2 k a  (old a).
// The coefficients are the same at every azimuth and depth (the operator is
// circulant and does not depend on z), so each level is one complex
// multiplier for the whole tile.  |a/b| < 1/2 (diagonal dominance) and
// q = a/b maps to q^2/(1 - 2 q^2): the levels stop once |a/b| <= 2^-60, where
// the remaining coupling is below FP64 resolution (about 12 levels at sigma
// = 600, 3-5 far from the source), and u_m = v_m / b.  Periodic lines wrap
// with period Ntheta; a sector (zero ghosts at m = -1 and m = Ntheta) is the
// restriction of the periodic line of period 2 Ntheta + 2 whose data are odd
// about the ghosts (v_{Ntheta+k} = -v_{Ntheta-k}, v_{-1} = 0), so a node
// outside 0..Ntheta-1 reads the mirrored node with its sign flipped.
// A workgroup's tile of td depths x Ntheta azimuths (td * Ntheta <=
// kPcrNodes) sits in LDS as FP64 complex, node m * td + dl, so consecutive
// threads load consecutive depths.  As in the chunked kernel the field is
// stored rounded to S and the next step's azimuth factor is applied to the
// rounded values before the store.
__host__ __device__ constexpr int pass_b_pcr_lds_bytes() { return kPcrNodes * 16; }

template <typename S, int NTHR = kPassBThreads>
__device__ __forceinline__ void pass_b_pcr_body(const ProbDesc& d, int tile, int koff, unsigned char* smem) {
  constexpr int NPT = kPcrNodes / NTHR;  // nodes per thread
  const int tid = lane_id<NTHR != kPassBThreads>();
  const int NT = d.nth, N = d.nz, TD = d.td;
  const int lgTD = 31 - __clz(TD);
  const int z0 = tile * TD;
  const int nn = TD * NT;
  D* V = reinterpret_cast<D*>(smem);
  const long long j = *d.jdev + koff;
  const bool last = (koff == d.nsteps - 1);
  const bool periodic = d.periodic != 0;
  const C<S>* __restrict__ src = (const C<S>*)d.scr;
  C<S>* __restrict__ dst = (C<S>*)(last ? d.u : d.scr);

  // ---- stage the tile (all loads issued first), FP64 in LDS; depths past
  //      the end of the column are zero and never stored
  {
    C<S> v[NPT];
    __builtin_amdgcn_s_setprio(2);
    #pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int n = tid + q * NTHR;
      const int m = n >> lgTD, z = z0 + (n & (TD - 1));
      v[q] = (n < nn && z < N) ? gload(src, unsigned(m * N + z)) : zero<S>();
    }
    __builtin_amdgcn_s_setprio(0);
    #pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int n = tid + q * NTHR;
      if (n < nn) V[n] = to_d(v[q]);
    }
  }
  const double sg = sigma_of(d, j);  // s = i sg
  D b = mk<double>(1.0, 2.0 * sg);
  D a = mk<double>(0.0, -sg);
  const int P = periodic ? NT : 2 * NT + 2;  // period of the (extended) line
  // node value at azimuth index i in [0, P) of the extended line, depth dl
  auto at = [&](int i, int dl) {
    if (periodic || i < NT) return V[(i << lgTD) + dl];
    if (i == NT || i == P - 1) return zero<double>();
    const D w = V[((2 * NT - i) << lgTD) + dl];
    return mk<double>(-w.re, -w.im);
  };
  __syncthreads();

  // ---- levels (uniform loop: the same a, b in every thread)
  int dist = 1 % P;  // level distance modulo the period
  for (int lvl = 0; lvl < 64; ++lvl) {
    const double qa = a.re * a.re + a.im * a.im, qb = b.re * b.re + b.im * b.im;
    if (!(qa > 0x1p-120 * qb)) break;
    const D k = cdiv(mk<double>(-a.re, -a.im), b);
    D nv[NPT];
    #pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int n = tid + q * NTHR;
      if (n < nn) {
        const int m = n >> lgTD, dl = n & (TD - 1);
        int lo = m - dist, hi = m + dist;
        if (lo < 0) lo += P;
        if (hi >= P) hi -= P;
        nv[q] = fma(k, add(at(lo, dl), at(hi, dl)), V[n]);
      }
    }
    __syncthreads();
    #pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int n = tid + q * NTHR;
      if (n < nn) V[n] = nv[q];
    }
    __syncthreads();
    b = fma(scl(2.0, k), a, b);
    a = mul(k, a);
    dist = (2 * dist) % P;
  }

  // ---- u = v / b rounded to S; the next step's factor w = u + s_{j+1} D_theta u
  //      from the rounded u (zero ghosts for a sector)
  const D ib = cdiv(one<double>(), b);
  C<S> u[NPT];
  #pragma unroll
  for (int q = 0; q < NPT; ++q) {
    const int n = tid + q * NTHR;
    if (n < nn) u[q] = from_d<S>(mul(V[n], ib));
  }
  if (!last) {
    __syncthreads();
    #pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int n = tid + q * NTHR;
      if (n < nn) V[n] = to_d(u[q]);
    }
    __syncthreads();
    const double s1 = sigma_of(d, j + 1);
    #pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int n = tid + q * NTHR;
      if (n < nn) {
        const int m = n >> lgTD, dl = n & (TD - 1);
        D ul = zero<double>(), ur = zero<double>();
        if (m > 0) ul = V[n - TD];
        else if (periodic) ul = V[((NT - 1) << lgTD) + dl];
        if (m < NT - 1) ur = V[n + TD];
        else if (periodic) ur = V[dl];
        const D c = V[n];
        const D dd = sub(add(ul, ur), scl(2.0, c));
        u[q] = from_d<S>(mk<double>(c.re - s1 * dd.im, c.im + s1 * dd.re));
      }
    }
  }
  #pragma unroll
  for (int q = 0; q < NPT; ++q) {
    const int n = tid + q * NTHR;
    const int m = n >> lgTD, z = z0 + (n & (TD - 1));
    if (n < nn && z < N) gstore(dst, unsigned(m * N + z), u[q]);
  }
}

// two workgroups per CU: one stages or stores its tile while the other computes
#define PE3D_PASS_B_OCC __attribute__((amdgpu_waves_per_eu(4, 4)))

template <typename S, int MM, bool EQ>
__global__ __launch_bounds__(kPassBThreads) PE3D_PASS_B_OCC void pass_b_single(ProbDesc d, int koff) {
  extern __shared__ __align__(16) unsigned char smem_b[];
  const int b = blockIdx.x;
  const int tile = pass_b_pairs(d.td, int(sizeof(C<S>))) ? pass_b_paired_tile(b, d.ntile_b) : b;
  pass_b_body<S, MM, EQ>(d, tile, koff, smem_b);
  medium_update_next(d, tile, koff);
}

// Batched launch over work items of problems of any class (a uniform branch).
template <typename S>
__global__ __launch_bounds__(kPassBThreads) PE3D_PASS_B_OCC void pass_b_batch(const ProbDesc* __restrict__ descs,
                                                              const WorkItem* __restrict__ items,
                                                              int koff) {
  extern __shared__ __align__(16) unsigned char smem_b[];
  const WorkItem it = items[blockIdx.x];
  const ProbDesc d = descs[it.prob];
  switch (d.bcls) {
    case 9: pass_b_body<S, 9, true>(d, it.tile, koff, smem_b); break;
    case 10: pass_b_body<S, 10, true>(d, it.tile, koff, smem_b); break;
    case 11: pass_b_body<S, 11, true>(d, it.tile, koff, smem_b); break;
    case 12: pass_b_body<S, 12, true>(d, it.tile, koff, smem_b); break;
    case 13: pass_b_body<S, 13, true>(d, it.tile, koff, smem_b); break;
    case 14: pass_b_body<S, 14, true>(d, it.tile, koff, smem_b); break;
    case 15: pass_b_body<S, 15, true>(d, it.tile, koff, smem_b); break;
    case 16: pass_b_body<S, 16, true>(d, it.tile, koff, smem_b); break;
    case kPcrClass: pass_b_pcr_body<S>(d, it.tile, koff, smem_b); break;
    default: pass_b_body<S, 16, false>(d, it.tile, koff, smem_b); break;
  }
}

template <typename S>
__global__ __launch_bounds__(kPassBThreads) void pass_b_pcr_single(ProbDesc d, int koff) {
  extern __shared__ __align__(16) unsigned char smem_b[];
  const int b = blockIdx.x;
  const int tile = pass_b_pairs(d.td, int(sizeof(C<S>))) ? pass_b_paired_tile(b, d.ntile_b) : b;
  pass_b_pcr_body<S>(d, tile, koff, smem_b);
  medium_update_next(d, tile, koff);
}

// ============================================================== persistent batched march
// One launch runs every step of a batched march (the paper's loop over
// frequencies, each marched through its range steps, carried onto one
// device): the workgroups, as many as fit on the device at once, take tasks
// from a list in list order, one atomic increment per task.  A task is nsub
// consecutive depth-pass tiles (spans of columns) or azimuth-pass tiles (of
// 256 lanes) of one problem at one step.  A problem's
// tasks enter the list step by step, the depth pass before the azimuth pass,
// and each task carries the number of the problem's tasks that must have
// finished before it may start: every task of the step's depth pass (for the
// azimuth pass), or of the previous step (for the depth pass).  A workgroup
// only ever waits for tasks that precede its own in the list, which were
// taken by workgroups already running; a workgroup publishes its finished
// tasks in small batches, but always before it waits and before it leaves,
// so every finished task is published within a few tasks of its workgroup
// and every wait ends without any assumption on how many workgroups are
// resident.  Each wait is also bounded
// in time: when it runs out, the workgroup counts the timeout
// (g_wait_timeouts), raises the launch's abort flag and leaves; workgroups
// that are waiting see the flag and leave too, so the kernel always ends
// (the fields of that call are then undefined).  Ordering: a task's stores
// are released at device scope before its problem's counter counts it,
// and a waiting workgroup acquires the counter at device scope before any of
// its lanes reads the field (the L2 caches of the XCDs are not coherent with
// each other without these fences).
__device__ unsigned long long g_wait_timeouts;

template <typename S>
__device__ __forceinline__ void persist_pass_a(const ProbDesc& d, int tile, int koff, unsigned char* smem) {
  switch (d.ma) {
    case 3: pass_a_body<S, 3, false, true>(d, tile, koff, smem); break;
    case 5: pass_a_body<S, 5, false, true>(d, tile, koff, smem); break;
    case 7: pass_a_body<S, 7, false, true>(d, tile, koff, smem); break;
    case 9: pass_a_body<S, 9, false, true>(d, tile, koff, smem); break;
    case 11: pass_a_body<S, 11, false, true>(d, tile, koff, smem); break;
    case 13: pass_a_body<S, 13, false, true>(d, tile, koff, smem); break;
    case 15: pass_a_body<S, 15, false, true>(d, tile, koff, smem); break;
    default: pass_a_body<S, 17, false, true>(d, tile, koff, smem); break;
  }
}

template <typename S>
__device__ __forceinline__ void persist_pass_b(const ProbDesc& d, int tile, int koff, unsigned char* smem) {
  switch (d.bcls) {
    case 9: pass_b_body<S, 9, true, kPersistThreads>(d, tile, koff, smem); break;
    case 10: pass_b_body<S, 10, true, kPersistThreads>(d, tile, koff, smem); break;
    case 11: pass_b_body<S, 11, true, kPersistThreads>(d, tile, koff, smem); break;
    case 12: pass_b_body<S, 12, true, kPersistThreads>(d, tile, koff, smem); break;
    case 13: pass_b_body<S, 13, true, kPersistThreads>(d, tile, koff, smem); break;
    case 14: pass_b_body<S, 14, true, kPersistThreads>(d, tile, koff, smem); break;
    case 15: pass_b_body<S, 15, true, kPersistThreads>(d, tile, koff, smem); break;
    case 16: pass_b_body<S, 16, true, kPersistThreads>(d, tile, koff, smem); break;
    case kPcrClass: pass_b_pcr_body<S, kPersistThreads>(d, tile, koff, smem); break;
    default: pass_b_body<S, 16, false, kPersistThreads>(d, tile, koff, smem); break;
  }
}

// ctl[0]: next task of the list, ctl[S]: abort flag; done[S p]: finished
// tasks of problem p (S = kPersistCounterStride: each word on a cache line of
// its own; all zero at launch).  wait_ticks: longest wait, in ticks of the
// device's constant-rate clock.
// Every branch around the barriers is uniform per wavefront (a scalar
// condition): the first wavefront takes and waits for the task with all of
// its lanes (lane 0 adds 1, the others add 0; the values it waits on are
// made scalar), and the other wavefronts wait at the barrier.  With a branch
// on a per-lane condition (thread 0 alone) the compiler may turn the loop
// into one in which the wavefront's other lanes go round the barrier and
// re-read the task index before lane 0 has taken the next task.
template <typename S>
__global__ __launch_bounds__(kPersistThreads) __attribute__((amdgpu_waves_per_eu(sizeof(S) == 8 ? 2 : 3)))
void march_persist(const ProbDesc* __restrict__ descs, const PTask* __restrict__ tasks, int ntasks, int* ctl,
                   int* done, long long wait_ticks) {
  extern __shared__ __align__(16) unsigned char smem_p[];
  __shared__ int s_task;
  const bool first_wave = __builtin_amdgcn_readfirstlane(threadIdx.x) < 64;  // uniform per wavefront
  const int one = (threadIdx.x & 63) == 0 ? 1 : 0;                           // lane 0 of the wavefront
  // finished tasks not yet published (first wavefront, scalar registers):
  // pend_n[i] tasks of problem pend_p[i], i < npend; published together after
  // one device-scope release
  constexpr int KP = kPersistPublishEvery;
  int pend_p[KP], pend_n[KP];
  int npend = 0, nfin = 0;
  auto publish = [&] {
    if (npend) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      #pragma unroll
      for (int i = 0; i < KP; ++i)
        if (i < npend)
          __hip_atomic_fetch_add(done + pend_p[i] * kPersistCounterStride, pend_n[i] * one, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
    }
    npend = 0;
    nfin = 0;
  };
  auto finished = [&](int prob) {
    bool found = false;
    #pragma unroll
    for (int i = 0; i < KP; ++i)
      if (i < npend && pend_p[i] == prob) {
        ++pend_n[i];
        found = true;
      }
    if (!found) {
      #pragma unroll
      for (int i = 0; i < KP; ++i)
        if (i == npend) {
          pend_p[i] = prob;
          pend_n[i] = 1;
        }
      ++npend;
    }
    if (++nfin >= KP) publish();
  };
  for (;;) {
    if (first_wave) {
      int t = __builtin_amdgcn_readfirstlane(
          __hip_atomic_fetch_add(&ctl[0], one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (t < ntasks) {
        const int prob = tasks[t].prob, need = tasks[t].need;
        int* const cnt = done + prob * kPersistCounterStride;
        auto count = [&] {
          return __builtin_amdgcn_readfirstlane(__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        };
        if (count() < need) {
          publish();  // never wait while holding unpublished tasks
          const long long t0 = (long long)wall_clock64();
          while (count() < need) {
            if (__builtin_amdgcn_readfirstlane(
                    __hip_atomic_load(&ctl[kPersistCounterStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0) {
              t = ntasks;
              break;
            }
            if ((long long)wall_clock64() - t0 > wait_ticks) {
              __hip_atomic_store(&ctl[kPersistCounterStride], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              atomicAdd(&g_wait_timeouts, (unsigned long long)one);
              t = ntasks;
              break;
            }
            __builtin_amdgcn_s_sleep(4);
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      if (t >= ntasks) publish();  // the workgroup leaves
      s_task = t;                  // every lane writes the same value
    }
    // (the first wavefront's acquire covers the CU: its caches are shared by
    // the workgroup's wavefronts, which read only after this barrier)
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(s_task);  // uniform: the task's data in scalar registers
    if (t >= ntasks) break;
    const PTask tk = tasks[t];
    const ProbDesc d = descs[tk.prob];
    // nsub consecutive tiles (the last task of a pass may reach past the
    // last tile)
    if (tk.kind == 0) {
      for (int q = 0; q < tk.nsub && tk.tile + q < d.ntile_a; ++q) {
        if (q) __syncthreads();  // the columns in LDS are free again
        persist_pass_a<S>(d, tk.tile + q, tk.k, smem_p);
      }
    } else {
      const int ntile = d.bcls == kPcrClass ? d.ntile_b : (d.nz + (kPersistThreads / d.wb) - 1) / (kPersistThreads / d.wb);
      for (int q = 0; q < tk.nsub && tk.tile + q < ntile; ++q) {
        if (q) __syncthreads();  // the tile in LDS is free again
        persist_pass_b<S>(d, tk.tile + q, tk.k, smem_p);
      }
    }
    // every wavefront waits for its stores to complete; the first wavefront
    // then counts the task as finished and publishes its finished tasks with
    // one device-scope release (a write-back of the XCD's L2, the kernel's
    // main overhead) once kPersistPublishEvery of them are pending, or
    // before it waits or leaves (LDS and s_task are then free for the next
    // task)
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (first_wave) finished(tk.prob);
  }
}

__global__ void fill_ints(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ============================================================== small kernels
// The medium of step j = the problem's step counter + koff for a problem with
// range rows (water nodes per column, one thread each; the water row),
// launched before every depth pass of a batched march, and of a single
// problem's march before the first step of a call and every step of an
// N x 2D march (later 3D steps take it from the single-problem azimuth pass;
// in the batched azimuth pass the same code cost 1.4 % on problems without
// range rows).
__global__ void medium_update_single(ProbDesc d, int koff) { medium_update(d, blockIdx.x, koff); }
__global__ void medium_update_batch(const ProbDesc* __restrict__ descs, const WorkItem* __restrict__ items,
                                    int koff) {
  const WorkItem it = items[blockIdx.x];
  medium_update(descs[it.prob], it.tile, koff);
}

__global__ void advance_kernel(long long* const* jdevs, const int* adds, int n, long long* js,
                               int add1) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (js) {
    if (i == 0) *js += add1;
  } else if (i < n) {
    *jdevs[i] += adds[i];
  }
}

template <typename R>
__global__ void starter_kernel(ProbDesc d, double zs, C<R>* u) {
  size_t n = (size_t)d.nz * d.nth;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n;
       idx += (size_t)gridDim.x * blockDim.x) {
    int l = int(idx % d.nz);
    double zz = d.dz * double(l + 1);
    double a = d.k0 * (zz - zs), b = d.k0 * (zz + zs);
    double val = sqrt(d.k0) * (exp(-0.5 * a * a) - exp(-0.5 * b * b));
    u[idx] = mk<R>(R(val), R(0));
  }
}

template <typename R>
__global__ void tl_kernel(ProbDesc d, const C<R>* u, float* tl) {
  size_t n = (size_t)d.nz * d.nth;
  double r = d.r0 + double(*d.jdev) * d.dr;
  double add = r > 0.0 ? 10.0 * log10(r) : 0.0;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n;
       idx += (size_t)gridDim.x * blockDim.x) {
    double a = hypot(double(u[idx].re), double(u[idx].im));
    tl[idx] = float(-20.0 * log10(a) + add);
  }
}

// p = u * H, H = H0^(1)(k0 r_j) evaluated on the host
template <typename R>
__global__ void scale_kernel(const C<R>* u, C<R>* p, size_t n, double hre, double him) {
  const D hh = mk<double>(hre, him);
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n;
       idx += (size_t)gridDim.x * blockDim.x)
    p[idx] = from_d<R>(mul(to_d(u[idx]), hh));
}

// ============================================================== launchers
// Raise a kernel's dynamic-LDS limit once per device (thread-safe).  The
// (device, kernel) pairs already done sit in a fixed table, so a launch
// never allocates; past its capacity the attribute is simply set again.
static hipError_t allow_lds(const void* fn, int bytes) {
  static std::mutex mu;
  constexpr int kCap = 512;
  static std::pair<int, const void*> done[kCap];
  static int ndone = 0;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  for (int i = 0; i < ndone; ++i)
    if (done[i].first == dev && done[i].second == fn) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess && ndone < kCap) done[ndone++] = {dev, fn};
  return e;
}

// Scratch field of pe3d_march_static: a file-scope device array, one copy on
// every GPU the library runs on, held until the process ends.  Host code
// never uses the array's name as an address (on the host it is a stand-in,
// not a device pointer): each device's address comes from
// hipGetSymbolAddress, called once per device with that device current.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch(void** ptr) {
  static std::mutex mu;
  constexpr int kMaxDevices = 64;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

template <typename S, int M>
static hipError_t run_a(const ProbDesc& d, int koff, int lds, hipStream_t st, bool multi) {
  // largest LDS any shape with this M can ask for: L = 4 lanes and nz = 3M - 1
  // (the host keeps nz <= (L-1) M - 1)
  constexpr int lds_max = pass_a_lds_bytes(int(sizeof(C<S>)), 4, 3 * M - 1, M);
  if (lds > lds_max) return hipErrorInvalidValue;
  const void* fn = multi ? reinterpret_cast<const void*>(&pass_a_multi<S, M>)
                         : reinterpret_cast<const void*>(&pass_a_single<S, M>);
  {
    const hipError_t e = allow_lds(fn, lds_max);
    if (e != hipSuccess) return e;
  }
  if (multi)
    hipLaunchKernelGGL((pass_a_multi<S, M>), dim3(d.ntile_a), dim3(kPassAThreads), lds, st, d);
  else
    hipLaunchKernelGGL((pass_a_single<S, M>), dim3(d.ntile_a), dim3(kPassAThreads), lds, st, d, koff);
  return hipGetLastError();
}

template <typename S>
static hipError_t run_a_batch(const ProbDesc* d_descs, const WorkItem* items, int nitems, int koff, int lds,
                              hipStream_t st) {
  constexpr int lds_max = pass_a_lds_bytes(int(sizeof(C<S>)), 4, 3 * 17 - 1, 17);
  if (lds > lds_max) return hipErrorInvalidValue;
  {
    const hipError_t e = allow_lds(reinterpret_cast<const void*>(&pass_a_batch<S>), lds_max);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((pass_a_batch<S>), dim3(nitems), dim3(kPassAThreads), lds, st, d_descs, items, koff);
  return hipGetLastError();
}

template <typename S, int MM, bool EQ>
static hipError_t run_b(const ProbDesc& d, int koff, int lds, hipStream_t st) {
  constexpr int lds_max = pass_b_lds_bytes(int(sizeof(C<S>)), 64, MM);  // W = 64 is the largest tile
  if (lds > lds_max) return hipErrorInvalidValue;
  {
    const hipError_t e = allow_lds(reinterpret_cast<const void*>(&pass_b_single<S, MM, EQ>), lds_max);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((pass_b_single<S, MM, EQ>), dim3(d.ntile_b), dim3(kPassBThreads), lds, st, d, koff);
  return hipGetLastError();
}

template <typename S>
static hipError_t run_b_pcr(const ProbDesc& d, int koff, int lds, hipStream_t st) {
  constexpr int lds_max = pass_b_pcr_lds_bytes();
  if (lds > lds_max) return hipErrorInvalidValue;
  {
    const hipError_t e = allow_lds(reinterpret_cast<const void*>(&pass_b_pcr_single<S>), lds_max);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((pass_b_pcr_single<S>), dim3(d.ntile_b), dim3(kPassBThreads), lds, st, d, koff);
  return hipGetLastError();
}

template <typename S>
static hipError_t run_b_batch(const ProbDesc* d_descs, const WorkItem* items, int nitems, int koff, int lds,
                              hipStream_t st) {
  constexpr int lds_max = pass_b_lds_bytes(int(sizeof(C<S>)), 64, 16);
  if (lds > lds_max) return hipErrorInvalidValue;
  {
    const hipError_t e = allow_lds(reinterpret_cast<const void*>(&pass_b_batch<S>), lds_max);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((pass_b_batch<S>), dim3(nitems), dim3(kPassBThreads), lds, st, d_descs, items, koff);
  return hipGetLastError();
}

int pass_a_lds(int prec, int L, int nz, int M) {
  return pass_a_lds_bytes(prec ? 16 : 8, L, nz, M);
}

template <typename S>
static hipError_t run_a_m(const ProbDesc& d, int koff, int lds, hipStream_t st, bool multi = false) {
  switch (d.ma) {
    case 3: return run_a<S, 3>(d, koff, lds, st, multi);
    case 5: return run_a<S, 5>(d, koff, lds, st, multi);
    case 7: return run_a<S, 7>(d, koff, lds, st, multi);
    case 9: return run_a<S, 9>(d, koff, lds, st, multi);
    case 11: return run_a<S, 11>(d, koff, lds, st, multi);
    case 13: return run_a<S, 13>(d, koff, lds, st, multi);
    case 15: return run_a<S, 15>(d, koff, lds, st, multi);
    case 17: return run_a<S, 17>(d, koff, lds, st, multi);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_pass_a_multi(int prec, const ProbDesc& d, int lds, hipStream_t st) {
  return prec == 0 ? run_a_m<float>(d, 0, lds, st, true) : run_a_m<double>(d, 0, lds, st, true);
}

hipError_t launch_pass_a(int prec, const ProbDesc* single, const ProbDesc* d_descs, const WorkItem* items,
                         int nitems, int koff, int lds, hipStream_t st) {
  if (single) return prec == 0 ? run_a_m<float>(*single, koff, lds, st) : run_a_m<double>(*single, koff, lds, st);
  return prec == 0 ? run_a_batch<float>(d_descs, items, nitems, koff, lds, st)
                   : run_a_batch<double>(d_descs, items, nitems, koff, lds, st);
}

int pass_b_lds(int prec, int W, int M, int nthr) {
  return W == 0 ? pass_b_pcr_lds_bytes() : pass_b_lds_bytes(prec ? 16 : 8, W, M, nthr);
}

// class: M in 9..16 for lines of exactly W*M azimuths, 0 for the general kernel
template <typename S>
static hipError_t run_b_cls(const ProbDesc& d, int koff, int lds, hipStream_t st) {
  switch (d.bcls) {
    case kPcrClass: return run_b_pcr<S>(d, koff, lds, st);
    case 0: return run_b<S, 16, false>(d, koff, lds, st);
    case 9: return run_b<S, 9, true>(d, koff, lds, st);
    case 10: return run_b<S, 10, true>(d, koff, lds, st);
    case 11: return run_b<S, 11, true>(d, koff, lds, st);
    case 12: return run_b<S, 12, true>(d, koff, lds, st);
    case 13: return run_b<S, 13, true>(d, koff, lds, st);
    case 14: return run_b<S, 14, true>(d, koff, lds, st);
    case 15: return run_b<S, 15, true>(d, koff, lds, st);
    case 16: return run_b<S, 16, true>(d, koff, lds, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_pass_b(int prec, const ProbDesc* single, const ProbDesc* d_descs, const WorkItem* items,
                         int nitems, int koff, int lds, hipStream_t st) {
  if (single) return prec == 0 ? run_b_cls<float>(*single, koff, lds, st) : run_b_cls<double>(*single, koff, lds, st);
  return prec == 0 ? run_b_batch<float>(d_descs, items, nitems, koff, lds, st)
                   : run_b_batch<double>(d_descs, items, nitems, koff, lds, st);
}

template <typename S>
static hipError_t run_persist(const ProbDesc* d_descs, const PTask* tasks, int ntasks, int* ctl_done, int nprob,
                              long long wait_ticks, int lds, hipStream_t st) {
  constexpr int esz = int(sizeof(C<S>));
  constexpr int la = pass_a_lds_bytes(esz, 4, 3 * 17 - 1, 17);
  constexpr int lb = pass_b_lds_bytes(esz, 64, 16, kPersistThreads);
  constexpr int lc = pass_b_pcr_lds_bytes();
  constexpr int lds_max = la > lb ? (la > lc ? la : lc) : (lb > lc ? lb : lc);
  if (lds > lds_max || ntasks < 1 || nprob < 1) return hipErrorInvalidValue;
  const void* fn = reinterpret_cast<const void*>(&march_persist<S>);
  hipError_t e = allow_lds(fn, lds_max);
  if (e != hipSuccess) return e;
  // resident workgroups of this LDS size, looked up once per (device, lds)
  static std::mutex mu;
  static std::map<std::pair<int, int>, int> cap;
  int dev = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  int grid = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cap.find({dev, lds});
    if (it != cap.end()) {
      grid = it->second;
    } else {
      int per_cu = 0, ncu = 0;
      if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kPersistThreads, lds)) != hipSuccess) return e;
      if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
      grid = std::max(1, per_cu) * std::max(1, ncu);
      cap[{dev, lds}] = grid;
    }
  }
  grid = std::min(grid, ntasks);
  const int nfill = persist_ctl_ints(nprob);
  hipLaunchKernelGGL(fill_ints, dim3((nfill + 255) / 256), dim3(256), 0, st, ctl_done, nfill, 0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((march_persist<S>), dim3(grid), dim3(kPersistThreads), lds, st, d_descs, tasks, ntasks,
                     ctl_done, ctl_done + 2 * kPersistCounterStride, wait_ticks);
  return hipGetLastError();
}

hipError_t launch_persist(int prec, const ProbDesc* d_descs, const PTask* tasks, int ntasks, int* ctl_done,
                          int nprob, long long wait_ticks, int lds, hipStream_t st) {
  return prec == 0 ? run_persist<float>(d_descs, tasks, ntasks, ctl_done, nprob, wait_ticks, lds, st)
                   : run_persist<double>(d_descs, tasks, ntasks, ctl_done, nprob, wait_ticks, lds, st);
}

hipError_t persist_take_timeouts(unsigned long long* n) {
  unsigned long long v = 0, z = 0;
  hipError_t e = hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_wait_timeouts), sizeof v, 0, hipMemcpyDeviceToHost);
  if (e == hipSuccess && v) e = hipMemcpyToSymbol(HIP_SYMBOL(g_wait_timeouts), &z, sizeof z, 0, hipMemcpyHostToDevice);
  *n = v;
  return e;
}

hipError_t launch_medium_update(const ProbDesc* single, const ProbDesc* d_descs, const WorkItem* items,
                               int nitems, int koff, hipStream_t st) {
  if (single)
    hipLaunchKernelGGL(medium_update_single, dim3(single->nbr ? (single->nth + 255) / 256 : 1), dim3(256), 0, st,
                       *single, koff);
  else
    hipLaunchKernelGGL(medium_update_batch, dim3(nitems), dim3(256), 0, st, d_descs, items, koff);
  return hipGetLastError();
}

hipError_t launch_advance(long long* const* jdevs_dev, const int* adds_dev, int n, long long* jsingle,
                          int add, hipStream_t st) {
  int blocks = jsingle ? 1 : (n + 255) / 256;
  hipLaunchKernelGGL(advance_kernel, dim3(blocks), dim3(256), 0, st, jdevs_dev, adds_dev, n, jsingle, add);
  return hipGetLastError();
}

hipError_t launch_starter(int prec, const ProbDesc& d, double zs, void* u, hipStream_t st) {
  size_t n = (size_t)d.nz * d.nth;
  int blocks = int(std::min<size_t>((n + 255) / 256, 4096));
  if (prec == 0)
    hipLaunchKernelGGL(starter_kernel<float>, dim3(blocks), dim3(256), 0, st, d, zs, (C<float>*)u);
  else
    hipLaunchKernelGGL(starter_kernel<double>, dim3(blocks), dim3(256), 0, st, d, zs, (C<double>*)u);
  return hipGetLastError();
}

hipError_t launch_scale(int prec, const ProbDesc& d, const void* u, void* p, double hre, double him,
                        hipStream_t st) {
  size_t n = (size_t)d.nz * d.nth;
  int blocks = int(std::min<size_t>((n + 255) / 256, 4096));
  if (prec == 0)
    hipLaunchKernelGGL(scale_kernel<float>, dim3(blocks), dim3(256), 0, st, (const C<float>*)u, (C<float>*)p, n,
                       hre, him);
  else
    hipLaunchKernelGGL(scale_kernel<double>, dim3(blocks), dim3(256), 0, st, (const C<double>*)u,
                       (C<double>*)p, n, hre, him);
  return hipGetLastError();
}

hipError_t launch_tl(int prec, const ProbDesc& d, const void* u, float* tl, hipStream_t st) {
  size_t n = (size_t)d.nz * d.nth;
  int blocks = int(std::min<size_t>((n + 255) / 256, 4096));
  if (prec == 0)
    hipLaunchKernelGGL(tl_kernel<float>, dim3(blocks), dim3(256), 0, st, d, (const C<float>*)u, tl);
  else
    hipLaunchKernelGGL(tl_kernel<double>, dim3(blocks), dim3(256), 0, st, d, (const C<double>*)u, tl);
  return hipGetLastError();
}

}  // namespace pe3d
