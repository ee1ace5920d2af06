// HIP kernels (gfx950) of the split Crank-Nicolson PE range march, Eq. (4).
//
// One range step is two passes over the field u[theta][z] (depth contiguous):
//
//  pass A (depth pass, Eqs. (5)/(7)): per azimuth column, R = [I + beta_+ X] w
//    with w = [I + s_j D_theta] u^j, then solve [I + beta_- X] v = R.
//    One 64-lane wavefront owns 64/L columns; each column is split into L
//    contiguous chunks of M rows, one per lane.  The column is staged through
//    LDS so that global loads and stores are coalesced along depth.  The
//    solve is a twisted factorisation: rows above the water/bottom interface
//    are eliminated top-down with the shared pivots of the all-water column,
//    rows below bottom-up with the shared pivots of the all-bottom column,
//    and the two interface rows form a 2x2 block.  Every first-order
//    recurrence of that elimination is split over the lanes: a local sweep
//    with zero carry, a segmented wavefront scan of the chunk's affine maps
//    (cross-lane shuffles), and a fix-up with the exact carry.
//
//  pass B (azimuth pass, Eqs. (6)/(8)): per depth, solve [I - s_j D_theta] u = v.
//    The operator is circulant (periodic) or Toeplitz (sector) with constant
//    coefficients and factors exactly as c (1 - rho S)(1 - rho S^-1), S the
//    cyclic shift, s rho^2 - (1 + 2s) rho + s = 0, |rho| < 1, c = s / rho.
//    The kernel solves for the defect e = u - v, B e = s D_theta v, i.e.
//    e = rho (1 - rho S^-1)^-1 (1 - rho S)^-1 D_theta v: two constant-coefficient
//    recurrences (forward, backward) split into azimuth chunks, with the
//    cross-chunk carries and the periodic wrap (a Sherman-Morrison rank-one
//    correction of each cyclic bidiagonal factor) evaluated in FP64; a sector
//    adds the rank-one correction of its first row.  Lanes are consecutive
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

template <typename R>
__device__ __forceinline__ C<R> from_d(C<double> z) { return mk<R>(R(z.re), R(z.im)); }
template <typename R>
__device__ __forceinline__ C<double> to_d(C<R> z) { return mk<double>(double(z.re), double(z.im)); }
using D = C<double>;

// ---------------------------------------------------------------- FP64 helpers
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
// root of s rho^2 - (1+2s) rho + s = 0 inside the unit circle, s = i sigma:
// rho = 2s / (1 + 2s + sqrt(1 + 4s))
__device__ __forceinline__ C<double> rho_of(double sigma) {
  C<double> s = mk<double>(0.0, sigma);
  C<double> q = csqrt(mk<double>(1.0, 4.0 * sigma));
  C<double> den = mk<double>(1.0 + q.re, 2.0 * sigma + q.im);
  return cdiv(mk<double>(2.0 * s.re, 2.0 * s.im), den);
}

// ============================================================== pass A
template <typename S, int MAXM>
__device__ __forceinline__ void pass_a_body(const ProbDesc& d, int tile, int koff, C<S>* lds) {
  const int lane = threadIdx.x;
  const int L = d.lpc;
  const int cpw = 64 / L;
  const int cw = lane / L;
  const int t = lane - cw * L;
  const int N = d.nz, NT = d.nth, M = d.ma;
  const int m0 = tile * cpw;
  const int m = m0 + cw;
  const bool colok = m < NT;
  const bool first = (koff == 0);
  const C<S>* __restrict__ src = (const C<S>*)(first ? d.u : d.scr);
  C<S>* __restrict__ dst = (C<S>*)d.scr;
  const int stride = L * (M + 1);
  const int ncols = min(cpw, NT - m0);
  D* slots = reinterpret_cast<D*>(lds + 64 * (MAXM + 1));  // 4 per column
  const float invM = 1.0f / float(M);

  for (int q = t; q < 4; q += L) slots[cw * 4 + q] = zero<double>();

  // ---- stage the columns into LDS; on the first step apply [I + s_0 D_theta]
  if (!first) {
    for (int c = 0; c < ncols; ++c) {
      const C<S>* col = src + (size_t)(m0 + c) * N;
      for (int r = lane; r < N; r += 64) {
        int q = int((float(r) + 0.5f) * invM);
        lds[c * stride + r + q] = col[r];
      }
    }
  } else {
    const long long j = *d.jdev + koff;
    const double s0 = sigma_of(d, j);  // s_0 = i * s0
    for (int c = 0; c < ncols; ++c) {
      const int mm = m0 + c;
      const C<S>* col = src + (size_t)mm * N;
      int ml = mm - 1, mr = mm + 1;
      bool hl = true, hr = true;
      if (d.periodic) {
        if (ml < 0) ml = NT - 1;
        if (mr >= NT) mr = 0;
      } else {
        hl = ml >= 0;
        hr = mr < NT;
      }
      const C<S>* coll = src + (size_t)(hl ? ml : mm) * N;
      const C<S>* colr = src + (size_t)(hr ? mr : mm) * N;
      for (int r = lane; r < N; r += 64) {
        D uc = to_d(col[r]);
        D ul = hl ? to_d(coll[r]) : zero<double>();
        D ur = hr ? to_d(colr[r]) : zero<double>();
        D dd = sub(add(ul, ur), scl(2.0, uc));
        D w = mk<double>(uc.re - s0 * dd.im, uc.im + s0 * dd.re);  // u + i s0 dd
        int q = int((float(r) + 0.5f) * invM);
        lds[c * stride + r + q] = from_d<S>(w);
      }
    }
  }
  __syncthreads();

  // ---- per-column constants (FP64)
  const double h = d.h;
  const D qb = mk<double>(d.qb_re, d.qb_im);
  const D bp = mk<double>(d.bp_re, d.bp_im);
  const D nbmh = mk<double>(-d.bm_re * d.h, -d.bm_im * d.h);
  const D* __restrict__ qw = (const D*)d.qw;
  const D* __restrict__ pw = (const D*)d.pw;
  const D* __restrict__ pb = (const D*)d.pb;
  int k = 0;
  ColBlock<double> B;
  if (colok) {
    k = d.kcol[m];
    B = ((const ColBlock<double>*)d.blk)[m];
  } else {
    B.xl0 = B.xd0 = B.xu0 = B.xl1 = B.xd1 = B.xu1 = zero<double>();
    B.fk = B.gk1 = B.i00 = B.i01 = B.i10 = B.i11 = zero<double>();
  }
  const bool rigid = d.rigid != 0;
  const D nbmh_floor = rigid ? scl(2.0, nbmh) : nbmh;  // lower coefficient of a rigid floor row
  const int r0 = t * M;
  const C<S>* my = lds + cw * stride + t * (M + 1);

  // ---- RHS R = w + beta_+ X w over the lane's rows (sliding window)
  C<S> Rv[MAXM];
  {
    D wm = (r0 >= 1 && r0 - 1 < N) ? to_d(my[-2]) : zero<double>();
    D wc = (r0 < N) ? to_d(my[0]) : zero<double>();
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      const int r = r0 + i;
      D wp = zero<double>();
      if (i < M && r + 1 < N) wp = to_d((i + 1 < M) ? my[i + 1] : my[M + 1]);
      D X;
      if (r < k) {
        D qv = (i < M && r < N) ? qw[r] : zero<double>();
        X = fma(mk<double>(qv.re - 2.0 * h, qv.im), wc, scl(h, add(wm, wp)));
      } else if (r > k + 1) {
        double hl = (rigid && r == N - 1) ? 2.0 * h : h;
        X = fma(mk<double>(qb.re - 2.0 * h, qb.im), wc, add(scl(hl, wm), scl(h, wp)));
      } else if (r == k) {
        X = fma(B.xl0, wm, fma(B.xd0, wc, mul(B.xu0, wp)));
      } else {
        X = fma(B.xl1, wm, fma(B.xd1, wc, mul(B.xu1, wp)));
      }
      Rv[i] = (i < M && r < N) ? from_d<S>(fma(bp, X, wc)) : zero<S>();
      wm = wc;
      wc = wp;
    }
  }

  // ---- elimination: top rows r < k downward, bottom rows r > k+1 upward
  D Ft = one<double>(), Et = zero<double>(), Gb = one<double>(), Sb = zero<double>();
#pragma unroll
  for (int i = 0; i < MAXM; ++i) {
    const int r = r0 + i;
    if (i < M && r < N && r < k) {
      D f = (r == 0) ? zero<double>() : mul(nbmh, pw[r - 1]);
      Et = fma(f, Et, to_d(Rv[i]));
      Ft = mul(Ft, f);
      Rv[i] = from_d<S>(Et);
    }
  }
#pragma unroll
  for (int i = MAXM - 1; i >= 0; --i) {
    const int r = r0 + i;
    if (i < M && r < N && r > k + 1) {
      D g = (r == N - 1) ? zero<double>() : mul(nbmh, pb[r + 1]);
      Sb = fma(g, Sb, to_d(Rv[i]));
      Gb = mul(Gb, g);
      Rv[i] = from_d<S>(Sb);
    }
  }
  // segmented scans over the L lanes of the column (FP64)
  {
    D A = Ft, Bv = Et, A2 = Gb, B2 = Sb;
    for (int dd = 1; dd < L; dd <<= 1) {
      D Ap = shfl_up(A, dd, L), Bp = shfl_up(Bv, dd, L);
      D A2p = shfl_down(A2, dd, L), B2p = shfl_down(B2, dd, L);
      if (t >= dd) {
        Bv = fma(A, Bp, Bv);
        A = mul(A, Ap);
      }
      if (t + dd < L) {
        B2 = fma(A2, B2p, B2);
        A2 = mul(A2, A2p);
      }
    }
    D ctop = shfl_up(Bv, 1, L);
    D cbot = shfl_down(B2, 1, L);
    if (t == 0) ctop = zero<double>();
    if (t == L - 1) cbot = zero<double>();
    D P = one<double>();
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      const int r = r0 + i;
      if (i < M && r < N && r < k) {
        D f = (r == 0) ? zero<double>() : mul(nbmh, pw[r - 1]);
        P = mul(P, f);
        Rv[i] = from_d<S>(fma(P, ctop, to_d(Rv[i])));
      }
    }
    P = one<double>();
#pragma unroll
    for (int i = MAXM - 1; i >= 0; --i) {
      const int r = r0 + i;
      if (i < M && r < N && r > k + 1) {
        D g = (r == N - 1) ? zero<double>() : mul(nbmh, pb[r + 1]);
        P = mul(P, g);
        Rv[i] = from_d<S>(fma(P, cbot, to_d(Rv[i])));
      }
    }
  }

  // ---- 2x2 interface block
#pragma unroll
  for (int i = 0; i < MAXM; ++i) {
    const int r = r0 + i;
    if (i < M && r < N) {
      if (r == k - 1) slots[cw * 4 + 0] = to_d(Rv[i]);
      if (r == k) slots[cw * 4 + 1] = to_d(Rv[i]);
      if (r == k + 1) slots[cw * 4 + 2] = to_d(Rv[i]);
      if (r == k + 2) slots[cw * 4 + 3] = to_d(Rv[i]);
    }
  }
  __syncthreads();
  D vk, vk1;
  {
    D ykm1 = slots[cw * 4 + 0], Rk = slots[cw * 4 + 1];
    D Rk1 = slots[cw * 4 + 2], zk2 = slots[cw * 4 + 3];
    D rk = fma(B.fk, ykm1, Rk);
    D rk1 = fma(B.gk1, zk2, Rk1);
    vk = fma(B.i00, rk, mul(B.i01, rk1));
    vk1 = fma(B.i10, rk, mul(B.i11, rk1));
  }

  // ---- back substitution: top rows upward from v_k, bottom rows downward from v_{k+1}
  D Ht = one<double>(), Eu = zero<double>(), Hb = one<double>(), Ed = zero<double>();
#pragma unroll
  for (int i = MAXM - 1; i >= 0; --i) {
    const int r = r0 + i;
    if (i < M && r < N) {
      if (r < k) {
        D p = pw[r];
        D hh = mul(nbmh, p);
        Eu = fma(hh, Eu, mul(p, to_d(Rv[i])));
        Ht = mul(Ht, hh);
        Rv[i] = from_d<S>(Eu);
      } else if (r == k) {
        Rv[i] = from_d<S>(vk);
      } else if (r == k + 1) {
        Rv[i] = from_d<S>(vk1);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < MAXM; ++i) {
    const int r = r0 + i;
    if (i < M && r < N && r > k + 1) {
      D p = pb[r];
      D hh = mul((r == N - 1) ? nbmh_floor : nbmh, p);
      Ed = fma(hh, Ed, mul(p, to_d(Rv[i])));
      Hb = mul(Hb, hh);
      Rv[i] = from_d<S>(Ed);
    }
  }
  {
    D A = Ht, Bv = Eu, A2 = Hb, B2 = Ed;
    for (int dd = 1; dd < L; dd <<= 1) {
      D Ap = shfl_down(A, dd, L), Bp = shfl_down(Bv, dd, L);
      D A2p = shfl_up(A2, dd, L), B2p = shfl_up(B2, dd, L);
      if (t + dd < L) {
        Bv = fma(A, Bp, Bv);
        A = mul(A, Ap);
      }
      if (t >= dd) {
        B2 = fma(A2, B2p, B2);
        A2 = mul(A2, A2p);
      }
    }
    // carries: the top chain enters from below with v_k, the bottom chain from above with v_{k+1}
    D An = shfl_down(A, 1, L), Bn = shfl_down(Bv, 1, L);
    D A2n = shfl_up(A2, 1, L), B2n = shfl_up(B2, 1, L);
    D cup = (t == L - 1) ? vk : fma(An, vk, Bn);
    D cdn = (t == 0) ? vk1 : fma(A2n, vk1, B2n);
    D P = one<double>();
#pragma unroll
    for (int i = MAXM - 1; i >= 0; --i) {
      const int r = r0 + i;
      if (i < M && r < N && r < k) {
        P = mul(P, mul(nbmh, pw[r]));
        Rv[i] = from_d<S>(fma(P, cup, to_d(Rv[i])));
      }
    }
    P = one<double>();
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      const int r = r0 + i;
      if (i < M && r < N && r > k + 1) {
        P = mul(P, mul((r == N - 1) ? nbmh_floor : nbmh, pb[r]));
        Rv[i] = from_d<S>(fma(P, cdn, to_d(Rv[i])));
      }
    }
  }

  // ---- write back through LDS, coalesced store
  __syncthreads();
  C<S>* myw = lds + cw * stride + t * (M + 1);
#pragma unroll
  for (int i = 0; i < MAXM; ++i) {
    if (i < M && r0 + i < N) myw[i] = Rv[i];
  }
  __syncthreads();
  for (int c = 0; c < ncols; ++c) {
    C<S>* col = dst + (size_t)(m0 + c) * N;
    for (int r = lane; r < N; r += 64) {
      int q = int((float(r) + 0.5f) * invM);
      col[r] = lds[c * stride + r + q];
    }
  }
}

template <typename S, int MAXM>
constexpr int pass_a_lds() {
  return int(sizeof(C<S>) * 64 * (MAXM + 1) + sizeof(D) * 4 * 64);
}

template <typename S, int MAXM>
__global__ __launch_bounds__(64) void pass_a_single(ProbDesc d, int koff) {
  extern __shared__ __align__(16) unsigned char smem_a[];
  pass_a_body<S, MAXM>(d, blockIdx.x, koff, (C<S>*)smem_a);
}

template <typename S, int MAXM>
__global__ __launch_bounds__(64) void pass_a_batch(const ProbDesc* __restrict__ descs,
                                                   const WorkItem* __restrict__ items, int koff) {
  extern __shared__ __align__(16) unsigned char smem_a[];
  const WorkItem it = items[blockIdx.x];
  const ProbDesc d = descs[it.prob];
  pass_a_body<S, MAXM>(d, it.tile, koff, (C<S>*)smem_a);
}

// ============================================================== pass B
template <typename S, int MAXM>
__device__ __forceinline__ void pass_b_body(const ProbDesc& d, int tile, int koff) {
  constexpr int NTHR = kPassBThreads;
  // sE1/sC1: forward chunk ends and carries, reused for the edge exchange;
  // sE2/sC2: backward chunk starts and carries, sE2 reused for the sector term
  __shared__ D sE1[NTHR], sC1[NTHR], sE2[NTHR], sC2[NTHR];
  __shared__ D sPow[MAXM + 2];

  const int tid = threadIdx.x;
  const int TD = d.td, NC = d.nc, M = d.mb;
  const int c = tid / TD;
  const int dl = tid - c * TD;
  const int N = d.nz, NT = d.nth;
  const int z = tile * TD + dl;
  const bool zok = z < N;
  const int m0 = c * M;
  const int len = (c < NC) ? min(M, NT - m0) : 0;
  const bool act = zok && len > 0;
  const long long j = *d.jdev + koff;
  const bool last = (koff == d.nsteps - 1);
  const bool periodic = d.periodic != 0;

  const double sig = sigma_of(d, j);
  const D rho = rho_of(sig);
  if (tid <= MAXM + 1) sPow[tid] = cpow(rho, tid);

  const C<S>* __restrict__ src = (const C<S>*)d.scr;
  C<S>* __restrict__ dst = (C<S>*)(last ? d.u : d.scr);

  // ---- load the chunk and its two azimuth neighbours
  C<S> v[MAXM];
  D x[MAXM];
  D vl = zero<double>(), vr = zero<double>();
  if (act) {
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      v[i] = (i < len) ? src[(size_t)(m0 + i) * N + z] : zero<S>();
    int ml = m0 - 1, mr = m0 + len;
    if (periodic) {
      if (ml < 0) ml = NT - 1;
      if (mr >= NT) mr = 0;
      vl = to_d(src[(size_t)ml * N + z]);
      vr = to_d(src[(size_t)mr * N + z]);
    } else {
      if (ml >= 0) vl = to_d(src[(size_t)ml * N + z]);
      if (mr < NT) vr = to_d(src[(size_t)mr * N + z]);
    }
  } else {
#pragma unroll
    for (int i = 0; i < MAXM; ++i) v[i] = zero<S>();
  }
  // ---- D_theta v, forward recurrence y_m = t_m + rho y_{m-1} with zero carry
  D E = zero<double>();
#pragma unroll
  for (int i = 0; i < MAXM; ++i) {
    if (i < len) {
      D a = (i == 0) ? vl : to_d(v[i - 1]);
      D b = (i + 1 < len) ? to_d(v[i + 1]) : vr;
      D tt = sub(add(a, b), scl(2.0, to_d(v[i])));
      E = fma(rho, E, tt);
      x[i] = E;
    } else {
      x[i] = zero<double>();
    }
  }
  sE1[tid] = E;
  __syncthreads();
  // ---- carries across chunks; periodic closure y_{-1} = y_{N-1}
  if (c == 0) {
    const D rM = cpow(rho, M);
    const D rL = cpow(rho, NT - (NC - 1) * M);
    D carry = zero<double>();
    if (periodic) {
      D tot = zero<double>();
      for (int cc = 0; cc < NC; ++cc) tot = add(mul(cc == NC - 1 ? rL : rM, tot), sE1[cc * TD + dl]);
      D rN = cpow(rho, NT);
      carry = cdiv(tot, mk<double>(1.0 - rN.re, -rN.im));
    }
    for (int cc = 0; cc < NC; ++cc) {
      sC1[cc * TD + dl] = carry;
      carry = add(mul(cc == NC - 1 ? rL : rM, carry), sE1[cc * TD + dl]);
    }
  }
  __syncthreads();
  {
    const D cin = sC1[tid];
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      if (i < len) x[i] = fma(sPow[i + 1], cin, x[i]);
  }
  // ---- backward recurrence x_m = y_m + rho x_{m+1} with zero carry
  D Sv = zero<double>();
#pragma unroll
  for (int i = MAXM - 1; i >= 0; --i) {
    if (i < len) {
      Sv = fma(rho, Sv, x[i]);
      x[i] = Sv;
    }
  }
  sE2[tid] = Sv;
  __syncthreads();
  if (c == 0) {
    const D rM = cpow(rho, M);
    const D rL = cpow(rho, NT - (NC - 1) * M);
    D carry = zero<double>();
    if (periodic) {
      D tot = zero<double>();
      for (int cc = NC - 1; cc >= 0; --cc) tot = add(mul(cc == NC - 1 ? rL : rM, tot), sE2[cc * TD + dl]);
      D rN = cpow(rho, NT);
      carry = cdiv(tot, mk<double>(1.0 - rN.re, -rN.im));
    }
    for (int cc = NC - 1; cc >= 0; --cc) {
      sC2[cc * TD + dl] = carry;
      carry = add(mul(cc == NC - 1 ? rL : rM, carry), sE2[cc * TD + dl]);
    }
  }
  __syncthreads();
  {
    const D cin = sC2[tid];
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      if (i < len) x[i] = fma(sPow[len - i], cin, x[i]);
  }
  // ---- u = v + rho x; sector: rank-one correction of the first row,
  //      e_m -= K (rho^m - rho^{2N-m}),  K = rho^2 e_0 / (1 - rho^{2N+2})
  if (!periodic) {
    if (c == 0) sE2[dl] = mul(rho, x[0]);
    __syncthreads();
    if (act) {
      const D e0 = sE2[dl];
      const D r2N2 = cpow(rho, 2 * (long long)NT + 2);
      const D K = cdiv(mul(mul(rho, rho), e0), mk<double>(1.0 - r2N2.re, -r2N2.im));
      const D pa = mul(K, cpow(rho, m0));                                  // K rho^m at i = 0
      const D pbk = mul(K, cpow(rho, 2 * (long long)NT - m0 - len + 1));   // K rho^{2N-m} at i = len-1
#pragma unroll
      for (int i = 0; i < MAXM; ++i)
        if (i < len) x[i] = sub(fma(rho, x[i], to_d(v[i])), sub(mul(pa, sPow[i]), mul(pbk, sPow[len - 1 - i])));
    }
  } else {
#pragma unroll
    for (int i = 0; i < MAXM; ++i) x[i] = fma(rho, x[i], to_d(v[i]));
  }
  // x now holds u^{j+1}.  Next step's azimuth factor w = u + s_{j+1} D_theta u, or store u.
  if (!last) {
    // start the next step from u^{j+1} as stored (rounded to S), exactly as a
    // new march call would: an interrupted and resumed march is bitwise equal
    // to an uninterrupted one
#pragma unroll
    for (int i = 0; i < MAXM; ++i) x[i] = to_d(from_d<S>(x[i]));
    D* sUf = sE1;
    D* sUl = sC1;
    sUf[tid] = x[0];
    D xl = zero<double>();
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      if (i == len - 1) xl = x[i];
    sUl[tid] = xl;
    __syncthreads();
    if (act) {
      D ul, ur;
      if (c > 0) ul = sUl[(c - 1) * TD + dl];
      else ul = periodic ? sUl[(NC - 1) * TD + dl] : zero<double>();
      if (c < NC - 1) ur = sUf[(c + 1) * TD + dl];
      else ur = periodic ? sUf[dl] : zero<double>();
      const double s1 = sigma_of(d, j + 1);
#pragma unroll
      for (int i = 0; i < MAXM; ++i) {
        if (i < len) {
          D a = (i == 0) ? ul : x[i - 1];
          D b = (i + 1 < len) ? x[i + 1] : ur;
          D dd = sub(add(a, b), scl(2.0, x[i]));
          dst[(size_t)(m0 + i) * N + z] = from_d<S>(mk<double>(x[i].re - s1 * dd.im, x[i].im + s1 * dd.re));
        }
      }
    }
  } else if (act) {
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      if (i < len) dst[(size_t)(m0 + i) * N + z] = from_d<S>(x[i]);
  }
}

template <typename S, int MAXM>
__global__ __launch_bounds__(kPassBThreads) void pass_b_single(ProbDesc d, int koff) {
  pass_b_body<S, MAXM>(d, blockIdx.x, koff);
}

template <typename S, int MAXM>
__global__ __launch_bounds__(kPassBThreads) void pass_b_batch(const ProbDesc* __restrict__ descs,
                                                              const WorkItem* __restrict__ items,
                                                              int koff) {
  const WorkItem it = items[blockIdx.x];
  const ProbDesc d = descs[it.prob];
  pass_b_body<S, MAXM>(d, it.tile, koff);
}

// ============================================================== small kernels
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

// ============================================================== launchers
template <typename S, int MAXM>
static hipError_t run_a(const ProbDesc* single, const ProbDesc* d_descs, const WorkItem* items,
                        int nitems, int koff, hipStream_t st) {
  constexpr int lds = pass_a_lds<S, MAXM>();
  if (single) {
    hipLaunchKernelGGL((pass_a_single<S, MAXM>), dim3(single->ntile_a), dim3(64), lds, st, *single, koff);
  } else {
    hipLaunchKernelGGL((pass_a_batch<S, MAXM>), dim3(nitems), dim3(64), lds, st, d_descs, items, koff);
  }
  return hipGetLastError();
}

template <typename S, int MAXM>
static hipError_t run_b(const ProbDesc* single, const ProbDesc* d_descs, const WorkItem* items,
                        int nitems, int koff, hipStream_t st) {
  if (single) {
    hipLaunchKernelGGL((pass_b_single<S, MAXM>), dim3(single->ntile_b), dim3(kPassBThreads), 0, st,
                       *single, koff);
  } else {
    hipLaunchKernelGGL((pass_b_batch<S, MAXM>), dim3(nitems), dim3(kPassBThreads), 0, st, d_descs,
                       items, koff);
  }
  return hipGetLastError();
}

hipError_t launch_pass_a(int prec, int maxm, const ProbDesc* single, const ProbDesc* d_descs,
                         const WorkItem* items, int nitems, int koff, hipStream_t st) {
  if (prec == 0) {
    switch (maxm) {
      case 16: return run_a<float, 16>(single, d_descs, items, nitems, koff, st);
      case 32: return run_a<float, 32>(single, d_descs, items, nitems, koff, st);
      case 64: return run_a<float, 64>(single, d_descs, items, nitems, koff, st);
    }
  } else {
    switch (maxm) {
      case 8: return run_a<double, 8>(single, d_descs, items, nitems, koff, st);
      case 16: return run_a<double, 16>(single, d_descs, items, nitems, koff, st);
      case 32: return run_a<double, 32>(single, d_descs, items, nitems, koff, st);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_pass_b(int prec, int maxm, const ProbDesc* single, const ProbDesc* d_descs,
                         const WorkItem* items, int nitems, int koff, hipStream_t st) {
  if (prec == 0) {
    switch (maxm) {
      case 8: return run_b<float, 8>(single, d_descs, items, nitems, koff, st);
      case 16: return run_b<float, 16>(single, d_descs, items, nitems, koff, st);
    }
  } else {
    switch (maxm) {
      case 8: return run_b<double, 8>(single, d_descs, items, nitems, koff, st);
      case 16: return run_b<double, 16>(single, d_descs, items, nitems, koff, st);
    }
  }
  return hipErrorInvalidValue;
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
