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
// Kernels are templated on the real type R (float: complex64 storage and
// arithmetic; double: complex128) and on the maximum chunk length.
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
  C<double> den = mk<double>(2.0 + q.re, 2.0 * sigma + q.im);
  return cdiv(mk<double>(2.0 * s.re, 2.0 * s.im), den);
}

// ============================================================== pass A
template <typename R, int MAXM>
__device__ __forceinline__ void pass_a_body(const ProbDesc& d, int tile, int koff, C<R>* lds) {
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
  const C<R>* __restrict__ src = (const C<R>*)(first ? d.u : d.scr);
  C<R>* __restrict__ dst = (C<R>*)d.scr;
  const int stride = L * (M + 1);
  const int ncols = min(cpw, NT - m0);
  C<R>* slots = lds + cpw * stride;  // 4 complex per column
  const float invM = 1.0f / float(M);

  for (int q = t; q < 4; q += L) slots[cw * 4 + q] = zero<R>();

  // ---- stage the columns into LDS; on the first step apply [I + s_0 D_theta]
  if (!first) {
    for (int c = 0; c < ncols; ++c) {
      const C<R>* col = src + (size_t)(m0 + c) * N;
      for (int r = lane; r < N; r += 64) {
        int q = int((float(r) + 0.5f) * invM);
        lds[c * stride + r + q] = col[r];
      }
    }
  } else {
    const long long j = *d.jdev + koff;
    const R s0 = R(sigma_of(d, j));  // s_0 = i * s0
    for (int c = 0; c < ncols; ++c) {
      const int mm = m0 + c;
      const C<R>* col = src + (size_t)mm * N;
      int ml = mm - 1, mr = mm + 1;
      bool hl = true, hr = true;
      if (d.periodic) {
        if (ml < 0) ml = NT - 1;
        if (mr >= NT) mr = 0;
      } else {
        hl = ml >= 0;
        hr = mr < NT;
      }
      const C<R>* coll = src + (size_t)(hl ? ml : mm) * N;
      const C<R>* colr = src + (size_t)(hr ? mr : mm) * N;
      for (int r = lane; r < N; r += 64) {
        C<R> uc = col[r];
        C<R> ul = hl ? coll[r] : zero<R>();
        C<R> ur = hr ? colr[r] : zero<R>();
        C<R> dd = sub(add(ul, ur), scl(R(2), uc));
        // w = u + i s0 dd
        C<R> w = mk<R>(uc.re - s0 * dd.im, uc.im + s0 * dd.re);
        int q = int((float(r) + 0.5f) * invM);
        lds[c * stride + r + q] = w;
      }
    }
  }
  __syncthreads();

  // ---- per-column constants
  const R h = R(d.h);
  const C<R> qb = mk<R>(R(d.qb_re), R(d.qb_im));
  const C<R> bp = mk<R>(R(d.bp_re), R(d.bp_im));
  const C<R> bmh = mk<R>(R(d.bm_re * d.h), R(d.bm_im * d.h));
  const C<R> nbmh = mk<R>(-bmh.re, -bmh.im);
  const C<R>* __restrict__ qw = (const C<R>*)d.qw;
  const C<R>* __restrict__ pw = (const C<R>*)d.pw;
  const C<R>* __restrict__ pb = (const C<R>*)d.pb;
  int k = 0;
  ColBlock<R> B;
  if (colok) {
    k = d.kcol[m];
    B = ((const ColBlock<R>*)d.blk)[m];
  } else {
    B.xl0 = B.xd0 = B.xu0 = B.xl1 = B.xd1 = B.xu1 = zero<R>();
    B.fk = B.gk1 = B.i00 = B.i01 = B.i10 = B.i11 = zero<R>();
  }
  const bool rigid = d.rigid != 0;
  const int r0 = t * M;
  const C<R>* my = lds + cw * stride + t * (M + 1);

  // ---- RHS R = w + beta_+ X w over the lane's rows (sliding window)
  C<R> Rv[MAXM];
  {
    C<R> wm = (r0 >= 1 && r0 - 1 < N) ? my[-2] : zero<R>();
    C<R> wc = (r0 < N) ? my[0] : zero<R>();
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      const int r = r0 + i;
      C<R> wp = zero<R>();
      if (i < M && r + 1 < N) wp = (i + 1 < M) ? my[i + 1] : my[M + 1];
      C<R> X;
      if (r < k) {
        C<R> qv = (i < M && r < N) ? qw[r] : zero<R>();
        C<R> dg = mk<R>(qv.re - R(2) * h, qv.im);
        X = fma(dg, wc, scl(h, add(wm, wp)));
      } else if (r > k + 1) {
        R hl = (rigid && r == N - 1) ? R(2) * h : h;
        C<R> dg = mk<R>(qb.re - R(2) * h, qb.im);
        X = fma(dg, wc, add(scl(hl, wm), scl(h, wp)));
      } else if (r == k) {
        X = fma(B.xl0, wm, fma(B.xd0, wc, mul(B.xu0, wp)));
      } else {
        X = fma(B.xl1, wm, fma(B.xd1, wc, mul(B.xu1, wp)));
      }
      Rv[i] = (i < M && r < N) ? fma(bp, X, wc) : zero<R>();
      wm = wc;
      wc = wp;
    }
  }

  // ---- elimination: top rows r < k downward, bottom rows r > k+1 upward
  C<R> Ft = one<R>(), Et = zero<R>(), Gb = one<R>(), Sb = zero<R>();
#pragma unroll
  for (int i = 0; i < MAXM; ++i) {
    const int r = r0 + i;
    if (i < M && r < N && r < k) {
      C<R> f = (r == 0) ? zero<R>() : mul(nbmh, pw[r - 1]);
      Et = fma(f, Et, Rv[i]);
      Ft = mul(Ft, f);
      Rv[i] = Et;
    }
  }
#pragma unroll
  for (int i = MAXM - 1; i >= 0; --i) {
    const int r = r0 + i;
    if (i < M && r < N && r > k + 1) {
      C<R> g = (r == N - 1) ? zero<R>() : mul(nbmh, pb[r + 1]);
      Sb = fma(g, Sb, Rv[i]);
      Gb = mul(Gb, g);
      Rv[i] = Sb;
    }
  }
  // segmented scans over the L lanes of the column
  {
    C<R> A = Ft, Bv = Et, A2 = Gb, B2 = Sb;
    for (int dd = 1; dd < L; dd <<= 1) {
      C<R> Ap = shfl_up(A, dd, L), Bp = shfl_up(Bv, dd, L);
      C<R> A2p = shfl_down(A2, dd, L), B2p = shfl_down(B2, dd, L);
      if (t >= dd) {
        Bv = fma(A, Bp, Bv);
        A = mul(A, Ap);
      }
      if (t + dd < L) {
        B2 = fma(A2, B2p, B2);
        A2 = mul(A2, A2p);
      }
    }
    C<R> ctop = shfl_up(Bv, 1, L);
    C<R> cbot = shfl_down(B2, 1, L);
    if (t == 0) ctop = zero<R>();
    if (t == L - 1) cbot = zero<R>();
    C<R> P = one<R>();
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      const int r = r0 + i;
      if (i < M && r < N && r < k) {
        C<R> f = (r == 0) ? zero<R>() : mul(nbmh, pw[r - 1]);
        P = mul(P, f);
        Rv[i] = fma(P, ctop, Rv[i]);
      }
    }
    P = one<R>();
#pragma unroll
    for (int i = MAXM - 1; i >= 0; --i) {
      const int r = r0 + i;
      if (i < M && r < N && r > k + 1) {
        C<R> g = (r == N - 1) ? zero<R>() : mul(nbmh, pb[r + 1]);
        P = mul(P, g);
        Rv[i] = fma(P, cbot, Rv[i]);
      }
    }
  }

  // ---- 2x2 interface block
#pragma unroll
  for (int i = 0; i < MAXM; ++i) {
    const int r = r0 + i;
    if (i < M && r < N) {
      if (r == k - 1) slots[cw * 4 + 0] = Rv[i];
      if (r == k) slots[cw * 4 + 1] = Rv[i];
      if (r == k + 1) slots[cw * 4 + 2] = Rv[i];
      if (r == k + 2) slots[cw * 4 + 3] = Rv[i];
    }
  }
  __syncthreads();
  C<R> vk, vk1;
  {
    C<R> ykm1 = slots[cw * 4 + 0], Rk = slots[cw * 4 + 1];
    C<R> Rk1 = slots[cw * 4 + 2], zk2 = slots[cw * 4 + 3];
    C<R> rk = fma(B.fk, ykm1, Rk);
    C<R> rk1 = fma(B.gk1, zk2, Rk1);
    vk = fma(B.i00, rk, mul(B.i01, rk1));
    vk1 = fma(B.i10, rk, mul(B.i11, rk1));
  }

  // ---- back substitution: top rows upward from v_k, bottom rows downward from v_{k+1}
  C<R> Ht = one<R>(), Eu = zero<R>(), Hb = one<R>(), Ed = zero<R>();
#pragma unroll
  for (int i = MAXM - 1; i >= 0; --i) {
    const int r = r0 + i;
    if (i < M && r < N) {
      if (r < k) {
        C<R> p = pw[r];
        C<R> hh = mul(nbmh, p);
        Eu = fma(hh, Eu, mul(p, Rv[i]));
        Ht = mul(Ht, hh);
        Rv[i] = Eu;
      } else if (r == k) {
        Rv[i] = vk;
      } else if (r == k + 1) {
        Rv[i] = vk1;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < MAXM; ++i) {
    const int r = r0 + i;
    if (i < M && r < N && r > k + 1) {
      C<R> p = pb[r];
      C<R> a = (rigid && r == N - 1) ? scl(R(2), nbmh) : nbmh;
      C<R> hh = mul(a, p);
      Ed = fma(hh, Ed, mul(p, Rv[i]));
      Hb = mul(Hb, hh);
      Rv[i] = Ed;
    }
  }
  {
    C<R> A = Ht, Bv = Eu, A2 = Hb, B2 = Ed;
    for (int dd = 1; dd < L; dd <<= 1) {
      C<R> Ap = shfl_down(A, dd, L), Bp = shfl_down(Bv, dd, L);
      C<R> A2p = shfl_up(A2, dd, L), B2p = shfl_up(B2, dd, L);
      if (t + dd < L) {
        Bv = fma(A, Bp, Bv);
        A = mul(A, Ap);
      }
      if (t >= dd) {
        B2 = fma(A2, B2p, B2);
        A2 = mul(A2, A2p);
      }
    }
    // carries: top chain enters from below with v_k, bottom chain from above with v_{k+1}
    C<R> An = shfl_down(A, 1, L), Bn = shfl_down(Bv, 1, L);
    C<R> A2n = shfl_up(A2, 1, L), B2n = shfl_up(B2, 1, L);
    C<R> cup = (t == L - 1) ? vk : fma(An, vk, Bn);
    C<R> cdn = (t == 0) ? vk1 : fma(A2n, vk1, B2n);
    C<R> P = one<R>();
#pragma unroll
    for (int i = MAXM - 1; i >= 0; --i) {
      const int r = r0 + i;
      if (i < M && r < N && r < k) {
        C<R> hh = mul(nbmh, pw[r]);
        P = mul(P, hh);
        Rv[i] = fma(P, cup, Rv[i]);
      }
    }
    P = one<R>();
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      const int r = r0 + i;
      if (i < M && r < N && r > k + 1) {
        C<R> a = (rigid && r == N - 1) ? scl(R(2), nbmh) : nbmh;
        C<R> hh = mul(a, pb[r]);
        P = mul(P, hh);
        Rv[i] = fma(P, cdn, Rv[i]);
      }
    }
  }

  // ---- write back through LDS, coalesced store
  __syncthreads();
  C<R>* myw = lds + cw * stride + t * (M + 1);
#pragma unroll
  for (int i = 0; i < MAXM; ++i) {
    if (i < M && r0 + i < N) myw[i] = Rv[i];
  }
  __syncthreads();
  for (int c = 0; c < ncols; ++c) {
    C<R>* col = dst + (size_t)(m0 + c) * N;
    for (int r = lane; r < N; r += 64) {
      int q = int((float(r) + 0.5f) * invM);
      col[r] = lds[c * stride + r + q];
    }
  }
}

template <typename R, int MAXM>
__global__ __launch_bounds__(64) void pass_a_single(ProbDesc d, int koff) {
  extern __shared__ __align__(16) unsigned char smem_a[];
  pass_a_body<R, MAXM>(d, blockIdx.x, koff, (C<R>*)smem_a);
}

template <typename R, int MAXM>
__global__ __launch_bounds__(64) void pass_a_batch(const ProbDesc* __restrict__ descs,
                                                   const WorkItem* __restrict__ items, int koff) {
  extern __shared__ __align__(16) unsigned char smem_a[];
  const WorkItem it = items[blockIdx.x];
  const ProbDesc d = descs[it.prob];
  pass_a_body<R, MAXM>(d, it.tile, koff, (C<R>*)smem_a);
}

// ============================================================== pass B
template <typename R, int MAXM>
__device__ __forceinline__ void pass_b_body(const ProbDesc& d, int tile, int koff) {
  constexpr int NTHR = kPassBThreads;
  __shared__ C<double> sE1[NTHR], sC1[NTHR], sE2[NTHR], sC2[NTHR];
  __shared__ C<R> sUf[NTHR], sUl[NTHR];
  __shared__ C<R> sPow[MAXM + 2];
  __shared__ C<double> sK[NTHR];

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
  const C<double> rho = rho_of(sig);
  const C<R> rhoR = from_d<R>(rho);
  if (tid <= MAXM + 1) sPow[tid] = from_d<R>(cpow(rho, tid));

  const C<R>* __restrict__ src = (const C<R>*)d.scr;
  C<R>* __restrict__ dst = (C<R>*)(last ? d.u : d.scr);

  // ---- load the chunk and its two azimuth neighbours
  C<R> v[MAXM], x[MAXM];
  C<R> vl = zero<R>(), vr = zero<R>();
  if (act) {
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      v[i] = (i < len) ? src[(size_t)(m0 + i) * N + z] : zero<R>();
    int ml = m0 - 1, mr = m0 + len;
    if (periodic) {
      if (ml < 0) ml = NT - 1;
      if (mr >= NT) mr = 0;
      vl = src[(size_t)ml * N + z];
      vr = src[(size_t)mr * N + z];
    } else {
      if (ml >= 0) vl = src[(size_t)ml * N + z];
      if (mr < NT) vr = src[(size_t)mr * N + z];
    }
  } else {
#pragma unroll
    for (int i = 0; i < MAXM; ++i) v[i] = zero<R>();
  }
  // ---- D_theta v, forward recurrence y_m = t_m + rho y_{m-1} with zero carry
  C<R> E = zero<R>();
#pragma unroll
  for (int i = 0; i < MAXM; ++i) {
    if (i < len) {
      C<R> a = (i == 0) ? vl : v[i - 1];
      C<R> b = (i + 1 < len) ? v[i + 1] : vr;
      C<R> tt = sub(add(a, b), scl(R(2), v[i]));
      E = fma(rhoR, E, tt);
      x[i] = E;
    } else {
      x[i] = zero<R>();
    }
  }
  sE1[tid] = to_d(E);
  __syncthreads();
  // ---- carries across chunks (FP64); periodic closure y_{-1} = y_{N-1}
  if (c == 0) {
    const C<double> rM = cpow(rho, M);
    const int lastlen = NT - (NC - 1) * M;
    const C<double> rL = cpow(rho, lastlen);
    C<double> carry = zero<double>();
    if (periodic) {
      C<double> tot = zero<double>();
      for (int cc = 0; cc < NC; ++cc) tot = add(mul(cc == NC - 1 ? rL : rM, tot), sE1[cc * TD + dl]);
      C<double> rN = cpow(rho, NT);
      carry = cdiv(tot, mk<double>(1.0 - rN.re, -rN.im));
    }
    for (int cc = 0; cc < NC; ++cc) {
      sC1[cc * TD + dl] = carry;
      carry = add(mul(cc == NC - 1 ? rL : rM, carry), sE1[cc * TD + dl]);
    }
  }
  __syncthreads();
  {
    C<R> cin = from_d<R>(sC1[tid]);
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      if (i < len) x[i] = fma(sPow[i + 1], cin, x[i]);
  }
  // ---- backward recurrence x_m = y_m + rho x_{m+1} with zero carry
  C<R> S = zero<R>();
#pragma unroll
  for (int i = MAXM - 1; i >= 0; --i) {
    if (i < len) {
      S = fma(rhoR, S, x[i]);
      x[i] = S;
    }
  }
  sE2[tid] = to_d(S);
  __syncthreads();
  if (c == 0) {
    const C<double> rM = cpow(rho, M);
    const int lastlen = NT - (NC - 1) * M;
    const C<double> rL = cpow(rho, lastlen);
    C<double> carry = zero<double>();
    if (periodic) {
      C<double> tot = zero<double>();
      for (int cc = NC - 1; cc >= 0; --cc) tot = add(mul(cc == NC - 1 ? rL : rM, tot), sE2[cc * TD + dl]);
      C<double> rN = cpow(rho, NT);
      carry = cdiv(tot, mk<double>(1.0 - rN.re, -rN.im));
    }
    for (int cc = NC - 1; cc >= 0; --cc) {
      sC2[cc * TD + dl] = carry;
      carry = add(mul(cc == NC - 1 ? rL : rM, carry), sE2[cc * TD + dl]);
    }
  }
  __syncthreads();
  {
    C<R> cin = from_d<R>(sC2[tid]);
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      if (i < len) x[i] = fma(sPow[len - i], cin, x[i]);
  }
  // ---- e = rho x; sector: rank-one correction of the first row,
  //      e_m -= K (rho^m - rho^{2N-m}),  K = rho^2 e_0 / (1 - rho^{2N+2})
  C<R> u[MAXM];
#pragma unroll
  for (int i = 0; i < MAXM; ++i) u[i] = fma(rhoR, x[i], v[i]);
  if (!periodic) {
    if (c == 0) sK[dl] = mul(rho, to_d(x[0]));
    __syncthreads();
    if (act) {
      C<double> e0 = sK[dl];
      C<double> r2N2 = cpow(rho, 2 * (long long)NT + 2);
      C<double> K = cdiv(mul(mul(rho, rho), e0), mk<double>(1.0 - r2N2.re, -r2N2.im));
      C<double> pa = mul(K, cpow(rho, m0));                          // K rho^m at i = 0
      C<double> pbk = mul(K, cpow(rho, 2 * (long long)NT - m0 - len + 1));  // K rho^{2N-m} at i = len-1
      C<R> paR = from_d<R>(pa), pbR = from_d<R>(pbk);
#pragma unroll
      for (int i = 0; i < MAXM; ++i) {
        if (i < len) {
          C<R> corr = sub(mul(paR, sPow[i]), mul(pbR, sPow[len - 1 - i]));
          u[i] = sub(u[i], corr);
        }
      }
    }
  }
  // ---- next step's azimuth factor w = u + s_{j+1} D_theta u, or store u
  if (!last) {
    sUf[tid] = u[0];
    sUl[tid] = zero<R>();
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      if (i == len - 1) sUl[tid] = u[i];
    __syncthreads();
    if (act) {
      C<R> ul, ur;
      if (c > 0) ul = sUl[(c - 1) * TD + dl];
      else ul = periodic ? sUl[(NC - 1) * TD + dl] : zero<R>();
      if (c < NC - 1) ur = sUf[(c + 1) * TD + dl];
      else ur = periodic ? sUf[dl] : zero<R>();
      const R s1 = R(sigma_of(d, j + 1));
#pragma unroll
      for (int i = 0; i < MAXM; ++i) {
        if (i < len) {
          C<R> a = (i == 0) ? ul : u[i - 1];
          C<R> b = (i + 1 < len) ? u[i + 1] : ur;
          C<R> dd = sub(add(a, b), scl(R(2), u[i]));
          dst[(size_t)(m0 + i) * N + z] = mk<R>(u[i].re - s1 * dd.im, u[i].im + s1 * dd.re);
        }
      }
    }
  } else if (act) {
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      if (i < len) dst[(size_t)(m0 + i) * N + z] = u[i];
  }
}

template <typename R, int MAXM>
__global__ __launch_bounds__(kPassBThreads) void pass_b_single(ProbDesc d, int koff) {
  pass_b_body<R, MAXM>(d, blockIdx.x, koff);
}

template <typename R, int MAXM>
__global__ __launch_bounds__(kPassBThreads) void pass_b_batch(const ProbDesc* __restrict__ descs,
                                                              const WorkItem* __restrict__ items,
                                                              int koff) {
  const WorkItem it = items[blockIdx.x];
  const ProbDesc d = descs[it.prob];
  pass_b_body<R, MAXM>(d, it.tile, koff);
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
int pass_a_lds_bytes(int prec, int maxm) {
  size_t csz = prec ? 16 : 8;
  return int(csz * (64 * (maxm + 1) + 4 * 64));
}

template <typename R, int MAXM>
static hipError_t run_a(const ProbDesc* single, const ProbDesc* d_descs, const WorkItem* items,
                        int nitems, int koff, hipStream_t st) {
  const int lds = int(sizeof(C<R>) * (64 * (MAXM + 1) + 4 * 64));
  if (single) {
    hipLaunchKernelGGL((pass_a_single<R, MAXM>), dim3(single->ntile_a), dim3(64), lds, st, *single, koff);
  } else {
    hipLaunchKernelGGL((pass_a_batch<R, MAXM>), dim3(nitems), dim3(64), lds, st, d_descs, items, koff);
  }
  return hipGetLastError();
}

template <typename R, int MAXM>
static hipError_t run_b(const ProbDesc* single, const ProbDesc* d_descs, const WorkItem* items,
                        int nitems, int koff, hipStream_t st) {
  if (single) {
    hipLaunchKernelGGL((pass_b_single<R, MAXM>), dim3(single->ntile_b), dim3(kPassBThreads), 0, st,
                       *single, koff);
  } else {
    hipLaunchKernelGGL((pass_b_batch<R, MAXM>), dim3(nitems), dim3(kPassBThreads), 0, st, d_descs,
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
      case 32: return run_b<float, 32>(single, d_descs, items, nitems, koff, st);
    }
  } else {
    switch (maxm) {
      case 4: return run_b<double, 4>(single, d_descs, items, nitems, koff, st);
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
