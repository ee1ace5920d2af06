// HIP kernels (gfx950) of the split Crank-Nicolson PE range march, Eq. (4).
//
// One range step is two passes over the field u[theta][z] (depth contiguous):
//
//  pass A (depth pass, Eqs. (5)/(7)): per azimuth column, R = [I + beta_+ X] w
//    with w = [I + s_j D_theta] u^j, then solve [I + beta_- X] v = R.
//    A 256-lane workgroup owns 256/L columns; each column is split into L
//    contiguous chunks of M <= 16 rows, one per lane (L up to 256 lanes, so
//    a column may span several wavefronts).  The column is staged through
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
// Workgroup of 256 lanes; a depth column is split over L lanes (L a power of
// two, 4..256), each lane holding M <= MAXM consecutive rows; 256/L <= 64
// columns per workgroup.  Columns wider than a wavefront (L > 64) combine the
// per-wavefront scan totals through LDS.
//
// A wavefront whose lanes all hold rows strictly above the interface rows of
// their column (or all strictly below) runs a branch-free path; lanes holding
// an interface row, or a partial chunk, run the general path.  With the
// rigid floor row pre-scaled by 1/2 on the host, every row of the bottom
// region has lower coefficient beta_- h.
constexpr int kPassAThreads = 256;

struct ChainPair {
  D down, up;
};
// Exclusive carries of a downward chain (lane t's map applied after lanes
// 0..t-1 of the column) and of an upward chain (after lanes t+1..L-1).  Each
// lane passes its chunk map (A, B): x -> A x + B.  tot: LDS scratch, 4 complex
// per wavefront.
__device__ __forceinline__ ChainPair scan_pair(D Ad, D Bd, D init_d, D Au, D Bu, D init_u, int t, int L,
                                               D* tot) {
  const int w = L < 64 ? L : 64;  // segment width inside a wavefront
  const int tw = t & (w - 1);     // lane within the segment
  D ad = Ad, bd = Bd, au = Au, bu = Bu;
  for (int dd = 1; dd < w; dd <<= 1) {
    D ap = shfl_up(ad, dd, w), bp = shfl_up(bd, dd, w);
    D aq = shfl_down(au, dd, w), bq = shfl_down(bu, dd, w);
    if (tw >= dd) {
      bd = fma(ad, bp, bd);
      ad = mul(ad, ap);
    }
    if (tw + dd < w) {
      bu = fma(au, bq, bu);
      au = mul(au, aq);
    }
  }
  D ade = shfl_up(ad, 1, w), bde = shfl_up(bd, 1, w);
  D aue = shfl_down(au, 1, w), bue = shfl_down(bu, 1, w);
  if (tw == 0) {
    ade = one<double>();
    bde = zero<double>();
  }
  if (tw == w - 1) {
    aue = one<double>();
    bue = zero<double>();
  }
  D xd = init_d, xu = init_u;
  if (L > 64) {
    const int wave = threadIdx.x >> 6;
    if (tw == w - 1) {
      tot[4 * wave + 0] = ad;
      tot[4 * wave + 1] = bd;
    }
    if (tw == 0) {
      tot[4 * wave + 2] = au;
      tot[4 * wave + 3] = bu;
    }
    __syncthreads();
    const int nw = L >> 6;
    const int wc = (t >> 6);
    const int w0 = wave - wc;
    for (int q = 0; q < wc; ++q) xd = fma(tot[4 * (w0 + q) + 0], xd, tot[4 * (w0 + q) + 1]);
    for (int q = nw - 1; q > wc; --q) xu = fma(tot[4 * (w0 + q) + 2], xu, tot[4 * (w0 + q) + 3]);
    __syncthreads();
  }
  ChainPair r;
  r.down = fma(ade, xd, bde);
  r.up = fma(aue, xu, bue);
  return r;
}

template <typename S, int MAXM>
__device__ __forceinline__ void pass_a_body(const ProbDesc& d, int tile, int koff, C<S>* lds) {
  const int lane = threadIdx.x;
  const int L = d.lpc;
  const int cpw = kPassAThreads / L;  // columns per workgroup
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
  D* slots = reinterpret_cast<D*>(lds + kPassAThreads * (MAXM + 1));  // 4 per column
  D* tot = slots + 4 * 64;                                              // 4 per wavefront
  const float invM = 1.0f / float(M);

  for (int q = t; q < 4; q += L) slots[cw * 4 + q] = zero<double>();

  // ---- stage the columns into LDS (coalesced); on the first step apply [I + s_0 D_theta]
  if (!first) {
    for (int c = 0; c < ncols; ++c) {
      const C<S>* col = src + (size_t)(m0 + c) * N;
      for (int r = lane; r < N; r += kPassAThreads) {
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
      for (int r = lane; r < N; r += kPassAThreads) {
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

  // ---- constants (FP64), lane classification, the lane's pivots (loaded once, coalesced)
  const double h = d.h;
  const D qb = mk<double>(d.qb_re, d.qb_im);
  const D bp = mk<double>(d.bp_re, d.bp_im);
  const D nbmh = mk<double>(-d.bm_re * d.h, -d.bm_im * d.h);
  const D* __restrict__ qwT = (const D*)d.qwT;
  const D* __restrict__ pwT = (const D*)d.pwT;
  const D* __restrict__ pbT = (const D*)d.pbT;
  const D* __restrict__ lt = (const D*)d.lane_tr;  // [4][L]: Ft, Gb, Ht, Hb of full lanes
  const int k = colok ? d.kcol[m] : 0;
  const ColBlock<double>* Bp = colok ? ((const ColBlock<double>*)d.blk) + m : nullptr;
  const bool rigid = d.rigid != 0;
  const int r0 = t * M;
  const bool full = colok && (r0 + M <= N);
  const bool ftop = full && (r0 + M <= k);   // every row above the interface rows
  const bool fbot = full && (r0 >= k + 2);   // every row below them
  const bool wave_top = __all(ftop);
  const bool wave_bot = __all(fbot);
  // piv[i]: reciprocal pivot of row r0-1+i (top-down above the interface rows,
  // bottom-up below them); zero outside the column
  __syncthreads();
  D piv[MAXM + 2];
#pragma unroll
  for (int i = 0; i < MAXM + 2; ++i) {
    const int r = r0 - 1 + i;
    piv[i] = (i < M + 2) ? (r < k ? pwT[i * L + t] : pbT[i * L + t]) : zero<double>();
  }
  const C<S>* my = lds + cw * stride + t * (M + 1);

  // ---- RHS R = w + beta_+ X w over the lane's rows (sliding window)
  D Rv[MAXM];
  {
    D wm = (r0 >= 1 && r0 - 1 < N) ? to_d(my[-2]) : zero<double>();
    D wc = (r0 < N) ? to_d(my[0]) : zero<double>();
    const D dgb = mk<double>(qb.re - 2.0 * h, qb.im);
    if (wave_top) {
#pragma unroll
      for (int i = 0; i < MAXM; ++i) {
        if (i < M) {
          const D wp = to_d((i + 1 < M) ? my[i + 1] : my[M + 1]);
          const D qv = qwT[i * L + t];
          const D X = fma(mk<double>(qv.re - 2.0 * h, qv.im), wc, scl(h, add(wm, wp)));
          Rv[i] = fma(bp, X, wc);
          wm = wc;
          wc = wp;
        }
      }
    } else if (wave_bot) {
      // a lane ending on a rigid floor: its last row has lower coefficient 2h
      // and is scaled by 1/2 (the host scales the floor row of the bottom system)
      const bool fl = rigid && (r0 + M == N);
#pragma unroll
      for (int i = 0; i < MAXM; ++i) {
        if (i < M) {
          const bool last = (i + 1 == M) && (r0 + M == N);
          const D wp = last ? zero<double>() : to_d((i + 1 < M) ? my[i + 1] : my[M + 1]);
          const D X = fma(dgb, wc, scl(h, add(wm, wp)));
          D R = fma(bp, X, wc);
          if (fl && i + 1 == M) R = scl(0.5, fma(bp, scl(h, wm), R));
          Rv[i] = R;
          wm = wc;
          wc = wp;
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < MAXM; ++i) {
        const int r = r0 + i;
        D wp = zero<double>();
        if (i < M && r + 1 < N) wp = to_d((i + 1 < M) ? my[i + 1] : my[M + 1]);
        D X;
        D R;
        if (r < k) {
          const D qv = (i < M && r < N) ? qwT[i * L + t] : zero<double>();
          X = fma(mk<double>(qv.re - 2.0 * h, qv.im), wc, scl(h, add(wm, wp)));
          R = fma(bp, X, wc);
        } else if (r > k + 1) {
          const bool flr = rigid && (r == N - 1);
          X = fma(dgb, wc, add(scl(flr ? 2.0 * h : h, wm), scl(h, wp)));
          R = fma(bp, X, wc);
          if (flr) R = scl(0.5, R);
        } else if (Bp == nullptr) {
          R = zero<double>();
        } else if (r == k) {
          X = fma(Bp->xl0, wm, fma(Bp->xd0, wc, mul(Bp->xu0, wp)));
          R = fma(bp, X, wc);
        } else {
          X = fma(Bp->xl1, wm, fma(Bp->xd1, wc, mul(Bp->xu1, wp)));
          R = fma(bp, X, wc);
        }
        Rv[i] = (i < M && r < N) ? R : zero<double>();
        wm = wc;
        wc = wp;
      }
    }
  }

  // ---- elimination: top rows downward, y_r = R_r + (-beta_- h) pivot_{r-1} y_{r-1};
  //      bottom rows upward, z_r = R_r + (-beta_- h) pivot_{r+1} z_{r+1}
  D Ft = one<double>(), Et = zero<double>(), Gb = one<double>(), Sb = zero<double>();
  if (wave_top) {
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      if (i < M) {
        Et = fma(nbmh, mul(piv[i], Et), Rv[i]);
        Rv[i] = Et;
      }
    Ft = lt[0 * L + t];
  } else if (wave_bot) {
#pragma unroll
    for (int i = MAXM - 1; i >= 0; --i)
      if (i < M) {
        Sb = fma(nbmh, mul(piv[i + 2], Sb), Rv[i]);
        Rv[i] = Sb;
      }
    Gb = lt[1 * L + t];
  } else {
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      const int r = r0 + i;
      if (i < M && r < N && r < k) {
        const D f = mul(nbmh, piv[i]);
        Et = fma(f, Et, Rv[i]);
        Ft = mul(Ft, f);
        Rv[i] = Et;
      }
    }
#pragma unroll
    for (int i = MAXM - 1; i >= 0; --i) {
      const int r = r0 + i;
      if (i < M && r < N && r > k + 1) {
        const D g = mul(nbmh, piv[i + 2]);
        Sb = fma(g, Sb, Rv[i]);
        Gb = mul(Gb, g);
        Rv[i] = Sb;
      }
    }
  }
  {
    const ChainPair cc = scan_pair(Ft, Et, zero<double>(), Gb, Sb, zero<double>(), t, L, tot);
    if (wave_top) {
      D dl = cc.down;
#pragma unroll
      for (int i = 0; i < MAXM; ++i)
        if (i < M) {
          dl = mul(nbmh, mul(piv[i], dl));
          Rv[i] = add(Rv[i], dl);
        }
    } else if (wave_bot) {
      D dl = cc.up;
#pragma unroll
      for (int i = MAXM - 1; i >= 0; --i)
        if (i < M) {
          dl = mul(nbmh, mul(piv[i + 2], dl));
          Rv[i] = add(Rv[i], dl);
        }
    } else {
      D dl = cc.down;
#pragma unroll
      for (int i = 0; i < MAXM; ++i) {
        const int r = r0 + i;
        if (i < M && r < N && r < k) {
          dl = mul(nbmh, mul(piv[i], dl));
          Rv[i] = add(Rv[i], dl);
        }
      }
      dl = cc.up;
#pragma unroll
      for (int i = MAXM - 1; i >= 0; --i) {
        const int r = r0 + i;
        if (i < M && r < N && r > k + 1) {
          dl = mul(nbmh, mul(piv[i + 2], dl));
          Rv[i] = add(Rv[i], dl);
        }
      }
    }
  }

  // ---- 2x2 interface block (rows k, k+1): the lanes holding rows k-1..k+2 publish them
  if (colok && r0 <= k + 2 && r0 + M > k - 1) {
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
  }
  __syncthreads();
  D vk = zero<double>(), vk1 = zero<double>();
  if (Bp) {
    const D ykm1 = slots[cw * 4 + 0], Rk = slots[cw * 4 + 1];
    const D Rk1 = slots[cw * 4 + 2], zk2 = slots[cw * 4 + 3];
    const D rk = fma(Bp->fk, ykm1, Rk);
    const D rk1 = fma(Bp->gk1, zk2, Rk1);
    vk = fma(Bp->i00, rk, mul(Bp->i01, rk1));
    vk1 = fma(Bp->i10, rk, mul(Bp->i11, rk1));
  }

  // ---- back substitution: top rows upward, v_r = pivot_r (y_r + (-beta_- h) v_{r+1});
  //      bottom rows downward, v_r = pivot_r (z_r + (-beta_- h) v_{r-1})
  D Ht = one<double>(), Eu = zero<double>(), Hb = one<double>(), Ed = zero<double>();
  if (wave_top) {
#pragma unroll
    for (int i = MAXM - 1; i >= 0; --i)
      if (i < M) {
        Eu = mul(piv[i + 1], fma(nbmh, Eu, Rv[i]));
        Rv[i] = Eu;
      }
    Ht = lt[2 * L + t];
  } else if (wave_bot) {
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      if (i < M) {
        Ed = mul(piv[i + 1], fma(nbmh, Ed, Rv[i]));
        Rv[i] = Ed;
      }
    Hb = lt[3 * L + t];
  } else {
#pragma unroll
    for (int i = MAXM - 1; i >= 0; --i) {
      const int r = r0 + i;
      if (i < M && r < N) {
        if (r < k) {
          const D p = piv[i + 1];
          Eu = mul(p, fma(nbmh, Eu, Rv[i]));
          Ht = mul(Ht, mul(nbmh, p));
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
        const D p = piv[i + 1];
        Ed = mul(p, fma(nbmh, Ed, Rv[i]));
        Hb = mul(Hb, mul(nbmh, p));
        Rv[i] = Ed;
      }
    }
  }
  {
    // the top chain runs upward and enters from below with v_k; the bottom
    // chain runs downward and enters from above with v_{k+1}
    const ChainPair cc = scan_pair(Hb, Ed, vk1, Ht, Eu, vk, t, L, tot);
    if (wave_top) {
      D dl = cc.up;
#pragma unroll
      for (int i = MAXM - 1; i >= 0; --i)
        if (i < M) {
          dl = mul(piv[i + 1], mul(nbmh, dl));
          Rv[i] = add(Rv[i], dl);
        }
    } else if (wave_bot) {
      D dl = cc.down;
#pragma unroll
      for (int i = 0; i < MAXM; ++i)
        if (i < M) {
          dl = mul(piv[i + 1], mul(nbmh, dl));
          Rv[i] = add(Rv[i], dl);
        }
    } else {
      D dl = cc.up;
#pragma unroll
      for (int i = MAXM - 1; i >= 0; --i) {
        const int r = r0 + i;
        if (i < M && r < N && r < k) {
          dl = mul(piv[i + 1], mul(nbmh, dl));
          Rv[i] = add(Rv[i], dl);
        }
      }
      dl = cc.down;
#pragma unroll
      for (int i = 0; i < MAXM; ++i) {
        const int r = r0 + i;
        if (i < M && r < N && r > k + 1) {
          dl = mul(piv[i + 1], mul(nbmh, dl));
          Rv[i] = add(Rv[i], dl);
        }
      }
    }
  }

  // ---- write back through LDS, coalesced store
  __syncthreads();
  C<S>* myw = lds + cw * stride + t * (M + 1);
#pragma unroll
  for (int i = 0; i < MAXM; ++i) {
    if (i < M && r0 + i < N) myw[i] = from_d<S>(Rv[i]);
  }
  __syncthreads();
  for (int c = 0; c < ncols; ++c) {
    C<S>* col = dst + (size_t)(m0 + c) * N;
    for (int r = lane; r < N; r += kPassAThreads) {
      int q = int((float(r) + 0.5f) * invM);
      col[r] = lds[c * stride + r + q];
    }
  }
}

template <typename S, int MAXM>
constexpr int pass_a_lds() {
  return int(sizeof(C<S>) * kPassAThreads * (MAXM + 1) + sizeof(D) * (4 * 64 + 16));
}

// two workgroups per CU: staging and compute of one overlap the other's memory traffic
#define PE3D_PASS_A_ATTR __launch_bounds__(kPassAThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))

template <typename S, int MAXM>
__global__ PE3D_PASS_A_ATTR void pass_a_single(ProbDesc d, int koff) {
  extern __shared__ __align__(16) unsigned char smem_a[];
  pass_a_body<S, MAXM>(d, blockIdx.x, koff, (C<S>*)smem_a);
}

template <typename S, int MAXM>
__global__ PE3D_PASS_A_ATTR void pass_a_batch(const ProbDesc* __restrict__ descs,
                                                              const WorkItem* __restrict__ items,
                                                              int koff) {
  extern __shared__ __align__(16) unsigned char smem_a[];
  const WorkItem it = items[blockIdx.x];
  const ProbDesc d = descs[it.prob];
  pass_a_body<S, MAXM>(d, it.tile, koff, (C<S>*)smem_a);
}

// ============================================================== pass B
// Per-workgroup FP64 constants of the azimuth solve for one range step.
struct BConst {
  D rho;     // root of s rho^2 - (1+2s) rho + s = 0 inside the unit circle
  D rM;      // rho^M
  D rL;      // rho^lastlen
  D winv;    // 1 / (1 - rho^N)   (periodic closure)
  D sinv;    // 1 / (1 - rho^(2N+2))  (sector first-row correction)
  D lev[6];  // rho^(M 2^l), multipliers of the chunk scan
  double s1; // sigma of the next step (its azimuth factor is applied on store)
};

template <typename S, int MAXM>
__device__ __forceinline__ void pass_b_body(const ProbDesc& d, int tile, int koff) {
  constexpr int NTHR = kPassBThreads;
  // sE1/sC1: forward chunk ends and carries, reused for the edge exchange;
  // sE2/sC2: backward chunk starts and carries, sE2 reused for the sector term
  __shared__ D sE1[NTHR], sC1[NTHR], sE2[NTHR], sC2[NTHR];
  __shared__ D sPow[MAXM + 2];   // rho^i
  __shared__ D sPowC[64];        // rho^(M c), chunk c
  __shared__ D sPowS[64];        // rho^(2N - m0 - len + 1), chunk c (sector)
  __shared__ BConst K;

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
  const int lastlen = NT - (NC - 1) * M;

  const C<S>* __restrict__ src = (const C<S>*)d.scr;
  C<S>* __restrict__ dst = (C<S>*)(last ? d.u : d.scr);

  // ---- load the chunk and its two azimuth neighbours (issued before the prologue)
  C<S> v[MAXM];
  C<S> vl = zero<S>(), vr = zero<S>();
  if (act) {
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      if (i < len) v[i] = src[(size_t)(m0 + i) * N + z];
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
  }

  // ---- FP64 step constants, once per workgroup
  if (tid == 0) {
    const D rho = rho_of(sigma_of(d, j));
    K.rho = rho;
    K.rM = cpow(rho, M);
    K.rL = cpow(rho, lastlen);
    const D rN = cpow(rho, NT);
    K.winv = cdiv(one<double>(), mk<double>(1.0 - rN.re, -rN.im));
    const D r2 = cpow(rho, 2 * (long long)NT + 2);
    K.sinv = cdiv(one<double>(), mk<double>(1.0 - r2.re, -r2.im));
    D lv = K.rM;
    for (int l = 0; l < 6; ++l) {
      K.lev[l] = lv;
      lv = mul(lv, lv);
    }
    K.s1 = sigma_of(d, j + 1);
  }
  __syncthreads();
  const D rho = K.rho;
  if (tid <= MAXM + 1) sPow[tid] = cpow(rho, tid);
  if (tid >= 64 && tid < 128 && tid - 64 < NC) sPowC[tid - 64] = cpow(K.rM, tid - 64);
  if (!periodic && tid >= 128 && tid < 192 && tid - 128 < NC) {
    const int cc = tid - 128;
    const int ln = min(M, NT - cc * M);
    sPowS[cc] = cpow(rho, 2 * (long long)NT - cc * M - ln + 1);
  }

  // ---- D_theta v, forward recurrence y_m = t_m + rho y_{m-1} with zero carry
  D x[MAXM];
  D E = zero<double>();
  {
    D a = to_d(vl), b = (len > 0) ? to_d(v[0]) : zero<double>();
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      if (i < len) {
        const D cdn = (i + 1 < len) ? to_d(v[i + 1]) : to_d(vr);
        const D tt = sub(add(a, cdn), scl(2.0, b));
        E = fma(rho, E, tt);
        x[i] = E;
        a = b;
        b = cdn;
      }
    }
  }
  sE1[tid] = E;
  __syncthreads();
  // ---- carries across chunks (FP64 segmented scan over the chunks of a depth)
  const int NCp = ncp_of(NC);
  if (tid < TD * NCp) {
    const int sd = tid / NCp, sc = tid - sd * NCp;
    const D e = (sc < NC) ? sE1[sc * TD + sd] : zero<double>();
    // inclusive scan over chunks 0..NC-2 (length M each)
    D Sv = (sc < NC - 1) ? e : zero<double>();
    for (int l = 0, dd = 1; dd < NCp; ++l, dd <<= 1) {
      const D up = shfl_up(Sv, dd, NCp);
      if (sc >= dd) Sv = fma(K.lev[l], up, Sv);
    }
    const D Slast = (NC >= 2) ? shfl_idx(Sv, NC - 2, NCp) : zero<double>();
    const D Elast = shfl_idx(e, NC - 1, NCp);
    const D c0 = periodic ? mul(fma(K.rL, Slast, Elast), K.winv) : zero<double>();
    D prev = shfl_up(Sv, 1, NCp);
    if (sc == 0) prev = zero<double>();
    if (sc < NC) sC1[sc * TD + sd] = fma(sPowC[sc], c0, prev);
  }
  __syncthreads();
  {
    const D cin = sC1[tid];
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      if (i < len) x[i] = fma(sPow[i + 1], cin, x[i]);
  }
  // ---- backward recurrence x_m = y_m + rho x_{m+1} with zero carry
  D Sb = zero<double>();
#pragma unroll
  for (int i = MAXM - 1; i >= 0; --i) {
    if (i < len) {
      Sb = fma(rho, Sb, x[i]);
      x[i] = Sb;
    }
  }
  sE2[tid] = Sb;
  __syncthreads();
  // backward chain scanned in reversed chunk order (chunk NC-1 first): the
  // chunk of length lastlen comes first, so only the wrap value sees rho^lastlen
  if (tid < TD * NCp) {
    const int sd = tid / NCp, sr = tid - sd * NCp;
    const D e = (sr < NC) ? sE2[(NC - 1 - sr) * TD + sd] : zero<double>();
    D Sv = e;
    for (int l = 0, dd = 1; dd < NCp; ++l, dd <<= 1) {
      const D up = shfl_up(Sv, dd, NCp);
      if (sr >= dd) Sv = fma(K.lev[l], up, Sv);
    }
    const D c0 = periodic ? mul(shfl_idx(Sv, NC - 1, NCp), K.winv) : zero<double>();
    D prev = shfl_up(Sv, 1, NCp);
    const D cin = (sr == 0) ? c0 : fma(mul(K.rL, sPowC[sr > 0 ? sr - 1 : 0]), c0, prev);
    if (sr < NC) sC2[(NC - 1 - sr) * TD + sd] = cin;
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
      const D Kc = mul(mul(mul(rho, rho), sE2[dl]), K.sinv);
      const D pa = mul(Kc, sPowC[c]);   // K rho^m at i = 0
      const D pbk = mul(Kc, sPowS[c]);  // K rho^{2N-m} at i = len-1
#pragma unroll
      for (int i = 0; i < MAXM; ++i)
        if (i < len)
          x[i] = sub(fma(rho, x[i], to_d(v[i])), sub(mul(pa, sPow[i]), mul(pbk, sPow[len - 1 - i])));
    }
  } else {
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      if (i < len) x[i] = fma(rho, x[i], to_d(v[i]));
  }
  // x now holds u^{j+1}.  Next step's azimuth factor w = u + s_{j+1} D_theta u, or store u.
  if (!last) {
    // start the next step from u^{j+1} as stored (rounded to S), exactly as a
    // new march call would: an interrupted and resumed march is bitwise equal
    // to an uninterrupted one
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      if (i < len) x[i] = to_d(from_d<S>(x[i]));
    D* sUf = sE1;
    D* sUl = sC1;
    sUf[tid] = (len > 0) ? x[0] : zero<double>();
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
      const double s1 = K.s1;
      D a = ul;
#pragma unroll
      for (int i = 0; i < MAXM; ++i) {
        if (i < len) {
          const D b = (i + 1 < len) ? x[i + 1] : ur;
          const D dd = sub(add(a, b), scl(2.0, x[i]));
          dst[(size_t)(m0 + i) * N + z] = from_d<S>(mk<double>(x[i].re - s1 * dd.im, x[i].im + s1 * dd.re));
          a = x[i];
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
  static bool attr = false;  // allow more than the default dynamic LDS once per kernel
  if (!attr) {
    hipError_t e1 = hipFuncSetAttribute(reinterpret_cast<const void*>(&pass_a_single<S, MAXM>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    hipError_t e2 = hipFuncSetAttribute(reinterpret_cast<const void*>(&pass_a_batch<S, MAXM>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e1 != hipSuccess || e2 != hipSuccess) return e1 != hipSuccess ? e1 : e2;
    attr = true;
  }
  if (single) {
    hipLaunchKernelGGL((pass_a_single<S, MAXM>), dim3(single->ntile_a), dim3(kPassAThreads), lds, st,
                       *single, koff);
  } else {
    hipLaunchKernelGGL((pass_a_batch<S, MAXM>), dim3(nitems), dim3(kPassAThreads), lds, st, d_descs,
                       items, koff);
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
  if (maxm == 16) {
    if (prec == 0) return run_a<float, 16>(single, d_descs, items, nitems, koff, st);
    return run_a<double, 16>(single, d_descs, items, nitems, koff, st);
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
