// Host runtime of the PE range march: argument validation, the FP64
// coefficient builder and depth-system factorisation, kernel shape choice,
// the plain per-problem march and the batched march with hipGraph replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <list>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <cstdio>
#include <new>
#include <vector>

#include "pe3d.h"
#include "pe3d_internal.h"

using namespace pe3d;
using cd = std::complex<double>;

namespace {

constexpr double kPi = 3.14159265358979323846;
// k = k_r (1 + i*eta*a) for an attenuation of a dB per wavelength, since
// a = 20 log10(e) k_i lambda
const double kEta = 1.0 / (40.0 * kPi * std::log10(std::exp(1.0)));

bool is_fin(double x) { return std::isfinite(x); }
bool is_periodic(double width) { return width >= 2.0 * kPi * (1.0 - 1e-12); }

int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// ------------------------------------------------------------------ uploads
// Host-to-device copies of set-up data (coefficient tables, batch plans) go
// through a non-blocking stream of the library's own, one per device, at the
// default priority, and only that stream is waited for: a copy does not wait
// for kernels the caller has queued (a copy on the legacy default stream
// would).
hipError_t upload(void* dst, const void* src, size_t n) {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  hipStream_t s = nullptr;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = streams.find(dev);
    if (it != streams.end()) {
      s = it->second;
    } else {
      e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
      if (e != hipSuccess) return e;
      streams[dev] = s;
    }
  }
  e = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

// ------------------------------------------------------------------ device pool
// Device memory of handles (tables, scratch field) and batch plans comes from
// a per-device pool: a released block is kept and handed to a later request
// of the same size class instead of being returned with hipFree, which waits
// for the whole device (a served stream creates and destroys handles while
// other requests' work runs).  Size classes: multiples of 64 KiB up to
// 1 MiB, then 8 steps per power of two (at most 12.5 % above the request).
// Pooled blocks are returned to the runtime only when an allocation fails.
size_t pool_class(size_t n) {
  const size_t g0 = size_t(64) << 10;
  if (n <= (size_t(1) << 20)) return (std::max<size_t>(n, 1) + g0 - 1) / g0 * g0;
  size_t p = size_t(1) << 20;
  while (p * 2 <= n) p *= 2;
  const size_t g = p / 8;
  return (n + g - 1) / g * g;
}
std::mutex g_pool_mu;
std::map<std::pair<int, size_t>, std::vector<void*>> g_pool_free;  // (device, class) -> blocks
std::map<void*, std::pair<int, size_t>> g_pool_live;               // live block -> (device, class)

hipError_t pool_alloc(void** out, size_t n) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const size_t c = pool_class(n);
  std::lock_guard<std::mutex> lk(g_pool_mu);
  auto it = g_pool_free.find({dev, c});
  if (it != g_pool_free.end() && !it->second.empty()) {
    *out = it->second.back();
    it->second.pop_back();
    g_pool_live[*out] = {dev, c};
    return hipSuccess;
  }
  e = hipMalloc(out, c);
  if (e != hipSuccess) {
    // give the pooled blocks of this device back and try once more
    (void)hipGetLastError();
    for (auto& kv : g_pool_free)
      if (kv.first.first == dev) {
        for (void* b : kv.second) (void)hipFree(b);
        kv.second.clear();
      }
    e = hipMalloc(out, c);
    if (e != hipSuccess) return e;
  }
  g_pool_live[*out] = {dev, c};
  return hipSuccess;
}

// Free every pooled (idle) block; returns the bytes freed.
size_t pool_trim() {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  size_t n = 0;
  for (auto& kv : g_pool_free) {
    for (void* b : kv.second) {
      (void)hipFree(b);
      n += kv.first.second;
    }
    kv.second.clear();
  }
  return n;
}

// The block must no longer be used by any enqueued work.
void pool_release(void* b) {
  if (!b) return;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  auto it = g_pool_live.find(b);
  if (it == g_pool_live.end()) return;
  g_pool_free[it->second].push_back(b);
  g_pool_live.erase(it);
}

// The device blocks of a destroyed handle, released to the pool when the
// last plan that used the handle is freed (its last work has finished).
struct HandleBlocks {
  void* tables = nullptr;
  void* scr = nullptr;
  ~HandleBlocks() {
    pool_release(scr);
    pool_release(tables);
  }
};

// ------------------------------------------------------------------ validation
pe3d_status validate(const pe3d_env* e, const pe3d_grid* g, const pe3d_freq* f) {
  if (!e || !g || !f) return PE3D_EINVAL;
  if (!is_fin(f->f_hz) || f->f_hz <= 0.0) return PE3D_EINVAL;
  if (!is_fin(e->c0) || e->c0 <= 0.0) return PE3D_EINVAL;
  if (e->n_ssp < 1 || !e->ssp_z || !e->ssp_c) return PE3D_EINVAL;
  if (e->n_ssp_r < 0 || e->n_ssp_r > 100000) return PE3D_EINVAL;
  if (e->n_ssp_r >= 2 && (!is_fin(e->ssp_r0) || !is_fin(e->ssp_dr) || e->ssp_dr <= 0.0)) return PE3D_EINVAL;
  for (int i = 0; i < e->n_ssp; ++i) {
    if (!is_fin(e->ssp_z[i])) return PE3D_EINVAL;
    if (i > 0 && !(e->ssp_z[i] > e->ssp_z[i - 1])) return PE3D_EINVAL;
  }
  for (long long i = 0; i < (long long)e->n_ssp * std::max(e->n_ssp_r, 1); ++i)
    if (!is_fin(e->ssp_c[i]) || e->ssp_c[i] <= 0.0) return PE3D_EINVAL;
  if (!is_fin(e->rho_w) || e->rho_w <= 0.0 || !is_fin(e->atten_w) || e->atten_w < 0.0) return PE3D_EINVAL;
  if (!is_fin(e->c_b) || e->c_b <= 0.0 || !is_fin(e->rho_b) || e->rho_b <= 0.0 ||
      !is_fin(e->atten_b) || e->atten_b < 0.0)
    return PE3D_EINVAL;
  if (e->n_bathy < 1 || !e->bathy_theta || !e->bathy_depth) return PE3D_EINVAL;
  if (e->n_bathy_r < 0 || e->n_bathy_r > 1000000) return PE3D_EINVAL;
  if (e->n_bathy_r >= 2 && (!is_fin(e->bathy_r0) || !is_fin(e->bathy_dr) || e->bathy_dr <= 0.0))
    return PE3D_EINVAL;
  for (int i = 0; i < e->n_bathy; ++i) {
    if (!is_fin(e->bathy_theta[i])) return PE3D_EINVAL;
    if (i > 0 && !(e->bathy_theta[i] > e->bathy_theta[i - 1])) return PE3D_EINVAL;
  }
  for (long long i = 0; i < (long long)e->n_bathy * std::max(e->n_bathy_r, 1); ++i)
    if (!is_fin(e->bathy_depth[i])) return PE3D_EINVAL;
  if (e->n_bathy > 1 && !(e->bathy_theta[e->n_bathy - 1] - e->bathy_theta[0] < 2.0 * kPi))
    return PE3D_EINVAL;
  if (!is_fin(e->zmax) || e->zmax <= 0.0) return PE3D_EINVAL;
  if (e->floor != PE3D_FLOOR_PRESSURE_RELEASE && e->floor != PE3D_FLOOR_RIGID) return PE3D_EINVAL;
  if (g->nz < 2) return PE3D_EINVAL;
  if (!is_fin(g->theta0) || !is_fin(g->width) || g->width <= 0.0) return PE3D_EINVAL;
  if (is_periodic(g->width) ? g->ntheta < 3 : g->ntheta < 1) return PE3D_EINVAL;
  if (!is_fin(g->dr) || g->dr <= 0.0 || !is_fin(g->r0) || g->r0 < 0.0) return PE3D_EINVAL;
  if (g->precision != PE3D_C64 && g->precision != PE3D_C128) return PE3D_EINVAL;
  if (g->mode != PE3D_MODE_3D && g->mode != PE3D_MODE_NX2D) return PE3D_EINVAL;
  auto pow2_in = [](int v, int lo, int hi) { return v == 0 || (v >= lo && v <= hi && (v & (v - 1)) == 0); };
  if (!pow2_in(g->depth_lanes, 4, 256) || !pow2_in(g->azimuth_lanes, 1, 64)) return PE3D_EINVAL;
  if (g->azimuth_solver != PE3D_AZIMUTH_CHUNKED && g->azimuth_solver != PE3D_AZIMUTH_PCR) return PE3D_EINVAL;
  if (g->azimuth_solver == PE3D_AZIMUTH_PCR && g->azimuth_lanes != 0) return PE3D_EINVAL;
  if (g->precision == PE3D_C64 && (g->nz > 4096 || g->ntheta > 1024)) return PE3D_EUNSUPPORTED;
  if (g->precision == PE3D_C128 && (g->nz > 4096 || g->ntheta > 1024)) return PE3D_EUNSUPPORTED;
  return PE3D_OK;
}

// ------------------------------------------------------------------ medium
double interp_ssp(const pe3d_env& e, double z) {
  const int n = e.n_ssp;
  if (n == 1 || z <= e.ssp_z[0]) return e.ssp_c[0];
  if (z >= e.ssp_z[n - 1]) return e.ssp_c[n - 1];
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (e.ssp_z[mid] <= z) lo = mid;
    else hi = mid;
  }
  // same evaluation order as the usual linear-interpolation formula:
  // slope * (z - z_lo) + c_lo
  double slope = (e.ssp_c[hi] - e.ssp_c[lo]) / (e.ssp_z[hi] - e.ssp_z[lo]);
  return slope * (z - e.ssp_z[lo]) + e.ssp_c[lo];
}

// D(theta) of one depth row dep[0..n_bathy-1]
double interp_bathy(const pe3d_env& e, const double* dep, double th) {
  const int n = e.n_bathy;
  if (n == 1) return dep[0];
  const double t0 = e.bathy_theta[0];
  double md = std::fmod(th - t0, 2.0 * kPi);
  if (md < 0.0) md += 2.0 * kPi;
  const double t = t0 + md;
  // segment i covers [theta_i, theta_{i+1}); the last one wraps to theta_0 + 2 pi
  for (int i = 0; i < n; ++i) {
    double a = e.bathy_theta[i];
    double b = (i + 1 < n) ? e.bathy_theta[i + 1] : t0 + 2.0 * kPi;
    if (t >= a && t < b) {
      double da = dep[i];
      double db = (i + 1 < n) ? dep[i + 1] : dep[0];
      if (t == a) return da;
      double slope = (db - da) / (b - a);
      return slope * (t - a) + da;
    }
  }
  return dep[0];
}

// D at range r from a column's depths dc[i] at ranges r_i = r0b + i*drb
// (i < nr, nr >= 2): the interval [r_i, r_{i+1}) holding r, the depth at an
// exact node, slope * (r - r_i) + dc[i] inside, the end values outside.  The
// depth kernel evaluates the same operations (no fused multiply-add), so
// both sides count the same water nodes.
double depth_in_range(const double* dc, int nr, double r0b, double drb, double r) {
  auto node = [&](int i) { return r0b + double(i) * drb; };
  if (r <= node(0)) return dc[0];
  if (r >= node(nr - 1)) return dc[nr - 1];
  int i = 0, hi = nr - 1;  // node(i) < r < node(hi)
  while (hi - i > 1) {
    const int mid = (i + hi) / 2;
    if (node(mid) <= r) i = mid; else hi = mid;
  }
  const double ra = node(i);
  if (r == ra) return dc[i];
  const double slope = (dc[i + 1] - dc[i]) / (node(i + 1) - ra);
  return slope * (r - ra) + dc[i];
}

// water nodes of a column of depth D: #{l = 1..N : l dz <= D}
int water_count(double D, double dz, int N) {
  int nw = 0;
  while (nw < N && double(nw + 1) * dz <= D) ++nw;
  return nw;
}

// FP64 problem description built on the host
struct Built {
  int N = 0, NT = 0, prec = 0, periodic = 0, rigid = 0;
  double k0 = 0, dz = 0, dth = 0, h = 0;
  cd qb, bp, bm;
  cd cbs;  // beta_+ h / (-beta_- h): off-diagonal of the scaled depth RHS
  std::vector<cd> qw, pw, pb;
  std::vector<cd> tabG, tabC, tabP;  // depth-kernel chain tables and lane products
  std::vector<int> nw, k;                // water nodes and interface row of each column at r0
  std::vector<std::array<cd, 12>> rec;  // interface rows by water count nw = 0..N
  std::vector<double> dcol;             // [NT][nbr] column depths at the range rows
  int nbr = 0;                          // range rows (0: range independent)
  double br0 = 0, bdr = 0;
  int nsr = 0;                          // water-profile rows (0: one profile)
  double sr0 = 0, sdr = 0;
  int la_req = 0, lb_req = 0;           // requested lanes (0: the rule)
  int bsolver = 0;                      // pe3d_azimuth_solver
  int lpc = 0, ma = 0, lt = 0, ntile_a = 0;
  int bconv[2] = {0, 0};   // first row of each chain's converged tail
  cd gtail[2], ctail[2];   // the tail's Gh and RHS diagonal / nbmh
  int wb = 0, nc = 0, td = 0, mb = 0, maxm_b = 0, ntile_b = 0;
};


// Kernel shapes (see pe3d_kernels.hip): pass A uses L lanes per column with M
// rows per lane; pass B uses nc azimuth chunks of mb nodes times td depths.
pe3d_status choose_shapes(Built& b) {
  const int N = b.N, NT = b.NT;
  // pass A: the fewest lanes L (power of two, 4..256) with M = ceil((nz+1)/(L-1))
  // rows per lane, rounded up to an odd number (conflict-free LDS strides),
  // at most 17; nz <= (L-1) M - 1 leaves room for the two chains' leading
  // zero slots in every column
  int L = b.la_req ? b.la_req : 4, M = 0;
  for (;; L *= 2) {
    if (L > 256) return PE3D_EUNSUPPORTED;
    M = (N + 1 + L - 2) / (L - 1);
    if (M % 2 == 0) ++M;
    if (M < 3) M = 3;
    if (M <= 17) break;
    if (b.la_req) return PE3D_EUNSUPPORTED;  // the requested lanes need > 17 rows each
  }
  b.lpc = L;
  b.ma = M;
  b.lt = (N + 3 * M - 1) / M;
  const int cpw = 256 / L;
  b.ntile_a = (NT + cpw - 1) / cpw;

  if (b.bsolver == PE3D_AZIMUTH_PCR) {
    // pass B by cyclic reduction: tiles of pcr_td(NT) depths, whole lines
    b.wb = 0;
    b.nc = 0;
    b.mb = 0;
    b.td = pcr_td(NT);
    b.maxm_b = kPcrClass;
    b.ntile_b = (N + b.td - 1) / b.td;
    return PE3D_OK;
  }
  // pass B: the fewest lanes W per depth line (power of two, 1..64) with chunks
  // of M = ceil(nth / W) <= 16 azimuths; lines of exactly W*M azimuths with
  // M >= 9 use the kernel specialised for M (class M), others the general
  // kernel (class 0)
  int W = 1;
  while ((NT + W - 1) / W > 16) W *= 2;
  if (W > 64) return PE3D_EUNSUPPORTED;
  if (b.lb_req) {
    if (b.lb_req < W) return PE3D_EUNSUPPORTED;  // > 16 azimuths per lane
    W = b.lb_req;
  }
  const int mb = (NT + W - 1) / W;
  b.wb = W;
  b.mb = mb;
  b.nc = (NT + mb - 1) / mb;
  b.td = kPassBThreads / W;
  b.maxm_b = (NT == W * mb && mb >= 9) ? mb : 0;
  b.ntile_b = (N + b.td - 1) / b.td;
  return PE3D_OK;
}

// Build the medium, the depth operator X and the factorisation of
// [I + beta_- X] (Eqs. (4), (5), (7)).  The medium is water above D(theta)
// and a homogeneous half-space below, so every column equals the all-water
// column above its interface rows and the all-bottom column below them; the
// shared pivots of those two columns (top-down and bottom-up) plus a 2x2
// interface block per column factor every depth system exactly.
pe3d_status build(const pe3d_env& e, const pe3d_grid& g, const pe3d_freq& f, Built& b) {
  const int N = g.nz, NT = g.ntheta;
  b.N = N;
  b.NT = NT;
  b.prec = g.precision;
  b.la_req = g.depth_lanes;
  b.lb_req = g.azimuth_lanes;
  b.bsolver = g.azimuth_solver;
  b.rigid = e.floor == PE3D_FLOOR_RIGID;
  b.periodic = is_periodic(g.width);
  b.k0 = 2.0 * kPi * f.f_hz / e.c0;
  b.dz = b.rigid ? e.zmax / N : e.zmax / (N + 1);
  b.dth = b.periodic ? 2.0 * kPi / NT : g.width / (NT + 1);
  b.h = 1.0 / ((b.k0 * b.dz) * (b.k0 * b.dz));
  b.bp = cd(1.0, b.k0 * g.dr) / 4.0;
  b.bm = cd(1.0, -b.k0 * g.dr) / 4.0;
  const double h = b.h;
  const cd bm = b.bm;
  auto nsq = [&](double c, double a) {
    cd n = cd(1.0, kEta * a);
    return (e.c0 / c) * (e.c0 / c) * n * n - 1.0;
  };
  b.qb = nsq(e.c_b, e.atten_b);
  b.qw.resize(N);
  for (int l = 0; l < N; ++l) b.qw[l] = nsq(interp_ssp(e, (l + 1) * b.dz), e.atten_w);

  // all-water and all-bottom columns: X diagonals with uniform density
  auto col_x = [&](int l, cd q, cd& xl, cd& xd, cd& xu) {
    xl = (l == 0) ? 0.0 : h;
    xu = (l == N - 1) ? 0.0 : h;
    xd = q - 2.0 * h;
    if (l == N - 1 && b.rigid) xl = 2.0 * h;
  };
  // top-down pivots of the all-water column
  b.pw.assign(N, 0.0);
  std::vector<cd> dw(N);
  {
    cd cprev = 0.0;
    for (int l = 0; l < N; ++l) {
      cd xl, xd, xu;
      col_x(l, b.qw[l], xl, xd, xu);
      cd a = bm * xl, bb = 1.0 + bm * xd, c = bm * xu;
      dw[l] = (l == 0) ? bb : bb - a * cprev / dw[l - 1];
      cprev = c;
      b.pw[l] = 1.0 / dw[l];
    }
  }
  // bottom-up pivots of the all-bottom column; a rigid floor row is divided
  // by 2 so that its lower coefficient is beta_- h like the other bottom rows
  b.pb.assign(N, 0.0);
  std::vector<cd> eb(N);
  const double floor_scale = b.rigid ? 0.5 : 1.0;
  {
    cd anext = 0.0;
    for (int l = N - 1; l >= 0; --l) {
      cd xl, xd, xu;
      col_x(l, b.qb, xl, xd, xu);
      cd a = bm * xl, bb = 1.0 + bm * xd, c = bm * xu;
      if (l == N - 1) {
        a *= floor_scale;
        bb *= floor_scale;
      }
      eb[l] = (l == N - 1) ? bb : bb - c * anext / eb[l + 1];
      anext = a;
      b.pb[l] = 1.0 / eb[l];
    }
  }
  // water nodes of every column: at r0 (the only depth when it has no range
  // rows); with range rows the column's depths at the row ranges, from which
  // the depth kernel finds the water nodes at r_{j+1} every step
  b.nbr = e.n_bathy_r >= 2 ? e.n_bathy_r : 0;
  b.br0 = e.bathy_r0;
  b.bdr = e.bathy_dr;
  b.nsr = e.n_ssp_r >= 2 ? e.n_ssp_r : 0;
  b.sr0 = e.ssp_r0;
  b.sdr = e.ssp_dr;
  b.nw.resize(NT);
  b.k.resize(NT);
  if (b.nbr) b.dcol.assign((size_t)NT * b.nbr, 0.0);
  int nwlo = N, nwhi = 0;
  for (int m = 0; m < NT; ++m) {
    double th = b.periodic ? g.theta0 + m * b.dth : g.theta0 - 0.5 * g.width + (m + 1) * b.dth;
    double D;
    if (b.nbr) {
      double* dc = b.dcol.data() + (size_t)m * b.nbr;
      for (int i = 0; i < b.nbr; ++i) {
        dc[i] = interp_bathy(e, e.bathy_depth + (size_t)i * e.n_bathy, th);
        // interpolated depths lie between row values: their water counts bound
        // every count the march meets (widened by one for rounding)
        const int c = water_count(dc[i], b.dz, N);
        nwlo = std::min(nwlo, std::max(c - 1, 0));
        nwhi = std::max(nwhi, std::min(c + 1, N));
      }
      D = depth_in_range(dc, b.nbr, b.br0, b.bdr, g.r0);
    } else {
      D = interp_bathy(e, e.bathy_depth, th);
    }
    const int nw = water_count(D, b.dz, N);
    b.nw[m] = nw;
    b.k[m] = std::min(std::max(nw - 1, 0), N - 2);
    nwlo = std::min(nwlo, nw);
    nwhi = std::max(nwhi, nw);
  }
  // interface record for every water count nw = 0..N (interface row
  // k = clamp(nw - 1, 0, N - 2)); the pivot check covers the counts met
  b.rec.assign(N + 1, {});
  double maxb = 0.0, minpiv = 1e300;
  const int kmin = std::min(std::max(nwlo - 1, 0), N - 2), kmax = std::min(std::max(nwhi - 1, 0), N - 2);
  const cd bp = b.bp;
  for (int nw = 0; nw <= N; ++nw) {
    const int k = std::min(std::max(nw - 1, 0), N - 2);
    const bool used = nw >= nwlo && nw <= nwhi;
    // the column's own X rows k-1..k+2 from the density-weighted operator
    auto rho_at = [&](int l) {
      l = std::min(std::max(l, 0), N - 1);  // ghost densities
      return l < nw ? e.rho_w : e.rho_b;
    };
    auto q_at = [&](int l) { return l < nw ? b.qw[l] : b.qb; };
    auto xrow = [&](int l, cd& xl, cd& xd, cd& xu) {
      double rm = rho_at(l - 1), r = rho_at(l), rp = rho_at(l + 1);
      double lm = 2.0 * r / (rm + r), lp = 2.0 * r / (r + rp);
      xl = (l == 0) ? 0.0 : h * lm;
      xd = q_at(l) - h * (lm + lp);
      xu = h * lp;
      if (l == N - 1) {
        if (b.rigid) xl += xu;
        xu = 0.0;
      }
    };
    cd xl0, xd0, xu0, xl1, xd1, xu1;
    xrow(k, xl0, xd0, xu0);
    xrow(k + 1, xl1, xd1, xu1);
    // eliminating row k-1 (top chain) into row k and row k+2 (bottom chain)
    // into row k+1 leaves the 2x2 block [[P, c01], [c10, Q]]
    const cd cft = -(bm * xl0), cfb = -(bm * xu1);
    cd P = 1.0 + bm * xd0, Q = 1.0 + bm * xd1;
    if (k >= 1) {
      cd pxl, pxd, pxu;
      xrow(k - 1, pxl, pxd, pxu);  // a water row: its upper coefficient is h
      P += cft * b.pw[k - 1] * (bm * pxu);
    }
    if (k + 2 <= N - 1) {
      cd nxl, nxd, nxu;
      xrow(k + 2, nxl, nxd, nxu);  // a bottom row (halved if it is the rigid floor)
      if (k + 2 == N - 1) nxl *= floor_scale;
      Q += cfb * b.pb[k + 2] * (bm * nxl);
    }
    cd c01 = bm * xu0, c10 = bm * xl1;
    cd det = P * Q - c01 * c10;
    if (!used) {
      if (det == 0.0 || !std::isfinite(std::abs(det))) continue;  // never read
    } else {
      maxb = std::max({maxb, std::abs(P), std::abs(Q)});
      minpiv = std::min(minpiv, std::abs(det) / std::max(std::abs(P), std::abs(Q)));
      if (det == 0.0 || !std::isfinite(std::abs(det))) return PE3D_EUNSUPPORTED;
    }
    cd id = 1.0 / det;
    // row k (top chain: previous row k-1, next row k+1), then row k+1
    // (bottom chain, reversed: previous row k+2, next row k).  The kernel
    // carries right-hand sides divided by nbmh = -beta_- h (see below), so
    // the RHS and elimination coefficients are divided by nbmh and the
    // inverse entries multiplied by it.
    const cd nb = -bm * h, inb = 1.0 / nb;
    b.rec[nw] = {(1.0 + bp * xd0) * inb, bp * xl0 * inb, bp * xu0 * inb, cft * inb, Q * id * nb, -c01 * id * nb,
                (1.0 + bp * xd1) * inb, bp * xu1 * inb, bp * xl1 * inb, cfb * inb, P * id * nb, -c10 * id * nb};
  }
  // pivots actually used: water rows < kmax, bottom rows > kmin + 1
  for (int l = 0; l < kmax; ++l) {
    minpiv = std::min(minpiv, std::abs(dw[l]));
    maxb = std::max(maxb, std::abs(1.0 + bm * (b.qw[l] - 2.0 * h)));
  }
  for (int l = kmin + 2; l < N; ++l) {
    minpiv = std::min(minpiv, std::abs(eb[l]));
    maxb = std::max(maxb, std::abs(1.0 + bm * (b.qb - 2.0 * h)));
  }
  if (!(minpiv > 1e-10 * maxb)) return PE3D_EUNSUPPORTED;
  pe3d_status st = choose_shapes(b);
  if (st != PE3D_OK) return st;

  // chain tables: chain 0 = rows 0..N-2 of the all-water column (top-down
  // pivots), chain 1 = rows N-1..1 of the all-bottom column (bottom-up
  // pivots, chain row bb = N-1-l); chain row r at [(r+M) % M][(r+M) / M].
  // With nbmh = -beta_- h (the off-diagonal of every non-interface row) and
  // right-hand sides carried divided by nbmh, the elimination is
  // yh_r = Gh_r (Rt_r + yh_{r-1}) and the back substitution
  // x_r = yh_r + Gh_r x_{r+1}, Gh_r = nbmh / pivot_r: tabG holds Gh and tabC
  // the diagonal of [I + beta_+ X] divided by nbmh.
  const int L = b.lpc, M = b.ma, LT = b.lt;
  const size_t MLT = (size_t)M * LT;
  const cd nbmh = -bm * h, inb = 1.0 / nbmh;
  b.cbs = bp * h * inb;
  b.tabG.assign(2 * MLT, 0.0);
  b.tabC.assign(2 * MLT, 0.0);
  auto tix = [&](int r) { const int rp = r + M; return (size_t)(rp % M) * LT + rp / M; };
  for (int r = 0; r <= N - 2; ++r) {
    b.tabG[tix(r)] = nbmh * b.pw[r];
    b.tabC[tix(r)] = (1.0 + bp * (b.qw[r] - 2.0 * h)) * inb;
  }
  for (int bb = 0; bb <= N - 2; ++bb) {
    b.tabG[MLT + tix(bb)] = nbmh * b.pb[N - 1 - bb];
    cd c = 1.0 + bp * (b.qb - 2.0 * h);
    if (bb == 0) c *= floor_scale;
    b.tabC[MLT + tix(bb)] = c * inb;
  }
  // converged tails: a uniform stretch of a chain (the whole bottom column;
  // the water column where the sound speed is constant) has a constant RHS
  // diagonal and pivots that converge geometrically.  From chain row
  // bconv[ch] on, every row's diagonal equals the chain's last one and its
  // Gh is within 2^-51 of the last one's; those rows take exactly the last
  // row's values (a change within the recurrence's own rounding).  Wavefronts
  // of the depth kernel whose lanes hold only tail and zero rows use these
  // constants instead of reading the tables.
  for (int ch = 0; ch < 2; ++ch) {
    const cd gl = b.tabG[ch * MLT + tix(N - 2)], cl = b.tabC[ch * MLT + tix(N - 2)];
    int bc = N - 2;
    while (bc > 0) {
      const cd g = b.tabG[ch * MLT + tix(bc - 1)], c = b.tabC[ch * MLT + tix(bc - 1)];
      if (c != cl || !(std::abs(g - gl) <= 0x1p-51 * std::abs(gl))) break;
      --bc;
    }
    for (int r = bc; r <= N - 2; ++r) b.tabG[ch * MLT + tix(r)] = gl;
    b.bconv[ch] = bc;
    b.gtail[ch] = gl;
    b.ctail[ch] = cl;
  }
  // lane products by (chain, leading zero slots sc = 1..M, lane in chain tc):
  // slot j of the lane holds chain row tc*M + j - sc
  b.tabP.assign((size_t)2 * (M + 1) * L, 0.0);
  for (int ch = 0; ch < 2; ++ch)
    for (int sc = 1; sc <= M; ++sc)
      for (int tc = 0; tc < L; ++tc) {
        cd p = 1.0;
        for (int j = 0; j < M; ++j) {
          const int r = tc * M + j - sc;
          p *= (r + M < (int)MLT) ? b.tabG[ch * MLT + tix(r)] : cd(0.0);
        }
        b.tabP[((size_t)ch * (M + 1) + sc) * L + tc] = p;
      }
  return PE3D_OK;
}

// Device image of a handle: one block of depth-pass tables per water row
// (tabG, tabC, tabP, the interface records), then the column depths at
// the depth rows, the water nodes per column, the table pointers of the
// current step and the step counter.  Coefficient tables are FP64 in both precisions.
struct Layout {
  size_t o_G, o_C, o_P, o_rec, row_bytes;  // within a row block
  size_t o_dc, o_k, o_cur, o_j, total;           // in the image
};
Layout layout(const Built& b) {
  const size_t csz = 16;
  Layout y;
  y.o_G = 0;
  y.o_C = y.o_G + 2 * (size_t)b.ma * b.lt * csz;
  y.o_P = y.o_C + 2 * (size_t)b.ma * b.lt * csz;
  y.o_rec = y.o_P + 2 * (size_t)(b.ma + 1) * b.lpc * csz;
  y.row_bytes = (y.o_rec + (size_t)(b.N + 1) * 12 * csz + 255) & ~size_t(255);
  y.o_dc = y.row_bytes * (size_t)std::max(b.nsr, 1);
  y.o_k = y.o_dc + (size_t)b.NT * b.nbr * sizeof(double);
  y.o_cur = (y.o_k + (size_t)b.NT * sizeof(int) + 63) & ~size_t(63);
  y.o_j = (y.o_cur + sizeof(TabPtrs) + 255) & ~size_t(255);
  y.total = y.o_j + 256;
  return y;
}
size_t table_bytes(const Built& b) { return layout(b).total; }
size_t field_bytes(const Built& b) { return (size_t)b.N * b.NT * (b.prec ? 16 : 8); }

template <typename R>
void pack(const std::vector<cd>& v, std::vector<unsigned char>& out, size_t off) {
  R* p = reinterpret_cast<R*>(out.data() + off);
  for (size_t i = 0; i < v.size(); ++i) {
    p[2 * i] = R(v[i].real());
    p[2 * i + 1] = R(v[i].imag());
  }
}

}  // namespace

// ------------------------------------------------------------------ handle


struct pe3d_handle_s {
  int prec = 0;
  int maxm_a = 0, maxm_b = 0;
  int lds_a = 0, lds_b = 0;  // dynamic LDS of a pass A / pass B workgroup
  ProbDesc desc{};
  void* d_tables = nullptr;
  void* d_scr = nullptr;
  long long* d_j = nullptr;
  long long j = 0;
  size_t bytes = 0;
  int device = 0;
  double r0 = 0, dr = 0;
  // the stream of the last work enqueued for the handle (destroy releases
  // the device memory only once that work has finished)
  bool used = false;
  hipStream_t last = nullptr;
};

namespace {

struct BatchPlan {
  std::vector<uintptr_t> key;
  std::vector<pe3d_handle> handles;
  int prec = 0;
  void* d_mem = nullptr;               // descs, items, jdev pointers, adds
  ProbDesc* d_descs = nullptr;
  long long** d_jdevs = nullptr;
  int* d_adds = nullptr;
  int n = 0;
  struct Class {
    int maxm;
    int lds = 0;                       // dynamic LDS (largest of the class)
    WorkItem* d_items = nullptr;
    std::vector<WorkItem> h_items;     // host copy until the image is uploaded
    std::vector<int> nitems_at;        // active items at step k (problems sorted by steps)
    std::vector<double> bytes_prefix;  // algorithmic bytes of the first i items
  };
  // A group of problems marched through all of its steps before the next
  // group of its chain starts (its field stays in the last-level cache).
  struct Group {
    int maxsteps = 0;
    std::vector<Class> a, b, u;        // depth pass, azimuth pass, medium update
  };
  // Chains are independent: chain 0 runs on the caller's stream, the others
  // on the device's side streams (shared by all plans of the device).
  std::vector<std::vector<Group>> chains;
  std::vector<hipGraphExec_t> execs;
  std::vector<hipGraph_t> graphs;
  std::vector<hipStream_t> side;       // chains 1.. (not owned)
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  hipEvent_t done = nullptr;           // recorded after the plan's latest use
  ~BatchPlan() {
    for (auto e : execs) (void)hipGraphExecDestroy(e);
    for (auto g : graphs) (void)hipGraphDestroy(g);
    for (auto e : join) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    if (done) (void)hipEventDestroy(done);
    pool_release(d_mem);
  }
  // device blocks of destroyed handles this plan used: released with it
  std::vector<std::shared_ptr<HandleBlocks>> keep;
  // persistent kernel (pe3d_set_batch_kernel): its task list, the launch's
  // control words and per-problem counters (persist_ctl_ints(n) ints, zeroed
  // by the launch)
  bool persist = false;
  PTask* d_tasks = nullptr;
  int ntasks = 0;
  int* d_ctl = nullptr;
  int lds_p = 0;
  double bytes_p = 0.0;       // algorithmic bytes of the whole call
  long long wait_ticks = 0;
};

// Batch schedule (pe3d_set_batch_schedule): independent chains replayed on
// concurrent streams, and the bytes of field a group may hold.
constexpr int kMaxChains = 4;
std::atomic<int> g_chains{2};
std::atomic<long long> g_group_bytes{112ll << 20};

// Batch kernel (pe3d_set_batch_kernel) and the persistent kernel's wait limit.
std::atomic<int> g_batch_kernel{PE3D_BATCH_LAUNCHES};
std::atomic<double> g_wait_limit_s{1.0};

constexpr int kBatchClass = -1;  // profiling name "batch"

std::mutex g_mu;
std::map<std::vector<uintptr_t>, std::unique_ptr<BatchPlan>> g_plans;
std::list<std::vector<uintptr_t>> g_lru;  // most recent first
constexpr size_t kMaxPlans = 64;

void touch(const std::vector<uintptr_t>& key) {
  for (auto it = g_lru.begin(); it != g_lru.end(); ++it)
    if (*it == key) {
      g_lru.erase(it);
      break;
    }
  g_lru.push_front(key);
}

// Evicted plans wait here until the work they enqueued has finished (their
// `done` event), so that eviction never waits for the device.
std::vector<std::unique_ptr<BatchPlan>> g_graveyard;

// Device blocks of destroyed handles waiting for the handle's last work
// (an event recorded on its last stream at destroy).
struct Deferred {
  hipEvent_t ev = nullptr;
  std::shared_ptr<HandleBlocks> blocks;
};
std::vector<Deferred> g_deferred;

// Caller holds g_mu.
void reap() {
  for (auto it = g_graveyard.begin(); it != g_graveyard.end();) {
    const hipEvent_t e = (*it)->done;
    if (!e || hipEventQuery(e) != hipErrorNotReady) it = g_graveyard.erase(it);
    else ++it;
  }
  for (auto it = g_deferred.begin(); it != g_deferred.end();) {
    if (!it->ev || hipEventQuery(it->ev) != hipErrorNotReady) {
      if (it->ev) (void)hipEventDestroy(it->ev);
      it = g_deferred.erase(it);
    } else {
      ++it;
    }
  }
}

// Caller holds g_mu.
void evict_if_full() {
  while (g_plans.size() >= kMaxPlans && !g_lru.empty()) {
    auto it = g_plans.find(g_lru.back());
    if (it != g_plans.end()) {
      g_graveyard.push_back(std::move(it->second));
      g_plans.erase(it);
    }
    g_lru.pop_back();
  }
  reap();
}

// Side streams per device (default priority, non-blocking), created on first
// use and kept until the process ends.  Caller holds g_mu.
std::map<int, std::vector<hipStream_t>> g_side_streams;

// ------------------------------------------------------------------ profiling
struct ProfRec {
  int name;
  double bytes;
  hipEvent_t a, b;
};
std::mutex g_pmu;
std::atomic<bool> g_prof{false};  // read on every launch without the lock
std::vector<std::string> g_pnames;
std::vector<ProfRec> g_precs;
std::vector<hipEvent_t> g_epool;

hipEvent_t take_event() {
  if (!g_epool.empty()) {
    hipEvent_t e = g_epool.back();
    g_epool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int prof_name(const char* pass, int prec, int maxm) {
  char buf[48];
  if (maxm < 0) std::snprintf(buf, sizeof buf, "%s<%s,batch>", pass, prec ? "c128" : "c64");
  else std::snprintf(buf, sizeof buf, "%s<%s,%d>", pass, prec ? "c128" : "c64", maxm);
  for (size_t i = 0; i < g_pnames.size(); ++i)
    if (g_pnames[i] == buf) return int(i);
  g_pnames.push_back(buf);
  return int(g_pnames.size() - 1);
}

// Launch through `fn`, bracketed by events when profiling is on (and the
// launch is not being captured into a graph: `allow` false).
template <typename F>
hipError_t prof_launch(const char* pass, int prec, int maxm, double bytes, hipStream_t st, F fn,
                       bool allow = true) {
  if (!allow || !g_prof.load(std::memory_order_relaxed)) return fn();
  std::lock_guard<std::mutex> lk(g_pmu);
  ProfRec r;
  r.name = prof_name(pass, prec, maxm);
  r.bytes = bytes;
  r.a = take_event();
  r.b = take_event();
  if (!r.a || !r.b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(r.a, st);
  if (e == hipSuccess) e = fn();
  if (e == hipSuccess) e = hipEventRecord(r.b, st);
  g_precs.push_back(r);
  return e;
}

// The plans that use a destroyed handle leave the cache for the graveyard,
// and the handle's device blocks go back to the pool once both the plans'
// last work (their `done` events) and the handle's last work (an event
// recorded now on the stream it last used) have finished: destroying a
// handle never waits for the device, where other requests' work may run.
void drop_plans_of(pe3d_handle h, std::shared_ptr<HandleBlocks> blocks) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (h->used) {
    Deferred df;
    df.blocks = blocks;
    if (hipEventCreateWithFlags(&df.ev, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(df.ev, h->last) != hipSuccess) {
      // cannot order the release after the handle's work: wait for the device
      (void)hipGetLastError();
      if (df.ev) (void)hipEventDestroy(df.ev);
      df.ev = nullptr;
      (void)hipDeviceSynchronize();
    }
    g_deferred.push_back(std::move(df));
  }
  for (auto it = g_plans.begin(); it != g_plans.end();) {
    auto& hs = it->second->handles;
    if (std::find(hs.begin(), hs.end(), h) != hs.end()) {
      g_lru.remove(it->first);
      g_graveyard.push_back(std::move(it->second));
      it = g_plans.erase(it);
    } else {
      ++it;
    }
  }
  // every plan in the graveyard that used the handle keeps its blocks
  for (auto& pl : g_graveyard) {
    auto& hs = pl->handles;
    if (std::find(hs.begin(), hs.end(), h) != hs.end()) pl->keep.push_back(blocks);
  }
  reap();
}

}  // namespace

extern "C" {

const char* pe3d_strerror(pe3d_status s) {
  switch (s) {
    case PE3D_OK: return "ok";
    case PE3D_EINVAL: return "invalid argument";
    case PE3D_ENOMEM: return "out of memory";
    case PE3D_EDEVICE: return "HIP runtime or kernel launch error";
    case PE3D_EUNSUPPORTED: return "outside the supported sizes or a vanishing depth pivot";
    case PE3D_ESTATE: return "invalid state";
  }
  return "unknown status";
}

pe3d_status pe3d_footprint(const pe3d_env* env, const pe3d_grid* grid, const pe3d_freq* freq,
                           size_t* bytes) {
  if (!bytes) return PE3D_EINVAL;
  pe3d_status st = validate(env, grid, freq);
  if (st != PE3D_OK) return st;
  Built b;
  b.N = grid->nz;
  b.NT = grid->ntheta;
  b.prec = grid->precision;
  b.nbr = env->n_bathy_r >= 2 ? env->n_bathy_r : 0;
  b.nsr = env->n_ssp_r >= 2 ? env->n_ssp_r : 0;
  b.la_req = grid->depth_lanes;
  b.lb_req = grid->azimuth_lanes;
  b.bsolver = grid->azimuth_solver;
  st = choose_shapes(b);
  if (st != PE3D_OK) return st;
  *bytes = table_bytes(b) + field_bytes(b);
  return PE3D_OK;
}

pe3d_status pe3d_host_tables(const pe3d_env* env, const pe3d_grid* grid, const pe3d_freq* freq,
                             double* qw, double* pw, double* pb, int32_t* kcol, double* blk) {
  if (!qw || !pw || !pb || !kcol || !blk) return PE3D_EINVAL;
  pe3d_status st = validate(env, grid, freq);
  if (st != PE3D_OK) return st;
  Built b;
  st = build(*env, *grid, *freq, b);
  if (st != PE3D_OK) return st;
  for (int l = 0; l < b.N; ++l) {
    qw[2 * l] = b.qw[l].real();
    qw[2 * l + 1] = b.qw[l].imag();
    pw[2 * l] = b.pw[l].real();
    pw[2 * l + 1] = b.pw[l].imag();
    pb[2 * l] = b.pb[l].real();
    pb[2 * l + 1] = b.pb[l].imag();
  }
  for (int m = 0; m < b.NT; ++m) {
    kcol[m] = b.k[m];
    for (int q = 0; q < 12; ++q) {
      blk[24 * m + 2 * q] = b.rec[b.nw[m]][q].real();
      blk[24 * m + 2 * q + 1] = b.rec[b.nw[m]][q].imag();
    }
  }
  return PE3D_OK;
}

pe3d_status pe3d_create(const pe3d_env* env, const pe3d_grid* grid, const pe3d_freq* freq,
                        pe3d_handle* out) {
  if (!out) return PE3D_EINVAL;
  *out = nullptr;
  pe3d_status st = validate(env, grid, freq);
  if (st != PE3D_OK) return st;
  Built b;
  st = build(*env, *grid, *freq, b);
  if (st != PE3D_OK) return st;
  // the depth-pass tables of every further water row (the same grid, shapes
  // and columns; only the water profile differs)
  std::vector<Built> more;
  for (int i = 1; i < b.nsr; ++i) {
    pe3d_env er = *env;
    er.ssp_c = env->ssp_c + (size_t)i * env->n_ssp;
    more.emplace_back();
    st = build(er, *grid, *freq, more.back());
    if (st != PE3D_OK) return st;
  }

  // host image of the coefficient tables (FP64 in both precisions)
  const Layout y = layout(b);
  const size_t tb = y.total;
  std::vector<unsigned char> img(tb, 0);
  for (int i = 0; i < std::max(b.nsr, 1); ++i) {
    const Built& t = i == 0 ? b : more[i - 1];
    const size_t ob = (size_t)i * y.row_bytes;
    std::vector<cd> recflat;
    recflat.reserve((size_t)(t.N + 1) * 12);
    for (auto& a : t.rec)
      for (auto& z : a) recflat.push_back(z);
    pack<double>(t.tabG, img, ob + y.o_G);
    pack<double>(t.tabC, img, ob + y.o_C);
    pack<double>(t.tabP, img, ob + y.o_P);
    pack<double>(recflat, img, ob + y.o_rec);
  }
  if (!b.dcol.empty()) std::memcpy(img.data() + y.o_dc, b.dcol.data(), b.dcol.size() * sizeof(double));
  std::memcpy(img.data() + y.o_k, b.nw.data(), b.NT * sizeof(int));

  pe3d_handle h = new (std::nothrow) pe3d_handle_s();
  if (!h) return PE3D_ENOMEM;
  h->prec = b.prec;
  h->maxm_a = b.ma;
  h->maxm_b = b.maxm_b;
  h->lds_a = pass_a_lds(b.prec, b.lpc, b.N, b.ma);
  h->lds_b = pass_b_lds(b.prec, b.wb, b.mb);
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return PE3D_EDEVICE;
  }
  if (pool_alloc(&h->d_tables, tb) != hipSuccess) {
    delete h;
    return PE3D_ENOMEM;
  }
  if (pool_alloc(&h->d_scr, field_bytes(b)) != hipSuccess) {
    pool_release(h->d_tables);
    delete h;
    return PE3D_ENOMEM;
  }
  {
    // the current step's tables start as row 0's (device addresses)
    unsigned char* dbase = static_cast<unsigned char*>(h->d_tables);
    TabPtrs t0;
    t0.tabG = dbase + y.o_G;
    t0.tabC = dbase + y.o_C;
    t0.tabP = dbase + y.o_P;
    t0.rec = dbase + y.o_rec;
    std::memcpy(img.data() + y.o_cur, &t0, sizeof t0);
  }
  if (upload(h->d_tables, img.data(), tb) != hipSuccess) {
    pool_release(h->d_tables);
    pool_release(h->d_scr);
    delete h;
    return PE3D_EDEVICE;
  }
  unsigned char* base = static_cast<unsigned char*>(h->d_tables);
  h->d_j = reinterpret_cast<long long*>(base + y.o_j);
  h->bytes = tb + field_bytes(b);
  h->r0 = grid->r0;
  h->dr = grid->dr;

  ProbDesc& d = h->desc;
  d.u = nullptr;
  d.scr = h->d_scr;
  d.jdev = h->d_j;
  d.nsteps = 0;
  d.nz = b.N;
  d.nth = b.NT;
  d.periodic = b.periodic;
  d.rigid = b.rigid;
  d.lpc = b.lpc;
  d.ma = b.ma;
  d.ntile_a = b.ntile_a;
  d.lt = b.lt;
  d.tabG = base + y.o_G;
  d.tabC = base + y.o_C;
  d.tabP = base + y.o_P;
  d.rec = base + y.o_rec;
  d.nwcol = reinterpret_cast<int*>(base + y.o_k);
  d.dcol = b.nbr ? reinterpret_cast<const double*>(base + y.o_dc) : nullptr;
  d.nbr = b.nbr;
  d.br0 = b.br0;
  d.bdr = b.bdr;
  d.nsr = b.nsr;
  d.sr0 = b.sr0;
  d.sdr = b.sdr;
  d.row_stride = (long long)y.row_bytes;
  d.cur = reinterpret_cast<TabPtrs*>(base + y.o_cur);
  // tail constants: the bottom chain's are the same in every water row (the
  // bottom half-space does not depend on the water profile); the water
  // chain's differ between rows, so with water rows the depth pass reads its
  // tables throughout (a tail row starts at nz - 1, past the last chain row)
  for (int ch = 0; ch < 2; ++ch) {
    d.bconv[ch] = b.bconv[ch];
    d.gt_re[ch] = b.gtail[ch].real();
    d.gt_im[ch] = b.gtail[ch].imag();
    d.ct_re[ch] = b.ctail[ch].real();
    d.ct_im[ch] = b.ctail[ch].imag();
  }
  if (b.nsr) d.bconv[0] = b.N - 1;
  d.h = b.h;
  d.qb_re = b.qb.real();
  d.qb_im = b.qb.imag();
  d.bp_re = b.bp.real();
  d.bp_im = b.bp.imag();
  d.bm_re = b.bm.real();
  d.bm_im = b.bm.imag();
  d.cbs_re = b.cbs.real();
  d.cbs_im = b.cbs.imag();
  d.wb = b.wb;
  d.nc = b.nc;
  d.td = b.td;
  d.mb = b.mb;
  d.ntile_b = b.ntile_b;
  d.bcls = b.maxm_b;
  d.k0 = b.k0;
  d.dr = grid->dr;
  d.r0 = grid->r0;
  d.dth = b.dth;
  d.dz = b.dz;
  d.nx2d = grid->mode == PE3D_MODE_NX2D;
  *out = h;
  return PE3D_OK;
}

pe3d_status pe3d_destroy(pe3d_handle h) {
  if (!h) return PE3D_OK;
  auto blocks = std::make_shared<HandleBlocks>();
  blocks->tables = h->d_tables;
  blocks->scr = h->d_scr;
  drop_plans_of(h, std::move(blocks));
  delete h;
  return PE3D_OK;
}

pe3d_status pe3d_get_step(pe3d_handle h, int64_t* j, double* r) {
  if (!h) return PE3D_EINVAL;
  if (j) *j = h->j;
  if (r) *r = h->r0 + double(h->j) * h->dr;
  return PE3D_OK;
}

pe3d_status pe3d_set_step(pe3d_handle h, int64_t j) {
  if (!h || j < 0) return PE3D_EINVAL;
  if (hipDeviceSynchronize() != hipSuccess) return PE3D_EDEVICE;
  long long jj = j;
  if (hipMemcpy(h->d_j, &jj, sizeof(jj), hipMemcpyHostToDevice) != hipSuccess) return PE3D_EDEVICE;
  h->j = j;
  return PE3D_OK;
}

pe3d_status pe3d_get_info(pe3d_handle h, pe3d_info* info) {
  if (!h || !info) return PE3D_EINVAL;
  const ProbDesc& d = h->desc;
  info->nz = d.nz;
  info->ntheta = d.nth;
  info->periodic = d.periodic;
  info->precision = h->prec;
  info->mode = d.nx2d ? PE3D_MODE_NX2D : PE3D_MODE_3D;
  info->k0 = d.k0;
  info->dz = d.dz;
  info->dtheta = d.dth;
  info->dr = d.dr;
  info->r0 = d.r0;
  info->pass_a_lanes = d.lpc;
  info->pass_a_chunk = d.ma;
  info->pass_b_chunks = d.nc;
  info->pass_b_depths = d.td;
  info->device_bytes = h->bytes;
  return PE3D_OK;
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // extern "C"

namespace {

// The plain march of one problem: the handle's scratch field (pe3d_march) or
// another of the same size or larger (pe3d_march_static); `profile` false
// records no events.  Arguments are checked by the callers.
pe3d_status march_impl(pe3d_handle h, int32_t nsteps, void* u_dev, hipStream_t st, void* scr, bool profile) {
  ProbDesc d = h->desc;
  d.u = u_dev;
  d.scr = scr;
  d.nsteps = nsteps;
  const double fbytes = 2.0 * double(d.nz) * d.nth * (h->prec ? 16.0 : 8.0);
  if (d.nx2d && !d.nbr && !d.nsr) {
    // N x 2D over a fixed medium: the columns march through every step of
    // the call inside one launch, in LDS (the same arithmetic and roundings
    // as one launch per step); algorithmic bytes: the field in and out once
    if (prof_launch("pass_a_nx2d", h->prec, h->maxm_a, fbytes, st, [&] {
          return launch_pass_a_multi(h->prec, d, h->lds_a, st);
        }, profile) != hipSuccess)
      return PE3D_EDEVICE;
    if (launch_advance(nullptr, nullptr, 0, h->d_j, nsteps, st) != hipSuccess) return PE3D_EDEVICE;
    h->j += nsteps;
    return PE3D_OK;
  }
  for (int k = 0; k < nsteps; ++k) {
    // the medium of step k: launched for the first step, and for every step
    // of an N x 2D march; a 3D march's azimuth pass writes it for the next
    if ((d.nbr || d.nsr) && (k == 0 || d.nx2d) && launch_medium_update(&d, nullptr, nullptr, 0, k, st) != hipSuccess)
      return PE3D_EDEVICE;
    if (prof_launch("pass_a", h->prec, h->maxm_a, fbytes, st, [&] {
          return launch_pass_a(h->prec, &d, nullptr, nullptr, 0, k, h->lds_a, st);
        }, profile) != hipSuccess)
      return PE3D_EDEVICE;
    if (!d.nx2d && prof_launch("pass_b", h->prec, h->maxm_b, fbytes, st, [&] {
          return launch_pass_b(h->prec, &d, nullptr, nullptr, 0, k, h->lds_b, st);
        }, profile) != hipSuccess)
      return PE3D_EDEVICE;
  }
  if (launch_advance(nullptr, nullptr, 0, h->d_j, nsteps, st) != hipSuccess) return PE3D_EDEVICE;
  h->j += nsteps;
  return PE3D_OK;
}

}  // namespace

extern "C" {

pe3d_status pe3d_march(pe3d_handle h, int32_t nsteps, void* u_dev, void* stream) {
  if (!h || !u_dev || nsteps < 0 || !aligned16(u_dev)) return PE3D_EINVAL;
  if (nsteps == 0) return PE3D_OK;
  h->used = true;
  h->last = static_cast<hipStream_t>(stream);
  return march_impl(h, nsteps, u_dev, static_cast<hipStream_t>(stream), h->d_scr, true);
}

pe3d_status pe3d_march_static(pe3d_handle h, int32_t nsteps, void* u_dev, void* stream) {
  if (!h || !u_dev || nsteps < 0 || !aligned16(u_dev)) return PE3D_EINVAL;
  if (nsteps == 0) return PE3D_OK;
  const size_t fb = (size_t)h->desc.nz * h->desc.nth * (h->prec ? 16u : 8u);
  if (fb > kStaticScratchBytes) return PE3D_EUNSUPPORTED;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return PE3D_EDEVICE;
  if (dev != h->device) return PE3D_ESTATE;
  void* scr = nullptr;
  if (static_scratch(&scr) != hipSuccess) return PE3D_EDEVICE;
  h->used = true;
  h->last = static_cast<hipStream_t>(stream);
  return march_impl(h, nsteps, u_dev, static_cast<hipStream_t>(stream), scr, false);
}

pe3d_status pe3d_starter(pe3d_handle h, double zs, void* u_dev, void* stream) {
  if (!h || !u_dev || !is_fin(zs) || zs < 0.0 || !aligned16(u_dev)) return PE3D_EINVAL;
  h->used = true;
  h->last = static_cast<hipStream_t>(stream);
  if (launch_starter(h->prec, h->desc, zs, u_dev, static_cast<hipStream_t>(stream)) != hipSuccess)
    return PE3D_EDEVICE;
  return PE3D_OK;
}

pe3d_status pe3d_tl(pe3d_handle h, const void* u_dev, float* tl_dev, void* stream) {
  if (!h || !u_dev || !tl_dev || !aligned16(u_dev)) return PE3D_EINVAL;
  h->used = true;
  h->last = static_cast<hipStream_t>(stream);
  if (launch_tl(h->prec, h->desc, u_dev, tl_dev, static_cast<hipStream_t>(stream)) != hipSuccess)
    return PE3D_EDEVICE;
  return PE3D_OK;
}

pe3d_status pe3d_pressure(pe3d_handle h, const void* u_dev, void* p_dev, void* stream) {
  if (!h || !u_dev || !p_dev || !aligned16(u_dev) || !aligned16(p_dev)) return PE3D_EINVAL;
  const double r = h->r0 + double(h->j) * h->dr;
  if (!(r > 0.0)) return PE3D_ESTATE;
  h->used = true;
  h->last = static_cast<hipStream_t>(stream);
  // H0^(1)(x) = J0(x) + i Y0(x), x = k0 r_j (C++17 special functions, FP64)
  const double x = h->desc.k0 * r;
  const double hre = std::cyl_bessel_j(0.0, x), him = std::cyl_neumann(0.0, x);
  if (launch_scale(h->prec, h->desc, u_dev, p_dev, hre, him, static_cast<hipStream_t>(stream)) != hipSuccess)
    return PE3D_EDEVICE;
  return PE3D_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batch
namespace {

// Partition of the stepping problems (indices into hs) into chains of
// groups: chains balanced by field bytes (largest problem to the lightest
// chain), each chain cut, in order of decreasing problem size, into the
// fewest groups of at most `group_bytes` of field each (a problem larger
// than that is a group of its own), of near-equal bytes.
std::vector<std::vector<std::vector<int>>> batch_partition(const pe3d_handle* hs, int n,
                                                           const int32_t* nsteps, int nchains,
                                                           long long group_bytes) {
  std::vector<int> ids;
  for (int i = 0; i < n; ++i)
    if (nsteps[i] > 0) ids.push_back(i);
  auto bytes_of = [&](int i) {
    return double(hs[i]->desc.nz) * hs[i]->desc.nth * (hs[i]->prec ? 16.0 : 8.0);
  };
  std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) { return bytes_of(a) > bytes_of(b); });
  nchains = std::max(1, std::min(nchains, int(ids.size())));
  std::vector<std::vector<int>> ch(nchains);
  std::vector<double> tot(nchains, 0.0);
  for (int i : ids) {
    int c = int(std::min_element(tot.begin(), tot.end()) - tot.begin());
    ch[c].push_back(i);
    tot[c] += bytes_of(i);
  }
  std::vector<std::vector<std::vector<int>>> out;
  for (int c = 0; c < nchains; ++c) {
    if (ch[c].empty()) continue;
    int ng = 1;
    if (group_bytes > 0) ng = std::max(1, int(std::ceil(tot[c] / double(group_bytes))));
    ng = std::min(ng, int(ch[c].size()));
    std::vector<std::vector<int>> gs(1);
    double acc = 0.0;
    for (size_t q = 0; q < ch[c].size(); ++q) {
      const int i = ch[c][q];
      // start a new group once more than half of this problem would lie
      // beyond the current group's share of the chain
      const double share = tot[c] * double(gs.size()) / ng;
      if (!gs.back().empty() && int(gs.size()) < ng && acc + 0.5 * bytes_of(i) > share)
        gs.emplace_back();
      gs.back().push_back(i);
      acc += bytes_of(i);
    }
    out.push_back(gs);
  }
  return out;
}

// The persistent kernel's task list.  Problem p has na depth-pass tiles
// taken asub at a time and nb azimuth-pass tiles (0: none) taken bsub at a
// time; its tasks of one step are the depth pass's ceil(na / asub) then the
// azimuth pass's ceil(nb / bsub), and a task waits for every task of the
// problem's earlier passes.  Per chain, the phases (one pass of one step of
// one group, over the group's problems still stepping) follow each group
// through its steps, groups in order; the chains' phases are interleaved,
// phase i of every chain before phase i + 1 of any, so that the wait of a
// phase for the previous phase of its group is covered by the other chains'
// work.  Every task's waits are on tasks earlier in the list.
struct PersistProb {
  int na, asub, nb, bsub, nsteps;
};
void persist_tasks(const std::vector<std::vector<std::vector<int>>>& chains, const std::vector<PersistProb>& pp,
                   std::vector<PTask>& out) {
  struct Phase {
    int g, k, kind;
  };
  std::vector<std::vector<Phase>> ph(chains.size());
  size_t most = 0;
  for (size_t c = 0; c < chains.size(); ++c) {
    for (int g = 0; g < int(chains[c].size()); ++g) {
      int ms = 0;
      bool azimuth = false;
      for (int p : chains[c][g]) {
        ms = std::max(ms, pp[p].nsteps);
        azimuth = azimuth || pp[p].nb > 0;
      }
      for (int k = 0; k < ms; ++k) {
        ph[c].push_back({g, k, 0});
        if (azimuth) ph[c].push_back({g, k, 1});
      }
    }
    most = std::max(most, ph[c].size());
  }
  out.clear();
  for (size_t i = 0; i < most; ++i)
    for (size_t c = 0; c < chains.size(); ++c) {
      if (i >= ph[c].size()) continue;
      const Phase f = ph[c][i];
      for (int p : chains[c][f.g]) {
        const PersistProb& q = pp[p];
        if (q.nsteps <= f.k) continue;
        const int nat = (q.na + q.asub - 1) / q.asub;
        const int nbt = q.nb > 0 ? (q.nb + q.bsub - 1) / q.bsub : 0;
        const int per_step = nat + nbt;
        if (f.kind == 0) {
          for (int t = 0; t < nat; ++t) out.push_back({p, t * q.asub, f.k, f.k * per_step, 0, short(q.asub)});
        } else {
          for (int t = 0; t < nbt; ++t)
            out.push_back({p, t * q.bsub, f.k, f.k * per_step + nat, 1, short(q.bsub)});
        }
      }
    }
}

// Tiles of the persistent kernel's tasks.  The depth pass's tiles are the
// launches' (256 / L columns each); the azimuth pass's hold 256 lanes.  A
// task takes consecutive tiles until it covers `points` grid points (at most
// kPersistMaxSub tiles), and an azimuth task at least enough tiles to fill a
// 128-byte line of each depth line it touches.  Finished tasks are published
// with device-scope releases (write-backs of the XCD's L2), the kernel's
// main overhead, so tasks hold kPersistTaskPoints points unless the batch is
// too small to give every resident workgroup two tasks per pass.
constexpr int kPersistTaskPoints = 16384;
constexpr int kPersistMaxSub = 16;
int persist_task_points(double batch_points, int resident) {
  const double per = batch_points / (2.0 * std::max(1, resident));
  return int(std::max(1.0, std::min(double(kPersistTaskPoints), per)));
}
void persist_shape(const pe3d_handle h, int points, PersistProb& q) {
  const ProbDesc& d = h->desc;
  const int esz = h->prec ? 16 : 8;
  auto sub_for = [points](int pts_per_tile, int at_least) {
    int s = std::max(at_least, (points + pts_per_tile - 1) / std::max(1, pts_per_tile));
    return std::max(1, std::min(kPersistMaxSub, s));
  };
  q.na = d.ntile_a;
  q.asub = sub_for((256 / d.lpc) * d.nz, 1);
  if (d.nx2d) {
    q.nb = 0;
    q.bsub = 1;
    return;
  }
  const int td = d.bcls == kPcrClass ? d.td : kPersistThreads / d.wb;
  q.nb = d.bcls == kPcrClass ? d.ntile_b : (d.nz + td - 1) / td;
  q.bsub = sub_for(td * d.nth, 128 / (td * esz));
}

// Task lists of at most this many tasks (20 bytes each); a longer call (the
// list grows with the steps) runs the launches.
constexpr long long kPersistMaxTasks = 1ll << 24;

// Grid points per task of the persistent kernel for these stepping problems.
int persist_points_for(const pe3d_handle* hs, int n, const int32_t* nsteps) {
  double batch_points = 0.0;
  for (int i = 0; i < n; ++i)
    if (nsteps[i] > 0) batch_points += double(hs[i]->desc.nz) * hs[i]->desc.nth;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, hs[0]->device) != hipSuccess || ncu < 1)
    ncu = 256;
  // resident workgroups: 3 per CU (the kernel's complex64 occupancy; 2 for complex128)
  return persist_task_points(batch_points, ncu * (hs[0]->prec ? 2 : 3));
}

// Length of the persistent kernel's task list for these problems.
long long persist_task_count(const pe3d_handle* hs, int n, const int32_t* nsteps) {
  const int points = persist_points_for(hs, n, nsteps);
  long long total = 0;
  for (int i = 0; i < n; ++i) {
    if (nsteps[i] <= 0) continue;
    PersistProb q{};
    persist_shape(hs[i], points, q);
    const long long per_step = (q.na + q.asub - 1) / q.asub + (q.nb > 0 ? (q.nb + q.bsub - 1) / q.bsub : 0);
    total += per_step * nsteps[i];
  }
  return total;
}

pe3d_status build_plan(const pe3d_handle* hs, int n, const int32_t* nsteps, void* const* u,
                       int nchains, long long group_bytes, bool persist, long long wait_ticks, BatchPlan& P) {
  // the persistent kernel takes one group per chain: its workgroups publish
  // finished tasks in batches, which leaves the short phases of cache-sized
  // groups waiting on each other
  auto part = batch_partition(hs, n, nsteps, nchains, persist ? 0 : group_bytes);
  // problem slots in the descriptor table, in partition order
  std::vector<int> order;
  for (auto& c : part)
    for (auto& g : c) order.insert(order.end(), g.begin(), g.end());
  const int np = int(order.size());
  P.n = np;
  P.prec = hs[0]->prec;
  std::vector<ProbDesc> descs(np);
  std::vector<long long*> jdevs(np);
  std::vector<int> adds(np);
  std::vector<int> slot(n, -1);
  for (int p = 0; p < np; ++p) {
    pe3d_handle h = hs[order[p]];
    slot[order[p]] = p;
    descs[p] = h->desc;
    descs[p].u = u[order[p]];
    descs[p].nsteps = nsteps[order[p]];
    jdevs[p] = h->d_j;
    adds[p] = nsteps[order[p]];
  }
  auto make_class = [](std::vector<WorkItem>& items, std::vector<int>& steps, std::vector<double>& bytes,
                       int lds, int maxsteps) {
    BatchPlan::Class c;
    c.maxm = kBatchClass;
    c.lds = lds;
    c.h_items = std::move(items);
    c.bytes_prefix.assign(bytes.size() + 1, 0.0);
    for (size_t i = 0; i < bytes.size(); ++i) c.bytes_prefix[i + 1] = c.bytes_prefix[i] + bytes[i];
    c.nitems_at.resize(maxsteps);
    for (int k = 0; k < maxsteps; ++k)  // steps is non-increasing: items whose problem has > k steps
      c.nitems_at[k] =
          int(std::lower_bound(steps.begin(), steps.end(), k, [](int a, int v) { return a > v; }) - steps.begin());
    return c;
  };
  std::vector<std::vector<std::vector<int>>> pchains;  // slots, in the groups' order
  for (auto& cpart : part) {
    std::vector<BatchPlan::Group> chain;
    pchains.emplace_back();
    for (auto g : cpart) {
      // within a group: problems sorted by steps (descending) so that the
      // problems still stepping at step k are a prefix of every item list,
      // and, among equal steps, deeper problems first (their heavier
      // workgroups are dispatched before the light ones, which shortens the
      // launch tail)
      std::stable_sort(g.begin(), g.end(), [&](int a, int b) {
        if (nsteps[a] != nsteps[b]) return nsteps[a] > nsteps[b];
        return hs[a]->desc.nz > hs[b]->desc.nz;
      });
      pchains.back().emplace_back();
      for (int i : g) pchains.back().back().push_back(slot[i]);
      if (persist) continue;
      BatchPlan::Group G;
      G.maxsteps = nsteps[g[0]];
      std::vector<WorkItem> ia, ib, iu;
      std::vector<int> sa, sb, su;
      std::vector<double> ba, bb, bu;
      int lds_a = 0, lds_b = 0;
      for (int i : g) {
        pe3d_handle h = hs[i];
        const int p = slot[i];
        const ProbDesc& hd = h->desc;
        const double esz = h->prec ? 16.0 : 8.0;
        const int cpw = 256 / hd.lpc;
        lds_a = std::max(lds_a, h->lds_a);
        for (int t = 0; t < hd.ntile_a; ++t) {
          ia.push_back({p, t});
          sa.push_back(nsteps[i]);
          const int ncol = std::min(cpw, hd.nth - t * cpw);
          ba.push_back(2.0 * esz * ncol * hd.nz);
        }
        // problems with range rows: water nodes of 256 columns per item (depth
        // rows), the water row in item 0 (water rows), before every step
        if (hd.nbr || hd.nsr)
          for (int t = 0; t < (hd.nbr ? (hd.nth + 255) / 256 : 1); ++t) {
            iu.push_back({p, t});
            su.push_back(nsteps[i]);
            bu.push_back(0.0);
          }
        // N x 2D problems have no azimuth pass: the items of the still-stepping
        // problems stay a prefix of the list, as the steps stay non-increasing
        if (hd.nx2d) continue;
        lds_b = std::max(lds_b, h->lds_b);
        const bool pairs = pass_b_pairs(hd.td, h->prec ? 16 : 8);
        for (int b = 0; b < hd.ntile_b; ++b) {
          const int t = pairs ? pass_b_paired_tile(b, hd.ntile_b) : b;
          ib.push_back({p, t});
          sb.push_back(nsteps[i]);
          const int nd = std::min(hd.td, hd.nz - t * hd.td);
          bb.push_back(2.0 * esz * nd * hd.nth);
        }
      }
      if (!ia.empty()) G.a.push_back(make_class(ia, sa, ba, lds_a, G.maxsteps));
      if (!ib.empty()) G.b.push_back(make_class(ib, sb, bb, lds_b, G.maxsteps));
      if (!iu.empty()) G.u.push_back(make_class(iu, su, bu, 0, G.maxsteps));
      chain.push_back(std::move(G));
    }
    P.chains.push_back(std::move(chain));
  }
  std::vector<PTask> tasks;
  if (persist) {
    std::vector<PersistProb> pp(np);
    const int points = persist_points_for(hs, n, nsteps);
    for (int p = 0; p < np; ++p) {
      pe3d_handle h = hs[order[p]];
      persist_shape(h, points, pp[p]);
      pp[p].nsteps = nsteps[order[p]];
      const double esz = h->prec ? 16.0 : 8.0;
      const double pts = double(h->desc.nz) * h->desc.nth;
      P.bytes_p += pp[p].nsteps * (pp[p].nb > 0 ? 4.0 : 2.0) * esz * pts;
      P.lds_p = std::max(P.lds_p, h->lds_a);
      if (pp[p].nb > 0)
        P.lds_p = std::max(P.lds_p, pass_b_lds(h->prec, h->desc.bcls == kPcrClass ? 0 : h->desc.wb,
                                               h->desc.mb, kPersistThreads));
    }
    persist_tasks(pchains, pp, tasks);
    if (tasks.size() > size_t(kPersistMaxTasks)) return PE3D_EUNSUPPORTED;  // checked by the caller
    P.persist = true;
    P.ntasks = int(tasks.size());
    P.wait_ticks = wait_ticks;
  }
  size_t nitems = 0;
  for (auto& c : P.chains)
    for (auto& g : c)
      for (auto* v : {&g.a, &g.b, &g.u})
        for (auto& k : *v) nitems += k.h_items.size();
  size_t off_desc = 0;
  size_t off_j = (off_desc + np * sizeof(ProbDesc) + 255) & ~size_t(255);
  size_t off_add = (off_j + np * sizeof(long long*) + 255) & ~size_t(255);
  size_t off_it = (off_add + np * sizeof(int) + 255) & ~size_t(255);
  size_t off_tk = (off_it + nitems * sizeof(WorkItem) + 255) & ~size_t(255);
  size_t off_ctl = (off_tk + tasks.size() * sizeof(PTask) + 255) & ~size_t(255);
  size_t total = off_ctl + (persist ? persist_ctl_ints(np) * sizeof(int) : 0) + 256;
  std::vector<unsigned char> img(total, 0);
  if (persist) std::memcpy(img.data() + off_tk, tasks.data(), tasks.size() * sizeof(PTask));
  std::memcpy(img.data() + off_desc, descs.data(), np * sizeof(ProbDesc));
  std::memcpy(img.data() + off_j, jdevs.data(), np * sizeof(long long*));
  std::memcpy(img.data() + off_add, adds.data(), np * sizeof(int));
  if (pool_alloc(&P.d_mem, total) != hipSuccess) return PE3D_ENOMEM;
  unsigned char* base = static_cast<unsigned char*>(P.d_mem);
  P.d_descs = reinterpret_cast<ProbDesc*>(base + off_desc);
  P.d_jdevs = reinterpret_cast<long long**>(base + off_j);
  P.d_adds = reinterpret_cast<int*>(base + off_add);
  if (persist) {
    P.d_tasks = reinterpret_cast<PTask*>(base + off_tk);
    P.d_ctl = reinterpret_cast<int*>(base + off_ctl);
  }
  size_t cur = off_it;
  for (auto& c : P.chains)
    for (auto& g : c)
      for (auto* v : {&g.a, &g.b, &g.u})
        for (auto& k : *v) {
          k.d_items = reinterpret_cast<WorkItem*>(base + cur);
          std::memcpy(img.data() + cur, k.h_items.data(), k.h_items.size() * sizeof(WorkItem));
          cur += k.h_items.size() * sizeof(WorkItem);
          std::vector<WorkItem>().swap(k.h_items);
        }
  if (upload(P.d_mem, img.data(), total) != hipSuccess) return PE3D_EDEVICE;
  return PE3D_OK;
}

// The launches of one chain: each group through all of its steps.
// profile: false while capturing (no event records inside a graph)
pe3d_status enqueue_chain(const BatchPlan& P, const std::vector<BatchPlan::Group>& chain, hipStream_t st,
                          bool profile) {
  for (const auto& g : chain)
    for (int k = 0; k < g.maxsteps; ++k) {
      for (auto& c : g.u) {
        int ni = c.nitems_at[k];
        if (ni > 0 && launch_medium_update(nullptr, P.d_descs, c.d_items, ni, k, st) != hipSuccess)
          return PE3D_EDEVICE;
      }
      for (auto& c : g.a) {
        int ni = c.nitems_at[k];
        if (ni > 0 && prof_launch("pass_a", P.prec, c.maxm, c.bytes_prefix[ni], st, [&] {
              return launch_pass_a(P.prec, nullptr, P.d_descs, c.d_items, ni, k, c.lds, st);
            }, profile) != hipSuccess)
          return PE3D_EDEVICE;
      }
      for (auto& c : g.b) {
        int ni = c.nitems_at[k];
        if (ni > 0 && prof_launch("pass_b", P.prec, c.maxm, c.bytes_prefix[ni], st, [&] {
              return launch_pass_b(P.prec, nullptr, P.d_descs, c.d_items, ni, k, c.lds, st);
            }, profile) != hipSuccess)
          return PE3D_EDEVICE;
      }
    }
  return PE3D_OK;
}

pe3d_status enqueue_advance(const BatchPlan& P, hipStream_t st) {
  return launch_advance(P.d_jdevs, P.d_adds, P.n, nullptr, 0, st) == hipSuccess ? PE3D_OK : PE3D_EDEVICE;
}

// The plan's side streams (from the device's pool) and fork/join events
// (created once; chains >= 1).  Caller holds g_mu.
pe3d_status ensure_side(BatchPlan& P) {
  const size_t nc = P.chains.size();
  if (nc > 1 && !P.fork && hipEventCreateWithFlags(&P.fork, hipEventDisableTiming) != hipSuccess)
    return PE3D_EDEVICE;
  if (P.side.size() + 1 < nc) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PE3D_EDEVICE;
    auto& pool = g_side_streams[dev];
    while (pool.size() + 1 < nc) {
      hipStream_t s;
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return PE3D_EDEVICE;
      pool.push_back(s);
    }
    P.side.assign(pool.begin(), pool.begin() + (nc - 1));
  }
  while (P.join.size() + 1 < nc) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return PE3D_EDEVICE;
    P.join.push_back(e);
  }
  return PE3D_OK;
}

// Chain 0 on the caller's stream, chain c >= 1 on side stream c-1 after the
// caller's prior work (fork event); the caller's stream then waits for every
// chain (join events) and advances the step counters.  run(c, stream)
// enqueues chain c.
template <typename F>
pe3d_status fork_join(const BatchPlan& P, hipStream_t st, F run) {
  const size_t nc = P.chains.size();
  if (nc > 1 && hipEventRecord(P.fork, st) != hipSuccess) return PE3D_EDEVICE;
  pe3d_status s = PE3D_OK;
  size_t joined = 1;  // side chains whose join event is recorded
  for (size_t c = 1; c < nc && s == PE3D_OK; ++c) {
    if (hipStreamWaitEvent(P.side[c - 1], P.fork, 0) != hipSuccess) {
      s = PE3D_EDEVICE;
      break;
    }
    s = run(c, P.side[c - 1]);
    // the join is recorded even after a failed enqueue, so that the caller's
    // stream never runs ahead of work already on a side stream
    if (hipEventRecord(P.join[c - 1], P.side[c - 1]) != hipSuccess && s == PE3D_OK) s = PE3D_EDEVICE;
    joined = c + 1;
  }
  if (s == PE3D_OK) s = run(0, st);
  for (size_t c = 1; c < joined; ++c)
    if (hipStreamWaitEvent(st, P.join[c - 1], 0) != hipSuccess && s == PE3D_OK) s = PE3D_EDEVICE;
  if (s != PE3D_OK) return s;
  return enqueue_advance(P, st);
}

// The persistent kernel (its counters zeroed first) on the caller's stream.
pe3d_status enqueue_persist(const BatchPlan& P, hipStream_t st, bool profile) {
  return prof_launch("persist", P.prec, kBatchClass, P.bytes_p, st, [&] {
           return launch_persist(P.prec, P.d_descs, P.d_tasks, P.ntasks, P.d_ctl, P.n, P.wait_ticks, P.lds_p, st);
         }, profile) == hipSuccess
             ? PE3D_OK
             : PE3D_EDEVICE;
}

// Direct launches, on the same streams as a graph replay.
pe3d_status enqueue_plan(BatchPlan& P, hipStream_t st) {
  if (P.persist) {
    pe3d_status s = enqueue_persist(P, st, true);
    return s == PE3D_OK ? enqueue_advance(P, st) : s;
  }
  pe3d_status s = ensure_side(P);
  if (s != PE3D_OK) return s;
  return fork_join(P, st, [&](size_t c, hipStream_t cs) { return enqueue_chain(P, P.chains[c], cs, true); });
}

// One graph per chain (persistent kernel: one graph), captured on a private
// stream.
pe3d_status capture_plan(BatchPlan& P) {
  const size_t ng = P.persist ? 1 : P.chains.size();
  for (size_t ci = 0; ci < ng; ++ci) {
    hipStream_t cap;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return PE3D_EDEVICE;
    pe3d_status s = PE3D_OK;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) s = PE3D_EDEVICE;
    if (s == PE3D_OK) s = P.persist ? enqueue_persist(P, cap, false) : enqueue_chain(P, P.chains[ci], cap, false);
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(cap, &g) != hipSuccess && s == PE3D_OK) s = PE3D_EDEVICE;
    (void)hipStreamDestroy(cap);
    if (g) P.graphs.push_back(g);
    if (s != PE3D_OK) return s;
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) return PE3D_EDEVICE;
    P.execs.push_back(x);
  }
  return P.persist ? PE3D_OK : ensure_side(P);
}

pe3d_status replay_plan(const BatchPlan& P, hipStream_t st) {
  if (P.persist) {
    if (hipGraphLaunch(P.execs[0], st) != hipSuccess) return PE3D_EDEVICE;
    return enqueue_advance(P, st);
  }
  return fork_join(P, st, [&](size_t c, hipStream_t cs) {
    return hipGraphLaunch(P.execs[c], cs) == hipSuccess ? PE3D_OK : PE3D_EDEVICE;
  });
}

}  // namespace

extern "C" pe3d_status pe3d_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_pmu);
  g_prof.store(on != 0);
  return PE3D_OK;
}

extern "C" pe3d_status pe3d_profile_read(pe3d_kernel_stat* stats, int32_t cap, int32_t* n) {
  if (!n || cap < 0 || (cap > 0 && !stats)) return PE3D_EINVAL;
  std::lock_guard<std::mutex> lk(g_pmu);
  std::vector<pe3d_kernel_stat> agg(g_pnames.size());
  std::vector<char> used(g_pnames.size(), 0);
  std::vector<int> order;
  pe3d_status st = PE3D_OK;
  for (auto& r : g_precs) {
    float ms = 0.0f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
      st = PE3D_EDEVICE;
    pe3d_kernel_stat& a = agg[r.name];
    if (!used[r.name]) {
      used[r.name] = 1;
      order.push_back(r.name);
      std::memset(&a, 0, sizeof a);
      std::snprintf(a.name, sizeof a.name, "%s", g_pnames[r.name].c_str());
    }
    a.launches += 1;
    a.total_ms += ms;
    a.algo_bytes += r.bytes;
    g_epool.push_back(r.a);
    g_epool.push_back(r.b);
  }
  g_precs.clear();
  *n = int(order.size());
  for (int i = 0; i < int(order.size()) && i < cap; ++i) stats[i] = agg[order[i]];
  return st;
}

extern "C" pe3d_status pe3d_release_pooled_memory(size_t* bytes) {
  {
    // blocks whose plans or handles have finished join the pool first
    std::lock_guard<std::mutex> lk(g_mu);
    reap();
  }
  const size_t n = pool_trim();
  if (bytes) *bytes = n;
  return hipGetLastError() == hipSuccess ? PE3D_OK : PE3D_EDEVICE;
}

extern "C" pe3d_status pe3d_set_batch_schedule(int32_t chains, int64_t group_bytes) {
  if (chains < 1 || chains > kMaxChains || group_bytes < 0) return PE3D_EINVAL;
  g_chains.store(chains);
  g_group_bytes.store(group_bytes);
  return PE3D_OK;
}

extern "C" pe3d_status pe3d_set_batch_kernel(int32_t kind, double wait_limit_s) {
  if (kind != PE3D_BATCH_LAUNCHES && kind != PE3D_BATCH_PERSISTENT) return PE3D_EINVAL;
  if (!(wait_limit_s >= 0.0 && wait_limit_s <= 3600.0)) return PE3D_EINVAL;  // NaN fails too
  g_batch_kernel.store(kind);
  g_wait_limit_s.store(wait_limit_s);
  return PE3D_OK;
}

extern "C" pe3d_status pe3d_batch_wait_timeouts(int64_t* count) {
  if (!count) return PE3D_EINVAL;
  unsigned long long v = 0;
  if (persist_take_timeouts(&v) != hipSuccess) return PE3D_EDEVICE;
  *count = int64_t(v);
  return PE3D_OK;
}

extern "C" pe3d_status pe3d_persist_schedule(int32_t n, const int32_t* na, const int32_t* asub, const int32_t* nb,
                                             const int32_t* bsub, const int32_t* nsteps, const int32_t* chain,
                                             const int32_t* group, int32_t* tasks, int64_t cap, int64_t* ntasks) {
  if (n < 1 || !na || !asub || !nb || !bsub || !nsteps || !chain || !group || !ntasks || cap < 0 ||
      (cap > 0 && !tasks))
    return PE3D_EINVAL;
  std::vector<std::vector<std::vector<int>>> chains;
  std::vector<PersistProb> pp(n);
  for (int i = 0; i < n; ++i) {
    if (na[i] < 1 || asub[i] < 1 || asub[i] > kPersistMaxSub || nb[i] < 0 || bsub[i] < 1 ||
        bsub[i] > kPersistMaxSub || nsteps[i] < 0 || chain[i] < 0 || chain[i] > 1024 || group[i] < 0 ||
        group[i] > 1 << 20)
      return PE3D_EINVAL;
    pp[i] = {na[i], asub[i], nb[i], bsub[i], nsteps[i]};
    if (int(chains.size()) <= chain[i]) chains.resize(chain[i] + 1);
    auto& c = chains[chain[i]];
    if (int(c.size()) <= group[i]) c.resize(group[i] + 1);
    c[group[i]].push_back(i);
  }
  std::vector<PTask> out;
  persist_tasks(chains, pp, out);
  *ntasks = int64_t(out.size());
  for (int64_t t = 0; t < std::min<int64_t>(cap, int64_t(out.size())); ++t) {
    const PTask& k = out[t];
    int32_t* o = tasks + 6 * t;
    o[0] = k.prob;
    o[1] = k.tile;
    o[2] = k.k;
    o[3] = k.kind;
    o[4] = k.nsub;
    o[5] = k.need;
  }
  return PE3D_OK;
}

constexpr int32_t kPrepareOnly = 2;  // pe3d_march_batch: build and capture, do not launch

extern "C" pe3d_status pe3d_march_batch(const pe3d_handle* hs, int32_t n, const int32_t* nsteps,
                                        void* const* u_devs, int32_t use_graph, void* stream) {
  if (!hs || !nsteps || !u_devs || n < 1) return PE3D_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!hs[i] || nsteps[i] < 0 || !u_devs[i] || !aligned16(u_devs[i])) return PE3D_EINVAL;
    if (hs[i]->prec != hs[0]->prec) return PE3D_EINVAL;
    for (int k = 0; k < i; ++k)
      if (hs[k] == hs[i] || u_devs[k] == u_devs[i]) return PE3D_EINVAL;
  }
  bool any = false;
  for (int i = 0; i < n; ++i) any = any || nsteps[i] > 0;
  if (!any) return PE3D_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);

  const int nchains = g_chains.load();
  const long long group_bytes = g_group_bytes.load();
  // the persistent kernel, unless a problem has range rows (its medium
  // changes from step to step)
  bool persist = g_batch_kernel.load() == PE3D_BATCH_PERSISTENT;
  for (int i = 0; i < n && persist; ++i)
    if (nsteps[i] > 0 && (hs[i]->desc.nbr || hs[i]->desc.nsr)) persist = false;
  // (and unless its task list would be too long)
  if (persist && persist_task_count(hs, n, nsteps) > kPersistMaxTasks) persist = false;
  const double wait_s = g_wait_limit_s.load();
  std::vector<uintptr_t> key;
  key.reserve(3 * n + 4);
  key.push_back(uintptr_t(nchains));
  key.push_back(uintptr_t(group_bytes));
  key.push_back(uintptr_t(persist));
  {
    uint64_t wb = 0;
    std::memcpy(&wb, &wait_s, sizeof wb);
    key.push_back(uintptr_t(persist ? wb : 0));
  }
  for (int i = 0; i < n; ++i) {
    key.push_back(reinterpret_cast<uintptr_t>(hs[i]));
    key.push_back(reinterpret_cast<uintptr_t>(u_devs[i]));
    key.push_back(uintptr_t(uint32_t(nsteps[i])));
  }
  // The plan cache, the graveyard and the side streams are shared: one
  // batched call at a time enqueues (the device work itself stays async).
  std::lock_guard<std::mutex> lk(g_mu);
  reap();
  BatchPlan* plan = nullptr;
  auto it = g_plans.find(key);
  if (it != g_plans.end()) {
    plan = it->second.get();
    touch(key);
  } else {
    std::unique_ptr<BatchPlan> fresh(new (std::nothrow) BatchPlan());
    if (!fresh) return PE3D_ENOMEM;
    fresh->key = key;
    fresh->handles.assign(hs, hs + n);
    long long ticks = 0;
    if (persist) {
      int dev = 0, khz = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
        khz = 100000;  // the constant-rate clock of CDNA devices: 100 MHz
      ticks = (long long)std::llround(wait_s * 1000.0 * khz);
    }
    pe3d_status s = build_plan(hs, n, nsteps, u_devs, nchains, group_bytes, persist, ticks, *fresh);
    if (s != PE3D_OK) return s;
    if (hipEventCreateWithFlags(&fresh->done, hipEventDisableTiming) != hipSuccess) return PE3D_EDEVICE;
    plan = fresh.get();
    evict_if_full();
    g_plans[key] = std::move(fresh);
    touch(key);
  }
  if (use_graph) {
    if (plan->execs.empty()) {
      pe3d_status s = capture_plan(*plan);
      if (s != PE3D_OK) {
        // leave no partial capture behind: the next call captures again
        for (auto e : plan->execs) (void)hipGraphExecDestroy(e);
        for (auto g : plan->graphs) (void)hipGraphDestroy(g);
        plan->execs.clear();
        plan->graphs.clear();
        return s;
      }
    }
    if (use_graph == kPrepareOnly) return PE3D_OK;  // captured, not run; steps unchanged
    pe3d_status s = replay_plan(*plan, st);
    if (s != PE3D_OK) return s;
  } else {
    pe3d_status s = enqueue_plan(*plan, st);
    if (s != PE3D_OK) return s;
  }
  if (hipEventRecord(plan->done, st) != hipSuccess) return PE3D_EDEVICE;
  for (int i = 0; i < n; ++i) {
    hs[i]->j += nsteps[i];
    hs[i]->used = true;
    hs[i]->last = st;
  }
  return PE3D_OK;
}
