// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pe3d {

// Complex number with the layout of float2 / double2 (re, im interleaved).
template <typename R>
struct alignas(2 * sizeof(R)) cplx {
  R re, im;
};

// Per-column data of the depth pass.  Row k(m) is the last water node of
// column m (clamped to 0..nz-2); rows k and k+1 hold the column's own depth
// operator coefficients (they straddle the water/bottom interface), all other
// rows use the shared all-water (above) or all-bottom (below) coefficients.
// fk, gk1: elimination multipliers that bring the top and bottom
// eliminations onto rows k and k+1; inv: inverse of the resulting 2x2 block.
// A rigid floor row that belongs to the bottom region is divided by 2 in the
// bottom system (its lower coefficient becomes beta_- h like every other
// bottom row; its right-hand side is halved to match).
template <typename R>
struct ColBlock {
  cplx<R> xl0, xd0, xu0;  // X diagonals of row k
  cplx<R> xl1, xd1, xu1;  // X diagonals of row k+1
  cplx<R> fk, gk1;
  cplx<R> i00, i01, i10, i11;
};

// Everything a kernel needs to march one problem.  Plain data; passed by
// value as a kernel argument (single-problem launches) or stored in a device
// array (batched launches).
struct ProbDesc {
  void* u;              // caller's field (first step reads it, last step writes it)
  void* scr;            // scratch field, same shape
  long long* jdev;      // device step counter (j of u on entry of the call)
  int nsteps;           // steps of the current call
  int nz, nth, periodic, rigid;
  // depth pass (pass A)
  int lpc;              // lanes per column (power of two, <= 64)
  int ma;               // rows per lane
  int ntile_a;          // number of 64-lane tiles = ceil(nth / (64/lpc))
  // lane-major tables (entry [i][t] at i*lpc + t, t = lane in the column), FP64 complex:
  const void* qwT;      // [ma][lpc]: n^2-1 of the water column at row t*ma + i
  const void* pwT;      // [ma+2][lpc]: 1/pivot of the all-water column (top-down) at row t*ma - 1 + i
  const void* pbT;      // [ma+2][lpc]: 1/pivot of the all-bottom column (bottom-up), same rows
  const void* lane_tr;  // [4][lpc]: chunk transfer products of a lane whose rows are all top
                        //   (elimination, back substitution) or all bottom
  const void* blk;      // [nth] ColBlock<double>
  const int* kcol;      // [nth] row k(m)
  double h;             // (k0 dz)^-2
  double qb_re, qb_im;  // n^2-1 of the bottom half-space
  double bp_re, bp_im;  // beta_+ = (1 + i k0 dr)/4
  double bm_re, bm_im;  // beta_- = (1 - i k0 dr)/4
  // azimuth pass (pass B)
  int nc;               // chunks per depth line
  int td;               // depths per workgroup (nc * td == kPassBThreads)
  int mb;               // azimuth nodes per chunk (nc * mb >= nth, all chunks non-empty)
  int ntile_b;          // ceil(nz / td)
  double k0, dr, r0, dth;
  double dz;            // starter / TL only
};

struct WorkItem {
  int prob;
  int tile;
};

constexpr int kPassBThreads = 512;

// kernel launchers (pe3d_kernels.hip); all return a hipError_t
// single != nullptr: one problem, grid from single->ntile_a / ntile_b, the
// descriptor passed by value.  Otherwise a batched launch over nitems items.
hipError_t launch_pass_a(int prec, int maxm, const ProbDesc* single, const ProbDesc* d_descs,
                         const WorkItem* items, int nitems, int koff, hipStream_t st);
hipError_t launch_pass_b(int prec, int maxm, const ProbDesc* single, const ProbDesc* d_descs,
                         const WorkItem* items, int nitems, int koff, hipStream_t st);
hipError_t launch_advance(long long* const* jdevs_dev, const int* adds_dev, int n,
                          long long* jsingle, int add, hipStream_t st);
hipError_t launch_starter(int prec, const ProbDesc& d, double zs, void* u, hipStream_t st);
hipError_t launch_tl(int prec, const ProbDesc& d, const void* u, float* tl, hipStream_t st);


}  // namespace pe3d
