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

// The depth-pass tables of the current step (see ProbDesc::cur).
struct TabPtrs {
  const void* tabG;
  const void* tabC;
  const void* tabP;
  const void* rec;
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
  // depth pass (pass A): L lanes per column, M rows per lane; see pe3d_kernels.hip
  int lpc;              // L, lanes per column (power of two, 4..256)
  int ma;               // M, rows per lane (odd, <= 17), nz <= (L-1) M - 1
  int ntile_a;          // workgroups = ceil(nth / (256 / L))
  int lt;               // LT, columns of the lane-major chain tables
  // chain tables, FP64 complex, [2][M][LT] (chain 0: all-water column top-down,
  // chain 1: all-bottom column bottom-up), chain row r at [(r+M) % M][(r+M) / M],
  // zero outside rows 0..nz-2; nbmh = -beta_- h:
  const void* tabG;     // nbmh / pivot of the chain row
  const void* tabC;     // diagonal of [I + beta_+ X] of the chain row, divided by nbmh
  const void* tabP;     // [2][M+1][L]: product of tabG over a lane's M slots,
                        //   by (chain, leading zero slots sc, lane in chain)
  const void* rec;      // [nz+1][12] interface rows of a column with nw water nodes
                        //   (interface row k = clamp(nw-1, 0, nz-2)): for row k then
                        //   row k+1: RHS diagonal, previous and next coefficient
                        //   along the chain, elimination multiplier (these four
                        //   divided by nbmh), and the two entries of the 2x2
                        //   block inverse that give its value (times nbmh)
  int* nwcol;           // [nth] water nodes of each column: fixed for a depth without
                        //   range rows, else rewritten for r_{j+1} before every depth pass
  const double* dcol;   // [nth][nbr] column depths at the range rows, or null
  int nbr;              // range rows (0: the depth does not depend on range)
  double br0, bdr;      // range of the first row, row spacing
  double h;             // (k0 dz)^-2
  double qb_re, qb_im;  // n^2-1 of the bottom half-space
  double bp_re, bp_im;  // beta_+ = (1 + i k0 dr)/4
  double bm_re, bm_im;  // beta_- = (1 - i k0 dr)/4
  double cbs_re, cbs_im;  // beta_+ h / nbmh, off-diagonal of the scaled depth RHS
  int bconv[2];         // per chain: rows >= bconv hold the tail values below
  double gt_re[2], gt_im[2], ct_re[2], ct_im[2];
  // range-dependent water: nsr >= 2 profile rows at ranges sr0 + i sdr, one
  // block of tables (tabG, tabC, tabP, rec) per row, row_stride bytes apart
  // from the row-0 pointers above.  The depth pass reads the tables of the
  // current step through *cur (the medium update points it at the step's
  // row before every depth pass; it holds the row-0 pointers from create
  // time on).  The bottom chain (chain 1) is the same in every row; the
  // water chain's tail constants are not used (bconv[0] = nz - 1).
  int nsr;
  double sr0, sdr;
  long long row_stride;
  TabPtrs* cur;
  // azimuth pass (pass B): W lanes per depth line, NC <= W chunks of M azimuths
  int wb;               // W, lanes per depth line (power of two, 1..64)
  int nc;               // NC = ceil(nth / M)
  int td;               // depths per workgroup = kPassBThreads / W
  int mb;               // M, azimuth nodes per chunk (<= 16)
  int ntile_b;          // ceil(nz / td)
  int bcls;             // kernel class: M (9..16) if nth == W*M, 0 (general) else,
                        //   kPcrClass for cyclic reduction (td from pcr_td; wb, nc, mb unused)
  double k0, dr, r0, dth;
  double dz;            // starter / TL only
  int nx2d;             // N x 2D mode (Y = 0): pass A writes the caller's field on
                        //   the last step, the first step reads it unchanged, and
                        //   pass B is not launched
};

struct WorkItem {
  int prob;
  int tile;
};

constexpr int kPassBThreads = 512;

// Persistent batched march (march_persist): workgroup lanes, and one task of
// its list (see pe3d_kernels.hip).  kind 0: depth-pass tiles tile ..
// tile+nsub-1 of problem `prob` at step k of the call; kind 1: azimuth-pass
// tiles tile .. tile+nsub-1 (tiles of kPersistThreads lanes).  need:
// finished tasks of the problem before this one may start.
constexpr int kPersistThreads = 256;
struct PTask {
  int prob;
  int tile;
  int k;
  int need;
  short kind;
  short nsub;
};

// Azimuth pass by parallel cyclic reduction (pass_b_pcr_body): class of the
// batched kernels' dispatch (ProbDesc::bcls), nodes (azimuth x depth) of one
// workgroup's tile held in LDS as FP64 complex, and its depths per tile: the
// largest power of two td <= 512 with td * nth <= kPcrNodes.
constexpr int kPcrClass = 1;
constexpr int kPcrNodes = 2048;
__host__ __device__ inline int pcr_td(int nth) {
  int td = 1;
  while (td < 512 && 2 * td * nth <= kPcrNodes) td *= 2;
  return td;
}

// Depth tiles of the azimuth pass: tile t covers depths [t td, (t+1) td).
// When a tile's row segment (td values) is half a 128-byte cache line, tiles
// 2q and 2q+1 share their lines.  Workgroups are dispatched round-robin over
// the 8 XCDs, each with its own L2, so such a pair goes to workgroups 8
// apart: the same XCD, dispatched together, one fetch of each line.  A
// bijection of [0, n): each group of 16 workgroups holds 8 pairs; a ragged
// last group keeps the identity.
__host__ __device__ inline int pass_b_paired_tile(int b, int n) {
  const int g = b >> 4, pos = b & 15;
  if ((g << 4) + 16 > n) return b;
  return (g << 4) + 2 * (pos & 7) + (pos >> 3);
}
__host__ __device__ inline bool pass_b_pairs(int td, int value_bytes) { return td * value_bytes < 128; }

// kernel launchers (pe3d_kernels.hip); all return a hipError_t
// single != nullptr: one problem, grid from single->ntile_a / ntile_b, the
// descriptor passed by value.  Otherwise a batched launch over nitems items
// of problems of any shape.  lds: dynamic LDS bytes (pass_a_lds / pass_b_lds,
// the largest over the problems of a batched launch).
hipError_t launch_pass_a(int prec, const ProbDesc* single, const ProbDesc* d_descs, const WorkItem* items,
                         int nitems, int koff, int lds, hipStream_t st);
int pass_a_lds(int prec, int L, int nz, int M);  // dynamic LDS bytes of one pass A workgroup
// every step of a call of one N x 2D problem without range rows in one launch
// (d.nsteps steps, the caller's field d.u in and out)
hipError_t launch_pass_a_multi(int prec, const ProbDesc& d, int lds, hipStream_t st);
hipError_t launch_pass_b(int prec, const ProbDesc* single, const ProbDesc* d_descs, const WorkItem* items,
                         int nitems, int koff, int lds, hipStream_t st);
// dynamic LDS bytes of one pass B workgroup of nthr lanes (W = 0: cyclic reduction)
int pass_b_lds(int prec, int W, int M, int nthr = kPassBThreads);
// Control words and per-problem counters of the persistent march: one
// 128-byte line each (the waiting workgroups poll them).
constexpr int kPersistCounterStride = 32;
// Finished tasks a workgroup of the persistent march publishes with one
// device-scope release (at most; fewer before a wait and at the end of the
// list).
constexpr int kPersistPublishEvery = 8;
inline int persist_ctl_ints(int nprob) { return (2 + nprob) * kPersistCounterStride; }
// The persistent batched march: ctl_done (persist_ctl_ints ints) zeroed, then
// march_persist over the task list with as many workgroups as fit on the
// device (at most ntasks).  lds: the largest dynamic LDS of the tasks' passes.
hipError_t launch_persist(int prec, const ProbDesc* d_descs, const PTask* tasks, int ntasks, int* ctl_done,
                          int nprob, long long wait_ticks, int lds, hipStream_t st);
// Waits of the persistent march that ran out since the last call (and reset).
hipError_t persist_take_timeouts(unsigned long long* n);
// the medium of the step at r_{j+1} for problems with range rows: the water
// nodes of every column (depth rows) and the water-profile row (water rows)
// (single: one problem; else nitems items of 256 columns each)
hipError_t launch_medium_update(const ProbDesc* single, const ProbDesc* d_descs, const WorkItem* items,
                               int nitems, int koff, hipStream_t st);
hipError_t launch_advance(long long* const* jdevs_dev, const int* adds_dev, int n,
                          long long* jsingle, int add, hipStream_t st);
hipError_t launch_starter(int prec, const ProbDesc& d, double zs, void* u, hipStream_t st);
hipError_t launch_tl(int prec, const ProbDesc& d, const void* u, float* tl, hipStream_t st);
hipError_t launch_scale(int prec, const ProbDesc& d, const void* u, void* p, double hre, double him,
                        hipStream_t st);  // p = u * (hre + i him)
// Bytes of the file-scope scratch field that pe3d_march_static uses (one copy
// per device); its address on the current device (looked up once per device).
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
hipError_t static_scratch(void** ptr);


}  // namespace pe3d
