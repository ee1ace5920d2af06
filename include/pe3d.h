/*
 * pe3d.h - C ABI of the MI355X (gfx950) 3D wide-angle parabolic-equation
 * range march.
 *
 * The library advances the PE envelope u(r, theta, z) by the split
 * Crank-Nicolson scheme of Xu, Wang, Chronopoulos & Yue, Eq. (4):
 *
 *   [1 + (1/4 - d/4) X][1 - (d/4) Y] u^{j+1} = [1 + (1/4 + d/4) X][1 + (d/4) Y] u^j,
 *   d = i k0 dr,
 *
 * solved each step by the two-step procedure of Eqs. (5)-(8): one complex
 * tridiagonal system in depth per azimuth, then one (periodic) complex
 * tridiagonal system in azimuth per depth.  X is the depth operator
 * (n^2 - 1) + k0^-2 d^2/dz^2 (density-weighted second difference) and Y the
 * azimuth operator (k0 r)^-2 d^2/dtheta^2 (3-point second difference), both
 * from Eq. (3).  The problem statement (frequency, source, sound-speed
 * profile, range step, boundary conditions, field and transmission loss)
 * follows the algorithm of Fig. 2.
 *
 * Conventions: lengths in m, speeds in m/s, densities in g/cm^3 (only ratios
 * matter), angles in rad, attenuation in dB per wavelength, frequency in Hz.
 * Every call returns a pe3d_status; nothing throws or aborts.
 *
 * Field layout: a field is a device array of ntheta rows of nz complex
 * values, depth contiguous (row-major [ntheta][nz]), interleaved (re, im).
 * Element type: float2 (complex64) for PE3D_C64, double2 (complex128) for
 * PE3D_C128.  It must be 16-byte aligned.  The caller owns it.
 *
 * Streams: a `stream` argument is a hipStream_t passed as void* (NULL is the
 * default stream).  Marching calls are asynchronous and stream ordered: they
 * return after enqueueing; device faults surface at the caller's next
 * synchronisation with that stream.
 *
 * Threads: a handle is not thread-safe; distinct handles are independent.
 * Calls that enqueue work on one handle from several streams race.
 */
#ifndef PE3D_H
#define PE3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pe3d_handle_s* pe3d_handle;

typedef enum {
  PE3D_OK = 0,
  PE3D_EINVAL = -1,       /* bad argument; nothing was changed or enqueued  */
  PE3D_ENOMEM = -2,       /* device or host allocation failed               */
  PE3D_EDEVICE = -3,      /* a HIP runtime call or kernel launch failed     */
  PE3D_EUNSUPPORTED = -4, /* valid but outside the built kernels' limits,
                             or a depth system with a vanishing pivot       */
  PE3D_ESTATE = -5        /* call not valid in the handle's current state   */
} pe3d_status;

typedef enum { PE3D_FLOOR_PRESSURE_RELEASE = 0, PE3D_FLOOR_RIGID = 1 } pe3d_floor;
typedef enum { PE3D_C64 = 0, PE3D_C128 = 1 } pe3d_precision;
/* Coupling between azimuths.  PE3D_MODE_3D: the full operator of Eq. (4).
 * PE3D_MODE_NX2D: the "weak 3D" (N x 2D) approximation contrasted with the
 * method in Sec. 1, which ignores the azimuthal coupling: Y = 0, so each step
 * is [1 + (1/4 - d/4) X] u^{j+1} = [1 + (1/4 + d/4) X] u^j per azimuth and
 * the azimuth pass is not run. */
typedef enum { PE3D_MODE_3D = 0, PE3D_MODE_NX2D = 1 } pe3d_mode;
/* Solver of the azimuth systems of Eq. (6)/(8) (the per-depth periodic or
 * sector tridiagonal systems [1 - (d/4) Y] u^{j+1} = v).
 * PE3D_AZIMUTH_CHUNKED: each lane runs the constant-coefficient recurrences
 * of the factored operator over a chunk of azimuths (a Thomas sweep), the
 * chunks joined by a wavefront scan of their affine maps (hybrid
 * Thomas / cyclic reduction; one lane per depth line, azimuth_lanes = 1, is
 * the plain per-lane Thomas solve for ntheta <= 16).
 * PE3D_AZIMUTH_PCR: parallel cyclic reduction of the whole line in LDS, one
 * uniform multiplier per level, as many levels as the coupling needs at that
 * range step (many near the source, few far from it). */
typedef enum { PE3D_AZIMUTH_CHUNKED = 0, PE3D_AZIMUTH_PCR = 1 } pe3d_azimuth_solver;

/* Ocean environment (the sound-speed profiles, bathymetry and bottom that
 * the set-up of Fig. 2 reads).  Water: sound speed c(z) piecewise linear through
 * (ssp_z[i], ssp_c[i]) with ssp_z strictly ascending, constant beyond the
 * ends; uniform density rho_w and attenuation atten_w.  Water depth D(theta)
 * is periodic piecewise linear through (bathy_theta[i], bathy_depth[i]) with
 * bathy_theta strictly ascending over less than 2*pi (n_bathy == 1: flat).
 * A node at depth z is water iff z <= D(theta); below it is a homogeneous
 * fluid half-space (c_b, rho_b, atten_b).  zmax is the computational floor
 * with boundary condition `floor`.  The surface is pressure release.
 * Index of refraction n^2 = (c0/c)^2 (1 + i*eta*atten)^2, eta = 1/(40 pi log10 e).
 * Range-dependent depth D(r, theta) (the per-step matrix update of Fig. 2):
 * n_bathy_r >= 2 rows at ranges bathy_r0 + i*bathy_dr (bathy_dr > 0), and
 * bathy_depth then holds n_bathy_r rows of n_bathy samples (row-major), each
 * row periodic piecewise linear in theta as above; D is linear in r between
 * rows (the usual interpolation formula, correctly rounded FP64, no fused
 * multiply-add) and constant before the first and after the last row.  The
 * step j -> j+1 uses the medium at r_{j+1} on both sides of Eq. (4).
 * n_bathy_r == 0 or 1: range independent, bathy_depth holds n_bathy samples.
 * Range-dependent water n(r, z) (Eq. (2); the same matrix update): n_ssp_r
 * >= 2 profiles at ranges ssp_r0 + i*ssp_dr (ssp_dr > 0), ssp_c then holding
 * n_ssp_r rows of n_ssp speeds (row-major) on the common depths ssp_z; a
 * row holds from its range until the next row's (stair-step in range), row
 * 0 also before it, and the step j -> j+1 uses the last row whose range is
 * <= r_{j+1} (correctly rounded FP64 comparisons).  The depth factorisation
 * of every row is built at create time (one block of tables per row; see
 * pe3d_footprint).  n_ssp_r == 0 or 1: one profile of n_ssp speeds.  Water
 * rows and depth rows may be combined.
 * The arrays are copied by pe3d_create; the caller may free them after. */
typedef struct {
  double c0;                  /* reference sound speed, k0 = 2 pi f / c0   */
  int32_t n_ssp;
  const double* ssp_z;
  const double* ssp_c;
  double rho_w, atten_w;
  double c_b, rho_b, atten_b;
  int32_t n_bathy;
  const double* bathy_theta;
  const double* bathy_depth;
  int32_t n_bathy_r;          /* range rows of bathy_depth (0 or 1: none) */
  double bathy_r0, bathy_dr;  /* range of the first row, row spacing      */
  double zmax;
  int32_t floor;              /* pe3d_floor */
  int32_t n_ssp_r;            /* water-profile rows of ssp_c (0 or 1: one) */
  double ssp_r0, ssp_dr;      /* range of the first row, row spacing       */
} pe3d_env;

/* Computational grid.  Depth nodes z_l = l*dz, l = 1..nz, with
 * dz = zmax/nz (rigid floor, node nz on the floor) or dz = zmax/(nz+1)
 * (pressure-release floor).  width >= 2*pi*(1 - 1e-12) is the full circle,
 * periodic in azimuth with dtheta = 2 pi/ntheta and theta_m = theta0 + m dtheta;
 * a smaller width is a sector centred on theta0 with dtheta = width/(ntheta+1),
 * theta_m = theta0 - width/2 + (m+1) dtheta and zero field on the two edge
 * azimuths.  The march starts at range r0 with range step dr (the range loop of Fig. 2):
 * r_j = r0 + j*dr.  mode selects the azimuthal coupling (pe3d_mode; a
 * zero-initialised grid is the full 3D march).  depth_lanes and
 * azimuth_lanes override the kernels' shape for this problem, and
 * azimuth_solver the algorithm of the azimuth pass (tuning; the results
 * agree with the defaults to rounding); a value the sizes do not allow gives
 * PE3D_EUNSUPPORTED, one that is not a power of two in range, an unknown
 * solver or azimuth lanes with PE3D_AZIMUTH_PCR PE3D_EINVAL. */
typedef struct {
  int32_t nz, ntheta;
  double theta0, width;
  double dr, r0;
  int32_t precision;          /* pe3d_precision */
  int32_t mode;               /* pe3d_mode */
  int32_t depth_lanes;        /* 0: the library's choice; else the lanes per
                                 depth column of the depth pass, a power of
                                 two 4..256 giving <= 17 rows per lane */
  int32_t azimuth_lanes;      /* 0: the library's choice; else the lanes per
                                 depth line of the azimuth pass, a power of
                                 two 1..64 giving <= 16 azimuths per lane
                                 (PE3D_AZIMUTH_CHUNKED only) */
  int32_t azimuth_solver;     /* pe3d_azimuth_solver (0: chunked) */
} pe3d_grid;

typedef struct { double f_hz; } pe3d_freq;

/* Build a march for one frequency (the set-up of Fig. 2): validates all
 * arguments before touching the device, builds the medium and the depth
 * operator in FP64 on the host, factors the depth system [1 + (1/4 - d/4) X]
 * once, and allocates the handle's device buffers (coefficient tables and one
 * scratch field).  Every column is the all-water column above its interface
 * and the all-bottom column below it, so the factorisation is two shared
 * pivot chains plus one 2x2 interface block per number of water nodes; with
 * a range-dependent depth the depth kernel finds each column's water nodes
 * at r_{j+1} every step, which is the exact factorisation of that step's
 * matrix.  The range counter starts at step j = 0 (range r0).
 * Limits of the built kernels: nz <= 4096 in both precisions,
 * ntheta <= 1024; nz >= 2; ntheta >= 3 (periodic) or >= 1 (sector).
 * Precision: in both modes every coefficient and every arithmetic operation
 * is FP64; PE3D_C64 stores the field (and values held between sweeps) in
 * complex64.  Errors: PE3D_EINVAL (null pointer, non-finite or non-positive
 * f, c0, dr, zmax, speeds or densities, negative attenuation, r0 < 0,
 * unordered samples, unknown enum, n_bathy_r < 0, non-positive bathy_dr), PE3D_EUNSUPPORTED
 * (outside the limits, or a depth pivot smaller than 1e-10 of the largest
 * diagonal), PE3D_ENOMEM, PE3D_EDEVICE.  On error *out is set to NULL. */
pe3d_status pe3d_create(const pe3d_env* env, const pe3d_grid* grid,
                        const pe3d_freq* freq, pe3d_handle* out);

/* Advance the field by nsteps range steps of Eq. (4) (the range loop of Fig. 2):
 * u_dev holds u^j on entry and u^{j+nsteps} on exit (in place).  Each step
 * forms RHS = [1 + (1/4 + d/4) X][1 + (d/4) Y] u^j, solves Eq. (5) per
 * azimuth column and Eq. (6) per depth (in PE3D_MODE_NX2D: Eq. (5) only).
 * Launches one kernel per pass per step on `stream` (the plain, per-problem
 * march).  nsteps == 0 is a no-op.
 * The handle's step counter advances by nsteps at enqueue.  Errors:
 * PE3D_EINVAL (null handle or field, nsteps < 0, misaligned field),
 * PE3D_EDEVICE (launch failure). */
pe3d_status pe3d_march(pe3d_handle h, int32_t nsteps, void* u_dev, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call hipMalloc, harnesses that forbid
 * it): pe3d_march with the march's scratch field taken from a file-scope
 * device array of the library instead of the handle's, and nothing allocated
 * (no hipMalloc, hipFree or event creation; no profiling records).  Same
 * arithmetic, kernels and results as pe3d_march, bit for bit.
 * Limit: the field (nz * ntheta * 8 bytes for PE3D_C64, * 16 for PE3D_C128)
 * must fit in PE3D_STATIC_SCRATCH_BYTES (32 MiB: every complex64 shape the
 * kernels accept, complex128 up to 2 Mi points such as 2048 x 1024), else
 * PE3D_EUNSUPPORTED with nothing enqueued.  The array (one per GPU, held until
 * the process ends) is shared by every call on that GPU and keeps the last
 * call's contents; nothing in it needs to start at zero.  Calls that overlap
 * on one GPU (two streams, two threads, or an unsynchronised host) race on
 * it: the caller serialises them.  The handle's device must be the current
 * device (else PE3D_ESTATE).  Errors otherwise as pe3d_march. */
#define PE3D_STATIC_SCRATCH_BYTES ((size_t)32 << 20)
pe3d_status pe3d_march_static(pe3d_handle h, int32_t nsteps, void* u_dev, void* stream);

/* Release every device and host resource of the handle.  NULL is OK.
 * Does not synchronise the device: the handle's device memory goes back to
 * the library's pool (reused by later handles and batch plans of the same
 * size class) once an event recorded now on the stream of the handle's last
 * enqueued work has passed, so that stream must still exist at this call;
 * the batch plans that used the handle are freed once their last work has
 * finished.  Work of the handle enqueued on other streams than its last one
 * must have finished. */
pe3d_status pe3d_destroy(pe3d_handle h);

/* Return the library's pooled device memory that no handle, plan or pending
 * work holds to the runtime (hipFree, which waits for the device), on every
 * device.  Pooled blocks are otherwise kept for reuse until the process ends,
 * or until an allocation fails.  *bytes (may be NULL) receives the bytes
 * returned.  Errors: PE3D_EDEVICE. */
pe3d_status pe3d_release_pooled_memory(size_t* bytes);

/* Device bytes pe3d_create would allocate for these arguments (coefficient
 * tables, one block per water-profile row, + scratch field), excluding the
 * caller's field.  Host only. */
pe3d_status pe3d_footprint(const pe3d_env* env, const pe3d_grid* grid,
                           const pe3d_freq* freq, size_t* bytes);

/* Current step index j and range r_j of the handle. */
pe3d_status pe3d_get_step(pe3d_handle h, int64_t* j, double* r);

/* Set the step index (resume from a saved field u^j: the march is Markov in
 * (u^j, j)).  j >= 0.  Synchronises the device with the handle's last
 * stream before writing. */
pe3d_status pe3d_set_step(pe3d_handle h, int64_t j);

/* Fill u_dev with the Gaussian starter field of a source at depth zs
 * (the initial field of Fig. 2; the same on every azimuth):
 *   u(z) = sqrt(k0) [exp(-k0^2 (z - zs)^2 / 2) - exp(-k0^2 (z + zs)^2 / 2)].
 * Asynchronous on `stream`.  Errors: PE3D_EINVAL (zs not finite or < 0). */
pe3d_status pe3d_starter(pe3d_handle h, double zs, void* u_dev, void* stream);

/* Advance n problems together (the frequency loop of Fig. 2, distributed
 * over MPI ranks in Sec. 3.2.3): problem i moves by
 * nsteps[i] >= 0 steps, its field u_devs[i] in place.  All handles must have
 * the same precision, be distinct and live on the current device.
 * Schedule (pe3d_set_batch_schedule): the problems are split into chains of
 * near-equal field bytes and each chain into groups of at most group_bytes of
 * field; a group runs through all of its steps, one launch per pass per step
 * over every problem of the group still stepping (a device work table of
 * (problem, tile) items; the kernels take each problem's shape from its
 * descriptor), before the next group of its chain starts, so that its field
 * stays in the last-level cache between the passes and the steps.  When
 * use_graph != 0 each chain is captured once into a hipGraph, kept in a
 * library-wide cache of at most 64 plans (least recently used evicted and
 * freed once the work they enqueued has finished, without waiting for the
 * device; plans of a destroyed handle dropped) under the exact argument
 * tuple (handles, steps, field pointers, schedule), and replayed on later
 * identical calls:
 * chain 0 on `stream`, the others on library streams of the device that
 * wait for `stream`'s prior work, and `stream` then waits for all of them.
 * Batched calls from several threads are serialised while they enqueue.  A plan
 * must not be run by two calls at once (they would share its fields and
 * streams).  use_graph == 0 enqueues the same launches directly, on the same
 * streams.  use_graph == 2 only builds the plan and
 * captures its graphs (a later call with use_graph == 1 and the same tuple
 * replays them): nothing runs, no field or step counter changes.  Results
 * are bitwise identical to pe3d_march of each problem alone, whatever the
 * schedule.  Errors: PE3D_EINVAL, PE3D_EDEVICE, PE3D_ENOMEM. */
pe3d_status pe3d_march_batch(const pe3d_handle* hs, int32_t n,
                             const int32_t* nsteps, void* const* u_devs,
                             int32_t use_graph, void* stream);

/* Schedule of later pe3d_march_batch plans (library-wide; plans already
 * built keep theirs): chains in 1..4 independent streams of work, and
 * group_bytes >= 0 the field bytes one group of a chain may hold (0: one
 * group per chain).  Defaults 2 and 112 MiB: two chains of groups whose
 * fields (about 2 x 108 MB for the 861 MB 64-frequency batch) fit together
 * in MI355X's 256 MB last-level cache.  Errors: PE3D_EINVAL. */
pe3d_status pe3d_set_batch_schedule(int32_t chains, int64_t group_bytes);

/* Kernel of later pe3d_march_batch plans (library-wide; plans already built
 * keep theirs):
 *   PE3D_BATCH_LAUNCHES (default): one launch per pass per step per group,
 *     as described at pe3d_march_batch;
 *   PE3D_BATCH_PERSISTENT: one persistent kernel per call runs every step of
 *     every problem (the frequency loop of Fig. 2 on one device).  Its
 *     workgroups (as many as are resident at once, 256 lanes each) take
 *     tasks from a device list in order: a run of depth-pass or azimuth-pass
 *     tiles of one problem at one step.  The list holds the launches' chains,
 *     one group per chain (group_bytes is not used), their phases (one pass
 *     of one step of the group) interleaved chain by chain.  A task starts once its
 *     problem's counter shows that the other pass of its step (depth pass)
 *     or of the previous step (azimuth pass) has finished; every such wait
 *     is bounded by wait_limit_s (>= 0, finite; default 1 s): when a wait
 *     runs out the call's workgroups leave early, the call's fields and step
 *     counters are then undefined, and pe3d_batch_wait_timeouts reports it.
 *     A call whose problems include range rows (depth or water), or whose
 *     task list would exceed 2^24 tasks (20 bytes each; about steps x grid
 *     points / 16384 tasks), uses the launches.  Results are bitwise
 *     identical to the launches.
 * Errors: PE3D_EINVAL (unknown kind, wait_limit_s negative, not finite or
 * above 3600). */
#define PE3D_BATCH_LAUNCHES 0
#define PE3D_BATCH_PERSISTENT 1
pe3d_status pe3d_set_batch_kernel(int32_t kind, double wait_limit_s);

/* Waits of persistent batched marches on the current device that ran out
 * since the last call (the count is then reset).  Synchronous: call it
 * after the marches' streams have been synchronised.  Errors: PE3D_EINVAL
 * (null), PE3D_EDEVICE. */
pe3d_status pe3d_batch_wait_timeouts(int64_t* count);

/* Host only, for tests of the persistent kernel's task list: the list the
 * library builds for n problems with na[i] depth-pass tiles taken asub[i] at
 * a time and nb[i] azimuth-pass tiles (0: no azimuth pass) taken bsub[i] at
 * a time (1..16), nsteps[i] steps, in group group[i] of chain chain[i]
 * (groups numbered from 0 within each chain, problems listed in their
 * group's order).  Writes up to `cap` tasks as 6 int32 each (problem, first
 * tile, step, kind 0 depth / 1 azimuth, tiles of the task, finished tasks of
 * the problem it waits for) and sets *ntasks to the list's length.
 * Errors: PE3D_EINVAL. */
pe3d_status pe3d_persist_schedule(int32_t n, const int32_t* na, const int32_t* asub, const int32_t* nb,
                                  const int32_t* bsub, const int32_t* nsteps, const int32_t* chain,
                                  const int32_t* group, int32_t* tasks, int64_t cap, int64_t* ntasks);

/* Transmission loss of a field at the handle's current step (Sec. 4.1,
 * Fig. 5): tl[m*nz + l] = -20 log10 |u| + 10 log10 r_j, in FP32, written to a
 * device array of ntheta*nz floats.  Asynchronous on `stream`. */
pe3d_status pe3d_tl(pe3d_handle h, const void* u_dev, float* tl_dev, void* stream);

/* Complex pressure of the handle's current step j (at enqueue) from the
 * envelope: p = u H0^(1)(k0 r_j), the outgoing Hankel factor split off by the
 * PE ansatz (Sec. 2.1).  u_dev and p_dev are fields of the handle's shape and
 * precision ([ntheta][nz], complex64 or complex128, 16-byte aligned, caller
 * owned; p_dev may equal u_dev).  H0^(1) is evaluated once in FP64 on the
 * host; the device multiplies in FP64 and rounds to the field type.
 * Asynchronous on `stream`.  Errors: PE3D_EINVAL (null or unaligned
 * pointer), PE3D_ESTATE (r_j <= 0, where H0^(1) is singular), PE3D_EDEVICE. */
pe3d_status pe3d_pressure(pe3d_handle h, const void* u_dev, void* p_dev, void* stream);

/* Static description of the handle (host memory, copied to *info). */
typedef struct {
  int32_t nz, ntheta, periodic, precision, mode;
  double k0, dz, dtheta, dr, r0;
  int32_t pass_a_lanes;   /* lanes per depth column in the depth pass  */
  int32_t pass_a_chunk;   /* rows per lane                              */
  int32_t pass_b_chunks;  /* azimuth chunks per depth in the azimuth pass */
  int32_t pass_b_depths;  /* depths per workgroup                       */
  size_t device_bytes;    /* what pe3d_footprint reports                */
} pe3d_info;
pe3d_status pe3d_get_info(pe3d_handle h, pe3d_info* info);

/* Measurement support.  While enabled, every kernel launch made by
 * pe3d_march and by pe3d_march_batch with use_graph == 0 is bracketed by a
 * pair of HIP events recorded on the launch stream, together with the
 * launch's algorithmic bytes (the field read once and written once over the
 * columns or depth lines the launch covers); with more than one chain in the
 * batch schedule the chains' launches overlap in time.  pe3d_profile_read waits for
 * those events, writes up to `cap` per-kernel aggregates (in first-launch
 * order) to `stats`, sets *n to the number of distinct kernels, and clears the
 * record.  Not thread-safe against concurrent marching calls. */
typedef struct {
  char name[48];
  int32_t launches;
  double total_ms;
  double algo_bytes;
} pe3d_kernel_stat;
pe3d_status pe3d_profile_enable(int32_t on);
pe3d_status pe3d_profile_read(pe3d_kernel_stat* stats, int32_t cap, int32_t* n);

/* Host only, for tests of the coefficient builder: the FP64 tables
 * pe3d_create would upload, without touching the device.  Arrays are
 * caller-allocated, complex values as (re, im) double pairs:
 *   qw[2*nz]  n^2 - 1 of the water column at z_l,
 *   pw[2*nz]  reciprocal top-down pivots of [1 + (1/4 - d/4) X] for the
 *             all-water column, pb[2*nz] reciprocal bottom-up pivots for the
 *             all-bottom column,
 *   kcol[ntheta]   interface row k(m) of each column,
 *   blk[24*ntheta] per column, 6 complex for row k then 6 for row k+1:
 *             diagonal of [1 + (1/4 + d/4) X], its coefficients on the
 *             previous and next row of the row's elimination order (row k:
 *             k-1 and k+1; row k+1: k+2 and k), the multiplier that
 *             eliminates that previous row, and the two entries of the
 *             inverse interface 2x2 block giving the row's value (own, other).
 * With water-profile rows, the tables of row 0.
 * Same validation and errors as pe3d_create (minus device errors). */
pe3d_status pe3d_host_tables(const pe3d_env* env, const pe3d_grid* grid, const pe3d_freq* freq,
                             double* qw, double* pw, double* pb, int32_t* kcol, double* blk);

/* Static string for a status code. */
const char* pe3d_strerror(pe3d_status s);

#ifdef __cplusplus
}
#endif
#endif /* PE3D_H */
