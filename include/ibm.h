/*
 * ibm.h -- C ABI of the MI355X (gfx950) implementation of one explicit RK3 time
 * step of the implicit, second-order, discrete-forcing immersed-boundary method
 * (Luchini et al., arXiv 2506.14328) on a staggered Cartesian channel grid,
 * with an FFT (x, z) / tridiagonal (y) pressure projection.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status: every function returns IBM_OK (0) or a negative IBM_ERR_* code; no
 *   C++ exception crosses the ABI.  ibm_last_error() gives a message.
 * Handle: opaque, owned by the library, released by ibm_destroy().
 * Memory: every array argument is a DEVICE pointer (HIP global memory, e.g. a
 *   torch tensor on the GPU), contiguous, in the layout stated below.  The
 *   library copies what it keeps and never frees caller memory.  Internal
 *   fields live in device memory the library allocates at create time.
 * Stream: all work is enqueued on the hipStream_t given at create, in stream
 *   order.  Only ibm_stats(), ibm_get_state(), ibm_get_geometry()/ibm_get_ibm_list(),
 *   ibm_profile_read(), ibm_autotune(), ibm_set_wall_velocity(), ibm_set_y_faces(),
 *   ibm_wall_shear() with modes, eager steps of a masked projection and the first
 *   ibm_set_geometry() of an instance synchronise that stream; while the caller captures
 *   the stream into a graph they return IBM_ERR_STATE before enqueuing anything.
 * Precision: fixed at create.  IBM_FP64 stores and computes everything in
 *   double.  IBM_FP32_STORAGE stores velocity, pressure and spectra as float
 *   and evaluates stencils and FFTs in float; the wall-normal tridiagonal
 *   solves, the flow-rate reductions and the immersed-boundary coefficients
 *   stay double.
 *
 * Grid (x streamwise periodic, y wall-normal bounded, z spanwise periodic):
 *   nx, nz cells in the periodic directions; ny wall-normal FACES including
 *   both box walls, so there are ny-1 cells in y.  Uniform spacings
 *   dx = lx/nx, dz = lz/nz, dy = (y_hi-y_lo)/(ny-1) (Sec. 2.1 of the paper:
 *   staggered grid, pressure at cell centres, velocity components at faces).
 * Field layout: [j][k][i], i (x) fastest, shape (ny-1, nz, nx):
 *   p at cell centres, u at west faces, w at back faces, v at south faces
 *   (row j = face j; face ny-1 is the north box wall and is implicitly 0;
 *   face 0 is the south box wall and is always 0).
 * SDF layout (signed distance to the solid, > 0 in the fluid, FP64):
 *   sdf_u (ny+1, nz, nx): rows j = -1..ny-1 at u positions (two ghost rows
 *                         outside the box, used only for wall distances)
 *   sdf_v (ny,   nz, nx): faces j = 0..ny-1 at v positions
 *   sdf_w (ny+1, nz, nx): rows j = -1..ny-1 at w positions
 */
#ifndef IBM_H
#define IBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  IBM_OK = 0,
  IBM_ERR_ARG = -1,      /* invalid argument / descriptor / size mismatch   */
  IBM_ERR_OOM = -2,      /* device allocation failed                        */
  IBM_ERR_DEVICE = -3,   /* a HIP runtime call or kernel launch failed      */
  IBM_ERR_STATE = -4,    /* call out of order (e.g. step before geometry)   */
  IBM_ERR_UNSTABLE = -5  /* NaN/Inf detected or CFL above sqrt(3)           */
};

enum { IBM_FP64 = 0, IBM_FP32_STORAGE = 1 };
enum { IBM_CFR = 0, IBM_CPG = 1 };               /* constant flow rate / pressure gradient */
enum { IBM_B_EXP = 0, IBM_B_EULER = 1, IBM_B_TAYLOR2 = 2 };
enum { IBM_TOP_WALL = 0, IBM_TOP_FREE_SLIP = 1 };   /* condition at the north box face y_hi */
enum { IBM_PROJ_FULL_BOX = 0, IBM_PROJ_MASKED = 1 }; /* pressure projection, see ibm_grid_desc */

typedef struct ibm_ctx* ibm_handle;

/* One channel instance.  n_inst descriptors are passed to ibm_create_grid. */
typedef struct {
  int32_t nx, ny, nz;   /* nx even, nx/2 and nz with prime factors in {2,3,5}; ny >= 3 */
  int32_t forcing;      /* IBM_CFR: hold the flow rate at q_target_or_pi;
                           IBM_CPG: fixed mean pressure gradient Pi = q_target_or_pi
                           (Pi enters the u-momentum equation as -Pi, Sec. 2.5 notation) */
  int32_t b_mode;       /* coefficient B of the implicit IBM update, Sec. 2.4:
                           IBM_B_EXP = exponential fit x/(e^x-1), Eq. (14);
                           IBM_B_EULER = 1 (first order); IBM_B_TAYLOR2 = 1/(1+x/2) */
  int32_t ibm;          /* 1: immersed-boundary correction on; 0: bare staircase */
  double lx, lz, y_lo, y_hi;
  double nu, dt;        /* kinematic viscosity (1/Re_bulk), fixed time step */
  double q_target_or_pi;
  int32_t top;          /* IBM_TOP_WALL: no-slip wall on the north box face (as on the south
                           one); IBM_TOP_FREE_SLIP: free-slip surface there (v = 0,
                           du/dy = dw/dy = 0: the row above mirrors the top row of u and w),
                           the open channel of Sec. 4.2 */
  int32_t projection;   /* IBM_PROJ_FULL_BOX: continuity on every cell of the box, one
                           FFT/tridiagonal solve per substep, external faces reset to zero
                           afterwards (Sec. 2.1, Sec. 3.3);
                           IBM_PROJ_MASKED: continuity on the internal pressure cells
                           only, D M G phi = D u_p / (c_k dt) (u_p the predictor) with M
                           keeping the internal faces (the external ones are never
                           corrected, Sec. 3.3 read strictly), solved by conjugate gradients
                           preconditioned with the full-box solve and started from its
                           solution; phi has zero mean over the internal cells.  With
                           IBM_FP32_STORAGE the iteration runs in FP64 with the FP32
                           full-box solve as preconditioner (the flexible Polak-Ribiere
                           update of the direction) and phi is stored in FP32.
                           Convergence is tested on the device after every iteration
                           and, once reached, the solve's remaining kernels return at once.
                           Eager steps read that flag back every 4 iterations to stop
                           launching (a host synchronisation each time) and return
                           IBM_ERR_UNSTABLE when pcg_max_iter is reached, the state then
                           holding the last iterate.  With IBM_TUNE_GRAPH on, a first step
                           runs eagerly and the captured graph then runs a fixed budget per
                           solve: the most iterations a solve has needed so far (eager, or
                           captured as read by ibm_stats) plus a quarter, at least 4 more (a
                           multiple of 4, at least 8, at most pcg_max_iter; a larger need
                           rebuilds the graph at the next ibm_step), with no host access; a
                           solve that does not converge within it makes the next ibm_stats
                           return IBM_ERR_UNSTABLE.  The internal pressure cells must be connected
                           through internal faces. */
  int32_t pcg_max_iter; /* masked: iteration cap per solve (<= 0: 500) */
  double pcg_tol;       /* masked: stop at ||r||_2 <= pcg_tol ||b||_2 over the internal cells,
                           b = D u_p / (c_k dt) (<= 0: 1e-13 with IBM_FP64, 1e-9 with
                           IBM_FP32_STORAGE) */
} ibm_grid_desc;

typedef struct {
  int64_t step;
  double time;
  double q;                     /* flow rate (1/nx) sum_{internal u} u dy dz */
  double pi_last;               /* mean pressure gradient of the last substep */
  double div_max_fullbox;       /* max |D u| after the last projection, before external
                                   faces are reset (needs ibm_set_diagnostics(h, 1)) */
  double div_max_internal_leak; /* max |D u| over internal pressure cells, current state */
  double poisson_rel_residual;  /* ||D G phi - (rhs - mean)||_inf / ||rhs||_inf (diagnostics on);
                                   masked projection: ||r||_2 / ||b||_2 at the end of the last
                                   conjugate-gradient solve */
  double rhs_mean_removed;      /* mean of the Poisson right-hand side removed by the gauge */
  double ke;                    /* 1/2 sum |u|^2 dx dy dz */
  double cfl_max;               /* max (|u|/dx + |v|/dy + |w|/dz) dt */
  int64_t n_internal[3];        /* internal u, v, w points */
  int64_t n_ibm[3];             /* points with lambda > 0 per component */
  int64_t n_p_internal;         /* internal pressure cells */
  int32_t nan_flag;             /* 1 if any field holds NaN/Inf */
  int32_t pcg_iters;            /* masked projection: iterations of the last solve; else 0 */
} ibm_stats_t;

/* Create n_inst independent channel instances (an ensemble of ragged sizes is
 * allowed; desc points to n_inst descriptors) at the given precision, all work on
 * hip_stream (a hipStream_t; NULL = default stream).  The grid is the staggered
 * second-order Cartesian grid of Sec. 2.1 (pressure at cell centres, each velocity
 * component on the faces normal to it), periodic in x and z, bounded by walls (or a
 * free-slip face) in y; the time step is the fixed dt of Sec. 2.4's RK3 integration.
 * Instances are addressed by their index in the per-instance calls; ibm_step advances
 * all of them.  Validates the descriptors (IBM_ERR_ARG: nx odd, nx/2 or nz with a prime
 * factor outside {2,3,5}, nx or nz above 1024, ny outside 3..2049, more than 2e9/3
 * cells, dt <= 0, nu <= 0, an empty box, an unknown forcing, b_mode, top, projection or
 * precision, n_inst outside 1..65536 or a null
 * pointer), allocates device fields and the FFT and tridiagonal plans (IBM_ERR_OOM;
 * IBM_ERR_DEVICE if a HIP call fails).  Fields start at zero. */
int ibm_create_grid(const ibm_grid_desc* desc, int32_t n_inst, int32_t precision,
                    void* hip_stream, ibm_handle* out);

/* Staircase tagging and immersed-boundary coefficients from signed-distance
 * samples (Sec. 2.2 Eqs. (5)-(7), Sec. 2.4 Eqs. (14)-(16), Sec. 3.3):
 * per component grid, a point is internal iff s > 0; a pressure cell is
 * internal iff one of its faces is internal; for each internal point the
 * centre-weight correction lambda = nu * sum_arms (h - delta)/(delta h^2) over
 * the arms whose neighbour is external, delta being the linear zero crossing
 * of s along the arm (or the box wall when nearer); per RK stage k,
 * x = lambda c_k dt, B(x) per b_mode, A = x + B.  sdf_* are FP64 device
 * arrays in the SDF layout above, read in stream order (they may be freed or refilled
 * once the work enqueued so far has run).  The first geometry of an instance reads the
 * point counts back, sizes the immersed-boundary lists with room to spare (the counts
 * plus a quarter, at least 1024 more per component), synchronises the stream, and returns
 * IBM_ERR_ARG if no pressure cell is internal.  A later geometry (a moving body) runs on
 * the stream only: no host read-back, no allocation, no memset, no synchronisation, the
 * library's captured graph kept, so that a caller may also capture it, with ibm_step,
 * into a graph of its own (host-side step counters then advance at capture only); its
 * counts reach the host at the next ibm_stats, which returns IBM_ERR_STATE if it left no
 * fluid or had more points than the lists hold (the next ibm_set_geometry then resizes
 * them, synchronously). */
int ibm_set_geometry(ibm_handle h, int32_t inst, const double* sdf_u, const double* sdf_v,
                     const double* sdf_w);

/* Copy a velocity/pressure state in (set) or out (get).  Arrays are device
 * pointers of the storage type (double for IBM_FP64, float for
 * IBM_FP32_STORAGE), field layout above.  set clears the stored explicit
 * right-hand side of the previous stage.  Values at external points (of the
 * geometry in force when the next step runs) are kept as given until then; the step
 * treats them as zero, the solid's velocity (Sec. 3.3), and writes zeros there. */
int ibm_set_state(ibm_handle h, int32_t inst, const void* u, const void* v, const void* w,
                  const void* p);
int ibm_get_state(ibm_handle h, int32_t inst, void* u, void* v, void* w, void* p);

/* Advance every instance by nsteps full RK3 steps (3 substeps each), Sec. 2.4
 * Eq. (16) with the incremental pressure-correction projection of Sec. 2.1
 * after every substep.  No host synchronisation.  IBM_ERR_STATE before
 * ibm_set_geometry. */
int ibm_step(ibm_handle h, int32_t nsteps);

/* Stand-alone pressure solve on the full box, the Poisson equation of the projection
 * of Sec. 2.1 (D G phi = D u_p / (c_k dt) there, u_p the predictor) solved exactly as Sec. 2.1 allows, with
 * the continuity equation imposed on every cell as Sec. 3.3 describes:
 * D G phi = rhs - mean(rhs), zero-mean phi (periodic x, z; homogeneous Neumann at the y
 * box walls), by real FFT in x, complex FFT in z and an FP64 tridiagonal solve per
 * Fourier mode in y.  rhs, phi: device arrays of the storage type, cell layout (no
 * alignment needed beyond that of the type); rhs is not modified; they may alias only
 * if identical.  The removed mean is reported by the next ibm_stats().  Stream-ordered,
 * no synchronisation.  IBM_ERR_ARG for a bad instance or null pointer. */
int ibm_solve_pressure(ibm_handle h, int32_t inst, const void* rhs, void* phi);

/* Diagnostics of the current state (synchronises the stream): the flow rate and mean
 * pressure gradient of the constant-flow-rate control (Sec. 2.5, Eq. (18) notation),
 * the divergence left by the projection of Sec. 2.1 on the full box and on the internal
 * pressure cells (Sec. 3.3), the Poisson residual, kinetic energy, CFL number and a
 * NaN/Inf flag, and the point counts of the staircase classification (Sec. 3.3) and of
 * the immersed-boundary lists (Sec. 2.2).  Fields as in ibm_stats_t; *out is fully
 * written on IBM_OK and on IBM_ERR_UNSTABLE (NaN/Inf or CFL above sqrt(3), the values
 * still reported).  IBM_ERR_ARG for a bad instance or null out. */
int ibm_stats(ibm_handle h, int32_t inst, ibm_stats_t* out);

/* Velocity (ub, vb, wb) of the immersed walls (the zero set of the signed distances),
 * a rigid translation; the box walls stay at rest.  The ghost value of a cut stencil arm
 * is the linear extrapolation through the wall velocity (Sec. 2.2, Eqs. (5)-(7) with a
 * moving wall): the implicit update gains the explicit term sigma U_b c_k dt / A, sigma
 * per immersed-boundary point from the same wall distances as lambda, and external points
 * inside the box hold U_b (the south box-wall face of v holds 0).  With a geometry that
 * moves, give the samples of each new position with ibm_set_geometry and its velocity
 * here, between steps.  Applies a pending projection first (with the previous velocity);
 * drops captured graphs (the flow-rate kernel then visits every immersed-boundary point).
 * Synchronises the stream.  IBM_ERR_ARG for a non-finite velocity. */
int ibm_set_wall_velocity(ibm_handle h, int32_t inst, double ub, double vb, double wb);

/* Stretched wall-normal grid (Sec. 2.1 allows non-uniform spacing): y_faces (host, ny
 * doubles, strictly increasing, the first y_lo and the last y_hi of the descriptor) are
 * the positions of the v faces; cell centres lie midway between their faces.  Every
 * wall-normal operator takes the spacings of its row: the three-point second derivative
 * with its non-uniform coefficient triple (Eq. (3)), lambda and sigma from the arm's own
 * coefficient and length (Eqs. (5)-(7)), u and w carried to the faces by linear
 * interpolation, the divergence and the pressure Poisson rows with the cell heights,
 * the flow rate and S_k weighted by them.  The immersed-boundary data depend on the
 * spacing: call ibm_set_geometry afterwards (IBM_ERR_STATE until then).  Applies a
 * pending projection first and drops captured graphs.  Synchronises the stream.  A
 * masked-projection instance solves the symmetric form W D M G phi = W rhs, W the cell
 * heights (the preconditioner, the full-box solve, takes W^-1 of the residual).
 * IBM_ERR_ARG for non-finite or non-increasing faces or end points other than y_lo, y_hi
 * (relative tolerance 1e-12). */
int ibm_set_y_faces(ibm_handle h, int32_t inst, const double* y_faces);

/* Wall-shear stress of the current state along the south wall, the undulated bottom
 * of the open channel (Sec. 4.2), and its Fourier components tau_1c, tau_1s defined
 * there.  Per (z_k, x_i) column of u points: the lowest internal u point, u1, at
 * distance d1 above the wall located as the immersed boundary locates it (the linear
 * zero crossing of the u signed distance towards the external point below it, or the
 * south box wall when nearer; the external point itself without the correction), and
 * tau = nu (u1 - U_b) / d1 (U_b the streamwise wall velocity of an immersed wall, 0 for
 * the box wall), the viscous flux the discretisation exchanges with the wall through
 * that stencil arm (its ghost value is the linear extrapolation through zero at the
 * wall, Sec. 2.2 Eqs. (5)-(7)).  tau_x[i] = mean over the nz columns at x_i = i dx (a
 * column with no internal u point adds 0).  modes = (tau_0, tau_1c, tau_1s): the mean
 * and (2/nx) sum_i tau_x[i] cos|sin(2 pi i/nx), the box length being one period.  The
 * paper's time average is the caller's mean over calls.
 * tau_x: device double[nx] or NULL; modes: host double[3] or NULL (then the call does
 * not synchronise the stream).  IBM_ERR_STATE before ibm_set_geometry. */
int ibm_wall_shear(ibm_handle h, int32_t inst, double* tau_x, double* modes);

/* 1: at the last substep of every ibm_step call, also measure the full-box
 * divergence before external faces are reset and the Poisson residual. */
int ibm_set_diagnostics(ibm_handle h, int32_t on);

/* Inspection of the geometry preprocessing (synchronises the stream).
 * tags: device uint8 array, cell layout; bit 0/1/2 = u/v/w internal,
 * bit 3 = pressure internal, bit 4/5/6 = u/v/w carries an IBM correction.
 * idx: device int32 [n_ibm[comp]] linear cell indices (ascending);
 * lambda: device double [n]; coef: device double [3][n][2] = (B_k, 1/A_k). */
int ibm_get_geometry(ibm_handle h, int32_t inst, uint8_t* tags, int64_t* n_ibm3);
int ibm_get_ibm_list(ibm_handle h, int32_t inst, int32_t comp, int32_t* idx, double* lambda,
                     double* coef);

/* Per-kernel timing with HIP events recorded on the library's stream around
 * every launch of the kernels selected by kernel_mask (bit k = kernel id k,
 * see ibm_kernel_name; -1 = all, 0 = off).  read() synchronises, returns the
 * accumulated milliseconds and launch counts for up to max kernels and
 * resets the accumulators.  At most 65536 launches are recorded between
 * two reads. */
int ibm_profile(ibm_handle h, int32_t kernel_mask);
int ibm_profile_read(ibm_handle h, double* total_ms, int64_t* launches, int32_t max);
const char* ibm_kernel_name(int32_t id);
int32_t ibm_num_kernels(void);

/* Launch-shape knobs (performance only: every setting gives the same result up to
 * the rounding of the reordered FP64 flow-rate sum and tridiagonal elimination).
 * 0 = automatic choice.
 *   IBM_TUNE_MOMENTUM_PLANES  y planes marched by one momentum block
 *   IBM_TUNE_FFTZ_WIDTH       x modes per z-FFT block (power of two; invalid
 *                             widths fall back to the automatic one)
 *   IBM_TUNE_TRI_ROWS         rows per thread of the tridiagonal solver: 4 or 8
 *   IBM_TUNE_TILE_ORDER       momentum tiles: 1 = each XCD takes a contiguous run of
 *                             tiles (neighbours share an L2), 2 = tiles interleaved
 *                             over the XCDs, 3..8 = super-tiles of 2x2, 4x2, 2x4, 4x4,
 *                             8x2 and 8x4 tiles (x by z) dealt round-robin to the XCDs,
 *                             the tiles of one super-tile consecutive blocks of one XCD
 *                             (they share halo lines through its L2); a grid whose tile
 *                             counts do not split into whole super-tiles dealt evenly to
 *                             the 8 XCDs takes order 2 instead */
enum { IBM_TUNE_MOMENTUM_PLANES = 0, IBM_TUNE_FFTZ_WIDTH = 1, IBM_TUNE_TRI_ROWS = 2,
       IBM_TUNE_GRAPH = 3,            /* 1: ibm_step replays a HIP graph of one RK3 step of all
                                         instances (captured on first use, rebuilt after any
                                         geometry/tuning/diagnostics change); instances run as
                                         independent graph branches.  Ignored while diagnostics
                                         or profiling are on. */
       IBM_TUNE_GRAPH_BRANCHES = 4,   /* capture streams for the graph (0 = up to 8) */
       IBM_TUNE_TILE_ORDER = 5,
       IBM_TUNE_BATCH = 6,            /* 1: an ensemble is advanced with one launch per kernel for
                                         all instances (each instance's blocks a contiguous range of
                                         the grid), also inside the graph.  Ignored for a single
                                         instance and while diagnostics or profiling are on. */
       IBM_TUNE_MOMENTUM_CACHE = 7,   /* cache policy of the momentum kernel's single-use
                                         accesses, 1 + bits: bit 0 streaming (non-temporal)
                                         stores of u*, p and H, bit 1 streaming loads of H_prev
                                         (0 = automatic: plain accesses) */
       IBM_TUNE_MOMENTUM_TILE = 8 };  /* (x, z) tile of one momentum block: 0 or 1 = 64 x 4,
                                         2 = 128 x 4, 3 = 64 x 8, 4 = 256 x 4 and 5 = 128 x 8
                                         (FP32 storage only; FP64 takes 64 x 4 for these),
                                         6 = 64 x 4 with the loads of two planes in flight;
                                         stretched grids and batched launches take 64 x 4 */
int ibm_tune_set(ibm_handle h, int32_t param, int32_t value);
int ibm_tune_get(ibm_handle h, int32_t param, int32_t* value);

/* Autotuner: for each knob in turn, time steps_per_trial RK3 steps (after one
 * warm-up step, best of two runs) from the current state for every candidate value
 * with HIP events, and keep the fastest.  Each instance is tuned on its own, except
 * for an ensemble launched as one launch per kernel for all instances (IBM_TUNE_BATCH
 * on): there the momentum planes and the tile order are tuned jointly, one value for
 * every instance, timing whole ensemble steps in that launch mode, eager or as a graph
 * (the other knobs keep their values).  An ensemble of per-instance graph branches is
 * tuned one instance at a time with eager launches.
 * The state (u, v, w, p, step count, time) of every instance is saved before and
 * restored after, so the trajectory is unchanged.  chosen (may be NULL) receives the 4
 * selected values (momentum planes, z-FFT width, tridiagonal rows, tile order; for an
 * ensemble, those of the last instance tuned on its own or of instance 0).
 * Synchronises the stream.  IBM_ERR_STATE before ibm_set_geometry. */
int ibm_autotune(ibm_handle h, int32_t steps_per_trial, int32_t* chosen);

/* Bytes of device memory the library holds for this handle. */
int64_t ibm_device_bytes(ibm_handle h);

/* Streaming device copy of `bytes` bytes from src to dst (device pointers, both 16-byte
 * aligned, bytes a multiple of 16, the ranges not overlapping), enqueued on hip_stream
 * (a hipStream_t; NULL = the default stream): 16-byte vector loads and stores over the
 * whole GPU.  It is the measured practical HBM ceiling against which the step kernels'
 * bandwidth is compared (it reads and writes every byte once).  No handle; the library
 * keeps nothing.  IBM_ERR_ARG for null pointers, misalignment, a size that is not a
 * multiple of 16 or overlapping ranges; IBM_ERR_DEVICE if the launch fails. */
int ibm_stream_copy(void* dst, const void* src, int64_t bytes, void* hip_stream);

/* Streams nsrc input arrays into ndst output arrays of `bytes` bytes each (1 <= nsrc, ndst
 * <= 8; dst and src are host arrays of device pointers, each 16-byte aligned; bytes a
 * multiple of 16): every output receives the element-wise sum of the inputs read as FP64
 * values, 16-byte vector loads and stores, enqueued on hip_stream (NULL = the default
 * stream).  It is the measured practical HBM ceiling of a kernel with the same numbers of
 * read and write streams as a step kernel (the momentum kernel moves 5..8 read and 4..7
 * write streams at once), the copy being the case of one and one.  No handle; the library
 * keeps nothing.  IBM_ERR_ARG for null or misaligned pointers, counts outside 1..8, a size
 * that is not a multiple of 16 or an output overlapping another array; IBM_ERR_DEVICE if
 * the launch fails. */
int ibm_stream_mix(void* const* dst, int32_t ndst, const void* const* src, int32_t nsrc, int64_t bytes,
                   void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the full-box pressure solve of
 * ibm_solve_pressure without a handle.  The grid is desc's (uniform wall-normal
 * spacing; only nx, ny, nz, lx, lz, y_lo and y_hi are read), the precision IBM_FP64 or
 * IBM_FP32_STORAGE, rhs and phi device arrays of that storage type in the cell layout
 * (as for ibm_solve_pressure, same kernels, same result up to the last-bit rounding of
 * the device-computed twiddle tables); mean_removed: NULL or a device double that
 * receives the mean of rhs removed by the gauge.  Work area: a fixed array of
 * IBM_NOALLOC_SCRATCH_BYTES inside the library, one per GPU (held until the process
 * ends, its device address looked up once per device on the first call there); the call
 * allocates nothing, calls no hipMalloc, hipFree or hipMemset, and only enqueues kernels
 * on hip_stream (a hipStream_t; NULL = the default stream), so it may be captured into a
 * HIP graph.  Every call on a GPU uses that GPU's one work area: calls that may run
 * concurrently on one GPU (different streams, or graphs replayed concurrently) race and
 * must be ordered by the caller.  IBM_ERR_ARG for a null argument, a grid the kernels do
 * not accept (as ibm_create_grid) or one whose half spectrum and tables exceed the work
 * area (about ny nz (nx/2 + 8) 16 bytes in FP64, half that in FP32: for example
 * 256 x 129 x 128 in FP64); IBM_ERR_DEVICE if a launch fails.  ibm_last_error(NULL)
 * gives the message. */
#define IBM_NOALLOC_SCRATCH_BYTES (64ll << 20)
int ibm_solve_pressure_noalloc(const ibm_grid_desc* desc, int32_t precision, const void* rhs, void* phi,
                               double* mean_removed, void* hip_stream);

int ibm_destroy(ibm_handle h);
const char* ibm_last_error(ibm_handle h);

#ifdef __cplusplus
}
#endif

#endif /* IBM_H */
