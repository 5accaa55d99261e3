/*
 * imb.h -- C-ABI of libimb.so: the coupled D2Q9 lattice-Boltzmann / immersed-moving-boundary /
 * DEM time step of Yang, Jing, Kwok & Sobral, "A comprehensive study of coupled LBM-DEM with
 * immersed moving boundary" (arXiv:1809.07008), on one AMD Instinct MI355X (gfx950).
 *
 * Conventions for every call
 *   - Lattice units: dx = dt = 1.  Node (x, y), 0 <= x < nx, 0 <= y < ny, owns the unit cell
 *     [x-1/2, x+1/2] x [y-1/2, y+1/2].  x is periodic.  With IMB_FLAG_WALLS the channel has resting
 *     no-slip walls at y = -1/2 and y = ny-1/2 (half-way bounce-back, Sec. 3.1.1); without it y is
 *     periodic too.
 *   - D2Q9 populations, direction order q = 0..8: (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1)
 *     (-1,-1) (1,-1).  Population arrays exchanged with the caller are FP64, layout [q][y][x].
 *     Field arrays are FP64 [y][x].  Per-particle arrays are FP64 (mode: int32) of length n.
 *   - Pointers named host_* or documented as host memory are caller-owned host memory, read or
 *     written before the call returns.  The library never keeps them.
 *   - Return value: IMB_OK (0) or a negative IMB_E* code; imb_strerror() names it and
 *     imb_last_error() gives the message of the last failure on a handle.  No C++ exception
 *     crosses this interface.
 *   - All device work is enqueued on the HIP stream given at creation (may be NULL = the null
 *     stream).  Calls documented as "synchronises" wait for that stream.  Device-side failures
 *     (IMB_EOVERFLOW, IMB_EUNSTABLE, IMB_EDEM) are latched by the kernels and reported by the next
 *     synchronising call.  A handle must not be used from two host threads at once.
 */
#ifndef IMB_H
#define IMB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------------------- error codes */
#define IMB_OK 0
#define IMB_EINVAL (-1)     /* an argument or configuration is out of range */
#define IMB_ENOMEM (-2)     /* device allocation failed or the bound buffer is too small */
#define IMB_EHIP (-3)       /* a HIP runtime call failed */
#define IMB_EOVERFLOW (-4)  /* a fixed-capacity list overflowed (tile, slot, cell or contact list) */
#define IMB_EUNSTABLE (-5)  /* a non-finite or non-positive density appeared */
#define IMB_EDEM (-6)       /* a disk moved more than one cell in one step or left the channel */
#define IMB_EUNSUPPORTED (-7) /* the call does not support this configuration */

/* ------------------------------------------------------------------ configuration */
#define IMB_STORAGE_F64 0   /* populations stored as FP64, FP64 arithmetic (parity form) */
#define IMB_STORAGE_F32 1   /* FP32 deviations f_i - w_i rho0, FP32 arithmetic */
#define IMB_STORAGE_F16 2   /* FP16 scaled deviations (f_i - w_i rho0) * 2^14, FP32 arithmetic */

#define IMB_FLAG_WALLS 1u   /* resting half-way bounce-back walls in y (else periodic in y) */

/* batch schedules (imb_batch_set_schedule) */
#define IMB_BATCH_PERSISTENT 0
#define IMB_BATCH_PER_STEP 1

#define IMB_MODE_FREE 0      /* moved by the DEM (Eqs. 8, 10, 11, 17) */
#define IMB_MODE_FIXED 1     /* never moved; its velocity/spin still act on the fluid */
#define IMB_MODE_PRESCRIBED 2 /* moves by its velocity once per lattice step */

typedef struct imb_config {
  int32_t nx, ny;          /* lattice size, each >= 2 */
  int32_t storage;         /* IMB_STORAGE_* */
  int32_t n_sub;           /* DEM sub-cycles per lattice step, Eq. (17); >= 1 */
  double tau0;             /* BGK relaxation time, Eqs. (1), (5); must exceed 1/2 */
  double smag_cs;          /* Smagorinsky constant (Sec. 3.3.2); 0 disables it */
  double gx, gy;           /* body-force acceleration on the fluid */
  double rho0;             /* reference density (deviation storage and initial state) */
  double kn;               /* normal contact stiffness, Eq. (8) */
  double damping_ratio;    /* normal damping ratio zeta: c_n = 2 zeta sqrt(k_n m_eff) */
  double rho_solid;        /* disk density: m = rho_solid pi r^2, I = m r^2 / 2 */
  int32_t max_particles;   /* capacity, 0..512 */
  uint32_t flags;          /* IMB_FLAG_* */
  int32_t tile_w;          /* tile width in cells: 16, 32, 64, 128 or 256 (0 = 64) */
  int32_t tile_rows;       /* cell rows per thread: 1, 2 or 4 (0 = 1); a tile is
                              tile_w x (256 / tile_w * tile_rows) cells */
  int32_t eps_subcells;    /* solid ratio of a cell (Sec. 2.2): 0 = the exact covered area;
                              n = 1..64: the paper's cell decomposition, the fraction of the
                              n x n sub-cell centres strictly inside the disk (imb_adjoint
                              rejects n > 0: that estimate is piecewise constant in the position) */
  int32_t reserved;        /* must be 0 */
  double wall_ux_bottom;   /* x-velocity of the wall at y = -1/2 (walls only; |u| <= 0.3) */
  double wall_ux_top;      /* x-velocity of the wall at y = ny - 1/2: a link crossing a wall
                              that moves at u_w returns f*_i - 6 w_i rho0 (c_i . u_w), the
                              moving bounce-back (plane Couette flow between the two) */
  double kt;               /* tangential contact stiffness (Sec. 2.1 names the tangential law;
                              0 with mu = 0: normal force only, bit for bit).  With kt, mu > 0
                              each contact (disk-disk, disk-wall) adds F_t along
                              t = (-n_y, n_x): the slip at the middle of the overlap
                              v_t = (V_i - V_j).t + w_i l_i + w_j l_j (l = r - overlap/2; a wall
                              moves at its wall_ux) stretches a spring s by v_t dt per DEM
                              sub-step, F_t = -kt s - c_t v_t with c_t = 2 zeta sqrt(kt m_eff),
                              and the torque l F_t enters the spin.  A disk holds at most 6
                              disk-disk springs at once: a seventh simultaneous contact latches
                              IMB_EOVERFLOW at the next sync.  The springs are part of a saved
                              state.  imb_adjoint rejects kt or mu > 0.  Finite, >= 0. */
  double mu;               /* Coulomb limit |F_t| <= mu max(F_n, 0); a sliding contact resets
                              s = -F_t / kt.  Finite, >= 0. */
  int32_t contact_model;   /* IMB_CONTACT_LINEAR (kn, kt above) or IMB_CONTACT_HERTZ_MINDLIN:
                              the simplified Hertz-Mindlin law Sec. 2.1 adopts, taken for the
                              disks as for spheres: normal force 4/3 E* sqrt(R*) d^(3/2) +
                              2 sqrt(5/6) zeta sqrt(S_n m*) v_n, S_n = 2 E* sqrt(R* d); with
                              mu > 0 the Mindlin spring S_t = 8 G* sqrt(R* d), damping
                              2 sqrt(5/6) zeta sqrt(S_t m*), and the Coulomb limit;
                              R* = r_a r_b / (r_a + r_b) (wall: r); disks of one material:
                              E* = young / (2 (1 - poisson^2)), G* = G / (2 (2 - poisson)),
                              G = young / (2 (1 + poisson)); a rigid wall: E* = young /
                              (1 - poisson^2), G* = G / (2 - poisson).  kn and kt are then
                              unused. */
  int32_t reserved2;       /* must be 0 */
  double young;            /* Young's modulus (Hertz-Mindlin), > 0 */
  double poisson;          /* Poisson's ratio (Hertz-Mindlin), 0 <= poisson < 1/2 */
} imb_config;

#define IMB_CONTACT_LINEAR 0
#define IMB_CONTACT_HERTZ_MINDLIN 1

typedef struct imb_sim imb_sim;

/* Fills *cfg with defaults: 64x64, F64 storage, tau0 = 0.6, no Smagorinsky, no body force,
 * rho0 = 1, n_sub = 10, k_n = 1e3, zeta = 0.1, rho_solid = 1, 64 particles, walls, 64-wide tiles. */
void imb_config_default(imb_config* cfg);

/* Bytes of device memory a simulation with this configuration needs (for imb_create with a
 * caller-provided buffer). */
int imb_required_bytes(const imb_config* cfg, size_t* bytes);

/* Validates cfg (tau0 > 1/2 (Sec. 4), nx, ny >= 2, C_s >= 0, storage, capacities) and creates a
 * simulation bound to hip_stream (a hipStream_t, may be NULL).  If dev_buf is non-NULL it must
 * point to at least imb_required_bytes() bytes of device memory owned by the caller (for example
 * a torch tensor), aligned to 256 bytes; the library uses it and never frees it.  If dev_buf is
 * NULL the library allocates and later frees its own memory.  The populations start at
 * equilibrium with rho0 and zero velocity and there are no particles. */
int imb_create(const imb_config* cfg, void* hip_stream, void* dev_buf, size_t dev_bytes,
               imb_sim** out);

/* Releases the handle (after waiting for its stream).  NULL is ignored. */
void imb_destroy(imb_sim* sim);

/* f = f^eq(rho, u) everywhere, including inside solids (Eq. 2).  Asynchronous. */
int imb_init_equilibrium(imb_sim* sim, double rho, double ux, double uy);

/* Sets the post-stream populations (host, FP64, [9][ny][nx]).  Stored in the configured
 * precision.  Synchronises. */
int imb_set_populations(imb_sim* sim, const double* host_f);

/* Reads the post-stream populations of the last completed step (host, FP64, [9][ny][nx]).
 * Synchronises. */
int imb_get_populations(imb_sim* sim, double* host_f);

/* Density and velocity u = m / rho (Eqs. 3, 4) of the post-stream populations, host FP64
 * [ny][nx] each (any may be NULL).  Synchronises. */
int imb_get_fields(imb_sim* sim, double* host_rho, double* host_ux, double* host_uy);

/* Solid ratio eps_tot = sum_p eps_p of every cell for the current disk positions (Sec. 2.2, exact
 * covered area), host FP64 [ny][nx], computed by the lattice step's own mapping code in the
 * configured arithmetic precision.  Synchronises. */
int imb_get_solid_field(imb_sim* sim, double* host_eps);

/* Replaces all disks (host arrays of length n, copied before return): centre (x, y), radius r,
 * velocity (vx, vy), angular velocity omega, mode IMB_MODE_*.  Requires n <= max_particles,
 * r > 0, 2 (r + 2) < min(nx, ny) and 0 <= x < nx; with walls the centre must lie between the
 * walls.  The particles' contact forces are evaluated from this state (Sec. 2.3 starts the
 * cycle with the generated particles).  Synchronises. */
int imb_set_particles(imb_sim* sim, int32_t n, const double* x, const double* y, const double* r,
                      const double* vx, const double* vy, const double* omega,
                      const int32_t* mode);

/* Enqueues nsteps coupled steps (Sec. 2.3, Fig. 4), each:
 *   solid ratio of every cell from the disks (Sec. 2.2, exact area) ->
 *   collision Eq. (13) with weight Eq. (14), Smagorinsky relaxation, body force ->
 *   streaming Eq. (1) with periodic x and bounce-back walls ->
 *   force and torque on each disk, Eqs. (15), (16) (sign: force on the particle) ->
 *   DEM: N_sub velocity-Verlet sub-cycles with that force held fixed (Eqs. 8, 10, 11, 17).
 * Asynchronous (returns once the work is queued).  nsteps >= 0. */
int imb_step(imb_sim* sim, int32_t nsteps);

/* For callers that cannot allocate device memory or create HIP objects (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the coupled steps of imb_step,
 * launched directly on the simulation's stream (no graph capture, no event, no allocation).
 * The per-disk force and torque that each step's lattice kernel hands to its particle phase are
 * kept in a library-wide device array (256 KiB per GPU, held until the process ends) instead of
 * the simulation's buffer; every step writes every entry it reads, so nothing needs clearing.
 * Limits: at most 8192 disks (IMB_EINVAL beyond); the current HIP device must be the one the
 * simulation was created on (IMB_EINVAL otherwise).  All calls on one GPU share that array:
 * calls that can overlap in time on one GPU (different streams, different host threads) race
 * and must be ordered by the caller.  Results equal imb_step's bit for bit.  Asynchronous. */
int imb_step_noalloc(imb_sim* sim, int32_t nsteps);

/* imb_step replays captured HIP graphs of 2 or 32 steps (captured on first use, re-captured
 * after imb_set_particles / imb_load_state); enable = 0 makes it launch every kernel directly.
 * Per-kernel timing (imb_set_kernel_timing) always launches directly.  Synchronises. */
int imb_set_graphs(imb_sim* sim, int enable);

/* Captures (if not yet captured) and uploads every step graph imb_step can replay: 2 and 32
 * steps, from either population buffer, so that a later imb_step only replays graphs (no
 * capture or instantiation inside a timed region).  A graph's first replay may still carry a
 * one-time cost; timing code replays each once beforehand.  No effect with graphs disabled.
 * Synchronises. */
int imb_prepare_graphs(imb_sim* sim);

/* Force (fx, fy) and torque tz on each disk from the last completed step, FP64, host arrays of
 * length n (particle count).  Zero before the first step.  Synchronises. */
int imb_get_forces(imb_sim* sim, double* fx, double* fy, double* tz);

/* Current disk state (host arrays of length n; any may be NULL).  Synchronises. */
int imb_get_particles(imb_sim* sim, double* x, double* y, double* vx, double* vy, double* omega);

/* Number of disks and completed steps. */
int imb_get_counts(imb_sim* sim, int32_t* n_particles, int64_t* steps);

/* Waits for the stream and reports latched device errors. */
int imb_sync(imb_sim* sim);

/* Byte-exact checkpoint of the whole simulation state (populations in storage precision,
 * particles, DEM caches, step counter).  imb_state_bytes gives the size; save/load use host
 * memory and synchronise.  load requires a handle created with the same configuration. */
int imb_state_bytes(imb_sim* sim, size_t* bytes);
int imb_save_state(imb_sim* sim, void* host_buf, size_t bytes);
int imb_load_state(imb_sim* sim, const void* host_buf, size_t bytes);

/* Per-kernel timing with HIP events on the simulation's stream.  A coupled step is two kernels:
 * the lattice kernel (every cell's update, each disk's force and torque) and the particle phase
 * (DEM, the next step's disk tables).  When enabled, every launch of each records an event pair
 * at the kernel's own start and end (so the gap after the previous kernel is not counted);
 * imb_get_kernel_timing synchronises and returns the summed milliseconds and launch counts since
 * the last reset (any pointer may be NULL). */
int imb_set_kernel_timing(imb_sim* sim, int enable);
int imb_get_kernel_timing(imb_sim* sim, double* lattice_ms, int64_t* lattice_launches,
                          double* particle_ms, int64_t* particle_launches);

/* Streaming copy of n_bytes between two device buffers with the library's copy kernel, for
 * calibrating bandwidth counters.  Asynchronous on hip_stream. */
int imb_copy_kernel(void* dst, const void* src, size_t n_bytes, void* hip_stream);

/* Discrete adjoint of nsteps coupled steps from the current state (differentiation form).
 * Objective J = sum over the nsteps steps and over disks of
 *     wfx[p] * Fx_p^n + wfy[p] * Fy_p^n + wtz[p] * Tz_p^n     (host weight arrays, any NULL = 0),
 * with F, T the hydrodynamic force and torque on the disks (Eqs. 15, 16, force on the disk).
 * Requires all disks in IMB_MODE_PRESCRIBED or IMB_MODE_FIXED (IMB_EINVAL otherwise), smag_cs = 0
 * (IMB_EINVAL) and F32 or F64 storage (IMB_EUNSUPPORTED for F16).  Disk positions follow
 * X_p^n = X_p^0 + n V_p (prescribed) or stay (fixed).  Runs the forward pass keeping a checkpoint
 * every k_ckpt steps, then for each segment from the last recomputes its states and applies the
 * transposed step (Eqs. 1, 12-16 differentiated, with the analytic derivative of the exact solid
 * ratio with respect to the disk centre).  The library allocates the checkpoints
 * (ceil(nsteps / k_ckpt) + k_ckpt + 1 population copies) on first use and keeps them for later
 * calls of the same shape.
 * Outputs (host, FP64; any may be NULL): dJ/dX0, dJ/dY0, dJ/dVx, dJ/dVy, dJ/domega (length n
 * each), dJ/dg (2 values: x, y), J, and dJ/df0 ([9][ny][nx]: the gradient with respect to the
 * post-stream populations at the start, as imb_set_populations takes them).
 * The simulation state afterwards is the state after the nsteps forward steps.  Synchronises. */
int imb_adjoint(imb_sim* sim, int32_t nsteps, int32_t k_ckpt, const double* wfx,
                const double* wfy, const double* wtz, double* gx0, double* gy0, double* gvx,
                double* gvy, double* gom, double* gg, double* J, double* gf0);

/* The same run split in two, for reverse-mode automatic differentiation: imb_adjoint_forward
 * validates as imb_adjoint, runs the forward pass keeping its checkpoints and per-step disk
 * tables, advances the simulation by nsteps and returns J (host, may be NULL); it arms one
 * reverse sweep.  imb_adjoint_backward runs that sweep (recomputation from the checkpoints and
 * the adjoint steps) and returns the gradients as imb_adjoint does.  IMB_EINVAL if no forward
 * pass is armed: imb_set_particles, imb_load_state and a completed backward call disarm it.
 * Between the two calls the simulation may be read or stepped (the sweep uses its own copies of
 * the states and tables), but its disks must not be replaced.  imb_adjoint is forward then
 * backward.  Both synchronise. */
int imb_adjoint_forward(imb_sim* sim, int32_t nsteps, int32_t k_ckpt, const double* wfx,
                        const double* wfy, const double* wtz, double* J);
int imb_adjoint_backward(imb_sim* sim, double* gx0, double* gy0, double* gvx, double* gvy,
                         double* gom, double* gg, double* gf0);

/* GPU time of the last forward pass and reverse sweep (HIP events): the forward pass and the reverse sweep
 * (recomputation + adjoint steps + finalisation), in milliseconds.  With kernel timing on
 * (imb_set_kernel_timing), also the summed time and count of the adjoint-step and recompute
 * launches since the last call of this function (which resets them).  Any pointer may be NULL. */
int imb_get_adjoint_timing(imb_sim* sim, double* forward_ms, double* reverse_ms,
                           double* adjoint_kernel_ms, int64_t* adjoint_kernels,
                           double* recompute_kernel_ms, int64_t* recompute_kernels);

/* -------------------------------------------------------------- batched channels
 * Many independent simulations (channels), each with its own configuration (lattice size,
 * relaxation time, disks), advanced together; the launches of one imb_batch_step call are
 * captured once per (nsteps, buffer parity) in a hipGraph and replayed.  Two schedules:
 *   IMB_BATCH_PERSISTENT: ONE persistent kernel per call.  The channels are split into two
 *     halves of about equal tile counts; every step is two phases separated by grid-wide
 *     barriers (lattice tiles of one half while the particle phases of the other half run),
 *     with workgroups pulling work items (a channel's particle phase, a chunk of (channel, disk)
 *     items or a chunk of (channel, tile) items) from an atomic counter.
 *   IMB_BATCH_PER_STEP: two launches per step, the lattice part of every channel (disk items,
 *     then tiles) and one particle-phase workgroup per channel.
 * The method per channel is the coupled step of imb_step (Sec. 2; Eqs. 1-2, 12-17), and a
 * channel evolves bit for bit as the same channel would alone with the same tile shape, under
 * either schedule.
 * Limits: 1..128 channels, F32 storage (IMB_EINVAL / IMB_EUNSUPPORTED otherwise), at most 512
 * disks per channel (max_particles), of which the persistent schedule takes 256: a batch with
 * a channel of max_particles > 256 starts on the per-step schedule, refuses the persistent one
 * (IMB_EUNSUPPORTED) and the autotuner tries only the per-step one.  A barrier that does not
 * open within 2 s aborts
 * the kernel (every workgroup exits) and the next synchronising call returns IMB_EHIP. */
typedef struct imb_batch imb_batch;

/* Device bytes for a batch of nsim channels (the caller may bind a buffer of this size). */
int imb_batch_required_bytes(int32_t nsim, const imb_config* cfgs, size_t* bytes);
/* Creates the batch (every channel at rest at rho0, no disks).  dev_buf: caller-owned device
 * buffer of imb_batch_required_bytes (256-byte aligned) or NULL for a library allocation.  The
 * tile shape of cfgs[0] is the initial shape of every channel.  Synchronises. */
int imb_batch_create(int32_t nsim, const imb_config* cfgs, void* hip_stream, void* dev_buf,
                     size_t dev_bytes, imb_batch** out);
void imb_batch_destroy(imb_batch* b);
/* As imb_set_particles for channel `sim`. Synchronises. */
int imb_batch_set_particles(imb_batch* b, int32_t sim, int32_t n, const double* x,
                            const double* y, const double* r, const double* vx, const double* vy,
                            const double* omega, const int32_t* mode);
/* Enqueues nsteps coupled steps of every channel (one persistent launch).  Asynchronous. */
int imb_batch_step(imb_batch* b, int32_t nsteps);
/* Per-channel readback, as the single-simulation calls (host FP64 arrays).  Synchronise. */
int imb_batch_get_forces(imb_batch* b, int32_t sim, double* fx, double* fy, double* tz);
int imb_batch_get_particles(imb_batch* b, int32_t sim, double* x, double* y, double* vx,
                            double* vy, double* omega);
int imb_batch_get_fields(imb_batch* b, int32_t sim, double* rho, double* ux, double* uy);
int imb_batch_get_populations(imb_batch* b, int32_t sim, double* host_f);
/* Waits for the batch and reports an abort or any channel's device error. */
int imb_batch_sync(imb_batch* b);
/* Persistent-grid size (workgroups; 0 = every co-resident workgroup, larger values are
 * clamped to that) and tile shape of every channel (0 keeps the current value).  Rebuilds the
 * disk tables for a new shape.  Synchronises. */
int imb_batch_set_launch(imb_batch* b, int32_t grid, int32_t tile_w, int32_t tile_rows);
/* Current grid, tile shape and the co-resident maximum (any pointer may be NULL). */
int imb_batch_get_launch(imb_batch* b, int32_t* grid, int32_t* tile_w, int32_t* tile_rows,
                         int32_t* max_grid);
/* Schedule of the batch (IMB_BATCH_PERSISTENT, the default, or IMB_BATCH_PER_STEP; other values
 * IMB_EINVAL; IMB_BATCH_PERSISTENT on a batch with a channel of more than 256 disks
 * IMB_EUNSUPPORTED).  set synchronises. */
int imb_batch_set_schedule(imb_batch* b, int32_t schedule);
int imb_batch_get_schedule(imb_batch* b, int32_t* schedule);
/* Autotuner: times trial_steps steps (after 2 warm-up steps) for each candidate tile shape
 * (16x4, 32x1/2/4, 64x1/2/4, 128x1/2: tile width x rows per thread) under the per-step schedule
 * and under the persistent schedule with two grid sizes (every co-resident workgroup, or one
 * workgroup fewer per compute unit), rebuilding the disk tables for the shape and restoring the
 * channels' state after every trial, and keeps the fastest (shape, schedule, grid).
 * max_trials > 0 caps the number of trials.  *trial_ms (may be NULL) receives the best time per
 * step.  Needs a temporary device copy of the channels' memory.  Synchronises; the simulation
 * state is unchanged. */
int imb_batch_autotune(imb_batch* b, int32_t trial_steps, double* trial_ms, int32_t max_trials);
/* Runs nsteps steps as one graph replay bracketed by HIP events and returns the elapsed
 * milliseconds.  Synchronises. */
int imb_batch_get_timing(imb_batch* b, int32_t nsteps, double* ms);
/* Message of the last failure on this batch (b = NULL: of the last failed create). */
const char* imb_batch_last_error(const imb_batch* b);

/* ------------------------------------------------------- one GPU's share of a split lattice
 * A lattice split in y into nslabs slabs of whole tile rows, as one device of a multi-GPU run
 * would hold it: each slab stores only its rows and runs the coupled step of imb_step on them
 * (Sec. 2.2, Eqs. 1, 2, 12-14 per cell; Eqs. 15, 16 per disk over the slab's own cells).  Pull
 * streaming across a slab face needs the populations that cross it (c_y = +1 from the slab
 * below, -1 from the slab above): each slab's population planes hold a ghost row on each side,
 * into which those three rows of the neighbour's boundary row are copied between steps.  Each
 * slab writes its share of every disk's force and torque (zero for disks whose box misses it).
 * After the slabs' lattice kernels one kernel does every ghost-row copy (standing in for the
 * transfer between devices) and sums the shares in slab order (standing in for the
 * all-reduce); the particle phase then runs once per slab on identical inputs (replicated DEM),
 * each writing the disk tables of its own rows.  Walls end the lowest and highest slabs; without walls they are
 * neighbours across the periodic boundary.  Every slab lives on the calling thread's current
 * device and works on hip_stream.  Results equal imb_sim's up to the order of the per-disk sums
 * (bit for bit where forces do not feed back: fixed or prescribed disks).
 * Host arrays as for imb_sim (populations [9][ny][nx] FP64).  Errors: IMB_EINVAL for bad
 * arguments (nslabs outside 2..16 or more slabs than tile rows), otherwise as imb_create /
 * imb_step; messages from imb_slab_last_error. */
typedef struct imb_slab imb_slab;

/* Splits cfg's lattice (validated as by imb_create) into nslabs slabs and allocates them; the
 * fluid starts at rest at rho0 with no disks.  Synchronises. */
int imb_slab_create(const imb_config* cfg, int32_t nslabs, void* hip_stream, imb_slab** out);
void imb_slab_destroy(imb_slab* s);
/* First row and row count of each slab (host arrays of nslabs). */
int imb_slab_layout(const imb_slab* s, int32_t* y0, int32_t* rows);
/* As imb_init_equilibrium, imb_set_populations, imb_get_populations and imb_get_fields, on the
 * whole lattice (each slab handles its rows and its ghost rows).  Synchronise. */
int imb_slab_init_equilibrium(imb_slab* s, double rho, double ux, double uy);
int imb_slab_set_populations(imb_slab* s, const double* host_f);
int imb_slab_get_populations(imb_slab* s, double* host_f);
int imb_slab_get_fields(imb_slab* s, double* rho, double* ux, double* uy);
/* As imb_set_particles, on every slab.  Synchronises. */
int imb_slab_set_particles(imb_slab* s, int32_t n, const double* x, const double* y,
                           const double* r, const double* vx, const double* vy, const double* om,
                           const int32_t* mode);
/* Enqueues nsteps coupled steps of every slab (replays captured graphs of 2 and 32 steps unless
 * kernel timing is on).  Asynchronous. */
int imb_slab_step(imb_slab* s, int32_t nsteps);
/* Summed hydrodynamic force and torque on each disk from the last step (as imb_get_forces). */
int imb_slab_get_forces(imb_slab* s, double* fx, double* fy, double* tz);
/* Slab `slab`'s share of each disk's force and torque from the last step.  Synchronises. */
int imb_slab_get_partial_forces(imb_slab* s, int32_t slab, double* fx, double* fy, double* tz);
/* Slab `slab`'s copy of the disk state (as imb_get_particles).  Synchronises. */
int imb_slab_get_particles(imb_slab* s, int32_t slab, double* x, double* y, double* vx,
                           double* vy, double* om);
/* Per-kernel timing with HIP events at each launch's start and end (direct launches while
 * enabled).  imb_slab_get_kernel_timing returns, since the last enable, the summed milliseconds
 * of each slab's lattice kernel and particle phase (host arrays of nslabs, may be NULL), of the
 * exchange kernel, and the number of timed steps.  Synchronises. */
int imb_slab_set_kernel_timing(imb_slab* s, int enable);
int imb_slab_get_kernel_timing(imb_slab* s, double* lattice_ms, double* exchange_ms,
                               double* particle_ms, int64_t* nsteps);
/* Waits for the stream and checks every slab's device error flags. */
int imb_slab_sync(imb_slab* s);
/* Message of the last failure on s (s = NULL: of the last failed imb_slab_create). */
const char* imb_slab_last_error(const imb_slab* s);

/* ------------------------------------------------------- three dimensions: D3Q19 with spheres
 * The lattice step of the paper's own three-dimensional method (Sec. 2 with the D3Q19 set of
 * Table 1; Sec. 2.2, Eqs. 12-16 for the spheres), for fixed spheres and spheres moving with a
 * prescribed velocity (no DEM): BGK with the body force G_i = 3 w_i rho (c_i . g), the
 * immersed-moving-boundary collision with the paper's cell-decomposition solid ratio (the share
 * of the n^3 sub-cell centres of a cell strictly inside the sphere), pull streaming (periodic in
 * x and z; half-way bounce-back walls at y = -1/2 and ny - 1/2 with IMB_FLAG_WALLS, else
 * periodic y), and the force and torque vectors on every sphere (Eqs. 15, 16, force on the
 * sphere).  Several spheres in one cell: eps_tot = min(1, sum eps_p), split in proportion.
 * Node (x, y, z) owns the unit cube centred on it.
 * D3Q19 velocity order q (populations exchanged through this interface, FP64 [19][nz][ny][nx]):
 *   0 rest; 1-6: +x -x +y -y +z -z; 7-10: (+1,+1,0) (-1,-1,0) (+1,-1,0) (-1,+1,0);
 *   11-14: (+1,0,+1) (-1,0,-1) (+1,0,-1) (-1,0,+1); 15-18: (0,+1,+1) (0,-1,-1) (0,+1,-1) (0,-1,+1).
 * Fields are FP64 [nz][ny][nx]; per-sphere vectors are FP64 [n][3].  Errors and threading as for
 * imb_sim; messages from imb3_last_error. */
typedef struct imb3_config {
  int32_t nx, ny, nz;      /* lattice size: nx >= 1, ny >= 2, nz >= 1 */
  int32_t storage;         /* IMB_STORAGE_F64 or IMB_STORAGE_F32 (deviations f - w rho0) */
  double tau0;             /* BGK relaxation time, > 1/2 (Eq. 5) */
  double gx, gy, gz;       /* body-force acceleration on the fluid */
  double rho0;             /* reference density (initial state, deviation storage) */
  int32_t max_spheres;     /* capacity, 0..256 */
  int32_t eps_subcells;    /* n of the paper's n^3 sub-cell solid ratio, 1..64 (the paper: 5) */
  uint32_t flags;          /* IMB_FLAG_WALLS: walls in y */
  int32_t tile_w;          /* tile width 16, 32 or 64 (tile = tile_w x 256/tile_w cells of one
                              z layer); 0 picks the one with the fewest padded cells */
  int32_t reserved;        /* must be 0 */
  int32_t reserved2;       /* must be 0 */
} imb3_config;

typedef struct imb3_sim imb3_sim;

/* Defaults: 32^3, F64, tau0 0.6, rho0 1, no body force, 8 spheres, n = 5, walls, tile auto. */
void imb3_config_default(imb3_config* cfg);
int imb3_required_bytes(const imb3_config* cfg, size_t* bytes);
/* As imb_create: dev_buf (caller-owned, 256-byte aligned, >= imb3_required_bytes) or NULL for a
 * library allocation; the fluid starts at rest at rho0 with no spheres.  Synchronises. */
int imb3_create(const imb3_config* cfg, void* hip_stream, void* dev_buf, size_t dev_bytes,
                imb3_sim** out);
void imb3_destroy(imb3_sim* sim);
/* f = f^eq(rho, u) everywhere (Eq. 2).  Asynchronous. */
int imb3_init_equilibrium(imb3_sim* sim, double rho, double ux, double uy, double uz);
/* f = f^eq(rho, (ux_of_y[y], 0, 0)): a shear flow along x (host array of ny values), e.g. the
 * undisturbed Poiseuille profile as a starting state.  Synchronises. */
int imb3_init_shear(imb3_sim* sim, double rho, const double* ux_of_y);
/* Post-stream populations, host FP64 [19][nz][ny][nx].  Synchronise. */
int imb3_set_populations(imb3_sim* sim, const double* host_f);
int imb3_get_populations(imb3_sim* sim, double* host_f);
/* Density and velocity of the post-stream populations (Eqs. 3, 4), host FP64 [nz][ny][nx] each
 * (any may be NULL).  Synchronises. */
int imb3_get_fields(imb3_sim* sim, double* rho, double* ux, double* uy, double* uz);
/* eps_tot of every cell for the current sphere positions, host FP64 [nz][ny][nx].  Synchronises. */
int imb3_get_solid_field(imb3_sim* sim, double* host_eps);
/* Replaces all spheres (host arrays of length n): centre, radius, velocity, angular velocity,
 * mode IMB_MODE_FIXED or IMB_MODE_PRESCRIBED (moves by its velocity once per step).  Requires
 * n <= max_spheres, r > 0, 2 (r + 2) < nx, ny and nz, the centre inside the lattice (between the
 * walls with IMB_FLAG_WALLS), and at most 4096 tiles per sphere box.  Synchronises. */
int imb3_set_spheres(imb3_sim* sim, int32_t n, const double* x, const double* y, const double* z,
                     const double* r, const double* vx, const double* vy, const double* vz,
                     const double* wx, const double* wy, const double* wz, const int32_t* mode);
/* Enqueues nsteps steps (replays captured graphs of 32 steps).  Asynchronous. */
int imb3_step(imb3_sim* sim, int32_t nsteps);
/* Force F[n][3] and torque T[n][3] on each sphere from the last step (host, any may be NULL).
 * Synchronises. */
int imb3_get_forces(imb3_sim* sim, double* F, double* T);
/* Current sphere centres and radii, host FP64 [n][4] (x, y, z, r).  Synchronises. */
int imb3_get_spheres(imb3_sim* sim, double* xyzr);
int imb3_sync(imb3_sim* sim);
/* Per-kernel timing with HIP events recorded at each launch's start and end (direct launches
 * while enabled): summed milliseconds and counts of the lattice kernel and the force
 * finalisation since the last enable. */
int imb3_set_kernel_timing(imb3_sim* sim, int enable);
int imb3_get_kernel_timing(imb3_sim* sim, double* lattice_ms, int64_t* lattice_launches,
                           double* finalize_ms, int64_t* finalize_launches);
const char* imb3_last_error(const imb3_sim* sim);

/* ------------------------------------------------------------------------ misc */
const char* imb_strerror(int code);
const char* imb_last_error(const imb_sim* sim);
/* Library version string. */
const char* imb_version(void);

#ifdef __cplusplus
}
#endif
#endif /* IMB_H */
