/*
 * enoao.h -- C ABI of the MI355X (gfx950) implementation of the ENO-AO
 * finite-difference method of H. Shen, "A class of ENO schemes with adaptive
 * order for solving hyperbolic conservation laws" (arXiv 2108.12742).
 *
 * Everything below runs on the GPU: the library launches hand-written HIP
 * kernels on the caller's stream and never computes a step of the method on
 * the host.
 *
 * ----------------------------------------------------------------------------
 * Problem (Section 2, Eq. 1DHCL_Eq and 1DWENOFD; Section 4 for the Euler
 * systems): u_t + f(u)_x [+ g(u)_y] = 0 on a uniform node grid
 *   x_i = x_lo + i*dx, i = 0..nx-1, dx = (x_hi - x_lo)/nx   (same in y),
 * semi-discretised as du_i/dt = -(fhat_{i+1/2} - fhat_{i-1/2})/dx [- same in y]
 * and advanced with the third-order TVD Runge-Kutta method.
 *   ENOAO_ADVECTION  f = a u (1 component)
 *   ENOAO_EULER1D    U = [rho, rho u, rho e]           (3 components)
 *   ENOAO_EULER2D    U = [rho, rho u, rho v, rho e]    (4 components)
 * with the ideal-gas law p = (gamma-1)(rho e - rho |v|^2/2).
 *
 * The numerical flux at every face (Section 3): global Lax-Friedrichs splitting
 * f^(+/-) = (f +/- alpha u)/2 with alpha = max|f'(u)| over the grid (for the
 * Euler systems per characteristic field, after projection on the left
 * eigenvectors of the face's Roe state); the candidate stencils from first
 * order to the designed order (5 or 7); the minimum-discrepancy smoothness
 * indicators IS = min(delta_L, delta_R) of Eq. New_Smoothness_Indicator; and
 * the reconstruction principle: among indicators <= delta the highest-priority
 * stencil, otherwise the smallest indicator (ties to the higher priority).
 *
 * ----------------------------------------------------------------------------
 * Data layout and ownership
 *   A state is a caller-owned DEVICE pointer to FP64 values, contiguous SoA
 *   [ncomp][ny][nx] (ny = 1 in 1D), grid nodes only (no ghost cells: periodic
 *   or transmissive boundaries are applied inside the kernels).  The library
 *   never frees or reallocates caller memory.  A plan owns its workspace
 *   (stage buffers, per-field maxima, time-loop control, optional selection
 *   record) and any HIP graphs it captured; enoao_plan_destroy releases them.
 *
 * Streams
 *   Every call takes a hipStream_t passed as void* (NULL = the legacy default
 *   stream).  Calls enqueue work and return without synchronising, except
 *   enoao_solve, enoao_plan_check and enoao_get_selection, which wait on the
 *   stream they are given.  Calls on one plan must not overlap in time.
 *
 * Errors
 *   Every function returns an enoao_status; nothing throws across the ABI.
 *   ENOAO_EINVAL: bad argument (NULL pointer, size, unsupported combination).
 *   ENOAO_ENOMEM: device allocation failed.  ENOAO_EDEVICE: a HIP call failed.
 *   ENOAO_ENONPHYSICAL: a state with rho <= 0, p <= 0 or a NaN was met by the
 *   device-side checks; asynchronous calls report it at the next synchronising
 *   call on the plan (enoao_solve or enoao_plan_check).
 */
#ifndef ENOAO_H
#define ENOAO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum enoao_status {
    ENOAO_OK = 0,
    ENOAO_EINVAL = 1,
    ENOAO_ENOMEM = 2,
    ENOAO_EDEVICE = 3,
    ENOAO_EUNSUPPORTED = 4,
    ENOAO_ENONPHYSICAL = 5
} enoao_status;

enum { ENOAO_ADVECTION = 0, ENOAO_EULER1D = 1, ENOAO_EULER2D = 2 };
enum { ENOAO_BC_PERIODIC = 0, ENOAO_BC_TRANSMISSIVE = 1 };
/* variables the Euler systems are split and reconstructed in */
enum { ENOAO_CHAR_ROE = 0, ENOAO_COMPONENT = 1 };
/* flags */
enum { ENOAO_F_RECORD_SELECTION = 1u };

/* Largest nx or ny (2^31 - 1024): node indices a tile forms beyond the last
 * node (its halo and the lanes past the end) stay within 32-bit range. */
#define ENOAO_MAX_EXTENT 2147482624

/* Caller-filled description of one problem; copied by the create calls. */
typedef struct enoao_problem {
    uint32_t struct_size; /* sizeof(enoao_problem): ABI version check                  */
    int32_t equation;     /* ENOAO_ADVECTION | ENOAO_EULER1D | ENOAO_EULER2D            */
    int32_t order;        /* designed order: 5 or 7 (Section 3.2 candidate lists)       */
    int32_t nx;           /* nodes along x, 1 .. ENOAO_MAX_EXTENT                       */
    int32_t ny;           /* nodes along y, 1 for the 1D equations; nx*ny <= 2^31       */
    int32_t recon_vars;   /* Euler systems: ENOAO_CHAR_ROE (0, default): characteristic */
                          /*   fields of the face's Roe state, alpha per field          */
                          /*   (Section 4); ENOAO_COMPONENT: the conserved components,  */
                          /*   one alpha = max(|u| + c) for all (the scalar splitting   */
                          /*   of Section 2 applied per component).  Advection: either. */
    double x_lo, x_hi;    /* dx = (x_hi - x_lo)/nx                                      */
    double y_lo, y_hi;    /* dy = (y_hi - y_lo)/ny (2D only)                            */
    int32_t bc_x, bc_y;   /* ENOAO_BC_PERIODIC | ENOAO_BC_TRANSMISSIVE (zero gradient)  */
    double gamma;         /* ratio of specific heats (Euler), > 1                       */
    double adv_speed;     /* a of the advection equation, != 0                          */
    double delta;         /* selection threshold, >= 0 (the paper uses 1e-5)            */
    uint32_t flags;       /* ENOAO_F_RECORD_SELECTION: keep the stencil choices of the  */
                          /* last evaluation of L for enoao_get_selection               */
    uint32_t reserved1;   /* must be 0                                                  */
} enoao_problem;

typedef struct enoao_plan enoao_plan;
typedef struct enoao_batch enoao_batch;
typedef struct enoao_pool enoao_pool;

/* Validates *prob, allocates the plan's device workspace on the current HIP
 * device and returns the plan in *out.  stream: used for initialisation. */
enoao_status enoao_plan_create(const enoao_problem *prob, void *stream, enoao_plan **out);
enoao_status enoao_plan_destroy(enoao_plan *plan);

/* Device bytes a plan for *prob allocates (0 on an invalid problem). */
size_t enoao_workspace_bytes(const enoao_problem *prob);

/* L = L(u), Eq. 1DWENOFD (plus the y-part in 2D), with alpha taken from u.
 * u, L: device arrays of ncomp*ny*nx doubles; u is read only; they must not
 * overlap. */
enoao_status enoao_rhs(enoao_plan *plan, const double *u, double *L, void *stream);

/* One third-order TVD Runge-Kutta step of size dt > 0, in place on u. */
enoao_status enoao_step(enoao_plan *plan, double *u, double dt, void *stream);

/* Advance u in place from t = 0 towards t_final, at most max_steps steps.
 * dt_fixed > 0: constant step dt_fixed; otherwise the CFL step
 * (advection cfl*dx/|a|; 1D Euler cfl*dx/max(|u|+c); 2D Euler
 * cfl/max((|u|+c)/dx + (|v|+c)/dy)), computed on the device from the state at
 * the start of each step.  The step that would reach t_final
 * (dt >= (t_final - t)(1 - 1e-10)) is shortened to land on it exactly.
 * Synchronises stream; *t_out / *steps_out (may be NULL) receive the final
 * time and the number of steps taken.  The steps run as replays of a captured
 * HIP graph of several steps (the whole budget when max_steps <= 256, else 64
 * CFL steps or up to 256 fixed ones per replay); the first call with a new
 * replay length captures its graph. */
enoao_status enoao_solve(enoao_plan *plan, double *u, double t_final, double cfl, double dt_fixed,
                         int64_t max_steps, double *t_out, int64_t *steps_out, void *stream);

/* Bytes of the per-device array that enoao_step_noalloc works in (64 MiB). */
#define ENOAO_NOALLOC_SCRATCH_BYTES 67108864

/* enoao_step without a plan and without any allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops
 * that forbid allocation): one third-order TVD Runge-Kutta step of size dt > 0
 * of the problem *prob, in place on the caller's device state u (layout as
 * above), enqueued on stream.  The result is bitwise that of enoao_step on a
 * plan of *prob (the same kernel launches).
 * Workspace: a file-scope device array of ENOAO_NOALLOC_SCRATCH_BYTES that each
 * GPU the library runs on holds until the process ends; the call uses
 * 1024 + B * (ncomp*nx*ny + 544) * 8 bytes of it (B = 3 buffers for Euler 2D,
 * 2 otherwise), e.g. up to about 836 x 836 nodes for Euler 2D or 1.39 million
 * for Euler 1D; a larger problem returns ENOAO_EINVAL, as do
 * ENOAO_F_RECORD_SELECTION and the arguments enoao_step rejects.  Every call on
 * a GPU shares that GPU's array: calls that overlap in time on one GPU (other
 * streams, other host threads) race and must be serialised by the caller.
 * A non-physical state is not reported (there is no plan to hold the flag).
 * ENOAO_EDEVICE if the array's device address cannot be obtained. */
enoao_status enoao_step_noalloc(const enoao_problem *prob, double *u, double dt, void *stream);

/* Synchronises stream and returns ENOAO_ENONPHYSICAL if any device-side check
 * of the plan failed since the last synchronising call (then clears it). */
enoao_status enoao_plan_check(enoao_plan *plan, void *stream);

/* Number of selection records of a plan (0 without ENOAO_F_RECORD_SELECTION):
 *   x block [ncomp][2 sides: plus, minus][ny][nx+1] (face i between nodes i-1 and i),
 *   y block [ncomp][2][ny+1][nx] (2D only, after the x block);
 * each record is the chosen candidate 0..K-1 (K = 6 for order 5, 9 for order 7)
 * numbered S_j^j, S_j^{j+1}, S_{j-1}^{j+1}, S_{j-2}^{j+1}, S_{j-1}^{j+2},
 * S_{j-2}^{j+2}[, S_{j-3}^{j+2}, S_{j-2}^{j+3}, S_{j-3}^{j+3}], i.e. in
 * increasing priority; entries are in characteristic fields for Euler
 * (conserved components with ENOAO_COMPONENT). */
size_t enoao_selection_size(const enoao_plan *plan);

/* Copies the selection records of the last evaluation of L (enoao_rhs, or the
 * third stage of the last step) to host memory host_out[n]; n must equal
 * enoao_selection_size.  Synchronises stream. */
enoao_status enoao_get_selection(enoao_plan *plan, uint8_t *host_out, size_t n, void *stream);

/* Copies the selection records of the three Runge-Kutta stages of the last
 * step (enoao_step, or the last step of enoao_solve) to host_out[n],
 * n = 3 * enoao_selection_size: stage 1 (input u^n), stage 2 (input u^(1)),
 * stage 3 (input u^(2)), each in the layout above (Section 2, third-order TVD
 * Runge-Kutta; Section 3.2 for the records).  Each stage's record is written
 * by that stage's kernels, so the three are those of one step only after a
 * step has run; after enoao_rhs only the first is updated.  ENOAO_EINVAL
 * without ENOAO_F_RECORD_SELECTION or for another n.  Synchronises stream. */
enoao_status enoao_get_step_selection(enoao_plan *plan, uint8_t *host_out, size_t n, void *stream);

/* ---- batches: many independent problems advanced together ----------------
 * One batch holds n problems of one equation and order (any sizes, geometry,
 * boundary conditions), each with its own CFL time step, time and step
 * count.  Every Runge-Kutta stage of every member is one persistent kernel
 * launch over the flattened list of line tiles of all members; a step is
 * captured once into a HIP graph and replayed.  (1D batches whose members all
 * fit one workgroup's LDS run on the LDS-resident solver instead, see
 * enoao_set_resident; results are the same.) */
enoao_status enoao_batch_create(const enoao_problem *probs, int32_t n, void *stream, enoao_batch **out);
enoao_status enoao_batch_destroy(enoao_batch *batch);

/* Advance every member i (state u[i], a device pointer, in place) by nsteps
 * CFL steps of its own size (cfl > 0), stopping a member early once it
 * reaches t_final[i] (t_final may be NULL: no end time).  Member times and
 * step counts persist across calls until enoao_batch_reset.  The call
 * synchronises stream once at its start (member controls are read and
 * updated on the host) and returns with the steps enqueued; member status is
 * reported by enoao_batch_query. */
enoao_status enoao_batch_step(enoao_batch *batch, double *const *u, int32_t nsteps, double cfl,
                              const double *t_final, void *stream);
enoao_status enoao_batch_reset(enoao_batch *batch, void *stream);

/* Synchronises stream; copies each member's time and step count (either
 * pointer may be NULL) and returns ENOAO_ENONPHYSICAL if a member failed a
 * device-side check (member_status[i] != 0 marks it; may be NULL; bit 1 of it
 * marks a failed grid barrier of the cooperative solver, see enoao_set_coop). */
enoao_status enoao_batch_query(enoao_batch *batch, double *t, int64_t *steps, int32_t *member_status,
                               void *stream);

/* ---- pools: members that join and leave between steps --------------------
 * A pool advances a changing set of problems of one equation, order, gamma
 * and delta (those of *like) with the batched kernels.  Member states and
 * stage workspaces live in one device arena of arena_bytes owned by the pool;
 * the step graph is captured once and stays valid as members come and go.
 * Intended for serving loops: admit requests as memory frees up, step, poll,
 * retire finished ones.
 *
 * enoao_pool_member_bytes: arena bytes a member needs (0 if invalid).  The
 *   pool keeps its members' states with rows padded to 128-byte multiples;
 *   admit and retire take and give the dense [ncomp][ny][nx] layout.
 * enoao_pool_admit: copies the initial state u0 (host memory if u0_on_host,
 *   else device memory) into the arena; the member runs CFL steps (cfl > 0)
 *   until t_final or max_steps.  *slot_out receives its slot (0..max_members-1).
 *   ENOAO_ENOMEM: no free slot or no arena space now (retry after a retire);
 *   ENOAO_EINVAL: bad arguments, or the member can never fit the arena.
 * enoao_pool_step: advances every active member by up to nsteps steps (a
 *   member that has finished is skipped).  Members admitted since the last
 *   step take alpha and their first step from their current state.
 * enoao_pool_poll: synchronises stream; per slot (arrays of max_members):
 *   done (1 finished, 0 running, -1 free slot), status (non-zero: non-
 *   physical state), steps taken, time reached.
 * enoao_pool_retire: copies the member's state to u_out (host or device, may
 *   be NULL), synchronises stream and frees the slot and its arena space.
 * enoao_pool_retire_async: the same without synchronising, for callers that
 *   keep several rounds in flight (a server that retires a member right after
 *   enqueuing its last step): enqueues on stream the copy of the state to u_out
 *   (device memory, dense [ncomp][ny][nx], may be NULL) and of the member's
 *   progress to info (device memory, 4 doubles: done flag, status, steps, time,
 *   as enoao_pool_poll reports them; may be NULL), and frees the slot and its
 *   arena space at once.  Later admissions reuse that space; their copies must
 *   be enqueued on the same stream (or ordered after this call's work).
 * enoao_pool_set_launch: grid of the pool's persistent sweeps, in workgroups
 *   per CU (0: the kernels' occupancy; default 24).  The grids are sized once
 *   for a full arena; each launch shares its tiles among as many of those
 *   workgroups as give 16 tiles each, and at least as many as the occupancy
 *   keeps resident, so a pool holding a few small members runs them as a plan
 *   would, and a full one runs many short chunks that the workgroups finishing
 *   early take up (members of uneven cost even out).
 * A member's result does not depend on the other members of the pool or on
 * the launch shape.  Every call that takes a stream enqueues its device work
 * there; calls on one pool are meant to use one stream. */
size_t enoao_pool_member_bytes(const enoao_problem *prob);
enoao_status enoao_pool_create(const enoao_problem *like, int32_t max_members, size_t arena_bytes, void *stream,
                               enoao_pool **out);
enoao_status enoao_pool_destroy(enoao_pool *pool);
enoao_status enoao_pool_set_launch(enoao_pool *pool, int32_t workgroups_per_cu);
enoao_status enoao_pool_admit(enoao_pool *pool, const enoao_problem *prob, const double *u0, int32_t u0_on_host,
                              double t_final, int64_t max_steps, double cfl, int32_t *slot_out, void *stream);
enoao_status enoao_pool_step(enoao_pool *pool, int32_t nsteps, void *stream);
enoao_status enoao_pool_poll(enoao_pool *pool, int32_t *done, int32_t *status, int64_t *steps, double *t,
                             int32_t n, void *stream);
enoao_status enoao_pool_retire(enoao_pool *pool, int32_t slot, double *u_out, int32_t u_out_on_host, void *stream);
enoao_status enoao_pool_retire_async(enoao_pool *pool, int32_t slot, double *u_out, double *info, void *stream);
enoao_status enoao_pool_usage(const enoao_pool *pool, size_t *arena_used, size_t *arena_total, int32_t *members);

/* ---- per-kernel timing -------------------------------------------------
 * enoao_profile(plan, 1): subsequent enoao_step / enoao_solve calls launch
 * eagerly (no graph replay) and record a hipEvent pair around every kernel on
 * the stream the kernel runs on.  enoao_profile_read synchronises stream and
 * returns, per kernel kind, the mean duration in ms and the number of
 * launches since profiling was enabled.  Kinds (n_kinds <= 10):
 *   0..2 x-sweep of stage 1..3, 3..5 y-sweep of stage 1..3 (2D only),
 *   6 time-step control, 7 initial per-field maxima, 8 LDS-resident solver,
 *   9 cooperative solver (8 and 9: one launch per call, all of its controlled
 *   steps). */
enoao_status enoao_profile(enoao_plan *plan, int32_t enable);
enoao_status enoao_profile_read(enoao_plan *plan, double *avg_ms, int64_t *count, int32_t n_kinds, void *stream);
enoao_status enoao_batch_profile(enoao_batch *batch, int32_t enable);
enoao_status enoao_batch_profile_read(enoao_batch *batch, double *avg_ms, int64_t *count, int32_t n_kinds,
                                      void *stream);

/* Launch shape of the persistent sweeps: workgroups resident per CU
 * (1..64; 0 = the occupancy the compiler's register and LDS use allow).
 * enoao_set_launch sets the default for plans and batches created afterwards
 * (reserved must be 0); the per-object calls change an existing plan or batch
 * (its captured graph is rebuilt on the next call).  Results do not depend on
 * the launch shape: every tile is computed the same way whichever workgroup
 * runs it. */
enoao_status enoao_set_launch(int32_t workgroups_per_cu, int32_t reserved);
enoao_status enoao_plan_set_launch(enoao_plan *plan, int32_t workgroups_per_cu);
enoao_status enoao_batch_set_launch(enoao_batch *batch, int32_t workgroups_per_cu);

/* Launch shape per kernel kind: workgroups_per_cu[k] (0..64) for kind k of
 * the stage kernels, k = 0..2 the x-sweep of stage 1..3 and 3..5 the y-sweep
 * of stage 1..3 (the kinds of enoao_profile_read); 0, or k >= n_kinds, keeps
 * the object's uniform setting (enoao_plan_set_launch / enoao_batch_set_launch,
 * which in turn clears these).  The sweeps of one stage can prefer different
 * shapes (on the 2048^2 2D Euler workload: the x-sweep 6 per CU, the first
 * y-sweep 2, the others 3).  ENOAO_EINVAL: n_kinds outside 0..6, a NULL array
 * with n_kinds > 0, or an entry outside 0..64.  The captured graphs are
 * rebuilt on the next call; results do not depend on the shapes. */
enoao_status enoao_plan_set_launch_kinds(enoao_plan *plan, const int32_t *workgroups_per_cu, int32_t n_kinds);
enoao_status enoao_batch_set_launch_kinds(enoao_batch *batch, const int32_t *workgroups_per_cu, int32_t n_kinds);

/* Tile width of the 2D y-sweep: columns per wave strip, 4 or 8 (0 = the
 * default: 8 for order 5, 4 for order 7).  A y tile is 4 strips wide and 64/w cell rows tall; wider
 * strips load longer row segments per wave, narrower ones stage fewer halo
 * rows per face.  The plan's or batch's tile lists are rebuilt (this
 * synchronises stream) and its captured graph is dropped.  1D problems have
 * no y-sweep and ignore the setting.  Results do not depend on it. */
enoao_status enoao_plan_set_tiles(enoao_plan *plan, int32_t y_strip_columns, void *stream);
enoao_status enoao_batch_set_tiles(enoao_batch *batch, int32_t y_strip_columns, void *stream);

/* LDS-resident solver for small 1D problems (advection and Euler 1D, any
 * order, no selection record).  When every member of a plan or batch fits one
 * workgroup's LDS (u^n and both stage states of the whole line plus each
 * wave's staging buffer: about 1890 nodes for Euler 1D and 6600 for advection
 * on gfx950), enoao_solve and enoao_batch_step run their time-step-controlled
 * steps in launches of many steps each (up to 1024 in enoao_solve, 128 in
 * enoao_batch_step) with one 4-wave workgroup per member: the state is read
 * from HBM at the start of a launch, every step and stage runs out of LDS, and
 * the state is written back at its end.  Members are grouped by how many of
 * their workgroups one CU holds (as many as fit its LDS, at most as many as the
 * kernel's registers allow: two groups at most for Euler 1D); each group is
 * one launch, and the groups run concurrently on streams the library forks
 * from and joins back into the caller's stream.  The arithmetic is the streaming kernels' (Sections 2 to 4
 * as above), so results are bitwise the same either way.  enable = 1 (default)
 * allows it for plans and batches used afterwards, 0 forces the streaming
 * kernels; other values return ENOAO_EINVAL.  enoao_step (host-given step) and
 * pools always stream. */
enoao_status enoao_set_resident(int32_t enable);

/* Cooperative solver of one mid-sized 1D problem.  A plan (or a one-member
 * batch) of a 1D problem whose line has at most one 63-cell segment per wave of
 * one 4-wave workgroup per CU (about 64K cells on MI355X), and that is too long
 * for the LDS-resident solver or fits it with more than 9 segments (Euler;
 * advection: 20; there this path measured faster), runs the time-step-
 * controlled steps of enoao_solve and enoao_batch_step in one cooperative
 * launch (hipLaunchCooperativeKernel: every workgroup resident) of many steps:
 * the stage states stay in the plan's HBM buffers, a grid barrier replaces the
 * kernel boundary after each stage, and every workgroup takes the same
 * time-step decision from the maxima the workgroups fold together.  On such a
 * line a kernel boundary costs about as much as a stage's work.  The
 * arithmetic is the streaming kernels' (Sections 2 to 4 as above), so results
 * are bitwise the same.  A barrier wait is bounded (the bound is never meant to
 * be reached): past it the launch stops stepping, the member's status gets
 * bit 1 (value 2) and enoao_solve returns ENOAO_EDEVICE.  Cooperative
 * launches do not overlap one another: callers that solve many such plans at
 * once on several streams do better on the streaming kernels (512 plans over 8
 * streams measured 1.1 to 2.7 times faster with it off).  enable = 1 (default) allows
 * it for plans and batches used afterwards; 0 leaves such problems to the
 * resident solver or the streaming kernels; other values return ENOAO_EINVAL.
 * Devices without cooperative launches never use it.  Where the runtime turns
 * a cooperative launch down (it does in a process started while another
 * process that has made cooperative launches holds the GPU), the plan or batch
 * takes the resident solver or the streaming kernels from then on, in the same
 * call, with the same results. */
enoao_status enoao_set_coop(int32_t enable);

/* Wave-uniform shortcut of the face kernels (Section 3.2, first principle):
 * when every face of a wave has the top candidate's indicator within delta on
 * both sides of a characteristic field, that field skips the other candidates'
 * indicators and the selection, and its value is the top candidate's, formed
 * directly from the conserved-variable differences and symmetric stencil of
 * that candidate.
 * Whenever the full selection picks the top candidate on both sides it uses
 * the same top indicator and value, so results do not depend on the shortcut.
 * enable = 1 (default) or 0 (every face takes the full selection; slower, for
 * checking that property); it applies to plans, batches and pools created
 * afterwards.  Other values return ENOAO_EINVAL. */
enoao_status enoao_set_shortcut(int32_t enable);

const char *enoao_status_string(enoao_status status);

#ifdef __cplusplus
}
#endif
#endif
