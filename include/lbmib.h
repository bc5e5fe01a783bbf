/*
 * lbmib.h -- C ABI of the MI355X (gfx950) implementation of the
 * distribution-function-correction immersed-boundary lattice Boltzmann method
 * of Tao, He, Chen and Huang (arXiv:1803.09380).
 *
 * One time step of a simulation, all on the GPU:
 *   1. fused D2Q9 collision (BGK, or the MRT operator of Eq. 2) and streaming
 *      (Eqs. 1, 3, 7), in place with the AA access pattern;
 *   2. boundary rules for populations entering through the lattice edge
 *      (half-way bounce-back as in Fig. 2, specular free slip, velocity inlet by
 *      non-equilibrium extrapolation as in Sec. 3.2, zero-gradient outflow);
 *   3. N sweeps of the distribution-function correction of Sec. 2.3: interpolate
 *      at each Lagrangian marker with the 4-point cosine delta of Eq. 15(c),
 *      form the deviation of Eq. 28, spread it back with the same delta
 *      (Eq. 26) and correct (Eq. 27); all markers of a body group read the
 *      same iterate (Jacobi);
 *   4. hydrodynamic force and torque of each body (Eqs. 29 and 38) reduced in
 *      FP64, and the rigid-body update of free circles (Eqs. 37, 39-42).
 *
 * Conventions.
 *   Lattice units: dx = dt = 1, c_s^2 = 1/3.  Node (x, y) sits at integer
 *   coordinates 0 <= x < nx, 0 <= y < ny; host field arrays are [ny][nx] with x
 *   fastest; population arrays are [9][ny][nx] in the order e0=(0,0), e1=(1,0),
 *   e2=(0,1), e3=(-1,0), e4=(0,-1), e5=(1,1), e6=(-1,1), e7=(-1,-1), e8=(1,-1)
 *   (the order fixed by the j_x and j_y rows of Eq. 5), weights 4/9, 1/9, 1/36.
 *   Host arrays passed in are copied before the call returns; output arrays are
 *   caller-owned.  Device pointers (the *_device variants) are HIP device
 *   allocations on the device that was current at lbm_create.
 *   Every call returns lbm_status and never aborts the process.  Calls on one
 *   handle must come from one thread at a time; distinct handles are
 *   independent.  lbm_step and lbm_batch_step only enqueue work on the handle's
 *   HIP stream; calls that return host data synchronise that stream.
 */
#ifndef LBMIB_H
#define LBMIB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_ERR_INVALID = 1,  /* bad argument; nothing was changed                */
    LBM_ERR_NOMEM = 2,    /* device memory or the batch's HBM budget exhausted */
    LBM_ERR_DEVICE = 3,   /* a HIP call failed; the handle should be destroyed */
    LBM_ERR_UNSTABLE = 4, /* a density went non-positive or non-finite         */
    LBM_ERR_STATE = 5     /* call not valid in the handle's current state      */
} lbm_status;

typedef enum {
    LBM_F64 = 0,         /* populations f_i stored and updated in FP64                 */
    LBM_F32_SHIFTED = 1  /* h_i = f_i - w_i rho0 stored and updated in FP32; marker
                            force, torque, residual and rigid bodies stay FP64        */
} lbm_precision;

typedef enum {
    LBM_BC_PERIODIC = 0, /* both sides of an axis                                   */
    LBM_BC_WALL = 1,     /* half-way bounce-back, wall half a spacing outside       */
    LBM_BC_FREESLIP = 2, /* south/north only: specular reflection                   */
    LBM_BC_VELOCITY = 3, /* west only: every population of column 0 is set to
                            f^eq(rho(1), u_in) + f(1) - f^eq(rho(1), u(1))           */
    LBM_BC_OUTFLOW = 4,  /* east only: populations entering from the east copy the
                            post-stream values of column nx-2                        */
    LBM_BC_PRESSURE = 5, /* east only, nx >= 5: every population of column nx-1 is set
                            to f^eq(rho0, u(nx-2)) + f(nx-2) - f^eq(rho(nx-2), u(nx-2))
                            (non-equilibrium extrapolation at fixed density, Sec. 3.2) */
    LBM_BC_DIRICHLET = 6 /* all four sides or none: prescribed velocity u_b of every
                            boundary node (lbm_set_boundary_velocity); each population
                            of a boundary node is f^eq(rho(n), u_b) + f(n) - f^eq(rho(n),
                            u(n)) with n the inward neighbour, the diagonal one at
                            corners (non-equilibrium extrapolation, Sec. 3.1.1)       */
} lbm_bc;

/* A population entering a corner node through both an west/east and a
 * south/north side follows the west/east rule. */

typedef struct {
    int32_t nx, ny;       /* lattice size, each >= 4                               */
    double tau;           /* BGK relaxation time, > 0.5; nu = (tau - 1/2)/3       */
    double rho0;          /* reference density (initial state, FP32 shift, rho_f) */
    int32_t precision;    /* lbm_precision                                         */
    int32_t bc_west, bc_east, bc_south, bc_north; /* lbm_bc                        */
    double u_in[2];       /* inlet velocity for LBM_BC_VELOCITY                    */
    double u_init[2];     /* initial uniform velocity: f = f^eq(rho0, u_init)      */
    int32_t ib_iters;     /* correction sweeps per step, N >= 0 (about 10)         */
    double gravity[2];    /* gravitational acceleration acting on free bodies      */
    int32_t collision;    /* lbm_collision                                         */
    double mrt_s[9];      /* LBM_MRT: relaxation rates of Eq. 6 in the moment order
                             of Eq. 5 (rho, e, epsilon, j_x, q_x, j_y, q_y, p_xx,
                             p_xy); the conserved ones (0, 3, 5) are not used      */
    int32_t delta;        /* discrete delta function of Eq. 15 used by the
                             correction: 2 (hat), 3 (three-point), 4 or 0 (cosine,
                             the paper's choice)                                   */
} lbm_params;

typedef enum {
    LBM_BGK = 0, /* f' = f - (f - f^eq)/tau                                      */
    LBM_MRT = 1  /* Eq. 2 with the moment matrix of Eq. 5 and the rates of Eq. 6;
                    with every rate 1/tau it equals LBM_BGK                        */
} lbm_collision;

typedef enum {
    IB_FIXED = 0, /* markers at given positions with given (or rigid-motion) velocities */
    IB_FREE = 1   /* rigid circle moved by Eqs. 37-42; markers generated on the circle  */
} ib_kind;

typedef struct {
    int32_t kind;   /* ib_kind                                                   */
    double xc[2];   /* centre: torque reference; free circles: centre of mass    */
    double U[2];    /* translational velocity                                   */
    double omega;   /* angular velocity, counter-clockwise positive             */
    double theta;   /* orientation of marker 0 (free circles)                   */
    double radius;  /* circle radius (free circles)                             */
    double rho_s;   /* solid density (free circles)                             */
} ib_body;

typedef struct lbm_sim lbm_sim;
typedef struct lbm_batch lbm_batch;

#define LBM_MAX_BODIES 8
#define LBM_MAX_GROUP_MARKERS 4096 /* markers in one group of interacting bodies     */
#define LBM_MAX_FREE_MARKERS 512   /* markers in a simulation that has free bodies  */

/* Create a simulation on the current HIP device: the lattice of Sec. 2.1
 * (D2Q9, Eq. 4), the relaxation of Eq. 2 (BGK with S = I/tau, or the MRT
 * rates of Eq. 6; viscosity from tau by Eq. 8), the boundary rules named
 * above (Fig. 2, Secs. 3.1.1 and 3.2), and every population at the
 * equilibrium of Eq. 3 for (rho0, u_init).  *p is copied; the handle owns its
 * device memory until lbm_destroy.  hip_stream is a hipStream_t (NULL: a
 * stream the handle creates and owns).  Errors: LBM_ERR_INVALID (sizes,
 * tau <= 1/2, boundary pairing: periodic sides come in pairs, FREESLIP only
 * south/north, VELOCITY only west, OUTFLOW/PRESSURE only east, PRESSURE with
 * nx < 5, DIRICHLET not on all four sides), LBM_ERR_NOMEM, LBM_ERR_DEVICE. */
lbm_status lbm_create(const lbm_params* p, void* hip_stream, lbm_sim** out);
void lbm_destroy(lbm_sim* s);
const char* lbm_last_error(const lbm_sim* s);

/* Set body body_id (0 <= body_id < LBM_MAX_BODIES) from n markers (n = 0 removes
 * it).  The interface Gamma of Sec. 2.2 is given by:
 *   IB_FIXED: xy[n][2] marker positions (required); uv[n][2] marker velocities
 *     or NULL for the rigid motion U + omega x (X - xc); ds[n] arc-length
 *     weights of Eq. 26 or NULL for half the distance to the two neighbours on a
 *     closed curve.
 *   IB_FREE: xy, uv, ds must be NULL; n markers are placed at angles
 *     theta + 2 pi l / n on the circle of body->radius around body->xc, each
 *     with ds = 2 pi R / n.
 * Bodies whose delta stencils (4 x 4 nodes each) share a node are corrected
 * together; a simulation with a free body corrects all its bodies together.
 * Markers must lie in the lattice: on a non-periodic axis within half a
 * spacing of the first and last nodes (-1/2 <= X <= n - 1/2, where half-way
 * bounce-back puts the wall), for a free circle the whole circle; on a
 * periodic axis within one period (0 <= X < n).
 * Errors: LBM_ERR_INVALID (a marker outside the lattice, marker counts above
 * LBM_MAX_GROUP_MARKERS or LBM_MAX_FREE_MARKERS, a body wider than a periodic
 * period, bad radius or density; the previous bodies stay), LBM_ERR_NOMEM,
 * LBM_ERR_STATE (the simulation is in a batch). */
lbm_status ib_set_markers(lbm_sim* s, int32_t body_id, int32_t n, const double* xy,
                          const double* uv, const double* ds, const ib_body* body);

/* LBM_BC_DIRICHLET simulations: velocities of the boundary nodes for the
 * following steps.  ub holds 2 doubles (u_x, u_y) per perimeter node in the
 * order: south row x = 0..nx-1, north row x = 0..nx-1, west column
 * y = 1..ny-2, east column y = 1..ny-2 (2 nx + 2 (ny - 2) nodes).  Host
 * memory, copied before return, ordered after the work already enqueued for
 * the simulation.  Errors: LBM_ERR_INVALID (null, not a DIRICHLET box),
 * LBM_ERR_STATE (simulation in a batch), LBM_ERR_DEVICE. */
lbm_status lbm_set_boundary_velocity(lbm_sim* s, const double* ub);

/* Replace the marker velocities uv[n][2] of FIXED body `id` (positions and
 * stencils unchanged; for boundaries whose velocity varies in time, such as
 * the Taylor-Green case of Sec. 3.1.1).  Host memory, copied before return.
 * Errors: LBM_ERR_INVALID (no such fixed body, null), LBM_ERR_STATE (in a
 * batch), LBM_ERR_DEVICE. */
lbm_status ib_set_marker_velocities(lbm_sim* s, int32_t id, const double* uv);

/* Enqueue nsteps time steps on the handle's stream (no host synchronisation).
 * One step: collision and streaming (Eqs. 1-3, 7), the boundary rules, N
 * correction sweeps of Sec. 2.3 (interpolation Eq. 22, deviation Eqs. 23-25
 * in the form of Eq. 28, spreading and correction Eqs. 26-27), force and
 * torque (Eqs. 29, 38) and the rigid-body update of free circles (Eqs. 37,
 * 39-42).  Errors: LBM_ERR_INVALID (nsteps < 0), LBM_ERR_STATE (in a batch),
 * LBM_ERR_DEVICE (a launch failed). */
lbm_status lbm_step(lbm_sim* s, int32_t nsteps);
/* Wait for the handle's stream; reports LBM_ERR_UNSTABLE once a density went bad. */
lbm_status lbm_sync(lbm_sim* s);
/* Steps taken so far (alone or in a batch; synchronises a batch it is in). */
int64_t lbm_step_count(lbm_sim* s);

/* Hydrodynamic force F[2] and torque T on body body_id in the last step
 * (Eqs. 29 and 38, the sum over the N sweeps, without the inertial terms of
 * Eqs. 37-38), reduced in FP64.  diag[2] (nullable): RMS of |rho* U - j*| over
 * the body's markers and max |U - u*| after the N sweeps.  state_out
 * (nullable): the body after the step (moved for free circles).  Synchronises. */
lbm_status ib_forces(lbm_sim* s, int32_t body_id, double F[2], double* T, double diag[2],
                     ib_body* state_out);

/* Density and velocity (Eq. 7: rho = sum_i f_i, rho u = sum_i e_i f_i) of
 * the corrected populations after the last step, written to caller-owned host
 * arrays of nx * ny doubles, [ny][nx] with x fastest; NULL skips an output.
 * Synchronises.  Errors: LBM_ERR_NOMEM, LBM_ERR_DEVICE, LBM_ERR_UNSTABLE
 * (the fields are still written). */
lbm_status lbm_fields(lbm_sim* s, double* rho, double* ux, double* uy);
/* lbm_fields for callers that cannot allocate device memory (tight serving
 * loops, harnesses that forbid hipMalloc): the same values, staged through a
 * static device array of 2^20 doubles (8 MiB) that each GPU the library runs
 * on holds until the process ends; no hipMalloc or hipFree.  Rows are staged
 * in chunks, so any lattice whose rows have at most 349,525 nodes is accepted
 * (LBM_ERR_INVALID beyond).  Every call on one GPU uses that GPU's array:
 * calls that overlap on one GPU, from any thread or handle, race.
 * Synchronises; errors as lbm_fields. */
lbm_status lbm_fields_noalloc(lbm_sim* s, double* rho, double* ux, double* uy);
/* Same into FP64 device arrays [ny][nx]; enqueued on the handle's stream. */
lbm_status lbm_fields_device(lbm_sim* s, void* rho, void* ux, void* uy);
/* Post-stream populations f_i (unshifted) as host FP64 [9][ny][nx].  Synchronises. */
lbm_status lbm_get_populations(lbm_sim* s, double* f);
/* Overwrite the state: populations f_i [9][ny][nx] (host FP64), or the
 * equilibrium of the given host fields [ny][nx].  Synchronises. */
lbm_status lbm_set_populations(lbm_sim* s, const double* f);
lbm_status lbm_set_fields(lbm_sim* s, const double* rho, const double* ux, const double* uy);
/* Device memory held by the handle, in bytes. */
size_t lbm_device_bytes(const lbm_sim* s);
/* Upper bound on lbm_device_bytes of a handle that lbm_create would make from
 * *p once its bodies are set, body k with markers[k] markers (k < nbodies;
 * 0 for an unused slot): for callers that admit work by a device-memory
 * budget before creating anything.  Host arithmetic only (no device call, no
 * allocation); for a 400 x 4000 FP32 lattice with two bodies of 126 markers
 * it exceeds the actual figure by well under 1 %.  Returns 0 when p is NULL,
 * nx or ny < 1, nbodies outside 0..LBM_MAX_BODIES, a count is negative, or
 * markers is NULL with nbodies > 0. */
size_t lbm_device_bytes_bound(const lbm_params* p, int32_t nbodies, const int32_t* markers);

/* ---- batching: many simulations of one precision advanced together ----
 * A batch owns no simulation state: admitted handles keep their device memory.
 * Each step is a fixed sequence of kernels over device-resident work tables
 * (cells of every admitted simulation, boundary nodes, body groups),
 * replayed from a HIP graph; admission and retirement rewrite the tables between
 * replays.  Results of a simulation do not depend on what else is in the batch. */

/* hbm_budget_bytes: upper bound on the summed lbm_device_bytes of admitted
 * simulations (0: unlimited).  hip_stream as in lbm_create. */
lbm_status lbm_batch_create(int32_t precision, size_t hbm_budget_bytes, void* hip_stream,
                            lbm_batch** out);
void lbm_batch_destroy(lbm_batch* b);
/* Admit s; it will advance `steps` more steps (<= 0: until retired) and then
 * stop by itself.  LBM_ERR_NOMEM: over budget (nothing changed).
 * LBM_ERR_INVALID: precision mismatch or s already admitted. */
lbm_status lbm_batch_admit(lbm_batch* b, lbm_sim* s, int64_t steps);
/* Remove s from the batch (waits for queued work); s stays valid. */
lbm_status lbm_batch_retire(lbm_batch* b, lbm_sim* s);
/* Enqueue nsteps batch steps (graph replays). */
lbm_status lbm_batch_step(lbm_batch* b, int32_t nsteps);
lbm_status lbm_batch_sync(lbm_batch* b);
/* Steps still to run for s in the batch (reads device state; synchronises). */
lbm_status lbm_batch_remaining(lbm_batch* b, lbm_sim* s, int64_t* remaining);
size_t lbm_batch_bytes(const lbm_batch* b);
/* Time every sweep tiling under each candidate lane schedule on the admitted
 * set (each candidate runs `trials` steps, after which the state is restored,
 * so it is not advanced) and keep the fastest pair.  The lane schedules
 * (lbm_batch_set_lanes) are the one requested, two interleaved halves
 * (lanes = 4) when the lanes are chosen automatically, and one lane (batches of
 * two simulations or more).  Tilings and lanes change scheduling only, never
 * the arithmetic.  chosen (nullable) receives the index of the tiling kept. */
lbm_status lbm_batch_autotune(lbm_batch* b, int32_t trials, int32_t* chosen);
/* Force a tiling index (0 .. lbm_tiling_count()-1). */
lbm_status lbm_batch_set_tiling(lbm_batch* b, int32_t tiling);
/* Index of the tiling the batch launches with now. */
int32_t lbm_batch_get_tiling(const lbm_batch* b);
/* The batch may split its simulations into two lanes replayed on two
 * streams: those whose largest body group has more than 400 markers, and the
 * rest, when both are non-empty and the first holds at most half of the nodes.
 * lanes = 2 replays each lane's captured graphs of several steps on its own
 * stream, independently; lanes = 3 interleaves the lanes step by step, their
 * sweeps in turn (the second lane's sweep of a step waits for the first
 * lane's, the first lane's next sweep for the second lane's), so that each
 * lane's boundary rules and correction run while the other lane sweeps;
 * steps are launched one by one from the host.
 * lanes = 4 interleaves two lanes the same way but splits the simulations
 * into two halves of about equal node count instead (at least two
 * simulations), so that either half's correction can run under the other
 * half's sweep.  In interleaved FP32 lanes the corrections run in 256-thread
 * kernels that fit beside sweep waves (groups of up to 1280 markers), each of
 * which also gathers and applies its group's band.  lanes = 0 (the default)
 * takes 3 for batches of at least 16 Mi nodes and 2 below; lanes = 1 keeps
 * one lane.  The second stream is ordered after
 * the batch stream's earlier work and the batch stream waits for it, so the
 * batch behaves as one stream to the caller.  Results do not depend on the
 * lanes.  lbm_batch_autotune may switch to one lane when it is faster.
 * LBM_ERR_INVALID for other values. */
lbm_status lbm_batch_set_lanes(lbm_batch* b, int32_t lanes);
/* Lanes in use now (1 or 2). */
int32_t lbm_batch_get_lanes(const lbm_batch* b);
/* The lane request in force (0 .. 4, as lbm_batch_set_lanes takes it; the
 * autotuner may have replaced the caller's), -1 for a null batch. */
int32_t lbm_batch_get_lane_mode(const lbm_batch* b);
/* Whether the second lane's stream was seen running kernels beside the batch
 * stream (the two reach the GPU through different hardware queues, which the
 * lanes need to overlap): 1 yes, 0 no (the lanes then run one after the other,
 * with the same results), -1 while no second lane has run (or a null batch).
 * The batch makes up to six candidate streams when the second lane first runs
 * and keeps the first that passes a bounded check (two tiny kernels, at most
 * about 0.2 ms each). */
int32_t lbm_batch_lanes_concurrent(const lbm_batch* b);
int32_t lbm_tiling_count(void);
/* Describe tiling k: threads along x, rows per block, rows per thread. */
lbm_status lbm_tiling_info(int32_t k, int32_t* tx, int32_t* ty, int32_t* rows_per_thread);

/* Run nsteps batch steps with direct launches and HIP events around every
 * kernel on the batch's stream (the state advances as with lbm_batch_step);
 * ms[4] receives the summed milliseconds of the sweep, boundary, correction
 * and bookkeeping kernels; cells (nullable) receives the lattice nodes that
 * one sweep launch updates (nodes of the simulations still stepping). */
lbm_status lbm_batch_profile(lbm_batch* b, int32_t nsteps, double ms[4], int64_t* cells);

/* Library version string. */
const char* lbm_version(void);

#ifdef __cplusplus
}
#endif
#endif
