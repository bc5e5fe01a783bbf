/*
 * lbm_oracle.h -- plain FP64 CPU oracle of the distribution-function-correction
 * immersed-boundary lattice Boltzmann method (Tao, He, Chen, Huang,
 * arXiv:1803.09380).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path.  It
 * shares no code, header, table or helper with the HIP library; only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It is written for readability, not speed: two population buffers,
 * push streaming, straightforward loops, double precision throughout.
 *
 * Conventions (lattice units, dx = dt = 1, c_s^2 = 1/3):
 *   populations f[i][y][x], i = 0..8, x fastest;
 *   D2Q9 order fixed by the rows j_x and j_y of the moment matrix (Eq. 5):
 *   e0=(0,0) e1=(1,0) e2=(0,1) e3=(-1,0) e4=(0,-1)
 *   e5=(1,1) e6=(-1,1) e7=(-1,-1) e8=(1,-1); weights 4/9, 1/9, 1/36 (Eq. 4).
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_PERIODIC = 0, OR_WALL = 1, OR_FREESLIP = 2, OR_VELOCITY = 3, OR_OUTFLOW = 4, OR_PRESSURE = 5,
       OR_DIRICHLET = 6 };
enum { OR_BGK = 0, OR_MRT = 1 };
enum { OR_ROUTE_LITERAL = 0, OR_ROUTE_SIMPLIFIED = 1 };
enum { OR_FIXED = 0, OR_FREE = 1 };
#define OR_MAX_BODIES 8

typedef struct {
    int nx, ny;
    double tau, rho0;
    int bc_west, bc_east, bc_south, bc_north;
    double u_in[2];
    double u_init[2];
    int ib_iters;        /* N of Sec. 2.3 (about 10 in the paper)                */
    int delta;           /* 2, 3 or 4: which kernel of Eq. 15 (a), (b), (c)      */
    int route;           /* OR_ROUTE_LITERAL: Eqs. 22-27; SIMPLIFIED: Eq. 28     */
    int collision;       /* OR_BGK or OR_MRT (Eqs. 2, 5, 6)                      */
    double mrt_s[9];     /* relaxation rates of Eq. 6 (only for OR_MRT)          */
    double gravity[2];   /* gravitational acceleration vector (Eq. 40)           */
} or_params;

typedef struct or_sim or_sim;

/* lifetime; returns NULL on invalid parameters */
or_sim* or_create(const or_params* p);
void or_destroy(or_sim* s);

/* state access: f is [9][ny][nx], fields are [ny][nx] */
void or_set_populations(or_sim* s, const double* f);
void or_get_populations(const or_sim* s, double* f);
void or_set_fields(or_sim* s, const double* rho, const double* ux, const double* uy);
void or_fields(const or_sim* s, double* rho, double* ux, double* uy);
long or_step_count(const or_sim* s);

/* bodies.  FIXED: markers xy[n][2] given, uv[n][2] or NULL (then U + omega x r),
 * ds[n] or NULL (then half the distance to the two neighbours on a closed curve).
 * FREE: rigid circle of radius R and density rho_s; markers are generated on the
 * circle from the state (xc, theta).  Returns 0 on success. */
int or_set_body(or_sim* s, int id, int kind, int n, const double* xy, const double* uv,
                const double* ds, const double xc[2], const double U[2], double omega,
                double theta, double radius, double rho_s);
int or_body_markers(const or_sim* s, int id, double* xy, double* uv, double* ds);

/* OR_DIRICHLET box (all four sides): velocity of every boundary node, ub[k][2]
 * in perimeter order (south row x = 0..nx-1, north row x = 0..nx-1, west column
 * y = 1..ny-2, east column y = 1..ny-2); used by the following steps.  Each
 * boundary node is rebuilt by non-equilibrium extrapolation from its inward
 * neighbour (the diagonal one at corners). */
int or_set_boundary_velocity(or_sim* s, const double* ub);
/* replace the marker velocities of a FIXED body (positions unchanged) */
int or_set_marker_velocities(or_sim* s, int id, const double* uv);

/* advance nsteps: collide, stream, boundary rules, N correction sweeps, rigid update */
void or_step(or_sim* s, int nsteps);
/* only the N correction sweeps (plus force accumulation) on the current field */
void or_ib_only(or_sim* s);

/* last step: hydrodynamic force and torque of Eqs. 29 and 38 (without the
 * inertial terms), diag[0] = RMS momentum mismatch after the sweeps,
 * diag[1] = max slip speed |U - u*| after the sweeps; state[6] =
 * xc, yc, Ux, Uy, omega, theta. */
int or_forces(const or_sim* s, int id, double F[2], double* T, double diag[2], double state[6]);
/* per-sweep RMS momentum mismatch of the last step, for all markers together */
int or_residual_history(const or_sim* s, double* out, int cap);

/* pure functions used by the pin tests */
double or_delta(int kind, double r);
void or_feq(double rho, double ux, double uy, double out[9]);
void or_collide_node(const or_sim* s, const double fin[9], double fout[9]);
void or_mrt_matrix(double M[81], double Minv[81]);
double or_couette_utheta(double r, double R1, double R2, double omega1);
double or_couette_torque_inner(double mu, double omega1, double R1, double R2);
void or_collision_force(const double xi[2], const double xj[2], double Ri, double Rj,
                        double cij, double eps, double xi_gap, double out[2]);
/* one step of the rigid-body integrator of Eqs. 37-42: st[7] = x, y, Ux, Uy,
 * omega, theta, and the previous Ux, Uy, omega in prev[3]; on return both are
 * advanced.  Fs, Ts: hydrodynamic force/torque (Eq. 29 part), Fc: collision
 * force, g: gravity vector, rho_f: fluid density. */
void or_rigid_step(double st[6], double prev[3], const double Fs[2], double Ts,
                   const double Fc[2], const double g[2], double rho_f, double rho_s,
                   double R);

#ifdef __cplusplus
}
#endif
#endif
