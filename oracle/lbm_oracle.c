/*
 * lbm_oracle.c -- plain FP64 CPU oracle of the distribution-function-correction
 * IB-LBM of Tao et al. (arXiv:1803.09380).
 *
 * TEST INFRASTRUCTURE ONLY: it checks the GPU path and is never called by it.
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * load it.  Everything is double precision, two population buffers, pull
 * streaming, loops in the order the paper states the method.
 *
 * One time step (the order is a reading of the paper, which places the
 * correction after streaming like the bounce-back treatment of Fig. 2):
 *   1. collision on every node (BGK, or MRT of Eqs. 2, 5, 6), equilibrium Eq. 3;
 *   2. streaming of Eq. 1 (pull from x - e_i), boundary rules for the
 *      populations whose source lies outside the lattice;
 *   3. N correction sweeps of Sec. 2.3 (Eqs. 22-27, or the Eq. 28 route),
 *      Jacobi over all markers, force and torque of Eqs. 29 and 38;
 *   4. rigid-body update of free circles (Eqs. 37-42, collision force Eq. 39).
 *
 * Parity pins live in tests/: delta identities, equilibrium moments, BGK as
 * MRT with S = I/tau, brute-force streaming, exact mass conservation, the
 * one-marker closed form of the sweep contraction, a dense-matrix rewrite of
 * the sweeps, the cylindrical Couette solution (Eq. 34) with its convergence
 * order, and closed forms of the rigid-body integrator and collision force.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define Q 9
static const int EX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double W[Q] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                            1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

typedef struct {
    int used, kind, n;
    double *X, *Y, *U, *V, *ds, *alpha;
    double xc[2], Uc[2], omega, theta, R, rho_s;
    double Uprev[2], omega_prev;
    double F[2], T, resid, maxslip;
} or_body;

struct or_sim {
    or_params p;
    int px, py; /* periodic axes */
    double* ub; /* OR_DIRICHLET: boundary velocities in perimeter order */
    double *f, *fp, *df;
    unsigned char* touched;
    double Minv[81], M[81];
    or_body b[OR_MAX_BODIES];
    long step;
    double hist[256];
    int nhist;
};

#define IDX(s, i, x, y) ((size_t)(i) * (size_t)(s)->p.nx * (size_t)(s)->p.ny + (size_t)(y) * (size_t)(s)->p.nx + (size_t)(x))

/* ---------------- lattice basics ---------------- */

/* Eq. 3 with c_s^2 = 1/3 */
void or_feq(double rho, double ux, double uy, double out[9]) {
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < Q; ++i) {
        double eu = EX[i] * ux + EY[i] * uy;
        out[i] = W[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    }
}

/* Eq. 7 */
static void moments(const double f[9], double* rho, double* ux, double* uy) {
    double r = 0, jx = 0, jy = 0;
    for (int i = 0; i < Q; ++i) {
        r += f[i];
        jx += EX[i] * f[i];
        jy += EY[i] * f[i];
    }
    *rho = r;
    *ux = jx / r;
    *uy = jy / r;
}

/* Eq. 5 (rows: rho, e, epsilon, j_x, q_x, j_y, q_y, p_xx, p_xy) */
static const double MROWS[81] = {
    1, 1, 1, 1, 1, 1, 1, 1, 1,
    -4, -1, -1, -1, -1, 2, 2, 2, 2,
    4, -2, -2, -2, -2, 1, 1, 1, 1,
    0, 1, 0, -1, 0, 1, -1, -1, 1,
    0, -2, 0, 2, 0, 1, -1, -1, 1,
    0, 0, 1, 0, -1, 1, 1, -1, -1,
    0, 0, -2, 0, 2, 1, 1, -1, -1,
    0, 1, -1, 1, -1, 0, 0, 0, 0,
    0, 0, 0, 0, 0, 1, -1, 1, -1};

/* The rows of M are mutually orthogonal, so M^-1 = M^T diag(1/|row|^2). */
void or_mrt_matrix(double M[81], double Minv[81]) {
    for (int k = 0; k < 81; ++k) M[k] = MROWS[k];
    for (int r = 0; r < 9; ++r) {
        double n2 = 0;
        for (int c = 0; c < 9; ++c) n2 += MROWS[r * 9 + c] * MROWS[r * 9 + c];
        for (int c = 0; c < 9; ++c) Minv[c * 9 + r] = MROWS[r * 9 + c] / n2;
    }
}

/* Collision of one node: BGK f - (f - feq)/tau, or MRT of Eq. 2. */
void or_collide_node(const or_sim* s, const double fin[9], double fout[9]) {
    double rho, ux, uy, feq[9];
    moments(fin, &rho, &ux, &uy);
    or_feq(rho, ux, uy, feq);
    if (s->p.collision == OR_BGK) {
        for (int i = 0; i < Q; ++i) fout[i] = fin[i] - (fin[i] - feq[i]) / s->p.tau;
        return;
    }
    double m[9], meq[9], dm[9];
    for (int r = 0; r < 9; ++r) {
        m[r] = 0;
        meq[r] = 0;
        for (int c = 0; c < 9; ++c) {
            m[r] += s->M[r * 9 + c] * fin[c];
            meq[r] += s->M[r * 9 + c] * feq[c];
        }
        dm[r] = s->p.mrt_s[r] * (m[r] - meq[r]);
    }
    for (int i = 0; i < Q; ++i) {
        double acc = 0;
        for (int r = 0; r < 9; ++r) acc += s->Minv[i * 9 + r] * dm[r];
        fout[i] = fin[i] - acc;
    }
}

/* ---------------- discrete delta functions, Eq. 15 ---------------- */

double or_delta(int kind, double r) {
    double a = fabs(r);
    if (kind == 2) return a <= 1.0 ? 1.0 - a : 0.0;
    if (kind == 3) {
        if (a < 0.5) return (1.0 + sqrt(1.0 - 3.0 * a * a)) / 3.0;
        if (a < 1.5) return (5.0 - 3.0 * a - sqrt(1.0 - 3.0 * (1.0 - a) * (1.0 - a))) / 6.0;
        return 0.0;
    }
    return a <= 2.0 ? 0.25 * (1.0 + cos(M_PI * a / 2.0)) : 0.0;
}

/* ---------------- analytic references ---------------- */

/* Eq. 34 with omega_2 = 0: u_theta = omega1 (R1^2 - R^2 r^2) / ((1 - R^2) r), R = R1/R2 */
double or_couette_utheta(double r, double R1, double R2, double omega1) {
    double Rr = R1 / R2;
    return (R1 * R1 - Rr * Rr * r * r) * omega1 / ((1.0 - Rr * Rr) * r);
}

/* Torque per unit depth exerted by the fluid on the inner cylinder of the
 * Couette flow of Eq. 34: T = 2 pi R1^2 tau_{r theta}(R1), with
 * tau_{r theta} = mu r d(u/r)/dr = -2 mu omega1 R1^2 R2^2 / ((R2^2 - R1^2) r^2). */
double or_couette_torque_inner(double mu, double omega1, double R1, double R2) {
    return -4.0 * M_PI * mu * omega1 * R1 * R1 * R2 * R2 / (R2 * R2 - R1 * R1);
}

/* ---------------- rigid body, Eqs. 37-42 and 39 ---------------- */

/* Eq. 39, reading the numerator symbol as the threshold gap xi. */
void or_collision_force(const double xi[2], const double xj[2], double Ri, double Rj, double cij,
                        double eps, double xi_gap, double out[2]) {
    double dx = xi[0] - xj[0], dy = xi[1] - xj[1];
    double d = sqrt(dx * dx + dy * dy);
    out[0] = out[1] = 0.0;
    if (d > Ri + Rj + xi_gap || d <= 0.0) return;
    double g = (d - Ri - Rj - xi_gap) / xi_gap;
    double mag = cij / eps * g * g;
    out[0] = mag * dx / d;
    out[1] = mag * dy / d;
}

void or_rigid_step(double st[6], double prev[3], const double Fs[2], double Ts, const double Fc[2],
                   const double g[2], double rho_f, double rho_s, double R) {
    double V = M_PI * R * R, Ms = rho_s * V, Is = 0.5 * Ms * R * R;
    double Ft[2], Tt;
    for (int k = 0; k < 2; ++k)
        Ft[k] = Fs[k] + rho_f * V * (st[2 + k] - prev[k]) + Fc[k] + (Ms - rho_f * V) * g[k];
    Tt = Ts + (rho_f / rho_s) * Is * (st[4] - prev[2]);
    /* Eq. 42 uses the velocities at level n, Eq. 41 then advances them */
    st[0] += st[2] + 0.5 * Ft[0] / Ms;
    st[1] += st[3] + 0.5 * Ft[1] / Ms;
    st[5] += st[4] + 0.5 * Tt / Is;
    prev[0] = st[2];
    prev[1] = st[3];
    prev[2] = st[4];
    st[2] += Ft[0] / Ms;
    st[3] += Ft[1] / Ms;
    st[4] += Tt / Is;
}

/* ---------------- lifetime and state ---------------- */

static int bc_ok(const or_params* p) {
    if (p->nx < 4 || p->ny < 4) return 0;
    {
        int nd = (p->bc_west == OR_DIRICHLET) + (p->bc_east == OR_DIRICHLET) + (p->bc_south == OR_DIRICHLET) +
                 (p->bc_north == OR_DIRICHLET);
        if (nd == 4) return 1;
        if (nd != 0) return 0;
    }
    if ((p->bc_west == OR_PERIODIC) != (p->bc_east == OR_PERIODIC)) return 0;
    if ((p->bc_south == OR_PERIODIC) != (p->bc_north == OR_PERIODIC)) return 0;
    if (p->bc_west != OR_PERIODIC && p->bc_west != OR_WALL && p->bc_west != OR_VELOCITY) return 0;
    if (p->bc_east != OR_PERIODIC && p->bc_east != OR_WALL && p->bc_east != OR_OUTFLOW &&
        p->bc_east != OR_PRESSURE)
        return 0;
    if (p->bc_east == OR_PRESSURE && p->nx < 5) return 0;
    if (p->bc_south != OR_PERIODIC && p->bc_south != OR_WALL && p->bc_south != OR_FREESLIP) return 0;
    if (p->bc_north != OR_PERIODIC && p->bc_north != OR_WALL && p->bc_north != OR_FREESLIP) return 0;
    return 1;
}

or_sim* or_create(const or_params* p) {
    if (!p || p->tau <= 0.5 || !bc_ok(p) || p->ib_iters < 0 ||
        (p->delta != 2 && p->delta != 3 && p->delta != 4))
        return NULL;
    or_sim* s = (or_sim*)calloc(1, sizeof(or_sim));
    s->p = *p;
    s->px = p->bc_west == OR_PERIODIC;
    s->py = p->bc_south == OR_PERIODIC;
    size_t n = (size_t)Q * p->nx * p->ny;
    s->f = (double*)malloc(n * sizeof(double));
    s->fp = (double*)malloc(n * sizeof(double));
    s->df = (double*)calloc(n, sizeof(double));
    s->touched = (unsigned char*)calloc((size_t)p->nx * p->ny, 1);
    or_mrt_matrix(s->M, s->Minv);
    if (p->bc_west == OR_DIRICHLET) s->ub = (double*)calloc((size_t)4 * (p->nx + p->ny), sizeof(double));
    double feq[9];
    or_feq(p->rho0, p->u_init[0], p->u_init[1], feq);
    for (int i = 0; i < Q; ++i)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) s->f[IDX(s, i, x, y)] = feq[i];
    return s;
}

static void free_body(or_body* b) {
    free(b->X);
    free(b->Y);
    free(b->U);
    free(b->V);
    free(b->ds);
    free(b->alpha);
    memset(b, 0, sizeof(*b));
}

void or_destroy(or_sim* s) {
    if (!s) return;
    for (int k = 0; k < OR_MAX_BODIES; ++k) free_body(&s->b[k]);
    free(s->f);
    free(s->fp);
    free(s->df);
    free(s->touched);
    free(s->ub);
    free(s);
}

static int perimeter_count(const or_sim* s) { return 2 * s->p.nx + 2 * (s->p.ny - 2); }

int or_set_boundary_velocity(or_sim* s, const double* ub) {
    if (!s || !s->ub || !ub) return -1;
    memcpy(s->ub, ub, sizeof(double) * 2 * perimeter_count(s));
    return 0;
}

int or_set_marker_velocities(or_sim* s, int id, const double* uv) {
    if (!s || id < 0 || id >= OR_MAX_BODIES || !s->b[id].used || s->b[id].kind != OR_FIXED || !uv) return -1;
    for (int l = 0; l < s->b[id].n; ++l) {
        s->b[id].U[l] = uv[2 * l];
        s->b[id].V[l] = uv[2 * l + 1];
    }
    return 0;
}

void or_set_populations(or_sim* s, const double* f) {
    memcpy(s->f, f, sizeof(double) * Q * s->p.nx * s->p.ny);
}
void or_get_populations(const or_sim* s, double* f) {
    memcpy(f, s->f, sizeof(double) * Q * s->p.nx * s->p.ny);
}
long or_step_count(const or_sim* s) { return s->step; }

void or_set_fields(or_sim* s, const double* rho, const double* ux, const double* uy) {
    double feq[9];
    for (int y = 0; y < s->p.ny; ++y)
        for (int x = 0; x < s->p.nx; ++x) {
            size_t c = (size_t)y * s->p.nx + x;
            or_feq(rho[c], ux[c], uy[c], feq);
            for (int i = 0; i < Q; ++i) s->f[IDX(s, i, x, y)] = feq[i];
        }
}

static void node_f(const or_sim* s, int x, int y, double f[9]) {
    for (int i = 0; i < Q; ++i) f[i] = s->f[IDX(s, i, x, y)];
}

void or_fields(const or_sim* s, double* rho, double* ux, double* uy) {
    double f[9], r, u, v;
    for (int y = 0; y < s->p.ny; ++y)
        for (int x = 0; x < s->p.nx; ++x) {
            node_f(s, x, y, f);
            moments(f, &r, &u, &v);
            size_t c = (size_t)y * s->p.nx + x;
            if (rho) rho[c] = r;
            if (ux) ux[c] = u;
            if (uy) uy[c] = v;
        }
}

/* ---------------- bodies ---------------- */

static void circle_markers(or_body* b) {
    for (int l = 0; l < b->n; ++l) {
        double a = b->alpha[l] + b->theta;
        b->X[l] = b->xc[0] + b->R * cos(a);
        b->Y[l] = b->xc[1] + b->R * sin(a);
        b->U[l] = b->Uc[0] - b->omega * (b->Y[l] - b->xc[1]);
        b->V[l] = b->Uc[1] + b->omega * (b->X[l] - b->xc[0]);
        b->ds[l] = 2.0 * M_PI * b->R / b->n;
    }
}

int or_set_body(or_sim* s, int id, int kind, int n, const double* xy, const double* uv,
                const double* ds, const double xc[2], const double U[2], double omega,
                double theta, double radius, double rho_s) {
    if (id < 0 || id >= OR_MAX_BODIES) return 1;
    or_body* b = &s->b[id];
    free_body(b);
    if (n <= 0) return 0;
    if (kind == OR_FREE && (radius <= 0 || rho_s <= 0 || xy)) return 1;
    if (kind == OR_FIXED && !xy) return 1;
    b->used = 1;
    b->kind = kind;
    b->n = n;
    b->X = (double*)malloc(n * sizeof(double));
    b->Y = (double*)malloc(n * sizeof(double));
    b->U = (double*)malloc(n * sizeof(double));
    b->V = (double*)malloc(n * sizeof(double));
    b->ds = (double*)malloc(n * sizeof(double));
    b->alpha = (double*)malloc(n * sizeof(double));
    b->xc[0] = xc ? xc[0] : 0.0;
    b->xc[1] = xc ? xc[1] : 0.0;
    b->Uc[0] = U ? U[0] : 0.0;
    b->Uc[1] = U ? U[1] : 0.0;
    b->omega = omega;
    b->theta = theta;
    b->R = radius;
    b->rho_s = rho_s;
    b->Uprev[0] = b->Uc[0];
    b->Uprev[1] = b->Uc[1];
    b->omega_prev = omega;
    if (kind == OR_FREE) {
        for (int l = 0; l < n; ++l) b->alpha[l] = 2.0 * M_PI * l / n;
        circle_markers(b);
        return 0;
    }
    for (int l = 0; l < n; ++l) {
        b->X[l] = xy[2 * l];
        b->Y[l] = xy[2 * l + 1];
        b->alpha[l] = 0.0;
    }
    for (int l = 0; l < n; ++l) {
        if (uv) {
            b->U[l] = uv[2 * l];
            b->V[l] = uv[2 * l + 1];
        } else {
            b->U[l] = b->Uc[0] - omega * (b->Y[l] - b->xc[1]);
            b->V[l] = b->Uc[1] + omega * (b->X[l] - b->xc[0]);
        }
        if (ds) {
            b->ds[l] = ds[l];
        } else {
            int a = (l + n - 1) % n, c = (l + 1) % n;
            double d1 = hypot(b->X[l] - b->X[a], b->Y[l] - b->Y[a]);
            double d2 = hypot(b->X[c] - b->X[l], b->Y[c] - b->Y[l]);
            b->ds[l] = 0.5 * (d1 + d2);
        }
    }
    return 0;
}

int or_body_markers(const or_sim* s, int id, double* xy, double* uv, double* ds) {
    if (id < 0 || id >= OR_MAX_BODIES || !s->b[id].used) return 0;
    const or_body* b = &s->b[id];
    for (int l = 0; l < b->n; ++l) {
        if (xy) {
            xy[2 * l] = b->X[l];
            xy[2 * l + 1] = b->Y[l];
        }
        if (uv) {
            uv[2 * l] = b->U[l];
            uv[2 * l + 1] = b->V[l];
        }
        if (ds) ds[l] = b->ds[l];
    }
    return b->n;
}

/* ---------------- collision + streaming + boundary rules ---------------- */

static void collide_all(or_sim* s) {
    const int nx = s->p.nx, ny = s->p.ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double fin[9], fout[9];
            node_f(s, x, y, fin);
            or_collide_node(s, fin, fout);
            for (int i = 0; i < Q; ++i) s->fp[IDX(s, i, x, y)] = fout[i];
        }
}

/* Post-collision value of population i at (x, y); (x, y) must be inside. */
static double fpost(const or_sim* s, int i, int x, int y) { return s->fp[IDX(s, i, x, y)]; }

static void stream_all(or_sim* s) {
    const int nx = s->p.nx, ny = s->p.ny;
    const int bw = s->p.bc_west, be = s->p.bc_east, bs = s->p.bc_south, bn = s->p.bc_north;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            for (int i = 0; i < Q; ++i) {
                int sx = x - EX[i], sy = y - EY[i];
                if (s->px) sx = (sx + nx) % nx;
                if (s->py) sy = (sy + ny) % ny;
                int outx = sx < 0 || sx >= nx, outy = sy < 0 || sy >= ny;
                double v;
                if (!outx && !outy) {
                    v = fpost(s, i, sx, sy); /* Eq. 1: f_i(x + e_i, t + 1) = f_i*(x, t) */
                } else if (outx) {
                    /* a west/east rule owns every population entering through that side */
                    int side = sx < 0 ? bw : be;
                    if (side == OR_WALL)
                        v = fpost(s, OPP[i], x, y); /* half-way bounce-back (Fig. 2) */
                    else
                        v = NAN; /* inlet / outlet: filled below */
                } else {
                    int side = sy < 0 ? bs : bn;
                    if (side == OR_DIRICHLET) {
                        v = NAN; /* rebuilt below */
                    } else if (side == OR_WALL) {
                        v = fpost(s, OPP[i], x, y);
                    } else { /* free slip: specular reflection of the mirrored population */
                        int mirror = -1;
                        for (int k = 0; k < Q; ++k)
                            if (EX[k] == EX[i] && EY[k] == -EY[i]) mirror = k;
                        int mx = x - EX[i];
                        if (s->px) mx = (mx + nx) % nx;
                        v = fpost(s, mirror, mx, y);
                    }
                }
                s->f[IDX(s, i, x, y)] = v;
            }
    /* zero-gradient outlet: the populations entering from the east copy column nx-2 */
    if (be == OR_OUTFLOW)
        for (int y = 0; y < ny; ++y)
            for (int i = 0; i < Q; ++i)
                if (EX[i] == -1) s->f[IDX(s, i, nx - 1, y)] = s->f[IDX(s, i, nx - 2, y)];
    /* prescribed velocities on a box (Sec. 3.1.1, non-equilibrium
     * extrapolation): every population of a boundary node is
     * f^eq(rho(n), u_b) + f(n) - f^eq(rho(n), u(n)) with n the inward neighbour */
    if (bw == OR_DIRICHLET) {
        int k = 0;
        for (int pass = 0; pass < 4; ++pass) {
            int cnt = pass < 2 ? nx : ny - 2;
            for (int t = 0; t < cnt; ++t, ++k) {
                int x = pass == 0 || pass == 1 ? t : (pass == 2 ? 0 : nx - 1);
                int y = pass == 0 ? 0 : (pass == 1 ? ny - 1 : t + 1);
                int xn = x < 1 ? 1 : (x > nx - 2 ? nx - 2 : x);
                int yn = y < 1 ? 1 : (y > ny - 2 ? ny - 2 : y);
                double fn[9], rn, un, vn, eqb[9], eqn[9];
                node_f(s, xn, yn, fn);
                moments(fn, &rn, &un, &vn);
                or_feq(rn, s->ub[2 * k], s->ub[2 * k + 1], eqb);
                or_feq(rn, un, vn, eqn);
                for (int i = 0; i < Q; ++i) s->f[IDX(s, i, x, y)] = eqb[i] + (fn[i] - eqn[i]);
            }
        }
    }
    /* pressure outlet by non-equilibrium extrapolation (Sec. 3.2): every
     * population of column nx-1 is f^eq(rho0, u(nx-2)) + f^neq(nx-2) */
    if (be == OR_PRESSURE)
        for (int y = 0; y < ny; ++y) {
            double f2[9], rho2, u2, v2, eqb[9], eq2[9];
            node_f(s, nx - 2, y, f2);
            moments(f2, &rho2, &u2, &v2);
            or_feq(s->p.rho0, u2, v2, eqb);
            or_feq(rho2, u2, v2, eq2);
            for (int i = 0; i < Q; ++i) s->f[IDX(s, i, nx - 1, y)] = eqb[i] + (f2[i] - eq2[i]);
        }
    /* velocity inlet by non-equilibrium extrapolation: every population of
     * column 0 is f^eq(rho(1), U_in) + f^neq(1) */
    if (bw == OR_VELOCITY)
        for (int y = 0; y < ny; ++y) {
            double f1[9], rho1, u1, v1, eqb[9], eq1[9];
            node_f(s, 1, y, f1);
            moments(f1, &rho1, &u1, &v1);
            or_feq(rho1, s->p.u_in[0], s->p.u_in[1], eqb);
            or_feq(rho1, u1, v1, eq1);
            for (int i = 0; i < Q; ++i) s->f[IDX(s, i, 0, y)] = eqb[i] + (f1[i] - eq1[i]);
        }
}

/* ---------------- the correction sweeps, Sec. 2.3 ---------------- */

typedef struct {
    int c[25]; /* cell index y * nx + x */
    double d[25];
    int n;
} stencil;

/* Nodes with non-zero D = phi(x - X) phi(y - Y) (Eq. 15, dx = 1); nodes past a
 * periodic edge wrap, nodes past any other edge are dropped. */
static void make_stencil(const or_sim* s, double X, double Y, stencil* st) {
    int fx = (int)floor(X), fy = (int)floor(Y);
    st->n = 0;
    for (int yy = fy - 2; yy <= fy + 2; ++yy) {
        double py = or_delta(s->p.delta, yy - Y);
        if (py == 0.0) continue;
        int wy = yy;
        if (s->py) wy = ((yy % s->p.ny) + s->p.ny) % s->p.ny;
        if (wy < 0 || wy >= s->p.ny) continue;
        for (int xx = fx - 2; xx <= fx + 2; ++xx) {
            double px = or_delta(s->p.delta, xx - X);
            if (px == 0.0) continue;
            int wx = xx;
            if (s->px) wx = ((xx % s->p.nx) + s->p.nx) % s->p.nx;
            if (wx < 0 || wx >= s->p.nx) continue;
            st->c[st->n] = wy * s->p.nx + wx;
            st->d[st->n] = px * py;
            st->n++;
        }
    }
}

typedef struct {
    int body, l;
} mref;

/* Node quantities of the current iterate: f_i, f^eq_i(rho(x), u(x)) and rho(x). */
typedef struct {
    double f[9], feq[9], rho;
} nodeval;

static void node_values(const or_sim* s, const int* band, int nband, nodeval* nv) {
    for (int k = 0; k < nband; ++k) {
        int x = band[k] % s->p.nx, y = band[k] / s->p.nx;
        double ux, uy;
        node_f(s, x, y, nv[k].f);
        moments(nv[k].f, &nv[k].rho, &ux, &uy);
        or_feq(nv[k].rho, ux, uy, nv[k].feq);
    }
}

/* For every marker (all bodies, ascending body then marker index): the
 * deviation delta f_i of Eq. 25 (literal route: Eqs. 22-25; simplified
 * route: Eq. 28), computed from the current field (Jacobi sweep).  Returns
 * the momentum mismatch sum_i e_i delta f_i in dm[2*k] and the interpolated
 * density in rstar[k]. */
static void deviations(const or_sim* s, const mref* refs, int nm, const stencil* sts,
                       const int* slot, const nodeval* nv, double* dev, double* dm, double* rstar) {
    for (int k = 0; k < nm; ++k) {
        const or_body* b = &s->b[refs[k].body];
        int l = refs[k].l;
        const stencil* st = &sts[k];
        double fs[9] = {0}, fneqs[9] = {0}, feqs[9] = {0}, rs = 0.0;
        for (int m = 0; m < st->n; ++m) {
            const nodeval* v = &nv[slot[st->c[m]]];
            double D = st->d[m];
            rs += D * v->rho;
            for (int i = 0; i < Q; ++i) {
                fs[i] += D * v->f[i];                  /* Eq. 22a */
                fneqs[i] += D * (v->f[i] - v->feq[i]); /* Eq. 22b */
                feqs[i] += D * v->feq[i];
            }
        }
        double eqb[9];
        or_feq(rs, b->U[l], b->V[l], eqb); /* f^eq(rho, U) at the boundary, rho = interpolated rho */
        double mx = 0, my = 0;
        for (int i = 0; i < Q; ++i) {
            double d;
            if (s->p.route == OR_ROUTE_LITERAL) {
                double desired = fneqs[i] + eqb[i]; /* Eqs. 23-24 */
                d = desired - fs[i];                /* Eq. 25 */
            } else {
                d = eqb[i] - feqs[i]; /* Eq. 28 */
            }
            dev[9 * k + i] = d;
            mx += EX[i] * d;
            my += EY[i] * d;
        }
        dm[2 * k] = mx;
        dm[2 * k + 1] = my;
        rstar[k] = rs;
    }
}

static int collect_markers(const or_sim* s, mref** out) {
    int nm = 0;
    for (int k = 0; k < OR_MAX_BODIES; ++k)
        if (s->b[k].used) nm += s->b[k].n;
    mref* r = (mref*)malloc(sizeof(mref) * (nm > 0 ? nm : 1));
    int c = 0;
    for (int k = 0; k < OR_MAX_BODIES; ++k)
        if (s->b[k].used)
            for (int l = 0; l < s->b[k].n; ++l) {
                r[c].body = k;
                r[c].l = l;
                ++c;
            }
    *out = r;
    return nm;
}

static void ib_sweeps(or_sim* s) {
    mref* refs;
    int nm = collect_markers(s, &refs);
    for (int k = 0; k < OR_MAX_BODIES; ++k) {
        s->b[k].F[0] = s->b[k].F[1] = s->b[k].T = 0.0;
        s->b[k].resid = s->b[k].maxslip = 0.0;
    }
    s->nhist = 0;
    if (nm == 0) {
        free(refs);
        return;
    }
    /* markers do not move during the sweeps: their stencils are fixed */
    stencil* sts = (stencil*)malloc(sizeof(stencil) * nm);
    int* band = (int*)malloc(sizeof(int) * 25 * nm);
    int nband = 0;
    for (int k = 0; k < nm; ++k) {
        const or_body* b = &s->b[refs[k].body];
        make_stencil(s, b->X[refs[k].l], b->Y[refs[k].l], &sts[k]);
        for (int m = 0; m < sts[k].n; ++m) {
            int c = sts[k].c[m];
            if (!s->touched[c]) {
                s->touched[c] = 1;
                band[nband++] = c;
            }
        }
    }
    int* slot = (int*)malloc(sizeof(int) * (size_t)s->p.nx * s->p.ny);
    for (int k = 0; k < nband; ++k) slot[band[k]] = k;
    nodeval* nv = (nodeval*)malloc(sizeof(nodeval) * nband);
    double* dev = (double*)malloc(sizeof(double) * 9 * nm);
    double* dm = (double*)malloc(sizeof(double) * 2 * nm);
    double* rs = (double*)malloc(sizeof(double) * nm);
    for (int n = 0; n < s->p.ib_iters; ++n) {
        node_values(s, band, nband, nv);
        deviations(s, refs, nm, sts, slot, nv, dev, dm, rs);
        double r2 = 0.0;
        for (int k = 0; k < nm; ++k) {
            or_body* b = &s->b[refs[k].body];
            int l = refs[k].l;
            /* Eq. 29: the body receives minus the momentum put into the fluid */
            double Fx = -b->ds[l] * dm[2 * k], Fy = -b->ds[l] * dm[2 * k + 1];
            b->F[0] += Fx;
            b->F[1] += Fy;
            /* Eq. 38 read as r x F with r = X - x_c */
            b->T += (b->X[l] - b->xc[0]) * Fy - (b->Y[l] - b->xc[1]) * Fx;
            r2 += dm[2 * k] * dm[2 * k] + dm[2 * k + 1] * dm[2 * k + 1];
        }
        if (s->nhist < 256) s->hist[s->nhist++] = sqrt(r2 / nm);
        /* Eq. 26: spread with the same delta function, ascending marker order */
        for (int k = 0; k < nm; ++k) {
            const or_body* b = &s->b[refs[k].body];
            int l = refs[k].l;
            for (int m = 0; m < sts[k].n; ++m) {
                double w = sts[k].d[m] * b->ds[l];
                size_t c = (size_t)sts[k].c[m], np = (size_t)s->p.nx * s->p.ny;
                for (int i = 0; i < Q; ++i) s->df[i * np + c] += w * dev[9 * k + i];
            }
        }
        /* Eq. 27: correct once, then clear the accumulator */
        for (int k = 0; k < nband; ++k) {
            size_t c = (size_t)band[k], np = (size_t)s->p.nx * s->p.ny;
            for (int i = 0; i < Q; ++i) {
                s->f[i * np + c] += s->df[i * np + c];
                s->df[i * np + c] = 0.0;
            }
        }
    }
    /* mismatch left after the last sweep (diagnostics only) */
    node_values(s, band, nband, nv);
    deviations(s, refs, nm, sts, slot, nv, dev, dm, rs);
    for (int k = 0; k < nm; ++k) {
        or_body* b = &s->b[refs[k].body];
        b->resid += dm[2 * k] * dm[2 * k] + dm[2 * k + 1] * dm[2 * k + 1];
        /* the slip U - j_star/rho_star equals dm/rho_star */
        double slip = sqrt(dm[2 * k] * dm[2 * k] + dm[2 * k + 1] * dm[2 * k + 1]) / rs[k];
        if (slip > b->maxslip) b->maxslip = slip;
    }
    for (int k = 0; k < OR_MAX_BODIES; ++k)
        if (s->b[k].used) s->b[k].resid = sqrt(s->b[k].resid / s->b[k].n);
    for (int k = 0; k < nband; ++k) s->touched[band[k]] = 0;
    free(nv);
    free(slot);
    free(band);
    free(sts);
    free(dev);
    free(dm);
    free(rs);
    free(refs);
}

void or_ib_only(or_sim* s) { ib_sweeps(s); }

/* ---------------- rigid update of free circles ---------------- */

static void rigid_all(or_sim* s) {
    double gmag = hypot(s->p.gravity[0], s->p.gravity[1]);
    double rho_f = s->p.rho0;
    double Fc[OR_MAX_BODIES][2];
    for (int k = 0; k < OR_MAX_BODIES; ++k) {
        Fc[k][0] = Fc[k][1] = 0.0;
        or_body* b = &s->b[k];
        if (!b->used || b->kind != OR_FREE) continue;
        double V = M_PI * b->R * b->R;
        double cij = (b->rho_s * V - rho_f * V) * gmag; /* buoyancy-reduced weight */
        double gap = 0.1 * b->R;                         /* xi = 0.05 D */
        for (int j = 0; j < OR_MAX_BODIES; ++j) {
            const or_body* o = &s->b[j];
            if (j == k || !o->used || o->kind != OR_FREE) continue;
            double f[2];
            or_collision_force(b->xc, o->xc, b->R, o->R, cij, 0.01, gap, f);
            Fc[k][0] += f[0];
            Fc[k][1] += f[1];
        }
        /* walls: a mirror particle of the same radius behind each solid side */
        double mir[4][2] = {{-1.0 - b->xc[0], b->xc[1]},
                            {2.0 * s->p.nx - 1.0 - b->xc[0], b->xc[1]},
                            {b->xc[0], -1.0 - b->xc[1]},
                            {b->xc[0], 2.0 * s->p.ny - 1.0 - b->xc[1]}};
        int sides[4] = {s->p.bc_west, s->p.bc_east, s->p.bc_south, s->p.bc_north};
        for (int w = 0; w < 4; ++w) {
            if (sides[w] != OR_WALL && sides[w] != OR_FREESLIP) continue;
            double f[2];
            or_collision_force(b->xc, mir[w], b->R, b->R, cij, 0.01, gap, f);
            Fc[k][0] += f[0];
            Fc[k][1] += f[1];
        }
    }
    for (int k = 0; k < OR_MAX_BODIES; ++k) {
        or_body* b = &s->b[k];
        if (!b->used || b->kind != OR_FREE) continue;
        double st[6] = {b->xc[0], b->xc[1], b->Uc[0], b->Uc[1], b->omega, b->theta};
        double prev[3] = {b->Uprev[0], b->Uprev[1], b->omega_prev};
        or_rigid_step(st, prev, b->F, b->T, Fc[k], s->p.gravity, rho_f, b->rho_s, b->R);
        b->xc[0] = st[0];
        b->xc[1] = st[1];
        b->Uc[0] = st[2];
        b->Uc[1] = st[3];
        b->omega = st[4];
        b->theta = st[5];
        b->Uprev[0] = prev[0];
        b->Uprev[1] = prev[1];
        b->omega_prev = prev[2];
        circle_markers(b);
    }
}

void or_step(or_sim* s, int nsteps) {
    for (int t = 0; t < nsteps; ++t) {
        collide_all(s);
        stream_all(s);
        ib_sweeps(s);
        rigid_all(s);
        s->step++;
    }
}

int or_forces(const or_sim* s, int id, double F[2], double* T, double diag[2], double state[6]) {
    if (id < 0 || id >= OR_MAX_BODIES || !s->b[id].used) return 1;
    const or_body* b = &s->b[id];
    if (F) {
        F[0] = b->F[0];
        F[1] = b->F[1];
    }
    if (T) *T = b->T;
    if (diag) {
        diag[0] = b->resid;
        diag[1] = b->maxslip;
    }
    if (state) {
        state[0] = b->xc[0];
        state[1] = b->xc[1];
        state[2] = b->Uc[0];
        state[3] = b->Uc[1];
        state[4] = b->omega;
        state[5] = b->theta;
    }
    return 0;
}

int or_residual_history(const or_sim* s, double* out, int cap) {
    int n = s->nhist < cap ? s->nhist : cap;
    for (int k = 0; k < n; ++k) out[k] = s->hist[k];
    return n;
}
