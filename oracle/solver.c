/*
 * solver.c -- whole-grid operators of the oracle: global Lax-Friedrichs
 * splitting, the conservative finite-difference operator, dimension-by-
 * dimension 2D, the third-order TVD Runge-Kutta step and the time loop.
 * TEST INFRASTRUCTURE ONLY (see enoao_ref.h).
 *
 * Paper references (Section 2 unless noted):
 *  - Eq. (1DWENOFD): du_j/dt = -(fhat_{j+1/2} - fhat_{j-1/2})/dx, fhat
 *    approximating the function h whose cell averages are the point values f;
 *  - Eq. (Flux_Split), (LF_Flux_Split): f^(+/-) = (f +/- alpha u)/2 with alpha
 *    the maximum of |f'(u)| over all mesh points;
 *  - Section 3.2: fhat^-_{j+1/2} is the mirror image of fhat^+ about x_{j+1/2};
 *  - dimension-by-dimension extension of the same 1D procedure;
 *  - third-order TVD Runge-Kutta time stepping (Shu-Osher form, coefficients
 *    not printed in the paper: u1 = u + dt L(u); u2 = 3/4 u + 1/4 (u1 + dt L(u1));
 *    u^{n+1} = 1/3 u + 2/3 (u2 + dt L(u2)));
 *  - Section 4: Roe-average characteristic decomposition for the Euler
 *    equations, CFL-limited time step.
 *
 * Readings where the paper is silent:
 *  - alpha is recomputed for every evaluation of L, over the grid nodes; for a
 *    system it is taken per characteristic field: alpha_s = max_j |lambda_s(U_j)|;
 *  - a system is split and reconstructed in characteristic variables: every
 *    stencil node is projected with the left eigenvectors of the face's Roe
 *    state, w^(+/-)_s = (L_s F + / - alpha_s L_s U)/2, reconstructed field by
 *    field, and mapped back with the right eigenvectors;
 *  - dt = cfl*dx/|a| (advection), cfl*dx/max(|u|+c) (1D Euler),
 *    cfl/max((|u|+c)/dx + (|v|+c)/dy) (2D Euler); the step that would reach
 *    t_final (dt >= (t_final - t)(1 - 1e-10)) is set to t_final - t and ends
 *    the loop at t = t_final exactly;
 *  - boundary conditions act on the stencil gather: periodic wrap, or
 *    zero-gradient ("non-reflective") copying of the end node;
 *  - the component-wise alternative (recon_vars = REF_COMPONENT) splits and
 *    reconstructs each conserved component of U and F directly, with the one
 *    alpha of the scalar splitting taken as the largest eigenvalue magnitude,
 *    max_j (|u| + c) along the sweep, for every component.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "enoao_ref.h"

static int ncomp_of(int eq)
{
    return eq == REF_ADVECTION ? 1 : eq == REF_EULER1D ? 3 : eq == REF_EULER2D ? 4 : 0;
}

static int check_problem(const ref_problem *p)
{
    if (!p) return REF_EINVAL;
    if (!ncomp_of(p->equation)) return REF_EINVAL;
    if (p->order != 5 && p->order != 7) return REF_EINVAL;
    if (p->nx < 1 || p->ny < 1) return REF_EINVAL;
    if (p->equation != REF_EULER2D && p->ny != 1) return REF_EINVAL;
    if (!(p->x_hi > p->x_lo)) return REF_EINVAL;
    if (p->equation == REF_EULER2D && !(p->y_hi > p->y_lo)) return REF_EINVAL;
    if (p->bc_x != REF_BC_PERIODIC && p->bc_x != REF_BC_TRANSMISSIVE) return REF_EINVAL;
    if (p->equation == REF_EULER2D && p->bc_y != REF_BC_PERIODIC && p->bc_y != REF_BC_TRANSMISSIVE)
        return REF_EINVAL;
    if (p->equation != REF_ADVECTION && !(p->gamma > 1.0)) return REF_EINVAL;
    if (p->recon_vars != REF_CHAR_ROE && p->recon_vars != REF_COMPONENT) return REF_EINVAL;
    if (p->equation == REF_ADVECTION && !(p->adv_speed != 0.0)) return REF_EINVAL;
    if (!(p->delta >= 0.0)) return REF_EINVAL;
    return REF_OK;
}

static double dx_of(const ref_problem *p) { return (p->x_hi - p->x_lo) / (double)p->nx; }
static double dy_of(const ref_problem *p) { return (p->y_hi - p->y_lo) / (double)p->ny; }

/* node index of a stencil position k in [-G, n+G) under the boundary condition */
static int bc_index(int k, int n, int bc)
{
    if (bc == REF_BC_PERIODIC) return ((k % n) + n) % n;
    return k < 0 ? 0 : (k >= n ? n - 1 : k);
}

/* Node values needed for alpha and dt: velocity along the sweep, sound speed. */
static int node_speed(int eq, double gamma, const double *U, double *un, double *ut, double *c)
{
    const double rho = U[0];
    if (!(rho > 0.0)) return REF_ENONPHYSICAL;
    double p;
    if (eq == REF_EULER1D) {
        *un = U[1] / rho;
        *ut = 0.0;
        p = (gamma - 1.0) * (U[2] - 0.5 * rho * ((*un) * (*un)));
    } else {
        *un = U[1] / rho;
        *ut = U[2] / rho;
        p = (gamma - 1.0) * (U[3] - 0.5 * rho * ((*un) * (*un) + (*ut) * (*ut)));
    }
    if (!(p > 0.0)) return REF_ENONPHYSICAL;
    *c = sqrt(gamma * p / rho);
    return REF_OK;
}

static void gather_node(const ref_problem *p, const double *u, int iy, int ix, double *U)
{
    const int nc = ncomp_of(p->equation);
    const size_t plane = (size_t)p->nx * (size_t)p->ny;
    for (int c = 0; c < nc; ++c) U[c] = u[(size_t)c * plane + (size_t)iy * p->nx + ix];
}

int ref_alpha(const ref_problem *p, const double *u, double *alpha_x, double *alpha_y)
{
    int st = check_problem(p);
    if (st) return st;
    const int nc = ncomp_of(p->equation);
    if (p->equation == REF_ADVECTION) {
        if (alpha_x) alpha_x[0] = fabs(p->adv_speed);
        if (alpha_y) alpha_y[0] = 0.0;
        return REF_OK;
    }
    double ax[4] = {0, 0, 0, 0}, ay[4] = {0, 0, 0, 0};
    for (int iy = 0; iy < p->ny; ++iy)
        for (int ix = 0; ix < p->nx; ++ix) {
            double U[4], un, ut, c;
            gather_node(p, u, iy, ix, U);
            if (node_speed(p->equation, p->gamma, U, &un, &ut, &c)) return REF_ENONPHYSICAL;
            /* x-direction eigenvalues: u-c, u, (u,) u+c */
            double lx[4], ly[4];
            if (nc == 3) { lx[0] = un - c; lx[1] = un; lx[2] = un + c; }
            else {
                lx[0] = un - c; lx[1] = un; lx[2] = un; lx[3] = un + c;
                ly[0] = ut - c; ly[1] = ut; ly[2] = ut; ly[3] = ut + c;
            }
            for (int s = 0; s < nc; ++s) {
                if (fabs(lx[s]) > ax[s]) ax[s] = fabs(lx[s]);
                if (nc == 4 && fabs(ly[s]) > ay[s]) ay[s] = fabs(ly[s]);
            }
        }
    for (int s = 0; s < nc; ++s) {
        if (alpha_x) alpha_x[s] = ax[s];
        if (alpha_y) alpha_y[s] = ay[s];
    }
    return REF_OK;
}

int64_t ref_selection_size(const ref_problem *p)
{
    if (check_problem(p)) return -1;
    const int64_t nc = ncomp_of(p->equation);
    int64_t n = nc * 2 * (int64_t)p->ny * (p->nx + 1);
    if (p->equation == REF_EULER2D) n += nc * 2 * (int64_t)(p->ny + 1) * p->nx;
    return n;
}

/*
 * One line of n nodes (a 1D problem, a row of a 2D problem, or a column of a
 * 2D problem with the two momentum components exchanged so that the line
 * direction reads as "x").  lin[c][G + k] holds node k (ghosts filled by the
 * boundary condition); fhat[c][i], i = 0..n, receives the numerical flux at
 * face i (between nodes i-1 and i).  sel/tie: pointer to the (component 0,
 * plus side) entry of this line and the distance between consecutive
 * (component, side) blocks, or NULL.
 */
static int line_fluxes(const ref_problem *p, int n, int G, double *const *lin,
                       const double *alpha, double **fhat, uint8_t *sel, uint8_t *tie,
                       const uint8_t *force, int64_t *nbad, int64_t face_stride, int64_t block_stride)
{
    const int eq = p->equation, nc = ncomp_of(eq), h = p->order == 5 ? 3 : 4;
    const int W = 2 * h + 2; /* stencil nodes j-h .. j+h+1 of face j+1/2 */
    double fplus[9], fminus[9], mplus[9], mminus[9];

    for (int i = 0; i <= n; ++i) {
        const int j = i - 1; /* face i is x_{j+1/2} with j = i-1 */
        if (eq == REF_ADVECTION) {
            for (int q = 0; q <= 2 * h; ++q) {
                const double up = lin[0][G + j - h + q];        /* node j-h+q   */
                const double um = lin[0][G + j + 1 + h - q];    /* node j+1+h-q */
                const double a = p->adv_speed;
                fplus[q] = 0.5 * (a * up + alpha[0] * up);
                fminus[q] = 0.5 * (a * um - alpha[0] * um);
                mplus[q] = 0.5 * (fabs(a * up) + alpha[0] * fabs(up));
                mminus[q] = 0.5 * (fabs(a * um) + alpha[0] * fabs(um));
            }
            double hp, hm;
            int sp, sm, tp, tm;
            const int fp = force ? force[i * face_stride] : -1;
            const int fm = force ? force[i * face_stride + block_stride] : -1;
            if (ref_reconstruct_replay(p->order, fplus, mplus, p->delta, fp, &hp, &sp, &tp, NULL)) ++*nbad;
            if (ref_reconstruct_replay(p->order, fminus, mminus, p->delta, fm, &hm, &sm, &tm, NULL)) ++*nbad;
            fhat[0][i] = hp + hm;
            if (sel) { sel[i * face_stride] = (uint8_t)sp; sel[i * face_stride + block_stride] = (uint8_t)sm; }
            if (tie) { tie[i * face_stride] = (uint8_t)tp; tie[i * face_stride + block_stride] = (uint8_t)tm; }
            continue;
        }
        const int dim = eq == REF_EULER1D ? 1 : 2;
        if (p->recon_vars == REF_COMPONENT) {
            /* conserved components: f^(+/-) = (F_c +/- alpha U_c)/2 with one alpha */
            const double a = alpha[0] > alpha[nc - 1] ? alpha[0] : alpha[nc - 1];
            double Uw[10][4], Fw[10][4];
            for (int t = 0; t < W; ++t) {
                for (int c = 0; c < nc; ++c) Uw[t][c] = lin[c][G + j - h + t];
                if (ref_euler_flux(dim, p->gamma, Uw[t], Fw[t])) return REF_ENONPHYSICAL;
            }
            for (int c = 0; c < nc; ++c) {
                for (int q = 0; q <= 2 * h; ++q) {
                    const int np = q, nm = 2 * h + 1 - q;
                    fplus[q] = 0.5 * (Fw[np][c] + a * Uw[np][c]);
                    fminus[q] = 0.5 * (Fw[nm][c] - a * Uw[nm][c]);
                    mplus[q] = 0.5 * (fabs(Fw[np][c]) + a * fabs(Uw[np][c]));
                    mminus[q] = 0.5 * (fabs(Fw[nm][c]) + a * fabs(Uw[nm][c]));
                }
                double hp, hm;
                int sp, sm, tp, tm;
                const int64_t o = (int64_t)c * 2 * block_stride + i * face_stride;
                const int fp = force ? force[o] : -1, fm = force ? force[o + block_stride] : -1;
                if (ref_reconstruct_replay(p->order, fplus, mplus, p->delta, fp, &hp, &sp, &tp, NULL)) ++*nbad;
                if (ref_reconstruct_replay(p->order, fminus, mminus, p->delta, fm, &hm, &sm, &tm, NULL)) ++*nbad;
                fhat[c][i] = hp + hm;
                if (sel) { sel[o] = (uint8_t)sp; sel[o + block_stride] = (uint8_t)sm; }
                if (tie) { tie[o] = (uint8_t)tp; tie[o + block_stride] = (uint8_t)tm; }
            }
            continue;
        }
        /* Euler: Roe state of the two nodes adjacent to the face */
        double UL[4], UR[4], R[16], Lm[16];
        for (int c = 0; c < nc; ++c) { UL[c] = lin[c][G + j]; UR[c] = lin[c][G + j + 1]; }
        if (ref_roe_eigen(dim, p->gamma, UL, UR, R, Lm, NULL)) return REF_ENONPHYSICAL;

        /* characteristic projection of U and F at every stencil node */
        double LU[4][10], LF[4][10], MU[4][10], MF[4][10];
        for (int t = 0; t < W; ++t) {
            double U[4], F[4];
            for (int c = 0; c < nc; ++c) U[c] = lin[c][G + j - h + t];
            if (ref_euler_flux(dim, p->gamma, U, F)) return REF_ENONPHYSICAL;
            for (int s = 0; s < nc; ++s) {
                double au = 0.0, af = 0.0, mu = 0.0, mf = 0.0;
                for (int c = 0; c < nc; ++c) {
                    au = au + Lm[s * nc + c] * U[c];
                    af = af + Lm[s * nc + c] * F[c];
                    mu = mu + fabs(Lm[s * nc + c]) * fabs(U[c]);
                    mf = mf + fabs(Lm[s * nc + c]) * fabs(F[c]);
                }
                LU[s][t] = au; LF[s][t] = af; MU[s][t] = mu; MF[s][t] = mf;
            }
        }
        /* split, reconstruct each field on both sides */
        double what[4];
        for (int s = 0; s < nc; ++s) {
            for (int q = 0; q <= 2 * h; ++q) {
                const int np = q, nm = 2 * h + 1 - q; /* node j-h+q and mirrored node j+1+h-q */
                fplus[q] = 0.5 * (LF[s][np] + alpha[s] * LU[s][np]);
                fminus[q] = 0.5 * (LF[s][nm] - alpha[s] * LU[s][nm]);
                mplus[q] = 0.5 * (MF[s][np] + alpha[s] * MU[s][np]);
                mminus[q] = 0.5 * (MF[s][nm] + alpha[s] * MU[s][nm]);
            }
            double hp, hm;
            int sp, sm, tp, tm;
            const int64_t o = (int64_t)s * 2 * block_stride + i * face_stride;
            const int fp = force ? force[o] : -1, fm = force ? force[o + block_stride] : -1;
            if (ref_reconstruct_replay(p->order, fplus, mplus, p->delta, fp, &hp, &sp, &tp, NULL)) ++*nbad;
            if (ref_reconstruct_replay(p->order, fminus, mminus, p->delta, fm, &hm, &sm, &tm, NULL)) ++*nbad;
            what[s] = hp + hm;
            if (sel) { sel[o] = (uint8_t)sp; sel[o + block_stride] = (uint8_t)sm; }
            if (tie) { tie[o] = (uint8_t)tp; tie[o + block_stride] = (uint8_t)tm; }
        }
        /* back to conserved variables */
        for (int c = 0; c < nc; ++c) {
            double acc = 0.0;
            for (int s = 0; s < nc; ++s) acc = acc + R[c * nc + s] * what[s];
            fhat[c][i] = acc;
        }
    }
    return REF_OK;
}

int ref_rhs(const ref_problem *p, const double *u, double *L, uint8_t *sel, uint8_t *tie)
{
    return ref_rhs_replay(p, u, L, NULL, sel, tie, NULL);
}

/* L(u) with the selections of another evaluation replayed at near ties: at every
 * face, field and side where force[] names a candidate other than the oracle's
 * own choice, that candidate is taken if it lies in the oracle's tie set there
 * (see ref_reconstruct_replay); otherwise the oracle keeps its own choice and
 * counts the face in *nbad.  Returns REF_EMISMATCH when *nbad > 0. */
int ref_rhs_replay(const ref_problem *p, const double *u, double *L, const uint8_t *force,
                   uint8_t *sel, uint8_t *tie, int64_t *nbad_out)
{
    int st = check_problem(p);
    if (st) return st;
    if (!u || !L) return REF_EINVAL;
    const int nc = ncomp_of(p->equation), nx = p->nx, ny = p->ny;
    const int G = (p->order == 5 ? 3 : 4) + 1;
    const size_t plane = (size_t)nx * ny;
    double ax[4], ay[4];
    st = ref_alpha(p, u, ax, ay);
    if (st) return st;

    const int nmax = nx > ny ? nx : ny;
    double *buf = (double *)malloc(sizeof(double) * (size_t)nc * ((nmax + 2 * G) + (nmax + 1)));
    if (!buf) return REF_EINVAL;
    double *lin[4], *fh[4];
    for (int c = 0; c < nc; ++c) {
        lin[c] = buf + (size_t)c * (nmax + 2 * G);
        fh[c] = buf + (size_t)nc * (nmax + 2 * G) + (size_t)c * (nmax + 1);
    }
    const double dx = dx_of(p);
    const int64_t xblock = (int64_t)ny * (nx + 1);
    int64_t nbad = 0;

    /* x-direction: every row */
    for (int iy = 0; iy < ny && !st; ++iy) {
        for (int k = -G; k < nx + G; ++k) {
            const int ix = bc_index(k, nx, p->bc_x);
            for (int c = 0; c < nc; ++c) lin[c][G + k] = u[c * plane + (size_t)iy * nx + ix];
        }
        st = line_fluxes(p, nx, G, lin, ax, fh, sel ? sel + (int64_t)iy * (nx + 1) : NULL,
                         tie ? tie + (int64_t)iy * (nx + 1) : NULL,
                         force ? force + (int64_t)iy * (nx + 1) : NULL, &nbad, 1, xblock);
        for (int c = 0; c < nc && !st; ++c)
            for (int ix = 0; ix < nx; ++ix)
                L[c * plane + (size_t)iy * nx + ix] = -(fh[c][ix + 1] - fh[c][ix]) / dx;
    }
    /* y-direction (2D): every column, momentum components exchanged */
    if (p->equation == REF_EULER2D && !st) {
        const double dy = dy_of(p);
        const int perm[4] = {0, 2, 1, 3};
        const int64_t ybase = (int64_t)nc * 2 * xblock, yblock = (int64_t)(ny + 1) * nx;
        for (int ix = 0; ix < nx && !st; ++ix) {
            for (int k = -G; k < ny + G; ++k) {
                const int iy = bc_index(k, ny, p->bc_y);
                for (int c = 0; c < nc; ++c) lin[c][G + k] = u[perm[c] * plane + (size_t)iy * nx + ix];
            }
            st = line_fluxes(p, ny, G, lin, ay, fh, sel ? sel + ybase + ix : NULL,
                             tie ? tie + ybase + ix : NULL, force ? force + ybase + ix : NULL, &nbad,
                             nx, yblock);
            for (int c = 0; c < nc && !st; ++c)
                for (int iy = 0; iy < ny; ++iy) {
                    const size_t o = perm[c] * plane + (size_t)iy * nx + ix;
                    L[o] = L[o] + (-(fh[c][iy + 1] - fh[c][iy]) / dy);
                }
        }
    }
    free(buf);
    if (nbad_out) *nbad_out = nbad;
    if (!st && nbad > 0) st = REF_EMISMATCH;
    return st;
}

int ref_step(const ref_problem *p, double *u, double dt)
{
    return ref_step_replay(p, u, dt, NULL, NULL);
}

/* One step with the selections of another evaluation replayed at near ties:
 * force[] holds three records of ref_selection_size(p) entries, one per stage;
 * a mismatch outside the tie set is counted in *nbad (summed over the stages)
 * and the step is completed with the oracle's own choice there. */
int ref_step_replay(const ref_problem *p, double *u, double dt, const uint8_t *force, int64_t *nbad_out)
{
    int st = check_problem(p);
    if (st) return st;
    const int64_t rec = ref_selection_size(p);
    int64_t nb[3] = {0, 0, 0};
    const size_t n = (size_t)ncomp_of(p->equation) * p->nx * p->ny;
    double *u1 = (double *)malloc(sizeof(double) * n * 3);
    if (!u1) return REF_EINVAL;
    double *u2 = u1 + n, *Lb = u1 + 2 * n;

    st = ref_rhs_replay(p, u, Lb, force, NULL, NULL, &nb[0]);
    if (st == REF_EMISMATCH) st = REF_OK;
    for (size_t i = 0; i < n && !st; ++i) u1[i] = u[i] + dt * Lb[i];
    if (!st) st = ref_rhs_replay(p, u1, Lb, force ? force + rec : NULL, NULL, NULL, &nb[1]);
    if (st == REF_EMISMATCH) st = REF_OK;
    for (size_t i = 0; i < n && !st; ++i) u2[i] = 0.75 * u[i] + 0.25 * (u1[i] + dt * Lb[i]);
    if (!st) st = ref_rhs_replay(p, u2, Lb, force ? force + 2 * rec : NULL, NULL, NULL, &nb[2]);
    if (st == REF_EMISMATCH) st = REF_OK;
    for (size_t i = 0; i < n && !st; ++i) u[i] = (1.0 / 3.0) * u[i] + (2.0 / 3.0) * (u2[i] + dt * Lb[i]);
    free(u1);
    if (nbad_out) *nbad_out = nb[0] + nb[1] + nb[2];
    if (!st && nb[0] + nb[1] + nb[2] > 0) st = REF_EMISMATCH;
    return st;
}

int ref_dt(const ref_problem *p, const double *u, double cfl, double *dt)
{
    int st = check_problem(p);
    if (st) return st;
    if (!(cfl > 0.0) || !dt) return REF_EINVAL;
    const double dx = dx_of(p);
    if (p->equation == REF_ADVECTION) {
        *dt = cfl * dx / fabs(p->adv_speed);
        return REF_OK;
    }
    double smax = 0.0;
    for (int iy = 0; iy < p->ny; ++iy)
        for (int ix = 0; ix < p->nx; ++ix) {
            double U[4], un, ut, c, s;
            gather_node(p, u, iy, ix, U);
            if (node_speed(p->equation, p->gamma, U, &un, &ut, &c)) return REF_ENONPHYSICAL;
            if (p->equation == REF_EULER1D) s = fabs(un) + c;
            else s = (fabs(un) + c) / dx + (fabs(ut) + c) / dy_of(p);
            if (s > smax) smax = s;
        }
    if (!(smax > 0.0)) return REF_ENONPHYSICAL;
    *dt = p->equation == REF_EULER1D ? cfl * dx / smax : cfl / smax;
    return REF_OK;
}

int ref_solve(const ref_problem *p, double *u, double t_final, double cfl, double dt_fixed,
              int64_t max_steps, double *t_out, int64_t *steps_out)
{
    int st = check_problem(p);
    if (st) return st;
    if (!u || !(t_final >= 0.0) || max_steps < 0) return REF_EINVAL;
    if (!(dt_fixed > 0.0) && !(cfl > 0.0)) return REF_EINVAL;
    double t = 0.0;
    int64_t steps = 0;
    while (steps < max_steps) {
        const double rem = t_final - t;
        if (!(rem > 0.0)) break;
        double dt;
        if (dt_fixed > 0.0) dt = dt_fixed;
        else if ((st = ref_dt(p, u, cfl, &dt))) break;
        /* the step that reaches t_final (within a relative 1e-10 of dt) lands on it exactly */
        const int last = dt >= rem * (1.0 - 1e-10);
        if (last) dt = rem;
        if ((st = ref_step(p, u, dt))) break;
        t = last ? t_final : t + dt;
        steps = steps + 1;
    }
    if (t_out) *t_out = t;
    if (steps_out) *steps_out = steps;
    return st;
}
