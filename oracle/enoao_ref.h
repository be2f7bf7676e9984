/*
 * enoao_ref.h -- plain FP64 CPU oracle for the ENO-AO finite-difference method
 * (H. Shen, "A class of ENO schemes with adaptive order for solving hyperbolic
 * conservation laws", arXiv 2108.12742).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code: only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no source, header, table or helper with
 * the HIP implementation; the only thing both sides share is the seeded input
 * generator, which holds none of the method's arithmetic.
 *
 * Build: gcc -O2 -ffp-contract=off (no FMA contraction, true IEEE division,
 * literal evaluation order), see oracle/build_oracle.py.
 *
 * Layout: a state is SoA FP64 [ncomp][ny][nx] over the grid nodes
 * x_i = x_lo + i*dx, i = 0..nx-1, dx = (x_hi-x_lo)/nx (node grid of Section 2;
 * a periodic grid drops the duplicated end node).  ncomp = 1 (advection),
 * 3 (1D Euler: rho, rho*u, rho*e), 4 (2D Euler: rho, rho*u, rho*v, rho*e).
 *
 * Faces: a line of n nodes has n+1 faces; face i sits between nodes i-1 and i
 * (face 0 and face n coincide on a periodic line).
 *
 * Return codes: 0 ok, 1 invalid argument, 5 non-physical state (rho<=0, p<=0,
 * NaN, or a non-positive Roe sound speed), 7 a replayed selection outside the
 * oracle's tie set (the *_replay calls below).
 */
#ifndef ENOAO_REF_H
#define ENOAO_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { REF_ADVECTION = 0, REF_EULER1D = 1, REF_EULER2D = 2 };
enum { REF_BC_PERIODIC = 0, REF_BC_TRANSMISSIVE = 1 };
enum { REF_CHAR_ROE = 0, REF_COMPONENT = 1 };
enum { REF_OK = 0, REF_EINVAL = 1, REF_ENONPHYSICAL = 5, REF_EMISMATCH = 7 };

typedef struct ref_problem {
    int32_t equation;   /* REF_ADVECTION | REF_EULER1D | REF_EULER2D            */
    int32_t order;      /* designed order: 5 or 7                                 */
    int32_t nx, ny;     /* nodes per direction, ny = 1 in 1D                      */
    double  x_lo, x_hi, y_lo, y_hi;
    int32_t bc_x, bc_y; /* REF_BC_PERIODIC | REF_BC_TRANSMISSIVE                  */
    double  gamma;      /* ideal-gas ratio of specific heats (Euler)              */
    double  adv_speed;  /* a in u_t + a u_x = 0 (advection)                       */
    double  delta;      /* selection threshold of the reconstruction principle    */
    int32_t recon_vars; /* Euler: REF_CHAR_ROE (characteristic fields of the Roe
                           state, the paper's choice) | REF_COMPONENT (conserved
                           components, one alpha = max(|u|+c) for all of them)  */
} ref_problem;

/* ---- single-face reconstruction (Section 3.2, Tables of fluxes and delta_L/delta_R) ----
 * f[0..2h] is the one-sided window of split-flux values around the target cell
 * j = f[h] (h = 3 for order 5, 4 for order 7); mag[] (may be NULL) holds a
 * magnitude bound for each f[] used only to scale the tie test. */
int ref_num_candidates(int order);
int ref_candidates(int order, const double *f, double *flux_k, double *is_k);
int ref_reconstruct(int order, const double *f, const double *mag, double delta,
                    double *fhat, int *sel, int *tie);
/* Replay of another evaluation's choice.  tie_set (may be NULL) receives a bit
 * mask of the candidates an evaluation of the same indicators with rounding
 * errors below the near-tie margin could select ({sel} when tie == 0).  With
 * forced >= 0: if forced is in that set, it is taken (fhat, sel = forced);
 * otherwise the oracle's own choice is returned with status REF_EMISMATCH.
 * forced < 0: the same as ref_reconstruct. */
int ref_reconstruct_replay(int order, const double *f, const double *mag, double delta, int forced,
                           double *fhat, int *sel, int *tie, unsigned *tie_set);
/* scale_k[k]: the forward-error scale of candidate k's indicator that the
 * near-tie margin multiplies (larger of the two delta rows' sum |c| mag). */
int ref_indicator_scales(int order, const double *f, const double *mag, double *scale_k);

/* ---- Euler building blocks (Section 4: Roe average, characteristic fields) ----
 * dim = 1 (3 components) or 2 (4 components, x-direction; the y-direction uses
 * the same with the two momentum components exchanged).  R, L are row-major
 * ncomp x ncomp, lam[ncomp] the Roe-state eigenvalues. */
int ref_euler_flux(int dim, double gamma, const double *U, double *F);
int ref_roe_eigen(int dim, double gamma, const double *UL, const double *UR,
                  double *R, double *L, double *lam);

/* ---- whole-grid operators ----
 * alpha: per characteristic field and direction, the global maximum of
 * |lambda_s| over all nodes (alpha_x[ncomp], alpha_y[ncomp]; advection: |a|).
 * rhs: L(u) of Eq. (1DWENOFD), summed over x and y in 2D.  sel/tie (may be
 * NULL) receive the selected candidate (0..K-1, order of increasing priority)
 * and the oracle's near-tie flag for every face, field and side, laid out as
 *   x: [ncomp][2 sides: plus, minus][ny][nx+1]
 *   y: [ncomp][2][ny+1][nx]           (2D only, directly after the x block)
 * step: one third-order TVD Runge-Kutta step of size dt, in place.
 * dt:   CFL time step (advection cfl*dx/|a|; 1D Euler cfl*dx/max(|u|+c);
 *       2D Euler cfl/max((|u|+c)/dx + (|v|+c)/dy)).
 * solve: steps to t_final, either with the CFL dt (dt_fixed <= 0) or the fixed
 *       dt_fixed, clipping the last step to land on t_final. */
int64_t ref_selection_size(const ref_problem *p);
int ref_alpha(const ref_problem *p, const double *u, double *alpha_x, double *alpha_y);
int ref_rhs(const ref_problem *p, const double *u, double *L, uint8_t *sel, uint8_t *tie);
int ref_step(const ref_problem *p, double *u, double dt);
/* The same with another evaluation's selection record force[] (layout of sel;
 * for a step three records, one per stage, each ref_selection_size entries)
 * replayed where the oracle's tie set allows it; faces where it does not are
 * counted in *nbad (may be NULL) and keep the oracle's choice, and the call
 * returns REF_EMISMATCH.  force == NULL gives ref_rhs / ref_step exactly. */
int ref_rhs_replay(const ref_problem *p, const double *u, double *L, const uint8_t *force,
                   uint8_t *sel, uint8_t *tie, int64_t *nbad);
int ref_step_replay(const ref_problem *p, double *u, double dt, const uint8_t *force, int64_t *nbad);
int ref_dt(const ref_problem *p, const double *u, double cfl, double *dt);
int ref_solve(const ref_problem *p, double *u, double t_final, double cfl, double dt_fixed,
              int64_t max_steps, double *t_out, int64_t *steps_out);

#ifdef __cplusplus
}
#endif
#endif
