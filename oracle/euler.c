/*
 * euler.c -- ideal-gas Euler building blocks for the oracle.
 * TEST INFRASTRUCTURE ONLY (see enoao_ref.h).
 *
 * Section 4 (1D Euler: U = [rho, rho u, rho e], F = [rho u, rho u^2 + p,
 * (rho e + p) u], e = p/(rho(gamma-1)) + u^2/2; 2D Euler: U = [rho, rho u,
 * rho v, rho e], F = [rho u, rho u^2 + p, rho u v, (rho e + p) u],
 * e = p/(rho(gamma-1)) + (u^2+v^2)/2).
 *
 * Characteristic decomposition uses the Roe average at the face (the paper's
 * numerical-examples section states that the Roe average is adopted for the
 * characteristic decomposition of the Euler equations).  The paper does not
 * print the eigenvectors; the reading taken is the textbook right eigenvectors
 * with unit first component (for the acoustic and entropy fields) and the
 * left eigenvectors as their exact inverse:
 *   1D  R = [[1,1,1],[u-c,u,u+c],[H-uc,u^2/2,H+uc]]
 *   2D  R columns (1,u-c,v,H-uc), (1,u,v,q^2/2), (0,0,1,v), (1,u+c,v,H+uc)
 * with b1 = (gamma-1)/c^2, b2 = b1 q^2/2 (q^2 = u^2 [+ v^2]).  The selection
 * threshold delta is absolute, so this scaling is part of the scheme's
 * definition for systems.
 */
#include <math.h>
#include "enoao_ref.h"

int ref_euler_flux(int dim, double gamma, const double *U, double *F)
{
    const double rho = U[0];
    if (!(rho > 0.0)) return REF_ENONPHYSICAL;
    if (dim == 1) {
        const double u = U[1] / rho;
        const double p = (gamma - 1.0) * (U[2] - 0.5 * rho * (u * u));
        if (!(p > 0.0)) return REF_ENONPHYSICAL;
        F[0] = U[1];
        F[1] = U[1] * u + p;
        F[2] = (U[2] + p) * u;
        return REF_OK;
    }
    if (dim == 2) {
        const double u = U[1] / rho, v = U[2] / rho;
        const double p = (gamma - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v));
        if (!(p > 0.0)) return REF_ENONPHYSICAL;
        F[0] = U[1];
        F[1] = U[1] * u + p;
        F[2] = U[1] * v;
        F[3] = (U[3] + p) * u;
        return REF_OK;
    }
    return REF_EINVAL;
}

/* primitive velocity(ies), pressure and total enthalpy H = (E+p)/rho */
static int primitives(int dim, double gamma, const double *U, double *u, double *v,
                      double *H)
{
    const double rho = U[0];
    if (!(rho > 0.0)) return REF_ENONPHYSICAL;
    double p;
    if (dim == 1) {
        *u = U[1] / rho;
        *v = 0.0;
        p = (gamma - 1.0) * (U[2] - 0.5 * rho * ((*u) * (*u)));
        *H = (U[2] + p) / rho;
    } else {
        *u = U[1] / rho;
        *v = U[2] / rho;
        p = (gamma - 1.0) * (U[3] - 0.5 * rho * ((*u) * (*u) + (*v) * (*v)));
        *H = (U[3] + p) / rho;
    }
    if (!(p > 0.0)) return REF_ENONPHYSICAL;
    return REF_OK;
}

int ref_roe_eigen(int dim, double gamma, const double *UL, const double *UR,
                  double *R, double *L, double *lam)
{
    if (dim != 1 && dim != 2) return REF_EINVAL;
    double uL, vL, HL, uR, vR, HR;
    if (primitives(dim, gamma, UL, &uL, &vL, &HL) || primitives(dim, gamma, UR, &uR, &vR, &HR))
        return REF_ENONPHYSICAL;
    /* Roe average: weights sqrt(rho) */
    const double sL = sqrt(UL[0]), sR = sqrt(UR[0]);
    const double u = (sL * uL + sR * uR) / (sL + sR);
    const double v = (sL * vL + sR * vR) / (sL + sR);
    const double H = (sL * HL + sR * HR) / (sL + sR);
    const double q2 = dim == 1 ? u * u : u * u + v * v;
    const double c2 = (gamma - 1.0) * (H - 0.5 * q2);
    if (!(c2 > 0.0)) return REF_ENONPHYSICAL;
    const double c = sqrt(c2);
    const double b1 = (gamma - 1.0) / c2;
    const double b2 = 0.5 * q2 * b1;

    if (dim == 1) {
        const double r[9] = {1.0, 1.0, 1.0,
                             u - c, u, u + c,
                             H - u * c, 0.5 * u * u, H + u * c};
        const double l[9] = {0.5 * (b2 + u / c), 0.5 * (-b1 * u - 1.0 / c), 0.5 * b1,
                             1.0 - b2, b1 * u, -b1,
                             0.5 * (b2 - u / c), 0.5 * (-b1 * u + 1.0 / c), 0.5 * b1};
        for (int i = 0; i < 9; ++i) { R[i] = r[i]; L[i] = l[i]; }
        if (lam) { lam[0] = u - c; lam[1] = u; lam[2] = u + c; }
    } else {
        const double r[16] = {1.0, 1.0, 0.0, 1.0,
                              u - c, u, 0.0, u + c,
                              v, v, 1.0, v,
                              H - u * c, 0.5 * q2, v, H + u * c};
        const double l[16] = {0.5 * (b2 + u / c), 0.5 * (-b1 * u - 1.0 / c), 0.5 * (-b1 * v), 0.5 * b1,
                              1.0 - b2, b1 * u, b1 * v, -b1,
                              -v, 0.0, 1.0, 0.0,
                              0.5 * (b2 - u / c), 0.5 * (-b1 * u + 1.0 / c), 0.5 * (-b1 * v), 0.5 * b1};
        for (int i = 0; i < 16; ++i) { R[i] = r[i]; L[i] = l[i]; }
        if (lam) { lam[0] = u - c; lam[1] = u; lam[2] = u; lam[3] = u + c; }
    }
    return REF_OK;
}
