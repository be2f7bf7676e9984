/*
 * recon.c -- ENO-AO reconstruction of one side of one face (oracle).
 * TEST INFRASTRUCTURE ONLY (see enoao_ref.h).
 *
 * What is computed (Section 3 of the paper):
 *  - candidate stencils S_{j-m}^{j+n}: for order 5 the six stencils listed in
 *    Section 3.2 (S_j^j, S_j^{j+1}, S_{j-1}^{j+1}, S_{j-2}^{j+1}, S_{j-1}^{j+2},
 *    S_{j-2}^{j+2}); for order 7 those plus S_{j-3}^{j+2}, S_{j-2}^{j+3},
 *    S_{j-3}^{j+3};
 *  - each candidate's value at x_{j+1/2}: the table of numerical fluxes on
 *    different stencils (Table "Flux_reconstruction");
 *  - each candidate's smoothness indicator IS = min(delta_L, delta_R) of
 *    Eq. (New_Smoothness_Indicator), with delta_L / delta_R in the closed forms
 *    of Tables "DeltaL" and "DeltaR" (the special averaged form for S_j^j);
 *  - the reconstruction principle (Section 3.2): when several indicators do not
 *    exceed delta, the highest-order one wins and, at equal order, the central
 *    stencil beats the upwind-biased one; otherwise the smallest indicator wins.
 *
 * Candidates are numbered in increasing priority, so "highest priority" is
 * "largest index".  Reading of two points the text leaves open:
 *  - "smaller than delta" is taken as IS <= delta (the paper's appendix code
 *    tests with <=);
 *  - a tie for the smallest indicator is resolved in favour of the candidate of
 *    higher priority (the appendix code keeps the last minimum in priority
 *    order).
 *
 * Near-tie flag (test policy, not part of the method): an implementation that
 * rounds differently may legitimately pick another candidate when a deciding
 * comparison is within rounding.  The flag is raised when any comparison that
 * decided the outcome (IS_k against delta for every candidate examined, and in
 * the fallback IS_k against the minimum) is within TIE_EPS of the forward-error
 * scale of the indicators involved, except for exact ties between two
 * indicators realised by one and the same undivided difference (the pairs of
 * identical rows in the delta tables), which every implementation reproduces,
 * and except for an indicator that is zero because one of its delta rows reads
 * only equal values: a difference of equal values is exactly zero however it is
 * evaluated, so the comparison with delta >= 0 is exact (such zeros are common:
 * flat regions of piecewise constant data, or the minus-side flux of advection
 * with a > 0, which is zero at every node).
 */
#include <math.h>
#include <stddef.h>
#include "enoao_ref.h"

#define TIE_EPS 1e-14
#define MAXC 9

typedef struct {
    int m, n;          /* stencil S_{j-m}^{j+n}                                   */
    int den;           /* divisor of the flux row                                 */
    int fc[7];         /* flux coefficients on f_{j-m} .. f_{j+n}                 */
    int nd;            /* number of terms of the delta rows (m+n+2); 0 for S_j^j  */
    int dl[8];         /* delta_L coefficients on f_{j-m-1} .. f_{j+n}            */
    int dr[8];         /* delta_R coefficients on f_{j-m} .. f_{j+n+1}            */
} cand_t;

/* Table of numerical fluxes and Tables DeltaL / DeltaR, rows of the candidate
 * stencils, in increasing priority. */
static const cand_t CANDS[MAXC] = {
    /* 0: S_j^j        f_j */
    {0, 0, 1, {1}, 0, {0}, {0}},
    /* 1: S_j^{j+1}    (f_j+f_{j+1})/2 */
    {0, 1, 2, {1, 1}, 3, {1, -2, 1}, {1, -2, 1}},
    /* 2: S_{j-1}^{j+1} (-f_{j-1}+5f_j+2f_{j+1})/6 */
    {1, 1, 6, {-1, 5, 2}, 4, {-1, 3, -3, 1}, {-1, 3, -3, 1}},
    /* 3: S_{j-2}^{j+1} (f_{j-2}-5f_{j-1}+13f_j+3f_{j+1})/12 */
    {2, 1, 12, {1, -5, 13, 3}, 5, {1, -4, 6, -4, 1}, {1, -4, 6, -4, 1}},
    /* 4: S_{j-1}^{j+2} (-f_{j-1}+7f_j+7f_{j+1}-f_{j+2})/12 */
    {1, 2, 12, {-1, 7, 7, -1}, 5, {1, -4, 6, -4, 1}, {1, -4, 6, -4, 1}},
    /* 5: S_{j-2}^{j+2} (2f_{j-2}-13f_{j-1}+47f_j+27f_{j+1}-3f_{j+2})/60 */
    {2, 2, 60, {2, -13, 47, 27, -3}, 6, {-1, 5, -10, 10, -5, 1}, {-1, 5, -10, 10, -5, 1}},
    /* 6: S_{j-3}^{j+2} (-f_{j-3}+7f_{j-2}-23f_{j-1}+57f_j+22f_{j+1}-2f_{j+2})/60 */
    {3, 2, 60, {-1, 7, -23, 57, 22, -2}, 7, {1, -6, 15, -20, 15, -6, 1}, {1, -6, 15, -20, 15, -6, 1}},
    /* 7: S_{j-2}^{j+3} (f_{j-2}-8f_{j-1}+37f_j+37f_{j+1}-8f_{j+2}+f_{j+3})/60 */
    {2, 3, 60, {1, -8, 37, 37, -8, 1}, 7, {1, -6, 15, -20, 15, -6, 1}, {1, -6, 15, -20, 15, -6, 1}},
    /* 8: S_{j-3}^{j+3} (-3f_{j-3}+25f_{j-2}-101f_{j-1}+319f_j+214f_{j+1}-38f_{j+2}+4f_{j+3})/420 */
    {3, 3, 420, {-3, 25, -101, 319, 214, -38, 4}, 8,
     {-1, 7, -21, 35, -35, 21, -7, 1}, {-1, 7, -21, 35, -35, 21, -7, 1}},
};

int ref_num_candidates(int order)
{
    if (order == 5) return 6;
    if (order == 7) return 9;
    return 0;
}

static int half_width(int order) { return order == 5 ? 3 : 4; }

/* sum_{t} c[t] * f[j + first + t], evaluated left to right, plus its magnitude
 * scale sum |c[t]| * mag[...] (mag may be NULL: then |f| is used). */
static double lin(const int *c, int nt, const double *f, const double *mag, int at,
                  double *scale)
{
    double acc = 0.0, s = 0.0;
    for (int t = 0; t < nt; ++t) {
        acc = acc + (double)c[t] * f[at + t];
        s = s + fabs((double)c[t]) * (mag ? mag[at + t] : fabs(f[at + t]));
    }
    if (scale) *scale = s;
    return acc;
}

/* Per candidate: flux value, delta_L, delta_R and their scales. */
typedef struct {
    double flux, dL, dR, sL, sR, is, s;
    int side;          /* 0: IS realised by delta_L, 1: by delta_R */
    int flat;          /* the nodes one of the delta rows reads hold equal values */
} eval_t;

/* whether f[a .. b] are all equal */
static int all_equal(const double *f, int a, int b)
{
    for (int t = a + 1; t <= b; ++t)
        if (f[t] != f[a]) return 0;
    return 1;
}

static void eval_candidates(int order, const double *f, const double *mag, eval_t *ev)
{
    const int K = ref_num_candidates(order), h = half_width(order);
    for (int k = 0; k < K; ++k) {
        const cand_t *c = &CANDS[k];
        const int j = h; /* index of f_j in the window */
        double fs;
        ev[k].flux = lin(c->fc, c->m + c->n + 1, f, mag, j - c->m, &fs) / (double)c->den;
        if (c->nd == 0) {
            ev[k].flat = all_equal(f, j - 2, j) || all_equal(f, j, j + 2);
            /* S_j^j: delta_L = (|f_j - f_{j-1}| + |f_{j-1} - f_{j-2}|)/2, delta_R mirrored */
            ev[k].dL = (fabs(f[j] - f[j - 1]) + fabs(f[j - 1] - f[j - 2])) / 2.0;
            ev[k].dR = (fabs(f[j] - f[j + 1]) + fabs(f[j + 1] - f[j + 2])) / 2.0;
            if (mag) {
                ev[k].sL = (mag[j] + 2.0 * mag[j - 1] + mag[j - 2]) / 2.0;
                ev[k].sR = (mag[j] + 2.0 * mag[j + 1] + mag[j + 2]) / 2.0;
            } else {
                ev[k].sL = (fabs(f[j]) + 2.0 * fabs(f[j - 1]) + fabs(f[j - 2])) / 2.0;
                ev[k].sR = (fabs(f[j]) + 2.0 * fabs(f[j + 1]) + fabs(f[j + 2])) / 2.0;
            }
        } else {
            ev[k].flat = all_equal(f, j - c->m - 1, j + c->n) || all_equal(f, j - c->m, j + c->n + 1);
            ev[k].dL = fabs(lin(c->dl, c->nd, f, mag, j - c->m - 1, &ev[k].sL));
            ev[k].dR = fabs(lin(c->dr, c->nd, f, mag, j - c->m, &ev[k].sR));
        }
        /* IS = MIN(delta_L, delta_R) */
        if (ev[k].dL <= ev[k].dR) { ev[k].is = ev[k].dL; ev[k].side = 0; }
        else                      { ev[k].is = ev[k].dR; ev[k].side = 1; }
        ev[k].s = ev[k].sL > ev[k].sR ? ev[k].sL : ev[k].sR;
    }
}

int ref_candidates(int order, const double *f, double *flux_k, double *is_k)
{
    eval_t ev[MAXC];
    const int K = ref_num_candidates(order);
    if (K == 0 || !f) return REF_EINVAL;
    eval_candidates(order, f, NULL, ev);
    for (int k = 0; k < K; ++k) {
        if (flux_k) flux_k[k] = ev[k].flux;
        if (is_k) is_k[k] = ev[k].is;
    }
    return REF_OK;
}

/* The undivided difference realising IS_k, as (first node offset from j, row):
 * two candidates realised by identical rows over identical nodes hold bitwise
 * equal indicators in every implementation that evaluates that row once. */
static int same_expression(const eval_t *ev, int a, int b)
{
    const cand_t *ca = &CANDS[a], *cb = &CANDS[b];
    if (ca->nd == 0 || cb->nd == 0 || ca->nd != cb->nd) return 0;
    const int *ra = ev[a].side ? ca->dr : ca->dl, *rb = ev[b].side ? cb->dr : cb->dl;
    const int oa = ev[a].side ? -ca->m : -ca->m - 1, ob = ev[b].side ? -cb->m : -cb->m - 1;
    if (oa != ob) return 0;
    for (int t = 0; t < ca->nd; ++t)
        if (ra[t] != rb[t]) return 0;
    return 1;
}

/* whether candidate k's choice of the smaller of delta_L, delta_R is robust */
static int side_robust(const eval_t *e)
{
    return fabs(e->dL - e->dR) > TIE_EPS * (e->sL + e->sR);
}

/*
 * The decision of one side of one face, and the set of candidates that an
 * evaluation of the same indicators with rounding errors below TIE_EPS times
 * their scale could select instead (the tie set; it is {chosen} when no
 * deciding comparison is within that margin).  Walking the candidates from the
 * highest priority down, a candidate near delta may go either way, so it joins
 * the set and the walk goes on; the first candidate clearly within delta ends
 * the walk; when no candidate is clearly within delta the second principle is
 * reachable and every candidate whose indicator is within the margin of the
 * smallest one joins the set (the smallest under perturbed values lies within
 * the sum of the two margins of the exact smallest).  The exceptions of the
 * near-tie flag apply alike: indicators that are exact zeros of equal values,
 * and exact ties of one and the same difference row, decide the same way in
 * every evaluation.
 */
static void decide(const eval_t *ev, int K, double delta, int *chosen_out, int *near_out, unsigned *set_out)
{
    int chosen = -1, near = 0, settled = 0;
    unsigned set = 0u;
    /* First principle, as the method takes it, and its near comparisons. */
    for (int k = K - 1; k >= 0; --k) {
        const int exact_zero = ev[k].is == 0.0 && ev[k].flat;
        if (fabs(ev[k].is - delta) <= TIE_EPS * ev[k].s && !exact_zero) near = 1;
        if (ev[k].is <= delta) { chosen = k; break; }
    }
    /* The walk of a perturbed evaluation. */
    for (int k = K - 1; k >= 0; --k) {
        const int exact_zero = ev[k].is == 0.0 && ev[k].flat;
        const int close = fabs(ev[k].is - delta) <= TIE_EPS * ev[k].s && !exact_zero;
        if (close) { set |= 1u << k; continue; }
        if (ev[k].is <= delta) { set |= 1u << k; settled = 1; break; }
    }
    /* Second principle: the smallest indicator; equal minima go to the
     * candidate of higher priority. */
    if (chosen < 0 || !settled) {
        int amin = 0;
        for (int k = 1; k < K; ++k)
            if (ev[k].is <= ev[amin].is) amin = k;
        const int taken = chosen < 0;
        if (!settled) set |= 1u << amin;
        for (int k = 0; k < K; ++k) {
            if (k == amin) continue;
            if (fabs(ev[k].is - ev[amin].is) > TIE_EPS * (ev[k].s + ev[amin].s)) continue;
            if (ev[k].is == ev[amin].is && same_expression(ev, k, amin) &&
                side_robust(&ev[k]) && side_robust(&ev[amin]))
                continue;
            if (taken) near = 1;
            if (!settled) set |= 1u << k;
        }
        if (taken) chosen = amin;
    }
    *chosen_out = chosen;
    *near_out = near;
    *set_out = set;
}

int ref_reconstruct(int order, const double *f, const double *mag, double delta,
                    double *fhat, int *sel, int *tie)
{
    return ref_reconstruct_replay(order, f, mag, delta, -1, fhat, sel, tie, NULL);
}

int ref_reconstruct_replay(int order, const double *f, const double *mag, double delta, int forced,
                           double *fhat, int *sel, int *tie, unsigned *tie_set)
{
    eval_t ev[MAXC];
    const int K = ref_num_candidates(order);
    if (K == 0 || !f || forced >= K) return REF_EINVAL;
    eval_candidates(order, f, mag, ev);
    int chosen, near;
    unsigned set;
    decide(ev, K, delta, &chosen, &near, &set);
    int status = REF_OK;
    if (forced >= 0 && forced != chosen) {
        if (set & (1u << forced)) chosen = forced;
        else status = REF_EMISMATCH;
    }
    if (fhat) *fhat = ev[chosen].flux;
    if (sel) *sel = chosen;
    if (tie) *tie = near;
    if (tie_set) *tie_set = set;
    return status;
}

int ref_indicator_scales(int order, const double *f, const double *mag, double *scale_k)
{
    eval_t ev[MAXC];
    const int K = ref_num_candidates(order);
    if (K == 0 || !f || !scale_k) return REF_EINVAL;
    eval_candidates(order, f, mag, ev);
    for (int k = 0; k < K; ++k) scale_k[k] = ev[k].s;
    return REF_OK;
}
