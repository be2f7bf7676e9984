// enoao_device.hpp -- per-face arithmetic of the ENO-AO method on gfx950.
//
// Everything here runs in registers of one lane: one lane owns one face.
//   * recon<ORDER>: one side of the reconstruction of Section 3.2 -- the
//     minimum-discrepancy indicators IS = min(delta_L, delta_R) of
//     Eq. (New_Smoothness_Indicator) in the closed forms of Tables DeltaL /
//     DeltaR, the reconstruction principle, and the selected row of the table
//     of numerical fluxes.
//   * Roe-state characteristic projection for the Euler systems (Section 4:
//     Roe average at the face for the characteristic decomposition).
//
// Implementation notes (same arithmetic as the paper, laid out for the VALU):
//   * the undivided differences of all candidates come from one difference
//     table (20 subtractions for order 5 instead of the literal rows); two
//     candidates whose delta rows coincide share one entry, so their indicators
//     are bitwise equal as the rows are;
//   * the two principles are evaluated branch-free: candidate k wins over the
//     candidates below it when IS_k <= delta, or when no lower candidate had
//     IS <= delta and IS_k <= min(lower IS); the last winner is the choice.
//     This is the highest-priority candidate with IS <= delta if any, else the
//     highest-priority one among the smallest indicators;
//   * only the chosen candidate's flux is evaluated, as a dot product of the
//     window with that row of the flux table (rows held in LDS);
//   * a window may be scaled by a power of two before reconstruction (the
//     factor 1/2 of the splitting is applied after it); scaling by 2^k is
//     exact, so indicators, comparisons and selections are unchanged when delta
//     is scaled alike.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace enoao {

// Wave-uniform early exit: when every lane of the wave has IS <= delta for the
// highest-priority candidate on both sides of a field, that candidate is every
// lane's choice (first principle), so the selection logic is skipped.  Each
// lane's result is bitwise the same as on the full path (same indicators, same
// row); only the work differs.
#ifndef ENOAO_EARLY_EXIT
#define ENOAO_EARLY_EXIT 1
#endif

// true when the predicate holds on every active lane of the wave (one ballot)
__device__ __forceinline__ bool wave_all(bool p) { return __builtin_amdgcn_ballot_w64(!p) == 0; }

template <int ORDER> struct ReconTraits;
template <> struct ReconTraits<5> { static constexpr int H = 3, K = 6; };
template <> struct ReconTraits<7> { static constexpr int H = 4, K = 9; };

// Rows of the table of numerical fluxes (Table "Flux_reconstruction") as
// weights on the whole window, candidates in increasing priority; row stride
// TW doubles (16-byte aligned).  The kernels copy the rows to LDS and each lane
// evaluates only its selected row.
template <int ORDER> struct FluxRows;
template <> struct FluxRows<5> {
    static constexpr int TW = 8;
    // window f_{j-3} .. f_{j+3}
    static constexpr double num[6][7] = {
        {0, 0, 0, 1, 0, 0, 0},        {0, 0, 0, 1, 1, 0, 0},       {0, 0, -1, 5, 2, 0, 0},
        {0, 1, -5, 13, 3, 0, 0},      {0, 0, -1, 7, 7, -1, 0},     {0, 2, -13, 47, 27, -3, 0}};
    static constexpr double den[6] = {1, 2, 6, 12, 12, 60};
};
template <> struct FluxRows<7> {
    static constexpr int TW = 10;
    // window f_{j-4} .. f_{j+4}
    static constexpr double num[9][9] = {
        {0, 0, 0, 0, 1, 0, 0, 0, 0},          {0, 0, 0, 0, 1, 1, 0, 0, 0},
        {0, 0, 0, -1, 5, 2, 0, 0, 0},         {0, 0, 1, -5, 13, 3, 0, 0, 0},
        {0, 0, 0, -1, 7, 7, -1, 0, 0},        {0, 0, 2, -13, 47, 27, -3, 0, 0},
        {0, -1, 7, -23, 57, 22, -2, 0, 0},    {0, 0, 1, -8, 37, 37, -8, 1, 0},
        {0, -3, 25, -101, 319, 214, -38, 4, 0}};
    static constexpr double den[9] = {1, 2, 6, 12, 12, 60, 60, 60, 420};
};

// Fill the LDS copy of the flux rows (weights num/den), all threads of a block.
template <int ORDER> __device__ __forceinline__ void load_flux_rows(double *tab)
{
    using R = FluxRows<ORDER>;
    constexpr int K = ReconTraits<ORDER>::K, W = 2 * ReconTraits<ORDER>::H + 1;
    for (int i = threadIdx.x; i < K * R::TW; i += blockDim.x) {
        const int k = i / R::TW, t = i % R::TW;
        tab[i] = t < W ? R::num[k][t] / R::den[k] : 0.0;
    }
}

// Two principles of Section 3.2 on the indicators is[0..K-1] (increasing
// priority): the highest-priority candidate with IS <= delta if there is one,
// else the last minimum.  The comparisons produce lane masks; the logic between
// them stays in scalar registers, the lane's index is one select per candidate.
template <int K>
__device__ __forceinline__ int select_candidate(const double (&is)[K], double delta)
{
    int s = 0;
    bool any = is[0] <= delta;
    double mn = is[0];
#pragma unroll
    for (int k = 1; k < K; ++k) {
        const bool le = is[k] <= delta;
        const bool win = le || (!any && is[k] <= mn);
        s = win ? k : s;
        any = any || le;
        mn = fmin(mn, is[k]);
    }
    return s;
}

// selected flux: one row of the table, as a dot product with the window
template <int W, int TW>
__device__ __forceinline__ double row_dot(const double (&f)[W], const double *tab, int s)
{
    const double *r = tab + s * TW;
    double q = r[0] * f[0];
#pragma unroll
    for (int t = 1; t < W; ++t) q = fma(r[t], f[t], q);
    return q;
}

// Indicators of all candidates of one window, in increasing priority.
// Order 5: f[0..6] = f_{j-3} .. f_{j+3}; candidates 0: S_j^j, 1: S_j^{j+1},
// 2: S_{j-1}^{j+1}, 3: S_{j-2}^{j+1}, 4: S_{j-1}^{j+2}, 5: S_{j-2}^{j+2}.
// Order 7: f[0..8] = f_{j-4} .. f_{j+4}; then 6: S_{j-3}^{j+2},
// 7: S_{j-2}^{j+3}, 8: S_{j-3}^{j+3}.
// delta_L / delta_R of every candidate are entries of one difference table
// (level k holds the k-th undivided differences); rows shared by two
// candidates are one entry.
__device__ __forceinline__ void indicators5(const double (&f)[7], double (&is)[6])
{
    const double a0 = f[1] - f[0], a1 = f[2] - f[1], a2 = f[3] - f[2];
    const double a3 = f[4] - f[3], a4 = f[5] - f[4], a5 = f[6] - f[5];
    const double b0 = a1 - a0, b1 = a2 - a1, b2 = a3 - a2, b3 = a4 - a3, b4 = a5 - a4;
    const double c0 = b1 - b0, c1 = b2 - b1, c2 = b3 - b2, c3 = b4 - b3;
    const double d0 = c1 - c0, d1 = c2 - c1, d2 = c3 - c2;
    const double e0 = d1 - d0, e1 = d2 - d1;
    const double ad1 = fabs(d1);
    is[0] = 0.5 * fmin(fabs(a2) + fabs(a1), fabs(a3) + fabs(a4)); // S_j^j (averaged form)
    is[1] = fmin(fabs(b2), fabs(b3));                              // S_j^{j+1}
    is[2] = fmin(fabs(c1), fabs(c2));                              // S_{j-1}^{j+1}
    is[3] = fmin(fabs(d0), ad1);                                   // S_{j-2}^{j+1}
    is[4] = fmin(ad1, fabs(d2));                                   // S_{j-1}^{j+2}
    is[5] = fmin(fabs(e0), fabs(e1));                              // S_{j-2}^{j+2}
}

__device__ __forceinline__ void indicators7(const double (&f)[9], double (&is)[9])
{
    double a[8], b[7], c[6], d[5], e[4], g[3], h[2];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = f[i + 1] - f[i];
#pragma unroll
    for (int i = 0; i < 7; ++i) b[i] = a[i + 1] - a[i];
#pragma unroll
    for (int i = 0; i < 6; ++i) c[i] = b[i + 1] - b[i];
#pragma unroll
    for (int i = 0; i < 5; ++i) d[i] = c[i + 1] - c[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) e[i] = d[i + 1] - d[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) g[i] = e[i + 1] - e[i];
#pragma unroll
    for (int i = 0; i < 2; ++i) h[i] = g[i + 1] - g[i];
    const double ad2 = fabs(d[2]), ag1 = fabs(g[1]);
    is[0] = 0.5 * fmin(fabs(a[3]) + fabs(a[2]), fabs(a[4]) + fabs(a[5])); // S_j^j
    is[1] = fmin(fabs(b[3]), fabs(b[4]));                                  // S_j^{j+1}
    is[2] = fmin(fabs(c[2]), fabs(c[3]));                                  // S_{j-1}^{j+1}
    is[3] = fmin(fabs(d[1]), ad2);                                         // S_{j-2}^{j+1}
    is[4] = fmin(ad2, fabs(d[3]));                                         // S_{j-1}^{j+2}
    is[5] = fmin(fabs(e[1]), fabs(e[2]));                                  // S_{j-2}^{j+2}
    is[6] = fmin(fabs(g[0]), ag1);                                         // S_{j-3}^{j+2}
    is[7] = fmin(ag1, fabs(g[2]));                                         // S_{j-2}^{j+3}
    is[8] = fmin(fabs(h[0]), fabs(h[1]));                                  // S_{j-3}^{j+3}
}

template <int ORDER> struct Recon {
    static constexpr int H = ReconTraits<ORDER>::H, K = ReconTraits<ORDER>::K, W = 2 * H + 1;
    __device__ __forceinline__ static void indicators(const double (&f)[W], double (&is)[K])
    {
        if constexpr (ORDER == 5) indicators5(f, is);
        else indicators7(f, is);
    }
    // One side of one field: the chosen candidate's value at x_{j+1/2}.  The
    // wave skips the other indicators and the selection when every lane's top
    // candidate has IS <= delta.
    __device__ __forceinline__ static double run(const double (&f)[W], double delta, const double *tab, int &sel)
    {
        if constexpr (ORDER == 5) {
            const double a0 = f[1] - f[0], a1 = f[2] - f[1], a2 = f[3] - f[2];
            const double a3 = f[4] - f[3], a4 = f[5] - f[4], a5 = f[6] - f[5];
            const double b0 = a1 - a0, b1 = a2 - a1, b2 = a3 - a2, b3 = a4 - a3, b4 = a5 - a4;
            const double c0 = b1 - b0, c1 = b2 - b1, c2 = b3 - b2, c3 = b4 - b3;
            const double d0 = c1 - c0, d1 = c2 - c1, d2 = c3 - c2;
            const double e0 = d1 - d0, e1 = d2 - d1;
            const double is_top = fmin(fabs(e0), fabs(e1));  // S_{j-2}^{j+2}
            if (ENOAO_EARLY_EXIT && wave_all(is_top <= delta)) {
                sel = 5;
                return row_dot<W, FluxRows<5>::TW>(f, tab, 5);
            }
            const double ad1 = fabs(d1);
            double is[6];
            is[0] = 0.5 * fmin(fabs(a2) + fabs(a1), fabs(a3) + fabs(a4)); // S_j^j (averaged form)
            is[1] = fmin(fabs(b2), fabs(b3));                              // S_j^{j+1}
            is[2] = fmin(fabs(c1), fabs(c2));                              // S_{j-1}^{j+1}
            is[3] = fmin(fabs(d0), ad1);                                   // S_{j-2}^{j+1}
            is[4] = fmin(ad1, fabs(d2));                                   // S_{j-1}^{j+2}
            is[5] = is_top;
            sel = select_candidate<6>(is, delta);
        } else {
            double is[9];
            indicators7(f, is);
            if (ENOAO_EARLY_EXIT && wave_all(is[8] <= delta)) {
                sel = 8;
                return row_dot<W, FluxRows<7>::TW>(f, tab, 8);
            }
            sel = select_candidate<9>(is, delta);
        }
        return row_dot<W, FluxRows<ORDER>::TW>(f, tab, sel);
    }
};

// ---------------------------------------------------------------------------
// Per-node quantities staged in LDS (computed once per node by the lane that
// loads it; faces read them from LDS).
//   advection: u
//   Euler 1D : rho, m, E | F0..F2 | sqrt(rho), u, H
//   Euler 2D : rho, m, n, E | F0..F3 | sqrt(rho), u, v, H
// (for a y-sweep the two momentum components arrive exchanged, so the same
//  x-direction formulas give the y-flux in exchanged order).
// 1/x for positive normal x: hardware reciprocal refined by two Newton steps
// (within an ulp or so; the kernels' reciprocals and quotients are rounding-level
// different from IEEE division).
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

template <int EQ> struct NodeTraits;
template <> struct NodeTraits<ADVECTION> { static constexpr int NC = 1, NQ = 1; };
template <> struct NodeTraits<EULER1D> { static constexpr int NC = 3, NQ = 9; };
template <> struct NodeTraits<EULER2D> { static constexpr int NC = 4, NQ = 12; };

// Returns false for a non-physical node (rho <= 0, p <= 0 or NaN).
template <int EQ>
__device__ __forceinline__ bool node_quantities(const double (&U)[NodeTraits<EQ>::NC], double gm1,
                                                double (&q)[NodeTraits<EQ>::NQ])
{
    if constexpr (EQ == ADVECTION) {
        q[0] = U[0];
        return U[0] == U[0];
    } else if constexpr (EQ == EULER1D) {
        const double rho = U[0], m = U[1], E = U[2];
        const double ir = rcp_nr(rho);
        const double u = m * ir;
        const double p = gm1 * (E - 0.5 * rho * (u * u));
        q[0] = rho; q[1] = m; q[2] = E;
        q[3] = m; q[4] = fma(m, u, p); q[5] = (E + p) * u;
        q[6] = sqrt(rho); q[7] = u; q[8] = (E + p) * ir;
        return rho > 0.0 && p > 0.0;
    } else {
        const double rho = U[0], m = U[1], n = U[2], E = U[3];
        const double ir = rcp_nr(rho);
        const double u = m * ir, v = n * ir;
        const double p = gm1 * (E - 0.5 * rho * fma(u, u, v * v));
        q[0] = rho; q[1] = m; q[2] = n; q[3] = E;
        q[4] = m; q[5] = fma(m, u, p); q[6] = m * v; q[7] = (E + p) * u;
        q[8] = sqrt(rho); q[9] = u; q[10] = v; q[11] = (E + p) * ir;
        return rho > 0.0 && p > 0.0;
    }
}

// Roe state of the two nodes adjacent to a face, with the factors of the
// characteristic projection.
struct RoeState {
    double u, v, H, c, ic, b1, b2, q2h;
};

__device__ __forceinline__ RoeState roe_state(double sL, double uL, double vL, double HL, double sR,
                                              double uR, double vR, double HR, double gm1)
{
    RoeState r;
    const double iw = rcp_nr(sL + sR);
    const double wL = sL * iw, wR = sR * iw;
    r.u = fma(wL, uL, wR * uR);
    r.v = fma(wL, vL, wR * vR);
    r.H = fma(wL, HL, wR * HR);
    r.q2h = 0.5 * fma(r.u, r.u, r.v * r.v);
    const double c2 = gm1 * (r.H - r.q2h);
    r.c = sqrt(c2);
    r.ic = rcp_nr(r.c);
    r.b1 = gm1 * r.ic * r.ic;
    r.b2 = r.q2h * r.b1;
    return r;
}

// Projection of a conserved-variable vector x on the left eigenvectors of the
// Roe state (right eigenvectors with unit first component):
//   2D: rows l0 = (b2+u/c, -b1 u-1/c, -b1 v, b1)/2, l1 = (1-b2, b1 u, b1 v, -b1),
//       l2 = (-v, 0, 1, 0), l3 = (b2-u/c, -b1 u+1/c, -b1 v, b1)/2
//   1D: the same without the v entries and without l2.
// Output scaled by (2, 1, 1, 2) in 2D and (2, 1, 2) in 1D: with
// A = b2 x0 - b1 (u x1 + v x2 - x3) and B = (u x0 - x1)/c,
// 2 l0.x = A + B, l1.x = x0 - A, l2.x = x2 - v x0, 2 l3.x = A - B.
template <int NC>
__device__ __forceinline__ void project(const RoeState &r, const double (&x)[NC], double (&w)[NC])
{
    if constexpr (NC == 4) {
        const double t = fma(r.u, x[1], fma(r.v, x[2], -x[3]));
        const double A = fma(r.b2, x[0], -r.b1 * t);
        const double B = fma(r.u, x[0], -x[1]) * r.ic;
        w[0] = A + B;
        w[1] = x[0] - A;
        w[2] = fma(-r.v, x[0], x[2]);
        w[3] = A - B;
    } else {
        const double t = fma(r.u, x[1], -x[2]);
        const double A = fma(r.b2, x[0], -r.b1 * t);
        const double B = fma(r.u, x[0], -x[1]) * r.ic;
        w[0] = A + B;
        w[1] = x[0] - A;
        w[2] = A - B;
    }
}

// scale of field s after project(): 2 for the acoustic fields, 1 otherwise
template <int NC> __device__ __forceinline__ constexpr double field_scale(int s)
{
    return (s == 0 || s == NC - 1) ? 2.0 : 1.0;
}

// Back to conserved variables: Fhat = R what, R columns (2D)
//   (1, u-c, v, H-uc), (1, u, v, q^2/2), (0, 0, 1, v), (1, u+c, v, H+uc)
// (1D: the same without v and without the third column).
template <int NC>
__device__ __forceinline__ void back_project(const RoeState &r, const double (&w)[NC], double (&F)[NC])
{
    if constexpr (NC == 4) {
        const double s03 = w[0] + w[3], d30 = w[3] - w[0];
        F[0] = s03 + w[1];
        F[1] = fma(r.u, F[0], r.c * d30);
        F[2] = fma(r.v, F[0], w[2]);
        F[3] = fma(r.H, s03, fma(r.u * r.c, d30, fma(r.q2h, w[1], r.v * w[2])));
    } else {
        const double s02 = w[0] + w[2], d20 = w[2] - w[0];
        F[0] = s02 + w[1];
        F[1] = fma(r.u, F[0], r.c * d20);
        F[2] = fma(r.H, s02, fma(r.u * r.c, d20, r.q2h * w[1]));
    }
}

}  // namespace enoao
