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
//   * the candidate fluxes of the table of numerical fluxes are taken in
//     Newton form on the same difference table: each candidate's row equals a
//     lower candidate's row plus a rational multiple of one undivided
//     difference (an exact identity of the table's rows, e.g. for order 5
//     S_{j-1}^{j+1} = S_j^{j+1} - 1/6 (f_{j+1} - 2 f_j + f_{j-1})), so all
//     candidates cost one multiply-add each and the chosen one is selected
//     with the index, without a table in memory;
//   * the top candidate also has a conserved-variable form (TopStencil): its
//     indicators and the sum of its two one-sided values are linear in the
//     window, so differences and a symmetric stencil of U and F are formed
//     first and projected on the characteristic fields afterwards;
//   * a window may be scaled by a power of two before reconstruction (the
//     factor 1/2 of the splitting is applied after it); scaling by 2^k is
//     exact, so indicators, comparisons and selections are unchanged when delta
//     is scaled alike.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Floating-point contraction is off from here on (the kernels include this
// header first): a multiply and an add are fused only where an fma() says so.
// Every inlined copy of the same arithmetic then rounds alike, which the
// kernels rely on: a value formed on two code paths, or in two kernels, agrees
// bit for bit.
#pragma clang fp contract(off)

namespace enoao {

// Wave-uniform shortcut: when every lane of the wave has IS <= delta for the
// top candidate on both sides of a field, that candidate is every lane's choice
// (first principle) and the field's value is the top candidate's alone;
// otherwise the field takes the full selection.  A lane's result does not
// depend on the path: the full selection uses the same top indicator and, when
// it picks the top candidate on both sides, the same value.  The kernels take
// a flag that turns the shortcut off (every face takes the full selection), so
// that property can be checked.

// true when the predicate holds on every active lane of the wave (one ballot)
__device__ __forceinline__ bool wave_all(bool p) { return __builtin_amdgcn_ballot_w64(!p) == 0; }

template <int ORDER> struct ReconTraits;
template <> struct ReconTraits<5> { static constexpr int H = 3, K = 6; };
template <> struct ReconTraits<7> { static constexpr int H = 4, K = 9; };

// Two principles of Section 3.2 on the indicators is[0..K-1] (increasing
// priority): the highest-priority candidate with IS <= delta if there is one,
// else the last minimum.  The comparisons produce lane masks; the logic between
// them stays in scalar registers, the lane's index and flux are one select each
// per candidate.
template <int K>
__device__ __forceinline__ double select_candidate(const double (&is)[K], const double (&h)[K], double delta,
                                                   int &sel)
{
    int s = 0;
    double v = h[0];
    bool any = is[0] <= delta;
    double mn = is[0];
#pragma unroll
    for (int k = 1; k < K; ++k) {
        const bool le = is[k] <= delta;
        const bool win = le || (!any && is[k] <= mn);
        s = win ? k : s;
        v = win ? h[k] : v;
        any = any || le;
        mn = fmin(mn, is[k]);
    }
    sel = s;
    return v;
}

// Candidates of one window, in increasing priority.
// Order 5: f[0..6] = f_{j-3} .. f_{j+3}; candidates 0: S_j^j, 1: S_j^{j+1},
// 2: S_{j-1}^{j+1}, 3: S_{j-2}^{j+1}, 4: S_{j-1}^{j+2}, 5: S_{j-2}^{j+2}.
// Order 7: f[0..8] = f_{j-4} .. f_{j+4}; then 6: S_{j-3}^{j+2},
// 7: S_{j-2}^{j+3}, 8: S_{j-3}^{j+3}.
// delta_L / delta_R of every candidate are entries of one difference table
// (level k holds the k-th undivided differences); rows shared by two
// candidates are one entry.
template <int ORDER> struct Recon {
    static constexpr int H = ReconTraits<ORDER>::H, K = ReconTraits<ORDER>::K, W = 2 * H + 1;
    // One side of one field: the chosen candidate's value at x_{j+1/2} and its
    // index, by the two principles.  The top candidate's indicator is_top is
    // given (it comes from the conserved-variable form below, so every path
    // takes the same decision on it).  Candidate values (the table of
    // numerical fluxes) in Newton form:
    //   order 5 (f_j = f[3]):  h0 = f_j, h1 = h0 + a3/2, h2 = h1 - b2/6,
    //     h3 = h2 - c1/12, h4 = h2 - c2/12, h5 = h3 - d1/20;
    //   order 7 (f_j = f[4]): the same on the shifted table, then
    //     h6 = h5 + e1/60, h7 = h5 + e2/60, h8 = h6 + g1/105,
    // (a, b, c, ... the 1st, 2nd, 3rd ... undivided differences, index = first
    // node).
    __device__ __forceinline__ static double select(const double (&f)[W], double delta, double is_top, int &sel)
    {
        if constexpr (ORDER == 5) {
            const double a0 = f[1] - f[0], a1 = f[2] - f[1], a2 = f[3] - f[2];
            const double a3 = f[4] - f[3], a4 = f[5] - f[4], a5 = f[6] - f[5];
            const double b1 = a2 - a1, b2 = a3 - a2, b3 = a4 - a3;
            const double c0 = b1 - (a1 - a0), c1 = b2 - b1, c2 = b3 - b2, c3 = (a5 - a4) - b3;
            const double d0 = c1 - c0, d1 = c2 - c1, d2 = c3 - c2;
            double h[6];
            h[0] = f[3];
            h[1] = fma(0.5, a3, h[0]);
            h[2] = fma(-1.0 / 6.0, b2, h[1]);
            h[3] = fma(-1.0 / 12.0, c1, h[2]);
            h[4] = fma(-1.0 / 12.0, c2, h[2]);
            h[5] = fma(-1.0 / 20.0, d1, h[3]);
            const double ad1 = fabs(d1);
            double is[6];
            is[0] = 0.5 * fmin(fabs(a2) + fabs(a1), fabs(a3) + fabs(a4)); // S_j^j (averaged form)
            is[1] = fmin(fabs(b2), fabs(b3));                              // S_j^{j+1}
            is[2] = fmin(fabs(c1), fabs(c2));                              // S_{j-1}^{j+1}
            is[3] = fmin(fabs(d0), ad1);                                   // S_{j-2}^{j+1}
            is[4] = fmin(ad1, fabs(d2));                                   // S_{j-1}^{j+2}
            is[5] = is_top;                                                // S_{j-2}^{j+2}
            return select_candidate<6>(is, h, delta, sel);
        } else {
            double a[8], b[7], c[6], d[5], e[4], g[3];
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
            double h[9];
            h[0] = f[4];
            h[1] = fma(0.5, a[4], h[0]);
            h[2] = fma(-1.0 / 6.0, b[3], h[1]);
            h[3] = fma(-1.0 / 12.0, c[2], h[2]);
            h[4] = fma(-1.0 / 12.0, c[3], h[2]);
            h[5] = fma(-1.0 / 20.0, d[2], h[3]);
            h[6] = fma(1.0 / 60.0, e[1], h[5]);
            h[7] = fma(1.0 / 60.0, e[2], h[5]);
            h[8] = fma(1.0 / 105.0, g[1], h[6]);
            const double ad2 = fabs(d[2]), ag1 = fabs(g[1]);
            double is[9];
            is[0] = 0.5 * fmin(fabs(a[3]) + fabs(a[2]), fabs(a[4]) + fabs(a[5])); // S_j^j
            is[1] = fmin(fabs(b[3]), fabs(b[4]));                                  // S_j^{j+1}
            is[2] = fmin(fabs(c[2]), fabs(c[3]));                                  // S_{j-1}^{j+1}
            is[3] = fmin(fabs(d[1]), ad2);                                         // S_{j-2}^{j+1}
            is[4] = fmin(ad2, fabs(d[3]));                                         // S_{j-1}^{j+2}
            is[5] = fmin(fabs(e[1]), fabs(e[2]));                                  // S_{j-2}^{j+2}
            is[6] = fmin(fabs(g[0]), ag1);                                         // S_{j-3}^{j+2}
            is[7] = fmin(ag1, fabs(g[2]));                                         // S_{j-2}^{j+3}
            is[8] = is_top;                                                        // S_{j-3}^{j+3}
            return select_candidate<9>(is, h, delta, sel);
        }
    }
};

// The top candidate (S_{j-2}^{j+2}, order 7: S_{j-3}^{j+3}) in conserved
// variables.  Its indicator and the sum of its values on the two sides are
// linear in the window, and so is the characteristic projection, so they can be
// formed on U and F once per node or face and projected afterwards.  Over a
// face's 2G nodes x_0 .. x_{2H+1}:
//   * D_p = (2H-1)-th undivided difference starting at node p:
//       order 5: (x5 - x0) + 5 (x1 - x4) + 10 (x3 - x2)            (shifted by p)
//       order 7: (x7 - x0) + 7 (x1 - x6) + 21 (x5 - x2) + 35 (x3 - x4)
//     plus side (window nodes 0 .. 2H):      IS_top = min(|D_0 g+|, |D_1 g+|);
//     minus side (mirror, nodes 2H+1 .. 1):  IS_top = min(|D_2 g-|, |D_1 g-|)
//     (reversing a window only flips the sign of an odd difference).
//   * plus value + minus value = S F + alpha kappa D_1 U, with the symmetric
//     stencil S in terms of the pair sums s_k = x_{H-k} + x_{H+1+k}:
//       order 5: S = s0 - 7/30 (s1 - s0) + 1/30 (s2 - s1),                   kappa = -1/30
//       order 7: S = s0 - 113/420 (s1 - s0) + 13/210 (s2 - s1) - 1/140 (s3 - s2), kappa = 1/140
//     (one-sided values 2,-13,47,27,-3 / 60 and -3,25,-101,319,214,-38,4 / 420
//     of the Newton forms above; their mirror difference is kappa D_1).
// Constant data give exactly zero differences and corrections.
template <int ORDER> struct TopStencil {
    static constexpr int H = ReconTraits<ORDER>::H;
    static constexpr double kappa = ORDER == 5 ? -1.0 / 30.0 : 1.0 / 140.0;
    // D starting at x[0], nodes x[0], x[ns], ...
    __device__ __forceinline__ static double diff(const double *x, int ns)
    {
        if constexpr (ORDER == 5) {
            const double r = fma(5.0, x[ns] - x[4 * ns], x[5 * ns] - x[0]);
            return fma(10.0, x[3 * ns] - x[2 * ns], r);
        } else {
            double r = fma(7.0, x[ns] - x[6 * ns], x[7 * ns] - x[0]);
            r = fma(21.0, x[5 * ns] - x[2 * ns], r);
            return fma(35.0, x[3 * ns] - x[4 * ns], r);
        }
    }
    // S over a face's nodes, x[0] = node 0
    __device__ __forceinline__ static double sym(const double *x, int ns)
    {
        const double s0 = x[H * ns] + x[(H + 1) * ns], s1 = x[(H - 1) * ns] + x[(H + 2) * ns];
        const double s2 = x[(H - 2) * ns] + x[(H + 3) * ns];
        if constexpr (ORDER == 5) {
            return fma(1.0 / 30.0, s2 - s1, fma(-7.0 / 30.0, s1 - s0, s0));
        } else {
            const double s3 = x[(H - 3) * ns] + x[(H + 4) * ns];
            double r = fma(-113.0 / 420.0, s1 - s0, s0);
            r = fma(13.0 / 210.0, s2 - s1, r);
            return fma(-1.0 / 140.0, s3 - s2, r);
        }
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

// sqrt(x) for positive normal x: hardware reciprocal square root refined by
// Goldschmidt's coupled iteration for sqrt(x) and 1/(2 sqrt(x)), with two
// Newton corrections of the root.  The compiler's sqrt takes the same steps
// plus a range scaling and special-value selects, which the kernels' operands
// (densities, squared sound speeds of physical states) never need; on them the
// results agree bit for bit.
__device__ __forceinline__ double sqrt_nr(double x)
{
    const double r = __builtin_amdgcn_rsq(x);
    double y = x * r;
    double h = 0.5 * r;
    const double e = fma(-h, y, 0.5);
    y = fma(y, e, y);
    h = fma(h, e, h);
    double d = fma(-y, y, x);
    y = fma(d, h, y);
    d = fma(-y, y, x);
    return fma(d, h, y);
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
        const double p = gm1 * fma(-0.5 * rho, u * u, E);
        q[0] = rho; q[1] = m; q[2] = E;
        q[3] = m; q[4] = fma(m, u, p); q[5] = (E + p) * u;
        q[6] = sqrt_nr(rho); q[7] = u; q[8] = (E + p) * ir;
        return rho > 0.0 && p > 0.0;
    } else {
        const double rho = U[0], m = U[1], n = U[2], E = U[3];
        const double ir = rcp_nr(rho);
        const double u = m * ir, v = n * ir;
        const double p = gm1 * fma(-0.5 * rho, fma(u, u, v * v), E);
        q[0] = rho; q[1] = m; q[2] = n; q[3] = E;
        q[4] = m; q[5] = fma(m, u, p); q[6] = m * v; q[7] = (E + p) * u;
        q[8] = sqrt_nr(rho); q[9] = u; q[10] = v; q[11] = (E + p) * ir;
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
    r.c = sqrt_nr(c2);
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
        const double Bc = fma(r.u, x[0], -x[1]);  // B c
        w[0] = fma(Bc, r.ic, A);
        w[1] = x[0] - A;
        w[2] = fma(-r.v, x[0], x[2]);
        w[3] = fma(-Bc, r.ic, A);
    } else {
        const double t = fma(r.u, x[1], -x[2]);
        const double A = fma(r.b2, x[0], -r.b1 * t);
        const double Bc = fma(r.u, x[0], -x[1]);  // B c
        w[0] = fma(Bc, r.ic, A);
        w[1] = x[0] - A;
        w[2] = fma(-Bc, r.ic, A);
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
