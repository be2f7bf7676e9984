// enoao_kernels.hip -- gfx950 kernels of the ENO-AO path.
//
// Per Runge-Kutta stage (Section 2: conservative finite differences, global
// Lax-Friedrichs splitting, third-order TVD Runge-Kutta; Section 3: ENO-AO
// reconstruction; Section 4: Roe characteristic decomposition):
//   1D:  sweep_x<STAGE s>   tile load + BC -> per-node flux and Roe inputs in
//        LDS -> one lane per face: projection, split, indicators, selection,
//        candidate flux, back-projection -> flux difference -> RK stage
//        combine -> per-field maxima of the new state for the next stage.
//   2D:  sweep_x<STAGE s> writes the x-part of L; sweep_y<STAGE s> adds the
//        y-part (dimension by dimension, both on the same stage state) and
//        does the RK combine and the maxima.
// Kernels are persistent: a grid of (CUs x occupancy) workgroups walks a
// contiguous chunk of the flattened tile list of all instances of a batch.
// Every face takes each field's top candidate in conserved-variable form and
// runs the full selection only for the fields of a wave that need it (the
// x-sweeps stage the top differences per node pair in LDS; the y-sweep and the
// LDS-resident solver form them per face, which their LDS budgets require).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "enoao_common.hpp"
#include "enoao_device.hpp"
#include "enoao_kernels.hpp"

// Tuning switches (defaults are the measured best on gfx950).
#ifndef ENOAO_NODE_PREFETCH
#define ENOAO_NODE_PREFETCH 1  // stencil nodes whose LDS reads are in flight ahead of use
#endif
#ifndef ENOAO_NODE_SCHED
#define ENOAO_NODE_SCHED 1     // stencil nodes between scheduling fences (0: none; bounds register use)
#endif

namespace enoao {

// Workgroups sharing a persistent launch's tile list of T tiles: the whole
// grid, or for a pool as many as give P.tiles_per_wg tiles each (at least
// P.grid_min, at most the grid).  A pool's grid covers the machine several
// times over; many small chunks let the workgroups that finish early take
// more of them, which evens out members of uneven cost, while a pool holding
// few tiles keeps chunks long enough for the y walks' row reuse.
__device__ __forceinline__ long long chunk_groups(const KParams &P, long long T)
{
    const long long g = gridDim.x;
    if (P.tiles_per_wg <= 0) return g;
    return min(g, max((long long)P.grid_min, T / P.tiles_per_wg));
}

__device__ __forceinline__ int bc_map(int k, int n, int bc)
{
    if (bc == BC_PERIODIC) {
        int r = k % n;
        return r < 0 ? r + n : r;
    }
    return k < 0 ? 0 : (k >= n ? n - 1 : k);
}

// Device-memory pointers.  The state and control pointers reach a kernel through
// the instance table in memory, so the compiler cannot tell that they address
// global memory and would emit flat instructions for them.  Flat loads and
// stores count against the LDS counter too, so every wait for an LDS read would
// also wait for the next tile's global prefetch in flight (and for the previous
// tile's stores).  Typed as global they compile to global instructions.
#define GMEM __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ GMEM T *gmem(T *p) { return (GMEM T *)p; }

// wave-uniform copy of a value (scalar registers)
template <typename T> __device__ __forceinline__ T uniform(T x)
{
    static_assert(sizeof(T) % 4 == 0, "32-bit multiple");
    union { T v; int w[sizeof(T) / 4]; } a;
    a.v = x;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) a.w[i] = __builtin_amdgcn_readfirstlane(a.w[i]);
    return a.v;
}

__device__ __forceinline__ double as_double(unsigned long long b) { return __longlong_as_double((long long)b); }
__device__ __forceinline__ unsigned long long as_bits(double d) { return (unsigned long long)__double_as_longlong(d); }

template <bool X>
__device__ __forceinline__ int find_inst(const Inst *inst, int n, long long tile)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const long long t0 = X ? inst[mid].xtile0 : inst[mid].ytile0;
        if (t0 <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Maxima of the per-field wave speeds of a state (for alpha of the next
// evaluation and for the CFL step), and the non-physical flag.
template <int EQ> struct Maxima {
    static constexpr int NV = EQ == EULER2D ? 7 : (EQ == EULER1D ? 3 : 0);  // values in use
    double v[7];
    int bad;
    __device__ void reset()
    {
#pragma unroll
        for (int i = 0; i < 7; ++i) v[i] = 0.0;
        bad = 0;
    }
    // U in the natural component order; idx, idy = 1/dx, 1/dy
    __device__ void add(const double *U, double gamma, double idx, double idy)
    {
        if constexpr (EQ == ADVECTION) {
            bad |= !(U[0] == U[0]);
        } else if constexpr (EQ == EULER1D) {
            const double rho = U[0], ir = rcp_nr(rho), u = U[1] * ir;
            const double p = (gamma - 1.0) * fma(-0.5 * rho, u * u, U[2]);
            const double c = sqrt_nr(gamma * p * ir);
            bad |= !(rho > 0.0 && p > 0.0);
            v[0] = fmax(v[0], fabs(u - c));
            v[1] = fmax(v[1], fabs(u));
            v[2] = fmax(v[2], fabs(u + c));
        } else {
            const double rho = U[0], ir = rcp_nr(rho), u = U[1] * ir, w = U[2] * ir;
            const double p = (gamma - 1.0) * fma(-0.5 * rho, fma(u, u, w * w), U[3]);
            const double c = sqrt_nr(gamma * p * ir);
            bad |= !(rho > 0.0 && p > 0.0);
            v[0] = fmax(v[0], fabs(u - c));
            v[1] = fmax(v[1], fabs(u));
            v[2] = fmax(v[2], fabs(u + c));
            v[3] = fmax(v[3], fabs(w - c));
            v[4] = fmax(v[4], fabs(w));
            v[5] = fmax(v[5], fabs(w + c));
            v[6] = fmax(v[6], fma(fabs(u) + c, idx, (fabs(w) + c) * idy));
        }
    }
    // workgroup reduction, then one atomic per value into the instance's slot
    __device__ void flush(GMEM unsigned long long *amax, GMEM Ctrl *ctrl, int slot, double *red)
    {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double x = v[i];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
            v[i] = x;
        }
        int b = bad;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) b |= __shfl_xor(b, o, 64);
        if (lane == 0) {
#pragma unroll
            for (int i = 0; i < NV; ++i) red[wave * 8 + i] = v[i];
            red[wave * 8 + 7] = (double)b;
        }
        __syncthreads();
        if (threadIdx.x < NV || threadIdx.x == 7) {
            double x = red[threadIdx.x];
            for (int w = 1; w < BLOCK / 64; ++w) x = fmax(x, red[w * 8 + threadIdx.x]);
            if (threadIdx.x < NV) {
                if (slot >= 0)
                    __hip_atomic_fetch_max(&amax[slot * AMAX_VALS + threadIdx.x], as_bits(x), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
            } else if (x != 0.0) {
                __hip_atomic_fetch_or(&ctrl->status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
        reset();
    }
};

// ---------------------------------------------------------------------------
// One face: window node t (t = 0 .. 2G-1) of face j+1/2 is node j-H+t; the
// plus side reads nodes j-H .. j+H, the minus side the mirror j+1+H .. j+1-H.

// Top candidate of every field of an Euler face in conserved-variable form
// (TopStencil): the projected differences D_0, D_1, D_2 of U and F and the
// projected symmetric stencil of F give both sides' top indicators and the sum
// of both sides' top values, on the window scale 2 field_scale (the windows
// below are g = P F +/- alpha P U with the scaled projection P).
// Reconstruction variables.  CH: the characteristic fields of the face's Roe
// state (Section 4), with the scaled projection and the field scales above;
// otherwise the conserved components themselves (identity projection, scale 1,
// and one alpha for all of them).
template <int NC, bool CH>
__device__ __forceinline__ void to_fields(const RoeState &r, const double (&x)[NC], double (&w)[NC])
{
    if constexpr (CH) {
        project<NC>(r, x, w);
    } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) w[c] = x[c];
    }
}

template <int NC, bool CH>
__device__ __forceinline__ void from_fields(const RoeState &r, const double (&w)[NC], double (&F)[NC])
{
    if constexpr (CH) {
        back_project<NC>(r, w, F);
    } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) F[c] = w[c];
    }
}

template <int NC, bool CH> __device__ __forceinline__ constexpr double fscale(int s)
{
    return CH ? field_scale<NC>(s) : 1.0;
}

template <int NC> struct TopForm {
    double is[NC][2];  // IS_top of the plus and minus side
    double hs[NC];     // plus + minus top value
};

// Staged differences (DSTAGED): d0 points at D_0 of quantity 0 of the face,
// quantities (U then F) dqs apart, positions dns apart.  Otherwise they are
// formed here from the window nodes.
template <int NC, int ORDER, bool DSTAGED, bool CH>
__device__ __forceinline__ void top_form(const double *w0, int qs, int ns, const double *d0, int dqs, int dns,
                                         const RoeState &r, const double *al, double delta, TopForm<NC> &tf)
{
    using T = TopStencil<ORDER>;
    constexpr int G = ReconTraits<ORDER>::H + 1;
    double dv[3][2][NC], sf[NC];
    if constexpr (DSTAGED) {
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int v = 0; v < 2; ++v)
#pragma unroll
                for (int c = 0; c < NC; ++c) dv[p][v][c] = d0[(v * NC + c) * dqs + p * dns];
#pragma unroll
        for (int c = 0; c < NC; ++c) sf[c] = T::sym(w0 + (NC + c) * qs, ns);
    } else {
        // one quantity's window at a time (bounds the live registers)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                double xw[2 * G];
#pragma unroll
                for (int t = 0; t < 2 * G; ++t) xw[t] = w0[(v * NC + c) * qs + t * ns];
#pragma unroll
                for (int p = 0; p < 3; ++p) dv[p][v][c] = T::diff(xw + p, 1);
                if (v == 1) sf[c] = T::sym(xw, 1);
                if (ENOAO_NODE_SCHED > 0 && c % 2 == 1) __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    double pd[3][2][NC], psf[NC];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int v = 0; v < 2; ++v) to_fields<NC, CH>(r, dv[p][v], pd[p][v]);
    to_fields<NC, CH>(r, sf, psf);
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        const double a = al[s];
        tf.is[s][0] = fmin(fabs(fma(a, pd[0][0][s], pd[0][1][s])), fabs(fma(a, pd[1][0][s], pd[1][1][s])));
        tf.is[s][1] = fmin(fabs(fma(-a, pd[2][0][s], pd[2][1][s])), fabs(fma(-a, pd[1][0][s], pd[1][1][s])));
        tf.hs[s] = fma(a * T::kappa, pd[1][0][s], psf[s]);
    }
}

// every lane of the wave has IS_top <= delta on both sides of field s
template <int NC, bool CH>
__device__ __forceinline__ bool top_wave_ok(const TopForm<NC> &tf, int s, double delta, bool shortcut)
{
    const double sd = 2.0 * fscale<NC, CH>(s) * delta;
    return wave_all(tf.is[s][0] <= sd && tf.is[s][1] <= sd) & shortcut;
}

// Full selection of the characteristic fields F0 (and F1 >= 0) of an Euler
// face: project U and F of every stencil node (the compiler drops the rows not
// used by these fields), split, select on both sides.  A field whose top
// candidate is within delta on every lane (bit s of okmask) keeps the top
// value; a lane whose selection takes the top candidate on both sides takes
// the same value, tf (the face's top form, formed once).  Taking the fields in
// two passes halves the live window registers.
template <int NC, int ORDER, int F0, int F1, bool CH>
__device__ __forceinline__ void field_pass(const double *w0, int qs, int ns, const RoeState &r, const double *al,
                                           double delta, int okmask, const TopForm<NC> &tf, double (&wh)[NC],
                                           int (&sel)[2 * NC])
{
    constexpr int H = ReconTraits<ORDER>::H, G = H + 1, W = 2 * H + 1, K = ReconTraits<ORDER>::K;
    constexpr int NF = F1 >= 0 ? 2 : 1;
    constexpr int fs[2] = {F0, F1 >= 0 ? F1 : F0};
    constexpr int pmask = (1 << F0) | (F1 >= 0 ? 1 << F1 : 0);
    double gp[NF][W], gm[NF][W];
    if ((okmask & pmask) != pmask) {
        // node t's LDS reads go out NODE_PREFETCH nodes ahead of its arithmetic
        constexpr int D = ENOAO_NODE_PREFETCH;
        double Uq[2 * G][NC], Fq[2 * G][NC];
#pragma unroll
        for (int t = 0; t < D && t < 2 * G; ++t) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                Uq[t][c] = w0[c * qs + t * ns];
                Fq[t][c] = w0[(NC + c) * qs + t * ns];
            }
        }
#pragma unroll
        for (int t = 0; t < 2 * G; ++t) {
            if (t + D < 2 * G) {
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    Uq[t + D][c] = w0[c * qs + (t + D) * ns];
                    Fq[t + D][c] = w0[(NC + c) * qs + (t + D) * ns];
                }
            }
            double PU[NC], PF[NC];
            to_fields<NC, CH>(r, Uq[t], PU);
            to_fields<NC, CH>(r, Fq[t], PF);
#pragma unroll
            for (int i = 0; i < NF; ++i) {
                const int s = fs[i];
                if (t < W) gp[i][t] = fma(al[s], PU[s], PF[s]);
                if (t >= 1) gm[i][2 * H + 1 - t] = fma(-al[s], PU[s], PF[s]);
            }
            // bound the live ranges: a scheduling fence every NODE_SCHED nodes
            if (ENOAO_NODE_SCHED > 0 && t % ENOAO_NODE_SCHED == ENOAO_NODE_SCHED - 1)
                __builtin_amdgcn_sched_barrier(0);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        const int s = fs[i];
        const double sc = 2.0 * fscale<NC, CH>(s);
        if (okmask & (1 << s)) {
            wh[s] = tf.hs[s] * (1.0 / sc);
            sel[2 * s] = sel[2 * s + 1] = K - 1;
        } else {
            int sp, sm;
            const double hp = Recon<ORDER>::select(gp[i], sc * delta, tf.is[s][0], sp);
            const double hm = Recon<ORDER>::select(gm[i], sc * delta, tf.is[s][1], sm);
            wh[s] = (sp == K - 1 && sm == K - 1 ? tf.hs[s] : hp + hm) * (1.0 / sc);
            sel[2 * s] = sp;
            sel[2 * s + 1] = sm;
        }
    }
}

// Numerical flux of one face from its 2G window nodes (w0: node 0, quantity
// stride qs, node stride ns; d0/dqs/dns: the staged top differences when
// DSTAGED, quantities U then F, for advection u only).  shortcut = false: every
// field takes the full selection (the result is the same).
template <int EQ, int ORDER, bool DSTAGED, bool CH>
__device__ __forceinline__ void face_flux(const double *w0, int qs, int ns, const double *d0, int dqs, int dns,
                                          const double *al, double gm1, double delta, double adv, bool shortcut,
                                          double (&Fh)[NodeTraits<EQ>::NC], int (&sel)[2 * NodeTraits<EQ>::NC])
{
    constexpr int H = ReconTraits<ORDER>::H, G = H + 1, W = 2 * H + 1, K = ReconTraits<ORDER>::K;
    if constexpr (EQ == ADVECTION) {
        // f^(+/-) = (a u +/- alpha u)/2, reconstructed as 2 f^(+/-); the
        // differences and the symmetric stencil of f = a u are a times those of u
        using T = TopStencil<ORDER>;
        double du[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) du[p] = DSTAGED ? d0[p * dns] : T::diff(w0 + p * ns, ns);
        const double a = al[0];
        const double isp = fmin(fabs(fma(a, du[0], adv * du[0])), fabs(fma(a, du[1], adv * du[1])));
        const double ism = fmin(fabs(fma(-a, du[2], adv * du[2])), fabs(fma(-a, du[1], adv * du[1])));
        const double hs = fma(a * T::kappa, du[1], adv * T::sym(w0, ns));
        if (wave_all(isp <= 2.0 * delta && ism <= 2.0 * delta) & shortcut) {
            Fh[0] = 0.5 * hs;
            sel[0] = sel[1] = K - 1;
            return;
        }
        double gp[W], gm[W];
#pragma unroll
        for (int t = 0; t < 2 * G; ++t) {
            const double u = w0[t * ns];
            const double au = adv * u;
            if (t < W) gp[t] = fma(a, u, au);
            if (t >= 1) gm[2 * H + 1 - t] = fma(-a, u, au);
        }
        int sp, sm;
        const double hp = Recon<ORDER>::select(gp, 2.0 * delta, isp, sp);
        const double hm = Recon<ORDER>::select(gm, 2.0 * delta, ism, sm);
        Fh[0] = 0.5 * (sp == K - 1 && sm == K - 1 ? hs : hp + hm);
        sel[0] = sp;
        sel[1] = sm;
    } else {
        constexpr int NC = NodeTraits<EQ>::NC, QR = 2 * NC;
        const double *nl = w0 + (G - 1) * ns, *nr = w0 + G * ns;
        RoeState r{};
        if constexpr (!CH) {
            // conserved components: no Roe state
        } else if constexpr (EQ == EULER1D)
            r = roe_state(nl[QR * qs], nl[(QR + 1) * qs], 0.0, nl[(QR + 2) * qs], nr[QR * qs],
                          nr[(QR + 1) * qs], 0.0, nr[(QR + 2) * qs], gm1);
        else
            r = roe_state(nl[QR * qs], nl[(QR + 1) * qs], nl[(QR + 2) * qs], nl[(QR + 3) * qs], nr[QR * qs],
                          nr[(QR + 1) * qs], nr[(QR + 2) * qs], nr[(QR + 3) * qs], gm1);
        double wh[NC];
        int okmask = 0;  // fields whose top candidate is within delta on every lane
        TopForm<NC> tf;
        top_form<NC, ORDER, DSTAGED, CH>(w0, qs, ns, d0, dqs, dns, r, al, delta, tf);
#pragma unroll
        for (int s = 0; s < NC; ++s)
            if (top_wave_ok<NC, CH>(tf, s, delta, shortcut)) okmask |= 1 << s;
        if (okmask == (1 << NC) - 1) {
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                wh[s] = tf.hs[s] * (1.0 / (2.0 * fscale<NC, CH>(s)));
                sel[2 * s] = sel[2 * s + 1] = K - 1;
            }
        } else if constexpr (NC == 4) {
            field_pass<4, ORDER, 0, 3, CH>(w0, qs, ns, r, al, delta, okmask, tf, wh, sel);
            field_pass<4, ORDER, 1, 2, CH>(w0, qs, ns, r, al, delta, okmask, tf, wh, sel);
        } else {
            field_pass<3, ORDER, 0, 2, CH>(w0, qs, ns, r, al, delta, okmask, tf, wh, sel);
            field_pass<3, ORDER, 1, -1, CH>(w0, qs, ns, r, al, delta, okmask, tf, wh, sel);
        }
        from_fields<NC, CH>(r, wh, Fh);
    }
}

// Staged top differences of two consecutive nodes i and i+1: D_0 of every
// staged quantity (U then F; advection: u) from nodes i .. i+2H, which the two
// share (one lane reads 2H+1 nodes for both instead of 2H for each).  x: node
// i, quantity stride qs, node stride ns; out: quantity stride oqs, node stride
// ons.  With two == false only node i's difference is formed, from nodes
// i .. i+2H-1 (node i+2H is not read).
template <int EQ, int ORDER>
__device__ __forceinline__ void stage_diff2(const double *x, int qs, int ns, double *out, int oqs, int ons, bool two)
{
    constexpr int ND = EQ == ADVECTION ? 1 : 2 * NodeTraits<EQ>::NC;
    constexpr int H = ReconTraits<ORDER>::H;
#pragma unroll
    for (int m = 0; m < ND; ++m) {
        double w[2 * H + 1];
#pragma unroll
        for (int t = 0; t < 2 * H; ++t) w[t] = x[m * qs + t * ns];
        w[2 * H] = two ? x[m * qs + 2 * H * ns] : 0.0;
        out[m * oqs] = TopStencil<ORDER>::diff(w, 1);
        if (two) out[m * oqs + ons] = TopStencil<ORDER>::diff(w + 1, 1);
    }
}

// RK stage combine (Shu-Osher form): s = 1: in + dt L; s = 2: 3/4 base +
// 1/4 (in + dt L); s = 3: 1/3 base + 2/3 (in + dt L).
template <int MODE>
__device__ __forceinline__ double rk_combine(double in, double base, double dt, double L)
{
    const double y = fma(dt, L, in);
    if constexpr (MODE == M_S1) return y;
    else if constexpr (MODE == M_S2) return fma(0.75, base, 0.25 * y);
    else return fma(1.0 / 3.0, base, (2.0 / 3.0) * y);
}

// 2D stages: the x-sweep writes its part of L, the y-sweep adds its own and
// applies the combine to L = L_x + L_y.

// Per-instance values of one sweep launch.  A workgroup walks a contiguous
// chunk of the tile list, so it reloads them only when the walk crosses into
// another instance; within an instance no tile reads a descriptor.
template <int EQ, int MODE> struct View {
    static constexpr int NC = NodeTraits<EQ>::NC;
    long long t0, t1;      // the instance's tiles in the batch list
    int k, nx, ny, pitch, per_row, bc;
    int active;            // the instance is still stepping
    const GMEM double *in;    // stage input
    GMEM double *out;         // stage output
    const GMEM double *base;  // u^n (stages 2 and 3)
    GMEM double *lx;          // x-part of L (2D) / L (rhs)
    GMEM uint8_t *sel;
    GMEM unsigned long long *amax;
    GMEM Ctrl *ctrl;
    double idx, idy, adv, dt;
    double al[NC];
};

// The view of the instance holding `tile`.  prev: the instance the walk was in
// (-1 at the start of a chunk: binary search); the tile lists are ordered by
// instance, so after the first the walk just moves on to the next instance
// that has tiles left.
template <int EQ, int MODE, bool Y, bool CH>
__device__ __forceinline__ View<EQ, MODE> load_view(const KParams &P, int n_inst, long long tile, int prev)
{
    constexpr int NC = NodeTraits<EQ>::NC;
    View<EQ, MODE> v;
    int k;
    if (prev < 0) {
        k = find_inst<!Y>(P.inst, n_inst, tile);
    } else {
        k = prev + 1;
        while (k < n_inst - 1 && tile >= (Y ? P.inst[k].ytile0 + P.inst[k].ytiles : P.inst[k].xtile0 + P.inst[k].xtiles))
            ++k;
    }
    v.k = uniform(k);
    const Inst &I = P.inst[v.k];
    v.t0 = uniform(Y ? I.ytile0 : I.xtile0);
    v.t1 = v.t0 + uniform(Y ? I.ytiles : I.xtiles);
    v.nx = uniform(I.nx);
    v.ny = uniform(I.ny);
    v.pitch = uniform(I.pitch);
    v.per_row = uniform(Y ? I.ytiles_per_row : I.segs_per_row);
    v.bc = uniform(Y ? I.bcy : I.bcx);
    v.ctrl = gmem(uniform(I.ctrl));
    v.active = uniform(v.ctrl->done) == 0;
    v.dt = uniform(v.ctrl->dt);
    v.in = gmem(uniform(MODE == M_S2 ? I.w1 : (MODE == M_S3 ? I.w2 : I.u)));
    v.out = gmem(uniform(MODE == M_S1 ? I.w1 : (MODE == M_S2 ? I.w2 : I.u)));
    v.base = gmem(uniform(I.u));
    v.lx = gmem(uniform(I.lx));
    v.sel = gmem(uniform(I.sel));
    if (v.sel && P.sel_slot > 0) {
        // records of one evaluation: x block [NC][2][ny][nx+1], then in 2D the y block [NC][2][ny+1][nx]
        const long long rec = (long long)NC * 2 * v.ny * (v.nx + 1) +
                              (EQ == EULER2D ? (long long)NC * 2 * (v.ny + 1) * v.nx : 0ll);
        v.sel += (long long)P.sel_slot * rec;
    }
    v.amax = gmem(uniform(I.amax));
    v.idx = 1.0 / uniform(I.dx);
    v.idy = 1.0 / uniform(I.dy);
    v.adv = uniform(I.adv);
    if constexpr (EQ == ADVECTION) {
        v.al[0] = fabs(v.adv);
    } else {
        const GMEM unsigned long long *a = v.amax + P.r_in * AMAX_VALS + (Y ? 3 : 0);
        const double m0 = uniform(as_double(a[0])), m1 = uniform(as_double(a[1])), m2 = uniform(as_double(a[2]));
        if constexpr (CH) {
            v.al[0] = m0;
            v.al[1] = m1;
            if (NC == 4) v.al[2] = m1;
            v.al[NC - 1] = m2;
        } else {
            // one alpha for all components: max(|u| + c) = max(max|u - c|, max|u + c|)
            const double a = fmax(m0, m2);
#pragma unroll
            for (int c = 0; c < NC; ++c) v.al[c] = a;
        }
    }
    return v;
}

// ---------------------------------------------------------------------------
// x-sweep.  Each wave: one segment of a grid line (64 faces, 63 cells) per
// tile, the wave's segments of a chunk in one contiguous run (a segment that
// continues the previous one along its line reuses its last 2G staged nodes).
// Tiles are software-pipelined: the global operands of tile t+1 are loaded into
// registers while tile t is reconstructed, so the memory latency hides behind
// the face arithmetic.  Waves per SIMD the register allocation must allow
// (measured: three for the x-sweep, whose LDS fits three workgroups per CU,
// except order 7, which spills at three; two for the y-sweep, whose LDS fits
// two, except order 7, which spills to scratch at two and runs faster at one
// with its whole working set in registers).
#ifndef ENOAO_X_WAVES_PER_EU
#define ENOAO_X_WAVES_PER_EU 3
#endif
#ifndef ENOAO_X7_WAVES_PER_EU
#define ENOAO_X7_WAVES_PER_EU 2  // order 7 (spills at three)
#endif
#ifndef ENOAO_Y_WAVES_PER_EU
#define ENOAO_Y_WAVES_PER_EU 2
#endif
#ifndef ENOAO_Y7_WAVES_PER_EU
#define ENOAO_Y7_WAVES_PER_EU 1  // order 7 (spills at two)
#endif

// a wave's segment within its instance: grid line and segment index along it
struct XCur {
    int row, segx;
};

// the segment of wave wseg in tile `tile` when the waves take consecutive
// segments (the maxima kernel's order)
__device__ __forceinline__ XCur x_cursor(long long tile, long long t0, int per_row, int wseg)
{
    // (segment counts of an instance fit 32 bits: ny * ceil(nx / 63))
    const unsigned seg = (unsigned)(tile - t0) * XW_SEGS + (unsigned)wseg;
    const unsigned row = seg / (unsigned)per_row;
    return XCur{(int)row, (int)(seg - row * (unsigned)per_row)};
}

// segment number seg of an instance (grid lines of per_row segments each)
__device__ __forceinline__ XCur x_segment(unsigned seg, int per_row)
{
    const unsigned row = seg / (unsigned)per_row;
    return XCur{(int)row, (int)(seg - row * (unsigned)per_row)};
}

// the next segment of an instance; it continues c along the same grid line
// unless it starts a new one (segx == 0)
__device__ __forceinline__ XCur x_next(XCur c, int per_row)
{
    if (++c.segx == per_row) {
        c.segx = 0;
        ++c.row;
    }
    return c;
}

// LDS exchange among the lanes of one wave: the wave's LDS operations are
// performed in order, so a wavefront-scope fence pair around a wave barrier
// orders each lane's writes before every lane's later reads.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// a lane's global operands of one x tile: the nodes it stages (segment
// positions lane and lane + 64; for a segment that continues the wave's
// previous one along its line only the 63 new nodes, positions 2G + lane) and,
// for a 1D stage 2 or 3, u^n at its cell.  Every register is written on every
// path (lanes and rows past the end load a clamped, in-bounds address whose
// value goes unused): a register that kept its old value would be copied while
// its previous load may still be in flight, and the copy's wait would stall on
// the prefetch just issued.
template <int NC> struct XPre {
    double U[2][NC];
    double base[NC];
};

template <int EQ, int MODE, int G>
__device__ __forceinline__ void x_prefetch(const View<EQ, MODE> &v, XCur c, bool cont, int lane,
                                           XPre<NodeTraits<EQ>::NC> &pre)
{
    constexpr int NC = NodeTraits<EQ>::NC, NN = XW_FACES + 2 * G - 1;
    const int nx = v.nx, sx = c.segx * XW_CELLS;
    const int row = min(c.row, v.ny - 1);
    const long long plane = (long long)v.pitch * v.ny;
    const GMEM double *rowp = v.in + (long long)row * v.pitch;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int i = cont ? min(2 * G + lane, NN - 1) : min(lane + 64 * j, NN - 1);
        const int x = bc_map(sx - G + i, nx, v.bc);
#pragma unroll
        for (int q = 0; q < NC; ++q) pre.U[j][q] = rowp[q * plane + x];
    }
    if constexpr ((MODE == M_S2 || MODE == M_S3) && EQ != EULER2D) {
        const int x = min(sx + lane, nx - 1);
        const GMEM double *b = v.base + (long long)row * v.pitch + x;
#pragma unroll
        for (int q = 0; q < NC; ++q) pre.base[q] = b[q * plane];
    }
}

template <int EQ, int ORDER, int MODE, bool REC, bool CH>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(ORDER == 7 ? ENOAO_X7_WAVES_PER_EU
                                                                  : ENOAO_X_WAVES_PER_EU))) void sweep_x(KParams P)
{
    constexpr int NC = NodeTraits<EQ>::NC, NQ = NodeTraits<EQ>::NQ;
    constexpr int H = ReconTraits<ORDER>::H, G = H + 1;
    constexpr int NN = XW_FACES + 2 * G - 1;  // nodes staged per segment
    constexpr int NNP = NN + 1;
    constexpr int ND = EQ == ADVECTION ? 1 : 2 * NC;  // staged top differences per node
    constexpr int NDN = XW_FACES + 2;                  // nodes with a staged difference
    constexpr bool FULL = (EQ != EULER2D) && (MODE != M_RHS);  // 1D stage: combine + maxima here
    __shared__ double lds[NQ * XW_SEGS * NNP];
    __shared__ double dif[ND * XW_SEGS * NDN];
    __shared__ double fh[NC * XW_SEGS * XW_FACES];
    __shared__ double red[(BLOCK / 64) * 8];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wseg = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n_inst = P.hdr->n_inst;
    const long long T = P.hdr->xtiles_total;
    const long long NG = chunk_groups(P, T);
    if (blockIdx.x >= NG) return;
    const long long t0 = (long long)blockIdx.x * T / NG, t1 = (long long)(blockIdx.x + 1) * T / NG;
    Maxima<EQ> mx;
    mx.reset();
    XPre<NC> pre;
    double *L = lds + wseg * NNP;
    double *Dl = dif + wseg * NDN;

    // Each wave owns its segment's LDS (nodes and face fluxes), so within the
    // tile loop the waves synchronise only with themselves.  The outer loop
    // runs once per instance met by the workgroup's chunk (uniform over the
    // workgroup, so the maxima flush, a workgroup reduction, is reached by all
    // waves together).
    int prev = -1;
    for (long long tile = t0; tile < t1;) {
        const View<EQ, MODE> v = load_view<EQ, MODE, false, CH>(P, n_inst, tile, prev);
        prev = v.k;
        const long long tend = v.t1 < t1 ? v.t1 : t1;
        if (!v.active) {
            tile = tend;
            continue;
        }
        if (MODE != M_RHS && P.r_zero >= 0 && tile == v.t0 && tid < AMAX_VALS)
            v.amax[P.r_zero * AMAX_VALS + tid] = 0ull;
        const int nx = v.nx;
        const long long plane = (long long)v.pitch * v.ny;
        // the waves take the instance's segments of this chunk in four contiguous
        // runs, so that a wave's next segment mostly continues its current one
        // along the grid line and shares its last 2G staged nodes
        const int T = (int)(tend - tile);
        XCur c = x_segment((unsigned)(tile - v.t0) * XW_SEGS + (unsigned)(wseg * T), v.per_row);
        bool cont = false;  // c continues the wave's previous segment
        x_prefetch<EQ, MODE, G>(v, c, cont, lane, pre);
        for (int k = 0; k < T; ++k) {
            const bool ok = c.row < v.ny;
            const int sx = c.segx * XW_CELLS;

            // stage this tile's nodes (flux, Roe inputs) into LDS
            if (ok) {
                if (cont) {
                    // the previous segment's nodes 63 .. 63 + 2G - 1 are this one's first
                    for (int t = lane; t < 2 * G * NQ; t += 64) {
                        const int m = t / (2 * G), i = t - m * (2 * G);
                        L[m * XW_SEGS * NNP + i] = L[m * XW_SEGS * NNP + XW_CELLS + i];
                    }
                }
                // nodes 2G + lane of a continuing segment, else lane and 64 + lane
                const int p0 = cont ? 2 * G + lane : lane;
                if (p0 < NN) {
                    double q[NQ];
                    node_quantities<EQ>(pre.U[0], P.gm1, q);
#pragma unroll
                    for (int m = 0; m < NQ; ++m) L[m * XW_SEGS * NNP + p0] = q[m];
                }
                if (!cont && lane + 64 < NN) {
                    double q[NQ];
                    node_quantities<EQ>(pre.U[1], P.gm1, q);
#pragma unroll
                    for (int m = 0; m < NQ; ++m) L[m * XW_SEGS * NNP + 64 + lane] = q[m];
                }
            }
            double base[NC];
#pragma unroll
            for (int q = 0; q < NC; ++q) base[q] = pre.base[q];
            // issue the next tile's loads before this tile's arithmetic
            const XCur cn = x_next(c, v.per_row);
            const bool cont_n = cn.segx != 0;
            if (k + 1 < T) x_prefetch<EQ, MODE, G>(v, cn, cont_n, lane, pre);
            wave_sync();
            // top differences of the nodes that start one (faces 0..63 read
            // 0..65), two consecutive nodes per lane
            static_assert(NDN % 2 == 0 && NDN / 2 <= 64, "one pair of nodes per lane");
            if (ok && lane < NDN / 2)
                stage_diff2<EQ, ORDER>(L + 2 * lane, XW_SEGS * NNP, 1, Dl + 2 * lane, XW_SEGS * NDN, 1, true);
            wave_sync();

            const int f = sx + lane;  // face index along the line
            if (ok) {
                double Fh[NC];
                int sel[2 * NC];
                face_flux<EQ, ORDER, true, CH>(L + lane, XW_SEGS * NNP, 1, Dl + lane, XW_SEGS * NDN, 1, v.al, P.gm1,
                                           P.delta, v.adv, (P.flags & KF_FULL_SELECTION) == 0, Fh, sel);
#pragma unroll
                for (int q = 0; q < NC; ++q) fh[(q * XW_SEGS + wseg) * XW_FACES + lane] = Fh[q];
                if (REC && v.sel && f <= nx) {
                    const long long xblock = (long long)v.ny * (nx + 1);
#pragma unroll
                    for (int s = 0; s < NC; ++s) {
                        const long long o = (long long)(2 * s) * xblock + (long long)c.row * (nx + 1) + f;
                        v.sel[o] = (uint8_t)sel[2 * s];
                        v.sel[o + xblock] = (uint8_t)sel[2 * s + 1];
                    }
                }
            }
            wave_sync();

            const int x = sx + lane;
            if (ok && lane < XW_CELLS && x < nx) {
                const long long o = (long long)c.row * v.pitch + x;
                double Lc[NC];
#pragma unroll
                for (int q = 0; q < NC; ++q)
                    Lc[q] = -(fh[(q * XW_SEGS + wseg) * XW_FACES + lane + 1] - fh[(q * XW_SEGS + wseg) * XW_FACES + lane]) * v.idx;
                if constexpr (!FULL) {  // L (rhs) or, in 2D, its x-part
#pragma unroll
                    for (int q = 0; q < NC; ++q) v.lx[q * plane + o] = Lc[q];
                } else {
                    double Un[NC];
#pragma unroll
                    for (int q = 0; q < NC; ++q) {
                        const double uin = L[q * XW_SEGS * NNP + lane + G];
                        Un[q] = rk_combine<MODE>(uin, base[q], v.dt, Lc[q]);
                        v.out[q * plane + o] = Un[q];
                    }
                    mx.add(Un, P.gamma, v.idx, v.idy);
                }
            }
            wave_sync();
            c = cn;
            cont = cont_n;
        }
        tile = tend;
        if (FULL) mx.flush(v.amax, v.ctrl, P.r_out, red);
    }
}

// ---------------------------------------------------------------------------
// y-sweep (2D).  A workgroup tile is 4 YW columns x 64/YW cell rows; each wave
// owns a strip of YW columns (lane = YW * row + column) and walks its tiles
// down the strip.  Successive tiles of a walk share node rows
// and one face row, so a walk keeps a rolling buffer: after its first tile, a
// tile copies the 2G-1 node rows it shares with the previous one, stages only
// 64/YW new rows, reuses the previous tile's last face row, and computes
// 64/YW new face rows -- one face and one staged node per lane and tile,
// and every face of the walk is computed once.  Each wave exchanges data only
// among its own lanes, so the tile loop has no workgroup barrier.  Momentum
// components are exchanged on load so the x-direction formulas apply.  The
// next tile's global operands are prefetched into registers.
// a tile's position within its instance: tile row along y, column group
struct YCur {
    int ty, cg;
};

__device__ __forceinline__ YCur y_cursor(long long tile, long long t0, int per_row)
{
    // (tile counts of an instance fit 32 bits)
    const unsigned tl = (unsigned)(tile - t0), cg = tl / (unsigned)per_row;
    return YCur{(int)(tl - cg * (unsigned)per_row), (int)cg};
}

__device__ __forceinline__ YCur y_advance(YCur c, int per_row)
{
    if (++c.ty == per_row) {
        c.ty = 0;
        ++c.cg;
    }
    return c;
}

// buffer rows of a walk: row b holds node row sy - G + b (sy = first cell row
// of the tile); face row k (k = 0..64/YW, the face below cell row sy + k)
// reads buffer rows k .. k + 2G - 1
template <int G, int YW> struct YBuf {
    static constexpr int CELLS = yt_cells(YW), COLS = yt_cols(YW);
    static constexpr int ROWS = CELLS + 2 * G;
    static constexpr int NODES = ROWS * YW;                // staged by a walk's first tile
    static constexpr int J = (NODES + 63) / 64;            // nodes per lane then
    static constexpr int FRESH = 2 * G;                    // first row a later tile stages
};

template <int G, int YW> struct YPre {
    double U[YBuf<G, YW>::J][4];
    double lx[4];    // x-part of L at the lane's cell
    double base[4];  // u^n at the lane's cell (stages 2 and 3)
};

// a lane's global operands of one y tile: the strip nodes it stages (all rows
// for the first tile of a walk, rows FRESH.. for the others), the x-part of L
// and, for stages 2 and 3, u^n at its cell (lanes past the grid's edge read a
// clamped, in-bounds address whose value goes unused).
template <int MODE, int G, int YW>
__device__ __forceinline__ void y_prefetch(const View<EULER2D, MODE> &v, YCur c, bool first, int wv, int lane,
                                           YPre<G, YW> &pre)
{
    using B = YBuf<G, YW>;
    const int perm[4] = {0, 2, 1, 3};
    const int nx = v.nx, ny = v.ny;
    const long long plane = (long long)v.pitch * ny;
    const int sy = c.ty * B::CELLS, cbase = c.cg * B::COLS + wv * YW;
    const int b0 = first ? 0 : B::FRESH;
#pragma unroll
    for (int j = 0; j < B::J; ++j) {
        const int i = b0 * YW + lane + 64 * j;
        if (i < B::NODES && (first || j == 0)) {
            const int r = i / YW, c0 = i % YW;
            const int y = bc_map(sy - G + r, ny, v.bc);
            const int x = min(cbase + c0, nx - 1);
            const GMEM double *p = v.in + (long long)y * v.pitch + x;
#pragma unroll
            for (int q = 0; q < 4; ++q) pre.U[j][q] = p[perm[q] * plane];
        }
    }
    const int fl = lane / YW, y = min(sy + fl, ny - 1), col = min(cbase + (lane % YW), nx - 1);
    const long long o = (long long)y * v.pitch + col;
#pragma unroll
    for (int q = 0; q < 4; ++q) pre.lx[q] = v.lx[q * plane + o];
    if constexpr (MODE == M_S2 || MODE == M_S3) {
#pragma unroll
        for (int q = 0; q < 4; ++q) pre.base[q] = v.base[q * plane + o];
    }
}

// one face of a y strip into the face buffer (and the selection record)
template <int ORDER, bool REC, int MODE, int YW, bool CH>
__device__ __forceinline__ void y_face(const View<EULER2D, MODE> &v, const KParams &P, const double *W, int QS,
                                       double *WF, int k, int cc, int col, int f)
{
    constexpr int NC = 4, CELLS = yt_cells(YW);
    double Fh[NC];
    int sel[2 * NC];
    face_flux<EULER2D, ORDER, false, CH>(W + k * YW + cc, QS, YW, nullptr, 0, 0, v.al, P.gm1, P.delta, 0.0,
                                     (P.flags & KF_FULL_SELECTION) == 0, Fh, sel);
#pragma unroll
    for (int q = 0; q < NC; ++q) WF[(q * (CELLS + 1) + k) * YW + cc] = Fh[q];
    if (REC && v.sel && col < v.nx && f <= v.ny) {
        const long long xblock = (long long)v.ny * (v.nx + 1), yblock = (long long)(v.ny + 1) * v.nx;
        const long long ybase = (long long)NC * 2 * xblock;
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const long long o = ybase + (long long)(2 * s) * yblock + (long long)f * v.nx + col;
            v.sel[o] = (uint8_t)sel[2 * s];
            v.sel[o + yblock] = (uint8_t)sel[2 * s + 1];
        }
    }
}

template <int ORDER, int MODE, bool REC, int YW, bool CH>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(ORDER == 7 ? ENOAO_Y7_WAVES_PER_EU
                                                                  : ENOAO_Y_WAVES_PER_EU))) void sweep_y(KParams P)
{
    constexpr int NC = 4, NQ = 12, NW = BLOCK / 64;
    constexpr int H = ReconTraits<ORDER>::H, G = H + 1;
    using B = YBuf<G, YW>;
    constexpr int CELLS = B::CELLS, COLS = B::COLS;
    constexpr int QS = B::NODES;  // a wave's LDS stride between quantities
    __shared__ double lds[NW * NQ * QS];
    __shared__ double fh[NW * NC * (CELLS + 1) * YW];
    __shared__ double red[NW * 8];
    // epilogue operands of the tile (x-part of L; u^n for stages 2 and 3),
    // staged from the prefetch registers so they are not held through the face
    // arithmetic
    constexpr bool BASE = MODE == M_S2 || MODE == M_S3;
    __shared__ double elx[NC * BLOCK];
    __shared__ double ebase[BASE ? NC * BLOCK : 1];
    const int perm[4] = {0, 2, 1, 3};

    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int cc = lane % YW, fl = lane / YW;
    double *W = lds + wv * NQ * QS;
    double *WF = fh + wv * NC * (CELLS + 1) * YW;
    const int n_inst = P.hdr->n_inst;
    const long long T = P.hdr->ytiles_total;
    const long long NG = chunk_groups(P, T);
    if (blockIdx.x >= NG) return;
    const long long t0 = (long long)blockIdx.x * T / NG, t1 = (long long)(blockIdx.x + 1) * T / NG;
    Maxima<EULER2D> mx;
    mx.reset();
    YPre<G, YW> pre;

    // one outer iteration per instance met by the workgroup's chunk (uniform
    // over the workgroup: the maxima flush is reached by all waves together)
    int prev = -1;
    for (long long tile = t0; tile < t1;) {
        const View<EULER2D, MODE> v = load_view<EULER2D, MODE, true, CH>(P, n_inst, tile, prev);
        prev = v.k;
        const long long tend = v.t1 < t1 ? v.t1 : t1;
        if (!v.active) {
            tile = tend;
            continue;
        }
        const int nx = v.nx, ny = v.ny;
        const long long plane = (long long)v.pitch * ny;
        YCur c = y_cursor(tile, v.t0, v.per_row);
        bool first = true;  // the tile starts a walk
        y_prefetch<MODE, G, YW>(v, c, true, wv, lane, pre);
        for (; tile < tend; ++tile) {
            if (!first) {
                // rows shared with the previous tile move up by 64/YW
                for (int i = YW + lane; i < B::FRESH * YW; i += 64) {
#pragma unroll
                    for (int m = 0; m < NQ; ++m) W[m * QS + i] = W[m * QS + i + CELLS * YW];
                }
                wave_sync();  // the new rows below overwrite rows other lanes just read
            }
#pragma unroll
            for (int j = 0; j < B::J; ++j) {
                const int i = (first ? 0 : B::FRESH * YW) + lane + 64 * j;
                if (i < B::NODES && (first || j == 0)) {
                    double q[NQ];
                    node_quantities<EULER2D>(pre.U[j], P.gm1, q);
#pragma unroll
                    for (int m = 0; m < NQ; ++m) W[m * QS + i] = q[m];
                }
            }
#pragma unroll
            for (int q = 0; q < NC; ++q) elx[q * BLOCK + tid] = pre.lx[q];
            if constexpr (BASE) {
#pragma unroll
                for (int q = 0; q < NC; ++q) ebase[q * BLOCK + tid] = pre.base[q];
            }
            const YCur cn = y_advance(c, v.per_row);
            const bool next_first = cn.ty == 0;
            if (tile + 1 < tend) y_prefetch<MODE, G, YW>(v, cn, next_first, wv, lane, pre);
            wave_sync();

            const int sy = c.ty * CELLS;
            const int col = c.cg * COLS + wv * YW + cc;
            // a walk's first tile also computes face row 0 (one call site, so the
            // face code is instantiated once)
#pragma unroll 1
            for (int pass = first ? 0 : 1; pass < 2; ++pass) {
                const int k = pass == 0 ? 0 : fl + 1;
                if (pass == 1 || lane < YW) y_face<ORDER, REC, MODE, YW, CH>(v, P, W, QS, WF, k, cc, col, sy + k);
            }
            wave_sync();

            const int y = sy + fl;
            if (y < ny && col < nx) {
                const long long o = (long long)y * v.pitch + col;
                double Ly[NC];  // natural component order
#pragma unroll
                for (int q = 0; q < NC; ++q)
                    Ly[perm[q]] = -(WF[(q * (CELLS + 1) + fl + 1) * YW + cc] - WF[(q * (CELLS + 1) + fl) * YW + cc]) *
                                  v.idy;
                if constexpr (MODE == M_RHS) {
#pragma unroll
                    for (int q = 0; q < NC; ++q) v.lx[q * plane + o] = elx[q * BLOCK + tid] + Ly[q];
                } else {
                    // stage input at the cell: buffer row fl + G (quantity perm[q]
                    // holds natural component q)
                    double Un[NC];
#pragma unroll
                    for (int q = 0; q < NC; ++q) {
                        const double uin = W[perm[q] * QS + (fl + G) * YW + cc];
                        const double base = BASE ? ebase[q * BLOCK + tid] : 0.0;
                        Un[q] = rk_combine<MODE>(uin, base, v.dt, elx[q * BLOCK + tid] + Ly[q]);
                        v.out[q * plane + o] = Un[q];
                    }
                    mx.add(Un, P.gamma, v.idx, v.idy);
                }
            }
            wave_sync();
            // the last face row is the next tile's first
            if (lane < YW) {
#pragma unroll
                for (int q = 0; q < NC; ++q) WF[(q * (CELLS + 1)) * YW + lane] = WF[(q * (CELLS + 1) + CELLS) * YW + lane];
            }
            wave_sync();
            c = cn;
            first = next_first;
        }
        if (MODE != M_RHS) mx.flush(v.amax, v.ctrl, P.r_out, red);
    }
}

// ---------------------------------------------------------------------------
// Maxima of the input state (alpha for the first evaluation, CFL step).
template <int EQ>
__global__ __launch_bounds__(BLOCK) void state_maxima(KParams P)
{
    constexpr int NC = NodeTraits<EQ>::NC;
    __shared__ double red[(BLOCK / 64) * 8];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wseg = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n_inst = P.hdr->n_inst;
    const long long T = P.hdr->xtiles_total;
    const long long NG = chunk_groups(P, T);
    if (blockIdx.x >= NG) return;
    const long long t0 = (long long)blockIdx.x * T / NG, t1 = (long long)(blockIdx.x + 1) * T / NG;
    Maxima<EQ> mx;
    mx.reset();
    int cur = -1;
    long long end = -1;
    int nx = 0, ny = 0, pitch = 0, spr = 1;
    long long first = 0;
    const GMEM double *u = nullptr;
    double idx = 0.0, idy = 0.0;
    for (long long tile = t0; tile < t1; ++tile) {
        if (tile >= end) {
            const int k = find_inst<true>(P.inst, n_inst, tile);
            if (cur >= 0) mx.flush(gmem(P.inst[cur].amax), gmem(P.inst[cur].ctrl), P.r_out, red);
            cur = k;
            const Inst &I = P.inst[k];
            first = I.xtile0;
            end = first + I.xtiles;
            nx = I.nx;
            ny = I.ny;
            pitch = I.pitch;
            spr = I.segs_per_row;
            u = gmem(I.u);
            idx = 1.0 / I.dx;
            idy = 1.0 / I.dy;
        }
        const long long plane = (long long)pitch * ny;
        const XCur c = x_cursor(tile, first, spr, wseg);
        const int x = c.segx * XW_CELLS + lane;
        if (c.row < ny && lane < XW_CELLS && x < nx) {
            double U[NC];
#pragma unroll
            for (int q = 0; q < NC; ++q) U[q] = u[q * plane + (long long)c.row * pitch + x];
            mx.add(U, P.gamma, idx, idy);
        }
    }
    if (cur >= 0) mx.flush(gmem(P.inst[cur].amax), gmem(P.inst[cur].ctrl), P.r_out, red);
}

// zero all maxima slots and the status of every instance
__global__ void reset_maxima(KParams P)
{
    const int n = P.hdr->n_inst;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n * AMAX_SLOTS * AMAX_VALS;
         k += gridDim.x * blockDim.x) {
        const int i = k / (AMAX_SLOTS * AMAX_VALS), j = k % (AMAX_SLOTS * AMAX_VALS);
        gmem(P.inst[i].amax)[j] = 0ull;
    }
}

// Time-step control of one instance: CFL (or fixed) step from the maxima m of
// the state at the start of the step (m[0], m[2]: max |u-c|, |u+c|; m[6]: the
// 2D sum), clipped to land on t_final.  Returns whether a step is taken.
template <int EQ>
__device__ __forceinline__ bool control_update(Ctrl &C, double m0, double m2, double m6, double dx, double adv)
{
    if (C.done) return false;
    if (C.status != 0 || C.steps >= C.max_steps) { C.done = 1; return false; }
    const double rem = C.t_final - C.t;
    if (!(rem > 0.0)) { C.done = 1; return false; }
    double dt;
    if (C.dt_fixed > 0.0) {
        dt = C.dt_fixed;
    } else {
        if constexpr (EQ == ADVECTION) {
            dt = C.cfl * dx / fabs(adv);
        } else if constexpr (EQ == EULER1D) {
            const double smax = fmax(m0, m2);  // max(|u|+c)
            if (!(smax > 0.0)) { C.status |= 1; C.done = 1; return false; }
            dt = C.cfl * dx / smax;
        } else {
            const double smax = m6;
            if (!(smax > 0.0)) { C.status |= 1; C.done = 1; return false; }
            dt = C.cfl / smax;
        }
    }
    const bool last = dt >= rem * (1.0 - 1e-10);
    if (last) dt = rem;
    C.dt = dt;
    C.t = last ? C.t_final : C.t + dt;
    C.steps = C.steps + 1;
    return true;
}

// one thread per instance; slot 0 of the maxima holds the state u^n
template <int EQ>
__global__ void step_control(KParams P)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.hdr->n_inst) return;
    const Inst &I = P.inst[k];
    const unsigned long long *a = I.amax;
    control_update<EQ>(*I.ctrl, as_double(a[0]), as_double(a[2]), as_double(a[6]), I.dx, I.adv);
}

// ---------------------------------------------------------------------------
// LDS-resident solver of small 1D members.  One workgroup per member runs
// `nsteps` controlled steps with u^n and both stage states in LDS: HBM is
// touched only to load the state and store it back.  Within a stage each wave
// owns 64-face line segments (63 cells each, taken round-robin) and works like
// a wave of the streaming x-sweep: it stages the segment's node quantities in
// its own LDS, computes the 64 face fluxes (top differences formed per face, as
// the y-sweep does: staging them costs a pass and two synchronisations more,
// and measured 15% slower here) and updates the 63 cells, synchronising only
// with itself.  The stages write distinct arrays
// (u^n -> w1 -> w2 -> u^n; stage 3 reads u^n only at the cell it writes), so
// no wave overwrites what another still reads, and one workgroup barrier per
// stage (which also publishes the per-wave maxima) is the only one.  Every
// arithmetic step is the streaming path's (same node quantities, staged top
// differences, face flux, flux difference, stage combine, maxima and step
// control), so a member's result is bitwise the one of the streaming kernels.
// A step of a member takes a fixed latency plus its segments over the waves
// (measured alone: 13 us at 128 nodes, 41 us at 1700), so a batch step lasts
// about as long as its largest member's.

// per-wave LDS of a resident workgroup: staged nodes, face fluxes
template <int EQ, int ORDER> struct ResWave {
    static constexpr int NQ = NodeTraits<EQ>::NQ, NC = NodeTraits<EQ>::NC;
    static constexpr int G = ReconTraits<ORDER>::H + 1;
    static constexpr int NN = XW_FACES + 2 * G - 1, NNP = NN + 1;
    static constexpr int DOUBLES = NQ * NNP + NC * XW_FACES;
};

// all threads: the maxima of the waves of stage `par` (every thread reads every
// wave's values, so no second barrier is needed); the non-physical flag goes to C
template <int EQ, int NW>
__device__ __forceinline__ void resident_maxima(const double *red, int par, double (&cm)[8], Ctrl &C)
{
    constexpr int NV = Maxima<EQ>::NV;
    const double *r = red + par * NW * 8;
#pragma unroll
    for (int i = 0; i < 8; ++i) cm[i] = 0.0;
    double bad = 0.0;
    for (int w = 0; w < NW; ++w) {
#pragma unroll
        for (int i = 0; i < NV; ++i) cm[i] = fmax(cm[i], r[w * 8 + i]);
        bad = fmax(bad, r[w * 8 + 7]);
    }
    if (bad != 0.0) C.status |= 1;
}

// a wave's maxima to red[par] (lane 0 writes; published by the next barrier)
template <int EQ, int NW>
__device__ __forceinline__ void resident_wave_maxima(Maxima<EQ> &mx, double *red, int par)
{
    constexpr int NV = Maxima<EQ>::NV;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double x = mx.v[i];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
        mx.v[i] = x;
    }
    int b = mx.bad;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) b |= __shfl_xor(b, o, 64);
    if (lane == 0) {
        double *r = red + (par * NW + wv) * 8;
#pragma unroll
        for (int i = 0; i < NV; ++i) r[i] = mx.v[i];
        r[7] = (double)b;
    }
}

// One stage over a 1D line for the waves of a resident or cooperative launch:
// segments first, first + stride, ... (63 cells each).  Each wave stages a
// segment's node quantities in its own LDS (wl), computes the segment's 64 face
// fluxes and updates its cells from `in` (and `base`: u^n) into `out`; alpha
// comes from cm, the maxima of the stage input, and the output's maxima
// accumulate in mx.
template <int EQ, int ORDER, int MODE, bool CH>
__device__ __forceinline__ void line_stage(const KParams &P, const Inst &I, int n, const double *in,
                                           const double *base, double *out, double *wl, const double (&cm)[8],
                                           double dt, int first, int stride, Maxima<EQ> &mx)
{
    using RW = ResWave<EQ, ORDER>;
    constexpr int NC = RW::NC, NQ = RW::NQ, G = RW::G, NN = RW::NN, NNP = RW::NNP;
    const int lane = threadIdx.x & 63;
    double al[NC];
    if constexpr (EQ == ADVECTION) {
        al[0] = fabs(I.adv);
    } else if constexpr (CH) {
        al[0] = cm[0];
        al[1] = cm[1];
        al[NC - 1] = cm[2];
    } else {
        const double a = fmax(cm[0], cm[2]);
#pragma unroll
        for (int c = 0; c < NC; ++c) al[c] = a;
    }
    double *q = wl, *fh = wl + NQ * NNP;
    const double idx = 1.0 / I.dx, idy = 1.0 / I.dy;
    const int nseg = (n + XW_CELLS - 1) / XW_CELLS;
    for (int seg = first; seg < nseg; seg += stride) {
        const int sx = seg * XW_CELLS;
        // node quantities of nodes sx - G .. sx + 63 + G - 1
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int i = lane + 64 * j;
            if (i < NN) {
                const int x = bc_map(sx - G + i, n, I.bcx);
                double U[NC], qq[NQ];
#pragma unroll
                for (int c = 0; c < NC; ++c) U[c] = in[c * n + x];
                node_quantities<EQ>(U, P.gm1, qq);
#pragma unroll
                for (int m = 0; m < NQ; ++m) q[m * NNP + i] = qq[m];
            }
        }
        wave_sync();
        double Fh[NC];
        int sel[2 * NC];
        face_flux<EQ, ORDER, false, CH>(q + lane, NNP, 1, nullptr, 0, 0, al, P.gm1, P.delta, I.adv,
                                        (P.flags & KF_FULL_SELECTION) == 0, Fh, sel);
#pragma unroll
        for (int c = 0; c < NC; ++c) fh[c * XW_FACES + lane] = Fh[c];
        wave_sync();
        const int x = sx + lane;
        if (lane < XW_CELLS && x < n) {
            double Un[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double Lc = -(fh[c * XW_FACES + lane + 1] - fh[c * XW_FACES + lane]) * idx;
                Un[c] = rk_combine<MODE>(q[c * NNP + lane + G], base[c * n + x], dt, Lc);
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) out[c * n + x] = Un[c];
            mx.add(Un, P.gamma, idx, idy);
        }
        wave_sync();  // the next segment overwrites the staged nodes and fluxes
    }
}

template <int EQ, int ORDER, int MODE, bool CH, int NW>
__device__ __forceinline__ void resident_stage(const KParams &P, const Inst &I, int n, const double *in,
                                               const double *base, double *out, double *wl, double *red, int par,
                                               double (&cm)[8], Ctrl &C, double dt)
{
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    Maxima<EQ> mx;
    mx.reset();
    line_stage<EQ, ORDER, MODE, CH>(P, I, n, in, base, out, wl, cm, dt, wv, NW, mx);
    resident_wave_maxima<EQ, NW>(mx, red, par);
    __syncthreads();  // the stage output and every wave's maxima are complete
    resident_maxima<EQ, NW>(red, par, cm, C);
}

// one launch covers members res_order[res_first .. res_first + gridDim.x) (the
// members of one LDS size class, largest first), one workgroup of NW waves each
template <int EQ, int ORDER, bool CH, int NW>
__global__ __launch_bounds__(64 * NW) void resident_1d(KParams P, int nsteps)
{
    using RW = ResWave<EQ, ORDER>;
    constexpr int NC = RW::NC;
    extern __shared__ double sm[];
    const int slot = P.res_first + (int)blockIdx.x;
    const Inst &I = P.inst[P.res_order ? P.res_order[slot] : slot];
    const int n = I.nx, pitch = I.pitch, tid = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    double *un = sm;
    double *w1 = un + NC * n;
    double *w2 = w1 + NC * n;
    double *wl = w2 + NC * n + wv * RW::DOUBLES;
    double *red = w2 + NC * n + NW * RW::DOUBLES;  // two parities of NW x 8 values
    GMEM double *ug = gmem(I.u);
#pragma unroll
    for (int c = 0; c < NC; ++c)
        for (int j = tid; j < n; j += 64 * NW) un[c * n + j] = ug[c * pitch + j];
    // every thread keeps the same copy of the member's time-loop control
    Ctrl C = *I.ctrl;
    double cm[8];
    {
        const double idx = 1.0 / I.dx, idy = 1.0 / I.dy;
        Maxima<EQ> mx;
        mx.reset();
        for (int j = tid; j < n; j += 64 * NW) {
            double U[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) U[c] = ug[c * pitch + j];
            mx.add(U, P.gamma, idx, idy);
        }
        resident_wave_maxima<EQ, NW>(mx, red, 1);
        __syncthreads();  // u^n loaded, maxima published
        resident_maxima<EQ, NW>(red, 1, cm, C);
    }
    for (int step = 0; step < nsteps; ++step) {
        if (!control_update<EQ>(C, cm[0], cm[2], cm[6], I.dx, I.adv)) break;  // the same in every thread
        const double dt = C.dt;
        // the maxima alternate between two parities from stage to stage (step 0's
        // first stage after the initial maxima's parity 1), so a wave that runs
        // ahead never overwrites values another wave has yet to read
        const int par = (3 * step) & 1;
        resident_stage<EQ, ORDER, M_S1, CH, NW>(P, I, n, un, un, w1, wl, red, par, cm, C, dt);
        resident_stage<EQ, ORDER, M_S2, CH, NW>(P, I, n, w1, un, w2, wl, red, par ^ 1, cm, C, dt);
        resident_stage<EQ, ORDER, M_S3, CH, NW>(P, I, n, w2, un, un, wl, red, par, cm, C, dt);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
        for (int j = tid; j < n; j += 64 * NW) ug[c * pitch + j] = un[c * n + j];
    if (tid == 0) *I.ctrl = C;
}

// ---------------------------------------------------------------------------
// Cooperative solver of one mid-sized 1D line (too long for one workgroup's
// LDS, short enough for one segment per wave of at most one workgroup per CU).
// A kernel boundary between stages costs several microseconds, about a stage's
// work on such a line; here one cooperative launch (every workgroup resident)
// runs every controlled step of a call, the stage states in the plan's HBM
// buffers, with a grid barrier after each stage.  Each wave takes its segments
// like a wave of the resident solver (line_stage: the same arithmetic, so a
// result is bitwise the streaming kernels'), each workgroup folds its maxima
// into the member's three-slot ring with one atomic max per value, and after
// the barrier every thread reads them and takes the same time-step decision.

constexpr unsigned COOP_SPIN_LIMIT = 1u << 19;  // polls of one barrier wait (about 0.5 s; never reached)

// Grid barrier: bar[0] counts arrivals (monotonic; the n-th barrier waits for
// n x grid), bar[1] is set when a wait outlasts its bound.  Every thread's
// stores before it are visible to every thread after it.  Returns false once
// a wait has failed (then it no longer waits).
__device__ __forceinline__ bool grid_barrier(GMEM unsigned *bar, unsigned target)
{
    __shared__ int ok;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int good = 1;
        for (unsigned spin = 0;; ++spin) {
            if (__hip_atomic_load(&bar[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
            if (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                spin >= COOP_SPIN_LIMIT) {
                __hip_atomic_store(&bar[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                good = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        ok = good;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok != 0;
}

// a workgroup's maxima into slot `slot` of the member: one atomic max per value,
// the non-physical flag as value 7
template <int EQ, int NW>
__device__ __forceinline__ void coop_publish(Maxima<EQ> &mx, double *red, GMEM unsigned long long *am, int slot)
{
    resident_wave_maxima<EQ, NW>(mx, red, 0);
    __syncthreads();
    const int t = threadIdx.x;
    if (t < Maxima<EQ>::NV || t == 7) {
        double x = red[t];
        for (int w = 1; w < NW; ++w) x = fmax(x, red[w * 8 + t]);
        __hip_atomic_fetch_max(&am[slot * AMAX_VALS + t], as_bits(x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// every thread: the maxima of slot `slot` (after the barrier that completes them)
template <int EQ>
__device__ __forceinline__ void coop_read(GMEM unsigned long long *am, int slot, double (&cm)[8], Ctrl &C)
{
#pragma unroll
    for (int i = 0; i < 8; ++i) cm[i] = 0.0;
#pragma unroll
    for (int i = 0; i < Maxima<EQ>::NV; ++i)
        cm[i] = as_double(__hip_atomic_load(&am[slot * AMAX_VALS + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (__hip_atomic_load(&am[slot * AMAX_VALS + 7], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0ull)
        C.status |= 1;
}

template <int EQ, int ORDER, int MODE, bool CH>
__device__ __forceinline__ bool coop_stage(const KParams &P, const Inst &I, const double *in, const double *base,
                                           double *out, double *wl, double *red, GMEM unsigned long long *am,
                                           GMEM unsigned *bar, unsigned &nb, int s, double (&cm)[8], Ctrl &C,
                                           double dt)
{
    constexpr int NW = RES_BLOCK / 64;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int slot = s % 3;  // stage s writes slot s mod 3 and clears the next one
    if (blockIdx.x == 0 && threadIdx.x < AMAX_VALS) am[((s + 1) % 3) * AMAX_VALS + threadIdx.x] = 0ull;
    Maxima<EQ> mx;
    mx.reset();
    line_stage<EQ, ORDER, MODE, CH>(P, I, I.nx, in, base, out, wl, cm, dt, (int)blockIdx.x * NW + wv,
                                    (int)gridDim.x * NW, mx);
    coop_publish<EQ, NW>(mx, red, am, slot);
    if (!grid_barrier(bar, ++nb * gridDim.x)) return false;
    coop_read<EQ>(am, slot, cm, C);
    return true;
}

// bar: the plan's barrier words; the member's maxima slots and bar are zero at launch
template <int EQ, int ORDER, bool CH>
__global__ __launch_bounds__(RES_BLOCK) void coop_1d(KParams P, int nsteps, unsigned *bar_)
{
    constexpr int NW = RES_BLOCK / 64, NC = NodeTraits<EQ>::NC;
    using RW = ResWave<EQ, ORDER>;
    __shared__ double wls[NW * RW::DOUBLES];
    __shared__ double red[NW * 8];
    const Inst &I = P.inst[0];
    const int n = I.nx, tid = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    double *wl = wls + wv * RW::DOUBLES;
    // global memory, so that the stage's loads and stores compile to global instructions
    double *un = (double *)gmem(I.u), *w1 = (double *)gmem(I.w1), *w2 = (double *)gmem(I.w2);
    GMEM unsigned long long *am = gmem(I.amax);
    GMEM unsigned *bar = gmem(bar_);
    Ctrl C = *I.ctrl;
    unsigned nb = 0;  // barriers passed
    double cm[8];
    bool ok;
    {
        // maxima of u^n into slot 0
        const double idx = 1.0 / I.dx, idy = 1.0 / I.dy;
        Maxima<EQ> mx;
        mx.reset();
        for (int j = (int)blockIdx.x * RES_BLOCK + tid; j < n; j += (int)gridDim.x * RES_BLOCK) {
            double U[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) U[c] = un[c * n + j];
            mx.add(U, P.gamma, idx, idy);
        }
        coop_publish<EQ, NW>(mx, red, am, 0);
        ok = grid_barrier(bar, ++nb * gridDim.x);
        if (ok) coop_read<EQ>(am, 0, cm, C);
    }
    for (int step = 0; ok && step < nsteps; ++step) {
        if (!control_update<EQ>(C, cm[0], cm[2], cm[6], I.dx, I.adv)) break;  // the same in every thread
        const double dt = C.dt;
        ok = coop_stage<EQ, ORDER, M_S1, CH>(P, I, un, un, w1, wl, red, am, bar, nb, 1, cm, C, dt) &&
             coop_stage<EQ, ORDER, M_S2, CH>(P, I, w1, un, w2, wl, red, am, bar, nb, 2, cm, C, dt) &&
             coop_stage<EQ, ORDER, M_S3, CH>(P, I, w2, un, un, wl, red, am, bar, nb, 3, cm, C, dt);
    }
    if (blockIdx.x == 0 && tid == 0) {
        if (!ok) C.status |= 2;
        *I.ctrl = C;
    }
}

// zero the member's maxima slots and the barrier words before a cooperative launch
__global__ void coop_reset(unsigned long long *amax, unsigned *bar)
{
    const int t = threadIdx.x;
    if (t < AMAX_SLOTS * AMAX_VALS) amax[t] = 0ull;
    if (t < 2) bar[t] = 0u;
}

// bind caller pointers into a member's descriptor (kernel arguments are
// captured at launch, so the host values need not outlive the call)
__global__ void patch_inst(Inst *inst, int k, const double *u, double *lx, int set_lx)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        inst[k].u = const_cast<double *>(u);
        if (set_lx) inst[k].lx = lx;
    }
}

// clear the done flag of every member (before an evaluation outside the time loop)
__global__ void clear_done(KParams P)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < P.hdr->n_inst) P.inst[k].ctrl->done = 0;
}

// replace a member's control block (pool admission and retirement); info, if
// given, receives the old block's done flag, status, step count and time
__global__ void set_ctrl(Ctrl *c, Ctrl v, double *info)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (info) {
            info[0] = c->done;
            info[1] = c->status;
            info[2] = (double)c->steps;
            info[3] = c->t;
        }
        *c = v;
    }
}

// copy between a dense and a row-padded layout (pool admission and retirement)
__global__ void copy_pitched(const double *src, long long sp, double *dst, long long dp, int width, long long rows)
{
    for (long long r = blockIdx.y; r < rows; r += gridDim.y)
        for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < width; x += gridDim.x * blockDim.x)
            dst[(long long)r * dp + x] = src[(long long)r * sp + x];
}

// host-given step size for a single step (all instances)
__global__ void set_dt(KParams P, double dt)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.hdr->n_inst) return;
    Ctrl &C = *P.inst[k].ctrl;
    C.dt = dt;
    C.done = 0;
}

// ---------------------------------------------------------------------------
// kernel selection and launchers
using KFn = void (*)(KParams);
using KFn2 = void (*)(KParams, int);

template <int EQ, int ORDER, bool REC, bool CH> static KFn pick_x_mode(int mode)
{
    switch (mode) {
    case M_RHS: return sweep_x<EQ, ORDER, M_RHS, REC, CH>;
    case M_S1: return sweep_x<EQ, ORDER, M_S1, REC, CH>;
    case M_S2: return sweep_x<EQ, ORDER, M_S2, REC, CH>;
    default: return sweep_x<EQ, ORDER, M_S3, REC, CH>;
    }
}
template <int EQ, bool REC, bool CH> static KFn pick_x_order(int order, int mode)
{
    return order == 7 ? pick_x_mode<EQ, 7, REC, CH>(mode) : pick_x_mode<EQ, 5, REC, CH>(mode);
}
template <int EQ, bool CH> static KFn pick_x_rec(int order, int mode, bool rec)
{
    return rec ? pick_x_order<EQ, true, CH>(order, mode) : pick_x_order<EQ, false, CH>(order, mode);
}
// ch: characteristic fields (advection has one variable and always takes this path)
static KFn pick_x(int eq, int order, int mode, bool rec, bool ch)
{
    if (eq == ADVECTION) return pick_x_rec<ADVECTION, true>(order, mode, rec);
    if (eq == EULER1D) return ch ? pick_x_rec<EULER1D, true>(order, mode, rec) : pick_x_rec<EULER1D, false>(order, mode, rec);
    return ch ? pick_x_rec<EULER2D, true>(order, mode, rec) : pick_x_rec<EULER2D, false>(order, mode, rec);
}
template <int ORDER, bool REC, int YW, bool CH> static KFn pick_y_mode(int mode)
{
    switch (mode) {
    case M_RHS: return sweep_y<ORDER, M_RHS, REC, YW, CH>;
    case M_S1: return sweep_y<ORDER, M_S1, REC, YW, CH>;
    case M_S2: return sweep_y<ORDER, M_S2, REC, YW, CH>;
    default: return sweep_y<ORDER, M_S3, REC, YW, CH>;
    }
}
template <int YW, bool CH> static KFn pick_y_w(int order, int mode, bool rec)
{
    if (order == 7) return rec ? pick_y_mode<7, true, YW, CH>(mode) : pick_y_mode<7, false, YW, CH>(mode);
    return rec ? pick_y_mode<5, true, YW, CH>(mode) : pick_y_mode<5, false, YW, CH>(mode);
}
static KFn pick_y(int order, int mode, bool rec, int yw, bool ch)
{
    if (ch) return yw == 4 ? pick_y_w<4, true>(order, mode, rec) : pick_y_w<8, true>(order, mode, rec);
    return yw == 4 ? pick_y_w<4, false>(order, mode, rec) : pick_y_w<8, false>(order, mode, rec);
}
static KFn pick_maxima(int eq)
{
    return eq == ADVECTION ? state_maxima<ADVECTION> : (eq == EULER1D ? state_maxima<EULER1D> : state_maxima<EULER2D>);
}
static KFn pick_control(int eq)
{
    return eq == ADVECTION ? step_control<ADVECTION> : (eq == EULER1D ? step_control<EULER1D> : step_control<EULER2D>);
}

static hipError_t launch(KFn fn, int grid, int block, const KParams &p, hipStream_t s)
{
    KParams copy = p;
    void *args[] = {&copy};
    return hipLaunchKernel((const void *)fn, dim3(grid > 0 ? grid : 1), dim3(block), args, 0, s);
}

static int occupancy(KFn fn)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void *)fn, BLOCK, 0) != hipSuccess || n < 1) n = 1;
    return n;
}

hipError_t launch_sweep_x(int eq, int order, int mode, bool rec, bool ch, const KParams &p, int grid, hipStream_t s)
{
    return launch(pick_x(eq, order, mode, rec, ch), grid, BLOCK, p, s);
}

hipError_t launch_sweep_y(int order, int mode, bool rec, bool ch, int yw, const KParams &p, int grid, hipStream_t s)
{
    return launch(pick_y(order, mode, rec, yw, ch), grid, BLOCK, p, s);
}

hipError_t launch_state_maxima(int eq, const KParams &p, int grid, hipStream_t s)
{
    return launch(pick_maxima(eq), grid, BLOCK, p, s);
}

hipError_t launch_reset_maxima(const KParams &p, int n_inst, hipStream_t s)
{
    const int total = n_inst * AMAX_SLOTS * AMAX_VALS;
    return launch(reset_maxima, (total + BLOCK - 1) / BLOCK, BLOCK, p, s);
}

hipError_t launch_step_control(int eq, const KParams &p, int n_inst, hipStream_t s)
{
    return launch(pick_control(eq), (n_inst + 63) / 64, 64, p, s);
}

hipError_t launch_set_dt(const KParams &p, int n_inst, double dt, hipStream_t s)
{
    KParams copy = p;
    void *args[] = {&copy, &dt};
    return hipLaunchKernel((const void *)set_dt, dim3((n_inst + 63) / 64), dim3(64), args, 0, s);
}

hipError_t launch_patch_inst(Inst *inst, int k, const double *u, double *lx, bool set_lx, hipStream_t s)
{
    int flag = set_lx ? 1 : 0;
    void *args[] = {&inst, &k, &u, &lx, &flag};
    return hipLaunchKernel((const void *)patch_inst, dim3(1), dim3(64), args, 0, s);
}

hipError_t launch_clear_done(const KParams &p, int n_inst, hipStream_t s)
{
    return launch(clear_done, (n_inst + 63) / 64, 64, p, s);
}

hipError_t launch_set_ctrl(Ctrl *c, const Ctrl &v, double *info, hipStream_t s)
{
    Ctrl copy = v;
    void *args[] = {&c, &copy, &info};
    return hipLaunchKernel((const void *)set_ctrl, dim3(1), dim3(64), args, 0, s);
}

hipError_t launch_copy_pitched(const double *src, long long sp, double *dst, long long dp, int width,
                               long long rows, hipStream_t s)
{
    if (width <= 0 || rows <= 0) return hipSuccess;
    const dim3 grid((unsigned)std::min((width + 255) / 256, 64), (unsigned)std::min(rows, 8192ll));
    void *args[] = {&src, &sp, &dst, &dp, &width, &rows};
    return hipLaunchKernel((const void *)copy_pitched, grid, dim3(256), args, 0, s);
}

using KFn2c = void (*)(KParams, int, unsigned *);

template <int NW> static KFn2 pick_resident_w(int eq, int order, bool ch)
{
    if (eq == ADVECTION) return order == 7 ? resident_1d<ADVECTION, 7, true, NW> : resident_1d<ADVECTION, 5, true, NW>;
    if (ch) return order == 7 ? resident_1d<EULER1D, 7, true, NW> : resident_1d<EULER1D, 5, true, NW>;
    return order == 7 ? resident_1d<EULER1D, 7, false, NW> : resident_1d<EULER1D, 5, false, NW>;
}

static KFn2 pick_resident(int eq, int order, bool ch) { return pick_resident_w<RES_BLOCK / 64>(eq, order, ch); }

hipError_t launch_resident(int eq, int order, bool ch, int block, const KParams &p, int n_inst, int nsteps,
                           size_t lds, hipStream_t s)
{
    if (eq == EULER2D || block != RES_BLOCK) return hipErrorInvalidValue;
    const KFn2 fn = pick_resident(eq, order, ch);
    // dynamic LDS beyond the default limit must be allowed per kernel
    const hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    KParams copy = p;
    void *args[] = {&copy, &nsteps};
    return hipLaunchKernel((const void *)fn, dim3(n_inst), dim3(block), args, lds, s);
}

static KFn2c pick_coop(int eq, int order, bool ch)
{
    if (eq == ADVECTION) return order == 7 ? coop_1d<ADVECTION, 7, true> : coop_1d<ADVECTION, 5, true>;
    if (ch) return order == 7 ? coop_1d<EULER1D, 7, true> : coop_1d<EULER1D, 5, true>;
    return order == 7 ? coop_1d<EULER1D, 7, false> : coop_1d<EULER1D, 5, false>;
}

int coop_max_groups(int eq, int order, bool ch)
{
    int dev = 0, cus = 0, coop = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)pick_coop(eq, order, ch), RES_BLOCK, 0) !=
        hipSuccess)
        return 0;
    return cus * per_cu;
}

hipError_t launch_coop(int eq, int order, bool ch, int groups, const KParams &p, int nsteps,
                       unsigned long long *amax, unsigned *bar, hipStream_t s, bool *refused)
{
    *refused = false;
    if (eq == EULER2D || groups < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(coop_reset, dim3(1), dim3(64), 0, s, amax, bar);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    KParams copy = p;
    void *args[] = {&copy, &nsteps, &bar};
    const hipError_t ce = hipLaunchCooperativeKernel((const void *)pick_coop(eq, order, ch), dim3(groups),
                                                     dim3(RES_BLOCK), args, 0, s);
    *refused = ce != hipSuccess;
    return ce;
}

size_t resident_lds_limit()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
    // the kernel's static LDS (control copy, flag) comes on top of the dynamic part
    return v > 256 ? (size_t)v - 256 : 0;
}

int resident_groups_per_cu(int eq, int order, bool ch)
{
    int n = 0;
    if (eq == EULER2D ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void *)pick_resident(eq, order, ch), RES_BLOCK, 0) !=
            hipSuccess)
        return 0;
    return n;
}

int occupancy_x(int eq, int order, int mode, bool rec, bool ch) { return occupancy(pick_x(eq, order, mode, rec, ch)); }
int occupancy_y(int order, int mode, bool rec, bool ch, int yw)
{
    return occupancy(pick_y(order, mode, rec, yw, ch));
}
int occupancy_maxima(int eq) { return occupancy(pick_maxima(eq)); }

}  // namespace enoao
