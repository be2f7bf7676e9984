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
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "enoao_common.hpp"
#include "enoao_device.hpp"
#include "enoao_kernels.hpp"

namespace enoao {

__device__ __forceinline__ int bc_map(int k, int n, int bc)
{
    if (bc == BC_PERIODIC) {
        int r = k % n;
        return r < 0 ? r + n : r;
    }
    return k < 0 ? 0 : (k >= n ? n - 1 : k);
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
    double v[7];
    int bad;
    __device__ void reset()
    {
#pragma unroll
        for (int i = 0; i < 7; ++i) v[i] = 0.0;
        bad = 0;
    }
    // U in the natural component order
    __device__ void add(const double *U, double gamma, double dx, double dy)
    {
        if constexpr (EQ == ADVECTION) {
            bad |= !(U[0] == U[0]);
        } else if constexpr (EQ == EULER1D) {
            const double rho = U[0], u = U[1] / rho;
            const double p = (gamma - 1.0) * (U[2] - 0.5 * rho * (u * u));
            const double c = sqrt(gamma * p / rho);
            bad |= !(rho > 0.0 && p > 0.0);
            v[0] = fmax(v[0], fabs(u - c));
            v[1] = fmax(v[1], fabs(u));
            v[2] = fmax(v[2], fabs(u + c));
        } else {
            const double rho = U[0], u = U[1] / rho, w = U[2] / rho;
            const double p = (gamma - 1.0) * (U[3] - 0.5 * rho * (u * u + w * w));
            const double c = sqrt(gamma * p / rho);
            bad |= !(rho > 0.0 && p > 0.0);
            v[0] = fmax(v[0], fabs(u - c));
            v[1] = fmax(v[1], fabs(u));
            v[2] = fmax(v[2], fabs(u + c));
            v[3] = fmax(v[3], fabs(w - c));
            v[4] = fmax(v[4], fabs(w));
            v[5] = fmax(v[5], fabs(w + c));
            v[6] = fmax(v[6], (fabs(u) + c) / dx + (fabs(w) + c) / dy);
        }
    }
    // workgroup reduction, then one atomic per value into the instance's slot
    __device__ void flush(const Inst &I, int slot, double *red)
    {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
        for (int i = 0; i < 7; ++i) {
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
            for (int i = 0; i < 7; ++i) red[wave * 8 + i] = v[i];
            red[wave * 8 + 7] = (double)b;
        }
        __syncthreads();
        if (threadIdx.x < 8) {
            double x = red[threadIdx.x];
            for (int w = 1; w < BLOCK / 64; ++w) x = fmax(x, red[w * 8 + threadIdx.x]);
            if (threadIdx.x < 7) {
                if (EQ != ADVECTION && slot >= 0)
                    atomicMax(&I.amax[slot * AMAX_VALS + threadIdx.x], as_bits(x));
            } else if (x != 0.0) {
                atomicOr(&I.ctrl->status, 1);
            }
        }
        __syncthreads();
        reset();
    }
};

// ---------------------------------------------------------------------------
// One face: window node t (t = 0 .. 2G-1) of face j+1/2 is node j-H+t; the
// plus side reads nodes j-H .. j+H, the minus side the mirror j+1+H .. j+1-H.

// Characteristic fields F0 (and F1 >= 0) of an Euler face: project U and F of
// every stencil node (the compiler drops the rows not used by these fields),
// split, reconstruct both sides.  Taking the fields in two passes halves the
// live window registers.
template <int NC, int ORDER, int F0, int F1>
__device__ __forceinline__ void field_pass(const double *w0, int qs, int ns, const RoeState &r, const double *al,
                                           double delta, double (&wh)[NC], int (&sel)[2 * NC])
{
    constexpr int H = ReconTraits<ORDER>::H, G = H + 1, W = 2 * H + 1;
    constexpr int NF = F1 >= 0 ? 2 : 1;
    constexpr int fs[2] = {F0, F1 >= 0 ? F1 : F0};
    double gp[NF][W], gm[NF][W];
    double U[NC], F[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        U[c] = w0[c * qs];
        F[c] = w0[(NC + c) * qs];
    }
#pragma unroll
    for (int t = 0; t < 2 * G; ++t) {
        // next node's LDS reads go out before this node's arithmetic
        double Un[NC], Fn[NC];
        if (t + 1 < 2 * G) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                Un[c] = w0[c * qs + (t + 1) * ns];
                Fn[c] = w0[(NC + c) * qs + (t + 1) * ns];
            }
        }
        double PU[NC], PF[NC];
        project<NC>(r, U, PU);
        project<NC>(r, F, PF);
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            const int s = fs[i];
            if (t < W) gp[i][t] = fma(al[s], PU[s], PF[s]);
            if (t >= 1) gm[i][2 * H + 1 - t] = fma(-al[s], PU[s], PF[s]);
        }
        if (t + 1 < 2 * G) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                U[c] = Un[c];
                F[c] = Fn[c];
            }
        }
        // bound the live ranges: at most two nodes' U and F in flight
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        const int s = fs[i];
        // window = 2 * field_scale * w^(+/-)
        const double sc = 2.0 * field_scale<NC>(s);
        int sp, sm;
        const double hp = Recon<ORDER>::run(gp[i], sc * delta, sp);
        const double hm = Recon<ORDER>::run(gm[i], sc * delta, sm);
        wh[s] = (hp + hm) * (1.0 / sc);
        sel[2 * s] = sp;
        sel[2 * s + 1] = sm;
    }
}

template <int EQ, int ORDER>
__device__ __forceinline__ void face_flux(const double *w0, int qs, int ns, const double *al, double gm1,
                                          double delta, double adv,
                                          double (&Fh)[NodeTraits<EQ>::NC], int (&sel)[2 * NodeTraits<EQ>::NC])
{
    constexpr int H = ReconTraits<ORDER>::H, G = H + 1, W = 2 * H + 1;
    if constexpr (EQ == ADVECTION) {
        // f^(+/-) = (a u +/- alpha u)/2, reconstructed as 2 f^(+/-)
        double gp[W], gm[W];
#pragma unroll
        for (int t = 0; t < 2 * G; ++t) {
            const double u = w0[t * ns];
            const double au = adv * u;
            if (t < W) gp[t] = fma(al[0], u, au);
            if (t >= 1) gm[2 * H + 1 - t] = fma(-al[0], u, au);
        }
        int sp, sm;
        const double hp = Recon<ORDER>::run(gp, 2.0 * delta, sp);
        const double hm = Recon<ORDER>::run(gm, 2.0 * delta, sm);
        Fh[0] = 0.5 * (hp + hm);
        sel[0] = sp;
        sel[1] = sm;
    } else {
        constexpr int NC = NodeTraits<EQ>::NC, QR = 2 * NC;
        const double *nl = w0 + (G - 1) * ns, *nr = w0 + G * ns;
        RoeState r;
        if constexpr (EQ == EULER1D)
            r = roe_state(nl[QR * qs], nl[(QR + 1) * qs], 0.0, nl[(QR + 2) * qs], nr[QR * qs],
                          nr[(QR + 1) * qs], 0.0, nr[(QR + 2) * qs], gm1);
        else
            r = roe_state(nl[QR * qs], nl[(QR + 1) * qs], nl[(QR + 2) * qs], nl[(QR + 3) * qs], nr[QR * qs],
                          nr[(QR + 1) * qs], nr[(QR + 2) * qs], nr[(QR + 3) * qs], gm1);
        double wh[NC];
        if constexpr (NC == 4) {
            field_pass<4, ORDER, 0, 3>(w0, qs, ns, r, al, delta, wh, sel);
            field_pass<4, ORDER, 1, 2>(w0, qs, ns, r, al, delta, wh, sel);
        } else {
            field_pass<3, ORDER, 0, 2>(w0, qs, ns, r, al, delta, wh, sel);
            field_pass<3, ORDER, 1, -1>(w0, qs, ns, r, al, delta, wh, sel);
        }
        back_project<NC>(r, wh, Fh);
    }
}

template <int EQ>
__device__ __forceinline__ void load_alpha(const Inst &I, int slot, bool ydir, double *al)
{
    constexpr int NC = NodeTraits<EQ>::NC;
    if constexpr (EQ == ADVECTION) {
        al[0] = fabs(I.adv);
    } else {
        const unsigned long long *a = I.amax + slot * AMAX_VALS + (ydir ? 3 : 0);
        const double m0 = as_double(a[0]), m1 = as_double(a[1]), m2 = as_double(a[2]);
        al[0] = m0;
        al[1] = m1;
        if (NC == 4) al[2] = m1;
        al[NC - 1] = m2;
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

template <int MODE> __device__ __forceinline__ const double *stage_in(const Inst &I)
{
    return MODE == M_S2 ? I.w1 : (MODE == M_S3 ? I.w2 : I.u);
}
template <int MODE> __device__ __forceinline__ double *stage_out(const Inst &I)
{
    return MODE == M_S1 ? I.w1 : (MODE == M_S2 ? I.w2 : I.u);
}

// ---------------------------------------------------------------------------
// x-sweep.  Each wave: one segment of a grid line (64 faces, 63 cells).
// Tiles are software-pipelined: the global operands of tile t+1 are loaded into
// registers while tile t is reconstructed, so the memory latency hides behind
// the face arithmetic.
#ifndef ENOAO_SWEEP_WAVES_PER_EU
#define ENOAO_SWEEP_WAVES_PER_EU 1
#endif

struct XSeg {
    int k;        // instance
    bool ok;      // this wave has a segment in the tile
    bool active;  // the instance is still stepping (uniform over the tile)
    int row, sx;  // grid line and first cell of the segment
};

// (segment counts of an instance fit 32 bits: ny * ceil(nx / 63) segments)
__device__ __forceinline__ XSeg x_segment(const KParams &P, int n_inst, long long tile, int wseg)
{
    XSeg g;
    g.k = find_inst<true>(P.inst, n_inst, tile);
    const Inst &I = P.inst[g.k];
    const unsigned seg = (unsigned)(tile - I.xtile0) * XW_SEGS + (unsigned)wseg;
    const unsigned spr = (unsigned)I.segs_per_row;
    g.ok = seg < (unsigned)I.ny * spr;
    const unsigned row = seg / spr;
    g.row = g.ok ? (int)row : 0;
    g.sx = g.ok ? (int)(seg - row * spr) * XW_CELLS : 0;
    g.active = I.ctrl->done == 0;
    return g;
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
// positions lane and lane + 64) and, for a 1D stage 2 or 3, u^n at its cell
template <int NC> struct XPre {
    double U[2][NC];
    double base[NC];
};

template <int EQ, int MODE, int G>
__device__ __forceinline__ void x_prefetch(const Inst &I, const XSeg &g, int lane, XPre<NodeTraits<EQ>::NC> &pre)
{
    constexpr int NC = NodeTraits<EQ>::NC, NN = XW_FACES + 2 * G - 1;
    if (!g.ok || !g.active) return;
    const int nx = I.nx;
    const long long plane = (long long)nx * I.ny;
    const double *rowp = stage_in<MODE>(I) + (long long)g.row * nx;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int i = lane + 64 * j;
        if (i < NN) {
            const int x = bc_map(g.sx - G + i, nx, I.bcx);
#pragma unroll
            for (int c = 0; c < NC; ++c) pre.U[j][c] = rowp[c * plane + x];
        }
    }
    if constexpr (EQ != EULER2D && (MODE == M_S2 || MODE == M_S3)) {
        const int x = g.sx + lane;
        if (lane < XW_CELLS && x < nx) {
            const double *b = I.u + (long long)g.row * nx + x;
#pragma unroll
            for (int c = 0; c < NC; ++c) pre.base[c] = b[c * plane];
        }
    }
}

template <int EQ, int ORDER, int MODE, bool REC>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(ENOAO_SWEEP_WAVES_PER_EU))) void sweep_x(KParams P)
{
    constexpr int NC = NodeTraits<EQ>::NC, NQ = NodeTraits<EQ>::NQ;
    constexpr int H = ReconTraits<ORDER>::H, G = H + 1;
    constexpr int NN = XW_FACES + 2 * G - 1;  // nodes staged per segment
    constexpr int NNP = NN + 1;
    constexpr bool FULL = (EQ != EULER2D) && (MODE != M_RHS);  // 1D stage: combine + maxima here
    __shared__ double lds[NQ * XW_SEGS * NNP];
    __shared__ double fh[NC * XW_SEGS * XW_FACES];
    __shared__ double red[(BLOCK / 64) * 8];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wseg = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n_inst = P.hdr->n_inst;
    const long long T = P.hdr->xtiles_total;
    const long long t0 = (long long)blockIdx.x * T / gridDim.x, t1 = (long long)(blockIdx.x + 1) * T / gridDim.x;
    Maxima<EQ> mx;
    mx.reset();
    int cur = -1;
    XPre<NC> pre;
    XSeg gn{};  // segment of the next tile
    if (t0 < t1) {
        gn = x_segment(P, n_inst, t0, wseg);
        x_prefetch<EQ, MODE, G>(P.inst[gn.k], gn, lane, pre);
    }

    // Each wave owns its segment's LDS (nodes and face fluxes), so within the
    // tile loop the waves synchronise only with themselves; all waves of a
    // workgroup walk the same tiles, so the maxima flush (a workgroup
    // reduction) is reached by all of them together.
    for (long long tile = t0; tile < t1; ++tile) {
        const XSeg g = gn;
        const Inst &I = P.inst[g.k];
        if (FULL && g.k != cur && cur >= 0) mx.flush(P.inst[cur], P.r_out, red);
        cur = g.k;
        if (g.active && MODE != M_RHS && P.r_zero >= 0 && tile == I.xtile0 && tid < AMAX_VALS)
            I.amax[P.r_zero * AMAX_VALS + tid] = 0ull;

        // stage this tile's nodes (flux, Roe inputs) into LDS
        double *L = lds + wseg * NNP;
        if (g.active && g.ok) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int i = lane + 64 * j;
                if (i < NN) {
                    double q[NQ];
                    node_quantities<EQ>(pre.U[j], P.gm1, q);
#pragma unroll
                    for (int m = 0; m < NQ; ++m) L[m * XW_SEGS * NNP + i] = q[m];
                }
            }
        }
        double base[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) base[c] = pre.base[c];
        // issue the next tile's loads before this tile's arithmetic
        if (tile + 1 < t1) {
            gn = x_segment(P, n_inst, tile + 1, wseg);
            x_prefetch<EQ, MODE, G>(P.inst[gn.k], gn, lane, pre);
        }
        if (!g.active) continue;  // uniform: all waves of a tile belong to one instance
        wave_sync();

        const int nx = I.nx, ny = I.ny;
        const long long plane = (long long)nx * ny;
        double al[NC];
        load_alpha<EQ>(I, P.r_in, false, al);
        const int f = g.sx + lane;  // face index along the line
        if (g.ok) {
            double Fh[NC];
            int sel[2 * NC];
            face_flux<EQ, ORDER>(L + lane, XW_SEGS * NNP, 1, al, P.gm1, P.delta, I.adv, Fh, sel);
#pragma unroll
            for (int c = 0; c < NC; ++c) fh[(c * XW_SEGS + wseg) * XW_FACES + lane] = Fh[c];
            if (REC && I.sel && f <= nx) {
                const long long xblock = (long long)ny * (nx + 1);
#pragma unroll
                for (int s = 0; s < NC; ++s) {
                    const long long o = (long long)(2 * s) * xblock + (long long)g.row * (nx + 1) + f;
                    I.sel[o] = (uint8_t)sel[2 * s];
                    I.sel[o + xblock] = (uint8_t)sel[2 * s + 1];
                }
            }
        }
        wave_sync();

        const int x = g.sx + lane;
        if (g.ok && lane < XW_CELLS && x < nx) {
            const double idx = -1.0 / I.dx;
            const long long o = (long long)g.row * nx + x;
            double Lc[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c)
                Lc[c] = (fh[(c * XW_SEGS + wseg) * XW_FACES + lane + 1] - fh[(c * XW_SEGS + wseg) * XW_FACES + lane]) * idx;
            if constexpr (!FULL) {
#pragma unroll
                for (int c = 0; c < NC; ++c) I.lx[c * plane + o] = Lc[c];
            } else {
                const double dt = I.ctrl->dt;
                double *out = stage_out<MODE>(I);
                double Un[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const double uin = L[c * XW_SEGS * NNP + lane + G];
                    Un[c] = rk_combine<MODE>(uin, base[c], dt, Lc[c]);
                    out[c * plane + o] = Un[c];
                }
                mx.add(Un, P.gamma, I.dx, I.dy);
            }
        }
        wave_sync();
    }
    if (FULL && cur >= 0) mx.flush(P.inst[cur], P.r_out, red);
}

// ---------------------------------------------------------------------------
// y-sweep (2D).  A workgroup: 16 columns x 16 faces along y, 16 x 15 cells.
// Momentum components are exchanged on load so the x-direction formulas apply.
// Pipelined like the x-sweep; the epilogue operands (x-part of L, u^n) are
// prefetched with the nodes.
struct YTile {
    int k;
    bool active;
    int sy, col0;  // first cell row, first column
};

__device__ __forceinline__ YTile y_tile(const KParams &P, int n_inst, long long tile)
{
    YTile t;
    t.k = find_inst<false>(P.inst, n_inst, tile);
    const Inst &I = P.inst[t.k];
    const long long tl = tile - I.ytile0;
    t.sy = (int)(tl % I.ytiles_per_row) * YT_CELLS;
    t.col0 = (int)(tl / I.ytiles_per_row) * YT_COLS;
    t.active = I.ctrl->done == 0;
    return t;
}

struct YPre {
    double U[2][4];
    double lx[4], base[4];
};

template <int MODE, int G>
__device__ __forceinline__ void y_prefetch(const Inst &I, const YTile &t, int tid, YPre &pre)
{
    constexpr int NR = YT_FACES + 2 * G - 1;
    const int perm[4] = {0, 2, 1, 3};
    if (!t.active) return;
    const int nx = I.nx, ny = I.ny;
    const long long plane = (long long)nx * ny;
    const double *in = stage_in<MODE>(I);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int i = tid + BLOCK * j;
        if (i < NR * YT_COLS) {
            const int r = i / YT_COLS, c0 = i % YT_COLS;
            const int y = bc_map(t.sy - G + r, ny, I.bcy);
            const int x = min(t.col0 + c0, nx - 1);
            const double *p = in + (long long)y * nx + x;
#pragma unroll
            for (int c = 0; c < 4; ++c) pre.U[j][c] = p[perm[c] * plane];
        }
    }
    const int fl = tid / YT_COLS, y = t.sy + fl, col = t.col0 + (tid & (YT_COLS - 1));
    if (fl < YT_CELLS && y < ny && col < nx) {
        const long long o = (long long)y * nx + col;
#pragma unroll
        for (int c = 0; c < 4; ++c) pre.lx[c] = I.lx[c * plane + o];
        if constexpr (MODE == M_S2 || MODE == M_S3) {
#pragma unroll
            for (int c = 0; c < 4; ++c) pre.base[c] = I.u[c * plane + o];
        }
    }
}

template <int ORDER, int MODE, bool REC>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(ENOAO_SWEEP_WAVES_PER_EU))) void sweep_y(KParams P)
{
    constexpr int NC = 4, NQ = 12;
    constexpr int H = ReconTraits<ORDER>::H, G = H + 1;
    constexpr int NR = YT_FACES + 2 * G - 1;  // node rows staged
    constexpr int QS = NR * YT_COLS;         // LDS stride between quantities
    __shared__ double lds[NQ * QS];
    __shared__ double fh[NC * YT_FACES * YT_COLS];
    __shared__ double red[(BLOCK / 64) * 8];
    // epilogue operands of the tile (x-part of L, u^n), staged from the prefetch
    // registers so they are not held through the face arithmetic
    constexpr bool BASE = MODE == M_S2 || MODE == M_S3;
    __shared__ double elx[NC * BLOCK];
    __shared__ double ebase[BASE ? NC * BLOCK : 1];
    const int perm[4] = {0, 2, 1, 3};

    const int tid = threadIdx.x, cc = tid & (YT_COLS - 1), fl = tid / YT_COLS;
    const int n_inst = P.hdr->n_inst;
    const long long T = P.hdr->ytiles_total;
    const long long t0 = (long long)blockIdx.x * T / gridDim.x, t1 = (long long)(blockIdx.x + 1) * T / gridDim.x;
    Maxima<EULER2D> mx;
    mx.reset();
    int cur = -1;
    YPre pre;
    if (t0 < t1) {
        const YTile y0 = y_tile(P, n_inst, t0);
        y_prefetch<MODE, G>(P.inst[y0.k], y0, tid, pre);
    }

    for (long long tile = t0; tile < t1; ++tile) {
        const YTile t = y_tile(P, n_inst, tile);
        const Inst &I = P.inst[t.k];
        if (MODE != M_RHS && t.k != cur && cur >= 0) mx.flush(P.inst[cur], P.r_out, red);
        cur = t.k;

        if (t.active) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int i = tid + BLOCK * j;
                if (i < NR * YT_COLS) {
                    double q[NQ];
                    node_quantities<EULER2D>(pre.U[j], P.gm1, q);
#pragma unroll
                    for (int m = 0; m < NQ; ++m) lds[m * QS + i] = q[m];
                }
            }
        }
        if (t.active) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                elx[c * BLOCK + tid] = pre.lx[c];
                if constexpr (BASE) ebase[c * BLOCK + tid] = pre.base[c];
            }
        }
        if (tile + 1 < t1) {
            const YTile tn = y_tile(P, n_inst, tile + 1);
            y_prefetch<MODE, G>(P.inst[tn.k], tn, tid, pre);
        }
        if (!t.active) continue;
        __syncthreads();

        const int nx = I.nx, ny = I.ny;
        const long long plane = (long long)nx * ny;
        double al[NC];
        load_alpha<EULER2D>(I, P.r_in, true, al);
        const int col = t.col0 + cc, f = t.sy + fl;
        {
            double Fh[NC];
            int sel[2 * NC];
            face_flux<EULER2D, ORDER>(lds + fl * YT_COLS + cc, QS, YT_COLS, al, P.gm1, P.delta, 0.0, Fh, sel);
#pragma unroll
            for (int c = 0; c < NC; ++c) fh[(c * YT_FACES + fl) * YT_COLS + cc] = Fh[c];
            if (REC && I.sel && col < nx && f <= ny) {
                const long long xblock = (long long)ny * (nx + 1), yblock = (long long)(ny + 1) * nx;
                const long long ybase = (long long)NC * 2 * xblock;
#pragma unroll
                for (int s = 0; s < NC; ++s) {
                    const long long o = ybase + (long long)(2 * s) * yblock + (long long)f * nx + col;
                    I.sel[o] = (uint8_t)sel[2 * s];
                    I.sel[o + yblock] = (uint8_t)sel[2 * s + 1];
                }
            }
        }
        __syncthreads();

        const int y = t.sy + fl;
        if (fl < YT_CELLS && y < ny && col < nx) {
            const double idy = -1.0 / I.dy;
            const long long o = (long long)y * nx + col;
            double Ly[NC];  // natural component order
#pragma unroll
            for (int c = 0; c < NC; ++c)
                Ly[perm[c]] = (fh[(c * YT_FACES + fl + 1) * YT_COLS + cc] - fh[(c * YT_FACES + fl) * YT_COLS + cc]) * idy;
            if constexpr (MODE == M_RHS) {
#pragma unroll
                for (int c = 0; c < NC; ++c) I.lx[c * plane + o] = elx[c * BLOCK + tid] + Ly[c];
            } else {
                const double dt = I.ctrl->dt;
                double *out = stage_out<MODE>(I);
                double Un[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const double uin = lds[perm[c] * QS + (fl + G) * YT_COLS + cc];
                    const double base = BASE ? ebase[c * BLOCK + tid] : 0.0;
                    Un[c] = rk_combine<MODE>(uin, base, dt, elx[c * BLOCK + tid] + Ly[c]);
                    out[c * plane + o] = Un[c];
                }
                mx.add(Un, P.gamma, I.dx, I.dy);
            }
        }
        __syncthreads();
    }
    if (MODE != M_RHS && cur >= 0) mx.flush(P.inst[cur], P.r_out, red);
}

// ---------------------------------------------------------------------------
// Maxima of the input state (alpha for the first evaluation, CFL step).
template <int EQ>
__global__ __launch_bounds__(BLOCK) void state_maxima(KParams P)
{
    constexpr int NC = NodeTraits<EQ>::NC;
    __shared__ double red[(BLOCK / 64) * 8];
    const int tid = threadIdx.x, wseg = tid >> 6, lane = tid & 63;
    const int n_inst = P.hdr->n_inst;
    const long long T = P.hdr->xtiles_total;
    const long long t0 = (long long)blockIdx.x * T / gridDim.x, t1 = (long long)(blockIdx.x + 1) * T / gridDim.x;
    Maxima<EQ> mx;
    mx.reset();
    int cur = -1;
    for (long long tile = t0; tile < t1; ++tile) {
        const int k = find_inst<true>(P.inst, n_inst, tile);
        const Inst &I = P.inst[k];
        if (k != cur && cur >= 0) mx.flush(P.inst[cur], P.r_out, red);
        cur = k;
        const int nx = I.nx, ny = I.ny;
        const long long plane = (long long)nx * ny;
        const long long seg = (tile - I.xtile0) * XW_SEGS + wseg;
        if (seg < (long long)ny * I.segs_per_row && lane < XW_CELLS) {
            const int row = (int)(seg / I.segs_per_row), x = (int)(seg % I.segs_per_row) * XW_CELLS + lane;
            if (x < nx) {
                double U[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) U[c] = I.u[c * plane + (long long)row * nx + x];
                mx.add(U, P.gamma, I.dx, I.dy);
            }
        }
    }
    if (cur >= 0) mx.flush(P.inst[cur], P.r_out, red);
}

// zero all maxima slots and the status of every instance
__global__ void reset_maxima(KParams P)
{
    const int n = P.hdr->n_inst;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n * AMAX_SLOTS * AMAX_VALS;
         k += gridDim.x * blockDim.x) {
        const int i = k / (AMAX_SLOTS * AMAX_VALS), j = k % (AMAX_SLOTS * AMAX_VALS);
        P.inst[i].amax[j] = 0ull;
    }
}

// Time-step control, one thread per instance: CFL (or fixed) step from the
// maxima of the state at the start of the step, clipped to land on t_final.
template <int EQ>
__global__ void step_control(KParams P)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.hdr->n_inst) return;
    const Inst &I = P.inst[k];
    Ctrl &C = *I.ctrl;
    if (C.done) return;
    if (C.status != 0 || C.steps >= C.max_steps) { C.done = 1; return; }
    const double rem = C.t_final - C.t;
    if (!(rem > 0.0)) { C.done = 1; return; }
    double dt;
    if (C.dt_fixed > 0.0) {
        dt = C.dt_fixed;
    } else {
        const unsigned long long *a = I.amax;  // slot 0: the state u^n
        if constexpr (EQ == ADVECTION) {
            dt = C.cfl * I.dx / fabs(I.adv);
        } else if constexpr (EQ == EULER1D) {
            const double smax = fmax(as_double(a[0]), as_double(a[2]));  // max(|u|+c)
            if (!(smax > 0.0)) { C.status |= 1; C.done = 1; return; }
            dt = C.cfl * I.dx / smax;
        } else {
            const double smax = as_double(a[6]);
            if (!(smax > 0.0)) { C.status |= 1; C.done = 1; return; }
            dt = C.cfl / smax;
        }
    }
    const bool last = dt >= rem * (1.0 - 1e-10);
    if (last) dt = rem;
    C.dt = dt;
    C.t = last ? C.t_final : C.t + dt;
    C.steps = C.steps + 1;
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

template <int EQ, int ORDER, bool REC> static KFn pick_x_mode(int mode)
{
    switch (mode) {
    case M_RHS: return sweep_x<EQ, ORDER, M_RHS, REC>;
    case M_S1: return sweep_x<EQ, ORDER, M_S1, REC>;
    case M_S2: return sweep_x<EQ, ORDER, M_S2, REC>;
    default: return sweep_x<EQ, ORDER, M_S3, REC>;
    }
}
template <int EQ, bool REC> static KFn pick_x_order(int order, int mode)
{
    return order == 7 ? pick_x_mode<EQ, 7, REC>(mode) : pick_x_mode<EQ, 5, REC>(mode);
}
template <int EQ> static KFn pick_x_rec(int order, int mode, bool rec)
{
    return rec ? pick_x_order<EQ, true>(order, mode) : pick_x_order<EQ, false>(order, mode);
}
static KFn pick_x(int eq, int order, int mode, bool rec)
{
    if (eq == ADVECTION) return pick_x_rec<ADVECTION>(order, mode, rec);
    if (eq == EULER1D) return pick_x_rec<EULER1D>(order, mode, rec);
    return pick_x_rec<EULER2D>(order, mode, rec);
}
template <int ORDER, bool REC> static KFn pick_y_mode(int mode)
{
    switch (mode) {
    case M_RHS: return sweep_y<ORDER, M_RHS, REC>;
    case M_S1: return sweep_y<ORDER, M_S1, REC>;
    case M_S2: return sweep_y<ORDER, M_S2, REC>;
    default: return sweep_y<ORDER, M_S3, REC>;
    }
}
static KFn pick_y(int order, int mode, bool rec)
{
    if (order == 7) return rec ? pick_y_mode<7, true>(mode) : pick_y_mode<7, false>(mode);
    return rec ? pick_y_mode<5, true>(mode) : pick_y_mode<5, false>(mode);
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

hipError_t launch_sweep_x(int eq, int order, int mode, bool rec, const KParams &p, int grid, hipStream_t s)
{
    return launch(pick_x(eq, order, mode, rec), grid, BLOCK, p, s);
}

hipError_t launch_sweep_y(int order, int mode, bool rec, const KParams &p, int grid, hipStream_t s)
{
    return launch(pick_y(order, mode, rec), grid, BLOCK, p, s);
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

int occupancy_x(int eq, int order, int mode, bool rec) { return occupancy(pick_x(eq, order, mode, rec)); }
int occupancy_y(int order, int mode, bool rec) { return occupancy(pick_y(order, mode, rec)); }
int occupancy_maxima(int eq) { return occupancy(pick_maxima(eq)); }

}  // namespace enoao
