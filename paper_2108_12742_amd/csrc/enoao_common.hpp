// enoao_common.hpp -- structures shared by the host runtime and the HIP kernels.
//
// A "batch" is the unit every kernel works on: an array of instance
// descriptors in device memory plus the flattened lists of line tiles of all
// instances.  A single plan is a batch of one instance, so the plain, batched
// and served paths run the same kernels.
#pragma once

#include <stdint.h>

namespace enoao {

enum Equation : int { ADVECTION = 0, EULER1D = 1, EULER2D = 2 };
enum Bc : int { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1 };

// x-sweep tiles: each wave reconstructs 64 consecutive faces of one grid line
// and updates the 63 cells between them; a workgroup holds 4 such segments.
constexpr int XW_FACES = 64;
constexpr int XW_CELLS = XW_FACES - 1;
constexpr int XW_SEGS = 4;
// y-sweep tiles: each of the 4 waves of a workgroup owns a strip of w columns
// (w = 4 or 8, chosen per plan or batch) and w * 64/w = 64 lanes; a tile is
// 4w columns x 64/w cell rows.
// Default strip width per order (measured on the 2048^2 Euler workloads: 8 for
// order 5; 4 for order 7, whose wider strips stage more halo rows per face
// than its one wave per SIMD can hide).
constexpr int yw_default(int order) { return order == 7 ? 4 : 8; }
constexpr int yt_cells(int w) { return 64 / w; }
constexpr int yt_cols(int w) { return 4 * w; }
constexpr int BLOCK = 256;

// per-field maxima kept per instance: three ring slots of 8 values each
// (non-negative doubles stored as their IEEE bit patterns so that unsigned
// integer max is the floating-point max):
//   [0..2] max |u-c|, |u|, |u+c| along x    [3..5] same along y (v)
//   [6]    max (|u|+c)/dx + (|v|+c)/dy (2D time step)
constexpr int AMAX_VALS = 8;
constexpr int AMAX_SLOTS = 3;

// Time-loop control of one instance (device memory).
struct Ctrl {
    double dt;          // step size of the step in flight
    double t;           // time reached (after the step in flight)
    double t_final;     // end time (+inf: none)
    double cfl;         // CFL number for the device-computed step (if dt_fixed <= 0)
    double dt_fixed;    // > 0: constant step
    long long steps;    // steps taken
    long long max_steps;
    int done;           // 1: no further steps; kernels skip the instance
    int status;         // bit 0: non-physical state met
    int pad0, pad1;
};

// One instance of a batch (device memory).
struct Inst {
    double *u;                  // u^n: caller state, updated in place by stage 3
    double *w1, *w2;            // stage-1 and stage-2 states
    double *lx;                 // 2D: x-part of L; rhs: the L output
    unsigned long long *amax;   // AMAX_SLOTS x AMAX_VALS
    Ctrl *ctrl;
    uint8_t *sel;               // selection record or nullptr
    int nx, ny;
    int bcx, bcy;
    double dx, dy;
    double adv;                 // advection speed
    int segs_per_row;           // ceil(nx / XW_CELLS)
    int ytiles_per_row;         // ceil(ny / yt_cells(w)) tiles per column group (w: y strip width)
    int ycol_groups;            // ceil(nx / yt_cols(w))
    int pitch;                  // row pitch of every state buffer, elements (>= nx; planes pitch * ny apart)
    long long xtile0, ytile0;   // first x / y tile of this instance in the batch lists
    long long xtiles, ytiles;   // number of x / y tiles
};

// LDS-resident solver of small 1D members: one workgroup of RES_BLOCK threads
// holds a member's state and both Runge-Kutta stage states in LDS for a whole
// call; each of its waves stages the nodes of one 64-face segment at a time,
// and that segment's face fluxes, in LDS of its own.
constexpr int RES_BLOCK = 256;

// dynamic LDS bytes of a resident member of n nodes (nc components, nq staged
// quantities per node, halo width g, block threads): u^n and the two stage
// states, each wave's segment staging (nodes and face fluxes), two parities of
// per-wave maxima
constexpr unsigned long long resident_lds_bytes(int nc, int nq, int g, long long n, int block = RES_BLOCK)
{
    const long long nnp = 64 + 2 * g, waves = block / 64;
    return 8ull * (unsigned long long)(3 * nc * n + waves * (nq * nnp + nc * 64) + 2 * waves * 8);
}

// Batch header (device memory): kernels read the instance count and the tile
// totals from here, so a captured graph stays valid when the active set changes.
struct BatchHdr {
    int n_inst;
    int pad;
    long long xtiles_total, ytiles_total;
};

}  // namespace enoao
