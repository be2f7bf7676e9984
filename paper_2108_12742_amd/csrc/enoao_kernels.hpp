// enoao_kernels.hpp -- launch interface of the gfx950 kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include "enoao_common.hpp"

namespace enoao {

// what a sweep kernel does with the flux difference
enum Mode : int {
    M_RHS = 0,  // evaluate L of the caller state (1D: write L; 2D: x writes Lx, y adds Ly)
    M_S1 = 1,   // Runge-Kutta stage 1: input u^n, output w1
    M_S2 = 2,   // stage 2: input w1, output w2
    M_S3 = 3    // stage 3: input w2, output u^{n+1} (in place)
};

struct KParams {
    const BatchHdr *hdr;
    const Inst *inst;
    double gamma, gm1, delta;
    int r_in;    // maxima slot holding alpha of the stage input
    int r_out;   // slot receiving the maxima of the stage output (-1: none)
    int r_zero;  // slot cleared by the first kernel of the stage (-1: none)
    int flags;   // KF_* below
    int sel_slot;  // selection record a recording launch writes (0..2: the stage's record)
    // LDS-resident launches: member run by workgroup b (members by decreasing
    // size, so the small ones fill the machine behind the large; null: member b)
    const int *res_order;
    int res_first;  // first entry of res_order a resident launch covers
    // Persistent sweeps of a pool: the grid is sized for a full arena, and the
    // workgroups that share the tile list are as many as give tiles_per_wg
    // tiles each, at least grid_min (0: the whole grid shares it).
    int tiles_per_wg;
    int grid_min;
};

// every face takes the full selection (no wave-uniform shortcut); results are
// the same either way, which this flag lets a caller check
constexpr int KF_FULL_SELECTION = 1;

// ch: reconstruct in the characteristic fields of the Roe state (false: in the
// conserved components; advection ignores it)
hipError_t launch_sweep_x(int eq, int order, int mode, bool rec, bool ch, const KParams &p, int grid, hipStream_t s);
// yw: columns per wave strip of the y tiles (4 or 8; the members' y tile lists
// must have been built for the same width)
hipError_t launch_sweep_y(int order, int mode, bool rec, bool ch, int yw, const KParams &p, int grid, hipStream_t s);
hipError_t launch_state_maxima(int eq, const KParams &p, int grid, hipStream_t s);
hipError_t launch_reset_maxima(const KParams &p, int n_inst, hipStream_t s);
hipError_t launch_step_control(int eq, const KParams &p, int n_inst, hipStream_t s);
hipError_t launch_set_dt(const KParams &p, int n_inst, double dt, hipStream_t s);
hipError_t launch_patch_inst(Inst *inst, int k, const double *u, double *lx, bool set_lx, hipStream_t s);
hipError_t launch_clear_done(const KParams &p, int n_inst, hipStream_t s);
// *c = v on the stream (v passed by value: no host buffer outlives the call);
// info (device, 4 doubles, may be null) receives the old done, status, steps, t
hipError_t launch_set_ctrl(Ctrl *c, const Ctrl &v, double *info, hipStream_t s);
// rows of `width` doubles from src (pitch sp) to dst (pitch dp), pitches in doubles
hipError_t launch_copy_pitched(const double *src, long long sp, double *dst, long long dp, int width,
                               long long rows, hipStream_t s);
// nsteps controlled steps of every member (all 1D, all fitting the LDS), one
// workgroup per member; lds = dynamic LDS bytes per workgroup
// block: RES_BLOCK threads per workgroup; n_inst members from p.res_order[p.res_first]
hipError_t launch_resident(int eq, int order, bool ch, int block, const KParams &p, int n_inst, int nsteps,
                           size_t lds, hipStream_t s);
// largest dynamic LDS a resident workgroup may use on this device (0: none)
size_t resident_lds_limit();
// resident workgroups one CU can hold as far as registers and waves allow (LDS
// aside; 0: unknown)
int resident_groups_per_cu(int eq, int order, bool ch);

// Cooperative solver of one 1D member (p.inst[0]): nsteps controlled steps in one
// cooperative launch of `groups` workgroups of RES_BLOCK threads (each wave one
// or more 63-cell segments per stage), after zeroing the member's maxima slots
// (amax) and the two barrier words (bar).  *refused is set when the runtime
// turned the cooperative launch itself down (its error is returned; the zeroing
// has been enqueued).  coop_max_groups: the most workgroups such a launch can
// keep resident on this device (0: no cooperative launch).
int coop_max_groups(int eq, int order, bool ch);
hipError_t launch_coop(int eq, int order, bool ch, int groups, const KParams &p, int nsteps,
                       unsigned long long *amax, unsigned *bar, hipStream_t s, bool *refused);

// resident workgroups per CU of each kernel (for persistent grid sizes)
int occupancy_x(int eq, int order, int mode, bool rec, bool ch);
int occupancy_y(int order, int mode, bool rec, bool ch, int yw);
int occupancy_maxima(int eq);

}  // namespace enoao
