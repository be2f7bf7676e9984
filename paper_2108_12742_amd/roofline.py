"""Algorithmic work per unit of the ENO-AO kernels, for roofline reporting.

Units: a "face" is one face of one sweep direction with all its characteristic
fields and both split sides; a "cell" is one node updated by one kernel launch.
Counts are the essential FP64 operations of the method as laid out in the
kernels (add, sub, mul, div, sqrt, min/max, compare = 1 flop; a fused
multiply-add = 2; fabs and negation free).  Two layouts of the same arithmetic:
  * window form: every stencil node projected and split, every indicator and
    one candidate flux per side (branch-free selection) -- the full selection,
    which the kernels run only for the fields of a wave that need it;
  * top form (every sweep and the LDS-resident solver): the top candidate's two
    indicators and the sum of its one-sided values from conserved-variable
    differences and a symmetric stencil, seven projected vectors per face.  The
    full selection that waves with a field off the top candidate add is
    data-dependent and not counted (the count is a lower bound there).
Bytes: algorithmic HBM traffic of a Runge-Kutta stage, per cell: the stage
reads its input state once (and u^n in stages 2 and 3) and writes its output
once -- 2 x, 3 x, 3 x the state's 8 * ncomp bytes, i.e. 64/96/96 = 256 B per 2D
cell-update, 48/72/72 = 192 B for 1D Euler.  Intermediate arrays of an
implementation (the x-part of L that the 2D x-sweep writes and the y-sweep
reads back, second reads of the stage input) are not algorithmic: a stage's
bytes belong to the kernel that completes the stage (the y-sweep in 2D), and
the 2D x-sweep carries none of its own.

Peaks (MI355X, published): HBM3E 8.0 TB/s; FP64 vector 78.6 TFLOP/s
(256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz).
"""

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6

# one side of one field: 20 (difference table: 6+5+4+3+2 subtractions for order 5;
# 8+7+...+2 = 35 for order 7) + indicators (S_j^j: 2 adds, 1 min, 1 mul; one min per
# other candidate) + keys (1 compare per candidate) + arg-min (K-1 compares) + the
# selected candidate flux (at most 5 / 7 multiply-adds and 1 scaling)
RECON_SIDE = {5: 20 + (4 + 5) + 6 + 5 + 9, 7: 35 + (4 + 8) + 9 + 8 + 13}


def face_flops(equation: str, order: int) -> int:
    r = RECON_SIDE[order]
    h = 3 if order == 5 else 4
    nodes = 2 * h + 2  # stencil nodes of one face
    if equation == "advection":
        # split: per window value 1 mul + 1 fma (2 windows of 2h+1), recon 2 sides,
        # combine 2, flux difference 2
        return 2 * (2 * h + 1) * 3 + 2 * r + 2 + 2
    nc = 3 if equation == "euler1d" else 4
    node = 15 if nc == 4 else 12            # conserved -> flux, sqrt(rho), u, (v,) H: once per node
    roe = 23 if nc == 4 else 19             # Roe average, c, 1/c, b1, b2
    proj_vec = 15 if nc == 4 else 11        # structured left-eigenvector product of one vector
    projection = 2 * nodes * proj_vec       # U and F at every stencil node
    split = 2 * (2 * h + 1) * nc * 2        # w+ and w- windows, one fma each
    recon = 2 * nc * r
    back = 2 * nc + (16 if nc == 4 else 12)  # (w+ + w-) scaling and R w
    diff = 2 * nc                            # flux difference per cell
    return node + roe + projection + split + recon + back + diff


# (2H-1)-th difference of one quantity at one node (order 5: 3 subtractions and
# 2 multiply-adds; order 7: 4 and 3) and the symmetric stencil of one quantity
# (pair sums, consecutive differences and multiply-adds: order 5 3+2+2, order 7 4+3+3)
TOP_DIFF = {5: 3 + 2 * 2, 7: 4 + 3 * 2}
TOP_SYM = {5: 3 + 2 + 2 * 2, 7: 4 + 3 + 3 * 2}


def face_flops_top(equation: str, order: int) -> int:
    """Top form of one face (common path): node quantities and the top
    differences of one node (the essential work; a kernel that forms them per
    face from the window does three nodes' worth), the symmetric stencil of F,
    the Roe state, seven projections (D_0, D_1, D_2 of U and F, S F), per field
    both sides' indicators (two fma, a min and a compare each) and the value sum
    (a multiply and an fma, then the window scaling), the back-projection and
    the flux difference."""
    d, sym = TOP_DIFF[order], TOP_SYM[order]
    if equation == "advection":
        # differences and stencil of u; per side two a*D products (mul + fma), min,
        # compare; value sum (mul, mul, fma) and the 1/2; flux difference
        return d + sym + 2 * (2 * 3 + 2) + 4 + 1 + 2
    nc = 3 if equation == "euler1d" else 4
    node = 15 if nc == 4 else 12
    roe = 23 if nc == 4 else 19
    proj_vec = 15 if nc == 4 else 11
    fields = nc * (2 * (2 * 2 + 1 + 1) + (1 + 2 + 1))
    back = 16 if nc == 4 else 12
    return node + 2 * nc * d + nc * sym + roe + 7 * proj_vec + fields + back + 2 * nc


def combine_flops(nc: int, stage: int) -> int:
    """Shu-Osher stage combine per cell: in + dt L (one fma per component), and for
    stages 2 and 3 the weighted sum with u^n (a multiply and an fma more)."""
    return 2 * nc if stage == 1 else 5 * nc


MAXIMA_FLOPS = {"advection": 1, "euler1d": 16, "euler2d": 28}  # per-field wave-speed maxima of a cell


def stage_cell_flops(equation: str, stage: int) -> int:
    """Per-cell work of a stage besides the faces, summed over the stage's kernels:
    1D: combine + maxima in the x-sweep; 2D: the y-sweep adds L_x and L_y (one add
    per component), combines and takes the maxima."""
    nc = {"advection": 1, "euler1d": 3, "euler2d": 4}[equation]
    extra = nc if equation == "euler2d" else 0
    return combine_flops(nc, stage) + MAXIMA_FLOPS[equation] + extra


def stage_bytes(equation: str, stage: int) -> int:
    """Algorithmic HBM bytes per cell of one stage (stage 0: one evaluation of L,
    read u, write L)."""
    w = 8 * {"advection": 1, "euler1d": 3, "euler2d": 4}[equation]
    return 2 * w if stage in (0, 1) else 3 * w


def algorithmic_bytes(equation: str, kernel: str, stage: int) -> int:
    """The stage's algorithmic bytes attributed to one kernel of it: all of them to
    the kernel that completes the stage (1D x-sweep, 2D y-sweep), none to the 2D
    x-sweep."""
    if equation == "euler2d" and kernel == "x":
        return 0
    return stage_bytes(equation, stage)


def sweep_bytes(equation: str, kernel: str, stage: int) -> int:
    """Compulsory HBM bytes per cell of one launch (stage 0: evaluation of L only).

    1D 'x': read the stage input (+ u^n for stages 2, 3), write the stage output.
    2D 'x': read the stage input, write L_x.
    2D 'y': read the stage input and L_x (+ u^n for stages 2, 3), write the stage
    output (rhs: L)."""
    nc = {"advection": 1, "euler1d": 3, "euler2d": 4}[equation]
    w = 8 * nc
    if equation == "euler2d":
        return 2 * w if kernel == "x" else 3 * w + (w if stage > 1 else 0)
    return 2 * w + (w if stage > 1 else 0)


def sweep_flops(equation: str, order: int, kernel: str, stage: int) -> int:
    """Algorithmic flops per cell of one launch (top form)."""
    nc = {"advection": 1, "euler1d": 3, "euler2d": 4}[equation]
    f = face_flops_top(equation, order)
    if stage == 0:
        return f
    if equation == "euler2d":
        return f if kernel == "x" else f + nc + combine_flops(nc, stage) + MAXIMA_FLOPS[equation]
    return f + combine_flops(nc, stage) + MAXIMA_FLOPS[equation]


def cell_update_flops(equation: str, order: int) -> int:
    dims = 2 if equation == "euler2d" else 1
    return 3 * dims * face_flops_top(equation, order) + sum(stage_cell_flops(equation, s) for s in (1, 2, 3))


def cell_update_bytes(equation: str) -> int:
    """Algorithmic HBM bytes of one cell-update (three stages): 256 B in 2D."""
    return sum(stage_bytes(equation, s) for s in (1, 2, 3))


def split_sweep_bytes(equation: str) -> int:
    """Compulsory bytes per cell-update of the split 2D layout (x-part of L written and
    read back, stage input read by both sweeps): the implementation's own minimum."""
    if equation == "euler2d":
        return sum(sweep_bytes(equation, "x", s) + sweep_bytes(equation, "y", s) for s in (1, 2, 3))
    return sum(sweep_bytes(equation, "x", s) for s in (1, 2, 3))


def hbm_entry(nbytes: float, seconds: float, traffic=None):
    """Roofline against HBM bandwidth (algorithmic bytes / time)."""
    gbs = nbytes / seconds / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": traffic}


def alu_entry(flops: float, seconds: float):
    """Roofline against the FP64 vector peak (flops / time)."""
    tf = flops / seconds / 1e12
    return {"bound": "alu", "achieved": round(tf, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tf / PEAK_FP64_TFLOPS, 4)}


def resident_bytes(equation: str, steps: int) -> float:
    """LDS-resident solver: the state is read once and written once per call, so the
    compulsory HBM bytes per cell-update are 2 * state / steps."""
    nc = {"advection": 1, "euler1d": 3, "euler2d": 4}[equation]
    return 2.0 * 8 * nc / max(steps, 1)


def roofline_entry(flops: float, nbytes: float, seconds: float, traffic=None):
    """The roof this launch is closer to, with achieved / peak."""
    gflops = flops / seconds / 1e12
    gbs = nbytes / seconds / 1e9
    f_alu = gflops / PEAK_FP64_TFLOPS
    f_hbm = gbs / PEAK_HBM_GBS
    if f_alu >= f_hbm:
        return {"bound": "alu", "achieved": round(gflops, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(f_alu, 4), "traffic": traffic}
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(f_hbm, 4), "traffic": traffic}
