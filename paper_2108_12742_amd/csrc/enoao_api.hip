// enoao_api.hip -- C ABI (include/enoao.h): plans, batches and the device-side
// time loop.  Host code only orders kernel launches; every arithmetic step of
// the method runs in the kernels of enoao_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/enoao.h"
#include "enoao_common.hpp"
#include "enoao_kernels.hpp"

using namespace enoao;

namespace {

int g_wg_per_cu = 0;  // 0: occupancy of each kernel
int g_resident = 1;   // small 1D members: LDS-resident solver for controlled steps
int g_coop = 1;       // one mid-sized 1D member: cooperative solver for controlled steps
int g_shortcut = 1;   // wave-uniform top-candidate shortcut of the face kernels

// Graph capture: one stream per device, shared by every plan, batch and pool of
// the process and created on first use, instead of a HIP stream per object (a
// few hundred plans made a few hundred streams, which the runtime maps onto its
// few hardware queues next to the caller's).  A capture only records launches;
// the mutex keeps two of them from using the stream at once.
constexpr int CAPTURE_MAX_DEVICES = 64;
std::mutex capture_mutex;
hipStream_t capture_streams[CAPTURE_MAX_DEVICES] = {};

// kernel kinds of the per-kernel timing (enoao_profile_read order)
enum {
    PROF_X1 = 0, PROF_X2, PROF_X3, PROF_Y1, PROF_Y2, PROF_Y3, PROF_CONTROL, PROF_MAXIMA, PROF_RESIDENT, PROF_COOP,
    PROF_KINDS
};

int ncomp_of(int eq) { return eq == ADVECTION ? 1 : eq == EULER1D ? 3 : eq == EULER2D ? 4 : 0; }

enoao_status check_problem(const enoao_problem *p)
{
    if (!p || p->struct_size != sizeof(enoao_problem)) return ENOAO_EINVAL;
    if (!ncomp_of(p->equation)) return ENOAO_EINVAL;
    if (p->order != 5 && p->order != 7) return ENOAO_EINVAL;
    if (p->nx < 1 || p->ny < 1 || p->reserved1 != 0) return ENOAO_EINVAL;
    if (p->recon_vars != ENOAO_CHAR_ROE && p->recon_vars != ENOAO_COMPONENT) return ENOAO_EINVAL;
    if (p->equation != EULER2D && p->ny != 1) return ENOAO_EINVAL;
    if (!(p->x_hi > p->x_lo)) return ENOAO_EINVAL;
    if (p->equation == EULER2D && !(p->y_hi > p->y_lo)) return ENOAO_EINVAL;
    if (p->bc_x != BC_PERIODIC && p->bc_x != BC_TRANSMISSIVE) return ENOAO_EINVAL;
    if (p->equation == EULER2D && p->bc_y != BC_PERIODIC && p->bc_y != BC_TRANSMISSIVE) return ENOAO_EINVAL;
    if (p->equation != ADVECTION && !(p->gamma > 1.0)) return ENOAO_EINVAL;
    if (p->equation == ADVECTION && !(std::isfinite(p->adv_speed) && p->adv_speed != 0.0)) return ENOAO_EINVAL;
    if (!(p->delta >= 0.0) || !std::isfinite(p->delta)) return ENOAO_EINVAL;
    if (p->nx > ENOAO_MAX_EXTENT || p->ny > ENOAO_MAX_EXTENT) return ENOAO_EINVAL;
    if ((long long)p->nx * p->ny > (1ll << 31)) return ENOAO_EINVAL;
    return ENOAO_OK;
}

size_t selection_count(const enoao_problem *p)
{
    const size_t nc = ncomp_of(p->equation);
    size_t n = nc * 2 * (size_t)p->ny * (p->nx + 1);
    if (p->equation == EULER2D) n += nc * 2 * (size_t)(p->ny + 1) * p->nx;
    return n;
}

// A member's state-sized buffers are laid out one after another with a gap of
// BUF_STAGGER doubles (4352 bytes) between them: buffers that a kernel streams
// together (stage input, x-part, stage output) then do not start at offsets
// that are multiples of a large power of two, which made their lines contend
// for the same cache sets and memory channels.
constexpr size_t BUF_STAGGER = 544;

// i-th state-sized buffer of a member block
inline double *member_buffer(double *m, size_t cells, int i) { return m + (size_t)i * (cells + BUF_STAGGER); }

// Row pitch of the states a pool owns: rows padded to a multiple of 16 doubles
// (128 bytes), so every row starts on a cache line.  A y-sweep wave reads 8-column
// strips of 8 rows; with rows at arbitrary 8-byte offsets those straddle two lines
// about half the time (batches of 2D members with nx = ny = 511 or 625 ran 19-20%
// below nx = ny = 512 or 624).  Caller-owned states (plans, batches) keep pitch nx.
inline int padded_pitch(int nx) { return (nx + 15) / 16 * 16; }

// device bytes of one member: w1, w2 (+ Lx for 2D) and the selection record
size_t member_bytes(const enoao_problem *p)
{
    const size_t n = (size_t)ncomp_of(p->equation) * p->nx * p->ny;
    const int bufs = p->equation == EULER2D ? 3 : 2;
    size_t b = bufs * (n + BUF_STAGGER) * sizeof(double);
    // three records: one per Runge-Kutta stage of a step (enoao_rhs uses the first)
    if (p->flags & ENOAO_F_RECORD_SELECTION) b += (3 * selection_count(p) + 255) / 256 * 256;
    return b;
}

size_t member_fixed_bytes() { return sizeof(Inst) + sizeof(Ctrl) + AMAX_SLOTS * AMAX_VALS * 8 + 256; }

#define HIP_TRY(x)                                    \
    do {                                              \
        if ((x) != hipSuccess) return ENOAO_EDEVICE;  \
    } while (0)

}  // namespace

// A runtime = a batch of members sharing equation and order (a plan is one member).
struct Runtime {
    int eq = 0, order = 5, nc = 1, n = 0;
    int n_cap = 0;   // members the control and reset launches cover (>= n)
    double gamma = 1.4, delta = 1e-5;
    bool rec = false;
    bool ch = true;    // characteristic reconstruction variables (ENOAO_CHAR_ROE)
    int last_sel = 0;  // record slot of the last evaluation of L enqueued (recording plans)
    int device = 0, cus = 256;
    std::vector<enoao_problem> probs;
    std::vector<Inst> h_inst;
    BatchHdr h_hdr{};
    // device memory
    void *d_block = nullptr;   // one allocation for everything
    BatchHdr *d_hdr = nullptr;
    Inst *d_inst = nullptr;
    Ctrl *d_ctrl = nullptr;
    unsigned long long *d_amax = nullptr;
    int *d_res_order = nullptr;  // LDS-resident launches: members by decreasing size
    Ctrl *h_ctrl = nullptr;    // pinned mirror
    // captured step graphs (k steps of control + stages), one per step count k
    // used so far (a pool's server varies k from round to round)
    std::vector<std::pair<int, hipGraphExec_t>> graphs;
    // one event per stream the object's work was enqueued on: destroy waits for
    // them instead of the whole device
    std::vector<std::pair<hipStream_t, hipEvent_t>> marks;
    int grid_x[4] = {0, 0, 0, 0}, grid_y[4] = {0, 0, 0, 0}, grid_m = 0;
    // pools: the fewest workgroups that share a tile list (the kernel's occupancy)
    int gmin_x[4] = {0, 0, 0, 0}, gmin_y[4] = {0, 0, 0, 0}, gmin_m = 0;
    int wg_per_cu = 0;  // resident workgroups per CU of the persistent sweeps (0: occupancy)
    // per kernel kind (x-sweep stages 1..3, y-sweep stages 1..3): workgroups per
    // CU of that launch (0: wg_per_cu)
    int wg_kind[6] = {0, 0, 0, 0, 0, 0};
    int yw = 8;  // columns per wave strip of the y-sweep tiles (4 or 8); set from the order at creation
    // every member 1D and small enough for the LDS-resident solver; controlled
    // steps then run there, one launch per LDS size class (below)
    bool resident = false;
    struct ResClass {
        int first, count;  // members res_order[first .. first + count)
        int block;         // threads per workgroup
        size_t lds;        // dynamic LDS bytes per workgroup
    };
    std::vector<ResClass> res_classes;
    std::vector<hipStream_t> res_streams;  // classes after the first run on these, concurrently
    std::vector<hipEvent_t> res_events;    // fork + one join per extra class
    bool use_resident() const { return resident && g_resident != 0; }
    // one 1D member too long for the resident solver but at most one segment per
    // wave of one workgroup per CU: the cooperative solver (coop_groups workgroups)
    bool coop = false;
    int coop_groups = 0;
    unsigned *d_bar = nullptr;  // its grid barrier words
    bool use_coop() const { return coop && g_coop != 0; }
    // A member that also fits the resident solver takes the cooperative one when
    // its line has more segments than this: a resident stage takes its segments
    // four at a time (one per wave), a cooperative one all at once but pays its
    // barrier and the HBM round trips (measured alone, Euler: 13.4 us per step
    // resident at 250 nodes, 20 cooperative; 25 against 20 at 630 nodes, 41
    // against 20 at 1700; advection: 7.8 against 9.9 at 800, 13 against 11 at 1600)
    int coop_over_resident_segs() const { return eq == ADVECTION ? 20 : 9; }
    bool coop_first = false;
    int kflags = g_shortcut ? 0 : KF_FULL_SELECTION;  // taken when the plan or batch is created
    // optional per-kernel timing: hipEvents recorded around every launch, on the
    // stream the kernel is launched on (eager launches, no graph)
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, int>> ev_pairs;  // (kind, first event index)
    double prof_ms[PROF_KINDS] = {};
    long long prof_n[PROF_KINDS] = {};

    hipError_t prof_begin(int kind, hipStream_t s, int &slot)
    {
        slot = -1;
        if (!profiling) return hipSuccess;
        const size_t need = ev_pairs.size() * 2 + 2;
        while (ev_pool.size() < need) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return hipErrorOutOfMemory;
            ev_pool.push_back(e);
        }
        slot = (int)ev_pairs.size() * 2;
        ev_pairs.push_back({kind, slot});
        return hipEventRecord(ev_pool[slot], s);
    }
    hipError_t prof_end(int slot, hipStream_t s)
    {
        if (slot < 0) return hipSuccess;
        return hipEventRecord(ev_pool[slot + 1], s);
    }
    // drop the pair just begun (its launch did not happen)
    void prof_cancel(int slot)
    {
        if (slot >= 0 && !ev_pairs.empty() && ev_pairs.back().second == slot) ev_pairs.pop_back();
    }
    // after a synchronisation: fold the recorded pairs into the per-kind totals
    void prof_collect()
    {
        bool failed = false;
        for (auto &pr : ev_pairs) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev_pool[pr.second], ev_pool[pr.second + 1]) == hipSuccess) {
                prof_ms[pr.first] += ms;
                prof_n[pr.first] += 1;
            } else {
                failed = true;
            }
        }
        ev_pairs.clear();
        if (failed) (void)hipGetLastError();  // a pair without a reading is skipped, not left as an error
    }

    KParams params(int r_in, int r_out, int r_zero, int sel_slot = 0) const
    {
        KParams p{};
        p.sel_slot = sel_slot;
        p.hdr = d_hdr;
        p.inst = d_inst;
        p.gamma = gamma;
        p.gm1 = gamma - 1.0;
        p.delta = delta;
        p.r_in = r_in;
        p.r_out = r_out;
        p.r_zero = r_zero;
        p.flags = kflags;
        p.res_order = d_res_order;
        return p;
    }

    // Pool: the tile totals change, so the grids cover the whole machine
    // (wg_per_cu workgroups per CU, POOL_WG_PER_CU unless set) and each launch
    // shares its tile list among as many of them as give POOL_TILES_PER_WG
    // tiles each, at least the kernel's occupancy (a pool with few tiles runs
    // as a plan would).  On the served mix of 128^2..1024^2 requests, 16 per CU
    // measured 4.7-5.0e9 cell-updates/s against 3.9-4.1e9 at the occupancy
    // (2-3 per CU); with long chunks only, a lone request's step took twice as
    // long at 16 per CU.  24 per CU with 16-tile chunks measured 3% above 16 with
    // 32 (64-tile chunks: 7% below); a lone request's time is the same at all.
    bool dynamic = false;
    static constexpr int POOL_WG_PER_CU = 24, POOL_TILES_PER_WG = 16;
    int grid_for(long long tiles, int occ, int kind_wg = 0) const
    {
        const int per_cu = kind_wg > 0 ? kind_wg : wg_per_cu > 0 ? wg_per_cu : occ;
        const long long g = dynamic ? (long long)cus * per_cu : std::min<long long>(tiles, (long long)cus * per_cu);
        return (int)std::max<long long>(g, 1);
    }
    KParams chunked(KParams p, int gmin) const
    {
        p.tiles_per_wg = dynamic ? POOL_TILES_PER_WG : 0;
        p.grid_min = gmin;
        return p;
    }

    enoao_status init(const enoao_problem *ps, int count, hipStream_t stream)
    {
        if (count < 1) return ENOAO_EINVAL;
        for (int i = 0; i < count; ++i) {
            if (check_problem(&ps[i])) return ENOAO_EINVAL;
            if (ps[i].equation != ps[0].equation || ps[i].order != ps[0].order) return ENOAO_EINVAL;
            if (ps[i].gamma != ps[0].gamma || ps[i].delta != ps[0].delta) return ENOAO_EINVAL;
            if (ps[i].recon_vars != ps[0].recon_vars) return ENOAO_EINVAL;
        }
        eq = ps[0].equation;
        order = ps[0].order;
        yw = yw_default(order);
        nc = ncomp_of(eq);
        n = count;
        n_cap = count;
        gamma = ps[0].gamma;
        delta = ps[0].delta;
        rec = (ps[0].flags & ENOAO_F_RECORD_SELECTION) != 0;
        ch = ps[0].recon_vars == ENOAO_CHAR_ROE;
        probs.assign(ps, ps + count);
        HIP_TRY(hipGetDevice(&device));
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));

        // layout of the single device allocation
        size_t off = 0;
        auto take = [&](size_t bytes) {
            const size_t o = off;
            off += (bytes + 255) / 256 * 256;
            return o;
        };
        const size_t o_hdr = take(sizeof(BatchHdr));
        const size_t o_inst = take(sizeof(Inst) * count);
        const size_t o_ctrl = take(sizeof(Ctrl) * count);
        const size_t o_amax = take(8ull * AMAX_SLOTS * AMAX_VALS * count);
        const size_t o_order = take(sizeof(int) * count);
        const size_t o_bar = take(2 * sizeof(unsigned));
        std::vector<size_t> o_mem(count);
        for (int i = 0; i < count; ++i) o_mem[i] = take(member_bytes(&ps[i]));
        if (hipMalloc(&d_block, off) != hipSuccess) {
            d_block = nullptr;
            return ENOAO_ENOMEM;
        }
        char *base = (char *)d_block;
        d_hdr = (BatchHdr *)(base + o_hdr);
        d_inst = (Inst *)(base + o_inst);
        d_ctrl = (Ctrl *)(base + o_ctrl);
        d_amax = (unsigned long long *)(base + o_amax);
        d_res_order = (int *)(base + o_order);
        d_bar = (unsigned *)(base + o_bar);
        if (hipHostMalloc((void **)&h_ctrl, sizeof(Ctrl) * count, hipHostMallocDefault) != hipSuccess) {
            h_ctrl = nullptr;
            return ENOAO_ENOMEM;
        }

        h_inst.resize(count);
        long long xt = 0, yt = 0;
        for (int i = 0; i < count; ++i) {
            double *m = (double *)(base + o_mem[i]);
            const size_t cells = (size_t)nc * ps[i].nx * ps[i].ny;
            fill_inst(h_inst[i], ps[i], nullptr, member_buffer(m, cells, 0), member_buffer(m, cells, 1),
                      eq == EULER2D ? member_buffer(m, cells, 2) : nullptr,
                      rec ? (uint8_t *)member_buffer(m, cells, eq == EULER2D ? 3 : 2) : nullptr,
                      d_amax + (size_t)i * AMAX_SLOTS * AMAX_VALS, d_ctrl + i, xt, yt);
        }
        h_hdr.n_inst = count;
        h_hdr.xtiles_total = xt;
        h_hdr.ytiles_total = yt;
        HIP_TRY(hipMemcpyAsync(d_hdr, &h_hdr, sizeof(BatchHdr), hipMemcpyHostToDevice, stream));
        HIP_TRY(hipMemcpyAsync(d_inst, h_inst.data(), sizeof(Inst) * count, hipMemcpyHostToDevice, stream));
        std::vector<Ctrl> c0(count);
        for (auto &c : c0) {
            std::memset(&c, 0, sizeof(Ctrl));
            c.t_final = INFINITY;
            c.max_steps = 0;
            c.done = 0;
        }
        HIP_TRY(hipMemcpyAsync(d_ctrl, c0.data(), sizeof(Ctrl) * count, hipMemcpyHostToDevice, stream));
        // LDS-resident launches take the members by decreasing size: the hardware
        // hands workgroups to free CUs in launch order, so the long members start
        // first and the short ones fill in behind them instead of a CU ending with
        // two long ones (512 members of 128..1700 nodes, one workgroup per CU:
        // 4.7-4.8e9 cell-updates/s against 3.9-4.0e9 in member order)
        std::vector<int> order_h(count);
        for (int i = 0; i < count; ++i) order_h[i] = i;
        std::stable_sort(order_h.begin(), order_h.end(),
                         [&](int a, int b) { return (long long)ps[a].nx * ps[a].ny > (long long)ps[b].nx * ps[b].ny; });
        HIP_TRY(hipMemcpyAsync(d_res_order, order_h.data(), sizeof(int) * count, hipMemcpyHostToDevice, stream));
        HIP_TRY(hipStreamSynchronize(stream));

        wg_per_cu = g_wg_per_cu;
        set_grids();
        if (eq != EULER2D && !rec) {
            if (enoao_status e = plan_resident(ps, order_h)) return e;
            if (count == 1) {
                const int segs = (ps[0].nx + XW_CELLS - 1) / XW_CELLS;
                const int groups = (segs + RES_BLOCK / 64 - 1) / (RES_BLOCK / 64);
                coop_groups = groups;
                coop = groups <= cus && groups <= coop_max_groups(eq, order, ch);
                coop_first = segs > coop_over_resident_segs();
            }
        }
        return ENOAO_OK;
    }

    // LDS size classes of the resident solver.  The dynamic LDS of a launch is the
    // same for all its workgroups, so one launch for all members would give every
    // member the largest one's and hold the CUs at the occupancy of the largest.
    // Members (largest first) are grouped by how many of their workgroups one CU
    // holds: as many as fit its LDS (4, 3, 2 or 1), at most as many as the kernel's
    // registers allow (two for Euler: more LDS classes would not raise occupancy,
    // only add launches).  Each class is one launch, and the classes run
    // concurrently on streams of their own (forked from and joined to the caller's
    // stream): every class needs a hardware queue of its own, since two classes
    // sharing one run one after the other (HIP spreads streams over few queues).
    // Workgroups of 4 waves: on the small-member batch 8-wave workgroups (one per
    // CU) for the mid-sized members measured 13% slower.
    enoao_status plan_resident(const enoao_problem *ps, const std::vector<int> &sorted)
    {
        const int nq = eq == ADVECTION ? 1 : 9, g = order == 5 ? 4 : 5;
        const size_t limit = resident_lds_limit();
        int per_cu = 0;
        if (hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) != hipSuccess ||
            per_cu <= 0)
            per_cu = (int)limit;
        int by_regs = resident_groups_per_cu(eq, order, ch);
        by_regs = by_regs < 1 ? 4 : by_regs;
        auto cls = [&](long long nx, int &block, size_t &lds) {
            block = RES_BLOCK;
            lds = resident_lds_bytes(nc, nq, g, nx, RES_BLOCK);
            for (int k = by_regs < 4 ? by_regs : 4; k >= 2; --k)
                if (lds + 1024 <= (size_t)per_cu / k) return k;  // 1 KiB for each workgroup's static LDS
            return lds <= limit ? 1 : 0;
        };
        res_classes.clear();
        int prev_k = -1;
        for (int i = 0; i < (int)sorted.size(); ++i) {
            int block;
            size_t lds;
            const int k = cls(ps[sorted[i]].nx, block, lds);
            if (k == 0) {  // a member too large for one workgroup's LDS: stream every member
                res_classes.clear();
                resident = false;
                return ENOAO_OK;
            }
            if (k != prev_k) {
                res_classes.push_back({i, 0, block, lds});  // the first member of a class is its largest
                prev_k = k;
            }
            res_classes.back().count++;
        }
        resident = !res_classes.empty();
        for (size_t c = 1; c < res_classes.size(); ++c) {
            hipStream_t st;
            HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            res_streams.push_back(st);
        }
        for (size_t c = 0; c < res_classes.size(); ++c) {
            hipEvent_t e;
            HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            res_events.push_back(e);
        }
        return ENOAO_OK;
    }

    // k controlled steps of every member on the resident solver
    enoao_status resident_steps(int k, hipStream_t s)
    {
        int slot;
        HIP_TRY(prof_begin(PROF_RESIDENT, s, slot));
        if (res_classes.size() > 1) HIP_TRY(hipEventRecord(res_events[0], s));
        for (size_t c = 0; c < res_classes.size(); ++c) {
            const ResClass &rc = res_classes[c];
            hipStream_t st = c == 0 ? s : res_streams[c - 1];
            if (c > 0) HIP_TRY(hipStreamWaitEvent(st, res_events[0], 0));
            KParams p = params(0, -1, -1);
            p.res_first = rc.first;
            HIP_TRY(launch_resident(eq, order, ch, rc.block, p, rc.count, k, rc.lds, st));
            if (c > 0) HIP_TRY(hipEventRecord(res_events[c], st));
        }
        for (size_t c = 1; c < res_classes.size(); ++c) HIP_TRY(hipStreamWaitEvent(s, res_events[c], 0));
        HIP_TRY(prof_end(slot, s));
        return ENOAO_OK;
    }

    // descriptor of one member; advances the running tile offsets
    void fill_inst(Inst &I, const enoao_problem &p, double *u, double *w1, double *w2, double *lx, uint8_t *sel,
                   unsigned long long *amax, Ctrl *ctrl, long long &xt, long long &yt, int pitch = 0) const
    {
        std::memset(&I, 0, sizeof(I));
        I.u = u;
        I.w1 = w1;
        I.w2 = w2;
        I.lx = lx;
        I.sel = sel;
        I.amax = amax;
        I.ctrl = ctrl;
        I.nx = p.nx;
        I.ny = p.ny;
        I.pitch = pitch > 0 ? pitch : p.nx;
        I.bcx = p.bc_x;
        I.bcy = eq == EULER2D ? p.bc_y : BC_PERIODIC;
        I.dx = (p.x_hi - p.x_lo) / p.nx;
        I.dy = eq == EULER2D ? (p.y_hi - p.y_lo) / p.ny : 1.0;
        I.adv = p.adv_speed;
        I.segs_per_row = (p.nx + XW_CELLS - 1) / XW_CELLS;
        I.ytiles_per_row = (p.ny + yt_cells(yw) - 1) / yt_cells(yw);
        I.ycol_groups = (p.nx + yt_cols(yw) - 1) / yt_cols(yw);
        I.xtile0 = xt;
        I.xtiles = ((long long)p.ny * I.segs_per_row + XW_SEGS - 1) / XW_SEGS;
        I.ytile0 = yt;
        I.ytiles = eq == EULER2D ? (long long)I.ytiles_per_row * I.ycol_groups : 0;
        xt += I.xtiles;
        yt += I.ytiles;
    }

    void set_grids()
    {
        const long long xt = h_hdr.xtiles_total, yt = h_hdr.ytiles_total;
        for (int m = 0; m < 4; ++m) {
            const int ox = occupancy_x(eq, order, m, false, ch);
            grid_x[m] = grid_for(xt, ox, m >= 1 ? wg_kind[m - 1] : 0);
            gmin_x[m] = std::min(grid_x[m], cus * ox);
            if (eq == EULER2D) {
                const int oy = occupancy_y(order, m, false, ch, yw);
                grid_y[m] = grid_for(yt, oy, m >= 1 ? wg_kind[2 + m] : 0);
                gmin_y[m] = std::min(grid_y[m], cus * oy);
            }
        }
        grid_m = grid_for(xt, occupancy_maxima(eq));
        gmin_m = std::min(grid_m, cus * occupancy_maxima(eq));
    }

    void drop_graphs()
    {
        for (auto &g : graphs) (void)hipGraphExecDestroy(g.second);
        graphs.clear();
    }

    // new launch shape: grids recomputed, the captured graphs dropped; a uniform
    // shape clears the per-kernel ones
    void set_launch(int wg)
    {
        wg_per_cu = wg;
        for (int &k : wg_kind) k = 0;
        set_grids();
        drop_graphs();
    }
    void set_launch_kinds(const int32_t *wg, int n)
    {
        for (int k = 0; k < 6; ++k) wg_kind[k] = k < n ? wg[k] : 0;
        set_grids();
        drop_graphs();
    }

    // the object's work enqueued on s so far ends before this stream's mark
    hipError_t mark(hipStream_t s)
    {
        for (auto &m : marks)
            if (m.first == s) return hipEventRecord(m.second, s);
        hipEvent_t e;
        hipError_t err = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (err != hipSuccess) return err;
        marks.push_back({s, e});
        return hipEventRecord(e, s);
    }

    // waits for the object's work on every stream it used
    void wait_marks()
    {
        for (auto &m : marks) (void)hipEventSynchronize(m.second);
    }

    // new y tile width: the members' y tile lists rebuilt and uploaded, grids
    // recomputed, the captured graph dropped
    enoao_status set_ytiles(int w, hipStream_t s)
    {
        if (w == yw) return ENOAO_OK;
        yw = w;
        long long yt = 0;
        for (int i = 0; i < n; ++i) {
            Inst &I = h_inst[i];
            I.ytiles_per_row = (I.ny + yt_cells(yw) - 1) / yt_cells(yw);
            I.ycol_groups = (I.nx + yt_cols(yw) - 1) / yt_cols(yw);
            I.ytile0 = yt;
            I.ytiles = eq == EULER2D ? (long long)I.ytiles_per_row * I.ycol_groups : 0;
            yt += I.ytiles;
        }
        h_hdr.ytiles_total = yt;
        HIP_TRY(hipMemcpyAsync(d_inst, h_inst.data(), sizeof(Inst) * n, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d_hdr, &h_hdr, sizeof(BatchHdr), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));  // the host copies are reused
        set_launch(wg_per_cu);
        return ENOAO_OK;
    }

    void release()
    {
        wait_marks();
        for (auto &m : marks) (void)hipEventDestroy(m.second);
        marks.clear();
        for (auto e : ev_pool) (void)hipEventDestroy(e);
        ev_pool.clear();
        for (auto st : res_streams) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
        res_streams.clear();
        for (auto e : res_events) (void)hipEventDestroy(e);
        res_events.clear();
        drop_graphs();
        if (h_ctrl) (void)hipHostFree(h_ctrl);
        if (d_block) (void)hipFree(d_block);
        h_ctrl = nullptr;
        d_block = nullptr;
    }

    // ---- building blocks, all enqueued on stream s ----
    enoao_status set_pointers(int k, const double *u, double *lx, hipStream_t s)
    {
        // patch the member's u (and L output) in the device descriptor
        HIP_TRY(launch_patch_inst(d_inst, k, u, lx, lx != nullptr, s));
        return ENOAO_OK;
    }

    enoao_status reset_and_maxima(hipStream_t s)
    {
        int slot;
        HIP_TRY(launch_reset_maxima(params(0, 0, -1), n_cap, s));
        HIP_TRY(prof_begin(PROF_MAXIMA, s, slot));
        HIP_TRY(launch_state_maxima(eq, chunked(params(-1, 0, -1), gmin_m), grid_m, s));
        HIP_TRY(prof_end(slot, s));
        return ENOAO_OK;
    }

    // one Runge-Kutta stage (1..3); slots: stage s reads s-1, writes s%3, clears (s+1)%3
    enoao_status stage(int s, bool record, hipStream_t st)
    {
        const int r_in = (s - 1) % 3, r_out = s % 3, r_zero = (s + 1) % 3;
        const int mode = s;  // M_S1..M_S3
        int slot;
        HIP_TRY(prof_begin(PROF_X1 + s - 1, st, slot));
        const KParams px = chunked(params(r_in, eq == EULER2D ? -1 : r_out, r_zero, s - 1), gmin_x[mode]);
        HIP_TRY(launch_sweep_x(eq, order, mode, record, ch, px, grid_x[mode], st));
        HIP_TRY(prof_end(slot, st));
        if (eq == EULER2D) {
            HIP_TRY(prof_begin(PROF_Y1 + s - 1, st, slot));
            const KParams py = chunked(params(r_in, r_out, -1, s - 1), gmin_y[mode]);
            HIP_TRY(launch_sweep_y(order, mode, record, ch, yw, py, grid_y[mode], st));
            HIP_TRY(prof_end(slot, st));
        }
        if (record) last_sel = s - 1;
        return ENOAO_OK;
    }

    enoao_status rhs(hipStream_t s)
    {
        HIP_TRY(launch_sweep_x(eq, order, M_RHS, rec, ch, chunked(params(0, -1, -1), gmin_x[M_RHS]), grid_x[M_RHS], s));
        if (eq == EULER2D)
            HIP_TRY(launch_sweep_y(order, M_RHS, rec, ch, yw, chunked(params(0, -1, -1), gmin_y[M_RHS]), grid_y[M_RHS],
                                   s));
        last_sel = 0;
        return ENOAO_OK;
    }

    enoao_status steps(int k, bool control, hipStream_t s)
    {
        if (control && use_coop() && (coop_first || !use_resident())) {
            int slot;
            bool refused = false;
            HIP_TRY(prof_begin(PROF_COOP, s, slot));
            const hipError_t e =
                launch_coop(eq, order, ch, coop_groups, params(0, -1, -1), k, h_inst[0].amax, d_bar, s, &refused);
            if (e == hipSuccess) {
                HIP_TRY(prof_end(slot, s));
                return ENOAO_OK;
            }
            if (!refused) return ENOAO_EDEVICE;
            // The runtime turned the cooperative launch down (it does while another
            // process that has made cooperative launches holds the device): clear the
            // error and leave the object to the other solvers from now on.  The zeroing
            // already enqueued cleared the maxima ring, so the maxima of the state at
            // this step boundary are taken again.
            (void)hipGetLastError();
            prof_cancel(slot);
            coop = false;
            if (enoao_status r = reset_and_maxima(s)) return r;
        }
        if (control && use_resident()) return resident_steps(k, s);
        for (int i = 0; i < k; ++i) {
            if (control) {
                int slot;
                HIP_TRY(prof_begin(PROF_CONTROL, s, slot));
                HIP_TRY(launch_step_control(eq, params(0, -1, -1), n_cap, s));
                HIP_TRY(prof_end(slot, s));
            }
            for (int st = 1; st <= 3; ++st)
                if (enoao_status e = stage(st, rec, s)) return e;
        }
        return ENOAO_OK;
    }

    // graph of k controlled steps, captured once per k and replayed
    hipGraphExec_t graph_for(int k) const
    {
        for (auto &g : graphs)
            if (g.first == k) return g.second;
        return nullptr;
    }

    enoao_status ensure_graph(int k)
    {
        if (graph_for(k)) return ENOAO_OK;
        // a bounded cache: the oldest graph goes when a ninth step count comes
        if (graphs.size() >= 8) {
            (void)hipGraphExecDestroy(graphs.front().second);
            graphs.erase(graphs.begin());
        }
        if (device < 0 || device >= CAPTURE_MAX_DEVICES) return ENOAO_EDEVICE;
        std::lock_guard<std::mutex> lock(capture_mutex);
        hipStream_t &cap = capture_streams[device];
        if (!cap) {  // on the object's device
            int cur = 0;
            HIP_TRY(hipGetDevice(&cur));
            if (cur != device) HIP_TRY(hipSetDevice(device));
            const hipError_t ce = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
            if (cur != device) HIP_TRY(hipSetDevice(cur));
            if (ce != hipSuccess) {
                cap = nullptr;
                return ENOAO_EDEVICE;
            }
        }
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        enoao_status e = steps(k, true, cap);
        const hipError_t ce = hipStreamEndCapture(cap, &g);
        if (e) {
            if (g) (void)hipGraphDestroy(g);
            return e;
        }
        if (ce != hipSuccess) return ENOAO_EDEVICE;
        hipGraphExec_t exec = nullptr;
        const hipError_t ie = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return ENOAO_EDEVICE;
        graphs.push_back({k, exec});
        return ENOAO_OK;
    }

    enoao_status read_ctrl(hipStream_t s)
    {
        HIP_TRY(hipMemcpyAsync(h_ctrl, d_ctrl, sizeof(Ctrl) * n_cap, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (profiling) prof_collect();
        return ENOAO_OK;
    }

    // k controlled steps: one graph replay, or eager launches when profiling
    enoao_status run_steps(int k, hipStream_t s)
    {
        if (profiling || use_resident() || use_coop()) return steps(k, true, s);  // (one launch already)
        if (enoao_status e = ensure_graph(k)) return e;
        HIP_TRY(hipGraphLaunch(graph_for(k), s));
        return ENOAO_OK;
    }
};

struct enoao_plan {
    Runtime rt;
    double *ws_lx = nullptr;  // 2D: Lx workspace (inside the runtime allocation)
};

// ---------------------------------------------------------------------------
// Allocation-free step (enoao_step_noalloc).  Its workspace -- the batch
// header, the member descriptor, the control block, the maxima ring and the
// stage buffers -- lives in one file-scope device array per GPU.  Host code
// never uses the array's name as an address: the device address is taken once
// per device with hipGetSymbolAddress and kept in noalloc_ptr.
namespace {

__device__ __align__(256) unsigned char scratch[ENOAO_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mutex;
void *noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// device address of this device's scratch array (nullptr on failure)
void *noalloc_scratch(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(noalloc_mutex);
    if (!noalloc_ptr[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        noalloc_ptr[device] = ptr;
    }
    return noalloc_ptr[device];
}

// scratch layout: header, descriptor, control, maxima ring, then the stage buffers
constexpr size_t NA_HDR = 0, NA_INST = 256, NA_CTRL = 512, NA_AMAX = 768, NA_MEM = 1024;
static_assert(sizeof(BatchHdr) <= 256 && sizeof(Inst) <= 256 && sizeof(Ctrl) <= 256 &&
                  AMAX_SLOTS * AMAX_VALS * 8 <= 256, "scratch header slots");

size_t noalloc_bytes(const enoao_problem *p)
{
    const size_t cells = (size_t)ncomp_of(p->equation) * p->nx * p->ny;
    return NA_MEM + (p->equation == EULER2D ? 3 : 2) * (cells + BUF_STAGGER) * sizeof(double);
}

// writes the descriptor, header and control block of the one member (kernel
// arguments by value: no host-to-device copy of pageable memory)
__global__ void noalloc_init(BatchHdr h, Inst I, Ctrl c, BatchHdr *dh, Inst *di, Ctrl *dc)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *dh = h;
        *di = I;
        *dc = c;
    }
}

}  // namespace

struct enoao_batch {
    Runtime rt;
    std::vector<const double *> bound;  // member states currently in the descriptors
    bool started = false;
};

// init-control kernel arguments go through a tiny device copy of a host Ctrl array
static enoao_status upload_ctrl(Runtime &rt, const std::vector<Ctrl> &c, hipStream_t s)
{
    std::memcpy(rt.h_ctrl, c.data(), sizeof(Ctrl) * rt.n);
    HIP_TRY(hipMemcpyAsync(rt.d_ctrl, rt.h_ctrl, sizeof(Ctrl) * rt.n, hipMemcpyHostToDevice, s));
    // the pinned mirror is reused by later calls: wait until the copy has read it
    HIP_TRY(hipStreamSynchronize(s));
    return ENOAO_OK;
}


// ---------------------------------------------------------------------------
// Pool: members join and leave between steps.  States and workspaces live in
// one device arena; the member list (descriptors, tile offsets) is rebuilt on
// the host and uploaded when it changes, while the captured step graph stays
// valid because the kernels read the list and its size from device memory.
struct enoao_pool {
    Runtime rt;
    int max_members = 0;
    size_t arena_bytes = 0;
    char *arena = nullptr;
    struct Slot {
        bool used = false;
        enoao_problem prob{};
        size_t off = 0, bytes = 0;
    };
    std::vector<Slot> slots;
    std::vector<std::pair<size_t, size_t>> free_list;  // (offset, size), sorted by offset
    // pinned copies of the header and instance list that rebuild uploads: two,
    // used in turn, each reused only after its last upload has completed, so a
    // rebuild does not wait for the stream
    char *h_pin[2] = {nullptr, nullptr};
    hipEvent_t ev_pin[2] = {nullptr, nullptr};
    int pin_cur = 0;
    bool dirty = false;
    int graph_steps = 0;

    static size_t align(size_t b) { return (b + 255) / 256 * 256; }

    bool arena_alloc(size_t bytes, size_t &off)
    {
        for (size_t i = 0; i < free_list.size(); ++i) {
            if (free_list[i].second >= bytes) {
                off = free_list[i].first;
                free_list[i].first += bytes;
                free_list[i].second -= bytes;
                if (free_list[i].second == 0) free_list.erase(free_list.begin() + i);
                return true;
            }
        }
        return false;
    }

    void arena_free(size_t off, size_t bytes)
    {
        auto it = std::lower_bound(free_list.begin(), free_list.end(), std::make_pair(off, (size_t)0));
        it = free_list.insert(it, {off, bytes});
        // merge with the neighbours
        size_t i = it - free_list.begin();
        if (i + 1 < free_list.size() && free_list[i].first + free_list[i].second == free_list[i + 1].first) {
            free_list[i].second += free_list[i + 1].second;
            free_list.erase(free_list.begin() + i + 1);
        }
        if (i > 0 && free_list[i - 1].first + free_list[i - 1].second == free_list[i].first) {
            free_list[i - 1].second += free_list[i].second;
            free_list.erase(free_list.begin() + i);
        }
    }

    enoao_status rebuild(hipStream_t s)
    {
        Runtime &r = rt;
        r.h_inst.clear();
        long long xt = 0, yt = 0;
        for (int k = 0; k < max_members; ++k) {
            if (!slots[k].used) continue;
            const enoao_problem &p = slots[k].prob;
            double *m = (double *)(arena + slots[k].off);
            const int pitch = padded_pitch(p.nx);
            const size_t cells = (size_t)r.nc * pitch * p.ny;
            Inst I;
            r.fill_inst(I, p, member_buffer(m, cells, 0), member_buffer(m, cells, 1), member_buffer(m, cells, 2),
                        r.eq == EULER2D ? member_buffer(m, cells, 3) : nullptr, nullptr,
                        r.d_amax + (size_t)k * AMAX_SLOTS * AMAX_VALS, r.d_ctrl + k, xt, yt, pitch);
            r.h_inst.push_back(I);
        }
        r.n = (int)r.h_inst.size();
        r.h_hdr.n_inst = r.n;
        r.h_hdr.xtiles_total = xt;
        r.h_hdr.ytiles_total = yt;
        pin_cur ^= 1;
        HIP_TRY(hipEventSynchronize(ev_pin[pin_cur]));  // this buffer's previous upload
        char *h = h_pin[pin_cur];
        std::memcpy(h, &r.h_hdr, sizeof(BatchHdr));
        if (r.n > 0) {
            std::memcpy(h + pin_inst_offset(), r.h_inst.data(), sizeof(Inst) * r.n);
            HIP_TRY(hipMemcpyAsync(r.d_inst, h + pin_inst_offset(), sizeof(Inst) * r.n, hipMemcpyHostToDevice, s));
        }
        HIP_TRY(hipMemcpyAsync(r.d_hdr, h, sizeof(BatchHdr), hipMemcpyHostToDevice, s));
        HIP_TRY(hipEventRecord(ev_pin[pin_cur], s));
        dirty = false;
        return ENOAO_OK;
    }

    static size_t pin_inst_offset() { return align(sizeof(BatchHdr)); }
    size_t pin_bytes() const { return pin_inst_offset() + sizeof(Inst) * (size_t)max_members; }

    void free_pins()
    {
        for (int i = 0; i < 2; ++i) {
            if (ev_pin[i]) (void)hipEventDestroy(ev_pin[i]);
            if (h_pin[i]) (void)hipHostFree(h_pin[i]);
            ev_pin[i] = nullptr;
            h_pin[i] = nullptr;
        }
    }

    // copy out (optional), stop the member, free its slot and arena space.  The
    // space is reused by later admissions, which enqueue their copies on the
    // stream after this call's work.
    enoao_status release_slot(int slot, double *u_out, bool u_out_on_host, double *info, hipStream_t s)
    {
        Runtime &r = rt;
        const enoao_problem &p = slots[slot].prob;
        if (u_out) {
            // the padded rows back to the dense layout (for a host result through the
            // member's w1 buffer: the member no longer steps)
            const int pitch = padded_pitch(p.nx);
            const long long rows = (long long)r.nc * p.ny;
            double *mem = (double *)(arena + slots[slot].off);
            const size_t cells = (size_t)r.nc * pitch * p.ny;
            double *dst = u_out_on_host ? member_buffer(mem, cells, 1) : u_out;
            HIP_TRY(launch_copy_pitched(member_buffer(mem, cells, 0), pitch, dst, p.nx, p.nx, rows, s));
            if (u_out_on_host)
                HIP_TRY(hipMemcpyAsync(u_out, dst, (size_t)rows * p.nx * sizeof(double), hipMemcpyDeviceToHost, s));
        }
        // the member stops stepping at once
        Ctrl c;
        std::memset(&c, 0, sizeof(Ctrl));
        c.done = 1;
        HIP_TRY(launch_set_ctrl(r.d_ctrl + slot, c, info, s));
        HIP_TRY(r.mark(s));
        arena_free(slots[slot].off, slots[slot].bytes);
        slots[slot].used = false;
        dirty = true;
        return ENOAO_OK;
    }
};

static size_t pool_member_bytes(const enoao_problem *p)
{
    const size_t cells = (size_t)ncomp_of(p->equation) * padded_pitch(p->nx) * p->ny;
    return enoao_pool::align((cells + BUF_STAGGER) * sizeof(double) * (p->equation == EULER2D ? 4 : 3));
}

extern "C" {

const char *enoao_status_string(enoao_status s)
{
    switch (s) {
    case ENOAO_OK: return "ok";
    case ENOAO_EINVAL: return "invalid argument";
    case ENOAO_ENOMEM: return "device out of memory";
    case ENOAO_EDEVICE: return "HIP runtime error";
    case ENOAO_EUNSUPPORTED: return "unsupported";
    case ENOAO_ENONPHYSICAL: return "non-physical state (rho <= 0, p <= 0 or NaN)";
    }
    return "unknown status";
}

size_t enoao_workspace_bytes(const enoao_problem *prob)
{
    if (check_problem(prob)) return 0;
    return sizeof(BatchHdr) + member_fixed_bytes() + member_bytes(prob);
}

enoao_status enoao_set_launch(int32_t workgroups_per_cu, int32_t reserved)
{
    if (workgroups_per_cu < 0 || workgroups_per_cu > 64 || reserved != 0) return ENOAO_EINVAL;
    g_wg_per_cu = workgroups_per_cu;
    return ENOAO_OK;
}

static bool valid_kinds(const int32_t *wg, int32_t n)
{
    if (n < 0 || n > 6 || (n > 0 && !wg)) return false;
    for (int k = 0; k < n; ++k)
        if (wg[k] < 0 || wg[k] > 64) return false;
    return true;
}

enoao_status enoao_plan_set_launch_kinds(enoao_plan *plan, const int32_t *workgroups_per_cu, int32_t n_kinds)
{
    if (!plan || !valid_kinds(workgroups_per_cu, n_kinds)) return ENOAO_EINVAL;
    plan->rt.set_launch_kinds(workgroups_per_cu, n_kinds);
    return ENOAO_OK;
}

enoao_status enoao_batch_set_launch_kinds(enoao_batch *batch, const int32_t *workgroups_per_cu, int32_t n_kinds)
{
    if (!batch || !valid_kinds(workgroups_per_cu, n_kinds)) return ENOAO_EINVAL;
    batch->rt.set_launch_kinds(workgroups_per_cu, n_kinds);
    return ENOAO_OK;
}

enoao_status enoao_plan_set_tiles(enoao_plan *plan, int32_t y_strip_columns, void *stream)
{
    if (!plan || (y_strip_columns != 0 && y_strip_columns != 4 && y_strip_columns != 8)) return ENOAO_EINVAL;
    return plan->rt.set_ytiles(y_strip_columns ? y_strip_columns : yw_default(plan->rt.order), (hipStream_t)stream);
}

enoao_status enoao_batch_set_tiles(enoao_batch *batch, int32_t y_strip_columns, void *stream)
{
    if (!batch || (y_strip_columns != 0 && y_strip_columns != 4 && y_strip_columns != 8)) return ENOAO_EINVAL;
    return batch->rt.set_ytiles(y_strip_columns ? y_strip_columns : yw_default(batch->rt.order), (hipStream_t)stream);
}

enoao_status enoao_set_resident(int32_t enable)
{
    if (enable != 0 && enable != 1) return ENOAO_EINVAL;
    g_resident = enable;
    return ENOAO_OK;
}

enoao_status enoao_set_coop(int32_t enable)
{
    if (enable != 0 && enable != 1) return ENOAO_EINVAL;
    g_coop = enable;
    return ENOAO_OK;
}

enoao_status enoao_set_shortcut(int32_t enable)
{
    if (enable != 0 && enable != 1) return ENOAO_EINVAL;
    g_shortcut = enable;
    return ENOAO_OK;
}

enoao_status enoao_plan_set_launch(enoao_plan *plan, int32_t workgroups_per_cu)
{
    if (!plan || workgroups_per_cu < 0 || workgroups_per_cu > 64) return ENOAO_EINVAL;
    plan->rt.set_launch(workgroups_per_cu);
    return ENOAO_OK;
}

enoao_status enoao_batch_set_launch(enoao_batch *batch, int32_t workgroups_per_cu)
{
    if (!batch || workgroups_per_cu < 0 || workgroups_per_cu > 64) return ENOAO_EINVAL;
    batch->rt.set_launch(workgroups_per_cu);
    return ENOAO_OK;
}

enoao_status enoao_plan_create(const enoao_problem *prob, void *stream, enoao_plan **out)
{
    if (!out) return ENOAO_EINVAL;
    *out = nullptr;
    if (check_problem(prob)) return ENOAO_EINVAL;
    enoao_plan *p = new (std::nothrow) enoao_plan();
    if (!p) return ENOAO_ENOMEM;
    enoao_status e = p->rt.init(prob, 1, (hipStream_t)stream);
    if (e) {
        p->rt.release();
        delete p;
        return e;
    }
    p->ws_lx = p->rt.h_inst[0].lx;
    *out = p;
    return ENOAO_OK;
}

enoao_status enoao_plan_destroy(enoao_plan *plan)
{
    if (!plan) return ENOAO_EINVAL;
    plan->rt.release();  // waits for the plan's work on the streams it was given
    delete plan;
    return ENOAO_OK;
}

enoao_status enoao_rhs(enoao_plan *plan, const double *u, double *L, void *stream)
{
    if (!plan || !u || !L || (const double *)L == u) return ENOAO_EINVAL;
    Runtime &rt = plan->rt;
    hipStream_t s = (hipStream_t)stream;
    if (enoao_status e = rt.set_pointers(0, u, L, s)) return e;
    HIP_TRY(launch_clear_done(rt.params(0, -1, -1), 1, s));
    if (enoao_status e = rt.reset_and_maxima(s)) return e;
    if (enoao_status e = rt.rhs(s)) return e;
    // restore the workspace Lx pointer for later steps
    if (rt.eq == EULER2D)
        if (enoao_status e = rt.set_pointers(0, u, plan->ws_lx, s)) return e;
    HIP_TRY(rt.mark(s));
    return ENOAO_OK;
}

enoao_status enoao_step(enoao_plan *plan, double *u, double dt, void *stream)
{
    if (!plan || !u || !(dt > 0.0) || !std::isfinite(dt)) return ENOAO_EINVAL;
    Runtime &rt = plan->rt;
    hipStream_t s = (hipStream_t)stream;
    if (enoao_status e = rt.set_pointers(0, u, plan->ws_lx, s)) return e;
    if (enoao_status e = rt.reset_and_maxima(s)) return e;
    HIP_TRY(launch_set_dt(rt.params(0, -1, -1), 1, dt, s));
    if (enoao_status e = rt.steps(1, false, s)) return e;
    HIP_TRY(rt.mark(s));
    return ENOAO_OK;
}

enoao_status enoao_solve(enoao_plan *plan, double *u, double t_final, double cfl, double dt_fixed,
                         int64_t max_steps, double *t_out, int64_t *steps_out, void *stream)
{
    if (!plan || !u || !(t_final >= 0.0) || !std::isfinite(t_final) || max_steps < 0) return ENOAO_EINVAL;
    if (!(dt_fixed > 0.0) && !(cfl > 0.0)) return ENOAO_EINVAL;
    Runtime &rt = plan->rt;
    hipStream_t s = (hipStream_t)stream;
    if (enoao_status e = rt.set_pointers(0, u, plan->ws_lx, s)) return e;
    std::vector<Ctrl> c(1);
    std::memset(c.data(), 0, sizeof(Ctrl));
    c[0].t = 0.0;
    c[0].t_final = t_final;
    c[0].cfl = cfl;
    c[0].dt_fixed = dt_fixed > 0.0 ? dt_fixed : 0.0;
    c[0].max_steps = max_steps;
    if (enoao_status e = upload_ctrl(rt, c, s)) return e;
    if (enoao_status e = rt.reset_and_maxima(s)) return e;

    // steps per graph replay: a guess of the total, bounded
    auto steps_per_launch = [&]() {
        int k = 16;
        if (dt_fixed > 0.0) {
            const double est = std::ceil(t_final / dt_fixed);
            k = (int)std::min(256.0, std::max(1.0, est));
        } else {
            // CFL steps: the end time may come early (the rest of a replay then only
            // checks its flag), unless the caller bounds the step count
            k = max_steps > 0 && max_steps <= 256 ? (int)max_steps : 64;
        }
        // the resident and cooperative solvers run many steps in one launch (they
        // stop by themselves at t_final): fewer, longer launches
        if (rt.use_resident() || rt.use_coop()) k = 1024;
        if (max_steps > 0) k = (int)std::min<int64_t>(k, max_steps);
        return std::max(k, 1);
    };
    enoao_status st = ENOAO_OK;
    int64_t taken = 0;  // steps known to be taken (host view)
    while (taken < max_steps) {
        // (again each time: a refused cooperative launch hands the plan to the others)
        const int k = steps_per_launch();
        // never enqueue more steps than the budget left: a partial batch runs eagerly
        const int64_t left = max_steps - taken;
        if (left >= k) {
            if (enoao_status e = rt.run_steps(k, s)) return e;
        } else {
            if (enoao_status e = rt.steps((int)left, true, s)) return e;
        }
        if (enoao_status e = rt.read_ctrl(s)) return e;
        const Ctrl &h = rt.h_ctrl[0];
        taken = h.steps;
        if (h.status) {  // bit 1: a grid barrier of the cooperative solver failed (it never should)
            st = (h.status & 2) ? ENOAO_EDEVICE : ENOAO_ENONPHYSICAL;
            break;
        }
        if (h.done || !(h.t < t_final)) break;
    }
    HIP_TRY(rt.mark(s));
    const Ctrl &h = rt.h_ctrl[0];
    if (t_out) *t_out = h.t;
    if (steps_out) *steps_out = h.steps;
    if (st == ENOAO_OK && h.status) st = ENOAO_ENONPHYSICAL;
    return st;
}

enoao_status enoao_step_noalloc(const enoao_problem *prob, double *u, double dt, void *stream)
{
    if (!prob || !u || !(dt > 0.0) || !std::isfinite(dt)) return ENOAO_EINVAL;
    if (check_problem(prob) || (prob->flags & ENOAO_F_RECORD_SELECTION)) return ENOAO_EINVAL;
    if (noalloc_bytes(prob) > (size_t)ENOAO_NOALLOC_SCRATCH_BYTES) return ENOAO_EINVAL;
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    char *base = (char *)noalloc_scratch(device);
    if (!base) return ENOAO_EDEVICE;
    hipStream_t s = (hipStream_t)stream;

    // a one-member runtime over the scratch array (nothing in it allocates)
    Runtime rt;
    rt.eq = prob->equation;
    rt.order = prob->order;
    rt.yw = yw_default(rt.order);
    rt.nc = ncomp_of(rt.eq);
    rt.n = rt.n_cap = 1;
    rt.gamma = prob->gamma;
    rt.delta = prob->delta;
    rt.rec = false;
    rt.ch = prob->recon_vars == ENOAO_CHAR_ROE;
    rt.device = device;
    HIP_TRY(hipDeviceGetAttribute(&rt.cus, hipDeviceAttributeMultiprocessorCount, device));
    rt.d_hdr = (BatchHdr *)(base + NA_HDR);
    rt.d_inst = (Inst *)(base + NA_INST);
    rt.d_ctrl = (Ctrl *)(base + NA_CTRL);
    rt.d_amax = (unsigned long long *)(base + NA_AMAX);
    rt.d_res_order = nullptr;
    double *m = (double *)(base + NA_MEM);
    const size_t cells = (size_t)rt.nc * prob->nx * prob->ny;
    Inst I;
    long long xt = 0, yt = 0;
    rt.fill_inst(I, *prob, u, member_buffer(m, cells, 0), member_buffer(m, cells, 1),
                 rt.eq == EULER2D ? member_buffer(m, cells, 2) : nullptr, nullptr, rt.d_amax, rt.d_ctrl, xt, yt);
    rt.h_hdr.n_inst = 1;
    rt.h_hdr.xtiles_total = xt;
    rt.h_hdr.ytiles_total = yt;
    rt.wg_per_cu = g_wg_per_cu;
    rt.set_grids();
    Ctrl c;
    std::memset(&c, 0, sizeof(Ctrl));
    c.t_final = INFINITY;
    // the same launches as enoao_step: descriptors, maxima of u, the step size, three stages
    hipLaunchKernelGGL(noalloc_init, dim3(1), dim3(64), 0, s, rt.h_hdr, I, c, rt.d_hdr, rt.d_inst, rt.d_ctrl);
    HIP_TRY(hipGetLastError());
    if (enoao_status e = rt.reset_and_maxima(s)) return e;
    HIP_TRY(launch_set_dt(rt.params(0, -1, -1), 1, dt, s));
    return rt.steps(1, false, s);
}

enoao_status enoao_plan_check(enoao_plan *plan, void *stream)
{
    if (!plan) return ENOAO_EINVAL;
    Runtime &rt = plan->rt;
    hipStream_t s = (hipStream_t)stream;
    if (enoao_status e = rt.read_ctrl(s)) return e;
    if (rt.h_ctrl[0].status) {
        static const int zero = 0;  // cleared by a copy, not a memset node, in case a caller records the stream
        HIP_TRY(hipMemcpyAsync(&rt.d_ctrl[0].status, &zero, sizeof(int), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
        return ENOAO_ENONPHYSICAL;
    }
    return ENOAO_OK;
}

static enoao_status profile_set(Runtime &rt, int32_t enable)
{
    if (enable) {
        rt.profiling = true;
        for (int i = 0; i < PROF_KINDS; ++i) { rt.prof_ms[i] = 0.0; rt.prof_n[i] = 0; }
        rt.ev_pairs.clear();
    } else {
        rt.profiling = false;
    }
    return ENOAO_OK;
}

static enoao_status profile_read(Runtime &rt, double *avg_ms, int64_t *count, int32_t n_kinds, void *stream)
{
    if (n_kinds < 0 || n_kinds > PROF_KINDS) return ENOAO_EINVAL;
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    rt.prof_collect();
    for (int i = 0; i < n_kinds; ++i) {
        if (avg_ms) avg_ms[i] = rt.prof_n[i] ? rt.prof_ms[i] / rt.prof_n[i] : 0.0;
        if (count) count[i] = rt.prof_n[i];
    }
    return ENOAO_OK;
}

enoao_status enoao_profile(enoao_plan *plan, int32_t enable)
{
    return plan ? profile_set(plan->rt, enable) : ENOAO_EINVAL;
}

enoao_status enoao_profile_read(enoao_plan *plan, double *avg_ms, int64_t *count, int32_t n_kinds, void *stream)
{
    return plan ? profile_read(plan->rt, avg_ms, count, n_kinds, stream) : ENOAO_EINVAL;
}

enoao_status enoao_batch_profile(enoao_batch *batch, int32_t enable)
{
    return batch ? profile_set(batch->rt, enable) : ENOAO_EINVAL;
}

enoao_status enoao_batch_profile_read(enoao_batch *batch, double *avg_ms, int64_t *count, int32_t n_kinds,
                                      void *stream)
{
    return batch ? profile_read(batch->rt, avg_ms, count, n_kinds, stream) : ENOAO_EINVAL;
}

size_t enoao_selection_size(const enoao_plan *plan)
{
    if (!plan || !plan->rt.rec) return 0;
    return selection_count(&plan->rt.probs[0]);
}

enoao_status enoao_get_selection(enoao_plan *plan, uint8_t *host_out, size_t n, void *stream)
{
    if (!plan || !host_out || !plan->rt.rec) return ENOAO_EINVAL;
    if (n != selection_count(&plan->rt.probs[0])) return ENOAO_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(host_out, plan->rt.h_inst[0].sel + (size_t)plan->rt.last_sel * n, n,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return ENOAO_OK;
}

enoao_status enoao_get_step_selection(enoao_plan *plan, uint8_t *host_out, size_t n, void *stream)
{
    if (!plan || !host_out || !plan->rt.rec) return ENOAO_EINVAL;
    if (n != 3 * selection_count(&plan->rt.probs[0])) return ENOAO_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(host_out, plan->rt.h_inst[0].sel, n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return ENOAO_OK;
}

// ---- batches ----
enoao_status enoao_batch_create(const enoao_problem *probs, int32_t n, void *stream, enoao_batch **out)
{
    if (!out || !probs || n < 1) return ENOAO_EINVAL;
    *out = nullptr;
    enoao_batch *b = new (std::nothrow) enoao_batch();
    if (!b) return ENOAO_ENOMEM;
    enoao_status e = b->rt.init(probs, n, (hipStream_t)stream);
    if (e) {
        b->rt.release();
        delete b;
        return e;
    }
    b->bound.assign(n, nullptr);
    *out = b;
    return ENOAO_OK;
}

enoao_status enoao_batch_destroy(enoao_batch *batch)
{
    if (!batch) return ENOAO_EINVAL;
    batch->rt.release();  // waits for the batch's work on the streams it was given
    delete batch;
    return ENOAO_OK;
}

enoao_status enoao_batch_reset(enoao_batch *batch, void *stream)
{
    if (!batch) return ENOAO_EINVAL;
    batch->started = false;
    (void)stream;
    return ENOAO_OK;
}

enoao_status enoao_batch_step(enoao_batch *batch, double *const *u, int32_t nsteps, double cfl,
                              const double *t_final, void *stream)
{
    if (!batch || !u || nsteps < 0 || !(cfl > 0.0)) return ENOAO_EINVAL;
    Runtime &rt = batch->rt;
    hipStream_t s = (hipStream_t)stream;
    bool rebind = false;
    for (int i = 0; i < rt.n; ++i) {
        if (!u[i]) return ENOAO_EINVAL;
        if (batch->bound[i] != u[i]) rebind = true;
    }
    if (rebind) {
        for (int i = 0; i < rt.n; ++i) rt.h_inst[i].u = u[i];
        HIP_TRY(hipMemcpyAsync(rt.d_inst, rt.h_inst.data(), sizeof(Inst) * rt.n, hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));  // h_inst is reused by later calls
        for (int i = 0; i < rt.n; ++i) batch->bound[i] = u[i];
    }
    // member control: continue times and step counts, extend the step budget
    if (!batch->started) {
        std::vector<Ctrl> c(rt.n);
        for (int i = 0; i < rt.n; ++i) {
            std::memset(&c[i], 0, sizeof(Ctrl));
            c[i].t_final = t_final ? t_final[i] : INFINITY;
            c[i].cfl = cfl;
            c[i].max_steps = nsteps;
        }
        if (enoao_status e = upload_ctrl(rt, c, s)) return e;
        if (enoao_status e = rt.reset_and_maxima(s)) return e;
        batch->started = true;
    } else {
        if (enoao_status e = rt.read_ctrl(s)) return e;
        std::vector<Ctrl> c(rt.h_ctrl, rt.h_ctrl + rt.n);
        for (int i = 0; i < rt.n; ++i) {
            c[i].cfl = cfl;
            if (t_final) c[i].t_final = t_final[i];
            c[i].max_steps = c[i].steps + nsteps;
            if (c[i].status == 0) c[i].done = 0;
        }
        if (enoao_status e = upload_ctrl(rt, c, s)) return e;
        // the caller may have changed the states since the last call
        if (enoao_status e = rt.reset_and_maxima(s)) return e;
    }
    if (nsteps > 0) {
        const int k = std::min(nsteps, 128);
        for (int done = 0; done < nsteps; done += k) {
            if (nsteps - done < k) {
                if (enoao_status e = rt.steps(nsteps - done, true, s)) return e;
                break;
            }
            if (enoao_status e = rt.run_steps(k, s)) return e;
        }
    }
    HIP_TRY(rt.mark(s));
    return ENOAO_OK;
}

enoao_status enoao_batch_query(enoao_batch *batch, double *t, int64_t *steps, int32_t *member_status,
                               void *stream)
{
    if (!batch) return ENOAO_EINVAL;
    Runtime &rt = batch->rt;
    if (enoao_status e = rt.read_ctrl((hipStream_t)stream)) return e;
    enoao_status st = ENOAO_OK;
    for (int i = 0; i < rt.n; ++i) {
        if (t) t[i] = rt.h_ctrl[i].t;
        if (steps) steps[i] = rt.h_ctrl[i].steps;
        if (member_status) member_status[i] = rt.h_ctrl[i].status;
        if (rt.h_ctrl[i].status) st = ENOAO_ENONPHYSICAL;
    }
    return st;
}

// ---- pools ----
size_t enoao_pool_member_bytes(const enoao_problem *prob)
{
    if (check_problem(prob) || (prob->flags & ENOAO_F_RECORD_SELECTION)) return 0;
    return pool_member_bytes(prob);
}

enoao_status enoao_pool_create(const enoao_problem *like, int32_t max_members, size_t arena_bytes, void *stream,
                               enoao_pool **out)
{
    if (!out || !like || max_members < 1 || arena_bytes < 256) return ENOAO_EINVAL;
    *out = nullptr;
    if (check_problem(like) || (like->flags & ENOAO_F_RECORD_SELECTION)) return ENOAO_EINVAL;
    enoao_pool *pl = new (std::nothrow) enoao_pool();
    if (!pl) return ENOAO_ENOMEM;
    Runtime &r = pl->rt;
    hipStream_t s = (hipStream_t)stream;
    auto fail = [&](enoao_status e) {
        pl->free_pins();
        r.release();
        delete pl;
        return e;
    };
    r.eq = like->equation;
    r.order = like->order;
    r.yw = yw_default(r.order);
    r.nc = ncomp_of(r.eq);
    r.gamma = like->gamma;
    r.delta = like->delta;
    r.rec = false;
    r.ch = like->recon_vars == ENOAO_CHAR_ROE;
    r.dynamic = true;
    r.n = 0;
    r.n_cap = max_members;
    r.probs.assign(1, *like);
    if (hipGetDevice(&r.device) != hipSuccess ||
        hipDeviceGetAttribute(&r.cus, hipDeviceAttributeMultiprocessorCount, r.device) != hipSuccess)
        return fail(ENOAO_EDEVICE);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += enoao_pool::align(bytes);
        return o;
    };
    const size_t o_hdr = take(sizeof(BatchHdr));
    const size_t o_inst = take(sizeof(Inst) * max_members);
    const size_t o_ctrl = take(sizeof(Ctrl) * max_members);
    const size_t o_amax = take(8ull * AMAX_SLOTS * AMAX_VALS * max_members);
    const size_t o_arena = take(arena_bytes);
    if (hipMalloc(&r.d_block, off) != hipSuccess) {
        r.d_block = nullptr;
        return fail(ENOAO_ENOMEM);
    }
    char *base = (char *)r.d_block;
    r.d_hdr = (BatchHdr *)(base + o_hdr);
    r.d_inst = (Inst *)(base + o_inst);
    r.d_ctrl = (Ctrl *)(base + o_ctrl);
    r.d_amax = (unsigned long long *)(base + o_amax);
    pl->arena = base + o_arena;
    pl->arena_bytes = arena_bytes / 256 * 256;
    pl->free_list.push_back({0, pl->arena_bytes});
    pl->max_members = max_members;
    pl->slots.assign(max_members, enoao_pool::Slot());
    if (hipHostMalloc((void **)&r.h_ctrl, sizeof(Ctrl) * max_members, hipHostMallocDefault) != hipSuccess) {
        r.h_ctrl = nullptr;
        return fail(ENOAO_ENOMEM);
    }
    for (int i = 0; i < 2; ++i) {
        if (hipHostMalloc((void **)&pl->h_pin[i], pl->pin_bytes(), hipHostMallocDefault) != hipSuccess) {
            pl->h_pin[i] = nullptr;
            return fail(ENOAO_ENOMEM);
        }
        if (hipEventCreateWithFlags(&pl->ev_pin[i], hipEventDisableTiming) != hipSuccess) {
            pl->ev_pin[i] = nullptr;
            return fail(ENOAO_EDEVICE);
        }
    }
    std::vector<Ctrl> c0(max_members);
    for (auto &c : c0) {
        std::memset(&c, 0, sizeof(Ctrl));
        c.done = 1;
    }
    if (hipMemcpyAsync(r.d_ctrl, c0.data(), sizeof(Ctrl) * max_members, hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(ENOAO_EDEVICE);
    r.wg_per_cu = Runtime::POOL_WG_PER_CU;
    r.set_grids();
    if (pl->rebuild(s)) return fail(ENOAO_EDEVICE);
    *out = pl;
    return ENOAO_OK;
}

enoao_status enoao_pool_destroy(enoao_pool *pool)
{
    if (!pool) return ENOAO_EINVAL;
    pool->rt.wait_marks();  // the pool's work on the streams it was given
    pool->free_pins();
    pool->rt.release();
    delete pool;
    return ENOAO_OK;
}

enoao_status enoao_pool_set_launch(enoao_pool *pool, int32_t workgroups_per_cu)
{
    if (!pool || workgroups_per_cu < 0 || workgroups_per_cu > 64) return ENOAO_EINVAL;
    pool->rt.set_launch(workgroups_per_cu);
    return ENOAO_OK;
}

enoao_status enoao_pool_admit(enoao_pool *pool, const enoao_problem *prob, const double *u0, int32_t u0_on_host,
                              double t_final, int64_t max_steps, double cfl, int32_t *slot_out, void *stream)
{
    if (!pool || !prob || !u0 || !slot_out || max_steps < 0 || !(cfl > 0.0) || !(t_final >= 0.0)) return ENOAO_EINVAL;
    Runtime &r = pool->rt;
    if (check_problem(prob) || (prob->flags & ENOAO_F_RECORD_SELECTION)) return ENOAO_EINVAL;
    if (prob->equation != r.eq || prob->order != r.order || prob->gamma != r.gamma || prob->delta != r.delta ||
        prob->recon_vars != r.probs[0].recon_vars)
        return ENOAO_EINVAL;
    const size_t bytes = pool_member_bytes(prob);
    if (bytes > pool->arena_bytes) return ENOAO_EINVAL;  // can never fit
    int slot = -1;
    for (int k = 0; k < pool->max_members; ++k)
        if (!pool->slots[k].used) { slot = k; break; }
    if (slot < 0) return ENOAO_ENOMEM;
    size_t off;
    if (!pool->arena_alloc(bytes, off)) return ENOAO_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    // dense rows of the caller into the member's padded rows (a host state goes
    // through the member's w1 buffer, unused until its first step)
    const int pitch = padded_pitch(prob->nx);
    const long long rows = (long long)r.nc * prob->ny;
    double *mem = (double *)(pool->arena + off);
    const size_t cells = (size_t)r.nc * pitch * prob->ny;
    const double *src = u0;
    if (u0_on_host) {
        double *tmp = member_buffer(mem, cells, 1);
        if (hipMemcpyAsync(tmp, u0, (size_t)rows * prob->nx * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess) {
            pool->arena_free(off, bytes);
            return ENOAO_EDEVICE;
        }
        src = tmp;
    }
    if (launch_copy_pitched(src, prob->nx, member_buffer(mem, cells, 0), pitch, prob->nx, rows, s) != hipSuccess) {
        pool->arena_free(off, bytes);
        return ENOAO_EDEVICE;
    }
    Ctrl c;
    std::memset(&c, 0, sizeof(Ctrl));
    c.t_final = t_final;
    c.cfl = cfl;
    c.max_steps = max_steps;
    if (launch_set_ctrl(r.d_ctrl + slot, c, nullptr, s) != hipSuccess) {
        pool->arena_free(off, bytes);
        return ENOAO_EDEVICE;
    }
    HIP_TRY(r.mark(s));
    pool->slots[slot].used = true;
    pool->slots[slot].prob = *prob;
    pool->slots[slot].off = off;
    pool->slots[slot].bytes = bytes;
    pool->dirty = true;
    *slot_out = slot;
    return ENOAO_OK;
}

enoao_status enoao_pool_step(enoao_pool *pool, int32_t nsteps, void *stream)
{
    if (!pool || nsteps < 1) return ENOAO_EINVAL;
    Runtime &r = pool->rt;
    hipStream_t s = (hipStream_t)stream;
    if (pool->dirty) {
        if (enoao_status e = pool->rebuild(s)) return e;
        if (r.n > 0) {
            // alpha and the first step of every member from its current state
            if (enoao_status e = r.reset_and_maxima(s)) return e;
        }
    }
    if (r.n > 0)
        if (enoao_status e = r.run_steps(nsteps, s)) return e;
    HIP_TRY(r.mark(s));
    return ENOAO_OK;
}

enoao_status enoao_pool_poll(enoao_pool *pool, int32_t *done, int32_t *status, int64_t *steps, double *t,
                             int32_t n, void *stream)
{
    if (!pool || n != pool->max_members) return ENOAO_EINVAL;
    Runtime &r = pool->rt;
    if (enoao_status e = r.read_ctrl((hipStream_t)stream)) return e;
    for (int k = 0; k < n; ++k) {
        const bool used = pool->slots[k].used;
        if (done) done[k] = used ? r.h_ctrl[k].done : -1;
        if (status) status[k] = used ? r.h_ctrl[k].status : 0;
        if (steps) steps[k] = used ? r.h_ctrl[k].steps : 0;
        if (t) t[k] = used ? r.h_ctrl[k].t : 0.0;
    }
    return ENOAO_OK;
}

enoao_status enoao_pool_retire(enoao_pool *pool, int32_t slot, double *u_out, int32_t u_out_on_host, void *stream)
{
    if (!pool || slot < 0 || slot >= pool->max_members || !pool->slots[slot].used) return ENOAO_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (enoao_status e = pool->release_slot(slot, u_out, u_out_on_host != 0, nullptr, s)) return e;
    HIP_TRY(hipStreamSynchronize(s));
    return ENOAO_OK;
}

enoao_status enoao_pool_retire_async(enoao_pool *pool, int32_t slot, double *u_out, double *info, void *stream)
{
    if (!pool || slot < 0 || slot >= pool->max_members || !pool->slots[slot].used) return ENOAO_EINVAL;
    return pool->release_slot(slot, u_out, false, info, (hipStream_t)stream);
}

enoao_status enoao_pool_usage(const enoao_pool *pool, size_t *arena_used, size_t *arena_total, int32_t *members)
{
    if (!pool) return ENOAO_EINVAL;
    size_t fr = 0;
    for (auto &f : pool->free_list) fr += f.second;
    if (arena_used) *arena_used = pool->arena_bytes - fr;
    if (arena_total) *arena_total = pool->arena_bytes;
    if (members) {
        int m = 0;
        for (auto &sl : pool->slots) m += sl.used;
        *members = m;
    }
    return ENOAO_OK;
}

}  // extern "C"
