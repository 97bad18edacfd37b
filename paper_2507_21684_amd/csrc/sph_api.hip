// sph_api.hip -- host side of libsph: plans, workspace layout, launch sequences and the
// C ABI declared in include/sph.h.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sph.h"
#include "sph_device.hpp"

using namespace sph;

namespace {

thread_local std::string g_err;

sph_status fail(sph_status code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(SPH_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define LAUNCH_CHECK(name)                                                                   \
    do {                                                                                     \
        hipError_t e_ = hipGetLastError();                                                   \
        if (e_ != hipSuccess) return fail(SPH_ERR_DEVICE, std::string("launch ") + name + ": " + hipGetErrorString(e_)); \
    } while (0)

#define RC_TRY(expr)                  \
    do {                              \
        sph_status rc_ = (expr);      \
        if (rc_ != SPH_OK) return rc_; \
    } while (0)

constexpr double kCellMargin = 1.0 + 1.0 / 1024.0;  // cell side exceeds H/sub by more than rounding
constexpr int64_t kGroupedBuildCells = 65536;         // 2D plans with this many cell slots build by 2 x 2 groups

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

uint64_t morton(int bx, int by, int bz, int dim)
{
    uint64_t code = 0;
    for (int b = 0; b < 21; ++b) {
        if (dim == 3) {
            code |= (uint64_t)((bx >> b) & 1) << (3 * b);
            code |= (uint64_t)((by >> b) & 1) << (3 * b + 1);
            code |= (uint64_t)((bz >> b) & 1) << (3 * b + 2);
        } else {
            code |= (uint64_t)((bx >> b) & 1) << (2 * b);
            code |= (uint64_t)((by >> b) & 1) << (2 * b + 1);
        }
    }
    return code;
}

struct SimHost {
    int64_t p0, n;
    int32_t cell0, blk0, nc, sub, B, nb, Bd, nblk, ncu;
};

// Per-step data kept in one tape slot: the sorted state, the packed per-particle data read
// by the sweeps, the original indices and the neighbour lists.
struct SlotLayout {
    size_t SA, jd0, jd1, orig, nbr, cnt;
};

}  // namespace

struct sph_plan {
    int32_t dim = 0, dtype = 0, nsims = 0, width = 0, tape_depth = 0, nslots = 2;
    int32_t lpp_fwd = 4, lpp_adj = 4;
    bool filter = false;      // some simulation has a skin: sweeps keep only pairs with r < H
    int32_t reuse = 1;        // a step rebuilds the cell list and the lists every `reuse` steps
    bool speed_skins = false; // per-particle half skins from the particles' speeds (else uniform)
    std::vector<int> list_of; // tape slot -> slot whose neighbour lists it uses
    // explicit Runge-Kutta tableau (0 stages: the semi-implicit Euler step)
    int32_t rk_stages = 0, rk_reserved = 0;
    double rk_A[kMaxStages * kMaxStages] = {}, rk_b[kMaxStages] = {};
    // symplectic Euler (uses the stage storage with two stages), optionally re-using the last
    // substep's rates as the next predictor's
    bool symplectic = false, symp_reuse = false, rate_tape = false;
    // delta-diffusion with the renormalised density gradient (records reserved once)
    bool renorm = false, renorm_reserved = false;
    size_t bytes_base = 0, state_block = 0;
    size_t o_rkU = 0, o_rkK = 0, o_rkUb = 0, o_rkB0 = 0, o_rkTape = 0, o_rkRate = 0;
    size_t o_jdG = 0, o_jdL = 0, o_gbar = 0;
    int64_t N = 0;
    int64_t ncell = 0, nblk = 0;
    std::vector<sph_params> prm;
    std::vector<SimHost> sim;
    std::vector<int32_t> h_blk_coord, h_blk_rank;
    std::vector<unsigned char> h_simc;
    // workspace layout (byte offsets)
    size_t o_simc = 0, o_psim = 0, o_cell_sim = 0, o_blk_coord = 0, o_blk_rank = 0;
    size_t o_cell_count = 0, o_cell_start = 0, o_part = 0, o_cell_of = 0, o_slot_of = 0, o_tmp = 0;
    size_t o_SB = 0, o_jdA = 0, o_jdB = 0, o_status = 0, o_part64 = 0, o_pairs = 0, o_ticket = 0, o_uref = 0;
    // status words of the neighbour export's own list build, kept apart from the plan's status
    // words (an overflow there is returned by sph_neighbors, not left for sph_poll)
    size_t o_status_x = 0;
    // staging of sph_poll_async: the pair total (8 bytes), then the status words
    size_t o_poll = 0;
    // two buffers of adjoint prologue records; adj_buf is the one in use, and adj_ready the tape
    // slot whose records an adjoint sweep has already written there (-1: none)
    size_t o_jdA2 = 0, o_jdB2 = 0;
    int adj_buf = 0, adj_ready = -1;
    std::vector<SlotLayout> slot;
    // Every write of a slot's sorted state or lists gives the slot a new generation number; the
    // last sph_rhs or sph_step call records the slot holding the sort and lists of its input
    // state, which the retained adjoint calls reuse while that slot keeps its generation.
    std::vector<uint64_t> slot_gen;
    uint64_t gen_counter = 0;
    int32_t kept_slot = -1;
    uint64_t kept_gen = 0;
    void touch(int sl) { slot_gen[(size_t)sl] = ++gen_counter; }
    void touch_all()
    {
        for (size_t k = 0; k < slot_gen.size(); ++k) slot_gen[k] = ++gen_counter;
    }
    void keep(int sl)
    {
        kept_slot = sl;
        kept_gen = sl >= 0 ? slot_gen[(size_t)sl] : 0;
    }
    // A semi-implicit Euler sph_step call of nsteps <= the tape slots keeps step t's sorted state
    // and lists in slot t (the forward tape).  A later sph_rollout_backward over the same steps and
    // the checkpoints that call wrote runs its adjoint steps on that tape, without recomputing the
    // segments, while every slot still has the generation the forward left.
    bool ftape = false;
    int32_t ftape_n = 0, ftape_every = 0;
    std::vector<uint64_t> ftape_gen;
    std::vector<uintptr_t> ftape_ckpt;
    int64_t nparts = 0, nparts64 = 0;
    size_t bytes = 0;
    char* ws = nullptr;
    bool bound = false;
    // bound to the static workspace of device scratch_dev by sph_bind_scratch (-1: the caller's
    // workspace), as that device's binding number scratch_gen
    int scratch_dev = -1;
    uint64_t scratch_gen = 0;
    // per-launch timing (sph_profile_enable)
    int32_t prof = 0;   // bit k: time launches of kernel class k
    struct Ev {
        hipEvent_t a, b;
        int kind;
    };
    std::vector<Ev> ev_used;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
    double prof_ms[SPH_KERN_COUNT] = {0, 0, 0, 0, 0};
    int64_t prof_n[SPH_KERN_COUNT] = {0, 0, 0, 0, 0};
    // executable graphs of whole sph_step / sph_rollout_backward calls (sph_set_graphs),
    // keyed by the call's arguments, least recently used evicted first
    struct GraphEntry {
        std::vector<uintptr_t> key;
        hipGraph_t graph;
        hipGraphExec_t exec;
        uint64_t used;
        int32_t kept_slot;  // slot whose retained sort the captured call leaves valid (-1: none)
        // the forward tape the captured step call leaves (ftape_n == 0: none)
        int32_t ftape_n, ftape_every;
        std::vector<uintptr_t> ftape_ckpt;
    };
    bool graphs = false;
    std::vector<GraphEntry> gcache;
    uint64_t gclock = 0;
    hipStream_t capture_stream = nullptr;
    void clear_graphs()
    {
        for (auto& g : gcache) {
            (void)hipGraphExecDestroy(g.exec);
            (void)hipGraphDestroy(g.graph);
        }
        gcache.clear();
    }
    ~sph_plan()
    {
        clear_graphs();
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
        for (auto& e : ev_used) {
            (void)hipEventDestroy(e.a);
            (void)hipEventDestroy(e.b);
        }
        for (auto& e : ev_pool) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    }
};

namespace {

template <typename T>
T* wsp(const sph_plan* p, size_t off) { return reinterpret_cast<T*>(p->ws + off); }

size_t tsize(const sph_plan* p) { return p->dtype == SPH_F64 ? 8 : 4; }

// The pointers of a state, appended to a key.
void key_state(std::vector<uintptr_t>& key, const sph_state* s)
{
    for (int k = 0; k < 3; ++k) {
        key.push_back((uintptr_t)s->x[k]);
        key.push_back((uintptr_t)s->v[k]);
    }
    key.push_back((uintptr_t)s->rho);
}

// Brackets a group of launches of one kernel class with HIP events on the launch stream
// when profiling is enabled.  A scope that holds exactly one kernel launch (one_kernel) gives
// its events to that launch instead (launch_k): hipExtLaunchKernelGGL sets them to the
// kernel's own start and end, without the gaps that events recorded around it would add.
struct ProfScope {
    sph_plan* P;
    hipStream_t st;
    int kind;
    bool one;
    bool launched = false;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(sph_plan* P_, hipStream_t st_, int kind_, bool one_kernel = false)
        : P(P_), st(st_), kind(kind_), one(one_kernel)
    {
        if (!((P->prof >> kind_) & 1)) return;
        if (P->ev_pool.empty()) {
            hipEvent_t e1, e2;
            if (hipEventCreate(&e1) != hipSuccess) return;
            if (hipEventCreate(&e2) != hipSuccess) {
                (void)hipEventDestroy(e1);
                return;
            }
            P->ev_pool.push_back({e1, e2});
        }
        a = P->ev_pool.back().first;
        b = P->ev_pool.back().second;
        P->ev_pool.pop_back();
        if (!one) (void)hipEventRecord(a, st);
    }
    ~ProfScope()
    {
        if (!a) return;
        if (!one) {
            (void)hipEventRecord(b, st);
            launched = true;
        }
        if (launched) P->ev_used.push_back({a, b, kind});
        else P->ev_pool.push_back({a, b});
    }
};

// Launch of `kern`; the kernel that a one-kernel profiling scope times carries its events.
template <typename... KArgs, typename... Args>
void launch_k(ProfScope* prof, void (*kern)(KArgs...), dim3 grid, dim3 block, hipStream_t st, Args... args)
{
    if (prof && prof->a && prof->one && !prof->launched) {
        hipExtLaunchKernelGGL(kern, grid, block, 0, st, prof->a, prof->b, 0, args...);
        prof->launched = true;
    } else {
        kern<<<grid, block, 0, st>>>(args...);
    }
}

template <typename T>
void fill_simconst(const sph_plan* P, std::vector<unsigned char>& out)
{
    out.assign(sizeof(SimConst<T>) * P->nsims, 0);
    SimConst<T>* sc = reinterpret_cast<SimConst<T>*>(out.data());
    const int d = P->dim;
    for (int s = 0; s < P->nsims; ++s) {
        const sph_params& q = P->prm[s];
        const SimHost& h = P->sim[s];
        SimConst<T> c;
        std::memset(&c, 0, sizeof(c));
        const double cd = (d == 2) ? 9.0 / M_PI : 495.0 / (32.0 * M_PI);
        c.L = (T)q.box;
        c.invL = T(1) / c.L;
        c.H = (T)q.support;
        c.H2 = c.H * c.H;
        {
            const T HL = (T)(q.support * (1.0 + q.skin));
            c.HL2 = HL * HL;
            c.hmax = (T)(0.5 * q.skin * q.support);
        }
        {
            // 1 / W(dx) at the initial spacing dx = (m / rho0)^(1/d), for particle shifting
            const double dx = std::pow(q.mass / q.rho0, 1.0 / d), qq = dx / q.support;
            const double t = 1.0 - qq;
            const double w = qq < 1.0 ? t * t * t * t * t * t * (1.0 + 6.0 * qq + (35.0 / 3.0) * qq * qq) : 0.0;
            const double W = cd / std::pow(q.support, d) * w;
            c.invW0 = W > 0.0 ? (T)(1.0 / W) : T(0);
        }
        c.invH = (T)(1.0 / q.support);
        c.cinv = (T)((double)h.nc / q.box);
        c.m = (T)q.mass;
        c.rho0 = (T)q.rho0;
        c.inv_rho0 = (T)(1.0 / q.rho0);
        c.c0sq = (T)(q.c0 * q.c0);
        c.dt = (T)q.dt;
        c.kW = (T)(cd / std::pow(q.support, d));
        c.kG = (T)(cd / std::pow(q.support, d + 2));
        c.kH = (T)(560.0 * cd / std::pow(q.support, d + 4));
        c.epsH2 = (T)(q.eps * q.support * q.support);
        c.cA = (T)(q.alpha * q.support * q.c0 * q.rho0);
        c.cD = (T)(2.0 * q.delta * q.support * q.c0);
        c.Bt = (T)(q.rho0 * q.c0 * q.c0 / 7.0);
        c.p0 = h.p0;
        c.n = h.n;
        c.cell0 = h.cell0;
        c.blk0 = h.blk0;
        c.nc = h.nc;
        c.sub = h.sub;
        c.B = h.B;
        c.nb = h.nb;
        c.Bd = h.Bd;
        c.ncu = h.ncu;
        sc[s] = c;
    }
}

inline unsigned grid_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

template <typename T, int D>
StatePtrs<T, D> user_state(const sph_state* s)
{
    StatePtrs<T, D> p;
    for (int k = 0; k < 3; ++k) {
        p.x[k] = (k < D) ? (T*)s->x[k] : nullptr;
        p.v[k] = (k < D) ? (T*)s->v[k] : nullptr;
    }
    p.rho = (T*)s->rho;
    return p;
}

template <typename T, int D>
StatePtrs<T, D> ws_state(const sph_plan* P, size_t off)
{
    StatePtrs<T, D> p;
    T* base = wsp<T>(P, off);
    for (int k = 0; k < 3; ++k) {
        p.x[k] = (k < D) ? base + (size_t)k * P->N : nullptr;
        p.v[k] = (k < D) ? base + (size_t)(D + k) * P->N : nullptr;
    }
    p.rho = base + (size_t)2 * D * P->N;
    return p;
}

// Exclusive scan in two launches: tile sums with the last workgroup scanning them, then the
// tiles' own scans plus their offsets.
template <typename I>
sph_status scan_exclusive(I* in, int64_t n, I* part, unsigned int* ticket, I* out, bool zero_in, hipStream_t st)
{
    if (n == 0) {
        k_fill<I><<<1, 1, 0, st>>>(out, 1, I(0));
        LAUNCH_CHECK("fill");
        return SPH_OK;
    }
    const unsigned g = grid_for(n, kScanTile);
    k_scan_reduce_last<I><<<g, kScanThreads, 0, st>>>(in, n, part, ticket);
    LAUNCH_CHECK("scan_reduce");
    k_scan_apply<I><<<g, kScanThreads, 0, st>>>(in, n, part, (int64_t)g, out, zero_in ? 1 : 0);
    LAUNCH_CHECK("scan_apply");
    return SPH_OK;
}

// Cell list of `src` (original indices in orig_in, or the identity when null) into tape slot
// `slot`: sorted state, packed sweep data and original indices.
template <typename T, int D>
sph_status sort_into(sph_plan* P, StatePtrs<T, D> src, const int32_t* orig_in, int slot, hipStream_t st,
                     bool assigned = false)
{
    P->touch(slot);
    const int64_t N = P->N;
    if (N == 0) return SPH_OK;
    const SlotLayout& L = P->slot[slot];
    int32_t* cell_count = wsp<int32_t>(P, P->o_cell_count);
    int32_t* cell_start = wsp<int32_t>(P, P->o_cell_start);
    int32_t* cell_of = wsp<int32_t>(P, P->o_cell_of);
    int32_t* slot_of = wsp<int32_t>(P, P->o_slot_of);
    int32_t* tmp = wsp<int32_t>(P, P->o_tmp);
    const int32_t* psim = wsp<int32_t>(P, P->o_psim);
    const SimConst<T>* simc = wsp<SimConst<T>>(P, P->o_simc);
    const int32_t* blk_rank = wsp<int32_t>(P, P->o_blk_rank);
    int32_t* status = wsp<int32_t>(P, P->o_status);
    int32_t* orig_out = wsp<int32_t>(P, L.orig);
    if (orig_in == orig_out) return fail(SPH_ERR_STATE, "sort source and destination slot coincide");
    const unsigned g = grid_for(N, 256);
    ProfScope prof(P, st, SPH_KERN_SORT);
    if (!assigned) {
        k_assign<T, D><<<g, 256, 0, st>>>(N, src, psim, simc, blk_rank, cell_count, cell_of, slot_of, status);
        LAUNCH_CHECK("assign");
    }
    RC_TRY(scan_exclusive<int32_t>(cell_count, P->ncell, wsp<int32_t>(P, P->o_part),
                                   wsp<unsigned int>(P, P->o_ticket), cell_start, true, st));
    k_scatter<<<g, 256, 0, st>>>(N, cell_of, slot_of, cell_start, tmp);
    LAUNCH_CHECK("scatter");
    k_order_gather<T, D><<<g, 256, 0, st>>>(N, tmp, cell_of, cell_start, orig_in, src, ws_state<T, D>(P, L.SA),
                                            orig_out, wsp<vec4_t<T>>(P, L.jd0), wsp<vec4_t<T>>(P, L.jd1), psim,
                                            simc, P->filter ? wsp<vec4_t<T>>(P, P->o_uref) : nullptr,
                                            (T)(P->speed_skins ? kSkinFloor : 1.0),
                                            (T)(P->speed_skins ? kSkinMargin * P->reuse : 0.0));
    LAUNCH_CHECK("order_gather");
    return SPH_OK;
}

// Neighbour lists of the state sorted into `slot` (needs the cell starts of that sort, so it
// runs before the next sort).
// Lists reach the support plus the skin, or exactly the support (`exact`, for the export).
// With a skin the pairs are counted by the forward sweeps, which filter them; without one,
// here.
template <typename T, int D>
sph_status build_lists(sph_plan* P, int slot, hipStream_t st, bool exact = false, int32_t* status = nullptr)
{
    if (P->N == 0 || P->ncell == 0) return SPH_OK;
    if (!status) status = wsp<int32_t>(P, P->o_status);
    const SlotLayout& L = P->slot[slot];
    P->list_of[slot] = slot;
    ProfScope prof(P, st, SPH_KERN_BUILD, true);
    // one wavefront per cell; in 2D with enough cells to fill the GPU four times over, one per
    // group of 2 x 2 cells, which shares the per-wavefront setup of cells with few particles
    const bool group = D == 2 && P->ncell >= kGroupedBuildCells;
    const unsigned groups = (unsigned)(group ? P->ncell / 4 : P->ncell);
    // lists with speed-scaled skins use the half skins of the sort that preceded this build
    if (group) {
        if (P->filter && P->speed_skins && !exact)
            launch_k(&prof, k_build_list<T, D, true, true>, dim3(groups), dim3(64), st,
                wsp<int32_t>(P, P->o_cell_sim), wsp<int32_t>(P, P->o_blk_coord), wsp<int32_t>(P, P->o_blk_rank),
                wsp<SimConst<T>>(P, P->o_simc),
                wsp<int32_t>(P, P->o_cell_start), wsp<vec4_t<T>>(P, L.jd0), P->width,
                wsp<int32_t>(P, L.nbr), wsp<int32_t>(P, L.cnt), status, (unsigned long long*)nullptr, 0,
                (const vec4_t<T>*)wsp<vec4_t<T>>(P, P->o_uref));
        else
            launch_k(&prof, k_build_list<T, D, false, true>, dim3(groups), dim3(64), st,
                wsp<int32_t>(P, P->o_cell_sim), wsp<int32_t>(P, P->o_blk_coord), wsp<int32_t>(P, P->o_blk_rank),
                wsp<SimConst<T>>(P, P->o_simc),
                wsp<int32_t>(P, P->o_cell_start), wsp<vec4_t<T>>(P, L.jd0), P->width,
                wsp<int32_t>(P, L.nbr), wsp<int32_t>(P, L.cnt), status,
                P->filter ? nullptr : wsp<unsigned long long>(P, P->o_pairs), exact ? 1 : 0,
                (const vec4_t<T>*)nullptr);
    } else if (P->filter && P->speed_skins && !exact)
        launch_k(&prof, k_build_list<T, D, true, false>, dim3(groups), dim3(64), st,
            wsp<int32_t>(P, P->o_cell_sim), wsp<int32_t>(P, P->o_blk_coord), wsp<int32_t>(P, P->o_blk_rank),
            wsp<SimConst<T>>(P, P->o_simc),
            wsp<int32_t>(P, P->o_cell_start), wsp<vec4_t<T>>(P, L.jd0), P->width,
            wsp<int32_t>(P, L.nbr), wsp<int32_t>(P, L.cnt), status, (unsigned long long*)nullptr, 0,
            (const vec4_t<T>*)wsp<vec4_t<T>>(P, P->o_uref));
    else
        launch_k(&prof, k_build_list<T, D, false, false>, dim3(groups), dim3(64), st,
            wsp<int32_t>(P, P->o_cell_sim), wsp<int32_t>(P, P->o_blk_coord), wsp<int32_t>(P, P->o_blk_rank),
            wsp<SimConst<T>>(P, P->o_simc),
            wsp<int32_t>(P, P->o_cell_start), wsp<vec4_t<T>>(P, L.jd0), P->width,
            wsp<int32_t>(P, L.nbr), wsp<int32_t>(P, L.cnt), status,
            P->filter ? nullptr : wsp<unsigned long long>(P, P->o_pairs), exact ? 1 : 0,
            (const vec4_t<T>*)nullptr);
    LAUNCH_CHECK("build_list");
    return SPH_OK;
}

// Renormalised density gradient of the state sorted into L, with the lists of LL (and L_i
// when `with_l`, for the adjoint).
template <typename T, int D, int LPP>
void launch_renorm(sph_plan* P, const SlotLayout& L, const SlotLayout& LL, hipStream_t st, bool with_l)
{
    const int64_t lanes = P->N * LPP;
    ProfScope prof(P, st, SPH_KERN_OTHER);
    k_renorm<T, D, LPP><<<grid_for(lanes, 256), 256, 0, st>>>(
        P->N, P->width, wsp<int32_t>(P, LL.nbr), wsp<int32_t>(P, LL.cnt), wsp<vec4_t<T>>(P, L.jd0),
        wsp<vec4_t<T>>(P, L.jd1), ws_state<T, D>(P, L.SA).rho, wsp<int32_t>(P, P->o_psim),
        wsp<SimConst<T>>(P, P->o_simc), P->filter ? 1 : 0, wsp<vec4_t<T>>(P, P->o_jdG),
        with_l ? wsp<vec4_t<T>>(P, P->o_jdL) : nullptr);
}

template <typename T, int D, int MODE, int LPP>
void launch_sweep(sph_plan* P, const SlotLayout& L, const SlotLayout& LL, StatePtrs<T, D> dst, T* drho, T* acc,
                  T* rhosum, NextCells next, NextSlot<T> ns, hipStream_t st, ProfScope* prof)
{
    const int64_t lanes = P->N * LPP;
    if (P->renorm) {
        launch_k(prof, k_sweep<T, D, MODE, LPP, true>, dim3(grid_for(lanes, 256)), dim3(256), st,
            P->N, P->width, wsp<int32_t>(P, LL.nbr), wsp<int32_t>(P, LL.cnt), wsp<vec4_t<T>>(P, L.jd0),
            wsp<vec4_t<T>>(P, L.jd1), ws_state<T, D>(P, L.SA), dst, wsp<int32_t>(P, L.orig), drho, acc, rhosum,
            wsp<int32_t>(P, P->o_psim), wsp<SimConst<T>>(P, P->o_simc), wsp<int32_t>(P, P->o_status), next, ns,
            P->filter ? 1 : 0, P->filter ? wsp<unsigned long long>(P, P->o_pairs) : nullptr,
            (const vec4_t<T>*)wsp<vec4_t<T>>(P, P->o_jdG));
        return;
    }
    launch_k(prof, k_sweep<T, D, MODE, LPP, false>, dim3(grid_for(lanes, 256)), dim3(256), st,
        P->N, P->width, wsp<int32_t>(P, LL.nbr), wsp<int32_t>(P, LL.cnt), wsp<vec4_t<T>>(P, L.jd0),
        wsp<vec4_t<T>>(P, L.jd1), ws_state<T, D>(P, L.SA), dst, wsp<int32_t>(P, L.orig), drho, acc, rhosum,
        wsp<int32_t>(P, P->o_psim), wsp<SimConst<T>>(P, P->o_simc), wsp<int32_t>(P, P->o_status), next, ns,
        P->filter ? 1 : 0, P->filter ? wsp<unsigned long long>(P, P->o_pairs) : nullptr,
        (const vec4_t<T>*)nullptr);
}

// Forward sweep over the state in `slot` with the lists of slot list_of[slot].  MODE step
// integrates into SB (same sorted order), or, with next_slot >= 0 (the next step reuses the
// lists), straight into that slot with its packed records; MODE rhs writes the derivatives
// to the caller's arrays in original order.  With assign_next (MODE step into SB) the sweep
// also does the cell assignment of the next sort.
template <typename T, int D, int MODE>
sph_status sweep(sph_plan* P, int slot, T* drho, T* acc, T* rhosum, hipStream_t st, bool assign_next = false,
                 int next_slot = -1)
{
    if (P->N == 0) return SPH_OK;
    const SlotLayout& L = P->slot[slot];
    const SlotLayout& LL = P->slot[P->list_of[slot]];
    NextCells next{wsp<int32_t>(P, P->o_blk_rank), nullptr, wsp<int32_t>(P, P->o_cell_of),
                   wsp<int32_t>(P, P->o_slot_of)};
    if (assign_next) next.cell_count = wsp<int32_t>(P, P->o_cell_count);
    NextSlot<T> ns{nullptr, nullptr, nullptr, nullptr};
    StatePtrs<T, D> dst = ws_state<T, D>(P, P->o_SB);
    if (next_slot >= 0) {
        P->touch(next_slot);
        const SlotLayout& N2 = P->slot[next_slot];
        dst = ws_state<T, D>(P, N2.SA);
        ns = NextSlot<T>{wsp<vec4_t<T>>(P, N2.jd0), wsp<vec4_t<T>>(P, N2.jd1), wsp<int32_t>(P, N2.orig),
                         wsp<vec4_t<T>>(P, P->o_uref)};
    }
    if (P->renorm) {
        switch (P->lpp_fwd) {
        case 2: launch_renorm<T, D, 2>(P, L, LL, st, false); break;
        case 8: launch_renorm<T, D, 8>(P, L, LL, st, false); break;
        default: launch_renorm<T, D, 4>(P, L, LL, st, false); break;
        }
        LAUNCH_CHECK("renorm");
    }
    ProfScope prof(P, st, SPH_KERN_SWEEP, true);
    switch (P->lpp_fwd) {
    case 2: launch_sweep<T, D, MODE, 2>(P, L, LL, dst, drho, acc, rhosum, next, ns, st, &prof); break;
    case 8: launch_sweep<T, D, MODE, 8>(P, L, LL, dst, drho, acc, rhosum, next, ns, st, &prof); break;
    default: launch_sweep<T, D, MODE, 4>(P, L, LL, dst, drho, acc, rhosum, next, ns, st, &prof); break;
    }
    LAUNCH_CHECK("sweep");
    return SPH_OK;
}

// Back to original order: the state `src` (sorted like `slot`) into dst.
template <typename T, int D>
sph_status unsort_from(sph_plan* P, StatePtrs<T, D> src, int slot, StatePtrs<T, D> dst, hipStream_t st)
{
    if (P->N == 0) return SPH_OK;
    ProfScope prof(P, st, SPH_KERN_OTHER);
    k_unsort<T, D><<<grid_for(P->N, 256), 256, 0, st>>>(P->N, src, wsp<int32_t>(P, P->slot[slot].orig), dst);
    LAUNCH_CHECK("unsort");
    return SPH_OK;
}

size_t jdA_off(const sph_plan* P, int buf) { return buf ? P->o_jdA2 : P->o_jdA; }
size_t jdB_off(const sph_plan* P, int buf) { return buf ? P->o_jdB2 : P->o_jdB; }

template <typename T, int D, int LPP>
void launch_adj(sph_plan* P, const SlotLayout& L, const SlotLayout& LL, StatePtrs<T, D> cot, hipStream_t st,
                bool vjp, ProfScope* prof, NextAdj<T> na)
{
    const int64_t lanes = P->N * LPP;
    if (P->renorm) {
        launch_k(prof, k_adj_sweep<T, D, LPP, true>, dim3(grid_for(lanes, 256)), dim3(256), st,
            P->N, P->width, wsp<int32_t>(P, LL.nbr), wsp<int32_t>(P, LL.cnt), wsp<vec4_t<T>>(P, L.jd0),
            wsp<vec4_t<T>>(P, L.jd1), wsp<vec4_t<T>>(P, jdA_off(P, P->adj_buf)),
            wsp<vec4_t<T>>(P, jdB_off(P, P->adj_buf)), wsp<int32_t>(P, L.orig), cot, wsp<int32_t>(P, P->o_psim),
            wsp<SimConst<T>>(P, P->o_simc), wsp<int32_t>(P, P->o_status), P->filter ? 1 : 0, vjp ? 1 : 0,
            (const vec4_t<T>*)wsp<vec4_t<T>>(P, P->o_jdG), (const vec4_t<T>*)wsp<vec4_t<T>>(P, P->o_jdL),
            wsp<vec4_t<T>>(P, P->o_gbar), na);
        return;
    }
    launch_k(prof, k_adj_sweep<T, D, LPP, false>, dim3(grid_for(lanes, 256)), dim3(256), st,
        P->N, P->width, wsp<int32_t>(P, LL.nbr), wsp<int32_t>(P, LL.cnt), wsp<vec4_t<T>>(P, L.jd0),
        wsp<vec4_t<T>>(P, L.jd1), wsp<vec4_t<T>>(P, jdA_off(P, P->adj_buf)),
        wsp<vec4_t<T>>(P, jdB_off(P, P->adj_buf)), wsp<int32_t>(P, L.orig), cot, wsp<int32_t>(P, P->o_psim),
        wsp<SimConst<T>>(P, P->o_simc), wsp<int32_t>(P, P->o_status), P->filter ? 1 : 0, vjp ? 1 : 0,
        (const vec4_t<T>*)nullptr, (const vec4_t<T>*)nullptr, (vec4_t<T>*)nullptr, na);
}

// Second pass of the renormalised diffusion's adjoint (after the adjoint sweep has written
// gbar), added to cot.
template <typename T, int D, int LPP>
void launch_renorm_adj(sph_plan* P, const SlotLayout& L, const SlotLayout& LL, StatePtrs<T, D> cot, hipStream_t st)
{
    const int64_t lanes = P->N * LPP;
    k_renorm_adj<T, D, LPP><<<grid_for(lanes, 256), 256, 0, st>>>(
        P->N, P->width, wsp<int32_t>(P, LL.nbr), wsp<int32_t>(P, LL.cnt), wsp<vec4_t<T>>(P, L.jd0),
        wsp<vec4_t<T>>(P, jdB_off(P, P->adj_buf)), wsp<vec4_t<T>>(P, P->o_jdG), wsp<vec4_t<T>>(P, P->o_gbar),
        wsp<int32_t>(P, L.orig), cot, wsp<int32_t>(P, P->o_psim), wsp<SimConst<T>>(P, P->o_simc),
        P->filter ? 1 : 0);
}

// Adjoint of the step that starts from the state in `slot` (sorted with its lists built).
// With vjp, the update function's VJP instead: cot holds the cotangents (kx, ka, krho) of
// (v, a, drho/dt) on entry and (xbar, vbar, rhobar) on exit.
// With next_slot >= 0 (a tape slot sharing this slot's particle order, whose adjoint runs next),
// the sweep also writes that step's prologue records into the other buffer, and the next call
// skips its prologue.
template <typename T, int D>
sph_status adjoint(sph_plan* P, int slot, StatePtrs<T, D> cot, hipStream_t st, bool vjp = false,
                   int next_slot = -1)
{
    if (P->N == 0) return SPH_OK;
    const SlotLayout& L = P->slot[slot];
    if (P->adj_ready != slot) {
        ProfScope prof(P, st, SPH_KERN_OTHER);
        k_adj_prologue<T, D><<<grid_for(P->N, 256), 256, 0, st>>>(
            P->N, wsp<int32_t>(P, L.orig), cot, ws_state<T, D>(P, L.SA), wsp<vec4_t<T>>(P, jdA_off(P, P->adj_buf)),
            wsp<vec4_t<T>>(P, jdB_off(P, P->adj_buf)), wsp<int32_t>(P, P->o_psim), wsp<SimConst<T>>(P, P->o_simc),
            vjp ? 1 : 0);
        LAUNCH_CHECK("adj_prologue");
    }
    P->adj_ready = -1;
    const bool fuse = next_slot >= 0 && !vjp && !P->renorm;
    NextAdj<T> na{nullptr, nullptr, nullptr};
    if (fuse)
        na = NextAdj<T>{wsp<vec4_t<T>>(P, jdA_off(P, 1 - P->adj_buf)), wsp<vec4_t<T>>(P, jdB_off(P, 1 - P->adj_buf)),
                        ws_state<T, D>(P, P->slot[next_slot].SA).rho};
    const SlotLayout& LL = P->slot[P->list_of[slot]];
    if (P->renorm) {
        // the step's renormalised gradients and L_i, recomputed from its sorted state
        switch (P->lpp_adj) {
        case 2: launch_renorm<T, D, 2>(P, L, LL, st, true); break;
        case 8: launch_renorm<T, D, 8>(P, L, LL, st, true); break;
        default: launch_renorm<T, D, 4>(P, L, LL, st, true); break;
        }
        LAUNCH_CHECK("renorm");
    }
    {
        ProfScope prof(P, st, SPH_KERN_ADJOINT, true);
        switch (P->lpp_adj) {
        case 2: launch_adj<T, D, 2>(P, L, LL, cot, st, vjp, &prof, na); break;
        case 8: launch_adj<T, D, 8>(P, L, LL, cot, st, vjp, &prof, na); break;
        default: launch_adj<T, D, 4>(P, L, LL, cot, st, vjp, &prof, na); break;
        }
        LAUNCH_CHECK("adj_sweep");
    }
    if (P->renorm) {
        ProfScope prof(P, st, SPH_KERN_OTHER);
        switch (P->lpp_adj) {
        case 2: launch_renorm_adj<T, D, 2>(P, L, LL, cot, st); break;
        case 8: launch_renorm_adj<T, D, 8>(P, L, LL, cot, st); break;
        default: launch_renorm_adj<T, D, 4>(P, L, LL, cot, st); break;
        }
        LAUNCH_CHECK("renorm_adj");
    }
    if (fuse) {
        P->adj_buf = 1 - P->adj_buf;
        P->adj_ready = next_slot;
    }
    return SPH_OK;
}

template <typename T, int D>
sph_status copy_state(sph_plan* P, StatePtrs<T, D> dst, StatePtrs<T, D> src, hipStream_t st)
{
    const size_t b = sizeof(T) * (size_t)P->N;
    if (b == 0) return SPH_OK;
    for (int k = 0; k < D; ++k) {
        HIP_TRY(hipMemcpyAsync(dst.x[k], src.x[k], b, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(dst.v[k], src.v[k], b, hipMemcpyDeviceToDevice, st));
    }
    HIP_TRY(hipMemcpyAsync(dst.rho, src.rho, b, hipMemcpyDeviceToDevice, st));
    return SPH_OK;
}

sph_status check_state(const sph_plan* P, const sph_state* s, const char* what)
{
    if (!s) return fail(SPH_ERR_INVALID_ARG, std::string(what) + " is null");
    if (P->N == 0) return SPH_OK;
    for (int k = 0; k < P->dim; ++k)
        if (!s->x[k] || !s->v[k]) return fail(SPH_ERR_INVALID_ARG, std::string(what) + " has a null array");
    if (!s->rho) return fail(SPH_ERR_INVALID_ARG, std::string(what) + " has a null density array");
    return SPH_OK;
}

// ---------------------------------------------------------------- static workspace
// The workspace of sph_bind_scratch: one array per device, held from the library's load to
// the end of the process.  Host code never uses its name as an address (on the host it is
// only a stand-in for the symbol): the device address comes from hipGetSymbolAddress, once
// per device, with that device current.
static __device__ __align__(256) unsigned char scratch[SPH_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;

struct ScratchSlot {
    void* ptr = nullptr;             // device address of `scratch` on this device
    std::atomic<uint64_t> gen{0};    // number of the latest sph_bind_scratch on this device
};

std::mutex g_scratch_mu;
ScratchSlot g_scratch[kMaxScratchDevices];

sph_status check_bound(const sph_plan* P)
{
    if (!P) return fail(SPH_ERR_INVALID_ARG, "plan is null");
    if (!P->bound) return fail(SPH_ERR_STATE, "plan has no workspace bound (call sph_bind)");
    if (P->scratch_dev >= 0) {
        int dev = -1;
        HIP_TRY(hipGetDevice(&dev));
        if (dev != P->scratch_dev)
            return fail(SPH_ERR_STATE, "plan is bound to the static workspace of device " +
                                           std::to_string(P->scratch_dev) + " but device " + std::to_string(dev) +
                                           " is current");
        if (g_scratch[dev].gen.load() != P->scratch_gen)
            return fail(SPH_ERR_STATE,
                        "the static workspace of this device was bound to another plan since (call sph_bind_scratch again)");
    }
    return SPH_OK;
}

#define DISPATCH(P, FN, ...)                                                       \
    ((P)->dtype == SPH_F32 ? ((P)->dim == 2 ? FN<float, 2>(__VA_ARGS__) : FN<float, 3>(__VA_ARGS__)) \
                           : ((P)->dim == 2 ? FN<double, 2>(__VA_ARGS__) : FN<double, 3>(__VA_ARGS__)))

// Particle shifting of a state in place, and its vector-Jacobian product, each on the state's
// own sort and lists.
template <typename T, int D, int LPP>
void launch_shift(sph_plan* P, StatePtrs<T, D> st_user, T beta, hipStream_t st)
{
    const SlotLayout& L = P->slot[0];
    k_shift<T, D, LPP><<<grid_for(P->N * LPP, 256), 256, 0, st>>>(
        P->N, P->width, wsp<int32_t>(P, L.nbr), wsp<int32_t>(P, L.cnt), wsp<vec4_t<T>>(P, L.jd0),
        wsp<int32_t>(P, L.orig), wsp<int32_t>(P, P->o_psim), wsp<SimConst<T>>(P, P->o_simc), P->filter ? 1 : 0, beta,
        st_user);
}

template <typename T, int D, int LPP>
void launch_shift_adj(sph_plan* P, StatePtrs<T, D> cot, T beta, hipStream_t st)
{
    const SlotLayout& L = P->slot[0];
    k_shift_adj<T, D, LPP><<<grid_for(P->N * LPP, 256), 256, 0, st>>>(
        P->N, P->width, wsp<int32_t>(P, L.nbr), wsp<int32_t>(P, L.cnt), wsp<vec4_t<T>>(P, L.jd0),
        wsp<vec4_t<T>>(P, P->o_jdA), ws_state<T, D>(P, L.SA).rho, wsp<int32_t>(P, L.orig), wsp<int32_t>(P, P->o_psim),
        wsp<SimConst<T>>(P, P->o_simc), P->filter ? 1 : 0, beta, cot);
}

template <typename T, int D>
sph_status do_shift(sph_plan* P, sph_state* s, double beta, hipStream_t st)
{
    if (P->N == 0) return SPH_OK;
    StatePtrs<T, D> u = user_state<T, D>(s);
    RC_TRY((sort_into<T, D>(P, u, nullptr, 0, st)));
    RC_TRY((build_lists<T, D>(P, 0, st)));
    ProfScope prof(P, st, SPH_KERN_OTHER);
    switch (P->lpp_fwd) {
    case 2: launch_shift<T, D, 2>(P, u, (T)beta, st); break;
    case 8: launch_shift<T, D, 8>(P, u, (T)beta, st); break;
    default: launch_shift<T, D, 4>(P, u, (T)beta, st); break;
    }
    LAUNCH_CHECK("shift");
    return SPH_OK;
}

template <typename T, int D>
sph_status do_shift_adjoint(sph_plan* P, const sph_state* s, sph_state* cot, double beta, hipStream_t st)
{
    if (P->N == 0) return SPH_OK;
    RC_TRY((sort_into<T, D>(P, user_state<T, D>(s), nullptr, 0, st)));
    RC_TRY((build_lists<T, D>(P, 0, st)));
    StatePtrs<T, D> c = user_state<T, D>(cot);
    ProfScope prof(P, st, SPH_KERN_OTHER);
    k_pack_xbar<T, D><<<grid_for(P->N, 256), 256, 0, st>>>(P->N, c, wsp<int32_t>(P, P->slot[0].orig),
                                                           wsp<vec4_t<T>>(P, P->o_jdA));
    LAUNCH_CHECK("pack_xbar");
    switch (P->lpp_adj) {
    case 2: launch_shift_adj<T, D, 2>(P, c, (T)beta, st); break;
    case 8: launch_shift_adj<T, D, 8>(P, c, (T)beta, st); break;
    default: launch_shift_adj<T, D, 4>(P, c, (T)beta, st); break;
    }
    LAUNCH_CHECK("shift_adj");
    return SPH_OK;
}

template <typename T, int D>
sph_status do_build_cells(sph_plan* P, const sph_state* s, hipStream_t st)
{
    return sort_into<T, D>(P, user_state<T, D>(s), nullptr, 0, st);
}

template <typename T, int D>
sph_status do_rhs(sph_plan* P, const sph_state* s, void* drho, void* acc, void* rhosum, hipStream_t st)
{
    // the last slot, so that a one-step call's sort of its input (slot 0) stays retained too
    const int sl = P->nslots - 1;
    RC_TRY((sort_into<T, D>(P, user_state<T, D>(s), nullptr, sl, st)));
    RC_TRY((build_lists<T, D>(P, sl, st)));
    P->keep(sl);
    return sweep<T, D, kModeRhs>(P, sl, (T*)drho, (T*)acc, (T*)rhosum, st);
}

// nsteps forward steps from `src` (original order).  Without a tape, steps alternate between
// slots 0 and 1; with a tape, step t keeps its sorted state in slot t.  Step t sorts and
// builds lists when t is a multiple of the plan's reuse interval; otherwise it uses the lists
// of the last build, its state already written into its slot by the previous sweep (same
// particle order).  The sweep of the last step is skipped when `last_sweep` is false (a
// recomputation needs only the states the adjoint steps start from).  *last_slot receives the
// slot of the last step.
template <typename T, int D>
sph_status run_steps(sph_plan* P, StatePtrs<T, D> src, int32_t nsteps, bool tape, bool last_sweep,
                     const sph_state* ckpt, int32_t every, int* last_slot, hipStream_t st)
{
    const int R = P->reuse;
    int slot = 0, list_slot = 0;
    for (int32_t t = 0; t < nsteps; ++t) {
        const int cur = tape ? t : (t & 1);
        if (t % R == 0) {
            if (t == 0) RC_TRY((sort_into<T, D>(P, src, nullptr, cur, st)));
            if (t == 0) P->keep(cur);  // the input state's sort; later writes of the slot retire it
            else
                RC_TRY((sort_into<T, D>(P, ws_state<T, D>(P, P->o_SB), wsp<int32_t>(P, P->slot[slot].orig), cur, st,
                                        true)));
            RC_TRY((build_lists<T, D>(P, cur, st)));
            list_slot = cur;
        }
        P->list_of[cur] = list_slot;
        slot = cur;
        const bool more = t + 1 < nsteps;
        const bool reuse_next = more && (t + 1) % R != 0;
        const int nxt = tape ? t + 1 : ((t + 1) & 1);
        if (more || last_sweep) {
            if (reuse_next) RC_TRY((sweep<T, D, kModeStep>(P, cur, nullptr, nullptr, nullptr, st, false, nxt)));
            else RC_TRY((sweep<T, D, kModeStep>(P, cur, nullptr, nullptr, nullptr, st, more)));
        }
        if (ckpt && (t + 1) % every == 0 && more) {
            if (reuse_next)
                RC_TRY((unsort_from<T, D>(P, ws_state<T, D>(P, P->slot[nxt].SA), nxt,
                                          user_state<T, D>(&ckpt[(t + 1) / every]), st)));
            else
                RC_TRY((unsort_from<T, D>(P, ws_state<T, D>(P, P->o_SB), cur, user_state<T, D>(&ckpt[(t + 1) / every]),
                                          st)));
        }
    }
    *last_slot = slot;
    return SPH_OK;
}

// ---------------------------------------------------------------- explicit Runge-Kutta steps

template <typename T, int D>
StatePtrs<T, D> rk_block(const sph_plan* P, size_t base, int i)
{
    return ws_state<T, D>(P, base + (size_t)i * P->state_block);
}

template <typename T, int D>
sph_status lincomb(sph_plan* P, StatePtrs<T, D> out, StatePtrs<T, D> base, double s0, bool s0_dt, int n,
                   const double* c, const StatePtrs<T, D>* K, bool c_dt, hipStream_t st)
{
    if (P->N == 0) return SPH_OK;
    LinComb<T, D> L{};
    L.out = out;
    L.base = base;
    L.s0 = (T)s0;
    L.s0_dt = s0_dt ? 1 : 0;
    L.c_dt = c_dt ? 1 : 0;
    L.nterm = n;
    for (int j = 0; j < n; ++j) {
        L.c[j] = (T)c[j];
        L.K[j] = K[j];
    }
    ProfScope prof(P, st, SPH_KERN_OTHER);
    k_lincomb<T, D><<<grid_for(P->N, 256), 256, 0, st>>>(P->N, L, wsp<int32_t>(P, P->o_psim),
                                                         wsp<SimConst<T>>(P, P->o_simc));
    LAUNCH_CHECK("lincomb");
    return SPH_OK;
}

// Puts a stage state w (original order) into slot 0 with neighbour lists for its sweeps.  The
// first stage of a step (`first`) sorts and builds; with a skin, later stages keep the first
// stage's particle order and lists (k_repack), the sweeps filtering them to r < H, which the
// skin covers as long as no particle moved more than half of it since the build (checked).
template <typename T, int D>
sph_status stage_into_slot0(sph_plan* P, StatePtrs<T, D> w, bool first, hipStream_t st)
{
    if (first || !P->filter) {
        RC_TRY((sort_into<T, D>(P, w, nullptr, 0, st)));
        return build_lists<T, D>(P, 0, st);
    }
    P->touch(0);
    if (P->N == 0) return SPH_OK;
    const SlotLayout& L = P->slot[0];
    ProfScope prof(P, st, SPH_KERN_SORT);
    k_repack<T, D><<<grid_for(P->N, 256), 256, 0, st>>>(
        P->N, wsp<int32_t>(P, L.orig), w, ws_state<T, D>(P, L.SA), wsp<vec4_t<T>>(P, L.jd0), wsp<vec4_t<T>>(P, L.jd1),
        wsp<vec4_t<T>>(P, P->o_uref), wsp<int32_t>(P, P->o_psim), wsp<SimConst<T>>(P, P->o_simc),
        wsp<int32_t>(P, P->o_status));
    LAUNCH_CHECK("repack");
    return SPH_OK;
}

// Stage states and rates of one Runge-Kutta step from u (original order): u_i = u + dt
// sum_{j<i} A_ij k_j (u_0 = u itself), k_i = f(u_i) = (v_i, a(u_i), drho/dt(u_i)), each rate
// from a sort, a list build and a right-hand-side sweep of the stage state.  The x-rate of
// a stage is its velocity, so K[i].x refers to U[i].v.
template <typename T, int D>
sph_status rk_stages(sph_plan* P, StatePtrs<T, D> u, StatePtrs<T, D>* U, StatePtrs<T, D>* K, hipStream_t st)
{
    const int s = P->rk_stages;
    for (int i = 0; i < s; ++i) {
        U[i] = (i == 0) ? u : rk_block<T, D>(P, P->o_rkU, i);
        if (i > 0) {
            double c[kMaxStages];
            StatePtrs<T, D> Ks[kMaxStages];
            int n = 0;
            for (int j = 0; j < i; ++j)
                if (P->rk_A[i * kMaxStages + j] != 0.0) {
                    c[n] = P->rk_A[i * kMaxStages + j];
                    Ks[n++] = K[j];
                }
            RC_TRY((lincomb<T, D>(P, U[i], u, 1.0, false, n, c, Ks, true, st)));
        }
        K[i] = rk_block<T, D>(P, P->o_rkK, i);
        RC_TRY((stage_into_slot0<T, D>(P, U[i], i == 0, st)));
        RC_TRY((sweep<T, D, kModeRhs>(P, 0, K[i].rho, K[i].v[0], nullptr, st)));
        for (int k = 0; k < 3; ++k) K[i].x[k] = U[i].v[k];
    }
    return SPH_OK;
}

// One Runge-Kutta step of u in place: u <- u + dt sum_i b_i k_i.
template <typename T, int D>
sph_status rk_step(sph_plan* P, StatePtrs<T, D> u, hipStream_t st)
{
    StatePtrs<T, D> U[kMaxStages], K[kMaxStages];
    RC_TRY((rk_stages<T, D>(P, u, U, K, st)));
    double c[kMaxStages];
    StatePtrs<T, D> Ks[kMaxStages];
    int n = 0;
    for (int i = 0; i < P->rk_stages; ++i)
        if (P->rk_b[i] != 0.0) {
            c[n] = P->rk_b[i];
            Ks[n++] = K[i];
        }
    return lincomb<T, D>(P, u, u, 1.0, false, n, c, Ks, true, st);
}

// Vector-Jacobian product of one Runge-Kutta step started at u, cot in place (output
// cotangents in, input cotangents out).  Stages in reverse: kbar_i = dt b_i ubar' + dt
// sum_{l>i} A_li Ubar_l, Ubar_i = (df/du at u_i)^T kbar_i (the adjoint sweep's VJP mode), and
// ubar = ubar' + sum_i Ubar_i.
template <typename T, int D>
sph_status rk_step_adjoint(sph_plan* P, StatePtrs<T, D> u, StatePtrs<T, D> cot, hipStream_t st)
{
    const int s = P->rk_stages;
    StatePtrs<T, D> U[kMaxStages], K[kMaxStages], Ub[kMaxStages];
    RC_TRY((rk_stages<T, D>(P, u, U, K, st)));
    const StatePtrs<T, D> B0 = rk_block<T, D>(P, P->o_rkB0, 0);
    RC_TRY((lincomb<T, D>(P, B0, cot, 1.0, false, 0, nullptr, nullptr, false, st)));
    for (int i = s - 1; i >= 0; --i) {
        Ub[i] = rk_block<T, D>(P, P->o_rkUb, i);
        double c[kMaxStages];
        StatePtrs<T, D> Ks[kMaxStages];
        int n = 0;
        for (int l = i + 1; l < s; ++l)
            if (P->rk_A[l * kMaxStages + i] != 0.0) {
                c[n] = P->rk_A[l * kMaxStages + i];
                Ks[n++] = Ub[l];
            }
        RC_TRY((lincomb<T, D>(P, Ub[i], B0, P->rk_b[i], true, n, c, Ks, true, st)));
        // the stages' lists are those rk_stages left in slot 0 (the first stage's, with a skin)
        RC_TRY((stage_into_slot0<T, D>(P, U[i], !P->filter, st)));
        RC_TRY((adjoint<T, D>(P, 0, Ub[i], st, true)));
    }
    double ones[kMaxStages] = {1.0, 1.0, 1.0, 1.0};
    return lincomb<T, D>(P, cot, B0, 1.0, false, s, ones, Ub, false, st);
}

// ---------------------------------------------------------------- symplectic Euler steps

// Rates (., a, D) = f(w) into r (original order) from a sort, a list build and a sweep of w.
template <typename T, int D>
sph_status rates_at(sph_plan* P, StatePtrs<T, D> w, StatePtrs<T, D> r, bool first, hipStream_t st)
{
    RC_TRY((stage_into_slot0<T, D>(P, w, first, st)));
    return sweep<T, D, kModeRhs>(P, 0, r.rho, r.v[0], nullptr, st);
}

template <typename T, int D>
sph_status symp_final(sph_plan* P, StatePtrs<T, D> u, StatePtrs<T, D> uh, StatePtrs<T, D> r2, hipStream_t st)
{
    if (P->N == 0) return SPH_OK;
    ProfScope prof(P, st, SPH_KERN_OTHER);
    k_symp_final<T, D><<<grid_for(P->N, 256), 256, 0, st>>>(P->N, u, uh, r2, wsp<int32_t>(P, P->o_psim),
                                                            wsp<SimConst<T>>(P, P->o_simc));
    LAUNCH_CHECK("symp_final");
    return SPH_OK;
}

// Predictor state u_h = u + (dt/2) (v, a1, D1) of the step from u whose predictor rates are in
// stage-rate block 0 (evaluated here from u when `fresh`, else left there by the caller), and
// the corrector's rates f(u_h) in stage-rate block 1.
template <typename T, int D>
sph_status symp_stages(sph_plan* P, StatePtrs<T, D> u, bool fresh, StatePtrs<T, D>& uh, StatePtrs<T, D>& r1,
                       StatePtrs<T, D>& r2, hipStream_t st)
{
    r1 = rk_block<T, D>(P, P->o_rkK, 0);
    r2 = rk_block<T, D>(P, P->o_rkK, 1);
    uh = rk_block<T, D>(P, P->o_rkU, 1);
    if (fresh) RC_TRY((rates_at<T, D>(P, u, r1, true, st)));
    StatePtrs<T, D> k1 = r1;
    for (int k = 0; k < 3; ++k) k1.x[k] = u.v[k];  // the predictor's x-rate is v
    const double half = 0.5;
    RC_TRY((lincomb<T, D>(P, uh, u, 1.0, false, 1, &half, &k1, true, st)));
    // with a fresh predictor the step's lists are u's, which the predictor state can keep
    return rates_at<T, D>(P, uh, r2, !fresh, st);
}

// One step of u in place.  With re-use the corrector's rates are copied to block 0 for the
// next step's predictor.
template <typename T, int D>
sph_status symp_step(sph_plan* P, StatePtrs<T, D> u, bool fresh, hipStream_t st)
{
    StatePtrs<T, D> uh, r1, r2;
    RC_TRY((symp_stages<T, D>(P, u, fresh, uh, r1, r2, st)));
    RC_TRY((symp_final<T, D>(P, u, uh, r2, st)));
    if (P->symp_reuse) RC_TRY((lincomb<T, D>(P, r1, r2, 1.0, false, 0, nullptr, nullptr, false, st)));
    return SPH_OK;
}

// Vector-Jacobian product of one step from u, cot in place.  The predictor's rates are f(u)
// when `fresh`, else the caller has put them in stage-rate block 0.  cb_in (has_cb) is the
// cotangent of this step's corrector rates where the next step re-used them; when not
// `fresh`, cb_out receives the cotangent of the re-used predictor rates.  Sequence: the
// corrector's transpose, the VJP of f at u_h (its lists are the last ones built), then the
// predictor's transpose: the VJP of f at u when fresh, else the hand-over to cb_out.
template <typename T, int D>
sph_status symp_step_adjoint(sph_plan* P, StatePtrs<T, D> u, StatePtrs<T, D> cot, bool fresh, bool has_cb,
                             StatePtrs<T, D> cb_in, StatePtrs<T, D> cb_out, hipStream_t st)
{
    StatePtrs<T, D> uh, r1, r2;
    RC_TRY((symp_stages<T, D>(P, u, fresh, uh, r1, r2, st)));
    const StatePtrs<T, D> kb2 = rk_block<T, D>(P, P->o_rkUb, 1);
    const StatePtrs<T, D> ubh = rk_block<T, D>(P, P->o_rkUb, 0);
    const StatePtrs<T, D> b0 = rk_block<T, D>(P, P->o_rkB0, 0);
    if (P->N > 0) {
        ProfScope prof(P, st, SPH_KERN_OTHER);
        k_symp_final_adj<T, D><<<grid_for(P->N, 256), 256, 0, st>>>(
            P->N, cot, u.rho, uh.rho, r2.rho, cb_in, has_cb ? 1 : 0, kb2, ubh, b0, wsp<int32_t>(P, P->o_psim),
            wsp<SimConst<T>>(P, P->o_simc));
        LAUNCH_CHECK("symp_final_adj");
    }
    RC_TRY((adjoint<T, D>(P, 0, kb2, st, true)));               // kb2 <- J_f(u_h)^T kb2
    const double one = 1.0;
    RC_TRY((lincomb<T, D>(P, ubh, ubh, 1.0, false, 1, &one, &kb2, false, st)));  // ubar_h
    RC_TRY((lincomb<T, D>(P, b0, b0, 1.0, false, 1, &one, &ubh, false, st)));
    RC_TRY((lincomb<T, D>(P, ubh, ubh, 0.5, true, 0, nullptr, nullptr, false, st)));  // kb1 = h ubar_h
    if (fresh) {
        RC_TRY((stage_into_slot0<T, D>(P, u, !P->filter, st)));
        RC_TRY((adjoint<T, D>(P, 0, ubh, st, true)));
        return lincomb<T, D>(P, cot, b0, 1.0, false, 1, &one, &ubh, false, st);
    }
    if (P->N == 0) return SPH_OK;
    ProfScope prof(P, st, SPH_KERN_OTHER);
    k_symp_pred_adj<T, D><<<grid_for(P->N, 256), 256, 0, st>>>(P->N, b0, ubh, cot, cb_out);
    LAUNCH_CHECK("symp_pred_adj");
    return SPH_OK;
}

template <typename T, int D>
sph_status do_step(sph_plan* P, sph_state* s, int32_t nsteps, const sph_state* ckpt, int32_t every, hipStream_t st)
{
    if (nsteps == 0) return SPH_OK;
    StatePtrs<T, D> user = user_state<T, D>(s);
    P->keep(-1);
    if (P->symplectic) {
        // with re-use the predictor's rates are evaluated afresh at the first step and at every
        // checkpoint, so that each checkpoint segment can be recomputed on its own
        for (int32_t t = 0; t < nsteps; ++t) {
            const bool at_ckpt = ckpt && t % every == 0;
            if (at_ckpt) RC_TRY((copy_state<T, D>(P, user_state<T, D>(&ckpt[t / every]), user, st)));
            RC_TRY((symp_step<T, D>(P, user, !P->symp_reuse || t == 0 || at_ckpt, st)));
        }
        return SPH_OK;
    }
    if (P->rk_stages > 0) {
        for (int32_t t = 0; t < nsteps; ++t) {
            if (ckpt && t % every == 0) RC_TRY((copy_state<T, D>(P, user_state<T, D>(&ckpt[t / every]), user, st)));
            RC_TRY((rk_step<T, D>(P, user, st)));
        }
        return SPH_OK;
    }
    if (ckpt) RC_TRY((copy_state<T, D>(P, user_state<T, D>(&ckpt[0]), user, st)));
    int last = 0;
    // with room for every step, step t keeps its sorted state and lists in slot t (forward tape)
    const bool tape = nsteps <= P->nslots && P->tape_depth >= nsteps;
    P->ftape = false;
    RC_TRY((run_steps<T, D>(P, user, nsteps, tape, true, ckpt, every, &last, st)));
    if (tape && ckpt) {
        P->ftape = true;
        P->ftape_n = nsteps;
        P->ftape_every = every;
        P->ftape_gen.assign(P->slot_gen.begin(), P->slot_gen.begin() + nsteps);
        P->ftape_ckpt.clear();
        for (int32_t k = 0; k < (nsteps + every - 1) / every; ++k) key_state(P->ftape_ckpt, &ckpt[k]);
    }
    return unsort_from<T, D>(P, ws_state<T, D>(P, P->o_SB), last, user, st);
}

template <typename T, int D>
sph_status do_step_adjoint(sph_plan* P, const sph_state* sn, sph_state* cot, hipStream_t st)
{
    if (P->symplectic)
        return symp_step_adjoint<T, D>(P, user_state<T, D>(sn), user_state<T, D>(cot), true, false,
                                       user_state<T, D>(cot), user_state<T, D>(cot), st);
    if (P->rk_stages > 0) return rk_step_adjoint<T, D>(P, user_state<T, D>(sn), user_state<T, D>(cot), st);
    RC_TRY((sort_into<T, D>(P, user_state<T, D>(sn), nullptr, 0, st)));
    RC_TRY((build_lists<T, D>(P, 0, st)));
    return adjoint<T, D>(P, 0, user_state<T, D>(cot), st);
}

// Checkpointed backward pass: segments in reverse; each is recomputed from its checkpoint
// with its sorted states and neighbour lists kept in the tape, then its adjoint steps run in
// reverse on the taped data.
template <typename T, int D>
sph_status do_rollout_backward(sph_plan* P, const sph_state* ckpt, int32_t nsteps, int32_t every, sph_state* cot,
                               hipStream_t st, bool use_tape)
{
    if (nsteps == 0) return SPH_OK;
    const int32_t nseg = (nsteps + every - 1) / every;
    StatePtrs<T, D> c = user_state<T, D>(cot);
    if (P->symplectic) {
        // each segment recomputed into the state tape (and, with re-use, the predictor rates of
        // each step into the rate tape), then the step VJPs in reverse; the cotangent of re-used
        // rates passes from a step to the one before it and never crosses a segment start, where
        // the forward evaluated the rates afresh
        const StatePtrs<T, D> r1 = rk_block<T, D>(P, P->o_rkK, 0);
        StatePtrs<T, D> cb[2] = {rk_block<T, D>(P, P->o_rkUb, 2), rk_block<T, D>(P, P->o_rkUb, 3)};
        for (int32_t seg = nseg - 1; seg >= 0; --seg) {
            const int32_t len = std::min(every, nsteps - seg * every);
            RC_TRY((copy_state<T, D>(P, rk_block<T, D>(P, P->o_rkTape, 0), user_state<T, D>(&ckpt[seg]), st)));
            for (int32_t t = 0; t + 1 < len; ++t) {
                RC_TRY((copy_state<T, D>(P, rk_block<T, D>(P, P->o_rkTape, t + 1), rk_block<T, D>(P, P->o_rkTape, t),
                                         st)));
                RC_TRY((symp_step<T, D>(P, rk_block<T, D>(P, P->o_rkTape, t + 1), !P->symp_reuse || t == 0, st)));
                if (P->symp_reuse) RC_TRY((copy_state<T, D>(P, rk_block<T, D>(P, P->o_rkRate, t + 1), r1, st)));
            }
            int cur = 0;
            bool has_cb = false;
            for (int32_t t = len - 1; t >= 0; --t) {
                const bool fresh = !P->symp_reuse || t == 0;
                if (!fresh) RC_TRY((copy_state<T, D>(P, r1, rk_block<T, D>(P, P->o_rkRate, t), st)));
                RC_TRY((symp_step_adjoint<T, D>(P, rk_block<T, D>(P, P->o_rkTape, t), c, fresh, has_cb, cb[cur],
                                                cb[1 - cur], st)));
                has_cb = !fresh;
                cur = 1 - cur;
            }
        }
        return SPH_OK;
    }
    if (P->rk_stages > 0) {
        // each segment's step states recomputed into the state tape, then the step VJPs
        for (int32_t seg = nseg - 1; seg >= 0; --seg) {
            const int32_t len = std::min(every, nsteps - seg * every);
            RC_TRY((copy_state<T, D>(P, rk_block<T, D>(P, P->o_rkTape, 0), user_state<T, D>(&ckpt[seg]), st)));
            for (int32_t t = 0; t + 1 < len; ++t) {
                RC_TRY((copy_state<T, D>(P, rk_block<T, D>(P, P->o_rkTape, t + 1), rk_block<T, D>(P, P->o_rkTape, t),
                                         st)));
                RC_TRY((rk_step<T, D>(P, rk_block<T, D>(P, P->o_rkTape, t + 1), st)));
            }
            for (int32_t t = len - 1; t >= 0; --t)
                RC_TRY((rk_step_adjoint<T, D>(P, rk_block<T, D>(P, P->o_rkTape, t), c, st)));
        }
        return SPH_OK;
    }
    if (use_tape) {
        // the forward's tape holds every step: the adjoint steps in reverse, no recomputation
        P->adj_buf = 0;
        P->adj_ready = -1;
        for (int32_t t = nsteps - 1; t >= 0; --t) {
            const int next = (t > 0 && P->list_of[t] == P->list_of[t - 1]) ? t - 1 : -1;
            RC_TRY((adjoint<T, D>(P, t, c, st, false, next)));
        }
        return SPH_OK;
    }
    for (int32_t seg = nseg - 1; seg >= 0; --seg) {
        const int32_t len = std::min(every, nsteps - seg * every);
        int last = 0;
        RC_TRY((run_steps<T, D>(P, user_state<T, D>(&ckpt[seg]), len, true, false, nullptr, 1, &last, st)));
        P->adj_buf = 0;
        P->adj_ready = -1;
        for (int32_t t = len - 1; t >= 0; --t) {
            // the step before shares this state's particle order when no sort happened in between
            const int next = (t > 0 && P->list_of[t] == P->list_of[t - 1]) ? t - 1 : -1;
            RC_TRY((adjoint<T, D>(P, t, c, st, false, next)));
        }
    }
    return SPH_OK;
}

// Whether sph_rollout_backward over (ckpt, nsteps, every) may run on the forward tape: the last
// sph_step call taped exactly these steps with these checkpoints, and no slot was written since.
bool forward_tape_intact(const sph_plan* P, const sph_state* ckpt, int32_t nsteps, int32_t every)
{
    if (!P->ftape || P->ftape_n != nsteps || P->ftape_every != every || P->symplectic || P->rk_stages > 0)
        return false;
    std::vector<uintptr_t> k;
    for (int32_t s2 = 0; s2 < (nsteps + every - 1) / every; ++s2) key_state(k, &ckpt[s2]);
    if (k != P->ftape_ckpt) return false;
    for (int32_t t = 0; t < nsteps; ++t)
        if (P->slot_gen[(size_t)t] != P->ftape_gen[(size_t)t]) return false;
    return true;
}

constexpr size_t kGraphCache = 8;

// Runs `issue(stream)` directly, or, with graphs enabled (and profiling off), as an executable
// graph: captured once per distinct key on a private stream (capture records the launches
// without running them), instantiated, kept, and launched on the caller's stream.
template <typename F>
sph_status run_graphed(sph_plan* P, std::vector<uintptr_t> key, hipStream_t st, F&& issue)
{
    if (!P->graphs || P->prof) return issue(st);
    key.push_back((uintptr_t)P->lpp_fwd);
    key.push_back((uintptr_t)P->lpp_adj);
    key.push_back((uintptr_t)P->reuse);
    key.push_back((uintptr_t)P->rk_stages);
    key.push_back((uintptr_t)(P->symplectic ? 1 + (P->symp_reuse ? 1 : 0) : 0));
    key.push_back((uintptr_t)(P->renorm ? 1 : 0));
    key.push_back((uintptr_t)(P->speed_skins ? 1 : 0));
    for (auto& g : P->gcache) {
        if (g.key == key) {
            g.used = ++P->gclock;
            HIP_TRY(hipGraphLaunch(g.exec, st));
            // the replay rewrites slots without the host bookkeeping of a direct call: every slot
            // gets a new generation, and what the captured call left (a retained sort, a forward
            // tape) is recorded again with them
            P->touch_all();
            P->ftape = false;
            if (g.kept_slot >= 0) P->keep(g.kept_slot);
            if (g.ftape_n > 0) {
                P->ftape = true;
                P->ftape_n = g.ftape_n;
                P->ftape_every = g.ftape_every;
                P->ftape_ckpt = g.ftape_ckpt;
                P->ftape_gen.assign(P->slot_gen.begin(), P->slot_gen.begin() + g.ftape_n);
            }
            return SPH_OK;
        }
    }
    if (!P->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&P->capture_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(P->capture_stream, hipStreamCaptureModeThreadLocal));
    const sph_status rc = issue(P->capture_stream);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(P->capture_stream, &graph);
    if (rc != SPH_OK || ec != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (rc != SPH_OK) return rc;
        return fail(SPH_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(SPH_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
    }
    if (P->gcache.size() >= kGraphCache) {
        auto lru = std::min_element(P->gcache.begin(), P->gcache.end(),
                                    [](const sph_plan::GraphEntry& a, const sph_plan::GraphEntry& b) {
                                        return a.used < b.used;
                                    });
        (void)hipGraphExecDestroy(lru->exec);
        (void)hipGraphDestroy(lru->graph);
        P->gcache.erase(lru);
    }
    // a step call leaves its input's sort retained (when valid at the end of the call)
    const int32_t kept = (key[0] == 1 && P->kept_slot >= 0 && P->slot_gen[(size_t)P->kept_slot] == P->kept_gen)
                             ? P->kept_slot
                             : -1;
    bool tape_left = key[0] == 1 && P->ftape;
    for (int32_t t = 0; tape_left && t < P->ftape_n; ++t) tape_left = P->slot_gen[(size_t)t] == P->ftape_gen[(size_t)t];
    P->gcache.push_back({std::move(key), graph, exec, ++P->gclock, kept, tape_left ? P->ftape_n : 0,
                         tape_left ? P->ftape_every : 0,
                         tape_left ? P->ftape_ckpt : std::vector<uintptr_t>()});
    HIP_TRY(hipGraphLaunch(exec, st));
    return SPH_OK;
}


template <typename T, int D, int LPP>
void launch_density_adj(sph_plan* P, const SlotLayout& L, const T* gs, T* xbar, hipStream_t st)
{
    const int64_t lanes = P->N * LPP;
    k_density_adj<T, D, LPP><<<grid_for(lanes, 256), 256, 0, st>>>(
        P->N, P->width, wsp<int32_t>(P, L.nbr), wsp<int32_t>(P, L.cnt), wsp<vec4_t<T>>(P, L.jd0), gs,
        wsp<int32_t>(P, L.orig), wsp<int32_t>(P, P->o_psim), wsp<SimConst<T>>(P, P->o_simc), xbar,
        P->filter ? 1 : 0);
}

// Summation-density VJP of the state s: sort, lists, the cotangent gathered into sorted
// order (adjoint scratch), then the pair sweep writing xbar in original order.
template <typename T, int D>
sph_status do_density_adjoint(sph_plan* P, const sph_state* s, const T* g, T* xbar, hipStream_t st,
                              int kept = -1)
{
    if (P->N == 0) return SPH_OK;
    int sl = kept;
    if (sl < 0) {
        sl = 0;
        RC_TRY((sort_into<T, D>(P, user_state<T, D>(s), nullptr, 0, st)));
        RC_TRY((build_lists<T, D>(P, 0, st)));
    }
    const SlotLayout& L = P->slot[sl];
    T* gs = wsp<T>(P, P->o_jdA);
    ProfScope prof(P, st, SPH_KERN_ADJOINT);
    k_gather_sorted<T><<<grid_for(P->N, 256), 256, 0, st>>>(P->N, g, wsp<int32_t>(P, L.orig), gs);
    LAUNCH_CHECK("gather_sorted");
    switch (P->lpp_adj) {
    case 2: launch_density_adj<T, D, 2>(P, L, gs, xbar, st); break;
    case 8: launch_density_adj<T, D, 8>(P, L, gs, xbar, st); break;
    default: launch_density_adj<T, D, 4>(P, L, gs, xbar, st); break;
    }
    LAUNCH_CHECK("density_adj");
    return SPH_OK;
}

// CSR export (original indices, rows ascending) of the lists in slot 0, whose build flagged its
// faults in the private status words xstat.  SYNCHRONOUS.
sph_status export_lists(sph_plan* P, const int32_t* xstat, int64_t* offsets, int32_t* nbr, int64_t capacity,
                        int64_t* total, hipStream_t st)
{
    const int64_t N = P->N;
    const SlotLayout& L = P->slot[0];
    const int32_t* orig = wsp<int32_t>(P, L.orig);
    int64_t* rowcnt = wsp<int64_t>(P, P->o_part64) + (P->nparts64 + 1);
    if (N > 0) {
        k_export_counts<<<grid_for(N, 256), 256, 0, st>>>(N, orig, wsp<int32_t>(P, L.cnt), P->width, rowcnt);
        LAUNCH_CHECK("export_counts");
    }
    RC_TRY(scan_exclusive<int64_t>(rowcnt, N, wsp<int64_t>(P, P->o_part64), wsp<unsigned int>(P, P->o_ticket),
                                   offsets, false, st));
    int64_t tot = 0;
    HIP_TRY(hipMemcpyAsync(&tot, offsets + N, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    std::vector<int32_t> stat(P->nsims, 0);
    HIP_TRY(hipMemcpyAsync(stat.data(), xstat, sizeof(int32_t) * P->nsims, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *total = tot;
    for (int s2 = 0; s2 < P->nsims; ++s2)
        if (stat[s2] & kFlagBadSupport)
            return fail(SPH_ERR_INVALID_ARG, "simulation " + std::to_string(s2) +
                                                 ": a particle's support is not in (0, H]");
    for (int s2 = 0; s2 < P->nsims; ++s2)
        if (stat[s2] & kFlagOverflow) return fail(SPH_ERR_CAPACITY, "a particle has more neighbours than max_neighbors");
    if (tot > capacity) return fail(SPH_ERR_CAPACITY, "neighbour capacity too small");
    if (N > 0) {
        k_export_rows<<<(unsigned)N, 64, 0, st>>>(N, P->width, orig, wsp<int32_t>(P, L.nbr), wsp<int32_t>(P, L.cnt),
                                                  offsets, nbr);
        LAUNCH_CHECK("export_rows");
    }
    HIP_TRY(hipStreamSynchronize(st));
    return SPH_OK;
}

template <typename T, int D>
sph_status do_neighbors(sph_plan* P, const sph_state* s, int64_t* offsets, int32_t* nbr, int64_t capacity,
                        int64_t* total, hipStream_t st)
{
    RC_TRY((sort_into<T, D>(P, user_state<T, D>(s), nullptr, 0, st)));
    // this build's overflow goes to private status words, cleared first: status bits left by
    // earlier calls neither fail the export nor get the export's overflow added to them
    int32_t* xstat = wsp<int32_t>(P, P->o_status_x);
    k_fill<int32_t><<<grid_for(P->nsims, 256), 256, 0, st>>>(xstat, P->nsims, 0);
    LAUNCH_CHECK("fill");
    RC_TRY((build_lists<T, D>(P, 0, st, true, xstat)));
    return export_lists(P, xstat, offsets, nbr, capacity, total, st);
}

// Lists with a support per particle: sort, supports into sorted order (in the sweep output
// block, free between steps), search radii by atomic maximum, the search with them, the export
// and the radii in original order.
template <typename T, int D>
sph_status do_neighbors_adaptive(sph_plan* P, const sph_state* s, const T* h, T* sr_out, int64_t* offsets,
                                 int32_t* nbr, int64_t capacity, int64_t* total, hipStream_t st)
{
    RC_TRY((sort_into<T, D>(P, user_state<T, D>(s), nullptr, 0, st)));
    int32_t* xstat = wsp<int32_t>(P, P->o_status_x);
    k_fill<int32_t><<<grid_for(P->nsims, 256), 256, 0, st>>>(xstat, P->nsims, 0);
    LAUNCH_CHECK("fill");
    const int64_t N = P->N;
    const SlotLayout& L = P->slot[0];
    P->list_of[0] = 0;
    if (N > 0) {
        T* hs = wsp<T>(P, P->o_SB);
        T* sr = hs + N;
        const int32_t* orig = wsp<int32_t>(P, L.orig);
        const int32_t* psim = wsp<int32_t>(P, P->o_psim);
        const SimConst<T>* simc = wsp<SimConst<T>>(P, P->o_simc);
        const int32_t* cstart = wsp<int32_t>(P, P->o_cell_start);
        const int32_t* brank = wsp<int32_t>(P, P->o_blk_rank);
        const vec4_t<T>* jd0 = wsp<vec4_t<T>>(P, L.jd0);
        const unsigned g = grid_for(N, 256);
        k_adapt_prepare<T><<<g, 256, 0, st>>>(N, h, orig, psim, simc, hs, sr, xstat);
        LAUNCH_CHECK("adapt_prepare");
        {
            ProfScope prof(P, st, SPH_KERN_BUILD);
            k_adapt_radius<T, D><<<g, 256, 0, st>>>(N, jd0, hs, sr, cstart, psim, simc, brank);
            LAUNCH_CHECK("adapt_radius");
            k_adapt_build<T, D><<<g, 256, 0, st>>>(N, jd0, hs, sr, cstart, psim, simc, brank, P->width,
                                                   wsp<int32_t>(P, L.nbr), wsp<int32_t>(P, L.cnt), xstat);
            LAUNCH_CHECK("adapt_build");
        }
        if (sr_out) {
            k_scatter_orig<T><<<g, 256, 0, st>>>(N, sr, orig, sr_out);
            LAUNCH_CHECK("scatter_orig");
        }
    }
    return export_lists(P, xstat, offsets, nbr, capacity, total, st);
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

const char* sph_last_error(void) { return g_err.c_str(); }

sph_status sph_plan_create(const sph_params* sims, int32_t nsims, const int64_t* counts, int32_t max_neighbors,
                           int32_t tape_depth, sph_plan** out)
{
    if (!out) return fail(SPH_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (nsims <= 0 || !sims || !counts) return fail(SPH_ERR_INVALID_ARG, "need nsims > 0, sims and counts");
    if (max_neighbors < 0) return fail(SPH_ERR_INVALID_ARG, "max_neighbors < 0");
    if (tape_depth < 0 || tape_depth > 4096) return fail(SPH_ERR_INVALID_ARG, "tape_depth out of range");
    sph_plan* P = new sph_plan();
    P->dim = sims[0].dim;
    P->dtype = sims[0].dtype;
    P->nsims = nsims;
    P->prm.assign(sims, sims + nsims);
    if (P->dim != 2 && P->dim != 3) {
        delete P;
        return fail(SPH_ERR_INVALID_ARG, "dim must be 2 or 3");
    }
    if (P->dtype != SPH_F32 && P->dtype != SPH_F64) {
        delete P;
        return fail(SPH_ERR_INVALID_ARG, "dtype must be SPH_F32 or SPH_F64");
    }
    const int d = P->dim;
    double nh_max = 0.0;
    int64_t p0 = 0, cell0 = 0, blk0 = 0;
    for (int s = 0; s < nsims; ++s) {
        const sph_params& q = sims[s];
        char buf[256];
        if (q.dim != d || q.dtype != P->dtype) {
            delete P;
            return fail(SPH_ERR_INVALID_ARG, "all simulations of a plan need the same dim and dtype");
        }
        if (counts[s] < 0) {
            delete P;
            return fail(SPH_ERR_INVALID_ARG, "negative particle count");
        }
        const double HL = q.support * (1.0 + q.skin);  // list radius
        if (!(q.skin >= 0) || !std::isfinite(q.skin) || !(2.0 * HL < q.box)) {
            std::snprintf(buf, sizeof buf, "simulation %d: need skin >= 0 and 2 H (1 + skin) < L", s);
            delete P;
            return fail(SPH_ERR_INVALID_ARG, buf);
        }
        if (q.skin > 0) P->filter = true;
        if (!(q.box > 0) || !(q.support > 0) || !(2.0 * q.support < q.box) || !(q.mass > 0) || !(q.rho0 > 0) ||
            !(q.c0 > 0) || !(q.eps > 0) || !std::isfinite(q.dt) || !std::isfinite(q.delta) ||
            !std::isfinite(q.alpha) || !std::isfinite(q.box)) {
            std::snprintf(buf, sizeof buf, "simulation %d: invalid parameters (need 0 < 2H < L, m, rho0, c0, eps > 0)", s);
            delete P;
            return fail(SPH_ERR_INVALID_ARG, buf);
        }
        SimHost h{};
        h.p0 = p0;
        h.n = counts[s];
        const double nc2 = std::floor(2.0 * q.box / (HL * kCellMargin));
        const double nc1 = std::floor(q.box / (HL * kCellMargin));
        if (nc2 >= 5) {
            h.sub = 2;
            h.nc = (int)std::min(nc2, 1e6);
        } else if (nc1 >= 3) {
            h.sub = 1;
            h.nc = (int)nc1;
        } else {
            std::snprintf(buf, sizeof buf, "simulation %d: fewer than 3 cells of side >= H per box side", s);
            delete P;
            return fail(SPH_ERR_TOO_FEW_CELLS, buf);
        }
        int B = (d == 3) ? 2 : 4;
        h.B = B;
        h.nb = (h.nc + B - 1) / B;
        if (h.nb > 1024) {
            delete P;
            return fail(SPH_ERR_UNSUPPORTED, "more than 1024 cell blocks per box side");
        }
        h.Bd = (d == 3) ? B * B * B : B * B;
        h.nblk = (d == 3) ? h.nb * h.nb * h.nb : h.nb * h.nb;
        h.cell0 = (int32_t)cell0;
        h.blk0 = (int32_t)blk0;
        const int sw = 2 * h.sub + 1;
        h.ncu = (d == 3) ? sw * sw * sw : sw * sw;
        cell0 += (int64_t)h.nblk * h.Bd;
        blk0 += h.nblk;
        if (cell0 >= ((int64_t)1 << kStencilIdBits) - 1) {
            delete P;
            return fail(SPH_ERR_UNSUPPORTED, "too many cells in one plan");
        }
        P->sim.push_back(h);
        p0 += counts[s];
        const double dxd = q.mass / q.rho0;
        const double vol = (d == 2) ? M_PI * HL * HL : 4.0 / 3.0 * M_PI * std::pow(HL, 3);
        nh_max = std::max(nh_max, vol / dxd);
    }
    // the sweeps gather per-particle records with 32-bit byte offsets
    const int64_t rec = (P->dtype == SPH_F64) ? 32 : 16;
    if (p0 * rec >= ((int64_t)1 << 32)) {
        delete P;
        return fail(SPH_ERR_UNSUPPORTED, "too many particles in one plan (records must fit 32-bit offsets)");
    }
    P->N = p0;
    P->ncell = cell0;
    P->nblk = blk0;
    P->width = max_neighbors > 0 ? (int32_t)align_up((size_t)max_neighbors, 8)
                                 : (int32_t)align_up((size_t)std::ceil(1.6 * nh_max), 8);
    if (P->width < 8) P->width = 8;
    P->tape_depth = tape_depth;
    P->nslots = std::max(2, tape_depth);
    // lanes per particle of the sweeps (the autotuner may change it; results do not depend on it)
    P->lpp_fwd = P->lpp_adj = 4;

    // host tables: block coordinates in Morton order of each simulation and the rank of every
    // row-major block index (the particle -> simulation and cell -> simulation tables are
    // filled on the device at bind time)
    P->h_blk_coord.resize((size_t)P->nblk);
    P->h_blk_rank.resize((size_t)P->nblk);
    for (int s = 0; s < nsims; ++s) {
        const SimHost& h = P->sim[s];
        std::vector<std::pair<uint64_t, int32_t>> blocks;
        blocks.reserve((size_t)h.nblk);
        for (int lin = 0; lin < h.nblk; ++lin) {
            int bx = lin % h.nb, by = (lin / h.nb) % h.nb, bz = (d == 3) ? lin / (h.nb * h.nb) : 0;
            blocks.push_back({morton(bx, by, bz, d), lin});
        }
        std::sort(blocks.begin(), blocks.end());
        for (int r = 0; r < h.nblk; ++r) {
            int lin = blocks[r].second;
            int bx = lin % h.nb, by = (lin / h.nb) % h.nb, bz = (d == 3) ? lin / (h.nb * h.nb) : 0;
            P->h_blk_coord[(size_t)(h.blk0 + r)] = bx | (by << 10) | (bz << 20);
            P->h_blk_rank[(size_t)(h.blk0 + lin)] = r;
        }
    }
    if (P->dtype == SPH_F32) fill_simconst<float>(P, P->h_simc);
    else fill_simconst<double>(P, P->h_simc);

    // workspace layout
    const size_t A = 256;
    const size_t N = (size_t)P->N, T = tsize(P), V4 = 4 * T;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1), A);
        return o;
    };
    P->nparts = (P->ncell + kScanTile - 1) / kScanTile;
    P->nparts64 = ((int64_t)N + kScanTile - 1) / kScanTile;
    P->o_simc = take(P->h_simc.size());
    P->o_psim = take(4 * N);
    P->o_cell_sim = take(4 * (size_t)P->ncell);
    P->o_blk_coord = take(4 * (size_t)P->nblk);
    P->o_blk_rank = take(4 * (size_t)P->nblk);
    P->o_cell_count = take(4 * (size_t)P->ncell);
    P->o_cell_start = take(4 * ((size_t)P->ncell + 1));
    P->o_part = take(4 * ((size_t)P->nparts + 1));
    P->o_cell_of = take(4 * N);
    P->o_slot_of = take(4 * N);
    P->o_tmp = take(4 * N);
    P->o_SB = take(T * N * (2 * d + 1));
    P->o_jdA = take(V4 * N);
    P->o_jdB = take(V4 * N);
    P->o_jdA2 = take(V4 * N);
    P->o_jdB2 = take(V4 * N);
    P->o_status = take(4 * (size_t)nsims);
    P->o_status_x = take(4 * (size_t)nsims);
    P->o_part64 = take(8 * ((size_t)P->nparts64 + 1) + 8 * (N + 1));
    P->o_pairs = take(8 * (size_t)kPairSlots * kPairStride);
    P->o_ticket = take(4);
    P->o_poll = take(8 + 4 * (size_t)nsims);
    P->o_uref = take(V4 * N);
    P->slot.resize((size_t)P->nslots);
    P->list_of.assign((size_t)P->nslots, 0);
    P->slot_gen.assign((size_t)P->nslots, 0);
    for (int k = 0; k < P->nslots; ++k) {
        SlotLayout& L = P->slot[k];
        L.SA = take(T * N * (2 * d + 1));
        L.jd0 = take(V4 * N);
        L.jd1 = take(V4 * N);
        L.orig = take(4 * N);
        L.nbr = take(4 * (size_t)P->width * N);
        L.cnt = take(4 * N);
    }
    P->bytes_base = off;
    P->state_block = align_up(T * N * (2 * d + 1), A);
    P->bytes = off;
    *out = P;
    return SPH_OK;
}

void sph_plan_destroy(sph_plan* plan) { delete plan; }

sph_status sph_workspace_size(const sph_plan* plan, size_t* bytes)
{
    if (!plan || !bytes) return fail(SPH_ERR_INVALID_ARG, "null argument");
    *bytes = plan->bytes;
    return SPH_OK;
}

sph_status sph_plan_info(const sph_plan* plan, int64_t* total_particles, int32_t* nsims, int32_t* max_neighbors)
{
    if (!plan) return fail(SPH_ERR_INVALID_ARG, "plan is null");
    if (total_particles) *total_particles = plan->N;
    if (nsims) *nsims = plan->nsims;
    if (max_neighbors) *max_neighbors = plan->width;
    return SPH_OK;
}

sph_status sph_set_tuning(sph_plan* plan, int32_t lanes_fwd, int32_t lanes_adj)
{
    if (!plan) return fail(SPH_ERR_INVALID_ARG, "plan is null");
    auto ok = [](int32_t v) { return v == 2 || v == 4 || v == 8; };
    if (!ok(lanes_fwd) || !ok(lanes_adj)) return fail(SPH_ERR_INVALID_ARG, "lanes per particle must be 2, 4 or 8");
    plan->lpp_fwd = lanes_fwd;
    plan->lpp_adj = lanes_adj;
    return SPH_OK;
}

}  // extern "C"

namespace {

// The optional workspace regions after the plan's base workspace, in a fixed order, each
// present once reserved: the renormalised-gradient records (G, L_i, gbar), then the stage
// storage (stage states, rates and cotangents, the output cotangent and a state tape of
// tape_depth blocks), then a tape of as many rate blocks (the symplectic scheme's re-used
// rates).  Setters that reserve call it before the workspace is bound.
void layout_extras(sph_plan* P)
{
    size_t off = P->bytes_base;
    const size_t sb = P->state_block;
    const size_t depth = (size_t)std::max(1, P->tape_depth);
    if (P->renorm_reserved) {
        const size_t v4 = align_up(4 * tsize(P) * (size_t)P->N, 256);
        P->o_jdG = off;
        off += v4;
        P->o_jdL = off;
        off += 2 * v4;
        P->o_gbar = off;
        off += v4;
    }
    if (P->rk_reserved == 0) {
        P->bytes = off;
        return;
    }
    P->o_rkU = off;
    off += kMaxStages * sb;
    P->o_rkK = off;
    off += kMaxStages * sb;
    P->o_rkUb = off;
    off += kMaxStages * sb;
    P->o_rkB0 = off;
    off += sb;
    P->o_rkTape = off;
    off += depth * sb;
    if (P->rate_tape) {
        P->o_rkRate = off;
        off += depth * sb;
    }
    P->bytes = off;
}

void reserve_stage_storage(sph_plan* P, bool rates)
{
    P->rk_reserved = kMaxStages;
    if (rates) P->rate_tape = true;
    layout_extras(P);
}

}  // namespace

extern "C" {

sph_status sph_set_diffusion(sph_plan* P, int32_t renormalised)
{
    if (!P) return fail(SPH_ERR_INVALID_ARG, "plan is null");
    if (renormalised && !P->renorm_reserved) {
        if (P->bound) return fail(SPH_ERR_CAPACITY, "renormalisation records were not reserved when the workspace was bound");
        P->renorm_reserved = true;
        layout_extras(P);
    }
    P->renorm = renormalised != 0;
    P->clear_graphs();
    return SPH_OK;
}

sph_status sph_set_symplectic(sph_plan* P, int32_t reuse_last_substep)
{
    if (!P) return fail(SPH_ERR_INVALID_ARG, "plan is null");
    if (P->rk_reserved < kMaxStages || !P->rate_tape) {
        if (P->bound) return fail(SPH_ERR_CAPACITY, "stage storage was not reserved when the workspace was bound");
        reserve_stage_storage(P, true);
    }
    // the predictor state is the midpoint tableau's second stage
    P->rk_stages = 2;
    std::fill(P->rk_A, P->rk_A + kMaxStages * kMaxStages, 0.0);
    std::fill(P->rk_b, P->rk_b + kMaxStages, 0.0);
    P->rk_A[1 * kMaxStages + 0] = 0.5;
    P->rk_b[1] = 1.0;
    P->symplectic = true;
    P->symp_reuse = reuse_last_substep != 0;
    P->clear_graphs();
    return SPH_OK;
}

sph_status sph_set_integrator(sph_plan* P, int32_t stages, const double* A, const double* b)
{
    if (!P) return fail(SPH_ERR_INVALID_ARG, "plan is null");
    if (stages < 0 || stages > kMaxStages) return fail(SPH_ERR_INVALID_ARG, "stages must be 0..4");
    if (stages > 0 && (!A || !b)) return fail(SPH_ERR_INVALID_ARG, "tableau arrays are null");
    for (int i = 0; i < stages; ++i) {
        if (!std::isfinite(b[i])) return fail(SPH_ERR_INVALID_ARG, "non-finite tableau weight");
        for (int j = 0; j < stages; ++j) {
            const double a = A[i * stages + j];
            if (!std::isfinite(a) || (j >= i && a != 0.0))
                return fail(SPH_ERR_INVALID_ARG, "the tableau must be explicit (A strictly lower triangular)");
        }
    }
    if (stages > P->rk_reserved) {
        if (P->bound) return fail(SPH_ERR_CAPACITY, "more stages than reserved when the workspace was bound");
        reserve_stage_storage(P, false);
    }
    P->symplectic = false;
    P->symp_reuse = false;
    P->rk_stages = stages;
    std::fill(P->rk_A, P->rk_A + kMaxStages * kMaxStages, 0.0);
    std::fill(P->rk_b, P->rk_b + kMaxStages, 0.0);
    for (int i = 0; i < stages; ++i) {
        P->rk_b[i] = b[i];
        for (int j = 0; j < i; ++j) P->rk_A[i * kMaxStages + j] = A[i * stages + j];
    }
    P->clear_graphs();
    return SPH_OK;
}

sph_status sph_set_reuse(sph_plan* plan, int32_t rebuild_every)
{
    if (!plan) return fail(SPH_ERR_INVALID_ARG, "plan is null");
    if (rebuild_every < 1) return fail(SPH_ERR_INVALID_ARG, "rebuild_every must be >= 1");
    if (rebuild_every > 1 && !plan->filter)
        return fail(SPH_ERR_INVALID_ARG, "reusing lists needs a skin (sph_params.skin > 0)");
    plan->reuse = rebuild_every;
    return SPH_OK;
}

sph_status sph_set_skin_mode(sph_plan* plan, int32_t speed_scaled)
{
    if (!plan) return fail(SPH_ERR_INVALID_ARG, "plan is null");
    if (speed_scaled && !plan->filter)
        return fail(SPH_ERR_INVALID_ARG, "speed-scaled skins need a skin (sph_params.skin > 0)");
    plan->speed_skins = speed_scaled != 0;
    return SPH_OK;
}

sph_status sph_set_graphs(sph_plan* plan, int32_t enable)
{
    if (!plan) return fail(SPH_ERR_INVALID_ARG, "plan is null");
    plan->graphs = enable != 0;
    if (!plan->graphs) plan->clear_graphs();
    return SPH_OK;
}

sph_status sph_get_tuning(const sph_plan* plan, int32_t* lanes_fwd, int32_t* lanes_adj)
{
    if (!plan) return fail(SPH_ERR_INVALID_ARG, "plan is null");
    if (lanes_fwd) *lanes_fwd = plan->lpp_fwd;
    if (lanes_adj) *lanes_adj = plan->lpp_adj;
    return SPH_OK;
}

sph_status sph_bind(sph_plan* P, void* workspace, size_t bytes, void* stream)
{
    if (!P) return fail(SPH_ERR_INVALID_ARG, "plan is null");
    if (!workspace) return fail(SPH_ERR_INVALID_ARG, "workspace is null");
    if (bytes < P->bytes) return fail(SPH_ERR_CAPACITY, "workspace smaller than sph_workspace_size()");
    if (((uintptr_t)workspace) % 256 != 0) return fail(SPH_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    P->clear_graphs();          // captured graphs hold addresses inside the old workspace
    P->scratch_dev = -1;
    P->ws = (char*)workspace;
    HIP_TRY(hipMemcpyAsync(P->ws + P->o_simc, P->h_simc.data(), P->h_simc.size(), hipMemcpyHostToDevice, st));
    if (P->nblk > 0) {
        HIP_TRY(hipMemcpyAsync(P->ws + P->o_blk_coord, P->h_blk_coord.data(), 4 * (size_t)P->nblk, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(P->ws + P->o_blk_rank, P->h_blk_rank.data(), 4 * (size_t)P->nblk, hipMemcpyHostToDevice, st));
    }
    if (P->N > 0 || P->ncell > 0) {
        const int64_t n = std::max<int64_t>(P->N, P->ncell);
        if (P->dtype == SPH_F32)
            k_sim_index<float><<<grid_for(n, 256), 256, 0, st>>>(P->N, P->ncell, P->nsims,
                                                                 wsp<SimConst<float>>(P, P->o_simc),
                                                                 wsp<int32_t>(P, P->o_psim), wsp<int32_t>(P, P->o_cell_sim));
        else
            k_sim_index<double><<<grid_for(n, 256), 256, 0, st>>>(P->N, P->ncell, P->nsims,
                                                                  wsp<SimConst<double>>(P, P->o_simc),
                                                                  wsp<int32_t>(P, P->o_psim), wsp<int32_t>(P, P->o_cell_sim));
        LAUNCH_CHECK("sim_index");
    }
    if (P->ncell > 0) {
        k_fill<int32_t><<<grid_for(P->ncell, 256), 256, 0, st>>>(wsp<int32_t>(P, P->o_cell_count), P->ncell, 0);
        LAUNCH_CHECK("fill");
    }
    k_fill<int32_t><<<grid_for(P->nsims, 256), 256, 0, st>>>(wsp<int32_t>(P, P->o_status), P->nsims, 0);
    LAUNCH_CHECK("fill");
    k_fill<unsigned int><<<1, 1, 0, st>>>(wsp<unsigned int>(P, P->o_ticket), 1, 0u);
    LAUNCH_CHECK("fill");
    k_fill<unsigned long long><<<grid_for(kPairSlots * kPairStride, 256), 256, 0, st>>>(
        wsp<unsigned long long>(P, P->o_pairs), kPairSlots * kPairStride, 0ull);
    LAUNCH_CHECK("fill");
    // the tables are copied from pageable host memory, which the runtime stages before the
    // copy call returns, so nothing here waits for the device
    P->bound = true;
    return SPH_OK;
}

sph_status sph_bind_scratch(sph_plan* P, void* stream)
{
    if (!P) return fail(SPH_ERR_INVALID_ARG, "plan is null");
    if (P->bytes > (size_t)SPH_SCRATCH_BYTES)
        return fail(SPH_ERR_CAPACITY, "plan needs a workspace of " + std::to_string(P->bytes) +
                                          " bytes; the static workspace holds " +
                                          std::to_string((size_t)SPH_SCRATCH_BYTES));
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices) return fail(SPH_ERR_UNSUPPORTED, "device index out of range");
    void* ptr = nullptr;
    uint64_t gen = 0;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch[dev].ptr) {
            HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
            if (!ptr || ((uintptr_t)ptr) % 256 != 0)
                return fail(SPH_ERR_DEVICE, "static workspace has no 256-byte aligned device address");
            g_scratch[dev].ptr = ptr;
        }
        ptr = g_scratch[dev].ptr;
        gen = g_scratch[dev].gen.fetch_add(1) + 1;
    }
    RC_TRY(sph_bind(P, ptr, (size_t)SPH_SCRATCH_BYTES, stream));
    P->scratch_dev = dev;
    P->scratch_gen = gen;
    return SPH_OK;
}

sph_status sph_build_cells(sph_plan* P, const sph_state* s, void* stream)
{
    RC_TRY(check_bound(P));
    RC_TRY(check_state(P, s, "state"));
    return DISPATCH(P, do_build_cells, P, s, (hipStream_t)stream);
}

sph_status sph_neighbors(sph_plan* P, const sph_state* s, int64_t* offsets, int32_t* nbr, int64_t capacity,
                         int64_t* total, void* stream)
{
    RC_TRY(check_bound(P));
    RC_TRY(check_state(P, s, "state"));
    if (!offsets || !total) return fail(SPH_ERR_INVALID_ARG, "offsets and total must not be null");
    if (capacity < 0 || (capacity > 0 && !nbr)) return fail(SPH_ERR_INVALID_ARG, "bad neighbour buffer");
    return DISPATCH(P, do_neighbors, P, s, offsets, nbr, capacity, total, (hipStream_t)stream);
}

sph_status sph_neighbors_adaptive(sph_plan* P, const sph_state* s, const void* support, void* search_radius,
                                  int64_t* offsets, int32_t* nbr, int64_t capacity, int64_t* total, void* stream)
{
    RC_TRY(check_bound(P));
    RC_TRY(check_state(P, s, "state"));
    if (!offsets || !total) return fail(SPH_ERR_INVALID_ARG, "offsets and total must not be null");
    if (P->N > 0 && !support) return fail(SPH_ERR_INVALID_ARG, "support must not be null");
    if (capacity < 0 || (capacity > 0 && !nbr)) return fail(SPH_ERR_INVALID_ARG, "bad neighbour buffer");
    hipStream_t st = (hipStream_t)stream;
    if (P->dtype == SPH_F32)
        return P->dim == 2 ? do_neighbors_adaptive<float, 2>(P, s, (const float*)support, (float*)search_radius,
                                                             offsets, nbr, capacity, total, st)
                           : do_neighbors_adaptive<float, 3>(P, s, (const float*)support, (float*)search_radius,
                                                             offsets, nbr, capacity, total, st);
    return P->dim == 2 ? do_neighbors_adaptive<double, 2>(P, s, (const double*)support, (double*)search_radius,
                                                          offsets, nbr, capacity, total, st)
                       : do_neighbors_adaptive<double, 3>(P, s, (const double*)support, (double*)search_radius,
                                                          offsets, nbr, capacity, total, st);
}

sph_status sph_rhs(sph_plan* P, const sph_state* s, void* drho, void* acc, void* rho_sum, void* stream)
{
    RC_TRY(check_bound(P));
    RC_TRY(check_state(P, s, "state"));
    if (P->N > 0 && (!drho || !acc)) return fail(SPH_ERR_INVALID_ARG, "drho and acc must not be null");
    return DISPATCH(P, do_rhs, P, s, drho, acc, rho_sum, (hipStream_t)stream);
}

sph_status sph_step(sph_plan* P, sph_state* s, int32_t nsteps, const sph_state* ckpt, int32_t ckpt_every,
                    void* stream)
{
    RC_TRY(check_bound(P));
    RC_TRY(check_state(P, s, "state"));
    if (nsteps < 0) return fail(SPH_ERR_INVALID_ARG, "nsteps < 0");
    if (ckpt) {
        if (ckpt_every <= 0) return fail(SPH_ERR_INVALID_ARG, "ckpt_every must be > 0");
        if (nsteps > ckpt_every && ckpt_every % P->reuse != 0)
            return fail(SPH_ERR_INVALID_ARG, "ckpt_every must be a multiple of the list reuse interval");
        const int32_t nslots = (nsteps + ckpt_every - 1) / ckpt_every;
        for (int32_t k = 0; k < nslots; ++k) RC_TRY(check_state(P, &ckpt[k], "checkpoint slot"));
    }
    std::vector<uintptr_t> key = {1u, (uintptr_t)nsteps, (uintptr_t)(ckpt ? ckpt_every : 0)};
    key_state(key, s);
    if (ckpt)
        for (int32_t k = 0; k < (nsteps + ckpt_every - 1) / ckpt_every; ++k) key_state(key, &ckpt[k]);
    return run_graphed(P, std::move(key), (hipStream_t)stream, [&](hipStream_t st) {
        return DISPATCH(P, do_step, P, s, nsteps, ckpt, ckpt_every, st);
    });
}

sph_status sph_step_adjoint(sph_plan* P, const sph_state* s_n, sph_state* cot, void* stream)
{
    RC_TRY(check_bound(P));
    RC_TRY(check_state(P, s_n, "state"));
    RC_TRY(check_state(P, cot, "cotangent"));
    P->adj_ready = -1;
    return DISPATCH(P, do_step_adjoint, P, s_n, cot, (hipStream_t)stream);
}

sph_status sph_retained_lists(const sph_plan* P, int32_t* slot, uint64_t* generation)
{
    if (!P || !slot || !generation) return fail(SPH_ERR_INVALID_ARG, "null argument");
    const bool valid = P->kept_slot >= 0 && P->slot_gen[(size_t)P->kept_slot] == P->kept_gen;
    *slot = valid ? P->kept_slot : -1;
    *generation = valid ? P->kept_gen : 0;
    return SPH_OK;
}

namespace {
// The retained slot when (slot, generation) still names it, else -1.
int retained(const sph_plan* P, int32_t slot, uint64_t generation)
{
    if (slot < 0 || slot >= P->nslots) return -1;
    return P->slot_gen[(size_t)slot] == generation && generation != 0 ? slot : -1;
}
}  // namespace

sph_status sph_step_adjoint_retained(sph_plan* P, const sph_state* s_n, sph_state* cot, int32_t slot,
                                     uint64_t generation, void* stream)
{
    RC_TRY(check_bound(P));
    RC_TRY(check_state(P, s_n, "state"));
    RC_TRY(check_state(P, cot, "cotangent"));
    P->adj_ready = -1;
    const int sl = retained(P, slot, generation);
    if (sl < 0 || P->symplectic || P->rk_stages > 0)
        return DISPATCH(P, do_step_adjoint, P, s_n, cot, (hipStream_t)stream);
    if (P->dtype == SPH_F32)
        return P->dim == 2 ? adjoint<float, 2>(P, sl, user_state<float, 2>(cot), (hipStream_t)stream)
                           : adjoint<float, 3>(P, sl, user_state<float, 3>(cot), (hipStream_t)stream);
    return P->dim == 2 ? adjoint<double, 2>(P, sl, user_state<double, 2>(cot), (hipStream_t)stream)
                       : adjoint<double, 3>(P, sl, user_state<double, 3>(cot), (hipStream_t)stream);
}

sph_status sph_density_adjoint_retained(sph_plan* P, const sph_state* s, const void* rho_sum_bar, void* x_bar,
                                        int32_t slot, uint64_t generation, void* stream)
{
    RC_TRY(check_bound(P));
    RC_TRY(check_state(P, s, "state"));
    if (P->N > 0 && (!rho_sum_bar || !x_bar)) return fail(SPH_ERR_INVALID_ARG, "rho_sum_bar and x_bar must not be null");
    const int sl = retained(P, slot, generation);
    hipStream_t st = (hipStream_t)stream;
    if (P->dtype == SPH_F32)
        return P->dim == 2 ? do_density_adjoint<float, 2>(P, s, (const float*)rho_sum_bar, (float*)x_bar, st, sl)
                           : do_density_adjoint<float, 3>(P, s, (const float*)rho_sum_bar, (float*)x_bar, st, sl);
    return P->dim == 2 ? do_density_adjoint<double, 2>(P, s, (const double*)rho_sum_bar, (double*)x_bar, st, sl)
                       : do_density_adjoint<double, 3>(P, s, (const double*)rho_sum_bar, (double*)x_bar, st, sl);
}

sph_status sph_density_adjoint(sph_plan* P, const sph_state* s, const void* rho_sum_bar, void* x_bar, void* stream)
{
    RC_TRY(check_bound(P));
    RC_TRY(check_state(P, s, "state"));
    if (P->N > 0 && (!rho_sum_bar || !x_bar)) return fail(SPH_ERR_INVALID_ARG, "rho_sum_bar and x_bar must not be null");
    hipStream_t st = (hipStream_t)stream;
    if (P->dtype == SPH_F32)
        return P->dim == 2 ? do_density_adjoint<float, 2>(P, s, (const float*)rho_sum_bar, (float*)x_bar, st)
                           : do_density_adjoint<float, 3>(P, s, (const float*)rho_sum_bar, (float*)x_bar, st);
    return P->dim == 2 ? do_density_adjoint<double, 2>(P, s, (const double*)rho_sum_bar, (double*)x_bar, st)
                       : do_density_adjoint<double, 3>(P, s, (const double*)rho_sum_bar, (double*)x_bar, st);
}

sph_status sph_shift(sph_plan* P, sph_state* s, double beta, void* stream)
{
    RC_TRY(check_bound(P));
    RC_TRY(check_state(P, s, "state"));
    if (!std::isfinite(beta)) return fail(SPH_ERR_INVALID_ARG, "beta must be finite");
    return DISPATCH(P, do_shift, P, s, beta, (hipStream_t)stream);
}

sph_status sph_shift_adjoint(sph_plan* P, const sph_state* s, sph_state* cot, double beta, void* stream)
{
    RC_TRY(check_bound(P));
    RC_TRY(check_state(P, s, "state"));
    RC_TRY(check_state(P, cot, "cotangent"));
    if (!std::isfinite(beta)) return fail(SPH_ERR_INVALID_ARG, "beta must be finite");
    return DISPATCH(P, do_shift_adjoint, P, s, cot, beta, (hipStream_t)stream);
}

sph_status sph_rollout_backward(sph_plan* P, const sph_state* ckpt, int32_t nsteps, int32_t ckpt_every,
                                sph_state* cot, void* stream)
{
    RC_TRY(check_bound(P));
    RC_TRY(check_state(P, cot, "cotangent"));
    if (nsteps < 0 || ckpt_every <= 0) return fail(SPH_ERR_INVALID_ARG, "need nsteps >= 0 and ckpt_every > 0");
    if (nsteps > 0 && !ckpt) return fail(SPH_ERR_INVALID_ARG, "checkpoints are null");
    if (std::min(ckpt_every, nsteps) > P->tape_depth)
        return fail(SPH_ERR_CAPACITY, "plan tape_depth is smaller than the checkpoint interval");
    if (nsteps > ckpt_every && ckpt_every % P->reuse != 0)
        return fail(SPH_ERR_INVALID_ARG, "ckpt_every must be a multiple of the list reuse interval");
    const int32_t nseg = nsteps > 0 ? (nsteps + ckpt_every - 1) / ckpt_every : 0;
    for (int32_t k = 0; k < nseg; ++k) RC_TRY(check_state(P, &ckpt[k], "checkpoint slot"));
    P->adj_ready = -1;
    const bool use_tape = nsteps > 0 && forward_tape_intact(P, ckpt, nsteps, ckpt_every);
    std::vector<uintptr_t> key = {2u, (uintptr_t)nsteps, (uintptr_t)ckpt_every, (uintptr_t)use_tape};
    key_state(key, cot);
    for (int32_t k = 0; k < nseg; ++k) key_state(key, &ckpt[k]);
    return run_graphed(P, std::move(key), (hipStream_t)stream, [&](hipStream_t st) {
        return DISPATCH(P, do_rollout_backward, P, ckpt, nsteps, ckpt_every, cot, st, use_tape);
    });
}

sph_status sph_poll(sph_plan* P, int32_t* per_sim_status, void* stream)
{
    RC_TRY(check_bound(P));
    if (!per_sim_status) return fail(SPH_ERR_INVALID_ARG, "per_sim_status is null");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(per_sim_status, P->ws + P->o_status, sizeof(int32_t) * P->nsims, hipMemcpyDeviceToHost, st));
    k_fill<int32_t><<<grid_for(P->nsims, 256), 256, 0, st>>>(wsp<int32_t>(P, P->o_status), P->nsims, 0);
    LAUNCH_CHECK("fill");
    HIP_TRY(hipStreamSynchronize(st));
    return SPH_OK;
}

sph_status sph_pair_count(sph_plan* P, int64_t* pairs, void* stream)
{
    RC_TRY(check_bound(P));
    if (!pairs) return fail(SPH_ERR_INVALID_ARG, "pairs is null");
    hipStream_t st = (hipStream_t)stream;
    std::vector<unsigned long long> v((size_t)kPairSlots * kPairStride, 0ull);
    HIP_TRY(hipMemcpyAsync(v.data(), P->ws + P->o_pairs, sizeof(unsigned long long) * v.size(), hipMemcpyDeviceToHost,
                           st));
    k_fill<unsigned long long><<<grid_for(kPairSlots * kPairStride, 256), 256, 0, st>>>(
        wsp<unsigned long long>(P, P->o_pairs), kPairSlots * kPairStride, 0ull);
    LAUNCH_CHECK("fill");
    HIP_TRY(hipStreamSynchronize(st));
    unsigned long long total = 0;
    for (int k = 0; k < kPairSlots; ++k) total += v[(size_t)k * kPairStride];
    *pairs = (int64_t)total;
    return SPH_OK;
}

sph_status sph_poll_async(sph_plan* P, int32_t* per_sim_status, int64_t* pairs, void* stream)
{
    RC_TRY(check_bound(P));
    if (!per_sim_status) return fail(SPH_ERR_INVALID_ARG, "per_sim_status is null");
    hipStream_t st = (hipStream_t)stream;
    unsigned long long* stage_pairs = wsp<unsigned long long>(P, P->o_poll);
    int32_t* stage_status = wsp<int32_t>(P, P->o_poll + 8);
    k_poll_stage<<<1, 256, 0, st>>>(P->nsims, wsp<int32_t>(P, P->o_status), wsp<unsigned long long>(P, P->o_pairs),
                                    stage_pairs, stage_status);
    LAUNCH_CHECK("poll_stage");
    HIP_TRY(hipMemcpyAsync(per_sim_status, stage_status, sizeof(int32_t) * P->nsims, hipMemcpyDeviceToHost, st));
    if (pairs) HIP_TRY(hipMemcpyAsync(pairs, stage_pairs, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    return SPH_OK;
}

sph_status sph_profile_enable(sph_plan* P, int32_t enable)
{
    if (!P) return fail(SPH_ERR_INVALID_ARG, "plan is null");
    P->prof = enable & ((1 << SPH_KERN_COUNT) - 1);
    return SPH_OK;
}

sph_status sph_profile_read(sph_plan* P, double* ms, int64_t* launches)
{
    if (!P) return fail(SPH_ERR_INVALID_ARG, "plan is null");
    for (auto& e : P->ev_used) {
        HIP_TRY(hipEventSynchronize(e.b));
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, e.a, e.b));
        P->prof_ms[e.kind] += t;
        P->prof_n[e.kind] += 1;
        P->ev_pool.push_back({e.a, e.b});
    }
    P->ev_used.clear();
    for (int k = 0; k < SPH_KERN_COUNT; ++k) {
        if (ms) ms[k] = P->prof_ms[k];
        if (launches) launches[k] = P->prof_n[k];
        P->prof_ms[k] = 0.0;
        P->prof_n[k] = 0;
    }
    return SPH_OK;
}

}  // extern "C"
