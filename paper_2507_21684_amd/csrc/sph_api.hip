// sph_api.hip -- host side of libsph: plans, workspace layout, launch sequences and the
// C ABI declared in include/sph.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
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

constexpr double kCellMargin = 1.0 + 1.0 / 1024.0;  // cell side exceeds H/sub by more than rounding

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
    int32_t cell0, blk0, nc, sub, B, nb, Bd, nblk;
};

}  // namespace

struct sph_plan {
    int32_t dim = 0, dtype = 0, nsims = 0, maxnbr = 0;
    int64_t N = 0, ld = 0;
    int64_t ncell = 0, nblk = 0;
    std::vector<sph_params> prm;
    std::vector<SimHost> sim;
    std::vector<int32_t> h_psim, h_blk_sim, h_blk_coord, h_blk_rank;
    std::vector<unsigned char> h_simc;
    // workspace layout (byte offsets)
    size_t o_simc = 0, o_psim = 0, o_blk_sim = 0, o_blk_coord = 0, o_blk_rank = 0;
    size_t o_cell_count = 0, o_cell_start = 0, o_part = 0, o_cell_of = 0, o_slot_of = 0, o_tmp = 0;
    size_t o_orig[2] = {0, 0}, o_SA = 0, o_SB = 0, o_jd0 = 0, o_jd1 = 0, o_jdA = 0, o_jdB = 0;
    size_t o_nbr = 0, o_cnt = 0, o_status = 0, o_part64 = 0;
    int64_t nparts = 0, nparts64 = 0;
    size_t bytes = 0;
    char* ws = nullptr;
    bool bound = false;
    int cur_orig = 0;  // index of the orig array written by the last sort
};

namespace {

template <typename T>
T* wsp(const sph_plan* p, size_t off) { return reinterpret_cast<T*>(p->ws + off); }

size_t tsize(const sph_plan* p) { return p->dtype == SPH_F64 ? 8 : 4; }

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

template <typename I>
sph_status scan_exclusive(sph_plan* P, I* in, int64_t n, I* part, int64_t np, I* out, bool zero_in, hipStream_t st)
{
    if (n == 0) {
        k_fill<I><<<1, 1, 0, st>>>(out, 1, I(0));
        LAUNCH_CHECK("fill");
        return SPH_OK;
    }
    unsigned g = grid_for(n, kScanTile);
    k_scan_reduce<I><<<g, kScanThreads, 0, st>>>(in, n, part);
    LAUNCH_CHECK("scan_reduce");
    k_scan_top<I><<<1, 1024, 0, st>>>(part, (int64_t)g);
    LAUNCH_CHECK("scan_top");
    k_scan_apply<I><<<g, kScanThreads, 0, st>>>(in, n, part, (int64_t)g, out, zero_in ? 1 : 0);
    LAUNCH_CHECK("scan_apply");
    (void)np;
    return SPH_OK;
}

// Sort `src` (orig ids in orig_in, or identity when null) into the workspace's sorted state SA.
template <typename T, int D>
sph_status sort_into_SA(sph_plan* P, StatePtrs<T, D> src, const int32_t* orig_in, hipStream_t st)
{
    const int64_t N = P->N;
    if (N == 0) return SPH_OK;
    int32_t* cell_count = wsp<int32_t>(P, P->o_cell_count);
    int32_t* cell_start = wsp<int32_t>(P, P->o_cell_start);
    int32_t* cell_of = wsp<int32_t>(P, P->o_cell_of);
    int32_t* slot_of = wsp<int32_t>(P, P->o_slot_of);
    int32_t* tmp = wsp<int32_t>(P, P->o_tmp);
    const int32_t* psim = wsp<int32_t>(P, P->o_psim);
    const SimConst<T>* simc = wsp<SimConst<T>>(P, P->o_simc);
    const int32_t* blk_rank = wsp<int32_t>(P, P->o_blk_rank);
    int32_t* status = wsp<int32_t>(P, P->o_status);
    const unsigned g = grid_for(N, 256);
    k_assign<T, D><<<g, 256, 0, st>>>(N, src, psim, simc, blk_rank, cell_count, cell_of, slot_of, status);
    LAUNCH_CHECK("assign");
    sph_status rc = scan_exclusive<int32_t>(P, cell_count, P->ncell, wsp<int32_t>(P, P->o_part), P->nparts, cell_start,
                                            true, st);
    if (rc != SPH_OK) return rc;
    k_scatter<<<g, 256, 0, st>>>(N, cell_of, slot_of, cell_start, tmp);
    LAUNCH_CHECK("scatter");
    const int out = orig_in == wsp<int32_t>(P, P->o_orig[0]) ? 1 : 0;
    int32_t* orig_out = wsp<int32_t>(P, P->o_orig[out]);
    k_order_gather<T, D><<<g, 256, 0, st>>>(N, tmp, cell_of, cell_start, orig_in, src, ws_state<T, D>(P, P->o_SA),
                                            orig_out, wsp<vec4_t<T>>(P, P->o_jd0), wsp<vec4_t<T>>(P, P->o_jd1), psim,
                                            simc);
    LAUNCH_CHECK("order_gather");
    P->cur_orig = out;
    return SPH_OK;
}

template <typename T, int D>
sph_status build_lists(sph_plan* P, hipStream_t st)
{
    if (P->N == 0 || P->nblk == 0) return SPH_OK;
    k_build_list<T, D><<<(unsigned)P->nblk, 64, 0, st>>>(
        wsp<int32_t>(P, P->o_blk_sim), wsp<int32_t>(P, P->o_blk_coord), wsp<int32_t>(P, P->o_blk_rank),
        wsp<SimConst<T>>(P, P->o_simc), wsp<int32_t>(P, P->o_cell_start), wsp<vec4_t<T>>(P, P->o_jd0), P->ld,
        P->maxnbr, wsp<int32_t>(P, P->o_nbr), wsp<int32_t>(P, P->o_cnt), wsp<int32_t>(P, P->o_status));
    LAUNCH_CHECK("build_list");
    return SPH_OK;
}

template <typename T, int D, int MODE>
sph_status sweep(sph_plan* P, T* drho, T* acc, T* rhosum, hipStream_t st)
{
    if (P->N == 0) return SPH_OK;
    k_sweep<T, D, MODE><<<grid_for(P->N, 256), 256, 0, st>>>(
        P->N, P->ld, P->maxnbr, wsp<int32_t>(P, P->o_nbr), wsp<int32_t>(P, P->o_cnt), wsp<vec4_t<T>>(P, P->o_jd0),
        wsp<vec4_t<T>>(P, P->o_jd1), ws_state<T, D>(P, P->o_SA), ws_state<T, D>(P, P->o_SB),
        wsp<int32_t>(P, P->o_orig[P->cur_orig]), drho, acc, rhosum, wsp<int32_t>(P, P->o_psim),
        wsp<SimConst<T>>(P, P->o_simc), wsp<int32_t>(P, P->o_status));
    LAUNCH_CHECK("sweep");
    return SPH_OK;
}

template <typename T, int D>
sph_status unsort_SB(sph_plan* P, StatePtrs<T, D> dst, hipStream_t st)
{
    if (P->N == 0) return SPH_OK;
    k_unsort<T, D><<<grid_for(P->N, 256), 256, 0, st>>>(P->N, ws_state<T, D>(P, P->o_SB),
                                                        wsp<int32_t>(P, P->o_orig[P->cur_orig]), dst);
    LAUNCH_CHECK("unsort");
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

sph_status check_bound(const sph_plan* P)
{
    if (!P) return fail(SPH_ERR_INVALID_ARG, "plan is null");
    if (!P->bound) return fail(SPH_ERR_STATE, "plan has no workspace bound (call sph_bind)");
    return SPH_OK;
}

#define DISPATCH(P, FN, ...)                                                       \
    ((P)->dtype == SPH_F32 ? ((P)->dim == 2 ? FN<float, 2>(__VA_ARGS__) : FN<float, 3>(__VA_ARGS__)) \
                           : ((P)->dim == 2 ? FN<double, 2>(__VA_ARGS__) : FN<double, 3>(__VA_ARGS__)))

template <typename T, int D>
sph_status do_build_cells(sph_plan* P, const sph_state* s, hipStream_t st)
{
    return sort_into_SA<T, D>(P, user_state<T, D>(s), nullptr, st);
}

template <typename T, int D>
sph_status do_rhs(sph_plan* P, const sph_state* s, void* drho, void* acc, void* rhosum, hipStream_t st)
{
    sph_status rc = sort_into_SA<T, D>(P, user_state<T, D>(s), nullptr, st);
    if (rc == SPH_OK) rc = build_lists<T, D>(P, st);
    if (rc == SPH_OK) rc = sweep<T, D, kModeRhs>(P, (T*)drho, (T*)acc, (T*)rhosum, st);
    return rc;
}

template <typename T, int D>
sph_status do_step(sph_plan* P, sph_state* s, int32_t nsteps, const sph_state* ckpt, int32_t every, hipStream_t st)
{
    StatePtrs<T, D> user = user_state<T, D>(s);
    if (ckpt && nsteps > 0) {
        sph_status rc = copy_state<T, D>(P, user_state<T, D>(&ckpt[0]), user, st);
        if (rc != SPH_OK) return rc;
    }
    for (int32_t t = 0; t < nsteps; ++t) {
        sph_status rc;
        if (t == 0) rc = sort_into_SA<T, D>(P, user, nullptr, st);
        else rc = sort_into_SA<T, D>(P, ws_state<T, D>(P, P->o_SB), wsp<int32_t>(P, P->o_orig[P->cur_orig]), st);
        if (rc == SPH_OK) rc = build_lists<T, D>(P, st);
        if (rc == SPH_OK) rc = sweep<T, D, kModeStep>(P, nullptr, nullptr, nullptr, st);
        if (rc != SPH_OK) return rc;
        if (ckpt && (t + 1) % every == 0 && t + 1 < nsteps) {
            rc = unsort_SB<T, D>(P, user_state<T, D>(&ckpt[(t + 1) / every]), st);
            if (rc != SPH_OK) return rc;
        }
    }
    if (nsteps > 0) return unsort_SB<T, D>(P, user, st);
    return SPH_OK;
}

template <typename T, int D>
sph_status do_step_adjoint(sph_plan* P, const sph_state* sn, sph_state* cot, hipStream_t st)
{
    sph_status rc = sort_into_SA<T, D>(P, user_state<T, D>(sn), nullptr, st);
    if (rc == SPH_OK) rc = build_lists<T, D>(P, st);
    if (rc != SPH_OK) return rc;
    if (P->N == 0) return SPH_OK;
    const unsigned g = grid_for(P->N, 256);
    const int32_t* orig = wsp<int32_t>(P, P->o_orig[P->cur_orig]);
    k_adj_prologue<T, D><<<g, 256, 0, st>>>(P->N, orig, user_state<T, D>(cot), ws_state<T, D>(P, P->o_SA),
                                            wsp<vec4_t<T>>(P, P->o_jdA), wsp<vec4_t<T>>(P, P->o_jdB),
                                            wsp<int32_t>(P, P->o_psim), wsp<SimConst<T>>(P, P->o_simc));
    LAUNCH_CHECK("adj_prologue");
    k_adj_sweep<T, D><<<g, 256, 0, st>>>(P->N, P->ld, P->maxnbr, wsp<int32_t>(P, P->o_nbr),
                                         wsp<int32_t>(P, P->o_cnt), wsp<vec4_t<T>>(P, P->o_jd0),
                                         wsp<vec4_t<T>>(P, P->o_jd1), wsp<vec4_t<T>>(P, P->o_jdA),
                                         wsp<vec4_t<T>>(P, P->o_jdB), orig, user_state<T, D>(cot),
                                         wsp<int32_t>(P, P->o_psim), wsp<SimConst<T>>(P, P->o_simc),
                                         wsp<int32_t>(P, P->o_status));
    LAUNCH_CHECK("adj_sweep");
    return SPH_OK;
}

template <typename T, int D>
sph_status do_neighbors(sph_plan* P, const sph_state* s, int64_t* offsets, int32_t* nbr, int64_t capacity,
                        int64_t* total, hipStream_t st)
{
    sph_status rc = sort_into_SA<T, D>(P, user_state<T, D>(s), nullptr, st);
    if (rc == SPH_OK) rc = build_lists<T, D>(P, st);
    if (rc != SPH_OK) return rc;
    const int64_t N = P->N;
    const int32_t* orig = wsp<int32_t>(P, P->o_orig[P->cur_orig]);
    int64_t* rowcnt = wsp<int64_t>(P, P->o_part64) + (P->nparts64 + 1);
    if (N > 0) {
        k_export_counts<<<grid_for(N, 256), 256, 0, st>>>(N, orig, wsp<int32_t>(P, P->o_cnt), P->maxnbr, rowcnt);
        LAUNCH_CHECK("export_counts");
    }
    rc = scan_exclusive<int64_t>(P, rowcnt, N, wsp<int64_t>(P, P->o_part64), P->nparts64, offsets, false, st);
    if (rc != SPH_OK) return rc;
    int64_t tot = 0;
    HIP_TRY(hipMemcpyAsync(&tot, offsets + N, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    std::vector<int32_t> stat(P->nsims, 0);
    if (P->nsims > 0)
        HIP_TRY(hipMemcpyAsync(stat.data(), wsp<int32_t>(P, P->o_status), sizeof(int32_t) * P->nsims,
                               hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *total = tot;
    for (int s2 = 0; s2 < P->nsims; ++s2)
        if (stat[s2] & kFlagOverflow)
            return fail(SPH_ERR_CAPACITY, "a particle has more neighbours than max_neighbors");
    if (tot > capacity) return fail(SPH_ERR_CAPACITY, "neighbour capacity too small");
    if (N > 0) {
        k_export_rows<<<(unsigned)N, 64, 0, st>>>(N, P->ld, orig, wsp<int32_t>(P, P->o_nbr),
                                                  wsp<int32_t>(P, P->o_cnt), P->maxnbr, offsets, nbr);
        LAUNCH_CHECK("export_rows");
    }
    HIP_TRY(hipStreamSynchronize(st));
    return SPH_OK;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

const char* sph_last_error(void) { return g_err.c_str(); }

sph_status sph_plan_create(const sph_params* sims, int32_t nsims, const int64_t* counts, int32_t max_neighbors,
                           sph_plan** out)
{
    if (!out) return fail(SPH_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (nsims <= 0 || !sims || !counts) return fail(SPH_ERR_INVALID_ARG, "need nsims > 0, sims and counts");
    if (max_neighbors < 0) return fail(SPH_ERR_INVALID_ARG, "max_neighbors < 0");
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
        if (!(q.box > 0) || !(q.support > 0) || !(2.0 * q.support < q.box) || !(q.mass > 0) || !(q.rho0 > 0) ||
            !(q.c0 > 0) || !(q.eps > 0) || !std::isfinite(q.dt) || !std::isfinite(q.delta) ||
            !std::isfinite(q.alpha)) {
            std::snprintf(buf, sizeof buf, "simulation %d: invalid parameters (need 0 < 2H < L, m, rho0, c0, eps > 0)", s);
            delete P;
            return fail(SPH_ERR_INVALID_ARG, buf);
        }
        SimHost h{};
        h.p0 = p0;
        h.n = counts[s];
        int nc2 = (int)std::floor(2.0 * q.box / (q.support * kCellMargin));
        int nc1 = (int)std::floor(q.box / (q.support * kCellMargin));
        if (nc2 >= 5) {
            h.sub = 2;
            h.nc = nc2;
        } else if (nc1 >= 3) {
            h.sub = 1;
            h.nc = nc1;
        } else {
            std::snprintf(buf, sizeof buf, "simulation %d: fewer than 3 cells of side >= H per box side", s);
            delete P;
            return fail(SPH_ERR_TOO_FEW_CELLS, buf);
        }
        if (h.nc > 1024 * 4) {
            delete P;
            return fail(SPH_ERR_UNSUPPORTED, "more than 4096 cells per box side");
        }
        int B = (d == 3) ? 2 : 4;
        while (B > 1 && B + 2 * h.sub > h.nc) --B;
        h.B = B;
        h.nb = (h.nc + B - 1) / B;
        h.Bd = (d == 3) ? B * B * B : B * B;
        h.nblk = (d == 3) ? h.nb * h.nb * h.nb : h.nb * h.nb;
        h.cell0 = (int32_t)cell0;
        h.blk0 = (int32_t)blk0;
        cell0 += (int64_t)h.nblk * h.Bd;
        blk0 += h.nblk;
        if (cell0 > (int64_t)1 << 30) {
            delete P;
            return fail(SPH_ERR_UNSUPPORTED, "too many cells in one plan");
        }
        P->sim.push_back(h);
        p0 += counts[s];
        const double dxd = q.mass / q.rho0;
        const double vol = (d == 2) ? M_PI * q.support * q.support : 4.0 / 3.0 * M_PI * std::pow(q.support, 3);
        nh_max = std::max(nh_max, vol / dxd);
    }
    if (p0 >= ((int64_t)1 << 31) - 1024) {
        delete P;
        return fail(SPH_ERR_UNSUPPORTED, "more than 2^31 particles in one plan");
    }
    P->N = p0;
    P->ncell = cell0;
    P->nblk = blk0;
    P->ld = (int64_t)align_up((size_t)std::max<int64_t>(P->N, 1), 64);
    P->maxnbr = max_neighbors > 0 ? max_neighbors : (int32_t)align_up((size_t)std::ceil(1.6 * nh_max), 8);
    if (P->maxnbr < 8) P->maxnbr = 8;

    // host tables: particle -> simulation, block tables in Morton order per simulation
    P->h_psim.resize((size_t)P->N);
    P->h_blk_sim.resize((size_t)P->nblk);
    P->h_blk_coord.resize((size_t)P->nblk);
    P->h_blk_rank.resize((size_t)P->nblk);
    for (int s = 0; s < nsims; ++s) {
        const SimHost& h = P->sim[s];
        for (int64_t i = 0; i < h.n; ++i) P->h_psim[(size_t)(h.p0 + i)] = s;
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
            P->h_blk_sim[(size_t)(h.blk0 + r)] = s;
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
    P->o_blk_sim = take(4 * (size_t)P->nblk);
    P->o_blk_coord = take(4 * (size_t)P->nblk);
    P->o_blk_rank = take(4 * (size_t)P->nblk);
    P->o_cell_count = take(4 * (size_t)P->ncell);
    P->o_cell_start = take(4 * ((size_t)P->ncell + 1));
    P->o_part = take(4 * ((size_t)P->nparts + 1));
    P->o_cell_of = take(4 * N);
    P->o_slot_of = take(4 * N);
    P->o_tmp = take(4 * N);
    P->o_orig[0] = take(4 * N);
    P->o_orig[1] = take(4 * N);
    P->o_SA = take(T * N * (2 * d + 1));
    P->o_SB = take(T * N * (2 * d + 1));
    P->o_jd0 = take(V4 * N);
    P->o_jd1 = take(V4 * N);
    P->o_jdA = take(V4 * N);
    P->o_jdB = take(V4 * N);
    P->o_nbr = take(4 * (size_t)P->ld * (size_t)P->maxnbr);
    P->o_cnt = take(4 * N);
    P->o_status = take(4 * (size_t)nsims);
    P->o_part64 = take(8 * ((size_t)P->nparts64 + 1) + 8 * (N + 1));
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
    if (max_neighbors) *max_neighbors = plan->maxnbr;
    return SPH_OK;
}

sph_status sph_bind(sph_plan* P, void* workspace, size_t bytes, void* stream)
{
    if (!P) return fail(SPH_ERR_INVALID_ARG, "plan is null");
    if (!workspace) return fail(SPH_ERR_INVALID_ARG, "workspace is null");
    if (bytes < P->bytes) return fail(SPH_ERR_CAPACITY, "workspace smaller than sph_workspace_size()");
    if (((uintptr_t)workspace) % 256 != 0) return fail(SPH_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    P->ws = (char*)workspace;
    HIP_TRY(hipMemcpyAsync(P->ws + P->o_simc, P->h_simc.data(), P->h_simc.size(), hipMemcpyHostToDevice, st));
    if (P->N > 0)
        HIP_TRY(hipMemcpyAsync(P->ws + P->o_psim, P->h_psim.data(), 4 * (size_t)P->N, hipMemcpyHostToDevice, st));
    if (P->nblk > 0) {
        HIP_TRY(hipMemcpyAsync(P->ws + P->o_blk_sim, P->h_blk_sim.data(), 4 * (size_t)P->nblk, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(P->ws + P->o_blk_coord, P->h_blk_coord.data(), 4 * (size_t)P->nblk, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(P->ws + P->o_blk_rank, P->h_blk_rank.data(), 4 * (size_t)P->nblk, hipMemcpyHostToDevice, st));
    }
    if (P->ncell > 0) {
        k_fill<int32_t><<<grid_for(P->ncell, 256), 256, 0, st>>>(wsp<int32_t>(P, P->o_cell_count), P->ncell, 0);
        LAUNCH_CHECK("fill");
    }
    k_fill<int32_t><<<grid_for(P->nsims, 256), 256, 0, st>>>(wsp<int32_t>(P, P->o_status), P->nsims, 0);
    LAUNCH_CHECK("fill");
    // the host tables must outlive the asynchronous copies
    HIP_TRY(hipStreamSynchronize(st));
    P->bound = true;
    return SPH_OK;
}

sph_status sph_build_cells(sph_plan* P, const sph_state* s, void* stream)
{
    sph_status rc = check_bound(P);
    if (rc == SPH_OK) rc = check_state(P, s, "state");
    if (rc != SPH_OK) return rc;
    return DISPATCH(P, do_build_cells, P, s, (hipStream_t)stream);
}

sph_status sph_neighbors(sph_plan* P, const sph_state* s, int64_t* offsets, int32_t* nbr, int64_t capacity,
                         int64_t* total, void* stream)
{
    sph_status rc = check_bound(P);
    if (rc == SPH_OK) rc = check_state(P, s, "state");
    if (rc != SPH_OK) return rc;
    if (!offsets || !total) return fail(SPH_ERR_INVALID_ARG, "offsets and total must not be null");
    if (capacity < 0 || (capacity > 0 && !nbr)) return fail(SPH_ERR_INVALID_ARG, "bad neighbour buffer");
    return DISPATCH(P, do_neighbors, P, s, offsets, nbr, capacity, total, (hipStream_t)stream);
}

sph_status sph_rhs(sph_plan* P, const sph_state* s, void* drho, void* acc, void* rho_sum, void* stream)
{
    sph_status rc = check_bound(P);
    if (rc == SPH_OK) rc = check_state(P, s, "state");
    if (rc != SPH_OK) return rc;
    if (P->N > 0 && (!drho || !acc)) return fail(SPH_ERR_INVALID_ARG, "drho and acc must not be null");
    return DISPATCH(P, do_rhs, P, s, drho, acc, rho_sum, (hipStream_t)stream);
}

sph_status sph_step(sph_plan* P, sph_state* s, int32_t nsteps, const sph_state* ckpt, int32_t ckpt_every,
                    void* stream)
{
    sph_status rc = check_bound(P);
    if (rc == SPH_OK) rc = check_state(P, s, "state");
    if (rc != SPH_OK) return rc;
    if (nsteps < 0) return fail(SPH_ERR_INVALID_ARG, "nsteps < 0");
    if (ckpt) {
        if (ckpt_every <= 0) return fail(SPH_ERR_INVALID_ARG, "ckpt_every must be > 0");
        int32_t nslots = (nsteps + ckpt_every - 1) / ckpt_every;
        for (int32_t k = 0; k < nslots; ++k) {
            rc = check_state(P, &ckpt[k], "checkpoint slot");
            if (rc != SPH_OK) return rc;
        }
    }
    return DISPATCH(P, do_step, P, s, nsteps, ckpt, ckpt_every, (hipStream_t)stream);
}

sph_status sph_step_adjoint(sph_plan* P, const sph_state* s_n, sph_state* cot, void* stream)
{
    sph_status rc = check_bound(P);
    if (rc == SPH_OK) rc = check_state(P, s_n, "state");
    if (rc == SPH_OK) rc = check_state(P, cot, "cotangent");
    if (rc != SPH_OK) return rc;
    return DISPATCH(P, do_step_adjoint, P, s_n, cot, (hipStream_t)stream);
}

sph_status sph_poll(sph_plan* P, int32_t* per_sim_status, void* stream)
{
    sph_status rc = check_bound(P);
    if (rc != SPH_OK) return rc;
    if (!per_sim_status) return fail(SPH_ERR_INVALID_ARG, "per_sim_status is null");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(per_sim_status, P->ws + P->o_status, sizeof(int32_t) * P->nsims, hipMemcpyDeviceToHost, st));
    k_fill<int32_t><<<grid_for(P->nsims, 256), 256, 0, st>>>(wsp<int32_t>(P, P->o_status), P->nsims, 0);
    LAUNCH_CHECK("fill");
    HIP_TRY(hipStreamSynchronize(st));
    return SPH_OK;
}

}  // extern "C"
