// sph_device.hpp -- gfx950 kernels of the weakly compressible delta-SPH hot path.
//
// Stages of one step (diffSPH, arXiv 2507.21684):
//   assign / scan / scatter / order  cell list by counting sort (App. B, steps 1-2)
//   build_list                       neighbour query over the cell stencil (App. B, step 3)
//   sweep                            Wendland-C4 kernel and gradient (App. A.1), summation
//                                    density, continuity + delta diffusion, Tait pressure and
//                                    artificial viscosity (Sec. 2.3), semi-implicit Euler (Sec. 3.4)
//   adj_prologue / adj_sweep         the vector-Jacobian product of one step (Sec. 2.2) with
//                                    the kernel Hessian (Sec. 3.3)
//
// Every pair sum is a gather: a particle adds its neighbours' terms in the order of its
// neighbour list, which is canonical (stencil cells by relative offset, then particles by
// original index), so results are deterministic and independent of tiling and batching.
// No floating-point atomics are used anywhere.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sph {

constexpr int kFlagNonfinite = 1;
constexpr int kFlagOverflow = 2;
constexpr int kFlagSkin = 4;  // a particle moved more than its half skin since its list was built

// Half skins of reused lists: particle i may move h_i between two list builds, and a pair is
// listed when r < H + h_i + h_j.  Uniform skins take h_i = hmax (half the simulation's skin);
// speed-scaled skins take h_i = min(hmax, kSkinFloor hmax + kSkinMargin R dt |v_i|) from the
// particle's speed when the lists are built (R the rebuild interval).  A pair that comes
// within H before the next build is therefore listed as long as neither particle has moved more
// than its own h_i, which every step checks (kFlagSkin).  The additive floor is every particle's
// allowance for acceleration over the interval: with hmax sized for 1.3 times the largest speed,
// a particle at rest may accelerate steadily to about a third of that speed; the margin covers
// 30 % more than its own speed.
constexpr double kSkinMargin = 1.3;
constexpr double kSkinFloor = 0.125;

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };
template <typename T> using vec4_t = typename Vec4<T>::type;

// Per-simulation constants.  Every floating-point field is rounded once, on the host,
// in the working precision T (H2 = H*H, invL = 1/L computed in T).
template <typename T>
struct SimConst {
    T L, invL, H, H2, invH, cinv;
    T m, rho0, inv_rho0, c0sq, dt;
    T kW;       // C_d / H^d
    T kG;       // C_d / H^(d+2)
    T kH;       // 560 C_d / H^(d+4): second coefficient of the kernel Hessian
    T epsH2;    // eps H^2
    T cA;       // alpha H c0 rho0
    T cD;       // 2 delta H c0
    T Bt;       // rho0 c0^2 / 7
    T HL2;      // (H (1 + skin))^2: list radius squared (= H2 without a skin)
    T hmax;     // skin H / 2: the largest half skin of a particle (the cells are sized for it)
    T invW0;    // 1 / W(dx), dx = (m / rho0)^(1/dim) the initial spacing (particle shifting)
    int64_t p0, n;      // packed particle range
    int32_t cell0;      // first global cell slot
    int32_t blk0;       // first global cell block
    int32_t nc;         // cells per box side
    int32_t sub;        // stencil half-width in cells (cell side >= H / sub)
    int32_t B;          // cells per block side
    int32_t nb;         // blocks per box side
    int32_t Bd;         // B^dim
    int32_t ncu;        // stencil cells per cell, (2 sub + 1)^dim
};

// Stencil entry: global cell id in the low 26 bits, periodic image shift (-1, 0, +1 box
// lengths, stored + 1) in two bits per axis above it.
constexpr int kStencilIdBits = 26;
constexpr int32_t kStencilIdMask = (1 << kStencilIdBits) - 1;

// Stencil cell u (u = 0 .. (2 sub + 1)^dim - 1, offsets in lexicographic order z, y, x) of the
// cell at coordinates cc of simulation S, as a stencil entry.  Cells are numbered block-major:
// blocks of B^dim cells in Morton order (blk_rank maps a row-major block index to its rank),
// cells row-major inside a block.
// Cells per block side: 4 in 2D, 2 in 3D (the host sets SimConst::B to the same values).
template <int DIM>
constexpr int kBlockSide = DIM == 3 ? 2 : 4;

// Offsets (x, y, z) of stencil cell u for a stencil of SW cells per side (SW = 2 sub + 1 = 3 or
// 5, a constant here so that the divisions are multiplications).
template <int DIM, int SW>
__device__ __forceinline__ void stencil_offsets(int u, int sub, int* o)
{
    const unsigned v = (unsigned)u;
    o[0] = (int)(v % SW) - sub;
    o[1] = (int)((v / SW) % SW) - sub;
    o[2] = (DIM == 3) ? (int)(v / (SW * SW)) - sub : 0;
}

template <int DIM, typename T, int EXT = 0>
__device__ __forceinline__ int32_t stencil_entry(const SimConst<T>& S, const int32_t* __restrict__ blk_rank,
                                                 const int* cc, int u)
{
    // EXT = 1: the (SW + 1)^DIM union stencil of a group of 2^DIM cells whose lowest cell is cc
    int o[3];
    if (S.sub == 2) stencil_offsets<DIM, 5 + EXT>(u, 2, o);
    else stencil_offsets<DIM, 3 + EXT>(u, 1, o);
    int c[3] = {0, 0, 0}, sh[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        int r = cc[k] + o[k];
        if (r < 0) {
            r += S.nc;
            sh[k] = -1;
        } else if (r >= S.nc) {
            r -= S.nc;
            sh[k] = 1;
        }
        c[k] = r;
    }
    constexpr unsigned B = kBlockSide<DIM>;
    const int bx = (int)((unsigned)c[0] / B), by = (int)((unsigned)c[1] / B), bz = (DIM == 3) ? (int)((unsigned)c[2] / B) : 0;
    const int lin = (DIM == 3) ? (bz * S.nb + by) * S.nb + bx : by * S.nb + bx;
    const int rk = blk_rank[S.blk0 + lin];
    const int wl = (DIM == 3) ? ((c[2] - bz * B) * B + (c[1] - by * B)) * B + (c[0] - bx * B)
                              : (c[1] - by * B) * B + (c[0] - bx * B);
    const int id = S.cell0 + rk * (DIM == 3 ? B * B * B : B * B) + wl;
    return id | ((sh[0] + 1) << kStencilIdBits) | ((sh[1] + 1) << (kStencilIdBits + 2)) |
           ((sh[2] + 1) << (kStencilIdBits + 4));
}

// Simulation index of every particle and every cell slot: the last simulation whose first
// particle (cell slot) is at or before it.  Empty simulations share their first index with the
// next one, so the last such simulation is the one that owns the index.
template <typename T>
__global__ void k_sim_index(int64_t N, int64_t ncell, int32_t nsims, const SimConst<T>* __restrict__ sims,
                            int32_t* __restrict__ psim, int32_t* __restrict__ cell_sim)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < N) {
        int lo = 0, hi = nsims - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sims[mid].p0 <= t) lo = mid;
            else hi = mid - 1;
        }
        psim[t] = lo;
    }
    if (t < ncell) {
        int lo = 0, hi = nsims - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sims[mid].cell0 <= t) lo = mid;
            else hi = mid - 1;
        }
        cell_sim[t] = lo;
    }
}

template <typename T, int DIM>
struct StatePtrs {
    T* x[3];
    T* v[3];
    T* rho;
};

// ---------------------------------------------------------------- helpers

// Workgroup index remapped so that each XCD (workgroups are dispatched round-robin over
// the 8 XCDs) receives one contiguous range of the logical index space: neighbouring
// tiles then share an L2.
__device__ __forceinline__ int xcd_remap(int wg, int nwg)
{
    const int nx = 8;
    int x = wg % nx, y = wg / nx;
    int q = nwg / nx, r = nwg % nx;
    return x * q + (x < r ? x : r) + y;
}

template <typename T>
__device__ __forceinline__ T wrap_pos(T x, T L, T invL)
{
#pragma clang fp contract(off)
    T k = floor(x * invL);
    T s = L * k;
    return x - s;
}

template <typename T>
__device__ __forceinline__ int cell_coord(T u, T cinv, int nc)
{
    T f = floor(u * cinv);
    int c = (int)f;
    c = c < 0 ? 0 : c;
    c = c > nc - 1 ? nc - 1 : c;
    return c;
}

template <typename T, int DIM>
__device__ __forceinline__ int global_cell(const SimConst<T>& S, const int32_t* __restrict__ blk_rank, int cx, int cy,
                                           int cz)
{
    constexpr int B = kBlockSide<DIM>;
    int bx = (int)((unsigned)cx / B), by = (int)((unsigned)cy / B), bz = (DIM == 3) ? (int)((unsigned)cz / B) : 0;
    int wx = cx - bx * B, wy = cy - by * B, wz = (DIM == 3) ? cz - bz * B : 0;
    int lin = (DIM == 3) ? ((bz * S.nb + by) * S.nb + bx) : (by * S.nb + bx);
    int rank = blk_rank[S.blk0 + lin];
    int w = (DIM == 3) ? ((wz * B + wy) * B + wx) : (wy * B + wx);
    return S.cell0 + rank * (DIM == 3 ? B * B * B : B * B) + w;
}

// r^2 of the minimum-image pair vector, every operation rounded in T (no contraction):
//   d = u_i - u_j; d = d - shift; r2 = ((d0 d0) + d1 d1) + d2 d2
// The shift (0 or +-L per axis) is the periodic image of the stencil cell the candidate
// was found in; for any pair within the support it equals L rint((u_i - u_j) / L).
template <typename T, int DIM>
__device__ __forceinline__ T dist2_exact(const T* ui, const T* uj, const T* sh)
{
#pragma clang fp contract(off)
    T r2 = T(0);
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        T d = ui[k] - uj[k];
        d = d - sh[k];
        T dd = d * d;
        r2 = r2 + dd;
    }
    return r2;
}

// FP32 sweeps use the hardware reciprocal and square root (about 1 ulp); FP64 keeps IEEE
// division and square root.
template <typename T> __device__ __forceinline__ T fast_rcp(T x) { return T(1) / x; }
template <> __device__ __forceinline__ float fast_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <typename T> __device__ __forceinline__ T fast_sqrt(T x) { return sqrt(x); }
template <> __device__ __forceinline__ float fast_sqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }

// Volume of a particle from its position record.  The 2D record (u, V, p V) holds it; the 3D
// record (u, rho) holds the density, and V = m / rho is recomputed with the arithmetic of the
// kernel that wrote the record, so it is the value that kernel had.
template <typename T, int DIM>
__device__ __forceinline__ T rec_volume(const vec4_t<T>& a, T m)
{
    return DIM == 3 ? m * fast_rcp(a.w) : a.z;
}

template <typename T>
__device__ __forceinline__ T tait(const SimConst<T>& S, T rho)
{
    T s = rho * S.inv_rho0;
    T s2 = s * s;
    T s3 = s2 * s;
    T s6 = s3 * s3;
    return S.Bt * (s6 * s - T(1));
}

template <typename T>
__device__ __forceinline__ T tait_slope(const SimConst<T>& S, T rho)
{
    T s = rho * S.inv_rho0;
    T s2 = s * s;
    T s3 = s2 * s;
    return S.c0sq * (s3 * s3);
}

template <typename I>
__device__ __forceinline__ I wave_incl_scan(I v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        I t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// ---------------------------------------------------------------- fill

template <typename I>
__global__ void k_fill(I* __restrict__ p, int64_t n, I val)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = val;
}

// ---------------------------------------------------------------- cell assignment

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_assign(int64_t N, StatePtrs<T, DIM> st, const int32_t* __restrict__ psim,
                                                const SimConst<T>* __restrict__ sims,
                                                const int32_t* __restrict__ blk_rank, int32_t* __restrict__ cell_count,
                                                int32_t* __restrict__ cell_of, int32_t* __restrict__ slot_of,
                                                int32_t* __restrict__ status)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int s = psim[p];
    const SimConst<T>& S = sims[s];
    int c[3] = {0, 0, 0};
    bool bad = false;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        T x = st.x[k][p];
        if (!isfinite(x)) {
            bad = true;
            x = T(0);
        }
        T u = wrap_pos(x, S.L, S.invL);
        c[k] = cell_coord(u, S.cinv, S.nc);
    }
    if (bad) atomicOr(&status[s], kFlagNonfinite);
    int gc = global_cell<T, DIM>(S, blk_rank, c[0], c[1], c[2]);
    cell_of[p] = gc;
    slot_of[p] = atomicAdd(&cell_count[gc], 1);
}

// ---------------------------------------------------------------- exclusive scan (3 phases)

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename I>
__device__ __forceinline__ I block_excl_scan(I v, I* smem /* >= 5 */, I* total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    I inc = wave_incl_scan(v);
    if (lane == 63) smem[wid] = inc;
    __syncthreads();
    I off = 0, tot = 0;
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) {
        I t = smem[w];
        if (w < wid) off += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// Tile sums, and the workgroup that finishes last (atomic ticket; no waiting on other
// workgroups) turns them into exclusive tile offsets, part[np] = grand total, and resets the
// ticket for the next scan.
template <typename I>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce_last(const I* __restrict__ in, int64_t n,
                                                                   I* __restrict__ part,
                                                                   unsigned int* __restrict__ ticket)
{
    __shared__ I smem[8];
    __shared__ I carry;
    __shared__ int is_last;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    I sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) sum += in[base + k];
    I tot;
    block_excl_scan<I>(sum, smem, &tot);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = tot;
        __threadfence();
        const unsigned int done = atomicAdd(ticket, 1u);
        is_last = (done == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    const int64_t np = gridDim.x;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b = 0; b < np; b += blockDim.x) {
        const int64_t i = b + threadIdx.x;
        const I v = (i < np) ? __atomic_load_n(&part[i], __ATOMIC_RELAXED) : I(0);
        I t2;
        const I ex = block_excl_scan<I>(v, smem, &t2);
        const I c0 = carry;
        if (i < np) part[i] = c0 + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry = c0 + t2;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[np] = carry;
        *ticket = 0u;
    }
}

// out[i] = exclusive prefix of in; out[n] = total; optionally zero `in` afterwards
template <typename I>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(I* __restrict__ in, int64_t n, const I* __restrict__ part,
                                                             int64_t np, I* __restrict__ out, int zero_in)
{
    __shared__ I smem[8];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    I v[kScanItems];
    I s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : I(0);
        s += v[k];
    }
    I tot;
    I ex = block_excl_scan<I>(s, smem, &tot) + part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) {
            out[base + k] = ex;
            if (zero_in) in[base + k] = 0;
        }
        ex += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = part[np];
}

// ---------------------------------------------------------------- scatter and within-cell order

__global__ __launch_bounds__(256) void k_scatter(int64_t N, const int32_t* __restrict__ cell_of,
                                                 const int32_t* __restrict__ slot_of,
                                                 const int32_t* __restrict__ cell_start, int32_t* __restrict__ tmp)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    tmp[cell_start[cell_of[p]] + slot_of[p]] = (int32_t)p;
}

// Final sorted position = cell start + rank of the particle's original index among its cell's
// members; gathers the state into that position and packs the per-particle data that the
// neighbour sweeps read (wrapped position, volume V = m / rho, p V, velocity).
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_order_gather(int64_t N, const int32_t* __restrict__ tmp,
                                                      const int32_t* __restrict__ cell_of,
                                                      const int32_t* __restrict__ cell_start,
                                                      const int32_t* __restrict__ orig_in, StatePtrs<T, DIM> src,
                                                      StatePtrs<T, DIM> dst, int32_t* __restrict__ orig_out,
                                                      vec4_t<T>* __restrict__ jd0, vec4_t<T>* __restrict__ jd1,
                                                      const int32_t* __restrict__ psim,
                                                      const SimConst<T>* __restrict__ sims,
                                                      vec4_t<T>* __restrict__ uref, T skin_floor,
                                                      T skin_steps)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const int p = tmp[q];
    const int c = cell_of[p];
    const int s0 = cell_start[c], s1 = cell_start[c + 1];
    const int op = orig_in ? orig_in[p] : p;
    int rank = 0;
    for (int r = s0; r < s1; ++r) {
        int pr = tmp[r];
        int o = orig_in ? orig_in[pr] : pr;
        rank += (o < op) ? 1 : 0;
    }
    const int d = s0 + rank;
    const SimConst<T>& S = sims[psim[d]];
    T x[3] = {0, 0, 0}, v[3] = {0, 0, 0}, u[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        x[k] = src.x[k][p];
        v[k] = src.v[k][p];
        dst.x[k][d] = x[k];
        dst.v[k][d] = v[k];
        u[k] = wrap_pos(isfinite(x[k]) ? x[k] : T(0), S.L, S.invL);
    }
    const T rho = src.rho[p];
    dst.rho[d] = rho;
    orig_out[d] = op;
    const T V = S.m * fast_rcp(rho);
    const T pr = tait(S, rho);
    const T pV = pr * V;
    vec4_t<T> a, b;
    if (DIM == 3) {
        a.x = u[0]; a.y = u[1]; a.z = u[2]; a.w = rho;
        b.x = v[0]; b.y = v[1]; b.z = v[2]; b.w = pr;
    } else {
        a.x = u[0]; a.y = u[1]; a.z = V; a.w = pV;
        b.x = v[0]; b.y = v[1]; b.z = rho; b.w = pr;
    }
    jd0[d] = a;
    jd1[d] = b;
    if (uref) {
        // the positions the lists are built from and the particle's half skin (list reuse):
        // speed-scaled with skin_floor = kSkinFloor, skin_steps = kSkinMargin R, uniform (hmax)
        // with skin_floor = 1, skin_steps = 0
        T v2 = T(0);
#pragma unroll
        for (int k = 0; k < DIM; ++k) v2 += v[k] * v[k];
        const T hv = skin_floor * S.hmax + skin_steps * S.dt * sqrt(v2);
        const T h = hv < S.hmax ? hv : S.hmax;   // a non-finite speed keeps hmax
        vec4_t<T> r;
        r.x = u[0]; r.y = u[1]; r.z = u[2]; r.w = h;
        uref[d] = r;
    }
}

// A state in original order gathered into the particle order of a slot that is already sorted
// and has lists (a later stage of a multistage step, with the lists of the step's first stage):
// the sorted state and the packed records as k_order_gather writes them, and the displacement
// since the lists were built checked against its half skin.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_repack(int64_t N, const int32_t* __restrict__ orig, StatePtrs<T, DIM> src,
                                                StatePtrs<T, DIM> dst, vec4_t<T>* __restrict__ jd0,
                                                vec4_t<T>* __restrict__ jd1, const vec4_t<T>* __restrict__ uref,
                                                const int32_t* __restrict__ psim,
                                                const SimConst<T>* __restrict__ sims, int32_t* __restrict__ status)
{
    int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= N) return;
    const int s = psim[d];
    const SimConst<T>& S = sims[s];
    const int p = orig[d];
    T x[3] = {0, 0, 0}, v[3] = {0, 0, 0}, u[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        x[k] = src.x[k][p];
        v[k] = src.v[k][p];
        dst.x[k][d] = x[k];
        dst.v[k][d] = v[k];
        u[k] = wrap_pos(isfinite(x[k]) ? x[k] : T(0), S.L, S.invL);
    }
    const T rho = src.rho[p];
    dst.rho[d] = rho;
    const T V = S.m * fast_rcp(rho);
    const T pr = tait(S, rho);
    const T pV = pr * V;
    vec4_t<T> a, b;
    if (DIM == 3) {
        a.x = u[0]; a.y = u[1]; a.z = u[2]; a.w = rho;
        b.x = v[0]; b.y = v[1]; b.z = v[2]; b.w = pr;
    } else {
        a.x = u[0]; a.y = u[1]; a.z = V; a.w = pV;
        b.x = v[0]; b.y = v[1]; b.z = rho; b.w = pr;
    }
    jd0[d] = a;
    jd1[d] = b;
    const vec4_t<T> ref = uref[d];
    const T rr[3] = {ref.x, ref.y, ref.z};
    T d2 = T(0);
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        T dk = u[k] - rr[k];
        dk -= S.L * rint(dk * S.invL);
        d2 += dk * dk;
    }
    if (!(d2 <= ref.w * ref.w)) atomicOr(&status[s], kFlagSkin);
}

template <typename T, int DIM>
__device__ __forceinline__ void unpack_u(const vec4_t<T>& a, T* u)
{
    u[0] = a.x;
    u[1] = a.y;
    if (DIM == 3) u[2] = a.z;
}

// ---------------------------------------------------------------- neighbour lists

// The pair counter is spread over kPairSlots words, one per 128-byte line, so that the
// wavefronts' integer atomics do not serialise on a single address.
constexpr int kPairSlots = 512;
constexpr int kPairStride = 16;
// Status read without a host wait: the pair total and the status words moved to a staging
// area and cleared, for one copy to the host in stream order.  One workgroup of 256 lanes.
__global__ __launch_bounds__(256) void k_poll_stage(int32_t nsims, int32_t* __restrict__ status,
                                                    unsigned long long* __restrict__ pair_slots,
                                                    unsigned long long* __restrict__ stage_pairs,
                                                    int32_t* __restrict__ stage_status)
{
    __shared__ unsigned long long part[256];
    unsigned long long sum = 0;
    for (int k = threadIdx.x; k < kPairSlots; k += blockDim.x) {
        sum += pair_slots[k * kPairStride];
        pair_slots[k * kPairStride] = 0ull;
    }
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *stage_pairs = part[0];
    for (int k = threadIdx.x; k < nsims; k += blockDim.x) {
        stage_status[k] = status[k];
        status[k] = 0;
    }
}

// Candidates (of the stencil of one cell) whose stencil cell is looked up in a byte table;
// later ones, in dense clusters only, search the prefix sums.
constexpr int kCandTable = 2048;

// One wavefront per cell.  The candidates of the cell's particles are the particles of the
// (2 sub + 1)^dim stencil cells, taken in lexicographic order of the cell offset (the
// precomputed stencil table lists them in that order), each cell's particles in sorted order
// (= original index inside a cell), which is the canonical list order.  The candidate stream
// is cut into chunks of 64; lane l holds candidate 64 c + l of chunk c in registers (the next
// chunk's gather is issued before the current chunk is tested; a candidate's stencil cell comes
// from a byte table in LDS, or a search of the prefix sums past it), and the cell's particles,
// staged in LDS, are taken one after the other with the same address in every lane.  For
// particle p one round tests all 64 candidates of the chunk; the ballot of the accepted ones
// gives each its rank, so the round appends a contiguous run to p's row, in candidate order.
// Lane p keeps p's running count.  Lists are row-major: entry k of particle i is
// nbr[i * width + k].
// With GROUP (2D) a wavefront serves a group of 2 x 2 cells (cell slots c, c + 1, c + B,
// c + B + 1 of a block, B = 4) over their 6 x 6 (or 4 x 4) union stencil, in the same lexicographic order:
// a particle's own stencil cells are a sub-grid of it in the same relative order, and the extra
// row and column of the union lie at least two cell sides, i.e. at least the list radius, away
// from it, so the strict distance test rejects them (also where a small box repeats a cell in
// the union under another periodic image).  Each particle's list is therefore the one of its own
// cell, while the stencil setup and the candidate stream are shared by four cells.
template <typename T, int DIM, bool PERPAIR, bool GROUP>
__global__ __launch_bounds__(64) void k_build_list(const int32_t* __restrict__ cell_sim,
                                                   const int32_t* __restrict__ blk_coord,
                                                   const int32_t* __restrict__ blk_rank,
                                                   const SimConst<T>* __restrict__ sims,
                                                   const int32_t* __restrict__ cell_start,
                                                   const vec4_t<T>* __restrict__ jd0, int32_t width,
                                                   int32_t* __restrict__ nbr, int32_t* __restrict__ nbr_count,
                                                   int32_t* __restrict__ status,
                                                   unsigned long long* __restrict__ pair_counter, int exact,
                                                   const vec4_t<T>* __restrict__ href)
{
    // PERPAIR: lists with per-particle half skins; positions and half skins come from href
    // (written by the sort), and the list radius of a pair is H + h_i + h_j
    const vec4_t<T>* __restrict__ rec = PERPAIR ? href : jd0;
    __shared__ vec4_t<T> pu[64];
    __shared__ int32_t uc_first[128];
    __shared__ int32_t uc_pref[129];
    __shared__ int32_t uc_code[128];
    __shared__ uint8_t uc_of[kCandTable];  // stencil cell of each of the first kCandTable candidates

    constexpr bool kGroup = GROUP && DIM == 2;
    constexpr int kExt = kGroup ? 1 : 0;
    const int gw = xcd_remap(blockIdx.x, gridDim.x);
    // lowest cell slot of the wavefront's cells (2D: group gw & 3 of block gw >> 2)
    const int gc = kGroup ? (gw >> 2) * 16 + ((gw >> 1) & 1) * 8 + (gw & 1) * 2 : gw;
    const int lane = threadIdx.x;
    const int s = cell_sim[gc];
    // particles: the range of cells gc (and gc + 1), then in 2D that of cells gc + 4, gc + 5
    const int i0 = cell_start[gc];
    const int n0 = cell_start[gc + (kGroup ? 2 : 1)] - i0;
    const int i1 = kGroup ? cell_start[gc + 4] : 0;
    const int n = n0 + (kGroup ? cell_start[gc + 6] - i1 : 0);
    if (n == 0) return;
    const SimConst<T> S = sims[s];
    const int sw1 = 2 * S.sub + 1 + kExt;
    const int ncu = kGroup ? sw1 * sw1 : S.ncu;
    const T R2 = exact ? S.H2 : S.HL2;  // list radius: the support, or the support plus the skin
    // the cell's coordinates from its block and its place inside the block
    int cc[3];
    {
        constexpr unsigned B = kBlockSide<DIM>, Bd = DIM == 3 ? B * B * B : B * B;
        const unsigned local = (unsigned)(gc - S.cell0);
        const int rank = (int)(local / Bd);
        const unsigned w = local % Bd;
        const int coord = blk_coord[S.blk0 + rank];
        cc[0] = (coord & 1023) * (int)B + (int)(w % B);
        cc[1] = ((coord >> 10) & 1023) * (int)B + (int)((w / B) % B);
        cc[2] = (DIM == 3) ? ((coord >> 20) & 1023) * (int)B + (int)(w / (B * B)) : 0;
    }

    // stencil cells: particle range and periodic image code, two per lane at most
    int carry = 0;
    const int halves = ncu > 64 ? 2 : 1;
    for (int half = 0; half < halves; ++half) {
        const int u = lane + 64 * half;
        int first = 0, count = 0, code = 0;
        if (u < ncu) {
            code = stencil_entry<DIM, T, kExt>(S, blk_rank, cc, u);
            const int id = code & kStencilIdMask;
            first = cell_start[id];
            count = cell_start[id + 1] - first;
        }
        const int inc = wave_incl_scan(count);
        const int beg = carry + inc - count;
        if (u < 128) {
            uc_first[u] = first;
            uc_pref[u] = beg;
            uc_code[u] = code;
        }
        const int end = (beg + count < kCandTable) ? beg + count : kCandTable;
        for (int m = beg; m < end; ++m) uc_of[m] = uint8_t(u);
        carry += __shfl(inc, 63, 64);
    }
    const int M = carry;
    if (lane == 0) uc_pref[ncu] = M;
    __syncthreads();

    // candidate m of the stream: sorted index, position and periodic shift
    auto fetch = [&](int m, int& j, vec4_t<T>& u, int& code) {
        int lo;  // the stencil cell holding candidate m: the last one whose prefix is <= m
        if (m < kCandTable) {
            lo = uc_of[m];
        } else {
            lo = 0;
            int hi = ncu - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (uc_pref[mid] <= m) lo = mid;
                else hi = mid - 1;
            }
        }
        j = uc_first[lo] + (m - uc_pref[lo]);
        code = uc_code[lo];
        u = rec[j];
    };

    // sorted index of the wavefront's particle q (the two ranges in order)
    auto pidx = [&](int q) { return q < n0 ? i0 + q : i1 + (q - n0); };
    int pairs_acc = 0;
    for (int pb = 0; pb < n; pb += 64) {
        const int nb = __builtin_amdgcn_readfirstlane((n - pb < 64) ? n - pb : 64);
        // batch positions [0, split) are in the first range, [split, nb) in the second
        const int split = __builtin_amdgcn_readfirstlane(n0 - pb < 0 ? 0 : (n0 - pb < nb ? n0 - pb : nb));
        __syncthreads();
        if (lane < nb) pu[lane] = rec[pidx(pb + lane)];
        __syncthreads();
        int cnt = 0;  // lane p: entries of the batch's particle p so far
        int jn = 0, coden = 0;
        vec4_t<T> un;
        un.x = un.y = un.z = un.w = T(0);
        if (lane < M) fetch(lane, jn, un, coden);
        for (int c0 = 0; c0 < M; c0 += 64) {
            const bool valid = c0 + lane < M;
            const int jc = jn;
            T uj[3] = {T(0), T(0), T(0)}, sh[3];
            unpack_u<T, DIM>(un, uj);
            sh[0] = T(((coden >> kStencilIdBits) & 3) - 1) * S.L;
            sh[1] = T(((coden >> (kStencilIdBits + 2)) & 3) - 1) * S.L;
            sh[2] = T(((coden >> (kStencilIdBits + 4)) & 3) - 1) * S.L;
            const T Aj = S.H + un.w;   // PERPAIR: H + h_j
            // PERPAIR lists only need to hold a superset of the pairs within H (the sweeps test
            // those exactly), so their distance takes the candidate's image once per chunk and
            // contracted products; exact lists keep the predicate's own arithmetic
            T ujs[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) ujs[k] = uj[k] + sh[k];
            if (c0 + 64 + lane < M) fetch(c0 + 64 + lane, jn, un, coden);  // next chunk in flight
            const unsigned long long vmask = __ballot(valid);
            // the rounds of batch positions [p0, p1), whose rows follow each other from row
            auto rounds = [&](int p0, int p1, int32_t* row) {
            for (int p = p0; p < p1; ++p, row += width) {
                T ui[3] = {T(0), T(0), T(0)};
                const vec4_t<T> rp = pu[p];
                unpack_u<T, DIM>(rp, ui);
                bool inr;
                if (PERPAIR) {
                    const T Rp = Aj + rp.w;
                    const T d0 = ui[0] - ujs[0];
                    T r2 = d0 * d0;
#pragma unroll
                    for (int k = 1; k < DIM; ++k) {
                        const T d = ui[k] - ujs[k];
                        r2 = fma(d, d, r2);
                    }
                    inr = r2 < Rp * Rp;
                } else {
                    inr = dist2_exact<T, DIM>(ui, uj, sh) < R2;
                }
                const unsigned long long mask = __ballot(inr) & vmask;
                const bool ok = valid & inr;
                const int base = __builtin_amdgcn_readlane(cnt, p);
                const int total = base + __popcll(mask);
                // base plus the accepted lanes below this one
                const unsigned pos = __builtin_amdgcn_mbcnt_hi(
                    unsigned(mask >> 32), __builtin_amdgcn_mbcnt_lo(unsigned(mask), unsigned(base)));
                if (total <= width) {           // wave-uniform: the whole run fits the row
                    if (ok) row[pos] = jc;
                } else if (ok && pos < unsigned(width)) {
                    row[pos] = jc;
                }
                cnt = (lane == p) ? total : cnt;  // lane p keeps p's count
            }
            };
            rounds(0, split, nbr + (int64_t)(i0 + pb) * width);
            if (kGroup) rounds(split, nb, nbr + (int64_t)pidx(pb + split) * width);
        }
        if (lane < nb) {
            const int i = pidx(pb + lane);
            nbr_count[i] = cnt;
            if (cnt > width) atomicOr(&status[s], kFlagOverflow);
            pairs_acc += cnt - 1;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) pairs_acc += __shfl_xor(pairs_acc, o, 64);
    if (lane == 0 && pair_counter)
        atomicAdd(&pair_counter[(gc & (kPairSlots - 1)) * kPairStride], (unsigned long long)pairs_acc);
}

// ---------------------------------------------------------------- canonical pair sums
//
// A particle's neighbour sum is split into eight partial sums s_q over list positions
// k = q (mod 8), each accumulated in increasing k, and combined by the balanced tree
// ((s0 + s1) + (s2 + s3)) + ((s4 + s5) + (s6 + s7)).  LPP lanes share a particle
// (LPP in {2, 4, 8}): lane r holds the 8 / LPP partial sums with q = r (mod LPP).  The
// first log2(LPP) levels of the tree combine lanes (xor shuffles; every lane of the group ends
// with the same value because floating-point addition commutes), the remaining levels combine
// a lane's own partial sums.  The result is bitwise the same for every LPP.
constexpr int kLeaves = 8;

template <int LPP, typename T>
__device__ __forceinline__ T combine_leaves(T* a /* [kLeaves / LPP] */)
{
    constexpr int NQ = kLeaves / LPP;
#pragma unroll
    for (int o = 1; o < LPP; o <<= 1) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) a[q] = a[q] + __shfl_xor(a[q], o, 64);
    }
    if (NQ == 1) return a[0];
    if (NQ == 2) return a[0] + a[1];
    return (a[0] + a[1]) + (a[2] + a[3]);
}

// ---------------------------------------------------------------- gathers and fast arithmetic

// Element `idx` of an array whose byte size fits 32 bits: a 32-bit byte offset from the
// array base, so the load uses a scalar base plus a vector offset.
template <typename V>
__device__ __forceinline__ V ldo(const V* __restrict__ base, uint32_t idx)
{
    return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + idx * (uint32_t)sizeof(V));
}

// List entries of lane r at its positions m0 .. m0 + U - 1 (position k = r + LPP m of the row);
// positions past the lane's count read as the particle itself, a valid index whose pair is
// skipped.  The sweeps load the next group's entries before computing the current one, so
// that only the record gathers stand between consecutive groups.
template <int LPP, int U>
__device__ __forceinline__ void load_entries(const int32_t* __restrict__ row, int r, int m0, int mcount, int self,
                                             int* jj)
{
#pragma unroll
    for (int u = 0; u < U; ++u) jj[u] = (m0 + u < mcount) ? row[r + LPP * (m0 + u)] : self;
}

// The same entries with every load issued unconditionally: the position is clamped to the row
// (width entries), so the load needs no branch, and past the lane's count the entry read is
// replaced by the particle itself.
template <int LPP, int U>
__device__ __forceinline__ void load_entries_clamped(const int32_t* __restrict__ row, int width, int r, int m0,
                                                     int mcount, int self, int* jj)
{
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int pos = r + LPP * (m0 + u);
        const int e = row[pos < width ? pos : width - 1];
        jj[u] = (m0 + u < mcount) ? e : self;
    }
}



// Four lanes per particle (adjoint sweep): each group of 16 list positions (16 g .. 16 g + 15,
// four per lane) is read as four 16-byte chunks, lane r reading positions 16 g + 4 r .. + 3, and
// a 4 x 4 transpose inside the lane quad gives lane r its positions r + 4 c (c = 0..3), the ones
// the canonical assignment gives it: one load instead of four.
// The chunk start is clamped to the row (width is a multiple of 8), so a chunk past the row end
// rereads its last chunk, whose positions the caller discards.  A lane leaves the loop after its
// own last position; the values it would pass to the lanes still looping are positions at or
// past the row's count (lane c stops once 4 c + 16 g >= count), which those lanes discard too.
__device__ __forceinline__ int4 load_chunk4(const int32_t* __restrict__ row, int width, int pos)
{
    pos = pos < width - 4 ? pos : width - 4;
    return *reinterpret_cast<const int4*>(row + pos);
}

template <int CTRL>
__device__ __forceinline__ int quad_perm(int v)
{
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}

__device__ __forceinline__ void quad_transpose(int r, const int4& m, int* out)
{
    const bool hi = (r & 2) != 0, odd = (r & 1) != 0;
    // exchange 2 x 2 blocks with lane r ^ 2 (quad permutation 2, 3, 0, 1)
    const int y0 = quad_perm<0x4E>(hi ? m.x : m.z);
    const int y1 = quad_perm<0x4E>(hi ? m.y : m.w);
    const int n0 = hi ? y0 : m.x, n1 = hi ? y1 : m.y, n2 = hi ? m.z : y0, n3 = hi ? m.w : y1;
    // exchange single elements with lane r ^ 1 (quad permutation 1, 0, 3, 2)
    const int z0 = quad_perm<0xB1>(odd ? n0 : n1);
    const int z1 = quad_perm<0xB1>(odd ? n2 : n3);
    out[0] = odd ? z0 : n0;
    out[1] = odd ? n1 : z0;
    out[2] = odd ? z1 : n2;
    out[3] = odd ? n3 : z1;
}

// Per-simulation constants the pair loops use, held in registers.
template <typename T>
struct PairConst {
    T L, invL, invH, kG, kH, epsH2, cA, cD, H2;
    T kGF;  // kG (-56/3): grad W = kGF t^5 (1 + 5 q) x_ij
    T m;    // particle mass
};

// Squared distance of a listed pair with the arithmetic of the neighbour predicate (per
// component the minimum image, then the sum of squares in component order, no contraction),
// so that a list with a skin can be filtered to exactly the pairs with r^2 < H^2.
// The minimum-image pair vector is returned in d.
template <typename T, int DIM>
__device__ __forceinline__ T r2_exact(const T* ui, const vec4_t<T>& a, T L, T invL, T* d)
{
#pragma clang fp contract(off)
    const T uj[3] = {a.x, a.y, a.z};
    T r2 = T(0);
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        T dk = ui[k] - uj[k];
        // L rint(.) is 0 or +-L exactly, so the fused form rounds once, as the separate
        // product and difference do
        dk = fma(-L, rint(dk * invL), dk);
        d[k] = dk;
        T dd = dk * dk;
        r2 = r2 + dd;
    }
    return r2;
}

// What the sweep that finishes a step does for the next step when that step reuses the lists
// (null jd0: the next step sorts and rebuilds): the next state goes straight into the next
// tape slot in the same particle order, with its packed records and original indices, and each
// particle's displacement since the list build is checked against its half skin.
template <typename T>
struct NextSlot {
    vec4_t<T>* jd0;
    vec4_t<T>* jd1;
    int32_t* orig;
    const vec4_t<T>* uref;
};

template <typename T>
__device__ __forceinline__ PairConst<T> pair_const(const SimConst<T>& S)
{
    PairConst<T> c;
    c.L = S.L;
    c.invL = S.invL;
    c.invH = S.invH;
    c.kG = S.kG;
    c.kH = S.kH;
    c.epsH2 = S.epsH2;
    c.cA = S.cA;
    c.cD = S.cD;
    c.H2 = S.H2;
    c.kGF = S.kG * T(-56.0 / 3.0);
    c.m = S.m;
    return c;
}

// ---------------------------------------------------------------- forward sweep

constexpr int kModeStep = 0;  // integrate into dst (sorted order)
constexpr int kModeRhs = 1;   // write drho, a, rho_sum to caller arrays (original order)
constexpr int kPairsInFlight = 4;  // list positions each lane loads before computing them

// ---------------------------------------------------------------- renormalised density gradient
//
// The corrected gradient of App. A.5 applied to the density:
//   G_i = L_i g_i,  L_i = M_i^-1,  M_i = sum_j V_j (x_j - x_i) (x) grad_i W_ij,
//   g_i = sum_j V_j (rho_j - rho_i) grad_i W_ij.
// With grad_i W_ij = gF d (d = x_i - x_j) every pair adds -V_j gF d d^T to M_i (symmetric)
// and V_j gF (rho_j - rho_i) d to g_i.  Same list traversal and eight canonical partial sums
// as the sweeps; a singular M_i gives G_i = 0.  G (and the symmetric L when requested) are
// written in sorted order: 2D L = (L00, L01, L11, 0); 3D L in two records
// (L00, L01, L02, L11), (L12, L22, 0, 0).

template <typename T, int DIM>
struct RenormAcc {
    T M[6];   // 2D: M00, M01, M11; 3D: M00, M01, M02, M11, M12, M22
    T g[3];
};

template <typename T, int DIM>
__device__ __forceinline__ bool inv_sym(const T* M, T* L)
{
    if (DIM == 2) {
        const T det = M[0] * M[2] - M[1] * M[1];
        if (!(det != T(0)) || !isfinite(det)) return false;
        const T id = T(1) / det;
        L[0] = M[2] * id;
        L[1] = -M[1] * id;
        L[2] = M[0] * id;
        return true;
    }
    const T a = M[0], b = M[1], c = M[2], d = M[3], e = M[4], f = M[5];
    const T c00 = d * f - e * e, c01 = c * e - b * f, c02 = b * e - c * d;
    const T det = a * c00 + b * c01 + c * c02;
    if (!(det != T(0)) || !isfinite(det)) return false;
    const T id = T(1) / det;
    L[0] = c00 * id;
    L[1] = c01 * id;
    L[2] = c02 * id;
    L[3] = (a * f - c * c) * id;
    L[4] = (b * c - a * e) * id;
    L[5] = (a * d - b * b) * id;
    return true;
}

// y = L x for the symmetric L stored as above.
template <typename T, int DIM>
__device__ __forceinline__ void sym_mul(const T* L, const T* x, T* y)
{
    if (DIM == 2) {
        y[0] = L[0] * x[0] + L[1] * x[1];
        y[1] = L[1] * x[0] + L[2] * x[1];
        y[2] = T(0);
    } else {
        y[0] = L[0] * x[0] + L[1] * x[1] + L[2] * x[2];
        y[1] = L[1] * x[0] + L[3] * x[1] + L[4] * x[2];
        y[2] = L[2] * x[0] + L[4] * x[1] + L[5] * x[2];
    }
}

template <typename T, int DIM, int LPP>
__global__ __launch_bounds__(256) void k_renorm(int64_t N, int32_t width, const int32_t* __restrict__ nbr,
                                                const int32_t* __restrict__ nbr_count,
                                                const vec4_t<T>* __restrict__ jd0, const vec4_t<T>* __restrict__ jd1,
                                                const T* __restrict__ rho3, const int32_t* __restrict__ psim,
                                                const SimConst<T>* __restrict__ sims, int filter,
                                                vec4_t<T>* __restrict__ G_out, vec4_t<T>* __restrict__ L_out)
{
    constexpr int NQ = kLeaves / LPP;
    constexpr int U = kPairsInFlight;
    constexpr int NM = DIM == 2 ? 3 : 6;
    const int64_t t = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int64_t i = t / LPP;
    const int r = (int)(t - i * LPP);
    if (i >= N) return;
    const SimConst<T>& S = sims[psim[i]];
    const PairConst<T> c = pair_const(S);
    T ui[3] = {0, 0, 0};
    unpack_u<T, DIM>(jd0[i], ui);
    const T rhoi = (DIM == 3) ? rho3[i] : jd1[i].z;
    int n = nbr_count[i];
    n = n < width ? n : width;
    const int mcount = (n - r + LPP - 1) / LPP;
    const int32_t* row = nbr + i * (int64_t)width;
    RenormAcc<T, DIM> acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
#pragma unroll
        for (int a = 0; a < 6; ++a) acc[q].M[a] = T(0);
        acc[q].g[0] = acc[q].g[1] = acc[q].g[2] = T(0);
    }
    int jn[U];
    load_entries<LPP, U>(row, r, 0, mcount, (int)i, jn);
    for (int m0 = 0; m0 < mcount; m0 += U) {
        vec4_t<T> a[U];
        T rj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            a[u] = ldo(jd0, (uint32_t)jn[u]);
            rj[u] = (DIM == 3) ? a[u].w : ldo(jd1, (uint32_t)jn[u]).z;
        }
        load_entries<LPP, U>(row, r, m0 + U, mcount, (int)i, jn);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (m0 + u >= mcount) continue;
            T d[3] = {0, 0, 0};
            const T r2 = r2_exact<T, DIM>(ui, a[u], c.L, c.invL, d);
            if (filter && !(r2 < c.H2)) continue;
            const T q = fast_sqrt(r2) * c.invH;
            const T tt = T(1) - q;
            const T t2 = tt * tt;
            const T gF = c.kG * (T(-56.0 / 3.0) * (t2 * t2 * tt) * (T(1) + T(5) * q));
            const T Vj = rec_volume<T, DIM>(a[u], S.m);
            const T f = Vj * gF;
            RenormAcc<T, DIM>& A = acc[u % NQ];
            if (DIM == 2) {
                A.M[0] -= f * d[0] * d[0];
                A.M[1] -= f * d[0] * d[1];
                A.M[2] -= f * d[1] * d[1];
            } else {
                A.M[0] -= f * d[0] * d[0];
                A.M[1] -= f * d[0] * d[1];
                A.M[2] -= f * d[0] * d[2];
                A.M[3] -= f * d[1] * d[1];
                A.M[4] -= f * d[1] * d[2];
                A.M[5] -= f * d[2] * d[2];
            }
            const T fr = f * (rj[u] - rhoi);
#pragma unroll
            for (int k = 0; k < DIM; ++k) A.g[k] += fr * d[k];
        }
    }
    T M[6], g[3] = {0, 0, 0}, tmp[NQ];
#pragma unroll
    for (int e = 0; e < NM; ++e) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) tmp[q] = acc[q].M[e];
        M[e] = combine_leaves<LPP>(tmp);
    }
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) tmp[q] = acc[q].g[k];
        g[k] = combine_leaves<LPP>(tmp);
    }
    if (r != 0) return;
    T L[6] = {0, 0, 0, 0, 0, 0}, G[3] = {0, 0, 0};
    if (inv_sym<T, DIM>(M, L)) sym_mul<T, DIM>(L, g, G);
    vec4_t<T> o;
    o.x = G[0];
    o.y = G[1];
    o.z = G[2];
    o.w = T(0);
    G_out[i] = o;
    if (L_out) {
        vec4_t<T> l0, l1;
        if (DIM == 2) {
            l0.x = L[0]; l0.y = L[1]; l0.z = L[2]; l0.w = T(0);
            L_out[i] = l0;
        } else {
            l0.x = L[0]; l0.y = L[1]; l0.z = L[2]; l0.w = L[3];
            l1.x = L[4]; l1.y = L[5]; l1.z = T(0); l1.w = T(0);
            L_out[2 * i] = l0;
            L_out[2 * i + 1] = l1;
        }
    }
}

template <typename T, int DIM>
struct FwdAcc {
    T ax[3];
    T rdv, rdd, rs, rdg;
};

// Per-particle sweep record of a neighbour (jd0, jd1; G with the renormalised diffusion).
template <typename T, int DIM>
struct FwdNbr {
    vec4_t<T> a, b, G;
};

// Forward pair terms of (i, j), added to acc:
//   a_i    += ((alpha H c0 rho0 pi_ij - p_i) V_j - p_j V_j) gW
//   drho_i += V_j (v_i - v_j).gW     (times rho_i later)   and   V_j (rho_i - rho_j) x_ij.gW / (r^2 + eps H^2)
//   rho_i  += W shape (times m C_d / H^d later)
// In 3D jd0 = (u, rho) and jd1 = (v, p), with V = m / rho recomputed as the writer computed it;
// in 2D jd0 = (u, V, p V) and jd1 = (v, rho, p).  Two records per neighbour either way, since
// the sweeps are bound by the vector L1's line rate, which counts gathers, not arithmetic.
// d and r2 are the pair vector x_ij and its square.  With keep false the pair leaves acc
// unchanged: MASK = false selects the old sums, MASK = true zeroes the kernel factors (every
// term carries gF or W) and adds, so the neighbour's records are consumed unconditionally and
// their loads stay ahead of the pair terms.  No implicit contraction: the products that are fused
// are written as fma, so a pair rounds the same whichever list position and lane count it has.
template <typename T, int DIM, bool RHOSUM, bool RENORM, bool MASK = false>
__device__ __forceinline__ void fwd_pair(const PairConst<T>& c, const T* vi, T rhoi, T pi, const FwdNbr<T, DIM>& nb,
                                         const T* Gi, const T* d, T r2, bool keep, FwdAcc<T, DIM>& acc)
{
#pragma clang fp contract(off)
    T vj[3];
    T Vj, pVj, rhoj;
    if (DIM == 3) {
        rhoj = nb.a.w;
        Vj = c.m * fast_rcp(rhoj);
        vj[0] = nb.b.x; vj[1] = nb.b.y; vj[2] = nb.b.z; pVj = nb.b.w * Vj;
    } else {
        Vj = nb.a.z; pVj = nb.a.w;
        vj[0] = nb.b.x; vj[1] = nb.b.y; rhoj = nb.b.z;
    }
    T ue = (vi[0] - vj[0]) * d[0];
#pragma unroll
    for (int k = 1; k < DIM; ++k) ue = fma(vi[k] - vj[k], d[k], ue);
    const T q = fast_sqrt(r2) * c.invH;
    const T t = T(1) - q;
    const T t2 = t * t;
    const T t4 = t2 * t2;
    const T t5 = t4 * t;
    T gF = c.kGF * (t5 * fma(T(5), q, T(1)));  // grad W = gF x_ij
    T wq = t4 * t2 * fma(q, fma(q, T(35.0 / 3.0), T(6)), T(1));   // W shape
    if (MASK) {
        const T kf = keep ? T(1) : T(0);
        gF = gF * kf;
        wq = wq * kf;
    }
    const T inv = fast_rcp(r2 + c.epsH2);
    const T pij = ue * inv;
    const T cg = fma(fma(c.cA, pij, -pi), Vj, -pVj) * gF;
    const T rdv = fma(Vj, gF * ue, acc.rdv);
    const T rdd = fma(Vj * (rhoi - rhoj), gF * r2 * inv, acc.rdd);
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const T ax = fma(cg, d[k], acc.ax[k]);
        acc.ax[k] = (MASK || keep) ? ax : acc.ax[k];
    }
    acc.rdv = (MASK || keep) ? rdv : acc.rdv;
    acc.rdd = (MASK || keep) ? rdd : acc.rdd;
    if (RHOSUM) acc.rs = (MASK || keep) ? acc.rs + wq : acc.rs;
    if (RENORM) {
        // V_j (G_i + G_j) . grad_i W_ij of the renormalised diffusion
        const T Gj[3] = {nb.G.x, nb.G.y, nb.G.z};
        T sg = (Gi[0] + Gj[0]) * d[0];
#pragma unroll
        for (int k = 1; k < DIM; ++k) sg = fma(Gi[k] + Gj[k], d[k], sg);
        const T rdg = fma(Vj, gF * sg, acc.rdg);
        acc.rdg = (MASK || keep) ? rdg : acc.rdg;
    }
}

// Cell assignment of the next step's sort, done by the sweep that produced the positions
// (same arithmetic as k_assign).  Null cell_count: no sort follows.
struct NextCells {
    const int32_t* blk_rank;
    int32_t* cell_count;
    int32_t* cell_of;
    int32_t* slot_of;
};

// The neighbour list positions of lane r among the LPP lanes of a particle are
// k = r + LPP m (m = 0, 1, ...); position k belongs to partial sum k mod 8, which is
// accumulator m mod (8 / LPP) of the lane.  Lanes gather the records of kPairsInFlight
// positions before computing them, in increasing m, with the list entries of the following
// group already in flight.
//
// In 3D the pairs of a group are computed without branches: a position past the lane's
// count or rejected by the filter is computed and dropped from the sums by a select (the
// accumulators start at +0 and never become -0, so adding nothing and skipping agree
// bitwise), which lets the compiler interleave the independent pairs of the group.  A 3D
// sweep keeps every SIMD busy with many wavefronts, and this takes the per-pair exec-mask
// branches out of its instruction stream.  In 2D with 2 or 8 lanes per particle the per-pair
// branches, which skip the tail positions that no lane of the wavefront holds, measured faster.
// In 2D with 4 lanes the list entries are read as quad chunks (a quarter of the entry loads, the
// vector L1's line rate being the bound) and the pairs again go without branches, dropped ones
// masked inside fwd_pair: with a branch per pair the compiler sinks a neighbour's gathers into
// it behind a full wait for the loads in flight.
template <typename T, int DIM, int MODE, int LPP, bool RENORM>
__global__ __launch_bounds__(256) void k_sweep(int64_t N, int32_t width, const int32_t* __restrict__ nbr,
                                               const int32_t* __restrict__ nbr_count,
                                               const vec4_t<T>* __restrict__ jd0, const vec4_t<T>* __restrict__ jd1,
                                               StatePtrs<T, DIM> cur, StatePtrs<T, DIM> dst,
                                               const int32_t* __restrict__ orig, T* __restrict__ drho_out,
                                               T* __restrict__ acc_out, T* __restrict__ rhosum_out,
                                               const int32_t* __restrict__ psim,
                                               const SimConst<T>* __restrict__ sims, int32_t* __restrict__ status,
                                               NextCells next, NextSlot<T> ns, int filter,
                                               unsigned long long* __restrict__ pair_counter,
                                               const vec4_t<T>* __restrict__ jdG)
{
    constexpr int NQ = kLeaves / LPP;
    constexpr int U = kPairsInFlight;
    static_assert(LPP >= 2 && LPP <= 8 && U % NQ == 0, "lanes per particle must be 2, 4 or 8");
    const int64_t t = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int64_t i = t / LPP;
    const int r = (int)(t - i * LPP);
    int accepted = 0;  // entries kept by the filter (lists with a skin), less the self entry
    if (i < N) {
    const int s = psim[i];
    const SimConst<T>& S = sims[s];
    const PairConst<T> c = pair_const(S);
    T ui[3] = {0, 0, 0}, vi[3] = {0, 0, 0};
    unpack_u<T, DIM>(jd0[i], ui);
#pragma unroll
    for (int k = 0; k < DIM; ++k) vi[k] = cur.v[k][i];
    const T rhoi = cur.rho[i];
    const T pi = tait(S, rhoi);
    T Gi[3] = {0, 0, 0};
    if (RENORM) {
        const vec4_t<T> g = jdG[i];
        Gi[0] = g.x;
        Gi[1] = g.y;
        Gi[2] = g.z;
    }
    int n = nbr_count[i];
    n = n < width ? n : width;
    const int mcount = (n - r + LPP - 1) / LPP;
    const int32_t* row = nbr + i * (int64_t)width;
    // every list holds its particle once, at r2 = 0, which the filter keeps
    if (r == 0 && n > 0) accepted = -1;
    FwdAcc<T, DIM> acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        acc[q].ax[0] = acc[q].ax[1] = acc[q].ax[2] = T(0);
        acc[q].rdv = acc[q].rdd = acc[q].rs = acc[q].rdg = T(0);
    }
    constexpr bool kSelect = DIM == 3;
    // four lanes per particle: list entries as 16-byte chunks and a quad transpose (one load
    // per lane and group of four positions instead of four), and no branch per position (the
    // positions past the count read the particle itself and are masked like dropped pairs), so
    // that no neighbour's gathers are sunk behind the pair terms of an earlier one
    constexpr bool kQuad = LPP == 4 && U == 4 && !kSelect;
    int jn[U];
    int4 chunk = make_int4(0, 0, 0, 0);
    if (kQuad) chunk = load_chunk4(row, width, 4 * r);
    else if (kSelect) load_entries_clamped<LPP, U>(row, width, r, 0, mcount, (int)i, jn);
    else load_entries<LPP, U>(row, r, 0, mcount, (int)i, jn);
    for (int m0 = 0; m0 < mcount; m0 += U) {
        if (kQuad) {
            int t4[4];
            quad_transpose(r, chunk, t4);
#pragma unroll
            for (int u = 0; u < U; ++u) jn[u] = (m0 + u < mcount) ? t4[u] : (int)i;
        }
        int jj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) jj[u] = jn[u];
        FwdNbr<T, DIM> nb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t j = (uint32_t)jj[u];
            nb[u].a = ldo(jd0, j);
            nb[u].b = ldo(jd1, j);
            if (RENORM) nb[u].G = ldo(jdG, j);
        }
        if (kQuad) chunk = load_chunk4(row, width, 4 * (m0 + U) + 4 * r);
        else if (kSelect) load_entries_clamped<LPP, U>(row, width, r, m0 + U, mcount, (int)i, jn);
        else load_entries<LPP, U>(row, r, m0 + U, mcount, (int)i, jn);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!kQuad && !kSelect && m0 + u >= mcount) continue;
            T d[3];
            const T r2 = r2_exact<T, DIM>(ui, nb[u].a, c.L, c.invL, d);
            const bool keep = (m0 + u < mcount) && (!filter || r2 < c.H2);
            if (!kQuad && !kSelect && !keep) continue;
            accepted += keep ? 1 : 0;
            if (kQuad)
                fwd_pair<T, DIM, MODE == kModeRhs, RENORM, true>(c, vi, rhoi, pi, nb[u], Gi, d, r2, keep, acc[u % NQ]);
            else
                fwd_pair<T, DIM, MODE == kModeRhs, RENORM>(c, vi, rhoi, pi, nb[u], Gi, d, r2, keep, acc[u % NQ]);
        }
    }
    T ax[3] = {0, 0, 0};
    T tmp[NQ];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) tmp[q] = acc[q].ax[k];
        ax[k] = combine_leaves<LPP>(tmp);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) tmp[q] = acc[q].rdv;
    const T rdv = combine_leaves<LPP>(tmp);
#pragma unroll
    for (int q = 0; q < NQ; ++q) tmp[q] = acc[q].rdd;
    const T rdd = combine_leaves<LPP>(tmp);
    T rs = 0;
    if (MODE == kModeRhs) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) tmp[q] = acc[q].rs;
        rs = combine_leaves<LPP>(tmp);
    }
    T rdg = 0;
    if (RENORM) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) tmp[q] = acc[q].rdg;
        rdg = combine_leaves<LPP>(tmp);
    }
    if (r == 0) {
    const T invrho = fast_rcp(rhoi);
    T a[3];
#pragma unroll
    for (int k = 0; k < DIM; ++k) a[k] = ax[k] * invrho;
    // renormalised diffusion: -delta H c0 sum_j V_j (G_i + G_j) . grad_i W_ij, cD = 2 delta H c0
    const T drho = RENORM ? rhoi * rdv + S.cD * rdd - T(0.5) * S.cD * rdg : rhoi * rdv + S.cD * rdd;
    if (MODE == kModeStep) {
        bool bad = !isfinite(drho);
        const T dt = S.dt;
        int cc[3] = {0, 0, 0};
        T xn[3] = {0, 0, 0}, vn[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            vn[k] = vi[k] + dt * a[k];
            xn[k] = cur.x[k][i] + dt * vn[k];
            dst.v[k][i] = vn[k];
            dst.x[k][i] = xn[k];
            bad = bad || !isfinite(vn[k]) || !isfinite(xn[k]);
            cc[k] = cell_coord(wrap_pos(isfinite(xn[k]) ? xn[k] : T(0), S.L, S.invL), S.cinv, S.nc);
        }
        const T rhon = rhoi + dt * drho;
        dst.rho[i] = rhon;
        if (bad) atomicOr(&status[s], kFlagNonfinite);
        if (next.cell_count) {
            const int gcell = global_cell<T, DIM>(S, next.blk_rank, cc[0], cc[1], cc[2]);
            next.cell_of[i] = gcell;
            next.slot_of[i] = atomicAdd(&next.cell_count[gcell], 1);
        }
        if (ns.jd0) {
            // packed records of the next step, as the sort would write them
            T u[3] = {0, 0, 0};
#pragma unroll
            for (int k = 0; k < DIM; ++k) u[k] = wrap_pos(isfinite(xn[k]) ? xn[k] : T(0), S.L, S.invL);
            const T V = S.m * fast_rcp(rhon);
            const T pn = tait(S, rhon);
            const T pV = pn * V;
            vec4_t<T> pa, pb;
            if (DIM == 3) {
                pa.x = u[0]; pa.y = u[1]; pa.z = u[2]; pa.w = rhon;
                pb.x = vn[0]; pb.y = vn[1]; pb.z = vn[2]; pb.w = pn;
            } else {
                pa.x = u[0]; pa.y = u[1]; pa.z = V; pa.w = pV;
                pb.x = vn[0]; pb.y = vn[1]; pb.z = rhon; pb.w = pn;
            }
            ns.jd0[i] = pa;
            ns.jd1[i] = pb;
            ns.orig[i] = orig[i];
            // displacement since the lists were built (minimum image)
            const vec4_t<T> ref = ns.uref[i];
            const T rr[3] = {ref.x, ref.y, ref.z};
            T d2 = T(0);
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                T d = u[k] - rr[k];
                d -= S.L * rint(d * S.invL);
                d2 += d * d;
            }
            if (!(d2 <= ref.w * ref.w)) atomicOr(&status[s], kFlagSkin);
        }
    } else {
        const int o = orig[i];
        drho_out[o] = drho;
#pragma unroll
        for (int k = 0; k < DIM; ++k) acc_out[(int64_t)k * N + o] = a[k];
        if (rhosum_out) rhosum_out[o] = S.m * S.kW * rs;
    }
    }
    }
    if (pair_counter) {
        // wave total of the filtered pairs, one integer atomic per wavefront
        int w = accepted;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o, 64);
        if ((threadIdx.x & 63) == 0 && w)
            atomicAdd(&pair_counter[(blockIdx.x & (kPairSlots - 1)) * kPairStride], (unsigned long long)w);
    }
}

// ---------------------------------------------------------------- density-summation adjoint
//
// Cotangent of the positions for cotangents g of the summation density rho_i = m sum_j W_ij
// (the backward benchmark of Sec. 4.1): xbar_k = m sum_{j != k} (g_k + g_j) grad_k W_kj, since
// x_k enters k's own sum and, through W_jk = W_kj, every neighbour's.  The self entry of the
// list has a zero pair vector and adds nothing.  Same list traversal and canonical partial
// sums as the forward sweep.

template <typename T>
__global__ __launch_bounds__(256) void k_gather_sorted(int64_t N, const T* __restrict__ in,
                                                       const int32_t* __restrict__ orig, T* __restrict__ out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < N) out[q] = in[orig[q]];
}

template <typename T, int DIM, int LPP>
__global__ __launch_bounds__(256) void k_density_adj(int64_t N, int32_t width, const int32_t* __restrict__ nbr,
                                                     const int32_t* __restrict__ nbr_count,
                                                     const vec4_t<T>* __restrict__ jd0, const T* __restrict__ gs,
                                                     const int32_t* __restrict__ orig,
                                                     const int32_t* __restrict__ psim,
                                                     const SimConst<T>* __restrict__ sims, T* __restrict__ xbar,
                                                     int filter)
{
    constexpr int NQ = kLeaves / LPP;
    constexpr int U = kPairsInFlight;
    static_assert(LPP >= 2 && LPP <= 8 && U % NQ == 0, "lanes per particle must be 2, 4 or 8");
    const int64_t t = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int64_t i = t / LPP;
    const int r = (int)(t - i * LPP);
    if (i >= N) return;
    const SimConst<T>& S = sims[psim[i]];
    const PairConst<T> c = pair_const(S);
    T ui[3] = {0, 0, 0};
    unpack_u<T, DIM>(jd0[i], ui);
    const T gi = gs[i];
    int n = nbr_count[i];
    n = n < width ? n : width;
    const int mcount = (n - r + LPP - 1) / LPP;
    const int32_t* row = nbr + i * (int64_t)width;
    T acc[NQ][3];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q][0] = acc[q][1] = acc[q][2] = T(0);
    int jn[U];
    load_entries<LPP, U>(row, r, 0, mcount, (int)i, jn);
    for (int m0 = 0; m0 < mcount; m0 += U) {
        vec4_t<T> a[U];
        T gj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            a[u] = ldo(jd0, (uint32_t)jn[u]);
            gj[u] = ldo(gs, (uint32_t)jn[u]);
        }
        load_entries<LPP, U>(row, r, m0 + U, mcount, (int)i, jn);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (m0 + u >= mcount) continue;
            T d[3] = {0, 0, 0};
            const T r2 = r2_exact<T, DIM>(ui, a[u], c.L, c.invL, d);
            if (filter && !(r2 < c.H2)) continue;
            const T q = fast_sqrt(r2) * c.invH;
            const T tt = T(1) - q;
            const T t2 = tt * tt;
            const T t5 = t2 * t2 * tt;
            const T gF = c.kGF * (t5 * (T(1) + T(5) * q));
            const T w = (gi + gj[u]) * gF;
#pragma unroll
            for (int k = 0; k < DIM; ++k) acc[u % NQ][k] += w * d[k];
        }
    }
    T out[3] = {0, 0, 0};
    T tmp[NQ];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) tmp[q] = acc[q][k];
        out[k] = combine_leaves<LPP>(tmp);
    }
    if (r != 0) return;
    const int o = orig[i];
#pragma unroll
    for (int k = 0; k < DIM; ++k) xbar[(int64_t)k * N + o] = S.m * out[k];
}

// ---------------------------------------------------------------- explicit Runge-Kutta stages

// out = s0 base + sum_j c[j] K[j] over every field of the states (original order), with up to
// four terms; out may be base (every element is read before it is written).  s0 and the c[j]
// are multiplied by the particle's simulation time step when s0_dt / c_dt are set.  Stage
// states u_i = u + dt sum_j A_ij k_j, the step's end u + dt sum_i b_i k_i, and the adjoint's
// stage cotangents are all of this form.
constexpr int kMaxStages = 4;

template <typename T, int DIM>
struct LinComb {
    StatePtrs<T, DIM> out, base;
    T s0;
    int s0_dt, c_dt, nterm;
    T c[kMaxStages];
    StatePtrs<T, DIM> K[kMaxStages];
};

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_lincomb(int64_t N, LinComb<T, DIM> L, const int32_t* __restrict__ psim,
                                                 const SimConst<T>* __restrict__ sims)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const T dt = sims[psim[i]].dt;
    const T s0 = L.s0_dt ? L.s0 * dt : L.s0;
    T x[3], v[3], r;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        x[k] = s0 * L.base.x[k][i];
        v[k] = s0 * L.base.v[k][i];
    }
    r = s0 * L.base.rho[i];
    for (int j = 0; j < L.nterm; ++j) {
        const T c = L.c_dt ? L.c[j] * dt : L.c[j];
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            x[k] += c * L.K[j].x[k][i];
            v[k] += c * L.K[j].v[k][i];
        }
        r += c * L.K[j].rho[i];
    }
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        L.out.x[k][i] = x[k];
        L.out.v[k][i] = v[k];
    }
    L.out.rho[i] = r;
}

// ---------------------------------------------------------------- symplectic Euler
//
// DualSPHysics' symplectic scheme (Sec. 3.4, App. C), h = dt/2: the predictor state
// u_h = (x + h v, v + h a1, rho + h D1) is formed by k_lincomb, the corrector's rates
// (a2, D2) = f(u_h) by a right-hand-side sweep, and the step ends with
//   v' = v + dt a2,  x' = x_h + h v',  rho' = rho (2 - e) / (2 + e),  e = -dt D2 / rho_h.
// All three kernels run in original particle order.

// The corrector, u in place; uh = predictor state, r2 = (., a2, D2).
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_symp_final(int64_t N, StatePtrs<T, DIM> u, StatePtrs<T, DIM> uh,
                                                    StatePtrs<T, DIM> r2, const int32_t* __restrict__ psim,
                                                    const SimConst<T>* __restrict__ sims)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const T dt = sims[psim[i]].dt;
    const T h = T(0.5) * dt;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const T vn = u.v[k][i] + dt * r2.v[k][i];
        u.v[k][i] = vn;
        u.x[k][i] = uh.x[k][i] + h * vn;
    }
    const T e = -dt * r2.rho[i] / uh.rho[i];
    u.rho[i] = u.rho[i] * (T(2) - e) / (T(2) + e);
}

// Transpose of the corrector.  cot = (xb', vb', rb') of u'; cb (null for none) = cotangent of
// (a2, D2) where the next step re-uses them.  With vt = vb' + h xb', g(e) = (2 - e)/(2 + e),
// eb = rb' rho g'(e):
//   kb2 = (0, dt vt + cb_a, -dt eb / rho_h + cb_D)       rates' cotangent, for the VJP at u_h
//   uhd = (xb', 0, eb dt D2 / rho_h^2)                    u_h's cotangent outside that VJP
//   b0  = (0, vt, rb' g)                                  u's cotangent outside the predictor
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_symp_final_adj(int64_t N, StatePtrs<T, DIM> cot, const T* __restrict__ rho,
                                                        const T* __restrict__ rho_h, const T* __restrict__ d2,
                                                        StatePtrs<T, DIM> cb, int has_cb, StatePtrs<T, DIM> kb2,
                                                        StatePtrs<T, DIM> uhd, StatePtrs<T, DIM> b0,
                                                        const int32_t* __restrict__ psim,
                                                        const SimConst<T>* __restrict__ sims)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const T dt = sims[psim[i]].dt;
    const T h = T(0.5) * dt;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const T xb = cot.x[k][i];
        const T vt = cot.v[k][i] + h * xb;
        kb2.x[k][i] = T(0);
        kb2.v[k][i] = dt * vt + (has_cb ? cb.v[k][i] : T(0));
        uhd.x[k][i] = xb;
        uhd.v[k][i] = T(0);
        b0.x[k][i] = T(0);
        b0.v[k][i] = vt;
    }
    const T rb = cot.rho[i], rh = rho_h[i], D2 = d2[i];
    const T e = -dt * D2 / rh;
    const T g = (T(2) - e) / (T(2) + e);
    const T gp = T(-4) / ((T(2) + e) * (T(2) + e));
    const T eb = rb * rho[i] * gp;
    kb2.rho[i] = -dt * eb / rh + (has_cb ? cb.rho[i] : T(0));
    uhd.rho[i] = eb * dt * D2 / (rh * rh);
    b0.rho[i] = rb * g;
}

// Transpose of the predictor when its rates were re-used (not evaluated from u): with
// kb1 = h ubar_h, u's cotangent is b0 + (0, kb1_x, 0) (the x-rate of the predictor is v) and
// the re-used rates receive (kb1_v, kb1_rho).
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_symp_pred_adj(int64_t N, StatePtrs<T, DIM> b0, StatePtrs<T, DIM> kb1,
                                                       StatePtrs<T, DIM> cot, StatePtrs<T, DIM> cb)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        cot.x[k][i] = b0.x[k][i];
        cot.v[k][i] = b0.v[k][i] + kb1.x[k][i];
        cb.v[k][i] = kb1.v[k][i];
    }
    cot.rho[i] = b0.rho[i];
    cb.rho[i] = kb1.rho[i];
}

// ---------------------------------------------------------------- unsort

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_unsort(int64_t N, StatePtrs<T, DIM> src, const int32_t* __restrict__ orig,
                                                StatePtrs<T, DIM> dst)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const int o = orig[q];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        dst.x[k][o] = src.x[k][q];
        dst.v[k][o] = src.v[k][q];
    }
    dst.rho[o] = src.rho[q];
}

// ---------------------------------------------------------------- adjoint

// Gathers the output cotangents into sorted order: jdA = (abar / rho, rbar) with
// vt = v'_bar + dt x'_bar, abar = dt vt, rbar = dt rho'_bar; jdB = (rho, p, rbar rho, dp/drho).
// The acceleration cotangent enters every pair term divided by its particle's density, so the
// record holds it divided once.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_adj_prologue(int64_t N, const int32_t* __restrict__ orig,
                                                      StatePtrs<T, DIM> cot, StatePtrs<T, DIM> cur,
                                                      vec4_t<T>* __restrict__ jdA, vec4_t<T>* __restrict__ jdB,
                                                      const int32_t* __restrict__ psim,
                                                      const SimConst<T>* __restrict__ sims, int vjp)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const SimConst<T>& S = sims[psim[q]];
    const int o = orig[q];
    T ab[3] = {0, 0, 0};
    T rb;
    if (vjp) {
        // the update function's VJP: cot holds the cotangents (kx, ka, krho) of (v, a, drho/dt)
#pragma unroll
        for (int k = 0; k < DIM; ++k) ab[k] = cot.v[k][o];
        rb = cot.rho[o];
    } else {
        // one semi-implicit Euler step: abar = dt (vbar' + dt xbar'), rbar = dt rhobar'
#pragma unroll
        for (int k = 0; k < DIM; ++k) ab[k] = S.dt * (cot.v[k][o] + S.dt * cot.x[k][o]);
        rb = S.dt * cot.rho[o];
    }
    const T rho = cur.rho[q];
    const T ir = fast_rcp(rho);
    vec4_t<T> a;
    if (DIM == 3) {
        a.x = ab[0] * ir; a.y = ab[1] * ir; a.z = ab[2] * ir; a.w = rb;
    } else {
        a.x = ab[0] * ir; a.y = ab[1] * ir; a.z = rb; a.w = rb * rho;
    }
    jdA[q] = a;
    vec4_t<T> b;
    b.x = rho;
    b.y = tait(S, rho);
    b.z = rb * rho;
    b.w = tait_slope(S, rho);
    jdB[q] = b;
}

// What the adjoint sweep of step t prepares for the adjoint of step t - 1 when both states share
// the particle order (a step within one list-reuse interval): the prologue records of step t - 1
// at the same sorted index, from the cotangents the sweep has just formed (null jdA: none).
template <typename T>
struct NextAdj {
    vec4_t<T>* jdA;
    vec4_t<T>* jdB;
    const T* rho;   // densities of state t - 1, sorted order
};

template <typename T, int DIM>
struct AdjAcc {
    T gx[3], gv[3];
    T gr;
    T Gb[3];   // cotangent of the renormalised density gradient
};

// Per-particle adjoint record of a neighbour: jd0 = (u, rho), jd1 = (v, p), jdA = (abar / rho, rbar)
// in 3D; jd0 = (u, V, p V), jd1 = (v, rho, p), jdA = (abar / rho, rbar, rbar rho) in 2D.  They
// hold everything a neighbour contributes (3D: V = m / rho and rbar rho recomputed), so the
// sweep gathers three records per neighbour; jdB = (rho, p, rbar rho, dp/drho) is read for the
// particle itself only.
template <typename T>
struct AdjNbr {
    vec4_t<T> a, b, A, G;
};

// Adjoint pair terms, gather form.  For particle k and a neighbour j != k: the partial
// derivatives, with respect to k's position, velocity and density, of the two directed pair
// terms (k,j) and (j,k) contracted with their particles' cotangents (abar, rbar).  With
// e = x_kj, G = gF e, the kernel Hessian Jg = gF I + hF e e^T, pi = (v_k - v_j).e / (r^2+eps H^2),
// s = e.G / (r^2+eps H^2), these partials reduce to the closed forms below.  The self pair
// contributes exactly zero.  The momentum term's factor 1/rho_k and 1/rho_j always multiplies
// the acceleration cotangent of the same particle, so both sides take abar / rho from their
// records (ak, aj here), and X = cA pi - p_k - p_j is the pressure-and-viscosity factor that
// Q_k = X / rho_k and Q_j = X / rho_j share.
//
// With RENORM, the renormalised diffusion T_i = c sum_j V_j (G_i + G_j) . grad_i W_ij
// (c = -delta H c0) adds, for q = rbar_k V_j - rbar_j V_k and s = G_k + G_j with the
// gradients held fixed: gx += c q Jg s, Gbar += c q gF e, gr += (V_k / rho_k) c rbar_j gF s.e.
template <typename T>
struct AdjSelf {
    T v[3], a[3];   // velocity, abar / rho
    T rb, V, rho, p, ir, dp;
    T rbr;          // rbar rho
    T Vir;          // V / rho
    T G[3];
};

template <typename T, int DIM, bool RENORM>
__device__ __forceinline__ void adj_pair(const PairConst<T>& c, const AdjSelf<T>& K, const AdjNbr<T>& nb,
                                         const T* e, T r2, bool keep, AdjAcc<T, DIM>& acc)
{
    T vj[3], aj[3];
    T Vj, rbj;
    if (DIM == 3) {
        Vj = c.m * fast_rcp(nb.a.w);
        vj[0] = nb.b.x; vj[1] = nb.b.y; vj[2] = nb.b.z;
        aj[0] = nb.A.x; aj[1] = nb.A.y; aj[2] = nb.A.z; rbj = nb.A.w;
    } else {
        Vj = nb.a.z;
        vj[0] = nb.b.x; vj[1] = nb.b.y;
        aj[0] = nb.A.x; aj[1] = nb.A.y; rbj = nb.A.z;
    }
    const T rhoj = (DIM == 3) ? nb.a.w : nb.b.z;
    const T pj = nb.b.w;
    const T rbrj = (DIM == 3) ? rbj * rhoj : nb.A.w;
    const T cA = c.cA, cD = c.cD;
    const T Vk = K.V, rbk = K.rb, rhok = K.rho;
    T u[3];
    T ue = 0, ake = 0, aje = 0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        u[k] = K.v[k] - vj[k];
        ue += u[k] * e[k];
        ake += K.a[k] * e[k];
        aje += aj[k] * e[k];
    }
    const T q = fast_sqrt(r2) * c.invH;
    const T t = T(1) - q;
    const T t2 = t * t;
    const T t4 = t2 * t2;
    const T gF = c.kGF * (t4 * t * (T(1) + T(5) * q));  // grad W = gF e
    const T hF = c.kH * t4;                                              // Hessian: gF I + hF e e^T
    const T inv = fast_rcp(r2 + c.epsH2);
    const T pij = ue * inv;
    const T sij = gF * r2 * inv;
    const T sig = inv * (T(2) * gF + hF * r2 - T(2) * sij);              // d s / d e = sig e
    const T aGk = gF * ake, aGj = gF * aje, uG = gF * ue;
    const T X = cA * pij - (K.p + pj);
    const T beta = cA * inv * (Vj * aGk - Vk * aGj);
    const T gam = Vj * K.rbr + Vk * rbrj;
    const T drho = rhok - rhoj;
    const T cdr = cD * sig * drho * (Vj * rbk - Vk * rbj);
    T w[3];
    T ew = 0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        w[k] = X * (Vj * K.a[k] - Vk * aj[k]) + gam * u[k];
        ew += e[k] * w[k];
    }
    const T ce = cdr - T(2) * beta * pij + hF * ew;  // coefficient of e in the position cotangent
    const T bg = beta + gam * gF;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        acc.gx[k] = keep ? fma(gF, w[k], fma(ce, e[k], fma(beta, u[k], acc.gx[k]))) : acc.gx[k];
        acc.gv[k] = keep ? fma(bg, e[k], acc.gv[k]) : acc.gv[k];
    }
    // density cotangent: the (k,j) and (j,k) terms' density partials; the (j,k) momentum term
    // enters through 1/rho_k as -(V_k / rho_k) P
    const T cds = cD * sij;
    const T rbjc = rbj * cds;
    const T P = rbrj * uG - X * aGj - drho * rbjc;
    const T dgr = Vj * (aGk * -(K.dp + X * K.ir) + rbk * (uG + cds)) - K.Vir * P + Vk * (aGj * K.dp - rbjc);
    acc.gr = keep ? acc.gr + dgr : acc.gr;
    if (RENORM) {
        const T cr = T(-0.5) * cD;
        const T Gj[3] = {nb.G.x, nb.G.y, nb.G.z};
        T sv[3], es = T(0);
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            sv[k] = K.G[k] + Gj[k];
            es += e[k] * sv[k];
        }
        const T qq = cr * (rbk * Vj - rbj * Vk);
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            acc.gx[k] = keep ? acc.gx[k] + qq * (gF * sv[k] + hF * es * e[k]) : acc.gx[k];
            acc.Gb[k] = keep ? acc.Gb[k] + qq * gF * e[k] : acc.Gb[k];
        }
        acc.gr = keep ? acc.gr + Vk * K.ir * cr * rbj * gF * es : acc.gr;
    }
}

template <typename T, int DIM, int LPP, bool RENORM>
__global__ __launch_bounds__(256) void k_adj_sweep(int64_t N, int32_t width, const int32_t* __restrict__ nbr,
                                                   const int32_t* __restrict__ nbr_count,
                                                   const vec4_t<T>* __restrict__ jd0,
                                                   const vec4_t<T>* __restrict__ jd1,
                                                   const vec4_t<T>* __restrict__ jdA,
                                                   const vec4_t<T>* __restrict__ jdB,
                                                   const int32_t* __restrict__ orig, StatePtrs<T, DIM> cot,
                                                   const int32_t* __restrict__ psim,
                                                   const SimConst<T>* __restrict__ sims, int32_t* __restrict__ status,
                                                   int filter, int vjp, const vec4_t<T>* __restrict__ jdG,
                                                   const vec4_t<T>* __restrict__ jdL, vec4_t<T>* __restrict__ gbar,
                                                   NextAdj<T> na)
{
    constexpr int NQ = kLeaves / LPP;
    constexpr int U = kPairsInFlight;
    static_assert(LPP >= 2 && LPP <= 8 && U % NQ == 0, "lanes per particle must be 2, 4 or 8");
    const int64_t t = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int64_t k = t / LPP;
    const int r = (int)(t - k * LPP);
    if (k >= N) return;
    const int s = psim[k];
    const SimConst<T>& S = sims[s];
    const PairConst<T> c = pair_const(S);
    T uk[3] = {0, 0, 0};
    AdjSelf<T> K;
    {
        const vec4_t<T> a = jd0[k], b = jd1[k], A = jdA[k];
        K.v[2] = K.a[2] = T(0);
        if (DIM == 3) {
            uk[0] = a.x; uk[1] = a.y; uk[2] = a.z; K.V = S.m * fast_rcp(a.w);
            K.v[0] = b.x; K.v[1] = b.y; K.v[2] = b.z;
            K.a[0] = A.x; K.a[1] = A.y; K.a[2] = A.z; K.rb = A.w;
        } else {
            uk[0] = a.x; uk[1] = a.y; K.V = a.z;
            K.v[0] = b.x; K.v[1] = b.y;
            K.a[0] = A.x; K.a[1] = A.y; K.rb = A.z;
        }
    }
    {
        const vec4_t<T> Bk = jdB[k];
        K.rho = Bk.x;
        K.p = Bk.y;
        K.rbr = Bk.z;
        K.dp = Bk.w;
        K.ir = fast_rcp(K.rho);
        K.Vir = K.V * K.ir;
    }
    K.G[0] = K.G[1] = K.G[2] = T(0);
    if (RENORM) {
        const vec4_t<T> g = jdG[k];
        K.G[0] = g.x;
        K.G[1] = g.y;
        K.G[2] = g.z;
    }
    int n = nbr_count[k];
    n = n < width ? n : width;
    const int mcount = (n - r + LPP - 1) / LPP;
    const int32_t* row = nbr + k * (int64_t)width;
    AdjAcc<T, DIM> acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
#pragma unroll
        for (int d = 0; d < 3; ++d) acc[q].gx[d] = acc[q].gv[d] = acc[q].Gb[d] = T(0);
        acc[q].gr = T(0);
    }
    int jn[U];
    int4 chunk = make_int4(0, 0, 0, 0);
    constexpr bool kQuad = LPP == 4 && U == 4;
    if (kQuad) chunk = load_chunk4(row, width, 4 * r);
    else load_entries<LPP, U>(row, r, 0, mcount, (int)k, jn);
    for (int m0 = 0; m0 < mcount; m0 += U) {
        if (kQuad) {
            int t4[4];
            quad_transpose(r, chunk, t4);
#pragma unroll
            for (int u = 0; u < U; ++u) jn[u] = (m0 + u < mcount) ? t4[u] : (int)k;
        }
        AdjNbr<T> nb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t j = (uint32_t)jn[u];
            nb[u].a = ldo(jd0, j);
            nb[u].b = ldo(jd1, j);
            nb[u].A = ldo(jdA, j);
            if (RENORM) nb[u].G = ldo(jdG, j);
        }
        if (kQuad) chunk = load_chunk4(row, width, 4 * (m0 + U) + 4 * r);
        else load_entries<LPP, U>(row, r, m0 + U, mcount, (int)k, jn);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // position m0 is below the count inside the loop; its pair is dropped by a select
            // rather than a branch, which keeps its gathers ahead of the pair terms
            if (u > 0 && m0 + u >= mcount) continue;
            T e[3];
            const T r2 = r2_exact<T, DIM>(uk, nb[u].a, c.L, c.invL, e);
            const bool keep = !filter || r2 < c.H2;
            if (u > 0 && !keep) continue;
            adj_pair<T, DIM, RENORM>(c, K, nb[u], e, r2, keep, acc[u % NQ]);
        }
    }
    T gx[3] = {0, 0, 0}, gv[3] = {0, 0, 0};
    T tmp[NQ];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) tmp[q] = acc[q].gx[d];
        gx[d] = combine_leaves<LPP>(tmp);
#pragma unroll
        for (int q = 0; q < NQ; ++q) tmp[q] = acc[q].gv[d];
        gv[d] = combine_leaves<LPP>(tmp);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) tmp[q] = acc[q].gr;
    const T gr = combine_leaves<LPP>(tmp);
    T Gb[3] = {0, 0, 0};
    if (RENORM) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) tmp[q] = acc[q].Gb[d];
            Gb[d] = combine_leaves<LPP>(tmp);
        }
    }
    if (r != 0) return;
    if (RENORM) {
        // gbar_k = L_k^T Gbar_k (L symmetric), for the second renormalisation pass
        T L[6] = {0, 0, 0, 0, 0, 0};
        if (DIM == 2) {
            const vec4_t<T> l0 = jdL[k];
            L[0] = l0.x; L[1] = l0.y; L[2] = l0.z;
        } else {
            const vec4_t<T> l0 = jdL[2 * k], l1 = jdL[2 * k + 1];
            L[0] = l0.x; L[1] = l0.y; L[2] = l0.z; L[3] = l0.w; L[4] = l1.x; L[5] = l1.y;
        }
        T gb[3];
        sym_mul<T, DIM>(L, Gb, gb);
        vec4_t<T> o4;
        o4.x = gb[0];
        o4.y = gb[1];
        o4.z = gb[2];
        o4.w = T(0);
        gbar[k] = o4;
    }
    const int o = orig[k];
    const T dt = S.dt;
    bool bad = !isfinite(gr);
    T xn[3] = {0, 0, 0}, vn[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const T xb = cot.x[d][o];
        const T vb = cot.v[d][o];
        if (vjp) {
            // (xbar, vbar, rhobar) = (J_x^T, kx + J_v^T, J_rho^T): dx/dt = v adds kx to vbar
            xn[d] = gx[d];
            vn[d] = xb + gv[d];
        } else {
            xn[d] = xb + gx[d];
            vn[d] = vb + dt * xb + gv[d];
        }
        cot.x[d][o] = xn[d];
        cot.v[d][o] = vn[d];
        bad = bad || !isfinite(gx[d]) || !isfinite(gv[d]);
    }
    const T rn = vjp ? gr : cot.rho[o] + gr;
    cot.rho[o] = rn;
    if (bad) atomicOr(&status[s], kFlagNonfinite);
    if (na.jdA) {
        // the prologue of the previous step's adjoint (same arithmetic as k_adj_prologue)
        T ab[3] = {0, 0, 0};
#pragma unroll
        for (int d = 0; d < DIM; ++d) ab[d] = dt * (vn[d] + dt * xn[d]);
        const T rb = dt * rn;
        const T rho = na.rho[k];
        const T ir = fast_rcp(rho);
        vec4_t<T> a;
        if (DIM == 3) {
            a.x = ab[0] * ir; a.y = ab[1] * ir; a.z = ab[2] * ir; a.w = rb;
        } else {
            a.x = ab[0] * ir; a.y = ab[1] * ir; a.z = rb; a.w = rb * rho;
        }
        na.jdA[k] = a;
        vec4_t<T> b;
        b.x = rho;
        b.y = tait(S, rho);
        b.z = rb * rho;
        b.w = tait_slope(S, rho);
        na.jdB[k] = b;
    }
}

// Second pass of the renormalised diffusion's adjoint: the cotangents of the moment sums
// M_i, g_i (Mbar_i = -gbar_i G_i^T, gbar_i = L_i Gbar_i from the adjoint sweep) carried to
// positions and densities, gathered over each particle's own sums and its neighbours':
//   own (e = x_k - x_j, w = gF e, Jg v = gF v + hF (e.v) e):
//     xbar_k += V_j [gbar_k (G_k.w) + Jg G_k (gbar_k.e)] + V_j (rho_j - rho_k) Jg gbar_k
//     rbar_k -= V_j (gbar_k.w)
//   neighbour's:
//     xbar_k += V_k [gbar_j (G_j.w) + Jg G_j (gbar_j.e)] - V_k (rho_k - rho_j) Jg gbar_j
//     rbar_k += -V_k (gbar_j.w) + (V_k / rho_k) [(rho_k - rho_j)(gbar_j.w) - (e.gbar_j)(G_j.w)]
// added to the cotangents (original order).  Same list traversal and partial sums.
template <typename T, int DIM, int LPP>
__global__ __launch_bounds__(256) void k_renorm_adj(int64_t N, int32_t width, const int32_t* __restrict__ nbr,
                                                    const int32_t* __restrict__ nbr_count,
                                                    const vec4_t<T>* __restrict__ jd0, const vec4_t<T>* __restrict__ jdB,
                                                    const vec4_t<T>* __restrict__ jdG,
                                                    const vec4_t<T>* __restrict__ gbar,
                                                    const int32_t* __restrict__ orig, StatePtrs<T, DIM> cot,
                                                    const int32_t* __restrict__ psim,
                                                    const SimConst<T>* __restrict__ sims, int filter)
{
    constexpr int NQ = kLeaves / LPP;
    constexpr int U = kPairsInFlight;
    const int64_t t = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int64_t k = t / LPP;
    const int r = (int)(t - k * LPP);
    if (k >= N) return;
    const SimConst<T>& S = sims[psim[k]];
    const PairConst<T> c = pair_const(S);
    const vec4_t<T> a0 = jd0[k];
    T uk[3] = {0, 0, 0};
    unpack_u<T, DIM>(a0, uk);
    const T Vk = rec_volume<T, DIM>(a0, S.m);
    const T rhok = jdB[k].x;
    const vec4_t<T> g4 = jdG[k], b4 = gbar[k];
    const T Gk[3] = {g4.x, g4.y, g4.z}, bk[3] = {b4.x, b4.y, b4.z};
    int n = nbr_count[k];
    n = n < width ? n : width;
    const int mcount = (n - r + LPP - 1) / LPP;
    const int32_t* row = nbr + k * (int64_t)width;
    T ax[NQ][3], ar[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) ax[q][0] = ax[q][1] = ax[q][2] = ar[q] = T(0);
    int jn[U];
    load_entries<LPP, U>(row, r, 0, mcount, (int)k, jn);
    for (int m0 = 0; m0 < mcount; m0 += U) {
        vec4_t<T> na[U], nB[U], nG[U], nb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t j = (uint32_t)jn[u];
            na[u] = ldo(jd0, j);
            nB[u] = ldo(jdB, j);
            nG[u] = ldo(jdG, j);
            nb[u] = ldo(gbar, j);
        }
        load_entries<LPP, U>(row, r, m0 + U, mcount, (int)k, jn);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (m0 + u >= mcount) continue;
            T e[3] = {0, 0, 0};
            const T r2 = r2_exact<T, DIM>(uk, na[u], c.L, c.invL, e);
            if (filter && !(r2 < c.H2)) continue;
            const T q = fast_sqrt(r2) * c.invH;
            const T tt = T(1) - q;
            const T t2 = tt * tt;
            const T t4 = t2 * t2;
            const T gF = c.kG * (T(-56.0 / 3.0) * t4 * tt * (T(1) + T(5) * q));
            const T hF = c.kH * t4;
            const T Vj = rec_volume<T, DIM>(na[u], S.m);
            const T rhoj = nB[u].x;
            const T Gj[3] = {nG[u].x, nG[u].y, nG[u].z}, bj[3] = {nb[u].x, nb[u].y, nb[u].z};
            T bke = 0, bje = 0, Gke = 0, Gje = 0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                Gke += Gk[d] * e[d];
                bke += bk[d] * e[d];
                Gje += Gj[d] * e[d];
                bje += bj[d] * e[d];
            }
            const T Gkw = gF * Gke, Gjw = gF * Gje, bkw = gF * bke, bjw = gF * bje;
            const T drk = rhoj - rhok;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                // Jg v = gF v + hF (e.v) e
                const T JGk = gF * Gk[d] + hF * Gke * e[d];
                const T Jbk = gF * bk[d] + hF * bke * e[d];
                const T JGj = gF * Gj[d] + hF * Gje * e[d];
                const T Jbj = gF * bj[d] + hF * bje * e[d];
                ax[u % NQ][d] += Vj * (bk[d] * Gkw + JGk * bke) + Vj * drk * Jbk +
                                 Vk * (bj[d] * Gjw + JGj * bje) + Vk * drk * Jbj;
            }
            ar[u % NQ] += -Vj * bkw - Vk * bjw + (Vk / rhok) * (-drk * bjw - bje * Gjw);
        }
    }
    T gx[3] = {0, 0, 0}, tmp[NQ];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) tmp[q] = ax[q][d];
        gx[d] = combine_leaves<LPP>(tmp);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) tmp[q] = ar[q];
    const T gr = combine_leaves<LPP>(tmp);
    if (r != 0) return;
    const int o = orig[k];
#pragma unroll
    for (int d = 0; d < DIM; ++d) cot.x[d][o] += gx[d];
    cot.rho[o] += gr;
}

// ---------------------------------------------------------------- particle shifting
//
// dr_i = -beta H^2 sum_j phi_ij V_j grad_i W_ij, phi = 1 + R (W_ij / W(dx))^4, R = 0.2 (the
// delta-plus form; a post-processing step on a state, x <- x + dr).  Same list traversal and
// partial sums as the sweeps; x is updated in original order.
constexpr double kShiftR = 0.2;

template <typename T, int DIM, int LPP>
__global__ __launch_bounds__(256) void k_shift(int64_t N, int32_t width, const int32_t* __restrict__ nbr,
                                               const int32_t* __restrict__ nbr_count,
                                               const vec4_t<T>* __restrict__ jd0, const int32_t* __restrict__ orig,
                                               const int32_t* __restrict__ psim,
                                               const SimConst<T>* __restrict__ sims, int filter, T beta,
                                               StatePtrs<T, DIM> state)
{
    constexpr int NQ = kLeaves / LPP;
    constexpr int U = kPairsInFlight;
    const int64_t t = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int64_t i = t / LPP;
    const int r = (int)(t - i * LPP);
    if (i >= N) return;
    const SimConst<T>& S = sims[psim[i]];
    const PairConst<T> c = pair_const(S);
    T ui[3] = {0, 0, 0};
    unpack_u<T, DIM>(jd0[i], ui);
    int n = nbr_count[i];
    n = n < width ? n : width;
    const int mcount = (n - r + LPP - 1) / LPP;
    const int32_t* row = nbr + i * (int64_t)width;
    T acc[NQ][3];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q][0] = acc[q][1] = acc[q][2] = T(0);
    int jn[U];
    load_entries<LPP, U>(row, r, 0, mcount, (int)i, jn);
    for (int m0 = 0; m0 < mcount; m0 += U) {
        vec4_t<T> a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = ldo(jd0, (uint32_t)jn[u]);
        load_entries<LPP, U>(row, r, m0 + U, mcount, (int)i, jn);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (m0 + u >= mcount) continue;
            T d[3] = {0, 0, 0};
            const T r2 = r2_exact<T, DIM>(ui, a[u], c.L, c.invL, d);
            if (filter && !(r2 < c.H2)) continue;
            const T q = fast_sqrt(r2) * c.invH;
            const T tt = T(1) - q;
            const T t2 = tt * tt;
            const T t4 = t2 * t2;
            const T gF = c.kG * (T(-56.0 / 3.0) * t4 * tt * (T(1) + T(5) * q));
            const T wr = S.kW * t4 * t2 * (T(1) + q * (T(6) + q * T(35.0 / 3.0))) * S.invW0;   // W / W(dx)
            const T w2 = wr * wr;
            const T phi = T(1) + T(kShiftR) * w2 * w2;
            const T f = phi * rec_volume<T, DIM>(a[u], S.m) * gF;
#pragma unroll
            for (int k = 0; k < DIM; ++k) acc[u % NQ][k] += f * d[k];
        }
    }
    T sum[3] = {0, 0, 0}, tmp[NQ];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) tmp[q] = acc[q][k];
        sum[k] = combine_leaves<LPP>(tmp);
    }
    if (r != 0) return;
    const int o = orig[i];
    const T cs = -beta * S.H2;
#pragma unroll
    for (int k = 0; k < DIM; ++k) state.x[k][o] += cs * sum[k];
}

// The position cotangents in sorted order, one record per particle, for k_shift_adj.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_pack_xbar(int64_t N, StatePtrs<T, DIM> cot, const int32_t* __restrict__ orig,
                                                   vec4_t<T>* __restrict__ xs)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int o = orig[k];
    vec4_t<T> a;
    a.x = cot.x[0][o];
    a.y = cot.x[1][o];
    a.z = (DIM == 3) ? cot.x[2][o] : T(0);
    a.w = T(0);
    xs[k] = a;
}

// Vector-Jacobian product of the shift for cotangents xb of the shifted positions (xs: xb in
// sorted order, one record per particle).  With D(e) = phi Jg + dphi (gF e)(gF e)^T the
// derivative of phi(e) grad W(e), dphi = 4 R (W / W(dx))^3 / W(dx), c = -beta H^2:
//   xbar_k += c sum_j D(e_kj) (V_j xb_k - V_k xb_j)
//   rbar_k += (V_k / rho_k) c sum_j phi gF (e_kj . xb_j)
// added to the cotangents (original order); velocities do not enter.
template <typename T, int DIM, int LPP>
__global__ __launch_bounds__(256) void k_shift_adj(int64_t N, int32_t width, const int32_t* __restrict__ nbr,
                                                   const int32_t* __restrict__ nbr_count,
                                                   const vec4_t<T>* __restrict__ jd0,
                                                   const vec4_t<T>* __restrict__ xs, const T* __restrict__ rho_s,
                                                   const int32_t* __restrict__ orig, const int32_t* __restrict__ psim,
                                                   const SimConst<T>* __restrict__ sims, int filter, T beta,
                                                   StatePtrs<T, DIM> cot)
{
    constexpr int NQ = kLeaves / LPP;
    constexpr int U = kPairsInFlight;
    const int64_t t = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int64_t k = t / LPP;
    const int r = (int)(t - k * LPP);
    if (k >= N) return;
    const SimConst<T>& S = sims[psim[k]];
    const PairConst<T> c = pair_const(S);
    const vec4_t<T> a0 = jd0[k];
    T uk[3] = {0, 0, 0};
    unpack_u<T, DIM>(a0, uk);
    const T Vk = rec_volume<T, DIM>(a0, S.m);
    const vec4_t<T> xk4 = xs[k];
    const T xbk[3] = {xk4.x, xk4.y, xk4.z};
    int n = nbr_count[k];
    n = n < width ? n : width;
    const int mcount = (n - r + LPP - 1) / LPP;
    const int32_t* row = nbr + k * (int64_t)width;
    T ax[NQ][3], ar[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) ax[q][0] = ax[q][1] = ax[q][2] = ar[q] = T(0);
    int jn[U];
    load_entries<LPP, U>(row, r, 0, mcount, (int)k, jn);
    for (int m0 = 0; m0 < mcount; m0 += U) {
        vec4_t<T> a[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            a[u] = ldo(jd0, (uint32_t)jn[u]);
            b[u] = ldo(xs, (uint32_t)jn[u]);
        }
        load_entries<LPP, U>(row, r, m0 + U, mcount, (int)k, jn);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (m0 + u >= mcount) continue;
            T e[3] = {0, 0, 0};
            const T r2 = r2_exact<T, DIM>(uk, a[u], c.L, c.invL, e);
            if (filter && !(r2 < c.H2)) continue;
            const T q = fast_sqrt(r2) * c.invH;
            const T tt = T(1) - q;
            const T t2 = tt * tt;
            const T t4 = t2 * t2;
            const T gF = c.kG * (T(-56.0 / 3.0) * t4 * tt * (T(1) + T(5) * q));
            const T hF = c.kH * t4;
            const T wr = S.kW * t4 * t2 * (T(1) + q * (T(6) + q * T(35.0 / 3.0))) * S.invW0;
            const T w2 = wr * wr;
            const T phi = T(1) + T(kShiftR) * w2 * w2;
            const T dphi = T(4.0 * kShiftR) * w2 * wr * S.invW0;
            const T Vj = rec_volume<T, DIM>(a[u], S.m);
            const T xbj[3] = {b[u].x, b[u].y, b[u].z};
            // z = V_j xb_k - V_k xb_j;  D z = phi (gF z + hF (e.z) e) + dphi gF^2 (e.z) e
            T z[3], ez = T(0), exj = T(0);
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                z[d] = Vj * xbk[d] - Vk * xbj[d];
                ez += e[d] * z[d];
                exj += e[d] * xbj[d];
            }
            const T ce = phi * hF * ez + dphi * gF * gF * ez;
#pragma unroll
            for (int d = 0; d < DIM; ++d) ax[u % NQ][d] += phi * gF * z[d] + ce * e[d];
            ar[u % NQ] += phi * gF * exj;
        }
    }
    T gx[3] = {0, 0, 0}, tmp[NQ];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) tmp[q] = ax[q][d];
        gx[d] = combine_leaves<LPP>(tmp);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) tmp[q] = ar[q];
    const T gr = combine_leaves<LPP>(tmp);
    if (r != 0) return;
    const int o = orig[k];
    const T cs = -beta * S.H2;
#pragma unroll
    for (int d = 0; d < DIM; ++d) cot.x[d][o] += cs * gx[d];
    cot.rho[o] += cs * (Vk / rho_s[k]) * gr;
}

// ---------------------------------------------------------------- neighbour export (CSR, original indices)

__global__ __launch_bounds__(256) void k_export_counts(int64_t N, const int32_t* __restrict__ orig,
                                                       const int32_t* __restrict__ nbr_count, int32_t width,
                                                       int64_t* __restrict__ rowcnt)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    int c = nbr_count[q];
    rowcnt[orig[q]] = c < width ? c : width;
}

// one wavefront per row: entries mapped to original indices and written in ascending order
// (each entry's rank in its row by comparison with every other entry of the row)
__global__ __launch_bounds__(64) void k_export_rows(int64_t N, int32_t width, const int32_t* __restrict__ orig,
                                                    const int32_t* __restrict__ nbr,
                                                    const int32_t* __restrict__ nbr_count,
                                                    const int64_t* __restrict__ offsets, int32_t* __restrict__ out)
{
    __shared__ int32_t row[1024];
    const int64_t q = (int64_t)xcd_remap(blockIdx.x, gridDim.x);
    if (q >= N) return;
    int c = nbr_count[q];
    c = c < width ? c : width;
    const int32_t* src = nbr + q * (int64_t)width;
    const int64_t base = offsets[orig[q]];
    for (int m0 = 0; m0 < c; m0 += 1024) {
        // rows longer than 1024 are handled by ranking each chunk against the full row
        const int mc = (c - m0 < 1024) ? c - m0 : 1024;
        for (int m = threadIdx.x; m < mc; m += 64) row[m] = orig[src[m0 + m]];
        __syncthreads();
        for (int m = threadIdx.x; m < mc; m += 64) {
            const int v = row[m];
            int rank = 0;
            for (int r2 = 0; r2 < c; ++r2) {
                const int w = (r2 >= m0 && r2 < m0 + mc) ? row[r2 - m0] : orig[src[r2]];
                rank += (w < v) ? 1 : 0;
            }
            out[base + rank] = v;
        }
        __syncthreads();
    }
}


// ---------------------------------------------------------------- per-particle support radii
//
// Neighbour search when every particle carries its own support h_i (Sec. 3.2, "Ensuring
// symmetric interactions"; App. B, the search-radius step).  A particle searching with its own
// support would miss partners whose larger support reaches it, so the search radius s_k
// starts at h_k and is raised by an integer atomic maximum on its bit pattern (positive IEEE
// values order like their bits) to h_i for every i that has k as a neighbour under h_i.  Each
// particle then searches with s_i and keeps the pairs with r_ij < max(h_i, h_j), a symmetric
// relation: if h_i >= h_j the pair lies within h_i <= s_i, else i is a neighbour of j under h_j
// and s_i >= h_j.  One thread per particle in sorted order, candidates from the stencil cells
// (the inner 3^dim when the radius fits half the list radius, on cells sized for that half),
// predicates with the arithmetic of the fixed-support search.  Supports must lie in (0, H].

constexpr int kFlagBadSupport = 8;  // a support outside (0, H] (status words of this search only)

// Stencil half-width a particle of search radius rad visits.
template <typename T>
__device__ __forceinline__ int reach_of(const SimConst<T>& S, T rad)
{
    return (S.sub == 2 && rad * rad <= T(0.25) * S.HL2) ? 1 : S.sub;
}

// Cell coordinates of a wrapped position, as the cell assignment computes them.
template <typename T, int DIM>
__device__ __forceinline__ void cell_of_u(const SimConst<T>& S, const T* u, int* cc)
{
    cc[0] = cell_coord(u[0], S.cinv, S.nc);
    cc[1] = cell_coord(u[1], S.cinv, S.nc);
    cc[2] = (DIM == 3) ? cell_coord(u[2], S.cinv, S.nc) : 0;
}

// Calls f(j, r2) for every particle j of the cells within `reach` of cell cc, in the canonical
// order (stencil offset lexicographic in z, y, x, then sorted order inside a cell).
template <typename T, int DIM, typename F>
__device__ __forceinline__ void for_each_candidate(const SimConst<T>& S, const int32_t* __restrict__ blk_rank,
                                                   const int32_t* __restrict__ cell_start,
                                                   const vec4_t<T>* __restrict__ jd0, const int* cc, const T* ui,
                                                   int reach, F&& f)
{
    const int sw = 2 * S.sub + 1;
    const int zr = (DIM == 3) ? reach : 0;
    for (int oz = -zr; oz <= zr; ++oz)
        for (int oy = -reach; oy <= reach; ++oy)
            for (int ox = -reach; ox <= reach; ++ox) {
                const int u = ((DIM == 3 ? (oz + S.sub) * sw : 0) + (oy + S.sub)) * sw + (ox + S.sub);
                const int code = stencil_entry<DIM>(S, blk_rank, cc, u);
                const int id = code & kStencilIdMask;
                T sh[3];
                sh[0] = T(((code >> kStencilIdBits) & 3) - 1) * S.L;
                sh[1] = T(((code >> (kStencilIdBits + 2)) & 3) - 1) * S.L;
                sh[2] = T(((code >> (kStencilIdBits + 4)) & 3) - 1) * S.L;
                const int j1 = cell_start[id + 1];
                for (int j = cell_start[id]; j < j1; ++j) {
                    T uj[3] = {T(0), T(0), T(0)};
                    unpack_u<T, DIM>(jd0[j], uj);
                    f(j, dist2_exact<T, DIM>(ui, uj, sh));
                }
            }
}

// s <- max(s, v) on the bits (v > 0).
__device__ __forceinline__ void raise_to(float* s, float v)
{
    atomicMax(reinterpret_cast<int*>(s), __float_as_int(v));
}
__device__ __forceinline__ void raise_to(double* s, double v)
{
    atomicMax(reinterpret_cast<unsigned long long*>(s), (unsigned long long)__double_as_longlong(v));
}

// Supports into sorted order, search radii initialised to them, supports checked.
template <typename T>
__global__ __launch_bounds__(256) void k_adapt_prepare(int64_t N, const T* __restrict__ h,
                                                       const int32_t* __restrict__ orig,
                                                       const int32_t* __restrict__ psim,
                                                       const SimConst<T>* __restrict__ sims, T* __restrict__ hs,
                                                       T* __restrict__ sr, int32_t* __restrict__ status)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const int s = psim[q];
    T v = h[orig[q]];
    if (!(v > T(0) && v <= sims[s].H)) {
        atomicOr(&status[s], kFlagBadSupport);
        v = sims[s].H;
    }
    hs[q] = v;
    sr[q] = v;
}

// Search radii: every k within h_i of particle i gets s_k >= h_i.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_adapt_radius(int64_t N, const vec4_t<T>* __restrict__ jd0,
                                                      const T* __restrict__ hs, T* __restrict__ sr,
                                                      const int32_t* __restrict__ cell_start,
                                                      const int32_t* __restrict__ psim,
                                                      const SimConst<T>* __restrict__ sims,
                                                      const int32_t* __restrict__ blk_rank)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const SimConst<T>& S = sims[psim[i]];
    T ui[3] = {T(0), T(0), T(0)};
    unpack_u<T, DIM>(jd0[i], ui);
    int cc[3];
    cell_of_u<T, DIM>(S, ui, cc);
    const T hi = hs[i];
    const T hi2 = hi * hi;
    for_each_candidate<T, DIM>(S, blk_rank, cell_start, jd0, cc, ui, reach_of(S, hi), [&](int j, T r2) {
        // only a partner with a smaller support can need its radius raised
        if (r2 < hi2 && hi > hs[j]) raise_to(sr + j, hi);
    });
}

// Lists: the search of radius s_i keeping r_ij < max(h_i, h_j), row-major (width entries per
// row), counts, overflow flagged.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_adapt_build(int64_t N, const vec4_t<T>* __restrict__ jd0,
                                                     const T* __restrict__ hs, const T* __restrict__ sr,
                                                     const int32_t* __restrict__ cell_start,
                                                     const int32_t* __restrict__ psim,
                                                     const SimConst<T>* __restrict__ sims,
                                                     const int32_t* __restrict__ blk_rank, int32_t width,
                                                     int32_t* __restrict__ nbr, int32_t* __restrict__ nbr_count,
                                                     int32_t* __restrict__ status)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int s = psim[i];
    const SimConst<T>& S = sims[s];
    T ui[3] = {T(0), T(0), T(0)};
    unpack_u<T, DIM>(jd0[i], ui);
    int cc[3];
    cell_of_u<T, DIM>(S, ui, cc);
    const T hi = hs[i];
    int32_t* row = nbr + i * (int64_t)width;
    int c = 0;
    for_each_candidate<T, DIM>(S, blk_rank, cell_start, jd0, cc, ui, reach_of(S, sr[i]), [&](int j, T r2) {
        const T hj = hs[j];
        const T hm = hi > hj ? hi : hj;
        const T hm2 = hm * hm;
        if (r2 < hm2) {
            if (c < width) row[c] = j;
            ++c;
        }
    });
    nbr_count[i] = c;
    if (c > width) atomicOr(&status[s], kFlagOverflow);
}

// Sorted-order values back to original order.
template <typename T>
__global__ __launch_bounds__(256) void k_scatter_orig(int64_t N, const T* __restrict__ in,
                                                      const int32_t* __restrict__ orig, T* __restrict__ out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < N) out[orig[q]] = in[q];
}

}  // namespace sph
