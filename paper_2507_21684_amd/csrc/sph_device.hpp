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
    int64_t p0, n;      // packed particle range
    int32_t cell0;      // first global cell slot
    int32_t blk0;       // first global cell block
    int32_t nc;         // cells per box side
    int32_t sub;        // stencil half-width in cells (cell side >= H / sub)
    int32_t B;          // cells per block side
    int32_t nb;         // blocks per box side
    int32_t Bd;         // B^dim
    int32_t pad;
};

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
    int bx = cx / S.B, by = cy / S.B, bz = (DIM == 3) ? cz / S.B : 0;
    int wx = cx - bx * S.B, wy = cy - by * S.B, wz = (DIM == 3) ? cz - bz * S.B : 0;
    int lin = (DIM == 3) ? ((bz * S.nb + by) * S.nb + bx) : (by * S.nb + bx);
    int rank = blk_rank[S.blk0 + lin];
    int w = (DIM == 3) ? ((wz * S.B + wy) * S.B + wx) : (wy * S.B + wx);
    return S.cell0 + rank * S.Bd + w;
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

template <typename I>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const I* __restrict__ in, int64_t n, I* __restrict__ part)
{
    __shared__ I smem[8];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    I s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += in[base + k];
    I tot;
    block_excl_scan<I>(s, smem, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// one workgroup: exclusive scan of part[0..np), part[np] = grand total
template <typename I>
__global__ __launch_bounds__(1024) void k_scan_top(I* __restrict__ part, int64_t np)
{
    __shared__ I smem[16];
    __shared__ I carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b = 0; b < np; b += blockDim.x) {
        int64_t i = b + threadIdx.x;
        I v = (i < np) ? part[i] : I(0);
        I tot;
        I ex = block_excl_scan<I>(v, smem, &tot);
        I c = carry;
        if (i < np) part[i] = c + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) part[np] = carry;
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
                                                      const SimConst<T>* __restrict__ sims)
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
    const T V = S.m / rho;
    const T pV = tait(S, rho) * V;
    vec4_t<T> a, b;
    if (DIM == 3) {
        a.x = u[0]; a.y = u[1]; a.z = u[2]; a.w = V;
        b.x = v[0]; b.y = v[1]; b.z = v[2]; b.w = pV;
    } else {
        a.x = u[0]; a.y = u[1]; a.z = V; a.w = pV;
        b.x = v[0]; b.y = v[1]; b.z = T(0); b.w = T(0);
    }
    jd0[d] = a;
    jd1[d] = b;
}

template <typename T, int DIM>
__device__ __forceinline__ void unpack_u(const vec4_t<T>& a, T* u)
{
    u[0] = a.x;
    u[1] = a.y;
    if (DIM == 3) u[2] = a.z;
}

// ---------------------------------------------------------------- neighbour lists

constexpr int kBuildTile = 512;  // candidates staged in LDS at a time

// One wavefront per cell block.  The block's particles (a contiguous sorted range) are tested
// against the union of their stencils, (B + 2 sub)^dim cells visited in lexicographic order of
// their offset from the block; candidate tiles are staged in LDS and read by all lanes at the
// same address.  Each lane appends its accepted neighbours to an ELL list (column-major, row
// stride `ld`), so each particle's list is ordered by stencil offset, then by original index.
template <typename T, int DIM>
__global__ __launch_bounds__(64) void k_build_list(const int32_t* __restrict__ blk_sim,
                                                   const int32_t* __restrict__ blk_coord,
                                                   const int32_t* __restrict__ blk_rank,
                                                   const SimConst<T>* __restrict__ sims,
                                                   const int32_t* __restrict__ cell_start,
                                                   const vec4_t<T>* __restrict__ jd0, int64_t ld, int32_t maxnbr,
                                                   int32_t* __restrict__ nbr, int32_t* __restrict__ nbr_count,
                                                   int32_t* __restrict__ status)
{
    __shared__ T su[DIM][kBuildTile];
    __shared__ T ssh[DIM][kBuildTile];
    __shared__ int32_t sj[kBuildTile];
    __shared__ int32_t uc_first[64];
    __shared__ int32_t uc_pref[65];
    __shared__ T uc_shift[DIM][64];

    const int gb = xcd_remap(blockIdx.x, gridDim.x);
    const int s = blk_sim[gb];
    const SimConst<T> S = sims[s];
    const int coord = blk_coord[gb];
    const int bc[3] = {coord & 1023, (coord >> 10) & 1023, (coord >> 20) & 1023};
    const int B = S.B, sub = S.sub, nc = S.nc;
    const int W = B + 2 * sub;
    const int ncu = (DIM == 3) ? W * W * W : W * W;
    const int cfirst = S.cell0 + (gb - S.blk0) * S.Bd;
    const int i0 = cell_start[cfirst], i1 = cell_start[cfirst + S.Bd];
    const int lane = threadIdx.x;

    for (int ib = i0; ib < i1; ib += 64) {
        const int i = ib + lane;
        const bool act = i < i1;
        T ui[3] = {0, 0, 0};
        if (act) unpack_u<T, DIM>(jd0[i], ui);
        int cnt = 0;
        for (int cu0 = 0; cu0 < ncu; cu0 += 64) {
            // lane's union cell: its particle range and periodic image shift
            const int cu = cu0 + lane;
            int first = 0, count = 0;
            T sh[3] = {0, 0, 0};
            if (cu < ncu) {
                int o[3] = {cu % W, (cu / W) % W, (DIM == 3) ? cu / (W * W) : 0};
                int cc[3] = {0, 0, 0};
#pragma unroll
                for (int k = 0; k < DIM; ++k) {
                    int r = bc[k] * B + o[k] - sub;
                    if (r < 0) {
                        r += nc;
                        sh[k] = -S.L;
                    } else if (r >= nc) {
                        r -= nc;
                        sh[k] = S.L;
                    }
                    cc[k] = r;
                }
                const int gc = global_cell<T, DIM>(S, blk_rank, cc[0], cc[1], cc[2]);
                first = cell_start[gc];
                count = cell_start[gc + 1] - first;
            }
            const int inc = wave_incl_scan(count);
            const int tot = __shfl(inc, 63, 64);
            __syncthreads();
            uc_first[lane] = first;
            uc_pref[lane] = inc - count;
            if (lane == 63) uc_pref[64] = inc;
#pragma unroll
            for (int k = 0; k < DIM; ++k) uc_shift[k][lane] = sh[k];
            __syncthreads();
            for (int m0 = 0; m0 < tot; m0 += kBuildTile) {
                const int mt = (tot - m0 < kBuildTile) ? tot - m0 : kBuildTile;
                for (int m = lane; m < mt; m += 64) {
                    const int gm = m0 + m;
                    int lo = 0, hi = 63;  // last union cell whose prefix is <= gm
                    while (lo < hi) {
                        int mid = (lo + hi + 1) >> 1;
                        if (uc_pref[mid] <= gm) lo = mid;
                        else hi = mid - 1;
                    }
                    const int j = uc_first[lo] + (gm - uc_pref[lo]);
                    T uj[3] = {0, 0, 0};
                    unpack_u<T, DIM>(jd0[j], uj);
#pragma unroll
                    for (int k = 0; k < DIM; ++k) {
                        su[k][m] = uj[k];
                        ssh[k][m] = uc_shift[k][lo];
                    }
                    sj[m] = j;
                }
                __syncthreads();
                if (act) {
                    for (int m = 0; m < mt; ++m) {
                        T uj[3], sh2[3];
#pragma unroll
                        for (int k = 0; k < DIM; ++k) {
                            uj[k] = su[k][m];
                            sh2[k] = ssh[k][m];
                        }
                        const T r2 = dist2_exact<T, DIM>(ui, uj, sh2);
                        if (r2 < S.H2) {
                            if (cnt < maxnbr) nbr[(int64_t)cnt * ld + i] = sj[m];
                            ++cnt;
                        }
                    }
                }
                __syncthreads();
            }
        }
        if (act) {
            nbr_count[i] = cnt;
            if (cnt > maxnbr) atomicOr(&status[s], kFlagOverflow);
        }
    }
}

// ---------------------------------------------------------------- forward sweep

constexpr int kModeStep = 0;  // integrate into dst (sorted order)
constexpr int kModeRhs = 1;   // write drho, a, rho_sum to caller arrays (original order)

template <typename T, int DIM, int MODE>
__global__ __launch_bounds__(256) void k_sweep(int64_t N, int64_t ld, int32_t maxnbr, const int32_t* __restrict__ nbr,
                                               const int32_t* __restrict__ nbr_count,
                                               const vec4_t<T>* __restrict__ jd0, const vec4_t<T>* __restrict__ jd1,
                                               StatePtrs<T, DIM> cur, StatePtrs<T, DIM> dst,
                                               const int32_t* __restrict__ orig, T* __restrict__ drho_out,
                                               T* __restrict__ acc_out, T* __restrict__ rhosum_out,
                                               const int32_t* __restrict__ psim,
                                               const SimConst<T>* __restrict__ sims, int32_t* __restrict__ status)
{
    const int64_t i = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int s = psim[i];
    const SimConst<T>& S = sims[s];
    T ui[3] = {0, 0, 0}, vi[3] = {0, 0, 0};
    unpack_u<T, DIM>(jd0[i], ui);
#pragma unroll
    for (int k = 0; k < DIM; ++k) vi[k] = cur.v[k][i];
    const T rhoi = cur.rho[i];
    const T pi = tait(S, rhoi);
    const T L = S.L, invL = S.invL, invH = S.invH, kG = S.kG, epsH2 = S.epsH2, cA = S.cA;
    int n = nbr_count[i];
    n = n < maxnbr ? n : maxnbr;
    T ax[3] = {0, 0, 0};
    T rdv = 0, rdd = 0, rs = 0;
    for (int k = 0; k < n; ++k) {
        const int j = nbr[(int64_t)k * ld + i];
        const vec4_t<T> a = jd0[j];
        const vec4_t<T> b = jd1[j];
        const T rhoj = cur.rho[j];
        T uj[3], vj[3], d[3];
        T Vj, pVj;
        if (DIM == 3) {
            uj[0] = a.x; uj[1] = a.y; uj[2] = a.z; Vj = a.w;
            vj[0] = b.x; vj[1] = b.y; vj[2] = b.z; pVj = b.w;
        } else {
            uj[0] = a.x; uj[1] = a.y; Vj = a.z; pVj = a.w;
            vj[0] = b.x; vj[1] = b.y;
        }
        T r2 = 0, ue = 0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            T dd = ui[c] - uj[c];
            dd -= L * rint(dd * invL);
            d[c] = dd;
            r2 += dd * dd;
            ue += (vi[c] - vj[c]) * dd;
        }
        const T q = sqrt(r2) * invH;
        const T t = T(1) - q;
        const T t2 = t * t;
        const T t4 = t2 * t2;
        const T t5 = t4 * t;
        const T gF = kG * (T(-56.0 / 3.0) * t5 * (T(1) + T(5) * q));  // grad W = gF x_ij
        const T inv = T(1) / (r2 + epsH2);
        const T pij = ue * inv;                                        // pi_ij
        const T cg = ((cA * pij - pi) * Vj - pVj) * gF;
#pragma unroll
        for (int c = 0; c < DIM; ++c) ax[c] += cg * d[c];
        rdv += Vj * (gF * ue);                                         // V_j (v_i - v_j).gW
        rdd += Vj * (rhoi - rhoj) * (gF * r2 * inv);                   // V_j (rho_i - rho_j) x_ij.gW / (r^2+eps H^2)
        if (MODE == kModeRhs) rs += t4 * t2 * (T(1) + q * (T(6) + q * T(35.0 / 3.0)));
    }
    const T invrho = T(1) / rhoi;
    T acc[3];
#pragma unroll
    for (int c = 0; c < DIM; ++c) acc[c] = ax[c] * invrho;
    const T drho = rhoi * rdv + S.cD * rdd;
    if (MODE == kModeStep) {
        bool bad = !isfinite(drho);
        const T dt = S.dt;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const T vn = vi[c] + dt * acc[c];
            const T xn = cur.x[c][i] + dt * vn;
            dst.v[c][i] = vn;
            dst.x[c][i] = xn;
            bad = bad || !isfinite(vn) || !isfinite(xn);
        }
        dst.rho[i] = rhoi + dt * drho;
        if (bad) atomicOr(&status[s], kFlagNonfinite);
    } else {
        const int o = orig[i];
        drho_out[o] = drho;
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc_out[(int64_t)c * N + o] = acc[c];
        if (rhosum_out) rhosum_out[o] = S.m * S.kW * rs;
    }
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

// Gathers the output cotangents into sorted order: jdA = (abar, rbar) with
// vt = v'_bar + dt x'_bar, abar = dt vt, rbar = dt rho'_bar; jdB = (rho, p, 1/rho, dp/drho).
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_adj_prologue(int64_t N, const int32_t* __restrict__ orig,
                                                      StatePtrs<T, DIM> cot, StatePtrs<T, DIM> cur,
                                                      vec4_t<T>* __restrict__ jdA, vec4_t<T>* __restrict__ jdB,
                                                      const int32_t* __restrict__ psim,
                                                      const SimConst<T>* __restrict__ sims)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const SimConst<T>& S = sims[psim[q]];
    const int o = orig[q];
    T ab[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < DIM; ++k) ab[k] = S.dt * (cot.v[k][o] + S.dt * cot.x[k][o]);
    const T rb = S.dt * cot.rho[o];
    vec4_t<T> a;
    if (DIM == 3) {
        a.x = ab[0]; a.y = ab[1]; a.z = ab[2]; a.w = rb;
    } else {
        a.x = ab[0]; a.y = ab[1]; a.z = rb; a.w = T(0);
    }
    jdA[q] = a;
    const T rho = cur.rho[q];
    vec4_t<T> b;
    b.x = rho;
    b.y = tait(S, rho);
    b.z = T(1) / rho;
    b.w = tait_slope(S, rho);
    jdB[q] = b;
}

// Adjoint sweep, gather form.  For particle k and each neighbour j != k it adds the partial
// derivatives, with respect to k's position, velocity and density, of the two directed pair
// terms (k,j) and (j,k) contracted with their particles' cotangents (abar, rbar).  With
// e = x_kj, G = gF e, the kernel Hessian Jg = gF I + hF e e^T, pi = (v_k - v_j).e / (r^2+eps H^2),
// s = e.G / (r^2+eps H^2), these partials reduce to the closed forms below.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_adj_sweep(int64_t N, int64_t ld, int32_t maxnbr,
                                                   const int32_t* __restrict__ nbr,
                                                   const int32_t* __restrict__ nbr_count,
                                                   const vec4_t<T>* __restrict__ jd0,
                                                   const vec4_t<T>* __restrict__ jd1,
                                                   const vec4_t<T>* __restrict__ jdA,
                                                   const vec4_t<T>* __restrict__ jdB,
                                                   const int32_t* __restrict__ orig, StatePtrs<T, DIM> cot,
                                                   const int32_t* __restrict__ psim,
                                                   const SimConst<T>* __restrict__ sims, int32_t* __restrict__ status)
{
    const int64_t k = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int s = psim[k];
    const SimConst<T>& S = sims[s];
    const T L = S.L, invL = S.invL, invH = S.invH, kG = S.kG, kH = S.kH, epsH2 = S.epsH2, cA = S.cA, cD = S.cD;
    T uk[3] = {0, 0, 0}, vk[3] = {0, 0, 0}, ak[3] = {0, 0, 0};
    T Vk, rbk;
    {
        const vec4_t<T> a = jd0[k], b = jd1[k], A = jdA[k];
        if (DIM == 3) {
            uk[0] = a.x; uk[1] = a.y; uk[2] = a.z; Vk = a.w;
            vk[0] = b.x; vk[1] = b.y; vk[2] = b.z;
            ak[0] = A.x; ak[1] = A.y; ak[2] = A.z; rbk = A.w;
        } else {
            uk[0] = a.x; uk[1] = a.y; Vk = a.z;
            vk[0] = b.x; vk[1] = b.y;
            ak[0] = A.x; ak[1] = A.y; rbk = A.z;
        }
    }
    const vec4_t<T> Bk = jdB[k];
    const T rhok = Bk.x, pk = Bk.y, irk = Bk.z, dpk = Bk.w;
    T gx[3] = {0, 0, 0}, gv[3] = {0, 0, 0};
    T gr = 0;
    int n = nbr_count[k];
    n = n < maxnbr ? n : maxnbr;
    for (int m = 0; m < n; ++m) {
        const int j = nbr[(int64_t)m * ld + k];
        const vec4_t<T> a = jd0[j], b = jd1[j], A = jdA[j], Bj = jdB[j];
        T uj[3], vj[3], aj[3];
        T Vj, rbj;
        if (DIM == 3) {
            uj[0] = a.x; uj[1] = a.y; uj[2] = a.z; Vj = a.w;
            vj[0] = b.x; vj[1] = b.y; vj[2] = b.z;
            aj[0] = A.x; aj[1] = A.y; aj[2] = A.z; rbj = A.w;
        } else {
            uj[0] = a.x; uj[1] = a.y; Vj = a.z;
            vj[0] = b.x; vj[1] = b.y;
            aj[0] = A.x; aj[1] = A.y; rbj = A.z;
        }
        const T rhoj = Bj.x, pj = Bj.y, irj = Bj.z;
        T e[3], u[3];
        T r2 = 0, ue = 0, ake = 0, aje = 0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            T dd = uk[c] - uj[c];
            dd -= L * rint(dd * invL);
            e[c] = dd;
            u[c] = vk[c] - vj[c];
            r2 += dd * dd;
            ue += u[c] * dd;
            ake += ak[c] * dd;
            aje += aj[c] * dd;
        }
        const T q = sqrt(r2) * invH;
        const T t = T(1) - q;
        const T t2 = t * t;
        const T t4 = t2 * t2;
        const T gF = kG * (T(-56.0 / 3.0) * t4 * t * (T(1) + T(5) * q));  // grad W = gF e
        const T hF = kH * t4;                                              // Hessian: gF I + hF e e^T
        const T inv = T(1) / (r2 + epsH2);
        const T pij = ue * inv;
        const T sij = gF * r2 * inv;
        const T sig = inv * (T(2) * gF + hF * r2 - T(2) * sij);            // d s / d e = sig e
        const T aGk = gF * ake, aGj = gF * aje, uG = gF * ue;
        const T Qk = (cA * pij - pk - pj) * irk;
        const T Qj = (cA * pij - pj - pk) * irj;
        const T beta = cA * inv * (Vj * aGk * irk - Vk * aGj * irj);
        const T gam = Vj * rbk * rhok + Vk * rbj * rhoj;
        const T cdr = cD * sig * (rhok - rhoj) * (Vj * rbk - Vk * rbj);
        T w[3];
        T ew = 0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            w[c] = Vj * Qk * ak[c] - Vk * Qj * aj[c] + gam * u[c];
            ew += e[c] * w[c];
        }
        const T hew = hF * ew;
        const T ce = cdr - T(2) * beta * pij + hew;   // coefficient of e in the position cotangent
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            gx[c] += beta * u[c] + ce * e[c] + gF * w[c];
            gv[c] += (beta + gam * gF) * e[c];
        }
        const T phi2 = Vk * (-Qj * aGj + rbj * rhoj * uG + rbj * cD * (rhoj - rhok) * sij);
        gr += Vj * (aGk * (-dpk - Qk) * irk + rbk * uG + rbk * cD * sij) - phi2 * irk +
              Vk * (aGj * dpk * irj - rbj * cD * sij);
    }
    const int o = orig[k];
    const T dt = S.dt;
    bool bad = !isfinite(gr);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        const T xb = cot.x[c][o];
        const T vb = cot.v[c][o];
        cot.x[c][o] = xb + gx[c];
        cot.v[c][o] = vb + dt * xb + gv[c];
        bad = bad || !isfinite(gx[c]) || !isfinite(gv[c]);
    }
    cot.rho[o] = cot.rho[o] + gr;
    if (bad) atomicOr(&status[s], kFlagNonfinite);
}

// ---------------------------------------------------------------- neighbour export (CSR, original indices)

__global__ __launch_bounds__(256) void k_export_counts(int64_t N, const int32_t* __restrict__ orig,
                                                       const int32_t* __restrict__ nbr_count, int32_t maxnbr,
                                                       int64_t* __restrict__ rowcnt)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    int c = nbr_count[q];
    rowcnt[orig[q]] = c < maxnbr ? c : maxnbr;
}

// one wavefront per row: entries mapped to original indices and written in ascending order
// (each entry's rank in its row by comparison with every other entry of the row)
__global__ __launch_bounds__(64) void k_export_rows(int64_t N, int64_t ld, const int32_t* __restrict__ orig,
                                                    const int32_t* __restrict__ nbr,
                                                    const int32_t* __restrict__ nbr_count, int32_t maxnbr,
                                                    const int64_t* __restrict__ offsets, int32_t* __restrict__ out)
{
    __shared__ int32_t row[1024];
    const int64_t q = (int64_t)xcd_remap(blockIdx.x, gridDim.x);
    if (q >= N) return;
    int c = nbr_count[q];
    c = c < maxnbr ? c : maxnbr;
    const int64_t base = offsets[orig[q]];
    for (int m0 = 0; m0 < c; m0 += 1024) {
        // rows longer than 1024 are handled by ranking each chunk against the full row
        const int mc = (c - m0 < 1024) ? c - m0 : 1024;
        for (int m = threadIdx.x; m < mc; m += 64) row[m] = orig[nbr[(int64_t)(m0 + m) * ld + q]];
        __syncthreads();
        for (int m = threadIdx.x; m < mc; m += 64) {
            const int v = row[m];
            int rank = 0;
            for (int r = 0; r < c; ++r) {
                const int w = (r >= m0 && r < m0 + mc) ? row[r - m0] : orig[nbr[(int64_t)r * ld + q]];
                rank += (w < v) ? 1 : 0;
            }
            out[base + rank] = v;
        }
        __syncthreads();
    }
}

}  // namespace sph
