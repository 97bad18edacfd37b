/*
 * sph_oracle.c -- plain, slow, double-precision CPU oracle for the weakly
 * compressible delta-SPH hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so and is
 * loaded by the test-suite, by the smoke check and by the CPU-baseline leg of
 * the benchmark.  The GPU library never links, loads or calls it, and it
 * shares no code, header, table or helper with the GPU library.
 *
 * What it computes, and where the paper defines it (diffSPH, arXiv 2507.21684):
 *   - Wendland-C4 kernel W(r,H) = C_d/H^d w(q), q = |r|/H, with
 *     w(q) = (1-q)^6_+ (1 + 6q + 35/3 q^2), C_2 = 9/pi, C_3 = 495/(32 pi)
 *     (App. A.1, kernel definition and Wendland-4 equation); its gradient
 *     r_hat C_d/H^(d+1) w'(q) (App. A.1, gradient equation) and its Hessian,
 *     the zero-epsilon limit of the regularised Hessian of Sec. 3.3.
 *   - Periodic domain: particles keep unwrapped positions; positions are
 *     mapped into the box with modulo arithmetic and pair vectors use the
 *     minimum image (Sec. 3.2 "Periodic Boundary Conditions", App. B).
 *   - Neighbour set N(i) = { j : |x_ij| < H }, self included, found with a
 *     bucket grid of cells of side >= H and a 3^d cell query (App. B,
 *     three-step procedure); a brute-force O(N^2) mode is kept for checks
 *     (Sec. 4.1, the "small"/"naive" searches).
 *   - Summation density rho_i = sum_j m_j W_ij (Sec. 2.3 eq. for rho_i,
 *     App. A.2).
 *   - Continuity with the difference divergence, Omega = 1 for a fixed
 *     support: drho_i/dt = -rho_i sum_j V_j (v_j - v_i).grad_i W_ij
 *     (Sec. 2.3 continuity equation, App. A.3 difference form).
 *   - delta-SPH density diffusion (cited in Sec. 2.3, not printed):
 *     delta H c0 sum_j V_j 2 (rho_j - rho_i) (x_ji . grad_i W_ij)/(r^2+eps H^2).
 *   - Tait equation of state p = rho0 c0^2/7 ((rho/rho0)^7 - 1) (Sec. 2.3).
 *   - Momentum: pressure with the summation gradient form
 *     -(1/rho_i) sum_j V_j (p_i + p_j) grad_i W_ij (App. A.3 summation form,
 *     the weakly compressible choice of Sec. 2.3) plus artificial viscosity
 *     alpha H c0 (rho0/rho_i) sum_j V_j pi_ij grad_i W_ij with
 *     pi_ij = (v_i - v_j).x_ij/(r^2 + eps H^2) (Sec. 2.3 dissipation
 *     equation, pairwise quantity of App. A.4).
 *   - Semi-implicit Euler with fixed dt (Sec. 3.4): v' = v + dt a,
 *     rho' = rho + dt drho/dt, x' = x + dt v'.
 *   - The adjoint: the exact vector-Jacobian product (dP/du)^T a of one step
 *     (Sec. 2.2), formed pair by pair from the partial derivatives of each
 *     directed pair's contribution, the neighbour list held fixed (Sec. 3.2
 *     "Differentiability").
 *
 *   - The vector-Jacobian product of the summation density alone (the
 *     backward benchmark of Sec. 4.1: summation density after a step,
 *     gradient with respect to the initial positions).
 *   - Explicit particle shifting as a post-processing step (Sec. 3.4,
 *     App. C; the delta-plus form) and its vector-Jacobian product.
 *   - DualSPHysics' symplectic Euler (Sec. 3.4, App. C), optionally with
 *     the last substep's rates re-used as the next step's first substep,
 *     and its vector-Jacobian products for one step and for a rollout.
 *   - Explicit Runge-Kutta steps from a Butcher tableau (Sec. 3.4, the
 *     multistage integrators) and their vector-Jacobian products.
 *   - Neighbour search with per-particle support radii h_i: a search radius
 *     s_k = max(h_k, max{h_i : |x_ik| < h_i}) (the atomic-maximum step), then
 *     the super-symmetric set |x_ij| < max(h_i, h_j) found by searching with s_i
 *     (Sec. 3.2 "Ensuring symmetric interactions", App. B).
 *   - The full delta-SPH diffusion with the renormalised density gradient
 *     <grad rho>_i = L_i sum_j V_j (rho_j - rho_i) grad_i W_ij,
 *     L_i = [sum_j V_j (x_j - x_i) (x) grad_i W_ij]^-1 (App. A.5, renormalised
 *     gradient; Sec. 2.3 cites the scheme), and its vector-Jacobian product.
 *
 * Readings taken where the paper is silent or garbled are listed in the
 * project's design notes; the ones that change arithmetic are: the minus
 * signs of the continuity and pressure terms, H (the support) in
 * delta H c0 and alpha H c0, eps = 0.01 in (r^2 + eps H^2), and the strict
 * r < H neighbour predicate evaluated in the working precision.  The time
 * step is an input (the callers pass dt = 0.25 h / c0 with h = H / 2).
 *
 * Layout: positions, velocities are SoA rows, x[k*n + i] for coordinate k.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

typedef struct {
    int32_t dim;    /* 2 or 3 */
    int32_t renorm; /* 1: delta-diffusion with the renormalised density gradient */
    double L;       /* periodic box side */
    double H;       /* kernel support radius */
    double m;       /* particle mass */
    double rho0;    /* rest density */
    double c0;      /* speed of sound */
    double delta;   /* delta-SPH diffusion coefficient */
    double alpha;   /* artificial viscosity coefficient */
    double eps;     /* regulariser in 1/(r^2 + eps H^2) */
    double dt;      /* fixed time step */
} orc_params;

/* ------------------------------------------------------------------ */
/* Wendland-C4 kernel (App. A.1)                                        */
/* ------------------------------------------------------------------ */

double orc_cd(int dim)
{
    if (dim == 2) return 9.0 / ORC_PI;
    if (dim == 3) return 495.0 / (32.0 * ORC_PI);
    return 0.0;
}

/* w(q) = (1-q)^6 (1 + 6q + 35/3 q^2) for q < 1, else 0 */
double orc_what(double q)
{
    if (q >= 1.0) return 0.0;
    double t = 1.0 - q;
    double t2 = t * t;
    double t6 = t2 * t2 * t2;
    return t6 * (1.0 + 6.0 * q + (35.0 / 3.0) * q * q);
}

/* dw/dq = -(56/3) q (1-q)^5 (1 + 5q) */
double orc_what_d1(double q)
{
    if (q >= 1.0) return 0.0;
    double t = 1.0 - q;
    double t5 = t * t * t * t * t;
    return -(56.0 / 3.0) * q * t5 * (1.0 + 5.0 * q);
}

/* d2w/dq2 = -(56/3) (1-q)^4 (1 + 4q - 35 q^2) */
double orc_what_d2(double q)
{
    if (q >= 1.0) return 0.0;
    double t = 1.0 - q;
    double t4 = t * t * t * t;
    return -(56.0 / 3.0) * t4 * (1.0 + 4.0 * q - 35.0 * q * q);
}

static double powi(double b, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

/* W(r, H) = C_d / H^d w(|r|/H) */
double orc_w(int dim, double H, const double* e)
{
    double r2 = 0.0;
    for (int k = 0; k < dim; ++k) r2 += e[k] * e[k];
    double q = sqrt(r2) / H;
    return orc_cd(dim) / powi(H, dim) * orc_what(q);
}

/* grad W = r_hat C_d/H^(d+1) w'(q); zero at r = 0 */
void orc_gradw(int dim, double H, const double* e, double* g)
{
    double r2 = 0.0;
    for (int k = 0; k < dim; ++k) r2 += e[k] * e[k];
    double r = sqrt(r2);
    for (int k = 0; k < dim; ++k) g[k] = 0.0;
    if (r == 0.0) return;
    double mag = orc_cd(dim) / powi(H, dim + 1) * orc_what_d1(r / H);
    for (int k = 0; k < dim; ++k) g[k] = e[k] / r * mag;
}

/* Hessian of W for r > 0: the radial-function Hessian
 *   C_d/H^(d+2) w''(q) r_hat r_hat^T + C_d/H^(d+1) w'(q)/r (I - r_hat r_hat^T),
 * i.e. the eps -> 0 limit of the regularised form of Sec. 3.3.  At r = 0 the
 * limit of both terms is C_d/H^(d+2) w''(0) I (w'(q)/q -> w''(0)). */
void orc_hessw(int dim, double H, const double* e, double* hess /* dim*dim */)
{
    double r2 = 0.0;
    for (int k = 0; k < dim; ++k) r2 += e[k] * e[k];
    double r = sqrt(r2);
    double c1 = orc_cd(dim) / powi(H, dim + 1);
    double c2 = orc_cd(dim) / powi(H, dim + 2);
    if (r == 0.0) {
        for (int a = 0; a < dim; ++a)
            for (int b = 0; b < dim; ++b)
                hess[a * dim + b] = (a == b) ? c2 * orc_what_d2(0.0) : 0.0;
        return;
    }
    double q = r / H;
    double d1 = c1 * orc_what_d1(q);
    double d2 = c2 * orc_what_d2(q);
    for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b) {
            double rr = e[a] / r * e[b] / r;
            double id = (a == b) ? 1.0 : 0.0;
            hess[a * dim + b] = d2 * rr + d1 / r * (id - rr);
        }
}

/* ------------------------------------------------------------------ */
/* Periodic mapping and the neighbour predicate (Sec. 3.2, App. B)      */
/* ------------------------------------------------------------------ */

/* Position mapped into [0, L): u = x - L floor(x / L), computed as
 * x - L * floor(x * (1/L)) with 1/L rounded once. */
static double wrap_f64(double x, double L, double invL)
{
    return x - L * floor(x * invL);
}

static float wrap_f32(float x, float L, float invL)
{
    float k = floorf(x * invL);
    float s = L * k;
    return x - s;
}

/* Strict r^2 < H^2 test on wrapped positions, minimum image per component:
 *   d = u_i - u_j;  d = d - L * rint(d * (1/L));  r2 = ((d0 d0) + d1 d1) + d2 d2
 * every product and sum rounded in the working precision (the file is built
 * with -ffp-contract=off, so no fused multiply-add is formed). */
static int within_f64(int dim, const double* ui, const double* uj, double L, double invL, double H2)
{
    double r2 = 0.0;
    for (int k = 0; k < dim; ++k) {
        double d = ui[k] - uj[k];
        double s = L * rint(d * invL);
        d = d - s;
        double dd = d * d;
        r2 = r2 + dd;
    }
    return r2 < H2;
}

static int within_f32(int dim, const float* ui, const float* uj, float L, float invL, float H2)
{
    float r2 = 0.0f;
    for (int k = 0; k < dim; ++k) {
        float d = ui[k] - uj[k];
        float s = L * rintf(d * invL);
        d = d - s;
        float dd = d * d;
        r2 = r2 + dd;
    }
    return r2 < H2;
}

/* minimum-image pair vector x_ij = x_i - x_j in double, from wrapped positions */
static void minimg(int dim, const double* ui, const double* uj, double L, double invL, double* e)
{
    for (int k = 0; k < dim; ++k) {
        double d = ui[k] - uj[k];
        e[k] = d - L * rint(d * invL);
    }
}

/* ------------------------------------------------------------------ */
/* Neighbour lists                                                      */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    int64_t* off;   /* n + 1 */
    int32_t* idx;   /* off[n] entries, each row ascending, self included */
} nblist;

static void nblist_free(nblist* nb)
{
    free(nb->off);
    free(nb->idx);
    nb->off = NULL;
    nb->idx = NULL;
}

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* Candidate iteration: either all particles (brute force) or the 3^d cells
 * around particle i in a bucket grid of side >= 1.01 H. */
typedef struct {
    int dim, nc, brute;
    int64_t n;
    int64_t* cstart;  /* nc^dim + 1 */
    int32_t* cmem;    /* members, grouped by cell */
    int32_t* cell3;   /* per particle: cell coordinate triplet */
} grid;

static void grid_build(grid* g, int dim, int64_t n, const double* u /* dim*n */, double L, double H, int brute)
{
    memset(g, 0, sizeof(*g));
    g->dim = dim;
    g->n = n;
    int nc = (int)floor(L / (1.01 * H));
    g->brute = brute || nc < 3;
    g->nc = nc;
    if (g->brute) return;
    int64_t ncell = 1;
    for (int k = 0; k < dim; ++k) ncell *= nc;
    g->cstart = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
    g->cmem = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    g->cell3 = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)(n > 0 ? n : 1));
    int64_t* cid = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        int64_t id = 0;
        for (int k = dim - 1; k >= 0; --k) {
            int c = (int)floor(u[k * n + i] / L * nc);
            if (c < 0) c = 0;
            if (c > nc - 1) c = nc - 1;
            g->cell3[3 * i + k] = c;
            id = id * nc + c;
        }
        cid[i] = id;
        g->cstart[id + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c) g->cstart[c + 1] += g->cstart[c];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)ncell);
    for (int64_t c = 0; c < ncell; ++c) fill[c] = g->cstart[c];
    for (int64_t i = 0; i < n; ++i) g->cmem[fill[cid[i]]++] = (int32_t)i;
    free(fill);
    free(cid);
}

static void grid_free(grid* g)
{
    free(g->cstart);
    free(g->cmem);
    free(g->cell3);
}

/* Collect the candidate list of particle i into buf (capacity n); returns count. */
static int64_t grid_candidates(const grid* g, int64_t i, int32_t* buf)
{
    if (g->brute) {
        for (int64_t j = 0; j < g->n; ++j) buf[j] = (int32_t)j;
        return g->n;
    }
    int dim = g->dim, nc = g->nc;
    int64_t cnt = 0;
    int dz_lo = (dim == 3) ? -1 : 0, dz_hi = (dim == 3) ? 1 : 0;
    for (int dz = dz_lo; dz <= dz_hi; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int c[3] = {g->cell3[3 * i + 0] + dx, g->cell3[3 * i + 1] + dy, 0};
                if (dim == 3) c[2] = g->cell3[3 * i + 2] + dz;
                int64_t id = 0;
                for (int k = dim - 1; k >= 0; --k) {
                    int ck = ((c[k] % nc) + nc) % nc;
                    id = id * nc + ck;
                }
                for (int64_t p = g->cstart[id]; p < g->cstart[id + 1]; ++p) buf[cnt++] = g->cmem[p];
            }
    return cnt;
}

/* Build neighbour lists.  prec: 0 = predicate in double, 1 = in float (the
 * positions are then first rounded to float).  Rows ascending, self included. */
static int build_lists(int dim, int64_t n, const double* x, double L, double H, int prec, int brute, nblist* out)
{
    out->n = n;
    out->off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    out->idx = NULL;
    double* u = (double*)malloc(sizeof(double) * (size_t)dim * (size_t)(n > 0 ? n : 1));
    float* uf = (float*)malloc(sizeof(float) * (size_t)dim * (size_t)(n > 0 ? n : 1));
    double invL = 1.0 / L;
    float Lf = (float)L, invLf = 1.0f / Lf;
    float Hf = (float)H;
    float H2f = Hf * Hf;
    double H2 = H * H;
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < dim; ++k) {
            if (prec == 1) {
                uf[k * n + i] = wrap_f32((float)x[k * n + i], Lf, invLf);
                u[k * n + i] = (double)uf[k * n + i];
            } else {
                u[k * n + i] = wrap_f64(x[k * n + i], L, invL);
            }
        }
    grid g;
    grid_build(&g, dim, n, u, L, H, brute);
    int64_t* cnt = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    int err = 0;
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            for (int64_t i = 0; i < n; ++i) out->off[i + 1] = out->off[i] + cnt[i];
            out->idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(out->off[n] > 0 ? out->off[n] : 1));
        }
#pragma omp parallel
        {
            int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 64)
            for (int64_t i = 0; i < n; ++i) {
                int64_t nc = grid_candidates(&g, i, buf);
                int64_t c = 0;
                double ui[3], uj[3];
                float fi[3], fj[3];
                for (int k = 0; k < dim; ++k) {
                    ui[k] = u[k * n + i];
                    fi[k] = uf[k * n + i];
                }
                int64_t base = (pass == 1) ? out->off[i] : 0;
                for (int64_t a = 0; a < nc; ++a) {
                    int64_t j = buf[a];
                    int ok;
                    if (prec == 1) {
                        for (int k = 0; k < dim; ++k) fj[k] = uf[k * n + j];
                        ok = within_f32(dim, fi, fj, Lf, invLf, H2f);
                    } else {
                        for (int k = 0; k < dim; ++k) uj[k] = u[k * n + j];
                        ok = within_f64(dim, ui, uj, L, invL, H2);
                    }
                    if (ok) {
                        if (pass == 1) out->idx[base + c] = (int32_t)j;
                        ++c;
                    }
                }
                if (pass == 0) cnt[i] = c;
                else qsort(out->idx + base, (size_t)c, sizeof(int32_t), cmp_i32);
            }
            free(buf);
        }
    }
    free(cnt);
    grid_free(&g);
    free(u);
    free(uf);
    return err;
}

/* Exported neighbour search.  Always writes offsets[0..n]; writes nbr only when
 * cap >= total.  Returns the total number of entries, or -1 on bad input. */
int64_t orc_neighbors(int dim, int64_t n, const double* x, double L, double H, int prec, int brute,
                      int64_t* offsets, int32_t* nbr, int64_t cap)
{
    if ((dim != 2 && dim != 3) || n < 0 || !(H > 0.0) || !(2.0 * H < L)) return -1;
    nblist nb;
    build_lists(dim, n, x, L, H, prec, brute, &nb);
    int64_t total = nb.off[n];
    memcpy(offsets, nb.off, sizeof(int64_t) * (size_t)(n + 1));
    if (nbr && cap >= total) memcpy(nbr, nb.idx, sizeof(int32_t) * (size_t)total);
    nblist_free(&nb);
    return total;
}

/* ------------------------------------------------------------------ */
/* Per-particle and per-pair physics (Sec. 2.3, App. A)                 */
/* ------------------------------------------------------------------ */

/* Tait EOS, n = 7: p = rho0 c0^2 / 7 ((rho/rho0)^7 - 1) */
static double tait_p(const orc_params* p, double rho)
{
    double s = rho / p->rho0;
    double s7 = s * s * s * s * s * s * s;
    return p->rho0 * p->c0 * p->c0 / 7.0 * (s7 - 1.0);
}

/* dp/drho = c0^2 (rho/rho0)^6 */
static double tait_dp(const orc_params* p, double rho)
{
    double s = rho / p->rho0;
    double s6 = s * s * s * s * s * s;
    return p->c0 * p->c0 * s6;
}

/* Contribution of the directed pair (i, j), j != i, to a_i and drho_i/dt.
 * e = x_ij (minimum image).  Returns 0 when |e| >= H. */
void orc_pair_terms(const orc_params* p, const double* e, const double* vi, const double* vj,
                    double rhoi, double rhoj, double* a_ij /* dim */, double* rdot_ij)
{
    int dim = p->dim;
    double G[3] = {0, 0, 0};
    orc_gradw(dim, p->H, e, G);
    double r2 = 0.0;
    for (int k = 0; k < dim; ++k) r2 += e[k] * e[k];
    double inv = 1.0 / (r2 + p->eps * p->H * p->H);
    double Vj = p->m / rhoj;
    double pi = tait_p(p, rhoi), pj = tait_p(p, rhoj);
    double vij_e = 0.0, div = 0.0, eG = 0.0;
    for (int k = 0; k < dim; ++k) {
        vij_e += (vi[k] - vj[k]) * e[k];
        div += (vj[k] - vi[k]) * G[k];
        eG += e[k] * G[k];
    }
    double piij = vij_e * inv;
    double kp = -(1.0 / rhoi) * Vj * (pi + pj);
    double ka = p->alpha * p->H * p->c0 * (p->rho0 / rhoi) * Vj * piij;
    for (int k = 0; k < dim; ++k) a_ij[k] = (kp + ka) * G[k];
    double dif = -eG * inv; /* x_ji . grad_i W_ij / (r^2 + eps H^2) */
    *rdot_ij = -rhoi * Vj * div + p->delta * p->H * p->c0 * Vj * 2.0 * (rhoj - rhoi) * dif;
}

typedef struct {
    double de[3];   /* d Phi / d x_ij */
    double dvi[3];
    double dvj[3];
    double dri;
    double drj;
} pair_grad;

/* Reverse-mode partial derivatives of Phi(i,j) = abar . a_ij + rbar rdot_ij
 * with respect to (x_ij, v_i, v_j, rho_i, rho_j), written by hand backwards
 * through the intermediates of orc_pair_terms. */
static void pair_partials(const orc_params* p, const double* e, const double* vi, const double* vj,
                          double rhoi, double rhoj, const double* abar, double rbar, pair_grad* out)
{
    int dim = p->dim;
    memset(out, 0, sizeof(*out));
    double r2 = 0.0;
    for (int k = 0; k < dim; ++k) r2 += e[k] * e[k];
    double r = sqrt(r2);
    if (r == 0.0 || r >= p->H) return;
    /* forward intermediates */
    double q = r / p->H;
    double c1 = orc_cd(dim) / powi(p->H, dim + 1);
    double c2 = orc_cd(dim) / powi(p->H, dim + 2);
    double gmag = c1 * orc_what_d1(q);     /* |grad W| signed magnitude */
    double dgmag = c2 * orc_what_d2(q);    /* d gmag / dr */
    double eh[3] = {0, 0, 0}, G[3] = {0, 0, 0}, vij[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) {
        eh[k] = e[k] / r;
        G[k] = eh[k] * gmag;
        vij[k] = vi[k] - vj[k];
    }
    double den = r2 + p->eps * p->H * p->H;
    double inv = 1.0 / den;
    double Vj = p->m / rhoj;
    double pi = tait_p(p, rhoi), pj = tait_p(p, rhoj);
    double vij_e = 0.0, vijG = 0.0, eG = 0.0, aG = 0.0;
    for (int k = 0; k < dim; ++k) {
        vij_e += vij[k] * e[k];
        vijG += vij[k] * G[k];
        eG += e[k] * G[k];
        aG += abar[k] * G[k];
    }
    double piij = vij_e * inv;
    double ca = p->alpha * p->H * p->c0;
    double cd = p->delta * p->H * p->c0;
    double kp = -(1.0 / rhoi) * Vj * (pi + pj);
    double ka = ca * (p->rho0 / rhoi) * Vj * piij;
    double div = -vijG;
    double dif = -eG * inv;

    /* adjoints of intermediates */
    double Gb[3] = {0, 0, 0}, eb[3] = {0, 0, 0}, vijb[3] = {0, 0, 0};
    double Vjb = 0.0, rib = 0.0, rjb = 0.0, pib = 0.0, pjb = 0.0, pib_ = 0.0, invb = 0.0;

    /* a_ij = (kp + ka) G */
    double kb = aG;
    for (int k = 0; k < dim; ++k) Gb[k] += (kp + ka) * abar[k];
    /* rdot = -rhoi Vj div + cd Vj 2 (rhoj - rhoi) dif */
    double divb = -rbar * rhoi * Vj;
    rib += -rbar * Vj * div;
    Vjb += -rbar * rhoi * div + rbar * cd * 2.0 * (rhoj - rhoi) * dif;
    double difb = rbar * cd * Vj * 2.0 * (rhoj - rhoi);
    rjb += rbar * cd * Vj * 2.0 * dif;
    rib += -rbar * cd * Vj * 2.0 * dif;
    /* dif = -(e.G) inv */
    for (int k = 0; k < dim; ++k) {
        eb[k] += -difb * inv * G[k];
        Gb[k] += -difb * inv * e[k];
    }
    invb += -difb * eG;
    /* div = -(vij . G) */
    for (int k = 0; k < dim; ++k) {
        vijb[k] += -divb * G[k];
        Gb[k] += -divb * vij[k];
    }
    /* kp = -(Vj / rhoi)(pi + pj) */
    Vjb += -kb * (pi + pj) / rhoi;
    rib += kb * Vj * (pi + pj) / (rhoi * rhoi);
    pib += -kb * Vj / rhoi;
    pjb += -kb * Vj / rhoi;
    /* ka = ca rho0 Vj piij / rhoi */
    Vjb += kb * ca * p->rho0 * piij / rhoi;
    double pijb = kb * ca * p->rho0 * Vj / rhoi;
    rib += -kb * ka / rhoi;
    /* piij = (vij . e) inv */
    for (int k = 0; k < dim; ++k) {
        vijb[k] += pijb * inv * e[k];
        eb[k] += pijb * inv * vij[k];
    }
    invb += pijb * vij_e;
    /* inv = 1/(r2 + eps H^2) */
    for (int k = 0; k < dim; ++k) eb[k] += invb * (-inv * inv) * 2.0 * e[k];
    /* G = eh gmag(r): dG/de = gmag/r (I - eh eh^T) + dgmag eh eh^T */
    double ehGb = 0.0;
    for (int k = 0; k < dim; ++k) ehGb += eh[k] * Gb[k];
    for (int k = 0; k < dim; ++k) eb[k] += gmag / r * (Gb[k] - eh[k] * ehGb) + dgmag * eh[k] * ehGb;
    /* Vj = m / rhoj */
    rjb += -Vjb * p->m / (rhoj * rhoj);
    /* p = Tait(rho) */
    rib += pib * tait_dp(p, rhoi);
    rjb += pjb * tait_dp(p, rhoj);
    (void)pib_;
    for (int k = 0; k < dim; ++k) {
        out->de[k] = eb[k];
        out->dvi[k] = vijb[k];
        out->dvj[k] = -vijb[k];
    }
    out->dri = rib;
    out->drj = rjb;
}

/* Exported for finite-difference checks of the partials. */
void orc_pair_partials(const orc_params* p, const double* e, const double* vi, const double* vj,
                       double rhoi, double rhoj, const double* abar, double rbar, double* out /* 3+3+3+2 */)
{
    pair_grad g;
    pair_partials(p, e, vi, vj, rhoi, rhoj, abar, rbar, &g);
    for (int k = 0; k < 3; ++k) {
        out[k] = g.de[k];
        out[3 + k] = g.dvi[k];
        out[6 + k] = g.dvj[k];
    }
    out[9] = g.dri;
    out[10] = g.drj;
}

static int valid_params(const orc_params* p)
{
    if (p->dim != 2 && p->dim != 3) return 0;
    if (!(p->H > 0.0) || !(2.0 * p->H < p->L)) return 0;
    if (!(p->m > 0.0) || !(p->rho0 > 0.0) || !(p->c0 > 0.0)) return 0;
    return 1;
}

static void wrap_all(const orc_params* p, int64_t n, const double* x, double* u)
{
    double invL = 1.0 / p->L;
    for (int k = 0; k < p->dim; ++k)
        for (int64_t i = 0; i < n; ++i) u[k * n + i] = wrap_f64(x[k * n + i], p->L, invL);
}

/* ---------------------------------------------------------------- renormalised gradient
 *
 * App. A.5 (kernel and gradient correction terms): the corrected gradient of a field A,
 *   <grad A>_i = L_i sum_j V_j (A_j - A_i) grad_i W_ij,
 *   L_i = [ sum_j V_j (x_j - x_i) (x) grad_i W_ij ]^-1,   V_j = m / rho_j.
 * The matrix M_i in the brackets is symmetric (grad_i W_ij is parallel to
 * x_i - x_j) and close to the identity for a full support, as in the periodic
 * box; it is inverted exactly (the paper allows a pseudo-inverse; a singular
 * M_i gives a zero gradient here). */

/* M_i and g_i = sum_j V_j (A_j - A_i) grad_i W_ij for particle i (dim x dim
 * row-major and dim). */
static void renorm_moments(const orc_params* p, int64_t n, const double* u, const double* rho, const double* A,
                           const nblist* nb, int64_t i, double* M, double* g)
{
    int dim = p->dim;
    double invL = 1.0 / p->L;
    double ui[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) ui[k] = u[k * n + i];
    for (int a = 0; a < 9; ++a) M[a] = 0.0;
    for (int a = 0; a < 3; ++a) g[a] = 0.0;
    for (int64_t q = nb->off[i]; q < nb->off[i + 1]; ++q) {
        int64_t j = nb->idx[q];
        if (j == i) continue;
        double uj[3] = {0, 0, 0}, e[3] = {0, 0, 0}, w[3] = {0, 0, 0};
        for (int k = 0; k < dim; ++k) uj[k] = u[k * n + j];
        minimg(dim, ui, uj, p->L, invL, e);        /* e = x_i - x_j */
        orc_gradw(dim, p->H, e, w);                /* grad_i W_ij */
        double Vj = p->m / rho[j];
        for (int a = 0; a < dim; ++a)
            for (int b = 0; b < dim; ++b) M[a * dim + b] += Vj * (-e[a]) * w[b];
        for (int b = 0; b < dim; ++b) g[b] += Vj * (A[j] - A[i]) * w[b];
    }
}

/* Inverse of a dim x dim matrix (cofactors); 0 if singular. */
static int inv_small(int dim, const double* M, double* L)
{
    if (dim == 2) {
        double det = M[0] * M[3] - M[1] * M[2];
        if (det == 0.0 || !isfinite(det)) return 0;
        L[0] = M[3] / det;
        L[1] = -M[1] / det;
        L[2] = -M[2] / det;
        L[3] = M[0] / det;
        return 1;
    }
    double c00 = M[4] * M[8] - M[5] * M[7], c01 = M[5] * M[6] - M[3] * M[8], c02 = M[3] * M[7] - M[4] * M[6];
    double det = M[0] * c00 + M[1] * c01 + M[2] * c02;
    if (det == 0.0 || !isfinite(det)) return 0;
    L[0] = c00 / det;
    L[1] = (M[2] * M[7] - M[1] * M[8]) / det;
    L[2] = (M[1] * M[5] - M[2] * M[4]) / det;
    L[3] = c01 / det;
    L[4] = (M[0] * M[8] - M[2] * M[6]) / det;
    L[5] = (M[2] * M[3] - M[0] * M[5]) / det;
    L[6] = c02 / det;
    L[7] = (M[1] * M[6] - M[0] * M[7]) / det;
    L[8] = (M[0] * M[4] - M[1] * M[3]) / det;
    return 1;
}

/* <grad A>_i for all particles into G (dim*n); Linv (dim*dim*n) receives L_i
 * when not NULL. */
static void renorm_gradient(const orc_params* p, int64_t n, const double* u, const double* rho, const double* A,
                            const nblist* nb, double* G, double* Linv)
{
    int dim = p->dim;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double M[9], g[3], L[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        renorm_moments(p, n, u, rho, A, nb, i, M, g);
        int ok = inv_small(dim, M, L);
        for (int a = 0; a < dim; ++a) {
            double s = 0.0;
            if (ok)
                for (int b = 0; b < dim; ++b) s += L[a * dim + b] * g[b];
            G[a * n + i] = s;
        }
        if (Linv)
            for (int a = 0; a < dim * dim; ++a) Linv[(size_t)a * n + i] = ok ? L[a] : 0.0;
    }
}

/* Exported for the checks of the operator itself: G (dim*n) = <grad A> with
 * V_j from rho. */
int orc_renorm_gradient(const orc_params* p, int64_t n, const double* x, const double* rho, const double* A,
                        double* G)
{
    if (!valid_params(p) || n < 0) return -1;
    double* u = (double*)malloc(sizeof(double) * (size_t)p->dim * (size_t)(n > 0 ? n : 1));
    wrap_all(p, n, x, u);
    nblist nb;
    build_lists(p->dim, n, x, p->L, p->H, 0, 0, &nb);
    renorm_gradient(p, n, u, rho, A, &nb, G, NULL);
    nblist_free(&nb);
    free(u);
    return 0;
}

/* The renormalised part of the delta-diffusion (Antuono et al.'s form, cited
 * in Sec. 2.3 through the delta-SPH scheme): with G = <grad rho>,
 *   drho_i/dt += -delta H c0 sum_j V_j (G_i + G_j) . grad_i W_ij,
 * added to drho (n). */
static void renorm_diffusion_add(const orc_params* p, int64_t n, const double* u, const double* rho,
                                 const nblist* nb, const double* G, double* drho)
{
    int dim = p->dim;
    double invL = 1.0 / p->L;
    double cd = p->delta * p->H * p->c0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double ui[3] = {0, 0, 0};
        for (int k = 0; k < dim; ++k) ui[k] = u[k * n + i];
        double t = 0.0;
        for (int64_t q = nb->off[i]; q < nb->off[i + 1]; ++q) {
            int64_t j = nb->idx[q];
            if (j == i) continue;
            double uj[3] = {0, 0, 0}, e[3] = {0, 0, 0}, w[3] = {0, 0, 0};
            for (int k = 0; k < dim; ++k) uj[k] = u[k * n + j];
            minimg(dim, ui, uj, p->L, invL, e);
            orc_gradw(dim, p->H, e, w);
            double sw = 0.0;
            for (int k = 0; k < dim; ++k) sw += (G[k * n + i] + G[k * n + j]) * w[k];
            t += (p->m / rho[j]) * sw;
        }
        drho[i] += -cd * t;
    }
}

/* Right-hand side of one evaluation of the update function: drho/dt, a, and
 * (optionally) the summation density.  Gather over the ascending neighbour
 * list; the self pair contributes only m W(0) to rho_sum. */
static void rhs_with_list(const orc_params* p, int64_t n, const double* u, const double* v, const double* rho,
                          const nblist* nb, double* drho, double* acc, double* rhosum)
{
    int dim = p->dim;
    double invL = 1.0 / p->L;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double ui[3] = {0, 0, 0}, vi[3] = {0, 0, 0};
        for (int k = 0; k < dim; ++k) {
            ui[k] = u[k * n + i];
            vi[k] = v[k * n + i];
        }
        double ai[3] = {0, 0, 0}, rd = 0.0, rs = 0.0;
        for (int64_t a = nb->off[i]; a < nb->off[i + 1]; ++a) {
            int64_t j = nb->idx[a];
            double uj[3] = {0, 0, 0}, vj[3] = {0, 0, 0}, e[3] = {0, 0, 0};
            for (int k = 0; k < dim; ++k) {
                uj[k] = u[k * n + j];
                vj[k] = v[k * n + j];
            }
            minimg(dim, ui, uj, p->L, invL, e);
            rs += p->m * orc_w(dim, p->H, e);
            if (j == i) continue;
            double aij[3] = {0, 0, 0}, rij = 0.0;
            orc_pair_terms(p, e, vi, vj, rho[i], rho[j], aij, &rij);
            for (int k = 0; k < dim; ++k) ai[k] += aij[k];
            rd += rij;
        }
        if (drho) drho[i] = rd;
        if (acc)
            for (int k = 0; k < dim; ++k) acc[k * n + i] = ai[k];
        if (rhosum) rhosum[i] = rs;
    }
    if (p->renorm && drho) {
        double* G = (double*)malloc(sizeof(double) * (size_t)dim * (size_t)(n > 0 ? n : 1));
        renorm_gradient(p, n, u, rho, rho, nb, G, NULL);
        renorm_diffusion_add(p, n, u, rho, nb, G, drho);
        free(G);
    }
}

int orc_rhs(const orc_params* p, int64_t n, const double* x, const double* v, const double* rho,
            double* drho, double* acc, double* rhosum)
{
    if (!valid_params(p) || n < 0) return -1;
    double* u = (double*)malloc(sizeof(double) * (size_t)p->dim * (size_t)(n > 0 ? n : 1));
    wrap_all(p, n, x, u);
    nblist nb;
    build_lists(p->dim, n, x, p->L, p->H, 0, 0, &nb);
    rhs_with_list(p, n, u, v, rho, &nb, drho, acc, rhosum);
    nblist_free(&nb);
    free(u);
    return 0;
}

/* Same quantities for the listed particles only, each found by a brute-force
 * pass over all particles (for sampled checks of large states). */
int orc_rhs_sample(const orc_params* p, int64_t n, const double* x, const double* v, const double* rho,
                   int64_t ns, const int64_t* sample, double* drho, double* acc /* dim*ns */, double* rhosum)
{
    if (!valid_params(p) || p->renorm || n < 0) return -1;
    int dim = p->dim;
    double invL = 1.0 / p->L;
    double H2 = p->H * p->H;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < ns; ++s) {
        int64_t i = sample[s];
        double ui[3] = {0, 0, 0}, vi[3] = {0, 0, 0};
        for (int k = 0; k < dim; ++k) {
            ui[k] = wrap_f64(x[k * n + i], p->L, invL);
            vi[k] = v[k * n + i];
        }
        double ai[3] = {0, 0, 0}, rd = 0.0, rs = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double uj[3] = {0, 0, 0}, vj[3] = {0, 0, 0}, e[3] = {0, 0, 0};
            for (int k = 0; k < dim; ++k) uj[k] = wrap_f64(x[k * n + j], p->L, invL);
            if (!within_f64(dim, ui, uj, p->L, invL, H2)) continue;
            for (int k = 0; k < dim; ++k) vj[k] = v[k * n + j];
            minimg(dim, ui, uj, p->L, invL, e);
            rs += p->m * orc_w(dim, p->H, e);
            if (j == i) continue;
            double aij[3] = {0, 0, 0}, rij = 0.0;
            orc_pair_terms(p, e, vi, vj, rho[i], rho[j], aij, &rij);
            for (int k = 0; k < dim; ++k) ai[k] += aij[k];
            rd += rij;
        }
        if (drho) drho[s] = rd;
        if (acc)
            for (int k = 0; k < dim; ++k) acc[k * ns + s] = ai[k];
        if (rhosum) rhosum[s] = rs;
    }
    return 0;
}

/* One semi-implicit Euler step in place (Sec. 3.4): kick, then drift. */
static void step_once(const orc_params* p, int64_t n, double* x, double* v, double* rho, double* work)
{
    int dim = p->dim;
    double* u = work;                       /* dim*n */
    double* acc = work + (size_t)dim * n;   /* dim*n */
    double* drho = acc + (size_t)dim * n;   /* n */
    wrap_all(p, n, x, u);
    nblist nb;
    build_lists(dim, n, x, p->L, p->H, 0, 0, &nb);
    rhs_with_list(p, n, u, v, rho, &nb, drho, acc, NULL);
    nblist_free(&nb);
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < dim; ++k) v[k * n + i] = v[k * n + i] + p->dt * acc[k * n + i];
        rho[i] = rho[i] + p->dt * drho[i];
        for (int k = 0; k < dim; ++k) x[k * n + i] = x[k * n + i] + p->dt * v[k * n + i];
    }
}

int orc_step(const orc_params* p, int64_t n, double* x, double* v, double* rho, int32_t nsteps)
{
    if (!valid_params(p) || n < 0 || nsteps < 0) return -1;
    double* work = (double*)malloc(sizeof(double) * ((size_t)2 * p->dim + 1) * (size_t)(n > 0 ? n : 1));
    for (int32_t s = 0; s < nsteps; ++s) step_once(p, n, x, v, rho, work);
    free(work);
    return 0;
}

/* The J^T terms of the update function's vector-Jacobian product (Sec. 2.2):
 * for cotangents abar of the accelerations and rbar of drho/dt, the
 * cotangents (gx, gv, gr) of the positions, velocities and densities, which
 * gather, for every particle k and neighbour j != k, the partials of the two
 * directed pairs (k,j) and (j,k) that involve k.  Outputs are overwritten. */
static void renorm_vjp_add(const orc_params* p, int64_t n, const double* u, const double* rho, const nblist* nb,
                           const double* rbar, double* gx, double* gr);

static void rhs_vjp_with_list(const orc_params* p, int64_t n, const double* u, const double* v,
                              const double* rho, const nblist* nb, const double* abar, const double* rbar,
                              double* gx, double* gv, double* gr)
{
    int dim = p->dim;
    double invL = 1.0 / p->L;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < n; ++k) {
        double uk[3] = {0, 0, 0}, vk[3] = {0, 0, 0}, ak[3] = {0, 0, 0};
        for (int c = 0; c < dim; ++c) {
            uk[c] = u[c * n + k];
            vk[c] = v[c * n + k];
            ak[c] = abar[c * n + k];
        }
        double sx[3] = {0, 0, 0}, sv[3] = {0, 0, 0}, sr = 0.0;
        for (int64_t a = nb->off[k]; a < nb->off[k + 1]; ++a) {
            int64_t j = nb->idx[a];
            if (j == k) continue;
            double uj[3] = {0, 0, 0}, vj[3] = {0, 0, 0}, aj[3] = {0, 0, 0};
            for (int c = 0; c < dim; ++c) {
                uj[c] = u[c * n + j];
                vj[c] = v[c * n + j];
                aj[c] = abar[c * n + j];
            }
            double ekj[3] = {0, 0, 0}, ejk[3] = {0, 0, 0};
            minimg(dim, uk, uj, p->L, invL, ekj);
            minimg(dim, uj, uk, p->L, invL, ejk);
            pair_grad g1, g2;
            pair_partials(p, ekj, vk, vj, rho[k], rho[j], ak, rbar[k], &g1); /* Phi(k,j) */
            pair_partials(p, ejk, vj, vk, rho[j], rho[k], aj, rbar[j], &g2); /* Phi(j,k) */
            for (int c = 0; c < dim; ++c) {
                sx[c] += g1.de[c] - g2.de[c];
                sv[c] += g1.dvi[c] + g2.dvj[c];
            }
            sr += g1.dri + g2.drj;
        }
        for (int c = 0; c < dim; ++c) {
            gx[c * n + k] = sx[c];
            gv[c * n + k] = sv[c];
        }
        gr[k] = sr;
    }
    if (p->renorm) renorm_vjp_add(p, n, u, rho, nb, rbar, gx, gr);
}

/* The renormalised diffusion's share of the update function's VJP, for
 * cotangents rbar of drho/dt, added to gx (positions) and gr (densities);
 * velocities do not enter.  In scatter form over the lists, sequentially:
 *  (a) with G fixed: T_i = c sum_j V_j s_ij . w_ij, s_ij = G_i + G_j,
 *      c = -delta H c0, w_ij = grad_i W_ij at e = x_i - x_j:
 *        Gbar_i += c rbar_i V_j w_ij,  Gbar_j += c rbar_i V_j w_ij,
 *        ebar = c rbar_i V_j Hess(e) s_ij   (x_i += ebar, x_j -= ebar),
 *        rho_j += -(V_j / rho_j) c rbar_i (s_ij . w_ij);
 *  (b) G_i = L_i g_i:  gbar_i = L_i^T Gbar_i,  Mbar_i = -gbar_i G_i^T;
 *  (c) M_i = sum_j V_j (-e) (x) w_ij,  g_i = sum_j V_j (rho_j - rho_i) w_ij:
 *        ebar = -V_j (Mbar_i w + Hess Mbar_i^T e) + V_j (rho_j - rho_i) Hess gbar_i,
 *        rho_j += V_j (gbar_i . w) - (V_j / rho_j) [(rho_j - rho_i)(gbar_i . w) - e^T Mbar_i w],
 *        rho_i -= V_j (gbar_i . w). */
static void renorm_vjp_add(const orc_params* p, int64_t n, const double* u, const double* rho, const nblist* nb,
                           const double* rbar, double* gx, double* gr)
{
    int dim = p->dim;
    double invL = 1.0 / p->L;
    double c = -p->delta * p->H * p->c0;
    size_t nn = (size_t)(n > 0 ? n : 1);
    double* G = (double*)malloc(sizeof(double) * (size_t)dim * nn);
    double* Linv = (double*)malloc(sizeof(double) * (size_t)dim * (size_t)dim * nn);
    double* Gb = (double*)calloc((size_t)dim * nn, sizeof(double));
    renorm_gradient(p, n, u, rho, rho, nb, G, Linv);
    for (int64_t i = 0; i < n; ++i) {
        double ui[3] = {0, 0, 0};
        for (int k = 0; k < dim; ++k) ui[k] = u[k * n + i];
        for (int64_t q = nb->off[i]; q < nb->off[i + 1]; ++q) {
            int64_t j = nb->idx[q];
            if (j == i) continue;
            double uj[3] = {0, 0, 0}, e[3] = {0, 0, 0}, w[3] = {0, 0, 0}, Hs[9], sv[3] = {0, 0, 0};
            for (int k = 0; k < dim; ++k) uj[k] = u[k * n + j];
            minimg(dim, ui, uj, p->L, invL, e);
            orc_gradw(dim, p->H, e, w);
            orc_hessw(dim, p->H, e, Hs);
            double Vj = p->m / rho[j], sw = 0.0;
            for (int k = 0; k < dim; ++k) {
                sv[k] = G[k * n + i] + G[k * n + j];
                sw += sv[k] * w[k];
            }
            for (int k = 0; k < dim; ++k) {
                Gb[k * n + i] += c * rbar[i] * Vj * w[k];
                Gb[k * n + j] += c * rbar[i] * Vj * w[k];
                double hs = 0.0;
                for (int b = 0; b < dim; ++b) hs += Hs[k * dim + b] * sv[b];
                gx[k * n + i] += c * rbar[i] * Vj * hs;
                gx[k * n + j] -= c * rbar[i] * Vj * hs;
            }
            gr[j] += -(Vj / rho[j]) * c * rbar[i] * sw;
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        double ui[3] = {0, 0, 0}, gbar[3] = {0, 0, 0}, Mb[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int k = 0; k < dim; ++k) ui[k] = u[k * n + i];
        for (int a = 0; a < dim; ++a)
            for (int b = 0; b < dim; ++b) gbar[a] += Linv[(size_t)(b * dim + a) * n + i] * Gb[b * n + i];
        for (int a = 0; a < dim; ++a)
            for (int b = 0; b < dim; ++b) Mb[a * dim + b] = -gbar[a] * G[b * n + i];
        for (int64_t q = nb->off[i]; q < nb->off[i + 1]; ++q) {
            int64_t j = nb->idx[q];
            if (j == i) continue;
            double uj[3] = {0, 0, 0}, e[3] = {0, 0, 0}, w[3] = {0, 0, 0}, Hs[9];
            for (int k = 0; k < dim; ++k) uj[k] = u[k * n + j];
            minimg(dim, ui, uj, p->L, invL, e);
            orc_gradw(dim, p->H, e, w);
            orc_hessw(dim, p->H, e, Hs);
            double Vj = p->m / rho[j];
            double Mw[3] = {0, 0, 0}, Mte[3] = {0, 0, 0}, gw = 0.0, eMw = 0.0;
            for (int a = 0; a < dim; ++a)
                for (int b = 0; b < dim; ++b) {
                    Mw[a] += Mb[a * dim + b] * w[b];
                    Mte[b] += Mb[a * dim + b] * e[a];
                }
            for (int k = 0; k < dim; ++k) {
                gw += gbar[k] * w[k];
                eMw += e[k] * Mw[k];
            }
            double drj = rho[j] - rho[i];
            for (int k = 0; k < dim; ++k) {
                double hm = 0.0, hg = 0.0;
                for (int b = 0; b < dim; ++b) {
                    hm += Hs[k * dim + b] * Mte[b];
                    hg += Hs[k * dim + b] * gbar[b];
                }
                double eb = -Vj * (Mw[k] + hm) + Vj * drj * hg;
                gx[k * n + i] += eb;
                gx[k * n + j] -= eb;
            }
            gr[j] += Vj * gw - (Vj / rho[j]) * (drj * gw - eMw);
            gr[i] -= Vj * gw;
        }
    }
    free(G);
    free(Linv);
    free(Gb);
}

/* Vector-Jacobian product of one step.  On entry (xb, vb, rb) hold the
 * cotangents of the step's output (x', v', rho'); on exit those of its input
 * (x, v, rho), the state at the start of the step.
 *   v' = v + dt a(x,v,rho);  rho' = rho + dt rdot(x,v,rho);  x' = x + dt v'
 * gives  vt = vb' + dt xb',  abar = dt vt,  rbar = dt rb',
 *        xb = xb' + (J_x)^T,  vb = vt + (J_v)^T,  rb = rb' + (J_rho)^T. */
static void step_adjoint_with_list(const orc_params* p, int64_t n, const double* u, const double* v,
                                   const double* rho, const nblist* nb, double* xb, double* vb, double* rb)
{
    int dim = p->dim;
    double* abar = (double*)malloc(sizeof(double) * (size_t)dim * (size_t)(n > 0 ? n : 1));
    double* rbar = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < dim; ++k) {
            double vt = vb[k * n + i] + p->dt * xb[k * n + i];
            vb[k * n + i] = vt;
            abar[k * n + i] = p->dt * vt;
        }
        rbar[i] = p->dt * rb[i];
    }
    double* gx = (double*)calloc((size_t)dim * (size_t)(n > 0 ? n : 1), sizeof(double));
    double* gv = (double*)calloc((size_t)dim * (size_t)(n > 0 ? n : 1), sizeof(double));
    double* gr = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    rhs_vjp_with_list(p, n, u, v, rho, nb, abar, rbar, gx, gv, gr);
    for (int64_t i = 0; i < n; ++i) {
        for (int c = 0; c < dim; ++c) {
            xb[c * n + i] += gx[c * n + i];
            vb[c * n + i] += gv[c * n + i];
        }
        rb[i] += gr[i];
    }
    free(gx);
    free(gv);
    free(gr);
    free(abar);
    free(rbar);
}

int orc_step_adjoint(const orc_params* p, int64_t n, const double* x, const double* v, const double* rho,
                     double* xb, double* vb, double* rb)
{
    if (!valid_params(p) || n < 0) return -1;
    double* u = (double*)malloc(sizeof(double) * (size_t)p->dim * (size_t)(n > 0 ? n : 1));
    wrap_all(p, n, x, u);
    nblist nb;
    build_lists(p->dim, n, x, p->L, p->H, 0, 0, &nb);
    step_adjoint_with_list(p, n, u, v, rho, &nb, xb, vb, rb);
    nblist_free(&nb);
    free(u);
    return 0;
}

/* Vector-Jacobian product of the summation density (Sec. 2.3 summation
 * density, Sec. 2.2 adjoint): for cotangents g_i of rho_i = sum_j m W_ij,
 *   xbar_k = sum_{j != k} m (g_k + g_j) grad_k W_kj,
 * because x_k enters both k's own sum (through W_kj) and every neighbour's
 * sum (through W_jk = W_kj, whose gradient with respect to x_k is again
 * grad_k W_kj).  The self pair has zero gradient.  xbar is overwritten. */
int orc_density_adjoint(const orc_params* p, int64_t n, const double* x, const double* g, double* xbar)
{
    if (!valid_params(p) || n < 0) return -1;
    int dim = p->dim;
    double invL = 1.0 / p->L;
    double* u = (double*)malloc(sizeof(double) * (size_t)dim * (size_t)(n > 0 ? n : 1));
    wrap_all(p, n, x, u);
    nblist nb;
    build_lists(dim, n, x, p->L, p->H, 0, 0, &nb);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < n; ++k) {
        double uk[3] = {0, 0, 0}, acc[3] = {0, 0, 0};
        for (int c = 0; c < dim; ++c) uk[c] = u[c * n + k];
        for (int64_t a = nb.off[k]; a < nb.off[k + 1]; ++a) {
            int64_t j = nb.idx[a];
            if (j == k) continue;
            double uj[3] = {0, 0, 0}, e[3] = {0, 0, 0}, gw[3] = {0, 0, 0};
            for (int c = 0; c < dim; ++c) uj[c] = u[c * n + j];
            minimg(dim, uk, uj, p->L, invL, e);
            orc_gradw(dim, p->H, e, gw);
            for (int c = 0; c < dim; ++c) acc[c] += p->m * (g[k] + g[j]) * gw[c];
        }
        for (int c = 0; c < dim; ++c) xbar[c * n + k] = acc[c];
    }
    nblist_free(&nb);
    free(u);
    return 0;
}

/* The adjoint-sweep increments (the J^T terms only, without the integrator
 * transpose) for listed particles, given abar and rbar of every particle;
 * each sampled particle is handled by a brute-force pass over all particles. */
int orc_adjoint_sweep_sample(const orc_params* p, int64_t n, const double* x, const double* v, const double* rho,
                             const double* abar, const double* rbar, int64_t ns, const int64_t* sample,
                             double* gx /* dim*ns */, double* gv /* dim*ns */, double* gr /* ns */)
{
    if (!valid_params(p) || p->renorm || n < 0) return -1;
    int dim = p->dim;
    double invL = 1.0 / p->L;
    double H2 = p->H * p->H;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < ns; ++s) {
        int64_t k = sample[s];
        double uk[3] = {0, 0, 0}, vk[3] = {0, 0, 0}, ak[3] = {0, 0, 0};
        for (int c = 0; c < dim; ++c) {
            uk[c] = wrap_f64(x[c * n + k], p->L, invL);
            vk[c] = v[c * n + k];
            ak[c] = abar[c * n + k];
        }
        double sx[3] = {0, 0, 0}, sv[3] = {0, 0, 0}, sr = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == k) continue;
            double uj[3] = {0, 0, 0}, vj[3] = {0, 0, 0}, aj[3] = {0, 0, 0};
            for (int c = 0; c < dim; ++c) uj[c] = wrap_f64(x[c * n + j], p->L, invL);
            if (!within_f64(dim, uk, uj, p->L, invL, H2)) continue;
            for (int c = 0; c < dim; ++c) {
                vj[c] = v[c * n + j];
                aj[c] = abar[c * n + j];
            }
            double ekj[3] = {0, 0, 0}, ejk[3] = {0, 0, 0};
            minimg(dim, uk, uj, p->L, invL, ekj);
            minimg(dim, uj, uk, p->L, invL, ejk);
            pair_grad g1, g2;
            pair_partials(p, ekj, vk, vj, rho[k], rho[j], ak, rbar[k], &g1);
            pair_partials(p, ejk, vj, vk, rho[j], rho[k], aj, rbar[j], &g2);
            for (int c = 0; c < dim; ++c) {
                sx[c] += g1.de[c] - g2.de[c];
                sv[c] += g1.dvi[c] + g2.dvj[c];
            }
            sr += g1.dri + g2.drj;
        }
        for (int c = 0; c < dim; ++c) {
            gx[c * ns + s] = sx[c];
            gv[c * ns + s] = sv[c];
        }
        gr[s] = sr;
    }
    return 0;
}

/* Full rollout and its gradient: T steps forward keeping every state, the
 * loss seed, then T adjoint steps.  loss_kind 0: L = sum_i |v_i(T)|^2;
 * loss_kind 1: L = 1/2 sum_i m |v_i(T)|^2.  Writes the final state and the
 * gradients of L with respect to the initial x, v, rho. */
int orc_rollout(const orc_params* p, int64_t n, const double* x0, const double* v0, const double* rho0,
                int32_t T, int32_t loss_kind, double* xT, double* vT, double* rhoT,
                double* gx0, double* gv0, double* grho0, double* loss)
{
    if (!valid_params(p) || n < 0 || T < 0) return -1;
    int dim = p->dim;
    size_t sd = (size_t)dim * (size_t)n, s1 = (size_t)n;
    double* xs = (double*)malloc(sizeof(double) * sd * (size_t)(T + 1) + 8);
    double* vs = (double*)malloc(sizeof(double) * sd * (size_t)(T + 1) + 8);
    double* rs = (double*)malloc(sizeof(double) * s1 * (size_t)(T + 1) + 8);
    double* work = (double*)malloc(sizeof(double) * ((size_t)2 * dim + 1) * (size_t)(n > 0 ? n : 1));
    memcpy(xs, x0, sizeof(double) * sd);
    memcpy(vs, v0, sizeof(double) * sd);
    memcpy(rs, rho0, sizeof(double) * s1);
    for (int32_t t = 0; t < T; ++t) {
        memcpy(xs + sd * (t + 1), xs + sd * t, sizeof(double) * sd);
        memcpy(vs + sd * (t + 1), vs + sd * t, sizeof(double) * sd);
        memcpy(rs + s1 * (t + 1), rs + s1 * t, sizeof(double) * s1);
        step_once(p, n, xs + sd * (t + 1), vs + sd * (t + 1), rs + s1 * (t + 1), work);
    }
    const double* vfin = vs + sd * T;
    double L = 0.0;
    for (size_t a = 0; a < sd; ++a) {
        if (loss_kind == 0) {
            L += vfin[a] * vfin[a];
            gv0[a] = 2.0 * vfin[a];
        } else {
            L += 0.5 * p->m * vfin[a] * vfin[a];
            gv0[a] = p->m * vfin[a];
        }
        gx0[a] = 0.0;
    }
    for (size_t a = 0; a < s1; ++a) grho0[a] = 0.0;
    if (loss) *loss = L;
    if (xT) memcpy(xT, xs + sd * T, sizeof(double) * sd);
    if (vT) memcpy(vT, vs + sd * T, sizeof(double) * sd);
    if (rhoT) memcpy(rhoT, rs + s1 * T, sizeof(double) * s1);
    for (int32_t t = T - 1; t >= 0; --t)
        orc_step_adjoint(p, n, xs + sd * t, vs + sd * t, rs + s1 * t, gx0, gv0, grho0);
    free(xs);
    free(vs);
    free(rs);
    free(work);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Explicit Runge-Kutta steps from a Butcher tableau (Sec. 3.4 and the  */
/* time-integration appendix: explicit schemes given by their tableau)  */
/* ------------------------------------------------------------------ */

/* The update function's vector-Jacobian product for one state: given the
 * cotangents abar of a and rbar of drho/dt, (xbar, vbar, rhobar) receive the
 * J^T terms (overwritten).  dx/dt = v is not part of it. */
int orc_rhs_vjp(const orc_params* p, int64_t n, const double* x, const double* v, const double* rho,
                const double* abar, const double* rbar, double* xbar, double* vbar, double* rhobar)
{
    if (!valid_params(p) || n < 0) return -1;
    double* u = (double*)malloc(sizeof(double) * (size_t)p->dim * (size_t)(n > 0 ? n : 1));
    wrap_all(p, n, x, u);
    nblist nb;
    build_lists(p->dim, n, x, p->L, p->H, 0, 0, &nb);
    rhs_vjp_with_list(p, n, u, v, rho, &nb, abar, rbar, xbar, vbar, rhobar);
    nblist_free(&nb);
    free(u);
    return 0;
}

/* Stage derivative k = f(u) = (v, a(u), drho/dt(u)) of the state u = (x, v, rho),
 * packed as [x-rate (dim*n) | v-rate (dim*n) | rho-rate (n)]. */
static void stage_rate(const orc_params* p, int64_t n, const double* x, const double* v, const double* rho,
                       double* k)
{
    int dim = p->dim;
    double* u = (double*)malloc(sizeof(double) * (size_t)dim * (size_t)(n > 0 ? n : 1));
    wrap_all(p, n, x, u);
    nblist nb;
    build_lists(dim, n, x, p->L, p->H, 0, 0, &nb);
    rhs_with_list(p, n, u, v, rho, &nb, k + (size_t)2 * dim * n, k + (size_t)dim * n, NULL);
    nblist_free(&nb);
    free(u);
    memcpy(k, v, sizeof(double) * (size_t)dim * (size_t)n);
}

/* Stage states of one step: u_i = u + dt sum_{j<i} A_ij k_j, k_i = f(u_i).
 * us and ks hold `stages` packed states / rates of (2 dim + 1) n each. */
static void rk_stages(const orc_params* p, int64_t n, const double* x, const double* v, const double* rho,
                      int stages, const double* A, double* us, double* ks)
{
    int dim = p->dim;
    size_t m = ((size_t)2 * dim + 1) * (size_t)n;
    for (int i = 0; i < stages; ++i) {
        double* ui = us + (size_t)i * m;
        memcpy(ui, x, sizeof(double) * (size_t)dim * (size_t)n);
        memcpy(ui + (size_t)dim * n, v, sizeof(double) * (size_t)dim * (size_t)n);
        memcpy(ui + (size_t)2 * dim * n, rho, sizeof(double) * (size_t)n);
        for (int j = 0; j < i; ++j) {
            double a = A[i * stages + j];
            if (a == 0.0) continue;
            const double* kj = ks + (size_t)j * m;
            for (size_t e = 0; e < m; ++e) ui[e] += p->dt * a * kj[e];
        }
        stage_rate(p, n, ui, ui + (size_t)dim * n, ui + (size_t)2 * dim * n, ks + (size_t)i * m);
    }
}

/* nsteps explicit Runge-Kutta steps with the tableau (A strictly lower
 * triangular, stages x stages, row-major; weights b): u' = u + dt sum_i b_i k_i. */
int orc_step_rk(const orc_params* p, int64_t n, double* x, double* v, double* rho, int32_t nsteps,
                int32_t stages, const double* A, const double* b)
{
    if (!valid_params(p) || n < 0 || nsteps < 0 || stages < 1 || stages > 8) return -1;
    int dim = p->dim;
    size_t m = ((size_t)2 * dim + 1) * (size_t)n;
    double* us = (double*)malloc(sizeof(double) * m * (size_t)stages + 1);
    double* ks = (double*)malloc(sizeof(double) * m * (size_t)stages + 1);
    for (int32_t t = 0; t < nsteps; ++t) {
        rk_stages(p, n, x, v, rho, stages, A, us, ks);
        for (int i = 0; i < stages; ++i) {
            const double* ki = ks + (size_t)i * m;
            double w = p->dt * b[i];
            if (w == 0.0) continue;
            for (int64_t e = 0; e < (int64_t)dim * n; ++e) x[e] += w * ki[e];
            for (int64_t e = 0; e < (int64_t)dim * n; ++e) v[e] += w * ki[(size_t)dim * n + e];
            for (int64_t e = 0; e < n; ++e) rho[e] += w * ki[(size_t)2 * dim * n + e];
        }
    }
    free(us);
    free(ks);
    return 0;
}

/* Vector-Jacobian product of one Runge-Kutta step.  On entry (xb, vb, rb) are
 * the cotangents of the step's output, on exit those of its input.  With the
 * stage states u_i recomputed, stages are taken in reverse:
 *   kbar_i = dt b_i ubar' + dt sum_{l>i} A_li Ubar_l,
 *   Ubar_i = (df/du at u_i)^T kbar_i
 *          = (J_x^T, kbar_x + J_v^T, J_rho^T) applied to (kbar_v, kbar_rho),
 * and ubar = ubar' + sum_i Ubar_i. */
int orc_step_rk_adjoint(const orc_params* p, int64_t n, const double* x, const double* v, const double* rho,
                        int32_t stages, const double* A, const double* b, double* xb, double* vb, double* rb)
{
    if (!valid_params(p) || n < 0 || stages < 1 || stages > 8) return -1;
    int dim = p->dim;
    size_t dn = (size_t)dim * (size_t)n, m = 2 * dn + (size_t)n;
    double* us = (double*)malloc(sizeof(double) * m * (size_t)stages + 1);
    double* ks = (double*)malloc(sizeof(double) * m * (size_t)stages + 1);
    double* Ub = (double*)calloc(m * (size_t)stages + 1, sizeof(double));
    double* kb = (double*)malloc(sizeof(double) * m + 1);
    double* out = (double*)malloc(sizeof(double) * m + 1);
    rk_stages(p, n, x, v, rho, stages, A, us, ks);
    for (int i = stages - 1; i >= 0; --i) {
        for (size_t e = 0; e < dn; ++e) kb[e] = p->dt * b[i] * xb[e];
        for (size_t e = 0; e < dn; ++e) kb[dn + e] = p->dt * b[i] * vb[e];
        for (size_t e = 0; e < (size_t)n; ++e) kb[2 * dn + e] = p->dt * b[i] * rb[e];
        for (int l = i + 1; l < stages; ++l) {
            double a = A[l * stages + i];
            if (a == 0.0) continue;
            const double* Ul = Ub + (size_t)l * m;
            for (size_t e = 0; e < m; ++e) kb[e] += p->dt * a * Ul[e];
        }
        const double* ui = us + (size_t)i * m;
        orc_rhs_vjp(p, n, ui, ui + dn, ui + 2 * dn, kb + dn, kb + 2 * dn, out, out + dn, out + 2 * dn);
        double* Ui = Ub + (size_t)i * m;
        for (size_t e = 0; e < dn; ++e) Ui[e] = out[e];
        for (size_t e = 0; e < dn; ++e) Ui[dn + e] = kb[e] + out[dn + e];
        for (size_t e = 0; e < (size_t)n; ++e) Ui[2 * dn + e] = out[2 * dn + e];
    }
    for (int i = 0; i < stages; ++i) {
        const double* Ui = Ub + (size_t)i * m;
        for (size_t e = 0; e < dn; ++e) xb[e] += Ui[e];
        for (size_t e = 0; e < dn; ++e) vb[e] += Ui[dn + e];
        for (size_t e = 0; e < (size_t)n; ++e) rb[e] += Ui[2 * dn + e];
    }
    free(us);
    free(ks);
    free(Ub);
    free(kb);
    free(out);
    return 0;
}

/* ---------------------------------------------------------------- symplectic Euler
 *
 * The symplectic scheme of DualSPHysics that the paper lists among its
 * integrators (Sec. 3.4 and App. C, citing Dominguez et al. 2022): a
 * position-Verlet predictor-corrector over the update function f = (a, D),
 * D = drho/dt, with h = dt/2:
 *   predictor  x_h = x + h v,  v_h = v + h a1,  rho_h = rho + h D1,
 *              (a1, D1) = f(x, v, rho)
 *   corrector  (a2, D2) = f(x_h, v_h, rho_h)
 *              v' = v + dt a2,  x' = x_h + h v',
 *              rho' = rho (2 - e) / (2 + e),  e = -dt D2 / rho_h.
 * With `reuse`, the rates of a step's last substep, (a2, D2), stand in for
 * f(x, v, rho) in the next step's predictor (the modified scheme of Sec. 3.4
 * and App. C that re-uses the last substep's update values), so a step costs
 * one evaluation of f.  A reusing rollout evaluates f(x, v, rho) afresh at
 * its first step and at every step whose index is a multiple of `restart`
 * (in a checkpointed rollout, the checkpoints, so that each segment can be
 * recomputed on its own).
 */

/* (a, D) = f(x, v, rho), packed as [a (dim*n) | D (n)]. */
static void rates_at(const orc_params* p, int64_t n, const double* x, const double* v, const double* rho,
                     double* r)
{
    int dim = p->dim;
    double* u = (double*)malloc(sizeof(double) * (size_t)dim * (size_t)(n > 0 ? n : 1));
    wrap_all(p, n, x, u);
    nblist nb;
    build_lists(dim, n, x, p->L, p->H, 0, 0, &nb);
    rhs_with_list(p, n, u, v, rho, &nb, r + (size_t)dim * n, r, NULL);
    nblist_free(&nb);
    free(u);
}

/* Predictor state u_h = [x_h | v_h | rho_h] from u and the predictor's rates r1. */
static void symp_predict(const orc_params* p, int64_t n, const double* x, const double* v, const double* rho,
                         const double* r1, double* uh)
{
    size_t dn = (size_t)p->dim * (size_t)n;
    double h = 0.5 * p->dt;
    for (size_t e = 0; e < dn; ++e) uh[e] = x[e] + h * v[e];
    for (size_t e = 0; e < dn; ++e) uh[dn + e] = v[e] + h * r1[e];
    for (int64_t i = 0; i < n; ++i) uh[2 * dn + i] = rho[i] + h * r1[dn + i];
}

/* One step in place with predictor rates r1; the corrector's rates go to r2. */
static void symp_step(const orc_params* p, int64_t n, double* x, double* v, double* rho, const double* r1,
                      double* uh, double* r2)
{
    size_t dn = (size_t)p->dim * (size_t)n;
    double h = 0.5 * p->dt;
    symp_predict(p, n, x, v, rho, r1, uh);
    rates_at(p, n, uh, uh + dn, uh + 2 * dn, r2);
    for (size_t e = 0; e < dn; ++e) {
        v[e] = v[e] + p->dt * r2[e];
        x[e] = uh[e] + h * v[e];
    }
    for (int64_t i = 0; i < n; ++i) {
        double e = -p->dt * r2[dn + i] / uh[2 * dn + i];
        rho[i] = rho[i] * (2.0 - e) / (2.0 + e);
    }
}

/* nsteps steps in place; *evals (if given) receives the number of evaluations of f. */
int orc_step_symplectic(const orc_params* p, int64_t n, double* x, double* v, double* rho, int32_t nsteps,
                        int32_t reuse, int32_t restart, int64_t* evals)
{
    if (!valid_params(p) || n < 0 || nsteps < 0 || (reuse && restart < 1)) return -1;
    size_t dn = (size_t)p->dim * (size_t)n, m = 2 * dn + (size_t)n;
    double* r1 = (double*)malloc(sizeof(double) * (dn + (size_t)n) + 1);
    double* r2 = (double*)malloc(sizeof(double) * (dn + (size_t)n) + 1);
    double* uh = (double*)malloc(sizeof(double) * m + 1);
    int64_t ne = 0;
    for (int32_t t = 0; t < nsteps; ++t) {
        if (!reuse || t % restart == 0) {
            rates_at(p, n, x, v, rho, r1);
            ++ne;
        }
        symp_step(p, n, x, v, rho, r1, uh, r2);
        ++ne;
        memcpy(r1, r2, sizeof(double) * (dn + (size_t)n));
    }
    if (evals) *evals = ne;
    free(r1);
    free(r2);
    free(uh);
    return 0;
}

/* Vector-Jacobian product of one step from u = (x, v, rho) with predictor
 * rates r1.  In: (xb, vb, rb), the cotangents of u', and cb2 (NULL for none),
 * the cotangent of the step's corrector rates (a2, D2) where a later step
 * re-uses them.  Out: (xb, vb, rb), the cotangents of u; if `fresh`, r1 is
 * f(u) and its dependence on u is included, otherwise cb1 receives the
 * cotangent of r1.  Transpose of the corrector, with vt = vb' + h xb':
 *   a2bar = dt vt,  ebar = rb' rho g'(e),  D2bar = -dt ebar / rho_h,
 *   the predictor state's cotangent = J_f(u_h)^T (a2bar, D2bar)
 *     + (xb', 0, ebar dt D2 / rho_h^2),
 * then of the predictor u_h = u + h (v, a1, D1). */
static void symp_step_adjoint(const orc_params* p, int64_t n, const double* x, const double* v,
                              const double* rho, const double* r1, int fresh, double* xb, double* vb, double* rb,
                              const double* cb2, double* cb1)
{
    size_t dn = (size_t)p->dim * (size_t)n, m = 2 * dn + (size_t)n;
    double h = 0.5 * p->dt, dt = p->dt;
    double* uh = (double*)malloc(sizeof(double) * m + 1);
    double* r2 = (double*)malloc(sizeof(double) * (dn + (size_t)n) + 1);
    double* r2b = (double*)malloc(sizeof(double) * (dn + (size_t)n) + 1);
    double* vt = (double*)malloc(sizeof(double) * dn + 1);
    double* rdir = (double*)malloc(sizeof(double) * (size_t)n + 1);
    double* uhb = (double*)calloc(m + 1, sizeof(double));
    symp_predict(p, n, x, v, rho, r1, uh);
    const double* rh = uh + 2 * dn;
    rates_at(p, n, uh, uh + dn, rh, r2);
    for (size_t e = 0; e < dn; ++e) {
        vt[e] = vb[e] + h * xb[e];
        r2b[e] = dt * vt[e] + (cb2 ? cb2[e] : 0.0);
    }
    double* rhb = (double*)malloc(sizeof(double) * (size_t)n + 1);
    for (int64_t i = 0; i < n; ++i) {
        double D2 = r2[dn + i];
        double e = -dt * D2 / rh[i];
        double g = (2.0 - e) / (2.0 + e);
        double gp = -4.0 / ((2.0 + e) * (2.0 + e));
        double eb = rb[i] * rho[i] * gp;
        r2b[dn + i] = -dt * eb / rh[i] + (cb2 ? cb2[dn + i] : 0.0);
        rhb[i] = eb * dt * D2 / (rh[i] * rh[i]);
        rdir[i] = rb[i] * g;
    }
    orc_rhs_vjp(p, n, uh, uh + dn, rh, r2b, r2b + dn, uhb, uhb + dn, uhb + 2 * dn);
    for (size_t e = 0; e < dn; ++e) uhb[e] += xb[e];
    for (int64_t i = 0; i < n; ++i) uhb[2 * dn + i] += rhb[i];
    /* the predictor u_h = (x + h v, v + h a1, rho + h D1) */
    for (size_t e = 0; e < dn; ++e) {
        xb[e] = uhb[e];
        vb[e] = vt[e] + uhb[dn + e] + h * uhb[e];
    }
    for (int64_t i = 0; i < n; ++i) rb[i] = rdir[i] + uhb[2 * dn + i];
    double* r1b = (double*)malloc(sizeof(double) * (dn + (size_t)n) + 1);
    for (size_t e = 0; e < dn; ++e) r1b[e] = h * uhb[dn + e];
    for (int64_t i = 0; i < n; ++i) r1b[dn + i] = h * uhb[2 * dn + i];
    if (fresh) {
        double* out = (double*)malloc(sizeof(double) * m + 1);
        orc_rhs_vjp(p, n, x, v, rho, r1b, r1b + dn, out, out + dn, out + 2 * dn);
        for (size_t e = 0; e < dn; ++e) {
            xb[e] += out[e];
            vb[e] += out[dn + e];
        }
        for (int64_t i = 0; i < n; ++i) rb[i] += out[2 * dn + i];
        free(out);
    } else {
        memcpy(cb1, r1b, sizeof(double) * (dn + (size_t)n));
    }
    free(uh);
    free(r2);
    free(r2b);
    free(vt);
    free(rdir);
    free(uhb);
    free(rhb);
    free(r1b);
}

/* VJP of one step whose predictor evaluates f(u) (a step without a re-used
 * substep): (xb, vb, rb) from the cotangents of u' to those of u. */
int orc_step_symplectic_adjoint(const orc_params* p, int64_t n, const double* x, const double* v,
                                const double* rho, double* xb, double* vb, double* rb)
{
    if (!valid_params(p) || n < 0) return -1;
    size_t dn = (size_t)p->dim * (size_t)n;
    double* r1 = (double*)malloc(sizeof(double) * (dn + (size_t)n) + 1);
    rates_at(p, n, x, v, rho, r1);
    symp_step_adjoint(p, n, x, v, rho, r1, 1, xb, vb, rb, NULL, NULL);
    free(r1);
    return 0;
}

/* Gradient through a whole rollout of nsteps steps from (x, v, rho): on
 * entry (xb, vb, rb) are the cotangents of the final state, on exit those of
 * the initial one.  With reuse, the re-used rates carry cotangents from each
 * step to the one before it. */
int orc_rollout_symplectic_adjoint(const orc_params* p, int64_t n, const double* x, const double* v,
                                   const double* rho, int32_t nsteps, int32_t reuse, int32_t restart, double* xb,
                                   double* vb, double* rb)
{
    if (!valid_params(p) || n < 0 || nsteps < 0 || (reuse && restart < 1)) return -1;
    size_t dn = (size_t)p->dim * (size_t)n, m = 2 * dn + (size_t)n, nr = dn + (size_t)n;
    double* us = (double*)malloc(sizeof(double) * m * (size_t)(nsteps + 1) + 1);
    double* rs = (double*)malloc(sizeof(double) * nr * (size_t)(nsteps + 1) + 1);
    double* uh = (double*)malloc(sizeof(double) * m + 1);
    double* r2 = (double*)malloc(sizeof(double) * nr + 1);
    double* cb = (double*)calloc(nr + 1, sizeof(double));
    double* cb_prev = (double*)calloc(nr + 1, sizeof(double));
    memcpy(us, x, sizeof(double) * dn);
    memcpy(us + dn, v, sizeof(double) * dn);
    memcpy(us + 2 * dn, rho, sizeof(double) * (size_t)n);
    for (int32_t t = 0; t < nsteps; ++t) {
        double* ut = us + (size_t)t * m;
        double* un = us + (size_t)(t + 1) * m;
        double* rt = rs + (size_t)t * nr;
        if (!reuse || t % restart == 0) rates_at(p, n, ut, ut + dn, ut + 2 * dn, rt);
        else memcpy(rt, r2, sizeof(double) * nr);
        memcpy(un, ut, sizeof(double) * m);
        symp_step(p, n, un, un + dn, un + 2 * dn, rt, uh, r2);
    }
    int carry = 0;  /* cb holds the cotangent of step t's corrector rates */
    for (int32_t t = nsteps - 1; t >= 0; --t) {
        double* ut = us + (size_t)t * m;
        int fresh = !reuse || t % restart == 0;
        symp_step_adjoint(p, n, ut, ut + dn, ut + 2 * dn, rs + (size_t)t * nr, fresh, xb, vb, rb,
                          carry ? cb : NULL, cb_prev);
        carry = !fresh;
        if (carry) memcpy(cb, cb_prev, sizeof(double) * nr);
    }
    free(us);
    free(rs);
    free(uh);
    free(r2);
    free(cb);
    free(cb_prev);
    return 0;
}

/* ---------------------------------------------------------------- particle shifting
 *
 * Explicit particle shifting, applied as a post-processing step to a state
 * (Sec. 3.4 and App. C place it at the end of a time step; the paper cites the
 * delta-plus scheme of Sun et al. without printing it).  The published form:
 *   dr_i = -beta H^2 sum_j [1 + R (W_ij / W(dx))^4] V_j grad_i W_ij,
 * R = 0.2, dx = (m / rho0)^(1/d) the initial spacing, V_j = m / rho_j, and
 * beta (the scheme's CFL Ma) a parameter; x <- x + dr, velocities and
 * densities unchanged.  With V_j = V the shift is a descent step on
 *   E = sum_i sum_j V [W_ij + R W_ij^5 / (5 W(dx)^4)].
 */
#define ORC_SHIFT_R 0.2

static double shift_w0(const orc_params* p)
{
    double dx = pow(p->m / p->rho0, 1.0 / p->dim);
    double e[3] = {dx, 0.0, 0.0};
    return orc_w(p->dim, p->H, e);
}

/* dr (dim*n) for the state (x, rho). */
int orc_shift(const orc_params* p, int64_t n, const double* x, const double* rho, double beta, double* dr)
{
    if (!valid_params(p) || n < 0) return -1;
    int dim = p->dim;
    double invL = 1.0 / p->L, w0 = shift_w0(p), c = -beta * p->H * p->H;
    double* u = (double*)malloc(sizeof(double) * (size_t)dim * (size_t)(n > 0 ? n : 1));
    wrap_all(p, n, x, u);
    nblist nb;
    build_lists(dim, n, x, p->L, p->H, 0, 0, &nb);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double ui[3] = {0, 0, 0}, s[3] = {0, 0, 0};
        for (int k = 0; k < dim; ++k) ui[k] = u[k * n + i];
        for (int64_t q = nb.off[i]; q < nb.off[i + 1]; ++q) {
            int64_t j = nb.idx[q];
            if (j == i) continue;
            double uj[3] = {0, 0, 0}, e[3] = {0, 0, 0}, w[3] = {0, 0, 0};
            for (int k = 0; k < dim; ++k) uj[k] = u[k * n + j];
            minimg(dim, ui, uj, p->L, invL, e);
            orc_gradw(dim, p->H, e, w);
            double rW = orc_w(dim, p->H, e) / w0;
            double phi = 1.0 + ORC_SHIFT_R * rW * rW * rW * rW;
            double Vj = p->m / rho[j];
            for (int k = 0; k < dim; ++k) s[k] += phi * Vj * w[k];
        }
        for (int k = 0; k < dim; ++k) dr[k * n + i] = c * s[k];
    }
    nblist_free(&nb);
    free(u);
    return 0;
}

/* Vector-Jacobian product of x' = x + dr(x, rho) for cotangents xb of x':
 * gx = J_x^T xb and gr = J_rho^T xb are written (the identity part, xb itself,
 * is the caller's).  Scatter form over the lists: with h(r) = phi(r) g(r),
 * grad_i W_ij = g e (e = x_i - x_j), dr_i += c V_j h e, c = -beta H^2:
 *   d(h e)/de = h I + (h'(r) / r) e e^T,
 *   x_i += c V_j D^T xb_i,  x_j -= c V_j D^T xb_i,
 *   rho_j += -(V_j / rho_j) c h (e . xb_i). */
int orc_shift_vjp(const orc_params* p, int64_t n, const double* x, const double* rho, double beta,
                  const double* xb, double* gx, double* gr)
{
    if (!valid_params(p) || n < 0) return -1;
    int dim = p->dim;
    double invL = 1.0 / p->L, w0 = shift_w0(p), c = -beta * p->H * p->H;
    double* u = (double*)malloc(sizeof(double) * (size_t)dim * (size_t)(n > 0 ? n : 1));
    wrap_all(p, n, x, u);
    nblist nb;
    build_lists(dim, n, x, p->L, p->H, 0, 0, &nb);
    for (int64_t e0 = 0; e0 < (int64_t)dim * n; ++e0) gx[e0] = 0.0;
    for (int64_t i = 0; i < n; ++i) gr[i] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double ui[3] = {0, 0, 0}, xbi[3] = {0, 0, 0};
        for (int k = 0; k < dim; ++k) {
            ui[k] = u[k * n + i];
            xbi[k] = xb[k * n + i];
        }
        for (int64_t q = nb.off[i]; q < nb.off[i + 1]; ++q) {
            int64_t j = nb.idx[q];
            if (j == i) continue;
            double uj[3] = {0, 0, 0}, e[3] = {0, 0, 0}, w[3] = {0, 0, 0}, Hs[9];
            for (int k = 0; k < dim; ++k) uj[k] = u[k * n + j];
            minimg(dim, ui, uj, p->L, invL, e);
            orc_gradw(dim, p->H, e, w);
            orc_hessw(dim, p->H, e, Hs);
            double Wr = orc_w(dim, p->H, e), rW = Wr / w0;
            double phi = 1.0 + ORC_SHIFT_R * rW * rW * rW * rW;
            /* d phi / de = 4 R (W/w0)^3 grad W / w0 */
            double dphi = 4.0 * ORC_SHIFT_R * rW * rW * rW / w0;
            double Vj = p->m / rho[j];
            /* the shift term t = phi(e) w(e); dt/de = phi Hess + w (dphi w)^T */
            double wx = 0.0;
            for (int k = 0; k < dim; ++k) wx += w[k] * xbi[k];
            for (int a = 0; a < dim; ++a) {
                double g = 0.0;
                for (int b = 0; b < dim; ++b) g += phi * Hs[b * dim + a] * xbi[b];
                g += dphi * w[a] * wx;
                gx[a * n + i] += c * Vj * g;
                gx[a * n + j] -= c * Vj * g;
            }
            gr[j] += -(Vj / rho[j]) * c * phi * wx;
        }
    }
    nblist_free(&nb);
    free(u);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Neighbour search with per-particle support radii (Sec. 3.2,         */
/* "Ensuring symmetric interactions"; App. B, the search-radius step)  */
/* ------------------------------------------------------------------ */

/* Each particle i carries its own support h_i.  Steps, in the paper's order:
 *   1. search radius: s_k starts at h_k and is raised to h_i for every particle
 *      i that has k as a neighbour under its own support (r_ik < h_i); written
 *      here as the definition s_k = max(h_k, max{h_i : r_ik < h_i}), gathered
 *      per k (the paper's atomic maximum reaches the same value in any order);
 *   2. neighbourhood construction: particle i searches with s_i and keeps the
 *      pairs of the super-symmetric set, r_ij < max(h_i, h_j).
 * Every pair with r_ij < max(h_i, h_j) is found by the search of step 2: if
 * h_i >= h_j it lies within h_i <= s_i, else i is a neighbour of j under h_j and
 * step 1 raised s_i to at least h_j.  Predicates as for a uniform support:
 * strict r^2 < h^2 with h^2 = h * h rounded once, on wrapped positions, in the
 * working precision (prec 1: positions and supports first rounded to float).
 * Candidates come from a bucket grid of cells of side >= 1.01 max_i h_i (or all
 * particles when brute != 0).  Rows ascending, self included.  s (n values) is
 * written when non-null.  Returns the total number of entries (offsets always
 * written, nbr when cap >= total), or -1 on bad input (h_i <= 0, non-finite h_i,
 * or 2 max h_i >= L). */
int64_t orc_neighbors_adaptive(int dim, int64_t n, const double* x, double L, const double* h, int prec,
                               int brute, int64_t* offsets, int32_t* nbr, int64_t cap, double* s_out)
{
    if ((dim != 2 && dim != 3) || n < 0) return -1;
    double hmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!(h[i] > 0.0) || !isfinite(h[i])) return -1;
        if (h[i] > hmax) hmax = h[i];
    }
    if (n > 0 && !(2.0 * hmax < L)) return -1;
    size_t nn = (size_t)(n > 0 ? n : 1);
    double* u = (double*)malloc(sizeof(double) * (size_t)dim * nn);
    float* uf = (float*)malloc(sizeof(float) * (size_t)dim * nn);
    double* hh = (double*)malloc(sizeof(double) * nn);   /* h_i in the working precision */
    double* sr = (double*)malloc(sizeof(double) * nn);   /* search radius s_i */
    double invL = 1.0 / L;
    float Lf = (float)L, invLf = 1.0f / Lf;
    for (int64_t i = 0; i < n; ++i) {
        hh[i] = prec == 1 ? (double)(float)h[i] : h[i];
        for (int k = 0; k < dim; ++k) {
            if (prec == 1) {
                uf[k * n + i] = wrap_f32((float)x[k * n + i], Lf, invLf);
                u[k * n + i] = (double)uf[k * n + i];
            } else {
                u[k * n + i] = wrap_f64(x[k * n + i], L, invL);
            }
        }
    }
    grid g;
    grid_build(&g, dim, n, u, L, hmax > 0.0 ? hmax : 0.25 * L, brute);

    /* r_ij^2 < rad^2 in the working precision */
#define ORC_WITHIN(i_, j_, rad_)                                                           \
    (prec == 1 ? within_f32(dim, fi_##i_, fj_##j_, Lf, invLf, (float)(rad_) * (float)(rad_)) \
               : within_f64(dim, di_##i_, dj_##j_, L, invL, (rad_) * (rad_)))

    /* step 1: search radii */
#pragma omp parallel
    {
        int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * nn);
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < n; ++k) {
            float fi_a[3] = {0, 0, 0}, fj_b[3] = {0, 0, 0};
            double di_a[3] = {0, 0, 0}, dj_b[3] = {0, 0, 0};
            for (int c = 0; c < dim; ++c) {
                fj_b[c] = uf[c * n + k];
                dj_b[c] = u[c * n + k];
            }
            double sk = hh[k];
            int64_t nc = grid_candidates(&g, k, buf);
            for (int64_t a = 0; a < nc; ++a) {
                int64_t i = buf[a];
                for (int c = 0; c < dim; ++c) {
                    fi_a[c] = uf[c * n + i];
                    di_a[c] = u[c * n + i];
                }
                /* is k a neighbour of i under i's own support? */
                if (ORC_WITHIN(a, b, hh[i]) && hh[i] > sk) sk = hh[i];
            }
            sr[k] = sk;
        }
        free(buf);
    }

    /* step 2: search with s_i, keep r_ij < max(h_i, h_j) */
    int64_t* cnt = (int64_t*)calloc(nn, sizeof(int64_t));
    offsets[0] = 0;
    int64_t total = 0;
    int32_t* idx = NULL;
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            for (int64_t i = 0; i < n; ++i) offsets[i + 1] = offsets[i] + cnt[i];
            total = offsets[n];
            idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
        }
#pragma omp parallel
        {
            int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * nn);
#pragma omp for schedule(dynamic, 64)
            for (int64_t i = 0; i < n; ++i) {
                float fi_a[3] = {0, 0, 0}, fj_b[3] = {0, 0, 0};
                double di_a[3] = {0, 0, 0}, dj_b[3] = {0, 0, 0};
                for (int c = 0; c < dim; ++c) {
                    fi_a[c] = uf[c * n + i];
                    di_a[c] = u[c * n + i];
                }
                int64_t nc = grid_candidates(&g, i, buf);
                int64_t c0 = 0, base = pass == 1 ? offsets[i] : 0;
                for (int64_t a = 0; a < nc; ++a) {
                    int64_t j = buf[a];
                    for (int c = 0; c < dim; ++c) {
                        fj_b[c] = uf[c * n + j];
                        dj_b[c] = u[c * n + j];
                    }
                    double hm = hh[i] > hh[j] ? hh[i] : hh[j];
                    if (ORC_WITHIN(a, b, sr[i]) && ORC_WITHIN(a, b, hm)) {
                        if (pass == 1) idx[base + c0] = (int32_t)j;
                        ++c0;
                    }
                }
                if (pass == 0) cnt[i] = c0;
                else qsort(idx + base, (size_t)c0, sizeof(int32_t), cmp_i32);
            }
            free(buf);
        }
    }
#undef ORC_WITHIN
    if (nbr && cap >= total && total > 0) memcpy(nbr, idx, sizeof(int32_t) * (size_t)total);
    if (s_out)
        for (int64_t i = 0; i < n; ++i) s_out[i] = sr[i];
    free(idx);
    free(cnt);
    grid_free(&g);
    free(u);
    free(uf);
    free(hh);
    free(sr);
    return total;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
