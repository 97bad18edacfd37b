/*
 * sph.h -- C ABI of libsph, the MI355X (gfx950) hot path of differentiable
 * weakly compressible SPH: cell-list neighbour search, the fused delta-SPH
 * pair sweeps, a fixed-step semi-implicit Euler integrator, and the adjoint
 * of one step.
 *
 * Paper: diffSPH, Winchenbach & Thuerey, arXiv 2507.21684.  The problem
 * statement the calls follow (Sec. 2.2): a state u = (x, f, sigma) is
 * advanced by a step P built from an update function f : P x C -> U (the
 * time derivatives, App. C) and a neighbourhood function g (App. B); its
 * gradient is the vector-Jacobian product (dP/du)^T a.
 *
 * Conventions shared by every call
 *  - Memory: the library never allocates device memory.  The caller owns the
 *    state, the outputs, the checkpoints and one workspace whose size
 *    sph_workspace_size() reports, or binds the library's static per-device
 *    workspace with sph_bind_scratch().  All pointers named "device" point to
 *    GPU memory; "host" pointers to CPU memory.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 *    stream).  Calls enqueue work asynchronously on it unless documented as
 *    synchronous.  Calls on one plan must be ordered (one stream, or the
 *    caller's own synchronisation); distinct plans are independent.
 *  - Batches: a plan describes nsims independent simulations of one
 *    dimension and one dtype, packed back to back: simulation s owns
 *    particles [off_s, off_s + counts[s]) of every array, off_s being the
 *    sum of the earlier counts.  A single simulation is a batch of one; there
 *    is one code path.
 *  - State layout: SoA in the plan's dtype (float for SPH_F32, double for
 *    SPH_F64), in the caller's particle order ("original order").
 *    x[k] is coordinate k (k < dim) of all packed particles, likewise v[k].
 *    Positions are unwrapped (absolute); the periodic box is applied inside
 *    (Sec. 3.2, "Periodic Boundary Conditions").
 *  - Errors: every call returns an sph_status; it never throws.  The return
 *    code covers argument checks and launch errors.  Faults detected on the
 *    device (non-finite values, neighbour-list overflow) are recorded per
 *    simulation and read with sph_poll().  sph_last_error() returns a
 *    thread-local message for the last failing call of the calling thread.
 *  - Determinism: results are bitwise reproducible for identical inputs, and
 *    a simulation's results do not depend on which other simulations share
 *    its batch (every particle sums its neighbours in a fixed order: stencil
 *    cells by relative offset, then particles by original index).
 */
#ifndef SPH_H
#define SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sph_status;

#define SPH_OK 0
#define SPH_ERR_INVALID_ARG (-1)   /* bad dim/dtype/pointer/size, or H >= L/2 */
#define SPH_ERR_TOO_FEW_CELLS (-2) /* fewer than 3 cells of side >= H per box side */
#define SPH_ERR_CAPACITY (-3)      /* an output or neighbour list is too small */
#define SPH_ERR_NONFINITE (-4)     /* a non-finite value was found on the device */
#define SPH_ERR_DEVICE (-5)        /* a HIP call failed */
#define SPH_ERR_UNSUPPORTED (-6)
#define SPH_ERR_STATE (-7)         /* call order violated (e.g. plan not bound) */

/* per-simulation device status bits, read by sph_poll() */
#define SPH_FLAG_NONFINITE 1
#define SPH_FLAG_NEIGHBOR_OVERFLOW 2
#define SPH_FLAG_SKIN 4 /* with list reuse: a particle moved more than its half skin h_i (see
                           sph_params.skin) since its lists were built, so a pair may be
                           missing; rerun with a larger skin or a shorter reuse interval */

#define SPH_F32 0
#define SPH_F64 1

/* Parameters of one simulation (Sec. 2.3 governing equations, App. A.1 kernel,
 * Sec. 3.4 fixed time step).  "support" is the kernel support radius H, the
 * distance at which the Wendland-C4 kernel vanishes; the paper stores the
 * support under the name h (App. A.1), and H is what enters delta*H*c0 and
 * alpha*H*c0.  The time step is the caller's `dt`: the workloads of this
 * library take dt = 0.25 h / c0 with the smoothing length h = H / 2, i.e.
 * dt = 0.125 H / c0 (the acoustic condition of Sec. 3.4 read with the
 * literature's H / h = 2 of App. A.1; with h = H the Taylor-Green flows blow
 * up within about a hundred steps). */
typedef struct sph_params {
    int32_t dim;      /* 2 or 3 */
    int32_t dtype;    /* SPH_F32 or SPH_F64; equal for every simulation of a plan */
    double box;       /* periodic box side L (the box is [0, L)^dim) */
    double support;   /* H; must satisfy 2 H < L */
    double mass;      /* particle mass m (equal for all particles of the simulation) */
    double rho0;      /* rest density of the Tait equation of state */
    double c0;        /* speed of sound */
    double delta;     /* delta-SPH density-diffusion coefficient */
    double alpha;     /* artificial-viscosity coefficient */
    double eps;       /* regulariser in 1/(r^2 + eps H^2) */
    double dt;        /* fixed time step */
    double skin;      /* neighbour-list skin as a fraction of the support.  Each particle
                         gets a half skin h_i (skin H / 2, or less with speed-scaled skins,
                         see sph_set_skin_mode), the lists hold the pairs with
                         r < H + h_i + h_j <= H (1 + skin), and the sweeps keep those with
                         r < H; 0 = lists of exactly the pairs with r < H.  Needs
                         2 H (1 + skin) < L.  Cells are sized for H (1 + skin). */
} sph_params;

/* Device pointers to one packed state in the plan's dtype.  Entries k >= dim
 * of x and v are ignored. */
typedef struct sph_state {
    void* x[3];
    void* v[3];
    void* rho;
} sph_state;

typedef struct sph_plan sph_plan;

/* Create a host-side plan for nsims simulations.  sims[s] (host) holds the
 * parameters of simulation s and counts[s] (host) its particle count (>= 0).
 * max_neighbors bounds the neighbours stored per particle, self included
 * (0 = automatic: 1.6 times the particles of a support sphere at the initial
 * spacing implied by mass and rho0; rounded up to a multiple of 8).
 * tape_depth is the number of steps whose sorted states and neighbour lists
 * the workspace can hold at once; sph_rollout_backward() needs it to be at
 * least the checkpoint interval (0 = no tape).  Allocates host memory only.
 * Errors: INVALID_ARG, TOO_FEW_CELLS (cells per side are chosen with side
 * >= H/2 (1 + 2^-10), at least 5 of them, else side >= H (1 + 2^-10), at
 * least 3 of them), UNSUPPORTED (more than 2^31 particles or 1024 cell blocks
 * of 4^2 / 2^3 cells per side). */
sph_status sph_plan_create(const sph_params* sims, int32_t nsims, const int64_t* counts,
                           int32_t max_neighbors, int32_t tape_depth, sph_plan** out);

/* Destroy a plan (host memory only; the workspace stays the caller's). */
void sph_plan_destroy(sph_plan* plan);

/* Workspace bytes the plan needs (host out-parameter). */
sph_status sph_workspace_size(const sph_plan* plan, size_t* bytes);

/* Total particles, simulations and the neighbour-list width of the plan. */
sph_status sph_plan_info(const sph_plan* plan, int64_t* total_particles, int32_t* nsims,
                         int32_t* max_neighbors);

/* Lanes that share one particle in the forward sweep and in the adjoint sweep
 * (2, 4 or 8; default 4).  A particle's pair sums are always formed as eight
 * partial sums over list positions k mod 8 combined by the balanced tree
 * ((s0 + s1) + (s2 + s3)) + ((s4 + s5) + (s6 + s7)), so results are bitwise
 * the same for every setting; only speed changes.  INVALID_ARG otherwise. */
sph_status sph_set_tuning(sph_plan* plan, int32_t lanes_fwd, int32_t lanes_adj);
sph_status sph_get_tuning(const sph_plan* plan, int32_t* lanes_fwd, int32_t* lanes_adj);

/* Time integrator (Sec. 3.4; the time-stepping appendix describes explicit
 * schemes by their Butcher tableau).  stages = 0 selects the default
 * semi-implicit Euler step (v' = v + dt a, rho' = rho + dt drho/dt,
 * x' = x + dt v').  stages = 1..4 selects the explicit Runge-Kutta scheme with
 * the tableau A (host, stages x stages, row-major, strictly lower triangular)
 * and weights b (host, stages) for the state u = (x, v, rho) with
 * du/dt = f(u) = (v, a(u), drho/dt(u)):
 *     u_i = u + dt sum_{j<i} A_ij k_j,  k_i = f(u_i),  u' = u + dt sum_i b_i k_i.
 * Without a list skin every stage sorts its state and builds its own neighbour
 * lists.  With a skin in the plan's parameters only the first stage of a step
 * sorts and builds; the later stages are gathered into its particle order, use
 * its lists filtered to r < H (so every stage still evaluates exactly its own
 * pair set), and set SPH_FLAG_SKIN when a particle moved more than its half
 * skin since the build.  The reuse interval of sph_set_reuse applies to the
 * semi-implicit Euler step only.  sph_step, sph_step_adjoint and
 * sph_rollout_backward then use the scheme; the adjoint reverses the stages
 * over the update function's VJP.  The first call with stages > 0 reserves the
 * stage storage and so grows sph_workspace_size(): make it before sph_bind
 * (CAPACITY afterwards).  INVALID_ARG for stages outside 0..4, null arrays,
 * non-finite entries, or a tableau that is not explicit. */
sph_status sph_set_integrator(sph_plan* plan, int32_t stages, const double* A, const double* b);

/* Symplectic Euler of DualSPHysics, the other integrator Sec. 3.4 and App. C
 * name: with h = dt/2 and (a, D) = f(u) the update function's acceleration and
 * density rate,
 *     predictor  u_h = (x + h v, v + h a1, rho + h D1),  (a1, D1) = f(u),
 *     corrector  (a2, D2) = f(u_h),  v' = v + dt a2,  x' = x_h + h v',
 *                rho' = rho (2 - e) / (2 + e),  e = -dt D2 / rho_h,
 * each evaluation of f with its own sort and neighbour lists; with a list
 * skin, a corrector that follows an evaluation of f(u) in the same step keeps
 * that evaluation's particle order and lists (filtered to r < H, displacement
 * checked against each particle's half skin as for Runge-Kutta stages).  With
 * reuse_last_substep != 0, the predictor takes the previous step's corrector
 * rates (a2, D2) instead of evaluating f(u) (the modified scheme of Sec. 3.4 /
 * App. C that re-uses the last substep's update values): one evaluation of f
 * per step.  The rates are evaluated afresh at the first step of every sph_step
 * call and, when the call writes checkpoints, at every checkpoint, so each
 * checkpoint segment can be recomputed on its own; sph_rollout_backward follows
 * the same schedule and carries the re-used rates' cotangents from step to step.
 * sph_step_adjoint is the adjoint of one step whose predictor evaluates f(u).
 * sph_set_integrator(plan, 0, NULL, NULL) returns to semi-implicit Euler.  The
 * first call reserves the stage storage and a tape of tape_depth rate blocks
 * and so grows sph_workspace_size(): make it before sph_bind (CAPACITY
 * afterwards).  Host-side setting. */
sph_status sph_set_symplectic(sph_plan* plan, int32_t reuse_last_substep);

/* delta-diffusion with the renormalised density gradient (the full delta-SPH
 * diffusion that Sec. 2.3 cites; the renormalisation of App. A.5).  With
 * renormalised != 0 every evaluation of the update function first forms, per
 * particle, G_i = L_i sum_j V_j (rho_j - rho_i) grad_i W_ij with
 * L_i = [sum_j V_j (x_j - x_i) (x) grad_i W_ij]^-1 (exact inverse; a singular
 * matrix gives G_i = 0), and adds
 *     -delta H c0 sum_j V_j (G_i + G_j) . grad_i W_ij
 * to drho_i/dt.  Applies to sph_rhs, sph_step, sph_step_adjoint and
 * sph_rollout_backward under every integrator; the adjoint adds the term's
 * vector-Jacobian product (two extra list passes).  0 returns to the
 * Molteni-Colagrossi term alone (the default).  The first call with a non-zero
 * value reserves three records per particle and so grows sph_workspace_size():
 * make it before sph_bind (CAPACITY afterwards).  Host-side setting. */
sph_status sph_set_diffusion(sph_plan* plan, int32_t renormalised);

/* Explicit particle shifting, the post-processing step Sec. 3.4 and App. C
 * apply at the end of a time step (the delta-plus form the paper cites):
 *     dr_i = -beta H^2 sum_j [1 + 0.2 (W_ij / W(dx))^4] V_j grad_i W_ij,
 * V_j = m / rho_j, dx = (m / rho0)^(1/dim) the initial spacing; x <- x + dr in
 * place (device state, original order; velocities and densities unchanged).
 * beta is the scheme's CFL Ma (dimensionless).  Sorts the state and builds its
 * lists (the plan's skin and lanes apply).  Compose it with sph_step calls of
 * one step to shift after every step.  INVALID_ARG for a non-finite beta. */
sph_status sph_shift(sph_plan* plan, sph_state* state, double beta, void* stream);

/* Vector-Jacobian product of sph_shift at `state` (the state before the shift):
 * cot holds the cotangents of the shifted state on entry and those of `state`
 * on exit (positions gain J_x^T xbar, densities J_rho^T xbar; velocities are
 * unchanged).  The state is not modified. */
sph_status sph_shift_adjoint(sph_plan* plan, const sph_state* state, sph_state* cot, double beta, void* stream);

/* Neighbour-list reuse (Verlet lists; the paper keeps one list for short rollouts,
 * Sec. 4.1).  With rebuild_every = R > 1 (needs a skin in every simulation's
 * parameters), a step sorts and rebuilds its lists only when its index within the
 * call is a multiple of R; the steps in between keep the particle order and the
 * lists of the last build, and their sweeps keep only the pairs with r < H, so
 * every step still evaluates exactly the pairs the method defines.  Each sweep
 * that hands its state to a reusing step checks every particle's displacement
 * since the build against its half skin h_i (see sph_params.skin) and sets
 * SPH_FLAG_SKIN if it is exceeded.
 * A call that spans more than one checkpoint interval needs the interval to be a
 * multiple of R (INVALID_ARG otherwise), so a backward recomputation, which starts
 * every segment with a build, follows the forward's build schedule exactly.  Results differ from R = 1 only
 * by summation order (the lists hold extra entries); they stay deterministic and
 * independent of the batch.  Host-side setting; default 1.  INVALID_ARG for
 * R < 1, or R > 1 without a skin. */
sph_status sph_set_reuse(sph_plan* plan, int32_t rebuild_every);

/* Half skins of the lists a skin gives (not in the paper, which keeps one list
 * radius; a choice of how many candidate pairs the lists carry).  Uniform
 * (speed_scaled = 0, the default): every particle's half skin is h = skin H / 2.
 * Speed-scaled (speed_scaled != 0): at each build particle i gets
 *     h_i = min(skin H / 2, skin H / 16 + 1.3 R dt |v_i|)
 * from its speed (R the reuse interval of sph_set_reuse, 1 by default, which also
 * covers the stages of a Runge-Kutta or symplectic step), so slow particles carry
 * shorter lists.  The
 * skin H / 16 term is every particle's allowance for acceleration between
 * builds; a skin sized as 2.6 v_max dt R / H for the simulation's largest speed
 * v_max lets a particle at rest accelerate steadily to about a third of v_max.
 * Either way the sweeps keep exactly the pairs with r < H, the displacement check
 * uses each particle's own h_i (SPH_FLAG_SKIN), and results stay deterministic
 * and independent of the batch; the two modes differ in summation order only.
 * Host-side setting.  INVALID_ARG for speed_scaled != 0 without a skin. */
sph_status sph_set_skin_mode(sph_plan* plan, int32_t speed_scaled);

/* Graph mode (default off; host-side switch, no device work).  When on, every
 * sph_step and sph_rollout_backward call is issued as one executable HIP graph
 * holding all of the call's launches (the fixed-step loop of Sec. 3.3 has no
 * data-dependent control flow, so a call's launch sequence depends only on its
 * arguments).  A graph is captured on the plan's private stream the first time
 * a given argument set is seen (nsteps, ckpt_every, every state, checkpoint
 * and cotangent pointer, the lanes settings), kept in a cache of 8 entries per
 * plan (least recently used evicted), and launched on the caller's stream;
 * later calls with the same arguments only launch it.  Results are bitwise
 * those of the direct path.  Calls made while profiling is enabled run
 * directly.  Turning the mode off, or sph_bind, drops the cached graphs.  The
 * graphs contain kernel and device-to-device copy nodes only (no memset nodes).
 * DEVICE if capture or instantiation fails. */
sph_status sph_set_graphs(sph_plan* plan, int32_t enable);

/* Bind a device workspace of at least sph_workspace_size() bytes, 256-byte
 * aligned: copies the per-simulation constants and the cell-block tables into
 * it and fills the particle -> simulation and cell -> simulation tables on the
 * device (asynchronous on stream; host work is O(simulations + cell blocks)).
 * The workspace must stay valid until the plan is destroyed or rebound.  A
 * plan may be rebound at any time, e.g. several plans taking turns on one
 * workspace on one stream; rebinding drops cached graphs and clears the
 * plan's status words and pair counter. */
sph_status sph_bind(sph_plan* plan, void* workspace, size_t bytes, void* stream);

/* Size in bytes of the static workspace of sph_bind_scratch (64 MiB per device). */
#define SPH_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): sph_bind with the library's own static
 * workspace instead of one the caller allocated.  The workspace is a device array of
 * SPH_SCRATCH_BYTES bytes that every device the library runs on holds from the library's
 * load until the process ends; its address on the current device is looked up on the first
 * call on that device.  The call allocates nothing (no hipMalloc/hipFree, no allocating
 * library routine); it copies the plan's tables into the array and clears the status words,
 * the pair counter and the sort's counters with fill kernels, as sph_bind does, so nothing
 * of an earlier plan's contents is read.  Every later call on the plan then works on that
 * array and must be made with the same device current (STATE otherwise).  One array per
 * device is shared by every plan bound to it: binding another plan there makes the calls of
 * the earlier one fail with STATE until it is bound again, and calls of plans that overlap
 * on one device race (call it from one thread per device, or order the calls yourself).
 * sph_bind() of the caller's own workspace ends the plan's use of the array.  Errors:
 * CAPACITY when sph_workspace_size() exceeds SPH_SCRATCH_BYTES (checked before any device
 * call), INVALID_ARG for a null plan, DEVICE when the array's address cannot be obtained. */
sph_status sph_bind_scratch(sph_plan* plan, void* stream);

/* Cell list of the state s (App. B, steps 1-2): every particle is mapped into
 * the box, assigned to its cell, and the particles are counting-sorted by
 * cell (cells in Morton order of cell blocks) with ties ordered by original
 * index.  The sorted copy lives in the workspace and is what the other calls
 * use; this call exists to time and test the sort on its own. */
sph_status sph_build_cells(sph_plan* plan, const sph_state* s, void* stream);

/* Neighbour lists of the state s (App. B step 3, Sec. 3.2): for every
 * particle i the set N(i) = { j : |x_i - x_j| < H } (minimum image, self
 * included) as CSR over original indices, each row ascending.  The
 * predicate is evaluated in the plan's dtype, in this order and with no fused
 * multiply-add: u = x - L floor(x (1/L)); d = u_i - u_j; d = d - L rint(d (1/L));
 * r2 = (d0 d0 + d1 d1) + d2 d2; r2 < H H.
 * offsets (device, int64[N+1]) receives row starts; nbr (device,
 * int32[capacity]) the entries.  *total (host) receives the number of
 * entries.  SYNCHRONOUS (waits on stream).  Returns CAPACITY, writing only
 * offsets and *total, when total > capacity; returns CAPACITY too when a
 * particle has more than max_neighbors neighbours.  That overflow is this
 * call's own: it is neither taken from nor added to the status words that
 * sph_poll() reads (a non-finite position found by the sort still is). */
sph_status sph_neighbors(sph_plan* plan, const sph_state* s, int64_t* offsets, int32_t* nbr,
                         int64_t capacity, int64_t* total, void* stream);

/* Neighbour lists with a support radius per particle (Sec. 3.2, "Ensuring
 * symmetric interactions"; App. B, the search-radius step).  support (device,
 * N values of the plan's dtype, original order) holds h_i with 0 < h_i <= H,
 * the simulation's support being the largest any of its particles may have
 * (cells are sized for it, or for H (1 + skin)).  A particle searching with its
 * own h_i would miss partners whose larger support reaches it, so:
 *   1. search radius: s_k = max(h_k, max{h_i : |x_i - x_k| < h_i}), formed on
 *      the device by an integer atomic maximum on the bit pattern of s_k (no
 *      floating-point atomics; positive values order like their bits);
 *   2. each particle searches with s_i and keeps the super-symmetric set
 *      N(i) = { j : |x_i - x_j| < max(h_i, h_j) }, self included, a symmetric
 *      relation that every particle's search finds in full.
 * Predicates as for sph_neighbors, with h^2 = h * h rounded once in the plan's
 * dtype.  Output as for sph_neighbors: CSR over original indices, each row
 * ascending, in offsets (device, int64[N+1]) and nbr (device, int32[capacity]),
 * *total (host) the entry count; search_radius (device, N values, original
 * order, nullable) receives s_i.  SYNCHRONOUS.  Errors: INVALID_ARG for a null
 * support or a support outside (0, H] (found on the device, reported after the
 * synchronisation, no entries written); CAPACITY as for sph_neighbors.  The
 * status words that sph_poll() reads are not touched (a non-finite position
 * found by the sort still is).  Steps and sweeps keep using the plan's fixed
 * support. */
sph_status sph_neighbors_adaptive(sph_plan* plan, const sph_state* s, const void* support, void* search_radius,
                                  int64_t* offsets, int32_t* nbr, int64_t capacity, int64_t* total,
                                  void* stream);

/* One evaluation of the update function f (App. C) at the state s:
 *   drho_i = -rho_i sum_j V_j (v_j - v_i).gW_ij
 *            + delta H c0 sum_j V_j 2 (rho_j - rho_i) (x_ji.gW_ij) / (r^2 + eps H^2)
 *   a_i    = -(1/rho_i) sum_j V_j (p_i + p_j) gW_ij
 *            + alpha H c0 (rho0/rho_i) sum_j V_j pi_ij gW_ij,
 *   pi_ij  = (v_i - v_j).x_ij / (r^2 + eps H^2),   V_j = m / rho_j,
 *   p      = rho0 c0^2 / 7 ((rho/rho0)^7 - 1)           (Tait, Sec. 2.3)
 *   rho_sum_i = m sum_j W_ij   (summation density, self included)
 * with the Wendland-C4 kernel W and gW_ij = grad_i W(x_ij) (App. A.1) and the
 * continuity, momentum and delta-SPH terms of Sec. 2.3 (signs as in the
 * physical equations).  drho (device, N), acc (device, dim*N, SoA rows)
 * and rho_sum (device, N, nullable) are in original order. */
sph_status sph_rhs(sph_plan* plan, const sph_state* s, void* drho, void* acc, void* rho_sum, void* stream);

/* Advance s in place by nsteps semi-implicit Euler steps (Sec. 3.4):
 *   v' = v + dt a,  rho' = rho + dt drho,  x' = x + dt v'.
 * If ckpt (host array of sph_state, device pointers inside) is non-NULL, it
 * must hold ceil(nsteps / ckpt_every) states; slot k receives the state at
 * step k * ckpt_every (slot 0 = the input state), in original order.  These
 * are the segment starts for checkpointed recomputation (Sec. 3: gradient
 * checkpointing with on-the-fly recompute).  When the plan's tape_depth is at
 * least nsteps (and the default integrator is in use), every step keeps its
 * sorted state and neighbour lists in its own tape slot (the forward tape),
 * which sph_rollout_backward then uses instead of recomputing. */
sph_status sph_step(sph_plan* plan, sph_state* s, int32_t nsteps, const sph_state* ckpt, int32_t ckpt_every,
                    void* stream);

/* Adjoint of one step (Sec. 2.2, vector-Jacobian product): s_n (device) is
 * the state at the START of the step; cot (device) holds on entry the
 * cotangents (x', v', rho') of the step's output and on exit those of
 * (x, v, rho), in place:
 *   vt = v'_bar + dt x'_bar,  abar = dt vt,  rbar = dt rho'_bar,
 *   x_bar = x'_bar + (da/dx)^T abar + (ddrho/dx)^T rbar,
 *   v_bar = vt     + (da/dv)^T abar + (ddrho/dv)^T rbar,
 *   rho_bar = rho'_bar + (da/drho)^T abar + (ddrho/drho)^T rbar.
 * The neighbour list is held fixed (Sec. 3.2: adjacency is not
 * differentiated; the kernel's compact support makes the omitted terms 0). */
sph_status sph_step_adjoint(sph_plan* plan, const sph_state* s_n, sph_state* cot, void* stream);

/* Gradient of a checkpointed rollout (Sec. 3: checkpoints of the particle
 * state only, intermediate quantities recomputed; Sec. 2.2: chained
 * vector-Jacobian products).  ckpt (host array of sph_state, device pointers)
 * holds the ceil(nsteps / ckpt_every) checkpoints that sph_step() wrote for the
 * same initial state, nsteps and ckpt_every.  cot (device) holds on entry the
 * cotangents of the state after nsteps steps and on exit those of the initial
 * state, in place.  Segments are processed last to first: each is recomputed
 * from its checkpoint keeping every step's sorted state and neighbour lists in
 * the workspace tape, then its steps' adjoints run in reverse on the taped
 * data (each equal to sph_step_adjoint() on that step's start state).
 * When the last sph_step call on the plan kept a forward tape of exactly these
 * nsteps with exactly these checkpoints (same pointers), and no call has
 * written any of its slots since (every write of a slot changes its
 * generation number, which is checked), the adjoint steps run on that tape and
 * nothing is recomputed; the result is bitwise the same.
 * Needs tape_depth >= min(ckpt_every, nsteps) (else CAPACITY). */
sph_status sph_rollout_backward(sph_plan* plan, const sph_state* ckpt, int32_t nsteps, int32_t ckpt_every,
                                sph_state* cot, void* stream);

/* Vector-Jacobian product of the summation density rho_i = sum_j m W_ij
 * (Sec. 2.3 summation density; the backward benchmark of Sec. 4.1 takes the
 * summation density after a step and differentiates it with respect to the
 * initial positions).  Given the state s and cotangents g = rho_sum_bar
 * (device, N values of the plan's dtype, original order), writes
 *     x_bar[k][i] = sum_{j != i} m (g_i + g_j) dW_ij/dx_i[k]
 * into x_bar (device, dim rows of N, overwritten; the cotangent of the
 * positions only: rho_sum depends on nothing else).  Rebuilds the cell list
 * and the neighbour lists of s; results are deterministic and do not depend on
 * the batch.  Compose with sph_step_adjoint (cotangent (x_bar, 0, 0)) for the
 * gradient through a step.  INVALID_ARG on null arrays. */
sph_status sph_density_adjoint(sph_plan* plan, const sph_state* s, const void* rho_sum_bar, void* x_bar,
                               void* stream);

/* Retained neighbour lists (the paper's backward reuses the adjacency that the forward pass
 * built, Sec. 3.2 and Sec. 4.1).  sph_rhs and semi-implicit Euler sph_step calls keep, in one
 * workspace slot, the sorted copy and the neighbour lists of their INPUT state (sph_rhs in the
 * last slot, sph_step in slot 0).  Every later write of that slot (any call that sorts into it,
 * a step's list-reusing sweep, a graph replay) gives the slot a new generation number.
 * sph_retained_lists (host out-parameters) returns the slot and generation that the last such
 * call left, or slot -1 when it is gone (or the call was a Runge-Kutta or symplectic step).
 * The *_retained variants of the step and density adjoints take that pair: while the slot still
 * has that generation they skip the sort and the list build and work on the retained copy, as
 * the adjoint of the call that built it; otherwise they do exactly what sph_step_adjoint and
 * sph_density_adjoint do with s.  Results are bitwise those of the plain calls on the state the
 * retaining call received.  The caller guarantees that s is that state (autograd saves it).
 * sph_step_adjoint_retained is for one-step calls of the default integrator (other schemes fall
 * back to the plain call). */
sph_status sph_retained_lists(const sph_plan* plan, int32_t* slot, uint64_t* generation);
sph_status sph_step_adjoint_retained(sph_plan* plan, const sph_state* s_n, sph_state* cot, int32_t slot,
                                     uint64_t generation, void* stream);
sph_status sph_density_adjoint_retained(sph_plan* plan, const sph_state* s, const void* rho_sum_bar, void* x_bar,
                                        int32_t slot, uint64_t generation, void* stream);

/* Copy the per-simulation status words (host int32[nsims], SPH_FLAG_* bits)
 * and clear them.  SYNCHRONOUS. */
sph_status sph_poll(sph_plan* plan, int32_t* per_sim_status, void* stream);

/* Number of directed neighbour pairs (i, j), j != i, with r < H, counted since the last
 * call (host out-parameter), then reset: by the neighbour-list builds for exact lists, or,
 * when the plan's lists carry a skin, by the forward sweeps that filter them (one count per
 * right-hand-side evaluation either way).  This is the unit of the pair interaction rate.
 * SYNCHRONOUS. */
sph_status sph_pair_count(sph_plan* plan, int64_t* pairs, void* stream);

/* sph_poll and sph_pair_count together, without waiting: enqueues on `stream` the copy of the
 * per-simulation status words into per_sim_status (host int32[nsims]) and of the directed pair
 * count (as sph_pair_count counts it) into *pairs (host; null skips it), then clears both on the
 * device.  The values are there once the stream has passed this point (hipStreamSynchronize, or
 * an event recorded after the call); a later call on the same plan reuses the device staging
 * area, so read the host copies before the stream reaches the next call.  The host buffers
 * should be page-locked (hipHostMalloc): with pageable memory the runtime may wait for the copy
 * before returning.  For callers that keep the device busy while they check many plans (one
 * host synchronisation for all of them).  INVALID_ARG on a null per_sim_status. */
sph_status sph_poll_async(sph_plan* plan, int32_t* per_sim_status, int64_t* pairs, void* stream);

/* Kernel classes timed by the profiler. */
#define SPH_KERN_SORT 0      /* cell assignment, scan, scatter, within-cell order, gather */
#define SPH_KERN_BUILD 1     /* neighbour-list build */
#define SPH_KERN_SWEEP 2     /* fused forward sweep (RHS + integrator) */
#define SPH_KERN_ADJOINT 3   /* adjoint sweep */
#define SPH_KERN_OTHER 4     /* unsort, adjoint prologue */
#define SPH_KERN_COUNT 5

/* Per-launch HIP-event timing of the plan's kernels: `classes` is a bit mask, bit k
 * selecting kernel class k (SPH_PROFILE_ALL for every class, 0 to stop).  The build, sweep
 * and adjoint classes are one kernel per launch group: their event pair is handed to that
 * launch (hipExtLaunchKernelGGL) and holds the kernel's own start and end.  The sort and
 * other classes span several kernels and are bracketed by events recorded on the stream,
 * each costing about a microsecond of device time, so time only the classes of interest
 * in a timed run.  While profiling is on, graph mode is not used. */
#define SPH_PROFILE_ALL ((1 << SPH_KERN_COUNT) - 1)
sph_status sph_profile_enable(sph_plan* plan, int32_t classes);

/* Accumulated device time in milliseconds (host double[SPH_KERN_COUNT]) and launch counts
 * (host int64[SPH_KERN_COUNT]) per kernel class since the last read, then reset.
 * SYNCHRONOUS (waits for the recorded events). */
sph_status sph_profile_read(sph_plan* plan, double* ms, int64_t* launches);

/* Message of the last failing call on this thread ("" if none). */
const char* sph_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPH_H */
