/*
 * lee.h -- C ABI of the MI355X library for one Runge-Kutta stage of the 2-D
 * linearized Euler equations with a ghost-point immersed boundary and a
 * mass-spring-damper impedance wall advanced by auxiliary differential
 * equations (ADE).
 *
 * The problem (paper Sec. 2.1, eq. LEE): dq/dt + dE/dx + dF/dy = S with
 * q = [p, u, v], rho0 = c0 = 1, S = [s, 0, 0]; advanced on a uniform grid
 * x_i = x0 + i h, y_j = y0 + j h (0 <= i < nx, 0 <= j < ny) at fluid nodes
 * only (Sec. 3.1).  Each stage fills the ghost points from a least-squares
 * fit on an elliptical cloud of fluid nodes extrapolated along the wall
 * normal (Sec. 3.1, eqs. ns-ellipse .. ns-ghost), coupled to the two-state
 * ADE of the impedance Z = M s + R + K/s (Sec. 2.5) through the six steps
 * of Sec. 3.2, then evaluates the DRP right-hand side (Sec. 2.2, eq. DRP_s)
 * and the low-storage RK4 stage update.
 *
 * Conventions common to every call:
 *   - every call returns a lee_status; nothing aborts or throws across the
 *     ABI; lee_last_error() returns a thread-local message for the last
 *     failing call on this thread;
 *   - host pointers are plain C arrays owned by the caller; device memory is
 *     owned by the caller (lee_bind) and never freed by the library;
 *   - all device work is asynchronous on the stream given to lee_bind,
 *     except the calls documented as synchronising;
 *   - an instance is not thread-safe: one thread at a time per instance.
 */
#ifndef LEE_H
#define LEE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lee_status;
#define LEE_OK 0
#define LEE_E_ARG (-1)               /* invalid argument or unsupported option */
#define LEE_E_GEOMETRY (-2)          /* wall/grid combination cannot be handled */
#define LEE_E_CRITICAL_DAMPING (-3)  /* R = 2 sqrt(KM): double pole (Sec. 2.5) */
#define LEE_E_ADE_STIFF (-4)         /* ADE or wall coupling unstable at this dt */
#define LEE_E_RANK (-5)              /* reserved: least-squares rank failure */
#define LEE_E_NOMEM (-6)             /* host allocation or device buffer too small */
#define LEE_E_DEVICE (-7)            /* a HIP runtime call failed */
#define LEE_E_STATE (-8)             /* call out of order (e.g. stage sequence) */
#define LEE_E_PROBE (-9)             /* probe stencil leaves the fluid */

#define LEE_F32 0
#define LEE_F64 1

#define LEE_WALL_NONE 0
#define LEE_WALL_LINE 1     /* through (cx, cy), unit normal (nx, ny) into the fluid */
#define LEE_WALL_CIRCLE 2   /* centre (cx, cy), radius rc, fluid outside */

#define LEE_IC_NONE 0
#define LEE_IC_PULSE 1      /* ic = {xs, ys, a, w}: p0 = a exp(-ln2 r^2 / w^2) (Sec. 4.2) */
#define LEE_IC_PACKET 2     /* ic = {xs, ys, dx, dy, a, alpha, k}: plane packet of Sec. 4.1
                               along (dx, dy): p0 = a/2 exp(-alpha^2 s^2) cos(2 pi k s),
                               s = (x - xs) dx + (y - ys) dy, (u0, v0) = p0 (dx, dy) */

#define LEE_SRC_NONE 0
#define LEE_SRC_MONOPOLE 1  /* src = {xs, ys, a, w, omega}:
                               s = a exp(-ln2 r^2 / w^2) sin(omega t) (Sec. 4.3) */

#define LEE_Z_RIGID 0       /* Y -> 0: u_n = 0, dp/dn = 0 (Sec. 2.4) */
#define LEE_Z_MSD 1         /* Z = M s + R + K / s (Sec. 2.5) */
#define LEE_Z_POLES 2       /* Y(s) = sum_k A_k / (s - lambda_k)
                               + sum_k [q_k / (s - s_k) + conj(q_k) / (s - conj(s_k))],
                               the multi-pole form of Sec. 2.3 (eq. Yrational) without a
                               direct term; one auxiliary state per real pole and two per
                               pair (eq. ADEgeneral), at most LEE_ADE_MAX_STATES */
#define LEE_ADE_MAX_STATES 8

/* Problem description (Sec. 2.1-2.2, 3.1, 4).  dt = cfl * h (c0 = 1). */
typedef struct {
    int32_t nx, ny;          /* grid nodes, each >= 16 */
    double x0, y0, h;        /* node (i, j) sits at (x0 + i h, y0 + j h) */
    int32_t stencil_half;    /* DRP half-width: 5 (11-point) or 3 (7-point, eq. DRP_s) */
    double cfl;              /* dt = cfl * h */
    double filter_sigma;     /* 11-point selective filter strength; 0 disables it
                                (requires stencil_half = 5 when > 0) */
    int32_t sponge_cells;    /* outer damping layer width in cells (0 = none) */
    double sponge_sigma;     /* its peak rate; sigma(e) = sigma ((W - e)/W)^2 */
    int32_t precision;       /* LEE_F32 or LEE_F64 field arithmetic */
    int32_t wall_kind;       /* LEE_WALL_* */
    double wall_cx, wall_cy, wall_nx, wall_ny, wall_rc;
    int32_t ic_kind;         /* LEE_IC_* */
    double ic[7];
    int32_t src_kind;        /* LEE_SRC_* */
    double src[5];
    /* Outer boundary (Sec. 2.2: one-sided stencils at the domain edges;
     * Sec. 4.1-4.2: the non-reflecting condition of Tam and Webb there).
     * 0: a zero frame around the domain (plus the sponge, if any).  1: at
     * the nodes closer than stencil_half nodes to an edge the stage solves
     * dq/dt = -(dq/dr + q/(2r)) for p, u and v, r and theta measured from
     * (rad_xc, rad_yc), with 7-node derivatives inside the domain (central
     * where three nodes lie on each side, else the one-sided maximal-order
     * set) and no filter term.  Requires every node within stencil_half + 6
     * of an edge to be fluid and the centre at least h from every band node
     * (else LEE_E_ARG); the tile sweeps only (LEE_SWEEP_MARCH -> LEE_E_ARG). */
    int32_t radiation;
    double rad_xc, rad_yc;
    /* Form of the selective filter (with filter_sigma > 0; Sec. 2.2 names
     * none, the paper runs without one).  0: the damping term
     * -(sigma/dt)(F_x + F_y)q in every stage's right-hand side.  1: the
     * explicit form, q <- q - sigma (F_x + F_y)q at the fluid nodes outside
     * the radiation band after every full step (one more launch per step),
     * the stages then without the damping term.  Both take the narrower
     * centred rows next to an immersed wall.  1 requires the tile sweep
     * (LEE_SWEEP_MARCH -> LEE_E_ARG); other values -> LEE_E_ARG. */
    int32_t filter_explicit;
} lee_case_desc;

typedef struct {
    int32_t kind;            /* LEE_Z_RIGID, LEE_Z_MSD or LEE_Z_POLES */
    double R, M, K;          /* LEE_Z_MSD: resistance, mass, stiffness per unit area (all > 0) */
    /* LEE_Z_POLES: n_real real poles lambda_k < 0 with residues A_k, and n_pair
       pole pairs s_k = alpha_k +- i beta_k (alpha_k < 0, beta_k > 0) with
       residues B_k +- i C_k; 1 <= n_real + 2 n_pair <= LEE_ADE_MAX_STATES */
    int32_t n_real;
    double real_pole[LEE_ADE_MAX_STATES], real_res[LEE_ADE_MAX_STATES];
    int32_t n_pair;
    double pair_alpha[LEE_ADE_MAX_STATES / 2], pair_beta[LEE_ADE_MAX_STATES / 2];
    double pair_B[LEE_ADE_MAX_STATES / 2], pair_C[LEE_ADE_MAX_STATES / 2];
} lee_impedance;

typedef struct {
    int32_t G;               /* ghost points */
    int64_t nnz;             /* total cloud entries */
    int32_t n_degraded;      /* ghosts fitted below degree 4 (or not at all) */
    int32_t n_cut;           /* ghosts whose ellipse leaves the domain (value 0) */
    double r_min, r_max;     /* range of r = d / h */
    double w_l1_max;         /* largest 1-norm of a composite weight row */
    int64_t fluid_nodes;     /* nodes advanced per stage */
    int32_t ade_kind;        /* 0 rigid, 1 complex pole pair, 2 two real poles, 3 multi-pole */
    double poles[4];         /* re s1, im s1, re s2, im s2 (multi-pole: the first two poles) */
    int32_t ade_states;      /* auxiliary states per ghost (2, or n_real + 2 n_pair) */
} lee_ghost_summary;

typedef struct lee_instance lee_instance;
typedef struct lee_batch lee_batch;

/* Thread-local message describing the last failing call on this thread. */
const char *lee_last_error(void);

/*
 * Grid set-up (host only, no device call): fluid mask (phi > 0, a node on the
 * wall is solid; Sec. 3.1), ghost list (solid nodes reached by a fluid
 * node's stencil along x or y), dt.  *out belongs to the library until
 * lee_destroy.  Unsupported descriptions -> LEE_E_ARG; a wall the kernels
 * cannot represent (more than two fluid intervals in a row, a ghost at a
 * circle centre) -> LEE_E_GEOMETRY.
 */
lee_status lee_setup_grid(const lee_case_desc *d, lee_instance **out);

/*
 * Ghost weights and ADE coefficients (host only, FP64).  For every ghost:
 * boundary point, normal and r (eq. ns-rotation), elliptical cloud
 * (eq. ns-ellipse, R_n = 2k, R_t = k/2 + 1), least-squares read-out at
 * P_0..P_4 by Householder QR (eqs. ns-vandermonde .. ns-readout), composed
 * with the 1-D Lagrange / Birkhoff extrapolation (eq. ns-ghost) into four
 * weights per cloud entry (p_BP, free, Dirichlet, Neumann).  degree must be
 * 4 (k = m = 4, Sec. 3.1); clouds that are too small or rank-deficient fall
 * back to degree 3, 2, 1, else zero; clouds cut by the domain edge are zero.
 * ADE: poles and residues of Y = 1/Z (Sec. 2.5); critical damping ->
 * LEE_E_CRITICAL_DAMPING; a pole outside the RK4 stability region or a wall
 * coupling gain h/M > 2 -> LEE_E_ADE_STIFF.  LEE_Z_POLES: the given terms
 * (Sec. 2.3); a pole off the open left half-plane, a pair with beta <= 0,
 * a non-finite value or a state count outside 1..8 -> LEE_E_ARG; a pole
 * outside the RK4 region or a coupling gain h (sum A_k + 2 sum B_k) > 2
 * (the limit of s Y(s), 1/M for the MSD) -> LEE_E_ADE_STIFF.  opt_out may
 * be NULL.
 * Must be called once, after lee_setup_grid and before lee_bind.
 */
lee_status lee_build_ghosts(lee_instance *inst, const lee_impedance *z, int32_t degree,
                            lee_ghost_summary *opt_out);

/* Device bytes lee_bind needs (fields: 3 register sets x 3 planes, ADE
 * states, ghost lists, probe buffers); valid after lee_build_ghosts and
 * after lee_set_probes. */
lee_status lee_required_bytes(const lee_instance *inst, size_t *dev_bytes);

/*
 * Bind caller-owned device memory (at least lee_required_bytes, 256-byte
 * aligned) and a HIP stream (hipStream_t, may be NULL for the default
 * stream) on the current device.  Uploads the lists and zeroes the state
 * asynchronously; lee_init_fields then applies the initial condition.  The
 * library never frees dev_ptr.
 */
lee_status lee_bind(lee_instance *inst, void *dev_ptr, size_t bytes, void *hip_stream);

/* Initial state (Sec. 2.1): q0 at fluid nodes, zero elsewhere, ADE states
 * zero, step counter 0, traces cleared.  Asynchronous. */
lee_status lee_init_fields(lee_instance *inst);

/*
 * One Runge-Kutta stage (stage = 0..3) on the bound stream, asynchronous:
 * ghost fill + ADE (Sec. 3.2 steps 1-5) then the stage sweep (step 6).  The
 * stages of a step must be issued in order 0, 1, 2, 3 (else LEE_E_STATE);
 * after stage 3 the step counter advances and the probes are sampled.  Four
 * calls give bit-identical results to lee_step_n(inst, 1).
 */
lee_status lee_rk_stage(lee_instance *inst, int32_t stage);

/* n full steps by replaying captured hipGraphs; asynchronous.  Requires that
 * no partial step is pending (else LEE_E_STATE).  The steps go in runs (one
 * captured graph each): the probes after each step but the last of a run are
 * sampled by extra workgroups of the next step's second stage, and a run ends
 * with the probes after its last step and one launch that advances the step
 * counter, so a step costs its four stage launches. */
lee_status lee_step_n(lee_instance *inst, int64_t n);

/*
 * Register recorded probes before lee_bind: np points (xy[2k], xy[2k+1]),
 * sampled after every step by 4 x 4 cubic Lagrange interpolation into a
 * device ring of `capacity` steps.  A stencil leaving the fluid ->
 * LEE_E_PROBE.  Optionally a running DFT of p at each probe over steps
 * [dft_start, dft_start + dft_count): P = (2i/N) sum p(t_n) exp(-i omega t_n)
 * (pass dft_count = 0 for none).
 */
lee_status lee_set_probes(lee_instance *inst, int32_t np, const double *xy, int64_t capacity,
                          double dft_omega, int64_t dft_start, int64_t dft_count);

/* Synchronising: sample q^n (after a full step) at np <= 256 arbitrary points;
 * out[3k + {0,1,2}] = p, u, v.  LEE_E_PROBE if a stencil leaves the fluid. */
lee_status lee_probe(lee_instance *inst, int32_t np, const double *xy, double *out);

/* Synchronising: copy recorded traces, oldest first, out[(s np + k) 3 + f];
 * *n receives the number of steps copied (at most cap and the ring size). */
lee_status lee_probe_traces(lee_instance *inst, double *out, int64_t cap, int64_t *n);

/* Synchronising: running DFT amplitudes over the window set by
 * lee_set_probes (N = dft_count steps), P_k = (2i/N) sum_n p_k(t_n)
 * exp(-i omega t_n) with t_n the time after step n, so that a harmonic
 * p_k(t) = Im(P_k exp(i omega t)) (App. C convention) gives back P_k;
 * out[2k] = Re P_k, out[2k+1] = Im P_k. */
lee_status lee_probe_dft(lee_instance *inst, double *out);

/*
 * Watched ghost (Coupling section, steps 1-3; Sec. 4.3, cylinder scattering a
 * harmonic monopole, for the comparison of the two normal velocities):
 * before lee_bind, choose the ghost whose boundary point is nearest (x, y)
 * (ties: the lowest index; *ghost receives its index, NULL allowed) and keep
 * a ring of `capacity` steps of three values at the first stage of each step,
 * in FP64: its boundary pressure p_BP, the ADE's wall normal velocity u_n,BP,
 * and the normal velocity read out of the fluid at the boundary point (the
 * least-squares fit's u.n at P_0, which the wall datum does not constrain),
 * both velocities positive into the wall.  With capacity 0 nothing is
 * recorded.  LEE_E_ARG without ghosts.
 */
lee_status lee_set_watch(lee_instance *inst, double x, double y, int64_t capacity, int32_t *ghost);

/* The last min(steps, capacity, cap) recorded (p_BP, u_n,BP, fluid u_n)
 * triples, oldest first, into out[3 * cap]; *n receives the count.
 * Synchronising. */
lee_status lee_watch_traces(lee_instance *inst, double *out, int64_t cap, int64_t *n);

/* Synchronising: copy q^n at the domain nodes into caller arrays of
 * ny * nx doubles (row-major, x fastest); any pointer may be NULL. */
lee_status lee_get_fields(lee_instance *inst, double *p, double *u, double *v);

/* Synchronising: overwrite q^n at fluid nodes from ny * nx doubles. */
lee_status lee_set_fields(lee_instance *inst, const double *p, const double *u, const double *v);

/* Synchronising: ADE states after the last full step, out[n g + k] with n
 * the summary's ade_states (states in the order of the real poles, then
 * each pair's two). */
lee_status lee_get_ade_states(lee_instance *inst, double *out);

/* Synchronising: overwrite the ADE states that the next step starts from
 * with in[n g + k], the layout lee_get_ade_states returns; nothing to do for
 * a rigid wall.  With lee_set_fields this sets the whole state of the scheme
 * (Sec. 2.3: the auxiliary states are part of the unknowns), as a linear
 * analysis of the step map needs. */
lee_status lee_set_ade_states(lee_instance *inst, const double *in);

/*
 * The semi-discrete operator at the current state (abstract: the spectral
 * analysis of the linearised operator; Sec. 3.2 steps 1-6 without the stage
 * update): the ghost fill and ADE derivative from (q^n, Psi^n) and the
 * right-hand side of the LEE at every fluid node, computed by the
 * instance's own stage kernels (its first stage, run once with an update
 * coefficient of one, then undone: q^n, Psi^n, the step counter and the
 * stage sequence are unchanged).  p, u, v (ny * nx doubles, row-major, any
 * may be NULL) receive the right-hand side at the fluid nodes and zero
 * elsewhere; psi (NULL allowed; ns * G doubles in the layout of
 * lee_get_ade_states) receives dPsi/dt (zero for a rigid wall).  The source
 * term, if any, is included at the current step's time.  Each value is the
 * difference of the stage output and q^n in the instance's precision, so an
 * FP32 instance carries FP32 rounding.  Synchronising; LEE_E_STATE while a
 * partial step is pending.
 */
lee_status lee_rhs(lee_instance *inst, double *p, double *u, double *v, double *psi);

/* Completed steps: the device's step counter once the stream is idle
 * (synchronising; budgets of a batch may have idled the instance); before
 * lee_bind, 0.  Reports a spent fused-stage wait as lee_synchronize does. */
lee_status lee_get_step(const lee_instance *inst, int64_t *step);

/*
 * Copy the set-up lists into caller arrays sized from the summary:
 * ghost_idx[G] (j nx + i, ascending), cloud_ptr[G+1], cloud_idx[nnz]
 * (j nx + i, ascending within a ghost), degree[G] (0 = zero ghost),
 * weights[4 nnz] as (w_BP, w_free, w_Dirichlet, w_Neumann) per entry and
 * beta[2 G] as (beta_D, beta_N) per ghost, geom[5 G] as (x_BP, y_BP, n_x,
 * n_y, r) per ghost.  Any pointer may be NULL.
 */
lee_status lee_export_lists(const lee_instance *inst, int32_t *ghost_idx, int32_t *cloud_ptr,
                            int32_t *cloud_idx, int8_t *degree, double *weights, double *beta,
                            double *geom);

/*
 * Stage-sweep kernel and tile shape.  LEE_SWEEP_TILE: a 256-thread workgroup
 * copies a cols x rows tile plus its 5-point halo into LDS and computes it;
 * shapes: FP32 cols 64 with rows 8, 16 or 32, cols 128 with rows 4, 8, 16 or
 * 32, cols 256 with rows 4, 8 or 16; FP64 cols 64 with rows 8, 16 or 32,
 * cols 128 with rows 4, 8 or 16, cols 256 with rows 4.  Default: cols 64, rows
 * 16 (FP32) or 8 (FP64), not fused.
 * LEE_SWEEP_MARCH: each wave marches a strip of 64 vec - 16 columns down
 * `rows` rows (>= 4) keeping an 11-row register window; vec 2 or 4 (FP32),
 * 2 (FP64); waves per workgroup 1, 2 or 4.  Other shapes -> LEE_E_ARG.
 * Invalidates the captured graph.  With `fused`, the ghost fill of a stage runs
 * in the first workgroups of the sweep launch, and only the tiles whose
 * stencils read ghost nodes wait for it; the results are bit-for-bit those
 * of the two-launch form.
 */
#define LEE_SWEEP_TILE 0
#define LEE_SWEEP_MARCH 1
typedef struct {
    int32_t kind;            /* LEE_SWEEP_TILE or LEE_SWEEP_MARCH */
    int32_t vec;             /* march: columns per lane */
    int32_t cols;            /* tile: columns per tile */
    int32_t rows;            /* rows per tile / per march */
    int32_t waves;           /* march: waves per workgroup */
    int32_t fused;           /* tile: 1 = a stage's ghost fill and sweep in one launch,
                                0 = two launches (the default); march: ignored */
} lee_tiling;

lee_status lee_set_tiling(lee_instance *inst, const lee_tiling *t);

/*
 * Steps per captured hipGraph for lee_step_n (and batches): steps > 0
 * captures that many consecutive steps in one graph (at most 256; a single-
 * step graph covers the remainder of n), 0 selects the built-in default (16
 * steps), a negative value launches every kernel eagerly without graphs.  Invalidates
 * the captured graphs.
 */
lee_status lee_set_graph_steps(lee_instance *inst, int32_t steps);
lee_status lee_get_tiling(const lee_instance *inst, lee_tiling *t);

/*
 * Bound on the polls of a fused stage's wait for each ghost value it reads
 * (the ghost values of the stage's carrier workgroups, Coupling section):
 * polls > 0 sets the bound (default 2^20, about a second), 0 restores the
 * default.  polls < 0 is for testing the error path: every wait then looks
 * for a tag that is never published, gives up after -polls polls and raises
 * the error flag, so the next lee_synchronize reports LEE_E_DEVICE (the
 * results of such stages are not valid; every kernel still ends).
 * Invalidates the captured graphs.
 */
lee_status lee_set_ghost_wait(lee_instance *inst, int32_t polls);

/*
 * Measurement (synchronising, on the bound stream).  Runs, each bracketed by
 * one pair of HIP events: 4n ghost launches (stages 0..3 in turn), 4n sweep
 * launches (the fused launch when the tiling is fused), then n eager steps.
 * Returns the mean per-launch ghost and sweep times and the mean step time
 * in microseconds; a mean over back-to-back launches includes the gap
 * between launches.  The repeated launches are not valid steps, so the
 * fields, ADE states, step counter and traces are reset to the initial
 * condition afterwards (as by lee_init_fields).
 */
lee_status lee_time_kernels(lee_instance *inst, int64_t n, double *sweep_us, double *ghost_us,
                            double *step_us);

/* Measurement utility: asynchronous device copy of `bytes` (multiple of 16,
 * 16-byte aligned buffers) on hip_stream.  Its traffic is exactly 2 x bytes,
 * which calibrates hardware byte counters and the achievable HBM rate. */
lee_status lee_stream_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

/* Wait for the instance's stream.  LEE_E_DEVICE if a fused stage's wait for
 * its ghost fill ran out of polls (the results of that stage are then not
 * valid; this does not happen while the device dispatches workgroups in
 * order).  lee_get_fields and lee_get_step report the same condition. */
lee_status lee_synchronize(lee_instance *inst);

/* Free host structures and device-side objects the library created (graph,
 * events); the bound device memory stays the caller's. */
void lee_destroy(lee_instance *inst);

/* ---------------- batches: many instances in one launch per phase -------- */

typedef struct {
    lee_tiling tiling;          /* sweep tiling for the whole batch (kind < 0: built-in default) */
    int32_t persistent_blocks;  /* 0 = one workgroup per work item */
    int32_t graph_steps;        /* as lee_set_graph_steps */
} lee_batch_opts;

/*
 * Group n bound instances of the same precision and stencil into a batch
 * advanced by one launch per phase (ghost fill and sweep, or one fused
 * launch) over a flat work list spanning all members, captured in hipGraphs
 * on the stream of the first member.  The instance table lives in device memory
 * owned by the batch (allocated by the library).  Members keep their own
 * step counters; lee_batch_set_budget lets finished members idle without
 * re-capturing.
 */
lee_status lee_batch_create(lee_instance *const *v, int32_t n, const lee_batch_opts *opts,
                            lee_batch **out);

/* Membership: add a bound instance (same precision, filter setting and
 * device; its own stream is synchronised first) or remove one (the batch's
 * stream is synchronised first).  The device table and work lists are
 * rebuilt in place: every list is padded with idle entries to a device
 * capacity and the launches cover the capacities, so the captured graphs
 * are kept.  Only a list that outgrows its capacity (capacities grow by
 * at least a quarter) or shrinks below three quarters of it drops them
 * (the capacities are then trimmed to the lists), and the next
 * lee_batch_step_n captures again.  In the fused form the ghost-fill workgroups of a batch come before
 * all tiles, sized by the ghost capacity.  A
 * batch may become empty (stepping it is then a no-op).  Budgets are per
 * position: set them again after a membership change. */
lee_status lee_batch_add(lee_batch *b, lee_instance *inst);
lee_status lee_batch_remove(lee_batch *b, lee_instance *inst);
lee_status lee_batch_size(const lee_batch *b, int32_t *n);

/* Several membership changes with one rebuild of the device table and work
 * lists: the nremove instances in `remove` (each a member, no repeats) leave
 * the batch, then the nadd instances in `add` (each bound, not a member
 * after the removals, no repeats, checked as lee_batch_add checks them)
 * join it at the end, in that order.  The result is the batch that the same
 * lee_batch_remove calls followed by the same lee_batch_add calls give, and
 * its graphs are kept or dropped by the same rule (applied once, to the
 * final membership); it costs one rebuild
 * instead of one per change (the rebuild covers every member, so a served
 * stream that retires and admits several requests between chunks of a
 * large batch pays it once).  The batch's stream and the added instances'
 * streams are synchronised first.  The arrays are the caller's; nothing is
 * changed when an argument is refused (LEE_E_ARG, LEE_E_STATE). */
lee_status lee_batch_update(lee_batch *b, lee_instance *const *add, int32_t nadd, lee_instance *const *remove,
                            int32_t nremove);

/* Number of step graphs the batch has captured so far (each run length
 * captured counts once); it grows only when graphs had to be dropped. */
lee_status lee_batch_graph_captures(const lee_batch *b, int64_t *n);

/* Per-member step budget (n entries, synchronising): member k takes the next
 * steps[k] steps and then idles (its fields, ADE states and step counter stay
 * as they are) until a new budget is set.  lee_init_fields (and so
 * lee_bind) makes an instance's budget unlimited. */
lee_status lee_batch_set_budget(lee_batch *b, const int64_t *steps);

/* n steps of every member with a positive budget; asynchronous. */
lee_status lee_batch_step_n(lee_batch *b, int64_t n);

/* The batch's sweep tiling (rebuilds its work list; synchronising) and steps
 * per captured graph, as lee_set_tiling and lee_set_graph_steps. */
lee_status lee_batch_set_tiling(lee_batch *b, const lee_tiling *t);
lee_status lee_batch_get_tiling(const lee_batch *b, lee_tiling *t);
lee_status lee_batch_set_graph_steps(lee_batch *b, int32_t steps);

/* Wait for the batch's stream; LEE_E_DEVICE as for lee_synchronize. */
lee_status lee_batch_synchronize(lee_batch *b);

/* As lee_time_kernels, over the whole batch; every member is reset to its
 * initial condition afterwards. */
lee_status lee_batch_time_kernels(lee_batch *b, int64_t n, double *sweep_us, double *ghost_us,
                                  double *step_us);

void lee_batch_destroy(lee_batch *b);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): advance the
 * bound instances v[0..n) together by `steps` steps, as lee_batch_step_n
 * does for a batch of the same members (lee_batch_create(v, n) with this
 * tiling, NULL for the batch default) -- the same kernels and the same per-node
 * arithmetic, so the same fields bit for bit -- but with the instance table,
 * the work lists and the error flag in a static device array of
 * LEE_NOALLOC_SCRATCH_BYTES per GPU instead of memory the library allocates.
 * Nothing is allocated on the device; the array is held by each GPU the
 * library runs on until the process ends.  Members as for lee_batch_create
 * (bound, same precision, filter setting and device, no partial step), run on
 * v[0]'s stream as eager launches (no graphs); each member takes the steps
 * below its budget (lee_batch_set_budget) as in a batch.  LEE_E_ARG when the
 * members' table and lists need more than the array holds (n at most
 * LEE_NOALLOC_MAX_MEMBERS).  The call waits until its lists are on the device
 * and returns with the steps queued; a ghost wait that ran out is reported by
 * lee_synchronize(v[0]).  Every call on a GPU shares that GPU's array, which
 * keeps the last call's contents (the error flag is cleared at each call):
 * calls that overlap on one GPU from different streams race.
 */
#define LEE_NOALLOC_SCRATCH_BYTES (16u << 20)
#define LEE_NOALLOC_MAX_MEMBERS 1024
lee_status lee_step_members_noalloc(lee_instance *const *v, int32_t n, const lee_tiling *tiling, int64_t steps);

#ifdef __cplusplus
}
#endif

#endif /* LEE_H */
