/*
 * pf.h -- C-ABI of libpf, an MI355X (gfx950) implementation of the explicit
 * method-of-lines time step for coupled multi-phase-field + concentration
 * models (Seiz & Takaki, "Numerical efficiency of explicit time integrators
 * for phase-field models", arXiv 2601.16522).
 *
 * The model (Sec. 2): N order parameters phi_a on the simplex, evolved by the
 * pairwise multi-phase Allen-Cahn equation with an obstacle potential
 * (eq. phieq), and one concentration c evolved by the KKS diffusion equation
 * with parabolic Gibbs energies (eqs. ceq, gibbs-energy).  Space: second-order
 * finite differences on a periodic, cell-centred Cartesian grid (Sec. 3).
 * Time: forward Euler, SSP(s)2, SSP(10)4, RKL1, RKL2 (Sec. 3.2), with the
 * simplex projection after every stage, and adaptive RKL/SSP steps with the
 * error estimates, norm and PID controller of Sec. 3.3.
 *
 * Field layout everywhere (host and device): a state vector is F = n_phi +
 * with_c planes of V = nx*ny*nz values, plane a < n_phi is phi_a, plane
 * n_phi is c; inside a plane x is fastest, then y, then z.  Host arrays are
 * always double; device arrays use the handle's precision (double for
 * PF_FP64, float for PF_FP32).
 *
 * Errors: every call returns a pf_status; a negative value is a failure and
 * leaves the state unchanged, except PF_ENONFINITE and PF_EDTMIN, which leave
 * the last accepted state.  pf_last_error() gives a message valid until the
 * next call on the same handle.
 * Ownership: the handle owns its device memory; host pointers are borrowed for
 * the duration of a call; device pointers passed in must be valid device
 * memory of the stated size and are only read during the call (stream
 * ordered on the handle's stream).
 * Threads: a handle is not thread safe; separate handles are independent.
 */
#ifndef PF_H
#define PF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pf_sim pf_sim;

typedef enum {
    PF_OK = 0,
    PF_EINVAL = -1,        /* bad argument or parameter */
    PF_ENOMEM = -2,        /* device or host allocation failed */
    PF_EHIP = -3,          /* HIP runtime error */
    PF_ENONFINITE = -4,    /* non-finite error norm three times in a row */
    PF_EDTMIN = -5,        /* adaptive step fell below 1e-12 dt_e */
    PF_ESTATE = -6,        /* call not valid in the current state (e.g. no fields) */
    PF_EUNSUPPORTED = -7   /* valid request that this library does not implement */
} pf_status;

/* Integrators of Sec. 3.2 (Table tab:ints). */
typedef enum {
    PF_FEULER = 0,    /* forward Euler */
    PF_SSP_S2 = 1,    /* SSP(s)2, s = pf_params.ssp_stages (Alg. ssp2) */
    PF_SSP_10_4 = 2,  /* SSP(10)4 (Ketcheson 2008, low storage) */
    PF_RKL1 = 3,      /* first-order Runge-Kutta-Legendre (Alg. sts1) */
    PF_RKL2 = 4       /* second-order Runge-Kutta-Legendre (eq. sts) */
} pf_integrator;

typedef enum {
    PF_FP64 = 0,  /* everything in double */
    PF_FP32 = 1   /* stencil, stage and projection arithmetic in float; time,
                     error norm and conservation sums in double */
} pf_precision;

/* Model and grid parameters.  Pair tables are symmetric n_types x n_types,
 * row-major; phase a has type type_of[a].  Pair constants follow Sec. 2:
 * A = 4 W gamma / pi, B = 4 gamma / (pi W), L = pi M / (4 W).  All arrays are
 * copied by pf_create. */
typedef struct {
    int dim;               /* 2 or 3 */
    int nx, ny, nz;        /* grid (nz = 1 for dim 2) */
    double dx;             /* grid spacing */
    double W;              /* interface parameter (interface width pi W) */
    int n_phi;             /* N, 2 <= N <= 16 (kernels exist for N in
                              pf_supported_nphi) */
    const int *type_of;    /* [n_phi], values in [0, n_types) */
    int n_types;           /* 1..4 */
    const double *gamma;   /* [n_types^2] interface energies */
    const double *mob;     /* [n_types^2] interface mobilities M */
    const double *k;       /* [n_types] Gibbs-energy curvatures (eq. gibbs-energy) */
    const double *c0;      /* [n_types] equilibrium concentrations */
    const double *D;       /* [n_types] diffusivities */
    int with_c;            /* 0: phase-field only (no c plane, no chemical term) */
    pf_precision prec;
    int ssp_stages;        /* s of SSP(s)2, >= 2 (0 selects 5) */
    /* Boundaries (Sec. 4: periodic unless stated).  bc[axis] (x, y, z): 0
     * periodic, 1 walls where phi and c have zero gradient (the neighbour
     * beyond a wall is the wall cell).  c_fixed[face] (faces x-, x+, y-, y+,
     * z-, z+) != 0 on a walled axis holds c at c_bc[face] beyond that face:
     * the ghost cell takes the wall cell's phi and c = c_bc (the Dirichlet
     * walls of the solutal Stefan problem, Sec. 5.2.2).  A zeroed tail means
     * periodic.  Batches take periodic instances only. */
    int bc[3];
    int c_fixed[6];
    double c_bc[6];
} pf_params;

/* Adaptive-step tolerances (Sec. 3.3): per-field relative r and absolute a,
 * the step cap in units of dt_e (<= 0 means 200) and the first step (<= 0
 * means 0.9 dt_e). */
typedef struct {
    double r_phi, a_phi, r_c, a_c;
    double dt_max_over_dte;
    double dt0;
} pf_tol;

/* Counters of a pf_step / pf_run_to call (RHS evaluations include the
 * estimator's extra one, Sec. 3.3 footnote). */
typedef struct {
    long long rhs_evals, stages, accepted, rejected;
    double t, last_dt, last_err;
} pf_stats;

/* Handle life cycle.  pf_create returns PF_EINVAL for inconsistent parameters
 * and PF_EUNSUPPORTED for an n_phi the library has no kernels for
 * (pf_supported_nphi) or a grid too large to address: the kernels split a
 * state vector's N + 1 planes into 1, 2 or 4 groups of ceil((N + 1) / groups)
 * planes, each group spanning less than 4 GiB (FP32 512^3 with N = 9 needs
 * two, FP64 four).  Walls need vectors that fit one group (else
 * PF_EUNSUPPORTED); walls on z of a 2D grid, bc values other than 0 and 1,
 * and a fixed c on a periodic axis, without c or not finite, are PF_EINVAL,
 * and so are pair tables that are not symmetric, finite and non-negative,
 * k <= 0, non-finite c0 or D, D < 0 and ssp_stages 1 or negative. */
pf_status pf_create(const pf_params *p, pf_sim **out);
pf_status pf_destroy(pf_sim *sim);

/* Use this HIP stream (hipStream_t) for every launch and copy of the handle;
 * NULL selects the null stream.  The stream must outlive its use.  On a change
 * of stream the call first waits for the handle's work on the previous stream,
 * so the two streams need not be ordered (PF_EHIP if that wait fails). */
pf_status pf_set_stream(pf_sim *sim, void *hip_stream);

/* Set the state from host doubles [F*V] (c may be NULL when with_c = 0, else
 * c is read from the same array after the phi planes when c == NULL) and the
 * time t0. phi is [n_phi*V], c is [V]. */
pf_status pf_init_fields(pf_sim *sim, const double *phi, const double *c, double t0);
/* Same from a device array of F*V values in the handle's precision. */
pf_status pf_init_fields_device(pf_sim *sim, const void *state, double t0);
/* Copy the state to host doubles (phi [n_phi*V], c [V] or NULL) and t. */
pf_status pf_get_fields(pf_sim *sim, double *phi, double *c, double *t);
/* Copy the state to a device array of F*V values in the handle's precision. */
pf_status pf_get_fields_device(pf_sim *sim, void *state);

/* One RHS evaluation of the current state (eqs. phieq, ceq; no projection)
 * into host doubles: dphi [n_phi*V], dc [V] (may be NULL). */
pf_status pf_rhs(pf_sim *sim, double *dphi, double *dc);
/* Same into a device array of F*V values in the handle's precision. */
pf_status pf_rhs_device(pf_sim *sim, void *out);

/* Stable forward-Euler step dt_e = 2 / max(lambda_phi, lambda_c) from the
 * Gershgorin-type estimates of Sec. 3.2 (formulas reconstructed from the
 * two-phase linearisation; reproduces the dt_e values of Table 3). */
pf_status pf_stable_dt(pf_sim *sim, double *dt_e);
/* RKL stage count for a step dt: smallest odd s with dt inside the exact real
 * stability interval scaled by the 0.9 safety factor (eq. sts-limit). */
pf_status pf_stage_count(pf_sim *sim, pf_integrator integ, double dt, int *s);

/* ---------------------------------------------------------------------------
 * Host-side helpers: the engine's own scalar computations, callable without a
 * handle or a device (no device memory, no launches).
 * -------------------------------------------------------------------------*/
/* pf_stable_dt of a parameter set (same validation as pf_create). */
pf_status pf_params_stable_dt(const pf_params *p, double *dt_e);
/* pf_stage_count for PF_RKL1 / PF_RKL2 given dt_e; PF_EINVAL for other
 * integrators or non-positive dt, dt_e. */
pf_status pf_rkl_stage_count(pf_integrator integ, double dt, double dt_e, int *s);

/* Step-size controller of Sec. 3.3 (PID form with gains 1.25, 0.5, -0.6, 0.25,
 * 0 on errors scaled by the bias b, limiter 1 + 5 atan((F - 1) / 5), bias
 * raised to sqrt(b) (at most 0.98) on acceptance and lowered to b^2 (at least
 * 0.1) on rejection; a step is accepted when err < 1, a non-finite err is a
 * rejection with factor 0).  pf_controller_update takes the error norm of a
 * step of size h of a method of order `order`, sets *accept and the proposed
 * next step *h_next, and advances the state as pf_run_to does. */
typedef struct {
    double b;     /* bias */
    int nhist;    /* accepted steps in the history (0..2) */
    double E1, E2, h1, h2; /* last two accepted scaled errors and steps */
} pf_controller;
pf_status pf_controller_init(pf_controller *c);
pf_status pf_controller_update(pf_controller *c, int order, double err, double h, int *accept,
                               double *h_next);

/* Exact output times (Sec. 5 opening): the step from t towards t_end has size
 * h unless the remainder is at most h (1 + 1e-10), in which case it is the
 * remainder and *last = 1 (an infinite h, as 0.9 dt_e is without mobility and
 * diffusion, always so).  Returns 1 with *h_use set, 0 when t_end is reached
 * (remainder at most 1e-12 h, or not positive for an infinite h), -1 for
 * invalid arguments. */
int pf_clip_step(double t, double t_end, double h, double *h_use, int *last);

/* One step of size dt (RKL stage count from pf_stage_count); dt must be
 * finite and > 0 (else PF_EINVAL).  stats may be NULL; otherwise it is
 * overwritten with this call's counters. */
pf_status pf_step(pf_sim *sim, pf_integrator integ, double dt, pf_stats *stats);

/* Integrate to t_end, landing on it exactly (Sec. 5 opening).  tol == NULL:
 * fixed steps of dt_fixed, the last clipped.  tol != NULL: adaptive RKL1,
 * RKL2 (estimate of Sec. 3.3 after Sommeijer), SSP(s)2 (embedded first-order
 * solution: the last Euler sub-step) or SSP(10)4 (embedded solution: the
 * tenth stage value, second order in general and third on linear problems),
 * PID controller with the method's order; steps are capped at
 * tol->dt_max_over_dte dt_e and, for SSP(s)2 and SSP(10)4, at 0.9 times their
 * stability limits (s - 1) dt_e and 6 dt_e; FE returns PF_EUNSUPPORTED.
 * t_end must be finite (else PF_EINVAL).  Where dt_e is infinite (no pair
 * mobility and no diffusivity: the right-hand side is zero) the first step,
 * 0.9 dt_e, is clipped to the remainder and lands on t_end. */
pf_status pf_run_to(pf_sim *sim, pf_integrator integ, double t_end, const pf_tol *tol,
                    double dt_fixed, pf_stats *stats);

/* Weighted RMS error norm of Sec. 3.3 (eq. error_norm) of a given local
 * error estimate, on host arrays: a pure function, no handle, no device.
 * e, u_old (u^n) and u_new (u^{n+1}) are F*cells doubles each in the state
 * layout, F = p->n_phi + (p->with_c != 0); only n_phi and with_c of p are
 * read.  Each entry is weighted by r max(|u^n|, |u^{n+1}|) + a with the
 * field's r and a from tol; the phi entries counted are those with e != 0
 * (the estimate's phi filter of Sec. 3.3 is the caller's, already in e), a
 * cell with none counts two degrees of freedom, and every c entry counts one.
 * Sums run over the cells in order (phi ascending, then c), so the result is
 * reproducible.  *out = sqrt(sum / N).  Errors: PF_EINVAL for null pointers,
 * cells < 1, n_phi outside 1..16 or negative tolerances; no other effect.
 * The adaptive steps of pf_run_to compute their norms on the device
 * (pf_error_norm_device); this form serves callers whose estimate is on the
 * host. */
pf_status pf_error_norm(const pf_params *p, long long cells, const double *e, const double *u_old,
                        const double *u_new, const pf_tol *tol, double *out);

/* The same norm with the estimate formed on the GPU from device state vectors
 * in the handle's precision, FP64 accumulation in a fixed order.  kind 0:
 * the estimate of Sec. 3.3 after Sommeijer from u_old = u^n, u_new = u^{n+1},
 * aux = rhs(u^n) and the step dt (one extra RHS of u_new is evaluated), with
 * the phi filter; kind 1: the embedded estimate e = u_new - aux.  Writes the
 * norm and, if non-NULL, the DoF count N.  Allocates the handle's per-tile
 * partial sums on first use. */
pf_status pf_error_norm_device(pf_sim *sim, int kind, double dt, const void *u_old,
                               const void *u_new, const void *aux, const pf_tol *tol,
                               double *norm, long long *ndof);

/* pf_error_norm_device for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same estimate, norm, arguments and result bits, but its
 * partial sums go to a static device array of the library (2 MiB, held by
 * each GPU the library runs on until the process ends) instead of memory the
 * handle allocates, and it creates no timing events.  It calls no hipMalloc,
 * hipFree or other allocating routine.  Limit: kind 0 needs one partial per
 * tile of the stage kernels (64 x 4 cells times the z extent of
 * pf_set_tiling in 3D; 64 x 8 cells in 2D with N <= 4, else 64 x 4), at most
 * 131072;
 * kind 1 needs 1024.  A larger request returns PF_EINVAL and launches
 * nothing.  Every call on one GPU uses that GPU's one array, so calls that
 * overlap on a GPU (other threads, other streams) race and must be
 * serialised by the caller; the array keeps the last call's contents, and
 * each call writes every entry it reads. */
pf_status pf_error_norm_device_noalloc(pf_sim *sim, int kind, double dt, const void *u_old,
                                       const void *u_new, const void *aux, const pf_tol *tol,
                                       double *norm, long long *ndof);

/* FP64 sum of c over all cells of the current state (GPU reduction, fixed
 * order, so repeated calls give identical bits). */
pf_status pf_conservation(pf_sim *sim, double *sum_c);
/* Constraint diagnostics of the current state: out[0] = sum c,
 * out[1] = max |sum_a phi_a - 1|, out[2] = min phi, out[3] = max phi,
 * out[4] = number of non-finite values. */
pf_status pf_diagnostics(pf_sim *sim, double out[5]);

/* Attempt log of the last pf_run_to: 4 doubles per attempt (dt, s, e,
 * accepted).  Copies min(n, cap) rows into buf and writes n. */
pf_status pf_get_trace(pf_sim *sim, double *buf, long long cap, long long *n);

/* Checkpoint: the state in the handle's precision plus t, the controller
 * state and the counters.  With buf == NULL, *len receives the size. */
pf_status pf_get_state(pf_sim *sim, void *buf, size_t *len);
pf_status pf_set_state(pf_sim *sim, const void *buf, size_t len);

/* Launch shape of the stencil kernels: the tile width tx (fixed by the
 * build: 64 cells, where a block of 256 threads covers 64 x 4 cells, or in 2D
 * 64 x 8 for N <= 4; a build option makes 3D tiles 32 x 8; pf_set_tiling takes
 * 0 or that width) and the number of z planes a block marches through (3D
 * only, >= 1).  pf_autotune times the RKL2 inner stage at
 * the z extents 4..256 (inputs: the current state and copies of it in three
 * work buffers, which it allocates if the handle has not yet; the state is only
 * read), in two interleaved passes keeping each extent's faster time, and
 * keeps the fastest extent.  Where fused stage pairs are built (below) it
 * also times pair launches (a fifth work buffer takes their second output;
 * in 3D at the pair z extents 8..128) and sets the fusion depth to 2 if a
 * pair takes less than two single stages, else to 1; on periodic 3D grids it
 * also times the stages that recompute R0 (pf_set_r0_recompute) at the same z
 * extents and turns that mode on if one is the fastest single stage, else
 * off; best_ms is then the time per stage of the choice.  The launch shape
 * and these modes never change a result bit. */
pf_status pf_set_tiling(pf_sim *sim, int tx, int zchunk);
pf_status pf_get_tiling(pf_sim *sim, int *tx, int *zchunk);
pf_status pf_autotune(pf_sim *sim, int *tx, int *zchunk, double *best_ms);

/* Least number of buffer groups per state vector (0: the fewest that address
 * the vectors, the default; 1, 2 or 4).  The stage kernels are compiled per
 * group count and read each field plane through its group's descriptor; more
 * groups than the grid needs address the same planes and give the same result
 * bits.  Errors: PF_EINVAL for other values or fewer groups than the grid
 * needs; PF_EUNSUPPORTED for more than one group on a grid with walls.
 * In 2D, fused RKL2 stage pairs (below) run only with one group.
 * pf_get_field_groups reports the count the kernels use. */
pf_status pf_set_field_groups(pf_sim *sim, int ng);
pf_status pf_get_field_groups(const pf_sim *sim, int *ng);

/* Sparse phase storage (Sec. 3.1 "Phase-field details"): with n_p > 0 each
 * cell of a state vector holds c, the values of at most n_p nonzero phases
 * (ascending phase order) and a 32-bit word of their phase ids (4 bits each),
 * instead of all N phase values; the stage kernels read the slots into the
 * dense values they compute with, so while no cell has more than n_p nonzero
 * phases the results equal dense storage bit for bit.  A projected stage with
 * more nonzero phases keeps the n_p largest (equal values: the lower phase),
 * divided by their sum; pf_sparse_cuts returns (and resets) the number of
 * cells so cut since pf_set_sparse_storage.  n_p = 0 returns to dense
 * storage.  The call frees the work buffers and clears the fields (call
 * pf_init_fields after it); host and device field arrays keep the dense
 * layout in every call.  Built for periodic grids whose vectors need one or
 * two buffer groups; it runs forward Euler, RKL1 and RKL2 fixed steps and the
 * RHS (SSP schemes, adaptive steps, error norms and checkpoints return
 * PF_EUNSUPPORTED; fused stage pairs are not used).  Errors: PF_EINVAL for n_p
 * outside 0..min(8, N); PF_EUNSUPPORTED for walls or more buffer groups. */
pf_status pf_set_sparse_storage(pf_sim *sim, int n_p);
pf_status pf_get_sparse_storage(const pf_sim *sim, int *n_p);
pf_status pf_sparse_cuts(pf_sim *sim, long long *cuts);

/* RKL2 inner stages per launch (eq. sts, stages j >= 2): 1, or 2 for stages j
 * and j + 1 in one pass over memory (four vectors read and two written per
 * pair instead of five per stage; a step with an odd count of inner stages
 * runs its first inner stage alone).  Depth 2 keeps a ring of four stage
 * vectors (one more work buffer than depth 1) and gives the same result bits
 * as depth 1.  It is built for periodic grids: in 2D where the vectors fit one
 * buffer group and the tile (64 x 8 cells with a two-cell halo, N + 3 planes,
 * and a one-cell ring of N + 2 planes) fits 64 KiB of LDS (single precision
 * N <= 8, double precision N = 2); in 3D (a tile of 32 x 8 cells marched
 * through the z extent of pf_set_pair_zchunk, 448 threads per block, one z
 * window of each stage per thread in registers) in single precision for
 * N <= 9 and in double precision for N <= 4, with any buffer-group count.
 * Errors: PF_EINVAL for another depth; PF_EUNSUPPORTED for depth 2 where it
 * is not built.  The default is 2 in 2D where it is built, else 1;
 * pf_autotune chooses by timing. */
pf_status pf_set_stage_fusion(pf_sim *sim, int depth);
pf_status pf_get_stage_fusion(const pf_sim *sim, int *depth);
/* RKL2 inner stages of periodic 3D grids (eq. sts, stages j >= 2) that
 * recompute R0 instead of reading it: on = 1 reads u^{n,0} as a second
 * stencil input and forms R0 = rhs(u^{n,0}) with the correction of the first
 * stage (Sec. 3.2, end) at every cell, so 4 (N + 1) values move per
 * cell-stage instead of 5 (N + 1), for a second right-hand side per cell.
 * The results are the same bits as with the stored R0 (which the first stage
 * still writes, for the error estimate).  on = 0 (the default) reads R0.
 * Built for single precision N <= 9 and double precision N <= 4 (two z
 * windows of N + 1 values per thread for two waves per SIMD).  Errors:
 * PF_EINVAL for other values; PF_EUNSUPPORTED for 2D grids, walls, sparse
 * storage or an N it is not built for.  With fused stage pairs (depth 2) the
 * pairs run instead.
 * pf_autotune times it at the single-stage z extents and keeps it where it
 * is faster. */
pf_status pf_set_r0_recompute(pf_sim *sim, int on);
pf_status pf_get_r0_recompute(const pf_sim *sim, int *on);
/* z planes per block of the 3D fused stage pairs (>= 1; default 32; the
 * autotuner times 8..128).  Never changes a result bit. */
pf_status pf_set_pair_zchunk(pf_sim *sim, int zchunk);
pf_status pf_get_pair_zchunk(const pf_sim *sim, int *zchunk);

/* Per-kernel timing with HIP events recorded on the handle's stream around
 * every launch while enabled.  Families: 0 stage kernels (all stage kinds),
 * 1 estimator, 2 reductions, 3 RKL2 inner stages (j >= 2) only, 4 FE stages.
 * pf_get_kernel_time synchronises the stream and returns the total ms and the
 * number of launches of a family since timing was enabled. */
pf_status pf_set_timing(pf_sim *sim, int enable);
/* The same for a subset of the families (bit f = family f; 0 disables):
 * events are recorded only around the selected families' launches, so that a
 * timed run carries no event between the launches of the others. */
pf_status pf_set_timing_families(pf_sim *sim, unsigned families);
pf_status pf_get_kernel_time(pf_sim *sim, int family, double *ms, long long *launches);

/* ---------------------------------------------------------------------------
 * Batch of independent 2D simulations.  All instances share dim = 2, n_phi,
 * with_c and the precision; grid sizes and every other parameter may differ.
 * Each instance's state must span less than 4 GiB and its boundaries must be
 * periodic (else PF_EUNSUPPORTED).
 * A launch of the batch advances every instance by one forward-Euler step
 * (Sec. 3.2), or by two (stage-fusion depth 2: a tile computes the first step
 * on itself and a one-cell ring, the second on itself, in one pass over HBM);
 * a persistent grid walks a tile list whose entries name their instance, the
 * per-instance parameters, state offsets and step sizes live in device
 * tables, and sequences of launches are replayed from a captured hipGraph.
 * Results do not depend on the depth or the grid size: every instance takes
 * bit for bit the steps of its own single-instance run.
 * -------------------------------------------------------------------------*/
typedef struct pf_batch pf_batch;

pf_status pf_batch_create(const pf_params *per_inst, int n, pf_batch **out);
pf_status pf_batch_destroy(pf_batch *b);
/* A non-null HIP stream for the batch's launches (graph capture needs one; by
 * default the batch owns a stream of its own).  On a change of stream the call
 * first waits for the batch's work on the previous stream. */
pf_status pf_batch_set_stream(pf_batch *b, void *hip_stream);
/* Instance i's state from host doubles [F*V_i] and its time. */
pf_status pf_batch_init_fields(pf_batch *b, int i, const double *u, double t0);
pf_status pf_batch_get_fields(pf_batch *b, int i, double *u, double *t);
pf_status pf_batch_stable_dt(pf_batch *b, int i, double *dt_e);
/* Fixed steps of every instance to its t_end[i] (steps dt[i], or 0.9 dt_e of
 * the instance when dt == NULL; the last step is clipped exactly as pf_run_to
 * clips it, so each instance takes the steps of its own single-instance run).
 * integ: PF_FEULER, or PF_RKL2 (eq. sts; each instance with its own stage
 * count per step, eq. sts-limit, and its coefficients from a device table; a
 * step is one launch per stage over all instances whose step has that stage;
 * the RKL2 ring, R0 and the table are allocated on the first RKL2 run and
 * kept); others return PF_EUNSUPPORTED.  graph_steps > 0 replays a graph of
 * that many launches (forward Euler) or steps (RKL2); 0 launches directly.
 * Every t_end[i] must be finite (else PF_EINVAL).  stats (optional) is [n]. */
pf_status pf_batch_run_to(pf_batch *b, pf_integrator integ, const double *t_end,
                          const double *dt, int graph_steps, pf_stats *stats);
/* Adaptive RKL2 steps of every instance to its t_end[i] (Sec. 3.3): each
 * instance runs the loop of pf_run_to with tol (Sommeijer estimate of eq.
 * sts with the phi filter, the weighted norm with its degree-of-freedom rule,
 * the PID controller with bias and limiter, exact t_end), with a controller of
 * its own that starts fresh (first step tol->dt0, or 0.9 dt_e of the instance
 * when tol->dt0 <= 0), so every instance takes bit for bit the steps of a fresh
 * single-instance pf_run_to(PF_RKL2, t_end[i], tol).  A batch step runs the
 * stages, the estimate and the norms of all instances still running in
 * batched launches and returns the norms to the host once; rejected instances
 * keep their state.  integ must be PF_RKL2 and the batch may hold at most
 * 65535 instances (else PF_EUNSUPPORTED).  Errors:
 * PF_EINVAL for negative tolerances, a field kind with zero weight or t_end[i]
 * before the instance's time or not finite; PF_EDTMIN on a step underflow; PF_ENONFINITE
 * after three non-finite norms of one instance in a row (the instances keep
 * their last accepted states).  Allocates the adaptive work buffers (the new
 * state, per-tile partials, norms) on the first call.  stats (optional) is [n]:
 * accepted and rejected steps, stages, RHS evaluations (estimate included),
 * last step, last norm and t of each instance. */
pf_status pf_batch_run_adaptive(pf_batch *b, pf_integrator integ, const double *t_end,
                                const pf_tol *tol, pf_stats *stats);
/* Times one launch for each persistent grid size (512..8192 blocks) and each
 * fusion depth the instances allow (the state is only read) and keeps the
 * fastest per step; best_ms is that time per step.  pf_batch_set_blocks sets
 * the grid size directly (rounded down to a multiple of 8, >= 8);
 * pf_batch_set_fusion the depth (1 or 2; depth 2 is built for n_phi <= 4,
 * where its LDS fits one workgroup in either precision, and returns
 * PF_EUNSUPPORTED otherwise);  pf_batch_get_config
 * reads both (either pointer may be NULL). */
pf_status pf_batch_autotune(pf_batch *b, int *nblocks, double *best_ms);
pf_status pf_batch_set_blocks(pf_batch *b, int nblocks);
pf_status pf_batch_set_fusion(pf_batch *b, int depth);
pf_status pf_batch_get_config(const pf_batch *b, int *nblocks, int *depth);
const char *pf_batch_last_error(const pf_batch *b);

/* Values of N for which kernels are compiled; returns the count. */
int pf_supported_nphi(int *out, int cap);

const char *pf_last_error(const pf_sim *sim);

#ifdef __cplusplus
}
#endif

#endif /* PF_H */
