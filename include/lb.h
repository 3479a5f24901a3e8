/*
 * lb.h -- C ABI of the MI355X multiscale lattice Boltzmann library.
 *
 * The library advances the discrete-velocity BGK equation (Meng, Zhang &
 * Shan, "Multiscale lattice Boltzmann approach to modeling gas flows",
 * Sec. 2.1, Eq. (lbgk)) on a 2D lattice with the forward-Euler / TVD-minmod
 * scheme of Sec. 3.1, diffuse-reflection walls (Sec. 3.2), a low-order
 * Gauss-Hermite velocity set in the core and a high-order set in bands next
 * to the walls, joined by an interface step (Sec. 2.2).
 *
 * Conventions
 *  - Every call returns an lb_status (LB_OK = 0, errors < 0); nothing throws
 *    or aborts across the ABI.  lb_last_error() returns a thread-local text
 *    for the last failure.
 *  - Units: grid spacing 1; velocities in units of sqrt(R T0), so the
 *    Gauss-Hermite abscissae are the particle speeds; temperatures in units
 *    of T0.  Isothermal lattices (the default) fix T = 1; thermal lattices
 *    (lb_params.thermal) take each node's T from its energy moment.  Node rows are
 *    j = 0..ny (ny + 1 rows); with walls, rows 0 and ny are the wall nodes and
 *    the channel height ny is the length of Eq. (KN): the relaxation time at
 *    density rho_ref is kn * ny.
 *  - A velocity set is named by its 1D point count n: 3 = D2Q9, 4 = D2Q16,
 *    6 = D2Q36 (tensor products of the n-point Gauss-Hermite rule, Sec. 2.1).
 *    Population alpha = p + n*q has velocity (x_p, x_q), abscissae ascending.
 *  - Host arrays of lattice fields are [ny+1][nx] doubles, row j slow.
 *    Population arrays are [Q][ny+1][nx] doubles.
 *  - Memory: the caller owns one device workspace per lattice (size from
 *    lb_workspace_bytes) and a HIP stream; lattice calls allocate no device
 *    memory.  Device allocations happen only in lb_batch_create (the batch's
 *    descriptor table and work lists, freed by lb_batch_destroy), in
 *    lb_mlp_forward / lb_mlp_loss_grad callers' workspaces (caller-owned) and
 *    in the lb_closure_eval test hook (a temporary weight copy); the
 *    allocation-free lb_mlp_forward_noalloc uses a library-owned device array.
 *    Host pointers are only read or written during the call.
 *  - Asynchrony: lb_step and the on-device variants enqueue work on the
 *    stream and return; errors found by kernels surface at the next call that
 *    synchronises (lb_conservation, host-side moments, get_* calls).
 */
#ifndef LB_H
#define LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LB_OK = 0,
    LB_EINVAL = -1,        /* invalid argument or parameter combination */
    LB_ENOMEM = -2,        /* workspace too small */
    LB_EDEVICE = -3,       /* a HIP runtime call failed */
    LB_EUNSTABLE = -4,     /* a reduction found a non-finite value */
    LB_EUNSUPPORTED = -5,  /* valid, but no kernel was built for it */
    LB_ESTATE = -6         /* call out of order (e.g. step before init) */
} lb_status;

typedef enum { LB_STORE_F64 = 0, LB_STORE_F32 = 1, LB_STORE_BF16 = 2 } lb_storage;
typedef enum { LB_IFACE_HERMITE = 0, LB_IFACE_PAPER = 1 } lb_iface;
typedef enum { LB_TAU_CONST = 0, LB_TAU_RHO = 1 } lb_tau_mode;
typedef enum { LB_XBC_PERIODIC = 0, LB_XBC_PRESSURE = 1 } lb_xbc;
/* LB_YBC_SHEAR (Kramers' problem, Sec. 3.3): a diffuse wall on row 0 and,
 * above the top row ny (an ordinary gas node), the far-field condition of
 * an imposed shear rate: ghost row k = 1, 2 holds the equilibrium at the top
 * node's density with its velocity raised by shear_top * k along x, plus the
 * top node's non-equilibrium part. */
typedef enum { LB_YBC_WALLS = 0, LB_YBC_PERIODIC = 1, LB_YBC_SHEAR = 2 } lb_ybc;

typedef struct lb_params {
    int32_t nx, ny;            /* nx columns (>= 2); ny intervals -> ny+1 rows (>= 4) */
    int32_t n_low, n_high;     /* 1D Gauss-Hermite points of the low / high set */
    int32_t eq_low, eq_high;   /* Hermite order of each set's equilibrium, Eq. (approxfeq) */
    int32_t force_low, force_high; /* order of the body-force expansion; 0 = eq order */
    int32_t tau_mode;          /* lb_tau_mode: constant, or kn*ny*rho_ref/rho */
    int32_t xbc, ybc;          /* lb_xbc, lb_ybc */
    int32_t iface;             /* lb_iface */
    int32_t storage;           /* lb_storage of the populations */
    int32_t tile_w;            /* columns per band tile; 0 = nx (one tile) */
    double kn;                 /* Knudsen number of Eq. (KN) at rho_ref */
    double rho_ref;            /* reference density (also the storage shift) */
    double cfl;                /* per-axis Courant number of the fastest abscissa */
    double dt;                 /* > 0 overrides cfl: explicit time step */
    double gx, gy;             /* body force per unit mass */
    double u_wall[4];          /* bottom (x, y), top (x, y) wall velocity */
    double rho_in, rho_out;    /* pressure x-boundary densities (LB_XBC_PRESSURE) */
    double u_osc, omega_osc;   /* oscillating bottom wall (oscillatory Couette flow,
                                  Sec. 3.5): its x velocity is u_wall[0] +
                                  u_osc sin(omega_osc t), with t = (n + 1) dt when
                                  step n -> n + 1 applies the wall condition */
    double shear_top;          /* LB_YBC_SHEAR: imposed du/dy above the top row */
    /* Thermal lattice (the non-isothermal form of Eq. (demoeq), Sec. 3.2 and
     * Sec. 2.2): thermal != 0 takes every node's temperature from its energy
     * moment, sum xi^2 f = rho (u^2 + 2 T), and uses it in the equilibrium's
     * Hermite coefficients (the Maxwellian's, to the set's order), in the
     * force, in the relaxation rate of LB_TAU_RHO (collision frequency p / mu
     * with p = rho T: tau = kn ny rho_ref / (rho T)), in the pressure and
     * shear ghost nodes (the edge node's T), in the interface (T_I, the
     * neighbours' average, LB_IFACE_PAPER; the projection's equilibria at
     * the node's T, LB_IFACE_HERMITE) and in the indicator (heat flux).
     * The diffuse walls emit S(T_wall, u_wall).  Built for FP64 and FP32
     * storage; not for batches or the learned closure.  Ignored when
     * thermal == 0 (T = 1 everywhere, walls included). */
    double T_wall[2];          /* bottom, top wall temperature (> 0) */
    int32_t thermal;           /* 0 = isothermal (default), 1 = thermal */
    int32_t reserved_;         /* 0 */
} lb_params;

typedef struct lb_lattice lb_lattice;

/* Text of the last error on this thread ("" if none). */
const char *lb_last_error(void);

/* Fill p with defaults: D2Q9 everywhere, eq order 2, HERMITE interface,
 * F64 storage, walls, periodic x, kn = 0.1, rho_ref = 1, cfl = 0.5,
 * isothermal, wall temperatures 1. */
lb_status lb_params_default(lb_params *p);

/* Device workspace needed for a lattice with parameters p (0 on invalid p). */
size_t lb_workspace_bytes(const lb_params *p);

/* Create a lattice in the caller's device workspace (>= lb_workspace_bytes,
 * 256-byte aligned), enqueuing on hip_stream (a hipStream_t; NULL = the null
 * stream).  Validates p (LB_EINVAL: sizes, orders above floor(n - 1/2)
 * (the quadrature-degree rule after Eq. (approxfeq)), Courant number above
 * 0.5, dt above the relaxation time; LB_EUNSUPPORTED: set pairs without a
 * kernel).  Regions start as all-low; populations are unset until
 * lb_init_equilibrium or lb_set_populations. */
lb_status lb_create_lattice(const lb_params *p, void *dev_workspace, size_t bytes,
                            void *hip_stream, lb_lattice **out);

void lb_destroy_lattice(lb_lattice *L);

/* Time step, relaxation time at rho_ref and number of band tiles. */
lb_status lb_get_info(const lb_lattice *L, double *dt, double *tau0, int32_t *ntiles);

/* Domain decomposition (Sec. 2.2 procedure): per band tile t, rows
 * j < band_lo[t] and j > ny - band_hi[t] use the high set, the rest the low
 * set.  With LB_IFACE_PAPER, the first row past each non-empty band is the
 * interface row of Sec. 2.2 (not evolved), and all tiles must have the same
 * bands.  Host arrays of ntiles entries.  Existing populations are not
 * converted: use lb_update_regions for that. */
lb_status lb_set_regions(lb_lattice *L, const int32_t *band_lo, const int32_t *band_hi);
lb_status lb_get_regions(const lb_lattice *L, int32_t *band_lo, int32_t *band_hi);

/* Equilibrium start (Eq. approxfeq) from host fields; NULL = rho_ref / 0. */
lb_status lb_init_equilibrium(lb_lattice *L, const double *rho, const double *ux, const double *uy);

/* The same with a temperature field T (host [ny+1][nx], NULL = 1): the
 * Maxwellian's Hermite expansion at (rho, u, T) to each set's order.
 * LB_EINVAL on an isothermal lattice when T is given. */
lb_status lb_init_equilibrium_thermal(lb_lattice *L, const double *rho, const double *ux, const double *uy,
                                      const double *T);

/* Advance nsteps time steps (Sec. 3.1 update, Sec. 3.2 walls, Sec. 2.2
 * interface).  Asynchronous on the lattice stream.  With an oscillating
 * bottom wall, the host recomputes that wall's equilibrium sums for every
 * step (time-dependent kernel arguments, no device-side state). */
lb_status lb_step(lb_lattice *L, int64_t nsteps);

/* Density and velocity of every node ([ny+1][nx], FP64): the zeroth and first
 * Hermite coefficients of Eq. (an), rho = sum f, rho u = sum xi f, in the
 * node's own set (interface rows report the interpolated values).
 * on_device != 0: the three pointers are device memory and the call is
 * asynchronous; else host memory and the call waits. */
lb_status lb_moments(lb_lattice *L, double *rho, double *ux, double *uy, int32_t on_device);

/* out[0..2] = sum rho, sum rho ux, sum rho uy over all nodes (the moments
 * of lb_moments, Eq. (an)), reduced in FP64 in a fixed order
 * (deterministic).  Waits.  LB_EUNSTABLE if not finite. */
lb_status lb_conservation(lb_lattice *L, double out[3]);

/* Temperature T = (sum xi^2 f / rho - u^2) / 2 and heat flux
 * q = 1/2 sum (xi - u) |xi - u|^2 f of every node ([ny+1][nx], FP64; the
 * heat flux of the 'B' parameter of Sec. 2.2).  Any lattice (an isothermal
 * one reports the temperature its populations carry).  on_device as for
 * lb_moments. */
lb_status lb_thermal_moments(lb_lattice *L, double *T, double *qx, double *qy, int32_t on_device);

/* *out = total energy, the sum over all nodes of 1/2 sum_alpha xi_alpha^2
 * f_alpha, reduced like lb_conservation (deterministic).  Waits.
 * Conserved by the update of a periodic thermal lattice. */
lb_status lb_energy(lb_lattice *L, double *out);

/* Populations of set which (0 = low, 1 = high) as FP64 host arrays
 * [Q][ny+1][nx].  get: nodes not evolved in that set (and not interface
 * rows) read as NaN.  set: only those nodes are read; the ghost, image and
 * interface entries are then rebuilt. */
lb_status lb_get_populations(lb_lattice *L, int32_t which, double *host);
lb_status lb_set_populations(lb_lattice *L, int32_t which, const double *host);

/* Raw state (both sets' population buffers + step counter) for
 * checkpointing; bit-exact round trip.  Waits. */
size_t lb_state_bytes(const lb_lattice *L);
lb_status lb_get_state(lb_lattice *L, void *host, size_t bytes);
lb_status lb_set_state(lb_lattice *L, const void *host, size_t bytes);
int64_t lb_step_count(const lb_lattice *L);

/* Non-equilibrium indicator per node (the 'B' breakdown parameter of
 * Sec. 2.2 made dimensionless), FP64 [ny+1][nx].  Isothermal lattices: max
 * over the second-order Hermite components of |a_km - rho ux^k uy^m| / rho.
 * Thermal lattices: max of |P_ij - p delta_ij| / p (ij = xx, xy, yy;
 * P_ij = sum c_i c_j f, c = xi - u, p = rho T) and |q_i| / (p sqrt(T)). */
lb_status lb_indicator(lb_lattice *L, double *B, int32_t on_device);

/* Re-decompose from the indicator: per tile, the bottom band reaches one row
 * past the highest lower-half row with B > theta (mirrored at the top),
 * clamped to [bmin, bmax].  Nodes that change set are converted by the
 * Hermite projection.  Waits (the band arrays come back to the host). */
lb_status lb_update_regions(lb_lattice *L, double theta, int32_t bmin, int32_t bmax);

/* Replace the decomposition with explicit bands, converting switched nodes
 * by the Hermite projection (lift to / restriction from the high set). */
lb_status lb_change_regions(lb_lattice *L, const int32_t *band_lo, const int32_t *band_hi);

/* Hermite-moment projection of n nodes from set (ns, eqs) to set (nd, eqd)
 * (Sec. 2.2 in moment form): equilibrium rebuilt in the target set from
 * rho, u; non-equilibrium coefficients carried where both sets resolve
 * them; missing ones from closure[nd*nd per node] (NULL = 0).  Device
 * arrays [node][Q] in FP64.  Asynchronous on hip_stream. */
lb_status lb_project(int32_t ns, int32_t eqs, int32_t nd, int32_t eqd, const double *f_src,
                     const double *closure, double *f_dst, int64_t n, void *hip_stream);

/* Kernel timing: enable = N >= 1 turns it on, and the update-kernel launches
 * of every Nth step (step count divisible by N; N = 1: every step) record
 * start and stop HIP events (hipExtLaunchKernelGGL) on the lattice stream;
 * 0 turns it off, a negative value is LB_EINVAL.  lb_kernel_times returns, for the
 * dominant update kernel (the set that moves the most bytes per step) and
 * for all update kernels, the summed duration in ms and the launch count,
 * then clears them.  Waits. */
lb_status lb_set_timing(lb_lattice *L, int32_t enable);
lb_status lb_kernel_times(lb_lattice *L, double *ms_high, int64_t *n_high, double *ms_all,
                          int64_t *n_all);

/* Update both sets in one kernel launch (on by default; used when the low
 * set is D2Q9 and both sets have nodes): the high set's work items and the
 * D2Q9 items share the launch instead of running back to back.  Results
 * are identical either way.  In timing mode the merged launch is the
 * dominant kernel reported by lb_kernel_times.  Thermal lattices with a
 * D2Q9 low set always use the merged launch (also when the high set has no
 * nodes): disabling it returns LB_EUNSUPPORTED, as do lb_set_concurrency(1)
 * and lb_autotune on them (both need the D2Q9 update launched alone). */
lb_status lb_set_merged_update(lb_lattice *L, int32_t enable);

/* Run the low set's update and its projection into the high set on a
 * second stream (created by the library on first use, default priority),
 * concurrently with the high set's update and projection; the streams join
 * before the end of every step, so lb_step stays ordered on the lattice's
 * stream.  Off by default: each step then adds two event records and two
 * stream waits on the host, which cost more than the overlap gains unless
 * the host is far ahead of the GPU; results are identical either way
 * (batches, whose steps replay from graphs, always overlap).  Timing mode
 * (lb_set_timing) launches everything on the lattice's stream. */
lb_status lb_set_concurrency(lb_lattice *L, int32_t enable);

/* Rows per work item of the update kernels (tuning; 0 = automatic: enough
 * items to fill the GPU, at most 16 rows). */
lb_status lb_set_strip_rows(lb_lattice *L, int32_t rows);

/* Current rows per work item of the low and high set's update kernel. */
lb_status lb_get_strip_rows(const lb_lattice *L, int32_t rows[2]);

/* Work shape of each set's update kernel: rows per work item (0 = automatic)
 * and item order (0 = XCD slabs of column groups, row-major inside; 1 =
 * column-major), low set first.  lb_autotune picks both; these reproduce
 * or inspect its choice. */
lb_status lb_set_work_shape(lb_lattice *L, const int32_t rows[2], const int32_t order[2]);
lb_status lb_get_work_shape(const lb_lattice *L, int32_t rows[2], int32_t order[2]);

/* Project-written autotuner: for each set, time the update kernel (kernel
 * events over `steps` steps, twice, the faster pass counting) for each
 * candidate strip height and item order
 * (per-XCD column slabs walked row-major, or column-major) and keep the
 * fastest; with two sets, then time the whole step for the strip heights
 * within one row of those choices (twice each) and keep the fastest.  The
 * lattice state is saved before and restored after, so the physics is not
 * advanced.  rows_out (may be NULL) receives the choice. */
lb_status lb_autotune(lb_lattice *L, int32_t steps, int32_t rows_out[2]);

/* Number of nodes in each region: [0] low set, [1] high set, [2] interface
 * rows (interpolation mode only). */
lb_status lb_region_counts(const lb_lattice *L, int64_t counts[3]);

/* ---------------------------------------------------------------------
 * Learned interface closure.  When low-order (D2Q9) populations are lifted
 * to the high-order set (D2Q36, order 4), the non-equilibrium Hermite
 * coefficients D2Q9 cannot carry are unknown (0 in the analytic
 * projection).  A perceptron 10 -> 64 -> 64 -> 8 (tanh, tanh, linear)
 * predicts the six of total order 3-4 -- (3,0), (0,3), (3,1), (1,3), (4,0),
 * (0,4) -- plus two logits of a region flag (indicator above threshold).
 * Inputs, from the node's D2Q9 populations: rho - 1, ux, uy, log Kn_loc and
 * the non-equilibrium coefficients (2,0), (1,1), (0,2), (2,1), (1,2), (2,2)
 * over rho; inputs and targets are standardised (norm = 10 input means,
 * 10 input deviations, 6 target means, 6 target deviations).  Parameters
 * are FP32, layout W1[64][10], b1[64], W2[64][64], b2[64], W3[8][64], b3[8].
 * Training runs in FP32; inference in the lift uses bf16 weights.
 * All pointers are device memory unless said otherwise. */
int64_t lb_mlp_param_count(void);
size_t lb_mlp_workspace_bytes(int64_t n);

/* y[n][8] = network(x[n][10]) in FP32. */
lb_status lb_mlp_forward(const float *params, const float *x, float *y, int64_t n, void *ws, void *hip_stream);

/* Allocation-free variant of lb_mlp_forward, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same kernels and results,
 * with the hidden activations in a library-owned device array of
 * 2 x 64 x LB_MLP_NOALLOC_MAX_N floats (8 MiB) that each GPU holds until the
 * process ends, in place of the caller's workspace.  n above
 * LB_MLP_NOALLOC_MAX_N is rejected with LB_EINVAL before anything is
 * enqueued.  The stream must belong to the current device.  Calls share
 * that device's array: calls that overlap on one GPU (other streams, other
 * host threads) race and must be ordered by the caller.  Nothing in the
 * array needs clearing: each layer writes its rows before the next reads
 * them.  Calls no hipMalloc / hipFree. */
#define LB_MLP_NOALLOC_MAX_N 16384
lb_status lb_mlp_forward_noalloc(const float *params, const float *x, float *y, int64_t n, void *hip_stream);

/* Gradient of the batch mean of [squared error of the 6 regression outputs
 * / 6 + cross-entropy of the 2 flag logits]; loss = that mean (device
 * float).  Deterministic. */
lb_status lb_mlp_loss_grad(const float *params, const float *x, const float *t, const int32_t *flag, int64_t n,
                           float *grad, float *loss, void *ws, void *hip_stream);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected), step >= 1. */
lb_status lb_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t step, float lr,
                      void *hip_stream);

/* Closure coefficients (row-major 6x6 Hermite indices, zero outside the six
 * predicted components) of n D2Q9 nodes given as FP64 absolute populations
 * [n][9]; norm is a host array of 32 floats.  Evaluated as in the lift:
 * bf16 weights on the matrix cores.  Test hook: allocates a temporary copy
 * of the weights (stream-ordered). */
lb_status lb_closure_eval(const float *params, const float *norm, double kn_ref, int32_t tau_rho, double rho_ref,
                          const double *f9, int64_t n, double *c36, void *hip_stream);

/* Training samples from a lattice whose listed nodes (j*nx + i) are in the
 * D2Q36 set: raw (unstandardised) features of the node restricted to D2Q9
 * x[n][10], raw targets t[n][6] (missing non-equilibrium coefficients over
 * rho) and flag[n] (indicator above theta).  A listed index outside the
 * lattice gets NaN features and targets and flag -1.  Asynchronous. */
lb_status lb_closure_samples(lb_lattice *L, const int32_t *nodes, int64_t n, double theta, float *x, float *t,
                             int32_t *flag);

/* Use the network in every D2Q9 -> D2Q36 lift of this lattice (params
 * device FP32, norm host [32]): the halo lift at the end of every step,
 * nodes switched to D2Q36 by a region change, and the halo rebuilt after
 * it.  params == NULL restores the analytic projection.  Waits. */
lb_status lb_set_closure(lb_lattice *L, const float *params, const float *norm);

/* Use the network's region flag (its two last outputs: does the node call
 * for the high-order set) in lb_update_regions, beside the indicator: every
 * node whose flag logits favour the high set counts as above the threshold
 * in the band rule.  Inputs are the node's D2Q9 populations, or its D2Q36
 * populations restricted to D2Q9 (Hermite projection).  Needs
 * lb_set_closure first (LB_ESTATE otherwise); lb_set_closure(NULL) turns it
 * off. */
lb_status lb_set_closure_flags(lb_lattice *L, int32_t enable);

/* ---------------------------------------------------------------------
 * Batches: many independent lattices (channels of different size, Kn and
 * velocity-set pair) advanced together.  Each step issues, in order on the
 * batch stream, one update launch covering every velocity set of every
 * lattice, one interface-projection launch covering the set pairs D2Q9 /
 * D2Q36, D2Q16 / D2Q36 and D2Q9 / D2Q16 (other pairs: one launch each),
 * and the finish passes of lattices that need them, instead of launches
 * per lattice; with a graph segment set, runs of that many steps are
 * captured once into a HIP graph and replayed.  Every step of every
 * lattice is the same computation as lb_step (bit-identical results).
 *
 * The lattices stay owned by the caller and must outlive the batch; they
 * must share a storage type, be isothermal, use the Hermite interface, have
 * no learned closure set and no oscillating wall (graph replays repeat the
 * captured kernel arguments), and be at the same copy parity (same step
 * count modulo 2).
 * A lattice stepped on its own in between makes lb_batch_step fail with
 * LB_ESTATE; region changes are picked up (the work lists are rebuilt).
 * The batch allocates its descriptor table and work lists with hipMalloc.
 * hip_stream must be a created stream (not the null stream) for graphs; the
 * batch orders itself after and before the lattices' own streams. */
typedef struct lb_batch lb_batch;

lb_status lb_batch_create(lb_lattice *const *lattices, int32_t n, void *hip_stream, lb_batch **out);
void lb_batch_destroy(lb_batch *B);

/* Persistent launches (off by default): one kernel launch advances every
 * lattice by a run of steps (up to 4096 per launch; with a graph segment
 * set, one launch per segment, captured).  Each workgroup owns whole
 * lattices, assigned largest-first by populations x nodes, and loops over
 * the steps with workgroup barriers only (no workgroup waits on another):
 * in each step its waves take the lattices' update items in turn, one wave
 * per item holding all of the item's populations, then its threads take the
 * projection entries.  Results are bit-identical to lb_step.  Lattices that
 * need a finish pass (periodic rows, pressure columns) or sets outside one
 * registered (D2Q36, D2Q16, D2Q9) order triple are refused with
 * LB_EUNSUPPORTED (the batch stays as it was).  Strip heights apply as for
 * the other launches (0 = 4 rows).  lb_batch_info reports 0 launches per
 * step in this mode. */
lb_status lb_batch_set_persistent(lb_batch *B, int32_t enable);

/* Steps per captured graph (0 = direct launches, the default).  Asynchronous
 * otherwise, like lb_step. */
lb_status lb_batch_set_graph(lb_batch *B, int32_t segment_steps);
lb_status lb_batch_step(lb_batch *B, int64_t steps);

/* Rows per work item of the low / high sets (0 = automatic), and the
 * autotuner that times candidates for `steps` steps each (twice, the faster
 * pass counting) and keeps the fastest (lattice states are restored). */
lb_status lb_batch_set_strip_rows(lb_batch *B, int32_t rows_low, int32_t rows_high);
lb_status lb_batch_autotune(lb_batch *B, int32_t steps, int32_t rows_out[2]);

/* Total nodes, kernel launches per step, velocity-set pairs present. */
lb_status lb_batch_info(const lb_batch *B, int64_t *nodes, int32_t *launches_per_step, int32_t *kinds);

#ifdef __cplusplus
}
#endif

#endif /* LB_H */
