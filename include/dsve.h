/*
 * dsve.h -- C ABI of libdsve.so: the A-DOT hot path for the 1-D de Saint
 * Venant-Exner system on one AMD Instinct MI355X (gfx950).
 *
 * Method (Carraro, Valiani, Caleffi, "Efficient analytical implementation of
 * the DOT Riemann solver for the de Saint Venant-Exner morphodynamic model"):
 *   state per cell W = (h, q, z): water depth, unit discharge, bed elevation
 *   (Sec. 2, Eq. W&A_definition); bed load q_s(h, q) from one of the closures of
 *   Sec. 2 (Eqs. Grass, GrassThr, MPM with Shields, vanRijn with u_star) or the
 *   power law of Sec. 5.1 (Eq. Soni_qs);
 *   DOT fluctuations D^{+-} = 1/2 sum_k w_k (A(Psi_k) +- |A(Psi_k)|)(W+ - W-)
 *   on the segment path with a G-point Gauss-Legendre rule (Sec. 3.1, Eqs. path,
 *   DOTjumpN), |A| = R |Lambda| R^-1 from the closed-form eigenstructure
 *   (Sec. 3.3, Eqs. lambda, parameters, RR, RR-1, ExAbsA); first-order update
 *   W_i <- W_i - dt/dx (D^-_{i+1/2} + D^+_{i-1/2}) + dt S(W_i) (Sec. 3, Eq. scheme)
 *   with S = (0, -g h s_f, 0), s_f = q|q| / (K_s^2 h^(10/3)) (Sec. 2) when a
 *   Strickler coefficient K_s is given, S = 0 otherwise (as in Sec. 4);
 *   dt = CFL dx / max_i max_m |lambda_m(W_i)|.
 *
 * Conventions shared by every entry point:
 *   - All state, fluctuation and time arrays are DEVICE pointers to float64
 *     (both precisions keep FP64 state in memory).  The caller owns them; the
 *     library never frees or reallocates them.
 *   - States are structure-of-arrays: h[i], q[i], z[i] for cell i.  Several
 *     channels are stored back to back; channel c owns cells [off[c], off[c+1]).
 *   - Edge e of a channel of N cells lies between cell e-1 and cell e, e = 0..N;
 *     cells -1 and N are the ghost cells given by the boundary conditions.
 *     Fluctuation arrays are [3][n] with component r of edge e at r*n + e.
 *   - Work is enqueued on the HIP stream given at init (NULL = the null stream)
 *     and returns without waiting.  Errors raised on the device (a non-finite
 *     CFL speed, complex eigenvalues) are deferred: dsve_sync() waits and
 *     reports them.  A failed call leaves its message in dsve_last_error().
 *     Errors are sticky per context until dsve_clear_error().
 *   - One context per stream; contexts share no state.  Calls that overlap on
 *     the same context from several host threads are not supported.
 *   - The library calls the HIP runtime it finds loaded (libamdhip64.so.7).  A
 *     caller whose streams and memory come from a HIP runtime of its own (one
 *     bundled with a framework) loads that runtime before this library, so that
 *     the process holds one runtime; with two, the caller's streams and pointers
 *     are unknown to the library's and init fails with DSVE_E_HIP.
 */
#ifndef DSVE_H
#define DSVE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DSVE_ABI_VERSION 5

typedef struct dsve_ctx dsve_ctx;

typedef enum {
    DSVE_OK = 0,
    DSVE_E_ARG = -1,            /* invalid argument (null pointer, size, parameter range) */
    DSVE_E_HIP = -2,            /* a HIP runtime call failed */
    DSVE_E_NONFINITE = -3,      /* a CFL speed was NaN/Inf or zero (e.g. h <= 0), or a non-finite
                                   arccos argument (an overflowed or NaN state) */
    DSVE_E_NONHYPERBOLIC = -4,  /* arccos argument outside [-1-1e-12, 1+1e-12] or k1 <= 0 (complex
                                   roots, Sec. 3.3), or exactly +-1 at a quadrature node: two
                                   eigenvalues coalesce to working precision and R^-1 (Eq. RR-1)
                                   does not exist (e.g. a fixed bed at Fr = +-1) */
    DSVE_E_UNSUPPORTED = -5     /* a valid request the library does not implement */
} dsve_status;

/* Boundary conditions: the ghost state W_{-1} (left) or W_N (right), from the adjacent cell
 * W_a = (h_a, q_a, z_a):
 *   TRANSMISSIVE  W_a
 *   PERIODIC      the cell at the other end (must be set on both sides)
 *   INFLOW_Q      (h_a, q_in, z_a): imposed discharge
 *   FIXED_DEPTH   (h_out, q_a, z_a): imposed depth, e.g. a downstream control (Sec. 5.1, 5.2)
 *   INFLOW_QH     (h_in, q_in, z_a): imposed discharge and depth; an imposed solid discharge
 *                 enters as the depth at which the closure gives it for q_in (Sec. 5.1)
 *   DIRICHLET     (h_d, q_d, z_d + t dz/dt) from dir_left / dir_right = {h_d, q_d, z_d, dz/dt},
 *                 t the channel's clock at the start of the step: a given ghost state whose bed
 *                 moves at a constant rate (the ghost cells of the analytical solution of
 *                 Sec. 4.2, Eq. berthon, whose bed falls linearly in time) */
enum { DSVE_BC_TRANSMISSIVE = 0, DSVE_BC_PERIODIC = 1, DSVE_BC_INFLOW_Q = 2,
       DSVE_BC_FIXED_DEPTH = 3, DSVE_BC_INFLOW_QH = 4, DSVE_BC_DIRICHLET = 5 };

/* Bed-load closures q_s(h, q), u = q/h, acting in the direction of the flow.  law_extra[]
 * holds the law's parameters; entries a law does not use must be zero.
 *   GRASS      q_s = A_g u^3                        (Sec. 2, Eq. Grass)     no parameters
 *   GRASS_THR  q_s = A_g sign(u) (|u| - u_cr)^3 for |u| > u_cr, else 0
 *                                                   (Sec. 2, Eq. GrassThr)  [0] = u_cr >= 0
 *   POWER      q_s = A_g sign(u) |u|^beta           (Sec. 5.1, Eq. Soni_qs) [0] = beta >= 1
 *   MPM        q_s = sign(q) 8 (theta - 0.047)^(3/2) sqrt(g (S_g-1) d50^3) for theta > 0.047,
 *              theta = s_f h / ((S_g-1) d50) with |s_f| (Sec. 2, Eqs. MPM, Shields)
 *                                                   [0] = d50 > 0, [1] = S_g > 1; needs ks > 0
 *   VANRIJN    q_s = sign(q) 0.053 T^2.1 / D_*^0.3 sqrt(g (S_g-1) d50^3) for T > 0,
 *              T = u_*^2 / u_*cr^2 - 1, u_*^2 = g h |s_f|, u_*cr^2 = theta_cr g (S_g-1) d50,
 *              D_* = d50 (g (S_g-1) / nu^2)^(1/3)    (Sec. 2, Eqs. vanRijn, u_star)
 *                                                   [0] = d50 > 0, [1] = S_g > 1, [2] = nu > 0,
 *                                                   [3] = theta_cr > 0; needs ks > 0
 * A_g is used by GRASS, GRASS_THR and POWER and must be zero for MPM and VANRIJN. */
enum { DSVE_LAW_GRASS = 0, DSVE_LAW_GRASS_THR = 1, DSVE_LAW_POWER = 2, DSVE_LAW_MPM = 3,
       DSVE_LAW_VANRIJN = 4 };
enum { DSVE_FP64 = 0, DSVE_MIXED = 1 };
/* Eigenstructure of the flux matrix at each quadrature node:
 *   ADOT  the closed form of Sec. 3.3 (the A-DOT scheme)
 *   DOT   a generic numerical eigen-decomposition, the original DOT solver of Sec. 3.1 (real
 *         Schur form by shifted QR, eigenvectors by back substitution, R^-1 by LU with partial
 *         pivoting, |A| = R |Lambda| R^-1): the baseline the closed form replaces; FP64 only */
enum { DSVE_SOLVER_ADOT = 0, DSVE_SOLVER_DOT = 1 };

/* Parameters of a context.
 *   g          gravitational acceleration (> 0)
 *   porosity   bed porosity p in [0, 1); xi = 1/(1-p)  (Sec. 2)
 *   law        DSVE_LAW_* (the closure of q_s)
 *   A_g        coefficient of the Grass-type laws (>= 0)
 *   law_extra  parameters of the law (see DSVE_LAW_*)
 *   n_gauss    quadrature points G in [1, 5] (Sec. 3.1 Eq. DOTjumpN); 3 is the default
 *   cfl        Courant number in (0, 1]
 *   dx         cell width (> 0)
 *   bc_left, bc_right   DSVE_BC_*
 *   q_in       unit discharge imposed by INFLOW_Q and INFLOW_QH
 *   h_in       depth imposed by INFLOW_QH (> 0 when used)
 *   h_out      depth imposed by FIXED_DEPTH (> 0 when used)
 *   dir_left, dir_right  DIRICHLET ghost {h > 0, q, z, dz/dt} of the left / right end
 *   ks         Strickler coefficient K_s of the friction slope (>= 0; 0 = no friction source;
 *              MPM and VANRIJN need ks > 0, their Shields stress and shear velocity use s_f)
 *   solver     DSVE_SOLVER_ADOT (default) or DSVE_SOLVER_DOT; DOT with DSVE_MIXED is
 *              DSVE_E_UNSUPPORTED
 *   precision  DSVE_FP64: all arithmetic in FP64.
 *              DSVE_MIXED: eigenstructure and quadrature in FP32; FP64 for the
 *              jumps W+ - W-, for the cubic's root solve and the eigenvector
 *              normalisation where the arccos argument is close to +-1
 *              (coalescing eigenvalues), and for the cell accumulation. */
typedef struct {
    double g;
    double porosity;
    int law;
    double A_g;
    double law_extra[4];
    int n_gauss;
    double cfl;
    double dx;
    int bc_left, bc_right;
    double q_in;
    int precision;
    double h_in;
    double h_out;
    double ks;
    double dir_left[4];
    double dir_right[4];
    int solver;
} dsve_params;

/* Per-channel parameters of a batched context (meaning and ranges as in dsve_params). */
typedef struct {
    double A_g;
    double porosity;
    double dx;
    double q_in;
    double h_in;
    double h_out;
    double ks;
    double law_extra[4];
    double dir_left[4];
    double dir_right[4];
    int bc_left, bc_right;
} dsve_channel;

/* Library ABI version (DSVE_ABI_VERSION). */
int dsve_abi_version(void);

/* Create a context for one channel of n_cells cells (n_cells >= 1).
 * Allocates device scratch: one ping-pong copy of the state (24 B per cell),
 * fluctuation scratch is not allocated.  hip_stream is a hipStream_t or NULL.
 * On error *out is NULL and the status says why (no context to query). */
dsve_status dsve_init(dsve_ctx **out, const dsve_params *p, int64_t n_cells, void *hip_stream);

/* Create a context for n_channels independent channels (n_channels >= 1).
 * HOST arrays:
 *   offsets[n_channels+1]  cell offsets, offsets[0] = 0, strictly increasing
 *   channels[n_channels]   per-channel parameters (each checked as in dsve_params)
 * g, law, n_gauss, cfl, precision and solver come from *common; its per-channel fields (A_g,
 * porosity, dx, bc_*, q_in, h_in, h_out, ks, law_extra, dir_*) are ignored.  All channels share the
 * closure law; its parameters may differ per channel.  Each channel gets its own time step
 * and clock (Sec. 3, Eq. scheme per channel).  The arrays are copied; the caller keeps them. */
dsve_status dsve_batch_init(dsve_ctx **out, int64_t n_channels, const int64_t *offsets,
                            const dsve_channel *channels, const dsve_params *common,
                            void *hip_stream);

/* Release the context and its device scratch (waits for its queued work). */
dsve_status dsve_destroy(dsve_ctx *ctx);

/* Pairwise DOT fluctuations of n independent edges (Sec. 3.1, Eq. DOTjumpN with
 * the segment path Eq. path; |A| from Sec. 3.3).  Left states (hL, qL, zL) and
 * right states (hR, qR, zR) are device arrays of n doubles; Dm and Dp receive
 * D^- and D^+ as [3][n] device arrays.  Uses the context's g, porosity, A_g,
 * n_gauss and precision (for a batched context: those of channel 0). */
dsve_status dot_edge_fluct(dsve_ctx *ctx, const double *hL, const double *qL, const double *zL,
                           const double *hR, const double *qR, const double *zR, int64_t n,
                           double *Dm, double *Dp);

/* Cell update of one channel (Sec. 3, Eq. scheme): for i = 0..N-1,
 *   W_i <- W_i - (dt/dx) (Dm[:, i+1] + Dp[:, i]) + dt S(W_i)
 * with Dm, Dp the [3][N+1] edge fluctuations (edge i is the left face of cell i),
 * dt_dev a device pointer to the time step, S the friction source of the context (zero
 * when ks = 0), and h, q, z updated in place.  The six arrays and dt_dev must not
 * overlap one another.  Single-channel contexts only. */
dsve_status cell_update(dsve_ctx *ctx, const double *Dm, const double *Dp, const double *dt_dev,
                        double *h, double *q, double *z);

/* CFL reduction of one channel: *amax_dev = max_i max_m |lambda_m(W_i)| over the
 * N real cells (eigenvalues of Sec. 3.3, Eq. lambda) and *dt_dev = cfl*dx/amax.
 * amax_dev and dt_dev are device pointers to one double each.  The maximum is
 * exact (order independent); a NaN speed wins it and is reported by dsve_sync.
 * Single-channel contexts only. */
dsve_status cfl_reduce(dsve_ctx *ctx, const double *h, const double *q, const double *z,
                       double *amax_dev, double *dt_dev);

/* Advance one channel by n_steps >= 0 time steps in place: per step, ghost
 * cells from the boundary conditions, dt = cfl*dx/amax(W^n), DOT fluctuations
 * at every edge, cell update with the friction source, and the CFL speed of W^{n+1} --
 * one fused kernel per step, or one launch for the whole run when the run is
 * channel-resident (dsve_set_resident).  With graph_steps > 0 (dsve_set_launch) the steps
 * are replayed from captured HIP graphs: n_steps / graph_steps replays of a graph of
 * graph_steps steps, then one replay of a graph of the remaining n_steps % graph_steps
 * steps; the graphs are captured at the first run that needs them and kept while the
 * arrays and the launch configuration stay the same (dsve_prepare_run captures them ahead).  *t_dev (device) is
 * increased by the sum of the time steps.  The result is in (h, q, z) when the
 * enqueued work completes, bitwise independent of the launch configuration. */
dsve_status adot_step(dsve_ctx *ctx, double *h, double *q, double *z, int n_steps, double *t_dev);

/* As adot_step for a batched context: h, q, z hold all channels back to back
 * (offsets as given to dsve_batch_init); t_dev[n_channels] receives each
 * channel's clock.  All channels run in one persistent kernel per step, or in one
 * launch for the whole run when it is channel-resident. */
dsve_status adot_step_batched(dsve_ctx *ctx, double *h, double *q, double *z, int n_steps,
                              double *t_dev);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): adot_step / adot_step_batched for a context created
 * beforehand, with the same results bit for bit, that allocates nothing -- no hipMalloc or
 * hipFree, no graph instantiation (every step is a direct launch; the caller may capture them).
 * The ping-pong copy of the state and clocks and the CFL slots live in a static device array
 * of the library (about 24.4 MiB, held by each device the library runs on until the process
 * ends) instead of the context's buffers, so the context may have at most 1048576 cells in at
 * most 4096 channels; larger contexts get DSVE_E_ARG and keep using adot_step.  All calls on one
 * device share that array: calls that overlap on one device (several streams or host threads)
 * race and are not supported.  Errors are deferred to dsve_sync as for adot_step. */
dsve_status adot_step_noalloc(dsve_ctx *ctx, double *h, double *q, double *z, int n_steps,
                              double *t_dev);

/* Capture ahead the HIP graphs a run of n_steps on these arrays will replay (see adot_step),
 * so that the run itself only replays them: graph capture and instantiation then fall
 * outside a timed or latency-critical region.  Enqueues no work; the arrays are not read.
 * Nothing to do for channel-resident runs or with graph_steps = 0. */
dsve_status dsve_prepare_run(dsve_ctx *ctx, double *h, double *q, double *z, int n_steps,
                             double *t_dev);

/* How the last run (adot_step, adot_step_batched) was launched: *graph_launches HIP graph
 * replays covering *graph_steps steps, and *direct_launches kernels launched one by one (step
 * kernels, or 1 for a channel-resident run).  Any pointer may be NULL. */
dsve_status dsve_get_last_run(const dsve_ctx *ctx, int *graph_launches, int *graph_steps,
                              int *direct_launches);

/* Wait for the context's queued work; report a deferred device error
 * (DSVE_E_NONFINITE, DSVE_E_NONHYPERBOLIC) raised since the last sync. */
dsve_status dsve_sync(dsve_ctx *ctx);

/* Message of the last error on this context ("" if none).  Valid until the
 * next call on the context. */
const char *dsve_last_error(const dsve_ctx *ctx);

/* Clear the sticky error state. */
dsve_status dsve_clear_error(dsve_ctx *ctx);

/* Launch configuration of the fused step kernel.
 *   tile           threads (= edges) per workgroup: 64, 128, 192 or 256
 *   blocks_per_cu  persistent workgroups per compute unit (1..1024); 0 = as many
 *                  as fit on a compute unit at once (occupancy of the kernel); more than
 *                  fit oversubscribes the grid (workgroups start as others finish).  The
 *                  grid is capped at one workgroup per tile, and each workgroup takes an
 *                  even contiguous run of the tiles
 *   graph_steps    steps per captured HIP graph: a multiple of 6 in [6, 600],
 *                  or 0 to launch every step directly
 * The results do not depend on these (each edge and cell is computed the same
 * way whatever tile it falls in). */
dsve_status dsve_set_launch(dsve_ctx *ctx, int tile, int blocks_per_cu, int graph_steps);
dsve_status dsve_get_launch(const dsve_ctx *ctx, int *tile, int *blocks_per_cu, int *graph_steps);

/* CFL sub-slots of the fused step kernel: each workgroup merges its partial
 * CFL maximum with an atomic into one of `split` sub-slots per channel (1, 2 or
 * 4; 0, the default, picks 4 when many workgroups share a channel and each
 * merges after a few tiles, else 1), and a workgroup reads the maximum over them
 * when its run of tiles enters a channel.
 * More sub-slots spread the atomics of a step over more addresses; fewer keep
 * the read to fewer loads.  The results do not depend on it.  The getter reports
 * the count in effect for the current launch configuration. */
dsve_status dsve_set_cfl_split(dsve_ctx *ctx, int split);
dsve_status dsve_get_cfl_split(const dsve_ctx *ctx, int *split);

/* Channel-resident runs (Sec. 3, Eq. scheme, run step after step on chip): when every
 * channel of the context has at most 511 cells, adot_step / adot_step_batched by default
 * run all n steps in one launch, one workgroup per channel at a time (256 threads, or 512
 * when a channel has more than 255 cells), with the state on chip and each channel's CFL
 * maximum reduced within its workgroup.  The results are
 * bitwise those of the per-step kernels; the per-step launch latency, which bounds such
 * small problems, is paid once.  mode 0: automatic (resident when eligible); 1: always
 * per-step kernels.  The launch configuration and CFL sub-slots do not apply to resident
 * runs.  dsve_get_resident reports whether the next run will be resident.  Resident runs
 * leave lanes idle in channels much shorter than their workgroup; dsve_autotune compares
 * them with the per-step kernels. */
dsve_status dsve_set_resident(dsve_ctx *ctx, int mode);
dsve_status dsve_get_resident(const dsve_ctx *ctx, int *active);

/* Autotuner: time candidate (tile, blocks_per_cu) pairs for `trial_steps`
 * fused steps each (rounded up to whole replays of a 12-step graph, after one warm-up
 * replay that captures it, when the context uses graphs) on a scratch copy of (h, q, z),
 * over tiles of 64..256 threads and 0..128 workgroups per compute unit, then the three
 * fastest with 1 and with 4 CFL sub-slots -- the caller's arrays are read, never written
 * -- and keep the fastest in the context.  If cache_path is not NULL, a JSON cache keyed
 * by device, precision, law, kernel closure and problem shape is read first (a hit sets the
 * launch and returns at once) and updated after tuning.
 * When the context can run channel-resident (and that is not turned off), a resident run
 * is timed too: it stays on if it is the fastest, else it is turned off (mode 1) for the
 * context.  Waits for completion.  Before the trials it waits for the work already
 * enqueued and returns that work's deferred error, as dsve_sync would; the trials' own
 * device error flags and CFL maxima are discarded, so a later dsve_sync reports only runs
 * made after tuning.  If a trial fails, the error is sticky and the context keeps the
 * launch it had before the call. */
dsve_status dsve_autotune(dsve_ctx *ctx, const double *h, const double *q, const double *z,
                          int trial_steps, const char *cache_path);

/* Number of compute units of the context's device. */
int dsve_device_cus(const dsve_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* DSVE_H */
