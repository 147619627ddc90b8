/*
 * empso.h - C ABI of the MI355X (gfx950) fitness-evaluation library.
 *
 * The library computes the fitness of velocity-model candidates for the
 * elitist-mutated particle swarm search of Mojica and Kukreja (arXiv
 * 1905.12795). The problem it solves is the one the paper states in its
 * Testing approach section: minimise, over control-node velocities x inside a
 * search box,
 *
 *     phi(x) = 1/2 sum_s || R u_s(B x) - d_s^obs ||^2
 *
 * where B is the bilinear two-grid map from control nodes to the FD grid,
 * u_s is the 2-D constant-density acoustic wavefield of shot s (finite
 * differences, second order in time, eighth order in space, damping absorbing
 * layer, Ricker source), R samples it at the receivers at every time step,
 * and the l2 misfit is summed over shots (Results section: a particle's
 * fitness needs all of its shots).
 *
 * Conventions (identical in every entry point):
 *   - Grid point (i, j) of the physical grid is at z = i*dz, x = j*dx; z points
 *     down; the origin is the top-left corner. The padded grid adds nbl points
 *     of absorbing layer on every side; beyond it the field is zero.
 *   - Scheme, with m = 1/v^2, damping d and a = d*dt/2:
 *       u^{n+1} = u^n + delta,
 *       delta = [ (1-a) (u^n - u^{n-1}) + (v dt)^2 (Lap_h u^n + f^n) ] / (1+a),
 *     which is the centred scheme u^{n+1} = [2u^n - (1-a)u^{n-1} + (v dt)^2
 *     (Lap_h u^n + f^n)]/(1+a) evaluated in increment form for FP32 accuracy
 *     (the increment u^n - u^{n-1} is formed before anything is added to it).
 *     Lap_h uses the eighth-order central weights (-205/72, 8/5, -1/5, 8/315,
 *     -1/560). u^0 = u^{-1} = 0.
 *   - Damping: d = d0 (l/nbl)^2 per axis, d0 = 3 vmax ln(1/R)/(2 nbl h), with l
 *     the depth into the layer in points; the z and x parts add.
 *   - Source: f^n = w(n dt)/(dz dx) at the source point, entering the step
 *     n -> n+1; w is a Ricker wavelet of peak frequency f0 delayed by 1/f0.
 *   - Traces: d[n][r] = u^n at receiver r, n = 0 .. nt-1 (every time step).
 *   - Misfit: 1/2 sum of squared residuals over time samples and receivers.
 *   - Sources and receivers must lie on grid points; all receivers of a
 *     problem share one grid row and occupy distinct columns (ENOTSUP
 *     otherwise).
 *
 * Memory: every device array (fields, traces, observed data, fitness,
 * workspace) is owned by the caller. Problem handles are owned by the library
 * and hold small device tables (wavelet, damping, receiver maps); they are
 * immutable after creation and may be shared between streams.
 *
 * Streams: entry points that take an empso_stream enqueue work on that HIP
 * stream (a hipStream_t; NULL means the default stream) and return; results
 * are valid once the stream has reached that point. Calls that overlap on
 * different streams must use different workspaces.
 *
 * Errors: every entry point returns EMPSO_OK (0) or a negative status. All
 * validation happens before anything is enqueued: on error nothing has been
 * enqueued and output arrays are untouched. empso_last_error() returns a
 * thread-local message describing the last failure.
 */
#ifndef EMPSO_H
#define EMPSO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EMPSO_OK          0
#define EMPSO_EINVAL     (-1)  /* null pointer, non-positive size, bad geometry          */
#define EMPSO_ECFL       (-2)  /* dt above the leapfrog stability limit at vmax          */
#define EMPSO_ERANGE     (-3)  /* a velocity outside [vmin, vmax] or not finite          */
#define EMPSO_EWORKSPACE (-4)  /* workspace too small                                     */
#define EMPSO_EHIP       (-5)  /* a HIP runtime call failed (see empso_last_error)        */
#define EMPSO_ENOTSUP    (-6)  /* valid request outside what this library implements      */

typedef void *empso_stream;                 /* hipStream_t */
typedef struct empso_problem empso_problem; /* opaque, immutable after creation */

/* One modelling problem: grid, time axis, acquisition, control-node grid.
 * All values on the host, SI units (m, s, m/s, Hz). Arrays are read during
 * empso_problem_create only. */
typedef struct {
    int32_t nz, nx;          /* physical grid points (z slow, x fast)                  */
    double dz, dx;           /* grid spacing                                            */
    int32_t nbl;             /* absorbing-layer points on every side (paper: nbpml)     */
    double dt;               /* time step; must satisfy dt <= stable limit at vmax      */
    int32_t nt;              /* time samples, t = 0 included                            */
    double f0;               /* Ricker peak frequency                                   */
    int32_t nshots;          /* number of shots                                         */
    const double *src_zx;    /* [nshots][2] source (z, x) positions                     */
    int32_t nrec;            /* receivers per shot (same spread for every shot)         */
    const double *rec_zx;    /* [nrec][2] receiver (z, x) positions                     */
    int32_t ncz, ncx;        /* regular control-node grid, corners included, >= 2 each  */
                             /* (layered grid: ncz = number of levels, ncx ignored)     */
    double vmin, vmax;       /* hard velocity bounds; dt is checked against vmax        */
    double damp_R;           /* target reflection coefficient of the layer (e.g. 1e-3)  */
    /* Optional layered node grid, the reading of the paper's irregular grid
     * (Testing approach section: nodes built from a 1-D prior with a water
     * layer on top). node_z == NULL selects the regular ncz x ncx grid.
     * Otherwise there are ncz >= 2 depth levels at depths node_z[ncz]
     * (metres, strictly increasing); level a holds level_nodes[a] >= 2 nodes
     * at x positions node_x (metres, strictly increasing within a level,
     * levels concatenated in order); the node vector of a particle lists the
     * nodes in the same order, D = sum(level_nodes). Interpolation: linear
     * along each level in x (constant beyond its first and last node), then
     * linear in z between the two levels around the point (constant above
     * the first and below the last level). A regular grid is the layered
     * grid whose levels all hold the same ncx evenly spaced nodes.         */
    const double *node_z;
    const int32_t *level_nodes;
    const double *node_x;
    int32_t water_rows;      /* physical rows 0 .. water_rows-1 hold v_water (either grid) */
    double v_water;          /* within [vmin, vmax] when water_rows > 0                  */
    /* Misfit of empso_fitness_batch, empso_gradient and empso_traces_misfit
     * (EMPSO_MISFIT_*). The paper scores fitness with the l2 misfit (Testing
     * approach section). The optional trace-normalised variant divides every
     * trace (one receiver of one shot, over the nt samples) of the modelled
     * and of the observed data by max(its l2 norm, w) before the l2 misfit,
     * w = EMPSO_TRACE_FLOOR times the largest trace norm of the same shot on
     * the same side (modelled or observed; a trace divided by zero stays
     * zero). This removes amplitude mismatches between modelled and
     * recorded sources: each side is invariant under a scale of all its
     * traces. The floor keeps traces that no arrival reaches (the scheme's
     * numerical precursor, orders of magnitude below any arrival) from being
     * raised to full weight. Per trace above both floors:
     * 1/2 |d/|d| - o/|o||^2 = 1 - d.o / (|d| |o|). */
    int32_t misfit;
} empso_geometry;

#define EMPSO_MISFIT_L2 0
#define EMPSO_MISFIT_TRACE_NORMALISED 1
#define EMPSO_TRACE_FLOOR 1e-4

/* Read-only facts about a problem (for sizing caller-owned arrays). */
typedef struct {
    int32_t nz, nx, nbl, nt, nshots, nrec, ncz, ncx;
    int32_t Nz, Nx;          /* padded grid: nz + 2 nbl, nx + 2 nbl                    */
    int32_t row_stride;      /* floats per stored row of an internal field              */
    int64_t updates_per_run; /* Nz * Nx * (nt - 1): point updates of one shot           */
    int32_t D;               /* node values per particle (ncz * ncx, or sum(level_nodes)) */
} empso_problem_info;

/* Tuning of the finite-difference kernels. Every valid tuning gives
 * bit-identical results; only the speed changes. */
typedef struct {
    int32_t variant;         /* reserved, 0                                             */
    int32_t bz;              /* target output rows per tile, a multiple of 20 in 20..1280;
                              * each grid's rows are split into equal strips of about
                              * this height, rounded up so that a strip's march (its
                              * 8 (tsteps - 1) queue-fill steps plus its rows) is a
                              * whole number of 10-step blocks; the last strip takes
                              * the rest                                                */
    int32_t tsteps;          /* time steps per launch (temporal-blocking depth): 1..4   */
    int32_t prefetch;        /* rows of u requested ahead of use: 1                     */
    int32_t use_graph;       /* 1: replay the time loop from a captured HIP graph       */
} empso_tuning;

/* Status name ("EMPSO_OK", ...). Never NULL. */
const char *empso_status_string(int status);

/* Thread-local description of the last error on this thread. Never NULL. */
const char *empso_last_error(void);

/* Largest stable time step of the scheme at velocity vmax (von Neumann limit
 * of the leapfrog with the eighth-order stencil):
 *   dt_stab = 2 / (vmax sqrt((2048/315) (1/dz^2 + 1/dx^2))).
 * Testing approach section: second order in time, eighth order in space. */
int empso_stable_dt(double vmax, double dz, double dx, double *dt_out);

/* Create a problem (Testing approach section: the grid, time axis, source,
 * receivers and control-node layout of the paper's modelling setup).
 * Validates the geometry (EINVAL, ECFL, ENOTSUP), builds the wavelet, damping
 * and receiver tables and uploads them to the current device. *out receives
 * the handle (NULL on error). ENOTSUP for a grid whose stored field (padded
 * grid plus a 16-point zero ring, rows rounded up to 64 floats) exceeds 2^27
 * floats (512 MiB): the kernels address a run's four fields with 32-bit
 * byte offsets. */
int empso_problem_create(const empso_geometry *geom, empso_problem **out);

/* Destroy a problem created by empso_problem_create (NULL is ignored). The
 * caller must make sure no enqueued work still uses it. */
void empso_problem_destroy(empso_problem *prob);

int empso_problem_get_info(const empso_problem *prob, empso_problem_info *info);

/* Two-grid interpolation (Testing approach section): control-node velocities
 * nodes_d[nmodels][D] (device, FP32) become vp_d[nmodels][nz][nx] (device,
 * FP32). Regular grid: nodes row-major z-major, node (a, b) at grid point
 * (a (nz-1)/(ncz-1), b (nx-1)/(ncx-1)), bilinear in each cell. Layered grid:
 * as described with empso_geometry. Rows above water_rows hold v_water. */
int empso_vp_from_nodes(const empso_problem *prob, int32_t nmodels, const float *nodes_d,
                        float *vp_d, empso_stream stream);

/* Workspace bytes for empso_forward_shots with nsh shots (0 for nsh = 0 and
 * on invalid arguments). */
size_t empso_forward_workspace_bytes(const empso_problem *prob, int32_t nsh);

/* Forward modelling of shots (Testing approach section: each shot is
 * modelled with the finite-difference scheme above and recorded at every
 * receiver at every time step; these are the traces the misfit compares).
 * Model shots shot0 .. shot0+nsh-1 in the physical-grid model vp_d[nz][nx]
 * (device, FP32; copied once to the host for the range check, so this call
 * waits for the stream) and write traces_d[nsh][nt][nrec] (device, FP32).
 * The model is extended into the absorbing layer by nearest-value copy.
 * ERANGE if a velocity lies outside [vmin, vmax]. tuning may be NULL: on the
 * first such call for a problem and shot count the library times the
 * candidate tunings (as empso_autotune_fitness does, on this call's workspace
 * and model) and keeps the fastest until the problem is destroyed. The graph
 * flag is ignored. The traces do not depend on the tuning.
 * nsh = 0 (with 0 <= shot0 <= nshots) is an empty range: EMPSO_OK, nothing is
 * enqueued and the pointer arguments are not used. EINVAL for nsh < 0 or a
 * range outside the problem's shots. */
int empso_forward_shots(const empso_problem *prob, const float *vp_d, int32_t shot0, int32_t nsh,
                        float *traces_d, void *ws, size_t ws_bytes, const empso_tuning *tuning,
                        empso_stream stream);

/* Workspace bytes for empso_misfit over n elements. */
size_t empso_misfit_workspace_bytes(int64_t n);

/* The paper's l2 misfit between two trace arrays (Testing approach section:
 * a model is scored by the l2 norm of its traces' difference from the
 * observed ones; here squared and halved):
 * out_d[0] = 1/2 sum_k (a_d[k] - b_d[k])^2 over n elements (device, FP32
 * inputs, FP64 accumulation in a fixed order, FP32 result). Deterministic.
 * n = 0 gives 0. EINVAL for NULL pointers or n < 0; EWORKSPACE if ws_bytes
 * is below empso_misfit_workspace_bytes(n). */
int empso_misfit(const float *a_d, const float *b_d, int64_t n, float *out_d,
                 void *ws, size_t ws_bytes, empso_stream stream);

/* Workspace bytes for empso_traces_misfit over nsh shots (0 on invalid arguments). */
size_t empso_traces_misfit_workspace_bytes(const empso_problem *prob, int32_t nsh);

/* The problem's misfit (l2 or trace-normalised, empso_geometry.misfit)
 * between modelled traces traces_d and observed traces obs_d, both device
 * FP32 [nsh][nt][nrec] (Testing approach section: the misfit that scores a
 * model), summed over the nsh shots: out_d[0] (device FP32). This is the
 * misfit empso_fitness_batch and empso_gradient compute inside their time
 * loops, for traces already recorded (a line search over physical models).
 * Per trace, FP64 sums over time in order, then a fixed-order sum over
 * traces: deterministic. +inf if a modelled trace is not finite.
 * nsh = 0 gives 0. EINVAL for NULL arguments or nsh < 0; EWORKSPACE if
 * ws_bytes is too small. */
int empso_traces_misfit(const empso_problem *prob, const float *traces_d, const float *obs_d, int32_t nsh,
                        float *out_d, void *ws, size_t ws_bytes, empso_stream stream);

/* empso_traces_misfit without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation). Its scratch (4 nsh nrec doubles) is a
 * fixed array of the library on each GPU, held until the process ends, so
 * the call allocates nothing; the result is bit-identical to
 * empso_traces_misfit's. Limit: nsh * nrec <= EMPSO_NOALLOC_MAX_TRACES
 * (ENOTSUP beyond it). Every call on a GPU uses that GPU's one scratch
 * array: calls that overlap on one GPU (different streams, or host threads
 * without ordering) race and give wrong results; calls ordered on one stream
 * are safe. Nothing in the scratch needs clearing between calls. */
#define EMPSO_NOALLOC_MAX_TRACES 262144
int empso_traces_misfit_noalloc(const empso_problem *prob, const float *traces_d, const float *obs_d, int32_t nsh,
                                float *out_d, empso_stream stream);

/* Workspace bytes for empso_fitness_batch over np particles; particle p uses
 * problem probs[prob_of_particle[p]] (host array). 0 for an empty batch
 * (np = 0) and on invalid arguments. */
size_t empso_fitness_workspace_bytes(const empso_problem *const *probs, int32_t nprob,
                                     const int32_t *prob_of_particle, int32_t np);

/* Fitness of np particles (Results section: a particle's fitness is the sum
 * over all shots of its problem of the l2 misfit, or of the trace-normalised
 * misfit when the problem selects it). All shots of all particles
 * advance together, one launch per time step or per block of time steps.
 *   probs[nprob]              problems (grids may differ; all must share nt; a batch
 *                             whose grids all have dz = dx uses the isotropic grouping
 *                             of the Laplacian, any other batch the general one, so
 *                             a grid's fitness is bit-identical across batches of
 *                             the same kind and equal to rounding otherwise)
 *   obs_d[nprob]              per problem, device FP32 [nshots][nt][nrec]
 *   prob_of_particle[np]      host, problem index of each particle
 *   nodes_h[np][ld_nodes]     host FP64 control-node velocities (ld_nodes >=
 *                             the largest ncz*ncx); range-checked on the host:
 *                             ERANGE if outside [vmin, vmax] or not finite
 *   fitness_d[np]             device FP32 output; +inf if the wavefield of
 *                             some shot became non-finite
 * tuning may be NULL (library default). np = 0 is an empty batch: EMPSO_OK,
 * nothing is enqueued and the other arguments are not used; np < 0 is
 * EINVAL. */
int empso_fitness_batch(const empso_problem *const *probs, int32_t nprob,
                        const float *const *obs_d, const int32_t *prob_of_particle, int32_t np,
                        const double *nodes_h, int32_t ld_nodes, float *fitness_d,
                        void *ws, size_t ws_bytes, const empso_tuning *tuning,
                        empso_stream stream);

/* The same evaluation as empso_fitness_batch, run in blocks of time steps:
 * one call performs the transitions n -> n+1 for n_begin <= n < n_end of
 * every run of the batch, so that a caller can bound the duration of a call
 * or interleave other work with a long evaluation. The state between calls
 * lives in the workspace.
 *   n_begin = 0       starts an evaluation: the particles' nodes_h (host
 *                     FP64, range-checked as in empso_fitness_batch) are
 *                     uploaded, the wavefields cleared and the coefficient
 *                     fields built;
 *   n_begin > 0       continues the evaluation that the previous call on this
 *                     batch, workspace and tuning left at step n_begin
 *                     (EINVAL otherwise); nodes_h is not read and may be NULL;
 *   n_end = nt - 1    finishes it: the last time sample is taken and
 *                     fitness_d[np] written. Before that call fitness_d is
 *                     not touched.
 * 0 <= n_begin <= n_end <= nt - 1; n_begin must be 0 or a multiple of
 * tuning->tsteps and n_end nt - 1 or a multiple of tuning->tsteps (EINVAL).
 * The launch sequence is the one empso_fitness_batch replays, so the fitness
 * values are bit-identical to it for the same tuning. Calls run without
 * graph replay (use_graph is ignored). np = 0 is an empty batch (EMPSO_OK,
 * nothing enqueued). */
int empso_fitness_batch_steps(const empso_problem *const *probs, int32_t nprob,
                              const float *const *obs_d, const int32_t *prob_of_particle, int32_t np,
                              const double *nodes_h, int32_t ld_nodes, float *fitness_d,
                              int32_t n_begin, int32_t n_end,
                              void *ws, size_t ws_bytes, const empso_tuning *tuning,
                              empso_stream stream);

/* Default tuning used when NULL is passed. */
int empso_default_tuning(empso_tuning *out);

/* Autotuner: with the same arguments as empso_fitness_batch, time a few
 * launches of the finite-difference kernel for every tile height of 20, 40,
 * 80, 160, 240, 320, 480, 720 and 1040 rows and temporal-blocking depth on
 * this batch (a
 * height that gives every grid the same strips as a lower one launches the
 * same tiles and is skipped), then time the three fastest again over about
 * one second of launches each (after as many untimed ones: short bursts
 * rank tilings that differ by a percent or two differently from a sustained
 * run), and write the fastest of those to *best (graph replay on) and its
 * time per time step in microseconds to *best_us_per_step (may be NULL).
 * Takes a few seconds on large batches. Every tuning gives bit-identical
 * results. Synchronises the stream; overwrites the workspace. */
int empso_autotune_fitness(const empso_problem *const *probs, int32_t nprob, const float *const *obs_d,
                           const int32_t *prob_of_particle, int32_t np, const double *nodes_h, int32_t ld_nodes,
                           void *ws, size_t ws_bytes, empso_tuning *best, float *best_us_per_step,
                           empso_stream stream);

/* Time one tuning the way the autotuner does: set the batch up, run one
 * untimed and `reps` timed launches of the finite-difference kernel from time
 * 0, and write the time per time step in microseconds. Used for tuning and
 * for hardware-counter collection on a few launches. Synchronises the
 * stream; overwrites the workspace. */
int empso_time_tuning(const empso_problem *const *probs, int32_t nprob, const float *const *obs_d,
                      const int32_t *prob_of_particle, int32_t np, const double *nodes_h, int32_t ld_nodes,
                      void *ws, size_t ws_bytes, const empso_tuning *tuning, int32_t reps, float *us_per_step,
                      empso_stream stream);

/* ------------------------------------------------------------------------
 * Misfit gradient for the local FWI that starts from the global search's best
 * model (Testing approach section: the best EMPSO model is the starting point
 * of a local full-waveform inversion of the same data with the same l2 misfit).
 *
 * The exact gradient of the discrete misfit J = 1/2 sum_s sum_n sum_r
 * (u_s^n(x_r) - d_s^n_r)^2 with respect to the physical model, by the discrete
 * adjoint: dividing the update by C = (v dt)^2 makes its operator symmetric,
 * so the adjoint runs the same damped scheme backwards in time with the
 * residuals injected at the receivers, and
 *   dJ/dC = sum_n psi^{n+1} [(1+a) u^{n+1} - 2 u^n + (1-a) u^{n-1}] / C^2,
 *   dJ/dv = 2 v dt^2 dJ/dC, folded onto the physical grid (an absorbing-layer
 * point adds into the edge point it copies) and summed over all shots.
 * Checkpointing: (u^n, u^{n-1}) are kept every K = checkpoint_every steps
 * (0: K = ceil(sqrt(2 (nt - 1)))), and each segment is recomputed during the
 * backward pass: about two forward passes and one adjoint pass of work, and
 * 2 (K + 2) + 6 + 2 ceil((nt - 1)/K) fields per shot of memory (two segment
 * buffers: the next segment is recomputed on a second stream of the library's
 * while the adjoint runs through the current one; the call's work still ends
 * on the caller's stream). Both forward passes run the fitness kernel (the
 * recomputation in a mode that keeps every time level). K >= nt - 1 keeps
 * every time level of one forward pass instead (one forward and one adjoint
 * pass; nt + 9 fields per shot, e.g. 234 GB for 16 shots of 381 x 1001 points
 * over 8114 steps). The adjoint advances up to three time steps per launch.
 * The same pass can return the source illumination
 * sum_s sum_{n>=1} u_s^n(x)^2, summed from the recomputed levels of each
 * segment and folded the same way, the usual diagonal scaling
 * (pseudo-Hessian) of the gradient; asking for it changes neither the
 * gradient nor the misfit (bit for bit).
 * ------------------------------------------------------------------------ */

/* Workspace bytes for empso_gradient (0 on invalid arguments). */
size_t empso_gradient_workspace_bytes(const empso_problem *prob, int32_t checkpoint_every);

/* Misfit and gradient of the physical model vp_d[nz][nx] (device FP32; copied
 * once to the host for the range check, so this call waits for the stream)
 * against obs_d[nshots][nt][nrec] (device FP32) over all shots:
 * grad_d[nz][nx] (device FP32) = dJ/dvp, misfit_d[0] (device FP32) = J,
 * illum_d[nz][nx] (device FP32, may be NULL) = the source illumination.
 * ERANGE if a velocity lies outside [vmin, vmax]; EINVAL for NULL arguments,
 * nt < 2 or a negative interval; EWORKSPACE if ws_bytes is too small; ENOTSUP
 * for a grid whose stored field (padded grid plus a 16-point ring, rows
 * rounded to 64 floats) takes 2^31 / 6 bytes or more. Calls on one device
 * share the library's second stream there. */
int empso_gradient(const empso_problem *prob, const float *vp_d, const float *obs_d, float *grad_d,
                   float *misfit_d, float *illum_d, int32_t checkpoint_every, void *ws, size_t ws_bytes,
                   empso_stream stream);

/* ------------------------------------------------------------------------
 * Surrogate network (not part of the paper): maps control-node velocities to
 * a standardised log-misfit so that candidates can be ranked before the
 * finite-difference fitness. x_hat = (x - lo)/(hi - lo); three hidden layers
 * h = GELU(W h + b) of width H (exact erf GELU); y = w4 . h3 + b4.
 * BF16 operands on MFMA with FP32 accumulation; FP32 master parameters and
 * Adam moments. All buffers are caller-owned device memory.
 * Shapes: 1 <= D, H <= 4096 and 1 <= n <= 2^22 rows; outside these bounds
 * the workspace size is 0 and every call returns EMPSO_EINVAL before it
 * touches any buffer.
 *
 * FP32 parameter layout (empso_mlp_param_count floats):
 *   W1 [H][D] | b1 [H] | W2 [H][H] | b2 [H] | W3 [H][H] | b3 [H] | w4 [H] | b4 [1]
 * BF16 weight copy (empso_mlp_bf16_count values, uint16 bit patterns):
 *   W1 [H][D] | W2 [H][H] | W3 [H][H]
 * Training target of a row with fitness f: (log(max(f, 1e-30)) - mu)/sigma;
 * loss = mean over the rows of (y - target)^2.
 * ---------------------------------------------------------------------- */
size_t empso_mlp_param_count(int32_t D, int32_t H);
size_t empso_mlp_bf16_count(int32_t D, int32_t H);
/* Workspace bytes for a pass over n rows. */
size_t empso_mlp_workspace_bytes(int32_t D, int32_t H, int32_t n);

/* Refresh the BF16 weight copy from the FP32 parameters. */
int empso_mlp_sync_bf16(int32_t D, int32_t H, const float *params_d, uint16_t *wbf16_d, empso_stream stream);

/* y_d[n] = network(X_d[n][D]); lo_d, hi_d: [D] input box. */
int empso_mlp_predict(int32_t D, int32_t H, const float *params_d, const uint16_t *wbf16_d, const float *lo_d,
                      const float *hi_d, const float *X_d, int32_t n, float *y_d, void *ws, size_t ws_bytes,
                      empso_stream stream);

/* Loss and its gradient (FP32, parameter layout) over n rows; row m is
 * X_d[idx_d[m]] with fitness fit_d[idx_d[m]] (idx_d may be NULL: row m).
 * grads_d [param_count] and loss_d [1] may be NULL. */
int empso_mlp_grad(int32_t D, int32_t H, const float *params_d, const uint16_t *wbf16_d, const float *lo_d,
                   const float *hi_d, const float *X_d, const float *fit_d, const int32_t *idx_d, int32_t n,
                   float mu, float sigma, float *grads_d, float *loss_d, void *ws, size_t ws_bytes,
                   empso_stream stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with the
 * 1-based step count) on the gradient of empso_mlp_grad, then refresh the
 * BF16 copy. loss_d [1] receives the loss before the step (may be NULL). */
int empso_mlp_train_step(int32_t D, int32_t H, float *params_d, uint16_t *wbf16_d, float *adam_m_d, float *adam_v_d,
                         int32_t step, float lr, const float *lo_d, const float *hi_d, const float *X_d,
                         const float *fit_d, const int32_t *idx_d, int32_t n, float mu, float sigma, float *loss_d,
                         void *ws, size_t ws_bytes, empso_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* EMPSO_H */
