/*
 * mm.h -- C ABI of the MI355X (gfx950) FFT-demagnetisation + LLG library.
 *
 * The library computes, for magnetisation M on an nx x ny x nz grid of equal
 * dx x dy x dz cells (R. Zhu, arXiv:1406.7459, Sec. 2, cell labelling),
 *   - the demagnetising field H_demag = K * M as a zero-padded discrete
 *     convolution evaluated by FFT on the 2nx x 2ny x 2nz grid (Sec. 2,
 *     eq. (7)-(16); zero-padding steps (1)-(5)); K = -N with N the
 *     cell-averaged Newell demagnetising tensor, whose transform is taken
 *     once at set-up (Sec. 3, remark after eq. (16));
 *   - the Landau-Lifshitz-Gilbert evolution, eq. (6), under the effective
 *     field of eq. (2): exchange (eq. (3)-(4), free boundaries), uniaxial
 *     anisotropy (eq. (5), easy-axis form), demag and Zeeman.
 *
 * Conventions shared by every entry point
 *   - Fields M and H are float32, structure-of-arrays [3][nz][ny][nx], x
 *     fastest, cells zero-indexed; SI units (A/m), lengths in metres.
 *   - Pointers named *_dev are device (HBM) pointers owned by the caller;
 *     the library never frees them.  Host pointers are named plainly.
 *   - Device memory: the library allocates none.  Every object (plan, batch,
 *     surrogate) reports the bytes it needs (mm_*_workspace_bytes) and works
 *     in a caller-allocated workspace bound to it (mm_*_bind_workspace; 256-
 *     byte aligned, owned by the caller, kept alive and untouched by the
 *     caller until the object is destroyed or re-bound).  The library owns
 *     only host-side metadata, a capture stream and HIP graphs.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All device work is enqueued asynchronously on it unless the entry point
 *     says it synchronises.
 *   - Every call returns MM_OK (0) or a negative MM_E* code; no C++
 *     exception crosses the ABI.  mm_last_error() gives a human-readable
 *     detail of the last failure on the calling thread.
 *   - A plan may be used from one host thread / stream at a time.
 */
#ifndef MM_H
#define MM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MM_OK = 0,
    MM_EINVAL = -1,       /* bad argument (n <= 0, d <= 0, NULL, unsupported length, ...) */
    MM_ENOMEM = -2,       /* device allocation failed */
    MM_ENODEV = -3,       /* no HIP device visible */
    MM_EHIP = -4,         /* a HIP runtime call failed (detail in mm_last_error) */
    MM_ENONFINITE = -5,   /* a reduction found NaN/Inf in the state */
    MM_ETUNE = -6,        /* the autotuner found no valid candidate */
    MM_EUNSUPPORTED = -7  /* valid request outside what the library implements */
};

enum { MM_RK4 = 0, MM_EULER = 1 };
enum { MM_EXACT = 0, MM_SURROGATE = 1 };

/* Opaque plan: grid, Newell spectrum, FFT launch configuration, workspace. */
typedef struct mm_plan_s *mm_plan;

/* Material and integration parameters (Sec. 2, eq. (1)-(6)).
 *  Ms      saturation magnetisation [A/m]
 *  A       exchange stiffness [J/m]; H_exch = 2A/(mu0 Ms^2) lap(M)
 *  Ku      uniaxial anisotropy [J/m^3]; H_anis = 2Ku/(mu0 Ms^2) (u.M) u
 *  axis    easy axis u (unit vector; the paper uses x)
 *  alpha   Gilbert damping
 *  gamma0  gamma*mu0 [m/(A s)], multiplies H in A/m in eq. (6)
 *  Hext    applied field [A/m]
 *  dt      time step [s]
 *  integrator MM_RK4 (classical, 4 field evaluations per step) or MM_EULER
 *  renorm  1: M <- Ms M/|M| after every step, 0: leave |M| free
 *  demag_mode MM_EXACT (FFT demag at every stage) or MM_SURROGATE (the
 *          learned increment attached with mm_sur_attach in RK stages 2-4)
 *  log_every  with a stats array, observables after every log_every steps
 *          (<= 0: only after the last step)
 *  sur_tol relative residual above which a surrogate step is redone exactly
 *  sur_check_every  surrogate steps run before the host reads their
 *          residuals (they are judged on the device); <= 1: every step.
 *          A group with a residual above sur_tol is redone from its first
 *          state with exact demag.  At most MM_SUR_CHECK_MAX.             */
typedef struct {
    double Ms, A, Ku;
    double axis[3];
    double alpha, gamma0;
    double Hext[3];
    double dt;
    int integrator;
    int renorm;
    int demag_mode;
    int log_every;
    double sur_tol;
    int sur_check_every;
} mm_llg_params;

#define MM_SUR_CHECK_MAX 256

/* Observables of a state (Sec. 2, eq. (1) with V = dx dy dz per cell):
 * energies in J, torque_max = max_i |M_i x H_eff,i| / Ms in A/m,
 * m_avg = (1/N) sum M/Ms, nonfinite = number of cells holding NaN/Inf;
 * steps = steps taken before the state was observed (in the call), and
 * fallbacks = surrogate steps redone exactly by then.                      */
typedef struct {
    double E_ex, E_an, E_d, E_z, E_tot;
    double torque_max;
    double m_avg[3];
    long long nonfinite;
    long long steps, fallbacks;
} mm_stats;

/* Plan description filled by mm_plan_query. */
typedef struct {
    int nx, ny, nz;
    int Lx, Ly, Lz;            /* padded FFT lengths >= 2nx, 2ny, 2nz (Lz = 1 when nz = 1: collapsed) */
    long long spectrum_count;  /* floats in the stored K~ octant: 6 (Lx/2+1)(Ly/2+1)(Lz/2+1), nz=1: 6(Lx/2+1)(Ly/2+1) */
    long long workspace_bytes; /* device bytes the plan works in (mm_plan_workspace_bytes) */
    int cfg[9];                /* launch tile per pass kind (see MM_PASS_*) */
    int tune_source;           /* 0 defaults or set by hand, 1 timed by mm_plan_autotune, 2 read from the tune cache */
} mm_plan_info;

/* Pass kinds of one demag evaluation, for tiles and per-kernel timing. */
enum {
    MM_PASS_XFWD = 0,   /* x: real rows -> nx+1 complex, upper half of the padded row zero  */
    MM_PASS_YFWD = 1,   /* y: forward, input rows j < ny                                     */
    MM_PASS_ZCONV = 2,  /* z: forward, K~ . M~ (eq. (13)/(15)), inverse, keep k < nz         */
    MM_PASS_YINV = 3,   /* y: inverse, keep j < ny                                           */
    MM_PASS_XINV = 4,   /* x: complex -> real, keep i < nx (eq. (16), keep first half)       */
    MM_PASS_YCONV = 5,  /* nz = 1: y forward, K~ . M~, y inverse in one pass                 */
    MM_PASS_STAGE = 6,  /* fused H_eff + LLG stage update                                    */
    MM_PASS_REDUCE = 7, /* observables reduction                                             */
    MM_PASS_XSTAGE = 8, /* fused: x inverse of the field, LLG stage, x forward of the result  */
    MM_PASS_COUNT = 9
};

/* Describe a plan for an nx x ny x nz grid of dx x dy x dz cells (Sec. 2,
 * cell labelling and eq. (7)-(12)): sizes, padded transform lengths, launch
 * configuration and the workspace it needs.  Allocates no device memory;
 * the plan computes nothing until a workspace is bound.
 * Any 1 <= n <= 512 per axis: each axis is padded to the smallest transform
 * length L >= 2n of 2, 4, 6, 8, 10, 12, 16, 20, 24, ..., 512, 640, 768, 1024
 * (2^a, 3*2^a and 5*2^a; radices 2, 3, 4, 5, 8, 16); the zero-padded
 * convolution needs L >= 2n - 1 (Sec. 2 zero padding), so L = 2n exactly
 * when n is 2^a, 3*2^a or 5*2^a and the result is the same convolution for
 * any L (mm_plan_info reports Lx, Ly, Lz).
 * Errors: MM_EINVAL (bad sizes), MM_ENODEV, MM_EHIP.                        */
int mm_demag_setup(int nx, int ny, int nz, double dx, double dy, double dz, mm_plan *out);

/* Device bytes the plan works in: K~, twiddles, reduction records and the
 * run-time buffers (half spectra X1 [3][nz][ny][xp] and X2 [3][nz][2ny][xp]
 * c64 with xp = nx+1 rounded up to 16, demag field and RK4 states 4 x
 * [3][nz][ny][nx] f32).                                                     */
int mm_plan_workspace_bytes(mm_plan plan, size_t *bytes);

/* Bind a caller-allocated device workspace of `bytes` >= the size above
 * (256-byte aligned) and compute K~ into it (set-up of the transform of the
 * demag kernel, remark after eq. (16)): the Newell tensor in FP64 on the
 * current device, its transform in FP64 by separable cosine/sine sums, and
 * the real, parity-folded octant of K~ = FFT(-N)/(2nx 2ny 2nz) stored in
 * FP32, one six-float record per frequency.  Synchronises the device.  A
 * second bind moves the plan to the new workspace (K~ is recomputed).
 * Errors: MM_EINVAL (NULL, misaligned), MM_ENOMEM (too small), MM_EHIP.   */
int mm_plan_bind_workspace(mm_plan plan, void *ws_dev, size_t bytes);

/* H_dev = demagnetising field of M_dev (eq. (11)-(16)).  M_dev, H_dev:
 * [3][nz][ny][nx] float32 device arrays, not aliased.  Asynchronous.
 * Errors: MM_EINVAL (NULL plan/pointer, M == H, no workspace bound), MM_EHIP. */
int mm_demag_apply(mm_plan plan, const float *M_dev, float *H_dev, void *stream);

/* For callers that cannot allocate device memory at all (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * mm_demag_apply with its half-spectrum buffers (X1 and X2 above) in a
 * fixed device array of the library, mm_demag_static_scratch_bytes() = 64
 * MiB on each GPU it runs on (held until the process ends), instead of the
 * plan's workspace; the plan still supplies K~ and the twiddles.  The
 * result equals mm_demag_apply's bitwise.  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (other streams, other
 * threads) race.  Allocates nothing.
 * Errors: MM_EINVAL (as mm_demag_apply, or a grid whose half spectra exceed
 * the array), MM_EHIP.                                                      */
int mm_demag_apply_static(mm_plan plan, const float *M_dev, float *H_dev, void *stream);
size_t mm_demag_static_scratch_bytes(void);

/* Advance M_dev (in place) by nsteps time steps of eq. (6) under H_eff of
 * eq. (2), with classical RK4 (four demag evaluations per step) or explicit
 * Euler (one); params->demag_mode MM_SURROGATE takes the attached learned
 * increment in RK stages 2-4 (see mm_llg_step_surrogate).  The steps are
 * replayed from a captured HIP graph after the first call with the same
 * (M_dev, params).
 * stats (host, nullable): NULL -> asynchronous.  Else the call fills
 * ceil(nsteps / e) records, e = log_every if 0 < log_every < nsteps, else
 * nsteps (one record; nsteps = 0 gives one record of the current state):
 * record k holds the observables (as mm_reduce) of the state after
 * min((k+1) e, nsteps) steps, each taken with one extra demag evaluation
 * and an FP64 reduction into device records, read back when RED_LOG (256)
 * are pending and at the end; the call then synchronises `stream` and
 * returns MM_ENONFINITE if a record holds a non-finite cell.
 * Errors: MM_EINVAL (NULL, nsteps < 0, Ms <= 0, dt not finite, no workspace,
 * MM_SURROGATE without an attached surrogate), MM_ENONFINITE, MM_EHIP.      */
int mm_llg_step(mm_plan plan, const mm_llg_params *params, float *M_dev, int nsteps, mm_stats *stats,
                void *stream);

/* Observables of state M_dev (energies per eq. (1), max torque, <m>, NaN
 * count) accumulated in FP64 with a deterministic two-pass wave64
 * reduction.  Synchronises `stream`.  Returns MM_ENONFINITE (with *out
 * filled) if any cell is not finite.                                        */
int mm_reduce(mm_plan plan, const mm_llg_params *params, const float *M_dev, mm_stats *out,
              void *stream);

/* Relax toward the minimum-energy state (the paper's benchmark runs, Sec. 4,
 * relax a cube under demag, exchange and anisotropy): step with `params`
 * until max_i |M_i x H_eff,i| / Ms <= torque_tol, checking every
 * `check_every` steps (mm_llg_step with a stats record), or until
 * max_steps.  Fills *out with the final observables (out->steps = steps
 * taken) and *steps_taken.  Synchronises at every check.                    */
int mm_llg_relax(mm_plan plan, const mm_llg_params *params, float *M_dev, double torque_tol, long long max_steps,
                 int check_every, mm_stats *out, long long *steps_taken, void *stream);

/* Newell tensor N in FP64 on the device for the octant of offsets
 * (i dx, j dy, k dz), 0 <= i < nx, 0 <= j < ny, 0 <= k < nz, written to
 * N_dev[6][nz][ny][nx] (order xx, yy, zz, xy, xz, yz); N_dev is caller
 * device memory of 6*nx*ny*nz doubles.  Exact f/g form for centre distance
 * < 8 cell edges (largest edge), tent-weighted Gauss-Legendre average of the
 * dipole kernel beyond.  Synchronises `stream`.                             */
int mm_newell_tensor(int nx, int ny, int nz, double dx, double dy, double dz, double *N_dev,
                     void *stream);

/* Copy the plan's stored K~ octant (FP32, [nzK][Ly/2+1][Lx/2+1][6] with the
 * six components xx, yy, zz, xy, xz, yz per frequency, nzK = Lz/2+1, or 1
 * when nz = 1; scale and sign folded in) to Kt_dev, which holds
 * `count` floats (>= mm_plan_info.spectrum_count).  Asynchronous.           */
int mm_plan_spectrum(mm_plan plan, float *Kt_dev, long long count, void *stream);

/* Describe a plan. */
int mm_plan_query(mm_plan plan, mm_plan_info *info);

/* Set the launch configuration of one pass kind: tile = P + 256 * variant,
 * P = transforms per workgroup (x rows, or kx columns for y/z; a power of
 * two <= 128), variant = schedule: for the single-component passes 0 = the
 * default values per thread E, 1 = 2E, 2 = radix order 1 (radix 16 first for
 * lengths 2^a, radix 3 then 4s for 3*2^a), 3 = radix order 2 (radix 4 only,
 * 2^a); for the product passes (ZCONV, YCONV) 0 = all three components in
 * one thread's registers, 1 = one component per thread group with the 3x3
 * product exchanged through LDS, 2 = as 1 with 2E, 3 and 4 = as 0 in radix
 * orders 1 and 2.  Tiles of one radix order compute bitwise the same result;
 * different orders agree to rounding.
 * For MM_PASS_STAGE the tile is the vector width W in {1, 2, 4}: W
 * consecutive cells of an x row per thread (nx % W == 0; default 4 when
 * nx % 4 == 0; a launch whose arrays are not aligned to 4W bytes falls back
 * to a narrower width).  For MM_PASS_XSTAGE the tile is P + 256 w: P = 2^k
 * pairs of cell rows per workgroup of the fused pass that runs, per RK
 * stage, the x inverse of the field, the stage and the x forward of its
 * result (the field is never stored; the default), with 2^w cells per stage
 * task, or 0 for the unfused path (XINV, stage kernel, XFWD).  Returns
 * MM_EINVAL for a configuration the pass cannot launch.                     */
int mm_plan_set_tile(mm_plan plan, int pass, int tile);

/* Time every candidate tile of every pass on this plan's buffers and keep
 * the fastest: a candidate is timed as `reps` complete demag evaluations
 * (hipEvents around the loop only), the other passes keeping their current
 * tiles, and the passes are swept twice; then the fused stage pass's tiles,
 * each timed as `reps` RK4 steps.  Candidates are the tile P, the schedule
 * variant and, for the product passes, the radix order (variants 3, 4);
 * one order's candidates agree bitwise, different orders within rounding.
 * Overwrites the plan's stage buffers.  The chosen tiles are readable with
 * mm_plan_query.  Synchronises.
 * Tune cache: when the environment variable MM_TUNE_CACHE names a file, a
 * plan whose (device architecture, compute units, grid) key is in it takes
 * the stored tiles without timing (tune_source 2); otherwise the timed
 * result is added to the file (one JSON object, one key per line).
 * Errors: MM_ETUNE if no candidate ran.                                     */
int mm_plan_autotune(mm_plan plan, int reps, void *stream);

/* Per-kernel timing: when enabled, every launch of the plan is timed with a
 * pair of HIP events and its duration accumulated per pass kind.  For the
 * passes of one kernel (the FFT passes and the stage kernel) the events
 * travel with the dispatch (hipExtLaunchKernelGGL) and time the kernel's
 * execution; the reduction's two kernels are bracketed by recorded events.
 * Steps run as direct launches while timing is on (no graph replay).
 * mm_plan_timing synchronises and returns total milliseconds and launch
 * counts per MM_PASS_* kind (arrays of MM_PASS_COUNT), then resets them.   */
int mm_plan_set_timing(mm_plan plan, int enable);
int mm_plan_timing(mm_plan plan, double *total_ms, long long *launches);

/* ------------------------------------------------------------------------ *
 * Batches: many independent grids of uneven sizes (e.g. the points of a
 * field sweep) stepped together.  Each instance is a full plan; the whole
 * step is replayed from one captured HIP graph.  Two launch modes:
 *   MM_BATCH_MERGED (default): one launch per pass kind over every instance
 *     and transform length (a task table of (instance, block, length),
 *     longest transform first; 3*2^a lengths in radix order 1): at most
 *     4 x 7 launches per RK4 step.  Results are bitwise those of per-instance
 *     plans whose tiles use the same radix orders.
 *   MM_BATCH_GROUPED: one launch per (pass kind, transform length), each
 *     group's tile tuned; bitwise the per-instance default results.
 * ------------------------------------------------------------------------ */
typedef struct mm_batch_s *mm_batch;
enum { MM_BATCH_GROUPED = 0, MM_BATCH_MERGED = 1 };

/* Describe `count` plans (arrays of per-instance sizes and cells, host
 * memory; each instance as in mm_demag_setup) and their task tables.
 * Allocates no device memory.
 * Errors: those of mm_demag_setup, MM_EINVAL (count < 1, NULL array).      */
int mm_batch_setup(int count, const int *nx, const int *ny, const int *nz, const double *dx, const double *dy,
                   const double *dz, mm_batch *out);

/* Device bytes of the batch: every instance's plan workspace, the task
 * tables (sized for the largest candidate tile) and the instance tables.   */
int mm_batch_workspace_bytes(mm_batch batch, size_t *bytes);

/* Bind a caller-allocated device workspace (>= the size above, 256-byte
 * aligned): binds every instance's plan (computing its K~) and uploads the
 * tables.  Synchronises.  Errors: MM_EINVAL, MM_ENOMEM (too small), MM_EHIP. */
int mm_batch_bind_workspace(mm_batch batch, void *ws_dev, size_t bytes);

/* Demag field of every instance: M_dev[i] -> H_dev[i] (host arrays of
 * `count` device pointers, layout as mm_demag_apply, not aliased).  Waits
 * for `stream` before updating the pointer table, then enqueues.            */
int mm_batch_demag(mm_batch batch, const float *const *M_dev, float *const *H_dev, void *stream);

/* nsteps steps of every instance (params: host array of `count`, one
 * integrator for all; M_dev: host array of `count` device pointers,
 * advanced in place).  A change of pointers or parameters re-uploads the
 * instance table (synchronising) and re-captures the step graph.           */
int mm_batch_step(mm_batch batch, const mm_llg_params *params, float *const *M_dev, int nsteps, void *stream);

/* Tune the tile of every (pass, length) group (the grouped mode's launches)
 * on the batch's buffers: a candidate is timed as `reps` complete batched
 * demag evaluations (hipEvents around the loop), the other groups keeping
 * their tiles.  The mode is left as it was.  Overwrites the instances' stage
 * buffers.  Synchronises.                                                   */
int mm_batch_autotune(mm_batch batch, int reps, void *stream);

/* Number of launch groups of the current mode ((pass, length) groups, or
 * pass kinds when merged), kernel launches per RK4 step, total cells.      */
int mm_batch_query(mm_batch batch, int *groups, int *launches_per_step, long long *cells);

/* Select the launch mode (MM_BATCH_MERGED or MM_BATCH_GROUPED).            */
int mm_batch_set_mode(mm_batch batch, int mode);

/* Pass kind (MM_PASS_*), transform length and tile of group `index`.       */
int mm_batch_group_tile(mm_batch batch, int index, int *pass, int *length, int *tile);

/* Release a batch, its plans and tables (NULL is ignored). */
void mm_batch_destroy(mm_batch batch);

/* ------------------------------------------------------------------------ *
 * Learned demag increment for RK stages 2-4 (not in the paper; an added
 * form).  Demag is linear, so a stage field is taken as
 *   H(M_s) = H_d(M_n) + Ms sigma Net((M_s - M_n) / (Ms sigma)),
 * with H_d(M_n) the exact stage-1 field and sigma the rms of the increment.
 * Net: six 3x3x3 convolutions, channels 3-32-32-32-32-32-3, zero "same"
 * padding, bias, GELU (tanh form) between layers; bfloat16 weights and
 * activations on the matrix cores with FP32 accumulation; FP32 master
 * weights trained with Adam (b1 0.9, b2 0.999, eps 1e-8) on the MSE loss.
 * Parameter layout (host arrays of mm_sur_param_count() floats): for each
 * layer, weights [co][ci][kz][ky][kx] then biases [co].
 * ------------------------------------------------------------------------ */
typedef struct mm_sur_s *mm_sur;

typedef struct {
    long long steps;      /* steps taken */
    long long checked;    /* accepted states judged against exact demag */
    long long fallbacks;  /* steps redone with exact demag */
    double last_residual, max_residual, sum_residual;  /* |H_s - H_d| / |H_d| */
} mm_sur_stats;

/* Describe a network for an nx x ny x nz grid of at most 2^25 cells whose
 * zero-padded x-y plane, (ny + 1) * roundup(nx + 1, 8) positions, is below
 * 2^27 (MM_EINVAL otherwise, before any device work).  Allocates no device
 * memory: bind a workspace before any other call.                          */
int mm_sur_create(int nx, int ny, int nz, mm_sur *out);

/* Device bytes of the network's weights, Adam state, activations and
 * training buffers (the zero-padded 8-channel BF16 network input, BF16
 * activations [N][32] of the later layers, padded channel-major copies for
 * the weight gradient, FP32 scratch fields).                               */
int mm_sur_workspace_bytes(mm_sur sur, size_t *bytes);

/* Bind a caller-allocated device workspace (>= the size above, 256-byte
 * aligned); zeroes the weights and Adam state.  Synchronises.
 * Errors: MM_EINVAL (NULL, misaligned), MM_ENOMEM (too small), MM_EHIP.   */
int mm_sur_bind_workspace(mm_sur sur, void *ws_dev, size_t bytes);

/* Attach a bound network to a plan of the same grid (NULL detaches), so
 * that mm_llg_step with params->demag_mode = MM_SURROGATE uses it in RK
 * stages 2-4 with params->sur_tol as the residual gate.                    */
int mm_sur_attach(mm_plan plan, mm_sur sur);
long long mm_sur_param_count(void);
int mm_sur_set_params(mm_sur sur, const float *params, long long n);  /* host; resets Adam state */
int mm_sur_get_params(mm_sur sur, float *params, long long n);
int mm_sur_zero(mm_sur sur);  /* Net == 0: stages 2-4 reuse the stage-1 field */

/* dh_dev = sigma Net(dm_dev / sigma), [3][nz][ny][nx] FP32 device arrays;
 * sigma = rms(dm) if normalize, else 1.  Asynchronous.                      */
int mm_sur_forward(mm_sur sur, const float *dm_dev, float *dh_dev, int normalize, void *stream);

/* MSE loss of Net(dm/sigma) against dh/sigma and its gradient with respect
 * to every parameter (host array, parameter layout; NULL to skip).
 * Synchronises.                                                             */
int mm_sur_gradients(mm_sur sur, const float *dm_dev, const float *dh_dev, int normalize, double *loss,
                     float *grads, long long n, void *stream);

/* One Adam step on that loss with learning rate lr.  Synchronises.          */
int mm_sur_train_step(mm_sur sur, const float *dm_dev, const float *dh_dev, float lr, int normalize,
                      double *loss, void *stream);

/* nsteps RK4 steps of M_dev with the learned increment in stages 2-4 and
 * exact demag at stage 1.  Every accepted state is judged against its exact
 * field, r = |H_s - H_d| / |H_d|, on the device.  The steps run in groups of
 * k = params->sur_check_every (1 if <= 1); the host reads a group's
 * residuals once, after its last step.  If any r > tol the group is redone
 * from its first state with exact demag and the surrogate is skipped for the
 * next step (tol < 0: never redo; tol = 0: always redo, i.e. the plain
 * exact path).  stats->checked counts judged steps, stats->fallbacks steps
 * redone.  Synchronises once per group.
 * Errors: MM_EINVAL (NULL, RK4 only, grids differ, k > MM_SUR_CHECK_MAX),
 * MM_EHIP.                                                                 */
int mm_llg_step_surrogate(mm_plan plan, mm_sur sur, const mm_llg_params *params, float *M_dev, int nsteps,
                          double tol, mm_sur_stats *stats, void *stream);

/* A training pair from the solver's own trajectory: advance M_dev by nsteps
 * exact steps; dm_dev = (M_after - M_before)/Ms, dh_dev = H_d(dm_dev).
 * Asynchronous.                                                             */
int mm_sur_make_pair(mm_plan plan, const mm_llg_params *params, float *M_dev, int nsteps, float *dm_dev,
                     float *dh_dev, void *stream);

void mm_sur_destroy(mm_sur sur);

/* Release a plan and its device memory (NULL is ignored). */
void mm_destroy(mm_plan plan);

/* Static description of a status code. */
const char *mm_status_string(int status);

/* Copy the calling thread's last error detail into buf (NUL-terminated,
 * truncated to n bytes).  Returns the number of bytes of the full detail. */
int mm_last_error(char *buf, size_t n);

#ifdef __cplusplus
}
#endif
#endif /* MM_H */
