/*
 * scps.h -- C ABI of the MI355X batched rMD / SCPS stepping library.
 *
 * The library advances many independent replicas of chain molecules under
 * Langevin dynamics, eq (Lang) of Orioli, a Beccara, Faccioli, "Self
 * Consistent Path Sampling" (arXiv:1705.02180), biased either by the
 * ratchet-and-pawl force on the contact-map coordinate z (rMD, eqs (FrMD),
 * (zrMD), (Cij)) or by the ratchets on the mean-field tube variables
 * s_lambda, w_lambda (SCPS, eqs (asXa), (awXa), (Fw), (Fs)), and
 * re-estimates the path-ensemble mean contact map, eq (avCij), from the
 * paths it generates.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every call returns scps_status.  On failure scps_last_error() returns a
 *   thread-local message.  INVALID_ARG, SHAPE and STATE leave the context
 *   usable.  HIP and NONFINITE poison it: afterwards only scps_sync() and
 *   scps_destroy() are accepted.  No C++ exception crosses the ABI.
 * - "device" pointers are HIP device allocations (e.g. torch tensors'
 *   data_ptr() on the same GPU); "host" pointers are ordinary memory and are
 *   read or written before the call returns.  The library never frees a
 *   caller's buffer.
 * - Device work is queued on the context's HIP stream and is asynchronous
 *   with respect to the host unless stated otherwise.  The caller keeps
 *   device buffers alive until that work has completed (torch tensors used
 *   on the same stream satisfy this).  An SCPS context in the default form
 *   holds a second stream of its own; when scps_autotune moves the nonbonded
 *   pass there, that part of each step is forked from and joined back to the
 *   context's stream through events within the call, so ordering with the
 *   caller's work on that stream is unchanged.
 * - The library cannot check the extent of a caller's buffer; the sizes
 *   stated below are the caller's contract.
 * - A context is not re-entrant: one thread, one stream at a time.
 *
 * Data layouts
 * ------------
 * - Particles of system s are numbered 0..N_s-1 along the chain.  Bonds join
 *   i and i+1.  Replica r runs system replica_system[r]; off_r is the sum of
 *   N over replicas 0..r-1 and Σ N is the sum over all replicas.
 * - Coordinates x, velocities v: float32, flat, replica r occupies
 *   [3*off_r, 3*off_r + 3*N_r) as [3][N_r] (all x, then all y, then all z).
 * - cvstate: float64 [R][SCPS_CV_STRIDE], see the SCPS_CV_* slots.  The
 *   running minima z_m, s_m, w_m start at +INFINITY; the first force
 *   evaluation then sets them to the current value (z_m(0) = z(X(0)), as in
 *   the rMD section of the paper); the bias functional T starts at 0.
 * - Contact maps are packed upper triangles over a system's contact set:
 *   for contact positions a<b (indices into contact_idx) the entry sits at
 *   a*n_c - a*(a+1)/2 + (b-a-1); P = n_c*(n_c-1)/2 entries per map.
 */
#ifndef SCPS_H
#define SCPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SCPS_OK = 0,
    SCPS_ERR_INVALID_ARG = -1, /* a NULL or out-of-range argument */
    SCPS_ERR_SHAPE = -2,       /* sizes that do not fit together */
    SCPS_ERR_OOM = -3,         /* device or host allocation failed */
    SCPS_ERR_HIP = -4,         /* a HIP runtime call failed (context poisoned) */
    SCPS_ERR_STATE = -5,       /* call not valid in the current state */
    SCPS_ERR_NONFINITE = -6,   /* a replica produced a non-finite coordinate (or overflowed its neighbour list) */
    SCPS_ERR_NO_SUCCESS = -7   /* update_reference_from_paths: no successful path */
} scps_status;

typedef struct scps_ctx scps_ctx;

#define SCPS_CV_STRIDE 8
#define SCPS_MAX_FRAMES 128   /* largest SCPS frame stack (the paper's protocol records ~72 frames per path) */
enum {
    SCPS_CV_Z = 0,   /* z(X) at the last force evaluation (rMD) */
    SCPS_CV_ZM = 1,  /* running minimum z_m (rMD) */
    SCPS_CV_EB = 2,  /* bias energy at the last force evaluation */
    SCPS_CV_S = 3,   /* s_lambda (SCPS) */
    SCPS_CV_W = 4,   /* w_lambda (SCPS), without the constant w0 */
    SCPS_CV_SM = 5,  /* running minimum s_m (SCPS) */
    SCPS_CV_WM = 6,  /* running minimum w_m (SCPS) */
    SCPS_CV_T = 7    /* bias functional T[X] accumulated along the path:
                        every force evaluation adds dt * sum_i |F_bias,i|^2 /
                        (m_i gamma) (rMD section and eq (T); the paper's
                        Gamma_i = 1/(4 gamma_i m_i k_B T) only rescales T).
                        The least biased path of an ensemble is the replica
                        with the smallest T.  Start it at 0. */
};

enum { SCPS_INTEGRATOR_OVERDAMPED = 0, SCPS_INTEGRATOR_BAOAB = 1 };
enum { SCPS_BIAS_RMD = 0, SCPS_BIAS_SCPS = 1 };
enum { SCPS_EXEC_AUTO = 0, SCPS_EXEC_PER_STEP = 1, SCPS_EXEC_PER_STEP_ALL_TILES = 2, SCPS_EXEC_PER_STEP_OVERLAP = 3 };
enum { SCPS_W_INV_LAMBDA = 0, SCPS_W_NO_INV_LAMBDA = 1 };

/* Physics and bias parameters (any consistent unit system; the protein-shaped
 * workloads use A, ps, kJ/mol, e and masses in kJ/mol ps^2/A^2). */
typedef struct {
    int32_t integrator;   /* SCPS_INTEGRATOR_*.  Overdamped: x += dt F/(m gamma) + sqrt(2 kT dt/(m gamma)) xi.
                             BAOAB: v holds the velocity right after the friction/noise substep, so each step is
                             v += dt F/m; x += dt/2 v; v = c1 v + sqrt((1-c1^2) kT/m) xi; x += dt/2 v, c1 = exp(-gamma dt) */
    int32_t bias_mode;    /* SCPS_BIAS_RMD: ratchet on z, eq (FrMD).  SCPS_BIAS_SCPS: ratchets on s, w, eqs (Fw),(Fs) */
    int32_t exec_mode;    /* SCPS_EXEC_AUTO: one persistent launch per call where a replica fits one workgroup
                             (short chains one or several to a wavefront; see scps_set_launch);
                             SCPS_EXEC_PER_STEP: a few kernel launches per step (always used for SCPS and large chains);
                             with r_cut_contact and r_cut_nb both > 0 in rMD mode, this path evaluates the pairs of
                             per-particle neighbour lists instead of every pair: radius (larger cutoff) + 2 A,
                             rebuilt for a replica when one of its particles has moved more than 1 A since the
                             last build (also by the caller between calls) or the reference map changed, at most
                             512 entries per particle
                             (scps_sync reports NONFINITE for a replica that would need more);
                             SCPS_EXEC_PER_STEP_ALL_TILES: the per-step path over every tile pair (no lists).
                             In SCPS mode the first two form the frame-weighted effective references on the fly,
                             inside the pass that applies the bias; SCPS_EXEC_PER_STEP_ALL_TILES writes them to
                             device memory first and reads them back in the pair pass (same results up to float
                             rounding order; it needs R x (contact tile pairs) x 16 KiB of device memory more).
                             SCPS_EXEC_PER_STEP_OVERLAP (SCPS bias only): as SCPS_EXEC_PER_STEP, with the
                             nonbonded pass on the context's second stream beside the distance pass; AUTO and
                             PER_STEP run it after the bias pass unless scps_autotune (AUTO) finds the
                             overlapped schedule more than 3% faster */
    int32_t nb_excl;      /* nonbonded pairs need |i-j| > nb_excl (>= 1) */
    int32_t min_seq_sep;  /* contact pairs need |i-j| > min_seq_sep; the paper's all-atom value is 35 */
    int32_t replica_base; /* replica r uses replica_base + r as its noise counter word, so a context that
                             holds one replica of a larger batch reproduces that replica's noise */
    int32_t w_form;       /* SCPS_W_*: SCPS_W_INV_LAMBDA (0) w = -(1/lambda) log sum_k exp(-lambda d_k), the
                             definition of eqs (wX) and (wXapp); SCPS_W_NO_INV_LAMBDA (1) w = -log sum_k
                             exp(-lambda d_k), as eq (awXa), the protocol and the toy model print it (w and
                             its gradient lambda times larger, so k_w means something else) */
    int32_t reserved;     /* 0 */
    double dt, gamma, kT;
    double k_bond, r_bond;        /* harmonic bond i,i+1 */
    double lj_eps, lj_sigma;      /* Lennard-Jones 12-6; lj_eps = 0 disables */
    double dh_prefactor, dh_kappa;/* Debye-Hueckel k_e/eps_r * q_i q_j exp(-kappa r)/r; prefactor 0 disables */
    double r0_contact;            /* r0 of eq (Cij) */
    double r_cut_contact;         /* <= 0: no cutoff; else C = 0 for r > r_cut (the linear-scaling remark after eq (Cij)) */
    double r_cut_nb;              /* <= 0: no cutoff; else a Lennard-Jones / Debye-Hueckel pair with r > r_cut_nb
                                     contributes nothing (plain truncation, like the contact cutoff).  With both
                                     cutoffs set, the per-step rMD path runs on neighbour lists (see exec_mode) */
    double k_R;                   /* rMD ratchet constant */
    double lambda, k_s, k_w;      /* SCPS tube variables and ratchet constants */
    uint64_t seed;                /* Philox4x32-10 key */
} scps_params;

/* Chains.  All arrays are host memory, copied during scps_init_system. */
typedef struct {
    int32_t n_systems;
    const int32_t *n_particles;   /* [n_systems], each in [2, 1<<20] */
    const int32_t *n_contact;     /* [n_systems], each in [0, N_s] */
    const int32_t *contact_idx;   /* concatenated per system, strictly ascending particle indices */
    const float *mass;            /* concatenated per particle, > 0 */
    const float *charge;          /* concatenated per particle */
} scps_topology;

/* Create a context for n_replicas replicas (1 .. 65535); replica r runs system
 * replica_system[r] (host array).  hip_stream: a hipStream_t, or NULL for the
 * null stream.  Allocates the context's device buffers.  Reference maps are
 * unset until scps_set_reference_map.  Errors: INVALID_ARG, SHAPE, OOM, HIP. */
scps_status scps_init_system(const scps_params *params, const scps_topology *topology,
                             int32_t n_replicas, const int32_t *replica_system,
                             void *hip_stream, scps_ctx **out);

/* Set a system's reference maps.
 *  n_maps == 1: the native map C0 used by z, eq (zrMD), and by the norm of the
 *    tube distance.  Either maps (host float64 [P]) or, when maps is NULL,
 *    native_xyz (host float64 [3][N]) from which C0 = C(X_N), eq (Cij), is
 *    computed on the device in float64.  z0_norm <= 0 sets Z0 to the sum of
 *    (C0_ij)^2 over the contact pairs with |i-j| > min_seq_sep, the
 *    denominator of the normalised distance ||C - C'||^2 of the SCPS
 *    section (its numerator sums over the same pairs); otherwise
 *    Z0 = z0_norm.
 *  n_maps >= 2: the SCPS frame stack <C(t_k)>, k = 0..n_maps-1, host float64
 *    [n_maps][P] in maps, at most SCPS_MAX_FRAMES (128) frames; native_xyz
 *    must be NULL and z0_norm is ignored.  The stack is kept as float32 for
 *    the per-step passes, with the float64 frame distances
 *    sum_p (R_jp - R_kp)^2 of every frame pair.
 * Blocks until the upload is done.  Errors: INVALID_ARG, SHAPE (more than
 * SCPS_MAX_FRAMES frames; the context stays usable), OOM, HIP. */
scps_status scps_set_reference_map(scps_ctx *ctx, int32_t system, int32_t n_maps,
                                   const double *maps, const double *native_xyz,
                                   double z0_norm);

/* Advance every replica by n_steps Langevin steps (eq (Lang)) with the bias
 * of params.bias_mode; global step indices step0 .. step0+n_steps-1.
 * Each step starts with a force evaluation at the current X, which updates
 * the running minima before the bias is applied (so the bias vanishes
 * whenever the collective variable reaches a new minimum).  The noise of
 * particle i of replica r at step t is Philox4x32-10 with key = seed and
 * counter = (i, replica_base + r, low32(t), high32(t)); each of the four 32-bit words w maps
 * to the uniform (2*(w>>9)+1)*2^-24 and Box-Muller turns words 0,1 into the
 * x, y normals and words 2,3 into the z normal.  Results therefore do not
 * depend on batching or on how the call is split into smaller calls.
 *   x, v: device float32 (layout above), in/out.  v may be NULL for the
 *         overdamped integrator and must not be NULL for BAOAB.
 *   cvstate: device float64 [R][SCPS_CV_STRIDE], in/out.
 *   record_every > 0: frames (device float32) receives X after local steps
 *         0, E, 2E, ... <= n_steps, each record being a full copy of the x
 *         layout, i.e. frames is [n_steps/E + 1][3 Σ N].  record_every == 0:
 *         frames is ignored.
 * Non-finite coordinates are flagged per replica on the device and reported
 * by scps_sync().  Requires the native map of every system (rMD) or the frame
 * stack and native map (SCPS).  Errors: INVALID_ARG, STATE, HIP. */
scps_status scps_step_replicas(scps_ctx *ctx, float *x, float *v, double *cvstate,
                               int64_t n_steps, uint64_t step0, int32_t record_every,
                               float *frames);

/* z(X) of eq (zrMD) against each replica's native map, and optionally its
 * gradient.  x: device float32 (layout above).  z: device float64 [R].
 * grad: device float32 (x layout) or NULL; receives coef_r * dz/dx for
 * replica r, where coef_r = grad_coef[r] (device float64 [R]) or 1 when
 * grad_coef is NULL.  C_ij is recomputed per pair; no map of the current
 * contacts is stored.  Errors: INVALID_ARG, STATE, HIP. */
scps_status scps_eval_z_and_grad(scps_ctx *ctx, const float *x, double *z, float *grad,
                                 const double *grad_coef);

/* Ratchet bias energy and its backward coefficient for a batch of z values
 * (rMD, eq (FrMD)): E_b[r] = 1/2 k_R (z - z_m)^2 theta(z - z_m), and, when
 * coef is not NULL, coef[r] = gz[r] + gE[r] * k_R (z - z_m) theta(z - z_m), the
 * factor that multiplies dz/dx in the gradient of gz*z + gE*E_b.  All
 * pointers are device float64 [R]; gz and gE may be NULL (taken as 0).
 * Errors: INVALID_ARG, HIP. */
scps_status scps_ratchet_energy(scps_ctx *ctx, const double *z, const double *z_m,
                                double *E_b, const double *gz, const double *gE,
                                double *coef);

/* out = coef[r] * in over the coordinates of every replica r (x layout; out
 * may equal in): with in = dz/dx kept from scps_eval_z_and_grad and coef from
 * scps_ratchet_energy, this is the gradient of gz*z + gE*E_b without a second
 * pass over the pairs (the backward of the differentiable z wrapper).
 *   in, out: device float32 [3 * sum N]; coef: device float64 [R].
 * Asynchronous.  Errors: INVALID_ARG, HIP. */
scps_status scps_scale_by_replica(scps_ctx *ctx, const float *in, const double *coef, float *out);

/* Forward of the differentiable rMD bias in one call (eq (zrMD) and the
 * ratchet energy of eq (FrMD)): z as scps_eval_z_and_grad computes it,
 * E_b[r] = 1/2 k_R (z - z_m)^2 theta(z - z_m) with theta(0) = 1, and, when
 * grad_z is not NULL, dz/dx.  The z sums, E_b and dz/dx leave the pair pass
 * in one launch (scps_eval_z_and_grad + scps_ratchet_energy take two more).
 *   x: device float32 (x layout); z_m, z, E_b: device float64 [R];
 *   grad_z: device float32 (x layout) or NULL.
 * Asynchronous.  Errors: INVALID_ARG (x, z_m, z or E_b NULL), STATE (a
 * system without its native map), HIP. */
scps_status scps_eval_zbias(scps_ctx *ctx, const float *x, const double *z_m, double *z,
                            double *E_b, float *grad_z);

/* Backward of the differentiable rMD bias in one launch: for every replica r,
 *   grad_x = grad_z * (g_z[r] + g_E[r] k_R (z - z_m) theta(z - z_m)),
 * the gradient of sum_r g_z[r] z_r + g_E[r] E_b,r with respect to x, from
 * dz/dx kept by scps_eval_zbias (scps_ratchet_energy's coef and
 * scps_scale_by_replica, fused).  g_z[r] is read at g_z[r * g_z_stride]
 * (stride 0: one value for every replica, as the gradient of a sum arrives)
 * and likewise g_E; either may be NULL (taken as 0).
 *   z, z_m: device float64 [R]; grad_z, grad_x: device float32 (x layout;
 *   grad_x may equal grad_z).
 * Asynchronous.  Errors: INVALID_ARG (a NULL array other than g_z / g_E, a
 * negative stride), HIP. */
scps_status scps_zbias_backward(scps_ctx *ctx, const double *z, const double *z_m,
                                const double *g_z, int64_t g_z_stride,
                                const double *g_E, int64_t g_E_stride,
                                const float *grad_z, float *grad_x);

/* Path-ensemble mean contact map, eq (avCij): for every recorded frame k,
 * <C(t_k)>_p = (1/|S|) sum over successful paths p of C(X_p(t_k)), summed in
 * float64, and install the result as the system's SCPS frame stack
 * (n_frames maps).  frames: device float32 [n_frames][n_paths][3][N] (the
 * layout step_replicas records when all replicas run this system).
 * success: host uint8 [n_paths], nonzero = path used (the paper keeps paths
 * that reached the native state).  maps_out: host float64 [n_frames][P] or
 * NULL.  n_frames <= SCPS_MAX_FRAMES (128).  Blocks until done.  Errors:
 * INVALID_ARG, SHAPE (n_frames > SCPS_MAX_FRAMES; stack unchanged), NO_SUCCESS
 * (stack unchanged), OOM, HIP. */
scps_status scps_update_reference_from_paths(scps_ctx *ctx, int32_t system, const float *frames,
                                             int32_t n_paths, int32_t n_frames,
                                             const uint8_t *success, double *maps_out);

/* Tube variables s_lambda, w_lambda, eqs (asXa), (awXa) discretised as in the
 * appendix, of every replica's configuration against the frame stack of system
 * stack_system, without ratchets or forces: distances d_k = sum_p (C_p -
 * R_kp)^2 / Z0 (Z0 of stack_system), s = 1 - (1/M) sum_k k p_k, w =
 * -(1/lambda) log sum_k exp(-lambda d_k) (without the 1/lambda for the
 * context's w_form SCPS_W_NO_INV_LAMBDA), p = softmax(-lambda d).  Several
 * initial conditions of one protein are several systems of the same chain,
 * each with the stack of its own runs; this measures any replica against any
 * of them.  Uses the context's lambda (any bias mode; it must be > 0).
 *   x: device float32 [3 * sum N], as for scps_step_replicas.
 *   s, w: device float64 [R] (either may be NULL, not both).
 * Every replica's system must have the same particles and contact set as
 * stack_system.  Asynchronous.  Errors: INVALID_ARG, STATE (stack_system has no
 * native map or no stack of >= 2 frames), SHAPE (a replica's system differs),
 * OOM, HIP. */
scps_status scps_eval_tube(scps_ctx *ctx, int32_t stack_system, const float *x, double *s, double *w);

/* Global progress coordinate sigma(X), eq (sigma): the mean over n_stacks
 * stacks (the systems stack_systems[0..n_stacks), one per initial condition)
 * of the time-weighted frame average that s_lambda measures, i.e.
 * sigma = (1/n_stacks) sum_k (1 - s_lambda^k(X)), in [0, 1] from the unfolded
 * to the folded end of the reference paths.
 *   stack_systems: host int32 [n_stacks]; sigma: device float64 [R].
 * Same conditions, asynchrony and errors as scps_eval_tube. */
scps_status scps_eval_sigma(scps_ctx *ctx, int32_t n_stacks, const int32_t *stack_systems, const float *x,
                            double *sigma);

/* Least-biased path selection, the last step of an SCPS iteration (the
 * method ranks the paths it generated by the bias functional T[X] of eq (T),
 * the weighted time integral of the squared bias force, and keeps the one
 * with the smallest value as its prediction of the most probable path).
 * Finds the replica r with the smallest cvstate[r][SCPS_CV_T] among those with
 * success[r] != 0; equal values go to the lowest r.
 *   cvstate: device float64 [R][SCPS_CV_STRIDE], as scps_step_replicas left it.
 *   success: host uint8 [R], nonzero = candidate; NULL = every replica.
 *   index:   host int32, receives r.
 *   t_min:   nullable host float64, receives T of replica r.
 * Queued behind earlier work on the context's stream; blocks until done.
 * Errors: INVALID_ARG (NULL cvstate or index, or a candidate whose T is NaN
 * or infinite; nothing is written), NO_SUCCESS (no candidate), OOM, HIP. */
scps_status scps_least_biased_path(scps_ctx *ctx, const double *cvstate, const uint8_t *success,
                                   int32_t *index, double *t_min);

/* Replace the stream later calls queue work on (a hipStream_t or NULL).  The
 * calls of a context share its device scratch buffers, so the new stream is
 * first made to wait (hipStreamWaitEvent) for the work still queued on the
 * previous one; nothing blocks the host.  Errors: HIP. */
scps_status scps_set_stream(scps_ctx *ctx, void *hip_stream);

/* Measurement of the SCPS step's two passes over the frame stack.  With
 * enable = k >= 1, every k-th later SCPS step (the first, then every k-th)
 * records HIP events on the context's stream right before and after its
 * distance pass and its bias pass (in the two-pass form: the effective
 * references and the pair pass together); the events are recycled in a ring
 * of 256 timed steps whose oldest entry is read back, waiting for it, before
 * reuse, so timing adds no device work and no full synchronisation.  A timed
 * step's kernels cannot overlap across the events, which shows on short
 * steps: timing every step of 32 replicas x 560 particles (60 us per step)
 * cost 16 % of the throughput, timing every 8th about 2 %.  Calling it
 * resets the sums; enable = 0 stops recording.  Steps run launch by launch
 * while timing is on (no graph replay).
 * Errors: INVALID_ARG (enable < 0), STATE (not an SCPS context), HIP. */
scps_status scps_time_passes(scps_ctx *ctx, int32_t enable);

/* The summed durations in ms (host float64 [2]: distance pass, bias pass) and
 * the number of timed steps (host int64 [2]) since scps_time_passes; waits for
 * the events still pending.  Errors: INVALID_ARG, HIP. */
scps_status scps_pass_times(scps_ctx *ctx, double *ms, int64_t *launches);

/* Wait for the context's stream and report replicas flagged non-finite:
 * *n_bad receives their count and, if bad_replicas is not NULL, up to R ids
 * (host int32 [R]).  Returns NONFINITE if any replica was flagged (and
 * poisons the context), HIP on a runtime error, OK otherwise. */
scps_status scps_sync(scps_ctx *ctx, int32_t *bad_replicas, int32_t *n_bad);

/* Autotuner for the batched stepping (running many replicas at once, SCPS
 * steps 2 and 4): times every launch configuration the context can use for
 * scps_step_replicas -- the persistent kernel with 256, 512 or 1024 threads per
 * replica where a replica's state fits in one workgroup's LDS (also 64, one
 * wavefront, for chains of at most 256 particles), the packed persistent
 * kernel for chains of at most 64 particles (floor(64 / n) replicas per
 * wavefront, n the longest chain, and 1, 2, 4 or 8 wavefronts per
 * workgroup), and the
 * per-step path -- for n_steps steps on private device copies of
 * (x, v, cvstate), in three rounds taken in turns after one untimed step
 * each, and keeps the one with the fastest run for the context's later calls
 * (exec_mode AUTO only).  An SCPS context has the per-step path alone; with
 * exec_mode AUTO the tuner times the two passes one after the other (the
 * default) against the nonbonded pass on the context's second stream beside
 * the distance pass, which it takes only when that is more than 3% faster;
 * other exec modes keep their schedule.
 *   x, v, cvstate: device buffers as for scps_step_replicas; read only.
 *   n_steps: steps timed per configuration, >= 1.
 *   chosen: nullable host int32[2]; receives {0 persistent / 1 per-step /
 *           2 packed, threads per workgroup of the persistent kernel,
 *           replicas per workgroup of the packed kernel, or for an SCPS
 *           context 1 when the nonbonded pass overlaps the distance pass and
 *           0 when it runs after the bias pass}.
 * Results of later calls differ from an untuned context's only by the order
 * of float64 additions.  Allocates three scratch buffers for the duration of
 * the call and synchronises the stream.  Errors: INVALID_ARG, OOM, HIP. */
scps_status scps_autotune(scps_ctx *ctx, const float *x, const float *v, const double *cvstate,
                          int64_t n_steps, int32_t *chosen);

/* Fixes the launch configuration of scps_step_replicas for a context with
 * exec_mode AUTO, as scps_autotune would (e.g. one it chose earlier):
 *   path 0: the persistent kernel, param = threads per workgroup (64, 256,
 *           512, 1024; the replica's state must fit one workgroup's LDS);
 *   path 1: the per-step path (param ignored; the only path of an SCPS
 *           context);
 *   path 2: the packed persistent kernel, param = wavefronts per workgroup
 *           (1 .. 8; every chain of at most 64 particles).
 * Without a call or a tuning, chains of at most 48 particles (at most 64
 * from 2048 replicas up) run packed with four wavefronts per workgroup and
 * longer ones on the persistent kernel where they fit (256 threads per
 * replica when a chain of at most 128 particles runs fewer than 512
 * replicas), else per step.  Results differ between configurations
 * only by the order of float32 and float64 additions.  Host only.
 * Errors: INVALID_ARG (unknown path or parameter; paths 0 and 2 of an SCPS
 * context), SHAPE (the chains do not fit the configuration), STATE
 * (exec_mode not AUTO). */
scps_status scps_set_launch(scps_ctx *ctx, int32_t path, int32_t param);

/* Steps per captured HIP graph on the per-step path (SCPS contexts, and rMD
 * chains too long for the persistent kernel): whole blocks of `steps` steps
 * replay one graph of their kernel launches, captured on first use for the
 * cvstate buffer of the call (again when that buffer, the largest frame stack
 * or `steps` changes).  The noise is that of the same steps launched one by
 * one.  Steps run launch by launch where a block does not fit (before a
 * recorded frame or the end of a call) and with neighbour lists or pass
 * timing.  The overlapped SCPS schedule is captured as two branches of the
 * graph (the nonbonded pass on the context's second stream).
 *   steps: 0 (no graphs, the default) .. SCPS_MAX_GRAPH_STEPS.  Measured
 *   on MI355X with ROCm 7.2: an SCPS step of 32 replicas x 560 particles
 *   is about 1 % faster replayed, one of 32 x 6000 no faster (the launch
 *   gaps are under 1 %), and an rMD step of a few microseconds was slower
 *   replayed, hence the default.
 * Synchronises the stream when the value changes.  Host only.
 * Errors: INVALID_ARG (NULL ctx, steps out of range), STATE (poisoned), HIP. */
#define SCPS_MAX_GRAPH_STEPS 256
scps_status scps_set_graph_steps(scps_ctx *ctx, int32_t steps);

/* Reports the launch configuration the next scps_step_replicas call takes,
 * the untuned defaults above resolved:
 *   launch: host int32[2]; receives {path, parameter} in scps_autotune's
 *           encoding (path 0: threads per workgroup; path 2: replicas per
 *           workgroup; path 1: 1 when an SCPS context overlaps the
 *           nonbonded pass with the distance pass, else 0).  Exec modes
 *           other than AUTO, and SCPS contexts, report path 1.
 * Host only.  Errors: INVALID_ARG (NULL ctx or launch), STATE (poisoned). */
scps_status scps_get_launch(scps_ctx *ctx, int32_t *launch);

/* Convergence measure of the iteration (the paper's Frobenius distance
 * between iterations I and J): the recorded frames of each iteration, projected
 * by the caller onto a plane (for Fip35, the RMSD to native of its two
 * hairpins), mark the cells they visit on an nx x ny grid of square cells of
 * side `cell` with lower corner (x0, y0) (cells half-open; points outside the
 * grid are ignored); each binary occupancy matrix is scaled to unit Frobenius
 * norm and D is the Frobenius norm of their difference, in [0, sqrt 2].  The
 * paper deems an iteration converged when D of consecutive pairs changes by
 * less than 10 %.
 *   xy_a, xy_b: device float32 [n][2] (x, y per frame); n_a, n_b >= 0.
 *   hip_stream: a hipStream_t or NULL.  D: host float64.  Needs no context;
 *   allocates 8 nx ny + 32 bytes of device scratch for the call and blocks.
 * Errors: INVALID_ARG (NULL arrays, bad grid, a set with no point inside the
 * grid), OOM, HIP. */
scps_status scps_path_distance(const float *xy_a, int64_t n_a, const float *xy_b, int64_t n_b, double x0,
                               double y0, double cell, int32_t nx, int32_t ny, void *hip_stream, double *D);

/* scps_path_distance for callers that cannot allocate device memory (code
 * under HIP graph capture or in tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and result, with the occupancy grids
 * and counts in a fixed device array that every GPU the library runs on
 * holds until the process ends (8 MiB + 32 bytes), so grids are limited to
 * nx ny <= 2^20 cells.  Calls no hipMalloc or hipFree; the scratch is cleared
 * by a kernel at every call.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (different streams or threads) race.  Blocks
 * until done.  Errors: INVALID_ARG (as scps_path_distance), SHAPE (more than
 * 2^20 cells), HIP. */
scps_status scps_path_distance_noalloc(const float *xy_a, int64_t n_a, const float *xy_b, int64_t n_b, double x0,
                                       double y0, double cell, int32_t nx, int32_t ny, void *hip_stream,
                                       double *D);

/* ---------------------------------------------------------------------------
 * Toy model (section "Diffusion in a 2-dimensional asymmetric funnel"): one
 * particle on the funnel of eq (U),
 *   U = w^2 r^4 - A1 s1^2/(r^2 + s1^2)^2 + A2 s2^2/(r^2 + s2^2)^2
 *       - A3 s3^2/((x - xm)^2 + (y - ym)^2 + s3^2)^2,   r^2 = x^2 + y^2,
 * (Table 1: A1 = 30, A2 = 20, A3 = 6, s1 = 1, s2 = 2, s3 = 0.5, w = 0.03,
 * xm = 1.5, ym = 0), many independent trajectories at once, float64.  It runs
 * the same protocol with the configuration itself in place of the contact
 * map: rMD on z = |X|, the mean path over the successful trajectories, then
 * the ratchets on the Euclidean tube variables around it.  Needs no context.
 * ------------------------------------------------------------------------- */
typedef struct {
    double A1, A2, A3, s1, s2, s3, w, xm, ym;   /* eq (U), Table 1 */
    double kT;
    double mobility_dt;   /* dt / (m gamma): X += mobility_dt F + sqrt(2 kT mobility_dt) xi (the paper's gamma dt) */
    int32_t bias_mode;    /* SCPS_BIAS_RMD: F_b = -k_R (z - z_m) grad z, z = |X|;
                             SCPS_BIAS_SCPS: ratchets (Fw),(Fs) on s, w of the Euclidean tube around the mean path */
    int32_t w_form;       /* SCPS_W_INV_LAMBDA: w = -(1/lambda) log sum_k exp(-lambda d_k); SCPS_W_NO_INV_LAMBDA:
                             w = -log sum_k exp(-lambda d_k), as the toy-model section prints it */
    double k_R, lambda, k_s, k_w;
    uint64_t seed;        /* Philox key; trajectory t draws from counter (0, first_id + t, step_lo, step_hi) and
                             uses the Box-Muller pair of the first two words for (x, y) */
} scps_funnel_params;

/* Advance n_traj trajectories by n_steps overdamped steps from global step
 * step0.  The discrete tube variables: d_k = |X - P_k|^2 over the mean-path
 * frames P_0..P_M, s = 1 - (1/M) sum_k k p_k, w = -(1/lambda) log sum_k
 * exp(-lambda d_k) (without the 1/lambda for w_form SCPS_W_NO_INV_LAMBDA),
 * p = softmax(-lambda d).
 *   xy: device float64 [n_traj][2], in/out.
 *   cvstate: device float64 [n_traj][SCPS_CV_STRIDE] as for the chains (z, z_m,
 *            E_b, s, w, s_m, w_m, T; minima start at +INFINITY, T at 0; T adds
 *            mobility_dt |F_b|^2 per step).
 *   record_every > 0: frames (device float64 [n_steps/record_every + 1][n_traj][2])
 *            receives X every record_every steps, the start first.
 *   mean_path: device float64 [n_path_frames][2], 2 .. 128 frames (bias_mode SCPS).
 * Asynchronous on hip_stream (a hipStream_t or NULL).  Errors: INVALID_ARG,
 * SHAPE, HIP. */
scps_status scps_funnel_steps(const scps_funnel_params *p, int32_t n_traj, int32_t first_id, double *xy,
                              double *cvstate, int64_t n_steps, uint64_t step0, int32_t record_every, double *frames,
                              int32_t n_path_frames, const double *mean_path, void *hip_stream);

/* The toy model's counterpart of eq (avCij): the mean over the trajectories
 * with success[t] != 0 of every recorded frame.
 *   frames: device float64 [n_frames][n_traj][2]; success: host uint8 [n_traj];
 *   mean_path: device float64 [n_frames][2].
 * Blocks until done.  Errors: INVALID_ARG, NO_SUCCESS, OOM, HIP. */
scps_status scps_funnel_mean_path(int32_t n_traj, int32_t n_frames, const double *frames, const uint8_t *success,
                                  double *mean_path, void *hip_stream);

/* Free the context and everything it owns; NULL is accepted. */
void scps_destroy(scps_ctx *ctx);

/* Message of the last failed call on this thread ("" if none). */
const char *scps_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SCPS_H */
