/*
 * slpic.h -- C ABI of the MI355X (gfx950) speed-limited PIC library.
 *
 * Method: Werner, Jenkins, Chap & Cary, "Speeding Up Simulations By Slowing
 * Down Particles: Speed-Limited Particle-in-Cell Simulation" (arXiv:1511.08225).
 *   Eq. (5)        f = beta g: macroparticles sample g; the physical density
 *                  is the beta-weighted sum over them.
 *   Eq. (10a,b)    dx/dt = beta v, dv/dt = beta a.
 *   Eq. (11a,b)    speed-limiting functions (smooth and step).
 *   Appendix A,    electrostatic SLPIC and its leapfrog discretisation, which
 *   Eq. (A1),(A2)  every step of this library implements: gather E^n(x^n),
 *                  v^{n+1/2} = v^{n-1/2} + (q/m) E^n int beta dt, x^{n+1} =
 *                  x^n + beta v^{n+1/2} dt, rho^{n+1} = sum w beta delta,
 *                  div E^{n+1} = rho^{n+1}.
 *
 * Geometry (1D3V electrostatic sheath): x in [0, L = nx*dx]; x = 0 is a
 * symmetry plane (specular particles, dphi/dx = 0), x = L a grounded
 * absorbing wall (phi = 0).  A thermal source injects electron/ion pairs in
 * the first source_cells cells, balancing the ion loss to the wall.
 *
 * Geometry SLPIC_GEOM_PLATES (the two-plate sheath of Sec. IV): conducting
 * plates at x = 0 (phi = 0) and x = L (phi = bias), both absorbing; the box
 * starts empty and both species enter through x = L with the one-sided flux
 * of a stationary Maxwellian of unit density, n0 v_t / sqrt(2 pi) per unit
 * area and time (the g-particles crossing carry the physical flux, Eq. 5):
 * v_x = -v_t sqrt(-2 ln(1 - U)), v_y and v_z Maxwellian, placed a uniform
 * fraction of the step's travel beta(|v|) |v_x| dt inside the plate (at most
 * source_cells cells).  The monitored potential is phi at node nx/2.
 *
 * Geometry SLPIC_GEOM_PERIODIC (the uniform plasma of the plasma-oscillation
 * section): positions wrap around [0, L), nothing is absorbed or injected;
 * node nx is the image of node 0 (the deposit on it is folded onto node 0 in
 * the solve), the mean charge is removed (a neutralising background) and
 * phi(0) = 0 fixes the gauge; E by centred differences around the ring.
 * The monitored value (history, steady detector, wall_potential) is the
 * fundamental sine amplitude of E, (2/nx) sum_{j<nx} E_j sin(2 pi j/nx).  slpic_moments uses the sheath's half volumes at both end
 * nodes, so its values at nodes 0 and nx are not those of a periodic box.
 * Normalised units: x in electron Debye lengths, t in 1/omega_pe, v in the
 * electron thermal speed, phi in T_e/e, density in n0; e = m_e = eps0 = 1.
 *
 * Memory and ownership.  The caller owns all device memory: one workspace of
 * slpic_workspace_bytes() bytes (256-byte aligned device pointer), plus the
 * output buffers passed to slpic_moments().  The library never allocates
 * device memory.  It owns only the host-side context and the HIP graphs and
 * events it creates, released by slpic_destroy().  "stream" arguments are
 * hipStream_t handles passed as void* (NULL = the default stream).
 *
 * Errors.  Every int-returning call returns SLPIC_OK (0) or a negative
 * SLPIC_E* code and never throws.  Faults found on the device (capacity
 * overflow, non-finite particle velocities) set sticky per-run flags that
 * slpic_status_query() reports; the affected particles are dropped and the
 * run keeps stepping.
 *
 * Threading.  One context is used by one host thread at a time.  Work is
 * enqueued on the stream given to each call; calls documented as "sync"
 * synchronise that stream before returning.
 */
#ifndef SLPIC_H
#define SLPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SLPIC_OK = 0,
    SLPIC_EINVAL = -1,     /* bad argument or configuration                */
    SLPIC_ENOMEM = -2,     /* workspace smaller than slpic_workspace_bytes */
    SLPIC_ECAPACITY = -3,  /* particle buffer full (sticky device flag)   */
    SLPIC_ENUMERIC = -4,   /* non-finite particle state (sticky flag)      */
    SLPIC_EHIP = -5,       /* a HIP runtime call failed                    */
    SLPIC_ESTATE = -6,     /* call not valid in the context's state        */
    SLPIC_ELIMIT = -7      /* input larger than an allocation-free call's  */
                           /* fixed scratch                                */
};

/* Speed-limiting function: Eq. (11b) (default) or Eq. (11a). */
enum { SLPIC_BETA_STEP = 0, SLPIC_BETA_SMOOTH = 1 };

/* Particle precision.  Grids, deposits and the field solve are FP64 in both.
 * SLPIC_F32: positions are int32 fixed-point grid coordinates, velocities
 * FP32; SLPIC_F64: positions and velocities FP64. */
enum { SLPIC_F32 = 0, SLPIC_F64 = 1 };

/* Geometry of a run (slpic_run_config.geometry). */
enum { SLPIC_GEOM_SHEATH = 0, SLPIC_GEOM_PLATES = 1, SLPIC_GEOM_PERIODIC = 2 };

/* Error flag bits reported in slpic_run_status.error_flags. */
enum { SLPIC_FLAG_CAPACITY = 1, SLPIC_FLAG_NUMERIC = 2 };

typedef struct {
    double charge;       /* in units of e (electron: -1)           */
    double mass;         /* in electron masses                       */
    double temperature;  /* in T_e                                   */
    int32_t ppc;         /* macroparticles per cell at load          */
    int32_t reserved;
} slpic_species;

typedef struct {
    int32_t nx;            /* cells, 4..2729; nodes 0..nx                       */
    int32_t beta_kind;     /* SLPIC_BETA_STEP / SLPIC_BETA_SMOOTH               */
    double dx, dt;         /* cell size, time step                              */
    double u;              /* speed limit v0; +INFINITY reduces to standard PIC */
    int32_t nspecies;      /* must be 2: species 0 electrons, 1 ions            */
    int32_t source_cells;  /* source region xt in [0, source_cells)            */
    slpic_species species[2];
    uint64_t seed;         /* Philox key                                         */
    int32_t run_id;        /* enters the Philox counter                          */
    int32_t steady_window; /* steps per wall-potential window; 0 = max(1, nx/4)  */
    double capacity_factor;/* particle slots per species = ceil(cf * nx * ppc)  */
    double steady_tol;     /* steady when the last three window means of Phi_w  */
                           /* lie within steady_tol * |their mean| of it;       */
                           /* 0 = default 0.02                                  */
    const double* warm_profile; /* NULL: cold load.  Else a host array of 7 x 256 */
                           /* doubles on x/L = k/255 (k = 0..255): phi, n_e,    */
                           /* n_i, Gamma_e, Gamma_i, T_e, T_i (physical; T in   */
                           /* T_e units, not positive = the species' source     */
                           /* temperature), read by slpic_workspace_bytes and    */
                           /* slpic_init only: each cell is loaded from the      */
                           /* Maxwellian of its temperature (vt = sqrt(T/m))     */
                           /* drifting at V = Gamma/n (|V| <= 4 vt) with         */
                           /* n dx <1/beta>/w g-particles sampled as f/beta      */
                           /* (Eq. 5)                                            */
    int32_t geometry;      /* SLPIC_GEOM_SHEATH (0), SLPIC_GEOM_PLATES or       */
                           /* SLPIC_GEOM_PERIODIC; the last two need no        */
                           /* warm_profile                                      */
    int32_t reserved;
    double bias;           /* SLPIC_GEOM_PLATES: phi(L) in T_e/e; else unused   */
    const double* limit_profile; /* NULL: the speed limit is u everywhere.  Else */
                           /* a host array of nx + 1 finite positive node      */
                           /* values of a limit v0(x) varying with position    */
                           /* (Sec. II lets beta depend on position), linear   */
                           /* between nodes, read by slpic_workspace_bytes and  */
                           /* slpic_init only; u must then be finite and only  */
                           /* sets the species weights (w = dx Z(u/vt)/ppc).   */
                           /* A step takes the limit at x^n for the velocity   */
                           /* map and the move (frozen over the step like      */
                           /* E^n(x^n)); the charge and the moments take it at */
                           /* the particle's position; the plates' wall source */
                           /* takes it at the plate.  The cold load goes cell  */
                           /* by cell (unit density at rest, g = f/beta at the */
                           /* limit of the cell centre, the mean of its nodes)  */
                           /* through the warm-load sampler; with warm_profile */
                           /* the warm cells take that limit too.  1D only.    */
} slpic_run_config;

typedef struct {
    int32_t precision;    /* SLPIC_F32 / SLPIC_F64 (all runs of a context)          */
    int32_t sort_every;   /* stable cell sort + compaction every k steps; 0 = never  */
    int32_t sort_bucket;  /* sort key = cell / bucket; 0 = compaction only (key 0)   */
    int32_t chunk;        /* particles per push wavefront: 64 P, P in {1, 2, 4, 8,  */
                          /* 16}; 0 = default (512 for F32, 256 for F64)             */
    int32_t block;        /* threads per push workgroup: 64, 128, 192 or 256, one   */
                          /* wavefront per chunk; 0 = default (128)                  */
    int32_t graph_steps;  /* steps captured per HIP graph; 0 = direct launches       */
    int32_t sort_tile;    /* particles per sort workgroup, at most 32768; 0 = 16384  */
    int32_t retire_steady;/* 1: a run stops advancing (push, source, field solve and */
                          /* step count frozen) from the step after its steady      */
                          /* detector flags it; 0 = every run always advances       */
    int32_t push_order;   /* order of the push launch's wavefronts: 0 = run by run,  */
                          /* each species' chunks in slot order; 1 = run by run,    */
                          /* the two species' chunks interleaved (by first slot).   */
                          /* Results do not depend on it (but for the order of the  */
                          /* charge atomics); the faster one depends on the size.   */
    int32_t record_perm;  /* 1: every sort also stores its permutation for         */
                          /* slpic_export_perm; 0 = not stored (the scatter writes */
                          /* the particles only, 4 B per particle less) and        */
                          /* slpic_export_perm returns SLPIC_EINVAL                 */
} slpic_tuning;

typedef struct {
    int64_t step;              /* completed steps                                  */
    int64_t nslots[2];         /* occupied slots per species (live + dead holes)   */
    int64_t capacity[2];
    int64_t absorbed_total[2]; /* particles absorbed at the wall since load        */
    int64_t injected_total[2]; /* particles injected by the source since load      */
    double acc_e;              /* fractional electron injection carried over       */
    double wall_potential;     /* phi(0) - phi(L) after the last field solve       */
                               /* (plates: phi at node nx/2; periodic: the sine     */
                               /* amplitude of E's fundamental mode)               */
    int32_t error_flags;       /* SLPIC_FLAG_* bits (sticky)                       */
    int32_t fixed_bits;        /* F32: fraction bits of the position fixed point   */
    double weight[2];          /* macroparticle weight per species, dx Z / ppc     */
    int64_t steady_step;       /* step count when the run became steady, -1 before */
    int64_t windows;           /* closed wall-potential windows                    */
    double window_mean[3];     /* the last three window means of Phi_w, newest first */
    int64_t moment_samples;    /* samples in the moment window (slpic_moments_sample) */
    double acc_flux[2];        /* plates: fractional wall injection per species     */
} slpic_run_status;

/* Bytes of device workspace needed for nruns runs (a sheath each) with the
 * given tuning (NULL = defaults).  Returns 0 on an invalid configuration. */
size_t slpic_workspace_bytes(const slpic_run_config* runs, int32_t nruns, const slpic_tuning* tuning);

/* Create a context over the caller's workspace and load every run cold
 * (or warm, from its warm_profile):
 * g0 = f0/beta (Eq. 5) sampled with Philox4x32-10 from each run's seed,
 * weight dx Z/ppc with Z = <1/beta> over the Maxwellian; then (if sort_every
 * > 0) the first cell sort, the beta-weighted deposit of rho^0 (Eq. A2c) and
 * the field solve (Eq. A2d).  Async on stream; *out is valid on return. */
int slpic_init(const slpic_run_config* runs, int32_t nruns, const slpic_tuning* tuning,
               void* d_workspace, size_t workspace_bytes, void* stream, void** out_ctx);

/* Advance every run by nsteps leapfrog steps of Eq. (A2a-d): push and
 * beta-weighted deposit, wall absorption, source injection, field solve,
 * and the periodic cell sort.  Async (enqueue only; HIP-graph replays when
 * tuning.graph_steps > 0). */
int slpic_step(void* ctx, int32_t nsteps, void* stream);

/* beta-weighted moments of the physical distribution f = beta g (Eq. 5) for
 * one run at its current state, written to the caller's device buffer d_out
 * of (1 + 3*2) * (nx+1) doubles, row-major: phi, then for species 0 and 1
 * the density n, the flux Gamma_x = n <v_x> and the kinetic-energy density.
 * Async on stream. */
int slpic_moments(void* ctx, int32_t run, double* d_out, void* stream);

/* Add the current moments of one run (run >= 0) or of every run (run = -1)
 * to the run's moment window on the device: the raw beta-weighted sums of
 * slpic_moments and phi, and one sample count.  Async; graph-free (call it
 * between slpic_step calls at the cadence wanted). */
int slpic_moments_sample(void* ctx, int32_t run, void* stream);

/* In-step sampling: from the next step on, every step whose count (the
 * context's step counter, as in slpic_step) is a multiple of `every` ends
 * with slpic_moments_sample(ctx, -1), inside the captured HIP graphs too, so
 * that time averages cost no host round trip; 0 turns it off.  With
 * tuning.graph_steps > 0, `every` must divide graph_steps (SLPIC_EINVAL
 * otherwise); the captured graph is rebuilt at the next replay.  Sync. */
int slpic_set_sampling(void* ctx, int32_t every);

/* The window mean of one run's moment samples, in the layout of
 * slpic_moments (all zero without samples), to the caller's device buffer;
 * reset != 0 then empties the window.  Async on stream. */
int slpic_moments_window(void* ctx, int32_t run, double* d_out, int32_t reset, void* stream);

/* Sync.  Copies the status of runs [0, nruns) to h_out. */
int slpic_status_query(void* ctx, slpic_run_status* h_out, int32_t nruns);

/* Sync.  The wall potential Phi_w after each of the last min(step, 4096)
 * steps of one run, oldest first, to h_out (at least 4096 doubles); *n
 * receives the count.  Step k (1-based) of the run is entry n - (step - k) - 1. */
#define SLPIC_HISTORY_LEN 4096
int slpic_wall_history(void* ctx, int32_t run, double* h_out, int64_t* n);

/* Sync.  Copies the nslots occupied slots of (run, species) to host arrays
 * of at least *n doubles: xt = x/dx (dead slots < 0), v_x and v_perp^2 =
 * v_y^2 + v_z^2.  On entry *n is the host capacity; on return the count.
 * Returns SLPIC_EINVAL if the arrays are too small. */
int slpic_export_particles(void* ctx, int32_t run, int32_t species, double* h_xt, double* h_vx,
                           double* h_vperp2, int64_t* n);

/* Sync.  Replaces the particles of (run, species) with n slots from host
 * arrays (layout as in export; F32 positions round to the fixed point).
 * Fields are not recomputed: call slpic_refresh_fields(). */
int slpic_import_particles(void* ctx, int32_t run, int32_t species, const double* h_xt,
                           const double* h_vx, const double* h_vperp2, int64_t n);

/* Sync.  Sets the step counter (enters the source's Philox counter) and the
 * fractional electron-injection accumulator of one run. */
int slpic_set_counters(void* ctx, int32_t run, int64_t step, double acc_e);

/* Sync.  Change the speed limit of one run mid-run to u (higher or lower;
 * +INFINITY turns it into standard PIC) with time step dt from the next
 * step on (the paper lets the limit vary in time, to adjust the
 * approximation during a simulation).  The physical distribution f = beta g
 * is kept: the species weights become those of a fresh load at u (w' = dx
 * Z(u)/ppc), and each live g-particle of the run, of velocity v, is
 * replaced by m copies, m = floor(p) + [U < p - floor(p)], p = (beta_old(|v|)
 * w) / (beta_u(|v|) w') (a raise: p <= w/w'; a lowering: p <= (beta_old /
 * beta_u) w/w', of order |v|/<|v|> for the fast particles; at most 255), U
 * the first draw of its own Philox stream (purpose 6, its slot, the step
 * count); the copies keep the slot order with dead slots dropped, in every
 * run of the context (the others keep each live particle once).  Then the
 * charge and fields are recomputed.  The last sort permutation is
 * overwritten.  Copies beyond the capacity are dropped with
 * SLPIC_FLAG_CAPACITY.  SLPIC_EINVAL for u <= 0, dt <= 0, a run with a
 * limit profile, a plates run whose wall flux per step would grow, or a
 * resampled total of 2^31 slots or more (then nothing has changed but the
 * last sort permutation). */
int slpic_set_speed_limit(void* ctx, int32_t run, double u, double dt, void* stream);

/* Sync.  With tuning.retire_steady, takes every run that has retired
 * (frozen at its steady step) and is not yet pruned out of the push and sort
 * work: its particles are copied into both particle buffers (the sort no
 * longer moves them), the push launch and captured graphs cover only the
 * remaining runs' chunks, and the sort keeps a pruned run's counts.  Its
 * state, moments, exports and refresh stay available.  *h_pruned (may be
 * NULL) receives the number of pruned runs.  Retired runs cost no push or
 * sort work only once pruned; call it at the cadence the status is polled. */
int slpic_prune_retired(void* ctx, int32_t* h_pruned, void* stream);

/* Sync.  Sets the fractional wall-injection accumulators of one run of the
 * plates geometry (h_acc: 2 doubles in [0, 1), electrons then ions). */
int slpic_set_flux_counters(void* ctx, int32_t run, const double* h_acc);

/* Recompute rho (Eq. A2c, from the stored particles) and the fields
 * (Eq. A2d) of every run without pushing.  Async. */
int slpic_refresh_fields(void* ctx, void* stream);

/* Sync.  Copies one run's last deposited charge per species (h_Q: 2*(nx+1)
 * doubles, Q_j = sum q w beta W_j, so rho_j = Q_j/dV_j), potential and
 * field at the nodes.  Any pointer may be NULL. */
int slpic_export_grid(void* ctx, int32_t run, double* h_Q, double* h_phi, double* h_E);

/* Run the stable cell sort (compaction) of every run now.  Async. */
int slpic_sort_now(void* ctx, void* stream);

/* Sync.  The permutation of the last sort of (run, species): h_perm[new] =
 * old slot, *n entries (capacity on entry, count on return).  Only in a
 * context whose tuning has record_perm = 1 (SLPIC_EINVAL otherwise). */
int slpic_export_perm(void* ctx, int32_t run, int32_t species, int32_t* h_perm, int64_t* n);

/* Kernel timing with HIP events on the launch stream (for roofline
 * accounting).  enable is a bitmask of kernel classes (bit 0 push-deposit,
 * bit 1 the plates wall injection (the sheath source runs inside the
 * field-solve launch), bit 2 source + field solve, bit 3 sort; 0 = off): an event
 * pair is recorded around every launch of an enabled class in slpic_step, and
 * previous records are cleared.  While profiling is on, slpic_step launches
 * every kernel directly (no graph replay).
 * slpic_profile_read (sync) returns the summed milliseconds and launch
 * counts per kernel class in that order (arrays of 4). */
int slpic_profile(void* ctx, int32_t enable);
int slpic_profile_read(void* ctx, double* h_ms, int64_t* h_launches);

/* Live particles advanced by all push launches since slpic_init (summed
 * over runs and species), for pushes/s accounting.  Sync. */
int slpic_total_slots(void* ctx, int64_t* h_total);

/* The velocity update of Eq. (A2a) alone, on caller device arrays of n
 * particles (float when precision = SLPIC_F32, double otherwise): d_out[i]
 * = v_x^{n+1/2} from d_vx[i] = v_x^{n-1/2}, d_vperp2[i] = v_y^2 + v_z^2 and
 * the acceleration d_a[i] = (q/m) E_x held fixed over the step, with the
 * integral of beta along the velocity path taken exactly (Eq. 11a or 11b
 * by beta_kind; u = +INFINITY gives v + a dt).  d_iters (nullable, int32)
 * receives the Newton iterations each particle used.  Async on stream;
 * SLPIC_EINVAL on bad arguments. */
int slpic_velocity_map(int32_t precision, int32_t beta_kind, double u, double dt, int64_t n,
                       const void* d_vx, const void* d_vperp2, const void* d_a, void* d_out,
                       int32_t* d_iters, void* stream);

/* Release the context (not the caller's workspace).  Safe on NULL. */
void slpic_destroy(void* ctx);

/* ------------------------------------------------------------------------
 * Test particles in a prescribed traveling wave (Sec. V, wave-particle
 * interactions): 1D1V particles (v_y = v_z = 0) in the periodic box
 * [0, length) under phi(x, t) = phi0(t) sin(k (x - v_phase t)),
 * k = 2 pi / length, phi0 rising linearly from 0 to phi_max over
 * [0, ramp_time] (0: phi_max from the start).  The particles do not act on
 * the field.
 * ------------------------------------------------------------------------ */
typedef struct {
    double length;      /* periodic box [0, length)                          */
    double v_phase;     /* phase velocity of the wave                        */
    double phi_max;     /* potential amplitude after the ramp                */
    double ramp_time;   /* duration of the linear ramp, >= 0                 */
    double qm;          /* charge / mass of the particles (electrons: -1)    */
    double dt;          /* time step                                         */
    double u;           /* speed limit v0; +INFINITY: standard PIC           */
    int32_t beta_kind;  /* SLPIC_BETA_STEP / SLPIC_BETA_SMOOTH               */
    int32_t reserved;
} slpic_wave_config;

/* Advance n particles (caller device arrays d_x, d_v of float for SLPIC_F32
 * or double for SLPIC_F64, updated in place: x in [0, length), v the
 * velocity v^{n-1/2}) through steps step0 .. step0 + nsteps - 1: at step m,
 * t = m dt, a = (q/m) E(x, t) with E = -dphi/dx evaluated at the particle,
 * v <- the exact map of Eq. (A2a) (1V), x <- x + beta(|v|) v dt wrapped into
 * [0, length).  One thread per particle carries it through all nsteps in
 * registers.  Async on stream; SLPIC_EINVAL on bad arguments. */
int slpic_wave_push(int32_t precision, const slpic_wave_config* cfg, void* d_x, void* d_v, int64_t n,
                    int64_t step0, int32_t nsteps, void* stream);

/* Static description of an SLPIC_* code. */
const char* slpic_strerror(int code);

/* ------------------------------------------------------------------------
 * Warm-start network (not in the paper): 4 -> 256 -> 256 -> 256 -> 1792,
 * ReLU after the hidden layers, mapping standardised sheath parameters to
 * standardised steady profiles.  BF16 weights, biases, inputs and stored
 * activations (round to nearest even from FP32), FP32 accumulation on the
 * matrix cores.  Parameter vector, element offsets identical in the BF16
 * and the FP32 copy: W1 [256][4], b1 [256], W2 [256][256], b2 [256],
 * W3 [256][256], b3 [256], W4 [1792][256], b4 [1792].  The caller owns every
 * buffer; batch must be a positive multiple of 16.  All calls are async on
 * stream and return SLPIC_EINVAL on bad arguments.
 * ------------------------------------------------------------------------ */
#define SLPIC_MLP_IN 4
#define SLPIC_MLP_HIDDEN 256
#define SLPIC_MLP_OUT 1792
#define SLPIC_MLP_PARAMS 593408

/* Bytes of the activation buffer written by forward and read by backward
 * (BF16 inputs and the three hidden activations), and of backward's
 * scratch buffer (BF16 output and hidden gradients). */
size_t slpic_mlp_act_bytes(int32_t batch);
size_t slpic_mlp_work_bytes(int32_t batch);

/* d_params_bf16 (uint16 BF16 bits) = BF16 rounding of d_params_fp32. */
int slpic_mlp_to_bf16(const float* d_params_fp32, void* d_params_bf16, void* stream);

/* d_y [batch][1792] (FP32) from d_x [batch][4] (FP32); d_act receives the
 * activations backward needs. */
int slpic_mlp_forward(const void* d_params_bf16, const float* d_x, float* d_y, int32_t batch, void* d_act,
                      void* stream);

/* Allocation-free variant of slpic_mlp_forward, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): the same kernels and the same d_y, with
 * the activations in a fixed array of the library's code object instead of
 * a caller buffer (SLPIC_MLP_NOALLOC_MAX_BATCH x 772 BF16 = 1.5 MiB, held on
 * every GPU the library runs on until the process ends).  It calls no
 * allocator.  The first call on a device (that device current) looks up the
 * array's address there.  batch beyond SLPIC_MLP_NOALLOC_MAX_BATCH returns
 * SLPIC_ELIMIT; nothing else is retained between calls (every call rewrites
 * the activations it reads).  Calls that overlap on one GPU (other streams,
 * other threads) share the array and race: serialise them. */
#define SLPIC_MLP_NOALLOC_MAX_BATCH 1024
int slpic_mlp_forward_noalloc(const void* d_params_bf16, const float* d_x, float* d_y, int32_t batch,
                              void* stream);

/* d_grads [SLPIC_MLP_PARAMS] (FP32, overwritten) = gradient of
 * sum(d_dy * y) for the batch whose activations forward left in d_act. */
int slpic_mlp_backward(const void* d_params_bf16, const void* d_act, const float* d_dy, float* d_grads,
                       int32_t batch, void* d_work, void* stream);

/* Mean squared error over n values: d_dy = 2 (y - t) / n, and the loss
 * sum (y - t)^2 / n added to *d_loss (one FP32, zeroed by the caller). */
int slpic_mlp_mse(const float* d_y, const float* d_t, float* d_dy, int64_t n, float* d_loss, void* stream);

/* One Adam step (step counts from 1) on the FP32 master parameters with
 * moment buffers d_m, d_v (FP32, zero before step 1), refreshing the BF16
 * copy. */
int slpic_mlp_adam(float* d_params_fp32, void* d_params_bf16, float* d_m, float* d_v, const float* d_grads,
                   float lr, float beta1, float beta2, float eps, int32_t step, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SLPIC_H */
