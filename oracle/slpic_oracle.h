/*
 * slpic_oracle.h -- FP64 CPU oracle for speed-limited PIC (SLPIC).
 *
 * TEST INFRASTRUCTURE ONLY.  This header and oracle/slpic_oracle.c are the
 * plain, slow reference that the GPU path is checked against.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or constant generator with the HIP
 * library, and the HIP library never calls it.
 *
 * Method (Werner, Jenkins, Chap & Cary, "Speeding Up Simulations By Slowing
 * Down Particles: Speed-Limited Particle-in-Cell Simulation"):
 *   - speed-limited equations of motion, Eq. (10a,b) and Appendix Eq. (A1a,b);
 *   - beta functions, Eq. (11a) (smooth) and Eq. (11b) (step, default);
 *   - leapfrog discretisation with the time integral of beta, Eq. (A2a-d);
 *   - beta-weighted charge deposit, Eq. (A1c)/(A2c);
 *   - Poisson solve, Eq. (A1d)/(A2d).
 *
 * Normalised units: x in electron Debye lengths, t in 1/omega_pe, v in the
 * electron thermal speed, phi in T_e/e, density in n0; eps0 = e = m_e = 1.
 * Positions are stored in grid units xt = x/dx.
 */
#ifndef SLPIC_ORACLE_H
#define SLPIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BETA_STEP = 0, ORC_BETA_SMOOTH = 1 };
enum { ORC_KICK_EXACT = 0, ORC_KICK_MMP = 1 };
enum { ORC_PURPOSE_LOAD = 1, ORC_PURPOSE_INJECT = 2, ORC_PURPOSE_WARM_COUNT = 3, ORC_PURPOSE_WARM = 4,
       ORC_PURPOSE_WALL = 5, ORC_PURPOSE_LIMIT = 6 };
/* Geometry: the sheath (symmetry plane at x = 0, grounded absorbing wall at
 * x = L, volume pair source), the two conducting plates of Sec. IV
 * (phi(0) = 0, phi(L) = bias, both absorbing, half-Maxwellian flux injected
 * from the plate at x = L; the box starts empty), or a periodic box (the
 * uniform plasma of the plasma-oscillation section: particles wrap, no
 * source, the field of the charge less its mean, gauge phi(0) = 0). */
enum { ORC_GEOM_SHEATH = 0, ORC_GEOM_PLATES = 1, ORC_GEOM_PERIODIC = 2 };

typedef struct {
    double charge, mass, temperature;
    int32_t ppc;
    int32_t pad;
} orc_species;

typedef struct {
    int32_t nx;            /* cells; nodes are 0..nx, wall at node nx        */
    int32_t beta_kind;     /* ORC_BETA_STEP / ORC_BETA_SMOOTH                */
    double dx, dt, u;      /* u = +INFINITY -> standard PIC                  */
    int32_t nspecies;      /* 2: species 0 electrons, species 1 ions         */
    int32_t source_cells;  /* injection region xt in [0, source_cells)       */
    orc_species species[2];
    uint64_t seed;
    int32_t run;           /* run index (enters the RNG counter)             */
    int32_t sort_every;    /* 0: never compact; k: stable sort every k steps */
    int32_t sort_bucket;   /* key = cell / bucket; <= 0: key 0 (compaction)  */
    int32_t kick;          /* ORC_KICK_EXACT / ORC_KICK_MMP                  */
    double mmp_tol;        /* relative tolerance of the modified midpoint    */
    double capacity_factor;
    int32_t steady_window; /* steps per wall-potential window; 0: max(1, nx/4) */
    int32_t pad;
    double steady_tol;     /* relative spread of three window means; 0: 0.02 */
    int32_t geometry;      /* ORC_GEOM_SHEATH / ORC_GEOM_PLATES / ORC_GEOM_PERIODIC */
    int32_t pad2;
    double bias;           /* plates: phi(L) in T_e/e                         */
    const double* limit;   /* NULL: the speed limit is u everywhere.  Else nx+1 */
                           /* node values of a limit varying with position:    */
                           /* v0(x) linear between nodes (u then only sets the  */
                           /* species weights, w = dx Z(u)/ppc)                 */
} orc_config;

/* Steady-state detector on the wall potential (a reading: the paper calls
 * the late state an equilibrium without a test).  Steps are grouped into
 * windows of W steps; each closed window's mean joins the last three, and
 * the run is steady at the first step count where the largest deviation of
 * those three means from their average is at most tol * |average|. */
typedef struct {
    int32_t window;        /* W */
    int32_t nopen;         /* steps in the open window */
    double tol;
    double sum;            /* sum of Phi_w over the open window */
    double mean[3];        /* last three window means, newest first */
    int64_t nwin;          /* closed windows */
    int64_t steady_step;   /* step count when first steady, -1 before */
} orc_steady;

void orc_steady_init(orc_steady* d, int32_t window, double tol);
/* Feed the wall potential after a step; step_count = steps completed. */
void orc_steady_feed(orc_steady* d, double phi_w, int64_t step_count);

typedef struct orc_run orc_run;

/* --- Philox4x32-10 counter-based generator (Salmon et al., SC'11) ------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u53(uint32_t a, uint32_t b);

/* --- beta and the velocity map ----------------------------------------- */
double orc_beta(int kind, double u, double speed);
double orc_G(double c2, double p);
double orc_fast_advance(double c2, double p0, double K);
void orc_kick_exact(int kind, double u, double dt, const double v[3],
                    const double a[3], double vout[3]);
int orc_kick_mmp(int kind, double u, double dt, const double v[3],
                 const double a[3], double tol, int nmax, double vout[3]);

/* --- loading helpers ---------------------------------------------------- */
double orc_Z(int kind, double u_over_vt);
double orc_weight(const orc_config* cfg, int s);
void orc_load_particle(const orc_config* cfg, int s, uint32_t i, double out[4]);
void orc_inject_particle(const orc_config* cfg, int s, uint32_t k, uint32_t step, double out[4]);

/* --- grid ---------------------------------------------------------------- */
void orc_poisson1d(int32_t nx, double dx, const double* Q, double* phi, double* E);
void orc_poisson1d_plates(int32_t nx, double dx, const double* Q, double bias, double* phi, double* E);
void orc_wall_inject_particle(const orc_config* cfg, int s, uint32_t k, uint32_t step, double out[4]);
double orc_wall_flux_per_step(const orc_config* cfg, int s);
void orc_poisson1d_periodic(int32_t nx, double dx, const double* Q, double* phi, double* E);
/* x in [0, nx) after a periodic move. */
double orc_wrap_periodic(double xt, int32_t nx);
/* (omega_s / omega_p)^2 = <(beta v_x)^2> / v_t^2 over the Maxwellian of
 * thermal speed vt (the long-wavelength plasma frequency of speed-limited
 * particles, plasma-oscillation section). */
double orc_slpic_plasma_freq2(int kind, double u, double vt);
/* The real root w > k u (omega_p = 1) of the full dispersion relation of
 * speed-limited particles for 1D perturbations exp(i(kx - wt)) of a uniform
 * Maxwellian (plasma-oscillation section). */
double orc_slpic_dispersion(int kind, double u, double vt, double k);

/* --- run ----------------------------------------------------------------- */
/* A run of cfg.  With a limit profile (cfg->limit, copied): the step takes
 * the limit at x^n for the velocity map and the move, frozen over the step
 * like E^n(x^n); the deposit and the moments take it at the particle's
 * position, the plates' wall source the limit at the plate; orc_load loads
 * cell by cell (unit density at rest, each cell's g-particles sampled as
 * f/beta at the limit of its centre, the mean of its two nodes) through the
 * warm loader (plates: nothing).  NULL for a profile node that is not finite
 * and positive, or an infinite u. */
orc_run* orc_create(const orc_config* cfg);
void orc_destroy(orc_run* r);
void orc_load(orc_run* r);
void orc_refresh_fields(orc_run* r);
void orc_step(orc_run* r, int32_t nsteps);
/* Warm load (replaces the particles, resets the counters, sorts if sorting
 * is on and refreshes the fields): profile = 7 x 256 doubles on x/L = k/255,
 * phi, n_e, n_i, Gamma_e, Gamma_i, T_e, T_i (a temperature not positive
 * stands for the species' source temperature). */
int orc_load_warm(orc_run* r, const double* profile);
double orc_warm_cell_vt(const orc_config* cfg, int s, const double* profile, int32_t c);
int64_t orc_warm_cell_count(const orc_config* cfg, int s, const double* profile, int32_t c, double w,
                            double* V_out, double* vt_out);
void orc_warm_particle(const orc_config* cfg, int s, uint32_t i, int32_t c, double V, double vt, double out[4]);
void orc_sort(orc_run* r, int32_t* perm0, int32_t* perm1);
void orc_keys(const orc_run* r, int32_t s, int32_t* keys);
void orc_moments(const orc_run* r, double* out);

int64_t orc_nslots(const orc_run* r, int32_t s);
int64_t orc_capacity(const orc_run* r, int32_t s);
int64_t orc_nlive(const orc_run* r, int32_t s);
int64_t orc_step_index(const orc_run* r);
double orc_acc_e(const orc_run* r);
int64_t orc_absorbed_total(const orc_run* r, int32_t s);
int64_t orc_injected_total(const orc_run* r, int32_t s);
void orc_get_particles(const orc_run* r, int32_t s, double* x, double* vx, double* vy, double* vz);
int orc_set_particles(orc_run* r, int32_t s, int64_t n, const double* x, const double* vx,
                      const double* vy, const double* vz);
void orc_set_counters(orc_run* r, int64_t step, double acc_e);
/* Plates: the fractional wall injection carried over, per species. */
double orc_acc_flux(const orc_run* r, int32_t s);
/* A new speed limit mid-run, higher or lower (u_new > 0, dt_new > 0): f =
 * beta g is kept by resampling the g-particles at the weight of a fresh
 * load at u_new; then the fields are recomputed.  Returns 0, or -1 for an
 * invalid argument or a run with a limit profile. */
int orc_set_speed_limit(orc_run* r, double u_new, double dt_new);
/* The current macroparticle weight of species s. */
double orc_run_weight(const orc_run* r, int32_t s);
/* The monitored value after the last field solve: Phi_w (sheath), phi at
 * node nx/2 (plates), the fundamental sine amplitude of E (periodic). */
double orc_monitor(const orc_run* r);
void orc_get_grid(const orc_run* r, double* Q0, double* Q1, double* phi, double* E);
void orc_get_steady(const orc_run* r, orc_steady* out);

/* Test particles in a prescribed traveling wave (1D1V, periodic x). */
typedef struct {
    double length, v_phase, phi_max, ramp_time, qm, dt, u;
    int32_t beta_kind, pad;
} orc_wave;
double orc_wave_phi0(const orc_wave* w, double t);
double orc_wave_accel(const orc_wave* w, double x, double t);
void orc_wave_push(const orc_wave* w, double* x, double* v, int64_t n, int64_t step0, int32_t nsteps);

/* 2D3V (y periodic, dy = dx): nodes (i, j) at i*ny + j, i = 0..nx. */
typedef struct orc2_run orc2_run;
orc2_run* orc2_create(const orc_config* cfg, int32_t ny, int32_t tile);
int64_t orc2_sort_key(int32_t ny, int32_t tile, double x, double y);
void orc2_destroy(orc2_run* r);
void orc2_load(orc2_run* r);
void orc2_step(orc2_run* r, int32_t nsteps);
void orc2_sort(orc2_run* r, int32_t* perm0, int32_t* perm1);
void orc2_refresh_fields(orc2_run* r);
void orc2_poisson(int32_t nx, int32_t ny, double dx, const double* Q, double* phi, double* Ex, double* Ey);
void orc2_load_particle(const orc_config* cfg, int32_t ny, int s, uint32_t i, double out[5]);
void orc2_inject_particle(const orc_config* cfg, int32_t ny, int s, uint32_t k, uint32_t step, double out[5]);
int64_t orc2_nslots(const orc2_run* r, int32_t s);
int64_t orc2_step_index(const orc2_run* r);
double orc2_acc_e(const orc2_run* r);
double orc2_weight(const orc2_run* r, int32_t s);
void orc2_get_particles(const orc2_run* r, int32_t s, double* x, double* y, double* vx, double* vy, double* vz);
void orc2_set_particles(orc2_run* r, int32_t s, int64_t n, const double* x, const double* y, const double* vx,
                        const double* vy, const double* vz);
void orc2_set_counters(orc2_run* r, int64_t step, double acc_e);
void orc2_get_grid(const orc2_run* r, double* Q0, double* Q1, double* phi, double* Ex, double* Ey);
/* The steady detector of a 2D run, fed with Phi_w = mean_y phi(0, y) after
 * every step (window max(1, nx/4) unless steady_window is set). */
void orc2_get_steady(const orc2_run* r, orc_steady* out);
/* beta-weighted node moments of a 2D run: 7 rows of (nx+1) ny values, phi
 * then n, Gamma_x, kinetic energy density per species (bilinear weights). */
void orc2_moments(const orc2_run* r, double* out);

#ifdef __cplusplus
}
#endif
#endif
