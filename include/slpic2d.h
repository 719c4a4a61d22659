/*
 * slpic2d.h -- C ABI of the 2D3V configuration of the MI355X (gfx950)
 * speed-limited PIC library (arXiv:1511.08225).
 *
 * The step is the one of slpic.h, Appendix A, Eq. (A2a-d), in two spatial
 * dimensions: gather E^n(x^n) by bilinear (cloud-in-cell) interpolation,
 * v^{n+1/2} from the exact frozen-field integral of beta with
 * a = (q/m)(E_x, E_y, 0), x^{n+1} = x^n + beta v^{n+1/2} dt per coordinate,
 * rho^{n+1} = sum w beta W (bilinear, Eq. 5), and the Poisson solve.
 *
 * Geometry: x in [0, L = nx dx] as in the 1D library (x = 0 a symmetry
 * plane with specular particles, x = L a grounded absorbing wall, the
 * thermal source in the first source_cells cells at any y); y periodic over
 * ny cells with dy = dx.  Nodes (i, j), i = 0..nx, j = 0..ny-1, are stored
 * row-major at i*ny + j.  Units as in slpic.h.  Poisson (eps0 = 1): the
 * five-point stencil, solved exactly by a Fourier transform along y and one
 * tridiagonal solve along x per mode; E = -grad phi by centred differences
 * (periodic in y; E_x = 0 at the symmetry plane, the one-sided second-order
 * difference at the wall).  Phi_w is the y-mean of phi at x = 0.
 *
 * One run per context; its particles are sorted every sort_every steps by
 * blocks of tile x tile cells (stable, dead slots dropped) so that each block
 * is pushed by one workgroup with its node window in LDS.
 *
 * Memory, ownership, errors and threading as in slpic.h: the caller owns one
 * 256-byte aligned device workspace of slpic2d_workspace_bytes() bytes; the
 * library never allocates device memory; every int-returning call returns
 * SLPIC_OK or a negative SLPIC_E* code; device faults (capacity, non-finite
 * velocities) set sticky flags reported by slpic2d_status_query().
 */
#ifndef SLPIC2D_H
#define SLPIC2D_H

#include <stddef.h>
#include <stdint.h>

#include "slpic.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t precision;   /* SLPIC_F32 (int32 fixed-point coordinates, float      */
                         /* velocities) or SLPIC_F64; grids are FP64 in both     */
    int32_t sort_every;  /* tile sort + compaction every k steps; 0 = never      */
    int32_t tile;        /* sort blocks of tile x tile cells, 1..64; 0 = 8;       */
                         /* ceil(nx/tile) * ceil(ny/tile) must not exceed 4096   */
    int32_t margin;      /* cells of the LDS node window beyond a block; 0 =     */
                         /* max(1, sort_every) (with dt <= dx/u no particle      */
                         /* leaves it between two sorts; those that do use the   */
                         /* grid directly)                                       */
    int32_t per_thread;  /* particles per push thread and pass: 1, 2, 4, 8; 0 = 1 */
    int32_t tail_groups; /* workgroups over the unsorted tail; 0 = 512           */
    int32_t sort_tile;   /* slots per sort workgroup, a multiple of 1024 up to   */
                         /* 32768; 0 = 32768                                     */
    int32_t graph_steps; /* > 0: slpic2d_step on a non-default stream replays     */
                         /* blocks of this many steps as one HIP graph (rounded  */
                         /* up to a multiple of sort_every; the graph is         */
                         /* captured on first use); 0 = direct launches          */
    int32_t record_perm; /* 1: every sort also stores its permutation for        */
                         /* slpic2d_export_perm (4 B per slot of workspace); 0 = */
                         /* not stored, slpic2d_export_perm returns SLPIC_EINVAL */
} slpic2d_tuning;

typedef struct {
    int64_t step;              /* completed steps                                   */
    int64_t nslots[2];         /* occupied slots per species (live + dead holes)    */
    int64_t nsorted[2];        /* slots in sorted blocks (the rest is the tail)     */
    int64_t capacity[2];
    int64_t absorbed_total[2];
    int64_t injected_total[2];
    int64_t pushed_total;      /* live particles advanced by push launches          */
    double acc_e;              /* fractional electron injection carried over        */
    double wall_potential;     /* y-mean of phi(0, y) after the last field solve     */
    int32_t error_flags;       /* SLPIC_FLAG_* bits (sticky)                        */
    int32_t fixed_bits;        /* F32: fraction bits of the coordinate fixed point  */
    double weight[2];          /* macroparticle weight per species, dx dy Z / ppc   */
    int64_t steady_step;       /* step count when the wall-potential detector first */
                               /* flagged the run steady (as slpic.h: three window  */
                               /* means of Phi_w within steady_tol of their mean;   */
                               /* steady_window and steady_tol of the run config,   */
                               /* 0 = max(1, nx/4) and 0.02), -1 before             */
    int64_t windows;           /* closed windows                                    */
    double window_mean[3];     /* the last three window means, newest first         */
} slpic2d_status;

/* Bytes of device workspace for one 2D run with ny cells along y (a power of
 * two, 4..2048) and the given tuning (NULL = defaults); run->geometry must be
 * SLPIC_GEOM_SHEATH.  run->nx, dx, dt, u,
 * beta_kind, species, source_cells, seed, run_id and capacity_factor are
 * used as in slpic.h (ppc per cell of dx x dy; warm_profile and
 * limit_profile must be NULL: one uniform limit).
 * Returns 0 on an invalid configuration. */
size_t slpic2d_workspace_bytes(const slpic_run_config* run, int32_t ny, const slpic2d_tuning* tuning);

/* Create a context over the caller's workspace and load the run cold: per
 * slot, x = nx U and y = ny U, then the g0 = f0/beta velocity draws of the
 * 1D loader, weight dx dy Z/ppc; then (if sort_every > 0) the first tile
 * sort, the deposit of rho^0 and the field solve.  Sync on stream. */
int slpic2d_init(const slpic_run_config* run, int32_t ny, const slpic2d_tuning* tuning, void* d_workspace,
                 size_t workspace_bytes, void* stream, void** out_ctx);

/* Advance by nsteps steps: push and deposit, wall absorption, source
 * injection, field solve, Phi_w into the history ring and the steady
 * detector, the periodic tile sort.  Async (HIP-graph replays when
 * tuning.graph_steps > 0 and stream is not the default stream). */
int slpic2d_step(void* ctx, int32_t nsteps, void* stream);

/* beta-weighted moments of f = beta g (Eq. 5) at the current state, to the
 * caller's device buffer d_out of 7 (nx+1) ny doubles: phi, then for species
 * 0 and 1 the density n, the flux Gamma_x = n <v_x> and the kinetic-energy
 * density, each (nx+1) x ny row-major at i*ny + j (bilinear weights with the
 * y wrap, node volume dx dy, halved at the x end nodes).  Async on stream. */
int slpic2d_moments(void* ctx, double* d_out, void* stream);

/* Sync.  Phi_w after each of the last min(step, 4096) steps, oldest first,
 * to h_out (at least 4096 doubles); *n receives the count. */
int slpic2d_wall_history(void* ctx, double* h_out, int64_t* n);

/* Recompute rho from the stored particles and the fields, without pushing.
 * Async. */
int slpic2d_refresh_fields(void* ctx, void* stream);

/* Replace the charge with the caller's device array d_Q (2 x (nx+1) x ny
 * doubles: Q per species, rho = Q/dV) and solve for phi and E.  Async. */
int slpic2d_solve_charge(void* ctx, const double* d_Q, void* stream);

/* Sync.  Copies the last deposited charge per species (h_Q: 2 (nx+1) ny
 * doubles), phi ((nx+1) ny) and E (h_E: 2 (nx+1) ny doubles, E_x then E_y)
 * to host arrays.  Any pointer may be NULL. */
int slpic2d_export_grid(void* ctx, double* h_Q, double* h_phi, double* h_E);

/* Sync.  The nslots occupied slots of one species to host arrays of at least
 * *n doubles: x/dx and y/dy (dead slots have x < 0), v_x, v_y, v_z^2.  On
 * entry *n is the capacity of the arrays, on return the count; SLPIC_EINVAL
 * if they are too small. */
int slpic2d_export_particles(void* ctx, int32_t species, double* h_x, double* h_y, double* h_vx, double* h_vy,
                             double* h_vz2, int64_t* n);

/* Sync.  Replaces the particles of one species with n slots from host arrays
 * (layout of export; F32 coordinates round to the fixed point).  The slots
 * count as unsorted until the next sort; fields are not recomputed. */
int slpic2d_import_particles(void* ctx, int32_t species, const double* h_x, const double* h_y,
                             const double* h_vx, const double* h_vy, const double* h_vz2, int64_t n);

/* Sync.  Sets the step counter (enters the source's Philox counter) and the
 * fractional electron-injection accumulator. */
int slpic2d_set_counters(void* ctx, int64_t step, double acc_e);

/* Run the stable tile sort now.  Async. */
int slpic2d_sort_now(void* ctx, void* stream);

/* Sync.  The permutation of the last sort of one species: h_perm[new] = old
 * slot, *n entries (capacity on entry, count on return). */
int slpic2d_export_perm(void* ctx, int32_t species, int32_t* h_perm, int64_t* n);

/* Sync.  The run status. */
int slpic2d_status_query(void* ctx, slpic2d_status* h_out);

/* Kernel timing with HIP events on the launch stream, as slpic_profile: bit 0
 * push-deposit, bit 1 source injection, bit 2 field solve, bit 3 sort;
 * slpic2d_profile_read (sync) returns summed milliseconds and launch counts
 * per class (arrays of 4) since the last slpic2d_profile call. */
int slpic2d_profile(void* ctx, int32_t enable);
int slpic2d_profile_read(void* ctx, double* h_ms, int64_t* h_launches);

/* Release the context (not the workspace).  Safe on NULL. */
void slpic2d_destroy(void* ctx);

#ifdef __cplusplus
}
#endif
#endif /* SLPIC2D_H */
