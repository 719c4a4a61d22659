// slpic2d_internal.h -- device-side data layout of the 2D3V library (one
// run: x in [0, nx) between the symmetry plane and the wall, y periodic in
// [0, ny), dy = dx; nodes (i, j), i = 0..nx, j = 0..ny-1, at i*ny + j).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace slpic {

constexpr int kCountSlots2 = 64;  // spread slots of the per-step particle counters
constexpr int kHistoryLen2 = 4096;  // wall-potential ring (the 1D length)

// Immutable run parameters.
struct Run2D {
    int32_t nx, ny, beta_kind, source_cells;
    int32_t fb;            // F32: fraction bits of the fixed-point coordinates
    int32_t uinf;          // 1 if u == +inf (beta == 1)
    int32_t tile;          // sort key: tile x tile blocks of cells
    int32_t ntx, nty, nkeys;
    int32_t margin;        // window margin in cells around a tile
    int32_t win;           // window side in nodes: tile + 2 margin + 1
    int32_t stiles[2];     // sort slot tiles per species
    int32_t sort_tile;     // slots per sort slot tile
    int32_t tile_shift;    // log2(tile) when tile is a power of two, else -1
    double dx, dt, u, u2, dtdx;
    double fscale, inv_fscale;
    double qm[2], qw[2], w[2], vt[2], mass[2], Ps[2], Pf[2], ut[2];
    double inj_ratio;
    uint32_t seed_lo, seed_hi, run_id, pad1;
    int64_t cap[2], poff[2], nload[2];
    int64_t hoff[2];       // first sort histogram entry per species
    int64_t nodes;         // (nx + 1) * ny
    int32_t steady_window; // steps per wall-potential window
    int32_t pad2;
    double steady_tol;     // relative spread of three window means that counts as steady
};

// Mutable run state, on the device.
struct alignas(64) State2D {
    int64_t nslots[2];          // occupied slots (live + dead holes)
    int64_t nsorted[2];         // slots covered by the tile ranges of the last sort
    int64_t absorbed_total[2];
    int64_t injected_total[2];
    int64_t step;
    int64_t pushed_total;
    double acc_e;
    double phi_w;               // y-mean of phi at x = 0 after the last solve
    int32_t error;
    int32_t win_n;              // steps in the open wall-potential window
    int64_t live[2];            // live particles counted by the sort histogram
    double win_sum;             // sum of phi_w over the open window
    double win_mean[3];         // the last three closed window means, newest first
    int64_t nwin;               // closed windows
    int64_t steady_step;        // step count when first steady, -1 before
};

// Source counts of the current step (computed from the push counters).
struct Inject2D {
    int64_t base[2], count[2], absorbed[2];
    int64_t pushed;
    double acc_e;
    int32_t overflow, pad;
};

struct Args2D {
    const Run2D* run;
    State2D* st;
    void* x[2];      // positions: int32 fixed point (F32) or double grid units
    void* y[2];
    void* vx[2];     // velocities: float or double
    void* vy[2];
    void* vz2[2];    // v_z^2 (a constant of the motion: E lies in the x-y plane)
    int* cur;        // which of the two particle buffers is current
    double* Q;       // deposited charge per species [2][nodes]
    double* phi;     // [nodes]
    double2* E;      // (Ex, Ey) [nodes]
    float2* E32;     // float copy of E
    double2* spec;   // y-Fourier modes of the field solve [nx][ny]
    const double* tpiv;  // elimination pivots of the x-system per y-mode [ny/2 + 1][nx]
    const double2* tw;   // exp(-2 pi i k / ny), k < ny/2
    int* hist;       // sort histograms [species][key][slot tile]
    long long* btot; // scan block totals
    int32_t* perm;   // last sort's permutation (new slot -> old slot), per species at poff; null
                     // unless sorts record it
    int64_t* tbeg;   // tile slot ranges after the last sort [2][nkeys + 1]
    int2* counts;    // [2][kCountSlots2]: (absorbed, pushed) of the last push
    Inject2D* inj;
    double* history; // wall-potential ring [kHistoryLen2]
};

}  // namespace slpic
