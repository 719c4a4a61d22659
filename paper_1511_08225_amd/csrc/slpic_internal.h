// slpic_internal.h -- device-side data layout shared by the library's HIP
// translation units (run table, run state, work tables, kernel arguments).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace slpic {

constexpr int kMaxSpecies = 2;
constexpr int kPurposeLoad = 1;
constexpr int kPurposeInject = 2;
constexpr int kPurposeWarmCount = 3;  // warm load: rounding of a cell's count
constexpr int kPurposeWarm = 4;       // warm load: one particle
constexpr int kPurposeWall = 5;       // plates: a particle entering through x = L
constexpr int kPurposeLimit = 6;      // a new speed limit: the resampling draw of a particle
constexpr int kLimitMaxCopies = 255;  // copies of one g-particle when the speed limit rises
constexpr int kGeomSheath = 0;        // symmetry plane at 0, grounded wall at L
constexpr int kGeomPlates = 1;        // conducting plates at 0 and L (bias)
constexpr int kGeomPeriodic = 2;      // periodic box, no walls, no source
// cells of a 1D run: a moments workgroup keeps 3 FP64 rows of nodes in its
// 64 KiB of LDS (3 * 8 * 2730 bytes)
constexpr int kMaxCells = 2729;
constexpr int kFieldThreads = 1024;   // field solve: threads of the per-run workgroup
constexpr int kFieldTmp = 32;         // field solve: LDS doubles after the node row (two scans' wave totals)
static_assert(2 * (kFieldThreads / 64) <= kFieldTmp, "each scan of the solve keeps its own wave totals");
// field solve: nodes per thread kept in registers (every run's cells fit the
// 1024-thread workgroup; a longer unrolled row would only cost registers)
constexpr int kFieldPer = (kMaxCells + kFieldThreads - 1) / kFieldThreads;
constexpr int kPlatesMaxSource = 511;   // plates: source_cells + 1 nodes fit the injection LDS window
constexpr int kInjectThreads = 128;     // plates: particles per wall-injection workgroup
constexpr int kHistoryLen = 4096;  // wall-potential ring per run
constexpr int kCountSlots = 64;    // spread slots of the per-step particle counters

// Immutable per-run parameters (device copy of the host plan).
struct RunInfo {
    int32_t nx, nodes, beta_kind, source_cells;
    int32_t fb;           // F32: fraction bits of the fixed-point position
    int32_t nkeys;        // sort keys (cells / bucket), at least 1
    int32_t bucket;       // sort key = cell / bucket (0: key 0)
    int32_t uinf;         // 1 if u == +inf (beta == 1)
    double dx, dt, u, u2, dtdx;
    double fscale, inv_fscale;  // 2^fb, 2^-fb
    double qm[kMaxSpecies], qw[kMaxSpecies], w[kMaxSpecies];
    double vt[kMaxSpecies], mass[kMaxSpecies];
    double Ps[kMaxSpecies], Pf[kMaxSpecies], ut[kMaxSpecies];  // loader mixture of Eq. (11b)
    double inj_ratio;     // w_ion / w_electron
    uint32_t seed_lo, seed_hi, run_id, pad0;
    int64_t cap[kMaxSpecies];    // slots per species
    int64_t poff[kMaxSpecies];   // first slot in the global particle arrays
    int64_t nload[kMaxSpecies];  // particles loaded cold
    int64_t goff;                // first node in the global node arrays
    int64_t hoff[kMaxSpecies];   // first entry of the sort histogram of (run, species)
    int32_t ntiles[kMaxSpecies]; // sort tiles of (run, species)
    int32_t chunk0[kMaxSpecies]; // first push chunk of (run, species)
    int32_t nchunk[kMaxSpecies]; // push chunks of (run, species)
    int32_t steady_window;       // steps per wall-potential window
    int32_t warm;                // 1: loaded from predicted profiles (k_load_warm), not cold
    int32_t retire;              // 1: frozen once steady (steady_step >= 0)
    int32_t geom;                // kGeomSheath / kGeomPlates
    double steady_tol;           // relative spread of three window means that counts as steady
    double bias;                 // plates: phi(L)
    double wall_flux[kMaxSpecies];  // plates: g-particles entering per step, per species
    int32_t ppc[kMaxSpecies];    // g-particles per cell at unit density (sets the weight)
    int32_t pruned;              // 1: retired and taken out of the push and sort work (its
                                 // particles then sit identical in both buffers)
    int32_t varlim;              // 1: the speed limit varies with position (node values at goff)
    double umax;                 // the largest speed limit of the run (its profile's largest node)
};

// A new (higher) speed limit for one run: the new limit and the new weights.
struct LimitArgs {
    int32_t run, uinf;
    double u, u2;
    double w[kMaxSpecies];
};

// Mutable per-run state, updated on the device.
struct alignas(64) RunState {
    int64_t nslots[kMaxSpecies];
    int64_t absorbed_step[kMaxSpecies];
    int64_t absorbed_total[kMaxSpecies];
    int64_t injected_total[kMaxSpecies];
    int64_t step;
    int64_t pushed_total;        // live particles advanced by push launches
    double acc_e;
    double phi_w;
    int32_t error;
    int32_t win_n;               // steps in the open wall-potential window
    double win_sum;              // sum of phi_w over the open window
    double win_mean[3];          // the last three closed window means, newest first
    int64_t nwin;                // closed windows
    int64_t steady_step;         // step count when first steady, -1 before
    int64_t msamples;            // moment samples in the window accumulator
    double acc_w[kMaxSpecies];   // plates: fractional wall injection carried over
};

// A run frozen under retire_steady: once its steady detector has flagged it,
// no push, source, field solve or step count.
__host__ __device__ inline bool retired(const RunInfo& R, const RunState& st) {
    return R.retire != 0 && st.steady_step >= 0;
}

// One cell of a warm load: `count` particles of (run, species) at slots
// start.., drawn from a Maxwellian of thermal speed vt drifting at V along x,
// as f/beta with the cell's speed limit u.
struct WarmCell {
    int32_t run, species, cell, count;
    int64_t start;
    double V, vt, u;
};

// A contiguous slot range of one (run, species): one push / load / moments
// workgroup.  begin/end count from the (run, species) first slot, base.
struct Chunk {
    int32_t run, species;
    int64_t begin, end;
    int64_t base;
};

// Particle SoA buffers (double-buffered for the sort); positions are int32
// fixed point (F32) or double (F64), velocities float or double.
struct Bufs {
    void* x[2];
    void* vx[2];
    void* vp2[2];
};

// A sort tile: contiguous slots of one (run, species), its index among the
// tiles of that (run, species).
struct Tile {
    int32_t run, species, index, pad;
    int64_t begin, end;
};

// Kernel arguments shared by every launch (device pointers into the workspace).
struct KArgs {
    const RunInfo* runs;
    RunState* state;
    const Chunk* chunks;
    const Tile* tiles;
    Bufs bufs;
    int* cur;             // which of the two particle buffers is current
    double* E;            // node field, per run at goff
    float* E32;           // float copy of the node field (float particles gather it)
    double* phi;          // node potential
    double* Qacc;         // deposit accumulators [run][species][nodes] at 2*goff
    double* Qlast;        // last step's charge per species, same layout
    double* history;      // wall-potential ring [run][kHistoryLen]
    int* hist;            // sort histogram, per (run, species) at hoff
    int64_t* totals;      // live slots after the sort [run][species]
    int2* counts;         // [run][species][kCountSlots]: (absorbed, pushed) of the last push
    int* push_err;        // [run]: error flags raised by the last push
    int32_t* perm;        // last sort's permutation (new slot -> old slot); scratch of a limit change
    int32_t* sort_perm;   // perm when sorts record their permutation, else null
    double* Macc;         // moment window accumulators [run]: 7 rows of nodes at 7*goff
    const int4* injb;     // plates: wall-injection workgroups (run, species, first particle, 0)
    int32_t ninjb;        // their count (0 without plates runs)
    const double* U;      // speed-limit profiles: node values per run at goff (runs with varlim)
    const float* U32;     // their float copy (float particles' velocity map and move)
};

}  // namespace slpic
