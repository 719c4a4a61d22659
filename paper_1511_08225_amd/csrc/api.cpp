// api.cpp -- the C ABI of include/slpic.h: run planning (run table, work
// tables, workspace layout), cold start, stepping with optional HIP-graph
// replay, sort scheduling, state import/export and event timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "slpic.h"
#include "host_math.h"
#include "launch.h"
#include "slpic_device.h"
#include "slpic_internal.h"

using namespace slpic;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// ---------------------------------------------------------------------------
// Warm load planning.  For cell c of species s: n and Gamma linearly
// interpolated from the 256-point profiles (x/L = k/255) at the cell centre,
// n clamped at 0, drift V = Gamma/n clamped to |V| <= 4 vt; the expected
// g-particle count is E = n dx Z / w with Z = <1/beta> over the Maxwellian
// drifting at V (f = beta g, Eq. 5), rounded up with probability frac(E)
// by the cell's Philox uniform.
// ---------------------------------------------------------------------------
struct GaussLegendre {
    static constexpr int n = 64;
    double x[n], w[n];  // on [-1, 1]
    GaussLegendre() {
        for (int i = 0; i < n; ++i) {
            double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = z;  // Legendre recurrence to P_n and its derivative
                for (int k = 2; k <= n; ++k) {
                    double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = pk;
                }
                dp = n * (z * p1 - p0) / (z * z - 1.0);
                const double dz = p1 / dp;
                z -= dz;
                if (std::fabs(dz) < 1e-16) break;
            }
            x[i] = z;
            w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
    }
};

// Density of |v| for v = V e_x + vt z, z standard normal in 3D (V -> 0: Maxwell).
static double drift_speed_pdf(double sp, double V, double vt) {
    const double g = sp / (vt * std::sqrt(2.0 * M_PI)) * std::exp(-(sp - V) * (sp - V) / (2.0 * vt * vt));
    const double q = 2.0 * sp * V / (vt * vt);
    return g * (q > 1e-300 ? -std::expm1(-q) / V : 2.0 * sp / (vt * vt));
}

// <1/beta> over the Maxwellian drifting at V: 64-point Gauss-Legendre in the
// speed on [lo, |V| + 12 vt] (lo = u for Eq. 11b, whose integrand is 1 below u).
static double drift_mean_inv_beta(int kind, double u, double V, double vt) {
    static const GaussLegendre gl;
    if (std::isinf(u)) return 1.0;
    V = std::fabs(V);
    const double hi = V + 12.0 * vt;
    const double lo = kind == SLPIC_BETA_STEP ? u : 0.0;
    if (lo >= hi) return 1.0;
    const double half = 0.5 * (hi - lo), mid = 0.5 * (hi + lo);
    double acc = 0.0;
    for (int i = 0; i < gl.n; ++i) {
        const double sp = mid + half * gl.x[i];
        const double f = kind == SLPIC_BETA_STEP ? sp / u - 1.0 : std::sqrt(1.0 + (sp / u) * (sp / u));
        acc += gl.w[i] * f * drift_speed_pdf(sp, V, vt);
    }
    acc *= half;
    return kind == SLPIC_BETA_STEP ? 1.0 + acc : acc;
}

static double profile_at(const double* p, double xi) {
    const double t = xi * 255.0;
    int k = (int)std::floor(t);
    k = std::max(0, std::min(254, k));
    const double f = t - (double)k;
    return p[k] * (1.0 - f) + p[k + 1] * f;
}

// Cells of one (run, species) loaded from the profiles prof (7 x 256),
// appended to out; returns the particle count.  A run with a limit profile
// samples each cell at the limit of its centre (the mean of its two nodes).
static int64_t plan_warm_species(const RunInfo& R, const slpic_run_config& c, const double* prof, int run, int s,
                                 std::vector<WarmCell>& out) {
    const double* pn = prof + 256 * (s == 0 ? 1 : 2);
    const double* pg = prof + 256 * (s == 0 ? 3 : 4);
    const double* pT = prof + 256 * (5 + s);
    const double* lim = c.limit_profile;
    int64_t start = 0;
    for (int cell = 0; cell < c.nx; ++cell) {
        const double uc = lim ? 0.5 * (lim[cell] + lim[cell + 1]) : c.u;
        const double xi = ((double)cell + 0.5) / (double)c.nx;
        const double T = profile_at(pT, xi);  // not positive: the source temperature
        const double vt = T > 0.0 ? std::sqrt(T / R.mass[s]) : R.vt[s];
        double n = profile_at(pn, xi);
        if (!(n > 0.0)) n = 0.0;
        const double G = profile_at(pg, xi);
        double V = n > 0.0 ? G / n : 0.0;
        V = std::max(-4.0 * vt, std::min(4.0 * vt, V));
        const double E = n * c.dx * drift_mean_inv_beta(c.beta_kind, uc, V, vt) / R.w[s];
        const double fl = std::floor(E);
        const U4 r = philox10((uint32_t)cell, 0u, R.run_id, ((uint32_t)kPurposeWarmCount << 24) | ((uint32_t)s << 20),
                              R.seed_lo, R.seed_hi);
        const int64_t cnt = (int64_t)fl + (u53(r.v[0], r.v[1]) < E - fl ? 1 : 0);
        if (cnt > 0) out.push_back(WarmCell{run, s, cell, (int32_t)cnt, start, V, vt, uc});
        start += cnt;
    }
    return start;
}

int ceil_log2(int64_t v) {
    int b = 0;
    while ((int64_t(1) << b) < v) ++b;
    return b;
}

struct Layout {
    size_t runs, state, chunks, tiles, cur, x[2], vx[2], vp2[2], perm, E, E32, phi, Qacc, Qlast, hist,
        totals, counts, push_err, Macc, btot, history, injb, active, U, U32, total;
};

struct Plan {
    int nruns = 0;
    slpic_tuning tun{};
    std::vector<RunInfo> runs;
    std::vector<Chunk> chunks;
    std::vector<int> run_chunk0, run_nchunks;
    std::vector<Tile> tiles;
    std::vector<WarmCell> warm_cells;
    std::vector<int4> injb;  // plates: wall-injection workgroups (run, species, first particle, 0)
    int64_t total_slots = 0, total_nodes = 0, hist_entries = 0;
    int max_nodes = 0, max_src = 0, max_nkeys = 0;
    bool all_sheath = true;  // no plates or periodic run: the push without their paths
    bool any_varlim = false; // a run with a limit profile: the push that reads the profiles
    std::vector<double> limit_nodes;  // every run's limit at its nodes (at goff)
    Layout L{};
};

int make_plan(const slpic_run_config* cfg, int nruns, const slpic_tuning* tin, Plan& P) {
    if (!cfg || nruns < 1) return SLPIC_EINVAL;
    slpic_tuning t{};
    if (tin) t = *tin;
    if (t.precision != SLPIC_F32 && t.precision != SLPIC_F64) return SLPIC_EINVAL;
    if (t.sort_every < 0 || t.sort_bucket < 0 || t.chunk < 0 || t.block < 0 || t.graph_steps < 0 ||
        t.sort_tile < 0 || (t.retire_steady != 0 && t.retire_steady != 1) ||
        (t.push_order != 0 && t.push_order != 1) || (t.record_perm != 0 && t.record_perm != 1))
        return SLPIC_EINVAL;
    if (t.block == 0) t.block = 128;
    if (t.chunk == 0) t.chunk = 64 * (t.precision == SLPIC_F32 ? 8 : 4);
    if (t.sort_tile == 0) t.sort_tile = 16384;
    // the scatter keeps per-wave offsets within a tile's run of one key in 16 bits
    if (t.sort_tile > 32768) return SLPIC_EINVAL;
    if (t.block < 64 || t.block > 256 || t.block % 64) return SLPIC_EINVAL;  // 1..4 push waves
    {   // one wavefront per push chunk: chunk = 64 * P, P in {1, 2, 4, 8, 16}
        const int per = t.chunk / 64;
        if (t.chunk % 64 || (per != 1 && per != 2 && per != 4 && per != 8 && per != 16)) return SLPIC_EINVAL;
    }
    if (t.sort_every > 0 && t.graph_steps > 0 && t.graph_steps % t.sort_every)
        t.graph_steps = (t.graph_steps / t.sort_every + 1) * t.sort_every;
    P.tun = t;
    P.nruns = nruns;
    P.runs.assign(nruns, RunInfo{});
    int64_t poff = 0, goff = 0, hoff = 0;
    for (int r = 0; r < nruns; ++r) {
        const slpic_run_config& c = cfg[r];
        if (c.nx < 4 || c.nx > kMaxCells || !(c.dx > 0) || !(c.dt > 0) || !(c.u > 0) || c.nspecies != 2 ||
            c.source_cells < 1 || c.source_cells > c.nx ||
            (c.beta_kind != SLPIC_BETA_STEP && c.beta_kind != SLPIC_BETA_SMOOTH))
            return SLPIC_EINVAL;
        const bool plates = c.geometry == SLPIC_GEOM_PLATES, periodic = c.geometry == SLPIC_GEOM_PERIODIC;
        if ((c.geometry != SLPIC_GEOM_SHEATH && !plates && !periodic) ||
            (plates && (c.warm_profile || c.source_cells > kPlatesMaxSource || !std::isfinite(c.bias))) ||
            (periodic && c.warm_profile))
            return SLPIC_EINVAL;
        double umax = c.u;
        if (c.limit_profile) {  // finite positive nodes, a finite u for the weights
            if (!std::isfinite(c.u)) return SLPIC_EINVAL;
            umax = 0.0;
            for (int j = 0; j <= c.nx; ++j) {
                const double v = c.limit_profile[j];
                if (!(v > 0.0) || !std::isfinite(v)) return SLPIC_EINVAL;
                umax = std::max(umax, v);
            }
            P.any_varlim = true;
        }
        RunInfo& R = P.runs[r];
        R.varlim = c.limit_profile ? 1 : 0;
        R.umax = umax;
        R.nx = c.nx;
        R.nodes = c.nx + 1;
        R.beta_kind = c.beta_kind;
        R.source_cells = c.source_cells;
        R.fb = std::min(24, 31 - ceil_log2((int64_t)c.nx + 1));
        R.bucket = t.sort_bucket;
        R.nkeys = t.sort_bucket > 0 ? (c.nx + t.sort_bucket - 1) / t.sort_bucket : 1;
        R.uinf = std::isinf(c.u) ? 1 : 0;
        R.dx = c.dx;
        R.dt = c.dt;
        R.u = c.u;
        R.u2 = c.u * c.u;
        R.dtdx = c.dt / c.dx;
        R.fscale = std::ldexp(1.0, R.fb);
        R.inv_fscale = std::ldexp(1.0, -R.fb);
        R.seed_lo = (uint32_t)(c.seed & 0xffffffffu);
        R.seed_hi = (uint32_t)(c.seed >> 32);
        R.run_id = (uint32_t)c.run_id;
        double cf = c.capacity_factor > 1.0 ? c.capacity_factor : 1.0;
        for (int s = 0; s < 2; ++s) {
            const slpic_species& sp = c.species[s];
            if (!(sp.mass > 0) || !(sp.temperature > 0) || sp.ppc < 1) return SLPIC_EINVAL;
            R.vt[s] = std::sqrt(sp.temperature / sp.mass);
            R.mass[s] = sp.mass;
            R.ut[s] = c.u / R.vt[s];
            double Z = mean_inv_beta(c.beta_kind, R.ut[s]);
            R.w[s] = c.dx * Z / (double)sp.ppc;
            R.qw[s] = sp.charge * R.w[s];
            R.qm[s] = sp.charge / sp.mass;
            if (R.uinf) {
                R.Ps[s] = 1.0;
                R.Pf[s] = 0.0;
            } else {
                step_mixture(R.ut[s], R.Ps[s], R.Pf[s]);
            }
            R.ppc[s] = sp.ppc;
            R.nload[s] = plates ? 0 : (int64_t)c.nx * sp.ppc;  // plates: the box starts empty
            // plates: the one-sided flux v_t / sqrt(2 pi) of unit density, in g-particles per step
            R.wall_flux[s] = plates ? R.vt[s] / std::sqrt(2.0 * M_PI) * c.dt / R.w[s] : 0.0;
            if (c.warm_profile || (c.limit_profile && !plates)) {
                // a limit profile loads cold cell by cell: unit density at rest,
                // the source temperatures (rows of zeros)
                static const std::vector<double> rest = [] {
                    std::vector<double> p(7 * 256, 0.0);
                    for (int k = 0; k < 256; ++k) p[256 + k] = p[512 + k] = 1.0;
                    return p;
                }();
                R.warm = 1;
                const int64_t nw =
                    plan_warm_species(R, c, c.warm_profile ? c.warm_profile : rest.data(), r, s, P.warm_cells);
                if (nw > ((int64_t)1 << 31) - 65) return SLPIC_ECAPACITY;
                R.cap[s] = std::max<int64_t>((int64_t)std::ceil(cf * (double)R.nload[s]), nw + 64);
                R.nload[s] = nw;
            } else {
                const int64_t nref = (int64_t)c.nx * sp.ppc;  // slots sized on the load density
                R.cap[s] = std::max<int64_t>((int64_t)std::ceil(cf * (double)nref), R.nload[s] + 64);
            }
            if (R.cap[s] > (int64_t(1) << 31) - 1) return SLPIC_EINVAL;
            R.poff[s] = poff;
            poff += R.cap[s];
            R.ntiles[s] = (int32_t)((R.cap[s] + t.sort_tile - 1) / t.sort_tile);
            R.hoff[s] = hoff;
            hoff += (int64_t)R.nkeys * R.ntiles[s];
        }
        R.inj_ratio = R.w[1] / R.w[0];
        R.geom = plates ? kGeomPlates : periodic ? kGeomPeriodic : kGeomSheath;
        if (plates || periodic) P.all_sheath = false;
        R.bias = plates ? c.bias : 0.0;
        if (c.steady_window < 0 || !(c.steady_tol >= 0.0)) return SLPIC_EINVAL;
        R.steady_window = c.steady_window > 0 ? c.steady_window : std::max(1, c.nx / 4);
        R.steady_tol = c.steady_tol > 0.0 ? c.steady_tol : 0.02;
        R.retire = t.retire_steady ? 1 : 0;
        R.goff = goff;
        goff += R.nodes;
        for (int j = 0; j <= c.nx; ++j) P.limit_nodes.push_back(c.limit_profile ? c.limit_profile[j] : c.u);
        P.max_nodes = std::max(P.max_nodes, R.nodes);
        P.max_src = std::max(P.max_src, c.source_cells + 1);
        P.max_nkeys = std::max(P.max_nkeys, R.nkeys);
    }
    if (poff > (int64_t(1) << 31) - 1) return SLPIC_EINVAL;  // sort offsets are int32
    P.total_slots = poff;
    P.total_nodes = goff;
    P.hist_entries = hoff;
    P.run_chunk0.assign(nruns, 0);
    P.run_nchunks.assign(nruns, 0);
    for (int r = 0; r < nruns; ++r) {
        P.run_chunk0[r] = (int)P.chunks.size();
        for (int s = 0; s < 2; ++s) {
            RunInfo& R = P.runs[r];
            R.chunk0[s] = (int32_t)P.chunks.size();
            for (int64_t b = 0; b < R.cap[s]; b += t.chunk)
                P.chunks.push_back(Chunk{r, s, b, std::min<int64_t>(b + t.chunk, R.cap[s]), R.poff[s]});
            R.nchunk[s] = (int32_t)P.chunks.size() - R.chunk0[s];
            for (int k = 0; k < R.ntiles[s]; ++k) {
                int64_t b = (int64_t)k * t.sort_tile;
                P.tiles.push_back(Tile{r, s, k, 0, b, std::min<int64_t>(b + t.sort_tile, R.cap[s])});
            }
        }
        P.run_nchunks[r] = (int)P.chunks.size() - P.run_chunk0[r];
    }
    // plates: the wall injection of a step (at most floor(wall_flux) + 1
    // particles per species), kInjectThreads particles per workgroup
    for (int r = 0; r < nruns; ++r) {
        const RunInfo& R = P.runs[r];
        if (R.geom != kGeomPlates) continue;
        for (int s = 0; s < 2; ++s) {
            const double most = std::floor(R.wall_flux[s]) + 1.0;
            if (!(most < 1e9)) return SLPIC_EINVAL;
            for (int64_t k = 0; k < (int64_t)most; k += kInjectThreads) P.injb.push_back(int4{r, s, (int)k, 0});
        }
    }
    if (P.injb.size() > (size_t)1 << 20) return SLPIC_EINVAL;
    const size_t psz = t.precision == SLPIC_F32 ? 4 : 8;  // int32 fixed point or double
    const size_t vsz = t.precision == SLPIC_F32 ? 4 : 8;
    Layout& L = P.L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + std::max<size_t>(bytes, 1));
        return at;
    };
    L.runs = take(sizeof(RunInfo) * nruns);
    L.state = take(sizeof(RunState) * nruns);
    L.chunks = take(sizeof(Chunk) * P.chunks.size());
    L.tiles = take(sizeof(Tile) * P.tiles.size());
    L.cur = take(sizeof(int));
    for (int b = 0; b < 2; ++b) {
        L.x[b] = take(psz * P.total_slots);
        L.vx[b] = take(vsz * P.total_slots);
        L.vp2[b] = take(vsz * P.total_slots);
    }
    L.perm = take(sizeof(int32_t) * P.total_slots);
    L.E = take(sizeof(double) * P.total_nodes);
    L.E32 = take(sizeof(float) * P.total_nodes);
    L.phi = take(sizeof(double) * P.total_nodes);
    L.Qacc = take(sizeof(double) * 2 * P.total_nodes);
    L.Qlast = take(sizeof(double) * 2 * P.total_nodes);
    L.hist = take(sizeof(int) * P.hist_entries);
    L.totals = take(sizeof(int64_t) * 2 * nruns);
    L.counts = take(sizeof(int2) * kMaxSpecies * kCountSlots * nruns);
    L.push_err = take(sizeof(int) * nruns);
    L.Macc = take(sizeof(double) * 7 * P.total_nodes);
    // block totals of the scans: the sort histogram, or one count per slot
    // (speed-limit resampling)
    L.btot = take(sizeof(long long) * (scan_blocks(std::max<int64_t>(P.hist_entries, P.total_slots)) + 1));
    L.history = take(sizeof(double) * kHistoryLen * nruns);
    L.injb = take(sizeof(int4) * P.injb.size());
    L.active = take(sizeof(Chunk) * P.chunks.size());  // the push's chunks: runs not pruned
    L.U = take(P.any_varlim ? sizeof(double) * P.total_nodes : 0);
    L.U32 = take(P.any_varlim ? sizeof(float) * P.total_nodes : 0);
    L.total = o;
    return SLPIC_OK;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
};

struct Context {
    Plan P;
    KArgs a{};
    unsigned char* ws = nullptr;
    long long* btot = nullptr;
    int64_t steps_done = 0;
    size_t field_lds = 0, source_field_lds = 0, sort_lds = 0, moments_lds = 0;
    size_t scatter_lds = 0;  // four waves' packed per-key offsets
    // threads of the per-run source + field workgroup (fewer waves helped the
    // 100-cell plates step by ~5 % but slowed the 2048-cell sheath by 10-20 %)
    int field_threads = kFieldThreads;
    hipGraphExec_t gexec = nullptr;
    int graph_len = 0;
    bool prof = false;
    int prof_mask = 0;  // kernel classes timed: bit k = class k
    std::vector<EventPair> ev[4];
    size_t ev_used[4] = {0, 0, 0, 0};
    int sample_every = 0;  // in-step moment sampling period (0: off)
    Chunk* active = nullptr;  // device: the chunks of runs not pruned (the push's work)
    int n_active = 0;
    std::vector<Chunk> active_host;  // its host copy (the source of the asynchronous upload)
    ~Context() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        for (auto& v : ev)
            for (auto& e : v) {
                if (e.a) (void)hipEventDestroy(e.a);
                if (e.b) (void)hipEventDestroy(e.b);
            }
    }
};

#define HIP_TRY(x)                                  \
    do {                                            \
        if ((x) != hipSuccess) return SLPIC_EHIP;   \
    } while (0)

int prec(const Context* c) { return c->P.tun.precision; }

void l_load(Context* c, hipStream_t s) {
    if (prec(c) == SLPIC_F32) launch_load_f32(c->a, (int)c->P.chunks.size(), 256, s);
    else launch_load_f64(c->a, (int)c->P.chunks.size(), 256, s);
}
// A pushing launch covers the chunks of the runs not pruned; a deposit-only
// launch (refresh) every chunk.
void l_push(Context* c, bool push, hipStream_t s) {
    const int per = c->P.tun.chunk / 64;
    const Chunk* ch = push ? c->active : c->a.chunks;
    const int n = push ? c->n_active : (int)c->P.chunks.size();
    if (prec(c) == SLPIC_F32)
        launch_push_f32(push, c->P.all_sheath, c->P.any_varlim, per, c->a, ch, n, c->P.tun.block, s);
    else
        launch_push_f64(push, c->P.all_sheath, c->P.any_varlim, per, c->a, ch, n, c->P.tun.block, s);
}
void l_wall_inject(Context* c, hipStream_t s) {
    if (prec(c) == SLPIC_F32) launch_wall_inject_f32(c->a, s);
    else launch_wall_inject_f64(c->a, s);
}
void l_source_field(Context* c, hipStream_t s) {
    if (prec(c) == SLPIC_F32) launch_source_field_f32(c->a, c->P.nruns, c->field_threads, c->source_field_lds, s);
    else launch_source_field_f64(c->a, c->P.nruns, c->field_threads, c->source_field_lds, s);
}

// timed launch wrapper: class k in {0 push, 1 source (inside the field launch), 2 field, 3 sort}
template <typename F>
int timed(Context* c, int k, hipStream_t s, F&& f) {
    if (!c->prof || !((c->prof_mask >> k) & 1)) {
        f();
        return hipGetLastError() == hipSuccess ? SLPIC_OK : SLPIC_EHIP;
    }
    if (c->ev_used[k] == c->ev[k].size()) {
        EventPair e;
        HIP_TRY(hipEventCreate(&e.a));
        HIP_TRY(hipEventCreate(&e.b));
        c->ev[k].push_back(e);
    }
    EventPair& e = c->ev[k][c->ev_used[k]++];
    HIP_TRY(hipEventRecord(e.a, s));
    f();
    HIP_TRY(hipEventRecord(e.b, s));
    return hipGetLastError() == hipSuccess ? SLPIC_OK : SLPIC_EHIP;
}

int do_sort(Context* c, hipStream_t s) {
    const int nt = (int)c->P.tiles.size();
    return timed(c, 3, s, [&] {
        // the (key, tile) counts start at zero: a tile writes only the keys it holds
        launch_zero_ints(c->a.hist, c->P.hist_entries, s);
        if (prec(c) == SLPIC_F32) launch_sort_hist_f32(c->a, nt, 256, c->sort_lds, s);
        else launch_sort_hist_f64(c->a, nt, 256, c->sort_lds, s);
        // both sort kernels run four waves per tile: scatter_lds is sized for them
        launch_sort_scan(c->a, c->P.hist_entries, c->btot, s);
        if (prec(c) == SLPIC_F32) launch_sort_scatter_f32(c->a, nt, 256, c->scatter_lds, s);
        else launch_sort_scatter_f64(c->a, nt, 256, c->scatter_lds, s);
        launch_sort_finish(c->a, c->P.nruns, c->P.hist_entries, c->btot, s);
    });
}

// One leapfrog step of every run; `local_step` decides the sort.
// The moments of every run added to their device windows (slpic_moments_sample).
void sample_all(Context* c, hipStream_t s) {
    if (prec(c) == SLPIC_F32)
        launch_moments_f32(c->a, 0, (int)c->P.chunks.size(), 256, c->moments_lds, c->a.Macc, 1, s);
    else
        launch_moments_f64(c->a, 0, (int)c->P.chunks.size(), 256, c->moments_lds, c->a.Macc, 1, s);
    launch_moments_sample_finish(c->a, 0, c->P.nruns, s);
}

int one_step(Context* c, int64_t local_step, hipStream_t s) {
    int rc;
    if (c->a.ninjb > 0 && (rc = timed(c, 1, s, [&] { l_wall_inject(c, s); }))) return rc;
    if ((rc = timed(c, 0, s, [&] { l_push(c, true, s); }))) return rc;
    if ((rc = timed(c, 2, s, [&] { l_source_field(c, s); }))) return rc;
    const int se = c->P.tun.sort_every;
    if (se > 0 && (local_step + 1) % se == 0)
        if ((rc = do_sort(c, s))) return rc;
    if (c->sample_every > 0 && (local_step + 1) % c->sample_every == 0) sample_all(c, s);
    return SLPIC_OK;
}

// Capture graph_steps steps into *out (with event records when profiling).
int capture_steps(Context* c, hipStream_t s, hipGraphExec_t* out) {
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    int rc = SLPIC_OK;
    for (int k = 0; k < c->P.tun.graph_steps && rc == SLPIC_OK; ++k) rc = one_step(c, k, s);
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc != SLPIC_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return rc != SLPIC_OK ? rc : SLPIC_EHIP;
    }
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        *out = nullptr;
        return SLPIC_EHIP;
    }
    return SLPIC_OK;
}

int build_graph(Context* c, hipStream_t s) {
    int rc = capture_steps(c, s, &c->gexec);
    if (rc == SLPIC_OK) c->graph_len = c->P.tun.graph_steps;
    return rc;
}

Context* ctx_of(void* p) { return static_cast<Context*>(p); }

// Both particle buffers of (run) hold the current one's slots.
// The push launch's chunk table: the chunks of the runs not pruned, run by
// run.  push_order 0 keeps the plan's order (each species' chunks in slot
// order); 1 interleaves a run's two species by first slot (a stable sort on
// (run, first slot)): electron and ion chunks cost different arithmetic, and
// alternating them spreads each kind over the launch, which pays when the
// whole launch is about one round of resident wavefronts; with many rounds
// the plan's order, whose neighbouring wavefronts share memory regions, is
// faster.  Either way a run's chunks past the occupied slots, which return
// at once, come after its live ones.
std::vector<Chunk> push_order(const Plan& P) {
    std::vector<Chunk> act;
    act.reserve(P.chunks.size());
    for (const Chunk& ch : P.chunks)
        if (!P.runs[ch.run].pruned) act.push_back(ch);
    if (P.tun.push_order == 1)
        std::stable_sort(act.begin(), act.end(), [](const Chunk& x, const Chunk& y) {
            return x.run != y.run ? x.run < y.run : x.begin < y.begin;
        });
    return act;
}

int mirror_run(Context* c, int run, hipStream_t s) {
    const RunInfo& R = c->P.runs[run];
    int b = 0;
    HIP_TRY(hipMemcpy(&b, c->a.cur, sizeof(int), hipMemcpyDeviceToHost));
    const size_t esz = prec(c) == SLPIC_F32 ? 4 : 8;
    for (int sp = 0; sp < 2; ++sp) {
        const size_t off = (size_t)R.poff[sp] * esz, bytes = (size_t)R.cap[sp] * esz;
        HIP_TRY(hipMemcpyAsync((char*)c->a.bufs.x[b ^ 1] + off, (char*)c->a.bufs.x[b] + off, bytes,
                               hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync((char*)c->a.bufs.vx[b ^ 1] + off, (char*)c->a.bufs.vx[b] + off, bytes,
                               hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync((char*)c->a.bufs.vp2[b ^ 1] + off, (char*)c->a.bufs.vp2[b] + off, bytes,
                               hipMemcpyDeviceToDevice, s));
    }
    return SLPIC_OK;
}

// The synchronous copies of the "sync" calls wait for the whole device
// first: work enqueued on a non-blocking stream is not ordered with the
// default stream that hipMemcpy uses.
int copy_d2h(void* dst, const void* src, size_t bytes) {
    if (!bytes) return SLPIC_OK;
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
    return SLPIC_OK;
}
int copy_h2d(void* dst, const void* src, size_t bytes) {
    if (!bytes) return SLPIC_OK;
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    return SLPIC_OK;
}

}  // namespace

extern "C" {

size_t slpic_workspace_bytes(const slpic_run_config* runs, int32_t nruns, const slpic_tuning* tuning) {
    Plan P;
    if (make_plan(runs, nruns, tuning, P) != SLPIC_OK) return 0;
    return P.L.total;
}

int slpic_init(const slpic_run_config* runs, int32_t nruns, const slpic_tuning* tuning, void* d_workspace,
               size_t workspace_bytes, void* stream, void** out_ctx) {
    if (!out_ctx) return SLPIC_EINVAL;
    *out_ctx = nullptr;
    Context* c = new (std::nothrow) Context();
    if (!c) return SLPIC_ENOMEM;
    int rc = make_plan(runs, nruns, tuning, c->P);
    if (rc) {
        delete c;
        return rc;
    }
    if (!d_workspace || ((uintptr_t)d_workspace % kAlign) != 0) {
        delete c;
        return SLPIC_EINVAL;
    }
    if (workspace_bytes < c->P.L.total) {
        delete c;
        return SLPIC_ENOMEM;
    }
    hipStream_t s = (hipStream_t)stream;
    unsigned char* w = (unsigned char*)d_workspace;
    const Layout& L = c->P.L;
    c->ws = w;
    KArgs& a = c->a;
    a.runs = (const RunInfo*)(w + L.runs);
    a.state = (RunState*)(w + L.state);
    a.chunks = (const Chunk*)(w + L.chunks);
    a.tiles = (const Tile*)(w + L.tiles);
    a.cur = (int*)(w + L.cur);
    for (int b = 0; b < 2; ++b) {
        a.bufs.x[b] = w + L.x[b];
        a.bufs.vx[b] = w + L.vx[b];
        a.bufs.vp2[b] = w + L.vp2[b];
    }
    a.perm = (int32_t*)(w + L.perm);
    a.sort_perm = c->P.tun.record_perm ? a.perm : nullptr;
    a.E = (double*)(w + L.E);
    a.E32 = (float*)(w + L.E32);
    a.phi = (double*)(w + L.phi);
    a.Qacc = (double*)(w + L.Qacc);
    a.Qlast = (double*)(w + L.Qlast);
    a.hist = (int*)(w + L.hist);
    a.totals = (int64_t*)(w + L.totals);
    a.counts = (int2*)(w + L.counts);
    a.push_err = (int*)(w + L.push_err);
    a.Macc = (double*)(w + L.Macc);
    a.history = (double*)(w + L.history);
    a.injb = (const int4*)(w + L.injb);
    a.ninjb = (int32_t)c->P.injb.size();
    a.U = c->P.any_varlim ? (const double*)(w + L.U) : nullptr;
    a.U32 = c->P.any_varlim ? (const float*)(w + L.U32) : nullptr;
    c->active = (Chunk*)(w + L.active);
    c->n_active = (int)c->P.chunks.size();
    c->btot = (long long*)(w + L.btot);
    c->field_lds = (size_t)(c->P.max_nodes + kFieldTmp) * 8;
    c->sort_lds = (size_t)c->P.max_nkeys * sizeof(int);  // the tile's key counts
    c->scatter_lds = (size_t)4 * ((c->P.max_nkeys + 1) / 2) * sizeof(uint32_t);
    c->source_field_lds = c->field_lds + (size_t)2 * c->P.max_src * 8;

    c->moments_lds = (size_t)3 * c->P.max_nodes * 8;
    if (c->sort_lds > 65536 || c->scatter_lds > 65536 || c->moments_lds > 65536 || c->source_field_lds > 65536) {
        delete c;
        return SLPIC_EINVAL;
    }
#define INIT_TRY(x)              \
    do {                         \
        int r_ = (x);            \
        if (r_) {                \
            delete c;            \
            return r_;           \
        }                        \
    } while (0)
    INIT_TRY(hipMemcpyAsync((void*)a.runs, c->P.runs.data(), sizeof(RunInfo) * nruns, hipMemcpyHostToDevice, s)
                 ? SLPIC_EHIP : SLPIC_OK);
    INIT_TRY(hipMemcpyAsync((void*)a.chunks, c->P.chunks.data(), sizeof(Chunk) * c->P.chunks.size(),
                            hipMemcpyHostToDevice, s) ? SLPIC_EHIP : SLPIC_OK);
    INIT_TRY(hipMemcpyAsync((void*)a.tiles, c->P.tiles.data(), sizeof(Tile) * c->P.tiles.size(),
                            hipMemcpyHostToDevice, s) ? SLPIC_EHIP : SLPIC_OK);
    c->active_host = push_order(c->P);
    INIT_TRY(hipMemcpyAsync((void*)c->active, c->active_host.data(), sizeof(Chunk) * c->active_host.size(),
                            hipMemcpyHostToDevice, s) ? SLPIC_EHIP : SLPIC_OK);
    if (!c->P.injb.empty())
        INIT_TRY(hipMemcpyAsync((void*)a.injb, c->P.injb.data(), sizeof(int4) * c->P.injb.size(),
                                hipMemcpyHostToDevice, s) ? SLPIC_EHIP : SLPIC_OK);
    std::vector<float> u32;
    if (c->P.any_varlim) {  // the limit profiles (pageable copies: synchronised before init returns)
        u32.assign(c->P.limit_nodes.begin(), c->P.limit_nodes.end());
        INIT_TRY(hipMemcpyAsync((void*)a.U, c->P.limit_nodes.data(), sizeof(double) * c->P.total_nodes,
                                hipMemcpyHostToDevice, s) ? SLPIC_EHIP : SLPIC_OK);
        INIT_TRY(hipMemcpyAsync((void*)a.U32, u32.data(), sizeof(float) * c->P.total_nodes, hipMemcpyHostToDevice,
                                s) ? SLPIC_EHIP : SLPIC_OK);
    }
    launch_init_state(a, nruns, s);
    launch_zero(a.Qacc, 2 * c->P.total_nodes, s);
    launch_zero(a.Macc, 7 * c->P.total_nodes, s);
    launch_zero(a.Qlast, 2 * c->P.total_nodes, s);
    launch_zero(a.E, c->P.total_nodes, s);
    launch_zero(a.phi, c->P.total_nodes, s);
    launch_zero(a.history, (int64_t)kHistoryLen * nruns, s);
    l_load(c, s);
    if (!c->P.warm_cells.empty()) {
        // the table goes to the second particle buffer, unused until the first sort
        const size_t tb = sizeof(WarmCell) * c->P.warm_cells.size();
        const size_t room = (size_t)c->P.total_slots * (c->P.tun.precision == SLPIC_F32 ? 4 : 8);
        if (tb > room) {
            delete c;
            return SLPIC_ENOMEM;
        }
        void* d_cells = w + L.x[1];
        INIT_TRY(hipMemcpyAsync(d_cells, c->P.warm_cells.data(), tb, hipMemcpyHostToDevice, s) ? SLPIC_EHIP
                                                                                               : SLPIC_OK);
        if (prec(c) == SLPIC_F32) launch_load_warm_f32(a, d_cells, (int)c->P.warm_cells.size(), s);
        else launch_load_warm_f64(a, d_cells, (int)c->P.warm_cells.size(), s);
    }
    if (c->P.tun.sort_every > 0) INIT_TRY(do_sort(c, s));
    l_push(c, false, s);
    launch_field(a, nruns, 0, c->field_lds, s);
    INIT_TRY(hipGetLastError() == hipSuccess ? SLPIC_OK : SLPIC_EHIP);
    INIT_TRY(hipStreamSynchronize(s) == hipSuccess ? SLPIC_OK : SLPIC_EHIP);
#undef INIT_TRY
    *out_ctx = c;
    return SLPIC_OK;
}

int slpic_step(void* ctx, int32_t nsteps, void* stream) {
    Context* c = ctx_of(ctx);
    if (!c || nsteps < 0) return SLPIC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int se = c->P.tun.sort_every;
    // graphs on a non-default stream; profiled steps launch directly (event
    // timings of graph-recorded events are not available)
    const bool graphs = c->P.tun.graph_steps > 0 && s != nullptr && !c->prof;
    int32_t done = 0;
    while (done < nsteps) {
        const int gl = c->P.tun.graph_steps;
        if (graphs && nsteps - done >= gl && (se == 0 || c->steps_done % se == 0) &&
            (c->sample_every == 0 || c->steps_done % c->sample_every == 0)) {
            if (!c->gexec) {
                int rc = build_graph(c, s);
                if (rc) return rc;
            }
            HIP_TRY(hipGraphLaunch(c->gexec, s));
            c->steps_done += gl;
            done += gl;
            continue;
        }
        int rc = one_step(c, c->steps_done, s);
        if (rc) return rc;
        c->steps_done += 1;
        done += 1;
    }
    return SLPIC_OK;
}

int slpic_moments(void* ctx, int32_t run, double* d_out, void* stream) {
    Context* c = ctx_of(ctx);
    if (!c || !d_out || run < 0 || run >= c->P.nruns) return SLPIC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const RunInfo& R = c->P.runs[run];
    launch_zero(d_out, (int64_t)7 * R.nodes, s);
    if (prec(c) == SLPIC_F32)
        launch_moments_f32(c->a, c->P.run_chunk0[run], c->P.run_nchunks[run], 256, c->moments_lds, d_out, 0, s);
    else
        launch_moments_f64(c->a, c->P.run_chunk0[run], c->P.run_nchunks[run], 256, c->moments_lds, d_out, 0, s);
    launch_moments_finish(c->a, run, d_out, s);
    return hipGetLastError() == hipSuccess ? SLPIC_OK : SLPIC_EHIP;
}

int slpic_moments_sample(void* ctx, int32_t run, void* stream) {
    Context* c = ctx_of(ctx);
    if (!c || run < -1 || run >= c->P.nruns) return SLPIC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int r0 = run < 0 ? 0 : run, nr = run < 0 ? c->P.nruns : 1;
    const int ch0 = c->P.run_chunk0[r0];
    const int nch = run < 0 ? (int)c->P.chunks.size() : c->P.run_nchunks[run];
    if (prec(c) == SLPIC_F32)
        launch_moments_f32(c->a, ch0, nch, 256, c->moments_lds, c->a.Macc, 1, s);
    else
        launch_moments_f64(c->a, ch0, nch, 256, c->moments_lds, c->a.Macc, 1, s);
    launch_moments_sample_finish(c->a, r0, nr, s);
    return hipGetLastError() == hipSuccess ? SLPIC_OK : SLPIC_EHIP;
}

int slpic_moments_window(void* ctx, int32_t run, double* d_out, int32_t reset, void* stream) {
    Context* c = ctx_of(ctx);
    if (!c || !d_out || run < 0 || run >= c->P.nruns) return SLPIC_EINVAL;
    launch_moments_window(c->a, run, d_out, reset != 0, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? SLPIC_OK : SLPIC_EHIP;
}

int slpic_status_query(void* ctx, slpic_run_status* h_out, int32_t nruns) {
    Context* c = ctx_of(ctx);
    if (!c || !h_out || nruns < 0 || nruns > c->P.nruns) return SLPIC_EINVAL;
    HIP_TRY(hipDeviceSynchronize());
    std::vector<RunState> st(nruns);
    if (int rc = copy_d2h(st.data(), c->a.state, sizeof(RunState) * nruns)) return rc;
    for (int r = 0; r < nruns; ++r) {
        const RunInfo& R = c->P.runs[r];
        slpic_run_status& o = h_out[r];
        std::memset(&o, 0, sizeof o);
        o.step = st[r].step;
        for (int s = 0; s < 2; ++s) {
            o.nslots[s] = st[r].nslots[s];
            o.capacity[s] = R.cap[s];
            o.absorbed_total[s] = st[r].absorbed_total[s];
            o.injected_total[s] = st[r].injected_total[s];
            o.weight[s] = R.w[s];
        }
        o.acc_e = st[r].acc_e;
        o.wall_potential = st[r].phi_w;
        o.error_flags = st[r].error;
        o.fixed_bits = c->P.tun.precision == SLPIC_F32 ? R.fb : 0;
        o.steady_step = st[r].steady_step;
        o.windows = st[r].nwin;
        for (int k = 0; k < 3; ++k) o.window_mean[k] = st[r].win_mean[k];
        o.moment_samples = st[r].msamples;
        o.acc_flux[0] = st[r].acc_w[0];
        o.acc_flux[1] = st[r].acc_w[1];
    }
    return SLPIC_OK;
}

int slpic_wall_history(void* ctx, int32_t run, double* h_out, int64_t* n) {
    Context* c = ctx_of(ctx);
    if (!c || !h_out || !n || run < 0 || run >= c->P.nruns) return SLPIC_EINVAL;
    static_assert(kHistoryLen == SLPIC_HISTORY_LEN, "history length");
    HIP_TRY(hipDeviceSynchronize());
    int64_t step = 0;
    if (int rc = copy_d2h(&step, &c->a.state[run].step, sizeof step)) return rc;
    std::vector<double> ring(kHistoryLen);
    if (int rc = copy_d2h(ring.data(), c->a.history + (int64_t)run * kHistoryLen, sizeof(double) * kHistoryLen))
        return rc;
    const int64_t cnt = std::min<int64_t>(step, kHistoryLen);
    for (int64_t j = 0; j < cnt; ++j) h_out[j] = ring[(step - cnt + j) % kHistoryLen];
    *n = cnt;
    return SLPIC_OK;
}

static int cur_buffer(Context* c, int* b) {
    HIP_TRY(hipDeviceSynchronize());
    return copy_d2h(b, c->a.cur, sizeof(int));
}

int slpic_export_particles(void* ctx, int32_t run, int32_t species, double* h_xt, double* h_vx,
                           double* h_vperp2, int64_t* n) {
    Context* c = ctx_of(ctx);
    if (!c || !n || run < 0 || run >= c->P.nruns || species < 0 || species > 1) return SLPIC_EINVAL;
    int b = 0;
    if (int rc = cur_buffer(c, &b)) return rc;
    RunState st;
    if (int rc = copy_d2h(&st, c->a.state + run, sizeof st)) return rc;
    const int64_t cnt = st.nslots[species];
    if (*n < cnt || (cnt && (!h_xt || !h_vx || !h_vperp2))) {
        *n = cnt;
        return SLPIC_EINVAL;
    }
    const RunInfo& R = c->P.runs[run];
    const int64_t po = R.poff[species];
    if (prec(c) == SLPIC_F32) {
        std::vector<int32_t> x(cnt);
        std::vector<float> vx(cnt), vp(cnt);
        if (int rc = copy_d2h(x.data(), (int32_t*)c->a.bufs.x[b] + po, 4 * cnt)) return rc;
        if (int rc = copy_d2h(vx.data(), (float*)c->a.bufs.vx[b] + po, 4 * cnt)) return rc;
        if (int rc = copy_d2h(vp.data(), (float*)c->a.bufs.vp2[b] + po, 4 * cnt)) return rc;
        for (int64_t i = 0; i < cnt; ++i) {
            h_xt[i] = x[i] < 0 ? -1.0 : (double)x[i] * R.inv_fscale;
            h_vx[i] = vx[i];
            h_vperp2[i] = vp[i];
        }
    } else {
        if (int rc = copy_d2h(h_xt, (double*)c->a.bufs.x[b] + po, 8 * cnt)) return rc;
        if (int rc = copy_d2h(h_vx, (double*)c->a.bufs.vx[b] + po, 8 * cnt)) return rc;
        if (int rc = copy_d2h(h_vperp2, (double*)c->a.bufs.vp2[b] + po, 8 * cnt)) return rc;
    }
    *n = cnt;
    return SLPIC_OK;
}

int slpic_import_particles(void* ctx, int32_t run, int32_t species, const double* h_xt, const double* h_vx,
                           const double* h_vperp2, int64_t n) {
    Context* c = ctx_of(ctx);
    if (!c || run < 0 || run >= c->P.nruns || species < 0 || species > 1 || n < 0) return SLPIC_EINVAL;
    const RunInfo& R = c->P.runs[run];
    if (n > R.cap[species] || (n && (!h_xt || !h_vx || !h_vperp2))) return SLPIC_EINVAL;
    int b = 0;
    if (int rc = cur_buffer(c, &b)) return rc;
    const int64_t po = R.poff[species];
    if (prec(c) == SLPIC_F32) {
        std::vector<int32_t> x(n);
        std::vector<float> vx(n), vp(n);
        for (int64_t i = 0; i < n; ++i) {
            double xt = h_xt[i];
            if (!(xt >= 0.0)) x[i] = -1;
            else if (!(xt < (double)R.nx)) return SLPIC_EINVAL;
            else x[i] = (int32_t)std::llrint(xt * R.fscale);
            if (x[i] >= (int32_t)((int64_t)R.nx << R.fb)) return SLPIC_EINVAL;
            vx[i] = (float)h_vx[i];
            vp[i] = (float)h_vperp2[i];
        }
        if (int rc = copy_h2d((int32_t*)c->a.bufs.x[b] + po, x.data(), 4 * n)) return rc;
        if (int rc = copy_h2d((float*)c->a.bufs.vx[b] + po, vx.data(), 4 * n)) return rc;
        if (int rc = copy_h2d((float*)c->a.bufs.vp2[b] + po, vp.data(), 4 * n)) return rc;
    } else {
        for (int64_t i = 0; i < n; ++i)
            if (h_xt[i] >= (double)R.nx) return SLPIC_EINVAL;
        if (int rc = copy_h2d((double*)c->a.bufs.x[b] + po, h_xt, 8 * n)) return rc;
        if (int rc = copy_h2d((double*)c->a.bufs.vx[b] + po, h_vx, 8 * n)) return rc;
        if (int rc = copy_h2d((double*)c->a.bufs.vp2[b] + po, h_vperp2, 8 * n)) return rc;
    }
    int64_t nn = n;
    if (int rc = copy_h2d(&c->a.state[run].nslots[species], &nn, sizeof nn)) return rc;
    if (R.pruned) {  // not sorted again: both buffers hold the new slots
        if (int rc = mirror_run(c, run, nullptr)) return rc;
        HIP_TRY(hipDeviceSynchronize());
    }
    return SLPIC_OK;
}

int slpic_set_counters(void* ctx, int32_t run, int64_t step, double acc_e) {
    Context* c = ctx_of(ctx);
    if (!c || run < 0 || run >= c->P.nruns || step < 0) return SLPIC_EINVAL;
    HIP_TRY(hipDeviceSynchronize());
    if (int rc = copy_h2d(&c->a.state[run].step, &step, sizeof step)) return rc;
    if (int rc = copy_h2d(&c->a.state[run].acc_e, &acc_e, sizeof acc_e)) return rc;
    c->steps_done = step;
    return SLPIC_OK;
}

int slpic_set_speed_limit(void* ctx, int32_t run, double u, double dt, void* stream) {
    Context* c = ctx_of(ctx);
    if (!c || run < 0 || run >= c->P.nruns || !(dt > 0.0) || !(u > 0.0)) return SLPIC_EINVAL;
    RunInfo Rn = c->P.runs[run];
    const RunInfo& R = c->P.runs[run];
    if (R.varlim) return SLPIC_EINVAL;  // a run with a limit profile keeps it
    Rn.uinf = std::isinf(u) ? 1 : 0;
    Rn.u = u;
    Rn.u2 = u * u;
    Rn.umax = u;
    Rn.dt = dt;
    Rn.dtdx = dt / R.dx;
    LimitArgs L{};
    L.run = run;
    L.uinf = Rn.uinf;
    L.u = u;
    L.u2 = Rn.u2;
    for (int s = 0; s < 2; ++s) {
        Rn.ut[s] = u / R.vt[s];
        Rn.w[s] = R.dx * mean_inv_beta(R.beta_kind, Rn.ut[s]) / (double)R.ppc[s];
        Rn.qw[s] = R.qw[s] / R.w[s] * Rn.w[s];  // the species charge times the new weight
        if (Rn.uinf) {
            Rn.Ps[s] = 1.0;
            Rn.Pf[s] = 0.0;
        } else {
            step_mixture(Rn.ut[s], Rn.Ps[s], Rn.Pf[s]);
        }
        if (R.geom == kGeomPlates) {
            Rn.wall_flux[s] = R.vt[s] / std::sqrt(2.0 * M_PI) * dt / Rn.w[s];
            // the injection workgroups were planned for the old flux per step
            if (Rn.wall_flux[s] > R.wall_flux[s]) return SLPIC_EINVAL;
        }
        L.w[s] = Rn.w[s];
    }
    Rn.inj_ratio = Rn.w[1] / Rn.w[0];
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipDeviceSynchronize());
    const int nch = (int)c->P.chunks.size();
    if (prec(c) == SLPIC_F32) launch_limit_f32(c->a, L, nch, 0, s);
    else launch_limit_f64(c->a, L, nch, 0, s);
    launch_scan_ints(c->a.perm, c->P.total_slots, c->btot, s);
    {   // the scan of copy counts runs in int32 over every slot: its exact
        // (64-bit) total must stay below 2^31 before any copy is written
        long long total = 0;
        HIP_TRY(hipMemcpyAsync(&total, c->btot + scan_blocks(c->P.total_slots), sizeof total,
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (total >= 2147483647LL) return SLPIC_EINVAL;
    }
    if (prec(c) == SLPIC_F32) launch_limit_f32(c->a, L, nch, 1, s);
    else launch_limit_f64(c->a, L, nch, 1, s);
    launch_limit_finish(c->a, c->P.nruns, c->P.total_slots, c->btot, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    for (int r = 0; r < c->P.nruns; ++r)  // pruned runs are not sorted: both buffers keep them
        if (c->P.runs[r].pruned)
            if (int rc = mirror_run(c, r, s)) return rc;
    // the new run parameters, once the resampling (which reads the old ones) is done
    c->P.runs[run] = Rn;
    if (int rc = copy_h2d((void*)(c->a.runs + run), &Rn, sizeof(RunInfo))) return rc;
    l_push(c, false, s);
    launch_field(c->a, c->P.nruns, 0, c->field_lds, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return SLPIC_OK;
}


int slpic_prune_retired(void* ctx, int32_t* h_pruned, void* stream) {
    Context* c = ctx_of(ctx);
    if (!c) return SLPIC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipDeviceSynchronize());
    std::vector<RunState> st(c->P.nruns);
    if (int rc = copy_d2h(st.data(), c->a.state, sizeof(RunState) * c->P.nruns)) return rc;
    int newly = 0, total = 0;
    for (int r = 0; r < c->P.nruns; ++r) {
        RunInfo& R = c->P.runs[r];
        if (!R.pruned && retired(R, st[r])) {
            if (int rc = mirror_run(c, r, s)) return rc;
            R.pruned = 1;
            HIP_TRY(hipMemcpyAsync((void*)(c->a.runs + r), &R, sizeof(RunInfo), hipMemcpyHostToDevice, s));
            ++newly;
        }
        total += R.pruned;
    }
    if (newly) {
        c->active_host = push_order(c->P);
        const std::vector<Chunk>& act = c->active_host;
        if (!act.empty())
            HIP_TRY(hipMemcpyAsync(c->active, act.data(), sizeof(Chunk) * act.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
        c->n_active = (int)act.size();
        if (c->gexec) {  // captured with the old push grid
            (void)hipGraphExecDestroy(c->gexec);
            c->gexec = nullptr;
        }
    }
    if (h_pruned) *h_pruned = total;
    return SLPIC_OK;
}

int slpic_set_flux_counters(void* ctx, int32_t run, const double* h_acc) {
    Context* c = ctx_of(ctx);
    if (!c || !h_acc || run < 0 || run >= c->P.nruns || c->P.runs[run].geom != kGeomPlates) return SLPIC_EINVAL;
    for (int s = 0; s < 2; ++s)
        if (!(h_acc[s] >= 0.0 && h_acc[s] < 1.0)) return SLPIC_EINVAL;
    HIP_TRY(hipDeviceSynchronize());
    return copy_h2d(&c->a.state[run].acc_w[0], h_acc, 2 * sizeof(double));
}

int slpic_refresh_fields(void* ctx, void* stream) {
    Context* c = ctx_of(ctx);
    if (!c) return SLPIC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    launch_zero(c->a.Qacc, 2 * c->P.total_nodes, s);
    l_push(c, false, s);
    launch_field(c->a, c->P.nruns, 0, c->field_lds, s);
    return hipGetLastError() == hipSuccess ? SLPIC_OK : SLPIC_EHIP;
}

int slpic_export_grid(void* ctx, int32_t run, double* h_Q, double* h_phi, double* h_E) {
    Context* c = ctx_of(ctx);
    if (!c || run < 0 || run >= c->P.nruns) return SLPIC_EINVAL;
    HIP_TRY(hipDeviceSynchronize());
    const RunInfo& R = c->P.runs[run];
    if (h_Q)
        if (int rc = copy_d2h(h_Q, c->a.Qlast + 2 * R.goff, sizeof(double) * 2 * R.nodes)) return rc;
    if (h_phi)
        if (int rc = copy_d2h(h_phi, c->a.phi + R.goff, sizeof(double) * R.nodes)) return rc;
    if (h_E)
        if (int rc = copy_d2h(h_E, c->a.E + R.goff, sizeof(double) * R.nodes)) return rc;
    return SLPIC_OK;
}

int slpic_sort_now(void* ctx, void* stream) {
    Context* c = ctx_of(ctx);
    if (!c) return SLPIC_EINVAL;
    return do_sort(c, (hipStream_t)stream);
}

int slpic_export_perm(void* ctx, int32_t run, int32_t species, int32_t* h_perm, int64_t* n) {
    Context* c = ctx_of(ctx);
    if (!c || !n || run < 0 || run >= c->P.nruns || species < 0 || species > 1 || !c->P.tun.record_perm)
        return SLPIC_EINVAL;
    HIP_TRY(hipDeviceSynchronize());
    RunState st;
    if (int rc = copy_d2h(&st, c->a.state + run, sizeof st)) return rc;
    const int64_t cnt = st.nslots[species];
    if (*n < cnt || (cnt && !h_perm)) {
        *n = cnt;
        return SLPIC_EINVAL;
    }
    const RunInfo& R = c->P.runs[run];
    if (int rc = copy_d2h(h_perm, c->a.perm + R.poff[species], sizeof(int32_t) * cnt)) return rc;
    *n = cnt;
    return SLPIC_OK;
}

int slpic_set_sampling(void* ctx, int32_t every) {
    Context* c = ctx_of(ctx);
    if (!c || every < 0) return SLPIC_EINVAL;
    const int gl = c->P.tun.graph_steps;
    if (every > 0 && gl > 0 && gl % every) return SLPIC_EINVAL;
    if (every == c->sample_every) return SLPIC_OK;
    HIP_TRY(hipDeviceSynchronize());
    if (c->gexec) {  // captured with the old step sequence
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    c->sample_every = every;
    return SLPIC_OK;
}

int slpic_profile(void* ctx, int32_t enable) {
    Context* c = ctx_of(ctx);
    if (!c) return SLPIC_EINVAL;
    HIP_TRY(hipDeviceSynchronize());
    c->prof = (enable & 15) != 0;
    c->prof_mask = enable & 15;
    for (auto& u : c->ev_used) u = 0;
    return SLPIC_OK;
}

int slpic_profile_read(void* ctx, double* h_ms, int64_t* h_launches) {
    Context* c = ctx_of(ctx);
    if (!c || !h_ms || !h_launches) return SLPIC_EINVAL;
    HIP_TRY(hipDeviceSynchronize());
    for (int k = 0; k < 4; ++k) {
        double sum = 0.0;
        int64_t n = 0;
        for (size_t i = 0; i < c->ev_used[k]; ++i) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, c->ev[k][i].a, c->ev[k][i].b));
            sum += ms;
            ++n;
        }
        h_ms[k] = sum;
        h_launches[k] = n;
    }
    return SLPIC_OK;
}

int slpic_total_slots(void* ctx, int64_t* h_total) {
    Context* c = ctx_of(ctx);
    if (!c || !h_total) return SLPIC_EINVAL;
    HIP_TRY(hipDeviceSynchronize());
    std::vector<RunState> st(c->P.nruns);
    if (int rc = copy_d2h(st.data(), c->a.state, sizeof(RunState) * c->P.nruns)) return rc;
    int64_t t = 0;
    for (auto& x : st) t += x.pushed_total;
    *h_total = t;
    return SLPIC_OK;
}

int slpic_velocity_map(int32_t precision, int32_t beta_kind, double u, double dt, int64_t n, const void* d_vx,
                       const void* d_vperp2, const void* d_a, void* d_out, int32_t* d_iters, void* stream) {
    if (n < 0 || (n > 0 && (!d_vx || !d_vperp2 || !d_a || !d_out)) || !(u > 0) || !(dt > 0) ||
        (beta_kind != SLPIC_BETA_STEP && beta_kind != SLPIC_BETA_SMOOTH))
        return SLPIC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (precision == SLPIC_F32)
        launch_velocity_map_f32(beta_kind, u, dt, n, d_vx, d_vperp2, d_a, d_out, d_iters, s);
    else if (precision == SLPIC_F64)
        launch_velocity_map_f64(beta_kind, u, dt, n, d_vx, d_vperp2, d_a, d_out, d_iters, s);
    else
        return SLPIC_EINVAL;
    return hipGetLastError() == hipSuccess ? SLPIC_OK : SLPIC_EHIP;
}

void slpic_destroy(void* ctx) { delete ctx_of(ctx); }

const char* slpic_strerror(int code) {
    switch (code) {
        case SLPIC_OK: return "ok";
        case SLPIC_EINVAL: return "invalid argument or configuration";
        case SLPIC_ENOMEM: return "workspace too small";
        case SLPIC_ECAPACITY: return "particle capacity exceeded";
        case SLPIC_ENUMERIC: return "non-finite particle state";
        case SLPIC_EHIP: return "HIP runtime error";
        case SLPIC_ESTATE: return "call not valid in this state";
        case SLPIC_ELIMIT: return "input larger than the allocation-free call's fixed scratch";
        default: return "unknown error";
    }
}

}  // extern "C"
