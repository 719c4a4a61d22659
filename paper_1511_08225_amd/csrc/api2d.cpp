// api2d.cpp -- the C ABI of include/slpic2d.h: planning of one 2D3V run
// (run table, workspace layout, field-solve tables), cold start, stepping,
// the tile sort, state import/export and event timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "host_math.h"
#include "launch.h"
#include "launch2d.h"
#include "slpic2d.h"
#include "slpic2d_internal.h"

using namespace slpic;

namespace {

constexpr size_t kAlign2 = 256;
size_t up2(size_t n) { return (n + kAlign2 - 1) / kAlign2 * kAlign2; }
constexpr int kInjectGroups2 = 256;  // source injection: a step's new particles (FP64 draws each) spread over the chip

#define HIP2_TRY(x)                                    \
    do {                                               \
        if ((x) != hipSuccess) return SLPIC_EHIP;      \
    } while (0)

struct Layout2 {
    size_t run, st, cur, inj, counts, x[2], y[2], vx[2], vy[2], vz2[2], perm, Q, phi, E, E32, spec, tpiv, tw,
        hist, btot, tbeg, history, total;
};

struct Plan2 {
    slpic2d_tuning tun{};
    Run2D R{};
    int64_t total_slots = 0, hist_entries = 0;
    size_t push_lds = 0, sort_lds = 0, scatter_lds = 0;
    Layout2 L{};
};

int clog2(int64_t v) {
    int b = 0;
    while ((int64_t(1) << b) < v) ++b;
    return b;
}

int make_plan2(const slpic_run_config* c, int ny, const slpic2d_tuning* tin, Plan2& P) {
    if (!c || c->geometry != SLPIC_GEOM_SHEATH) return SLPIC_EINVAL;  // the plates geometry is 1D only
    slpic2d_tuning t{};
    if (tin) t = *tin;
    if (t.precision != SLPIC_F32 && t.precision != SLPIC_F64) return SLPIC_EINVAL;
    if (t.sort_every < 0 || t.tile < 0 || t.margin < 0 || t.per_thread < 0 || t.tail_groups < 0 || t.sort_tile < 0 ||
        t.graph_steps < 0 || (t.record_perm != 0 && t.record_perm != 1))
        return SLPIC_EINVAL;
    // a captured block of steps starts at a multiple of the sort period
    if (t.sort_every > 0 && t.graph_steps > 0 && t.graph_steps % t.sort_every)
        t.graph_steps = (t.graph_steps / t.sort_every + 1) * t.sort_every;
    if (t.tile == 0) t.tile = 8;
    if (t.margin == 0) t.margin = std::max(1, t.sort_every);
    if (t.per_thread == 0) t.per_thread = 1;
    if (t.tail_groups == 0) t.tail_groups = 512;
    if (t.sort_tile == 0) t.sort_tile = 32768;  // 512 x 512 sheath: 0.392 ms per step (65536: 0.402)
    // the scatter keeps per-wave offsets within a tile's run of one key in 16 bits
    if (t.sort_tile < 1024 || t.sort_tile > 32768 || (t.sort_tile & 1023)) return SLPIC_EINVAL;
    if (t.tile > 64 || t.margin > 32 || t.tail_groups > 65536) return SLPIC_EINVAL;
    if (t.per_thread != 1 && t.per_thread != 2 && t.per_thread != 4 && t.per_thread != 8) return SLPIC_EINVAL;
    if (ny < 4 || ny > 2048 || (ny & (ny - 1))) return SLPIC_EINVAL;
    if (c->nx < 4 || c->nx > 1024 || !(c->dx > 0) || !(c->dt > 0) || !(c->u > 0) || c->nspecies != 2 ||
        c->source_cells < 1 || c->source_cells > c->nx || c->warm_profile || c->limit_profile ||
        (c->beta_kind != SLPIC_BETA_STEP && c->beta_kind != SLPIC_BETA_SMOOTH) || c->steady_window < 0 ||
        !(c->steady_tol >= 0.0))
        return SLPIC_EINVAL;
    P.tun = t;
    Run2D& R = P.R;
    R.nx = c->nx;
    R.ny = ny;
    R.beta_kind = c->beta_kind;
    R.source_cells = c->source_cells;
    R.fb = std::min(24, 31 - clog2((int64_t)std::max(c->nx, ny) + 1));
    R.uinf = std::isinf(c->u) ? 1 : 0;
    R.tile = t.tile;
    R.ntx = (c->nx + t.tile - 1) / t.tile;
    R.nty = (ny + t.tile - 1) / t.tile;
    R.nkeys = R.ntx * R.nty;
    if (R.nkeys > 4096) return SLPIC_EINVAL;
    R.margin = t.margin;
    R.win = t.tile + 2 * t.margin + 1;
    R.sort_tile = t.sort_tile;
    R.tile_shift = (t.tile & (t.tile - 1)) ? -1 : clog2(t.tile);
    R.dx = c->dx;
    R.dt = c->dt;
    R.u = c->u;
    R.u2 = c->u * c->u;
    R.dtdx = c->dt / c->dx;
    R.fscale = std::ldexp(1.0, R.fb);
    R.inv_fscale = std::ldexp(1.0, -R.fb);
    R.seed_lo = (uint32_t)(c->seed & 0xffffffffu);
    R.seed_hi = (uint32_t)(c->seed >> 32);
    R.run_id = (uint32_t)c->run_id;
    R.nodes = (int64_t)(c->nx + 1) * ny;
    R.steady_window = c->steady_window > 0 ? c->steady_window : std::max(1, c->nx / 4);
    R.steady_tol = c->steady_tol > 0.0 ? c->steady_tol : 0.02;
    const double cf = c->capacity_factor > 1.0 ? c->capacity_factor : 1.0;
    int64_t poff = 0, hoff = 0;
    for (int s = 0; s < 2; ++s) {
        const slpic_species& sp = c->species[s];
        if (!(sp.mass > 0) || !(sp.temperature > 0) || sp.ppc < 1) return SLPIC_EINVAL;
        R.vt[s] = std::sqrt(sp.temperature / sp.mass);
        R.mass[s] = sp.mass;
        R.ut[s] = c->u / R.vt[s];
        R.w[s] = c->dx * c->dx * mean_inv_beta(c->beta_kind, R.ut[s]) / (double)sp.ppc;
        R.qw[s] = sp.charge * R.w[s];
        R.qm[s] = sp.charge / sp.mass;
        if (R.uinf) {
            R.Ps[s] = 1.0;
            R.Pf[s] = 0.0;
        } else {
            step_mixture(R.ut[s], R.Ps[s], R.Pf[s]);
        }
        R.nload[s] = (int64_t)c->nx * ny * sp.ppc;
        R.cap[s] = std::max<int64_t>((int64_t)std::ceil(cf * (double)R.nload[s]), R.nload[s] + 64);
        if (R.cap[s] > (int64_t(1) << 31) - 1) return SLPIC_EINVAL;
        R.poff[s] = poff;
        poff += R.cap[s];
        R.stiles[s] = (int32_t)((R.cap[s] + t.sort_tile - 1) / t.sort_tile);
        R.hoff[s] = hoff;
        hoff += (int64_t)R.nkeys * R.stiles[s];
    }
    if (poff > (int64_t(1) << 31) - 1 || hoff > (int64_t(1) << 31) - 1) return SLPIC_EINVAL;
    R.inj_ratio = R.w[1] / R.w[0];
    P.total_slots = poff;
    P.hist_entries = hoff;
    const size_t tsz = t.precision == SLPIC_F32 ? 4 : 8;
    P.push_lds = (size_t)R.win * R.win * (2 * tsz + 8);
    P.sort_lds = (size_t)R.nkeys * sizeof(int);  // the tile's key counts
    // four waves' packed per-key offsets
    P.scatter_lds = (size_t)4 * ((R.nkeys + 1) / 2) * sizeof(uint32_t);
    if (P.push_lds > 65536 || P.sort_lds > 65536 || P.scatter_lds > 65536) return SLPIC_EINVAL;
    Layout2& L = P.L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = up2(o + std::max<size_t>(bytes, 1));
        return at;
    };
    L.run = take(sizeof(Run2D));
    L.st = take(sizeof(State2D));
    L.cur = take(sizeof(int));
    L.inj = take(sizeof(Inject2D));
    L.counts = take(sizeof(int2) * 2 * kCountSlots2);
    for (int b = 0; b < 2; ++b) {
        L.x[b] = take(tsz * P.total_slots);
        L.y[b] = take(tsz * P.total_slots);
        L.vx[b] = take(tsz * P.total_slots);
        L.vy[b] = take(tsz * P.total_slots);
        L.vz2[b] = take(tsz * P.total_slots);
    }
    L.perm = take(t.record_perm ? sizeof(int32_t) * P.total_slots : 0);
    L.Q = take(sizeof(double) * 2 * R.nodes);
    L.phi = take(sizeof(double) * R.nodes);
    L.E = take(sizeof(double2) * R.nodes);
    L.E32 = take(sizeof(float2) * R.nodes);
    L.spec = take(sizeof(double2) * (size_t)R.nx * ny);
    L.tpiv = take(sizeof(double) * (size_t)(ny / 2 + 1) * R.nx);
    L.tw = take(sizeof(double2) * (size_t)(ny / 2));
    L.hist = take(sizeof(int) * P.hist_entries);
    L.btot = take(sizeof(long long) * (scan_blocks(P.hist_entries) + 1));
    L.tbeg = take(sizeof(int64_t) * 2 * (R.nkeys + 1));
    L.history = take(sizeof(double) * kHistoryLen2);
    L.total = o;
    return SLPIC_OK;
}

struct Ev2 {
    hipEvent_t a = nullptr, b = nullptr;
};

struct Ctx2 {
    Plan2 P;
    Args2D a{};
    unsigned char* ws = nullptr;
    int64_t steps_done = 0;
    int prof = 0;
    std::vector<Ev2> ev[4];
    size_t ev_used[4] = {0, 0, 0, 0};
    hipGraphExec_t gexec = nullptr;  // graph_steps captured steps (built on first use)
    ~Ctx2() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        for (auto& v : ev)
            for (auto& e : v) {
                if (e.a) (void)hipEventDestroy(e.a);
                if (e.b) (void)hipEventDestroy(e.b);
            }
    }
};

Ctx2* ctx2(void* p) { return static_cast<Ctx2*>(p); }
bool f32(const Ctx2* c) { return c->P.tun.precision == SLPIC_F32; }

// Launch wrapper: an event pair around the launches of class k when enabled.
template <typename F>
int timed2(Ctx2* c, int k, hipStream_t s, F&& f) {
    if (!((c->prof >> k) & 1)) {
        f();
        return hipGetLastError() == hipSuccess ? SLPIC_OK : SLPIC_EHIP;
    }
    if (c->ev_used[k] == c->ev[k].size()) {
        Ev2 e;
        HIP2_TRY(hipEventCreate(&e.a));
        HIP2_TRY(hipEventCreate(&e.b));
        c->ev[k].push_back(e);
    }
    Ev2& e = c->ev[k][c->ev_used[k]++];
    HIP2_TRY(hipEventRecord(e.a, s));
    f();
    HIP2_TRY(hipEventRecord(e.b, s));
    return hipGetLastError() == hipSuccess ? SLPIC_OK : SLPIC_EHIP;
}

int push2(Ctx2* c, bool push, hipStream_t s) {
    const Plan2& P = c->P;
    int rc = 0;
    if (f32(c)) rc = launch2d_push_f32(push, P.tun.per_thread, c->a, P.R.nkeys, P.tun.tail_groups, P.push_lds, s);
    else rc = launch2d_push_f64(push, P.tun.per_thread, c->a, P.R.nkeys, P.tun.tail_groups, P.push_lds, s);
    return rc ? SLPIC_EINVAL : SLPIC_OK;
}

int sort2(Ctx2* c, hipStream_t s) {
    const Plan2& P = c->P;
    const int nt = P.R.stiles[0] + P.R.stiles[1];
    return timed2(c, 3, s, [&] {
        // the (key, tile) counts start at zero: a tile writes only the keys it holds
        launch_zero_ints(c->a.hist, P.hist_entries, s);
        if (f32(c)) launch2d_sort_hist_f32(c->a, nt, P.sort_lds, s);
        else launch2d_sort_hist_f64(c->a, nt, P.sort_lds, s);
        launch_scan_ints(c->a.hist, P.hist_entries, c->a.btot, s);
        if (f32(c)) launch2d_sort_scatter_f32(c->a, nt, P.scatter_lds, s);
        else launch2d_sort_scatter_f64(c->a, nt, P.scatter_lds, s);
        launch2d_sort_finish(c->a, scan_blocks(P.hist_entries), s);
    });
}

int field2(Ctx2* c, hipStream_t s, int advance = 0) {
    return timed2(c, 2, s, [&] { launch2d_field(c->a, c->P.R.nx, c->P.R.ny, advance, s); });
}

int refresh2(Ctx2* c, hipStream_t s) {
    launch2d_fill(c->a.Q, 2 * c->P.R.nodes, s);
    int rc = push2(c, false, s);
    if (rc) return rc;
    return field2(c, s);
}

// One step; `index` is the step's number modulo the capture (it decides the
// periodic sort); the caller counts it.
int one_step2(Ctx2* c, int64_t index, hipStream_t s) {
    int rc;
    launch2d_fill(c->a.Q, 2 * c->P.R.nodes, s);
    int prc = SLPIC_OK;
    if ((rc = timed2(c, 0, s, [&] { prc = push2(c, true, s); }))) return rc;
    if (prc) return prc;
    if ((rc = timed2(c, 1, s, [&] {
             if (f32(c)) launch2d_inject_f32(c->a, kInjectGroups2, s);
             else launch2d_inject_f64(c->a, kInjectGroups2, s);
             launch2d_finish(c->a, s);
         })))
        return rc;
    if ((rc = field2(c, s, 1))) return rc;  // with Phi_w into the history ring and the steady detector
    const int se = c->P.tun.sort_every;
    if (se > 0 && (index + 1) % se == 0)
        if ((rc = sort2(c, s))) return rc;
    return SLPIC_OK;
}

// graph_steps steps captured from a step index that is a multiple of the
// sort period (the launches read every count from the device).
int build_graph2(Ctx2* c, hipStream_t s) {
    hipGraph_t g = nullptr;
    HIP2_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    int rc = SLPIC_OK;
    for (int k = 0; k < c->P.tun.graph_steps && rc == SLPIC_OK; ++k) rc = one_step2(c, k, s);
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc != SLPIC_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return rc != SLPIC_OK ? rc : SLPIC_EHIP;
    }
    e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->gexec = nullptr;
        return SLPIC_EHIP;
    }
    return SLPIC_OK;
}

int read_state(Ctx2* c, State2D& st) {
    HIP2_TRY(hipMemcpy(&st, c->a.st, sizeof(State2D), hipMemcpyDeviceToHost));
    return SLPIC_OK;
}

int cur_buf(Ctx2* c, int* b) {
    HIP2_TRY(hipMemcpy(b, c->a.cur, sizeof(int), hipMemcpyDeviceToHost));
    return SLPIC_OK;
}

}  // namespace

extern "C" {

size_t slpic2d_workspace_bytes(const slpic_run_config* run, int32_t ny, const slpic2d_tuning* tuning) {
    Plan2 P;
    if (make_plan2(run, ny, tuning, P) != SLPIC_OK) return 0;
    return P.L.total;
}

int slpic2d_init(const slpic_run_config* run, int32_t ny, const slpic2d_tuning* tuning, void* d_workspace,
                 size_t workspace_bytes, void* stream, void** out_ctx) {
    if (!out_ctx) return SLPIC_EINVAL;
    *out_ctx = nullptr;
    Ctx2* c = new (std::nothrow) Ctx2();
    if (!c) return SLPIC_ENOMEM;
    int rc = make_plan2(run, ny, tuning, c->P);
    if (rc == SLPIC_OK && (!d_workspace || ((uintptr_t)d_workspace % kAlign2) != 0)) rc = SLPIC_EINVAL;
    if (rc == SLPIC_OK && workspace_bytes < c->P.L.total) rc = SLPIC_ENOMEM;
    if (rc) {
        delete c;
        return rc;
    }
    hipStream_t s = (hipStream_t)stream;
    unsigned char* w = (unsigned char*)d_workspace;
    const Layout2& L = c->P.L;
    const Run2D& R = c->P.R;
    c->ws = w;
    Args2D& a = c->a;
    a.run = (const Run2D*)(w + L.run);
    a.st = (State2D*)(w + L.st);
    a.cur = (int*)(w + L.cur);
    a.inj = (Inject2D*)(w + L.inj);
    a.counts = (int2*)(w + L.counts);
    for (int b = 0; b < 2; ++b) {
        a.x[b] = w + L.x[b];
        a.y[b] = w + L.y[b];
        a.vx[b] = w + L.vx[b];
        a.vy[b] = w + L.vy[b];
        a.vz2[b] = w + L.vz2[b];
    }
    a.perm = c->P.tun.record_perm ? (int32_t*)(w + L.perm) : nullptr;
    a.Q = (double*)(w + L.Q);
    a.phi = (double*)(w + L.phi);
    a.E = (double2*)(w + L.E);
    a.E32 = (float2*)(w + L.E32);
    a.spec = (double2*)(w + L.spec);
    a.tpiv = (const double*)(w + L.tpiv);
    a.tw = (const double2*)(w + L.tw);
    a.hist = (int*)(w + L.hist);
    a.btot = (long long*)(w + L.btot);
    a.tbeg = (int64_t*)(w + L.tbeg);
    a.history = (double*)(w + L.history);
    // field-solve tables: twiddles exp(-2 pi i k/ny) and, per y-mode m <=
    // ny/2, the pivots of the elimination of its x-system (diagonal 2 +
    // 4 sin^2(pi m/ny) with dy = dx, off-diagonals -1, row 0 coupled to row 1
    // by -2): p_i = 1 / (diag + c'_{i-1}), c'_0 = -2 p_0, c'_i = -p_i
    std::vector<double2> tw(ny / 2);
    for (int k = 0; k < ny / 2; ++k) {
        const double ang = 2.0 * M_PI * (double)k / (double)ny;
        tw[k] = make_double2(std::cos(ang), -std::sin(ang));
    }
    std::vector<double> piv((size_t)(ny / 2 + 1) * R.nx);
    for (int m = 0; m <= ny / 2; ++m) {
        const double sm = std::sin(M_PI * (double)m / (double)ny);
        const double diag = 2.0 + 4.0 * sm * sm;
        double cp = 0.0;
        for (int i = 0; i < R.nx; ++i) {
            const double p = 1.0 / (diag + cp);
            piv[(size_t)m * R.nx + i] = p;
            cp = (i == 0 ? -2.0 : -1.0) * p;
        }
    }
    State2D st{};
    for (int sp = 0; sp < 2; ++sp) st.nslots[sp] = R.nload[sp];
    st.steady_step = -1;
#define INIT2_TRY(x)             \
    do {                         \
        if ((x) != hipSuccess) { \
            delete c;            \
            return SLPIC_EHIP;   \
        }                        \
    } while (0)
    INIT2_TRY(hipMemsetAsync(w, 0, L.total, s));
    INIT2_TRY(hipMemcpyAsync((void*)a.run, &R, sizeof(Run2D), hipMemcpyHostToDevice, s));
    INIT2_TRY(hipMemcpyAsync(a.st, &st, sizeof(State2D), hipMemcpyHostToDevice, s));
    INIT2_TRY(hipMemcpyAsync((void*)a.tw, tw.data(), sizeof(double2) * tw.size(), hipMemcpyHostToDevice, s));
    INIT2_TRY(hipMemcpyAsync((void*)a.tpiv, piv.data(), sizeof(double) * piv.size(), hipMemcpyHostToDevice, s));
    if (f32(c)) launch2d_load_f32(a, s);
    else launch2d_load_f64(a, s);
    rc = SLPIC_OK;
    if (c->P.tun.sort_every > 0) rc = sort2(c, s);
    if (rc == SLPIC_OK) rc = refresh2(c, s);
    if (rc == SLPIC_OK && hipStreamSynchronize(s) != hipSuccess) rc = SLPIC_EHIP;
#undef INIT2_TRY
    if (rc) {
        delete c;
        return rc;
    }
    *out_ctx = c;
    return SLPIC_OK;
}

int slpic2d_step(void* ctx, int32_t nsteps, void* stream) {
    Ctx2* c = ctx2(ctx);
    if (!c || nsteps < 0) return SLPIC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int se = c->P.tun.sort_every, gl = c->P.tun.graph_steps;
    // graph replay on a non-default stream; profiled steps launch directly
    const bool graphs = gl > 0 && s != nullptr && !c->prof;
    int32_t done = 0;
    while (done < nsteps) {
        if (graphs && nsteps - done >= gl && (se == 0 || c->steps_done % se == 0)) {
            if (!c->gexec) {
                int rc = build_graph2(c, s);
                if (rc) return rc;
            }
            HIP2_TRY(hipGraphLaunch(c->gexec, s));
            c->steps_done += gl;
            done += gl;
            continue;
        }
        int rc = one_step2(c, c->steps_done, s);
        if (rc) return rc;
        c->steps_done += 1;
        done += 1;
    }
    return SLPIC_OK;
}

int slpic2d_moments(void* ctx, double* d_out, void* stream) {
    Ctx2* c = ctx2(ctx);
    if (!c || !d_out) return SLPIC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const Run2D& R = c->P.R;
    launch2d_fill(d_out, 7 * R.nodes, s);
    if (f32(c)) launch2d_moments_f32(c->a, std::max(R.cap[0], R.cap[1]), d_out, s);
    else launch2d_moments_f64(c->a, std::max(R.cap[0], R.cap[1]), d_out, s);
    launch2d_moments_finish(c->a, R.nodes, d_out, s);
    return hipGetLastError() == hipSuccess ? SLPIC_OK : SLPIC_EHIP;
}

int slpic2d_wall_history(void* ctx, double* h_out, int64_t* n) {
    Ctx2* c = ctx2(ctx);
    if (!c || !h_out || !n) return SLPIC_EINVAL;
    static_assert(kHistoryLen2 == SLPIC_HISTORY_LEN, "history length");
    HIP2_TRY(hipDeviceSynchronize());
    State2D st;
    int rc = read_state(c, st);
    if (rc) return rc;
    std::vector<double> ring(kHistoryLen2);
    HIP2_TRY(hipMemcpy(ring.data(), c->a.history, sizeof(double) * kHistoryLen2, hipMemcpyDeviceToHost));
    const int64_t cnt = std::min<int64_t>(st.step, kHistoryLen2);
    for (int64_t j = 0; j < cnt; ++j) h_out[j] = ring[(st.step - cnt + j) % kHistoryLen2];
    *n = cnt;
    return SLPIC_OK;
}

int slpic2d_refresh_fields(void* ctx, void* stream) {
    Ctx2* c = ctx2(ctx);
    if (!c) return SLPIC_EINVAL;
    return refresh2(c, (hipStream_t)stream);
}

int slpic2d_solve_charge(void* ctx, const double* d_Q, void* stream) {
    Ctx2* c = ctx2(ctx);
    if (!c || !d_Q) return SLPIC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    HIP2_TRY(hipMemcpyAsync(c->a.Q, d_Q, sizeof(double) * 2 * c->P.R.nodes, hipMemcpyDeviceToDevice, s));
    return field2(c, s);
}

int slpic2d_export_grid(void* ctx, double* h_Q, double* h_phi, double* h_E) {
    Ctx2* c = ctx2(ctx);
    if (!c) return SLPIC_EINVAL;
    HIP2_TRY(hipDeviceSynchronize());
    const int64_t nodes = c->P.R.nodes;
    if (h_Q) HIP2_TRY(hipMemcpy(h_Q, c->a.Q, sizeof(double) * 2 * nodes, hipMemcpyDeviceToHost));
    if (h_phi) HIP2_TRY(hipMemcpy(h_phi, c->a.phi, sizeof(double) * nodes, hipMemcpyDeviceToHost));
    if (h_E) {
        std::vector<double2> e(nodes);
        HIP2_TRY(hipMemcpy(e.data(), c->a.E, sizeof(double2) * nodes, hipMemcpyDeviceToHost));
        for (int64_t n = 0; n < nodes; ++n) {
            h_E[n] = e[n].x;
            h_E[nodes + n] = e[n].y;
        }
    }
    return SLPIC_OK;
}

int slpic2d_export_particles(void* ctx, int32_t species, double* h_x, double* h_y, double* h_vx, double* h_vy,
                             double* h_vz2, int64_t* n) {
    Ctx2* c = ctx2(ctx);
    if (!c || species < 0 || species > 1 || !n || !h_x || !h_y || !h_vx || !h_vy || !h_vz2) return SLPIC_EINVAL;
    HIP2_TRY(hipDeviceSynchronize());
    State2D st;
    int rc = read_state(c, st);
    if (rc) return rc;
    int b;
    if ((rc = cur_buf(c, &b))) return rc;
    const int64_t m = st.nslots[species];
    if (*n < m) return SLPIC_EINVAL;
    *n = m;
    const Run2D& R = c->P.R;
    const int64_t off = R.poff[species];
    if (f32(c)) {
        std::vector<int32_t> X(m), Y(m);
        std::vector<float> VX(m), VY(m), VZ(m);
        HIP2_TRY(hipMemcpy(X.data(), (int32_t*)c->a.x[b] + off, 4 * m, hipMemcpyDeviceToHost));
        HIP2_TRY(hipMemcpy(Y.data(), (int32_t*)c->a.y[b] + off, 4 * m, hipMemcpyDeviceToHost));
        HIP2_TRY(hipMemcpy(VX.data(), (float*)c->a.vx[b] + off, 4 * m, hipMemcpyDeviceToHost));
        HIP2_TRY(hipMemcpy(VY.data(), (float*)c->a.vy[b] + off, 4 * m, hipMemcpyDeviceToHost));
        HIP2_TRY(hipMemcpy(VZ.data(), (float*)c->a.vz2[b] + off, 4 * m, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < m; ++i) {
            h_x[i] = X[i] < 0 ? -1.0 : (double)X[i] * R.inv_fscale;
            h_y[i] = (double)Y[i] * R.inv_fscale;
            h_vx[i] = VX[i];
            h_vy[i] = VY[i];
            h_vz2[i] = VZ[i];
        }
    } else {
        HIP2_TRY(hipMemcpy(h_x, (double*)c->a.x[b] + off, 8 * m, hipMemcpyDeviceToHost));
        HIP2_TRY(hipMemcpy(h_y, (double*)c->a.y[b] + off, 8 * m, hipMemcpyDeviceToHost));
        HIP2_TRY(hipMemcpy(h_vx, (double*)c->a.vx[b] + off, 8 * m, hipMemcpyDeviceToHost));
        HIP2_TRY(hipMemcpy(h_vy, (double*)c->a.vy[b] + off, 8 * m, hipMemcpyDeviceToHost));
        HIP2_TRY(hipMemcpy(h_vz2, (double*)c->a.vz2[b] + off, 8 * m, hipMemcpyDeviceToHost));
    }
    return SLPIC_OK;
}

int slpic2d_import_particles(void* ctx, int32_t species, const double* h_x, const double* h_y,
                             const double* h_vx, const double* h_vy, const double* h_vz2, int64_t n) {
    Ctx2* c = ctx2(ctx);
    if (!c || species < 0 || species > 1 || n < 0 || (n > 0 && (!h_x || !h_y || !h_vx || !h_vy || !h_vz2)))
        return SLPIC_EINVAL;
    const Run2D& R = c->P.R;
    if (n > R.cap[species]) return SLPIC_ECAPACITY;
    for (int64_t i = 0; i < n; ++i) {  // coordinates inside the domain (dead slots: x < 0)
        if (h_x[i] >= 0 && !(h_x[i] < (double)R.nx && h_y[i] >= 0 && h_y[i] < (double)R.ny)) return SLPIC_EINVAL;
    }
    HIP2_TRY(hipDeviceSynchronize());
    State2D st;
    int rc = read_state(c, st);
    if (rc) return rc;
    int b;
    if ((rc = cur_buf(c, &b))) return rc;
    const int64_t off = R.poff[species];
    if (f32(c)) {
        std::vector<int32_t> X(n), Y(n);
        std::vector<float> VX(n), VY(n), VZ(n);
        auto enc = [&](double v, int lim) {
            int64_t q = std::llrint(v * R.fscale);
            const int64_t top = ((int64_t)lim << R.fb) - 1;
            return (int32_t)std::min(std::max<int64_t>(q, 0), top);
        };
        for (int64_t i = 0; i < n; ++i) {
            X[i] = h_x[i] < 0 ? -1 : enc(h_x[i], R.nx);
            Y[i] = h_x[i] < 0 ? 0 : enc(h_y[i], R.ny);
            VX[i] = (float)h_vx[i];
            VY[i] = (float)h_vy[i];
            VZ[i] = (float)h_vz2[i];
        }
        HIP2_TRY(hipMemcpy((int32_t*)c->a.x[b] + off, X.data(), 4 * n, hipMemcpyHostToDevice));
        HIP2_TRY(hipMemcpy((int32_t*)c->a.y[b] + off, Y.data(), 4 * n, hipMemcpyHostToDevice));
        HIP2_TRY(hipMemcpy((float*)c->a.vx[b] + off, VX.data(), 4 * n, hipMemcpyHostToDevice));
        HIP2_TRY(hipMemcpy((float*)c->a.vy[b] + off, VY.data(), 4 * n, hipMemcpyHostToDevice));
        HIP2_TRY(hipMemcpy((float*)c->a.vz2[b] + off, VZ.data(), 4 * n, hipMemcpyHostToDevice));
    } else {
        std::vector<double> X(h_x, h_x + n), Y(h_y, h_y + n);
        for (int64_t i = 0; i < n; ++i) {
            if (X[i] < 0) {
                X[i] = -1.0;
                Y[i] = 0.0;
            }
        }
        HIP2_TRY(hipMemcpy((double*)c->a.x[b] + off, X.data(), 8 * n, hipMemcpyHostToDevice));
        HIP2_TRY(hipMemcpy((double*)c->a.y[b] + off, Y.data(), 8 * n, hipMemcpyHostToDevice));
        HIP2_TRY(hipMemcpy((double*)c->a.vx[b] + off, h_vx, 8 * n, hipMemcpyHostToDevice));
        HIP2_TRY(hipMemcpy((double*)c->a.vy[b] + off, h_vy, 8 * n, hipMemcpyHostToDevice));
        HIP2_TRY(hipMemcpy((double*)c->a.vz2[b] + off, h_vz2, 8 * n, hipMemcpyHostToDevice));
    }
    st.nslots[species] = n;
    st.nsorted[species] = 0;
    HIP2_TRY(hipMemcpy(c->a.st, &st, sizeof(State2D), hipMemcpyHostToDevice));
    return SLPIC_OK;
}

int slpic2d_set_counters(void* ctx, int64_t step, double acc_e) {
    Ctx2* c = ctx2(ctx);
    if (!c || step < 0 || !(acc_e >= 0.0 && acc_e < 1.0)) return SLPIC_EINVAL;
    HIP2_TRY(hipDeviceSynchronize());
    State2D st;
    int rc = read_state(c, st);
    if (rc) return rc;
    st.step = step;
    st.acc_e = acc_e;
    HIP2_TRY(hipMemcpy(c->a.st, &st, sizeof(State2D), hipMemcpyHostToDevice));
    c->steps_done = step;
    return SLPIC_OK;
}

int slpic2d_sort_now(void* ctx, void* stream) {
    Ctx2* c = ctx2(ctx);
    if (!c) return SLPIC_EINVAL;
    return sort2(c, (hipStream_t)stream);
}

int slpic2d_export_perm(void* ctx, int32_t species, int32_t* h_perm, int64_t* n) {
    Ctx2* c = ctx2(ctx);
    if (!c || species < 0 || species > 1 || !n || !h_perm || !c->a.perm) return SLPIC_EINVAL;
    HIP2_TRY(hipDeviceSynchronize());
    State2D st;
    int rc = read_state(c, st);
    if (rc) return rc;
    const int64_t m = st.live[species];
    if (*n < m) return SLPIC_EINVAL;
    *n = m;
    HIP2_TRY(hipMemcpy(h_perm, c->a.perm + c->P.R.poff[species], sizeof(int32_t) * m, hipMemcpyDeviceToHost));
    return SLPIC_OK;
}

int slpic2d_status_query(void* ctx, slpic2d_status* h_out) {
    Ctx2* c = ctx2(ctx);
    if (!c || !h_out) return SLPIC_EINVAL;
    HIP2_TRY(hipDeviceSynchronize());
    State2D st;
    int rc = read_state(c, st);
    if (rc) return rc;
    const Run2D& R = c->P.R;
    slpic2d_status o{};
    o.step = st.step;
    for (int s = 0; s < 2; ++s) {
        o.nslots[s] = st.nslots[s];
        o.nsorted[s] = st.nsorted[s];
        o.capacity[s] = R.cap[s];
        o.absorbed_total[s] = st.absorbed_total[s];
        o.injected_total[s] = st.injected_total[s];
        o.weight[s] = R.w[s];
    }
    o.pushed_total = st.pushed_total;
    o.acc_e = st.acc_e;
    o.wall_potential = st.phi_w;
    o.error_flags = st.error;
    o.fixed_bits = c->P.tun.precision == SLPIC_F32 ? R.fb : 0;
    o.steady_step = st.steady_step;
    o.windows = st.nwin;
    for (int k = 0; k < 3; ++k) o.window_mean[k] = st.win_mean[k];
    *h_out = o;
    return SLPIC_OK;
}

int slpic2d_profile(void* ctx, int32_t enable) {
    Ctx2* c = ctx2(ctx);
    if (!c || enable < 0 || enable > 15) return SLPIC_EINVAL;
    c->prof = enable;
    for (auto& u : c->ev_used) u = 0;
    return SLPIC_OK;
}

int slpic2d_profile_read(void* ctx, double* h_ms, int64_t* h_launches) {
    Ctx2* c = ctx2(ctx);
    if (!c || !h_ms || !h_launches) return SLPIC_EINVAL;
    HIP2_TRY(hipDeviceSynchronize());
    for (int k = 0; k < 4; ++k) {
        double tot = 0.0;
        for (size_t j = 0; j < c->ev_used[k]; ++j) {
            float ms = 0.0f;
            HIP2_TRY(hipEventElapsedTime(&ms, c->ev[k][j].a, c->ev[k][j].b));
            tot += ms;
        }
        h_ms[k] = tot;
        h_launches[k] = (int64_t)c->ev_used[k];
    }
    return SLPIC_OK;
}

void slpic2d_destroy(void* ctx) { delete ctx2(ctx); }

}  // extern "C"
