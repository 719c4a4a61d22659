// wave.hip -- test particles in a prescribed traveling wave (the paper's
// wave-particle test): 1D1V particles (v_y = v_z = 0) in a periodic box
// [0, L) under phi(x, t) = phi0(t) sin(k (x - v_phi t)), k = 2 pi / L, with
// phi0 rising linearly from 0 to phi_max over ramp_time.  The particles do
// not act on the field, so each thread carries its particle through all the
// requested steps in registers: one load and one store per particle per
// launch.  Each step is App. Eq. (A2a, A2b) with the exact velocity map
// (c = 0: G_0(p) = p|p|/2), E evaluated exactly at (x^n, t^n = n dt).
#include <hip/hip_runtime.h>

#include <cmath>

#include "slpic.h"
#include "slpic_device.h"

namespace slpic {

struct WaveArgs {
    double L, vph, phimax, ramp, qm, dt, u;
    int bk;
};

template <typename T, int BK>
__global__ void k_wave_push(WaveArgs w, T* __restrict__ X, T* __restrict__ V, int64_t n, int64_t step0,
                            int nsteps) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool uinf = isinf(w.u);
    const T u = uinf ? T(0) : (T)w.u, u2 = u * u, dt = (T)w.dt, L = (T)w.L;
    const double k = 6.283185307179586 / w.L;
    T x = X[i], v = V[i];
    for (int s = 0; s < nsteps; ++s) {
        const double t = (double)(step0 + s) * w.dt;
        const double phi0 = (w.ramp > 0.0 && t < w.ramp) ? w.phimax * (t / w.ramp) : w.phimax;
        T a;
        if constexpr (sizeof(T) == 8) {
            a = -w.qm * phi0 * k * cos(k * (x - w.vph * t));
        } else {
            // phase in turns: (x - v_phi t) / L, the wave offset reduced in FP64
            const double off = fmod(w.vph * t, w.L);
            const float turns = (x - (float)off) * (float)(1.0 / w.L);
            a = (float)(-w.qm * phi0 * k) * __builtin_amdgcn_cosf(turns);
        }
        v = kick1d<BK, T>(v, T(0), a, dt, u, u2, uinf);
        const T b = beta_s2<BK, T>(v * v, u, u2, uinf);
        x = x + b * v * dt;
        if (x < T(0) || x >= L) {
            x = fmod(x, L);
            if (x < T(0)) x += L;
            if (x >= L) x = T(0);
        }
    }
    X[i] = x;
    V[i] = v;
}

}  // namespace slpic

using namespace slpic;

extern "C" int slpic_wave_push(int32_t precision, const slpic_wave_config* cfg, void* d_x, void* d_v, int64_t n,
                               int64_t step0, int32_t nsteps, void* stream) {
    if (!cfg || n < 0 || nsteps < 0 || step0 < 0 || (n > 0 && (!d_x || !d_v))) return SLPIC_EINVAL;
    if (!(cfg->length > 0) || !(cfg->dt > 0) || !(cfg->u > 0) || !std::isfinite(cfg->v_phase) ||
        !std::isfinite(cfg->phi_max) || !std::isfinite(cfg->qm) || !(cfg->ramp_time >= 0) ||
        (cfg->beta_kind != SLPIC_BETA_STEP && cfg->beta_kind != SLPIC_BETA_SMOOTH) ||
        (precision != SLPIC_F32 && precision != SLPIC_F64))
        return SLPIC_EINVAL;
    if (n == 0 || nsteps == 0) return SLPIC_OK;
    WaveArgs w{cfg->length, cfg->v_phase, cfg->phi_max, cfg->ramp_time, cfg->qm, cfg->dt, cfg->u, cfg->beta_kind};
    hipStream_t s = (hipStream_t)stream;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    const bool smooth = cfg->beta_kind == SLPIC_BETA_SMOOTH;
    if (precision == SLPIC_F32) {
        if (smooth) hipLaunchKernelGGL((k_wave_push<float, kBetaSmooth>), grid, block, 0, s, w, (float*)d_x, (float*)d_v, n, step0, nsteps);
        else hipLaunchKernelGGL((k_wave_push<float, kBetaStep>), grid, block, 0, s, w, (float*)d_x, (float*)d_v, n, step0, nsteps);
    } else {
        if (smooth) hipLaunchKernelGGL((k_wave_push<double, kBetaSmooth>), grid, block, 0, s, w, (double*)d_x, (double*)d_v, n, step0, nsteps);
        else hipLaunchKernelGGL((k_wave_push<double, kBetaStep>), grid, block, 0, s, w, (double*)d_x, (double*)d_v, n, step0, nsteps);
    }
    return hipGetLastError() == hipSuccess ? SLPIC_OK : SLPIC_EHIP;
}
