// slpic_device.h -- device math of the SLPIC particle step: the counter-based
// generator, the speed-limiting functions and the exact frozen-field
// velocity map of Eq. (A2a), written for gfx950 in float or double.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "slpic_internal.h"

namespace slpic {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32->64-bit multiplies; the key is bumped by a Weyl sequence between
// rounds.  One call gives four 32-bit words.
// ---------------------------------------------------------------------------
struct U4 { uint32_t v[4]; };

__host__ __device__ __forceinline__ uint32_t mulhi32(uint32_t a, uint32_t b) {
    return (uint32_t)(((uint64_t)a * b) >> 32);
}
__host__ __device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint32_t lo0 = 0xD2511F53u * c0, hi0 = mulhi32(0xD2511F53u, c0);
        uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = mulhi32(0xCD9E8D57u, c2);
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    U4 o;
    o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

// 53-bit uniform in [0,1): 27 high bits of a, 26 high bits of b.
__host__ __device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

// Per-particle uniform stream: counter (index, step, run, purpose|species|call).
struct Stream {
    uint32_t c0, c1, c2, c3, k0, k1;
    U4 buf;
    int pos;
    __device__ Stream(const RunInfo& R, uint32_t index, uint32_t step, int purpose, int species)
        : Stream(R.run_id, R.seed_lo, R.seed_hi, index, step, purpose, species) {}
    __device__ Stream(uint32_t run_id, uint32_t seed_lo, uint32_t seed_hi, uint32_t index, uint32_t step,
                      int purpose, int species)
        : c0(index), c1(step), c2(run_id), c3(((uint32_t)purpose << 24) | ((uint32_t)species << 20)),
          k0(seed_lo), k1(seed_hi), pos(4) {}
    __device__ double next() {
        if (pos >= 4) {
            buf = philox10(c0, c1, c2, c3, k0, k1);
            c3 += 1u;
            pos = 0;
        }
        double r = u53(buf.v[pos], buf.v[pos + 1]);
        pos += 2;
        return r;
    }
    // Box-Muller: two normals from one pair, the third from the next pair.
    __device__ void normal3(double z[3]) {
        double u1 = next(), u2 = next();
        double r = sqrt(-2.0 * log(1.0 - u1));
        double sn, cs;
        sincos(6.283185307179586 * u2, &sn, &cs);
        z[0] = r * cs;
        z[1] = r * sn;
        double u3 = next(), u4 = next();
        double r2 = sqrt(-2.0 * log(1.0 - u3));
        z[2] = r2 * cos(6.283185307179586 * u4);
    }
};

// ---------------------------------------------------------------------------
// Elementary functions of the particle arithmetic.  Float uses the gfx950
// hardware instructions (v_sqrt/v_rcp/v_rsq/v_log_f32, ~1 ulp), which the
// float tolerances absorb; double keeps the correctly rounded library forms.
// ---------------------------------------------------------------------------
template <typename T> struct Fm;
template <> struct Fm<float> {
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    static __device__ __forceinline__ float log(float x) { return __builtin_amdgcn_logf(x) * 0.6931471805599453f; }
    // log(1 + y) for small y: log(w) * y / (w - 1) with w = 1 + y keeps the
    // relative accuracy of y (the rounding of w cancels).
    static __device__ __forceinline__ float log1p(float y) {
        const float w = 1.0f + y;
        return (w == 1.0f) ? y : log(w) * div(y, w - 1.0f);
    }
};
template <> struct Fm<double> {
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double rsqrt(double x) { return 1.0 / ::sqrt(x); }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
    static __device__ __forceinline__ double log(double x) { return ::log(x); }
    static __device__ __forceinline__ double log1p(double y) { return ::log1p(y); }
};

// ---------------------------------------------------------------------------
// Speed-limiting functions of the squared speed.
// ---------------------------------------------------------------------------
enum { kBetaStep = 0, kBetaSmooth = 1 };

template <int BK, typename T>
__device__ __forceinline__ T beta_s2(T s2, T u, T u2, bool uinf) {
    if (uinf) return T(1);
    if (sizeof(T) == 8) {  // double: the correctly rounded forms
        if (BK == kBetaSmooth) return T(1) / sqrt(T(1) + s2 / u2);  // Eq. (11a)
        return (s2 <= u2) ? T(1) : u / sqrt(s2);                    // Eq. (11b), beta(v0) = 1
    }
    if (BK == kBetaSmooth) return Fm<T>::rsqrt(T(1) + Fm<T>::div(s2, u2));
    return (s2 <= u2) ? T(1) : u * Fm<T>::rsqrt(s2);
}

// beta of Eq. (11a)/(11b) in FP64 from the stored particle velocity, for the
// charge deposit, injected particles and the moments (float particles: the
// float hardware reciprocal square root refined by one FP64 Newton step,
// ~1e-14; double particles: the correctly rounded form).
template <int BK, typename T>
__device__ __forceinline__ double beta_deposit(T vx, T c2, double u, double u2, bool uinf) {
    if (uinf) return 1.0;
    const double v = (double)vx;
    const double s2 = v * v + (double)c2;
    if (BK == kBetaSmooth) return 1.0 / sqrt(1.0 + s2 / u2);
    if (s2 <= u2) return 1.0;
    if (sizeof(T) == 8) return u / sqrt(s2);
    // float seed (~1e-7), one Newton step in FP64: ~1.5e-14, always from below
    double y = (double)__builtin_amdgcn_rsqf((float)s2);
    y = y * (1.5 - 0.5 * s2 * y * y);
    return u * y;
}

// ---------------------------------------------------------------------------
// Cold load: g0 = f0/beta (Eq. 5).  Speeds from the g-speed density of
// Eq. (11b) (a mixture of the Maxwell speed density below v0 and
// s^3 e^{-s^2/2} above it), or of Eq. (11a) by rejection from it; isotropic
// directions; uniform positions.  The uniform draws of one particle come in
// a fixed order from its own counter-based stream, so runs are reproducible.
// ---------------------------------------------------------------------------
__device__ inline double sample_g_speed_step(Stream& st, double ut, double Ps, double Pf) {
    double usel = st.next();
    if (usel * (Ps + Pf) < Ps) {
        for (int attempt = 0; attempt < 100000; ++attempt) {
            if (ut <= 1.0) {
                double s = ut * cbrt(st.next());
                double acc = st.next();
                if (acc < exp(-0.5 * s * s)) return s;
            } else {
                double z[3];
                st.normal3(z);
                double s = sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
                if (s <= ut) return s;
            }
        }
        return 0.0;
    }
    double t0 = 0.5 * ut * ut;
    double uc = st.next();
    double y = -log(1.0 - st.next());
    if (!(uc * (t0 + 1.0) < t0)) {
        double y2 = -log(1.0 - st.next());
        y += y2;
    }
    return sqrt(2.0 * (t0 + y));
}

__device__ inline double sample_g_speed(Stream& st, int bk, double ut, double Ps, double Pf) {
    if (bk == kBetaStep) return sample_g_speed_step(st, ut, Ps, Pf);
    for (int attempt = 0; attempt < 100000; ++attempt) {
        double s = sample_g_speed_step(st, ut, Ps, Pf);
        double r = sqrt(1.0 + (s / ut) * (s / ut)) / (sqrt(2.0) * fmax(1.0, s / ut));
        if (st.next() < r) return s;
    }
    return 0.0;
}

template <typename T> struct Eps;
template <> struct Eps<float> { static constexpr float v = 1.1920929e-7f; };
template <> struct Eps<double> { static constexpr double v = 2.220446049250313e-16; };

// G_c(p) = (p s + c^2 asinh(p/c)) / 2, s = sqrt(p^2 + c^2): the integral of
// the speed along the velocity path, which fast segments advance linearly in
// time (s dp = |a| v0 dt).  asinh r = log1p(r + r^2 / (1 + sqrt(1 + r^2))) for
// every r >= 0 (one branch-free form; sqrt(1 + r^2) = s/c).
template <typename T>
__device__ __forceinline__ T G_of(T c2, T c, T p, T s) {
    if (c2 == T(0)) return T(0.5) * p * fabs(p);
    const T ic = Fm<T>::rcp(c);
    const T r = fabs(p) * ic;
    const T ash = Fm<T>::log1p(r + Fm<T>::div(r * r, T(1) + s * ic));
    return T(0.5) * (p * s + copysign(c2 * ash, p));
}

// Series inverse of the speed integral around p0: with alpha = p0/s0 and
// kappa = K/s0^2, p1 = p0 + s0 d where
//   d = sum_n c_n kappa^n,  c_1 = 1, c_2 = -alpha/2, c_3 = (4 alpha^2 - 1)/6, ...
// (the inverse of int_0^d sqrt(1 + 2 alpha t + t^2) dt = kappa, whose
// coefficients are polynomials in alpha; the integrand's singularities lie at
// |t| = 1).  Truncated after kappa^8, the error is below 7e-9 s0 for
// kappa <= 0.1 and 4e-5 s0 at kappa = 1/4, for every |alpha| <= 1.
template <typename T>
__device__ __forceinline__ T series_inverse(T al, T kap) {
    const T a2 = al * al;
    const T c2 = T(-0.5) * al;
    const T c3 = (T(4) * a2 - T(1)) * T(1.0 / 6.0);
    const T c4 = al * (T(13) - T(28) * a2) * T(1.0 / 24.0);
    const T c5 = ((T(280) * a2 - T(188)) * a2 + T(13)) * T(1.0 / 120.0);
    const T c6 = al * ((T(-3640) * a2 + T(3188)) * a2 - T(493)) * T(1.0 / 720.0);
    const T c7 = (((T(58240) * a2 - T(62832)) * a2 + T(15480)) * a2 - T(493)) * T(1.0 / 5040.0);
    const T c8 = al * (((T(-1106560) * a2 + T(1417584)) * a2 - T(483528)) * a2 + T(37369)) * T(1.0 / 40320.0);
    return kap * (T(1) + kap * (c2 + kap * (c3 + kap * (c4 + kap * (c5 + kap * (c6 + kap * (c7 + kap * c8)))))));
}

// The same series through kappa^4: for kappa <= 0.03 the omitted terms sum
// to at most 2.2e-8 s0 for every |alpha| <= 1 (the leading one, c_5 kappa^5
// with |c_5| <= 0.875), under the float rounding of s0.
template <typename T>
__device__ __forceinline__ T series_inverse4(T al, T kap) {
    const T a2 = al * al;
    const T c2 = T(-0.5) * al;
    const T c3 = (T(4) * a2 - T(1)) * T(1.0 / 6.0);
    const T c4 = al * (T(13) - T(28) * a2) * T(1.0 / 24.0);
    return kap * (T(1) + kap * (c2 + kap * (c3 + kap * c4)));
}

// p1 >= p0 with G_c(p1) - G_c(p0) = K.
//  - c = 0: closed form, p1|p1| = p0|p0| + 2K.
//  - kappa = K/s0^2 < 1/4: the series inverse, used as is in float when
//    kappa <= 0.11 (truncation below float rounding; through kappa^4 when
//    every active lane of the wave has kappa <= 0.03), else refined by
//    Newton steps on G;
//  - larger kicks: Newton on G from the upper bound min(c = 0 solution,
//    p0 + K/c), bracketed by bisection (G is monotone).
// Newton stops when the step falls below a few ulps of |p| + c (the rounding
// floor of G differences), or at the iteration cap.
template <typename T>
__device__ __forceinline__ T fast_advance(T c2, T p0, T K, int* iters = nullptr) {
    if (!(K > T(0))) return p0;
    const T eps = Eps<T>::v;
    const bool f32 = sizeof(T) == 4;
    T pser = T(0);
    const bool small = c2 > T(0) && K < T(0.25) * (p0 * p0 + c2);  // kappa < 1/4
    if (small) {
        const T s0 = Fm<T>::sqrt(p0 * p0 + c2);
        const T inv_s0 = Fm<T>::rcp(s0);
        const T kap = K * inv_s0 * inv_s0;
        if (f32 && __all(kap <= T(0.03))) {  // the whole wave's kicks are small: four terms
            if (iters) *iters += 1;
            return p0 + s0 * series_inverse4(p0 * inv_s0, kap);
        }
        pser = p0 + s0 * series_inverse(p0 * inv_s0, kap);
        if (f32 && kap <= T(0.11)) {
            if (iters) *iters += 1;
            return pser;
        }
    }
    const T Q = T(0.5) * p0 * fabs(p0) + K;
    const T pc0 = (Q >= T(0)) ? Fm<T>::sqrt(T(2) * Q) : -Fm<T>::sqrt(-T(2) * Q);
    if (c2 == T(0)) return pc0;
    const T c = Fm<T>::sqrt(c2);
    T hi = fmin(pc0, p0 + Fm<T>::div(K, c));
    T lo = p0;
    T p = hi;
    int nmax = f32 ? 12 : 60;
    if (small) {
        if (pser > lo && pser <= hi) p = pser;
        nmax = f32 ? 3 : 6;
    }
    const T s0 = Fm<T>::sqrt(p0 * p0 + c2);
    const T Gt = G_of(c2, c, p0, s0) + K;
    // rounding floor of a Newton step: G differences carry ~eps (|p| + c) / s
    const T tol_rel = f32 ? T(8) * eps : T(4) * eps;
    // A step leaving the bracket first lands on the bound it crossed (the
    // c = 0 bound is often within rounding of the root when c << |p|); a
    // second exit in a row bisects.
    bool clamped = false;
    int it = 0;
    for (; it < nmax; ++it) {
        const T s = Fm<T>::sqrt(p * p + c2);
        const T r = G_of(c2, c, p, s) - Gt;
        if (r == T(0)) break;
        if (r > T(0)) hi = p;
        else lo = p;
        const T step = Fm<T>::div(r, s);
        T pn = p - step;
        if (fabs(step) <= tol_rel * (fabs(p) + c)) {  // converged: accept the last step
            p = pn;
            break;
        }
        if (!(pn > lo && pn < hi)) {
            pn = clamped ? T(0.5) * (lo + hi) : (pn >= hi ? hi : lo);
            clamped = true;
        } else {
            clamped = false;
        }
        p = pn;
    }
    if (iters) *iters += it + 1;
    return p;
}

// Eq. (A2a) in 1D3V: E along x, so v moves along x with c^2 = v_perp^2 fixed;
// p = sign(a) v_x obeys dp/dt = |a| beta(sqrt(p^2 + c^2)) with a frozen.  The
// path is split into its segments first, so that every lane makes at most
// one fast_advance call (divergent lanes of a wave then share it).
template <int BK, typename T>
__device__ __forceinline__ T kick1d(T vx, T c2, T a, T dt, T u, T u2, bool uinf, int* iters = nullptr) {
    if (a == T(0)) return vx;
    if (uinf) return vx + a * dt;  // beta == 1: standard leapfrog
    if (BK == kBetaStep) {
        // |v|^2 is convex along the path: both ends inside the band => beta = 1 throughout
        if (vx * vx + c2 <= u2) {
            T vt = vx + a * dt;
            if (vt * vt + c2 <= u2) return vt;
        }
    }
    const T sg = (a > T(0)) ? T(1) : T(-1);
    const T A = fabs(a);
    const T p0 = sg * vx;
    // the last segment: fast from pf over time rem with constant c^2 = cf
    T cf = c2, pf = p0, rem = dt;
    bool fast = true;
    if (BK == kBetaSmooth) {
        cf = c2 + u2;  // Eq. (11a): the speed integral with c^2 + u^2
    } else if (c2 < u2) {
        // Eq. (11b): fast toward the band, slow inside |p| <= ps, fast beyond
        const T ps = Fm<T>::sqrt(u2 - c2);
        // reaching the band from p0 < -ps takes the speed integral
        // G(-ps) - G(p0) >= (p0^2 - ps^2)/2 (the speed is at least |p|): when
        // that bound already exceeds the step's A u dt, the two G evaluations
        // (two logarithms) are skipped
        if (p0 < -ps && T(0.5) * (p0 * p0 - ps * ps) < A * u * dt) {
            const T c = Fm<T>::sqrt(c2);
            const T Kneed = G_of(c2, c, -ps, u) - G_of(c2, c, p0, Fm<T>::sqrt(p0 * p0 + c2));
            if (Kneed < A * u * dt) {  // reaches the band
                rem = dt - Fm<T>::div(Kneed, A * u);
                pf = -ps;
            }
        }
        if (pf >= -ps && pf <= ps) {
            const T tb = Fm<T>::div(ps - pf, A);
            if (tb >= rem) {
                pf = pf + A * rem;  // ends inside the band
                fast = false;
            } else {
                rem -= tb;
                pf = ps;
            }
        }
    }
    if (fast) pf = fast_advance(cf, pf, A * u * rem, iters);
    return sg * pf;
}

// ---------------------------------------------------------------------------
// Positions: F32 runs store int32 fixed point (fb fraction bits) so the cell
// is an exact shift and the CIC fraction an exact float; F64 runs store the
// grid coordinate xt = x/dx as a double.  Dead slots are negative.
// ---------------------------------------------------------------------------
// The cell map of a run (fraction bits of the fixed point), copied into
// registers: kernels that store particles read it once, before any store.
struct CellMap {
    int fb;
    float inv_fscale;
    __device__ __forceinline__ explicit CellMap(const RunInfo& R) : fb(R.fb), inv_fscale((float)R.inv_fscale) {}
    __device__ __forceinline__ CellMap(int fb_, float inv_fscale_) : fb(fb_), inv_fscale(inv_fscale_) {}
};
template <typename T> struct PosT;
template <> struct PosT<float> {
    using S = int32_t;
    static __device__ __forceinline__ bool alive(S x) { return x >= 0; }
    static __device__ __forceinline__ void cell_frac(S x, const CellMap& m, int& c, float& f) {
        c = x >> m.fb;
        f = (float)(x & ((1 << m.fb) - 1)) * m.inv_fscale;
    }
    static __device__ __forceinline__ void cell_frac(S x, const RunInfo& R, int& c, float& f) {
        cell_frac(x, CellMap(R), c, f);
    }
    static __device__ __forceinline__ S dead() { return -1; }
};
template <> struct PosT<double> {
    using S = double;
    static __device__ __forceinline__ bool alive(S x) { return x >= 0.0; }
    static __device__ __forceinline__ void cell_frac(S x, const CellMap&, int& c, double& f) {
        c = (int)x;
        f = x - (double)c;
    }
    static __device__ __forceinline__ void cell_frac(S x, const RunInfo&, int& c, double& f) {
        c = (int)x;
        f = x - (double)c;
    }
    static __device__ __forceinline__ S dead() { return -1.0; }
};

// The lanes of the wave that hold the same sort key as this one (keys >= 0;
// a lane with k < 0 gets 0), for the counting sorts.  The distinct keys of a
// row are peeled one at a time, the lowest remaining lane's key each round
// (a row of cell-sorted particles holds one or two keys); lanes left after
// kPeelKeys rounds are grouped by the bits of their keys, one ballot per bit
// of nbits.
constexpr int kPeelKeys = 4;
__device__ __forceinline__ uint64_t key_peers(int k, int nbits) {
    uint64_t todo = __ballot(k >= 0);
    uint64_t peers = 0;
    for (int it = 0; it < kPeelKeys && todo; ++it) {
        const int k0 = __builtin_amdgcn_readlane(k, __builtin_ctzll(todo));  // wave-uniform
        const uint64_t m = __ballot(k == k0);
        peers = (k == k0) ? m : peers;
        todo &= ~m;
    }
    if (todo) {
        const bool mine = (todo >> (threadIdx.x & 63)) & 1;
        uint64_t p = todo;
        for (int bit = 0; bit < nbits; ++bit) {
            const bool on = (k >> bit) & 1;
            const uint64_t m = __ballot(mine && on);
            p &= on ? m : ~m;
        }
        peers = mine ? p : peers;
    }
    return peers;
}

// Runs of equal keys in a row (lane order): a lane heads a run when its key
// differs from the previous lane's.  key_runs returns the mask of heads and
// the previous lane's key (lane 0: its own); run_length the size of the run
// a head lane starts.
__device__ __forceinline__ uint64_t key_runs(int k, int lane, int& kprev) {
    kprev = __shfl_up(k, 1);
    return __ballot(lane == 0 || k != kprev);
}
__device__ __forceinline__ int run_length(uint64_t heads, int lane) {
    const uint64_t after = heads & ~((2ull << lane) - 1);  // heads above this lane (lane 63: none)
    return (after ? (int)__builtin_ctzll(after) : 64) - lane;
}

// Stable rank of a lane among the lanes of its row holding its key, and
// (for the lowest such lane, rank 0) their number.  A row whose keys do not
// decrease in lane order (a sorted row) holds each key in one run: the rank
// is the distance to the run's head.  Other rows group lanes by key_peers.
__device__ __forceinline__ void key_rank(int k, int nbits, int lane, int& rank, int& count) {
    int kprev;
    const uint64_t heads = key_runs(k, lane, kprev);
    if (__ballot(lane > 0 && k < kprev) == 0) {  // wave-uniform: keys non-decreasing
        const int head = 63 - (int)__builtin_clzll(heads & ((2ull << lane) - 1));
        rank = lane - head;
        count = rank == 0 ? run_length(heads, lane) : 0;
    } else {
        const uint64_t peers = key_peers(k, nbits);
        const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        rank = (int)__popcll(peers & lt);
        count = (int)__popcll(peers);
    }
}

// Steady-state detection on the wall potential Phi_w (1D: phi(0) - phi(L);
// 2D: the y-mean of phi(0, y); the paper calls the final state an
// equilibrium without a formal test): steps are grouped into windows of
// steady_window steps; when a window closes, its mean joins the last three
// means, and the run is steady at the first step where the three means lie
// within steady_tol * |their mean| of it (the largest deviation from their
// average).  The step count then stays as steady_step.  Called by one thread
// per run after each advancing solve, with st->step already counting it.
// RI / ST: the run parameters and run state of the 1D or the 2D library.
template <typename RI, typename ST>
__device__ __forceinline__ void steady_feed(const RI& R, ST* st, double pw) {
    st->win_sum += pw;
    st->win_n += 1;
    if (st->win_n < R.steady_window) return;
    const double m = st->win_sum / (double)R.steady_window;
    st->win_mean[2] = st->win_mean[1];
    st->win_mean[1] = st->win_mean[0];
    st->win_mean[0] = m;
    st->nwin += 1;
    st->win_sum = 0.0;
    st->win_n = 0;
    if (st->nwin >= 3 && st->steady_step < 0) {
        const double m0 = st->win_mean[0], m1 = st->win_mean[1], m2 = st->win_mean[2];
        const double mbar = (m0 + m1 + m2) / 3.0;
        const double dev = fmax(fmax(fabs(m0 - mbar), fabs(m1 - mbar)), fabs(m2 - mbar));
        if (dev <= R.steady_tol * fabs(mbar)) st->steady_step = st->step;
    }
}

// Orders a wave's LDS accesses: everything before is complete and visible to
// the other lanes of the wave before anything after.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

}  // namespace slpic
