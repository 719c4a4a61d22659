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

__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    U4 o;
    o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

// 53-bit uniform in [0,1): 27 high bits of a, 26 high bits of b.
__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

// Per-particle uniform stream: counter (index, step, run, purpose|species|call).
struct Stream {
    uint32_t c0, c1, c2, c3, k0, k1;
    U4 buf;
    int pos;
    __device__ Stream(const RunInfo& R, uint32_t index, uint32_t step, int purpose, int species)
        : c0(index), c1(step), c2(R.run_id),
          c3(((uint32_t)purpose << 24) | ((uint32_t)species << 20)), k0(R.seed_lo), k1(R.seed_hi),
          pos(4) {}
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
// Speed-limiting functions of the squared speed.
// ---------------------------------------------------------------------------
enum { kBetaStep = 0, kBetaSmooth = 1 };

template <int BK, typename T>
__device__ __forceinline__ T beta_s2(T s2, T u, T u2, bool uinf) {
    if (uinf) return T(1);
    if (BK == kBetaSmooth) return T(1) / sqrt(T(1) + s2 / u2);  // Eq. (11a)
    return (s2 <= u2) ? T(1) : u / sqrt(s2);                    // Eq. (11b), beta(v0) = 1
}

template <typename T> struct Eps;
template <> struct Eps<float> { static constexpr float v = 1.1920929e-7f; };
template <> struct Eps<double> { static constexpr double v = 2.220446049250313e-16; };

// G_c(p) = (p s + c^2 asinh(p/c)) / 2, s = sqrt(p^2 + c^2): the integral of
// the speed along the velocity path, which fast segments advance linearly in
// time (s dp = |a| v0 dt).
template <typename T>
__device__ __forceinline__ T G_of(T c2, T c, T p, T s) {
    if (c2 == T(0)) return T(0.5) * p * fabs(p);
    T ap = fabs(p);
    T r = ap / c;
    T ash;
    if (r < T(0.5)) {
        T q = sqrt(T(1) + r * r);
        ash = log1p(r + r * r / (T(1) + q));
    } else {
        ash = log((ap + s) / c);
    }
    return T(0.5) * (p * s + copysign(c2 * ash, p));
}

// p1 >= p0 with G_c(p1) - G_c(p0) = K.  Small kicks (K << s0^2) use the
// series inverse of the integral around p0 (alpha = p0/s0, gamma = c^2/s0^2,
// kappa = K/s0^2):
//   dp/s0 = k - a/2 k^2 + (a^2/2 - g/6) k^3 + (-5/8 a^3 + 13/24 a g) k^4 + O(k^5);
// otherwise (and always in double) Newton on G, bracketed by the bounds
// sqrt(p^2+c^2) >= |p| (c = 0 solution) and >= c (p0 + K/c).
template <typename T>
__device__ __forceinline__ T fast_advance(T c2, T p0, T K) {
    if (!(K > T(0))) return p0;
    const T eps = Eps<T>::v;
    T s0 = sqrt(p0 * p0 + c2);
    T inv_s0 = T(1) / s0;
    T kap = K * inv_s0 * inv_s0;
    T p;
    bool series = kap < T(0.25);
    if (series) {
        T al = p0 * inv_s0, ga = c2 * inv_s0 * inv_s0;
        T c4 = T(-0.625) * al * al * al + T(13.0 / 24.0) * al * ga;
        T c3 = T(0.5) * al * al - ga * T(1.0 / 6.0);
        T d = kap * (T(1) + kap * (T(-0.5) * al + kap * (c3 + kap * c4)));
        p = p0 + s0 * d;
        if (sizeof(T) == 4 && kap < T(0.02)) return p;
    }
    T c = sqrt(c2);
    T Gt = G_of(c2, c, p0, s0) + K;
    T Q = T(0.5) * p0 * fabs(p0) + K;
    T hi = (Q >= T(0)) ? sqrt(T(2) * Q) : -sqrt(-T(2) * Q);
    if (c2 > T(0)) hi = fmin(hi, p0 + K / c);
    T lo = p0;
    if (!series || !(p > lo && p <= hi)) p = hi;
    for (int it = 0; it < 40; ++it) {
        T s = sqrt(p * p + c2);
        T r = G_of(c2, c, p, s) - Gt;
        if (r > T(0)) hi = p;
        else if (r < T(0)) lo = p;
        else break;
        T pn = (s > T(0)) ? p - r / s : T(0.5) * (lo + hi);
        if (!(pn > lo && pn < hi)) pn = T(0.5) * (lo + hi);
        T dl = fabs(pn - p);
        p = pn;
        if (dl <= T(4) * eps * fabs(pn) || hi - lo <= T(4) * eps * fmax(fabs(lo), fabs(hi))) break;
    }
    return p;
}

// Eq. (A2a) in 1D3V: E along x, so v moves along x with c^2 = v_perp^2 fixed;
// p = sign(a) v_x obeys dp/dt = |a| beta(sqrt(p^2 + c^2)) with a frozen.
template <int BK, typename T>
__device__ __forceinline__ T kick1d(T vx, T c2, T a, T dt, T u, T u2, bool uinf) {
    if (a == T(0)) return vx;
    if (uinf) return vx + a * dt;  // beta == 1: standard leapfrog
    if (BK == kBetaStep) {
        // |v|^2 is convex along the path: both ends inside the band => beta = 1 throughout
        if (vx * vx + c2 <= u2) {
            T vt = vx + a * dt;
            if (vt * vt + c2 <= u2) return vt;
        }
    }
    T sg = (a > T(0)) ? T(1) : T(-1);
    T A = fabs(a);
    T p0 = sg * vx;
    T p1;
    if (BK == kBetaSmooth) {
        p1 = fast_advance(c2 + u2, p0, A * u * dt);
    } else if (c2 >= u2) {
        p1 = fast_advance(c2, p0, A * u * dt);
    } else {
        // Eq. (11b): fast toward the band, slow inside |p| <= ps, fast beyond
        T ps = sqrt(u2 - c2);
        T p = p0, rem = dt;
        bool done = false;
        p1 = p0;
        if (p < -ps) {
            T c = sqrt(c2);
            T s = sqrt(p * p + c2);
            T Kneed = G_of(c2, c, -ps, u) - G_of(c2, c, p, s);
            T Kav = A * u * rem;
            if (Kneed >= Kav) {
                p1 = fast_advance(c2, p, Kav);
                done = true;
            } else {
                rem -= Kneed / (A * u);
                p = -ps;
            }
        }
        if (!done && p <= ps) {
            T tb = (ps - p) / A;
            if (tb >= rem) {
                p1 = p + A * rem;
                done = true;
            } else {
                rem -= tb;
                p = ps;
            }
        }
        if (!done) p1 = fast_advance(c2, p, A * u * rem);
    }
    return sg * p1;
}

// ---------------------------------------------------------------------------
// Positions: F32 runs store int32 fixed point (fb fraction bits) so the cell
// is an exact shift and the CIC fraction an exact float; F64 runs store the
// grid coordinate xt = x/dx as a double.  Dead slots are negative.
// ---------------------------------------------------------------------------
template <typename T> struct PosT;
template <> struct PosT<float> {
    using S = int32_t;
    static __device__ __forceinline__ bool alive(S x) { return x >= 0; }
    static __device__ __forceinline__ void cell_frac(S x, const RunInfo& R, int& c, float& f) {
        c = x >> R.fb;
        f = (float)(x & ((1 << R.fb) - 1)) * (float)R.inv_fscale;
    }
    static __device__ __forceinline__ S dead() { return -1; }
};
template <> struct PosT<double> {
    using S = double;
    static __device__ __forceinline__ bool alive(S x) { return x >= 0.0; }
    static __device__ __forceinline__ void cell_frac(S x, const RunInfo& R, int& c, double& f) {
        c = (int)x;
        f = x - (double)c;
    }
    static __device__ __forceinline__ S dead() { return -1.0; }
};

// ---------------------------------------------------------------------------
// Wavefront reductions (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = min(v, __shfl_xor(v, m, 64));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m, 64));
    return v;
}

// CIC deposit of (w0 -> node n, w1 -> node n+1) from every lane into an LDS
// FP64 grid.  When the wave's nodes fall in a window of five (cell-sorted
// particles), the window is summed across the wave first and one lane adds
// it; otherwise each lane adds its own pair.
__device__ __forceinline__ void wave_deposit(double* Ql, bool valid, int n, double w0, double w1) {
    int nmin = wave_min(valid ? n : 0x7fffffff);
    if (nmin == 0x7fffffff) return;
    int nmax = wave_max(valid ? n : -0x7fffffff);
    if (nmax - nmin <= 3) {
        int k = valid ? n - nmin : -10;
        double acc[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            double a = (k == j) ? w0 : 0.0;
            a += (k + 1 == j) ? w1 : 0.0;
            acc[j] = wave_sum(a);
        }
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int j = 0; j < 5; ++j)
                if (acc[j] != 0.0) atomicAdd(&Ql[nmin + j], acc[j]);
        }
    } else if (valid) {
        atomicAdd(&Ql[n], w0);
        atomicAdd(&Ql[n + 1], w1);
    }
}

}  // namespace slpic
