/*
 * slpic_oracle.c -- FP64 CPU oracle for speed-limited PIC (SLPIC), 1D3V.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark.  Plain, slow and written to be checked by
 * eye against the paper; it shares no code with the HIP library.
 *
 * Paper: Werner, Jenkins, Chap & Cary, arXiv:1511.08225.
 *   Sec. II, Eq. (5)       f = beta g  (particles sample g, physical f is beta-weighted)
 *   Sec. II, Eq. (10a,b)   dx/dt = beta v, dv/dt = beta a
 *   Sec. II, Eq. (11a,b)   the two speed-limiting functions
 *   Appendix, Eq. (A1a-d)  electrostatic SLPIC with beta(|v|)
 *   Appendix, Eq. (A2a-d)  leapfrog discretisation; the integral of beta over
 *                          the step in (A2a) is evaluated along the velocity
 *                          path with E frozen at E^n(x^n)
 *
 * Readings where the paper is silent (identical on the GPU side, documented
 * with the design):
 *   - beta_step(|v| = v0) = 1;
 *   - the integral of beta in (A2a) is evaluated exactly along the frozen-field
 *     velocity characteristic (the converged limit of the paper's adaptive
 *     modified-midpoint quadrature, which is available as ORC_KICK_MMP);
 *   - cloud-in-cell weights, node-centred grid, half-volume end nodes,
 *     symmetry plane at x = 0 (specular particles, dphi/dx = 0) and a grounded
 *     absorbing wall at x = L (phi = 0);
 *   - thermal source: pairs balanced by ion loss, uniform in
 *     xt in [0, source_cells), Maxwellian velocity (the source term of g equals
 *     the physical source term once the right-hand side of Eq. (7) is dropped);
 *   - initial load samples g0 = f0/beta with weight dx*Z/ppc, Z = <1/beta>.
 *
 * Parity pins: see tests/test_oracle_*.py (closed forms, limits, brute force).
 */
#include "slpic_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define TWO_PI 6.283185307179586
#define SQRT_2_OVER_PI 0.7978845608028654

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the definition in Salmon, Moraes, Dror & Shaw,        */
/* "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two  */
/* 32x32->64 multiplies with a Weyl-sequence key schedule.                   */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53-bit uniform in [0,1) from two 32-bit words (27 + 26 bits). */
double orc_u53(uint32_t a, uint32_t b) {
    double hi = (double)(a >> 5);
    double lo = (double)(b >> 6);
    return (hi * 67108864.0 + lo) * (1.0 / 9007199254740992.0);
}

/* A per-particle stream of uniforms: counter = (index, step, run, tag|sub);
 * every Philox call yields two uniforms, sub counts the calls. */
typedef struct {
    uint32_t ctr[4];
    uint32_t key[2];
    uint32_t buf[4];
    int pos;
} orc_stream;

static void stream_init(orc_stream* st, const orc_config* cfg, uint32_t index, uint32_t step,
                        int purpose, int species) {
    st->ctr[0] = index;
    st->ctr[1] = step;
    st->ctr[2] = (uint32_t)cfg->run;
    st->ctr[3] = ((uint32_t)purpose << 24) | ((uint32_t)species << 20);
    st->key[0] = (uint32_t)(cfg->seed & 0xffffffffu);
    st->key[1] = (uint32_t)(cfg->seed >> 32);
    st->pos = 4;
}

static double stream_next(orc_stream* st) {
    if (st->pos >= 4) {
        orc_philox4x32_10(st->ctr, st->key, st->buf);
        st->ctr[3] += 1u;
        st->pos = 0;
    }
    double u = orc_u53(st->buf[st->pos], st->buf[st->pos + 1]);
    st->pos += 2;
    return u;
}

/* Three independent standard normals by the Box-Muller transform. */
static void stream_normal3(orc_stream* st, double z[3]) {
    double u1 = stream_next(st);
    double u2 = stream_next(st);
    double r = sqrt(-2.0 * log(1.0 - u1));
    double th = TWO_PI * u2;
    z[0] = r * cos(th);
    z[1] = r * sin(th);
    double u3 = stream_next(st);
    double u4 = stream_next(st);
    double r2 = sqrt(-2.0 * log(1.0 - u3));
    z[2] = r2 * cos(TWO_PI * u4);
}

/* ------------------------------------------------------------------------ */
/* beta, Eq. (11a) and Eq. (11b).                                           */
/* ------------------------------------------------------------------------ */
static double beta_of_s2(int kind, double u, double s2) {
    if (isinf(u)) return 1.0;
    if (kind == ORC_BETA_SMOOTH) return 1.0 / sqrt(1.0 + s2 / (u * u)); /* Eq. (11a) */
    /* Eq. (11b), with beta = 1 on the boundary |v| = v0 */
    if (s2 <= u * u) return 1.0;
    return u / sqrt(s2);
}

double orc_beta(int kind, double u, double speed) { return beta_of_s2(kind, u, speed * speed); }

/* |v|^2 = vx^2 + (vy^2 + vz^2): the perpendicular part is a constant of the
 * 1D motion, so it is summed first. */
static double norm2(const double v[3]) { return v[0] * v[0] + (v[1] * v[1] + v[2] * v[2]); }

/* ------------------------------------------------------------------------ */
/* The velocity update of Eq. (A2a).                                        */
/*                                                                          */
/* With a = (q/m) E^n(x^n) frozen over the step, Eq. (A1b) moves v along    */
/* the line through v parallel to a: write v = vperp + p ahat with c =      */
/* |vperp| fixed; then dp/dt = |a| beta(sqrt(p^2 + c^2)).  Where beta = 1   */
/* the motion is dp/dt = |a|.  Where beta = v0/|v| (Eq. 11b, fast) or       */
/* v0/sqrt(|v|^2 + v0^2) (Eq. 11a, with c^2 -> c^2 + v0^2),                 */
/*   sqrt(p^2 + c^2) dp = |a| v0 dt,                                        */
/* whose antiderivative is G_c(p) = (p sqrt(p^2+c^2) + c^2 asinh(p/c))/2.   */
/* The integral of beta over the step is then (p_end - p_start)/|a|.        */
/* ------------------------------------------------------------------------ */
double orc_G(double c2, double p) {
    if (c2 == 0.0) return 0.5 * p * fabs(p);
    double c = sqrt(c2);
    return 0.5 * (p * sqrt(p * p + c2) + c2 * asinh(p / c));
}

/* p1 >= p0 with G_c(p1) - G_c(p0) = K (K >= 0): Newton on the monotone G,
 * safeguarded by bisection inside a bracket.  Upper bounds: sqrt(p^2+c^2)
 * >= |p| gives the c = 0 solution, sqrt(p^2+c^2) >= c gives p0 + K/c. */
double orc_fast_advance(double c2, double p0, double K) {
    if (!(K > 0.0)) return p0;
    double Gt = orc_G(c2, p0) + K;
    double Q = 0.5 * p0 * fabs(p0) + K;
    double hi = (Q >= 0.0) ? sqrt(2.0 * Q) : -sqrt(-2.0 * Q);
    if (c2 > 0.0) {
        double hi2 = p0 + K / sqrt(c2);
        if (hi2 < hi) hi = hi2;
    }
    double lo = p0;
    double p = hi;
    for (int it = 0; it < 400; ++it) {
        double r = orc_G(c2, p) - Gt;
        if (r == 0.0) return p;
        if (r > 0.0) hi = p; else lo = p;
        double s = sqrt(p * p + c2);
        double pn = (s > 0.0) ? p - r / s : 0.5 * (lo + hi);
        if (!(pn > lo && pn < hi)) pn = 0.5 * (lo + hi);
        double scale = fmax(fabs(lo), fabs(hi));
        if (fabs(pn - p) <= 4.0 * DBL_EPSILON * fabs(pn) || hi - lo <= 4.0 * DBL_EPSILON * scale)
            return pn;
        p = pn;
    }
    return p;
}

void orc_kick_exact(int kind, double u, double dt, const double v[3], const double a[3],
                    double vout[3]) {
    double A2 = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
    if (A2 == 0.0) {
        vout[0] = v[0]; vout[1] = v[1]; vout[2] = v[2];
        return;
    }
    if (isinf(u)) { /* beta == 1: standard leapfrog, Eq. (4) */
        vout[0] = v[0] + a[0] * dt;
        vout[1] = v[1] + a[1] * dt;
        vout[2] = v[2] + a[2] * dt;
        return;
    }
    double u2 = u * u;
    if (kind == ORC_BETA_STEP && norm2(v) <= u2) {
        /* |v|^2 is convex along the straight velocity path: if both ends of
         * the unlimited trial step are inside the band, beta = 1 throughout */
        double vt[3] = {v[0] + a[0] * dt, v[1] + a[1] * dt, v[2] + a[2] * dt};
        if (norm2(vt) <= u2) {
            vout[0] = vt[0]; vout[1] = vt[1]; vout[2] = vt[2];
            return;
        }
    }
    double A = sqrt(A2);
    double ah[3] = {a[0] / A, a[1] / A, a[2] / A};
    double p0 = v[0] * ah[0] + v[1] * ah[1] + v[2] * ah[2];
    double vp[3] = {v[0] - p0 * ah[0], v[1] - p0 * ah[1], v[2] - p0 * ah[2]};
    double c2 = vp[0] * vp[0] + (vp[1] * vp[1] + vp[2] * vp[2]);
    double p1;
    if (kind == ORC_BETA_SMOOTH) {
        p1 = orc_fast_advance(c2 + u2, p0, A * u * dt);
    } else if (c2 >= u2) {
        p1 = orc_fast_advance(c2, p0, A * u * dt);
    } else {
        /* Eq. (11b): fast approaching the band, slow inside |p| <= ps, fast leaving */
        double ps = sqrt(u2 - c2);
        double p = p0;
        double rem = dt;
        int done = 0;
        p1 = p0;
        if (p < -ps) {
            double Kneed = orc_G(c2, -ps) - orc_G(c2, p);
            double Kav = A * u * rem;
            if (Kneed >= Kav) {
                p1 = orc_fast_advance(c2, p, Kav);
                done = 1;
            } else {
                rem -= Kneed / (A * u);
                p = -ps;
            }
        }
        if (!done && p <= ps) {
            double tb = (ps - p) / A;
            if (tb >= rem) {
                p1 = p + A * rem;
                done = 1;
            } else {
                rem -= tb;
                p = ps;
            }
        }
        if (!done) p1 = orc_fast_advance(c2, p, A * u * rem);
    }
    vout[0] = vp[0] + ah[0] * p1;
    vout[1] = vp[1] + ah[1] * p1;
    vout[2] = vp[2] + ah[2] * p1;
}

/* The paper's own quadrature (Appendix): the modified midpoint method
 * applied to dv/dt = beta(|v|) a, dI/dt = beta(|v|), with the number of
 * substeps doubled until I (the integral of beta over the step) changes by
 * at most tol relative; then v^{n+1/2} = v^{n-1/2} + a I as in Eq. (A2a).
 * Returns the number of substeps used. */
static void mmp_rhs(int kind, double u, const double a[3], const double y[4], double f[4]) {
    double b = beta_of_s2(kind, u, norm2(y));
    f[0] = b * a[0];
    f[1] = b * a[1];
    f[2] = b * a[2];
    f[3] = b;
}

int orc_kick_mmp(int kind, double u, double dt, const double v[3], const double a[3], double tol,
                 int nmax, double vout[3]) {
    double y0[4] = {v[0], v[1], v[2], 0.0};
    double prev = 0.0, I = 0.0;
    int n;
    for (n = 2; n <= nmax; n *= 2) {
        double h = dt / n;
        double z0[4], z1[4], z2[4], f[4];
        memcpy(z0, y0, sizeof z0);
        mmp_rhs(kind, u, a, z0, f);
        for (int k = 0; k < 4; ++k) z1[k] = z0[k] + h * f[k];
        for (int m = 1; m < n; ++m) {
            mmp_rhs(kind, u, a, z1, f);
            for (int k = 0; k < 4; ++k) z2[k] = z0[k] + 2.0 * h * f[k];
            memcpy(z0, z1, sizeof z0);
            memcpy(z1, z2, sizeof z1);
        }
        mmp_rhs(kind, u, a, z1, f);
        I = 0.5 * (z1[3] + z0[3] + h * f[3]);
        if (n > 2 && fabs(I - prev) <= tol * fabs(I)) break;
        prev = I;
    }
    if (n > nmax) n = nmax;
    vout[0] = v[0] + a[0] * I;
    vout[1] = v[1] + a[1] * I;
    vout[2] = v[2] + a[2] * I;
    return n;
}

/* ------------------------------------------------------------------------ */
/* Loading g0 = f0/beta (Eq. 5) and the thermal source.                      */
/* ------------------------------------------------------------------------ */

/* Maxwell speed density (units of vt): sqrt(2/pi) s^2 exp(-s^2/2). */
static double maxwell_speed_pdf(double s) { return SQRT_2_OVER_PI * s * s * exp(-0.5 * s * s); }

/* Z = <1/beta> over the Maxwellian.  Eq. (11b): closed form from the split
 * at s = ut (slow part is the Maxwell mass below ut, fast part integrates
 * s/ut times the density).  Eq. (11a): Simpson quadrature of
 * sqrt(1 + s^2/ut^2) against the Maxwell speed density. */
static void step_mixture(double ut, double* Ps, double* Pf) {
    double e = exp(-0.5 * ut * ut);
    *Ps = erf(ut / sqrt(2.0)) - SQRT_2_OVER_PI * ut * e;
    *Pf = SQRT_2_OVER_PI * (ut * ut + 2.0) * e / ut;
}

double orc_Z(int kind, double ut) {
    if (isinf(ut)) return 1.0;
    if (kind == ORC_BETA_STEP) {
        double Ps, Pf;
        step_mixture(ut, &Ps, &Pf);
        return Ps + Pf;
    }
    const int n = 1 << 17;
    const double smax = 48.0;
    double h = smax / n, sum = 0.0;
    for (int k = 0; k <= n; ++k) {
        double s = k * h;
        double fk = maxwell_speed_pdf(s) * sqrt(1.0 + (s / ut) * (s / ut));
        double wk = (k == 0 || k == n) ? 1.0 : ((k & 1) ? 4.0 : 2.0);
        sum += wk * fk;
    }
    return sum * h / 3.0;
}

static double species_vt(const orc_config* cfg, int s) {
    return sqrt(cfg->species[s].temperature / cfg->species[s].mass);
}

double orc_weight(const orc_config* cfg, int s) {
    double ut = cfg->u / species_vt(cfg, s);
    return cfg->dx * orc_Z(cfg->beta_kind, ut) / (double)cfg->species[s].ppc;
}

/* speed (units of vt) from the g-speed density of Eq. (11b):
 * proportional to s^2 e^{-s^2/2} max(1, s/ut) */
static double sample_g_speed_step(orc_stream* st, double ut) {
    double Ps, Pf;
    step_mixture(ut, &Ps, &Pf);
    double usel = stream_next(st);
    if (usel * (Ps + Pf) < Ps) {
        for (int attempt = 0; attempt < 100000; ++attempt) {
            if (ut <= 1.0) {
                double s = ut * cbrt(stream_next(st));
                double acc = stream_next(st);
                if (acc < exp(-0.5 * s * s)) return s;
            } else {
                double z[3];
                stream_normal3(st, z);
                double s = sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
                if (s <= ut) return s;
            }
        }
        return 0.0;
    }
    /* s^3 e^{-s^2/2} on s > ut: with t = s^2/2, density (t0 + y) e^{-y},
     * y = t - t0 >= 0: an Exp(1) / Gamma(2) mixture with weights t0 : 1 */
    double t0 = 0.5 * ut * ut;
    double uc = stream_next(st);
    double y = -log(1.0 - stream_next(st));
    if (!(uc * (t0 + 1.0) < t0)) {
        double y2 = -log(1.0 - stream_next(st));
        y += y2;
    }
    return sqrt(2.0 * (t0 + y));
}

static double sample_g_speed(orc_stream* st, int kind, double ut) {
    if (kind == ORC_BETA_STEP) return sample_g_speed_step(st, ut);
    /* Eq. (11a): rejection from the Eq. (11b) g-density; the ratio
     * sqrt(1 + s^2/ut^2) / max(1, s/ut) lies in [1, sqrt 2] */
    for (int attempt = 0; attempt < 100000; ++attempt) {
        double s = sample_g_speed_step(st, ut);
        double r = sqrt(1.0 + (s / ut) * (s / ut)) / (sqrt(2.0) * fmax(1.0, s / ut));
        if (stream_next(st) < r) return s;
    }
    return 0.0;
}

void orc_load_particle(const orc_config* cfg, int s, uint32_t i, double out[4]) {
    orc_stream st;
    stream_init(&st, cfg, i, 0u, ORC_PURPOSE_LOAD, s);
    double vt = species_vt(cfg, s);
    out[0] = (double)cfg->nx * stream_next(&st);
    if (out[0] >= (double)cfg->nx) out[0] = nextafter((double)cfg->nx, 0.0); /* rounding onto the wall */
    if (isinf(cfg->u)) {
        double z[3];
        stream_normal3(&st, z);
        out[1] = vt * z[0]; out[2] = vt * z[1]; out[3] = vt * z[2];
        return;
    }
    double sp = sample_g_speed(&st, cfg->beta_kind, cfg->u / vt);
    double mu = 2.0 * stream_next(&st) - 1.0;
    double ph = TWO_PI * stream_next(&st);
    double sn = sqrt(fmax(0.0, 1.0 - mu * mu));
    out[1] = vt * sp * mu;
    out[2] = vt * sp * (sn * cos(ph));
    out[3] = vt * sp * (sn * sin(ph));
}

void orc_inject_particle(const orc_config* cfg, int s, uint32_t k, uint32_t step, double out[4]) {
    orc_stream st;
    stream_init(&st, cfg, k, step, ORC_PURPOSE_INJECT, s);
    double vt = species_vt(cfg, s);
    out[0] = (double)cfg->source_cells * stream_next(&st);
    if (out[0] >= (double)cfg->source_cells) out[0] = nextafter((double)cfg->source_cells, 0.0);
    double z[3];
    stream_normal3(&st, z);
    out[1] = vt * z[0]; out[2] = vt * z[1]; out[3] = vt * z[2];
}

/* ------------------------------------------------------------------------ */
/* Poisson, Eq. (A2d) with eps0 = 1: -phi'' = rho on nodes 0..nx.            */
/* Node 0: symmetry plane, -2(phi1 - phi0)/dx^2 = rho0; node nx: phi = 0.    */
/* rho_j = Q_j / dV_j with dV = dx inside and dx/2 at both end nodes.       */
/* Solved by the Thomas algorithm; E by centred differences, E_0 = 0 and a  */
/* one-sided second-order difference at the wall.                           */
/* ------------------------------------------------------------------------ */
void orc_poisson1d(int32_t nx, double dx, const double* Q, double* phi, double* E) {
    int n = nx; /* unknowns phi_0..phi_{nx-1} */
    double* cp = (double*)malloc(sizeof(double) * (size_t)n);
    double* dp = (double*)malloc(sizeof(double) * (size_t)n);
    double dx2 = dx * dx;
    for (int j = 0; j < n; ++j) {
        double dV = (j == 0) ? 0.5 * dx : dx;
        double rhs = (Q[j] / dV) * dx2;
        double aj = (j == 0) ? 0.0 : -1.0;
        double bj = 2.0;
        double cj = (j == 0) ? -2.0 : -1.0;
        if (j == 0) {
            cp[0] = cj / bj;
            dp[0] = rhs / bj;
        } else {
            double m = bj - aj * cp[j - 1];
            cp[j] = cj / m;
            dp[j] = (rhs - aj * dp[j - 1]) / m;
        }
    }
    phi[nx] = 0.0;
    phi[n - 1] = dp[n - 1];
    for (int j = n - 2; j >= 0; --j) phi[j] = dp[j] - cp[j] * phi[j + 1];
    E[0] = 0.0;
    for (int j = 1; j < nx; ++j) E[j] = -(phi[j + 1] - phi[j - 1]) / (2.0 * dx);
    E[nx] = -(3.0 * phi[nx] - 4.0 * phi[nx - 1] + phi[nx - 2]) / (2.0 * dx);
    free(cp);
    free(dp);
}

/* Poisson with two conducting plates (Sec. IV): phi_0 = 0, phi_nx = bias,   */
/* the interior rows of the three-point stencil solved by the Thomas         */
/* algorithm; E by centred differences inside and one-sided second-order     */
/* differences at both plates.                                              */
void orc_poisson1d_plates(int32_t nx, double dx, const double* Q, double bias, double* phi, double* E) {
    int n = nx - 1; /* unknowns phi_1..phi_{nx-1} */
    double* cp = (double*)malloc(sizeof(double) * (size_t)n);
    double* dp = (double*)malloc(sizeof(double) * (size_t)n);
    double dx2 = dx * dx;
    for (int k = 0; k < n; ++k) {
        int j = k + 1;
        double rhs = (Q[j] / dx) * dx2;
        if (j == nx - 1) rhs += bias;  /* phi_nx = bias moves to the right-hand side */
        double a = (k == 0) ? 0.0 : -1.0, b = 2.0, c = (k == n - 1) ? 0.0 : -1.0;
        if (k == 0) {
            cp[0] = c / b;
            dp[0] = rhs / b;
        } else {
            double m = b - a * cp[k - 1];
            cp[k] = c / m;
            dp[k] = (rhs - a * dp[k - 1]) / m;
        }
    }
    phi[0] = 0.0;
    phi[nx] = bias;
    phi[n] = dp[n - 1];
    for (int k = n - 2; k >= 0; --k) phi[k + 1] = dp[k] - cp[k] * phi[k + 2];
    E[0] = -(-3.0 * phi[0] + 4.0 * phi[1] - phi[2]) / (2.0 * dx);
    for (int j = 1; j < nx; ++j) E[j] = -(phi[j + 1] - phi[j - 1]) / (2.0 * dx);
    E[nx] = -(3.0 * phi[nx] - 4.0 * phi[nx - 1] + phi[nx - 2]) / (2.0 * dx);
    free(cp);
    free(dp);
}

/* Periodic box (plasma-oscillation section): nodes 0..nx-1 with node nx the
 * image of node 0.  The charge of node nx is folded onto node 0, the mean
 * charge (a uniform neutralising background) is removed, and with the gauge
 * phi_0 = 0 periodicity gives phi_nx = 0 too: the rows of nodes 1..nx-1 are
 * then the two-plate system with zero bias (the row of node 0 follows from
 * them because the charge sums to zero).  E by centred differences around
 * the ring; node nx repeats node 0. */
void orc_poisson1d_periodic(int32_t nx, double dx, const double* Q, double* phi, double* E) {
    double* Qp = (double*)calloc((size_t)nx + 1, sizeof(double));
    double tot = 0.0;
    for (int j = 0; j < nx; ++j) {
        Qp[j] = Q[j] + (j == 0 ? Q[nx] : 0.0);
        tot += Qp[j];
    }
    double mean = tot / (double)nx;
    for (int j = 0; j < nx; ++j) Qp[j] -= mean;
    Qp[nx] = 0.0;
    orc_poisson1d_plates(nx, dx, Qp, 0.0, phi, E);
    phi[nx] = phi[0];
    E[0] = -(phi[1] - phi[nx - 1]) / (2.0 * dx);
    for (int j = 1; j < nx; ++j) E[j] = -(phi[j + 1] - phi[j - 1]) / (2.0 * dx);
    E[nx] = E[0];
    free(Qp);
}

double orc_wrap_periodic(double xt, int32_t nx) {
    double L = (double)nx;
    if (xt < 0.0 || xt >= L) {
        xt -= L * floor(xt / L);
        if (xt >= L) xt = 0.0; /* a tiny negative position rounds onto L: its image is 0 */
    }
    if (!(xt >= 0.0 && xt < L)) xt = -1.0; /* no image (a non-finite move): the slot is dropped */
    return xt;
}

/* <(beta v_x)^2>/v_t^2 for the 3D Maxwellian: beta depends on the speed
 * only, so <beta^2 v_x^2> = <beta^2 s^2>/3 over the Maxwell speed density
 * 4 pi s^2 (2 pi vt^2)^(-3/2) exp(-s^2 / 2 vt^2); the speed integral is taken
 * by the composite Simpson rule on [0, 12 vt] with 24000 panels (its tail
 * is below 1e-28), split at s = u for the step form's kink. */
static double simpson_p(double (*f)(double, const double*), const double* p, double a, double b, int n) {
    if (b <= a) return 0.0;
    if (n % 2) n += 1;
    double h = (b - a) / n, sum = f(a, p) + f(b, p);
    for (int i = 1; i < n; ++i) sum += f(a + i * h, p) * ((i % 2) ? 4.0 : 2.0);
    return sum * h / 3.0;
}

static double pf2_integrand(double s, const double* p) {
    /* p = {kind, u, vt} */
    double b = beta_of_s2((int)p[0], p[1], s * s);
    return b * b * s * s / 3.0 * maxwell_speed_pdf(s / p[2]) / p[2];
}

double orc_slpic_plasma_freq2(int kind, double u, double vt) {
    double p[3] = {(double)kind, u, vt};
    double top = 12.0 * vt;
    double val;
    if (isinf(u) || u >= top) {
        val = simpson_p(pf2_integrand, p, 0.0, top, 24000);
    } else {
        int n1 = (int)(24000.0 * u / top) + 2;
        val = simpson_p(pf2_integrand, p, 0.0, u, n1) + simpson_p(pf2_integrand, p, u, top, 24000 - n1 + 2);
    }
    return val / (vt * vt);
}

/* The full long-time dispersion relation of the plasma-oscillation section
 * for 1D perturbations exp(i(kx - wt)) of a uniform Maxwellian (omega_p = 1):
 *   D(w) = 1 - (1/w^2) < (beta^2 + (d beta/d v_x) w/k) / (1 - k beta v_x/w)^2 >.
 * beta depends on the speed s only: v_x = s mu, d beta/d v_x = beta'(s) mu,
 * and the average over the direction cosine mu (uniform on [-1, 1]) is
 * done in closed form with c = k beta(s) s / w < 1:
 *   (1/2) int (A + B mu)/(1 - c mu)^2 dmu = A/(1 - c^2)
 *       + (B/(2c^2)) (2c/(1 - c^2) + ln((1 - c)/(1 + c))),
 * with A = beta(s)^2 and B = beta'(s) w/k; for c < 1e-3 the
 * bracket over c^2 is replaced by its series 4c/3 + 8c^3/5.  The speed integral is
 * the composite Simpson rule on [0, 12 vt] (split at u).  Since beta s <= u
 * for both speed limits, no particle resonates once w > k u, and D rises
 * from -inf (w -> k u) to 1 (w -> inf): the root is found by bisection.
 * For u = inf this is the fluid limit of the resonant relation (no Landau
 * term), used only where k v_t << w. */
static double beta_prime(int kind, double u, double s) {
    if (isinf(u)) return 0.0;
    if (kind == ORC_BETA_SMOOTH) return -(s / (u * u)) * pow(1.0 + s * s / (u * u), -1.5);
    return s <= u ? 0.0 : -u / (s * s);
}

static double disp_integrand(double s, const double* p) {
    /* p = {kind, u, vt, k, w} */
    int kind = (int)p[0];
    double u = p[1], vt = p[2], k = p[3], w = p[4];
    double b = beta_of_s2(kind, u, s * s);
    double A = b * b, B = beta_prime(kind, u, s) * w / k;
    double c = k * b * s / w;
    double mu_avg;
    if (c < 1e-3) {
        mu_avg = A / (1.0 - c * c) + (B / 2.0) * (4.0 * c / 3.0 + 8.0 * c * c * c / 5.0);
    } else {
        mu_avg = A / (1.0 - c * c) + (B / (2.0 * c * c)) * (2.0 * c / (1.0 - c * c) + log((1.0 - c) / (1.0 + c)));
    }
    return mu_avg * maxwell_speed_pdf(s / vt) / vt;
}

static double dispersion_D(int kind, double u, double vt, double k, double w) {
    double p[5] = {(double)kind, u, vt, k, w};
    double top = 12.0 * vt;
    double avg;
    if (isinf(u) || u >= top) {
        avg = simpson_p(disp_integrand, p, 0.0, top, 24000);
    } else {
        int n1 = (int)(24000.0 * u / top) + 2;
        /* the step form's d beta/d|v| jumps at u: the upper piece starts just
         * above it so that its first node takes the right-hand value */
        avg = simpson_p(disp_integrand, p, 0.0, u, n1) +
              simpson_p(disp_integrand, p, nextafter(u, INFINITY), top, 24000 - n1 + 2);
    }
    return 1.0 - avg / (w * w);
}

double orc_slpic_dispersion(int kind, double u, double vt, double k) {
    double vmax = isinf(u) ? 12.0 * vt : u;  /* the largest beta |v| */
    double lo = k * vmax * (1.0 + 1e-12) + 1e-300, hi = 1.0;
    while (dispersion_D(kind, u, vt, k, hi) < 0.0) hi *= 2.0;
    for (int it = 0; it < 200 && hi - lo > 1e-14 * hi; ++it) {
        double mid = 0.5 * (lo + hi);
        if (dispersion_D(kind, u, vt, k, mid) < 0.0) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Expected g-particles entering through the plate at x = L per step: the
 * one-sided flux n0 v_t / sqrt(2 pi) of a stationary Maxwellian (n0 = 1)
 * times dt, over the weight (each entering g-particle carries w physical
 * particles across the plate: its flux beta v g equals v f, Eq. 5). */
double orc_wall_flux_per_step(const orc_config* cfg, int s) {
    return species_vt(cfg, s) / sqrt(TWO_PI) * cfg->dt / orc_weight(cfg, s);
}

/* Particle k entering through the plate at x = L in step `step`: v_x from
 * the flux-weighted half Maxwellian (v_x = -v_t sqrt(-2 ln(1 - U))), v_y, v_z
 * Maxwellian, and a position a uniform fraction of this step's travel
 * beta(|v|) |v_x| dt inside the plate (held within source_cells; beta with
 * the limit at the plate). */
void orc_wall_inject_particle(const orc_config* cfg, int s, uint32_t k, uint32_t step, double out[4]) {
    orc_stream st;
    stream_init(&st, cfg, k, step, ORC_PURPOSE_WALL, s);
    double vt = species_vt(cfg, s);
    double vx = -vt * sqrt(-2.0 * log(1.0 - stream_next(&st)));
    double z[3];
    stream_normal3(&st, z);
    double vy = vt * z[0], vz = vt * z[1];
    double s2 = vx * vx + (vy * vy + vz * vz);
    double ul = cfg->limit ? cfg->limit[cfg->nx] : cfg->u;
    double depth = beta_of_s2(cfg->beta_kind, ul, s2) * fabs(vx) * cfg->dt / cfg->dx * stream_next(&st);
    if (depth > (double)cfg->source_cells) depth = (double)cfg->source_cells;
    double x = (double)cfg->nx - depth;
    if (x >= (double)cfg->nx) x = nextafter((double)cfg->nx, 0.0);
    out[0] = x; out[1] = vx; out[2] = vy; out[3] = vz;
}

/* ------------------------------------------------------------------------ */
/* A run: particle slots (dead slots have xt < 0 until compaction), grids.   */
/* ------------------------------------------------------------------------ */
/* ---------------------------------------------------------------- steady */
void orc_steady_init(orc_steady* d, int32_t window, double tol) {
    memset(d, 0, sizeof *d);
    d->window = window;
    d->tol = tol;
    d->steady_step = -1;
}

void orc_steady_feed(orc_steady* d, double phi_w, int64_t step_count) {
    d->sum += phi_w;
    d->nopen += 1;
    if (d->nopen < d->window) return;
    double m = d->sum / (double)d->window;
    d->mean[2] = d->mean[1];
    d->mean[1] = d->mean[0];
    d->mean[0] = m;
    d->nwin += 1;
    d->sum = 0.0;
    d->nopen = 0;
    if (d->nwin >= 3 && d->steady_step < 0) {
        double avg = (d->mean[0] + d->mean[1] + d->mean[2]) / 3.0;
        double dev = 0.0;
        for (int k = 0; k < 3; ++k) {
            double e = fabs(d->mean[k] - avg);
            if (e > dev) dev = e;
        }
        if (dev <= d->tol * fabs(avg)) d->steady_step = step_count;
    }
}

struct orc_run {
    orc_steady steady;
    orc_config cfg;
    double* U;  /* nodes of a position-dependent speed limit (NULL: uniform) */
    double w[2], qw[2], qm[2], vt[2];
    int64_t n[2], cap[2];
    double *x[2], *vx[2], *vy[2], *vz[2];
    double *Q[2], *phi, *E;
    double acc_e;
    double acc_flux[2];  /* plates: fractional g-particles carried per species */
    int64_t step;
    int64_t absorbed_total[2], injected_total[2];
};

static void ensure_capacity(orc_run* r, int s, int64_t need) {
    if (need <= r->cap[s]) return;
    int64_t cap = r->cap[s] > 0 ? r->cap[s] : 16;
    while (cap < need) cap *= 2;
    r->x[s] = (double*)realloc(r->x[s], sizeof(double) * (size_t)cap);
    r->vx[s] = (double*)realloc(r->vx[s], sizeof(double) * (size_t)cap);
    r->vy[s] = (double*)realloc(r->vy[s], sizeof(double) * (size_t)cap);
    r->vz[s] = (double*)realloc(r->vz[s], sizeof(double) * (size_t)cap);
    r->cap[s] = cap;
}

/* The speed limit at position xt (grid units) of a run: the node values of
 * its limit profile interpolated linearly, or the uniform limit u. */
static double run_limit(const orc_run* r, double xt) {
    if (!r->U) return r->cfg.u;
    int c = (int)floor(xt);
    if (c < 0) c = 0;
    if (c > r->cfg.nx - 1) c = r->cfg.nx - 1;
    double f = xt - (double)c;
    return r->U[c] * (1.0 - f) + r->U[c + 1] * f;
}

/* The speed limit at the centre of cell c of a configuration (the loaders). */
static double cell_limit(const orc_config* cfg, int32_t c) {
    return cfg->limit ? 0.5 * (cfg->limit[c] + cfg->limit[c + 1]) : cfg->u;
}

orc_run* orc_create(const orc_config* cfg) {
    if (cfg->limit) {  /* finite positive nodes */
        if (!isfinite(cfg->u)) return NULL;
        for (int j = 0; j <= cfg->nx; ++j)
            if (!(cfg->limit[j] > 0.0) || !isfinite(cfg->limit[j])) return NULL;
    }
    orc_run* r = (orc_run*)calloc(1, sizeof(orc_run));
    r->cfg = *cfg;
    if (cfg->limit) {  /* the run keeps its own copy of the limit profile */
        r->U = (double*)malloc(sizeof(double) * (size_t)(cfg->nx + 1));
        memcpy(r->U, cfg->limit, sizeof(double) * (size_t)(cfg->nx + 1));
        r->cfg.limit = r->U;
    }
    orc_steady_init(&r->steady, cfg->steady_window > 0 ? cfg->steady_window : (cfg->nx / 4 > 1 ? cfg->nx / 4 : 1),
                    cfg->steady_tol > 0.0 ? cfg->steady_tol : 0.02);
    int nodes = cfg->nx + 1;
    for (int s = 0; s < cfg->nspecies; ++s) {
        r->vt[s] = species_vt(cfg, s);
        r->w[s] = orc_weight(cfg, s);
        r->qw[s] = cfg->species[s].charge * r->w[s];
        r->qm[s] = cfg->species[s].charge / cfg->species[s].mass;
        r->Q[s] = (double*)calloc((size_t)nodes, sizeof(double));
        int64_t n0 = (int64_t)cfg->nx * cfg->species[s].ppc;
        double cf = cfg->capacity_factor > 1.0 ? cfg->capacity_factor : 1.0;
        ensure_capacity(r, s, (int64_t)ceil(cf * (double)n0) + 1);
    }
    r->phi = (double*)calloc((size_t)nodes, sizeof(double));
    r->E = (double*)calloc((size_t)nodes, sizeof(double));
    return r;
}

void orc_destroy(orc_run* r) {
    if (!r) return;
    for (int s = 0; s < 2; ++s) {
        free(r->x[s]); free(r->vx[s]); free(r->vy[s]); free(r->vz[s]); free(r->Q[s]);
    }
    free(r->phi);
    free(r->E);
    free(r->U);
    free(r);
}

/* Eq. (A2c): Q_j = sum_p q w beta(|v^{n+1/2}|) W_j(x^{n+1}) with CIC W (a
 * limit varying with position: beta with the limit at x^{n+1}). */
static void deposit(orc_run* r) {
    int nodes = r->cfg.nx + 1;
    for (int s = 0; s < r->cfg.nspecies; ++s) {
        memset(r->Q[s], 0, sizeof(double) * (size_t)nodes);
        for (int64_t i = 0; i < r->n[s]; ++i) {
            double xt = r->x[s][i];
            if (xt < 0.0) continue;
            double v[3] = {r->vx[s][i], r->vy[s][i], r->vz[s][i]};
            double b = beta_of_s2(r->cfg.beta_kind, run_limit(r, xt), norm2(v));
            int c = (int)floor(xt);
            double f = xt - (double)c;
            double wb = r->qw[s] * b;
            r->Q[s][c] += wb * (1.0 - f);
            r->Q[s][c + 1] += wb * f;
        }
    }
}

static void solve_fields(orc_run* r) {
    int nodes = r->cfg.nx + 1;
    double* Qt = (double*)calloc((size_t)nodes, sizeof(double));
    for (int j = 0; j < nodes; ++j)
        for (int s = 0; s < r->cfg.nspecies; ++s) Qt[j] += r->Q[s][j];
    if (r->cfg.geometry == ORC_GEOM_PLATES)
        orc_poisson1d_plates(r->cfg.nx, r->cfg.dx, Qt, r->cfg.bias, r->phi, r->E);
    else if (r->cfg.geometry == ORC_GEOM_PERIODIC)
        orc_poisson1d_periodic(r->cfg.nx, r->cfg.dx, Qt, r->phi, r->E);
    else
        orc_poisson1d(r->cfg.nx, r->cfg.dx, Qt, r->phi, r->E);
    free(Qt);
}

void orc_refresh_fields(orc_run* r) {
    deposit(r);
    solve_fields(r);
}

void orc_keys(const orc_run* r, int32_t s, int32_t* keys) {
    int b = r->cfg.sort_bucket;
    for (int64_t i = 0; i < r->n[s]; ++i) {
        double xt = r->x[s][i];
        if (xt < 0.0) keys[i] = -1;
        else keys[i] = (b > 0) ? (int32_t)floor(xt) / b : 0;
    }
}

/* Stable counting sort by key, dead slots dropped; perm[new] = old. */
void orc_sort(orc_run* r, int32_t* perm0, int32_t* perm1) {
    for (int s = 0; s < r->cfg.nspecies; ++s) {
        int64_t n = r->n[s];
        int32_t* keys = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
        orc_keys(r, s, keys);
        int nkeys = (r->cfg.sort_bucket > 0) ? (r->cfg.nx + r->cfg.sort_bucket - 1) / r->cfg.sort_bucket : 1;
        int64_t* start = (int64_t*)calloc((size_t)nkeys + 1, sizeof(int64_t));
        for (int64_t i = 0; i < n; ++i)
            if (keys[i] >= 0) start[keys[i] + 1] += 1;
        for (int k = 0; k < nkeys; ++k) start[k + 1] += start[k];
        int64_t nlive = start[nkeys];
        double* nx_ = (double*)malloc(sizeof(double) * (size_t)(nlive + 1));
        double* nvx = (double*)malloc(sizeof(double) * (size_t)(nlive + 1));
        double* nvy = (double*)malloc(sizeof(double) * (size_t)(nlive + 1));
        double* nvz = (double*)malloc(sizeof(double) * (size_t)(nlive + 1));
        int32_t* perm = (s == 0) ? perm0 : perm1;
        for (int64_t i = 0; i < n; ++i) {
            if (keys[i] < 0) continue;
            int64_t d = start[keys[i]]++;
            nx_[d] = r->x[s][i];
            nvx[d] = r->vx[s][i];
            nvy[d] = r->vy[s][i];
            nvz[d] = r->vz[s][i];
            if (perm) perm[d] = (int32_t)i;
        }
        memcpy(r->x[s], nx_, sizeof(double) * (size_t)nlive);
        memcpy(r->vx[s], nvx, sizeof(double) * (size_t)nlive);
        memcpy(r->vy[s], nvy, sizeof(double) * (size_t)nlive);
        memcpy(r->vz[s], nvz, sizeof(double) * (size_t)nlive);
        r->n[s] = nlive;
        free(nx_); free(nvx); free(nvy); free(nvz); free(start); free(keys);
    }
}

static int load_cells(orc_run* r, const double* profile);

void orc_load(orc_run* r) {
    if (r->U && r->cfg.geometry != ORC_GEOM_PLATES) {
        /* g0 = f0/beta with the limit of each cell: cell by cell, at n0 = 1 and rest */
        double* uni = (double*)calloc(7 * 256, sizeof(double));
        for (int k = 0; k < 256; ++k) uni[256 + k] = uni[512 + k] = 1.0;
        load_cells(r, uni);
        free(uni);
        return;
    }
    for (int s = 0; s < r->cfg.nspecies; ++s) {
        int64_t n0 = r->cfg.geometry == ORC_GEOM_PLATES ? 0 : (int64_t)r->cfg.nx * r->cfg.species[s].ppc;
        ensure_capacity(r, s, n0);
        for (int64_t i = 0; i < n0; ++i) {
            double p[4];
            orc_load_particle(&r->cfg, s, (uint32_t)i, p);
            r->x[s][i] = p[0]; r->vx[s][i] = p[1]; r->vy[s][i] = p[2]; r->vz[s][i] = p[3];
        }
        r->n[s] = n0;
    }
    r->step = 0;
    r->acc_e = 0.0;
    r->acc_flux[0] = r->acc_flux[1] = 0.0;
    if (r->cfg.sort_every > 0) orc_sort(r, NULL, NULL);
    orc_refresh_fields(r);
}

/* ------------------------------------------------------------------------ */
/* Warm load from predicted steady profiles (a reading; the paper loads     */
/* cold).  profile: 7 x 256 values on x/L = k/255: phi, n_e, n_i, Gamma_e,    */
/* Gamma_i, T_e, T_i (physical; T in T_e units).  In cell c (centre x/L =    */
/* (c + 1/2)/nx), species s: n, Gamma and T by linear interpolation (n       */
/* clamped at 0; T not positive: the species' source temperature), thermal  */
/* speed vt = sqrt(T/m), drift V = Gamma/n clamped to |V| <= 4 vt,           */
/* f = n Maxwellian(V e_x, vt) and                                          */
/* g = f/beta (Eq. 5): the cell holds E = n dx Z / w g-particles, Z = <1/beta> */
/* over the drifting Maxwellian, w the run's constant weight; the count is   */
/* floor(E) + [U < frac(E)].  Positions uniform in the cell; velocities from */
/* f/beta by rejection from the drifting Maxwellian against                  */
/* M = 1/beta(|V| + 8 vt) (a proposal beyond 8 vt is accepted).  Particles   */
/* are stored cell by cell.                                                  */
/* ------------------------------------------------------------------------ */
static double inv_beta(int kind, double u, double s) {
    if (isinf(u)) return 1.0;
    if (kind == ORC_BETA_SMOOTH) return sqrt(1.0 + (s / u) * (s / u));
    return s <= u ? 1.0 : s / u;
}

/* Density of |v| for v = V e_x + vt z (z standard normal in 3D):
 * p(s) = s/(vt sqrt(2 pi)) exp(-(s - V)^2 / (2 vt^2)) (1 - exp(-2 s V / vt^2)) / V,
 * whose V -> 0 limit is the Maxwell speed density. */
static double drift_speed_density(double s, double V, double vt) {
    double a = s / (vt * sqrt(TWO_PI)) * exp(-(s - V) * (s - V) / (2.0 * vt * vt));
    double q = 2.0 * s * V / (vt * vt);
    double f = q > 1e-300 ? -expm1(-q) / V : 2.0 * s / (vt * vt);
    return a * f;
}

/* Z = <1/beta> over the drifting Maxwellian: composite Simpson, 4096 panels,
 * on [lo, hi] with hi = |V| + 12 vt (beyond: < 1e-30 of the mass); for the
 * step form the integrand is 1 below u, so Z = 1 + int_u^hi (s/u - 1) p. */
static double warm_Z(int kind, double u, double V, double vt) {
    if (isinf(u)) return 1.0;
    V = fabs(V);
    double hi = V + 12.0 * vt;
    int n = 4096;
    double lo = 0.0;
    if (kind == ORC_BETA_STEP) {
        if (u >= hi) return 1.0;
        lo = u;
    }
    double h = (hi - lo) / n, acc = 0.0;
    for (int k = 0; k <= n; ++k) {
        double s = lo + h * k;
        double g = (kind == ORC_BETA_STEP) ? (s / u - 1.0) : sqrt(1.0 + (s / u) * (s / u));
        double w = (k == 0 || k == n) ? 1.0 : ((k & 1) ? 4.0 : 2.0);
        acc += w * g * drift_speed_density(s, V, vt);
    }
    acc *= h / 3.0;
    return kind == ORC_BETA_STEP ? 1.0 + acc : acc;
}

static double interp_profile(const double* p, double xi) {
    double t = xi * 255.0;
    int k = (int)floor(t);
    if (k < 0) k = 0;
    if (k > 254) k = 254;
    double f = t - (double)k;
    return p[k] * (1.0 - f) + p[k + 1] * f;
}

/* The thermal speed of cell c of a warm load: sqrt(T/m) from the profile's
 * temperature row of species s at the cell centre, or the species' own
 * (source) temperature where that row is not positive. */
double orc_warm_cell_vt(const orc_config* cfg, int s, const double* profile, int32_t c) {
    double T = interp_profile(profile + 256 * (5 + s), ((double)c + 0.5) / (double)cfg->nx);
    return T > 0.0 ? sqrt(T / cfg->species[s].mass) : species_vt(cfg, s);
}

int64_t orc_warm_cell_count(const orc_config* cfg, int s, const double* profile, int32_t c, double w,
                            double* V_out, double* vt_out) {
    double vt = orc_warm_cell_vt(cfg, s, profile, c);
    double xi = ((double)c + 0.5) / (double)cfg->nx;
    const double* pn = profile + 256 * (s == 0 ? 1 : 2);
    const double* pg = profile + 256 * (s == 0 ? 3 : 4);
    double n = interp_profile(pn, xi);
    if (!(n > 0.0)) n = 0.0;
    double G = interp_profile(pg, xi);
    double V = n > 0.0 ? G / n : 0.0;
    if (V > 4.0 * vt) V = 4.0 * vt;
    if (V < -4.0 * vt) V = -4.0 * vt;
    if (V_out) *V_out = V;
    if (vt_out) *vt_out = vt;
    double E = n * cfg->dx * warm_Z(cfg->beta_kind, cell_limit(cfg, c), V, vt) / w;
    double fl = floor(E);
    orc_stream st;
    stream_init(&st, cfg, (uint32_t)c, 0u, ORC_PURPOSE_WARM_COUNT, s);
    return (int64_t)fl + (stream_next(&st) < E - fl ? 1 : 0);
}

void orc_warm_particle(const orc_config* cfg, int s, uint32_t i, int32_t c, double V, double vt, double out[4]) {
    orc_stream st;
    stream_init(&st, cfg, i, 0u, ORC_PURPOSE_WARM, s);
    double u = cell_limit(cfg, c);
    out[0] = (double)c + stream_next(&st);
    if (out[0] >= (double)(c + 1)) out[0] = nextafter((double)(c + 1), 0.0);
    double M = inv_beta(cfg->beta_kind, u, fabs(V) + 8.0 * vt);
    double v[3] = {V, 0.0, 0.0};
    for (int attempt = 0; attempt < 100000; ++attempt) {
        double z[3];
        stream_normal3(&st, z);
        v[0] = V + vt * z[0];
        v[1] = vt * z[1];
        v[2] = vt * z[2];
        double sp = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        double w = inv_beta(cfg->beta_kind, u, sp);
        if (w >= M || stream_next(&st) * M < w) break;
    }
    out[1] = v[0]; out[2] = v[1]; out[3] = v[2];
}

int orc_load_warm(orc_run* r, const double* profile) { return load_cells(r, profile); }

static int load_cells(orc_run* r, const double* profile) {
    for (int s = 0; s < r->cfg.nspecies; ++s) {
        int64_t i = 0;
        for (int32_t c = 0; c < r->cfg.nx; ++c) {
            double V, vt;
            int64_t cnt = orc_warm_cell_count(&r->cfg, s, profile, c, r->w[s], &V, &vt);
            ensure_capacity(r, s, i + cnt);
            for (int64_t k = 0; k < cnt; ++k, ++i) {
                double p[4];
                orc_warm_particle(&r->cfg, s, (uint32_t)i, c, V, vt, p);
                r->x[s][i] = p[0]; r->vx[s][i] = p[1]; r->vy[s][i] = p[2]; r->vz[s][i] = p[3];
            }
        }
        r->n[s] = i;
    }
    r->step = 0;
    r->acc_e = 0.0;
    if (r->cfg.sort_every > 0) orc_sort(r, NULL, NULL);
    orc_refresh_fields(r);
    return 0;
}

static void inject(orc_run* r, int s, int64_t count) {
    ensure_capacity(r, s, r->n[s] + count);
    for (int64_t k = 0; k < count; ++k) {
        double p[4];
        orc_inject_particle(&r->cfg, s, (uint32_t)k, (uint32_t)r->step, p);
        int64_t i = r->n[s] + k;
        r->x[s][i] = p[0]; r->vx[s][i] = p[1]; r->vy[s][i] = p[2]; r->vz[s][i] = p[3];
    }
    r->n[s] += count;
    r->injected_total[s] += count;
}

/* The quantity the steady detector and the history watch: Phi_w = phi(0) -
 * phi(L) for the sheath; for the plates, whose end potentials are fixed, phi
 * at the mid-plane node; for the periodic box, the amplitude of the
 * fundamental sin(2 pi x/L) mode of E, (2/nx) sum_j E_j sin(2 pi j/nx) (the
 * field of a cos(2 pi x/L) density perturbation). */
static double orc_monitor_potential(const orc_run* r) {
    if (r->cfg.geometry == ORC_GEOM_PLATES) return r->phi[r->cfg.nx / 2];
    if (r->cfg.geometry == ORC_GEOM_PERIODIC) {
        double a = 0.0;
        for (int j = 0; j < r->cfg.nx; ++j) a += r->E[j] * sin(TWO_PI * (double)j / (double)r->cfg.nx);
        return 2.0 * a / (double)r->cfg.nx;
    }
    return r->phi[0] - r->phi[r->cfg.nx];
}

double orc_monitor(const orc_run* r) { return orc_monitor_potential(r); }
double orc_run_weight(const orc_run* r, int32_t s) { return r->w[s]; }

/* A new speed limit mid-run (the paper allows the limit to vary in time, to
 * adjust the approximation during a simulation).  The physical distribution
 * f = beta g is kept: the species weight becomes that of a fresh load at
 * the new limit, w' = dx Z(u')/ppc, and each live g-particle of velocity v,
 * in slot order, is replaced by m copies, m = floor(p) + [U < p - floor(p)]
 * with p = (beta_u(|v|) w) / (beta_u'(|v|) w'), so that the expected
 * beta' w' g' equals beta w g at every velocity.  A raise has beta' >= beta
 * and p <= w/w'; a lowering has p <= (beta/beta') (w/w'), a ratio of order
 * |v| / <|v|> for the fast particles, and the slow ones (beta' = beta) are
 * thinned by w/w' < 1.  m is capped at 255 copies.  U is the first draw of
 * the particle's own stream (purpose 6, its slot index, the current step).
 * Then dt becomes dt' and the charge and fields are recomputed.  A run with
 * a limit profile keeps it (-1). */
int orc_set_speed_limit(orc_run* r, double u_new, double dt_new) {
    orc_config nc = r->cfg;
    if (!(u_new > 0.0) || !(dt_new > 0.0) || r->U) return -1;
    nc.u = u_new;
    nc.dt = dt_new;
    for (int s = 0; s < r->cfg.nspecies; ++s) {
        double w_old = r->w[s], w_new = orc_weight(&nc, s);
        int64_t n = r->n[s], total = 0;
        int32_t* m = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
        for (int64_t i = 0; i < n; ++i) {
            if (r->x[s][i] < 0.0) continue;
            double v[3] = {r->vx[s][i], r->vy[s][i], r->vz[s][i]};
            double s2 = norm2(v);
            double p = (beta_of_s2(r->cfg.beta_kind, r->cfg.u, s2) * w_old) /
                       (beta_of_s2(r->cfg.beta_kind, u_new, s2) * w_new);
            orc_stream st;
            stream_init(&st, &r->cfg, (uint32_t)i, (uint32_t)r->step, ORC_PURPOSE_LIMIT, s);
            double fl = floor(p);
            int64_t c = (int64_t)fl + (stream_next(&st) < p - fl ? 1 : 0);
            m[i] = (int32_t)(c < 255 ? c : 255);
            total += m[i];
        }
        double* nxs = (double*)malloc(sizeof(double) * (size_t)(total + 1));
        double* nvx = (double*)malloc(sizeof(double) * (size_t)(total + 1));
        double* nvy = (double*)malloc(sizeof(double) * (size_t)(total + 1));
        double* nvz = (double*)malloc(sizeof(double) * (size_t)(total + 1));
        int64_t k = 0;
        for (int64_t i = 0; i < n; ++i)
            for (int32_t c = 0; c < m[i]; ++c, ++k) {
                nxs[k] = r->x[s][i]; nvx[k] = r->vx[s][i]; nvy[k] = r->vy[s][i]; nvz[k] = r->vz[s][i];
            }
        ensure_capacity(r, s, total + 1);
        memcpy(r->x[s], nxs, sizeof(double) * (size_t)total);
        memcpy(r->vx[s], nvx, sizeof(double) * (size_t)total);
        memcpy(r->vy[s], nvy, sizeof(double) * (size_t)total);
        memcpy(r->vz[s], nvz, sizeof(double) * (size_t)total);
        r->n[s] = total;
        free(nxs); free(nvx); free(nvy); free(nvz); free(m);
        r->w[s] = w_new;
        r->qw[s] = r->cfg.species[s].charge * w_new;
    }
    r->cfg = nc;
    orc_refresh_fields(r);
    return 0;
}

/* One step of Eq. (A2a-d). */
void orc_step(orc_run* r, int32_t nsteps) {
    const orc_config* cfg = &r->cfg;
    double dtdx = cfg->dt / cfg->dx;
    for (int32_t it = 0; it < nsteps; ++it) {
        int64_t absorbed[2] = {0, 0};
        for (int s = 0; s < cfg->nspecies; ++s) {
            for (int64_t i = 0; i < r->n[s]; ++i) {
                double xt = r->x[s][i];
                if (xt < 0.0) continue;
                /* gather E^n(x^n), CIC */
                int c = (int)floor(xt);
                double f = xt - (double)c;
                double Ex = r->E[c] * (1.0 - f) + r->E[c + 1] * f;
                double a[3] = {r->qm[s] * Ex, 0.0, 0.0};
                double v[3] = {r->vx[s][i], r->vy[s][i], r->vz[s][i]};
                double v1[3];
                /* the speed limit of the step: at x^n, frozen like E^n(x^n) */
                double up = run_limit(r, xt);
                if (cfg->kick == ORC_KICK_MMP)
                    orc_kick_mmp(cfg->beta_kind, up, cfg->dt, v, a, cfg->mmp_tol, 1 << 20, v1);
                else
                    orc_kick_exact(cfg->beta_kind, up, cfg->dt, v, a, v1);
                /* Eq. (A2b): x^{n+1} = x^n + beta(|v^{n+1/2}|) v^{n+1/2} dt */
                double b = beta_of_s2(cfg->beta_kind, up, norm2(v1));
                double xn = xt + b * v1[0] * dtdx;
                int left_out = 0;
                if (cfg->geometry == ORC_GEOM_PERIODIC) {
                    xn = orc_wrap_periodic(xn, cfg->nx);
                } else if (xn < 0.0) {
                    if (cfg->geometry == ORC_GEOM_PLATES) {
                        left_out = 1; /* absorbing plate */
                    } else {      /* symmetry plane: specular reflection */
                        xn = -xn;
                        v1[0] = -v1[0];
                    }
                }
                r->vx[s][i] = v1[0];
                r->vy[s][i] = v1[1];
                r->vz[s][i] = v1[2];
                if (left_out || xn >= (double)cfg->nx) { /* absorbing wall */
                    r->x[s][i] = -1.0;
                    absorbed[s] += 1;
                } else {
                    r->x[s][i] = xn;
                }
            }
            r->absorbed_total[s] += absorbed[s];
        }
        if (cfg->geometry == ORC_GEOM_PLATES) {
            /* flux injection through the plate at x = L, both species */
            for (int s = 0; s < cfg->nspecies; ++s) {
                r->acc_flux[s] += orc_wall_flux_per_step(cfg, s);
                int64_t m = (int64_t)floor(r->acc_flux[s]);
                r->acc_flux[s] -= (double)m;
                ensure_capacity(r, s, r->n[s] + m);
                for (int64_t k = 0; k < m; ++k) {
                    double p[4];
                    orc_wall_inject_particle(cfg, s, (uint32_t)k, (uint32_t)r->step, p);
                    int64_t i = r->n[s] + k;
                    r->x[s][i] = p[0]; r->vx[s][i] = p[1]; r->vy[s][i] = p[2]; r->vz[s][i] = p[3];
                }
                r->n[s] += m;
                r->injected_total[s] += m;
            }
        } else if (cfg->nspecies == 2 && cfg->geometry == ORC_GEOM_SHEATH) {
            /* thermal source: ion-loss-balanced pairs */
            int64_t ni = absorbed[1];
            r->acc_e += (double)ni * (r->w[1] / r->w[0]);
            int64_t ne = (int64_t)floor(r->acc_e);
            r->acc_e -= (double)ne;
            inject(r, 1, ni);
            inject(r, 0, ne);
        }
        deposit(r);
        solve_fields(r);
        r->step += 1;
        orc_steady_feed(&r->steady, orc_monitor_potential(r), r->step);
        if (cfg->sort_every > 0 && r->step % cfg->sort_every == 0) orc_sort(r, NULL, NULL);
    }
}

/* beta-weighted moments at nodes: phi, then per species density n,
 * flux Gamma_x = sum w beta vx W / dV and kinetic energy density
 * sum w beta (m |v|^2 / 2) W / dV (f = beta g, Eq. 5). */
void orc_moments(const orc_run* r, double* out) {
    int nodes = r->cfg.nx + 1;
    int ns = r->cfg.nspecies;
    memset(out, 0, sizeof(double) * (size_t)(nodes * (1 + 3 * ns)));
    memcpy(out, r->phi, sizeof(double) * (size_t)nodes);
    for (int s = 0; s < ns; ++s) {
        double* n = out + (size_t)nodes * (1 + 3 * s);
        double* G = n + nodes;
        double* K = G + nodes;
        for (int64_t i = 0; i < r->n[s]; ++i) {
            double xt = r->x[s][i];
            if (xt < 0.0) continue;
            double v[3] = {r->vx[s][i], r->vy[s][i], r->vz[s][i]};
            double v2 = norm2(v);
            double wb = r->w[s] * beta_of_s2(r->cfg.beta_kind, run_limit(r, xt), v2);
            int c = (int)floor(xt);
            double f = xt - (double)c;
            double w0 = wb * (1.0 - f), w1 = wb * f;
            double ke = 0.5 * r->cfg.species[s].mass * v2;
            n[c] += w0; n[c + 1] += w1;
            G[c] += w0 * v[0]; G[c + 1] += w1 * v[0];
            K[c] += w0 * ke; K[c + 1] += w1 * ke;
        }
        for (int j = 0; j < nodes; ++j) {
            double dV = (j == 0 || j == nodes - 1) ? 0.5 * r->cfg.dx : r->cfg.dx;
            n[j] /= dV; G[j] /= dV; K[j] /= dV;
        }
    }
}

int64_t orc_nslots(const orc_run* r, int32_t s) { return r->n[s]; }
int64_t orc_capacity(const orc_run* r, int32_t s) { return r->cap[s]; }
int64_t orc_nlive(const orc_run* r, int32_t s) {
    int64_t k = 0;
    for (int64_t i = 0; i < r->n[s]; ++i) k += (r->x[s][i] >= 0.0);
    return k;
}
int64_t orc_step_index(const orc_run* r) { return r->step; }
double orc_acc_e(const orc_run* r) { return r->acc_e; }
int64_t orc_absorbed_total(const orc_run* r, int32_t s) { return r->absorbed_total[s]; }
int64_t orc_injected_total(const orc_run* r, int32_t s) { return r->injected_total[s]; }

void orc_get_particles(const orc_run* r, int32_t s, double* x, double* vx, double* vy, double* vz) {
    size_t n = (size_t)r->n[s];
    memcpy(x, r->x[s], n * sizeof(double));
    memcpy(vx, r->vx[s], n * sizeof(double));
    memcpy(vy, r->vy[s], n * sizeof(double));
    memcpy(vz, r->vz[s], n * sizeof(double));
}

int orc_set_particles(orc_run* r, int32_t s, int64_t n, const double* x, const double* vx,
                      const double* vy, const double* vz) {
    ensure_capacity(r, s, n);
    memcpy(r->x[s], x, (size_t)n * sizeof(double));
    memcpy(r->vx[s], vx, (size_t)n * sizeof(double));
    memcpy(r->vy[s], vy, (size_t)n * sizeof(double));
    memcpy(r->vz[s], vz, (size_t)n * sizeof(double));
    r->n[s] = n;
    return 0;
}

void orc_set_counters(orc_run* r, int64_t step, double acc_e) {
    r->step = step;
    r->acc_e = acc_e;
}

double orc_acc_flux(const orc_run* r, int32_t s) { return r->acc_flux[s]; }

void orc_get_grid(const orc_run* r, double* Q0, double* Q1, double* phi, double* E) {
    size_t nodes = (size_t)r->cfg.nx + 1;
    if (Q0) memcpy(Q0, r->Q[0], nodes * sizeof(double));
    if (Q1 && r->cfg.nspecies > 1) memcpy(Q1, r->Q[1], nodes * sizeof(double));
    if (phi) memcpy(phi, r->phi, nodes * sizeof(double));
    if (E) memcpy(E, r->E, nodes * sizeof(double));
}

void orc_get_steady(const orc_run* r, orc_steady* out) { *out = r->steady; }

/* ======================================================================== */
/* 2D3V: x in [0, nx) with the symmetry plane at x = 0 and the grounded     */
/* absorbing wall at x = nx (as in 1D), y periodic in [0, ny); dy = dx.      */
/* Nodes (i, j), i = 0..nx, j = 0..ny-1, stored at i*ny + j.  E lies in the  */
/* (x, y) plane, so v_z is a constant of the motion.                          */
/* ======================================================================== */
struct orc2_run {
    orc_steady steady; /* fed with Phi_w (the y-mean of phi(0, y)) after every step */
    orc_config cfg;
    int32_t ny, tile; /* sort key: the tile x tile block of cells holding the particle */
    double w[2], qw[2], qm[2];
    int64_t n[2], cap[2];
    double *x[2], *y[2], *vx[2], *vy[2], *vz[2];
    double *Q[2], *phi, *Ex, *Ey;
    double acc_e;
    int64_t step;
    int64_t absorbed_total[2], injected_total[2];
};

static void ensure2(orc2_run* r, int s, int64_t need) {
    if (need <= r->cap[s]) return;
    int64_t cap = r->cap[s] > 0 ? r->cap[s] : 16;
    while (cap < need) cap *= 2;
    double** arrs[5] = {&r->x[s], &r->y[s], &r->vx[s], &r->vy[s], &r->vz[s]};
    for (int k = 0; k < 5; ++k) *arrs[k] = (double*)realloc(*arrs[k], sizeof(double) * (size_t)cap);
    r->cap[s] = cap;
}

orc2_run* orc2_create(const orc_config* cfg, int32_t ny, int32_t tile) {
    if (cfg->limit) return NULL;  /* 2D runs take one uniform limit */
    orc2_run* r = (orc2_run*)calloc(1, sizeof(orc2_run));
    r->cfg = *cfg;
    r->ny = ny;
    orc_steady_init(&r->steady, cfg->steady_window > 0 ? cfg->steady_window : (cfg->nx / 4 > 1 ? cfg->nx / 4 : 1),
                    cfg->steady_tol > 0.0 ? cfg->steady_tol : 0.02);
    r->tile = tile > 0 ? tile : 1;
    size_t nodes = (size_t)(cfg->nx + 1) * (size_t)ny;
    for (int s = 0; s < cfg->nspecies; ++s) {
        /* weight: dx dy Z / ppc, the 2D cell area holding ppc g-particles */
        r->w[s] = orc_weight(cfg, s) * cfg->dx;
        r->qw[s] = cfg->species[s].charge * r->w[s];
        r->qm[s] = cfg->species[s].charge / cfg->species[s].mass;
        r->Q[s] = (double*)calloc(nodes, sizeof(double));
    }
    r->phi = (double*)calloc(nodes, sizeof(double));
    r->Ex = (double*)calloc(nodes, sizeof(double));
    r->Ey = (double*)calloc(nodes, sizeof(double));
    return r;
}

void orc2_destroy(orc2_run* r) {
    if (!r) return;
    for (int s = 0; s < 2; ++s) {
        free(r->x[s]); free(r->y[s]); free(r->vx[s]); free(r->vy[s]); free(r->vz[s]); free(r->Q[s]);
    }
    free(r->phi); free(r->Ex); free(r->Ey);
    free(r);
}

/* Cold load in 2D: x = nx U, y = ny U, then the velocity draws of the 1D
 * loader (g = f/beta, Eq. 5). */
void orc2_load_particle(const orc_config* cfg, int32_t ny, int s, uint32_t i, double out[5]) {
    orc_stream st;
    stream_init(&st, cfg, i, 0u, ORC_PURPOSE_LOAD, s);
    double vt = species_vt(cfg, s);
    out[0] = (double)cfg->nx * stream_next(&st);
    if (out[0] >= (double)cfg->nx) out[0] = nextafter((double)cfg->nx, 0.0);
    out[1] = (double)ny * stream_next(&st);
    if (out[1] >= (double)ny) out[1] = nextafter((double)ny, 0.0);
    if (isinf(cfg->u)) {
        double z[3];
        stream_normal3(&st, z);
        out[2] = vt * z[0]; out[3] = vt * z[1]; out[4] = vt * z[2];
        return;
    }
    double sp = sample_g_speed(&st, cfg->beta_kind, cfg->u / vt);
    double mu = 2.0 * stream_next(&st) - 1.0;
    double ph = TWO_PI * stream_next(&st);
    double sn = sqrt(fmax(0.0, 1.0 - mu * mu));
    out[2] = vt * sp * mu;
    out[3] = vt * sp * (sn * cos(ph));
    out[4] = vt * sp * (sn * sin(ph));
}

void orc2_inject_particle(const orc_config* cfg, int32_t ny, int s, uint32_t k, uint32_t step, double out[5]) {
    orc_stream st;
    stream_init(&st, cfg, k, step, ORC_PURPOSE_INJECT, s);
    double vt = species_vt(cfg, s);
    out[0] = (double)cfg->source_cells * stream_next(&st);
    if (out[0] >= (double)cfg->source_cells) out[0] = nextafter((double)cfg->source_cells, 0.0);
    out[1] = (double)ny * stream_next(&st);
    if (out[1] >= (double)ny) out[1] = nextafter((double)ny, 0.0);
    double z[3];
    stream_normal3(&st, z);
    out[2] = vt * z[0]; out[3] = vt * z[1]; out[4] = vt * z[2];
}

/* Poisson in 2D, eps0 = 1: -lap phi = rho = Q/dV (dV = dx dy, half at the x
 * end nodes).  A discrete Fourier transform in y (periodic) turns the
 * five-point stencil into, per mode m, the 1D three-point system of
 * orc_poisson1d plus kappa_m phi with kappa_m = (4/dy^2) sin^2(pi m/ny);
 * node 0 symmetric, phi = 0 at node nx; Thomas per mode (real and imaginary
 * parts separately), inverse transform.  E = -grad phi by centred
 * differences (periodic in y; in x: E_x = 0 at node 0, the one-sided
 * second-order difference at the wall). */
void orc2_poisson(int32_t nx, int32_t ny, double dx, const double* Q, double* phi, double* Ex, double* Ey) {
    int nodes_x = nx + 1;
    double* re = (double*)calloc((size_t)nodes_x * ny, sizeof(double));
    double* im = (double*)calloc((size_t)nodes_x * ny, sizeof(double));
    for (int i = 0; i < nodes_x; ++i) {
        double dV = (i == 0 || i == nx) ? 0.5 * dx * dx : dx * dx;
        for (int m = 0; m < ny; ++m) {
            double sr = 0.0, si = 0.0;
            for (int j = 0; j < ny; ++j) {
                double ang = TWO_PI * (double)((int64_t)m * j % ny) / (double)ny;
                double rho = Q[(size_t)i * ny + j] / dV;
                sr += rho * cos(ang);
                si -= rho * sin(ang);
            }
            re[(size_t)i * ny + m] = sr;
            im[(size_t)i * ny + m] = si;
        }
    }
    double* cp = (double*)malloc(sizeof(double) * nx);
    double* dpr = (double*)malloc(sizeof(double) * nx);
    double* dpi = (double*)malloc(sizeof(double) * nx);
    double dx2 = dx * dx;
    for (int m = 0; m < ny; ++m) {
        double sm = sin(0.5 * TWO_PI * (double)m / (double)ny);
        double kd = 4.0 * sm * sm; /* kappa_m dx^2 with dy = dx */
        for (int i = 0; i < nx; ++i) {
            double a = (i == 0) ? 0.0 : -1.0, b = 2.0 + kd, c = (i == 0) ? -2.0 : -1.0;
            double rr = re[(size_t)i * ny + m] * dx2, ri = im[(size_t)i * ny + m] * dx2;
            if (i == 0) {
                cp[0] = c / b; dpr[0] = rr / b; dpi[0] = ri / b;
            } else {
                double den = b - a * cp[i - 1];
                cp[i] = c / den;
                dpr[i] = (rr - a * dpr[i - 1]) / den;
                dpi[i] = (ri - a * dpi[i - 1]) / den;
            }
        }
        re[(size_t)nx * ny + m] = 0.0;
        im[(size_t)nx * ny + m] = 0.0;
        re[(size_t)(nx - 1) * ny + m] = dpr[nx - 1];
        im[(size_t)(nx - 1) * ny + m] = dpi[nx - 1];
        for (int i = nx - 2; i >= 0; --i) {
            re[(size_t)i * ny + m] = dpr[i] - cp[i] * re[(size_t)(i + 1) * ny + m];
            im[(size_t)i * ny + m] = dpi[i] - cp[i] * im[(size_t)(i + 1) * ny + m];
        }
    }
    for (int i = 0; i < nodes_x; ++i)
        for (int j = 0; j < ny; ++j) {
            double s = 0.0;
            for (int m = 0; m < ny; ++m) {
                double ang = TWO_PI * (double)((int64_t)m * j % ny) / (double)ny;
                s += re[(size_t)i * ny + m] * cos(ang) - im[(size_t)i * ny + m] * sin(ang);
            }
            phi[(size_t)i * ny + j] = (i == nx) ? 0.0 : s / (double)ny;
        }
    for (int i = 0; i < nodes_x; ++i)
        for (int j = 0; j < ny; ++j) {
            const double* p = phi;
            size_t o = (size_t)i * ny + j;
            if (i == 0) Ex[o] = 0.0;
            else if (i < nx) Ex[o] = -(p[o + ny] - p[o - ny]) / (2.0 * dx);
            else Ex[o] = -(3.0 * p[o] - 4.0 * p[o - ny] + p[o - 2 * (size_t)ny]) / (2.0 * dx);
            int jp = (j + 1) % ny, jm = (j + ny - 1) % ny;
            Ey[o] = -(p[(size_t)i * ny + jp] - p[(size_t)i * ny + jm]) / (2.0 * dx);
        }
    free(re); free(im); free(cp); free(dpr); free(dpi);
}

/* beta-weighted bilinear (2D CIC) deposit of both species. */
static void deposit2(orc2_run* r) {
    int ny = r->ny;
    size_t nodes = (size_t)(r->cfg.nx + 1) * ny;
    for (int s = 0; s < r->cfg.nspecies; ++s) {
        memset(r->Q[s], 0, sizeof(double) * nodes);
        for (int64_t i = 0; i < r->n[s]; ++i) {
            double xt = r->x[s][i];
            if (xt < 0.0) continue;
            double yt = r->y[s][i];
            double v[3] = {r->vx[s][i], r->vy[s][i], r->vz[s][i]};
            double wb = r->qw[s] * beta_of_s2(r->cfg.beta_kind, r->cfg.u, norm2(v));
            int cx = (int)floor(xt), cy = (int)floor(yt);
            double fx = xt - cx, fy = yt - cy;
            int cy1 = (cy + 1) % ny;
            r->Q[s][(size_t)cx * ny + cy] += wb * (1.0 - fx) * (1.0 - fy);
            r->Q[s][(size_t)(cx + 1) * ny + cy] += wb * fx * (1.0 - fy);
            r->Q[s][(size_t)cx * ny + cy1] += wb * (1.0 - fx) * fy;
            r->Q[s][(size_t)(cx + 1) * ny + cy1] += wb * fx * fy;
        }
    }
}

/* Phi_w of a 2D run: the y-mean of phi at x = 0 (phi = 0 at the wall). */
static double orc2_wall_potential(const orc2_run* r) {
    double a = 0.0;
    for (int j = 0; j < r->ny; ++j) a += r->phi[j];
    return a / (double)r->ny;
}

static void solve2(orc2_run* r) {
    size_t nodes = (size_t)(r->cfg.nx + 1) * r->ny;
    double* Qt = (double*)calloc(nodes, sizeof(double));
    for (size_t k = 0; k < nodes; ++k)
        for (int s = 0; s < r->cfg.nspecies; ++s) Qt[k] += r->Q[s][k];
    orc2_poisson(r->cfg.nx, r->ny, r->cfg.dx, Qt, r->phi, r->Ex, r->Ey);
    free(Qt);
}

void orc2_refresh_fields(orc2_run* r) {
    deposit2(r);
    solve2(r);
}

/* Stable counting sort by the block of tile x tile cells holding each
 * particle, blocks numbered x-major: key = (cx/tile) * nty + cy/tile with
 * nty = ceil(ny/tile) (tile = 1: the cell index cx*ny + cy).  Dead slots are
 * dropped; perm (new slot -> old slot) when given. */
int64_t orc2_sort_key(int32_t ny, int32_t tile, double x, double y) {
    if (x < 0.0) return -1;
    int64_t nty = (ny + tile - 1) / tile;
    return ((int64_t)floor(x) / tile) * nty + (int64_t)floor(y) / tile;
}

void orc2_sort(orc2_run* r, int32_t* perm0, int32_t* perm1) {
    int ny = r->ny, T = r->tile;
    int64_t nkeys = (int64_t)((r->cfg.nx + T - 1) / T) * ((ny + T - 1) / T);
    for (int s = 0; s < r->cfg.nspecies; ++s) {
        int64_t n = r->n[s];
        int64_t* keys = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
        int64_t* start = (int64_t*)calloc((size_t)nkeys + 1, sizeof(int64_t));
        for (int64_t i = 0; i < n; ++i) {
            keys[i] = orc2_sort_key(ny, T, r->x[s][i], r->y[s][i]);
            if (keys[i] >= 0) start[keys[i] + 1] += 1;
        }
        for (int64_t k = 0; k < nkeys; ++k) start[k + 1] += start[k];
        int64_t nlive = start[nkeys];
        double* tmp[5];
        double* src[5] = {r->x[s], r->y[s], r->vx[s], r->vy[s], r->vz[s]};
        for (int a = 0; a < 5; ++a) tmp[a] = (double*)malloc(sizeof(double) * (size_t)(nlive + 1));
        int32_t* perm = (s == 0) ? perm0 : perm1;
        for (int64_t i = 0; i < n; ++i) {
            if (keys[i] < 0) continue;
            int64_t d = start[keys[i]]++;
            for (int a = 0; a < 5; ++a) tmp[a][d] = src[a][i];
            if (perm) perm[d] = (int32_t)i;
        }
        for (int a = 0; a < 5; ++a) {
            memcpy(src[a], tmp[a], sizeof(double) * (size_t)nlive);
            free(tmp[a]);
        }
        r->n[s] = nlive;
        free(keys); free(start);
    }
}

void orc2_load(orc2_run* r) {
    int64_t cells = (int64_t)r->cfg.nx * r->ny;
    for (int s = 0; s < r->cfg.nspecies; ++s) {
        int64_t n0 = cells * r->cfg.species[s].ppc;
        ensure2(r, s, n0);
        for (int64_t i = 0; i < n0; ++i) {
            double p[5];
            orc2_load_particle(&r->cfg, r->ny, s, (uint32_t)i, p);
            r->x[s][i] = p[0]; r->y[s][i] = p[1]; r->vx[s][i] = p[2]; r->vy[s][i] = p[3]; r->vz[s][i] = p[4];
        }
        r->n[s] = n0;
    }
    r->step = 0;
    r->acc_e = 0.0;
    if (r->cfg.sort_every > 0) orc2_sort(r, NULL, NULL);
    orc2_refresh_fields(r);
}

static void inject2(orc2_run* r, int s, int64_t count) {
    ensure2(r, s, r->n[s] + count);
    for (int64_t k = 0; k < count; ++k) {
        double p[5];
        orc2_inject_particle(&r->cfg, r->ny, s, (uint32_t)k, (uint32_t)r->step, p);
        int64_t i = r->n[s] + k;
        r->x[s][i] = p[0]; r->y[s][i] = p[1]; r->vx[s][i] = p[2]; r->vy[s][i] = p[3]; r->vz[s][i] = p[4];
    }
    r->n[s] += count;
    r->injected_total[s] += count;
}

/* One step of App. Eq. (A2) in 2D: bilinear gather of E^n(x^n), the exact
 * velocity map with a = (q/m)(E_x, E_y, 0) frozen, x += beta vx dt/dx,
 * y += beta vy dt/dy (periodic), the walls in x, source, deposit, solve. */
void orc2_step(orc2_run* r, int32_t nsteps) {
    const orc_config* cfg = &r->cfg;
    int ny = r->ny;
    double dtdx = cfg->dt / cfg->dx;
    for (int32_t it = 0; it < nsteps; ++it) {
        int64_t absorbed[2] = {0, 0};
        for (int s = 0; s < cfg->nspecies; ++s) {
            for (int64_t i = 0; i < r->n[s]; ++i) {
                double xt = r->x[s][i];
                if (xt < 0.0) continue;
                double yt = r->y[s][i];
                int cx = (int)floor(xt), cy = (int)floor(yt);
                double fx = xt - cx, fy = yt - cy;
                int cy1 = (cy + 1) % ny;
                size_t o00 = (size_t)cx * ny + cy, o10 = (size_t)(cx + 1) * ny + cy;
                size_t o01 = (size_t)cx * ny + cy1, o11 = (size_t)(cx + 1) * ny + cy1;
                double w00 = (1.0 - fx) * (1.0 - fy), w10 = fx * (1.0 - fy), w01 = (1.0 - fx) * fy, w11 = fx * fy;
                double ex = r->Ex[o00] * w00 + r->Ex[o10] * w10 + r->Ex[o01] * w01 + r->Ex[o11] * w11;
                double ey = r->Ey[o00] * w00 + r->Ey[o10] * w10 + r->Ey[o01] * w01 + r->Ey[o11] * w11;
                double a[3] = {r->qm[s] * ex, r->qm[s] * ey, 0.0};
                double v[3] = {r->vx[s][i], r->vy[s][i], r->vz[s][i]};
                double v1[3];
                orc_kick_exact(cfg->beta_kind, cfg->u, cfg->dt, v, a, v1);
                double b = beta_of_s2(cfg->beta_kind, cfg->u, norm2(v1));
                double xn = xt + b * v1[0] * dtdx;
                double yn = yt + b * v1[1] * dtdx;
                if (yn < 0.0 || yn >= (double)ny) { /* periodic in y: the remainder */
                    yn = fmod(yn, (double)ny);
                    if (yn < 0.0) yn += (double)ny;
                    if (yn >= (double)ny) yn = 0.0; /* a tiny negative rounded onto ny */
                }
                if (xn < 0.0) {
                    xn = -xn;
                    v1[0] = -v1[0];
                }
                r->vx[s][i] = v1[0];
                r->vy[s][i] = v1[1];
                r->vz[s][i] = v1[2];
                if (xn >= (double)cfg->nx) {
                    r->x[s][i] = -1.0;
                    absorbed[s] += 1;
                } else {
                    r->x[s][i] = xn;
                    r->y[s][i] = yn;
                }
            }
            r->absorbed_total[s] += absorbed[s];
        }
        if (cfg->nspecies == 2) {
            int64_t ni = absorbed[1];
            r->acc_e += (double)ni * (r->w[1] / r->w[0]);
            int64_t ne = (int64_t)floor(r->acc_e);
            r->acc_e -= (double)ne;
            inject2(r, 1, ni);
            inject2(r, 0, ne);
        }
        deposit2(r);
        solve2(r);
        r->step += 1;
        orc_steady_feed(&r->steady, orc2_wall_potential(r), r->step);
        if (cfg->sort_every > 0 && r->step % cfg->sort_every == 0) orc2_sort(r, NULL, NULL);
    }
}

void orc2_get_steady(const orc2_run* r, orc_steady* out) { *out = r->steady; }

/* beta-weighted moments at the nodes (f = beta g, Eq. 5), as in 1D: rows phi,
 * then per species n, Gamma_x = sum w beta v_x W / dV and the kinetic energy
 * density sum w beta (m |v|^2 / 2) W / dV, W bilinear with the y wrap, dV =
 * dx dy (halved at the x end nodes); each row (nx + 1) ny values at i*ny + j. */
void orc2_moments(const orc2_run* r, double* out) {
    int ny = r->ny;
    size_t nodes = (size_t)(r->cfg.nx + 1) * (size_t)ny;
    int ns = r->cfg.nspecies;
    memset(out, 0, sizeof(double) * nodes * (size_t)(1 + 3 * ns));
    memcpy(out, r->phi, sizeof(double) * nodes);
    for (int s = 0; s < ns; ++s) {
        double* n = out + nodes * (size_t)(1 + 3 * s);
        double* G = n + nodes;
        double* K = G + nodes;
        for (int64_t i = 0; i < r->n[s]; ++i) {
            double xt = r->x[s][i];
            if (xt < 0.0) continue;
            double yt = r->y[s][i];
            double v[3] = {r->vx[s][i], r->vy[s][i], r->vz[s][i]};
            double v2 = norm2(v);
            double wb = r->w[s] * beta_of_s2(r->cfg.beta_kind, r->cfg.u, v2);
            double ke = 0.5 * r->cfg.species[s].mass * v2;
            int cx = (int)floor(xt), cy = (int)floor(yt);
            double fx = xt - cx, fy = yt - cy;
            int cy1 = (cy + 1) % ny;
            size_t idx[4] = {(size_t)cx * ny + cy, (size_t)(cx + 1) * ny + cy, (size_t)cx * ny + cy1,
                             (size_t)(cx + 1) * ny + cy1};
            double wt[4] = {(1.0 - fx) * (1.0 - fy), fx * (1.0 - fy), (1.0 - fx) * fy, fx * fy};
            for (int k = 0; k < 4; ++k) {
                n[idx[k]] += wb * wt[k];
                G[idx[k]] += wb * wt[k] * v[0];
                K[idx[k]] += wb * wt[k] * ke;
            }
        }
        for (size_t k = 0; k < nodes; ++k) {
            int ix = (int)(k / (size_t)ny);
            double dV = r->cfg.dx * r->cfg.dx * ((ix == 0 || ix == r->cfg.nx) ? 0.5 : 1.0);
            n[k] /= dV; G[k] /= dV; K[k] /= dV;
        }
    }
}

int64_t orc2_nslots(const orc2_run* r, int32_t s) { return r->n[s]; }
int64_t orc2_step_index(const orc2_run* r) { return r->step; }
double orc2_acc_e(const orc2_run* r) { return r->acc_e; }
double orc2_weight(const orc2_run* r, int32_t s) { return r->w[s]; }
void orc2_get_particles(const orc2_run* r, int32_t s, double* x, double* y, double* vx, double* vy, double* vz) {
    size_t b = sizeof(double) * (size_t)r->n[s];
    memcpy(x, r->x[s], b); memcpy(y, r->y[s], b); memcpy(vx, r->vx[s], b); memcpy(vy, r->vy[s], b);
    memcpy(vz, r->vz[s], b);
}
void orc2_set_particles(orc2_run* r, int32_t s, int64_t n, const double* x, const double* y, const double* vx,
                        const double* vy, const double* vz) {
    ensure2(r, s, n);
    size_t b = sizeof(double) * (size_t)n;
    memcpy(r->x[s], x, b); memcpy(r->y[s], y, b); memcpy(r->vx[s], vx, b); memcpy(r->vy[s], vy, b);
    memcpy(r->vz[s], vz, b);
    r->n[s] = n;
}
void orc2_set_counters(orc2_run* r, int64_t step, double acc_e) {
    r->step = step;
    r->acc_e = acc_e;
}
void orc2_get_grid(const orc2_run* r, double* Q0, double* Q1, double* phi, double* Ex, double* Ey) {
    size_t b = sizeof(double) * (size_t)(r->cfg.nx + 1) * r->ny;
    if (Q0) memcpy(Q0, r->Q[0], b);
    if (Q1) memcpy(Q1, r->Q[1], b);
    if (phi) memcpy(phi, r->phi, b);
    if (Ex) memcpy(Ex, r->Ex, b);
    if (Ey) memcpy(Ey, r->Ey, b);
}

/* ======================================================================== */
/* Test particles in a prescribed traveling wave (Sec. V, wave-particle     */
/* interactions): 1D1V (v_y = v_z = 0), periodic x in [0, L), potential     */
/* phi(x, t) = phi0(t) sin(k (x - v_phi t)), k = 2 pi / L, with phi0 rising   */
/* linearly from 0 to phi_max over ramp_time and constant after (reading: a  */
/* linear ramp; the paper says only that it rises slowly over twenty wave    */
/* periods).  The field is evaluated exactly at (x^n, t^n = n dt); the       */
/* particles do not act on it.  Each step is App. Eq. (A2a, A2b) with the    */
/* exact velocity map and x wrapped into [0, L).                            */
/* ======================================================================== */
double orc_wave_phi0(const orc_wave* w, double t) {
    if (!(w->ramp_time > 0.0) || t >= w->ramp_time) return w->phi_max;
    return w->phi_max * (t / w->ramp_time);
}

/* acceleration (q/m) E_x with E_x = -dphi/dx */
double orc_wave_accel(const orc_wave* w, double x, double t) {
    double k = TWO_PI / w->length;
    return -w->qm * orc_wave_phi0(w, t) * k * cos(k * (x - w->v_phase * t));
}

void orc_wave_push(const orc_wave* w, double* x, double* v, int64_t n, int64_t step0, int32_t nsteps) {
    for (int64_t i = 0; i < n; ++i) {
        double xi = x[i], vi = v[i];
        for (int32_t s = 0; s < nsteps; ++s) {
            double t = (double)(step0 + s) * w->dt;
            double a[3] = {orc_wave_accel(w, xi, t), 0.0, 0.0};
            double v0[3] = {vi, 0.0, 0.0}, v1[3];
            orc_kick_exact(w->beta_kind, w->u, w->dt, v0, a, v1);
            vi = v1[0];
            double b = beta_of_s2(w->beta_kind, w->u, vi * vi);
            xi = xi + b * vi * w->dt;
            if (xi < 0.0 || xi >= w->length) {
                xi = fmod(xi, w->length);
                if (xi < 0.0) xi += w->length;
                if (xi >= w->length) xi = 0.0;
            }
        }
        x[i] = xi;
        v[i] = vi;
    }
}
