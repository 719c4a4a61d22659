// field2d.hip -- the 2D3V field solve (Eq. A2d with eps0 = 1) and the
// precision-independent step kernels of the 2D library.
//
// -lap phi = rho on the (nx+1) x ny nodes, y periodic, dy = dx, node 0 a
// symmetry plane, phi = 0 at node nx.  A discrete Fourier transform along y
// (rows are contiguous: one workgroup per x-row, a radix-2 FFT in LDS)
// turns the five-point stencil into one tridiagonal system along x per mode
// m with diagonal 2 + 4 sin^2(pi m/ny); those are solved by elimination with
// precomputed pivots, its two recurrences evaluated as scans in LDS (one
// workgroup per mode), then the inverse transform gives phi and centred
// differences give E.
#include <hip/hip_runtime.h>

#include "launch2d.h"
#include "slpic_device.h"
#include "slpic2d_internal.h"

namespace slpic {

__global__ void k_fill2d(double* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// In-place radix-2 decimation-in-time transform of buf (ny complex values,
// input in bit-reversed order): X_m = sum_j x_j exp(-+2 pi i m j / ny) with
// tw[k] = exp(-2 pi i k / ny), k < ny/2, conjugated for the inverse.  The
// workgroup has ny/2 threads: one butterfly each per stage.
__device__ void fft_rows(double2* buf, int ny, const double2* __restrict__ tw, bool inverse) {
    const int t = threadIdx.x;
    for (int len = 2; len <= ny; len <<= 1) {
        const int half = len >> 1;
        const int g = t / half, p = t - g * half;
        const int i1 = g * len + p, i2 = i1 + half;
        double2 w = tw[p * (ny / len)];
        if (inverse) w.y = -w.y;
        const double2 u = buf[i1], v = buf[i2];
        const double2 vw = make_double2(v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x);
        buf[i1] = make_double2(u.x + vw.x, u.y + vw.y);
        buf[i2] = make_double2(u.x - vw.x, u.y - vw.y);
        __syncthreads();
    }
}

__device__ __forceinline__ int bitrev(int j, int lg) { return (int)(__brev((unsigned)j) >> (32 - lg)); }

// Row i < nx: the right-hand side rho dx^2 = Q dx^2/dV (dV = dx dy, half at
// node 0, so Q or 2Q) to y-modes.
__global__ void k_fft_fwd2d(Args2D a, int lg) {
    const Run2D& R = *a.run;
    const int ny = R.ny, i = blockIdx.x;
    extern __shared__ __align__(16) unsigned char smem[];
    double2* buf = (double2*)smem;
    const double* Q0 = a.Q + (int64_t)i * ny;
    const double* Q1 = Q0 + R.nodes;
    const double sc = (i == 0) ? 2.0 : 1.0;
    for (int j = threadIdx.x; j < ny; j += blockDim.x) buf[bitrev(j, lg)] = make_double2((Q0[j] + Q1[j]) * sc, 0.0);
    __syncthreads();
    fft_rows(buf, ny, a.tw, false);
    double2* out = a.spec + (int64_t)i * ny;
    for (int m = threadIdx.x; m < ny; m += blockDim.x) out[m] = buf[m];
}

// Mode m: rows 0..nx-1 of (2 + kappa_m dx^2) phi_i - phi_{i+1} - phi_{i-1} =
// r_i, with phi_{-1} = phi_1 at the symmetry plane (coefficient -2 towards
// row 1 in row 0) and phi_nx = 0.  Gaussian elimination without pivoting
// (the Thomas algorithm) with the pivots p_i precomputed per mode: forward
// d_i = p_i (r_i + d_{i-1}), back phi_i = d_i + e_i p_i phi_{i+1} (e_0 = 2,
// e_i = 1).  Both are first-order linear recurrences, i.e. compositions of
// affine maps, evaluated as inclusive scans in LDS (one thread per row,
// ceil(log2 nx) doubling steps each way): the same terms as the sequential
// recurrence, summed as a tree.  Real input makes mode ny - m the complex
// conjugate of mode m (same coefficients): modes 0..ny/2 are solved and the
// others written as conjugates.
__global__ void k_tri2d(Args2D a) {
    const Run2D& R = *a.run;
    const int ny = R.ny, n = R.nx, m = blockIdx.x;
    const int i = threadIdx.x;
    extern __shared__ __align__(16) unsigned char smem[];
    double2* Bs = (double2*)smem;
    double* As = (double*)(Bs + n);
    const bool row = i < n;
    const double p = row ? a.tpiv[(int64_t)m * n + i] : 0.0;
    const double2 r = row ? a.spec[(int64_t)i * ny + m] : make_double2(0.0, 0.0);
    // forward: F_i = f_i o f_{i-1} o ... o f_0 with f_i(x) = p_i x + p_i r_i
    double A = p;
    double2 B = make_double2(p * r.x, p * r.y);
    for (int s = 1; s < n; s <<= 1) {
        if (row) {
            As[i] = A;
            Bs[i] = B;
        }
        __syncthreads();
        if (row && i >= s) {
            const double A1 = As[i - s];
            const double2 B1 = Bs[i - s];
            B = make_double2(A * B1.x + B.x, A * B1.y + B.y);
            A = A * A1;
        }
        __syncthreads();
    }
    // back: G_i = g_i o g_{i+1} o ... o g_{n-1} with g_i(y) = e_i p_i y + d_i, at y = 0
    A = (i == 0 ? 2.0 : 1.0) * p;
    for (int s = 1; s < n; s <<= 1) {
        if (row) {
            As[i] = A;
            Bs[i] = B;
        }
        __syncthreads();
        if (row && i + s < n) {
            const double A2 = As[i + s];
            const double2 B2 = Bs[i + s];
            B = make_double2(A * B2.x + B.x, A * B2.y + B.y);
            A = A * A2;
        }
        __syncthreads();
    }
    if (!row) return;
    a.spec[(int64_t)i * ny + m] = B;
    if (m > 0 && m < ny / 2) a.spec[(int64_t)i * ny + (ny - m)] = make_double2(B.x, -B.y);
}

// Row i < nx: phi from its y-modes; row 0 also gives Phi_w = mean_y phi(0, y)
// (phi = 0 at the wall) and, after an advancing step (already counted by
// k_finish2d), puts it into the history ring and the steady detector.
__global__ void k_fft_inv2d(Args2D a, int lg, int advance) {
    const Run2D& R = *a.run;
    const int ny = R.ny, i = blockIdx.x;
    extern __shared__ __align__(16) unsigned char smem[];
    double2* buf = (double2*)smem;
    const double2* in = a.spec + (int64_t)i * ny;
    for (int m = threadIdx.x; m < ny; m += blockDim.x) buf[bitrev(m, lg)] = in[m];
    __syncthreads();
    fft_rows(buf, ny, a.tw, true);
    const double inv = 1.0 / (double)ny;
    double* phi = a.phi + (int64_t)i * ny;
    double part = 0.0;
    for (int j = threadIdx.x; j < ny; j += blockDim.x) {
        const double v = buf[j].x * inv;
        phi[j] = v;
        part += v;
    }
    if (i != 0) return;  // workgroup-uniform
    __syncthreads();
    double* red = (double*)smem;  // buf is no longer read
    red[threadIdx.x] = part;
    __syncthreads();
    for (int h = blockDim.x >> 1; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        State2D* st = a.st;
        const double pw = red[0] * inv;
        st->phi_w = pw;
        if (advance) {
            a.history[(st->step - 1) % kHistoryLen2] = pw;
            steady_feed(R, st, pw);
        }
    }
}

// E = -grad phi at every node: centred differences (periodic in y; in x:
// zero at the symmetry plane, the one-sided second-order difference at the
// wall), in FP64 and as a float copy for float particles.
__global__ void k_efield2d(Args2D a) {
    const Run2D& R = *a.run;
    const int ny = R.ny, nx = R.nx;
    const double h = 0.5 / R.dx;
    const int64_t nodes = R.nodes;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nodes; n += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(n / ny), j = (int)(n - (int64_t)i * ny);
        const double* p = a.phi;
        double ex;
        if (i == 0) ex = 0.0;
        else if (i < nx) ex = -(p[n + ny] - p[n - ny]) * h;
        else ex = -(3.0 * p[n] - 4.0 * p[n - ny] + p[n - 2 * ny]) * h;
        const int jp = (j + 1 == ny) ? 0 : j + 1, jm = (j == 0) ? ny - 1 : j - 1;
        const int64_t r = (int64_t)i * ny;
        const double ey = -(p[r + jp] - p[r + jm]) * h;
        a.E[n] = make_double2(ex, ey);
        a.E32[n] = make_float2((float)ex, (float)ey);
    }
}

// End of a step's particle work: the source plan and push counters applied
// to the run state, the counters cleared for the next push.
__global__ void k_finish2d(Args2D a) {
    State2D* st = a.st;
    Inject2D* ip = a.inj;
    if (threadIdx.x == 0) {
        for (int s = 0; s < 2; ++s) {
            st->nslots[s] = ip->base[s] + ip->count[s];
            st->absorbed_total[s] += ip->absorbed[s];
            st->injected_total[s] += ip->count[s];
        }
        st->pushed_total += ip->pushed;
        st->acc_e = ip->acc_e;
        st->error |= ip->overflow;
        ip->overflow = 0;
        st->step += 1;
    }
    for (int j = threadIdx.x; j < 2 * kCountSlots2; j += blockDim.x) a.counts[j] = make_int2(0, 0);
}

// Moments: phi into row 0, the six accumulated rows divided by the node
// volume dx dy (half at the x end nodes).
__global__ void k_moments2d_finish(Args2D a, double* out) {
    const Run2D& R = *a.run;
    const int64_t nodes = R.nodes;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nodes; k += (int64_t)gridDim.x * blockDim.x) {
        out[k] = a.phi[k];
        const int ix = (int)(k / R.ny);
        const double inv = 1.0 / (R.dx * R.dx * ((ix == 0 || ix == R.nx) ? 0.5 : 1.0));
        for (int row = 1; row < 7; ++row) out[row * nodes + k] *= inv;
    }
}

// After the sort scatter: the sorted buffer becomes current and holds exactly
// the live particles; tile k of species s owns slots [tbeg[k], tbeg[k+1]).
__global__ void k_sort2d_finish(Args2D a, int nblk) {
    const Run2D& R = *a.run;
    State2D* st = a.st;
    const int nk = R.nkeys;
    for (int s = 0; s < 2; ++s) {
        const int* hs = a.hist + R.hoff[s];
        const int base = hs[0];
        const int64_t end_entry = R.hoff[s] + (int64_t)nk * R.stiles[s];
        const long long end = (s == 0) ? (long long)a.hist[end_entry] : a.btot[nblk];
        const int64_t live = end - base;
        int64_t* tb = a.tbeg + (int64_t)s * (nk + 1);
        for (int k = threadIdx.x; k < nk; k += blockDim.x) tb[k] = hs[(int64_t)k * R.stiles[s]] - base;
        if (threadIdx.x == 0) {
            tb[nk] = live;
            st->nslots[s] = live;
            st->nsorted[s] = live;
            st->live[s] = live;
        }
    }
    if (threadIdx.x == 0) *a.cur ^= 1;
}

void launch2d_fill(double* p, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill2d, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, s, p, n);
}

void launch2d_field(const Args2D& a, int nx, int ny, int advance, hipStream_t s) {
    int lg = 0;
    while ((1 << lg) < ny) ++lg;
    const size_t lds = sizeof(double2) * (size_t)ny;
    hipLaunchKernelGGL(k_fft_fwd2d, dim3(nx), dim3(ny / 2), lds, s, a, lg);
    const int rows = (nx + 63) / 64 * 64;
    hipLaunchKernelGGL(k_tri2d, dim3(ny / 2 + 1), dim3(rows), (size_t)nx * 24, s, a);
    hipLaunchKernelGGL(k_fft_inv2d, dim3(nx), dim3(ny / 2), lds, s, a, lg, advance);
    const int64_t nodes = (int64_t)(nx + 1) * ny;
    hipLaunchKernelGGL(k_efield2d, dim3((unsigned)std::min<int64_t>((nodes + 255) / 256, 8192)), dim3(256), 0, s, a);
}

void launch2d_finish(const Args2D& a, hipStream_t s) {
    hipLaunchKernelGGL(k_finish2d, dim3(1), dim3(128), 0, s, a);
}

void launch2d_sort_finish(const Args2D& a, int nblk, hipStream_t s) {
    hipLaunchKernelGGL(k_sort2d_finish, dim3(1), dim3(256), 0, s, a, nblk);
}

void launch2d_moments_finish(const Args2D& a, int64_t nodes, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_moments2d_finish, dim3((unsigned)std::min<int64_t>((nodes + 255) / 256, 4096)), dim3(256), 0,
                       s, a, out);
}

}  // namespace slpic
