// kernels_common.hip -- precision-independent kernels: run-state setup, the
// 1D field solve (Eq. A2d), the scan stage of the cell sort and the
// finishing pass of the moments.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "slpic_device.h"

namespace slpic {

__global__ void k_init_state(KArgs a, int nruns) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) *a.cur = 0;
    if (r >= nruns) return;
    RunState* st = a.state + r;
    const RunInfo& R = a.runs[r];
    for (int s = 0; s < kMaxSpecies; ++s) {
        st->nslots[s] = R.nload[s];
        st->absorbed_step[s] = 0;
        st->absorbed_total[s] = 0;
        st->injected_total[s] = 0;
    }
    st->step = 0;
    st->pushed_total = 0;
    st->acc_e = 0.0;
    st->phi_w = 0.0;
    st->error = 0;
}

// Block-wide exclusive scans of one value per thread, in thread order
// (prefix) or reverse thread order (suffix): wave64 shuffles, then the wave
// totals in LDS.  Fixed summation order, so results are reproducible.
template <typename V>
__device__ V block_scan(V v, V* tmp, bool suffix) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    V inc = v;
    if (!suffix) {
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            V t = __shfl_up(inc, d, 64);
            if (lane >= d) inc += t;
        }
    } else {
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            V t = __shfl_down(inc, d, 64);
            if (lane + d < 64) inc += t;
        }
    }
    V exc = suffix ? __shfl_down(inc, 1, 64) : __shfl_up(inc, 1, 64);
    if (suffix ? lane == 63 : lane == 0) exc = V(0);
    if (suffix ? lane == 0 : lane == 63) tmp[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        V run = V(0);
        for (int k = 0; k < nw; ++k) {
            int kk = suffix ? nw - 1 - k : k;
            V t = tmp[kk];
            tmp[kk] = run;
            run += t;
        }
        tmp[nw] = run;
    }
    __syncthreads();
    V r = tmp[w] + exc;
    __syncthreads();
    return r;
}

// Field solve of one run (one workgroup).  Charge Q_j = sum_s Q_{s,j};
// rho_j = Q_j/dV_j with half volumes at both ends.  With the symmetry plane
// at node 0 and phi = 0 at node nx, the three-point system
//   -2(phi_1 - phi_0)/dx^2 = rho_0,  -(phi_{j+1} - 2 phi_j + phi_{j-1})/dx^2 = rho_j
// has the exact two-pass solution
//   D_j = phi_j - phi_{j+1} = dx * sum_{i<=j} Q_i        (Gauss's law)
//   phi_j = sum_{k=j}^{nx-1} D_k,
// computed as a prefix scan and a suffix scan.  E_j = -(phi_{j+1} -
// phi_{j-1})/(2dx) = (D_{j-1} + D_j)/(2dx), E_0 = 0, and the one-sided
// second-order difference at the wall, E_nx = (3 D_{nx-1} - D_{nx-2})/(2dx).
__global__ void k_field(KArgs a, int advance) {
    const int run = blockIdx.x;
    const RunInfo& R = a.runs[run];
    RunState* st = a.state + run;
    const int nx = R.nx, nodes = R.nodes;
    extern __shared__ __align__(16) unsigned char smem[];
    double* D = (double*)smem;  // [nodes]
    double* tmp = D + nodes;    // [nwaves + 1]
    double* Qa = a.Qacc + 2 * R.goff;
    double* Ql = a.Qlast + 2 * R.goff;
    for (int j = threadIdx.x; j < nodes; j += blockDim.x) {
        double q0 = Qa[j], q1 = Qa[nodes + j];
        Ql[j] = q0;
        Ql[nodes + j] = q1;
        Qa[j] = 0.0;
        Qa[nodes + j] = 0.0;
        D[j] = q0 + q1;
    }
    __syncthreads();
    const int per = (nx + blockDim.x - 1) / blockDim.x;
    const int j0 = threadIdx.x * per, j1 = min(j0 + per, nx);
    {   // prefix: D_j = dx * sum_{i<=j} Q_i
        double loc = 0.0;
        for (int j = j0; j < j1; ++j) loc += D[j];
        double run_s = block_scan(loc, tmp, false);
        for (int j = j0; j < j1; ++j) {
            run_s += D[j];
            D[j] = R.dx * run_s;
        }
    }
    __syncthreads();
    double* phi = a.phi + R.goff;
    {   // suffix: phi_j = sum_{k>=j} D_k
        double loc = 0.0;
        for (int j = j1 - 1; j >= j0; --j) loc += D[j];
        double run_s = block_scan(loc, tmp, true);
        for (int j = j1 - 1; j >= j0; --j) {
            run_s += D[j];
            phi[j] = run_s;
        }
    }
    double* E = a.E + R.goff;
    for (int j = threadIdx.x; j < nodes; j += blockDim.x) {
        double e;
        if (j == 0) e = 0.0;
        else if (j < nx) e = (D[j - 1] + D[j]) / (2.0 * R.dx);
        else e = (3.0 * D[nx - 1] - D[nx - 2]) / (2.0 * R.dx);
        E[j] = e;
        if (j == nx) phi[j] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double pw = phi[0];
        st->phi_w = pw;
        if (advance) {
            a.history[(int64_t)run * kHistoryLen + (st->step % kHistoryLen)] = pw;
            st->step += 1;
        }
    }
}

// Exclusive scan of the sort histogram, in place, over all (run, species)
// segments at once: block sums, a scan of the block sums, then each block
// rescanned with its offset.  A segment's first entry is then its base and
// the next segment's first entry (or the grand total) its end.
constexpr int kScanBlock = 8192;

__global__ void k_scan_blocks(int* h, int64_t n, long long* btot) {
    __shared__ long long tmp[17];
    const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
    const int64_t b1 = min(b0 + kScanBlock, n);
    long long loc = 0;
    for (int64_t j = b0 + threadIdx.x; j < b1; j += blockDim.x) loc += h[j];
    // block total via the scan helper
    long long ex = block_scan<long long>(loc, tmp, false);
    if (threadIdx.x == blockDim.x - 1) btot[blockIdx.x] = ex + loc;
}

__global__ void k_scan_top(long long* btot, int nblk) {
    __shared__ long long tmp[17];
    const int per = (nblk + blockDim.x - 1) / blockDim.x;
    const int j0 = threadIdx.x * per, j1 = min(j0 + per, nblk);
    long long loc = 0;
    for (int j = j0; j < j1; ++j) loc += btot[j];
    long long run = block_scan<long long>(loc, tmp, false);
    for (int j = j0; j < j1; ++j) {
        long long c = btot[j];
        btot[j] = run;
        run += c;
    }
    if (threadIdx.x == blockDim.x - 1) btot[nblk] = run;  // grand total
}

__global__ void k_scan_apply(int* h, int64_t n, const long long* btot) {
    __shared__ long long tmp[17];
    const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
    const int64_t b1 = min(b0 + kScanBlock, n);
    const int per = (kScanBlock + blockDim.x - 1) / blockDim.x;
    const int64_t j0 = b0 + (int64_t)threadIdx.x * per, j1 = min(j0 + per, b1);
    long long loc = 0;
    for (int64_t j = j0; j < j1; ++j) loc += h[j];
    long long run = btot[blockIdx.x] + block_scan<long long>(loc, tmp, false);
    for (int64_t j = j0; j < j1; ++j) {
        long long c = h[j];
        h[j] = (int)run;
        run += c;
    }
}

// After the scatter: the sorted buffer becomes current and holds exactly the
// live particles of each (run, species).
__global__ void k_sort_finish(KArgs a, int nruns, int64_t hist_entries, const long long* btot, int nblk) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) *a.cur ^= 1;
    if (r >= nruns) return;
    const RunInfo& R = a.runs[r];
    for (int s = 0; s < kMaxSpecies; ++s) {
        const int64_t e = R.hoff[s] + (int64_t)R.nkeys * R.ntiles[s];
        const long long base = a.hist[R.hoff[s]];
        const long long end = e < hist_entries ? (long long)a.hist[e] : btot[nblk];
        a.state[r].nslots[s] = end - base;
    }
}

__global__ void k_zero(double* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0.0;
}

// Moments: potential into row 0, accumulated sums divided by the node volume.
__global__ void k_moments_finish(KArgs a, int run, double* out) {
    const RunInfo& R = a.runs[run];
    const int nodes = R.nodes;
    const double* phi = a.phi + R.goff;
    for (int j = threadIdx.x + blockIdx.x * blockDim.x; j < nodes; j += blockDim.x * gridDim.x) {
        double dV = (j == 0 || j == nodes - 1) ? 0.5 * R.dx : R.dx;
        out[j] = phi[j];
        for (int r = 1; r < 7; ++r) out[(int64_t)r * nodes + j] /= dV;
    }
}

void launch_init_state(const KArgs& a, int nruns, hipStream_t s) {
    hipLaunchKernelGGL(k_init_state, dim3((nruns + 255) / 256), dim3(256), 0, s, a, nruns);
}
void launch_field(const KArgs& a, int nruns, int advance, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL(k_field, dim3(nruns), dim3(1024), lds, s, a, advance);
}
int scan_blocks(int64_t n) { return (int)((n + kScanBlock - 1) / kScanBlock); }
void launch_sort_scan(const KArgs& a, int64_t hist_entries, long long* btot, hipStream_t s) {
    const int nblk = scan_blocks(hist_entries);
    hipLaunchKernelGGL(k_scan_blocks, dim3(nblk), dim3(1024), 0, s, a.hist, hist_entries, btot);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, btot, nblk);
    hipLaunchKernelGGL(k_scan_apply, dim3(nblk), dim3(1024), 0, s, a.hist, hist_entries, (const long long*)btot);
}
void launch_sort_finish(const KArgs& a, int nruns, int64_t hist_entries, const long long* btot,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_sort_finish, dim3((nruns + 255) / 256), dim3(256), 0, s, a, nruns, hist_entries,
                       btot, scan_blocks(hist_entries));
}
void launch_zero(double* p, int64_t n, hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
}
void launch_moments_finish(const KArgs& a, int run, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_moments_finish, dim3(8), dim3(256), 0, s, a, run, out);
}

}  // namespace slpic
