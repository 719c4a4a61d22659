// kernels_common.hip -- precision-independent kernels: run-state setup, the
// 1D field solve (Eq. A2d), the scan stage of the cell sort and the
// finishing pass of the moments.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "slpic_device.h"
#include "field.inc"

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
    for (int j = 0; j < kMaxSpecies * kCountSlots; ++j)
        a.counts[(int64_t)r * kMaxSpecies * kCountSlots + j] = make_int2(0, 0);
    a.push_err[r] = 0;
    st->acc_e = 0.0;
    st->phi_w = 0.0;
    st->error = 0;
    st->win_n = 0;
    st->win_sum = 0.0;
    for (int k = 0; k < 3; ++k) st->win_mean[k] = 0.0;
    st->nwin = 0;
    st->steady_step = -1;
    st->msamples = 0;
    st->acc_w[0] = 0.0;
    st->acc_w[1] = 0.0;
}

__global__ __launch_bounds__(kFieldThreads) void k_field(KArgs a, int advance) {
    extern __shared__ __align__(16) unsigned char smem[];
    double* D = (double*)smem;
    const RunInfo& R = a.runs[blockIdx.x];
    ChargeRegs qc;
    load_charge(a, R, qc);
    field_solve(a, R, blockIdx.x, a.state + blockIdx.x, advance, D, D + R.nodes, qc);
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

// Launched with kScanThreads threads: each holds kScanPer consecutive
// entries in registers (two 16-byte loads and stores where all are in range;
// h is 16-byte aligned).
constexpr int kScanThreads = 1024;
constexpr int kScanPer = kScanBlock / kScanThreads;
static_assert(kScanPer == 8, "two int4 per thread");
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(int* h, int64_t n, const long long* btot) {
    __shared__ long long tmp[17];
    const int64_t j0 = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
    const bool full = j0 + kScanPer <= n;
    int v[kScanPer];
    if (full) {
        const int4 a = *(const int4*)(h + j0), b = *(const int4*)(h + j0 + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int i = 0; i < kScanPer; ++i) v[i] = j0 + i < n ? h[j0 + i] : 0;
    }
    long long loc = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) loc += v[i];
    long long run = btot[blockIdx.x] + block_scan<long long>(loc, tmp, false);
    int o[kScanPer];
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        o[i] = (int)run;
        run += v[i];
    }
    if (full) {
        *(int4*)(h + j0) = make_int4(o[0], o[1], o[2], o[3]);
        *(int4*)(h + j0 + 4) = make_int4(o[4], o[5], o[6], o[7]);
    } else {
#pragma unroll
        for (int i = 0; i < kScanPer; ++i)
            if (j0 + i < n) h[j0 + i] = o[i];
    }
}

// After the scatter: the sorted buffer becomes current and holds exactly the
// live particles of each (run, species).
__global__ void k_sort_finish(KArgs a, int nruns, int64_t hist_entries, const long long* btot, int nblk) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) *a.cur ^= 1;
    if (r >= nruns) return;
    const RunInfo& R = a.runs[r];
    if (R.pruned) return;  // not sorted: its counts stand
    for (int s = 0; s < kMaxSpecies; ++s) {
        const int64_t e = R.hoff[s] + (int64_t)R.nkeys * R.ntiles[s];
        const long long base = a.hist[R.hoff[s]];
        const long long end = e < hist_entries ? (long long)a.hist[e] : btot[nblk];
        a.state[r].nslots[s] = end - base;
    }
}

// After a speed-limit resampling: every (run, species) segment's new count
// from the scanned copy counts (the next segment's first entry, or the
// grand total), capped at the capacity with the sticky flag, and the
// particle buffers swapped.
__global__ void k_limit_finish(KArgs a, int nruns, int64_t total_slots, const long long* btot, int nblk) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) *a.cur ^= 1;
    if (r >= nruns) return;
    const RunInfo& R = a.runs[r];
    for (int s = 0; s < kMaxSpecies; ++s) {
        const int64_t e = R.poff[s] + R.cap[s];
        const long long base = a.perm[R.poff[s]];
        const long long end = e < total_slots ? (long long)a.perm[e] : btot[nblk];
        const long long n = end - base;
        if (n > R.cap[s]) a.state[r].error |= 1;
        a.state[r].nslots[s] = n < R.cap[s] ? n : R.cap[s];
    }
}

__global__ void k_zero(double* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0.0;
}

__global__ void k_zero_ints(int* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

// Moments: potential into row 0, accumulated sums divided by the node volume.
// Window means of the moment samples of one run (phi, then per species n,
// Gamma_x, energy density, each node's sums over dV), optionally clearing
// the window afterwards.  One workgroup.
__global__ void k_moments_window(KArgs a, int run, double* out, int reset) {
    const RunInfo& R = a.runs[run];
    RunState* st = a.state + run;
    const int nodes = R.nodes;
    double* M = a.Macc + 7 * R.goff;
    const int64_t ns = st->msamples;
    const double inv = ns > 0 ? 1.0 / (double)ns : 0.0;
    for (int j = threadIdx.x; j < nodes; j += blockDim.x) {
        const double dV = (j == 0 || j == nodes - 1) ? 0.5 * R.dx : R.dx;
        out[j] = M[j] * inv;
        for (int r = 1; r < 7; ++r) out[(int64_t)r * nodes + j] = M[(int64_t)r * nodes + j] * inv / dV;
    }
    if (reset) {
        __syncthreads();
        for (int j = threadIdx.x; j < 7 * nodes; j += blockDim.x) M[j] = 0.0;
        if (threadIdx.x == 0) st->msamples = 0;
    }
}

// After the raw moment sums of a sample were added to the accumulators: add
// phi and count the sample.  One workgroup per run.
__global__ void k_moments_sample_finish(KArgs a, int run0) {
    const int run = run0 + blockIdx.x;
    const RunInfo& R = a.runs[run];
    double* M = a.Macc + 7 * R.goff;
    const double* phi = a.phi + R.goff;
    for (int j = threadIdx.x; j < R.nodes; j += blockDim.x) M[j] += phi[j];
    if (threadIdx.x == 0) a.state[run].msamples += 1;
}

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
    hipLaunchKernelGGL(k_field, dim3(nruns), dim3(kFieldThreads), lds, s, a, advance);
}
int scan_blocks(int64_t n) { return (int)((n + kScanBlock - 1) / kScanBlock); }
void launch_scan_ints(int* h, int64_t n, long long* btot, hipStream_t s) {
    const int nblk = scan_blocks(n);
    hipLaunchKernelGGL(k_scan_blocks, dim3(nblk), dim3(1024), 0, s, h, n, btot);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, btot, nblk);
    hipLaunchKernelGGL(k_scan_apply, dim3(nblk), dim3(kScanThreads), 0, s, h, n, (const long long*)btot);
}
void launch_sort_scan(const KArgs& a, int64_t hist_entries, long long* btot, hipStream_t s) {
    launch_scan_ints(a.hist, hist_entries, btot, s);
}
void launch_sort_finish(const KArgs& a, int nruns, int64_t hist_entries, const long long* btot,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_sort_finish, dim3((nruns + 255) / 256), dim3(256), 0, s, a, nruns, hist_entries,
                       btot, scan_blocks(hist_entries));
}
void launch_limit_finish(const KArgs& a, int nruns, int64_t total_slots, const long long* btot, hipStream_t s) {
    hipLaunchKernelGGL(k_limit_finish, dim3((nruns + 255) / 256), dim3(256), 0, s, a, nruns, total_slots, btot,
                       scan_blocks(total_slots));
}
void launch_zero_ints(int* p, int64_t n, hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_zero_ints, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
}
void launch_zero(double* p, int64_t n, hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
}
void launch_moments_window(const KArgs& a, int run, double* out, int reset, hipStream_t s) {
    hipLaunchKernelGGL(k_moments_window, dim3(1), dim3(256), 0, s, a, run, out, reset);
}
void launch_moments_sample_finish(const KArgs& a, int run0, int nruns, hipStream_t s) {
    hipLaunchKernelGGL(k_moments_sample_finish, dim3(nruns), dim3(256), 0, s, a, run0);
}
void launch_moments_finish(const KArgs& a, int run, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_moments_finish, dim3(8), dim3(256), 0, s, a, run, out);
}

}  // namespace slpic
