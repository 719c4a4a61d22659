// launch.h -- host launchers of the library's kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "slpic_internal.h"

namespace slpic {

#define SLPIC_DECLARE_LAUNCHERS(sfx)                                                                   \
    void launch_load_##sfx(const KArgs& a, int nchunks, int block, hipStream_t s);                     \
    void launch_load_warm_##sfx(const KArgs& a, const void* cells, int ncells, hipStream_t s);         \
    void launch_push_##sfx(bool push, bool sheath, bool varlim, int per_thread, const KArgs& a,        \
                           const Chunk* chunks, int nchunks, int block, hipStream_t s);                \
    void launch_velocity_map_##sfx(int beta_kind, double u, double dt, int64_t n, const void* vx,      \
                                   const void* c2, const void* acc, void* out, int* iters,             \
                                   hipStream_t s);                                                     \
    void launch_source_field_##sfx(const KArgs& a, int nruns, int threads, size_t lds, hipStream_t s); \
    void launch_wall_inject_##sfx(const KArgs& a, hipStream_t s);                                      \
    void launch_limit_##sfx(const KArgs& a, const LimitArgs& L, int nchunks, int scatter, hipStream_t s); \
    void launch_moments_##sfx(const KArgs& a, int chunk0, int nchunks, int block, size_t lds,          \
                              double* out, int per_run, hipStream_t s);                                \
    void launch_sort_hist_##sfx(const KArgs& a, int ntiles, int block, size_t lds, hipStream_t s);     \
    void launch_sort_scatter_##sfx(const KArgs& a, int ntiles, int block, size_t lds, hipStream_t s);

SLPIC_DECLARE_LAUNCHERS(f32)
SLPIC_DECLARE_LAUNCHERS(f64)
#undef SLPIC_DECLARE_LAUNCHERS

// precision-independent kernels
void launch_init_state(const KArgs& a, int nruns, hipStream_t s);
void launch_field(const KArgs& a, int nruns, int advance, size_t lds, hipStream_t s);
int scan_blocks(int64_t hist_entries);
void launch_sort_scan(const KArgs& a, int64_t hist_entries, long long* btot, hipStream_t s);
// exclusive scan of n ints in place; btot[scan_blocks(n)] receives the total
void launch_scan_ints(int* h, int64_t n, long long* btot, hipStream_t s);
void launch_sort_finish(const KArgs& a, int nruns, int64_t hist_entries, const long long* btot,
                        hipStream_t s);
void launch_zero(double* p, int64_t n, hipStream_t s);
void launch_zero_ints(int* p, int64_t n, hipStream_t s);
void launch_limit_finish(const KArgs& a, int nruns, int64_t total_slots, const long long* btot, hipStream_t s);
void launch_moments_finish(const KArgs& a, int run, double* out, hipStream_t s);
void launch_moments_window(const KArgs& a, int run, double* out, int reset, hipStream_t s);
void launch_moments_sample_finish(const KArgs& a, int run0, int nruns, hipStream_t s);

}  // namespace slpic
