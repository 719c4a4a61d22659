// launch2d.h -- host launchers of the 2D3V kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "slpic2d_internal.h"

namespace slpic {

#define SLPIC2_DECLARE_LAUNCHERS(sfx)                                                                    \
    void launch2d_load_##sfx(const Args2D& a, hipStream_t s);                                            \
    int launch2d_push_##sfx(bool push, int per_thread, const Args2D& a, int nkeys, int ntail, size_t lds, \
                            hipStream_t s);                                                              \
    void launch2d_inject_##sfx(const Args2D& a, int groups, hipStream_t s);                              \
    void launch2d_sort_hist_##sfx(const Args2D& a, int ntiles, size_t lds, hipStream_t s);               \
    void launch2d_sort_scatter_##sfx(const Args2D& a, int ntiles, size_t lds, hipStream_t s);          \
    void launch2d_moments_##sfx(const Args2D& a, int64_t slots, double* out, hipStream_t s);

SLPIC2_DECLARE_LAUNCHERS(f32)
SLPIC2_DECLARE_LAUNCHERS(f64)
#undef SLPIC2_DECLARE_LAUNCHERS

void launch2d_fill(double* p, int64_t n, hipStream_t s);
// advance: the solve ends an advancing step (Phi_w into the history ring
// and the steady detector)
void launch2d_field(const Args2D& a, int nx, int ny, int advance, hipStream_t s);
void launch2d_finish(const Args2D& a, hipStream_t s);
void launch2d_sort_finish(const Args2D& a, int nblk, hipStream_t s);
void launch2d_moments_finish(const Args2D& a, int64_t nodes, double* out, hipStream_t s);

}  // namespace slpic
