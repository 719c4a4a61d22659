// kernels2d_f32.hip -- 2D3V kernels for FP32 particles (int32 fixed-point
// coordinates, float velocities) with FP64 grids.
#define SLPIC_T float
#define SLPIC_SUFFIX f32
#include "kernels2d.inc"
