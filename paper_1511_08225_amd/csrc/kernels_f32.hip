// kernels_f32.hip -- FP32 particles (int32 fixed-point positions, float
// velocities) with FP64 grids.
#include "kernels.inc"
#include "launch.h"

#define SLPIC_T float
#define SLPIC_SUFFIX f32
#include "launchers.inc"
