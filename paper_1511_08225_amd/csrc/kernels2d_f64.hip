// kernels2d_f64.hip -- 2D3V kernels for FP64 particles.
#define SLPIC_T double
#define SLPIC_SUFFIX f64
#include "kernels2d.inc"
