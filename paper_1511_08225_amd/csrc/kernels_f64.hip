// kernels_f64.hip -- FP64 particles and grids.  Built without floating-point
// contraction so that the beta = 1 path is the standard leapfrog arithmetic.
#include "kernels.inc"
#include "launch.h"

#define SLPIC_T double
#define SLPIC_SUFFIX f64
#include "launchers.inc"
