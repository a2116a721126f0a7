// Local Metropolis sampler (placeholder translation unit, filled in below).
#include "common.h"
#include "kernels.h"
