// Fused persistent kernel instantiations for FP8 E4M3 codes.
#include "fused_impl.h"

HNTL_FUSED_TU(2)
