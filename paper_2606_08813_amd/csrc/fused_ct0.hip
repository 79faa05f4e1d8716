// Fused persistent kernel instantiations for FP32 codes.
#include "fused_impl.h"

HNTL_FUSED_TU(0)
