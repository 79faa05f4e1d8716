// Fused persistent kernel instantiations for BF16 codes.
#include "fused_impl.h"

HNTL_FUSED_TU(1)
