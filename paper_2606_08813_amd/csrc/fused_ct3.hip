// Fused persistent kernel instantiations for the int16 codes of eq. 5.
#include "fused_impl.h"

HNTL_FUSED_TU(3)
