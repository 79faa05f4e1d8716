// Scan kernels for int16 codes (eq. 5) (one translation unit per code form).
#include "scan_impl.h"

namespace hntl {

void launch_scan_ct3(const Index& ix, const float* T, const float* epsq, int P, int C, const Buckets& b, int list,
                      uint64_t* part, const uint64_t* bound_lists, bool prune, unsigned long long* scored,
                      hipStream_t s) {
  scan_detail::launch_ct<3>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s);
}

}  // namespace hntl
