// Backward kernels for (2n+1)x(2n+1) windows with n = 1.
#include "backward_impl.hpp"

namespace msibm {
hipError_t launch_backward_n1(int nc, const BackArgs& a, hipStream_t s) { return dispatch_backward<1>(nc, a, s); }
hipError_t launch_backward_multi_n1(int nc, const MultiArgs& a, int blocks, hipStream_t s)
{
    return dispatch_backward_multi<1>(nc, a, blocks, s);
}
hipError_t launch_backward_levels_n1(int nc, const BackLevels& a, int blocks, hipStream_t s)
{
    return dispatch_backward_levels<1>(nc, a, blocks, s);
}
}  // namespace msibm
