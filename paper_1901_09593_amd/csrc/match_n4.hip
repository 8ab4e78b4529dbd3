// Matching kernels for (2n+1)x(2n+1) windows with n = 4.
#include "match_impl.hpp"

namespace msibm {
hipError_t launch_match_n4(int dtype, int mode, int nc, const MatchArgs& a, hipStream_t s)
{
    return dispatch_match<4>(dtype, mode, nc, a, s);
}
hipError_t launch_match_multi_n4(int dtype, int mode, int nc, const MultiArgs& a, int blocks, hipStream_t s)
{
    return dispatch_match_multi<4>(dtype, mode, nc, a, blocks, s);
}
}  // namespace msibm
