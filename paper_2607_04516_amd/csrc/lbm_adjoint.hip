// Discrete adjoint of the D3Q19 LBM-LES step (not yet built: reports an error).
#include "lbm_launch.h"

namespace lbm {

hipError_t launch_adjoint(const DevCtx&, const void*, const void*, void*, const int*, int, const void*, void*,
                          hipStream_t)
{
    return hipErrorNotSupported;
}

}  // namespace lbm
