// Fused engine (one kernel per iteration, int8 MFMA contraction).
#include "kernels.hpp"

namespace qap {

hipError_t launch_fused_step(const InstDesc&, int*, hipStream_t, hipEvent_t*) { return hipErrorNotSupported; }

hipError_t launch_eval_mfma(const InstDesc&, const uint8_t*, int, long long*, long long*, hipStream_t)
{
    return hipErrorNotSupported;
}

}  // namespace qap
