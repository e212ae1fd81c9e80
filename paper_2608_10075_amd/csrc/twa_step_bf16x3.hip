// Step kernels of the BF16 x3 (split) contraction (see twa_step_impl.h).
#include "twa_step_impl.h"

namespace twa {

template int launch_gemm_p<TWA_PREC_BF16X3>(const Geometry&, const EnsembleBuffers&, const StepConsts&, int, bool, int, bool, bool,
                               hipStream_t);
template int grouped_prepare_p<TWA_PREC_BF16X3>(const std::vector<Geometry>&, const std::vector<EnsembleBuffers>&,
                                   const std::vector<StepConsts>&, int64_t*, bool, GroupedPlan&, hipStream_t);
template int grouped_launch_p<TWA_PREC_BF16X3>(const GroupedPlan&, int, int, int, hipStream_t);
template int launch_call_p<TWA_PREC_BF16X3>(const Geometry&, const GemmCall&, hipStream_t);

}  // namespace twa
