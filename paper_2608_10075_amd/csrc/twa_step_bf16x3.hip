// Step kernels of the BF16 x3 (split) contraction (see twa_step_impl.h).
#include "twa_step_impl.h"

namespace twa {

template int launch_gemm_p<TWA_PREC_BF16X3>(const Geometry&, const EnsembleBuffers&, const StepConsts&, int, bool, int, bool, bool,
                               hipStream_t);

}  // namespace twa
