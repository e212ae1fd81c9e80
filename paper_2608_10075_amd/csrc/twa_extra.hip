// Batched-scan entry points (the grouped scan is not part of this build yet:
// twa_run_batch reports TWA_EINVAL).
#include "twa_internal.h"

extern "C" {

TWA_API void twa_batch_opts_default(twa_batch_opts* o) {
    if (!o) return;
    *o = twa_batch_opts{};
    o->n_traj = 512;
    o->n_steps = 1000;
    o->burnin = -1;
    o->gamma = 1.0;
    o->s0z = 1.0;
    o->precision = TWA_PREC_FP32;
    o->use_graph = 1;
    o->steps_per_graph = 16;
}

TWA_API int twa_run_batch(const twa_point*, int, const twa_batch_opts*, twa_observables*) {
    twa::set_error("twa_run_batch: not available in this build");
    return TWA_EINVAL;
}


}
