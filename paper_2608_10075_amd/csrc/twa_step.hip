// Dispatch of the step kernels (templates in twa_step_impl.h, one translation
// unit per contraction precision): tile configurations, the launchers of the
// forward, response, store and adjoint contractions, and the grouped launches
// of the batched scan.
#include <algorithm>
#include <vector>

#include "twa_internal.h"

namespace twa {

// ---------------------------------------------------------------------------
// tile configurations
static const TileCfg kCfgs[] = {
    {0, 16, 32, 64, 1, 1, 2, "16x32 K64B 1w 2st"},
    {1, 64, 64, 64, 2, 2, 4, "64x64 K64B 4w 4st"},
    {2, 128, 128, 128, 2, 2, 4, "128x128 K128B 4w 4st"},
    {3, 128, 128, 64, 2, 2, 8, "128x128 K64B 4w 8st"},
    {4, 256, 128, 64, 4, 1, 6, "256x128 K64B 4w 6st"},
    {5, 128, 256, 64, 2, 2, 6, "128x256 K64B 4w 6st"},
    {6, 256, 128, 64, 4, 2, 4, "256x128 K64B 8w 4st"},
    {7, 320, 256, 128, 4, 2, 2, "320x256 K128B 8w 2st"},
    {8, 320, 256, 64, 4, 2, 4, "320x256 K64B 8w 4st"},
};
int n_tile_cfgs() { return (int)(sizeof(kCfgs) / sizeof(kCfgs[0])); }
const TileCfg& tile_cfg(int id) { return kCfgs[id]; }

int launch_gemm(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, int stage, bool tangent,
                int cur, bool store_y2, bool keep_dlt, hipStream_t st) {
    switch (g.precision) {
        case TWA_PREC_FP64: return launch_gemm_p<TWA_PREC_FP64>(g, b, c, stage, tangent, cur, store_y2, keep_dlt, st);
        case TWA_PREC_FP32: return launch_gemm_p<TWA_PREC_FP32>(g, b, c, stage, tangent, cur, store_y2, keep_dlt, st);
        case TWA_PREC_BF16: return launch_gemm_p<TWA_PREC_BF16>(g, b, c, stage, tangent, cur, store_y2, keep_dlt, st);
        case TWA_PREC_FP16: return launch_gemm_p<TWA_PREC_FP16>(g, b, c, stage, tangent, cur, store_y2, keep_dlt, st);
        case TWA_PREC_BF16X3:
            return launch_gemm_p<TWA_PREC_BF16X3>(g, b, c, stage, tangent, cur, store_y2, keep_dlt, st);
    }
    set_error("unknown precision");
    return TWA_EINVAL;
}

int launch_gemm_call(const Geometry& g, const GemmCall& c, hipStream_t st) {
    switch (g.precision) {
        case TWA_PREC_FP64: return launch_call_p<TWA_PREC_FP64>(g, c, st);
        case TWA_PREC_FP32: return launch_call_p<TWA_PREC_FP32>(g, c, st);
        case TWA_PREC_BF16: return launch_call_p<TWA_PREC_BF16>(g, c, st);
        case TWA_PREC_FP16: return launch_call_p<TWA_PREC_FP16>(g, c, st);
        case TWA_PREC_BF16X3: return launch_call_p<TWA_PREC_BF16X3>(g, c, st);
    }
    set_error("unknown precision");
    return TWA_EINVAL;
}


int grouped_prepare(const std::vector<Geometry>& gs, const std::vector<EnsembleBuffers>& bs,
                    const std::vector<StepConsts>& cs, int64_t* step, bool tangents, GroupedPlan& pl,
                    hipStream_t st) {
    if (gs.empty()) return TWA_EINVAL;
    switch (gs[0].precision) {
        case TWA_PREC_FP32: return grouped_prepare_p<TWA_PREC_FP32>(gs, bs, cs, step, tangents, pl, st);
        case TWA_PREC_BF16: return grouped_prepare_p<TWA_PREC_BF16>(gs, bs, cs, step, tangents, pl, st);
        case TWA_PREC_FP16: return grouped_prepare_p<TWA_PREC_FP16>(gs, bs, cs, step, tangents, pl, st);
        case TWA_PREC_FP64: return grouped_prepare_p<TWA_PREC_FP64>(gs, bs, cs, step, tangents, pl, st);
        case TWA_PREC_BF16X3: return grouped_prepare_p<TWA_PREC_BF16X3>(gs, bs, cs, step, tangents, pl, st);
    }
    set_error("unknown precision");
    return TWA_EINVAL;
}

int grouped_launch(const GroupedPlan& pl, int stage, int cur, int variant, hipStream_t st) {
    if (variant < 0 || variant >= GV_COUNT || (variant != GV_PRIMAL && !pl.tangents)) {
        set_error("grouped launch: variant not prepared");
        return TWA_EINVAL;
    }
    switch (pl.precision) {
        case TWA_PREC_FP32: return grouped_launch_p<TWA_PREC_FP32>(pl, stage, cur, variant, st);
        case TWA_PREC_BF16: return grouped_launch_p<TWA_PREC_BF16>(pl, stage, cur, variant, st);
        case TWA_PREC_FP16: return grouped_launch_p<TWA_PREC_FP16>(pl, stage, cur, variant, st);
        case TWA_PREC_FP64: return grouped_launch_p<TWA_PREC_FP64>(pl, stage, cur, variant, st);
        case TWA_PREC_BF16X3: return grouped_launch_p<TWA_PREC_BF16X3>(pl, stage, cur, variant, st);
    }
    set_error("unknown precision");
    return TWA_EINVAL;
}

void grouped_free(GroupedPlan& pl) {
    for (int v = 0; v < GV_COUNT; ++v)
        for (int s = 0; s < 2; ++s)
            for (int c = 0; c < 2; ++c) hipFree(pl.d_args[v][s][c]);
    for (int t = 0; t < 2; ++t) hipFree(pl.d_tiles[t]);
    pl = GroupedPlan();
}

}  // namespace twa
