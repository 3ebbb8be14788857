// Launchers of the network kernels (kf_mlp.hip) for the C-ABI layer.
#pragma once

#include "kf_mlp.hpp"

namespace kfmi {

hipError_t launch_mlp_features(const kf_ctx* ctx, const kf_tracks* t, const int32_t* target,
                               float* feats, int prec, hipStream_t s);
hipError_t launch_mlp_targets(const float* feats, const float* path, int64_t n, int64_t ld,
                              float* target, hipStream_t s);
hipError_t launch_mlp_forward(const MlpDev& m, const float* feats, int64_t n, int64_t ld, float* out,
                              hipStream_t s);
// scratch bytes of one training step over `batch` rows
size_t mlp_partial_bytes(int batch);
// mode 0: gradient and loss only; mode 1: Adam update of the master weights
hipError_t launch_mlp_step(const MlpBuffers& mb, const float* feats, const float* target, int64_t n,
                           int64_t ld, const int32_t* rows, int batch, void* scratch, int mode,
                           const AdamStep& ad, float* grad_out, float* loss_out, hipStream_t s);
hipError_t launch_mlp_publish(const MlpBuffers& mb, hipStream_t s);

}  // namespace kfmi
