// Internal declarations shared by the C-ABI layer and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/kf.h"
#include "kf_matmap.hpp"
#include "kf_steer.hpp"

namespace kfmi {

constexpr int kMaxLayers = 64;
constexpr int kMaxDevices = 64;   // devices the static scratch of kf_find_noalloc tracks

// Device-resident workspace, grown on demand and reused between calls.
struct Workspace {
    void* ptr = nullptr;
    size_t bytes = 0;
    // returns nullptr on failure
    void* get(size_t need);
    void release();
};

// Device copies of the learned guess's weights read by the forward pass
// (rounded to bf16).
struct MlpDev {
    const uint16_t* w1;    // [64][16] W1 [out][in] twice along K (high and low input parts)
    const uint16_t* w2;    // [64][64] W2 [out][in]
    const uint16_t* w2t;   // [64][64] W2 transposed [in][out]
    const float* bias;     // [193] b1 [0,64), b2 [64,128), w3 [128,192), b3 [192]
};

// Device state of the network: FP32 master weights and Adam moments (flat
// parameter order), and the copies the forward pass reads.
struct MlpBuffers {
    float* master = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    float* bias = nullptr;
    uint16_t* w1 = nullptr;
    uint16_t* w2 = nullptr;
    uint16_t* w2t = nullptr;
    MlpDev dev() const { return MlpDev{w1, w2, w2t, bias}; }
};

// One Adam update: step size, moment decays, epsilon and the bias
// corrections 1 / (1 - beta^t) of this step.
struct AdamStep {
    float lr, beta1, beta2, eps, c1, c2;
};

// The captured finding pass of kf_find_batched: seeding, seed fit, binning,
// seed order and the finding kernel as child graphs, separated by event-record
// nodes whose events are swapped per launch (timing or not).
constexpr int kPhaseEvents = 5;
struct FindGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t ev_node[kPhaseEvents] = {};
    uint64_t key[40] = {};          // everything the captured launches depend on
    int nkey = 0;
    bool timed = false;             // ev_node currently point at a timing set
};

}  // namespace kfmi

struct kf_ctx {
    int32_t n_layers = 0;
    kf_layer layers[kfmi::kMaxLayers];
    kf_params params;
    kf_layer* d_layers = nullptr;     // device copy of the geometry
    float* d_mat = nullptr;           // device copy of the material map (x0 then xi)
    kfmi::MatMap mat{};               // its view (x0 == nullptr: no map)
    kfmi::SteerDev* d_steer = nullptr;  // device copy of the tracking regions (nullptr: none)
    int device = 0;
    std::string err;
    kfmi::Workspace ws;               // general scratch of the find path
    int n_cu = 0;                     // compute units of the device
    int max_lds = 0;                  // LDS bytes a workgroup may use
    int find_width = 64;              // lanes per workgroup of the finding kernel
    int find_largest_first = 0;       // tile order
    int occ_cache[2][2][2][2][2][9] = {};  // resident workgroups per CU by (field, steering,
                                           // material map, learned, precision, log2 width)
    int timing_cap = 0;               // event sets available (0: timing off)
    int timing_used = 0;              // event sets recorded since kf_set_timing
    int timing_n = 0;                 // sets requested by kf_set_timing
    hipEvent_t* ev = nullptr;         // [timing_cap][kPhaseEvents] phase boundaries
    hipStream_t cap_stream = nullptr; // private stream the batched pass is captured on
    hipEvent_t idle_ev[kfmi::kPhaseEvents] = {};  // record targets of an untimed graph launch
    kfmi::FindGraph fg;
    void* noalloc_scratch = nullptr;  // device address of kf_find_noalloc's static scratch
    uint64_t setup_gen = 0;           // bumped by every change of the material map or the
                                      // steering, which captured launches take by value
    void* mlp_mem = nullptr;          // device block holding the network buffers
    kfmi::MlpBuffers mlp;             // views into mlp_mem
    bool mlp_loaded = false;
    int64_t mlp_step = 0;             // Adam steps taken since kf_mlp_load
    kfmi::Workspace mlp_ws;           // partial gradients of a training step
};

namespace kfmi {

// Launchers (kernels in kf_fit.hip).  Return hipError_t.
hipError_t launch_seed(const kf_ctx* ctx, const kf_hits* h, const int32_t* seed_hits,
                       kf_tracks* out, int flags, hipStream_t s);
hipError_t launch_propagate(const kf_ctx* ctx, kf_tracks* t, const int32_t* target,
                            float* path_len, int32_t* iters, int flags, hipStream_t s);
hipError_t launch_fit(const kf_ctx* ctx, kf_tracks* t, const kf_hits* h, const int32_t* layer_seq,
                      const int32_t* hit_idx, int32_t max_steps, int flags, hipStream_t s);

}  // namespace kfmi
