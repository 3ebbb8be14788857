// Device copy of the tracking regions and their layer plans (kf_set_steering).
#pragma once

#include <stdint.h>

namespace kfmi {

constexpr int kMaxRegions = 8;
constexpr int kMaxPlan = 64;

struct SteerDev {
    int32_t n;                              // regions
    int32_t len[kMaxRegions];               // plan lengths
    double eta_lo[kMaxRegions], eta_hi[kMaxRegions];
    uint8_t layers[kMaxRegions][kMaxPlan];  // plans
};

}  // namespace kfmi
