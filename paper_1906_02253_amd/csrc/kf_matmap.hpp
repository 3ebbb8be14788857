// Device view of the r-z material map (kf_set_material).
#pragma once

#include <stdint.h>

namespace kfmi {

// x0 == nullptr: no map (the layers' own x0, no energy loss).  Arrays
// [nr][nz]: radiation-length fraction and areal density [g/cm^2].
struct MatMap {
    const float* x0;
    const float* xi;
    int32_t nr, nz;
    double r_max, z_min, z_max;
};

}  // namespace kfmi
