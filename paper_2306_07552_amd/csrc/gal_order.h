// Raster queue order computed inside the robot-step launch (not part of the
// ABI): one extra workgroup of the robot kernel sorts the work items by the
// previous step's measured times while the other workgroups step the envs,
// so the order costs no launch of its own on the step's critical path.
#pragma once

#include "gal_internal.h"

namespace gal {

struct ItemOrder {
    const uint32_t *cost;   // [n] last step's time per work item
    int32_t n;              // items to order (0: no ordering in this launch)
    uint32_t *order;        // [n] out: queue position -> work item
};

hipError_t launch_robot_step(const RobotParams &rp, const SimBuffers &sb, const float *actions,
                             const StepOutputs &out, uint32_t *queue_reset, int lanes_per_env,
                             const ItemOrder &ord, hipStream_t s);

}  // namespace gal
