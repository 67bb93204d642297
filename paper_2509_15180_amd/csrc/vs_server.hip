// vs_server.hip -- gfx950 kernel that gives server robots a starting state.
//
// A growth step depends on the robot's state only through its joint angles and its
// link and step counts (Alg. 1: the next step appends a link at zero angle to the
// current chain and solves from there), so a robot queued with the first s links of an
// earlier rollout and their joint angles continues that rollout exactly: the batched
// planner (Alg. 2) propagates a child T steps from its parent's state this way instead
// of growing the whole design again.

#include <hip/hip_runtime.h>

#include "vs_device.h"

namespace vs {

// One block per robot of a group, after the group's slots were cleared: robot slots[i]
// takes start[i] links (0: it starts empty and nothing is written) with joint angles
// theta0[row .. row + start[i]), row being its first theta element.  start and theta0
// are pinned host memory at device-visible addresses, written before the launch.
__global__ void slot_start_kernel(KData D, const int* slots, const int* start,
                                  const double* theta0, int count) {
  if ((int)blockIdx.x >= count) return;
  const int s0 = start[blockIdx.x];
  if (s0 <= 0) return;
  const size_t b = (size_t)slots[blockIdx.x];
  const int row = D.ii[kII * b + kThetaOff];
  for (int j = threadIdx.x; j < s0; j += blockDim.x) D.theta[row + j] = theta0[row + j];
  if (threadIdx.x == 0) {
    D.ncur[b] = s0;
    D.tcur[b] = s0;
  }
}

hipError_t launch_slot_start(const KData& D, const int* slots, const int* start,
                             const double* theta0, int count, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  if (!D.ii || !D.theta || !D.ncur || !D.tcur || !slots || !start || !theta0)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(slot_start_kernel, dim3(count), dim3(64), 0, stream, D, slots, start,
                     theta0, count);
  return hipGetLastError();
}

}  // namespace vs
