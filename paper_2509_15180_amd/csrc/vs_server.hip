// vs_server.hip -- gfx950 kernels of the serving loop's data movement.
//
// Each group of admitted robots is loaded with one launch and read back with one launch:
// a block per robot reads its inputs from the pinned host staging (at the device-visible
// address of that memory) and writes the slab, or reads the slab and writes its results
// to the staging; the host then only polls events.
//
// A growth step depends on the robot's state only through its joint angles and its link
// and step counts (Alg. 1: the next step appends a link at zero angle to the current
// chain and solves from there), so a robot queued with the first s links of an earlier
// rollout and their joint angles continues that rollout exactly: the batched planner
// (Alg. 2) propagates a child T steps from its parent's state this way instead of growing
// the whole design again.

#include "vs_server.h"

namespace vs {

__global__ void slot_load_kernel(SlotInputs in, SlotStage st, int first, int count) {
  if ((int)blockIdx.x >= count) return;
  const int b = st.order[first + blockIdx.x];
  const int* sii = st.ii + (size_t)kII * b;
  const int n = sii[kNTarget], row = sii[kCoverOff], oo = sii[kObsOff], K = sii[kObsCnt];
  const int t = threadIdx.x;
  if (t == 0) in.order[first + blockIdx.x] = b;
  if (t < kII) in.ii[(size_t)kII * b + t] = sii[t];
  if (t < 6) in.dd[6 * (size_t)b + t] = st.dd[6 * (size_t)b + t];
  for (int j = t; j < 2 * n; j += blockDim.x) in.cover[2 * (size_t)row + j] = st.cover[2 * (size_t)row + j];
  for (int k = t; k < K; k += blockDim.x) in.okind[oo + k] = st.okind[oo + k];
  for (int k = t; k < 4 * K; k += blockDim.x) in.obs[4 * (size_t)oo + k] = st.obs[4 * (size_t)oo + k];
}

__global__ void slot_start_kernel(KData D, SlotStage st, int first, int count) {
  if ((int)blockIdx.x >= count) return;
  const int s0 = st.start[first + blockIdx.x];
  if (s0 <= 0) return;
  const size_t b = (size_t)D.order[first + blockIdx.x];
  const int row = D.ii[kII * b + kThetaOff];
  for (int j = threadIdx.x; j < s0; j += blockDim.x) D.theta[row + j] = st.theta[row + j];
  if (threadIdx.x == 0) {
    D.ncur[b] = s0;
    D.tcur[b] = s0;
  }
}

__global__ void slot_store_kernel(KData D, SlotStage st, int first, int count) {
  if ((int)blockIdx.x >= count) return;
  const size_t b = (size_t)D.order[first + blockIdx.x];
  const int* ii = D.ii + kII * b;
  const int n = ii[kNTarget], row = ii[kThetaOff], rec = ii[kRecOff];
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    st.theta[row + j] = D.theta[row + j];
    st.status[row + j] = D.status[rec + j];
  }
  if (threadIdx.x < 3 && n > 0)
    st.tip[3 * ((size_t)row + n - 1) + threadIdx.x] = D.tip[3 * ((size_t)rec + n - 1) + threadIdx.x];
}

hipError_t launch_slot_load(const SlotInputs& in, const SlotStage& st, int first, int count,
                            hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  if (!in.ii || !in.dd || !in.cover || !in.okind || !in.obs || !in.order || !st.ii || !st.dd ||
      !st.cover || !st.okind || !st.obs || !st.order)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(slot_load_kernel, dim3(count), dim3(64), 0, stream, in, st, first, count);
  return hipGetLastError();
}

hipError_t launch_slot_start(const KData& D, const SlotStage& st, int first, int count,
                             hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  if (!D.ii || !D.order || !D.theta || !D.ncur || !D.tcur || !st.start || !st.theta)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(slot_start_kernel, dim3(count), dim3(64), 0, stream, D, st, first, count);
  return hipGetLastError();
}

hipError_t launch_slot_store(const KData& D, const SlotStage& st, int first, int count,
                             hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  if (!D.ii || !D.order || !D.theta || !D.status || !D.tip || !st.theta || !st.status || !st.tip)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(slot_store_kernel, dim3(count), dim3(64), 0, stream, D, st, first, count);
  return hipGetLastError();
}

}  // namespace vs
