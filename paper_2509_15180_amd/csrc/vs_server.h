// vs_server.h -- data movement of the serving loop between its pinned host staging and
// the device slab, by kernels that read and write the staging at its device-visible
// addresses (one launch per group instead of a copy call per robot and array).
#pragma once

#include <hip/hip_runtime.h>

#include "vs_device.h"

namespace vs {

// Pinned host staging (hipHostMalloc) at device-visible addresses
// (hipHostGetDevicePointer), laid out at the slab's offsets: per slot, per pool row, per
// obstacle-pool entry, per order entry.
struct SlotStage {
  const int* ii;        // [slots][kII]
  const double* dd;     // [slots][6]
  const double* cover;  // [rows][2]
  const int* okind;     // [obstacle entries]
  const double* obs;    // [obstacle entries][4]
  const int* order;     // each group's slots at its order offsets
  const int* start;     // links each robot of a group starts with, at the order offsets
  double* theta;        // [rows]: starting angles in, final angles out
  double* tip;          // [rows][3]: the final tip pose at the robot's last row
  int* status;          // [rows]: per-step status
};

// Writable views of the slab's input arrays (the ones KData reads).
struct SlotInputs {
  int* ii;
  double* dd;
  double* cover;
  int* okind;
  double* obs;
  int* order;
};

// Inputs of the group's robots (slots st.order[first, first + count)) from staging into
// the slab, and the group's order entries.
hipError_t launch_slot_load(const SlotInputs& in, const SlotStage& st, int first, int count,
                            hipStream_t stream);
// After the slots were cleared: robots with a nonzero start take their starting state.
hipError_t launch_slot_start(const KData& D, const SlotStage& st, int first, int count,
                             hipStream_t stream);
// Results of a finished group into staging: joint angles, per-step statuses, final tip.
hipError_t launch_slot_store(const KData& D, const SlotStage& st, int first, int count,
                             hipStream_t stream);

}  // namespace vs
