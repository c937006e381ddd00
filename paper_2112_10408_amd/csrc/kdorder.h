// Device construction of the kd order of segments into blocks and of the
// point offsets in that order: the launchers of the kernels in build.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "host.h"

namespace tnn {

// perm[i] = i for i < n.
hipError_t launch_iota(int32_t *perm, int64_t n, hipStream_t st);

// One level of the kd order (the splits of host::kd_splits for that level,
// n_splits of them, in device memory): each split range of perm is
// partitioned in place along its widest key axis, with tmp (as long as
// perm) as the staging area.  keys: 4 float32 per segment, indexed by the
// entries of perm.
hipError_t launch_kd_level(const float *keys, int32_t *perm, int32_t *tmp,
                           const host::KdSplit *splits, int64_t n_splits, hipStream_t st);

// After the last level: inside every block of kBlockSegs entries of perm
// (the last one shorter) the splits continue down to single entries, a range
// of n entries splitting into its n/2 smallest along its widest axis and the
// rest.
hipError_t launch_kd_leaves(const float *keys, int32_t *perm, int64_t n_seg, hipStream_t st);

// dpstart[i] = sum over j < i of the member count of segment perm[j]
// (cnt_flags bits 0..15); the total must fit in int32.
hipError_t launch_point_offsets(const int32_t *perm, const int32_t *cnt_flags, int64_t n_seg,
                                int32_t *dpstart, hipStream_t st);

}  // namespace tnn
