// lbrb_analysis.h -- the pose recorder used by rb_record_poses (the trajectory analysis
// itself is the C-ABI lb_traj_* in include/lbrb.h, implemented in lbrb_analysis.hip).
#ifndef LBRB_ANALYSIS_H
#define LBRB_ANALYSIS_H

#include <hip/hip_runtime.h>

#include "lbrb_core.h"

namespace lbrb {

// frame[7 b + (0..2)] = centre, frame[7 b + (3..6)] = quaternion (w,x,y,z) of body b
void launch_record_poses(const Body* bodies, int n_bodies, double* frame, hipStream_t s);

}  // namespace lbrb

#endif
