// literal.h -- the assignment step on a distance image kept across
// iterations, the literal reading of the loops of Sec. 2.2 and Sec. 3.1 (d is
// set to infinity once, in stage 1).
#pragma once
#include "sslic_internal.h"

namespace sslic {

// One assignment step on dist (FP32 squared distances D^2 [N], +inf where no
// centre has reached yet): for every voxel x, the least D^2 over the centres
// of `it` whose closed window holds x, ties to the smaller k; where it is
// strictly below dist[x], labels[x] and dist[x] take the centre and its D^2.
// Elsewhere both are left as they are, except that with `first` a voxel no
// window holds gets the label of its grid cell (the starting labels of the
// run, written here instead of in a pass of their own).  Needs the records
// and the bin index of the centres (launch_prep, launch_bins).  Returns at
// once when the iteration loop's stop flag is set.
hipError_t launch_assign_persist(const Geo& g, const void* img, const Iter& it, int32_t* labels,
                                 float* dist, int first, hipStream_t s);

}  // namespace sslic
