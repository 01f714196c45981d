// collide_ilp.hip -- the batched collision kernel of the mixed form without
// the composition mix and the event log, for either event budget and for
// fixed event counts only, and the FP64 form's for fixed event counts,
// instantiated here so that they can be compiled with the scheduling strategy
// that maximises instruction-level parallelism (the build gives this file
// that flag); launched from collide.hip.
#include "collide_device.hpp"

namespace mcd {

template __global__ void collide_batched<float, 4, true, false, false>(CollideArgs A);
template __global__ void collide_batched<float, 4, true, false, false, kFixedCount>(CollideArgs A);
template __global__ void collide_batched<double, 4, false, false, false, kFixedCount>(CollideArgs A);

}  // namespace mcd
