// Instantiation of the block H.V kernels in FP32 (separate unit so the two precisions compile in parallel).
#include "hv_kern.h"

namespace trbl {
template void dispatch_hv<float>(HVArgs<float>&, const HVPlan&, hipStream_t, int, unsigned);
}  // namespace trbl
