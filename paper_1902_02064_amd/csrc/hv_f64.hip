// Instantiation of the block H.V kernels in FP64 (separate unit so the two precisions compile in parallel).
#include "hv_kern.h"

namespace trbl {
template void dispatch_hv<double>(HVArgs<double>&, const HVPlan&, hipStream_t, int, unsigned);
}  // namespace trbl
