// Chain kernels instantiated for state dimension 14.
#include "chain_impl.h"

namespace pg {
template hipError_t launch_chain_n<14>(const DevState&, int, int, int, hipStream_t);
template hipError_t launch_prior_costs_n<14>(const DevState&, int, int, hipStream_t);
template hipError_t launch_iteration_n<14>(const DevState&, int, int, int, hipStream_t);
}  // namespace pg
