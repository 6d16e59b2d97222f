// Instantiation of the evaluation and quantize launchers for BF16 storage.
#include "blip_launch.hpp"

namespace blip {
template hipError_t launch_eval<BF16>(const KArgs&, const Cfg&, hipStream_t);
template hipError_t launch_ratio<BF16>(const KArgs&, const Cfg&, hipStream_t);
template hipError_t launch_quantize<BF16>(const float*, char*, int64_t, int, int64_t, float,
                                          hipStream_t);
}  // namespace blip
