// Instantiation of the evaluation and quantize launchers for F32 storage.
#include "blip_launch.hpp"

namespace blip {
template hipError_t launch_eval<F32>(const KArgs&, const Cfg&, hipStream_t);
template hipError_t launch_ratio<F32>(const KArgs&, const Cfg&, hipStream_t);
template hipError_t launch_quantize<F32>(const float*, char*, int64_t, int, int64_t, float,
                                          hipStream_t);
}  // namespace blip
