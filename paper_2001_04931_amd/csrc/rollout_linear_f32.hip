// F32 instantiation of the linear-model rollout (rollout_linear.hpp).
#include "rollout_linear.hpp"

namespace empc {
template hipError_t launch_linear<float>(const ProbView<float> &, const float *, const float *, int64_t,
                                        int64_t, float *, hipStream_t, const Events &, int);
}  // namespace empc
