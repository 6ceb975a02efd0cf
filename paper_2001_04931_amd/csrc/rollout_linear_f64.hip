// F64 instantiation of the linear-model rollout (rollout_linear.hpp).
#include "rollout_linear.hpp"

namespace empc {
template hipError_t launch_linear<double>(const ProbView<double> &, const double *, const double *, int64_t,
                                        int64_t, double *, hipStream_t, const Events &, int);
}  // namespace empc
