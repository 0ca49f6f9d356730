// 2D step kernels, state type double, 4 cells per lane.
#include "she_step_nd.hpp"

namespace she {
template hipError_t step2d_e<double, 4>(int, int, int, hipStream_t, const ParamsND &, const void *, void *,
                                         const StepArg &, double *, InstAcc *, const SkRows *);
}  // namespace she
