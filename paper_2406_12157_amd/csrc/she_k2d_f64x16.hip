// 2D step kernels, state type double, 16 cells per lane.
#include "she_step_nd.hpp"

namespace she {
template hipError_t step2d_e<double, 16>(int, int, int, hipStream_t, const ParamsND &, const void *, void *,
                                         const StepArg &, double *, InstAcc *, const SkRows *);
}  // namespace she
