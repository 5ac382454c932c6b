// Fibre projections with FP32 input and FP64 output (instantiations of
// the templates in k_fiber.hpp).
#include "k_fiber.hpp"

namespace st {

hipError_t launch_fiber_fd(const FiberIn &in, const FiberW &w, int m0, int mcount,
                           const FiberOut &out, double *partials, Prec prec, hipStream_t s,
                           int *nparts) {
  return fk::launch_fiber_typed<float, double>(in, w, m0, mcount, out, partials, prec, s, nparts);
}

}  // namespace st
