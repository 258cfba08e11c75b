// 2-D instantiations of the fused stage kernel (rhd_stage.hpp). They sit in a
// file of their own because they are compiled with the default scheduler: the
// plain 2-D kernels run four waves per SIMD, which fits their registers without
// spills only under that scheduler, while the 1-D and 3-D kernels in
// rhd_forward.hip schedule for instruction-level parallelism.
#include "rhd_stage.hpp"

namespace rhd {

hipError_t launch_stage_2d(const DevParams& P, int mode, bool mixed, const double* ysten,
                           const double* yown, double* yout, const double* rho, const double* kP,
                           const double* kF, double dt, unsigned long long* err, hipStream_t s) {
  return launch_stage_nd<2>(P, mode, mixed, ysten, yown, yout, rho, kP, kF, dt, err, s);
}

}  // namespace rhd
