// mixed.hip -- FP16 matrix-core Rademacher sketch (in progress).
#include "common.h"
#include "kernels.h"

namespace rcq {

hipError_t launch_sketch_mixed(const float*, int64_t, int, int64_t, int, uint64_t,
                               const SketchPlan&, double*, double*, int64_t, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace rcq
