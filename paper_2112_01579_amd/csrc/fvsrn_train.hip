// Training kernels (placeholder until the trainer lands).
#include "fvsrn_common.hpp"

namespace fvsrn_detail {

size_t train_workspace_bytes(const NetDev&, long long) { return 0; }

int launch_train(const NetDev&, float*, float*, float*, float*, const float*, long long, const float*, const float*,
                 int, float, float, float, float, float, int, float*, float*, float*, float*, float*, void*, size_t,
                 void*) {
  return 1;
}

}  // namespace fvsrn_detail
