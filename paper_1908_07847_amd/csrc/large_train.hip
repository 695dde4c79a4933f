// Large-N minibatch trainer (placeholder until the persistent kernel lands).
#include "mlp_large.hpp"

namespace mlph {

mlp_status large_workspace_bytes(const mlp_config &, size_t *bytes) {
  *bytes = 0;
  return MLP_ERR_UNSUPPORTED;
}

mlp_status large_train(const mlp_config &, const mlp_params &, float *, void *, size_t, int,
                       const float *, const float *, int, float *, hipStream_t,
                       std::string *err) {
  *err = "no large-N trainer for this configuration";
  return MLP_ERR_UNSUPPORTED;
}

}  // namespace mlph
