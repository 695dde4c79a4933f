// Large-N minibatch trainer (host-side entry points).
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "mlp.h"

namespace mlph {

// Workspace bytes for training cfg on the large-N path (MLP_ERR_UNSUPPORTED
// when no kernel here covers cfg).
mlp_status large_workspace_bytes(const mlp_config &cfg, size_t *bytes);

// Launch hint for the Gi x Gj grid (0, 0: automatic).
void set_large_grid_hint(int row_blocks, int hidden_blocks);

// Minibatch training for shapes outside the small trainer.
mlp_status large_train(const mlp_config &cfg, const mlp_params &theta, float *comp, void *ws,
                       size_t ws_bytes, int n_cu, const float *X, const float *T, int epochs,
                       float *loss_hist, hipStream_t s, std::string *err);

}  // namespace mlph
