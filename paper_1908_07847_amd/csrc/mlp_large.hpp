// Large-N minibatch trainer (host-side entry points).
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "mlp.h"

namespace mlph {

// Workspace bytes for training n_nets nets of shape cfg on the large-N path
// (MLP_ERR_UNSUPPORTED when no kernel here covers cfg).
mlp_status large_workspace_bytes(const mlp_config &cfg, int n_nets, size_t *bytes);

// Launch hint for the Gi x Gj grid (0, 0: automatic).
void set_large_grid_hint(int row_blocks, int hidden_blocks);

// Minibatch training for shapes outside the small trainer: n_nets nets of
// shape cfg, parameters packed back to back from theta.W1 (and comp), all
// on the same X and T; lrs (host, n_nets) or cfg.lr for every net.
mlp_status large_train(const mlp_config &cfg, int n_nets, const float *lrs, const mlp_params &theta,
                       float *comp, void *ws, size_t ws_bytes, int n_cu, const float *X, const float *T,
                       int epochs, float *loss_hist, hipStream_t s, std::string *err);

// Grid-barrier probe (cooperative launch of n_wg workgroups, `rounds`
// barriers); ws holds barrier_probe_workspace_bytes() of counters.
mlp_status barrier_probe(int n_wg, int rounds, void *ws, hipStream_t s, std::string *err);
size_t barrier_probe_workspace_bytes();

}  // namespace mlph
