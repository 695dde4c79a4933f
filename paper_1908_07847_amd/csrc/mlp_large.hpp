// Large-N minibatch trainer (host-side entry points).
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "mlp.h"

namespace mlph {

// Workspace bytes for training n_nets nets of shape cfg on the large-N path
// (MLP_ERR_UNSUPPORTED when no kernel here covers cfg).
mlp_status large_workspace_bytes(const mlp_config &cfg, int n_nets, size_t *bytes);

// The plan the trainer would launch for n_nets nets of shape cfg on n_cu
// CUs: {Gi, Gj, waves, rows staged per piece}.
mlp_status large_plan(const mlp_config &cfg, int n_nets, int n_cu, int shape[5], std::string *err);

// Launch hint for the Gi x Gj grid (0, 0: automatic) and the waves per
// workgroup (0: automatic, else 4 or 8).
void set_large_grid_hint(int row_blocks, int hidden_blocks, int waves);

// Longest a grid-barrier wait may take before it gives up (microseconds;
// negative: the default of 5 s).
void set_wait_limit_us(int64_t us);

// Bytes at the head of a workspace that hold the barrier counters and the
// status words of the last training launch on it.
constexpr size_t kStatusBytes = 2048;

// Zero the status block (stream-ordered).
hipError_t launch_clear_status(void *status_block, hipStream_t s);
// Set the status block's non-finite word if a[0..na) or b[0..nb) holds a NaN
// or an infinity (stream-ordered).
hipError_t launch_check_finite(const float *a, int64_t na, const float *b, int64_t nb, void *status_block,
                               hipStream_t s);
// Synchronise the stream, then map the status words to MLP_OK,
// MLP_ERR_TIMEOUT or MLP_ERR_NONFINITE.
mlp_status read_status(const void *status_block, hipStream_t s, std::string *err);

// Minibatch training for shapes outside the small trainer: n_nets nets of
// shape cfg, parameters packed back to back from theta.W1 (and comp), all
// on the same X and T; lrs (host, n_nets) or cfg.lr for every net.
mlp_status large_train(const mlp_config &cfg, int n_nets, const float *lrs, const mlp_params &theta,
                       float *comp, void *ws, size_t ws_bytes, int n_cu, const float *X, const float *T,
                       int epochs, float *loss_hist, hipStream_t s, std::string *err);

// Bytes of the static scratch behind mlp_train_shared_static (per device).
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;

// large_train on the static scratch of the current device (nothing is
// allocated); MLP_ERR_WORKSPACE when the plan needs more than it holds.
mlp_status large_train_static(const mlp_config &cfg, int n_nets, const float *lrs, const mlp_params &theta,
                              float *comp, int n_cu, const float *X, const float *T, int epochs, float *loss_hist,
                              hipStream_t s, std::string *err);

// Grid-barrier probe (cooperative launch of n_wg workgroups, `rounds`
// barriers); ws holds barrier_probe_workspace_bytes() of counters.
mlp_status barrier_probe(int n_wg, int rounds, void *ws, hipStream_t s, std::string *err);
size_t barrier_probe_workspace_bytes();

// Contraction probe on the trainer's matrix-core instruction (C = A B^T;
// M, N multiples of 16, Kd a multiple of 32).
hipError_t launch_mfma_probe(int prec, const float *A, const float *B, float *C, int M, int N, int Kd,
                             hipStream_t s);

}  // namespace mlph
