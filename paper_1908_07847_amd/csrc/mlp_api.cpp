// Host side of libmlp: argument validation, workspace sizing and dispatch
// to the HIP kernels.  Validation never calls HIP, so a rejected call
// leaves nothing on the stream and can be tested without a GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "mlp.h"
#include "deep.hpp"
#include "mlp_device.hpp"
#include "mlp_large.hpp"

struct mlp_net {
  mlp_config cfg;
  mlp_params theta;
  float *comp;
  void *ws;
  size_t ws_bytes;
  int device;
  int n_cu;
  float mu;         // momentum rate (0: plain gradient descent)
  float *velocity;  // [P] packed, device; null without momentum
};

namespace {

thread_local std::string g_last_error;
mlp_launch_hint g_hint{};

mlp_status fail(mlp_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

mlp_status hip_fail(hipError_t e, const char *where) {
  return fail(MLP_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
bool aligned4(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

int64_t n_params(int64_t D, int64_t H, int64_t K) { return D * H + H + H * K + K; }

mlp_status check_config(const mlp_config *c) {
  if (!c) return fail(MLP_ERR_ARG, "config is NULL");
  if (c->n_in <= 0 || c->n_hidden <= 0 || c->n_out <= 0 || c->n_rows <= 0)
    return fail(MLP_ERR_SHAPE, "n_in, n_hidden, n_out and n_rows must be positive (got %d, %d, %d, %lld)",
                c->n_in, c->n_hidden, c->n_out, (long long)c->n_rows);
  if (c->batch < 0) return fail(MLP_ERR_SHAPE, "batch must be >= 0");
  if (c->n_out > mlpk::kLayerMaxOut)
    return fail(MLP_ERR_SHAPE, "n_out %d above the supported %d", c->n_out, mlpk::kLayerMaxOut);
  if (c->n_in > (1 << 20) || c->n_hidden > (1 << 20))
    return fail(MLP_ERR_SHAPE, "n_in / n_hidden above 2^20");
  if (c->prec != MLP_FP32 && c->prec != MLP_BF16 && c->prec != MLP_FP8_E4M3)
    return fail(MLP_ERR_ARG, "unknown precision %d", c->prec);
  if (c->flags & ~(uint32_t)(MLP_F_COMPENSATED | MLP_F_DETERMINISTIC | MLP_F_CHECK_FINITE | MLP_F_TANH_HIDDEN))
    return fail(MLP_ERR_ARG, "unknown flag bits 0x%x", c->flags);
  if (!(c->lr >= 0.0f) || c->lr > 1e6f) return fail(MLP_ERR_ARG, "lr must be finite and >= 0");
  return MLP_OK;
}

mlp_status check_params(mlp_params p, const char *what) {
  if (!p.W1 || !p.b1 || !p.W2 || !p.b2) return fail(MLP_ERR_ARG, "%s: a parameter pointer is NULL", what);
  if (!aligned4(p.W1) || !aligned4(p.b1) || !aligned4(p.W2) || !aligned4(p.b2))
    return fail(MLP_ERR_ALIGN, "%s: parameter pointers must be 4-byte aligned", what);
  return MLP_OK;
}

int64_t eff_batch(const mlp_config &c) { return (c.batch <= 0 || c.batch >= c.n_rows) ? c.n_rows : c.batch; }

bool small_path(const mlp_config &c) {
  return c.prec == MLP_FP32 && eff_batch(c) == c.n_rows && c.n_rows <= MLP_SMALL_MAX_ROWS &&
         c.n_hidden <= MLP_SMALL_MAX_HIDDEN && c.n_in <= MLP_SMALL_MAX_IN &&
         c.n_out <= MLP_SMALL_MAX_OUT;
}

int act_of(const mlp_config &c) { return (c.flags & MLP_F_TANH_HIDDEN) ? 1 : 0; }

size_t backward_ws_bytes(const mlp_config &c) {
  const int64_t rows = std::min<int64_t>(c.n_rows, mlph::kBackwardChunk);
  return sizeof(float) * (size_t)rows * (size_t)(c.n_hidden + c.n_out + 1);
}

}  // namespace

extern "C" {

const char *mlp_status_string(mlp_status s) {
  switch (s) {
    case MLP_OK: return "ok";
    case MLP_ERR_ARG: return "invalid argument";
    case MLP_ERR_SHAPE: return "unsupported or inconsistent shape";
    case MLP_ERR_ALIGN: return "misaligned device pointer";
    case MLP_ERR_WORKSPACE: return "workspace missing or too small";
    case MLP_ERR_UNSUPPORTED: return "unsupported request";
    case MLP_ERR_HIP: return "HIP runtime error";
    case MLP_ERR_TIMEOUT: return "a grid-wide wait gave up";
    case MLP_ERR_NONFINITE: return "non-finite parameter or loss";
  }
  return "unknown status";
}

const char *mlp_last_error(void) { return g_last_error.c_str(); }

mlp_status mlp_set_launch_hint(const mlp_launch_hint *hint) {
  if (!hint) {
    g_hint = mlp_launch_hint{};
    mlph::set_large_grid_hint(0, 0, 0);
    return MLP_OK;
  }
  const int t = hint->small_threads;
  if (t != 0 && t != 64 && t != 128 && t != 256 && t != 512)
    return fail(MLP_ERR_ARG, "small_threads must be 0, 64, 128, 256 or 512");
  if (hint->large_row_blocks < 0 || hint->large_row_blocks > 256 || hint->large_hidden_blocks < 0 ||
      hint->large_hidden_blocks > 16)
    return fail(MLP_ERR_ARG, "large grid hint outside [0,256] x [0,16]");
  if ((hint->large_row_blocks == 0) != (hint->large_hidden_blocks == 0))
    return fail(MLP_ERR_ARG, "give both large grid dimensions or neither");
  if (hint->large_waves != 0 && hint->large_waves != 4 && hint->large_waves != 8)
    return fail(MLP_ERR_ARG, "large_waves must be 0, 4 or 8");
  g_hint = *hint;
  mlph::set_large_grid_hint(hint->large_row_blocks, hint->large_hidden_blocks, hint->large_waves);
  return MLP_OK;
}

mlp_status mlp_large_plan(const mlp_config *cfg, int32_t n_nets, int32_t n_cu, int32_t shape[5]) {
  mlp_status s = check_config(cfg);
  if (s != MLP_OK) return s;
  if (!shape) return fail(MLP_ERR_ARG, "shape is NULL");
  if (n_cu < 1) return fail(MLP_ERR_ARG, "n_cu must be >= 1");
  if (n_nets < 1 || n_nets > MLP_MAX_SHARED_NETS) return fail(MLP_ERR_ARG, "n_nets must be in 1..%d", MLP_MAX_SHARED_NETS);
  int out[5] = {0, 0, 0, 0, 0};
  s = mlph::large_plan(*cfg, n_nets, n_cu, out, &g_last_error);
  if (s != MLP_OK) return s;
  for (int i = 0; i < 5; ++i) shape[i] = out[i];
  return MLP_OK;
}

mlp_status mlp_workspace_size(const mlp_config *cfg, size_t *bytes) {
  mlp_status s = check_config(cfg);
  if (s != MLP_OK) return s;
  if (!bytes) return fail(MLP_ERR_ARG, "bytes is NULL");
  size_t need = mlph::kStatusBytes + backward_ws_bytes(*cfg);
  if (!small_path(*cfg)) {
    size_t lw = 0;
    s = mlph::large_workspace_bytes(*cfg, 1, &lw);
    if (s != MLP_OK && s != MLP_ERR_UNSUPPORTED) return s;
    if (s == MLP_OK) need = std::max(need, lw);
  }
  *bytes = (need + 255) / 256 * 256;
  return MLP_OK;
}

mlp_status mlp_init(mlp_net **out, const mlp_config *cfg, mlp_params theta, float *comp,
                    void *workspace, size_t ws_bytes) {
  if (!out) return fail(MLP_ERR_ARG, "out is NULL");
  *out = nullptr;
  mlp_status s = check_config(cfg);
  if (s != MLP_OK) return s;
  if ((s = check_params(theta, "theta")) != MLP_OK) return s;
  if ((cfg->flags & MLP_F_COMPENSATED) && !comp)
    return fail(MLP_ERR_ARG, "MLP_F_COMPENSATED needs a compensation buffer");
  if (comp && !aligned4(comp)) return fail(MLP_ERR_ALIGN, "comp must be 4-byte aligned");
  size_t need = 0;
  mlp_workspace_size(cfg, &need);
  if (ws_bytes < need || (need > 0 && !workspace))
    return fail(MLP_ERR_WORKSPACE, "workspace of %zu bytes given, %zu needed", ws_bytes, need);
  if (workspace && !aligned16(workspace)) return fail(MLP_ERR_ALIGN, "workspace must be 16-byte aligned");
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
  mlp_net *n = new (std::nothrow) mlp_net;
  if (!n) return fail(MLP_ERR_ARG, "out of host memory");
  n->cfg = *cfg;
  n->theta = theta;
  n->comp = (cfg->flags & MLP_F_COMPENSATED) ? comp : nullptr;
  n->ws = workspace;
  n->ws_bytes = ws_bytes;
  n->device = dev;
  n->n_cu = ncu;
  n->mu = 0.0f;
  n->velocity = nullptr;
  *out = n;
  return MLP_OK;
}

mlp_status mlp_destroy(mlp_net *net) {
  if (!net) return fail(MLP_ERR_ARG, "net is NULL");
  delete net;
  return MLP_OK;
}

mlp_status mlp_forward(mlp_net *net, const float *X, int64_t n, float *A, float *Y, void *stream) {
  if (!net) return fail(MLP_ERR_ARG, "net is NULL");
  if (!X || !Y) return fail(MLP_ERR_ARG, "X and Y must not be NULL");
  if (n <= 0) return fail(MLP_ERR_SHAPE, "n must be positive");
  if (!aligned16(X) || !aligned4(Y) || (A && !aligned4(A)))
    return fail(MLP_ERR_ALIGN, "X must be 16-byte and A, Y 4-byte aligned");
  const mlp_config &c = net->cfg;
  hipError_t e = mlph::launch_forward(n, c.n_in, c.n_hidden, c.n_out, X, net->theta, A, Y, act_of(c),
                                      (hipStream_t)stream);
  return e == hipSuccess ? MLP_OK : hip_fail(e, "mlp_forward launch");
}

mlp_status mlp_predict(mlp_net *net, const float *X, int64_t n, float *Y, int32_t *labels, const float *T,
                       int32_t *correct, void *stream) {
  if (!net) return fail(MLP_ERR_ARG, "net is NULL");
  if (!X || !Y || !labels) return fail(MLP_ERR_ARG, "X, Y and labels must not be NULL");
  if ((T == nullptr) != (correct == nullptr)) return fail(MLP_ERR_ARG, "give T and correct together");
  if (n <= 0) return fail(MLP_ERR_SHAPE, "n must be positive");
  if (!aligned16(X) || !aligned4(Y) || !aligned4(labels) || (T && !aligned4(T)) || (correct && !aligned4(correct)))
    return fail(MLP_ERR_ALIGN, "X must be 16-byte and Y, labels, T, correct 4-byte aligned");
  const mlp_config &c = net->cfg;
  hipError_t e = mlph::launch_predict(n, c.n_in, c.n_hidden, c.n_out, X, net->theta, Y, labels, T, correct,
                                      act_of(c), (hipStream_t)stream);
  return e == hipSuccess ? MLP_OK : hip_fail(e, "mlp_predict launch");
}

mlp_status mlp_backward(mlp_net *net, const float *X, const float *A, const float *Y,
                        const float *dY, const float *T, int64_t n, mlp_params grads, float *dX,
                        float *loss, void *stream) {
  if (!net) return fail(MLP_ERR_ARG, "net is NULL");
  if (!X || !A || !Y) return fail(MLP_ERR_ARG, "X, A and Y must not be NULL");
  if (!dY && !T) return fail(MLP_ERR_ARG, "either dY or T must be given");
  if (n <= 0) return fail(MLP_ERR_SHAPE, "n must be positive");
  const mlp_config &c = net->cfg;
  mlp_status s = check_params(grads, "grads");
  if (s != MLP_OK) return s;
  const void *ptrs[] = {A, Y, dY, T, dX, loss};
  for (const void *p : ptrs)
    if (p && !aligned4(p)) return fail(MLP_ERR_ALIGN, "device pointers must be 4-byte aligned");
  if (!aligned16(X)) return fail(MLP_ERR_ALIGN, "X must be 16-byte aligned");
  if (!net->ws || net->ws_bytes < mlph::kStatusBytes + backward_ws_bytes(c))
    return fail(MLP_ERR_WORKSPACE, "backward needs %zu workspace bytes",
                mlph::kStatusBytes + backward_ws_bytes(c));
  const int64_t ws_rows = std::min<int64_t>(c.n_rows, mlph::kBackwardChunk);
  // the workspace's head holds the status block of training launches
  float *scratch = reinterpret_cast<float *>(static_cast<char *>(net->ws) + mlph::kStatusBytes);
  hipError_t e = mlph::launch_backward(n, ws_rows, c.n_in, c.n_hidden, c.n_out, X, A, Y, dY, T,
                                       net->theta, grads, dX, loss, scratch, act_of(c), (hipStream_t)stream);
  return e == hipSuccess ? MLP_OK : hip_fail(e, "mlp_backward launch");
}

mlp_status mlp_step(mlp_net *net, mlp_params grads, float lr, void *stream) {
  if (!net) return fail(MLP_ERR_ARG, "net is NULL");
  mlp_status s = check_params(grads, "grads");
  if (s != MLP_OK) return s;
  if (!(lr >= 0.0f) || lr > 1e6f) return fail(MLP_ERR_ARG, "lr must be finite and >= 0");
  const mlp_config &c = net->cfg;
  hipError_t e = mlph::launch_step(c.n_in, c.n_hidden, c.n_out, net->theta, grads, net->comp, lr, net->mu,
                                   net->velocity, (hipStream_t)stream);
  return e == hipSuccess ? MLP_OK : hip_fail(e, "mlp_step launch");
}

mlp_status mlp_train(mlp_net *net, const float *X, const float *T, int32_t epochs,
                     float *loss_hist, void *stream) {
  if (!net) return fail(MLP_ERR_ARG, "net is NULL");
  if (!X || !T) return fail(MLP_ERR_ARG, "X and T must not be NULL");
  if (epochs < 0) return fail(MLP_ERR_ARG, "epochs must be >= 0");
  if (!aligned16(X) || !aligned16(T) || (loss_hist && !aligned4(loss_hist)))
    return fail(MLP_ERR_ALIGN, "X and T must be 16-byte and loss_hist 4-byte aligned");
  if (epochs == 0) return MLP_OK;
  const mlp_config &c = net->cfg;
  const mlp_params &p = net->theta;
  if (small_path(c)) {
    // The small trainer reads the parameters packed; a single net whose
    // four arrays are laid out back to back is trained in place, any other
    // layout is rejected rather than silently copied.
    const int64_t D = c.n_in, H = c.n_hidden, K = c.n_out;
    if (p.b1 != p.W1 + D * H || p.W2 != p.b1 + H || p.b2 != p.W2 + H * K)
      return fail(MLP_ERR_UNSUPPORTED,
                  "full-batch small training needs W1, b1, W2, b2 contiguous in packed order");
    mlp_batch_item one{};
    one.n_rows = (int32_t)c.n_rows;
    one.n_hidden = (int32_t)H;
    one.lr = c.lr;
    one.x_off = 0;
    one.p_off = 0;
    // the tanh variant runs 8 waves per net (its only instances)
    const int threads = act_of(c) ? 512 : mlph::small_threads(1, g_hint.small_threads);
    if (act_of(c) && mlph::small_lds_bytes((int)c.n_rows, (int)H, (int)D, 512, net->velocity != nullptr) >
                         160 * 1024)
      return fail(MLP_ERR_UNSUPPORTED, "the tanh variant's 8-wave plan does not fit in LDS at this shape");
    hipError_t e = mlph::launch_clear_status(net->ws, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mlp_train status block");
    e = mlph::launch_small_train(nullptr, one, 1, (int)D, (int)K, (int)c.n_rows, (int)H, X, T, p.W1, net->comp,
                                 epochs, loss_hist, act_of(c), net->mu, net->velocity, threads, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mlp_train (small) launch");
    if (c.flags & MLP_F_CHECK_FINITE) {
      e = mlph::launch_check_finite(p.W1, n_params(D, H, K), loss_hist, loss_hist ? epochs : 0, net->ws,
                                    (hipStream_t)stream);
      if (e != hipSuccess) return hip_fail(e, "mlp_train finite check");
    }
    return MLP_OK;
  }
  if (act_of(c) != 0 || net->velocity)
    return fail(MLP_ERR_UNSUPPORTED, "the large-N trainer (minibatches or large shapes) trains the sigmoid "
                                     "network without momentum only");
  return mlph::large_train(net->cfg, 1, nullptr, net->theta, net->comp, net->ws, net->ws_bytes, net->n_cu,
                           X, T, epochs, loss_hist, (hipStream_t)stream, &g_last_error);
}

mlp_status mlp_train_batched(const mlp_batch_item *items_host, const mlp_batch_item *items_dev,
                             int32_t n_nets, int32_t n_in, int32_t n_out, const float *X_packed,
                             const float *T_packed, int64_t total_rows, float *theta_packed,
                             float *comp_packed, int64_t total_params, int32_t epochs,
                             float *loss_hist, void *stream) {
  if (!items_host || !items_dev) return fail(MLP_ERR_ARG, "item tables must not be NULL");
  if (n_nets <= 0) return fail(MLP_ERR_SHAPE, "n_nets must be positive");
  if (n_in <= 0 || n_in > MLP_SMALL_MAX_IN || n_out <= 0 || n_out > MLP_SMALL_MAX_OUT)
    return fail(MLP_ERR_SHAPE, "n_in must be in [1,%d] and n_out in [1,%d]", MLP_SMALL_MAX_IN,
                MLP_SMALL_MAX_OUT);
  if (!X_packed || !T_packed || !theta_packed) return fail(MLP_ERR_ARG, "X, T, theta must not be NULL");
  if (epochs < 0) return fail(MLP_ERR_ARG, "epochs must be >= 0");
  const void *ptrs[] = {items_dev, X_packed, T_packed};
  for (const void *p : ptrs)
    if (p && !aligned16(p)) return fail(MLP_ERR_ALIGN, "items, X and T must be 16-byte aligned");
  const void *ptrs4[] = {theta_packed, comp_packed, loss_hist};
  for (const void *p : ptrs4)
    if (p && !aligned4(p)) return fail(MLP_ERR_ALIGN, "theta, comp, loss_hist must be 4-byte aligned");
  for (int32_t i = 0; i < n_nets; ++i) {
    const mlp_batch_item &it = items_host[i];
    if (it.n_rows <= 0 || it.n_rows > MLP_SMALL_MAX_ROWS || it.n_hidden <= 0 ||
        it.n_hidden > MLP_SMALL_MAX_HIDDEN)
      return fail(MLP_ERR_SHAPE, "net %d: n_rows %d / n_hidden %d outside [1,%d] / [1,%d]", i,
                  it.n_rows, it.n_hidden, MLP_SMALL_MAX_ROWS, MLP_SMALL_MAX_HIDDEN);
    if (it.reserved != 0) return fail(MLP_ERR_ARG, "net %d: reserved field must be 0", i);
    if (!(it.lr >= 0.0f) || it.lr > 1e6f) return fail(MLP_ERR_ARG, "net %d: bad lr", i);
    if (it.x_off < 0 || it.x_off + it.n_rows > total_rows)
      return fail(MLP_ERR_SHAPE, "net %d: rows [%lld, %lld) outside the %lld packed rows", i,
                  (long long)it.x_off, (long long)(it.x_off + it.n_rows), (long long)total_rows);
    if (it.p_off < 0 || it.p_off + n_params(n_in, it.n_hidden, n_out) > total_params)
      return fail(MLP_ERR_SHAPE, "net %d: parameters outside the %lld packed floats", i,
                  (long long)total_params);
  }
  if (epochs == 0) return MLP_OK;
  int max_rows = 0, max_h = 0;
  for (int32_t i = 0; i < n_nets; ++i) {
    max_rows = std::max(max_rows, items_host[i].n_rows);
    max_h = std::max(max_h, items_host[i].n_hidden);
  }
  mlp_batch_item none{};
  hipError_t e = mlph::launch_small_train(items_dev, none, n_nets, n_in, n_out, max_rows, max_h, X_packed,
                                          T_packed, theta_packed, comp_packed, epochs, loss_hist, 0, 0.0f,
                                          nullptr, mlph::small_threads(n_nets, g_hint.small_threads),
                                          (hipStream_t)stream);
  return e == hipSuccess ? MLP_OK : hip_fail(e, "mlp_train_batched launch");
}

mlp_status mlp_eval_batched(const mlp_batch_item *items_host, const mlp_batch_item *items_dev, int32_t n_nets,
                            int32_t n_in, int32_t n_out, const float *X_packed, const float *T_packed,
                            int64_t total_rows, const float *theta_packed, int64_t total_params, float *loss,
                            int32_t *correct, void *stream) {
  if (!items_host || !items_dev) return fail(MLP_ERR_ARG, "item tables must not be NULL");
  if (n_nets <= 0) return fail(MLP_ERR_SHAPE, "n_nets must be positive");
  if (n_in <= 0 || n_in > (1 << 20) || n_out <= 0 || n_out > MLP_SMALL_MAX_OUT)
    return fail(MLP_ERR_SHAPE, "n_in must be in [1,2^20] and n_out in [1,%d]", MLP_SMALL_MAX_OUT);
  if (!X_packed || !T_packed || !theta_packed || !loss) return fail(MLP_ERR_ARG, "X, T, theta, loss must not be NULL");
  if (!aligned16(items_dev) || !aligned16(X_packed) || !aligned16(T_packed))
    return fail(MLP_ERR_ALIGN, "items, X and T must be 16-byte aligned");
  if (!aligned4(theta_packed) || !aligned4(loss) || (correct && !aligned4(correct)))
    return fail(MLP_ERR_ALIGN, "theta, loss, correct must be 4-byte aligned");
  for (int32_t i = 0; i < n_nets; ++i) {
    const mlp_batch_item &it = items_host[i];
    if (it.n_rows <= 0 || it.n_hidden <= 0 || it.n_hidden > (1 << 20))
      return fail(MLP_ERR_SHAPE, "net %d: n_rows %d / n_hidden %d must be positive (n_hidden <= 2^20)", i,
                  it.n_rows, it.n_hidden);
    if (it.reserved != 0) return fail(MLP_ERR_ARG, "net %d: reserved field must be 0", i);
    if (it.x_off < 0 || it.x_off + it.n_rows > total_rows)
      return fail(MLP_ERR_SHAPE, "net %d: rows [%lld, %lld) outside the %lld packed rows", i,
                  (long long)it.x_off, (long long)(it.x_off + it.n_rows), (long long)total_rows);
    if (it.p_off < 0 || it.p_off + n_params(n_in, it.n_hidden, n_out) > total_params)
      return fail(MLP_ERR_SHAPE, "net %d: parameters outside the %lld packed floats", i, (long long)total_params);
  }
  hipError_t e = mlph::launch_eval_batched(items_dev, n_nets, n_in, n_out, X_packed, T_packed, theta_packed, loss,
                                           correct, (hipStream_t)stream);
  return e == hipSuccess ? MLP_OK : hip_fail(e, "mlp_eval_batched launch");
}

mlp_status mlp_cv_select(const float *loss, const int32_t *group, int32_t n_nets, int32_t n_groups,
                         float *group_mean, int32_t *best, void *stream) {
  if (!loss || !group || !group_mean || !best) return fail(MLP_ERR_ARG, "loss, group, group_mean, best must not be NULL");
  if (n_nets < 1) return fail(MLP_ERR_SHAPE, "n_nets must be positive");
  if (n_groups < 1 || n_groups > 65536) return fail(MLP_ERR_SHAPE, "n_groups must be in [1, 65536]");
  const void *ptrs[] = {loss, group, group_mean, best};
  for (const void *p : ptrs)
    if (!aligned4(p)) return fail(MLP_ERR_ALIGN, "loss, group, group_mean, best must be 4-byte aligned");
  hipError_t e = mlph::launch_cv_select(loss, group, n_nets, n_groups, group_mean, best, (hipStream_t)stream);
  return e == hipSuccess ? MLP_OK : hip_fail(e, "mlp_cv_select launch");
}

mlp_status mlp_shared_workspace_size(const mlp_config *cfg, int32_t n_nets, size_t *bytes) {
  mlp_status s = check_config(cfg);
  if (s != MLP_OK) return s;
  if (!bytes) return fail(MLP_ERR_ARG, "bytes is NULL");
  if (n_nets < 1 || n_nets > MLP_MAX_SHARED_NETS)
    return fail(MLP_ERR_SHAPE, "n_nets %d outside [1,%d]", n_nets, MLP_MAX_SHARED_NETS);
  size_t need = 0;
  s = mlph::large_workspace_bytes(*cfg, n_nets, &need);
  if (s != MLP_OK)
    return fail(s, "no shared-X trainer for this shape (n_in <= 64, n_out <= 4, batch a multiple of 32)");
  *bytes = (need + 255) / 256 * 256;
  return MLP_OK;
}

namespace {
// Argument checks shared by mlp_train_shared and mlp_train_shared_static
// (host only, before any HIP call).
mlp_status check_shared(const mlp_config *cfg, int32_t n_nets, const float *lr, const float *X, const float *T,
                        const float *theta, const float *comp, int32_t epochs, const float *loss_hist,
                        size_t *ws_need) {
  mlp_status s = mlp_shared_workspace_size(cfg, n_nets, ws_need);
  if (s != MLP_OK) return s;
  if (!X || !T || !theta) return fail(MLP_ERR_ARG, "X, T and theta must not be NULL");
  if ((cfg->flags & MLP_F_COMPENSATED) && !comp)
    return fail(MLP_ERR_ARG, "MLP_F_COMPENSATED needs a compensation buffer");
  if (epochs < 0) return fail(MLP_ERR_ARG, "epochs must be >= 0");
  if (cfg->prec == MLP_FP8_E4M3 && n_nets > 1)
    return fail(MLP_ERR_UNSUPPORTED, "e4m3 operands need n_nets == 1 (per-tensor scales)");
  if (cfg->flags & MLP_F_TANH_HIDDEN)
    return fail(MLP_ERR_UNSUPPORTED, "nets sharing X are sigmoid networks");
  if (lr)
    for (int32_t i = 0; i < n_nets; ++i)
      if (!(lr[i] >= 0.0f) || lr[i] > 1e6f) return fail(MLP_ERR_ARG, "net %d: lr must be finite and >= 0", i);
  if (!aligned16(X) || !aligned16(T)) return fail(MLP_ERR_ALIGN, "X and T must be 16-byte aligned");
  if (!aligned4(theta) || (comp && !aligned4(comp)) || (loss_hist && !aligned4(loss_hist)))
    return fail(MLP_ERR_ALIGN, "theta, comp and loss_hist must be 4-byte aligned");
  return MLP_OK;
}

mlp_status device_cus(int *ncu) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  e = hipDeviceGetAttribute(ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
  return MLP_OK;
}
}  // namespace

mlp_status mlp_train_shared(const mlp_config *cfg, int32_t n_nets, const float *lr, const float *X,
                            const float *T, float *theta, float *comp, int32_t epochs, float *loss_hist,
                            void *workspace, size_t ws_bytes, void *stream) {
  size_t need = 0;
  mlp_status s = check_shared(cfg, n_nets, lr, X, T, theta, comp, epochs, loss_hist, &need);
  if (s != MLP_OK) return s;
  if (!workspace || ws_bytes < need)
    return fail(MLP_ERR_WORKSPACE, "workspace of %zu bytes given, %zu needed", workspace ? ws_bytes : 0, need);
  if (!aligned16(workspace)) return fail(MLP_ERR_ALIGN, "workspace must be 16-byte aligned");
  if (epochs == 0) return MLP_OK;
  int ncu = 0;
  if ((s = device_cus(&ncu)) != MLP_OK) return s;
  const int64_t D = cfg->n_in, H = cfg->n_hidden, K = cfg->n_out;
  mlp_params p{theta, theta + D * H, theta + D * H + H, theta + D * H + H + H * K};
  return mlph::large_train(*cfg, n_nets, lr, p, (cfg->flags & MLP_F_COMPENSATED) ? comp : nullptr, workspace,
                           ws_bytes, ncu, X, T, epochs, loss_hist, (hipStream_t)stream, &g_last_error);
}

mlp_status mlp_train_shared_static(const mlp_config *cfg, int32_t n_nets, const float *lr, const float *X,
                                   const float *T, float *theta, float *comp, int32_t epochs, float *loss_hist,
                                   void *stream) {
  size_t need = 0;
  mlp_status s = check_shared(cfg, n_nets, lr, X, T, theta, comp, epochs, loss_hist, &need);
  if (s != MLP_OK) return s;
  if (cfg->flags & MLP_F_CHECK_FINITE)
    return fail(MLP_ERR_UNSUPPORTED, "the finite check reports through a workspace; use mlp_train_shared");
  if (epochs == 0) return MLP_OK;
  int ncu = 0;
  if ((s = device_cus(&ncu)) != MLP_OK) return s;
  const int64_t D = cfg->n_in, H = cfg->n_hidden, K = cfg->n_out;
  mlp_params p{theta, theta + D * H, theta + D * H + H, theta + D * H + H + H * K};
  return mlph::large_train_static(*cfg, n_nets, lr, p, (cfg->flags & MLP_F_COMPENSATED) ? comp : nullptr, ncu, X, T,
                                  epochs, loss_hist, (hipStream_t)stream, &g_last_error);
}

mlp_status mlp_barrier_probe(int32_t n_workgroups, int32_t rounds, void *workspace, size_t ws_bytes,
                             void *stream) {
  if (rounds < 0 || rounds > 1000000) return fail(MLP_ERR_ARG, "rounds must be in 0 .. 1000000");
  if (!workspace || ws_bytes < MLP_BARRIER_PROBE_WS_BYTES || ws_bytes < mlph::barrier_probe_workspace_bytes())
    return fail(MLP_ERR_WORKSPACE, "workspace of %zu bytes given, %d needed", workspace ? ws_bytes : 0,
                MLP_BARRIER_PROBE_WS_BYTES);
  if (!aligned16(workspace)) return fail(MLP_ERR_ALIGN, "workspace must be 16-byte aligned");
  if (n_workgroups < 1) return fail(MLP_ERR_ARG, "n_workgroups must be >= 1");
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
  if (n_workgroups > ncu) return fail(MLP_ERR_ARG, "n_workgroups %d above the %d CUs", n_workgroups, ncu);
  return mlph::barrier_probe(n_workgroups, rounds, workspace, (hipStream_t)stream, &g_last_error);
}

mlp_status mlp_mfma_probe(int32_t prec, const float *A, const float *B, float *C, int32_t M, int32_t N,
                          int32_t Kd, void *stream) {
  if (prec != MLP_FP32 && prec != MLP_BF16 && prec != MLP_FP8_E4M3) return fail(MLP_ERR_ARG, "unknown precision %d", prec);
  if (!A || !B || !C) return fail(MLP_ERR_ARG, "A, B and C must not be NULL");
  if (M <= 0 || N <= 0 || Kd <= 0 || M % 16 || N % 16 || Kd % 32 || M > 4096 || N > 4096 || Kd > (1 << 20))
    return fail(MLP_ERR_SHAPE, "M, N multiples of 16 up to 4096 and Kd a multiple of 32 up to 2^20 required");
  if (!aligned4(A) || !aligned4(B) || !aligned4(C)) return fail(MLP_ERR_ALIGN, "device pointers must be 4-byte aligned");
  hipError_t e = mlph::launch_mfma_probe(prec, A, B, C, M, N, Kd, (hipStream_t)stream);
  return e == hipSuccess ? MLP_OK : hip_fail(e, "mlp_mfma_probe launch");
}

mlp_status mlp_set_wait_limit(int64_t microseconds) {
  mlph::set_wait_limit_us(microseconds);
  return MLP_OK;
}

mlp_status mlp_workspace_status(const void *workspace, size_t ws_bytes, void *stream) {
  if (!workspace) return fail(MLP_ERR_ARG, "workspace is NULL");
  if (ws_bytes < mlph::kStatusBytes)
    return fail(MLP_ERR_WORKSPACE, "a training workspace holds at least %zu bytes", mlph::kStatusBytes);
  if (!aligned16(workspace)) return fail(MLP_ERR_ALIGN, "workspace must be 16-byte aligned");
  const mlp_status s = mlph::read_status(workspace, (hipStream_t)stream, &g_last_error);
  return s;
}

mlp_status mlp_query_status(mlp_net *net, void *stream) {
  if (!net) return fail(MLP_ERR_ARG, "net is NULL");
  return mlp_workspace_status(net->ws, net->ws_bytes, stream);
}

mlp_status mlp_set_momentum(mlp_net *net, float mu, float *velocity) {
  if (!net) return fail(MLP_ERR_ARG, "net is NULL");
  if (!(mu >= 0.0f) || !(mu < 1.0f)) return fail(MLP_ERR_ARG, "mu must be in [0, 1)");
  if (mu > 0.0f && !velocity) return fail(MLP_ERR_ARG, "momentum needs a velocity buffer");
  if (velocity && !aligned4(velocity)) return fail(MLP_ERR_ALIGN, "velocity must be 4-byte aligned");
  net->mu = mu;
  net->velocity = mu > 0.0f ? velocity : nullptr;
  return MLP_OK;
}

mlp_status mlp_dense_forward(const float *X, int64_t n, int32_t d_in, int32_t d_out, const float *W,
                             const float *b, int32_t act, float *Y, void *stream) {
  if (!X || !W || !b || !Y) return fail(MLP_ERR_ARG, "X, W, b and Y must not be NULL");
  if (n <= 0 || d_in <= 0 || d_out <= 0 || d_in > 65536 || d_out > 65536)
    return fail(MLP_ERR_SHAPE, "n >= 1 and d_in, d_out in 1 .. 65536 required");
  if (act != 0 && act != 1) return fail(MLP_ERR_ARG, "act must be 0 (sigmoid) or 1 (tanh)");
  if (!aligned4(X) || !aligned4(W) || !aligned4(b) || !aligned4(Y))
    return fail(MLP_ERR_ALIGN, "device pointers must be 4-byte aligned");
  hipError_t e = mlph::launch_dense_forward(n, d_in, d_out, X, W, b, act, Y, (hipStream_t)stream);
  return e == hipSuccess ? MLP_OK : hip_fail(e, "mlp_dense_forward launch");
}

mlp_status mlp_dense_backward(const float *X, const float *Y, const float *dY, int64_t n, int32_t d_in,
                              int32_t d_out, const float *W, int32_t act, float *gW, float *gb, float *dX,
                              void *workspace, size_t ws_bytes, void *stream) {
  if (!X || !Y || !dY || !W || !gW || !gb) return fail(MLP_ERR_ARG, "X, Y, dY, W, gW and gb must not be NULL");
  if (n <= 0 || d_in <= 0 || d_out <= 0 || d_in > 65536 || d_out > 65536)
    return fail(MLP_ERR_SHAPE, "n >= 1 and d_in, d_out in 1 .. 65536 required");
  if (act != 0 && act != 1) return fail(MLP_ERR_ARG, "act must be 0 (sigmoid) or 1 (tanh)");
  const void *ptrs[] = {X, Y, dY, W, gW, gb, dX, workspace};
  for (const void *p : ptrs)
    if (p && !aligned4(p)) return fail(MLP_ERR_ALIGN, "device pointers must be 4-byte aligned");
  const size_t need = sizeof(float) * (size_t)n * (size_t)d_out;
  if (!workspace || ws_bytes < need)
    return fail(MLP_ERR_WORKSPACE, "workspace of %zu bytes given, %zu needed", workspace ? ws_bytes : 0, need);
  hipError_t e = mlph::launch_dense_backward(n, d_in, d_out, X, Y, dY, W, act, gW, gb, dX,
                                             static_cast<float *>(workspace), (hipStream_t)stream);
  return e == hipSuccess ? MLP_OK : hip_fail(e, "mlp_dense_backward launch");
}

mlp_status mlp_update(float *theta, const float *grad, float *comp, int64_t P, float lr, void *stream) {
  if (!theta || !grad) return fail(MLP_ERR_ARG, "theta and grad must not be NULL");
  if (P <= 0) return fail(MLP_ERR_SHAPE, "P must be positive");
  if (!(lr >= 0.0f) || lr > 1e6f) return fail(MLP_ERR_ARG, "lr must be finite and >= 0");
  if (!aligned4(theta) || !aligned4(grad) || (comp && !aligned4(comp)))
    return fail(MLP_ERR_ALIGN, "device pointers must be 4-byte aligned");
  hipError_t e = mlph::launch_update(P, theta, grad, comp, lr, (hipStream_t)stream);
  return e == hipSuccess ? MLP_OK : hip_fail(e, "mlp_update launch");
}

mlp_status mlp_mse_grad(const float *Y, const float *T, int64_t n, int32_t k, float *dY, float *loss,
                        void *stream) {
  if (!Y || !T || !dY) return fail(MLP_ERR_ARG, "Y, T and dY must not be NULL");
  if (n <= 0 || k <= 0 || n * (int64_t)k > ((int64_t)1 << 26)) return fail(MLP_ERR_SHAPE, "need n, k >= 1, n k <= 2^26");
  if (!aligned4(Y) || !aligned4(T) || !aligned4(dY) || (loss && !aligned4(loss)))
    return fail(MLP_ERR_ALIGN, "device pointers must be 4-byte aligned");
  hipError_t e = mlph::launch_mse_grad(n, k, Y, T, dY, loss, (hipStream_t)stream);
  return e == hipSuccess ? MLP_OK : hip_fail(e, "mlp_mse_grad launch");
}

mlp_status mlp_deep_train(const float *X, const float *T, int64_t n, int32_t n_layers, const int32_t *widths,
                          int32_t act, float *theta, float *comp, float lr, int32_t epochs, float *loss_hist,
                          void *stream) {
  if (!X || !T || !theta || !widths) return fail(MLP_ERR_ARG, "X, T, theta and widths must not be NULL");
  if (n_layers < 1 || n_layers > mlph::kDeepMaxLayers)
    return fail(MLP_ERR_SHAPE, "n_layers must be in 1 .. %d", mlph::kDeepMaxLayers);
  for (int l = 0; l <= n_layers; ++l)
    if (widths[l] < 1 || widths[l] > mlph::kDeepMaxWidth)
      return fail(MLP_ERR_SHAPE, "widths[%d] = %d outside 1 .. %d", l, widths[l], mlph::kDeepMaxWidth);
  if (n <= 0) return fail(MLP_ERR_SHAPE, "n must be positive");
  if (act != 0 && act != 1) return fail(MLP_ERR_ARG, "act must be 0 (sigmoid) or 1 (tanh)");
  if (!(lr >= 0.0f) || lr > 1e6f) return fail(MLP_ERR_ARG, "lr must be finite and >= 0");
  if (epochs < 0) return fail(MLP_ERR_ARG, "epochs must be >= 0");
  const void *ptrs[] = {X, T, theta, comp, loss_hist};
  for (const void *p : ptrs)
    if (p && !aligned4(p)) return fail(MLP_ERR_ALIGN, "device pointers must be 4-byte aligned");
  mlph::DeepPlan plan;
  if (!mlph::deep_plan(n_layers, widths, n, 160 * 1024, &plan))
    return fail(MLP_ERR_UNSUPPORTED, "rows, activations, deltas and parameters of this network do not fit in "
                                     "one workgroup's 160 KiB of LDS");
  if (epochs == 0) return MLP_OK;
  hipError_t e = mlph::launch_deep_train(plan, act, X, T, theta, comp, lr, epochs, loss_hist, (hipStream_t)stream);
  return e == hipSuccess ? MLP_OK : hip_fail(e, "mlp_deep_train launch");
}

}  // extern "C"
