/*
 * mlp.h -- C ABI of libmlp: one-hidden-layer sigmoid MLP training on gfx950.
 *
 * The method (arxiv 1908.07847, section 2.2): a fully connected feed-forward
 * network with one hidden layer, the logistic sigmoid of Equation 1 at both
 * layers, trained by gradient descent through backpropagation with a fixed
 * learning rate and no momentum.  Data and weights are flat float arrays;
 * the input-to-hidden weights hold (hidden neurons x columns) entries.
 *
 *   forward:   A = sigma(X W1^T + b1),  Y = sigma(A W2^T + b2)
 *   error:     L = sum (Y - T)^2 / (m K)     (mean over rows and outputs)
 *   backward:  delta2 = dL/dY . Y(1-Y);  delta1 = (delta2 W2) . A(1-A)
 *              gW2 = delta2^T A, gb2 = sum delta2, gW1 = delta1^T X,
 *              gb1 = sum delta1  (delta1 uses the pre-update W2)
 *   update:    theta <- theta - lr * g   (all four at once)
 *
 * Conventions for every function:
 *   - Arrays are float32, row-major: X[n][D], T[n][K], A[n][H], Y[n][K],
 *     W1[H][D], b1[H], W2[K][H], b2[K].  "Packed" parameters are
 *     [W1 | b1 | W2 | b2] back to back (P = D*H + H + H*K + K floats).
 *   - Every array argument is a DEVICE pointer unless marked "host".  The
 *     caller allocates every device buffer (inputs, outputs, parameters,
 *     compensation, workspace) and keeps it alive until the stream has run
 *     the work; the library never allocates or frees device memory.
 *   - `stream` is a hipStream_t passed as void* (NULL: the null stream).
 *     All device work is enqueued on it and is asynchronous: execution
 *     errors surface at the caller's next synchronisation.
 *   - Every function returns an mlp_status and never aborts.  Argument,
 *     shape and alignment checks happen before any HIP call, so a rejected
 *     call leaves no work on the stream.  mlp_last_error() gives a
 *     thread-local message for the last failure.
 *   - Device pointers must be 4-byte aligned; X, T, the workspace and the
 *     batched item table must be 16-byte aligned.
 *   - NaN/Inf in inputs propagate; nothing checks for them on the hot path
 *     unless the configuration sets MLP_F_CHECK_FINITE.
 *   - Errors that only the device can see (a grid-wide wait of the
 *     minibatch trainer that gave up, the finite check) are written to a
 *     status block at the head of the training workspace; mlp_query_status
 *     and mlp_workspace_status synchronise the stream and report them.
 *
 * Beyond the method, the library offers the build's own extensions, each
 * marked where it is declared: reduced-precision operands for the two large
 * contractions, many networks in one launch (independent rows, or one shared
 * X), class predictions and a held-out read-out, a tanh hidden activation
 * and momentum, one dense layer for networks with several hidden layers,
 * and a grid-barrier probe for measurement.
 */
#ifndef MLP_H_
#define MLP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MLP_OK = 0,
  MLP_ERR_ARG = 1,         /* NULL pointer, non-positive size, bad flag */
  MLP_ERR_SHAPE = 2,       /* sizes outside what the kernels support */
  MLP_ERR_ALIGN = 3,       /* device pointer not 16-byte aligned */
  MLP_ERR_WORKSPACE = 4,   /* workspace missing or too small */
  MLP_ERR_UNSUPPORTED = 5, /* valid request no kernel here implements */
  MLP_ERR_HIP = 6,         /* the HIP runtime reported an error */
  MLP_ERR_TIMEOUT = 7,     /* a grid-wide wait of the last training launch
                            * gave up (see mlp_set_wait_limit): parameters
                            * and losses of that launch are not valid */
  MLP_ERR_NONFINITE = 8    /* MLP_F_CHECK_FINITE found a NaN or infinity */
} mlp_status;

/* Operand precision of the two large contractions (X W1^T and delta1^T X).
 * Master parameters, biases, sigmoid, the output layer, the loss and the
 * update are float32 in every precision.  Reduced precisions are the
 * build's own extension (the paper trains in float). */
typedef enum { MLP_FP32 = 0, MLP_BF16 = 1, MLP_FP8_E4M3 = 2 } mlp_precision;

/* Flags. */
enum {
  /* Compensated (Kahan) float32 parameter update, using the caller's
   * compensation buffer.  Same update, computed more exactly. */
  MLP_F_COMPENSATED = 1u,
  /* Accepted for interface completeness: every kernel here reduces in a
   * fixed order, so results are bitwise repeatable with or without it. */
  MLP_F_DETERMINISTIC = 2u,
  /* After each mlp_train / mlp_train_shared launch, scan the trained
   * parameters (and loss_hist, when given) for NaN or infinity; a hit is
   * reported as MLP_ERR_NONFINITE by mlp_query_status /
   * mlp_workspace_status.  One extra pass over the parameters; off the
   * training loop. */
  MLP_F_CHECK_FINITE = 4u,
  /* Hidden neurons apply tanh (derivative 1 - tanh^2) instead of the
   * sigmoid of Equation 1; the output neurons stay sigmoid.  A variant of
   * section 2.2's network (the paper's neurons are all sigmoid), honoured by
   * mlp_forward, mlp_backward, mlp_predict and the full-batch small trainer
   * of mlp_train; the minibatch / large-shape trainer and mlp_train_shared
   * return MLP_ERR_UNSUPPORTED for it. */
  MLP_F_TANH_HIDDEN = 8u
};

typedef struct {
  int32_t n_in;     /* D, features per row                         */
  int32_t n_hidden; /* H, hidden neurons                           */
  int32_t n_out;    /* K, output neurons                           */
  int32_t prec;     /* mlp_precision                               */
  int64_t n_rows;   /* N, rows of the training set                 */
  int64_t batch;    /* rows per gradient step; 0 or >= N: full batch */
  float lr;         /* learning rate (section 2.2 uses 0.1)        */
  uint32_t flags;   /* MLP_F_*                                     */
} mlp_config;

typedef struct {
  float *W1, *b1, *W2, *b2; /* device, W1[H][D] b1[H] W2[K][H] b2[K] */
} mlp_params;

typedef struct mlp_net mlp_net; /* opaque host handle; owns no device memory */

/* Bytes of device workspace that mlp_init must be given for this
 * configuration (host out).  Pure host computation. */
mlp_status mlp_workspace_size(const mlp_config *cfg /*host*/, size_t *bytes /*host out*/);

/* Create a handle bound to caller-owned parameters (updated in place by
 * mlp_step / mlp_train), an optional compensation buffer comp[P] (packed
 * order; required when MLP_F_COMPENSATED is set; zero it before the first
 * training call) and a workspace of at least mlp_workspace_size bytes.
 * Queries the current device once.  One handle per stream; not
 * thread-safe. */
mlp_status mlp_init(mlp_net **out /*host out*/, const mlp_config *cfg /*host*/, mlp_params theta,
                    float *comp, void *workspace, size_t ws_bytes);

/* Release the handle (host memory only). */
mlp_status mlp_destroy(mlp_net *net);

/* Heavy-ball momentum for the handle's updates (a variant: section 2.2
 * trains without momentum, which is mu = 0, the default):
 *   v <- mu v + g,  theta <- theta - lr v   (compensated like the plain step)
 * for every parameter, simultaneously.  velocity [P] (device, packed order
 * W1 | b1 | W2 | b2, 4-byte aligned, caller-owned; zero it before the first
 * update) carries v across calls, so training a then b epochs equals a+b.
 * Applies to mlp_step and to the full-batch small trainer of mlp_train; the
 * minibatch / large-shape trainer returns MLP_ERR_UNSUPPORTED while it is
 * set.  mu in [0, 1); mu > 0 needs velocity; mu = 0 turns momentum off. */
mlp_status mlp_set_momentum(mlp_net *net, float mu, float *velocity);

/* Feed-forward pass over n rows (section 2.2, Equation 1):
 * A[n][H] (may be NULL) and Y[n][K] are overwritten.  Any n >= 1. */
mlp_status mlp_forward(mlp_net *net, const float *X, int64_t n, float *A, float *Y, void *stream);

/* Backpropagation over n rows, from the A and Y of mlp_forward at the
 * current parameters.  dY[n][K] is the upstream gradient dL/dY; when dY is
 * NULL the mean-squared-error reading is used against T[n][K]
 * (dL/dY = 2 (Y - T) / (n K)) and, if loss is non-NULL, loss[0] receives
 * L.  grads (device, same shapes as the parameters) are overwritten with
 * the parameter gradients; dX[n][D] (may be NULL) receives delta1 W1.
 * Row sums are reduced in a fixed order: repeated calls are bitwise equal. */
mlp_status mlp_backward(mlp_net *net, const float *X, const float *A, const float *Y,
                        const float *dY, const float *T, int64_t n, mlp_params grads, float *dX,
                        float *loss, void *stream);

/* theta <- theta - lr * grads (section 2.2: fixed rate, no momentum),
 * compensated when the handle was created with MLP_F_COMPENSATED. */
mlp_status mlp_step(mlp_net *net, mlp_params grads, float lr, void *stream);

/* Train for `epochs` epochs on X[N][D], T[N][K]: per epoch, ceil(N/batch)
 * contiguous minibatches in stored order, each a forward pass, the MSE
 * error, backpropagation and an update.  loss_hist[epochs] (may be NULL)
 * receives, per epoch, the mean over its minibatches of the minibatch loss
 * at the pre-update parameters.  With the compensation buffer, training a
 * then b epochs is bitwise equal to training a+b epochs. */
mlp_status mlp_train(mlp_net *net, const float *X, const float *T, int32_t epochs,
                     float *loss_hist, void *stream);

/* Status of the last mlp_train launch on this handle's workspace: waits for
 * the stream, then returns MLP_ERR_TIMEOUT if a grid-wide wait of the
 * minibatch / large-shape trainer gave up (the launch then ended early in
 * every workgroup; loss_hist entries from the failing epoch on are NaN and
 * the parameters may hold a partial update), MLP_ERR_NONFINITE if the
 * finite check (MLP_F_CHECK_FINITE) found a NaN or infinity, else MLP_OK.
 * Valid until the next training launch on the same workspace. */
mlp_status mlp_query_status(mlp_net *net, void *stream);

/* The same for a caller-held training workspace (mlp_train_shared, or a
 * handle's workspace): waits for the stream and reads the status block at
 * the workspace's head.  ws_bytes >= 2048, workspace 16-byte aligned. */
mlp_status mlp_workspace_status(const void *workspace, size_t ws_bytes, void *stream);

/* Longest time one grid-wide wait of the minibatch / large-shape trainer
 * (and of mlp_barrier_probe) may take before it gives up, in microseconds
 * of the device's constant-rate wall clock; process-wide, read at launch.
 * Negative: the default, 5 s.  0: a wait that is not already satisfied
 * gives up at once (for testing the failure path).  A launch whose wait
 * gives up ends early in every workgroup -- nothing hangs -- and reports
 * MLP_ERR_TIMEOUT through mlp_query_status / mlp_workspace_status. */
mlp_status mlp_set_wait_limit(int64_t microseconds);

/* Class predictions: the network outputs Y = sigma(sigma(X W1^T + b1) W2^T
 * + b2) of section 2.2 read as a class, the index of the largest output
 * (the lowest index on ties), as in the paper's evaluation of the trained
 * network; with one output (K = 1, the two-class good/poor-control
 * reading) class 1 when the output is above 1/2, else 0.  X [n][D]; Y [n][K]
 * (out, the outputs themselves); labels [n] (out, int32).  With targets
 * T [n][K] (one-hot, or 0/1 for K = 1; may be NULL), correct [1] (out,
 * int32, device) receives the number of rows whose class equals the
 * target's (same rule applied to T); correct must be non-NULL iff T is.
 * Uses the parameters bound to net; X 16-byte aligned, the rest 4. */
mlp_status mlp_predict(mlp_net *net, const float *X, int64_t n, float *Y, int32_t *labels,
                       const float *T, int32_t *correct, void *stream);

/* ---- many independent small networks in one launch ---------------------- */

typedef struct {
  int32_t n_rows;   /* N_i: rows of net i (full batch)                     */
  int32_t n_hidden; /* H_i                                                  */
  float lr;         /* lr_i                                                 */
  int32_t reserved; /* must be 0                                            */
  int64_t x_off;    /* first row of net i in X_packed and T_packed          */
  int64_t p_off;    /* first float of net i's [W1|b1|W2|b2] in theta_packed */
} mlp_batch_item;   /* 32 bytes */

/* Limits of the batched (and small full-batch) trainer. */
#define MLP_SMALL_MAX_ROWS 128
#define MLP_SMALL_MAX_HIDDEN 64
#define MLP_SMALL_MAX_IN 48
#define MLP_SMALL_MAX_OUT 4

/* Train n_nets independent networks, each full batch on its own rows, for
 * `epochs` epochs, in one kernel launch (capturable in a hipGraph).  The
 * item table is given twice with identical contents: items_host (host) is
 * validated and drives the launch, items_dev (device) is read by the
 * kernel.  Nets are started in table order, so listing them by decreasing
 * N_i*H_i gives a longest-first schedule.  theta_packed and comp_packed
 * (may be NULL: plain update) are updated in place; loss_hist
 * [n_nets][epochs] (may be NULL) is indexed by table position.  Every net's
 * result is independent of the others and of the table order. */
mlp_status mlp_train_batched(const mlp_batch_item *items_host, const mlp_batch_item *items_dev,
                             int32_t n_nets, int32_t n_in, int32_t n_out, const float *X_packed,
                             const float *T_packed, int64_t total_rows, float *theta_packed,
                             float *comp_packed, int64_t total_params, int32_t epochs,
                             float *loss_hist, void *stream);

/* Evaluate n_nets networks, each on its own rows of X_packed / T_packed (for
 * instance the held-out fold of a cross-validation split), in one launch:
 * loss[i] = sum (Y - T)^2 / (N_i K) of net i's forward pass (section 2.2)
 * and, if correct is not NULL, correct[i] (int32) = rows whose class (index
 * of the largest output, lowest on ties) equals the target's.  The item
 * table is the batched trainer's (n_rows, n_hidden, x_off, p_off of each
 * net; lr is ignored), given on the host (validated) and on the device
 * (read by the kernel); n_hidden and n_rows may exceed the trainer's
 * limits, n_out <= MLP_SMALL_MAX_OUT.  Sums over rows use a fixed order. */
mlp_status mlp_eval_batched(const mlp_batch_item *items_host, const mlp_batch_item *items_dev, int32_t n_nets,
                            int32_t n_in, int32_t n_out, const float *X_packed, const float *T_packed,
                            int64_t total_rows, const float *theta_packed, int64_t total_params, float *loss,
                            int32_t *correct, void *stream);

/* Cross-validation model selection over the nets of a batched run (the
 * under/overfitting question of section 1 answered on a hidden-size grid),
 * on the device: group_mean[g] = the mean of loss[i] over the nets i with
 * group[i] == g, summed in increasing i in float32 (+inf for a group with no
 * net or a non-finite mean), and best[0] = the group with the lowest mean,
 * the lowest index on ties (0 when every mean is +inf).  loss [n_nets] (for
 * instance mlp_eval_batched's held-out losses), group [n_nets] (int32),
 * group_mean [n_groups] and best [1] are device pointers, 4-byte aligned;
 * 1 <= n_nets, 1 <= n_groups <= 65536.  A net whose group index lies outside
 * [0, n_groups) belongs to no group (the kernel cannot report it).  One
 * launch on the stream, no allocation. */
mlp_status mlp_cv_select(const float *loss, const int32_t *group, int32_t n_nets, int32_t n_groups,
                         float *group_mean, int32_t *best, void *stream);

/* ---- networks sharing one dataset --------------------------------------- */

#define MLP_MAX_SHARED_NETS 64

/* Workspace bytes for mlp_train_shared with n_nets nets of shape cfg. */
mlp_status mlp_shared_workspace_size(const mlp_config *cfg /*host*/, int32_t n_nets, size_t *bytes /*host out*/);

/* Train n_nets independent networks of the shape in cfg on the same X[N][D]
 * and T[N][K], in one kernel launch: the training loop of section 2.2 (the
 * same minibatches, loss and update as mlp_train) for every net, with its
 * own initial parameters and learning rate -- a grid over learning rates and
 * initialisations evaluated on one dataset.  The nets exchange nothing; the
 * launch shares the staging of X's row blocks between them.
 *   cfg        shape, minibatch, operand precision and flags of every net;
 *              n_in <= 64, n_out <= 4, batch a multiple of 32; FP8_E4M3
 *              needs n_nets == 1 (its scales are per tensor)
 *   n_nets     1 .. MLP_MAX_SHARED_NETS
 *   lr         host [n_nets] learning rates, or NULL for cfg->lr for all
 *   theta      [n_nets][P] packed parameters, updated in place
 *   comp       [n_nets][P] compensation terms (needed iff MLP_F_COMPENSATED)
 *   loss_hist  [n_nets][epochs] per-epoch losses as in mlp_train, or NULL
 *   workspace  >= mlp_shared_workspace_size bytes, 16-byte aligned; its
 *              contents on entry do not matter; its head holds the
 *              launch's status block (mlp_workspace_status)
 * Results of net i equal mlp_train of net i alone up to float summation
 * order; for a fixed device and n_nets they are bitwise repeatable. */
mlp_status mlp_train_shared(const mlp_config *cfg /*host*/, int32_t n_nets, const float *lr /*host*/,
                            const float *X, const float *T, float *theta, float *comp, int32_t epochs,
                            float *loss_hist, void *workspace, size_t ws_bytes, void *stream);

/* Allocation-free form of mlp_train_shared, for callers that cannot
 * allocate device memory or pass a workspace (code under HIP-graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * semantics and results (bitwise equal to mlp_train_shared on the same
 * device and shape) except that the scratch the kernels need lives in a
 * fixed device array inside the library: 32 MiB (MLP_STATIC_SCRATCH_BYTES),
 * one copy per GPU the library runs on, held until the process ends.  The
 * call allocates nothing, looks the array's address up on its first call on
 * a device, and rejects with MLP_ERR_WORKSPACE a shape whose grid needs more
 * scratch than that (e.g. the 64-1024-3 net fits; 64 such nets sharing X do
 * not -- use mlp_train_shared).  Every call on one GPU shares its array:
 * calls that overlap on that GPU (different streams, threads or processes
 * without ordering) race and must not be made.  The status block is not
 * reachable by the caller: a grid-barrier wait that gave up shows as NaN in
 * loss_hist, and MLP_F_CHECK_FINITE is rejected (MLP_ERR_UNSUPPORTED). */
#define MLP_STATIC_SCRATCH_BYTES (32u << 20)
mlp_status mlp_train_shared_static(const mlp_config *cfg /*host*/, int32_t n_nets, const float *lr /*host*/,
                                   const float *X, const float *T, float *theta, float *comp, int32_t epochs,
                                   float *loss_hist, void *stream);

/* ---- networks with several hidden layers ----------------------------------- */

/* One fully connected layer of a deeper network (section 2.2's layer,
 * stacked; the paper's network has one hidden layer):
 *   Y = act(X W^T + b),  X [n][d_in], W [d_out][d_in], b [d_out], Y [n][d_out]
 * act 0: the sigmoid of Equation 1; 1: tanh.  n >= 1; d_in, d_out in
 * 1 .. 65536.  Device pointers, 4-byte aligned. */
mlp_status mlp_dense_forward(const float *X, int64_t n, int32_t d_in, int32_t d_out, const float *W,
                             const float *b, int32_t act, float *Y, void *stream);

/* Adjoint of mlp_dense_forward from dY = dL/dY [n][d_out] and the layer's
 * own output Y:  dZ = dY . act'(Y),  gW = dZ^T X,  gb = sum over rows of dZ,
 * dX = dZ W (dX may be NULL).  gW [d_out][d_in], gb [d_out] are
 * overwritten; row sums run in a fixed order (bitwise repeatable).
 * workspace: >= n * d_out * 4 bytes (dZ), 4-byte aligned. */
mlp_status mlp_dense_backward(const float *X, const float *Y, const float *dY, int64_t n, int32_t d_in,
                              int32_t d_out, const float *W, int32_t act, float *gW, float *gb, float *dX,
                              void *workspace, size_t ws_bytes, void *stream);

/* theta <- theta - lr g over P packed parameters (any network), Kahan-
 * compensated with comp [P] when comp is not NULL. */
mlp_status mlp_update(float *theta, const float *grad, float *comp, int64_t P, float lr, void *stream);

/* The error of section 2.2 as the mean squared error of outputs Y [n][K]
 * against targets T [n][K]: loss[0] = sum (Y-T)^2 / (n K) (loss may be NULL)
 * and dY = dL/dY = 2 (Y-T) / (n K) [n][K].  One workgroup, fixed summation
 * order; n K <= 2^26. */
mlp_status mlp_mse_grad(const float *Y, const float *T, int64_t n, int32_t k, float *dY, float *loss,
                        void *stream);

/* Full-batch training of a network with several hidden layers in one launch:
 * section 2.2's loop (feed forward layer by layer, the mean squared error,
 * backpropagation from the top layer down using each layer's pre-update
 * weights, then theta <- theta - lr g for every layer at once), `epochs`
 * times, one workgroup holding the rows, activations, deltas and
 * parameters in LDS.  The same epochs as DeepNet's per-layer calls
 * (mlp_dense_forward, mlp_mse_grad, mlp_dense_backward, mlp_update) up to
 * float summation order.
 *   X          [n][widths[0]] rows, T [n][widths[n_layers]] targets
 *   n_layers   weight layers, 1 .. 8; widths (host) [n_layers + 1], each
 *              1 .. 1024
 *   act        hidden layers' activation, 0: the sigmoid of Equation 1,
 *              1: tanh; the top layer applies the sigmoid
 *   theta      [P] parameters packed layer after layer, each as W_l
 *              [widths[l+1]][widths[l]] then b_l [widths[l+1]]; updated
 *              in place
 *   comp       [P] Kahan compensation terms (updated in place), or NULL for
 *              the plain update
 *   loss_hist  [epochs] the error at each epoch's pre-update parameters, or
 *              NULL
 * Device pointers, 4-byte aligned.  MLP_ERR_UNSUPPORTED when n rows of
 * every layer's activations, two delta arrays and 2 + RS copies of the P
 * parameters (RS >= 1 row segments of the gradient sums) exceed 160 KiB.
 * Bitwise repeatable.  Asynchronous on the stream; argument errors return
 * before any launch; epochs = 0 launches nothing. */
mlp_status mlp_deep_train(const float *X, const float *T, int64_t n, int32_t n_layers,
                          const int32_t *widths /*host*/, int32_t act, float *theta, float *comp, float lr,
                          int32_t epochs, float *loss_hist, void *stream);

/* ---- measurement ---------------------------------------------------------- */

/* Bytes of workspace mlp_barrier_probe needs. */
#define MLP_BARRIER_PROBE_WS_BYTES 2048

/* Grid-barrier latency probe for the sync-adjusted bound of the large-N
 * trainer: one cooperative launch of n_workgroups workgroups (256 threads
 * each, at most one per CU on the device) that pass `rounds` grid barriers
 * of the kind the large-N trainer passes three times per minibatch step
 * (section 2.2's loop: forward, backpropagation, update), and do nothing
 * else.  Timing two launches with different round counts on the stream
 * gives the time one barrier adds.
 *   n_workgroups  1 .. the device's CU count
 *   rounds        0 .. 1,000,000
 *   workspace     >= MLP_BARRIER_PROBE_WS_BYTES device bytes, 16-byte
 *                 aligned; overwritten (barrier counters).  A barrier wait
 *                 that does not complete within the wait limit
 *                 (mlp_set_wait_limit) sets the 32-bit word at index 16 to
 *                 nonzero and ends the launch instead of hanging;
 *                 mlp_workspace_status reports it.
 * Asynchronous on the stream; argument errors return before any launch. */
mlp_status mlp_barrier_probe(int32_t n_workgroups, int32_t rounds, void *workspace, size_t ws_bytes,
                             void *stream);

/* Accuracy probe of the matrix-core contraction the minibatch trainer runs
 * for its two large products (measurement, no part of training):
 *   C[M][N] = sum over k < Kd of A[M][Kd] B[N][Kd]
 * on the instruction the trainer uses for operand precision prec (float32:
 * 16x16x4 steps; bf16 and e4m3: 16x16x32 steps), with its operand layout and
 * its chained float32 accumulation over k.  A and B hold float32 values that
 * the kernel converts to the format (round to nearest even; e4m3 saturates
 * at +-448, no scale); values already representable convert exactly, so C
 * then differs from the exact sum only by the matrix core's own summation.
 * M, N multiples of 16 (<= 4096), Kd a multiple of 32 (<= 2^20); device
 * pointers, 4-byte aligned, row-major; C is overwritten. */
mlp_status mlp_mfma_probe(int32_t prec, const float *A, const float *B, float *C, int32_t M, int32_t N,
                          int32_t Kd, void *stream);

/* ---- launch-shape hints -------------------------------------------------- */

/* Overrides of launch shapes that do not change results beyond summation
 * order (0 = the library's own choice).  Process-wide; set it before the
 * calls it should affect, not concurrently with them.  It exists for an
 * autotuner that times candidate shapes and remembers the fastest:
 *   small_threads        threads per net in the small / batched trainer:
 *                        128, 256 or 512, the waves splitting the rows
 *                        (fewer are used when the larger count's LDS plan
 *                        would not fit), or 64: one wave per 16 hidden
 *                        units of the widest net, the waves splitting the
 *                        hidden layer (sigmoid without momentum; the
 *                        variants then run on 128 threads);
 *   large_row_blocks,    the Gi x Gj grid of the large-N trainer (row blocks
 *   large_hidden_blocks  of >= 32 rows, hidden blocks of <= 256 units);
 *   large_waves          waves per workgroup of the large-N trainer, 4 or 8
 *                        (0: 8 for hidden blocks of at least 128 units,
 *                        else 4). */
typedef struct {
  int32_t small_threads;
  int32_t large_row_blocks;
  int32_t large_hidden_blocks;
  int32_t large_waves;
} mlp_launch_hint;

mlp_status mlp_set_launch_hint(const mlp_launch_hint *hint /*host; NULL resets*/);

/* The launch shape the large-N trainer (minibatch shapes outside the small
 * trainer, and mlp_train_shared) picks for n_nets nets of shape *cfg on a
 * device with n_cu compute units, under the current launch hint: shape[0]
 * the row blocks Gi, shape[1] the hidden blocks Gj (the grid has Gi x n_nets
 * x Gj workgroups, one per CU), shape[2] the waves per workgroup (4 or 8),
 * shape[3] the rows of a block staged in LDS at a time, shape[4] the hidden
 * tiles of 16 units a wave owns at most (the kernel instance: 1 when a
 * 4-wave block has at most one tile per wave, else 16 / waves).  The default grid
 * gives one net row blocks of at least 64 rows (32 for nets sharing X) and
 * hidden blocks of 64..256 units, filling the CUs.  Host-only arithmetic (no
 * device call): *cfg and shape are host pointers.  MLP_ERR_ARG for a NULL
 * pointer, n_cu < 1 or n_nets outside 1..64; MLP_ERR_UNSUPPORTED when no
 * grid covers the shape (mlp_last_error says why). */
mlp_status mlp_large_plan(const mlp_config *cfg, int32_t n_nets, int32_t n_cu, int32_t shape[5]);

const char *mlp_status_string(mlp_status s);
const char *mlp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MLP_H_ */
