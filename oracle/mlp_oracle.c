/*
 * FP64 CPU oracle for one-hidden-layer sigmoid MLP training by full-batch
 * (or contiguous-minibatch) gradient descent with backpropagation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the ground truth the HIP path is
 * checked against.  Only the tests, the smoke check and the benchmark's CPU
 * baseline load it; the product library never links it and shares no code,
 * header, table or helper with it.
 *
 * What it follows (arxiv 1908.07847):
 *   - section 2.2: a fully connected feed-forward multi-layer perceptron with
 *     one hidden layer; every neuron applies the logistic sigmoid of
 *     Equation 1, sigma(x) = 1/(1+e^-x);
 *   - section 2.2: supervised learning by gradient descent performed through
 *     backpropagation, learning rate 0.1, no momentum;
 *   - section 2.2: after each feed-forward pass the difference between the
 *     outputs and the true values drives the backpropagation step; training
 *     runs for a number of epochs;
 *   - section 2.2: data and weights are flat arrays; the input-to-hidden
 *     weight array holds (hidden neurons x columns) entries, i.e. W1[H][D].
 * Readings where the paper is silent (documented with the build):
 *   - the error is the mean squared error over the batch rows and outputs,
 *     L = sum (Y-T)^2 / (m*K), so dL/dY = 2 (Y-T) / (m*K);
 *   - both layers carry biases; all four gradients come from one forward
 *     pass and are applied simultaneously (the hidden delta uses the
 *     pre-update W2);
 *   - minibatches are contiguous row slices in stored order; a short last
 *     slice uses its own m.
 *
 * Everything is plain float64 loops with no blocking or reordering: the
 * order of operations is the order of the method.  On large inputs the
 * independent outputs of a loop (rows of the forward pass and of delta1,
 * entries of a gradient) are shared among OpenMP threads; each output is
 * still formed by the same loop in the same order, so the result does not
 * depend on the thread count (bit for bit; tested).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Loops with at least this much work are shared among threads (inside
 * ora_train_many, which runs one net per thread, nested regions stay on
 * their thread). */
#define ORA_PAR(work) ((int64_t)(work) >= ((int64_t)1 << 18))

/* Equation 1. exp(-z) overflowing to +inf gives 0, the correct limit. */
static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

/* Feed-forward pass (section 2.2): A = sigma(X W1^T + b1), Y = sigma(A W2^T + b2). */
void ora_forward(int64_t n, int d, int h, int k, const double *X, const double *W1,
                 const double *b1, const double *W2, const double *b2, double *A, double *Y) {
#pragma omp parallel for schedule(static) if (ORA_PAR(n * h * d))
  for (int64_t r = 0; r < n; ++r) {
    for (int j = 0; j < h; ++j) {
      double z = b1[j];
      for (int i = 0; i < d; ++i) z += X[r * d + i] * W1[(int64_t)j * d + i];
      A[r * h + j] = sigmoid(z);
    }
    for (int o = 0; o < k; ++o) {
      double z = b2[o];
      for (int j = 0; j < h; ++j) z += A[r * h + j] * W2[(int64_t)o * h + j];
      Y[r * k + o] = sigmoid(z);
    }
  }
}

/* Mean squared error over rows and outputs (the loss reading of section 2.2). */
double ora_mse(int64_t n, int k, const double *Y, const double *T) {
  double s = 0.0;
  for (int64_t r = 0; r < n; ++r)
    for (int o = 0; o < k; ++o) {
      double e = Y[r * k + o] - T[r * k + o];
      s += e * e;
    }
  return s / ((double)n * (double)k);
}

/*
 * Backpropagation (section 2.2) from an upstream gradient dY = dL/dY.
 *   delta2 = dY . Y(1-Y)                  (output delta; sigma' = sigma(1-sigma))
 *   gW2 = delta2^T A,  gb2 = sum_rows delta2
 *   delta1 = (delta2 W2) . A(1-A)         (hidden delta, pre-update W2)
 *   gW1 = delta1^T X,  gb1 = sum_rows delta1
 *   dX = delta1 W1                        (optional input gradient)
 * Gradients are overwritten.  dX may be NULL.
 */
void ora_backward(int64_t n, int d, int h, int k, const double *X, const double *A,
                  const double *Y, const double *dY, const double *W1, const double *W2,
                  double *gW1, double *gb1, double *gW2, double *gb2, double *dX) {
  double *delta2 = (double *)malloc(sizeof(double) * (size_t)(n * k));
  double *delta1 = (double *)malloc(sizeof(double) * (size_t)(n * h));
  for (int64_t r = 0; r < n; ++r)
    for (int o = 0; o < k; ++o) {
      double y = Y[r * k + o];
      delta2[r * k + o] = dY[r * k + o] * y * (1.0 - y);
    }
#pragma omp parallel for schedule(static) if (ORA_PAR(n * h * k))
  for (int64_t r = 0; r < n; ++r)
    for (int j = 0; j < h; ++j) {
      double s = 0.0;
      for (int o = 0; o < k; ++o) s += delta2[r * k + o] * W2[(int64_t)o * h + j];
      double a = A[r * h + j];
      delta1[r * h + j] = s * a * (1.0 - a);
    }
  for (int o = 0; o < k; ++o) {
#pragma omp parallel for schedule(static) if (ORA_PAR(n * h))
    for (int j = 0; j < h; ++j) {
      double s = 0.0;
      for (int64_t r = 0; r < n; ++r) s += delta2[r * k + o] * A[r * h + j];
      gW2[(int64_t)o * h + j] = s;
    }
    double s = 0.0;
    for (int64_t r = 0; r < n; ++r) s += delta2[r * k + o];
    gb2[o] = s;
  }
#pragma omp parallel for schedule(static) if (ORA_PAR(n * h * d))
  for (int j = 0; j < h; ++j) {
    for (int i = 0; i < d; ++i) {
      double s = 0.0;
      for (int64_t r = 0; r < n; ++r) s += delta1[r * h + j] * X[r * d + i];
      gW1[(int64_t)j * d + i] = s;
    }
    double s = 0.0;
    for (int64_t r = 0; r < n; ++r) s += delta1[r * h + j];
    gb1[j] = s;
  }
  if (dX) {
#pragma omp parallel for schedule(static) if (ORA_PAR(n * h * d))
    for (int64_t r = 0; r < n; ++r)
      for (int i = 0; i < d; ++i) {
        double s = 0.0;
        for (int j = 0; j < h; ++j) s += delta1[r * h + j] * W1[(int64_t)j * d + i];
        dX[r * d + i] = s;
      }
  }
  free(delta2);
  free(delta1);
}

/* Loss and gradient of the MSE reading at the given parameters; returns L. */
double ora_loss_grad(int64_t n, int d, int h, int k, const double *X, const double *T,
                     const double *W1, const double *b1, const double *W2, const double *b2,
                     double *gW1, double *gb1, double *gW2, double *gb2) {
  double *A = (double *)malloc(sizeof(double) * (size_t)(n * h));
  double *Y = (double *)malloc(sizeof(double) * (size_t)(n * k));
  double *dY = (double *)malloc(sizeof(double) * (size_t)(n * k));
  ora_forward(n, d, h, k, X, W1, b1, W2, b2, A, Y);
  double L = ora_mse(n, k, Y, T);
  for (int64_t r = 0; r < n; ++r)
    for (int o = 0; o < k; ++o)
      dY[r * k + o] = 2.0 * (Y[r * k + o] - T[r * k + o]) / ((double)n * (double)k);
  ora_backward(n, d, h, k, X, A, Y, dY, W1, W2, gW1, gb1, gW2, gb2, NULL);
  free(A);
  free(Y);
  free(dY);
  return L;
}

/*
 * Training loop (section 2.2): for every epoch, for every contiguous
 * minibatch (batch <= 0 or batch >= n means full batch): feed forward,
 * error, backpropagation, then theta <- theta - lr * g (no momentum).
 * loss_hist[e] (may be NULL) is the mean over the epoch's minibatches of the
 * minibatch loss at the pre-update parameters.  Parameters are updated in
 * place.
 */
void ora_train(int64_t n, int d, int h, int k, int64_t batch, const double *X, const double *T,
               double *W1, double *b1, double *W2, double *b2, double lr, int epochs,
               double *loss_hist) {
  if (batch <= 0 || batch > n) batch = n;
  int64_t steps = (n + batch - 1) / batch;
  double *gW1 = (double *)malloc(sizeof(double) * (size_t)h * d);
  double *gb1 = (double *)malloc(sizeof(double) * (size_t)h);
  double *gW2 = (double *)malloc(sizeof(double) * (size_t)k * h);
  double *gb2 = (double *)malloc(sizeof(double) * (size_t)k);
  for (int e = 0; e < epochs; ++e) {
    double acc = 0.0;
    for (int64_t s = 0; s < steps; ++s) {
      int64_t r0 = s * batch;
      int64_t m = (r0 + batch <= n) ? batch : n - r0;
      acc += ora_loss_grad(m, d, h, k, X + r0 * d, T + r0 * k, W1, b1, W2, b2, gW1, gb1, gW2,
                           gb2);
      for (int64_t q = 0; q < (int64_t)h * d; ++q) W1[q] -= lr * gW1[q];
      for (int j = 0; j < h; ++j) b1[j] -= lr * gb1[j];
      for (int64_t q = 0; q < (int64_t)k * h; ++q) W2[q] -= lr * gW2[q];
      for (int o = 0; o < k; ++o) b2[o] -= lr * gb2[o];
    }
    if (loss_hist) loss_hist[e] = acc / (double)steps;
  }
  free(gW1);
  free(gb1);
  free(gW2);
  free(gb2);
}

/*
 * Many independent networks (one per row of the item tables), each trained
 * full batch on its own rows for the same number of epochs.  Packed layout:
 * net i's rows start at row x_off[i] of X and T; its parameters are
 * [W1 | b1 | W2 | b2] starting at float p_off[i] of theta.  loss_hist (may be
 * NULL) is [n_nets][epochs].  Nets share nothing, so they may be run on
 * several threads (threads <= 0: the OpenMP default).
 */
void ora_train_many(int n_nets, const int32_t *n_rows, const int32_t *n_hidden, const double *lr,
                    const int64_t *x_off, const int64_t *p_off, int d, int k, const double *X,
                    const double *T, double *theta, int epochs, double *loss_hist, int threads) {
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int i = 0; i < n_nets; ++i) {
    int h = n_hidden[i];
    double *W1 = theta + p_off[i];
    double *b1 = W1 + (int64_t)h * d;
    double *W2 = b1 + h;
    double *b2 = W2 + (int64_t)k * h;
    ora_train(n_rows[i], d, h, k, 0, X + x_off[i] * d, T + x_off[i] * k, W1, b1, W2, b2, lr[i],
              epochs, loss_hist ? loss_hist + (int64_t)i * epochs : NULL);
  }
}

int ora_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads for the shared loops of later calls (<= 0: the OpenMP default). */
void ora_set_threads(int threads) {
#ifdef _OPENMP
  omp_set_num_threads(threads > 0 ? threads : omp_get_num_procs());
#else
  (void)threads;
#endif
}
