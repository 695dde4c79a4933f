/*
 * FP64 CPU oracle for networks with several hidden layers (the build's
 * extension of section 2.2's one-hidden-layer network to L layers).
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of oracle/.
 *
 * Layer l (l = 0 .. L-1) maps width w[l] to w[l+1] with weights W_l
 * [w[l+1]][w[l]] and biases b_l [w[l+1]]; hidden layers apply the hidden
 * activation act (0 sigma, 1 tanh), the last layer the sigmoid of
 * Equation 1.  The error is the mean squared error over rows and outputs;
 * backpropagation runs the layers in reverse (section 2.2), each layer's
 * delta using the pre-update weights of the layer above; every layer is
 * then updated by theta <- theta - lr g, simultaneously.  Parameters are
 * packed layer after layer, each as W_l then b_l.  Plain float64 loops.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static double sig(double z) { return 1.0 / (1.0 + exp(-z)); }

static int64_t layer_off(const int32_t *w, int l) {
  int64_t o = 0;
  for (int j = 0; j < l; ++j) o += (int64_t)w[j + 1] * w[j] + w[j + 1];
  return o;
}

/* loss at theta and its gradient g (same packing); acts[l] holds layer l's output */
double ora_deep_loss_grad(int64_t n, int L, const int32_t *w, int act, const double *X, const double *T,
                          const double *theta, double *g) {
  double **A = (double **)malloc(sizeof(double *) * (size_t)(L + 1));
  double **Dl = (double **)malloc(sizeof(double *) * (size_t)(L + 1));
  A[0] = (double *)X;
  for (int l = 1; l <= L; ++l) {
    A[l] = (double *)malloc(sizeof(double) * (size_t)(n * w[l]));
    Dl[l] = (double *)malloc(sizeof(double) * (size_t)(n * w[l]));
  }
  /* feed forward, layer by layer */
  for (int l = 0; l < L; ++l) {
    const double *W = theta + layer_off(w, l), *b = W + (int64_t)w[l + 1] * w[l];
    for (int64_t r = 0; r < n; ++r)
      for (int o = 0; o < w[l + 1]; ++o) {
        double z = b[o];
        for (int i = 0; i < w[l]; ++i) z += A[l][r * w[l] + i] * W[(int64_t)o * w[l] + i];
        A[l + 1][r * w[l + 1] + o] = (l == L - 1 || act == 0) ? sig(z) : tanh(z);
      }
  }
  /* error and the last layer's delta */
  const int K = w[L];
  double loss = 0.0;
  for (int64_t r = 0; r < n; ++r)
    for (int o = 0; o < K; ++o) {
      double y = A[L][r * K + o], e = y - T[r * K + o];
      loss += e * e;
      Dl[L][r * K + o] = 2.0 * e / ((double)n * (double)K) * y * (1.0 - y);
    }
  loss /= (double)n * (double)K;
  /* backpropagation through the layers, top down */
  for (int l = L - 1; l >= 0; --l) {
    const double *W = theta + layer_off(w, l);
    double *gW = g + layer_off(w, l), *gb = gW + (int64_t)w[l + 1] * w[l];
    for (int o = 0; o < w[l + 1]; ++o) {
      for (int i = 0; i < w[l]; ++i) {
        double s = 0.0;
        for (int64_t r = 0; r < n; ++r) s += Dl[l + 1][r * w[l + 1] + o] * A[l][r * w[l] + i];
        gW[(int64_t)o * w[l] + i] = s;
      }
      double s = 0.0;
      for (int64_t r = 0; r < n; ++r) s += Dl[l + 1][r * w[l + 1] + o];
      gb[o] = s;
    }
    if (l > 0)   /* delta of the hidden layer below, with this layer's pre-update W */
      for (int64_t r = 0; r < n; ++r)
        for (int i = 0; i < w[l]; ++i) {
          double s = 0.0;
          for (int o = 0; o < w[l + 1]; ++o) s += Dl[l + 1][r * w[l + 1] + o] * W[(int64_t)o * w[l] + i];
          double a = A[l][r * w[l] + i];
          Dl[l][r * w[l] + i] = s * (act == 1 ? 1.0 - a * a : a * (1.0 - a));
        }
  }
  for (int l = 1; l <= L; ++l) {
    free(A[l]);
    free(Dl[l]);
  }
  free(A);
  free(Dl);
  return loss;
}

/* full-batch training for `epochs` epochs; theta updated in place */
void ora_deep_train(int64_t n, int L, const int32_t *w, int act, const double *X, const double *T, double *theta,
                    double lr, int epochs, double *loss_hist) {
  const int64_t P = layer_off(w, L);
  double *g = (double *)malloc(sizeof(double) * (size_t)P);
  for (int e = 0; e < epochs; ++e) {
    double loss = ora_deep_loss_grad(n, L, w, act, X, T, theta, g);
    for (int64_t q = 0; q < P; ++q) theta[q] -= lr * g[q];
    if (loss_hist) loss_hist[e] = loss;
  }
  free(g);
}
