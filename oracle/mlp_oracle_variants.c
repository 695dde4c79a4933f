/*
 * FP64 CPU oracle for two variants of the training method: a tanh hidden
 * activation and gradient descent with momentum.
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of oracle/: the product library
 * never links it and shares nothing with it.
 *
 * The method is the one of section 2.2 (one hidden layer, sigmoid output
 * neurons of Equation 1, mean squared error, backpropagation, simultaneous
 * update of all four parameter arrays, contiguous minibatches).  Section 2.2
 * fixes the sigmoid for every neuron and trains without momentum; these two
 * variants are the build's own extensions, named as such:
 *   act = 0: hidden activation sigma (the paper's network);
 *   act = 1: hidden activation tanh, derivative 1 - tanh^2;
 *   mu  = 0: plain gradient descent theta <- theta - lr g (the paper);
 *   mu  > 0: heavy-ball momentum, v <- mu v + g, theta <- theta - lr v, with
 *            the velocity v (packed like the parameters: W1 | b1 | W2 | b2)
 *            carried across steps and calls.
 * Plain float64 loops in the order of the method.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

static double act_fn(int act, double z) { return act == 1 ? tanh(z) : sigmoid(z); }

/* derivative of the hidden activation from its value a */
static double act_slope(int act, double a) { return act == 1 ? 1.0 - a * a : a * (1.0 - a); }

/* One minibatch: loss at the given parameters and the four gradients. */
static double loss_grad_var(int64_t n, int d, int h, int k, int act, const double *X, const double *T,
                            const double *W1, const double *b1, const double *W2, const double *b2,
                            double *gW1, double *gb1, double *gW2, double *gb2) {
  double *A = (double *)malloc(sizeof(double) * (size_t)(n * h));
  double *Y = (double *)malloc(sizeof(double) * (size_t)(n * k));
  double *delta2 = (double *)malloc(sizeof(double) * (size_t)(n * k));
  double *delta1 = (double *)malloc(sizeof(double) * (size_t)(n * h));
  /* feed forward */
  for (int64_t r = 0; r < n; ++r) {
    for (int j = 0; j < h; ++j) {
      double z = b1[j];
      for (int i = 0; i < d; ++i) z += X[r * d + i] * W1[(int64_t)j * d + i];
      A[r * h + j] = act_fn(act, z);
    }
    for (int o = 0; o < k; ++o) {
      double z = b2[o];
      for (int j = 0; j < h; ++j) z += A[r * h + j] * W2[(int64_t)o * h + j];
      Y[r * k + o] = sigmoid(z);
    }
  }
  /* error and output delta */
  double L = 0.0;
  for (int64_t r = 0; r < n; ++r)
    for (int o = 0; o < k; ++o) {
      double e = Y[r * k + o] - T[r * k + o];
      L += e * e;
      double y = Y[r * k + o];
      delta2[r * k + o] = 2.0 * e / ((double)n * (double)k) * y * (1.0 - y);
    }
  L /= (double)n * (double)k;
  /* hidden delta with the pre-update W2 */
  for (int64_t r = 0; r < n; ++r)
    for (int j = 0; j < h; ++j) {
      double s = 0.0;
      for (int o = 0; o < k; ++o) s += delta2[r * k + o] * W2[(int64_t)o * h + j];
      delta1[r * h + j] = s * act_slope(act, A[r * h + j]);
    }
  /* gradients */
  for (int o = 0; o < k; ++o) {
    for (int j = 0; j < h; ++j) {
      double s = 0.0;
      for (int64_t r = 0; r < n; ++r) s += delta2[r * k + o] * A[r * h + j];
      gW2[(int64_t)o * h + j] = s;
    }
    double s = 0.0;
    for (int64_t r = 0; r < n; ++r) s += delta2[r * k + o];
    gb2[o] = s;
  }
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
  free(A);
  free(Y);
  free(delta2);
  free(delta1);
  return L;
}

/* the update of one parameter: plain, or heavy-ball with velocity v */
static void update(double *w, double *v, double g, double lr, double mu) {
  if (v) {
    *v = mu * *v + g;
    *w -= lr * *v;
  } else {
    *w -= lr * g;
  }
}

/*
 * Training loop as ora_train, with the hidden activation `act` and momentum
 * mu; velocity [P] (packed W1 | b1 | W2 | b2) is required when mu != 0 and
 * updated in place (NULL with mu == 0: plain gradient descent).
 */
void ora_train_var(int64_t n, int d, int h, int k, int64_t batch, int act, double mu, const double *X,
                   const double *T, double *W1, double *b1, double *W2, double *b2, double lr, int epochs,
                   double *velocity, double *loss_hist) {
  if (batch <= 0 || batch > n) batch = n;
  int64_t steps = (n + batch - 1) / batch;
  double *gW1 = (double *)malloc(sizeof(double) * (size_t)h * d);
  double *gb1 = (double *)malloc(sizeof(double) * (size_t)h);
  double *gW2 = (double *)malloc(sizeof(double) * (size_t)k * h);
  double *gb2 = (double *)malloc(sizeof(double) * (size_t)k);
  double *vW1 = velocity, *vb1 = velocity ? vW1 + (int64_t)h * d : NULL;
  double *vW2 = velocity ? vb1 + h : NULL, *vb2 = velocity ? vW2 + (int64_t)k * h : NULL;
  for (int e = 0; e < epochs; ++e) {
    double acc = 0.0;
    for (int64_t s = 0; s < steps; ++s) {
      int64_t r0 = s * batch;
      int64_t m = (r0 + batch <= n) ? batch : n - r0;
      acc += loss_grad_var(m, d, h, k, act, X + r0 * d, T + r0 * k, W1, b1, W2, b2, gW1, gb1, gW2, gb2);
      for (int64_t q = 0; q < (int64_t)h * d; ++q) update(W1 + q, vW1 ? vW1 + q : NULL, gW1[q], lr, mu);
      for (int j = 0; j < h; ++j) update(b1 + j, vb1 ? vb1 + j : NULL, gb1[j], lr, mu);
      for (int64_t q = 0; q < (int64_t)k * h; ++q) update(W2 + q, vW2 ? vW2 + q : NULL, gW2[q], lr, mu);
      for (int o = 0; o < k; ++o) update(b2 + o, vb2 ? vb2 + o : NULL, gb2[o], lr, mu);
    }
    if (loss_hist) loss_hist[e] = acc / (double)steps;
  }
  free(gW1);
  free(gb1);
  free(gW2);
  free(gb2);
}

/* Loss and gradients at the given parameters for the hidden activation act. */
double ora_loss_grad_var(int64_t n, int d, int h, int k, int act, const double *X, const double *T,
                         const double *W1, const double *b1, const double *W2, const double *b2, double *gW1,
                         double *gb1, double *gW2, double *gb2) {
  return loss_grad_var(n, d, h, k, act, X, T, W1, b1, W2, b2, gW1, gb1, gW2, gb2);
}
