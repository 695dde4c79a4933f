/*
 * FP64 CPU oracle for the reduced-precision forms of the trainer.
 *
 * TEST INFRASTRUCTURE ONLY (same rules as mlp_oracle.c: only tests, the
 * smoke check and the benchmark's CPU baseline load it).
 *
 * The paper trains in float (section 2.2) and says nothing about lower
 * precision; these forms are the build's own.  Their definition: the method
 * of mlp_oracle.c, unchanged, except that the operands of the two large
 * contractions -- the hidden pre-activation X W1^T and the input-layer
 * gradient delta1^T X -- are rounded to a narrow format before the
 * (exact) products are summed.  Everything else (biases, sigmoid, the
 * output layer, both deltas, gb1, gW2, gb2, the loss and the update of the
 * master parameters) stays in full precision.
 *
 *   prec 1 (bf16): operands rounded to 8 significant bits, round to nearest
 *                  even, exponent range of float32.
 *   prec 2 (e4m3): OCP FP8 E4M3 (4 significant bits, smallest normal 2^-6,
 *                  largest finite 448, no infinities) with a per-tensor
 *                  power-of-two scale s: an operand v is represented as
 *                  q(v*s)/s where q rounds to nearest even and saturates to
 *                  +-448.  s = 2^e with e the largest integer such that
 *                  amax*2^e <= 448 (e = 0 when amax = 0):
 *                    X:      amax over the whole dataset, once;
 *                    W1:     amax of the master W1 at the current step;
 *                    delta1: amax of delta1 over the previous minibatch
 *                            (delayed scaling); at the first step the bound
 *                            max_j sum_o |W2[o][j]| / (8 m K), which no
 *                            delta1 of that step can exceed since
 *                            |Y-T| <= 1 and sigma(1-sigma) <= 1/4.
 *                            That bound is formed in float32, left to right.
 * With prec 0 no operand is rounded and the result equals mlp_oracle.c.
 * Large loops share their independent outputs among OpenMP threads, each
 * output formed by the same loop in the same order (thread-count
 * independent, bit for bit; the amax is a maximum, exact in any order).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Round v to p significant bits, smallest normal exponent emin, saturating
 * at +-maxv; ties to even (C's default rounding mode for nearbyint). */
double ora_round_format(double v, int p, int emin, double maxv) {
  if (v == 0.0 || isnan(v)) return v;
  int ex;
  frexp(fabs(v), &ex);            /* |v| = f * 2^ex, f in [0.5, 1) */
  int e = ex - 1;                 /* exponent of the leading bit */
  if (e < emin) e = emin;         /* subnormal range: fixed spacing */
  double ulp = ldexp(1.0, e - (p - 1));
  double r = nearbyint(v / ulp) * ulp;
  if (r > maxv) r = maxv;
  if (r < -maxv) r = -maxv;
  return r;
}

double ora_round_bf16(double v) { return ora_round_format(v, 8, -126, 3.3895313892515355e38); }
double ora_round_e4m3(double v) { return ora_round_format(v, 4, -6, 448.0); }

/* e such that amax*2^e <= 448 < amax*2^(e+1); 0 for amax == 0. */
int ora_e4m3_scale_exp(double amax) {
  if (!(amax > 0.0)) return 0;
  int ex;
  double f = frexp(amax, &ex);    /* amax = f * 2^ex; 448 = 0.875 * 2^9 */
  return (f <= 0.875) ? 9 - ex : 8 - ex;
}

static double q_op(double v, int prec, int sexp) {
  if (prec == 1) return ora_round_bf16(v);
  if (prec == 2) return ldexp(ora_round_e4m3(ldexp(v, sexp)), -sexp);
  return v;
}

static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

#define ORA_PAR(work) ((int64_t)(work) >= ((int64_t)1 << 18))

/* Round n values to the operand format of prec with scale 2^sexp (e4m3). */
void ora_round_array(int prec, int sexp, const double *in, double *out, int64_t n) {
  for (int64_t q = 0; q < n; ++q) out[q] = q_op(in[q], prec, sexp);
}

/*
 * Training loop with rounded contraction operands.  Same loop, loss and
 * update as ora_train.  scale_log (may be NULL) receives, per step, the three
 * scale exponents used (X, W1, delta1); it is written only for prec 2.
 * d1_first and bp_first (may be NULL; [batch][h]) receive, for the first
 * step, delta1 and its back-propagated factor delta2 W2 before the sigmoid
 * derivative is applied.
 */
void ora_train_lowp(int64_t n, int d, int h, int k, int64_t batch, const double *X,
                    const double *T, double *W1, double *b1, double *W2, double *b2, double lr,
                    int epochs, int prec, double *loss_hist, int32_t *scale_log, double *d1_first,
                    double *bp_first) {
  if (batch <= 0 || batch > n) batch = n;
  int64_t steps = (n + batch - 1) / batch;
  int64_t bmax = batch;
  double *A = (double *)malloc(sizeof(double) * (size_t)(bmax * h));
  double *Y = (double *)malloc(sizeof(double) * (size_t)(bmax * k));
  double *delta2 = (double *)malloc(sizeof(double) * (size_t)(bmax * k));
  double *delta1 = (double *)malloc(sizeof(double) * (size_t)(bmax * h));
  double *gW1 = (double *)malloc(sizeof(double) * (size_t)h * d);
  double *gb1 = (double *)malloc(sizeof(double) * (size_t)h);
  double *gW2 = (double *)malloc(sizeof(double) * (size_t)k * h);
  double *gb2 = (double *)malloc(sizeof(double) * (size_t)k);
  double *Xq = (double *)malloc(sizeof(double) * (size_t)(n * d));
  double *W1q = (double *)malloc(sizeof(double) * (size_t)h * d);
  double *delta1q = (double *)malloc(sizeof(double) * (size_t)(bmax * h));

  int ex = 0;
  if (prec == 2) {
    double amax = 0.0;
    for (int64_t q = 0; q < n * d; ++q) amax = fmax(amax, fabs(X[q]));
    ex = ora_e4m3_scale_exp(amax);
  }
  for (int64_t q = 0; q < n * d; ++q) Xq[q] = q_op(X[q], prec, ex);
  double amax_d1_prev = -1.0;  /* < 0: first step, use the bound */
  int64_t step_no = 0;

  for (int e = 0; e < epochs; ++e) {
    double acc = 0.0;
    for (int64_t s = 0; s < steps; ++s, ++step_no) {
      int64_t r0 = s * batch;
      int64_t m = (r0 + batch <= n) ? batch : n - r0;
      const double *Xqb = Xq + r0 * d;
      const double *Tb = T + r0 * k;
      int ew = 0, ed = 0;
      if (prec == 2) {
        double amax = 0.0;
        for (int64_t q = 0; q < (int64_t)h * d; ++q) amax = fmax(amax, fabs(W1[q]));
        ew = ora_e4m3_scale_exp(amax);
        if (amax_d1_prev < 0.0) {
          float bound = 0.0f;
          for (int j = 0; j < h; ++j) {
            float col = 0.0f;
            for (int o = 0; o < k; ++o) col = col + fabsf((float)W2[(int64_t)o * h + j]);
            if (col > bound) bound = col;
          }
          bound = bound / (float)(8 * m * k);
          ed = ora_e4m3_scale_exp((double)bound);
        } else {
          ed = ora_e4m3_scale_exp(amax_d1_prev);
        }
        if (scale_log) {
          scale_log[step_no * 3 + 0] = ex;
          scale_log[step_no * 3 + 1] = ew;
          scale_log[step_no * 3 + 2] = ed;
        }
      }
      for (int64_t q = 0; q < (int64_t)h * d; ++q) W1q[q] = q_op(W1[q], prec, ew);
      /* feed forward */
#pragma omp parallel for schedule(static) if (ORA_PAR(m * h * d))
      for (int64_t r = 0; r < m; ++r) {
        for (int j = 0; j < h; ++j) {
          double z = 0.0;
          for (int i = 0; i < d; ++i) z += Xqb[r * d + i] * W1q[(int64_t)j * d + i];
          A[r * h + j] = sigmoid(z + b1[j]);
        }
        for (int o = 0; o < k; ++o) {
          double z = b2[o];
          for (int j = 0; j < h; ++j) z += A[r * h + j] * W2[(int64_t)o * h + j];
          Y[r * k + o] = sigmoid(z);
        }
      }
      /* error and deltas */
      double L = 0.0;
      for (int64_t r = 0; r < m; ++r)
        for (int o = 0; o < k; ++o) {
          double y = Y[r * k + o], t = Tb[r * k + o];
          L += (y - t) * (y - t);
          delta2[r * k + o] = 2.0 * (y - t) / ((double)m * (double)k) * y * (1.0 - y);
        }
      acc += L / ((double)m * (double)k);
      double amax_d1 = 0.0;
#pragma omp parallel for schedule(static) reduction(max : amax_d1) if (ORA_PAR(m * h * k))
      for (int64_t r = 0; r < m; ++r)
        for (int j = 0; j < h; ++j) {
          double sum = 0.0;
          for (int o = 0; o < k; ++o) sum += delta2[r * k + o] * W2[(int64_t)o * h + j];
          double a = A[r * h + j];
          delta1[r * h + j] = sum * a * (1.0 - a);
          amax_d1 = fmax(amax_d1, fabs(delta1[r * h + j]));
          if (step_no == 0 && d1_first) d1_first[r * h + j] = delta1[r * h + j];
          if (step_no == 0 && bp_first) bp_first[r * h + j] = sum;
        }
      for (int64_t q = 0; q < m * h; ++q) delta1q[q] = q_op(delta1[q], prec, ed);
      /* gradients */
      for (int o = 0; o < k; ++o) {
#pragma omp parallel for schedule(static) if (ORA_PAR(m * h))
        for (int j = 0; j < h; ++j) {
          double sum = 0.0;
          for (int64_t r = 0; r < m; ++r) sum += delta2[r * k + o] * A[r * h + j];
          gW2[(int64_t)o * h + j] = sum;
        }
        double sum = 0.0;
        for (int64_t r = 0; r < m; ++r) sum += delta2[r * k + o];
        gb2[o] = sum;
      }
#pragma omp parallel for schedule(static) if (ORA_PAR(m * h * d))
      for (int j = 0; j < h; ++j) {
        for (int i = 0; i < d; ++i) {
          double sum = 0.0;
          for (int64_t r = 0; r < m; ++r) sum += delta1q[r * h + j] * Xqb[r * d + i];
          gW1[(int64_t)j * d + i] = sum;
        }
        double sum = 0.0;
        for (int64_t r = 0; r < m; ++r) sum += delta1[r * h + j];
        gb1[j] = sum;
      }
      amax_d1_prev = amax_d1;
      /* simultaneous update, no momentum */
      for (int64_t q = 0; q < (int64_t)h * d; ++q) W1[q] -= lr * gW1[q];
      for (int j = 0; j < h; ++j) b1[j] -= lr * gb1[j];
      for (int64_t q = 0; q < (int64_t)k * h; ++q) W2[q] -= lr * gW2[q];
      for (int o = 0; o < k; ++o) b2[o] -= lr * gb2[o];
    }
    if (loss_hist) loss_hist[e] = acc / (double)steps;
  }
  free(A); free(Y); free(delta2); free(delta1);
  free(gW1); free(gb1); free(gW2); free(gb2);
  free(Xq); free(W1q); free(delta1q);
}
