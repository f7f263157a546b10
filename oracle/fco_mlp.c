/*
 * fco_mlp.c -- the learned-tagging network of the CPU oracle (test
 * infrastructure only).  Not part of the paper: an extension that predicts
 * the refine / keep / coarsen tags of the Sec. 5 criterion a few steps
 * ahead from per-patch statistics (fco_features).
 *
 * Network: 16 inputs -> 64 -> 64 -> 3 logits, GELU after both hidden layers
 * in its exact form z * Phi(z) (Phi the standard normal distribution
 * function, through erf).  Inputs are standardised, x_n = (x - mu) / sigma.
 * Parameter vector, 5443 values:
 *   W1[16][64] b1[64] W2[64][64] b2[64] W3[64][3] b3[3]
 * (row index = input unit, column = output unit).
 * Loss: scale * sum_r w[y_r] * (-log softmax(z_r)[y_r]).
 *
 * With round = 1 every operand of a matrix product is first rounded to
 * bfloat16 (8 significant bits, round to nearest, ties to even): the
 * standardised inputs, the three weight matrices, both hidden activations,
 * and in the backward pass the logit gradient and both pre-activation
 * gradients; biases and element-wise work stay unrounded.  The standardised
 * input that is rounded is formed in FP32 (see standardise32).  Everything
 * else is evaluated in FP64, so the result is the exact value (to FP64 rounding)
 * of the network on those rounded operands.  With round = 0 it is the plain
 * FP64 network, whose gradient is exactly the derivative of its loss.
 *
 * Adam: Kingma and Ba (2015), Algorithm 1, with bias correction.
 */
#include "fco.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { NI = 16, NH = 64, NO = 3 };
enum { OW1 = 0, OB1 = OW1 + NI * NH, OW2 = OB1 + NH, OB2 = OW2 + NH * NH,
       OW3 = OB2 + NH, OB3 = OW3 + NH * NO, NPARAM = OB3 + NO };

double fco_bf16(double x) {
  if (x == 0.0 || !isfinite(x)) return x;
  int e;
  double f = frexp(x, &e);                 /* x = f 2^e, 0.5 <= |f| < 1 */
  return ldexp(nearbyint(ldexp(f, 8)), e - 8);
}

static double rnd(double x, int round) { return round ? fco_bf16(x) : x; }

/* The rounded network standardises its inputs in FP32, (x - mu) * (1 / sigma)
 * with each operation rounded to FP32, because the bfloat16 code of the
 * result is a decision taken in the precision of the matrix-core network;
 * the plain network standardises in FP64. */
static double standardise32(double x, double mu, double sigma) {
  const float d = (float)x - (float)mu;
  const float is = 1.0f / (float)sigma;
  const float v = d * is;
  return (double)v;
}

static double gelu(double z) { return 0.5 * z * (1.0 + erf(z / sqrt(2.0))); }

/* d/dz [z Phi(z)] = Phi(z) + z phi(z) */
static double gelu_d(double z) {
  const double two_pi = 6.28318530717958647692;
  return 0.5 * (1.0 + erf(z / sqrt(2.0))) + z * exp(-0.5 * z * z) / sqrt(two_pi);
}

double fco_mlp(const double *P, const double *norm, int64_t M, const double *x,
               const int32_t *y, const double *cw, double scale, int32_t round,
               double *logits, double *grad) {
  double W1[NI * NH], W2[NH * NH], W3[NH * NO];
  for (int t = 0; t < NI * NH; ++t) W1[t] = rnd(P[OW1 + t], round);
  for (int t = 0; t < NH * NH; ++t) W2[t] = rnd(P[OW2 + t], round);
  for (int t = 0; t < NH * NO; ++t) W3[t] = rnd(P[OW3 + t], round);
  const double *b1 = P + OB1, *b2 = P + OB2, *b3 = P + OB3;
  if (grad) memset(grad, 0, sizeof(double) * NPARAM);
  double loss = 0.0;
  for (int64_t r = 0; r < M; ++r) {
    /* forward */
    double xn[NI], z1[NH], h1[NH], z2[NH], h2[NH], z3[NO];
    for (int f = 0; f < NI; ++f)
      xn[f] = round ? fco_bf16(standardise32(x[r * NI + f], norm[f], norm[NI + f]))
                    : (x[r * NI + f] - norm[f]) / norm[NI + f];
    for (int o = 0; o < NH; ++o) {
      double s = 0.0;
      for (int f = 0; f < NI; ++f) s += xn[f] * W1[f * NH + o];
      z1[o] = s + b1[o];
      h1[o] = rnd(gelu(z1[o]), round);
    }
    for (int o = 0; o < NH; ++o) {
      double s = 0.0;
      for (int f = 0; f < NH; ++f) s += h1[f] * W2[f * NH + o];
      z2[o] = s + b2[o];
      h2[o] = rnd(gelu(z2[o]), round);
    }
    for (int o = 0; o < NO; ++o) {
      double s = 0.0;
      for (int f = 0; f < NH; ++f) s += h2[f] * W3[f * NO + o];
      z3[o] = s + b3[o];
      if (logits) logits[r * NO + o] = z3[o];
    }
    if (!y) continue;
    /* softmax cross-entropy, weighted */
    double zm = fmax(z3[0], fmax(z3[1], z3[2]));
    double e[NO], se = 0.0;
    for (int o = 0; o < NO; ++o) {
      e[o] = exp(z3[o] - zm);
      se += e[o];
    }
    const int c = y[r];
    const double w = scale * cw[c];
    loss += w * (log(se) + zm - z3[c]);
    if (!grad) continue;
    /* backward: dL/dz3 = w (softmax - onehot) */
    double g3[NO], d2[NH], d1[NH];
    for (int o = 0; o < NO; ++o) g3[o] = rnd(w * (e[o] / se - (o == c ? 1.0 : 0.0)), round);
    for (int o = 0; o < NO; ++o) {
      grad[OB3 + o] += g3[o];
      for (int f = 0; f < NH; ++f) grad[OW3 + f * NO + o] += h2[f] * g3[o];
    }
    for (int f = 0; f < NH; ++f) {
      double s = 0.0;
      for (int o = 0; o < NO; ++o) s += g3[o] * W3[f * NO + o];
      d2[f] = rnd(s * gelu_d(z2[f]), round);
    }
    for (int o = 0; o < NH; ++o) {
      grad[OB2 + o] += d2[o];
      for (int f = 0; f < NH; ++f) grad[OW2 + f * NH + o] += h1[f] * d2[o];
    }
    for (int f = 0; f < NH; ++f) {
      double s = 0.0;
      for (int o = 0; o < NH; ++o) s += d2[o] * W2[f * NH + o];
      d1[f] = rnd(s * gelu_d(z1[f]), round);
    }
    for (int o = 0; o < NH; ++o) {
      grad[OB1 + o] += d1[o];
      for (int f = 0; f < NI; ++f) grad[OW1 + f * NH + o] += xn[f] * d1[o];
    }
  }
  return loss;
}

void fco_adam(int64_t n, double *P, const double *g, double *m1, double *m2,
              int32_t t, double lr, double beta1, double beta2, double eps) {
  const double c1 = 1.0 - pow(beta1, t), c2 = 1.0 - pow(beta2, t);
  for (int64_t i = 0; i < n; ++i) {
    m1[i] = beta1 * m1[i] + (1.0 - beta1) * g[i];
    m2[i] = beta2 * m2[i] + (1.0 - beta2) * g[i] * g[i];
    P[i] -= lr * (m1[i] / c1) / (sqrt(m2[i] / c2) + eps);
  }
}

/* Tags from logits (class 0 refine, 1 keep, 2 coarsen), with the plain
 * criterion as fallback: a patch the plain criterion tags +1 stays +1, and
 * where the largest softmax probability is below `confidence` the plain tag
 * is used; otherwise the most likely class (lowest class on ties). */
void fco_learned_tags(int64_t M, const double *logits, const int8_t *plain,
                      double confidence, int8_t *tags) {
  for (int64_t r = 0; r < M; ++r) {
    const double *z = logits + r * NO;
    int best = 0;
    for (int o = 1; o < NO; ++o)
      if (z[o] > z[best]) best = o;
    double se = 0.0;
    for (int o = 0; o < NO; ++o) se += exp(z[o] - z[best]);
    const double pmax = 1.0 / se;
    if (plain[r] == 1 || pmax < confidence)
      tags[r] = plain[r];
    else
      tags[r] = (int8_t)(1 - best);
  }
}
