// Host-side evaluation of the learned selector (variant and block size from
// the problem shape; the block-size study of Section 5.1 turned into a model):
// a multilayer perceptron in FP32 that predicts the log time per flop of one
// configuration from (order, batch count, precision, variant, block size);
// every candidate configuration of the shape is scored and the smallest wins.
#include "../../include/mlu.h"

#include <cmath>

namespace {

constexpr int kHeader = 12;
constexpr int kFeatures = 9;
constexpr int kMaxHidden = 1024;

// The features of (n, batch, precision, variant, nb), as the trainer computes
// them: log2 n scaled, its square, log2 batch scaled, the FP32 flag, the
// variant one-hot (RL, LL, LA, batched), log2 nb scaled.
void features(int n, int batch, int precision, int variant, int nb, float* f) {
  const float x = (float)((std::log2((double)n) - 6.0) / 9.0);
  f[0] = x;
  f[1] = x * x;
  f[2] = (float)(std::log2((double)batch) / 14.3);
  f[3] = precision == MLU_PREC_FP32 ? 1.f : 0.f;
  for (int v = 0; v < 4; ++v) f[4 + v] = v == variant ? 1.f : 0.f;
  f[8] = (float)((std::log2((double)nb) - 4.0) / 5.0);
}

// The perceptron's output for one input (three dense layers, ReLU between).
float evaluate(const float* p, int hidden, const float* in) {
  float h1[kMaxHidden], h2[kMaxHidden];
  const int dims[4] = {kFeatures, hidden, hidden, 1};
  const float* src = in;
  float* bufs[2] = {h1, h2};
  float out = 0.f;
  for (int l = 0; l < 3; ++l) {
    const int din = dims[l], dout = dims[l + 1];
    const float* W = p;
    const float* b = p + (size_t)dout * din;
    p = b + dout;
    for (int o = 0; o < dout; ++o) {
      float acc = 0.f;
      for (int i = 0; i < din; ++i) acc += W[(size_t)o * din + i] * src[i];
      acc += b[o];
      if (l < 2) bufs[l][o] = acc > 0.f ? acc : 0.f;
      else out = acc;
    }
    if (l < 2) src = bufs[l];
  }
  return out;
}

}  // namespace

extern "C" {

int mlu_select(const float* model, int model_len, int n, int batch, int precision, int* variant, int* nb,
               int* fallback) {
  if (!model) return -1;
  if (model_len < kHeader) return -2;
  if (n < 1) return -3;
  if (batch < 1) return -4;
  if (precision != MLU_PREC_FP64 && precision != MLU_PREC_FP32) return -5;
  if (!variant) return -6;
  if (!nb) return -7;
  if (!fallback) return -8;
  const int version = (int)model[0], n_in = (int)model[1], hidden = (int)model[2], n_layers = (int)model[3];
  const int n_cand = (int)model[4];
  if (version != 2 || n_in != kFeatures || hidden < 1 || hidden > kMaxHidden || n_layers != 3 || n_cand < 1 ||
      n_cand > 4096)
    return -1;
  const long long need = kHeader + 2LL * n_cand + (long long)hidden * kFeatures + hidden +
                         (long long)hidden * hidden + hidden + hidden + 1;
  if (model_len < need) return -2;
  const float n_lo = model[5], n_hi = model[6], batch_hi = model[7], margin_min = model[8], sd = model[9];
  const int ll_max_panels = (int)model[10], batch_max_n = (int)model[11];
  const float* cand = model + kHeader;
  const float* weights = cand + 2 * n_cand;
  // candidates: the batched kernel's configurations for a batch of small
  // matrices, else the single-matrix ones (left-looking only up to a number
  // of panels)
  const bool batched = batch > 1 && n <= batch_max_n;
  float best = 0.f, second = 0.f;
  int arg = -1;
  bool has_second = false;
  float f[kFeatures];
  for (int c = 0; c < n_cand; ++c) {
    const int v = (int)cand[2 * c], b = (int)cand[2 * c + 1];
    if (b < 1 || v < 0 || v > 3) return -1;
    if (batched != (v == 3)) continue;
    if (v == MLU_LL && (n + b - 1) / b > ll_max_panels) continue;
    features(n, batch, precision, v, b, f);
    const float s = evaluate(weights, hidden, f);
    if (arg < 0) {               // the first candidate
      best = s;
      arg = c;
    } else if (s < best) {       // a new best (the first of equal scores stays)
      second = best;
      has_second = true;
      best = s;
      arg = c;
    } else if (!has_second || s < second) {
      second = s;
      has_second = true;
    }
  }
  if (arg < 0) return -1;
  *variant = (int)cand[2 * arg];
  *nb = (int)cand[2 * arg + 1];
  // scores are (log time - mean) / sd: the runner-up's predicted relative gap
  const double margin = has_second ? std::exp((double)(second - best) * sd) - 1.0 : INFINITY;
  const bool outside = n < n_lo || n > n_hi || batch > batch_hi;
  *fallback = (outside || margin < margin_min) ? 1 : 0;
  return 0;
}

}  // extern "C"
