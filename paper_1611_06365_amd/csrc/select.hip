// Host-side evaluation of the learned selector (variant and block size from
// the problem size; the block-size study of Section 5.1 turned into a model):
// a multilayer perceptron in FP32 whose outputs are the predicted
// log time per flop of every configuration; the smallest wins.
#include "../../include/mlu.h"

#include <cmath>

extern "C" {

int mlu_select(const float* model, int model_len, int n, int precision, int* variant, int* nb) {
  if (!model) return -1;
  if (model_len < 4) return -2;
  if (n < 1) return -3;
  if (precision != MLU_PREC_FP64 && precision != MLU_PREC_FP32) return -4;
  if (!variant) return -5;
  if (!nb) return -6;
  const int n_in = (int)model[0], hidden = (int)model[1], n_out = (int)model[2], n_layers = (int)model[3];
  if (n_in != 3 || hidden < 1 || hidden > 4096 || n_out < 1 || n_out > 4096 || n_layers != 3) return -1;
  const long long need = 4LL + 2LL * n_out + (long long)hidden * n_in + hidden + (long long)hidden * hidden + hidden +
                         (long long)n_out * hidden + n_out;
  if (model_len < need) return -2;
  const float* cfg = model + 4;
  const float* p = cfg + 2 * n_out;
  // features: log2 n scaled, its square, the FP32 flag
  const float x = (float)((std::log2((double)n) - 6.0) / 9.0);
  float in[3] = {x, x * x, precision == MLU_PREC_FP32 ? 1.f : 0.f};
  float h1[4096], h2[4096];
  const int dims[4] = {n_in, hidden, hidden, n_out};
  const float* src = in;
  float* bufs[3] = {h1, h2, h1};
  float best = 0.f;
  int arg = -1;
  for (int l = 0; l < 3; ++l) {
    const int din = dims[l], dout = dims[l + 1];
    const float* W = p;
    const float* b = p + (size_t)dout * din;
    p = b + dout;
    float* dst = bufs[l];
    for (int o = 0; o < dout; ++o) {
      float acc = 0.f;
      for (int i = 0; i < din; ++i) acc += W[(size_t)o * din + i] * src[i];
      acc += b[o];
      if (l < 2) {
        dst[o] = acc > 0.f ? acc : 0.f;
      } else if (arg < 0 || acc < best) {
        best = acc;
        arg = o;
      }
    }
    src = dst;
  }
  *variant = (int)cfg[2 * arg];
  *nb = (int)cfg[2 * arg + 1];
  return 0;
}

}  // extern "C"
