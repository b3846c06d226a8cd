// C ABI of the convolutional surrogate: single conv layers (forward, input
// gradient, weight gradient, weight packing), Adam, and the whole 5-level
// encoder-decoder as one object that owns its parameters, moments,
// activations and gradients in device memory.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>
#include <utility>
#include <vector>

#include "nn.hpp"
#include "vlbm.h"

namespace vlbm {
int set_error(int code, const char* fmt, ...);   // capi.hip
}

namespace {

using vlbm::nn::Conv;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return vlbm::set_error(code, "%s", buf);
}

int ok() { return vlbm::set_error(VLBM_OK, "%s", ""); }

#define NN_TRY(expr)                                                               \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) return fail(VLBM_ERR_DEVICE, "%s", hipGetErrorString(e_)); \
  } while (0)

int conv_of(const vlbm_conv_desc* d, Conv* c) {
  if (!d) return fail(VLBM_ERR_ARG, "null conv descriptor");
  c->N = d->batch;
  c->H = d->height;
  c->W = d->width;
  c->cin = d->c_in;
  c->cskip = d->c_skip;
  c->up = d->upsample ? 1 : 0;
  c->stride = d->stride;
  c->cout = d->c_out;
  c->relu = d->relu ? 1 : 0;
  c->OH = c->stride > 0 ? (c->H + c->stride - 1) / c->stride : 0;
  c->OW = c->stride > 0 ? (c->W + c->stride - 1) / c->stride : 0;
  if (const char* why = vlbm::nn::check(*c)) return fail(VLBM_ERR_ARG, "conv layer: %s", why);
  return VLBM_OK;
}

// ---- the network ----------------------------------------------------------

constexpr int kLevels = 5;
constexpr int kChannels[kLevels] = {32, 64, 128, 256, 256};
constexpr int kIn = 8;        // stored input channels (features padded with zeros)
constexpr int kOut = 16;      // stored output channels
constexpr int kFeatures = 3;  // caller's input channels
constexpr int kTargets = 3;   // caller's output channels

struct Layer {
  Conv c;
  int src, skip;           // producing layers of the primary and skip inputs (-1: network input)
  int64_t w_off, b_off;    // offsets in the parameter vector
  int64_t act_off;         // offset in the activation pools (per sample * max batch)
  int64_t out_per_sample;  // output elements per sample
};

struct Net {
  int H = 0, W = 0, max_batch = 0;
  hipStream_t stream = nullptr;
  std::vector<Layer> layers;
  int64_t nparams = 0, nweights16 = 0, act_total = 0, max_out = 0;
  float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
  uint16_t *w16 = nullptr, *wt16 = nullptr;
  uint16_t* in16 = nullptr;
  uint16_t* act = nullptr;   // BF16 outputs of every layer but the head
  float* gact = nullptr;     // their FP32 gradients
  float* out32 = nullptr;    // head output [pixels][kOut]
  float* gout = nullptr;
  uint16_t* gy16 = nullptr;
  uint16_t* gy16b = nullptr;  // the next layer's BF16 output gradient, formed by this layer's input gradient
  double* loss = nullptr;
  double* lossp = nullptr;   // per-block loss partials (ordered reduction)
  float* wwork = nullptr;    // partial weight-gradient tiles (ordered reduction)
  int64_t wwork_n = 0;
  int64_t step = 0;
};

// Layer order and parameter layout: per layer the weights [c_out][3][3][c_in + c_skip]
// then the bias [c_out]; encoder levels 0..4 (two convs each, the first of
// levels 1..4 with stride 2), decoder levels 3..0 (the first conv reads the
// 2x-upsampled tensor from below followed by the encoder output of its level),
// then the head.
void build_layers(Net* n, int batch) {
  n->layers.clear();
  const int H = n->H, W = n->W;
  auto add = [&](int h, int w, int cin, int cskip, int up, int stride, int cout, int relu, int src, int skip) {
    Layer L{};
    L.c.N = batch;
    L.c.H = h;
    L.c.W = w;
    L.c.cin = cin;
    L.c.cskip = cskip;
    L.c.up = up;
    L.c.stride = stride;
    L.c.cout = cout;
    L.c.relu = relu;
    L.c.OH = (h + stride - 1) / stride;
    L.c.OW = (w + stride - 1) / stride;
    L.src = src;
    L.skip = skip;
    n->layers.push_back(L);
  };
  int enc_out[kLevels];
  for (int l = 0; l < kLevels; ++l) {
    const int hin = l == 0 ? H : (H >> (l - 1)), win = l == 0 ? W : (W >> (l - 1));
    add(hin, win, l == 0 ? kIn : kChannels[l - 1], 0, 0, l == 0 ? 1 : 2, kChannels[l], 1,
        l == 0 ? -1 : enc_out[l - 1], -1);
    add(H >> l, W >> l, kChannels[l], 0, 0, 1, kChannels[l], 1, (int)n->layers.size() - 1, -1);
    enc_out[l] = (int)n->layers.size() - 1;
  }
  int below = enc_out[kLevels - 1];
  for (int l = kLevels - 2; l >= 0; --l) {
    add(H >> l, W >> l, kChannels[l + 1], kChannels[l], 1, 1, kChannels[l], 1, below, enc_out[l]);
    add(H >> l, W >> l, kChannels[l], 0, 0, 1, kChannels[l], 1, (int)n->layers.size() - 1, -1);
    below = (int)n->layers.size() - 1;
  }
  add(H, W, kChannels[0], 0, 0, 1, kOut, 0, below, -1);
  int64_t p = 0, a = 0, mo = 0;
  for (Layer& L : n->layers) {
    L.w_off = p;
    p += (int64_t)L.c.cout * 9 * L.c.ctot();
    L.b_off = p;
    p += L.c.cout;
    L.out_per_sample = (int64_t)L.c.OH * L.c.OW * L.c.cout;
    L.act_off = a;
    a += L.out_per_sample * n->max_batch;
    mo = std::max<int64_t>(mo, L.out_per_sample);
  }
  n->nparams = p;
  n->act_total = a;
  n->max_out = mo;
}

void set_batch(Net* n, int batch) {
  for (Layer& L : n->layers) L.c.N = batch;
}

void free_net(Net* n) {
  if (!n) return;
  if (n->stream) (void)hipStreamSynchronize(n->stream);
  void* ptrs[] = {n->params, n->grads, n->m, n->v, n->w16, n->wt16, n->in16, n->act, n->gact, n->out32,
                  n->gout, n->gy16, n->gy16b, n->loss, n->lossp, n->wwork};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete n;
}

template <class T>
hipError_t alloc(T** p, int64_t count) {
  return hipMalloc((void**)p, sizeof(T) * (size_t)(count > 0 ? count : 1));
}

const uint16_t* input_of(const Net* n, int idx) {
  if (idx < 0) return n->in16;
  return n->act + n->layers[idx].act_off;
}

float* grad_of(const Net* n, int idx) { return idx < 0 ? nullptr : n->gact + n->layers[idx].act_off; }

int pack_all(Net* n) {
  std::vector<Conv> convs;
  std::vector<int64_t> offs;
  for (const Layer& L : n->layers) {
    convs.push_back(L.c);
    offs.push_back(L.w_off);
  }
  NN_TRY(vlbm::nn::pack_weights_all((int)convs.size(), convs.data(), offs.data(), n->params, n->w16, n->wt16,
                                    n->stream));
  return VLBM_OK;
}

int forward(Net* n, const float* x, int batch) {
  if (!x || batch <= 0 || batch > n->max_batch) return fail(VLBM_ERR_ARG, "surrogate: bad input or batch size");
  set_batch(n, batch);
  const int64_t pixels = (int64_t)batch * n->H * n->W;
  NN_TRY(vlbm::nn::pack_input(x, n->in16, pixels, kFeatures, kIn, n->stream));
  const int last = (int)n->layers.size() - 1;
  for (int i = 0; i <= last; ++i) {
    const Layer& L = n->layers[i];
    const uint16_t* skip = L.skip >= 0 ? input_of(n, L.skip) : nullptr;
    NN_TRY(vlbm::nn::conv_forward(L.c, input_of(n, L.src), skip, n->w16 + L.w_off, n->params + L.b_off,
                                  i == last ? nullptr : n->act + L.act_off, i == last ? n->out32 : nullptr,
                                  n->stream));
  }
  return VLBM_OK;
}

int gradient(Net* n, const float* x, const float* t, int batch) {
  if (!t) return fail(VLBM_ERR_ARG, "surrogate: null target");
  int rc = forward(n, x, batch);
  if (rc) return rc;
  const int64_t pixels = (int64_t)batch * n->H * n->W;
  // a layer output's gradient is stored by its first contribution in backward
  // order (its highest-numbered consumer) and added to by the others, so it
  // needs no clearing
  std::vector<int> first(n->layers.size(), -1);
  for (int i = 0; i < (int)n->layers.size(); ++i) {
    const Layer& L = n->layers[i];
    if (L.src >= 0) first[L.src] = std::max(first[L.src], i);
    if (L.skip >= 0) first[L.skip] = std::max(first[L.skip], i);
  }
  NN_TRY(vlbm::nn::mse(n->out32, t, n->gout, n->loss, pixels, kOut, kTargets, n->lossp, n->stream));
  const int last = (int)n->layers.size() - 1;
  // Layer i's output gradient is complete once layer i + 1, its last consumer
  // in backward order, has added its input gradient (a decoder reading it as
  // skip runs earlier); that input gradient then also forms the BF16 ReLU
  // gradient layer i starts from, into the second buffer.
  uint16_t* gcur = n->gy16;
  uint16_t* gnext = n->gy16b;
  bool ready = false;
  for (int i = last; i >= 0; --i) {
    const Layer& L = n->layers[i];
    const int64_t nout = L.out_per_sample * batch;
    if (!ready) {
      const float* g = i == last ? n->gout : n->gact + L.act_off;
      NN_TRY(vlbm::nn::relu_grad(g, i == last ? nullptr : n->act + L.act_off, gcur, nout, L.c.relu, n->stream));
    }
    const uint16_t* skip = L.skip >= 0 ? input_of(n, L.skip) : nullptr;
    // each layer's weight and bias gradients are formed once: stored, not added
    NN_TRY(vlbm::nn::conv_backward_weight(L.c, input_of(n, L.src), skip, gcur, n->grads + L.w_off,
                                          n->grads + L.b_off, n->stream, n->wwork, n->wwork_n, 1));
    ready = false;
    if (L.src >= 0) {
      const Layer& S = n->layers[L.src];
      const bool fuse = L.src == i - 1;
      NN_TRY(vlbm::nn::conv_backward_data(L.c, gcur, n->wt16 + L.w_off, grad_of(n, L.src),
                                          L.skip >= 0 ? grad_of(n, L.skip) : nullptr, n->stream,
                                          fuse ? n->act + S.act_off : nullptr, S.c.relu, fuse ? gnext : nullptr,
                                          first[L.src] == i, L.skip >= 0 && first[L.skip] == i));
      ready = fuse;
    }
    std::swap(gcur, gnext);
  }
  return VLBM_OK;
}

int adam_update(Net* n, const vlbm_adam* hp) {
  if (!hp || !(hp->lr > 0) || !(hp->beta1 >= 0 && hp->beta1 < 1) || !(hp->beta2 >= 0 && hp->beta2 < 1) ||
      !(hp->eps > 0))
    return fail(VLBM_ERR_ARG, "adam: bad hyper-parameters");
  n->step++;
  const double c1 = 1.0 / (1.0 - std::pow(hp->beta1, (double)n->step));
  const double c2 = 1.0 / (1.0 - std::pow(hp->beta2, (double)n->step));
  NN_TRY(vlbm::nn::adam(n->params, n->grads, n->m, n->v, n->nparams, (float)hp->lr, (float)hp->beta1,
                        (float)hp->beta2, (float)hp->eps, (float)c1, (float)c2, n->stream));
  return pack_all(n);
}

int read_loss(Net* n, double* loss) {
  if (!loss) return VLBM_OK;
  NN_TRY(hipMemcpyAsync(loss, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->stream));
  NN_TRY(hipStreamSynchronize(n->stream));
  return VLBM_OK;
}

}  // namespace

extern "C" {

int vlbm_conv2d_forward(const vlbm_conv_desc* d, const uint16_t* x, const uint16_t* skip, const uint16_t* w,
                        const float* bias, uint16_t* y_bf16, float* y_f32, void* stream) {
  Conv c;
  if (int rc = conv_of(d, &c)) return rc;
  if (!x || !w || (c.cskip && !skip) || (!y_bf16 && !y_f32)) return fail(VLBM_ERR_ARG, "conv forward: null pointer");
  NN_TRY(vlbm::nn::conv_forward(c, x, skip, w, bias, y_bf16, y_f32, static_cast<hipStream_t>(stream)));
  return ok();
}

int vlbm_conv2d_backward_data(const vlbm_conv_desc* d, const uint16_t* gy, const uint16_t* wt, float* gx,
                              float* gskip, void* stream) {
  Conv c;
  if (int rc = conv_of(d, &c)) return rc;
  if (!gy || !wt || (!gx && !gskip)) return fail(VLBM_ERR_ARG, "conv backward-data: null pointer");
  NN_TRY(vlbm::nn::conv_backward_data(c, gy, wt, gx, gskip, static_cast<hipStream_t>(stream)));
  return ok();
}

int vlbm_conv2d_backward_weight(const vlbm_conv_desc* d, const uint16_t* x, const uint16_t* skip,
                                const uint16_t* gy, float* gw, float* gb, void* stream) {
  Conv c;
  if (int rc = conv_of(d, &c)) return rc;
  if (!x || !gy || !gw || !gb || (c.cskip && !skip)) return fail(VLBM_ERR_ARG, "conv backward-weight: null pointer");
  NN_TRY(vlbm::nn::conv_backward_weight(c, x, skip, gy, gw, gb, static_cast<hipStream_t>(stream)));
  return ok();
}

int vlbm_conv2d_pack_weights(const vlbm_conv_desc* d, const float* w, uint16_t* w_bf16, uint16_t* wt_bf16,
                             void* stream) {
  Conv c;
  if (int rc = conv_of(d, &c)) return rc;
  if (!w || !w_bf16 || !wt_bf16) return fail(VLBM_ERR_ARG, "pack weights: null pointer");
  NN_TRY(vlbm::nn::pack_weights(c, w, w_bf16, wt_bf16, static_cast<hipStream_t>(stream)));
  return ok();
}

int vlbm_adam_step(float* p, const float* g, float* m, float* v, int64_t n, const vlbm_adam* hp, int64_t step,
                   void* stream) {
  if (!p || !g || !m || !v || n < 0 || !hp || step < 1) return fail(VLBM_ERR_ARG, "vlbm_adam_step: bad argument");
  const double c1 = 1.0 / (1.0 - std::pow(hp->beta1, (double)step));
  const double c2 = 1.0 / (1.0 - std::pow(hp->beta2, (double)step));
  NN_TRY(vlbm::nn::adam(p, g, m, v, n, (float)hp->lr, (float)hp->beta1, (float)hp->beta2, (float)hp->eps,
                        (float)c1, (float)c2, static_cast<hipStream_t>(stream)));
  return ok();
}

int vlbm_surrogate_param_count(int height, int width, int64_t* n) {
  if (!n || height <= 0 || width <= 0 || height % 16 || width % 16)
    return fail(VLBM_ERR_ARG, "surrogate: height and width must be positive multiples of 16");
  Net tmp;
  tmp.H = height;
  tmp.W = width;
  tmp.max_batch = 1;
  build_layers(&tmp, 1);
  *n = tmp.nparams;
  return ok();
}

int vlbm_surrogate_create(int height, int width, int max_batch, const float* params, void* stream,
                          vlbm_surrogate* out) {
  if (!out || !params || max_batch <= 0 || height <= 0 || width <= 0 || height % 16 || width % 16)
    return fail(VLBM_ERR_ARG, "vlbm_surrogate_create: bad argument (sizes must be multiples of 16)");
  *out = nullptr;
  Net* n = new (std::nothrow) Net();
  if (!n) return fail(VLBM_ERR_NOMEM, "host allocation failed");
  n->H = height;
  n->W = width;
  n->max_batch = max_batch;
  n->stream = static_cast<hipStream_t>(stream);
  build_layers(n, max_batch);
  const int64_t pixels = (int64_t)max_batch * height * width;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  A(alloc(&n->params, n->nparams));
  A(alloc(&n->grads, n->nparams));
  A(alloc(&n->m, n->nparams));
  A(alloc(&n->v, n->nparams));
  A(alloc(&n->w16, n->nparams));
  A(alloc(&n->wt16, n->nparams));
  A(alloc(&n->in16, pixels * kIn));
  A(alloc(&n->act, n->act_total));
  A(alloc(&n->gact, n->act_total));
  A(alloc(&n->out32, pixels * kOut));
  A(alloc(&n->gout, pixels * kOut));
  A(alloc(&n->gy16, n->max_out * max_batch));
  A(alloc(&n->gy16b, n->max_out * max_batch));
  A(alloc(&n->loss, 1));
  A(alloc(&n->lossp, vlbm::nn::kMseBlocks));
  // the weight gradients add their split partial sums in a fixed order, so
  // training is bit-reproducible; the workspace fits the largest layer at any
  // batch size
  for (const Layer& L : n->layers) {
    const int64_t need = vlbm::nn::conv_backward_weight_workspace(L.c);
    if (need > n->wwork_n) n->wwork_n = need;
  }
  A(alloc(&n->wwork, n->wwork_n));
  if (e != hipSuccess) {
    free_net(n);
    return fail(VLBM_ERR_NOMEM, "surrogate: device allocation failed (%s)", hipGetErrorString(e));
  }
  A(hipMemcpyAsync(n->params, params, sizeof(float) * n->nparams, hipMemcpyDefault, n->stream));
  if (e == hipSuccess) e = vlbm::nn::fill(n->m, n->nparams, 0.f, n->stream);
  if (e == hipSuccess) e = vlbm::nn::fill(n->v, n->nparams, 0.f, n->stream);
  if (e == hipSuccess) e = vlbm::nn::fill(n->grads, n->nparams, 0.f, n->stream);
  if (e != hipSuccess) {
    free_net(n);
    return fail(VLBM_ERR_DEVICE, "surrogate: %s", hipGetErrorString(e));
  }
  if (int rc = pack_all(n)) {
    free_net(n);
    return rc;
  }
  *out = reinterpret_cast<vlbm_surrogate>(n);
  return ok();
}

int vlbm_surrogate_forward(vlbm_surrogate s, const float* x, int batch, float* y) {
  Net* n = reinterpret_cast<Net*>(s);
  if (!n || !y) return fail(VLBM_ERR_ARG, "vlbm_surrogate_forward: null argument");
  if (int rc = forward(n, x, batch)) return rc;
  NN_TRY(vlbm::nn::unpack_output(n->out32, y, (int64_t)batch * n->H * n->W, kOut, kTargets, n->stream));
  return ok();
}

int vlbm_surrogate_gradient(vlbm_surrogate s, const float* x, const float* target, int batch, double* loss,
                            float* grad) {
  Net* n = reinterpret_cast<Net*>(s);
  if (!n) return fail(VLBM_ERR_ARG, "null surrogate");
  if (int rc = gradient(n, x, target, batch)) return rc;
  if (grad) NN_TRY(hipMemcpyAsync(grad, n->grads, sizeof(float) * n->nparams, hipMemcpyDefault, n->stream));
  if (int rc = read_loss(n, loss)) return rc;
  return ok();
}

int vlbm_surrogate_adam(vlbm_surrogate s, const vlbm_adam* hp) {
  Net* n = reinterpret_cast<Net*>(s);
  if (!n) return fail(VLBM_ERR_ARG, "null surrogate");
  if (int rc = adam_update(n, hp)) return rc;
  return ok();
}

int vlbm_surrogate_train_step(vlbm_surrogate s, const float* x, const float* target, int batch,
                              const vlbm_adam* hp, double* loss) {
  Net* n = reinterpret_cast<Net*>(s);
  if (!n) return fail(VLBM_ERR_ARG, "null surrogate");
  if (int rc = gradient(n, x, target, batch)) return rc;
  if (int rc = adam_update(n, hp)) return rc;
  if (int rc = read_loss(n, loss)) return rc;
  return ok();
}

int vlbm_surrogate_params(vlbm_surrogate s, float* out, int64_t* step) {
  Net* n = reinterpret_cast<Net*>(s);
  if (!n || !out) return fail(VLBM_ERR_ARG, "vlbm_surrogate_params: null argument");
  NN_TRY(hipMemcpyAsync(out, n->params, sizeof(float) * n->nparams, hipMemcpyDefault, n->stream));
  NN_TRY(hipStreamSynchronize(n->stream));
  if (step) *step = n->step;
  return ok();
}

int vlbm_surrogate_destroy(vlbm_surrogate s) {
  free_net(reinterpret_cast<Net*>(s));
  return VLBM_OK;
}

}  // extern "C"
