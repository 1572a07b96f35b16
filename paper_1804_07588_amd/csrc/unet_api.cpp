// C ABI of the learned warm start: a 3-D U-Net (two poolings, skip
// connections by channel concatenation) trained and evaluated with the
// kernels of unet_kernels.hip.  The host side only sequences launches and
// owns no device memory: the caller binds one workspace.
#include "fdlbm_unet.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "unet_launch.h"

namespace {

// layer table: input channels (padded), output channels, level (edge R >> level)
struct Layer {
  int ci, co, level, relu;
};
constexpr int CP = FDLBM_UNET_CPAD;  // padded input / output channels
// enc1 a,b | enc2 a,b | bottleneck a,b | dec2 a,b | dec1 a,b | head
constexpr int C1 = 32, C2 = 64, C3 = 160;
const Layer LAYERS[FDLBM_UNET_LAYERS] = {
    {CP, C1, 0, 1},      {C1, C1, 0, 1},      {C1, C2, 1, 1}, {C2, C2, 1, 1},
    {C2, C3, 2, 1},      {C3, C3, 2, 1},      {C3 + C2, C2, 1, 1}, {C2, C2, 1, 1},
    {C2 + C1, C1, 0, 1}, {C1, C1, 0, 1},      {C1, CP, 0, 0}};
constexpr int NL = FDLBM_UNET_LAYERS;

size_t wcount(const Layer &l) { return (size_t)l.co * 27 * l.ci; }

}  // namespace

struct fdlbm_unet {
  int R = 0, nmax = 0, cin = 0, nout = 0;
  hipStream_t stream = nullptr;
  std::string err;
  size_t nparam = 0, woff[NL]{}, boff[NL]{};  // offsets (floats) of W and b in the parameter vector
  size_t bwoff[NL]{};                         // offsets (bf16) of each layer's W / WT copies
  char *ws = nullptr;
  size_t total = 0;
  // workspace offsets (bytes)
  size_t o_p = 0, o_g = 0, o_m = 0, o_v = 0, o_w = 0, o_wt = 0, o_loss = 0;
  size_t o_red = 0;  // per-block partials of the fixed-order reductions
  size_t o_in = 0, o_a[NL]{}, o_p1 = 0, o_p2 = 0, o_c1 = 0, o_c2 = 0, o_out = 0;
  size_t o_gout = 0, o_ga[NL]{}, o_gc1 = 0, o_gc2 = 0, o_gp1 = 0, o_gp2 = 0, o_gb = 0;
  int64_t t_adam = 0;
  bool bound = false, have_params = false;
};

static int uerr(fdlbm_unet *u, int code, const char *fmt, ...) {
  if (u) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    u->err = buf;
  }
  return code;
}

#define UCHK(u, call)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) return uerr(u, FDLBM_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

static size_t npos(const fdlbm_unet *u, int level, int n) {
  const size_t r = (size_t)(u->R >> level);
  return (size_t)n * r * r * r;
}

int fdlbm_unet_create(int R, int n_max, int cin, int nout, void *hip_stream, fdlbm_unet **out) {
  if (!out) return FDLBM_E_INVALID;
  *out = nullptr;
  if (R < 16 || R % 4 || R > 256 || n_max < 1 || cin < 1 || cin > CP || nout < 1 || nout > CP)
    return FDLBM_E_INVALID;
  auto *u = new fdlbm_unet;
  u->R = R;
  u->nmax = n_max;
  u->cin = cin;
  u->nout = nout;
  u->stream = (hipStream_t)hip_stream;
  size_t p = 0, bw = 0;
  for (int l = 0; l < NL; ++l) {
    u->woff[l] = p;
    p += wcount(LAYERS[l]);
    u->boff[l] = p;
    p += LAYERS[l].co;
    u->bwoff[l] = bw;
    bw += wcount(LAYERS[l]);
  }
  u->nparam = p;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  const int n = n_max;
  u->o_p = take(p * 4);
  u->o_g = take(p * 4);
  u->o_m = take(p * 4);
  u->o_v = take(p * 4);
  u->o_w = take(bw * 2);
  u->o_wt = take(bw * 2);
  u->o_loss = take(8);
  {
    // the largest partial set of any reduction (they run one after another
    // on the network's stream and share the region)
    size_t red = (size_t)unet::LOSS_BLOCKS * 8;
    for (int l = 0; l < NL; ++l) {
      const Layer &L = LAYERS[l];
      const int Rl = R >> L.level;
      red = std::max(red, (size_t)unet::wgrad_chunks(Rl, n_max) * wcount(L) * 4);
      red = std::max(red, (size_t)unet::act_bwd_blocks(npos(u, L.level, n_max) * L.co, L.co) * L.co * 4);
    }
    u->o_red = take(red);
  }
  u->o_in = take(npos(u, 0, n) * CP * 2);
  for (int l = 0; l < NL - 1; ++l) u->o_a[l] = take(npos(u, LAYERS[l].level, n) * LAYERS[l].co * 2);
  u->o_p1 = take(npos(u, 1, n) * C1 * 2);
  u->o_p2 = take(npos(u, 2, n) * C2 * 2);
  u->o_c2 = take(npos(u, 1, n) * (C3 + C2) * 2);
  u->o_c1 = take(npos(u, 0, n) * (C2 + C1) * 2);
  u->o_out = take(npos(u, 0, n) * CP * 4);
  u->o_gout = take(npos(u, 0, n) * CP * 4);
  for (int l = 0; l < NL - 1; ++l) u->o_ga[l] = take(npos(u, LAYERS[l].level, n) * LAYERS[l].co * 4);
  u->o_gc1 = take(npos(u, 0, n) * (C2 + C1) * 4);
  u->o_gc2 = take(npos(u, 1, n) * (C3 + C2) * 4);
  u->o_gp1 = take(npos(u, 1, n) * C1 * 4);
  u->o_gp2 = take(npos(u, 2, n) * C2 * 4);
  u->o_gb = take(npos(u, 0, n) * CP * 2);  // largest pre-activation gradient (bf16)
  u->total = off;
  *out = u;
  return FDLBM_OK;
}

void fdlbm_unet_destroy(fdlbm_unet *u) { delete u; }

const char *fdlbm_unet_last_error(const fdlbm_unet *u) { return u ? u->err.c_str() : "null network"; }

int fdlbm_unet_param_count(const fdlbm_unet *u, size_t *n) {
  if (!u || !n) return FDLBM_E_INVALID;
  *n = u->nparam;
  return FDLBM_OK;
}

int fdlbm_unet_workspace_bytes(const fdlbm_unet *u, size_t *bytes) {
  if (!u || !bytes) return FDLBM_E_INVALID;
  *bytes = u->total;
  return FDLBM_OK;
}

int fdlbm_unet_bind_workspace(fdlbm_unet *u, void *dev, size_t bytes) {
  if (!u) return FDLBM_E_INVALID;
  if (!dev || ((uintptr_t)dev & 255u) || bytes < u->total)
    return uerr(u, FDLBM_E_ALIGN, "workspace must be >= %zu bytes and 256-byte aligned", u->total);
  u->ws = (char *)dev;
  u->bound = true;
  u->have_params = false;
  return FDLBM_OK;
}

template <typename T>
static T *at(fdlbm_unet *u, size_t off) {
  return reinterpret_cast<T *>(u->ws + off);
}

// bf16 copies of the weights (and the flipped transposes for the backward pass)
static int refresh_weights(fdlbm_unet *u) {
  for (int l = 0; l < NL; ++l)
    UCHK(u, unet::wcast(at<float>(u, u->o_p) + u->woff[l], LAYERS[l].co, LAYERS[l].ci,
                        at<__bf16>(u, u->o_w) + u->bwoff[l], at<__bf16>(u, u->o_wt) + u->bwoff[l], u->stream));
  return FDLBM_OK;
}

int fdlbm_unet_set_params(fdlbm_unet *u, const float *host, size_t n) {
  if (!u || !host) return FDLBM_E_INVALID;
  if (!u->bound) return uerr(u, FDLBM_E_STATE, "bind the workspace first");
  if (n != u->nparam) return uerr(u, FDLBM_E_INVALID, "expected %zu parameters", u->nparam);
  UCHK(u, hipMemcpyAsync(u->ws + u->o_p, host, n * 4, hipMemcpyHostToDevice, u->stream));
  UCHK(u, hipMemsetAsync(u->ws + u->o_m, 0, n * 4, u->stream));
  UCHK(u, hipMemsetAsync(u->ws + u->o_v, 0, n * 4, u->stream));
  const int rc = refresh_weights(u);
  if (rc != FDLBM_OK) return rc;
  UCHK(u, hipStreamSynchronize(u->stream));
  u->t_adam = 0;
  u->have_params = true;
  return FDLBM_OK;
}

int fdlbm_unet_get_params(fdlbm_unet *u, float *host, size_t n) {
  if (!u || !host) return FDLBM_E_INVALID;
  if (!u->have_params) return uerr(u, FDLBM_E_STATE, "no parameters set");
  if (n != u->nparam) return uerr(u, FDLBM_E_INVALID, "expected %zu parameters", u->nparam);
  UCHK(u, hipMemcpyAsync(host, u->ws + u->o_p, n * 4, hipMemcpyDeviceToHost, u->stream));
  UCHK(u, hipStreamSynchronize(u->stream));
  return FDLBM_OK;
}

static int check_call(fdlbm_unet *u, int n) {
  if (!u->bound || !u->have_params) return uerr(u, FDLBM_E_STATE, "bind the workspace and set parameters first");
  if (n < 1 || n > u->nmax) return uerr(u, FDLBM_E_INVALID, "sample count must be in 1..%d", u->nmax);
  return FDLBM_OK;
}

// forward pass of n samples; the activations stay in the workspace
static int forward(fdlbm_unet *u, const float *x, int n) {
  hipStream_t st = u->stream;
  const int R = u->R, r1 = R / 2, r2 = R / 4;
  auto A = [&](int l) { return at<__bf16>(u, u->o_a[l]); };
  auto Wl = [&](int l) { return at<__bf16>(u, u->o_w) + u->bwoff[l]; };
  auto Bl = [&](int l) { return at<float>(u, u->o_p) + u->boff[l]; };
  auto conv = [&](int l, const __bf16 *in, void *out, int mode) {
    const Layer &L = LAYERS[l];
    return unet::conv(in, L.ci, Wl(l), Bl(l), L.co, R >> L.level, n, mode, L.relu, out, st);
  };
  UCHK(u, unet::input(x, u->cin, CP, npos(u, 0, n), at<__bf16>(u, u->o_in), st));
  UCHK(u, conv(0, at<__bf16>(u, u->o_in), A(0), 0));
  UCHK(u, conv(1, A(0), A(1), 0));
  UCHK(u, unet::pool(A(1), R, C1, n, at<__bf16>(u, u->o_p1), st));
  UCHK(u, conv(2, at<__bf16>(u, u->o_p1), A(2), 0));
  UCHK(u, conv(3, A(2), A(3), 0));
  UCHK(u, unet::pool(A(3), r1, C2, n, at<__bf16>(u, u->o_p2), st));
  UCHK(u, conv(4, at<__bf16>(u, u->o_p2), A(4), 0));
  UCHK(u, conv(5, A(4), A(5), 0));
  UCHK(u, unet::up(A(5), r2, C3, n, at<__bf16>(u, u->o_c2), C3 + C2, 0, st));
  UCHK(u, unet::copy_ch(A(3), C2, at<__bf16>(u, u->o_c2), C3 + C2, C3, npos(u, 1, n), st));
  UCHK(u, conv(6, at<__bf16>(u, u->o_c2), A(6), 0));
  UCHK(u, conv(7, A(6), A(7), 0));
  UCHK(u, unet::up(A(7), r1, C2, n, at<__bf16>(u, u->o_c1), C2 + C1, 0, st));
  UCHK(u, unet::copy_ch(A(1), C1, at<__bf16>(u, u->o_c1), C2 + C1, C2, npos(u, 0, n), st));
  UCHK(u, conv(8, at<__bf16>(u, u->o_c1), A(8), 0));
  UCHK(u, conv(9, A(8), A(9), 0));
  UCHK(u, conv(10, A(9), at<float>(u, u->o_out), 1));
  return FDLBM_OK;
}

// backward pass after forward(): parameter gradients into o_g (zeroed here)
static int backward(fdlbm_unet *u, int n) {
  hipStream_t st = u->stream;
  const int R = u->R, r1 = R / 2, r2 = R / 4;
  float *G = at<float>(u, u->o_g);
  __bf16 *gb = at<__bf16>(u, u->o_gb);
  UCHK(u, hipMemsetAsync(G, 0, u->nparam * 4, st));
  UCHK(u, hipMemsetAsync(u->ws + u->o_ga[1], 0, npos(u, 0, n) * C1 * 4, st));
  UCHK(u, hipMemsetAsync(u->ws + u->o_ga[3], 0, npos(u, 1, n) * C2 * 4, st));
  auto GA = [&](int l) { return at<float>(u, u->o_ga[l]); };
  auto A = [&](int l) { return at<__bf16>(u, u->o_a[l]); };
  // layer l: gradient of its output g (f32) -> bias and weight gradients and,
  // unless l == 0, the gradient of its input (f32) into gin
  auto layer_bwd = [&](int l, const float *g, const __bf16 *y, const __bf16 *in, float *gin) -> int {
    const Layer &L = LAYERS[l];
    const int Rl = R >> L.level;
    float *part = at<float>(u, u->o_red);
    UCHK(u, unet::act_bwd(g, L.relu ? y : nullptr, npos(u, L.level, n) * L.co, L.co, gb, G + u->boff[l], part,
                          st));
    UCHK(u, unet::wgrad(gb, L.co, in, L.ci, Rl, n, G + u->woff[l], part, st));
    if (gin)
      UCHK(u, unet::conv(gb, L.co, at<__bf16>(u, u->o_wt) + u->bwoff[l], nullptr, L.ci, Rl, n, 1, 0, gin, st));
    return FDLBM_OK;
  };
  int rc;
  if ((rc = layer_bwd(10, at<float>(u, u->o_gout), nullptr, A(9), GA(9)))) return rc;
  if ((rc = layer_bwd(9, GA(9), A(9), A(8), GA(8)))) return rc;
  if ((rc = layer_bwd(8, GA(8), A(8), at<__bf16>(u, u->o_c1), at<float>(u, u->o_gc1)))) return rc;
  UCHK(u, unet::up_bwd(at<float>(u, u->o_gc1), r1, C2, C2 + C1, 0, n, GA(7), st));
  UCHK(u, unet::copy_ch_bwd(at<float>(u, u->o_gc1), C1, C2 + C1, C2, npos(u, 0, n), GA(1), st));
  if ((rc = layer_bwd(7, GA(7), A(7), A(6), GA(6)))) return rc;
  if ((rc = layer_bwd(6, GA(6), A(6), at<__bf16>(u, u->o_c2), at<float>(u, u->o_gc2)))) return rc;
  UCHK(u, unet::up_bwd(at<float>(u, u->o_gc2), r2, C3, C3 + C2, 0, n, GA(5), st));
  UCHK(u, unet::copy_ch_bwd(at<float>(u, u->o_gc2), C2, C3 + C2, C3, npos(u, 1, n), GA(3), st));
  if ((rc = layer_bwd(5, GA(5), A(5), A(4), GA(4)))) return rc;
  if ((rc = layer_bwd(4, GA(4), A(4), at<__bf16>(u, u->o_p2), at<float>(u, u->o_gp2)))) return rc;
  UCHK(u, unet::pool_bwd(at<float>(u, u->o_gp2), r1, C2, n, GA(3), st));
  if ((rc = layer_bwd(3, GA(3), A(3), A(2), GA(2)))) return rc;
  if ((rc = layer_bwd(2, GA(2), A(2), at<__bf16>(u, u->o_p1), at<float>(u, u->o_gp1)))) return rc;
  UCHK(u, unet::pool_bwd(at<float>(u, u->o_gp1), R, C1, n, GA(1), st));
  if ((rc = layer_bwd(1, GA(1), A(1), A(0), GA(0)))) return rc;
  if ((rc = layer_bwd(0, GA(0), A(0), at<__bf16>(u, u->o_in), nullptr))) return rc;
  return FDLBM_OK;
}

static int loss_grad(fdlbm_unet *u, const float *t, const float *w, int n, double wsum, double *loss) {
  if (!(wsum > 0)) return uerr(u, FDLBM_E_INVALID, "the weight sum must be positive");
  UCHK(u, hipMemsetAsync(u->ws + u->o_loss, 0, 8, u->stream));
  UCHK(u, unet::loss(at<float>(u, u->o_out), CP, t, w, u->nout, npos(u, 0, n), 1.0 / wsum,
                     at<float>(u, u->o_gout), at<double>(u, u->o_loss), at<double>(u, u->o_red), u->stream));
  if (loss) {
    UCHK(u, hipMemcpyAsync(loss, u->ws + u->o_loss, 8, hipMemcpyDeviceToHost, u->stream));
    UCHK(u, hipStreamSynchronize(u->stream));
  }
  return FDLBM_OK;
}

int fdlbm_unet_forward(fdlbm_unet *u, const float *x, int n, float *y) {
  if (!u || !x || !y) return FDLBM_E_INVALID;
  int rc = check_call(u, n);
  if (rc) return rc;
  if ((rc = forward(u, x, n))) return rc;
  // the first nout channels of every position
  UCHK(u, hipMemcpy2DAsync(y, (size_t)u->nout * 4, u->ws + u->o_out, (size_t)CP * 4, (size_t)u->nout * 4,
                           npos(u, 0, n), hipMemcpyDeviceToDevice, u->stream));
  return FDLBM_OK;
}

int fdlbm_unet_gradient(fdlbm_unet *u, const float *x, const float *t, const float *w, int n, double wsum,
                        double *loss, float *grad_host) {
  if (!u || !x || !t || !w) return FDLBM_E_INVALID;
  int rc = check_call(u, n);
  if (rc) return rc;
  if ((rc = forward(u, x, n))) return rc;
  if ((rc = loss_grad(u, t, w, n, wsum, nullptr))) return rc;
  if ((rc = backward(u, n))) return rc;
  if (loss) UCHK(u, hipMemcpyAsync(loss, u->ws + u->o_loss, 8, hipMemcpyDeviceToHost, u->stream));
  if (grad_host) UCHK(u, hipMemcpyAsync(grad_host, u->ws + u->o_g, u->nparam * 4, hipMemcpyDeviceToHost, u->stream));
  UCHK(u, hipStreamSynchronize(u->stream));
  return FDLBM_OK;
}

int fdlbm_unet_train_step(fdlbm_unet *u, const float *x, const float *t, const float *w, int n, double wsum,
                          float lr, double *loss) {
  if (!u || !x || !t || !w || !(lr > 0)) return FDLBM_E_INVALID;
  int rc = check_call(u, n);
  if (rc) return rc;
  if ((rc = forward(u, x, n))) return rc;
  if ((rc = loss_grad(u, t, w, n, wsum, nullptr))) return rc;
  if ((rc = backward(u, n))) return rc;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  ++u->t_adam;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, (double)u->t_adam)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, (double)u->t_adam)));
  UCHK(u, unet::adam(at<float>(u, u->o_p), at<float>(u, u->o_m), at<float>(u, u->o_v), at<float>(u, u->o_g),
                     u->nparam, lr, b1, b2, eps, c1, c2, u->stream));
  if ((rc = refresh_weights(u))) return rc;
  if (loss) {
    UCHK(u, hipMemcpyAsync(loss, u->ws + u->o_loss, 8, hipMemcpyDeviceToHost, u->stream));
    UCHK(u, hipStreamSynchronize(u->stream));
  }
  return FDLBM_OK;
}
