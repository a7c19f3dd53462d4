// Host side of the learned preconditioner: the network object, its forward pass (used by
// flexible CG), the loss gradient, and an Adam trainer.  All arithmetic on lattice fields runs
// in the kernels of net.hip; the host only updates the few thousand weights.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <numeric>
#include <random>

#include "net.h"
#include "runtime.h"

using cplx = std::complex<double>;

struct stag_net_s {
  stag_lattice_s* lat = nullptr;
  int layers = 0;
  int channels = 0;
  bool herm = false;                         // second half of the layers = adjoints of the first half
  std::vector<int> ch;                       // ch[0] = 1, ch[L] = 1
  std::vector<std::vector<cplx>> w;          // per layer [9][cout][cin]
  stag::DevBuf wdev;                         // complex64 weights of all layers, then their adjoints
  std::vector<size_t> woff, aoff;            // float2 offsets per layer
  std::vector<stag::DevBuf> act;             // L+1 activations [2][ch][V/2][3] complex64
  std::vector<std::array<bool, 2>> nz;       // which parities of each activation are nonzero
  stag::DevBuf gbuf[2];                      // activation gradients [2][Cmax][V/2][3]
  stag::DevBuf partial;                      // weight-gradient partials
  stag::DevBuf gacc;                         // accumulated weight gradients, complex128, all layers
  stag::DevBuf lossbuf;                      // per-pair losses and norms
  stag::DevBuf vy, vt, vu;                   // FP64 even-site vectors of the residual loss
  std::vector<std::vector<double>> am, av;   // Adam moments per layer (re, im interleaved)
  long adam_t = 0;
  ~stag_net_s() {
    (void)hipDeviceSynchronize();
    wdev.release();
    for (auto& a : act) a.release();
    gbuf[0].release();
    gbuf[1].release();
    partial.release();
    gacc.release();
    lossbuf.release();
    vy.release();
    vt.release();
    vu.release();
  }
};

namespace stag {

namespace {

constexpr int kWgradBlocks = 240;

// adj(W)[d'][a][b] = conj(W[d][b][a]) with d' the opposite direction: the weights of the adjoint layer.
std::vector<cplx> adjoint_weights(const std::vector<cplx>& W, int ci, int co) {
  std::vector<cplx> A(W.size());
  for (int d = 0; d < 9; ++d) {
    const int dp = d == 0 ? 0 : (d <= 4 ? d + 4 : d - 4);
    for (int a = 0; a < ci; ++a)
      for (int b = 0; b < co; ++b) A[(dp * ci + a) * co + b] = std::conj(W[(d * co + b) * ci + a]);
  }
  return A;
}

void tie_weights(stag_net_s* n) {
  if (!n->herm) return;
  for (int l = 0; l < n->layers / 2; ++l)
    n->w[n->layers - 1 - l] = adjoint_weights(n->w[l], n->ch[l], n->ch[l + 1]);
}

int nweights(const stag_net_s* n, int l) { return 9 * n->ch[l] * n->ch[l + 1]; }

float2* wptr(stag_net_s* n, size_t off) { return reinterpret_cast<float2*>(n->wdev.ptr) + off; }

float2* act_par(stag_net_s* n, int l, int p) {
  const size_t per = (size_t)n->ch[l] * n->lat->g.half * 3;
  return reinterpret_cast<float2*>(n->act[l].ptr) + p * per;
}

float2* grad_par(stag_net_s* n, int which, int c, int p) {
  const size_t per = (size_t)c * n->lat->g.half * 3;
  return reinterpret_cast<float2*>(n->gbuf[which].ptr) + p * per;
}

hipError_t upload_weights(stag_net_s* n, hipStream_t st) {
  std::vector<float2> h;
  size_t total = 0;
  for (int l = 0; l < n->layers; ++l) total += 2 * nweights(n, l);
  h.resize(total);
  size_t off = 0;
  n->woff.assign(n->layers, 0);
  n->aoff.assign(n->layers, 0);
  for (int l = 0; l < n->layers; ++l) {
    n->woff[l] = off;
    for (int i = 0; i < nweights(n, l); ++i) h[off + i] = make_float2((float)n->w[l][i].real(), (float)n->w[l][i].imag());
    off += nweights(n, l);
  }
  for (int l = 0; l < n->layers; ++l) {
    n->aoff[l] = off;
    // adjoint layer (used by the backward pass): direction d' = opposite(d), weights W_d^H ([ci][co])
    const std::vector<cplx> A = adjoint_weights(n->w[l], n->ch[l], n->ch[l + 1]);
    for (int i = 0; i < nweights(n, l); ++i) h[off + i] = make_float2((float)A[i].real(), (float)A[i].imag());
    off += nweights(n, l);
  }
  hipError_t e = n->wdev.ensure(total * sizeof(float2));
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(n->wdev.ptr, h.data(), total * sizeof(float2), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

NetLayerArgs layer_args(stag_net_s* n, int p) {
  NetLayerArgs a{};
  a.g = n->lat->g;
  a.links = reinterpret_cast<const char*>(n->lat->links[P32][p].ptr);
  a.out_par = p;
  return a;
}

}  // namespace

stag_lattice_s* net_lattice(stag_net_s* n) { return n->lat; }

// Forward pass: in (device complex128 even vector) -> out (same), activations kept in n->act.
hipError_t net_forward(stag_net_s* n, const void* in, void* out, hipStream_t st) {
  const long half = n->lat->g.half;
  hipError_t e = launch_net_embed(in, act_par(n, 0, 0), half, st);
  if (e != hipSuccess) return e;
  n->nz.assign(n->layers + 1, {false, false});
  n->nz[0] = {true, false};
  for (int l = 0; l < n->layers; ++l) {
    const bool last = l == n->layers - 1;
    for (int p = 0; p < (last ? 1 : 2); ++p) {
      NetLayerArgs a = layer_args(n, p);
      a.in_same = n->nz[l][p] ? act_par(n, l, p) : nullptr;
      a.in_other = n->nz[l][1 - p] ? act_par(n, l, 1 - p) : nullptr;
      if (!a.in_same && !a.in_other) continue;
      a.out = act_par(n, l + 1, p);
      a.w = wptr(n, n->woff[l]);
      e = launch_net_layer(a, n->ch[l], n->ch[l + 1], st);
      if (e != hipSuccess) return e;
      n->nz[l + 1][p] = true;
    }
  }
  if (!out) return hipSuccess;
  if (!n->nz[n->layers][0]) return hipMemsetAsync(out, 0, (size_t)half * 48, st);
  return launch_net_extract(act_par(n, n->layers, 0), out, half, st);
}

// Loss and weight gradients of one pair, accumulated into n->gacc (complex128 dL/dconj W); loss to *loss_dev.
// Output gradient of the loss for one pair and the unscaled loss numerator in *loss_dev:
//   kind 0: g = (N(b) - x) / |x|^2,            *loss_dev = |N(b) - x|^2            (inv = 1/|x|^2)
//   kind 1: g = M (M N(b) - b) / |b|^2,        *loss_dev = |M N(b) - b|^2          (inv = 1/|b|^2)
// (M Hermitian, so the gradient of |M y - b|^2 with respect to conj(y) is M (M y - b)).
hipError_t net_backward_pair(stag_net_s* n, const void* b, const void* x, double inv, int kind, double mass,
                             double* loss_dev, hipStream_t st) {
  const long half = n->lat->g.half;
  hipError_t e = net_forward(n, b, kind == 1 ? n->vy.ptr : nullptr, st);
  if (e != hipSuccess) return e;
  int cur = 0;
  std::array<bool, 2> gnz = {true, false};
  double* part = reinterpret_cast<double*>(n->partial.ptr);
  if (kind == 0) {
    e = launch_net_loss(act_par(n, n->layers, 0), x, inv, grad_par(n, cur, 1, 0), part, loss_dev, half, st);
    if (e != hipSuccess) return e;
  } else {
    if (stag_apply_m(n->lat, &mass, n->vy.ptr, n->vu.ptr, 1, st) != STAG_OK) return hipErrorUnknown;
    e = launch_sub_norm(n->vu.ptr, b, n->vt.ptr, part, loss_dev, half, st);
    if (e != hipSuccess) return e;
    if (stag_apply_m(n->lat, &mass, n->vt.ptr, n->vu.ptr, 1, st) != STAG_OK) return hipErrorUnknown;
    e = launch_scale_to_f32(n->vu.ptr, inv, grad_par(n, cur, 1, 0), half, st);
    if (e != hipSuccess) return e;
  }
  size_t goff = 0;
  std::vector<size_t> gofs(n->layers);
  for (int l = 0; l < n->layers; ++l) {
    gofs[l] = goff;
    goff += 2 * (size_t)nweights(n, l);
  }
  for (int l = n->layers - 1; l >= 0; --l) {
    const int ci = n->ch[l], co = n->ch[l + 1];
    for (int p = 0; p < 2; ++p) {
      NetLayerArgs a = layer_args(n, p);
      a.in_same = n->nz[l][p] ? act_par(n, l, p) : nullptr;
      a.in_other = n->nz[l][1 - p] ? act_par(n, l, 1 - p) : nullptr;
      const float2* gy = gnz[p] ? grad_par(n, cur, co, p) : nullptr;
      e = launch_net_wgrad(a, gy, part, ci, co, kWgradBlocks, st);
      if (e != hipSuccess) return e;
    }
    e = launch_net_wgrad_reduce(part, ci, co, kWgradBlocks, 2, reinterpret_cast<double*>(n->gacc.ptr) + gofs[l], st);
    if (e != hipSuccess) return e;
    if (l == 0) break;
    std::array<bool, 2> nnz = {false, false};
    for (int p = 0; p < 2; ++p) {
      NetLayerArgs a = layer_args(n, p);
      a.in_same = gnz[p] ? grad_par(n, cur, co, p) : nullptr;
      a.in_other = gnz[1 - p] ? grad_par(n, cur, co, 1 - p) : nullptr;
      if (!a.in_same && !a.in_other) continue;
      a.out = grad_par(n, 1 - cur, ci, p);
      a.w = wptr(n, n->aoff[l]);
      e = launch_net_layer(a, co, ci, st);
      if (e != hipSuccess) return e;
      nnz[p] = true;
    }
    gnz = nnz;
    cur = 1 - cur;
  }
  return hipSuccess;
}

size_t net_grad_count(const stag_net_s* n) {
  size_t t = 0;
  for (int l = 0; l < n->layers; ++l) t += 2 * (size_t)nweights(n, l);
  return t;
}

}  // namespace stag

using namespace stag;

namespace {

stag_status net_arg(const char* m) {
  set_error(m);
  return STAG_ERR_ARG;
}

}  // namespace

// The transports read the lattice's FP32 links at every launch: they must still be loaded (a later
// stag_load_links may have dropped them), and the lattice's device must be current.
stag_status stag::net_check(stag_net_s* n) {
  const stag_lattice_s* lat = n->lat;
  if (!lat->loaded || !(lat->built & STAG_PREC_BIT(STAG_F32)) || !lat->links[P32][0].ptr) {
    set_error("the network transports need the lattice's FP32 links: load them with STAG_PREC_BIT(STAG_F32)");
    return STAG_ERR_STATE;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != lat->device) return net_arg("the current HIP device is not the lattice's device");
  return STAG_OK;
}

namespace {

hipError_t net_alloc(stag_net_s* n) {
  const size_t half = n->lat->g.half;
  const int cmax = *std::max_element(n->ch.begin(), n->ch.end());
  n->act.resize(n->layers + 1);
  for (int l = 0; l <= n->layers; ++l) {
    hipError_t e = n->act[l].ensure(2 * (size_t)n->ch[l] * half * 3 * sizeof(float2));
    if (e != hipSuccess) return e;
  }
  for (int i = 0; i < 2; ++i) {
    hipError_t e = n->gbuf[i].ensure(2 * (size_t)cmax * half * 3 * sizeof(float2));
    if (e != hipSuccess) return e;
  }
  hipError_t e = n->partial.ensure(std::max<size_t>(2 * 9 * (size_t)cmax * cmax * kWgradBlocks * 2,
                                                    (half * 3 + 255) / 256) * sizeof(double));
  if (e != hipSuccess) return e;
  e = n->gacc.ensure(net_grad_count(n) * sizeof(double));
  if (e != hipSuccess) return e;
  e = n->vy.ensure(half * 48);
  if (e == hipSuccess) e = n->vt.ensure(half * 48);
  if (e == hipSuccess) e = n->vu.ensure(half * 48);
  if (e != hipSuccess) return e;
  return n->lossbuf.ensure(64 * sizeof(double));
}

void zero_adam(stag_net_s* n) {
  n->am.assign(n->layers, {});
  n->av.assign(n->layers, {});
  for (int l = 0; l < n->layers; ++l) {
    n->am[l].assign(2 * 9 * n->ch[l] * n->ch[l + 1], 0.0);
    n->av[l].assign(2 * 9 * n->ch[l] * n->ch[l + 1], 0.0);
  }
  n->adam_t = 0;
}

// L = sum_i ||N(b_i) - x_i||^2 / ||x_i||^2 over the pairs idx; gradients accumulated in n->gacc.
stag_status loss_grad(stag_net_s* n, const char* b, const char* x, const std::vector<int>& idx, int kind,
                      double mass, double* loss, hipStream_t st) {
  const long half = n->lat->g.half;
  const size_t vb = (size_t)half * 48;
  double* lb = reinterpret_cast<double*>(n->lossbuf.ptr);
  double* part = reinterpret_cast<double*>(n->partial.ptr);
  double total = 0.0;
  for (int i : idx) {
    double nx = 0.0;
    STAG_HIP_TRY(launch_norm2_c128((kind == 0 ? x : b) + i * vb, part, lb + 8, half, st));
    STAG_HIP_TRY(hipMemcpyAsync(&nx, lb + 8, sizeof(double), hipMemcpyDeviceToHost, st));
    STAG_HIP_TRY(hipStreamSynchronize(st));
    if (!(nx > 0.0)) {
      set_error("a training vector (x for the solution loss, b for the residual loss) is zero");
      return STAG_ERR_ARG;
    }
    hipError_t e = net_backward_pair(n, b + i * vb, x + i * vb, 1.0 / nx, kind, mass, lb, st);
    if (e == hipErrorUnknown) return STAG_ERR_HIP;  // stag_apply_m failed and set the message
    STAG_HIP_TRY(e);
    double l2 = 0.0;
    STAG_HIP_TRY(hipMemcpyAsync(&l2, lb, sizeof(double), hipMemcpyDeviceToHost, st));
    STAG_HIP_TRY(hipStreamSynchronize(st));
    total += l2 / nx;
  }
  *loss = total;
  return STAG_OK;
}

}  // namespace

// No exception may cross the C ABI.
#define STAG_NET_GUARD_BEGIN try {
#define STAG_NET_GUARD_END                                    \
  }                                                           \
  catch (const std::bad_alloc&) {                             \
    set_error("host allocation failed");                      \
    return STAG_ERR_NOMEM;                                    \
  }                                                           \
  catch (const std::exception& ex) {                          \
    set_error(std::string("internal error: ") + ex.what());   \
    return STAG_ERR_STATE;                                    \
  }

extern "C" {

stag_status stag_net_create(stag_lattice_t lat, int32_t layers, int32_t channels, uint32_t flags, uint64_t seed,
                            stag_net_t* out) {
  try {
    if (!lat || !out) return net_arg("lattice and out must not be NULL");
    *out = nullptr;
    if (layers < 1 || layers > 16) return net_arg("layers must be in [1, 16]");
    if (flags & ~STAG_NET_HERMITIAN) return net_arg("unknown network flags");
    if ((flags & STAG_NET_HERMITIAN) && (layers % 2)) return net_arg("a Hermitian network needs an even layer count");
    if (channels != 1 && channels != 2 && channels != 4 && channels != 8) return net_arg("channels must be 1, 2, 4 or 8");
    if (!lat->loaded || !(lat->built & STAG_PREC_BIT(STAG_F32))) {
      set_error("the network transports need FP32 links: call stag_load_links with STAG_PREC_BIT(STAG_F32)");
      return STAG_ERR_STATE;
    }
    auto* n = new stag_net_s();
    n->lat = lat;
    n->layers = layers;
    n->channels = channels;
    n->herm = (flags & STAG_NET_HERMITIAN) != 0;
    n->ch.assign(layers + 1, channels);
    n->ch.front() = 1;
    n->ch.back() = 1;
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd;
    n->w.resize(layers);
    for (int l = 0; l < layers; ++l) {
      const double s = 0.1 / std::sqrt(9.0 * n->ch[l]);
      n->w[l].resize(9 * n->ch[l] * n->ch[l + 1]);
      for (auto& v : n->w[l]) v = cplx(s * nd(rng), s * nd(rng));
    }
    tie_weights(n);
    hipError_t e = net_alloc(n);
    if (e == hipSuccess) e = upload_weights(n, nullptr);
    if (e != hipSuccess) {
      set_error(std::string("network allocation: ") + hipGetErrorString(e));
      delete n;
      return STAG_ERR_HIP;
    }
    zero_adam(n);
    *out = n;
    return STAG_OK;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return STAG_ERR_NOMEM;
  }
}

stag_status stag_net_destroy(stag_net_t net) {
  STAG_NET_GUARD_BEGIN
  if (!net) return net_arg("network is NULL");
  delete net;
  return STAG_OK;
  STAG_NET_GUARD_END
}

stag_status stag_net_num_weights(stag_net_t net, int64_t* n_complex) {
  if (!net || !n_complex) return net_arg("network and n_complex must not be NULL");
  int64_t t = 0;
  for (int l = 0; l < net->layers; ++l) t += nweights(net, l);
  *n_complex = t;
  return STAG_OK;
}

stag_status stag_net_set_weights(stag_net_t net, const double* w, int64_t n_complex) {
  STAG_NET_GUARD_BEGIN
  if (!net || !w) return net_arg("network and weights must not be NULL");
  int64_t t = 0;
  for (int l = 0; l < net->layers; ++l) t += nweights(net, l);
  if (n_complex != t) return net_arg("weight count does not match the network");
  for (int64_t i = 0; i < 2 * t; ++i)
    if (!std::isfinite(w[i])) return net_arg("weights must be finite");
  int64_t k = 0;
  for (int l = 0; l < net->layers; ++l)
    for (auto& v : net->w[l]) {
      v = cplx(w[2 * k], w[2 * k + 1]);
      ++k;
    }
  tie_weights(net);
  STAG_HIP_TRY(upload_weights(net, nullptr));
  zero_adam(net);
  return STAG_OK;
  STAG_NET_GUARD_END
}

stag_status stag_net_get_weights(stag_net_t net, double* w, int64_t n_complex) {
  STAG_NET_GUARD_BEGIN
  if (!net || !w) return net_arg("network and weights must not be NULL");
  int64_t t = 0;
  for (int l = 0; l < net->layers; ++l) t += nweights(net, l);
  if (n_complex != t) return net_arg("weight count does not match the network");
  int64_t k = 0;
  for (int l = 0; l < net->layers; ++l)
    for (const auto& v : net->w[l]) {
      w[2 * k] = v.real();
      w[2 * k + 1] = v.imag();
      ++k;
    }
  return STAG_OK;
  STAG_NET_GUARD_END
}

stag_status stag_net_apply(stag_net_t net, const void* in, void* out, int32_t nrhs, void* stream) {
  STAG_NET_GUARD_BEGIN
  if (!net || !in || !out) return net_arg("network, in and out must not be NULL");
  if (in == out) return net_arg("in and out must not overlap");
  if (nrhs < 1) return net_arg("nrhs must be >= 1");
  stag_status s = net_check(net);
  if (s != STAG_OK) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const size_t vb = (size_t)net->lat->g.half * 48;
  for (int r = 0; r < nrhs; ++r)
    STAG_HIP_TRY(net_forward(net, reinterpret_cast<const char*>(in) + r * vb, reinterpret_cast<char*>(out) + r * vb, st));
  return STAG_OK;
  STAG_NET_GUARD_END
}

stag_status stag_net_loss_grad(stag_net_t net, const void* b, const void* x, int32_t npairs, int32_t loss_kind,
                               double mass, double* loss, double* grad, void* stream) {
  STAG_NET_GUARD_BEGIN
  if (!net || !b || !x || !loss) return net_arg("network, b, x and loss must not be NULL");
  if (npairs < 1) return net_arg("npairs must be >= 1");
  if (loss_kind != 0 && loss_kind != 1) return net_arg("loss_kind must be 0 or 1");
  if (!std::isfinite(mass)) return net_arg("mass must be finite");
  if (loss_kind == 1 && !(net->lat->built & STAG_PREC_BIT(STAG_F64))) return net_arg("the residual loss needs FP64 links");
  {
    const stag_status c = net_check(net);
    if (c != STAG_OK) return c;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const size_t ng = net_grad_count(net);
  STAG_HIP_TRY(hipMemsetAsync(net->gacc.ptr, 0, ng * sizeof(double), st));
  std::vector<int> idx(npairs);
  std::iota(idx.begin(), idx.end(), 0);
  stag_status s = loss_grad(net, reinterpret_cast<const char*>(b), reinterpret_cast<const char*>(x), idx, loss_kind,
                            mass, loss, st);
  if (s != STAG_OK) return s;
  if (grad) {
    STAG_HIP_TRY(hipMemcpyAsync(grad, net->gacc.ptr, ng * sizeof(double), hipMemcpyDeviceToHost, st));
    STAG_HIP_TRY(hipStreamSynchronize(st));
  }
  return STAG_OK;
  STAG_NET_GUARD_END
}

void stag_train_params_default(stag_train_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->epochs = 10;
  p->batch = 8;
  p->lr = 1e-3;
  p->beta1 = 0.9;
  p->beta2 = 0.999;
  p->eps = 1e-8;
  p->seed = 1;
  p->loss_kind = 1;
  p->mass = 0.0;
}

stag_status stag_net_train(stag_net_t net, const void* b, const void* x, int32_t npairs, const stag_train_params* prm_in,
                           stag_train_info* info, void* stream) {
  STAG_NET_GUARD_BEGIN
  const auto t0 = std::chrono::steady_clock::now();
  if (!net || !b || !x) return net_arg("network, b and x must not be NULL");
  if (npairs < 1) return net_arg("npairs must be >= 1");
  stag_train_params prm;
  if (prm_in) prm = *prm_in; else stag_train_params_default(&prm);
  if (prm.epochs < 1 || prm.batch < 1 || !(prm.lr > 0.0) || !(prm.beta1 >= 0.0 && prm.beta1 < 1.0) ||
      !(prm.beta2 >= 0.0 && prm.beta2 < 1.0) || !(prm.eps > 0.0) || (prm.loss_kind != 0 && prm.loss_kind != 1) ||
      !std::isfinite(prm.mass))
    return net_arg("invalid training parameters");
  {
    const stag_status c = net_check(net);
    if (c != STAG_OK) return c;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const size_t ng = net_grad_count(net);
  std::vector<double> g(ng);
  std::vector<int> order(npairs);
  std::iota(order.begin(), order.end(), 0);
  std::mt19937_64 rng(prm.seed);
  double first = 0.0, last = 0.0;
  int steps = 0;
  for (int ep = 0; ep < prm.epochs; ++ep) {
    std::shuffle(order.begin(), order.end(), rng);
    double ep_loss = 0.0;
    for (int s0 = 0; s0 < npairs; s0 += prm.batch) {
      std::vector<int> idx(order.begin() + s0, order.begin() + std::min(npairs, s0 + prm.batch));
      STAG_HIP_TRY(hipMemsetAsync(net->gacc.ptr, 0, ng * sizeof(double), st));
      double l = 0.0;
      stag_status s = loss_grad(net, reinterpret_cast<const char*>(b), reinterpret_cast<const char*>(x), idx,
                                prm.loss_kind, prm.mass, &l, st);
      if (s != STAG_OK) return s;
      ep_loss += l;
      STAG_HIP_TRY(hipMemcpyAsync(g.data(), net->gacc.ptr, ng * sizeof(double), hipMemcpyDeviceToHost, st));
      STAG_HIP_TRY(hipStreamSynchronize(st));
      // tied layers: W_{L-1-l} = adj(W_l), so dL/dconj(W_l)[d][b][a] gains conj(dL/dconj(W_{L-1-l})[d'][a][b])
      std::vector<size_t> goff(net->layers + 1, 0);
      for (int li = 0; li < net->layers; ++li) goff[li + 1] = goff[li] + 2 * (size_t)nweights(net, li);
      if (net->herm)
        for (int li = 0; li < net->layers / 2; ++li) {
          const int lt = net->layers - 1 - li;
          const int ci = net->ch[li], co = net->ch[li + 1];
          for (int d = 0; d < 9; ++d) {
            const int dp = d == 0 ? 0 : (d <= 4 ? d + 4 : d - 4);
            for (int b = 0; b < co; ++b)
              for (int a = 0; a < ci; ++a) {
                const size_t i0 = goff[li] + 2 * (size_t)((d * co + b) * ci + a);
                const size_t i1 = goff[lt] + 2 * (size_t)((dp * ci + a) * co + b);
                g[i0] += g[i1];
                g[i0 + 1] -= g[i1 + 1];
              }
          }
        }
      // Adam on (Re W, Im W): d L / d(Re, Im) = 2 (Re, Im) of d L / d conj W, averaged over the batch
      net->adam_t += 1;
      const double b1t = 1.0 - std::pow(prm.beta1, (double)net->adam_t);
      const double b2t = 1.0 - std::pow(prm.beta2, (double)net->adam_t);
      const int free_layers = net->herm ? net->layers / 2 : net->layers;
      for (int li = 0; li < free_layers; ++li) {
        size_t k = goff[li];
        for (size_t j = 0; j < net->w[li].size(); ++j) {
          double pr[2] = {net->w[li][j].real(), net->w[li][j].imag()};
          for (int c = 0; c < 2; ++c, ++k) {
            const double gr = 2.0 * g[k] / idx.size();
            double& m = net->am[li][2 * j + c];
            double& v = net->av[li][2 * j + c];
            m = prm.beta1 * m + (1.0 - prm.beta1) * gr;
            v = prm.beta2 * v + (1.0 - prm.beta2) * gr * gr;
            pr[c] -= prm.lr * (m / b1t) / (std::sqrt(v / b2t) + prm.eps);
          }
          net->w[li][j] = cplx(pr[0], pr[1]);
        }
      }
      tie_weights(net);
      STAG_HIP_TRY(upload_weights(net, st));
      ++steps;
    }
    ep_loss /= npairs;
    if (ep == 0) first = ep_loss;
    last = ep_loss;
    if (!std::isfinite(ep_loss)) {
      set_error("training loss is not finite");
      return STAG_ERR_NAN;
    }
  }
  if (info) {
    info->loss_first = first;
    info->loss_last = last;
    info->epochs = prm.epochs;
    info->steps = steps;
    info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return STAG_OK;
  STAG_NET_GUARD_END
}

}  // extern "C"
