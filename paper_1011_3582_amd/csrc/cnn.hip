// C ABI of the warm-start network: workspace layout, the per-layer implicit-GEMM launches
// of the forward pass, the backward pass and Adam, and the warm-start transform.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <new>

#include "cnn.hpp"
#include "fftlb.h"
#include "fftlb_cnn.h"

using namespace fftlb::cnn;

static_assert(kParams == FFTLB_CNN_PARAMS, "parameter count of the header");

namespace {

thread_local char g_cnn_error[256] = "";

size_t align_up(size_t v) { return (v + 255) / 256 * 256; }

struct CnnLayout {
  size_t theta, grad, m, v, z[kLayers], a[kLayers], dz[kLayers], y, x, wpart, part, sums, total;
};

// Pixels per K chunk of the weight-gradient GEMM (each chunk of each sample writes one
// partial gradient).
constexpr int kWChunk = 1024;

// Output size of layer l for an h x w input.
void layer_out(int l, int h, int w, int* ho, int* wo) {
  int H = h, W = w;
  for (int i = 0; i <= l; ++i) {
    if (kKind[i] == KIND_S2) H /= 2, W /= 2;
    if (kKind[i] == KIND_UP) H *= 2, W *= 2;
  }
  *ho = H;
  *wo = W;
}

CnnLayout make_layout(int h, int w, int nmax) {
  CnnLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.theta = take(kParams * sizeof(float));
  L.grad = take(kParams * sizeof(float));
  L.m = take(kParams * sizeof(float));
  L.v = take(kParams * sizeof(float));
  for (int l = 0; l < kLayers; ++l) {
    int ho, wo;
    layer_out(l, h, w, &ho, &wo);
    const size_t bytes = (size_t)nmax * kCout[l] * ho * wo * sizeof(float);
    L.z[l] = take(bytes);
    L.a[l] = l < kLayers - 1 ? take(bytes) : 0;
    L.dz[l] = take(bytes);
  }
  L.y = take((size_t)nmax * 2 * h * w * sizeof(float));
  L.x = take((size_t)3 * h * w * sizeof(float));
  size_t wp = 0;  // largest per-layer set of weight-gradient partials
  for (int l = 0; l < kLayers; ++l) {
    int ho, wo;
    layer_out(l, h, w, &ho, &wo);
    const size_t chunks = ((size_t)ho * wo + kWChunk - 1) / kWChunk;
    wp = std::max(wp, (size_t)nmax * chunks * kCout[l] * (kCin[l] * 9 + 1));
  }
  L.wpart = take(wp * sizeof(float));
  L.part = take((size_t)kWsMaxBlocks * kWsSums * sizeof(double));
  L.sums = take(8 * sizeof(double));
  L.total = o;
  return L;
}

bool shape_ok(int h, int w, int nmax) {
  return h >= 8 && w >= 8 && h <= 4096 && w <= 4096 && h % 4 == 0 && w % 4 == 0 && nmax >= 1 && nmax <= 4096;
}

template <class Pb>
int launch_gemm(const Pb& pb, int M, int N, int Z, hipStream_t s) {
  hipLaunchKernelGGL(k_gemm<Pb>, dim3((N + 255) / 256, (M + 31) / 32, Z), dim3(256), 0, s, pb);
  return hipGetLastError() == hipSuccess ? FFTLB_OK : FFTLB_EHIP;
}

int grid_for(long count) { return (int)std::min<long>(4096, (count + 255) / 256); }

// Grid of the kernels that write per-block partial sums (at most kWsMaxBlocks blocks).
int sum_grid(long count) { return (int)std::min<long>(kWsMaxBlocks, (count + 255) / 256); }

}  // namespace

struct fftlb_cnn {
  int h, w, nmax, device;
  CnnLayout L;
  char* ws;
  float* theta;
  float* grad;
  float* m;
  float* v;
  double* sums;   // [0] sum of squared errors; warm start: M0, M, sum w, sum T, M after the shift
  double* part;   // per-block partial sums
  float* wpart;   // weight-gradient partials
  int adam_t;
  int have_grad;
  float* ptr(size_t off) const { return reinterpret_cast<float*>(ws + off); }
  Geom geom(int l) const {
    int hi = h, wi = w, ho, wo;
    if (l > 0) layer_out(l - 1, h, w, &hi, &wi);
    layer_out(l, h, w, &ho, &wo);
    return Geom{kCin[l], kCout[l], hi, wi, ho, wo, kKind[l]};
  }
};

namespace {

// Forward pass of n samples of x [n][3][h][w]; output [n][2][h][w] into the internal y.
int forward(fftlb_cnn* c, const float* x, int n, hipStream_t s) {
  const float* in = x;
  long in_stride = 3L * c->h * c->w;
  for (int l = 0; l < kLayers; ++l) {
    const Geom g = c->geom(l);
    const long P = (long)g.hout * g.wout;
    FwdProblem pb{};
    pb.g = g;
    pb.X = in;
    pb.W = c->theta + param_offset(l);
    pb.bias = pb.W + (long)g.cout * g.cin * 9;
    pb.Z = c->ptr(c->L.z[l]);
    pb.A = l < kLayers - 1 ? c->ptr(c->L.a[l]) : nullptr;
    pb.resid = l == kLayers - 1 ? x : nullptr;
    pb.Y = l == kLayers - 1 ? c->ptr(c->L.y) : nullptr;
    pb.xs = in_stride;
    pb.zs = g.cout * P;
    pb.rs = 3L * c->h * c->w;
    if (launch_gemm(pb, g.cout, (int)P, n, s)) return FFTLB_EHIP;
    in = pb.A;
    in_stride = pb.zs;
  }
  return FFTLB_OK;
}

// Backward pass after forward(): loss, dL/dZ of every layer and the parameter gradient.
int backward(fftlb_cnn* c, const float* x, const float* target, int n, hipStream_t s) {
  const long out_count = (long)n * 2 * c->h * c->w;
  const int mse_blocks = sum_grid(out_count);
  hipLaunchKernelGGL(k_mse, dim3(mse_blocks), dim3(256), 0, s, c->ptr(c->L.y), target,
                     c->ptr(c->L.dz[kLayers - 1]), out_count, c->part);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, c->part, mse_blocks, 1, 1, c->sums);
  for (int l = kLayers - 1; l >= 0; --l) {
    const Geom g = c->geom(l);
    const long P = (long)g.hout * g.wout;
    const float* X = l == 0 ? x : c->ptr(c->L.a[l - 1]);
    const long xs = l == 0 ? 3L * c->h * c->w : (long)g.cin * g.hin * g.win;
    WGradProblem wg{};
    wg.g = g;
    wg.X = X;
    wg.dZ = c->ptr(c->L.dz[l]);
    wg.part = c->wpart;
    wg.xs = xs;
    wg.zs = g.cout * P;
    wg.chunk = kWChunk;
    wg.nchunks = (int)((P + wg.chunk - 1) / wg.chunk);
    const int ncol = g.cin * 9 + 1;
    if (launch_gemm(wg, g.cout, ncol, n * wg.nchunks, s)) return FFTLB_EHIP;
    float* dW = c->grad + param_offset(l);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((g.cout * ncol + 63) / 64), dim3(256), 0, s, c->wpart,
                       n * wg.nchunks, g.cout, ncol, dW, dW + (long)g.cout * g.cin * 9);
    if (l == 0) break;
    BwdDataProblem bd{};
    bd.g = g;
    bd.W = c->theta + param_offset(l);
    bd.dZ = c->ptr(c->L.dz[l]);
    bd.Zprev = c->ptr(c->L.z[l - 1]);
    bd.dZprev = c->ptr(c->L.dz[l - 1]);
    bd.zs = g.cout * P;
    bd.ps = (long)g.cin * g.hin * g.win;
    if (launch_gemm(bd, g.cin, g.hin * g.win, n, s)) return FFTLB_EHIP;
  }
  return FFTLB_OK;
}

__global__ void k_mean(const double* sse, double count, double* out) { *out = *sse / count; }

int check(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    std::snprintf(g_cnn_error, sizeof g_cnn_error, "%s: %s", what, hipGetErrorString(e));
    return FFTLB_EHIP;
  }
  return FFTLB_OK;
}

// The warm-start transform of a prediction pred [2][h][w] (normalised density and
// temperature) into rho_out, T_out (see fftlb_cnn_project); the network input buffer holds
// the filter's intermediate and then the interface weights.
int project(fftlb_cnn* c, const float* pred, const float* rho0, float rho_c, float T_c, float rho_max, float* rho_out,
            float* T_out, hipStream_t s) {
  const long P = (long)c->h * c->w;
  const int G = sum_grid(P);
  float* tmp = c->ptr(c->L.x);
  const float rmin = 1e-3f * rho_c;
  hipLaunchKernelGGL(k_ws_clip, dim3(G), dim3(256), 0, s, pred, rho_out, P, rho_c, rmin, rho_max);
  hipLaunchKernelGGL(k_ws_smooth_x, dim3(G), dim3(256), 0, s, rho_out, tmp, c->h, c->w);
  hipLaunchKernelGGL(k_ws_smooth_y, dim3(G), dim3(256), 0, s, tmp, rho_out, c->h, c->w);
  hipLaunchKernelGGL(k_ws_weights, dim3(G), dim3(256), 0, s, rho0, rho_out, pred + P, tmp, c->h, c->w, T_c, c->part);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, c->part, G, kWsSums, 4, c->sums);
  hipLaunchKernelGGL(k_ws_shift, dim3(G), dim3(256), 0, s, rho_out, tmp, P, rmin, rho_max, c->sums, c->part);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, c->part, G, kWsSums, 1, c->sums + 4);
  hipLaunchKernelGGL(k_ws_finish, dim3(G), dim3(256), 0, s, rho_out, T_out, P, 1e-2f * T_c, c->sums);
  return check("cnn warm-start transform");
}

}  // namespace

extern "C" {

int fftlb_cnn_workspace_bytes(int32_t h, int32_t w, int32_t max_batch, size_t* bytes) {
  if (!bytes || !shape_ok(h, w, max_batch)) return FFTLB_EINVAL;
  *bytes = make_layout(h, w, max_batch).total;
  return FFTLB_OK;
}

int fftlb_cnn_create(int32_t h, int32_t w, int32_t max_batch, void* workspace, size_t ws_bytes, const float* params,
                     void* stream, fftlb_cnn** out) {
  if (!out) return FFTLB_EINVAL;
  *out = nullptr;
  if (!shape_ok(h, w, max_batch) || !params) return FFTLB_EINVAL;
  const CnnLayout L = make_layout(h, w, max_batch);
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 || ws_bytes < L.total) return FFTLB_ENOSPC;
  fftlb_cnn* c = new (std::nothrow) fftlb_cnn();
  if (!c) return FFTLB_EINVAL;
  c->h = h;
  c->w = w;
  c->nmax = max_batch;
  c->L = L;
  c->ws = static_cast<char*>(workspace);
  c->theta = c->ptr(L.theta);
  c->grad = c->ptr(L.grad);
  c->m = c->ptr(L.m);
  c->v = c->ptr(L.v);
  c->sums = reinterpret_cast<double*>(c->ws + L.sums);
  c->part = reinterpret_cast<double*>(c->ws + L.part);
  c->wpart = c->ptr(L.wpart);
  c->adam_t = 0;
  c->have_grad = 0;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return FFTLB_EHIP;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(c->theta, params, kParams * sizeof(float), hipMemcpyDeviceToDevice, s) != hipSuccess) {
    delete c;
    return FFTLB_EHIP;
  }
  hipLaunchKernelGGL(k_fill, dim3(grid_for(kParams)), dim3(256), 0, s, c->m, (long)kParams, 0.0f);
  hipLaunchKernelGGL(k_fill, dim3(grid_for(kParams)), dim3(256), 0, s, c->v, (long)kParams, 0.0f);
  if (check("cnn create")) {
    delete c;
    return FFTLB_EHIP;
  }
  *out = c;
  return FFTLB_OK;
}

int fftlb_cnn_forward(fftlb_cnn* c, const float* x, float* y, int32_t n, void* stream) {
  if (!c || !x || n < 1 || n > c->nmax) return FFTLB_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (forward(c, x, n, s)) return check("cnn forward");
  if (y && hipMemcpyAsync(y, c->ptr(c->L.y), (size_t)n * 2 * c->h * c->w * sizeof(float), hipMemcpyDeviceToDevice,
                          s) != hipSuccess)
    return FFTLB_EHIP;
  return check("cnn forward");
}

int fftlb_cnn_gradient(fftlb_cnn* c, const float* x, const float* target, int32_t n, float* grad, double* loss,
                       void* stream) {
  if (!c || !x || !target || n < 1 || n > c->nmax) return FFTLB_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (forward(c, x, n, s) || backward(c, x, target, n, s)) return check("cnn gradient");
  if (loss) hipLaunchKernelGGL(k_mean, dim3(1), dim3(1), 0, s, c->sums, (double)n * 2 * c->h * c->w, loss);
  if (grad && hipMemcpyAsync(grad, c->grad, kParams * sizeof(float), hipMemcpyDeviceToDevice, s) != hipSuccess)
    return FFTLB_EHIP;
  c->have_grad = 1;
  return check("cnn gradient");
}

int fftlb_cnn_adam_step(fftlb_cnn* c, float lr, void* stream) {
  if (!c || !c->have_grad || !(lr > 0.0f)) return FFTLB_EINVAL;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  c->adam_t += 1;
  const float bc1 = (float)(1.0 - std::pow(0.9, c->adam_t));
  const float bc2 = (float)(1.0 - std::pow(0.999, c->adam_t));
  hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                     c->theta, c->grad, c->m, c->v, kParams, lr, b1, b2, eps, bc1, bc2);
  return check("cnn adam");
}

int fftlb_cnn_get_params(const fftlb_cnn* c, float* params, void* stream) {
  if (!c || !params) return FFTLB_EINVAL;
  return hipMemcpyAsync(params, c->theta, kParams * sizeof(float), hipMemcpyDeviceToDevice,
                        reinterpret_cast<hipStream_t>(stream)) == hipSuccess
             ? FFTLB_OK
             : FFTLB_EHIP;
}

int fftlb_cnn_set_params(fftlb_cnn* c, const float* params, void* stream) {
  if (!c || !params) return FFTLB_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(c->theta, params, kParams * sizeof(float), hipMemcpyDeviceToDevice, s) != hipSuccess)
    return FFTLB_EHIP;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(kParams)), dim3(256), 0, s, c->m, (long)kParams, 0.0f);
  hipLaunchKernelGGL(k_fill, dim3(grid_for(kParams)), dim3(256), 0, s, c->v, (long)kParams, 0.0f);
  c->adam_t = 0;
  c->have_grad = 0;
  return check("cnn set params");
}

int fftlb_cnn_read_buffer(const fftlb_cnn* c, int32_t layer, int32_t kind, float* dst, size_t count,
                          void* stream) {
  if (!c || !dst || layer < 1 || layer > kLayers || kind < 0 || kind > 2) return FFTLB_EINVAL;
  const int l = layer - 1;
  int ho, wo;
  layer_out(l, c->h, c->w, &ho, &wo);
  const size_t cap = (size_t)c->nmax * (l == kLayers - 1 && kind == 2 ? 2 : kCout[l]) * ho * wo;
  if (count > cap) return FFTLB_EINVAL;
  const float* src = kind == 0 ? c->ptr(c->L.z[l])
                     : kind == 1 ? c->ptr(c->L.dz[l])
                                 : (l == kLayers - 1 ? c->ptr(c->L.y) : c->ptr(c->L.a[l]));
  return hipMemcpyAsync(dst, src, count * sizeof(float), hipMemcpyDeviceToDevice,
                        reinterpret_cast<hipStream_t>(stream)) == hipSuccess
             ? FFTLB_OK
             : FFTLB_EHIP;
}

int fftlb_cnn_project(fftlb_cnn* c, const float* pred, const float* rho0, float rho_c, float T_c, float rho_max,
                      float* rho_out, float* T_out, void* stream) {
  if (!c || !pred || !rho0 || !rho_out || !T_out || !(rho_c > 0.0f) || !(T_c > 0.0f) || !(rho_max > 1e-3f * rho_c))
    return FFTLB_EINVAL;
  return project(c, pred, rho0, rho_c, T_c, rho_max, rho_out, T_out, reinterpret_cast<hipStream_t>(stream));
}

int fftlb_cnn_warm_start(fftlb_cnn* c, const float* rho0, const float* T0, float T_target, float rho_c, float T_c,
                         float rho_max, float* rho_out, float* T_out, void* stream) {
  if (!c || !rho0 || !T0 || !rho_out || !T_out || !(rho_c > 0.0f) || !(T_c > 0.0f) || !(T_target > 0.0f) ||
      !(rho_max > 1e-3f * rho_c))
    return FFTLB_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const long P = (long)c->h * c->w;
  float* x = c->ptr(c->L.x);
  hipLaunchKernelGGL(k_ws_input, dim3(grid_for(P)), dim3(256), 0, s, rho0, T0, x, P, 1.0f / rho_c, 1.0f / T_c,
                     T_target / T_c);
  if (forward(c, x, 1, s)) return check("cnn warm start");
  return project(c, c->ptr(c->L.y), rho0, rho_c, T_c, rho_max, rho_out, T_out, s);
}

int fftlb_cnn_destroy(fftlb_cnn* c) {
  if (!c) return FFTLB_EINVAL;
  delete c;
  return FFTLB_OK;
}

}  // extern "C"
