// net.hip -- the warm-start network: a 4-level convolutional encoder-decoder
// (about 165k parameters) that maps per-node statistics of an instance to a
// prediction of (u, mean_j y_j, mean_j p_j).  Forward, backward and Adam run in
// the kernels of net.h (BF16 matrix cores, FP32 accumulation); the master
// weights, their gradients and the Adam moments are FP32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/smg.h"
#include "net.h"

using namespace smgnet;

namespace {

struct Layer {
  int cin, cout, taps, stride, up, skip, act;
};

// encoder 16/32/48/48 channels at H, H/2, H/4, H/8; decoder by nearest
// upsampling + 3x3 convolution with additive skips; 1x1 output to 3 channels
const Layer kArch[] = {
    {4, 16, 9, 1, 0, -1, 1},  {16, 16, 9, 1, 0, -1, 1}, {16, 32, 9, 2, 0, -1, 1}, {32, 32, 9, 1, 0, -1, 1},
    {32, 48, 9, 2, 0, -1, 1}, {48, 48, 9, 1, 0, -1, 1}, {48, 48, 9, 2, 0, -1, 1}, {48, 48, 9, 1, 0, -1, 1},
    {48, 48, 9, 1, 1, 5, 1},  {48, 48, 9, 1, 0, -1, 1}, {48, 32, 9, 1, 1, 3, 1},  {32, 32, 9, 1, 0, -1, 1},
    {32, 16, 9, 1, 1, 1, 1},  {16, 16, 9, 1, 0, -1, 1}, {16, 3, 1, 1, 0, -1, 0},
};
constexpr int kLayers = sizeof(kArch) / sizeof(kArch[0]);

int coutp(int c) { return (c + 3) & ~3; }

size_t param_count() {
  size_t s = 0;
  for (const auto& l : kArch) s += (size_t)l.cout * l.taps * l.cin + l.cout;
  return s;
}

}  // namespace

struct smg_net {
  int B = 0, H = 0;
  hipStream_t stream = nullptr;
  std::string err;
  size_t np = 0;
  float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  uint16_t* xin = nullptr;
  size_t woff[kLayers], boff[kLayers];
  uint16_t* W16[kLayers];
  uint16_t* WT[kLayers];
  float* z[kLayers];
  uint16_t* a[kLayers];
  float* dA[kLayers];
  int Hout[kLayers], Hin[kLayers];
  float* dz32 = nullptr;
  uint16_t* dz16 = nullptr;
  float* wpart = nullptr;
  size_t wpart_len = 0;
  float* lpart = nullptr;
  float* lossd = nullptr;
  int adam_t = 0;
  float* host = nullptr;
};

namespace {

constexpr int kChunk = 4096;      // output pixels per weight-gradient partial
constexpr int kLossBlocks = 512;

struct NCarver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

size_t net_plan(int B, int H, smg_net* N, void* base) {
  NCarver cv{(char*)base};
  N->np = param_count();
  N->theta = cv.take<float>(N->np);
  N->grad = cv.take<float>(N->np);
  N->m = cv.take<float>(N->np);
  N->v = cv.take<float>(N->np);
  N->xin = cv.take<uint16_t>((size_t)B * H * H * 4);
  size_t o = 0, maxpc = 0, maxwp = 0;
  int h = H;
  for (int l = 0; l < kLayers; ++l) {
    const Layer& L = kArch[l];
    N->Hin[l] = h;
    const int ho = L.up ? 2 * h : (h + L.stride - 1) / L.stride;
    N->Hout[l] = ho;
    h = ho;
    const size_t K = (size_t)L.taps * L.cin;
    N->woff[l] = o;
    o += L.cout * K;
    N->boff[l] = o;
    o += L.cout;
    N->W16[l] = cv.take<uint16_t>(L.cout * K);
    N->WT[l] = cv.take<uint16_t>(coutp(L.cout) * K);
    const size_t P = (size_t)B * ho * ho;
    N->z[l] = cv.take<float>(P * L.cout);
    N->a[l] = cv.take<uint16_t>(P * L.cout);
    N->dA[l] = cv.take<float>(P * L.cout);
    maxpc = std::max(maxpc, P * coutp(L.cout));
    const size_t nch = (P + kChunk - 1) / kChunk;
    maxwp = std::max(maxwp, nch * L.cout * K);
  }
  N->dz32 = cv.take<float>(maxpc);
  N->dz16 = cv.take<uint16_t>(maxpc);
  N->wpart = cv.take<float>(maxwp);
  N->wpart_len = maxwp;
  N->lpart = cv.take<float>(kLossBlocks);
  N->lossd = cv.take<float>(1);
  return cv.off + 256;
}

ConvGeom geom(const smg_net* N, int l) {
  const Layer& L = kArch[l];
  ConvGeom g;
  g.B = N->B; g.Hin = N->Hin[l]; g.Win = N->Hin[l]; g.Hout = N->Hout[l]; g.Wout = N->Hout[l];
  g.Cin = L.cin; g.Cout = L.cout; g.CoutP = coutp(L.cout); g.taps = L.taps; g.stride = L.stride; g.up = L.up;
  return g;
}

int gridn(size_t n) {
  size_t b = (n + 255) / 256;
  return (int)std::max<size_t>(1, std::min<size_t>(b, 8192));
}

#define NHIP(call)                                                          \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      N->err = std::string(#call) + ": " + hipGetErrorString(e_);           \
      return SMG_EHIP;                                                      \
    }                                                                       \
  } while (0)

int cast_weights(smg_net* N) {
  for (int l = 0; l < kLayers; ++l) {
    const Layer& L = kArch[l];
    const int tot = coutp(L.cout) * L.taps * L.cin;
    hipLaunchKernelGGL(k_cast_weights, dim3(gridn(tot)), dim3(256), 0, N->stream, L.cout, coutp(L.cout), L.taps,
                       L.cin, (const float*)(N->theta + N->woff[l]), N->W16[l], N->WT[l]);
  }
  NHIP(hipGetLastError());
  return SMG_OK;
}

int forward(smg_net* N, const float* x) {
  const size_t nin = (size_t)N->B * N->H * N->H * 4;
  hipLaunchKernelGGL(k_f32_to_bf16, dim3(gridn(nin)), dim3(256), 0, N->stream, nin, x, N->xin);
  for (int l = 0; l < kLayers; ++l) {
    const Layer& L = kArch[l];
    const ConvGeom g = geom(N, l);
    const size_t P = (size_t)g.B * g.Hout * g.Wout;
    const int waves = (int)((P + 15) / 16);
    const int blocks = (waves + 3) / 4;
    const uint16_t* in = l == 0 ? N->xin : N->a[l - 1];
    const uint16_t* skip = L.skip >= 0 ? N->a[L.skip] : nullptr;
    hipLaunchKernelGGL(k_conv_fwd, dim3(blocks), dim3(kNetBlock), 0, N->stream, g, in,
                       (const uint16_t*)N->W16[l], (const float*)(N->theta + N->boff[l]), skip, L.act, N->z[l],
                       N->a[l]);
  }
  NHIP(hipGetLastError());
  return SMG_OK;
}

// loss (device, in N->lossd) and d loss / d theta into N->grad
int backward(smg_net* N, const float* target, int valid) {
  for (int l = 0; l < kLayers; ++l) {
    const size_t P = (size_t)N->B * N->Hout[l] * N->Hout[l];
    hipLaunchKernelGGL(k_fillf, dim3(gridn(P * kArch[l].cout)), dim3(256), 0, N->stream, P * kArch[l].cout,
                       N->dA[l], 0.f);
  }
  const int last = kLayers - 1;
  const float cnt = (float)N->B * valid * valid * 3.f;
  hipLaunchKernelGGL(k_mse, dim3(kLossBlocks), dim3(kNetBlock), 0, N->stream, N->B, N->H, valid,
                     (const float*)N->z[last], target, 1.f / cnt, N->dA[last], N->lpart);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, N->stream, kLossBlocks, (const float*)N->lpart,
                     1.f / cnt, N->lossd);
  for (int l = last; l >= 0; --l) {
    const Layer& L = kArch[l];
    const ConvGeom g = geom(N, l);
    const int P = g.B * g.Hout * g.Wout;
    hipLaunchKernelGGL(k_silu_bwd, dim3(gridn((size_t)P * g.CoutP)), dim3(256), 0, N->stream, P, L.cout, g.CoutP,
                       L.act, (const float*)N->dA[l], (const float*)N->z[l], N->dz32, N->dz16,
                       L.skip >= 0 ? N->dA[L.skip] : (float*)nullptr);
    const int K = L.taps * L.cin;
    const int nch = (P + kChunk - 1) / kChunk;
    const int waves = ((L.cout + 15) / 16) * ((K + 15) / 16) * nch;
    const uint16_t* in = l == 0 ? N->xin : N->a[l - 1];
    hipLaunchKernelGGL(k_conv_bwd_weight, dim3((waves + 3) / 4), dim3(kNetBlock), 0, N->stream, g, in,
                       (const uint16_t*)N->dz16, kChunk, nch, N->wpart);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(gridn((size_t)L.cout * K)), dim3(256), 0, N->stream, L.cout, K, nch,
                       (const float*)N->wpart, N->grad + N->woff[l]);
    hipLaunchKernelGGL(k_bias_grad, dim3(L.cout), dim3(kNetBlock), 0, N->stream, P, L.cout,
                       (const float*)N->dz32, N->grad + N->boff[l]);
    if (l > 0) {
      const int Pin = g.B * g.Hin * g.Win;
      const int wv = (Pin + 15) / 16;
      hipLaunchKernelGGL(k_conv_bwd_data, dim3((wv + 3) / 4), dim3(kNetBlock), 0, N->stream, g,
                         (const uint16_t*)N->dz16, (const uint16_t*)N->WT[l], N->dA[l - 1]);
    }
  }
  NHIP(hipGetLastError());
  return SMG_OK;
}

}  // namespace

extern "C" {

int smg_net_param_count(void) { return (int)param_count(); }

size_t smg_net_workspace_bytes(int batch, int H) {
  if (batch < 1 || H < 8 || (H % 8) != 0) return 0;
  smg_net tmp;
  return net_plan(batch, H, &tmp, nullptr);
}

int smg_net_setup(int batch, int H, void* workspace, size_t bytes, void* stream, smg_net** out) {
  if (!out) return SMG_EINVAL;
  *out = nullptr;
  if (batch < 1 || H < 8 || (H % 8) != 0) return SMG_EINVAL;
  smg_net* N = new smg_net();
  N->B = batch;
  N->H = H;
  N->stream = (hipStream_t)stream;
  const size_t need = net_plan(batch, H, N, workspace);
  if (!workspace || bytes < need || ((uintptr_t)workspace & 255) != 0) { delete N; return SMG_EWORKSPACE; }
  if (hipHostMalloc((void**)&N->host, 64, hipHostMallocDefault) != hipSuccess) { delete N; return SMG_EHIP; }
  *out = N;
  return SMG_OK;
}

void smg_net_destroy(smg_net* N) {
  if (!N) return;
  if (N->host) (void)hipHostFree(N->host);
  delete N;
}

const char* smg_net_last_error(const smg_net* N) { return N ? N->err.c_str() : ""; }

int smg_net_set_params(smg_net* N, const float* theta) {
  if (!N || !theta) return SMG_EINVAL;
  NHIP(hipMemcpyAsync(N->theta, theta, N->np * sizeof(float), hipMemcpyDeviceToDevice, N->stream));
  hipLaunchKernelGGL(k_fillf, dim3(gridn(N->np)), dim3(256), 0, N->stream, N->np, N->m, 0.f);
  hipLaunchKernelGGL(k_fillf, dim3(gridn(N->np)), dim3(256), 0, N->stream, N->np, N->v, 0.f);
  N->adam_t = 0;
  return cast_weights(N);
}

int smg_net_get_params(smg_net* N, float* theta) {
  if (!N || !theta) return SMG_EINVAL;
  NHIP(hipMemcpyAsync(theta, N->theta, N->np * sizeof(float), hipMemcpyDeviceToDevice, N->stream));
  return SMG_OK;
}

int smg_net_forward(smg_net* N, const float* x, float* out) {
  if (!N || !x || !out) return SMG_EINVAL;
  int rc = forward(N, x);
  if (rc != SMG_OK) return rc;
  const size_t n = (size_t)N->B * N->H * N->H * 3;
  NHIP(hipMemcpyAsync(out, N->z[kLayers - 1], n * sizeof(float), hipMemcpyDeviceToDevice, N->stream));
  return SMG_OK;
}

int smg_net_grad(smg_net* N, const float* x, const float* target, int valid, float* grad, float* loss) {
  if (!N || !x || !target || valid < 1 || valid > N->H) return SMG_EINVAL;
  int rc = forward(N, x);
  if (rc == SMG_OK) rc = backward(N, target, valid);
  if (rc != SMG_OK) return rc;
  if (grad) NHIP(hipMemcpyAsync(grad, N->grad, N->np * sizeof(float), hipMemcpyDeviceToDevice, N->stream));
  if (loss) {
    NHIP(hipMemcpyAsync(N->host, N->lossd, sizeof(float), hipMemcpyDeviceToHost, N->stream));
    NHIP(hipStreamSynchronize(N->stream));
    *loss = N->host[0];
  }
  return SMG_OK;
}

int smg_net_train_step(smg_net* N, const float* x, const float* target, int valid, float lr, float* loss) {
  if (!N || !x || !target || valid < 1 || valid > N->H || !(lr > 0.f)) return SMG_EINVAL;
  int rc = forward(N, x);
  if (rc == SMG_OK) rc = backward(N, target, valid);
  if (rc != SMG_OK) return rc;
  N->adam_t += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - std::pow(b1, (float)N->adam_t), c2 = 1.f - std::pow(b2, (float)N->adam_t);
  hipLaunchKernelGGL(k_adam, dim3(gridn(N->np)), dim3(256), 0, N->stream, N->np, N->theta, (const float*)N->grad,
                     N->m, N->v, lr, b1, b2, eps, c1, c2);
  NHIP(hipGetLastError());
  rc = cast_weights(N);
  if (rc != SMG_OK) return rc;
  if (loss) {
    NHIP(hipMemcpyAsync(N->host, N->lossd, sizeof(float), hipMemcpyDeviceToHost, N->stream));
    NHIP(hipStreamSynchronize(N->stream));
    *loss = N->host[0];
  }
  return SMG_OK;
}

}  // extern "C"
