// netio.h -- glue between an instance and the warm-start network (gfx950):
// per-node input features from the solver's own data, training targets from a
// solution, and the lift of a prediction to an initial guess x0.
#pragma once
#include "common.h"

namespace smg {

struct NetNorm {
  float mean[3], std[3];   // normalization of the three predicted fields
};

// feat[k][x][0..3] on an H x H grid (H >= n, zero beyond the instance's nodes):
//   mean_j and standard deviation over samples of the node log-coefficient
//   l_j = (log kW + log kE + log kS + log kN) / 4,
//   the target state y_d = f_Y,0 / c_0 and log10(nu) + 4, nu = g / h^2.
__global__ void k_net_features(int n, int N, int H, const double* __restrict__ kx, const double* __restrict__ ky,
                               const double* __restrict__ fY, double inv_c0, float lognu4,
                               float* __restrict__ feat) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= H * H) return;
  const int k = i / H, x = i - k * H;
  float* o = feat + (size_t)i * 4;
  if (k >= n || x >= n) { o[0] = 0.f; o[1] = 0.f; o[2] = 0.f; o[3] = 0.f; return; }
  const size_t node = (size_t)k * n + x;
  const size_t kxb = ((size_t)k * (n + 1) + x) * N, kyb = node * N, rowN = (size_t)n * N;
  double s = 0.0, s2 = 0.0;
  for (int j = 0; j < N; ++j) {
    const double l = 0.25 * ((log(kx[kxb + j]) + log(kx[kxb + N + j])) + (log(ky[kyb + j]) + log(ky[kyb + rowN + j])));
    s += l;
    s2 += l * l;
  }
  const double mean = s / N;
  const double var = fmax(s2 / N - mean * mean, 0.0);
  o[0] = (float)mean;
  o[1] = (float)sqrt(var);
  o[2] = (float)(fY[node * N] * inv_c0);
  o[3] = lognu4;
}

// tgt[k][x][0..2] = normalized (u, mean_j y_j, mean_j p_j); zero beyond the nodes.
__global__ void k_net_targets(int n, int N, int H, const double* __restrict__ xv, NetNorm nm,
                              float* __restrict__ tgt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= H * H) return;
  const int k = i / H, x = i - k * H;
  float* o = tgt + (size_t)i * 3;
  if (k >= n || x >= n) { o[0] = 0.f; o[1] = 0.f; o[2] = 0.f; return; }
  const size_t nn = (size_t)n * n, node = (size_t)k * n + x;
  double sy = 0.0, sp = 0.0;
  for (int j = 0; j < N; ++j) {
    sy += xv[node * N + j];
    sp += xv[(size_t)(N + 1) * nn + node * N + j];
  }
  const double v[3] = {xv[(size_t)N * nn + node], sy / N, sp / N};
  for (int c = 0; c < 3; ++c) o[c] = (float)((v[c] - nm.mean[c]) / nm.std[c]);
}

// x0: y_j = ybar, p_j = pbar for every sample, u = u, from the normalized prediction.
__global__ void k_net_lift(int n, int N, int H, const float* __restrict__ pred, NetNorm nm, double* __restrict__ x0) {
  const size_t nn = (size_t)n * n;
  const size_t tot = nn * N;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
    const size_t node = t / N;
    const int j = (int)(t - node * N);
    const int k = (int)(node / n), x = (int)(node - (size_t)k * n);
    const float* q = pred + ((size_t)k * H + x) * 3;
    x0[node * N + j] = (double)(q[1] * nm.std[1] + nm.mean[1]);
    x0[(size_t)(N + 1) * nn + node * N + j] = (double)(q[2] * nm.std[2] + nm.mean[2]);
    if (j == 0) x0[(size_t)N * nn + node] = (double)(q[0] * nm.std[0] + nm.mean[0]);
  }
}

}  // namespace smg
