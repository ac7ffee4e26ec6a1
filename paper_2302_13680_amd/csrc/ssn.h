// ssn.h -- pointwise kernels of the semismooth Newton method for the control
// problem with an L^1 penalty and box constraints (Section 5, Algorithm 2).
//
// Vectors in the node layout (Y block [n][n][N], U block [n][n], P block
// [n][n][N]); the adjoint is carried rescaled by the sample weights, so
// E[p] = sum_j zeta_j p_j is the plain sum of the P block's samples at a node.
#pragma once
#include "common.h"

namespace smg {

constexpr int kSsnGammas = 8;          // step lengths priced by one merit pass
constexpr int kSsnMeritBlocks = 1024;  // grid of the merit pass (at most)

struct SsnArgs {
  double nu, beta;
  double nub, nua;   // nu b, nu a (infinite for a missing bound)
};

// F(u) of the discrete optimality condition (Section 5): u minus 1/nu times the
// sum of the four clipped terms, in the printed order.
__device__ __forceinline__ double ssn_F(double u, double w, const SsnArgs& a) {
  const double s = ((fmax(0.0, w - a.beta) + fmin(0.0, w + a.beta)) - fmax(0.0, (w - a.beta) - a.nub)) -
                   fmin(0.0, (w + a.beta) - a.nua);
  return u - s / a.nu;
}

// Indicator of I+ u I- (eq. activesets).
__device__ __forceinline__ double ssn_active(double w, const SsnArgs& a) {
  const double wp = w - a.beta, wm = w + a.beta;
  return ((wp >= 0.0 && wp <= a.nub) || (wm >= a.nua && wm <= 0.0)) ? 1.0 : 0.0;
}

// Per node (W lanes, JM samples per lane): w = sum_j p~_j of x's P block; when
// F is given also F(u, w), the active-set indicator chi, -mass F into rU (if
// given: the U block of the Newton right-hand side) and per-block sums of F^2
// into partials[blockIdx.x].
template <int W, int JM>
__global__ __launch_bounds__(kBlock) void k_ssn_eval(int nn, int N, const double* __restrict__ x, SsnArgs a,
                                                     double mass, double* __restrict__ w, double* __restrict__ F,
                                                     double* __restrict__ chi, double* __restrict__ rU,
                                                     double* __restrict__ partials) {
  const int lane = threadIdx.x & (W - 1);
  const int slot = group_slot<W>(blockIdx.x);
  double s = 0.0;
  if (slot < nn) {
    const double* p = x + (size_t)(N + 1) * nn + (size_t)slot * N;
#pragma unroll
    for (int q = 0; q < JM; ++q) {
      const int j = lane + q * W;
      s += j < N ? p[j] : 0.0;
    }
  }
  s = group_sum<W>(s);
  double f2[1] = {0.0};
  if (slot < nn && lane == 0) {
    w[slot] = s;
    if (F) {
      const double Fv = ssn_F(x[(size_t)N * nn + slot], s, a);
      F[slot] = Fv;
      chi[slot] = ssn_active(s, a);
      if (rU) rU[slot] = -mass * Fv;
      f2[0] = Fv * Fv;
    }
  }
  if (partials) {
    block_sum<1>(f2);
    if (threadIdx.x == 0) partials[blockIdx.x] = f2[0];
  }
}

struct SsnGammas {
  double g[kSsnGammas];
};

// Per-block sums of F(u + g du, w + g dw)^2 for ng <= kSsnGammas step lengths g
// (the line search of Algorithm 2: E[p] is affine in u, so the trial E[p] is
// w + g dw).  partials[blockIdx.x][q]; grid-stride over the nn nodes.
__global__ __launch_bounds__(kBlock) void k_ssn_merit(int nn, const double* __restrict__ u,
                                                      const double* __restrict__ du, const double* __restrict__ w,
                                                      const double* __restrict__ dw, SsnArgs a, SsnGammas G, int ng,
                                                      double* __restrict__ partials) {
  double acc[kSsnGammas];
#pragma unroll
  for (int q = 0; q < kSsnGammas; ++q) acc[q] = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < nn; i += gridDim.x * kBlock) {
    const double ui = u[i], dui = du[i], wi = w[i], dwi = dw[i];
#pragma unroll
    for (int q = 0; q < kSsnGammas; ++q) {
      if (q < ng) {
        const double Fv = ssn_F(ui + G.g[q] * dui, wi + G.g[q] * dwi, a);
        acc[q] += Fv * Fv;
      }
    }
  }
  block_sum<kSsnGammas>(acc);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kSsnGammas; ++q) partials[(size_t)blockIdx.x * kSsnGammas + q] = acc[q];
  }
}

// x += g dx over len values.
__global__ __launch_bounds__(kBlock) void k_axpy(size_t len, double* __restrict__ x, double g,
                                                 const double* __restrict__ dx) {
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < len; i += (size_t)gridDim.x * kBlock)
    x[i] += g * dx[i];
}

// U block of y: mass * u (the right-hand side that fixes u = u0 when D_j = 0).
__global__ __launch_bounds__(kBlock) void k_scale(int nn, const double* __restrict__ u, double mass,
                                                  double* __restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < nn) out[i] = mass * u[i];
}

}  // namespace smg
