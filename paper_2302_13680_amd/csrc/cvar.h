// cvar.h -- per-sample kernels of the risk-averse (smoothed CVaR) problem
// (Section 6, eq. discretized_nonlinearsystem and the Newton matrix
// eq. optmality_systeMmoothed_discretized).
//
// Y-block vectors are [n][n][N] (node-major, samples contiguous), so one pass
// over the nodes with a thread per sample reads every row coalesced.
#pragma once
#include "common.h"

namespace smg {

constexpr int kSampleBlocks = 240;   // node ranges of the per-sample reductions

// z_j = mass (y_j - y_d) on the domain (dom NULL: everywhere), 0 outside.
__global__ __launch_bounds__(kBlock) void k_cvar_z(int nn, int N, double mass, const double* __restrict__ Y,
                                                   const double* __restrict__ yd, const double* __restrict__ dom,
                                                   double* __restrict__ Z) {
  const size_t len = (size_t)nn * N;
  for (size_t k = blockIdx.x * (size_t)kBlock + threadIdx.x; k < len; k += (size_t)gridDim.x * kBlock) {
    const size_t i = k / N;
    Z[k] = (!dom || dom[i] != 0.0) ? mass * (Y[k] - yd[i]) : 0.0;
  }
}

// part[b][j] = sum over block b's node range of A_j(i) B_j(i).
__global__ __launch_bounds__(kBlock) void k_sample_dots(int nn, int N, const double* __restrict__ A,
                                                        const double* __restrict__ B, double* __restrict__ part) {
  const int per = (nn + gridDim.x - 1) / gridDim.x;
  const int i0 = blockIdx.x * per, i1 = min(nn, i0 + per);
  for (int j = threadIdx.x; j < N; j += kBlock) {
    double s = 0.0;
    for (int i = i0; i < i1; ++i) s += A[(size_t)i * N + j] * B[(size_t)i * N + j];
    part[(size_t)blockIdx.x * N + j] = s;
  }
}

// out_j = scale_j sum_b part[b][j] (scale NULL: 1).  A block takes 64
// samples; its 4 waves sum every fourth partial (independent loads in flight)
// and meet in LDS.
constexpr int kFinalizeSamples = 64;
__global__ __launch_bounds__(kBlock) void k_sample_finalize(int nb, int N, const double* __restrict__ part,
                                                            const double* __restrict__ scale,
                                                            double* __restrict__ out) {
  constexpr int kSlices = kBlock / kFinalizeSamples;
  __shared__ double acc[kSlices][kFinalizeSamples];
  const int jl = threadIdx.x % kFinalizeSamples, slice = threadIdx.x / kFinalizeSamples;
  const int j = blockIdx.x * kFinalizeSamples + jl;
  double s = 0.0;
  if (j < N) {
#pragma unroll 8
    for (int b = slice; b < nb; b += kSlices) s += part[(size_t)b * N + j];
  }
  acc[slice][jl] = s;
  __syncthreads();
  if (slice == 0 && j < N) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kSlices; ++q) t += acc[q][jl];
    out[j] = scale ? scale[j] * t : t;
  }
}

// Y_j += sign coef_j z_j (the rank-one terms w_j z_j (z_j . x_j) once coef_j =
// w_j (z_j . x_j)).
__global__ __launch_bounds__(kBlock) void k_lowrank_add(int nn, int N, double sign, const double* __restrict__ coef,
                                                        const double* __restrict__ Z, double* __restrict__ Y) {
  const size_t len = (size_t)nn * N;
  for (size_t k = blockIdx.x * (size_t)kBlock + threadIdx.x; k < len; k += (size_t)gridDim.x * kBlock)
    Y[k] += sign * coef[k % N] * Z[k];
}

// Y block of the right-hand side b(c) = [c_j y_d | f_U | f_P]: c_j y_d on the
// domain, 0 outside.
__global__ __launch_bounds__(kBlock) void k_cvar_rhs(int nn, int N, const double* __restrict__ c,
                                                     const double* __restrict__ yd, const double* __restrict__ dom,
                                                     double* __restrict__ fY) {
  const size_t len = (size_t)nn * N;
  for (size_t k = blockIdx.x * (size_t)kBlock + threadIdx.x; k < len; k += (size_t)gridDim.x * kBlock) {
    const size_t i = k / N;
    fY[k] = (!dom || dom[i] != 0.0) ? c[k % N] * yd[i] : 0.0;
  }
}

}  // namespace smg
