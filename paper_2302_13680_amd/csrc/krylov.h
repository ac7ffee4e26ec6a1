// krylov.h -- vector kernels of the Krylov and refinement drivers (gfx950).
#pragma once
#include "common.h"

namespace smg {

// ---------------------------------------------------------- vector kernels
template <typename TI, typename TO>
__global__ void k_convert(size_t len, const TI* __restrict__ in, TO* __restrict__ out) {
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < len; i += (size_t)gridDim.x * kBlock)
    out[i] = (TO)in[i];
}

template <typename T>
__global__ void k_fill(size_t len, T* __restrict__ p, T v) {
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < len; i += (size_t)gridDim.x * kBlock) p[i] = v;
}

// x += (double) d
template <typename TD>
__global__ void k_add(size_t len, double* __restrict__ x, const TD* __restrict__ d) {
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < len; i += (size_t)gridDim.x * kBlock)
    x[i] += (double)d[i];
}

// Block reduction of acc[0..nv) and acc[KM] (the squared-norm slot, when
// with_norm) into partials[blockIdx.x][i] and partials[blockIdx.x][kMaxBasis].
template <int KM>
__device__ __forceinline__ void store_block_partials(double (&acc)[KM + 1], int nv, int with_norm,
                                                     double* __restrict__ partials) {
  __shared__ double red[kBlock / 64][KM + 1];
  const int lane = threadIdx.x & 63, wvi = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i <= KM; ++i) {
    if (i < nv || (i == KM && with_norm)) {
      const double s = group_sum<64>(acc[i]);
      if (lane == 0) red[wvi][i] = s;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= KM; i += kBlock) {
    if (i < nv || (i == KM && with_norm)) {
      double s = red[0][i];
      for (int q = 1; q < kBlock / 64; ++q) s += red[q][i];
      partials[(size_t)blockIdx.x * (kMaxBasis + 1) + (i == KM ? kMaxBasis : i)] = s;
    }
  }
}

// partials[b][i] = block sum of w * V_i (i < nv <= KM); slot kMaxBasis = block sum
// of w * w when with_norm.  V may be null when nv == 0.
template <typename TV, int KM>
__global__ __launch_bounds__(kBlock) void k_mdot(size_t len, const double* __restrict__ w,
                                                 const TV* __restrict__ V, size_t ldv, int nv,
                                                 int with_norm, double* __restrict__ partials) {
  double acc[KM + 1];
#pragma unroll
  for (int i = 0; i <= KM; ++i) acc[i] = 0.0;
  for (size_t t = blockIdx.x * (size_t)kBlock + threadIdx.x; t < len; t += (size_t)gridDim.x * kBlock) {
    double vv[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i) vv[i] = i < nv ? (double)V[(size_t)i * ldv + t] : 0.0;
    const double wv = w[t];
#pragma unroll
    for (int i = 0; i < KM; ++i) acc[i] += wv * vv[i];
    acc[KM] += wv * wv;
  }
  store_block_partials<KM>(acc, nv, with_norm, partials);
}

// out[i] = sum_b partials[b][i] for every requested slot i (i < nv, and slot
// kMaxBasis when with_norm); one block per slot, fixed summation order.  If
// accumulate, out[i] += the sum.
__global__ __launch_bounds__(kBlock) void k_mdot_finalize(const double* __restrict__ partials, int nb, int nv,
                                                          int with_norm, double* __restrict__ out,
                                                          int accumulate) {
  const int i = blockIdx.x;
  if (!(i < nv || (i == kMaxBasis && with_norm))) return;
  double v[1] = {0.0};
  for (int b = threadIdx.x; b < nb; b += kBlock) v[0] += partials[(size_t)b * (kMaxBasis + 1) + i];
  block_sum<1>(v);
  if (threadIdx.x == 0) out[i] = accumulate ? out[i] + v[0] : v[0];
}

// Second Gram-Schmidt pass fused with the update of the first:
//   w <- w - sum_i h_i V_i   (h = first-pass coefficients, on the device)
//   partials[b][i] = block sum of V_i * w (new w), slot kMaxBasis = block sum of w^2
template <typename TV, int KM>
__global__ __launch_bounds__(kBlock) void k_gs_update_mdot(size_t len, double* __restrict__ w,
                                                           const TV* __restrict__ V, size_t ldv, int nv,
                                                           const double* __restrict__ h,
                                                           double* __restrict__ partials) {
  double acc[KM + 1], hh[KM];
#pragma unroll
  for (int i = 0; i <= KM; ++i) acc[i] = 0.0;
#pragma unroll
  for (int i = 0; i < KM; ++i) hh[i] = i < nv ? h[i] : 0.0;
  for (size_t t = blockIdx.x * (size_t)kBlock + threadIdx.x; t < len; t += (size_t)gridDim.x * kBlock) {
    double vv[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i) vv[i] = i < nv ? (double)V[(size_t)i * ldv + t] : 0.0;
    double s = w[t];
#pragma unroll
    for (int i = 0; i < KM; ++i) s -= hh[i] * vv[i];
    w[t] = s;
#pragma unroll
    for (int i = 0; i < KM; ++i) acc[i] += s * vv[i];
    acc[KM] += s * s;
  }
  store_block_partials<KM>(acc, nv, 1, partials);
}

// Last Gram-Schmidt update fused with the normalization: out = s (w - sum_i h_i V_i).
template <typename TV, int KM>
__global__ __launch_bounds__(kBlock) void k_gs_final(size_t len, const double* __restrict__ w,
                                                     const TV* __restrict__ V, size_t ldv, int nv,
                                                     const double* __restrict__ h, double* __restrict__ out,
                                                     double s) {
  double hh[KM];
#pragma unroll
  for (int i = 0; i < KM; ++i) hh[i] = i < nv ? h[i] : 0.0;
  for (size_t t = blockIdx.x * (size_t)kBlock + threadIdx.x; t < len; t += (size_t)gridDim.x * kBlock) {
    double v = w[t];
#pragma unroll
    for (int i = 0; i < KM; ++i)
      if (i < nv) v -= hh[i] * (double)V[(size_t)i * ldv + t];
    out[t] = v * s;
  }
}

// v = s w
__global__ void k_scale(size_t len, const double* __restrict__ w, double* __restrict__ v, double s) {
  for (size_t t = blockIdx.x * (size_t)kBlock + threadIdx.x; t < len; t += (size_t)gridDim.x * kBlock)
    v[t] = w[t] * s;
}

// x += sum_i y_i Z_i  (y on the device)
template <typename TZ, int KM>
__global__ __launch_bounds__(kBlock) void k_basis_axpy(size_t len, double* __restrict__ x,
                                                       const TZ* __restrict__ Z, size_t ldz, int nz,
                                                       const double* __restrict__ y) {
  double yy[KM];
#pragma unroll
  for (int i = 0; i < KM; ++i) yy[i] = i < nz ? y[i] : 0.0;
  for (size_t t = blockIdx.x * (size_t)kBlock + threadIdx.x; t < len; t += (size_t)gridDim.x * kBlock) {
    double s = x[t];
#pragma unroll
    for (int i = 0; i < KM; ++i)
      if (i < nz) s += yy[i] * (double)Z[(size_t)i * ldz + t];
    x[t] = s;
  }
}

}  // namespace smg
