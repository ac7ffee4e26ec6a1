// transfer.h -- restriction and prolongation between grid levels (gfx950).
#pragma once
#include "common.h"

namespace smg {

// coarse = R fine, R = P^T: coarse node (X, K) sits on fine node (2X+1, 2K+1)
// and gathers its 3x3 fine neighbourhood with weights w(dx) w(dk).  One group
// of W lanes per coarse node; the slot-th coarse node in strips of cstrip
// coarse columns (strip_node).
template <typename T, int JM, int VW = 1>
__device__ __forceinline__ void restrict_node(int nf, int N, const T* __restrict__ fine,
                                              T* __restrict__ coarse, int slot, int lane, int W, int cstrip) {
  static_assert(JM % VW == 0, "whole chunks per lane");
  constexpr int NCH = JM / VW;
  const int nc = (nf - 1) / 2;
  const size_t nnf = (size_t)nf * nf, nnc = (size_t)nc * nc;
  int X, K;
  strip_node(slot, nc, cstrip, X, K);
  const int cnode = K * nc + X;
  const size_t c0 = (size_t)(2 * K + 1) * nf + (2 * X + 1);
  const T* fY = fine;
  const T* fP = fine + (size_t)(N + 1) * nnf;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    // loads for a chunk past N read the last chunk (in bounds); only the stores
    // are guarded, so all loads of the node can be in flight together
    const int j0 = VW * (lane + c * W);
    const int j = j0 < N ? j0 : N - VW;
    T sY[VW], sP[VW];
#pragma unroll
    for (int u = 0; u < VW; ++u) { sY[u] = T(0); sP[u] = T(0); }
#pragma unroll
    for (int dk = -1; dk <= 1; ++dk)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const T w = (T)(lin_w(dx) * lin_w(dk));
        const size_t fi = (size_t)((long)c0 + (long)dk * nf + dx) * N + j;
        T vy[VW], vp[VW];
        ldv<VW>(fY + fi, vy);
        ldv<VW>(fP + fi, vp);
#pragma unroll
        for (int u = 0; u < VW; ++u) {
          sY[u] += w * vy[u];
          sP[u] += w * vp[u];
        }
      }
    if (j0 < N) {
      stv<VW>(coarse + (size_t)cnode * N + j, sY);
      stv<VW>(coarse + (size_t)(N + 1) * nnc + (size_t)cnode * N + j, sP);
    }
  }
  if (lane == 0) {
    const T* fU = fine + (size_t)N * nnf;
    T sU = 0;
#pragma unroll
    for (int dk = -1; dk <= 1; ++dk)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx)
        sU += (T)(lin_w(dx) * lin_w(dk)) * fU[(long)c0 + (long)dk * nf + dx];
    coarse[(size_t)N * nnc + cnode] = sU;
  }
}

template <typename T, int W, int JM, int VW>
__global__ __launch_bounds__(kBlock) void k_restrict(int nf, int N, const T* __restrict__ fine,
                                                     T* __restrict__ coarse, int cstrip) {
  const int nc = (nf - 1) / 2;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x & (W - 1);
  const int slot = b * (kBlock / W) + threadIdx.x / W;
  if (slot >= nc * nc) return;
  restrict_node<T, JM, VW>(nf, N, fine, coarse, slot, lane, W, cstrip);
}

// fine += P coarse, bilinear interpolation gathered per fine node.
template <typename T, int W, int JM>
__global__ __launch_bounds__(kBlock) void k_prolong_add(int nc, int N, const T* __restrict__ coarse,
                                                        T* __restrict__ fine) {
  const int nf = 2 * nc + 1;
  const size_t nnf = (size_t)nf * nf, nnc = (size_t)nc * nc;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x & (W - 1);
  const int slot = b * (kBlock / W) + threadIdx.x / W;
  if (slot >= (int)nnf) return;
  const int k = slot / nf, xx = slot - k * nf;
  // coarse columns/rows touching this fine node and their weights
  int cx[2], ck[2];
  T wx[2], wk[2];
  int nx = 0, nk = 0;
  if (xx & 1) { cx[nx] = (xx - 1) / 2; wx[nx++] = T(1); }
  else {
    if (xx / 2 - 1 >= 0) { cx[nx] = xx / 2 - 1; wx[nx++] = T(0.5); }
    if (xx / 2 < nc) { cx[nx] = xx / 2; wx[nx++] = T(0.5); }
  }
  if (k & 1) { ck[nk] = (k - 1) / 2; wk[nk++] = T(1); }
  else {
    if (k / 2 - 1 >= 0) { ck[nk] = k / 2 - 1; wk[nk++] = T(0.5); }
    if (k / 2 < nc) { ck[nk] = k / 2; wk[nk++] = T(0.5); }
  }
  const T* cY = coarse;
  const T* cP = coarse + (size_t)(N + 1) * nnc;
#pragma unroll
  for (int q = 0; q < JM; ++q) {
    const int j = lane + q * W;
    if (j < N) {
      T sY = 0, sP = 0;
      for (int a = 0; a < nk; ++a)
        for (int c = 0; c < nx; ++c) {
          const T w = wk[a] * wx[c];
          const size_t ci = ((size_t)ck[a] * nc + cx[c]) * N + j;
          sY += w * cY[ci];
          sP += w * cP[ci];
        }
      fine[(size_t)slot * N + j] += sY;
      fine[(size_t)(N + 1) * nnf + (size_t)slot * N + j] += sP;
    }
  }
  if (lane == 0) {
    const T* cU = coarse + (size_t)N * nnc;
    T sU = 0;
    for (int a = 0; a < nk; ++a)
      for (int c = 0; c < nx; ++c) sU += wk[a] * wx[c] * cU[(size_t)ck[a] * nc + cx[c]];
    fine[(size_t)N * nnf + slot] += sU;
  }
}

}  // namespace smg
