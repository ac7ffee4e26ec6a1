// jacobi.h -- damped collective Jacobi step (gfx950), the smoother of the
// paper's experiments; an option of the V-cycle next to the red-black
// Gauss-Seidel half-sweeps of smoother.h.
#pragma once
#include "common.h"

namespace smg {

// One damped collective Jacobi step (eq. collective_smoothing) at one node by a
// group of W lanes: the node's residual rows r = f - S xin, formed as
// residual_node forms them, the node system S~_i d = r solved as in
// halfsweep_node (with the residual rows as right-hand sides and no neighbour
// terms), and xout_i = xin_i + theta d.  Out of place: xin and xout must not
// alias (every node reads its neighbours' old values).
// dsum and num summed over the node's group: W <= 64 lanes within a wave;
// WT = kBlock (a block per node, for many samples) across its waves in LDS.
template <int WT, typename T>
__device__ __forceinline__ void jacobi_group_sums(T& a, T& b, int W) {
  if constexpr (WT > 64) {
    static_assert(WT == kBlock, "a wide group is one block");
    __shared__ T sa[kBlock / 64], sb[kBlock / 64];
    a = group_sum<64>(a);
    b = group_sum<64>(b);
    if ((threadIdx.x & 63) == 0) { sa[threadIdx.x >> 6] = a; sb[threadIdx.x >> 6] = b; }
    __syncthreads();
    T ra = 0, rb = 0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) { ra += sa[q]; rb += sb[q]; }
    a = ra;
    b = rb;
  } else {
    a = group_sum_w(a, W);
    b = group_sum_w(b, W);
  }
}

template <typename T, int JM, int VW = 1, bool MK = true, int WT = 0>
__device__ __forceinline__ void jacobi_node(const LevelArgs<T>& L, const T* __restrict__ xin, T* __restrict__ xout,
                                            const T* __restrict__ f, T theta, int slot, int lane, int W) {
  static_assert(JM % VW == 0, "whole chunks per lane");
  constexpr int NCH = JM / VW;
  const int n = L.n, N = L.N;
  const size_t nn = (size_t)n * n, rowN = (size_t)n * N;
  int xx, k;
  strip_node(slot, n, L.strip, xx, k);
  const size_t node = (size_t)k * n + xx;
  const T* Y = xin;
  const T* P = xin + (size_t)(N + 1) * nn;
  const T* fY = f;
  const T* fP = f + (size_t)(N + 1) * nn;
  const size_t kxb = ((size_t)k * (n + 1) + xx) * N;
  const size_t kyb = node * N;
  const bool hw = xx > 0, he = xx < n - 1, hs = k > 0, hn = k < n - 1;
  // missing neighbours read the node itself and are selected away; a chunk
  // past N reads the last chunk and is masked out of the sums
  const ptrdiff_t ow = hw ? -(ptrdiff_t)N : 0, oe = he ? (ptrdiff_t)N : 0;
  const ptrdiff_t os = hs ? -(ptrdiff_t)rowN : 0, on = hn ? (ptrdiff_t)rowN : 0;
  const T u = xin[(size_t)N * nn + node], fu = f[(size_t)N * nn + node], gd = L.gden[node];
  const NodeFactors<T> mf = node_factors<MK>(L, node);
  T rYq[JM], rPq[JM], ia[JM], cq[JM], eq[JM], yo[JM], po[JM];
  T dsum = 0, num = 0;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int j0 = VW * (lane + c * W);
    const bool act = j0 < N;
    const int j = act ? j0 : N - VW;
    const size_t base = node * N + j;
    T kw[VW], ke[VW], ks[VW], kn[VW], cj[VW], dj[VW], ej[VW], fy[VW], fp[VW];
    ldv<VW>(L.kx + kxb + j, kw);
    ldv<VW>(L.kx + kxb + N + j, ke);
    ldv<VW>(L.ky + kyb + j, ks);
    ldv<VW>(L.ky + kyb + rowN + j, kn);
    ldv<VW>(L.c + j, cj);
    ldv<VW>(L.d + j, dj);
    ldv<VW>(L.e + j, ej);
    ldv<VW>(fY + base, fy);
    ldv<VW>(fP + base, fp);
    T y0[VW], p0[VW], yw[VW], ye[VW], ys[VW], yn[VW], pw[VW], pe[VW], ps[VW], pn[VW];
    ldv<VW>(Y + base, y0); ldv<VW>(P + base, p0);
    ldv<VW>(Y + base + ow, yw); ldv<VW>(Y + base + oe, ye); ldv<VW>(Y + base + os, ys); ldv<VW>(Y + base + on, yn);
    ldv<VW>(P + base + ow, pw); ldv<VW>(P + base + oe, pe); ldv<VW>(P + base + os, ps); ldv<VW>(P + base + on, pn);
#pragma unroll
    for (int v = 0; v < VW; ++v) {
      const int q = c * VW + v;
      auto nbsum = [&](T vw, T ve, T vs, T vn) -> T {
        return ((hw ? kw[v] * vw : T(0)) + (he ? ke[v] * ve : T(0))) +
               ((hs ? ks[v] * vs : T(0)) + (hn ? kn[v] * vn : T(0)));
      };
      const T sy = nbsum(yw[v], ye[v], ys[v], yn[v]);
      const T sp = nbsum(pw[v], pe[v], ps[v], pn[v]);
      const T a = (kw[v] + ke[v]) + (ks[v] + kn[v]);
      const T rY = fy[v] - (cj[v] * y0[v] + (a * p0[v] - sp));   // Y row: C_j y_j + A_j^T p_j
      const T rP = fp[v] - ((a * y0[v] - sy) + (mf.e * ej[v]) * u);   // P row: A_j y_j + E_j u
      dsum += act ? (mf.d * dj[v]) * p0[v] : T(0);
      const T ai = T(1) / a;
      const T t = cj[v] * ai * ai;
      num += act ? (mf.d * dj[v]) * (t * rP - ai * rY) : T(0);
      rYq[q] = rY; rPq[q] = rP; ia[q] = ai; cq[q] = cj[v]; eq[q] = mf.e * ej[v]; yo[q] = y0[v]; po[q] = p0[v];
    }
  }
  jacobi_group_sums<WT>(dsum, num, W);
  const T rU = fu - (L.g * u + dsum);                         // U row: G u + sum_j D_j p_j
  const T du = (rU + num) / gd;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int j = VW * (lane + c * W);
    if (j < N) {
      const size_t base = node * N + j;
      T yv[VW], pv[VW];
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        const int q = c * VW + v;
        const T dy = ia[q] * (rPq[q] - eq[q] * du);
        const T dp = ia[q] * (rYq[q] - cq[q] * dy);
        yv[v] = node_live(mf) ? yo[q] + theta * dy : T(0);   // outside the domain: zero
        pv[v] = node_live(mf) ? po[q] + theta * dp : T(0);
      }
      stv<VW>(xout + base, yv);
      stv<VW>(xout + (size_t)(N + 1) * nn + base, pv);
    }
  }
  if (lane == 0) xout[(size_t)N * nn + node] = node_live(mf) ? u + theta * du : T(0);
}

template <typename T, int W, int JM, int VW, bool MK>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, JM >= 4 ? 3 : 8)))
void k_jacobi(LevelArgs<T> L, const T* __restrict__ xin, T* __restrict__ xout, const T* __restrict__ f, T theta) {
  const int b = xcd_remap(blockIdx.x, group_blocks<W>(L.n * L.n));
  const int lane = threadIdx.x & (W - 1);
  const int slot = group_slot<W>(b);
  if (slot >= L.n * L.n) return;
  jacobi_node<T, JM, VW, MK, W>(L, xin, xout, f, theta, slot, lane, W);
}

}  // namespace smg
