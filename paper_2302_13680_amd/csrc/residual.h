// residual.h -- N-batched residual / operator application and its norms (gfx950).
#pragma once
#include "common.h"

namespace smg {

// Residual rows of one node (slot = k n + x) by a group of W lanes:
// out = f - S x (mode 0) or out = S x (mode 1), block rows of eq. (2):
//   Y rows: C_j y_j + A_j^T p_j,  U row: G u + sum_j D_j p_j,  P rows: A_j y_j + E_j u.
// Faces and arithmetic in T, x and f in TX, out in TO (out may be null).
// acc[0..2] accumulate the squared Y, U (lane 0) and P residual entries, acc[3]
// the squared entries of f (mode 0), which gives ||f|| in the same pass.
template <typename T, typename TX, typename TO, int JM, int VW = 1, bool MK = true>
__device__ __forceinline__ void residual_node(const LevelArgs<T>& L, const TX* __restrict__ x,
                                              const TX* __restrict__ f, TO* __restrict__ out, int mode,
                                              int slot, int lane, int W, double (&acc)[4]) {
  static_assert(JM % VW == 0, "whole chunks per lane");
  constexpr int NCH = JM / VW;
  const int n = L.n, N = L.N;
  const size_t nn = (size_t)n * n, rowN = (size_t)n * N;
  int xx, k;
  strip_node(slot, n, L.strip, xx, k);   // strips keep the rows above and below in L2
  const size_t node = (size_t)k * n + xx;
  const TX* Y = x;
  const TX* P = x + (size_t)(N + 1) * nn;
  const T u = (T)x[(size_t)N * nn + node];
  const NodeFactors<T> mf = node_factors<MK>(L, node);
  const size_t kxb = ((size_t)k * (n + 1) + xx) * N;
  const size_t kyb = node * N;
  const bool hw = xx > 0, he = xx < n - 1, hs = k > 0, hn = k < n - 1;
  // Unconditional loads: a missing neighbour reads the node itself and a chunk
  // past N reads the last chunk; both are selected away (see halfsweep_node).
  const ptrdiff_t ow = hw ? -(ptrdiff_t)N : 0, oe = he ? (ptrdiff_t)N : 0;
  const ptrdiff_t os = hs ? -(ptrdiff_t)rowN : 0, on = hn ? (ptrdiff_t)rowN : 0;
  T dsum = 0;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int j0 = VW * (lane + c * W);
    const bool act = j0 < N;
    const int j = act ? j0 : N - VW;
    T kw[VW], ke[VW], ks[VW], kn[VW];
    ldv<VW>(L.kx + kxb + j, kw);
    ldv<VW>(L.kx + kxb + N + j, ke);
    ldv<VW>(L.ky + kyb + j, ks);
    ldv<VW>(L.ky + kyb + rowN + j, kn);
    const size_t base = node * N + j;
    TX y0[VW], p0[VW], yw[VW], ye[VW], ys[VW], yn[VW], pw[VW], pe[VW], ps[VW], pn[VW];
    ldv<VW>(Y + base, y0); ldv<VW>(P + base, p0);
    ldv<VW>(Y + base + ow, yw); ldv<VW>(Y + base + oe, ye); ldv<VW>(Y + base + os, ys); ldv<VW>(Y + base + on, yn);
    ldv<VW>(P + base + ow, pw); ldv<VW>(P + base + oe, pe); ldv<VW>(P + base + os, ps); ldv<VW>(P + base + on, pn);
    T cj[VW], dj[VW], ej[VW];
    ldv<VW>(L.c + j, cj);
    ldv<VW>(L.d + j, dj);
    ldv<VW>(L.e + j, ej);
    TX fyv[VW], fpv[VW];
    if (mode == 0) {
      ldv<VW>(f + base, fyv);
      ldv<VW>(f + (size_t)(N + 1) * nn + base, fpv);
    }
    TO ry[VW], rp[VW];
#pragma unroll
    for (int q = 0; q < VW; ++q) {
      auto nbsum = [&](T vw, T ve, T vs, T vn) -> T {
        return ((hw ? kw[q] * vw : T(0)) + (he ? ke[q] * ve : T(0))) +
               ((hs ? ks[q] * vs : T(0)) + (hn ? kn[q] * vn : T(0)));
      };
      const T sy = nbsum((T)yw[q], (T)ye[q], (T)ys[q], (T)yn[q]);
      const T sp = nbsum((T)pw[q], (T)pe[q], (T)ps[q], (T)pn[q]);
      const T a = (kw[q] + ke[q]) + (ks[q] + kn[q]);
      const T yq = (T)y0[q], pq = (T)p0[q];
      T rY = cj[q] * yq + (a * pq - sp);     // C_j y_j + A_j^T p_j
      T rP = (a * yq - sy) + (mf.e * ej[q]) * u;   // A_j y_j + E_j u
      dsum += act ? (mf.d * dj[q]) * pq : T(0);
      double ff = 0.0;
      if (mode == 0) {
        const T fy = (T)fyv[q], fp = (T)fpv[q];
        rY = fy - rY;
        rP = fp - rP;
        ff = (double)fy * (double)fy + (double)fp * (double)fp;
      }
      rY = node_live(mf) ? rY : T(0);   // zero rows outside the domain
      rP = node_live(mf) ? rP : T(0);
      ry[q] = (TO)rY;
      rp[q] = (TO)rP;
      if (act) {
        acc[0] += (double)rY * (double)rY;
        acc[2] += (double)rP * (double)rP;
        acc[3] += ff;
      }
    }
    if (act && out) {
      stv_nt<VW>(out + base, ry);
      stv_nt<VW>(out + (size_t)(N + 1) * nn + base, rp);
    }
  }
  dsum = group_sum_w(dsum, W);
  if (lane == 0) {
    T rU = L.g * u + dsum;                    // G u + sum_j D_j p_j
    if (mode == 0) {
      const T fu = (T)f[(size_t)N * nn + node];
      rU = fu - rU;
      acc[3] += (double)fu * (double)fu;
    }
    rU = node_live(mf) ? rU : T(0);
    if (out) out[(size_t)N * nn + node] = (TO)rU;
    acc[1] = (double)rU * (double)rU;
  }
}

// One refinement update fused with the next residual: x_next = x + d (d: the
// FP32 correction of the cycle) and out = f - S x_next rounded to FP32, by a group
// of W lanes for one node; the neighbours' x + d are formed on the fly with the
// same FP64 addition their own groups store, so no group reads x_next.  acc as
// in residual_node.  x_next must not alias x.
template <int JM, int VW = 1, bool MK = true>
__device__ __forceinline__ void residual_add_node(const LevelArgs<double>& L, const double* __restrict__ x,
                                                  const float* __restrict__ d, double* __restrict__ xn,
                                                  const double* __restrict__ f, float* __restrict__ out,
                                                  int slot, int lane, int W, double (&acc)[4]) {
  static_assert(JM % VW == 0, "whole chunks per lane");
  constexpr int NCH = JM / VW;
  const int n = L.n, N = L.N;
  const size_t nn = (size_t)n * n, rowN = (size_t)n * N;
  int xx, k;
  strip_node(slot, n, L.strip, xx, k);
  const size_t node = (size_t)k * n + xx;
  const size_t oU = (size_t)N * nn, oP = (size_t)(N + 1) * nn;
  const double u = x[oU + node] + (double)d[oU + node];
  const NodeFactors<double> mf = node_factors<MK>(L, node);
  const size_t kxb = ((size_t)k * (n + 1) + xx) * N;
  const size_t kyb = node * N;
  const bool hw = xx > 0, he = xx < n - 1, hs = k > 0, hn = k < n - 1;
  const ptrdiff_t ow = hw ? -(ptrdiff_t)N : 0, oe = he ? (ptrdiff_t)N : 0;
  const ptrdiff_t os = hs ? -(ptrdiff_t)rowN : 0, on = hn ? (ptrdiff_t)rowN : 0;
  // x + d of VW samples at element offset i of the Y (o = 0) or P (o = oP) block
  auto xd = [&](size_t i, double (&v)[VW]) {
    double xv[VW];
    float dv[VW];
    ldv<VW>(x + i, xv);
    ldv<VW>(d + i, dv);
#pragma unroll
    for (int q = 0; q < VW; ++q) v[q] = xv[q] + (double)dv[q];
  };
  double dsum = 0;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int j0 = VW * (lane + c * W);
    const bool act = j0 < N;
    const int j = act ? j0 : N - VW;
    double kw[VW], ke[VW], ks[VW], kn[VW], cj[VW], dj[VW], ej[VW], fy[VW], fp[VW];
    ldv<VW>(L.kx + kxb + j, kw);
    ldv<VW>(L.kx + kxb + N + j, ke);
    ldv<VW>(L.ky + kyb + j, ks);
    ldv<VW>(L.ky + kyb + rowN + j, kn);
    ldv<VW>(L.c + j, cj);
    ldv<VW>(L.d + j, dj);
    ldv<VW>(L.e + j, ej);
    const size_t base = node * N + j;
    double y0[VW], p0[VW], yw[VW], ye[VW], ys[VW], yn[VW], pw[VW], pe[VW], ps[VW], pn[VW];
    xd(base, y0); xd(oP + base, p0);
    xd(base + ow, yw); xd(base + oe, ye); xd(base + os, ys); xd(base + on, yn);
    xd(oP + base + ow, pw); xd(oP + base + oe, pe); xd(oP + base + os, ps); xd(oP + base + on, pn);
    ldv<VW>(f + base, fy);
    ldv<VW>(f + oP + base, fp);
    float ry[VW], rp[VW];
#pragma unroll
    for (int q = 0; q < VW; ++q) {
      auto nbsum = [&](double vw, double ve, double vs, double vn) {
        return ((hw ? kw[q] * vw : 0.0) + (he ? ke[q] * ve : 0.0)) + ((hs ? ks[q] * vs : 0.0) + (hn ? kn[q] * vn : 0.0));
      };
      const double sy = nbsum(yw[q], ye[q], ys[q], yn[q]);
      const double sp = nbsum(pw[q], pe[q], ps[q], pn[q]);
      const double a = (kw[q] + ke[q]) + (ks[q] + kn[q]);
      const double rY = node_live(mf) ? fy[q] - (cj[q] * y0[q] + (a * p0[q] - sp)) : 0.0;   // zero rows outside
      const double rP = node_live(mf) ? fp[q] - ((a * y0[q] - sy) + (mf.e * ej[q]) * u) : 0.0;
      dsum += act ? (mf.d * dj[q]) * p0[q] : 0.0;
      ry[q] = (float)rY;
      rp[q] = (float)rP;
      if (act) {
        acc[0] += rY * rY;
        acc[2] += rP * rP;
        acc[3] += fy[q] * fy[q] + fp[q] * fp[q];
      }
    }
    if (act) {
      stv_nt<VW>(xn + base, y0);
      stv_nt<VW>(xn + oP + base, p0);
      stv_nt<VW>(out + base, ry);
      stv_nt<VW>(out + oP + base, rp);
    }
  }
  dsum = group_sum_w(dsum, W);
  if (lane == 0) {
    const double fu = f[oU + node];
    const double rU = node_live(mf) ? fu - (L.g * u + dsum) : 0.0;
    xn[oU + node] = u;
    out[oU + node] = (float)rU;
    acc[1] = rU * rU;
    acc[3] += fu * fu;
  }
}

template <int W, int JM, int VW, bool MK>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, JM >= 4 ? 3 : 8)))
void k_residual_add(LevelArgs<double> L, const double* __restrict__ x, const float* __restrict__ d,
                    double* __restrict__ xn, const double* __restrict__ f, float* __restrict__ out,
                    double* __restrict__ partials) {
  const int b = xcd_remap(blockIdx.x, group_blocks<W>(L.n * L.n));
  const int lane = threadIdx.x & (W - 1);
  const int slot = group_slot<W>(b);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (slot < L.n * L.n) residual_add_node<JM, VW, MK>(L, x, d, xn, f, out, slot, lane, W, acc);
  block_sum<4>(acc);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) partials[4 * (size_t)b + i] = acc[i];
  }
}

// out = f - S x (mode 0) or out = S x (mode 1) over every node.  partials (if not
// null) receives per block { sum r_Y^2, sum r_U^2, sum r_P^2, sum f^2 }.
template <typename T, typename TX, typename TO, int W, int JM, int VW, bool MK>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, JM >= 4 ? 3 : 8)))
void k_residual(LevelArgs<T> L, const TX* __restrict__ x, const TX* __restrict__ f, TO* __restrict__ out,
                int mode, double* __restrict__ partials) {
  const int b = xcd_remap(blockIdx.x, group_blocks<W>(L.n * L.n));
  const int lane = threadIdx.x & (W - 1);
  const int slot = group_slot<W>(b);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (slot < L.n * L.n) residual_node<T, TX, TO, JM, VW, MK>(L, x, f, out, mode, slot, lane, W, acc);
  if (partials) {
    block_sum<4>(acc);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) partials[4 * (size_t)b + i] = acc[i];
    }
  }
}

// First stage of the norm reduction for many partials: block b sums the b-th
// contiguous chunk of the nb block partials into out[b][0..3] (fixed order).
__global__ __launch_bounds__(kBlock) void k_norms_stage(const double* __restrict__ partials, int nb,
                                                      double* __restrict__ out) {
  const int chunk = (nb + gridDim.x - 1) / gridDim.x;
  const int lo = blockIdx.x * chunk, hi = min(nb, lo + chunk);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = lo + threadIdx.x; i < hi; i += kBlock) {
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] += partials[4 * (size_t)i + c];
  }
  block_sum<4>(acc);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) out[4 * (size_t)blockIdx.x + c] = acc[c];
  }
}

// norms[0..4] = { ||r||, ||r_Y||, ||r_U||, ||r_P||, ||f|| } from nb block
// partials (one block of 1024 threads, fixed summation order).
__global__ __launch_bounds__(1024) void k_finalize_norms(const double* __restrict__ partials, int nb,
                                                         double* __restrict__ norms) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nb; i += 1024) {
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] += partials[4 * (size_t)i + c];
  }
  block_sum<4, 1024>(acc);
  if (threadIdx.x == 0) {
    norms[0] = sqrt(acc[0] + acc[1] + acc[2]);
    norms[1] = sqrt(acc[0]);
    norms[2] = sqrt(acc[1]);
    norms[3] = sqrt(acc[2]);
    norms[4] = sqrt(acc[3]);
  }
}

}  // namespace smg
