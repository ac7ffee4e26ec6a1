// smoother.h -- collective Gauss-Seidel half-sweep (gfx950).
#pragma once
#include "common.h"

namespace smg {

// Neighbour values the half-sweep reads, by source:
//   kPlain   : the level iterate x (the other colour)
//   kZero    : a zero iterate (first red half-sweep of a cycle started from 0)
//   kProlong : x + P e_c, the iterate after the coarse correction of Alg. 1,
//              interpolated on the fly from the coarse correction e_c (the other
//              colour is overwritten by the following half-sweep, so the
//              corrected values never need to be stored)
enum NbSource { kPlain = 0, kZero = 1, kProlong = 2 };

// Coarse corrections (P e)(nb) of the four neighbours W, E, S, N of a fine node
// with x + k even (the red colour), for one sample field of the coarse vector e
// (nc x nc coarse grid, stride N between nodes).  Such a node either coincides
// with coarse node (X, K) (x, k odd) or is the centre of a coarse cell (x, k
// even); every neighbour lies on a coarse edge, so bilinear interpolation there
// averages two coarse values.  Coarse nodes outside the grid are zero.
template <int VW, typename T>
__device__ __forceinline__ void prolong_nb(const T* __restrict__ e, int nc, int N, int j, int x, int k,
                                           T (&cw)[VW], T (&ce)[VW], T (&cs)[VW], T (&cn)[VW]) {
  // Five unconditional loads (clamped into the grid, outside values selected to
  // zero) for both cases, so that they are in flight together with the node's
  // other loads.  x odd: v0 = (X, K) and its W, E, S, N coarse neighbours
  // v1..v4; x even: v1..v4 = the cell corners (X-1, K-1), (X, K-1), (X-1, K),
  // (X, K) (v0 = v4 is read twice).  VW consecutive samples from j.
  auto at = [&](int X, int K, T (&v)[VW]) {
    const bool in = X >= 0 && X < nc && K >= 0 && K < nc;
    const int Xc = X < 0 ? 0 : (X >= nc ? nc - 1 : X), Kc = K < 0 ? 0 : (K >= nc ? nc - 1 : K);
    ldv<VW>(e + ((size_t)Kc * nc + Xc) * N + j, v);
#pragma unroll
    for (int u = 0; u < VW; ++u) v[u] = in ? v[u] : T(0);
  };
  const bool odd = x & 1;
  const int X = odd ? (x - 1) >> 1 : x >> 1, K = odd ? (k - 1) >> 1 : k >> 1;
  T v0[VW], v1[VW], v2[VW], v3[VW], v4[VW];
  at(X, K, v0);
  at(X - 1, odd ? K : K - 1, v1);
  at(odd ? X + 1 : X, odd ? K : K - 1, v2);
  at(odd ? X : X - 1, odd ? K - 1 : K, v3);
  at(X, odd ? K + 1 : K, v4);
#pragma unroll
  for (int u = 0; u < VW; ++u) {
    cw[u] = T(0.5) * (v1[u] + (odd ? v0[u] : v3[u]));
    ce[u] = T(0.5) * ((odd ? v0[u] : v2[u]) + (odd ? v2[u] : v4[u]));
    cs[u] = T(0.5) * ((odd ? v3[u] : v1[u]) + (odd ? v0[u] : v2[u]));
    cn[u] = T(0.5) * ((odd ? v0[u] : v3[u]) + v4[u]);
  }
}

// Half-sweep update of the slot-th node of `colour` by one group of W lanes
// (lane = index in the group; JM samples per lane in chunks of VW, see
// common.h).  The node is replaced by the solution of its (2N+1)x(2N+1) system
// (eq. solution_reduced_system) with the opposite-colour neighbours fixed:
//   bP_j = fY_j + sum_nb k_nb p_j,nb      (rhs of the C_j / A_j^T row)
//   bY_j = fP_j + sum_nb k_nb y_j,nb      (rhs of the A_j / E_j row)
//   u    = (fU + sum_j d_j (c_j bY_j / a_j^2 - bP_j / a_j)) / (g + sum_j d_j c_j e_j / a_j^2)
//   y_j  = (bY_j - e_j u) / a_j,   p_j = (bP_j - c_j y_j) / a_j
// The denominator of u depends on the operator only and is read from L.gden
// (node_den, at setup).
// theta != 1 (relaxation) is supported for SRC == kPlain only; kProlong needs
// colour 0.  W is a compile-time constant after inlining in the single-instance
// kernel and a per-instance value in the batched one; the arithmetic is the same.
template <typename T, int JM, int SRC, int VW = 1, bool MK = true>
__device__ __forceinline__ void halfsweep_node(const LevelArgs<T>& L, T* __restrict__ x,
                                               const T* __restrict__ f, int colour, T theta, int slot,
                                               int lane, int W, const T* __restrict__ ec) {
  static_assert(JM % VW == 0, "whole chunks per lane");
  constexpr int NCH = JM / VW;
  const int n = L.n, N = L.N;
  const size_t nn = (size_t)n * n, rowN = (size_t)n * N;
  int xx, k;
  colour_node(slot, n, colour, L.strip, xx, k);
  const size_t node = (size_t)k * n + xx;
  T* __restrict__ Y = x;
  T* __restrict__ U = x + (size_t)N * nn;
  T* __restrict__ P = x + (size_t)(N + 1) * nn;
  const T* __restrict__ fY = f;
  const T* __restrict__ fU = f + (size_t)N * nn;
  const T* __restrict__ fP = f + (size_t)(N + 1) * nn;
  const size_t kxb = ((size_t)k * (n + 1) + xx) * N;
  const size_t kyb = node * N;
  const bool hw = xx > 0, he = xx < n - 1, hs = k > 0, hn = k < n - 1;
  const int nc = (n - 1) / 2;
  const size_t nnc = (size_t)nc * nc;
  const T* eY = ec;
  const T* eP = ec + (size_t)(N + 1) * nnc;
  // Neighbour offsets; a missing (boundary) neighbour reads the node itself and
  // is discarded by a select (the node's own old value may be stale, e.g. the
  // other colour right after a zero-start sweep), so every load is
  // unconditional.  A chunk past N (ragged last lane group) reads the last
  // chunk and is masked out of the sums.
  const ptrdiff_t ow = hw ? -(ptrdiff_t)N : 0, oe = he ? (ptrdiff_t)N : 0;
  const ptrdiff_t os = hs ? -(ptrdiff_t)rowN : 0, on = hn ? (ptrdiff_t)rowN : 0;
  // per-node values first, so that their loads are in flight with the rest
  const T fu = fU[node], gd = L.gden[node];
  const NodeFactors<T> mf = node_factors<MK>(L, node);
  T bP[JM], bY[JM], ia[JM], cq[JM], eq[JM];
  T num = 0;
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
    // every load of the chunk is written before the arithmetic that uses it, so
    // that the compiler issues them together
    T cj[VW], dj[VW], ej[VW], fy[VW], fp[VW];
    ldv<VW>(L.c + j, cj);
    ldv<VW>(L.d + j, dj);
    ldv<VW>(L.e + j, ej);
    ldv<VW>(fY + base, fy);
    ldv<VW>(fP + base, fp);
    // sum over existing neighbours of face * value (missing ones selected away)
    auto nbsum = [&](int u, T vw, T ve, T vs, T vn) -> T {
      return ((hw ? kw[u] * vw : T(0)) + (he ? ke[u] * ve : T(0))) +
             ((hs ? ks[u] * vs : T(0)) + (hn ? kn[u] * vn : T(0)));
    };
    T sy[VW], sp[VW];
#pragma unroll
    for (int u = 0; u < VW; ++u) { sy[u] = T(0); sp[u] = T(0); }
    if constexpr (SRC != kZero) {
      T yw[VW], ye[VW], ys[VW], yn[VW], pw[VW], pe[VW], ps[VW], pn[VW];
      ldv<VW>(Y + base + ow, yw); ldv<VW>(Y + base + oe, ye); ldv<VW>(Y + base + os, ys); ldv<VW>(Y + base + on, yn);
      ldv<VW>(P + base + ow, pw); ldv<VW>(P + base + oe, pe); ldv<VW>(P + base + os, ps); ldv<VW>(P + base + on, pn);
      T cwy[VW], cey[VW], csy[VW], cny[VW], cwp[VW], cep[VW], csp[VW], cnp[VW];
      if constexpr (SRC == kProlong) {
        prolong_nb<VW>(eY, nc, N, j, xx, k, cwy, cey, csy, cny);
        prolong_nb<VW>(eP, nc, N, j, xx, k, cwp, cep, csp, cnp);
      }
#pragma unroll
      for (int u = 0; u < VW; ++u) {
        sy[u] = nbsum(u, yw[u], ye[u], ys[u], yn[u]);
        sp[u] = nbsum(u, pw[u], pe[u], ps[u], pn[u]);
        if constexpr (SRC == kProlong) {
          sy[u] += nbsum(u, cwy[u], cey[u], csy[u], cny[u]);
          sp[u] += nbsum(u, cwp[u], cep[u], csp[u], cnp[u]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < VW; ++u) {
      const int q = c * VW + u;
      const T a = (kw[u] + ke[u]) + (ks[u] + kn[u]);
      const T ai = T(1) / a;
      const T bp = fy[u] + sp[u], by = fp[u] + sy[u];
      const T t = cj[u] * ai * ai;
      num += act ? (mf.d * dj[u]) * (t * by - ai * bp) : T(0);
      bP[q] = bp; bY[q] = by; ia[q] = ai; cq[q] = cj[u]; eq[q] = mf.e * ej[u];
    }
  }
  // e_j is first used after the sum over samples; without this the compiler
  // sinks its load there and every wave waits a full memory latency at the end
#pragma unroll
  for (int q = 0; q < JM; ++q) asm volatile("" ::"v"(eq[q]));
  num = group_sum_w(num, W);
  const T un = (fu + num) / gd;
  const bool relax = SRC == kPlain && theta != T(1);
  const bool live = node_live(mf);   // outside the domain: held at zero
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int j = VW * (lane + c * W);
    if (j < N) {
      const size_t base = node * N + j;
      T yv[VW], pv[VW];
#pragma unroll
      for (int u = 0; u < VW; ++u) {
        const int q = c * VW + u;
        yv[u] = ia[q] * (bY[q] - eq[q] * un);
        pv[u] = ia[q] * (bP[q] - cq[q] * yv[u]);
      }
      if (relax) {
        T yo[VW], po[VW];
        ldv<VW>(Y + base, yo);
        ldv<VW>(P + base, po);
#pragma unroll
        for (int u = 0; u < VW; ++u) {
          yv[u] = (T(1) - theta) * yo[u] + theta * yv[u];
          pv[u] = (T(1) - theta) * po[u] + theta * pv[u];
        }
      }
#pragma unroll
      for (int u = 0; u < VW; ++u) {
        yv[u] = live ? yv[u] : T(0);
        pv[u] = live ? pv[u] : T(0);
      }
      stv<VW>(Y + base, yv);
      stv<VW>(P + base, pv);
    }
  }
  if (lane == 0) U[node] = !live ? T(0) : relax ? (T(1) - theta) * U[node] + theta * un : un;
}

// Denominator of the control update of the node solve, per node, by a group
// of W lanes: gden = g + sum_j d_j c_j e_j / a_j^2, a_j the sum of the node's
// four faces of sample j (eq. solution_reduced_system; positive whenever the
// faces are and d_j c_j e_j >= 0).  Set up once per level, since it depends on
// the operator only.
template <typename T, int JM, int VW = 1>
__device__ __forceinline__ void node_den(const LevelArgs<T>& L, T* __restrict__ gden, int node, int lane, int W) {
  static_assert(JM % VW == 0, "whole chunks per lane");
  constexpr int NCH = JM / VW;
  const int n = L.n, N = L.N;
  const int k = node / n, xx = node - k * n;
  const size_t kxb = ((size_t)k * (n + 1) + xx) * N, kyb = (size_t)node * N, rowN = (size_t)n * N;
  const NodeFactors<T> mf = node_factors<true>(L, node);
  T den = 0;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int j0 = VW * (lane + c * W);
    const bool act = j0 < N;
    const int j = act ? j0 : N - VW;
    T kw[VW], ke[VW], ks[VW], kn[VW], cj[VW], dj[VW], ej[VW];
    ldv<VW>(L.kx + kxb + j, kw);
    ldv<VW>(L.kx + kxb + N + j, ke);
    ldv<VW>(L.ky + kyb + j, ks);
    ldv<VW>(L.ky + kyb + rowN + j, kn);
    ldv<VW>(L.c + j, cj);
    ldv<VW>(L.d + j, dj);
    ldv<VW>(L.e + j, ej);
#pragma unroll
    for (int u = 0; u < VW; ++u) {
      const T a = (kw[u] + ke[u]) + (ks[u] + kn[u]);
      const T ai = T(1) / a;
      const T t = cj[u] * ai * ai;
      den += act ? (mf.d * dj[u]) * t * (mf.e * ej[u]) : T(0);
    }
  }
  den = group_sum_w(den, W);
  if (lane == 0) gden[node] = L.g + den;
}

template <typename T, int W, int JM, int VW>
__global__ __launch_bounds__(kBlock) void k_node_den(LevelArgs<T> L, T* __restrict__ gden) {
  const int lane = threadIdx.x & (W - 1);
  const int node = group_slot<W>(blockIdx.x);
  if (node >= L.n * L.n) return;
  node_den<T, JM, VW>(L, gden, node, lane, W);
}

// Waves per SIMD the compiler schedules the half-sweep for.  With JM >= 4
// samples per lane a node issues ~70 loads; at 3 waves per SIMD (up to 168
// VGPRs) they are all in flight before the first wait, which measured 6% (FP64)
// and 14% (FP32) faster at 511x511, N=256 than the default 8-wave schedule.
// The prolongation variant holds more live values and stays on the default.
template <int JM, int SRC>
constexpr int halfsweep_waves() { return SRC == kProlong ? (JM <= 2 ? 4 : 8) : (JM >= 4 ? 3 : 8); }

// One half-sweep of collective Gauss-Seidel over every node of `colour`.
template <typename T, int W, int JM, int SRC, int VW, bool MK>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, halfsweep_waves<JM, SRC>())))
void k_halfsweep(LevelArgs<T> L, T* __restrict__ x, const T* __restrict__ f, int colour, T theta, int nactive,
                 const T* __restrict__ ec) {
  const int b = xcd_remap(blockIdx.x, group_blocks<W>(nactive));
  const int lane = threadIdx.x & (W - 1);
  const int slot = group_slot<W>(b);
  if (slot >= nactive) return;  // whole W-lane groups leave together
  halfsweep_node<T, JM, SRC, VW, MK>(L, x, f, colour, theta, slot, lane, W, ec);
}

}  // namespace smg
