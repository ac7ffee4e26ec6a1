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

// coarse = R (f - S x) for coarse node (X, K) by one group of W lanes, without
// storing the fine residual: the Y and P residual rows of the 3x3 fine nodes
// around (2X+1, 2K+1) are formed as residual_node forms them (mode 0) and summed
// with restrict_node's weights in its order.  The y and p values of the 5x5 fine
// window (corners unused), its 24 faces and the 9 right-hand sides are loaded
// once per chunk; window entries outside the grid read a clamped in-bounds node
// and are replaced by the boundary value 0 (so every face product of a missing
// neighbour is 0, as in residual_node).  The U row uses
//   sum_f w_f r_U(f) = sum_f w_f (f_U(f) - g u(f)) - sum_j d_j sum_f w_f p_j(f),
// one sum over samples instead of nine (a different rounding order only).
// L, x, f: fine level.
// The Y and P rows of coarse node (X, K) by lane `lane` of a group of W lanes
// (W <= 256: groups wider than a wave span several waves); returns the lane's
// part of sum_j d_j sum_f w_f p_j(f), which residual_restrict_urow completes.
template <typename T, int JM, int VW = 1, bool MK = true>
__device__ __forceinline__ T residual_restrict_rows(const LevelArgs<T>& L, const T* __restrict__ x,
                                                    const T* __restrict__ f, T* __restrict__ coarse, int X,
                                                    int K, int lane, int W) {
  static_assert(JM % VW == 0, "whole chunks per lane");
  constexpr int NCH = JM / VW;
  const int n = L.n, N = L.N;
  const int nc = (n - 1) / 2;
  const size_t nn = (size_t)n * n, nnc = (size_t)nc * nc;
  const int xc = 2 * X + 1, kc = 2 * K + 1;   // fine centre, 1 <= xc, kc <= n - 2
  const int cnode = K * nc + X;
  const T* Y = x;
  const T* U = x + (size_t)N * nn;
  const T* P = x + (size_t)(N + 1) * nn;
  const T* fY = f;
  const T* fP = f + (size_t)(N + 1) * nn;
  // window row / column i <-> fine row kc - 2 + i / column xc - 2 + i; only
  // rows / columns 0 and 4 can lie outside the grid
  const bool r0in = kc >= 2, r4in = kc + 2 < n, c0in = xc >= 2, c4in = xc + 2 < n;
  const int wrow0 = r0in ? kc - 2 : 0, wrow4 = r4in ? kc + 2 : n - 1;
  const int wcol0 = c0in ? xc - 2 : 0, wcol4 = c4in ? xc + 2 : n - 1;
  auto wrow = [&](int i) { return i == 0 ? wrow0 : (i == 4 ? wrow4 : kc - 2 + i); };
  auto wcol = [&](int k) { return k == 0 ? wcol0 : (k == 4 ? wcol4 : xc - 2 + k); };
  auto win = [&](int i, int k) {
    return (i == 0 ? r0in : (i == 4 ? r4in : true)) && (k == 0 ? c0in : (k == 4 ? c4in : true));
  };
  T dw = 0;   // this lane's sum_j d_j sum_f w_f p_j(f)
  // one chunk at a time: a chunk already keeps ~90 loads per lane in flight
#pragma unroll 1
  for (int c = 0; c < NCH; ++c) {
    const int j0 = VW * (lane + c * W);
    const bool act = j0 < N;
    const int j = act ? j0 : N - VW;
    T yv[5][5][VW], pv[5][5][VW];
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        if ((i == 0 || i == 4) && (k == 0 || k == 4)) continue;
        const size_t o = ((size_t)wrow(i) * n + wcol(k)) * N + j;
        ldv<VW>(Y + o, yv[i][k]);
        ldv<VW>(P + o, pv[i][k]);
      }
    // faces: kx[row][face] for fine rows kc-1..kc+1, faces xc-1..xc+2;
    // ky[face row][col] for face rows kc-1..kc+2, columns xc-1..xc+1
    T kxv[3][4][VW], kyv[4][3][VW];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 4; ++k) ldv<VW>(L.kx + ((size_t)(kc - 1 + i) * (n + 1) + (xc - 1 + k)) * N + j, kxv[i][k]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) ldv<VW>(L.ky + ((size_t)(kc - 1 + i) * n + (xc - 1 + k)) * N + j, kyv[i][k]);
    T fyv[3][3][VW], fpv[3][3][VW];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const size_t o = ((size_t)(kc - 1 + i) * n + (xc - 1 + k)) * N + j;
        ldv<VW>(fY + o, fyv[i][k]);
        ldv<VW>(fP + o, fpv[i][k]);
      }
    T cj[VW], dj[VW], ej[VW];
    ldv<VW>(L.c + j, cj);
    ldv<VW>(L.d + j, dj);
    ldv<VW>(L.e + j, ej);
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        if ((i == 0 || i == 4) && (k == 0 || k == 4)) continue;
        if (i != 0 && i != 4 && k != 0 && k != 4) continue;
        const bool in = win(i, k);
#pragma unroll
        for (int q = 0; q < VW; ++q) {
          yv[i][k][q] = in ? yv[i][k][q] : T(0);
          pv[i][k][q] = in ? pv[i][k][q] : T(0);
        }
      }
    T sY[VW], sP[VW];
#pragma unroll
    for (int q = 0; q < VW; ++q) { sY[q] = T(0); sP[q] = T(0); }
#pragma unroll
    for (int i = 0; i < 3; ++i)       // fine row kc - 1 + i (dk = i - 1)
#pragma unroll
      for (int k = 0; k < 3; ++k) {   // fine column xc - 1 + k (dx = k - 1)
        const int wi = i + 1, wk = k + 1;
        // a fine node outside the domain has no residual rows
        const NodeFactors<T> nf = node_factors<MK>(L, (size_t)(kc - 1 + i) * n + (xc - 1 + k));
        const T w = node_live(nf) ? (T)(lin_w(k - 1) * lin_w(i - 1)) : T(0);
        const T u = U[(size_t)(kc - 1 + i) * n + (xc - 1 + k)];
        const T mf = nf.e;
#pragma unroll
        for (int q = 0; q < VW; ++q) {
          const T kw = kxv[i][k][q], ke = kxv[i][k + 1][q], ks = kyv[i][k][q], kn = kyv[i + 1][k][q];
          auto nbsum = [&](T vw, T ve, T vs, T vn) -> T { return (kw * vw + ke * ve) + (ks * vs + kn * vn); };
          const T sy = nbsum(yv[wi][wk - 1][q], yv[wi][wk + 1][q], yv[wi - 1][wk][q], yv[wi + 1][wk][q]);
          const T sp = nbsum(pv[wi][wk - 1][q], pv[wi][wk + 1][q], pv[wi - 1][wk][q], pv[wi + 1][wk][q]);
          const T a = (kw + ke) + (ks + kn);
          const T yq = yv[wi][wk][q], pq = pv[wi][wk][q];
          const T rY = fyv[i][k][q] - (cj[q] * yq + (a * pq - sp));
          const T rP = fpv[i][k][q] - ((a * yq - sy) + (mf * ej[q]) * u);
          sY[q] += w * rY;
          sP[q] += w * rP;
        }
      }
#pragma unroll
    for (int q = 0; q < VW; ++q) {
      // restricted p of this sample, weighted like the residual rows
      T wp = 0;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k)
          wp += ((T)(lin_w(k - 1) * lin_w(i - 1)) * node_factors<MK>(L, (size_t)(kc - 1 + i) * n + (xc - 1 + k)).d) *
                pv[i + 1][k + 1][q];
      dw += act ? dj[q] * wp : T(0);
    }
    if (act) {
      // a coarse node outside the domain (the fine node it sits on is) has no equation
      const bool clive = node_live(node_factors<MK>(L, (size_t)kc * n + xc));
#pragma unroll
      for (int q = 0; q < VW; ++q) {
        sY[q] = clive ? sY[q] : T(0);
        sP[q] = clive ? sP[q] : T(0);
      }
      stv<VW>(coarse + (size_t)cnode * N + j, sY);
      stv<VW>(coarse + (size_t)(N + 1) * nnc + (size_t)cnode * N + j, sP);
    }
  }
  return dw;
}

// U row of coarse node (X, K): sum_f w_f (f_U(f) - g u(f)) - D, with D the
// group's sum of the residual_restrict_rows partials.  The U residual is
// restricted within the control space: fine nodes without a control carry
// weight 0, and a coarse node whose coincident fine node has none gets a zero
// U row (coarse factors by injection: the coarse node has none either).
template <typename T, bool MK = true>
__device__ __forceinline__ void residual_restrict_urow(const LevelArgs<T>& L, const T* __restrict__ x,
                                                       const T* __restrict__ f, T* __restrict__ coarse, int X,
                                                       int K, T D) {
  const int n = L.n, N = L.N, nc = (n - 1) / 2;
  const size_t nn = (size_t)n * n;
  const int xc = 2 * X + 1, kc = 2 * K + 1;
  const T* U = x + (size_t)N * nn;
  const T* fU = f + (size_t)N * nn;
  T sU = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const size_t o = (size_t)(kc - 1 + i) * n + (xc - 1 + k);
      const T w = node_control(node_factors<MK>(L, o)) ? (T)(lin_w(k - 1) * lin_w(i - 1)) : T(0);
      sU += w * (fU[o] - L.g * U[o]);
    }
  const bool cctrl = node_control(node_factors<MK>(L, (size_t)kc * n + xc));
  coarse[(size_t)N * nc * nc + (size_t)K * nc + X] = cctrl ? sU - D : T(0);
}

// Group of W <= 64 lanes (one wave or part of one) per coarse node.
template <typename T, int JM, int VW = 1, bool MK = true>
__device__ __forceinline__ void residual_restrict_node(const LevelArgs<T>& L, const T* __restrict__ x,
                                                       const T* __restrict__ f, T* __restrict__ coarse,
                                                       int slot, int lane, int W, int cstrip) {
  int X, K;
  strip_node(slot, (L.n - 1) / 2, cstrip, X, K);
  const T dw = residual_restrict_rows<T, JM, VW, MK>(L, x, f, coarse, X, K, lane, W);
  const T D = group_sum_w(dw, W);
  if (lane == 0) residual_restrict_urow<T, MK>(L, x, f, coarse, X, K, D);
}

// coarse = R (f - S x) over every coarse node, W lanes per node (W <= 256; a
// node of W > 64 lanes spans W / 64 waves whose partial sums meet in LDS).
template <typename T, int W, int JM, int VW, bool MK>
__global__ __launch_bounds__(kBlock) void k_residual_restrict(LevelArgs<T> L, const T* __restrict__ x,
                                                              const T* __restrict__ f, T* __restrict__ coarse,
                                                              int cstrip) {
  static_assert(W >= 1 && W <= kBlock && (W & (W - 1)) == 0, "power-of-two group");
  const int nc = (L.n - 1) / 2;
  const int b = xcd_remap(blockIdx.x, group_blocks<W>(nc * nc));
  const int lane = threadIdx.x & (W - 1);
  const int slot = group_slot<W>(b);
  if constexpr (W <= 64) {
    if (slot >= nc * nc) return;
    residual_restrict_node<T, JM, VW, MK>(L, x, f, coarse, slot, lane, W, cstrip);
  } else {
    __shared__ T part[kBlock / 64];
    const bool live = slot < nc * nc;
    int X = 0, K = 0;
    if (live) strip_node(slot, nc, cstrip, X, K);
    T dw = live ? residual_restrict_rows<T, JM, VW, MK>(L, x, f, coarse, X, K, lane, W) : T(0);
    dw = group_sum<64>(dw);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = dw;
    __syncthreads();
    if (live && lane == 0) {
      const int w0 = (threadIdx.x >> 6);
      T D = part[w0];
      for (int q = 1; q < W / 64; ++q) D += part[w0 + q];
      residual_restrict_urow<T, MK>(L, x, f, coarse, X, K, D);
    }
  }
}

// U entries of the n x n level vector u zeroed at nodes without a control,
// read from factors mk of an nm x nm level at node (s k + s - 1, s x + s - 1)
// (s = 1: the same level; s = 2: the coincident node of the finer level).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_control_rows(int n, int s, int nm, const T* __restrict__ mk,
                                                         T* __restrict__ u) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n * n) return;
  const int k = i / n, x = i - k * n;
  if (!node_control(load_factors(mk, (size_t)(s * k + s - 1) * nm + (s * x + s - 1)))) u[i] = T(0);
}

template <typename T, int W, int JM, int VW>
__global__ __launch_bounds__(kBlock) void k_restrict(int nf, int N, const T* __restrict__ fine,
                                                     T* __restrict__ coarse, int cstrip) {
  const int nc = (nf - 1) / 2;
  const int b = xcd_remap(blockIdx.x, group_blocks<W>(nc * nc));
  const int lane = threadIdx.x & (W - 1);
  const int slot = group_slot<W>(b);
  if (slot >= nc * nc) return;
  restrict_node<T, JM, VW>(nf, N, fine, coarse, slot, lane, W, cstrip);
}

// fine += P coarse, bilinear interpolation gathered per fine node; with MK the
// U block only at fine nodes with a control (fmk: the fine level's factors).
template <typename T, int W, int JM, bool MK>
__global__ __launch_bounds__(kBlock) void k_prolong_add(int nc, int N, const T* __restrict__ coarse,
                                                        T* __restrict__ fine, const T* __restrict__ fmk) {
  const int nf = 2 * nc + 1;
  const size_t nnf = (size_t)nf * nf, nnc = (size_t)nc * nc;
  const int b = xcd_remap(blockIdx.x, group_blocks<W>((int)nnf));
  const int lane = threadIdx.x & (W - 1);
  const int slot = group_slot<W>(b);
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
    if constexpr (MK) {
      if (!node_control(load_factors(fmk, slot))) return;
    }
    const T* cU = coarse + (size_t)N * nnc;
    T sU = 0;
    for (int a = 0; a < nk; ++a)
      for (int c = 0; c < nx; ++c) sU += wk[a] * wx[c] * cU[(size_t)ck[a] * nc + cx[c]];
    fine[(size_t)N * nnf + slot] += sU;
  }
}

}  // namespace smg
