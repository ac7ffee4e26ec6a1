// rrwalk.h -- the residual of a level restricted to the next coarser one, in
// column walks (gfx950): coarse = R (f - S x), R = P^T full weighting.
//
// The per-coarse-node form (k_residual_restrict, transfer.h) loads the 5x5 fine
// window of every coarse node; neighbouring windows overlap, so each fine value
// is requested about five times and, at 511x511 with N = 256, 1.26x the
// algorithmic bytes reach HBM.  Here a wavefront owns coarse column X, i.e. fine
// columns 2X, 2X+1, 2X+2, over a segment of coarse rows, and walks the fine rows
// upwards one at a time.  At fine row r it forms the Y and P residual rows of its
// three fine nodes (eq. (2)'s block rows with the neighbours of the previous and
// next rows), weights them across the columns by (1/2, 1, 1/2) into h(r), and
// adds h(r) to the coarse row it belongs to: coarse row K gathers
// h(2K)/2 + h(2K+1) + h(2K+2)/2.  The fine rows r-1 and r of its own columns, and
// the S faces of row r, stay in registers from the previous step, so a step
// loads the next row of x, the two side neighbours, the row's faces and
// right-hand sides once.  The U row uses
//   sum_f w_f r_U(f) = sum_f w_f (f_U(f) - g u(f)) - sum_j d_j sum_f w_f p_j(f),
// one sum over samples per coarse node.  Column 2X + 2 is formed by this wave and
// by the wave of column X + 1 (at about the same time, from L2).  No node
// factors and no domain (distributed control on the square); 64 lanes per node.
#pragma once
#include "sweep.h"

namespace smg {

template <typename T, int JM, int VW>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 2)))
void k_rr_walk(LevelArgs<T> L, const T* __restrict__ x, const T* __restrict__ f, T* __restrict__ coarse,
               int seg) {
  constexpr int kWaves = kBlock / 64;
  const int n = L.n, N = L.N;
  const int nc = (n - 1) / 2;
  __shared__ T cde[3 * 64 * JM];
  for (int j = threadIdx.x; j < N; j += kBlock) {
    cde[j] = L.c[j];
    cde[N + j] = L.d[j];
    cde[2 * N + j] = L.e[j];
  }
  __syncthreads();
  const size_t nn = (size_t)n * n, nnc = (size_t)nc * nc;
  const int npg = (nc + kWaves - 1) / kWaves, nseg = (nc + seg - 1) / seg;
  const int t = xcd_remap(blockIdx.x, npg * nseg);
  const int g = t / npg, pg = t - g * npg;
  const int X = __builtin_amdgcn_readfirstlane(pg * kWaves + (int)threadIdx.x / 64);
  const int lane = threadIdx.x & 63;
  if (X >= nc) return;   // whole waves; no barriers below
  const int K0 = g * seg, K1 = min(nc, K0 + seg);
  if (K0 >= K1) return;
  const int c0 = 2 * X;                       // columns c0, c0 + 1, c0 + 2
  auto cl = [&](int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); };
  auto nd = [&](int col, int row) { return (size_t)cl(row, n - 1) * n + cl(col, n - 1); };
  auto kxp = [&](int row, int fc) { return L.kx + ((size_t)cl(row, n - 1) * (n + 1) + cl(fc, n)) * N; };
  auto kyp = [&](int fr, int col) { return L.ky + ((size_t)cl(fr, n) * n + cl(col, n - 1)) * N; };
  const T* __restrict__ fY = f;
  const T* __restrict__ fU = f + (size_t)N * nn;
  const T* __restrict__ fP = f + (size_t)(N + 1) * nn;
  const T* __restrict__ U = x + (size_t)N * nn;
  const bool hw0 = c0 > 0, he2 = c0 + 2 < n - 1;   // W of column c0, E of column c0 + 2
  auto st_cached = [&](T* p, const T (&v)[JM]) {
#pragma unroll
    for (int c = 0; c < JM / VW; ++c) {
      const int j0 = VW * (lane + c * 64);
      if (j0 < N) {
        T t2[VW];
#pragma unroll
        for (int u = 0; u < VW; ++u) t2[u] = v[c * VW + u];
        stv<VW>(p + j0, t2);
      }
    }
  };

  // carried: x of rows r-1 and r (own columns), S faces of row r
  NodeYP<T, JM> xp[3], xc[3];
  T ks[3][JM];
  const int r0 = 2 * K0, r1 = 2 * K1;          // fine rows r0..r1
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    ld_yp<T, JM, VW>(x, nn, N, nd(c0 + c, r0 - 1), lane, xp[c]);
    ld_yp<T, JM, VW>(x, nn, N, nd(c0 + c, r0), lane, xc[c]);
    ldn<T, JM, VW>(kyp(r0, c0 + c), N, lane, ks[c]);
  }
  // coarse row being gathered: Y and P rows, the weighted p for the U row, and
  // the weighted f_U - g u
  T aY[JM], aP[JM], aQ[JM];
  T aU = T(0);
#pragma unroll
  for (int q = 0; q < JM; ++q) aY[q] = aP[q] = aQ[q] = T(0);
  for (int r = r0; r <= r1; ++r) {
    const bool hs = r > 0, hn = r < n - 1;
    // ---- loads of the step
    NodeYP<T, JM> xn[3], sw, se;
    T kxv[4][JM], kn[3][JM], fyv[3][JM], fpv[3][JM];
#pragma unroll
    for (int c = 0; c < 3; ++c) ld_yp<T, JM, VW>(x, nn, N, nd(c0 + c, r + 1), lane, xn[c]);
    ld_yp<T, JM, VW>(x, nn, N, nd(c0 - 1, r), lane, sw);
    ld_yp<T, JM, VW>(x, nn, N, nd(c0 + 3, r), lane, se);
#pragma unroll
    for (int c = 0; c < 4; ++c) ldn<T, JM, VW>(kxp(r, c0 + c), N, lane, kxv[c]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      ldn<T, JM, VW>(kyp(r + 1, c0 + c), N, lane, kn[c]);
      ldn<T, JM, VW>(fY + nd(c0 + c, r) * N, N, lane, fyv[c]);
      ldn<T, JM, VW>(fP + nd(c0 + c, r) * N, N, lane, fpv[c]);
    }
    T uu[3], fu[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      uu[c] = U[nd(c0 + c, r)];
      fu[c] = fU[nd(c0 + c, r)];
    }
    // ---- residual rows of the three nodes of row r, weighted across columns
    T hY[JM], hP[JM], hQ[JM];
#pragma unroll
    for (int q = 0; q < JM; ++q) {
      const int j = VW * (lane + (q / VW) * 64) + q % VW;
      const T cj = cde[j < N ? j : N - 1], ej = cde[2 * N + (j < N ? j : N - 1)];
      T sY = T(0), sP = T(0);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const bool hw = c > 0 || hw0, he = c < 2 || he2;
        const T kw = kxv[c][q], ke = kxv[c + 1][q], kS = ks[c][q], kN = kn[c][q];
        const T yW = c == 0 ? sw.y[q] : xc[c - 1].y[q], yE = c == 2 ? se.y[q] : xc[c + 1].y[q];
        const T pW = c == 0 ? sw.p[q] : xc[c - 1].p[q], pE = c == 2 ? se.p[q] : xc[c + 1].p[q];
        auto nbsum = [&](T vw, T ve, T vs, T vn) -> T {
          return ((hw ? kw * vw : T(0)) + (he ? ke * ve : T(0))) + ((hs ? kS * vs : T(0)) + (hn ? kN * vn : T(0)));
        };
        const T sy = nbsum(yW, yE, xp[c].y[q], xn[c].y[q]);
        const T sp = nbsum(pW, pE, xp[c].p[q], xn[c].p[q]);
        const T a = (kw + ke) + (kS + kN);
        const T yq = xc[c].y[q], pq = xc[c].p[q];
        const T rY = fyv[c][q] - (cj * yq + (a * pq - sp));
        const T rP = fpv[c][q] - ((a * yq - sy) + ej * uu[c]);
        const T w = c == 1 ? T(1) : T(0.5);
        sY += w * rY;
        sP += w * rP;
      }
      hY[q] = sY;
      hP[q] = sP;
      hQ[q] = (T(0.5) * xc[0].p[q] + xc[1].p[q]) + T(0.5) * xc[2].p[q];
    }
    const T hU = (T(0.5) * (fu[0] - L.g * uu[0]) + (fu[1] - L.g * uu[1])) + T(0.5) * (fu[2] - L.g * uu[2]);
    // ---- gather into the coarse rows: row r = 2K + 1 is the middle of coarse
    //      row K, an even row ends coarse row r/2 - 1 and starts row r/2
    if (r & 1) {
#pragma unroll
      for (int q = 0; q < JM; ++q) { aY[q] += hY[q]; aP[q] += hP[q]; aQ[q] += hQ[q]; }
      aU += hU;
    } else {
      if (r > r0) {   // coarse row K = r/2 - 1 complete
        const int K = r / 2 - 1;
        T dl = T(0);
#pragma unroll
        for (int q = 0; q < JM; ++q) {
          aY[q] += T(0.5) * hY[q];
          aP[q] += T(0.5) * hP[q];
          aQ[q] += T(0.5) * hQ[q];
          const int j = VW * (lane + (q / VW) * 64) + q % VW;
          dl += j < N ? cde[N + j] * aQ[q] : T(0);
        }
        aU += T(0.5) * hU;
        const size_t cn = (size_t)K * nc + X;
        st_cached(coarse + cn * N, aY);   // read by the next level right away
        st_cached(coarse + (size_t)(N + 1) * nnc + cn * N, aP);
        const T D = group_sum<64>(dl);
        if (lane == 0) coarse[(size_t)N * nnc + cn] = aU - D;
      }
      if (r < r1) {   // start coarse row r/2
#pragma unroll
        for (int q = 0; q < JM; ++q) { aY[q] = T(0.5) * hY[q]; aP[q] = T(0.5) * hP[q]; aQ[q] = T(0.5) * hQ[q]; }
        aU = T(0.5) * hU;
      }
    }
    // ---- shift the carried rows
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xp[c] = xc[c];
      xc[c] = xn[c];
      cpy(ks[c], kn[c]);
    }
  }
}

// The same restriction right after a Gauss-Seidel sweep xold -> xnew (theta = 1,
// red then black), from the black nodes' change alone.  Every node solve makes
// its own block row of eq. (2) exact for the neighbour values it read: a black
// node read the final reds, so its residual is zero; a red node read the old
// blacks, so its residual is what the blacks' change adds to the coupling
// terms, r_Y = sum_nb k (p_new - p_old)_nb and r_P = sum_nb k (y_new - y_old)_nb
// over its four faces; and the U row couples no neighbours, so it is zero at
// every node.  The result equals R (f - S xnew) up to the rounding of the node
// solves, without reading f, u or the red values: 2 words per node-sample of
// faces and 2 of black values (old and new) instead of 6.  Full weighting then
// takes the centre of each 3 x 3 fine window (weight 1) and its four corners
// (1/4), the red ones.  A wave owns coarse column X, walks fine rows two at a
// time (an odd row: the centre red 2X+1; an even row: the corner reds 2X and
// 2X+2) and keeps the black changes of the last two rows in registers.
template <typename T, int JM, int VW>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 2)))
void k_rr_gs_walk(LevelArgs<T> L, const T* __restrict__ xold, const T* __restrict__ xnew, T* __restrict__ coarse,
                  int seg) {
  constexpr int kWaves = kBlock / 64;
  const int n = L.n, N = L.N;
  const int nc = (n - 1) / 2;
  const size_t nn = (size_t)n * n, nnc = (size_t)nc * nc;
  const int npg = (nc + kWaves - 1) / kWaves, nseg = (nc + seg - 1) / seg;
  const int t = xcd_remap(blockIdx.x, npg * nseg);
  const int g = t / npg, pg = t - g * npg;
  const int X = __builtin_amdgcn_readfirstlane(pg * kWaves + (int)threadIdx.x / 64);
  const int lane = threadIdx.x & 63;
  if (X >= nc) return;   // whole waves; no barriers in this kernel
  const int K0 = g * seg, K1 = min(nc, K0 + seg);
  if (K0 >= K1) return;
  const int c0 = 2 * X;                       // fine columns c0, c0 + 1, c0 + 2
  auto cl = [&](int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); };
  auto nd = [&](int col, int row) { return (size_t)cl(row, n - 1) * n + cl(col, n - 1); };
  auto kxp = [&](int row, int fc) { return L.kx + ((size_t)cl(row, n - 1) * (n + 1) + cl(fc, n)) * N; };
  auto kyp = [&](int fr, int col) { return L.ky + ((size_t)cl(fr, n) * n + cl(col, n - 1)) * N; };
  // new minus old y and p of a node (indices clamped; off-grid ones are never used)
  auto dl = [&](int col, int row, NodeYP<T, JM>& o) {
    NodeYP<T, JM> a;
    ld_yp<T, JM, VW>(xnew, nn, N, nd(col, row), lane, o);
    ld_yp<T, JM, VW>(xold, nn, N, nd(col, row), lane, a);
#pragma unroll
    for (int q = 0; q < JM; ++q) {
      o.y[q] -= a.y[q];
      o.p[q] -= a.p[q];
    }
  };
  // residual of the red node (xx, r) from its neighbours' changes
  auto red = [&](int xx, int r, const T (&kw)[JM], const T (&ke)[JM], const T (&kS)[JM], const T (&kN)[JM],
                 const NodeYP<T, JM>& w, const NodeYP<T, JM>& e, const NodeYP<T, JM>& so,
                 const NodeYP<T, JM>& no, T (&rY)[JM], T (&rP)[JM]) {
    const bool hw = xx > 0, he = xx < n - 1, hs = r > 0, hn = r < n - 1;
#pragma unroll
    for (int q = 0; q < JM; ++q) {
      auto nbsum = [&](T vw, T ve, T vs, T vn) -> T {
        return ((hw ? kw[q] * vw : T(0)) + (he ? ke[q] * ve : T(0))) + ((hs ? kS[q] * vs : T(0)) + (hn ? kN[q] * vn : T(0)));
      };
      rY[q] = nbsum(w.p[q], e.p[q], so.p[q], no.p[q]);
      rP[q] = nbsum(w.y[q], e.y[q], so.y[q], no.y[q]);
    }
  };
  // even row r: the corner reds c0 and c0 + 2, weighted 1/2 across the columns;
  // E: black changes of row r at c0 - 1, c0 + 1, c0 + 3; Os, On: rows r - 1 and
  // r + 1 at c0, c0 + 2
  auto even_row = [&](int r, const NodeYP<T, JM> (&E)[3], const NodeYP<T, JM> (&Os)[2],
                      const NodeYP<T, JM> (&On)[2], T (&hY)[JM], T (&hP)[JM]) {
    T k0[JM], k1[JM], k2[JM], k3[JM], s0[JM], n0[JM], s2[JM], n2[JM];
    ldn<T, JM, VW>(kxp(r, c0), N, lane, k0);
    ldn<T, JM, VW>(kxp(r, c0 + 1), N, lane, k1);
    ldn<T, JM, VW>(kxp(r, c0 + 2), N, lane, k2);
    ldn<T, JM, VW>(kxp(r, c0 + 3), N, lane, k3);
    ldn<T, JM, VW>(kyp(r, c0), N, lane, s0);
    ldn<T, JM, VW>(kyp(r + 1, c0), N, lane, n0);
    ldn<T, JM, VW>(kyp(r, c0 + 2), N, lane, s2);
    ldn<T, JM, VW>(kyp(r + 1, c0 + 2), N, lane, n2);
    T uY[JM], uP[JM], vY[JM], vP[JM];
    red(c0, r, k0, k1, s0, n0, E[0], E[1], Os[0], On[0], uY, uP);
    red(c0 + 2, r, k2, k3, s2, n2, E[1], E[2], Os[1], On[1], vY, vP);
#pragma unroll
    for (int q = 0; q < JM; ++q) {
      hY[q] = T(0.5) * uY[q] + T(0.5) * vY[q];
      hP[q] = T(0.5) * uP[q] + T(0.5) * vP[q];
    }
  };
  auto st_cached = [&](T* p, const T (&v)[JM]) {
#pragma unroll
    for (int c = 0; c < JM / VW; ++c) {
      const int j0 = VW * (lane + c * 64);
      if (j0 < N) {
        T t2[VW];
#pragma unroll
        for (int u = 0; u < VW; ++u) t2[u] = v[c * VW + u];
        stv<VW>(p + j0, t2);
      }
    }
  };

  // the first even row 2 K0 starts coarse row K0 with weight 1/2
  NodeYP<T, JM> Ec[3], Oc[2], Op[2];
  const int rb = 2 * K0;
  dl(c0, rb - 1, Op[0]);
  dl(c0 + 2, rb - 1, Op[1]);
  dl(c0 - 1, rb, Ec[0]);
  dl(c0 + 1, rb, Ec[1]);
  dl(c0 + 3, rb, Ec[2]);
  dl(c0, rb + 1, Oc[0]);
  dl(c0 + 2, rb + 1, Oc[1]);
  T aY[JM], aP[JM];
  {
    T hY[JM], hP[JM];
    even_row(rb, Ec, Op, Oc, hY, hP);
#pragma unroll
    for (int q = 0; q < JM; ++q) { aY[q] = T(0.5) * hY[q]; aP[q] = T(0.5) * hP[q]; }
  }
  for (int K = K0; K < K1; ++K) {
    const int ro = 2 * K + 1, re = 2 * K + 2;   // the centre row, then the even row ending K
    NodeYP<T, JM> En[3], On[2];
    dl(c0 - 1, re, En[0]);
    dl(c0 + 1, re, En[1]);
    dl(c0 + 3, re, En[2]);
    dl(c0, re + 1, On[0]);
    dl(c0 + 2, re + 1, On[1]);
    // centre red (c0 + 1, ro): W, E the blacks of row ro, S, N column c0 + 1 of rows ro -/+ 1
    {
      T kw[JM], ke[JM], kS[JM], kN[JM], rY[JM], rP[JM];
      ldn<T, JM, VW>(kxp(ro, c0 + 1), N, lane, kw);
      ldn<T, JM, VW>(kxp(ro, c0 + 2), N, lane, ke);
      ldn<T, JM, VW>(kyp(ro, c0 + 1), N, lane, kS);
      ldn<T, JM, VW>(kyp(ro + 1, c0 + 1), N, lane, kN);
      red(c0 + 1, ro, kw, ke, kS, kN, Oc[0], Oc[1], Ec[1], En[1], rY, rP);
#pragma unroll
      for (int q = 0; q < JM; ++q) { aY[q] += rY[q]; aP[q] += rP[q]; }
    }
    T hY[JM], hP[JM];
    even_row(re, En, Oc, On, hY, hP);
#pragma unroll
    for (int q = 0; q < JM; ++q) { aY[q] += T(0.5) * hY[q]; aP[q] += T(0.5) * hP[q]; }
    const size_t cn = (size_t)K * nc + X;
    st_cached(coarse + cn * N, aY);   // read by the next level right away
    st_cached(coarse + (size_t)(N + 1) * nnc + cn * N, aP);
    if (lane == 0) coarse[(size_t)N * nnc + cn] = T(0);
#pragma unroll
    for (int q = 0; q < JM; ++q) { aY[q] = T(0.5) * hY[q]; aP[q] = T(0.5) * hP[q]; }
#pragma unroll
    for (int c = 0; c < 3; ++c) Ec[c] = En[c];
#pragma unroll
    for (int c = 0; c < 2; ++c) Oc[c] = On[c];
  }
}

}  // namespace smg

namespace smg {

// One FP32-refinement update fused with the next residual, in column walks:
// x_next = x + d (d: the FP32 correction of the cycle) and out = f - S x_next
// rounded to FP32, the arithmetic of residual_add_node (residual.h) per node.
// The per-node form reads x and d of all four neighbours of every node (about
// five times each overall); here a wavefront owns one column c over a segment of
// rows and walks it upwards, keeping x + d of rows r-1 and r and the S face of
// row r in registers, so a step loads x and d of (c, r+1) and of the two side
// neighbours once.  Per-block squared norms {r_Y, r_U, r_P, f} into partials
// (every wave of a block takes part in the final block sum).  No node factors,
// no domain; 64 lanes per node.
template <int JM, int VW>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 2)))
void k_residual_add_walk(LevelArgs<double> L, const double* __restrict__ x, const float* __restrict__ d,
                         double* __restrict__ xn, const double* __restrict__ f, float* __restrict__ out,
                         double* __restrict__ partials, int seg) {
  constexpr int kWaves = kBlock / 64;
  const int n = L.n, N = L.N;
  __shared__ double cde[3 * 64 * JM];
  for (int j = threadIdx.x; j < N; j += kBlock) {
    cde[j] = L.c[j];
    cde[N + j] = L.d[j];
    cde[2 * N + j] = L.e[j];
  }
  __syncthreads();
  const size_t nn = (size_t)n * n;
  const size_t oU = (size_t)N * nn, oP = (size_t)(N + 1) * nn;
  const int npg = (n + kWaves - 1) / kWaves, nseg = (n + seg - 1) / seg;
  const int t = xcd_remap(blockIdx.x, npg * nseg);
  const int g = t / npg, pg = t - g * npg;
  const int c = __builtin_amdgcn_readfirstlane(pg * kWaves + (int)threadIdx.x / 64);
  const int lane = threadIdx.x & 63;
  const int r0 = g * seg, r1 = min(n, r0 + seg);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (c < n && r0 < r1) {
    auto cl = [&](int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); };
    auto nd = [&](int col, int row) { return (size_t)cl(row, n - 1) * n + cl(col, n - 1); };
    // x + d of VW samples per access, both fields of node k
    auto xd = [&](size_t k, NodeYP<double, JM>& o) {
#pragma unroll
      for (int ch = 0; ch < JM / VW; ++ch) {
        const int j0 = VW * (lane + ch * 64);
        const int j = j0 < N ? j0 : N - VW;
        double xv[VW], xw[VW];
        float dv[VW], dw[VW];
        ldv<VW>(x + k * N + j, xv);
        ldv<VW>(d + k * N + j, dv);
        ldv<VW>(x + oP + k * N + j, xw);
        ldv<VW>(d + oP + k * N + j, dw);
#pragma unroll
        for (int u = 0; u < VW; ++u) {
          o.y[ch * VW + u] = xv[u] + (double)dv[u];
          o.p[ch * VW + u] = xw[u] + (double)dw[u];
        }
      }
    };
    const bool hw = c > 0, he = c < n - 1;
    NodeYP<double, JM> xp, xc;
    double ks[JM];
    xd(nd(c, r0 - 1), xp);
    xd(nd(c, r0), xc);
    ldn<double, JM, VW>(L.ky + ((size_t)r0 * n + c) * N, N, lane, ks);
    for (int r = r0; r < r1; ++r) {
      const bool hs = r > 0, hn = r < n - 1;
      const size_t node = (size_t)r * n + c;
      NodeYP<double, JM> xq, xw, xe;
      double kw[JM], ke[JM], kn[JM], fy[JM], fp[JM];
      xd(nd(c, r + 1), xq);
      xd(nd(c - 1, r), xw);
      xd(nd(c + 1, r), xe);
      ldn<double, JM, VW>(L.kx + ((size_t)r * (n + 1) + c) * N, N, lane, kw);
      ldn<double, JM, VW>(L.kx + ((size_t)r * (n + 1) + c + 1) * N, N, lane, ke);
      ldn<double, JM, VW>(L.ky + ((size_t)(r + 1) * n + c) * N, N, lane, kn);
      ldn<double, JM, VW>(f + node * N, N, lane, fy);
      ldn<double, JM, VW>(f + oP + node * N, N, lane, fp);
      const double u = x[oU + node] + (double)d[oU + node];
      double dsum = 0.0;
      float ry[JM], rp[JM];
#pragma unroll
      for (int q = 0; q < JM; ++q) {
        const int j = VW * (lane + (q / VW) * 64) + q % VW;
        const bool act = j < N;
        const int jj = act ? j : N - 1;
        auto nbsum = [&](double vw, double ve, double vs, double vn) {
          return ((hw ? kw[q] * vw : 0.0) + (he ? ke[q] * ve : 0.0)) + ((hs ? ks[q] * vs : 0.0) + (hn ? kn[q] * vn : 0.0));
        };
        const double sy = nbsum(xw.y[q], xe.y[q], xp.y[q], xq.y[q]);
        const double sp = nbsum(xw.p[q], xe.p[q], xp.p[q], xq.p[q]);
        const double a = (kw[q] + ke[q]) + (ks[q] + kn[q]);
        const double rY = fy[q] - (cde[jj] * xc.y[q] + (a * xc.p[q] - sp));
        const double rP = fp[q] - ((a * xc.y[q] - sy) + cde[2 * N + jj] * u);
        dsum += act ? cde[N + jj] * xc.p[q] : 0.0;
        ry[q] = (float)rY;
        rp[q] = (float)rP;
        if (act) {
          acc[0] += rY * rY;
          acc[2] += rP * rP;
          acc[3] += fy[q] * fy[q] + fp[q] * fp[q];
        }
      }
#pragma unroll
      for (int ch = 0; ch < JM / VW; ++ch) {
        const int j0 = VW * (lane + ch * 64);
        if (j0 < N) {
          double ty[VW], tp[VW];
          float sy2[VW], sp2[VW];
#pragma unroll
          for (int u2 = 0; u2 < VW; ++u2) {
            ty[u2] = xc.y[ch * VW + u2];
            tp[u2] = xc.p[ch * VW + u2];
            sy2[u2] = ry[ch * VW + u2];
            sp2[u2] = rp[ch * VW + u2];
          }
          stv_nt<VW>(xn + node * N + j0, ty);
          stv_nt<VW>(xn + oP + node * N + j0, tp);
          stv_nt<VW>(out + node * N + j0, sy2);
          stv_nt<VW>(out + oP + node * N + j0, sp2);
        }
      }
      const double D = group_sum<64>(dsum);
      if (lane == 0) {
        const double fu = f[oU + node];
        const double rU = fu - (L.g * u + D);
        xn[oU + node] = u;
        out[oU + node] = (float)rU;
        acc[1] += rU * rU;
        acc[3] += fu * fu;
      }
      xp = xc;
      xc = xq;
      cpy(ks, kn);
    }
  }
  block_sum<4>(acc);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) partials[4 * (size_t)blockIdx.x + i] = acc[i];
  }
}

}  // namespace smg

namespace smg {

// The residual or operator application of residual_node (residual.h), out =
// f - S x (mode 0) or S x (mode 1) with the same arithmetic per node, in column
// walks: the per-node form reads x of all four neighbours of every node (about
// five times each overall); here a wavefront owns one column c over a segment of
// rows and walks it upwards, keeping x of rows r-1 and r and the S face of row r
// in registers, so a step loads x of (c, r+1) and of the two side neighbours
// (shared with the neighbouring columns' waves, from L2), the row's faces and
// right-hand sides once.  FP64 faces, x and f in TX, out in TO (may be null);
// per-block squared norms {r_Y, r_U, r_P, f} into partials when given (every
// wave of a block takes part in the final block sum).  No node factors, no
// domain; 64 lanes per node.
template <typename TX, typename TO, int JM, int VW>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 2)))
void k_residual_walk(LevelArgs<double> L, const TX* __restrict__ x, const TX* __restrict__ f, TO* __restrict__ out,
                     int mode, double* __restrict__ partials, int seg) {
  constexpr int kWaves = kBlock / 64;
  const int n = L.n, N = L.N;
  __shared__ double cde[3 * 64 * JM];
  for (int j = threadIdx.x; j < N; j += kBlock) {
    cde[j] = L.c[j];
    cde[N + j] = L.d[j];
    cde[2 * N + j] = L.e[j];
  }
  __syncthreads();
  const size_t nn = (size_t)n * n;
  const size_t oU = (size_t)N * nn, oP = (size_t)(N + 1) * nn;
  const int npg = (n + kWaves - 1) / kWaves, nseg = (n + seg - 1) / seg;
  const int t = xcd_remap(blockIdx.x, npg * nseg);
  const int g = t / npg, pg = t - g * npg;
  const int c = __builtin_amdgcn_readfirstlane(pg * kWaves + (int)threadIdx.x / 64);
  const int lane = threadIdx.x & 63;
  const int r0 = g * seg, r1 = min(n, r0 + seg);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (c < n && r0 < r1) {
    auto cl = [&](int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); };
    auto nd = [&](int col, int row) { return (size_t)cl(row, n - 1) * n + cl(col, n - 1); };
    // both fields of node k, VW samples per access, widened to FP64
    auto ldx = [&](size_t k, NodeYP<double, JM>& o) {
#pragma unroll
      for (int ch = 0; ch < JM / VW; ++ch) {
        const int j0 = VW * (lane + ch * 64);
        const int j = j0 < N ? j0 : N - VW;
        TX yv[VW], pv[VW];
        ldv<VW>(x + k * N + j, yv);
        ldv<VW>(x + oP + k * N + j, pv);
#pragma unroll
        for (int u = 0; u < VW; ++u) {
          o.y[ch * VW + u] = (double)yv[u];
          o.p[ch * VW + u] = (double)pv[u];
        }
      }
    };
    const bool hw = c > 0, he = c < n - 1;
    NodeYP<double, JM> xp, xc;
    double ks[JM];
    ldx(nd(c, r0 - 1), xp);
    ldx(nd(c, r0), xc);
    ldn<double, JM, VW>(L.ky + ((size_t)r0 * n + c) * N, N, lane, ks);
    for (int r = r0; r < r1; ++r) {
      const bool hs = r > 0, hn = r < n - 1;
      const size_t node = (size_t)r * n + c;
      NodeYP<double, JM> xq, xw, xe;
      double kw[JM], ke[JM], kn[JM];
      TX fy[JM], fp[JM];
      ldx(nd(c, r + 1), xq);
      ldx(nd(c - 1, r), xw);
      ldx(nd(c + 1, r), xe);
      ldn<double, JM, VW>(L.kx + ((size_t)r * (n + 1) + c) * N, N, lane, kw);
      ldn<double, JM, VW>(L.kx + ((size_t)r * (n + 1) + c + 1) * N, N, lane, ke);
      ldn<double, JM, VW>(L.ky + ((size_t)(r + 1) * n + c) * N, N, lane, kn);
      if (mode == 0) {
        ldn<TX, JM, VW>(f + node * N, N, lane, fy);
        ldn<TX, JM, VW>(f + oP + node * N, N, lane, fp);
      }
      const double u = (double)x[oU + node];
      double dsum = 0.0;
      TO ry[JM], rp[JM];
#pragma unroll
      for (int q = 0; q < JM; ++q) {
        const int j = VW * (lane + (q / VW) * 64) + q % VW;
        const bool act = j < N;
        const int jj = act ? j : N - 1;
        auto nbsum = [&](double vw, double ve, double vs, double vn) {
          return ((hw ? kw[q] * vw : 0.0) + (he ? ke[q] * ve : 0.0)) + ((hs ? ks[q] * vs : 0.0) + (hn ? kn[q] * vn : 0.0));
        };
        const double sy = nbsum(xw.y[q], xe.y[q], xp.y[q], xq.y[q]);
        const double sp = nbsum(xw.p[q], xe.p[q], xp.p[q], xq.p[q]);
        const double a = (kw[q] + ke[q]) + (ks[q] + kn[q]);
        double rY = cde[jj] * xc.y[q] + (a * xc.p[q] - sp);
        double rP = (a * xc.y[q] - sy) + cde[2 * N + jj] * u;
        dsum += act ? cde[N + jj] * xc.p[q] : 0.0;
        double ff = 0.0;
        if (mode == 0) {
          const double fyq = (double)fy[q], fpq = (double)fp[q];
          rY = fyq - rY;
          rP = fpq - rP;
          ff = fyq * fyq + fpq * fpq;
        }
        ry[q] = (TO)rY;
        rp[q] = (TO)rP;
        if (act) {
          acc[0] += rY * rY;
          acc[2] += rP * rP;
          acc[3] += ff;
        }
      }
      if (out) {
        stn<TO, JM, VW>(out + node * N, N, lane, ry);
        stn<TO, JM, VW>(out + oP + node * N, N, lane, rp);
      }
      const double D = group_sum<64>(dsum);
      if (lane == 0) {
        double rU = L.g * u + D;
        if (mode == 0) {
          const double fu = (double)f[oU + node];
          rU = fu - rU;
          acc[3] += fu * fu;
        }
        if (out) out[oU + node] = (TO)rU;
        acc[1] += rU * rU;
      }
      xp = xc;
      xc = xq;
      cpy(ks, kn);
    }
  }
  if (partials) {
    block_sum<4>(acc);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) partials[4 * (size_t)blockIdx.x + i] = acc[i];
    }
  }
}

}  // namespace smg
