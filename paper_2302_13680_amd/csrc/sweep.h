// sweep.h -- one whole red+black sweep of collective Gauss-Seidel in a single
// launch, out of place (xin -> xout), every face coefficient read once (gfx950).
//
// A half-sweep per colour reads every face twice per sweep (each face borders
// one red and one black node).  Here a wavefront owns a pair of grid columns
// (a, a+1) over a segment of rows [r0, r1) and walks it upwards.  At step s it
//   1. solves the red node of row s outside the pair that borders the pair's
//      black node of row s (a "halo" red, owned by the neighbouring pair and
//      recomputed here, so that no wave waits for another),
//   2. solves its own red node of row s (column a + (s & 1)),
//   3. solves its own black node of row s - 1 in the same column, whose four
//      red neighbours are now all in registers: the own reds of steps s and
//      s - 2 (same column), the own red of step s - 1 (other column of the
//      pair) and the halo red of step s - 1.
// Reds read their black neighbours from xin (the values before the sweep), so
// the result is the red half-sweep followed by the black half-sweep, node for
// node the arithmetic of halfsweep_node (smoother.h).  The coarse correction
// ahead of post-smoothing is a separate pass over the black nodes only
// (k_prolong_black below; the reds never read the old red values): folded into
// the sweep as in the half-sweeps, the reds' interpolation of their four black
// neighbours re-read the coarse vector and cost 1.79 ms per sweep at 511x511,
// N=256 FP64 against 0.90 ms for a plain sweep; the black pass plus a plain
// sweep take about 1.2 ms, and 11 FP64 V-cycles to 1e-8 went from 90.4 to
// 83.0 ms.  Faces, black values and
// right-hand sides that two solves of the same wave need are kept in registers
// between steps; what a wave shares with its neighbour pair is read by both
// from memory at about the same time (neighbouring pairs run in the same
// workgroup or on the same XCD), so it is fetched from HBM once.
//
// Needs 64 lanes per node (N > 32 samples, or N > 64 in FP32 pairs), theta = 1,
// no node factors (distributed control on the square).  Segments: the row
// below r0 and the row r1 are solved as reds too (not written), for the blacks
// at the segment's ends.
#pragma once
#include "smoother.h"

namespace smg {

// One field of one node, JM samples per lane (chunks of VW, see common.h).
template <typename T, int JM, int VW>
__device__ __forceinline__ void ldn(const T* __restrict__ p, int N, int lane, T (&v)[JM]) {
#pragma unroll
  for (int c = 0; c < JM / VW; ++c) {
    const int j0 = VW * (lane + c * 64);
    T t[VW];
    ldv<VW>(p + (j0 < N ? j0 : N - VW), t);
#pragma unroll
    for (int u = 0; u < VW; ++u) v[c * VW + u] = t[u];
  }
}
template <typename T, int JM, int VW>
__device__ __forceinline__ void stn(T* __restrict__ p, int N, int lane, const T (&v)[JM]) {
#pragma unroll
  for (int c = 0; c < JM / VW; ++c) {
    const int j0 = VW * (lane + c * 64);
    if (j0 < N) {
      T t[VW];
#pragma unroll
      for (int u = 0; u < VW; ++u) t[u] = v[c * VW + u];
      stv_nt<VW>(p + j0, t);
    }
  }
}
template <typename T, int JM>
__device__ __forceinline__ void cpy(T (&d)[JM], const T (&s)[JM]) {
#pragma unroll
  for (int q = 0; q < JM; ++q) d[q] = s[q];
}

template <typename T, int JM>
struct NodeYP {
  T y[JM], p[JM];
};

// Where a sweep's fields live.
template <typename T>
struct SweepPtrs {
  const T* __restrict__ xin;   // iterate before the sweep (unused with kZero)
  T* __restrict__ xout;        // iterate after the sweep
  const T* __restrict__ f;
};

// The node solve of eq. solution_reduced_system in two phases, arithmetic as
// halfsweep_node with MK = false and theta = 1: prep forms the right-hand sides
// b_P, b_Y, 1/a_j and this lane's part of the sum over samples from the faces,
// the neighbour values (missing ones discarded by the boundary selects) and the
// node's f; finish completes the sum over the 64 lanes and the update.  Two
// independent nodes can then share the latency of their sums.  SRC: kPlain or
// kZero (no neighbour terms).  cde: c_j, d_j, e_j in LDS.
template <typename T, int JM>
struct NodePrep {
  T bP[JM], bY[JM], ia[JM], cq[JM], eq[JM];
  T num;
};

template <typename T, int JM, int VW, int SRC>
__device__ __forceinline__ void prep_node(const LevelArgs<T>& L, const T* cde, int xx,
                                          int k, int lane, const T (&kw)[JM], const T (&ke)[JM],
                                          const T (&ks)[JM], const T (&kn)[JM], const NodeYP<T, JM>& w,
                                          const NodeYP<T, JM>& e, const NodeYP<T, JM>& s,
                                          const NodeYP<T, JM>& nb, const T (&fy)[JM], const T (&fp)[JM],
                                          NodePrep<T, JM>& o) {
  constexpr int NCH = JM / VW;
  const int n = L.n, N = L.N;
  static_assert(SRC == kPlain || SRC == kZero, "one-launch sweep: plain or zero-start neighbours");
  const bool hw = xx > 0, he = xx < n - 1, hs = k > 0, hn = k < n - 1;
  o.num = T(0);
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int j0 = VW * (lane + c * 64);
    const bool act = j0 < N;
    const int j = act ? j0 : N - VW;
    T cj[VW], dj[VW], ej[VW];
    ldv<VW>(cde + j, cj);
    ldv<VW>(cde + N + j, dj);
    ldv<VW>(cde + 2 * N + j, ej);
#pragma unroll
    for (int u = 0; u < VW; ++u) {
      const int q = c * VW + u;
      auto nbsum = [&](T vw, T ve, T vs, T vn) -> T {
        return ((hw ? kw[q] * vw : T(0)) + (he ? ke[q] * ve : T(0))) +
               ((hs ? ks[q] * vs : T(0)) + (hn ? kn[q] * vn : T(0)));
      };
      T sy = T(0), sp = T(0);
      if constexpr (SRC != kZero) {
        sy = nbsum(w.y[q], e.y[q], s.y[q], nb.y[q]);
        sp = nbsum(w.p[q], e.p[q], s.p[q], nb.p[q]);
      }
      const T a = (kw[q] + ke[q]) + (ks[q] + kn[q]);
      const T ai = T(1) / a;
      const T bp = fy[q] + sp, by = fp[q] + sy;
      const T t = cj[u] * ai * ai;
      o.num += act ? (T(1) * dj[u]) * (t * by - ai * bp) : T(0);
      o.bP[q] = bp; o.bY[q] = by; o.ia[q] = ai; o.cq[q] = cj[u]; o.eq[q] = T(1) * ej[u];
    }
  }
}

template <typename T, int JM>
__device__ __forceinline__ void finish_node(const NodePrep<T, JM>& o, T num, T fu, T gd, NodeYP<T, JM>& out,
                                            T& uout) {
  const T un = (fu + num) / gd;
#pragma unroll
  for (int q = 0; q < JM; ++q) {
    out.y[q] = o.ia[q] * (o.bY[q] - o.eq[q] * un);
    out.p[q] = o.ia[q] * (o.bP[q] - o.cq[q] * out.y[q]);
  }
  uout = un;
}

// y and p of node `node` from vector v (a Y block and a P block of nn nodes).
template <typename T, int JM, int VW>
__device__ __forceinline__ void ld_yp(const T* __restrict__ v, size_t nn, int N, size_t node, int lane,
                                      NodeYP<T, JM>& o) {
  ldn<T, JM, VW>(v + node * N, N, lane, o.y);
  ldn<T, JM, VW>(v + (size_t)(N + 1) * nn + node * N, N, lane, o.p);
}
template <typename T, int JM, int VW>
__device__ __forceinline__ void st_ypu(T* __restrict__ v, size_t nn, int N, size_t node, int lane,
                                       const NodeYP<T, JM>& o, T u) {
  stn<T, JM, VW>(v + node * N, N, lane, o.y);
  stn<T, JM, VW>(v + (size_t)(N + 1) * nn + node * N, N, lane, o.p);
  if (lane == 0) v[(size_t)N * nn + node] = u;
}

// x += P e_c at the black nodes (x + k odd) only, Y and P blocks: the coarse
// correction of Alg. 1 ahead of a one-launch post-smoothing sweep.  The sweep's
// reds read only black neighbours, its blacks only the new reds, and no solve
// reads a node's own old value or any u, so the red values and U block of x
// after the correction are never used.  A black node lies on a coarse edge:
// (P e)(x, k) is the mean of the two coarse nodes at its ends (zero outside the
// coarse grid).  One wave per black node, 64 lanes, JM samples per lane.
template <typename T, int JM, int VW>
__global__ __launch_bounds__(kBlock) void k_prolong_black(int n, int N, const T* __restrict__ ec,
                                                          T* __restrict__ x) {
  constexpr int kWaves = kBlock / 64;
  const int nc = (n - 1) / 2;
  const size_t nn = (size_t)n * n, nnc = (size_t)nc * nc;
  const int nblack = (int)(nn / 2), nb = (nblack + kWaves - 1) / kWaves;
  const int slot = __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, nb) * kWaves + (int)threadIdx.x / 64);
  const int lane = threadIdx.x & 63;
  if (slot >= nblack) return;
  // rows 2m and 2m+1 hold n blacks: (n-1)/2 at odd x in row 2m, (n+1)/2 at even x in row 2m+1
  const int m = slot / n, rem = slot - m * n, h = (n - 1) / 2;
  const bool krow_even = rem < h;
  const int k = krow_even ? 2 * m : 2 * m + 1, xx = krow_even ? 2 * rem + 1 : 2 * (rem - h);
  // the two coarse ends: along the row (x even, k odd) or along the column (x odd, k even)
  int X0, K0, X1, K1;
  if (krow_even) { X0 = X1 = (xx - 1) / 2; K0 = k / 2 - 1; K1 = k / 2; }
  else { K0 = K1 = (k - 1) / 2; X0 = xx / 2 - 1; X1 = xx / 2; }
  const bool in0 = X0 >= 0 && K0 >= 0, in1 = X1 < nc && K1 < nc;
  const size_t c0 = in0 ? (size_t)K0 * nc + X0 : 0, c1 = in1 ? (size_t)K1 * nc + X1 : 0;
  const size_t node = (size_t)k * n + xx;
  T ey0[JM], ey1[JM], ep0[JM], ep1[JM], y[JM], p[JM];
  ldn<T, JM, VW>(ec + c0 * N, N, lane, ey0);
  ldn<T, JM, VW>(ec + c1 * N, N, lane, ey1);
  ldn<T, JM, VW>(ec + (size_t)(N + 1) * nnc + c0 * N, N, lane, ep0);
  ldn<T, JM, VW>(ec + (size_t)(N + 1) * nnc + c1 * N, N, lane, ep1);
  ldn<T, JM, VW>(x + node * N, N, lane, y);
  ldn<T, JM, VW>(x + (size_t)(N + 1) * nn + node * N, N, lane, p);
#pragma unroll
  for (int q = 0; q < JM; ++q) {
    y[q] += T(0.5) * ((in0 ? ey0[q] : T(0)) + (in1 ? ey1[q] : T(0)));
    p[q] += T(0.5) * ((in0 ? ep0[q] : T(0)) + (in1 ? ep1[q] : T(0)));
  }
  stn<T, JM, VW>(x + node * N, N, lane, y);
  stn<T, JM, VW>(x + (size_t)(N + 1) * nn + node * N, N, lane, p);
}

// Pair-walking waves: kBlock / 64 consecutive pairs of one row segment per
// workgroup; blocks remapped so that each XCD takes contiguous segments.  Every
// load of a step is issued before its arithmetic (one memory round trip per
// step); c_j, d_j, e_j sit in LDS.  ALL = false writes the blacks' y and p only:
// no solve reads a red value, a u or a node's own old value, so only the last
// sweep before a consumer of the whole vector needs to store them (the others
// feed the next sweep, the restriction from the blacks' change and the black
// prolongation): 7 words per node-sample instead of 8.
template <typename T, int JM, int VW, int SRC, bool ALL = true>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 2)))
void k_sweep_fused(LevelArgs<T> L, SweepPtrs<T> P, int seg_rows) {
  constexpr int kWaves = kBlock / 64;
  const int n = L.n, N = L.N;
  __shared__ T cde[3 * 64 * JM];
  for (int j = threadIdx.x; j < N; j += kBlock) {
    cde[j] = L.c[j];
    cde[N + j] = L.d[j];
    cde[2 * N + j] = L.e[j];
  }
  __syncthreads();
  const size_t nn = (size_t)n * n;
  const int npair = (n + 1) / 2, npg = (npair + kWaves - 1) / kWaves;
  const int nseg = (n + seg_rows - 1) / seg_rows;
  const int t = xcd_remap(blockIdx.x, npg * nseg);
  const int g = t / npg, pg = t - g * npg;
  const int pair = __builtin_amdgcn_readfirstlane(pg * kWaves + (int)threadIdx.x / 64);
  const int lane = threadIdx.x & 63;
  if (pair >= npair) return;   // whole waves; no barriers below
  const int a = 2 * pair;
  const int r0 = g * seg_rows, r1 = min(n, r0 + seg_rows);
  auto colok = [&](int x) { return x >= 0 && x < n; };
  auto cl = [&](int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); };
  // faces kx(k, f) (f = 0..n) and ky(g, x) (g = 0..n); indices clamped into the arrays
  auto kxp = [&](int k, int f) { return L.kx + ((size_t)cl(k, n - 1) * (n + 1) + cl(f, n)) * N; };
  auto kyp = [&](int g2, int x) { return L.ky + ((size_t)cl(g2, n) * n + cl(x, n - 1)) * N; };
  auto nd = [&](int x, int k) { return (size_t)cl(k, n - 1) * n + cl(x, n - 1); };
  const T* __restrict__ fY = P.f;
  const T* __restrict__ fU = P.f + (size_t)N * nn;
  const T* __restrict__ fP = P.f + (size_t)(N + 1) * nn;

  // carried between steps
  NodeYP<T, JM> R1, R2, H1;       // own red of step s-1, s-2; halo red of step s-1
  T kxin1[JM], kxh1[JM];          // faces of row s-1: kx(a+1), and kx between xo and the halo
  T kyn1[JM], kyn2[JM];           // ky(s, xr(s-1)), ky(s-1, xr(s-2)): N faces of the own reds
  NodeYP<T, JM> obIn, obS;        // old blacks: (xo, s) and (xr, s-1)
  bool carry = false;             // obIn / obS hold this step's values
#pragma unroll
  for (int q = 0; q < JM; ++q) {
    kxin1[q] = kxh1[q] = kyn2[q] = T(0);
    R1.y[q] = R1.p[q] = R2.y[q] = R2.p[q] = H1.y[q] = H1.p[q] = T(0);
    obIn.y[q] = obIn.p[q] = obS.y[q] = obS.p[q] = T(0);
  }
  const int s_first = r0 > 0 ? r0 - 1 : 0;
  // the S face of the first black when no earlier red supplied it (r0 = 0)
  ldn<T, JM, VW>(kyp(s_first, a + ((s_first + 1) & 1)), N, lane, kyn1);
  for (int s = s_first; s <= r1; ++s) {
    const bool odd = s & 1;
    const int xr = a + (odd ? 1 : 0), xo = a + (odd ? 0 : 1);
    const bool row = s < n;                                 // row s exists
    const bool red_ok = row && colok(xr);                    // own red (xr, s)
    const bool blk = s - 1 >= r0 && colok(xr);              // own black (xr, s-1), s - 1 < r1 always
    const int xh = odd ? a - 1 : a + 2;                      // halo column (next to xo)
    const bool halo_ok = s >= r0 && s < r1 && colok(xo) && colok(xh);
    const size_t nh = nd(xh, s), nr = nd(xr, s), nb = nd(xr, s - 1);
    // ---- every load of the step: faces of row s around the pair (kx(a..a+2),
    // the halo's outer kx, the ky faces of the own and halo columns), the old
    // blacks the two reds read, the right-hand sides of the three nodes
    T F0[JM], F1[JM], F2[JM], Fh[JM], kys0[JM], kyn0[JM], ksh[JM], knh[JM];
    NodeYP<T, JM> vo, vs, vn, vq, obN;
    T fyh[JM], fph[JM], fyr[JM], fpr[JM], fyb[JM], fpb[JM];
    ldn<T, JM, VW>(kxp(s, a), N, lane, F0);
    ldn<T, JM, VW>(kxp(s, a + 1), N, lane, F1);
    ldn<T, JM, VW>(kxp(s, a + 2), N, lane, F2);
    ldn<T, JM, VW>(kxp(s, odd ? a - 1 : a + 3), N, lane, Fh);
    ldn<T, JM, VW>(kyp(s, xr), N, lane, kys0);        // also the black's N face
    ldn<T, JM, VW>(kyp(s + 1, xr), N, lane, kyn0);
    ldn<T, JM, VW>(kyp(s, xh), N, lane, ksh);
    ldn<T, JM, VW>(kyp(s + 1, xh), N, lane, knh);
    ldn<T, JM, VW>(fY + nh * N, N, lane, fyh);
    ldn<T, JM, VW>(fP + nh * N, N, lane, fph);
    ldn<T, JM, VW>(fY + nr * N, N, lane, fyr);
    ldn<T, JM, VW>(fP + nr * N, N, lane, fpr);
    ldn<T, JM, VW>(fY + nb * N, N, lane, fyb);
    ldn<T, JM, VW>(fP + nb * N, N, lane, fpb);
    const T fuh = fU[nh], gdh = L.gden[nh], fur = fU[nr], gdr = L.gden[nr], fub = fU[nb], gdb = L.gden[nb];
    if constexpr (SRC != kZero) {
      ld_yp<T, JM, VW>(P.xin, nn, N, nd(odd ? xh - 1 : xh + 1, s), lane, vo);
      ld_yp<T, JM, VW>(P.xin, nn, N, nd(xh, s - 1), lane, vs);
      ld_yp<T, JM, VW>(P.xin, nn, N, nd(xh, s + 1), lane, vn);
      ld_yp<T, JM, VW>(P.xin, nn, N, nd(odd ? xr + 1 : xr - 1, s), lane, vq);
      ld_yp<T, JM, VW>(P.xin, nn, N, nd(xr, s + 1), lane, obN);
      if (!carry) {   // first step: the carried old blacks, read afresh
        ld_yp<T, JM, VW>(P.xin, nn, N, nd(xo, s), lane, obIn);
        ld_yp<T, JM, VW>(P.xin, nn, N, nd(xr, s - 1), lane, obS);
      }
    } else {
#pragma unroll
      for (int q = 0; q < JM; ++q)
        vo.y[q] = vo.p[q] = vs.y[q] = vs.p[q] = vn.y[q] = vn.p[q] = vq.y[q] = vq.p[q] = obN.y[q] = obN.p[q] = T(0);
    }
    // ---- 1+2. halo red (xh, s) and own red (xr, s), their sums together
    NodePrep<T, JM> ph, pr;
    if (odd) {
      prep_node<T, JM, VW, SRC>(L, cde, xh, s, lane, Fh, F0, ksh, knh, vo, obIn, vs, vn, fyh, fph, ph);
      prep_node<T, JM, VW, SRC>(L, cde, xr, s, lane, F1, F2, kys0, kyn0, obIn, vq, obS, obN, fyr, fpr, pr);
    } else {
      prep_node<T, JM, VW, SRC>(L, cde, xh, s, lane, F2, Fh, ksh, knh, obIn, vo, vs, vn, fyh, fph, ph);
      prep_node<T, JM, VW, SRC>(L, cde, xr, s, lane, F0, F1, kys0, kyn0, vq, obIn, obS, obN, fyr, fpr, pr);
    }
#pragma unroll
    for (int q = 0; q < JM; ++q) asm volatile("" ::"v"(ph.eq[q]), "v"(pr.eq[q]));
    const T numh = group_sum<64>(ph.num), numr = group_sum<64>(pr.num);
    NodeYP<T, JM> H0, R0;
    T uH, uR;
    finish_node<T, JM>(ph, numh, fuh, gdh, H0, uH);
    finish_node<T, JM>(pr, numr, fur, gdr, R0, uR);
    if (!halo_ok) {   // no halo red this step: nothing for the next black
#pragma unroll
      for (int q = 0; q < JM; ++q) H0.y[q] = H0.p[q] = T(0);
    }
    if constexpr (ALL) {
      if (red_ok && s >= r0 && s < r1) st_ypu<T, JM, VW>(P.xout, nn, N, (size_t)s * n + xr, lane, R0, uR);
    }
    // ---- 3. own black (xr, s-1): W/E = pair partner (R1) and halo (H1) of step
    //         s-1, S = own red of step s-2 (R2), N = own red of step s (R0)
    if (blk) {
      NodePrep<T, JM> pb;
      if (odd)
        prep_node<T, JM, VW, kPlain>(L, cde, xr, s - 1, lane, kxin1, kxh1, kyn2, kys0, R1, H1, R2, R0, fyb, fpb,
                                     pb);
      else
        prep_node<T, JM, VW, kPlain>(L, cde, xr, s - 1, lane, kxh1, kxin1, kyn2, kys0, H1, R1, R2, R0, fyb, fpb,
                                     pb);
#pragma unroll
      for (int q = 0; q < JM; ++q) asm volatile("" ::"v"(pb.eq[q]));
      NodeYP<T, JM> Bv;
      T uB;
      finish_node<T, JM>(pb, group_sum<64>(pb.num), fub, gdb, Bv, uB);
      if constexpr (ALL) {
        st_ypu<T, JM, VW>(P.xout, nn, N, (size_t)(s - 1) * n + xr, lane, Bv, uB);
      } else {
        const size_t node = (size_t)(s - 1) * n + xr;
        stn<T, JM, VW>(P.xout + node * N, N, lane, Bv.y);
        stn<T, JM, VW>(P.xout + (size_t)(N + 1) * nn + node * N, N, lane, Bv.p);
      }
    }
    // ---- shift the carried values to step s+1
    R2 = R1; R1 = R0; H1 = H0;
    cpy(kyn2, kyn1); cpy(kyn1, kyn0);
    cpy(kxin1, F1); cpy(kxh1, odd ? F0 : F2);
    obS = obIn; obIn = obN;
    carry = red_ok;
  }
}

}  // namespace smg
