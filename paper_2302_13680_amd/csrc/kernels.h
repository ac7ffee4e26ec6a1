// kernels.h -- gfx950 kernels of the collective multigrid V-cycle.
//
// Layout (see include/smg.h): samples innermost.  A level vector is
//   Y [n][n][N] | U [n][n] | P [n][n][N];  faces kx [n][n+1][N], ky [n+1][n][N].
// A node's N samples are contiguous, so a group of W lanes of one wavefront
// (W = 1..64, a power of two) holds one node and each lane handles JM samples
// j = lane, lane + W, ...; the reductions over samples that the node solve and
// the control row need are butterfly shuffles inside that group.  Every lane
// of a group ends with the bitwise-same sum (IEEE addition is commutative), so
// all lanes agree on u_i.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smg {

constexpr int kBlock = 256;
constexpr int kNumXcd = 8;
constexpr int kMaxCoarse = 49;   // unknowns per field on the coarsest grid (n_c <= 7)
constexpr int kMaxBasis = 32;    // Krylov vectors handled by one multi-dot pass
constexpr int kPartials = 1024;  // fixed block count of grid-stride reductions

template <typename T>
struct LevelArgs {
  int n, N;
  const T* __restrict__ kx;
  const T* __restrict__ ky;
  const T* __restrict__ c;
  const T* __restrict__ d;
  const T* __restrict__ e;
  T g;
};

// MI355X dispatches workgroup b to XCD b % 8.  Remap so that every XCD works on
// one contiguous range of logical tiles (neighbouring grid rows then share that
// XCD's L2).  Bijective on [0, nblocks).
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
  const int q = nblocks / kNumXcd, r = nblocks % kNumXcd;
  const int xcd = b % kNumXcd, idx = b / kNumXcd;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

template <int W, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
  return v;
}

// Block-wide sum of NV values, deterministic order; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
  __shared__ double red[kBlock / 64][NV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = group_sum<64>(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wv][i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = red[0][i];
      for (int w = 1; w < kBlock / 64; ++w) s += red[w][i];
      v[i] = s;
    }
  }
}

// Node (x, k) of the slot-th node of colour `colour` ((x + k) % 2 == colour),
// n odd, row-major order.  A pair of rows holds n nodes of each colour.
__device__ __forceinline__ void colour_node(int slot, int n, int colour, int& x, int& k) {
  const int pr = slot / n, rem = slot - pr * n;
  const int c0 = (n - colour + 1) >> 1;  // nodes of this colour on the even row of the pair
  if (rem < c0) { k = 2 * pr; x = colour + 2 * rem; }
  else { k = 2 * pr + 1; x = (1 - colour) + 2 * (rem - c0); }
}

__host__ __device__ inline int colour_count(int n, int colour) {
  return ((n - 1) / 2) * n + (n - colour + 1) / 2;
}

// ---------------------------------------------------------------- smoother
// One half-sweep of collective Gauss-Seidel: each node of `colour` is replaced
// by the solution of its (2N+1)x(2N+1) system (eq. solution_reduced_system)
// with the opposite-colour neighbours fixed:
//   bP_j = fY_j + sum_nb k_nb p_j,nb      (rhs of the C_j / A_j^T row)
//   bY_j = fP_j + sum_nb k_nb y_j,nb      (rhs of the A_j / E_j row)
//   u    = (fU + sum_j d_j (c_j bY_j / a_j^2 - bP_j / a_j)) / (g + sum_j d_j c_j e_j / a_j^2)
//   y_j  = (bY_j - e_j u) / a_j,   p_j = (bP_j - c_j y_j) / a_j
template <typename T, int W, int JM>
__global__ __launch_bounds__(kBlock) void k_halfsweep(LevelArgs<T> L, T* __restrict__ x,
                                                      const T* __restrict__ f, int colour,
                                                      T theta, int nactive) {
  const int n = L.n, N = L.N;
  const size_t nn = (size_t)n * n, rowN = (size_t)n * N;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x & (W - 1);
  const int slot = b * (kBlock / W) + threadIdx.x / W;
  if (slot >= nactive) return;  // whole W-lane groups leave together
  int xx, k;
  colour_node(slot, n, colour, xx, k);
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
  T bP[JM], bY[JM], ia[JM];
  T num = 0, den = 0;
#pragma unroll
  for (int q = 0; q < JM; ++q) {
    const int j = lane + q * W;
    bP[q] = 0; bY[q] = 0; ia[q] = 0;
    if (j < N) {
      const T kw = L.kx[kxb + j], ke = L.kx[kxb + N + j];
      const T ks = L.ky[kyb + j], kn = L.ky[kyb + rowN + j];
      const size_t base = node * N + j;
      T sy = 0, sp = 0;
      if (hw) { sy += kw * Y[base - N]; sp += kw * P[base - N]; }
      if (he) { sy += ke * Y[base + N]; sp += ke * P[base + N]; }
      if (hs) { sy += ks * Y[base - rowN]; sp += ks * P[base - rowN]; }
      if (hn) { sy += kn * Y[base + rowN]; sp += kn * P[base + rowN]; }
      const T a = (kw + ke) + (ks + kn);
      const T ai = T(1) / a;
      const T cj = L.c[j], dj = L.d[j], ej = L.e[j];
      const T bp = fY[base] + sp, by = fP[base] + sy;
      const T t = cj * ai * ai;
      num += dj * (t * by - ai * bp);
      den += dj * t * ej;
      bP[q] = bp; bY[q] = by; ia[q] = ai;
    }
  }
  num = group_sum<W>(num);
  den = group_sum<W>(den);
  const T un = (fU[node] + num) / (L.g + den);
  const bool relax = theta != T(1);
#pragma unroll
  for (int q = 0; q < JM; ++q) {
    const int j = lane + q * W;
    if (j < N) {
      const size_t base = node * N + j;
      T yn = ia[q] * (bY[q] - L.e[j] * un);
      T pn = ia[q] * (bP[q] - L.c[j] * yn);
      if (relax) {
        yn = (T(1) - theta) * Y[base] + theta * yn;
        pn = (T(1) - theta) * P[base] + theta * pn;
      }
      Y[base] = yn;
      P[base] = pn;
    }
  }
  if (lane == 0) U[node] = relax ? (T(1) - theta) * U[node] + theta * un : un;
}

// ---------------------------------------------------------------- residual
// out = f - S x (mode 0) or out = S x (mode 1) over every node; the block rows
// are those of eq. (2).  Faces and arithmetic in T, x and f in TX, out in TO.
// out may be null (norms only).  partials (if not null) receives per block
// { sum r_Y^2, sum r_U^2, sum r_P^2 }.
template <typename T, typename TX, typename TO, int W, int JM>
__global__ __launch_bounds__(kBlock) void k_residual(LevelArgs<T> L, const TX* __restrict__ x,
                                                     const TX* __restrict__ f,
                                                     TO* __restrict__ out, int mode,
                                                     double* __restrict__ partials) {
  const int n = L.n, N = L.N;
  const size_t nn = (size_t)n * n, rowN = (size_t)n * N;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x & (W - 1);
  const int slot = b * (kBlock / W) + threadIdx.x / W;
  double acc[3] = {0.0, 0.0, 0.0};
  if (slot < (int)nn) {
    const int k = slot / n, xx = slot - k * n;
    const size_t node = (size_t)slot;
    const TX* Y = x;
    const TX* P = x + (size_t)(N + 1) * nn;
    const T u = (T)x[(size_t)N * nn + node];
    const size_t kxb = ((size_t)k * (n + 1) + xx) * N;
    const size_t kyb = node * N;
    const bool hw = xx > 0, he = xx < n - 1, hs = k > 0, hn = k < n - 1;
    T dsum = 0;
#pragma unroll
    for (int q = 0; q < JM; ++q) {
      const int j = lane + q * W;
      if (j < N) {
        const T kw = L.kx[kxb + j], ke = L.kx[kxb + N + j];
        const T ks = L.ky[kyb + j], kn = L.ky[kyb + rowN + j];
        const size_t base = node * N + j;
        const T y0 = (T)Y[base], p0 = (T)P[base];
        T sy = 0, sp = 0;
        if (hw) { sy += kw * (T)Y[base - N]; sp += kw * (T)P[base - N]; }
        if (he) { sy += ke * (T)Y[base + N]; sp += ke * (T)P[base + N]; }
        if (hs) { sy += ks * (T)Y[base - rowN]; sp += ks * (T)P[base - rowN]; }
        if (hn) { sy += kn * (T)Y[base + rowN]; sp += kn * (T)P[base + rowN]; }
        const T a = (kw + ke) + (ks + kn);
        T rY = L.c[j] * y0 + (a * p0 - sp);     // C_j y_j + A_j^T p_j
        T rP = (a * y0 - sy) + L.e[j] * u;      // A_j y_j + E_j u
        dsum += L.d[j] * p0;
        if (mode == 0) {
          rY = (T)f[base] - rY;
          rP = (T)f[(size_t)(N + 1) * nn + base] - rP;
        }
        if (out) {
          out[base] = (TO)rY;
          out[(size_t)(N + 1) * nn + base] = (TO)rP;
        }
        acc[0] += (double)rY * (double)rY;
        acc[2] += (double)rP * (double)rP;
      }
    }
    dsum = group_sum<W>(dsum);
    if (lane == 0) {
      T rU = L.g * u + dsum;                    // G u + sum_j D_j p_j
      if (mode == 0) rU = (T)f[(size_t)N * nn + node] - rU;
      if (out) out[(size_t)N * nn + node] = (TO)rU;
      acc[1] = (double)rU * (double)rU;
    }
  }
  if (partials) {
    block_sum<3>(acc);
    if (threadIdx.x == 0) {
      partials[3 * (size_t)b + 0] = acc[0];
      partials[3 * (size_t)b + 1] = acc[1];
      partials[3 * (size_t)b + 2] = acc[2];
    }
  }
}

// norms[0..3] = { ||r||, ||r_Y||, ||r_U||, ||r_P|| } from nb block partials.
__global__ __launch_bounds__(kBlock) void k_finalize_norms3(const double* __restrict__ partials,
                                                            int nb, double* __restrict__ norms) {
  double acc[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nb; i += kBlock) {
    acc[0] += partials[3 * (size_t)i + 0];
    acc[1] += partials[3 * (size_t)i + 1];
    acc[2] += partials[3 * (size_t)i + 2];
  }
  block_sum<3>(acc);
  if (threadIdx.x == 0) {
    norms[0] = sqrt(acc[0] + acc[1] + acc[2]);
    norms[1] = sqrt(acc[0]);
    norms[2] = sqrt(acc[1]);
    norms[3] = sqrt(acc[2]);
  }
}

// ----------------------------------------------------------------- transfers
// Weights of 1D linear interpolation: 1 at the coinciding node, 1/2 next to it.
__device__ __forceinline__ double lin_w(int d) { return d == 0 ? 1.0 : 0.5; }

// coarse = R fine, R = P^T: coarse node (X, K) sits on fine node (2X+1, 2K+1)
// and gathers its 3x3 fine neighbourhood with weights w(dx) w(dk).
template <typename T, int W, int JM>
__global__ __launch_bounds__(kBlock) void k_restrict(int nf, int N, const T* __restrict__ fine,
                                                     T* __restrict__ coarse) {
  const int nc = (nf - 1) / 2;
  const size_t nnf = (size_t)nf * nf, nnc = (size_t)nc * nc;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x & (W - 1);
  const int slot = b * (kBlock / W) + threadIdx.x / W;
  if (slot >= (int)nnc) return;
  const int K = slot / nc, X = slot - K * nc;
  const size_t c0 = (size_t)(2 * K + 1) * nf + (2 * X + 1);
  const T* fY = fine;
  const T* fP = fine + (size_t)(N + 1) * nnf;
#pragma unroll
  for (int q = 0; q < JM; ++q) {
    const int j = lane + q * W;
    if (j < N) {
      T sY = 0, sP = 0;
#pragma unroll
      for (int dk = -1; dk <= 1; ++dk)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const T w = (T)(lin_w(dx) * lin_w(dk));
          const size_t fi = (size_t)((long)c0 + (long)dk * nf + dx) * N + j;
          sY += w * fY[fi];
          sP += w * fP[fi];
        }
      coarse[(size_t)slot * N + j] = sY;
      coarse[(size_t)(N + 1) * nnc + (size_t)slot * N + j] = sP;
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
    coarse[(size_t)N * nnc + slot] = sU;
  }
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

// ------------------------------------------------------------------- setup
// Coarse faces by rediscretization: mean of the two fine faces under a coarse face.
template <typename T>
__global__ void k_coarsen_faces(int nf, int N, const T* __restrict__ kxf, const T* __restrict__ kyf,
                                T* __restrict__ kxc, T* __restrict__ kyc) {
  const int nc = (nf - 1) / 2;
  const size_t tot = (size_t)nc * (nc + 1) * N;
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < tot; i += (size_t)gridDim.x * kBlock) {
    const int j = (int)(i % N);
    const size_t r = i / N;
    {  // kx: (K, F)
      const int F = (int)(r % (nc + 1)), K = (int)(r / (nc + 1));
      const size_t fb = ((size_t)(2 * K + 1) * (nf + 1) + 2 * F) * N + j;
      kxc[i] = T(0.5) * (kxf[fb] + kxf[fb + N]);
    }
    {  // ky: (G, X)
      const int X = (int)(r % nc), G = (int)(r / nc);
      const size_t fb = ((size_t)(2 * G) * nf + 2 * X + 1) * N + j;
      kyc[i] = T(0.5) * (kyf[fb] + kyf[fb + (size_t)nf * N]);
    }
  }
}

// flags[0] = 1 if any face is not finite or <= 0 (A_j would lose its positive diagonal).
__global__ void k_check_faces(size_t len, const double* __restrict__ a, const double* __restrict__ b,
                              int* __restrict__ flag) {
  int bad = 0;
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < len; i += (size_t)gridDim.x * kBlock) {
    const double u = a[i], v = b[i];
    if (!(u > 0.0) || !(v > 0.0) || !isfinite(u) || !isfinite(v)) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

// In-place Gauss-Jordan inversion of an m x m matrix held in LDS (no pivoting:
// used on symmetric positive definite matrices only).  All threads call it.
__device__ void lds_invert_spd(double* A, double* col, int m) {
  for (int p = 0; p < m; ++p) {
    __syncthreads();
    const double piv = A[p * m + p];
    for (int i = threadIdx.x; i < m; i += blockDim.x) col[i] = A[i * m + p];
    __syncthreads();
    const double ip = 1.0 / piv;
    for (int j = threadIdx.x; j < m; j += blockDim.x) A[p * m + j] = (j == p) ? ip : A[p * m + j] * ip;
    __syncthreads();
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
      const int i = idx / m, j = idx - i * m;
      if (i == p) continue;
      const double fct = col[i];
      A[idx] = (j == p) ? -fct * ip : A[idx] - fct * A[p * m + j];
    }
  }
  __syncthreads();
}

// One block per sample: assemble the coarsest A_j (m = n^2) from its faces and invert it.
__global__ __launch_bounds__(kBlock) void k_coarse_invert_A(int n, int N, const double* __restrict__ kx,
                                                            const double* __restrict__ ky,
                                                            double* __restrict__ Ainv) {
  __shared__ double A[kMaxCoarse * kMaxCoarse];
  __shared__ double col[kMaxCoarse];
  const int j = blockIdx.x, m = n * n;
  for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) A[idx] = 0.0;
  __syncthreads();
  for (int r = threadIdx.x; r < m; r += blockDim.x) {
    const int k = r / n, x = r - k * n;
    const double kw = kx[((size_t)k * (n + 1) + x) * N + j], ke = kx[((size_t)k * (n + 1) + x + 1) * N + j];
    const double ks = ky[((size_t)k * n + x) * N + j], kn = ky[((size_t)(k + 1) * n + x) * N + j];
    A[r * m + r] = (kw + ke) + (ks + kn);
    if (x > 0) A[r * m + r - 1] = -kw;
    if (x < n - 1) A[r * m + r + 1] = -ke;
    if (k > 0) A[r * m + r - n] = -ks;
    if (k < n - 1) A[r * m + r + n] = -kn;
  }
  lds_invert_spd(A, col, m);
  for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) Ainv[(size_t)j * m * m + idx] = A[idx];
}

// terms[j] = d_j c_j e_j Ainv_j Ainv_j   (one block per sample)
__global__ __launch_bounds__(kBlock) void k_coarse_schur_terms(int m, const double* __restrict__ Ainv,
                                                               const double* __restrict__ c,
                                                               const double* __restrict__ d,
                                                               const double* __restrict__ e,
                                                               double* __restrict__ terms) {
  __shared__ double A[kMaxCoarse * kMaxCoarse];
  const int j = blockIdx.x;
  for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) A[idx] = Ainv[(size_t)j * m * m + idx];
  __syncthreads();
  const double s = d[j] * c[j] * e[j];
  for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
    const int i = idx / m, q = idx - i * m;
    double t = 0.0;
    for (int r = 0; r < m; ++r) t += A[i * m + r] * A[r * m + q];
    terms[(size_t)j * m * m + idx] = s * t;
  }
}

// Schur complement g I + sum_j terms[j] (fixed order over j), inverted in place; one block.
__global__ __launch_bounds__(kBlock) void k_coarse_schur_invert(int m, int N, const double* __restrict__ terms,
                                                                double g, double* __restrict__ Sinv) {
  __shared__ double A[kMaxCoarse * kMaxCoarse];
  __shared__ double col[kMaxCoarse];
  for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
    double s = (idx / m == idx % m) ? g : 0.0;
    for (int j = 0; j < N; ++j) s += terms[(size_t)j * m * m + idx];
    A[idx] = s;
  }
  lds_invert_spd(A, col, m);
  for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) Sinv[idx] = A[idx];
}

// ------------------------------------------------------------ coarsest solve
// Block elimination of eq. (2) on the coarsest grid, one block per sample j:
//   phase 1: ds_j = d_j A_j^{-1} (F_Y,j - c_j A_j^{-1} F_P,j)
//   phase 2: u = Sinv (F_U - sum_j ds_j);  y_j = A_j^{-1}(F_P,j - e_j u);
//            p_j = A_j^{-1}(F_Y,j - c_j y_j)
// Vectors in the level layout (type TV), arithmetic in FP64.
__device__ __forceinline__ double row_dot(const double* __restrict__ M, int m, int i, const double* v) {
  double s = 0.0;
  for (int c = 0; c < m; ++c) s += M[(size_t)i * m + c] * v[c];
  return s;
}

template <typename TV>
__global__ __launch_bounds__(64) void k_coarse_phase1(int m, int N, const double* __restrict__ Ainv,
                                                      const double* __restrict__ c, const double* __restrict__ d,
                                                      const TV* __restrict__ F, double* __restrict__ ds) {
  __shared__ double sF[kMaxCoarse], sT[kMaxCoarse];
  const int j = blockIdx.x, i = threadIdx.x;
  const double* Aj = Ainv + (size_t)j * m * m;
  const TV* FY = F;
  const TV* FP = F + (size_t)(N + 1) * m;
  if (i < m) sF[i] = (double)FP[(size_t)i * N + j];
  __syncthreads();
  if (i < m) sT[i] = (double)FY[(size_t)i * N + j] - c[j] * row_dot(Aj, m, i, sF);
  __syncthreads();
  if (i < m) ds[(size_t)j * m + i] = d[j] * row_dot(Aj, m, i, sT);
}

template <typename TV>
__global__ __launch_bounds__(64) void k_coarse_phase2(int m, int N, const double* __restrict__ Ainv,
                                                      const double* __restrict__ Sinv,
                                                      const double* __restrict__ c, const double* __restrict__ e,
                                                      const TV* __restrict__ F, const double* __restrict__ ds,
                                                      TV* __restrict__ X) {
  __shared__ double sR[kMaxCoarse], sU[kMaxCoarse], sT[kMaxCoarse], sY[kMaxCoarse];
  const int j = blockIdx.x, i = threadIdx.x;
  const double* Aj = Ainv + (size_t)j * m * m;
  const TV* FY = F;
  const TV* FU = F + (size_t)N * m;
  const TV* FP = F + (size_t)(N + 1) * m;
  if (i < m) {
    double s = (double)FU[i];
    for (int q = 0; q < N; ++q) s -= ds[(size_t)q * m + i];
    sR[i] = s;
  }
  __syncthreads();
  if (i < m) sU[i] = row_dot(Sinv, m, i, sR);
  __syncthreads();
  if (i < m) sT[i] = (double)FP[(size_t)i * N + j] - e[j] * sU[i];
  __syncthreads();
  if (i < m) sY[i] = row_dot(Aj, m, i, sT);
  __syncthreads();
  if (i < m) sT[i] = (double)FY[(size_t)i * N + j] - c[j] * sY[i];
  __syncthreads();
  if (i < m) {
    const double p = row_dot(Aj, m, i, sT);
    X[(size_t)i * N + j] = (TV)sY[i];
    X[(size_t)(N + 1) * m + (size_t)i * N + j] = (TV)p;
    if (j == 0) X[(size_t)N * m + i] = (TV)sU[i];
  }
}

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

// partials[b][i] = sum over the block's elements of w * V_i, i < nv (nv <= kMaxBasis).
// Also (slot nv) the block's sum of w*w when with_norm.
template <typename TV>
__global__ __launch_bounds__(kBlock) void k_mdot(size_t len, const double* __restrict__ w,
                                                 const TV* __restrict__ V, size_t ldv, int nv,
                                                 int with_norm, double* __restrict__ partials) {
  double acc[kMaxBasis + 1];
#pragma unroll
  for (int i = 0; i <= kMaxBasis; ++i) acc[i] = 0.0;
  for (size_t t = blockIdx.x * (size_t)kBlock + threadIdx.x; t < len; t += (size_t)gridDim.x * kBlock) {
    const double wv = w[t];
#pragma unroll
    for (int i = 0; i < kMaxBasis; ++i)
      if (i < nv) acc[i] += wv * (double)V[(size_t)i * ldv + t];
    if (with_norm) acc[kMaxBasis] += wv * wv;
  }
  __shared__ double red[kBlock / 64][kMaxBasis + 1];
  const int lane = threadIdx.x & 63, wvi = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i <= kMaxBasis; ++i) {
    if (i < nv || (i == kMaxBasis && with_norm)) {
      const double s = group_sum<64>(acc[i]);
      if (lane == 0) red[wvi][i] = s;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= kMaxBasis; i += kBlock) {
    if (i < nv || (i == kMaxBasis && with_norm)) {
      double s = red[0][i];
      for (int q = 1; q < kBlock / 64; ++q) s += red[q][i];
      partials[(size_t)blockIdx.x * (kMaxBasis + 1) + i] = s;
    }
  }
}

// out[i] = sum_b partials[b][i] (fixed order), i <= kMaxBasis; out[kMaxBasis] is the
// squared norm slot.  If accumulate, out[i] += the sum.
__global__ __launch_bounds__(kBlock) void k_mdot_finalize(const double* __restrict__ partials, int nb, int nv,
                                                          int with_norm, double* __restrict__ out,
                                                          int accumulate) {
  const int i = threadIdx.x;
  if (i > kMaxBasis) return;
  if (!(i < nv || (i == kMaxBasis && with_norm))) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += partials[(size_t)b * (kMaxBasis + 1) + i];
  out[i] = accumulate ? out[i] + s : s;
}

// w -= sum_i h_i V_i  (h on the device)
template <typename TV>
__global__ void k_gs_update(size_t len, double* __restrict__ w, const TV* __restrict__ V, size_t ldv,
                            int nv, const double* __restrict__ h) {
  for (size_t t = blockIdx.x * (size_t)kBlock + threadIdx.x; t < len; t += (size_t)gridDim.x * kBlock) {
    double s = w[t];
    for (int i = 0; i < nv; ++i) s -= h[i] * (double)V[(size_t)i * ldv + t];
    w[t] = s;
  }
}

// v = s w
__global__ void k_scale(size_t len, const double* __restrict__ w, double* __restrict__ v, double s) {
  for (size_t t = blockIdx.x * (size_t)kBlock + threadIdx.x; t < len; t += (size_t)gridDim.x * kBlock)
    v[t] = w[t] * s;
}

// x += sum_i y_i Z_i  (y on the device)
template <typename TZ>
__global__ void k_basis_axpy(size_t len, double* __restrict__ x, const TZ* __restrict__ Z, size_t ldz,
                             int nz, const double* __restrict__ y) {
  for (size_t t = blockIdx.x * (size_t)kBlock + threadIdx.x; t < len; t += (size_t)gridDim.x * kBlock) {
    double s = x[t];
    for (int i = 0; i < nz; ++i) s += y[i] * (double)Z[(size_t)i * ldz + t];
    x[t] = s;
  }
}

}  // namespace smg
