// coarse.h -- hierarchy setup and the coarsest-level direct solve (gfx950).
#pragma once
#include "common.h"

namespace smg {

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

// Node factor pairs (md, me) of the finest level from the caller's arrays md,
// me ([n][n], null: 1).
__global__ void k_node_factors(int nn, const double* __restrict__ md, const double* __restrict__ me,
                               double* __restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= nn) return;
  out[2 * (size_t)i] = md ? md[i] : 1.0;
  out[2 * (size_t)i + 1] = me ? me[i] : 1.0;
}

// Node factor pairs of a level with nc x nc nodes from those of the level above
// (nf = 2 nc + 1): coarse node (X, K) takes fine node (2X+1, 2K+1) (full = 0,
// injection) or the full-weighting average of the 3 x 3 fine nodes around it,
// weights (1/4)(1/2)^(|dx|+|dk|) (full = 1: the diagonal of R diag(v) P lumped
// by rows, R = P^T / 4).  Every such fine node is interior.
__global__ void k_coarsen_factors(int nc, int full, const double* __restrict__ fine, double* __restrict__ coarse) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= nc * nc) return;
  const int nf = 2 * nc + 1;
  const int K = i / nc, X = i - K * nc;
  const size_t c = (size_t)(2 * K + 1) * nf + (2 * X + 1);
  double d = fine[2 * c], e = fine[2 * c + 1];
  if (full) {
    d = 0.0;
    e = 0.0;
    for (int dk = -1; dk <= 1; ++dk)
      for (int dx = -1; dx <= 1; ++dx) {
        const double w = (dx ? 0.5 : 1.0) * (dk ? 0.5 : 1.0) * 0.25;
        const size_t f = (size_t)((ptrdiff_t)c + (ptrdiff_t)dk * nf + dx);
        d += w * fine[2 * f];
        e += w * fine[2 * f + 1];
      }
  }
  coarse[2 * (size_t)i] = d;
  coarse[2 * (size_t)i + 1] = e;
}

// Domain of a level from the level above (nf = 2 nc + 1) by injection.
__global__ void k_inject_domain(int nc, const double* __restrict__ fine, double* __restrict__ coarse) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= nc * nc) return;
  const int K = i / nc, X = i - K * nc;
  coarse[i] = fine[(size_t)(2 * K + 1) * (2 * nc + 1) + (2 * X + 1)];
}

// Factor pairs of the nodes outside the domain set to (0, -0) (see node_live).
__global__ void k_apply_domain(int nn, const double* __restrict__ dom, double* __restrict__ pairs) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= nn || dom[i] != 0.0) return;
  pairs[2 * (size_t)i] = 0.0;
  pairs[2 * (size_t)i + 1] = -0.0;
}

// Every field of x set to zero at the nodes outside the domain (y, p: N samples each, u).
__global__ void k_zero_outside(int nn, int N, const double* __restrict__ dom, double* __restrict__ x) {
  const size_t t = blockIdx.x * (size_t)kBlock + threadIdx.x;
  const size_t per = 2 * (size_t)N + 1;
  if (t >= (size_t)nn * per) return;
  const int i = (int)(t / per);
  const size_t r = t - (size_t)i * per;
  if (dom[i] != 0.0) return;
  if (r < (size_t)N) x[(size_t)i * N + r] = 0.0;                                   // y_j
  else if (r == (size_t)N) x[(size_t)N * nn + i] = 0.0;                            // u
  else x[(size_t)(N + 1) * nn + (size_t)i * N + (r - N - 1)] = 0.0;                // p_j
}

// flags[0] = 1 if any value is not finite or lies outside [0, 1].
__global__ void k_check_unit(size_t len, const double* __restrict__ a, int* __restrict__ flag) {
  int bad = 0;
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < len; i += (size_t)gridDim.x * kBlock) {
    const double v = a[i];
    if (!(v >= 0.0 && v <= 1.0)) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
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

// In-place Gauss-Jordan inversion of an m x m matrix held in LDS, without pivoting:
// used on the SPD A_j and on Schur complements g I + diag(md) K diag(me) (K SPD,
// g > 0, factors >= 0), whose leading minors are all positive (their eigenvalues
// are those of g I + a symmetric positive semidefinite matrix).  All threads call it.
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
// dom (null: no domain): nodes outside (0) get identity rows; the couplings of the
// nodes inside to them act on values that are zero.
__global__ __launch_bounds__(kBlock) void k_coarse_invert_A(int n, int N, const double* __restrict__ kx,
                                                            const double* __restrict__ ky,
                                                            const double* __restrict__ dom,
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
  __syncthreads();
  if (dom)
    for (int r = threadIdx.x; r < m; r += blockDim.x)
      if (dom[r] == 0.0) {
        for (int q = 0; q < m; ++q) A[r * m + q] = 0.0;
        A[r * m + r] = 1.0;
      }
  lds_invert_spd(A, col, m);
  // stored transposed: AinvT[c][r] = Ainv[r][c], so that a thread per row reads coalesced
  for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
    const int r = idx / m, q = idx - r * m;
    Ainv[(size_t)j * m * m + (size_t)q * m + r] = A[idx];
  }
}

// terms[j] = (d_j c_j e_j diag(md) Ainv_j Ainv_j diag(me))^T from the transposed
// inverses (one block per sample; mk: node factor pairs (md, me))
__global__ __launch_bounds__(kBlock) void k_coarse_schur_terms(int m, const double* __restrict__ Ainv,
                                                               const double* __restrict__ c,
                                                               const double* __restrict__ d,
                                                               const double* __restrict__ e,
                                                               const double* __restrict__ mk,
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
    terms[(size_t)j * m * m + idx] = (mk[2 * q] * s * mk[2 * i + 1]) * t;   // row q, column i
  }
}

// Pre-reduction of the Schur terms over samples: part[q] = sum of terms[j] over
// the samples j of chunk q (kSchurChunk consecutive samples, in order), one
// block per chunk, so that the single-block inversion below sums N / kSchurChunk
// partials instead of N terms.
constexpr int kSchurChunk = 64;
__global__ __launch_bounds__(kBlock) void k_coarse_schur_chunks(int m, int N, const double* __restrict__ terms,
                                                                double* __restrict__ part) {
  const int j0 = blockIdx.x * kSchurChunk, j1 = min(N, j0 + kSchurChunk);
  for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
    double s = 0.0;
    for (int q0 = j0; q0 < j1; q0 += 16) {
      double t[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) t[u] = terms[(size_t)(q0 + u < j1 ? q0 + u : j1 - 1) * m * m + idx];
#pragma unroll
      for (int u = 0; u < 16; ++u) s += q0 + u < j1 ? t[u] : 0.0;
    }
    part[(size_t)blockIdx.x * m * m + idx] = s;
  }
}

// Transposed Schur complement (g I + sum of the terms)^T inverted in place; the
// result is the transposed storage of its inverse.  One block.  `terms` holds the
// N = ceil(samples / kSchurChunk) chunk partials of k_coarse_schur_chunks, summed
// here in order: the sum over samples is two-stage, in sample order within each
// chunk of 64, then over the chunks in order.
__global__ __launch_bounds__(kBlock) void k_coarse_schur_invert(int m, int N, const double* __restrict__ terms,
                                                                double g, double* __restrict__ Sinv) {
  __shared__ double A[kMaxCoarse * kMaxCoarse];
  __shared__ double col[kMaxCoarse];
  for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
    // summed in sample order; 16 loads in flight per round trip
    double s = (idx / m == idx % m) ? g : 0.0;
    for (int q0 = 0; q0 < N; q0 += 16) {
      double t[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) t[u] = terms[(size_t)(q0 + u < N ? q0 + u : N - 1) * m * m + idx];
#pragma unroll
      for (int u = 0; u < 16; ++u) s += q0 + u < N ? t[u] : 0.0;
    }
    A[idx] = s;
  }
  lds_invert_spd(A, col, m);
  for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) Sinv[idx] = A[idx];
}

// ------------------------------------------------------------ coarsest solve
// Block elimination of eq. (2) on the coarsest grid, one block per sample j:
//   phase 1: ds_j = D_j A_j^{-1} (F_Y,j - c_j A_j^{-1} F_P,j)
//   phase 2: u = Sinv (F_U - sum_j ds_j);  y_j = A_j^{-1}(F_P,j - E_j u);
//            (up to kCoarseUMin samples every block forms u itself from the N ds_j in
//            sample order; above that k_coarse_u forms it once, summing the ds_j
//            in sixteen interleaved slices, and the blocks read it as `upre`)
// with D_j = d_j diag(md), E_j = e_j diag(me) (mk: node factor pairs (md, me));
//            p_j = A_j^{-1}(F_Y,j - c_j y_j)
// Vectors in the level layout (type TV), arithmetic in FP64.
// (M v)_i with M stored transposed (MT[c][i] = M[i][c]): coalesced across threads i.
// Row i of M stored transposed (MT[c][i] = M[i][c]; coalesced across threads i)
// into registers: all kMaxCoarse loads are issued before the first use (indices
// past m are clamped into the matrix), so a row costs one memory round trip and
// is reused for every product with M.
__device__ __forceinline__ void load_row(const double* __restrict__ MT, int m, int i, double (&a)[kMaxCoarse]) {
#pragma unroll
  for (int c = 0; c < kMaxCoarse; ++c) a[c] = MT[(size_t)(c < m ? c : m - 1) * m + i];
}
// (M v)_i from the row in registers, summed over c = 0..m-1 in order.
__device__ __forceinline__ double dot_row(const double (&a)[kMaxCoarse], int m, const double* v) {
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kMaxCoarse; ++c) s += c < m ? a[c] * v[c] : 0.0;
  return s;
}

// Phase 1 for sample j (one block of >= m threads).
template <typename TV>
__device__ __forceinline__ void coarse_phase1_sample(int j, int m, int N, const double* __restrict__ Ainv,
                                                     const double* __restrict__ c, const double* __restrict__ d,
                                                     const double* __restrict__ mk, const TV* __restrict__ F,
                                                     double* __restrict__ ds) {
  __shared__ double sF[kMaxCoarse], sT[kMaxCoarse];
  const int i = threadIdx.x;
  const double* Aj = Ainv + (size_t)j * m * m;
  const TV* FY = F;
  const TV* FP = F + (size_t)(N + 1) * m;
  double a[kMaxCoarse];
  double dm = 0.0;   // this row's D_j entry, loaded with the rest
  if (i < m) {
    load_row(Aj, m, i, a);
    sF[i] = (double)FP[(size_t)i * N + j];
    dm = mk[2 * i] * d[j];
  }
  __syncthreads();
  if (i < m) sT[i] = (double)FY[(size_t)i * N + j] - c[j] * dot_row(a, m, sF);
  __syncthreads();
  if (i < m) ds[(size_t)j * m + i] = dm * dot_row(a, m, sT);
}

// Phase 2 for sample j (one block of >= m threads); block j = 0 also writes u.
// Without upre the block computes u from the N ds_j; with upre (N > kCoarseUMin)
// it takes the u that k_coarse_u computed once.
template <typename TV>
__device__ __forceinline__ void coarse_phase2_sample(int j, int m, int N, const double* __restrict__ Ainv,
                                                     const double* __restrict__ Sinv,
                                                     const double* __restrict__ c, const double* __restrict__ e,
                                                     const double* __restrict__ mk, const TV* __restrict__ F,
                                                     const double* __restrict__ ds, TV* __restrict__ X,
                                                     const double* __restrict__ upre = nullptr) {
  __shared__ double sR[kMaxCoarse], sU[kMaxCoarse], sT[kMaxCoarse], sY[kMaxCoarse];
  const int i = threadIdx.x;
  const double* Aj = Ainv + (size_t)j * m * m;
  const TV* FY = F;
  const TV* FU = F + (size_t)N * m;
  const TV* FP = F + (size_t)(N + 1) * m;
  double a[kMaxCoarse], si[kMaxCoarse];
  double em = 0.0;   // this row's E_j entry, loaded with the rest
  if (i < m) {
    load_row(Aj, m, i, a);
    em = mk[2 * i + 1] * e[j];
    if (upre) {                 // u computed once for all samples (k_coarse_u)
      sU[i] = upre[i];
    } else {
      load_row(Sinv, m, i, si);
      // F_U - sum_j ds_j, in sample order; 16 loads in flight per round trip
      double s = (double)FU[i];
      for (int q0 = 0; q0 < N; q0 += 16) {
        double t[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) t[u] = ds[(size_t)(q0 + u < N ? q0 + u : N - 1) * m + i];
#pragma unroll
        for (int u = 0; u < 16; ++u) s -= q0 + u < N ? t[u] : 0.0;
      }
      sR[i] = s;
    }
  }
  __syncthreads();
  if (!upre && i < m) sU[i] = dot_row(si, m, sR);
  __syncthreads();
  if (i < m) sT[i] = (double)FP[(size_t)i * N + j] - em * sU[i];
  __syncthreads();
  if (i < m) sY[i] = dot_row(a, m, sT);
  __syncthreads();
  if (i < m) sT[i] = (double)FY[(size_t)i * N + j] - c[j] * sY[i];
  __syncthreads();
  if (i < m) {
    const double p = dot_row(a, m, sT);
    X[(size_t)i * N + j] = (TV)sY[i];
    X[(size_t)(N + 1) * m + (size_t)i * N + j] = (TV)p;
    if (j == 0) X[(size_t)N * m + i] = (TV)sU[i];
  }
}

template <typename TV>
__global__ __launch_bounds__(64) void k_coarse_phase1(int m, int N, const double* __restrict__ Ainv,
                                                      const double* __restrict__ c, const double* __restrict__ d,
                                                      const double* __restrict__ mk, const TV* __restrict__ F,
                                                      double* __restrict__ ds) {
  coarse_phase1_sample<TV>(blockIdx.x, m, N, Ainv, c, d, mk, F, ds);
}

template <typename TV>
__global__ __launch_bounds__(64) void k_coarse_phase2(int m, int N, const double* __restrict__ Ainv,
                                                      const double* __restrict__ Sinv,
                                                      const double* __restrict__ c, const double* __restrict__ e,
                                                      const double* __restrict__ mk, const TV* __restrict__ F,
                                                      const double* __restrict__ ds, TV* __restrict__ X,
                                                      const double* __restrict__ upre) {
  coarse_phase2_sample<TV>(blockIdx.x, m, N, Ainv, Sinv, c, e, mk, F, ds, X, upre);
}

// u = Sinv (F_U - sum_j ds_j) once for all samples, for many samples (every
// phase-2 block would otherwise sum all N of them): 16 slices of 64 lanes sum
// the samples j = slice (mod 16), then meet in LDS in slice order.  One block.
constexpr int kCoarseUSlices = 16;
template <typename TV>
__global__ __launch_bounds__(64 * kCoarseUSlices) void k_coarse_u(int m, int N, const double* __restrict__ Sinv,
                                                                   const TV* __restrict__ F,
                                                                   const double* __restrict__ ds,
                                                                   double* __restrict__ u) {
  __shared__ double part[kCoarseUSlices][kMaxCoarse];
  __shared__ double sR[kMaxCoarse];
  const int i = threadIdx.x % 64, sl = threadIdx.x / 64;
  if (i < m) {
    double s = 0.0;
    for (int j0 = sl; j0 < N; j0 += 8 * kCoarseUSlices) {
      double t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int jj = j0 + q * kCoarseUSlices;
        t[q] = jj < N ? ds[(size_t)jj * m + i] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) s += t[q];
    }
    part[sl][i] = s;
  }
  __syncthreads();
  if (sl == 0 && i < m) {
    double r = (double)F[(size_t)N * m + i];
#pragma unroll
    for (int q = 0; q < kCoarseUSlices; ++q) r -= part[q][i];
    sR[i] = r;
  }
  __syncthreads();
  if (sl == 0 && i < m) {
    double si[kMaxCoarse];
    load_row(Sinv, m, i, si);
    u[i] = dot_row(si, m, sR);
  }
}

}  // namespace smg
