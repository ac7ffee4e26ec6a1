// common.h -- shared device helpers of the collective multigrid kernels (gfx950).
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
  int strip;   // columns per strip of the colour traversal (colour_node)
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

// Sum over a group of W lanes (W a power of two <= 64, runtime or constant).
template <typename T>
__device__ __forceinline__ T group_sum_w(T v, int W) {
  for (int off = W >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
  return v;
}

// Block-wide sum of NV values over BS threads, deterministic order; result valid in thread 0.
template <int NV, int BS = kBlock>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
  __shared__ double red[BS / 64][NV];
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
      for (int w = 1; w < BS / 64; ++w) s += red[w][i];
      v[i] = s;
    }
  }
}

// Node (x, k) of the slot-th node of colour `colour` ((x + k) % 2 == colour),
// n odd.  The grid is cut into vertical strips of S columns (S even; S >= n is
// plain row-major order) and each strip is traversed row by row, strips one
// after another.  Rows above and below a node are then visited soon after it
// within a strip, so opposite-colour values shared between neighbouring rows are
// read again while still in L2.  In a strip of width w a pair of rows (even k
// first) holds w nodes of each colour.
__host__ __device__ inline void colour_node(int slot, int n, int colour, int S, int& x, int& k) {
  int x0 = 0, w = n, l = slot;
  if (S < n) {
    const int per = n * (S >> 1);   // nodes of either colour in a full strip
    const int s = slot / per;
    x0 = s * S;
    w = n - x0 < S ? n - x0 : S;
    l = slot - s * per;
  }
  const int pr = l / w, rem = l - pr * w;
  const int c0 = (w - colour + 1) >> 1;  // nodes of this colour on the even row of the pair
  if (rem < c0) { k = 2 * pr; x = x0 + colour + 2 * rem; }
  else { k = 2 * pr + 1; x = x0 + (1 - colour) + 2 * (rem - c0); }
}

// Weights of 1D linear interpolation: 1 at the coinciding node, 1/2 next to it.
__device__ __forceinline__ double lin_w(int d) { return d == 0 ? 1.0 : 0.5; }

__host__ __device__ inline int colour_count(int n, int colour) {
  return ((n - 1) / 2) * n + (n - colour + 1) / 2;
}

}  // namespace smg
