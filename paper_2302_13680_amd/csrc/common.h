// common.h -- shared device helpers of the collective multigrid kernels (gfx950).
//
// Layout (see include/smg.h): samples innermost.  A level vector is
//   Y [n][n][N] | U [n][n] | P [n][n][N];  faces kx [n][n+1][N], ky [n+1][n][N].
// A node's N samples are contiguous, so a group of W lanes of one wavefront
// (W = 1..64, a power of two) holds one node and each lane handles JM samples,
// in chunks of VW consecutive ones: chunk c of a lane holds samples
// VW (lane + c W) + [0, VW) (VW = 2 needs N even; FP32 uses it so that every
// access is 8 bytes); the reductions over samples that the node solve and
// the control row need stay inside that group (DPP lane moves and reads of row
// sums, group_sum).  Every lane of a group ends with the bitwise-same sum (IEEE
// addition is commutative), so all lanes agree on u_i.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

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
  const T* __restrict__ gden;   // [n][n] per node: g + sum_j d_j c_j e_j / a_j^2 (set up once)
  const T* __restrict__ mk;     // [n][n][2] node factors (md_i, me_i): the node entries of D_j
                                // and E_j are md_i d_j and me_i e_j (local control: both the
                                // control mask; the semismooth Newton system: md = active set)
  int strip;   // columns per strip of the colour traversal (colour_node)
};

template <typename T>
struct NodeFactors {
  T d, e;   // factors of the node entries of D_j and E_j
};

// A node outside the domain (the L-shape's removed quadrant: a homogeneous
// Dirichlet node held at zero) carries the factor pair (0, -0): both factors
// vanish, and the sign bit of the E factor marks it.  Kernels compiled with
// MK = false (no factors, no domain) see every node inside.
template <typename T>
__device__ __forceinline__ bool node_live(const NodeFactors<T>& f) {
  return !signbit(f.e);
}

// A node with a control: a U unknown coupled to the state and adjoint rows
// (md or me nonzero; never outside the domain).  The control space spans these
// nodes only, so restriction and prolongation of the U block stay inside it.
template <typename T>
__device__ __forceinline__ bool node_control(const NodeFactors<T>& f) {
  return f.d != T(0) || f.e != T(0);
}

// the factor pair of node i from a [n][n][2] array, one 2-element load
template <typename T>
__device__ __forceinline__ NodeFactors<T> load_factors(const T* __restrict__ mk, size_t i) {
  using V = typename std::conditional<std::is_same<T, double>::value, double2, float2>::type;
  const V v = *reinterpret_cast<const V*>(mk + 2 * i);
  return {v.x, v.y};
}

// node factors of node i; kernels compiled with MK = false (contexts whose
// factors are all 1) use 1 without a load
template <bool MK, typename T>
__device__ __forceinline__ NodeFactors<T> node_factors(const LevelArgs<T>& L, size_t i) {
  if constexpr (MK) {
    return load_factors(L.mk, i);
  } else {
    return {T(1), T(1)};
  }
}

// MI355X dispatches workgroup b to XCD b % 8.  Remap so that every XCD works on
// one contiguous range of logical tiles (neighbouring grid rows then share that
// XCD's L2).  Bijective on [0, nblocks).
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
  const int q = nblocks / kNumXcd, r = nblocks % kNumXcd;
  const int xcd = b % kNumXcd, idx = b / kNumXcd;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// Blocks of a launch that gives each of `units` groups W lanes: the grid every
// per-node kernel is launched with.  Computed from an argument that the kernel
// loads anyway, rather than read from the dispatch's hidden arguments, which
// would cost each block's start one more kernel-argument cache line (measured:
// a few percent on the latency-bound coarse levels).
template <int W>
__device__ __forceinline__ int group_blocks(int units) {
  constexpr int per = kBlock / W;
  return (units + per - 1) / per;
}

// Index of this thread's group of W lanes in a launch of kBlock-thread blocks
// (b: the remapped block index).  A group of 64 or more lanes holds whole
// waves, so its index is wave-uniform; readfirstlane tells the compiler, which
// then keeps the node's index arithmetic and addresses in scalar registers.
template <int W>
__device__ __forceinline__ int group_slot(int b) {
  const int s = b * (kBlock / W) + (int)threadIdx.x / W;
  if constexpr (W >= 64) return __builtin_amdgcn_readfirstlane(s);
  else return s;
}

// VW consecutive samples as one access (VW = 2: an 8-byte float2 or a 16-byte
// double2; VW = 4: a 16-byte float4; the address is a multiple of VW elements
// from a 256-byte aligned base).
template <int VW, typename T>
__device__ __forceinline__ void ldv(const T* __restrict__ p, T (&v)[VW]) {
  if constexpr (VW == 1) {
    v[0] = *p;
  } else if constexpr (VW == 4) {
    static_assert(std::is_same<T, float>::value, "four samples per access: FP32 only");
    const float4 t = *reinterpret_cast<const float4*>(p);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  } else {
    static_assert(VW == 2, "one, two or four samples per access");
    using V2 = typename std::conditional<std::is_same<T, float>::value, float2, double2>::type;
    const V2 t = *reinterpret_cast<const V2*>(p);
    v[0] = t.x;
    v[1] = t.y;
  }
}
template <int VW, typename T>
__device__ __forceinline__ void stv(T* __restrict__ p, const T (&v)[VW]) {
  if constexpr (VW == 1) {
    *p = v[0];
  } else if constexpr (VW == 4) {
    static_assert(std::is_same<T, float>::value, "four samples per access: FP32 only");
    *reinterpret_cast<float4*>(p) = float4{v[0], v[1], v[2], v[3]};
  } else {
    using V2 = typename std::conditional<std::is_same<T, float>::value, float2, double2>::type;
    V2 t;
    t.x = v[0];
    t.y = v[1];
    *reinterpret_cast<V2*>(p) = t;
  }
}

// stv with the nontemporal hint, for level vectors no cache will hold until
// they are read again (one access per element: 4- or 8-byte stores).
template <int VW, typename T>
__device__ __forceinline__ void stv_nt(T* __restrict__ p, const T (&v)[VW]) {
#pragma unroll
  for (int u = 0; u < VW; ++u) __builtin_nontemporal_store(v[u], p + u);
}

// Move a value between lanes of a row of 16 lanes with DPP (CTRL: 0xB1 = xor 1
// and 0x4E = xor 2 inside quads, 0x141 = mirror inside 8 lanes, 0x140 = mirror
// inside 16 lanes).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_value(double v, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                          __builtin_amdgcn_readlane(__double2loint(v), lane));
}
__device__ __forceinline__ float lane_value(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Sum over aligned groups of W lanes (W a power of two <= 64); every lane of a
// group gets the bitwise-same sum (each step adds two values that the partner
// lane adds in the other order).  Within a 16-lane row the partners come by DPP:
// xor 1 and xor 2 inside quads, then the 8-lane and 16-lane mirrors, each of
// which pairs a lane with one in the other half of its block.  Groups of 32 and
// 64 lanes add the row sums read from lanes 0, 16, 32, 48.  Lanes of other
// groups are never read into a group's sum, so groups of a wave may be inactive.
template <int W, typename T>
__device__ __forceinline__ T group_sum(T v) {
  if constexpr (W >= 2) v += dpp_move<0xB1>(v);
  if constexpr (W >= 4) v += dpp_move<0x4E>(v);
  if constexpr (W >= 8) v += dpp_move<0x141>(v);
  if constexpr (W >= 16) v += dpp_move<0x140>(v);
  if constexpr (W == 32) {
    const T r0 = lane_value(v, 0), r1 = lane_value(v, 16), r2 = lane_value(v, 32), r3 = lane_value(v, 48);
    v = (__lane_id() & 32) ? r2 + r3 : r0 + r1;
  } else if constexpr (W == 64) {
    const T r0 = lane_value(v, 0), r1 = lane_value(v, 16), r2 = lane_value(v, 32), r3 = lane_value(v, 48);
    v = (r0 + r1) + (r2 + r3);
  }
  return v;
}

// group_sum for a group width known at run time (uniform across the wave).
template <typename T>
__device__ __forceinline__ T group_sum_w(T v, int W) {
  switch (W) {
    case 1: return v;
    case 2: return group_sum<2>(v);
    case 4: return group_sum<4>(v);
    case 8: return group_sum<8>(v);
    case 16: return group_sum<16>(v);
    case 32: return group_sum<32>(v);
    default: return group_sum<64>(v);
  }
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

// Node (x, k) of the slot-th node of an n x n grid (any n) traversed in vertical
// strips of S columns (S >= n: row-major order), each strip row by row.
__host__ __device__ inline void strip_node(int slot, int n, int S, int& x, int& k) {
  int x0 = 0, w = n, l = slot;
  if (S < n) {
    const int per = n * S;
    const int s = slot / per;
    x0 = s * S;
    w = n - x0 < S ? n - x0 : S;
    l = slot - s * per;
  }
  k = l / w;
  x = x0 + (l - k * w);
}

// Strip width on the next coarser grid that covers the same fine columns.
__host__ __device__ inline int coarse_strip(int fine_strip) { return fine_strip >= 4 ? fine_strip / 2 : 2; }

// Weights of 1D linear interpolation: 1 at the coinciding node, 1/2 next to it.
__device__ __forceinline__ double lin_w(int d) { return d == 0 ? 1.0 : 0.5; }

__host__ __device__ inline int colour_count(int n, int colour) {
  return ((n - 1) / 2) * n + (n - colour + 1) / 2;
}

}  // namespace smg
