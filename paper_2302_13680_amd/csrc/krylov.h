// krylov.h -- vector kernels of the Krylov and refinement drivers (gfx950).
#pragma once
#include "common.h"

namespace smg {

// ---------------------------------------------------------- vector kernels
// Streaming copy (the achievable-bandwidth reference): each lane keeps four
// 16-byte loads in flight (coalesced, kBlock apart) before their stores, and
// both bypass the caches' retention (non-temporal), which measured 6.0-6.1 TB/s
// on MI355X against 4.6 TB/s for one 16-byte access per step.
constexpr int kCopyUnroll = 4;
__global__ __launch_bounds__(kBlock) void k_stream_copy(size_t n16, const double2* __restrict__ src,
                                                        double2* __restrict__ dst) {
  const size_t stride = (size_t)gridDim.x * kBlock * kCopyUnroll;
  for (size_t b = blockIdx.x * (size_t)kBlock * kCopyUnroll + threadIdx.x; b < n16; b += stride) {
    double lo[kCopyUnroll], hi[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const size_t i = b + (size_t)u * kBlock;
      const double* p = reinterpret_cast<const double*>(src + (i < n16 ? i : b));
      lo[u] = __builtin_nontemporal_load(p);
      hi[u] = __builtin_nontemporal_load(p + 1);
    }
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const size_t i = b + (size_t)u * kBlock;
      if (i < n16) {
        double* q = reinterpret_cast<double*>(dst + i);
        __builtin_nontemporal_store(lo[u], q);
        __builtin_nontemporal_store(hi[u], q + 1);
      }
    }
  }
}

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

// Block reduction of acc[0..nv) and acc[KM] (the squared-norm slot, when
// with_norm) into partials[blockIdx.x][i] and partials[blockIdx.x][kMaxBasis].
template <int KM>
__device__ __forceinline__ void store_block_partials(double (&acc)[KM + 1], int nv, int with_norm,
                                                     double* __restrict__ partials) {
  __shared__ double red[kBlock / 64][KM + 1];
  const int lane = threadIdx.x & 63, wvi = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i <= KM; ++i) {
    if (i < nv || (i == KM && with_norm)) {
      const double s = group_sum<64>(acc[i]);
      if (lane == 0) red[wvi][i] = s;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= KM; i += kBlock) {
    if (i < nv || (i == KM && with_norm)) {
      double s = red[0][i];
      for (int q = 1; q < kBlock / 64; ++q) s += red[q][i];
      partials[(size_t)blockIdx.x * (kMaxBasis + 1) + (i == KM ? kMaxBasis : i)] = s;
    }
  }
}

// partials[b][i] = block sum of w * V_i (i < nv <= KM); slot kMaxBasis = block sum
// of w * w when with_norm.  V may be null when nv == 0.
template <typename TV, int KM>
__global__ __launch_bounds__(kBlock) void k_mdot(size_t len, const double* __restrict__ w,
                                                 const TV* __restrict__ V, size_t ldv, int nv,
                                                 int with_norm, double* __restrict__ partials) {
  double acc[KM + 1];
#pragma unroll
  for (int i = 0; i <= KM; ++i) acc[i] = 0.0;
  for (size_t t = blockIdx.x * (size_t)kBlock + threadIdx.x; t < len; t += (size_t)gridDim.x * kBlock) {
    double vv[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i) vv[i] = i < nv ? (double)V[(size_t)i * ldv + t] : 0.0;
    const double wv = w[t];
#pragma unroll
    for (int i = 0; i < KM; ++i) acc[i] += wv * vv[i];
    acc[KM] += wv * wv;
  }
  store_block_partials<KM>(acc, nv, with_norm, partials);
}

// out[i] = sum_b partials[b][i] for every requested slot i (i < nv, and slot
// kMaxBasis when with_norm); one block per slot, fixed summation order.  If
// accumulate, out[i] += the sum.
__global__ __launch_bounds__(kBlock) void k_mdot_finalize(const double* __restrict__ partials, int nb, int nv,
                                                          int with_norm, double* __restrict__ out,
                                                          int accumulate) {
  const int i = blockIdx.x;
  if (!(i < nv || (i == kMaxBasis && with_norm))) return;
  double v[1] = {0.0};
  for (int b = threadIdx.x; b < nb; b += kBlock) v[0] += partials[(size_t)b * (kMaxBasis + 1) + i];
  block_sum<1>(v);
  if (threadIdx.x == 0) out[i] = accumulate ? out[i] + v[0] : v[0];
}

// ------------------------------------------- Arnoldi with delayed reorthogonalization
// One Arnoldi step touches the basis in two passes.  The stored vectors V_i are
// never rewritten: the orthonormal basis is V' = V T with an upper-triangular T
// kept on the host (it holds the normalizations and the second projections).
// On entry V_k is the previous step's projected vector (scaled to about unit
// norm, not yet projected a second time) and w = S z_k.
//   dots:   R = V_{<k}^T V_k, B = V_{<k}^T w, c = V_k.V_k, d = V_k.w, e = w.w
//   update: V_{k+1} = (w - V_{<=k} g) / rho
// where the host turns R, B into projections on V' (s = T^T R, b = T^T B),
// derives alpha^2 = c - |s|^2, h_kk = (d - s.b) / alpha, the new column of T and
// the combination g = T [b; h_kk].
constexpr int kArnSlots = 2 * kMaxBasis + 4;   // partial slots of the dots pass

template <int KM>
struct ArnSlots {
  static constexpr int kC = 2 * KM, kD = 2 * KM + 1, kE = 2 * KM + 2, kCount = 2 * KM + 3;
};

// partials[b][slot], slots: [0,KM) R_i, [KM,2KM) B_i, then c, d, e (ArnSlots).
// Pairs of entries per access (16 bytes; the basis stride ldv is even), the odd
// last entry of an odd len by the first thread.
template <int KM>
__global__ __launch_bounds__(kBlock) void k_arnoldi_dots(size_t len, const double* __restrict__ V, size_t ldv,
                                                         int k, const double* __restrict__ w,
                                                         double* __restrict__ partials) {
  using S = ArnSlots<KM>;
  double acc[S::kCount];
#pragma unroll
  for (int i = 0; i < S::kCount; ++i) acc[i] = 0.0;
  const double* __restrict__ vk = V + (size_t)k * ldv;
  auto add = [&](const double (&vv)[KM], double v, double wv) {
#pragma unroll
    for (int i = 0; i < KM; ++i) {
      acc[i] += vv[i] * v;
      acc[KM + i] += vv[i] * wv;
    }
    acc[S::kC] += v * v;
    acc[S::kD] += v * wv;
    acc[S::kE] += wv * wv;
  };
  const size_t np = len / 2;
  for (size_t t = blockIdx.x * (size_t)kBlock + threadIdx.x; t < np; t += (size_t)gridDim.x * kBlock) {
    double2 vv2[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i)
      vv2[i] = i < k ? *reinterpret_cast<const double2*>(V + (size_t)i * ldv + 2 * t) : double2{0.0, 0.0};
    const double2 v2 = *reinterpret_cast<const double2*>(vk + 2 * t);
    const double2 w2 = *reinterpret_cast<const double2*>(w + 2 * t);
    double va[KM], vb[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i) { va[i] = vv2[i].x; vb[i] = vv2[i].y; }
    add(va, v2.x, w2.x);
    add(vb, v2.y, w2.y);
  }
  if ((len & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    double vv[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i) vv[i] = i < k ? V[(size_t)i * ldv + len - 1] : 0.0;
    add(vv, vk[len - 1], w[len - 1]);
  }
  __shared__ double red[kBlock / 64][S::kCount];
  const int lane = threadIdx.x & 63, wvi = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < S::kCount; ++i) {
    const double s = group_sum<64>(acc[i]);
    if (lane == 0) red[wvi][i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < S::kCount; i += kBlock) {
    double s = red[0][i];
    for (int q = 1; q < kBlock / 64; ++q) s += red[q][i];
    partials[(size_t)blockIdx.x * kArnSlots + i] = s;
  }
}

// out[i] = sum_b partials[b][i], one block per slot, fixed order.
__global__ __launch_bounds__(kBlock) void k_partials_finalize(const double* __restrict__ partials, int nb,
                                                              int stride, double* __restrict__ out) {
  const int i = blockIdx.x;
  double v[1] = {0.0};
  for (int b = threadIdx.x; b < nb; b += kBlock) v[0] += partials[(size_t)b * stride + i];
  block_sum<1>(v);
  if (threadIdx.x == 0) out[i] = v[0];
}

// Copy nv FP64 values into host-mapped memory, then store seq into the host
// publish word; the system-scope fence orders the values before the word, so a
// host that reads seq reads complete values (one wave).
__global__ __launch_bounds__(64) void k_publish(const double* __restrict__ src, int nv, double* __restrict__ dst,
                                                unsigned* __restrict__ word, unsigned seq) {
  for (int i = threadIdx.x; i < nv; i += 64) dst[i] = src[i];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(word, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

struct ArnCoef {
  double g[kMaxBasis];   // coefficients of V_0..V_k
  double inv_rho;
};

// The update pass V_{k+1} = (w - sum_{i<=k} g_i V_i) * inv_rho (KM >= k + 1).  If
// norm_partials is not null, partials[b] = block sum of the squared entries of
// the unscaled vector.  Pairs of entries per access, as k_arnoldi_dots.
template <int KM>
__global__ __launch_bounds__(kBlock) void k_arnoldi_update(size_t len, double* __restrict__ V, size_t ldv, int k,
                                                           const double* __restrict__ w, ArnCoef cf,
                                                           double* __restrict__ norm_partials) {
  double* __restrict__ vn = V + (size_t)(k + 1) * ldv;
  double acc[1] = {0.0};
  const size_t np = len / 2;
  for (size_t t = blockIdx.x * (size_t)kBlock + threadIdx.x; t < np; t += (size_t)gridDim.x * kBlock) {
    double2 vv2[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i)
      vv2[i] = i <= k ? *reinterpret_cast<const double2*>(V + (size_t)i * ldv + 2 * t) : double2{0.0, 0.0};
    const double2 w2 = *reinterpret_cast<const double2*>(w + 2 * t);
    double wa = w2.x, wb = w2.y;
#pragma unroll
    for (int i = 0; i < KM; ++i) {
      wa -= cf.g[i] * vv2[i].x;
      wb -= cf.g[i] * vv2[i].y;
    }
    __builtin_nontemporal_store(wa * cf.inv_rho, vn + 2 * t);
    __builtin_nontemporal_store(wb * cf.inv_rho, vn + 2 * t + 1);
    acc[0] += wa * wa;
    acc[0] += wb * wb;
  }
  if ((len & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    double ws = w[len - 1];
#pragma unroll
    for (int i = 0; i < KM; ++i) ws -= cf.g[i] * (i <= k ? V[(size_t)i * ldv + len - 1] : 0.0);
    vn[len - 1] = ws * cf.inv_rho;
    acc[0] += ws * ws;
  }
  if (norm_partials) {
    block_sum<1>(acc);
    if (threadIdx.x == 0) norm_partials[blockIdx.x] = acc[0];
  }
}

struct BasisCoef {
  double y[kMaxBasis];
};

// x += sum_i y_i Z_i, pairs of entries per access (ldz even) where x is 16-byte
// aligned, else one entry per access.
template <typename TZ, int KM>
__global__ __launch_bounds__(kBlock) void k_basis_axpy(size_t len, double* __restrict__ x,
                                                       const TZ* __restrict__ Z, size_t ldz, int nz, BasisCoef cf) {
  using Z2 = typename std::conditional<std::is_same<TZ, float>::value, float2, double2>::type;
  if (reinterpret_cast<uintptr_t>(x) & 15) {
    for (size_t t = blockIdx.x * (size_t)kBlock + threadIdx.x; t < len; t += (size_t)gridDim.x * kBlock) {
      double s = x[t];
#pragma unroll
      for (int i = 0; i < KM; ++i)
        if (i < nz) s += cf.y[i] * (double)Z[(size_t)i * ldz + t];
      x[t] = s;
    }
    return;
  }
  const size_t np = len / 2;
  for (size_t t = blockIdx.x * (size_t)kBlock + threadIdx.x; t < np; t += (size_t)gridDim.x * kBlock) {
    double2 s = *reinterpret_cast<const double2*>(x + 2 * t);
#pragma unroll
    for (int i = 0; i < KM; ++i)
      if (i < nz) {
        const Z2 z = *reinterpret_cast<const Z2*>(Z + (size_t)i * ldz + 2 * t);
        s.x += cf.y[i] * (double)z.x;
        s.y += cf.y[i] * (double)z.y;
      }
    *reinterpret_cast<double2*>(x + 2 * t) = s;
  }
  if ((len & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    double s = x[len - 1];
#pragma unroll
    for (int i = 0; i < KM; ++i)
      if (i < nz) s += cf.y[i] * (double)Z[(size_t)i * ldz + len - 1];
    x[len - 1] = s;
  }
}

}  // namespace smg
