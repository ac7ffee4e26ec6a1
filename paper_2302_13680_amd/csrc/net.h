// net.h -- kernels of the warm-start network: 3x3 / 1x1 convolutions as
// implicit GEMMs on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16: BF16
// operands, FP32 accumulation, K = 32 per instruction), SiLU, masked MSE loss
// and Adam.
//
// Tensors are NHWC.  Activations feeding a matrix product are BF16; pre-
// activations, gradients of activations, weight gradients and the master
// weights are FP32.  MFMA operand layout (one wavefront, 16x16x32; checked on
// the device with small integer matrices):
//   A (16 x 32, M x K): lane l holds A[l % 16][8 (l / 16) + j], j = 0..7
//   B (32 x 16, K x N): lane l holds B[8 (l / 16) + j][l % 16]
//   D (16 x 16, M x N): lane l holds D[4 (l / 16) + i][l % 16], i = 0..3
// Each lane's eight K values are two runs of four (channel counts are multiples
// of four), loaded as two 8-byte accesses.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smgnet {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8s __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// acc += A B for one 16x16x32 tile (operands as 8 BF16 bit patterns per lane)
__device__ __forceinline__ f32x4 mfma_k32(bf16x4 alo, bf16x4 ahi, bf16x4 blo, bf16x4 bhi, f32x4 acc) {
  const bf16x8s a = __builtin_shufflevector(alo, ahi, 0, 1, 2, 3, 4, 5, 6, 7);
  const bf16x8s b = __builtin_shufflevector(blo, bhi, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), acc,
                                                 0, 0, 0);
}

constexpr int kNetBlock = 256;   // 4 wavefronts

// float -> bfloat16 bits, round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + __expf(-z)); }

struct ConvGeom {
  int B, Hin, Win, Hout, Wout, Cin, Cout, CoutP, taps, stride, up;
  // CoutP: Cout rounded up to a multiple of 4 (channel stride of BF16 gradients)
};

// Input coordinate read by output pixel (yo, xo) through tap (ky, kx); false
// if it falls in the zero padding.
__device__ __forceinline__ bool tap_src(const ConvGeom& g, int yo, int xo, int tap, int& yi, int& xi) {
  const int k = g.taps == 9 ? 3 : 1, pad = k >> 1;
  const int ky = tap / k, kx = tap - ky * k;
  if (g.up) {
    const int yu = yo + ky - pad, xu = xo + kx - pad;   // upsampled grid = output grid
    if (yu < 0 || yu >= g.Hout || xu < 0 || xu >= g.Wout) return false;
    yi = yu >> 1; xi = xu >> 1;
    return true;
  }
  yi = g.stride * yo + ky - pad;
  xi = g.stride * xo + kx - pad;
  return yi >= 0 && yi < g.Hin && xi >= 0 && xi < g.Win;
}

// ----------------------------------------------------------------- forward
// z = conv(in) + bias (+ skip), a = SiLU(z) (act) or a = z; out pre-activation z
// in FP32 and the BF16 activation a (if a != null).  One wavefront computes 16
// output pixels x every output channel (up to 4 tiles of 16).
__global__ __launch_bounds__(kNetBlock) void k_conv_fwd(ConvGeom g, const uint16_t* __restrict__ in,
                                                        const uint16_t* __restrict__ W,
                                                        const float* __restrict__ bias,
                                                        const uint16_t* __restrict__ skip, int act,
                                                        float* __restrict__ z, uint16_t* __restrict__ a) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * kNetBlock + threadIdx.x) >> 6;
  const int P = g.B * g.Hout * g.Wout;
  const int p0 = wave * 16;
  if (p0 >= P) return;
  const int K = g.taps * g.Cin;
  const int NT = (g.Cout + 15) >> 4;
  // the A-row pixel of this lane
  const int pr = p0 + (lane & 15);
  int rb = 0, ryo = 0, rxo = 0;
  const bool rvalid = pr < P;
  if (rvalid) { rb = pr / (g.Hout * g.Wout); const int rem = pr - rb * g.Hout * g.Wout; ryo = rem / g.Wout; rxo = rem - ryo * g.Wout; }
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kq = 4 * (lane >> 4);      // D rows of this lane
  const int k8 = 8 * (lane >> 4);      // first of this lane's eight K values
  for (int k0 = 0; k0 < K; k0 += 32) {
    bf16x4 av[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k4 = k0 + k8 + 4 * h;
      av[h] = bf16x4{0, 0, 0, 0};
      if (rvalid && k4 < K) {
        const int tap = k4 / g.Cin, ci = k4 - tap * g.Cin;
        int yi, xi;
        if (tap_src(g, ryo, rxo, tap, yi, xi))
          av[h] = *(const bf16x4*)(in + (((size_t)rb * g.Hin + yi) * g.Win + xi) * g.Cin + ci);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t < NT) {
        const int co = 16 * t + (lane & 15);
        bf16x4 bv[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int k4 = k0 + k8 + 4 * h;
          bv[h] = bf16x4{0, 0, 0, 0};
          if (co < g.Cout && k4 < K) bv[h] = *(const bf16x4*)(W + (size_t)co * K + k4);
        }
        acc[t] = mfma_k32(av[0], av[1], bv[0], bv[1], acc[t]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (t >= NT) continue;
    const int co = 16 * t + (lane & 15);
    if (co >= g.Cout) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p = p0 + kq + i;
      if (p >= P) continue;
      float v = acc[t][i] + bias[co];
      if (skip) v += bf2f(skip[(size_t)p * g.Cout + co]);
      z[(size_t)p * g.Cout + co] = v;
      if (a) a[(size_t)p * g.Cout + co] = f2bf(act ? v * sigm(v) : v);
    }
  }
}

// ------------------------------------------------------- backward: gradients
// dz = dA * SiLU'(z) (act) or dA; writes dz in FP32 (for the bias gradient) and
// BF16 with channel stride CoutP (zero pad channels); adds dz into dskip (the
// gradient of the skip tensor) when given.
__global__ void k_silu_bwd(int P, int Cout, int CoutP, int act, const float* __restrict__ dA,
                           const float* __restrict__ z, float* __restrict__ dz32, uint16_t* __restrict__ dz16,
                           float* __restrict__ dskip) {
  const size_t tot = (size_t)P * CoutP;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < tot; i += (size_t)gridDim.x * blockDim.x) {
    const size_t p = i / CoutP;
    const int c = (int)(i - p * CoutP);
    float d = 0.f;
    if (c < Cout) {
      const size_t o = p * Cout + c;
      d = dA[o];
      if (act) { const float zz = z[o]; const float s = sigm(zz); d *= s * (1.f + zz * (1.f - s)); }
      dz32[o] = d;
      if (dskip) dskip[o] += d;
    }
    dz16[i] = f2bf(d);
  }
}

// dIn[pixel][ci] (+)= sum_{co, tap} W[co][tap][ci] dz[out pixel(s) reading it][co].
// GEMM with rows = input pixels, columns = ci, reduction over (tap, sub, co);
// for upsampled inputs each tap reaches 2x2 output pixels (sub = 0..3).
// WT: BF16 weights transposed to [ci][tap][CoutP].
__global__ __launch_bounds__(kNetBlock) void k_conv_bwd_data(ConvGeom g, const uint16_t* __restrict__ dz16,
                                                             const uint16_t* __restrict__ WT,
                                                             float* __restrict__ dIn) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * kNetBlock + threadIdx.x) >> 6;
  const int P = g.B * g.Hin * g.Win;
  const int p0 = wave * 16;
  if (p0 >= P) return;
  const int NT = (g.Cin + 15) >> 4;
  const int pr = p0 + (lane & 15);
  const bool rvalid = pr < P;
  int rb = 0, ryi = 0, rxi = 0;
  if (rvalid) { rb = pr / (g.Hin * g.Win); const int rem = pr - rb * g.Hin * g.Win; ryi = rem / g.Win; rxi = rem - ryi * g.Win; }
  const int k = g.taps == 9 ? 3 : 1, pad = k >> 1;
  const int nsub = g.up ? 4 : 1;
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kq = 4 * (lane >> 4);      // D rows of this lane
  const int k8 = 8 * (lane >> 4);      // first of this lane's eight reduction values
  for (int tap = 0; tap < g.taps; ++tap) {
    const int ky = tap / k, kx = tap - ky * k;
    for (int sub = 0; sub < nsub; ++sub) {
      // the output pixel that reads input (ryi, rxi) through this tap (and sub-position)
      int yo, xo;
      bool ok = rvalid;
      if (g.up) {
        yo = 2 * ryi + (sub >> 1) - ky + pad;
        xo = 2 * rxi + (sub & 1) - kx + pad;
      } else {
        const int ny = ryi - ky + pad, nx = rxi - kx + pad;
        ok = ok && ny >= 0 && nx >= 0 && (ny % g.stride) == 0 && (nx % g.stride) == 0;
        yo = ny / g.stride;
        xo = nx / g.stride;
      }
      ok = ok && yo >= 0 && yo < g.Hout && xo >= 0 && xo < g.Wout;
      const size_t orow = ((size_t)rb * g.Hout + (ok ? yo : 0)) * g.Wout + (ok ? xo : 0);
      for (int c0 = 0; c0 < g.CoutP; c0 += 32) {
        bf16x4 av[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int co = c0 + k8 + 4 * h;
          av[h] = bf16x4{0, 0, 0, 0};
          if (ok && co < g.CoutP) av[h] = *(const bf16x4*)(dz16 + orow * g.CoutP + co);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          if (t < NT) {
            const int ci = 16 * t + (lane & 15);
            bf16x4 bv[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int co = c0 + k8 + 4 * h;
              bv[h] = bf16x4{0, 0, 0, 0};
              if (ci < g.Cin && co < g.CoutP)
                bv[h] = *(const bf16x4*)(WT + ((size_t)ci * g.taps + tap) * g.CoutP + co);
            }
            acc[t] = mfma_k32(av[0], av[1], bv[0], bv[1], acc[t]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (t >= NT) continue;
    const int ci = 16 * t + (lane & 15);
    if (ci >= g.Cin) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p = p0 + kq + i;
      if (p < P) dIn[(size_t)p * g.Cin + ci] += acc[t][i];
    }
  }
}

// Partial weight gradients over one chunk of output pixels:
//   part[chunk][co][k] = sum_{p in chunk} dz[p][co] im2col(in)[p][k],  k = tap Cin + ci.
// One wavefront per (co tile, k tile, chunk): GEMM rows co, columns k, reduction
// over pixels 16 at a time.
__global__ __launch_bounds__(kNetBlock) void k_conv_bwd_weight(ConvGeom g, const uint16_t* __restrict__ in,
                                                               const uint16_t* __restrict__ dz16, int chunk,
                                                               int nchunks, float* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * kNetBlock + threadIdx.x) >> 6;
  const int K = g.taps * g.Cin;
  const int nct = (g.Cout + 15) >> 4, nkt = (K + 15) >> 4;
  if (wave >= nct * nkt * nchunks) return;
  const int ch = wave / (nct * nkt);
  const int rem = wave - ch * nct * nkt;
  const int ct = rem / nkt, kt = rem - ct * nkt;
  const int P = g.B * g.Hout * g.Wout;
  const int pbeg = ch * chunk, pend = min(P, pbeg + chunk);
  const int co_r = 16 * ct + (lane & 15);        // A row (co) of this lane
  const int kcol = 16 * kt + (lane & 15);        // B column (k) of this lane
  const int tap = kcol / g.Cin, ci = kcol - (kcol / g.Cin) * g.Cin;
  const bool colv = kcol < K;
  const int kq = 4 * (lane >> 4);      // D rows of this lane
  const int k8 = 8 * (lane >> 4);      // first of this lane's eight pixels
  f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int q0 = pbeg; q0 < pend; q0 += 32) {
    bf16x4 av[2], bv[2];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int p = q0 + k8 + j;
      short aj = 0, bj = 0;
      if (p < pend) {
        if (co_r < g.Cout) aj = (short)dz16[(size_t)p * g.CoutP + co_r];
        if (colv) {
          const int b = p / (g.Hout * g.Wout);
          const int r = p - b * g.Hout * g.Wout;
          const int yo = r / g.Wout, xo = r - (r / g.Wout) * g.Wout;
          int yi, xi;
          if (tap_src(g, yo, xo, tap, yi, xi)) bj = (short)in[(((size_t)b * g.Hin + yi) * g.Win + xi) * g.Cin + ci];
        }
      }
      av[j >> 2][j & 3] = aj;
      bv[j >> 2][j & 3] = bj;
    }
    acc = mfma_k32(av[0], av[1], bv[0], bv[1], acc);
  }
  // D[co = 16 ct + kq + i][k = kcol]
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int co = 16 * ct + kq + i;
    if (co < g.Cout && colv) part[((size_t)ch * g.Cout + co) * K + kcol] = acc[i];
  }
}

// dW[co][k] = sum over chunks (fixed order); db[co] = sum_p dz32[p][co].
__global__ void k_wgrad_reduce(int Cout, int K, int nchunks, const float* __restrict__ part,
                               float* __restrict__ dW) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Cout * K) return;
  float s = 0.f;
  for (int c = 0; c < nchunks; ++c) s += part[(size_t)c * Cout * K + i];
  dW[i] = s;
}

__global__ __launch_bounds__(kNetBlock) void k_bias_grad(int P, int Cout, const float* __restrict__ dz32,
                                                         float* __restrict__ db) {
  // one block per output channel, fixed order
  const int co = blockIdx.x;
  __shared__ float red[kNetBlock];
  float s = 0.f;
  for (int p = threadIdx.x; p < P; p += kNetBlock) s += dz32[(size_t)p * Cout + co];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kNetBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[co] = red[0];
}

// --------------------------------------------------------------- loss, Adam
// Masked MSE over pixels with y, x < valid and the 3 channels; dA = d loss / d out.
// Per-block partial sums of the squared error (deterministic reduction after).
__global__ __launch_bounds__(kNetBlock) void k_mse(int B, int H, int valid, const float* __restrict__ out,
                                                   const float* __restrict__ tgt, float inv_cnt,
                                                   float* __restrict__ dA, float* __restrict__ part) {
  __shared__ float red[kNetBlock];
  const size_t tot = (size_t)B * H * H * 3;
  float s = 0.f;
  for (size_t i = blockIdx.x * (size_t)kNetBlock + threadIdx.x; i < tot; i += (size_t)gridDim.x * kNetBlock) {
    const size_t pix = i / 3;
    const int x = (int)(pix % H), y = (int)((pix / H) % H);
    const bool in = y < valid && x < valid;
    const float d = in ? out[i] - tgt[i] : 0.f;
    dA[i] = 2.f * d * inv_cnt;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kNetBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum_partials(int n, const float* __restrict__ part, float scale, float* __restrict__ out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = s * scale;
  }
}

// Adam (Kingma and Ba 2015): bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t from the host.
__global__ void k_adam(size_t n, float* __restrict__ th, const float* __restrict__ gr, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float g = gr[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// BF16 weights of one layer from the FP32 master: W16[co][k] and the transposed
// WT[ci][tap][CoutP] (zero pad channels) used by the data gradient.
__global__ void k_cast_weights(int Cout, int CoutP, int taps, int Cin, const float* __restrict__ Wm,
                               uint16_t* __restrict__ W16, uint16_t* __restrict__ WT) {
  const int K = taps * Cin;
  const int tot = CoutP * K;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += gridDim.x * blockDim.x) {
    const int co = i / K, k = i - co * K;
    const int tap = k / Cin, ci = k - tap * Cin;
    const uint16_t b = co < Cout ? f2bf(Wm[(size_t)co * K + k]) : (uint16_t)0;
    if (co < Cout) W16[(size_t)co * K + k] = b;
    WT[((size_t)ci * taps + tap) * CoutP + co] = b;
  }
}

__global__ void k_f32_to_bf16(size_t n, const float* __restrict__ in, uint16_t* __restrict__ out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = f2bf(in[i]);
}

__global__ void k_fillf(size_t n, float* __restrict__ p, float v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

}  // namespace smgnet
