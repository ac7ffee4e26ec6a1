// smg.hip -- runtime and C ABI of the collective multigrid library (see include/smg.h).
//
// Host side of the method: the level hierarchy (nested grids n -> (n-1)/2,
// rediscretized coarse operators), the V-cycle of Alg. 1 as a sequence of
// kernel launches on the caller's stream, the coarsest direct solve, the
// stationary and GMRES drivers and FP64 iterative refinement around an FP32
// V-cycle.  All device memory comes from the caller's workspace, carved here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <mutex>
#include <vector>

#include "../../include/smg.h"
#include "kernels.h"
#include "sweep.h"
#include "rrwalk.h"

using namespace smg;

namespace {

constexpr int kMaxLevels = 16;
constexpr int kMaxSamples = 2048;
constexpr int kCoarseUMin = 512;   // above this many samples the coarsest u is computed once

template <typename T>
struct Level {
  int n = 0;
  T* kx = nullptr;   // [n][n+1][N]
  T* ky = nullptr;   // [n+1][n][N]
  T* c = nullptr;    // [N]
  T* d = nullptr;
  T* e = nullptr;
  T g = 0;
  T* gden = nullptr; // [n][n]: g + sum_j d_j c_j e_j / a_j^2 (node_den)
  T* mk = nullptr;   // [n][n][2] node factor pairs (md, me); (0, -0) outside the domain
  T* dom = nullptr;  // [n][n] domain (FP64 levels, contexts with a domain): 1 inside, 0 outside
  T* x = nullptr;    // level iterate (levels >= 1, and level 0 of the FP32 cycle)
  T* f = nullptr;    // level right-hand side
  T* xa = nullptr;   // second iterate of the one-launch sweep (levels >= 1 where it runs)
};

template <int V>
using IC = std::integral_constant<int, V>;

// lanes per node W and samples per lane JM for N samples
// compile-time width KM >= nv of the Krylov multi-vector kernels
constexpr int kNormStage = 128;       // blocks of the first norm-reduction stage
constexpr int kNormStageMin = 4096;   // partials above which the two-stage reduction is used

// Register width of the multi-vector kernels for nv basis vectors.
int km_width(int nv) { return nv <= 4 ? 4 : nv <= 8 ? 8 : nv <= 16 ? 16 : 32; }

template <typename F>
void km_dispatch(int nv, F&& fn) {
  switch (km_width(nv)) {
    case 4: fn(IC<4>{}); break;
    case 8: fn(IC<8>{}); break;
    case 16: fn(IC<16>{}); break;
    default: fn(IC<32>{}); break;
  }
}

template <typename F>
void seg_dispatch(int N, F&& fn) {
  if (N <= 1) fn(IC<1>{}, IC<1>{});
  else if (N <= 2) fn(IC<2>{}, IC<1>{});
  else if (N <= 4) fn(IC<4>{}, IC<1>{});
  else if (N <= 8) fn(IC<8>{}, IC<1>{});
  else if (N <= 16) fn(IC<16>{}, IC<1>{});
  else if (N <= 32) fn(IC<32>{}, IC<1>{});
  else if (N <= 64) fn(IC<64>{}, IC<1>{});
  else if (N <= 128) fn(IC<64>{}, IC<2>{});
  else if (N <= 256) fn(IC<64>{}, IC<4>{});
  else if (N <= 512) fn(IC<64>{}, IC<8>{});
  else if (N <= 1024) fn(IC<64>{}, IC<16>{});
  else fn(IC<64>{}, IC<32>{});
}

// Lanes per node W, samples per lane JM and samples per access VW of a
// context's level kernels.  FP64 contexts, and FP32 contexts with odd N: one
// sample per access, W = min(64, pow2ceil(N)).  FP32 contexts with even N:
// W = min(64, pow2ceil(N/2)) lanes with two samples per access in FP32
// arithmetic (8-byte accesses; 4-byte ones stream at ~65% of the 8-byte rate);
// the FP64 kernels of such a context keep one sample per access on the same W
// and JM, so the batched solver (which uses the same widths) reproduces them.
bool vec2_ctx(int precision, int N) { return precision == SMG_F32 && (N & 1) == 0; }

// The FP32 half-sweep keeps one sample per access with four or more samples per
// lane: measured at 511x511, N=256 it runs 271 us that way against 283-291 us
// with pairs (the residual and restriction gain from pairs at every N).
constexpr int halfsweep_vw(int vw, int jm) { return vw == 2 && jm == 2 ? 2 : 1; }

// Kernels compiled without the control mask (MK = false) for contexts whose
// control acts on every node, with it otherwise.
template <typename F>
void mask_dispatch(bool masked, F&& fn) {
  if (masked) fn(std::true_type{}); else fn(std::false_type{});
}

template <bool kVec2, typename F>
void lane_dispatch(int precision, int N, F&& fn) {
  if (vec2_ctx(precision, N)) {
    auto go = [&](auto Wc, auto Jc) {
      if constexpr (kVec2) fn(Wc, Jc, IC<2>{}); else fn(Wc, Jc, IC<1>{});
    };
    if (N <= 2) go(IC<1>{}, IC<2>{});
    else if (N <= 4) go(IC<2>{}, IC<2>{});
    else if (N <= 8) go(IC<4>{}, IC<2>{});
    else if (N <= 16) go(IC<8>{}, IC<2>{});
    else if (N <= 32) go(IC<16>{}, IC<2>{});
    else if (N <= 64) go(IC<32>{}, IC<2>{});
    else if (N <= 128) go(IC<64>{}, IC<2>{});
    else if (N <= 256) go(IC<64>{}, IC<4>{});
    else if (N <= 512) go(IC<64>{}, IC<8>{});
    else if (N <= 1024) go(IC<64>{}, IC<16>{});
    else go(IC<64>{}, IC<32>{});
  } else {
    seg_dispatch(N, [&](auto Wc, auto Jc) { fn(Wc, Jc, IC<1>{}); });
  }
}

// Lanes per coarse node of the fused residual + restriction: the smoother's
// widths while one chunk of VW samples per lane covers N (up to 64 lanes), then
// groups of 128 or 256 lanes (several waves) so that every lane still handles
// one chunk: with all ~90 loads of a chunk in flight at once, a second chunk per
// lane would need more registers than two waves per SIMD leave.  (FP64 in
// 16-byte accesses, 128 lanes of two samples at N = 256, was slower at 511x511:
// 1.20 against 1.01 ms for the finest level.)
template <bool kVec2, typename F>
void rr_dispatch(int precision, int N, F&& fn) {
  const bool v2 = kVec2 && vec2_ctx(precision, N);
  const int M = v2 ? N / 2 : N;   // accesses per node and field
  if (M <= 64) {
    if (v2) lane_dispatch<kVec2>(precision, N, fn);
    else seg_dispatch(N, [&](auto Wc, auto Jc) { fn(Wc, Jc, IC<1>{}); });
    return;
  }
  auto go = [&](auto Wc, auto Cc) {   // Cc: chunks per lane
    constexpr int C = decltype(Cc)::value;
    if constexpr (kVec2) {
      if (v2) {
        fn(Wc, IC<2 * C>{}, IC<2>{});
        return;
      }
    }
    fn(Wc, IC<C>{}, IC<1>{});
  };
  if (M <= 128) go(IC<128>{}, IC<1>{});
  else if (M <= 256) go(IC<256>{}, IC<1>{});
  else if (M <= 512) go(IC<256>{}, IC<2>{});
  else if (M <= 1024) go(IC<256>{}, IC<4>{});
  else go(IC<256>{}, IC<8>{});
}

// Lanes per node W and samples per lane JM of the smoother's layout.
void smoother_layout(int precision, int N, int* W, int* JM) {
  lane_dispatch<true>(precision, N, [&](auto Wc, auto Jc, auto) {
    *W = decltype(Wc)::value;
    *JM = decltype(Jc)::value;
  });
}

// Where a sweep runs as one launch (k_sweep_fused).  The one-launch sweep reads
// every face once but recomputes the reds at the pair borders and walks each
// column in serial steps of one memory round trip each, so it needs enough work
// per step (two or more samples per lane, N = 65..256) and a level that streams
// from HBM.  Measured (one-launch against two half-sweeps, us, 16-byte FP64
// pairs): 511x511, N=256 FP64 788 / 1225, FP32 428 / 518; N=192 (three samples
// per lane, one per access) 255x255 FP64 213 / 323, FP32 107 / 151; N=128
// 511x511 FP64 450 / 755, FP32 323 / 397, 255x255 FP64 128 / 198; but with one
// sample per lane (N = 64) 511x511 FP64 384 / 393, and 255x255, N=64 FP64 59 /
// 54 (cache resident).
constexpr double kOneLaunchMinBytes = 512e6;
constexpr int kOneLaunchMinJM = 2;

// Levels of this descriptor whose sweeps can run as one launch (the context's
// node factors and domain are checked at run time).
bool one_launch_desc(const smg_desc& d, int n) {
  if (d.flags & (SMG_FLAG_HALFSWEEPS | SMG_FLAG_UNFUSED | SMG_FLAG_JACOBI)) return false;
  if (d.theta != 1.0) return false;
  const double word = d.precision == SMG_F32 ? 4.0 : 8.0;
  if (d.sweep_rows == 0 && 10.0 * d.nsamples * (double)n * n * word < kOneLaunchMinBytes) return false;
  int W = 0, JM = 0;
  smoother_layout(d.precision, d.nsamples, &W, &JM);
  if (W != 64 || JM > 4) return false;
  return d.sweep_rows > 0 || JM >= kOneLaunchMinJM;
}

int count_levels(int n, int nc) {
  int nl = 1, t = n;
  while (t > nc) {
    if ((t & 1) == 0) return -1;
    t = (t - 1) / 2;
    if (++nl > kMaxLevels) return -1;
  }
  return t == nc ? nl : -1;
}

size_t vlen(int n, int N) { return (size_t)(2 * N + 1) * n * n; }

}  // namespace

struct smg_ctx {
  smg_desc desc{};
  int nlev = 0, N = 0;
  hipStream_t stream = nullptr;
  int device = 0;              // the device current at setup (the stream's)
  std::string err;
  Level<double> L64[kMaxLevels];
  Level<float> L32[kMaxLevels];
  double* r64 = nullptr;       // level-0 sized residual scratch of the FP64 cycle
  float* r32 = nullptr;        // same for the FP32 cycle
  int m = 0;                   // coarsest unknowns per field
  double* Ainv = nullptr;      // [N][m][m]
  double* Sinv = nullptr;      // [m][m]
  double* ds = nullptr;        // [N][m]
  double* terms = nullptr;     // [N][m][m], setup only
  double* schur_part = nullptr;   // [ceil(N / kSchurChunk)][m][m]: terms summed per chunk of samples
  double* cu = nullptr;           // [m]: the coarsest u, computed once when N > kCoarseUMin
  double* partials = nullptr;  // [npart][4] per-block squared norms of a residual and of f
  size_t npart = 0;
  double* partials2 = nullptr; // [kNormStage][4] first-stage sums of many partials
  double* norms = nullptr;     // [4]
  double* mdp = nullptr;       // [kPartials][kArnSlots] partials of the Krylov reductions
  double* hdev = nullptr;      // [3][kMaxBasis+1]
  int* flag = nullptr;
  double* V = nullptr;         // [(m+1)][ldk] Krylov basis
  double* Z64 = nullptr;       // [m][ldk] preconditioned basis (FP64 cycle)
  float* Z32 = nullptr;        // [m][ldk] preconditioned basis (FP32 cycle)
  size_t ldk = 0;              // basis stride: len0 rounded up to 64 (16-byte aligned pairs)
  double* w = nullptr;         // [len0]
  double* rr = nullptr;        // [len0]
  size_t len0 = 0;
  double* host = nullptr;      // host-mapped staging of read-back values (pinned, coherent)
  double* host_dev = nullptr;  // the same memory as the device addresses it
  unsigned* pub_host = nullptr;   // publish word after the values, host and device views
  unsigned* pub_dev = nullptr;
  unsigned pub_seq = 0;
  bool masked = false;         // node factors other than 1 somewhere (local control, Newton systems)
  bool domain = false;         // a domain other than the square (nodes held at zero outside)
  // semismooth Newton buffers (SMG_FLAG_SSN): increment, right-hand side, node vectors
  // E[p], E[dp], F, chi, per-block partials and their sums
  double *sdx = nullptr, *sr = nullptr, *sw = nullptr, *sdw = nullptr, *sF = nullptr, *schi = nullptr;
  double *spart = nullptr, *sout = nullptr;
  // risk-averse buffers (SMG_FLAG_CVAR): rank-one vectors z_j [nn][N], weights w_j,
  // per-sample scratch, partials, c_j on the device; right-hand side b(c), residual
  // -F_1, Newton increment, saved iterate, J_12, J_11^{-1} J_12, residual scratch
  double *cz = nullptr, *cwv = nullptr, *cs = nullptr, *cpart = nullptr, *cc = nullptr;
  double *cb = nullptr, *cr = nullptr, *cdx = nullptr, *cxk = nullptr, *cj12 = nullptr, *cxi = nullptr,
         *clr = nullptr, *cxt = nullptr;
  bool lr_on = false;          // rank-one terms in the finest-level operator
  size_t used_bytes = 0;
  // captured V-cycles, one per (x, f, kind); kind = precision * 2 + zero_first
  struct Graph {
    const void* x;
    const void* f;
    int kind;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
  hipStream_t cap_stream = nullptr;  // private stream used only while capturing
};

namespace {

struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

bool desc_valid(const smg_desc& d, std::string* why) {
  auto fail = [&](const char* m) { if (why) *why = m; return false; };
  if (d.nsamples < 1 || d.nsamples > kMaxSamples) return fail("nsamples must be in [1, 2048]");
  if (d.coarsest_n < 1 || d.coarsest_n > 7 || (d.coarsest_n & 1) == 0) return fail("coarsest_n must be odd and <= 7");
  if (d.n < 1 || count_levels(d.n, d.coarsest_n) < 1) return fail("n must be (coarsest_n+1)*2^k - 1");
  if (d.pre < 0 || d.post < 0 || d.pre > 64 || d.post > 64) return fail("pre/post out of range");
  if (!(d.theta > 0.0 && d.theta < 2.0)) return fail("theta must lie in (0, 2)");
  if (d.precision != SMG_F64 && d.precision != SMG_F32) return fail("precision must be SMG_F64 or SMG_F32");
  if (d.gmres_restart < 0 || d.gmres_restart > kMaxBasis - 1) return fail("gmres_restart must be in [0, 31]");
  if (d.flags & ~(SMG_FLAG_EAGER | SMG_FLAG_UNFUSED | SMG_FLAG_JACOBI | SMG_FLAG_SSN | SMG_FLAG_CVAR |
                  SMG_FLAG_HALFSWEEPS))
    return fail("unknown flag bits");
  if (d.sweep_rows < 0) return fail("sweep_rows must be >= 0");
  if ((d.flags & SMG_FLAG_CVAR) && d.precision != SMG_F64) return fail("SMG_FLAG_CVAR needs SMG_F64");
  if (d.strip < 0 || (d.strip & 1)) return fail("strip must be 0 or a positive even number");
  return true;
}

smg_desc normalized(const smg_desc& in) {
  smg_desc d = in;
  if (d.coarsest_n == 0) d.coarsest_n = 7;
  if (d.theta == 0.0) d.theta = 1.0;
  return d;
}

// Lay out (base == null: only size) every device buffer of a context.
size_t plan(const smg_desc& d, smg_ctx* C, void* base) {
  Carver cv(base);
  const int N = d.nsamples, nl = count_levels(d.n, d.coarsest_n);
  const bool f32 = d.precision == SMG_F32;
  int n = d.n;
  for (int l = 0; l < nl; ++l) {
    Level<double>& L = C->L64[l];
    L.n = n;
    const size_t fx = (size_t)n * (n + 1) * N, len = vlen(n, N);
    if (l > 0) { L.kx = cv.take<double>(fx); L.ky = cv.take<double>(fx); }
    L.c = cv.take<double>(N); L.d = cv.take<double>(N); L.e = cv.take<double>(N);
    L.gden = cv.take<double>((size_t)n * n);
    if (l > 0 && !f32) { L.x = cv.take<double>(len); L.f = cv.take<double>(len); }
    if (f32) {
      Level<float>& M = C->L32[l];
      M.n = n;
      M.kx = cv.take<float>(fx); M.ky = cv.take<float>(fx);
      M.c = cv.take<float>(N); M.d = cv.take<float>(N); M.e = cv.take<float>(N);
      M.gden = cv.take<float>((size_t)n * n);
      M.x = cv.take<float>(len); M.f = cv.take<float>(len);
    }
    n = (n - 1) / 2;
  }
  const size_t len0 = vlen(d.n, N);
  C->len0 = len0;
  if (f32) C->r32 = cv.take<float>(len0); else C->r64 = cv.take<double>(len0);
  const int m = d.coarsest_n * d.coarsest_n;
  C->m = m;
  C->Ainv = cv.take<double>((size_t)N * m * m);
  C->Sinv = cv.take<double>((size_t)m * m);
  C->ds = cv.take<double>((size_t)N * m);
  C->terms = cv.take<double>((size_t)N * m * m);
  C->npart = ((size_t)d.n * d.n + 3) / 4 + 1;   // residual blocks hold >= 4 nodes
  C->partials = cv.take<double>(C->npart * 4);
  C->partials2 = cv.take<double>((size_t)kNormStage * 4);
  C->norms = cv.take<double>(5);
  C->mdp = cv.take<double>((size_t)kPartials * kArnSlots);
  C->hdev = cv.take<double>(3 * (kMaxBasis + 1));
  C->flag = cv.take<int>(1);
  C->w = cv.take<double>(len0);
  C->rr = cv.take<double>(len0);
  const int mr = d.gmres_restart;
  if (mr > 0) {
    C->ldk = (len0 + 63) & ~(size_t)63;
    C->V = cv.take<double>(C->ldk * (mr + 1));
    if (f32) C->Z32 = cv.take<float>(C->ldk * mr); else C->Z64 = cv.take<double>(C->ldk * mr);
  }
  if (d.flags & SMG_FLAG_SSN) {
    const size_t nn = (size_t)d.n * d.n;
    C->sdx = cv.take<double>(len0);
    C->sr = cv.take<double>(len0);
    C->sw = cv.take<double>(nn);
    C->sdw = cv.take<double>(nn);
    C->sF = cv.take<double>(nn);
    C->schi = cv.take<double>(nn);
    C->spart = cv.take<double>(std::max(nn / 4 + 1, (size_t)kSsnMeritBlocks * kSsnGammas));
    C->sout = cv.take<double>(kSsnGammas);
  }
  if (d.flags & SMG_FLAG_CVAR) {
    const size_t nn = (size_t)d.n * d.n, N = d.nsamples;
    C->cz = cv.take<double>(nn * N);
    C->cwv = cv.take<double>(N);
    C->cs = cv.take<double>(N);
    C->cc = cv.take<double>(N);
    C->cpart = cv.take<double>((size_t)kSampleBlocks * N);
    C->cb = cv.take<double>(len0);
    C->cr = cv.take<double>(len0);
    C->cdx = cv.take<double>(len0);
    C->cxk = cv.take<double>(len0);
    C->cj12 = cv.take<double>(len0);
    C->cxi = cv.take<double>(len0);
    C->clr = cv.take<double>(len0);
    C->cxt = cv.take<double>(len0);
  }
  C->schur_part = cv.take<double>((size_t)((N + kSchurChunk - 1) / kSchurChunk) * m * m);
  C->cu = cv.take<double>((size_t)m);
  // node factor pairs last: the other buffers keep the places they have without them
  for (int l = 0; l < nl; ++l) {
    const size_t nn = (size_t)C->L64[l].n * C->L64[l].n;
    C->L64[l].mk = cv.take<double>(2 * nn);
    if (f32) C->L32[l].mk = cv.take<float>(2 * nn);
    C->L64[l].dom = cv.take<double>(nn);
  }
  // second iterates of the one-launch sweep on the coarse levels that use it
  // (level 0 uses the cycle's level-0 scratch)
  for (int l = 1; l < nl; ++l) {
    const int nl_n = C->L64[l].n;
    if (!one_launch_desc(d, nl_n)) continue;
    if (f32) C->L32[l].xa = cv.take<float>(vlen(nl_n, N));
    else C->L64[l].xa = cv.take<double>(vlen(nl_n, N));
  }
  return cv.off + 256;
}

int hip_fail(smg_ctx* C, hipError_t e, const char* where) {
  C->err = std::string(where) + ": " + hipGetErrorString(e);
  return SMG_EHIP;
}

#define HIP_TRY(call)                                      \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return hip_fail(C, e_, #call);   \
  } while (0)

#define LAUNCH_CHECK() HIP_TRY(hipGetLastError())
#define TRY(expr)                  \
  do {                             \
    int rc_ = (expr);              \
    if (rc_ != SMG_OK) return rc_; \
  } while (0)

int grid_for(size_t len) {
  size_t b = (len + kBlock - 1) / kBlock;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (int)b;
}

// Strip width of the smoother's traversal (colour_node): the requested one, or
// by default 64 columns on grids wider than 128 nodes (measured on the 511x511,
// N=256 finest level: 3.5% faster than row-major order, which re-reads rows
// evicted from L2; neutral at 255x255, N=64) and row-major order below.
int strip_for(int n, int requested) {
  const int s = requested > 0 ? requested : (n > 128 ? 64 : 0);
  return s > 0 && s < n ? s : n + 1;
}

template <typename T>
LevelArgs<T> args(const Level<T>& L, int N, int strip = 0) {
  LevelArgs<T> a;
  a.n = L.n; a.N = N; a.kx = L.kx; a.ky = L.ky; a.c = L.c; a.d = L.d; a.e = L.e; a.g = L.g; a.gden = L.gden; a.mk = L.mk;
  a.strip = strip_for(L.n, strip);
  return a;
}

template <typename T>
int fill(smg_ctx* C, T* p, size_t len, T v) {
  hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(len)), dim3(kBlock), 0, C->stream, len, p, v);
  LAUNCH_CHECK();
  return SMG_OK;
}

template <typename TI, typename TO>
int convert(smg_ctx* C, const TI* in, TO* out, size_t len) {
  hipLaunchKernelGGL((k_convert<TI, TO>), dim3(grid_for(len)), dim3(kBlock), 0, C->stream, len, in, out);
  LAUNCH_CHECK();
  return SMG_OK;
}

// src: kPlain (neighbours from x), kZero (x is zero), kProlong (x + P ec).
template <typename T>
int halfsweep(smg_ctx* C, const Level<T>& L, T* x, const T* f, int colour, int src = kPlain,
              const T* ec = nullptr) {
  const int nact = colour_count(L.n, colour);
  const T theta = (T)C->desc.theta;
  const LevelArgs<T> a = args(L, C->N, C->desc.strip);
  lane_dispatch<std::is_same<T, float>::value>(C->desc.precision, C->N, [&](auto Wc, auto Jc, auto Vc) {
    constexpr int W = decltype(Wc)::value, JM = decltype(Jc)::value;
    constexpr int VW = halfsweep_vw(decltype(Vc)::value, JM);
    const int per = kBlock / W, nb = (nact + per - 1) / per;
    mask_dispatch(C->masked, [&](auto Mc) {
      constexpr bool MK = decltype(Mc)::value;
      if (src == kZero)
        hipLaunchKernelGGL((k_halfsweep<T, W, JM, kZero, VW, MK>), dim3(nb), dim3(kBlock), 0, C->stream, a, x, f,
                           colour, theta, nact, ec);
      else if (src == kProlong)
        hipLaunchKernelGGL((k_halfsweep<T, W, JM, kProlong, VW, MK>), dim3(nb), dim3(kBlock), 0, C->stream, a, x, f,
                           colour, theta, nact, ec);
      else
        hipLaunchKernelGGL((k_halfsweep<T, W, JM, kPlain, VW, MK>), dim3(nb), dim3(kBlock), 0, C->stream, a, x, f,
                           colour, theta, nact, ec);
    });
  });
  LAUNCH_CHECK();
  return SMG_OK;
}

// Whether level L's sweeps run as one launch now (descriptor, second buffer,
// and neither node factors nor a domain in the context).
template <typename T>
bool one_launch(const smg_ctx* C, const Level<T>& L, const T* alt) {
  return alt && !C->masked && !C->domain && one_launch_desc(C->desc, L.n);
}

// Rows per segment of the one-launch sweep: as many pair-walking waves as the
// device holds at once (`resident`), so that every segment runs in the first
// and only round (measured at 511x511, N=256: 903 us with 1024 waves of 128
// rows against 920-953 us with two rounds of shorter segments, FP64; FP32 at
// two waves per SIMD is fastest with 2048 waves of 64 rows).
int sweep_rows_for(int n, int requested, int resident) {
  if (requested > 0) return std::min(requested, n);
  const int npair = (n + 1) / 2;
  const int nseg = std::max(1, resident / npair);
  return (n + nseg - 1) / nseg;
}

// Waves of kernel `fn` (kBlock threads per block) the device holds at once.
int resident_waves(const void* fn) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kBlock, 0) != hipSuccess || cus <= 0 || per <= 0)
    return 1024;
  return cus * per * (kBlock / 64);
}

// Samples per access of the one-launch sweep and the black prolongation: FP32
// as the half-sweeps take them (vw); FP64 two samples (one 16-byte access)
// wherever N is even and a lane holds two or more samples.  On 511x511,
// N = 256, 16-byte accesses took the FP64 operator residual from 937 to 742 us.
template <typename T, int JM, typename F>
void sweep_vw_dispatch(int vw, int N, F&& fn) {
  if constexpr (std::is_same<T, double>::value && JM >= 2 && JM % 2 == 0) {
    if (N % 2 == 0) { fn(IC<2>{}); return; }
    fn(IC<1>{});
  } else {
    if constexpr (JM == 4) {
      if (N % 4 == 0) { fn(IC<4>{}); return; }
    }
    if constexpr (JM % 2 == 0) {
      if (vw == 2) { fn(IC<2>{}); return; }
    }
    fn(IC<1>{});
  }
}

// One whole red+black sweep, xin -> xout (must not alias); src: kPlain or
// kZero (xin taken as zero, not read); all = false: only the blacks' y and p
// of xout are written (the rest of xout keeps what it held).
template <typename T>
int sweep_one_launch(smg_ctx* C, const Level<T>& L, const T* xin, T* xout, const T* f, int src, bool all = true) {
  const LevelArgs<T> a = args(L, C->N, C->desc.strip);
  const SweepPtrs<T> P{xin, xout, f};
  const int npair = (L.n + 1) / 2, npg = (npair + kBlock / 64 - 1) / (kBlock / 64);
  bool launched = false;
  lane_dispatch<std::is_same<T, float>::value>(C->desc.precision, C->N, [&](auto Wc, auto Jc, auto Vc) {
    constexpr int W = decltype(Wc)::value, JM = decltype(Jc)::value;
    if constexpr (W == 64 && JM <= 4) {
      sweep_vw_dispatch<T, JM>(halfsweep_vw(decltype(Vc)::value, JM), C->N, [&](auto Vk) {
        constexpr int VW = decltype(Vk)::value;
        auto go = [&](auto kern) {
          static const int resident = resident_waves(reinterpret_cast<const void*>(kern));
          const int rows = sweep_rows_for(L.n, C->desc.sweep_rows, resident);
          const int nb = npg * ((L.n + rows - 1) / rows);
          hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlock), 0, C->stream, a, P, rows);
        };
        if (src == kZero) {
          if (all) go(k_sweep_fused<T, JM, VW, kZero, true>);
          else go(k_sweep_fused<T, JM, VW, kZero, false>);
        } else {
          if (all) go(k_sweep_fused<T, JM, VW, kPlain, true>);
          else go(k_sweep_fused<T, JM, VW, kPlain, false>);
        }
      });
      launched = true;
    }
  });
  if (!launched) {
    C->err = "one-launch sweep: layout without 64 lanes per node";
    return SMG_EINVAL;
  }
  LAUNCH_CHECK();
  return SMG_OK;
}

// x += P ec at the black nodes of level L (Y and P blocks), ahead of a
// one-launch sweep (see k_prolong_black).
template <typename T>
int prolong_black(smg_ctx* C, const Level<T>& L, T* x, const T* ec) {
  bool launched = false;
  lane_dispatch<std::is_same<T, float>::value>(C->desc.precision, C->N, [&](auto Wc, auto Jc, auto Vc) {
    constexpr int W = decltype(Wc)::value, JM = decltype(Jc)::value;
    if constexpr (W == 64 && JM <= 4) {
      const int nblack = L.n * L.n / 2, nb = (nblack + kBlock / 64 - 1) / (kBlock / 64);
      sweep_vw_dispatch<T, JM>(halfsweep_vw(decltype(Vc)::value, JM), C->N, [&](auto Vk) {
        hipLaunchKernelGGL((k_prolong_black<T, JM, decltype(Vk)::value>), dim3(nb), dim3(kBlock), 0, C->stream, L.n,
                           C->N, ec, x);
      });
      launched = true;
    }
  });
  if (!launched) {
    C->err = "black prolongation: layout without 64 lanes per node";
    return SMG_EINVAL;
  }
  LAUNCH_CHECK();
  return SMG_OK;
}

// count >= 1 sweeps of collective Gauss-Seidel on x (level L), the first with
// neighbour source src (kProlong: x + P ec): one launch per sweep between x and
// alt (an even number, ending in x), an odd count starting with one sweep in
// place by half-sweeps; with kProlong and an even count the correction is added
// at the black nodes first (the only old values a sweep reads).  The one-launch
// sweeps write the blacks' y and p only, except the last one when last_all: the
// red values and u of a sweep are read by nothing but a consumer of the whole
// vector.
template <typename T>
int sweeps_one_launch(smg_ctx* C, const Level<T>& L, T* x, T* alt, const T* f, int count, int src,
                      const T* ec, bool last_all) {
  int s = 0;
  if (count & 1) {
    TRY(halfsweep<T>(C, L, x, f, 0, src, ec));
    TRY(halfsweep<T>(C, L, x, f, 1));
    s = 1;
    src = kPlain;
  }
  if (s < count && src == kProlong) {   // the correction at the blacks, then plain sweeps
    TRY(prolong_black<T>(C, L, x, ec));
    src = kPlain;
  }
  for (; s < count; s += 2, src = kPlain) {
    TRY(sweep_one_launch<T>(C, L, x, alt, f, src, false));
    TRY(sweep_one_launch<T>(C, L, alt, x, f, kPlain, last_all && s + 2 >= count));
  }
  return SMG_OK;
}

// xout = xin + theta D^{-1} (f - S xin): one damped collective Jacobi step
// (D the node block diagonal); xin and xout must not alias.
template <typename T>
int jacobi(smg_ctx* C, const Level<T>& L, const T* xin, T* xout, const T* f) {
  const int nn = L.n * L.n;
  const T theta = (T)C->desc.theta;
  const LevelArgs<T> a = args(L, C->N, C->desc.strip);
  if (C->N > 512) {   // many samples: a block of 256 lanes per node (4 or 8 samples per lane), 4x the waves
    auto go = [&](auto Jc) {
      constexpr int JM = decltype(Jc)::value;
      mask_dispatch(C->masked, [&](auto Mc) {
        hipLaunchKernelGGL((k_jacobi<T, kBlock, JM, 1, decltype(Mc)::value>), dim3(nn), dim3(kBlock), 0, C->stream,
                           a, xin, xout, f, theta);
      });
    };
    if (C->N <= 1024) go(IC<4>{}); else go(IC<8>{});
    LAUNCH_CHECK();
    return SMG_OK;
  }
  lane_dispatch<std::is_same<T, float>::value>(C->desc.precision, C->N, [&](auto Wc, auto Jc, auto Vc) {
    constexpr int W = decltype(Wc)::value, JM = decltype(Jc)::value;
    constexpr int VW = halfsweep_vw(decltype(Vc)::value, JM);
    const int per = kBlock / W, nb = (nn + per - 1) / per;
    mask_dispatch(C->masked, [&](auto Mc) {
      hipLaunchKernelGGL((k_jacobi<T, W, JM, VW, decltype(Mc)::value>), dim3(nb), dim3(kBlock), 0, C->stream, a, xin,
                         xout, f, theta);
    });
  });
  LAUNCH_CHECK();
  return SMG_OK;
}

// L.gden = g + sum_j d_j c_j e_j / a_j^2 per node, in the lane layout (and so
// the summation order) of the level's half-sweep.
template <typename T>
int node_den_level(smg_ctx* C, const Level<T>& L) {
  const int nn = L.n * L.n;
  const LevelArgs<T> a = args(L, C->N, C->desc.strip);
  lane_dispatch<std::is_same<T, float>::value>(C->desc.precision, C->N, [&](auto Wc, auto Jc, auto Vc) {
    constexpr int W = decltype(Wc)::value, JM = decltype(Jc)::value;
    constexpr int VW = halfsweep_vw(decltype(Vc)::value, JM);
    const int per = kBlock / W, nb = (nn + per - 1) / per;
    hipLaunchKernelGGL((k_node_den<T, W, JM, VW>), dim3(nb), dim3(kBlock), 0, C->stream, a, L.gden);
  });
  LAUNCH_CHECK();
  return SMG_OK;
}

// Node factor pairs of every level from the finest level's md, me (device
// [n][n], null: 1), coarse levels by injection (full = 0) or full weighting
// (full = 1), FP32 copies for the FP32 cycle; then what depends on them: the
// per-node denominators and the coarsest Schur complement (A_j^{-1} must be in
// place).
int node_terms(smg_ctx* C);

int factors_setup(smg_ctx* C, const double* md, const double* me, int full) {
  const bool f32 = C->desc.precision == SMG_F32;
  const int n0 = C->desc.n;
  hipLaunchKernelGGL(k_node_factors, dim3((n0 * n0 + kBlock - 1) / kBlock), dim3(kBlock), 0, C->stream, n0 * n0,
                     md, me, C->L64[0].mk);
  for (int l = 0; l < C->nlev; ++l) {
    const int nl = C->L64[l].n, nb = (nl * nl + kBlock - 1) / kBlock;
    if (l > 0)
      hipLaunchKernelGGL(k_coarsen_factors, dim3(nb), dim3(kBlock), 0, C->stream, nl, full,
                         (const double*)C->L64[l - 1].mk, C->L64[l].mk);
    if (C->domain)   // nodes outside the domain: (0, -0)
      hipLaunchKernelGGL(k_apply_domain, dim3(nb), dim3(kBlock), 0, C->stream, nl * nl,
                         (const double*)C->L64[l].dom, C->L64[l].mk);
  }
  LAUNCH_CHECK();
  if (f32)
    for (int l = 0; l < C->nlev; ++l)
      TRY((convert<double, float>(C, C->L64[l].mk, C->L32[l].mk, 2 * (size_t)C->L64[l].n * C->L64[l].n)));
  return node_terms(C);
}

// Per-node control denominators of every level and the coarsest Schur
// complement, from the current blocks and node factors.
int node_terms(smg_ctx* C) {
  const bool f32 = C->desc.precision == SMG_F32;
  for (int l = 0; l < C->nlev; ++l) {
    TRY(node_den_level<double>(C, C->L64[l]));
    if (f32) TRY(node_den_level<float>(C, C->L32[l]));
  }
  const Level<double>& Lc = C->L64[C->nlev - 1];
  hipLaunchKernelGGL(k_coarse_schur_terms, dim3(C->N), dim3(kBlock), 0, C->stream, C->m, C->Ainv, Lc.c, Lc.d, Lc.e,
                     (const double*)Lc.mk, C->terms);
  const int nchunks = (C->N + kSchurChunk - 1) / kSchurChunk;
  hipLaunchKernelGGL(k_coarse_schur_chunks, dim3(nchunks), dim3(kBlock), 0, C->stream, C->m, C->N,
                     (const double*)C->terms, C->schur_part);
  hipLaunchKernelGGL(k_coarse_schur_invert, dim3(1), dim3(kBlock), 0, C->stream, C->m, nchunks,
                     (const double*)C->schur_part, Lc.g, C->Sinv);
  LAUNCH_CHECK();
  return SMG_OK;
}

// x (a finest-level FP64 vector) set to zero outside the domain: the kernels
// keep those values at zero and read them as the Dirichlet values of the nodes
// inside, so every solver starts from such an x.
int zero_outside(smg_ctx* C, double* x) {
  if (!C->domain) return SMG_OK;
  const int nn = C->desc.n * C->desc.n;
  const size_t tot = (size_t)nn * (2 * (size_t)C->N + 1);
  hipLaunchKernelGGL(k_zero_outside, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, C->stream, nn,
                     C->N, (const double*)C->L64[0].dom, x);
  LAUNCH_CHECK();
  return SMG_OK;
}

// Kernels with node factors from now on (factors != 1 somewhere): captured
// V-cycles hold the other instantiation, so they are dropped when this changes.
void set_masked(smg_ctx* C, bool masked) {
  if (C->masked == masked) return;
  for (auto& g : C->graphs) (void)hipGraphExecDestroy(g.exec);
  C->graphs.clear();
  C->masked = masked;
}

// out = f - S x (mode 0) or S x (mode 1); when want_norm, C->norms receives
// { ||r||, ||r_Y||, ||r_U||, ||r_P||, ||f|| } (||f|| = 0 in mode 1).
// Blocks of the residual kernel on a level of n x n nodes (one partial sum per block).
int residual_blocks(const smg_ctx* C, int n) {
  int nb = 0;
  lane_dispatch<false>(C->desc.precision, C->N, [&](auto Wc, auto, auto) {
    const int per = kBlock / decltype(Wc)::value;
    nb = (int)(((size_t)n * n + per - 1) / per);
  });
  return nb;
}

// out = f - S x (mode 0) or S x (mode 1); with partials given, also the five
// norms { ||r||, ||r_Y||, ||r_U||, ||r_P||, ||f|| } into norms (device), the
// per-block sums in partials (residual_blocks x 4) and, above kNormStageMin
// blocks, partials2 (kNormStage x 4).
template <typename T, typename TX, typename TO>
int residual_into(smg_ctx* C, const Level<T>& L, const TX* x, const TX* f, TO* out, int mode, double* partials,
                  double* partials2, double* norms) {
  const size_t nn = (size_t)L.n * L.n;
  // column walks (k_residual_walk) on an FP64-face level that streams from HBM
  const bool walk = std::is_same<T, double>::value && !C->masked && !C->domain && one_launch_desc(C->desc, L.n);
  lane_dispatch<std::is_same<T, float>::value>(C->desc.precision, C->N, [&](auto Wc, auto Jc, auto Vc) {
    constexpr int W = decltype(Wc)::value, JM = decltype(Jc)::value, VW = decltype(Vc)::value;
    const int per = kBlock / W;
    int nb = (int)((nn + per - 1) / per);
    bool walked = false;
    if constexpr (std::is_same<T, double>::value && W == 64 && JM <= 4) {
      if (walk) {
        auto go = [&](auto kern) {
          static const int resident = resident_waves(reinterpret_cast<const void*>(kern));
          const int nseg = std::max(1, resident / L.n), seg = (L.n + nseg - 1) / nseg;
          nb = ((L.n + kBlock / 64 - 1) / (kBlock / 64)) * ((L.n + seg - 1) / seg);
          hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlock), 0, C->stream, args(L, C->N, C->desc.strip), x, f, out,
                             mode, partials, seg);
        };
        if (JM % 2 == 0 && C->N % 2 == 0) go(k_residual_walk<TX, TO, JM, (JM % 2 == 0 ? 2 : 1)>);
        else go(k_residual_walk<TX, TO, JM, 1>);
        walked = true;
      }
    }
    if (!walked) mask_dispatch(C->masked, [&](auto Mc) {
      // FP64 faces with an even N of 65..512: two samples per lane and access
      // (16-byte FP64, 8-byte FP32 iterates)
      if constexpr (std::is_same<T, double>::value && W == 64 && VW == 1 && JM >= 2 && JM <= 8) {
        if (C->N % 2 == 0) {
          hipLaunchKernelGGL((k_residual<T, TX, TO, 64, (JM + 1) / 2 * 2, 2, decltype(Mc)::value>), dim3(nb),
                             dim3(kBlock), 0, C->stream, args(L, C->N, C->desc.strip), x, f, out, mode, partials);
          return;
        }
      }
      hipLaunchKernelGGL((k_residual<T, TX, TO, W, JM, VW, decltype(Mc)::value>), dim3(nb), dim3(kBlock), 0,
                         C->stream, args(L, C->N, C->desc.strip), x, f, out, mode, partials);
    });
    if (partials) {
      if (nb > kNormStageMin) {   // two stages: one block alone reads partials at ~50 GB/s
        hipLaunchKernelGGL(k_norms_stage, dim3(kNormStage), dim3(kBlock), 0, C->stream, (const double*)partials, nb,
                           partials2);
        hipLaunchKernelGGL(k_finalize_norms, dim3(1), dim3(1024), 0, C->stream, (const double*)partials2,
                           kNormStage, norms);
      } else {
        hipLaunchKernelGGL(k_finalize_norms, dim3(1), dim3(1024), 0, C->stream, (const double*)partials, nb, norms);
      }
    }
  });
  LAUNCH_CHECK();
  return SMG_OK;
}

template <typename T, typename TX, typename TO>
int residual(smg_ctx* C, const Level<T>& L, const TX* x, const TX* f, TO* out, int mode, bool want_norm) {
  return residual_into<T, TX, TO>(C, L, x, f, out, mode, want_norm ? C->partials : nullptr, C->partials2, C->norms);
}

// x_next = x + d, out = f - S x_next (FP32), norms into C->norms (FP32 refinement).
int residual_add(smg_ctx* C, const double* x, const float* d, double* xn, const double* f, float* out) {
  const Level<double>& L = C->L64[0];
  const size_t nn = (size_t)L.n * L.n;
  // column walks (k_residual_add_walk) on a level that streams from HBM
  const bool walk = !C->masked && !C->domain && one_launch_desc(C->desc, L.n);
  lane_dispatch<false>(C->desc.precision, C->N, [&](auto Wc, auto Jc, auto) {
    constexpr int W = decltype(Wc)::value, JM = decltype(Jc)::value;
    const int per = kBlock / W;
    int nb = (int)((nn + per - 1) / per);
    bool walked = false;
    if constexpr (W == 64 && JM <= 4) {
      if (walk) {
        auto go = [&](auto kern) {
          static const int resident = resident_waves(reinterpret_cast<const void*>(kern));
          const int nseg = std::max(1, resident / L.n), seg = (L.n + nseg - 1) / nseg;
          nb = ((L.n + kBlock / 64 - 1) / (kBlock / 64)) * ((L.n + seg - 1) / seg);
          hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlock), 0, C->stream, args(L, C->N, C->desc.strip), x, d, xn, f,
                             out, C->partials, seg);
        };
        if (JM % 2 == 0 && C->N % 2 == 0) go(k_residual_add_walk<JM, (JM % 2 == 0 ? 2 : 1)>);
        else go(k_residual_add_walk<JM, 1>);
        walked = true;
      }
    }
    if (!walked) mask_dispatch(C->masked, [&](auto Mc) {
      // two samples per access (16-byte FP64, 8-byte FP32) where N is even
      if constexpr (W == 64 && JM % 2 == 0) {
        if (C->N % 2 == 0) {
          hipLaunchKernelGGL((k_residual_add<W, JM, 2, decltype(Mc)::value>), dim3(nb), dim3(kBlock), 0, C->stream,
                             args(L, C->N, C->desc.strip), x, d, xn, f, out, C->partials);
          return;
        }
      }
      hipLaunchKernelGGL((k_residual_add<W, JM, 1, decltype(Mc)::value>), dim3(nb), dim3(kBlock), 0, C->stream,
                         args(L, C->N, C->desc.strip), x, d, xn, f, out, C->partials);
    });
    if (nb > kNormStageMin) {
      hipLaunchKernelGGL(k_norms_stage, dim3(kNormStage), dim3(kBlock), 0, C->stream, C->partials, nb, C->partials2);
      hipLaunchKernelGGL(k_finalize_norms, dim3(1), dim3(1024), 0, C->stream, C->partials2, kNormStage, C->norms);
    } else {
      hipLaunchKernelGGL(k_finalize_norms, dim3(1), dim3(1024), 0, C->stream, C->partials, nb, C->norms);
    }
  });
  LAUNCH_CHECK();
  return SMG_OK;
}

template <typename T>
int restrict_to(smg_ctx* C, int nf, const T* fine, T* coarse) {
  const int nc = (nf - 1) / 2;
  lane_dispatch<std::is_same<T, float>::value>(C->desc.precision, C->N, [&](auto Wc, auto Jc, auto Vc) {
    constexpr int W = decltype(Wc)::value, JM = decltype(Jc)::value, VW = decltype(Vc)::value;
    const int per = kBlock / W, nb = (nc * nc + per - 1) / per;
    hipLaunchKernelGGL((k_restrict<T, W, JM, VW>), dim3(nb), dim3(kBlock), 0, C->stream, nf, C->N, fine, coarse,
                       coarse_strip(strip_for(nf, C->desc.strip)));
  });
  LAUNCH_CHECK();
  return SMG_OK;
}

// coarse = R (f - S x) in one pass (the fine residual is never stored).
// The column-walk form (k_rr_walk) where the level's sweeps run in one launch:
// 64 lanes per node, at most four samples per lane, no node factors or domain.
template <typename T>
bool rr_walk(smg_ctx* C, const Level<T>& L, const T* x, const T* f, T* coarse) {
  if (C->masked || C->domain || !one_launch_desc(C->desc, L.n) || L.n < 3) return false;
  const int nc = (L.n - 1) / 2;
  const LevelArgs<T> a = args(L, C->N, C->desc.strip);
  bool launched = false;
  lane_dispatch<std::is_same<T, float>::value>(C->desc.precision, C->N, [&](auto Wc, auto Jc, auto Vc) {
    constexpr int W = decltype(Wc)::value, JM = decltype(Jc)::value;
    if constexpr (W == 64 && JM <= 4) {
      sweep_vw_dispatch<T, JM>(halfsweep_vw(decltype(Vc)::value, JM), C->N, [&](auto Vk) {
        constexpr int VW = decltype(Vk)::value;
        auto kern = k_rr_walk<T, JM, VW>;
        static const int resident = resident_waves(reinterpret_cast<const void*>(kern));
        const int nseg = std::max(1, resident / nc), seg = (nc + nseg - 1) / nseg;
        const int npg = (nc + kBlock / 64 - 1) / (kBlock / 64);
        const int nb = npg * ((nc + seg - 1) / seg);
        hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlock), 0, C->stream, a, x, f, coarse, seg);
      });
      launched = true;
    }
  });
  return launched;
}

// coarse = R (f - S xnew) where xnew is one Gauss-Seidel sweep of xold (theta =
// 1, same f), from the blacks' change (k_rr_gs_walk) on the levels the column
// walk takes; false elsewhere (the caller then forms the residual from f).
template <typename T>
bool rr_gs_walk(smg_ctx* C, const Level<T>& L, const T* xold, const T* xnew, T* coarse) {
  if (C->desc.theta != 1.0 || C->masked || C->domain || !one_launch_desc(C->desc, L.n) || L.n < 3) return false;
  const int nc = (L.n - 1) / 2;
  const LevelArgs<T> a = args(L, C->N, C->desc.strip);
  bool launched = false;
  lane_dispatch<std::is_same<T, float>::value>(C->desc.precision, C->N, [&](auto Wc, auto Jc, auto Vc) {
    constexpr int W = decltype(Wc)::value, JM = decltype(Jc)::value;
    if constexpr (W == 64 && JM <= 4) {
      sweep_vw_dispatch<T, JM>(halfsweep_vw(decltype(Vc)::value, JM), C->N, [&](auto Vk) {
        constexpr int VW = decltype(Vk)::value;
        auto kern = k_rr_gs_walk<T, JM, VW>;
        static const int resident = resident_waves(reinterpret_cast<const void*>(kern));
        const int nseg = std::max(1, resident / nc), seg = (nc + nseg - 1) / nseg;
        const int npg = (nc + kBlock / 64 - 1) / (kBlock / 64);
        const int nb = npg * ((nc + seg - 1) / seg);
        hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlock), 0, C->stream, a, xold, xnew, coarse, seg);
      });
      launched = true;
    }
  });
  return launched;
}

template <typename T>
int residual_restrict(smg_ctx* C, const Level<T>& L, const T* x, const T* f, T* coarse) {
  const int nc = (L.n - 1) / 2;
  if (rr_walk<T>(C, L, x, f, coarse)) {
    LAUNCH_CHECK();
    return SMG_OK;
  }
  const LevelArgs<T> a = args(L, C->N, C->desc.strip);
  rr_dispatch<std::is_same<T, float>::value>(C->desc.precision, C->N, [&](auto Wc, auto Jc, auto Vc) {
    constexpr int W = decltype(Wc)::value, JM = decltype(Jc)::value, VW = decltype(Vc)::value;
    const int per = kBlock / W, nb = (nc * nc + per - 1) / per;
    mask_dispatch(C->masked, [&](auto Mc) {
      hipLaunchKernelGGL((k_residual_restrict<T, W, JM, VW, decltype(Mc)::value>), dim3(nb), dim3(kBlock), 0,
                         C->stream, a, x, f, coarse, coarse_strip(a.strip));
    });
  });
  LAUNCH_CHECK();
  return SMG_OK;
}

// fine += P coarse; fmk: the fine level's node factors (the U block is
// prolongated into the control space only)
template <typename T>
int prolong_add(smg_ctx* C, int nc, const T* coarse, T* fine, const T* fmk) {
  const int nf = 2 * nc + 1;
  if (C->N > 512) {   // many samples: 256 lanes per fine node (4 or 8 samples per lane), 4x the waves
    auto go = [&](auto Jc) {
      constexpr int JM = decltype(Jc)::value;
      mask_dispatch(C->masked, [&](auto Mc) {
        hipLaunchKernelGGL((k_prolong_add<T, 256, JM, decltype(Mc)::value>), dim3(nf * nf), dim3(kBlock), 0,
                           C->stream, nc, C->N, coarse, fine, fmk);
      });
    };
    if (C->N <= 1024) go(IC<4>{}); else go(IC<8>{});
    LAUNCH_CHECK();
    return SMG_OK;
  }
  lane_dispatch<false>(C->desc.precision, C->N, [&](auto Wc, auto Jc, auto) {
    constexpr int W = decltype(Wc)::value, JM = decltype(Jc)::value;
    const int per = kBlock / W, nb = (nf * nf + per - 1) / per;
    mask_dispatch(C->masked, [&](auto Mc) {
      hipLaunchKernelGGL((k_prolong_add<T, W, JM, decltype(Mc)::value>), dim3(nb), dim3(kBlock), 0, C->stream, nc,
                         C->N, coarse, fine, fmk);
    });
  });
  LAUNCH_CHECK();
  return SMG_OK;
}

// The unfused restriction's control space, as the fused residual-restriction
// has it: U entries of the fine residual r (level F; before restricting) or of
// the restricted coarse vector fc (after) zeroed at nodes without a control.
template <typename T>
int control_rows(smg_ctx* C, const Level<T>& F, T* r, T* fc) {
  if (!C->masked) return SMG_OK;
  const int nf = F.n, nc = (nf - 1) / 2, N = C->N;
  if (r)
    hipLaunchKernelGGL(k_control_rows<T>, dim3((nf * nf + kBlock - 1) / kBlock), dim3(kBlock), 0, C->stream, nf, 1,
                       nf, (const T*)F.mk, r + (size_t)N * nf * nf);
  if (fc)
    hipLaunchKernelGGL(k_control_rows<T>, dim3((nc * nc + kBlock - 1) / kBlock), dim3(kBlock), 0, C->stream, nc, 2,
                       nf, (const T*)F.mk, fc + (size_t)N * nc * nc);
  LAUNCH_CHECK();
  return SMG_OK;
}

template <typename TV>
int coarse_solve(smg_ctx* C, const TV* F, TV* X) {
  const Level<double>& L = C->L64[C->nlev - 1];
  hipLaunchKernelGGL((k_coarse_phase1<TV>), dim3(C->N), dim3(64), 0, C->stream, C->m, C->N, C->Ainv, L.c, L.d,
                     (const double*)L.mk, F, C->ds);
  LAUNCH_CHECK();
  // many samples: u once (k_coarse_u) instead of a sum over all samples in every block
  const bool upre = C->N > kCoarseUMin;
  if (upre) {
    hipLaunchKernelGGL((k_coarse_u<TV>), dim3(1), dim3(64 * kCoarseUSlices), 0, C->stream, C->m, C->N,
                       (const double*)C->Sinv, F, (const double*)C->ds, C->cu);
    LAUNCH_CHECK();
  }
  hipLaunchKernelGGL((k_coarse_phase2<TV>), dim3(C->N), dim3(64), 0, C->stream, C->m, C->N, C->Ainv, C->Sinv,
                     L.c, L.e, (const double*)L.mk, F, C->ds, X, upre ? (const double*)C->cu : nullptr);
  LAUNCH_CHECK();
  return SMG_OK;
}

// count damped collective Jacobi steps on x, alternating between x and the
// scratch t (an odd count ends with a copy back).
template <typename T>
int jacobi_steps(smg_ctx* C, const Level<T>& L, T* x, T* t, const T* f, int count) {
  for (int s = 0; s < count; ++s) TRY(s % 2 == 0 ? jacobi<T>(C, L, x, t, f) : jacobi<T>(C, L, t, x, f));
  if (count % 2) TRY((convert<T, T>(C, t, x, vlen(L.n, C->N))));
  return SMG_OK;
}

// Alg. 1 with the damped collective Jacobi smoother (SMG_FLAG_JACOBI): the
// smoothing steps are out of place through the level-0-sized scratch t, the
// residual is restricted in the pass that forms it (unless unfused), and the
// coarse correction is a separate prolongation pass.
template <typename T>
int vcycle_level_jacobi(smg_ctx* C, Level<T>* Ls, T* t, int l, T* x, const T* f, bool x_zero) {
  if (l == C->nlev - 1) return coarse_solve<T>(C, f, x);
  const Level<T>& L = Ls[l];
  if (x_zero) TRY(fill<T>(C, x, vlen(L.n, C->N), T(0)));
  TRY(jacobi_steps<T>(C, L, x, t, f, C->desc.pre));
  Level<T>& Lc = Ls[l + 1];
  if (!(C->desc.flags & SMG_FLAG_UNFUSED)) {
    TRY(residual_restrict<T>(C, L, x, f, Lc.f));
  } else {
    TRY((residual<T, T, T>(C, L, x, f, t, 0, false)));
    TRY(control_rows<T>(C, L, t, nullptr));
    TRY(restrict_to<T>(C, L.n, t, Lc.f));
    TRY(control_rows<T>(C, L, nullptr, Lc.f));
  }
  TRY(vcycle_level_jacobi<T>(C, Ls, t, l + 1, Lc.x, Lc.f, true));
  TRY(prolong_add<T>(C, Lc.n, Lc.x, x, L.mk));
  return jacobi_steps<T>(C, L, x, t, f, C->desc.post);
}

// Alg. 1 on level l (Levels Ls of type T), x and f of that level; x_zero: x
// holds (or is to be taken as) zero on entry.
//
// With theta = 1 the launch sequence is fused without changing the iteration:
//  - from a zero guess the first red half-sweep reads no neighbours (kZero) and
//    no zero fill is written;
//  - the coarse correction x += P e_c is folded into the first post-smoothing red
//    half-sweep (kProlong): red nodes read their black neighbours corrected on
//    the fly, and the black half-sweep that follows overwrites every black node;
//    on levels swept in one launch per sweep it is added at the black nodes only.
// For any theta the residual is restricted in the same pass that forms it.
template <typename T>
int vcycle_level(smg_ctx* C, Level<T>* Ls, T* r, int l, T* x, const T* f, bool x_zero) {
  if (C->desc.flags & SMG_FLAG_JACOBI) return vcycle_level_jacobi<T>(C, Ls, r, l, x, f, x_zero);
  if (l == C->nlev - 1) return coarse_solve<T>(C, f, x);
  const Level<T>& L = Ls[l];
  const bool fused = C->desc.theta == 1.0 && !(C->desc.flags & SMG_FLAG_UNFUSED);
  T* alt = l == 0 ? r : L.xa;
  if (fused && one_launch<T>(C, L, alt) && C->desc.pre > 0 && C->desc.post > 0) {
    // whole sweeps in one launch each (k_sweep_fused), the same iteration
    // two or more pre-smoothing sweeps end with one from alt into x and the
    // residual is restricted from the blacks' change, which reads no red value
    // and no u: then no pre-smoothing sweep writes them
    const bool gs_rr = C->desc.pre >= 2;
    TRY(sweeps_one_launch<T>(C, L, x, alt, f, C->desc.pre, x_zero ? kZero : kPlain, nullptr, !gs_rr));
    Level<T>& Lc = Ls[l + 1];
    if (gs_rr) {
      if (!rr_gs_walk<T>(C, L, alt, x, Lc.f)) {
        C->err = "restriction after a sweep: layout without 64 lanes per node";
        return SMG_EINVAL;
      }
      LAUNCH_CHECK();
    } else {
      TRY(residual_restrict<T>(C, L, x, f, Lc.f));
    }
    TRY(vcycle_level<T>(C, Ls, r, l + 1, Lc.x, Lc.f, true));
    return sweeps_one_launch<T>(C, L, x, alt, f, C->desc.post, kProlong, Lc.x, true);
  }
  int s0 = 0;
  if (x_zero) {
    if (fused && C->desc.pre > 0) {
      TRY(halfsweep<T>(C, L, x, f, 0, kZero));
      TRY(halfsweep<T>(C, L, x, f, 1));
      s0 = 1;
    } else {
      TRY(fill<T>(C, x, vlen(L.n, C->N), T(0)));
    }
  }
  for (int s = s0; s < C->desc.pre; ++s) {
    TRY(halfsweep<T>(C, L, x, f, 0));
    TRY(halfsweep<T>(C, L, x, f, 1));
  }
  Level<T>& Lc = Ls[l + 1];
  if (!(C->desc.flags & SMG_FLAG_UNFUSED)) {
    TRY(residual_restrict<T>(C, L, x, f, Lc.f));
  } else {
    TRY((residual<T, T, T>(C, L, x, f, r, 0, false)));
    TRY(control_rows<T>(C, L, r, nullptr));
    TRY(restrict_to<T>(C, L.n, r, Lc.f));
    TRY(control_rows<T>(C, L, nullptr, Lc.f));
  }
  TRY(vcycle_level<T>(C, Ls, r, l + 1, Lc.x, Lc.f, true));
  int p0 = 0;
  if (fused && C->desc.post > 0) {
    TRY(halfsweep<T>(C, L, x, f, 0, kProlong, Lc.x));
    TRY(halfsweep<T>(C, L, x, f, 1));
    p0 = 1;
  } else {
    TRY(prolong_add<T>(C, Lc.n, Lc.x, x, L.mk));
  }
  for (int s = p0; s < C->desc.post; ++s) {
    TRY(halfsweep<T>(C, L, x, f, 0));
    TRY(halfsweep<T>(C, L, x, f, 1));
  }
  return SMG_OK;
}

template <typename T>
int cycle_eager(smg_ctx* C, T* x, const T* f, bool zero_first) {
  Level<T>* Ls;
  T* r;
  if constexpr (std::is_same<T, double>::value) { Ls = C->L64; r = C->r64; }
  else { Ls = C->L32; r = C->r32; }
  return vcycle_level<T>(C, Ls, r, 0, x, f, zero_first);
}

constexpr size_t kMaxGraphs = 128;

// One V-cycle on the finest level (x <- Vcycle(x, f), or from zero when
// zero_first).  Unless the context is eager, the launch sequence is captured
// once per (x, f) pair into a hipGraph on a private stream and replayed on the
// caller's stream; graphs hold no memset nodes.
template <typename T>
int run_cycle(smg_ctx* C, T* x, const T* f, bool zero_first) {
  if ((C->desc.flags & SMG_FLAG_EAGER) || !C->cap_stream) return cycle_eager<T>(C, x, f, zero_first);
  const int kind = (std::is_same<T, double>::value ? 0 : 2) + (zero_first ? 1 : 0);
  for (auto& g : C->graphs)
    if (g.x == x && g.f == f && g.kind == kind) {
      HIP_TRY(hipGraphLaunch(g.exec, C->stream));
      return SMG_OK;
    }
  if (C->graphs.size() >= kMaxGraphs) return cycle_eager<T>(C, x, f, zero_first);
  hipStream_t user = C->stream;
  C->stream = C->cap_stream;
  hipError_t e = hipStreamBeginCapture(C->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) { C->stream = user; return hip_fail(C, e, "hipStreamBeginCapture"); }
  const int rc = cycle_eager<T>(C, x, f, zero_first);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(C->cap_stream, &graph);
  C->stream = user;
  if (rc != SMG_OK) { if (graph) (void)hipGraphDestroy(graph); return rc; }
  if (e != hipSuccess) return hip_fail(C, e, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(C, e, "hipGraphInstantiate");
  C->graphs.push_back({x, f, kind, exec});
  HIP_TRY(hipGraphLaunch(exec, C->stream));
  return SMG_OK;
}

int vcycle64(smg_ctx* C, double* x, const double* f) { return run_cycle<double>(C, x, f, false); }
int vcycle32(smg_ctx* C, float* x, const float* f) { return run_cycle<float>(C, x, f, false); }

int sync(smg_ctx* C) {
  HIP_TRY(hipStreamSynchronize(C->stream));
  return SMG_OK;
}

// Bring nv FP64 values from device memory to C->host[0..nv) at the current
// point of the stream: a one-wave kernel stores them into the host-mapped
// staging and then a sequence number into the publish word; the host spins on
// that word (a few microseconds after the kernel, instead of a copy and a
// stream synchronization) and falls back to querying the stream, so an error
// is reported and a completed stream always ends the wait.
int readback(smg_ctx* C, const double* src, int nv) {
  const unsigned seq = ++C->pub_seq;
  hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, C->stream, src, nv, C->host_dev, C->pub_dev, seq);
  LAUNCH_CHECK();
  for (unsigned long it = 1;; ++it) {
    if (__atomic_load_n(C->pub_host, __ATOMIC_ACQUIRE) == seq) return SMG_OK;
    if ((it & 255) == 0) {
      const hipError_t q = hipStreamQuery(C->stream);
      if (q == hipSuccess) {
        if (__atomic_load_n(C->pub_host, __ATOMIC_ACQUIRE) == seq) return SMG_OK;
        C->err = "readback: stream complete without the published values";
        return SMG_EHIP;
      }
      if (q != hipErrorNotReady) return hip_fail(C, q, "hipStreamQuery");
    }
  }
}

// ||v||_2 (one multi-dot pass with no basis vectors).
int vec_norm(smg_ctx* C, const double* v, size_t len, double* out) {
  hipLaunchKernelGGL((k_mdot<double, 4>), dim3(kPartials), dim3(kBlock), 0, C->stream, len, v,
                     (const double*)nullptr, (size_t)0, 0, 1, C->mdp);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_mdot_finalize, dim3(kMaxBasis + 1), dim3(kBlock), 0, C->stream, C->mdp, kPartials, 0, 1, C->hdev, 0);
  LAUNCH_CHECK();
  TRY(readback(C, C->hdev + kMaxBasis, 1));
  *out = std::sqrt(C->host[0]);
  return SMG_OK;
}

// out_j = scale_j sum_i A_j(i) B_j(i) over the finest level's nodes (device, N values).
int sample_dots(smg_ctx* C, const double* A, const double* B, const double* scale, double* out) {
  const int nn = C->desc.n * C->desc.n, N = C->N, nb = std::min(kSampleBlocks, nn);
  hipLaunchKernelGGL(k_sample_dots, dim3(nb), dim3(kBlock), 0, C->stream, nn, N, A, B, C->cpart);
  hipLaunchKernelGGL(k_sample_finalize, dim3((N + kFinalizeSamples - 1) / kFinalizeSamples), dim3(kBlock), 0,
                     C->stream, nb, N,
                     (const double*)C->cpart, scale, out);
  LAUNCH_CHECK();
  return SMG_OK;
}

// out_Y += sign sum_j w_j z_j (z_j . x_Y,j): the rank-one terms of the finest
// level (nothing unless they are set).
int lowrank_add(smg_ctx* C, const double* x, double* out, double sign) {
  if (!C->lr_on) return SMG_OK;
  const int nn = C->desc.n * C->desc.n, N = C->N;
  TRY(sample_dots(C, C->cz, x, C->cwv, C->cs));
  hipLaunchKernelGGL(k_lowrank_add, dim3(grid_for((size_t)nn * N)), dim3(kBlock), 0, C->stream, nn, N, sign,
                     (const double*)C->cs, (const double*)C->cz, out);
  LAUNCH_CHECK();
  return SMG_OK;
}

// FP64 residual of the finest level into out (may be null); norms to host
// h[0..4] = { ||r||, ||r_Y||, ||r_U||, ||r_P||, ||f|| }.  With rank-one terms
// the residual is corrected and its block norms taken again.
int residual_norms64(smg_ctx* C, const double* x, const double* f, double* out, double* h) {
  double* o = out ? out : C->clr;
  TRY((residual<double, double, double>(C, C->L64[0], x, f, C->lr_on ? o : out, 0, true)));
  TRY(readback(C, C->norms, 5));
  for (int i = 0; i < 5; ++i) h[i] = C->host[i];
  if (C->lr_on) {
    const size_t nn = (size_t)C->desc.n * C->desc.n, N = C->N;
    TRY(lowrank_add(C, x, o, -1.0));
    TRY(vec_norm(C, o, N * nn, &h[1]));
    h[0] = std::sqrt(h[1] * h[1] + h[2] * h[2] + h[3] * h[3]);
  }
  return SMG_OK;
}

void stats_begin(smg_stats* st) {
  if (!st) return;
  st->iterations = 0; st->inner_iterations = 0; st->restarts = 0;
  st->relres = st->relres_y = st->relres_u = st->relres_p = NAN;
  st->history_len = 0;
}

void stats_push(smg_stats* st, double v) {
  if (st && st->history && st->history_len < st->history_cap) st->history[st->history_len++] = v;
}

void stats_norms(smg_stats* st, const double* h, double fn) {
  if (!st) return;
  st->relres = h[0] / fn; st->relres_y = h[1] / fn; st->relres_u = h[2] / fn; st->relres_p = h[3] / fn;
}

// Apply the preconditioner to V_k and the operator to the result:
//   Z_k = Vcycle(0, V_k);  w = S Z_k.
int precond_and_apply(smg_ctx* C, int k) {
  const size_t len = C->len0;
  double* vk = C->V + (size_t)k * C->ldk;
  if (C->desc.precision == SMG_F64) {
    double* zk = C->Z64 + (size_t)k * C->ldk;
    TRY(run_cycle<double>(C, zk, vk, true));
    TRY((residual<double, double, double>(C, C->L64[0], zk, (const double*)nullptr, C->w, 1, false)));
    TRY(lowrank_add(C, zk, C->w, 1.0));
  } else {
    float* zk = C->Z32 + (size_t)k * C->ldk;
    TRY((convert<double, float>(C, vk, C->L32[0].f, len)));
    TRY(run_cycle<float>(C, zk, C->L32[0].f, true));
    TRY((residual<double, float, double>(C, C->L64[0], zk, (const float*)nullptr, C->w, 1, false)));
  }
  return SMG_OK;
}

// Least squares min |g0 e_1 - H y| over the first nc columns of the
// (m+1) x m upper Hessenberg H (row-major, row stride m), by Givens rotations
// from scratch.  Returns the residual norm; writes y[0..nc) if y is not null.
double hessenberg_lsq(const std::vector<double>& H, int m, int nc, double g0, double* y) {
  std::vector<double> R(H.begin(), H.begin() + (size_t)(nc + 1) * m), g(nc + 1, 0.0), cs(nc), sn(nc);
  g[0] = g0;
  for (int j = 0; j < nc; ++j) {
    for (int i = 0; i < j; ++i) {
      const double a = R[(size_t)i * m + j], b = R[(size_t)(i + 1) * m + j];
      R[(size_t)i * m + j] = cs[i] * a + sn[i] * b;
      R[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
    }
    const double a = R[(size_t)j * m + j], b = R[(size_t)(j + 1) * m + j];
    const double rr = std::sqrt(a * a + b * b);
    cs[j] = rr > 0.0 ? a / rr : 1.0;
    sn[j] = rr > 0.0 ? b / rr : 0.0;
    R[(size_t)j * m + j] = rr;
    R[(size_t)(j + 1) * m + j] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
  }
  if (y) {
    for (int i = nc - 1; i >= 0; --i) {
      double s = g[i];
      for (int q = i + 1; q < nc; ++q) s -= R[(size_t)i * m + q] * y[q];
      y[i] = s / R[(size_t)i * m + i];
    }
  }
  return std::fabs(g[nc]);
}

// One restart cycle of right-preconditioned (flexible) GMRES.  The Arnoldi
// process is classical Gram-Schmidt applied twice, with the second projection
// of each basis vector delayed to the next step, where it shares one pass over
// the basis with the first projection of the new vector (Hernandez, Roman and
// Tomas 2007; Bielich et al. 2022): per step one V-cycle, one operator apply,
// one pass of dot products, one host synchronization and one update pass that
// writes only the new vector (the second projections and normalizations live in
// the triangular factor T of V' = V T on the host).  The preconditioner sees
// each basis vector before its second projection, which flexible GMRES allows
// (x += Z y with A Z = V' H holds for any Z).  The provisional subdiagonal |w'|
// of a step is replaced by the exact norm after the second projection in the
// next step, and the least-squares problem is re-solved from scratch each step.
// On entry V_0 holds r0 = f - S x itself (norm beta), and r0 = g0 V'_0 with
// g0 = |r0| from the first dots pass.  Iterates until the recurrence residual
// <= target, m steps, or *budget runs out; x += Z y at the end.  Returns its in
// *its_done and the last recurrence residual in *est.
int gmres_cycle(smg_ctx* C, double* x, double beta, int m, double target, int budget, int* its_done,
                double* est, smg_stats* st, double fn) {
  const size_t len = C->len0;
  const int m1 = m + 1;
  std::vector<double> H((size_t)m1 * m, 0.0);
  // Orthonormal basis V' = V T (T upper triangular, T[l * m1 + i] = weight of
  // stored V_l in V'_i); the stored vectors are never rewritten.
  std::vector<double> T((size_t)m1 * m1, 0.0);
  std::vector<double> s(m1), b(m1);
  double g0 = beta, rho = 1.0;   // V_k as stored = (projected vector) / rho
  int k = 0, done = 0;
  double res = beta;
  for (; k < m && done < budget; ++k) {
    TRY(precond_and_apply(C, k));
    const int KMv = km_width(k);
    const int nslots = 2 * KMv + 3;
    km_dispatch(k, [&](auto Kc) {
      constexpr int KM = decltype(Kc)::value;
      hipLaunchKernelGGL((k_arnoldi_dots<KM>), dim3(kPartials), dim3(kBlock), 0, C->stream, len,
                         (const double*)C->V, C->ldk, k, (const double*)C->w, C->mdp);
    });
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_partials_finalize, dim3(nslots), dim3(kBlock), 0, C->stream, (const double*)C->mdp,
                       kPartials, kArnSlots, C->hdev);
    LAUNCH_CHECK();
    TRY(readback(C, C->hdev, nslots));
    const double* R = C->host;          // stored V_l . V_k
    const double* B = C->host + KMv;    // stored V_l . w
    const double c = C->host[2 * KMv], d = C->host[2 * KMv + 1], e = C->host[2 * KMv + 2];
    // projections on the orthonormal basis: s = T^T R, b = T^T B
    double ss = 0.0, sb = 0.0, bb = 0.0;
    for (int i = 0; i < k; ++i) {
      double si = 0.0, bi = 0.0;
      for (int l = 0; l <= i; ++l) {
        si += T[(size_t)l * m1 + i] * R[l];
        bi += T[(size_t)l * m1 + i] * B[l];
      }
      s[i] = si; b[i] = bi;
      ss += si * si;
      sb += si * bi;
      bb += bi * bi;
    }
    const double a2 = c - ss;
    if (!std::isfinite(a2) || !std::isfinite(d) || !std::isfinite(e)) {
      C->err = "non-finite Arnoldi coefficients";
      return SMG_ENONFINITE;
    }
    if (!(a2 > 0.0)) {
      // V_k lies in the span of V_{<k}: the Krylov space is invariant and the
      // previous step's solution is exact.
      if (k > 0) H[(size_t)k * m + k - 1] = 0.0;
      break;
    }
    const double alpha = std::sqrt(a2);
    // V'_k = (V_k - sum_{i<k} s_i V'_i) / alpha
    for (int l = 0; l <= k; ++l) {
      double t = l == k ? 1.0 : 0.0;
      for (int i = l; i < k; ++i) t -= s[i] * T[(size_t)l * m1 + i];
      T[(size_t)l * m1 + k] = t / alpha;
    }
    if (k == 0) {
      g0 = alpha;
    } else {
      for (int i = 0; i < k; ++i) H[(size_t)i * m + k - 1] += rho * s[i];
      H[(size_t)k * m + k - 1] = rho * alpha;
    }
    const double hkk = (d - sb) / alpha;
    for (int i = 0; i < k; ++i) H[(size_t)i * m + k] = b[i];
    H[(size_t)k * m + k] = hkk;
    // w' = w - sum_{i<k} b_i V'_i - hkk V'_k = w - sum_{l<=k} g_l V_l
    ArnCoef cf;
    for (int l = 0; l < kMaxBasis; ++l) {
      double g = 0.0;
      if (l <= k) {
        for (int i = l; i < k; ++i) g += T[(size_t)l * m1 + i] * b[i];
        g += T[(size_t)l * m1 + k] * hkk;
      }
      cf.g[l] = g;
    }
    // |w'|^2 from the dots; trusted unless cancellation takes more than four digits
    const double wn2 = e - bb - hkk * hkk;
    const bool estimated = wn2 > 1e-4 * e;
    double hn;
    bool updated = false;
    if (estimated) {
      hn = std::sqrt(wn2);
    } else {
      cf.inv_rho = 1.0;
      km_dispatch(k + 1, [&](auto Kc) {
        constexpr int KM = decltype(Kc)::value;
        hipLaunchKernelGGL((k_arnoldi_update<KM>), dim3(kPartials), dim3(kBlock), 0, C->stream, len, C->V, C->ldk,
                           k, (const double*)C->w, cf, C->mdp);
      });
      LAUNCH_CHECK();
      hipLaunchKernelGGL(k_partials_finalize, dim3(1), dim3(kBlock), 0, C->stream, (const double*)C->mdp, kPartials,
                         1, C->hdev);
      LAUNCH_CHECK();
      TRY(readback(C, C->hdev, 1));
      hn = std::sqrt(std::max(C->host[0], 0.0));
      updated = true;
    }
    if (!std::isfinite(hn) || !std::isfinite(hkk)) {
      C->err = "non-finite Arnoldi coefficients";
      return SMG_ENONFINITE;
    }
    H[(size_t)(k + 1) * m + k] = hn;
    res = hessenberg_lsq(H, m, k + 1, g0, nullptr);
    ++done;
    stats_push(st, res / fn);
    if (res <= target || hn == 0.0 || k + 1 == m || done == budget) { ++k; break; }
    if (!updated) {
      cf.inv_rho = 1.0 / hn;
      km_dispatch(k + 1, [&](auto Kc) {
        constexpr int KM = decltype(Kc)::value;
        hipLaunchKernelGGL((k_arnoldi_update<KM>), dim3(grid_for(len)), dim3(kBlock), 0, C->stream, len, C->V,
                           C->ldk, k, (const double*)C->w, cf, (double*)nullptr);
      });
      LAUNCH_CHECK();
      rho = hn;
    } else {
      rho = 1.0;
    }
  }
  const int kend = k;
  if (kend > 0) {
    BasisCoef y;
    for (int i = 0; i < kMaxBasis; ++i) y.y[i] = 0.0;
    hessenberg_lsq(H, m, kend, g0, y.y);
    km_dispatch(kend, [&](auto Kc) {
      constexpr int KM = decltype(Kc)::value;
      if (C->desc.precision == SMG_F64)
        hipLaunchKernelGGL((k_basis_axpy<double, KM>), dim3(grid_for(len)), dim3(kBlock), 0, C->stream, len, x,
                           (const double*)C->Z64, C->ldk, kend, y);
      else
        hipLaunchKernelGGL((k_basis_axpy<float, KM>), dim3(grid_for(len)), dim3(kBlock), 0, C->stream, len, x,
                           (const float*)C->Z32, C->ldk, kend, y);
    });
    LAUNCH_CHECK();
  }
  *its_done = done;
  *est = res;
  return SMG_OK;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int check_level(const smg_ctx* C, int level, int need_coarser) {
  if (level < 0 || level >= C->nlev) return SMG_EINVAL;
  if (need_coarser && level + 1 >= C->nlev) return SMG_EINVAL;
  return SMG_OK;
}

}  // namespace

// ============================================================ batched solves
// Many independent instances advance together: one refinement step of every
// unretired instance (FP64 outer residual, convergence check, one correction
// V-cycle from zero, x += correction) is a fixed list of batched launches,
// each covering one phase for all instances at the same hierarchy depth, and
// the whole step is captured once into a hipGraph.
// One group of instances advanced in lockstep (the whole batch is split into
// groups of equal grid size, each on its own stream).
struct BatchGroup {
  std::vector<smg_ctx*> ctx;
  std::vector<double*> xs;   // the instances' iterates (solutions out)
  int count = 0, precision = SMG_F64, jm = 1;
  int vw = 1;                // samples per access of the correction kernels (2: FP32, every N even)
  hipStream_t stream = nullptr, cap_stream = nullptr;
  std::string err;
  std::vector<int> lanes;
  std::vector<double> fnorm;
  struct Phase {
    int kind, colour, src;
    size_t off;       // byte offset of the task table in the workspace
    int ntasks, nblocks;
  };
  std::vector<Phase> phases;
  char* base = nullptr;      // workspace
  int* done = nullptr;
  int* iters = nullptr;
  double* relres = nullptr;
  long long* tdone = nullptr;
  long long* t0 = nullptr;
  double* partials = nullptr;
  BCheck* chk = nullptr;
  hipGraphExec_t graph = nullptr;   // one refinement step, for (cap_tol, cap_maxit)
  double cap_tol = -1.0;
  int cap_maxit = -1;
  void* host = nullptr;      // pinned staging
  size_t bytes = 0;
};

namespace {

enum BPhaseKind { kbOuter, kbCheck, kbSweep, kbResRestrict, kbCoarse1, kbCoarse2, kbAdd };

// Lanes per node of an instance by default (the single-instance widths).
int default_lanes(int N, int precision) {
  const int M = vec2_ctx(precision, N) ? N / 2 : N;
  int W = 1;
  while (W < M && W < 64) W <<= 1;
  return W;
}

// Samples per lane of an instance with W lanes and vw samples per access.
int samples_per_lane(int N, int W, int vw) { return vw * ((N + vw * W - 1) / (vw * W)); }

int pow2_ok(int W) { return W >= 1 && W <= 64 && (W & (W - 1)) == 0; }

// Layout of the batch workspace: every task table and the per-instance state.
// With base == null only sizes are computed.  T is the correction arithmetic.
template <typename T>
size_t batch_build(BatchGroup* B, double* const* x, const double* const* f, std::vector<char>* blob) {
  const int cnt = B->count;
  Level<T>* (*levels)(smg_ctx*) = [](smg_ctx* C) -> Level<T>* {
    if constexpr (std::is_same<T, double>::value) return C->L64; else return C->L32;
  };
  auto x0 = [](smg_ctx* C) -> T* {
    if constexpr (std::is_same<T, double>::value) return C->w; else return C->L32[0].x;
  };
  auto f0 = [](smg_ctx* C) -> T* {
    if constexpr (std::is_same<T, double>::value) return C->rr; else return C->L32[0].f;
  };
  // level d of instance i (d = 0 is the finest): x, f, operator
  auto lvl_x = [&](int i, int d) -> T* { return d == 0 ? x0(B->ctx[i]) : levels(B->ctx[i])[d].x; };
  auto lvl_f = [&](int i, int d) -> T* { return d == 0 ? f0(B->ctx[i]) : levels(B->ctx[i])[d].f; };
  auto lvl_args = [&](int i, int d) -> LevelArgs<T> {
    return args(levels(B->ctx[i])[d], B->ctx[i]->N, B->ctx[i]->desc.strip);
  };
  int maxD = 0;
  for (int i = 0; i < cnt; ++i) maxD = std::max(maxD, B->ctx[i]->nlev);
  B->phases.clear();
  blob->clear();
  auto align = [&]() { while (blob->size() % 256) blob->push_back(0); };
  auto add_phase = [&](int kind, int colour, int src, const void* tasks, size_t tbytes, int ntasks, int nblocks) {
    align();
    BatchGroup::Phase p{kind, colour, src, blob->size(), ntasks, nblocks};
    const char* c = (const char*)tasks;
    blob->insert(blob->end(), c, c + tbytes);
    B->phases.push_back(p);
  };
  auto groups = [&](int i, int items) {
    const int per = kBlock / B->lanes[i];
    return (items + per - 1) / per;
  };
  // --- outer FP64 residual into the correction right-hand side, with norm partials
  std::vector<BOuterTask<T>> outer;
  std::vector<BCheck> chk(cnt);
  int nb = 0;
  for (int i = 0; i < cnt; ++i) {
    smg_ctx* C = B->ctx[i];
    const int n = C->L64[0].n;
    BOuterTask<T> t{};
    t.inst = i; t.W = B->lanes[i]; t.nitems = n * n; t.block0 = nb;
    t.L = args(C->L64[0], C->N, C->desc.strip); t.x = x ? x[i] : nullptr; t.f = f ? f[i] : nullptr;
    t.out = f0(C);
    if constexpr (std::is_same<T, float>::value) { t.w = C->w; t.d = x0(C); }   // fused update
    else { t.w = nullptr; t.d = nullptr; }
    const int blocks = groups(i, n * n);
    chk[i].pb0 = nb; chk[i].pnb = blocks; chk[i].fnorm = 1.0;
    nb += blocks;
    outer.push_back(t);
  }
  const int outer_blocks = nb;
  add_phase(kbOuter, 0, 0, outer.data(), sizeof(BOuterTask<T>) * outer.size(), cnt, nb);
  add_phase(kbCheck, 0, 0, nullptr, 0, cnt, cnt);
  // --- correction V-cycle from zero, in lockstep by depth
  auto sweep_phase = [&](int d, int colour, int src, bool down) {
    std::vector<BTask<T>> ts;
    int blocks = 0;
    for (int i = 0; i < cnt; ++i) {
      if (d >= B->ctx[i]->nlev - 1) continue;
      BTask<T> t{};
      t.inst = i; t.W = B->lanes[i]; t.L = lvl_args(i, d);
      t.nitems = colour_count(t.L.n, colour); t.block0 = blocks;
      t.x = lvl_x(i, d); t.f = lvl_f(i, d);
      t.b = src == kProlong ? lvl_x(i, d + 1) : nullptr;
      blocks += groups(i, t.nitems);
      ts.push_back(t);
    }
    (void)down;
    if (!ts.empty()) add_phase(kbSweep, colour, src, ts.data(), sizeof(BTask<T>) * ts.size(), (int)ts.size(), blocks);
  };
  for (int d = 0; d + 1 < maxD; ++d) {
    const int pre = B->ctx[0]->desc.pre;
    sweep_phase(d, 0, kZero, true);
    sweep_phase(d, 1, kPlain, true);
    for (int s = 1; s < pre; ++s) { sweep_phase(d, 0, kPlain, true); sweep_phase(d, 1, kPlain, true); }
    std::vector<BTask<T>> rr;
    int brr = 0;
    for (int i = 0; i < cnt; ++i) {
      if (d >= B->ctx[i]->nlev - 1) continue;
      BTask<T> t{};
      t.inst = i; t.W = B->lanes[i]; t.L = lvl_args(i, d);
      t.x = lvl_x(i, d); t.f = lvl_f(i, d); t.a = lvl_f(i, d + 1);
      const int nc = (t.L.n - 1) / 2;
      t.nitems = nc * nc; t.block0 = brr;
      brr += groups(i, t.nitems);
      rr.push_back(t);
    }
    if (!rr.empty()) add_phase(kbResRestrict, 0, 0, rr.data(), sizeof(BTask<T>) * rr.size(), (int)rr.size(), brr);
  }
  {
    std::vector<BTask<T>> cs;
    int blocks = 0;
    for (int i = 0; i < cnt; ++i) {
      smg_ctx* C = B->ctx[i];
      const int d = C->nlev - 1;
      BTask<T> t{};
      t.inst = i; t.W = B->lanes[i]; t.L = lvl_args(i, d);
      t.x = lvl_x(i, d); t.f = lvl_f(i, d);
      t.m = C->m; t.Ainv = C->Ainv; t.Sinv = C->Sinv; t.ds = C->ds;
      t.c64 = C->L64[d].c; t.d64 = C->L64[d].d; t.e64 = C->L64[d].e; t.mk64 = C->L64[d].mk;
      t.nitems = C->N; t.block0 = blocks;
      blocks += C->N;
      cs.push_back(t);
    }
    add_phase(kbCoarse1, 0, 0, cs.data(), sizeof(BTask<T>) * cs.size(), cnt, blocks);
    add_phase(kbCoarse2, 0, 0, cs.data(), sizeof(BTask<T>) * cs.size(), cnt, blocks);
  }
  for (int d = maxD - 2; d >= 0; --d) {
    const int post = B->ctx[0]->desc.post;
    sweep_phase(d, 0, kProlong, false);
    sweep_phase(d, 1, kPlain, false);
    for (int s = 1; s < post; ++s) { sweep_phase(d, 0, kPlain, false); sweep_phase(d, 1, kPlain, false); }
  }
  if constexpr (std::is_same<T, double>::value) {   // FP32 corrections are added by the next outer pass
    std::vector<BAddTask<T>> as;
    int blocks = 0;
    for (int i = 0; i < cnt; ++i) {
      smg_ctx* C = B->ctx[i];
      BAddTask<T> t{};
      t.inst = i; t.block0 = blocks; t.len = C->len0; t.x = x ? x[i] : nullptr; t.d = x0(C);
      t.nblk = (int)std::min<size_t>((C->len0 + kBlock - 1) / kBlock, 1024);
      blocks += t.nblk;
      as.push_back(t);
    }
    add_phase(kbAdd, 0, 0, as.data(), sizeof(BAddTask<T>) * as.size(), cnt, blocks);
  }
  // per-instance state after the tables
  align();
  const size_t st = blob->size();
  size_t off = st;
  auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) & ~(size_t)255; return o; };
  const size_t o_done = take(sizeof(int) * cnt), o_iters = take(sizeof(int) * cnt);
  const size_t o_rel = take(sizeof(double) * cnt), o_td = take(sizeof(long long) * cnt);
  const size_t o_t0 = take(sizeof(long long)), o_chk = take(sizeof(BCheck) * cnt);
  // partials sized for the smallest lane width (most blocks)
  size_t maxpb = 0;
  for (int i = 0; i < cnt; ++i) maxpb += ((size_t)B->ctx[i]->L64[0].n * B->ctx[i]->L64[0].n + 3) / 4 + 1;
  const size_t o_part = take(sizeof(double) * 3 * std::max<size_t>(maxpb, (size_t)outer_blocks));
  if (B->base) {
    B->done = (int*)(B->base + o_done); B->iters = (int*)(B->base + o_iters);
    B->relres = (double*)(B->base + o_rel); B->tdone = (long long*)(B->base + o_td);
    B->t0 = (long long*)(B->base + o_t0); B->chk = (BCheck*)(B->base + o_chk);
    B->partials = (double*)(B->base + o_part);
    for (int i = 0; i < cnt; ++i) chk[i].fnorm = B->fnorm[i];
    // the check table travels with the blob
    blob->resize(off, 0);
    memcpy(blob->data() + o_chk, chk.data(), sizeof(BCheck) * cnt);
  }
  return off + 256;
}

template <typename F>
void jm_dispatch(int jm, F&& fn) {
  if (jm <= 1) fn(IC<1>{});
  else if (jm <= 2) fn(IC<2>{});
  else if (jm <= 4) fn(IC<4>{});
  else fn(IC<8>{});
}

// (JM, VW) of the batched correction kernels in arithmetic T (two samples per
// access only for FP32, JM then even).
template <typename T, typename F>
void jmv_dispatch(int jm, int vw, F&& fn) {
  if constexpr (std::is_same<T, float>::value) {
    if (vw == 2) {
      if (jm <= 2) fn(IC<2>{}, IC<2>{});
      else if (jm <= 4) fn(IC<4>{}, IC<2>{});
      else fn(IC<8>{}, IC<2>{});
      return;
    }
  }
  jm_dispatch(jm, [&](auto Jc) { fn(Jc, IC<1>{}); });
}

#define BHIP(call)                                                           \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) {                                                  \
      B->err = std::string(#call) + ": " + hipGetErrorString(e_);            \
      return SMG_EHIP;                                                       \
    }                                                                        \
  } while (0)

template <typename T>
int batch_launch_step(BatchGroup* B, hipStream_t s, double tol, int maxit) {
  for (const auto& p : B->phases) {
    const void* tasks = B->base + p.off;
    const int nt = p.ntasks, nbk = p.nblocks;
    switch (p.kind) {
      case kbOuter:
        jm_dispatch(B->jm, [&](auto Jc) {
          constexpr int JM = decltype(Jc)::value;
          auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(nbk), dim3(kBlock), 0, s, (const BOuterTask<T>*)tasks, nt,
                               (const int*)B->done, (const int*)B->iters, B->partials);
          };
          if constexpr (JM % 2 == 0) {
            if (B->vw == 2) { go(kb_outer_residual<T, JM, 2>); return; }   // two samples per access
          }
          go(kb_outer_residual<T, JM, 1>);
        });
        break;
      case kbCheck:
        hipLaunchKernelGGL(kb_check, dim3(B->count), dim3(kBlock), 0, s, (const BCheck*)B->chk,
                           (const double*)B->partials, tol, maxit, B->done, B->iters, B->relres, B->tdone);
        break;
      case kbSweep:
        jmv_dispatch<T>(B->jm, B->vw, [&](auto Jc, auto Vc) {
          constexpr int JM = decltype(Jc)::value, VW = halfsweep_vw(decltype(Vc)::value, JM);
          if (p.src == kZero)
            hipLaunchKernelGGL((kb_halfsweep<T, JM, kZero, VW>), dim3(nbk), dim3(kBlock), 0, s,
                               (const BTask<T>*)tasks, nt, p.colour, (const int*)B->done);
          else if (p.src == kProlong)
            hipLaunchKernelGGL((kb_halfsweep<T, JM, kProlong, VW>), dim3(nbk), dim3(kBlock), 0, s,
                               (const BTask<T>*)tasks, nt, p.colour, (const int*)B->done);
          else
            hipLaunchKernelGGL((kb_halfsweep<T, JM, kPlain, VW>), dim3(nbk), dim3(kBlock), 0, s,
                               (const BTask<T>*)tasks, nt, p.colour, (const int*)B->done);
        });
        break;
      case kbResRestrict:
        jmv_dispatch<T>(B->jm, B->vw, [&](auto Jc, auto Vc) {
          constexpr int JM = decltype(Jc)::value, VW = decltype(Vc)::value;
          hipLaunchKernelGGL((kb_residual_restrict<T, JM, VW>), dim3(nbk), dim3(kBlock), 0, s,
                             (const BTask<T>*)tasks, nt, (const int*)B->done);
        });
        break;
      case kbCoarse1:
        hipLaunchKernelGGL((kb_coarse1<T>), dim3(nbk), dim3(64), 0, s, (const BTask<T>*)tasks, nt,
                           (const int*)B->done);
        break;
      case kbCoarse2:
        hipLaunchKernelGGL((kb_coarse2<T>), dim3(nbk), dim3(64), 0, s, (const BTask<T>*)tasks, nt,
                           (const int*)B->done);
        break;
      case kbAdd:
        hipLaunchKernelGGL((kb_add<T>), dim3(nbk), dim3(kBlock), 0, s, (const BAddTask<T>*)tasks, nt,
                           (const int*)B->done);
        break;
    }
    BHIP(hipGetLastError());
  }
  return SMG_OK;
}

int batch_step(BatchGroup* B, double tol, int maxit) {
  if (B->precision == SMG_F32) return batch_launch_step<float>(B, B->stream, tol, maxit);
  return batch_launch_step<double>(B, B->stream, tol, maxit);
}

}  // namespace

// =================================================================== C ABI
extern "C" {

size_t smg_workspace_bytes(const smg_desc* desc) {
  if (!desc) return 0;
  const smg_desc d = normalized(*desc);
  if (!desc_valid(d, nullptr)) return 0;
  smg_ctx tmp;
  return plan(d, &tmp, nullptr);
}

const char* smg_strerror(int code) {
  switch (code) {
    case SMG_OK: return "ok";
    case SMG_NOT_CONVERGED: return "not converged within the iteration limit";
    case SMG_EINVAL: return "invalid argument";
    case SMG_ESINGULAR: return "singular or non-positive block";
    case SMG_EHIP: return "HIP runtime error";
    case SMG_ENONFINITE: return "non-finite residual";
    case SMG_EWORKSPACE: return "workspace missing or too small";
    default: return "unknown error";
  }
}

const char* smg_last_error(const smg_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }
int smg_num_levels(const smg_ctx* ctx) { return ctx ? ctx->nlev : 0; }
int smg_level_n(const smg_ctx* ctx, int level) {
  return (ctx && level >= 0 && level < ctx->nlev) ? ctx->L64[level].n : 0;
}

void smg_destroy(smg_ctx* ctx) {
  if (!ctx) return;
  for (auto& g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
  ctx->graphs.clear();
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->host) (void)hipHostFree(ctx->host);
  delete ctx;
}

int smg_setup(const smg_desc* desc_in, const smg_blocks* B, void* workspace, size_t workspace_bytes,
              void* stream, smg_ctx** out) {
  if (!out) return SMG_EINVAL;
  *out = nullptr;
  if (!desc_in || !B || !B->kx || !B->ky || !B->c || !B->d || !B->e) return SMG_EINVAL;
  const smg_desc d = normalized(*desc_in);
  std::string why;
  if (!desc_valid(d, &why)) return SMG_EINVAL;
  const int N = d.nsamples;
  // node denominators g + sum_j d_j c_j e_j / a_j^2 stay positive for every a_j > 0
  if (!(B->g > 0.0) || !std::isfinite(B->g)) return SMG_ESINGULAR;
  if (B->control_growth != 0.0 && !(B->control_growth > 0.0 && B->control_growth <= 16.0)) return SMG_EINVAL;
  for (int j = 0; j < N; ++j) {
    if (!(B->c[j] > 0.0) || !std::isfinite(B->c[j]) || !std::isfinite(B->d[j]) || !std::isfinite(B->e[j]))
      return SMG_ESINGULAR;
    if (B->d[j] * B->c[j] * B->e[j] < 0.0) return SMG_ESINGULAR;
  }
  if (B->ctrl)
    for (size_t i = 0; i < (size_t)d.n * d.n; ++i)
      if (!(B->ctrl[i] >= 0.0 && B->ctrl[i] <= 1.0)) return SMG_EINVAL;
  if (B->domain)
    for (size_t i = 0; i < (size_t)d.n * d.n; ++i)
      if (!(B->domain[i] == 0.0 || B->domain[i] == 1.0)) return SMG_EINVAL;
  smg_ctx* C = new smg_ctx();
  C->desc = d;
  C->N = N;
  C->nlev = count_levels(d.n, d.coarsest_n);
  C->stream = (hipStream_t)stream;
  if (hipGetDevice(&C->device) != hipSuccess) C->device = 0;
  const size_t need = plan(d, C, workspace);
  if (!workspace || workspace_bytes < need || ((uintptr_t)workspace & 255) != 0) {
    delete C;
    return SMG_EWORKSPACE;
  }
  C->used_bytes = need;
  auto fail = [&](int rc) { smg_destroy(C); return rc; };
  {
    const size_t nd = 4 * (kMaxBasis + 1);
    if (hipHostMalloc((void**)&C->host, sizeof(double) * nd + 256, hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer((void**)&C->host_dev, C->host, 0) != hipSuccess)
      return fail(SMG_EHIP);
    C->pub_host = (unsigned*)(C->host + nd);
    C->pub_dev = (unsigned*)(C->host_dev + nd);
    *C->pub_host = 0;
  }
  if (!(d.flags & SMG_FLAG_EAGER) &&
      hipStreamCreateWithFlags(&C->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return fail(SMG_EHIP);
  // level 0 references the caller's faces; coarse faces by rediscretization
  C->L64[0].kx = const_cast<double*>(B->kx);
  C->L64[0].ky = const_cast<double*>(B->ky);
  std::vector<double> cc(B->c, B->c + N), dd(B->d, B->d + N), ee(B->e, B->e + N);
  double g = B->g;
  const double growth = B->control_growth == 0.0 ? 4.0 : B->control_growth;
  std::vector<float> cf(N), df(N), ef(N);
  for (int l = 0; l < C->nlev; ++l) {
    Level<double>& L = C->L64[l];
    L.g = g;
    if (hipMemcpy(L.c, cc.data(), sizeof(double) * N, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(L.d, dd.data(), sizeof(double) * N, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(L.e, ee.data(), sizeof(double) * N, hipMemcpyHostToDevice) != hipSuccess)
      return fail(SMG_EHIP);
    if (d.precision == SMG_F32) {
      Level<float>& M = C->L32[l];
      M.g = (float)g;
      for (int j = 0; j < N; ++j) { cf[j] = (float)cc[j]; df[j] = (float)dd[j]; ef[j] = (float)ee[j]; }
      if (hipMemcpy(M.c, cf.data(), sizeof(float) * N, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(M.d, df.data(), sizeof(float) * N, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(M.e, ef.data(), sizeof(float) * N, hipMemcpyHostToDevice) != hipSuccess)
        return fail(SMG_EHIP);
    }
    // the state mass carries h^2 (x4 per coarsening); the control blocks grow by
    // control_growth (x4 too for an area control, x2 for a control on a line)
    for (int j = 0; j < N; ++j) { cc[j] *= 4.0; dd[j] *= growth; ee[j] *= growth; }
    g *= growth;
  }
  const size_t fx0 = (size_t)d.n * (d.n + 1) * N;
  if (hipMemsetAsync(C->flag, 0, sizeof(int), C->stream) != hipSuccess) return fail(SMG_EHIP);
  hipLaunchKernelGGL(k_check_faces, dim3(grid_for(fx0)), dim3(kBlock), 0, C->stream, fx0, B->kx, B->ky, C->flag);
  if (hipGetLastError() != hipSuccess) return fail(SMG_EHIP);
  for (int l = 1; l < C->nlev; ++l) {
    const Level<double>& F = C->L64[l - 1];
    Level<double>& L = C->L64[l];
    const size_t tot = (size_t)L.n * (L.n + 1) * N;
    hipLaunchKernelGGL((k_coarsen_faces<double>), dim3(grid_for(tot)), dim3(kBlock), 0, C->stream, F.n, N, F.kx,
                       F.ky, L.kx, L.ky);
    if (hipGetLastError() != hipSuccess) return fail(SMG_EHIP);
  }
  if (d.precision == SMG_F32) {
    for (int l = 0; l < C->nlev; ++l) {
      const size_t fx = (size_t)C->L64[l].n * (C->L64[l].n + 1) * N;
      if (convert<double, float>(C, C->L64[l].kx, C->L32[l].kx, fx) != SMG_OK ||
          convert<double, float>(C, C->L64[l].ky, C->L32[l].ky, fx) != SMG_OK)
        return fail(SMG_EHIP);
    }
  }
  // domain on every level (the caller's on the finest, coarse levels by injection)
  C->domain = B->domain != nullptr;
  if (C->domain) {
    if (hipMemcpyAsync(C->L64[0].dom, B->domain, sizeof(double) * d.n * d.n, hipMemcpyHostToDevice, C->stream) !=
        hipSuccess)
      return fail(SMG_EHIP);
    for (int l = 1; l < C->nlev; ++l) {
      const int nl = C->L64[l].n;
      hipLaunchKernelGGL(k_inject_domain, dim3((nl * nl + kBlock - 1) / kBlock), dim3(kBlock), 0, C->stream, nl,
                         (const double*)C->L64[l - 1].dom, C->L64[l].dom);
    }
    if (hipGetLastError() != hipSuccess) return fail(SMG_EHIP);
  }
  // coarsest factorization (FP64): A_j^{-1}
  const Level<double>& Lc = C->L64[C->nlev - 1];
  hipLaunchKernelGGL(k_coarse_invert_A, dim3(N), dim3(kBlock), 0, C->stream, Lc.n, N, Lc.kx, Lc.ky,
                     C->domain ? (const double*)Lc.dom : (const double*)nullptr, C->Ainv);
  if (hipGetLastError() != hipSuccess) return fail(SMG_EHIP);
  // control mask (local control): the caller's, as both node factors (staged
  // through the scratch vector rr); all ones without one
  {
    const double* mk = nullptr;
    C->masked = C->domain;
    if (B->ctrl) {
      for (size_t i = 0; i < (size_t)d.n * d.n; ++i) C->masked |= (B->ctrl[i] != 1.0);
      if (hipMemcpyAsync(C->rr, B->ctrl, sizeof(double) * d.n * d.n, hipMemcpyHostToDevice, C->stream) != hipSuccess)
        return fail(SMG_EHIP);
      mk = C->rr;
    }
    if (factors_setup(C, mk, mk, SMG_COARSEN_INJECT) != SMG_OK) return fail(SMG_EHIP);
  }
  int flag = 0;
  if (hipMemcpyAsync(&flag, C->flag, sizeof(int), hipMemcpyDeviceToHost, C->stream) != hipSuccess) return fail(SMG_EHIP);
  if (hipStreamSynchronize(C->stream) != hipSuccess) return fail(SMG_EHIP);
  if (flag) return fail(SMG_ESINGULAR);
  *out = C;
  return SMG_OK;
}

int smg_set_node_factors(smg_ctx* C, const double* md, const double* me, int coarsening) {
  if (!C || (coarsening != SMG_COARSEN_INJECT && coarsening != SMG_COARSEN_FULL)) return SMG_EINVAL;
  const size_t nn = (size_t)C->desc.n * C->desc.n;
  HIP_TRY(hipMemsetAsync(C->flag, 0, sizeof(int), C->stream));
  for (const double* a : {md, me})
    if (a) hipLaunchKernelGGL(k_check_unit, dim3(grid_for(nn)), dim3(kBlock), 0, C->stream, nn, a, C->flag);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(C->host, C->flag, sizeof(int), hipMemcpyDeviceToHost, C->stream));
  TRY(sync(C));
  if (*(const int*)C->host) return SMG_EINVAL;
  set_masked(C, md || me || C->domain);
  return factors_setup(C, md, me, coarsening);
}

int smg_apply(smg_ctx* C, const double* x, double* Sx) {
  if (!C || !x || !Sx) return SMG_EINVAL;
  TRY((residual<double, double, double>(C, C->L64[0], x, (const double*)nullptr, Sx, 1, false)));
  return lowrank_add(C, x, Sx, 1.0);
}

}  // extern "C"

// ============================================== allocation-free residual
// The library's own device scratch for smg_residual_static: the residual's
// per-block partial sums (and the first stage of their reduction).  Each GPU the
// library runs on holds its own copy until the process ends.  Host code uses
// only the address hipGetSymbolAddress gives for the current device, never the
// array's name.
constexpr size_t kScratchDoubles = ((size_t)1 << 20) + 4 * kNormStage;   // 8.4 MB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the context's device, looked up once per
// device with that device current (the caller's current device is restored).
int scratch_address(smg_ctx* C, double** out) {
  const int dev = C->device;
  if (dev < 0 || dev >= kMaxDevices) {
    C->err = "smg_residual_static: device index beyond the library's table";
    return SMG_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != dev) HIP_TRY(hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) HIP_TRY(hipSetDevice(cur));
    if (e != hipSuccess || !p) return hip_fail(C, e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return SMG_OK;
}
}  // namespace

extern "C" {

int smg_residual_static(smg_ctx* C, const double* x, const double* f, double* r, double* norms_dev) {
  if (!C || !x || !f || !r || !norms_dev) return SMG_EINVAL;
  if (C->lr_on) {
    C->err = "smg_residual_static: the rank-one terms are not supported (use smg_residual)";
    return SMG_EINVAL;
  }
  const int nb = residual_blocks(C, C->desc.n);
  const size_t need = 4 * (size_t)nb + 4 * (size_t)kNormStage;
  if (need > kScratchDoubles) {
    C->err = "smg_residual_static: this grid needs " + std::to_string(need) + " doubles of scratch, the library holds " +
             std::to_string(kScratchDoubles);
    return SMG_EWORKSPACE;
  }
  double* s = nullptr;
  TRY(scratch_address(C, &s));
  // every partial is written before it is read: nothing needs clearing
  return residual_into<double, double, double>(C, C->L64[0], x, f, r, 0, s, s + 4 * (size_t)nb, norms_dev);
}

int smg_residual(smg_ctx* C, const double* x, const double* f, double* r, double* norms) {
  if (!C || !x || !f || !r) return SMG_EINVAL;
  if (norms) {
    double h[5];
    TRY(residual_norms64(C, x, f, r, h));
    for (int i = 0; i < 4; ++i) norms[i] = h[i];
    return SMG_OK;
  }
  TRY((residual<double, double, double>(C, C->L64[0], x, f, r, 0, false)));
  return lowrank_add(C, x, r, -1.0);
}

int smg_smooth(smg_ctx* C, int level, int colour, double* x, const double* f) {
  if (!C || !x || !f || (colour != 0 && colour != 1)) return SMG_EINVAL;
  TRY(check_level(C, level, 0));
  return halfsweep<double>(C, C->L64[level], x, f, colour);
}

}  // extern "C"

namespace {
template <typename T>
int sweep_abi(smg_ctx* C, const Level<T>& L, T* alt_hint, const T* xin, T* xout, const T* f, int* one) {
  const size_t len = vlen(L.n, C->N);
  if (xin + len > xout && xout + len > xin) return SMG_EINVAL;   // overlapping vectors
  if (C->desc.theta != 1.0) return SMG_EINVAL;
  const bool fast = one_launch<T>(C, L, alt_hint);
  if (one) *one = fast ? 1 : 0;
  if (fast) return sweep_one_launch<T>(C, L, xin, xout, f, kPlain);
  HIP_TRY(hipMemcpyAsync(xout, xin, sizeof(T) * len, hipMemcpyDeviceToDevice, C->stream));
  TRY(halfsweep<T>(C, L, xout, f, 0));
  return halfsweep<T>(C, L, xout, f, 1);
}
}  // namespace

extern "C" {

int smg_sweep(smg_ctx* C, int level, const double* xin, double* xout, const double* f, int* one) {
  if (!C || !xin || !xout || !f || C->desc.precision != SMG_F64) return SMG_EINVAL;
  TRY(check_level(C, level, 0));
  const Level<double>& L = C->L64[level];
  return sweep_abi<double>(C, L, level == 0 ? C->r64 : L.xa, xin, xout, f, one);
}

int smg_sweep32(smg_ctx* C, int level, const float* xin, float* xout, const float* f, int* one) {
  if (!C || !xin || !xout || !f || C->desc.precision != SMG_F32) return SMG_EINVAL;
  TRY(check_level(C, level, 0));
  const Level<float>& L = C->L32[level];
  return sweep_abi<float>(C, L, level == 0 ? C->r32 : L.xa, xin, xout, f, one);
}

int smg_stream_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src || (bytes & 15) || (((uintptr_t)dst | (uintptr_t)src) & 15)) return SMG_EINVAL;
  const size_t n16 = bytes / 16;
  if (n16 == 0) return SMG_OK;
  const size_t blocks = std::min<size_t>((n16 + kBlock * kCopyUnroll - 1) / (kBlock * kCopyUnroll), 16384);
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(kBlock), 0, (hipStream_t)stream, n16,
                     (const double2*)src, (double2*)dst);
  return hipGetLastError() == hipSuccess ? SMG_OK : SMG_EHIP;
}

int smg_smooth32(smg_ctx* C, int level, int colour, float* x, const float* f) {
  if (!C || !x || !f || (colour != 0 && colour != 1) || C->desc.precision != SMG_F32) return SMG_EINVAL;
  TRY(check_level(C, level, 0));
  return halfsweep<float>(C, C->L32[level], x, f, colour);
}

int smg_restrict(smg_ctx* C, int level, const double* fine, double* coarse) {
  if (!C || !fine || !coarse) return SMG_EINVAL;
  TRY(check_level(C, level, 1));
  return restrict_to<double>(C, C->L64[level].n, fine, coarse);
}

int smg_residual_restrict(smg_ctx* C, int level, const double* x, const double* f, double* coarse) {
  if (!C || !x || !f || !coarse) return SMG_EINVAL;
  TRY(check_level(C, level, 1));
  return residual_restrict<double>(C, C->L64[level], x, f, coarse);
}

int smg_residual_restrict_after_sweep(smg_ctx* C, int level, const double* xold, const double* xnew,
                                      const double* f, double* coarse, int* from_change) {
  if (!C || !xold || !xnew || !f || !coarse || xold == xnew) return SMG_EINVAL;
  TRY(check_level(C, level, 1));
  const bool walk = rr_gs_walk<double>(C, C->L64[level], xold, xnew, coarse);
  if (from_change) *from_change = walk ? 1 : 0;
  if (walk) {
    LAUNCH_CHECK();
    return SMG_OK;
  }
  return residual_restrict<double>(C, C->L64[level], xnew, f, coarse);
}

int smg_jacobi(smg_ctx* C, int level, const double* x, double* xout, const double* f) {
  if (!C || !x || !xout || !f || x == xout) return SMG_EINVAL;
  TRY(check_level(C, level, 0));
  return jacobi<double>(C, C->L64[level], x, xout, f);
}

int smg_prolong_add(smg_ctx* C, int level, const double* coarse, double* fine) {
  if (!C || !fine || !coarse) return SMG_EINVAL;
  TRY(check_level(C, level, 1));
  return prolong_add<double>(C, C->L64[level + 1].n, coarse, fine, C->L64[level].mk);
}

int smg_coarse_solve(smg_ctx* C, const double* F, double* X) {
  if (!C || !F || !X) return SMG_EINVAL;
  return coarse_solve<double>(C, F, X);
}

int smg_level_faces(smg_ctx* C, int level, double* kx, double* ky) {
  if (!C || !kx || !ky) return SMG_EINVAL;
  TRY(check_level(C, level, 0));
  const int n = C->L64[level].n;
  const size_t bytes = (size_t)n * (n + 1) * C->N * sizeof(double);
  HIP_TRY(hipMemcpyAsync(kx, C->L64[level].kx, bytes, hipMemcpyDeviceToDevice, C->stream));
  HIP_TRY(hipMemcpyAsync(ky, C->L64[level].ky, bytes, hipMemcpyDeviceToDevice, C->stream));
  return SMG_OK;
}

int smg_vcycle(smg_ctx* C, double* x, const double* f, int ncycles) {
  if (!C || !x || !f || ncycles < 0) return SMG_EINVAL;
  TRY(zero_outside(C, x));
  if (C->desc.precision == SMG_F64) {
    for (int i = 0; i < ncycles; ++i) TRY(vcycle64(C, x, f));
    return SMG_OK;
  }
  Level<float>& L = C->L32[0];
  TRY((convert<double, float>(C, x, L.x, C->len0)));
  TRY((convert<double, float>(C, f, L.f, C->len0)));
  for (int i = 0; i < ncycles; ++i) TRY(vcycle32(C, L.x, L.f));
  TRY((convert<float, double>(C, L.x, x, C->len0)));
  return SMG_OK;
}

int smg_gmres_precond(smg_ctx* C, double* x, const double* f, int restart, double rtol, int maxit,
                      smg_stats* st) {
  if (!C || !x || !f || restart < 1 || restart > C->desc.gmres_restart || !(rtol > 0) || maxit < 1)
    return SMG_EINVAL;
  TRY(zero_outside(C, x));
  const double t0 = now_ms();
  stats_begin(st);
  double h[5];
  TRY(residual_norms64(C, x, f, C->V, h));
  const double fn = h[4] > 0.0 ? h[4] : 1.0;
  stats_push(st, h[0] / fn);
  int its = 0, restarts = 0, rc = SMG_NOT_CONVERGED;
  while (true) {
    if (!std::isfinite(h[0])) { rc = SMG_ENONFINITE; break; }
    if (h[0] <= rtol * fn) { rc = SMG_OK; break; }
    if (its >= maxit) break;
    int done = 0;
    double est = 0;
    TRY(gmres_cycle(C, x, h[0], restart, rtol * fn, maxit - its, &done, &est, st, fn));
    its += done;
    TRY(residual_norms64(C, x, f, C->V, h));
    if (h[0] > rtol * fn && its < maxit) ++restarts;
  }
  if (st) {
    stats_norms(st, h, fn);
    st->iterations = its;
    st->inner_iterations = its;
    st->restarts = restarts;
    st->time_ms = now_ms() - t0;
  }
  return rc;
}

int smg_solve(smg_ctx* C, double* x, const double* f, int method, double rtol, int maxit, smg_stats* st) {
  if (!C || !x || !f || !(rtol > 0) || maxit < 1) return SMG_EINVAL;
  if (method != SMG_VCYCLE && method != SMG_GMRES) return SMG_EINVAL;
  if (C->lr_on && method != SMG_GMRES) return SMG_EINVAL;
  TRY(zero_outside(C, x));
  const double t0 = now_ms();
  const bool f32 = C->desc.precision == SMG_F32;
  if (method == SMG_GMRES && !f32) {
    const int m = C->desc.gmres_restart;
    if (m < 1) return SMG_EINVAL;
    return smg_gmres_precond(C, x, f, m, rtol, maxit, st);
  }
  if (method == SMG_GMRES && C->desc.gmres_restart < 1) return SMG_EINVAL;
  stats_begin(st);
  double fn = -1.0;   // ||f||, from the first residual pass
  double h[5];
  int its = 0, inner = 0, rc = SMG_NOT_CONVERGED;
  // FP32 stationary refinement keeps its iterate in x or in the scratch vector
  // C->w, alternately: each update x + d is fused with the next residual.
  double* xc = x;
  while (true) {
    if (!f32) {
      TRY(residual_norms64(C, x, f, nullptr, h));
    } else if (method == SMG_VCYCLE) {
      if (its == 0) {
        // FP64 residual rounded straight into the FP32 cycle's right-hand side
        TRY((residual<double, double, float>(C, C->L64[0], x, f, C->L32[0].f, 0, true)));
      } else {
        double* xo = xc == x ? C->w : x;
        TRY(residual_add(C, xc, C->L32[0].x, xo, f, C->L32[0].f));
        xc = xo;
      }
      TRY(readback(C, C->norms, 5));
      for (int i = 0; i < 5; ++i) h[i] = C->host[i];
    } else {
      TRY(residual_norms64(C, x, f, C->V, h));   // r0 straight into the Krylov basis
    }
    if (fn < 0.0) fn = h[4] > 0.0 ? h[4] : 1.0;
    stats_push(st, h[0] / fn);
    if (!std::isfinite(h[0])) { rc = SMG_ENONFINITE; break; }
    if (h[0] <= rtol * fn) { rc = SMG_OK; break; }
    if (its >= maxit) break;
    if (!f32) {
      TRY(vcycle64(C, x, f));
      ++inner;
    } else if (method == SMG_VCYCLE) {
      TRY(run_cycle<float>(C, C->L32[0].x, C->L32[0].f, true));   // the update waits for the next residual
      ++inner;
    } else {
      int done = 0;
      double est = 0;
      const double inner_rtol = 1e-5;
      TRY(gmres_cycle(C, x, h[0], C->desc.gmres_restart, inner_rtol * h[0], C->desc.gmres_restart, &done, &est,
                      nullptr, fn));
      inner += done;
    }
    ++its;
  }
  if (xc != x) HIP_TRY(hipMemcpyAsync(x, xc, C->len0 * sizeof(double), hipMemcpyDeviceToDevice, C->stream));
  TRY(sync(C));
  if (st) {
    stats_norms(st, h, fn);
    st->iterations = its;
    st->inner_iterations = inner;
    st->time_ms = now_ms() - t0;
  }
  return rc;
}

}  // extern "C"

// ======================================================= semismooth Newton
namespace {

SsnArgs ssn_args(const smg_ssn_params& p) { return {p.nu, p.beta, p.nu * p.b, p.nu * p.a}; }

bool ssn_params_valid(const smg_ssn_params& p) {
  return p.nu > 0 && std::isfinite(p.nu) && p.beta >= 0 && std::isfinite(p.beta) && p.a < 0 && p.b > 0 &&
         !std::isnan(p.a) && !std::isnan(p.b) && p.mass > 0 && std::isfinite(p.mass) && p.tol > 0 &&
         p.inner_rtol > 0 && p.maxit >= 0 && p.inner_maxit >= 1 &&
         (p.inner_method == SMG_VCYCLE || p.inner_method == SMG_GMRES) && p.sigma >= 0 && p.sigma < 1 &&
         p.rho >= 0 && p.rho < 1;
}

// w = E[p] of x per node; with F: also F, chi, -mass F into rU (if given) and
// the merit sqrt(mass sum F^2) into *phi (if given; reads it back).
int ssn_eval(smg_ctx* C, const double* x, const SsnArgs& a, double mass, double* w, double* F, double* chi,
             double* rU, double* phi) {
  const int nn = C->desc.n * C->desc.n;
  int nb = 0;
  seg_dispatch(C->N, [&](auto Wc, auto Jc) {
    constexpr int W = decltype(Wc)::value, JM = decltype(Jc)::value;
    const int per = kBlock / W;
    nb = (nn + per - 1) / per;
    hipLaunchKernelGGL((k_ssn_eval<W, JM>), dim3(nb), dim3(kBlock), 0, C->stream, nn, C->N, x, a, mass, w, F, chi,
                       rU, F ? C->spart : (double*)nullptr);
  });
  LAUNCH_CHECK();
  if (F && phi) {
    hipLaunchKernelGGL(k_partials_finalize, dim3(1), dim3(kBlock), 0, C->stream, C->spart, nb, 1, C->sout);
    LAUNCH_CHECK();
    TRY(readback(C, C->sout, 1));
    *phi = std::sqrt(mass * C->host[0]);
  }
  return SMG_OK;
}

// phis[q] = merit at u + gammas[q] du (trial E[p] = w + gammas[q] dw), q < ng.
int ssn_merit(smg_ctx* C, const double* u, const double* du, const double* w, const double* dw, const SsnArgs& a,
              double mass, const double* gammas, int ng, double* phis) {
  const int nn = C->desc.n * C->desc.n;
  const int nb = std::min(kSsnMeritBlocks, (nn + kBlock - 1) / kBlock);
  SsnGammas G{};
  for (int q = 0; q < ng; ++q) G.g[q] = gammas[q];
  hipLaunchKernelGGL(k_ssn_merit, dim3(nb), dim3(kBlock), 0, C->stream, nn, u, du, w, dw, a, G, ng, C->spart);
  hipLaunchKernelGGL(k_partials_finalize, dim3(ng), dim3(kBlock), 0, C->stream, C->spart, nb, kSsnGammas, C->sout);
  LAUNCH_CHECK();
  TRY(readback(C, C->sout, ng));
  for (int q = 0; q < ng; ++q) phis[q] = std::sqrt(mass * C->host[q]);
  return SMG_OK;
}

void ssn_push(smg_ssn_stats* st, double phi, double gamma, int inner) {
  if (!st) return;
  const int k = st->len;
  if (st->phi && k < st->cap) st->phi[k] = phi;
  if (k > 0 && k - 1 < st->cap) {
    if (st->gamma) st->gamma[k - 1] = gamma;
    if (st->inner) st->inner[k - 1] = inner;
  }
  st->len = k + 1;
}

}  // namespace

extern "C" {

int smg_ssn_eval(smg_ctx* C, const double* x, const smg_ssn_params* p, double* w, double* F, double* chi,
                 double* phi) {
  if (!C || !x || !p || !w || ((F == nullptr) != (chi == nullptr)) || !ssn_params_valid(*p)) return SMG_EINVAL;
  if (!(C->desc.flags & SMG_FLAG_SSN)) return SMG_EINVAL;
  double ph = 0.0;
  TRY(ssn_eval(C, x, ssn_args(*p), p->mass, w, F, chi, nullptr, F ? &ph : nullptr));
  if (phi) *phi = F ? ph : 0.0;
  return SMG_OK;
}

int smg_ssn_merit(smg_ctx* C, const double* u, const double* du, const double* w, const double* dw,
                  const smg_ssn_params* p, int ng, const double* gammas, double* phis) {
  if (!C || !u || !du || !w || !dw || !p || !gammas || !phis || ng < 1 || ng > kSsnGammas || !ssn_params_valid(*p))
    return SMG_EINVAL;
  if (!(C->desc.flags & SMG_FLAG_SSN)) return SMG_EINVAL;
  return ssn_merit(C, u, du, w, dw, ssn_args(*p), p->mass, gammas, ng, phis);
}

int smg_ssn_solve(smg_ctx* C, double* x, const double* f, const smg_ssn_params* prm, smg_ssn_stats* st) {
  if (!C || !x || !f || !prm || !ssn_params_valid(*prm)) return SMG_EINVAL;
  if (!(C->desc.flags & SMG_FLAG_SSN)) return SMG_EINVAL;
  if (prm->inner_method == SMG_GMRES && C->desc.gmres_restart < 1) return SMG_EINVAL;
  TRY(zero_outside(C, x));
  const double t0 = now_ms();
  const smg_ssn_params& p = *prm;
  const double sigma = p.sigma > 0 ? p.sigma : 1e-4, rho = p.rho > 0 ? p.rho : 0.5;
  const SsnArgs a = ssn_args(p);
  const int N = C->N, nn = C->desc.n * C->desc.n;
  const size_t len = C->len0;
  double* const xU = x + (size_t)N * nn;
  if (st) { st->iterations = 0; st->inner_total = 0; st->init_iterations = 0; st->len = 0; st->phi_final = 0.0; }
  set_masked(C, true);
  // Algorithm 2, first step: the state and adjoint equations for u0 = x's U
  // block, as the system with D_j = 0 (md = 0) whose U row M u = M u0 fixes u
  TRY(fill(C, C->schi, (size_t)nn, 0.0));
  TRY(factors_setup(C, C->schi, nullptr, SMG_COARSEN_FULL));
  HIP_TRY(hipMemcpyAsync(C->sr, f, len * sizeof(double), hipMemcpyDeviceToDevice, C->stream));
  hipLaunchKernelGGL(k_scale, dim3((nn + kBlock - 1) / kBlock), dim3(kBlock), 0, C->stream, nn, xU, p.mass,
                     C->sr + (size_t)N * nn);
  LAUNCH_CHECK();
  smg_stats ist{};
  int rc = smg_solve(C, x, C->sr, p.inner_method, p.inner_rtol, p.inner_maxit, &ist);
  if (rc < 0) return rc;
  if (st) st->init_iterations = ist.iterations;
  if (rc != SMG_OK) { C->err = "initial state and adjoint solve did not converge"; return SMG_NOT_CONVERGED; }
  // Newton right-hand side: zero but for its U block, -M F(u^k), which every
  // evaluation rewrites
  TRY(fill(C, C->sr, len, 0.0));
  double* const rU = C->sr + (size_t)N * nn;
  double phi = 0.0;
  TRY(ssn_eval(C, x, a, p.mass, C->sw, C->sF, C->schi, rU, &phi));
  ssn_push(st, phi, 0.0, 0);
  int k = 0, inner_total = 0;
  rc = SMG_NOT_CONVERGED;
  while (true) {
    if (!std::isfinite(phi)) { rc = SMG_ENONFINITE; break; }
    if (phi <= p.tol) { rc = SMG_OK; break; }
    if (k >= p.maxit) break;
    // Newton system of the current active set (md = chi, E_j unchanged; coarse
    // levels by full weighting), solved from zero
    TRY(factors_setup(C, C->schi, nullptr, SMG_COARSEN_FULL));
    TRY(fill(C, C->sdx, len, 0.0));
    smg_stats ns{};
    const int lr = smg_solve(C, C->sdx, C->sr, p.inner_method, p.inner_rtol, p.inner_maxit, &ns);
    if (lr < 0) return lr;
    inner_total += ns.iterations;
    TRY(ssn_eval(C, C->sdx, a, p.mass, C->sdw, nullptr, nullptr, nullptr, nullptr));
    // line search: the first of 1, rho, rho^2, ... (at most 64) with sufficient
    // decrease of the merit, priced kSsnGammas at a time
    double g[kSsnGammas], phis[kSsnGammas], gamma = 0.0, next = 1.0;
    bool found = false;
    for (int batch = 0; batch < 64 / kSsnGammas && !found; ++batch) {
      for (int q = 0; q < kSsnGammas; ++q) { g[q] = next; next *= rho; }
      TRY(ssn_merit(C, xU, C->sdx + (size_t)N * nn, C->sw, C->sdw, a, p.mass, g, kSsnGammas, phis));
      for (int q = 0; q < kSsnGammas && !found; ++q)
        if (phis[q] - phi <= -sigma * phi) { gamma = g[q]; found = true; }
    }
    if (!found) { C->err = "line search found no decrease of the merit"; rc = SMG_NOT_CONVERGED; break; }
    hipLaunchKernelGGL(k_axpy, dim3(grid_for(len)), dim3(kBlock), 0, C->stream, len, x, gamma, C->sdx);
    LAUNCH_CHECK();
    TRY(ssn_eval(C, x, a, p.mass, C->sw, C->sF, C->schi, rU, &phi));
    ++k;
    ssn_push(st, phi, gamma, ns.iterations);
  }
  TRY(sync(C));
  if (st) {
    st->iterations = k;
    st->inner_total = inner_total;
    st->phi_final = phi;
    st->time_ms = now_ms() - t0;
  }
  return rc;
}

}  // extern "C"

// ======================================================= risk-averse (CVaR)
namespace {

// The C^2 smoothing of max(0, x) (eq. smoothapproximation; middle branch in
// s = x + eps/2: s^3/eps^2 - s^4/(2 eps^3)) and its first two derivatives.
double cv_dg(double x, double eps) {
  if (x <= -0.5 * eps) return 0.0;
  if (x >= 0.5 * eps) return 1.0;
  const double s = x + 0.5 * eps;
  return 3.0 * s * s / (eps * eps) - 2.0 * s * s * s / (eps * eps * eps);
}
double cv_ddg(double x, double eps) {
  if (x <= -0.5 * eps || x >= 0.5 * eps) return 0.0;
  const double s = x + 0.5 * eps;
  return 6.0 * s / (eps * eps) - 6.0 * s * s / (eps * eps * eps);
}

int set_sample_c(smg_ctx* C, const double* c) {
  const int N = C->N;
  std::vector<double> cc(c, c + N);
  for (int l = 0; l < C->nlev; ++l) {
    if (l > 0)
      for (int j = 0; j < N; ++j) cc[j] *= 4.0;
    HIP_TRY(hipMemcpyAsync(C->L64[l].c, cc.data(), sizeof(double) * N, hipMemcpyHostToDevice, C->stream));
    TRY(sync(C));   // cc is reused for the next level
  }
  return node_terms(C);
}

struct CvarRun {
  smg_ctx* C;
  const smg_cvar_params* p;
  const double* f;
  const double* yd;
  std::vector<double> q, w, c;   // per sample: Q_j + t, w_j, c_j
  int inner_total = 0, lin_solves = 0, lin_total = 0, inner_capped = 0, inner_stalled = 0;
  std::vector<int> counts;       // Newton steps of every evaluation of h(t)

  double F4(double t) const {
    double s = 0.0;
    for (int j = 0; j < C->N; ++j) s += p->zeta[j] * cv_dg(q[j] - t, p->eps);
    return 1.0 - s / (1.0 - p->lambda);
  }
  // z at x into C->cz; q_j = z_j . z_j / (2 mass) to the host
  int zq(const double* x) {
    const int nn = C->desc.n * C->desc.n, N = C->N;
    hipLaunchKernelGGL(k_cvar_z, dim3(grid_for((size_t)nn * N)), dim3(kBlock), 0, C->stream, nn, N, p->mass, x, yd,
                       C->domain ? (const double*)C->L64[0].dom : (const double*)nullptr, C->cz);
    LAUNCH_CHECK();
    TRY(sample_dots(C, C->cz, C->cz, nullptr, C->cs));
    HIP_TRY(hipMemcpyAsync(q.data(), C->cs, sizeof(double) * N, hipMemcpyDeviceToHost, C->stream));
    TRY(sync(C));
    for (int j = 0; j < N; ++j) q[j] *= 0.5 / p->mass;
    return SMG_OK;
  }
  // C_j = c_j(x, t) I, b(c) into C->cb, C->cr = b - S(c) x = -F_1; ||F_1|| to fn
  int F1(const double* x, double t, double* fn) {
    const int nn = C->desc.n * C->desc.n, N = C->N;
    TRY(zq(x));
    for (int j = 0; j < N; ++j) c[j] = p->zeta[j] * cv_dg(q[j] - t, p->eps) * p->mass / (1.0 - p->lambda);
    TRY(set_sample_c(C, c.data()));
    HIP_TRY(hipMemcpyAsync(C->cc, c.data(), sizeof(double) * N, hipMemcpyHostToDevice, C->stream));
    HIP_TRY(hipMemcpyAsync(C->cb, f, sizeof(double) * C->len0, hipMemcpyDeviceToDevice, C->stream));
    hipLaunchKernelGGL(k_cvar_rhs, dim3(grid_for((size_t)nn * N)), dim3(kBlock), 0, C->stream, nn, N,
                       (const double*)C->cc, yd, C->domain ? (const double*)C->L64[0].dom : (const double*)nullptr,
                       C->cb);
    LAUNCH_CHECK();
    C->lr_on = false;
    double h[5];
    TRY(residual_norms64(C, x, C->cb, C->cr, h));
    *fn = h[0];
    return SMG_OK;
  }
  // w_j at (q, t) to the host and the device; rank-one terms on where any is nonzero
  int set_w(double t, bool* any) {
    *any = false;
    for (int j = 0; j < C->N; ++j) {
      w[j] = p->zeta[j] * cv_ddg(q[j] - t, p->eps) / (1.0 - p->lambda);
      *any = *any || w[j] != 0.0;
    }
    HIP_TRY(hipMemcpyAsync(C->cwv, w.data(), sizeof(double) * C->N, hipMemcpyHostToDevice, C->stream));
    return SMG_OK;
  }
  // sol = J_11^{-1} rhs by GMRES from zero (rank-one terms as set_w left them)
  int solve(double* sol, const double* rhs, bool lowrank) {
    HIP_TRY(hipMemsetAsync(sol, 0, sizeof(double) * C->len0, C->stream));
    C->lr_on = lowrank;
    smg_stats st{};
    const int rc = smg_gmres_precond(C, sol, rhs, C->desc.gmres_restart, p->lin_rtol, p->lin_maxit, &st);
    C->lr_on = false;
    if (rc != SMG_OK && rc != SMG_NOT_CONVERGED) return rc;
    ++lin_solves;
    lin_total += st.iterations;
    return SMG_OK;
  }
  // h(t): Newton on F_1(.; t) = 0 from x, each step halved until ||F_1||
  // decreases (full steps: an option; they cycle on the Monte Carlo problems),
  // stopped once both the relative and the absolute residual are at most
  // inner_tol (Section 6, the rules stated with the risk-averse table; min of
  // the two: an option), or when no halving decreases ||F_1|| although the
  // absolute part is met (the rounding floor: the step is not taken).
  int inner(double* x, double t) {
    double fn, f0;
    TRY(F1(x, t, &fn));
    f0 = fn;
    const size_t bytes = sizeof(double) * C->len0;
    const bool use_min = p->inner_rule == SMG_CVAR_INNER_MIN;
    int k = 0;
    for (; k < p->inner_maxit; ++k) {
      const double part = use_min ? std::min(fn / f0, fn) : std::max(fn / f0, fn);
      if (fn == 0.0 || part <= p->inner_tol) break;
      bool any;
      TRY(set_w(t, &any));
      TRY(solve(C->cdx, C->cr, any));
      double ft = 0.0;
      if (p->inner_full_steps) {
        hipLaunchKernelGGL(k_axpy, dim3(grid_for(C->len0)), dim3(kBlock), 0, C->stream, C->len0, x, 1.0,
                           (const double*)C->cdx);
        LAUNCH_CHECK();
        TRY(F1(x, t, &ft));
      } else {
        double a = 1.0;
        bool ok = false;
        for (int ls = 0; ls <= 30; ++ls) {
          HIP_TRY(hipMemcpyAsync(C->cxt, x, bytes, hipMemcpyDeviceToDevice, C->stream));
          hipLaunchKernelGGL(k_axpy, dim3(grid_for(C->len0)), dim3(kBlock), 0, C->stream, C->len0, C->cxt, a,
                             (const double*)C->cdx);
          LAUNCH_CHECK();
          TRY(F1(C->cxt, t, &ft));
          if (ft <= (1.0 - 1e-4 * a) * fn) { ok = true; break; }
          if (ls < 30) a *= 0.5;
        }
        if (!ok && fn <= p->inner_tol) {   // the rounding floor: keep x, C_j back at x
          TRY(F1(x, t, &ft));
          ++inner_stalled;
          counts.push_back(k);
          return SMG_OK;
        }
        HIP_TRY(hipMemcpyAsync(x, C->cxt, bytes, hipMemcpyDeviceToDevice, C->stream));
      }
      fn = ft;
      ++inner_total;
    }
    if (k >= p->inner_maxit) ++inner_capped;
    counts.push_back(k);
    return SMG_OK;
  }
  // the root of F_2(x; t) = 0 in t for the current q (bisection)
  double split_t() const {
    double lo = q[0], hi = q[0];
    for (double v : q) { lo = std::min(lo, v); hi = std::max(hi, v); }
    lo -= p->eps;
    hi += p->eps;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid == lo || mid == hi) break;
      if (F4(mid) < 0.0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
  }
};

bool cvar_params_valid(const smg_cvar_params& p, int N) {
  if (!(p.lambda >= 0.0 && p.lambda < 1.0) || !(p.eps > 0.0 && std::isfinite(p.eps)) ||
      !(p.mass > 0.0 && std::isfinite(p.mass)) || !p.zeta || !(p.tol > 0) || !(p.inner_tol > 0) ||
      !(p.lin_rtol > 0) || p.maxit < 0 || p.inner_maxit < 1 || p.lin_maxit < 1 || !(p.sigma >= 0 && p.sigma < 1) ||
      !(p.rho >= 0 && p.rho < 1) || (p.inner_rule != SMG_CVAR_INNER_MAX && p.inner_rule != SMG_CVAR_INNER_MIN) ||
      (p.inner_full_steps != 0 && p.inner_full_steps != 1))
    return false;
  for (int j = 0; j < N; ++j)
    if (!(p.zeta[j] >= 0.0 && std::isfinite(p.zeta[j]))) return false;
  return true;
}

}  // namespace

extern "C" {

int smg_set_sample_weights(smg_ctx* C, const double* c) {
  if (!C || !c) return SMG_EINVAL;
  for (int j = 0; j < C->N; ++j)
    if (!(c[j] >= 0.0 && std::isfinite(c[j]))) return SMG_EINVAL;
  return set_sample_c(C, c);
}

int smg_set_lowrank(smg_ctx* C, const double* z, const double* w) {
  if (!C || !(C->desc.flags & SMG_FLAG_CVAR) || (!z) != (!w)) return SMG_EINVAL;
  if (!z) { C->lr_on = false; return SMG_OK; }
  const size_t nn = (size_t)C->desc.n * C->desc.n;
  HIP_TRY(hipMemcpyAsync(C->cz, z, sizeof(double) * nn * C->N, hipMemcpyDeviceToDevice, C->stream));
  HIP_TRY(hipMemcpyAsync(C->cwv, w, sizeof(double) * C->N, hipMemcpyDeviceToDevice, C->stream));
  C->lr_on = true;
  return SMG_OK;
}

int smg_cvar_solve(smg_ctx* C, double* x, const double* f, const double* yd, double* t,
                   const smg_cvar_params* prm, smg_cvar_stats* st) {
  if (!C || !x || !f || !yd || !t || !prm || !std::isfinite(*t)) return SMG_EINVAL;
  if (!(C->desc.flags & SMG_FLAG_CVAR) || C->desc.gmres_restart < 1) return SMG_EINVAL;
  smg_cvar_params p = *prm;
  if (p.sigma == 0.0) p.sigma = 1e-4;
  if (p.rho == 0.0) p.rho = 0.5;
  if (!cvar_params_valid(p, C->N)) return SMG_EINVAL;
  const double t0ms = now_ms();
  TRY(zero_outside(C, x));
  const int N = C->N;
  CvarRun R{C, &p, f, yd, std::vector<double>(N), std::vector<double>(N), std::vector<double>(N)};
  double tk = *t;
  if (st) st->len = 0;
  auto push = [&](double v) { if (st && st->F && st->len < st->cap) st->F[st->len++] = v; };
  TRY(R.inner(x, tk));
  int k = 0, rc = SMG_NOT_CONVERGED;
  double Fk = NAN;
  while (true) {
    Fk = R.F4(tk);
    push(std::fabs(Fk));
    if (!std::isfinite(Fk)) { rc = SMG_ENONFINITE; break; }
    if (std::fabs(Fk) <= p.tol) { rc = SMG_OK; break; }
    if (k >= p.maxit) break;
    bool any = false;
    for (int j = 0; j < N && !any; ++j) any = cv_ddg(R.q[j] - tk, p.eps) != 0.0;
    if (!any) {   // eq. condition: the split step
      TRY(R.inner(x, tk));
      tk = R.split_t();
      TRY(R.inner(x, tk));   // F(t) = F_2(h(t), t): the next test needs h at the new t
    } else {
      double fn;
      TRY(R.F1(x, tk, &fn));                       // S(c) and z at (x^k, t^k)
      TRY(R.set_w(tk, &any));
      const size_t nn = (size_t)C->desc.n * C->desc.n;
      HIP_TRY(hipMemsetAsync(C->cj12, 0, sizeof(double) * C->len0, C->stream));
      hipLaunchKernelGGL(k_lowrank_add, dim3(grid_for(nn * N)), dim3(kBlock), 0, C->stream, (int)nn, N, -1.0,
                         (const double*)C->cwv, (const double*)C->cz, C->cj12);   // J_12 = -w_j z_j
      LAUNCH_CHECK();
      TRY(R.solve(C->cxi, C->cj12, true));
      TRY(sample_dots(C, C->cz, C->cxi, C->cwv, C->cs));
      std::vector<double> zx(N);
      HIP_TRY(hipMemcpyAsync(zx.data(), C->cs, sizeof(double) * N, hipMemcpyDeviceToHost, C->stream));
      TRY(sync(C));
      double Fp = 0.0;
      for (int j = 0; j < N; ++j) Fp += R.w[j] + zx[j];
      const double d = -Fk / Fp;
      HIP_TRY(hipMemcpyAsync(C->cxk, x, sizeof(double) * C->len0, hipMemcpyDeviceToDevice, C->stream));
      double gamma = 1.0;
      for (int ls = 0; ls <= 30; ++ls) {
        if (ls > 0)
          HIP_TRY(hipMemcpyAsync(x, C->cxk, sizeof(double) * C->len0, hipMemcpyDeviceToDevice, C->stream));
        TRY(R.inner(x, tk + gamma * d));
        if (std::fabs(R.F4(tk + gamma * d)) - std::fabs(Fk) <= -p.sigma * std::fabs(Fk)) break;
        if (ls < 30) gamma *= p.rho;
      }
      tk += gamma * d;
    }
    ++k;
  }
  C->lr_on = false;
  TRY(sync(C));
  *t = tk;
  if (st) {
    st->outer = k;
    st->inner_total = R.inner_total;
    st->linear_solves = R.lin_solves;
    st->linear_total = R.lin_total;
    st->t = tk;
    st->F_final = std::fabs(Fk);
    st->time_ms = now_ms() - t0ms;
    st->inner_capped = R.inner_capped;
    st->inner_stalled = R.inner_stalled;
    st->inner_len = 0;
    if (st->inner_counts)
      for (int c : R.counts)
        if (st->inner_len < st->inner_cap) st->inner_counts[st->inner_len++] = c;
  }
  return rc;
}

}  // extern "C"

// ================================================================ batch C ABI
extern "C" {

}  // extern "C"

// A batch: its instances in groups (the smallest instances, then one finest grid
// size per group), smallest first;
// every group is a lockstep batch of its own (BatchGroup) and the groups run one
// after another on the contexts' stream.  Small instances then retire after
// steps of their own size, not steps as long as the largest instance's.
struct smg_batch {
  std::vector<BatchGroup*> groups;
  std::vector<int> gidx, gpos;      // group of instance i and its index there
  std::vector<hipEvent_t> ev;       // per group: done flags copied
  hipStream_t stream = nullptr;     // the contexts' stream
  int count = 0;
  std::string err;
};

namespace {

int group_validate(smg_ctx* const* ctxs, int count, const int* lanes, BatchGroup* B) {
  if (!ctxs || count < 1) return SMG_EINVAL;
  B->count = count;
  B->ctx.assign(ctxs, ctxs + count);
  B->lanes.resize(count);
  B->fnorm.assign(count, 1.0);
  B->precision = ctxs[0] ? ctxs[0]->desc.precision : 0;
  B->jm = 1;
  B->vw = B->precision == SMG_F32 ? 2 : 1;
  for (int i = 0; i < count; ++i) {
    if (!ctxs[i]) return SMG_EINVAL;
    if (!vec2_ctx(B->precision, ctxs[i]->N)) B->vw = 1;
  }
  for (int i = 0; i < count; ++i) {
    smg_ctx* C = ctxs[i];
    if (C->desc.precision != B->precision || C->desc.theta != 1.0 || (C->desc.flags & SMG_FLAG_JACOBI) || C->domain ||
        C->desc.pre < 1 || C->desc.post < 1 ||
        C->desc.pre != ctxs[0]->desc.pre || C->desc.post != ctxs[0]->desc.post || C->stream != ctxs[0]->stream)
      return SMG_EINVAL;
    const int W = lanes ? lanes[i] : default_lanes(C->N, C->desc.precision);
    if (!pow2_ok(W) || samples_per_lane(C->N, W, B->vw) > 8) return SMG_EINVAL;
    B->lanes[i] = W;
    B->jm = std::max(B->jm, samples_per_lane(C->N, W, B->vw));
  }
  B->stream = ctxs[0]->stream;
  return SMG_OK;
}

// Bytes one V-cycle correction of an instance touches: its level iterates,
// right-hand sides and faces in the cycle's precision, the FP64 outer vectors.
double instance_bytes(const smg_ctx* C) {
  const double w = C->desc.precision == SMG_F32 ? 4.0 : 8.0;
  double b = 0.0;
  for (int l = 0; l < C->nlev; ++l) {
    const double n = C->L64[l].n;
    b += w * (2.0 * (2.0 * C->N + 1.0) * n * n + 2.0 * C->N * n * (n + 1.0));
  }
  return b + 8.0 * 3.0 * (double)C->len0;
}

// Groups of instances: the smallest instances (a correction cycle that touches
// at most kFastLaneBytes: their steps run at the launch-latency floor) in one
// group of their own, the others one group per finest grid size; groups in order
// of the bytes a correction cycle of their largest instance touches (smallest
// first), instances in input order.  Measured on 64 uneven instances (n 63..255,
// N 16..128), retirement of the 63x63, N=16 instances / solves per second:
// this grouping 2.1 ms / 618; one group per grid size 4.5 ms / 626; one group
// per (n, N) 1.7 ms / 574; the small instances then all others in one lockstep
// group 2.1 ms / 630 (but the 127x127 instances retire with the 255x255 ones,
// at 92 ms instead of 20); all in one lockstep group 79 ms / 642; groups packed
// to fit the Infinity Cache lost a quarter of the throughput.
constexpr double kFastLaneBytes = 16e6;

std::vector<std::vector<int>> group_members(smg_ctx* const* ctxs, int count) {
  std::vector<int> ns;
  std::vector<double> cost;
  std::vector<std::vector<int>> g;
  for (int i = 0; i < count; ++i) {
    const int n = instance_bytes(ctxs[i]) <= kFastLaneBytes ? 0 : ctxs[i]->desc.n;   // group key
    size_t k = 0;
    while (k < ns.size() && ns[k] != n) ++k;
    if (k == ns.size()) { ns.push_back(n); g.emplace_back(); cost.push_back(0.0); }
    g[k].push_back(i);
    cost[k] = std::max(cost[k], instance_bytes(ctxs[i]));
  }
  std::vector<int> order(g.size());
  for (size_t k = 0; k < g.size(); ++k) order[k] = (int)k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] < cost[b]; });
  std::vector<std::vector<int>> out;
  for (int k : order) out.push_back(g[k]);
  return out;
}

size_t group_bytes(BatchGroup* G) {
  std::vector<char> blob;
  const size_t b = G->precision == SMG_F32 ? batch_build<float>(G, nullptr, nullptr, &blob)
                                           : batch_build<double>(G, nullptr, nullptr, &blob);
  return (b + 255) & ~(size_t)255;
}

void group_destroy(BatchGroup* G) {
  if (!G) return;
  if (G->graph) (void)hipGraphExecDestroy(G->graph);
  if (G->cap_stream) (void)hipStreamDestroy(G->cap_stream);
  if (G->host) (void)hipHostFree(G->host);
  delete G;
}

// One group's state and tables into its slice of the workspace.
int group_setup(BatchGroup* B, double* const* x, const double* const* f, void* workspace, size_t bytes) {
  B->xs.assign(x, x + B->count);
  for (int i = 0; i < B->count; ++i) {
    double fn = 0.0;
    const int rc = vec_norm(B->ctx[i], f[i], B->ctx[i]->len0, &fn);
    if (rc != SMG_OK) { B->err = B->ctx[i]->err; return rc; }
    B->fnorm[i] = fn > 0.0 ? fn : 1.0;
  }
  std::vector<char> blob;
  B->base = (char*)workspace;
  const size_t need = B->precision == SMG_F32 ? batch_build<float>(B, x, f, &blob)
                                              : batch_build<double>(B, x, f, &blob);
  if (!workspace || bytes < need || ((uintptr_t)workspace & 255) != 0) return SMG_EWORKSPACE;
  B->bytes = need;
  BHIP(hipMemcpyAsync(workspace, blob.data(), blob.size(), hipMemcpyHostToDevice, B->stream));
  BHIP(hipStreamSynchronize(B->stream));
  BHIP(hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking));
  BHIP(hipHostMalloc(&B->host, (sizeof(int) + sizeof(double) + 2 * sizeof(long long)) * (B->count + 2),
                     hipHostMallocDefault));
  return SMG_OK;
}

// Start a solve of group B on its stream: clear the state, stamp t0 (the first
// group's stamp is the batch's start), capture the refinement step's graph (per
// tolerance and limit) if needed.
int group_begin(BatchGroup* B, double rtol, int maxit) {
  hipStream_t s = B->stream;
  BHIP(hipMemsetAsync(B->done, 0, sizeof(int) * B->count, s));
  BHIP(hipMemsetAsync(B->iters, 0, sizeof(int) * B->count, s));
  hipLaunchKernelGGL(kb_stamp, dim3(1), dim3(64), 0, s, B->t0);
  BHIP(hipGetLastError());
  if (!B->graph || B->cap_tol != rtol || B->cap_maxit != maxit) {
    if (B->graph) { (void)hipGraphExecDestroy(B->graph); B->graph = nullptr; }
    BHIP(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal));
    const hipStream_t keep = B->stream;
    B->stream = B->cap_stream;
    const int rc = batch_step(B, rtol, maxit);
    B->stream = keep;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(B->cap_stream, &g);
    if (rc != SMG_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
    BHIP(e);
    const hipError_t ei = hipGraphInstantiate(&B->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    BHIP(ei);
    B->cap_tol = rtol;
    B->cap_maxit = maxit;
  }
  return SMG_OK;
}

// Results of group B after its last step (on its stream, synchronized).
int group_finish(BatchGroup* B, smg_stats* const* stats, int* rc_out, const long long* t0dev) {
  hipStream_t s = B->stream;
  const int cnt = B->count;
  std::vector<int> its(cnt), dn(cnt);
  std::vector<double> rel(cnt);
  std::vector<long long> td(cnt);
  long long t0 = 0;
  BHIP(hipMemcpyAsync(dn.data(), B->done, sizeof(int) * cnt, hipMemcpyDeviceToHost, s));
  BHIP(hipMemcpyAsync(its.data(), B->iters, sizeof(int) * cnt, hipMemcpyDeviceToHost, s));
  BHIP(hipMemcpyAsync(rel.data(), B->relres, sizeof(double) * cnt, hipMemcpyDeviceToHost, s));
  BHIP(hipMemcpyAsync(td.data(), B->tdone, sizeof(long long) * cnt, hipMemcpyDeviceToHost, s));
  BHIP(hipMemcpyAsync(&t0, t0dev, sizeof(long long), hipMemcpyDeviceToHost, s));
  BHIP(hipStreamSynchronize(s));
  if (B->precision == SMG_F32) {
    // iterates after an odd number of FP32 corrections live in the context's w
    for (int i = 0; i < cnt; ++i)
      if (its[i] & 1)
        BHIP(hipMemcpyAsync(B->xs[i], B->ctx[i]->w, B->ctx[i]->len0 * sizeof(double), hipMemcpyDeviceToDevice, s));
    BHIP(hipStreamSynchronize(s));
  }
  int dev = 0, khz = 0;
  BHIP(hipGetDevice(&dev));
  BHIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  for (int i = 0; i < cnt; ++i) {
    if (dn[i] != 1 && *rc_out == SMG_OK) *rc_out = SMG_NOT_CONVERGED;
    if (!std::isfinite(rel[i])) *rc_out = SMG_ENONFINITE;
    if (stats && stats[i]) {
      smg_stats* st = stats[i];
      st->iterations = its[i];
      st->inner_iterations = its[i];
      st->restarts = 0;
      st->relres = rel[i];
      st->relres_y = st->relres_u = st->relres_p = NAN;
      st->time_ms = dn[i] && khz > 0 ? (double)(td[i] - t0) / (double)khz : NAN;
      st->history_len = 0;
    }
  }
  return SMG_OK;
}

}  // namespace

extern "C" {

size_t smg_batch_workspace_bytes(smg_ctx* const* ctxs, int count) {
  if (!ctxs || count < 1) return 0;
  for (int i = 0; i < count; ++i)
    if (!ctxs[i]) return 0;
  BatchGroup all;
  if (group_validate(ctxs, count, nullptr, &all) != SMG_OK) return 0;
  size_t total = 0;
  for (const auto& m : group_members(ctxs, count)) {
    std::vector<smg_ctx*> sub;
    for (int i : m) sub.push_back(ctxs[i]);
    BatchGroup G;
    if (group_validate(sub.data(), (int)sub.size(), nullptr, &G) != SMG_OK) return 0;
    total += group_bytes(&G);
  }
  return total + 256;
}

void smg_batch_destroy(smg_batch* B) {
  if (!B) return;
  for (BatchGroup* G : B->groups) group_destroy(G);
  for (hipEvent_t e : B->ev) (void)hipEventDestroy(e);
  delete B;
}

const char* smg_batch_last_error(const smg_batch* B) { return B ? B->err.c_str() : ""; }

int smg_batch_setup(smg_ctx* const* ctxs, int count, double* const* x, const double* const* f, const int* lanes,
                    void* workspace, size_t workspace_bytes, smg_batch** out) {
  if (!out) return SMG_EINVAL;
  *out = nullptr;
  if (!x || !f || !ctxs || count < 1) return SMG_EINVAL;
  for (int i = 0; i < count; ++i)
    if (!ctxs[i] || !x[i] || !f[i]) return SMG_EINVAL;
  {
    BatchGroup all;   // the batch-wide rules (same precision, pre/post, stream, ...)
    const int rc = group_validate(ctxs, count, lanes, &all);
    if (rc != SMG_OK) return rc;
  }
  smg_batch* B = new smg_batch();
  B->count = count;
  B->stream = ctxs[0]->stream;
  B->gidx.assign(count, 0);
  B->gpos.assign(count, 0);
  char* base = (char*)workspace;
  size_t off = 0;
  auto fail = [&](int rc, const std::string& why) {
    B->err = why;
    const std::string keep = B->err;
    smg_batch_destroy(B);
    (void)keep;
    return rc;
  };
  if (!workspace || ((uintptr_t)workspace & 255) != 0) { smg_batch_destroy(B); return SMG_EWORKSPACE; }
  const auto members = group_members(ctxs, count);
  for (size_t g = 0; g < members.size(); ++g) {
    std::vector<smg_ctx*> sub;
    std::vector<double*> sx;
    std::vector<const double*> sf;
    std::vector<int> sl;
    for (size_t k = 0; k < members[g].size(); ++k) {
      const int i = members[g][k];
      sub.push_back(ctxs[i]); sx.push_back(x[i]); sf.push_back(f[i]);
      sl.push_back(lanes ? lanes[i] : default_lanes(ctxs[i]->N, ctxs[i]->desc.precision));
      B->gidx[i] = (int)g;
      B->gpos[i] = (int)k;
    }
    BatchGroup* G = new BatchGroup();
    B->groups.push_back(G);
    int rc = group_validate(sub.data(), (int)sub.size(), sl.data(), G);
    if (rc != SMG_OK) return fail(rc, "group validation");
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return fail(SMG_EHIP, "hipEventCreate");
    B->ev.push_back(e);
    const size_t gb = group_bytes(G);
    if (off + gb > workspace_bytes) { smg_batch_destroy(B); return SMG_EWORKSPACE; }
    rc = group_setup(G, sx.data(), sf.data(), base + off, gb);
    if (rc != SMG_OK) return fail(rc, G->err);
    off += gb;
  }
  *out = B;
  return SMG_OK;
}

// Solve every instance to ||f_i - S_i x_i|| <= rtol ||f_i|| (x_i: initial guess
// in, solution out), at most maxit correction cycles each.  The groups run one
// after another on the contexts' stream, each replaying its refinement step's
// graph until all its instances are retired; the next group's first steps are
// queued before the current group's done flags are read.  stats (may be null)
// receives count entries: iterations = correction V-cycles, relres, time_ms =
// device time from the start of the first group to the step that retired the
// instance.  wall_ms (may be null) receives the host wall time of the whole
// batch.
int smg_batch_solve(smg_batch* B, double rtol, int maxit, smg_stats* stats, double* wall_ms) {
  if (!B || !(rtol > 0) || maxit < 1) return SMG_EINVAL;
  const double t_start = now_ms();
  const int ng = (int)B->groups.size();
  for (int g = 0; g < ng; ++g) {
    const int rc = group_begin(B->groups[g], rtol, maxit);
    if (rc != SMG_OK) { B->err = B->groups[g]->err; return rc; }
  }
  const int first = std::min(maxit + 2, 8);   // typical refinement steps to 1e-8
  std::vector<int> steps(ng, 0);
  auto launch = [&](int g, int k) -> int {
    for (int i = 0; i < k; ++i) { BHIP(hipGraphLaunch(B->groups[g]->graph, B->stream)); ++steps[g]; }
    return SMG_OK;
  };
  auto flags = [&](int g) -> int {
    BatchGroup* G = B->groups[g];
    BHIP(hipMemcpyAsync(G->host, G->done, sizeof(int) * G->count, hipMemcpyDeviceToHost, B->stream));
    BHIP(hipEventRecord(B->ev[g], B->stream));
    return SMG_OK;
  };
  // A group's steps are not queued behind the next group's: the next group
  // starts once the host has seen every instance of this one retire (one host
  // round trip of idle GPU per group and per check).
  for (int g = 0; g < ng; ++g) {
    TRY(launch(g, first));
    TRY(flags(g));
    BatchGroup* G = B->groups[g];
    while (true) {
      BHIP(hipEventSynchronize(B->ev[g]));
      bool all = true;
      for (int i = 0; i < G->count; ++i) all = all && ((int*)G->host)[i] != 0;
      if (all || steps[g] >= maxit + 2) break;
      TRY(launch(g, 2));
      TRY(flags(g));
    }
  }
  int rc = SMG_OK;
  for (int g = 0; g < ng; ++g) {
    std::vector<smg_stats*> sp(B->groups[g]->count, nullptr);
    if (stats)
      for (int i = 0; i < B->count; ++i)
        if (B->gidx[i] == g) sp[B->gpos[i]] = &stats[i];
    const int r = group_finish(B->groups[g], sp.data(), &rc, B->groups[0]->t0);
    if (r != SMG_OK) { B->err = B->groups[g]->err; return r; }
  }
  if (wall_ms) *wall_ms = now_ms() - t_start;
  return rc;
}

// Autotuner of the lanes-per-node width of one context's half-sweep: times the
// finest-level red half-sweep (the batched kernel, one task) for every
// power-of-two width W up to default_lanes with at most 8 samples per lane.
// lanes/us receive up to `cap` candidates, *ncand their number, *best the
// fastest width.  Uses the context's correction buffers as scratch.
int smg_tune_lanes(smg_ctx* C, int cap, int* lanes, double* us, int* ncand, int* best) {
  if (!C || cap < 1 || !lanes || !us || !ncand || !best) return SMG_EINVAL;
  const bool f32 = C->desc.precision == SMG_F32;
  const int N = C->N, top = default_lanes(N, C->desc.precision);
  const int vw = vec2_ctx(C->desc.precision, N) ? 2 : 1;
  int k = 0;
  double best_us = 1e300;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipMemsetAsync(C->flag, 0, sizeof(int), C->stream));
  auto run = [&](auto tag, int W) -> int {
    using T = decltype(tag);
    Level<T>* Lp;
    T* xs;
    T* fs;
    if constexpr (std::is_same<T, float>::value) { Lp = &C->L32[0]; xs = C->L32[0].x; fs = C->L32[0].f; }
    else { Lp = &C->L64[0]; xs = C->w; fs = C->rr; }
    Level<T>& L = *Lp;
    TRY(fill<T>(C, xs, C->len0, T(0)));
    TRY(fill<T>(C, fs, C->len0, T(1)));
    BTask<T> t{};
    t.inst = 0; t.W = W; t.L = args(L, N); t.nitems = colour_count(L.n, 0); t.block0 = 0;
    t.x = xs; t.f = fs;
    const int per = kBlock / W, nbk = (t.nitems + per - 1) / per;
    HIP_TRY(hipMemcpyAsync(C->mdp, &t, sizeof(t), hipMemcpyHostToDevice, C->stream));
    const int jm = samples_per_lane(N, W, vw);
    auto launch = [&]() {
      jmv_dispatch<T>(jm, vw, [&](auto Jc, auto Vc) {
        constexpr int JM = decltype(Jc)::value, VW = halfsweep_vw(decltype(Vc)::value, JM);
        hipLaunchKernelGGL((kb_halfsweep<T, JM, kPlain, VW>), dim3(nbk), dim3(kBlock), 0, C->stream,
                           (const BTask<T>*)C->mdp, 1, 0, (const int*)C->flag);
      });
    };
    for (int r = 0; r < 3; ++r) launch();
    HIP_TRY(hipEventRecord(e0, C->stream));
    const int reps = 20;
    for (int r = 0; r < reps; ++r) launch();
    HIP_TRY(hipEventRecord(e1, C->stream));
    HIP_TRY(hipEventSynchronize(e1));
    LAUNCH_CHECK();
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    const double u = 1e3 * ms / reps;
    lanes[k] = W; us[k] = u; ++k;
    if (u < best_us) { best_us = u; *best = W; }
    return SMG_OK;
  };
  for (int W = 64; W >= 1 && k < cap; W >>= 1) {
    if (W > top || samples_per_lane(N, W, vw) > 8) continue;
    const int rc = f32 ? run(float(0), W) : run(double(0), W);
    if (rc != SMG_OK) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); return rc; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ncand = k;
  return k > 0 ? SMG_OK : SMG_EINVAL;
}

}  // extern "C"

// ============================================================ network glue
extern "C" {

int smg_net_features(smg_ctx* C, const double* f, int H, float* feat) {
  if (!C || !f || !feat || H < C->L64[0].n) return SMG_EINVAL;
  const Level<double>& L = C->L64[0];
  std::vector<double> c0(1);
  HIP_TRY(hipMemcpy(c0.data(), L.c, sizeof(double), hipMemcpyDeviceToHost));
  const double h = 1.0 / (L.n + 1);
  const float lognu4 = (float)(std::log10(L.g / (h * h)) + 4.0);
  hipLaunchKernelGGL(k_net_features, dim3((H * H + 255) / 256), dim3(256), 0, C->stream, L.n, C->N, H,
                     (const double*)L.kx, (const double*)L.ky, f, 1.0 / c0[0], lognu4, feat);
  LAUNCH_CHECK();
  return SMG_OK;
}

int smg_net_targets(smg_ctx* C, const double* x, int H, const float* norm, float* tgt) {
  if (!C || !x || !norm || !tgt || H < C->L64[0].n) return SMG_EINVAL;
  NetNorm nm;
  for (int c = 0; c < 3; ++c) { nm.mean[c] = norm[c]; nm.std[c] = norm[3 + c]; }
  hipLaunchKernelGGL(k_net_targets, dim3((H * H + 255) / 256), dim3(256), 0, C->stream, C->L64[0].n, C->N, H, x,
                     nm, tgt);
  LAUNCH_CHECK();
  return SMG_OK;
}

int smg_net_lift(smg_ctx* C, const float* pred, int H, const float* norm, double* x0) {
  if (!C || !pred || !norm || !x0 || H < C->L64[0].n) return SMG_EINVAL;
  NetNorm nm;
  for (int c = 0; c < 3; ++c) { nm.mean[c] = norm[c]; nm.std[c] = norm[3 + c]; }
  const size_t tot = (size_t)C->L64[0].n * C->L64[0].n * C->N;
  hipLaunchKernelGGL(k_net_lift, dim3(grid_for(tot)), dim3(kBlock), 0, C->stream, C->L64[0].n, C->N, H, pred, nm,
                     x0);
  LAUNCH_CHECK();
  return SMG_OK;
}

}  // extern "C"
