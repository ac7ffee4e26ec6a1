// batch.h -- batched kernels: one launch runs one phase of the refinement step
// for many independent instances (different n, N, nu) at once.  A launch is a
// list of tasks, one per instance, each owning a contiguous range of (logical)
// blocks; a block finds its task by binary search over the task offsets.
// Instances whose residual already met the tolerance are retired by a device
// flag and their blocks exit at once.  The per-node arithmetic is the same
// device code as the single-instance kernels.
#pragma once
#include "coarse.h"
#include "common.h"
#include "residual.h"
#include "smoother.h"
#include "transfer.h"

namespace smg {

template <typename T>
struct BTask {
  int inst;            // instance index (retire flag, statistics)
  int W;               // lanes per node of this instance
  int nitems;          // node groups (or samples, or elements) of this task
  int block0;          // first logical block of the task
  LevelArgs<T> L;      // level operator
  T* x;                // level iterate / coarsest solution
  const T* f;          // level right-hand side
  T* a;                // phase output: coarse right-hand side
  const T* b;          // phase input: coarse correction
  int m;               // coarsest unknowns per field
  const double* Ainv;  // coarsest factors (transposed storage) and scratch
  const double* Sinv;
  double* ds;
  const double* c64;   // coarsest diagonal blocks in FP64
  const double* d64;
  const double* e64;
  const double* mk64;  // coarsest control mask in FP64
};

// FP64 outer residual of one instance, rounded into the reduced-precision
// right-hand side of its correction cycle; the task also owns a range of
// norm partials (one triple per block).  With FP32 corrections (w set) the
// update of the previous step is fused in: after c correction cycles the
// iterate lives in x (c even) or w (c odd), and the pass forms it as the other
// buffer plus the pending correction d.
template <typename TO>
struct BOuterTask {
  int inst, W, nitems, block0;
  LevelArgs<double> L;
  double* x;
  const double* f;
  TO* out;
  double* w;           // second iterate buffer, or null (separate update pass)
  const TO* d;         // pending correction of the last cycle
};

template <typename TD>
struct BAddTask {
  int inst, block0, nblk;
  size_t len;
  double* x;
  const TD* d;
};

struct BCheck {
  int pb0, pnb;        // partial-block range of the instance's outer residual
  double fnorm;        // ||f|| of the instance
};

template <typename Task>
__device__ __forceinline__ int find_task(const Task* __restrict__ tasks, int ntasks, int b) {
  __shared__ int s_idx;
  if (threadIdx.x == 0) {
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tasks[mid].block0 <= b) lo = mid; else hi = mid - 1;
    }
    s_idx = lo;
  }
  __syncthreads();
  return s_idx;
}

template <typename T, int JM, int SRC, int VW>
__global__ __launch_bounds__(kBlock) void kb_halfsweep(const BTask<T>* __restrict__ tasks, int ntasks, int colour,
                                                       const int* __restrict__ done) {
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const BTask<T>& t = tasks[find_task(tasks, ntasks, b)];
  if (done[t.inst]) return;
  const int W = t.W;
  const int lane = threadIdx.x & (W - 1);
  const int slot = (b - t.block0) * (kBlock / W) + threadIdx.x / W;
  if (slot >= t.nitems) return;
  halfsweep_node<T, JM, SRC, VW>(t.L, t.x, t.f, colour, T(1), slot, lane, W, t.b);
}

// coarse right-hand side t.a = R (t.f - S t.x) of level t.L (fine residual never stored)
template <typename T, int JM, int VW>
__global__ __launch_bounds__(kBlock) void kb_residual_restrict(const BTask<T>* __restrict__ tasks, int ntasks,
                                                               const int* __restrict__ done) {
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const BTask<T>& t = tasks[find_task(tasks, ntasks, b)];
  if (done[t.inst]) return;
  const int W = t.W;
  const int lane = threadIdx.x & (W - 1);
  const int slot = (b - t.block0) * (kBlock / W) + threadIdx.x / W;
  if (slot >= t.nitems) return;
  residual_restrict_node<T, JM, VW>(t.L, t.x, t.f, t.a, slot, lane, W, coarse_strip(t.L.strip));
}

// coarsest direct solve, one block per (instance, sample)
template <typename T>
__global__ __launch_bounds__(64) void kb_coarse1(const BTask<T>* __restrict__ tasks, int ntasks,
                                                 const int* __restrict__ done) {
  const int b = blockIdx.x;
  const BTask<T>& t = tasks[find_task(tasks, ntasks, b)];
  if (done[t.inst]) return;
  coarse_phase1_sample<T>(b - t.block0, t.m, t.L.N, t.Ainv, t.c64, t.d64, t.mk64, t.f, t.ds);
}

template <typename T>
__global__ __launch_bounds__(64) void kb_coarse2(const BTask<T>* __restrict__ tasks, int ntasks,
                                                 const int* __restrict__ done) {
  const int b = blockIdx.x;
  const BTask<T>& t = tasks[find_task(tasks, ntasks, b)];
  if (done[t.inst]) return;
  coarse_phase2_sample<T>(b - t.block0, t.m, t.L.N, t.Ainv, t.Sinv, t.c64, t.e64, t.mk64, t.f, t.ds, t.x);
}

// FP64 outer residual, rounded into t.out; per-block squared norms into partials.
// VW samples per access (2: every instance's N even).
template <typename TO, int JM, int VW>
__global__ __launch_bounds__(kBlock) void kb_outer_residual(const BOuterTask<TO>* __restrict__ tasks, int ntasks,
                                                            const int* __restrict__ done,
                                                            const int* __restrict__ iters,
                                                            double* __restrict__ partials) {
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const BOuterTask<TO>& t = tasks[find_task(tasks, ntasks, b)];
  if (done[t.inst]) return;
  const int W = t.W;
  const int lane = threadIdx.x & (W - 1);
  const int slot = (b - t.block0) * (kBlock / W) + threadIdx.x / W;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int c = t.w ? iters[t.inst] : 0;
  if (slot < t.nitems) {
    if constexpr (std::is_same<TO, float>::value) {
      if (c > 0) {
        double* cur = (c & 1) ? t.w : t.x;
        const double* prev = (c & 1) ? t.x : t.w;
        residual_add_node<JM, VW>(t.L, prev, t.d, cur, t.f, t.out, slot, lane, W, acc);
      } else {
        residual_node<double, double, TO, JM, VW>(t.L, t.x, t.f, t.out, 0, slot, lane, W, acc);
      }
    } else {
      residual_node<double, double, TO, JM, VW>(t.L, t.x, t.f, t.out, 0, slot, lane, W, acc);
    }
  }
  double r3[3] = {acc[0], acc[1], acc[2]};
  block_sum<3>(r3);
  if (threadIdx.x == 0) {
    partials[3 * (size_t)b + 0] = r3[0];
    partials[3 * (size_t)b + 1] = r3[1];
    partials[3 * (size_t)b + 2] = r3[2];
  }
}

// One block per instance: relative residual from the partials; retire the
// instance (flag, device wall-clock stamp) once it meets tol, otherwise count
// the correction cycle this step is about to apply (at most maxit).
__global__ __launch_bounds__(kBlock) void kb_check(const BCheck* __restrict__ chk, const double* __restrict__ partials,
                                                   double tol, int maxit, int* __restrict__ done,
                                                   int* __restrict__ iters, double* __restrict__ relres,
                                                   long long* __restrict__ tdone) {
  const int i = blockIdx.x;
  if (done[i]) return;
  double acc[1] = {0.0};
  const BCheck c = chk[i];
  for (int q = threadIdx.x; q < c.pnb; q += kBlock) {
    const double* p = partials + 3 * (size_t)(c.pb0 + q);
    acc[0] += (p[0] + p[1]) + p[2];
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) {
    const double rel = sqrt(acc[0]) / c.fnorm;
    relres[i] = rel;
    if (!(rel > tol)) {            // converged (a NaN also retires: flagged by relres)
      done[i] = 1;
      tdone[i] = wall_clock64();
    } else if (iters[i] >= maxit) {
      done[i] = 2;                 // iteration limit
      tdone[i] = wall_clock64();
    } else {
      iters[i] += 1;
    }
  }
}

template <typename TD>
__global__ __launch_bounds__(kBlock) void kb_add(const BAddTask<TD>* __restrict__ tasks, int ntasks,
                                                 const int* __restrict__ done) {
  const int b = blockIdx.x;
  const BAddTask<TD>& t = tasks[find_task(tasks, ntasks, b)];
  if (done[t.inst]) return;
  for (size_t i = (size_t)(b - t.block0) * kBlock + threadIdx.x; i < t.len; i += (size_t)t.nblk * kBlock)
    t.x[i] += (double)t.d[i];
}

// device wall clock at the start of a batched solve
__global__ void kb_stamp(long long* __restrict__ t0) {
  if (threadIdx.x == 0) *t0 = wall_clock64();
}

}  // namespace smg
