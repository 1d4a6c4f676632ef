// Contractions of several vertex tensors (Sec. 3.1 "Tensor contractions": amplitudes with many
// vertices contract vertex tensors over the intertwiners of their bulk edges; Sec. 3.3 "Tensor
// contractions on CPU and GPU"; the Delta_3 amplitude of Sec. 4.2).
//
//   vertices:  F = sum_i A(i1..i5) B(i1..i5)                                  (real)
//   trailing:  T(i1..i_{5-m}) = sum over the last m intertwiners of A psi_1 .. psi_m
//   delta3:    F = (-1)^x (2x+1) sum_{k1,k2,k3} (-1)^{k1+k2+k3} TA[k1][k2] TB[k3][k1] TC[k2][k3]
//
// All three read their operands once and are bound by memory bandwidth (or, for delta3 on its
// small matrices, by launch latency).  Sums run in a fixed order: every block sums a fixed
// contiguous range with a fixed tree, and partial sums are added in block order, so results
// are bitwise repeatable.
#include "eprl_internal.hpp"

namespace eprl {

namespace {

struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx load_c(const double *p, int64_t i) { return {p[2 * i], p[2 * i + 1]}; }

constexpr int kDotThreads = 256;
constexpr int kTrailThreads = 64;

template <typename T>
__device__ T tree_sum(T v, T *sh, T (*add)(T, T)) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w) sh[tid] = add(sh[tid], sh[tid + w]);
    __syncthreads();
  }
  T r = sh[0];
  __syncthreads();
  return r;
}

__device__ double dadd(double a, double b) { return a + b; }
__device__ cplx cadd_f(cplx a, cplx b) { return cadd(a, b); }

// Block b sums A * B over [b * per, (b + 1) * per).
__global__ __launch_bounds__(kDotThreads) void vertices_partial_kernel(const double *A, const double *B,
                                                                       int64_t total, int nblocks,
                                                                       double *partial) {
  __shared__ double sh[kDotThreads];
  const int64_t per = (total + nblocks - 1) / nblocks;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = b0 + per < total ? b0 + per : total;
  double acc = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) acc += A[i] * B[i];
  const double s = tree_sum<double>(acc, sh, dadd);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kDotThreads) void vertices_final_kernel(const double *partial, int nblocks,
                                                                     double *F) {
  __shared__ double sh[kDotThreads];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) acc += partial[b];
  const double s = tree_sum<double>(acc, sh, dadd);
  if (threadIdx.x == 0) F[0] = s;
}

// Block (lead, split): the entries [split * per, (split + 1) * per) of the contiguous trailing
// block of row `lead`, each times the product of the m vectors at its trailing indices.
__global__ __launch_bounds__(kTrailThreads) void trailing_kernel(TrailParams tp) {
  __shared__ cplx sh[kTrailThreads];
  const int64_t lead = blockIdx.x / tp.nsplit;
  const int split = (int)(blockIdx.x % tp.nsplit);
  const int64_t per = (tp.S + tp.nsplit - 1) / tp.nsplit;
  const int64_t s0 = (int64_t)split * per;
  const int64_t s1 = s0 + per < tp.S ? s0 + per : tp.S;
  const double *row = tp.A + lead * tp.S;
  cplx acc{0.0, 0.0};
  for (int64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
    int64_t r = s;
    cplx w{row[s], 0.0};
    for (int q = tp.m - 1; q >= 0; --q) {
      const int i = (int)(r % tp.n[q]);
      r /= tp.n[q];
      w = cmul(w, load_c(tp.psi[q], i));
    }
    acc = cadd(acc, w);
  }
  const cplx v = tree_sum<cplx>(acc, sh, cadd_f);
  if (threadIdx.x == 0) {
    double *dst = tp.nsplit == 1 ? tp.T + 2 * lead : tp.partial + 2 * (lead * tp.nsplit + split);
    dst[0] = v.re;
    dst[1] = v.im;
  }
}

// One thread per leading row: its nsplit partial sums in order.
__global__ void trailing_final_kernel(TrailParams tp, int64_t nlead) {
  const int64_t lead = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (lead >= nlead) return;
  cplx acc{0.0, 0.0};
  for (int q = 0; q < tp.nsplit; ++q) acc = cadd(acc, load_c(tp.partial, lead * tp.nsplit + q));
  tp.T[2 * lead] = acc.re;
  tp.T[2 * lead + 1] = acc.im;
}

// One block: thread t takes the (k1, k2) pairs t, t + blockDim, ... and sums over k3.
__global__ __launch_bounds__(kDotThreads) void delta3_kernel(int n, int two_klo, int two_x,
                                                             const double *TA, const double *TB,
                                                             const double *TC, double *F) {
  __shared__ cplx sh[kDotThreads];
  cplx acc{0.0, 0.0};
  for (int p = threadIdx.x; p < n * n; p += blockDim.x) {
    const int k1 = p / n, k2 = p % n;
    cplx inner{0.0, 0.0};
    for (int k3 = 0; k3 < n; ++k3) {
      cplx t = cmul(load_c(TB, (int64_t)k3 * n + k1), load_c(TC, (int64_t)k2 * n + k3));
      if (((two_klo >> 1) + k3) & 1) t = {-t.re, -t.im};
      inner = cadd(inner, t);
    }
    cplx v = cmul(load_c(TA, (int64_t)k1 * n + k2), inner);
    if ((2 * (two_klo >> 1) + k1 + k2) & 1) v = {-v.re, -v.im};
    acc = cadd(acc, v);
  }
  const cplx s = tree_sum<cplx>(acc, sh, cadd_f);
  if (threadIdx.x == 0) {
    const double pre = (((two_x >> 1) & 1) ? -1.0 : 1.0) * (double)(two_x + 1);
    F[0] = pre * s.re;
    F[1] = pre * s.im;
  }
}

}  // namespace

hipError_t launch_contract_vertices(const double *A, const double *B, int64_t total, int nblocks,
                                    double *partial, double *F, hipStream_t s) {
  vertices_partial_kernel<<<nblocks, kDotThreads, 0, s>>>(A, B, total, nblocks, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  vertices_final_kernel<<<1, kDotThreads, 0, s>>>(partial, nblocks, F);
  return hipGetLastError();
}

int trailing_splits(int64_t nlead, int64_t S) {
  // About 16 entries per thread of a block, at most 64 blocks per row.
  int64_t ns = (S + 16 * kTrailThreads - 1) / (16 * kTrailThreads);
  if (ns > 64) ns = 64;
  (void)nlead;
  return ns < 1 ? 1 : (int)ns;
}

hipError_t launch_contract_trailing(const TrailParams &tp, int64_t nlead, hipStream_t s) {
  trailing_kernel<<<(unsigned)(nlead * tp.nsplit), kTrailThreads, 0, s>>>(tp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || tp.nsplit == 1) return e;
  trailing_final_kernel<<<(unsigned)((nlead + 255) / 256), 256, 0, s>>>(tp, nlead);
  return hipGetLastError();
}

hipError_t launch_delta3(int n, int two_klo, int two_x, const double *TA, const double *TB,
                         const double *TC, double *F, hipStream_t s) {
  delta3_kernel<<<1, kDotThreads, 0, s>>>(n, two_klo, two_x, TA, TB, TC, F);
  return hipGetLastError();
}

}  // namespace eprl
