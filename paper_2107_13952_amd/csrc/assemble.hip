// Vertex-tensor assembly: steps 5-6 of the framed algorithm of Sec. 3.1.
//
// For every shell l = (l23, l24, l25, l34, l35, l45) (one element of the (dl+1)^6 grid):
//   (i)   W(i1, k2, k3, k4, k5) = (-1)^R sum_x (2x+1) S1 S2 S3 S4 S5       (eq. (15j))
//   (ii)  the booster blocks M_e = (2k_e+1) B_e(l_e) of the four edges     (eq. (vertex-ampl))
//   (iii) T = W x_{k5} M5 x_{k4} M4 x_{k3} M3 x_{k2} M2, one mode at a time
//   (iv)  A += T
// Then A *= prod_e sqrt(2 i_e + 1) (eq. (vertex-ampl)) in the reduction kernel.
//
// Work decomposition on the GPU (one workgroup per (chunk of shells, i1)):
//  * the shell header (k ranges, booster offsets, phase) is derived from the shell index in
//    registers: shell enumeration and triangle pruning happen inside the kernel;
//  * the four booster blocks of the shell, weighted by (2k+1)(-1)^{k - k_lo}, are staged in
//    LDS (zero-padded to D x D);
//  * k2 is processed in chunks of KC values.  Step A builds a row W(i1, k2, k3, k4, :) in
//    registers (sum over the x values allowed by the triads of that row, 6j values read from
//    the 6j tables) and multiplies it by M5 at once (mode k5), writing T1(k2, k3, k4, i5) to
//    LDS; steps B and C apply M4 and M3 through LDS; step D applies M2 and accumulates into
//    A(i1, i2, i3, i4, i5), which stays in registers across all shells of the chunk;
//  * the per-chunk partial tensors are summed in a fixed order by the reduction kernel, so
//    the result does not depend on scheduling (no floating-point atomics).
#include "eprl_internal.hpp"

namespace eprl {

namespace {

struct ShellHeader {
  int o[6];
  int t[4];        // booster triple index per edge 2..5
  int klo[4];      // lowest two_k of k2..k5
  int kn[4];       // sizes of k2..k5
  int l[10];       // virtual spins of all ten links
  double sign;     // (-1)^{R0}, R0 = R at the lowest intertwiners
  bool live;
};

__device__ __forceinline__ ShellHeader shell_header(const VertexParams &vp, int64_t s) {
  ShellHeader h;
  const int nd = vp.nd;
  int64_t r = s;
  for (int q = 5; q >= 0; --q) {
    h.o[q] = (int)(r % nd);
    r /= nd;
  }
  h.t[0] = (h.o[0] * nd + h.o[1]) * nd + h.o[2];  // e2: (l23, l24, l25)
  h.t[1] = (h.o[3] * nd + h.o[4]) * nd + h.o[0];  // e3: (l34, l35, l23)
  h.t[2] = (h.o[5] * nd + h.o[1]) * nd + h.o[3];  // e4: (l45, l24, l34)
  h.t[3] = (h.o[2] * nd + h.o[4]) * nd + h.o[5];  // e5: (l25, l35, l45)
  const int nd3 = nd * nd * nd;
  h.live = true;
  for (int e = 0; e < 4; ++e) {
    h.klo[e] = vp.kr[(e * nd3 + h.t[e]) * 2 + 0];
    h.kn[e] = vp.kr[(e * nd3 + h.t[e]) * 2 + 1];
    h.live = h.live && h.kn[e] > 0;
  }
  for (int q = 0; q < 4; ++q) h.l[q] = vp.two_j[q];
  for (int q = 0; q < 6; ++q) h.l[4 + q] = vp.two_j[4 + q] + 2 * h.o[q];
  int base = vp.i_lo2[0];
  for (int q = 0; q < 10; ++q) base += h.l[q];
  for (int e = 0; e < 4; ++e) base += h.klo[e];
  h.sign = ((base / 2) & 1) ? -1.0 : 1.0;
  return h;
}

__device__ __forceinline__ int iabs(int v) { return v < 0 ? -v : v; }
__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }
__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

// W(i1, k2, k3, k4, k5) for k5 = 0..D-1 (zero beyond the k5 range), including (-1)^R.
// n1, k2, k3, k4 are indices into their ranges.
template <int D>
__device__ __forceinline__ void w_row(const VertexParams &vp, const ShellHeader &h, int n1, int k2,
                                      int k3, int k4, double (&w)[D]) {
#pragma unroll
  for (int q = 0; q < D; ++q) w[q] = 0.0;
  const int two_i1 = vp.i_lo2[0] + 2 * n1;
  const int two_k2 = h.klo[0] + 2 * k2, two_k3 = h.klo[1] + 2 * k3, two_k4 = h.klo[2] + 2 * k4;
  const int l24 = h.l[L24], l25 = h.l[L25], l35 = h.l[L35], j13 = h.l[L13];
  // x closes (i1 l25 x), (j13 k2 x), (l24 k3 x), (l35 k4 x); (k5 j14 x) is handled by the
  // zeros of the first table.
  int lo = imax(imax(iabs(two_i1 - l25), iabs(j13 - two_k2)),
                imax(iabs(l24 - two_k3), iabs(l35 - two_k4)));
  int hi = imin(imin(two_i1 + l25, j13 + two_k2), imin(l24 + two_k3, l35 + two_k4));
  lo = imax(lo, vp.X_lo2);
  hi = imin(hi, vp.X_lo2 + 2 * (vp.NX - 1));
  if (lo > hi) return;
  const int nd = vp.nd, NX = vp.NX;
  const int n_i1 = vp.i_n[0];
  const int nK2 = vp.K_n[0], nK3 = vp.K_n[1], nK4 = vp.K_n[2], nK5 = vp.K_n[3];
  const int k2g = (two_k2 - vp.K_lo2[0]) / 2, k3g = (two_k3 - vp.K_lo2[1]) / 2;
  const int k4g = (two_k4 - vp.K_lo2[2]) / 2, k5g0 = (h.klo[3] - vp.K_lo2[3]) / 2;
  const int64_t b3 = ((((int64_t)h.o[1] * nd + h.o[3]) * nd + h.o[4]) * nK4 + k4g) * nK3 * NX +
                     (int64_t)k3g * NX;
  const int64_t b4 = ((((int64_t)h.o[0] * nd + h.o[1]) * nK3 + k3g) * nK2 + k2g) * NX;
  const int64_t b5 = (((int64_t)h.o[2] * nK2 + k2g) * n_i1 + n1) * NX;
  const int64_t b1 = (((int64_t)h.o[2] * n_i1 + n1) * nK5 + k5g0) * NX;
  const int64_t b2 = ((((int64_t)h.o[4] * nd + h.o[5]) * nK5 + k5g0) * nK4 + k4g) * NX;
  const int nk5 = h.kn[3];
  const double sgn = (n1 & 1) ? -h.sign : h.sign;
  for (int x2 = lo; x2 <= hi; x2 += 2) {
    const int xg = (x2 - vp.X_lo2) / 2;
    const double r = vp.T3[b3 + xg] * vp.T4[b4 + xg] * vp.T5[b5 + xg] * (double)(x2 + 1);
    if (r == 0.0) continue;
#pragma unroll
    for (int k5 = 0; k5 < D; ++k5) {
      if (k5 < nk5) {
        w[k5] += vp.T1[b1 + (int64_t)k5 * NX + xg] * vp.T2[b2 + (int64_t)k5 * nK4 * NX + xg] * r;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < D; ++q) w[q] *= sgn;
}

// Stage the weighted booster blocks M_e(i, k) = (2k+1) (-1)^{k - k_lo} B_e(i, k) of a shell.
template <int D>
__device__ __forceinline__ void stage_boosters(const VertexParams &vp, const ShellHeader &h,
                                               double *Ms, int tid, int nt) {
  const int nd3 = vp.nd * vp.nd * vp.nd;
  for (int idx = tid; idx < 4 * D * D; idx += nt) {
    const int e = idx / (D * D), i = (idx / D) % D, k = idx % D;
    double v = 0.0;
    if (i < vp.i_n[e + 1] && k < h.kn[e]) {
      const int64_t off = vp.boff[e * nd3 + h.t[e]];
      v = vp.B[off + (int64_t)i * h.kn[e] + k] * (double)(h.klo[e] + 2 * k + 1);
      if (k & 1) v = -v;
    }
    Ms[idx] = v;
  }
}

template <int D, int KC, int NT, int OS, int I2S>
__global__ __launch_bounds__(NT) void assemble_kernel(VertexParams vp) {
  // Each thread owns NP positions (i3, i4, i5) of the accumulator and I2S values of i2.
  constexpr int NP = D * D * D / NT;
  __shared__ double Ms[4 * D * D];
  __shared__ double buf1[KC * D * D * D];
  __shared__ double buf2[KC * D * D * D];
  const int tid = threadIdx.x;
  const int chunk = blockIdx.x, n1 = blockIdx.y, i2base = blockIdx.z * I2S;
  const int d2 = vp.i_n[1], d3 = vp.i_n[2], d4 = vp.i_n[3], d5 = vp.i_n[4];
  double acc[NP][I2S];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int j = 0; j < I2S; ++j) acc[p][j] = 0.0;

  const int64_t s0 = vp.shell_begin + (int64_t)chunk * vp.chunk;
  const int64_t s1 = s0 + vp.chunk < vp.shell_end ? s0 + vp.chunk : vp.shell_end;
  for (int64_t s = s0; s < s1; ++s) {
    const ShellHeader h = shell_header(vp, s);
    if (!h.live) continue;
    stage_boosters<D>(vp, h, Ms, tid, NT);
    __syncthreads();
    const int dk2 = h.kn[0], dk3 = h.kn[1], dk4 = h.kn[2];
    for (int k2c = 0; k2c < dk2; k2c += KC) {
      const int kc = dk2 - k2c < KC ? dk2 - k2c : KC;
      // Step A: W rows and mode k5 -> buf1[kk][k3][k4][i5]
      for (int u = tid; u < kc * dk3 * dk4 * OS; u += NT) {
        const int q = u % OS, row = u / OS;
        const int k4 = row % dk4, k3 = (row / dk4) % dk3, kk = row / (dk4 * dk3);
        double w[D];
        w_row<D>(vp, h, n1, k2c + kk, k3, k4, w);
        const double *m5 = Ms + 3 * D * D;
        double *dst = buf1 + ((kk * D + k3) * D + k4) * D;
        for (int c = 0; c < D / OS; ++c) {
          const int i5 = q + c * OS;
          double t = 0.0;
#pragma unroll
          for (int k5 = 0; k5 < D; ++k5) t += m5[i5 * D + k5] * w[k5];
          dst[i5] = t;
        }
      }
      __syncthreads();
      // Step B: mode k4 -> buf2[kk][k3][i4][i5]
      for (int u = tid; u < kc * dk3 * d5 * OS; u += NT) {
        const int q = u % OS, row = u / OS;
        const int i5 = row % d5, k3 = (row / d5) % dk3, kk = row / (d5 * dk3);
        const double *m4 = Ms + 2 * D * D;
        const double *src = buf1 + (kk * D + k3) * D * D + i5;
        double v[D];
#pragma unroll
        for (int k4 = 0; k4 < D; ++k4) v[k4] = k4 < dk4 ? src[k4 * D] : 0.0;
        double *dst = buf2 + (kk * D + k3) * D * D + i5;
        for (int c = 0; c < D / OS; ++c) {
          const int i4 = q + c * OS;
          double t = 0.0;
#pragma unroll
          for (int k4 = 0; k4 < D; ++k4) t += m4[i4 * D + k4] * v[k4];
          dst[i4 * D] = t;
        }
      }
      __syncthreads();
      // Step C: mode k3 -> buf1[kk][i3][i4][i5]
      for (int u = tid; u < kc * d4 * d5 * OS; u += NT) {
        const int q = u % OS, row = u / OS;
        const int i5 = row % d5, i4 = (row / d5) % d4, kk = row / (d5 * d4);
        const double *m3 = Ms + 1 * D * D;
        const double *src = buf2 + kk * D * D * D + i4 * D + i5;
        double v[D];
#pragma unroll
        for (int k3 = 0; k3 < D; ++k3) v[k3] = k3 < dk3 ? src[k3 * D * D] : 0.0;
        double *dst = buf1 + kk * D * D * D + i4 * D + i5;
        for (int c = 0; c < D / OS; ++c) {
          const int i3 = q + c * OS;
          double t = 0.0;
#pragma unroll
          for (int k3 = 0; k3 < D; ++k3) t += m3[i3 * D + k3] * v[k3];
          dst[i3 * D * D] = t;
        }
      }
      __syncthreads();
      // Step D: mode k2 and accumulation into the register-resident A(i1, i2, ...).  Padded
      // rows of M2 are zero, so positions and i2 values outside the ranges stay zero.
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const int pos = tid + p * NT;
        double v[KC];
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) v[kk] = kk < kc ? buf1[kk * D * D * D + pos] : 0.0;
#pragma unroll
        for (int j = 0; j < I2S; ++j) {
          const int i2 = i2base + j;
          double t = acc[p][j];
#pragma unroll
          for (int kk = 0; kk < KC; ++kk) {
            const int k2 = k2c + kk;
            t += (kk < kc ? Ms[i2 * D + k2] : 0.0) * v[kk];
          }
          acc[p][j] = t;
        }
      }
      __syncthreads();
    }
  }
  // Flush this chunk's partial A(i1, i2-group, ...).
  const int64_t slice = (int64_t)d2 * d3 * d4 * d5;
  double *out = vp.partial + ((int64_t)chunk * vp.i_n[0] + n1) * slice;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int pos = tid + p * NT;
    const int i5 = pos % D, i4 = (pos / D) % D, i3 = pos / (D * D);
    if (i3 < d3 && i4 < d4 && i5 < d5) {
#pragma unroll
      for (int j = 0; j < I2S; ++j) {
        const int i2 = i2base + j;
        if (i2 < d2) out[((i2 * d3 + i3) * d4 + i4) * d5 + i5] = acc[p][j];
      }
    }
  }
}

// A = (accumulate ? A : 0) + prod_e sqrt(2 i_e + 1) * sum_chunks partial.  A workgroup of
// RW wavefronts owns 64 consecutive entries; wavefront w sums the w-th of RW contiguous runs of
// chunks in chunk order, then the RW run sums are added in run order: a fixed order for a given
// chunk count, with enough loads in flight to stream the partials at HBM rate.
constexpr int RW = 16;
__global__ __launch_bounds__(64 * RW) void reduce_kernel(ReduceParams rp) {
  __shared__ double run[RW][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t idx = (int64_t)blockIdx.x * 64 + lane;
  const bool in = idx < rp.a_size;
  const int c0 = (int)((int64_t)rp.nchunk * w / RW), c1 = (int)((int64_t)rp.nchunk * (w + 1) / RW);
  double s = 0.0;
  if (in) {
    const double *p = rp.partial + idx;
    int c = c0;
    for (; c + 8 <= c1; c += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = p[(int64_t)(c + q) * rp.a_size];
#pragma unroll
      for (int q = 0; q < 8; ++q) s += v[q];
    }
    for (; c < c1; ++c) s += p[(int64_t)c * rp.a_size];
  }
  run[w][lane] = s;
  __syncthreads();
  if (w != 0 || !in) return;
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < RW; ++q) t += run[q][lane];
  int64_t r = idx;
  double norm = 1.0;
  for (int e = 4; e >= 0; --e) {
    const int n = (int)(r % rp.i_n[e]);
    r /= rp.i_n[e];
    norm *= __builtin_sqrt((double)(rp.i_lo2[e] + 2 * n + 1));
  }
  const double v = t * norm;
  rp.A[idx] = rp.accumulate ? rp.A[idx] + v : v;
}

template <int D>
__global__ void shell_fifteenj_kernel(VertexParams vp, int64_t shell, double *W) {
  const ShellHeader h = shell_header(vp, shell);
  if (!h.live) return;
  const int dk2 = h.kn[0], dk3 = h.kn[1], dk4 = h.kn[2], dk5 = h.kn[3];
  const int rows = vp.i_n[0] * dk2 * dk3 * dk4;
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= rows) return;
  const int k4 = u % dk4, k3 = (u / dk4) % dk3, k2 = (u / (dk4 * dk3)) % dk2, n1 = u / (dk4 * dk3 * dk2);
  double w[D];
  w_row<D>(vp, h, n1, k2, k3, k4, w);
  // The assembly folds (-1)^{k - k_lo} of every virtual intertwiner into the booster blocks;
  // restore it here so that W carries the full (-1)^R.
  const double s = ((k2 + k3 + k4) & 1) ? -1.0 : 1.0;
  for (int k5 = 0; k5 < dk5; ++k5) W[(int64_t)u * dk5 + k5] = (k5 & 1) ? -s * w[k5] : s * w[k5];
}

// SU(2) BF vertex (Sec. 3.2 "BF vertex (15j) tensors"; the Delta l = 0, no-booster limit of
// eq. (vertex-ampl)): A(i1..i5) = prod_e sqrt(2 i_e + 1) {15j}(j; i1..i5).  At dl = 0 every
// virtual range k_e is the boundary range i_e and the tables hold the 6j symbols of the single
// shell, so an entry is the x sum of w_row for one k5, with the phase (-1)^R restored in full.
// One thread per entry: no register tile, so any intertwiner dimension is handled.
__global__ void bf_vertex_kernel(VertexParams vp, double *A, int64_t total) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= total) return;
  const ShellHeader h = shell_header(vp, 0);
  int64_t r = u;
  const int k5 = (int)(r % h.kn[3]); r /= h.kn[3];
  const int k4 = (int)(r % h.kn[2]); r /= h.kn[2];
  const int k3 = (int)(r % h.kn[1]); r /= h.kn[1];
  const int k2 = (int)(r % h.kn[0]); r /= h.kn[0];
  const int n1 = (int)r;
  const int two_i1 = vp.i_lo2[0] + 2 * n1;
  const int two_k2 = h.klo[0] + 2 * k2, two_k3 = h.klo[1] + 2 * k3, two_k4 = h.klo[2] + 2 * k4;
  const int two_k5 = h.klo[3] + 2 * k5;
  const int l24 = h.l[L24], l25 = h.l[L25], l35 = h.l[L35], j13 = h.l[L13], j14 = h.l[L14];
  // x closes the five triads (i1 l25 x), (k5 j14 x), (l35 k4 x), (l24 k3 x), (j13 k2 x).
  int lo = imax(imax(iabs(two_i1 - l25), iabs(j13 - two_k2)),
                imax(imax(iabs(l24 - two_k3), iabs(l35 - two_k4)), iabs(j14 - two_k5)));
  int hi = imin(imin(two_i1 + l25, j13 + two_k2),
                imin(imin(l24 + two_k3, l35 + two_k4), j14 + two_k5));
  lo = imax(lo, vp.X_lo2);
  hi = imin(hi, vp.X_lo2 + 2 * (vp.NX - 1));
  const int NX = vp.NX, n_i1 = vp.i_n[0];
  const int nK2 = vp.K_n[0], nK3 = vp.K_n[1], nK4 = vp.K_n[2], nK5 = vp.K_n[3];
  const int k2g = (two_k2 - vp.K_lo2[0]) / 2, k3g = (two_k3 - vp.K_lo2[1]) / 2;
  const int k4g = (two_k4 - vp.K_lo2[2]) / 2, k5g = (two_k5 - vp.K_lo2[3]) / 2;
  const double *t1 = vp.T1 + ((int64_t)n1 * nK5 + k5g) * NX;
  const double *t2 = vp.T2 + ((int64_t)k5g * nK4 + k4g) * NX;
  const double *t3 = vp.T3 + ((int64_t)k4g * nK3 + k3g) * NX;
  const double *t4 = vp.T4 + ((int64_t)k3g * nK2 + k2g) * NX;
  const double *t5 = vp.T5 + ((int64_t)k2g * n_i1 + n1) * NX;
  double w = 0.0;
  for (int x2 = lo; x2 <= hi; x2 += 2) {
    const int xg = (x2 - vp.X_lo2) / 2;
    w += t1[xg] * t2[xg] * t3[xg] * t4[xg] * t5[xg] * (double)(x2 + 1);
  }
  // (-1)^R: the header's phase at the lowest intertwiners, one sign per unit step of each.
  const double sgn = ((n1 + k2 + k3 + k4 + k5) & 1) ? -h.sign : h.sign;
  double norm = __builtin_sqrt((double)(two_i1 + 1));
  norm *= __builtin_sqrt((double)(two_k2 + 1)) * __builtin_sqrt((double)(two_k3 + 1));
  norm *= __builtin_sqrt((double)(two_k4 + 1)) * __builtin_sqrt((double)(two_k5 + 1));
  A[u] = sgn * w * norm;
}

}  // namespace

hipError_t launch_bf_vertex(const VertexParams &vp, double *A, int64_t total, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  bf_vertex_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(vp, A, total);
  return hipGetLastError();
}

hipError_t launch_assemble(const VertexParams &vp, int D, hipStream_t s) {
  if (D == 8) {
    dim3 grid(vp.nchunk, vp.i_n[0], 1);
    assemble_kernel<8, 4, 256, 1, 8><<<grid, 256, 0, s>>>(vp);
  } else if (D == 16) {
    dim3 grid(vp.nchunk, vp.i_n[0], (vp.i_n[1] + 7) / 8);
    assemble_kernel<16, 1, 512, 2, 8><<<grid, 512, 0, s>>>(vp);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reduce(const ReduceParams &rp, hipStream_t s) {
  const int64_t blocks = (rp.a_size + 63) / 64;
  reduce_kernel<<<(unsigned)blocks, 64 * RW, 0, s>>>(rp);
  return hipGetLastError();
}

hipError_t launch_shell_fifteenj(const VertexParams &vp, int64_t shell, double *W, hipStream_t s) {
  // The largest row count of any shell bounds the grid; threads beyond the shell's rows exit.
  int maxk = 1;
  for (int e = 0; e < 4; ++e) maxk = maxk > vp.K_n[e] ? maxk : vp.K_n[e];
  const int64_t rows = (int64_t)vp.i_n[0] * maxk * maxk * maxk;
  const unsigned blocks = (unsigned)((rows + 255) / 256);
  if (vp.K_n[0] <= 8 && vp.K_n[1] <= 8 && vp.K_n[2] <= 8 && vp.K_n[3] <= 8)
    shell_fifteenj_kernel<8><<<blocks, 256, 0, s>>>(vp, shell, W);
  else
    shell_fifteenj_kernel<16><<<blocks, 256, 0, s>>>(vp, shell, W);
  return hipGetLastError();
}

}  // namespace eprl
