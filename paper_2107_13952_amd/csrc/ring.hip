// Factorised ("ring") evaluation of the vertex tensor, eq. (vertex-ampl) with eq. (15j).
//
// For fixed x the sum over k2..k5 of W times the four booster blocks is a closed chain
//   U1(i1,k5) M5(i5,k5) U2(k5,k4) M4(i4,k4) U3(k4,k3) M3(i3,k3) U4(k3,k2) M2(i2,k2) U5(k2,i1)
// (U = signed 6j tables, M_e = (2k_e+1) B_e).  The six shell spins enter as
//   U1, U5: l25      U2: l35, l45     U3: l24, l34, l35     U4: l23, l24
//   M5: (l25, l35, l45)   M4: (l45, l24, l34)   M3: (l34, l35, l23)   M2: (l23, l24, l25)
// so with the "core" (l24, l25, l34, l35) fixed, l45 only touches the half chain on the k5/k4
// side and l23 only the half chain on the k2/k3 side.  Both sums are done first:
//   G(i5, i4, k4) = sum_{l45} [sum_{k5} U1(i1,k5) M5(i5,k5) U2(k5,k4)] M4(i4,k4)
//   H(k3, i3, i2) = sum_{l23} M3(i3,k3) [sum_{k2} U4(k3,k2) M2(i2,k2) U5(k2,i1)]
//   P(i5, i4, k3) = sum_{k4} G(i5,i4,k4) U3(k4,k3)                            (FP64 MFMA)
//   A(i1; i5 i4, i3 i2) += sum_{k3} P(i5 i4, k3) H(k3, i3 i2)                   (FP64 MFMA)
// which is the same sum as the framed algorithm of Sec. 3.1 regrouped by linearity; with the
// index ranges that the triads leave active at each x it needs about 17x fewer
// multiply-adds than the per-shell mode products at j = 3, dl = 8.
//
// Work decomposition: one workgroup (4 wavefronts) per (chunk of cores, i1).  The
// A(i1, ...) slice (rows (i5, i4), columns (i3, i2), padded to 64 x 64) lives in MFMA
// accumulators for the whole chunk; wavefront w owns row tile w.  Per x: G on lanes
// (i5, k4), H on lanes (k3, i2), both VALU, through LDS into two 16x16x4 FP64 MFMA
// contractions.  Partial slices are reduced in fixed order by the shell-path reduction.
#include "eprl_internal.hpp"

namespace eprl {

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int RT = 256;  // threads per workgroup

__device__ __forceinline__ int iabs(int v) { return v < 0 ? -v : v; }
__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }
__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

// One work item: cores [chunk * rp.chunk, ...) of rp, boundary intertwiner i1 = n1.
template <int KW>
__device__ void ring_item(const RingParams &rp, int64_t chunk_index, int n1, double *smem) {
  constexpr int GS = KW + 1;  // padded row stride of G and P
  const int nd = rp.nd, nd3 = nd * nd * nd;
  double *Gs = smem;                  // [64][GS]  rows (i5, i4), cols k4
  double *Ps = Gs + 64 * GS;          // [64][GS]  rows (i5, i4), cols k3
  double *Hs = Ps + 64 * GS;          // [KW][64]  rows k3, cols (i3, i2)
  double *U3s = Hs + KW * 64;         // [KW][KW]  k4 x k3
  double *Mb = U3s + KW * KW;         // [4][nd][8][8]: M5, M4 (per o45), M2, M3 (per o23)
  double *U2s = Mb + 4 * nd * 64;     // [nd][8][KW]  per o45: active k5 x core-window k4
  double *U4s = U2s + nd * 8 * KW;    // [nd][KW][8]  per o23: core-window k3 x active k2
  double *U1s = U4s + nd * KW * 8;    // [nd][8]      per o45: active k5
  double *U5s = U1s + nd * 8;         // [nd][8]      per o23: active k2
  int *rng = reinterpret_cast<int *>(U5s + nd * 8);  // [8][nd]: lo/n of k5, k4, k2, k3

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int *J = rp.two_j;
  const int two_i1 = rp.i_lo2[0] + 2 * n1;
  const int d1 = rp.i_n[0], d2 = rp.i_n[1], d3 = rp.i_n[2], d4 = rp.i_n[3], d5 = rp.i_n[4];
  const int NX = rp.NX, nK2 = rp.K_n[0], nK3 = rp.K_n[1], nK4 = rp.K_n[2], nK5 = rp.K_n[3];
  const int xhi_g = rp.X_lo2 + 2 * (NX - 1);

  d4v acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = d4v{0.0, 0.0, 0.0, 0.0};

  const int64_t c0 = rp.core_begin + chunk_index * rp.chunk;
  const int64_t c1 = c0 + rp.chunk < rp.core_end ? c0 + rp.chunk : rp.core_end;
  for (int64_t core = c0; core < c1; ++core) {
    const int o24 = (int)(core / (nd * nd * nd)), o25 = (int)((core / (nd * nd)) % nd);
    const int o34 = (int)((core / nd) % nd), o35 = (int)(core % nd);
    const int l24 = J[L24] + 2 * o24, l25 = J[L25] + 2 * o25;
    const int l34 = J[L34] + 2 * o34, l35 = J[L35] + 2 * o35;
    // Ranges of k5, k4 for every l45 and of k2, k3 for every l23 (empty when either
    // range of that edge pair is empty, so the spin does not contribute).
    __syncthreads();  // previous core's readers of rng / Mb are done
    for (int o = tid; o < nd; o += RT) {
      const int t5 = (o25 * nd + o35) * nd + o, t4 = (o * nd + o24) * nd + o34;
      const int t2 = (o * nd + o24) * nd + o25, t3 = (o34 * nd + o35) * nd + o;
      int n5 = rp.kr[(3 * nd3 + t5) * 2 + 1], n4 = rp.kr[(2 * nd3 + t4) * 2 + 1];
      int n2 = rp.kr[(0 * nd3 + t2) * 2 + 1], n3 = rp.kr[(1 * nd3 + t3) * 2 + 1];
      if (n5 == 0 || n4 == 0) n5 = n4 = 0;
      if (n2 == 0 || n3 == 0) n2 = n3 = 0;
      rng[0 * nd + o] = rp.kr[(3 * nd3 + t5) * 2];
      rng[1 * nd + o] = n5;
      rng[2 * nd + o] = rp.kr[(2 * nd3 + t4) * 2];
      rng[3 * nd + o] = n4;
      rng[4 * nd + o] = rp.kr[(0 * nd3 + t2) * 2];
      rng[5 * nd + o] = n2;
      rng[6 * nd + o] = rp.kr[(1 * nd3 + t3) * 2];
      rng[7 * nd + o] = n3;
    }
    __syncthreads();
    // Core windows of k4 (over l45) and k3 (over l23).
    int w4lo = 1 << 30, w4hi = -1, w3lo = 1 << 30, w3hi = -1;
    for (int o = 0; o < nd; ++o) {
      if (rng[3 * nd + o] > 0) {
        w4lo = imin(w4lo, rng[2 * nd + o]);
        w4hi = imax(w4hi, rng[2 * nd + o] + 2 * (rng[3 * nd + o] - 1));
      }
      if (rng[7 * nd + o] > 0) {
        w3lo = imin(w3lo, rng[6 * nd + o]);
        w3hi = imax(w3hi, rng[6 * nd + o] + 2 * (rng[7 * nd + o] - 1));
      }
    }
    if (w4hi < 0 || w3hi < 0) continue;  // uniform: no live shell in this core
    // Stage the weighted booster blocks of this core.
    for (int idx = tid; idx < 4 * nd * 64; idx += RT) {
      const int e = idx / (nd * 64), o = (idx / 64) % nd, i = (idx / 8) % 8, k = idx % 8;
      // e: 0 = M5 (o45), 1 = M4 (o45), 2 = M2 (o23), 3 = M3 (o23)
      const int edge = e == 0 ? 3 : (e == 1 ? 2 : (e == 2 ? 0 : 1));
      const int t = e == 0 ? (o25 * nd + o35) * nd + o
                  : e == 1 ? (o * nd + o24) * nd + o34
                  : e == 2 ? (o * nd + o24) * nd + o25
                           : (o34 * nd + o35) * nd + o;
      const int klo = rp.kr[(edge * nd3 + t) * 2], kn = rp.kr[(edge * nd3 + t) * 2 + 1];
      const int ni = rp.i_n[edge + 1];
      double v = 0.0;
      if (i < ni && k < kn)
        v = rp.B[rp.boff[edge * nd3 + t] + (int64_t)i * kn + k] * (double)(klo + 2 * k + 1);
      Mb[idx] = v;
    }
    // x closes (i1 l25 x); the other triads restrict the k ranges at each x.
    const int xlo = imax(iabs(two_i1 - l25), rp.X_lo2), xhi = imin(two_i1 + l25, xhi_g);
    const int64_t u3base = (((int64_t)o24 * nd + o34) * nd + o35) * NX;
    for (int x = xlo; x <= xhi; x += 2) {
      const int xg = (x - rp.X_lo2) / 2;
      const int a4 = imax(w4lo, iabs(l35 - x)), b4 = imin(w4hi, l35 + x);
      const int a3 = imax(w3lo, iabs(l24 - x)), b3 = imin(w3hi, l24 + x);
      if (a4 > b4 || a3 > b3) continue;  // uniform
      const int a4l = (a4 - w4lo) / 2, b4l = (b4 - w4lo) / 2;
      const int a3l = (a3 - w3lo) / 2, b3l = (b3 - w3lo) / 2;
      __syncthreads();  // previous x's readers of Gs / Hs / U3s / Ps are done
      // Stage every 6j slice this x needs, zero outside the active windows:
      // U3 (k4 x k3); per l45 the active k5 of its range (at most 8) with U1 and U2 (k5 x k4
      // window); per l23 the active k2 of its range with U5 and U4 (k3 window x k2).
      const int x14lo = iabs(x - J[L14]), x14hi = x + J[L14];
      const int x13lo = iabs(J[L13] - x), x13hi = J[L13] + x;
      const int k4g0 = (w4lo - rp.K_lo2[2]) / 2, k3g0 = (w3lo - rp.K_lo2[1]) / 2;
      {
        const int n_u3 = KW * KW, n_u2 = nd * 8 * KW, n_u4 = nd * KW * 8, n_v = 2 * nd * 8;
        const int total = n_u3 + n_u2 + n_u4 + n_v;
        for (int idx = tid; idx < total; idx += RT) {
          double v = 0.0;
          if (idx < n_u3) {
            const int k4l = idx / KW, k3l = idx % KW;
            if (k4l >= a4l && k4l <= b4l && k3l >= a3l && k3l <= b3l)
              v = rp.U3[((u3base + xg) * nK4 + k4g0 + k4l) * nK3 + k3g0 + k3l];
            U3s[idx] = v;
          } else if (idx < n_u3 + n_u2) {
            const int q = idx - n_u3, o = q / (8 * KW), k5i = (q / KW) % 8, k4l = q % KW;
            const int lo5 = rng[0 * nd + o], n5 = rng[1 * nd + o];
            const int b5 = imax(lo5, x14lo), e5 = imin(lo5 + 2 * (n5 - 1), x14hi);
            const int k5 = b5 + 2 * k5i;
            if (n5 > 0 && k5 <= e5 && k4l >= a4l && k4l <= b4l)
              v = rp.U2[((((int64_t)o35 * nd + o) * NX + xg) * nK5 + (k5 - rp.K_lo2[3]) / 2) * nK4 +
                        k4g0 + k4l];
            U2s[q] = v;
          } else if (idx < n_u3 + n_u2 + n_u4) {
            const int q = idx - n_u3 - n_u2, o = q / (KW * 8), k3l = (q / 8) % KW, k2i = q % 8;
            const int lo2 = rng[4 * nd + o], n2 = rng[5 * nd + o];
            const int b2 = imax(lo2, x13lo), e2 = imin(lo2 + 2 * (n2 - 1), x13hi);
            const int k2 = b2 + 2 * k2i;
            if (n2 > 0 && k2 <= e2 && k3l >= a3l && k3l <= b3l)
              v = rp.U4[((((int64_t)o * nd + o24) * NX + xg) * nK3 + k3g0 + k3l) * nK2 +
                        (k2 - rp.K_lo2[0]) / 2];
            U4s[q] = v;
          } else {
            const int q = idx - n_u3 - n_u2 - n_u4, side = q / (nd * 8), o = (q / 8) % nd, i = q % 8;
            if (side == 0) {  // U1 for the active k5 of l45 = o
              const int lo5 = rng[0 * nd + o], n5 = rng[1 * nd + o];
              const int b5 = imax(lo5, x14lo), e5 = imin(lo5 + 2 * (n5 - 1), x14hi);
              const int k5 = b5 + 2 * i;
              if (n5 > 0 && k5 <= e5)
                v = rp.U1[(((int64_t)o25 * NX + xg) * d1 + n1) * nK5 + (k5 - rp.K_lo2[3]) / 2];
              U1s[o * 8 + i] = v;
            } else {  // U5 for the active k2 of l23 = o
              const int lo2 = rng[4 * nd + o], n2 = rng[5 * nd + o];
              const int b2 = imax(lo2, x13lo), e2 = imin(lo2 + 2 * (n2 - 1), x13hi);
              const int k2 = b2 + 2 * i;
              if (n2 > 0 && k2 <= e2)
                v = rp.U5[(((int64_t)o25 * NX + xg) * nK2 + (k2 - rp.K_lo2[0]) / 2) * d1 + n1];
              U5s[o * 8 + i] = v;
            }
          }
        }
      }
      __syncthreads();
      // Half chains.  KW = 16: G on threads 0..127 and H on 128..255 at the same time.
      for (int pass = 0; pass < (KW == 16 ? 1 : 2); ++pass) {
        const bool doG = KW == 16 ? tid < 128 : pass == 0;
        const int u = KW == 16 ? (tid & 127) : tid;
        if (doG) {
          const int i5 = u / KW, k4l = u % KW;
          double g[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) g[q] = 0.0;
          if (k4l >= a4l && k4l <= b4l) {
            const int k4 = w4lo + 2 * k4l;
            for (int o = 0; o < nd; ++o) {
              const int n5 = rng[1 * nd + o], lo4 = rng[2 * nd + o], n4 = rng[3 * nd + o];
              if (n5 == 0 || k4 < lo4 || k4 > lo4 + 2 * (n4 - 1)) continue;
              // active k5 of this l45: its range intersected with the (k5 j14 x) triad
              const int lo5 = rng[0 * nd + o];
              const int b5 = imax(lo5, x14lo), e5 = imin(lo5 + 2 * (n5 - 1), x14hi);
              const int c5 = e5 >= b5 ? (e5 - b5) / 2 + 1 : 0;
              const double *m5 = Mb + (0 * nd + o) * 64 + i5 * 8 + (b5 - lo5) / 2;
              const double *u2 = U2s + o * 8 * KW + k4l;
              const double *u1 = U1s + o * 8;
              double t = 0.0;
#pragma unroll
              for (int k5i = 0; k5i < 8; ++k5i)
                if (k5i < c5) t += u1[k5i] * m5[k5i] * u2[k5i * KW];
              const double *m4 = Mb + (1 * nd + o) * 64 + (k4 - lo4) / 2;
#pragma unroll
              for (int i4 = 0; i4 < 8; ++i4) g[i4] += t * m4[i4 * 8];
            }
          }
#pragma unroll
          for (int i4 = 0; i4 < 8; ++i4) Gs[(i5 * 8 + i4) * GS + k4l] = g[i4];
        } else {
          const int k3l = u / 8, i2 = u % 8;
          double hq[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) hq[q] = 0.0;
          if (k3l >= a3l && k3l <= b3l) {
            const int k3 = w3lo + 2 * k3l;
            for (int o = 0; o < nd; ++o) {
              const int lo2 = rng[4 * nd + o], n2 = rng[5 * nd + o];
              const int lo3 = rng[6 * nd + o], n3 = rng[7 * nd + o];
              if (n2 == 0 || k3 < lo3 || k3 > lo3 + 2 * (n3 - 1)) continue;
              const int b2 = imax(lo2, x13lo), e2 = imin(lo2 + 2 * (n2 - 1), x13hi);
              const int c2 = e2 >= b2 ? (e2 - b2) / 2 + 1 : 0;
              const double *m2 = Mb + (2 * nd + o) * 64 + i2 * 8 + (b2 - lo2) / 2;
              const double *u4 = U4s + (o * KW + k3l) * 8;
              const double *u5 = U5s + o * 8;
              double t = 0.0;
#pragma unroll
              for (int k2i = 0; k2i < 8; ++k2i)
                if (k2i < c2) t += u4[k2i] * m2[k2i] * u5[k2i];
              const double *m3 = Mb + (3 * nd + o) * 64 + (k3 - lo3) / 2;
#pragma unroll
              for (int i3 = 0; i3 < 8; ++i3) hq[i3] += t * m3[i3 * 8];
            }
          }
#pragma unroll
          for (int i3 = 0; i3 < 8; ++i3) Hs[k3l * 64 + i3 * 8 + i2] = hq[i3];
        }
      }
      __syncthreads();
      // P = G U3 (rows (i5, i4), cols k3): wavefront `wave` owns row tile `wave`.
      {
        const int r = wave * 16 + (lane & 15), kq = lane >> 4;
#pragma unroll
        for (int cb = 0; cb < KW / 16; ++cb) {
          d4v c = {0.0, 0.0, 0.0, 0.0};
          for (int ks = a4l & ~3; ks <= b4l; ks += 4) {
            const double a = Gs[r * GS + ks + kq];
            const double b = U3s[(ks + kq) * KW + cb * 16 + (lane & 15)];
            c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) Ps[(wave * 16 + 4 * kq + j) * GS + cb * 16 + (lane & 15)] = c[j];
        }
      }
      __syncthreads();
      // A(i1; rows, cols) += P H over the active k3 window.
      {
        const int r = wave * 16 + (lane & 15), kq = lane >> 4;
        for (int ks = a3l & ~3; ks <= b3l; ks += 4) {
          const double a = Ps[r * GS + ks + kq];
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) {
            const double b = Hs[(ks + kq) * 64 + cb * 16 + (lane & 15)];
            acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[cb], 0, 0, 0);
          }
        }
      }
    }
  }
  // Flush the chunk's partial A(i1, ...): row (i5, i4), column (i3, i2).
  const int64_t slice = (int64_t)d2 * d3 * d4 * d5;
  double *out = rp.partial + (chunk_index * d1 + n1) * slice;
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = wave * 16 + 4 * (lane >> 4) + j, c = cb * 16 + (lane & 15);
      const int i5 = r >> 3, i4 = r & 7, i3 = c >> 3, i2 = c & 7;
      if (i2 < d2 && i3 < d3 && i4 < d4 && i5 < d5)
        out[((i2 * d3 + i3) * d4 + i4) * d5 + i5] = acc[cb][j];
    }
  }
  __syncthreads();  // the next item reuses the LDS
}

template <int KW>
__global__ __launch_bounds__(RT) void ring_kernel(RingParams rp) {
  extern __shared__ double smem[];
  ring_item<KW>(rp, blockIdx.x, blockIdx.y, smem);
}

// Persistent variant for batches: every workgroup walks a static, longest-first list of
// (configuration, chunk, i1) items with stride gridDim.x; no atomics, so the assignment of
// items to workgroups (and every partial sum) is fixed.
template <int KW>
__global__ __launch_bounds__(RT) void ring_batch_kernel(const RingParams *cfgs, const int *items,
                                                        int nitems) {
  extern __shared__ double smem[];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int c = items[3 * it], chunk = items[3 * it + 1], n1 = items[3 * it + 2];
    ring_item<KW>(cfgs[c], chunk, n1, smem);
  }
}

}  // namespace

size_t ring_smem_bytes(int KW, int nd) {
  const int GS = KW + 1;
  return sizeof(double) * (size_t)(2 * 64 * GS + KW * 64 + KW * KW + 4 * nd * 64 +
                                   2 * nd * 8 * KW + 2 * nd * 8) +
         sizeof(int) * (size_t)(8 * nd);
}

// Allow the ring kernels the dynamic LDS of the largest supported configuration.  Called once
// per process before any launch (not a stream operation, so never inside a graph capture).
hipError_t ring_init_attributes() {
  const int bytes = (int)ring_smem_bytes(32, kRingMaxNd);
  const void *fns[4] = {(const void *)ring_kernel<16>, (const void *)ring_kernel<32>,
                        (const void *)ring_batch_kernel<16>, (const void *)ring_batch_kernel<32>};
  for (const void *f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_ring(const RingParams &rp, int KW, hipStream_t s) {
  dim3 grid(rp.nchunk, rp.i_n[0], 1);
  const size_t shm = ring_smem_bytes(KW, rp.nd);
  if (KW == 16) {
    ring_kernel<16><<<grid, RT, shm, s>>>(rp);
  } else if (KW == 32) {
    ring_kernel<32><<<grid, RT, shm, s>>>(rp);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ring_batch(const RingParams *cfgs_dev, const int *items_dev, int nitems, int KW,
                             int max_nd, int grid, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  const size_t shm = ring_smem_bytes(KW, max_nd);
  if (KW == 16) {
    ring_batch_kernel<16><<<grid, RT, shm, s>>>(cfgs_dev, items_dev, nitems);
  } else if (KW == 32) {
    ring_batch_kernel<32><<<grid, RT, shm, s>>>(cfgs_dev, items_dev, nitems);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace eprl
