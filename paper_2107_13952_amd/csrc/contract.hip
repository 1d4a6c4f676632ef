// Boundary contraction of the vertex tensor (Sec. 3.2, `contract`) and its adjoint.
//
//   F = sum_i A(i1..i5) psi1(i1) psi2(i2) psi3(i3) psi4(i4) psi5(i5)        (no conjugation)
//
// Adjoint with respect to the boundary vectors: dF/dpsi_a = A contracted with the other four.
// Adjoint with respect to the boosters (eq. (vertex-ampl) differentiated): with
// p(i) = sqrt(2i+1) psi(i) and u_e(k) = sum_i p_e(i) (2k+1) B_e(i, k),
//
//   dF/dB_e(i, k; l_e) = p_e(i) (2k+1) sum_{shells with triple l_e} G_e(k),
//   G_e(k_e) = sum_{i1, k_b (b != e)} p_1(i1) prod_{b != e} u_b(k_b) W(i1, k2..k5).
//
// With the boundary vectors inserted, W never has to be formed: writing the x-sum of eq. (15j)
// as a trace around the ring of 6j matrices
//   S1(i1,k5) S2(k5,k4) S3(k4,k3) S4(k3,k2) S5(k2,i1)        (one set per x)
// every G_e is a diagonal of a cyclic matrix product, O(d^3) per x instead of O(d^5).
// Each shell is recomputed independently; per-shell G vectors are then summed per booster
// block in a fixed order (deterministic, no atomics).
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
__device__ __forceinline__ cplx cscale(cplx a, double s) { return {a.re * s, a.im * s}; }

constexpr int kContractThreads = 256;

// Block-level deterministic sum of a complex value (fixed tree order).
__device__ cplx block_sum(cplx v, cplx *sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w) sh[tid] = cadd(sh[tid], sh[tid + w]);
    __syncthreads();
  }
  cplx r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ cplx load_c(const double *p, int i) { return {p[2 * i], p[2 * i + 1]}; }

// Stage 1: each block sums a fixed contiguous range of entries.
__global__ void contract_partial_kernel(ContractParams cp, int64_t total) {
  __shared__ cplx sh[kContractThreads];
  const int64_t per = (total + cp.nblocks - 1) / cp.nblocks;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = b0 + per < total ? b0 + per : total;
  cplx acc{0.0, 0.0};
  for (int64_t idx = b0 + threadIdx.x; idx < b1; idx += blockDim.x) {
    int64_t r = idx;
    int ii[5];
    for (int e = 4; e >= 0; --e) {
      ii[e] = (int)(r % cp.n[e]);
      r /= cp.n[e];
    }
    cplx t{cp.A[idx], 0.0};
    for (int e = 0; e < 5; ++e) t = cmul(t, load_c(cp.psi[e], ii[e]));
    acc = cadd(acc, t);
  }
  cplx s = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    cp.partial[2 * blockIdx.x] = s.re;
    cp.partial[2 * blockIdx.x + 1] = s.im;
  }
}

__global__ void contract_final_kernel(const double *partial, int nblocks, double *F) {
  __shared__ cplx sh[kContractThreads];
  cplx acc{0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) acc = cadd(acc, load_c(partial, b));
  cplx s = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    F[0] = s.re;
    F[1] = s.im;
  }
}

// One block per (a, i_a): g * sum over the other four indices.
__global__ void grad_psi_kernel(ContractParams cp, double gre, double gim, GradPsiOut out) {
  __shared__ cplx sh[kContractThreads];
  int a = 0, rem = blockIdx.x;
  while (rem >= cp.n[a]) {
    rem -= cp.n[a];
    ++a;
  }
  const int ia = rem;
  int dims[4], axes[4], na = 0;
  int64_t m = 1;
  for (int e = 0; e < 5; ++e)
    if (e != a) {
      dims[na] = cp.n[e];
      axes[na++] = e;
      m *= cp.n[e];
    }
  cplx acc{0.0, 0.0};
  for (int64_t r0 = threadIdx.x; r0 < m; r0 += blockDim.x) {
    int ii[5];
    ii[a] = ia;
    int64_t r = r0;
    for (int q = 3; q >= 0; --q) {
      ii[axes[q]] = (int)(r % dims[q]);
      r /= dims[q];
    }
    int64_t idx = 0;
    for (int e = 0; e < 5; ++e) idx = idx * cp.n[e] + ii[e];
    cplx t{cp.A[idx], 0.0};
    for (int q = 0; q < 4; ++q) t = cmul(t, load_c(cp.psi[axes[q]], ii[axes[q]]));
    acc = cadd(acc, t);
  }
  cplx s = block_sum(acc, sh);
  if (threadIdx.x == 0 && out.p[a]) {
    cplx g = cmul(s, {gre, gim});
    out.p[a][2 * ia] = g.re;
    out.p[a][2 * ia + 1] = g.im;
  }
}

}  // namespace

// Partial sums of the contraction for callers that cannot allocate: a fixed device array,
// one copy per GPU, held until the process ends.  Host code never passes its name to a kernel
// (on the host it is only a stand-in for the symbol); it passes the device address that
// contract_scratch_address returns for the current device.
static __device__ __align__(256) double scratch[2 * kContractScratchSlots];

hipError_t contract_scratch_address(double **ptr) {
  void *p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  *ptr = e == hipSuccess ? static_cast<double *>(p) : nullptr;
  return e;
}

hipError_t launch_contract(const ContractParams &cp, double *F, hipStream_t s) {
  int64_t total = 1;
  for (int e = 0; e < 5; ++e) total *= cp.n[e];
  contract_partial_kernel<<<cp.nblocks, kContractThreads, 0, s>>>(cp, total);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  contract_final_kernel<<<1, kContractThreads, 0, s>>>(cp.partial, cp.nblocks, F);
  return hipGetLastError();
}

hipError_t launch_grad_psi(const ContractParams &cp, double gre, double gim, double *const out[5],
                           hipStream_t s) {
  GradPsiOut o;
  int blocks = 0;
  for (int e = 0; e < 5; ++e) {
    o.p[e] = out[e];
    blocks += cp.n[e];
  }
  grad_psi_kernel<<<blocks, kContractThreads, 0, s>>>(cp, gre, gim, o);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Booster adjoint.

namespace {

// Threads per shell: enough for one KD x KD product per round (two wavefronts up to KD = 10,
// four above).
template <int KD>
constexpr int adj_threads() { return KD <= 10 ? 128 : 256; }
// The per-shell matrices are padded to KD x KD (KD in 8, 10, 12, 16: the smallest that holds
// the configuration's dimensions), so that the LDS of a workgroup, and with it the number of
// workgroups resident per CU, follows the actual dimensions.

struct AdjShell {
  int o[6], t[4], klo[4], kn[4];
  double sign;
  bool live;
};

__device__ AdjShell adj_header(const VertexParams &vp, int64_t s) {
  AdjShell h;
  const int nd = vp.nd;
  int64_t r = s;
  for (int q = 5; q >= 0; --q) {
    h.o[q] = (int)(r % nd);
    r /= nd;
  }
  h.t[0] = (h.o[0] * nd + h.o[1]) * nd + h.o[2];
  h.t[1] = (h.o[3] * nd + h.o[4]) * nd + h.o[0];
  h.t[2] = (h.o[5] * nd + h.o[1]) * nd + h.o[3];
  h.t[3] = (h.o[2] * nd + h.o[4]) * nd + h.o[5];
  const int nd3 = nd * nd * nd;
  h.live = true;
  for (int e = 0; e < 4; ++e) {
    h.klo[e] = vp.kr[(e * nd3 + h.t[e]) * 2 + 0];
    h.kn[e] = vp.kr[(e * nd3 + h.t[e]) * 2 + 1];
    h.live = h.live && h.kn[e] > 0;
  }
  int base = vp.i_lo2[0];
  for (int q = 0; q < 10; ++q) base += vp.two_j[q];
  for (int q = 0; q < 6; ++q) base += 2 * h.o[q];
  for (int e = 0; e < 4; ++e) base += h.klo[e];
  h.sign = ((base / 2) & 1) ? -1.0 : 1.0;
  return h;
}

// C(rows x cols) = A(rows x inner) * diag(dg) * B(inner x cols), all in LDS, KD-strided.
// dg may be null (identity).  Complex A, real or complex B handled by the caller through
// separate real/imaginary planes: here everything is complex.
template <int KD>
__device__ void cmatmul(const cplx *A, const cplx *dg, const cplx *B, cplx *C, int rows, int inner,
                        int cols) {
  for (int idx = threadIdx.x; idx < rows * cols; idx += blockDim.x) {
    const int r = idx / cols, c = idx % cols;
    cplx t{0.0, 0.0};
    for (int q = 0; q < inner; ++q) {
      cplx a = A[r * KD + q];
      if (dg) a = cmul(a, dg[q]);
      t = cadd(t, cmul(a, B[q * KD + c]));
    }
    C[r * KD + c] = t;
  }
}

template <int KD>
__global__ __launch_bounds__(adj_threads<KD>()) void adjoint_shell_kernel(AdjointParams ap) {
  const VertexParams &vp = ap.v;
  const int64_t s = vp.shell_begin + blockIdx.x;
  if (s >= vp.shell_end) return;
  const AdjShell h = adj_header(vp, s);
  cplx *gout = reinterpret_cast<cplx *>(ap.shell_g) + (int64_t)blockIdx.x * 4 * ap.kpad;
  if (!h.live) {
    for (int q = threadIdx.x; q < 4 * ap.kpad; q += blockDim.x) gout[q] = {0.0, 0.0};
    return;
  }
  __shared__ cplx S[5][KD * KD];         // S1 (i1 x k5), S2 (k5 x k4), S3 (k4 x k3), S4 (k3 x k2), S5 (k2 x i1)
  __shared__ cplx Ra[KD * KD], Rb[KD * KD], E[KD * KD], H[KD * KD], Y[KD * KD];
  __shared__ cplx P1[KD], U[4][KD];      // diag factors with (-1)^n; U[0..3] = k2..k5
  __shared__ cplx G[4][KD];
  const int n1 = vp.i_n[0];
  const int dk[4] = {h.kn[0], h.kn[1], h.kn[2], h.kn[3]};
  const int nd = vp.nd, nd3 = nd * nd * nd, NX = vp.NX;
  // Diagonal factors.
  for (int q = threadIdx.x; q < KD; q += blockDim.x) {
    cplx p{0.0, 0.0};
    if (q < n1) {
      p = cscale(load_c(ap.psi[0], q), __builtin_sqrt((double)(vp.i_lo2[0] + 2 * q + 1)));
      if (q & 1) p = cscale(p, -1.0);
    }
    P1[q] = p;
    for (int e = 0; e < 4; ++e) {
      cplx u{0.0, 0.0};
      if (q < dk[e]) {
        const int64_t off = vp.boff[e * nd3 + h.t[e]];
        const double wk = (double)(h.klo[e] + 2 * q + 1);
        for (int i = 0; i < vp.i_n[e + 1]; ++i) {
          cplx pi = cscale(load_c(ap.psi[e + 1], i), __builtin_sqrt((double)(vp.i_lo2[e + 1] + 2 * i + 1)));
          u = cadd(u, cscale(pi, vp.B[off + (int64_t)i * dk[e] + q] * wk));
        }
        if (q & 1) u = cscale(u, -1.0);
      }
      U[e][q] = u;
      G[e][q] = {0.0, 0.0};
    }
  }
  const int nK2 = vp.K_n[0], nK3 = vp.K_n[1], nK4 = vp.K_n[2], nK5 = vp.K_n[3];
  const int k2g = (h.klo[0] - vp.K_lo2[0]) / 2, k3g = (h.klo[1] - vp.K_lo2[1]) / 2;
  const int k4g = (h.klo[2] - vp.K_lo2[2]) / 2, k5g = (h.klo[3] - vp.K_lo2[3]) / 2;
  const int *o = h.o;
  __syncthreads();
  for (int xg = 0; xg < NX; ++xg) {
    const double cx = (double)(vp.X_lo2 + 2 * xg + 1) * h.sign;
    // Load the five 6j matrices of this x.
    for (int idx = threadIdx.x; idx < KD * KD; idx += blockDim.x) {
      const int r = idx / KD, c = idx % KD;
      double v1 = 0, v2 = 0, v3 = 0, v4 = 0, v5 = 0;
      if (r < n1 && c < dk[3])
        v1 = vp.T1[(((int64_t)o[2] * n1 + r) * nK5 + k5g + c) * NX + xg];
      if (r < dk[3] && c < dk[2])
        v2 = vp.T2[((((int64_t)o[4] * nd + o[5]) * nK5 + k5g + r) * nK4 + k4g + c) * NX + xg];
      if (r < dk[2] && c < dk[1])
        v3 = vp.T3[(((((int64_t)o[1] * nd + o[3]) * nd + o[4]) * nK4 + k4g + r) * nK3 + k3g + c) * NX + xg];
      if (r < dk[1] && c < dk[0])
        v4 = vp.T4[((((int64_t)o[0] * nd + o[1]) * nK3 + k3g + r) * nK2 + k2g + c) * NX + xg];
      if (r < dk[0] && c < n1)
        v5 = vp.T5[(((int64_t)o[2] * nK2 + k2g + r) * n1 + c) * NX + xg];
      S[0][idx] = {v1 * cx, 0.0};
      S[1][idx] = {v2, 0.0};
      S[2][idx] = {v3, 0.0};
      S[3][idx] = {v4, 0.0};
      S[4][idx] = {v5, 0.0};
    }
    __syncthreads();
    // Ra = S5 P1 S1 (k2 x k5);  Rb = S2 U4 S3 (k5 x k3)
    cmatmul<KD>(S[4], P1, S[0], Ra, dk[0], n1, dk[3]);
    cmatmul<KD>(S[1], U[2], S[2], Rb, dk[3], dk[2], dk[1]);
    __syncthreads();
    // E = S4 U2 Ra (k3 x k5);  Y = Rb U3 S4 (k5 x k2)
    cmatmul<KD>(S[3], U[0], Ra, E, dk[1], dk[0], dk[3]);
    cmatmul<KD>(Rb, U[1], S[3], Y, dk[3], dk[1], dk[0]);
    __syncthreads();
    // H = E U5 S2 (k3 x k4)
    cmatmul<KD>(E, U[3], S[1], H, dk[1], dk[3], dk[2]);
    __syncthreads();
    // Diagonals:
    //  G5(k5) = sum_k3 Rb(k5,k3) U3(k3) E(k3,k5)     G3(k3) = sum_k5 E(k3,k5) U5(k5) Rb(k5,k3)
    //  G4(k4) = sum_k3 S3(k4,k3) U3(k3) H(k3,k4)     G2(k2) = sum_k5 Ra(k2,k5) U5(k5) Y(k5,k2)
    for (int q = threadIdx.x; q < 4 * KD; q += blockDim.x) {
      const int e = q / KD, k = q % KD;
      if (k >= dk[e]) continue;
      cplx t{0.0, 0.0};
      if (e == 3) {
        for (int c = 0; c < dk[1]; ++c) t = cadd(t, cmul(cmul(Rb[k * KD + c], U[1][c]), E[c * KD + k]));
      } else if (e == 1) {
        for (int c = 0; c < dk[3]; ++c) t = cadd(t, cmul(cmul(E[k * KD + c], U[3][c]), Rb[c * KD + k]));
      } else if (e == 2) {
        for (int c = 0; c < dk[1]; ++c) t = cadd(t, cmul(cmul(S[2][k * KD + c], U[1][c]), H[c * KD + k]));
      } else {
        for (int c = 0; c < dk[3]; ++c) t = cadd(t, cmul(cmul(Ra[k * KD + c], U[3][c]), Y[c * KD + k]));
      }
      G[e][k] = cadd(G[e][k], t);
    }
    __syncthreads();
  }
  // (-1)^{n_k} of the differentiated index.
  for (int q = threadIdx.x; q < 4 * ap.kpad; q += blockDim.x) {
    const int e = q / ap.kpad, k = q % ap.kpad;
    cplx v{0.0, 0.0};
    if (k < dk[e] && k < KD) v = (k & 1) ? cscale(G[e][k], -1.0) : G[e][k];
    gout[q] = v;
  }
}

// One thread per booster entry: sum the per-shell G over the shells that use its block.
__global__ void adjoint_reduce_kernel(AdjointParams ap, double gre, double gim, double *grad_b) {
  const VertexParams &vp = ap.v;
  const int nd = vp.nd, nd3 = nd * nd * nd;
  const int64_t total = vp.boff[4 * nd3];
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  // Locate the block (edge e, triple t) by binary search over the offsets.
  int lo = 0, hi = 4 * nd3 - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (vp.boff[mid] <= idx) lo = mid; else hi = mid - 1;
  }
  const int e = lo / nd3, t = lo % nd3;
  const int kn = vp.kr[(e * nd3 + t) * 2 + 1], klo = vp.kr[(e * nd3 + t) * 2];
  const int64_t within = idx - vp.boff[lo];
  const int i = (int)(within / kn), k = (int)(within % kn);
  const int a = t / (nd * nd), b = (t / nd) % nd, c = t % nd;
  // Shell coordinates (o23, o24, o25, o34, o35, o45) of the block's triple; the other three
  // coordinates run over 0..dl in lexicographic order.
  cplx sum{0.0, 0.0};
  for (int f = 0; f < nd3; ++f) {
    const int p = f / (nd * nd), q = (f / nd) % nd, r = f % nd;
    int o[6];
    if (e == 0) { o[0] = a; o[1] = b; o[2] = c; o[3] = p; o[4] = q; o[5] = r; }
    else if (e == 1) { o[3] = a; o[4] = b; o[0] = c; o[1] = p; o[2] = q; o[5] = r; }
    else if (e == 2) { o[5] = a; o[1] = b; o[3] = c; o[0] = p; o[2] = q; o[4] = r; }
    else { o[2] = a; o[4] = b; o[5] = c; o[0] = p; o[1] = q; o[3] = r; }
    int64_t sh = 0;
    for (int z = 0; z < 6; ++z) sh = sh * nd + o[z];
    if (sh < vp.shell_begin || sh >= vp.shell_end) continue;
    const cplx *g = reinterpret_cast<const cplx *>(ap.shell_g) + (sh - vp.shell_begin) * 4 * ap.kpad;
    sum = cadd(sum, g[e * ap.kpad + k]);
  }
  cplx pe = cscale(load_c(ap.psi[e + 1], i), __builtin_sqrt((double)(vp.i_lo2[e + 1] + 2 * i + 1)));
  cplx v = cmul(cscale(cmul(pe, sum), (double)(klo + 2 * k + 1)), {gre, gim});
  grad_b[2 * idx] = v.re;
  grad_b[2 * idx + 1] = v.im;
}

}  // namespace

hipError_t launch_adjoint_shells(const AdjointParams &ap, hipStream_t s) {
  const int64_t n = ap.v.shell_end - ap.v.shell_begin;
  if (n <= 0) return hipSuccess;
  const int d = ap.v.i_n[0] > ap.kpad ? ap.v.i_n[0] : ap.kpad;
  if (d > 16) return hipErrorInvalidValue;
  if (d <= 8)
    adjoint_shell_kernel<8><<<(unsigned)n, adj_threads<8>(), 0, s>>>(ap);
  else if (d <= 10)
    adjoint_shell_kernel<10><<<(unsigned)n, adj_threads<10>(), 0, s>>>(ap);
  else if (d <= 12)
    adjoint_shell_kernel<12><<<(unsigned)n, adj_threads<12>(), 0, s>>>(ap);
  else
    adjoint_shell_kernel<16><<<(unsigned)n, adj_threads<16>(), 0, s>>>(ap);
  return hipGetLastError();
}

hipError_t launch_adjoint_reduce(const AdjointParams &ap, int64_t total, double gre, double gim,
                                 double *grad_b, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  adjoint_reduce_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(ap, gre, gim, grad_b);
  return hipGetLastError();
}

}  // namespace eprl
