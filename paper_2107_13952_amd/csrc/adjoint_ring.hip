// Adjoint of the boundary contraction in the factorised (ring) order.
//
// With the boundary vectors inserted (p_a(i) = sqrt(2i+1) psi_a(i), and for the four boosted
// edges u_e(k; l_e) = sum_i p_e(i) M_e(l_e)[i, k], M_e = (2k+1) B_e), eq. (vertex-ampl) contracted
// with psi is, for each x of eq. (15j) and each shell, the trace of a closed chain of the signed
// 6j tables (the ones of the factorised vertex kernels, whose x-sum gives W exactly):
//   F = sum_{shells, x} sum_{i1} p1(i1) [U1 D5 U2 D4 U3 D3 U4 D2 U5](i1, i1),   D_e = diag(u_e).
// The derivative with respect to a booster entry is
//   dF/dB_e(l_e)[i, k] = (2k+1) p_e(i) G_e(k; l_e),
//   G_e(k; l_e) = sum over the shells containing l_e and over x of the chain with u_e(k) taken out.
// With the core (l24, l25, l34, l35) and x fixed, l45 enters only the left half of the chain and
// l23 only the right half, so (all matrices at most 16 x 32):
//   V2_o(k3, i1)  = sum_k2 U4(k3, k2; l23=o) u2(k2; o) U5(k2, i1)          X2 = sum_o D3_o V2_o
//   R4(k4, i1)    = sum_k3 U3(k4, k3) X2(k3, i1)
//   Z5_o(i1, k4)  = sum_k5 p1(i1) U1(i1, k5) u5(k5; l45=o) U2(k5, k4; o)   X5 = sum_o Z5_o D4_o
//   G4_o(k4)     += sum_i1 Z5_o(i1, k4) R4(k4, i1)
//   G5_o(k5)     += sum_i1 p1(i1) U1(i1, k5) sum_k4 U2(k5, k4; o) u4(k4; o) R4(k4, i1)
//   R3(i1, k3)    = sum_k4 X5(i1, k4) U3(k4, k3)
//   G3_o(k3)     += sum_i1 R3(i1, k3) V2_o(k3, i1)
//   G2_o(k2)     += sum_i1 U5(k2, i1) sum_k3 R3(i1, k3) u3(k3; o) U4(k3, k2; o)
// per core and x: O(nd d^3) complex multiply-adds instead of the O(nd^2 d^3) of the per-shell
// traces.  One workgroup per core accumulates its G vectors over x and writes them out; a second
// kernel sums, for every booster entry, the G of the cores that share its block, in a fixed
// order (no atomics: the result is bitwise repeatable).
#include <algorithm>

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
__device__ __forceinline__ cplx cfma(cplx acc, cplx a, double s) {
  return {acc.re + a.re * s, acc.im + a.im * s};
}
__device__ __forceinline__ cplx load_c(const double *p, int i) { return {p[2 * i], p[2 * i + 1]}; }
__device__ __forceinline__ int iabs(int v) { return v < 0 ? -v : v; }
__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }
__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

constexpr int AT = 512;  // threads per workgroup

// Division by a size that is the same for the whole kernel, as a multiply-high by the rounded-up
// reciprocal: exact for dividends and divisors below 2^16 (the item indices of the loops below),
// and one instruction where the generic integer division takes dozens.
struct FastDiv {
  uint32_t m;
  int d;
  __device__ explicit FastDiv(int d_)
      : m(d_ > 1 ? (uint32_t)((0x100000000ull + (uint64_t)d_ - 1) / (uint64_t)d_) : 0u), d(d_) {}
  __device__ int operator()(int q) const { return d > 1 ? (int)__umulhi((uint32_t)q, m) : q; }
};

// The five boundary vectors (device, complex interleaved), passed by value.
struct PsiPtrs {
  const double *p[5];
};
// LDS layout (complex unless noted), sized by the configuration: kl = largest k range of a spin,
// iw = number of i1 values, kw = widest core window of k5, k4, k3 or k2 (union over l45 or l23).
// Per-spin arrays are [nd][kl].  The two halves take their spins (l45, then l23) ng at a time,
// Z5, Q5 and S2 holding one [iw][kl] / [kl][iw] block per spin of the group.  R3 reuses X2 (dead
// once R4 is formed) and S2 reuses Z5 (dead after the left half).
struct AdjGeom {
  int kl, iw, kw, ng;
  int p1, u5, u4, u2, u3, g5, g4, g3, g2;     // [iw] and [nd][kl] vectors
  int v2;                                      // [nd][kl k3][iw]
  int x2, r4, x5, r3;                          // [kw][iw] or [iw][kw]
  int z5, q5, s2;                              // [ng][iw][kl], [ng][kl][iw], [ng][iw][kl] scratch
  int u1s, u5s, u3s;                           // real: [iw][kw], [kw][iw], [kw][kw]
  int meta;                                    // ints: rng [8][nd], then int64 bo [4][nd]
  size_t bytes;
};

__host__ __device__ inline AdjGeom adj_geom(int nd, int kl, int iw, int kw, int ng) {
  AdjGeom g;
  g.kl = kl;
  g.iw = iw;
  g.kw = kw;
  g.ng = ng;
  int c = 0;  // in complex units (16 bytes)
  g.p1 = c; c += iw;
  g.u5 = c; c += nd * kl;
  g.u4 = c; c += nd * kl;
  g.u2 = c; c += nd * kl;
  g.u3 = c; c += nd * kl;
  g.g5 = c; c += nd * kl;
  g.g4 = c; c += nd * kl;
  g.g3 = c; c += nd * kl;
  g.g2 = c; c += nd * kl;
  g.v2 = c; c += nd * kl * iw;
  g.x2 = c; c += kw * iw;
  g.r4 = c; c += kw * iw;
  g.x5 = c; c += iw * kw;
  g.r3 = g.x2;
  g.z5 = c; c += ng * iw * kl;
  g.q5 = c; c += ng * kl * iw;
  g.s2 = g.z5;
  int d = 2 * c;  // in doubles
  g.u1s = d; d += iw * kw;
  g.u5s = d; d += kw * iw;
  g.u3s = d; d += kw * kw;
  g.meta = d;
  g.bytes = sizeof(double) * (size_t)d + sizeof(int) * 8 * (size_t)nd + sizeof(int64_t) * 4 * (size_t)nd;
  return g;
}

__global__ __launch_bounds__(AT) void adjoint_ring_kernel(RingParams rp, const int *__restrict__ order,
                                                          PsiPtrs psi, double *gbuf,
                                                          int KLr, int IWr, int KWr, int NGr) {
  extern __shared__ double sm[];
  const int nd = rp.nd, nd3 = nd * nd * nd;
  const AdjGeom geo = adj_geom(nd, KLr, IWr, KWr, NGr);
  const int kl = geo.kl, iw = geo.iw, kw = geo.kw, ng = geo.ng;
  const FastDiv by_kw(kw), by_kl(kl), by_iw(iw), by_kliw(kl * iw), by_2kliw(2 * kl * iw);
  cplx *cs = reinterpret_cast<cplx *>(sm);
  cplx *P1 = cs + geo.p1, *u5 = cs + geo.u5, *u4 = cs + geo.u4, *u2 = cs + geo.u2, *u3 = cs + geo.u3;
  cplx *G5 = cs + geo.g5, *G4 = cs + geo.g4, *G3 = cs + geo.g3, *G2 = cs + geo.g2;
  cplx *V2 = cs + geo.v2, *X2 = cs + geo.x2, *R4 = cs + geo.r4, *X5 = cs + geo.x5, *R3 = cs + geo.r3;
  cplx *Z5 = cs + geo.z5, *Q5 = cs + geo.q5, *S2 = cs + geo.s2;
  double *U1s = sm + geo.u1s, *U5s = sm + geo.u5s, *U3s = sm + geo.u3s;
  int *rng = reinterpret_cast<int *>(sm + geo.meta);
  int64_t *bo = reinterpret_cast<int64_t *>(rng + 8 * nd);

  const int tid = threadIdx.x;
  const int core = order[blockIdx.x];  // cores longest first
  const int o24 = core / nd3, o25 = (core / (nd * nd)) % nd, o34 = (core / nd) % nd, o35 = core % nd;
  const int *J = rp.two_j;
  const int l24 = J[L24] + 2 * o24, l25 = J[L25] + 2 * o25, l35 = J[L35] + 2 * o35;
  const int d1 = rp.i_n[0];
  const int NX = rp.NX, nK2 = rp.K_n[0], nK3 = rp.K_n[1], nK4 = rp.K_n[2], nK5 = rp.K_n[3];
  const double *B = rp.B;

  for (int o = tid; o < nd; o += AT) {
    const int t5 = (o25 * nd + o35) * nd + o, t4 = (o * nd + o24) * nd + o34;
    const int t2 = (o * nd + o24) * nd + o25, t3 = (o34 * nd + o35) * nd + o;
    int n5 = rp.kr[(3 * nd3 + t5) * 2 + 1], n4 = rp.kr[(2 * nd3 + t4) * 2 + 1];
    int n2 = rp.kr[(0 * nd3 + t2) * 2 + 1], n3 = rp.kr[(1 * nd3 + t3) * 2 + 1];
    // A spin whose pair of ranges has an empty member closes no shell.
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
    bo[0 * nd + o] = rp.boff[3 * nd3 + t5];
    bo[1 * nd + o] = rp.boff[2 * nd3 + t4];
    bo[2 * nd + o] = rp.boff[0 * nd3 + t2];
    bo[3 * nd + o] = rp.boff[1 * nd3 + t3];
  }
  for (int q = tid; q < 4 * nd * kl; q += AT) G5[q] = cplx{0.0, 0.0};  // G5, G4, G3, G2 are adjacent
  for (int q = tid; q < iw; q += AT)
    P1[q] = q < d1 ? cscale(load_c(psi.p[0], q), __builtin_sqrt((double)(rp.i_lo2[0] + 2 * q + 1)))
                   : cplx{0.0, 0.0};
  __syncthreads();
  // Contracted boosters u_e(k; l) of this core: edge slot s = 0 u5 (l45), 1 u4 (l45), 2 u2 (l23),
  // 3 u3 (l23); psi of edges 5, 4, 2, 3.
  for (int q = tid; q < 4 * nd * kl; q += AT) {
    const int s = q / (nd * kl), o = (q / kl) % nd, k = q % kl;
    const int ri = s == 0 ? 0 : s == 1 ? 2 : s == 2 ? 4 : 6;
    const int lo = rng[ri * nd + o], n = rng[(ri + 1) * nd + o];
    const int e = s == 0 ? 4 : s == 1 ? 3 : s == 2 ? 1 : 2;  // boundary index of the edge
    cplx u{0.0, 0.0};
    if (k < n) {
      const double w = (double)(lo + 2 * k + 1);
      const int64_t off = bo[s * nd + o];
      for (int i = 0; i < rp.i_n[e]; ++i) {
        const cplx p = cscale(load_c(psi.p[e], i), __builtin_sqrt((double)(rp.i_lo2[e] + 2 * i + 1)));
        u = cfma(u, p, B[off + (int64_t)i * n + k] * w);
      }
    }
    cs[(s == 0 ? geo.u5 : s == 1 ? geo.u4 : s == 2 ? geo.u2 : geo.u3) + o * kl + k] = u;
  }
  // Core windows of k4 (over l45), k3 (over l23), k5 (over l45) and k2 (over l23).
  int w4lo = 1 << 30, w4hi = -1, w3lo = 1 << 30, w3hi = -1, w5lo = 1 << 30, w2lo = 1 << 30;
  int w5hi = -1, w2hi = -1;
  for (int o = 0; o < nd; ++o) {
    if (rng[3 * nd + o] > 0) {
      w4lo = imin(w4lo, rng[2 * nd + o]);
      w4hi = imax(w4hi, rng[2 * nd + o] + 2 * (rng[3 * nd + o] - 1));
      w5lo = imin(w5lo, rng[0 * nd + o]);
      w5hi = imax(w5hi, rng[0 * nd + o] + 2 * (rng[1 * nd + o] - 1));
    }
    if (rng[7 * nd + o] > 0) {
      w3lo = imin(w3lo, rng[6 * nd + o]);
      w3hi = imax(w3hi, rng[6 * nd + o] + 2 * (rng[7 * nd + o] - 1));
      w2lo = imin(w2lo, rng[4 * nd + o]);
      w2hi = imax(w2hi, rng[4 * nd + o] + 2 * (rng[5 * nd + o] - 1));
    }
  }
  const bool live = w4hi >= 0 && w3hi >= 0;
  const int nw4 = live ? (w4hi - w4lo) / 2 + 1 : 0, nw3 = live ? (w3hi - w3lo) / 2 + 1 : 0;
  const int nw5 = live ? (w5hi - w5lo) / 2 + 1 : 0, nw2 = live ? (w2hi - w2lo) / 2 + 1 : 0;
  const int64_t u3base = (((int64_t)o24 * nd + o34) * nd + o35) * NX;
  const int xhi_g = rp.X_lo2 + 2 * (NX - 1);
  // x closes (i1 l25 x) for some i1, (k4 l35 x) and (k3 l24 x) for some k4, k3 of the windows.
  int xlo = 0, xhi = -1;
  if (live) {
    const int i1lo = rp.i_lo2[0], i1hi = rp.i_lo2[0] + 2 * (d1 - 1);
    xlo = imax(rp.X_lo2, l25 > i1hi ? l25 - i1hi : (i1lo > l25 ? i1lo - l25 : ((l25 - i1lo) & 1)));
    xhi = imin(xhi_g, i1hi + l25);
  }
  // x values with both core windows non-empty, in increasing order.
  auto active = [&](int x) {
    return imax(w4lo, iabs(l35 - x)) <= imin(w4hi, l35 + x) && imax(w3lo, iabs(l24 - x)) <= imin(w3hi, l24 + x);
  };
  auto next_active = [&](int x) {
    while (x <= xhi && !active(x)) x += 2;
    return x;
  };
  // Table slices of an x (U1(i1, k5), U5(k2, i1), U3(k4, k3) over the core windows), read into
  // registers one x ahead of their use: this thread's entries q = tid (U1, U5) and tid, tid + AT
  // (U3) of the slices (iw kw <= AT and kw kw <= 2 AT, checked at launch).
  double pf1 = 0.0, pf5 = 0.0, pf3[2] = {0.0, 0.0};
  auto fetch = [&](int x) {
    const int xg = (x - rp.X_lo2) / 2;
    pf1 = pf5 = 0.0;
    if (tid < iw * kw) {
      const int i = by_kw(tid), p = tid - i * kw;
      if (i < d1 && p < nw5)
        pf1 = rp.U1[(((int64_t)o25 * NX + xg) * d1 + i) * nK5 + ((w5lo - rp.K_lo2[3]) >> 1) + p];
      if (i < d1 && p < nw2)
        pf5 = rp.U5[(((int64_t)o25 * NX + xg) * nK2 + ((w2lo - rp.K_lo2[0]) >> 1) + p) * d1 + i];
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = tid + h * AT, p4 = by_kw(q), p3 = q - p4 * kw;
      pf3[h] = 0.0;
      if (q < kw * kw && p4 < nw4 && p3 < nw3)
        pf3[h] = rp.U3[((u3base + xg) * nK4 + ((w4lo - rp.K_lo2[2]) >> 1) + p4) * nK3 +
                       ((w3lo - rp.K_lo2[1]) >> 1) + p3];
    }
  };
  int x = live ? next_active(xlo) : xhi + 2;
  if (x <= xhi) fetch(x);
  while (x <= xhi) {
    const int a4 = imax(w4lo, iabs(l35 - x)), b4 = imin(w4hi, l35 + x);
    const int a3 = imax(w3lo, iabs(l24 - x)), b3 = imin(w3hi, l24 + x);
    const int xg = (x - rp.X_lo2) / 2;
    const int xn = next_active(x + 2);
    __syncthreads();  // previous x's readers are done
    if (tid < iw * kw) {
      const int i = by_kw(tid), p = tid - i * kw;
      U1s[i * kw + p] = pf1;
      U5s[p * iw + i] = pf5;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (tid + h * AT < kw * kw) U3s[tid + h * AT] = pf3[h];
    if (xn <= xhi) fetch(xn);  // in flight during this x's stages
    __syncthreads();
    // V2_o(k3, i1) = sum_k2 U4(k3, k2; o) u2(k2; o) U5(k2, i1) for every l23 = o.
    for (int q = tid; q < nd * kl * iw; q += AT) {
      const int o = by_kliw(q), rr = q - o * (kl * iw), k3i = by_iw(rr), i = rr - k3i * iw;
      const int lo2 = rng[4 * nd + o], n2 = rng[5 * nd + o], lo3 = rng[6 * nd + o], n3 = rng[7 * nd + o];
      cplx v{0.0, 0.0};
      if (k3i < n3 && i < d1) {
        const int k3g = (lo3 + 2 * k3i - rp.K_lo2[1]) >> 1;
        const double *u4r = rp.U4 + ((((int64_t)o * nd + o24) * NX + xg) * nK3 + k3g) * nK2 +
                            ((lo2 - rp.K_lo2[0]) >> 1);
        const int p2 = (lo2 - w2lo) >> 1;
#pragma unroll 4
        for (int k2i = 0; k2i < n2; ++k2i)
          v = cfma(v, u2[o * kl + k2i], u4r[k2i] * U5s[(p2 + k2i) * iw + i]);
      }
      V2[q] = v;
    }
    __syncthreads();
    // X2(k3, i1) = sum_o u3(k3; o) V2_o(k3, i1), k3 over the core window.
    for (int q = tid; q < kw * iw; q += AT) {
      const int p3 = by_iw(q), i = q - p3 * iw;
      cplx v{0.0, 0.0};
      if (p3 < nw3) {
        const int k3 = w3lo + 2 * p3;
        for (int o = 0; o < nd; ++o) {
          const int lo3 = rng[6 * nd + o], n3 = rng[7 * nd + o], k3i = (k3 - lo3) >> 1;
          if (n3 > 0 && k3 >= lo3 && k3i < n3) v = cadd(v, cmul(u3[o * kl + k3i], V2[(o * kl + k3i) * iw + i]));
        }
      }
      X2[q] = v;
    }
    __syncthreads();
    // R4(k4, i1) = sum_k3 U3(k4, k3) X2(k3, i1); X5 cleared.
    for (int q = tid; q < kw * iw; q += AT) {
      const int p4 = by_iw(q), i = q - p4 * iw;
      cplx v{0.0, 0.0};
      if (p4 < nw4)
        for (int p3 = 0; p3 < nw3; ++p3) v = cfma(v, X2[p3 * iw + i], U3s[p4 * kw + p3]);
      R4[q] = v;
      X5[q] = cplx{0.0, 0.0};
    }
    __syncthreads();
    // Left half, the l45 = o values ng at a time.
    for (int og = 0; og < nd; og += ng) {
      const int gn = imin(ng, nd - og);
      // Z5_o(i1, k4) = p1(i1) sum_k5 U1(i1, k5) u5(k5) U2(k5, k4);  Q5_o(k5, i1) = sum_k4 U2(k5, k4)
      // u4(k4) R4(k4, i1), for every o of the group.
      for (int q = tid; q < gn * 2 * iw * kl; q += AT) {
        const int gi = by_2kliw(q), r = q - gi * (2 * iw * kl), o = og + gi;
        const int lo5 = rng[0 * nd + o], n5 = rng[1 * nd + o], lo4 = rng[2 * nd + o], n4 = rng[3 * nd + o];
        const int p5 = (lo5 - w5lo) >> 1, p4 = (lo4 - w4lo) >> 1;
        const double *u2b = rp.U2 + ((((int64_t)o35 * nd + o) * NX + xg) * nK5 + ((lo5 - rp.K_lo2[3]) >> 1)) * nK4 +
                            ((lo4 - rp.K_lo2[2]) >> 1);
        cplx v{0.0, 0.0};
        if (r < iw * kl) {
          const int i = by_kl(r), k4i = r - i * kl;
          if (i < d1 && k4i < n4) {
            const double *u2c = u2b + k4i;  // column k4i of U2, advanced a row (nK4) per k5
#pragma unroll 4
            for (int k5i = 0; k5i < n5; ++k5i, u2c += nK4)
              v = cfma(v, u5[o * kl + k5i], U1s[i * kw + p5 + k5i] * *u2c);
            v = cmul(v, P1[i]);
          }
          Z5[gi * iw * kl + r] = v;
        } else {
          const int r2 = r - iw * kl, k5i = by_iw(r2), i = r2 - k5i * iw;
          if (k5i < n5 && i < d1) {
            const double *u2r = u2b + (int64_t)k5i * nK4;  // row k5i of U2
#pragma unroll 4
            for (int k4i = 0; k4i < n4; ++k4i)
              v = cadd(v, cmul(u4[o * kl + k4i], cscale(R4[(p4 + k4i) * iw + i], u2r[k4i])));
          }
          Q5[gi * kl * iw + r2] = v;
        }
      }
      __syncthreads();
      // G4_o(k4) += sum_i1 Z5_o(i1, k4) R4(k4, i1);  G5_o(k5) += sum_i1 p1(i1) U1(i1, k5) Q5_o(k5, i1);
      // X5(i1, k4) += Z5_o(i1, k4) u4_o(k4), the group's o in increasing order.
      for (int q = tid; q < gn * 2 * kl + iw * kw; q += AT) {
        if (q < gn * kl) {
          const int gi = by_kl(q), k4i = q - gi * kl, o = og + gi;
          const int n4 = rng[3 * nd + o], p4 = (rng[2 * nd + o] - w4lo) >> 1;
          if (k4i < n4) {
            cplx v{0.0, 0.0};
            for (int i = 0; i < d1; ++i) v = cadd(v, cmul(Z5[(gi * iw + i) * kl + k4i], R4[(p4 + k4i) * iw + i]));
            G4[o * kl + k4i] = cadd(G4[o * kl + k4i], v);
          }
        } else if (q < gn * 2 * kl) {
          const int qq = q - gn * kl, gi = by_kl(qq), k5i = qq - gi * kl, o = og + gi;
          const int n5 = rng[1 * nd + o], p5 = (rng[0 * nd + o] - w5lo) >> 1;
          if (k5i < n5) {
            cplx v{0.0, 0.0};
            for (int i = 0; i < d1; ++i)
              v = cadd(v, cmul(P1[i], cscale(Q5[(gi * kl + k5i) * iw + i], U1s[i * kw + p5 + k5i])));
            G5[o * kl + k5i] = cadd(G5[o * kl + k5i], v);
          }
        } else {
          const int r = q - gn * 2 * kl, i = by_kw(r), p = r - i * kw;
          if (i < d1) {
            cplx v = X5[r];
            for (int gi = 0; gi < gn; ++gi) {
              const int o = og + gi, n4 = rng[3 * nd + o], k4i = p - ((rng[2 * nd + o] - w4lo) >> 1);
              if (k4i >= 0 && k4i < n4) v = cadd(v, cmul(Z5[(gi * iw + i) * kl + k4i], u4[o * kl + k4i]));
            }
            X5[r] = v;
          }
        }
      }
      __syncthreads();
    }
    // R3(i1, k3) = sum_k4 X5(i1, k4) U3(k4, k3)
    for (int q = tid; q < iw * kw; q += AT) {
      const int i = by_kw(q), p3 = q - i * kw;
      cplx v{0.0, 0.0};
      if (p3 < nw3)
        for (int p4 = 0; p4 < nw4; ++p4) v = cfma(v, X5[i * kw + p4], U3s[p4 * kw + p3]);
      R3[q] = v;
    }
    __syncthreads();
    // Right half, the l23 = o values ng at a time.
    for (int og = 0; og < nd; og += ng) {
      const int gn = imin(ng, nd - og);
      // G3_o(k3) += sum_i1 R3(i1, k3) V2_o(k3, i1);  S2_o(i1, k2) = sum_k3 R3(i1, k3) u3(k3) U4(k3, k2)
      for (int q = tid; q < gn * (kl + iw * kl); q += AT) {
        if (q < gn * kl) {
          const int gi = by_kl(q), k3i = q - gi * kl, o = og + gi;
          const int n3 = rng[7 * nd + o], p3 = (rng[6 * nd + o] - w3lo) >> 1;
          if (k3i < n3) {
            cplx v{0.0, 0.0};
            for (int i = 0; i < d1; ++i) v = cadd(v, cmul(R3[i * kw + p3 + k3i], V2[(o * kl + k3i) * iw + i]));
            G3[o * kl + k3i] = cadd(G3[o * kl + k3i], v);
          }
        } else {
          const int qq = q - gn * kl, gi = by_kliw(qq), r = qq - gi * (iw * kl), o = og + gi;
          const int lo2 = rng[4 * nd + o], n2 = rng[5 * nd + o], lo3 = rng[6 * nd + o], n3 = rng[7 * nd + o];
          const int p3 = (lo3 - w3lo) >> 1;
          const int i = by_kl(r), k2i = r - i * kl;
          cplx v{0.0, 0.0};
          if (i < d1 && k2i < n2) {
            const double *u4b = rp.U4 + ((((int64_t)o * nd + o24) * NX + xg) * nK3 + ((lo3 - rp.K_lo2[1]) >> 1)) * nK2 +
                                ((lo2 - rp.K_lo2[0]) >> 1);
            const double *u4c = u4b + k2i;  // column k2i of U4, advanced a row (nK2) per k3
#pragma unroll 4
            for (int k3i = 0; k3i < n3; ++k3i, u4c += nK2)
              v = cadd(v, cmul(u3[o * kl + k3i], cscale(R3[i * kw + p3 + k3i], *u4c)));
          }
          S2[gi * iw * kl + r] = v;
        }
      }
      __syncthreads();
      // G2_o(k2) += sum_i1 S2_o(i1, k2) U5(k2, i1)
      for (int q = tid; q < gn * kl; q += AT) {
        const int gi = by_kl(q), k2i = q - gi * kl, o = og + gi;
        const int n2 = rng[5 * nd + o], p2 = (rng[4 * nd + o] - w2lo) >> 1;
        if (k2i < n2) {
          cplx v{0.0, 0.0};
          for (int i = 0; i < d1; ++i) v = cfma(v, S2[(gi * iw + i) * kl + k2i], U5s[(p2 + k2i) * iw + i]);
          G2[o * kl + k2i] = cadd(G2[o * kl + k2i], v);
        }
      }
      __syncthreads();
    }
    x = xn;
  }
  __syncthreads();
  // gbuf[core][slot][o][k], slots in booster-edge order: 0 G2, 1 G3, 2 G4, 3 G5.
  double *out = gbuf + (int64_t)core * 4 * nd * kl * 2;
  for (int q = tid; q < 4 * nd * kl; q += AT) {
    const int s = q / (nd * kl), r = q % (nd * kl);
    const cplx v = (s == 0 ? G2 : s == 1 ? G3 : s == 2 ? G4 : G5)[r];
    out[2 * q] = v.re;
    out[2 * q + 1] = v.im;
  }
}

// One thread per booster entry (edge e, triple t, row i, column k): the sum over the nd^2 cores
// that contain the block, in a fixed order, times g (2k+1) p_e(i).
__global__ void adjoint_ring_reduce_kernel(RingParams rp, PsiPtrs psi, const double *gbuf, int kl,
                                           double gre, double gim, double *grad_b) {
  const int nd = rp.nd, nd3 = nd * nd * nd;
  const int64_t total = rp.boff[4 * nd3];
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  int lo = 0, hi = 4 * nd3 - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (rp.boff[mid] <= idx) lo = mid; else hi = mid - 1;
  }
  const int e = lo / nd3, t = lo % nd3;
  const int kn = rp.kr[(e * nd3 + t) * 2 + 1], klo = rp.kr[(e * nd3 + t) * 2];
  const int64_t within = idx - rp.boff[lo];
  const int i = (int)(within / kn), k = (int)(within % kn);
  const int a = t / (nd * nd), b = (t / nd) % nd, c = t % nd;
  // The block's triple in shell coordinates and the core coordinates (o24, o25, o34, o35) that
  // run free: e2 (l23, l24, l25): o = a, (o24, o25) = (b, c), free (o34, o35);
  // e3 (l34, l35, l23): o = c, (o34, o35) = (a, b), free (o24, o25);
  // e4 (l45, l24, l34): o = a, (o24, o34) = (b, c), free (o25, o35);
  // e5 (l25, l35, l45): o = c, (o25, o35) = (a, b), free (o24, o34).
  const int o = (e == 0 || e == 2) ? a : c;
  double sre = 0.0, sim = 0.0;
  for (int f = 0; f < nd * nd; ++f) {
    const int p = f / nd, q = f % nd;
    int o24, o25, o34, o35;
    if (e == 0) { o24 = b; o25 = c; o34 = p; o35 = q; }
    else if (e == 1) { o34 = a; o35 = b; o24 = p; o25 = q; }
    else if (e == 2) { o24 = b; o34 = c; o25 = p; o35 = q; }
    else { o25 = a; o35 = b; o24 = p; o34 = q; }
    const int core = ((o24 * nd + o25) * nd + o34) * nd + o35;
    const double *g = gbuf + (((int64_t)core * 4 + e) * nd + o) * kl * 2 + 2 * k;
    sre += g[0];
    sim += g[1];
  }
  const cplx pe = cscale(load_c(psi.p[e + 1], i), __builtin_sqrt((double)(rp.i_lo2[e + 1] + 2 * i + 1)));
  const cplx v = cmul(cscale(cmul(pe, cplx{sre, sim}), (double)(klo + 2 * k + 1)), cplx{gre, gim});
  grad_b[2 * idx] = v.re;
  grad_b[2 * idx + 1] = v.im;
}

}  // namespace

void adjoint_ring_dims(const Plan &p, int &kl, int &iw, int &kw, int &ng) {
  const int nd = p.nd, nd3 = nd * nd * nd;
  kl = std::max(1, p.kmax);
  iw = std::max(1, p.i[0].n);
  kw = 1;
  // Widest window of k5 and k4 over l45, and of k3 and k2 over l23, of any core (spins whose pair
  // of ranges has an empty member left out, as in the kernel).
  for (int core = 0; core < nd * nd3; ++core) {
    const int o24 = core / nd3, o25 = (core / (nd * nd)) % nd, o34 = (core / nd) % nd, o35 = core % nd;
    int lo[4] = {1 << 30, 1 << 30, 1 << 30, 1 << 30}, hi[4] = {-1, -1, -1, -1};
    for (int o = 0; o < nd; ++o) {
      const int t5 = (o25 * nd + o35) * nd + o, t4 = (o * nd + o24) * nd + o34;
      const int t2 = (o * nd + o24) * nd + o25, t3 = (o34 * nd + o35) * nd + o;
      const int n5 = p.kr[(3 * nd3 + t5) * 2 + 1], n4 = p.kr[(2 * nd3 + t4) * 2 + 1];
      const int n2 = p.kr[(0 * nd3 + t2) * 2 + 1], n3 = p.kr[(1 * nd3 + t3) * 2 + 1];
      const int l5 = p.kr[(3 * nd3 + t5) * 2], l4 = p.kr[(2 * nd3 + t4) * 2];
      const int l2 = p.kr[(0 * nd3 + t2) * 2], l3 = p.kr[(1 * nd3 + t3) * 2];
      if (n5 > 0 && n4 > 0) {
        lo[0] = std::min(lo[0], l5); hi[0] = std::max(hi[0], l5 + 2 * (n5 - 1));
        lo[1] = std::min(lo[1], l4); hi[1] = std::max(hi[1], l4 + 2 * (n4 - 1));
      }
      if (n2 > 0 && n3 > 0) {
        lo[2] = std::min(lo[2], l3); hi[2] = std::max(hi[2], l3 + 2 * (n3 - 1));
        lo[3] = std::min(lo[3], l2); hi[3] = std::max(hi[3], l2 + 2 * (n2 - 1));
      }
    }
    for (int q = 0; q < 4; ++q)
      if (hi[q] >= 0) kw = std::max(kw, (hi[q] - lo[q]) / 2 + 1);
  }
  // Spins per group of the two halves: as many as keep two workgroups on a CU (half the LDS),
  // or, when even one does not, as many as fit one workgroup.
  const size_t two = kAdjRingMaxLds / 2 - 1024;
  const size_t cap = adj_geom(nd, kl, iw, kw, 1).bytes <= two ? two : kAdjRingMaxLds;
  ng = 1;
  while (ng < nd && adj_geom(nd, kl, iw, kw, ng + 1).bytes <= cap) ++ng;
  // Each thread holds one U1/U5 entry and two U3 entries of the next x's slices.
  if (iw * kw > AT || kw * kw > 2 * AT) kl = 0;
}

void adjoint_ring_order(const Plan &p, std::vector<int> &order) {
  const int nd = p.nd, nd3 = nd * nd * nd, ncore = nd * nd3;
  const int *J = p.two_j;
  const int i1lo = p.i[0].lo2, i1hi = p.i[0].lo2 + 2 * (p.i[0].n - 1);
  const int xhi_g = p.X.lo2 + 2 * (p.X.n - 1);
  std::vector<double> cost(ncore, 0.0);
  for (int core = 0; core < ncore; ++core) {
    const int o24 = core / nd3, o25 = (core / (nd * nd)) % nd, o34 = (core / nd) % nd, o35 = core % nd;
    int w4lo = 1 << 30, w4hi = -1, w3lo = 1 << 30, w3hi = -1, width = 0;
    for (int o = 0; o < nd; ++o) {
      const int t5 = (o25 * nd + o35) * nd + o, t4 = (o * nd + o24) * nd + o34;
      const int t2 = (o * nd + o24) * nd + o25, t3 = (o34 * nd + o35) * nd + o;
      const int n5 = p.kr[(3 * nd3 + t5) * 2 + 1], n4 = p.kr[(2 * nd3 + t4) * 2 + 1];
      const int n2 = p.kr[(0 * nd3 + t2) * 2 + 1], n3 = p.kr[(1 * nd3 + t3) * 2 + 1];
      if (n5 > 0 && n4 > 0) {
        const int l4 = p.kr[(2 * nd3 + t4) * 2];
        w4lo = std::min(w4lo, l4);
        w4hi = std::max(w4hi, l4 + 2 * (n4 - 1));
        width += n5 + n4;
      }
      if (n2 > 0 && n3 > 0) {
        const int l3 = p.kr[(1 * nd3 + t3) * 2];
        w3lo = std::min(w3lo, l3);
        w3hi = std::max(w3hi, l3 + 2 * (n3 - 1));
        width += n2 + n3;
      }
    }
    if (w4hi < 0 || w3hi < 0) continue;
    const int l24 = J[L24] + 2 * o24, l25 = J[L25] + 2 * o25, l35 = J[L35] + 2 * o35;
    const int xlo = std::max(p.X.lo2, l25 > i1hi ? l25 - i1hi : (i1lo > l25 ? i1lo - l25 : ((l25 - i1lo) & 1)));
    const int xhi = std::min(xhi_g, i1hi + l25);
    int nx = 0;
    for (int x = xlo; x <= xhi; x += 2)
      if (std::max(w4lo, std::abs(l35 - x)) <= std::min(w4hi, l35 + x) &&
          std::max(w3lo, std::abs(l24 - x)) <= std::min(w3hi, l24 + x))
        ++nx;
    cost[core] = (double)nx * (1 + width);
  }
  order.resize(ncore);
  for (int k = 0; k < ncore; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
}

size_t adjoint_ring_smem(int nd, int kl, int iw, int kw, int ng) { return adj_geom(nd, kl, iw, kw, ng).bytes; }
size_t adjoint_ring_gbuf_bytes(int nd, int kl) {
  return sizeof(double) * 2 * (size_t)nd * nd * nd * nd * 4 * nd * kl;
}

hipError_t adjoint_ring_init_attributes() {
  return hipFuncSetAttribute((const void *)adjoint_ring_kernel,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kAdjRingMaxLds);
}

hipError_t launch_adjoint_ring(const RingParams &rp, int kl, int iw, int kw, int ng,
                               const int *order, const double *const psi[5], double *gbuf,
                               int64_t total, double gre, double gim, double *grad_b, hipStream_t s) {
  PsiPtrs pp;
  for (int a = 0; a < 5; ++a) pp.p[a] = psi[a];
  const int nd = rp.nd;
  const size_t bytes = adj_geom(nd, kl, iw, kw, ng).bytes;
  if (nd > kAdjRingMaxNd || ng < 1 || bytes > kAdjRingMaxLds) return hipErrorInvalidValue;
  if (iw * kw > AT || kw * kw > 2 * AT) return hipErrorInvalidValue;  // the slices' prefetch
  adjoint_ring_kernel<<<nd * nd * nd * nd, AT, bytes, s>>>(rp, order, pp, gbuf, kl, iw, kw, ng);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (total <= 0) return hipSuccess;
  adjoint_ring_reduce_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(rp, pp, gbuf, kl, gre, gim,
                                                                            grad_b);
  return hipGetLastError();
}

}  // namespace eprl
