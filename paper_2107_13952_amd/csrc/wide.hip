// Factorised ("ring") evaluation of the vertex tensor for intertwiner dimensions up to 16, with
// every stage on FP64 matrix-core tiles and the (i5, i4) and (i3, i2) pairs packed densely.
//
// The sum regrouped by linearity (eq. (vertex-ampl) with eq. (15j); the same regrouping as the
// 8-wide kernel of ring.hip, which describes the chain U1 M5 U2 M4 U3 M3 U4 M2 U5): for a fixed
// i1, core (l24, l25, l34, l35) and x of eq. (15j),
//   T5(l45; i5, k4) = sum_k5 M5(i5, k5) [U1(k5) U2(k5, k4)]          one 16x16 tile per l45
//   T2(l23; i2, k3) = sum_k2 M2(i2, k2) [U5(k2) U4(k3, k2)]          one 16x16 tile per l23
//   G(i5, i4; k4)   = sum_l45 T5(l45; i5, k4) M4(l45; i4, k4)        one 16x16 tile per k4
//   H(k3; i3, i2)   = sum_l23 M3(l23; i3, k3) T2(l23; i2, k3)        one 16x16 tile per k3
//   P(rho; k3)      = sum_k4 G(rho; k4) U3(k4, k3)                    rho = i5 d4 + i4
//   A(i1; rho, sig) += sum_k3 P(rho; k3) H(k3; sig)                   sig = i3 d2 + i2
// (M_e = (2k_e + 1) B_e, U = signed 6j tables, k4 / k3 over the core's windows).  All six are
// v_mfma_f64_16x16x4 contractions; the last one, a rank-n3 update of the whole R x C slice
// (R = d5 d4, C = d3 d2, padded to multiples of 16 only), is where the work is.
// Lane layout of v_mfma_f64_16x16x4 (lane l = 16 g + c, measured on the device): operand A[c][g],
// operand B[g][c], result register r = D[g + 4 r][c].
//
// One workgroup of 8 wavefronts owns a block of rows of A(i1; rho, sig) (all rows when the
// slice's tiles fit in 14 accumulator tiles per wavefront, else the rows split into row blocks)
// for a chunk of cores, and keeps it in MFMA accumulators.  LDS holds the T5/T2 tiles, G (then
// P, in place) for the block's rows, H, the U3 slice of the current x and, when they fit, the
// core's weighted booster blocks; the other 6j values (and booster entries otherwise) are read
// from global memory (L1/L2) straight into the MFMA operands.  Stages are separated by workgroup
// barriers.
#include <type_traits>

#include "eprl_internal.hpp"

namespace eprl {

namespace {

// Device buffers reached through pointers held in memory (the batch kernel's parameter array)
// are read and written as global memory: the compiler then emits global rather than generic
// accesses, and waits on LDS reads no longer wait for them (a generic access counts for both).
__device__ __forceinline__ double ldg(const double *p) {
  return *(const __attribute__((address_space(1))) double *)p;
}
__device__ __forceinline__ void stg(double *p, double v) { *(__attribute__((address_space(1))) double *)p = v; }

typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int WT = 512;          // threads per workgroup
constexpr int WW = WT / 64;      // wavefronts per workgroup
constexpr int kMaxAcc = 14;      // accumulator tiles per wavefront
constexpr int kAccGroup = 3;     // accumulator tiles per branch of the A update
constexpr size_t kLdsBytes = 160 * 1024;

__device__ __forceinline__ int iabs(int v) { return v < 0 ? -v : v; }
__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }
__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

__device__ __forceinline__ d4v mfma(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// LDS geometry of one configuration (all sizes in doubles).
struct WideGeom {
  int R, C, RT, CT, RTb, GS, HS;
  int t5, t2, g, h, u3, mb, meta;  // offsets
};

// Row stride of the U3 slice in LDS (rows: k4 positions, columns: k3 positions 0..31; the two
// halves of a row read by one matrix-core operand fall on opposite halves of the banks).
constexpr int kU3S = 48;

// stg: the core's four weighted booster blocks are staged in LDS (16 x 16 each per spin value,
// zero outside the block) for the operands of T5 / T2 and G / H.
__host__ __device__ inline WideGeom wide_geom(int nd, const int *i_n, int kw, int nrb, bool stg) {
  WideGeom w;
  w.R = i_n[4] * i_n[3];
  w.C = i_n[2] * i_n[1];
  w.RT = (w.R + 15) / 16;
  w.CT = (w.C + 15) / 16;
  w.RTb = (w.RT + nrb - 1) / nrb;
  w.GS = kw + 1;
  w.HS = w.CT * 16 + 1;
  w.t5 = 0;
  w.t2 = w.t5 + nd * 256;
  w.g = w.t2 + nd * 256;
  w.h = w.g + w.RTb * 16 * w.GS;
  w.u3 = w.h + kw * w.HS;
  w.mb = w.u3 + kw * kU3S;
  w.meta = w.mb + (stg ? 4 * nd * 256 : 0);
  return w;
}

// Bytes of LDS: the double buffers plus the per-core range table (8 ints per spin value) and
// booster offsets (4 int64 per spin value).
__host__ __device__ inline size_t wide_bytes(int nd, const int *i_n, int kw, int nrb, bool stg) {
  const WideGeom w = wide_geom(nd, i_n, kw, nrb, stg);
  return sizeof(double) * (size_t)w.meta + sizeof(int) * 8 * (size_t)nd + sizeof(int64_t) * 4 * (size_t)nd;
}

// One work item: cores [bounds[i1][chunk], bounds[i1][chunk + 1]) of rp, boundary intertwiner
// i1 = n1, row block rb of A(i1; rho, sig).
template <bool STG>
__device__ void wide_item(const RingParams &rp, int chunk_index, int n1, int rb, double *smem) {
  const int nd = rp.nd, nd3 = nd * nd * nd;
  const int d1 = rp.i_n[0], d2 = rp.i_n[1], d3 = rp.i_n[2], d4 = rp.i_n[3], d5 = rp.i_n[4];
  const int KW = rp.kw;
  const WideGeom geo = wide_geom(nd, rp.i_n, KW, rp.nrb, STG);
  const int rt0 = rb * geo.RTb;
  const int rtn = imin(geo.RTb, geo.RT - rt0);  // row tiles of this block
  if (rtn <= 0) return;                          // uniform over the workgroup
  const int rho0 = rt0 * 16, nrow = rtn * 16;
  const int ntile = rtn * geo.CT;                // accumulator tiles of the block
  const int GS = geo.GS, HS = geo.HS, CT = geo.CT;
  double *T5s = smem + geo.t5;    // [l45][i5][k4 - lo4(l45)]
  double *T2s = smem + geo.t2;    // [l23][i2][k3 - lo3(l23)]
  double *Gs = smem + geo.g;      // [rho - rho0][k4 position], then P: [rho - rho0][k3 position]
  double *Hs = smem + geo.h;      // [k3 position][sig]
  double *U3s = smem + geo.u3;    // [k4 position][k3 position]: U3 at x inside the active windows, else 0
  double *Mb = smem + geo.mb;     // [slot: M5, M4, M2, M3][spin value][i][k - lo], when STG
  int *rng = reinterpret_cast<int *>(smem + geo.meta);             // [8][nd]
  int64_t *bo = reinterpret_cast<int64_t *>(rng + 8 * nd);         // [4][nd]

  // The wavefront index read through a scalar register, so that branches on it are uniform.
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, g = l >> 4,
            c = l & 15;
  const int ntw = (ntile - w + WW - 1) / WW;  // accumulator tiles held by this wavefront
  const int ctm = (2048 + CT - 1) / CT;          // t / CT = (t * ctm) >> 11 for t < 128
  const int *J = rp.two_j;
  const int two_i1 = rp.i_lo2[0] + 2 * n1;
  const int NX = rp.NX, nK2 = rp.K_n[0], nK3 = rp.K_n[1], nK4 = rp.K_n[2], nK5 = rp.K_n[3];
  const int xhi_g = rp.xhi2, tnd = rp.tnd;
  const double *B = rp.B;

  d4v acc[kMaxAcc];
#pragma unroll
  for (int j = 0; j < kMaxAcc; ++j) acc[j] = d4v{0.0, 0.0, 0.0, 0.0};
  // Rows and columns of G / P and H that the stages never write (padding of the last tile)
  // must read as zeros.
  for (int q = tid; q < nrow * GS; q += WT) Gs[q] = 0.0;
  for (int q = tid; q < KW * HS; q += WT) Hs[q] = 0.0;

  const int c0 = rp.bounds[(int64_t)n1 * (rp.nchunk + 1) + chunk_index];
  const int c1 = rp.bounds[(int64_t)n1 * (rp.nchunk + 1) + chunk_index + 1];
  for (int core = c0; core < c1; ++core) {
    // Core index ((l24 * nd + l25) * nd + l34) * nd + l35 in offsets from the lowest spins.
    const int o24 = core / nd3, o25 = (core / (nd * nd)) % nd, o34 = (core / nd) % nd, o35 = core % nd;
    const int l24 = J[L24] + 2 * o24, l25 = J[L25] + 2 * o25, l35 = J[L35] + 2 * o35;
    __syncthreads();  // previous readers of rng / bo (and of the LDS tiles) are done
    for (int o = tid; o < nd; o += WT) {
      const int t5 = (o25 * nd + o35) * nd + o, t4 = (o * nd + o24) * nd + o34;
      const int t2 = (o * nd + o24) * nd + o25, t3 = (o34 * nd + o35) * nd + o;
      int n5 = rp.kr[(3 * nd3 + t5) * 2 + 1], n4 = rp.kr[(2 * nd3 + t4) * 2 + 1];
      int n2 = rp.kr[(0 * nd3 + t2) * 2 + 1], n3 = rp.kr[(1 * nd3 + t3) * 2 + 1];
      // A spin whose pair of ranges has an empty member does not contribute.
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
      bo[0 * nd + o] = rp.boff[3 * nd3 + t5];  // M5
      bo[1 * nd + o] = rp.boff[2 * nd3 + t4];  // M4
      bo[2 * nd + o] = rp.boff[0 * nd3 + t2];  // M2
      bo[3 * nd + o] = rp.boff[1 * nd3 + t3];  // M3
    }
    __syncthreads();
    if (STG) {
      // Weighted booster blocks (2k+1) B of this core, zero outside each block: block so =
      // slot nd + o (slot 0 M5, 1 M4, 2 M2, 3 M3), entry (i, k) = thread (tid >> 4 & 15, tid & 15)
      // of blocks tid >> 8, + 2, + 4, ...; the reads of eight blocks are in flight together.
      {
        const int i = (tid >> 4) & 15, k = tid & 15;
        constexpr int kSB = 8;
        for (int so0 = tid >> 8; so0 < 4 * nd; so0 += 2 * kSB) {
          double v[kSB], wt[kSB];
#pragma unroll
          for (int j = 0; j < kSB; ++j) {
            const int so = so0 + 2 * j;
            const int slot = (so >= nd) + (so >= 2 * nd) + (so >= 3 * nd), o = so - slot * nd;
            const int lo = rng[2 * slot * nd + o], n = rng[(2 * slot + 1) * nd + o];
            const int di = slot == 0 ? d5 : slot == 1 ? d4 : slot == 2 ? d2 : d3;
            wt[j] = (double)(lo + 2 * k + 1);
            v[j] = 0.0;
            if (so < 4 * nd && i < di && k < n) v[j] = ldg(B + bo[slot * nd + o] + (int64_t)i * n + k);
          }
#pragma unroll
          for (int j = 0; j < kSB; ++j)
            if (so0 + 2 * j < 4 * nd) Mb[(so0 + 2 * j) * 256 + (tid & 255)] = v[j] * wt[j];
        }
      }
      __syncthreads();
    }
    // Core windows of k4 (over l45) and of k3 (over l23).
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
    const int xlo = imax(iabs(two_i1 - l25), rp.xlo2), xhi = imin(two_i1 + l25, xhi_g);
    const int64_t u3base = (((int64_t)o24 * tnd + o34) * tnd + o35) * NX;
    auto windows = [&](int x, int &a4, int &b4, int &a3, int &b3) {
      a4 = imax(w4lo, iabs(l35 - x));
      b4 = imin(w4hi, l35 + x);
      a3 = imax(w3lo, iabs(l24 - x));
      b3 = imin(w3hi, l24 + x);
      return a4 <= b4 && a3 <= b3;
    };
    for (int x = xlo; x <= xhi; x += 2) {
      int a4, b4, a3, b3;
      if (!windows(x, a4, b4, a3, b3)) continue;  // uniform
      const int a4l = (a4 - w4lo) / 2, b4l = (b4 - w4lo) / 2;
      const int a3l = (a3 - w3lo) / 2, b3l = (b3 - w3lo) / 2;
      const int xg = (x - rp.X_lo2) / 2;
      // No barrier here: the T stage writes only T5s / T2s (last read in the previous x's G / H
      // stage) and U3s (last read in its P stage), which barriers already separate; a wavefront
      // that finishes the previous x's A update early starts the T stage's global reads while
      // the others are still multiplying.  The barrier after the T stage keeps the G / H writes
      // behind every wavefront's A update.

      // The U3 slice at x (zero outside the active k4 and k3 windows) is read from global memory
      // here and written to LDS after the T stage, for the P stage.
      constexpr int NU3 = 32 * 32 / WT;
      double u3v[NU3];
      {
        const double *u3row = rp.U3 + (u3base + xg) * nK4 * nK3 + ((w3lo - rp.K_lo2[1]) >> 1);
        const int k4g0 = (w4lo - rp.K_lo2[2]) >> 1;
#pragma unroll
        for (int q = 0; q < NU3; ++q) {
          const int idx = tid + q * WT, kp = idx >> 5, k3l = idx & 31;
          u3v[q] = 0.0;
          if (kp >= a4l && kp <= b4l && k3l >= a3l && k3l <= b3l) u3v[q] = ldg(u3row + (int64_t)(k4g0 + kp) * nK3 + k3l);
        }
      }

      // ---- T5 (per l45) and T2 (per l23): 16x16 tiles, K over the k5 (k2) values active at x.
      // A operand: the booster block M5 (M2) of that spin, row c; B operand: the product of the
      // two 6j columns, column c the k4 (k3) of that spin's range.  All loads of a task are issued
      // before its multiply-adds (addresses clamped into range, values masked afterwards).
      // The two sides as two copies of the task (the side is uniform per task): strides and
      // table pointers known per copy.
      auto t_task = [&](int u, auto side) {
        constexpr bool s5 = decltype(side)::value;
        const int o = s5 ? u : u - nd;
        const int lo = rng[(s5 ? 0 : 4) * nd + o], n = rng[(s5 ? 1 : 5) * nd + o];
        const int lop = rng[(s5 ? 2 : 6) * nd + o], np = rng[(s5 ? 3 : 7) * nd + o];
        const int jq = s5 ? J[L14] : J[L13];
        const int ka = imax(lo, iabs(x - jq)), kb = imin(lo + 2 * (n - 1), x + jq);
        d4v t = d4v{0.0, 0.0, 0.0, 0.0};
        if (kb >= ka) {  // uniform
          const int ia = (ka - lo) >> 1, ib = (kb - lo) >> 1, kk0 = ia & ~3;
          const bool rowok = c < (s5 ? d5 : d2), colok = c < np;
          const int cr = rowok ? c : 0, cc = colok ? c : 0;
          const double *bm = B + bo[(s5 ? 0 : 2) * nd + o] + (int64_t)cr * n;
          const double *P, *Q;
          int sP, sQ, kgb;
          if (s5) {
            kgb = (lo - rp.K_lo2[3]) >> 1;
            P = rp.U1 + (((int64_t)o25 * NX + xg) * d1 + n1) * nK5;
            Q = rp.U2 + (((int64_t)o35 * tnd + o) * NX + xg) * nK5 * nK4 + ((lop + 2 * cc - rp.K_lo2[2]) >> 1);
            sP = 1;
            sQ = nK4;
          } else {
            kgb = (lo - rp.K_lo2[0]) >> 1;
            P = rp.U5 + ((int64_t)o25 * NX + xg) * nK2 * d1 + n1;
            Q = rp.U4 + ((((int64_t)o * tnd + o24) * NX + xg) * nK3 + ((lop + 2 * cc - rp.K_lo2[1]) >> 1)) * nK2;
            sP = d1;
            sQ = 1;
          }
          constexpr int TS = 5;  // k steps of 4 covering at most 16 active values
          double av[TS], bv[TS];
#pragma unroll
          for (int s = 0; s < TS; ++s) {
            const int ki = kk0 + 4 * s + g;
            const bool kin = ki >= ia && ki <= ib;
            const int kc = kin ? ki : ia;
            const double a = STG ? Mb[((s5 ? 0 : 2) * nd + o) * 256 + cr * 16 + kc]
                                 : ldg(bm + kc) * (double)(lo + 2 * kc + 1);
            const double b = ldg(P + (int64_t)(kgb + kc) * sP) * ldg(Q + (int64_t)(kgb + kc) * sQ);
            // k values outside [ia, ib] add nothing: zeroing one (finite) operand is enough.  Rows
            // c >= d5 (d2) and columns c >= np of T read clamped entries and are never used.
            av[s] = kin ? a : 0.0;
            bv[s] = b;
          }
          // Steps 0..2 unconditionally (zero operands past ib), 3..4 when active.
#pragma unroll
          for (int s = 0; s < 3; ++s) t = mfma(av[s], bv[s], t);
          if (kk0 + 12 <= ib) {  // uniform
#pragma unroll
            for (int s = 3; s < TS; ++s) t = mfma(av[s], bv[s], t);
          }
        }
        double *Ts = s5 ? T5s : T2s;
#pragma unroll
        for (int r = 0; r < 4; ++r) Ts[(o * 16 + g + 4 * r) * 16 + c] = t[r];
      };
      for (int u = w; u < 2 * nd; u += WW) {
        if (u < nd)
          t_task(u, std::true_type{});
        else
          t_task(u, std::false_type{});
      }
#pragma unroll
      for (int q = 0; q < NU3; ++q) {
        const int idx = tid + q * WT, kp = idx >> 5;
        if (kp < KW) U3s[kp * kU3S + (idx & 31)] = u3v[q];
      }
      __syncthreads();

      // ---- G (per k4 position) and H (per k3 position): 16x16 tiles, K over l45 (l23), whose
      // spin values sit in at most three groups of four.  A task takes four consecutive positions
      // of G or of H, sharing the spin ranges it looks up.
      const int g0 = a4l & ~3, nG = (b4l | 3) - g0 + 1;  // multiples of 4
      const int h0 = a3l & ~3, nH = (b3l | 3) - h0 + 1;
      for (int u = w; u < (nG + nH) / 4; u += WW) {
        const bool sg = u < nG / 4;
        const int p0 = sg ? g0 + 4 * u : h0 + 4 * u - nG;
        const int wlo = sg ? w4lo : w3lo;
        const int pa = sg ? a4l : a3l, pb = sg ? b4l : b3l;
        const int rlo = sg ? 2 : 6, mslot = sg ? 1 : 3;
        const bool cin = c < (sg ? d4 : d3);
        const int cm = cin ? c : 0;
        const double *Ts = sg ? T5s : T2s;
        constexpr int GS3 = 3;  // kWideMaxNd <= 12
        // Per spin group s (this lane's spin value o = 4s + g): position p of the window is
        // entry kb + p of the spin's k range, in range when 0 <= kb + p < nk (nk = 0 for a spin
        // beyond nd or with an empty range); the operand rows of this lane start at tr and mr.
        int kb[GS3], nk[GS3], tr[GS3], mr[GS3];
        const double *bp[GS3];
#pragma unroll
        for (int s = 0; s < GS3; ++s) {
          const int o = 4 * s + g, oc = o < nd ? o : 0;
          const int lok = rng[rlo * nd + oc];
          nk[s] = o < nd ? rng[(rlo + 1) * nd + oc] : 0;
          kb[s] = (wlo - lok) >> 1;
          tr[s] = (oc * 16 + c) * 16 + kb[s];
          mr[s] = (mslot * nd + oc) * 256 + cm * 16 + kb[s];
          bp[s] = B + bo[mslot * nd + oc] + (int64_t)cm * nk[s] + kb[s];
        }
        // Two positions at a time: the operand reads of both are in flight together and their
        // two chains of multiply-adds interleave.  Both stages multiply T (lane c = row i5 or i2)
        // by M (lane c = column i4 or i3): H comes out transposed, (i2, i3).
#pragma unroll
        for (int pp = 0; pp < 2; ++pp) {
          double av[2][GS3], bv[2][GS3];
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int p = p0 + 2 * pp + q, kv = wlo + 2 * p;
            const bool act = p >= pa && p <= pb;  // uniform
#pragma unroll
            for (int s = 0; s < GS3; ++s) {
              double x1 = 0.0, x2 = 0.0;
              if (act && (unsigned)(kb[s] + p) < (unsigned)nk[s]) {
                x1 = Ts[tr[s] + p];
                x2 = STG ? Mb[mr[s] + p] : ldg(bp[s] + p) * (double)(kv + 1);
              }
              av[q][s] = x1;
              bv[q][s] = x2;
            }
          }
          d4v t[2] = {d4v{0.0, 0.0, 0.0, 0.0}, d4v{0.0, 0.0, 0.0, 0.0}};
#pragma unroll
          for (int s = 0; s < GS3; ++s) {
            if (4 * s >= nd) break;  // uniform
#pragma unroll
            for (int q = 0; q < 2; ++q) t[q] = mfma(av[q][s], bv[q][s], t[q]);  // zero operands when idle
          }
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int p = p0 + 2 * pp + q;
            // Entries outside the block go to a padding slot that nothing reads (column KW of
            // G row c, column 16 CT of H row c), so the stores need no branch.
            if (sg) {
              // rows i5 = g + 4r, column i4 = c  ->  rho = i5 d4 + i4
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int rho = (g + 4 * r) * d4 + c - rho0;
                const bool ok = g + 4 * r < d5 && c < d4 && rho >= 0 && rho < nrow;
                Gs[ok ? rho * GS + p : c * GS + KW] = t[q][r];
              }
            } else {
              // rows i2 = g + 4r, column i3 = c  ->  sig = i3 d2 + i2
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const bool ok = g + 4 * r < d2 && c < d3;
                Hs[ok ? p * HS + c * d2 + g + 4 * r : (c < KW ? c : 0) * HS + 16 * CT] = t[q][r];
              }
            }
          }
        }
      }
      __syncthreads();

      // ---- P = G U3 for the block's rows, written over G row tile by row tile (a wavefront
      // reads and writes only its own row tiles, and finishes reading before it writes).  The
      // operands of four k4 steps are loaded (from LDS) before their multiply-adds.
      const int nq = ((b3l | 3) + 16) / 16;  // k3 column tiles (1 or 2)
      for (int rt = w; rt < rtn; rt += WW) {
        d4v pq0 = d4v{0.0, 0.0, 0.0, 0.0}, pq1 = d4v{0.0, 0.0, 0.0, 0.0};
        for (int ks = g0; ks <= b4l; ks += 16) {
          double av[4], b0[4], b1[4];
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            // Positions past the window's last multiple of four are never multiplied: clamp.
            const int kp = ks + 4 * s + g, kr = kp < KW ? kp : KW - 1;
            av[s] = Gs[(rt * 16 + c) * GS + kr];
            b0[s] = U3s[kr * kU3S + c];
            b1[s] = U3s[kr * kU3S + 16 + c];
          }
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            if (ks + 4 * s > b4l) break;  // uniform
            pq0 = mfma(av[s], b0[s], pq0);
            if (nq > 1) pq1 = mfma(av[s], b1[s], pq1);
          }
        }
        // Columns up to KW - 1 only: a row of G / P holds KW positions (the A update reads no
        // further than the last active k3 position rounded up to 4, which is below KW).
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (c < KW) Gs[(rt * 16 + g + 4 * r) * GS + c] = pq0[r];
          if (nq > 1 && 16 + c < KW) Gs[(rt * 16 + g + 4 * r) * GS + 16 + c] = pq1[r];
        }
      }
      __syncthreads();

      // ---- A(i1; rho, sig) += P H over the active k3 positions.  This wavefront's tiles are
      // t = w + 8 j, j < ntw (row tile t / CT by a multiply-shift, exact for t < 128 and
      // CT <= 16), taken in groups of kAccGroup: a group is skipped when it holds no tile of the
      // wavefront, else all of its multiply-adds run (a tile past the end reads tile 0's operands
      // into an accumulator that is never written out), with no branch per tile; the operands of
      // a group are read from LDS, all reads in flight together, before its multiply-adds.
      const double *pa = Gs + c * GS + g, *pb = Hs + g * HS + c;  // this lane's parts of both operands
      for (int ks = h0; ks <= b3l; ks += 4) {
#pragma unroll
        for (int j0 = 0; j0 < kMaxAcc; j0 += kAccGroup) {
          if (j0 < ntw) {  // uniform
            double av[kAccGroup], bv[kAccGroup];
#pragma unroll
            for (int jj = 0; jj < kAccGroup; ++jj) {
              if (j0 + jj >= kMaxAcc) break;
              const int t = w + WW * (j0 + jj), tc = t < ntile ? t : 0;
              const int rt = (tc * ctm) >> 11, ct = tc - rt * CT;
              av[jj] = pa[rt * 16 * GS + ks];
              bv[jj] = pb[ks * HS + ct * 16];
            }
#pragma unroll
            for (int jj = 0; jj < kAccGroup; ++jj) {
              if (j0 + jj >= kMaxAcc) break;
              acc[j0 + jj] = mfma(av[jj], bv[jj], acc[j0 + jj]);
            }
          }
        }
      }
    }
  }
  // Flush the block's partial A(i1, ...): row rho = i5 d4 + i4, column sig = i3 d2 + i2.
  const int64_t slice = (int64_t)d2 * d3 * d4 * d5;
  double *out = rp.partial + ((int64_t)chunk_index * d1 + n1) * slice;
#pragma unroll
  for (int j = 0; j < kMaxAcc; ++j) {
    const int t = w + WW * j;
    if (t >= ntile) continue;
    const int rt = t / CT, ct = t - rt * CT;
    const int sig = ct * 16 + c;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rho = rho0 + rt * 16 + g + 4 * r;
      if (rho < geo.R && sig < geo.C) {
        const int i5 = rho / d4, i4 = rho - i5 * d4, i3 = sig / d2, i2 = sig - i3 * d2;
        stg(out + ((i2 * d3 + i3) * d4 + i4) * d5 + i5, acc[j][r]);
      }
    }
  }
  __syncthreads();  // the next item reuses the LDS
}

// Workgroups are dispatched to the eight XCDs round-robin (workgroup b on XCD b % 8; checked on
// the device against the XCC_ID hardware register, which the kernels read).  The persistent
// kernels give each XCD its own lists of work items so that the items of one chunk of cores, all
// (i1, row block) of it, run on one XCD one after the other: with the chunk bounds shared by
// every i1, those items read the same 6j table slices and booster blocks, which then stay in
// that XCD's L2.
// XCD this workgroup runs on (hardware register XCC_ID, bits 3:0).
__device__ __forceinline__ int xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | 20) & 7; }

// Plain call, persistent: XCD x owns the chunks c with c % 8 == x, item j of its list being
// chunk (j / (d1 nrb)) * 8 + x, i1 and row block from j % (d1 nrb).  A workgroup takes items
// from its own XCD's list through that list's counter (next[x], zeroed before the launch), then
// from the other lists in turn; every item writes its own partial slice, so which workgroup runs
// it does not matter.  The loop ends for every workgroup once all eight counters have passed the
// ends of their lists.
template <bool STG>
__global__ __launch_bounds__(WT, 1) void wide_kernel(RingParams rp, int *next) {
  extern __shared__ double smem[];
  __shared__ int it_s;
  const int per_chunk = rp.i_n[0] * rp.nrb;
  const int home = xcc_id();
  for (int v = 0; v < 8; ++v) {
    const int qx = (home + v) & 7;
    const int n = (qx < rp.nchunk ? (rp.nchunk - qx + 7) / 8 : 0) * per_chunk;
    for (;;) {
      if (threadIdx.x == 0) it_s = atomicAdd(next + qx, 1);
      __syncthreads();
      const int it = __builtin_amdgcn_readfirstlane(it_s);
      __syncthreads();
      if (it >= n) break;
      const int chunk = (it / per_chunk) * 8 + qx, r = it % per_chunk;
      wide_item<STG>(rp, chunk, r / rp.nrb, r % rp.nrb, smem);
    }
  }
}

// Persistent variant for batches: the (configuration, chunk, i1, row block) items are split into
// eight lists, one per XCD (whole chunks per list, balanced by cost, longest chunks first, the
// items of a chunk together), list x holding items [xoff[x], xoff[x + 1]).  A workgroup takes
// items from its own XCD's list through that list's counter, then from the other lists in turn;
// every item writes its own partial slice, so which workgroup runs it does not matter.  The loop
// ends for every workgroup once all eight counters have passed the ends of their lists.
template <bool STG>
__global__ __launch_bounds__(WT, 1) void wide_batch_kernel(const RingParams *__restrict__ cfgs,
                                                          const int *__restrict__ items,
                                                          const int *__restrict__ xoff, int *next) {
  extern __shared__ double smem[];
  __shared__ int it_s;
  const int home = xcc_id();
  for (int v = 0; v < 8; ++v) {
    const int qx = (home + v) & 7;
    const int lo = __builtin_amdgcn_readfirstlane(xoff[qx]);
    const int n = __builtin_amdgcn_readfirstlane(xoff[qx + 1]) - lo;
    for (;;) {
      if (threadIdx.x == 0) it_s = atomicAdd(next + qx, 1);
      __syncthreads();
      // The item and its fields are the same for the whole workgroup: read them through scalar
      // registers, so that the configuration's parameters are scalar loads too.
      const int it = __builtin_amdgcn_readfirstlane(it_s);
      __syncthreads();
      if (it >= n) break;
      const int *p = items + 4 * (lo + it);
      const int q0 = __builtin_amdgcn_readfirstlane(p[0]), q1 = __builtin_amdgcn_readfirstlane(p[1]);
      const int q2 = __builtin_amdgcn_readfirstlane(p[2]), q3 = __builtin_amdgcn_readfirstlane(p[3]);
      wide_item<STG>(cfgs[q0], q1, q2, q3, smem);
    }
  }
}

}  // namespace

size_t wide_smem_bytes(int nd, const int i_n[5], int kw, int nrb, bool stg) {
  return wide_bytes(nd, i_n, kw, nrb, stg);
}

int wide_row_blocks(const int i_n[5]) {
  const int RT = (i_n[4] * i_n[3] + 15) / 16, CT = (i_n[2] * i_n[1] + 15) / 16;
  for (int nrb = 1; nrb <= RT; ++nrb)
    if (((RT + nrb - 1) / nrb) * CT <= WW * kMaxAcc) return nrb;
  return 0;  // a single row tile already needs more accumulators than a workgroup holds
}

bool wide_fits(int nd, const int i_n[5], int kw, int nrb, bool stg) {
  return nrb > 0 && kw <= 32 && wide_bytes(nd, i_n, kw, nrb, stg) <= kLdsBytes - 256;
}

hipError_t wide_init_attributes() {
  const int bytes = (int)(kLdsBytes - 256);
  const void *fns[4] = {(const void *)wide_kernel<false>, (const void *)wide_kernel<true>,
                        (const void *)wide_batch_kernel<false>, (const void *)wide_batch_kernel<true>};
  for (const void *f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_wide(const RingParams &rp, int *next, int ncu, hipStream_t s) {
  const int items = rp.nchunk * rp.i_n[0] * rp.nrb;
  const unsigned grid = (unsigned)(items < ncu ? items : ncu);
  if (grid == 0) return hipSuccess;
  hipError_t e = launch_reset_counters(next, 8, s);
  if (e != hipSuccess) return e;
  if (wide_fits(rp.nd, rp.i_n, rp.kw, rp.nrb, true))
    wide_kernel<true><<<grid, WT, wide_bytes(rp.nd, rp.i_n, rp.kw, rp.nrb, true), s>>>(rp, next);
  else
    wide_kernel<false><<<grid, WT, wide_bytes(rp.nd, rp.i_n, rp.kw, rp.nrb, false), s>>>(rp, next);
  return hipGetLastError();
}

hipError_t launch_wide_batch(const RingParams *cfgs_dev, const int *items_dev, const int *xoff_dev,
                             int nitems, size_t smem, bool stg, int grid, int *next, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (stg)
    wide_batch_kernel<true><<<grid, WT, smem, s>>>(cfgs_dev, items_dev, xoff_dev, next);
  else
    wide_batch_kernel<false><<<grid, WT, smem, s>>>(cfgs_dev, items_dev, xoff_dev, next);
  return hipGetLastError();
}

}  // namespace eprl
