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
// Tiles: boundary intertwiners padded to DI (8 or 16), virtual ones to DK (8 or 16), the
// union over l45 (l23) of the k4 (k3) ranges of a core to KW (16 or 32).  A(i1; rows, cols)
// has DI^2 rows (i5, i4) and DI^2 columns (i3, i2).  One workgroup (4 wavefronts) owns a
// block of 64 rows (all of them for DI = 8, a quarter for DI = 16) of A(i1, ...) for a chunk
// of cores and keeps it in MFMA accumulators; wavefront w owns row tile w and every column
// tile.  Per x: the two half chains on VALU in two stages through LDS (step 1: T5 per (l45, k4)
// and T2 per (l23, k3), each 6j column read once per workgroup; step 2: G and H over l45 and
// l23 with the core's weighted booster blocks staged in LDS as far as they fit), the U3 slice in
// LDS, then two 16x16x4 FP64 MFMA contractions.  The cores of each i1 are split into chunks of
// equal estimated cost; partial slices are reduced in a fixed order by the reduction kernel.
#include "eprl_internal.hpp"

namespace eprl {

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int RT = 256;  // threads per workgroup
constexpr size_t kLdsBytes = 160 * 1024 - 256;  // LDS of a CU, less room for static LDS

__device__ __forceinline__ int iabs(int v) { return v < 0 ? -v : v; }
__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }
__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

// An empty asm taking the N values as register operands: the LDS reads that produce them are
// all issued before the first use, rather than one by one between the multiply-adds that the
// register-frugal schedule would otherwise interleave them with (one wait instead of N / 2).
template <int N>
__device__ __forceinline__ void ready(double (&v)[N]) {
  static_assert(N % 8 == 0, "groups of eight");
#pragma unroll
  for (int g = 0; g < N; g += 8)
    asm volatile("" : "+v"(v[g]), "+v"(v[g + 1]), "+v"(v[g + 2]), "+v"(v[g + 3]), "+v"(v[g + 4]),
                 "+v"(v[g + 5]), "+v"(v[g + 6]), "+v"(v[g + 7]));
}

// One work item: cores [bounds[i1][chunk], bounds[i1][chunk + 1]) of rp, boundary intertwiner
// i1 = n1, row block rb (rows rb * 64 .. rb * 64 + 63 of A(i1; rows, cols)).
// STG: booster blocks of a core staged in LDS: 2 all four (M5, M4, M2, M3), 1 the two read in
// the second half-chain stage (M4, M3), 0 none (read from global memory).
template <int DI, int DK, int KW, int STG>
__device__ void ring_item(const RingParams &rp, int64_t chunk_index, int n1, int rb, double *smem) {
  constexpr bool STAGE = STG == 2;   // M5, M2 in LDS (first stage)
  constexpr bool STAGE2 = STG >= 1;  // M4, M3 in LDS (second stage)
  constexpr int NBLK = STG == 2 ? 4 : 2 * STG;
  // 8-wide tiles (always fully staged) look up the step-2 operands of each (l45, k4) and
  // (l23, k3) in a per-core table instead of testing the k ranges per l45 / l23.
  constexpr bool TAB = DI == 8 && STAGE2;
  constexpr int ZN = TAB ? 8 * DK : 0;  // zero column read by table entries of inactive spins
  constexpr int GS = KW + 1;       // padded row stride of G and P
  constexpr int CC = DI * DI;      // columns (i3, i2)
  constexpr int CT = CC / 16;      // column tiles
  constexpr int IB = 64 / DI;      // i5 values per row block
  // LDS strides, padded so that the access patterns below spread over the 64 banks.
  constexpr int HS = CC + 8;                     // row of H
  constexpr int U3S = KW == 32 ? KW + 8 : KW;    // row of the U3 slice
  constexpr int T5S = IB * DK + 8;               // one l45 of T5
  constexpr int T2S = DI * DK + 8;               // one l23 of T2
  constexpr int MBS = DI * DK + 2;               // one booster block
  const int nd = rp.nd, nd3 = nd * nd * nd;
  double *Gs = smem;                  // [64][GS]  rows (i5, i4) of this block: G (cols k4), then P (cols k3)
  double *Hs = Gs + 64 * GS;          // [KW][HS]  rows k3, cols (i3, i2)
  double *U3s = Hs + KW * HS;         // [KW][U3S] k4 x k3
  double *T5 = U3s + KW * U3S;        // [nd][T5S] per l45: sum_k5 U1 M5 U2 as [i5 of block][k4]
  double *T2 = T5 + nd * T5S;         // [nd][T2S] per l23: sum_k2 U4 M2 U5 as [i2][k3]
  double *Mb = T2 + nd * T2S;         // [NBLK][nd][MBS] weighted boosters as [i][k]
  double *Zc = Mb + NBLK * nd * MBS;  // [ZN] zeros
  int64_t *bo = reinterpret_cast<int64_t *>(Zc + ZN);  // [4][nd]
  // Offset in Mb of the block of edge slot e (0 M5, 1 M4, 2 M2, 3 M3) for the spin index o.
  auto mb = [&](int e, int o) { return ((STG == 2 ? e : (e == 1 ? 0 : 1)) * nd + o) * MBS; };
  // [2][nd][KW] step-2 table: LDS byte offsets of the T5 (T2) entry and the M4 (M3) column of
  // spin index o at window position k4l (k3l); inactive pairs point at the zero column.
  int2 *tab = reinterpret_cast<int2 *>(bo + 4 * nd);
  int *rng = reinterpret_cast<int *>(tab + (TAB ? 2 * nd * KW : 0));  // [8][nd] lo/n of k5, k4, k2, k3

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int *J = rp.two_j;
  const int two_i1 = rp.i_lo2[0] + 2 * n1;
  const int d1 = rp.i_n[0], d2 = rp.i_n[1], d3 = rp.i_n[2], d4 = rp.i_n[3], d5 = rp.i_n[4];
  const int NX = rp.NX, nK2 = rp.K_n[0], nK3 = rp.K_n[1], nK4 = rp.K_n[2], nK5 = rp.K_n[3];
  const int xhi_g = rp.xhi2, tnd = rp.tnd;
  const double *B = rp.B;

  // This thread's first step-1 item (u = tid): side 0 (T5, per l45) or 1 (T2, per l23).
  const bool first_item = tid < 2 * nd * DK;
  const int f_side = tid / (nd * DK), f_o = (tid / DK) % nd, f_ki = tid % DK;

  d4v acc[CT];
#pragma unroll
  for (int cb = 0; cb < CT; ++cb) acc[cb] = d4v{0.0, 0.0, 0.0, 0.0};
  // The two pad entries after each staged booster block are read (times zero) by the
  // branch-free step 1 and never written by the staging: clear them once.
  for (int q = tid; q < NBLK * nd; q += RT) Mb[q * MBS + DI * DK] = Mb[q * MBS + DI * DK + 1] = 0.0;
  for (int q = tid; q < ZN; q += RT) Zc[q] = 0.0;

  const int64_t c0 = rp.bounds[(int64_t)n1 * (rp.nchunk + 1) + chunk_index];
  const int64_t c1 = rp.bounds[(int64_t)n1 * (rp.nchunk + 1) + chunk_index + 1];
  for (int64_t core = c0; core < c1; ++core) {
    const int o24 = (int)(core / (nd * nd * nd)), o25 = (int)((core / (nd * nd)) % nd);
    const int o34 = (int)((core / nd) % nd), o35 = (int)(core % nd);
    const int l24 = J[L24] + 2 * o24, l25 = J[L25] + 2 * o25;
    const int l35 = J[L35] + 2 * o35;
    // Ranges of k5, k4 for every l45 and of k2, k3 for every l23 (empty when either range of
    // the pair is empty, so that spin does not contribute), and the booster block offsets.
    __syncthreads();  // previous readers of rng / bo are done
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
      bo[0 * nd + o] = rp.boff[3 * nd3 + t5];  // M5
      bo[1 * nd + o] = rp.boff[2 * nd3 + t4];  // M4
      bo[2 * nd + o] = rp.boff[0 * nd3 + t2];  // M2
      bo[3 * nd + o] = rp.boff[1 * nd3 + t3];  // M3
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
    if (TAB) {
      // Entry (side, o, kl): k4 = w4lo + 2 kl against the k4 range of l45 = o (side 0), or
      // k3 = w3lo + 2 kl against the k3 range of l23 = o (side 1); read after the x loop's
      // first barrier.
      for (int q = tid; q < 2 * nd * KW; q += RT) {
        const int side = q / (nd * KW), o = (q / KW) % nd, kl = q % KW;
        const int kk = (side == 0 ? w4lo : w3lo) + 2 * kl;
        const int nf = rng[(side == 0 ? 1 : 5) * nd + o], lo = rng[(side == 0 ? 2 : 6) * nd + o];
        const int n = rng[(side == 0 ? 3 : 7) * nd + o], ki = (kk - lo) >> 1;
        const bool ok = nf > 0 && kk >= lo && ki < n;
        const double *tv = ok ? (side == 0 ? T5 + o * T5S : T2 + o * T2S) + ki : Zc;
        const double *mv = Mb + mb(side == 0 ? 1 : 3, o) + (ok ? ki : 0);
        tab[q] = int2{(int)((tv - smem) * sizeof(double)), (int)((mv - smem) * sizeof(double))};
      }
    }
    if (STG > 0) {
      // Weighted booster blocks (2k+1) B of this core: e = 0 M5, 1 M4 (per l45), 2 M2, 3 M3
      // (per l23); rows i, columns k relative to the lowest k of the block; zero outside the
      // block, pads included (reads below run past a row end and multiply by zero there).
      constexpr int BS = DI * DK;  // entries of a block (a power of two; its pads stay zero)
      for (int idx = tid; idx < NBLK * nd * BS; idx += RT) {
        const int bi = idx / BS, r = idx % BS;
        const int blk = bi / nd, o = bi - blk * nd;
        const int e = STG == 2 ? blk : (blk == 0 ? 1 : 3);
        const int i = r / DK, k = r % DK;
        const int lo = rng[(e == 0 ? 0 : e == 1 ? 2 : e == 2 ? 4 : 6) * nd + o];
        const int kn = rng[(e == 0 ? 1 : e == 1 ? 3 : e == 2 ? 5 : 7) * nd + o];
        const int ni = e == 0 ? d5 : e == 1 ? d4 : e == 2 ? d2 : d3;
        double v = 0.0;
        if (i < ni && k < kn) v = B[bo[e * nd + o] + (int64_t)i * kn + k] * (double)(lo + 2 * k + 1);
        Mb[bi * MBS + r] = v;
      }
    }
    // x closes (i1 l25 x); the other triads restrict the k ranges at each x.
    const int xlo = imax(iabs(two_i1 - l25), rp.xlo2), xhi = imin(two_i1 + l25, xhi_g);
    const int64_t u3base = (((int64_t)o24 * tnd + o34) * tnd + o35) * NX;
    // Active k4 and k3 windows at x (triads (k4 l35 x) and (k3 l24 x)); false if one is empty.
    auto windows = [&](int x, int &a4, int &b4, int &a3, int &b3) {
      a4 = imax(w4lo, iabs(l35 - x));
      b4 = imin(w4hi, l35 + x);
      a3 = imax(w3lo, iabs(l24 - x));
      b3 = imin(w3hi, l24 + x);
      return a4 <= b4 && a3 <= b3;
    };
    auto next_x = [&](int x) {  // first x >= x (same parity) with both windows non-empty
      int a4, b4, a3, b3;
      while (x <= xhi && !windows(x, a4, b4, a3, b3)) x += 2;
      return x;
    };
    // Step-1 item u at x: its 6j column (pointers, stride, count c of active k5 or k2), the
    // first active k (ka) and its index in the booster block (kk0).
    auto item = [&](int u, int x, const double *&pa, const double *&pb, int &sb, int &c, int &ka,
                    int &kk0) {
      const int side = u / (nd * DK), o = (u / DK) % nd, ki = u % DK;
      const int xg = (x - rp.X_lo2) / 2;
      int a4, b4, a3, b3;
      windows(x, a4, b4, a3, b3);
      if (side == 0) {
        const int lo5 = rng[0 * nd + o], n5 = rng[1 * nd + o], lo4 = rng[2 * nd + o], n4 = rng[3 * nd + o];
        const int k4 = lo4 + 2 * ki;
        ka = imax(lo5, iabs(x - J[L14]));
        const int kb = imin(lo5 + 2 * (n5 - 1), x + J[L14]);
        c = (n5 > 0 && ki < n4 && k4 >= a4 && k4 <= b4 && kb >= ka) ? (kb - ka) / 2 + 1 : 0;
        const int g0 = (ka - rp.K_lo2[3]) / 2, k4g = (k4 - rp.K_lo2[2]) / 2;
        kk0 = c > 0 ? (ka - lo5) / 2 : 0;
        pa = rp.U1 + (((int64_t)o25 * NX + xg) * d1 + n1) * nK5 + g0;
        pb = rp.U2 + ((((int64_t)o35 * tnd + o) * NX + xg) * nK5 + g0) * nK4 + k4g;
        sb = nK4;
      } else {
        const int lo2 = rng[4 * nd + o], n2 = rng[5 * nd + o], lo3 = rng[6 * nd + o], n3 = rng[7 * nd + o];
        const int k3 = lo3 + 2 * ki;
        ka = imax(lo2, iabs(J[L13] - x));
        const int kb = imin(lo2 + 2 * (n2 - 1), J[L13] + x);
        c = (n2 > 0 && ki < n3 && k3 >= a3 && k3 <= b3 && kb >= ka) ? (kb - ka) / 2 + 1 : 0;
        const int g0 = (ka - rp.K_lo2[0]) / 2, k3g = (k3 - rp.K_lo2[1]) / 2;
        kk0 = c > 0 ? (ka - lo2) / 2 : 0;
        pa = rp.U4 + ((((int64_t)o * tnd + o24) * NX + xg) * nK3 + k3g) * nK2 + g0;
        pb = rp.U5 + (((int64_t)o25 * NX + xg) * nK2 + g0) * d1 + n1;
        sb = d1;
      }
    };
    auto load_item = [&](int u, int x, double (&a)[DK], double (&b)[DK]) {
      const double *pa, *pb;
      int sb, c, ka, kk0;
      item(u, x, pa, pb, sb, c, ka, kk0);
#pragma unroll
      for (int q = 0; q < DK; ++q) {
        a[q] = q < c ? pa[q] : 0.0;
        b[q] = q < c ? pb[(int64_t)q * sb] : 0.0;
      }
    };
    // U3 slice at x, zero outside the active windows; this thread's entries.
    constexpr int NU3 = (KW * KW + RT - 1) / RT;
    auto load_u3 = [&](int x, double (&v)[NU3]) {
      int a4, b4, a3, b3;
      windows(x, a4, b4, a3, b3);
      const int a4l = (a4 - w4lo) / 2, b4l = (b4 - w4lo) / 2, a3l = (a3 - w3lo) / 2, b3l = (b3 - w3lo) / 2;
      const int xg = (x - rp.X_lo2) / 2;
#pragma unroll
      for (int q = 0; q < NU3; ++q) {
        const int idx = tid + q * RT, k4l = idx / KW, k3l = idx % KW;
        v[q] = 0.0;
        if (idx < KW * KW && k4l >= a4l && k4l <= b4l && k3l >= a3l && k3l <= b3l) {
          const int k4g = (w4lo - rp.K_lo2[2]) / 2 + k4l, k3g = (w3lo - rp.K_lo2[1]) / 2 + k3l;
          v[q] = rp.U3[((u3base + xg) * nK4 + k4g) * nK3 + k3g];
        }
      }
    };
    // Step 1 for item u from its loaded column:
    //   T5(l45; i5, k4) = sum_k5 U1(k5) M5(i5, k5) U2(k5, k4)      (k5 active at this x)
    //   T2(l23; i2, k3) = sum_k2 U4(k3, k2) M2(i2, k2) U5(k2)      (k2 active at this x)
    // The rows of step 1 for item (side, o, ki) from its loaded column: a[q], b[q] hold the q-th
    // active k5 (k2), zero for q >= c; ka is the first active k, kk0 its index in the block.
    auto step1_rows = [&](int side, int o, int ki, int c, int ka, int kk0, double (&a)[DK],
                          const double (&b)[DK]) {
#pragma unroll
      for (int q = 0; q < DK; ++q) a[q] *= b[q];
      const int e = side == 0 ? 0 : 2, ni = side == 0 ? d5 : d2, nrow = side == 0 ? IB : DI;
      const int r0 = side == 0 ? rb * IB : 0;
      // a[q] is zero for q >= c: staged sums run over all DK terms without branches (rows read
      // past their end into finite values); global rows load only the c active entries.
      for (int il = 0; il < nrow; ++il) {
        const int i = r0 + il;
        double t = 0.0;
        if (STAGE) {
          const double *m = Mb + mb(e, o) + i * DK + kk0;
          double mv[DK];
#pragma unroll
          for (int q = 0; q < DK; ++q) mv[q] = m[q];
          ready(mv);
#pragma unroll
          for (int q = 0; q < DK; ++q) t += a[q] * mv[q];
        } else if (c > 0 && i < ni) {
          const int kn = rng[(e == 0 ? 1 : 5) * nd + o];
          const double *m = B + bo[e * nd + o] + (int64_t)i * kn + kk0;
          double mv[DK];  // the row's c active entries, all reads in flight together
#pragma unroll
          for (int q = 0; q < DK; ++q) mv[q] = q < c ? m[q] : 0.0;
          ready(mv);
#pragma unroll
          for (int q = 0; q < DK; ++q) t += a[q] * (mv[q] * (double)(ka + 2 * q + 1));
        }
        if (side == 0)
          T5[o * T5S + il * DK + ki] = t;
        else
          T2[o * T2S + il * DK + ki] = t;
      }
    };
    auto step1 = [&](int u, int x, double (&a)[DK], const double (&b)[DK]) {
      const double *pa, *pb;
      int sb, c, ka, kk0;
      item(u, x, pa, pb, sb, c, ka, kk0);
      step1_rows(u / (nd * DK), (u / DK) % nd, u % DK, c, ka, kk0, a, b);
    };
    // This thread's first step-1 item u = tid (the same for every core): its geometry for this
    // core is set up once here; per x only the active k range and one pointer offset change.
    int f_lo = 0, f_n = 0, f_kc = 0, f_sb = 0;
    bool f_kv = false;
    const double *f_pa = rp.U1, *f_pb = rp.U1;
    int64_t f_pax = 0, f_pbx = 0;
    if (first_item) {
      const int sh = f_side == 0 ? 0 : 4;
      f_lo = rng[(sh + 0) * nd + f_o];
      f_n = rng[(sh + 1) * nd + f_o];
      f_kc = rng[(sh + 2) * nd + f_o] + 2 * f_ki;
      f_kv = f_n > 0 && f_ki < rng[(sh + 3) * nd + f_o];
      if (f_side == 0) {
        const int g0 = (f_lo - rp.K_lo2[3]) / 2, kg = (f_kc - rp.K_lo2[2]) / 2;
        f_pa = rp.U1 + ((int64_t)o25 * NX * d1 + n1) * nK5 + g0;                     // U1[o25][x][i1][k5]
        f_pax = (int64_t)d1 * nK5;
        f_pb = rp.U2 + (((int64_t)o35 * tnd + f_o) * NX * nK5 + g0) * nK4 + kg;        // U2[o35][o45][x][k5][k4]
        f_pbx = (int64_t)nK5 * nK4;
        f_sb = nK4;
      } else {
        const int g0 = (f_lo - rp.K_lo2[0]) / 2, kg = (f_kc - rp.K_lo2[1]) / 2;
        f_pa = rp.U4 + (((int64_t)f_o * tnd + o24) * NX * nK3 + kg) * nK2 + g0;        // U4[o23][o24][x][k3][k2]
        f_pax = (int64_t)nK3 * nK2;
        f_pb = rp.U5 + ((int64_t)o25 * NX * nK2 + g0) * d1 + n1;                      // U5[o25][x][k2][i1]
        f_pbx = (int64_t)nK2 * d1;
        f_sb = d1;
      }
    }
    double pu3[NU3];
    int x = next_x(xlo);
    while (x <= xhi) {
      int a4, b4, a3, b3;
      windows(x, a4, b4, a3, b3);
      const int a4l = (a4 - w4lo) / 2, b4l = (b4 - w4lo) / 2;
      const int a3l = (a3 - w3lo) / 2, b3l = (b3 - w3lo) / 2;
      const int xn = next_x(x + 2);
      __syncthreads();  // previous x's readers of Gs / Hs / U3s / T5 / T2 are done
      load_u3(x, pu3);
      if (first_item) {
        // Active k5 (k2) values at x: the triad (k5 j14 x) (or (j13 k2 x)) and the block range;
        // the item is empty unless its k4 (k3) lies in the active window.
        const int jq = f_side == 0 ? J[L14] : J[L13];
        const int ka = imax(f_lo, iabs(x - jq)), kb = imin(f_lo + 2 * (f_n - 1), x + jq);
        const bool inw = f_side == 0 ? (f_kc >= a4 && f_kc <= b4) : (f_kc >= a3 && f_kc <= b3);
        const bool ok = f_kv && inw && kb >= ka;
        const int c = ok ? (kb - ka) / 2 + 1 : 0, kk0 = ok ? (ka - f_lo) / 2 : 0;
        const int xg = (x - rp.X_lo2) / 2;
        const double *pa = f_pa + xg * f_pax + kk0, *pb = f_pb + xg * f_pbx + (int64_t)kk0 * f_sb;
        double a[DK], b[DK];
#pragma unroll
        for (int q = 0; q < DK; ++q) {
          a[q] = q < c ? pa[q] : 0.0;
          b[q] = q < c ? pb[(int64_t)q * f_sb] : 0.0;
        }
        step1_rows(f_side, f_o, f_ki, c, f_lo + 2 * kk0, kk0, a, b);
      }
      for (int u = tid + RT; u < 2 * nd * DK; u += RT) {
        double a[DK], b[DK];
        load_item(u, x, a, b);
        step1(u, x, a, b);
      }
#pragma unroll
      for (int q = 0; q < NU3; ++q)
        if (tid + q * RT < KW * KW) U3s[((tid + q * RT) / KW) * U3S + (tid + q * RT) % KW] = pu3[q];
      __syncthreads();
      // Step 2: G(i5, i4, k4) = sum_l45 T5 M4 and H(k3, i3, i2) = sum_l23 M3 T2.
      for (int u = tid; u < IB * KW + KW * DI; u += RT) {
        if (u < IB * KW) {
          const int i5l = u / KW, k4l = u % KW, i5 = rb * IB + i5l;
          double g[DI];
#pragma unroll
          for (int q = 0; q < DI; ++q) g[q] = 0.0;
          if (TAB && k4l >= a4l && k4l <= b4l && i5 < d5) {
            const int2 *te = tab + k4l;
            const char *sb = reinterpret_cast<const char *>(smem);
            const int tr = i5l * DK * (int)sizeof(double);
            int2 e = te[0];
            for (int o = 0; o < nd; ++o) {
              // One LDS round trip per spin: this spin's operands and the next spin's table
              // entry are all in flight before the first multiply-add.
              const double t = *reinterpret_cast<const double *>(sb + e.x + tr);
              const double *m4 = reinterpret_cast<const double *>(sb + e.y);
              double mv[DI];
#pragma unroll
              for (int q = 0; q < DI; ++q) mv[q] = m4[q * DK];
              int2 en = te[(o + 1 < nd ? o + 1 : o) * KW];
              ready(mv);
              asm volatile("" : "+v"(en.x), "+v"(en.y));
#pragma unroll
              for (int q = 0; q < DI; ++q) g[q] += t * mv[q];
              e = en;
            }
          } else if (!TAB && k4l >= a4l && k4l <= b4l && i5 < d5) {
            const int k4 = w4lo + 2 * k4l;
#pragma unroll 2
            for (int o = 0; o < nd; ++o) {
              const int n5 = rng[1 * nd + o], lo4 = rng[2 * nd + o], n4 = rng[3 * nd + o];
              const int k4i = (k4 - lo4) >> 1;
              const bool ok = n5 > 0 && k4 >= lo4 && k4i < n4;
              if (STAGE2) {
                // Branch-free: an l45 whose k4 range misses k4 contributes t = 0.
                const int kc = ok ? k4i : 0;
                const double t = ok ? T5[o * T5S + i5l * DK + kc] : 0.0;
                const double *m4 = Mb + mb(1, o) + kc;
                double mv[DI];
#pragma unroll
                for (int i4 = 0; i4 < DI; ++i4) mv[i4] = m4[i4 * DK];
                ready(mv);
#pragma unroll
                for (int i4 = 0; i4 < DI; ++i4) g[i4] += t * mv[i4];
              } else {
                if (!ok) continue;
                const double t = T5[o * T5S + i5l * DK + k4i];
                const double w4 = (double)(k4 + 1);
                const double *m4 = B + bo[1 * nd + o] + k4i;
                double mv[DI];
#pragma unroll
                for (int i4 = 0; i4 < DI; ++i4) mv[i4] = i4 < d4 ? m4[(int64_t)i4 * n4] : 0.0;
                ready(mv);
#pragma unroll
                for (int i4 = 0; i4 < DI; ++i4) g[i4] += t * (mv[i4] * w4);
              }
            }
          }
#pragma unroll
          for (int i4 = 0; i4 < DI; ++i4) Gs[(i5l * DI + i4) * GS + k4l] = g[i4];
        } else {
          const int v = u - IB * KW, k3l = v / DI, i2 = v % DI;
          double hq[DI];
#pragma unroll
          for (int q = 0; q < DI; ++q) hq[q] = 0.0;
          if (TAB && k3l >= a3l && k3l <= b3l && i2 < d2) {
            const int2 *te = tab + nd * KW + k3l;
            const char *sb = reinterpret_cast<const char *>(smem);
            const int tr = i2 * DK * (int)sizeof(double);
            int2 e = te[0];
            for (int o = 0; o < nd; ++o) {
              // One LDS round trip per spin: this spin's operands and the next spin's table
              // entry are all in flight before the first multiply-add.
              const double t = *reinterpret_cast<const double *>(sb + e.x + tr);
              const double *m3 = reinterpret_cast<const double *>(sb + e.y);
              double mv[DI];
#pragma unroll
              for (int q = 0; q < DI; ++q) mv[q] = m3[q * DK];
              int2 en = te[(o + 1 < nd ? o + 1 : o) * KW];
              ready(mv);
              asm volatile("" : "+v"(en.x), "+v"(en.y));
#pragma unroll
              for (int q = 0; q < DI; ++q) hq[q] += t * mv[q];
              e = en;
            }
          } else if (!TAB && k3l >= a3l && k3l <= b3l && i2 < d2) {
            const int k3 = w3lo + 2 * k3l;
#pragma unroll 2
            for (int o = 0; o < nd; ++o) {
              const int n2 = rng[5 * nd + o], lo3 = rng[6 * nd + o], n3 = rng[7 * nd + o];
              const int k3i = (k3 - lo3) >> 1;
              const bool ok = n2 > 0 && k3 >= lo3 && k3i < n3;
              if (STAGE2) {
                const int kc = ok ? k3i : 0;
                const double t = ok ? T2[o * T2S + i2 * DK + kc] : 0.0;
                const double *m3 = Mb + mb(3, o) + kc;
                double mv[DI];
#pragma unroll
                for (int i3 = 0; i3 < DI; ++i3) mv[i3] = m3[i3 * DK];
                ready(mv);
#pragma unroll
                for (int i3 = 0; i3 < DI; ++i3) hq[i3] += t * mv[i3];
              } else {
                if (!ok) continue;
                const double t = T2[o * T2S + i2 * DK + k3i];
                const double w3 = (double)(k3 + 1);
                const double *m3 = B + bo[3 * nd + o] + k3i;
                double mv[DI];
#pragma unroll
                for (int i3 = 0; i3 < DI; ++i3) mv[i3] = i3 < d3 ? m3[(int64_t)i3 * n3] : 0.0;
                ready(mv);
#pragma unroll
                for (int i3 = 0; i3 < DI; ++i3) hq[i3] += t * (mv[i3] * w3);
              }
            }
          }
#pragma unroll
          for (int i3 = 0; i3 < DI; ++i3) Hs[k3l * HS + i3 * DI + i2] = hq[i3];
        }
      }
      __syncthreads();
      // P = G U3 (rows (i5, i4) of this block, cols k3): wavefront `wave` owns row tile `wave`
      // and reads and writes only those rows, so P replaces G in place with no barrier (LDS
      // operations of one wavefront complete in order).
      {
        const int r = wave * 16 + (lane & 15), kq = lane >> 4;
        d4v c[KW / 16];
#pragma unroll
        for (int cb = 0; cb < KW / 16; ++cb) {
          c[cb] = d4v{0.0, 0.0, 0.0, 0.0};
          for (int ks = a4l & ~3; ks <= b4l; ks += 4) {
            const double a = Gs[r * GS + ks + kq];
            const double b = U3s[(ks + kq) * U3S + cb * 16 + (lane & 15)];
            c[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[cb], 0, 0, 0);
          }
        }
#pragma unroll
        for (int cb = 0; cb < KW / 16; ++cb)
#pragma unroll
          for (int j = 0; j < 4; ++j) Gs[(wave * 16 + 4 * kq + j) * GS + cb * 16 + (lane & 15)] = c[cb][j];
        __builtin_amdgcn_wave_barrier();  // keeps the reads below after these writes
      }
      // A(i1; rows, cols) += P H over the active k3 window.
      {
        const int r = wave * 16 + (lane & 15), kq = lane >> 4;
        for (int ks = a3l & ~3; ks <= b3l; ks += 4) {
          const double a = Gs[r * GS + ks + kq];
#pragma unroll
          for (int cb = 0; cb < CT; ++cb) {
            const double b = Hs[(ks + kq) * HS + cb * 16 + (lane & 15)];
            acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[cb], 0, 0, 0);
          }
        }
      }
      x = xn;
    }
  }
  // Flush the partial A(i1, ...): row (i5, i4), column (i3, i2).
  const int64_t slice = (int64_t)d2 * d3 * d4 * d5;
  double *out = rp.partial + (chunk_index * d1 + n1) * slice;
#pragma unroll
  for (int cb = 0; cb < CT; ++cb) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = rb * 64 + wave * 16 + 4 * (lane >> 4) + j, c = cb * 16 + (lane & 15);
      const int i5 = r / DI, i4 = r % DI, i3 = c / DI, i2 = c % DI;
      if (i2 < d2 && i3 < d3 && i4 < d4 && i5 < d5)
        out[((i2 * d3 + i3) * d4 + i4) * d5 + i5] = acc[cb][j];
    }
  }
  __syncthreads();  // the next item reuses the LDS
}

// Wavefronts per SIMD that the LDS of a tile class allows at the usual nd (<= 11): the register
// budget is capped to match, so registers never limit occupancy below LDS.
template <int DI, int DK, int KW>
constexpr int ring_waves() {
  return (DI == 8 && DK == 8 && KW == 16) ? 3 : (DI == 8 && (DK == 8 || KW == 16)) ? 2 : 1;
}

template <int DI, int DK, int KW, int STG>
__global__ __launch_bounds__(RT, (ring_waves<DI, DK, KW>())) void ring_kernel(RingParams rp) {
  extern __shared__ double smem[];
  ring_item<DI, DK, KW, STG>(rp, blockIdx.x, blockIdx.y, blockIdx.z, smem);
}

// Persistent variant for batches: workgroups take (configuration, chunk, i1, row block) items
// of a longest-first list from a counter (see below).
template <int DI, int DK, int KW, int STG>
__global__ __launch_bounds__(RT, (ring_waves<DI, DK, KW>())) void ring_batch_kernel(const RingParams *cfgs, const int *items,
                                                        int nitems, int *next) {
  extern __shared__ double smem[];
  __shared__ int it_s;
  // Items are taken from a counter in list order (longest first); which workgroup runs an
  // item does not matter for the result: every item writes its own partial slice.  The loop
  // ends for every workgroup once the counter passes nitems.
  for (;;) {
    if (threadIdx.x == 0) it_s = atomicAdd(next, 1);
    __syncthreads();
    // The item and its fields are the same for the whole workgroup: read them through scalar
    // registers, so that the configuration's parameters are scalar loads too.
    const int it = __builtin_amdgcn_readfirstlane(it_s);
    __syncthreads();
    if (it >= nitems) break;
    const int *p = items + 4 * it;
    const int q0 = __builtin_amdgcn_readfirstlane(p[0]), q1 = __builtin_amdgcn_readfirstlane(p[1]);
    const int q2 = __builtin_amdgcn_readfirstlane(p[2]), q3 = __builtin_amdgcn_readfirstlane(p[3]);
    ring_item<DI, DK, KW, STG>(cfgs[q0], q1, q2, q3, smem);
  }
}

// Resets the work-queue counters of a batch (a kernel, so that graph replays start from 0).
__global__ void reset_counters(int *c, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) c[i] = 0;
}

template <int DI, int DK, int KW, int STG>
struct RingVariant {
  static constexpr int stg = STG;
  static constexpr size_t smem(int nd) {
    const size_t stage = (size_t)(STG == 2 ? 4 : 2 * STG) * nd * (DI * DK + 2);
    const bool tab = DI == 8 && STG >= 1;
    return sizeof(double) * ((size_t)(64 * (KW + 1) + KW * (DI * DI + 8) + KW * (KW == 32 ? KW + 8 : KW)) +
                             (size_t)nd * ((64 / DI + DI) * DK + 16) + stage + (tab ? 8 * DK : 0)) +
           sizeof(int64_t) * (size_t)(4 * nd) + 2 * sizeof(int) * (size_t)(tab ? 2 * nd * KW : 0) +
           sizeof(int) * (size_t)(8 * nd);
  }
  static constexpr bool fits(int nd) { return smem(nd) <= kLdsBytes; }
  static hipError_t init() {
    int nd = kRingMaxNd;
    while (nd > 1 && !fits(nd)) --nd;
    const int bytes = (int)smem(nd);
    hipError_t e = hipFuncSetAttribute((const void *)ring_kernel<DI, DK, KW, STG>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)ring_batch_kernel<DI, DK, KW, STG>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  }
  static hipError_t launch(const RingParams &rp, hipStream_t s) {
    dim3 grid(rp.nchunk, rp.i_n[0], DI == 16 ? 4 : 1);
    ring_kernel<DI, DK, KW, STG><<<grid, RT, smem(rp.nd), s>>>(rp);
    return hipGetLastError();
  }
  static hipError_t launch_batch(const RingParams *cfgs, const int *items, int nitems, int max_nd,
                                 int grid, int *next, hipStream_t s) {
    ring_batch_kernel<DI, DK, KW, STG><<<grid, RT, smem(max_nd), s>>>(cfgs, items, nitems, next);
    return hipGetLastError();
  }
};

static_assert(RingVariant<8, 16, 32, 2>::fits(kRingMaxNd) && RingVariant<8, 8, 32, 2>::fits(kRingMaxNd),
              "8-wide tiles must fit with all booster blocks staged");
static_assert(RingVariant<16, 16, 32, 0>::fits(kRingMaxNd), "16-wide tiles must fit unstaged");

// Staging level for a 16-wide tile class at nd: the most booster blocks that fit in LDS.
// (stg = 0, 1 or 2 asks for that level when it fits; -1 takes the most that fits.)
template <int DI, int DK, int KW, typename F>
hipError_t pick_stage(int nd, F &&f, int stg = -1) {
  if (stg == 0) return f(RingVariant<DI, DK, KW, 0>());
  if (stg == 1 && RingVariant<DI, DK, KW, 1>::fits(nd)) return f(RingVariant<DI, DK, KW, 1>());
  if (RingVariant<DI, DK, KW, 2>::fits(nd)) return f(RingVariant<DI, DK, KW, 2>());
  if (RingVariant<DI, DK, KW, 1>::fits(nd)) return f(RingVariant<DI, DK, KW, 1>());
  return f(RingVariant<DI, DK, KW, 0>());
}

// Dispatch over the eight tile classes (and, for 16-wide tiles, the staging level at nd).
// 8-wide tiles always stage all four blocks; nd = 0 visits every variant (attribute set-up).
template <typename F>
hipError_t dispatch(int cls, int nd, F &&f, int stg = -1) {
  if (nd == 0 && cls >= 4) {
    hipError_t e = hipSuccess;
    auto all = [&](auto v0, auto v1, auto v2) {
      if (e == hipSuccess) e = f(v0);
      if (e == hipSuccess) e = f(v1);
      if (e == hipSuccess) e = f(v2);
      return e;
    };
    switch (cls) {
      case 4: return all(RingVariant<16, 8, 16, 0>(), RingVariant<16, 8, 16, 1>(), RingVariant<16, 8, 16, 2>());
      case 5: return all(RingVariant<16, 8, 32, 0>(), RingVariant<16, 8, 32, 1>(), RingVariant<16, 8, 32, 2>());
      case 6: return all(RingVariant<16, 16, 16, 0>(), RingVariant<16, 16, 16, 1>(), RingVariant<16, 16, 16, 2>());
      default: return all(RingVariant<16, 16, 32, 0>(), RingVariant<16, 16, 32, 1>(), RingVariant<16, 16, 32, 2>());
    }
  }
  switch (cls) {
    case 0: return f(RingVariant<8, 8, 16, 2>());
    case 1: return f(RingVariant<8, 8, 32, 2>());
    case 2: return f(RingVariant<8, 16, 16, 2>());
    case 3: return f(RingVariant<8, 16, 32, 2>());
    case 4: return pick_stage<16, 8, 16>(nd, f, stg);
    case 5: return pick_stage<16, 8, 32>(nd, f, stg);
    case 6: return pick_stage<16, 16, 16>(nd, f, stg);
    case 7: return pick_stage<16, 16, 32>(nd, f, stg);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int ring_class(int DI, int DK, int KW) {
  if ((DI != 8 && DI != 16) || (DK != 8 && DK != 16) || (KW != 16 && KW != 32)) return -1;
  return (DI == 16 ? 4 : 0) + (DK == 16 ? 2 : 0) + (KW == 32 ? 1 : 0);
}

int ring_row_blocks(const Plan &p) {
  if (p.ring_cls == kWideClass) return p.ring_nrb;
  return p.ring_cls >= 4 ? 4 : 1;
}

size_t ring_smem_bytes(int cls, int nd, int stg) {
  size_t out = 0;
  if (cls == kWideClass) return 0;  // sized per configuration (wide_smem_bytes)
  dispatch(
      cls, nd,
      [&](auto v) {
        out = decltype(v)::smem(nd);
        return hipSuccess;
      },
      stg);
  return out;
}

int ring_stage_levels(int cls, int nd, int levels[3]) {
  if (cls == kWideClass) {  // reads boosters straight into the matrix-core operands
    levels[0] = 0;
    return 1;
  }
  if (cls < 4) {
    levels[0] = 2;
    return 1;
  }
  int n = 0;
  for (int stg = 2; stg >= 0; --stg) {
    int got = -1;
    dispatch(
        cls, nd,
        [&](auto v) {
          got = decltype(v)::stg;
          return hipSuccess;
        },
        stg);
    if (got == stg) levels[n++] = stg;
  }
  return n;
}

// Allow the ring kernels the dynamic LDS of the largest supported configuration.  Called once
// per process before any launch (not a stream operation, so never inside a graph capture).
hipError_t ring_init_attributes() {
  for (int cls = 0; cls < 8; ++cls) {
    hipError_t e = dispatch(cls, 0, [](auto v) { return decltype(v)::init(); });
    if (e != hipSuccess) return e;
  }
  hipError_t e = wide_init_attributes();
  if (e != hipSuccess) return e;
  return adjoint_ring_init_attributes();
}

hipError_t launch_ring(const RingParams &rp, int cls, int stg, hipStream_t s) {
  return dispatch(
      cls, rp.nd, [&](auto v) { return decltype(v)::launch(rp, s); }, stg);
}

hipError_t launch_ring_batch(const RingParams *cfgs_dev, const int *items_dev, int nitems, int cls,
                             int max_nd, int stg, int grid, int *next, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  return dispatch(
      cls, max_nd,
      [&](auto v) {
        return decltype(v)::launch_batch(cfgs_dev, items_dev, nitems, max_nd, grid, next, s);
      },
      stg);
}

hipError_t launch_reset_counters(int *c, int n, hipStream_t s) {
  reset_counters<<<1, 64, 0, s>>>(c, n);
  return hipGetLastError();
}

}  // namespace eprl
