// Host planner: admissibility, intertwiner ranges, packed booster layout, global index
// windows of the 6j tables (Sec. 2 eq. (vertex-ampl); Sec. 3.1 framed algorithm, steps 1-4).
#include <algorithm>
#include <cstdlib>
#include <sstream>

#include "eprl_internal.hpp"

namespace eprl {

namespace {

// The four links of each edge; the intertwiner couples (first, second) and (third, fourth).
const int kEdgeLinks[5][4] = {
    {L12, L13, L14, L15}, {L23, L24, L25, L12}, {L34, L35, L13, L23},
    {L45, L14, L24, L34}, {L15, L25, L35, L45}};
// Virtual links of the booster of edges 2..5, in packing order.
const int kEdgeTriple[4][3] = {{L23, L24, L25}, {L34, L35, L23}, {L45, L24, L34}, {L25, L35, L45}};
// Shell coordinate of each virtual link (-1 for the four gauge-fixed links).
const int kShellSlot[10] = {-1, -1, -1, -1, 0, 1, 2, 3, 4, 5};

Range coupled(int a, int b, int c, int d) {
  Range r;
  if ((a + b + c + d) % 2) return r;
  int lo = std::max(std::abs(a - b), std::abs(c - d));
  int hi = std::min(a + b, c + d);
  if (lo > hi) return r;
  r.lo2 = lo;
  r.n = (hi - lo) / 2 + 1;
  return r;
}

// Smallest |a - b| and largest a + b over a in range ra and fixed b.
int min_gap(Range ra, int b) {
  int hi = ra.lo2 + 2 * (ra.n - 1);
  if (b < ra.lo2) return ra.lo2 - b;
  if (b > hi) return b - hi;
  return (b - ra.lo2) % 2;  // 0 or 1: parity of the triad fixes the lowest reachable value
}

}  // namespace

std::vector<int> primes_upto(int n) {
  std::vector<char> sieve(std::max(n + 1, 2), 1);
  std::vector<int> out;
  for (int q = 2; q <= n; ++q) {
    if (!sieve[q]) continue;
    out.push_back(q);
    for (int m = 2 * q; m <= n; m += q) sieve[m] = 0;
  }
  return out;
}

int make_plan(const int two_j[10], int dl, Plan &p, std::string &err) {
  std::ostringstream msg;
  if (!two_j) {
    err = "two_j is NULL";
    return EPRL_EINVAL;
  }
  if (dl < 0) {
    err = "the number of shells dl must be >= 0";
    return EPRL_EINVAL;
  }
  for (int n = 0; n < 10; ++n) {
    if (two_j[n] < 0) {
      err = "spins must be non-negative";
      return EPRL_EINVAL;
    }
    p.two_j[n] = two_j[n];
  }
  // Spin limit: the largest virtual spin 2 (j + dl) must keep every factorial argument of
  // the 6j evaluation below the prime-exponent table limit.
  int maxtwo = 0;
  for (int n = 0; n < 10; ++n) maxtwo = std::max(maxtwo, two_j[n] + 2 * dl);
  if (maxtwo > kSixjMaxTwo) {
    msg << "spin 2j + 2dl = " << maxtwo << " exceeds the supported " << kSixjMaxTwo;
    err = msg.str();
    return EPRL_ERANGE;
  }
  p.dl = dl;
  p.nd = dl + 1;
  for (int e = 0; e < 5; ++e) {
    const int *L = kEdgeLinks[e];
    p.i[e] = coupled(two_j[L[0]], two_j[L[1]], two_j[L[2]], two_j[L[3]]);
    if (p.i[e].n == 0) {
      msg << "node " << (e + 1) << " admits no intertwiner (parity or polygon inequality)";
      err = msg.str();
      return EPRL_EINVAL;
    }
  }
  const int nd = p.nd, nd3 = nd * nd * nd;
  p.nshell = (int64_t)nd3 * nd3;
  p.kr.assign(4 * nd3 * 2, 0);
  p.boff.assign(4 * (size_t)nd3 + 1, 0);
  p.kmax = 0;
  for (int e = 0; e < 4; ++e) {
    int klo = 1 << 30, khi = -1;
    for (int t = 0; t < nd3; ++t) {
      int o[3] = {t / (nd * nd), (t / nd) % nd, t % nd};
      int l[10];
      for (int n = 0; n < 10; ++n) l[n] = two_j[n];
      for (int q = 0; q < 3; ++q) l[kEdgeTriple[e][q]] += 2 * o[q];
      const int *L = kEdgeLinks[e + 1];
      Range k = coupled(l[L[0]], l[L[1]], l[L[2]], l[L[3]]);
      p.kr[(e * nd3 + t) * 2 + 0] = k.lo2;
      p.kr[(e * nd3 + t) * 2 + 1] = k.n;
      size_t slot = (size_t)e * nd3 + t;
      p.boff[slot + 1] = p.boff[slot] + (int64_t)p.i[e + 1].n * k.n;
      if (k.n > 0) {
        klo = std::min(klo, k.lo2);
        khi = std::max(khi, k.lo2 + 2 * (k.n - 1));
        p.kmax = std::max(p.kmax, k.n);
      }
    }
    if (khi < 0) {
      err = "no shell has a non-empty virtual intertwiner range";
      return EPRL_EINVAL;
    }
    p.K[e].lo2 = klo;
    p.K[e].n = (khi - klo) / 2 + 1;
  }
  // Global x window: x closes the triads (i1 l25 x), (k5 j14 x), (l35 k4 x), (l24 k3 x),
  // (j13 k2 x) of eq. (15j).
  auto spin_range = [&](int link) {
    Range r;
    r.lo2 = two_j[link];
    r.n = kShellSlot[link] < 0 ? 1 : nd;
    return r;
  };
  struct Pair {
    Range a;
    Range b;
  } pairs[5] = {{p.i[0], spin_range(L25)}, {p.K[3], spin_range(L14)}, {spin_range(L35), p.K[2]},
                {spin_range(L24), p.K[1]}, {spin_range(L13), p.K[0]}};
  int xlo = 0, xhi = 1 << 30;
  for (auto &pr : pairs) {
    int gap = 1 << 30;
    for (int q = 0; q < pr.b.n; ++q) gap = std::min(gap, min_gap(pr.a, pr.b.lo2 + 2 * q));
    xlo = std::max(xlo, gap);
    xhi = std::min(xhi, pr.a.lo2 + 2 * (pr.a.n - 1) + pr.b.lo2 + 2 * (pr.b.n - 1));
  }
  if (xlo > xhi) {
    err = "empty summation range for x";
    return EPRL_EINVAL;
  }
  p.X.lo2 = xlo;
  p.X.n = (xhi - xlo) / 2 + 1;
  int dmax = p.kmax;
  for (int e = 0; e < 5; ++e) dmax = std::max(dmax, p.i[e].n);
  p.D = dmax <= 8 ? 8 : (dmax <= 16 ? 16 : 0);
  // Largest factorial argument of any 6j in the tables: (a + b + c)/2 + 1 for a triad and the
  // sums of four entries; bounded by the largest two-spin met times 2, plus 1.
  int xmax2 = p.X.lo2 + 2 * (p.X.n - 1);
  int kmax2 = 0;
  for (int e = 0; e < 4; ++e) kmax2 = std::max(kmax2, p.K[e].lo2 + 2 * (p.K[e].n - 1));
  int imax2 = 0;
  for (int e = 0; e < 5; ++e) imax2 = std::max(imax2, p.i[e].lo2 + 2 * (p.i[e].n - 1));
  int big = std::max(std::max(maxtwo, xmax2), std::max(kmax2, imax2));
  if (big > kSixjMaxTwo) {
    msg << "a 6j argument of the tables reaches 2j = " << big << ", above the supported "
        << kSixjMaxTwo;
    err = msg.str();
    return EPRL_ERANGE;
  }
  p.fact_max = 2 * big + 2;
  // 6j table sizes (doubles): T1[nd][n_i1][nK5][NX], T2[nd][nd][nK5][nK4][NX],
  // T3[nd][nd][nd][nK4][nK3][NX], T4[nd][nd][nK3][nK2][NX], T5[nd][nK2][n_i1][NX].
  const int64_t NX = p.X.n, n1 = p.i[0].n;
  const int64_t nK2 = p.K[0].n, nK3 = p.K[1].n, nK4 = p.K[2].n, nK5 = p.K[3].n;
  p.tsize[0] = nd * n1 * nK5 * NX;
  p.tsize[1] = (int64_t)nd * nd * nK5 * nK4 * NX;
  p.tsize[2] = (int64_t)nd * nd * nd * nK4 * nK3 * NX;
  p.tsize[3] = (int64_t)nd * nd * nK3 * nK2 * NX;
  p.tsize[4] = nd * nK2 * n1 * NX;
  p.toff[0] = 0;
  for (int t = 0; t < 5; ++t) p.toff[t + 1] = p.toff[t] + ((p.tsize[t] + 31) / 32) * 32;
  p.a_size = 1;
  for (int e = 0; e < 5; ++e) p.a_size *= p.i[e].n;
  // Widest core windows of the factorised path.
  p.ring_w4 = p.ring_w3 = 0;
  for (int a = 0; a < nd; ++a) {
    for (int b = 0; b < nd; ++b) {
      int lo4 = 1 << 30, hi4 = -1, lo3 = 1 << 30, hi3 = -1;
      for (int o = 0; o < nd; ++o) {
        // edge 4 triple (l45, l24, l34) with (o24, o34) = (a, b)
        const int t4 = (o * nd + a) * nd + b;
        const int klo4 = p.kr[(2 * nd3 + t4) * 2], kn4 = p.kr[(2 * nd3 + t4) * 2 + 1];
        if (kn4 > 0) {
          lo4 = std::min(lo4, klo4);
          hi4 = std::max(hi4, klo4 + 2 * (kn4 - 1));
        }
        // edge 3 triple (l34, l35, l23) with (o34, o35) = (a, b)
        const int t3 = (a * nd + b) * nd + o;
        const int klo3 = p.kr[(1 * nd3 + t3) * 2], kn3 = p.kr[(1 * nd3 + t3) * 2 + 1];
        if (kn3 > 0) {
          lo3 = std::min(lo3, klo3);
          hi3 = std::max(hi3, klo3 + 2 * (kn3 - 1));
        }
      }
      if (hi4 >= 0) p.ring_w4 = std::max(p.ring_w4, (hi4 - lo4) / 2 + 1);
      if (hi3 >= 0) p.ring_w3 = std::max(p.ring_w3, (hi3 - lo3) / 2 + 1);
    }
  }
  int imaxn = 0;
  for (int e = 0; e < 5; ++e) imaxn = std::max(imaxn, p.i[e].n);
  const int w = std::max(p.ring_w4, p.ring_w3);
  p.ring_DI = imaxn <= 8 ? 8 : (imaxn <= 16 ? 16 : 0);
  p.ring_DK = p.kmax <= 8 ? 8 : (p.kmax <= 16 ? 16 : 0);
  p.ring_KW = w <= 16 ? 16 : (w <= 32 ? 32 : 0);
  if (p.ring_DI == 0 || p.ring_DK == 0 || p.ring_KW == 0 || nd > kRingMaxNd) p.ring_KW = 0;
  p.ring_cls = p.ring_KW ? ring_class(p.ring_DI, p.ring_DK, p.ring_KW) : -1;
  p.ring_cls8 = p.ring_cls;
  // Boundary dimensions above 8: the all-matrix-core kernel, when its tiles fit in LDS.
  int dims[5];
  for (int e = 0; e < 5; ++e) dims[e] = p.i[e].n;
  p.ring_kw = (w + 3) / 4 * 4;
  p.ring_nrb = wide_row_blocks(dims);
  if (p.ring_cls >= 4 && nd <= kWideMaxNd && wide_fits(nd, dims, p.ring_kw, p.ring_nrb))
    p.ring_cls = kWideClass;
  return EPRL_OK;
}

int ring_schedule(const Plan &p, int target_wg, std::vector<int> &bounds,
                  std::vector<double> *chunk_cost, int core_lo, int core_hi) {
  const int nd = p.nd, nd3 = nd * nd * nd, d1 = p.i[0].n;
  const int ncore = nd * nd3;
  if (core_hi < 0) core_hi = ncore;
  const int nrange = std::max(1, core_hi - core_lo);
  const int nrb = p.ring_cls >= 0 ? ring_row_blocks(p) : 1;
  int nchunk = std::max(1, target_wg / (d1 * nrb));
  nchunk = (int)std::min<int64_t>(nchunk, std::max<int64_t>(1, (int64_t)(kRingMaxPartialBytes / ((size_t)p.a_size * sizeof(double)))));
  nchunk = std::min(nchunk, nrange);
  const int *J = p.two_j;
  const int xlo_g = p.X.lo2, xhi_g = p.X.lo2 + 2 * (p.X.n - 1);
  std::vector<double> cost((size_t)d1 * ncore, 0.0);
  for (int core = core_lo; core < core_hi; ++core) {
    // Core order of the kernels: (l24, l25, l34, l35) with l35 fastest.
    const int o24 = core / nd3, o25 = (core / (nd * nd)) % nd;
    const int o34 = (core / nd) % nd, o35 = core % nd;
    // Windows of k4 over l45 and of k3 over l23 (pairs with an empty range left out), as the
    // kernel forms them.
    int w4lo = 1 << 30, w4hi = -1, w3lo = 1 << 30, w3hi = -1;
    for (int o = 0; o < nd; ++o) {
      const int t5 = (o25 * nd + o35) * nd + o, t4 = (o * nd + o24) * nd + o34;
      const int t2 = (o * nd + o24) * nd + o25, t3 = (o34 * nd + o35) * nd + o;
      const int n5 = p.kr[(3 * nd3 + t5) * 2 + 1], n4 = p.kr[(2 * nd3 + t4) * 2 + 1];
      const int n2 = p.kr[(0 * nd3 + t2) * 2 + 1], n3 = p.kr[(1 * nd3 + t3) * 2 + 1];
      if (n5 > 0 && n4 > 0) {
        const int lo = p.kr[(2 * nd3 + t4) * 2];
        w4lo = std::min(w4lo, lo);
        w4hi = std::max(w4hi, lo + 2 * (n4 - 1));
      }
      if (n2 > 0 && n3 > 0) {
        const int lo = p.kr[(1 * nd3 + t3) * 2];
        w3lo = std::min(w3lo, lo);
        w3hi = std::max(w3hi, lo + 2 * (n3 - 1));
      }
    }
    if (w4hi < 0 || w3hi < 0) {
      for (int n1 = 0; n1 < d1; ++n1) cost[(size_t)n1 * ncore + core] = 0.1;
      continue;
    }
    const int l24 = J[L24] + 2 * o24, l25 = J[L25] + 2 * o25, l35 = J[L35] + 2 * o35;
    // x runs over (i1 l25 x) in steps of 2; both windows are non-empty exactly on
    // max(w4lo - l35, l35 - w4hi) <= x <= l35 + w4hi and the same with (l24, w3).
    const int lo_w = std::max(std::max(w4lo - l35, l35 - w4hi), std::max(w3lo - l24, l24 - w3hi));
    const int hi_w = std::min(l35 + w4hi, l24 + w3hi);
    for (int n1 = 0; n1 < d1; ++n1) {
      const int i1 = p.i[0].lo2 + 2 * n1;
      const int xlo = std::max(std::abs(i1 - l25), xlo_g), xhi = std::min(i1 + l25, xhi_g);
      int lo = std::max(xlo, lo_w);
      if ((lo - xlo) & 1) ++lo;
      const int hi = std::min(xhi, hi_w);
      const int nx = hi >= lo ? (hi - lo) / 2 + 1 : 0;
      cost[(size_t)n1 * ncore + core] = 1.0 + nx;
    }
  }
  bounds.assign((size_t)d1 * (nchunk + 1), 0);
  if (chunk_cost) chunk_cost->assign((size_t)d1 * nchunk, 0.0);
  // The wide kernel splits the cores the same way for every i1 (by the cost summed over i1):
  // the work items of one chunk then read the same 6j table slices and booster blocks, which
  // the XCD-aware launch order keeps in one L2.
  const bool shared = p.ring_cls == kWideClass;
  std::vector<double> sum_cost;
  if (shared) {
    sum_cost.assign(ncore, 0.0);
    for (int n1 = 0; n1 < d1; ++n1)
      for (int k = core_lo; k < core_hi; ++k) sum_cost[k] += cost[(size_t)n1 * ncore + k];
  }
  for (int n1 = 0; n1 < d1; ++n1) {
    const double *cs = shared ? sum_cost.data() : cost.data() + (size_t)n1 * ncore;
    double total = 0.0;
    for (int k = core_lo; k < core_hi; ++k) total += cs[k];
    int *bd = bounds.data() + (size_t)n1 * (nchunk + 1);
    double run = 0.0;
    int k = core_lo;
    for (int ch = 1; ch < nchunk; ++ch) {
      const double target = total * ch / nchunk;
      while (k < core_hi && run + 0.5 * cs[k] < target) run += cs[k++];
      bd[ch] = k;
    }
    bd[0] = core_lo;
    bd[nchunk] = core_hi;
    if (chunk_cost)
      for (int ch = 0; ch < nchunk; ++ch)
        for (int q = bd[ch]; q < bd[ch + 1]; ++q)
          (*chunk_cost)[(size_t)n1 * nchunk + ch] += cost[(size_t)n1 * ncore + q];
  }
  return nchunk;
}

void count_terms(const Plan &p, int64_t &live, double &terms) {
  const int nd = p.nd, nd3 = nd * nd * nd;
  live = 0;
  terms = 0.0;
  for (int64_t s = 0; s < p.nshell; ++s) {
    int o[6];
    int64_t r = s;
    for (int q = 5; q >= 0; --q) {
      o[q] = (int)(r % nd);
      r /= nd;
    }
    // edge triples in (o23, o24, o25, o34, o35, o45) coordinates
    const int t[4] = {(o[0] * nd + o[1]) * nd + o[2], (o[3] * nd + o[4]) * nd + o[0],
                      (o[5] * nd + o[1]) * nd + o[3], (o[2] * nd + o[4]) * nd + o[5]};
    double prod = p.i[0].n;
    bool ok = true;
    for (int e = 0; e < 4; ++e) {
      int kn = p.kr[(e * nd3 + t[e]) * 2 + 1];
      if (kn == 0) {
        ok = false;
        break;
      }
      prod *= kn;
    }
    if (!ok) continue;
    ++live;
    terms += prod;
  }
}

namespace {

// Number of values v = lo, lo + 2, ... (n of them) with |a - v| <= x <= a + v, i.e. in the
// triad (a, v, x).  All two-units.
int triad_count(int lo, int n, int a, int x) {
  if (n <= 0) return 0;
  const int hi = lo + 2 * (n - 1);
  const int vlo = std::max(lo, std::abs(x - a)), vhi = std::min(hi, x + a);
  if (vlo > vhi) return 0;
  if (((vlo - lo) & 1) != 0) return 0;  // parity mismatch: no value closes the triad
  return (vhi - vlo) / 2 + 1;
}

}  // namespace

// Accumulator tiles the wide kernel's A update multiplies per k step, summed over the row
// blocks and the eight wavefronts of a workgroup: wavefront w holds the tiles w + 8 j of its
// block and runs them in groups of three (the last group of the fourteen holds two), a group
// whole once it holds one of them.
// k steps of four the wide kernel's T stage multiplies for a spin value with s active steps:
// three unconditionally, the last two when the fourth is active.
static int t_steps(int s) { return s <= 3 ? 3 : 5; }

static int wide_update_tiles(int RT, int CT, int nrb) {
  const int RTb = (RT + nrb - 1) / nrb;
  int total = 0;
  for (int rb = 0; rb < nrb; ++rb) {
    const int ntile = std::max(0, std::min(RTb, RT - rb * RTb)) * CT;
    for (int w = 0; w < 8; ++w) {
      const int ntw = std::max(0, (ntile - w + 7) / 8);
      total += std::min(14, (ntw + 2) / 3 * 3);
    }
  }
  return total;
}

void count_work(const Plan &p, double out[5]) {
  const int nd = p.nd, nd3 = nd * nd * nd;
  const int *J = p.two_j;
  const int d1 = p.i[0].n, d2 = p.i[1].n, d3 = p.i[2].n, d4 = p.i[3].n, d5 = p.i[4].n;
  const int xlo = p.X.lo2, xhi = p.X.lo2 + 2 * (p.X.n - 1);
  double terms = 0, modes = 0, xterms = 0;
  for (int64_t s = 0; s < p.nshell; ++s) {
    int o[6];
    int64_t r = s;
    for (int q = 5; q >= 0; --q) {
      o[q] = (int)(r % nd);
      r /= nd;
    }
    const int t[4] = {(o[0] * nd + o[1]) * nd + o[2], (o[3] * nd + o[4]) * nd + o[0],
                      (o[5] * nd + o[1]) * nd + o[3], (o[2] * nd + o[4]) * nd + o[5]};
    int klo[4], kn[4];
    bool live = true;
    for (int e = 0; e < 4; ++e) {
      klo[e] = p.kr[(e * nd3 + t[e]) * 2];
      kn[e] = p.kr[(e * nd3 + t[e]) * 2 + 1];
      live = live && kn[e] > 0;
    }
    if (!live) continue;
    const double k2 = kn[0], k3 = kn[1], k4 = kn[2], k5 = kn[3];
    terms += d1 * k2 * k3 * k4 * k5;
    modes += d1 * k2 * k3 * k4 * k5 * d5 + d1 * k2 * k3 * k4 * d5 * d4 + d1 * k2 * k3 * d4 * d5 * d3 +
             d1 * k2 * d3 * d4 * d5 * d2;
    const int l24 = J[L24] + 2 * o[1], l25 = J[L25] + 2 * o[2], l35 = J[L35] + 2 * o[4];
    for (int x = xlo; x <= xhi; x += 2) {
      xterms += (double)triad_count(p.i[0].lo2, d1, l25, x) * triad_count(klo[3], kn[3], J[L14], x) *
                triad_count(klo[2], kn[2], l35, x) * triad_count(klo[1], kn[1], l24, x) *
                triad_count(klo[0], kn[0], J[L13], x);
    }
  }
  out[0] = terms;
  out[1] = 2.0 * modes + 6.0 * xterms;
  // Factorised order: useful flops and MFMA-executed flops (padded tiles), as the ring
  // kernel evaluates them: per (core, i1, x) with non-empty active k4 and k3 windows.
  double useful = 0, executed = 0;
  const int KW = p.ring_KW > 0 ? p.ring_KW : 16;
  const int DI = p.ring_DI > 0 ? p.ring_DI : 8;
  const double rows = (double)DI * DI, cols = (double)DI * DI;  // padded tile rows / columns
  for (int o24 = 0; o24 < nd; ++o24)
    for (int o25 = 0; o25 < nd; ++o25)
      for (int o34 = 0; o34 < nd; ++o34)
        for (int o35 = 0; o35 < nd; ++o35) {
          const int l24 = J[L24] + 2 * o24, l25 = J[L25] + 2 * o25;
          const int l34 = J[L34] + 2 * o34, l35 = J[L35] + 2 * o35;
          (void)l34;
          int lo5[64], n5[64], lo4[64], n4[64], lo2[64], n2[64], lo3[64], n3[64];
          int w4lo = 1 << 30, w4hi = -1, w3lo = 1 << 30, w3hi = -1;
          for (int o = 0; o < nd && o < 64; ++o) {
            const int t5 = (o25 * nd + o35) * nd + o, t4 = (o * nd + o24) * nd + o34;
            const int t2 = (o * nd + o24) * nd + o25, t3 = (o34 * nd + o35) * nd + o;
            lo5[o] = p.kr[(3 * nd3 + t5) * 2];
            n5[o] = p.kr[(3 * nd3 + t5) * 2 + 1];
            lo4[o] = p.kr[(2 * nd3 + t4) * 2];
            n4[o] = p.kr[(2 * nd3 + t4) * 2 + 1];
            lo2[o] = p.kr[(0 * nd3 + t2) * 2];
            n2[o] = p.kr[(0 * nd3 + t2) * 2 + 1];
            lo3[o] = p.kr[(1 * nd3 + t3) * 2];
            n3[o] = p.kr[(1 * nd3 + t3) * 2 + 1];
            if (n5[o] == 0 || n4[o] == 0) n5[o] = n4[o] = 0;
            if (n2[o] == 0 || n3[o] == 0) n2[o] = n3[o] = 0;
            if (n4[o] > 0) {
              w4lo = std::min(w4lo, lo4[o]);
              w4hi = std::max(w4hi, lo4[o] + 2 * (n4[o] - 1));
            }
            if (n3[o] > 0) {
              w3lo = std::min(w3lo, lo3[o]);
              w3hi = std::max(w3hi, lo3[o] + 2 * (n3[o] - 1));
            }
          }
          if (w4hi < 0 || w3hi < 0) continue;
          for (int n1 = 0; n1 < d1; ++n1) {
            const int i1 = p.i[0].lo2 + 2 * n1;
            const int xa = std::max(std::abs(i1 - l25), xlo), xb = std::min(i1 + l25, xhi);
            for (int x = xa; x <= xb; x += 2) {
              const int a4 = std::max(w4lo, std::abs(l35 - x)), b4 = std::min(w4hi, l35 + x);
              const int a3 = std::max(w3lo, std::abs(l24 - x)), b3 = std::min(w3hi, l24 + x);
              if (a4 > b4 || a3 > b3) continue;
              const int na4 = (b4 - a4) / 2 + 1, na3 = (b3 - a3) / 2 + 1;
              for (int o = 0; o < nd && o < 64; ++o) {
                if (n5[o] > 0) {
                  const int c4 = triad_count(lo4[o], n4[o], l35, x);
                  const int c5 = triad_count(lo5[o], n5[o], J[L14], x);
                  useful += (double)d5 * c4 * (3.0 * c5 + 2.0 * d4);
                }
                if (n2[o] > 0) {
                  const int c3 = triad_count(lo3[o], n3[o], l24, x);
                  const int c2 = triad_count(lo2[o], n2[o], J[L13], x);
                  useful += (double)d2 * c3 * (3.0 * c2 + 2.0 * d3);
                }
              }
              useful += 2.0 * d5 * d4 * na4 * na3 + 2.0 * d5 * d4 * na3 * d3 * d2;
              const int s4 = ((b4 - w4lo) / 2) / 4 - ((a4 - w4lo) / 2) / 4 + 1;
              const int s3 = ((b3 - w3lo) / 2) / 4 - ((a3 - w3lo) / 2) / 4 + 1;
              if (p.ring_cls == kWideClass) {
                // Every stage on 16x16x4 tiles (2048 flops each): T5 / T2 over the active k5 /
                // k2 values in steps of 4 (at least three steps, else five), G / H per k4 / k3
                // position of the windows rounded out to multiples of 4 over the spin values in
                // steps of 4 (repeated per row block), P over the row tiles and one or two k3
                // column tiles, the update over the wavefronts' groups of tiles.
                int tsteps = 0;
                for (int o = 0; o < nd && o < 64; ++o) {
                  if (n5[o] > 0) {
                    const int ka = std::max(lo5[o], std::abs(x - J[L14]));
                    const int kb = std::min(lo5[o] + 2 * (n5[o] - 1), x + J[L14]);
                    if (kb >= ka) tsteps += t_steps(((kb - lo5[o]) / 2) / 4 - ((ka - lo5[o]) / 2) / 4 + 1);
                  }
                  if (n2[o] > 0) {
                    const int ka = std::max(lo2[o], std::abs(J[L13] - x));
                    const int kb = std::min(lo2[o] + 2 * (n2[o] - 1), J[L13] + x);
                    if (kb >= ka) tsteps += t_steps(((kb - lo2[o]) / 2) / 4 - ((ka - lo2[o]) / 2) / 4 + 1);
                  }
                }
                const int RT = (d5 * d4 + 15) / 16, CT = (d3 * d2 + 15) / 16;
                const int nq = ((((b3 - w3lo) / 2) | 3) + 16) / 16;
                const int upd_tiles = wide_update_tiles(RT, CT, p.ring_nrb);
                const int nG = (((b4 - w4lo) / 2) | 3) - (((a4 - w4lo) / 2) & ~3) + 1;
                const int nH = (((b3 - w3lo) / 2) | 3) - (((a3 - w3lo) / 2) & ~3) + 1;
                const double per_block = tsteps + (double)(nG + nH) * ((nd + 3) / 4);
                executed += 2048.0 * (p.ring_nrb * per_block + (double)RT * nq * s4 + (double)upd_tiles * s3);
              } else {
                executed += 2.0 * rows * KW * 4 * s4 + 2.0 * rows * cols * 4 * s3;
              }
            }
          }
        }
  out[2] = useful;
  out[3] = executed;
  out[4] = p.ring_cls;
}

// Booster blocks of a configuration in packing order (eq. (booster); edges 2..5, offset
// triples of their virtual links): the boundary and virtual spins of the edge's four links,
// the intertwiner ranges and the block's offset in the packed buffer.  Empty blocks are left out.
void booster_blocks(const Plan &p, std::vector<BoosterBlock> &out) {
  out.clear();
  const int nd = p.nd, nd3 = nd * nd * nd;
  for (int e = 0; e < 4; ++e)
    for (int t = 0; t < nd3; ++t) {
      const int kn = p.kr[(e * nd3 + t) * 2 + 1];
      if (kn == 0 || p.i[e + 1].n == 0) continue;
      const int o[3] = {t / (nd * nd), (t / nd) % nd, t % nd};
      int l[10];
      for (int n = 0; n < 10; ++n) l[n] = p.two_j[n];
      for (int q = 0; q < 3; ++q) l[kEdgeTriple[e][q]] += 2 * o[q];
      BoosterBlock b;
      b.edge = e;
      const int *L = kEdgeLinks[e + 1];
      for (int a = 0; a < 4; ++a) {
        b.jb[a] = p.two_j[L[a]];
        b.lb[a] = l[L[a]];
      }
      b.two_ilo = p.i[e + 1].lo2;
      b.idim = p.i[e + 1].n;
      b.two_klo = p.kr[(e * nd3 + t) * 2];
      b.kdim = kn;
      b.off = p.boff[(size_t)e * nd3 + t];
      out.push_back(b);
    }
}

}  // namespace eprl
