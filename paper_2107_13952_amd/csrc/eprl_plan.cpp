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
  if (maxtwo > 400) {
    msg << "spin 2j + 2dl = " << maxtwo << " exceeds the supported 400";
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
  return EPRL_OK;
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

}  // namespace eprl
