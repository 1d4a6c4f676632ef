// FP64 6j symbols on the device and the five 6j tables of the vertex computation
// (Sec. 3.1 framed algorithm, step 4; the tensors S of eq. (15j)).
//
// Racah's single-sum formula (Racah 1942):
//   {a b c; d e f} = sqrt(P) sum_t (-1)^t (t+1)! / [prod_i (t - alpha_i)! prod_j (beta_j - t)!]
//   alpha = (a+b+c, a+e+f, d+b+f, d+e+c),  beta = (a+b+d+e, a+c+d+f, b+c+e+f),
//   P = prod over the four triads (x y z) of (x+y-z)! (x-y+z)! (-x+y+z)! / (x+y+z+1)!.
//
// Evaluation, designed so that the result is within a few ulp of the exact value:
//  * The common factor sqrt(P) * T0 (T0 = |first term|) is an exact rational square root.
//    Its prime factorisation is assembled from a table of prime exponents of n! (Legendre's
//    formula), and the product prod_p sqrt(p)^{E_p} is formed in double-double arithmetic
//    with a separate binary exponent, so no factorial is ever rounded.
//  * The remaining sum is 1 + r_0 + r_0 r_1 + ... with exact integer ratios
//    r_t = -(t+2) prod_j (beta_j - t) / prod_i (t + 1 - alpha_i); the ratios and the running
//    products and sum are carried in double-double, which removes the effect of the
//    alternating-sign cancellation at the spins handled here.
// Double-double primitives follow Dekker (1971) and Knuth (TAOCP vol. 2, 4.2.2).
#include "eprl_internal.hpp"

// The error-free transformations below need every product and sum rounded exactly as
// written: fusing p = a*b into a later p + e (the default contraction of device code) would
// destroy the error terms.
#pragma clang fp contract(off)

namespace eprl {

namespace {

struct dd {
  double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

__device__ __forceinline__ dd fast_two_sum(double a, double b) {
  double s = a + b;
  return {s, b - (s - a)};
}

__device__ __forceinline__ dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ dd dd_mul(dd a, dd b) {
  double p = a.hi * b.hi;
  double e = __builtin_fma(a.hi, b.hi, -p);
  e += a.hi * b.lo + a.lo * b.hi;
  return fast_two_sum(p, e);
}

// Quotient of two exactly representable integers as a double-double.
__device__ __forceinline__ dd dd_ratio(double num, double den) {
  double q = num / den;
  double r = __builtin_fma(-q, den, num);  // exact remainder
  return fast_two_sum(q, r / den);
}

// Double-double with a separate power-of-two exponent: value = (hi + lo) * 2^e.
struct dde {
  double hi, lo;
  int e;
};

__device__ __forceinline__ void normalise(dde &v) {
  int k;
  double h = __builtin_frexp(v.hi, &k);
  v.lo = __builtin_ldexp(v.lo, -k);
  v.hi = h;
  v.e += k;
}

__device__ __forceinline__ dde dde_mul(dde a, dde b) {
  dd m = dd_mul({a.hi, a.lo}, {b.hi, b.lo});
  dde r{m.hi, m.lo, a.e + b.e};
  normalise(r);
  return r;
}

// sqrt(q) of a small integer q as a double-double.
__device__ __forceinline__ dd dd_sqrt_int(double q) {
  double s = __builtin_sqrt(q);
  double r = __builtin_fma(-s, s, q);
  return fast_two_sum(s, r / (2.0 * s));
}

// base^n, n >= 0, by binary powering.
__device__ dde dde_pow(dd base, int n) {
  dde result{1.0, 0.0, 0};
  dde b{base.hi, base.lo, 0};
  normalise(b);
  while (n > 0) {
    if (n & 1) result = dde_mul(result, b);
    n >>= 1;
    if (n) b = dde_mul(b, b);
  }
  return result;
}

__device__ __forceinline__ bool triad_ok(int a, int b, int c) {
  return ((a + b + c) & 1) == 0 && c >= (a > b ? a - b : b - a) && c <= a + b;
}

// {a b c; d e f}, all arguments in two-units.  `fexp` holds v_p(n!) for n <= fact_max.
__device__ double sixj_device(int a, int b, int c, int d, int e, int f, const uint16_t *fexp,
                              const int *primes, int nprime) {
  if (!(triad_ok(a, b, c) && triad_ok(a, e, f) && triad_ok(d, b, f) && triad_ok(d, e, c)))
    return 0.0;
  const int al[4] = {(a + b + c) / 2, (a + e + f) / 2, (d + b + f) / 2, (d + e + c) / 2};
  const int be[3] = {(a + b + d + e) / 2, (a + c + d + f) / 2, (b + c + e + f) / 2};
  int tmin = al[0], tmax = be[0];
  for (int q = 1; q < 4; ++q) tmin = al[q] > tmin ? al[q] : tmin;
  for (int q = 1; q < 3; ++q) tmax = be[q] < tmax ? be[q] : tmax;
  // Factorial arguments with their exponent in P * T0^2.
  const int tri[4][3] = {{a, b, c}, {a, e, f}, {d, b, f}, {d, e, c}};
  int arg[24], coef[24];
  int na = 0, top = tmin + 1;
  for (int q = 0; q < 4; ++q) {
    const int x = tri[q][0], y = tri[q][1], z = tri[q][2];
    arg[na] = (x + y - z) / 2; coef[na++] = 1;
    arg[na] = (x - y + z) / 2; coef[na++] = 1;
    arg[na] = (-x + y + z) / 2; coef[na++] = 1;
    arg[na] = (x + y + z) / 2 + 1; coef[na++] = -1;
    if ((x + y + z) / 2 + 1 > top) top = (x + y + z) / 2 + 1;
  }
  arg[na] = tmin + 1; coef[na++] = 2;
  for (int q = 0; q < 4; ++q) { arg[na] = tmin - al[q]; coef[na++] = -2; }
  for (int q = 0; q < 3; ++q) { arg[na] = be[q] - tmin; coef[na++] = -2; }
  // prod_p sqrt(p)^{E_p}: numerator and denominator powers kept apart.
  dde num{0.5, 0.0, 1}, den{0.5, 0.0, 1};
  for (int ip = 0; ip < nprime; ++ip) {
    const int pr = primes[ip];
    if (pr > top) break;
    int E = 0;
    for (int q = 0; q < na; ++q) E += coef[q] * (int)fexp[arg[q] * nprime + ip];
    if (E == 0) continue;
    dd sp = dd_sqrt_int((double)pr);
    if (E > 0)
      num = dde_mul(num, dde_pow(sp, E));
    else
      den = dde_mul(den, dde_pow(sp, -E));
  }
  // Series in double-double.  Terms can grow far beyond the first one before they fall off:
  // the running term and sum are scaled down together by 2^-768 (exact) whenever the term
  // passes 2^768, and the scale is put back at the end.
  dd rho{1.0, 0.0}, sum{1.0, 0.0};
  int sexp = 0;
  for (int t = tmin; t < tmax; ++t) {
    double nu = -(double)(t + 2) * (double)(be[0] - t) * (double)(be[1] - t) * (double)(be[2] - t);
    double de = (double)(t + 1 - al[0]) * (double)(t + 1 - al[1]) * (double)(t + 1 - al[2]) *
                (double)(t + 1 - al[3]);
    rho = dd_mul(rho, dd_ratio(nu, de));
    sum = dd_add(sum, rho);
    if (__builtin_fabs(rho.hi) > 0x1p768) {
      rho = {__builtin_ldexp(rho.hi, -768), __builtin_ldexp(rho.lo, -768)};
      sum = {__builtin_ldexp(sum.hi, -768), __builtin_ldexp(sum.lo, -768)};
      sexp += 768;
    }
  }
  // value = (-1)^tmin * num / den * sum
  dd q;
  {
    // num / den in double-double: q = num.hi / den.hi, then one correction step.
    double qh = num.hi / den.hi;
    dd prod = dd_mul({qh, 0.0}, {den.hi, den.lo});
    dd diff = dd_add({num.hi, num.lo}, {-prod.hi, -prod.lo});
    q = fast_two_sum(qh, diff.hi / den.hi);
  }
  dd v = dd_mul(q, sum);
  double r = __builtin_ldexp(v.hi + v.lo, num.e - den.e + sexp);
  return (tmin & 1) ? -r : r;
}

// Wigner 3jm symbol (j1 j2 j3; m1 m2 m3), arguments in two-units, by Racah's single sum
//   (-1)^(j1-j2-m3) sqrt(D(j1 j2 j3) prod_a (j_a+m_a)! (j_a-m_a)!)
//     * sum_t (-1)^t / [t! (j3-j2+t+m1)! (j3-j1+t-m2)! (j1+j2-j3-t)! (j1-t-m1)! (j2-t+m2)!],
// D(abc) = (a+b-c)! (a-b+c)! (-a+b+c)! / (a+b+c+1)!, evaluated like the 6j symbol above: the
// common factor sqrt(D prod (j +- m)!) T0 as an exact square root from prime exponents, the
// series 1 + r_0 + r_0 r_1 + ... with exact integer ratios in double-double.
__device__ double threejm_device(int j1, int j2, int j3, int m1, int m2, int m3, const uint16_t *fexp,
                                 const int *primes, int nprime) {
  if (m1 + m2 + m3 != 0 || !triad_ok(j1, j2, j3)) return 0.0;
  const int jj[3] = {j1, j2, j3}, mm[3] = {m1, m2, m3};
  for (int q = 0; q < 3; ++q)
    if (mm[q] > jj[q] || -mm[q] > jj[q] || ((jj[q] - mm[q]) & 1)) return 0.0;
  // Integer (not two-unit) quantities.
  const int a1 = (j1 + j2 - j3) / 2, a2 = (j1 - m1) / 2, a3 = (j2 + m2) / 2;   // (. - t)!
  const int b1 = (j3 - j2 + m1) / 2, b2 = (j3 - j1 - m2) / 2;                   // (. + t)!
  int tmin = 0, tmax = a1;
  if (-b1 > tmin) tmin = -b1;
  if (-b2 > tmin) tmin = -b2;
  if (a2 < tmax) tmax = a2;
  if (a3 < tmax) tmax = a3;
  if (tmin > tmax) return 0.0;
  int arg[16], coef[16];
  int na = 0;
  arg[na] = (j1 + j2 - j3) / 2; coef[na++] = 1;
  arg[na] = (j1 - j2 + j3) / 2; coef[na++] = 1;
  arg[na] = (-j1 + j2 + j3) / 2; coef[na++] = 1;
  arg[na] = (j1 + j2 + j3) / 2 + 1; coef[na++] = -1;
  for (int q = 0; q < 3; ++q) {
    arg[na] = (jj[q] + mm[q]) / 2; coef[na++] = 1;
    arg[na] = (jj[q] - mm[q]) / 2; coef[na++] = 1;
  }
  arg[na] = tmin; coef[na++] = -2;
  arg[na] = b1 + tmin; coef[na++] = -2;
  arg[na] = b2 + tmin; coef[na++] = -2;
  arg[na] = a1 - tmin; coef[na++] = -2;
  arg[na] = a2 - tmin; coef[na++] = -2;
  arg[na] = a3 - tmin; coef[na++] = -2;
  const int top = (j1 + j2 + j3) / 2 + 1;
  dde num{0.5, 0.0, 1}, den{0.5, 0.0, 1};
  for (int ip = 0; ip < nprime; ++ip) {
    const int pr = primes[ip];
    if (pr > top) break;
    int E = 0;
    for (int q = 0; q < na; ++q) E += coef[q] * (int)fexp[arg[q] * nprime + ip];
    if (E == 0) continue;
    dd sp = dd_sqrt_int((double)pr);
    if (E > 0)
      num = dde_mul(num, dde_pow(sp, E));
    else
      den = dde_mul(den, dde_pow(sp, -E));
  }
  // term(t+1) / term(t) = -(a1 - t)(a2 - t)(a3 - t) / ((t + 1)(b1 + t + 1)(b2 + t + 1))
  dd rho{1.0, 0.0}, sum{1.0, 0.0};
  for (int t = tmin; t < tmax; ++t) {
    const double nu = -(double)(a1 - t) * (double)(a2 - t) * (double)(a3 - t);
    const double de = (double)(t + 1) * (double)(b1 + t + 1) * (double)(b2 + t + 1);
    rho = dd_mul(rho, dd_ratio(nu, de));
    sum = dd_add(sum, rho);
  }
  dd q;
  {
    double qh = num.hi / den.hi;
    dd prod = dd_mul({qh, 0.0}, {den.hi, den.lo});
    dd diff = dd_add({num.hi, num.lo}, {-prod.hi, -prod.lo});
    q = fast_two_sum(qh, diff.hi / den.hi);
  }
  dd v = dd_mul(q, sum);
  const double r = __builtin_ldexp(v.hi + v.lo, num.e - den.e);
  const int ph = (j1 - j2 - m3) / 2 + tmin;
  return (ph & 1) ? -r : r;
}

// 4jm(j1 j2 j3 j4; m1 m2 m3 m4)^(i): (j1 j2) coupled to i, then i with (j3 j4),
//   (-1)^(i - mi) (j1 j2 i; m1 m2 mi) (i j3 j4; -mi m3 m4),  mi = -(m1 + m2).
__device__ double fourjm_device(const int *j, const int *m, int i, const uint16_t *fexp,
                                const int *primes, int nprime) {
  const int mi = -(m[0] + m[1]);
  if (mi - m[2] - m[3] != 0) return 0.0;
  const double v = threejm_device(j[0], j[1], i, m[0], m[1], mi, fexp, primes, nprime) *
                   threejm_device(i, j[2], j[3], -mi, m[2], m[3], fexp, primes, nprime);
  return (((i - mi) / 2) & 1) ? -v : v;
}

// Coefficient tables of the booster contraction: set s (blockIdx.y), entry (m, i) of its
// M x n table = 4jm(j; m-tuple m; two_lo + 2 i).
__global__ void fourjm_table_kernel(const FourjmSet *sets, const int *mtuples, double *out,
                                    const uint16_t *fexp, const int *primes, int nprime) {
  const FourjmSet st = sets[blockIdx.y];
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= st.M * st.n) return;
  const int m = idx / st.n, i = idx % st.n;
  out[st.out + idx] = fourjm_device(st.j, mtuples + st.mt + 4 * m, st.two_lo + 2 * i, fexp, primes,
                                    nprime);
}

__global__ void threejm_batch_kernel(const int *args, int n, double *out, const uint16_t *fexp,
                                     const int *primes, int nprime, int fact_max) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int *a = args + 6 * idx;
  out[idx] = threejm_device(a[0], a[1], a[2], a[3], a[4], a[5], fexp, primes, nprime);
}

__global__ void fexp_kernel(uint16_t *fexp, int fact_max, const int *primes, int nprime) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (fact_max + 1) * nprime) return;
  const int n = idx / nprime, p = primes[idx % nprime];
  // Legendre: v_p(n!) = sum_k floor(n / p^k)
  int v = 0;
  for (long long pk = p; pk <= n; pk *= p) v += (int)(n / pk);
  fexp[idx] = (uint16_t)v;
}

// One thread per table entry.  Table t (0..4), its linear index decomposed row-major.
__global__ void sixj_table_kernel(TableParams tp, int64_t total) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  int t = 0;
  while (t < 4 && g >= tp.toff[t + 1]) ++t;
  int64_t idx = g - tp.toff[t];
  const int nd = tp.nd;
  const int *J = tp.two_j;
  const int NX = tp.NX;
  int64_t size;
  switch (t) {
    case 0: size = (int64_t)nd * tp.i1_n * tp.K_n[3] * NX; break;
    case 1: size = (int64_t)nd * nd * tp.K_n[3] * tp.K_n[2] * NX; break;
    case 2: size = (int64_t)nd * nd * nd * tp.K_n[2] * tp.K_n[1] * NX; break;
    case 3: size = (int64_t)nd * nd * tp.K_n[1] * tp.K_n[0] * NX; break;
    default: size = (int64_t)nd * tp.K_n[0] * tp.i1_n * NX; break;
  }
  if (idx >= size) return;  // alignment padding between tables
  const int x = tp.X_lo2 + 2 * (int)(idx % NX);
  int64_t r = idx / NX;
  int args[6];
  if (t == 0) {  // T1[o25][i1][k5][x] = {i1 l25 x; k5 j14 j15}
    int k5 = tp.K_lo2[3] + 2 * (int)(r % tp.K_n[3]); r /= tp.K_n[3];
    int i1 = tp.i1_lo2 + 2 * (int)(r % tp.i1_n); r /= tp.i1_n;
    int l25 = J[L25] + 2 * (int)r;
    int a6[6] = {i1, l25, x, k5, J[L14], J[L15]};
    for (int q = 0; q < 6; ++q) args[q] = a6[q];
  } else if (t == 1) {  // T2[o35][o45][k5][k4][x] = {j14 k5 x; l35 k4 l45}
    int k4 = tp.K_lo2[2] + 2 * (int)(r % tp.K_n[2]); r /= tp.K_n[2];
    int k5 = tp.K_lo2[3] + 2 * (int)(r % tp.K_n[3]); r /= tp.K_n[3];
    int l45 = J[L45] + 2 * (int)(r % nd); r /= nd;
    int l35 = J[L35] + 2 * (int)r;
    int a6[6] = {J[L14], k5, x, l35, k4, l45};
    for (int q = 0; q < 6; ++q) args[q] = a6[q];
  } else if (t == 2) {  // T3[o24][o34][o35][k4][k3][x] = {k4 l35 x; k3 l24 l34}
    int k3 = tp.K_lo2[1] + 2 * (int)(r % tp.K_n[1]); r /= tp.K_n[1];
    int k4 = tp.K_lo2[2] + 2 * (int)(r % tp.K_n[2]); r /= tp.K_n[2];
    int l35 = J[L35] + 2 * (int)(r % nd); r /= nd;
    int l34 = J[L34] + 2 * (int)(r % nd); r /= nd;
    int l24 = J[L24] + 2 * (int)r;
    int a6[6] = {k4, l35, x, k3, l24, l34};
    for (int q = 0; q < 6; ++q) args[q] = a6[q];
  } else if (t == 3) {  // T4[o23][o24][k3][k2][x] = {l24 k3 x; j13 k2 l23}
    int k2 = tp.K_lo2[0] + 2 * (int)(r % tp.K_n[0]); r /= tp.K_n[0];
    int k3 = tp.K_lo2[1] + 2 * (int)(r % tp.K_n[1]); r /= tp.K_n[1];
    int l24 = J[L24] + 2 * (int)(r % nd); r /= nd;
    int l23 = J[L23] + 2 * (int)r;
    int a6[6] = {l24, k3, x, J[L13], k2, l23};
    for (int q = 0; q < 6; ++q) args[q] = a6[q];
  } else {  // T5[o25][k2][i1][x] = {k2 j13 x; i1 l25 j12}
    int i1 = tp.i1_lo2 + 2 * (int)(r % tp.i1_n); r /= tp.i1_n;
    int k2 = tp.K_lo2[0] + 2 * (int)(r % tp.K_n[0]); r /= tp.K_n[0];
    int l25 = J[L25] + 2 * (int)r;
    int a6[6] = {k2, J[L13], x, i1, l25, J[L12]};
    for (int q = 0; q < 6; ++q) args[q] = a6[q];
  }
  tp.tables[g] = sixj_device(args[0], args[1], args[2], args[3], args[4], args[5], tp.fexp,
                             tp.primes, tp.nprime);
}

// Signed, x-major tables for the factorised (ring) assembly.  The phase (-1)^R of eq. (15j)
// splits over the five closed triads (i1 j12 j13), (k2 l23 l24), (k3 l34 l35), (k4 j14 l45),
// (k5 j15 l25), each with an integer half-sum r_n; every factor goes into the one table that
// carries all of its spins, and (2x+1) goes into the first table:
//   U1[o25][x][i1][k5]  = (2x+1) (-1)^{r1 + r5} {i1 l25 x; k5 j14 j15}
//   U2[o35][o45][x][k5][k4] = (-1)^{r4} {j14 k5 x; l35 k4 l45}
//   U3[o24][o34][o35][x][k4][k3] = (-1)^{r3} {k4 l35 x; k3 l24 l34}
//   U4[o23][o24][x][k3][k2] = (-1)^{r2} {l24 k3 x; j13 k2 l23}
//   U5[o25][x][k2][i1]  = {k2 j13 x; i1 l25 j12}
// so that W(i1, k2..k5) = sum_x U1 U2 U3 U4 U5 exactly.
__global__ void ring_table_kernel(TableParams tp, int64_t total) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  int t = 0;
  while (t < 4 && g >= tp.toff[t + 1]) ++t;
  int64_t idx = g - tp.toff[t];
  const int nd = tp.nd;
  const int *J = tp.two_j;
  const int NX = tp.NX;
  const int n1 = tp.i1_n, nK2 = tp.K_n[0], nK3 = tp.K_n[1], nK4 = tp.K_n[2], nK5 = tp.K_n[3];
  int64_t size;
  switch (t) {
    case 0: size = (int64_t)nd * NX * n1 * nK5; break;
    case 1: size = (int64_t)nd * nd * NX * nK5 * nK4; break;
    case 2: size = (int64_t)nd * nd * nd * NX * nK4 * nK3; break;
    case 3: size = (int64_t)nd * nd * NX * nK3 * nK2; break;
    default: size = (int64_t)nd * NX * nK2 * n1; break;
  }
  if (idx >= size) return;
  int64_t r = idx;
  double v = 0.0;
  int ph = 0;  // exponent of -1 (two-units, halved below)
  if (t == 0) {
    const int k5 = tp.K_lo2[3] + 2 * (int)(r % nK5); r /= nK5;
    const int i1 = tp.i1_lo2 + 2 * (int)(r % n1); r /= n1;
    const int x = tp.X_lo2 + 2 * (int)(r % NX); r /= NX;
    const int l25 = J[L25] + 2 * (int)r;
    v = (double)(x + 1) * sixj_device(i1, l25, x, k5, J[L14], J[L15], tp.fexp, tp.primes, tp.nprime);
    ph = (i1 + J[L12] + J[L13]) / 2 + (k5 + J[L15] + l25) / 2;
  } else if (t == 1) {
    const int k4 = tp.K_lo2[2] + 2 * (int)(r % nK4); r /= nK4;
    const int k5 = tp.K_lo2[3] + 2 * (int)(r % nK5); r /= nK5;
    const int x = tp.X_lo2 + 2 * (int)(r % NX); r /= NX;
    const int l45 = J[L45] + 2 * (int)(r % nd); r /= nd;
    const int l35 = J[L35] + 2 * (int)r;
    v = sixj_device(J[L14], k5, x, l35, k4, l45, tp.fexp, tp.primes, tp.nprime);
    ph = (k4 + J[L14] + l45) / 2;
  } else if (t == 2) {
    const int k3 = tp.K_lo2[1] + 2 * (int)(r % nK3); r /= nK3;
    const int k4 = tp.K_lo2[2] + 2 * (int)(r % nK4); r /= nK4;
    const int x = tp.X_lo2 + 2 * (int)(r % NX); r /= NX;
    const int l35 = J[L35] + 2 * (int)(r % nd); r /= nd;
    const int l34 = J[L34] + 2 * (int)(r % nd); r /= nd;
    const int l24 = J[L24] + 2 * (int)r;
    v = sixj_device(k4, l35, x, k3, l24, l34, tp.fexp, tp.primes, tp.nprime);
    ph = (k3 + l34 + l35) / 2;
  } else if (t == 3) {
    const int k2 = tp.K_lo2[0] + 2 * (int)(r % nK2); r /= nK2;
    const int k3 = tp.K_lo2[1] + 2 * (int)(r % nK3); r /= nK3;
    const int x = tp.X_lo2 + 2 * (int)(r % NX); r /= NX;
    const int l24 = J[L24] + 2 * (int)(r % nd); r /= nd;
    const int l23 = J[L23] + 2 * (int)r;
    v = sixj_device(l24, k3, x, J[L13], k2, l23, tp.fexp, tp.primes, tp.nprime);
    ph = (k2 + l23 + l24) / 2;
  } else {
    const int i1 = tp.i1_lo2 + 2 * (int)(r % n1); r /= n1;
    const int k2 = tp.K_lo2[0] + 2 * (int)(r % nK2); r /= nK2;
    const int x = tp.X_lo2 + 2 * (int)(r % NX); r /= NX;
    const int l25 = J[L25] + 2 * (int)r;
    v = sixj_device(k2, J[L13], x, i1, l25, J[L12], tp.fexp, tp.primes, tp.nprime);
    ph = 0;
  }
  tp.tables[g] = (ph & 1) ? -v : v;
}

__global__ void sixj_batch_kernel(const int *args, int n, double *out, const uint16_t *fexp,
                                  const int *primes, int nprime, int fact_max) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int *a = args + 6 * i;
  // Arguments beyond the factorial table are rejected by the host; guard anyway.
  int s = 0;
  for (int q = 0; q < 6; ++q) s = a[q] > s ? a[q] : s;
  if (2 * s + 2 > fact_max) {
    out[i] = __builtin_nan("");
    return;
  }
  out[i] = sixj_device(a[0], a[1], a[2], a[3], a[4], a[5], fexp, primes, nprime);
}

}  // namespace

hipError_t launch_fexp_table(uint16_t *fexp, int fact_max, const int *primes, int nprime,
                             hipStream_t s) {
  int total = (fact_max + 1) * nprime;
  fexp_kernel<<<(total + 255) / 256, 256, 0, s>>>(fexp, fact_max, primes, nprime);
  return hipGetLastError();
}

hipError_t launch_sixj_tables(const TableParams &tp, int64_t total, hipStream_t s) {
  int64_t blocks = (total + 255) / 256;
  sixj_table_kernel<<<(unsigned)blocks, 256, 0, s>>>(tp, total);
  return hipGetLastError();
}

hipError_t launch_ring_tables(const TableParams &tp, int64_t total, hipStream_t s) {
  int64_t blocks = (total + 255) / 256;
  ring_table_kernel<<<(unsigned)blocks, 256, 0, s>>>(tp, total);
  return hipGetLastError();
}

hipError_t launch_fourjm_tables(const FourjmSet *sets_dev, int nsets, int max_entries,
                                const int *mtuples_dev, double *out, const uint16_t *fexp,
                                const int *primes, int nprime, hipStream_t s) {
  if (nsets <= 0 || max_entries <= 0) return hipSuccess;
  dim3 grid((unsigned)((max_entries + 255) / 256), (unsigned)nsets);
  fourjm_table_kernel<<<grid, 256, 0, s>>>(sets_dev, mtuples_dev, out, fexp, primes, nprime);
  return hipGetLastError();
}

hipError_t launch_threejm_batch(const int *args, int n, double *out, const uint16_t *fexp,
                                const int *primes, int nprime, int fact_max, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  threejm_batch_kernel<<<(n + 255) / 256, 256, 0, s>>>(args, n, out, fexp, primes, nprime, fact_max);
  return hipGetLastError();
}

hipError_t launch_sixj_batch(const int *args, int n, double *out, const uint16_t *fexp,
                             const int *primes, int nprime, int fact_max, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  sixj_batch_kernel<<<(n + 255) / 256, 256, 0, s>>>(args, n, out, fexp, primes, nprime,
                                                    fact_max);
  return hipGetLastError();
}

}  // namespace eprl
