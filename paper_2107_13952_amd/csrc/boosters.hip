// Booster functions of eq. (booster) by quadrature on the device (Sec. 3.1 "Booster
// coefficients"):
//
//   B4(j, l; i, k) = sum_{m1..m4} 4jm(j; m; i) 4jm(l; m; k)
//                    * int_0^inf dr sinh^2(r) / (4 pi) prod_a d^{(rho_a, j_a)}_{j_a l_a m_a}(r),
//   rho_a = gamma (j_a + 1)  (the Y-map of eq. (booster)).
//
// The boost matrix elements d are computed from the principal-series realisation of SL(2,C) on
// functions on SU(2): a boost of rapidity r acts on the polar angle of SU(2) and multiplies by a
// power of the modulus of its lower-triangular factor, which gives
//
//   d_{jlm}(r) = sqrt((2j+1)(2l+1)) / (2 sinh r) int_{-r}^{r} ds e^{i rho s}
//                d^j_{j m}(beta(s)) d^l_{j m}(beta'(s)),
//   cos^2(beta/2) = (e^s - e^{-r}) / (2 sinh r),  sin^2(beta/2) = (e^r - e^s) / (2 sinh r),
//   cos^2(beta'/2) = e^{r-s} cos^2(beta/2),        sin^2(beta'/2) = e^{-r-s} sin^2(beta/2),
//
// times a phase exp(-i phi_{jl}) that fixes the basis convention (purely imaginary generator
// elements between l and l + 1, and d_{j l -m} = (-1)^{l-j} conj(d_{j l m}), under which the
// boosters are real).  The s integral is a Gauss-Legendre sum (the integrand is analytic); the
// SU(2) functions are evaluated in their Jacobi-polynomial form
//   d^J_{m' m}(beta) = xi sqrt(s! (s+mu+nu)! / ((s+mu)! (s+nu)!)) sin^mu(beta/2) cos^nu(beta/2)
//                      P_s^{(mu, nu)}(cos beta),   mu = |m - m'|, nu = |m + m'|,
// with the stable three-term recurrence of P in its degree, cos beta = cos^2 - sin^2 and the
// half-angle functions as square roots of the expressions above (no angle is formed).
//
// The r integral follows the quadrature of Sec. 3.1: u = e^{-r} maps it to (0, 1], cut into n
// subintervals growing linearly from u = 0; each gets a 30- and a 61-point Gauss-Legendre rule
// (the host builds the nodes); the 61-point sum is the value and |61 - 30| the error estimate.
//
// Kernels: (1) d on every (j, l, m) and r node (one wavefront per pair, lanes over the s
// nodes); (2) per booster block and m-tuple the r integral of the product of its four d
// (one wavefront each, lanes over the r nodes); (3) per block the contraction with the 4jm
// coefficient tables (sixj.hip) and the error and magnitude statistics.  All sums run in a fixed
// order.
#include "eprl_internal.hpp"

namespace eprl {

namespace {

__device__ __forceinline__ double ipow(double x, int n) {
  double r = 1.0;
  for (int q = 0; q < n; ++q) r *= x;
  return r;
}

// Jacobi polynomial P_n^{(a, b)}(x) by the recurrence in the degree.
__device__ double jacobi(int n, int a, int b, double x) {
  if (n == 0) return 1.0;
  double p0 = 1.0, p1 = (a + 1) + 0.5 * (a + b + 2) * (x - 1.0);
  for (int k = 2; k <= n; ++k) {
    const double c = 2.0 * k + a + b;
    const double a1 = 2.0 * k * (k + a + b) * (c - 2.0);
    const double a2 = (c - 1.0) * ((double)a * a - (double)b * b);
    const double a3 = (c - 1.0) * c * (c - 2.0);
    const double a4 = 2.0 * (k + a - 1.0) * (k + b - 1.0) * c;
    const double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// SU(2) d in Jacobi form from cos^2 and sin^2 of the half angle.
__device__ __forceinline__ double dsu2(double norm, int mu, int nu, int s, double c2, double s2) {
  const double sh = __builtin_sqrt(s2 > 0.0 ? s2 : 0.0), ch = __builtin_sqrt(c2 > 0.0 ? c2 : 0.0);
  return norm * ipow(sh, mu) * ipow(ch, nu) * jacobi(s, mu, nu, c2 - s2);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  return v;
}

// (1) d_{jlm}(r) for key `key` and r node `ir`: one wavefront, lanes over the s nodes.
__global__ __launch_bounds__(256) void booster_dfun_kernel(BoosterParams bp) {
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= (int64_t)bp.nkeys * bp.nr) return;  // uniform over the wavefront
  const int key = (int)(wave / bp.nr), ir = (int)(wave % bp.nr);
  const DKey K = bp.keys[key];
  const double r = bp.r[ir];
  const double sh2 = 2.0 * sinh(r), emr = exp(-r);
  double re = 0.0, im = 0.0;
  for (int q = lane; q < bp.ns; q += 64) {
    const double x = bp.sx[q], w = bp.sw[q];
    const double s = r * x;
    // e^s - e^-r = e^-r expm1(r (1 + x)) and e^r - e^s = e^s expm1(r (1 - x)): no cancellation
    // at small r.
    const double ep = expm1(r * (1.0 + x)), em = expm1(r * (1.0 - x));
    const double es = exp(s), ems = exp(-s);
    const double c2 = emr * ep / sh2, s2 = es * em / sh2;
    const double c2p = ems * ep / sh2, s2p = emr * em / sh2;
    const double f = w * dsu2(K.nj, K.muj, K.nuj, K.sj, c2, s2) * dsu2(K.nl, K.mul, K.nul, K.sl, c2p, s2p);
    double sn, cs;
    sincos(K.rho * s, &sn, &cs);
    re += f * cs;
    im += f * sn;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) {
    const double scale = K.pre * r / sh2;
    bp.dtab[2 * wave] = scale * (re * K.ph_re - im * K.ph_im);
    bp.dtab[2 * wave + 1] = scale * (re * K.ph_im + im * K.ph_re);
  }
}

// (2) Per block (blockIdx.y) and m-tuple (one wavefront each): the two rules' integrals of the
// product of the block's four d functions.
__global__ __launch_bounds__(256) void booster_integrals_kernel(BoosterParams bp) {
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int mi = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int *bi = bp.binfo + 9 * b;
  const int e = bi[0], M = bi[3], moff = bi[4];
  if (mi >= M) return;
  const int *mt = bp.mtuples + bp.mt_edge[e] + 4 * mi;
  const double *d[4];
  for (int a = 0; a < 4; ++a) {
    // row of (j_a, l_a, m_a): the key base of (j_a, l_a) at m = -j_a, plus (m_a + j_a) / 2
    const int row = bi[5 + a] + (mt[a] + bp.jb_edge[e][a]) / 2;
    d[a] = bp.dtab + 2 * (int64_t)row * bp.nr;
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int rule = 0; rule < 2; ++rule) {
    const int q0 = rule ? bp.nr30 : 0, q1 = rule ? bp.nr : bp.nr30;
    double re = 0.0, im = 0.0;
    for (int q = q0 + lane; q < q1; q += 64) {
      double pr = d[0][2 * q], pi = d[0][2 * q + 1];
      for (int a = 1; a < 4; ++a) {
        const double xr = d[a][2 * q], xi = d[a][2 * q + 1];
        const double t = pr * xr - pi * xi;
        pi = pr * xi + pi * xr;
        pr = t;
      }
      re += bp.rw[q] * pr;
      im += bp.rw[q] * pi;
    }
    acc[2 * rule] = wave_sum(re);
    acc[2 * rule + 1] = wave_sum(im);
  }
  if (lane == 0)
    for (int q = 0; q < 4; ++q) bp.I[4 * (int64_t)(moff + mi) + q] = acc[q];
}

// (3) One workgroup per block: entry (i, k) = sum over the m-tuples of 4jm(j; m; i) 4jm(l; m; k)
// times each rule's integral; the 61-point real part is the booster, |61 - 30| its error.
__global__ __launch_bounds__(256) void booster_assemble_kernel(BoosterParams bp) {
  __shared__ double red[3][256];
  const int b = blockIdx.x;
  const int *bi = bp.binfo + 9 * b;
  const int e = bi[0], idim = bi[1], kdim = bi[2], M = bi[3], moff = bi[4];
  const double *ci = bp.ci + bp.ci_edge[e];
  const double *ck = bp.ck + bp.boffs[2 * b + 1];
  double *out = bp.B + bp.boffs[2 * b];
  double err = 0.0, mag = 0.0, imag = 0.0;
  for (int idx = threadIdx.x; idx < idim * kdim; idx += blockDim.x) {
    const int i = idx / kdim, k = idx % kdim;
    double g30r = 0.0, g30i = 0.0, g61r = 0.0, g61i = 0.0;
    for (int m = 0; m < M; ++m) {
      const double c = ci[(int64_t)m * idim + i] * ck[(int64_t)m * kdim + k];
      const double *I = bp.I + 4 * (int64_t)(moff + m);
      g30r += c * I[0];
      g30i += c * I[1];
      g61r += c * I[2];
      g61i += c * I[3];
    }
    out[idx] = g61r;
    err = fmax(err, hypot(g61r - g30r, g61i - g30i));
    mag = fmax(mag, hypot(g61r, g61i));
    imag = fmax(imag, __builtin_fabs(g61i));
  }
  red[0][threadIdx.x] = err;
  red[1][threadIdx.x] = mag;
  red[2][threadIdx.x] = imag;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = fmax(red[q][threadIdx.x], red[q][threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x < 3) bp.stat[3 * b + threadIdx.x] = red[threadIdx.x][0];
}

// Maxima of the per-block statistics.
__global__ __launch_bounds__(256) void booster_stat_kernel(const double *stat, int nblocks, double *out) {
  __shared__ double red[3][256];
  double v[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
    for (int q = 0; q < 3; ++q) v[q] = fmax(v[q], stat[3 * b + q]);
  for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = fmax(red[q][threadIdx.x], red[q][threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x < 3) out[threadIdx.x] = red[threadIdx.x][0];
}

}  // namespace

hipError_t launch_booster_dfun(const BoosterParams &bp, hipStream_t s) {
  const int64_t waves = (int64_t)bp.nkeys * bp.nr;
  if (waves == 0) return hipSuccess;
  booster_dfun_kernel<<<(unsigned)((waves + 3) / 4), 256, 0, s>>>(bp);
  return hipGetLastError();
}

hipError_t launch_booster_integrals(const BoosterParams &bp, hipStream_t s) {
  if (bp.nblocks == 0 || bp.Mmax == 0) return hipSuccess;
  dim3 grid((unsigned)((bp.Mmax + 3) / 4), (unsigned)bp.nblocks);
  booster_integrals_kernel<<<grid, 256, 0, s>>>(bp);
  return hipGetLastError();
}

hipError_t launch_booster_assemble(const BoosterParams &bp, double *stat3, hipStream_t s) {
  if (bp.nblocks == 0) return hipSuccess;
  booster_assemble_kernel<<<bp.nblocks, 256, 0, s>>>(bp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  booster_stat_kernel<<<1, 256, 0, s>>>(bp.stat, bp.nblocks, stat3);
  return hipGetLastError();
}

}  // namespace eprl
