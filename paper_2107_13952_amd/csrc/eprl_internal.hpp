// Internal declarations shared by the host planner, the kernels and the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/eprl.h"

namespace eprl {

// A range of spins in two-units: values lo2, lo2 + 2, ..., lo2 + 2 (n - 1).
struct Range {
  int lo2 = 0;
  int n = 0;
};

// Link indices in the order (12, 13, 14, 15, 23, 24, 25, 34, 35, 45).
enum Link { L12 = 0, L13, L14, L15, L23, L24, L25, L34, L35, L45 };

// Everything the kernels need to know about one configuration (two_j, dl); built on the host.
struct Plan {
  int two_j[10];
  int dl = 0;
  int nd = 1;                 // dl + 1
  Range i[5];                 // boundary intertwiners i1..i5
  Range K[4];                 // union over shells of the k2..k5 ranges (global windows)
  Range X;                    // global window of the x summation spin
  int kmax = 0;               // largest k range of any shell
  int D = 0;                  // padded tile dimension of the assembly kernel (8 or 16)
  int64_t nshell = 0;         // (dl + 1)^6
  std::vector<int64_t> boff;  // packed booster offsets, 4 nd^3 + 1
  std::vector<int> kr;        // [4][nd^3][2]: lowest two_k and size of k_e per edge triple
  int fact_max = 0;           // largest factorial argument met by any 6j of the tables
  // 6j tables: sizes in doubles and offsets into one allocation.
  int64_t tsize[5] = {0, 0, 0, 0, 0};
  int64_t toff[6] = {0, 0, 0, 0, 0, 0};
  int64_t a_size = 0;         // entries of the vertex tensor
  // Factorised (ring) path: widest union over l45 of the k4 ranges of a core
  // (l24, l34 fixed) and over l23 of the k3 ranges (l34, l35 fixed); the ring kernel needs
  // them to fit its KW-wide LDS tiles, and all i and k ranges to fit 8.
  int ring_w4 = 0, ring_w3 = 0;
  int ring_KW = 0;            // 16 or 32 when the ring path applies, else 0
  int ring_DI = 0, ring_DK = 0;  // padded boundary / virtual intertwiner tile sizes (8 or 16)
  int ring_cls = -1;          // tile class of the ring kernel, -1 when it does not apply
  // Wide (all-matrix-core) kernel, tile class kWideClass: k windows padded to a multiple of 4
  // and the number of row blocks of A(i1) per work item.
  int ring_kw = 0, ring_nrb = 1;
  int ring_cls8 = -1;         // class among 0..7 (half chains on vector ALUs), -1 when none
};

// Largest 6j argument (two-units) the device evaluation is built for: up to it the alternating
// Racah sum cancels by at most ~1e15, which double-double arithmetic absorbs with a few ulp to
// spare; beyond it the cancellation grows past what 106 bits hold.
constexpr int kSixjMaxTwo = 200;

// Build a plan; returns EPRL_OK or an error code with a message in `err`.
int make_plan(const int two_j[10], int dl, Plan &p, std::string &err);
// Live-shell and term counts (host enumeration).
void count_terms(const Plan &p, int64_t &live, double &terms);
// Exact work counts: terms, per-shell-order flops, factorised-order useful and executed flops.
void count_work(const Plan &p, double out[5]);
// Primes up to n.
std::vector<int> primes_upto(int n);

// ---- kernel-side parameter blocks (passed by value) ----

struct TableParams {
  int two_j[10];
  int nd;
  int i1_lo2, i1_n;
  int K_lo2[4], K_n[4];
  int X_lo2, NX;
  int64_t toff[6];
  double *tables;
  const uint16_t *fexp;  // [fact_max + 1][nprime]
  const int *primes;
  int nprime;
};

struct VertexParams {
  int two_j[10];
  int nd;
  int i_lo2[5], i_n[5];
  int K_lo2[4], K_n[4];
  int X_lo2, NX;
  const double *T1, *T2, *T3, *T4, *T5;
  const double *B;
  const int64_t *boff;
  const int *kr;
  double *partial;        // [nchunk][i1][i2][i3][i4][i5]
  int64_t shell_begin, shell_end, chunk;
  int nchunk;
};

struct RingParams {
  int two_j[10];
  int nd;
  int i_lo2[5], i_n[5];
  // Index ranges of the ring tables U1..U5 (virtual spins, x) and the spin count tnd that strides
  // them: the configuration's own, or those of a configuration of the same spins at a larger dl
  // whose tables it shares (every index range of its own lies inside them).
  int K_lo2[4], K_n[4];
  int X_lo2, NX;
  int tnd;
  int xlo2, xhi2;         // the configuration's own x range (the loops' bounds)
  const double *U1, *U2, *U3, *U4, *U5;
  const double *B;
  const int64_t *boff;
  const int *kr;
  double *partial;        // [nchunk][i1][i2][i3][i4][i5]
  const int *bounds;      // [i1][nchunk + 1]: first core of each chunk of that i1
  int nchunk;
  int kw, nrb;            // wide kernel: padded k window, row blocks of A(i1)
};

struct ReduceParams {
  const double *partial;
  int nchunk;
  int64_t a_size;
  int i_lo2[5], i_n[5];
  double *A;
  int accumulate;
};

// Kernel launchers (defined in the .hip files).  They return hipSuccess or the launch error.
hipError_t launch_fexp_table(uint16_t *fexp, int fact_max, const int *primes, int nprime,
                             hipStream_t s);
hipError_t launch_sixj_tables(const TableParams &tp, int64_t total, hipStream_t s);
hipError_t launch_ring_tables(const TableParams &tp, int64_t total, hipStream_t s);
hipError_t launch_sixj_batch(const int *args, int n, double *out, const uint16_t *fexp,
                             const int *primes, int nprime, int fact_max, hipStream_t s);
hipError_t launch_assemble(const VertexParams &vp, int D, hipStream_t s);
hipError_t launch_reduce(const ReduceParams &rp, hipStream_t s);
int ring_class(int DI, int DK, int KW);
// Tile classes: 0..7 the 8/16-wide kernels of ring.hip, kWideClass the all-matrix-core kernel of
// wide.hip (boundary dimensions above 8).
constexpr int kWideClass = 8;
constexpr int kRingClasses = 9;
// Largest dl + 1 the wide kernel takes (its per-spin tiles must fit in LDS beside G and H).
constexpr int kWideMaxNd = 11;
// LDS bytes of the wide kernel; stg: with the core's booster blocks staged.
size_t wide_smem_bytes(int nd, const int i_n[5], int kw, int nrb, bool stg);
// Row blocks of A(i1) per work item so that each wavefront holds at most 12 accumulator tiles
// (0 when even one row tile needs more).
int wide_row_blocks(const int i_n[5]);
bool wide_fits(int nd, const int i_n[5], int kw, int nrb, bool stg = false);
hipError_t wide_init_attributes();
// Plain call, persistent (one workgroup per CU, ncu of them at most); next: eight device ints
// of scratch for the per-XCD counters (reset by the launch).
hipError_t launch_wide(const RingParams &rp, int *next, int ncu, hipStream_t s);
// Persistent launch over per-XCD item lists: list x is items [xoff[x], xoff[x + 1]) of
// items_dev (offsets relative to items_dev, device memory), next[0..7] its counters (zeroed).
hipError_t launch_wide_batch(const RingParams *cfgs_dev, const int *items_dev, const int *xoff_dev,
                             int nitems, size_t smem, bool stg, int grid, int *next, hipStream_t s);
// Splits the cores of the factorised path, for each i1, into chunks of equal estimated cost
// (x iterations plus the per-core set-up), about target_wg workgroups in all and at most
// kRingMaxPartialBytes of partial sums; fills bounds ([i1][nchunk + 1]) and, if asked for, the
// estimated cost of each chunk ([i1][nchunk], in x iterations) and returns nchunk.  Only the
// cores [core_lo, core_hi) are split (core_hi < 0: all); core index
// ((o24 * nd + o25) * nd + o34) * nd + o35 over the offsets of l24, l25, l34, l35.
constexpr size_t kRingMaxPartialBytes = size_t(256) << 20;
int ring_schedule(const Plan &p, int target_wg, std::vector<int> &bounds,
                  std::vector<double> *chunk_cost = nullptr, int core_lo = 0, int core_hi = -1);
int ring_row_blocks(const Plan &p);
// LDS bytes of the tile class at nd with staging level stg (-1: the most that fits).
size_t ring_smem_bytes(int cls, int nd, int stg = -1);
// Booster staging levels of the tile class that fit in LDS at nd, most first; returns their count.
int ring_stage_levels(int cls, int nd, int levels[3]);
// Largest dl + 1 the ring kernels stage booster blocks for.
constexpr int kRingMaxNd = 16;
hipError_t ring_init_attributes();
hipError_t launch_ring(const RingParams &rp, int cls, int stg, hipStream_t s);
hipError_t launch_ring_batch(const RingParams *cfgs_dev, const int *items_dev, int nitems, int cls,
                             int max_nd, int stg, int grid, int *next, hipStream_t s);
hipError_t launch_reset_counters(int *c, int n, hipStream_t s);
hipError_t launch_shell_fifteenj(const VertexParams &vp, int64_t shell, double *W,
                                 hipStream_t s);
// BF vertex of a plan made with dl = 0 (tables of the per-shell layout); total = entries of A.
hipError_t launch_bf_vertex(const VertexParams &vp, double *A, int64_t total, hipStream_t s);

struct ContractParams {
  int n[5];
  const double *A;
  const double *psi[5];
  double *partial;  // complex partial sums
  int nblocks;
};
struct GradPsiOut {
  double *p[5];
};
hipError_t launch_contract(const ContractParams &cp, double *F, hipStream_t s);
// Complex partial-sum slots of the fixed device scratch of the contraction (one per block of
// contract_partial_kernel) and its device address on the current device.
constexpr int kContractScratchSlots = 256;
hipError_t contract_scratch_address(double **ptr);
hipError_t launch_grad_psi(const ContractParams &cp, double gre, double gim, double *const out[5],
                           hipStream_t s);

// Booster builder (boosters.hip; 4jm coefficient tables in sixj.hip).
// One booster block: edge e (0..3 for edges 2..5), boundary and virtual spins of its four links
// (two-units, pairing (first second)(third fourth)), intertwiner ranges, packed offset.
struct BoosterBlock {
  int edge;
  int jb[4], lb[4];
  int two_ilo, idim, two_klo, kdim;
  int64_t off;
};
void booster_blocks(const Plan &p, std::vector<BoosterBlock> &out);
// A table of 4jm coefficients: out[o + m n + i] = 4jm(j; m-tuple m; two_lo + 2 i) for the M
// m-tuples at mtuples[mt + 4 m ..].
struct FourjmSet {
  int j[4];
  int two_lo, n;
  int M, mt;
  int64_t out;
};
hipError_t launch_fourjm_tables(const FourjmSet *sets_dev, int nsets, int max_entries,
                                const int *mtuples_dev, double *out, const uint16_t *fexp,
                                const int *primes, int nprime, hipStream_t s);
hipError_t launch_threejm_batch(const int *args, int n, double *out, const uint16_t *fexp,
                                const int *primes, int nprime, int fact_max, hipStream_t s);
// A boost matrix element d^{(rho, k = j)}_{j l m}(r): spins, the Y-map rho = gamma (j + 1), the
// phase factor of the basis convention, and the Jacobi-form constants of the two SU(2) d
// functions it integrates, d^j_{j m} and d^l_{j m}.
struct DKey {
  double rho, ph_re, ph_im, pre;      // pre = sqrt((2j+1)(2l+1))
  double nj, nl;                      // xi * sqrt(s! (s+mu+nu)! / ((s+mu)! (s+nu)!)) of each d
  int muj, nuj, sj, mul, nul, sl;     // Jacobi parameters of each d
};
struct BoosterParams {
  const DKey *keys;
  int nkeys;
  const double *sx, *sw;   // Gauss-Legendre nodes and weights of the s integral on [-1, 1]
  int ns;
  const double *r, *rw;    // r nodes (30-point rule, then 61-point rule) and their weights,
  int nr, nr30;            //   rw including sinh^2 r / (4 pi) and the Jacobian of u = e^{-r}
  double *dtab;            // complex [key][r]
  // blocks
  const int *binfo;        // per block: edge, idim, kdim, M, moff, kb[4]  (9 ints)
  const int64_t *boffs;    // per block: packed offset, ck offset
  const int *mtuples;      // per edge: its m-tuples (4 ints each), edge e at mt_edge[e]
  int mt_edge[4];
  int jb_edge[4][4];       // boundary spins of each edge's four links
  const double *ci;        // per edge: M x idim 4jm of the boundary spins, edge e at ci_edge[e]
  int64_t ci_edge[4];
  const double *ck;        // per block: M x kdim 4jm of the virtual spins
  double *I;               // per block and m-tuple: the two rules' integrals, complex (4 doubles)
  double *B;               // packed boosters (real parts of the 61-point values)
  double *stat;            // per block: max |G61 - G30|, max |G61|, max |Im G61|
  int nblocks, Mmax;
};
hipError_t launch_booster_dfun(const BoosterParams &bp, hipStream_t s);
hipError_t launch_booster_integrals(const BoosterParams &bp, hipStream_t s);
hipError_t launch_booster_assemble(const BoosterParams &bp, double *stat3, hipStream_t s);

// Multi-vertex contractions (network.hip).
struct TrailParams {
  const double *A;        // [lead][S] row-major
  int m;                  // trailing intertwiners contracted
  int n[5];               // their dimensions
  const double *psi[5];   // their vectors (complex)
  int64_t S;              // prod n[0..m-1]
  int nsplit;             // blocks per leading row
  double *T;              // complex [lead]
  double *partial;        // complex [lead][nsplit] when nsplit > 1
};
hipError_t launch_contract_vertices(const double *A, const double *B, int64_t total, int nblocks,
                                    double *partial, double *F, hipStream_t s);
int trailing_splits(int64_t nlead, int64_t S);
hipError_t launch_contract_trailing(const TrailParams &tp, int64_t nlead, hipStream_t s);
hipError_t launch_delta3(int n, int two_klo, int two_x, const double *TA, const double *TB,
                         const double *TC, double *F, hipStream_t s);

struct AdjointParams {
  VertexParams v;
  const double *psi[5];
  double *shell_g;        // [nshell][4][kmaxpad] complex
  int kpad;
};
hipError_t launch_adjoint_shells(const AdjointParams &ap, hipStream_t s);
// Adjoint in the factorised order (one workgroup per core, then a fixed-order sum per booster
// entry of `total`); the per-core G vectors go to gbuf (adjoint_ring_gbuf_bytes).  Applies where
// the factorised vertex kernels do, with dl + 1 <= kAdjRingMaxNd.
constexpr int kAdjRingMaxNd = 11;
constexpr size_t kAdjRingMaxLds = 160 * 1024 - 256;
// LDS sizes of the kernel for a configuration: kl = largest k range of a spin, iw = number of i1
// values, kw = widest core window of k5, k4 (over l45), k3 or k2 (over l23), ng = spins per group
// of the two halves.  kl = 0 when the windows are too wide for the kernel.
void adjoint_ring_dims(const Plan &p, int &kl, int &iw, int &kw, int &ng);
size_t adjoint_ring_smem(int nd, int kl, int iw, int kw, int ng);
size_t adjoint_ring_gbuf_bytes(int nd, int kl);
// Launch order of the adjoint's cores, longest first by an estimate of their work (the x values
// with both core windows non-empty, times the windows' widths), so that the last workgroups to
// start are short ones; every core writes its own G vectors, so the order changes no result.
void adjoint_ring_order(const Plan &p, std::vector<int> &order);
hipError_t adjoint_ring_init_attributes();
hipError_t launch_adjoint_ring(const RingParams &rp, int kl, int iw, int kw, int ng,
                               const int *order, const double *const psi[5], double *gbuf,
                               int64_t total, double gre, double gim, double *grad_b, hipStream_t s);
hipError_t launch_adjoint_reduce(const AdjointParams &ap, int64_t total, double gre, double gim,
                                 double *grad_b, hipStream_t s);

}  // namespace eprl
