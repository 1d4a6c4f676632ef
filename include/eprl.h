/*
 * eprl.h - C ABI of the MI355X (gfx950) library for the EPRL vertex tensor in the booster
 * decomposition (Gozzini, "A high-performance code for EPRL spin foam amplitudes",
 * arXiv:2107.13952).
 *
 * What is computed (Sec. 2, eq. (vertex-ampl) and eq. (15j)):
 *
 *   A(i1..i5) = prod_{e=1..5} sqrt(2 i_e + 1)
 *               sum_{shells l} sum_{k2..k5} prod_{e=2..5} (2 k_e + 1) B_e(i_e, k_e; l)
 *               {15j}(l; i1, k2, k3, k4, k5)
 *
 *   {15j} = (-1)^R sum_x (2x+1) {i1 l25 x; k5 j14 j15} {j14 k5 x; l35 k4 l45}
 *                                {k4 l35 x; k3 l24 l34} {l24 k3 x; j13 k2 l23}
 *                                {k2 j13 x; i1 l25 j12},      R = sum of the 15 entries.
 *
 * Conventions shared by every entry point:
 *  - Spins are passed as two_j = 2 j (non-negative ints), ten of them in link order
 *    (12, 13, 14, 15, 23, 24, 25, 34, 35, 45) (the order of the spin list in Sec. 4.1).
 *  - dl = number of shells (Delta s of Sec. 2): l_ab = j_ab + o_ab, o_ab = 0..dl, on the six
 *    links 23, 24, 25, 34, 35, 45; l12..l15 stay at the boundary spins (gauge fixing of
 *    eq. (vertex-ampl)).  Shells are the tuples (o23, o24, o25, o34, o35, o45) numbered
 *    lexicographically, o45 fastest: there are (dl+1)^6 of them.
 *  - Edge e couples its four links (p q)(r s):  e1 (12 13)(14 15), e2 (23 24)(25 12),
 *    e3 (34 35)(13 23), e4 (45 14)(24 34), e5 (15 25)(35 45) (the booster tensors of step 3
 *    of the framed algorithm of Sec. 3.1).  Boundary intertwiner i_e and virtual k_e run in
 *    unit steps from max(|p-q|,|r-s|) to min(p+q,r+s); index n <-> lowest value + n.
 *  - The vertex tensor is FP64, row-major [i1][i2][i3][i4][i5] (i5 fastest); this is the
 *    byte layout of the paper's column-major A^{i5 i4 i3 i2 i1} (Sec. 3.1, step 7).
 *  - Boosters (eq. (booster)) are the raw B4 values, without the (2k+1) factor, packed
 *    FP64: for e = 2..5, for the triple of virtual spins of that edge
 *        e2: (l23, l24, l25)  e3: (l34, l35, l23)  e4: (l45, l24, l34)  e5: (l25, l35, l45)
 *    with offsets (o1, o2, o3) enumerated lexicographically (o3 fastest), one block of
 *    dim(i_e) x dim(k_e) values, row-major (k fastest).  An empty k range is an empty block.
 *    eprl_layout() returns the offsets.
 *  - Complex numbers are interleaved (re, im) FP64 pairs.
 *  - Device pointers are HIP device allocations owned by the caller; the library never
 *    frees or retains them beyond the call.  Every device-side call is enqueued on the
 *    context's stream and returns without synchronising unless stated otherwise.
 *  - Return value 0 on success, a negative EPRL_E* code on failure; the message is then
 *    available from eprl_last_error().  The library never aborts the process.
 */
#ifndef EPRL_H
#define EPRL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EPRL_OK 0
#define EPRL_EINVAL (-1) /* inadmissible spins, dl < 0, null or mismatched argument    */
#define EPRL_ENOMEM (-2) /* device or host allocation failed                           */
#define EPRL_EHIP (-3)   /* a HIP runtime call or kernel launch failed                 */
#define EPRL_ERANGE (-4) /* spins or dimensions beyond what the kernels are built for  */

typedef struct eprl_ctx eprl_ctx;

/* Create a context bound to HIP device `device` and stream `hip_stream` (a hipStream_t; NULL
 * means the null stream).  The context owns a grow-only device workspace (6j tables,
 * per-chunk partial sums) that is freed by eprl_destroy.  Returns EPRL_EHIP when the device
 * cannot be selected. */
int eprl_create(eprl_ctx **out, int device, void *hip_stream);
void eprl_destroy(eprl_ctx *ctx);
/* Text of the last error on this context; valid until the next call on it. */
const char *eprl_last_error(const eprl_ctx *ctx);
/* Change the stream subsequent calls are enqueued on.  When it differs from the current one,
 * the new stream is made to wait (an event, no host synchronisation) for the work already
 * enqueued on the old stream, which may still use the context's workspace. */
int eprl_set_stream(eprl_ctx *ctx, void *hip_stream);

/* How eprl_vertex_tensor evaluates the shell sum (both give the same tensor up to rounding):
 *  EPRL_ALGO_SHELL  the framed algorithm of Sec. 3.1 literally: per shell the {15j} tensor W
 *                   and the four booster mode products k5, k4, k3, k2, accumulated over shells;
 *  EPRL_ALGO_RING   the same sum regrouped by linearity: for each x of eq. (15j) and each
 *                   (l24, l25, l34, l35) the l45 and l23 sums are taken inside the two halves
 *                   of the closed chain of 6j and booster matrices, then contracted over k4 and
 *                   k3 with FP64 matrix-core tiles.  Needs every i and k range <= 16 and at
 *                   most 16 values per virtual spin (dl <= 15); used for full-range calls
 *                   only (EPRL_ERANGE when forced where it does not apply);
 *  EPRL_ALGO_AUTO   (default) RING where it applies, SHELL otherwise;
 *  EPRL_ALGO_RING_VALU  RING restricted to the kernels that take the l45 / l23 half chains on
 *                   vector ALUs (tile classes 0..7): for boundary dimensions above 8 RING
 *                   otherwise runs every stage on matrix-core tiles (class 8); kept as a
 *                   cross-check and for shell counts above 11 (EPRL_ERANGE where neither
 *                   applies).  Same sum, results agree to rounding. */
#define EPRL_ALGO_AUTO 0
#define EPRL_ALGO_SHELL 1
#define EPRL_ALGO_RING 2
#define EPRL_ALGO_RING_VALU 3
int eprl_set_algorithm(eprl_ctx *ctx, int algo);

/* Work split of the factorised order per tile class (the class is out[4] of eprl_count_work):
 * the shell sum is cut into chunks of cores of equal estimated cost, about target_workgroups
 * workgroups per launch (0: the default, 8192), and staging_level picks how many booster blocks
 * of a core are held in LDS (2: all four, 1: the two of the second stage, 0: none, -1: the
 * most that fits; a level that does not fit falls back to the next lower one).  The paper
 * adapts the split of its loops to the machine in the same spirit (Sec. 3.1,
 * "Parallelization").  The split changes the order of the floating-point sums (results agree
 * to rounding) but every call with the same setting is bitwise repeatable, and plain and
 * batched calls use the same setting.  EPRL_EINVAL for values out of range. */
int eprl_set_tuning(eprl_ctx *ctx, int tile_class, int target_workgroups, int staging_level);

/* Autotuner: times the vertex tensor of this configuration (boosters device, A device scratch
 * of prod(dims_i) doubles, overwritten) in the factorised order for target workgroups
 * 2048, 4096, 8192, 16384 and every staging level that fits (one warm-up call, then the
 * fastest of three timed calls per setting), keeps the fastest setting for
 * the configuration's tile class on this context (as eprl_set_tuning would) and writes
 * out[0] = tile class, out[1] = target workgroups, out[2] = staging level.  Synchronises the
 * context's stream.  EPRL_ERANGE when the factorised order does not apply. */
int eprl_autotune(eprl_ctx *ctx, const int two_j[10], int dl, const double *boosters, double *A,
                  int out[3]);

/* Host-only (no GPU use).  Ranges of the vertex tensor (eq. (vertex-ampl)) and the packed
 * booster layout described above.  Every call that plans a configuration returns EPRL_ERANGE
 * when a 6j symbol of its tables would have an argument above two_j = 200 (j + dl, the
 * intertwiners and x all at most 100), the range of the device 6j evaluation.
 *   dims_i[5]        out: dim(i1) .. dim(i5)
 *   two_ilo[5]       out (may be NULL): lowest two_i of each boundary intertwiner
 *   booster_offsets  out (may be NULL): 4 (dl+1)^3 + 1 offsets in doubles; the last one is
 *                    the total size of the booster buffer.
 * Returns EPRL_EINVAL for inadmissible input. */
int eprl_layout(const int two_j[10], int dl, int dims_i[5], int two_ilo[5],
                int64_t *booster_offsets);

/* Host-only.  Number of live shells (every k_e range non-empty) among the (dl+1)^6, and the
 * number of {15j} x booster terms sum_{live shells} dim(i1) prod_e dim(k_e). */
int eprl_count_terms(const int two_j[10], int dl, int64_t *live_shells, double *terms);

/* Host-only.  Exact work of one vertex tensor, for rooflines:
 *   out[0] = {15j} x booster terms (as eprl_count_terms);
 *   out[1] = FP64 flops of the per-shell order: 2 x (multiply-adds of the four mode products)
 *            + 6 per (term, allowed x) for the {15j} sums;
 *   out[2] = useful FP64 flops of the factorised order (active index ranges only);
 *   out[3] = FP64 flops its matrix-core tiles execute (16x16x4 tiles, padding included);
 *   out[4] = tile class of the factorised kernel for this configuration (0..7), or -1 when
 *            the configuration falls back to the per-shell order. */
int eprl_count_work(const int two_j[10], int dl, double out[5]);

/* The vertex tensor of eq. (vertex-ampl): the sum of the framed algorithm of Sec. 3.1 (6j
 * tables (step 4); per shell the {15j} tensor W (6(i)) contracted with the booster
 * sub-matrices (6(ii)) over k5, k4, k3, k2 (6(iii)) and accumulated (6(iv)); finally
 * A *= prod_e sqrt(2 i_e + 1)), evaluated in the order set by eprl_set_algorithm.
 *   boosters  device, booster_offsets[last] doubles in the packed layout
 *   A         device, prod(dims_i) doubles, overwritten
 *   gamma     the Barbero-Immirzi parameter the boosters were computed with; it enters A only
 *             through the boosters and is checked to be finite and positive.
 * The shell sum is evaluated in a fixed order: repeated calls give bitwise identical A. */
int eprl_vertex_tensor(eprl_ctx *ctx, const int two_j[10], int dl, double gamma,
                       const double *boosters, double *A);

/* The SU(2) BF vertex tensor, the "BF vertex (15j) tensors" of the interface of Sec. 3.2 and
 * the vertex of the BF studies of Sec. 4.2: eq. (vertex-ampl) with no shells (dl = 0) and no
 * boosters,
 *     A(i1..i5) = prod_{e=1..5} sqrt(2 i_e + 1) {15j}(j; i1, i2, i3, i4, i5),
 * the {15j} of eq. (15j) at l = j and k_e = i_e.  A: device, prod(dims_i) doubles in the
 * layout of eprl_vertex_tensor ([i1..i5] row-major, dims from eprl_layout with dl = 0),
 * overwritten.  Any intertwiner dimension is accepted (one thread per entry); spins are
 * limited only by the 6j range (EPRL_ERANGE above it). */
int eprl_bf_vertex_tensor(eprl_ctx *ctx, const int two_j[10], double *A);

/* Same, restricted to shells with index in [shell_begin, shell_end) of the (dl+1)^6
 * enumeration.  accumulate = 0 overwrites A, 1 adds to it.  Since A is a sum over shells,
 * consecutive ranges reproduce the full tensor: this is the resume / sharding unit. */
int eprl_vertex_tensor_range(eprl_ctx *ctx, const int two_j[10], int dl, double gamma,
                             const double *boosters, int64_t shell_begin, int64_t shell_end,
                             int accumulate, double *A);

/* Same, restricted to the shells of the "cores" [core_begin, core_end) in the factorised order
 * (regrouping by linearity of the shell sum of eq. (vertex-ampl); the paper distributes shells
 * over workers, Sec. 3.1 "Parallelization"): core index
 *     ((o24 (dl+1) + o25) (dl+1) + o34) (dl+1) + o35,   o_ab = (l_ab - j_ab) in [0, dl],
 * with every l23 and l45 of each core included.  accumulate = 0 overwrites A, 1 adds to it;
 * consecutive core ranges reproduce the full tensor, and the range [0, (dl+1)^4) gives the same
 * bits as eprl_vertex_tensor.  This is the resume / sharding unit of the factorised order (the
 * shell-range call evaluates in the per-shell order).  EPRL_EINVAL for a range outside
 * [0, (dl+1)^4] or when the per-shell order is forced; EPRL_ERANGE when the configuration has
 * no factorised evaluation (intertwiner or k dimension above 16, core window above 32). */
int eprl_vertex_tensor_cores(eprl_ctx *ctx, const int two_j[10], int dl, double gamma,
                             const double *boosters, int64_t core_begin, int64_t core_end,
                             int accumulate, double *A);

/* n independent vertex tensors (configuration c: two_j[10 c .. 10 c + 9], dl[c],
 * boosters[c], A[c]); the host arrays of pointers hold device pointers.  The 6j tables, one
 * persistent launch per tile class over a longest-first work queue of all configurations and
 * the reductions are captured into a HIP graph, replayed while the configurations, pointers
 * and algorithm are unchanged.  Results are bitwise equal to n calls of eprl_vertex_tensor. */
int eprl_vertex_tensor_batched(eprl_ctx *ctx, int n, const int *two_j, const int *dl,
                               double gamma, const double *const *boosters, double *const *A);

/* Shell scan: the vertex tensors A(dl) for dl = 0, 1, ..., dl_max of one spin configuration, as
 * needed for the convergence of the shell sum (Sec. 4.1 and the "EPRL vertex" study of Sec. 4.2:
 * A(dl) = A(dl - 1) + the shells whose largest offset is dl).  boosters: device, packed for
 * dl_max (eprl_layout(two_j, dl_max)); each A(dl) reads the blocks of its own shells from it.
 * A: device, (dl_max + 1) prod(dims_i) doubles, A(dl) at offset dl prod(dims_i), overwritten.
 * The dl_max + 1 tensors run as one batch (one graph of table builds, persistent launches and
 * reductions; see eprl_vertex_tensor_batched): every A(dl) has the bits of
 * eprl_vertex_tensor(two_j, dl) on its own packed boosters.  Errors as eprl_vertex_tensor. */
int eprl_vertex_tensor_scan(eprl_ctx *ctx, const int two_j[10], int dl_max, double gamma,
                            const double *boosters, double *A);

/* Boundary contraction (Sec. 3.2, `contract`):
 *   F = sum_{i1..i5} A(i1..i5) psi1(i1) psi2(i2) psi3(i3) psi4(i4) psi5(i5)
 * without complex conjugation.  A device FP64 [i1..i5]; psi[a] device complex vectors of
 * length dims_i[a]; F device, one complex number. */
int eprl_contract_boundary(eprl_ctx *ctx, const int dims_i[5], const double *A,
                           const double *const psi[5], double *F);

/* Same contraction for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): identical arguments, kernels
 * and result (bitwise) as eprl_contract_boundary, but the 256 complex partial sums live in a
 * fixed device array of the library (4 KiB per GPU, held until the process ends) instead of the
 * context's workspace, and no hipMalloc, hipFree or other allocating call is made.  The array
 * holds 256 partial sums, which every contraction uses whatever the size of A (EPRL_ERANGE if
 * a call ever needed more).  All calls on one GPU share the array: calls that overlap in time
 * on that GPU (different streams or contexts) race and must be ordered by the caller. */
int eprl_contract_boundary_noalloc(eprl_ctx *ctx, const int dims_i[5], const double *A,
                                   const double *const psi[5], double *F);

/* Complete contraction of two vertex tensors (the two-vertex test of Sec. 3.3 "Tensor
 * contractions on CPU and GPU"; vertex tensors glued over all five intertwiners, Sec. 3.1
 * "Tensor contractions"):
 *   F = sum_{i1..i5} A(i1..i5) B(i1..i5).
 * A, B: device FP64, prod(dims_i) entries each in the same layout; F: device, one double.
 * Summed in a fixed order (bitwise repeatable).  EPRL_EINVAL for a non-positive dimension. */
int eprl_contract_vertices(eprl_ctx *ctx, const int dims_i[5], const double *A, const double *B,
                           double *F);

/* Partial contraction of a vertex with boundary vectors on its last m intertwiners, leaving a
 * tensor in the first 5 - m (each vertex of the Delta_3 amplitude of Sec. 4.2 keeps its two
 * bulk intertwiners; the paper's contract(v, c3, c2, c1) on its column-major A^{i5..i1} pairs
 * c3 with i5, c2 with i4, c1 with i3, i.e. psi = {c1, c2, c3} here):
 *   T(i1..i_{5-m}) = sum_{i_{6-m}..i5} A(i1..i5) psi[0](i_{6-m}) ... psi[m-1](i5)
 * without complex conjugation.  A: device FP64 [i1..i5]; psi: host array of m device complex
 * vectors (interleaved re, im) of lengths dims_i[5-m..4]; T: device complex, row-major over
 * (i1..i_{5-m}) (one complex number for m = 5, which is eprl_contract_boundary).  Fixed-order
 * sums.  EPRL_EINVAL for m outside 1..5 or a null vector. */
int eprl_contract_trailing(eprl_ctx *ctx, const int dims_i[5], const double *A, int m,
                           const double *const *psi, double *T);

/* Delta_3 amplitude from its three partially contracted vertices (Sec. 4.2, the Delta_3
 * listing): with the bulk intertwiners k = (two_klo + 2 n') / 2, n' = 0..n-1, and the spin x of
 * the internal face,
 *   F = (-1)^x (2x + 1) sum_{k1, k2, k3} (-1)^(k1 + k2 + k3) TA[k1][k2] TB[k3][k1] TC[k2][k3]
 * (each matrix is the eprl_contract_trailing output of one vertex, m = 3, row-major over its
 * first two intertwiners; the triangle runs k1 -> k2 -> k3 -> k1).  TA, TB, TC: device complex
 * n x n; F: device complex.  EPRL_EINVAL unless 1 <= n <= 256 and two_klo, two_x are even
 * (integer spins: the phases are then real). */
int eprl_contract_delta3(eprl_ctx *ctx, int n, int two_klo, int two_x, const double *TA,
                         const double *TB, const double *TC, double *F);

/* Adjoint of the boundary contraction composed with the vertex tensor.  With g = grad_F
 * (host complex), writes g * dF/dpsi_a (device, complex, length dims_i[a]) and
 * g * dF/dB (device, complex, same packing and size as the boosters) where the derivatives
 * are the holomorphic ones of the multilinear function F(psi, B).  The {15j} tensors are
 * recomputed shell by shell; no per-shell data is stored.  grad_psi entries or
 * grad_boosters may be NULL to skip them. */
int eprl_contract_boundary_adjoint(eprl_ctx *ctx, const int two_j[10], int dl,
                                   const double *boosters, const double *A,
                                   const double *const psi[5], const double grad_F[2],
                                   double *const grad_psi[5], double *grad_boosters);

/* Booster functions of eq. (booster) for every block of a configuration, in the packed layout
 * of eprl_layout (edges 2..5, offset triples of their virtual links, rows i, columns k), by the
 * quadrature of Sec. 3.1 "Booster coefficients":
 *   B4(j, l; i, k) = sum_m 4jm(j; m; i) 4jm(l; m; k)
 *                    int_0^inf dr sinh^2 r / (4 pi) prod_a d^{(gamma (j_a+1), j_a)}_{j_a l_a m_a}(r)
 * (Y-map of eq. (booster); 4jm couples (first second)(third fourth) links of the edge).  The r
 * integral maps u = e^{-r} to (0, 1] and cuts it into n subintervals growing linearly from u = 0,
 * each with 30- and 61-point Gauss-Legendre rules; n doubles from 16 (at most 512) until the
 * largest |61-point - 30-point| entry is at most tol times the largest entry.  The boost matrix
 * elements d come from the principal-series realisation on SU(2) (an s integral of two SU(2) d
 * functions, 256 Gauss-Legendre points), in the basis convention under which the boosters are
 * real; B receives the real parts.
 *   B     device, booster_offsets[last] doubles, overwritten
 *   info  host, 3 doubles or NULL: the largest error estimate, the largest |imaginary part| of an
 *         entry, and the n used.
 * Synchronises with the context's stream once per n tried (the convergence test).  EPRL_EINVAL
 * for inadmissible spins or non-positive gamma or tol. */
int eprl_boosters(eprl_ctx *ctx, const int two_j[10], int dl, double gamma, double tol,
                  double *B, double info[3]);

/* Diagnostic: n Wigner 3jm symbols (j1 j2 j3; m1 m2 m3) (args: n x 6 two-unit values, host
 * int32, |value| <= 200, EPRL_ERANGE otherwise) with the device routine of the booster builder
 * (Racah's single sum, exact prefactor, double-double series); out: n doubles (device). */
int eprl_threejm_batch(eprl_ctx *ctx, int n, const int *args, double *out);

/* Diagnostic: evaluate n 6j symbols {a b c; d e f} (args: n x 6 two_j values, host int32,
 * each in 0..200, EPRL_ERANGE otherwise) with the same device routine the table builder uses;
 * out: n doubles (device).  Up to two_j = 200 the alternating Racah sum cancels by at most
 * ~1e15, which its double-double evaluation absorbs: results are within a few ulp. */
int eprl_sixj_batch(eprl_ctx *ctx, int n, const int *args, double *out);

/* Diagnostic: the {15j} tensor W(i1, k2, k3, k4, k5) of one shell (the intermediate of
 * step 6(i), including the (-1)^R phase), written to W (device, row-major, dims
 * dim(i1) x dim(k2) x ... x dim(k5)); kdims[4] (host, out) receives dim(k2..k5). */
int eprl_shell_fifteenj(eprl_ctx *ctx, const int two_j[10], int dl, int64_t shell,
                        int kdims[4], double *W, int64_t capacity);

/* Per-kernel timing with HIP events recorded on the context's stream around each launch.
 * kernel ids: 0 = 6j table builder, 1 = per-shell vertex assembly, 2 = shell-sum reduction,
 * 3 = adjoint shell kernel, 4 = factorised (ring) vertex assembly, 5 = BF vertex,
 * 6 = persistent factorised assembly of a batch (one launch per tile class).  While timing is
 * on, eprl_vertex_tensor_batched enqueues its launch sequence directly instead of replaying
 * the captured graph (same kernels, same results), so that each launch can be bracketed.
 * eprl_timing_enable(ctx, 1) starts recording (clearing earlier records), 0 stops.
 * eprl_timing_read synchronises the stream and returns the summed duration in milliseconds and
 * the number of launches recorded for `kernel`. */
int eprl_timing_enable(eprl_ctx *ctx, int enable);
int eprl_timing_read(eprl_ctx *ctx, int kernel, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* EPRL_H */
