/*
 * pdsink.h - C ABI of the MI355X (gfx950) persistence-diagram Sinkhorn library.
 *
 * Method: Lacombe, Cuturi, Oudot, "Large Scale computation of Means and
 * Clusters for Persistence Diagrams using Optimal Transport" (NeurIPS 2018).
 * A diagram is a d x d histogram on [0,1]^2 plus a diagonal bin Delta
 * (section 3, "Discretization"); the Gibbs kernel K of the (d^2+1)-point
 * ground space is applied in separable form (Proposition 2) and the
 * transport cost in separable form (Proposition 3).
 *
 * Conventions for every entry point below:
 *  - Pointers marked (device) are device memory of the context's GPU;
 *    pointers marked (host) are host memory.  The caller owns every buffer;
 *    the library owns only the context's small constant tables.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it and its outputs are valid once it has completed.
 *  - Return 0 on success, a negative PDSINK_E* code otherwise.  Argument
 *    errors are detected on the host before anything is enqueued; nothing is
 *    thrown across the boundary.  pdsink_strerror() names each code.
 *  - Histograms are float32, row-major d x d, row index = birth cell,
 *    column index = death cell: cell (i, j) holds the mass of the points
 *    with floor(birth d) = i and floor(death d) = j (index d-1 for 1.0).
 *  - Ground cost (readings of section 3): c(i,k) = (|i-k|/d)^p per axis, so
 *    C((i,j),(k,l)) = c(i,k) + c(j,l), and the diagonal cost
 *    c_Delta(i,j) = 2 (|j-i|/(2d))^p; gamma is in the same cost units.
 *  - A context is immutable after creation; calls on different streams are
 *    safe when each uses its own workspace.
 */
#ifndef PDSINK_H
#define PDSINK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PDSINK_OK        0
#define PDSINK_EINVAL   -1   /* bad argument (size, pointer, parameter, point) */
#define PDSINK_ENOMEM   -2   /* workspace too small or device allocation failed */
#define PDSINK_EDEVICE  -3   /* HIP runtime error (launch, copy, device) */
#define PDSINK_ERANGE   -4   /* a result was not representable (see status bits) */

/* Precision of the grid contractions (the two GEMMs of Proposition 2). */
#define PDSINK_FP32        0  /* FP32 operands on MFMA, FP32 accumulation          */
#define PDSINK_BF16_REFINE 1  /* BF16 operands until err <= switch_tol, then FP32  */

/* Distance kernel of a context (pdsink_params.kernel).  Both compute the same
 * iteration, stopping rule and cost (Algorithm 1, Propositions 2 and 3); they
 * differ in tiling and padding.  The general kernel pads d to 32, 64, 128 or
 * 256 and contracts over the padded grid; the resident kernel (grids 33 to
 * 100) contracts over d rounded up to 16 and keeps the scaled kernels of both
 * half steps in LDS between refits of the scales.  Pairs with a warm-start
 * state, barycenter solves, bounds and pairs the resident kernel cannot hold
 * (supports beyond 512 cells or below the diagonal) always run in the general
 * kernel, at its own padding (a context at d <= 64 holds the resident
 * kernel's 128-padded tables beside the general kernel's). */
#define PDSINK_KERNEL_AUTO      0  /* resident for 33 <= d <= 100 with BF16_REFINE and
                                    * for 65 <= d <= 100 with FP32; general otherwise */
#define PDSINK_KERNEL_RESIDENT  1  /* resident kernel; d in [33, 100], else PDSINK_EINVAL */
#define PDSINK_KERNEL_GENERAL   2  /* general kernel at every d */

/* Per-pair status bits written by sinkhorn_dist_batch / kmeans_assign. */
#define PDSINK_ST_CONVERGED  0  /* err <= tol                                      */
#define PDSINK_ST_MAX_ITER   1  /* stopped at max_iter with err > tol              */
#define PDSINK_ST_NONFINITE  2  /* a kernel product vanished or overflowed: cost = NaN */
#define PDSINK_ST_RANGE      4  /* scaling residual left the representable range  */
#define PDSINK_ST_LOG_PATH   8  /* solved again in the log domain after NONFINITE or
                                 * RANGE (then those two bits are clear)          */

typedef struct pdsink_ctx pdsink_ctx;

typedef struct {
  int32_t d;            /* grid size, 2 <= d <= 256                                    */
  double  p;            /* ground exponent, p >= 1 (the paper's experiments use 2)     */
  double  gamma;        /* entropic parameter, >= 1e-5, in cost units of [0,1]^2       */
  double  tol;          /* stop when (||P1-a||_1 + |.|_Delta)/m <= tol; 0 = run max_iter */
  int32_t max_iter;     /* cap on full (u, v) iterations, >= 1                         */
  int32_t precision;    /* PDSINK_FP32 or PDSINK_BF16_REFINE                           */
  double  switch_tol;   /* BF16_REFINE: switch to FP32 once err <= switch_tol (or after
                         * max_iter / 2 iterations); stopping is decided in FP32 only */
  int32_t kernel;       /* PDSINK_KERNEL_*: tiling of the distance solves (0 = AUTO)   */
} pdsink_params;

/* Create a context for `params` on HIP device `device`: validates the
 * parameters and uploads the per-(d, gamma, p) tables of the 1-D kernels
 * k = exp(-c/gamma), k_Delta and costs c, c_Delta (section 3, the tables
 * before Propositions 2 and 3), as exact (exponent, mantissa) pairs.
 * (host) params, (host) out.  Returns PDSINK_EINVAL for d outside [2, 256],
 * p < 1, gamma < 1e-5 (the integer log2 scales of the iterates, about
 * 1.44 / gamma octaves, must stay far inside the int32 range the kernels
 * use), tol < 0, max_iter < 1, an unknown precision or kernel, or
 * PDSINK_KERNEL_RESIDENT outside d in [33, 100]. */
int pdsink_ctx_create(const pdsink_params* params, int device, pdsink_ctx** out);

/* Release the context's device tables.  NULL is a no-op. */
void pdsink_ctx_destroy(pdsink_ctx* ctx);

/* Parameters the context was created with (host out). */
int pdsink_ctx_params(const pdsink_ctx* ctx, pdsink_params* out);

#define PDSINK_OP_DIST        0
#define PDSINK_OP_KMEANS      1
#define PDSINK_OP_BARYCENTER  2
#define PDSINK_OP_DIST_WARM   3   /* sinkhorn_dist_batch with a warm-start state */
/* Workspace (device bytes) an operation needs for `n_items` (pairs for DIST and
 * DIST_WARM, diagrams x centroids for KMEANS, diagrams for BARYCENTER).
 * (host) bytes. */
int pdsink_workspace_bytes(const pdsink_ctx* ctx, int op, int64_t n_items, size_t* bytes);

/* Discretisation (section 3, "Discretization"; supplementary, error control
 * due to discretisation).  Diagram n owns points [offsets[n], offsets[n+1])
 * of `pts`, each (birth, death) in float32.  Writes hist[n] (d x d counts,
 * overwritten) and mass[n] = number of points kept.  A point outside [0,1]^2,
 * non-finite, or with birth > death is not counted; the number of such points
 * is added to *n_bad.  The cell index floor(x d) is taken in exact arithmetic.
 *   pts     (device) float32 [total, 2]
 *   offsets (device) int64   [n_diag + 1], non-decreasing, offsets[0] = 0
 *   hist    (device) float32 [n_diag, d, d]  out
 *   mass    (device) double  [n_diag]        out
 *   n_bad   (device) int32   [1]             in/out (accumulated), may be NULL
 * n_diag = 0 is a no-op. */
int pd_discretize(pdsink_ctx* ctx, const float* pts, const int64_t* offsets, int64_t n_diag,
                  float* hist, double* mass, int32_t* n_bad, void* stream);

/* Algorithm 1 for a batch of pairs.  Pair q transports
 * a = (hist_a[ia[q]], |hist_b[ib[q]]|) onto b = (hist_b[ib[q]], |hist_a[ia[q]]|)
 * (Proposition 1: D1 + R D2 onto D2 + R D1).  Iterates the Sinkhorn map
 * (section 2) in alternating form from an initial v (Algorithm 1's initial
 * (u, v): the first half step computes u from v, so only v is an input),
 * u-update first, applying K by Proposition 2, until the marginal error
 * dist(P, Pi(a,b)) / m <= tol or max_iter iterations, then returns the
 * Sinkhorn cost <P_t, C> of Proposition 3, reduced in FP64.
 *   hist_a, hist_b (device) float32 [*, d, d]  histogram pools (may alias)
 *   ia, ib         (device) int32   [n_pairs]  indices into the pools
 *   state          (device) double  [n_pairs, d*d + 1] in/out, may be NULL:
 *                  natural log of v on the grid cells (row-major, as the
 *                  histograms) and on the diagonal bin (last entry); -inf is
 *                  v = 0.  NULL starts from v = 1 on every cell and the bin.
 *                  Given, the solve starts from this v on supp(b) and the bin
 *                  (entries off supp(b) are read as 0: the first v-update
 *                  zeroes them anyway) and, on return, state holds log v_t
 *                  (-inf off supp(b)).  A v whose log2 spans more than about
 *                  200 octaves within the grid after row and column scaling
 *                  sets PDSINK_ST_RANGE.  With a state the workspace is
 *                  pdsink_workspace_bytes(DIST_WARM, n_pairs), the pairs run
 *                  in the general kernels (not the resident d <= 100 variant),
 *                  and pairs flagged NONFINITE or RANGE keep their flags (no
 *                  log-domain re-solve: its iterates have no scaled v).
 *   cost           (device) double  [n_pairs]  out: <P_t, C>
 *   iters          (device) int32   [n_pairs, 2] out: iterations in BF16, in FP32
 *   err            (device) float   [n_pairs]  out: marginal error / m at stopping
 *   status         (device) int32   [n_pairs]  out: PDSINK_ST_* bits
 *   ws, ws_bytes   (device) workspace of at least pdsink_workspace_bytes(DIST, n_pairs)
 *                  bytes (DIST_WARM with a state); PDSINK_ENOMEM if smaller
 * Masses are the histogram sums.  n_pairs = 0 is a no-op.  Any support size
 * is accepted: pairs whose supports exceed the register lists (512 cells per
 * side) run again with their lists in the workspace, from the same launch
 * sequence.  A pair whose scaled solve ends NONFINITE or RANGE (a kernel so
 * sharp that one grid step costs tens of octaves, gamma d^2 well below 1) is
 * solved again from the start by the same iteration in log-sum-exp form over
 * the two supports (up to 1024 cells per side; larger pairs keep their
 * flags): maxima, logarithms, sums and the cost in FP64, the exponentials
 * FP32-accurate (exponent split in FP64, hardware base-2 exponential), so the
 * result matches the FP64 log-domain iteration to the FP32 tolerance.  Status
 * PDSINK_ST_LOG_PATH, iterations reported in the FP32 slot. */
int sinkhorn_dist_batch(pdsink_ctx* ctx, int64_t n_pairs,
                        const float* hist_a, const float* hist_b,
                        const int32_t* ia, const int32_t* ib, double* state,
                        double* cost, int32_t* iters, float* err, int32_t* status,
                        void* ws, size_t ws_bytes, void* stream);

/* Completion record of one pair (sinkhorn_dist_batch_notify): the pair's
 * outputs, then `tag`, which the device stores last with release ordering at
 * system scope.  A host thread that reads tag equal to the call's tag, and
 * only then the other fields, sees the pair's final outputs.  32 bytes. */
typedef struct {
  double   cost;
  float    err;
  int32_t  status;
  int32_t  iters[2];
  uint32_t tag;
  uint32_t reserved;    /* not written */
} pdsink_done;

/* sinkhorn_dist_batch (state NULL; same iteration, outputs and workspace,
 * Algorithm 1 of section 3) that also posts each pair's outputs to done[q] as
 * soon as they are final, while the launches of the call still run: for a
 * serving loop that completes a request when its own pairs are done, not when
 * the whole batch is.  A pair's outputs are final at the end of its solve,
 * or, when that solve flags it NONFINITE or RANGE, after the log-domain
 * re-solve (the last launch of the call posts those pairs).  Every pair is
 * posted exactly once per call, before the call's work on `stream` is done.
 *   done  pdsink_done [n_pairs] out: host memory the device can write
 *         (hipHostMalloc, e.g. pinned torch tensors) or device memory;
 *         records are written whole, tag last; `reserved` is not written
 *   tag   non-zero value written to done[q].tag; use a new tag per call on
 *         reused records, so that a record of an earlier call is not taken
 *         for this one
 * PDSINK_EINVAL when done is NULL or tag is 0 (n_pairs > 0); otherwise as
 * sinkhorn_dist_batch. */
int sinkhorn_dist_batch_notify(pdsink_ctx* ctx, int64_t n_pairs,
                               const float* hist_a, const float* hist_b,
                               const int32_t* ia, const int32_t* ib,
                               double* cost, int32_t* iters, float* err, int32_t* status,
                               pdsink_done* done, uint32_t tag,
                               void* ws, size_t ws_bytes, void* stream);

/* sinkhorn_dist_batch with no workspace argument and no device allocation, for
 * callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The routing flags, launch order
 * and support-list slots live in one static device array of
 * PDSINK_NOALLOC_SCRATCH_BYTES, which every GPU the library runs on holds from
 * the loading of the library's code until the process ends; its address is
 * looked up when a context is created.  The caller passes inputs and outputs
 * as for sinkhorn_dist_batch with state = NULL, and the results are the same
 * bit for bit: the
 * same kernels run, with as many list slots as the array holds (all of them at
 * grids up to 128; 15 at grids beyond 128, where every launch strides over the
 * batch, so there the call is slower).
 * Errors: PDSINK_ENOMEM when n_pairs > PDSINK_NOALLOC_MAX_PAIRS; PDSINK_EDEVICE
 * when the array's address could not be found on the context's device; others
 * as sinkhorn_dist_batch.  Every call on one GPU uses that GPU's one array, and
 * the array keeps the last call's contents (every byte a call reads is written
 * by the same call first): calls that overlap on one GPU, from different
 * streams or threads, race and must be serialised by the caller. */
#define PDSINK_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
#define PDSINK_NOALLOC_MAX_PAIRS     ((int64_t)1 << 18)
int sinkhorn_dist_batch_noalloc(pdsink_ctx* ctx, int64_t n_pairs,
                                const float* hist_a, const float* hist_b,
                                const int32_t* ia, const int32_t* ib,
                                double* cost, int32_t* iters, float* err, int32_t* status,
                                void* stream);

/* sinkhorn_dist_batch plus the error control of section 3 ("Upper and Lower
 * Bounds"; Algorithm 1's optional outputs) for the final (u_t, v_t):
 *   upper (device) double [n_pairs] out, may be NULL: <R_t, C>, R_t the
 *         rounding of P_t = diag(u_t) K diag(v_t) onto Pi(a, b) (rounding
 *         algorithm of the supplementary material), priced by Proposition 4
 *   lower (device) double [n_pairs] out, may be NULL: <alpha^{c cbar}, a> +
 *         <alpha^c, b> with alpha = gamma log u_t, both c-transforms (inf over
 *         the ground space, every grid cell and the diagonal bin) computed
 *         by separable min-plus passes over the grid
 * so that lower <= L_C(a, b) <= upper up to rounding.  Both are NaN for a pair
 * whose status has PDSINK_ST_NONFINITE, and 0 for an empty pair; a pair solved
 * by the log-domain path (PDSINK_ST_LOG_PATH) gets them from its log
 * scalings, by the same definitions.  The K
 * applications inside are exact sums over the two supports, O(|supp a| |supp b|)
 * per pair; the transforms cost O(d^3) per pair.  Other arguments, errors and
 * the workspace are those of sinkhorn_dist_batch. */
int sinkhorn_dist_bounds_batch(pdsink_ctx* ctx, int64_t n_pairs,
                               const float* hist_a, const float* hist_b,
                               const int32_t* ia, const int32_t* ib,
                               double* cost, int32_t* iters, float* err, int32_t* status,
                               double* upper, double* lower,
                               void* ws, size_t ws_bytes, void* stream);

/* Algorithm 2: smoothed barycenter of the diagrams hist[0..n_diag) (section 4).
 * Pairs (z + R a_i, a_i + R z) are iterated to `tol` of the context
 * (warm-started), the gradient of Proposition 5 averaged over the diagrams,
 * gamma (mean_i log u_i + log v_i,Delta), and z <- z * exp(-lambda grad).
 * Stops when |E_t / E_{t-1} - 1| < energy_rtol or after max_outer steps,
 * where E_t = mean_i S(z_t + R a_i, a_i + R z_t) (Algorithm 2, energy step).
 *   hist     (device) float32 [n_diag, d, d]
 *   z        (device) float32 [d, d] in/out: initial z if init_uniform == 0,
 *            otherwise overwritten with the uniform measure on cells j >= i of
 *            total mass = mean diagram mass; on return, z_t.
 *   energy   (host)   double out, E_t;  outer (host) int32 out, t
 * The outer steps are all enqueued on `stream` at once: the energy and the
 * stopping test run on the device, and the launches of the steps after the
 * stop do nothing; the call synchronises `stream` once, at the end, to read
 * the energy and the step count.  n_diag >= 1.  PDSINK_ERANGE when an inner solve ends with
 * PDSINK_ST_NONFINITE or PDSINK_ST_RANGE (its iterates left the scaled
 * representation, gamma d^2 of order 1 or below): the energy and the step
 * would then be wrong, and these warm-started solves do not take the
 * log-domain path; z holds the last good iterate. */
int pd_barycenter(pdsink_ctx* ctx, int64_t n_diag, const float* hist,
                  double lambda, int32_t max_outer, double energy_rtol, int32_t init_uniform,
                  float* z, double* energy, int32_t* outer,
                  void* ws, size_t ws_bytes, void* stream);

/* Entropic sharpening of smoothed barycenters (section 4, the paragraph after
 * Algorithm 2: the barycenters are smeared, and sharpening is the paper's
 * pointer to more spiked ones).  For each histogram z[i] (d x d, in place),
 * with M its mass and p = z[i] / M on its positive cells: if the Shannon
 * entropy -sum p log p exceeds h0, z[i] <- M p^beta / sum p^beta with the
 * beta > 1 at which that entropy equals h0 (FP64 bisection to adjacent
 * doubles); if h0 <= log n_max, n_max the number of cells at the maximum,
 * z[i] becomes M / n_max on those cells (beta = +inf, the limit).  Mass,
 * support (but for the limit) and the order of the cells are kept.
 *   z    (device) float32 [n, d, d] in/out
 *   h0   target entropy in nats, finite and >= 0, else PDSINK_EINVAL
 *   beta (device) double  [n] out, may be NULL: the exponent used (1 = unchanged)
 * n = 0 is a no-op. */
int pd_sharpen(pdsink_ctx* ctx, int64_t n, float* z, double h0, double* beta, void* stream);

/* Quantisation of smoothed barycenters to point counts (section 4, the
 * paragraph after Algorithm 2: quantisation is the paper's other pointer to
 * spikier barycenters; reading: each cell's mass, in point units, rounded to
 * the nearest integer, halves upwards).  q may alias z; the result is a
 * histogram of integer counts (a diagram on the grid) that the other calls
 * take as any histogram.
 *   z (device) float32 [n, d, d]
 *   q (device) float32 [n, d, d] out: floor(z + 1/2), exact
 * n = 0 is a no-op. */
int pd_quantize(pdsink_ctx* ctx, int64_t n, const float* z, float* q, void* stream);

/* k-means assignment step (section 5): the distance of diagram n to centroid
 * c is the Algorithm 1 cost of (hist[n] + R z_c, z_c + R hist[n]); assign[n]
 * is the index of the smallest distance, ties to the lowest index.
 *   hist      (device) float32 [n_diag, d, d]
 *   centroids (device) float32 [k, d, d]
 *   assign    (device) int32   [n_diag]      out
 *   dist      (device) double  [n_diag, k]   out, may be NULL
 *   status    (device) int32   [n_diag, k]   out, may be NULL
 *   ws, ws_bytes (device) at least pdsink_workspace_bytes(KMEANS, n_diag * k) */
int kmeans_assign(pdsink_ctx* ctx, int64_t n_diag, const float* hist,
                  int32_t k, const float* centroids,
                  int32_t* assign, double* dist, int32_t* status,
                  void* ws, size_t ws_bytes, void* stream);

/* k-means (section 5) by Lloyd rounds.  Each round assigns every diagram to
 * its nearest centroid (as kmeans_assign) and then replaces each centroid that
 * has members by the Algorithm 2 barycenter of its members, started from the
 * uniform measure (as pd_barycenter with init_uniform); a centroid without
 * members is kept.
 *   hist      (device) float32 [n_diag, d, d]
 *   init      (host)   int32   [k]  indices of the initial centroids, distinct, in [0, n_diag)
 *   centroids (device) float32 [k, d, d]  out: centroids after the last round
 *   assign    (device) int32   [n_diag]   out: the last round's assignment
 *   objective (host)   double  [rounds]   out, may be NULL: per round, the sum over
 *             the diagrams of the distance to the assigned centroid
 *   ws, ws_bytes (device) at least pdsink_lloyd_workspace_bytes(n_diag, k)
 * Synchronises `stream` once per round (its assignment) and once per
 * barycenter.
 * PDSINK_ERANGE if a distance or barycenter step is not finite. */
int pdsink_lloyd_workspace_bytes(const pdsink_ctx* ctx, int64_t n_diag, int32_t k, size_t* bytes);
int kmeans_lloyd(pdsink_ctx* ctx, int64_t n_diag, const float* hist, int32_t k, const int32_t* init,
                 int32_t rounds, double lambda, int32_t max_outer, double energy_rtol,
                 float* centroids, int32_t* assign, double* objective,
                 void* ws, size_t ws_bytes, void* stream);

/* Phase cycle counters of the resident-kernel distance path, for performance
 * work.  Only a library built with PDSINK_PROFILE=1 (python -m
 * paper_1805_08331_amd.build --profile, libpdsink_prof.so) records them; the
 * plain library returns PDSINK_EINVAL.  Copies PDSINK_NPHASE counters summed
 * over every pair that path solved on the current device since the last
 * reset into out (host), in the order: cycles of setup, scale normalisers,
 * BF16 kernel builds, contraction 1, contraction 2, first update pass,
 * suspects, refits, final update pass, cost; then the numbers of half steps,
 * refits, kernel builds, normaliser computations, half steps with suspects
 * and pairs.  Cycles are those of the shader clock counter between workgroup
 * barriers, as seen by the first wave.  reset != 0 clears the counters.
 * Synchronises the device. */
#define PDSINK_NPHASE 16
int pdsink_phase_profile(uint64_t* out, int reset);

/* Static string for a PDSINK_* return code. */
const char* pdsink_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* PDSINK_H */
