/*
 * shot.h -- C ABI of libshot: heat-kernel Sinkhorn on the sphere S^2 on AMD
 * Instinct MI355X (gfx950).
 *
 * Method (arXiv 2605.18389, "Spherical Harmonic Optimal Transport"):
 *   HeatConv(v) = F^{-1}( h (.) F(v) ), h_l = exp(-t l(l+1)), l < L      (Sec. 3.2)
 *   F = semi-naive SHT: FFT along latitude rows, then per-order Legendre
 *       projection with quadrature weights                              (App. C.1)
 *   Sinkhorn scaling loop, balanced and unbalanced, potentials and cost (Alg. 1, App. C.2)
 *   Sinkhorn divergence S = OT(p,q) - (OT(p,p)+OT(q,q))/2 + eps/2 (m(p)-m(q))^2  (Def. 2.3)
 *   its gradient with respect to the input measure                      (Sec. 4.2.2)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grids.  Iso-latitude grids of nlat rows x nlon columns.  Row 0 is the
 *   northernmost row (colatitude closest to 0), column k sits at longitude
 *   2*pi*k/nlon.  The band limit L keeps degrees and orders l, m < L and needs
 *   nlon >= 2L-1; nlat and nlon are at least 2 (SHOT_E_INVALID otherwise).
 *   nlon must be at most 2048 (any factorisation: prime factors
 *   above 5 run as direct stages, slower than radices 2 to 5), and
 *   (2*ceil(nlat/2) + L) complex values of the field precision must fit in
 *   60 KiB (SHOT_E_UNSUPPORTED otherwise).  Area weights a_{jk} = w_j * 2*pi/nlon
 *   sum to 4*pi.
 * Items.  A call processes nitems independent items; item i lives on grid
 *   grid_of_item[i] (an index into the plan's grids).  nitems (npairs) must be
 *   at least 1: an empty batch returns SHOT_E_INVALID before any launch.  Field arrays hold the
 *   items back to back, item i starting at element sum_{i'<i} nlat*nlon of
 *   grid_of_item[i'], each item row-major [nlat][nlon].
 * Precision.  SHOT_FP64 plans take and return double fields and compute in
 *   float64.  SHOT_FP32, SHOT_BF16_MFMA and SHOT_BF16X3_MFMA plans take and
 *   return float fields; FFTs and pointwise updates run in float32, the
 *   Legendre stage in float32 (SHOT_FP32), in bfloat16 operands on matrix cores
 *   with float32 accumulation (SHOT_BF16_MFMA), or in split bfloat16 operands
 *   (SHOT_BF16X3_MFMA: each operand is the sum of two bfloat16 numbers, hi and
 *   lo, and a product is formed as hi*hi + hi*lo + lo*hi on matrix cores,
 *   about 2^-16 relative error per product against 2^-8 for plain bfloat16;
 *   recurrence Legendre mode only).  With SHOT_LEG_RECURRENCE the bfloat16
 *   forms generate P_l^m in float64 and round it to the operand form inside
 *   the kernel; the separate SHT entry points (shot_sht_analysis/synthesis) of
 *   such plans compute in float32.  Quadrature, Legendre recurrence
 *   coefficients and every final reduction (cost, divergence, norms) are
 *   float64 in all plans.
 * Memory.  Pointers documented "device" must be device memory of the GPU
 *   that was current when the plan was made; "host" pointers are ordinary
 *   host memory.  The caller owns every argument buffer; the plan owns its
 *   tables and its workspace.  Calls on one plan must be serialised (they share
 *   the workspace).  `stream` is a hipStream_t (NULL = default stream); work is
 *   enqueued on it, and entry points that return host results synchronise it.
 * Errors.  Every entry point validates its arguments before any launch and
 *   returns SHOT_E_INVALID (nothing launched) on a bad argument, SHOT_E_NOMEM
 *   when device memory cannot be obtained, SHOT_E_HIP on a HIP runtime error.
 *   Solver entry points return the worst per-item status.  Nothing is clamped
 *   silently: a non-positive or non-finite heat-kernel output is reported as
 *   SHOT_E_BREAKDOWN with the first iteration at which it happened (App. C.4).
 */
#ifndef SHOT_H
#define SHOT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct shot_plan_s* shot_plan_t;

typedef enum {
  SHOT_OK = 0,
  SHOT_E_INVALID = 1,
  SHOT_E_NOMEM = 2,
  SHOT_E_HIP = 3,
  SHOT_E_UNSUPPORTED = 4,
  SHOT_W_NOT_CONVERGED = 16, /* tol > 0 and e_marg >= tol after max_iter iterations */
  SHOT_E_BREAKDOWN = 17      /* heat-kernel output <= 0 or non-finite (App. C.4)   */
} shot_status;

enum { SHOT_GRID_GAUSS_LEGENDRE = 0, SHOT_GRID_CLENSHAW_CURTIS = 1, SHOT_GRID_HEALPIX = 2, SHOT_GRID_LOBATTO = 3 };
enum { SHOT_FP64 = 0, SHOT_FP32 = 1, SHOT_BF16_MFMA = 2, SHOT_BF16X3_MFMA = 3 };
enum { SHOT_LEG_AUTO = 0, SHOT_LEG_TABLE = 1, SHOT_LEG_RECURRENCE = 2 };

/* One grid.  kind: SHOT_GRID_GAUSS_LEGENDRE (rows at the roots of P_nlat),
 * SHOT_GRID_CLENSHAW_CURTIS (equiangular rows theta_j = j*pi/(nlat-1), poles
 * included) or SHOT_GRID_LOBATTO (rows at the poles and at the zeros of
 * P'_{nlat-1}, Gauss-Lobatto weights, exact to degree 2 nlat - 3) -- App. C.1:
 * a field is [nlat][nlon] row-major, requires nlon >= 2L-1, nlon <= 2048.
 *
 * SHOT_GRID_HEALPIX (Sec. 3.3, App. C.1; Gorski et al. 2005): nlat = 4 Nside - 1
 * iso-latitude rings, nlon = 4 Nside (the longest ring), Nside <= 512; a field
 * holds the 12 Nside^2 equal-area pixels in RING order (rings from the north,
 * pixels of a ring by increasing longitude from that ring's first pixel, see
 * shot_plan_ring).  No sampling theorem holds, so the transform is
 * pseudo-spectral: the analysis is the area-weighted pixel sum (every pixel
 * has area 4 pi / Npix) and any band limit L >= 1 is accepted. */
typedef struct {
  int32_t kind;
  int32_t nlat;
  int32_t nlon;
  int32_t L;
} shot_grid_desc;

/* Alg. 1 inputs other than the marginals (its REQUIRE list).  The heat time is
 * t = eps/4 (Alg. 1, first step). */
typedef struct {
  double eps;          /* entropic parameter, > 0                                  */
  double tau;          /* marginal penalty, > 0; +INFINITY selects the balanced branch */
  int32_t max_iter;    /* T >= 1                                                   */
  int32_t check_every; /* C >= 1: e_marg is evaluated when k mod C == 0 (App. C.3)  */
  double tol;          /* delta >= 0: stop when e_marg < delta; 0 runs exactly T    */
} shot_params;

/* Per-solve report. */
typedef struct {
  double cost;            /* Alg. 1 return value (float64 reduction)                  */
  double err;             /* e_marg of the returned scalings (App. C.3)               */
  int32_t iters;          /* iterations run                                           */
  int32_t status;         /* shot_status of this item                                 */
  int32_t breakdown_iter; /* first iteration with K. <= 0 or non-finite, 0 if none     */
  int32_t reserved;
  double kratio;          /* min over the iterations' heat applies of min(K.)/max(K.),
                             -inf once an output was non-finite: how close the run came
                             to the positivity breakdown of App. C.4                  */
} shot_solve_info;

/* Build a plan for `ngrids` grids (host array).  Computes the float64
 * quadrature (App. C.1), the FFT factorisations and, for SHOT_LEG_TABLE, the
 * table of orthonormal P_l^m(x_j) on the northern rows (App. B normalisation
 * N_lm), stored in the plan's Legendre precision; SHOT_LEG_RECURRENCE instead
 * keeps O(L^2 + L*nlat) recurrence coefficients and seeds and generates
 * P_l^m in float64 inside the kernels (the O(n) memory claim of Sec. 3.2).
 * SHOT_LEG_AUTO picks per grid.  `precision` is SHOT_FP64, SHOT_FP32 or
 * SHOT_BF16_MFMA.  On success *out holds the plan; on failure *out is NULL. */
shot_status shot_sht_plan(shot_plan_t* out, const shot_grid_desc* grids, int32_t ngrids,
                          int32_t precision, int32_t legendre_mode, void* stream);

/* Free a plan and everything it owns.  NULL is accepted. */
shot_status shot_plan_destroy(shot_plan_t plan);

/* Copy grid `grid`'s float64 nodes x_j = cos(colatitude_j) and latitude
 * weights w_j (sum 2) into host arrays of nlat entries each (either may be NULL). */
shot_status shot_plan_grid(shot_plan_t plan, int32_t grid, double* x_out, double* w_out);

/* Ring layout of grid `grid`: for each of its nlat rows (HEALPix: rings), the
 * number of points and the longitude of the first point (point k of the row
 * sits at phi0 + 2 pi k / npix).  Host arrays of nlat entries (either may be
 * NULL).  Latitude-longitude grids report nlon and 0 for every row. */
shot_status shot_plan_ring(shot_plan_t plan, int32_t grid, int32_t* npix_out, double* phi0_out);

/* Area weights of grid `grid` in field order (App. C.2: the discrete measure
 * of point (j, k) of a latitude-longitude grid is a_{jk} = w_j * 2 pi / nlon;
 * every HEALPix pixel has the area 4 pi / Npix).  a_out: host, one float64 per
 * point of a field (nlat * nlon, or 12 Nside^2).  They sum to 4 pi. */
shot_status shot_plan_area_weights(shot_plan_t plan, int32_t grid, double* a_out);

/* Forward SHT (App. B: f_lm = <f, Y_lm>, evaluated by App. C.1's semi-naive
 * algorithm).  f: device, fields of the items.  coeffs: device, per item
 * L(L+1)/2 complex values (real, imag interleaved, field precision), ordered by
 * m then l: f_lm for m = 0..L-1, l = m..L-1, at index m*L - m(m-1)/2 + (l-m).
 * Items are packed back to back in that layout. */
shot_status shot_sht_analysis(shot_plan_t plan, const int32_t* grid_of_item, int32_t nitems,
                              const void* f, void* coeffs, void* stream);

/* Inverse SHT of coefficients in shot_sht_analysis's layout (orders m >= 0;
 * negative orders follow from the field being real). coeffs, f: device. */
shot_status shot_sht_synthesis(shot_plan_t plan, const int32_t* grid_of_item, int32_t nitems,
                                const void* coeffs, void* f, void* stream);

/* HeatConv (Sec. 3.2): out_i = F^{-1}(h (.) F(v_i)) with h_l = exp(-t[i] l(l+1)).
 * t: host, nitems heat times >= 0.  v, out: device fields (may not alias).
 * transpose != 0 applies the transpose of that linear map instead,
 * out = a (.) HeatConv(v / a), used by adjoints. */
shot_status shot_heat_apply(shot_plan_t plan, const int32_t* grid_of_item, int32_t nitems,
                            const double* t, const void* v, void* out, int32_t transpose,
                            void* stream);

/* shot_heat_apply for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, result and kernels as shot_heat_apply, but the per-call
 * workspace (item descriptors, folded spectra, heat multipliers) lives in a
 * fixed device array of SHOT_NOALLOC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends; the call allocates no device
 * memory.  Needs a plan made on the current device (plan creation fetches the
 * array's address).  A call whose workspace exceeds the array (about 4.2 MB per
 * float32 item at 721 x 1440, 2 x L x ceil(nlat/2) complex values per item in
 * general) returns SHOT_E_INVALID before any launch, with the sizes in
 * shot_last_error().  Every call on one GPU shares that GPU's array, so calls
 * that overlap on one GPU (other streams or threads, any plan) race; serialise
 * them. */
#define SHOT_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
shot_status shot_heat_apply_noalloc(shot_plan_t plan, const int32_t* grid_of_item, int32_t nitems,
                                    const double* t, const void* v, void* out, int32_t transpose,
                                    void* stream);

/* Alg. 1 on nitems independent items.  params: host, one per item.  p, q:
 * device marginals (densities with respect to the area weights, positive).
 * An item whose marginals do not both have positive, finite area-weighted mass
 * m = sum a p gets status SHOT_E_INVALID (found from the masses the solve
 * computes, so after its launches; shot_last_error() names the item), and the
 * call then returns SHOT_E_INVALID; this applies to the divergence and
 * gradient entry points as well.  Otherwise the call returns the largest
 * per-item status.
 * phi, psi: device outputs, eps*log(u) and eps*log(v) (either may be NULL).
 * info: host, nitems reports.  Synchronises `stream`. */
shot_status shot_sinkhorn_solve(shot_plan_t plan, const int32_t* grid_of_item, int32_t nitems,
                                const shot_params* params, const void* p, const void* q,
                                void* phi, void* psi, shot_solve_info* info, void* stream);

/* Sinkhorn divergence (Def. 2.3) of npairs pairs: three Alg. 1 solves per pair,
 * (p,q), (p,p) and (q,q), advanced together, combined in float64 as
 * S = R(p,q) - (R(p,p)+R(q,q))/2 + eps/2 (m(p)-m(q))^2, m(p) = sum a p.
 * params: host, one per pair.  S_out: host, npairs.  info: host, 3*npairs
 * reports in the order (p,q),(p,p),(q,q) per pair, or NULL.  Synchronises. */
shot_status shot_sinkhorn_divergence(shot_plan_t plan, const int32_t* grid_of_pair, int32_t npairs,
                                     const shot_params* params, const void* p, const void* q,
                                     double* S_out, shot_solve_info* info, void* stream);

/* Divergence and its gradient with respect to the density array p (Sec. 4.2.2),
 * with tol = 0; the pairs of one call are all balanced (tau = +INFINITY) or all
 * unbalanced (SHOT_E_UNSUPPORTED otherwise).
 * mode 0: exact reverse-mode derivative of the T-iteration computation
 *         (hand-written adjoint of Alg. 1, both branches, and of HeatConv).  The
 *         reverse sweep reads the forward iterates of `checkpoint_every`
 *         iterations at a time, recomputed from checkpoints of v.  With 0 the
 *         library keeps the whole history in one segment (one forward pass, no
 *         recomputation) when 2 T fields per (p,q) and (p,p) solve take at most
 *         half the free device memory and 64 GiB, else checkpoints every
 *         ceil(sqrt(T)) iterations.  The workspace stays with the plan.
 * mode 1: envelope gradient from the potentials (balanced pairs only),
 *         a (.) (phi_pq - (phi_pp + psi_pp)/2) + eps (m(p)-m(q)) a.
 * dS_dp: device, layout of p.  Other arguments as shot_sinkhorn_divergence. */
shot_status shot_sinkhorn_divergence_grad(shot_plan_t plan, const int32_t* grid_of_pair,
                                          int32_t npairs, const shot_params* params,
                                          const void* p, const void* q, double* S_out,
                                          void* dS_dp, int32_t mode, int32_t checkpoint_every,
                                          shot_solve_info* info, void* stream);

/* Regional attribution of a gradient (Sec. 4.2.2, "Gradient-based regional
 * attribution"): for each pair, g = dS_dp / a (a: point areas) is centred by
 * its area-weighted mean over the sphere, and its area-weighted RMS over each
 * latitude band is returned.  dS_dp: device, the layout of
 * shot_sinkhorn_divergence_grad's output for these pairs.  bands: host,
 * nbands (lat_lo, lat_hi) pairs in degrees; a row (ring) belongs to a band
 * when lat_lo < its latitude < lat_hi (rows on an edge are excluded; a
 * latitude within 1e-9 degree of a bound counts as on it, so that rounding of
 * the arcsine cannot move a row across a bound).
 * rms_out: host, npairs * nbands (NaN for a band holding no row).  The
 * per-row sums run on the device in float64, the band combination on the
 * host.  Synchronises `stream`. */
shot_status shot_gradient_regional_rms(shot_plan_t plan, const int32_t* grid_of_pair, int32_t npairs,
                                       const void* dS_dp, const double* bands, int32_t nbands,
                                       double* rms_out, void* stream);

/* Launch configuration of grid `grid`'s Legendre kernel: items advanced per
 * workgroup of the VALU kernels (1, 2, 4 or 8; 0 = automatic, capped by LDS;
 * for SHOT_LEG_RECURRENCE grids of float plans 8 or 16 select the
 * recurrence-fed matrix-core kernel with that many items per workgroup, which
 * bfloat16 plans always use) and, as the second value, for SHOT_LEG_RECURRENCE grids the latitude chains
 * per thread of the latitude-split kernel (1, 2 or 4, at most 256 threads per
 * workgroup; 0 = the row-split kernel), for SHOT_LEG_TABLE grids of float32 and
 * bfloat16 plans the matrix-core kernel's column tiles per workgroup (1, 2 or 4
 * tiles of 16 columns = 8, 16 or 32 items; 0 = automatic: matrix cores for any
 * number of items, 1 tile below 16 items, 2 from 16, 4 from 32, fewer while
 * they overflow 60 KiB of LDS; -1 = VALU kernel only; a table whose single
 * tile would need more than 150 KiB of LDS runs the VALU kernel).
 * SHOT_E_INVALID otherwise. */
shot_status shot_plan_set_tuning(shot_plan_t plan, int32_t grid, int32_t items_per_block,
                                 int32_t chains_per_thread);
shot_status shot_plan_get_tuning(shot_plan_t plan, int32_t grid, int32_t* items_per_block,
                                 int32_t* chains_per_thread);

/* Autotuner: times every valid launch configuration of grid `grid`'s fused
 * Legendre kernel for a batch of `nitems` items (synthetic spectrum, HIP
 * events on `stream`) and keeps the fastest on the plan.  Synchronises. */
shot_status shot_autotune(shot_plan_t plan, int32_t grid, int32_t nitems, void* stream);

/* Fixed-T solves (tol = 0) record their iteration loop once as a HIP graph
 * per plan and call layout and replay it on later calls with the same layout
 * (the per-call inputs live in device memory).  enable = 0 launches every
 * kernel eagerly instead.  Default: enabled. */
shot_status shot_plan_set_graphs(shot_plan_t plan, int32_t enable);

/* Kernel timing.  When enabled, every launch of the Legendre kernels (class 0)
 * and of the row-FFT kernels (class 1) is bracketed by HIP events on the
 * launch stream; shot_profile_read synchronises and returns the number of
 * timed launches and their summed duration in milliseconds for one class.
 * shot_profile_enable(plan, 0) stops timing; enabling again resets the counts.
 * While timing is enabled, solves launch eagerly (no graph replay). */
shot_status shot_profile_enable(shot_plan_t plan, int32_t enable);
shot_status shot_profile_read(shot_plan_t plan, int32_t kernel_class, int64_t* launches,
                              double* total_ms);

/* Identifier of the sources this library was built from (a hash the build
 * script computes over the C, HIP and header files and the compile flags;
 * static storage).  Loaders compare it with the sources next to the library
 * so that a stale build is refused instead of being run. */
const char* shot_build_id(void);

/* Human-readable name of a status code (static storage). */
const char* shot_status_string(int32_t status);

/* Description of the most recent HIP runtime failure seen by libshot on the
 * calling thread (the call, its source line and the HIP error string), or ""
 * if none.  Valid until the next libshot call on this thread. */
const char* shot_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SHOT_H */
