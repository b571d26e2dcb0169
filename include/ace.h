/*
 * ace.h — C-ABI of the MI355X (gfx950) adaptively compressed exchange build.
 *
 * The calls follow the statement of the problem in arXiv 2110.07670,
 * section "HF Exchange Operator" (Eq. (1)-(4)) and section "ACE Operator":
 *
 *   ace_build  : W = alpha V_X Phi (Eq. (2)), one periodic Poisson solve per
 *                orbital pair (Eq. (3), evaluated in reciprocal space),
 *                M = dV Phi^T W, -M = L L^T, projectors xi = W L^{-T} (the
 *                paper's P_k), and E_x = tr(M) = alpha E_X^HF (Eq. (4)).
 *   ace_apply  : V_ACE psi = -xi (dV xi^T psi)  (the ACE application formula).
 *   exx_energy : E_x from forward transforms only (Parseval form of Eq. (4)),
 *                optionally the energy of every pair.
 *
 * Conventions (the paper leaves them open; these are the library's readings):
 *   - Gamma point, real orbitals phi_i sampled on an n1 x n2 x n3 grid of an
 *     orthorhombic cell with edges L1, L2, L3 (bohr); Omega = L1 L2 L3,
 *     N = n1 n2 n3, dV = Omega / N, <f, g> = dV sum_r f(r) g(r).
 *   - Coulomb kernel K(G) = 4 pi / |G|^2 with K(0) = 0, G = 2 pi m_a / L_a,
 *     m in numpy FFT order (the Nyquist plane is kept); unnormalised forward
 *     transform, 1/N on the inverse.
 *   - W_i = -alpha sum_j v_ij phi_j includes alpha and the minus sign; every
 *     unordered pair i <= j is solved once (v_ij = v_ji) and updates both
 *     W_i and W_j.  Closed shell: no factor 1/2 in E_x.
 *   - L is lower triangular with a positive diagonal; a non-positive leading
 *     minor of -M is reported through *info (LAPACK style); xi is then left
 *     untouched.
 *
 * Layout: phi, W, xi, psi, out are orbital-major [k][n1][n2][n3] float64 in C
 * order (z fastest, each orbital contiguous).  M is [n_orb][n_orb] row-major.
 * ex and info are single device values.  pair_mask and pair_e are described
 * at their calls.
 *
 * Ownership: every array is caller-owned device memory, except pair_mask
 * (host memory).  The library never allocates device memory (a batch owns
 * its streams, events and a pinned host table copy) and never frees caller
 * memory; each call copies its small tables (twiddles, pair schedule)
 * into the caller's workspace, stream-ordered.  A plan is immutable host data
 * and may be shared by several streams if each stream has its own workspace.
 * Calls that overlap on one workspace race.
 *
 * Errors: every argument is validated on the host before any device work; the
 * return value is an ace_status.  Calls are asynchronous on `stream` (a
 * hipStream_t; NULL is the default stream): read ex / info after
 * synchronising the stream.
 */
#ifndef ACE_H_
#define ACE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ace_plan ace_plan;

enum ace_precision {
  ACE_FP64 = 0, /* all stages in FP64 */
  ACE_FP32 = 1  /* pair densities, transforms and Coulomb multiply in FP32
                   (from an FP32 copy of phi, which the W update also reads);
                   the W products and sums, M, Cholesky, xi and E_x in FP64 */
};

enum ace_status {
  ACE_OK = 0,
  ACE_ERR_ARG = 1,       /* null pointer, bad count or cell, aliasing outputs */
  ACE_ERR_SIZE = 2,      /* grid not supported (see ace_plan_create) or n_orb too large */
  ACE_ERR_WORKSPACE = 3, /* workspace smaller than the call needs */
  ACE_ERR_HIP = 4,       /* a HIP launch or runtime call failed: see ace_last_hip_error() */
  ACE_ERR_NODEV = 5      /* no HIP device is visible */
};

typedef struct {
  int n[3];        /* grid points per axis; currently n1 = n2 = n3 and n in
                      {16,24,32,40,48,64,80,96,120,128,144,160,192} (factors 2, 3, 5) */
  double cell[3];  /* orthorhombic edge lengths L1, L2, L3 in bohr, > 0 */
  int n_orb;       /* occupied orbitals, 1 .. 512 */
  int precision;   /* enum ace_precision */
  double alpha;    /* exact-exchange fraction (0.25 for PBE0) */
} ace_desc;

/* Create a host-only plan for one grid / cell / orbital count.  Touches no
 * device.  Returns ACE_ERR_ARG for a null pointer, n_orb < 1, a non-positive
 * or non-finite cell edge, an unknown precision or a non-finite alpha;
 * ACE_ERR_SIZE for a grid outside the supported set or n_orb > 512.  On
 * success *plan owns host memory released by ace_plan_destroy. */
int ace_plan_create(ace_plan **plan, const ace_desc *desc);
void ace_plan_destroy(ace_plan *plan);

/* Device workspace bytes that ace_build and exx_energy need (0 on a null plan). */
size_t ace_workspace_bytes(const ace_plan *plan);
/* Device workspace bytes that ace_apply needs for n_vec vectors. */
size_t ace_apply_workspace_bytes(const ace_plan *plan, int n_vec);

/* The ACE build (see the file comment).
 *   phi       [n_orb][N] input orbitals, orthonormal under dV (not checked)
 *   pair_mask host [n_orb][n_orb] uint8 or NULL; only the upper triangle
 *             (i <= j) is read; a zero entry skips pair (i, j) for both W_i
 *             and W_j (the s-MTACE screening of the paper); NULL = all pairs
 *   W         [n_orb][N] output, alpha V_X phi
 *   M         [n_orb][n_orb] output, dV Phi^T W
 *   xi        [n_orb][N] output projectors; untouched when *info != 0
 *   ex        device double: tr(M)
 *   info      device int: 0, or k when the k-th leading minor of -M is not
 *             positive
 * phi, W and xi must not overlap. */
int ace_build(const ace_plan *plan, void *stream, void *ws, size_t ws_bytes, const double *phi,
              const uint8_t *pair_mask, double *W, double *M, double *xi, double *ex, int *info);

/* out[v] = -sum_k xi_k <xi_k, psi_v>, v < n_vec.  xi [n_orb][N] from ace_build,
 * psi and out [n_vec][N]; out must not overlap xi or psi. */
int ace_apply(const ace_plan *plan, void *stream, void *ws, size_t ws_bytes, const double *xi,
              const double *psi, int n_vec, double *out);

/* ace_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same result as ace_apply (up to rounding: the split-K products may be
 * split into fewer partials) with no workspace argument.  Its scratch, the
 * n_vec x n_orb coefficients and their split-K partial products, lives in a
 * static device array of ACE_NOALLOC_SCRATCH_BYTES that the library holds on
 * every device it runs on until the process ends; the call itself allocates
 * nothing (no hipMalloc, no allocating library routine).  Returns
 * ACE_ERR_SIZE (before any device work) when the coefficients and one
 * partial product, 8 n_vec n_orb bytes each (the first rounded up to a
 * multiple of 256), exceed that size, and the argument errors of ace_apply.  Every call on one device shares that device's array and leaves
 * its contents behind: calls that overlap in time on one device (different
 * streams or threads) race and must be serialised by the caller. */
#define ACE_NOALLOC_SCRATCH_BYTES (32u << 20)
int ace_apply_noalloc(const ace_plan *plan, void *stream, const double *xi, const double *psi,
                      int n_vec, double *out);

/* E_x = -alpha sum_{i<=j} (2 - delta_ij) (ij|ji) with
 * (ij|ji) = (Omega / N^2) sum_m K(m) |FFT(phi_i phi_j)(m)|^2.
 *   pair_mask as in ace_build.
 *   ex      device double output.
 *   pair_e  NULL, or device [n_orb][n_orb] double: entry (i, j), i <= j, gets
 *           that pair's share -alpha (2 - delta_ij) (ij|ji); other entries are
 *           left untouched.  Requesting pair_e solves one pair per transform
 *           instead of two. */
int exx_energy(const ace_plan *plan, void *stream, void *ws, size_t ws_bytes, const double *phi,
               const uint8_t *pair_mask, double *ex, double *pair_e);

/* Pair screening (section "s-MTACE Method": pairs whose orbitals barely
 * overlap are left out of the exchange build).  The outputs feed pair_mask.
 *
 * ace_overlap_integrals: S[i][j] = dV sum_r |phi_i(r)| |phi_j(r)|, the
 *   paper's screening integral, for all i, j ([n_orb][n_orb] device double);
 *   keeping pair (i, j) when S[i][j] >= rho_cut is the s-MTACE screen.
 *   Needs the ace_build workspace.
 * ace_wannier: Berry-phase moments of each orbital density,
 *   z[i][2a], z[i][2a+1] = Re, Im of dV sum_r phi_i(r)^2 exp(2 pi i r_a / L_a)
 *   ([n_orb][6] device double), and features feat[i] = (centre_x, centre_y,
 *   centre_z, spread) ([n_orb][4] device double) with
 *   centre_a = L_a/(2 pi) arg z_a in [0, L_a) and
 *   spread^2 = sum_a (L_a/(2 pi))^2 (-ln |z_a|^2).
 * ace_mlp_screen: for i <= j, pred[i][j] = MLP(d_ij, min(s_i, s_j),
 *   max(s_i, s_j)) ([n_orb][n_orb] device float; entries j < i untouched),
 *   d_ij the minimum-image distance of the centres; a 3-64-64-1 ReLU network
 *   in FP32 predicting log10 |e_ij| of the pair energy.  weights: device
 *   float[ace_mlp_weight_count()] laid out as mean[3] std[3] W1[64][3] b1[64]
 *   W2[64][64] b2[64] w3[64] b3 (inputs standardised by mean and std). */
int ace_overlap_integrals(const ace_plan *plan, void *stream, void *ws, size_t ws_bytes,
                          const double *phi, double *S);
int ace_wannier(const ace_plan *plan, void *stream, const double *phi, double *z, double *feat);
int ace_mlp_screen(const ace_plan *plan, void *stream, const double *feat, const float *weights,
                   float *pred);
int ace_mlp_weight_count(void);

/* The screening decision (section "s-MTACE Method"): which pairs ace_build
 * skips, from the overlap integrals or from the learned pair-energy
 * predictions, with the all-pairs build as the fallback.
 *
 * ace_screen_desc:
 *   kind        ACE_SCREEN_OVERLAP: keep (i, j) when S_ij >= rho_cut (the
 *               paper's criterion, S as from ace_overlap_integrals);
 *               ACE_SCREEN_MLP: skip the pairs of smallest predicted |e_ij|,
 *               in increasing order, while their predicted sum stays at most
 *               budget / safety (predictions as from ace_mlp_screen, read as
 *               log10 of the expected |e_ij| in Ha).
 *   rho_cut     overlap threshold (ACE_SCREEN_OVERLAP).
 *   budget      Ha: the largest exchange energy the skipped pairs may carry.
 *   safety      >= 1; the MLP screen keeps the predicted skipped energy at
 *               most budget / safety.
 *   mlp_weights device float[ace_mlp_weight_count()] or NULL.  Required for
 *               ACE_SCREEN_MLP; with ACE_SCREEN_OVERLAP, when given, the
 *               predicted energy of the skipped pairs is reported and checked
 *               against the budget.
 * ace_screen_report: kept and total unordered pairs, the predicted energy of
 *   the skipped pairs (Ha; NaN without weights) and fallback = 1 when that
 *   prediction exceeds the budget, in which case the mask keeps every pair.
 * Diagonal pairs are always kept.  The mask is host [n_orb][n_orb] uint8,
 * upper triangle written (i <= j), the rest zero, ready for ace_build.
 *
 * ace_screen_mask: computes the inputs on the device (in the ace_build
 *   workspace), copies them to the host and decides; it synchronises
 *   `stream`.
 * ace_screen_mask_host: the decision alone from host arrays S ([n][n]
 *   double, or NULL for ACE_SCREEN_MLP) and pred ([n][n] float, upper
 *   triangle read; NULL when no predictions are available).  Touches no
 *   device.  ACE_ERR_ARG for a null mask, report or desc, n < 1, an unknown
 *   kind, a missing input for the kind, budget < 0 or safety < 1. */
#define ACE_SCREEN_OVERLAP 0
#define ACE_SCREEN_MLP 1
typedef struct {
  int kind;
  double rho_cut;
  double budget;
  double safety;
  const float *mlp_weights;
} ace_screen_desc;
typedef struct {
  int64_t pairs_kept;
  int64_t pairs_total;
  double predicted_skipped;
  int fallback;
} ace_screen_report;
int ace_screen_mask(const ace_plan *plan, void *stream, void *ws, size_t ws_bytes,
                    const double *phi, const ace_screen_desc *desc, uint8_t *mask,
                    ace_screen_report *report);
int ace_screen_mask_host(int n_orb, const ace_screen_desc *desc, const double *S,
                         const float *pred, uint8_t *mask, ace_screen_report *report);

/* Static text for a status code. */
const char *ace_error_string(int code);
/* The hipError_t behind the calling thread's last ACE_ERR_HIP (0 if none). */
int ace_last_hip_error(void);

/* Stage timing.  With profiling on, the calls above record a pair of HIP
 * events around every launch on their stream; ace_profile_read waits for
 * them, returns per-stage totals in milliseconds and launch counts, and
 * clears the record.  Stages: 0 yz-forward, 1 x-Poisson, 2 yz-inverse,
 * 3 W-accumulate, 4 M product, 5 Cholesky + inverse, 6 xi product,
 * 7 small kernels and table copies, 8 apply products, 9 x-energy.
 * out_ms and out_count must hold ACE_N_STAGES entries. */
#define ACE_N_STAGES 10
int ace_set_profiling(ace_plan *plan, int on);
int ace_profile_read(ace_plan *plan, double *out_ms, int *out_count);

/* Launch-shape knobs, for the tuner: orbital block of the pair tiles
 * (8 or 16; a new plan takes 16, or 8 where only block 8 has the three-pass
 * schedule: FP64 120^3 and 128^3), the packed transforms per forward/inverse
 * launch (0 = a whole tile) and the x-pass pencils per workgroup (8, 16 or
 * 32 dividing n; 0 = the default).  chunk and pencils change no result bit; block changes
 * which pairs share a transform and the order of the W sums, so results move
 * by rounding only.  block changes ace_workspace_bytes (the scratch holds
 * one tile's transforms: block^2 / 2 complex grids).
 * ACE_ERR_ARG for a value outside these sets. */
int ace_plan_set_tiling(ace_plan *plan, int block, int chunk, int pencils);
/* The plan's current launch shape (any pointer may be NULL). */
int ace_plan_tiling(const ace_plan *plan, int *block, int *chunk, int *pencils);

/* Transform schedule.  ACE_SCHEDULE_AUTO: full pair tiles (block x block
 * orbitals, every pair kept; block 8 or 16) take three passes over the
 * scratch grids where the grid's plane fits a workgroup's LDS (FP64 n <= 96,
 * FP32 n <= 128; from 48^3 up the forward pass takes each plane two slabs
 * at a time so that several workgroups share a compute unit), or where a
 * workgroup can take a plane slab by slab (FP64 120^3 and 128^3, block 8),
 * and four elsewhere; in all of these the
 * inverse z transform feeds the W update directly.  Every other tile takes
 * four passes with the W update a pass of its own.
 * ACE_SCHEDULE_FOUR_PASS: four passes everywhere.  Both give the same result
 * up to rounding (the order of the W sums differs). */
#define ACE_SCHEDULE_AUTO 0
#define ACE_SCHEDULE_FOUR_PASS 1
int ace_plan_set_schedule(ace_plan *plan, int schedule);
/* The passes the plan's current shape and schedule give (host-side, for
 * byte accounting): *full_tiles is ACE_TILES_THREE_PASS (forward, middle,
 * inverse z with W), ACE_TILES_ROWS_FUSED (forward, x, inverse y, inverse z
 * rows with W) or ACE_TILES_FOUR_PASS (forward, x, inverse y/z, W), the
 * schedule of full tiles; other tiles take four passes.  *plane is 1 where
 * a (y, z) plane fits LDS (a four-pass inverse y/z is one plane pass) and 0
 * where it does not (a four-pass inverse y/z is a line pass plus a row
 * pass); the forward pass moves the same bytes in either case. */
#define ACE_TILES_THREE_PASS 0
#define ACE_TILES_ROWS_FUSED 1
#define ACE_TILES_FOUR_PASS 2
int ace_plan_schedule(const ace_plan *plan, int *full_tiles, int *plane);

/* ---- Batches of independent systems (uneven grids and orbital counts).
 *
 * One ace_build per instance (each with its own plan, launch shapes and
 * optional pair mask), recorded once into a HIP graph; later calls with the
 * same pointers replay the recorded graph.  Instances with the same grid
 * (48, 64, 80 or 96 points per axis), bulk precision and the automatic
 * schedule form a lane: round r of a lane takes tile r of each of its
 * instances, every whole three-pass tile of the round in one persistent
 * launch per pass (workgroups draining a shared work queue of the
 * instances' transform planes and point blocks), the lane's other tiles
 * after them.  Lanes and the remaining instances run concurrently on the
 * graph's branches, largest first, balanced by estimated work.  Every
 * instance's result is bitwise that of a separate ace_build with the same
 * plan and mask (the same arithmetic in the same order per instance).
 *
 * ace_batch_create: plans[count] (1 <= count <= ACE_BATCH_MAX) must outlive
 *   the batch and keep the launch shapes they had at creation (a changed
 *   shape makes ace_batch_build return ACE_ERR_ARG).  pair_masks may be NULL
 *   (all pairs everywhere) or hold count host pointers, each NULL or an
 *   n_orb x n_orb mask as for ace_build; the masks are read here and not kept.
 * ace_batch_workspace_bytes: device bytes of the one workspace the batch
 *   slices into per-instance workspaces (256-byte aligned).
 * ace_batch_build: phi, W, M, xi are host arrays of count device pointers,
 *   laid out as for ace_build; ex[count] and info[count] are device arrays.
 *   Outputs of different instances may not overlap each other or any phi.
 *   The first call on a device creates the batch's streams, events and a
 *   pinned host copy of the tables; the tables are copied into the workspace
 *   on `stream` ahead of the work at every call.  flags: 0 replays (or first
 *   records) the graph, launched on `stream`; ACE_BATCH_EAGER launches the
 *   same work directly on the branch streams, joined back into `stream`;
 *   ACE_BATCH_NO_LANES (with or without EAGER) runs every instance's own
 *   launch sequence on its branch instead of the lanes' shared pass
 *   launches (same results bit for bit; which is faster depends on the
 *   batch, and the batch tuner times both).
 *   A later call on another device returns ACE_ERR_ARG.
 * ace_batch_destroy: only after the batch's last build has completed.
 * ace_batch_lanes: host-side description of the schedule: *lanes lanes,
 *   *batch_tiles tiles in the shared pass launches, *other_tiles tiles on
 *   the single-system kernels (any pointer may be NULL). */
#define ACE_BATCH_MAX 1024
#define ACE_BATCH_EAGER 1
#define ACE_BATCH_NO_LANES 2
typedef struct ace_batch ace_batch;
int ace_batch_create(ace_batch **batch, const ace_plan *const *plans,
                     const uint8_t *const *pair_masks, int count);
void ace_batch_destroy(ace_batch *batch);
size_t ace_batch_workspace_bytes(const ace_batch *batch);
int ace_batch_build(ace_batch *batch, void *stream, void *ws, size_t ws_bytes,
                    const double *const *phi, double *const *W, double *const *M,
                    double *const *xi, double *ex, int *info, int flags);
int ace_batch_lanes(const ace_batch *batch, int *lanes, int64_t *batch_tiles,
                    int64_t *other_tiles);

/* ---- SCDM localisation (section "s-MTACE Method": a rank-revealing QR of
 * Psi^* selects columns of the density matrix Gamma = Psi Psi^*, which are
 * orthonormalised; section "s'-MTACE Method": only grid points with
 * rho > <rho> and |grad rho| < <|grad rho|> enter the QR).
 *
 * Readings (the paper gives no formulas): rho = sum_i phi_i^2; grad rho by
 * second-order central differences on the periodic grid, compared by its
 * Euclidean norm; averages over all grid points; the QR is Householder with
 * Businger-Golub column pivoting (largest residual column norm, the first
 * on a tie); the selected columns are orthonormalised symmetrically
 * (Loewdin): phi_loc = U^T Phi with U the orthogonal polar factor of
 * A_C = Psi^*(:, C), computed by Newton-Schulz iteration.
 *
 * scdm_workspace_bytes: device bytes for scdm_preselect (m = 0) or for
 *   both calls with m kept points.
 * scdm_preselect: points (device int[n1 n2 n3], caller-owned capacity for
 *   every grid point) receives the kept flat C-order point indices in
 *   increasing order, *count (device int) their number.
 * scdm_localize: the k = n_orb pivoted-QR steps over the m points
 *   (points NULL: every grid point, m = n1 n2 n3; otherwise m >= n_orb
 *   device ints); pivots (device int[n_orb]) receives the selected grid
 *   points in selection order; phi_loc (device, laid out like phi, not
 *   overlapping it) the localised orbitals, row j localised at pivots[j];
 *   *info (device int) 0, s + 1 if step s met a zero residual column (the
 *   orbitals are rank deficient on the points), or n_orb + 1 if the polar
 *   iteration did not converge (phi_loc is then not orthonormal).
 * Argument errors as elsewhere (ACE_ERR_ARG for m out of range). */
size_t scdm_workspace_bytes(const ace_plan *plan, int m);
int scdm_preselect(const ace_plan *plan, void *stream, void *ws, size_t ws_bytes,
                   const double *phi, int *points, int *count);
int scdm_localize(const ace_plan *plan, void *stream, void *ws, size_t ws_bytes,
                  const double *phi, const int *points, int m, int *pivots,
                  double *phi_loc, int *info);

#ifdef __cplusplus
}
#endif

#endif /* ACE_H_ */
