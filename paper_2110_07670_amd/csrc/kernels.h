// Internal launch interface between the host runtime and the gfx950 kernels.
// Not part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace acex {

// One packed transform carries two real pairs: rho = phi_a phi_b + i phi_c phi_d.
// c = d = -1 marks a transform carrying a single pair.
struct Pack {
  int a, b, c, d;
};

struct GridArgs {
  int n;              // points per axis (cubic grid)
  int prec;           // 0: FP64 bulk, 1: FP32 bulk
  int64_t npts;       // n^3
  double g2[3];       // (2 pi / L_a)^2 per axis
  double kscale;      // multiplies 4 pi / G^2 (1/N for the Poisson pass, 1 for energy)
  const void* tw;     // n twiddles w_n^k = exp(-2 pi i k / n), bulk precision
  int cus;            // compute units of the device (persistent grids), a multiple of 8
  int pencils = 0;    // x-pass pencils per workgroup: 8, 16, 32 or 0 (default)
};

// Is `pencils` a valid x-pass shape for grid n (0 is always valid)?
bool pencils_ok(int n, int pencils);

// Does one (y, z) plane of the bulk type fit in a workgroup's LDS?
bool plane_fits(int n, int prec);
bool supported_n(int n);

// Forward (y,z) transforms of the pair densities of `npack` packed pairs.
// phi: FP64 orbitals (prec 0) or FP32 copy (prec 1), orbital-major.
// S: npack complex grids of the bulk type, written in position order,
// as S[x][ky][kz], or S[kz][x][ky] with zxy (plane-fitting grids only).
hipError_t launch_fwd_yz(const GridArgs& g, const void* phi, const Pack* packs, int npack,
                         void* S, hipStream_t s, bool zxy = false);

// Three-pass schedule for full tiles (three_pass_ok):
// launch_fwd_yz(zxy) -> launch_mid (forward x, K/N, inverse x, inverse y
// per kz plane, in place) -> launch_zinv_acc (inverse z of the tile's
// transforms, S + 0 .. npack-1 in the canonical row order, folded into W of
// the tile's orbitals orbs[0..2 block)).
bool three_pass_ok(int n, int prec, int block);
// Large-grid schedule for full tiles where a plane does not fit
// (fused_rows_ok): launch_fwd_yz -> launch_poisson_x -> launch_inv_y (the
// inverse y lines only) -> launch_zinv_acc (inverse z rows folded into W).
bool fused_rows_ok(int n, int prec, int block);
hipError_t launch_inv_y(const GridArgs& g, void* S, int npack, hipStream_t s);
hipError_t launch_mid(const GridArgs& g, void* S, int npack, hipStream_t s);
// phi: the orbitals in the bulk precision (FP64, or the FP32 copy).  With
// S2 (and orbs2) one launch also does a second tile of the same kind whose
// orbital blocks are disjoint from the first's.
hipError_t launch_zinv_acc(const GridArgs& g, int block, bool diag, const void* S,
                           const void* phi, double* W, const int* orbs, double alpha,
                           hipStream_t s, const void* S2 = nullptr,
                           const int* orbs2 = nullptr);
// x transforms with the Coulomb multiply between forward and inverse, in place.
hipError_t launch_poisson_x(const GridArgs& g, void* S, int npack, hipStream_t s);
// x forward transform and sum of K |Z|^2 per workgroup into part[npack][parts_per_pack].
hipError_t launch_energy_x(const GridArgs& g, const void* S, int npack, double* part,
                           hipStream_t s);
int energy_parts_per_pack(int n);
// Inverse (y,z) transforms back to real space, natural order, in place.
hipError_t launch_inv_yz(const GridArgs& g, void* S, int npack, hipStream_t s);

// W tile update: W_I -= alpha sum_j v_ij phi_j, W_J -= alpha sum_i v_ij phi_i.
// meta[p] = a0 | b0 << 8 | a1 << 16 | b1 << 24: local positions of the pairs
// in the real / imaginary half of transform p (a1 = 255: single pair);
// meta == nullptr: a full unmasked B x B tile in the canonical a-major order.
// orbs: the tile's 2B orbital indices (I list, then J list); useI / useJ:
// local orbitals with at least one pair.
// phi: the orbitals in the bulk precision (FP64, or the FP32 copy).
hipError_t launch_accumulate(int prec, int block, bool diag, const void* S, const void* phi,
                             double* W, const int* meta, int npack, const int* orbs,
                             unsigned useI, unsigned useJ, double alpha, int64_t npts,
                             hipStream_t s);

// ---- Batches: one persistent launch per pass over the three-pass tiles of
// many systems of one grid size, bulk precision and block.  A launch drains a work
// queue (an atomic counter) of items; segment k covers items item0 ..
// item0 + count - 1 of one system's current tile: forward (pass 0) and
// middle (pass 1) items are (x or kz, transform), N npack of them; fused
// inverse-z/W items (pass 2) are the N N / 8 point blocks.  Each item does
// the work of one workgroup of the single-system kernels, with the same
// arithmetic, so results are bitwise those of the system's own build.
struct BatchSeg {
  const void* phi;      // orbitals in the bulk precision
  const Pack* packs;    // the tile's transforms (pass 0)
  void* S;              // the system's transform scratch
  const void* tw;       // n twiddles, bulk precision
  double* W;            // pass 2
  const int* orbs;      // the tile's 2 block orbital indices (pass 2)
  int64_t npts;
  double g2[3];         // (2 pi / L_a)^2 (pass 1)
  double kscale;        // 1 / N (pass 1)
  double alpha;         // pass 2
  int n, npack, block, diag;
  int item0, count;
};
// Is a three-pass tile of this grid, bulk precision and block run by the
// batch kernels?
bool batch_ok(int n, int prec, int block);
int batch_items(int pass, int n, int npack);
// One launch of pass `pass` over the segments of one grid size n, bulk
// precision and block; counter must read 0 when the launch starts.
hipError_t launch_batch_pass(int prec, int pass, int n, int block, const BatchSeg* segs, int nseg,
                             int total, int* counter, int cus, hipStream_t s);
hipError_t launch_fill_i32(int* p, int v, int64_t count, hipStream_t s);

// Pair energies from the per-workgroup partial sums.
// e_pack[p] = sum of the parts of pack p (fixed order) * omega / N^2.
hipError_t launch_energy_reduce(const double* part, int npack, int parts, double factor,
                                double* e_pack, hipStream_t s);

// Small utility kernels.
hipError_t launch_fill_f64(double* p, double v, int64_t count, hipStream_t s);
hipError_t launch_cast_f64_f32(const double* in, float* out, int64_t count, hipStream_t s);

// Dense FP64 kernels (MFMA) and the small factorisation.
// C[m][n] = scale * sum_k A[m][k] B[n][k] for A (m x K), B (n x K) row-major,
// split over K into `nsplit` partial products reduced in a fixed order.
hipError_t launch_gemm_abt(const double* A, const double* B, int m, int n, int64_t K,
                           double scale, double* C, double* partial, int nsplit,
                           bool abs_inputs, const int* skip_if_nonzero, hipStream_t s);
int gemm_abt_splits(int m, int n, int64_t K);
// Out[m][r] = scale * sum_k A[m][k] B[k][r]; A (m x k) row-major small, B (k x R) row-major.
hipError_t launch_gemm_ab(const double* A, const double* B, int m, int k, int64_t R,
                          double scale, double* Out, const int* skip_if_nonzero, hipStream_t s);
// -M = L L^T (lower), then Linv = L^{-1}; info = 0 or the order of the first
// non-positive leading minor.  work: n*n doubles.
hipError_t launch_cholesky_inv(const double* M, int n, double* L, double* Linv, int* info,
                               hipStream_t s);
hipError_t launch_trace(const double* M, int n, double* out, hipStream_t s);
// out = sum_i w[i] e[i] in a fixed order (single workgroup)
hipError_t launch_weighted_sum(const double* e, const double* w, int count, double* out,
                               hipStream_t s);
hipError_t launch_scatter_pair_energies(const double* e_pack, const int* pair_of_pack,
                                        int npack, int n_orb, double weight_scale,
                                        double* pair_e, hipStream_t s);

// Pair screening (screen.hip): Berry-phase moments z[orb][6], Wannier
// features feat[orb][4] = (centre xyz, spread), MLP pair predictions.
hipError_t launch_moments(const double* phi, int n, int n_orb, int64_t npts, double dV, double* z,
                          hipStream_t s);
hipError_t launch_wannier_features(const double* z, int n_orb, const double* L, double* feat,
                                   hipStream_t s);
int mlp_weight_count();
hipError_t launch_mlp_pairs(const double* feat, int n_orb, const double* L, const float* wts,
                            float* pred, hipStream_t s);

// SCDM localisation (scdm.hip).
// Preselection: rho, g (|grad rho|) npts doubles each; part 2 * scdm_sum_blocks()
// doubles; means 2 doubles; cnt, off scdm_sel_blocks(npts) ints; points
// (capacity npts) and *count receive the kept points in increasing order.
int64_t scdm_sel_blocks(int64_t npts);
int scdm_sum_blocks();
hipError_t launch_scdm_preselect(const double* phi, int n, int k, const double* L, double* rho,
                                 double* g, double* part, double* means, int* cnt, int* off,
                                 int* points, int* count, hipStream_t s);
// Pivoted QR of the k x m matrix phi(:, points) (points == nullptr: all m = npts
// points): A m*k doubles, nrm m doubles, perm m ints, v k doubles, tau 1,
// rdiag k; pivots[k] = the chosen grid points; info = s + 1 on a zero
// residual column at step s (must be 0 on entry).
hipError_t launch_scdm_qr(const double* phi, const int* points, int m, int k, int64_t npts,
                          double* A, double* nrm, int* perm, double* v, double* tau,
                          double* rdiag, int* pivots, int* info, hipStream_t s);
// Newton-Schulz polar factor of A_C^T (A_C = phi at the pivots) into Y (k x k);
// G, Z k*k doubles, partial nsplit*k*k (nsplit = gemm_abt_splits(k, k, k)),
// state 3 ints; info = k + 1 if max_iter steps do not converge.
hipError_t launch_scdm_polar(const double* phi, const int* pivots, int k, int64_t npts, double* Y,
                             double* G, double* Z, double* partial, int nsplit, int* state,
                             int* info, int max_iter, hipStream_t s);
hipError_t launch_set_int(int* p, int v, hipStream_t s);

}  // namespace acex

// The apply stage of the host runtime (api.cpp), shared by the entry points
// that take their scratch from the caller's workspace and from the library's
// static array.  apply_check validates on the host (ACE_OK or a status);
// apply_enqueue launches C = dV psi xi^T (split over K into ns fixed-order
// partials held in part[ns][n_vec][n_orb]) and out = -C xi on stream s.
struct ace_plan;
namespace acex {
int apply_check(const ace_plan* p, const double* xi, const double* psi, int n_vec,
                const double* out);
int apply_splits(const ace_plan* p, int n_vec);
int apply_orbitals(const ace_plan* p);
int apply_enqueue(const ace_plan* p, hipStream_t s, double* C, double* part, int ns,
                  const double* xi, const double* psi, int n_vec, double* out);
int apply_device_present();
int apply_hip_fail(hipError_t e);
}  // namespace acex
