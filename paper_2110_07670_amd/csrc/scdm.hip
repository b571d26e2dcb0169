// SCDM localisation on gfx950 (arXiv 2110.07670, section "s-MTACE Method":
// a rank-revealing QR of Psi^* picks columns of the density matrix, which are
// orthonormalised; section "s'-MTACE Method": only grid points with
// rho > <rho> and |grad rho| < <|grad rho|> enter the QR).
//
//   preselection : k_density, k_grad_norm (central differences, periodic),
//                  fixed-order means, and an ordered compaction of the kept
//                  points (count per block, one scan, in-block prefix);
//   pivoted QR   : Businger-Golub column pivoting on the n_orb x m matrix,
//                  stored point-major (each column contiguous); per step one
//                  workgroup picks the pivot (largest residual norm, first
//                  index on a tie), swaps, and forms the Householder vector,
//                  then one wave per remaining column applies it and
//                  recomputes that column's residual norm;
//   orthonormalisation : Newton-Schulz iteration Y <- (3 Y - Y Y^T Y) / 2
//                  from Y = A_C^T / ||A_C||_F, which converges to the
//                  orthogonal polar factor; the MFMA products of dense.hip.
#include "kernels.h"

namespace acex {

namespace {

constexpr int kSelBlock = 1024;  // points per compaction block (256 threads x 4)
constexpr int kScdmSumBlocks = 1024;  // partial sums of the means

__device__ __forceinline__ double block_sum_1024(double v, double* red) {
  // fixed-order: wave tree, then the wave partials in order
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = (blockDim.x + 63) >> 6;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// rho(r) = sum_i phi_i(r)^2, products and sums rounded one by one, in order
__global__ void k_density(const double* __restrict__ phi, int k, int64_t npts,
                          double* __restrict__ rho) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= npts) return;
  double acc = 0.0;
  for (int i = 0; i < k; ++i) {
    const double f = phi[(int64_t)i * npts + r];
    acc = __dadd_rn(acc, __dmul_rn(f, f));
  }
  rho[r] = acc;
}

__global__ void k_grad_norm(const double* __restrict__ rho, int n, double two_h0, double two_h1,
                            double two_h2, double* __restrict__ g) {
  const int64_t npts = (int64_t)n * n * n;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= npts) return;
  const int z = (int)(r % n), y = (int)((r / n) % n), x = (int)(r / ((int64_t)n * n));
  const int64_t nn = (int64_t)n * n;
  const int xp = x + 1 == n ? 0 : x + 1, xm = x == 0 ? n - 1 : x - 1;
  const int yp = y + 1 == n ? 0 : y + 1, ym = y == 0 ? n - 1 : y - 1;
  const int zp = z + 1 == n ? 0 : z + 1, zm = z == 0 ? n - 1 : z - 1;
  const int64_t base_x = (int64_t)y * n + z, base_y = (int64_t)x * nn + z,
                base_z = (int64_t)x * nn + (int64_t)y * n;
  const double dx = (rho[xp * nn + base_x] - rho[xm * nn + base_x]) / two_h0;
  const double dy = (rho[base_y + (int64_t)yp * n] - rho[base_y + (int64_t)ym * n]) / two_h1;
  const double dz = (rho[base_z + zp] - rho[base_z + zm]) / two_h2;
  double s = 0.0;
  s = __dadd_rn(s, __dmul_rn(dx, dx));
  s = __dadd_rn(s, __dmul_rn(dy, dy));
  s = __dadd_rn(s, __dmul_rn(dz, dz));
  g[r] = sqrt(s);
}

// per-block partial sums of a and b over a grid-stride range
__global__ __launch_bounds__(256) void k_sum2_partial(const double* __restrict__ a,
                                                      const double* __restrict__ b, int64_t n,
                                                      double* __restrict__ part) {
  __shared__ double red[4];
  double sa = 0.0, sb = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    sa += a[i];
    sb += b[i];
  }
  const double ta = block_sum_1024(sa, red);
  const double tb = block_sum_1024(sb, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ta;
    part[2 * blockIdx.x + 1] = tb;
  }
}

__global__ __launch_bounds__(256) void k_sum2_final(const double* __restrict__ part, int nblk,
                                                    int64_t n, double* __restrict__ means) {
  __shared__ double red[4];
  double sa = 0.0, sb = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) {
    sa += part[2 * i];
    sb += part[2 * i + 1];
  }
  const double ta = block_sum_1024(sa, red);
  const double tb = block_sum_1024(sb, red);
  if (threadIdx.x == 0) {
    means[0] = ta / (double)n;
    means[1] = tb / (double)n;
  }
}

__device__ __forceinline__ bool kept(const double* rho, const double* g, const double* means,
                                     int64_t r) {
  return rho[r] > means[0] && g[r] < means[1];
}

// kept points per block of kSelBlock consecutive points
__global__ __launch_bounds__(256) void k_sel_count(const double* __restrict__ rho,
                                                   const double* __restrict__ g,
                                                   const double* __restrict__ means, int64_t npts,
                                                   int* __restrict__ cnt) {
  __shared__ int red[4];
  const int64_t r0 = (int64_t)blockIdx.x * kSelBlock;
  int c = 0;
  for (int q = 0; q < kSelBlock / 256; ++q) {
    const int64_t r = r0 + q * 256 + threadIdx.x;
    if (r < npts && kept(rho, g, means, r)) ++c;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) cnt[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// exclusive scan of the block counts (one thread; a few thousand blocks)
__global__ void k_sel_scan(const int* __restrict__ cnt, int nblk, int* __restrict__ off,
                           int* __restrict__ total) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int s = 0;
  for (int i = 0; i < nblk; ++i) {
    off[i] = s;
    s += cnt[i];
  }
  *total = s;
}

// write the kept points of each block, in increasing order
__global__ __launch_bounds__(256) void k_sel_write(const double* __restrict__ rho,
                                                   const double* __restrict__ g,
                                                   const double* __restrict__ means, int64_t npts,
                                                   const int* __restrict__ off,
                                                   int* __restrict__ points) {
  __shared__ int wsum[4];
  const int64_t r0 = (int64_t)blockIdx.x * kSelBlock;
  int base = off[blockIdx.x];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int q = 0; q < kSelBlock / 256; ++q) {
    const int64_t r = r0 + q * 256 + threadIdx.x;
    const bool f = r < npts && kept(rho, g, means, r);
    const unsigned long long bal = __ballot(f);
    const int below = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wid] = __popcll(bal);
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wid; ++w) before += wsum[w];
    if (f) points[base + before + below] = (int)r;
    const int tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    base += tot;
  }
}

// A (point-major, column j = point points[j], k values), residual norms, order
__global__ __launch_bounds__(256) void k_qr_gather(const double* __restrict__ phi,
                                                   const int* __restrict__ points, int m, int k,
                                                   int64_t npts, double* __restrict__ A,
                                                   double* __restrict__ nrm,
                                                   int* __restrict__ perm) {
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= m) return;
  const int64_t pt = points ? (int64_t)points[j] : (int64_t)j;
  double s = 0.0;
  for (int i = lane; i < k; i += 64) {
    const double v = phi[(int64_t)i * npts + pt];
    A[(int64_t)j * k + i] = v;
    s += v * v;
  }
  s = wave_sum(s);
  if (lane == 0) {
    nrm[j] = s;
    perm[j] = j;
  }
}

// Step s: pivot (largest residual norm over columns s..m-1, first on a tie),
// swap it into column s, Householder vector v (v[s] = 1, zeros above s) and
// tau with (I - tau v v^T) A[s:, s] = beta e_s; info = s + 1 on a zero column.
__global__ __launch_bounds__(1024) void k_qr_pivot(int s, int m, int k, double* __restrict__ A,
                                                   double* __restrict__ nrm,
                                                   int* __restrict__ perm, double* __restrict__ v,
                                                   double* __restrict__ tau,
                                                   double* __restrict__ rdiag,
                                                   int* __restrict__ info) {
  __shared__ double bv[16];
  __shared__ int bi[16];
  __shared__ double red[16];
  __shared__ double sx0, sbeta;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  double best = -1.0;
  int bidx = m;
  for (int j = s + tid; j < m; j += 1024) {
    const double x = nrm[j];
    if (x > best) {  // strided scan visits increasing j: keeps the first maximum
      best = x;
      bidx = j;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ob = __shfl_xor(best, off, 64);
    const int oi = __shfl_xor(bidx, off, 64);
    if (ob > best || (ob == best && oi < bidx)) {
      best = ob;
      bidx = oi;
    }
  }
  if (lane == 0) {
    bv[wid] = best;
    bi[wid] = bidx;
  }
  __syncthreads();
  if (tid == 0) {
    double b = bv[0];
    int ix = bi[0];
    for (int w = 1; w < 16; ++w)
      if (bv[w] > b || (bv[w] == b && bi[w] < ix)) {
        b = bv[w];
        ix = bi[w];
      }
    bi[0] = ix;
  }
  __syncthreads();
  const int p = bi[0] < m ? bi[0] : s;  // no column compares (NaN norms): keep s
  __syncthreads();
  if (p != s) {
    for (int i = tid; i < k; i += 1024) {
      const double t = A[(int64_t)s * k + i];
      A[(int64_t)s * k + i] = A[(int64_t)p * k + i];
      A[(int64_t)p * k + i] = t;
    }
    if (tid == 0) {
      const double t = nrm[s];
      nrm[s] = nrm[p];
      nrm[p] = t;
      const int q = perm[s];
      perm[s] = perm[p];
      perm[p] = q;
    }
  }
  __syncthreads();
  double* col = A + (int64_t)s * k;
  double ss = 0.0;
  for (int i = s + tid; i < k; i += 1024) ss += col[i] * col[i];
  const double nx2 = block_sum_1024(ss, red);
  if (tid == 0) {
    const double x0 = col[s];
    const double nx = sqrt(nx2);
    if (nx == 0.0) {
      sbeta = 0.0;
      tau[0] = 0.0;
      rdiag[s] = 0.0;
      if (*info == 0) *info = s + 1;
    } else {
      const double beta = x0 >= 0.0 ? -nx : nx;
      sbeta = beta;
      tau[0] = (beta - x0) / beta;
      rdiag[s] = beta;
    }
    sx0 = x0;
  }
  __syncthreads();
  const double beta = sbeta, x0 = sx0;
  for (int i = tid; i < k; i += 1024) {
    double vi = 0.0;
    if (i == s) vi = beta == 0.0 ? 0.0 : 1.0;
    else if (i > s && beta != 0.0) vi = col[i] / (x0 - beta);
    v[i] = vi;
  }
}

// Step s, every column j > s: A[s:, j] -= tau v (v^T A[s:, j]); residual norm
// over rows s+1.. recomputed.  One wave per column.
__global__ __launch_bounds__(256) void k_qr_apply(int s, int m, int k, double* __restrict__ A,
                                                  double* __restrict__ nrm,
                                                  const double* __restrict__ v,
                                                  const double* __restrict__ tau) {
  const int j = s + 1 + blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= m) return;
  double* col = A + (int64_t)j * k;
  const double t = tau[0];
  double w = 0.0;
  for (int i = s + lane; i < k; i += 64) w += v[i] * col[i];
  w = wave_sum(w);
  double r = 0.0;
  for (int i = s + lane; i < k; i += 64) {
    const double a = col[i] - t * v[i] * w;
    col[i] = a;
    if (i > s) r += a * a;
  }
  r = wave_sum(r);
  if (lane == 0) nrm[j] = r;
}

__global__ void k_pivot_points(const int* __restrict__ perm, const int* __restrict__ points,
                               int k, int* __restrict__ pivots) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  pivots[j] = points ? points[perm[j]] : perm[j];
}

// Y[j][i] = phi_i(pivot_j) / ||.||_F ; state flags cleared
__global__ __launch_bounds__(1024) void k_ns_init(const double* __restrict__ phi,
                                                  const int* __restrict__ pivots, int k,
                                                  int64_t npts, double* __restrict__ Y,
                                                  int* __restrict__ state) {
  __shared__ double red[16];
  double s = 0.0;
  for (int e = threadIdx.x; e < k * k; e += 1024) {
    const int j = e / k, i = e % k;
    const double x = phi[(int64_t)i * npts + pivots[j]];
    Y[e] = x;
    s += x * x;
  }
  const double fro = sqrt(block_sum_1024(s, red));
  __syncthreads();
  const double inv = fro > 0.0 ? 1.0 / fro : 0.0;
  for (int e = threadIdx.x; e < k * k; e += 1024) Y[e] *= inv;
  if (threadIdx.x == 0) {
    state[0] = 0;  // done: the products skip
    state[1] = 0;  // polishing iterations taken
    state[2] = 0;  // iterations taken
  }
}

// err = max |G - I| with G = Y Y^T.  Below 1e-10 two more steps polish the
// result (the iteration converges quadratically there); then done.
__global__ __launch_bounds__(1024) void k_ns_update(double* __restrict__ Y,
                                                    const double* __restrict__ G,
                                                    const double* __restrict__ Z, int k,
                                                    int* __restrict__ state) {
  if (state[0] != 0) return;
  __shared__ double red[16];
  __shared__ int go;
  double e = 0.0;
  for (int q = threadIdx.x; q < k * k; q += 1024) {
    const int j = q / k, i = q % k;
    const double d = fabs(G[q] - (i == j ? 1.0 : 0.0));
    e = d > e ? d : e;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl_xor(e, off, 64);
    e = o > e ? o : e;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int w = 0; w < 16; ++w) mx = red[w] > mx ? red[w] : mx;
    int pol = state[1];
    if (mx < 1e-10) ++pol;
    go = pol <= 2;
    state[1] = pol;
    state[2] += 1;
  }
  __syncthreads();
  if (!go) {
    if (threadIdx.x == 0) state[0] = 1;
    return;
  }
  for (int q = threadIdx.x; q < k * k; q += 1024) Y[q] = 1.5 * Y[q] - 0.5 * Z[q];
}

__global__ void k_set_int(int* __restrict__ p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void k_ns_finish(const int* __restrict__ state, int k, int* __restrict__ info) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && *info == 0 && state[0] == 0) *info = k + 1;
}

}  // namespace

int64_t scdm_sel_blocks(int64_t npts) { return (npts + kSelBlock - 1) / kSelBlock; }
int scdm_sum_blocks() { return kScdmSumBlocks; }

hipError_t launch_set_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_scdm_preselect(const double* phi, int n, int k, const double* L, double* rho,
                                 double* g, double* part, double* means, int* cnt, int* off,
                                 int* points, int* count, hipStream_t s) {
  const int64_t npts = (int64_t)n * n * n;
  const unsigned blocks = (unsigned)((npts + 255) / 256);
  hipLaunchKernelGGL(k_density, dim3(blocks), dim3(256), 0, s, phi, k, npts, rho);
  const double h0 = L[0] / n, h1 = L[1] / n, h2 = L[2] / n;
  hipLaunchKernelGGL(k_grad_norm, dim3(blocks), dim3(256), 0, s, rho, n, 2.0 * h0, 2.0 * h1,
                     2.0 * h2, g);
  hipLaunchKernelGGL(k_sum2_partial, dim3(kScdmSumBlocks), dim3(256), 0, s, rho, g, npts, part);
  hipLaunchKernelGGL(k_sum2_final, dim3(1), dim3(256), 0, s, part, kScdmSumBlocks, npts, means);
  const int64_t nb = scdm_sel_blocks(npts);
  hipLaunchKernelGGL(k_sel_count, dim3((unsigned)nb), dim3(256), 0, s, rho, g, means, npts, cnt);
  hipLaunchKernelGGL(k_sel_scan, dim3(1), dim3(64), 0, s, cnt, (int)nb, off, count);
  hipLaunchKernelGGL(k_sel_write, dim3((unsigned)nb), dim3(256), 0, s, rho, g, means, npts, off,
                     points);
  return hipGetLastError();
}

hipError_t launch_scdm_qr(const double* phi, const int* points, int m, int k, int64_t npts,
                          double* A, double* nrm, int* perm, double* v, double* tau,
                          double* rdiag, int* pivots, int* info, hipStream_t s) {
  hipLaunchKernelGGL(k_qr_gather, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, phi, points, m,
                     k, npts, A, nrm, perm);
  for (int st = 0; st < k; ++st) {
    hipLaunchKernelGGL(k_qr_pivot, dim3(1), dim3(1024), 0, s, st, m, k, A, nrm, perm, v, tau,
                       rdiag, info);
    const int rest = m - st - 1;
    if (rest > 0)
      hipLaunchKernelGGL(k_qr_apply, dim3((unsigned)((rest + 3) / 4)), dim3(256), 0, s, st, m, k,
                         A, nrm, v, tau);
  }
  hipLaunchKernelGGL(k_pivot_points, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, s, perm,
                     points, k, pivots);
  return hipGetLastError();
}

hipError_t launch_scdm_polar(const double* phi, const int* pivots, int k, int64_t npts, double* Y,
                             double* G, double* Z, double* partial, int nsplit, int* state,
                             int* info, int max_iter, hipStream_t s) {
  hipLaunchKernelGGL(k_ns_init, dim3(1), dim3(1024), 0, s, phi, pivots, k, npts, Y, state);
  hipError_t e = hipSuccess;
  for (int it = 0; it < max_iter; ++it) {
    e = launch_gemm_abt(Y, Y, k, k, k, 1.0, G, partial, nsplit, false, state, s);
    if (e != hipSuccess) return e;
    e = launch_gemm_ab(G, Y, k, k, k, 1.0, Z, state, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ns_update, dim3(1), dim3(1024), 0, s, Y, G, Z, k, state);
  }
  hipLaunchKernelGGL(k_ns_finish, dim3(1), dim3(64), 0, s, state, k, info);
  return hipGetLastError();
}

}  // namespace acex
