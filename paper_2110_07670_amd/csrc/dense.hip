// Dense FP64 stages of the ACE build on gfx950 (arXiv 2110.07670, section
// "ACE Operator"): the overlap matrix M = dV Phi^T W, the Cholesky factor of
// -M, the projectors xi = W L^{-T} and their application
// V_ACE psi = -xi (dV xi^T psi).  The products run on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64); the small factorisation runs in one workgroup.
//
// MFMA f64 16x16x4 operand layout (per wave, lane l):
//   A fragment: A[i = l % 16][k = l / 16]
//   B fragment: B[k = l / 16][j = l % 16]
//   D (4 doubles): D[i = 4*(l / 16) + v][j = l % 16], v = 0..3
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace acex {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma16x16x4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------ C = A B^T, split K
// Workgroup: 256 threads (4 waves in 2 x 2), output tile 128 x 128, each wave
// 64 x 64 = 4 x 4 MFMA blocks.  K staged through LDS in slabs of KT.
constexpr int kAbtTile = 128;
constexpr int kAbtKT = 16;
constexpr int kAbtPitch = kAbtKT + 1;

__global__ __launch_bounds__(256) void k_gemm_abt(const double* __restrict__ A,
                                                  const double* __restrict__ B, int m, int n,
                                                  int64_t K, int64_t kchunk, int tiles_n,
                                                  bool abs_in, double* __restrict__ partial,
                                                  const int* __restrict__ skip) {
  if (skip && *skip != 0) return;
  __shared__ double sA[kAbtTile * kAbtPitch];
  __shared__ double sB[kAbtTile * kAbtPitch];
  const int tile = blockIdx.x;
  const int split = blockIdx.y;
  const int tm = tile / tiles_n, tn = tile % tiles_n;
  const int m0 = tm * kAbtTile, n0 = tn * kAbtTile;
  const int64_t kbeg = (int64_t)split * kchunk;
  int64_t kend = kbeg + kchunk;
  if (kend > K) kend = K;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  for (int64_t k0 = kbeg; k0 < kend; k0 += kAbtKT) {
    // stage A[m0..m0+128)[k0..k0+KT) and B likewise; 2048 elements each
#pragma unroll
    for (int e = tid; e < kAbtTile * kAbtKT; e += 256) {
      const int r = e / kAbtKT, c = e % kAbtKT;
      const int64_t k = k0 + c;
      double va = 0.0, vb = 0.0;
      if (k < kend) {
        if (m0 + r < m) va = A[(int64_t)(m0 + r) * K + k];
        if (n0 + r < n) vb = B[(int64_t)(n0 + r) * K + k];
      }
      if (abs_in) {
        va = fabs(va);
        vb = fabs(vb);
      }
      sA[r * kAbtPitch + c] = va;
      sB[r * kAbtPitch + c] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kAbtKT; kk += 4) {
      double af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        af[i] = sA[(wm * 64 + i * 16 + (lane & 15)) * kAbtPitch + kk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        bf[j] = sB[(wn * 64 + j * 16 + (lane & 15)) * kAbtPitch + kk + (lane >> 4)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma16x16x4(af[i], bf[j], acc[i][j]);
    }
    __syncthreads();
  }
  double* out = partial + (int64_t)split * m * n;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + v;
        const int col = n0 + wn * 64 + j * 16 + (lane & 15);
        if (row < m && col < n) out[(int64_t)row * n + col] = acc[i][j][v];
      }
}

__global__ void k_reduce_splits(const double* __restrict__ partial, int nsplit, int64_t count,
                                double scale, double* __restrict__ C, const int* __restrict__ skip) {
  if (skip && *skip != 0) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double s = 0.0;
  for (int k = 0; k < nsplit; ++k) s += partial[(int64_t)k * count + i];
  C[i] = scale * s;
}

int gemm_abt_splits(int m, int n, int64_t K) {
  const int tiles = ((m + kAbtTile - 1) / kAbtTile) * ((n + kAbtTile - 1) / kAbtTile);
  // aim for about 1024 workgroups, at least 4 K-slabs each
  int64_t ns = (1024 + tiles - 1) / tiles;
  const int64_t maxs = (K + 4 * kAbtKT - 1) / (4 * kAbtKT);
  if (ns > maxs) ns = maxs;
  if (ns < 1) ns = 1;
  return (int)ns;
}

hipError_t launch_gemm_abt(const double* A, const double* B, int m, int n, int64_t K,
                           double scale, double* C, double* partial, int nsplit, bool abs_inputs,
                           const int* skip, hipStream_t s) {
  const int tiles_m = (m + kAbtTile - 1) / kAbtTile, tiles_n = (n + kAbtTile - 1) / kAbtTile;
  int64_t kchunk = (K + nsplit - 1) / nsplit;
  kchunk = ((kchunk + kAbtKT - 1) / kAbtKT) * kAbtKT;
  hipLaunchKernelGGL(k_gemm_abt, dim3(tiles_m * tiles_n, nsplit), dim3(256), 0, s, A, B, m, n, K,
                     kchunk, tiles_n, abs_inputs, partial, skip);
  const int64_t count = (int64_t)m * n;
  hipLaunchKernelGGL(k_reduce_splits, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                     partial, nsplit, count, scale, C, skip);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Out = A B (A small)
// Workgroup: 256 threads, output tile 64 rows x 128 columns; wave w owns
// rows [16 w, 16 w + 16) x 128 columns = 8 MFMA blocks.  Rows beyond 64 are
// covered by more workgroups along grid y.
constexpr int kAbRows = 64;
constexpr int kAbCols = 128;
constexpr int kAbKT = 16;

__global__ __launch_bounds__(256) void k_gemm_ab(const double* __restrict__ A,
                                                 const double* __restrict__ B, int m, int k,
                                                 int64_t R, double scale, double* __restrict__ Out,
                                                 const int* __restrict__ skip) {
  if (skip && *skip != 0) return;
  __shared__ double sA[kAbRows * (kAbKT + 1)];
  __shared__ double sB[kAbKT * kAbCols];
  const int64_t r0 = (int64_t)blockIdx.x * kAbCols;
  const int m0 = blockIdx.y * kAbRows;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  d4 acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < k; k0 += kAbKT) {
    for (int e = tid; e < kAbRows * kAbKT; e += 256) {
      const int r = e / kAbKT, c = e % kAbKT;
      double v = 0.0;
      if (m0 + r < m && k0 + c < k) v = A[(int64_t)(m0 + r) * k + k0 + c];
      sA[r * (kAbKT + 1) + c] = v;
    }
    for (int e = tid; e < kAbKT * kAbCols; e += 256) {
      const int kr = e / kAbCols, c = e % kAbCols;
      double v = 0.0;
      if (k0 + kr < k && r0 + c < R) v = B[(int64_t)(k0 + kr) * R + r0 + c];
      sB[kr * kAbCols + c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kAbKT; kk += 4) {
      const double af = sA[(wave * 16 + (lane & 15)) * (kAbKT + 1) + kk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const double bf = sB[(kk + (lane >> 4)) * kAbCols + j * 16 + (lane & 15)];
        acc[j] = mfma16x16x4(af, bf, acc[j]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = m0 + wave * 16 + 4 * (lane >> 4) + v;
      const int64_t col = r0 + j * 16 + (lane & 15);
      if (row < m && col < R) Out[(int64_t)row * R + col] = scale * acc[j][v];
    }
}

hipError_t launch_gemm_ab(const double* A, const double* B, int m, int k, int64_t R, double scale,
                          double* Out, const int* skip, hipStream_t s) {
  const dim3 grid((unsigned)((R + kAbCols - 1) / kAbCols), (unsigned)((m + kAbRows - 1) / kAbRows));
  hipLaunchKernelGGL(k_gemm_ab, grid, dim3(256), 0, s, A, B, m, k, R, scale, Out, skip);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Cholesky and L^{-1}
// One workgroup.  Right-looking: for column j, pivot d = A[j][j] (already
// updated), L[j][j] = sqrt(d), scale the column, update the trailing lower
// triangle.  A non-positive (or NaN) pivot stops with info = j + 1.
__global__ __launch_bounds__(1024) void k_cholesky(const double* __restrict__ M, int n,
                                                   double* __restrict__ L, int* __restrict__ info) {
  const int tid = threadIdx.x;
  __shared__ int bad;
  for (int64_t e = tid; e < (int64_t)n * n; e += 1024) {
    const int i = (int)(e / n), j = (int)(e % n);
    L[e] = (j <= i) ? -M[e] : 0.0;
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double d = L[(int64_t)j * n + j];
    if (!(d > 0.0)) {
      if (tid == 0) bad = j + 1;
      break;
    }
    const double ljj = sqrt(d);
    __syncthreads();
    if (tid == 0) L[(int64_t)j * n + j] = ljj;
    for (int i = j + 1 + tid; i < n; i += 1024) L[(int64_t)i * n + j] /= ljj;
    __syncthreads();
    const int rem = n - j - 1;
    for (int64_t e = tid; e < (int64_t)rem * rem; e += 1024) {
      const int ii = (int)(e / rem), kk = (int)(e % rem);
      if (kk > ii) continue;
      const int i = j + 1 + ii, k = j + 1 + kk;
      L[(int64_t)i * n + k] -= L[(int64_t)i * n + j] * L[(int64_t)k * n + j];
    }
    __syncthreads();
  }
  __syncthreads();
  if (tid == 0) *info = bad;
}

// Linv = L^{-1} (lower); thread j owns column j: forward substitution.
__global__ __launch_bounds__(256) void k_tri_inv(const double* __restrict__ L, int n,
                                                 double* __restrict__ X, const int* __restrict__ info) {
  if (*info != 0) return;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  for (int i = 0; i < j; ++i) X[(int64_t)i * n + j] = 0.0;
  for (int i = j; i < n; ++i) {
    double s = (i == j) ? 1.0 : 0.0;
    for (int k = j; k < i; ++k) s -= L[(int64_t)i * n + k] * X[(int64_t)k * n + j];
    X[(int64_t)i * n + j] = s / L[(int64_t)i * n + i];
  }
}

hipError_t launch_cholesky_inv(const double* M, int n, double* L, double* Linv, int* info,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(1024), 0, s, M, n, L, info);
  hipLaunchKernelGGL(k_tri_inv, dim3((n + 255) / 256), dim3(256), 0, s, L, n, Linv, info);
  return hipGetLastError();
}

// ------------------------------------------------------------------ reductions
__global__ void k_trace(const double* __restrict__ M, int n, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += M[(int64_t)i * n + i];
    *out = s;
  }
}

hipError_t launch_trace(const double* M, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(64), 0, s, M, n, out);
  return hipGetLastError();
}

// Fixed-order weighted sum: 256 contiguous chunks, then the chunk sums in order.
__global__ __launch_bounds__(256) void k_weighted_sum(const double* __restrict__ e,
                                                      const double* __restrict__ w, int count,
                                                      double* __restrict__ out) {
  __shared__ double part[256];
  const int tid = threadIdx.x;
  const int per = (count + 255) / 256;
  double s = 0.0;
  const int b = tid * per;
  for (int i = b; i < b + per && i < count; ++i) s += w[i] * e[i];
  part[tid] = s;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int i = 0; i < 256; ++i) t += part[i];
    *out = t;
  }
}

hipError_t launch_weighted_sum(const double* e, const double* w, int count, double* out,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_weighted_sum, dim3(1), dim3(256), 0, s, e, w, count, out);
  return hipGetLastError();
}

// pair_e[i][j] = weight * e_pack[p] for packs carrying one pair (i, j)
__global__ void k_scatter_pairs(const double* __restrict__ e_pack, const int* __restrict__ pair_of_pack,
                                int npack, int n_orb, double wscale, double* __restrict__ pair_e) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npack) return;
  const int code = pair_of_pack[p];
  const int i = code / n_orb, j = code % n_orb;
  pair_e[(int64_t)i * n_orb + j] = wscale * (i == j ? 1.0 : 2.0) * e_pack[p];
}

hipError_t launch_scatter_pair_energies(const double* e_pack, const int* pair_of_pack, int npack,
                                        int n_orb, double weight_scale, double* pair_e,
                                        hipStream_t s) {
  if (npack <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_pairs, dim3((npack + 255) / 256), dim3(256), 0, s, e_pack,
                     pair_of_pack, npack, n_orb, weight_scale, pair_e);
  return hipGetLastError();
}

}  // namespace acex
