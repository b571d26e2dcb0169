// Dense FP64 stages of the ACE build on gfx950 (arXiv 2110.07670, section
// "ACE Operator"): the overlap matrix M = dV Phi^T W, the Cholesky factor of
// -M, the projectors xi = W L^{-T} and their application
// V_ACE psi = -xi (dV xi^T psi).  The products run on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64); the small factorisation runs in one workgroup.
//
// MFMA f64 16x16x4 operand layout (per wave, lane l):
//   A fragment: A[i = l % 16][k = l / 16]
//   B fragment: B[k = l / 16][j = l % 16]
//   D (4 doubles): D[i = l / 16 + 4 v][j = l % 16], v = 0..3
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace acex {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma16x16x4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------ C = A B^T, split K
// Workgroup: 256 threads (4 waves in 2 x 2), output tile 128 x 128, each wave
// 64 x 64 = 4 x 4 MFMA blocks.  K staged through LDS in slabs of KT; the next
// slab is loaded into registers while the current one feeds the MFMAs.
constexpr int kAbtTile = 128;
constexpr int kAbtKT = 32;
constexpr int kAbtPitch = kAbtKT + 1;
constexpr int kAbtPer = kAbtTile * kAbtKT / 256;  // elements per thread per operand

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

  double ra[kAbtPer], rb[kAbtPer];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < kAbtPer; ++q) {
      const int e = tid + q * 256;
      const int r = e / kAbtKT, c = e % kAbtKT;
      const int64_t k = k0 + c;
      double va = 0.0, vb = 0.0;
      if (k < kend) {
        if (m0 + r < m) va = A[(int64_t)(m0 + r) * K + k];
        if (n0 + r < n) vb = B[(int64_t)(n0 + r) * K + k];
      }
      ra[q] = abs_in ? fabs(va) : va;
      rb[q] = abs_in ? fabs(vb) : vb;
    }
  };
  if (kbeg < kend) fetch(kbeg);
  for (int64_t k0 = kbeg; k0 < kend; k0 += kAbtKT) {
#pragma unroll
    for (int q = 0; q < kAbtPer; ++q) {
      const int e = tid + q * 256;
      const int r = e / kAbtKT, c = e % kAbtKT;
      sA[r * kAbtPitch + c] = ra[q];
      sB[r * kAbtPitch + c] = rb[q];
    }
    __syncthreads();
    if (k0 + kAbtKT < kend) fetch(k0 + kAbtKT);
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
        const int row = m0 + wm * 64 + i * 16 + (lane >> 4) + 4 * v;
        const int col = n0 + wn * 64 + j * 16 + (lane & 15);
        if (row < m && col < n) out[(int64_t)row * n + col] = acc[i][j][v];
      }
}

// C[i] = scale * sum_s partial[s][i]: 64 outputs per workgroup, four threads
// per output each summing a fixed residue class of s, combined in a fixed order.
__global__ __launch_bounds__(256) void k_reduce_splits(const double* __restrict__ partial,
                                                       int nsplit, int64_t count, double scale,
                                                       double* __restrict__ C,
                                                       const int* __restrict__ skip) {
  if (skip && *skip != 0) return;
  __shared__ double red[4][64];
  const int o = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + o;
  double s0 = 0.0, s1 = 0.0;
  if (i < count) {
    int k = g;
    for (; k + 4 < nsplit; k += 8) {
      s0 += partial[(int64_t)k * count + i];
      s1 += partial[(int64_t)(k + 4) * count + i];
    }
    if (k < nsplit) s0 += partial[(int64_t)k * count + i];
  }
  red[g][o] = s0 + s1;
  __syncthreads();
  if (g == 0 && i < count) C[i] = scale * ((red[0][o] + red[1][o]) + (red[2][o] + red[3][o]));
}

int gemm_abt_splits(int m, int n, int64_t K) {
  const int tiles = ((m + kAbtTile - 1) / kAbtTile) * ((n + kAbtTile - 1) / kAbtTile);
  // aim for about 1024 workgroups, at least 8 K-slabs each
  int64_t ns = (1024 + tiles - 1) / tiles;
  const int64_t maxs = (K + 8 * kAbtKT - 1) / (8 * kAbtKT);
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
  hipLaunchKernelGGL(k_reduce_splits, dim3((unsigned)((count + 63) / 64)), dim3(256), 0, s,
                     partial, nsplit, count, scale, C, skip);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Out = A B (A small)
// Workgroup: 256 threads, output tile 64 rows x 128 columns; wave w owns
// rows [16 w, 16 w + 16) x 128 columns = 8 MFMA blocks.  Rows beyond 64 are
// covered by more workgroups (row blocks).  Next K-slab prefetched into
// registers.
constexpr int kAbRows = 64;
constexpr int kAbCols = 128;
constexpr int kAbKT = 16;
constexpr int kAbPerA = kAbRows * kAbKT / 256;
constexpr int kAbPerB = kAbKT * kAbCols / 256;

__global__ __launch_bounds__(256) void k_gemm_ab(const double* __restrict__ A,
                                                 const double* __restrict__ B, int m, int k,
                                                 int64_t R, double scale, double* __restrict__ Out,
                                                 const int* __restrict__ skip) {
  if (skip && *skip != 0) return;
  __shared__ double sA[kAbRows * (kAbKT + 1)];
  __shared__ double sB[kAbKT * kAbCols];
  // Workgroup b runs on XCD b mod 8: the row blocks of one column block are
  // consecutive on one XCD, so B's columns are read from HBM once and the
  // other row blocks find them in that XCD's L2.
  const int nrb = (m + kAbRows - 1) / kAbRows;
  const int64_t ncb = (R + kAbCols - 1) / kAbCols;
  const int64_t g = blockIdx.x >> 3;
  const int xcd = blockIdx.x & 7;
  const int rblk = (int)(g % nrb);
  const int64_t cblk = (g / nrb) * 8 + xcd;
  if (cblk >= ncb) return;
  const int64_t r0 = cblk * kAbCols;
  const int m0 = rblk * kAbRows;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  d4 acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
  double ra[kAbPerA], rb[kAbPerB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < kAbPerA; ++q) {
      const int e = tid + q * 256;
      const int r = e / kAbKT, c = e % kAbKT;
      ra[q] = (m0 + r < m && k0 + c < k) ? A[(int64_t)(m0 + r) * k + k0 + c] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kAbPerB; ++q) {
      const int e = tid + q * 256;
      const int kr = e / kAbCols, c = e % kAbCols;
      rb[q] = (k0 + kr < k && r0 + c < R) ? B[(int64_t)(k0 + kr) * R + r0 + c] : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < k; k0 += kAbKT) {
#pragma unroll
    for (int q = 0; q < kAbPerA; ++q) {
      const int e = tid + q * 256;
      sA[(e / kAbKT) * (kAbKT + 1) + e % kAbKT] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < kAbPerB; ++q) {
      const int e = tid + q * 256;
      sB[(e / kAbCols) * kAbCols + e % kAbCols] = rb[q];
    }
    __syncthreads();
    if (k0 + kAbKT < k) fetch(k0 + kAbKT);
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
      const int row = m0 + wave * 16 + (lane >> 4) + 4 * v;
      const int64_t col = r0 + j * 16 + (lane & 15);
      if (row < m && col < R) Out[(int64_t)row * R + col] = scale * acc[j][v];
    }
}

hipError_t launch_gemm_ab(const double* A, const double* B, int m, int k, int64_t R, double scale,
                          double* Out, const int* skip, hipStream_t s) {
  const int64_t ncb = (R + kAbCols - 1) / kAbCols;
  const int64_t nrb = (m + kAbRows - 1) / kAbRows;
  const int64_t blocks = ((ncb + 7) / 8) * 8 * nrb;  // column blocks padded to the 8 XCDs
  hipLaunchKernelGGL(k_gemm_ab, dim3((unsigned)blocks), dim3(256), 0, s, A, B, m, k, R, scale,
                     Out, skip);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Cholesky and L^{-1}
// One workgroup of 1024 threads.  The matrix lives in LDS when n <= 128 and
// in the Linv output buffer otherwise.
//  1. A = -M (lower triangle read).
//  2. Right-looking Cholesky: pivot d = A[j][j]; a non-positive (or NaN)
//     pivot stops with info = j + 1; L[j][j] = sqrt(d); scale the column;
//     update the trailing lower triangle.
//  3. L -> global.
//  4. In-place inverse, columns from the last: with X = L^{-1} already in the
//     trailing block, X[j][j] = 1 / L[j][j] and
//     X[i][j] = -X[j][j] sum_{k=j+1..i} X[i][k] L[k][j]  (i > j);
//     eight threads share each dot product (fixed-order shuffle sum).
constexpr int kCholLdsN = 128;
constexpr int kCholMaxN = 512;

template <bool LDS>
__global__ __launch_bounds__(1024) void k_chol_inv(const double* __restrict__ M, int n,
                                                   double* __restrict__ L,
                                                   double* __restrict__ Linv,
                                                   int* __restrict__ info) {
  __shared__ double smat[LDS ? kCholLdsN * (kCholLdsN + 1) : 1];
  __shared__ double col[kCholMaxN];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int P = LDS ? n + 1 : n;
  double* A = LDS ? smat : Linv;
  for (int64_t e = tid; e < (int64_t)n * n; e += 1024) {
    const int i = (int)(e / n), j = (int)(e % n);
    A[(int64_t)i * P + j] = (j <= i) ? -M[e] : 0.0;
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double d = A[(int64_t)j * P + j];
    if (!(d > 0.0)) {
      if (tid == 0) bad = j + 1;
      break;
    }
    const double ljj = sqrt(d);
    __syncthreads();
    if (tid == 0) A[(int64_t)j * P + j] = ljj;
    for (int i = j + 1 + tid; i < n; i += 1024) A[(int64_t)i * P + j] /= ljj;
    __syncthreads();
    const int rem = n - j - 1;
    for (int64_t e = tid; e < (int64_t)rem * rem; e += 1024) {
      const int ii = (int)(e / rem), kk = (int)(e % rem);
      if (kk > ii) continue;
      const int i = j + 1 + ii, k = j + 1 + kk;
      A[(int64_t)i * P + k] -= A[(int64_t)i * P + j] * A[(int64_t)k * P + j];
    }
    __syncthreads();
  }
  __syncthreads();
  const int failed = bad;
  if (tid == 0) *info = failed;
  if (failed) return;
  for (int64_t e = tid; e < (int64_t)n * n; e += 1024) {
    const int i = (int)(e / n), j = (int)(e % n);
    L[e] = (j <= i) ? A[(int64_t)i * P + j] : 0.0;
  }
  __syncthreads();
  const int g = tid & 7, row0 = tid >> 3;  // 128 row slots, 8 threads each
  for (int j = n - 1; j >= 0; --j) {
    for (int k = j + 1 + tid; k < n; k += 1024) col[k] = A[(int64_t)k * P + j];
    __syncthreads();
    const double djj = 1.0 / A[(int64_t)j * P + j];
    for (int i0 = j + 1; i0 < n; i0 += 128) {
      const int i = i0 + row0;
      double s = 0.0;
      if (i < n)
        for (int k = j + 1 + g; k <= i; k += 8) s += A[(int64_t)i * P + k] * col[k];
      s += __shfl_xor(s, 1, 64);
      s += __shfl_xor(s, 2, 64);
      s += __shfl_xor(s, 4, 64);
      if (i < n && g == 0) A[(int64_t)i * P + j] = -djj * s;
    }
    __syncthreads();
    if (tid == 0) A[(int64_t)j * P + j] = djj;
    __syncthreads();
  }
  for (int64_t e = tid; e < (int64_t)n * n; e += 1024) {
    const int i = (int)(e / n), j = (int)(e % n);
    if (LDS) Linv[e] = (j <= i) ? A[(int64_t)i * P + j] : 0.0;
    else if (j > i) Linv[e] = 0.0;
  }
}

hipError_t launch_cholesky_inv(const double* M, int n, double* L, double* Linv, int* info,
                               hipStream_t s) {
  if (n > kCholMaxN) return hipErrorInvalidValue;
  if (n <= kCholLdsN)
    hipLaunchKernelGGL((k_chol_inv<true>), dim3(1), dim3(1024), 0, s, M, n, L, Linv, info);
  else
    hipLaunchKernelGGL((k_chol_inv<false>), dim3(1), dim3(1024), 0, s, M, n, L, Linv, info);
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
