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
// 64 x 64 = 4 x 4 MFMA blocks.  K staged through two LDS buffers in slabs of
// KT: while the MFMAs read one slab, the next one (loaded into registers
// behind them) is stored into the other buffer, so each slab costs one
// barrier.  VEC (even K, 16-byte aligned operands): two consecutive k per
// load and per LDS store, rows padded to 18 (16-byte aligned, and the MFMA
// operand reads of 32 lanes still fall on distinct banks); else one k per
// access, rows padded to 17.
constexpr int kAbtTile = 128;
constexpr int kAbtKT = 16;
constexpr int kAbtPer = kAbtTile * kAbtKT / 256;  // elements per thread per operand

template <bool VEC>
__global__ __launch_bounds__(256) void k_gemm_abt(const double* __restrict__ A,
                                                  const double* __restrict__ B, int m, int n,
                                                  int64_t K, int64_t kchunk, int tiles_n,
                                                  bool abs_in, double* __restrict__ partial,
                                                  const int* __restrict__ skip) {
  if (skip && *skip != 0) return;
  constexpr int kAbtPitch = VEC ? kAbtKT + 2 : kAbtKT + 1;
  __shared__ __align__(16) double sA[2][kAbtTile * kAbtPitch];
  __shared__ __align__(16) double sB[2][kAbtTile * kAbtPitch];
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
    if constexpr (VEC) {
      // element pairs (r, c), (r, c + 1), c even; kend is even
#pragma unroll
      for (int q = 0; q < kAbtPer / 2; ++q) {
        const int e = tid + q * 256;
        const int r = e / (kAbtKT / 2), c = 2 * (e % (kAbtKT / 2));
        const int64_t k = k0 + c;
        double2 va = {0.0, 0.0}, vb = {0.0, 0.0};
        if (k < kend) {
          if (m0 + r < m) va = *reinterpret_cast<const double2*>(A + (int64_t)(m0 + r) * K + k);
          if (n0 + r < n) vb = *reinterpret_cast<const double2*>(B + (int64_t)(n0 + r) * K + k);
        }
        ra[2 * q] = abs_in ? fabs(va.x) : va.x;
        ra[2 * q + 1] = abs_in ? fabs(va.y) : va.y;
        rb[2 * q] = abs_in ? fabs(vb.x) : vb.x;
        rb[2 * q + 1] = abs_in ? fabs(vb.y) : vb.y;
      }
    } else {
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
    }
  };
  auto stage = [&](int buf) {
    if constexpr (VEC) {
#pragma unroll
      for (int q = 0; q < kAbtPer / 2; ++q) {
        const int e = tid + q * 256;
        const int r = e / (kAbtKT / 2), c = 2 * (e % (kAbtKT / 2));
        *reinterpret_cast<double2*>(&sA[buf][r * kAbtPitch + c]) = double2{ra[2 * q], ra[2 * q + 1]};
        *reinterpret_cast<double2*>(&sB[buf][r * kAbtPitch + c]) = double2{rb[2 * q], rb[2 * q + 1]};
      }
    } else {
#pragma unroll
      for (int q = 0; q < kAbtPer; ++q) {
        const int e = tid + q * 256;
        const int r = e / kAbtKT, c = e % kAbtKT;
        sA[buf][r * kAbtPitch + c] = ra[q];
        sB[buf][r * kAbtPitch + c] = rb[q];
      }
    }
  };
  if (kbeg < kend) {
    fetch(kbeg);
    stage(0);
  }
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += kAbtKT) {
    const bool more = k0 + kAbtKT < kend;
    if (more) fetch(k0 + kAbtKT);
#pragma unroll
    for (int kk = 0; kk < kAbtKT; kk += 4) {
      double af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        af[i] = sA[buf][(wm * 64 + i * 16 + (lane & 15)) * kAbtPitch + kk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        bf[j] = sB[buf][(wn * 64 + j * 16 + (lane & 15)) * kAbtPitch + kk + (lane >> 4)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma16x16x4(af[i], bf[j], acc[i][j]);
    }
    if (more) stage(buf ^ 1);
    __syncthreads();
    buf ^= 1;
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
  const bool vec = K % 2 == 0 && reinterpret_cast<uintptr_t>(A) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(B) % 16 == 0;
  if (vec)
    hipLaunchKernelGGL(k_gemm_abt<true>, dim3(tiles_m * tiles_n, nsplit), dim3(256), 0, s, A, B,
                       m, n, K, kchunk, tiles_n, abs_inputs, partial, skip);
  else
    hipLaunchKernelGGL(k_gemm_abt<false>, dim3(tiles_m * tiles_n, nsplit), dim3(256), 0, s, A, B,
                       m, n, K, kchunk, tiles_n, abs_inputs, partial, skip);
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
// -M = L L^T (lower, positive diagonal), then X = L^{-1}, in blocks of 32
// columns (a partial last block when 32 does not divide n).
//
// k_chol_left: one workgroup of 1024 threads, left-looking, L built in place
// in the L buffer (at these sizes it stays in the CU's caches).  Block column
// J (columns j0 .. j0 + w - 1):
//   1. the finished columns 0 .. j0-1 of its rows are staged in LDS,
//      transposed: lj[k][c] = L[j0 + c][k];
//   2. every row i >= j0: A[i][j0 + c] -= sum_{k < j0} L[i][k] lj[k][c]
//      (thread = (row, c), k in increasing order);
//   3. the diagonal block is factored in LDS, unblocked; a non-positive (or
//      NaN) pivot stops the factorisation with info = column + 1;
//   4. the rows below it are solved against it, L[i][J] = A[i][J] D^{-T}
//      (one thread per row, the row in registers).
// k_tri_inv: one workgroup per block column J of X; forward block
// substitution down the row blocks I >= J with the block column in LDS:
//   X[I][J] = D_I^{-1} (delta - sum_{J <= K < I} L[I][K] X[K][J]),
// the triangular solve by one thread per column with the column in
// registers.  Both are skipped after a failed factorisation (X undefined).
constexpr int kCholNB = 32;
constexpr int kCholMaxN = 512;

__global__ __launch_bounds__(1024) void k_chol_left(const double* __restrict__ M, int n,
                                                    double* __restrict__ L,
                                                    int* __restrict__ info) {
  __shared__ double lj[kCholMaxN - kCholNB][kCholNB];
  __shared__ double dblk[kCholNB][kCholNB + 1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int c = tid % kCholNB, il = tid / kCholNB;
  for (int64_t e = tid; e < (int64_t)n * n; e += 1024) {
    const int i = (int)(e / n), j = (int)(e % n);
    L[e] = (j <= i) ? -M[e] : 0.0;
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j0 = 0; j0 < n; j0 += kCholNB) {
    const int w = min(kCholNB, n - j0);
    // 1. stage the block's rows of the finished columns
    for (int e = tid; e < j0 * kCholNB; e += 1024) {
      const int k = e / kCholNB, cc = e % kCholNB;
      lj[k][cc] = cc < w ? L[(int64_t)(j0 + cc) * n + k] : 0.0;
    }
    __syncthreads();
    // 2. left-looking update of the block column
    if (c < w) {
      for (int i = j0 + il; i < n; i += 1024 / kCholNB) {
        const double* __restrict__ li = L + (int64_t)i * n;
        double s = li[j0 + c];
#pragma unroll 8
        for (int k = 0; k < j0; ++k) s -= li[k] * lj[k][c];
        L[(int64_t)i * n + j0 + c] = s;
      }
    }
    __syncthreads();
    // 3. the diagonal block, factored in LDS
    for (int e = tid; e < w * w; e += 1024) {
      const int r = e / w, cc = e % w;
      dblk[r][cc] = L[(int64_t)(j0 + r) * n + j0 + cc];
    }
    __syncthreads();
    for (int j = 0; j < w; ++j) {
      const double d = dblk[j][j];
      if (!(d > 0.0)) {
        if (tid == 0) bad = j0 + j + 1;
        break;
      }
      const double ljj = sqrt(d);
      __syncthreads();
      if (tid == 0) dblk[j][j] = ljj;
      if (tid > j && tid < w) dblk[tid][j] /= ljj;
      __syncthreads();
      const int rem = w - j - 1;
      for (int e = tid; e < rem * rem; e += 1024) {
        const int rr = e / rem, kk = e % rem;
        if (kk <= rr) dblk[j + 1 + rr][j + 1 + kk] -= dblk[j + 1 + rr][j] * dblk[j + 1 + kk][j];
      }
      __syncthreads();
    }
    __syncthreads();
    if (bad) break;
    for (int e = tid; e < w * w; e += 1024) {
      const int r = e / w, cc = e % w;
      L[(int64_t)(j0 + r) * n + j0 + cc] = cc <= r ? dblk[r][cc] : 0.0;
    }
    // 4. rows below: forward substitution against the diagonal block (w = 32
    // whenever rows remain below it)
    const int i = j0 + kCholNB + tid;
    if (w == kCholNB && i < n) {
      double* __restrict__ li = L + (int64_t)i * n + j0;
      double x[kCholNB];
#pragma unroll
      for (int cc = 0; cc < kCholNB; ++cc) x[cc] = li[cc];
#pragma unroll
      for (int cc = 0; cc < kCholNB; ++cc) {
#pragma unroll
        for (int k = 0; k < cc; ++k) x[cc] -= x[k] * dblk[cc][k];
        x[cc] /= dblk[cc][cc];
      }
#pragma unroll
      for (int cc = 0; cc < kCholNB; ++cc) li[cc] = x[cc];
    }
    __syncthreads();
  }
  __syncthreads();
  if (tid == 0) *info = bad;
}

__global__ __launch_bounds__(1024) void k_tri_inv(const double* __restrict__ L, int n,
                                                  double* __restrict__ X,
                                                  const int* __restrict__ info) {
  __shared__ double xs[kCholMaxN][kCholNB];  // rows j0 .. n-1 of the block column
  __shared__ double dblk[kCholNB][kCholNB + 1];
  if (*info != 0) return;
  const int j0 = blockIdx.x * kCholNB;
  const int w = min(kCholNB, n - j0);
  const int tid = threadIdx.x, c = tid % kCholNB, il = tid / kCholNB;
  for (int i0 = j0; i0 < n; i0 += kCholNB) {
    const int h = min(kCholNB, n - i0);
    // right-hand sides of row block I
    if (il < h && c < w) {
      const int i = i0 + il;
      const double* __restrict__ li = L + (int64_t)i * n;
      double s = (i == j0 + c) ? 1.0 : 0.0;
#pragma unroll 8
      for (int k = j0; k < i0; ++k) s -= li[k] * xs[k - j0][c];
      xs[i - j0][c] = s;
    }
    for (int e = tid; e < h * h; e += 1024) {
      const int r = e / h, cc = e % h;
      dblk[r][cc] = L[(int64_t)(i0 + r) * n + i0 + cc];
    }
    __syncthreads();
    // X[I][J] = D_I^{-1} (right-hand sides): one thread per column
    if (tid < w) {
      double x[kCholNB];
#pragma unroll
      for (int r = 0; r < kCholNB; ++r) x[r] = r < h ? xs[i0 - j0 + r][tid] : 0.0;
#pragma unroll
      for (int r = 0; r < kCholNB; ++r) {
        if (r < h) {
#pragma unroll
          for (int k = 0; k < r; ++k) x[r] -= dblk[r][k] * x[k];
          x[r] /= dblk[r][r];
        }
      }
#pragma unroll
      for (int r = 0; r < kCholNB; ++r)
        if (r < h) xs[i0 - j0 + r][tid] = x[r];
    }
    __syncthreads();
  }
  for (int e = tid; e < n * kCholNB; e += 1024) {
    const int i = e / kCholNB, cc = e % kCholNB;
    if (cc >= w) continue;
    const int col = j0 + cc;
    X[(int64_t)i * n + col] = (i >= col) ? xs[i - j0][cc] : 0.0;
  }
}

hipError_t launch_cholesky_inv(const double* M, int n, double* L, double* Linv, int* info,
                               hipStream_t s) {
  if (n > kCholMaxN || n < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chol_left, dim3(1), dim3(1024), 0, s, M, n, L, info);
  hipLaunchKernelGGL(k_tri_inv, dim3((n + kCholNB - 1) / kCholNB), dim3(1024), 0, s, L, n, Linv,
                     info);
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
