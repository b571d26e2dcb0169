// Pair screening on gfx950 (arXiv 2110.07670, section "s-MTACE Method":
// orbital pairs with a negligible overlap integral are left out of the
// exchange build).  Two screens feed the same pair mask:
//   * the paper's overlap integral dV sum_r |phi_i phi_j| (an FP64 MFMA
//     product of |Phi| with itself, in dense.hip);
//   * a small learned predictor of the pair energy from the distance of the
//     orbitals' Wannier centres and their spreads (this file).
// Wannier centres and spreads come from Berry-phase moments of each orbital
// density on the periodic cell, z_a = dV sum_r phi(r)^2 exp(2 pi i r_a / L_a):
// centre_a = L_a/(2 pi) arg z_a, spread^2 = sum_a (L_a/(2 pi))^2 (-ln |z_a|^2).
#include <hip/hip_runtime.h>
#include <math.h>

#include "kernels.h"

namespace acex {

// One workgroup per orbital; fixed-order reduction.
__global__ __launch_bounds__(256) void k_moments(const double* __restrict__ phi, int n,
                                                 int64_t npts, double dV, double* __restrict__ z) {
  __shared__ double cs[3][192], sn[3][192];  // per-axis cos/sin(2 pi p / n), n <= 192
  __shared__ double red[6][4];
  const int orb = blockIdx.x, tid = threadIdx.x;
  for (int p = tid; p < n; p += 256) {
    double s, c;
    sincospi(2.0 * (double)p / (double)n, &s, &c);
    for (int a = 0; a < 3; ++a) {
      cs[a][p] = c;
      sn[a][p] = s;
    }
  }
  __syncthreads();
  const double* __restrict__ f = phi + (int64_t)orb * npts;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const int64_t nn = (int64_t)n * n;
  for (int64_t r = tid; r < npts; r += 256) {
    const int px = (int)(r / nn);
    const int64_t rem = r - (int64_t)px * nn;
    const int py = (int)(rem / n);
    const int pz = (int)(rem - (int64_t)py * n);
    const double w = f[r] * f[r];
    acc[0] += w * cs[0][px];
    acc[1] += w * sn[0][px];
    acc[2] += w * cs[1][py];
    acc[3] += w * sn[1][py];
    acc[4] += w * cs[2][pz];
    acc[5] += w * sn[2][pz];
  }
  const int lane = tid & 63, wid = tid >> 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double v = acc[k];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[k][wid] = v;
  }
  __syncthreads();
  if (tid < 6) {
    const double s = ((red[tid][0] + red[tid][1]) + (red[tid][2] + red[tid][3]));
    z[(int64_t)orb * 6 + tid] = dV * s;
  }
}

// feat[i] = (centre_x, centre_y, centre_z, spread) from the moments.
__global__ void k_wannier_features(const double* __restrict__ z, int n_orb, double L0, double L1,
                                   double L2, double* __restrict__ feat) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_orb) return;
  const double L[3] = {L0, L1, L2};
  double s2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double re = z[(int64_t)i * 6 + 2 * a], im = z[(int64_t)i * 6 + 2 * a + 1];
    const double scale = L[a] / (2.0 * M_PI);
    double c = scale * atan2(im, re);
    if (c < 0.0) c += L[a];
    feat[(int64_t)i * 4 + a] = c;
    const double mod2 = re * re + im * im;
    s2 += scale * scale * (-log(mod2));
  }
  feat[(int64_t)i * 4 + 3] = sqrt(s2 > 0.0 ? s2 : 0.0);
}

// MLP 3 -> H -> H -> 1 (ReLU), FP32, one thread per pair (i <= j).
// Inputs: minimum-image centre distance, smaller spread, larger spread,
// standardised by (mean, std).  Output: predicted log10 |e_ij|.
// Weight layout (floats): mean[3] std[3] W1[H][3] b1[H] W2[H][H] b2[H] w3[H] b3.
constexpr int kMlpH = 64;
constexpr int kMlpFloats = 6 + kMlpH * 3 + kMlpH + kMlpH * kMlpH + kMlpH + kMlpH + 1;

__global__ __launch_bounds__(256) void k_mlp_pairs(const double* __restrict__ feat, int n_orb,
                                                   double L0, double L1, double L2,
                                                   const float* __restrict__ wts,
                                                   float* __restrict__ pred) {
  __shared__ float w[kMlpFloats];
  for (int k = threadIdx.x; k < kMlpFloats; k += 256) w[k] = wts[k];
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)n_orb * n_orb) return;
  const int i = (int)(t / n_orb), j = (int)(t % n_orb);
  if (j < i) return;
  const double L[3] = {L0, L1, L2};
  double d2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    double d = feat[(int64_t)i * 4 + a] - feat[(int64_t)j * 4 + a];
    d -= L[a] * rint(d / L[a]);
    d2 += d * d;
  }
  const double si = feat[(int64_t)i * 4 + 3], sj = feat[(int64_t)j * 4 + 3];
  float x[3] = {(float)sqrt(d2), (float)fmin(si, sj), (float)fmax(si, sj)};
  const float* mean = w;
  const float* sd = w + 3;
  const float* W1 = w + 6;
  const float* b1 = W1 + kMlpH * 3;
  const float* W2 = b1 + kMlpH;
  const float* b2 = W2 + kMlpH * kMlpH;
  const float* w3 = b2 + kMlpH;
  const float b3 = w3[kMlpH];
  for (int a = 0; a < 3; ++a) x[a] = (x[a] - mean[a]) / sd[a];
  float h1[kMlpH];
#pragma unroll
  for (int u = 0; u < kMlpH; ++u) {
    const float v = b1[u] + W1[u * 3] * x[0] + W1[u * 3 + 1] * x[1] + W1[u * 3 + 2] * x[2];
    h1[u] = v > 0.f ? v : 0.f;
  }
  float y = b3;
  for (int u = 0; u < kMlpH; ++u) {
    float v = b2[u];
#pragma unroll
    for (int q = 0; q < kMlpH; ++q) v += W2[u * kMlpH + q] * h1[q];
    y += w3[u] * (v > 0.f ? v : 0.f);
  }
  pred[t] = y;
}

hipError_t launch_moments(const double* phi, int n, int n_orb, int64_t npts, double dV, double* z,
                          hipStream_t s) {
  if (n > 192) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_moments, dim3(n_orb), dim3(256), 0, s, phi, n, npts, dV, z);
  return hipGetLastError();
}

hipError_t launch_wannier_features(const double* z, int n_orb, const double* L, double* feat,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_wannier_features, dim3((n_orb + 63) / 64), dim3(64), 0, s, z, n_orb, L[0],
                     L[1], L[2], feat);
  return hipGetLastError();
}

int mlp_weight_count() { return kMlpFloats; }

hipError_t launch_mlp_pairs(const double* feat, int n_orb, const double* L, const float* wts,
                            float* pred, hipStream_t s) {
  const int64_t total = (int64_t)n_orb * n_orb;
  hipLaunchKernelGGL(k_mlp_pairs, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, feat,
                     n_orb, L[0], L[1], L[2], wts, pred);
  return hipGetLastError();
}

}  // namespace acex
