// Per-pair periodic Poisson solves on gfx950 (arXiv 2110.07670, Eq. (3) in
// reciprocal space, accumulated into V_X phi as in Eq. (2)).
//
// One packed transform carries two real pair densities,
// rho = phi_a phi_b + i phi_c phi_d; since the Coulomb kernel K(G) = 4 pi/|G|^2
// is real and even in G, the real and imaginary parts of IFFT(K FFT(rho)) are
// exactly the two pair potentials.
//
// A 3-D transform is done in three passes over a complex grid S[x][y][z]:
//   fwd_yz : pair density, then y and z transforms of each x plane held in
//            LDS (plane kernel), written in "position order";
//   poisson_x : x transform of z-adjacent pencils, multiply by K/N, inverse
//            x transform, in place;
//   inv_yz : inverse y and z transforms of each x plane, natural order.
// Position order: after the forward four-step transform of length N = N1*N2,
// position a + N2*b holds frequency b + N1*a; the inverse consumes it, so no
// reordering pass exists anywhere.  Where a plane does not fit the 160 KiB
// LDS, the y/z stage is split into a row (z) pass and a column (y) pass.
#include <algorithm>
#include <atomic>

#include "fft_core.h"
#include "kernels.h"

namespace acex {

// ------------------------------------------------------------------ sizes

template <typename T>
constexpr int cx_bytes() { return int(sizeof(cx<T>)); }

constexpr int kLdsBytes = 163840;

template <typename T, int N>
constexpr bool plane_ok() {
  return ((long)N * (N + 1) + N) * (long)sizeof(cx<T>) + 64 <= kLdsBytes;
}

// threads per plane workgroup: a multiple of 64 and of N2
template <int N>
constexpr int plane_threads() {
  switch (N) {
    case 16: return 64;
    case 24: return 128;
    case 32: return 256;
    case 40: return 320;
    case 48: return 384;
    case 64: return 512;
    case 80: return 640;
    case 96: return 768;
    case 120: return 640;
    case 128: return 1024;
    case 144: return 576;
    case 160: return 640;
    default: return 768;
  }
}

// threads of the persistent forward plane workgroup: fewer than the inverse
// kernel so that the prefetched orbital values of the next plane fit in
// registers next to the transform working set.
template <int N>
constexpr int fwd_threads() {
  switch (N) {
    default: return plane_threads<N>();
  }
}

// pencils per strided-lines workgroup (consecutive z positions)
template <int N>
constexpr int line_chunk() { return (N % 16 == 0) ? 16 : 8; }

// pencils per y-lines workgroup (large grids): 32 where they divide n
template <int N>
constexpr int yline_chunk() { return N % 32 == 0 ? 32 : line_chunk<N>(); }

template <int N, int C = line_chunk<N>()>
constexpr int line_threads() {
  constexpr int N2 = fft_split<N>::N2;
  constexpr int t = C * N2;
  return ((t + 63) / 64) * 64;
}

// rows per row-pass workgroup (fallback)
constexpr int kRowsPerBlock = 16;
template <int N>
constexpr int row_threads() {
  constexpr int n1 = fft_split<N>::N1, n2 = fft_split<N>::N2;
  constexpr int t = kRowsPerBlock * (n1 > n2 ? n1 : n2);
  return ((t + 63) / 64) * 64;
}

// Streaming (non-temporal) vector load and store of one complex value: for
// scratch data that is written once and read once by a later pass.
template <typename T>
__device__ __forceinline__ cx<T> ld_stream(const cx<T>* p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return {v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void st_stream(cx<T>* p, cx<T> c) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 v = {c.re, c.im};
  __builtin_nontemporal_store(v, reinterpret_cast<v2*>(p));
}

// Workgroup barrier that orders LDS only: waits for this wave's LDS accesses
// (lgkmcnt) but not for its global loads and stores, which stay in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The thread index as a value the compiler cannot see through: in the
// persistent batch loops this keeps the per-thread index arithmetic of an
// item inside the item instead of hoisted out of the loop and held in
// registers across all of them (which cost the loops their occupancy).
template <int NT>
__device__ __forceinline__ int opaque_tid() {
  int t = threadIdx.x;
  __asm__ volatile("" : "+v"(t));
  __builtin_assume(t >= 0 && t < NT);
  return t;
}

template <typename T, int N>
__device__ __forceinline__ T coulomb_k(int kx, int ky, int kz, T g0, T g1, T g2, T kscale) {
  const int mx = kx <= N / 2 ? kx : kx - N;
  const int my = ky <= N / 2 ? ky : ky - N;
  const int mz = kz <= N / 2 ? kz : kz - N;
  const T G2 = g0 * T(mx * mx) + g1 * T(my * my) + g2 * T(mz * mz);
  return G2 > T(0) ? (T(4.0 * kPi) * kscale) / G2 : T(0);
}

// ------------------------------------------------------------------ y/z plane, forward
// Persistent: each workgroup walks items (x, pack) with a stride of the grid
// size, as many workgroups per CU as are resident at once.  The orbital
// values of the next item are loaded into registers while the current item
// is transformed, so their latency hides behind its last steps and its
// stores (on the larger grids one such workgroup fills a CU, so there is no
// second workgroup to overlap with): FP32 ones once the z transform is done,
// FP64 ones after the first y step (measured per precision: issued after the
// z transform, FP32 passes take 8% (96^3) and 10% (128^3) less time, the FP64
// one 3% more).  Barriers order LDS only, leaving these loads and the stores
// in flight.
//
// Every pack carries pairs (a, b) and (a, d) that share their first orbital,
// or the single pair (a, b) (c = d = -1): rho = phi_a (phi_b + i phi_d).
template <typename T, int N>
__device__ __forceinline__ void plane_item(int item, int npack, int& x, int& p) {
  const int xcd = item & 7;
  const int q = item >> 3;
  const int xh = q / npack;
  p = q - xh * npack;
  x = xcd + 8 * xh;
}

// ZXY: write the result as S[kz][x][ky] (the three-pass schedule, whose middle
// pass reads one kz plane contiguously) instead of S[x][ky][kz].
// The loop of one forward-plane workgroup of NT threads over the items that
// the source Q hands it: Q::first() (called by every thread), Q::ask() at the
// top of an item and Q::post() before its first barrier (a queue fetches
// the next item there), Q::next(item) after that barrier, Q::more(item), and
// Q::at(item, phi, pack, out, x): the orbitals, the pack, the transform's
// scratch grid and the plane x of an item.  lds holds N (N + 1) values,
// stw N.
template <typename T, int N, bool ZXY, int NT, class Q>
__device__ __forceinline__ void plane_fwd_loop(Q& q, const cx<T>* __restrict__ tw, int64_t npts,
                                               cx<T>* __restrict__ lds, cx<T>* __restrict__ stw) {
  constexpr int N1 = fft_split<N>::N1, N2 = fft_split<N>::N2, P = N + 1;
  constexpr int Q1 = (N * N2 + NT - 1) / NT;  // z-step-1 tasks per thread
  static_assert(NT % N2 == 0, "threads must be a multiple of N2");
  constexpr bool EARLY = sizeof(T) == 4;  // where the next item's loads are issued
  const int tid = threadIdx.x;
  const int t2 = tid % N2;
  for (int i = tid; i < N; i += NT) stw[i] = tw[(i % N2) * (i / N2)];  // stw[k1 N2 + t2] = w^(t2 k1)
  int item = q.first();
  __syncthreads();

  // row of z-step-1 task group g: with eight lanes per row, the two halves of
  // each 16 lanes take rows 8 apart (offset 8 on the odd pitch: distinct
  // banks) instead of adjacent rows; a permutation within blocks of 16 rows
  auto zrow = [](int g) __attribute__((always_inline)) {
    if constexpr (N2 == 8 && N % 16 == 0)
      return (g & ~15) | ((g & 1) << 3) | ((g >> 1) & 7);
    else
      return g;
  };
  // phi_a, phi_b, phi_d of one item at this thread's z-step-1 elements
  T fa[Q1][N1], fb[Q1][N1], fd[Q1][N1];
  auto fetch = [&](int it) __attribute__((always_inline)) {
    const T* phi;
    Pack pk;
    cx<T>* o;
    int x;
    q.at(it, phi, pk, o, x);
    const int64_t plane = (int64_t)x * N * N;
    const T* __restrict__ pa = phi + (int64_t)pk.a * npts + plane;
    const T* __restrict__ pb = phi + (int64_t)pk.b * npts + plane;
    const T* __restrict__ pd = phi + (int64_t)(pk.c >= 0 ? pk.d : pk.b) * npts + plane;
#pragma unroll
    for (int q = 0; q < Q1; ++q) {
      const int task = tid + q * NT;
      const int y = zrow((task < N * N2 ? task : 0) / N2);
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) {
        const int off = y * N + t2 + N2 * j1;
        fa[q][j1] = pa[off];
        fb[q][j1] = pb[off];
        fd[q][j1] = pd[off];
      }
    }
  };

  if (q.more(item)) fetch(item);
  while (q.more(item)) {
    const T* phi_unused;
    Pack pk;
    cx<T>* S;
    int x;
    q.at(item, phi_unused, pk, S, x);
    q.ask();
    const T dmask = pk.c >= 0 ? T(1) : T(0);
    const int64_t plane = (int64_t)x * N * N;
    // z step 1: tasks (y, t2), t2 fastest (coalesced along z)
#pragma unroll
    for (int q = 0; q < Q1; ++q) {
      const int task = tid + q * NT;
      if (task < N * N2) {
        const int y = zrow(task / N2);
        cx<T> v[N1];
#pragma unroll
        for (int j1 = 0; j1 < N1; ++j1)
          v[j1] = {fa[q][j1] * fb[q][j1], fa[q][j1] * (dmask * fd[q][j1])};
        dft<N1, false>(v);
#pragma unroll
        for (int k1 = 1; k1 < N1; ++k1) v[k1] = cmul(v[k1], stw[k1 * N2 + t2]);
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) lds[y * P + t2 + N2 * k1] = v[k1];
      }
    }
    q.post();
    lds_barrier();
    const int next = q.next(item);
    // z step 2: tasks (y, k1), y fastest
#pragma unroll 1
    for (int task = tid; task < N * N1; task += NT) {
      const int y = task % N, k1 = task / N;
      cx<T> v[N2];
#pragma unroll
      for (int t = 0; t < N2; ++t) v[t] = lds[y * P + t + N2 * k1];
      dft<N2, false>(v);
#pragma unroll
      for (int t = 0; t < N2; ++t) lds[y * P + t + N2 * k1] = v[t];
    }
    if constexpr (EARLY) {
      __builtin_amdgcn_sched_barrier(0);  // keep the prefetch below the z-step-2 work
      if (q.more(next)) fetch(next);
      __builtin_amdgcn_sched_barrier(0);
    }
    lds_barrier();
    // y step 1: tasks (pz, u2), pz fastest (LDS only: consecutive threads on
    // consecutive pz keep the column accesses of the odd-pitch rows apart)
    for (int task = tid; task < N * N2; task += NT) {
      const int pz = task % N, u2 = task / N;
      cx<T> v[N1];
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) v[j1] = lds[(u2 + N2 * j1) * P + pz];
      dft<N1, false>(v);
#pragma unroll
      for (int k1 = 1; k1 < N1; ++k1) v[k1] = cmul(v[k1], stw[k1 * N2 + u2]);
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) lds[(u2 + N2 * k1) * P + pz] = v[k1];
    }
    if constexpr (!EARLY) {
      __builtin_amdgcn_sched_barrier(0);  // keep the prefetch below the y-step-1 work
      if (q.more(next)) fetch(next);
      __builtin_amdgcn_sched_barrier(0);
    }
    lds_barrier();
    if constexpr (!ZXY) {
      // y step 2 -> global: tasks (pz, k1), pz fastest (coalesced)
      cx<T>* __restrict__ out = S + plane;
#pragma unroll 1
      for (int task = tid; task < N * N1; task += NT) {
        const int pz = task % N, k1 = task / N;
        cx<T> v[N2];
#pragma unroll
        for (int t = 0; t < N2; ++t) v[t] = lds[(t + N2 * k1) * P + pz];
        dft<N2, false>(v);
#pragma unroll
        for (int t = 0; t < N2; ++t) out[(t + N2 * k1) * N + pz] = v[t];
      }
    } else {
      // y step 2 in place, then the plane leaves transposed: S[kz][x][ky],
      // consecutive threads on consecutive ky (column reads of the odd-pitch
      // LDS rows are conflict-free), with streaming stores (the middle pass
      // reads each value once)
#pragma unroll 1
      for (int task = tid; task < N * N1; task += NT) {
        const int pz = task % N, k1 = task / N;
        cx<T> v[N2];
#pragma unroll
        for (int t = 0; t < N2; ++t) v[t] = lds[(t + N2 * k1) * P + pz];
        dft<N2, false>(v);
#pragma unroll
        for (int t = 0; t < N2; ++t) lds[(t + N2 * k1) * P + pz] = v[t];
      }
      lds_barrier();
      cx<T>* __restrict__ out = S + (int64_t)x * N;
#pragma unroll 1
      for (int e = tid; e < N * N; e += NT) {
        const int ky = e % N, pz = e / N;
        st_stream(&out[(int64_t)pz * N * N + ky], lds[ky * P + pz]);
      }
    }
    lds_barrier();
    item = next;
  }
}

// Items of one tile: (x, pack) in plane_item order, strided by the grid.
template <typename T, int N>
struct FwdTile {
  const T* phi;
  const Pack* packs;
  cx<T>* S;
  int npack;
  int64_t npts;
  __device__ __forceinline__ int first() const { return blockIdx.x; }
  __device__ __forceinline__ void ask() {}
  __device__ __forceinline__ void post() {}
  __device__ __forceinline__ int next(int it) const { return it + gridDim.x; }
  __device__ __forceinline__ bool more(int it) const { return it < N * npack; }
  __device__ __forceinline__ void at(int it, const T*& f, Pack& pk, cx<T>*& o, int& x) const {
    int p;
    plane_item<T, N>(it, npack, x, p);
    f = phi;
    pk = packs[p];
    o = S + (int64_t)p * npts;
  }
};

template <typename T, int N, bool ZXY>
__global__ __launch_bounds__(fwd_threads<N>()) void k_plane_fwd(
    const T* __restrict__ phi, const Pack* __restrict__ packs, const cx<T>* __restrict__ tw,
    cx<T>* __restrict__ S, int npack, int64_t npts) {
  __shared__ cx<T> lds[N * (N + 1)];
  __shared__ cx<T> stw[N];
  FwdTile<T, N> q{phi, packs, S, npack, npts};
  plane_fwd_loop<T, N, ZXY, fwd_threads<N>()>(q, tw, npts, lds, stw);
}

// ------------------------------------------------------------------ y/z plane, inverse
template <typename T, int N>
__global__ __launch_bounds__(plane_threads<N>()) void k_plane_inv(
    cx<T>* __restrict__ S, const cx<T>* __restrict__ tw, int npack, int64_t npts) {
  constexpr int N1 = fft_split<N>::N1, N2 = fft_split<N>::N2, P = N + 1;
  constexpr int NT = plane_threads<N>();
  __shared__ cx<T> lds[N * P];
  const int bid = blockIdx.x;
  const int x = bid % N, p = bid / N;
  const int tid = threadIdx.x;
  const int t2 = tid % N2;
  cx<T> w[N1];
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) w[k1] = tw[t2 * k1];
  cx<T>* __restrict__ io = S + (int64_t)p * npts + (int64_t)x * N * N;

  // y step 2 inverse: global positions -> LDS, tasks (pz, k1), pz fastest
  for (int task = tid; task < N * N1; task += NT) {
    const int pz = task % N, k1 = task / N;
    cx<T> v[N2];
#pragma unroll
    for (int t = 0; t < N2; ++t) v[t] = io[(t + N2 * k1) * N + pz];
    dft<N2, true>(v);
#pragma unroll
    for (int t = 0; t < N2; ++t) lds[(t + N2 * k1) * P + pz] = v[t];
  }
  __syncthreads();
  // y step 1 inverse: tasks (pz, t2)
  for (int task = tid; task < N * N2; task += NT) {
    const int pz = task / N2;
    cx<T> v[N1];
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) v[k1] = cmulc(lds[(t2 + N2 * k1) * P + pz], w[k1]);
    dft<N1, true>(v);
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) lds[(t2 + N2 * j1) * P + pz] = v[j1];
  }
  __syncthreads();
  // z step 2 inverse: tasks (y, k1), y fastest
  for (int task = tid; task < N * N1; task += NT) {
    const int y = task % N, k1 = task / N;
    cx<T> v[N2];
#pragma unroll
    for (int t = 0; t < N2; ++t) v[t] = lds[y * P + t + N2 * k1];
    dft<N2, true>(v);
#pragma unroll
    for (int t = 0; t < N2; ++t) lds[y * P + t + N2 * k1] = v[t];
  }
  __syncthreads();
  // z step 1 inverse -> global natural order: tasks (y, t2)
  for (int task = tid; task < N * N2; task += NT) {
    const int y = task / N2;
    cx<T> v[N1];
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) v[k1] = cmulc(lds[y * P + t2 + N2 * k1], w[k1]);
    dft<N1, true>(v);
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) io[y * N + t2 + N2 * j1] = v[j1];
  }
}

// The same inverse, a slab of kz positions at a time: per slab the inverse
// y transform of its ZC columns and the in-slab inverse z step; each thread
// keeps its share of the first slab's z-step outputs in registers, and after
// the second slab the first inverse z step runs on the held values and the
// plane leaves in natural order, in place (every slab has been read by
// then).  Half a plane of LDS and 512 threads, so that two workgroups share
// a CU; the same values, bit for bit, as the plane kernel (inv_slabs says
// where it is used).
template <typename T, int N>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_slab_inv(
    cx<T>* __restrict__ S, const cx<T>* __restrict__ tw, int npack, int64_t npts) {
  constexpr int N1 = fft_split<N>::N1, N2 = fft_split<N>::N2;
  constexpr int SL = 2, ZC = N / SL, K1S = ZC / N2, PZ = ZC + 1;
  constexpr int NT = 512;
  constexpr int Q = (N * N2 + NT - 1) / NT;  // final-step tasks (y, t2) per thread
  static_assert(N % SL == 0 && ZC % N2 == 0, "whole second-step blocks per slab");
  __shared__ cx<T> lds[N * PZ];
  __shared__ cx<T> stw[N];
  const int bid = blockIdx.x;
  const int x = bid % N, p = bid / N;
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NT) stw[i] = tw[(i % N2) * (i / N2)];
  cx<T>* __restrict__ io = S + (int64_t)p * npts + (int64_t)x * N * N;
  cx<T> hold[Q][K1S];
  sfor<0, SL>([&](auto sc) {
    constexpr int sl = decltype(sc)::value;
    __syncthreads();  // twiddles in place / the previous slab read out of LDS
    // y step 2 inverse: the slab's columns -> LDS, tasks (pz, k1), pz fastest
    for (int task = tid; task < ZC * N1; task += NT) {
      const int pz = task % ZC, k1 = task / ZC;
      cx<T> v[N2];
#pragma unroll
      for (int t = 0; t < N2; ++t) v[t] = io[(int64_t)(t + N2 * k1) * N + sl * ZC + pz];
      dft<N2, true>(v);
#pragma unroll
      for (int t = 0; t < N2; ++t) lds[(t + N2 * k1) * PZ + pz] = v[t];
    }
    __syncthreads();
    // y step 1 inverse to natural y: tasks (pz, t2), pz fastest
    for (int task = tid; task < ZC * N2; task += NT) {
      const int pz = task % ZC, t2 = task / ZC;
      cx<T> v[N1];
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) v[k1] = cmulc(lds[(t2 + N2 * k1) * PZ + pz], stw[k1 * N2 + t2]);
      dft<N1, true>(v);
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) lds[(t2 + N2 * j1) * PZ + pz] = v[j1];
    }
    __syncthreads();
    // z step 2 inverse within the slab's blocks: tasks (y, k), y fastest
    for (int task = tid; task < N * K1S; task += NT) {
      const int y = task % N, k = task / N;
      cx<T> v[N2];
#pragma unroll
      for (int t = 0; t < N2; ++t) v[t] = lds[y * PZ + t + N2 * k];
      dft<N2, true>(v);
#pragma unroll
      for (int t = 0; t < N2; ++t) lds[y * PZ + t + N2 * k] = v[t];
    }
    __syncthreads();
    if constexpr (sl == 0) {
      // this thread's tasks (y, t2), t2 fastest: the slab's K1S values
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int task = tid + q * NT;
        if (task < N * N2) {
          const int t2 = task % N2, y = task / N2;
#pragma unroll
          for (int k = 0; k < K1S; ++k) hold[q][k] = lds[y * PZ + t2 + N2 * k];
        }
      }
    } else {
      // z step 1 inverse -> global, natural order: tasks (y, t2)
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int task = tid + q * NT;
        if (task < N * N2) {
          const int t2 = task % N2, y = task / N2;
          cx<T> v[N1];
#pragma unroll
          for (int k1 = 0; k1 < N1; ++k1) {
            const cx<T> u = k1 < K1S ? hold[q][k1 < K1S ? k1 : 0] : lds[y * PZ + t2 + N2 * (k1 - K1S)];
            v[k1] = cmulc(u, stw[k1 * N2 + t2]);
          }
          dft<N1, true>(v);
#pragma unroll
          for (int j1 = 0; j1 < N1; ++j1) io[(int64_t)y * N + t2 + N2 * j1] = v[j1];
        }
      }
    }
  });
}

// Full, unmasked tile: the schedule packs the pairs of each row a two per
// transform, (a, b) and (a, b + 1), with a row's odd leftover alone, so the
// pair -> (transform, half) map is known at compile time and each transform
// is read once as one complex value.
template <int B, bool DIAG>
constexpr int row_packs(int a) { return DIAG ? (B - a + 1) / 2 : B / 2; }
template <int B, bool DIAG>
constexpr int row_pack0(int a) {
  int s = 0;
  for (int r = 0; r < a; ++r) s += row_packs<B, DIAG>(r);
  return s;
}

// ------------------------------------------------------------------ three-pass schedule
// For full tiles where a plane fits LDS the solve takes three passes
// instead of four:
//   k_plane_fwd<ZXY> : pair density, y and z transforms, written S[kz][x][ky];
//   k_plane_mid      : one kz plane [x][ky] (contiguous): forward x, multiply
//                      by K/N, inverse x, inverse y, written S[kz][x][y];
//   k_zinv_acc       : inverse z of a tile's transforms at the points
//                      (x, y0..y0+7, all z), folded straight into W.
// The potentials never make a round trip through HBM in real space.
// The work of one middle-pass workgroup of NT threads: item bid = (kz
// position, transform); lds holds N (N + 1) values, stw N.
template <typename T, int N, int NT, bool LOOP = false>
__device__ __forceinline__ void plane_mid_item(cx<T>* __restrict__ S, const cx<T>* __restrict__ tw,
                                               int64_t npts, T g0, T g1, T g2, T kscale, int bid,
                                               cx<T>* __restrict__ lds, cx<T>* __restrict__ stw) {
  constexpr int N1 = fft_split<N>::N1, N2 = fft_split<N>::N2, P = N + 1;
  const int pz = bid % N, p = bid / N;
  const int tid = LOOP ? opaque_tid<NT>() : (int)threadIdx.x;
  for (int i = tid; i < N; i += NT) stw[i] = tw[(i % N2) * (i / N2)];  // stw[k1 N2 + t2] = w^(t2 k1)
  cx<T>* __restrict__ io = S + (int64_t)p * npts + (int64_t)pz * N * N;
  const int kz = freq_of_pos<N>(pz);
  __syncthreads();

  // x forward step 1: tasks (py, t2), py fastest (coalesced rows)
  for (int task = tid; task < N * N2; task += NT) {
    const int py = task % N, t2 = task / N;
    cx<T> v[N1];
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) v[j1] = io[(t2 + N2 * j1) * N + py];
    dft<N1, false>(v);
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) v[k1] = cmul(v[k1], stw[k1 * N2 + t2]);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) lds[(t2 + N2 * k1) * P + py] = v[k1];
  }
  __syncthreads();
  // x forward step 2, Coulomb multiply, x inverse step 2: tasks (py, k1)
  for (int task = tid; task < N * N1; task += NT) {
    const int py = task % N, k1 = task / N;
    const int ky = freq_of_pos<N>(py);
    cx<T> v[N2];
#pragma unroll
    for (int t = 0; t < N2; ++t) v[t] = lds[(t + N2 * k1) * P + py];
    dft<N2, false>(v);
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2)
      v[k2] = scale(v[k2], coulomb_k<T, N>(k1 + N1 * k2, ky, kz, g0, g1, g2, kscale));
    dft<N2, true>(v);
#pragma unroll
    for (int t = 0; t < N2; ++t) lds[(t + N2 * k1) * P + py] = v[t];
  }
  __syncthreads();
  // x inverse step 1 to natural x, in place: tasks (py, t2)
  for (int task = tid; task < N * N2; task += NT) {
    const int py = task % N, t2 = task / N;
    cx<T> v[N1];
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) v[k1] = cmulc(lds[(t2 + N2 * k1) * P + py], stw[k1 * N2 + t2]);
    dft<N1, true>(v);
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) lds[(t2 + N2 * j1) * P + py] = v[j1];
  }
  __syncthreads();
  // y inverse step 2 along the rows: tasks (x, k1), x fastest
  for (int task = tid; task < N * N1; task += NT) {
    const int x = task % N, k1 = task / N;
    cx<T> v[N2];
#pragma unroll
    for (int t = 0; t < N2; ++t) v[t] = lds[x * P + t + N2 * k1];
    dft<N2, true>(v);
#pragma unroll
    for (int t = 0; t < N2; ++t) lds[x * P + t + N2 * k1] = v[t];
  }
  __syncthreads();
  // y inverse step 1 -> global, natural y: tasks (x, t2), t2 fastest; with
  // eight lanes per row the two halves of each 16 lanes take rows 8 apart
  // (distinct banks on the odd pitch), a permutation within blocks of 16 rows
  for (int task = tid; task < N * N2; task += NT) {
    const int t2 = task % N2, g = task / N2;
    const int x = (N2 == 8 && N % 16 == 0) ? ((g & ~15) | ((g & 1) << 3) | ((g >> 1) & 7)) : g;
    cx<T> v[N1];
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) v[k1] = cmulc(lds[x * P + t2 + N2 * k1], stw[k1 * N2 + t2]);
    dft<N1, true>(v);
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) io[x * N + t2 + N2 * j1] = v[j1];
  }
}

template <typename T, int N>
__global__ __launch_bounds__(plane_threads<N>()) void k_plane_mid(
    cx<T>* __restrict__ S, const cx<T>* __restrict__ tw, int npack, int64_t npts, T g0, T g1,
    T g2, T kscale) {
  __shared__ cx<T> lds[N * (N + 1)];
  __shared__ cx<T> stw[N];
  plane_mid_item<T, N, plane_threads<N>()>(S, tw, npts, g0, g1, g2, kscale, blockIdx.x, lds, stw);
}

// ------------------------------------------------------------------ slab sizes
// The fewest slabs that fit (more slabs, for more workgroups per CU,
// measured slower: the recomputed first step and orbital loads grow with
// the slab count).
template <typename T, int N>
constexpr int slab_count() {
  constexpr int N2 = fft_split<N>::N2;
  for (int sl = 2; sl <= 8; ++sl)
    if (N % sl == 0 && (N / sl) % N2 == 0 &&
        ((long)N * (N / sl + 1) + N) * (long)sizeof(cx<T>) + 64 <= kLdsBytes)
      return sl;
  return 0;
}

template <typename T, int N>
constexpr bool slab_ok() { return !plane_ok<T, N>() && slab_count<T, N>() > 0; }

// A workgroup takes SPW consecutive slabs of its plane from one first step:
// the outputs of its first slab go to LDS, those of the others wait in
// registers (at most 72 per thread with 512 FP64 threads, 48 with 768, 32
// with 1024 FP32 threads: beyond that the kernels spill).  The first step is
// recomputed SL / SPW times per plane.  On grids whose plane fits LDS (the
// two-slab forward pass below) FP32 workgroups have 512 threads too, so that
// two of them share a CU.
template <typename T, int N, int SPW>
constexpr int slab_threads() {
  constexpr int SL = slab_count<T, N>();
  if constexpr (sizeof(T) == 4) return plane_ok<T, N>() ? 512 : 1024;
  else return SPW == SL ? 512 : 768;
}

template <typename T, int N>
constexpr int slab_spw() {
  constexpr int N2 = fft_split<N>::N2, SL = slab_count<T, N>();
  if (SL == 0) return 1;
  constexpr int K1S = N / SL / N2;
  for (int spw = SL; spw > 1; --spw) {
    if (SL % spw) continue;
    const int nt = sizeof(T) == 4 ? 1024 : (spw == SL ? 512 : 768);
    const int q = (N * N2 + nt - 1) / nt;
    const int cap = sizeof(T) == 4 ? 32 : (spw == SL ? 72 : 48);
    if ((spw - 1) * K1S * q * int(sizeof(cx<T>) / 4) <= cap) return spw;
  }
  return 1;
}

template <typename T, int N>
constexpr bool slab3_ok() {
  return slab_ok<T, N>() && slab_spw<T, N>() == slab_count<T, N>();
}

// Plane-fitting grids from 48^3 up also run the forward pass as two slabs
// (both layouts): one 512-thread workgroup per plane takes both slabs from one
// first step, holding the second slab's first-step outputs in registers;
// half a plane of LDS lets two or more such workgroups share a CU, so that
// one's transform steps overlap another's loads and stores.  (A plane
// workgroup's waves all move through the same phase between barriers, so
// its memory traffic barely overlaps its arithmetic, and the large planes
// leave room for one per CU.)  Measured, one 128-transform launch, slabs
// against planes: FP64 96^3 551 / 606 us, 80^3 333 / 381, 64^3 118 / 125,
// 48^3 58 / 71; FP32 128^3 752 / 864, 120^3 734 / 967 (both with the plane
// kernel's earlier FP32 prefetch placement), 96^3 300 / 341, 80^3 122 / 198,
// 64^3 62 / 65, 48^3 52 / 57.  Per build, the forward pass of the 96^3 FP64
// build of 128 orbitals 17.4 -> 16.1 ms, of the 128^3 FP32 build of 256
// orbitals 105 -> 101 ms.  In the four-pass layout S[x][ky][kz]: FP64 96^3
// 510 / 668 us, 64^3 100 / 184; FP32 128^3 657 / 804, 96^3 271 / 352, 48^3
// 49 / 58.
template <typename T, int N>
constexpr bool fwd_slabs() {
  return plane_ok<T, N>() && N >= 48 && slab_count<T, N>() == 2;
}

// Rows of y per inverse-z workgroup (one workgroup: rows x N points).  Eight
// rows read 128 B (FP64) of each scratch row per transform; four FP64 rows
// (64 B segments, two workgroups per CU) measured slower, even with the two
// halves of each segment dispatched back to back on one XCD.  Grids past
// 128 (more than 1024 points in eight rows) take four.
// ROWS: the large-grid schedule, whose scratch is S[x][y][kz] (each z row
// contiguous, so four rows per workgroup read whole rows).
template <typename T, int N, bool ROWS = false>
constexpr int zinv_rows() { return (ROWS || 8 * N > 1024) ? 4 : 8; }

template <typename T, int N, bool ROWS = false>
constexpr int zinv_threads() { return zinv_rows<T, N, ROWS>() * N; }

template <typename T, int N, int B, bool ROWS>
constexpr bool zinv_fits() {
  return zinv_threads<T, N, ROWS>() <= 1024 &&
         ((long)(B / 2) * zinv_rows<T, N, ROWS>() * (N + 1) + N) * (long)sizeof(cx<T>) + 64 <=
             kLdsBytes;
}

// The plane form (scratch S[kz][x][y]) serves the three-pass schedules, of
// plane-fitting grids and of slab grids; the row form (S[x][y][kz]) the
// large-grid four-pass one where those do not apply.
// On slab grids the plane form also needs its registers: above 768 threads
// (128 registers each) the block-16 form spills, so there only block 8; and
// eight rows per workgroup (at 160^3 FP32 the four-row form, 32-byte
// segments, took 1.44 s per 512-orbital build against 0.83 s for the row
// form, more than the middle pass saves).
template <typename T, int N, int B, bool ROWS = false>
constexpr bool zinv_ok() {
  constexpr bool three =
      zinv_fits<T, N, B, false>() &&
      (plane_ok<T, N>() || (slab3_ok<T, N>() && zinv_rows<T, N, false>() == 8 &&
                            (B == 8 || zinv_threads<T, N, false>() <= 768)));
  if constexpr (!ROWS) return three;
  else return !plane_ok<T, N>() && !three && zinv_fits<T, N, B, true>();
}

// A workgroup owns the points (x, y0 .. y0 + YC - 1, all z) of a full B x B tile and
// walks its rows a: the transforms of row a (pairs (a, b0) and (a, b0 + 1))
// are inverse-transformed along z in LDS; then each thread, one point, folds
// them into the W sums it keeps in registers.  Off-diagonal tiles: W_a is
// updated once per row (sum_b v_ab phi_b) and the B sums of W_J at the end;
// diagonal tiles: all B sums at the end.  Fixed order, no atomics.
// The work of one such workgroup of NT >= YC N threads (threads past YC N
// take part in the transforms and barriers but own no point): item bid =
// (x, y0); lds holds B / 2 YC (N + 1) values, stw N.
template <typename T, int N, int B, bool DIAG, bool ROWS, int NT, bool LOOP = false>
__device__ __forceinline__ void zinv_item(const cx<T>* __restrict__ S,
                                          const cx<T>* __restrict__ tw, const T* __restrict__ phi,
                                          double* __restrict__ W, const int* __restrict__ orbs,
                                          double alpha, int64_t npts, int bid,
                                          cx<T>* __restrict__ lds, cx<T>* __restrict__ stw) {
  constexpr int N1 = fft_split<N>::N1, N2 = fft_split<N>::N2, P = N + 1;
  constexpr int G = B / 2, YC = zinv_rows<T, N, ROWS>();
  constexpr int ACT = zinv_threads<T, N, ROWS>();  // threads that own a point
  static_assert(NT >= ACT, "a thread per point");
  // kz positions and rows in the scratch: S[kz][x][y] (kz stride N^2, rows
  // adjacent) or, with ROWS, S[x][y][kz] (kz adjacent, rows N apart)
  constexpr int64_t KS = ROWS ? 1 : (int64_t)N * N;
  constexpr int64_t CS = ROWS ? N : 1;
  static_assert(B % 2 == 0, "rows of a full tile pack evenly");
  const int tid = LOOP ? opaque_tid<NT>() : (int)threadIdx.x;
  const bool act = NT == ACT || tid < ACT;
  int x, y0;
  // workgroups per 128-byte scratch segment (FP32: two)
  constexpr int H = YC * int(sizeof(cx<T>)) < 128 ? 128 / (YC * int(sizeof(cx<T>))) : 1;
  if constexpr (!ROWS && H > 1 && N % (H * YC) == 0) {
    // the H workgroups sharing a segment run back to back on one XCD
    // (workgroup b runs on XCD b mod 8), so the later ones find the lines in
    // L2; only where whole segments tile the y rows (else the plain order)
    const int g = bid >> 3, xcd = bid & 7;
    const int seg = (g / H) * 8 + xcd;
    y0 = (seg % (N / (H * YC))) * (H * YC) + (g % H) * YC;
    x = seg / (N / (H * YC));
  } else {
    y0 = (bid % (N / YC)) * YC;
    x = bid / (N / YC);
  }
  for (int i = tid; i < N; i += NT) stw[i] = tw[(i % N2) * (i / N2)];  // stw[k1 N2 + t2] = w^(t2 k1)
  // this thread's point for the W update (consecutive threads: consecutive
  // z); a thread without one reads point (x, y0, z) and writes nothing
  const int c = act ? tid / N : 0, z = tid % N;
  const int64_t r = ((int64_t)x * N + y0 + c) * N + z;
  const cx<T>* __restrict__ sx =
      S + (ROWS ? ((int64_t)x * N + y0) * N : (int64_t)x * N + y0);  // + pack npts + c CS + pz KS
  // step-2 task -> (row, k1, transform): row fastest for S[kz][x][y] (the
  // rows' values at one kz are adjacent), k1 fastest with ROWS (a row's
  // positions are adjacent)
  auto task_map = [&](int task, int& cc, int& k1, int& m) __attribute__((always_inline)) {
    if constexpr (ROWS) {
      k1 = task % N1;
      cc = (task / N1) % YC;
    } else {
      cc = task % YC;
      k1 = (task / YC) % N1;
    }
    m = task / (YC * N1);
  };

  // W is read and written with streaming accesses: the rows of a W update
  // are far apart in time, and kept out of the caches they leave room for
  // the orbital rows that the next tile's forward pass reads again (measured:
  // forward pass 19.9 to 17.5 ms per build at 96^3).  The orbitals come in
  // the bulk precision (with FP32 transforms, the FP32 copy the forward pass
  // reads: half the bytes and registers; the products and sums stay FP64).
  // off-diagonal: ph = phi_J, acc = W_J sums; diagonal: the tile's B orbitals
  T ph[B];
  double acc[B];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    ph[b] = phi[(int64_t)orbs[(DIAG ? 0 : B) + b] * npts + r];
    acc[b] = 0.0;
  }
  __syncthreads();

  // inverse z step 2, tasks (c, k1, m) with c fastest, Q2 per thread.  With
  // FP32 transforms the loads of row a + 1 are issued before row a's W update
  // so that they are in flight while it runs (the barriers order LDS only);
  // with FP64 ones the registers for that do not fit next to the W sums
  // (measured slower with the spills) and each row loads at its start, with
  // streaming loads in the plane form (4% faster at 96^3; the row form and
  // the prefetched FP32 form measured slower with them: 42 to 77 ms per
  // build at 120^3).  With
  // the prefetch the four-step twiddles are applied at the end of step 2,
  // which keeps step 1 light; without it, at the start of step 1.
  constexpr int T2MAX = YC * N1 * G;
  // every thread has exactly one step-2 task in every row: no bounds test
  constexpr bool EXACT = !DIAG && T2MAX == NT;
  constexpr bool PF = sizeof(T) == 4;
  constexpr int Q2 = PF ? (T2MAX + NT - 1) / NT : 1;
  cx<T> pre[Q2][N2];
  auto fetch = [&](int q0n, int gan) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < Q2; ++q) {
      const int task = tid + q * NT;
      if (EXACT || task < YC * N1 * gan) {
        int cc, k1, m;
        task_map(task, cc, k1, m);
        const cx<T>* __restrict__ src = sx + (int64_t)(q0n + m) * npts + cc * CS;
#pragma unroll
        for (int t = 0; t < N2; ++t) pre[q][t] = src[(int64_t)(t + N2 * k1) * KS];
      }
    }
  };
  if constexpr (PF) fetch(0, DIAG ? (B + 1) / 2 : G);

  int q0 = 0;  // first transform of row a
#pragma unroll 1
  for (int a = 0; a < B; ++a) {
    const int ga = DIAG ? (B - a + 1) / 2 : G;  // transforms in row a
    const int64_t oa = (int64_t)orbs[a] * npts + r;
    T phA = T(0);
    double wA = 0.0;
    if constexpr (!DIAG) {
      phA = phi[oa];
      wA = __builtin_nontemporal_load(&W[oa]);
    }
    if constexpr (PF) {
#pragma unroll
      for (int q = 0; q < Q2; ++q) {
        const int task = tid + q * NT;
        if (EXACT || task < YC * N1 * ga) {
          int cc, k1, m;
          task_map(task, cc, k1, m);
          dft<N2, true>(pre[q]);
          lds[(m * YC + cc) * P + N2 * k1] = pre[q][0];
#pragma unroll
          for (int t = 1; t < N2; ++t)
            lds[(m * YC + cc) * P + t + N2 * k1] = cmulc(pre[q][t], stw[k1 * N2 + t]);
        }
      }
    } else {
      for (int task = tid; task < YC * N1 * ga; task += NT) {
        int cc, k1, m;
        task_map(task, cc, k1, m);
        const cx<T>* __restrict__ src = sx + (int64_t)(q0 + m) * npts + cc * CS;
        cx<T> v[N2];
#pragma unroll
        for (int t = 0; t < N2; ++t)
          v[t] = ROWS ? src[(int64_t)(t + N2 * k1) * KS] : ld_stream(&src[(int64_t)(t + N2 * k1) * KS]);
        dft<N2, true>(v);
#pragma unroll
        for (int t = 0; t < N2; ++t) lds[(m * YC + cc) * P + t + N2 * k1] = v[t];
      }
    }
    lds_barrier();
    // inverse z step 1 to natural z: tasks (t2, c, m), t2 fastest; in the
    // plane form then m (the row offset of a transform, 8 rows of the odd
    // pitch, keeps the two halves of each 16 lanes on distinct banks), in the
    // row form then c
    for (int task = tid; task < YC * N2 * ga; task += NT) {
      const int t2 = task % N2;
      const int cc = ROWS ? (task / N2) % YC : task / (N2 * ga);
      const int m = ROWS ? task / (N2 * YC) : (task / N2) % ga;
      cx<T> v[N1];
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) {
        v[k1] = lds[(m * YC + cc) * P + t2 + N2 * k1];
        if constexpr (!PF) v[k1] = cmulc(v[k1], stw[k1 * N2 + t2]);
      }
      dft<N1, true>(v);
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) lds[(m * YC + cc) * P + t2 + N2 * j1] = v[j1];
    }
    lds_barrier();
    if constexpr (PF) {
      __builtin_amdgcn_sched_barrier(0);
      if (a + 1 < B) fetch(q0 + ga, DIAG ? (B - a) / 2 : G);
      __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (!DIAG) {
      double accA = 0.0;
#pragma unroll
      for (int m = 0; m < G; ++m) {
        const cx<T> vv = lds[(m * YC + c) * P + z];
        const double v0 = double(vv.re), v1 = double(vv.im);
        accA += v0 * ph[2 * m] + v1 * ph[2 * m + 1];
        acc[2 * m] += v0 * phA;
        acc[2 * m + 1] += v1 * phA;
      }
      if (act) __builtin_nontemporal_store(wA - alpha * accA, &W[oa]);
    } else {
      // row a at compile time, so every register index is static
      sfor<0, B>([&](auto ac) {
        constexpr int ar = decltype(ac)::value;
        if (a == ar) {
          sfor<0, row_packs<B, true>(ar)>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            constexpr int b0 = ar + 2 * m;
            const cx<T> vv = lds[(m * YC + c) * P + z];
            const double v0 = double(vv.re), v1 = double(vv.im);
            acc[ar] += v0 * ph[b0];
            if constexpr (b0 != ar) acc[b0] += v0 * ph[ar];
            if constexpr (b0 + 1 < B) {
              acc[ar] += v1 * ph[b0 + 1];
              acc[b0 + 1] += v1 * ph[ar];
            }
          });
        }
      });
    }
    q0 += ga;
    lds_barrier();
  }
  // all B rows of W are read before any is written: a store followed by the
  // next row's load would have to wait for that load (the compiler cannot
  // tell the rows apart), one memory round trip per row
  double wold[B];
#pragma unroll
  for (int b = 0; b < B; ++b)
    wold[b] = __builtin_nontemporal_load(&W[(int64_t)orbs[(DIAG ? 0 : B) + b] * npts + r]);
  if (act) {
#pragma unroll
    for (int b = 0; b < B; ++b)
      __builtin_nontemporal_store(wold[b] - alpha * acc[b],
                                  &W[(int64_t)orbs[(DIAG ? 0 : B) + b] * npts + r]);
  }
}

// One launch may serve two tiles with disjoint orbital blocks (their W rows
// differ): workgroups nb and up take the second tile's scratch S2 and
// orbitals orbs2 (nb, the workgroups of one tile, is a multiple of 8, so
// every workgroup keeps its XCD order).  Two tiles' 2 nb workgroups fill
// whole rounds of the chip where one tile's leave the last round half empty.
template <typename T, int N, int B, bool DIAG, bool ROWS>
__global__ __launch_bounds__((zinv_threads<T, N, ROWS>())) void k_zinv_acc(
    const cx<T>* __restrict__ S, const cx<T>* __restrict__ tw, const T* __restrict__ phi,
    double* __restrict__ W, const int* __restrict__ orbs, double alpha, int64_t npts,
    const cx<T>* __restrict__ S2, const int* __restrict__ orbs2, int nb) {
  __shared__ cx<T> lds[(B / 2) * zinv_rows<T, N, ROWS>() * (N + 1)];
  __shared__ cx<T> stw[N];
  const int second = (int)blockIdx.x >= nb;
  zinv_item<T, N, B, DIAG, ROWS, zinv_threads<T, N, ROWS>()>(
      second ? S2 : S, tw, phi, W, second ? orbs2 : orbs, alpha, npts,
      (int)blockIdx.x - (second ? nb : 0), lds, stw);
}

// ------------------------------------------------------------------ y/z slabs, forward
// Where a whole plane does not fit LDS, the forward y and z transforms of a
// plane are still done in one pass, a slab of z positions at a time: of the
// first z step (N1-point DFTs) of all the plane's rows, the K1S = ZC / N2
// outputs per row that land in a slab go to LDS, where the z transform and
// the whole y transform of the slab's ZC columns are finished and written
// once, in position order S[x][ky][kz].  The scratch is written once instead
// of written, read and written again by a z-row pass and a y-line pass.


// ZXY: write S[kz][x][ky] (the large-grid three-pass schedule) instead of
// S[x][ky][kz], through LDS so that the stores run along ky.
// The work of one slab workgroup of NT threads on plane x of one transform
// (pack pk, scratch grid Sp), slab group grp: lds holds N (ZC + 1) values,
// stw the N four-step twiddles, filled (and a barrier passed) before the
// call.  The slab kernel runs one item per workgroup; the batch forward
// items on the grids that take the two-slab form run the same function
// with the same thread count, so their results are bitwise the same.  The
// caller puts a barrier between two calls (the last step reads LDS).
template <typename T, int N, int SPW, bool ZXY, int NT>
__device__ __forceinline__ void slab_fwd_item(const T* __restrict__ phi, const Pack pk,
                                              cx<T>* __restrict__ Sp, int x, int grp,
                                              int64_t npts, cx<T>* __restrict__ lds,
                                              const cx<T>* __restrict__ stw) {
  constexpr int N1 = fft_split<N>::N1, N2 = fft_split<N>::N2;
  constexpr int SL = slab_count<T, N>(), ZC = N / SL, K1S = ZC / N2, PZ = ZC + 1;
  constexpr int NG = SL / SPW;                          // workgroups per plane
  constexpr int Q = (N * N2 + NT - 1) / NT;            // first-step tasks per thread
  constexpr int KH = SPW > 1 ? (SPW - 1) * K1S : 1;    // outputs held per task
  static_assert(SL > 0 && ZC % N2 == 0 && SL % SPW == 0, "whole second-step blocks per slab");
  const int tid = threadIdx.x;
  const int64_t plane = (int64_t)x * N * N;
  const T* __restrict__ pa = phi + (int64_t)pk.a * npts + plane;
  const T* __restrict__ pb = phi + (int64_t)pk.b * npts + plane;
  const T* __restrict__ pd = phi + (int64_t)(pk.c >= 0 ? pk.d : pk.b) * npts + plane;
  const T dmask = pk.c >= 0 ? T(1) : T(0);
  cx<T> hold[Q][KH];
  // z step 1 over every row: tasks (y, t2), t2 fastest; the outputs of the
  // group's first slab go to LDS, those of its other slabs to registers
  // (static indices: the group is a compile-time case, the test uniform)
  sfor<0, NG>([&](auto gc) {
    constexpr int G = decltype(gc)::value;
    constexpr int K0 = G * SPW * K1S;  // first step-1 output of the group
    if (grp == G) {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int task = tid + q * NT;
        if (task < N * N2) {
          const int y = task / N2, t2 = task % N2;
          cx<T> v[N1];
#pragma unroll
          for (int j1 = 0; j1 < N1; ++j1) {
            const int off = y * N + t2 + N2 * j1;
            const T fa = pa[off];
            v[j1] = {fa * pb[off], fa * (dmask * pd[off])};
          }
          dft<N1, false>(v);
#pragma unroll
          for (int k1 = K0; k1 < K0 + SPW * K1S; ++k1) {
            const cx<T> w = k1 == 0 ? v[0] : cmul(v[k1], stw[k1 * N2 + t2]);
            if (k1 < K0 + K1S) lds[y * PZ + t2 + N2 * (k1 - K0)] = w;
            else hold[q][k1 - K0 - K1S] = w;
          }
        }
      }
    }
  });
  // the rest of the transform for one slab whose first-step outputs are in LDS
  auto finish = [&](int sl) __attribute__((always_inline)) {
    __syncthreads();
    // z step 2 of the slab's blocks: tasks (y, k), y fastest
    for (int task = tid; task < N * K1S; task += NT) {
      const int y = task % N, k = task / N;
      cx<T> v[N2];
#pragma unroll
      for (int t = 0; t < N2; ++t) v[t] = lds[y * PZ + t + N2 * k];
      dft<N2, false>(v);
#pragma unroll
      for (int t = 0; t < N2; ++t) lds[y * PZ + t + N2 * k] = v[t];
    }
    __syncthreads();
    // y step 1: tasks (pz, u2), pz fastest
    for (int task = tid; task < ZC * N2; task += NT) {
      const int pz = task % ZC, u2 = task / ZC;
      cx<T> v[N1];
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) v[j1] = lds[(u2 + N2 * j1) * PZ + pz];
      dft<N1, false>(v);
#pragma unroll
      for (int k1 = 1; k1 < N1; ++k1) v[k1] = cmul(v[k1], stw[k1 * N2 + u2]);
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) lds[(u2 + N2 * k1) * PZ + pz] = v[k1];
    }
    __syncthreads();
    if constexpr (!ZXY) {
      // y step 2 -> global: tasks (pz, k1), pz fastest (a slab row is contiguous)
      cx<T>* __restrict__ out = Sp + plane + sl * ZC;
      for (int task = tid; task < ZC * N1; task += NT) {
        const int pz = task % ZC, k1 = task / ZC;
        cx<T> v[N2];
#pragma unroll
        for (int t = 0; t < N2; ++t) v[t] = lds[(t + N2 * k1) * PZ + pz];
        dft<N2, false>(v);
#pragma unroll
        for (int t = 0; t < N2; ++t) st_stream(&out[(int64_t)(t + N2 * k1) * N + pz], v[t]);
      }
    } else {
      // y step 2 in place, then the slab leaves transposed, consecutive
      // threads on consecutive ky (column reads of the odd-pitch rows)
      for (int task = tid; task < ZC * N1; task += NT) {
        const int pz = task % ZC, k1 = task / ZC;
        cx<T> v[N2];
#pragma unroll
        for (int t = 0; t < N2; ++t) v[t] = lds[(t + N2 * k1) * PZ + pz];
        dft<N2, false>(v);
#pragma unroll
        for (int t = 0; t < N2; ++t) lds[(t + N2 * k1) * PZ + pz] = v[t];
      }
      __syncthreads();
      cx<T>* __restrict__ out = Sp + (int64_t)x * N;
      for (int e = tid; e < N * ZC; e += NT) {
        const int ky = e % N, pz = e / N;
        st_stream(&out[(int64_t)(sl * ZC + pz) * N * N + ky], lds[ky * PZ + pz]);
      }
    }
  };
  finish(grp * SPW);
  sfor<1, SPW>([&](auto sc) {
    constexpr int h = decltype(sc)::value;
    __syncthreads();  // the previous slab read out of LDS
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int task = tid + q * NT;
      if (task < N * N2) {
        const int y = task / N2, t2 = task % N2;
#pragma unroll
        for (int k = 0; k < K1S; ++k) lds[y * PZ + t2 + N2 * k] = hold[q][(h - 1) * K1S + k];
      }
    }
    finish(grp * SPW + h);
  });
}

// On the two-slab grids, at most 128 registers: two 512-thread workgroups per CU.
template <typename T, int N>
constexpr int slab_fwd_waves() { return fwd_slabs<T, N>() ? 4 : 1; }

template <typename T, int N, int SPW, bool ZXY>
__global__ __launch_bounds__((slab_threads<T, N, SPW>()))
__attribute__((amdgpu_waves_per_eu(slab_fwd_waves<T, N>()))) void k_slab_fwd(
    const T* __restrict__ phi, const Pack* __restrict__ packs, const cx<T>* __restrict__ tw,
    cx<T>* __restrict__ S, int npack, int64_t npts) {
  constexpr int N2 = fft_split<N>::N2;
  constexpr int SL = slab_count<T, N>(), PZ = N / SL + 1, NG = SL / SPW;
  constexpr int NT = slab_threads<T, N, SPW>();
  __shared__ cx<T> lds[N * PZ];
  __shared__ cx<T> stw[N];
  // item: (x, transform, slab group); the groups of one plane are
  // consecutive on one XCD (workgroup b runs on XCD b mod 8), so its orbital
  // rows are in that L2
  const int i = blockIdx.x;
  const int r = i >> 3, grp = r % NG;
  int x, p;
  plane_item<T, N>((r / NG) * 8 + (i & 7), npack, x, p);
  const Pack pk = packs[p];
  for (int k = threadIdx.x; k < N; k += NT) stw[k] = tw[(k % N2) * (k / N2)];
  __syncthreads();
  slab_fwd_item<T, N, SPW, ZXY, NT>(phi, pk, S + (int64_t)p * npts, x, grp, npts, lds, stw);
}

// Large-grid three-pass schedule: where a workgroup holds all slabs of a
// plane (slab_spw == slab_count), the forward pass writes S[kz][x][ky] and
// the middle pass below does, per kz plane [x][ky], slab by slab of ky:
// forward x, Coulomb multiply, inverse x and the second inverse y step
// (within the slab's blocks), keeping each thread's share of the slab in
// registers; after the last slab the first inverse y step runs on the held
// values and the plane leaves in natural y, in place.  The inverse z and W
// pass is then the plane-fitting grids' one.

// The work of one slab middle-pass workgroup of NT threads: item bid = (kz
// position, transform); lds holds N (ZC + 1) values, stw the N four-step
// twiddles, filled before the call (the first slab starts with a barrier).
// The slab kernel runs one item per workgroup; the batch middle items on
// the grids that take this form run the same function with the same
// thread count, so their results are bitwise the same.
template <typename T, int N, int NT>
__device__ __forceinline__ void slab_mid_item(cx<T>* __restrict__ S, int64_t npts, T g0, T g1,
                                              T g2, T kscale, int bid, cx<T>* __restrict__ lds,
                                              const cx<T>* __restrict__ stw) {
  constexpr int N1 = fft_split<N>::N1, N2 = fft_split<N>::N2;
  constexpr int SL = slab_count<T, N>(), ZC = N / SL, K1S = ZC / N2, PZ = ZC + 1;
  constexpr int Q = (N * N2 + NT - 1) / NT;   // final-step tasks (x, t2) per thread
  constexpr int KH = (SL - 1) * K1S;          // values held per task
  const int pz = bid % N, p = bid / N;
  const int tid = threadIdx.x;
  cx<T>* __restrict__ io = S + (int64_t)p * npts + (int64_t)pz * N * N;
  const int kz = freq_of_pos<N>(pz);
  cx<T> hold[Q][KH];
  sfor<0, SL>([&](auto sc) {
    constexpr int sl = decltype(sc)::value;
    __syncthreads();  // twiddles in place / the previous slab read out of LDS
    // x forward step 1 from global: tasks (py, t2), py fastest
    for (int task = tid; task < ZC * N2; task += NT) {
      const int py = task % ZC, t2 = task / ZC;
      cx<T> v[N1];
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) v[j1] = io[(int64_t)(t2 + N2 * j1) * N + sl * ZC + py];
      dft<N1, false>(v);
#pragma unroll
      for (int k1 = 1; k1 < N1; ++k1) v[k1] = cmul(v[k1], stw[k1 * N2 + t2]);
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) lds[(t2 + N2 * k1) * PZ + py] = v[k1];
    }
    __syncthreads();
    // x forward step 2, Coulomb multiply, x inverse step 2: tasks (py, k1)
    for (int task = tid; task < ZC * N1; task += NT) {
      const int py = task % ZC, k1 = task / ZC;
      const int ky = freq_of_pos<N>(sl * ZC + py);
      cx<T> v[N2];
#pragma unroll
      for (int t = 0; t < N2; ++t) v[t] = lds[(t + N2 * k1) * PZ + py];
      dft<N2, false>(v);
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2)
        v[k2] = scale(v[k2], coulomb_k<T, N>(k1 + N1 * k2, ky, kz, g0, g1, g2, kscale));
      dft<N2, true>(v);
#pragma unroll
      for (int t = 0; t < N2; ++t) lds[(t + N2 * k1) * PZ + py] = v[t];
    }
    __syncthreads();
    // x inverse step 1 to natural x, in place: tasks (py, t2)
    for (int task = tid; task < ZC * N2; task += NT) {
      const int py = task % ZC, t2 = task / ZC;
      cx<T> v[N1];
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) v[k1] = cmulc(lds[(t2 + N2 * k1) * PZ + py], stw[k1 * N2 + t2]);
      dft<N1, true>(v);
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) lds[(t2 + N2 * j1) * PZ + py] = v[j1];
    }
    __syncthreads();
    // y inverse step 2 within the slab's blocks: tasks (x, k), x fastest
    for (int task = tid; task < N * K1S; task += NT) {
      const int x = task % N, k = task / N;
      cx<T> v[N2];
#pragma unroll
      for (int t = 0; t < N2; ++t) v[t] = lds[x * PZ + t + N2 * k];
      dft<N2, true>(v);
#pragma unroll
      for (int t = 0; t < N2; ++t) lds[x * PZ + t + N2 * k] = v[t];
    }
    __syncthreads();
    if constexpr (sl + 1 < SL) {
      // this thread's tasks (x, t2), t2 fastest: the slab's K1S values
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int task = tid + q * NT;
        if (task < N * N2) {
          const int t2 = task % N2, x = task / N2;
#pragma unroll
          for (int k = 0; k < K1S; ++k) hold[q][sl * K1S + k] = lds[x * PZ + t2 + N2 * k];
        }
      }
    } else {
      // y inverse step 1 -> global, natural y, in place (every slab of the
      // plane has been read): tasks (x, t2), t2 fastest
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int task = tid + q * NT;
        if (task < N * N2) {
          const int t2 = task % N2, x = task / N2;
          cx<T> v[N1];
#pragma unroll
          for (int k1 = 0; k1 < N1; ++k1) {
            const cx<T> u = k1 < KH ? hold[q][k1 < KH ? k1 : 0] : lds[x * PZ + t2 + N2 * (k1 - KH)];
            v[k1] = cmulc(u, stw[k1 * N2 + t2]);
          }
          dft<N1, true>(v);
#pragma unroll
          for (int j1 = 0; j1 < N1; ++j1) io[(int64_t)x * N + t2 + N2 * j1] = v[j1];
        }
      }
    }
  });
}

// Plane-fitting grids whose plane workgroup takes more than half of a CU's
// LDS (FP64 80^3 and 96^3, FP32 120^3 and 128^3) run the middle pass slab by
// slab too: 512 threads and half a plane of LDS, two workgroups per CU.
// One 128-transform launch, slabs against planes: FP64 96^3 714 / 750 us,
// 80^3 409 / 483; FP32 128^3 838 / 1011, 120^3 810 / 1018 (FP32 96^3, whose
// plane workgroups already fit twice, 397 / 371).
template <typename T, int N>
constexpr bool mid_slabs() {
  return plane_ok<T, N>() && slab_count<T, N>() == 2 &&
         2 * (((long)N * (N + 1) + N) * (long)sizeof(cx<T>) + 64) > kLdsBytes;
}

template <typename T, int N>
__global__ __launch_bounds__((slab_threads<T, N, slab_count<T, N>()>()))
__attribute__((amdgpu_waves_per_eu(mid_slabs<T, N>() ? 4 : 1))) void
k_slab_mid(cx<T>* __restrict__ S, const cx<T>* __restrict__ tw, int npack, int64_t npts, T g0,
           T g1, T g2, T kscale) {
  constexpr int N2 = fft_split<N>::N2;
  constexpr int SL = slab_count<T, N>(), PZ = N / SL + 1;
  constexpr int NT = slab_threads<T, N, SL>();
  __shared__ cx<T> lds[N * PZ];
  __shared__ cx<T> stw[N];
  for (int i = threadIdx.x; i < N; i += NT) stw[i] = tw[(i % N2) * (i / N2)];
  slab_mid_item<T, N, NT>(S, npts, g0, g1, g2, kscale, blockIdx.x, lds, stw);
}

// ------------------------------------------------------------------ z rows (fallback)
// Forward: pair density + z transform of kRowsPerBlock consecutive rows,
// written in position order with streaming stores (the y pass reads them
// once).  Twiddles in LDS as stw[k1 N2 + t2].
template <typename T, int N>
__global__ __launch_bounds__(row_threads<N>()) void k_rows_fwd(
    const T* __restrict__ phi, const Pack* __restrict__ packs, const cx<T>* __restrict__ tw,
    cx<T>* __restrict__ S, int npack, int64_t npts) {
  constexpr int N1 = fft_split<N>::N1, N2 = fft_split<N>::N2, P = N + 1;
  constexpr int NT = row_threads<N>(), R = kRowsPerBlock;
  __shared__ cx<T> lds[R * P];
  __shared__ cx<T> stw[N];
  // transform fastest: consecutive workgroups share the row block, so the
  // orbital rows stay in L2 across the tile's transforms
  const int p = blockIdx.x % npack, rb = blockIdx.x / npack;
  const Pack pk = packs[p];
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NT) stw[i] = tw[(i % N2) * (i / N2)];
  const int64_t row0 = (int64_t)rb * R * N;
  const T* __restrict__ pa = phi + (int64_t)pk.a * npts + row0;
  const T* __restrict__ pb = phi + (int64_t)pk.b * npts + row0;
  const bool two = pk.c >= 0;
  const T* __restrict__ pd = phi + (int64_t)(two ? pk.d : pk.b) * npts + row0;
  __syncthreads();
  for (int task = tid; task < R * N2; task += NT) {
    const int y = task / N2, t2 = task % N2;
    cx<T> v[N1];
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) {
      const int off = y * N + t2 + N2 * j1;
      const T fa = pa[off];
      v[j1] = {fa * pb[off], two ? fa * pd[off] : T(0)};
    }
    dft<N1, false>(v);
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) v[k1] = cmul(v[k1], stw[k1 * N2 + t2]);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) lds[y * P + t2 + N2 * k1] = v[k1];
  }
  __syncthreads();
  for (int task = tid; task < R * N1; task += NT) {
    const int y = task % R, k1 = task / R;
    cx<T> v[N2];
#pragma unroll
    for (int t = 0; t < N2; ++t) v[t] = lds[y * P + t + N2 * k1];
    dft<N2, false>(v);
#pragma unroll
    for (int t = 0; t < N2; ++t) lds[y * P + t + N2 * k1] = v[t];
  }
  __syncthreads();
  cx<T>* __restrict__ out = S + (int64_t)p * npts + row0;
  for (int e = tid; e < R * N; e += NT) st_stream(&out[e], lds[(e / N) * P + (e % N)]);
}

// Inverse z transform of position-ordered rows to natural order.
template <typename T, int N>
__global__ __launch_bounds__(row_threads<N>()) void k_rows_inv(
    cx<T>* __restrict__ S, const cx<T>* __restrict__ tw, int npack, int64_t npts) {
  constexpr int N1 = fft_split<N>::N1, N2 = fft_split<N>::N2, P = N + 1;
  constexpr int NT = row_threads<N>(), R = kRowsPerBlock;
  __shared__ cx<T> lds[R * P];
  __shared__ cx<T> stw[N];
  constexpr int nrb = N * N / R;
  const int rb = blockIdx.x % nrb, p = blockIdx.x / nrb;
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NT) stw[i] = tw[(i % N2) * (i / N2)];
  cx<T>* __restrict__ io = S + (int64_t)p * npts + (int64_t)rb * R * N;
  for (int e = tid; e < R * N; e += NT) lds[(e / N) * P + (e % N)] = io[e];
  __syncthreads();
  for (int task = tid; task < R * N1; task += NT) {
    const int y = task % R, k1 = task / R;
    cx<T> v[N2];
#pragma unroll
    for (int t = 0; t < N2; ++t) v[t] = lds[y * P + t + N2 * k1];
    dft<N2, true>(v);
#pragma unroll
    for (int t = 0; t < N2; ++t) lds[y * P + t + N2 * k1] = v[t];
  }
  __syncthreads();
  for (int task = tid; task < R * N2; task += NT) {
    const int y = task / N2, t2 = task % N2;
    cx<T> v[N1];
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) v[k1] = cmulc(lds[y * P + t2 + N2 * k1], stw[k1 * N2 + t2]);
    dft<N1, true>(v);
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) io[y * N + t2 + N2 * j1] = v[j1];
  }
}

// ------------------------------------------------------------------ strided lines
// A workgroup owns C lines that are adjacent in memory (consecutive z
// positions) and runs length-N transforms along a strided axis:
//   MODE_POISSON : x lines, forward, * K / N, inverse (in place);
//   MODE_ENERGY  : x lines, forward, sum K |Z|^2 (S unchanged);
//   MODE_FWD     : y lines, forward only, written in position order;
//   MODE_INV     : y lines, inverse only, natural order.
enum { MODE_POISSON = 0, MODE_ENERGY = 1, MODE_FWD = 2, MODE_INV = 3 };

template <typename T>
__device__ __forceinline__ double block_sum(double v, double* red) {
  // fixed-order reduction: wave shuffles, then wave partials in LDS
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
  }
  return s;
}

template <typename T, int N, int MODE, int C = line_chunk<N>()>
__global__ __launch_bounds__((line_threads<N, C>())) void k_lines(
    cx<T>* __restrict__ S, const cx<T>* __restrict__ tw, int npack, int64_t npts, int64_t estride,
    int64_t ostride, T g0, T g1, T g2, T kscale, double* __restrict__ part) {
  constexpr int N1 = fft_split<N>::N1, N2 = fft_split<N>::N2;
  constexpr int NT = line_threads<N, C>(), NCH = N / C;
  static_assert(N % C == 0, "pencils per workgroup must divide the grid");
  __shared__ cx<T> lds[N * C];
  __shared__ cx<T> stw[N];
  __shared__ double red[NT / 64 + 1];
  const int bid = blockIdx.x;
  const int chunk = bid % NCH;
  const int outer = (bid / NCH) % N;
  const int p = bid / (NCH * N);
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NT) stw[i] = tw[(i % N2) * (i / N2)];  // stw[k1 N2 + t2] = w^(t2 k1)
  cx<T>* __restrict__ base = S + (int64_t)p * npts + (int64_t)outer * ostride + chunk * C;
  __syncthreads();

  if constexpr (MODE != MODE_INV) {
    // forward step 1: global -> LDS, tasks (c, t2) with c fastest
    for (int task = tid; task < C * N2; task += NT) {
      const int c = task % C, t2 = task / C;
      cx<T> v[N1];
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) v[j1] = base[(int64_t)(t2 + N2 * j1) * estride + c];
      dft<N1, false>(v);
#pragma unroll
      for (int k1 = 1; k1 < N1; ++k1) v[k1] = cmul(v[k1], stw[k1 * N2 + t2]);
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) lds[(t2 + N2 * k1) * C + c] = v[k1];
    }
    __syncthreads();
    double acc = 0.0;
    const int ky = freq_of_pos<N>(outer);
    for (int task = tid; task < C * N1; task += NT) {
      const int c = task % C, k1 = task / C;
      cx<T> v[N2];
#pragma unroll
      for (int t = 0; t < N2; ++t) v[t] = lds[(t + N2 * k1) * C + c];
      dft<N2, false>(v);
      if constexpr (MODE == MODE_FWD) {
#pragma unroll
        for (int t = 0; t < N2; ++t) base[(int64_t)(t + N2 * k1) * estride + c] = v[t];
      } else {
        const int kz = freq_of_pos<N>(chunk * C + c);
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) {
          const T kk = coulomb_k<T, N>(k1 + N1 * k2, ky, kz, g0, g1, g2, kscale);
          if constexpr (MODE == MODE_POISSON) {
            v[k2] = scale(v[k2], kk);
          } else {
            acc += double(kk) * (double(v[k2].re) * double(v[k2].re) +
                                 double(v[k2].im) * double(v[k2].im));
          }
        }
        if constexpr (MODE == MODE_POISSON) {
          dft<N2, true>(v);
#pragma unroll
          for (int t = 0; t < N2; ++t) lds[(t + N2 * k1) * C + c] = v[t];
        }
      }
    }
    if constexpr (MODE == MODE_ENERGY) {
      const double s = block_sum<T>(acc, red);
      if (tid == 0) part[bid] = s;
      return;
    }
    if constexpr (MODE == MODE_FWD) return;
    __syncthreads();
  } else {
    // inverse step 2: global positions -> LDS
    for (int task = tid; task < C * N1; task += NT) {
      const int c = task % C, k1 = task / C;
      cx<T> v[N2];
#pragma unroll
      for (int t = 0; t < N2; ++t) v[t] = base[(int64_t)(t + N2 * k1) * estride + c];
      dft<N2, true>(v);
#pragma unroll
      for (int t = 0; t < N2; ++t) lds[(t + N2 * k1) * C + c] = v[t];
    }
    __syncthreads();
  }
  // inverse step 1: LDS -> global natural order
  for (int task = tid; task < C * N2; task += NT) {
    const int c = task % C, t2 = task / C;
    cx<T> v[N1];
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) v[k1] = cmulc(lds[(t2 + N2 * k1) * C + c], stw[k1 * N2 + t2]);
    dft<N1, true>(v);
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) base[(int64_t)(t2 + N2 * j1) * estride + c] = v[j1];
  }
}

// ------------------------------------------------------------------ W accumulation
// One thread per grid point; the tile's pairs are visited in a fixed order
// (no atomics), so W is bitwise reproducible.  orbs: the tile's orbitals,
// I list (B entries) then J list (B entries).
//
// General (masked) tiles: meta[p] = a0 | b0 << 8 | a1 << 16 | b1 << 24 gives
// the local positions of transform p's pair in the real (a0, b0) and
// imaginary (a1, b1; a1 = 255 when absent) half; useI / useJ flag the
// orbitals with at least one pair.  Transforms come row-major in a (both
// halves share it), so a thread keeps the current row's orbital value and
// accumulator in registers and the other side's values and accumulators in
// LDS, laid out [orbital][thread]: each thread reads and writes only its own
// column (no barriers, no bank conflicts), and the runtime positions b index
// LDS instead of select chains over registers.  The sums run in the same
// order as a per-orbital register accumulator would take them.
constexpr int kAccThreads = 128;
constexpr int kAccAhead = 8;  // transforms whose loads are issued ahead

// W -= d with streaming accesses (as in the fused pass: W rows are touched
// far apart in time).  The orbitals come in the bulk precision, as in the
// fused pass.
__device__ __forceinline__ void w_sub(double* p, double d) {
  __builtin_nontemporal_store(__builtin_nontemporal_load(p) - d, p);
}

template <typename TS, int B, bool DIAG>
__global__ __launch_bounds__(kAccThreads) void k_accumulate(
    const cx<TS>* __restrict__ S, const TS* __restrict__ phi, double* __restrict__ W,
    const int* __restrict__ meta, int npack, const int* __restrict__ orbs, unsigned useI,
    unsigned useJ, double alpha, int64_t npts) {
  __shared__ TS sph[B][kAccThreads];
  __shared__ double sacc[B][kAccThreads];
  const int t = threadIdx.x;
  const int64_t r = (int64_t)blockIdx.x * kAccThreads + t;
  if (r >= npts) return;  // no barriers below
  // the other side: the J list off the diagonal, the tile's one list on it
  const unsigned use = DIAG ? useI : useJ;
  const int* side = DIAG ? orbs : orbs + B;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    sph[b][t] = ((use >> b) & 1u) ? phi[(int64_t)side[b] * npts + r] : TS(0);
    sacc[b][t] = 0.0;
  }
  int cur = -1;  // current row a
  double phA = 0.0, accA = 0.0;
  auto pair = [&](int b, double v) __attribute__((always_inline)) {
    if (DIAG && b == cur) {
      accA += v * phA;
    } else {
      accA += v * sph[b][t];
      sacc[b][t] += v * phA;
    }
  };
  for (int p0 = 0; p0 < npack; p0 += kAccAhead) {
    cx<TS> z[kAccAhead];
    int m[kAccAhead];
#pragma unroll
    for (int u = 0; u < kAccAhead; ++u) {
      const int p = min(p0 + u, npack - 1);
      z[u] = S[(int64_t)p * npts + r];
      m[u] = meta[p];
    }
#pragma unroll
    for (int u = 0; u < kAccAhead; ++u) {
      if (p0 + u >= npack) break;
      const int a = m[u] & 255, b0 = (m[u] >> 8) & 255, a1 = (m[u] >> 16) & 255,
                b1 = (m[u] >> 24) & 255;
      if (a != cur) {
        if (cur >= 0) {
          if constexpr (DIAG) sacc[cur][t] = accA;
          else w_sub(&W[(int64_t)orbs[cur] * npts + r], alpha * accA);
        }
        cur = a;
        if constexpr (DIAG) {
          phA = sph[a][t];
          accA = sacc[a][t];  // contributions of earlier rows, where a was the column
        } else {
          phA = phi[(int64_t)orbs[a] * npts + r];
          accA = 0.0;
        }
      }
      pair(b0, double(z[u].re));
      if (a1 != 255) pair(b1, double(z[u].im));
    }
  }
  if (cur >= 0) {
    if constexpr (DIAG) sacc[cur][t] = accA;
    else w_sub(&W[(int64_t)orbs[cur] * npts + r], alpha * accA);
  }
  // the other side's rows: all read before any is written (one round trip)
  double wold[B];
#pragma unroll
  for (int b = 0; b < B; ++b)
    wold[b] = ((use >> b) & 1u) ? __builtin_nontemporal_load(&W[(int64_t)side[b] * npts + r]) : 0.0;
#pragma unroll
  for (int b = 0; b < B; ++b)
    if ((use >> b) & 1u)
      __builtin_nontemporal_store(wold[b] - alpha * sacc[b][t], &W[(int64_t)side[b] * npts + r]);
}

template <typename TS, int B, bool DIAG>
__global__ __launch_bounds__(256) void k_accumulate_full(
    const cx<TS>* __restrict__ S, const TS* __restrict__ phi, double* __restrict__ W,
    const int* __restrict__ orbs, double alpha, int64_t npts) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= npts) return;
  static_assert(DIAG || B % 2 == 0, "off-diagonal rows pack evenly");
  TS phI[B], phJ[DIAG ? 1 : B];
  double accI[B], accJ[DIAG ? 1 : B];
#pragma unroll
  for (int a = 0; a < B; ++a) {
    phI[a] = phi[(int64_t)orbs[a] * npts + r];
    accI[a] = 0.0;
  }
  if constexpr (!DIAG) {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      phJ[b] = phi[(int64_t)orbs[B + b] * npts + r];
      accJ[b] = 0.0;
    }
  }
  sfor<0, B>([&](auto ac) {
    constexpr int a = decltype(ac)::value;
    sfor<0, row_packs<B, DIAG>(a)>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      constexpr int q = row_pack0<B, DIAG>(a) + c;
      constexpr int b0 = (DIAG ? a : 0) + 2 * c;
      const cx<TS> z = S[(int64_t)q * npts + r];
      const double v0 = double(z.re), v1 = double(z.im);
      if constexpr (DIAG) {
        accI[a] += v0 * phI[b0];
        if constexpr (b0 != a) accI[b0] += v0 * phI[a];
        if constexpr (b0 + 1 < B) {
          accI[a] += v1 * phI[b0 + 1];
          accI[b0 + 1] += v1 * phI[a];
        }
      } else {
        accI[a] += v0 * phJ[b0] + v1 * phJ[b0 + 1];
        accJ[b0] += v0 * phI[a];
        accJ[b0 + 1] += v1 * phI[a];
      }
    });
  });
  // every W row read before any is written (one round trip, not one per row)
  double wI[B], wJ[DIAG ? 1 : B];
#pragma unroll
  for (int a = 0; a < B; ++a) wI[a] = W[(int64_t)orbs[a] * npts + r];
  if constexpr (!DIAG) {
#pragma unroll
    for (int b = 0; b < B; ++b) wJ[b] = W[(int64_t)orbs[B + b] * npts + r];
  }
#pragma unroll
  for (int a = 0; a < B; ++a) W[(int64_t)orbs[a] * npts + r] = wI[a] - alpha * accI[a];
  if constexpr (!DIAG) {
#pragma unroll
    for (int b = 0; b < B; ++b) W[(int64_t)orbs[B + b] * npts + r] = wJ[b] - alpha * accJ[b];
  }
}

// ------------------------------------------------------------------ small kernels
__global__ void k_energy_reduce(const double* __restrict__ part, int parts, double factor,
                                double* __restrict__ e_pack) {
  __shared__ double red[16];
  const int p = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < parts; i += blockDim.x) acc += part[(int64_t)p * parts + i];
  const double s = block_sum<double>(acc, red);
  if (threadIdx.x == 0) e_pack[p] = s * factor;
}

__global__ void k_fill_f64(double* __restrict__ p, double v, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = i; k < count; k += stride) p[k] = v;
}

__global__ void k_cast_f64_f32(const double* __restrict__ in, float* __restrict__ out,
                               int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = i; k < count; k += stride) out[k] = float(in[k]);
}

// ------------------------------------------------------------------ batches
// Persistent pass kernels over the whole three-pass tiles of many systems of
// one grid size and bulk precision (a lane round: segment k of the table
// covers items item0 .. item0 + count - 1 of one system's tile).  Forward
// items (one plane of one transform) all cost the same, so each workgroup
// takes every grid-th item of the round; middle and inverse-z/W items are
// taken from a work queue (one atomic counter per launch) until it is empty
// (middle items strided like the forward ones measured slower inside a
// batch graph: 233 against 228 ms for config 4).
// Each item runs the single-system code for its grid, block and diagonal
// flag with the single-system thread count (the two-slab forward code on
// these grids), so every result is bitwise the system's own build.
// One kernel per grid size (48, 64, 80, 96: a plane fits one workgroup's
// LDS in FP64 and FP32): one kernel over all sizes took the register
// allocation of the largest into every path, and a common thread count
// idled threads on the smaller grids.
#define ACEX_BATCH_SIZES(X) X(48) X(64) X(80) X(96)

// Threads of a batch pass workgroup: 8 N (the single-system middle and
// inverse-z workgroups'), or, for forward items on grids whose own forward
// pass takes the two-slab form, that kernel's.
template <typename T, int PASS, int N>
constexpr int batch_threads() {
  return (PASS == 0 && fwd_slabs<T, N>()) || (PASS == 1 && mid_slabs<T, N>())
             ? slab_threads<T, N, 2>()
             : 8 * N;
}

// LDS values of a batch pass workgroup.
template <typename T, int PASS, int N, int B>
constexpr int batch_lds() {
  if constexpr (PASS == 2) return (B / 2) * zinv_rows<T, N>() * (N + 1) + N;
  else if constexpr ((PASS == 0 && fwd_slabs<T, N>()) || (PASS == 1 && mid_slabs<T, N>()))
    return N * (N / 2 + 1) + N;
  else return N * (N + 1) + N;
}

// the last segment that starts at or before item (uniform across the workgroup)
__device__ __forceinline__ int batch_seg(const BatchSeg* __restrict__ segs, int nseg, int item) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].item0 <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Forward items of a lane round, strided by the grid.
template <typename T, int N>
struct FwdLane {
  const BatchSeg* segs;
  int nseg, total;
  int64_t npts;
  __device__ __forceinline__ int first() const { return blockIdx.x; }
  __device__ __forceinline__ void ask() {}
  __device__ __forceinline__ void post() {}
  __device__ __forceinline__ int next(int it) const { return it + gridDim.x; }
  __device__ __forceinline__ bool more(int it) const { return it < total; }
  __device__ __forceinline__ void at(int it, const T*& f, Pack& pk, cx<T>*& o, int& x) const {
    const BatchSeg& g = segs[batch_seg(segs, nseg, it)];
    int p;
    plane_item<T, N>(it - g.item0, g.npack, x, p);
    f = static_cast<const T*>(g.phi);
    pk = g.packs[p];
    o = static_cast<cx<T>*>(g.S) + (int64_t)p * npts;
  }
};

// Middle (PASS 1) and inverse-z/W (PASS 2, block B) items.
template <typename T, int PASS, int N, int B>
__device__ __forceinline__ void batch_item(const BatchSeg& g, int local, cx<T>* __restrict__ smem) {
  constexpr int NT = batch_threads<T, PASS, N>();
  if constexpr (PASS == 1 && mid_slabs<T, N>()) {
    // twiddles filled once per launch (the same for every segment)
    slab_mid_item<T, N, NT>(static_cast<cx<T>*>(g.S), g.npts, T(g.g2[0]), T(g.g2[1]),
                            T(g.g2[2]), T(g.kscale), local, smem, smem + N * (N / 2 + 1));
  } else if constexpr (PASS == 1) {
    plane_mid_item<T, N, NT, true>(static_cast<cx<T>*>(g.S), static_cast<const cx<T>*>(g.tw),
                                   g.npts, T(g.g2[0]), T(g.g2[1]), T(g.g2[2]), T(g.kscale), local,
                                   smem, smem + N * (N + 1));
  } else {
    cx<T>* stw = smem + (B / 2) * zinv_rows<T, N>() * (N + 1);
    const cx<T>* S = static_cast<const cx<T>*>(g.S);
    const cx<T>* tw = static_cast<const cx<T>*>(g.tw);
    const T* phi = static_cast<const T*>(g.phi);
    if (g.diag)
      zinv_item<T, N, B, true, false, NT, true>(S, tw, phi, g.W, g.orbs, g.alpha, g.npts, local,
                                                smem, stw);
    else
      zinv_item<T, N, B, false, false, NT, true>(S, tw, phi, g.W, g.orbs, g.alpha, g.npts, local,
                                                 smem, stw);
  }
}

// Waves per SIMD each batch kernel is compiled for: the workgroups per CU of
// the single-system kernel of the same pass and grid (their registers and
// LDS), where the persistent loop would otherwise take more registers and
// fit fewer (1: no bound beyond the workgroup size).
template <typename T, int PASS, int N, int B>
constexpr int batch_waves() {
  constexpr bool F = sizeof(T) == 4;
  if (PASS == 1) {
    if (N == 48) return F ? 1 : 6;
    if (N == 64 || N == 80) return F ? 8 : 1;
    return F ? 6 : 1;
  }
  return 1;
}

// PASS 0 and 1 take B = 0; PASS 2 one kernel per block.
template <typename T, int PASS, int N, int B>
__global__ __launch_bounds__((batch_threads<T, PASS, N>()))
__attribute__((amdgpu_waves_per_eu(batch_waves<T, PASS, N, B>()))) void k_batch_pass(
    const BatchSeg* __restrict__ segs, int nseg, int total, int* __restrict__ counter) {
  __shared__ cx<T> smem[batch_lds<T, PASS, N, B>()];
  constexpr int NT = batch_threads<T, PASS, N>();
  if constexpr (PASS == 0 && fwd_slabs<T, N>()) {
    // the single-system slab kernel's items, one after another
    constexpr int N2 = fft_split<N>::N2;
    constexpr int64_t npts = (int64_t)N * N * N;
    FwdLane<T, N> q{segs, nseg, total, npts};
    cx<T>* stw = smem + N * (N / 2 + 1);
    const cx<T>* tw = static_cast<const cx<T>*>(segs[0].tw);
    for (int k = threadIdx.x; k < N; k += NT) stw[k] = tw[(k % N2) * (k / N2)];
    __syncthreads();
    for (int item = q.first(); q.more(item); item = q.next(item)) {
      const T* phi;
      Pack pk;
      cx<T>* o;
      int x;
      q.at(item, phi, pk, o, x);
      slab_fwd_item<T, N, 2, true, NT>(phi, pk, o, x, 0, npts, smem, stw);
      __syncthreads();  // the item's last step read LDS
    }
  } else if constexpr (PASS == 0) {
    FwdLane<T, N> q{segs, nseg, total, (int64_t)N * N * N};
    plane_fwd_loop<T, N, true, NT>(q, static_cast<const cx<T>*>(segs[0].tw), (int64_t)N * N * N,
                                   smem, smem + N * (N + 1));
  } else {
    __shared__ int s_item;
    if constexpr (PASS == 1 && mid_slabs<T, N>()) {
      constexpr int N2 = fft_split<N>::N2;
      cx<T>* stw = smem + N * (N / 2 + 1);
      const cx<T>* tw = static_cast<const cx<T>*>(segs[0].tw);
      for (int k = threadIdx.x; k < N; k += NT) stw[k] = tw[(k % N2) * (k / N2)];
    }
    for (;;) {
      if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
      __syncthreads();
      const int item = __builtin_amdgcn_readfirstlane(s_item);
      // every thread has its item (and has left the previous one) before
      // thread 0 takes the next or anyone reuses the LDS
      __syncthreads();
      if (item >= total) break;  // the same for the whole workgroup
      const int k = batch_seg(segs, nseg, item);
      batch_item<T, PASS, N, B>(segs[k], item - segs[k].item0, smem);
    }
  }
}

bool batch_ok(int n, int prec, int block) {
  if (block != 8 && block != 16) return false;
  switch (n) {
#define X(NN) case NN:
    ACEX_BATCH_SIZES(X)
#undef X
    break;
    default: return false;
  }
  return three_pass_ok(n, prec, block);
}

int batch_items(int pass, int n, int npack) {
  return pass == 2 ? n * (n / 8) : n * npack;  // eight rows per item on these grids
}

// Workgroups of a batch pass resident per CU (LDS and registers), looked up
// once per kernel.
template <typename T, int PASS, int N, int B>
static int batch_per_cu() {
  static std::atomic<int> cached{0};
  const int v = cached.load(std::memory_order_relaxed);
  if (v > 0) return v;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batch_pass<T, PASS, N, B>,
                                                   batch_threads<T, PASS, N>(), 0) != hipSuccess ||
      occ < 1)
    occ = 1;
  cached.store(occ, std::memory_order_relaxed);
  return occ;
}

template <typename T, int PASS, int N, int B>
static hipError_t batch_launch(const BatchSeg* segs, int nseg, int total, int* counter, int cus,
                               hipStream_t s) {
  static_assert(PASS != 2 || zinv_threads<T, N>() <= batch_threads<T, PASS, N>(),
                "a thread per inverse-z point");
  static_assert(plane_ok<T, N>(), "a plane per workgroup");
  // persistent, the whole chip (one workgroup per item measured slower,
  // 246-255 against 228 ms for config 4, and so did half or a quarter of
  // the chip per launch, 249 and 383 ms)
  const int grid = std::min(total, cus * batch_per_cu<T, PASS, N, B>());
  hipLaunchKernelGGL((k_batch_pass<T, PASS, N, B>), dim3(grid), dim3(batch_threads<T, PASS, N>()), 0, s,
                     segs, nseg, total, counter);
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t batch_t(int pass, int block, const BatchSeg* segs, int nseg, int total,
                          int* counter, int cus, hipStream_t s) {
  if (pass == 0) return batch_launch<T, 0, N, 0>(segs, nseg, total, counter, cus, s);
  if (pass == 1) return batch_launch<T, 1, N, 0>(segs, nseg, total, counter, cus, s);
  if (pass == 2 && block == 16) return batch_launch<T, 2, N, 16>(segs, nseg, total, counter, cus, s);
  if (pass == 2 && block == 8) return batch_launch<T, 2, N, 8>(segs, nseg, total, counter, cus, s);
  return hipErrorInvalidValue;
}

hipError_t launch_batch_pass(int prec, int pass, int n, int block, const BatchSeg* segs, int nseg,
                             int total, int* counter, int cus, hipStream_t s) {
  if (nseg <= 0 || total <= 0) return hipSuccess;
  switch (n) {
#define X(NN)                                                                               \
  case NN:                                                                                  \
    return prec == 0 ? batch_t<double, NN>(pass, block, segs, nseg, total, counter, cus, s) \
                     : batch_t<float, NN>(pass, block, segs, nseg, total, counter, cus, s);
    ACEX_BATCH_SIZES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

__global__ void k_fill_i32(int* __restrict__ p, int v, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

hipError_t launch_fill_i32(int* p, int v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, v,
                     count);
  return hipGetLastError();
}

// ------------------------------------------------------------------ dispatch

#define ACEX_SIZES(X) \
  X(16) X(24) X(32) X(40) X(48) X(64) X(80) X(96) X(120) X(128) X(144) X(160) X(192)

bool supported_n(int n) {
  switch (n) {
#define X(N) case N:
    ACEX_SIZES(X)
#undef X
    return true;
    default: return false;
  }
}

template <typename T>
static bool plane_fits_t(int n) {
  switch (n) {
#define X(N) \
  case N: return plane_ok<T, N>();
    ACEX_SIZES(X)
#undef X
    default: return false;
  }
}

bool plane_fits(int n, int prec) { return prec == 0 ? plane_fits_t<double>(n) : plane_fits_t<float>(n); }

int energy_parts_per_pack(int n) {
  switch (n) {
#define X(N) \
  case N: return N * (N / line_chunk<N>());
    ACEX_SIZES(X)
#undef X
    default: return 0;
  }
}

// Forward plane workgroups resident per CU (registers and LDS permitting,
// up to three on the small grids): the persistent grid is that many per CU.
// One launch of 128 transforms, one against two or three per CU: FP32 48^3
// 83 -> 59 us, 64^3 92 -> 61 us; FP64 48^3 83 -> 66 us, 64^3 151 -> 123 us.
template <typename T, int N, bool ZXY>
static int fwd_per_cu() {
  static std::atomic<int> cached{0};
  const int v = cached.load(std::memory_order_relaxed);
  if (v > 0) return v;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_plane_fwd<T, N, ZXY>,
                                                   fwd_threads<N>(), 0) != hipSuccess ||
      occ < 1)
    occ = 1;
  cached.store(occ, std::memory_order_relaxed);
  return occ;
}

template <typename T, int N>
static hipError_t fwd_yz_t(const GridArgs& g, const void* phi, const Pack* packs, int npack,
                           void* S, bool zxy, hipStream_t s) {
  const cx<T>* tw = static_cast<const cx<T>*>(g.tw);
  if constexpr (fwd_slabs<T, N>()) {
    if (zxy)
      hipLaunchKernelGGL((k_slab_fwd<T, N, 2, true>), dim3(N * npack),
                         dim3(slab_threads<T, N, 2>()), 0, s, static_cast<const T*>(phi), packs,
                         tw, static_cast<cx<T>*>(S), npack, g.npts);
    else
      hipLaunchKernelGGL((k_slab_fwd<T, N, 2, false>), dim3(N * npack),
                         dim3(slab_threads<T, N, 2>()), 0, s, static_cast<const T*>(phi), packs,
                         tw, static_cast<cx<T>*>(S), npack, g.npts);
    return hipGetLastError();
  }
  if constexpr (plane_ok<T, N>()) {
    const int items = N * npack;
    const int cap = g.cus * (zxy ? fwd_per_cu<T, N, true>() : fwd_per_cu<T, N, false>());
    const int grid = items < cap ? ((items + 7) / 8) * 8 : cap;
    if (zxy)
      hipLaunchKernelGGL((k_plane_fwd<T, N, true>), dim3(grid), dim3(fwd_threads<N>()), 0, s,
                         static_cast<const T*>(phi), packs, tw, static_cast<cx<T>*>(S), npack,
                         g.npts);
    else
      hipLaunchKernelGGL((k_plane_fwd<T, N, false>), dim3(grid), dim3(fwd_threads<N>()), 0, s,
                         static_cast<const T*>(phi), packs, tw, static_cast<cx<T>*>(S), npack,
                         g.npts);
  } else if constexpr (slab_ok<T, N>()) {
    constexpr int SPW = slab_spw<T, N>(), SL = slab_count<T, N>();
    if (zxy) {
      if constexpr (slab3_ok<T, N>())
        hipLaunchKernelGGL((k_slab_fwd<T, N, SPW, true>), dim3(N * npack * (SL / SPW)),
                           dim3(slab_threads<T, N, SPW>()), 0, s, static_cast<const T*>(phi),
                           packs, tw, static_cast<cx<T>*>(S), npack, g.npts);
      else
        return hipErrorInvalidValue;
    } else {
      hipLaunchKernelGGL((k_slab_fwd<T, N, SPW, false>), dim3(N * npack * (SL / SPW)),
                         dim3(slab_threads<T, N, SPW>()), 0, s, static_cast<const T*>(phi),
                         packs, tw, static_cast<cx<T>*>(S), npack, g.npts);
    }
  } else {
    if (zxy) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_rows_fwd<T, N>), dim3((N * N / kRowsPerBlock) * npack),
                       dim3(row_threads<N>()), 0, s, static_cast<const T*>(phi), packs, tw,
                       static_cast<cx<T>*>(S), npack, g.npts);
    hipLaunchKernelGGL((k_lines<T, N, MODE_FWD, yline_chunk<N>()>),
                       dim3((N / yline_chunk<N>()) * N * npack),
                       dim3(line_threads<N, yline_chunk<N>()>()), 0, s, static_cast<cx<T>*>(S), tw, npack, g.npts,
                       (int64_t)N, (int64_t)N * N, T(0), T(0), T(0), T(0), (double*)nullptr);
  }
  return hipGetLastError();
}

// The slab inverse on the FP32 grids whose plane takes more than half of
// LDS: one 128-transform launch at 128^3 808 against 1016 us; at FP64 96^3
// and 80^3 the plane kernel already moves 5.2 TB/s and the slab form is no
// faster (713 / 695 us, 406 / 405), at FP32 96^3 slower (354 / 333).
template <typename T, int N>
constexpr bool inv_slabs() { return sizeof(T) == 4 && mid_slabs<T, N>(); }

template <typename T, int N>
static hipError_t inv_yz_t(const GridArgs& g, void* S, int npack, hipStream_t s) {
  const cx<T>* tw = static_cast<const cx<T>*>(g.tw);
  if constexpr (inv_slabs<T, N>()) {
    hipLaunchKernelGGL((k_slab_inv<T, N>), dim3(N * npack), dim3(512), 0, s,
                       static_cast<cx<T>*>(S), tw, npack, g.npts);
  } else if constexpr (plane_ok<T, N>()) {
    hipLaunchKernelGGL((k_plane_inv<T, N>), dim3(N * npack), dim3(plane_threads<N>()), 0, s,
                       static_cast<cx<T>*>(S), tw, npack, g.npts);
  } else {
    hipLaunchKernelGGL((k_lines<T, N, MODE_INV, yline_chunk<N>()>),
                       dim3((N / yline_chunk<N>()) * N * npack),
                       dim3(line_threads<N, yline_chunk<N>()>()), 0, s, static_cast<cx<T>*>(S), tw, npack, g.npts,
                       (int64_t)N, (int64_t)N * N, T(0), T(0), T(0), T(0), (double*)nullptr);
    hipLaunchKernelGGL((k_rows_inv<T, N>), dim3((N * N / kRowsPerBlock) * npack),
                       dim3(row_threads<N>()), 0, s, static_cast<cx<T>*>(S), tw, npack, g.npts);
  }
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t mid_t(const GridArgs& g, void* S, int npack, hipStream_t s) {
  if constexpr (mid_slabs<T, N>()) {
    constexpr int SL = slab_count<T, N>();
    hipLaunchKernelGGL((k_slab_mid<T, N>), dim3(N * npack), dim3(slab_threads<T, N, SL>()), 0,
                       s, static_cast<cx<T>*>(S), static_cast<const cx<T>*>(g.tw), npack, g.npts,
                       T(g.g2[0]), T(g.g2[1]), T(g.g2[2]), T(g.kscale));
    return hipGetLastError();
  } else if constexpr (plane_ok<T, N>()) {
    hipLaunchKernelGGL((k_plane_mid<T, N>), dim3(N * npack), dim3(plane_threads<N>()), 0, s,
                       static_cast<cx<T>*>(S), static_cast<const cx<T>*>(g.tw), npack, g.npts,
                       T(g.g2[0]), T(g.g2[1]), T(g.g2[2]), T(g.kscale));
    return hipGetLastError();
  } else if constexpr (slab3_ok<T, N>()) {
    constexpr int SL = slab_count<T, N>();
    hipLaunchKernelGGL((k_slab_mid<T, N>), dim3(N * npack), dim3(slab_threads<T, N, SL>()), 0,
                       s, static_cast<cx<T>*>(S), static_cast<const cx<T>*>(g.tw), npack, g.npts,
                       T(g.g2[0]), T(g.g2[1]), T(g.g2[2]), T(g.kscale));
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

template <typename T, int N, int B, bool ROWS>
static hipError_t zinv_launch(const GridArgs& g, bool diag, const void* S, const void* phi,
                              double* W, const int* orbs, double alpha, hipStream_t s,
                              const void* S2, const int* orbs2) {
  if constexpr (zinv_ok<T, N, B, ROWS>()) {
    const int nb = N * (N / zinv_rows<T, N, ROWS>());
    static_assert((N * (N / zinv_rows<T, N, ROWS>())) % 8 == 0, "whole XCD groups per tile");
    const dim3 grid(S2 ? 2 * nb : nb), block(zinv_threads<T, N, ROWS>());
    const cx<T>* s2 = static_cast<const cx<T>*>(S2 ? S2 : S);
    const int* o2 = S2 ? orbs2 : orbs;
    if (diag)
      hipLaunchKernelGGL((k_zinv_acc<T, N, B, true, ROWS>), grid, block, 0, s,
                         static_cast<const cx<T>*>(S), static_cast<const cx<T>*>(g.tw),
                         static_cast<const T*>(phi), W, orbs, alpha, g.npts, s2, o2, nb);
    else
      hipLaunchKernelGGL((k_zinv_acc<T, N, B, false, ROWS>), grid, block, 0, s,
                         static_cast<const cx<T>*>(S), static_cast<const cx<T>*>(g.tw),
                         static_cast<const T*>(phi), W, orbs, alpha, g.npts, s2, o2, nb);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

template <typename T, int N, int B>
static hipError_t zinv_t(const GridArgs& g, bool diag, const void* S, const void* phi,
                         double* W, const int* orbs, double alpha, hipStream_t s,
                         const void* S2, const int* orbs2) {
  if constexpr (zinv_ok<T, N, B, false>())
    return zinv_launch<T, N, B, false>(g, diag, S, phi, W, orbs, alpha, s, S2, orbs2);
  else
    return zinv_launch<T, N, B, true>(g, diag, S, phi, W, orbs, alpha, s, S2, orbs2);
}

// the large-grid schedule's inverse y lines (its inverse z is fused with W)
template <typename T, int N>
static hipError_t inv_y_t(const GridArgs& g, void* S, int npack, hipStream_t s) {
  if constexpr (!plane_ok<T, N>()) {
    hipLaunchKernelGGL((k_lines<T, N, MODE_INV, yline_chunk<N>()>),
                       dim3((N / yline_chunk<N>()) * N * npack),
                       dim3(line_threads<N, yline_chunk<N>()>()), 0, s, static_cast<cx<T>*>(S),
                       static_cast<const cx<T>*>(g.tw), npack, g.npts, (int64_t)N, (int64_t)N * N,
                       T(0), T(0), T(0), T(0), (double*)nullptr);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

template <typename T, int N, int MODE, int C>
static void x_launch(const GridArgs& g, void* S, int npack, double* part, hipStream_t s) {
  const cx<T>* tw = static_cast<const cx<T>*>(g.tw);
  hipLaunchKernelGGL((k_lines<T, N, MODE, C>), dim3((N / C) * N * npack),
                     dim3(line_threads<N, C>()), 0, s, static_cast<cx<T>*>(S), tw, npack, g.npts,
                     (int64_t)N * N, (int64_t)N, T(g.g2[0]), T(g.g2[1]), T(g.g2[2]),
                     T(g.kscale), part);
}

// The Poisson pass takes its pencils per workgroup from g.pencils (8, 16 or
// 32 where they divide N; anything else: the default); the energy pass keeps
// the default, which fixes its partial-sum layout.
template <typename T, int N, int MODE>
static hipError_t x_t(const GridArgs& g, void* S, int npack, double* part, hipStream_t s) {
  if constexpr (MODE == MODE_POISSON) {
    if constexpr (N % 8 == 0 && line_chunk<N>() != 8) {
      if (g.pencils == 8) {
        x_launch<T, N, MODE, 8>(g, S, npack, part, s);
        return hipGetLastError();
      }
    }
    if constexpr (N % 32 == 0) {
      if (g.pencils == 32) {
        x_launch<T, N, MODE, 32>(g, S, npack, part, s);
        return hipGetLastError();
      }
    }
  }
  x_launch<T, N, MODE, line_chunk<N>()>(g, S, npack, part, s);
  return hipGetLastError();
}

bool pencils_ok(int n, int pencils) {
  if (pencils == 0) return true;
  if (pencils != 8 && pencils != 16 && pencils != 32) return false;
  return n % pencils == 0;
}

hipError_t launch_fwd_yz(const GridArgs& g, const void* phi, const Pack* packs, int npack,
                         void* S, hipStream_t s, bool zxy) {
  if (npack <= 0) return hipSuccess;
  switch (g.n) {
#define X(N)                                                                   \
  case N:                                                                      \
    return g.prec == 0 ? fwd_yz_t<double, N>(g, phi, packs, npack, S, zxy, s)  \
                       : fwd_yz_t<float, N>(g, phi, packs, npack, S, zxy, s);
    ACEX_SIZES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

bool three_pass_ok(int n, int prec, int block) {
  switch (n) {
#define X(N)                                                                        \
  case N:                                                                           \
    if (block == 16) return prec == 0 ? zinv_ok<double, N, 16>() : zinv_ok<float, N, 16>(); \
    if (block == 8) return prec == 0 ? zinv_ok<double, N, 8>() : zinv_ok<float, N, 8>();    \
    return false;
    ACEX_SIZES(X)
#undef X
    default: return false;
  }
}

bool fused_rows_ok(int n, int prec, int block) {
  switch (n) {
#define X(N)                                                                                \
  case N:                                                                                   \
    if (block == 16)                                                                        \
      return prec == 0 ? zinv_ok<double, N, 16, true>() : zinv_ok<float, N, 16, true>();    \
    if (block == 8)                                                                         \
      return prec == 0 ? zinv_ok<double, N, 8, true>() : zinv_ok<float, N, 8, true>();      \
    return false;
    ACEX_SIZES(X)
#undef X
    default: return false;
  }
}

hipError_t launch_inv_y(const GridArgs& g, void* S, int npack, hipStream_t s) {
  if (npack <= 0) return hipSuccess;
  switch (g.n) {
#define X(N) \
  case N: return g.prec == 0 ? inv_y_t<double, N>(g, S, npack, s) : inv_y_t<float, N>(g, S, npack, s);
    ACEX_SIZES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_mid(const GridArgs& g, void* S, int npack, hipStream_t s) {
  if (npack <= 0) return hipSuccess;
  switch (g.n) {
#define X(N) \
  case N: return g.prec == 0 ? mid_t<double, N>(g, S, npack, s) : mid_t<float, N>(g, S, npack, s);
    ACEX_SIZES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_zinv_acc(const GridArgs& g, int block, bool diag, const void* S,
                           const void* phi, double* W, const int* orbs, double alpha,
                           hipStream_t s, const void* S2, const int* orbs2) {
  switch (g.n) {
#define X(N)                                                                                 \
  case N:                                                                                    \
    if (block == 16)                                                                         \
      return g.prec == 0 ? zinv_t<double, N, 16>(g, diag, S, phi, W, orbs, alpha, s, S2, orbs2) \
                         : zinv_t<float, N, 16>(g, diag, S, phi, W, orbs, alpha, s, S2, orbs2); \
    if (block == 8)                                                                          \
      return g.prec == 0 ? zinv_t<double, N, 8>(g, diag, S, phi, W, orbs, alpha, s, S2, orbs2)  \
                         : zinv_t<float, N, 8>(g, diag, S, phi, W, orbs, alpha, s, S2, orbs2);  \
    return hipErrorInvalidValue;
    ACEX_SIZES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_inv_yz(const GridArgs& g, void* S, int npack, hipStream_t s) {
  if (npack <= 0) return hipSuccess;
  switch (g.n) {
#define X(N) \
  case N: return g.prec == 0 ? inv_yz_t<double, N>(g, S, npack, s) : inv_yz_t<float, N>(g, S, npack, s);
    ACEX_SIZES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_poisson_x(const GridArgs& g, void* S, int npack, hipStream_t s) {
  if (npack <= 0) return hipSuccess;
  switch (g.n) {
#define X(N)                                                              \
  case N:                                                                 \
    return g.prec == 0 ? x_t<double, N, MODE_POISSON>(g, S, npack, nullptr, s) \
                       : x_t<float, N, MODE_POISSON>(g, S, npack, nullptr, s);
    ACEX_SIZES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_energy_x(const GridArgs& g, const void* S, int npack, double* part,
                           hipStream_t s) {
  if (npack <= 0) return hipSuccess;
  void* Sm = const_cast<void*>(S);
  switch (g.n) {
#define X(N)                                                             \
  case N:                                                                \
    return g.prec == 0 ? x_t<double, N, MODE_ENERGY>(g, Sm, npack, part, s) \
                       : x_t<float, N, MODE_ENERGY>(g, Sm, npack, part, s);
    ACEX_SIZES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

template <typename TS, int B>
static hipError_t acc_t(bool diag, const void* S, const void* phi_v, double* W, const int* meta,
                        int npack, const int* orbs, unsigned useI, unsigned useJ, double alpha,
                        int64_t npts, hipStream_t s) {
  const TS* phi = static_cast<const TS*>(phi_v);
  if (meta == nullptr) {
    const dim3 grid((unsigned)((npts + 255) / 256));
    if (diag)
      hipLaunchKernelGGL((k_accumulate_full<TS, B, true>), grid, dim3(256), 0, s,
                         static_cast<const cx<TS>*>(S), phi, W, orbs, alpha, npts);
    else
      hipLaunchKernelGGL((k_accumulate_full<TS, B, false>), grid, dim3(256), 0, s,
                         static_cast<const cx<TS>*>(S), phi, W, orbs, alpha, npts);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)((npts + kAccThreads - 1) / kAccThreads));
  if (diag)
    hipLaunchKernelGGL((k_accumulate<TS, B, true>), grid, dim3(kAccThreads), 0, s,
                       static_cast<const cx<TS>*>(S), phi, W, meta, npack, orbs, useI, useJ,
                       alpha, npts);
  else
    hipLaunchKernelGGL((k_accumulate<TS, B, false>), grid, dim3(kAccThreads), 0, s,
                       static_cast<const cx<TS>*>(S), phi, W, meta, npack, orbs, useI, useJ,
                       alpha, npts);
  return hipGetLastError();
}

hipError_t launch_accumulate(int prec, int block, bool diag, const void* S, const void* phi,
                             double* W, const int* meta, int npack, const int* orbs,
                             unsigned useI, unsigned useJ, double alpha, int64_t npts,
                             hipStream_t s) {
  if (block == 16)
    return prec == 0 ? acc_t<double, 16>(diag, S, phi, W, meta, npack, orbs, useI, useJ, alpha,
                                         npts, s)
                     : acc_t<float, 16>(diag, S, phi, W, meta, npack, orbs, useI, useJ, alpha,
                                        npts, s);
  if (block == 8)
    return prec == 0 ? acc_t<double, 8>(diag, S, phi, W, meta, npack, orbs, useI, useJ, alpha,
                                        npts, s)
                     : acc_t<float, 8>(diag, S, phi, W, meta, npack, orbs, useI, useJ, alpha,
                                       npts, s);
  return hipErrorInvalidValue;
}

hipError_t launch_energy_reduce(const double* part, int npack, int parts, double factor,
                                double* e_pack, hipStream_t s) {
  if (npack <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_energy_reduce, dim3(npack), dim3(256), 0, s, part, parts, factor, e_pack);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, double v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)blocks), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}

hipError_t launch_cast_f64_f32(const double* in, float* out, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_cast_f64_f32, dim3((unsigned)blocks), dim3(256), 0, s, in, out, count);
  return hipGetLastError();
}

}  // namespace acex
