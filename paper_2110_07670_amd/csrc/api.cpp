// Host runtime behind include/ace.h: plan, argument validation, the pair
// schedule and the stream-ordered launch sequence.  Every check runs on the
// host before the first device call, so argument errors are reported
// without a GPU.
#include "../../include/ace.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "kernels.h"

using acex::Pack;

namespace {

thread_local int g_last_hip = 0;
// set while this thread records a graph: stage timing events stay out of it
thread_local bool g_capturing = false;

constexpr double kTwoPi = 6.28318530717958647692;
constexpr int kBatchBranches = 4;  // concurrent graph branches of a batch

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Tile {
  int i0, j0, bi, bj;
  bool diag;
  int pack0, npack;
  unsigned useI, useJ;  // local orbitals with at least one kept pair
  bool complete;        // every pair of the tile kept: canonical pack order
};

struct ProfRec {
  int stage;
  hipEvent_t a, b;
};

}  // namespace

struct ace_plan {
  int n;
  double L[3];
  int n_orb;
  int prec;
  double alpha;
  int64_t npts;
  double omega, dV;
  int block;
  int chunk;
  int pencils;  // x-pass pencils per workgroup (0: the kernel's default)
  int schedule;  // ACE_SCHEDULE_AUTO or ACE_SCHEDULE_FOUR_PASS
  // workspace layout (bytes)
  size_t off_tab, tab_bytes, off_phi32, off_S, off_part, off_L, off_Linv, off_epart, off_epack,
      total;
  size_t s_grid_bytes;  // one complex grid of the bulk type
  size_t s_buf_bytes;   // one tile's transforms
  int max_pack_tile;
  int nsplit;
  int eparts;
  std::vector<unsigned char> tw_host;  // n twiddles in the bulk type
  bool profiling = false;
  std::mutex prof_mu;
  std::vector<ProfRec> prof;
};

namespace {
struct BuildTables {
  std::vector<unsigned char> host;  // packs | meta | twiddles | tile orbitals
  size_t o_packs = 0, o_meta = 0, o_tw = 0, o_orbs = 0, used = 0;
  std::vector<Tile> tiles;
  bool masked = false;
};
}  // namespace

namespace {
// Instances of a batch with one grid size, bulk precision and block whose full tiles
// run in shared persistent pass launches.  Round r takes tile r of every
// instance: the whole three-pass tiles as one launch per pass, the others
// (partial, masked, chunked) with the single-system kernels after them.
struct BatchLane {
  int prec = 0, n = 0, block = 0, branch = 0;
  double cost = 0.0;
  std::vector<int> inst;  // instances, largest first
  struct Round {
    size_t seg0 = 0;        // pass q's segments: seg0 + q nseg ...
    int nseg = 0;
    int total[3] = {0, 0, 0};
    int ctr = 0;            // pass q's queue counter: ctr + q
    std::vector<std::pair<int, int>> rest;  // (position in inst, tile)
  };
  std::vector<Round> rounds;
};
}  // namespace

struct ace_batch {
  int count = 0;
  std::vector<const ace_plan*> plans;
  std::vector<int> shape;             // (block, chunk, pencils, schedule) per plan at creation
  std::vector<BuildTables> tables;
  std::vector<size_t> ws_off;         // each instance's workspace slice
  size_t total = 0;
  std::vector<int> order;             // instances, largest first
  std::vector<int> branch;            // graph branch of each instance
  std::vector<int> branch_alone;      // its branch when every instance runs alone
  int nbranch = 0;
  int device = -1;
  hipStream_t cap = nullptr;          // capture stream
  std::vector<hipStream_t> streams;   // one per branch
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  unsigned char* pinned = nullptr;    // every instance's tables, back to back
  std::vector<size_t> pin_off;
  size_t pin_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> key;       // pointers the recorded graph was made for
  // the batch passes
  std::vector<char> fused;            // instance belongs to a lane
  std::vector<BatchLane> lanes;
  std::vector<acex::BatchSeg> segs;   // sizes and counts; pointers filled per call
  std::vector<std::pair<int, int>> seg_of;  // (instance, tile) of each segment
  size_t off_seg = 0, off_ctr = 0;    // in the workspace, after the instances
  int nctr = 0;
  acex::BatchSeg* seg_pinned = nullptr;
  hipEvent_t seg_ev = nullptr;        // the last upload of seg_pinned
  bool seg_pending = false;
  std::vector<const void*> seg_key;   // pointers seg_pinned holds
};

namespace {

int64_t n_pairs(int k) { return (int64_t)k * (k + 1) / 2; }

void layout(ace_plan* p) {
  const int B = p->block;
  const int nb = (p->n_orb + B - 1) / B;
  const int64_t ntiles = (int64_t)nb * (nb + 1) / 2;
  const int64_t npair = n_pairs(p->n_orb);
  const size_t bulk = p->prec == 0 ? sizeof(double) : sizeof(float);
  p->s_grid_bytes = align256((size_t)p->npts * 2 * bulk);
  p->max_pack_tile = (B * B + 1) / 2;
  p->nsplit = acex::gemm_abt_splits(p->n_orb, p->n_orb, p->npts);
  p->eparts = acex::energy_parts_per_pack(p->n);
  size_t off = 0;
  p->off_tab = off;
  p->tab_bytes = align256((size_t)ntiles * 2 * B * sizeof(int)) +
                 align256((size_t)npair * sizeof(Pack)) + align256((size_t)npair * sizeof(int)) +
                 align256((size_t)p->n * 2 * bulk) + align256((size_t)npair * sizeof(int)) +
                 align256((size_t)npair * sizeof(double));
  off += align256(p->tab_bytes);
  p->off_phi32 = off;
  if (p->prec == 1) off += align256((size_t)p->n_orb * p->npts * sizeof(float));
  p->off_S = off;
  // the transform scratch also holds the screening inputs of ace_screen_mask
  const size_t nn = (size_t)p->n_orb * p->n_orb;
  const size_t screen_bytes = nn * sizeof(double) + (size_t)p->n_orb * 10 * sizeof(double) +
                              nn * sizeof(float);
  // FP32 bulk: two tiles' transforms where full tiles take a fused
  // inverse-z/W pass (two disjoint tiles then share one launch of it)
  p->s_buf_bytes = align256(p->s_grid_bytes * (size_t)p->max_pack_tile);
  const size_t nbuf = (p->prec == ACE_FP32 && (acex::three_pass_ok(p->n, p->prec, B) ||
                                                acex::fused_rows_ok(p->n, p->prec, B)))
                          ? 2
                          : 1;
  off += std::max(p->s_buf_bytes * nbuf, align256(screen_bytes));
  p->off_part = off;
  off += align256((size_t)p->nsplit * p->n_orb * p->n_orb * sizeof(double));
  p->off_L = off;
  off += align256((size_t)p->n_orb * p->n_orb * sizeof(double));
  p->off_Linv = off;
  off += align256((size_t)p->n_orb * p->n_orb * sizeof(double));
  p->off_epart = off;
  off += align256((size_t)p->max_pack_tile * p->eparts * sizeof(double));
  p->off_epack = off;
  off += align256((size_t)npair * sizeof(double));
  p->total = off;
}

void make_twiddles(ace_plan* p) {
  const int n = p->n;
  p->tw_host.assign((size_t)n * 2 * (p->prec == 0 ? 8 : 4), 0);
  for (int k = 0; k < n; ++k) {
    const long double ang = -2.0L * 3.141592653589793238462643383279502884L * (long double)k / n;
    const long double c = std::cos(ang), s = std::sin(ang);
    if (p->prec == 0) {
      double* t = reinterpret_cast<double*>(p->tw_host.data());
      t[2 * k] = (double)c;
      t[2 * k + 1] = (double)s;
    } else {
      float* t = reinterpret_cast<float*>(p->tw_host.data());
      t[2 * k] = (float)c;
      t[2 * k + 1] = (float)s;
    }
  }
}

bool mask_on(const uint8_t* mask, int n_orb, int i, int j) {
  return mask == nullptr || mask[(size_t)i * n_orb + j] != 0;
}

// Orbital order for the pair tiles.  Without a mask: 0, 1, 2, ...  With a
// mask: greedy clusters of B orbitals joined by many kept pairs, so that the
// kept pairs of spatially close orbitals gather in few, dense tiles (a band
// order such as reverse Cuthill-McKee leaves the tiles of a 3-D system
// sparse: measured on the 512-orbital screen, 30% more orbital traffic in
// the W update and 7% more transforms).  A cluster starts at the unplaced
// orbital with the fewest unplaced partners (ties: lowest index) and grows
// by the unplaced orbital with the most kept pairs into the cluster (ties:
// fewest unplaced partners, then lowest index); when no unplaced orbital has
// a partner in the cluster, the start rule picks the next one.
std::vector<int> pair_order(int k, int B, const uint8_t* mask) {
  std::vector<int> ord;
  ord.reserve(k);
  if (!mask) {
    for (int i = 0; i < k; ++i) ord.push_back(i);
    return ord;
  }
  std::vector<std::vector<int>> adj(k);
  for (int i = 0; i < k; ++i)
    for (int j = i + 1; j < k; ++j)
      if (mask[(size_t)i * k + j]) {
        adj[i].push_back(j);
        adj[j].push_back(i);
      }
  std::vector<int> free_deg(k), conn(k, 0), cand;
  std::vector<char> placed(k, 0);
  for (int i = 0; i < k; ++i) free_deg[i] = (int)adj[i].size();
  auto place = [&](int v) {
    placed[v] = 1;
    ord.push_back(v);
    for (int w : adj[v]) {
      --free_deg[w];
      if (!placed[w] && conn[w]++ == 0) cand.push_back(w);
    }
  };
  auto start = [&]() {
    int best = -1;
    for (int v = 0; v < k; ++v)
      if (!placed[v] && (best < 0 || free_deg[v] < free_deg[best])) best = v;
    return best;
  };
  while ((int)ord.size() < k) {
    for (int w : cand) conn[w] = 0;  // partners counted per cluster
    cand.clear();
    place(start());
    for (int n = 1; n < B && (int)ord.size() < k; ++n) {
      int best = -1;
      for (int w : cand) {
        if (placed[w]) continue;
        if (best < 0 || conn[w] > conn[best] ||
            (conn[w] == conn[best] &&
             (free_deg[w] < free_deg[best] || (free_deg[w] == free_deg[best] && w < best))))
          best = w;
      }
      place(best >= 0 ? best : start());
    }
  }
  return ord;
}

// Pair tiles for ace_build: blocks of B consecutive orbitals of `ord`; tile
// (I, J), I <= J; pairs visited a-major inside a tile (local positions).  Two
// pairs share one transform only when they share their first orbital, (a, b)
// and (a, d) with d the next kept column of row a; a row's odd leftover is a
// single-pair transform.  meta receives, per transform, the local positions
// of its pairs (a0 | b0 << 8 | a1 << 16 | b1 << 24, a1 = 255 for a single
// pair); orbs receives, per kept tile, its 2B orbital indices (I list, then
// J list; -1 past a partial block).
// Block pairs (I, J), I <= J, in build order.  FP64 bulk: row by row, so
// that consecutive tiles share their first block's orbital rows in the
// last-level cache.  FP32 bulk: diagonal tiles, then the others, each kind
// row by row, except that each tile is followed by the first later tile of
// the same kind (diagonal or not, full or not) with no block in common, so
// that consecutive tiles can share one launch of the fused inverse-z/W pass
// (their W rows differ).  Measured at 96^3, 128 orbitals: FP32 201,700 to
// 206,700 pairs/s; FP64 127,400 to 123,300 (its forward pass loses more to
// the lost orbital reuse, 17.6 to 20.2 ms, than the paired W pass saves,
// 19.8 to 19.1 ms).
std::vector<std::pair<int, int>> tile_order(int nb, bool last_full, bool paired) {
  if (!paired) {
    std::vector<std::pair<int, int>> out;
    for (int I = 0; I < nb; ++I)
      for (int J = I; J < nb; ++J) out.emplace_back(I, J);
    return out;
  }
  std::vector<std::pair<int, int>> kinds[4];  // (diag, full) classes
  for (int I = 0; I < nb; ++I)
    for (int J = I; J < nb; ++J) {
      const bool full = last_full || (I < nb - 1 && J < nb - 1);
      kinds[(I == J ? 0 : 2) + (full ? 0 : 1)].emplace_back(I, J);
    }
  std::vector<std::pair<int, int>> out;
  for (auto& list : kinds) {
    std::vector<char> used(list.size(), 0);
    for (size_t a = 0; a < list.size(); ++a) {
      if (used[a]) continue;
      used[a] = 1;
      out.push_back(list[a]);
      for (size_t b = a + 1; b < list.size(); ++b) {
        const auto& x = list[a];
        const auto& y = list[b];
        if (!used[b] && x.first != y.first && x.first != y.second && x.second != y.first &&
            x.second != y.second) {
          used[b] = 1;
          out.push_back(y);
          break;
        }
      }
    }
  }
  return out;
}

void build_schedule(const ace_plan* p, const uint8_t* mask, std::vector<Pack>& packs,
                    std::vector<int>& meta, std::vector<int>& orbs, std::vector<Tile>& tiles) {
  const int B = p->block, k = p->n_orb;
  const int nb = (k + B - 1) / B;
  const std::vector<int> ord = pair_order(k, B, mask);
  packs.clear();
  tiles.clear();
  meta.clear();
  orbs.clear();
  for (const auto& IJ : tile_order(nb, k % B == 0, p->prec == ACE_FP32)) {
    {
      const int I = IJ.first, J = IJ.second;
      Tile t;
      t.i0 = I * B;
      t.j0 = J * B;
      t.bi = std::min(B, k - t.i0);
      t.bj = std::min(B, k - t.j0);
      t.diag = (I == J);
      t.pack0 = (int)packs.size();
      t.useI = t.useJ = 0u;
      int local = 0, kept = 0;
      for (int a = 0; a < t.bi; ++a) {
        int half = 0;
        Pack cur{-1, -1, -1, -1};
        int code = 0;
        for (int b = t.diag ? a : 0; b < t.bj; ++b) {
          const int i = ord[t.i0 + a], j = ord[t.j0 + b];
          if (!mask_on(mask, k, std::min(i, j), std::max(i, j))) continue;
          ++kept;
          t.useI |= 1u << a;
          if (t.diag) t.useI |= 1u << b;
          else t.useJ |= 1u << b;
          if (half == 0) {
            cur = Pack{i, j, -1, -1};
            code = a | (b << 8);
            half = 1;
          } else {
            cur.c = i;
            cur.d = j;
            packs.push_back(cur);
            meta.push_back(code | (a << 16) | (b << 24));
            ++local;
            half = 0;
          }
        }
        if (half == 1) {
          packs.push_back(cur);
          meta.push_back(code | (255 << 16));
          ++local;
        }
      }
      t.npack = local;
      t.complete = kept == (t.diag ? t.bi * (t.bi + 1) / 2 : t.bi * t.bj);
      if (t.npack > 0) {
        tiles.push_back(t);
        for (int a = 0; a < B; ++a) orbs.push_back(a < t.bi ? ord[t.i0 + a] : -1);
        for (int b = 0; b < B; ++b) orbs.push_back(b < t.bj ? ord[t.j0 + b] : -1);
      } else {
        packs.resize(t.pack0);
        meta.resize(t.pack0);
      }
    }
  }
}

// Energy schedule: off-diagonal pairs (i, j), (i, j') of one row share a
// transform (both halves then carry the weight 2); diagonal pairs are
// single-pair transforms.  One pair per transform when per-pair energies are
// wanted.
void build_energy_schedule(const ace_plan* p, const uint8_t* mask, bool single,
                           std::vector<Pack>& packs, std::vector<double>& weight,
                           std::vector<int>& code) {
  const int k = p->n_orb;
  packs.clear();
  weight.clear();
  code.clear();
  for (int i = 0; i < k; ++i) {
    if (mask_on(mask, k, i, i)) {
      packs.push_back(Pack{i, i, -1, -1});
      weight.push_back(-p->alpha);
      code.push_back(i * k + i);
    }
    int half = 0;
    Pack cur{-1, -1, -1, -1};
    for (int j = i + 1; j < k; ++j) {
      if (!mask_on(mask, k, i, j)) continue;
      if (single) {
        packs.push_back(Pack{i, j, -1, -1});
        weight.push_back(-2.0 * p->alpha);
        code.push_back(i * k + j);
        continue;
      }
      if (half == 0) {
        cur = Pack{i, j, -1, -1};
        half = 1;
      } else {
        cur.c = i;
        cur.d = j;
        packs.push_back(cur);
        weight.push_back(-2.0 * p->alpha);
        code.push_back(-1);
        half = 0;
      }
    }
    if (half == 1) {
      packs.push_back(cur);
      weight.push_back(-2.0 * p->alpha);
      code.push_back(-1);
    }
  }
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + nb && y < x + na;
}

int hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return ACE_ERR_HIP;
}

int device_present() {
  int count = 0;
  const hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    return 0;
  }
  return 1;
}

// Compute units of the current device, rounded down to a multiple of the 8
// XCDs (persistent grids keep a workgroup on one XCD).  Cached per device.
int device_cus() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cache[dev] == 0) {
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cu < 8)
      cu = 256;
    cache[dev] = (cu / 8) * 8;
  }
  return cache[dev];
}

struct ProfScope {
  ace_plan* p;
  int stage;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(const ace_plan* plan, int st, hipStream_t strm)
      : p(const_cast<ace_plan*>(plan)), stage(st), s(strm) {
    if (!p->profiling || g_capturing) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      a = b = nullptr;
      return;
    }
    (void)hipEventRecord(a, s);
  }
  ~ProfScope() {
    if (!a) return;
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> g(p->prof_mu);
    p->prof.push_back(ProfRec{stage, a, b});
  }
};

// ---------------------------------------------------------------- the build sequence

int check_build_args(const ace_plan* p, const void* ws, size_t ws_bytes, const double* phi,
                     const double* W, const double* M, const double* xi, const double* ex,
                     const int* info) {
  if (!p || !ws || !phi || !W || !M || !xi || !ex || !info) return ACE_ERR_ARG;
  const size_t orb_bytes = (size_t)p->n_orb * p->npts * sizeof(double);
  if (overlaps(phi, orb_bytes, W, orb_bytes) || overlaps(phi, orb_bytes, xi, orb_bytes) ||
      overlaps(W, orb_bytes, xi, orb_bytes))
    return ACE_ERR_ARG;
  if (ws_bytes < p->total) return ACE_ERR_WORKSPACE;
  return ACE_OK;
}

// A0: the pair schedule and the tables the kernels read, built on the host.
int prepare_tables(const ace_plan* p, const uint8_t* pair_mask, BuildTables& bt) {
  std::vector<Pack> packs;
  std::vector<int> meta;
  std::vector<int> orbs;
  build_schedule(p, pair_mask, packs, meta, orbs, bt.tiles);
  bt.masked = pair_mask != nullptr;
  const size_t bulk = p->prec == 0 ? 8 : 4;
  bt.o_packs = 0;
  bt.o_meta = bt.o_packs + align256(std::max<size_t>(packs.size(), 1) * sizeof(Pack));
  bt.o_tw = bt.o_meta + align256(std::max<size_t>(meta.size(), 1) * sizeof(int));
  bt.o_orbs = bt.o_tw + align256((size_t)p->n * 2 * bulk);
  bt.used = bt.o_orbs + align256(std::max<size_t>(orbs.size(), 1) * sizeof(int));
  if (bt.used > p->tab_bytes) return ACE_ERR_SIZE;
  bt.host.assign(bt.used, 0);
  if (!packs.empty())
    std::memcpy(bt.host.data() + bt.o_packs, packs.data(), packs.size() * sizeof(Pack));
  if (!meta.empty()) std::memcpy(bt.host.data() + bt.o_meta, meta.data(), meta.size() * sizeof(int));
  std::memcpy(bt.host.data() + bt.o_tw, p->tw_host.data(), p->tw_host.size());
  if (!orbs.empty()) std::memcpy(bt.host.data() + bt.o_orbs, orbs.data(), orbs.size() * sizeof(int));
  return ACE_OK;
}

// One stream-ordered copy of the tables into the workspace.  The source is
// pageable host memory, which the runtime stages before the call returns.
int upload_tables(const ace_plan* p, hipStream_t s, char* w, const BuildTables& bt) {
  ProfScope ps(p, 7, s);
  const hipError_t e =
      hipMemcpyAsync(w + p->off_tab, bt.host.data(), bt.used, hipMemcpyHostToDevice, s);
  return e == hipSuccess ? ACE_OK : hip_fail(e);
}

// One build's launch context: the plan, its workspace and tables, the grid
// arguments and the orbitals in the bulk precision.
struct BuildCtx {
  const ace_plan* p = nullptr;
  char* w = nullptr;
  const BuildTables* bt = nullptr;
  acex::GridArgs g;
  const void* phi_bulk = nullptr;
  const Pack* d_packs = nullptr;
  const int* d_meta = nullptr;
  const int* d_orbs = nullptr;
  bool three_ok = false, rows_ok = false;
};

// Launch arguments and the W / FP32-copy prologue of a build on stream s,
// reading tables already resident in the workspace.
int build_begin(const ace_plan* p, hipStream_t s, char* w, const double* phi,
                const BuildTables& bt, double* W, BuildCtx& c) {
  hipError_t e;
  c.p = p;
  c.w = w;
  c.bt = &bt;
  c.d_packs = reinterpret_cast<const Pack*>(w + p->off_tab + bt.o_packs);
  c.d_meta = reinterpret_cast<const int*>(w + p->off_tab + bt.o_meta);
  c.d_orbs = reinterpret_cast<const int*>(w + p->off_tab + bt.o_orbs);
  acex::GridArgs& g = c.g;
  g.n = p->n;
  g.prec = p->prec;
  g.npts = p->npts;
  for (int a = 0; a < 3; ++a) g.g2[a] = (kTwoPi / p->L[a]) * (kTwoPi / p->L[a]);
  g.kscale = 1.0 / (double)p->npts;
  g.tw = w + p->off_tab + bt.o_tw;
  g.cus = device_cus();
  g.pencils = p->pencils;
  const bool fuse_ok = p->schedule == ACE_SCHEDULE_AUTO;
  c.three_ok = fuse_ok && acex::three_pass_ok(p->n, p->prec, p->block);
  c.rows_ok = fuse_ok && acex::fused_rows_ok(p->n, p->prec, p->block);
  c.phi_bulk = phi;
  ProfScope ps(p, 7, s);
  if (p->prec == 1) {
    e = acex::launch_cast_f64_f32(phi, reinterpret_cast<float*>(w + p->off_phi32),
                                  (int64_t)p->n_orb * p->npts, s);
    if (e != hipSuccess) return hip_fail(e);
    c.phi_bulk = w + p->off_phi32;
  }
  e = acex::launch_fill_f64(W, 0.0, (int64_t)p->n_orb * p->npts, s);
  if (e != hipSuccess) return hip_fail(e);
  return ACE_OK;
}

// Does the tile take the three-pass schedule as one launch per pass, with a
// grid the batch kernels run?
bool tile_batch_whole(const ace_plan* p, const Tile& t) {
  const int B = p->block;
  return p->schedule == ACE_SCHEDULE_AUTO && acex::batch_ok(p->n, p->prec, B) && t.bi == B &&
         t.bj == B && t.complete && (p->chunk == 0 || p->chunk >= t.npack);
}

// A1-A4 for tile ti: pair densities and Poisson solves into scratch S
// (forward and middle passes; four-pass tiles also x and the inverse y/z).
// Full tiles take three passes where the kernels fit (the inverse z
// transform then feeds the W update directly); the others take four.
int tile_transforms(const BuildCtx& c, hipStream_t s, size_t ti, void* S) {
  hipError_t e;
  const ace_plan* p = c.p;
  const acex::GridArgs& g = c.g;
  const int B = p->block;
  const Tile& t = c.bt->tiles[ti];
  // a full block x block tile with every pair kept (masked builds too)
  const bool full = t.bi == B && t.bj == B && t.complete;
  const bool three = c.three_ok && full;           // plane-fitting grids
  const bool fused = (c.three_ok || c.rows_ok) && full;
  const int chunk = p->chunk > 0 ? p->chunk : t.npack;
  for (int c0 = 0; c0 < t.npack; c0 += chunk) {
    const int cnt = std::min(chunk, t.npack - c0);
    void* Sc = static_cast<char*>(S) + (size_t)c0 * p->s_grid_bytes;
    {
      ProfScope ps(p, 0, s);
      e = acex::launch_fwd_yz(g, c.phi_bulk, c.d_packs + t.pack0 + c0, cnt, Sc, s, three);
      if (e != hipSuccess) return hip_fail(e);
    }
    {
      ProfScope ps(p, 1, s);
      e = three ? acex::launch_mid(g, Sc, cnt, s) : acex::launch_poisson_x(g, Sc, cnt, s);
      if (e != hipSuccess) return hip_fail(e);
    }
    if (!three) {
      ProfScope ps(p, 2, s);
      e = fused ? acex::launch_inv_y(g, Sc, cnt, s) : acex::launch_inv_yz(g, Sc, cnt, s);
      if (e != hipSuccess) return hip_fail(e);
    }
  }
  return ACE_OK;
}

// Does tile ti take the fused inverse-z/W pass?
bool tile_fused(const BuildCtx& c, size_t ti) {
  const Tile& t = c.bt->tiles[ti];
  const int B = c.p->block;
  return (c.three_ok || c.rows_ok) && t.bi == B && t.bj == B && t.complete;
}

// A5 for tile ti (and, with S2, a second fused tile tj of the same kind and
// no block in common, in the same launch): the W update from the
// transforms in scratch.
int tile_accumulate(const BuildCtx& c, hipStream_t s, size_t ti, const void* S, double* W,
                    size_t tj = 0, const void* S2 = nullptr) {
  hipError_t e;
  const ace_plan* p = c.p;
  const acex::GridArgs& g = c.g;
  const int B = p->block;
  const Tile& t = c.bt->tiles[ti];
  const bool full = t.bi == B && t.bj == B && t.complete;
  const int* t_orbs = c.d_orbs + ti * (size_t)2 * B;
  ProfScope ps(p, 3, s);
  if (tile_fused(c, ti)) {
    e = acex::launch_zinv_acc(g, B, t.diag, S, c.phi_bulk, W, t_orbs, p->alpha, s, S2,
                              S2 ? c.d_orbs + tj * (size_t)2 * B : nullptr);
  } else {
    e = acex::launch_accumulate(p->prec, B, t.diag, S, c.phi_bulk, W,
                                full ? nullptr : c.d_meta + t.pack0, t.npack, t_orbs, t.useI,
                                t.useJ, p->alpha, p->npts, s);
  }
  return e == hipSuccess ? ACE_OK : hip_fail(e);
}

// A1-A5 for tile ti alone, in the first scratch buffer.
int build_tile(const BuildCtx& c, hipStream_t s, size_t ti, double* W) {
  void* S = c.w + c.p->off_S;
  const int rc = tile_transforms(c, s, ti, S);
  return rc != ACE_OK ? rc : tile_accumulate(c, s, ti, S, W);
}

// Can tiles ti and ti + 1 share one fused-pass launch?
bool tiles_pair(const BuildCtx& c, size_t ti) {
  const std::vector<Tile>& tl = c.bt->tiles;
  if (ti + 1 >= tl.size() || !tile_fused(c, ti) || !tile_fused(c, ti + 1)) return false;
  const Tile& a = tl[ti];
  const Tile& b = tl[ti + 1];
  return a.diag == b.diag && a.i0 != b.i0 && a.i0 != b.j0 && a.j0 != b.i0 && a.j0 != b.j0 &&
         c.p->s_buf_bytes > 0 && c.p->off_part - c.p->off_S >= 2 * c.p->s_buf_bytes;
}

// A6-A10 once W is complete: M, the Cholesky factor and its inverse, xi, E_x.
int build_end(const ace_plan* p, hipStream_t s, char* w, const double* phi, double* W, double* M,
              double* xi, double* ex, int* info) {
  hipError_t e;
  // ---- A6: M = dV Phi^T W
  double* part = reinterpret_cast<double*>(w + p->off_part);
  {
    ProfScope ps(p, 4, s);
    e = acex::launch_gemm_abt(phi, W, p->n_orb, p->n_orb, p->npts, p->dV, M, part, p->nsplit,
                              false, nullptr, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  // ---- A7: -M = L L^T, L^{-1}
  double* L = reinterpret_cast<double*>(w + p->off_L);
  double* Linv = reinterpret_cast<double*>(w + p->off_Linv);
  {
    ProfScope ps(p, 5, s);
    e = acex::launch_cholesky_inv(M, p->n_orb, L, Linv, info, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  // ---- A8: xi = W L^{-T}, i.e. xi_k = sum_i Linv[k][i] W_i
  {
    ProfScope ps(p, 6, s);
    e = acex::launch_gemm_ab(Linv, W, p->n_orb, p->n_orb, p->npts, 1.0, xi, info, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  // ---- A10: E_x = tr(M)
  {
    ProfScope ps(p, 7, s);
    e = acex::launch_trace(M, p->n_orb, ex, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  return ACE_OK;
}

// A1-A10 on stream s, reading tables already resident in the workspace.
int enqueue_build(const ace_plan* p, hipStream_t s, char* w, const double* phi,
                  const BuildTables& bt, double* W, double* M, double* xi, double* ex, int* info) {
  BuildCtx c;
  int rc = build_begin(p, s, w, phi, bt, W, c);
  if (rc != ACE_OK) return rc;
  for (size_t ti = 0; ti < bt.tiles.size(); ++ti) {
    if (tiles_pair(c, ti)) {
      // both tiles' transforms, then one fused-pass launch for the two
      void* S0 = w + p->off_S;
      void* S1 = w + p->off_S + p->s_buf_bytes;
      if ((rc = tile_transforms(c, s, ti, S0)) != ACE_OK) return rc;
      if ((rc = tile_transforms(c, s, ti + 1, S1)) != ACE_OK) return rc;
      if ((rc = tile_accumulate(c, s, ti, S0, W, ti + 1, S1)) != ACE_OK) return rc;
      ++ti;
      continue;
    }
    rc = build_tile(c, s, ti, W);
    if (rc != ACE_OK) return rc;
  }
  return build_end(p, s, w, phi, W, M, xi, ex, info);
}

}  // namespace

// ------------------------------------------------------------------ the apply, shared
// by ace_apply (scratch in the caller's workspace) and ace_apply_noalloc
// (scratch in the library's static device array).

namespace acex {

int apply_check(const ace_plan* p, const double* xi, const double* psi, int n_vec,
                const double* out) {
  if (!p || !xi || !psi || !out) return ACE_ERR_ARG;
  if (n_vec < 1) return ACE_ERR_ARG;
  const size_t xi_bytes = (size_t)p->n_orb * p->npts * sizeof(double);
  const size_t v_bytes = (size_t)n_vec * p->npts * sizeof(double);
  if (overlaps(out, v_bytes, xi, xi_bytes) || overlaps(out, v_bytes, psi, v_bytes))
    return ACE_ERR_ARG;
  return ACE_OK;
}

int apply_splits(const ace_plan* p, int n_vec) {
  return gemm_abt_splits(n_vec, p->n_orb, p->npts);
}

int apply_orbitals(const ace_plan* p) { return p->n_orb; }

int apply_enqueue(const ace_plan* p, hipStream_t s, double* C, double* part, int ns,
                  const double* xi, const double* psi, int n_vec, double* out) {
  ProfScope ps(p, 8, s);
  // C[v][k] = dV <psi_v, xi_k>
  hipError_t e = launch_gemm_abt(psi, xi, n_vec, p->n_orb, p->npts, p->dV, C, part, ns, false,
                                 nullptr, s);
  if (e != hipSuccess) return hip_fail(e);
  // out[v] = -sum_k C[v][k] xi_k
  e = launch_gemm_ab(C, xi, n_vec, p->n_orb, p->npts, -1.0, out, nullptr, s);
  if (e != hipSuccess) return hip_fail(e);
  return ACE_OK;
}

int apply_device_present() { return device_present(); }

int apply_hip_fail(hipError_t e) { return hip_fail(e); }

}  // namespace acex

// ====================================================================== C-ABI

extern "C" {

const char* ace_error_string(int code) {
  switch (code) {
    case ACE_OK: return "ok";
    case ACE_ERR_ARG: return "invalid argument";
    case ACE_ERR_SIZE: return "unsupported size";
    case ACE_ERR_WORKSPACE: return "workspace too small";
    case ACE_ERR_HIP: return "HIP runtime error";
    case ACE_ERR_NODEV: return "no HIP device";
    default: return "unknown status";
  }
}

int ace_last_hip_error(void) { return g_last_hip; }

int ace_plan_create(ace_plan** plan, const ace_desc* d) {
  if (!plan || !d) return ACE_ERR_ARG;
  *plan = nullptr;
  if (d->n_orb < 1) return ACE_ERR_ARG;
  for (int a = 0; a < 3; ++a)
    if (!(d->cell[a] > 0.0) || !std::isfinite(d->cell[a])) return ACE_ERR_ARG;
  if (d->precision != ACE_FP64 && d->precision != ACE_FP32) return ACE_ERR_ARG;
  if (!std::isfinite(d->alpha)) return ACE_ERR_ARG;
  if (d->n[0] != d->n[1] || d->n[1] != d->n[2]) return ACE_ERR_SIZE;
  if (!acex::supported_n(d->n[0])) return ACE_ERR_SIZE;
  if (d->n_orb > 512) return ACE_ERR_SIZE;
  ace_plan* p = new ace_plan();
  p->n = d->n[0];
  for (int a = 0; a < 3; ++a) p->L[a] = d->cell[a];
  p->n_orb = d->n_orb;
  p->prec = d->precision;
  p->alpha = d->alpha;
  p->npts = (int64_t)p->n * p->n * p->n;
  p->omega = d->cell[0] * d->cell[1] * d->cell[2];
  p->dV = p->omega / (double)p->npts;
  // block 16, unless only block 8 has the three-pass schedule on this grid
  p->block = (!acex::three_pass_ok(p->n, p->prec, 16) && acex::three_pass_ok(p->n, p->prec, 8))
                 ? 8
                 : 16;
  p->chunk = 0;
  p->pencils = 0;
  p->schedule = ACE_SCHEDULE_AUTO;
  layout(p);
  make_twiddles(p);
  *plan = p;
  return ACE_OK;
}

void ace_plan_destroy(ace_plan* plan) {
  if (!plan) return;
  for (auto& r : plan->prof) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  delete plan;
}

size_t ace_workspace_bytes(const ace_plan* plan) { return plan ? plan->total : 0; }

size_t ace_apply_workspace_bytes(const ace_plan* plan, int n_vec) {
  if (!plan || n_vec < 1) return 0;
  const int ns = acex::gemm_abt_splits(n_vec, plan->n_orb, plan->npts);
  return align256((size_t)n_vec * plan->n_orb * sizeof(double)) +
         align256((size_t)ns * n_vec * plan->n_orb * sizeof(double));
}

int ace_plan_set_tiling(ace_plan* plan, int block, int chunk, int pencils) {
  if (!plan) return ACE_ERR_ARG;
  if (block != 8 && block != 16) return ACE_ERR_ARG;
  if (chunk < 0) return ACE_ERR_ARG;
  if (!acex::pencils_ok(plan->n, pencils)) return ACE_ERR_ARG;
  plan->block = block;
  plan->chunk = chunk;
  plan->pencils = pencils;
  layout(plan);
  return ACE_OK;
}

int ace_plan_tiling(const ace_plan* plan, int* block, int* chunk, int* pencils) {
  if (!plan) return ACE_ERR_ARG;
  if (block) *block = plan->block;
  if (chunk) *chunk = plan->chunk;
  if (pencils) *pencils = plan->pencils;
  return ACE_OK;
}

int ace_plan_schedule(const ace_plan* plan, int* full_tiles, int* plane) {
  if (!plan) return ACE_ERR_ARG;
  const bool fuse_ok = plan->schedule == ACE_SCHEDULE_AUTO;
  int kind = ACE_TILES_FOUR_PASS;
  if (fuse_ok && acex::three_pass_ok(plan->n, plan->prec, plan->block))
    kind = ACE_TILES_THREE_PASS;
  else if (fuse_ok && acex::fused_rows_ok(plan->n, plan->prec, plan->block))
    kind = ACE_TILES_ROWS_FUSED;
  if (full_tiles) *full_tiles = kind;
  if (plane) *plane = acex::plane_fits(plan->n, plan->prec) ? 1 : 0;
  return ACE_OK;
}

int ace_plan_set_schedule(ace_plan* plan, int schedule) {
  if (!plan) return ACE_ERR_ARG;
  if (schedule != ACE_SCHEDULE_AUTO && schedule != ACE_SCHEDULE_FOUR_PASS) return ACE_ERR_ARG;
  plan->schedule = schedule;
  return ACE_OK;
}

int ace_set_profiling(ace_plan* plan, int on) {
  if (!plan) return ACE_ERR_ARG;
  plan->profiling = on != 0;
  return ACE_OK;
}

int ace_profile_read(ace_plan* plan, double* out_ms, int* out_count) {
  if (!plan || !out_ms || !out_count) return ACE_ERR_ARG;
  for (int i = 0; i < ACE_N_STAGES; ++i) {
    out_ms[i] = 0.0;
    out_count[i] = 0;
  }
  std::lock_guard<std::mutex> g(plan->prof_mu);
  int rc = ACE_OK;
  for (auto& r : plan->prof) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) rc = hip_fail(e);
    if (r.stage >= 0 && r.stage < ACE_N_STAGES) {
      out_ms[r.stage] += ms;
      out_count[r.stage] += 1;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  plan->prof.clear();
  return rc;
}

int ace_build(const ace_plan* p, void* stream, void* ws, size_t ws_bytes, const double* phi,
              const uint8_t* pair_mask, double* W, double* M, double* xi, double* ex, int* info) {
  int rc = check_build_args(p, ws, ws_bytes, phi, W, M, xi, ex, info);
  if (rc != ACE_OK) return rc;
  if (!device_present()) return ACE_ERR_NODEV;
  BuildTables bt;
  rc = prepare_tables(p, pair_mask, bt);
  if (rc != ACE_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  rc = upload_tables(p, s, static_cast<char*>(ws), bt);
  if (rc != ACE_OK) return rc;
  return enqueue_build(p, s, static_cast<char*>(ws), phi, bt, W, M, xi, ex, info);
}

int ace_apply(const ace_plan* p, void* stream, void* ws, size_t ws_bytes, const double* xi,
              const double* psi, int n_vec, double* out) {
  int rc = acex::apply_check(p, xi, psi, n_vec, out);
  if (rc != ACE_OK) return rc;
  if (!ws) return ACE_ERR_ARG;
  if (ws_bytes < ace_apply_workspace_bytes(p, n_vec)) return ACE_ERR_WORKSPACE;
  if (!device_present()) return ACE_ERR_NODEV;
  char* w = static_cast<char*>(ws);
  double* C = reinterpret_cast<double*>(w);
  double* part = reinterpret_cast<double*>(w + align256((size_t)n_vec * p->n_orb * sizeof(double)));
  return acex::apply_enqueue(p, static_cast<hipStream_t>(stream), C, part,
                             acex::apply_splits(p, n_vec), xi, psi, n_vec, out);
}

int exx_energy(const ace_plan* p, void* stream, void* ws, size_t ws_bytes, const double* phi,
               const uint8_t* pair_mask, double* ex, double* pair_e) {
  if (!p || !ws || !phi || !ex) return ACE_ERR_ARG;
  if (ws_bytes < p->total) return ACE_ERR_WORKSPACE;
  if (!device_present()) return ACE_ERR_NODEV;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  hipError_t e;
  std::vector<Pack> packs;
  std::vector<double> weight;
  std::vector<int> code;
  build_energy_schedule(p, pair_mask, pair_e != nullptr, packs, weight, code);
  const int np = (int)packs.size();
  const size_t bulk = p->prec == 0 ? 8 : 4;
  const size_t o_packs = 0;
  const size_t o_tw = o_packs + align256(std::max<size_t>(np, 1) * sizeof(Pack));
  const size_t o_w = o_tw + align256((size_t)p->n * 2 * bulk);
  const size_t o_code = o_w + align256(std::max<size_t>(np, 1) * sizeof(double));
  const size_t tab_used = o_code + align256(std::max<size_t>(np, 1) * sizeof(int));
  if (tab_used > p->tab_bytes) return ACE_ERR_SIZE;
  std::vector<unsigned char> host(tab_used, 0);
  if (np) {
    std::memcpy(host.data() + o_packs, packs.data(), (size_t)np * sizeof(Pack));
    std::memcpy(host.data() + o_w, weight.data(), (size_t)np * sizeof(double));
    std::memcpy(host.data() + o_code, code.data(), (size_t)np * sizeof(int));
  }
  std::memcpy(host.data() + o_tw, p->tw_host.data(), p->tw_host.size());
  {
    ProfScope ps(p, 7, s);
    e = hipMemcpyAsync(w + p->off_tab, host.data(), tab_used, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  const Pack* d_packs = reinterpret_cast<const Pack*>(w + p->off_tab + o_packs);
  const double* d_w = reinterpret_cast<const double*>(w + p->off_tab + o_w);
  const int* d_code = reinterpret_cast<const int*>(w + p->off_tab + o_code);
  acex::GridArgs g;
  g.n = p->n;
  g.prec = p->prec;
  g.npts = p->npts;
  for (int a = 0; a < 3; ++a) g.g2[a] = (kTwoPi / p->L[a]) * (kTwoPi / p->L[a]);
  g.kscale = 1.0;
  g.tw = w + p->off_tab + o_tw;
  g.cus = device_cus();
  const void* phi_bulk = phi;
  if (p->prec == 1) {
    ProfScope ps(p, 7, s);
    e = acex::launch_cast_f64_f32(phi, reinterpret_cast<float*>(w + p->off_phi32),
                                  (int64_t)p->n_orb * p->npts, s);
    if (e != hipSuccess) return hip_fail(e);
    phi_bulk = w + p->off_phi32;
  }
  void* S = w + p->off_S;
  double* epart = reinterpret_cast<double*>(w + p->off_epart);
  double* epack = reinterpret_cast<double*>(w + p->off_epack);
  const double factor = p->omega / ((double)p->npts * (double)p->npts);
  const int chunk = p->max_pack_tile;
  for (int c0 = 0; c0 < np; c0 += chunk) {
    const int cnt = std::min(chunk, np - c0);
    {
      ProfScope ps(p, 0, s);
      e = acex::launch_fwd_yz(g, phi_bulk, d_packs + c0, cnt, S, s);
      if (e != hipSuccess) return hip_fail(e);
    }
    {
      ProfScope ps(p, 9, s);
      e = acex::launch_energy_x(g, S, cnt, epart, s);
      if (e != hipSuccess) return hip_fail(e);
      e = acex::launch_energy_reduce(epart, cnt, p->eparts, factor, epack + c0, s);
      if (e != hipSuccess) return hip_fail(e);
    }
  }
  ProfScope ps(p, 7, s);
  if (np == 0) {
    e = acex::launch_fill_f64(ex, 0.0, 1, s);
  } else {
    e = acex::launch_weighted_sum(epack, d_w, np, ex, s);
  }
  if (e != hipSuccess) return hip_fail(e);
  if (pair_e && np) {
    e = acex::launch_scatter_pair_energies(epack, d_code, np, p->n_orb, -p->alpha, pair_e, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  return ACE_OK;
}

int ace_wannier(const ace_plan* p, void* stream, const double* phi, double* z, double* feat) {
  if (!p || !phi || !z || !feat) return ACE_ERR_ARG;
  if (!device_present()) return ACE_ERR_NODEV;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = acex::launch_moments(phi, p->n, p->n_orb, p->npts, p->dV, z, s);
  if (e != hipSuccess) return hip_fail(e);
  e = acex::launch_wannier_features(z, p->n_orb, p->L, feat, s);
  if (e != hipSuccess) return hip_fail(e);
  return ACE_OK;
}

int ace_overlap_integrals(const ace_plan* p, void* stream, void* ws, size_t ws_bytes,
                          const double* phi, double* S) {
  if (!p || !ws || !phi || !S) return ACE_ERR_ARG;
  if (ws_bytes < p->total) return ACE_ERR_WORKSPACE;
  if (!device_present()) return ACE_ERR_NODEV;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* part = reinterpret_cast<double*>(static_cast<char*>(ws) + p->off_part);
  const hipError_t e = acex::launch_gemm_abt(phi, phi, p->n_orb, p->n_orb, p->npts, p->dV, S, part,
                                             p->nsplit, true, nullptr, s);
  if (e != hipSuccess) return hip_fail(e);
  return ACE_OK;
}

int ace_mlp_weight_count(void) { return acex::mlp_weight_count(); }

int ace_mlp_screen(const ace_plan* p, void* stream, const double* feat, const float* weights,
                   float* pred) {
  if (!p || !feat || !weights || !pred) return ACE_ERR_ARG;
  if (!device_present()) return ACE_ERR_NODEV;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const hipError_t e = acex::launch_mlp_pairs(feat, p->n_orb, p->L, weights, pred, s);
  if (e != hipSuccess) return hip_fail(e);
  return ACE_OK;
}

// ------------------------------------------------------------------ screening decision

int ace_screen_mask_host(int n, const ace_screen_desc* d, const double* S, const float* pred,
                         uint8_t* mask, ace_screen_report* rep) {
  if (!d || !mask || !rep || n < 1) return ACE_ERR_ARG;
  if (d->kind != ACE_SCREEN_OVERLAP && d->kind != ACE_SCREEN_MLP) return ACE_ERR_ARG;
  if (!(d->budget >= 0.0) || !(d->safety >= 1.0)) return ACE_ERR_ARG;
  if (d->kind == ACE_SCREEN_OVERLAP && !S) return ACE_ERR_ARG;
  if (d->kind == ACE_SCREEN_MLP && !pred) return ACE_ERR_ARG;
  const size_t nn = (size_t)n * n;
  std::memset(mask, 0, nn);
  for (int i = 0; i < n; ++i) mask[(size_t)i * n + i] = 1;
  // predicted |e_ij| of the off-diagonal pairs, upper triangle in row order
  auto energy = [&](int i, int j) { return std::pow(10.0, (double)pred[(size_t)i * n + j]); };
  double skipped = 0.0;
  if (d->kind == ACE_SCREEN_OVERLAP) {
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) {
        if (S[(size_t)i * n + j] >= d->rho_cut) mask[(size_t)i * n + j] = 1;
        else if (pred) skipped += energy(i, j);
      }
  } else {
    std::vector<std::pair<double, int64_t>> e;
    e.reserve((size_t)n * (n - 1) / 2);
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) e.push_back({energy(i, j), (int64_t)i * n + j});
    // smallest first; ties in row order
    std::stable_sort(e.begin(), e.end(),
                     [](const std::pair<double, int64_t>& x, const std::pair<double, int64_t>& y) {
                       return x.first < y.first;
                     });
    const double limit = d->budget / d->safety;
    size_t k = 0;
    for (; k < e.size(); ++k) {
      if (skipped + e[k].first > limit) break;
      skipped += e[k].first;
    }
    for (size_t q = k; q < e.size(); ++q) mask[e[q].second] = 1;
  }
  rep->pairs_total = (int64_t)n * (n + 1) / 2;
  rep->predicted_skipped = pred ? skipped : std::nan("");
  rep->fallback = (pred && skipped > d->budget) ? 1 : 0;
  if (rep->fallback)
    for (int i = 0; i < n; ++i)
      for (int j = i; j < n; ++j) mask[(size_t)i * n + j] = 1;
  int64_t kept = 0;
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) kept += mask[(size_t)i * n + j];
  rep->pairs_kept = kept;
  return ACE_OK;
}

int ace_screen_mask(const ace_plan* p, void* stream, void* ws, size_t ws_bytes, const double* phi,
                    const ace_screen_desc* d, uint8_t* mask, ace_screen_report* rep) {
  if (!p || !ws || !phi || !d || !mask || !rep) return ACE_ERR_ARG;
  if (d->kind != ACE_SCREEN_OVERLAP && d->kind != ACE_SCREEN_MLP) return ACE_ERR_ARG;
  if (d->kind == ACE_SCREEN_MLP && !d->mlp_weights) return ACE_ERR_ARG;
  if (!(d->budget >= 0.0) || !(d->safety >= 1.0)) return ACE_ERR_ARG;
  if (ws_bytes < p->total) return ACE_ERR_WORKSPACE;
  if (!device_present()) return ACE_ERR_NODEV;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  const int n = p->n_orb;
  const size_t nn = (size_t)n * n;
  // inputs in the transform scratch: S [n][n] double, z [n][6], feat [n][4], pred [n][n] float
  double* dS = reinterpret_cast<double*>(w + p->off_S);
  double* dz = dS + nn;
  double* dfeat = dz + (size_t)n * 6;
  float* dpred = reinterpret_cast<float*>(dfeat + (size_t)n * 4);
  hipError_t e;
  if (d->kind == ACE_SCREEN_OVERLAP) {
    e = acex::launch_gemm_abt(phi, phi, n, n, p->npts, p->dV, dS,
                              reinterpret_cast<double*>(w + p->off_part), p->nsplit, true, nullptr,
                              s);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (d->mlp_weights) {
    e = acex::launch_moments(phi, p->n, n, p->npts, p->dV, dz, s);
    if (e != hipSuccess) return hip_fail(e);
    e = acex::launch_wannier_features(dz, n, p->L, dfeat, s);
    if (e != hipSuccess) return hip_fail(e);
    e = acex::launch_mlp_pairs(dfeat, n, p->L, d->mlp_weights, dpred, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  std::vector<double> S;
  std::vector<float> pred;
  if (d->kind == ACE_SCREEN_OVERLAP) {
    S.resize(nn);
    if ((e = hipMemcpyAsync(S.data(), dS, nn * sizeof(double), hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
      return hip_fail(e);
  }
  if (d->mlp_weights) {
    pred.resize(nn);
    if ((e = hipMemcpyAsync(pred.data(), dpred, nn * sizeof(float), hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
      return hip_fail(e);
  }
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e);
  return ace_screen_mask_host(n, d, S.empty() ? nullptr : S.data(),
                              pred.empty() ? nullptr : pred.data(), mask, rep);
}

// ------------------------------------------------------------------ batches

int ace_batch_create(ace_batch** batch, const ace_plan* const* plans,
                     const uint8_t* const* pair_masks, int count) {
  if (!batch || !plans) return ACE_ERR_ARG;
  *batch = nullptr;
  if (count < 1 || count > ACE_BATCH_MAX) return ACE_ERR_ARG;
  for (int k = 0; k < count; ++k)
    if (!plans[k]) return ACE_ERR_ARG;
  ace_batch* b = new ace_batch();
  b->count = count;
  size_t off = 0, pin = 0;
  std::vector<double> cost(count);
  for (int k = 0; k < count; ++k) {
    const ace_plan* p = plans[k];
    b->plans.push_back(p);
    b->shape.insert(b->shape.end(), {p->block, p->chunk, p->pencils, p->schedule});
    BuildTables bt;
    const int rc = prepare_tables(p, pair_masks ? pair_masks[k] : nullptr, bt);
    if (rc != ACE_OK) {
      delete b;
      return rc;
    }
    int64_t packs = 0;
    for (const Tile& t : bt.tiles) packs += t.npack;
    cost[k] = (double)packs * (double)p->npts * std::log2((double)p->npts);
    b->tables.push_back(std::move(bt));
    b->ws_off.push_back(off);
    off += align256(p->total);
    b->pin_off.push_back(pin);
    pin += align256(b->tables.back().used);
  }
  b->total = off;
  b->pin_bytes = pin;
  // largest first, each onto the branch with the least work so far
  b->order.resize(count);
  for (int k = 0; k < count; ++k) b->order[k] = k;
  std::stable_sort(b->order.begin(), b->order.end(),
                   [&](int x, int y) { return cost[x] > cost[y]; });
  // lanes: instances with at least one whole three-pass tile, by (precision, grid, block)
  b->fused.assign(count, 0);
  std::vector<std::vector<char>> whole(count);
  for (int k : b->order) {
    const ace_plan* p = b->plans[k];
    const std::vector<Tile>& tl = b->tables[k].tiles;
    whole[k].assign(tl.size(), 0);
    for (size_t ti = 0; ti < tl.size(); ++ti) {
      whole[k][ti] = tile_batch_whole(p, tl[ti]) ? 1 : 0;
      if (whole[k][ti]) b->fused[k] = 1;
    }
    if (!b->fused[k]) continue;
    BatchLane* lane = nullptr;
    for (BatchLane& l : b->lanes)
      if (l.prec == p->prec && l.n == p->n && l.block == p->block) lane = &l;
    if (!lane) {
      b->lanes.emplace_back();
      lane = &b->lanes.back();
      lane->prec = p->prec;
      lane->n = p->n;
      lane->block = p->block;
    }
    lane->inst.push_back(k);
    lane->cost += cost[k];
  }
  for (BatchLane& l : b->lanes) {
    size_t R = 0;
    for (int k : l.inst) R = std::max(R, b->tables[k].tiles.size());
    l.rounds.resize(R);
    for (size_t r = 0; r < R; ++r) {
      BatchLane::Round& rd = l.rounds[r];
      rd.seg0 = b->segs.size();
      for (int q = 0; q < 3; ++q) {
        int items = 0, nseg = 0;
        for (size_t pos = 0; pos < l.inst.size(); ++pos) {
          const int k = l.inst[pos];
          const ace_plan* p = b->plans[k];
          const std::vector<Tile>& tl = b->tables[k].tiles;
          if (r >= tl.size()) continue;
          if (!whole[k][r]) {
            if (q == 0) rd.rest.emplace_back((int)pos, (int)r);
            continue;
          }
          acex::BatchSeg sg{};
          sg.npts = p->npts;
          for (int a = 0; a < 3; ++a) sg.g2[a] = (kTwoPi / p->L[a]) * (kTwoPi / p->L[a]);
          sg.kscale = 1.0 / (double)p->npts;
          sg.alpha = p->alpha;
          sg.n = p->n;
          sg.npack = tl[r].npack;
          sg.block = p->block;
          sg.diag = tl[r].diag ? 1 : 0;
          sg.item0 = items;
          sg.count = acex::batch_items(q, p->n, tl[r].npack);
          items += sg.count;
          ++nseg;
          b->segs.push_back(sg);
          b->seg_of.emplace_back(k, (int)r);
        }
        rd.nseg = nseg;
        rd.total[q] = items;
      }
      rd.ctr = b->nctr;
      b->nctr += 3;
    }
  }
  if (!b->segs.empty()) {
    b->off_seg = off;
    off += align256(b->segs.size() * sizeof(acex::BatchSeg));
    b->off_ctr = off;
    off += align256((size_t)b->nctr * sizeof(int));
    b->total = off;
  }
  // branches: lanes and the other instances, largest first, each onto the
  // branch with the least work so far
  std::vector<std::pair<double, int>> units;  // (cost, lane l as -1 - l, or instance)
  for (size_t l = 0; l < b->lanes.size(); ++l) units.emplace_back(b->lanes[l].cost, -1 - (int)l);
  for (int k : b->order)
    if (!b->fused[k]) units.emplace_back(cost[k], k);
  std::stable_sort(units.begin(), units.end(),
                   [](const std::pair<double, int>& x, const std::pair<double, int>& y) {
                     return x.first > y.first;
                   });
  b->nbranch = std::min(count, kBatchBranches);
  {
    std::vector<double> alone(b->nbranch, 0.0);
    b->branch_alone.assign(count, 0);
    for (int k : b->order) {
      const int j = (int)(std::min_element(alone.begin(), alone.end()) - alone.begin());
      b->branch_alone[k] = j;
      alone[j] += cost[k];
    }
  }
  std::vector<double> load(std::min((int)units.size(), b->nbranch), 0.0);
  b->branch.assign(count, 0);
  for (const auto& u : units) {
    const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    if (u.second < 0)
      b->lanes[-1 - u.second].branch = j;
    else
      b->branch[u.second] = j;
    load[j] += u.first;
  }
  for (int k = 0; k < count; ++k)
    if (b->fused[k])
      for (const BatchLane& l : b->lanes)
        for (int kk : l.inst)
          if (kk == k) b->branch[k] = l.branch;
  *batch = b;
  return ACE_OK;
}

void ace_batch_destroy(ace_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (hipStream_t st : b->streams) (void)hipStreamDestroy(st);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (hipEvent_t ev : b->join) (void)hipEventDestroy(ev);
  if (b->pinned) (void)hipHostFree(b->pinned);
  if (b->seg_ev) (void)hipEventDestroy(b->seg_ev);
  if (b->seg_pinned) (void)hipHostFree(b->seg_pinned);
  delete b;
}

size_t ace_batch_workspace_bytes(const ace_batch* b) { return b ? b->total : 0; }

int ace_batch_lanes(const ace_batch* b, int* lanes, int64_t* batch_tiles, int64_t* other_tiles) {
  if (!b) return ACE_ERR_ARG;
  int64_t all = 0;
  for (const BuildTables& bt : b->tables) all += (int64_t)bt.tiles.size();
  const int64_t whole = (int64_t)b->seg_of.size() / 3;
  if (lanes) *lanes = (int)b->lanes.size();
  if (batch_tiles) *batch_tiles = whole;
  if (other_tiles) *other_tiles = all - whole;
  return ACE_OK;
}

int ace_batch_build(ace_batch* b, void* stream, void* ws, size_t ws_bytes,
                    const double* const* phi, double* const* W, double* const* M,
                    double* const* xi, double* ex, int* info, int flags) {
  if (!b || !ws || !phi || !W || !M || !xi || !ex || !info) return ACE_ERR_ARG;
  if (flags & ~(ACE_BATCH_EAGER | ACE_BATCH_NO_LANES)) return ACE_ERR_ARG;
  const bool lanes = !(flags & ACE_BATCH_NO_LANES);
  if (ws_bytes < b->total) return ACE_ERR_WORKSPACE;
  char* w = static_cast<char*>(ws);
  for (int k = 0; k < b->count; ++k) {
    const ace_plan* p = b->plans[k];
    if (p->block != b->shape[4 * k] || p->chunk != b->shape[4 * k + 1] ||
        p->pencils != b->shape[4 * k + 2] || p->schedule != b->shape[4 * k + 3])
      return ACE_ERR_ARG;
    const int rc = check_build_args(p, w + b->ws_off[k], p->total, phi[k], W[k], M[k], xi[k],
                                    ex + k, info + k);
    if (rc != ACE_OK) return rc;
  }
  // outputs of different instances must not share memory with any input or output
  for (int k = 0; k < b->count; ++k) {
    const size_t bk = (size_t)b->plans[k]->n_orb * b->plans[k]->npts * sizeof(double);
    for (int l = 0; l < b->count; ++l) {
      if (l == k) continue;
      const size_t bl = (size_t)b->plans[l]->n_orb * b->plans[l]->npts * sizeof(double);
      if (overlaps(W[k], bk, W[l], bl) || overlaps(W[k], bk, xi[l], bl) ||
          overlaps(xi[k], bk, xi[l], bl) || overlaps(W[k], bk, phi[l], bl) ||
          overlaps(xi[k], bk, phi[l], bl))
        return ACE_ERR_ARG;
    }
  }
  if (!device_present()) return ACE_ERR_NODEV;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  if (b->device < 0) {
    e = hipHostMalloc(reinterpret_cast<void**>(&b->pinned), std::max<size_t>(b->pin_bytes, 1),
                      hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e);
    for (int k = 0; k < b->count; ++k)
      std::memcpy(b->pinned + b->pin_off[k], b->tables[k].host.data(), b->tables[k].used);
    if ((e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming)) != hipSuccess)
      return hip_fail(e);
    if (!b->segs.empty()) {
      e = hipHostMalloc(reinterpret_cast<void**>(&b->seg_pinned),
                        b->segs.size() * sizeof(acex::BatchSeg), hipHostMallocDefault);
      if (e != hipSuccess) return hip_fail(e);
      if ((e = hipEventCreateWithFlags(&b->seg_ev, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e);
    }
    for (int j = 0; j < b->nbranch; ++j) {
      hipStream_t st = nullptr;
      hipEvent_t ev = nullptr;
      if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e);
      b->streams.push_back(st);
      if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e);
      b->join.push_back(ev);
    }
    b->device = dev;
  } else if (dev != b->device) {
    return ACE_ERR_ARG;
  }
  (void)device_cus();
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the tables go in ahead of the work, in stream order, from batch-owned pinned memory
  for (int k = 0; k < b->count; ++k) {
    e = hipMemcpyAsync(w + b->ws_off[k] + b->plans[k]->off_tab, b->pinned + b->pin_off[k],
                       b->tables[k].used, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e);
  }

  // the batch-pass segments: device pointers of this call's arrays, written
  // into the pinned copy only when they change (after its last upload has
  // been read), uploaded in stream order like the tables
  acex::BatchSeg* d_segs = reinterpret_cast<acex::BatchSeg*>(w + b->off_seg);
  int* d_ctr = reinterpret_cast<int*>(w + b->off_ctr);
  if (!b->segs.empty()) {
    std::vector<const void*> sk;
    sk.reserve(2 * b->count + 1);
    sk.push_back(ws);
    for (int k = 0; k < b->count; ++k) {
      sk.push_back(phi[k]);
      sk.push_back(W[k]);
    }
    if (sk != b->seg_key) {
      if (b->seg_pending && (e = hipEventSynchronize(b->seg_ev)) != hipSuccess)
        return hip_fail(e);
      for (size_t i = 0; i < b->segs.size(); ++i) {
        const int k = b->seg_of[i].first, ti = b->seg_of[i].second;
        const ace_plan* p = b->plans[k];
        const BuildTables& bt = b->tables[k];
        char* pw = w + b->ws_off[k];
        acex::BatchSeg sg = b->segs[i];
        sg.phi = p->prec == 0 ? static_cast<const void*>(phi[k]) : pw + p->off_phi32;
        sg.packs = reinterpret_cast<const Pack*>(pw + p->off_tab + bt.o_packs) + bt.tiles[ti].pack0;
        sg.S = pw + p->off_S;
        sg.tw = pw + p->off_tab + bt.o_tw;
        sg.W = W[k];
        sg.orbs = reinterpret_cast<const int*>(pw + p->off_tab + bt.o_orbs) + (size_t)ti * 2 * p->block;
        b->seg_pinned[i] = sg;
      }
      b->seg_key = std::move(sk);
    }
    e = hipMemcpyAsync(d_segs, b->seg_pinned, b->segs.size() * sizeof(acex::BatchSeg),
                       hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e);
    if ((e = hipEventRecord(b->seg_ev, s)) != hipSuccess) return hip_fail(e);
    b->seg_pending = true;
  }

  // one lane on stream st: the instances' prologues, the rounds (batch passes,
  // then the lane's other tiles of the round), the instances' dense tails
  auto run_lane = [&](const BatchLane& l, hipStream_t st) -> int {
    std::vector<BuildCtx> ctx(l.inst.size());
    int rc = ACE_OK;
    for (size_t pos = 0; pos < l.inst.size(); ++pos) {
      const int k = l.inst[pos];
      rc = build_begin(b->plans[k], st, w + b->ws_off[k], phi[k], b->tables[k], W[k], ctx[pos]);
      if (rc != ACE_OK) return rc;
    }
    const int cus = device_cus();
    for (const BatchLane::Round& rd : l.rounds) {
      for (int q = 0; q < 3; ++q) {
        const hipError_t er =
            acex::launch_batch_pass(l.prec, q, l.n, l.block, d_segs + rd.seg0 + (size_t)q * rd.nseg, rd.nseg,
                                    rd.total[q], d_ctr + rd.ctr + q, cus, st);
        if (er != hipSuccess) return hip_fail(er);
      }
      for (const auto& pt : rd.rest) {
        rc = build_tile(ctx[pt.first], st, (size_t)pt.second, W[l.inst[pt.first]]);
        if (rc != ACE_OK) return rc;
      }
    }
    for (size_t pos = 0; pos < l.inst.size(); ++pos) {
      const int k = l.inst[pos];
      rc = build_end(b->plans[k], st, w + b->ws_off[k], phi[k], W[k], M[k], xi[k], ex + k,
                     info + k);
      if (rc != ACE_OK) return rc;
    }
    return ACE_OK;
  };

  // fork from `head` onto the branch streams (lanes and the other instances
  // on their branches), join back
  auto record = [&](hipStream_t head) -> int {
    hipError_t er;
    if (lanes && b->nctr > 0 &&
        (er = acex::launch_fill_i32(d_ctr, 0, b->nctr, head)) != hipSuccess)
      return hip_fail(er);
    if ((er = hipEventRecord(b->fork, head)) != hipSuccess) return hip_fail(er);
    for (hipStream_t st : b->streams)
      if ((er = hipStreamWaitEvent(st, b->fork, 0)) != hipSuccess) return hip_fail(er);
    int rc = ACE_OK;
    if (lanes) {
      for (const BatchLane& l : b->lanes) {
        rc = run_lane(l, b->streams[l.branch]);
        if (rc != ACE_OK) break;
      }
    }
    for (int k : b->order) {
      if (rc != ACE_OK || (lanes && b->fused[k])) continue;
      const int br = lanes ? b->branch[k] : b->branch_alone[k];
      rc = enqueue_build(b->plans[k], b->streams[br], w + b->ws_off[k], phi[k], b->tables[k],
                         W[k], M[k], xi[k], ex + k, info + k);
    }
    // the join is recorded even after an error, so that a capture always closes
    for (int j = 0; j < b->nbranch; ++j) {
      if ((er = hipEventRecord(b->join[j], b->streams[j])) != hipSuccess) return hip_fail(er);
      if ((er = hipStreamWaitEvent(head, b->join[j], 0)) != hipSuccess) return hip_fail(er);
    }
    return rc;
  };

  if (flags & ACE_BATCH_EAGER) return record(s);

  std::vector<const void*> key;
  key.reserve(4 * b->count + 3);
  key.push_back(ws);
  key.push_back(ex);
  key.push_back(info);
  key.push_back(reinterpret_cast<const void*>(static_cast<uintptr_t>(lanes ? 1 : 2)));
  for (int k = 0; k < b->count; ++k) {
    key.push_back(phi[k]);
    key.push_back(W[k]);
    key.push_back(M[k]);
    key.push_back(xi[k]);
  }
  if (!b->exec || key != b->key) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->key.clear();
    e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e);
    g_capturing = true;
    const int rc = record(b->cap);
    g_capturing = false;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(b->cap, &graph);
    if (rc != ACE_OK || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc != ACE_OK ? rc : hip_fail(e);
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_fail(e);
    }
    b->graph = graph;
    b->exec = exec;
    b->key = std::move(key);
  }
  e = hipGraphLaunch(b->exec, s);
  return e == hipSuccess ? ACE_OK : hip_fail(e);
}

}  // extern "C"

// ------------------------------------------------------------------ SCDM localisation

namespace {

struct ScdmLayout {
  size_t rho, g, part, means, cnt, off, pre_total;
  size_t A, nrm, perm, v, tau, rdiag, Y, G, Z, partial, state, loc_total;
  int nsplit;
};

ScdmLayout scdm_layout(const ace_plan* p, int m) {
  ScdmLayout l{};
  const int64_t nb = acex::scdm_sel_blocks(p->npts);
  size_t o = 0;
  l.rho = o;
  o += align256((size_t)p->npts * 8);
  l.g = o;
  o += align256((size_t)p->npts * 8);
  l.part = o;
  o += align256((size_t)2 * acex::scdm_sum_blocks() * 8);
  l.means = o;
  o += align256(16);
  l.cnt = o;
  o += align256((size_t)nb * 4);
  l.off = o;
  o += align256((size_t)nb * 4);
  l.pre_total = o;
  const int k = p->n_orb;
  l.nsplit = acex::gemm_abt_splits(k, k, k);
  o = 0;
  l.A = o;
  o += align256((size_t)std::max(m, 1) * k * 8);
  l.nrm = o;
  o += align256((size_t)std::max(m, 1) * 8);
  l.perm = o;
  o += align256((size_t)std::max(m, 1) * 4);
  l.v = o;
  o += align256((size_t)k * 8);
  l.tau = o;
  o += align256(8);
  l.rdiag = o;
  o += align256((size_t)k * 8);
  l.Y = o;
  o += align256((size_t)k * k * 8);
  l.G = o;
  o += align256((size_t)k * k * 8);
  l.Z = o;
  o += align256((size_t)k * k * 8);
  l.partial = o;
  o += align256((size_t)l.nsplit * k * k * 8);
  l.state = o;
  o += align256(16);
  l.loc_total = o;
  return l;
}

constexpr int kPolarMaxIter = 100;

}  // namespace

extern "C" {

size_t scdm_workspace_bytes(const ace_plan* p, int m) {
  if (!p || m < 0) return 0;
  const ScdmLayout l = scdm_layout(p, m);
  return m > 0 ? std::max(l.pre_total, l.loc_total) : l.pre_total;
}

int scdm_preselect(const ace_plan* p, void* stream, void* ws, size_t ws_bytes, const double* phi,
                   int* points, int* count) {
  if (!p || !ws || !phi || !points || !count) return ACE_ERR_ARG;
  const ScdmLayout l = scdm_layout(p, 0);
  if (ws_bytes < l.pre_total) return ACE_ERR_WORKSPACE;
  if (!device_present()) return ACE_ERR_NODEV;
  char* w = static_cast<char*>(ws);
  const hipError_t e = acex::launch_scdm_preselect(
      phi, p->n, p->n_orb, p->L, reinterpret_cast<double*>(w + l.rho),
      reinterpret_cast<double*>(w + l.g), reinterpret_cast<double*>(w + l.part),
      reinterpret_cast<double*>(w + l.means), reinterpret_cast<int*>(w + l.cnt),
      reinterpret_cast<int*>(w + l.off), points, count, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? ACE_OK : hip_fail(e);
}

int scdm_localize(const ace_plan* p, void* stream, void* ws, size_t ws_bytes, const double* phi,
                  const int* points, int m, int* pivots, double* phi_loc, int* info) {
  if (!p || !ws || !phi || !pivots || !phi_loc || !info) return ACE_ERR_ARG;
  if (m < p->n_orb || (int64_t)m > p->npts) return ACE_ERR_ARG;
  if (!points && (int64_t)m != p->npts) return ACE_ERR_ARG;
  const size_t orb_bytes = (size_t)p->n_orb * p->npts * sizeof(double);
  if (overlaps(phi, orb_bytes, phi_loc, orb_bytes)) return ACE_ERR_ARG;
  const ScdmLayout l = scdm_layout(p, m);
  if (ws_bytes < l.loc_total) return ACE_ERR_WORKSPACE;
  if (!device_present()) return ACE_ERR_NODEV;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  const int k = p->n_orb;
  hipError_t e = acex::launch_set_int(info, 0, s);
  if (e != hipSuccess) return hip_fail(e);
  e = acex::launch_scdm_qr(phi, points, m, k, p->npts, reinterpret_cast<double*>(w + l.A),
                           reinterpret_cast<double*>(w + l.nrm), reinterpret_cast<int*>(w + l.perm),
                           reinterpret_cast<double*>(w + l.v), reinterpret_cast<double*>(w + l.tau),
                           reinterpret_cast<double*>(w + l.rdiag), pivots, info, s);
  if (e != hipSuccess) return hip_fail(e);
  double* Y = reinterpret_cast<double*>(w + l.Y);
  e = acex::launch_scdm_polar(phi, pivots, k, p->npts, Y, reinterpret_cast<double*>(w + l.G),
                              reinterpret_cast<double*>(w + l.Z),
                              reinterpret_cast<double*>(w + l.partial), l.nsplit,
                              reinterpret_cast<int*>(w + l.state), info, kPolarMaxIter, s);
  if (e != hipSuccess) return hip_fail(e);
  e = acex::launch_gemm_ab(Y, phi, k, k, p->npts, 1.0, phi_loc, nullptr, s);
  return e == hipSuccess ? ACE_OK : hip_fail(e);
}

}  // extern "C"
