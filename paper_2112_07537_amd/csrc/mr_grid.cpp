// Host driver of the multiresolution block-octree hot path: linear octree,
// owner maps, ghost-patch layout and work lists, adaptation policy, and the
// C ABI of include/mr.h.
//
// Method: Gillis & van Rees, MURPHY (arXiv 2112.07537).  Section 2.2 (block
// operations), section 2.2.5 (criterion, thresholds), the ghosting
// algorithms (Part 1 / Part 2) and the grid-adaptation algorithm of the
// supplementary algorithms section.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "mr.h"
#include "mr_internal.h"

namespace mr {

static thread_local std::string g_errmsg;

static mr_status fail(mr_status s, const std::string& m) {
  g_errmsg = m;
  return s;
}

#define HIPCHK(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(MR_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));       \
  } while (0)

struct Key {
  int32_t L, i, j, k;
};

static inline uint64_t pack(int L, int i, int j, int k) {
  return (uint64_t(L) << 60) | (uint64_t(i) << 40) | (uint64_t(j) << 20) | uint64_t(k);
}

static inline uint64_t spread3(uint64_t v) {
  uint64_t r = 0;
  for (int b = 0; b < 20; ++b) r |= ((v >> b) & 1ull) << (3 * b);
  return r;
}

// Morton order of leaves: interleave origin coordinates at level 19.
static inline uint64_t morton(const Key& b) {
  const int s = 19 - b.L;
  return spread3(uint64_t(b.i) << s) | (spread3(uint64_t(b.j) << s) << 1) |
         (spread3(uint64_t(b.k) << s) << 2);
}

// Leaf key -> block index: open addressing with linear probing (the map is
// rebuilt after every tree change and queried a few million times then).
struct LeafIndex {
  static constexpr uint64_t kEmpty = ~0ull;
  std::vector<uint64_t> keys;
  std::vector<int32_t> vals;
  uint64_t mask = 0;
  static uint64_t mix(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    return x;
  }
  void build(size_t n) {
    size_t cap = 16;
    while (cap < 2 * n + 16) cap <<= 1;
    keys.assign(cap, kEmpty);
    vals.assign(cap, -1);
    mask = cap - 1;
  }
  void insert(uint64_t key, int32_t v) {
    uint64_t h = mix(key) & mask;
    while (keys[h] != kEmpty && keys[h] != key) h = (h + 1) & mask;
    keys[h] = key;
    vals[h] = v;
  }
  int32_t find(uint64_t key) const {
    if (keys.empty()) return -1;
    uint64_t h = mix(key) & mask;
    while (keys[h] != kEmpty) {
      if (keys[h] == key) return vals[h];
      h = (h + 1) & mask;
    }
    return -1;
  }
};

// Device buffer: library-owned (hipMalloc, grow on demand) or a fixed slice
// of a caller-owned pool (never freed or grown by the library).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool owned = true;
  hipError_t ensure(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    if (!owned) return hipErrorOutOfMemory;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    size_t want = std::max<size_t>(n, 256);
    hipError_t e = hipMalloc(&p, want);
    if (e == hipSuccess) bytes = want;
    return e;
  }
  void adopt(void* q, size_t n) {
    p = q;
    bytes = n;
    owned = false;
  }
  void release() {
    if (p && owned) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    owned = true;
  }
};

struct Lists {
  std::vector<GItem> g;   // c->f patch items (one launch)
  std::vector<GItem> s;   // substitution items (one launch, after the patches)
  std::vector<RItem> r;
  int lds_g = 0, lds_s = 0;
  // f->c items grouped by pass-1 column length (extent along y or z):
  // classes <= 3, <= 6, <= 12 at [rcls[c], rcls[c+1]) with their LDS sizes
  int rcls[4] = {0, 0, 0, 0};
  int lds_rc[3] = {0, 0, 0};
  int64_t out_points = 0;
  // values each launch of the reconstruction writes and reads (the
  // algorithmic traffic of the lists): c->f patch values / coarse samples,
  // substituted points / staged points, f->c values / fine window points
  int64_t cf_w = 0, cf_r = 0, sb_w = 0, sb_r = 0, fc_w = 0, fc_r = 0;
  DevBuf dg, ds, dr;
};

struct Prof {
  bool on = false;
  struct Rec {
    hipEvent_t a, b;
    int fam;
  };
  std::vector<Rec> recs;
  int64_t points[5] = {0, 0, 0, 0, 0};
};

static const int kNumFam = 5;
static const char* kFam[kNumFam] = {"rhs", "details", "ghost_refine", "ghost_restrict",
                                    "ghost_subst"};

// Host-side phases of an adaptation (wall clock, stream work included where
// the phase waits for it): criterion (ghosts + transform + norms to host),
// plan (flags + policy), apply (refine / coarsen / update passes), commit
// (owner map, patch offsets, work lists, uploads).
static const char* kHostPhase[4] = {"adapt_criterion", "adapt_plan", "adapt_apply", "tree_commit"};
struct HostTimer {
  double ms[4] = {0, 0, 0, 0};
  int64_t n[4] = {0, 0, 0, 0};
};
static double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace mr

using namespace mr;

// Defaults of the launch-shape knobs (mr_tuning).  LDS per work item is
// bounded by tiling: every workgroup of a launch reserves the largest item's
// LDS, so smaller tiles raise the number of resident workgroups.  The c->f
// and substitution values do not depend on the tiling; the rounding order of
// an f->c sum follows its tile's thinnest axis.
static const int kLdsBudgetRefine = 20 * 1024;
static const int kLdsBudgetRestrict = 24 * 1024;
static const int kLdsBudgetSubst = 37 * 1024;
static const int kSubstThreads = 512;

struct mr_grid {
  mr_config cfg{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // second stream (default priority) for the detail pass of a fused step,
  // which runs beside the first stage's RHS; fork / join events
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  HostTimer htime;
  DevBuf ad_pairs, ad_items, ad_scr, ad_det, ad_slot, ad_dirs;   // adaptation scratch
  std::vector<DevBuf> backup;   // fields at the start of an mr_adapt call
  bool f32 = false;
  int nb = 16, N = 4, Nt = 0, G = 2, Dw = 4;
  mr_tuning tune{kLdsBudgetRefine, kLdsBudgetRestrict, kLdsBudgetSubst, kSubstThreads, {0, 0, 0, 0}};
  int Ef = 0, Eb = 0;
  size_t esz = 8;
  // tree
  std::vector<Key> leaves;
  LeafIndex index;
  std::vector<int32_t> cmap;
  std::vector<int64_t> poff;
  std::vector<int32_t> cdir_host;   // per block: bit r = region r is coarser
  std::vector<uint64_t> stab_host;  // per block: 512-bit slab table (8 words)
  int64_t patch_elems = 0;
  // device
  std::vector<DevBuf> fields, alts;
  DevBuf tmpA, tmpB;
  DevBuf d_lev, d_ijk, d_cmap, d_poff, d_patch, d_err, d_cbase, d_cstep, d_stab;
  // second patch buffer of the same layout, for the later stages of a fused
  // step while the detail pass still reads the first (allocated on demand)
  DevBuf d_patch2;
  DevBuf d_bands, d_norms, d_icpar, d_mom;
  Lists stage, wide;
  Prof prof;
  // hipGraphs of a whole RK3 step and of a fused detail pass + RK3 step,
  // each re-captured when the tree, the field, dt or the velocity changes
  struct StepGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double dt = 0;
    mr_velocity vel{};
    int field = -1;
    int64_t version = -1;
    void reset() {
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      exec = nullptr;
      graph = nullptr;
    }
  };
  StepGraph rk3_graph, fused_graph;
  int64_t tree_version = 0;
};

namespace mr {

// ---------------------------------------------------------------- helpers
static int find_leaf(const mr_grid* g, int L, int i, int j, int k) {
  if (L < 0) return -1;
  const int n = 1 << L;
  i = ((i % n) + n) % n;
  j = ((j % n) + n) % n;
  k = ((k % n) + n) % n;
  return g->index.find(pack(L, i, j, k));
}

// Leaf containing the level-Lc cell (I, J, K) (periodic), searching the cell
// itself and its ancestors; -1 when the cell is subdivided.
static int leaf_containing(const mr_grid* g, int Lc, int I, int J, int K) {
  for (int l = Lc; l >= 0; --l) {
    const int s = Lc - l;
    const int n = 1 << Lc;
    const int ii = ((I % n) + n) % n, jj = ((J % n) + n) % n, kk = ((K % n) + n) % n;
    const int id = find_leaf(g, l, ii >> s, jj >> s, kk >> s);
    if (id >= 0) return id;
  }
  return -1;
}

// Type of the neighbour cell of block b in direction d: 0 same level,
// -1 inside a coarser leaf (id returned), +1 subdivided (finer).
static int neighbor_kind(const mr_grid* g, int b, int dx, int dy, int dz, int* id_out) {
  const Key& k = g->leaves[b];
  int id = find_leaf(g, k.L, k.i + dx, k.j + dy, k.k + dz);
  if (id >= 0) {
    *id_out = id;
    return 0;
  }
  for (int l = k.L - 1; l >= 0; --l) {
    const int s = k.L - l;
    const int n = 1 << k.L;
    int ii = (((k.i + dx) % n) + n) % n, jj = (((k.j + dy) % n) + n) % n,
        kk = (((k.k + dz) % n) + n) % n;
    id = find_leaf(g, l, ii >> s, jj >> s, kk >> s);
    if (id >= 0) {
      *id_out = id;
      return -1;
    }
  }
  *id_out = -1;
  return 1;
}

static void rebuild_index(mr_grid* g) {
  g->index.build(g->leaves.size());
  for (size_t b = 0; b < g->leaves.size(); ++b) {
    const Key& k = g->leaves[b];
    g->index.insert(pack(k.L, k.i, k.j, k.k), int32_t(b));
  }
}

static void sort_leaves(std::vector<Key>& v) {
  std::vector<std::pair<uint64_t, Key>> t(v.size());
  for (size_t i = 0; i < v.size(); ++i) t[i] = {morton(v[i]), v[i]};
  std::sort(t.begin(), t.end(), [](const std::pair<uint64_t, Key>& a, const std::pair<uint64_t, Key>& b) {
    return a.first < b.first;
  });
  for (size_t i = 0; i < v.size(); ++i) v[i] = t[i].second;
}

// Owner map (4x4x4 half-block cells around each block) and 2:1 check.
// Run body(lo, hi) over [0, n) split into contiguous chunks on host threads.
template <typename F>
static void parallel_for(size_t n, F body) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const unsigned nt = std::min<unsigned>(16, hw);
  if (n < 2 || nt == 1) {
    body(size_t(0), n);
    return;
  }
  std::vector<std::thread> th;
  const size_t chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    const size_t lo = t * chunk, hi = std::min(n, lo + chunk);
    if (lo >= hi) break;
    th.emplace_back(body, lo, hi);
  }
  for (auto& x : th) x.join();
}

// Owner map (4x4x4 half-block cells around each block) and 2:1 check.  The
// cells of one of the 27 regions around a block share the owner unless the
// region is subdivided, so each region costs one or two lookups.
static mr_status build_cmap(mr_grid* g) {
  const size_t n = g->leaves.size();
  g->cmap.assign(n * 64, -1);
  std::atomic<int64_t> bad{-1};
  parallel_for(n, [&](size_t lo, size_t hi) {
    for (size_t b = lo; b < hi; ++b) {
      const Key& k = g->leaves[b];
      for (int r = 0; r < 27; ++r) {
        const int rr[3] = {r % 3, (r / 3) % 3, r / 9};
        int id = find_leaf(g, k.L, k.i + rr[0] - 1, k.j + rr[1] - 1, k.k + rr[2] - 1);
        if (id < 0 && k.L > 0) {
          const int m = 1 << k.L;
          const int ii = ((k.i + rr[0] - 1) % m + m) % m, jj = ((k.j + rr[1] - 1) % m + m) % m,
                    kk = ((k.k + rr[2] - 1) % m + m) % m;
          id = find_leaf(g, k.L - 1, ii >> 1, jj >> 1, kk >> 1);
        }
        const int c0[3] = {rr[0] == 0 ? 0 : (rr[0] == 1 ? 1 : 3), rr[1] == 0 ? 0 : (rr[1] == 1 ? 1 : 3),
                           rr[2] == 0 ? 0 : (rr[2] == 1 ? 1 : 3)};
        const int c1[3] = {rr[0] == 1 ? 2 : c0[0], rr[1] == 1 ? 2 : c0[1], rr[2] == 1 ? 2 : c0[2]};
        for (int cz = c0[2]; cz <= c1[2]; ++cz)
          for (int cy = c0[1]; cy <= c1[1]; ++cy)
            for (int cx = c0[0]; cx <= c1[0]; ++cx) {
              int cid = id;
              if (cid < 0)   // subdivided (or not 2:1): resolve the cell itself
                cid = leaf_containing(g, k.L + 1, 2 * k.i + cx - 1, 2 * k.j + cy - 1, 2 * k.k + cz - 1);
              if (cid < 0 || std::abs(g->leaves[cid].L - k.L) > 1) {
                int64_t expect = -1;
                bad.compare_exchange_strong(expect, int64_t(b));
                cid = -1;
              }
              g->cmap[b * 64 + (cz * 4 + cy) * 4 + cx] = cid;
            }
      }
    }
  });
  if (bad.load() >= 0) {
    const Key& k = g->leaves[size_t(bad.load())];
    return fail(MR_EINVAL, "tree is not 2:1 balanced around block (" + std::to_string(k.L) + "," +
                               std::to_string(k.i) + "," + std::to_string(k.j) + "," +
                               std::to_string(k.k) + ")");
  }
  return MR_OK;
}

static int region_level(const mr_grid* g, int b, int r) {
  const int rx = r % 3, ry = (r / 3) % 3, rz = r / 9;
  const int cx = rx == 0 ? 0 : (rx == 1 ? 1 : 3);
  const int cy = ry == 0 ? 0 : (ry == 1 ? 1 : 3);
  const int cz = rz == 0 ? 0 : (rz == 1 ? 1 : 3);
  return g->leaves[g->cmap[b * 64 + (cz * 4 + cy) * 4 + cx]].L;
}

static void region_box(int nb, int D, int r, int lo[3], int hi[3]) {
  const int rr[3] = {r % 3, (r / 3) % 3, r / 9};
  for (int a = 0; a < 3; ++a) {
    if (rr[a] == 0) { lo[a] = -D; hi[a] = 0; }
    else if (rr[a] == 1) { lo[a] = 0; hi[a] = nb; }
    else { lo[a] = nb; hi[a] = nb + D; }
  }
}

static int64_t box_size(const int lo[3], const int hi[3]) {
  return int64_t(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
}

static int floordiv(int a, int b) {
  int q = a / b;
  return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// Sample range of a refinement box along one axis: pairs p0..p1 of fine
// points (2c, 2c+1) need the samples p0 + 1 - N/2 .. p1 + N/2.
static void gview_samples(int lo, int hi, int N, int* clo, int* cs) {
  const int p0 = floordiv(lo, 2), p1 = floordiv(hi - 1, 2);
  *clo = p0 + 1 - N / 2;
  *cs = p1 - p0 + N;
}

static int gview_lds(const GItem& it, int N, size_t esz) {
  int cs[3], fs[3];
  for (int a = 0; a < 3; ++a) {
    int clo;
    gview_samples(it.lo[a], it.hi[a], N, &clo, &cs[a]);
    fs[a] = it.hi[a] - it.lo[a];
  }
  return int(esz * (size_t(fs[0]) * cs[1] * cs[2] +
                    std::max(size_t(cs[0]) * cs[1] * cs[2], size_t(fs[0]) * fs[1] * cs[2])));
}

static int rview_lds(const RItem& it, int H, size_t esz) {
  int qs[3], xs[3];
  for (int a = 0; a < 3; ++a) {
    qs[a] = it.hi[a] - it.lo[a];
    xs[a] = 2 * (qs[a] - 1) + 1 + 2 * H;
  }
  const int n = qs[1] <= qs[2] ? 1 : 2;   // pass 1 never runs along x
  const int a1 = 0, a2 = n == 2 ? 1 : 2;
  return int(esz * (size_t(qs[n]) * xs[a1] * xs[a2] + size_t(qs[n]) * qs[a1] * xs[a2]));
}


// LDS of a substitution item (k_subst): the lattice of its box (per axis
// the even coordinates within N-1 of the box and the odd ones inside it),
// one value per point padded to 8 bytes, one flag bit per point in 64-bit
// words, then the larger of the degree-2 temporaries ((x, y) and (x, z)
// classes together, or the (y, z) class) and the degree-3 ones.
static int subst_lds(const GItem& it, int N, size_t esz) {
  const int R = N - 1;
  int nE[3], nO[3], nL[3];
  for (int a = 0; a < 3; ++a) {
    const int lo = it.lo[a], hi = it.hi[a];
    const int s = lo - R, e0 = s + (s & 1), o0 = lo | 1;
    nE[a] = (hi + R - e0 + 1) >> 1;
    nO[a] = hi > o0 ? (hi - o0 + 1) >> 1 : 0;
    nL[a] = nE[a] + nO[a];
  }
  const size_t nV = size_t(nL[0]) * nL[1] * nL[2];
  const size_t t2 = std::max(size_t(nE[2]) * nO[1] * nL[0] + size_t(nO[2]) * nE[1] * nL[0],
                             size_t(nO[2]) * nL[1] * nE[0]);
  const size_t t3 = size_t(nO[2]) * nL[1] * nL[0] + size_t(nO[2]) * nO[1] * nL[0];
  const size_t head = ((nV * esz + 7) & ~size_t(7)) + (nV + 63) / 64 * 8;
  return int(head + std::max(t2, t3) * esz);
}

// Split a box along its longest axis until the LDS estimate fits the budget.
template <typename Item, typename F>
static void push_tiled(std::vector<Item>& out, Item it, F lds_of, int kLdsBudget) {
  std::vector<Item> todo{it};
  while (!todo.empty()) {
    Item c = todo.back();
    todo.pop_back();
    if (lds_of(c) <= kLdsBudget) {
      out.push_back(c);
      continue;
    }
    int ax = 0;
    for (int a = 1; a < 3; ++a)
      if (c.hi[a] - c.lo[a] > c.hi[ax] - c.lo[ax]) ax = a;
    const int mid = c.lo[ax] + (c.hi[ax] - c.lo[ax]) / 2;
    if (mid == c.lo[ax]) {  // cannot split further
      out.push_back(c);
      continue;
    }
    Item a = c, b = c;
    a.hi[ax] = mid;
    b.lo[ax] = mid;
    todo.push_back(a);
    todo.push_back(b);
  }
}

static int Hreach(int N, int Nt) { return Nt ? N : 0; }

// Box a minus box b as disjoint boxes, appended to out (other fields of a).
static void box_subtract(const GItem& a, const GItem& b, std::vector<GItem>& out) {
  for (int c = 0; c < 3; ++c)
    if (a.hi[c] <= b.lo[c] || b.hi[c] <= a.lo[c]) {
      out.push_back(a);
      return;
    }
  GItem rest = a;
  for (int c = 0; c < 3; ++c) {
    if (rest.lo[c] < b.lo[c]) {
      GItem p = rest;
      p.hi[c] = b.lo[c];
      out.push_back(p);
      rest.lo[c] = b.lo[c];
    }
    if (rest.hi[c] > b.hi[c]) {
      GItem p = rest;
      p.lo[c] = b.hi[c];
      out.push_back(p);
      rest.hi[c] = b.hi[c];
    }
  }
  // what is left of a lies inside b
}

// Work lists of one ghost reconstruction at depth D, in launch order
// (READING R-ORDER, the ghosting algorithms' Part 1 before Part 2): c->f
// patches (refined from the samples as they stand), then the substitution of
// every fine block's slabs (reading those patches), then f->c restrictions by
// the fine blocks (reading their substituted values and their c->f
// patches).  c->f patches are filled to max(D, reach of H^a, N-1): a fine
// block's restriction window and its substitution stencils are covered by
// its own ghost layer.
static mr_status build_lists(mr_grid* g, int D, Lists& L) {
  L.g.clear();
  L.s.clear();
  L.r.clear();
  L.out_points = 0;
  const int nb = g->nb, N = g->N, Nt = g->Nt, Dw = g->Dw;
  const int H = Hreach(N, Nt);
  const int Dc = std::min(Dw, std::max(std::max(D, H), N - 1));
  const size_t esz = g->esz;
  auto glds = [&](const GItem& it) { return gview_lds(it, N, esz); };
  auto slds = [&](const GItem& it) { return subst_lds(it, N, esz); };
  auto rlds = [&](const RItem& it) { return rview_lds(it, H, esz); };
  const int n = int(g->leaves.size());
  const int hb = nb / 2;
  // blocks are split into contiguous chunks built on host threads; the
  // chunks' items are concatenated in block order
  struct Part {
    std::vector<GItem> g, s;
    std::vector<RItem> r;
    int64_t pts = 0;
    bool ok = true;
  };
  auto one_block = [&](int b, Part& P) -> bool {
    const int Lb = g->leaves[b].L;
    std::vector<GItem> slabs;   // made disjoint below
    for (int r = 0; r < 27; ++r) {
      if (r == 13) continue;
      const int lr = region_level(g, b, r);
      if (lr == Lb) continue;
      const int rr[3] = {r % 3, (r / 3) % 3, r / 9};
      int rlo[3], rhi[3], blo[3], bhi[3];
      region_box(nb, Dw, r, rlo, rhi);
      if (lr < Lb) {
        // c->f patches are merged per side below
        // substitution slab of this interface (READING R-SUB), unless a
        // coarser region facing a proper subset of the same axes exists: its
        // slab contains this one
        GItem sb{};
        sb.blk = b;
        sb.sel = (Nt ? 8 : 0) | 16;
        int facing = 0;
        for (int a = 0; a < 3; ++a)
          if (rr[a] != 1) facing |= (1 << a);
        bool sempty = false;
        for (int a = 0; a < 3; ++a) {
          const int d = rr[a] - 1;
          if (d == 0) { sb.lo[a] = 0; sb.hi[a] = nb; }
          else if (Nt) {
            if (d < 0) { sb.lo[a] = 0; sb.hi[a] = N; }
            else { sb.lo[a] = nb - N + 1; sb.hi[a] = nb; }
          } else {
            if (d < 0) { sb.lo[a] = 0; sb.hi[a] = N - 1; }
            else { sb.lo[a] = nb - N + 2; sb.hi[a] = nb; }
          }
          if (sb.hi[a] <= sb.lo[a]) sempty = true;
        }
        bool covered = false;
        for (int sub = 1; sub < 8 && !covered; ++sub) {
          if ((sub & facing) != sub || sub == facing) continue;
          int r2 = 0, mul = 1;
          for (int a = 0; a < 3; ++a, mul *= 3) r2 += mul * ((sub >> a) & 1 ? rr[a] : 1);
          if (region_level(g, b, r2) < Lb) covered = true;
        }
        if (!sempty && !covered) slabs.push_back(sb);
      } else {
        // f->c: each finer leaf covering this region restricts its part
        region_box(nb, D, r, blo, bhi);
        int c0[3], c1[3];
        for (int a = 0; a < 3; ++a) {
          c0[a] = rr[a] == 0 ? 0 : (rr[a] == 1 ? 1 : 3);
          c1[a] = rr[a] == 0 ? 0 : (rr[a] == 1 ? 2 : 3);
        }
        for (int cz = c0[2]; cz <= c1[2]; ++cz)
          for (int cy = c0[1]; cy <= c1[1]; ++cy)
            for (int cx = c0[0]; cx <= c1[0]; ++cx) {
              const int cc[3] = {cx, cy, cz};
              RItem it{};
              it.fblk = g->cmap[size_t(b) * 64 + (cz * 4 + cy) * 4 + cx];
              it.cblk = b;
              it.off = g->poff[size_t(b) * 27 + r];
              bool empty = false;
              for (int a = 0; a < 3; ++a) {
                const int lo = (cc[a] - 1) * hb, hi = cc[a] * hb;
                it.lo[a] = std::max(blo[a], lo);
                it.hi[a] = std::min(bhi[a], hi);
                it.sh[a] = lo;
                it.rlo[a] = rlo[a];
                it.rsz[a] = rhi[a] - rlo[a];
                if (it.hi[a] <= it.lo[a]) empty = true;
              }
              if (empty) continue;
              if (g->leaves[it.fblk].L != Lb + 1)
                return false;
              P.pts += box_size(it.lo, it.hi);
              push_tiled(P.r, it, rlds, g->tune.lds_restrict);
            }
      }
    }
    // c->f patches, merged per side: a coarser region goes to the side of
    // its lowest facing axis; the item's box is the bounding box of the
    // side's regions at depth Dc, and only those regions are written
    for (int a = 0; a < 3; ++a)
      for (int side = 0; side <= 2; side += 2) {
        GItem pt{};
        pt.blk = b;
        pt.sel = Nt ? 8 : 0;
        int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
        for (int r = 0; r < 27; ++r) {
          if (r == 13) continue;
          const int rr[3] = {r % 3, (r / 3) % 3, r / 9};
          int low = -1;
          for (int c = 2; c >= 0; --c)
            if (rr[c] != 1) low = c;
          if (low != a || rr[a] != side) continue;
          if (region_level(g, b, r) >= Lb) continue;
          int blo[3], bhi[3];
          region_box(nb, Dc, r, blo, bhi);
          for (int c = 0; c < 3; ++c) {
            lo[c] = std::min(lo[c], blo[c]);
            hi[c] = std::max(hi[c], bhi[c]);
          }
          pt.rmask |= 1 << r;
          P.pts += box_size(blo, bhi);
        }
        if (!pt.rmask) continue;
        for (int c = 0; c < 3; ++c) {
          pt.lo[c] = lo[c];
          pt.hi[c] = hi[c];
        }
        push_tiled(P.g, pt, glds, g->tune.lds_refine);
      }
    // Overlapping slabs (two faces meet along an edge) are cut into disjoint
    // boxes, so each point is written by exactly one item; the kernel decides
    // per point from all of the block's coarser regions whether it is taken.
    if (!slabs.empty()) {
      std::vector<GItem> acc, pieces, next;
      for (const GItem& sl : slabs) {
        pieces.assign(1, sl);
        for (const GItem& q : acc) {
          next.clear();
          for (const GItem& pc : pieces) box_subtract(pc, q, next);
          pieces.swap(next);
        }
        acc.insert(acc.end(), pieces.begin(), pieces.end());
      }
      for (const GItem& pc : acc) push_tiled(P.s, pc, slds, g->tune.lds_subst);
    }
    return true;
  };
  const int nchunk = std::max(1, std::min(64, n / 256));
  std::vector<Part> parts(nchunk);
  parallel_for(size_t(nchunk), [&](size_t c0, size_t c1) {
    for (size_t c = c0; c < c1; ++c) {
      const int lo = int(int64_t(n) * int64_t(c) / nchunk), hi = int(int64_t(n) * int64_t(c + 1) / nchunk);
      for (int b = lo; b < hi && parts[c].ok; ++b) parts[c].ok = one_block(b, parts[c]);
    }
  });
  // per part on the host threads: item checks, algorithmic traffic, LDS
  // maxima, and the restriction items split by column-length class
  auto cls = [](const RItem& it) {
    const int q = std::min(it.hi[1] - it.lo[1], it.hi[2] - it.lo[2]);
    return q <= 3 ? 0 : (q <= 6 ? 1 : (q <= 12 ? 2 : 3));
  };
  struct Post {
    int err = 0;   // 1 samples leave the map, 2 c->f too wide, 3 substitution too wide, 4 restriction too wide
    int64_t cf_w = 0, cf_r = 0, sb_w = 0, sb_r = 0, fc_w = 0, fc_r = 0;
    int lds_g = 0, lds_s = 0, lds_rc[3] = {0, 0, 0};
    std::vector<RItem> rc[3];
  };
  std::vector<Post> post(parts.size());
  parallel_for(parts.size(), [&](size_t c0, size_t c1) {
    for (size_t c = c0; c < c1; ++c) {
      const Part& P = parts[c];
      Post& Q = post[c];
      if (!P.ok) continue;
      // sample boxes of c->f items stay inside the owner map and fit the
      // kernel's per-axis cell table (32 samples)
      for (const GItem& it : P.g) {
        int64_t r = 1;
        for (int a = 0; a < 3; ++a) {
          int clo, cs;
          gview_samples(it.lo[a], it.hi[a], N, &clo, &cs);
          if (2 * clo < -nb / 2 || 2 * (clo + cs - 1) >= 3 * nb / 2) Q.err = Q.err ? Q.err : 1;
          if (cs > 32) Q.err = Q.err ? Q.err : 2;
          r *= cs;
        }
        Q.cf_r += r;
        for (int rr = 0; rr < 27; ++rr) {
          if (!((it.rmask >> rr) & 1)) continue;
          int blo[3], bhi[3];
          region_box(nb, Dc, rr, blo, bhi);
          int64_t v = 1;
          for (int a = 0; a < 3; ++a)
            v *= std::max(0, std::min(bhi[a], it.hi[a]) - std::max(blo[a], it.lo[a]));
          Q.cf_w += v;
        }
        Q.lds_g = std::max(Q.lds_g, gview_lds(it, N, esz));
      }
      // substitution items: slab points (every point of the box but the
      // all-even ones) and staged lattice points (per axis the even
      // coordinates of [lo-N+1, hi+N-1) and the odd ones of [lo, hi), at
      // most 32, the kernel's per-axis tables)
      for (const GItem& it : P.s) {
        int64_t vol = 1, ev = 1, lat = 1;
        for (int a = 0; a < 3; ++a) {
          const int lo = it.lo[a], hi = it.hi[a];
          vol *= hi - lo;
          ev *= (hi - lo + (lo & 1 ? 0 : 1)) / 2;
          const int s0 = lo - (N - 1), e0 = s0 + (s0 & 1), o0 = lo | 1;
          const int nE = (hi + N - e0) >> 1, nO = hi > o0 ? (hi - o0 + 1) >> 1 : 0;
          if (nE + nO > 32) Q.err = Q.err ? Q.err : 3;
          lat *= nE + nO;
        }
        Q.sb_r += lat;
        Q.sb_w += vol - ev;
        Q.lds_s = std::max(Q.lds_s, subst_lds(it, N, esz));
      }
      for (const RItem& it : P.r) {
        int64_t w = 1, r = 1;
        for (int a = 0; a < 3; ++a) {
          const int q = it.hi[a] - it.lo[a];
          w *= q;
          r *= 2 * (q - 1) + 1 + 2 * H;
        }
        Q.fc_w += w;
        Q.fc_r += r;
        const int k = cls(it);
        if (k > 2) {
          Q.err = Q.err ? Q.err : 4;
          continue;
        }
        Q.rc[k].push_back(it);
        Q.lds_rc[k] = std::max(Q.lds_rc[k], rview_lds(it, H, esz));
      }
    }
  });
  static const char* kPostErr[5] = {"", "refinement samples leave the owner map",
                                    "refinement item too wide", "substitution item too wide",
                                    "restriction item wider than 12 coarse points"};
  size_t ng = 0, ns = 0, nr[3] = {0, 0, 0};
  L.cf_w = L.cf_r = L.sb_w = L.sb_r = L.fc_w = L.fc_r = 0;
  L.lds_g = L.lds_s = 0;
  L.lds_rc[0] = L.lds_rc[1] = L.lds_rc[2] = 0;
  for (size_t c = 0; c < parts.size(); ++c) {
    if (!parts[c].ok) return fail(MR_EINVAL, "finer region not covered by level+1 leaves");
    const Post& Q = post[c];
    if (Q.err) return fail(MR_EINVAL, kPostErr[Q.err]);
    ng += parts[c].g.size();
    ns += parts[c].s.size();
    for (int k = 0; k < 3; ++k) {
      nr[k] += Q.rc[k].size();
      L.lds_rc[k] = std::max(L.lds_rc[k], Q.lds_rc[k]);
    }
    L.cf_w += Q.cf_w;
    L.cf_r += Q.cf_r;
    L.sb_w += Q.sb_w;
    L.sb_r += Q.sb_r;
    L.fc_w += Q.fc_w;
    L.fc_r += Q.fc_r;
    L.lds_g = std::max(L.lds_g, Q.lds_g);
    L.lds_s = std::max(L.lds_s, Q.lds_s);
    L.out_points += parts[c].pts;
  }
  // concatenation in part order (restriction items by class, then part),
  // copied on the host threads
  L.rcls[0] = 0;
  L.rcls[1] = int(nr[0]);
  L.rcls[2] = int(nr[0] + nr[1]);
  L.rcls[3] = int(nr[0] + nr[1] + nr[2]);
  L.g.resize(ng);
  L.s.resize(ns);
  L.r.resize(size_t(L.rcls[3]));
  std::vector<size_t> og(parts.size()), os(parts.size()), orr[3];
  for (int k = 0; k < 3; ++k) orr[k].resize(parts.size());
  {
    size_t a = 0, b = 0, r[3] = {0, 0, 0};
    for (size_t c = 0; c < parts.size(); ++c) {
      og[c] = a;
      os[c] = b;
      a += parts[c].g.size();
      b += parts[c].s.size();
      for (int k = 0; k < 3; ++k) {
        orr[k][c] = size_t(L.rcls[k]) + r[k];
        r[k] += post[c].rc[k].size();
      }
    }
  }
  parallel_for(parts.size(), [&](size_t c0, size_t c1) {
    for (size_t c = c0; c < c1; ++c) {
      std::copy(parts[c].g.begin(), parts[c].g.end(), L.g.begin() + og[c]);
      std::copy(parts[c].s.begin(), parts[c].s.end(), L.s.begin() + os[c]);
      for (int k = 0; k < 3; ++k)
        std::copy(post[c].rc[k].begin(), post[c].rc[k].end(), L.r.begin() + orr[k][c]);
    }
  });
  const int lds_r = std::max(L.lds_rc[0], std::max(L.lds_rc[1], L.lds_rc[2]));
  if (L.lds_g > 64 * 1024 || lds_r > 64 * 1024 || L.lds_s > 64 * 1024)
    return fail(MR_EINVAL, "ghost work item exceeds LDS");
  HIPCHK(L.dg.ensure(std::max<size_t>(1, L.g.size()) * sizeof(GItem)));
  HIPCHK(L.ds.ensure(std::max<size_t>(1, L.s.size()) * sizeof(GItem)));
  HIPCHK(L.dr.ensure(std::max<size_t>(1, L.r.size()) * sizeof(RItem)));
  if (!L.g.empty())
    HIPCHK(hipMemcpyAsync(L.dg.p, L.g.data(), L.g.size() * sizeof(GItem), hipMemcpyHostToDevice, g->stream));
  if (!L.s.empty())
    HIPCHK(hipMemcpyAsync(L.ds.p, L.s.data(), L.s.size() * sizeof(GItem), hipMemcpyHostToDevice, g->stream));
  if (!L.r.empty())
    HIPCHK(hipMemcpyAsync(L.dr.p, L.r.data(), L.r.size() * sizeof(RItem), hipMemcpyHostToDevice, g->stream));
  return MR_OK;
}

// Per coarser region r around a block: bit (lo | hi << 3 | parity << 6) set
// when a point whose per-axis front / back slab range membership is lo / hi
// and whose index parities are `parity` (not all even) lies in the slab
// toward r (front along axes where r lies below, back where above).
static const std::array<std::array<uint64_t, 8>, 27>& slab_region_tables() {
  static const std::array<std::array<uint64_t, 8>, 27> t = [] {
    std::array<std::array<uint64_t, 8>, 27> t{};
    for (int r = 0; r < 27; ++r) {
      if (r == 13) continue;
      const int d[3] = {r % 3 - 1, (r / 3) % 3 - 1, r / 9 - 1};
      for (int idx = 0; idx < 512; ++idx) {
        const int lo = idx & 7, hi = (idx >> 3) & 7, par = idx >> 6;
        bool ok = par != 0;
        for (int a = 0; a < 3; ++a) {
          if (d[a] < 0 && !((lo >> a) & 1)) ok = false;
          if (d[a] > 0 && !((hi >> a) & 1)) ok = false;
        }
        if (ok) t[r][idx >> 6] |= 1ull << (idx & 63);
      }
    }
    return t;
  }();
  return t;
}

// Upload tree metadata and rebuild every derived structure.
static mr_status commit_tree_impl(mr_grid* g);
static void build_cell_tables(mr_grid* g);
static mr_status commit_tree(mr_grid* g) {
  const double t0 = now_ms();
  mr_status st = commit_tree_impl(g);
  g->htime.ms[3] += now_ms() - t0;
  g->htime.n[3] += 1;
  return st;
}

static mr_status commit_tree_impl(mr_grid* g) {
  rebuild_index(g);
  mr_status st = build_cmap(g);
  if (st != MR_OK) return st;
  const int n = int(g->leaves.size());
  const int nb = g->nb, Dw = g->Dw;
  // patch offsets: per-block patch sizes on host threads, then a prefix sum
  g->poff.assign(size_t(n) * 27, -1);
  std::vector<int64_t> bsize(n);
  parallel_for(size_t(n), [&](size_t lo_b, size_t hi_b) {
    for (size_t b = lo_b; b < hi_b; ++b) {
      int64_t sz = 0;
      for (int r = 0; r < 27; ++r) {
        if (r == 13 || region_level(g, int(b), r) == g->leaves[b].L) continue;
        int lo[3], hi[3];
        region_box(nb, Dw, r, lo, hi);
        g->poff[b * 27 + r] = sz;   // offset inside the block's patches
        sz += box_size(lo, hi);
      }
      bsize[b] = sz;
    }
  });
  int64_t cur = 0;
  for (int b = 0; b < n; ++b) {
    const int64_t base = cur;
    cur += bsize[b];
    if (bsize[b] == 0) continue;
    for (int r = 0; r < 27; ++r)
      if (g->poff[size_t(b) * 27 + r] >= 0) g->poff[size_t(b) * 27 + r] += base;
  }
  g->patch_elems = cur;
  std::vector<int32_t> lev(n), ijk(3 * size_t(n));
  std::vector<int32_t>& cdir = g->cdir_host;
  cdir.assign(n, 0);
  parallel_for(size_t(n), [&](size_t lo_b, size_t hi_b) {
    for (size_t b = lo_b; b < hi_b; ++b) {
      int32_t m = 0;
      for (int r = 0; r < 27; ++r)
        if (r != 13 && region_level(g, int(b), r) < g->leaves[b].L) m |= 1 << r;
      cdir[b] = m;
    }
  });
  // slab tables (READING R-SUB): bit (lo | hi << 3 | parity << 6) of a block
  // is set when a point whose per-axis front / back slab range membership is
  // lo / hi and whose index parities are `parity` lies in one of the slabs
  // of the block's coarser regions and passes that slab's selector (every
  // detail of the slab, both families); a block's table is the union of the
  // tables of its coarser regions, each built once
  {
    const auto& region_table = slab_region_tables();
    g->stab_host.assign(size_t(n) * 8, 0);
    parallel_for(size_t(n), [&](size_t lo_b, size_t hi_b) {
      for (size_t b = lo_b; b < hi_b; ++b) {
        const int32_t m = cdir[b];
        for (int r = 0; r < 27; ++r)
          if ((m >> r) & 1)
            for (int w = 0; w < 8; ++w) g->stab_host[b * 8 + w] |= region_table[r][w];
      }
    });
  }
  for (int b = 0; b < n; ++b) {
    lev[b] = g->leaves[b].L;
    ijk[3 * b] = g->leaves[b].i;
    ijk[3 * b + 1] = g->leaves[b].j;
    ijk[3 * b + 2] = g->leaves[b].k;
  }
  HIPCHK(g->d_lev.ensure(std::max(1, n) * sizeof(int32_t)));
  HIPCHK(g->d_ijk.ensure(std::max(1, 3 * n) * sizeof(int32_t)));
  HIPCHK(g->d_cmap.ensure(std::max(1, 64 * n) * sizeof(int32_t)));
  HIPCHK(g->d_poff.ensure(std::max(1, 27 * n) * sizeof(int64_t)));
  HIPCHK(g->d_stab.ensure(std::max(1, n) * 8 * sizeof(uint64_t)));
  HIPCHK(g->d_patch.ensure(std::max<int64_t>(1, cur) * g->esz));
  HIPCHK(g->d_bands.ensure(std::max(1, 27 * n) * sizeof(double)));
  HIPCHK(g->d_norms.ensure(std::max(1, n) * sizeof(double)));
  if (n) {
    HIPCHK(hipMemcpyAsync(g->d_lev.p, lev.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, g->stream));
    HIPCHK(hipMemcpyAsync(g->d_ijk.p, ijk.data(), 3 * n * sizeof(int32_t), hipMemcpyHostToDevice, g->stream));
    HIPCHK(hipMemcpyAsync(g->d_cmap.p, g->cmap.data(), 64 * size_t(n) * sizeof(int32_t), hipMemcpyHostToDevice, g->stream));
    HIPCHK(hipMemcpyAsync(g->d_poff.p, g->poff.data(), 27 * size_t(n) * sizeof(int64_t), hipMemcpyHostToDevice, g->stream));
    HIPCHK(hipMemcpyAsync(g->d_stab.p, g->stab_host.data(), size_t(n) * 8 * sizeof(uint64_t), hipMemcpyHostToDevice, g->stream));
    HIPCHK(g->d_cbase.ensure(64 * size_t(n) * sizeof(int64_t)));
    HIPCHK(g->d_cstep.ensure(64 * size_t(n) * sizeof(int32_t)));
    build_cell_tables(g);
  }
  // the stage-depth and wide work lists are independent: build them on two
  // threads (the error message of the other thread is carried over)
  mr_status st_w = MR_OK;
  std::string msg_w;
  std::thread tw([&] {
    st_w = build_lists(g, g->Dw, g->wide);
    if (st_w != MR_OK) msg_w = g_errmsg;
  });
  st = build_lists(g, g->G, g->stage);
  tw.join();
  if (st != MR_OK) return st;
  if (st_w != MR_OK) {
    g_errmsg = msg_w;
    return st_w;
  }
  HIPCHK(hipStreamSynchronize(g->stream));  // host vectors above are staged
  ++g->tree_version;
  return MR_OK;
}

template <typename T>
static DevGrid<T> view(mr_grid* g, void* field, void* patch = nullptr) {
  DevGrid<T> d{};
  d.nb = g->nb;
  d.nblk = int32_t(g->leaves.size());
  d.lev = static_cast<const int32_t*>(g->d_lev.p);
  d.ijk = static_cast<const int32_t*>(g->d_ijk.p);
  d.cmap = static_cast<const int32_t*>(g->d_cmap.p);
  d.poff = static_cast<const int64_t*>(g->d_poff.p);
  d.stab = static_cast<const uint64_t*>(g->d_stab.p);
  d.cbase = static_cast<const int64_t*>(g->d_cbase.p);
  d.cstep = static_cast<const int32_t*>(g->d_cstep.p);
  d.field = static_cast<T*>(field);
  d.patch = static_cast<T*>(patch ? patch : g->d_patch.p);
  d.dw = g->Dw;
  d.err = static_cast<int32_t*>(g->d_err.p);
  return d;
}

struct AnyView {
  alignas(16) unsigned char raw[sizeof(DevGrid<double>)];
};
static AnyView anyview(mr_grid* g, void* field, void* patch = nullptr) {
  AnyView v;
  if (g->f32) {
    DevGrid<float> d = view<float>(g, field, patch);
    std::memcpy(v.raw, &d, sizeof(d));
  } else {
    DevGrid<double> d = view<double>(g, field, patch);
    std::memcpy(v.raw, &d, sizeof(d));
  }
  return v;
}

// Per-block coarse-sample address tables (depend on the tree only).
static void build_cell_tables(mr_grid* g) {
  AnyView v = anyview(g, nullptr);
  launch_cell_tables(g->f32, v.raw, int(g->leaves.size()), g->stream);
}

// Kernel timers: events stamped by the runtime at the start and end of the
// timed launch (hipExtLaunchKernel), or around a sequence of launches in the
// plain (one launch per block) mode.
static void prof_begin(mr_grid* g, int fam, hipEvent_t* a, hipEvent_t* b, bool tight) {
  (void)fam;
  *a = *b = nullptr;
  if (!g->prof.on) return;
  (void)hipEventCreate(a);
  (void)hipEventCreate(b);
  if (tight) set_launch_events(*a, *b);
  else (void)hipEventRecord(*a, g->stream);
}
static void prof_end(mr_grid* g, int fam, hipEvent_t a, hipEvent_t b, bool tight, int64_t points) {
  if (!g->prof.on) return;
  if (tight) set_launch_events(nullptr, nullptr);
  else (void)hipEventRecord(b, g->stream);
  g->prof.recs.push_back({a, b, fam});
  g->prof.points[fam] = points;
}

// Ghost reconstruction of `field` at depth D (stage G or wide Dw).
static void ghost_fill(mr_grid* g, void* field, Lists& L, void* patch = nullptr) {
  AnyView v = anyview(g, field, patch);
  const Wavelet w{g->N, g->Nt};
  const bool plain = g->cfg.exec_mode == 1;
  hipEvent_t a = nullptr, b = nullptr;
  // c->f patches, then the substitution (which reads them), each one launch
  const GItem* gi = static_cast<const GItem*>(L.dg.p);
  const GItem* si = static_cast<const GItem*>(L.ds.p);
  const int ng = int(L.g.size()), ns = int(L.s.size());
  if (ng) {
    prof_begin(g, 2, &a, &b, !plain);
    if (plain) {
      for (int i = 0; i < ng; ++i) launch_gview(g->f32, v.raw, w, gi + i, 1, L.lds_g, g->stream);
    } else {
      launch_gview(g->f32, v.raw, w, gi, ng, L.lds_g, g->stream);
    }
    prof_end(g, 2, a, b, !plain, L.out_points);
  }
  if (ns) {
    prof_begin(g, 4, &a, &b, !plain);
    if (plain) {
      for (int i = 0; i < ns; ++i)
        launch_subst(g->f32, v.raw, w, si + i, 1, L.lds_s, g->tune.subst_threads, g->stream);
    } else {
      launch_subst(g->f32, v.raw, w, si, ns, L.lds_s, g->tune.subst_threads, g->stream);
    }
    prof_end(g, 4, a, b, !plain, L.out_points);
  }
  // one launch per column-length class (the classes are independent)
  static const int kMaxq[3] = {3, 6, 12};
  const RItem* ritems = static_cast<const RItem*>(L.dr.p);
  for (int c = 0; c < 3; ++c) {
    const int i0 = L.rcls[c], i1 = L.rcls[c + 1];
    if (i1 <= i0) continue;
    prof_begin(g, 3, &a, &b, !plain);
    if (plain) {
      for (int i = i0; i < i1; ++i)
        launch_rview(g->f32, v.raw, w, ritems + i, 1, L.lds_rc[c], kMaxq[c], g->stream);
    } else {
      launch_rview(g->f32, v.raw, w, ritems + i0, i1 - i0, L.lds_rc[c], kMaxq[c], g->stream);
    }
    prof_end(g, 3, a, b, !plain, L.out_points);
  }
}

static void rhs_stage(mr_grid* g, void* y, const void* un, void* out, double a_un, double b_y,
                      double dt, const VelDev& vel, void* patch = nullptr, double c_y = 1.0) {
  AnyView v = anyview(g, y, patch);
  const int n = int(g->leaves.size());
  hipEvent_t a = nullptr, e = nullptr;
  const bool plain = g->cfg.exec_mode == 1;
  prof_begin(g, 0, &a, &e, !plain);
  if (plain) {
    for (int b = 0; b < n; ++b)
      launch_rhs(g->f32, v.raw, un, out, g->cfg.fd_order, g->G, a_un, b_y, c_y, dt, vel, b, 1,
                 g->stream);
  } else {
    launch_rhs(g->f32, v.raw, un, out, g->cfg.fd_order, g->G, a_un, b_y, c_y, dt, vel, 0, n,
               g->stream);
  }
  prof_end(g, 0, a, e, !plain, int64_t(n) * g->nb * g->nb * g->nb);
}

static void details_pass(mr_grid* g, void* field, const int32_t* det_slot, double* det_out,
                         hipStream_t st = nullptr, double* bands = nullptr,
                         double* norms = nullptr) {
  const hipStream_t strm = st ? st : g->stream;
  if (!bands) bands = static_cast<double*>(g->d_bands.p);
  if (!norms) norms = static_cast<double*>(g->d_norms.p);
  AnyView v = anyview(g, field);
  const int n = int(g->leaves.size());
  const Wavelet w{g->N, g->Nt};
  hipEvent_t a = nullptr, e = nullptr;
  const bool plain = g->cfg.exec_mode == 1;
  prof_begin(g, 1, &a, &e, !plain);
  if (plain) {
    for (int b = 0; b < n; ++b)
      launch_details(g->f32, v.raw, w, g->Ef, g->Eb, bands, det_slot, det_out, b, 1, strm);
  } else {
    launch_details(g->f32, v.raw, w, g->Ef, g->Eb, bands, det_slot, det_out, 0, n, strm);
  }
  prof_end(g, 1, a, e, !plain, int64_t(n) * g->nb * g->nb * g->nb);
  // a pass for the discarded details of an adaptation visits only the
  // blocks with a slot and leaves the norms alone
  if (!det_out) launch_combine(v.raw, bands, g->cfg.detail_ext, norms, n, strm);
}

static mr_status check_err(mr_grid* g) {
  int32_t e = 0;
  HIPCHK(hipMemcpyAsync(&e, g->d_err.p, sizeof(int32_t), hipMemcpyDeviceToHost, g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  if (e) {
    int32_t z = 0;
    HIPCHK(hipMemcpy(g->d_err.p, &z, sizeof(z), hipMemcpyHostToDevice));
    return fail(MR_EINVAL, "unsupported tree geometry met by a ghost or adaptation kernel");
  }
  return MR_OK;
}

// ------------------------------------------------------------ adaptation
enum { S_SAME = 0, S_FINER = 1, S_COARSER = -1 };

struct Plan {
  std::vector<char> refine;                     // per old block
  std::vector<Key> parents;                     // coarsening parents
  int refined = 0, coarsened = 0;
};

static void plan_from_flags(mr_grid* g, const std::vector<int>& flag,
                            const std::unordered_set<uint64_t>& created, bool allow_coarsen,
                            Plan& plan);

// Flags (READING R-TIE: >= eps_r refines, <= eps_c may coarsen) and the
// policy of the grid-adaptation supplement.
static void make_plan(mr_grid* g, const std::vector<double>& norms,
                      const std::unordered_set<uint64_t>& created, bool allow_coarsen,
                      Plan& plan, int* in_band) {
  const int n = int(g->leaves.size());
  std::vector<int> flag(n, S_SAME);
  int band = 0;
  for (int b = 0; b < n; ++b) {
    const Key& k = g->leaves[b];
    const double v = norms[b];
    if (std::fabs(v - g->cfg.eps_refine) <= 1e-4 * g->cfg.eps_refine ||
        std::fabs(v - g->cfg.eps_coarsen) <= 1e-4 * g->cfg.eps_coarsen)
      ++band;
    if (v >= g->cfg.eps_refine && k.L < g->cfg.level_max) flag[b] = S_FINER;
    else if (v <= g->cfg.eps_coarsen && k.L > g->cfg.level_min) flag[b] = S_COARSER;
  }
  if (in_band) *in_band = band;
  plan_from_flags(g, flag, created, allow_coarsen, plan);
}

// The adaptation policy of the grid-adaptation supplement on given block
// statuses: refinement has priority and propagates to coarser neighbours
// (2:1 after refining); a sibling set coarsens only if all eight leaves are
// flagged, none was created by refinement in this adaptation, and no
// neighbour is finer or refining.
static void plan_from_flags(mr_grid* g, const std::vector<int>& flag,
                            const std::unordered_set<uint64_t>& created, bool allow_coarsen,
                            Plan& plan) {
  const int n = int(g->leaves.size());
  plan.refine.assign(n, 0);
  std::vector<int> todo;
  for (int b = 0; b < n; ++b)
    if (flag[b] == S_FINER) {
      plan.refine[b] = 1;
      todo.push_back(b);
    }
  // refinement propagates to coarser 26-neighbours (2:1 after refining)
  while (!todo.empty()) {
    const int b = todo.back();
    todo.pop_back();
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          if (!dx && !dy && !dz) continue;
          int id;
          if (neighbor_kind(g, b, dx, dy, dz, &id) == -1 && !plan.refine[id]) {
            plan.refine[id] = 1;
            todo.push_back(id);
          }
        }
  }
  plan.parents.clear();
  if (allow_coarsen) {
    std::unordered_map<uint64_t, int> groups;
    for (int b = 0; b < n; ++b) {
      const Key& k = g->leaves[b];
      if (flag[b] != S_COARSER || plan.refine[b]) continue;
      if (created.count(pack(k.L, k.i, k.j, k.k))) continue;
      groups[pack(k.L - 1, k.i >> 1, k.j >> 1, k.k >> 1)]++;
    }
    // complete sibling sets, checked for finer or refining neighbours on
    // host threads (the parents keep the sets' order)
    std::vector<uint64_t> cand;
    for (auto& kv : groups)
      if (kv.second == 8) cand.push_back(kv.first);
    std::vector<char> ok(cand.size(), 1);
    parallel_for(cand.size(), [&](size_t c0, size_t c1) {
      for (size_t ci = c0; ci < c1; ++ci) {
        const uint64_t key = cand[ci];
        const int Lp = int(key >> 60);
        const int pi = int((key >> 40) & 0xFFFFF), pj = int((key >> 20) & 0xFFFFF),
                  pk = int(key & 0xFFFFF);
        bool good = true;
        for (int c = 0; c < 8 && good; ++c) {
          const int b = find_leaf(g, Lp + 1, 2 * pi + (c & 1), 2 * pj + ((c >> 1) & 1),
                                  2 * pk + ((c >> 2) & 1));
          for (int dz = -1; dz <= 1 && good; ++dz)
            for (int dy = -1; dy <= 1 && good; ++dy)
              for (int dx = -1; dx <= 1 && good; ++dx) {
                if (!dx && !dy && !dz) continue;
                int id;
                const int kind = neighbor_kind(g, b, dx, dy, dz, &id);
                if (kind == 1) good = false;                           // finer neighbour
                else if (kind == 0 && plan.refine[id]) good = false;   // refining neighbour
              }
        }
        ok[ci] = good;
      }
    });
    for (size_t ci = 0; ci < cand.size(); ++ci)
      if (ok[ci]) {
        const uint64_t key = cand[ci];
        plan.parents.push_back({int(key >> 60), int((key >> 40) & 0xFFFFF),
                                int((key >> 20) & 0xFFFFF), int(key & 0xFFFFF)});
      }
  }
  plan.refined = 0;
  for (int b = 0; b < n; ++b) plan.refined += plan.refine[b];
  plan.coarsened = int(plan.parents.size());
}

static mr_status ensure_fields(mr_grid* g) {
  const size_t bytes = size_t(g->cfg.max_blocks) * g->nb * g->nb * g->nb * g->esz;
  for (int f = 0; f < g->cfg.n_fields; ++f) {
    if (g->fields[f].bytes < bytes) HIPCHK(g->fields[f].ensure(bytes));
    if (g->alts[f].bytes < bytes) HIPCHK(g->alts[f].ensure(bytes));
  }
  if (g->tmpA.bytes < bytes) HIPCHK(g->tmpA.ensure(bytes));
  if (g->tmpB.bytes < bytes) HIPCHK(g->tmpB.ensure(bytes));
  return MR_OK;
}

// Apply a plan: new tree, refine / coarsen / copy / update every field.
static mr_status apply_plan(mr_grid* g, const Plan& plan, std::unordered_set<uint64_t>* created,
                            bool resample_only) {
  const int n_old = int(g->leaves.size());
  const int nb = g->nb;
  LeafIndex coarsen_child;   // children of the coarsened parents -> 1
  coarsen_child.build(8 * plan.parents.size());
  for (const Key& p : plan.parents)
    for (int c = 0; c < 8; ++c)
      coarsen_child.insert(pack(p.L + 1, 2 * p.i + (c & 1), 2 * p.j + ((c >> 1) & 1), 2 * p.k + ((c >> 2) & 1)), 1);
  std::vector<Key> nl;
  nl.reserve(n_old + 7 * plan.refined);
  for (int b = 0; b < n_old; ++b) {
    const Key& k = g->leaves[b];
    if (plan.refine[b]) {
      for (int c = 0; c < 8; ++c)
        nl.push_back({k.L + 1, 2 * k.i + (c & 1), 2 * k.j + ((c >> 1) & 1), 2 * k.k + ((c >> 2) & 1)});
    } else if (coarsen_child.find(pack(k.L, k.i, k.j, k.k)) < 0) {
      nl.push_back(k);
    }
  }
  for (const Key& p : plan.parents) nl.push_back(p);
  if (int64_t(nl.size()) > g->cfg.max_blocks)
    return fail(MR_ECAPACITY, "adaptation needs " + std::to_string(nl.size()) + " blocks, capacity " +
                                  std::to_string(g->cfg.max_blocks));
  sort_leaves(nl);
  LeafIndex nidx;
  nidx.build(nl.size());
  for (size_t i = 0; i < nl.size(); ++i) nidx.insert(pack(nl[i].L, nl[i].i, nl[i].j, nl[i].k), int32_t(i));
  if (created)
    for (int b = 0; b < n_old; ++b)
      if (plan.refine[b]) {
        const Key& k = g->leaves[b];
        for (int c = 0; c < 8; ++c)
          created->insert(pack(k.L + 1, 2 * k.i + (c & 1), 2 * k.j + ((c >> 1) & 1), 2 * k.k + ((c >> 2) & 1)));
      }
  if (!resample_only) {
    // ---- device work on the old tree
    const Wavelet w{g->N, g->Nt};
    std::vector<int32_t> pairs;
    std::vector<PItem> ref[3], crs[3], upd[3];
    int64_t scr = 0;
    // slots of coarsening children for their detail arrays
    std::vector<int32_t> slot(n_old, -1);
    int nslot = 0;
    for (int b = 0; b < n_old; ++b) {
      const Key& k = g->leaves[b];
      if (coarsen_child.find(pack(k.L, k.i, k.j, k.k)) >= 0) slot[b] = nslot++;
    }
    // kept blocks with a same-level neighbour in a coarsening sibling set,
    // and the directions of those neighbours (host threads, one block each)
    std::vector<char> touches(n_old, 0);
    std::vector<int32_t> tdirs(n_old, 0);
    parallel_for(size_t(n_old), [&](size_t b0, size_t b1) {
      for (size_t b = b0; b < b1; ++b) {
        if (slot[b] >= 0) continue;
        const Key& k = g->leaves[b];
        int32_t m = 0;
        for (int r = 0; r < 27; ++r) {
          if (r == 13) continue;
          const int id = find_leaf(g, k.L, k.i + r % 3 - 1, k.j + (r / 3) % 3 - 1, k.k + r / 9 - 1);
          if (id >= 0 && slot[id] >= 0) m |= 1 << r;
        }
        touches[b] = m != 0;
        tdirs[b] = m;
      }
    });
    // discarded details per slot: all of a child's; of a kept neighbour,
    // its coarse-extension slab toward the coarsening children (the update
    // of section 2.2.1 discards those too, up to the coarse region
    // extension of Table 3)
    std::vector<int32_t> dirs(nslot, kDiscardAll);
    for (int b = 0; b < n_old; ++b) {
      if (!touches[b]) continue;
      slot[b] = nslot++;
      dirs.push_back(tdirs[b]);
    }
    const int H = Hreach(g->N, g->Nt);
    // item sets in block order: 8 refinement sets per refined block, one
    // coarsening set per coarsening child, one copy pair and possibly one
    // update set per kept block; each set takes two scratch boxes of fixed
    // size.  Counted, then written, per contiguous chunk of blocks on host
    // threads, with offsets and scratch in block order.
    const int hb2 = nb / 2;
    const int Rup = std::max(g->Nt ? 1 : 0, g->Nt ? g->N : g->N - 1);
    const int64_t ref_sc = int64_t(nb) * (hb2 + g->N) * (hb2 + g->N) + int64_t(nb) * nb * (hb2 + g->N);
    const int64_t crs_sc = int64_t(hb2) * (nb - 1 + 2 * H) * (nb - 1 + 2 * H) +
                           int64_t(hb2) * hb2 * (nb - 1 + 2 * H);
    const int64_t upd_sc = int64_t(nb + 2 * Rup) * (nb + 2 * Rup) * nb + int64_t(nb + 2 * Rup) * nb * nb;
    const int nch = std::max(1, std::min(64, n_old / 256));
    struct Cnt {
      size_t ref = 0, crs = 0, upd = 0, pairs = 0;
      int64_t sc = 0;
    };
    std::vector<Cnt> cnt(nch + 1);
    auto chunk_lo = [&](size_t c) { return int(int64_t(n_old) * int64_t(c) / nch); };
    parallel_for(size_t(nch), [&](size_t c0, size_t c1) {
      for (size_t c = c0; c < c1; ++c) {
        Cnt& C = cnt[c + 1];
        for (int b = chunk_lo(c); b < chunk_lo(c + 1); ++b) {
          const Key& k = g->leaves[b];
          if (plan.refine[b]) {
            C.ref += 8;
            C.sc += 8 * ref_sc;
          } else if (coarsen_child.find(pack(k.L, k.i, k.j, k.k)) >= 0) {
            C.crs += 1;
            C.sc += crs_sc;
          } else {
            C.pairs += 1;
            if (touches[b]) {
              C.upd += 1;
              C.sc += upd_sc;
            }
          }
        }
      }
    });
    for (int c = 0; c < nch; ++c) {
      cnt[c + 1].ref += cnt[c].ref;
      cnt[c + 1].crs += cnt[c].crs;
      cnt[c + 1].upd += cnt[c].upd;
      cnt[c + 1].pairs += cnt[c].pairs;
      cnt[c + 1].sc += cnt[c].sc;
    }
    for (int p = 0; p < 3; ++p) {
      ref[p].resize(cnt[nch].ref);
      crs[p].resize(cnt[nch].crs);
      upd[p].resize(cnt[nch].upd);
    }
    pairs.resize(2 * cnt[nch].pairs);
    scr = cnt[nch].sc;
    std::vector<char> layout_ok(nch, 1);
    parallel_for(size_t(nch), [&](size_t c0, size_t c1) {
      for (size_t ch = c0; ch < c1; ++ch) {
        size_t ir = cnt[ch].ref, ic = cnt[ch].crs, iu = cnt[ch].upd, ip = cnt[ch].pairs;
        int64_t sc = cnt[ch].sc;
        const int blo = chunk_lo(ch), bhi = chunk_lo(ch + 1);
        for (int b = blo; b < bhi; ++b) {
          const Key& k = g->leaves[b];
          const uint64_t key = pack(k.L, k.i, k.j, k.k);
          if (plan.refine[b]) {
            for (int c = 0; c < 8; ++c) {
              const int o[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
              const int child = nidx.find(pack(k.L + 1, 2 * k.i + o[0], 2 * k.j + o[1], 2 * k.k + o[2]));
              int flo[3], fhi[3], clo[3], chi[3];
              for (int a = 0; a < 3; ++a) {
                flo[a] = o[a] * nb;
                fhi[a] = flo[a] + nb;
                clo[a] = o[a] * nb / 2 - g->N / 2;
                chi[a] = o[a] * nb / 2 + nb / 2 + g->N / 2;
              }
              PItem p0{}, p1{}, p2{};
              p0.src_blk = p1.src_blk = p2.src_blk = b;
              p0.dst_blk = p1.dst_blk = p2.dst_blk = child;
              const int b0lo[3] = {flo[0], clo[1], clo[2]}, b0hi[3] = {fhi[0], chi[1], chi[2]};
              const int b1lo[3] = {flo[0], flo[1], clo[2]}, b1hi[3] = {fhi[0], fhi[1], chi[2]};
              for (int a = 0; a < 3; ++a) {
                p0.lo[a] = b0lo[a]; p0.hi[a] = b0hi[a];
                p1.lo[a] = b1lo[a]; p1.hi[a] = b1hi[a];
                p1.ilo[a] = b0lo[a]; p1.isz[a] = b0hi[a] - b0lo[a];
                p2.lo[a] = flo[a]; p2.hi[a] = fhi[a];
                p2.ilo[a] = b1lo[a]; p2.isz[a] = b1hi[a] - b1lo[a];
                p2.dlo[a] = flo[a];
              }
              p0.out_off = sc;
              p1.in_off = sc;
              sc += box_size(b0lo, b0hi);
              p1.out_off = sc;
              p2.in_off = sc;
              sc += box_size(b1lo, b1hi);
              ref[0][ir] = p0;
              ref[1][ir] = p1;
              ref[2][ir] = p2;
              ++ir;
            }
          } else if (coarsen_child.find(key) >= 0) {
            const int o[3] = {k.i & 1, k.j & 1, k.k & 1};
            const int parent = nidx.find(pack(k.L - 1, k.i >> 1, k.j >> 1, k.k >> 1));
            const int hb = nb / 2;
            const int b0lo[3] = {0, -H, -H}, b0hi[3] = {hb, nb - 1 + H, nb - 1 + H};
            const int b1lo[3] = {0, 0, -H}, b1hi[3] = {hb, hb, nb - 1 + H};
            const int b2lo[3] = {0, 0, 0}, b2hi[3] = {hb, hb, hb};
            PItem p0{}, p1{}, p2{};
            p0.src_blk = p1.src_blk = p2.src_blk = b;
            p0.dst_blk = p1.dst_blk = p2.dst_blk = parent;
            for (int a = 0; a < 3; ++a) {
              p0.lo[a] = b0lo[a]; p0.hi[a] = b0hi[a];
              p1.lo[a] = b1lo[a]; p1.hi[a] = b1hi[a];
              p1.ilo[a] = b0lo[a]; p1.isz[a] = b0hi[a] - b0lo[a];
              p2.lo[a] = b2lo[a]; p2.hi[a] = b2hi[a];
              p2.ilo[a] = b1lo[a]; p2.isz[a] = b1hi[a] - b1lo[a];
              p2.dlo[a] = -o[a] * hb;
            }
            p0.out_off = sc;
            p1.in_off = sc;
            sc += box_size(b0lo, b0hi);
            p1.out_off = sc;
            p2.in_off = sc;
            sc += box_size(b1lo, b1hi);
            crs[0][ic] = p0;
            crs[1][ic] = p1;
            crs[2][ic] = p2;
            ++ic;
          } else {
            const int nid = nidx.find(key);
            pairs[2 * ip] = nid;
            pairs[2 * ip + 1] = b;
            ++ip;
            // update step on kept blocks next to a coarsening sibling set of
            // their own level (Table 3, update after neighbour has coarsened)
            if (touches[b]) {
              int r = 0;
              const int Jr = g->Nt ? 1 : 0, Kr = g->Nt ? g->N : g->N - 1;
              r = std::max(Jr, Kr);
              const int b0lo[3] = {-r, -r, 0}, b0hi[3] = {nb + r, nb + r, nb};
              const int b1lo[3] = {-r, 0, 0}, b1hi[3] = {nb + r, nb, nb};
              const int b2lo[3] = {0, 0, 0}, b2hi[3] = {nb, nb, nb};
              PItem p0{}, p1{}, p2{};
              p0.src_blk = p1.src_blk = p2.src_blk = b;
              p0.dst_blk = p1.dst_blk = p2.dst_blk = nid;
              for (int a = 0; a < 3; ++a) {
                p0.lo[a] = b0lo[a]; p0.hi[a] = b0hi[a];
                p1.lo[a] = b1lo[a]; p1.hi[a] = b1hi[a];
                p1.ilo[a] = b0lo[a]; p1.isz[a] = b0hi[a] - b0lo[a];
                p2.lo[a] = b2lo[a]; p2.hi[a] = b2hi[a];
                p2.ilo[a] = b1lo[a]; p2.isz[a] = b1hi[a] - b1lo[a];
                p2.dlo[a] = 0;
              }
              p0.out_off = sc;
              p1.in_off = sc;
              sc += box_size(b0lo, b0hi);
              p1.out_off = sc;
              p2.in_off = sc;
              sc += box_size(b1lo, b1hi);
              upd[0][iu] = p0;
              upd[1][iu] = p1;
              upd[2][iu] = p2;
              ++iu;
            }
          }
        }
        if (sc != cnt[ch + 1].sc) layout_ok[ch] = 0;
      }
    });
    for (int c = 0; c < nch; ++c)
      if (!layout_ok[c]) return fail(MR_EINVAL, "adaptation scratch layout does not add up");
    // grow-only buffers kept by the grid (no allocation per adaptation)
    DevBuf& d_pairs = g->ad_pairs;
    DevBuf& d_items = g->ad_items;
    DevBuf& d_scr = g->ad_scr;
    DevBuf& d_det = g->ad_det;
    DevBuf& d_slot = g->ad_slot;
    // per slot the table of discarded details: all details of a coarsening
    // child, the union of the slabs toward its directions for a kept block
    DevBuf& d_dirs = g->ad_dirs;
    std::vector<uint64_t> dtab(size_t(std::max(1, nslot)) * 8, 0);
    {
      const auto& rt = slab_region_tables();
      for (int sl = 0; sl < nslot; ++sl) {
        uint64_t* t = &dtab[size_t(sl) * 8];
        if (dirs[sl] == kDiscardAll) {
          for (int w = 1; w < 8; ++w) t[w] = ~0ull;   // every point with an odd index
        } else {
          for (int r = 0; r < 27; ++r)
            if ((dirs[sl] >> r) & 1)
              for (int w = 0; w < 8; ++w) t[w] |= rt[r][w];
        }
      }
    }
    HIPCHK(d_dirs.ensure(dtab.size() * sizeof(uint64_t)));
    if (nslot)
      HIPCHK(hipMemcpyAsync(d_dirs.p, dtab.data(), size_t(nslot) * 8 * sizeof(uint64_t),
                            hipMemcpyHostToDevice, g->stream));
    HIPCHK(d_scr.ensure(std::max<int64_t>(1, scr) * sizeof(double)));
    HIPCHK(d_det.ensure(std::max<int64_t>(1, int64_t(nslot) * nb * nb * nb) * sizeof(double)));
    HIPCHK(d_slot.ensure(std::max(1, n_old) * sizeof(int32_t)));
    HIPCHK(hipMemcpyAsync(d_slot.p, slot.data(), n_old * sizeof(int32_t), hipMemcpyHostToDevice, g->stream));
    HIPCHK(d_pairs.ensure(std::max<size_t>(1, pairs.size()) * sizeof(int32_t)));
    if (!pairs.empty())
      HIPCHK(hipMemcpyAsync(d_pairs.p, pairs.data(), pairs.size() * sizeof(int32_t), hipMemcpyHostToDevice, g->stream));
    // all pass items in one upload: [ref0 ref1 ref2 crs0 crs1 crs2 upd0 upd1 upd2]
    std::vector<PItem> all;
    size_t offs[10];
    size_t cur = 0;
    std::vector<PItem>* groups[3] = {ref, crs, upd};
    for (int gi = 0; gi < 3; ++gi)
      for (int p = 0; p < 3; ++p) {
        offs[gi * 3 + p] = cur;
        all.insert(all.end(), groups[gi][p].begin(), groups[gi][p].end());
        cur += groups[gi][p].size();
      }
    offs[9] = cur;
    HIPCHK(d_items.ensure(std::max<size_t>(1, all.size()) * sizeof(PItem)));
    if (!all.empty())
      HIPCHK(hipMemcpyAsync(d_items.p, all.data(), all.size() * sizeof(PItem), hipMemcpyHostToDevice, g->stream));
    const PItem* items = static_cast<const PItem*>(d_items.p);
    double* scrp = static_cast<double*>(d_scr.p);
    for (int f = 0; f < g->cfg.n_fields; ++f) {
      void* src = g->fields[f].p;
      void* dst = g->alts[f].p;
      ghost_fill(g, src, g->wide);
      AnyView v = anyview(g, src);
      if (nslot && !upd[0].empty())
        details_pass(g, src, static_cast<const int32_t*>(d_slot.p), static_cast<double*>(d_det.p));
      launch_copy_blocks(g->f32, src, dst, static_cast<const int32_t*>(d_pairs.p), int(pairs.size() / 2), nb, g->stream);
      // refine: x, y, z passes of the zero-detail refinement
      for (int p = 0; p < 3; ++p)
        launch_pass(g->f32, v.raw, w, F_REFINE, p, p == 0 ? 0 : 1, p == 2 ? 1 : 0, items + offs[p],
                    int(ref[p].size()), scrp, scrp, nullptr, nullptr, nullptr, dst, g->stream);
      for (int p = 0; p < 3; ++p)
        launch_pass(g->f32, v.raw, w, F_RESTRICT, p, p == 0 ? 0 : 1, p == 2 ? 1 : 0, items + offs[3 + p],
                    int(crs[p].size()), scrp, scrp, nullptr, nullptr, nullptr, dst, g->stream);
      // update: synthesis of the discarded details along z, then y, then x
      const int ax[3] = {2, 1, 0};
      for (int p = 0; p < 3; ++p)
        launch_pass(g->f32, v.raw, w, F_SYNTH, ax[p], p == 0 ? 2 : 1, p == 2 ? 2 : 0, items + offs[6 + p],
                    int(upd[p].size()), scrp, scrp, static_cast<const double*>(d_det.p),
                    static_cast<const int32_t*>(d_slot.p), static_cast<const uint32_t*>(d_dirs.p),
                    dst, g->stream);
    }
    mr_status st = check_err(g);
    HIPCHK(hipStreamSynchronize(g->stream));
    if (st != MR_OK) return st;
    for (int f = 0; f < g->cfg.n_fields; ++f) std::swap(g->fields[f], g->alts[f]);
  }
  g->leaves = nl;
  return commit_tree(g);
}

static mr_status norms_to_host(mr_grid* g, int field, std::vector<double>& out) {
  ghost_fill(g, g->fields[field].p, g->wide);
  details_pass(g, g->fields[field].p, nullptr, nullptr);
  out.resize(g->leaves.size());
  if (!out.empty())
    HIPCHK(hipMemcpyAsync(out.data(), g->d_norms.p, out.size() * sizeof(double), hipMemcpyDeviceToHost, g->stream));
  mr_status st = check_err(g);
  if (st != MR_OK) return st;
  for (double v : out)
    if (!std::isfinite(v)) return fail(MR_ENONFINITE, "non-finite detail norm");
  return MR_OK;
}

// One adaptation iteration with caller-given block statuses (no criterion).
static mr_status adapt_with_flags(mr_grid* g, const int8_t* user, mr_adapt_stats* stats) {
  const int n = int(g->leaves.size());
  std::vector<int> flag(n, S_SAME);
  for (int b = 0; b < n; ++b) {
    const Key& k = g->leaves[b];
    if (user[b] > 0 && k.L < g->cfg.level_max) flag[b] = S_FINER;
    else if (user[b] < 0 && k.L > g->cfg.level_min) flag[b] = S_COARSER;
  }
  Plan plan;
  plan_from_flags(g, flag, {}, true, plan);
  mr_adapt_stats s{};
  if (plan.refined || plan.coarsened) {
    int64_t nn = int64_t(n) + 7 * int64_t(plan.refined) - 7 * int64_t(plan.coarsened);
    if (nn > g->cfg.max_blocks)
      return fail(MR_ECAPACITY, "adaptation needs " + std::to_string(nn) + " blocks, capacity " +
                                    std::to_string(g->cfg.max_blocks));
    mr_status st = apply_plan(g, plan, nullptr, false);
    if (st != MR_OK) return st;
    s.iters = 1;
    s.refined = plan.refined;
    s.coarsened = plan.coarsened;
  }
  s.n_blocks = int64_t(g->leaves.size());
  if (stats) *stats = s;
  return MR_OK;
}

static mr_status adapt_iterations(mr_grid* g, int field, int max_iter, mr_adapt_stats* stats,
                                  const int8_t* user_flags = nullptr) {
  if (user_flags) return adapt_with_flags(g, user_flags, stats);
  std::unordered_set<uint64_t> created;
  mr_adapt_stats s{};
  HostTimer& ht = g->htime;
  for (int it = 0; it < max_iter; ++it) {
    std::vector<double> norms;
    double t0 = now_ms();
    mr_status st = norms_to_host(g, field, norms);
    ht.ms[0] += now_ms() - t0;
    ht.n[0] += 1;
    if (st != MR_OK) return st;
    Plan plan;
    int band = 0;
    t0 = now_ms();
    make_plan(g, norms, created, true, plan, &band);
    ht.ms[1] += now_ms() - t0;
    ht.n[1] += 1;
    s.in_band = band;
    if (plan.refined == 0 && plan.coarsened == 0) break;
    int64_t nn = int64_t(g->leaves.size()) + 7 * int64_t(plan.refined) - 7 * int64_t(plan.coarsened);
    if (nn > g->cfg.max_blocks)
      return fail(MR_ECAPACITY, "adaptation needs " + std::to_string(nn) + " blocks, capacity " +
                                    std::to_string(g->cfg.max_blocks));
    t0 = now_ms();
    const double c0 = ht.ms[3];
    st = apply_plan(g, plan, &created, false);
    ht.ms[2] += now_ms() - t0 - (ht.ms[3] - c0);   // the commit is timed on its own
    ht.n[2] += 1;
    if (st != MR_OK) return st;
    s.iters++;
    s.refined += plan.refined;
    s.coarsened += plan.coarsened;
  }
  s.n_blocks = int64_t(g->leaves.size());
  if (stats) *stats = s;
  return MR_OK;
}

// mr_adapt is transactional over the whole call: the tree and every field
// (which the ghost reconstructions of the criterion substitute in place) are
// saved first; when the call fails with MR_ECAPACITY or MR_ENONFINITE they
// are restored bit for bit.
static mr_status adapt_impl(mr_grid* g, int field, int max_iter, mr_adapt_stats* stats,
                            const int8_t* user_flags = nullptr) {
  const std::vector<Key> saved = g->leaves;
  const size_t bytes = g->leaves.size() * size_t(g->nb) * g->nb * g->nb * g->esz;
  g->backup.resize(g->cfg.n_fields);
  for (int f = 0; f < g->cfg.n_fields; ++f) {
    HIPCHK(g->backup[f].ensure(bytes));
    HIPCHK(hipMemcpyAsync(g->backup[f].p, g->fields[f].p, bytes, hipMemcpyDeviceToDevice, g->stream));
  }
  mr_status st = adapt_iterations(g, field, max_iter, stats, user_flags);
  if (st != MR_ECAPACITY && st != MR_ENONFINITE) return st;
  const std::string msg = g_errmsg;
  (void)hipStreamSynchronize(g->stream);
  for (int f = 0; f < g->cfg.n_fields; ++f)
    HIPCHK(hipMemcpyAsync(g->fields[f].p, g->backup[f].p, bytes, hipMemcpyDeviceToDevice, g->stream));
  if (g->leaves.size() != saved.size() || !std::equal(saved.begin(), saved.end(), g->leaves.begin(),
                                                      [](const Key& a, const Key& b) {
                                                        return a.L == b.L && a.i == b.i &&
                                                               a.j == b.j && a.k == b.k;
                                                      })) {
    g->leaves = saved;
    mr_status c = commit_tree(g);
    if (c != MR_OK) return c;
  }
  HIPCHK(hipStreamSynchronize(g->stream));
  g_errmsg = msg;
  return st;
}

static mr_status upload_ic(mr_grid* g, int field, const mr_ic* ic) {
  int np = ic->kind == MR_IC_GAUSS_SUM ? 5 * ic->n : 4;
  if (np <= 0 || !ic->params) return fail(MR_EINVAL, "initial condition without parameters");
  HIPCHK(g->d_icpar.ensure(np * sizeof(double)));
  HIPCHK(hipMemcpyAsync(g->d_icpar.p, ic->params, np * sizeof(double), hipMemcpyHostToDevice, g->stream));
  IcDev d{ic->kind, ic->n, static_cast<const double*>(g->d_icpar.p)};
  AnyView v = anyview(g, g->fields[field].p);
  launch_sample_ic(g->f32, v.raw, d, g->stream);
  HIPCHK(hipStreamSynchronize(g->stream));
  return MR_OK;
}

static double usum(const mr_velocity& v) {
  if (v.kind == MR_VEL_SHEAR) return 3.0;
  if (v.kind == MR_VEL_ROTATING)
    return std::max(std::fabs(v.p[1]), std::fabs(1 - v.p[1])) +
           std::max(std::fabs(v.p[0]), std::fabs(1 - v.p[0])) + std::fabs(v.p[2]);
  return std::fabs(v.p[0]) + std::fabs(v.p[1]) + std::fabs(v.p[2]);
}

// One SSP-RK3 step: each stage reconstructs the ghosts of its input, then
// applies the RHS and the stage update.
static void enqueue_rk3(mr_grid* g, int field, double dt, const VelDev& vd) {
  void* u = g->fields[field].p;
  void* A = g->tmpA.p;
  void* B = g->tmpB.p;
  ghost_fill(g, u, g->stage);
  rhs_stage(g, u, u, A, 0.0, 1.0, dt, vd);
  ghost_fill(g, A, g->stage);
  rhs_stage(g, A, u, B, 0.75, 0.25, dt, vd);
  ghost_fill(g, B, g->stage);
  rhs_stage(g, B, u, u, 1.0 / 3.0, 2.0 / 3.0, dt, vd);
}

// Detail pass + RK3 step.  The wide reconstruction of the field serves both
// the detail pass and the first stage (its patches hold every value of the
// stage depth).  The detail pass reads only the field and those patches, so
// it runs on the second stream while the step goes on: the later stages
// reconstruct into the second patch buffer, and the last stage, which
// overwrites the field, waits for the detail pass.  With the kernel timers
// on, everything runs in order on the grid's stream.
static void enqueue_fused(mr_grid* g, int field, double dt, const VelDev& vd) {
  void* u = g->fields[field].p;
  void* A = g->tmpA.p;
  void* B = g->tmpB.p;
  ghost_fill(g, u, g->wide);
  const bool fork = g->aux && !g->prof.on && g->d_patch2.p;
  void* p2 = fork ? g->d_patch2.p : nullptr;
  if (fork) {
    (void)hipEventRecord(g->ev_fork, g->stream);
    (void)hipStreamWaitEvent(g->aux, g->ev_fork, 0);
    details_pass(g, u, nullptr, nullptr, g->aux);
    (void)hipEventRecord(g->ev_join, g->aux);
  } else {
    details_pass(g, u, nullptr, nullptr);
  }
  rhs_stage(g, u, u, A, 0.0, 1.0, dt, vd);
  ghost_fill(g, A, g->stage, p2);
  rhs_stage(g, A, u, B, 0.75, 0.25, dt, vd, p2);
  ghost_fill(g, B, g->stage, p2);
  if (fork) (void)hipStreamWaitEvent(g->stream, g->ev_join, 0);
  rhs_stage(g, B, u, u, 1.0 / 3.0, 2.0 / 3.0, dt, vd, p2);
}

static mr_status check_step_args(mr_grid* g, int32_t field, double dt, const mr_velocity* vel,
                                 VelDev& vd) {
  if (!g || !vel || field < 0 || field >= g->cfg.n_fields) return fail(MR_EINVAL, "bad argument");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(MR_EINVAL, "dt must be positive");
  if (vel->kind < 0 || vel->kind > 3) return fail(MR_EINVAL, "unknown velocity kind");
  if (vel->kind == MR_VEL_DIFFUSION &&
      (g->cfg.fd_order % 2 != 0 || !(vel->p[0] >= 0) || !std::isfinite(vel->p[0])))
    return fail(MR_EINVAL, "diffusion needs fd_order 2, 4 or 6 and a finite nu >= 0");
  vd = VelDev{};
  vd.kind = vel->kind;
  for (int i = 0; i < 8; ++i) vd.p[i] = vel->p[i];
  return MR_OK;
}

// Enqueue `work` on the grid's stream, through a captured graph in graph
// mode (re-captured when the tree, the field, dt or the velocity changed).
template <typename F>
static mr_status run_step(mr_grid* g, mr_grid::StepGraph& sg, int32_t field, double dt,
                          const mr_velocity* vel, F&& work) {
  if (g->cfg.exec_mode == 2 && !g->prof.on) {
    const bool same = sg.exec && sg.version == g->tree_version && sg.dt == dt &&
                      sg.field == field && std::memcmp(&sg.vel, vel, sizeof(mr_velocity)) == 0;
    if (!same) {
      sg.reset();
      HIPCHK(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
      work();
      HIPCHK(hipStreamEndCapture(g->stream, &sg.graph));
      HIPCHK(hipGraphInstantiate(&sg.exec, sg.graph, nullptr, nullptr, 0));
      sg.version = g->tree_version;
      sg.dt = dt;
      sg.field = field;
      sg.vel = *vel;
    }
    HIPCHK(hipGraphLaunch(sg.exec, g->stream));
    return MR_OK;
  }
  work();
  return MR_OK;
}

// Release everything a grid holds (also on the error paths of creation).
static void free_grid(mr_grid* g) {
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  if (g->aux) (void)hipStreamSynchronize(g->aux);
  g->rk3_graph.reset();
  g->fused_graph.reset();
  for (auto& r : g->prof.recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto& b : g->fields) b.release();
  for (auto& b : g->alts) b.release();
  for (auto& b : g->backup) b.release();
  DevBuf* bufs[] = {&g->tmpA, &g->tmpB, &g->d_lev, &g->d_ijk, &g->d_cmap, &g->d_poff, &g->d_patch,
                    &g->d_err, &g->d_bands, &g->d_norms, &g->d_icpar, &g->d_mom,
                    &g->stage.dg, &g->stage.ds, &g->stage.dr, &g->wide.dg, &g->wide.ds,
                    &g->wide.dr, &g->ad_pairs, &g->d_cbase, &g->d_cstep, &g->d_stab, &g->d_patch2,
                    &g->ad_items, &g->ad_scr, &g->ad_det, &g->ad_slot, &g->ad_dirs};
  for (DevBuf* b : bufs) b->release();
  if (g->aux) {
    (void)hipEventDestroy(g->ev_fork);
    (void)hipEventDestroy(g->ev_join);
    (void)hipStreamDestroy(g->aux);
  }
  if (g->own_stream) (void)hipStreamDestroy(g->stream);
  delete g;
}

}  // namespace mr

// =================================================================== C ABI
extern "C" {

const char* mr_last_error(void) { return g_errmsg.c_str(); }

// Bytes of the fixed-capacity field buffers (fields, their adaptation
// alternates and two work buffers), each a 256-byte-aligned slice.
static size_t pool_need(const mr_config& c) {
  const size_t esz = c.prec == MR_F32 ? 4 : 8;
  const size_t one = (size_t(c.max_blocks) * c.nb * c.nb * c.nb * esz + 255) / 256 * 256;
  return one * (2 * size_t(c.n_fields) + 2);
}

mr_status mr_pool_bytes(const mr_config* cfg, size_t* bytes) {
  if (!cfg || !bytes) return fail(MR_EINVAL, "null argument");
  if (cfg->n_fields < 1 || cfg->n_fields > 8 || cfg->max_blocks < 1 ||
      (cfg->nb != 8 && cfg->nb != 16 && cfg->nb != 24) || (cfg->prec != MR_F64 && cfg->prec != MR_F32))
    return fail(MR_EINVAL, "invalid configuration");
  *bytes = pool_need(*cfg);
  return MR_OK;
}

mr_status mr_grid_create(const mr_config* cfg, void* hip_stream, void* dev_pool, size_t pool_bytes,
                         mr_grid** out) {
  if (!cfg || !out) return fail(MR_EINVAL, "null argument");
  const mr_config& c = *cfg;
  if (c.nb != 8 && c.nb != 16 && c.nb != 24) return fail(MR_EINVAL, "nb must be 8, 16 or 24");
  if (c.wavelet_N != 2 && c.wavelet_N != 4 && c.wavelet_N != 6) return fail(MR_EINVAL, "wavelet_N must be 2, 4 or 6");
  if (c.wavelet_Nt != 0 && c.wavelet_Nt != 2) return fail(MR_EINVAL, "wavelet_Nt must be 0 or 2");
  if (c.fd_order < 2 || c.fd_order > 6)
    return fail(MR_EINVAL, "fd_order must be 2, 4 or 6 (central) or 3 or 5 (CONS-3 / CONS-5)");
  if (c.level_min < 0 || c.level_max < c.level_min || c.level_max > 12)
    return fail(MR_EINVAL, "need 0 <= level_min <= level_max <= 12");
  if (c.prec != MR_F64 && c.prec != MR_F32) return fail(MR_EINVAL, "prec must be MR_F64 or MR_F32");
  if (c.n_fields < 1 || c.n_fields > 8) return fail(MR_EINVAL, "n_fields must be 1..8");
  if (c.exec_mode < 0 || c.exec_mode > 2) return fail(MR_EINVAL, "exec_mode must be 0, 1 or 2");
  if (!(c.eps_refine > c.eps_coarsen) || !(c.eps_coarsen >= 0))
    return fail(MR_EINVAL, "need eps_refine > eps_coarsen >= 0");
  const int64_t n0 = int64_t(1) << (3 * c.level_min);
  if (c.max_blocks < n0 || c.max_blocks > (int64_t(1) << 31))
    return fail(MR_EINVAL, "max_blocks must hold the level_min tree and fit int32");
  if (dev_pool && (reinterpret_cast<uintptr_t>(dev_pool) % 256 != 0))
    return fail(MR_EINVAL, "dev_pool must be 256-byte aligned");
  if (dev_pool && pool_bytes < pool_need(c))
    return fail(MR_EINVAL, "dev_pool holds " + std::to_string(pool_bytes) + " bytes, the fields need " +
                               std::to_string(pool_need(c)) + " (mr_pool_bytes)");
  mr_grid* g = new mr_grid();
  g->cfg = c;
  g->stream = static_cast<hipStream_t>(hip_stream);
  if (!g->stream) {
    // a private non-blocking stream (default priority): the legacy NULL
    // stream cannot be captured into a graph
    if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess) {
      free_grid(g);
      return fail(MR_EHIP, "hipStreamCreateWithFlags failed");
    }
    g->own_stream = true;
  }
  if (hipStreamCreateWithFlags(&g->aux, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&g->ev_join, hipEventDisableTiming) != hipSuccess) {
    // without them the fused step runs its detail pass in order
    if (g->ev_fork) (void)hipEventDestroy(g->ev_fork);
    if (g->aux) (void)hipStreamDestroy(g->aux);
    g->aux = nullptr;
    g->ev_fork = g->ev_join = nullptr;
    (void)hipGetLastError();
  }
  g->f32 = c.prec == MR_F32;
  g->esz = g->f32 ? 4 : 8;
  g->nb = c.nb;
  g->N = c.wavelet_N;
  g->Nt = c.wavelet_Nt;
  g->G = (c.fd_order + 1) / 2;   // FD2: 1, FD4 / CONS-3: 2, FD6 / CONS-5: 3
  const int H = Hreach(g->N, g->Nt);
  const int tf = std::max(H, g->N - 2), tb = std::max(H - 1, g->N - 1);
  g->Dw = std::max({g->G, tf, tb, g->N / 2, H});
  static const int ext[2][7][2] = {{{0, 0}, {0, 0}, {0, 1}, {0, 0}, {2, 3}, {0, 0}, {4, 5}},
                                   {{0, 0}, {0, 0}, {1, 2}, {0, 0}, {3, 4}, {0, 0}, {5, 6}}};
  g->Ef = ext[g->Nt / 2][g->N][0];
  g->Eb = ext[g->Nt / 2][g->N][1];
  // every sample of a ghost reconstruction must lie in the half-block shell
  // covered by the owner map: coarse samples reach ceil(Dw/2) + N/2 coarse
  // points beyond the block
  if (2 * ((g->Dw + 1) / 2 + g->N / 2) > g->nb / 2) {
    const int Dw = g->Dw;
    free_grid(g);
    return fail(MR_EINVAL, "nb too small for this wavelet: ghost depth " + std::to_string(Dw) +
                               " plus the refinement reach must fit in nb/2");
  }
  g->fields.resize(c.n_fields);
  g->alts.resize(c.n_fields);
  if (dev_pool) {
    // fixed-capacity field buffers as slices of the caller's pool
    const size_t one = pool_need(c) / (2 * size_t(c.n_fields) + 2);
    unsigned char* q = static_cast<unsigned char*>(dev_pool);
    for (int f = 0; f < c.n_fields; ++f) {
      g->fields[f].adopt(q, one);
      q += one;
      g->alts[f].adopt(q, one);
      q += one;
    }
    g->tmpA.adopt(q, one);
    q += one;
    g->tmpB.adopt(q, one);
  }
  std::string warn;
  if (c.eps_refine / std::max(c.eps_coarsen, 1e-300) <= double(1 << g->N))
    warn = "warning: eps_refine/eps_coarsen <= 2^N may flip-flop (section 2.2.5)";
  if (g->d_err.ensure(sizeof(int32_t)) != hipSuccess || g->d_mom.ensure(4 * sizeof(double)) != hipSuccess) {
    free_grid(g);
    return fail(MR_ENOMEM, "device allocation failed");
  }
  int32_t z = 0;
  if (hipMemcpy(g->d_err.p, &z, sizeof(z), hipMemcpyHostToDevice) != hipSuccess) {
    free_grid(g);
    return fail(MR_EHIP, "hipMemcpy failed");
  }
  mr_status st = ensure_fields(g);
  if (st != MR_OK) {
    free_grid(g);
    return fail(MR_ENOMEM, "field allocation failed: " + g_errmsg);
  }
  const int n = 1 << c.level_min;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) g->leaves.push_back({c.level_min, i, j, k});
  sort_leaves(g->leaves);
  st = commit_tree(g);
  if (st != MR_OK) {
    free_grid(g);
    return st;
  }
  for (int f = 0; f < c.n_fields; ++f)
    launch_fill(g->f32, g->fields[f].p, g->leaves.size() * size_t(g->nb * g->nb * g->nb), g->stream);
  if (hipStreamSynchronize(g->stream) != hipSuccess) {
    free_grid(g);
    return fail(MR_EHIP, "stream synchronize failed");
  }
  *out = g;
  g_errmsg = warn;
  return MR_OK;
}

mr_status mr_grid_destroy(mr_grid* g) {
  if (!g) return fail(MR_EINVAL, "null grid");
  free_grid(g);
  return MR_OK;
}

mr_status mr_set_tree(mr_grid* g, int64_t n, const int32_t* level, const int32_t* ijk) {
  if (!g || n <= 0 || !level || !ijk) return fail(MR_EINVAL, "null or empty tree");
  if (n > g->cfg.max_blocks) return fail(MR_ECAPACITY, "tree exceeds max_blocks");
  std::vector<Key> nl(n);
  std::unordered_set<uint64_t> seen;
  int Lmax = 0;
  for (int64_t b = 0; b < n; ++b) {
    const int L = level[b];
    if (L < 0 || L > 12) return fail(MR_EINVAL, "level out of range");
    const int m = 1 << L;
    const int i = ijk[3 * b], j = ijk[3 * b + 1], k = ijk[3 * b + 2];
    if (i < 0 || j < 0 || k < 0 || i >= m || j >= m || k >= m) return fail(MR_EINVAL, "block index out of range");
    if (!seen.insert(pack(L, i, j, k)).second) return fail(MR_EINVAL, "duplicate leaf");
    nl[b] = {L, i, j, k};
    Lmax = std::max(Lmax, L);
  }
  // tiling: no leaf is an ancestor of another and the volumes add up
  long double vol = 0;
  for (const Key& k : nl) {
    vol += std::ldexp(1.0L, -3 * k.L);
    for (int l = k.L - 1; l >= 0; --l)
      if (seen.count(pack(l, k.i >> (k.L - l), k.j >> (k.L - l), k.k >> (k.L - l))))
        return fail(MR_EINVAL, "overlapping leaves");
  }
  if (std::fabs(double(vol - 1.0L)) > 1e-12) return fail(MR_EINVAL, "leaves do not tile the unit cube");
  std::vector<Key> saved = g->leaves;
  sort_leaves(nl);
  g->leaves = nl;
  mr_status st = commit_tree(g);
  if (st != MR_OK) {
    std::string msg = g_errmsg;
    g->leaves = saved;
    commit_tree(g);
    return fail(st, msg);
  }
  for (int f = 0; f < g->cfg.n_fields; ++f)
    launch_fill(g->f32, g->fields[f].p, g->leaves.size() * size_t(g->nb * g->nb * g->nb), g->stream);
  HIPCHK(hipStreamSynchronize(g->stream));
  return MR_OK;
}

mr_status mr_sample_ic(mr_grid* g, int32_t field, const mr_ic* ic) {
  if (!g || !ic || field < 0 || field >= g->cfg.n_fields) return fail(MR_EINVAL, "bad argument");
  if (ic->kind != MR_IC_GAUSS_SUM && ic->kind != MR_IC_TANH_SHELL) return fail(MR_EINVAL, "unknown IC kind");
  return upload_ic(g, field, ic);
}

mr_status mr_init_ic(mr_grid* g, int32_t field, const mr_ic* ic, int32_t max_iter, mr_adapt_stats* stats) {
  if (!g || !ic || field < 0 || field >= g->cfg.n_fields) return fail(MR_EINVAL, "bad argument");
  if (ic->kind != MR_IC_GAUSS_SUM && ic->kind != MR_IC_TANH_SHELL) return fail(MR_EINVAL, "unknown IC kind");
  if (max_iter <= 0) max_iter = 64;
  g->leaves.clear();
  const int n = 1 << g->cfg.level_min;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) g->leaves.push_back({g->cfg.level_min, i, j, k});
  sort_leaves(g->leaves);
  mr_status st = commit_tree(g);
  if (st != MR_OK) return st;
  st = upload_ic(g, field, ic);
  if (st != MR_OK) return st;
  for (int it = 0; it < max_iter; ++it) {
    std::vector<double> norms;
    st = norms_to_host(g, field, norms);
    if (st != MR_OK) return st;
    Plan plan;
    std::unordered_set<uint64_t> none;
    make_plan(g, norms, none, false, plan, nullptr);
    if (plan.refined == 0) break;
    int64_t nn = int64_t(g->leaves.size()) + 7 * int64_t(plan.refined);
    if (nn > g->cfg.max_blocks) return fail(MR_ECAPACITY, "initial grid exceeds max_blocks");
    st = apply_plan(g, plan, nullptr, true);
    if (st != MR_OK) return st;
    st = upload_ic(g, field, ic);
    if (st != MR_OK) return st;
  }
  return adapt_impl(g, field, 64, stats);
}

mr_status mr_ghost(mr_grid* g, int32_t field, int32_t depth) {
  if (!g || field < 0 || field >= g->cfg.n_fields) return fail(MR_EINVAL, "bad argument");
  if (depth == 0) depth = g->G;
  if (depth == g->G) ghost_fill(g, g->fields[field].p, g->stage);
  else if (depth == g->Dw) ghost_fill(g, g->fields[field].p, g->wide);
  else return fail(MR_EINVAL, "depth must be 0, the stencil depth or the wide depth " + std::to_string(g->Dw));
  return MR_OK;
}

mr_status mr_ghost_get(mr_grid* g, int32_t field, int32_t depth, int64_t b0, int64_t nblk, void* host,
                       size_t bytes) {
  if (!g || !host || field < 0 || field >= g->cfg.n_fields) return fail(MR_EINVAL, "bad argument");
  if (depth < 0 || depth > g->Dw) return fail(MR_EINVAL, "depth exceeds the patch depth");
  if (b0 < 0 || nblk < 0 || b0 + nblk > int64_t(g->leaves.size())) return fail(MR_EINVAL, "block range");
  const int64_t e = g->nb + 2 * depth;
  if (bytes != size_t(nblk * e * e * e) * g->esz) return fail(MR_EINVAL, "size mismatch");
  DevBuf tmp;
  HIPCHK(tmp.ensure(bytes));
  AnyView v = anyview(g, g->fields[field].p);
  launch_gather_ext(g->f32, v.raw, depth, b0, nblk, tmp.p, g->stream);
  HIPCHK(hipMemcpyAsync(host, tmp.p, bytes, hipMemcpyDeviceToHost, g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  tmp.release();
  return check_err(g);
}

mr_status mr_details(mr_grid* g, int32_t field, double* norms, int32_t on_device) {
  if (!g || (!norms && !on_device) || field < 0 || field >= g->cfg.n_fields)
    return fail(MR_EINVAL, "bad argument");
  ghost_fill(g, g->fields[field].p, g->wide);
  details_pass(g, g->fields[field].p, nullptr, nullptr);
  const size_t n = g->leaves.size();
  if (on_device) {
    if (norms && n)
      HIPCHK(hipMemcpyAsync(norms, g->d_norms.p, n * sizeof(double), hipMemcpyDeviceToDevice, g->stream));
    return MR_OK;
  }
  HIPCHK(hipMemcpyAsync(norms, g->d_norms.p, n * sizeof(double), hipMemcpyDeviceToHost, g->stream));
  mr_status st = check_err(g);
  if (st != MR_OK) return st;
  for (size_t b = 0; b < n; ++b)
    if (!std::isfinite(norms[b])) return fail(MR_ENONFINITE, "non-finite detail norm");
  return MR_OK;
}

mr_status mr_details_noalloc(mr_grid* g, int32_t field, double* dev_norms) {
  if (!g || !dev_norms || field < 0 || field >= g->cfg.n_fields)
    return fail(MR_EINVAL, "bad argument");
  const int64_t n = int64_t(g->leaves.size());
  if (n > static_band_blocks())
    return fail(MR_ECAPACITY, "mr_details_noalloc holds " + std::to_string(static_band_blocks()) +
                                  " blocks at most, the grid has " + std::to_string(n));
  double* bands = nullptr;
  HIPCHK(static_band_scratch(&bands));
  ghost_fill(g, g->fields[field].p, g->wide);
  details_pass(g, g->fields[field].p, nullptr, nullptr, nullptr, bands, dev_norms);
  return MR_OK;
}

mr_status mr_adapt(mr_grid* g, int32_t field, int32_t max_iter, mr_adapt_stats* stats) {
  if (!g || field < 0 || field >= g->cfg.n_fields) return fail(MR_EINVAL, "bad argument");
  if (max_iter <= 0) max_iter = 64;
  return adapt_impl(g, field, max_iter, stats);
}

mr_status mr_adapt_flags(mr_grid* g, const int8_t* flags, mr_adapt_stats* stats) {
  if (!g || !flags) return fail(MR_EINVAL, "bad argument");
  for (size_t b = 0; b < g->leaves.size(); ++b)
    if (flags[b] < -1 || flags[b] > 1) return fail(MR_EINVAL, "block status must be -1, 0 or 1");
  return adapt_impl(g, 0, 1, stats, flags);
}

mr_status mr_stage(mr_grid* g, int32_t y, int32_t un, int32_t out, double a_un, double b,
                   double c_y, double dt, const mr_velocity* vel) {
  VelDev vd;
  mr_status st = check_step_args(g, y, dt, vel, vd);
  if (st != MR_OK) return st;
  if (un < 0 || un >= g->cfg.n_fields || out < 0 || out >= g->cfg.n_fields || out == y)
    return fail(MR_EINVAL, "stage fields: un, out in range and out != y");
  if (!std::isfinite(a_un) || !std::isfinite(b) || !std::isfinite(c_y))
    return fail(MR_EINVAL, "non-finite stage coefficient");
  ghost_fill(g, g->fields[y].p, g->stage);
  rhs_stage(g, g->fields[y].p, g->fields[un].p, g->fields[out].p, a_un, b, dt, vd, nullptr, c_y);
  return MR_OK;
}

mr_status mr_set_tuning(mr_grid* g, const mr_tuning* t) {
  if (!g || !t) return fail(MR_EINVAL, "null argument");
  mr_tuning n = g->tune;
  const int32_t* in[3] = {&t->lds_refine, &t->lds_restrict, &t->lds_subst};
  int32_t* out[3] = {&n.lds_refine, &n.lds_restrict, &n.lds_subst};
  for (int k = 0; k < 3; ++k) {
    if (*in[k] == 0) continue;
    if (*in[k] < 4096 || *in[k] > 65536) return fail(MR_EINVAL, "LDS budget out of [4096, 65536]");
    *out[k] = *in[k];
  }
  if (t->subst_threads != 0) {
    if (t->subst_threads != 256 && t->subst_threads != 512)
      return fail(MR_EINVAL, "subst_threads must be 256 or 512");
    n.subst_threads = t->subst_threads;
  }
  g->tune = n;
  if (!g->leaves.empty()) {
    HIPCHK(hipStreamSynchronize(g->stream));
    return commit_tree(g);
  }
  return MR_OK;
}

mr_status mr_device_arch(char* out, size_t n) {
  if (!out || n == 0) return fail(MR_EINVAL, "null argument");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  std::string a(prop.gcnArchName);
  a = a.substr(0, a.find(':'));
  std::snprintf(out, n, "%s", a.c_str());
  return MR_OK;
}

mr_status mr_get_tuning(mr_grid* g, mr_tuning* t) {
  if (!g || !t) return fail(MR_EINVAL, "null argument");
  *t = g->tune;
  return MR_OK;
}

mr_status mr_set_thresholds(mr_grid* g, double eps_refine, double eps_coarsen) {
  if (!g) return fail(MR_EINVAL, "null grid");
  if (!(eps_refine > eps_coarsen) || !(eps_coarsen >= 0))
    return fail(MR_EINVAL, "need eps_refine > eps_coarsen >= 0");
  g->cfg.eps_refine = eps_refine;
  g->cfg.eps_coarsen = eps_coarsen;
  return MR_OK;
}

mr_status mr_rk3_step(mr_grid* g, int32_t field, double dt, const mr_velocity* vel) {
  VelDev vd;
  mr_status st = check_step_args(g, field, dt, vel, vd);
  if (st != MR_OK) return st;
  return run_step(g, g->rk3_graph, field, dt, vel, [&] { enqueue_rk3(g, field, dt, vd); });
}

mr_status mr_details_rk3_step(mr_grid* g, int32_t field, double dt, const mr_velocity* vel,
                              double* norms, int32_t on_device) {
  VelDev vd;
  mr_status st = check_step_args(g, field, dt, vel, vd);
  if (st != MR_OK) return st;
  if (!norms && !on_device) return fail(MR_EINVAL, "bad argument");
  // the second patch buffer is allocated outside any graph capture
  if (g->aux && !g->prof.on)
    HIPCHK(g->d_patch2.ensure(std::max<int64_t>(1, g->patch_elems) * g->esz));
  st = run_step(g, g->fused_graph, field, dt, vel, [&] { enqueue_fused(g, field, dt, vd); });
  if (st != MR_OK) return st;
  const size_t n = g->leaves.size();
  if (on_device) {
    if (norms && n)
      HIPCHK(hipMemcpyAsync(norms, g->d_norms.p, n * sizeof(double), hipMemcpyDeviceToDevice, g->stream));
    return MR_OK;
  }
  HIPCHK(hipMemcpyAsync(norms, g->d_norms.p, n * sizeof(double), hipMemcpyDeviceToHost, g->stream));
  st = check_err(g);
  if (st != MR_OK) return st;
  for (size_t b = 0; b < n; ++b)
    if (!std::isfinite(norms[b])) return fail(MR_ENONFINITE, "non-finite detail norm");
  return MR_OK;
}

mr_status mr_cfl_dt(const mr_grid* g, const mr_velocity* vel, double cfl, double* dt) {
  if (!g || !vel || !dt || !(cfl > 0)) return fail(MR_EINVAL, "bad argument");
  int Lf = 0;
  for (const Key& k : g->leaves) Lf = std::max(Lf, k.L);
  const double h = 1.0 / double(g->nb << Lf);
  if (vel->kind == MR_VEL_DIFFUSION) {
    if (!(vel->p[0] > 0)) return fail(MR_EINVAL, "diffusion dt needs nu > 0");
    *dt = cfl * h * h / (6.0 * vel->p[0]);   // explicit diffusion: h^2 / (2 d nu)
    return MR_OK;
  }
  *dt = cfl * h / usum(*vel);
  return MR_OK;
}

mr_status mr_block_meta(const mr_grid* g, int64_t n_cap, int64_t* n, int32_t* level, int32_t* ijk) {
  if (!g || !n) return fail(MR_EINVAL, "null argument");
  *n = int64_t(g->leaves.size());
  if (!level && !ijk) return MR_OK;
  if (n_cap < *n) return fail(MR_EINVAL, "n_cap smaller than the leaf count");
  for (size_t b = 0; b < g->leaves.size(); ++b) {
    if (level) level[b] = g->leaves[b].L;
    if (ijk) {
      ijk[3 * b] = g->leaves[b].i;
      ijk[3 * b + 1] = g->leaves[b].j;
      ijk[3 * b + 2] = g->leaves[b].k;
    }
  }
  return MR_OK;
}

mr_status mr_field_get(mr_grid* g, int32_t field, void* host, size_t bytes) {
  if (!g || !host || field < 0 || field >= g->cfg.n_fields) return fail(MR_EINVAL, "bad argument");
  const size_t want = g->leaves.size() * size_t(g->nb * g->nb * g->nb) * g->esz;
  if (bytes != want) return fail(MR_EINVAL, "size mismatch: expected " + std::to_string(want));
  HIPCHK(hipMemcpyAsync(host, g->fields[field].p, bytes, hipMemcpyDeviceToHost, g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  return MR_OK;
}

mr_status mr_field_set(mr_grid* g, int32_t field, const void* host, size_t bytes) {
  if (!g || !host || field < 0 || field >= g->cfg.n_fields) return fail(MR_EINVAL, "bad argument");
  const size_t want = g->leaves.size() * size_t(g->nb * g->nb * g->nb) * g->esz;
  if (bytes != want) return fail(MR_EINVAL, "size mismatch: expected " + std::to_string(want));
  HIPCHK(hipMemcpyAsync(g->fields[field].p, host, bytes, hipMemcpyHostToDevice, g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  return MR_OK;
}

mr_status mr_field_ptr(mr_grid* g, int32_t field, void** dev_ptr) {
  if (!g || !dev_ptr || field < 0 || field >= g->cfg.n_fields) return fail(MR_EINVAL, "bad argument");
  *dev_ptr = g->fields[field].p;
  return MR_OK;
}

// Neumaier's compensated sum of the per-block partials (column c of rows of
// width w): the result does not depend on the order the blocks ran in.
static double compensated_sum(const std::vector<double>& a, int w, int c) {
  double s = 0.0, comp = 0.0;
  for (size_t i = c; i < a.size(); i += w) {
    const double t = s + a[i];
    comp += std::fabs(s) >= std::fabs(a[i]) ? (s - t) + a[i] : (a[i] - t) + s;
    s = t;
  }
  return s + comp;
}

mr_status mr_moments(mr_grid* g, int32_t field, double out[4]) {
  if (!g || !out || field < 0 || field >= g->cfg.n_fields) return fail(MR_EINVAL, "bad argument");
  const int n = int(g->leaves.size());
  for (int k = 0; k < 4; ++k) out[k] = 0.0;
  if (n == 0) return MR_OK;
  HIPCHK(g->d_mom.ensure(4 * size_t(n) * sizeof(double)));
  AnyView v = anyview(g, g->fields[field].p);
  launch_moments(g->f32, v.raw, static_cast<double*>(g->d_mom.p), g->stream);
  std::vector<double> part(4 * size_t(n));
  HIPCHK(hipMemcpyAsync(part.data(), g->d_mom.p, part.size() * sizeof(double),
                        hipMemcpyDeviceToHost, g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  for (int k = 0; k < 4; ++k) out[k] = compensated_sum(part, 4, k);
  return MR_OK;
}

mr_status mr_ic_error(mr_grid* g, int32_t field, const mr_ic* ic, double out[2]) {
  if (!g || !ic || !out || field < 0 || field >= g->cfg.n_fields)
    return fail(MR_EINVAL, "bad argument");
  if (ic->kind != MR_IC_GAUSS_SUM && ic->kind != MR_IC_TANH_SHELL)
    return fail(MR_EINVAL, "unknown initial condition kind");
  const int np = ic->kind == MR_IC_GAUSS_SUM ? 5 * ic->n : 4;
  if (np <= 0 || !ic->params) return fail(MR_EINVAL, "initial condition without parameters");
  out[0] = out[1] = 0.0;
  const int n = int(g->leaves.size());
  if (n == 0) return MR_OK;
  HIPCHK(g->d_icpar.ensure(np * sizeof(double)));
  HIPCHK(hipMemcpyAsync(g->d_icpar.p, ic->params, np * sizeof(double), hipMemcpyHostToDevice,
                        g->stream));
  HIPCHK(g->d_mom.ensure(4 * size_t(n) * sizeof(double)));
  IcDev d{ic->kind, ic->n, static_cast<const double*>(g->d_icpar.p)};
  AnyView v = anyview(g, g->fields[field].p);
  launch_ic_error(g->f32, v.raw, d, static_cast<double*>(g->d_mom.p), g->stream);
  std::vector<double> part(2 * size_t(n));
  HIPCHK(hipMemcpyAsync(part.data(), g->d_mom.p, part.size() * sizeof(double),
                        hipMemcpyDeviceToHost, g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  for (int b = 0; b < n; ++b) out[0] = std::max(out[0], part[2 * size_t(b)]);
  out[1] = std::sqrt(compensated_sum(part, 2, 1));
  return MR_OK;
}

mr_status mr_prof_enable(mr_grid* g, int32_t on) {
  if (!g) return fail(MR_EINVAL, "null grid");
  (void)hipStreamSynchronize(g->stream);
  for (auto& r : g->prof.recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g->prof.recs.clear();
  g->prof.on = on != 0;
  g->htime = HostTimer{};
  return MR_OK;
}

mr_status mr_prof_read(mr_grid* g, const char* kernel, double* total_ms, int64_t* launches,
                       int64_t* points_per_launch) {
  if (!g || !kernel || !total_ms || !launches) return fail(MR_EINVAL, "null argument");
  int fam = -1;
  for (int f = 0; f < kNumFam; ++f)
    if (std::strcmp(kernel, kFam[f]) == 0) fam = f;
  for (int f = 0; f < 4; ++f)
    if (std::strcmp(kernel, kHostPhase[f]) == 0) {
      *total_ms = g->htime.ms[f];
      *launches = g->htime.n[f];
      if (points_per_launch) *points_per_launch = 0;
      return MR_OK;
    }
  if (fam < 0) return fail(MR_EINVAL, "unknown kernel family");
  HIPCHK(hipStreamSynchronize(g->stream));
  double ms = 0;
  int64_t cnt = 0;
  for (auto& r : g->prof.recs) {
    if (r.fam != fam) continue;
    float t = 0;
    HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
    ms += t;
    ++cnt;
  }
  *total_ms = ms;
  *launches = cnt;
  if (points_per_launch) *points_per_launch = g->prof.points[fam];
  return MR_OK;
}

mr_status mr_sync(mr_grid* g) {
  if (!g) return fail(MR_EINVAL, "null grid");
  HIPCHK(hipStreamSynchronize(g->stream));
  return check_err(g);
}

mr_status mr_tree_stats(const mr_grid* g, int64_t out[22]) {
  if (!g || !out) return fail(MR_EINVAL, "null argument");
  int lo = 99, hi = -1;
  for (const Key& k : g->leaves) {
    lo = std::min(lo, k.L);
    hi = std::max(hi, k.L);
  }
  out[0] = int64_t(g->leaves.size());
  out[1] = g->stage.out_points;
  out[2] = int64_t(g->stage.s.size());
  out[3] = hi;
  out[4] = lo;
  out[5] = int64_t(g->stage.g.size());
  out[6] = int64_t(g->stage.r.size());
  out[7] = g->stage.lds_g;
  out[8] = std::max(g->stage.lds_rc[0], std::max(g->stage.lds_rc[1], g->stage.lds_rc[2]));
  out[9] = g->patch_elems;
  out[10] = g->stage.cf_w;
  out[11] = g->stage.cf_r;
  out[12] = g->stage.sb_w;
  out[13] = g->stage.sb_r;
  out[14] = g->stage.fc_w;
  out[15] = g->stage.fc_r;
  out[16] = g->wide.cf_w;
  out[17] = g->wide.cf_r;
  out[18] = g->wide.sb_w;
  out[19] = g->wide.sb_r;
  out[20] = g->wide.fc_w;
  out[21] = g->wide.fc_r;
  return MR_OK;
}

}  // extern "C"
