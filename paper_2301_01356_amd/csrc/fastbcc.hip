// FAST-BCC on gfx950: phase kernels and the C ABI declared in fastbcc.h.
//
// Pipeline (paper: Algorithm 1 and Section "Algorithmic Details"; the
// GPU-specific readings are listed in the design notes):
//
//   First-CC   union-find over all arcs, the hooking edge of every hooked root
//              kept as a spanning-forest edge; a few sampling rounds first,
//              then the full sweep skips rows already in the largest set
//              (optionally after a low-diameter decomposition, whose BFS
//              edges are forest edges too).
//   Rooting    forest edges numbered densely, arcs 2e and 2e + 1 (twins by
//              a ^ 1); each vertex's out-arcs in a linked list built by
//              atomic exchange; Euler circuit by "arc u->v continues with the
//              arc after v->u in v's cyclic list" (paper: "Euler Tour
//              Technique"); all trees' tours plus one entry node per root of
//              a tree with edges are chained into ONE list, so list ranking
//              yields global positions directly; ruling-set list ranking
//              (rulers at every K-th node index, each walks to the next ruler)
//              and pointer jumping over the rulers.  Trees are rooted at hubs.
//   Tagging    down arcs (rank(u->v) < rank(v->u)) give parent and preorder
//              number first[v] = #entries before (scan of entry flags);
//              last[v] = first[v] + |T_v| - 1; w1/w2 = min/max of first over
//              v and its neighbours (one arc-balanced sweep, or sampled
//              neighbours with exact sweeps only under undecided vertices);
//              low/high by range min/max over the preorder interval (blocked
//              sparse table); fence bit per vertex.
//   Last-CC    union-find on the skeleton: plain tree edges linked per
//              vertex, non-tree arcs kept iff neither endpoint is an ancestor
//              of the other (cross edges); fence and back edges skipped.
//   Read-out   head(l[u]) = p(u) where l[u] != l[p(u)]; articulation points;
//              canonical label per BCC = its smallest arc (found in the row
//              of the BCC's smallest vertex); arc x->y lies in l[x] unless x
//              heads l[y]; with sorted rows those arcs are found from y's side
//              and every arc is written once with its final label.
//
// Every kernel is enqueued on the caller's stream; data-dependent sizes
// (number of trees, tree arcs, rulers) stay in device memory and grids are
// sized by upper bounds, so a solve needs no host synchronisation.

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "fastbcc.h"
#include "prims.hpp"

using namespace fastbcc;

struct fastbcc_trace {
  struct Pending {
    const char* name;
    hipEvent_t a, b;
  };
  struct Total {
    const char* name;
    double ms;
    int64_t launches;
  };
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<Pending> pending;
  std::vector<Total> totals;
  int64_t dropped = 0;
};

namespace {

constexpr int BLOCK = 256;
constexpr int MODE_SAMPLES = 1024;
constexpr int MIN_RULER_SHIFT = 3;
constexpr int MAX_RULER_SHIFT = 10;
constexpr int DEF_RULER_SHIFT = 5;
constexpr int LR2_SHIFT = 4;             // second ruling level: every 16th ruler
constexpr int LR2_MIN_RULERS = 1 << 16;  // below this, pointer jumping over all rulers
constexpr int DEF_SAMPLE_ROUNDS = 2;
constexpr int MIN_TILE_ARCS = 256;  // workspace is sized for this tile size
constexpr int DEF_TILE_SHIFT = 2;   // 4 windows of 64 arcs
constexpr int MAX_TILE_SHIFT = 6;
constexpr int ROWS_TILE_WINDOWS = 64;  // windows per wave in the row-wise label fill
constexpr int TAG_ROWS_GRID = 2048;    // blocks of the exact-tag pass over listed rows
constexpr int HUB_DEG = 4096;    // graph degree from which tree-degree counters are sharded
constexpr int HUB_SHARDS = 32;   // counters per hub (power of two, <= 32: 5 bits of a slot)

// scalar slots at the head of the workspace
enum Scalar : int {
  S_STATUS = 0,
  S_BIG_CC = 1,
  S_BIG_LAB = 2,
  S_LBIG = 3,       // final Last-CC root of the sampled largest skeleton component
  S_CANON_BIG = 4,  // canonical label of that component's BCC (-1 if it is no BCC)
  S_NODES = 8,      // list nodes of the Euler tour
  S_ENTRIES = 9,    // entry flags over the tour
  S_LDD_HUGE = 10,  // two slots: long rows listed by a decomposition round
  S_BIG_ROOT = 12,  // Last-CC root of the sampled largest set (priority hooking)
  S_BIG_MIN = 13,   // its smallest member
  S_HUBS = 14,      // hubs numbered so far
  S_DIRTY = 15,     // rows listed for exact tags
  S_GRAPH_NEXT = 16,  // next graph of a per-graph First-CC
  S_GRAPH_NEXT_LCC = 17,  // next graph of a per-graph Last-CC
  S_COUNT = 64,
};

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int ilog2_floor(int64_t x) {
  int l = 0;
  while ((int64_t(1) << (l + 1)) <= x) ++l;
  return l;
}

// ------------------------------------------------------------ workspace
struct Layout {
  size_t total = 0;
  size_t scalars, off32, cc, hook, toff, su, sv, tadj, twin, rootidx, roots, next, ol, ol2, rnext2, rlen2, rlen,
      rnext, rval0,
      rval1, rnx0, rnx1, pos, eflag, first, w1, w2, W, pre, suf, tab, rec, lab, head,
      rootlab, minid, canon, bsum, heads, foff, frank, frow, fstart, ftile, hubidx, shard, bigbits, dbits, tile_row, scan_tmp;
  int64_t nb = 0;      // rmq blocks of 64
  int levels = 0;      // sparse-table levels
  int64_t rmax = 0;    // ruler capacity
  int64_t rmax2 = 0;   // second-level ruler capacity
  int64_t tiles = 0;   // tile capacity
  int64_t scan_blocks = 0;
  int64_t hubs = 0;    // hub capacity (sharded tree-degree counters)
};

inline size_t take(size_t& cur, size_t bytes) {
  size_t at = cur;
  cur += (bytes + 255) & ~size_t(255);
  return at;
}

Layout make_layout(int64_t n, int64_t A) {
  Layout L;
  size_t c = 0;
  const int64_t n1 = n + 1, n2 = 2 * n + 1;
  L.nb = cdiv(n > 0 ? n : 1, 64);
  L.levels = ilog2_floor(L.nb) + 1;
  L.rmax = cdiv(n2, int64_t(1) << MIN_RULER_SHIFT) + 1;
  L.rmax2 = cdiv(L.rmax, int64_t(1) << LR2_SHIFT) + 1;
  L.tiles = cdiv(A > 0 ? A : 1, MIN_TILE_ARCS) + 1;
  L.scan_blocks = cdiv(n2, SCAN_TILE) + 1;
  const size_t I = sizeof(int);
  L.scalars = take(c, S_COUNT * I);
  L.off32 = take(c, n1 * I);
  L.cc = take(c, n * I);
  L.hook = take(c, n * sizeof(int2));  // First-CC's hooking edge per vertex (x < 0: none)
  L.toff = take(c, n1 * I);
  L.su = take(c, n * I);
  L.sv = take(c, n * I);
  L.tadj = take(c, n2 * I);
  L.twin = take(c, n2 * I);
  L.rootidx = take(c, n1 * I);
  L.roots = take(c, n * I);
  L.next = take(c, n2 * I);
  L.ol = take(c, n2 * 2 * I);
  L.rlen = take(c, L.rmax * I);
  L.rnext = take(c, L.rmax * I);
  L.rval0 = take(c, L.rmax * I);
  L.rval1 = take(c, L.rmax * I);
  L.rnx0 = take(c, L.rmax * I);
  L.rnx1 = take(c, L.rmax * I);
  L.ol2 = take(c, L.rmax * 2 * I);
  L.rnext2 = take(c, L.rmax2 * I);
  L.rlen2 = take(c, L.rmax2 * I);
  L.pos = take(c, n2 * I);
  L.eflag = take(c, n2 * I);
  L.first = take(c, n * I);
  L.w1 = take(c, n * I);
  L.w2 = take(c, n * I);
  L.W = take(c, n * 4 * I);
  L.pre = take(c, n * 2 * I);
  L.suf = take(c, n * 2 * I);
  L.tab = take(c, (size_t)L.levels * L.nb * 2 * I);
  L.rec = take(c, n * sizeof(int4));
  L.lab = take(c, n * I);
  L.head = take(c, n * I);
  L.rootlab = take(c, n * I);
  L.minid = take(c, n * I);
  L.canon = take(c, n * I);
  L.bsum = take(c, (cdiv(n > 0 ? n : 1, BLOCK) + 1) * I);
  L.heads = take(c, n);
  L.foff = take(c, n1 * I);
  L.frank = take(c, n1 * I);
  L.frow = take(c, n1 * I);
  L.fstart = take(c, n1 * I);
  L.ftile = take(c, L.tiles * I);
  L.hubs = (A / HUB_DEG) + 1;  // at most arcs / HUB_DEG vertices reach the hub degree
  L.hubidx = take(c, n1 * I);
  L.shard = take(c, (size_t)L.hubs * HUB_SHARDS * I);
  L.bigbits = take(c, (size_t)cdiv(n > 0 ? n : 1, 64) * 8);
  L.dbits = take(c, (size_t)cdiv(A > 0 ? A : 1, 64) * 8);
  L.tile_row = take(c, L.tiles * I);
  L.scan_tmp = take(c, L.scan_blocks * I);
  L.total = c;
  return L;
}

struct Tune {
  int ruler_shift = DEF_RULER_SHIFT;
  int sample_rounds = DEF_SAMPLE_ROUNDS;
  int tile_windows = 1 << DEF_TILE_SHIFT;
  bool cc_prio = false;  // First-CC hooks by hashed priority instead of by id
  int ldd = 0;           // First-CC starts with a low-diameter decomposition, beta = 2^-ldd (0 = off)
  bool sampled_tags = false;  // fences certified from sampled tags, exact tags only where needed
  int tag_samples = 4;        // sampled neighbours per vertex in that mode
  bool first_round_free = false;  // First-CC's first sampling round links without atomics
  bool lcc_prio = false;          // Last-CC hooks by hashed priority, then relabels to smallest members
  int lcc_rounds = -1;            // Last-CC sampling rounds (-1: as First-CC)
  int vertex_block = BLOCK;       // threads per block of the hot per-vertex kernels
  bool compress_free = false;     // flatten the sets after the atomic-free round too
  bool xcd = false;               // per-vertex launches in XCD-ordered shape
  bool graph_cc = false;          // batches: First-CC per graph, one workgroup each
};

bool decode_flags(uint32_t flags, Tune& t) {
  const uint32_t known = FASTBCC_FLAG_VALIDATE | FASTBCC_FLAG_SORTED_ROWS | FASTBCC_FLAG_NO_SELF_LOOPS |
                         (0xFu << FASTBCC_TUNE_RULER_SHIFT) |
                         (0x3u << FASTBCC_TUNE_SAMPLE_SHIFT) | (0x7u << FASTBCC_TUNE_TILE_SHIFT) |
                         FASTBCC_TUNE_CC_PRIORITY | (0x3u << FASTBCC_TUNE_LDD_SHIFT) |
                         FASTBCC_TUNE_SAMPLED_TAGS | (0x3u << FASTBCC_TUNE_TAG_SAMPLES_SHIFT) |
                         FASTBCC_TUNE_FREE_FIRST_ROUND | FASTBCC_TUNE_LCC_PRIORITY |
                         (0x3u << FASTBCC_TUNE_LCC_ROUNDS_SHIFT) | (0x3u << FASTBCC_TUNE_VERTEX_BLOCK_SHIFT) |
                         FASTBCC_TUNE_COMPRESS_FREE_ROUND | FASTBCC_TUNE_XCD_ORDER | FASTBCC_TUNE_GRAPH_CC;
  {
    const uint32_t lr = (flags >> FASTBCC_TUNE_LCC_ROUNDS_SHIFT) & 0x3;
    t.lcc_rounds = lr == 0 ? -1 : (int)lr - 1;
  }
  {
    static const int kBlock[4] = {BLOCK, 64, 128, 512};
    t.vertex_block = kBlock[(flags >> FASTBCC_TUNE_VERTEX_BLOCK_SHIFT) & 0x3];
  }
  t.first_round_free = (flags & FASTBCC_TUNE_FREE_FIRST_ROUND) != 0;
  t.compress_free = (flags & FASTBCC_TUNE_COMPRESS_FREE_ROUND) != 0;
  t.xcd = (flags & FASTBCC_TUNE_XCD_ORDER) != 0;
  t.graph_cc = (flags & FASTBCC_TUNE_GRAPH_CC) != 0;
  t.lcc_prio = (flags & FASTBCC_TUNE_LCC_PRIORITY) != 0;
  t.sampled_tags = (flags & FASTBCC_TUNE_SAMPLED_TAGS) != 0;
  static const int kSamples[4] = {4, 2, 3, 1};
  t.tag_samples = kSamples[(flags >> FASTBCC_TUNE_TAG_SAMPLES_SHIFT) & 0x3];
  t.cc_prio = (flags & FASTBCC_TUNE_CC_PRIORITY) != 0;
  t.ldd = (int)((flags >> FASTBCC_TUNE_LDD_SHIFT) & 0x3);
  if (flags & ~known) return false;
  uint32_t r = (flags >> FASTBCC_TUNE_RULER_SHIFT) & 0xF;
  uint32_t s = (flags >> FASTBCC_TUNE_SAMPLE_SHIFT) & 0x3;
  uint32_t w = (flags >> FASTBCC_TUNE_TILE_SHIFT) & 0x7;
  if (r) {
    if (r < MIN_RULER_SHIFT || r > MAX_RULER_SHIFT) return false;
    t.ruler_shift = (int)r;
  }
  if (s) t.sample_rounds = (s == 3) ? 0 : (int)s;
  if (w) {
    if (w < 2 || w > MAX_TILE_SHIFT) return false;
    t.tile_windows = 1 << w;
  }
  return true;
}

// ------------------------------------------------------------ XCD-ordered launches
// MI355X hands workgroup i of a launch to XCD i mod 8, and each XCD has its
// own L2.  A per-vertex launch of shape (8, per) puts the logical blocks
// k*per .. k*per + per - 1 (one contiguous run of vertices) on XCD k, so a
// kernel whose accesses stay near its own vertex (the graphs of a batch,
// lattices) keeps them in one L2.  The Euler tour's per-node and per-ruler
// launches take the same shape: its nodes are numbered graph by graph too.  The index below is the logical one for
// both shapes: a plain launch (blocks, 1) gives the usual numbering.
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int vertex_index() {
  return (int)(((int64_t)blockIdx.x * gridDim.y + blockIdx.y) * blockDim.x + threadIdx.x);
}

// ------------------------------------------------------------ small kernels
__global__ void k_fill_i32(int* p, int v, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_i64(int64_t* p, int64_t v, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// tile_row[t] = row holding arc t*tile_arcs (count from the device if given).
__global__ void k_tile_rows(const int* __restrict__ off, int n, int64_t A, const int* rows_dev, int64_t tile_arcs,
                            int* __restrict__ tile_row) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (rows_dev) {  // rows and arc count both on the device: off[rows] = arcs
    n = *rows_dev;
    A = off[n];
  }
  if (t * tile_arcs >= A) return;
  const int64_t a = t * tile_arcs;
  int lo = 0, hi = n;  // off[lo] <= a < off[hi]
  while (hi - lo > 1) {
    int mid = lo + (hi - lo) / 2;
    if ((int64_t)off[mid] <= a) lo = mid;
    else hi = mid;
  }
  tile_row[t] = lo;
}

// Frontier of a connectivity sweep: the rows outside the sampled largest set
// (their sampled arcs are visited again; re-linking joined ends costs two
// finds).  One scan over fdeg gives each frontier row both its rank (the
// count of non-zero degrees before it) and its first virtual arc (the sum of
// degrees before it), and its last pass writes the compacted rows (row id +
// start), so the virtual CSR has no empty rows for a wave to walk over.
// Frontier rows: those outside the sampled largest set.  Flattens the
// parent array on the way (every parent becomes its root), so the pass
// before it need not.
__global__ void k_frontier_deg(const int* __restrict__ off, int* comp, const int* __restrict__ scal, int slot, int n,
                               const uint8_t* __restrict__ mark, int* __restrict__ fdeg) {
  int v = vertex_index();
  if (v >= n) return;
  const int r = uf_find(comp, v);
  if (ld_relaxed(comp + v) != r) st_relaxed(comp + v, r);
  const int d = off[v + 1] - off[v];
  // skipped: the sampled largest set, or in a batch each graph's marked set
  const bool skip = mark ? mark[r] != 0 : r == scal[slot];
  const bool in = d > 0 && !skip;
  fdeg[v] = in ? d : 0;
}

// Per graph of a batch: the most frequent set among up to 256 evenly spaced
// vertices gets its root marked, and the frontier skips the rows of marked
// sets as it skips the largest set of a single graph.  No edge joins two
// graphs and each graph has one marked set, so every edge between a marked
// and another set is still seen from the other set's rows.
constexpr int GRAPH_MODE_SAMPLES = 256;
__global__ void __launch_bounds__(GRAPH_MODE_SAMPLES) k_mark_graph_modes(int* p, const int* __restrict__ vbegin,
                                                                         int n, uint8_t* __restrict__ mark) {
  __shared__ int s[GRAPH_MODE_SAMPLES];
  __shared__ int best_len[GRAPH_MODE_SAMPLES / WAVE];
  __shared__ int best_val[GRAPH_MODE_SAMPLES / WAVE];
  const int g = blockIdx.x, i = threadIdx.x;
  // clamped like the per-graph count: a graph range is never read past n
  const int v0 = min(max(vbegin[g], 0), n), ng = min(max(vbegin[g + 1], v0), n) - v0;
  if (ng <= 0) return;  // the whole block
  const int S = ng < GRAPH_MODE_SAMPLES ? ng : GRAPH_MODE_SAMPLES;
  s[i] = i < S ? uf_find(p, v0 + (int)((int64_t)i * ng / S)) : INT32_MAX;
  __syncthreads();
  for (int k = 2; k <= GRAPH_MODE_SAMPLES; k <<= 1) {  // bitonic sort, padding last
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int ix = i ^ j;
      if (ix > i) {
        const int a = s[i], b = s[ix];
        if ((a > b) == ((i & k) == 0)) {
          s[i] = b;
          s[ix] = a;
        }
      }
      __syncthreads();
    }
  }
  int len = 0, val = s[i];
  if (val != INT32_MAX && (i == 0 || s[i - 1] != val)) {
    int j = i;
    while (j < GRAPH_MODE_SAMPLES && s[j] == val) ++j;
    len = j - i;
  }
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const int l2 = __shfl_down(len, o, WAVE), v2 = __shfl_down(val, o, WAVE);
    if (l2 > len) {
      len = l2;
      val = v2;
    }
  }
  if (lane_id() == 0) {
    best_len[i / WAVE] = len;
    best_val[i / WAVE] = val;
  }
  __syncthreads();
  if (i == 0) {
    int bl = 0, bv = -1;
    for (int w = 0; w < GRAPH_MODE_SAMPLES / WAVE; ++w)
      if (best_len[w] > bl) {
        bl = best_len[w];
        bv = best_val[w];
      }
    if (bv >= 0) mark[bv] = 1;
  }
}

// Per scan tile of fdeg: the sum of degrees into bsum[tile] and the count of
// frontier rows into bsum[tiles + tile].
__global__ void __launch_bounds__(SCAN_BLOCK) k_fscan_reduce(const int* __restrict__ fdeg, int64_t n,
                                                              int* __restrict__ bsum, int tiles) {
  __shared__ int lds[SCAN_BLOCK / WAVE];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  load_items(fdeg, base, n, v);
  int s = 0, k = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    s += v[i];
    k += v[i] > 0;
  }
  int total;
  block_exclusive_scan(s, lds, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
  block_exclusive_scan(k, lds, total);
  if (threadIdx.x == 0) bsum[tiles + blockIdx.x] = total;
}

// The frontier rows in order, with their first arc in the virtual CSR, from
// the tiles' exclusive sums (bsum after the spine); fstart[rows] closes the
// last row with the frontier's arc count.
__global__ void __launch_bounds__(SCAN_BLOCK) k_fscan_compact(const int* __restrict__ fdeg, int64_t n,
                                                               const int* __restrict__ bsum, int tiles,
                                                               const int* __restrict__ rows, const int* __restrict__ arcs,
                                                               int* __restrict__ frow, int* __restrict__ fstart) {
  __shared__ int lds[SCAN_BLOCK / WAVE];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  load_items(fdeg, base, n, v);  // zero past n: no row there
  int s = 0, k = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    s += v[i];
    k += v[i] > 0;
  }
  int total;
  int start = block_exclusive_scan(s, lds, total) + bsum[blockIdx.x];
  int rank = block_exclusive_scan(k, lds, total) + bsum[tiles + blockIdx.x];
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    if (v[i] > 0) {
      frow[rank] = (int)(base + i);
      fstart[rank] = start;
      ++rank;
    }
    start += v[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) fstart[*rows] = *arcs;
}

// Tree roots: every component with a sampled vertex is rooted at its
// highest-degree sampled vertex, the others at their union-find root.  Any
// root is valid; a hub almost surely lies in its component's largest BCC, and
// a root inside the largest BCC keeps the subtrees below fence vertices small
// (what the sampled-tag certification needs).  Only the samples touch the
// per-component slots, so even the largest component sees few atomics.
constexpr int ROOT_SAMPLES = 65536;

__device__ __forceinline__ int root_sample(int i, int n) {
  return (int)(((int64_t)i * n) / ROOT_SAMPLES);
}

// Largest sampled degree per component.  Samples without edges are skipped
// (their trees have no tour).  Most samples fall in one component, whose
// counter would serialise one atomic per wave: each block first folds the
// samples of its first sampled component in LDS, then the rest reduce runs of
// equal components per wave.  Launched with ROOT_BLOCK threads per block.
constexpr int ROOT_BLOCK = 1024;
__global__ void __launch_bounds__(ROOT_BLOCK) k_root_degree(const int* __restrict__ off, const int* __restrict__ cc,
                                                          int n, int* rdeg) {
  __shared__ int first_t, key, kmax;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int c = -1, d = -1;
  if (i < ROOT_SAMPLES) {
    const int v = root_sample(i, n);
    if (i == 0 || v != root_sample(i - 1, n)) {  // n < ROOT_SAMPLES: each vertex once
      d = off[v + 1] - off[v];
      if (d > 0) c = cc[v];
    }
  }
  if (threadIdx.x == 0) {
    first_t = INT32_MAX;
    key = -1;
    kmax = -1;
  }
  __syncthreads();
  if (c >= 0) atomicMin(&first_t, (int)threadIdx.x);
  __syncthreads();
  if ((int)threadIdx.x == first_t) key = c;
  __syncthreads();
  if (c >= 0 && c == key) {
    atomicMax(&kmax, d);
    c = -1;
  }
  __syncthreads();
  if (threadIdx.x == 0 && key >= 0) atomicMax(rdeg + key, kmax);
  // the other components: runs of equal components within the wave, one atomic each
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int c2 = __shfl_up(c, o, WAVE), d2 = __shfl_up(d, o, WAVE);
    if (lane >= o && c2 == c && d2 > d) d = d2;
  }
  const int cn = __shfl_down(c, 1, WAVE);
  if (c >= 0 && (lane == WAVE - 1 || cn != c)) atomicMax(rdeg + c, d);
}

__global__ void k_root_select(const int* __restrict__ off, const int* __restrict__ cc, int n,
                              const int* __restrict__ rdeg, int* __restrict__ rsel) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int v = -1, c = -1;
  if (i < ROOT_SAMPLES) {
    v = root_sample(i, n);
    c = cc[v];
    if (off[v + 1] - off[v] != rdeg[c]) c = -1;  // not of largest degree
  }
  // any sampled vertex of largest degree: one store per run of equal components in the wave
  const int cn = __shfl_down(c, 1, WAVE);
  if (c >= 0 && (lane_id() == WAVE - 1 || cn != c)) rsel[c] = v;
}

// Most frequent value of p[] over a stratified sample of vertices (one
// block): the samples' roots are counted in an LDS hash table with twice as
// many slots as samples (linear probing always finds a slot), then the block
// takes the slot with the largest count.
constexpr int MODE_SLOTS = 2 * MODE_SAMPLES;
__global__ void __launch_bounds__(MODE_SAMPLES) k_pick_mode(int* p, int n, int* out) {
  __shared__ int key[MODE_SLOTS];
  __shared__ int cnt[MODE_SLOTS];
  __shared__ int best_len[MODE_SAMPLES / WAVE];
  __shared__ int best_val[MODE_SAMPLES / WAVE];
  const int i = threadIdx.x;
  for (int k = i; k < MODE_SLOTS; k += MODE_SAMPLES) {
    key[k] = -1;
    cnt[k] = 0;
  }
  int64_t stride = n / MODE_SAMPLES;
  if (stride < 1) stride = 1;
  // jitter inside each stride: Knuth's multiplicative hash (2654435761 =
  // 2^32 / golden ratio) of the sample index, then a multiply / xor-shift mix
  uint32_t h = (uint32_t)i * 2654435761u + 0x9e3779b9u;
  h ^= h >> 15;
  h *= 0x2c1b3c6du;
  h ^= h >> 12;
  const int64_t v = ((int64_t)i * stride + (int64_t)(h % (uint32_t)stride)) % n;
  const int r = uf_find(p, (int)v);  // the sets need not be flattened yet
  __syncthreads();
  uint32_t slot = ((uint32_t)r * 2654435761u) % (uint32_t)MODE_SLOTS;
  for (;;) {
    const int k = atomicCAS(&key[slot], -1, r);
    if (k == -1 || k == r) {
      atomicAdd(&cnt[slot], 1);
      break;
    }
    slot = slot + 1 == (uint32_t)MODE_SLOTS ? 0 : slot + 1;
  }
  __syncthreads();
  int len = -1, val = 0;
  for (int k = i; k < MODE_SLOTS; k += MODE_SAMPLES)
    if (cnt[k] > len) {
      len = cnt[k];
      val = key[k];
    }
  // block argmax of (len, val)
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    int l2 = __shfl_down(len, o, WAVE), v2 = __shfl_down(val, o, WAVE);
    if (l2 > len) {
      len = l2;
      val = v2;
    }
  }
  if (lane_id() == 0) {
    best_len[i / WAVE] = len;
    best_val[i / WAVE] = val;
  }
  __syncthreads();
  if (i == 0) {
    int bl = -1, bv = 0;
    for (int w = 0; w < MODE_SAMPLES / WAVE; ++w)
      if (best_len[w] > bl) {
        bl = best_len[w];
        bv = best_val[w];
      }
    out[0] = bv;
  }
}

__global__ void k_compress(int* p, int n) {
  int v = vertex_index();
  if (v >= n) return;
  int r = uf_find(p, v);
  if (ld_relaxed(p + v) != r) st_relaxed(p + v, r);
}

// Every entry onto its root, guaranteed: reads only, writes its own entry.
// Run after a path-halving pass, whose concurrent writes can leave a few
// entries on an ancestor below the root (those walks are then short); the
// passes that read p[v] as the set's id (Rooting's component ids, the
// read-out's labels, the relabelling) need every entry on its root.
__global__ void k_flatten(int* p, int n) {
  int v = vertex_index();
  if (v >= n) return;
  const int r = uf_root_ro(p, v);
  if (ld_relaxed(p + v) != r) st_relaxed(p + v, r);
}

// ------------------------------------------------------------ validation
// Graph g of a batch owns vertices [vbegin[g], vbegin[g+1]) (vbegin already
// checked to be nondecreasing from 0 to n).
__device__ __forceinline__ int graph_index(const int* __restrict__ vbegin, int G, int v) {
  int lo = 0, hi = G;  // vbegin[lo] <= v < vbegin[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (vbegin[mid] <= v) lo = mid;
    else hi = mid;
  }
  return lo;
}

// The graph ranges of a batch: vbegin[0] = 0, vbegin[G] = n, nondecreasing.
__global__ void k_validate_vbegin(const int* __restrict__ vbegin, int G, int n, int* status) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g > G) return;
  bool bad = false;
  if (g == 0 && vbegin[0] != 0) bad = true;
  if (g == G && vbegin[G] != n) bad = true;
  if (g < G && vbegin[g] > vbegin[g + 1]) bad = true;
  if (bad) atomicExch(status, (int)FASTBCC_ERR_INVALID_GRAPH);
}

template <typename OffT>
__global__ void k_validate_rows(const OffT* __restrict__ off, int n, int64_t A, int* status) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v > n) return;
  bool bad = false;
  if (v == 0 && off[0] != 0) bad = true;
  if (v == n && (int64_t)off[n] != A) bad = true;
  if (v < n && off[v] > off[v + 1]) bad = true;
  if (bad) atomicExch(status, (int)FASTBCC_ERR_INVALID_GRAPH);
}

__global__ void k_validate_arcs(const int* __restrict__ off, const int* __restrict__ adj, int n, int64_t A,
                                const int* __restrict__ tile_row, int tw, bool no_loops, const int* __restrict__ vbegin,
                                int G, int* status) {
  arc_tiles(off, n, A, tile_row, tw, [&](int64_t a, int x, bool ok) {
    if (!ok) return;
    const int y = adj[a];
    bool bad = (y < 0 || y >= n) || (no_loops && y == x);
    // in a batch every arc stays inside its own graph
    if (!bad && G > 1 && graph_index(vbegin, G, y) != graph_index(vbegin, G, x)) bad = true;
    if (!bad && a > (int64_t)off[x] && adj[a - 1] > y) bad = true;  // rows sorted
    if (!bad) {
      // x must occur in row y (binary search; rows sorted)
      int64_t lo = off[y], hi = off[y + 1];
      while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (adj[mid] < x) lo = mid + 1;
        else hi = mid;
      }
      if (lo >= (int64_t)off[y + 1] || adj[lo] != x) bad = true;
    }
    if (bad) atomicExch(status, (int)FASTBCC_ERR_INVALID_GRAPH);
  });
}

// ------------------------------------------------------------ First-CC
__global__ void k_cc_init(int* __restrict__ cc, int2* __restrict__ hook, int n) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  cc[v] = v;
  hook[v] = make_int2(-1, -1);
}

// Position of the neighbour a vertex samples in round r: a hash of (v, r)
// over its row, so sampled links do not all point to each row's smallest id
// (sorted rows would otherwise build long union-find chains).  The hash is
// an ad-hoc multiply / xor-shift mix (golden-ratio multiplier for v); the
// results never depend on which neighbour is sampled, only the speed does.
__device__ __forceinline__ int64_t sample_pos(int v, int r, int64_t deg) {
  uint32_t h = (uint32_t)v * 0x9E3779B1u ^ (uint32_t)(r + 1) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  return (int64_t)(h % (uint32_t)deg);
}

template <bool PRIO>
__device__ __forceinline__ void cc_link(int* cc, int u, int v, int2* hook) {
  if (PRIO) uf_link_record_prio(cc, u, v, hook);
  else uf_link_record(cc, u, v, hook);
}

// Sampling round r: every vertex links to one hashed neighbour.
template <bool PRIO>
__global__ void k_cc_sample(const int* __restrict__ off, const int* __restrict__ adj, int n, int r, int* cc,
                            int2* hook) {
  int v = vertex_index();
  if (v >= n) return;
  const int64_t b = off[v], e = off[v + 1];
  if (e > b) {
    int w = adj[b + sample_pos(v, r, e - b)];
    if (w != v) cc_link<PRIO>(cc, v, w, hook);
  }
}

// First sampling round from all-singleton sets, without atomics: v points to
// the higher-ranked of two sampled neighbours when it ranks above v (smaller
// id, or higher hashed priority), which keeps the pointers acyclic; the edge
// is recorded at v as a hooked root's edge would be.  About three quarters
// of the vertices link; the next rounds link the rest with the full
// union-find.
template <bool PRIO>
__device__ __forceinline__ bool ranks_above(int w, int v) {
  return PRIO ? uf_prio(w) > uf_prio(v) : w < v;
}

template <bool PRIO>
__global__ void k_cc_first_round(const int* __restrict__ off, const int* __restrict__ adj, int n, int* cc,
                                 int2* __restrict__ hook) {
  int v = vertex_index();
  if (v >= n) return;
  const int64_t b = off[v], e = off[v + 1];
  int w = v;
  if (e > b) {
    const int w1 = adj[b + sample_pos(v, 0, e - b)];
    const int w2 = adj[b + sample_pos(v, 16, e - b)];
    w = ranks_above<PRIO>(w2, w1) ? w2 : w1;
    if (!ranks_above<PRIO>(w, v)) w = v;
  }
  // this pass also initialises every set (cc[v] = v, no hook edge)
  cc[v] = w;
  hook[v] = make_int2(w == v ? -1 : v, w);
}

// Full sweep over the frontier: rows whose set is the sampled largest one
// are skipped (every edge they share with another set is seen from that
// set's side, and a row found in the largest set stays connected to it).
template <bool PRIO>
__global__ void k_cc_sweep(const int* __restrict__ off, const int* __restrict__ frow, const int* __restrict__ fstart,
                           const int* __restrict__ adj, const int* __restrict__ frows, const int* __restrict__ ftile,
                           int tw, int* cc, int2* hook) {
  const int R = *frows;
  const int64_t F = fstart[R];
  arc_tiles(fstart, R, F, ftile, tw, [&](int64_t k, int i, bool ok) {
    if (!ok) return;
    const int x = frow[i];
    const int64_t a = (int64_t)off[x] + (k - (int64_t)fstart[i]);
    const int w = adj[a];
    if (w != x) cc_link<PRIO>(cc, x, w, hook);
  });
}

// ------------------------------------------------- low-diameter decomposition
// Optional First-CC front end (paper: connectivity by LDD-UF-JTB, Section
// "Implementation Details" and the appendix on its cost): a Miller-Peng-Xu
// decomposition grows BFS clusters from centres that wake up at exponentially
// distributed times, then union-find joins the clusters over the remaining
// edges (the sampling rounds and the frontier sweep that follow).  Vertex v
// draws a shift d_v ~ Exp(beta) and wakes in round T0 - floor(d_v) (clamped
// to [0, T0], T0 = ceil(ln n / beta)) unless a cluster reached it first; every
// vertex is claimed by round T0.  The local-search analog: a lane that claims
// a vertex of small degree expands it at once, so clusters grow two hops per
// round through sparse regions.  A claimed vertex records its BFS edge the way
// a hooked root records its union-find edge, so the recorded edges still form
// a spanning forest.
constexpr int LDD_SMALL = 32;    // rows up to this degree are expanded by one lane
constexpr int LDD_HUGE = 2048;   // longer rows are queued in chunks for the whole grid
constexpr int LDD_CHUNK = 1024;  // arcs per queued chunk (<= LDD_HUGE)
constexpr int LDD_HUGE_GRID = 1024;

// ------------------------------------------------------------ per-graph First-CC (batches)
// With FASTBCC_TUNE_GRAPH_CC a batch's First-CC runs per graph instead of
// over the whole union (a BCC never spans two graphs, and neither does a
// component): one workgroup at a time takes the next graph from a counter
// the solve zeroed, runs union-find over its arcs -- each edge once, from its
// smaller endpoint; the larger root goes under the smaller; the hooking edge
// is kept at the hooked root, as uf_link_record keeps it -- and leaves cc[v]
// on the graph's root.  The parents of a graph of at most 2^16 vertices live
// in LDS as 16-bit local ids, two to a word: a hook is a 32-bit CAS on the
// word, so a path-halving store into the other half makes it retry and never
// loses an update.  A larger graph runs the same loop on the device-memory
// union-find.
// Two sampling rounds (an atomic-free one over two hashed neighbours, then a
// union-find one over a third) hook most vertices of a connected graph into
// one set; the sweep then gives thread t the rows t, t + 1024, ..., tests
// each row's set in LDS and reads only the rows outside the sampled largest
// set, their arcs spread over the wave's lanes.
constexpr int GCC_THREADS = 1024;
constexpr int GCC_LDS_VERTICES = 1 << 16;
constexpr int GCC_SB = 4;  // vertices per thread with their loads in flight together in the row pass
constexpr int GCC_GRID = 1024;  // workgroups of the launch (more than one per compute unit waits)

__device__ __forceinline__ int p16_get(const uint32_t* P, int x) {
  const uint32_t w = __hip_atomic_load(P + (x >> 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  return (int)((x & 1) ? (w >> 16) : (w & 0xFFFFu));
}
__device__ __forceinline__ void p16_set(uint32_t* P, int x, int val) {
  reinterpret_cast<volatile uint16_t*>(P)[x] = (uint16_t)val;
}
__device__ __forceinline__ bool p16_cas(uint32_t* P, int x, int expect, int val) {
  uint32_t* w = P + (x >> 1);
  const int sh = (x & 1) * 16;
  uint32_t old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  for (;;) {
    if (((old >> sh) & 0xFFFFu) != (uint32_t)expect) return false;
    const uint32_t nw = (old & ~(0xFFFFu << sh)) | ((uint32_t)val << sh);
    const uint32_t prev = atomicCAS(w, old, nw);
    if (prev == old) return true;
    old = prev;  // the word changed (either half): test again
  }
}
// Parents only point to smaller local ids, so both walks end.
__device__ __forceinline__ int p16_find(uint32_t* P, int x) {
  int px = p16_get(P, x);
  while (px != x) {
    const int gx = p16_get(P, px);
    if (gx == px) return px;
    p16_set(P, x, gx);  // path halving: an ancestor of x
    x = gx;
    px = p16_get(P, x);
  }
  return x;
}
__device__ __forceinline__ int p16_root(const uint32_t* P, int x) {
  int px = p16_get(P, x);
  while (px != x) {
    x = px;
    px = p16_get(P, x);
  }
  return x;
}

// The per-graph passes take the graphs largest first: a workgroup that takes
// a big graph near the end keeps running while the rest of the GPU idles
// (claimed in index order, a mixed batch of 4096 graphs of 64-65536 vertices
// would end about 1.6x after its mean load per compute unit; largest first,
// within 1.1x).  One workgroup sorts the graphs into size classes by their
// work (arcs plus twice the vertices; two classes per power of two): it
// counts the classes, scans them from the largest down and scatters each
// graph's index into its class's range.  The order within a class is
// whatever the LDS atomics give; no result depends on which workgroup solves
// which graph, or when.
constexpr int GORDER_CLASSES = 128;
constexpr int GORDER_THREADS = 1024;

__device__ __forceinline__ int graph_size_class(const int* __restrict__ vbegin, int n, const int* __restrict__ off,
                                                int g) {
  const int v0 = min(max(vbegin[g], 0), n), v1 = min(max(vbegin[g + 1], v0), n);
  const int64_t work = (int64_t)max(off[v1] - off[v0], 0) + 2 * (int64_t)(v1 - v0);
  if (work == 0) return GORDER_CLASSES - 1;
  const int bl = 64 - __clzll((unsigned long long)work);  // 1..34: arcs and vertices are below 2^31
  const int half = bl >= 2 ? (int)((work >> (bl - 2)) & 1) : 0;
  return GORDER_CLASSES - 1 - (2 * bl + half);  // larger work, smaller class (>= 58)
}

__global__ void __launch_bounds__(GORDER_THREADS) k_graph_order(const int* __restrict__ vbegin, int G, int n,
                                                                const int* __restrict__ off, int* __restrict__ order) {
  __shared__ int cls[GORDER_CLASSES];
  const int tid = threadIdx.x;
  for (int i = tid; i < GORDER_CLASSES; i += GORDER_THREADS) cls[i] = 0;
  __syncthreads();
  for (int g = tid; g < G; g += GORDER_THREADS) atomicAdd(&cls[graph_size_class(vbegin, n, off, g)], 1);
  __syncthreads();
  if (tid == 0) {
    int s = 0;
    for (int i = 0; i < GORDER_CLASSES; ++i) {
      const int k = cls[i];
      cls[i] = s;
      s += k;
    }
  }
  __syncthreads();
  for (int g = tid; g < G; g += GORDER_THREADS) order[atomicAdd(&cls[graph_size_class(vbegin, n, off, g)], 1)] = g;
}

// The sweep's arcs spread over a wave: each lane holds at most one row to
// read, [rb, re) (empty if none); the wave walks the concatenation of its
// lanes' rows 64 arcs at a time, each lane finding the row of its arc by a
// binary search over the wave's prefix sums of the row lengths (kept rows are
// few and short, so one row per lane would leave most lanes idle).
// body(owner lane, arc or -1) runs on all 64 lanes together, so it may shuffle.
template <typename Body>
__device__ __forceinline__ void wave_row_arcs(int rb, int re, Body&& body) {
  const int lane = lane_id(), d = re - rb;
  int incl = d;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int t = __shfl_up(incl, o, WAVE);
    if (lane >= o) incl += t;
  }
  const int excl = incl - d, total = __shfl(incl, WAVE - 1, WAVE);
  for (int c = 0; c < total; c += WAVE) {
    const int k = c + lane;
    int lo = 0;  // the last lane whose rows start at or before arc k: its row holds k
#pragma unroll
    for (int step = WAVE / 2; step > 0; step >>= 1)
      if (__shfl(excl, lo + step, WAVE) <= k) lo += step;
    const int a = __shfl(rb, lo, WAVE) + (k - __shfl(excl, lo, WAVE));
    body(lo, k < total ? a : -1);
  }
}

// The next graph of a per-graph pass: the i-th claim takes order[i] (index
// order without an order).
__device__ __forceinline__ int claim_graph(int* next_graph, const int* __restrict__ order, int G) {
  const int i = atomicAdd(next_graph, 1);
  return (order != nullptr && i < G) ? order[i] : i;
}

__global__ void __launch_bounds__(GCC_THREADS) k_graph_cc(const int* __restrict__ vbegin, int G, int n,
                                                          const int* __restrict__ off, const int* __restrict__ adj,
                                                          int* cc, int2* hook, int* next_graph,
                                                          const int* __restrict__ order) {
  __shared__ uint32_t P[GCC_LDS_VERTICES / 2];
  __shared__ int g_s, big_s;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) g_s = claim_graph(next_graph, order, G);
    __syncthreads();
    const int g = g_s;
    __syncthreads();  // everyone has read g_s before it is rewritten
    if (g >= G) break;
    const int v0 = min(max(vbegin[g], 0), n), v1 = min(max(vbegin[g + 1], v0), n), ng = v1 - v0;
    if (ng == 0) continue;
    const bool in_lds = ng <= GCC_LDS_VERTICES;
    const int a0 = off[v0], A = max(off[v1] - a0, 0);
    // Every set starts here.  With parents in LDS this is also the first
    // sampling round, without atomics: v points to the smaller of two sampled
    // neighbours when that id is below v's (pointers to smaller ids are
    // acyclic and keep each set's root its smallest member, as min-id hooking
    // does), and the edge is kept at v as a hooked root's would be -- one
    // coalesced store per vertex.  GCC_SB vertices per thread with their
    // loads in flight together.
    for (int base = 0; base < ng; base += GCC_THREADS * GCC_SB) {
      int w[GCC_SB];
      {
        int rb[GCC_SB], re[GCC_SB];
#pragma unroll
        for (int j = 0; j < GCC_SB; ++j) {
          const int v = base + j * GCC_THREADS + tid;
          rb[j] = re[j] = 0;
          if (in_lds && v < ng) {
            rb[j] = min(max(off[v0 + v] - a0, 0), A);
            re[j] = min(max(off[v0 + v + 1] - a0, rb[j]), A);
          }
        }
        int w2[GCC_SB];
#pragma unroll
        for (int j = 0; j < GCC_SB; ++j) {
          const int v = base + j * GCC_THREADS + tid, d = re[j] - rb[j];
          w[j] = d > 0 ? adj[a0 + rb[j] + (int)sample_pos(v0 + v, 0, d)] - v0 : v;
          w2[j] = d > 0 ? adj[a0 + rb[j] + (int)sample_pos(v0 + v, 16, d)] - v0 : v;
        }
#pragma unroll
        for (int j = 0; j < GCC_SB; ++j) {
          const int v = base + j * GCC_THREADS + tid;
          const int c1 = w[j] >= 0 && w[j] < v ? w[j] : v, c2 = w2[j] >= 0 && w2[j] < v ? w2[j] : v;
          w[j] = c1 < c2 ? c1 : c2;  // v unless a sampled neighbour of the graph has a smaller id
        }
      }
#pragma unroll
      for (int j = 0; j < GCC_SB; ++j) {
        const int v = base + j * GCC_THREADS + tid;
        if (v >= ng) continue;
        hook[v0 + v] = w[j] == v ? make_int2(-1, -1) : make_int2(v0 + v, v0 + w[j]);
        if (in_lds) p16_set(P, v, w[j]);
        else cc[v0 + v] = v0 + v;
      }
    }
    __syncthreads();
    // hook the sets of local x and y, keeping the hooking edge
    auto link16 = [&](int x, int y) {
      if (p16_get(P, x) == p16_get(P, y)) return;  // same parent: same set
      int ru = p16_find(P, x), rv = p16_find(P, y);
      while (ru != rv) {
        const int h = ru > rv ? ru : rv, l = ru > rv ? rv : ru;
        if (p16_cas(P, h, h, l)) {
          hook[v0 + h] = make_int2(v0 + x, v0 + y);
          return;
        }
        ru = p16_find(P, ru);
        rv = p16_find(P, rv);
      }
    };
    // The second sampling round (parents in LDS): each vertex links to one
    // more hashed neighbour by union-find.
    for (int base = 0; in_lds && base < ng; base += GCC_THREADS * GCC_SB) {
      int ys[GCC_SB];
      {
        int rb[GCC_SB], re[GCC_SB];
#pragma unroll
        for (int j = 0; j < GCC_SB; ++j) {
          const int v = base + j * GCC_THREADS + tid;
          rb[j] = re[j] = 0;
          if (v < ng) {
            rb[j] = min(max(off[v0 + v] - a0, 0), A);
            re[j] = min(max(off[v0 + v + 1] - a0, rb[j]), A);
          }
        }
#pragma unroll
        for (int j = 0; j < GCC_SB; ++j) {
          const int v = base + j * GCC_THREADS + tid, d = re[j] - rb[j];
          ys[j] = d > 0 ? adj[a0 + rb[j] + (int)sample_pos(v0 + v, 1, d)] - v0 : -1;
        }
      }
#pragma unroll
      for (int j = 0; j < GCC_SB; ++j) {
        const int v = base + j * GCC_THREADS + tid, y = ys[j];
        if (y != v && y >= 0 && y < ng) link16(v, y);  // -1 unless sampled
      }
    }
    __syncthreads();
    int big = -1;  // sets rooted with big (sampled largest set) skip their rows below
    if (in_lds) {
      // the set most of 64 evenly spread vertices fall in
      if (tid < WAVE) {
        const int r = p16_root(P, (int)((int64_t)tid * ng / WAVE));
        int cnt = 0;
        for (int j = 0; j < WAVE; ++j) cnt += __shfl(r, j, WAVE) == r ? 1 : 0;
        int best_c = cnt, best_r = r;
        for (int o = WAVE / 2; o > 0; o >>= 1) {
          const int oc = __shfl_xor(best_c, o, WAVE), orr = __shfl_xor(best_r, o, WAVE);
          if (oc > best_c || (oc == best_c && orr < best_r)) {
            best_c = oc;
            best_r = orr;
          }
        }
        if (tid == 0) big_s = best_r;
      }
      __syncthreads();
      big = big_s;
    }
    // the sweep: every arc of every row outside the big set (an edge between
    // two rows that are both skipped lies inside the big set already); rows
    // are tested in LDS, so the skipped ones (most, once sampling found the
    // big set) cost no global load
    for (int xb = 0; xb < ng; xb += GCC_THREADS) {  // the same trip count on every wave
      const int xo = xb + tid;
      int rb = 0, re = 0;
      if (xo < ng && !(in_lds && p16_find(P, xo) == p16_find(P, big))) {
        rb = min(max(off[v0 + xo] - a0, 0), A);
        re = min(max(off[v0 + xo + 1] - a0, rb), A);
      }
      wave_row_arcs(rb, re, [&](int owner, int a) {
        const int x = __shfl(xo, owner, WAVE);
        if (a < 0) return;
        const int y = adj[a0 + a] - v0;
        if (y == x || y < 0 || y >= ng) return;  // self-loops and foreign ids skipped
        if (in_lds) link16(x, y);
        else if (y > x) uf_link_record(cc, v0 + x, v0 + y, hook);  // each edge once
      });
    }
    __syncthreads();
    if (in_lds)
      for (int v = tid; v < ng; v += GCC_THREADS) cc[v0 + v] = v0 + p16_root(P, v);
    __syncthreads();  // the next graph reuses P
  }
}

// Start round from a splitmix64 hash of the vertex id (Steele, Lea and Flood,
// "Fast splittable pseudorandom number generators").
__device__ __forceinline__ int ldd_start(int v, int T0, float inv_beta) {
  uint64_t z = (uint64_t)(uint32_t)v * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const float u = (float)((z >> 40) + 1) * (1.0f / 16777216.0f);  // (0, 1]
  const int d = (int)(-logf(u) * inv_beta);
  const int s = T0 - d;
  return s < 0 ? 0 : s;
}

__global__ void k_ldd_init(int* __restrict__ cc, int2* __restrict__ hook, int* __restrict__ rnd, int n, int* scal) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v == 0) scal[S_LDD_HUGE] = scal[S_LDD_HUGE + 1] = 0;
  if (v >= n) return;
  cc[v] = -1;
  hook[v] = make_int2(-1, -1);
  rnd[v] = -1;
}

__device__ __forceinline__ bool ldd_claim(int* cc, int* rnd, int2* hook, int u, int cu, int w, int r) {
  if (ld_relaxed(cc + w) != -1 || atomicCAS(cc + w, -1, cu) != -1) return false;
  hook[w] = make_int2(u, w);
  rnd[w] = r + 1;  // expands next round (unless expanded at once)
  return true;
}

// Round r: wake the centres due now, then every vertex of round r claims its
// unclaimed neighbours.  Rows longer than LDD_SMALL are expanded by the whole
// wave, 64 arcs at a time; rows longer than LDD_HUGE are queued as chunks of
// LDD_CHUNK arcs, (row, first arc) each, for k_ldd_huge.  The queue length
// alternates between two slots, so this round can clear the slot of the round
// before while appending to its own.  Queue capacity: a row of d > LDD_HUGE
// arcs takes ceil(d / LDD_CHUNK) < 2d / LDD_CHUNK entries, so all rows together
// need fewer than 2A / LDD_CHUNK.
__global__ void k_ldd_round(const int* __restrict__ off, const int* __restrict__ adj, int n, int r, int T0,
                            float inv_beta, int* cc, int* rnd, int2* __restrict__ hook,
                            int2* __restrict__ queue, int* scal) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v == 0) scal[S_LDD_HUGE + ((r + 1) & 1)] = 0;
  bool active = false;
  int b = 0, e = 0, cv = -1;
  if (v < n) {
    if (ld_relaxed(cc + v) == -1 && ldd_start(v, T0, inv_beta) <= r && atomicCAS(cc + v, -1, v) == -1) rnd[v] = r;
    if (ld_relaxed(rnd + v) == r) {
      active = true;
      b = off[v];
      e = off[v + 1];
      cv = ld_relaxed(cc + v);
    }
  }
  if (active && e - b > LDD_HUGE) {
    const int chunks = (e - b + LDD_CHUNK - 1) / LDD_CHUNK;
    const int at = atomicAdd(scal + S_LDD_HUGE + (r & 1), chunks);
    for (int k = 0; k < chunks; ++k) queue[at + k] = make_int2(v, b + k * LDD_CHUNK);
    active = false;
  }
  if (active && e - b <= LDD_SMALL) {
    for (int a = b; a < e; ++a) {
      const int w = adj[a];
      if (w == v || !ldd_claim(cc, rnd, hook, v, cv, w, r)) continue;
      const int wb = off[w], we = off[w + 1];
      if (we - wb > LDD_SMALL) continue;
      rnd[w] = -2;  // expanded here
      for (int k = wb; k < we; ++k) {
        const int x = adj[k];
        if (x != w) ldd_claim(cc, rnd, hook, w, cv, x, r);
      }
    }
  }
  uint64_t big = __ballot(active && e - b > LDD_SMALL);
  while (big) {
    const int j = __builtin_ctzll(big);
    big &= big - 1;
    const int u = __shfl(v, j, WAVE), cu = __shfl(cv, j, WAVE);
    const int ub = __shfl(b, j, WAVE), ue = __shfl(e, j, WAVE);
    for (int a = ub + lane_id(); a < ue; a += WAVE) {
      const int w = adj[a];
      if (w != u) ldd_claim(cc, rnd, hook, u, cu, w, r);
    }
  }
}

// The queued chunks of round r, one wave per chunk.
__global__ void k_ldd_huge(const int* __restrict__ off, const int* __restrict__ adj, int r,
                           const int2* __restrict__ queue, const int* scal, int* cc, int* rnd,
                           int2* __restrict__ hook) {
  const int count = scal[S_LDD_HUGE + (r & 1)];
  const int waves = gridDim.x * (blockDim.x / WAVE);
  for (int i = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE; i < count; i += waves) {
    const int2 q = queue[i];
    const int u = q.x, cu = ld_relaxed(cc + q.x);
    const int64_t e = off[u + 1];
    const int64_t end = (int64_t)q.y + LDD_CHUNK < e ? (int64_t)q.y + LDD_CHUNK : e;
    for (int64_t a = q.y + lane_id(); a < end; a += WAVE) {
      const int w = adj[a];
      if (w != u) ldd_claim(cc, rnd, hook, u, cu, w, r);
    }
  }
}

// ------------------------------------------------------------ Rooting
// The forest edges (one record per hooked vertex) are numbered densely, edge
// e = (eu[e], ev[e]); its two arcs are list nodes 2e (eu -> ev) and 2e + 1
// (ev -> eu), so an arc's twin is a ^ 1.  Each vertex keeps its out-arcs in a
// linked list built by atomic exchange on a list head (nxt[a] = previous
// head); that list order is the cyclic order the Euler tour uses.  A vertex
// of graph degree >= HUB_DEG may get a huge tree degree, and one head would
// serialise every exchange on one address: such hubs get HUB_SHARDS lists,
// picked by edge number, chained shard after shard.
__device__ __forceinline__ bool is_hub(const int* __restrict__ off, int x) { return off[x + 1] - off[x] >= HUB_DEG; }

// Hub test of the tour kernels: one bit per vertex (a 64-bit word per 64
// vertices), which stays in cache where the row starts would not.
__device__ __forceinline__ bool hub_bit(const unsigned long long* __restrict__ hubbits, int x) {
  return (hubbits[x >> 6] >> (x & 63)) & 1ull;
}

// Per vertex, first pass of Rooting: edge flag for the dense numbering,
// First-CC's sets flattened, the out-list head cleared, hubs numbered (in any
// order: the number only picks the hub's counters) and their bits set (a
// wave covers 64 consecutive vertices from a multiple of 64: one word).
__global__ void k_edge_flags(const int* __restrict__ off, const int2* __restrict__ hook, int n, int* cc,
                             int* __restrict__ eid, int* __restrict__ headp, int* __restrict__ hubidx, int* scal,
                             unsigned long long* __restrict__ hubbits) {
  const int h = vertex_index();
  const bool hub = h < n && is_hub(off, h);
  const unsigned long long bits = __ballot(hub);
  if (lane_id() == 0 && h < n) hubbits[h >> 6] = bits;
  if (h >= n) return;
  eid[h] = hook[h].x >= 0 ? 1 : 0;
  const int r = uf_find(cc, h);
  if (ld_relaxed(cc + h) != r) st_relaxed(cc + h, r);
  headp[h] = -1;
  if (hub) hubidx[h] = atomicAdd(scal + S_HUBS, 1);
}

__global__ void k_edge_compact(const int2* __restrict__ hook, const int* __restrict__ eid, int n,
                               int* __restrict__ eu, int* __restrict__ ev) {
  int h = vertex_index();
  if (h >= n) return;
  const int2 r = hook[h];
  if (r.x < 0) return;
  const int e = eid[h];
  eu[e] = r.x;
  ev[e] = r.y;
}

__device__ __forceinline__ int arc_src(const int* __restrict__ eu, const int* __restrict__ ev, int a) {
  return (a & 1) ? ev[a >> 1] : eu[a >> 1];
}

__global__ void k_tree_link(const unsigned long long* __restrict__ hubbits, const int* __restrict__ hubidx,
                            const int* __restrict__ eid, int n, const int* __restrict__ eu, const int* __restrict__ ev,
                            int* headp, int* shard, int* __restrict__ nxt) {
  const int a = vertex_index();
  if (a >= 2 * eid[n]) return;
  const int s = arc_src(eu, ev, a);
  int* slot = hub_bit(hubbits, s) ? shard + (size_t)hubidx[s] * HUB_SHARDS + ((a >> 1) & (HUB_SHARDS - 1))
                                  : headp + s;
  nxt[a] = atomicExch(slot, a);
}

// Per hub: its first arc (head of the first non-empty shard) into headp, and
// every shard slot rewritten to the head of the next non-empty shard in
// cyclic order, stored as -2 - head when that step wraps around.  Then, for
// every vertex, the root flags: roots of trees with at least one edge get a
// list entry node; a one-vertex tree (an isolated vertex, or one with only
// self-loops) stays out of the Euler tour and takes a preorder number after
// all others.  rdeg is cleared for the root choice.
__global__ void k_hub_lists(const int* __restrict__ off, const int* __restrict__ hubidx,
                            const int* __restrict__ cc, int n, int* headp, int* shard, int* __restrict__ rootidx,
                            int* __restrict__ lone, int* __restrict__ rdeg) {
  int v = vertex_index();
  if (v >= n) return;
  rdeg[v] = -1;
  int hv = headp[v];
  if (is_hub(off, v)) {
    int* sh = shard + (size_t)hubidx[v] * HUB_SHARDS;
    int head[HUB_SHARDS];
    int firsts = -1;
    for (int k = 0; k < HUB_SHARDS; ++k) {
      head[k] = sh[k];
      if (firsts < 0 && head[k] >= 0) firsts = k;
    }
    hv = firsts >= 0 ? head[firsts] : -1;
    headp[v] = hv;
    if (firsts >= 0) {
      for (int k = 0; k < HUB_SHARDS; ++k) {
        int j = k + 1;
        while (j < HUB_SHARDS && head[j] < 0) ++j;
        sh[k] = j < HUB_SHARDS ? head[j] : -2 - head[firsts];
      }
    }
  }
  const bool root = cc[v] == v;
  const bool alone = root && hv < 0;
  rootidx[v] = root && !alone ? 1 : 0;
  lone[v] = alone ? 1 : 0;
}

__global__ void k_root_list(const int* __restrict__ cc, const int* __restrict__ headp,
                            const int* __restrict__ rootidx, const int* __restrict__ rdeg,
                            const int* __restrict__ rsel, const int* __restrict__ scal, int n,
                            int* __restrict__ roots) {
  int v = vertex_index();
  if (v >= n) return;
  if (cc[v] != v || headp[v] < 0) return;
  roots[rootidx[v]] = rdeg[v] >= 0 ? rsel[v] : v;
}

// One-vertex trees: first = last = n - S + (rank among them), S of them in
// all.  Done by the per-vertex pass that starts Tagging.
__device__ __forceinline__ bool lone_tags(const int* __restrict__ lone, int n, int v, int* __restrict__ first,
                                          int4* __restrict__ rec) {
  const int k = lone[v];
  if (lone[v + 1] == k) return false;
  const int f = n - lone[n] + k;
  first[v] = f;
  rec[v] = make_int4(f, f, -1, 0);
  return true;
}

// Exact tags: w1/w2 start empty for the sweep's atomics.
__global__ void k_tag_init(const int* __restrict__ lone, int n, int* __restrict__ first, int4* __restrict__ rec,
                           int* __restrict__ w1, int* __restrict__ w2) {
  int v = vertex_index();
  if (v >= n) return;
  lone_tags(lone, n, v, first, rec);
  w1[v] = INT32_MAX;
  w2[v] = INT32_MIN;
}

// List nodes: [0, C) one entry node per root of a tree with edges (root
// order), then C + [0, 2T) the tree arcs.  The chain runs entry_0, tour_0,
// entry_1, ...  The successor of arc u->v is the arc after v->u in v's cyclic
// out-list; when that step wraps around at the tour's root, the tour of this
// tree is complete and the chain continues with the next entry node.
__device__ __forceinline__ int node_count(const int* __restrict__ rootidx, const int* __restrict__ eid, int n) {
  return rootidx[n] + 2 * eid[n];
}

__global__ void k_euler_next(const unsigned long long* __restrict__ hubbits, const int* __restrict__ hubidx,
                             const int* __restrict__ eid, const int* __restrict__ eu, const int* __restrict__ ev,
                             const int* __restrict__ headp, const int* __restrict__ shard,
                             const int* __restrict__ nxt, const int* __restrict__ cc,
                             const int* __restrict__ rootidx, const int* __restrict__ roots, int n,
                             int* __restrict__ next) {
  const int C = rootidx[n], NL = node_count(rootidx, eid, n);
  int i = vertex_index();
  if (i >= NL) return;
  if (i < C) {
    next[i] = C + headp[roots[i]];
    return;
  }
  const int t = (i - C) ^ 1;  // v -> u, the twin of this arc u -> v
  const int nx = nxt[t];
  if (nx >= 0) {
    next[i] = C + nx;
    return;
  }
  const int v = arc_src(eu, ev, t);
  int head;
  bool wrap;
  if (hub_bit(hubbits, v)) {
    const int q = shard[(size_t)hubidx[v] * HUB_SHARDS + ((t >> 1) & (HUB_SHARDS - 1))];
    wrap = q < 0;
    head = wrap ? -2 - q : q;
  } else {
    wrap = true;
    head = headp[v];
  }
  if (wrap) {
    const int k = rootidx[cc[v]];
    if (roots[k] == v) {  // closes the tour of v's tree: continue with the next tree
      next[i] = k + 1 < C ? k + 1 : -1;
      return;
    }
  }
  next[i] = C + head;
}

__global__ void k_node_count(const int* __restrict__ rootidx, const int* __restrict__ eid, int n, int* out) {
  *out = node_count(rootidx, eid, n);
}

// Each ruler (node index multiple of K) walks to the next ruler.
__global__ void k_lr_walk(const int* __restrict__ next, const int* __restrict__ rootidx,
                          const int* __restrict__ eid, int n, int shift, int2* __restrict__ ol,
                          int* __restrict__ rnext, int* __restrict__ rlen) {
  const int NL = node_count(rootidx, eid, n);
  const int R = (NL + (1 << shift) - 1) >> shift;
  int r = vertex_index();
  if (r >= R) return;
  const int mask = (1 << shift) - 1;
  int i = r << shift, cnt = 0, nr = -1;
  for (int steps = 0; steps < NL; ++steps) {
    ol[i] = make_int2(r, cnt++);
    int j = next[i];
    if (j < 0) break;
    if ((j & mask) == 0) {
      nr = j >> shift;
      break;
    }
    i = j;
  }
  rnext[r] = nr;
  rlen[r] = cnt;
}

// Second level of the ruling set, over the rulers' own list (weighted by
// segment lengths): every 2^shift2-th ruler walks it to the next such ruler,
// recording for each ruler it passes the weight before it.  Pointer jumping
// then runs over 2^shift2 times fewer elements.
__global__ void k_lr_walk2(const int* __restrict__ rootidx, const int* __restrict__ eid, int n, int shift,
                           int shift2, const int* __restrict__ rnext, const int* __restrict__ rlen,
                           int2* __restrict__ ol2, int* __restrict__ rnext2, int* __restrict__ rlen2) {
  const int NL = node_count(rootidx, eid, n);
  const int R = (NL + (1 << shift) - 1) >> shift;
  const int R2 = (R + (1 << shift2) - 1) >> shift2;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= R2) return;
  const int mask = (1 << shift2) - 1;
  int r = q << shift2, acc = 0, nq = -1;
  for (int steps = 0; steps < R; ++steps) {
    ol2[r] = make_int2(q, acc);
    acc += rlen[r];
    const int j = rnext[r];
    if (j < 0) break;
    if ((j & mask) == 0) {
      nq = j >> shift2;
      break;
    }
    r = j;
  }
  rnext2[q] = nq;
  rlen2[q] = acc;
}

// Rulers' suffix sums from the second level's: suf[r] = suf2[q] - (weight
// between q's first ruler and r).  Written over rlen.
__global__ void k_lr_suf(const int* __restrict__ rootidx, const int* __restrict__ eid, int n, int shift,
                         int shift2, const int2* __restrict__ ol2, const int* __restrict__ suf2,
                         int* __restrict__ suf, int* status) {
  const int NL = node_count(rootidx, eid, n);
  const int R = (NL + (1 << shift) - 1) >> shift;
  const int R2 = (R + (1 << shift2) - 1) >> shift2;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int2 o = ol2[r];
  if (o.x < 0 || o.x >= R2) {  // a ruler no second-level walk passed: the tour is broken
    atomicExch(status, (int)FASTBCC_ERR_HIP);
    suf[r] = 0;
    return;
  }
  suf[r] = suf2[o.x] - o.y;
}

// One pointer-jumping round over rulers: suffix sums of segment lengths.
__global__ void k_lr_jump(const int* __restrict__ rootidx, const int* __restrict__ eid, int n, int shift,
                          const int* __restrict__ vin, const int* __restrict__ nin, int* __restrict__ vout,
                          int* __restrict__ nout) {
  const int NL = node_count(rootidx, eid, n);
  const int R = (NL + (1 << shift) - 1) >> shift;
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  int nx = nin[r];
  if (nx >= 0) {
    vout[r] = vin[r] + vin[nx];
    nout[r] = nin[nx];
  } else {
    vout[r] = vin[r];
    nout[r] = -1;
  }
}

// Global position of every node, then its entry flag scattered by position.
__global__ void k_lr_pos(const int* __restrict__ rootidx, const int* __restrict__ eid, int n, int shift,
                         const int2* __restrict__ ol, const int* __restrict__ suf, int* __restrict__ pos,
                         int* status) {
  const int NL = node_count(rootidx, eid, n);
  const int R = (NL + (1 << shift) - 1) >> shift;
  int i = vertex_index();
  if (i >= NL) return;
  int2 o = ol[i];
  if (o.x < 0 || o.x >= R) {  // a node no ruler walked over: the tour is broken
    atomicExch(status, (int)FASTBCC_ERR_HIP);
    pos[i] = -1;
    return;
  }
  pos[i] = NL - suf[o.x] + o.y;
}

__global__ void k_enter_flags(const int* __restrict__ rootidx, const int* __restrict__ eid, int n,
                              const int* __restrict__ pos, int* __restrict__ eflag, int* status) {
  const int C = rootidx[n], NL = node_count(rootidx, eid, n);
  int i = vertex_index();
  if (i >= NL) return;
  int f = 1;
  if (i >= C) f = pos[i] < pos[C + ((i - C) ^ 1)] ? 1 : 0;  // the down arc comes first
  const int p = pos[i];
  if (p < 0 || p >= NL) {
    atomicExch(status, (int)FASTBCC_ERR_HIP);
    return;
  }
  eflag[p] = f;
}

// first/last/parent from the ranked tour: one 16-byte record per vertex plus
// a compact first[] (the array every arc sweep gathers from).
__global__ void k_tags(const int* __restrict__ rootidx, const int* __restrict__ roots,
                       const int* __restrict__ eid, const int* __restrict__ eu, const int* __restrict__ ev,
                       const int* __restrict__ lone, int n, const int* __restrict__ pos,
                       const int* __restrict__ escan, int* __restrict__ first, int4* __restrict__ rec, int* status) {
  const int C = rootidx[n], NL = node_count(rootidx, eid, n);
  int i = vertex_index();
  if (i >= NL) return;
  int v, f, l, p;
  if (i < C) {
    const int pi = pos[i], pn = (i + 1 < C) ? pos[i + 1] : 0;
    if (pi < 0 || pi >= NL || pn < 0 || pn >= NL) {
      atomicExch(status, (int)FASTBCC_ERR_HIP);
      return;
    }
    v = roots[i];
    f = escan[pi];
    int nf = (i + 1 < C) ? escan[pn] : n - lone[n];
    l = nf - 1;
    p = -1;
  } else {
    const int a = i - C, tw = C + (a ^ 1);
    const int pi = pos[i], pt = pos[tw];
    if (pi < 0 || pi >= NL || pt < 0 || pt >= NL) {
      atomicExch(status, (int)FASTBCC_ERR_HIP);
      return;
    }
    if (pi > pt) return;  // up arc
    v = arc_src(eu, ev, a ^ 1);  // the arc runs p -> v
    p = arc_src(eu, ev, a);
    f = escan[pi];
    l = f + (pt - pi - 1) / 2;
  }
  if (v < 0 || v >= n) {
    atomicExch(status, (int)FASTBCC_ERR_HIP);
    return;
  }
  first[v] = f;
  rec[v] = make_int4(f, l, p, 0);
}

// ------------------------------------------------------------ Tagging
// w1[x] = min, w2[x] = max of first[] over x and all its neighbours.  Using
// every neighbour instead of non-tree ones only adds first[p(x)] and values
// inside T_x; neither changes any fence decision.  The gathered first[y] also
// tells whether y is a proper descendant of x (first[x] < first[y] <=
// last[x]); that bit is kept per arc (one ballot word per 64-arc window) for
// the edge-label read-out.
__global__ void k_tag_sweep(const int* __restrict__ off, const int* __restrict__ adj, int n, int64_t A,
                            const int* __restrict__ tile_row, int tw, const int* __restrict__ first,
                            const int4* __restrict__ rec, int* __restrict__ w1, int* __restrict__ w2,
                            unsigned long long* __restrict__ dbits) {
  arc_windows2(
      off, adj, n, A, tile_row, tw,
      [&](int x, int y, bool) {
        const int2 fl = reinterpret_cast<const int2*>(rec)[2 * (int64_t)x];  // (first[x], last[x])
        return make_int3(first[y], fl.x, fl.y);
      },
      [&](int64_t a, int x, bool ok, int y, int3 g) {
        int mn = INT32_MAX, mx = INT32_MIN;
        bool desc = false;
        const int key = ok ? x : -1;
        if (ok && y != x) {
          mn = mx = g.x;
          desc = g.x > g.y && g.x <= g.z;
        }
        const int lane = lane_id();
        const uint64_t dm = __ballot(desc);
        if (lane == 0) dbits[a / WAVE] = dm;  // lane 0 holds the window's first arc, a multiple of 64
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
          int k2 = __shfl_up(key, o, WAVE);
          int m2 = __shfl_up(mn, o, WAVE);
          int x2 = __shfl_up(mx, o, WAVE);
          if (lane >= o && k2 == key) {
            mn = m2 < mn ? m2 : mn;
            mx = x2 > mx ? x2 : mx;
          }
        }
        const int knext = __shfl_down(key, 1, WAVE);
        const bool tail = (lane == WAVE - 1) || knext != key;
        if (tail && key >= 0 && mn != INT32_MAX) {
          atomicMin(w1 + key, mn);
          atomicMax(w2 + key, mx);
        }
      });
}

// Per preorder slot f: (min, max) of the tags, the vertex at that slot and
// whether its tags are exact, one 16-byte record, so a range query gathers
// both tags at once and the preorder map costs no second line.
__global__ void k_rmq_scatter(const int* __restrict__ first, const int* __restrict__ w1, const int* __restrict__ w2,
                              int n, int4* __restrict__ W, int* status) {
  int v = vertex_index();
  if (v >= n) return;
  int f = first[v];
  if (f < 0 || f >= n) {  // preorder numbers must be a permutation of [0, n)
    atomicExch(status, (int)FASTBCC_ERR_HIP);
    return;
  }
  int a = w1[v], b = w2[v];
  W[f] = make_int4(a < f ? a : f, b > f ? b : f, v, 1);
}

__device__ __forceinline__ int2 mm(int2 p, int2 q) {
  return make_int2(q.x < p.x ? q.x : p.x, q.y > p.y ? q.y : p.y);
}

// In-block prefix/suffix (min, max) (block = 64 consecutive preorder slots
// = one wave), block (min, max) into sparse-table level 0.
// With `only`, blocks whose flag is clear are left as they are (a rebuild
// after a few slots changed).
__global__ void k_rmq_block(const int4* __restrict__ W, int n, int64_t nb, const uint8_t* __restrict__ only,
                            int2* __restrict__ pre, int2* __restrict__ suf, int2* __restrict__ tab) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = lane_id();
  if (only && i / WAVE < nb && !only[i / WAVE]) return;  // the whole wave: one block per wave
  const bool in = i < n;
  const int4 w4 = in ? W[i] : make_int4(INT32_MAX, INT32_MIN, 0, 0);
  const int2 w = make_int2(w4.x, w4.y);
  int2 p = w, q = w;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int2 t = make_int2(__shfl_up(p.x, o, WAVE), __shfl_up(p.y, o, WAVE));
    const int2 u = make_int2(__shfl_down(q.x, o, WAVE), __shfl_down(q.y, o, WAVE));
    if (lane >= o) p = mm(p, t);
    if (lane + o < WAVE) q = mm(q, u);
  }
  if (in) {
    pre[i] = p;
    suf[i] = q;
  }
  const int64_t blk = i / WAVE;
  if (lane == 0 && blk < nb) tab[blk] = q;
}

// Sparse-table levels j and, when two_levels, j + 1, both from level j - 1
// (level j + 1 takes four entries of level j - 1), so a launch builds two
// levels.  Entries past the last block are left out of a minimum.
__global__ void k_rmq_level(int2* __restrict__ tab, int64_t nb, int j, bool two_levels) {
  int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int64_t h = int64_t(1) << (j - 1);
  const int2* pt = tab + (size_t)(j - 1) * nb;
  int2 m = pt[b];
  if (b + h < nb) m = mm(m, pt[b + h]);
  tab[(size_t)j * nb + b] = m;
  if (!two_levels) return;
  if (b + 2 * h < nb) m = mm(m, pt[b + 2 * h]);
  if (b + 3 * h < nb) m = mm(m, pt[b + 3 * h]);
  tab[(size_t)(j + 1) * nb + b] = m;
}

// low/high over [first, last]; fence(p(v), v) = first[p] <= low[v] and
// last[p] >= high[v] (paper: Algorithm 1, function Fence).  Updates the
// vertex record in place (only its fence field changes).  Modes:
//   QUERY_EXACT    tags are exact: fence bit 0/1;
//   QUERY_CERTIFY  tags are sampled (low can only be higher, high only lower):
//                  a failed fence test certifies "no fence" (0); a child of a
//                  root is always a fence (1); otherwise the vertex stays
//                  undecided (2) and its preorder interval is counted in cover[]
//                  (difference array) so that its subtree gets exact tags;
//   QUERY_RECHECK  exact test for the undecided vertices only.
enum QueryMode : int { QUERY_EXACT = 0, QUERY_CERTIFY = 1, QUERY_RECHECK = 2 };

//   Thread t handles the vertex at preorder slot t (by_slot), or vertex t:
//   in preorder the range reads of neighbouring threads fall on neighbouring
//   slots, since most subtrees are small.
__global__ void k_rmq_query(int n, int64_t nb, const int4* __restrict__ W, const int2* __restrict__ pre,
                            const int2* __restrict__ suf, const int2* __restrict__ tab, int4* rec, int mode,
                            bool by_slot, int* __restrict__ cover, int* status) {
  const int t = vertex_index();
  if (t >= n) return;
  // the recheck by slot visits only covered slots (cover holds the scanned counts then)
  if (mode == QUERY_RECHECK && cover && cover[t + 1] <= 0) return;
  const int v = by_slot ? W[t].z : t;
  if (v < 0 || v >= n) {  // only if first[] was no permutation (already reported)
    atomicExch(status, (int)FASTBCC_ERR_HIP);
    return;
  }
  const int4 me = rec[v];
  if (mode == QUERY_RECHECK && me.w != 2) return;
  const int l = me.x, r = me.y;
  if (l < 0 || r < l || r >= n) {
    atomicExch(status, (int)FASTBCC_ERR_HIP);
    rec[v] = make_int4(0, n - 1, -1, 0);
    return;
  }
  const int p = me.z;
  if (p < 0) return;
  const int4 pr = rec[p];
  if (mode == QUERY_CERTIFY && pr.z < 0) {
    rec[v].w = 1;
    return;
  }
  const int bl = l / WAVE, br = r / WAVE;
  int2 m;
  bool exact = false;  // every row of the subtree read whole (known for small subtrees)
  if (bl == br) {
    m = make_int2(W[l].x, W[l].y);
    exact = W[l].w != 0;
    for (int k = l + 1; k <= r; ++k) {
      const int4 wk = W[k];
      m = mm(m, make_int2(wk.x, wk.y));
      exact = exact && wk.w != 0;
    }
  } else {
    m = mm(suf[l], pre[r]);
    const int len = br - bl - 1;
    if (len > 0) {
      const int j = 31 - __clz(len);
      const size_t lv = (size_t)j * nb;
      m = mm(m, mm(tab[lv + bl + 1], tab[lv + br - (1 << j)]));
    }
  }
  const bool fence = pr.x <= m.x && pr.y >= m.y;
  if (mode == QUERY_CERTIFY) {
    if (fence && exact) {
      rec[v].w = 1;  // every row under v was read whole: the tags, and so the test, are exact
    } else if (fence) {
      rec[v].w = 2;
      atomicAdd(cover + l, 1);
      atomicAdd(cover + r + 1, -1);
    }
  } else if (mode == QUERY_RECHECK || fence) {
    rec[v].w = fence ? 1 : 0;
  }
}

// ------------------------------------------------------------ sampled tags
// Tags from a sample of each row: ks consecutive neighbours from a hashed
// start, or the whole row when it is no longer (then the tags are exact).
// Sampled w1 can only be higher and w2 only lower than the exact ones, which
// is what the certification pass relies on.
__global__ void k_tag_sample(const int* __restrict__ off, const int* __restrict__ adj, const int* __restrict__ lone,
                             int* __restrict__ first, int4* __restrict__ rec, int n, int ks, int4* __restrict__ W,
                             int* __restrict__ cover, int* scal, int* status) {
  const int x = vertex_index();
  if (x < 2) cover[n + x] = 0;  // the certification's difference array (n + 2 slots) starts at zero
  if (x == 0) scal[S_DIRTY] = 0;
  if (x >= n) return;
  cover[x] = 0;
  int f, mn, mx;
  bool exact = true;  // the tags are exact unless the row was sampled
  if (lone_tags(lone, n, x, first, rec)) {  // no neighbour but itself: its tags are its own
    f = mn = mx = first[x];
  } else {
    f = mn = mx = first[x];
    const int b = off[x], d = off[x + 1] - b;
    exact = d <= ks;
    if (d <= ks) {
      for (int k = 0; k < d; ++k) {
        const int y = adj[b + k];
        if (y == x) continue;
        const int fy = first[y];
        mn = fy < mn ? fy : mn;
        mx = fy > mx ? fy : mx;
      }
    } else {
      // ks consecutive arcs from a hashed start: one adjacency line instead
      // of ks (any subset of the row keeps the sampled tags sound)
      const int s0 = b + sample_pos(x, 0, d - ks + 1);
      for (int k = 0; k < ks; ++k) {
        const int y = adj[s0 + k];
        if (y == x) continue;
        const int fy = first[y];
        mn = fy < mn ? fy : mn;
        mx = fy > mx ? fy : mx;
      }
    }
  }
  if (f < 0 || f >= n) {  // preorder numbers must be a permutation of [0, n)
    atomicExch(status, (int)FASTBCC_ERR_HIP);
    return;
  }
  // straight into the RMQ input, by preorder slot, with the vertex and
  // whether the tags are exact
  W[f] = make_int4(mn, mx, x, exact ? 1 : 0);
}

// Slot i of the preorder: its vertex's row needs exact tags when an undecided
// interval covers i (cover = exclusive scan of the difference array, so the
// count at i is cover[i + 1]) and its tags were sampled.  Such rows are
// appended to a list, one counter atomic per block.
__global__ void __launch_bounds__(BLOCK) k_dirty_list(const int* __restrict__ off, const int4* __restrict__ W,
                                                      const int* __restrict__ cover, int n, int ks,
                                                      int* __restrict__ list, int* count) {
  __shared__ int wsum[BLOCK / WAVE];
  __shared__ int base;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int x = -1;
  if (i < n && cover[i + 1] > 0) {
    const int y = W[i].z;
    if (y >= 0 && y < n && off[y + 1] - off[y] > ks) x = y;  // else first[] was no permutation (reported)
  }
  const unsigned long long m = __ballot(x >= 0);
  const int lane = lane_id(), wid = threadIdx.x / WAVE;
  if (lane == 0) wsum[wid] = __builtin_popcountll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int k = 0; k < BLOCK / WAVE; ++k) {
      const int c = wsum[k];
      wsum[k] = t;
      t += c;
    }
    base = t ? atomicAdd(count, t) : 0;
  }
  __syncthreads();
  if (x >= 0) list[base + wsum[wid] + __builtin_popcountll(m & ((1ull << lane) - 1))] = x;
}

// Exact w1/w2 of the listed rows: a wave per row (grid-stride over the list)
// takes min/max of first[] over the whole row and folds them into the row's
// RMQ slot (each row is listed once), whose block is then rebuilt.
__global__ void k_tag_rows(const int* __restrict__ off, const int* __restrict__ adj, const int* __restrict__ list,
                           const int* __restrict__ count, const int* __restrict__ first, int4* __restrict__ W,
                           uint8_t* __restrict__ dirty_block) {
  const int lane = lane_id();
  const int nw = (int)(((int64_t)gridDim.x * blockDim.x) / WAVE);
  const int cnt = *count;
  for (int r = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE); r < cnt; r += nw) {
    const int x = list[r];
    const int b = off[x], e = off[x + 1];
    int mn = INT32_MAX, mx = INT32_MIN;
    for (int a = b + lane; a < e; a += WAVE) {
      const int y = adj[a];
      if (y == x) continue;
      const int fy = first[y];
      mn = fy < mn ? fy : mn;
      mx = fy > mx ? fy : mx;
    }
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
      const int m2 = __shfl_xor(mn, o, WAVE), x2 = __shfl_xor(mx, o, WAVE);
      mn = m2 < mn ? m2 : mn;
      mx = x2 > mx ? x2 : mx;
    }
    if (lane == 0 && mn != INT32_MAX) {
      const int f = first[x];
      int4 wf = W[f];
      wf.x = mn < wf.x ? mn : wf.x;
      wf.y = mx > wf.y ? mx : wf.y;
      W[f] = wf;
      dirty_block[f / WAVE] = 1;
    }
  }
}

// ------------------------------------------------------------ Last-CC

// Last-CC hooks by id (a set's root is its smallest member, which the
// read-out relies on) or, as a tuning variant, by hashed priority (shallower
// trees on lattices and long paths) followed by a relabelling to the smallest
// member.  One rule per solve: mixing rules could hook two roots under each
// other.
template <bool PRIO>
__device__ __forceinline__ void lcc_link(int* lab, int u, int v) {
  if (PRIO) uf_link_prio(lab, u, v);
  else uf_link(lab, u, v);
}

// Plain (non-fence) tree edges are skeleton edges.  First without atomics,
// from all-singleton sets: v points to its parent when the parent ranks
// above it (the hooking rule's order, so the pointers are acyclic and every
// set's root is still the member the rule would leave on top); this pass also
// initialises every set.  Then the other plain tree edges by union-find.
template <bool PRIO>
__global__ void k_lcc_tree_free(const int4* __restrict__ rec, int n, int* __restrict__ lab) {
  int v = vertex_index();
  if (v >= n) return;
  const int4 r = rec[v];
  lab[v] = (r.z >= 0 && r.w == 0 && ranks_above<PRIO>(r.z, v)) ? r.z : v;
}

template <bool PRIO>
__global__ void k_lcc_tree(const int4* __restrict__ rec, int n, int* lab) {
  int v = vertex_index();
  if (v >= n) return;
  int4 r = rec[v];
  if (r.z >= 0 && r.w == 0 && !ranks_above<PRIO>(r.z, v)) lcc_link<PRIO>(lab, v, r.z);
}

// Non-tree arc x-y is a skeleton edge iff neither endpoint is an ancestor of
// the other (paper: InSkeleton and Back).  Tree arcs (either endpoint the
// other's parent; also repeated copies of a tree edge) are left to k_lcc_tree.
__device__ __forceinline__ bool cross_edge(int x, int4 rx, int y, int4 ry) {
  if (ry.z == x || rx.z == y) return false;
  const bool y_under_x = rx.x <= ry.x && ry.x <= rx.y;
  const bool x_under_y = ry.x <= rx.x && rx.x <= ry.y;
  return !y_under_x && !x_under_y;
}

// Last-CC per graph of a batch (FASTBCC_TUNE_GRAPH_CC): the union-find of
// k_graph_cc on the skeleton instead of the graph -- plain tree edges and
// cross edges (InSkeleton: neither endpoint an ancestor of the other) --
// hooked by id, so each set's root is its smallest member, as the read-out
// needs.  The row pass links each vertex's plain tree edge and, of the two
// neighbours at hashed positions of its row, those across cross edges; the
// sweep then reads every arc of the rows outside the sampled largest set.  Graphs above the
// LDS size run on the device-memory union-find (flattened afterwards).
__global__ void __launch_bounds__(GCC_THREADS) k_graph_lcc(const int* __restrict__ vbegin, int G, int n,
                                                           const int* __restrict__ off, const int* __restrict__ adj,
                                                           const int4* __restrict__ rec, int* lab, int* next_graph,
                                                           const int* __restrict__ order) {
  __shared__ uint32_t P[GCC_LDS_VERTICES / 2];
  __shared__ int g_s, big_s;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) g_s = claim_graph(next_graph, order, G);
    __syncthreads();
    const int g = g_s;
    __syncthreads();  // everyone has read g_s before it is rewritten
    if (g >= G) break;
    const int v0 = min(max(vbegin[g], 0), n), v1 = min(max(vbegin[g + 1], v0), n), ng = v1 - v0;
    if (ng == 0) continue;
    const bool in_lds = ng <= GCC_LDS_VERTICES;
    // Sets start from the plain tree edges to a parent of smaller id, without
    // atomics (pointers to smaller ids are acyclic, and each pointer tree's
    // root is its smallest member, as min-id hooking keeps it); the plain
    // tree edges to a parent of larger id are linked after the barrier.
    for (int v = tid; v < ng; v += GCC_THREADS) {
      const int4 r = rec[v0 + v];
      const bool up = r.z >= v0 && r.z < v0 + v && r.w == 0;
      if (in_lds) p16_set(P, v, up ? r.z - v0 : v);
      else lab[v0 + v] = up ? r.z : v0 + v;
    }
    __syncthreads();
    const int a0 = off[v0], A = max(off[v1] - a0, 0);
    auto link = [&](int x, int y) {
      if (!in_lds) {
        uf_link(lab, v0 + x, v0 + y);
        return;
      }
      if (p16_get(P, x) == p16_get(P, y)) return;  // same parent: same set
      int ru = p16_find(P, x), rv = p16_find(P, y);
      while (ru != rv) {
        const int h = ru > rv ? ru : rv, l = ru > rv ? rv : ru;
        if (p16_cas(P, h, h, l)) return;
        ru = p16_find(P, ru);
        rv = p16_find(P, rv);
      }
    };
    for (int v = tid; v < ng; v += GCC_THREADS) {
      const int4 r = rec[v0 + v];
      if (r.z > v0 + v && r.z < v1 && r.w == 0) link(v, r.z - v0);
    }
    __syncthreads();
    int big = -1;
    if (in_lds) {
      if (tid < WAVE) {
        const int r = p16_root(P, (int)((int64_t)tid * ng / WAVE));
        int cnt = 0;
        for (int j = 0; j < WAVE; ++j) cnt += __shfl(r, j, WAVE) == r ? 1 : 0;
        int best_c = cnt, best_r = r;
        for (int o = WAVE / 2; o > 0; o >>= 1) {
          const int oc = __shfl_xor(best_c, o, WAVE), orr = __shfl_xor(best_r, o, WAVE);
          if (oc > best_c || (oc == best_c && orr < best_r)) {
            best_c = oc;
            best_r = orr;
          }
        }
        if (tid == 0) big_s = best_r;
      }
      __syncthreads();
      big = big_s;
    }
    for (int xb = 0; xb < ng; xb += GCC_THREADS) {  // the same trip count on every wave
      const int xo = xb + tid;
      int rb = 0, re = 0;
      int4 ro = make_int4(0, -1, -1, 0);
      if (xo < ng && !(in_lds && p16_find(P, xo) == p16_find(P, big))) {
        rb = min(max(off[v0 + xo] - a0, 0), A);
        re = min(max(off[v0 + xo + 1] - a0, rb), A);
        if (re > rb) ro = rec[v0 + xo];
      }
      wave_row_arcs(rb, re, [&](int owner, int a) {
        const int x = __shfl(xo, owner, WAVE);
        const int4 rx = make_int4(__shfl(ro.x, owner, WAVE), __shfl(ro.y, owner, WAVE), __shfl(ro.z, owner, WAVE),
                                  __shfl(ro.w, owner, WAVE));
        if (a < 0) return;
        const int y = adj[a0 + a] - v0;
        // each edge once in memory mode
        if (y == x || y < 0 || y >= ng || (!in_lds && y < x)) return;
        if (cross_edge(v0 + x, rx, v0 + y, rec[v0 + y])) link(x, y);
      });
    }
    __syncthreads();
    if (in_lds)
      for (int v = tid; v < ng; v += GCC_THREADS) lab[v0 + v] = v0 + p16_root(P, v);
    __syncthreads();  // the next graph reuses P
  }
}

template <bool PRIO>
__global__ void k_lcc_sample(const int* __restrict__ off, const int* __restrict__ adj, const int4* __restrict__ rec,
                             int n, int r, int* lab) {
  int v = vertex_index();
  if (v >= n) return;
  const int64_t b = off[v], e = off[v + 1];
  if (e > b) {
    int y = adj[b + sample_pos(v, r, e - b)];
    if (y != v && cross_edge(v, rec[v], y, rec[y])) lcc_link<PRIO>(lab, v, y);
  }
}

template <bool PRIO>
__global__ void k_lcc_sweep(const int* __restrict__ off, const int* __restrict__ frow, const int* __restrict__ fstart,
                            const int* __restrict__ adj, const int* __restrict__ frows, const int* __restrict__ ftile,
                            int tw, const int4* __restrict__ rec, int* lab) {
  const int R = *frows;
  const int64_t F = fstart[R];
  arc_tiles(fstart, R, F, ftile, tw, [&](int64_t k, int i, bool ok) {
    if (!ok) return;
    const int x = frow[i];
    const int64_t a = (int64_t)off[x] + (k - (int64_t)fstart[i]);
    const int y = adj[a];
    if (y != x && cross_edge(x, rec[x], y, rec[y])) lcc_link<PRIO>(lab, x, y);
  });
}

// After priority hooking: every label becomes the smallest member of its set.
// The largest set (sampled label big) takes a two-level reduction (block
// minima, then one block over them); the others take the minimum of their
// members with one atomic per run of equal labels in a wave.
__global__ void k_big_min_part(const int* __restrict__ lab, int n, const int* __restrict__ scal,
                               int* __restrict__ part) {
  __shared__ int wmin[BLOCK / WAVE];
  const int big = lab[scal[S_BIG_LAB]];
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  int m = (v < n && lab[v] == big) ? v : INT32_MAX;
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const int m2 = __shfl_down(m, o, WAVE);
    m = m2 < m ? m2 : m;
  }
  if (lane_id() == 0) wmin[threadIdx.x / WAVE] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < BLOCK / WAVE; ++w) m = wmin[w] < m ? wmin[w] : m;
    part[blockIdx.x] = m;
  }
}

__global__ void __launch_bounds__(1024) k_big_min(const int* __restrict__ lab, const int* __restrict__ part,
                                                  int parts, int* scal) {
  __shared__ int wmin[1024 / WAVE];
  int m = INT32_MAX;
  for (int i = threadIdx.x; i < parts; i += blockDim.x) m = part[i] < m ? part[i] : m;
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const int m2 = __shfl_down(m, o, WAVE);
    m = m2 < m ? m2 : m;
  }
  if (lane_id() == 0) wmin[threadIdx.x / WAVE] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 1024 / WAVE; ++w) m = wmin[w] < m ? wmin[w] : m;
    scal[S_BIG_ROOT] = lab[scal[S_BIG_LAB]];
    scal[S_BIG_MIN] = m;
  }
}

__global__ void k_label_min(const int* __restrict__ lab, int n, const int* __restrict__ scal, int* minv) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  int L = -1;
  if (v < n) L = lab[v];
  if (L == scal[S_BIG_ROOT]) L = -1;
  int m = v;
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int l2 = __shfl_up(L, o, WAVE), m2 = __shfl_up(m, o, WAVE);
    if (lane >= o && l2 == L && m2 < m) m = m2;
  }
  const int ln = __shfl_down(L, 1, WAVE);
  // minima only fall, so a read that already shows m or less makes the
  // atomic moot; blocks run roughly in vertex order, so the first visitor of
  // a label usually holds its minimum and the rest only read
  if (L >= 0 && (lane == WAVE - 1 || ln != L) && m < minv[L]) atomicMin(minv + L, m);
}

__global__ void k_relabel(int* lab, int n, const int* __restrict__ scal, const int* __restrict__ minv) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int L = lab[v];
  lab[v] = L == scal[S_BIG_ROOT] ? scal[S_BIG_MIN] : minv[L];
}

// ------------------------------------------------------------ read-out
__global__ void k_readout_init(int n, int* __restrict__ head, uint8_t* __restrict__ heads, int* __restrict__ rootlab,
                               int* __restrict__ minid, uint8_t* __restrict__ ap) {
  int v = vertex_index();
  if (v >= n) return;
  head[v] = -1;
  heads[v] = 0;
  rootlab[v] = -1;
  minid[v] = INT32_MAX;
  if (ap) ap[v] = 0;
}

// head(l[u]) = p(u) when l[u] != l[p(u)] (paper: Algorithm 1, component
// heads).  A non-root head is an articulation point; a tree root is one iff
// it heads two different labels.
// A BCC label is a Last-CC root that is not a tree root (a tree root is a
// singleton of the skeleton and heads, but never labels, a BCC).
__device__ __forceinline__ bool is_bcc_label(const int4* __restrict__ rec, const int* __restrict__ lab, int v) {
  return lab[v] == v && rec[v].z >= 0;
}

// Heads, head flags and articulation points; with bsum also the block's
// count of BCC labels, which shares this pass's reads of rec and lab.
__global__ void __launch_bounds__(BLOCK) k_bcc_heads(const int4* __restrict__ rec, const int* __restrict__ lab, int n,
                                                     int* __restrict__ head, uint8_t* __restrict__ heads,
                                                     int* rootlab, uint8_t* __restrict__ ap, int* __restrict__ bsum) {
  __shared__ int part[BLOCK / WAVE];
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  bool is_label = false;
  if (v < n) {
    const int4 r = rec[v];
    const int p = r.z;
    const int L = lab[v];
    is_label = L == v && p >= 0;  // is_bcc_label on the values at hand
    // a plain (non-fence) tree edge joins v and p in Last-CC: same label, no head
    if (p >= 0 && r.w != 0 && L != lab[p]) {
      head[L] = p;
      heads[p] = 1;
      if (ap != nullptr) {
        if (rec[p].z >= 0) {
          ap[p] = 1;
        } else {
          int old = atomicCAS(rootlab + p, -1, L);
          if (old != -1 && old != L) ap[p] = 1;
        }
      }
    }
  }
  if (bsum == nullptr) return;  // uniform
  const uint64_t m = __ballot(is_label);
  if (lane_id() == 0) part[threadIdx.x / WAVE] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < BLOCK / WAVE; ++w) t += part[w];
    bsum[blockIdx.x] = t;
  }
}

// BCC count of a batch, a wave per graph: the whole BLOCK-vertex blocks
// inside the graph come from the exclusive scan P of k_bcc_heads' block
// counts, the partial blocks at its two ends are counted here.
__global__ void k_graph_count(const int4* __restrict__ rec, const int* __restrict__ lab, int n,
                              const int* __restrict__ vbegin, int G, const int* __restrict__ P,
                              int64_t* __restrict__ nbcc) {
  const int g = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE);
  if (g >= G) return;  // the whole wave
  const int a = min(max(vbegin[g], 0), n), b = min(max(vbegin[g + 1], a), n);
  const int ba = (a + BLOCK - 1) / BLOCK, bb = b / BLOCK;  // whole blocks [ba, bb)
  int64_t t = 0;
  int lo_end = b, hi_start = b;  // no whole block: count [a, b) directly
  if (ba < bb) {
    t = P[bb] - P[ba];
    lo_end = ba * BLOCK;
    hi_start = bb * BLOCK;
  }
  const int lane = lane_id();
  for (int v = a + lane; v - lane < lo_end; v += WAVE)
    t += __popcll(__ballot(v < lo_end && is_bcc_label(rec, lab, v)));
  for (int v = hi_start + lane; v - lane < b; v += WAVE)
    t += __popcll(__ballot(v < b && is_bcc_label(rec, lab, v)));
  if (lane == 0) nbcc[g] = t;
}

// Sum of nblocks ints into *out, which the solve zeroed: SUM_PER_LANE
// values per lane, one 64-bit atomic per block.
constexpr int SUM_PER_LANE = 4;
__global__ void __launch_bounds__(1024) k_sum_blocks(const int* __restrict__ bsum, int nblocks, int64_t* out) {
  __shared__ long long part[1024 / WAVE];
  const int base = blockIdx.x * blockDim.x * SUM_PER_LANE + threadIdx.x;
  long long t = 0;
#pragma unroll
  for (int k = 0; k < SUM_PER_LANE; ++k) {
    const int j = base + k * (int)blockDim.x;
    const int x = bsum[min(j, nblocks - 1)];  // in bounds for every lane, so the loads overlap
    t += j < nblocks ? x : 0;
  }
  for (int o = WAVE / 2; o > 0; o >>= 1) t += __shfl_down(t, o, WAVE);
  if (lane_id() == 0) part[threadIdx.x / WAVE] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long s = 0;
    for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) s += part[w];
    if (s) atomicAdd((unsigned long long*)out, (unsigned long long)s);
  }
}

// The label of the largest skeleton component (the giant BCC on power-law
// graphs) and a bitmap of its members: 1 bit per vertex (4 MB at n = 2^25)
// stays in L2, so most arcs of head rows learn l[y] without a gather.
__global__ void k_lbig(const int* __restrict__ lab, int* scal) { scal[S_LBIG] = lab[scal[S_BIG_LAB]]; }

__global__ void k_big_bitmap(const int* __restrict__ lab, int n, const int* __restrict__ scal,
                             unsigned long long* __restrict__ bits) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int big = scal[S_LBIG];
  const uint64_t m = __ballot(v < n && lab[v] == big);
  if (lane_id() == 0 && v < n) bits[v / WAVE] = m;
}

// The canonical label of the largest label's BCC, computed before pass 1 by
// scanning the one row that holds its smallest arc (the row of its smallest
// vertex, see pass 1), so pass 1 can write final labels for its arcs.
__global__ void __launch_bounds__(BLOCK) k_big_canon(const int* __restrict__ off, const int* __restrict__ adj,
                                                      const int4* __restrict__ rec, const int* __restrict__ lab,
                                                      const int* __restrict__ head,
                                                      const uint8_t* __restrict__ heads,
                                                      const int* __restrict__ vbegin, int G, int* scal) {
  __shared__ int part[BLOCK / WAVE];
  const int Lb = scal[S_LBIG];
  if (rec[Lb].z < 0 || lab[Lb] != Lb) {  // a tree root or an isolated vertex: labels no arc
    if (threadIdx.x == 0) scal[S_CANON_BIG] = -1;
    return;
  }
  const int hb = head[Lb];
  const int x = (hb >= 0 && hb < Lb) ? hb : Lb;
  const int lx = lab[x], hx = head[lx];
  int best = INT32_MAX;
  for (int64_t a = (int64_t)off[x] + threadIdx.x; a < off[x + 1]; a += blockDim.x) {
    const int y = adj[a];
    if (y == x) continue;
    int L;
    if (!heads[x]) {
      L = lx;
    } else {
      const int ly = lab[y];
      L = (ly == lx || hx == y) ? lx : ly;
    }
    if (L == Lb && (int)a < best) best = (int)a;
  }
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    int b2 = __shfl_down(best, o, WAVE);
    best = b2 < best ? b2 : best;
  }
  if (lane_id() == 0) part[threadIdx.x / WAVE] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < BLOCK / WAVE; ++w) best = part[w] < best ? part[w] : best;
    if (best != INT32_MAX && G > 1) best -= off[vbegin[graph_index(vbegin, G, Lb)]];
    scal[S_CANON_BIG] = best == INT32_MAX ? -1 : best;
  }
}

// Pass 1 over the arcs.  Arc x->y lies in the BCC whose vertex set holds both
// endpoints: the label of x when l[x] == l[y] or y heads l[x] (x's BCC is
// {l == l[x]} plus its head), else the label of y (then x heads l[y]).  Two
// BCCs share at most one vertex, so this is the edge's unique BCC.  A vertex
// that heads no BCC lies in exactly one BCC, so its row needs no gather.  In
// a head row, an arc whose target is not a proper descendant of x (the tag
// sweep's bit) lies on a cycle through the tree edge (x, p(x)), or that edge
// itself, whose BCC is l[x]: no gather either.  The remaining arcs read l[y]
// from the giant-label bitmap when its bit is set.  The
// smallest arc of BCC L lies in the row of its smallest vertex
// m(L) = min(L, head(L)) (L is the smallest non-head vertex, the Last-CC
// root); arcs of that row update minid[L].  Arcs of the largest label get
// its final canonical label; the others get the raw label encoded as -2 - L
// (self-loops -1), resolved by pass 2.
// How pass 1 learns l[y] in the rows of heads (unsorted rows; sorted rows
// take the one-pass read-out below):
//   LABEL_BITMAP  every arc gathers (bitmap bit, else the record of y);
//   LABEL_DBITS   only arcs to proper descendants (bits from the tag sweep).
enum LabelMode : int { LABEL_BITMAP = 0, LABEL_DBITS = 1 };

__device__ __forceinline__ int bcc_min_vertex(int L, int h) { return (h >= 0 && h < L) ? h : L; }

template <int MODE>
__global__ void k_bcc_label(const int* __restrict__ off, const int* __restrict__ adj, int n, int64_t A,
                            const int* __restrict__ tile_row, int tw, const int4* __restrict__ vlh,
                            const uint8_t* __restrict__ heads, const unsigned long long* __restrict__ bits,
                            const unsigned long long* __restrict__ dbits, const int* __restrict__ head,
                            const int* __restrict__ scal, int* __restrict__ minid, int* __restrict__ out) {
  const int big = scal[S_LBIG];
  const int hbig = head[big];
  const int4 rbig = make_int4(big, hbig, bcc_min_vertex(big, hbig), 0);
  const int canon_big = scal[S_CANON_BIG];
  arc_windows2(
      off, adj, n, A, tile_row, tw,
      [&](int x, int, bool) { return vlh[x]; },
      [&](int64_t a, int x, bool ok, int y, int4 rx) {
        if (!ok) return;
        if (y == x) {
          __builtin_nontemporal_store(-1, out + a);
          return;
        }
        // rx = (l[x], head(l[x]), smallest vertex of l[x]'s BCC, exact-row flag)
        int L = rx.x, m = rx.z;
        bool look;
        if (MODE == LABEL_DBITS) look = heads[x] && ((dbits[a / WAVE] >> (a % WAVE)) & 1ull);
        else look = heads[x] != 0;
        if (look) {
          const int4 ry = ((bits[y / WAVE] >> (y % WAVE)) & 1ull) ? rbig : vlh[y];
          if (ry.x != rx.x && rx.y != y) {
            L = ry.x;
            m = ry.z;
          }
        }
        const bool final_big = L == big && canon_big >= 0;
        __builtin_nontemporal_store(final_big ? canon_big : -2 - L, out + a);
        if (m == x && !final_big) atomicMin(minid + L, (int)a);
      });
}

// Per vertex: (l, head(l), smallest vertex of the BCC, exact-row flag).  A
// head row stays exact (gathers per arc in the mirror mode) when x is a tree
// root, heads the largest label, or is the smallest vertex of its own BCC
// (its arcs update minid[l[x]], so none may be mislabelled there first).
__global__ void k_vertex_lh(const int* __restrict__ lab, const int* __restrict__ head,
                            const uint8_t* __restrict__ heads, const int4* __restrict__ rec,
                            const int* __restrict__ scal, int n, int4* __restrict__ vlh) {
  int v = vertex_index();
  if (v >= n) return;
  const int l = lab[v], h = head[l], m = bcc_min_vertex(l, h);
  const bool exact = heads[v] && (rec[v].z < 0 || v == head[scal[S_LBIG]] || m == v);
  vlh[v] = make_int4(l, h, m, exact ? 1 : 0);
}

// ---- final labels in one pass (sorted rows): canonical labels first
// The smallest arc of BCC L lies in the row of its smallest vertex m(L).
// When m(L) is the head h, that arc is h->y for the smallest member y next to
// h: the mirror search below finds every arc h->y anyway.  Otherwise m(L) = L
// (a member, the Last-CC root): a non-head's row lies wholly in L, so its
// first arc that is not a self-loop; a head's row is scanned with the exact
// rule until its first arc in L.

// Binary search of y in h's row (first copy), -1 if absent.
__device__ __forceinline__ int row_lower(const int* __restrict__ off, const int* __restrict__ adj, int h, int y) {
  int lo = off[h], hi = off[h + 1];
  const int e = hi;
  while (lo < hi) {
    const int mid = lo + ((hi - lo) >> 1);
    if (adj[mid] < y) lo = mid + 1;
    else hi = mid;
  }
  return (lo < e && adj[lo] == y) ? lo : -1;
}

// Per vertex y of a non-largest BCC L with head h: where the arcs h->y start
// in h's row and how many copies there are (mpos, mcnt; -1 / 0 if h and y
// are not adjacent), and minid[L] when h is the smallest vertex of the BCC.
__global__ void k_mirror_find(const int* __restrict__ off, const int* __restrict__ adj, int n,
                              const int4* __restrict__ vlh, const int* __restrict__ scal, int* __restrict__ minid,
                              int* __restrict__ mpos, int* __restrict__ mcnt) {
  const int y = vertex_index();
  if (y >= n) return;
  const int4 r = vlh[y];  // (l, head(l), smallest vertex of the BCC, exact-row flag)
  int a = -1, k = 0;
  if (r.y >= 0 && r.x != scal[S_LBIG]) {
    a = row_lower(off, adj, r.y, y);
    if (a >= 0) {
      if (r.z == r.y) atomicMin(minid + r.x, a);
      const int e = off[r.y + 1];
      do ++k;
      while (a + k < e && adj[a + k] == y);
    }
  }
  mpos[y] = a;
  mcnt[y] = k;
}

// canon[L] for every BCC label, graph-local for batches.
__global__ void k_canon_first(const int* __restrict__ off, const int* __restrict__ adj, int n,
                              const int4* __restrict__ rec, const int* __restrict__ lab,
                              const int4* __restrict__ vlh, const uint8_t* __restrict__ heads,
                              const unsigned long long* __restrict__ bits, const int* __restrict__ scal,
                              const int* __restrict__ minid, const int* __restrict__ vbegin, int G,
                              int* __restrict__ canon) {
  const int v = vertex_index();
  const int big = scal[S_LBIG];
  bool label = v < n && is_bcc_label(rec, lab, v);
  int c = -1;
  bool scan = false;
  int4 r = make_int4(0, -1, 0, 0);
  if (label) {
    r = vlh[v];  // v is a label, so r = (v, head(v), m(v), exact)
    if (v == big && scal[S_CANON_BIG] >= 0) {
      canon[v] = scal[S_CANON_BIG];
      label = false;
    } else if (r.z == r.y) {
      c = minid[v];
    } else if (!heads[v]) {
      int a = off[v];
      const int e = off[v + 1];
      while (a < e && adj[a] == v) ++a;
      c = a;
    } else {
      scan = true;
    }
  }
  // rows of heads: the wave scans each one 64 arcs at a time
  uint64_t todo = __ballot(scan);
  while (todo) {
    const int j = __builtin_ctzll(todo);
    todo &= todo - 1;
    const int x = __shfl(v, j, WAVE), hx = __shfl(r.y, j, WAVE);
    const int b = off[x], e = off[x + 1];
    int found = -1;
    for (int base = b; base < e && found < 0; base += WAVE) {
      const int a = base + lane_id();
      bool in = false;
      if (a < e) {
        const int y = adj[a];
        if (y != x) {
          const int ly = ((bits[y / WAVE] >> (y % WAVE)) & 1ull) ? big : lab[y];
          in = ly == x || hx == y;
        }
      }
      const uint64_t hit = __ballot(in);
      if (hit) found = base + __builtin_ctzll(hit);
    }
    if (lane_id() == j) c = found;
  }
  if (label) {
    if (G > 1 && c >= 0) c -= off[vbegin[graph_index(vbegin, G, v)]];
    canon[v] = c;
  }
}

// Records for the final pass: z becomes canon(l) (canon is -1 where l labels
// no BCC).
__global__ void k_vertex_canon(const int* __restrict__ canon, int n, int4* __restrict__ vlh) {
  const int v = vertex_index();
  if (v >= n) return;
  vlh[v].z = canon[vlh[v].x];
}

// One pass: every arc gets its final label; rows marked exact gather per arc.
__global__ void k_bcc_final(const int* __restrict__ off, const int* __restrict__ adj, int n, int64_t A,
                            const int* __restrict__ tile_row, int tw, const int4* __restrict__ vlh,
                            const unsigned long long* __restrict__ bits, const int* __restrict__ scal,
                            int* __restrict__ out) {
  const int big = scal[S_LBIG];
  const int4 rbig = vlh[big];
  arc_windows2(
      off, adj, n, A, tile_row, tw,
      [&](int x, int, bool) { return vlh[x]; },
      [&](int64_t a, int x, bool ok, int y, int4 rx) {
        if (!ok) return;
        if (y == x) {
          __builtin_nontemporal_store(-1, out + a);
          return;
        }
        // rx = (l[x], head(l[x]), canon(l[x]), exact-row flag)
        int c = rx.z;
        if (rx.w) {
          const int4 ry = ((bits[y / WAVE] >> (y % WAVE)) & 1ull) ? rbig : vlh[y];
          if (ry.x != rx.x && rx.y != y) c = ry.z;
        }
        __builtin_nontemporal_store(c, out + a);
      });
}

// Number of the 64 row ends held in `e` (ascending over the lanes) that are
// <= a: a binary search over the lanes.
__device__ __forceinline__ int block_count(int e, int a) {
  int pos = 0;
#pragma unroll
  for (int step = 32; step >= 1; step >>= 1)
    if (__shfl(e, pos + step - 1, WAVE) <= a) pos += step;
  if (pos == WAVE - 1 && __builtin_amdgcn_readlane(e, WAVE - 1) <= a) pos = WAVE;
  return pos;
}

// The same pass for inputs without self-loops (sorted rows): only exact rows
// read their targets; every other arc takes its row's label, so the pass is
// a row-wise fill.  A wave walks its tile's 64-arc windows holding a block of
// 64 consecutive rows in registers, per lane the end of one row and that
// row's label with the exact-row flag in bit 31.  Most arcs lie in windows
// inside one row (high-degree rows hold most arcs): such a window costs one
// compare.  The few row ends inside other windows are counted from a ballot,
// lane by lane.  Loads happen only when the walk leaves the block (the block
// then restarts at the window's first row), for exact rows, and for windows
// spanning more than 64 rows; waits for them also wait for the stores in
// flight, so the windows between them run without any wait.
typedef int v4i __attribute__((ext_vector_type(4)));

__global__ void k_bcc_rows(const int* __restrict__ off, const int* __restrict__ adj, int n, int64_t A,
                           const int* __restrict__ tile_row, int tw, int stride, const int4* __restrict__ vlh,
                           const unsigned long long* __restrict__ bits, const int* __restrict__ scal,
                           bool out16, int* __restrict__ out) {
  const int lane = lane_id();
  const int64_t wave =
      __builtin_amdgcn_readfirstlane((int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE));
  const int64_t tile_arcs = (int64_t)WAVE * tw * stride;
  const int64_t tbeg = wave * tile_arcs;
  if (tbeg >= A) return;
  const int64_t tend = tbeg + tile_arcs < A ? tbeg + tile_arcs : A;
  const int4 rbig = vlh[scal[S_LBIG]];
  auto pack = [](int4 q) { return (q.z & 0x7fffffff) | (q.w ? (int)0x80000000 : 0); };
  // Every load below is used on its own path before paths join, so no load
  // is in flight where a window begins: the compiler waits only on paths
  // that load (a wait for a load also waits for the stores in flight).
  int rb = tile_row[wave * stride];  // the row holding arc tbeg
  int e = 0, p = 0;                  // rows rb .. rb+63 (rows past n end at A)
  bool stale = true;                 // the block must be loaded at rb
  auto block = [&]() {
    const int v = rb + lane;
    e = off[v < n ? v + 1 : n];
    p = pack(vlh[v < n ? v : n - 1]);
  };
  for (int64_t base = tbeg; base < tend; base += WAVE) {
    const int64_t a64 = base + lane;
    const bool ok = a64 < tend;
    const int a = (int)(ok ? a64 : tend - 1);
    const int b = (int)base;
    const int wend = (int)(base + WAVE < tend ? base + WAVE : tend);
    unsigned long long live = __ballot(e > b);  // rows of the block ending after b
    if (stale) {
      block();
      live = __ballot(e > b);
      stale = false;
    }
    if (live == 0 || __builtin_amdgcn_readlane(e, WAVE - 1) < wend) {
      // restart the block at the row holding arc b
      while (live == 0) {
        rb += WAVE;
        block();
        live = __ballot(e > b);
      }
      rb += __builtin_ctzll(live);
      block();
      live = __ballot(e > b);
    }
    const int rp = __builtin_ctzll(live);  // block row holding arc b
    // four windows inside one row that is not exact: a 16-byte store per lane
    // (out16: the labels are 16-byte aligned; windows start at multiples of 64)
    if (out16 && base + 4 * WAVE <= tend && (int64_t)__builtin_amdgcn_readlane(e, rp) >= base + 4 * WAVE) {
      const int q4 = __builtin_amdgcn_readlane(p, rp);
      if (q4 >= 0) {
        const v4i c4 = {q4, q4, q4, q4};
        __builtin_nontemporal_store(c4, reinterpret_cast<v4i*>(out + base) + lane);
        base += 3 * WAVE;  // and the loop's own step
        continue;
      }
    }
    int pos, q, x;
    if (__builtin_amdgcn_readlane(e, rp) >= wend) {  // one row holds the whole window
      q = __builtin_amdgcn_readlane(p, rp);
      x = rb + rp;
    } else {
      const unsigned long long m = __ballot(e < wend) & (~0ull << rp);  // row ends inside
      if (__builtin_popcountll(m) > 8) {
        pos = block_count(e, a);
      } else {
        pos = rp;
        for (unsigned long long k = m; k; k &= k - 1)
          pos += a >= __builtin_amdgcn_readlane(e, __builtin_ctzll(k)) ? 1 : 0;
      }
      q = __shfl(p, pos & (WAVE - 1), WAVE);
      x = rb + pos;
      if (m >> (WAVE - 1)) {
        // more than 64 rows in the window: the rest from the offsets, then
        // the block restarts at the row of the window's last arc
        bool far = pos >= WAVE;  // every lane, so the last lane's row is known
        for (int lo = rb + WAVE; __any(far) && lo < n; lo += WAVE) {
          const int ev = off[lo + 1 + lane < n ? lo + 1 + lane : n];
          const int k = block_count(ev, a);
          if (far && k < WAVE) {
            x = lo + k;
            q = pack(vlh[x]);
            far = false;
          }
        }
        rb = __builtin_amdgcn_readlane(x, WAVE - 1);
        stale = true;
      }
    }
    int c = q & 0x7fffffff;
    if (__any(ok && q < 0)) {
      if (ok && q < 0) {
        // exact row: rx = (l[x], head(l[x]), canon(l[x]), 1)
        const int4 rx = vlh[x];
        const int y = adj[a];
        const int4 ry = ((bits[y / WAVE] >> (y % WAVE)) & 1ull) ? rbig : vlh[y];
        if (ry.x != rx.x && rx.y != y) c = ry.z;
      }
    }
    if (ok) __builtin_nontemporal_store(c, out + a64);
  }
}

// The arcs h->y of the mirror search get y's BCC.
__global__ void k_mirror_write(int n, const int4* __restrict__ vlh, const int* __restrict__ mpos,
                               const int* __restrict__ mcnt, int* __restrict__ out) {
  const int y = vertex_index();
  if (y >= n) return;
  const int a0 = mpos[y];
  if (a0 < 0) return;
  const int c = vlh[y].z, k = mcnt[y];
  for (int a = a0; a < a0 + k; ++a) out[a] = c;
}

// canon[L] = smallest arc of BCC L, made graph-local for batches (the
// largest label's was found before pass 1, which then skips its minid).
__global__ void k_bcc_canon(const int4* __restrict__ rec, const int* __restrict__ lab,
                            const int* __restrict__ minid, int n, const int* __restrict__ vbegin, int G,
                            const int* __restrict__ off, const int* __restrict__ scal, int* __restrict__ canon) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || !is_bcc_label(rec, lab, v)) return;
  if (v == scal[S_LBIG] && scal[S_CANON_BIG] >= 0) {
    canon[v] = scal[S_CANON_BIG];
    return;
  }
  int c = minid[v];
  if (G > 1) c -= off[vbegin[graph_index(vbegin, G, v)]];
  canon[v] = c;
}

// Pass 2: encoded raw label -> canonical label (elementwise, 4 arcs per
// thread); a vector holding only final labels is not written back.
__device__ __forceinline__ int resolve(int q, const int* __restrict__ canon) { return q <= -2 ? canon[-2 - q] : q; }

__global__ void k_bcc_remap4(int4* __restrict__ out, int64_t n4, const int* __restrict__ canon) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
    int4 q = out[i];
    if ((q.x | q.y | q.z | q.w) >= 0 || (q.x > -2 && q.y > -2 && q.z > -2 && q.w > -2)) continue;
    q.x = resolve(q.x, canon);
    q.y = resolve(q.y, canon);
    q.z = resolve(q.z, canon);
    q.w = resolve(q.w, canon);
    out[i] = q;
  }
}

__global__ void k_bcc_remap1(int* __restrict__ out, int64_t begin, int64_t end, const int* __restrict__ canon) {
  int64_t i = begin + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= end) return;
  out[i] = resolve(out[i], canon);
}

// BC-labeling read-out: home BCC (canonical id) and its head per vertex.
__global__ void k_vertex_labels(const int4* __restrict__ rec, const int* __restrict__ lab,
                                const int* __restrict__ head, const int* __restrict__ canon, int n,
                                const int* __restrict__ vbegin, int G, int* __restrict__ home,
                                int* __restrict__ home_head) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int c = -1, h = -1;
  if (rec[v].z >= 0) {
    const int L = lab[v];
    c = canon[L];
    h = head[L];
    if (G > 1 && h >= 0) h -= vbegin[graph_index(vbegin, G, v)];
  }
  if (home) home[v] = c;
  if (home_head) home_head[v] = h;
}

// ------------------------------------------------------------ BC labeling: labels, bridges, block-cut tree
// After a solve, from its workspace.  A BCC with exactly one edge is a bridge.
// Its two vertices are a tree edge (u, p(u)) (a bridge lies on every spanning
// tree), u is the only non-head member of the label l[u] (the label's vertex
// set plus its head is the BCC's vertex set), and the edge u-p(u) has no
// parallel copy.  mark[L] = 1 when some vertex other than L carries label L.
__global__ void k_bc_mark(const int4* __restrict__ rec, const int* __restrict__ lab, int n, int* __restrict__ mark) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || rec[v].z < 0) return;
  const int L = lab[v];
  if (L != v && ld_relaxed(mark + L) == 0) mark[L] = 1;  // idempotent store, tested first
}

// Per vertex: the paper's label l[v] and the tree parent (graph-local), the
// block-cut tree parent of a cut vertex (the BCC in which it is a non-head
// member), and, for the lone member u of a two-vertex BCC, whether u-p(u) is
// a single edge; if so, the bit of its BCC's canonical id goes into `bits`.
__global__ void k_bc_vertex(const int* __restrict__ off, const int* __restrict__ adj, const int4* __restrict__ rec,
                            const int* __restrict__ lab, const int* __restrict__ canon, const int* __restrict__ mark,
                            int n, bool sorted_rows, const int* __restrict__ vbegin, int G,
                            const int* __restrict__ edge_label, const uint8_t* __restrict__ is_ap,
                            unsigned long long* __restrict__ bits, int* __restrict__ abase,
                            int* __restrict__ out_label, int* __restrict__ out_parent,
                            int* __restrict__ out_cut_parent) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int p = rec[u].z;
  const int base = G > 1 ? vbegin[graph_index(vbegin, G, u)] : 0;
  const int ab = G > 1 ? off[base] : 0;  // first arc of u's graph: canonical ids are graph-local
  if (G > 1 && abase) abase[u] = ab;
  const int L = p >= 0 ? lab[u] : -1;
  if (out_label) out_label[u] = L >= 0 ? L - base : -1;
  if (out_parent) out_parent[u] = p >= 0 ? p - base : -1;
  if (out_cut_parent) out_cut_parent[u] = (p >= 0 && is_ap != nullptr && is_ap[u]) ? canon[L] : -1;
  if (bits == nullptr || p < 0 || L != u || mark[u] != 0) return;
  // u alone in its label: the BCC is {u, p}; a bridge iff row u holds p once
  const int b = off[u], e = off[u + 1];
  int pos = -1, copies = 0;
  if (sorted_rows) {
    int lo = b, hi = e;
    while (lo < hi) {
      const int mid = lo + ((hi - lo) >> 1);
      if (adj[mid] < p) lo = mid + 1;
      else hi = mid;
    }
    if (lo < e && adj[lo] == p) {
      pos = lo;
      copies = (lo + 1 < e && adj[lo + 1] == p) ? 2 : 1;
    }
  } else {
    for (int a = b; a < e && copies < 2; ++a)
      if (adj[a] == p) {
        pos = a;
        ++copies;
      }
  }
  if (copies == 1) {
    const int c = edge_label[pos];  // the BCC's canonical id, shared by both arcs of the edge
    if (c >= 0) atomicOr(bits + ((c + ab) >> 6), 1ull << ((c + ab) & 63));
  }
}

// Per arc: a bridge arc is one whose BCC's canonical id is marked (made
// global with the first arc of the row's graph in a batch).
template <bool BATCH>
__global__ void k_bc_bridges(const int* __restrict__ off, int n, int64_t A, const int* __restrict__ tile_row, int tw,
                             const int* __restrict__ edge_label, const int* __restrict__ abase,
                             const unsigned long long* __restrict__ bits, uint8_t* __restrict__ out) {
  if (!BATCH) {
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < A; a += (int64_t)gridDim.x * blockDim.x) {
      const int c = edge_label[a];
      out[a] = c >= 0 ? (uint8_t)((bits[c >> 6] >> (c & 63)) & 1) : 0;
    }
    return;
  }
  arc_tiles(off, n, A, tile_row, tw, [&](int64_t a, int x, bool ok) {
    if (!ok) return;
    const int c = edge_label[a];
    const int g = c + abase[x];
    out[a] = c >= 0 ? (uint8_t)((bits[g >> 6] >> (g & 63)) & 1) : 0;
  });
}

// ------------------------------------------------------------ batch input check
// Per-graph check of a batch of untrusted graphs (fastbcc_check_batched).
// Every access stays inside the arrays whatever the input holds: a row is
// read only after its bounds were found inside its graph's arc range, which
// lies inside [0, A); targets are range-checked before they index anything.
constexpr int CHECK_LANE_ROW = 256;  // longer rows are checked by a whole wave

struct GraphRange {
  int lo, hi;      // vertex range [lo, hi)
  int64_t ga, gb;  // arc range [ga, gb)
  bool ok;
};

__device__ __forceinline__ GraphRange graph_range(const int* __restrict__ off, int n, int64_t A,
                                                  const int* __restrict__ vbegin, int G, int v, int* g_out) {
  GraphRange r;
  const int g = G > 1 ? graph_index(vbegin, G, v) : 0;
  r.lo = G > 1 ? vbegin[g] : 0;
  r.hi = G > 1 ? vbegin[g + 1] : n;
  r.ga = off[r.lo];
  r.gb = off[r.hi];
  r.ok = r.ga >= 0 && r.ga <= r.gb && r.gb <= A;
  *g_out = g;
  return r;
}

// Arc a of row x (rows of x's graph are known to lie in [ga, gb)).
__device__ __forceinline__ bool arc_ok(const int* __restrict__ off, const int* __restrict__ adj, const GraphRange& r,
                                       int x, int64_t b, int64_t a, bool sorted, bool no_loops, bool symmetric) {
  const int y = adj[a];
  if (y < r.lo || y >= r.hi) return false;
  if (no_loops && y == x) return false;
  if (sorted && a > b && adj[a - 1] > y) return false;
  if (symmetric) {  // x occurs in row y (sorted rows: binary search)
    int64_t lo = off[y], hi = off[y + 1];
    lo = lo < r.ga ? r.ga : lo;
    hi = hi > r.gb ? r.gb : hi;
    const int64_t end = hi;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (adj[mid] < x) lo = mid + 1;
      else hi = mid;
    }
    if (lo >= end || adj[lo] != x) return false;
  }
  return true;
}

__global__ void k_check_rows(const int* __restrict__ off, const int* __restrict__ adj, int n, int64_t A,
                             const int* __restrict__ vbegin, int G, bool sorted, bool no_loops, bool symmetric,
                             int* __restrict__ status) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  int g = 0;
  bool bad = false, wave_row = false;
  GraphRange r{0, 0, 0, 0, false};
  int64_t b = 0, e = 0;
  if (v < n) {
    r = graph_range(off, n, A, vbegin, G, v, &g);
    b = off[v];
    e = off[v + 1];
    bad = !r.ok || b < r.ga || e > r.gb || b > e;
    if (!bad && e - b <= CHECK_LANE_ROW) {
      for (int64_t a = b; a < e; ++a)
        if (!arc_ok(off, adj, r, v, b, a, sorted, no_loops, symmetric)) {
          bad = true;
          break;
        }
    } else if (!bad) {
      wave_row = true;
    }
  }
  uint64_t big = __ballot(wave_row);
  while (big) {
    const int j = __builtin_ctzll(big);
    big &= big - 1;
    const int x = __shfl(v, j, WAVE);
    const int64_t xb = shfl64(b, j), xe = shfl64(e, j);
    GraphRange xr;
    xr.lo = __shfl(r.lo, j, WAVE);
    xr.hi = __shfl(r.hi, j, WAVE);
    xr.ga = shfl64(r.ga, j);
    xr.gb = shfl64(r.gb, j);
    xr.ok = true;
    bool lane_bad = false;
    for (int64_t a = xb + lane_id(); a < xe; a += WAVE)
      lane_bad = lane_bad || !arc_ok(off, adj, xr, x, xb, a, sorted, no_loops, symmetric);
    if (__any(lane_bad) && lane_id() == j) bad = true;
  }
  if (bad) atomicExch(status + g, (int)FASTBCC_ERR_INVALID_GRAPH);
}

// A graph that failed becomes valid in place: every arc a self-loop of its
// first vertex, its other rows empty.  One block per graph (grid-stride).
__global__ void k_repair_graphs(int* __restrict__ off, int* __restrict__ adj, int n, int64_t A,
                                const int* __restrict__ vbegin, int G, const int* __restrict__ status) {
  for (int g = blockIdx.x; g < G; g += gridDim.x) {
    if (status[g] == 0) continue;  // uniform per block
    const int lo = G > 1 ? vbegin[g] : 0, hi = G > 1 ? vbegin[g + 1] : n;
    int64_t ga = off[lo], gb = off[hi];
    ga = ga < 0 ? 0 : (ga > A ? A : ga);
    gb = gb < ga ? ga : (gb > A ? A : gb);
    __syncthreads();  // every lane has read the bounds before any row start changes
    for (int v = lo + 1 + threadIdx.x; v < hi; v += blockDim.x) off[v] = (int)gb;
    for (int64_t a = ga + threadIdx.x; a < gb; a += blockDim.x) adj[a] = lo;
  }
}

// ------------------------------------------------------------ batch assembly
// Graph-local ids and row starts made global: graph g's arcs get vbegin[g]
// added to their targets and its rows abegin[g] added to their starts.  A
// thread finds its element's graph by binary search over the (short, cached)
// range arrays.
__global__ void k_rebase_arcs(const int* __restrict__ abegin, const int* __restrict__ vbegin, int G, int64_t A,
                              int* __restrict__ adj) {
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < A; a += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = G;  // abegin[lo] <= a < abegin[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (abegin[mid] <= a) lo = mid;
      else hi = mid;
    }
    adj[a] += vbegin[lo];
  }
}

__global__ void k_rebase_rows(const int* __restrict__ abegin, const int* __restrict__ vbegin, int G, int64_t n,
                              int* __restrict__ off) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = G;  // vbegin[lo] <= v < vbegin[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (vbegin[mid] <= v) lo = mid;
      else hi = mid;
    }
    off[v] += abegin[lo];
  }
}

// int64 offsets are narrowed once (every offset is < 2^31 because arcs are).
__global__ void k_narrow_offsets(const int64_t* __restrict__ in, int64_t count, int* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (int)in[i];
}

// ------------------------------------------------------------ host driver
inline unsigned grid_for(int64_t count, int block = BLOCK) { return (unsigned)cdiv(count, block); }

// Grid of a per-vertex launch: plain, or XCD-ordered (8, per) when asked and
// the second dimension allows it.
inline dim3 vertex_grid(int64_t count, int block, bool xcd) {
  const int64_t blocks = cdiv(count, block);
  const int64_t per = cdiv(blocks, NUM_XCD);
  if (xcd && per > 0 && per <= 65535) return dim3(NUM_XCD, (unsigned)per);
  return dim3((unsigned)blocks);
}

struct Ctx {
  hipStream_t st;
  fastbcc_trace* trace = nullptr;
  bool ok = true;
  hipEvent_t pending_start = nullptr;
  void check() {
    if (hipGetLastError() != hipSuccess) ok = false;
  }
  void before() {
    pending_start = nullptr;
    if (!trace) return;
    if (trace->used + 2 > trace->pool.size()) {
      ++trace->dropped;
      return;
    }
    pending_start = trace->pool[trace->used++];
    if (hipEventRecord(pending_start, st) != hipSuccess) ok = false;
  }
  void after(const char* name) {
    if (!trace || !pending_start) return;
    hipEvent_t e = trace->pool[trace->used++];
    if (hipEventRecord(e, st) != hipSuccess) ok = false;
    trace->pending.push_back({name, pending_start, e});
    pending_start = nullptr;
  }
};

inline bool grid_nonempty(unsigned g) { return g > 0; }
inline bool grid_nonempty(dim3 g) { return g.x > 0 && g.y > 0 && g.z > 0; }
#define LAUNCH(ctx, kern, grid, block, ...)                                              \
  do {                                                                                   \
    if (grid_nonempty(grid)) {                                                           \
      (ctx).before();                                                                    \
      hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, (ctx).st, __VA_ARGS__);      \
      (ctx).check();                                                                     \
      (ctx).after(#kern);                                                                \
    }                                                                                    \
  } while (0)

void fill_i32(Ctx& c, int* p, int v, int64_t count) {
  if (count <= 0) return;
  unsigned g = grid_for(count);
  if (g > 65536) g = 65536;
  LAUNCH(c, k_fill_i32, g, BLOCK, p, v, count);
}


// Exclusive scan in place over max_count ints (count from device if given);
// the total goes to data[count] when total_out is null, else to *total_out.
void scan_inplace(Ctx& c, int* data, int64_t max_count, const int* count_dev, int* tmp, int* total_out) {
  if (max_count <= 0) return;
  const int64_t nbk = cdiv(max_count, SCAN_TILE);
  LAUNCH(c, k_scan_reduce, (unsigned)nbk, SCAN_BLOCK, data, max_count, count_dev, tmp);
  LAUNCH(c, k_scan_spine, 1, 1024, tmp, (int)nbk, total_out);
  LAUNCH(c, k_scan_down, (unsigned)nbk, SCAN_BLOCK, data, data, max_count, count_dev, tmp);
}

// The solve proper, on int32 offsets.
fastbcc_status solve_core(const Layout& L, Ctx& c, int n, int64_t A, const int* off, const int* adj, int G,
                          const int* vbegin, int* out_label, uint8_t* out_ap, int64_t* out_nbcc, char* w,
                          const Tune& tune, bool validate, bool sorted_rows, bool no_loops) {
  auto I = [&](size_t o) { return (int*)(w + o); };
  int* scal = I(L.scalars);
  const int tw = tune.tile_windows;
  const int64_t tile_arcs = (int64_t)WAVE * tw;
  const int64_t ntiles = cdiv(A, tile_arcs);
  int* tile_row = I(L.tile_row);
  const unsigned tile_grid = (unsigned)cdiv(ntiles * WAVE, BLOCK);
  LAUNCH(c, k_tile_rows, grid_for(ntiles), BLOCK, off, n, A, (const int*)nullptr, tile_arcs, tile_row);
  int *foff = I(L.foff), *frank = I(L.frank), *frow = I(L.frow), *fstart = I(L.fstart), *ftile = I(L.ftile);
  int* frows = frank + n;  // number of compacted frontier rows (scan total)
  // frontier virtual CSR of the rows a sweep still has to visit
  // in a batch the per-graph marks live in the head flags (unused until the read-out)
  uint8_t* gmark = G > 1 ? (uint8_t*)(w + L.heads) : nullptr;
  auto frontier = [&](int* comp, int slot) {
    if (gmark) {
      fill_i32(c, (int*)gmark, 0, cdiv(n, 4));  // n bytes, the allocation is padded to 256
      LAUNCH(c, k_mark_graph_modes, (unsigned)G, GRAPH_MODE_SAMPLES, comp, vbegin, n, gmark);
    }
    LAUNCH(c, k_frontier_deg, vertex_grid(n, BLOCK, tune.xcd), BLOCK, off, comp, scal, slot, n, (const uint8_t*)gmark,
           foff);
    // one scan of the degrees for both the ranks and the starts (the scratch
    // holds 2 * tiles sums: cdiv(2n + 1, SCAN_TILE) + 1 >= 2 * cdiv(n, SCAN_TILE))
    const int tiles = (int)cdiv(n, SCAN_TILE);
    int* tsum = I(L.scan_tmp);
    LAUNCH(c, k_fscan_reduce, (unsigned)tiles, SCAN_BLOCK, foff, (int64_t)n, tsum, tiles);
    LAUNCH(c, k_scan_spine, 1, 1024, tsum, tiles, foff + n);           // arcs of the frontier
    LAUNCH(c, k_scan_spine, 1, 1024, tsum + tiles, tiles, frows);      // its rows
    LAUNCH(c, k_fscan_compact, (unsigned)tiles, SCAN_BLOCK, foff, (int64_t)n, tsum, tiles, frows, foff + n, frow,
           fstart);
    LAUNCH(c, k_tile_rows, grid_for(ntiles), BLOCK, fstart, n, A, frows, tile_arcs, ftile);
  };

  if (validate) {
    int h = 0;
    LAUNCH(c, k_validate_arcs, tile_grid, BLOCK, off, adj, n, A, tile_row, tw, no_loops, vbegin, G > 1 ? G : 1,
           scal + S_STATUS);
    if (!c.ok || hipMemcpyAsync(&h, scal + S_STATUS, sizeof(int), hipMemcpyDeviceToHost, c.st) != hipSuccess ||
        hipStreamSynchronize(c.st) != hipSuccess)
      return FASTBCC_ERR_HIP;
    if (h != 0) return FASTBCC_ERR_INVALID_GRAPH;
  }

  const unsigned gn = grid_for(n);
  // the per-vertex kernels of the hot phases take the tuned block size
  const int VB = tune.vertex_block;
  const dim3 gv = vertex_grid(n, VB, tune.xcd);
  const dim3 gx = vertex_grid(n, BLOCK, tune.xcd);  // compression and frontier passes
  int* cc = I(L.cc);
  int2* hook = (int2*)(w + L.hook);

  // ---- First-CC (spanning forest)
  // the per-graph passes' largest-first order (the read-out's root labels are
  // free until then; a batch of more graphs than vertices keeps index order)
  int* gorder = (tune.graph_cc && G > 1 && vbegin != nullptr && G <= n) ? I(L.rootlab) : nullptr;
  if (gorder) LAUNCH(c, k_graph_order, 1, GORDER_THREADS, vbegin, G, n, off, gorder);
  if (tune.graph_cc && G > 1 && vbegin != nullptr) {
    LAUNCH(c, k_graph_cc, (unsigned)(G < GCC_GRID ? G : GCC_GRID), GCC_THREADS, vbegin, G, n, off, adj, cc, hook,
           scal + S_GRAPH_NEXT, (const int*)gorder);
  } else {
    if (tune.ldd) {
      int* rnd = I(L.su);  // the tree-slot array is free until Rooting
      int2* queue = (int2*)(w + L.dbits);  // A/8 bytes, free until Tagging; the queue needs < A/64
      const float beta = 1.0f / (float)(1 << tune.ldd);
      const int T0 = (int)ceil(log((double)(n > 2 ? n : 2)) / beta);
      LAUNCH(c, k_ldd_init, gn, BLOCK, cc, hook, rnd, n, scal);
      for (int r = 0; r <= T0; ++r) {
        LAUNCH(c, k_ldd_round, gn, BLOCK, off, adj, n, r, T0, 1.0f / beta, cc, rnd, hook, queue, scal);
        LAUNCH(c, k_ldd_huge, LDD_HUGE_GRID, BLOCK, off, adj, r, queue, scal, cc, rnd, hook);
      }
    } else if (!(tune.first_round_free && tune.sample_rounds > 0)) {
      LAUNCH(c, k_cc_init, gn, BLOCK, cc, hook, n);  // else the atomic-free round initialises
    }
    // compress after every round: the next round's finds then take one hop
    for (int r = 0; r < tune.sample_rounds; ++r) {
      const bool free_round = r == 0 && tune.first_round_free && !tune.ldd;
      if (free_round) {
        if (tune.cc_prio) LAUNCH(c, k_cc_first_round<true>, gv, VB, off, adj, n, cc, hook);
        else LAUNCH(c, k_cc_first_round<false>, gv, VB, off, adj, n, cc, hook);
      } else if (tune.cc_prio) {
        LAUNCH(c, k_cc_sample<true>, gv, VB, off, adj, n, r, cc, hook);
      } else {
        LAUNCH(c, k_cc_sample<false>, gv, VB, off, adj, n, r, cc, hook);
      }
      // flattened for the next round, except after the atomic-free round (its
      // chains are short and the next round's finds walk them anyway) and
      // after the last one (the frontier pass flattens)
      if ((!free_round || tune.compress_free) && r + 1 < tune.sample_rounds) LAUNCH(c, k_compress, gx, BLOCK, cc, n);
    }
    LAUNCH(c, k_pick_mode, 1, MODE_SAMPLES, cc, n, scal + S_BIG_CC);
    frontier(cc, S_BIG_CC);
    if (tune.cc_prio)
      LAUNCH(c, k_cc_sweep<true>, tile_grid, BLOCK, off, frow, fstart, adj, frows, ftile, tw, cc, hook);
    else
      LAUNCH(c, k_cc_sweep<false>, tile_grid, BLOCK, off, frow, fstart, adj, frows, ftile, tw, cc, hook);
  }
  // (Rooting's first pass flattens the sets)

  // ---- Rooting
  int *eid = I(L.toff), *eu = I(L.su), *ev = I(L.sv), *headp = I(L.tadj), *nxt = I(L.twin);
  int *rootidx = I(L.rootidx), *roots = I(L.roots), *next = I(L.next), *tmp = I(L.scan_tmp);
  int *hubidx = I(L.hubidx), *shard = I(L.shard);
  fill_i32(c, shard, -1, L.hubs * HUB_SHARDS);
  unsigned long long* hubbits = (unsigned long long*)(w + L.bigbits);  // free until the read-out
  LAUNCH(c, k_edge_flags, gx, BLOCK, off, hook, n, cc, eid, headp, hubidx, scal, hubbits);
  LAUNCH(c, k_flatten, gx, BLOCK, cc, n);  // Rooting reads cc[v] as the component id
  scan_inplace(c, eid, n, nullptr, tmp, eid + n);
  LAUNCH(c, k_edge_compact, gx, BLOCK, hook, eid, n, eu, ev);
  const int64_t arcs_max = 2 * (int64_t)n;  // 2T <= 2n - 2
  // plain order: its atomics gain nothing from one XCD's L2 and lose issue
  // rate when one graph's all land there
  LAUNCH(c, k_tree_link, grid_for(arcs_max), BLOCK, (const unsigned long long*)hubbits, hubidx, eid, n, eu, ev, headp,
         shard, nxt);
  int* lone = I(L.frank);  // free from here until Last-CC's frontier rewrites its row count (frank[n])
  int *rdeg = I(L.pos), *rsel = I(L.eflag);  // free until list ranking
  LAUNCH(c, k_hub_lists, gx, BLOCK, off, hubidx, cc, n, headp, shard, rootidx, lone, rdeg);
  scan_inplace(c, rootidx, n, nullptr, tmp, rootidx + n);
  scan_inplace(c, lone, n, nullptr, tmp, lone + n);
  LAUNCH(c, k_root_degree, grid_for(ROOT_SAMPLES, ROOT_BLOCK), ROOT_BLOCK, off, cc, n, rdeg);
  LAUNCH(c, k_root_select, grid_for(ROOT_SAMPLES), BLOCK, off, cc, n, rdeg, rsel);
  LAUNCH(c, k_root_list, gx, BLOCK, cc, headp, rootidx, rdeg, rsel, scal, n, roots);
  const int64_t nodes_max = 2 * (int64_t)n;  // C + 2T <= 2n - 1
  const dim3 gnode = vertex_grid(nodes_max, BLOCK, tune.xcd);
  LAUNCH(c, k_euler_next, gnode, BLOCK, (const unsigned long long*)hubbits, hubidx, eid, eu, ev, headp, shard, nxt, cc,
         rootidx, roots, n, next);

  // list ranking: ruling set + pointer jumping over rulers
  const int sh = tune.ruler_shift;
  const int64_t rmax = cdiv(nodes_max, int64_t(1) << sh);
  int2* ol = (int2*)(w + L.ol);
  int *rlen = I(L.rlen), *rnext = I(L.rnext);
  LAUNCH(c, k_lr_walk, vertex_grid(rmax, BLOCK, tune.xcd), BLOCK, next, rootidx, eid, n, sh, ol, rnext, rlen);
  int* bufv[2] = {I(L.rval0), I(L.rval1)};
  int* bufn[2] = {I(L.rnx0), I(L.rnx1)};
  auto jump = [&](const int* vin, const int* nin, int shift, int64_t count) {  // suffix sums
    const int rounds = ilog2_floor(count) + 1;  // 2^rounds > ruler count
    for (int k = 0; k < rounds; ++k) {
      LAUNCH(c, k_lr_jump, grid_for(count), BLOCK, rootidx, eid, n, shift, vin, nin, bufv[k & 1], bufn[k & 1]);
      vin = bufv[k & 1];
      nin = bufn[k & 1];
    }
    return vin;
  };
  const int* rsuf;  // suffix sums of the rulers' segment lengths
  if (rmax >= LR2_MIN_RULERS) {
    // a second ruling level over the rulers, then pointer jumping over its rulers
    const int sh2 = LR2_SHIFT;
    const int64_t rmax2 = cdiv(rmax, int64_t(1) << sh2);
    int2* ol2 = (int2*)(w + L.ol2);
    int *rnext2 = I(L.rnext2), *rlen2 = I(L.rlen2);
    LAUNCH(c, k_lr_walk2, grid_for(rmax2), BLOCK, rootidx, eid, n, sh, sh2, rnext, rlen, ol2, rnext2, rlen2);
    const int* suf2 = jump(rlen2, rnext2, sh + sh2, rmax2);
    LAUNCH(c, k_lr_suf, grid_for(rmax), BLOCK, rootidx, eid, n, sh, sh2, ol2, suf2, rlen, scal + S_STATUS);
    rsuf = rlen;
  } else {
    rsuf = jump(rlen, rnext, sh, rmax);
  }
  int* pos = I(L.pos);
  int* eflag = I(L.eflag);
  LAUNCH(c, k_lr_pos, gnode, BLOCK, rootidx, eid, n, sh, ol, rsuf, pos, scal + S_STATUS);
  LAUNCH(c, k_enter_flags, gnode, BLOCK, rootidx, eid, n, pos, eflag, scal + S_STATUS);
  int* nl_dev = scal + S_NODES;  // number of list nodes, for the scan of entry flags
  LAUNCH(c, k_node_count, 1, 1, rootidx, eid, n, nl_dev);
  scan_inplace(c, eflag, nodes_max, nl_dev, tmp, scal + S_ENTRIES);

  // ---- Tagging
  int *first = I(L.first), *w1 = I(L.w1), *w2 = I(L.w2);
  int4* rec = (int4*)(w + L.rec);
  LAUNCH(c, k_tags, gnode, BLOCK, rootidx, roots, eid, eu, ev, lone, n, pos, eflag, first, rec, scal + S_STATUS);
  unsigned long long* dbits = (unsigned long long*)(w + L.dbits);
  int4* W = (int4*)(w + L.W);
  int2 *pre = (int2*)(w + L.pre), *suf = (int2*)(w + L.suf), *tab = (int2*)(w + L.tab);
  auto rmq_tables = [&](const uint8_t* only) {
    LAUNCH(c, k_rmq_block, (unsigned)cdiv(L.nb * WAVE, BLOCK), BLOCK, W, n, L.nb, only, pre, suf, tab);
    for (int j = 1; j < L.levels; j += 2)
      LAUNCH(c, k_rmq_level, grid_for(L.nb), BLOCK, tab, L.nb, j, j + 1 < L.levels);
  };
  if (!tune.sampled_tags) {
    LAUNCH(c, k_tag_init, gx, BLOCK, lone, n, first, rec, w1, w2);
    LAUNCH(c, k_tag_sweep, tile_grid, BLOCK, off, adj, n, A, tile_row, tw, first, rec, w1, w2, dbits);
    LAUNCH(c, k_rmq_scatter, gx, BLOCK, first, w1, w2, n, W, scal + S_STATUS);
    rmq_tables(nullptr);
    LAUNCH(c, k_rmq_query, gv, VB, n, L.nb, W, pre, suf, tab, rec, (int)QUERY_EXACT, true, (int*)nullptr,
           scal + S_STATUS);
  } else {
    // sampled tags certify most non-fences; exact tags for the subtrees of the
    // undecided vertices only
    int* cover = eflag;  // difference array over preorder slots (2n + 1 >= n + 2 ints)
    LAUNCH(c, k_tag_sample, gv, VB, off, adj, lone, first, rec, n, tune.tag_samples, W, cover, scal,
           scal + S_STATUS);
    rmq_tables(nullptr);
    LAUNCH(c, k_rmq_query, gv, VB, n, L.nb, W, pre, suf, tab, rec, (int)QUERY_CERTIFY, true, cover,
           scal + S_STATUS);
    scan_inplace(c, cover, (int64_t)n + 1, nullptr, tmp, cover + n + 1);
    int* dirty = w1;  // rows listed for exact tags (w1/w2 are unused with sampled tags)
    LAUNCH(c, k_dirty_list, gn, BLOCK, off, W, cover, n, tune.tag_samples, dirty, scal + S_DIRTY);
    uint8_t* dirty_block = (uint8_t*)(w + L.heads);  // nb <= n bytes, unused until the read-out
    fill_i32(c, (int*)dirty_block, 0, cdiv(L.nb, 4));
    LAUNCH(c, k_tag_rows, TAG_ROWS_GRID, BLOCK, off, adj, dirty, scal + S_DIRTY, first, W, dirty_block);
    rmq_tables(dirty_block);
    LAUNCH(c, k_rmq_query, gv, VB, n, L.nb, W, pre, suf, tab, rec, (int)QUERY_RECHECK, true, cover,
           scal + S_STATUS);
  }

  // ---- Last-CC on the implicit skeleton
  int* lab = I(L.lab);
  if (tune.graph_cc && G > 1 && vbegin != nullptr) {
    LAUNCH(c, k_graph_lcc, (unsigned)(G < GCC_GRID ? G : GCC_GRID), GCC_THREADS, vbegin, G, n, off, adj,
           (const int4*)rec, lab, scal + S_GRAPH_NEXT_LCC, (const int*)gorder);
    LAUNCH(c, k_flatten, gx, BLOCK, lab, n);  // graphs above the LDS size leave chains
    LAUNCH(c, k_pick_mode, 1, MODE_SAMPLES, lab, n, scal + S_BIG_LAB);
  } else {
    if (tune.lcc_prio) {
      LAUNCH(c, k_lcc_tree_free<true>, gv, VB, rec, n, lab);
      LAUNCH(c, k_lcc_tree<true>, gv, VB, rec, n, lab);
    } else {
      LAUNCH(c, k_lcc_tree_free<false>, gv, VB, rec, n, lab);
      LAUNCH(c, k_lcc_tree<false>, gv, VB, rec, n, lab);
    }
    // flattened before each sampling round; the frontier pass flattens the last state
    const int lcc_rounds = tune.lcc_rounds < 0 ? tune.sample_rounds : tune.lcc_rounds;
    for (int r = 0; r < lcc_rounds; ++r) {
      LAUNCH(c, k_compress, gx, BLOCK, lab, n);
      if (tune.lcc_prio) LAUNCH(c, k_lcc_sample<true>, gv, VB, off, adj, rec, n, r, lab);
      else LAUNCH(c, k_lcc_sample<false>, gv, VB, off, adj, rec, n, r, lab);
    }
    LAUNCH(c, k_pick_mode, 1, MODE_SAMPLES, lab, n, scal + S_BIG_LAB);
    frontier(lab, S_BIG_LAB);
    if (tune.lcc_prio)
      LAUNCH(c, k_lcc_sweep<true>, tile_grid, BLOCK, off, frow, fstart, adj, frows, ftile, tw, rec, lab);
    else
      LAUNCH(c, k_lcc_sweep<false>, tile_grid, BLOCK, off, frow, fstart, adj, frows, ftile, tw, rec, lab);
    LAUNCH(c, k_compress, gx, BLOCK, lab, n);
    LAUNCH(c, k_flatten, gx, BLOCK, lab, n);  // the relabelling and the read-out read lab[v] as the label
    if (tune.lcc_prio) {
      int* minv = I(L.minid);  // refilled by the read-out
      fill_i32(c, minv, INT32_MAX, n);
      int* part = I(L.bsum);  // cdiv(n, BLOCK) + 1 slots, used again by the BCC count
      LAUNCH(c, k_big_min_part, gn, BLOCK, lab, n, scal, part);
      LAUNCH(c, k_big_min, 1, 1024, lab, part, (int)gn, scal);
      LAUNCH(c, k_label_min, gn, BLOCK, lab, n, scal, minv);
      LAUNCH(c, k_relabel, gn, BLOCK, lab, n, scal, minv);
    }
  }

  // ---- heads, articulation points, canonical labels
  int *head = I(L.head), *rootlab = I(L.rootlab), *minid = I(L.minid), *canon = I(L.canon), *bsum = I(L.bsum);
  uint8_t* heads = (uint8_t*)(w + L.heads);
  LAUNCH(c, k_readout_init, gx, BLOCK, n, head, heads, rootlab, minid, out_ap);
  LAUNCH(c, k_bcc_heads, gn, BLOCK, rec, lab, n, head, heads, rootlab, out_ap, out_nbcc ? bsum : nullptr);
  if (out_nbcc) {
    if (G <= 1) {
      LAUNCH(c, k_sum_blocks, grid_for(gn, 1024 * SUM_PER_LANE), 1024, bsum, (int)gn, out_nbcc);
    } else {
      // exclusive scan with the total in bsum[gn]: a graph that ends on the
      // last block boundary (n a multiple of BLOCK) reads P[gn]
      scan_inplace(c, bsum, gn, nullptr, I(L.scan_tmp), bsum + gn);
      LAUNCH(c, k_graph_count, grid_for((int64_t)G * WAVE), BLOCK, rec, lab, n, vbegin, G, bsum, out_nbcc);
    }
  }
  unsigned long long* bigbits = (unsigned long long*)(w + L.bigbits);
  LAUNCH(c, k_lbig, 1, 1, lab, scal);
  LAUNCH(c, k_big_bitmap, (unsigned)cdiv((int64_t)n, BLOCK), BLOCK, lab, n, scal, bigbits);
  LAUNCH(c, k_big_canon, 1, BLOCK, off, adj, rec, lab, head, heads, vbegin, G, scal);
  int4* vlh = (int4*)(w + L.ol);  // the list-ranking array (16n + 8 bytes) is dead by now
  LAUNCH(c, k_vertex_lh, gv, VB, lab, head, heads, rec, scal, n, vlh);
  if (sorted_rows) {
    // canonical labels first, then every arc once with its final label
    int *mpos = I(L.w1), *mcnt = I(L.w2);  // tags are done
    LAUNCH(c, k_mirror_find, gv, VB, off, adj, n, vlh, scal, minid, mpos, mcnt);
    fill_i32(c, canon, -1, n);
    LAUNCH(c, k_canon_first, gv, VB, off, adj, n, rec, lab, vlh, heads, bigbits, scal, minid, vbegin, G, canon);
    LAUNCH(c, k_vertex_canon, gx, BLOCK, canon, n, vlh);
    if (no_loops) {
      const int stride = tw >= ROWS_TILE_WINDOWS ? 1 : ROWS_TILE_WINDOWS / tw;
      const unsigned rows_grid = (unsigned)cdiv(cdiv(ntiles, stride) * WAVE, BLOCK);
      const bool out16 = ((uintptr_t)out_label & 15) == 0;
      LAUNCH(c, k_bcc_rows, rows_grid, BLOCK, off, adj, n, A, tile_row, tw, stride, vlh, bigbits, scal, out16,
             out_label);
    } else {
      LAUNCH(c, k_bcc_final, tile_grid, BLOCK, off, adj, n, A, tile_row, tw, vlh, bigbits, scal, out_label);
    }
    LAUNCH(c, k_mirror_write, gx, BLOCK, n, vlh, mpos, mcnt, out_label);
    return c.ok ? FASTBCC_OK : FASTBCC_ERR_HIP;
  }
  if (!tune.sampled_tags)
    LAUNCH(c, k_bcc_label<LABEL_DBITS>, tile_grid, BLOCK, off, adj, n, A, tile_row, tw, vlh, heads, bigbits, dbits,
           head, scal, minid, out_label);
  else
    LAUNCH(c, k_bcc_label<LABEL_BITMAP>, tile_grid, BLOCK, off, adj, n, A, tile_row, tw, vlh, heads, bigbits, dbits,
           head, scal, minid, out_label);
  LAUNCH(c, k_bcc_canon, gn, BLOCK, rec, lab, minid, n, vbegin, G, off, scal, canon);
  if (A > 0) {
    if (((uintptr_t)out_label & 15) == 0) {
      const int64_t n4 = A / 4;
      unsigned g4 = grid_for(n4);
      if (g4 > 65536) g4 = 65536;
      LAUNCH(c, k_bcc_remap4, g4, BLOCK, (int4*)out_label, n4, canon);
      LAUNCH(c, k_bcc_remap1, grid_for(A - 4 * n4), BLOCK, out_label, 4 * n4, A, canon);
    } else {
      LAUNCH(c, k_bcc_remap1, grid_for(A), BLOCK, out_label, (int64_t)0, A, canon);
    }
  }
  return c.ok ? FASTBCC_OK : FASTBCC_ERR_HIP;
}

template <typename OffT>
fastbcc_status solve_impl(int64_t n64, int64_t A, const OffT* off, const int* adj, int G, const int* vbegin,
                          int* out_label, uint8_t* out_ap, int64_t* out_nbcc, void* ws, size_t ws_bytes,
                          uint32_t flags, hipStream_t st, fastbcc_trace* trace = nullptr) {
  Tune tune;
  if (!decode_flags(flags, tune)) return FASTBCC_ERR_INVALID_ARGUMENT;
  if (n64 < 0 || A < 0) return FASTBCC_ERR_INVALID_ARGUMENT;
  if (n64 >= (int64_t(1) << 30) || A >= (int64_t(1) << 31)) return FASTBCC_ERR_TOO_LARGE;
  if (n64 > 0 && off == nullptr) return FASTBCC_ERR_INVALID_ARGUMENT;
  if (A > 0 && (adj == nullptr || out_label == nullptr)) return FASTBCC_ERR_INVALID_ARGUMENT;
  if (G > 1 && vbegin == nullptr) return FASTBCC_ERR_INVALID_ARGUMENT;
  const Layout L = make_layout(n64, A);
  if (ws == nullptr || ws_bytes < L.total) return FASTBCC_ERR_WORKSPACE_TOO_SMALL;
  if (((uintptr_t)ws & 255) != 0) return FASTBCC_ERR_INVALID_ARGUMENT;

  Ctx c{st, trace};
  char* w = (char*)ws;
  int* scal = (int*)(w + L.scalars);
  const int n = (int)n64;
  const int GG = G < 1 ? 1 : G;

  fill_i32(c, scal, 0, S_COUNT);
  if (out_nbcc) {
    LAUNCH(c, k_fill_i64, 1, BLOCK, out_nbcc, (int64_t)0, (int64_t)GG);
  }
  if (n == 0) return c.ok ? FASTBCC_OK : FASTBCC_ERR_HIP;

  const bool validate = (flags & FASTBCC_FLAG_VALIDATE) != 0;
  const bool sorted_rows = (flags & FASTBCC_FLAG_SORTED_ROWS) != 0;
  const bool no_loops = (flags & FASTBCC_FLAG_NO_SELF_LOOPS) != 0;
  if (validate) {
    LAUNCH(c, k_validate_rows<OffT>, grid_for(n64 + 1), BLOCK, off, n, A, scal + S_STATUS);
    if (GG > 1) LAUNCH(c, k_validate_vbegin, grid_for((int64_t)GG + 1), BLOCK, vbegin, GG, n, scal + S_STATUS);
    int h = 0;
    if (!c.ok || hipMemcpyAsync(&h, scal + S_STATUS, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return FASTBCC_ERR_HIP;
    if (h != 0) return FASTBCC_ERR_INVALID_GRAPH;
  }
  const int* off32;
  if (sizeof(OffT) == 8) {
    int* o = (int*)(w + L.off32);
    unsigned g = grid_for(n64 + 1);
    if (g > 65536) g = 65536;
    LAUNCH(c, k_narrow_offsets, g, BLOCK, (const int64_t*)off, n64 + 1, o);
    off32 = o;
  } else {
    off32 = (const int*)off;
  }
  return solve_core(L, c, n, A, off32, adj, G, vbegin, out_label, out_ap, out_nbcc, w, tune, validate, sorted_rows,
                    no_loops);
}

}  // namespace

// ------------------------------------------------------------ allocation-free entry point
// Workspace of fastbcc_solve_noalloc: one static array per GPU, living as long
// as the process.  In host code `scratch` names only a host-side stand-in;
// its device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[FASTBCC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of the current device's scratch, looked up on the first
// call made with that device current.
fastbcc_status scratch_for_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return FASTBCC_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return FASTBCC_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FASTBCC_OK;
}

}  // namespace

extern "C" {

fastbcc_status fastbcc_workspace_size(int64_t n, int64_t num_arcs, int32_t num_graphs, size_t* bytes) {
  if (bytes == nullptr || n < 0 || num_arcs < 0 || num_graphs < 0) return FASTBCC_ERR_INVALID_ARGUMENT;
  if (n >= (int64_t(1) << 30) || num_arcs >= (int64_t(1) << 31)) return FASTBCC_ERR_TOO_LARGE;
  *bytes = make_layout(n, num_arcs).total;
  return FASTBCC_OK;
}

fastbcc_status fastbcc_solve(int64_t n, int64_t num_arcs, const int32_t* offsets, const int32_t* adj,
                             int32_t* out_edge_label, uint8_t* out_is_ap, int64_t* out_num_bcc, void* workspace,
                             size_t workspace_bytes, uint32_t flags, void* stream) {
  return solve_impl<int>(n, num_arcs, offsets, adj, 1, nullptr, out_edge_label, out_is_ap, out_num_bcc, workspace,
                         workspace_bytes, flags, (hipStream_t)stream);
}

fastbcc_status fastbcc_solve_noalloc(int64_t n, int64_t num_arcs, const int32_t* offsets, const int32_t* adj,
                                     int32_t* out_edge_label, uint8_t* out_is_ap, int64_t* out_num_bcc,
                                     uint32_t flags, void* stream) {
  if (n < 0 || num_arcs < 0) return FASTBCC_ERR_INVALID_ARGUMENT;
  if (n >= (int64_t(1) << 30) || num_arcs >= (int64_t(1) << 31)) return FASTBCC_ERR_TOO_LARGE;
  if (make_layout(n, num_arcs).total > (size_t)FASTBCC_NOALLOC_SCRATCH_BYTES) return FASTBCC_ERR_SCRATCH_TOO_SMALL;
  void* ws = nullptr;
  const fastbcc_status s = scratch_for_current_device(&ws);
  if (s != FASTBCC_OK) return s;
  return solve_impl<int>(n, num_arcs, offsets, adj, 1, nullptr, out_edge_label, out_is_ap, out_num_bcc, ws,
                         (size_t)FASTBCC_NOALLOC_SCRATCH_BYTES, flags, (hipStream_t)stream);
}

fastbcc_status fastbcc_solve_off64(int64_t n, int64_t num_arcs, const int64_t* offsets, const int32_t* adj,
                                   int32_t* out_edge_label, uint8_t* out_is_ap, int64_t* out_num_bcc,
                                   void* workspace, size_t workspace_bytes, uint32_t flags, void* stream) {
  return solve_impl<int64_t>(n, num_arcs, offsets, adj, 1, nullptr, out_edge_label, out_is_ap, out_num_bcc,
                             workspace, workspace_bytes, flags, (hipStream_t)stream);
}

fastbcc_status fastbcc_solve_batched(int32_t num_graphs, const int32_t* graph_vbegin, int64_t n_total,
                                     int64_t num_arcs, const int32_t* offsets, const int32_t* adj,
                                     int32_t* out_edge_label, uint8_t* out_is_ap, int64_t* out_num_bcc,
                                     void* workspace, size_t workspace_bytes, uint32_t flags, void* stream) {
  if (num_graphs < 1 || graph_vbegin == nullptr) return FASTBCC_ERR_INVALID_ARGUMENT;
  return solve_impl<int>(n_total, num_arcs, offsets, adj, num_graphs, graph_vbegin, out_edge_label, out_is_ap,
                         out_num_bcc, workspace, workspace_bytes, flags, (hipStream_t)stream);
}

fastbcc_status fastbcc_vertex_labels(int64_t n, int64_t num_arcs, int32_t num_graphs, const int32_t* graph_vbegin,
                                     const void* workspace, size_t workspace_bytes, int32_t* out_home,
                                     int32_t* out_home_head, void* stream) {
  if (n < 0 || num_arcs < 0 || num_graphs < 1 || (num_graphs > 1 && graph_vbegin == nullptr))
    return FASTBCC_ERR_INVALID_ARGUMENT;
  if (n >= (int64_t(1) << 30) || num_arcs >= (int64_t(1) << 31)) return FASTBCC_ERR_TOO_LARGE;
  const Layout L = make_layout(n, num_arcs);
  if (workspace == nullptr || workspace_bytes < L.total) return FASTBCC_ERR_WORKSPACE_TOO_SMALL;
  if (n == 0 || (out_home == nullptr && out_home_head == nullptr)) return FASTBCC_OK;
  const char* w = (const char*)workspace;
  Ctx c{(hipStream_t)stream};
  LAUNCH(c, k_vertex_labels, grid_for(n), BLOCK, (const int4*)(w + L.rec), (const int*)(w + L.lab),
         (const int*)(w + L.head), (const int*)(w + L.canon), (int)n, graph_vbegin, num_graphs, out_home,
         out_home_head);
  return c.ok ? FASTBCC_OK : FASTBCC_ERR_HIP;
}

fastbcc_status fastbcc_bc_labeling(int64_t n, int64_t num_arcs, int32_t num_graphs, const int32_t* graph_vbegin,
                                   const void* offsets, int32_t offsets_bits, const int32_t* adj,
                                   const int32_t* edge_label, const uint8_t* is_ap, void* workspace,
                                   size_t workspace_bytes, uint32_t flags, int32_t* out_label, int32_t* out_parent,
                                   int32_t* out_cut_parent, uint8_t* out_is_bridge, void* stream) {
  if (n < 0 || num_arcs < 0 || num_graphs < 1 || (num_graphs > 1 && graph_vbegin == nullptr))
    return FASTBCC_ERR_INVALID_ARGUMENT;
  if (offsets_bits != 32 && offsets_bits != 64) return FASTBCC_ERR_INVALID_ARGUMENT;
  if (n >= (int64_t(1) << 30) || num_arcs >= (int64_t(1) << 31)) return FASTBCC_ERR_TOO_LARGE;
  const Layout L = make_layout(n, num_arcs);
  if (workspace == nullptr || workspace_bytes < L.total) return FASTBCC_ERR_WORKSPACE_TOO_SMALL;
  if (((uintptr_t)workspace & 255) != 0) return FASTBCC_ERR_INVALID_ARGUMENT;
  const bool bridges = out_is_bridge != nullptr && num_arcs > 0;
  if (n > 0 && offsets == nullptr) return FASTBCC_ERR_INVALID_ARGUMENT;
  if (bridges && (adj == nullptr || edge_label == nullptr)) return FASTBCC_ERR_INVALID_ARGUMENT;
  if (out_cut_parent != nullptr && n > 0 && is_ap == nullptr) return FASTBCC_ERR_INVALID_ARGUMENT;
  if (n == 0) return FASTBCC_OK;
  char* w = (char*)workspace;
  Ctx c{(hipStream_t)stream};
  const int nn = (int)n;
  const int* off32 = (const int*)offsets;
  if (offsets_bits == 64) {  // narrowed into the workspace, as the solve does
    int* o = (int*)(w + L.off32);
    unsigned g = grid_for(n + 1);
    if (g > 65536) g = 65536;
    LAUNCH(c, k_narrow_offsets, g, BLOCK, (const int64_t*)offsets, n + 1, o);
    off32 = o;
  }
  // arrays of the solve's tagging phase serve as scratch here: the read-out
  // state that the BC labeling reads (records, labels, heads, canonical ids)
  // is left as the solve left it
  int* mark = (int*)(w + L.w1);
  int* abase = (int*)(w + L.w2);
  unsigned long long* bits = (unsigned long long*)(w + L.dbits);  // one bit per arc
  if (bridges) {
    fill_i32(c, mark, 0, n);
    fill_i32(c, (int*)bits, 0, 2 * cdiv(num_arcs, 64));
    LAUNCH(c, k_bc_mark, grid_for(n), BLOCK, (const int4*)(w + L.rec), (const int*)(w + L.lab), nn, mark);
  }
  LAUNCH(c, k_bc_vertex, grid_for(n), BLOCK, off32, adj, (const int4*)(w + L.rec), (const int*)(w + L.lab),
         (const int*)(w + L.canon), (const int*)mark, nn, (flags & FASTBCC_FLAG_SORTED_ROWS) != 0, graph_vbegin,
         (int)num_graphs, edge_label, is_ap, bridges ? bits : nullptr, abase, out_label, out_parent, out_cut_parent);
  if (bridges) {
    if (num_graphs > 1) {
      constexpr int tw = MIN_TILE_ARCS / WAVE;  // the tile array holds tiles of at least this many arcs
      int* tile_row = (int*)(w + L.tile_row);
      const int64_t ntiles = cdiv(num_arcs, (int64_t)WAVE * tw);
      LAUNCH(c, k_tile_rows, grid_for(ntiles), BLOCK, off32, nn, num_arcs, (const int*)nullptr, (int64_t)WAVE * tw,
             tile_row);
      LAUNCH(c, k_bc_bridges<true>, (unsigned)cdiv(ntiles * WAVE, BLOCK), BLOCK, off32, nn, num_arcs,
             (const int*)tile_row, tw, edge_label, (const int*)abase, (const unsigned long long*)bits, out_is_bridge);
    } else {
      unsigned g = grid_for(num_arcs);
      if (g > 65536) g = 65536;
      LAUNCH(c, k_bc_bridges<false>, g, BLOCK, off32, nn, num_arcs, (const int*)nullptr, 0, edge_label,
             (const int*)nullptr, (const unsigned long long*)bits, out_is_bridge);
    }
  }
  return c.ok ? FASTBCC_OK : FASTBCC_ERR_HIP;
}

fastbcc_status fastbcc_check_batched(int32_t num_graphs, const int32_t* graph_vbegin, int64_t n, int64_t num_arcs,
                                     int32_t* offsets, int32_t* adj, uint32_t flags, int32_t* out_graph_status,
                                     void* stream) {
  if (n < 0 || num_arcs < 0 || num_graphs < 1 || (num_graphs > 1 && graph_vbegin == nullptr) ||
      out_graph_status == nullptr)
    return FASTBCC_ERR_INVALID_ARGUMENT;
  if (n >= (int64_t(1) << 30) || num_arcs >= (int64_t(1) << 31)) return FASTBCC_ERR_TOO_LARGE;
  const uint32_t known = FASTBCC_FLAG_VALIDATE | FASTBCC_FLAG_SORTED_ROWS | FASTBCC_FLAG_NO_SELF_LOOPS |
                         FASTBCC_FLAG_REPAIR;
  if (flags & ~known) return FASTBCC_ERR_INVALID_ARGUMENT;
  const bool sorted = (flags & FASTBCC_FLAG_SORTED_ROWS) != 0;
  const bool symmetric = (flags & FASTBCC_FLAG_VALIDATE) != 0;
  if (symmetric && !sorted) return FASTBCC_ERR_INVALID_ARGUMENT;  // the symmetry test searches sorted rows
  if (offsets == nullptr || (num_arcs > 0 && adj == nullptr)) return FASTBCC_ERR_INVALID_ARGUMENT;
  Ctx c{(hipStream_t)stream};
  fill_i32(c, out_graph_status, 0, num_graphs);
  if (n > 0) {
    LAUNCH(c, k_check_rows, grid_for(n), BLOCK, (const int*)offsets, (const int*)adj, (int)n, num_arcs, graph_vbegin,
           (int)num_graphs, sorted, (flags & FASTBCC_FLAG_NO_SELF_LOOPS) != 0, symmetric, out_graph_status);
    if (flags & FASTBCC_FLAG_REPAIR) {
      const unsigned blocks = num_graphs < 65535 ? (unsigned)num_graphs : 65535u;
      LAUNCH(c, k_repair_graphs, blocks, BLOCK, offsets, adj, (int)n, num_arcs, graph_vbegin, (int)num_graphs,
             (const int*)out_graph_status);
    }
  }
  return c.ok ? FASTBCC_OK : FASTBCC_ERR_HIP;
}

fastbcc_status fastbcc_batch_rebase(int32_t num_graphs, const int32_t* graph_vbegin, const int32_t* graph_abegin,
                                    int64_t n, int64_t num_arcs, int32_t* offsets, int32_t* adj, void* stream) {
  if (num_graphs < 1 || n < 0 || num_arcs < 0 || graph_vbegin == nullptr || graph_abegin == nullptr)
    return FASTBCC_ERR_INVALID_ARGUMENT;
  if ((n > 0 && offsets == nullptr) || (num_arcs > 0 && adj == nullptr)) return FASTBCC_ERR_INVALID_ARGUMENT;
  if (n >= (int64_t(1) << 30) || num_arcs >= (int64_t(1) << 31)) return FASTBCC_ERR_TOO_LARGE;
  Ctx c{(hipStream_t)stream};
  if (num_arcs > 0) {
    unsigned g = grid_for(num_arcs);
    if (g > 65536) g = 65536;
    LAUNCH(c, k_rebase_arcs, g, BLOCK, graph_abegin, graph_vbegin, (int)num_graphs, num_arcs, adj);
  }
  if (n > 0) {
    unsigned g = grid_for(n);
    if (g > 65536) g = 65536;
    LAUNCH(c, k_rebase_rows, g, BLOCK, graph_abegin, graph_vbegin, (int)num_graphs, n, offsets);
  }
  return c.ok ? FASTBCC_OK : FASTBCC_ERR_HIP;
}

fastbcc_status fastbcc_read_device_status(const void* workspace, void* stream, int32_t* out_status) {
  if (workspace == nullptr || out_status == nullptr) return FASTBCC_ERR_INVALID_ARGUMENT;
  hipStream_t st = (hipStream_t)stream;
  const int* scal = (const int*)workspace;  // scalars sit at offset 0
  int h = 0;
  if (hipMemcpyAsync(&h, scal + S_STATUS, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return FASTBCC_ERR_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return FASTBCC_ERR_HIP;
  *out_status = h;
  return FASTBCC_OK;
}

fastbcc_status fastbcc_solve_traced(int32_t num_graphs, const int32_t* graph_vbegin, int64_t n, int64_t num_arcs,
                                    const void* offsets, int32_t offsets_bits, const int32_t* adj,
                                    int32_t* out_edge_label, uint8_t* out_is_ap, int64_t* out_num_bcc, void* workspace,
                                    size_t workspace_bytes, uint32_t flags, void* stream, fastbcc_trace* trace) {
  if (num_graphs < 1 || (num_graphs > 1 && graph_vbegin == nullptr)) return FASTBCC_ERR_INVALID_ARGUMENT;
  if (offsets_bits == 32)
    return solve_impl<int>(n, num_arcs, (const int*)offsets, adj, num_graphs, graph_vbegin, out_edge_label, out_is_ap,
                           out_num_bcc, workspace, workspace_bytes, flags, (hipStream_t)stream, trace);
  if (offsets_bits == 64)
    return solve_impl<int64_t>(n, num_arcs, (const int64_t*)offsets, adj, num_graphs, graph_vbegin, out_edge_label,
                               out_is_ap, out_num_bcc, workspace, workspace_bytes, flags, (hipStream_t)stream, trace);
  return FASTBCC_ERR_INVALID_ARGUMENT;
}

fastbcc_trace* fastbcc_trace_create(int32_t max_launches) {
  if (max_launches < 1) return nullptr;
  fastbcc_trace* t = new fastbcc_trace;
  t->pool.resize((size_t)max_launches * 2);
  for (auto& e : t->pool) {
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
  }
  for (auto e : t->pool)
    if (!e) {
      fastbcc_trace_destroy(t);
      return nullptr;
    }
  return t;
}

void fastbcc_trace_destroy(fastbcc_trace* t) {
  if (!t) return;
  for (auto e : t->pool)
    if (e) (void)hipEventDestroy(e);
  delete t;
}

fastbcc_status fastbcc_trace_collect(fastbcc_trace* t) {
  if (!t) return FASTBCC_ERR_INVALID_ARGUMENT;
  fastbcc_status rc = FASTBCC_OK;
  for (auto& p : t->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) != hipSuccess || hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) {
      rc = FASTBCC_ERR_HIP;
      continue;
    }
    bool found = false;
    for (auto& tot : t->totals)
      if (strcmp(tot.name, p.name) == 0) {
        tot.ms += ms;
        tot.launches += 1;
        found = true;
        break;
      }
    if (!found) t->totals.push_back({p.name, (double)ms, 1});
  }
  t->pending.clear();
  t->used = 0;
  return rc;
}

int32_t fastbcc_trace_count(const fastbcc_trace* t) { return t ? (int32_t)t->totals.size() : 0; }

fastbcc_status fastbcc_trace_entry(const fastbcc_trace* t, int32_t i, const char** name, double* total_ms,
                                   int64_t* launches) {
  if (!t || i < 0 || (size_t)i >= t->totals.size()) return FASTBCC_ERR_INVALID_ARGUMENT;
  if (name) *name = t->totals[i].name;
  if (total_ms) *total_ms = t->totals[i].ms;
  if (launches) *launches = t->totals[i].launches;
  return FASTBCC_OK;
}

int64_t fastbcc_trace_dropped(const fastbcc_trace* t) { return t ? t->dropped : 0; }

void fastbcc_trace_reset(fastbcc_trace* t) {
  if (!t) return;
  t->totals.clear();
  t->dropped = 0;
}

const char* fastbcc_status_string(fastbcc_status s) {
  switch (s) {
    case FASTBCC_OK: return "ok";
    case FASTBCC_ERR_INVALID_ARGUMENT: return "invalid argument";
    case FASTBCC_ERR_TOO_LARGE: return "graph too large (n >= 2^30 or arcs >= 2^31)";
    case FASTBCC_ERR_WORKSPACE_TOO_SMALL: return "workspace too small or missing";
    case FASTBCC_ERR_HIP: return "HIP runtime error";
    case FASTBCC_ERR_INVALID_GRAPH: return "input is not a valid symmetric CSR";
    case FASTBCC_ERR_SCRATCH_TOO_SMALL:
      return "graph needs a larger workspace than the static scratch of fastbcc_solve_noalloc holds";
  }
  return "unknown status";
}

const char* fastbcc_version(void) { return "0.1.0"; }

}  // extern "C"
