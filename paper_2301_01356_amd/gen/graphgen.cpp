// Seeded synthetic graph generators (host C++, OpenMP).
//
// These build the input workloads that both the HIP path and the CPU oracle
// consume.  They hold none of the biconnectivity arithmetic: every function
// here only draws random numbers and assembles a symmetric CSR (sorted rows,
// self-loops dropped, parallel edges merged).  Output is deterministic for a
// given seed, whatever the thread count: each structure draws from its own
// xoshiro256** stream, seeded through splitmix64 from (seed, stream id).
//
// Workload shapes follow the experiments section of the paper (low-diameter
// power-law graphs, large-diameter grids and chains, k-NN graphs); the exact
// recipes are stated in the design notes and repeated above each function.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>
#include <omp.h>

namespace {

inline uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9e3779b97f4a7c15ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// xoshiro256** (Blackman & Vigna), seeded from splitmix64 of (seed, stream).
struct Rng {
  uint64_t s[4];
  Rng(uint64_t seed, uint64_t stream) {
    uint64_t x = seed;
    uint64_t h = splitmix64(x);
    x = h ^ (stream * 0xd1b54a32d192ed03ULL + 0x8bb84b93962eacc9ULL);
    for (int i = 0; i < 4; ++i) s[i] = splitmix64(x);
  }
  static inline uint64_t rotl(uint64_t v, int k) { return (v << k) | (v >> (64 - k)); }
  inline uint64_t next() {
    const uint64_t r = rotl(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t; s[3] = rotl(s[3], 45);
    return r;
  }
  // integer in [0, n) by multiply-shift (bias < n / 2^64, irrelevant here)
  inline uint64_t below(uint64_t n) {
    return (uint64_t)(((__uint128_t)next() * (__uint128_t)n) >> 64);
  }
  inline double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

// Stream ids: one per structure so adding a structure never shifts another.
enum : uint64_t {
  S_BASE = 1, S_PENDANT = 2, S_CYCLE = 3, S_GRID_ROW = 1ull << 40, S_PATH = 5,
  S_RMAT_CHUNK = 1ull << 41, S_PERM = 7, S_MIX = 1ull << 42, S_FAMILY = 9,
};

struct Edges {
  std::vector<int32_t> u, v;
  void add(int64_t a, int64_t b) { u.push_back((int32_t)a); v.push_back((int32_t)b); }
};

struct Graph {
  int64_t n = 0;
  std::vector<int64_t> off;   // n + 1
  std::vector<int32_t> adj;   // off[n]
  std::vector<int32_t> vbegin; // for concatenated batches: G + 1 entries
  std::vector<int64_t> meta;  // generator facts a test may want (documented per generator)
};

// Symmetric CSR from an undirected edge list: both directions stored, rows
// sorted ascending, self-loops dropped, repeated edges merged.
void build_csr(int64_t n, const int32_t* eu, const int32_t* ev, int64_t m, Graph& g) {
  g.n = n;
  std::vector<std::atomic<int64_t>> cnt(n);
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) cnt[i].store(0, std::memory_order_relaxed);
  #pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    int32_t a = eu[e], b = ev[e];
    if (a == b) continue;
    cnt[a].fetch_add(1, std::memory_order_relaxed);
    cnt[b].fetch_add(1, std::memory_order_relaxed);
  }
  std::vector<int64_t> off(n + 1);
  off[0] = 0;
  for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + cnt[i].load(std::memory_order_relaxed);
  std::vector<int32_t> raw(off[n]);
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) cnt[i].store(off[i], std::memory_order_relaxed);
  #pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    int32_t a = eu[e], b = ev[e];
    if (a == b) continue;
    raw[cnt[a].fetch_add(1, std::memory_order_relaxed)] = b;
    raw[cnt[b].fetch_add(1, std::memory_order_relaxed)] = a;
  }
  std::vector<int64_t> deg(n);
  #pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i) {
    int32_t* b = raw.data() + off[i];
    int32_t* e = raw.data() + off[i + 1];
    std::sort(b, e);
    deg[i] = std::unique(b, e) - b;
  }
  g.off.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) g.off[i + 1] = g.off[i] + deg[i];
  g.adj.resize(g.off[n]);
  #pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i)
    std::memcpy(g.adj.data() + g.off[i], raw.data() + off[i], sizeof(int32_t) * deg[i]);
}

void build_csr(int64_t n, const Edges& e, Graph& g) {
  build_csr(n, e.u.data(), e.v.data(), (int64_t)e.u.size(), g);
}

// ---------------------------------------------------------------- families
// Random recursive tree on [base, base + s): vertex i > 0 joins a uniform j < i.
void recursive_tree(Rng& r, int64_t base, int64_t s, Edges& e, std::vector<int64_t>* parent) {
  for (int64_t i = 1; i < s; ++i) {
    int64_t j = (int64_t)r.below((uint64_t)i);
    e.add(base + j, base + i);
    if (parent) (*parent)[i] = j;
  }
}

// family 0: uniform random graph with about n*d/2 edges (endpoints uniform).
void fam_random(Rng& r, int64_t n, double d, Edges& e) {
  int64_t m = (int64_t)std::llround(n * d / 2.0);
  for (int64_t i = 0; i < m; ++i) {
    int64_t a = (int64_t)r.below(n), b = (int64_t)r.below(n);
    e.add(a, b);
  }
}

// family 1: open lattice with about sqrt(n) columns holding n vertices
// row-major (last row partial); each lattice edge kept with probability p.
void fam_lattice(Rng& r, int64_t n, double p, Edges& e) {
  int64_t rows = std::max<int64_t>(1, (int64_t)std::floor(std::sqrt((double)n)));
  int64_t cols = (n + rows - 1) / rows;
  for (int64_t id = 0; id < n; ++id) {
    int64_t c = id % cols;
    if (c + 1 < cols && id + 1 < n && r.uniform() < p) e.add(id, id + 1);
    if (id + cols < n && r.uniform() < p) e.add(id, id + cols);
  }
}

// family 2: k nearest neighbours (Euclidean, ties by index) of n uniform
// points in the unit square; each point links to its k nearest, symmetrised.
// The neighbour search runs in parallel over points (inside an already
// parallel region it runs serially); edges are appended in point order, so
// the result does not depend on the thread count.
void fam_knn(Rng& r, int64_t n, int k, Edges& e) {
  std::vector<double> x(n), y(n);
  for (int64_t i = 0; i < n; ++i) { x[i] = r.uniform(); y[i] = r.uniform(); }
  int64_t g = std::max<int64_t>(1, (int64_t)std::floor(std::sqrt((double)n / 2.0)));
  double cs = 1.0 / (double)g;
  std::vector<int64_t> cell_of(n), cstart(g * g + 1, 0), items(n);
  for (int64_t i = 0; i < n; ++i) {
    int64_t cx = std::min<int64_t>(g - 1, (int64_t)(x[i] * g));
    int64_t cy = std::min<int64_t>(g - 1, (int64_t)(y[i] * g));
    cell_of[i] = cy * g + cx;
    cstart[cell_of[i] + 1]++;
  }
  for (int64_t c = 0; c < g * g; ++c) cstart[c + 1] += cstart[c];
  {
    std::vector<int64_t> cur(cstart.begin(), cstart.end() - 1);
    for (int64_t i = 0; i < n; ++i) items[cur[cell_of[i]]++] = i;
  }
  const int kk = (int)std::min<int64_t>(k, n - 1);
  std::vector<int32_t> nbr((size_t)n * (kk > 0 ? kk : 1), -1);
  #pragma omp parallel if (n >= 65536 && !omp_in_parallel())
  {
    std::vector<std::pair<double, int64_t>> cand;
    #pragma omp for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
      int64_t cx = cell_of[i] % g, cy = cell_of[i] / g;
      for (int64_t rad = 1;; ++rad) {
        cand.clear();
        for (int64_t yy = std::max<int64_t>(0, cy - rad); yy <= std::min<int64_t>(g - 1, cy + rad); ++yy)
          for (int64_t xx = std::max<int64_t>(0, cx - rad); xx <= std::min<int64_t>(g - 1, cx + rad); ++xx) {
            int64_t c = yy * g + xx;
            for (int64_t t = cstart[c]; t < cstart[c + 1]; ++t) {
              int64_t j = items[t];
              if (j == i) continue;
              double dx = x[i] - x[j], dy = y[i] - y[j];
              cand.emplace_back(dx * dx + dy * dy, j);
            }
          }
        bool covers_all = (cx - rad <= 0 && cy - rad <= 0 && cx + rad >= g - 1 && cy + rad >= g - 1);
        if ((int64_t)cand.size() >= kk) {
          std::partial_sort(cand.begin(), cand.begin() + kk, cand.end());
          double reach = (double)rad * cs;  // every point within this distance is in the window
          if (covers_all || cand[kk - 1].first <= reach * reach) break;
        } else if (covers_all) {
          break;
        }
      }
      int take = (int)std::min<int64_t>(kk, (int64_t)cand.size());
      for (int t = 0; t < take; ++t) nbr[(size_t)i * kk + t] = (int32_t)cand[t].second;
    }
  }
  for (int64_t i = 0; i < n; ++i)
    for (int t = 0; t < kk; ++t)
      if (nbr[(size_t)i * kk + t] >= 0) e.add(i, nbr[(size_t)i * kk + t]);
}

// family 3: random recursive tree plus floor(f*n) extra edges, each from a
// uniform vertex to one of its proper ancestors above its parent.
void fam_tree_back(Rng& r, int64_t n, double f, Edges& e) {
  std::vector<int64_t> parent(n, -1);
  recursive_tree(r, 0, n, e, &parent);
  int64_t nb = (int64_t)std::floor(f * (double)n);
  for (int64_t t = 0; t < nb && n > 2; ++t) {
    int64_t v = 1 + (int64_t)r.below(n - 1);
    int64_t a = parent[v];
    int64_t hops = 1 + (int64_t)r.below(6);
    for (int64_t h = 0; h < hops && a > 0; ++h) a = parent[a];
    if (a >= 0 && a != parent[v]) e.add(a, v);
  }
}

// One graph of the mixed-family workload: family uniform over the four above,
// n log-uniform in [nmin, nmax]; random-graph degree d ~ U[dmin, dmax],
// lattice p ~ U[0.6, 0.9], k-NN k = 5, tree back-edge fraction f ~ U[0.05, 0.5].
void mixed_graph(uint64_t seed, int64_t index, int64_t nmin, int64_t nmax, double dmin, double dmax,
                 Graph& g, int* family_out) {
  Rng r(seed, S_MIX + (uint64_t)index);
  double lo = std::log((double)nmin), hi = std::log((double)nmax);
  int64_t n = (int64_t)std::llround(std::exp(lo + (hi - lo) * r.uniform()));
  n = std::max<int64_t>(nmin, std::min<int64_t>(nmax, n));
  int fam = (int)r.below(4);
  double pd = dmin + (dmax - dmin) * r.uniform();
  double pp = 0.6 + 0.3 * r.uniform();
  double pf = 0.05 + 0.45 * r.uniform();
  Rng rg(seed, (S_MIX + (uint64_t)index) ^ 0x5bd1e995ULL);
  Edges e;
  switch (fam) {
    case 0: fam_random(rg, n, pd, e); break;
    case 1: fam_lattice(rg, n, pp, e); break;
    case 2: fam_knn(rg, n, 5, e); break;
    default: fam_tree_back(rg, n, pf, e); break;
  }
  build_csr(n, e, g);
  if (family_out) *family_out = fam;
}

}  // namespace

extern "C" {

// Plain workload: n_base vertices with m_base uniform endpoint pairs, then
// n_pendant random recursive trees of U{pmin..pmax} vertices each joined by
// one edge to a uniform base vertex, then n_cycles cycles of U{cmin..cmax}
// vertices each joined by one bridge to a uniform base vertex.  Appended
// vertices are numbered after the base in generation order.
// meta = [n_base, sum of pendant tree sizes, number of cycles].
void* gg_plain(uint64_t seed, int64_t n_base, int64_t m_base, int64_t n_pendant, int64_t pmin,
               int64_t pmax, int64_t n_cycles, int64_t cmin, int64_t cmax) {
  Graph* g = new Graph;
  Edges e;
  Rng rb(seed, S_BASE), rp(seed, S_PENDANT), rc(seed, S_CYCLE);
  for (int64_t i = 0; i < m_base; ++i) {
    int64_t a = (int64_t)rb.below(n_base), b = (int64_t)rb.below(n_base);
    e.add(a, b);
  }
  int64_t next = n_base, pend_total = 0;
  for (int64_t t = 0; t < n_pendant; ++t) {
    int64_t s = pmin + (int64_t)rp.below((uint64_t)(pmax - pmin + 1));
    recursive_tree(rp, next, s, e, nullptr);
    e.add(next, (int64_t)rp.below(n_base));
    next += s;
    pend_total += s;
  }
  for (int64_t c = 0; c < n_cycles; ++c) {
    int64_t L = cmin + (int64_t)rc.below((uint64_t)(cmax - cmin + 1));
    for (int64_t i = 0; i < L; ++i) e.add(next + i, next + (i + 1) % L);
    e.add(next, (int64_t)rc.below(n_base));
    next += L;
  }
  build_csr(next, e, *g);
  g->meta = {n_base, pend_total, n_cycles};
  return g;
}

// Large-diameter workload: rows x cols lattice (vertex r*cols+c), open, or
// circular in both directions when wrap != 0 (the paper's SQR/REC grids), each
// edge kept with probability p; then a path of path_len vertices numbered
// after the lattice, joined by one edge to a seeded corner of the lattice,
// with one chord (a, b), b - a >= 2, inside every block of chord_block path
// vertices (blocks shorter than 3 vertices get none).
// meta = [rows, cols, path_len, corner vertex].
void* gg_grid(uint64_t seed, int64_t rows, int64_t cols, double p, int64_t path_len, int64_t chord_block,
              int wrap) {
  Graph* g = new Graph;
  int nt = omp_get_max_threads();
  std::vector<Edges> parts(nt);
  #pragma omp parallel
  {
    Edges& loc = parts[omp_get_thread_num()];
    #pragma omp for schedule(static)
    for (int64_t rr = 0; rr < rows; ++rr) {
      Rng r(seed, S_GRID_ROW + (uint64_t)rr);
      for (int64_t c = 0; c < cols; ++c) {
        int64_t id = rr * cols + c;
        if (c + 1 < cols) {
          if (r.uniform() < p) loc.add(id, id + 1);
        } else if (wrap && cols > 2) {
          if (r.uniform() < p) loc.add(id, rr * cols);
        }
        if (rr + 1 < rows) {
          if (r.uniform() < p) loc.add(id, id + cols);
        } else if (wrap && rows > 2) {
          if (r.uniform() < p) loc.add(id, c);
        }
      }
    }
  }
  Edges e;
  for (auto& pt : parts) {
    e.u.insert(e.u.end(), pt.u.begin(), pt.u.end());
    e.v.insert(e.v.end(), pt.v.begin(), pt.v.end());
  }
  int64_t base = rows * cols, corner = 0;
  if (path_len > 0) {
    Rng r(seed, S_PATH);
    const int64_t corners[4] = {0, cols - 1, (rows - 1) * cols, rows * cols - 1};
    corner = corners[r.below(4)];
    e.add(corner, base);
    for (int64_t i = 0; i + 1 < path_len; ++i) e.add(base + i, base + i + 1);
    for (int64_t s = 0; s < path_len; s += chord_block) {
      int64_t end = std::min(path_len, s + chord_block);
      if (end - s < 3) continue;
      int64_t a = s + (int64_t)r.below((uint64_t)(end - s - 2));
      int64_t b = a + 2 + (int64_t)r.below((uint64_t)(end - a - 2));
      e.add(base + a, base + b);
    }
  }
  build_csr(base + path_len, e, *g);
  g->meta = {rows, cols, path_len, corner};
  return g;
}

// R-MAT (Chakrabarti, Zhan, Faloutsos): 2^scale vertices, edge_factor*2^scale
// samples, quadrant probabilities (a, b, c, 1-a-b-c) at every level, no noise;
// then symmetrised, merged, self-loops dropped and (if permute) vertex ids
// relabelled by a seeded uniform permutation.
void* gg_rmat(uint64_t seed, int scale, int64_t edge_factor, double a, double b, double c, int permute) {
  Graph* g = new Graph;
  const int64_t n = (int64_t)1 << scale;
  const int64_t m = edge_factor * n;
  const uint64_t ta = (uint64_t)(a * 4294967296.0);
  const uint64_t tb = (uint64_t)((a + b) * 4294967296.0);
  const uint64_t tc = (uint64_t)((a + b + c) * 4294967296.0);
  std::vector<int32_t> eu(m), ev(m);
  const int64_t chunk = 1 << 16;
  const int64_t nchunks = (m + chunk - 1) / chunk;
  #pragma omp parallel for schedule(dynamic, 4)
  for (int64_t ch = 0; ch < nchunks; ++ch) {
    Rng r(seed, S_RMAT_CHUNK + (uint64_t)ch);
    int64_t e0 = ch * chunk, e1 = std::min(m, e0 + chunk);
    for (int64_t e = e0; e < e1; ++e) {
      uint32_t u = 0, v = 0;
      uint64_t bits = 0;
      for (int l = 0; l < scale; ++l) {
        if ((l & 1) == 0) bits = r.next();
        uint64_t x = (l & 1) ? (bits >> 32) : (bits & 0xffffffffULL);
        uint32_t bu = (x >= tb) ? 1u : 0u;
        uint32_t bv = (x >= ta && x < tb) || (x >= tc) ? 1u : 0u;
        u = (u << 1) | bu;
        v = (v << 1) | bv;
      }
      eu[e] = (int32_t)u;
      ev[e] = (int32_t)v;
    }
  }
  if (permute) {
    std::vector<int32_t> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    Rng r(seed, S_PERM);
    for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[(int64_t)r.below((uint64_t)(i + 1))]);
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) { eu[e] = perm[eu[e]]; ev[e] = perm[ev[e]]; }
  }
  build_csr(n, eu.data(), ev.data(), m, *g);
  g->meta = {scale, edge_factor};
  return g;
}

// One graph of a single family (see fam_* above) with explicit parameters.
void* gg_family(uint64_t seed, int family, int64_t n, double param) {
  Graph* g = new Graph;
  Rng r(seed, S_FAMILY);
  Edges e;
  switch (family) {
    case 0: fam_random(r, n, param, e); break;
    case 1: fam_lattice(r, n, param, e); break;
    case 2: fam_knn(r, n, (int)param, e); break;
    default: fam_tree_back(r, n, param, e); break;
  }
  build_csr(n, e, *g);
  g->meta = {family};
  return g;
}

// One graph of the mixed-family workload, drawn from stream (seed, index).
// meta = [family].
void* gg_mixed(uint64_t seed, int64_t index, int64_t nmin, int64_t nmax, double dmin, double dmax) {
  Graph* g = new Graph;
  int fam = 0;
  mixed_graph(seed, index, nmin, nmax, dmin, dmax, *g, &fam);
  g->meta = {fam};
  return g;
}

// Disjoint union of graphs gg_mixed(seed, i, ...) for i in [0, count): graph i
// owns vertices [vbegin[i], vbegin[i+1]) and its arcs hold global vertex ids.
// meta = family of each graph.
void* gg_batch(uint64_t seed, int64_t count, int64_t nmin, int64_t nmax, double dmin, double dmax) {
  std::vector<Graph> parts(count);
  std::vector<int> fams(count);
  #pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < count; ++i) mixed_graph(seed, i, nmin, nmax, dmin, dmax, parts[i], &fams[i]);
  Graph* g = new Graph;
  g->vbegin.assign(count + 1, 0);
  std::vector<int64_t> abeg(count + 1, 0);
  for (int64_t i = 0; i < count; ++i) {
    g->vbegin[i + 1] = g->vbegin[i] + (int32_t)parts[i].n;
    abeg[i + 1] = abeg[i] + (int64_t)parts[i].adj.size();
  }
  g->n = g->vbegin[count];
  g->off.assign(g->n + 1, 0);
  g->adj.resize(abeg[count]);
  #pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < count; ++i) {
    const Graph& p = parts[i];
    int64_t vb = g->vbegin[i];
    for (int64_t v = 0; v <= p.n; ++v) g->off[vb + v] = abeg[i] + p.off[v];
    for (size_t t = 0; t < p.adj.size(); ++t) g->adj[abeg[i] + t] = (int32_t)(p.adj[t] + vb);
  }
  g->meta.assign(fams.begin(), fams.end());
  return g;
}

// CSR from an explicit undirected edge list (merged, self-loops dropped).
void* gg_from_edges(int64_t n, int64_t m, const int32_t* u, const int32_t* v) {
  Graph* g = new Graph;
  build_csr(n, u, v, m, *g);
  return g;
}

int64_t gg_num_vertices(void* h) { return ((Graph*)h)->n; }
int64_t gg_num_arcs(void* h) { return (int64_t)((Graph*)h)->adj.size(); }
int64_t gg_num_graphs(void* h) {
  Graph* g = (Graph*)h;
  return g->vbegin.empty() ? 0 : (int64_t)g->vbegin.size() - 1;
}
int64_t gg_meta_len(void* h) { return (int64_t)((Graph*)h)->meta.size(); }

// Copy out: offsets as int64 and/or int32 (either may be null), adj, vbegin.
void gg_copy(void* h, int64_t* off64, int32_t* off32, int32_t* adj, int32_t* vbegin, int64_t* meta) {
  Graph* g = (Graph*)h;
  if (off64) std::memcpy(off64, g->off.data(), sizeof(int64_t) * (g->n + 1));
  if (off32) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i <= g->n; ++i) off32[i] = (int32_t)g->off[i];
  }
  if (adj) std::memcpy(adj, g->adj.data(), sizeof(int32_t) * g->adj.size());
  if (vbegin && !g->vbegin.empty()) std::memcpy(vbegin, g->vbegin.data(), sizeof(int32_t) * g->vbegin.size());
  if (meta && !g->meta.empty()) std::memcpy(meta, g->meta.data(), sizeof(int64_t) * g->meta.size());
}

void gg_free(void* h) { delete (Graph*)h; }

}  // extern "C"
