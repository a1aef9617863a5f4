// Fused batched solve of small graphs (the C ABI's fastbcc_solve_small).
//
// A batch of small graphs is a disconnected input whose components are
// independent (paper: Algorithm 1, First-CC processes the connected
// components in parallel), so a run of consecutive graphs (a pack) is solved
// by ONE workgroup, start to end, as one disjoint union with every
// per-vertex array of the pipeline in LDS: one launch per size class, each
// workgroup looping over the packs (persistent), and no workspace.  The
// adjacency is read from device memory (arc-parallel, a chunk of arcs per
// thread in flight at once); a pack's rows are small enough to stay in L2
// between the passes that read them.
//
// Steps per pack (each ends with a workgroup barrier):
//   First-CC   union-find in LDS over the graph's edges, each edge once from
//              its smaller endpoint, min-id hooking by CAS; a hooked root
//              keeps the edge that hooked it, so the kept edges form a
//              spanning forest and each set's root is its smallest vertex.
//   Rooting    the edge kept at v gives tree arcs 2v and 2v + 1 (twins by
//              x ^ 1); per-vertex lists of tree arcs by count, scan and
//              scatter; Euler circuit successor of u->v = the arc after
//              v->u in v's cyclic list (paper: Euler tour technique); each
//              tree's circuit is cut before its root's first arc; list ranking
//              by pointer jumping gives each arc its distance to the tour's
//              end.  Of two twins the one with the larger distance is the
//              down arc (its tail is the parent); preorder numbers come from a
//              scan of down-arc flags in tour order, subtree sizes from the
//              twins' distances: first[v] and last[v] = first[v] + |T_v| - 1.
//   Tagging    w1/w2 = min/max of first[] over each vertex and all its
//              neighbours (paper: Section "Tagging"; the extra tree
//              neighbours cannot change a fence decision), placed by preorder;
//              low/high by range min/max over [first[v], last[v]] (32-slot
//              blocks with in-block prefix and suffix extrema plus a sparse
//              table over the blocks); tree edge p(v)-v is a fence iff
//              first[p] <= low[v] and high[v] <= last[p].
//   Last-CC    union-find over the skeleton: plain (non-fence) tree edges and
//              cross edges (neither endpoint an ancestor of the other); fence
//              and back edges are left out.
//   Read-out   head(l[v]) = p(v) for a fence child v with l[v] != l[p(v)];
//              such a p is an articulation point unless it is a tree root,
//              which is one iff it heads two labels; arc x->y lies in l[x]
//              unless x heads l[y]; the canonical label of a BCC is its
//              smallest arc (LDS atomic minimum) made graph-local; a BCC is
//              a Last-CC root that is not a tree root, counted per graph.
//
// Results are exactly those of fastbcc_solve_batched (the BCC partition is
// unique and so is its canonical labelling); the spanning forest may differ.

#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include <mutex>

#include "fastbcc.h"

namespace {

constexpr int SW = 64;  // wavefront width of gfx950

__device__ __forceinline__ int lds_ld(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Union-find in LDS.  Parents only ever point to smaller ids (a hook puts the
// larger root under the smaller one; path halving stores an ancestor), so
// every walk ends.
__device__ __forceinline__ int s_find(int* p, int x) {
  int px = lds_ld(p + x);
  while (px != x) {
    const int gx = lds_ld(p + px);
    if (gx == px) return px;
    lds_st(p + x, gx);
    x = gx;
    px = lds_ld(p + x);
  }
  return x;
}

// Root without writes: the flattening pass reads only, so no concurrent
// path-halving store can leave an entry on a stale ancestor.
__device__ __forceinline__ int s_root(const int* p, int x) {
  int px = lds_ld(p + x);
  while (px != x) {
    x = px;
    px = lds_ld(p + x);
  }
  return x;
}

// Joins the set entered at su (u itself, or a root found for u earlier: a
// root only ever gains ancestors, so its find is u's find) with v's set;
// returns the root it hooked, or -1 when they were already one set, and
// leaves u's root as found in ru_found.  At a successful CAS the two sets are
// disjoint, so an edge recorded per hooked root is a spanning-forest edge.
__device__ __forceinline__ int s_link_at(int* p, int su, int v, int& ru_found) {
  int ru = s_find(p, su), rv = s_find(p, v);
  ru_found = ru;
  while (ru != rv) {
    const int hi = ru > rv ? ru : rv, lo = ru > rv ? rv : ru;
    if (atomicCAS(p + hi, hi, lo) == hi) return hi;
    ru = s_find(p, ru);
    rv = s_find(p, rv);
  }
  return -1;
}

__device__ __forceinline__ int s_link(int* p, int u, int v) {
  int ru;
  return s_link_at(p, u, v, ru);
}

// Exclusive scan in place of a[0, m) by T threads (contiguous chunks per
// thread, wave scans, one pass over the wave totals); returns the total.
// ws: T / SW + 1 ints of LDS.  Called by the whole workgroup.
template <int T>
__device__ int s_scan(int* a, int m, int* ws) {
  const int tid = threadIdx.x, lane = tid & (SW - 1), wid = tid / SW;
  const int c = (m + T - 1) / T;
  const int b = min(tid * c, m), e = min(b + c, m);
  int s = 0;
  for (int i = b; i < e; ++i) s += a[i];
  int x = s;
#pragma unroll
  for (int o = 1; o < SW; o <<= 1) {
    const int y = __shfl_up(x, o, SW);
    if (lane >= o) x += y;
  }
  if (lane == SW - 1) ws[wid] = x;
  __syncthreads();
  if (tid == 0) {
    int t = 0;
    for (int w = 0; w < T / SW; ++w) {
      const int q = ws[w];
      ws[w] = t;
      t += q;
    }
    ws[T / SW] = t;
  }
  __syncthreads();
  int run = ws[wid] + x - s;
  for (int i = b; i < e; ++i) {
    const int q = a[i];
    a[i] = run;
    run += q;
  }
  const int total = ws[T / SW];
  __syncthreads();
  return total;
}

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }

constexpr int RMQ_B = 32;  // preorder slots per range-query block

// LDS words of one workgroup for graphs of up to NS vertices.
template <int NS, int T>
struct SmallLayout {
  static constexpr int NB = NS / RMQ_B;
  static constexpr int LOGB = ilog2c(NB) + 1;
  static constexpr int R0 = 0;              // union-find | W1 | Last-CC labels
  static constexpr int R1 = NS;             // edge end u (TB at roots) | W2 | head of label
  static constexpr int R2 = 2 * NS;         // edge end w (VB at roots) | prefix min | head flag
  static constexpr int R3 = 3 * NS;         // list fill counters | first tree arc | suffix min | root label
  static constexpr int R4 = 4 * NS;         // tree-list starts (NS + 1) | parent
  static constexpr int R5 = 5 * NS + 64;    // 2 NS: tree lists | down flags | prefix/suffix max | AP, min arc
  static constexpr int R6 = 7 * NS + 64;    // 2 NS: list positions | tour distances | fence flags
  static constexpr int R7 = 9 * NS + 64;    // 2 NS: successors | first, last
  static constexpr int R8 = 11 * NS + 64;   // sparse tables (min, max): 2 * LOGB * NB
  static constexpr int R9 = R8 + 2 * LOGB * NB;  // scan wave totals (T / SW + 1), counter
  static constexpr int R10 = R9 + T / SW + 8;    // graph-local row starts (NS + 1)
  static constexpr int WORDS = R10 + NS + 64;
};

constexpr int ARC_CHUNK = 8;  // arcs per thread loaded before any is used

// One pack per workgroup at a time: the consecutive graphs [pack_begin[p],
// pack_begin[p + 1]) solved as one disjoint union (a graph per pack without
// pack_begin), so the fixed cost of the pipeline's barriers is paid once for
// many small graphs.  Packs with lo_n < n <= NS vertices are this class's;
// with reject, larger ones get num_bcc = -1 for all their graphs.  The loop
// bounds and every branch around a barrier depend only on the pack, so all
// threads reach every barrier.
template <int NS, int T>
__global__ void __launch_bounds__(T) k_small_bcc(const int* __restrict__ vbegin, int G,
                                                 const int* __restrict__ pack_begin, int P, int64_t n_total,
                                                 int64_t num_arcs, const int* __restrict__ off,
                                                 const int* __restrict__ adj, int lo_n, bool reject,
                                                 int* __restrict__ out_label, uint8_t* __restrict__ out_ap,
                                                 int64_t* __restrict__ out_nbcc) {
  using Lay = SmallLayout<NS, T>;
  constexpr int VPT = NS / T;  // vertices per thread
  constexpr int NB = Lay::NB;
  static_assert(NS % T == 0 && T % SW == 0 && NS % RMQ_B == 0 && SW % RMQ_B == 0, "class shape");
  __shared__ int S[Lay::WORDS];
  int* const UF = S + Lay::R0;
  int* const TU = S + Lay::R1;
  int* const TW = S + Lay::R2;
  int* const FILL = S + Lay::R3;
  int* const FA = S + Lay::R3;
  int* const TST = S + Lay::R4;
  int* const PAR = S + Lay::R4;
  int* const TADJ = S + Lay::R5;
  int* const E = S + Lay::R5;
  int* const LPOS = S + Lay::R6;
  int* const DIST = S + Lay::R6;
  int* const NX = S + Lay::R7;
  int* const FIRST = S + Lay::R7;
  int* const LAST = S + Lay::R7 + NS;
  int* const ST1 = S + Lay::R8;
  int* const ST2 = S + Lay::R8 + Lay::LOGB * NB;
  int* const WS = S + Lay::R9;
  int* const OFF = S + Lay::R10;
  const int tid = threadIdx.x;

  for (int p = blockIdx.x; p < P; p += gridDim.x) {
    const int gb = pack_begin ? pack_begin[p] : p, ge = pack_begin ? pack_begin[p + 1] : p + 1;
    if (gb < 0 || ge < gb || ge > G) continue;  // not a pack of this batch: nothing to read or write
    const int ng = ge - gb;
    auto mark_all = [&](int64_t val) {
      for (int k = tid; k < ng; k += T) out_nbcc[gb + k] = val;
    };
    const int v0 = vbegin[gb], v1 = vbegin[ge];
    const int n = v1 - v0;
    if (v0 < 0 || v1 > n_total || n < 0) {  // not a valid range: nothing is read
      mark_all(-1);
      continue;
    }
    if (n <= lo_n) continue;  // a smaller class's pack
    if (n > NS) {
      if (reject) mark_all(-1);
      continue;
    }
    if (ng > NS) {  // more graphs than LDS slots for their starts
      mark_all(-1);
      continue;
    }
    if (n == 0) {
      mark_all(0);
      continue;
    }
    const int a0 = off[v0], a1 = off[v1];
    if (a0 < 0 || a1 < a0 || a1 > num_arcs) {
      mark_all(-1);
      continue;
    }
    const int A = a1 - a0;
    // Arc passes are arc-parallel: thread t takes the t-th contiguous run of
    // ceil(A / T) arcs, finds the row of its first arc by bisection over the
    // row starts in LDS and walks forward from there; it loads ARC_CHUNK
    // targets at once (one memory latency per chunk).  body(local arc,
    // source, local target); a target outside [0, n) is a foreign id,
    // ignored by every pass.  No barrier inside.
    auto row_of = [&](int a) {
      int lo = 0, hi = n;  // OFF[lo] <= a < OFF[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (OFF[mid] <= a) lo = mid;
        else hi = mid;
      }
      return lo;
    };
    const int64_t per = ((int64_t)A + T - 1) / T;  // 64-bit: tid * per may pass 2^31 before the clamp
    const int ab = (int)min((int64_t)tid * per, (int64_t)A), ae = (int)min((int64_t)ab + per, (int64_t)A);
    auto for_arcs = [&](auto&& body) {
      if (ab >= ae) return;
      int v = row_of(ab);
      for (int c0 = ab; c0 < ae; c0 += ARC_CHUNK) {  // c0 + ARC_CHUNK < 2^31: the entry point bounds the arcs
        int tg[ARC_CHUNK];
#pragma unroll
        for (int k = 0; k < ARC_CHUNK; ++k) tg[k] = c0 + k < ae ? adj[a0 + c0 + k] - v0 : -1;
#pragma unroll
        for (int k = 0; k < ARC_CHUNK; ++k) {
          const int a = c0 + k;
          if (a >= ae) break;
          while (OFF[v + 1] <= a) ++v;  // OFF[n] = A > a ends the walk
          body(a, v, tg[k]);
        }
      }
    };

    // ---------------------------------------------------------- First-CC
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * T;
      if (v < n) {
        UF[v] = v;
        TU[v] = -1;
        TST[v] = 0;
        FILL[v] = 0;
        OFF[v] = min(max(off[v0 + v] - a0, 0), A);
      }
    }
    if (tid == 0) OFF[n] = A;
    __syncthreads();
    int cv = -1, cr = 0;  // the run's last source and the root found for it
    for_arcs([&](int, int v, int y) {
      if (y <= v || y >= n) return;  // each edge once; self-loops and foreign ids skipped
      const int h = s_link_at(UF, v == cv ? cr : v, y, cr);
      cv = v;
      if (h >= 0) {
        TU[h] = v;
        TW[h] = y;
      }
    });
    __syncthreads();
    // ---------------------------------------------------------- Rooting
    int rr[VPT];
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * T;
      rr[i] = v < n ? s_root(UF, v) : 0;
      if (v < n && TU[v] >= 0) {
        atomicAdd(TST + TU[v], 1);
        atomicAdd(TST + TW[v], 1);
      }
    }
    __syncthreads();
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * T;
      if (v < n) UF[v] = rr[i];  // every entry now holds its tree's root
    }
    __syncthreads();
    {
      const int tot = s_scan<T>(TST, n, WS);
      if (tid == 0) TST[n] = tot;
    }
    __syncthreads();
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * T;
      if (v >= n || UF[v] == v) continue;  // a non-root holds the edge that hooked it
      const int u = TU[v], w = TW[v];
      int s = TST[u] + atomicAdd(FILL + u, 1);
      TADJ[s] = 2 * v;  // u -> w
      LPOS[2 * v] = s;
      s = TST[w] + atomicAdd(FILL + w, 1);
      TADJ[s] = 2 * v + 1;  // w -> u
      LPOS[2 * v + 1] = s;
    }
    __syncthreads();
    for (int k = 0; k < 2 * VPT; ++k) {
      const int x = tid + k * T;
      if (x >= 2 * n) continue;
      const int e = x >> 1;
      if (UF[e] == e) continue;
      const int b = (x & 1) ? TU[e] : TW[e];  // head of arc x
      const int st = TST[b], deg = TST[b + 1] - st;
      int k2 = LPOS[x ^ 1] - st + 1;
      if (k2 == deg) k2 = 0;
      NX[x] = (k2 == 0 && UF[b] == b) ? -1 : TADJ[st + k2];  // back at the root's first arc: end
    }
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * T;
      if (v < n && UF[v] == v) FA[v] = TST[v + 1] > TST[v] ? TADJ[TST[v]] : -1;
    }
    __syncthreads();
    // list ranking by pointer jumping: DIST[x] = arcs after x in its tour
    for (int k = 0; k < 2 * VPT; ++k) {
      const int x = tid + k * T;
      if (x < 2 * n && UF[x >> 1] != (x >> 1)) DIST[x] = NX[x] >= 0 ? 1 : 0;
    }
    __syncthreads();
    // a list of at most 2 NS arcs is ranked in ilog2(2 NS) + 1 rounds; the
    // bound only guards the loop
    for (int round = 0; round < ilog2c(2 * NS) + 2; ++round) {
      int nd[2 * VPT], nn[2 * VPT];
      int more = 0;
#pragma unroll
      for (int k = 0; k < 2 * VPT; ++k) {
        const int x = tid + k * T;
        nn[k] = -1;
        nd[k] = 0;
        if (x < 2 * n && UF[x >> 1] != (x >> 1)) {
          const int nx = NX[x];
          if (nx >= 0) {
            nd[k] = DIST[x] + DIST[nx];
            nn[k] = NX[nx];
          } else {
            nn[k] = -2;  // finished: nothing to write
          }
        } else {
          nn[k] = -2;
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 2 * VPT; ++k) {
        const int x = tid + k * T;
        if (nn[k] != -2) {
          DIST[x] = nd[k];
          NX[x] = nn[k];
          more |= nn[k] >= 0;
        }
      }
      if (!__syncthreads_or(more)) break;
    }
    // per tree: tour length and vertex count, scanned into the tree's offset
    // in the concatenated tours (kept at the root in TU) and in preorder (TW)
    int* const TL = NX;
    int* const TS = NX + NS;
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * T;
      if (v >= n) continue;
      int L = 0, c = 0;
      if (UF[v] == v) {
        L = FA[v] >= 0 ? DIST[FA[v]] + 1 : 0;
        c = L / 2 + 1;
      }
      TL[v] = L;
      TS[v] = c;
    }
    __syncthreads();
    const int M = s_scan<T>(TL, n, WS);
    s_scan<T>(TS, n, WS);
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * T;
      if (v < n && UF[v] == v) {
        TU[v] = TL[v];
        TW[v] = TS[v];
      }
    }
    for (int k = 0; k < 2 * VPT; ++k) {
      const int x = tid + k * T;
      if (x < M) E[x] = 0;
    }
    __syncthreads();
    // down arcs: parents, and a flag at each down arc's tour position
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * T;
      if (v >= n) continue;
      if (UF[v] == v) {
        PAR[v] = -1;
        continue;
      }
      const bool fwd = DIST[2 * v] > DIST[2 * v + 1];  // arc 2v (TU -> TW) comes first
      const int child = fwd ? TW[v] : TU[v], parent = fwd ? TU[v] : TW[v];
      const int down = fwd ? 2 * v : 2 * v + 1;
      const int r = UF[v];
      const int L = DIST[FA[r]] + 1;
      E[TU[r] + (L - 1 - DIST[down])] = 1;
      PAR[child] = parent;
    }
    __syncthreads();
    s_scan<T>(E, M, WS);
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * T;
      if (v >= n) continue;
      const int r = UF[v];
      if (r == v) {
        const int L = FA[v] >= 0 ? DIST[FA[v]] + 1 : 0;
        FIRST[v] = TW[v];
        LAST[v] = TW[v] + L / 2;
        continue;
      }
      const bool fwd = DIST[2 * v] > DIST[2 * v + 1];
      const int child = fwd ? TW[v] : TU[v];
      const int down = fwd ? 2 * v : 2 * v + 1;
      const int L = DIST[FA[r]] + 1;
      const int pos = TU[r] + (L - 1 - DIST[down]);
      const int f = TW[r] + 1 + E[pos] - E[TU[r]];
      FIRST[child] = f;
      LAST[child] = f + (DIST[down] - DIST[down ^ 1] + 1) / 2 - 1;
    }
    __syncthreads();
    // ---------------------------------------------------------- Tagging
    int* const W1 = S + Lay::R0;
    int* const W2 = S + Lay::R1;
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * T;
      if (v < n) {
        const int f = FIRST[v];
        W1[f] = f;
        W2[f] = f;
      }
    }
    __syncthreads();
    for_arcs([&](int, int v, int y) {
      if (y == v || y < 0 || y >= n) return;
      const int f = FIRST[v], fy = FIRST[y];
      if (fy < f) atomicMin(W1 + f, fy);
      if (fy > f) atomicMax(W2 + f, fy);
    });
    __syncthreads();
    int* const P1 = S + Lay::R2;
    int* const S1 = S + Lay::R3;
    int* const P2 = S + Lay::R5;
    int* const S2 = S + Lay::R5 + NS;
    const int nb = (n + RMQ_B - 1) / RMQ_B;
    // in-block prefix and suffix extrema by segmented wave scans: slot
    // tid + k T sits in lane tid % 64, so each 32-lane half of a wave holds
    // one whole block; slots past n take the identity
    for (int k = 0; k < VPT; ++k) {
      const int i = tid + k * T;
      const bool in = i < n;
      const int sl = tid & (RMQ_B - 1);
      int p1 = in ? W1[i] : INT_MAX, p2 = in ? W2[i] : INT_MIN;
      int s1 = p1, s2 = p2;
#pragma unroll
      for (int o = 1; o < RMQ_B; o <<= 1) {
        const int u1 = __shfl_up(p1, o, RMQ_B), u2 = __shfl_up(p2, o, RMQ_B);
        const int d1 = __shfl_down(s1, o, RMQ_B), d2 = __shfl_down(s2, o, RMQ_B);
        if (sl >= o) {
          p1 = min(p1, u1);
          p2 = max(p2, u2);
        }
        if (sl + o < RMQ_B) {
          s1 = min(s1, d1);
          s2 = max(s2, d2);
        }
      }
      if (in) {
        P1[i] = p1;
        P2[i] = p2;
        S1[i] = s1;
        S2[i] = s2;
        if (sl == 0) {  // a block's suffix at its first slot is the block's extremum
          ST1[i / RMQ_B] = s1;
          ST2[i / RMQ_B] = s2;
        }
      }
    }
    __syncthreads();
    for (int j = 1; (1 << j) <= nb; ++j) {
      const int h = 1 << (j - 1);
      for (int b = tid; b + (1 << j) <= nb; b += T) {
        ST1[j * NB + b] = min(ST1[(j - 1) * NB + b], ST1[(j - 1) * NB + b + h]);
        ST2[j * NB + b] = max(ST2[(j - 1) * NB + b], ST2[(j - 1) * NB + b + h]);
      }
      __syncthreads();
    }
    int* const FEN = S + Lay::R6;
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * T;
      if (v >= n) continue;
      const int p = PAR[v];
      int fen = 0;
      if (p >= 0) {
        const int l = FIRST[v], r = LAST[v];
        const int bl = l / RMQ_B, br = r / RMQ_B;
        int mn, mx;
        if (bl == br) {
          mn = W1[l];
          mx = W2[l];
          for (int k = l + 1; k <= r; ++k) {
            mn = min(mn, W1[k]);
            mx = max(mx, W2[k]);
          }
        } else {
          mn = min(S1[l], P1[r]);
          mx = max(S2[l], P2[r]);
          const int len = br - bl - 1;
          if (len > 0) {
            const int j = 31 - __clz(len);
            mn = min(mn, min(ST1[j * NB + bl + 1], ST1[j * NB + br - (1 << j)]));
            mx = max(mx, max(ST2[j * NB + bl + 1], ST2[j * NB + br - (1 << j)]));
          }
        }
        fen = (FIRST[p] <= mn && LAST[p] >= mx) ? 1 : 0;
      }
      FEN[v] = fen;
    }
    __syncthreads();
    // ---------------------------------------------------------- Last-CC
    int* const LAB = S + Lay::R0;
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * T;
      if (v < n) LAB[v] = v;
    }
    __syncthreads();
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * T;
      if (v >= n) continue;
      const int p = PAR[v];
      if (p >= 0 && !FEN[v]) s_link(LAB, v, p);  // plain tree edge
    }
    cv = -1;
    for_arcs([&](int, int v, int y) {
      if (y <= v || y >= n || y == PAR[v] || PAR[y] == v) return;  // each edge once; tree arcs left out
      const int fv = FIRST[v], fy = FIRST[y];
      const bool y_under_v = fv <= fy && fy <= LAST[v];
      const bool v_under_y = fy <= fv && fv <= LAST[y];
      if (!y_under_v && !v_under_y) {  // cross edge
        s_link_at(LAB, v == cv ? cr : v, y, cr);
        cv = v;
      }
    });
    __syncthreads();
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * T;
      rr[i] = v < n ? s_root(LAB, v) : 0;
    }
    __syncthreads();
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * T;
      if (v < n) LAB[v] = rr[i];  // the smallest member of v's skeleton component
    }
    // ---------------------------------------------------------- read-out
    int* const HEAD = S + Lay::R1;
    int* const ISH = S + Lay::R2;
    int* const RLAB = S + Lay::R3;
    int* const APF = S + Lay::R5;
    int* const MINA = S + Lay::R5 + NS;
    int* const GK = S + Lay::R7;       // the pack's graph of each vertex
    int* const GV = S + Lay::R7 + NS;  // first vertex of each of the pack's graphs (ng + 1 words; the
                                       // last may reach into the dead sparse tables)
    int* const GCNT = S + Lay::R6;     // BCCs per graph (once the fence flags are read)
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * T;
      if (v < n) {
        HEAD[v] = -1;
        ISH[v] = 0;
        RLAB[v] = -1;
        APF[v] = 0;
        MINA[v] = INT_MAX;
      }
    }
    for (int k = tid; k <= ng; k += T) GV[k] = vbegin[gb + k] - v0;
    __syncthreads();
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * T;
      if (v >= n) continue;
      const int p = PAR[v];
      if (p < 0 || !FEN[v]) continue;
      const int L = LAB[v];
      if (L == LAB[p]) continue;
      HEAD[L] = p;
      ISH[p] = 1;
      if (PAR[p] >= 0) {
        APF[p] = 1;
      } else {
        const int old = atomicCAS(RLAB + p, -1, L);
        if (old != -1 && old != L) APF[p] = 1;
      }
    }
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * T;
      if (v >= n) continue;
      int lo = 0, hi = ng;  // GV[lo] <= v < GV[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (GV[mid] <= v) lo = mid;
        else hi = mid;
      }
      GK[v] = lo;
    }
    __syncthreads();
    for (int k = tid; k < ng; k += T) GCNT[k] = 0;
    auto arc_label = [&](int v, int y) {
      const int Lv = LAB[v];
      if (ISH[v]) {
        const int Ly = LAB[y];
        if (Ly != Lv && HEAD[Lv] != y) return Ly;  // v heads y's BCC
      }
      return Lv;
    };
    int last_label = -1;  // a thread's arcs ascend: only the first arc of a label run can be its minimum
    for_arcs([&](int a, int v, int y) {
      if (y == v || y < 0 || y >= n) return;
      const int L = arc_label(v, y);
      if (L != last_label) atomicMin(MINA + L, a);
      last_label = L;
    });
    __syncthreads();
    // graph-local labels: the pack-local smallest arc minus its graph's first arc
    for_arcs([&](int a, int v, int y) {
      const bool skip = y == v || y < 0 || y >= n;
      out_label[a0 + a] = skip ? -1 : MINA[arc_label(v, y)] - OFF[GV[GK[v]]];
    });
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * T;
      if (v >= n) continue;
      if (out_ap != nullptr) out_ap[v0 + v] = (uint8_t)APF[v];
      if (LAB[v] == v && PAR[v] >= 0) atomicAdd(GCNT + GK[v], 1);
    }
    __syncthreads();
    for (int k = tid; k < ng; k += T) out_nbcc[gb + k] = GCNT[k];
    __syncthreads();  // the next pack reuses every LDS word
  }
}

// ------------------------------------------------------------ classes
struct SmallClass {
  int max_n;
  int threads;
  const void* kernel;
};

template <int NS, int T>
SmallClass small_class() {
  return SmallClass{NS, T, reinterpret_cast<const void*>(&k_small_bcc<NS, T>)};
}

const SmallClass kClasses[] = {small_class<256, 256>(), small_class<1024, 256>(),
                               small_class<FASTBCC_SMALL_MAX_VERTICES, 1024>()};
constexpr int kNumClasses = sizeof(kClasses) / sizeof(kClasses[0]);
static_assert(FASTBCC_SMALL_MAX_VERTICES % 1024 == 0, "largest class shape");

// Resident workgroups per GPU for each class (occupancy x compute units),
// per device, found once.
constexpr int kMaxDevices = 64;
int g_resident[kMaxDevices][kNumClasses];
std::once_flag g_resident_once[kMaxDevices];

bool resident_groups(int dev, int* out) {
  if (dev < 0 || dev >= kMaxDevices) return false;
  bool ok = true;
  std::call_once(g_resident_once[dev], [&] {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    for (int c = 0; c < kNumClasses; ++c) {
      int per = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kClasses[c].kernel, kClasses[c].threads, 0) !=
              hipSuccess ||
          per <= 0)
        per = 1;
      g_resident[dev][c] = per * cus;
    }
  });
  for (int c = 0; c < kNumClasses; ++c) out[c] = g_resident[dev][c];
  return ok;
}

}  // namespace

extern "C" {

FASTBCC_API fastbcc_status fastbcc_solve_small(int32_t num_graphs, const int32_t* graph_vbegin, int32_t num_packs,
                                               const int32_t* pack_begin, int64_t n_total, int64_t num_arcs,
                                               const int32_t* offsets, const int32_t* adj, int32_t* out_edge_label,
                                               uint8_t* out_is_ap, int64_t* out_num_bcc, uint32_t flags,
                                               void* stream) {
  const uint32_t allowed = FASTBCC_FLAG_SORTED_ROWS | FASTBCC_FLAG_NO_SELF_LOOPS;
  if (num_graphs < 1 || graph_vbegin == nullptr || offsets == nullptr || out_num_bcc == nullptr || n_total < 0 ||
      num_arcs < 0 || (flags & ~allowed) != 0)
    return FASTBCC_ERR_INVALID_ARGUMENT;
  if (pack_begin == nullptr) num_packs = num_graphs;
  else if (num_packs < 1) return FASTBCC_ERR_INVALID_ARGUMENT;
  // arcs stay 64 below 2^31 so that a thread's chunk index never wraps
  if (n_total >= (int64_t(1) << 30) || num_arcs >= (int64_t(1) << 31) - 64) return FASTBCC_ERR_TOO_LARGE;
  if (num_arcs > 0 && (adj == nullptr || out_edge_label == nullptr)) return FASTBCC_ERR_INVALID_ARGUMENT;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return FASTBCC_ERR_HIP;
  int resident[kNumClasses];
  if (!resident_groups(dev, resident)) return FASTBCC_ERR_HIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int lo = -1;  // the first class also takes the empty graphs
  for (int c = 0; c < kNumClasses; ++c) {
    const SmallClass& k = kClasses[c];
    const int grid = num_packs < resident[c] ? num_packs : resident[c];
    bool reject = c == kNumClasses - 1;
    void* args[] = {(void*)&graph_vbegin, (void*)&num_graphs, (void*)&pack_begin,     (void*)&num_packs,
                    (void*)&n_total,      (void*)&num_arcs,   (void*)&offsets,        (void*)&adj,
                    (void*)&lo,           (void*)&reject,     (void*)&out_edge_label, (void*)&out_is_ap,
                    (void*)&out_num_bcc};
    if (hipLaunchKernel(k.kernel, dim3(grid), dim3(k.threads), args, 0, s) != hipSuccess) return FASTBCC_ERR_HIP;
    lo = k.max_n;
  }
  return FASTBCC_OK;
}

}  // extern "C"
