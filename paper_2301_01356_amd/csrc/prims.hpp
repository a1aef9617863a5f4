// Device primitives for the FAST-BCC kernels (gfx950, wave64).
//
//  * wave helpers (64-bit shuffles, lane id)
//  * exclusive prefix scan over int32 (reduce -> spine -> downsweep), with an
//    optional element count read from device memory so a launch sequence
//    needs no host round trip for data-dependent sizes
//  * union-find on an acyclic parent array: find with path halving, link by
//    CAS of the larger root under the smaller one (so a set's root is its
//    smallest member) or, for connectivity that only needs some root, of the
//    lower hashed priority under the higher; variants record the edge behind
//    every successful hook (the spanning-forest by-product of connectivity,
//    paper: Section "Implementation Details", "Spanning Forest")
//  * arc tiles: a wave walks a contiguous range of arcs 64 at a time and
//    finds the source row of every arc by a shuffle binary search over 64
//    consecutive row ends, so every sweep over the CSR is arc-balanced and
//    reads adjacency coalesced no matter how skewed the degrees are.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fastbcc {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

__device__ __forceinline__ int64_t shfl64(int64_t v, int src) {
  int lo = __shfl((int)(uint32_t)(uint64_t)v, src, WAVE);
  int hi = __shfl((int)(uint32_t)((uint64_t)v >> 32), src, WAVE);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

__device__ __forceinline__ int ld_relaxed(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------ scan
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

// Exclusive scan of one value per thread over the block; `total` gets the sum.
__device__ __forceinline__ int block_exclusive_scan(int v, int* lds, int& total) {
  const int lane = lane_id(), wid = threadIdx.x / WAVE;
  int x = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    int y = __shfl_up(x, o, WAVE);
    if (lane >= o) x += y;
  }
  if (lane == WAVE - 1) lds[wid] = x;
  __syncthreads();
  int before = 0, sum = 0;
  const int nw = blockDim.x / WAVE;
  for (int w = 0; w < nw; ++w) {
    int s = lds[w];
    if (w < wid) before += s;
    sum += s;
  }
  __syncthreads();
  total = sum;
  return before + x - v;
}

__device__ __forceinline__ int64_t scan_count(int64_t max_count, const int* count_dev) {
  if (count_dev == nullptr) return max_count;
  int64_t c = (int64_t)*count_dev;
  return c < max_count ? (c < 0 ? 0 : c) : max_count;
}

__device__ __forceinline__ void load_items(const int* in, int64_t base, int64_t count, int (&v)[SCAN_ITEMS]) {
  if (base + SCAN_ITEMS <= count) {
    const int4* p = reinterpret_cast<const int4*>(in + base);
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS / 4; ++k) {
      int4 q = p[k];
      v[4 * k] = q.x; v[4 * k + 1] = q.y; v[4 * k + 2] = q.z; v[4 * k + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) v[k] = (base + k < count) ? in[base + k] : 0;
  }
}

__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_reduce(const int* __restrict__ in, int64_t max_count,
                                                             const int* count_dev, int* __restrict__ bsum) {
  __shared__ int lds[SCAN_BLOCK / WAVE];
  const int64_t count = scan_count(max_count, count_dev);
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  load_items(in, base, count, v);
  int s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) s += v[k];
  int total;
  block_exclusive_scan(s, lds, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// One block scans the per-block sums in place (exclusive) and stores the total.
__global__ void __launch_bounds__(1024) k_scan_spine(int* __restrict__ bsum, int nblocks, int* total_out) {
  __shared__ int lds[1024 / WAVE];
  int carry = 0;
  for (int base = 0; base < nblocks; base += 1024 * 4) {
    int v[4];
    int s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int i = base + threadIdx.x * 4 + k;
      v[k] = i < nblocks ? bsum[i] : 0;
      s += v[k];
    }
    int tot;
    int ex = block_exclusive_scan(s, lds, tot) + carry;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int i = base + threadIdx.x * 4 + k;
      if (i < nblocks) bsum[i] = ex;
      ex += v[k];
    }
    carry += tot;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_down(const int* in, int* out, int64_t max_count,
                                                           const int* count_dev, const int* __restrict__ bsum) {
  __shared__ int lds[SCAN_BLOCK / WAVE];
  const int64_t count = scan_count(max_count, count_dev);
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  load_items(in, base, count, v);
  int s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) s += v[k];
  int total;
  int ex = block_exclusive_scan(s, lds, total) + bsum[blockIdx.x];
  if (base + SCAN_ITEMS <= count) {
    int4* p = reinterpret_cast<int4*>(out + base);
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS / 4; ++k) {
      int4 q;
      q.x = ex; ex += v[4 * k];
      q.y = ex; ex += v[4 * k + 1];
      q.z = ex; ex += v[4 * k + 2];
      q.w = ex; ex += v[4 * k + 3];
      p[k] = q;
    }
  } else {
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
      if (base + k < count) out[base + k] = ex;
      ex += v[k];
    }
  }
}

// ------------------------------------------------------------ union-find
// Parent pointers form a forest (every hook puts a root under another
// set's root), so find loops always end.
__device__ __forceinline__ int uf_find(int* p, int x) {
  int px = ld_relaxed(p + x);
  while (px != x) {
    int gx = ld_relaxed(p + px);
    if (gx == px) return px;
    st_relaxed(p + x, gx);  // path halving: an ancestor of x, same set
    x = gx;
    px = ld_relaxed(p + x);
  }
  return x;
}

// Root of x without writing anything.  Used where one pass must leave every
// entry pointing at its root: path-halving writes of concurrent finds can
// store a stale ancestor over an entry that its own thread had just set to
// the root, so a flattening pass that needs a guarantee reads only and writes
// nothing but its own entry.
__device__ __forceinline__ int uf_root_ro(const int* p, int x) {
  int px = ld_relaxed(p + x);
  while (px != x) {
    x = px;
    px = ld_relaxed(p + x);
  }
  return x;
}

// Union by CAS: the larger root goes under the smaller one.  Two vertices
// with the same parent are in the same set: that common case returns without
// touching the (hot) root slot.
__device__ __forceinline__ void uf_link(int* p, int u, int v) {
  if (ld_relaxed(p + u) == ld_relaxed(p + v)) return;
  int ru = uf_find(p, u), rv = uf_find(p, v);
  while (ru != rv) {
    int hi = ru > rv ? ru : rv, lo = ru > rv ? rv : ru;
    // test before the CAS: when many threads race to hook the same root,
    // only the ones that still see it as a root pay for an atomic
    if (ld_relaxed(p + hi) == hi && atomicCAS(p + hi, hi, lo) == hi) return;
    ru = uf_find(p, ru);
    rv = uf_find(p, rv);
  }
}

// As uf_link; a successful hook of root h stores the edge (u, v) at h (one
// 8-byte store: the two ends share a line).  At the CAS, u's set (rooted at
// the hooked root) and v's set are disjoint, so the recorded edges form a
// spanning forest.
__device__ __forceinline__ void uf_link_record(int* p, int u, int v, int2* hook) {
  if (ld_relaxed(p + u) == ld_relaxed(p + v)) return;
  int ru = uf_find(p, u), rv = uf_find(p, v);
  while (ru != rv) {
    int hi = ru > rv ? ru : rv, lo = ru > rv ? rv : ru;
    if (ld_relaxed(p + hi) == hi && atomicCAS(p + hi, hi, lo) == hi) {
      hook[hi] = make_int2(u, v);
      return;
    }
    ru = uf_find(p, ru);
    rv = uf_find(p, rv);
  }
}

// Hook by hashed priority instead of by id: the root whose (bijectively
// mixed) id is smaller goes under the other.  Roots are then arbitrary
// members, which connectivity with forest recording allows, and structured
// ids (lattices, chains) no longer line up into long hook chains.  The mixer
// is the 32-bit finaliser "fmix32" of Austin Appleby's public-domain
// MurmurHash3 (xor-shift 16, multiply, xor-shift 13, multiply, xor-shift
// 16); every step is invertible, so distinct ids get distinct priorities.
__device__ __forceinline__ uint32_t uf_prio(int x) {
  uint32_t h = (uint32_t)x;
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

__device__ __forceinline__ void uf_link_prio(int* p, int u, int v) {
  if (ld_relaxed(p + u) == ld_relaxed(p + v)) return;
  int ru = uf_find(p, u), rv = uf_find(p, v);
  while (ru != rv) {
    const bool u_low = uf_prio(ru) < uf_prio(rv);
    const int lo = u_low ? ru : rv, hi = u_low ? rv : ru;
    if (ld_relaxed(p + lo) == lo && atomicCAS(p + lo, lo, hi) == lo) return;
    ru = uf_find(p, ru);
    rv = uf_find(p, rv);
  }
}

__device__ __forceinline__ void uf_link_record_prio(int* p, int u, int v, int2* hook) {
  if (ld_relaxed(p + u) == ld_relaxed(p + v)) return;
  int ru = uf_find(p, u), rv = uf_find(p, v);
  while (ru != rv) {
    const bool u_low = uf_prio(ru) < uf_prio(rv);
    const int lo = u_low ? ru : rv, hi = u_low ? rv : ru;
    if (ld_relaxed(p + lo) == lo && atomicCAS(p + lo, lo, hi) == lo) {
      hook[lo] = make_int2(u, v);
      return;
    }
    ru = uf_find(p, ru);
    rv = uf_find(p, rv);
  }
}

// ------------------------------------------------------------- arc tiles
// A wave owns arcs [t*tile_arcs, (t+1)*tile_arcs).  tile_row[t] is the row
// containing the tile's first arc.  `body(a, x, ok)` is called by all 64
// lanes for every 64-arc window; ok says whether arc a (source row x) exists.
template <typename OffT, typename Body>
__device__ __forceinline__ void arc_tiles(const OffT* __restrict__ off, int n, int64_t A,
                                          const int* __restrict__ tile_row, int tile_windows, Body&& body) {
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t tile_arcs = (int64_t)WAVE * tile_windows;
  const int64_t tbeg = wave * tile_arcs;
  if (tbeg >= A) return;
  const int64_t tend = tbeg + tile_arcs < A ? tbeg + tile_arcs : A;
  int row = tile_row[wave];
  for (int64_t base = tbeg; base < tend; base += WAVE) {
    const int64_t a = base + lane;
    int my_row = -1;
    int lo = row;
    while (lo < n) {
      int idx = lo + 1 + lane;
      idx = idx < n ? idx : n;
      const int64_t e = (int64_t)off[idx];  // end of row lo + lane
      const int64_t e_last = shfl64(e, WAVE - 1);
      // pos = number of the 64 row ends that are <= a (0..64)
      int pos = 0;
#pragma unroll
      for (int step = 32; step >= 1; step >>= 1) {
        int64_t ej = shfl64(e, pos + step - 1);
        if (ej <= a) pos += step;
      }
      if (pos == WAVE - 1 && e_last <= a) pos = WAVE;
      if (my_row < 0 && pos < WAVE) my_row = lo + pos;
      const bool need = (a < tend) && my_row < 0;
      if (!__any(need)) break;
      lo += WAVE;
    }
    const bool ok = (a < tend) && my_row >= 0 && my_row < n;
    body(a, ok ? my_row : -1, ok);
    int last = __shfl(my_row, WAVE - 1, WAVE);
    row = last >= 0 ? last : row;
  }
}

// The same tiling for sweeps over the arcs themselves, software-pipelined:
// the next window's targets and row ends are loaded before the current
// window's body runs, so the body's gathers overlap them (vector loads of a
// wave return in issue order, so a load is only useful early if nothing the
// wave waits for before it was issued later).  `body(a, x, ok, y)` also gets
// y = adj[a], loaded nontemporally (the adjacency is streamed once).
template <typename Body>
__device__ __forceinline__ void arc_windows(const int* __restrict__ off, const int* __restrict__ adj, int n,
                                            int64_t A, const int* __restrict__ tile_row, int tile_windows,
                                            Body&& body) {
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t tile_arcs = (int64_t)WAVE * tile_windows;
  const int64_t tbeg = wave * tile_arcs;
  if (tbeg >= A) return;
  const int64_t tend = tbeg + tile_arcs < A ? tbeg + tile_arcs : A;
  int row = tile_row[wave];
  int y = tbeg + lane < tend ? __builtin_nontemporal_load(adj + tbeg + lane) : -1;
  int e = 0;
  if (row < n) e = off[row + 1 + lane < n ? row + 1 + lane : n];
  for (int64_t base = tbeg; base < tend; base += WAVE) {
    const int64_t a = base + lane;
    int my_row = -1;
    int lo = row;
    int ev = e;  // end of row lo + lane
    while (lo < n) {
      const int64_t e_last = __shfl(ev, WAVE - 1, WAVE);
      int pos = 0;  // number of the 64 row ends that are <= a (0..64)
#pragma unroll
      for (int step = 32; step >= 1; step >>= 1) {
        const int64_t ej = __shfl(ev, pos + step - 1, WAVE);
        if (ej <= a) pos += step;
      }
      if (pos == WAVE - 1 && e_last <= a) pos = WAVE;
      if (my_row < 0 && pos < WAVE) my_row = lo + pos;
      const bool need = (a < tend) && my_row < 0;
      if (!__any(need)) break;
      lo += WAVE;
      if (lo < n) ev = off[lo + 1 + lane < n ? lo + 1 + lane : n];
    }
    const bool ok = (a < tend) && my_row >= 0 && my_row < n;
    const int last = __shfl(my_row, WAVE - 1, WAVE);
    row = last >= 0 ? last : row;
    // next window: its targets and the row ends from its first row on
    const int64_t an = a + WAVE;
    const int yn = an < tend ? __builtin_nontemporal_load(adj + an) : -1;
    int en = 0;
    if (base + WAVE < tend && row < n) en = off[row + 1 + lane < n ? row + 1 + lane : n];
    body(a, ok ? my_row : -1, ok, y);
    y = yn;
    e = en;
  }
}

// Row of every arc of one window, from the 64 row ends starting at `row`
// (held in `e`, loaded by the caller).  Only a window spanning more than 64
// rows takes the branch that loads further blocks of row ends.
__device__ __forceinline__ int window_pos(int ev, int64_t a) {
  // number of the 64 row ends in ev that are <= a (0..64)
  const int64_t e_last = __shfl(ev, WAVE - 1, WAVE);
  int pos = 0;
#pragma unroll
  for (int step = 32; step >= 1; step >>= 1) {
    const int64_t ej = __shfl(ev, pos + step - 1, WAVE);
    if (ej <= a) pos += step;
  }
  if (pos == WAVE - 1 && e_last <= a) pos = WAVE;
  return pos;
}

__device__ __forceinline__ int window_row(const int* __restrict__ off, int n, int64_t a, int64_t tend, int row,
                                          int e) {
  const int pos = window_pos(e, a);
  int my_row = pos < WAVE ? row + pos : -1;
  if (__any(a < tend && my_row < 0)) {
    const int lane = lane_id();
    for (int lo = row + WAVE; lo < n; lo += WAVE) {
      const int ev = off[lo + 1 + lane < n ? lo + 1 + lane : n];
      const int p = window_pos(ev, a);
      if (my_row < 0 && p < WAVE) my_row = lo + p;
      if (!__any(a < tend && my_row < 0)) break;
    }
  }
  return my_row;
}

// arc_windows pipelined two windows deep: while window k's body waits for
// its per-row gathers (`fetch(x, y, ok)`, issued one window earlier), window
// k+1's rows are already found and its gathers are in flight.  A wave's vector
// loads complete in issue order and the compiler can only wait for them by
// count, so every load here is unconditional (out-of-range lanes read a
// clamped address and ignore the value) and the loop is unrolled twice with
// one register set per parity: no branch and no register copy of a value in
// flight forces a wait for all loads.  body(a, x, ok, y, fetched).
template <typename Fetch, typename Body>
__device__ __forceinline__ void arc_windows2(const int* __restrict__ off, const int* __restrict__ adj, int n,
                                             int64_t A, const int* __restrict__ tile_row, int tile_windows,
                                             Fetch&& fetch, Body&& body) {
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t tile_arcs = (int64_t)WAVE * tile_windows;
  const int64_t tbeg = wave * tile_arcs;
  if (tbeg >= A) return;
  const int64_t tend = tbeg + tile_arcs < A ? tbeg + tile_arcs : A;
  auto row_ends = [&](int r) {  // r < n
    const int idx = r + 1 + lane;
    return off[idx < n ? idx : n];
  };
  auto target = [&](int64_t a) {
    return __builtin_nontemporal_load(adj + (a < tend ? a : tend - 1));
  };
  using F = decltype(fetch(0, 0, false));
  int row = tile_row[wave];
  int eA = row_ends(row);
  int yA = target(tbeg + lane);
  int xA = window_row(off, n, tbeg + lane, tend, row, eA);
  bool okA = tbeg + lane < tend && xA >= 0 && xA < n;
  int last = __shfl(xA, WAVE - 1, WAVE);
  row = last >= 0 ? last : row;
  int eB = row_ends(row);
  int yB = target(tbeg + WAVE + lane);
  F fA = fetch(okA ? xA : 0, yA, okA), fB;
  int xB = -1;
  bool okB = false;
  int64_t base = tbeg;
  // one window: find the next window's rows, load the window after next,
  // fetch for the next window, then run this window's body
  auto step = [&](int& xc, bool& okc, int& yc, F& fc, int& ec, int& xn, bool& okn, int& yn, F& fn, int& en) {
    const int64_t an = base + WAVE + lane;
    xn = window_row(off, n, an, tend, row, en);
    okn = an < tend && xn >= 0 && xn < n;
    last = __shfl(xn, WAVE - 1, WAVE);
    row = last >= 0 ? last : row;
    ec = row_ends(row);
    fn = fetch(okn ? xn : 0, yn, okn);
    body(base + lane, okc ? xc : -1, okc, yc, fc);
    yc = target(base + 2 * WAVE + lane);
    base += WAVE;
  };
  for (;;) {
    step(xA, okA, yA, fA, eA, xB, okB, yB, fB, eB);
    if (base >= tend) break;
    step(xB, okB, yB, fB, eB, xA, okA, yA, fA, eA);
    if (base >= tend) break;
  }
}

}  // namespace fastbcc
