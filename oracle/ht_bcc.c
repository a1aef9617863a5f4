/*
 * CPU oracle for biconnected components -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg may load
 * this code.  The product path never calls it and shares nothing with it.
 *
 * What it computes (the plain definition, reached by the textbook method):
 *   The biconnected components (BCCs) of an undirected graph are the classes
 *   of edges under "e1 ~ e2 iff e1 = e2 or both lie on one simple cycle";
 *   equivalently the maximal subgraphs that stay connected after deleting any
 *   single vertex (paper: Introduction / Preliminaries, definitions of BCC,
 *   articulation point and bridge).  An articulation point is a vertex whose
 *   removal increases the number of connected components.
 *
 * How: the sequential Hopcroft-Tarjan algorithm (paper, Section "Existing BCC
 * Algorithms", subsection "The Hopcroft-Tarjan Algorithm"): a depth-first
 * search assigns each vertex its preorder number first[v] and
 *   low[v] = min over the DFS subtree of v of w1[u],
 *   w1[u]   = min({first[u]} U {first[u'] : u-u' a non-tree edge});
 * edges are pushed on a stack as they are first traversed, and when a child u
 * of v returns with low[u] >= first[v] the stack is popped down to the tree
 * edge v-u: the popped edges form one BCC.  v is an articulation point when
 * this happens for a non-root v, or at least twice for the DFS root.
 *
 * Output conventions (readings of the paper stated in the design notes):
 *   - arcs: the CSR stores each undirected edge as two arcs (u->w in row u,
 *     w->u in row w); the id of an edge is the smaller of its two arc indices;
 *   - out_label[a] = smallest edge id in the BCC of arc a, the same for both
 *     arcs of an edge; -1 for self-loop arcs;
 *   - out_ap[v] = 1 iff v is an articulation point;
 *   - isolated vertices and self-loops belong to no BCC and are not counted;
 *   - parallel copies of an edge form a 2-cycle, hence share a BCC.
 *
 * The DFS is iterative (explicit frame stack) so paths of millions of
 * vertices do not overflow the C stack.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

typedef struct {
  int32_t nbr;
  int64_t arc;
} nbr_arc;

static int cmp_nbr_arc(const void* a, const void* b) {
  const nbr_arc* x = (const nbr_arc*)a;
  const nbr_arc* y = (const nbr_arc*)b;
  if (x->nbr != y->nbr) return x->nbr < y->nbr ? -1 : 1;
  return x->arc < y->arc ? -1 : (x->arc > y->arc);
}

/*
 * rev[a] = index of the reverse arc of a.  Within every row, arcs are taken
 * in ascending (neighbour, arc index) order; for u ascending, each arc u->w
 * with w > u is paired with the next unpaired arc w->u of row w.  Parallel
 * copies are thereby paired in order.  Self-loop arcs pair with themselves.
 * Returns 0, or -1 when the CSR is not symmetric (an arc has no reverse).
 */
static int pair_reverse_arcs(int64_t n, const int64_t* off, const int32_t* adj, int64_t* rev) {
  int64_t A = off[n];
  int sorted = 1;
  for (int64_t u = 0; u < n && sorted; ++u)
    for (int64_t a = off[u] + 1; a < off[u + 1]; ++a)
      if (adj[a - 1] > adj[a]) { sorted = 0; break; }
  /* order[k] = arc at sorted position k (identity when rows are sorted) */
  int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(A > 0 ? A : 1));
  if (!order) return -2;
  if (sorted) {
    for (int64_t a = 0; a < A; ++a) order[a] = a;
  } else {
    nbr_arc* tmp = NULL;
    int64_t cap = 0;
    for (int64_t u = 0; u < n; ++u) {
      int64_t d = off[u + 1] - off[u];
      if (d > cap) {
        cap = d;
        free(tmp);
        tmp = (nbr_arc*)malloc(sizeof(nbr_arc) * (size_t)cap);
        if (!tmp) { free(order); return -2; }
      }
      for (int64_t k = 0; k < d; ++k) { tmp[k].nbr = adj[off[u] + k]; tmp[k].arc = off[u] + k; }
      qsort(tmp, (size_t)d, sizeof(nbr_arc), cmp_nbr_arc);
      for (int64_t k = 0; k < d; ++k) order[off[u] + k] = tmp[k].arc;
    }
    free(tmp);
  }
  for (int64_t a = 0; a < A; ++a) rev[a] = -1;
  /* cur[w]: next sorted position in row w whose arc points to a smaller vertex */
  int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!cur) { free(order); return -2; }
  for (int64_t w = 0; w < n; ++w) cur[w] = off[w];
  int ok = 1;
  for (int64_t u = 0; u < n && ok; ++u) {
    for (int64_t k = off[u]; k < off[u + 1]; ++k) {
      int64_t a = order[k];
      int32_t w = adj[a];
      if (w < 0 || w >= n) { ok = 0; break; }
      if (w == u) { rev[a] = a; continue; }
      if (w < u) continue;
      int64_t pos = cur[w];
      if (pos >= off[w + 1] || adj[order[pos]] != (int32_t)u) { ok = 0; break; }
      int64_t b = order[pos];
      rev[a] = b;
      rev[b] = a;
      cur[w] = pos + 1;
    }
  }
  for (int64_t a = 0; a < A && ok; ++a)
    if (rev[a] < 0) ok = 0;
  free(cur);
  free(order);
  return ok ? 0 : -1;
}

/*
 * Hopcroft-Tarjan BCC.  offsets int64[n+1], adj int32[offsets[n]], symmetric.
 * Outputs: out_label int32[A], out_ap uint8[n], *out_num_bcc.
 * Timings (seconds) of the reverse-arc pairing ("prep") and of the DFS with
 * labelling ("ht") are stored when the pointers are non-null.
 * Returns 0 on success, -1 for a non-symmetric or out-of-range CSR, -2 when
 * memory runs out.
 */
int ht_bcc(int64_t n, const int64_t* off, const int32_t* adj, int32_t* out_label, uint8_t* out_ap,
           int64_t* out_num_bcc, double* prep_s, double* ht_s) {
  int64_t A = off[n];
  double t0 = now_s();
  int64_t* rev = (int64_t*)malloc(sizeof(int64_t) * (size_t)(A > 0 ? A : 1));
  if (!rev) return -2;
  int rc = pair_reverse_arcs(n, off, adj, rev);
  if (rc != 0) { free(rev); return rc; }
  double t1 = now_s();

  int64_t* first = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* low = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  /* DFS frame per depth: vertex, next arc to scan, arc used to enter it */
  int64_t* fv = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* fcur = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* fin = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  /* edge stack holds arcs in traversal direction; each edge pushed once */
  int64_t* stk = (int64_t*)malloc(sizeof(int64_t) * (size_t)(A / 2 + 1));
  if (!first || !low || !fv || !fcur || !fin || !stk) {
    free(rev); free(first); free(low); free(fv); free(fcur); free(fin); free(stk);
    return -2;
  }
  for (int64_t v = 0; v < n; ++v) { first[v] = -1; out_ap[v] = 0; }
  for (int64_t a = 0; a < A; ++a) out_label[a] = -1;
  int64_t timer = 0, nbcc = 0, sp = 0;

  for (int64_t s = 0; s < n; ++s) {
    if (first[s] >= 0 || off[s + 1] == off[s]) continue;
    int64_t depth = 0, root_children = 0;
    fv[0] = s; fcur[0] = off[s]; fin[0] = -1;
    first[s] = low[s] = timer++;
    while (depth >= 0) {
      int64_t v = fv[depth];
      if (fcur[depth] < off[v + 1]) {
        int64_t a = fcur[depth]++;
        int64_t w = adj[a];
        if (w == v) continue;                                 /* self-loop */
        if (fin[depth] >= 0 && a == rev[fin[depth]]) continue; /* the tree edge back up */
        if (first[w] < 0) {                                   /* tree edge: descend */
          stk[sp++] = a;
          ++depth;
          fv[depth] = w; fcur[depth] = off[w]; fin[depth] = a;
          first[w] = low[w] = timer++;
        } else if (first[w] < first[v]) {                     /* back edge to an ancestor */
          stk[sp++] = a;
          if (first[w] < low[v]) low[v] = first[w];
        }
        /* first[w] > first[v]: already pushed from w's side */
      } else {
        /* v is finished: return to its parent */
        int64_t ein = fin[depth];
        --depth;
        if (depth < 0) break;
        int64_t p = fv[depth];
        if (low[v] < low[p]) low[p] = low[v];
        if (low[v] >= first[p]) {
          /* pop one BCC: down to and including the tree arc p->v */
          int64_t lab = INT64_MAX, base = sp;
          do {
            --base;
            int64_t e = stk[base];
            int64_t id = e < rev[e] ? e : rev[e];
            if (id < lab) lab = id;
          } while (stk[base] != ein);
          for (int64_t k = base; k < sp; ++k) {
            int64_t e = stk[k];
            out_label[e] = (int32_t)lab;
            out_label[rev[e]] = (int32_t)lab;
          }
          sp = base;
          ++nbcc;
          if (depth > 0) out_ap[p] = 1;
          else if (++root_children >= 2) out_ap[p] = 1;
        }
      }
    }
  }
  double t2 = now_s();
  *out_num_bcc = nbcc;
  if (prep_s) *prep_s = t1 - t0;
  if (ht_s) *ht_s = t2 - t1;
  free(rev); free(first); free(low); free(fv); free(fcur); free(fin); free(stk);
  return 0;
}
