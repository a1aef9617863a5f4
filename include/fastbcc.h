/*
 * fastbcc -- biconnected components on one MI355X (gfx950), C ABI.
 *
 * The problem (paper: Introduction and Preliminaries): given an undirected
 * graph G = (V, E), partition E into biconnected components (BCCs) -- the
 * classes of "e1 ~ e2 iff e1 = e2 or both lie on a common simple cycle" --
 * and report the articulation points (vertices whose removal increases the
 * number of connected components).
 *
 * The method is FAST-BCC (paper: Section "The FAST-BCC Algorithm",
 * Algorithm 1): First-CC builds a spanning forest, Rooting roots it by an
 * Euler tour and list ranking, Tagging computes first/last/low/high per
 * vertex (low/high by range-min/max queries over preorder), Last-CC runs
 * connectivity on the implicit skeleton (plain tree edges and cross edges;
 * fence and back edges skipped), and every label gets its component head.
 * All of it runs as hand-written HIP kernels; this header is the only way in.
 *
 * Graph format: symmetric CSR.  offsets[n+1] (int32 or int64), adj[num_arcs]
 * (int32 vertex ids).  Every undirected edge u-w is stored as two arcs,
 * u->w in row u and w->u in row w.  Parallel edges are allowed (they always
 * share a BCC); self-loop arcs are allowed and get label -1.  Rows need not
 * be sorted for the solve (FASTBCC_FLAG_VALIDATE requires sorted rows);
 * FASTBCC_FLAG_SORTED_ROWS lets the edge-label read-out use that they are.
 *
 * Output conventions:
 *   out_edge_label[a]  smallest arc index of the BCC that arc a belongs to
 *                      (the "edge id" of an edge is the smaller of its two
 *                      arc indices, so both arcs of an edge get the same
 *                      value); -1 for a self-loop arc.
 *   out_is_ap[v]       1 if v is an articulation point, else 0.
 *   out_num_bcc[g]     number of BCCs (isolated vertices and self-loops form
 *                      none).
 *
 * Memory: every pointer argument is DEVICE memory unless marked (host).
 * All buffers -- inputs, outputs and the workspace -- are owned by the
 * caller.  The solve allocates nothing, keeps no state between calls, and
 * issues no host synchronisation (unless FASTBCC_FLAG_VALIDATE is set): it
 * only enqueues kernels on `stream`, so it may be captured into a HIP graph.
 * Calls on distinct workspaces may run concurrently on distinct streams.
 *
 * Limits: n < 2^30 vertices, num_arcs < 2^31 (labels are int32 arc ids).
 */
#ifndef FASTBCC_H
#define FASTBCC_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define FASTBCC_API __attribute__((visibility("default")))
#else
#define FASTBCC_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fastbcc_status {
  FASTBCC_OK = 0,
  FASTBCC_ERR_INVALID_ARGUMENT = 1,    /* null pointer, negative size, bad flag bits */
  FASTBCC_ERR_TOO_LARGE = 2,           /* n >= 2^30 or num_arcs >= 2^31 */
  FASTBCC_ERR_WORKSPACE_TOO_SMALL = 3, /* workspace_bytes < fastbcc_workspace_size() */
  FASTBCC_ERR_HIP = 4,                 /* a HIP launch or API call failed */
  FASTBCC_ERR_INVALID_GRAPH = 5,       /* FASTBCC_FLAG_VALIDATE found a malformed CSR */
  FASTBCC_ERR_SCRATCH_TOO_SMALL = 6    /* fastbcc_solve_noalloc: the graph's workspace exceeds
                                          FASTBCC_NOALLOC_SCRATCH_BYTES */
} fastbcc_status;

/* flags */
#define FASTBCC_FLAG_VALIDATE 0x1u /* check the CSR on the device first, then
                                      synchronise `stream` and return
                                      FASTBCC_ERR_INVALID_GRAPH if it is not a
                                      symmetric CSR with sorted rows and ids in
                                      range; nothing else is launched then */
#define FASTBCC_FLAG_SORTED_ROWS 0x2u /* the caller guarantees ascending rows:
                                         the edge-label read-out then finds
                                         reverse arcs by binary search instead
                                         of gathering per arc.  Unsorted rows
                                         with this flag give wrong labels (no
                                         access leaves its row). */
#define FASTBCC_FLAG_NO_SELF_LOOPS 0x4u /* the caller guarantees no arc v->v:
                                           with FASTBCC_FLAG_SORTED_ROWS the
                                           edge-label pass then writes labels
                                           without reading the adjacency (rows
                                           that need per-arc care still read
                                           it).  A self-loop with this flag
                                           gets a BCC label instead of -1;
                                           with FASTBCC_FLAG_VALIDATE it is
                                           reported as an invalid graph. */
#define FASTBCC_FLAG_REPAIR 0x8u /* fastbcc_check_batched only: rewrite every
                                     graph that failed into a valid one */
/* Tuning fields (0 = built-in default).  They change speed, never results.
 *   bits 8-11  log2 of the list-ranking ruler spacing, 3..10
 *   bits 12-13 union-find sampling rounds before the full sweep, 0..3 (value 3 = none)
 *   bits 14-16 log2 of 64-arc windows per wave tile, 2..6
 *   bit  17    First-CC union-find variant: 0 = hook the larger root id under
 *              the smaller, 1 = hook by hashed random priority
 *   bits 18-19 First-CC low-diameter decomposition (Miller-Peng-Xu, the LDD
 *              of the paper's LDD-UF-JTB connectivity) before union-find:
 *              0 = off, k = on with beta = 2^-k
 *   bit  20    Tagging from sampled tags: fences are certified from a few
 *              sampled neighbours per vertex (the tags of Section "Tagging"
 *              computed on a subset of the edges) and exact tags are swept
 *              only for the subtrees still undecided
 *   bits 21-22 sampled neighbours per vertex in that mode: 0 = 4, 1 = 2,
 *              2 = 3, 3 = 1
 *   bit  23    First-CC's first sampling round links each vertex to its
 *              sample only when the sample ranks above it, without atomics
 *   bit  24    Last-CC hooks by hashed priority, then relabels every set to
 *              its smallest member
 *   bits 25-26 Last-CC sampling rounds: 0 = as First-CC, k = k - 1 rounds
 *   bits 27-28 threads per block of the per-vertex kernels of the hot phases
 *              (union-find sampling, tag sampling and range queries, Last-CC
 *              tree and sampling passes, read-out searches): 0 = 256, 1 = 64,
 *              2 = 128, 3 = 512
 *   bit  29    flatten First-CC's sets after its atomic-free first round too
 *              (the next sampling round's finds then take one hop)
 *   bit  30    XCD-ordered per-vertex launches (and the Euler tour's per-node
 *              and per-ruler ones): each of the GPU's 8 XCDs (each with its
 *              own L2) takes one contiguous run of vertices or tour nodes,
 *              which keeps graph-local accesses (a batch's graphs, lattices)
 *              in one L2
 *   bit  31    batches only (fastbcc_solve_batched): First-CC and Last-CC
 *              per graph, one workgroup per graph running union-find over the
 *              graph's arcs (or its skeleton), parents in LDS for graphs of up
 *              to 2^16 vertices (larger ones in device memory, slowly),
 *              graphs taken largest first when there are no more graphs than
 *              vertices; for batches of many graphs, never for few huge ones;
 *              ignored by single-graph solves */
#define FASTBCC_TUNE_RULER_SHIFT 8
#define FASTBCC_TUNE_SAMPLE_SHIFT 12
#define FASTBCC_TUNE_TILE_SHIFT 14
#define FASTBCC_TUNE_CC_PRIORITY 0x20000u
#define FASTBCC_TUNE_LDD_SHIFT 18
#define FASTBCC_TUNE_SAMPLED_TAGS 0x100000u
#define FASTBCC_TUNE_TAG_SAMPLES_SHIFT 21
#define FASTBCC_TUNE_FREE_FIRST_ROUND 0x800000u
#define FASTBCC_TUNE_LCC_PRIORITY 0x1000000u
#define FASTBCC_TUNE_LCC_ROUNDS_SHIFT 25
#define FASTBCC_TUNE_VERTEX_BLOCK_SHIFT 27
#define FASTBCC_TUNE_COMPRESS_FREE_ROUND 0x20000000u
#define FASTBCC_TUNE_XCD_ORDER 0x40000000u
#define FASTBCC_TUNE_GRAPH_CC 0x80000000u

/*
 * Workspace bytes needed for a graph with n vertices and num_arcs arcs split
 * into num_graphs graphs (1 for a single graph).  O(n + num_arcs/4 +
 * num_graphs); independent of flags.  `bytes` is host memory.
 * The paper's space bound (Theorem on cost bounds: O(n) auxiliary words) is
 * kept up to bit-level bookkeeping: what grows with the number of arcs is at
 * most 1/4 byte per arc (arc tiles, sharded hub counters and one
 * descendant bit per arc that saves the edge-label pass a gather), against
 * the 4 bytes per arc of the input and of the output.
 */
FASTBCC_API fastbcc_status fastbcc_workspace_size(int64_t n, int64_t num_arcs, int32_t num_graphs, size_t* bytes);

/*
 * Solve one graph (Algorithm 1 of the paper plus the edge-label and
 * articulation-point read-out).  offsets: int32[n+1]; adj: int32[num_arcs];
 * out_edge_label: int32[num_arcs]; out_is_ap: uint8[n] (may be null);
 * out_num_bcc: int64[1] (may be null); workspace: >= fastbcc_workspace_size
 * bytes, 256-byte aligned; stream: a hipStream_t (null = default stream).
 * Asynchronous: returns after enqueueing.  Inputs must stay valid and
 * unmodified until the work on `stream` completes.
 */
FASTBCC_API fastbcc_status fastbcc_solve(int64_t n, int64_t num_arcs, const int32_t* offsets, const int32_t* adj,
                             int32_t* out_edge_label, uint8_t* out_is_ap, int64_t* out_num_bcc,
                             void* workspace, size_t workspace_bytes, uint32_t flags, void* stream);

/*
 * Allocation-free variant of fastbcc_solve, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  Same arguments, results and asynchrony as
 * fastbcc_solve, without the workspace: the library keeps one static
 * workspace of FASTBCC_NOALLOC_SCRATCH_BYTES per GPU (a __device__ array,
 * held from the code object's load on that GPU until the process ends) and
 * solves in it.  No call allocates or frees memory.  The device is the
 * current HIP device; `stream` must belong to it.
 *   - A graph whose fastbcc_workspace_size(n, num_arcs, 1) exceeds
 *     FASTBCC_NOALLOC_SCRATCH_BYTES is refused with
 *     FASTBCC_ERR_SCRATCH_TOO_SMALL before anything is enqueued (64 MiB hold,
 *     e.g., about 3 * 10^5 vertices with 2.4 * 10^6 arcs).
 *   - Every call on one GPU shares that GPU's scratch, which keeps the last
 *     call's contents (each solve initialises what it reads).  Calls whose
 *     work overlaps on one GPU -- on different streams, or from different
 *     threads without ordering -- race on it and give undefined results:
 *     order them on one stream, or use fastbcc_solve with a workspace each.
 *   - fastbcc_read_device_status and fastbcc_vertex_labels need a caller's
 *     workspace, so they do not apply to this entry point.
 */
#define FASTBCC_NOALLOC_SCRATCH_BYTES (64u << 20)
FASTBCC_API fastbcc_status fastbcc_solve_noalloc(int64_t n, int64_t num_arcs, const int32_t* offsets,
                                                 const int32_t* adj, int32_t* out_edge_label, uint8_t* out_is_ap,
                                                 int64_t* out_num_bcc, uint32_t flags, void* stream);

/* As fastbcc_solve, with int64 offsets (graphs whose arc count needs them
 * in memory layout; num_arcs must still be < 2^31). */
FASTBCC_API fastbcc_status fastbcc_solve_off64(int64_t n, int64_t num_arcs, const int64_t* offsets, const int32_t* adj,
                                   int32_t* out_edge_label, uint8_t* out_is_ap, int64_t* out_num_bcc,
                                   void* workspace, size_t workspace_bytes, uint32_t flags, void* stream);

/*
 * Solve many independent graphs in one launch sequence.  The graphs are
 * concatenated into one CSR: graph g owns vertices [graph_vbegin[g],
 * graph_vbegin[g+1]) and arcs [offsets[graph_vbegin[g]], offsets[graph_vbegin[g+1]]),
 * and its arcs hold GLOBAL vertex ids that stay inside its own range.
 * graph_vbegin: int32[num_graphs+1] on the device, graph_vbegin[0] = 0,
 * graph_vbegin[num_graphs] = n_total, nondecreasing.
 * Results are graph-local: out_edge_label[a] is the label graph g would get
 * if solved alone (its arc indices counted from offsets[graph_vbegin[g]]);
 * out_num_bcc: int64[num_graphs].  A BCC never spans two graphs (the paper
 * processes the connected components of a disconnected input in parallel),
 * so the union is solved as one graph and only the read-out is per graph.
 */
FASTBCC_API fastbcc_status fastbcc_solve_batched(int32_t num_graphs, const int32_t* graph_vbegin, int64_t n_total,
                                     int64_t num_arcs, const int32_t* offsets, const int32_t* adj,
                                     int32_t* out_edge_label, uint8_t* out_is_ap, int64_t* out_num_bcc,
                                     void* workspace, size_t workspace_bytes, uint32_t flags, void* stream);

/*
 * Batched solve of SMALL graphs by persistent fused kernels (paper:
 * Algorithm 1 -- First-CC, Rooting, Tagging, Last-CC and the head
 * assignment -- with the connected components of a disconnected input
 * solved in parallel): one workgroup solves a whole pack of consecutive
 * graphs as one disjoint union, every per-vertex array of every phase in
 * its LDS, and loops over the packs; one launch per size class (packs of up
 * to 256, 1024 and FASTBCC_SMALL_MAX_VERTICES vertices).  Same graph layout,
 * results (graph-local labels, AP flags, per-graph counts) and asynchrony as
 * fastbcc_solve_batched, but no workspace: nothing but the outputs is
 * written, and the call may be captured into a HIP graph.
 *   - pack_begin: int32[num_packs + 1] on the device, pack p = graphs
 *     [pack_begin[p], pack_begin[p + 1]), from 0 to num_graphs,
 *     nondecreasing; null = one graph per pack (num_packs ignored).  Packing
 *     many tiny graphs together pays the pipeline's fixed per-pack cost once.
 *   - A pack with more than FASTBCC_SMALL_MAX_VERTICES vertices or graphs (or
 *     whose vertex or arc range does not fit the arrays) is not solved: its
 *     graphs' out_num_bcc is -1 and their labels and AP flags are not
 *     written.
 *   - Arcs whose target lies outside their graph are ignored (label -1), as
 *     are self-loops (label -1).
 *   - flags: FASTBCC_FLAG_SORTED_ROWS and FASTBCC_FLAG_NO_SELF_LOOPS are
 *     accepted and not needed; any other bit is FASTBCC_ERR_INVALID_ARGUMENT.
 *   - out_is_ap may be null; out_edge_label may be null only when
 *     num_arcs == 0.  num_arcs >= 2^31 - 64 is FASTBCC_ERR_TOO_LARGE.
 */
#define FASTBCC_SMALL_MAX_VERTICES 3072
FASTBCC_API fastbcc_status fastbcc_solve_small(int32_t num_graphs, const int32_t* graph_vbegin, int32_t num_packs,
                                               const int32_t* pack_begin, int64_t n_total, int64_t num_arcs,
                                               const int32_t* offsets, const int32_t* adj, int32_t* out_edge_label,
                                               uint8_t* out_is_ap, int64_t* out_num_bcc, uint32_t flags,
                                               void* stream);

/*
 * BC-labeling read-out (paper: Section "Space-Efficient BCC Representation"
 * and the component heads of Algorithm 1).  Call after a solve on the same
 * workspace with the same n, num_arcs and graphs (enqueue on the solve's
 * stream or after it).  For every vertex v:
 *   out_home[v]      canonical id (smallest arc index, graph-local for
 *                    batches) of the BCC in which v is a non-head member;
 *   out_home_head[v] the head vertex of that BCC (graph-local for batches);
 * both -1 for a spanning-tree root (every isolated vertex is one).  Each BCC
 * c is {v : out_home[v] = c} plus the shared out_home_head of those v, so the
 * whole partition takes O(n) space.  Either output may be null.
 * graph_vbegin may be null when num_graphs == 1.  Device pointers.
 */
FASTBCC_API fastbcc_status fastbcc_vertex_labels(int64_t n, int64_t num_arcs, int32_t num_graphs,
                                                 const int32_t* graph_vbegin, const void* workspace,
                                                 size_t workspace_bytes, int32_t* out_home,
                                                 int32_t* out_home_head, void* stream);

/*
 * Batch assembly: graphs copied into one CSR with their own (graph-local)
 * ids and row starts get them made global in place.  Graph g owns vertices
 * [graph_vbegin[g], graph_vbegin[g+1]) and arcs [graph_abegin[g],
 * graph_abegin[g+1]); every arc of g gets graph_vbegin[g] added to its
 * target, every row start of g gets graph_abegin[g] added (offsets[n] is not
 * touched).  Both range arrays: int32[num_graphs + 1] on the device, from 0
 * to n and to num_arcs, nondecreasing.  Enqueue-only on `stream`.  (The
 * batched solve itself takes global ids; this is how a batch is built from
 * requests that arrive with local ones.)
 */
FASTBCC_API fastbcc_status fastbcc_batch_rebase(int32_t num_graphs, const int32_t* graph_vbegin,
                                                const int32_t* graph_abegin, int64_t n, int64_t num_arcs,
                                                int32_t* offsets, int32_t* adj, void* stream);

/*
 * Per-graph input check of a batch, for graphs from untrusted sources
 * (serving): enqueue-only on `stream`, no host synchronisation, nothing
 * allocated.  The layout is that of fastbcc_solve_batched (global ids;
 * graph_vbegin may be null when num_graphs == 1), and the caller vouches for
 * the layout itself: graph_vbegin runs from 0 to n without decreasing, and
 * the graphs' first row starts offsets[graph_vbegin[g]] run from 0 to
 * num_arcs without decreasing.  Everything inside a graph is checked, with
 * every access kept inside the arrays whatever they hold:
 *   - each row lies inside its graph's arc range, offsets nondecreasing;
 *   - each arc's target lies in its graph's vertex range;
 *   - with FASTBCC_FLAG_SORTED_ROWS, rows ascend; with
 *     FASTBCC_FLAG_NO_SELF_LOOPS, no arc v->v; with FASTBCC_FLAG_VALIDATE
 *     (needs FASTBCC_FLAG_SORTED_ROWS), every arc has its reverse.
 * out_graph_status[g] (int32[num_graphs], device) = 0 if graph g passed, else
 * FASTBCC_ERR_INVALID_GRAPH.  With FASTBCC_FLAG_REPAIR every graph that
 * failed is rewritten in place (offsets and adj): all its arcs become
 * self-loops of its first vertex and its other rows empty, so a batched solve
 * of the whole batch can follow at once, safely; the results of a failed
 * graph mean nothing and the caller drops them.  Graphs that passed are left
 * untouched.  Rows longer than 256 arcs are checked by a whole wave.
 */
FASTBCC_API fastbcc_status fastbcc_check_batched(int32_t num_graphs, const int32_t* graph_vbegin, int64_t n,
                                                 int64_t num_arcs, int32_t* offsets, int32_t* adj, uint32_t flags,
                                                 int32_t* out_graph_status, void* stream);

/*
 * The rest of the BC labeling of the last solve on `workspace` (paper:
 * Section "The BC-labeling Technique", Section "Space-Efficient BCC
 * Representation" and Algorithm 1's labels and heads), plus the bridges and
 * the block-cut tree.  Call after a solve on the same workspace, with the same
 * graph (n, num_arcs, graphs, offsets, adj) and that solve's outputs
 * edge_label and is_ap, enqueued on the solve's stream or after it.  It
 * overwrites workspace arrays the solve no longer needs; what
 * fastbcc_vertex_labels reads stays valid.  For every vertex v:
 *   out_label[v]      l[v], the paper's vertex label: the vertex that
 *                     represents v's Last-CC component (its smallest
 *                     member); the BCC labelled l is {u : l[u] = l} plus
 *                     its head; -1 for a spanning-tree root;
 *   out_parent[v]     parent of v in the solve's spanning forest (the tree
 *                     the labels refer to: head(l[u]) = p(u) whenever
 *                     l[u] != l[p(u)]); -1 for a root;
 *   out_cut_parent[v] for an articulation point v that is not a tree root:
 *                     the canonical id of the BCC in which v is a non-head
 *                     member, its parent in the block-cut tree; else -1.
 * The block-cut tree (a forest, one tree per connected component with an
 * edge): BCC nodes are canonical ids c, cut nodes are articulation points.
 * The parent of BCC node c is its head (out_home_head of
 * fastbcc_vertex_labels) when the head is an articulation point, else c is a
 * root; the parent of cut node v is out_cut_parent[v] (-1: v is a root,
 * a tree root heading two or more BCCs).  Each (cut vertex, BCC containing
 * it) pair is exactly one tree edge.
 * For every arc a:
 *   out_is_bridge[a]  1 if a belongs to a bridge, a BCC with exactly one
 *                     edge (parallel copies make a 2-cycle, not a bridge),
 *                     else 0 (0 for self-loops).
 * Vertex ids and canonical ids are graph-local in a batch.  offsets_bits is
 * 32 or 64; flags: FASTBCC_FLAG_SORTED_ROWS (rows are searched instead of
 * scanned), other bits ignored.  Outputs may be null (not computed);
 * out_is_bridge needs adj and edge_label, out_cut_parent needs is_ap.
 */
FASTBCC_API fastbcc_status fastbcc_bc_labeling(int64_t n, int64_t num_arcs, int32_t num_graphs,
                                               const int32_t* graph_vbegin, const void* offsets, int32_t offsets_bits,
                                               const int32_t* adj, const int32_t* edge_label, const uint8_t* is_ap,
                                               void* workspace, size_t workspace_bytes, uint32_t flags,
                                               int32_t* out_label, int32_t* out_parent, int32_t* out_cut_parent,
                                               uint8_t* out_is_bridge, void* stream);

/*
 * Synchronise `stream` and copy the device status word kept in `workspace`
 * (0 = fine; otherwise a fastbcc_status written by a device-side check) to
 * *out_status (host).
 */
FASTBCC_API fastbcc_status fastbcc_read_device_status(const void* workspace, void* stream, int32_t* out_status);

/*
 * Per-kernel timing (profiling aid).  A trace owns a pool of HIP events
 * (created by fastbcc_trace_create, freed by fastbcc_trace_destroy).
 * fastbcc_solve_traced enqueues the same kernels as the plain entry points
 * with an event pair around every launch; fastbcc_trace_collect waits for
 * the recorded events and adds each launch's duration to a per-kernel
 * total.  Launches beyond the pool's capacity are not timed (counted in
 * fastbcc_trace_dropped).  A trace must not be shared by concurrent solves.
 */
typedef struct fastbcc_trace fastbcc_trace;

FASTBCC_API fastbcc_trace* fastbcc_trace_create(int32_t max_launches);
FASTBCC_API void fastbcc_trace_destroy(fastbcc_trace* trace);
/* General solve with tracing: offsets_bits is 32 or 64; graph_vbegin may be
 * null when num_graphs == 1; other arguments as in fastbcc_solve_batched. */
FASTBCC_API fastbcc_status fastbcc_solve_traced(int32_t num_graphs, const int32_t* graph_vbegin, int64_t n,
                                                int64_t num_arcs, const void* offsets, int32_t offsets_bits,
                                                const int32_t* adj, int32_t* out_edge_label, uint8_t* out_is_ap,
                                                int64_t* out_num_bcc, void* workspace, size_t workspace_bytes,
                                                uint32_t flags, void* stream, fastbcc_trace* trace);
FASTBCC_API fastbcc_status fastbcc_trace_collect(fastbcc_trace* trace);
/* Number of distinct kernels seen; entry i: kernel name (static string),
 * summed milliseconds and number of timed launches (all host pointers). */
FASTBCC_API int32_t fastbcc_trace_count(const fastbcc_trace* trace);
FASTBCC_API fastbcc_status fastbcc_trace_entry(const fastbcc_trace* trace, int32_t i, const char** name,
                                               double* total_ms, int64_t* launches);
FASTBCC_API int64_t fastbcc_trace_dropped(const fastbcc_trace* trace);
FASTBCC_API void fastbcc_trace_reset(fastbcc_trace* trace);

/* Static string for a status code. */
FASTBCC_API const char* fastbcc_status_string(fastbcc_status status);

/* Library version as "major.minor.patch" (static string). */
FASTBCC_API const char* fastbcc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FASTBCC_H */
