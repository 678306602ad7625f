/* pierce.h - C ABI of the MI355X mesh-join refinement library (libpierce_hip.so).
 *
 * The library implements the refinement step of a 3D spatial join over closed
 * triangle meshes by the edge-as-segment reformulation of Pierce (arXiv
 * 2609.24513): the unique edges of each mesh of a candidate pair are cast as
 * segments against a BVH built over the other mesh's triangles (Section 3.1,
 * Steps I and II), in both directions (Section 3.2, "Bidirectional tracing").
 * Decisions use closed sets on the exact values of the FP32 coordinates, so a
 * pair is TRUE iff the two triangulated surfaces share at least one point
 * (touching counts); this equals an exact triangle-triangle test over all
 * triangle pairs.
 *
 * Conventions shared by every entry point:
 *  - Pointers documented "dev" are device pointers (HIP global memory) owned
 *    by the caller; "host" pointers are ordinary host memory.  The library
 *    never allocates or frees memory in these calls; scratch space comes
 *    from the caller's workspace `ws` (refine_intersects_static: from a
 *    static device buffer of the library).  The only state kept between
 *    calls is a per-device cache of launch figures (compute-unit count,
 *    resident blocks per compute unit of each persistent kernel) and of the
 *    static buffer's address, filled on first use.
 *  - Work is enqueued on `stream` (a hipStream_t passed as void*); nothing
 *    synchronises the host.  Results are valid once the stream has reached
 *    the end of the call.
 *  - Return value: PR_OK (0) or a negative PR_E_* code.  Argument errors that
 *    the host can see are reported before any work is enqueued (PR_E_ARG,
 *    PR_E_CAPACITY for a too-small workspace or blob).  A HIP runtime failure
 *    returns PR_E_DEVICE.  pr_last_error() gives a message for the calling
 *    thread's last failure.
 *  - Errors found on the device (bad geometry) are written to a caller-owned
 *    device status word, read by the caller after synchronising.
 *  - Calls are reentrant; blobs are immutable after their build and may be
 *    read by several concurrent calls on different streams.
 */
#ifndef PIERCE_H
#define PIERCE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PR_ABI_VERSION 8

enum {
  PR_OK = 0,
  PR_E_ARG = -1,        /* invalid argument (null pointer, negative size, bad params) */
  PR_E_CAPACITY = -2,   /* blob or workspace smaller than the size query returned */
  PR_E_GEOMETRY = -3,   /* device status: non-finite coordinate, bad face id, degenerate triangle */
  PR_E_DEVICE = -4,     /* HIP runtime error; pr_last_error() has hipGetErrorString */
  PR_E_UNSUPPORTED = -5 /* size beyond the library's index ranges, or blob/params mismatch */
};

/* Message describing the calling thread's most recent failure ("" if none). */
const char* pr_last_error(void);

/* PR_ABI_VERSION of the loaded library. */
int pr_abi_version(void);

/* ------------------------------------------------------------------------ */
/* BVH build (Section 3.1 Step I edge preparation; Section 2 BVH; the build
 * replaces the paper's per-dataset acceleration-structure build, Section 4.1).
 *
 * One blob holds, for every mesh of a dataset: its exact box, a width-W BVH
 * (W in {2,4,8}) over its triangles with at most `leaf_size` (1,2,4,8)
 * triangles per leaf, the triangles in leaf order, and its unique edges
 * (pairs of vertex ids, deduplicated within the mesh as in Section 3.1)
 * stored as FP32 segment endpoints in groups of 64.  The blob contains only
 * offsets, never pointers, so it can be copied or moved as raw bytes.
 */
typedef struct {
  int32_t width;      /* 2, 4 or 8 children per node */
  int32_t leaf_size;  /* 1, 2, 4 or 8 triangles per leaf at most */
  int32_t builder;    /* LBVH (Morton order, Karras radix tree) collapsed to width W by
                         greedy expansion: 0 opens the child of largest surface area,
                         1 the child of largest surface area x triangle count (its term
                         of the surface-area cost) */
  int32_t reserved;   /* must be 0 */
} pr_bvh_params;

/* Upper bounds, in bytes, of the blob and of the build workspace for a
 * dataset of n_meshes meshes with f_total faces and v_total vertices.
 * Returns PR_OK or PR_E_ARG / PR_E_UNSUPPORTED (f_total >= 2^28,
 * v_total >= 2^31, n_meshes >= 2^24) / PR_E_DEVICE. */
int build_mesh_bvh_sizes(int64_t n_meshes, int64_t f_total, int64_t v_total,
                         const pr_bvh_params* params, size_t* blob_bytes, size_t* ws_bytes);

/* The blob bound alone: bytes of the blob of such a dataset (an upper
 * bound), or 0 when the arguments are rejected (pr_last_error says why). */
size_t build_mesh_bvh_bytes(int64_t n_meshes, int64_t f_total, int64_t v_total,
                            const pr_bvh_params* params);

/* Builds the blob of a dataset.
 *  verts     dev f32[v_total][3]    vertex coordinates
 *  vert_off  dev i64[n_meshes+1]    mesh m owns verts[vert_off[m] .. vert_off[m+1])
 *  faces     dev i32[f_total][3]    vertex ids local to the face's mesh
 *  face_off  dev i64[n_meshes+1]    mesh m owns faces[face_off[m] .. face_off[m+1])
 *  params    host                   see pr_bvh_params
 *  blob      dev, blob_bytes        output; at least build_mesh_bvh_sizes' bound
 *  ws        dev, ws_bytes          scratch; at least build_mesh_bvh_sizes' bound
 *  dev_status dev i32[1]            out: -1 if the geometry is valid, else the
 *                                   smallest global face index that has an id
 *                                   out of range, a non-finite coordinate or
 *                                   three exactly collinear vertices (the paper
 *                                   leaves degenerate triangles to
 *                                   preprocessing, Section 3.6).  The blob
 *                                   must not be used when it is not -1.
 * Offsets must be non-decreasing with vert_off[0] = face_off[0] = 0; a mesh may
 * have zero faces (it then never intersects anything). */
int build_mesh_bvh(const float* verts, const int64_t* vert_off, const int32_t* faces,
                   const int64_t* face_off, int64_t n_meshes, int64_t v_total, int64_t f_total,
                   const pr_bvh_params* params, void* blob, size_t blob_bytes, void* ws,
                   size_t ws_bytes, int32_t* dev_status, void* stream);

/* Copies the exact per-mesh boxes out of a blob:
 * boxes dev f32[n_meshes][6] = (lo_x, lo_y, lo_z, hi_x, hi_y, hi_z). */
int blob_mesh_boxes(const void* blob, int64_t n_meshes, float* boxes, void* stream);

/* Copies each mesh's unique-edge count out of a blob: counts dev i32[n_meshes]. */
int blob_edge_counts(const void* blob, int64_t n_meshes, int32_t* counts, void* stream);

/* Copies the exponent range of the blob's coordinates: exps dev i32[2] =
 * (lowest exponent of a set bit, highest exponent of a set bit) over every
 * non-zero coordinate of every face; (INT32_MAX, INT32_MIN) when there is
 * none.  Two blobs whose joint range spans at most 14 (highest - lowest)
 * lie on one small power-of-two grid: refinement precision 3 then decides
 * every test the FP32 filter leaves open exactly, in place. */
int blob_coord_exponents(const void* blob, int32_t* exps, void* stream);

/* ------------------------------------------------------------------------ */
/* Candidate filter (the classic filter step that the paper's single traversal
 * fuses with refinement, Section 1 "Challenges" and Section 3 introduction).
 *
 * Writes every (i, j), i a mesh of blob_a and j a mesh of blob_b, whose
 * closed boxes overlap on all three axes (touching boxes are candidates), and,
 * when query_box is given, whose boxes both overlap the closed query box and
 * whose common box part meets it.  Output is sorted by (i, j).
 *  query_box dev f32[6] or NULL
 *  pairs     dev i32[cap][2]   out: first min(total, cap) pairs
 *  dev_count dev i64[1]        out: exact total (may exceed cap; the caller
 *                              relaunches with a larger buffer, the paper's
 *                              abort-and-relaunch convention of Section 3.5)
 *  ws, ws_bytes                scratch of at least filter_aabb_pairs_ws_bytes */
int filter_aabb_pairs_ws_bytes(int64_t n_meshes_a, int64_t n_meshes_b, size_t* ws_bytes);
int filter_aabb_pairs(const void* blob_a, int64_t n_meshes_a, const void* blob_b,
                      int64_t n_meshes_b, const float* query_box, int32_t* pairs, int64_t cap,
                      int64_t* dev_count, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Refinement (Section 3.1 Steps I-II, Section 3.2 bidirectional tracing).
 *
 * For every candidate pair (i, j) the edges of A_i are traced as closed
 * segments against the BVH of B_j and the edges of B_j against the BVH of
 * A_i.  Internal nodes use a conservative segment-box test (never rejects a
 * box the segment touches); leaves use a closed segment-triangle test whose
 * orientation signs are filtered in FP32 with a forward error bound; signs
 * the bound cannot certify are re-decided on the GPU in FP64 and, if still
 * uncertain, in exact FP64 expansion arithmetic (the exact arithmetic the
 * paper calls for on degenerate configurations, Section 3.6).  Any hit
 * decides the pair, so the search stops early per pair.
 */
typedef struct {
  int32_t bvh_width;   /* width the blobs were built with (2, 4 or 8) */
  int32_t persistent;  /* 1: one persistent pass over all pairs (batched): the groups of
                          segments of every (pair, direction) are culled against the top
                          of the target tree and the survivors traced by persistent waves;
                          0: one launch per pair (plain), wave-per-pair packets */
  int32_t precision;   /* 0: FP32 filter, uncertain tests deferred and re-decided in
                             FP64/exact after the traversal
                          1: every leaf test decided in FP64/exact directly
                          2: every leaf test deferred to the FP64/exact pass (test mode)
                          3: as 0, but a test the FP32 filter leaves open is first decided
                             exactly in place when its five points lie on one small
                             power-of-two grid (coordinate bit span <= 14; see
                             blob_coord_exponents), so a pair whose only contacts are
                             exact touches still ends early; other tests are deferred */
  int32_t queue_cap;   /* capacity of the deferred-test queues (0 = default 1<<20, split
                          over 8 queues); a pair whose tests overflow them is traced
                          again with every leaf test decided in FP64/exact */
  int32_t grid_blocks; /* persistent launch: blocks of 256 threads of the tracing kernel
                          (0 = default: every block the GPU holds at once) */
  uint32_t seg_live_max; /* schedule 0: per target-size bucket (byte k: targets below
                          2^10, 2^13, 2^16 triangles, and larger), the largest number
                          of a group's segments meeting the target box for which the
                          group is traced wave-per-segment (the autotuner's table);
                          0 = every group wave-per-pair (measured best on the
                          workloads here) */
  int32_t schedule;    /* persistent launch (Section 3.2, edges traced in parallel):
                          0 = auto: per group, by the seg_live_max table (0: as 1);
                          1 = wave-per-pair: a wave traces 64 segments of one
                              (pair, direction) together, one per lane, walking the
                              target tree as one packet;
                          2 = wave-per-segment: the lanes of a wave are W children x
                              64/W segments, each segment walking its own path with its
                              own stack in LDS */
  int32_t survivor_cap; /* total capacity of the surviving-group queues, 16 bytes per
                          entry (0 = default 1<<24); a group beyond it sends its pair to
                          the rerun pass (every group of the pair traced again, leaf
                          tests in FP64/exact) */
  void* ev_begin;      /* optional hipEvent_t (or NULL) for timing the traversal kernels
                          alone: with persistent = 1 it takes the start time stamp of the
                          cull dispatch on `stream` (attached to the dispatch, no extra
                          packet); with persistent = 0 it is recorded on `stream` just
                          before the per-pair launches */
  void* ev_end;        /* optional hipEvent_t (or NULL): the end time stamp of the last
                          traversal dispatch (persistent = 1), or recorded just after the
                          launches (persistent = 0) */
  const int64_t* dev_n_pairs; /* optional device i64[1] (or NULL): the pairs processed are the
                          first min(*dev_n_pairs, n_pairs), so a count left on the device
                          by filter_aabb_pairs feeds the refinement without a host round
                          trip; n_pairs is then the capacity of pairs[] and flags[] (it
                          sizes the workspace), and flags past the count are not written */
  int32_t trace_budget; /* persistent: 0 = default: a wave whose queues are drained takes
                          pending stack entries (subtrees) that the other waves of its
                          block hand over on seeing it wait; > 0: instead, a group still
                          running after that many traversal steps hands its pending
                          entries to a continuation pass spread over all waves; -1 = no
                          hand-over of either kind */
  int32_t lds_stack;   /* persistent: 0 = the packet traversal keeps its first 64 stack
                          entries in VGPR lanes and the rest in LDS; 1 = the first
                          entries in LDS and only those beyond the LDS part in VGPR
                          lanes (no hand-over of stack entries then) */
} pr_refine_params;

typedef struct {
  uint64_t segments;              /* segments started (64-segment groups picked up x live lanes) */
  uint64_t node_visits;           /* wave-level BVH node fetches */
  uint64_t tri_tests;             /* segment-triangle tests (per segment) */
  uint64_t fp32_ambiguous;        /* tests the FP32 bound could not decide */
  uint64_t fp64_filter_ambiguous; /* tests needing exact expansions after the FP64 bound */
  uint64_t exact_decided;         /* tests decided in FP64/exact (deferred or in place) */
  uint64_t pairs_true;            /* pairs found intersecting */
  uint64_t queue_overflow;        /* deferred tests that did not fit in the queue */
  uint64_t groups;                /* 64-segment groups picked up */
  uint64_t tri_fetches;           /* wave-level leaf triangle loads */
  uint64_t groups_box_pass;       /* groups whose box meets the target mesh box (segments loaded) */
  uint64_t groups_traversed;      /* groups with a segment meeting the target mesh box */
  uint64_t max_group_node_visits; /* most node visits of one traced group */
  uint64_t max_group_leaf_fetches;/* most leaf triangle fetches of one traced group */
} pr_refine_stats;

/* Workspace bytes for refine_intersects on n_pairs pairs. */
int refine_workspace_bytes(int64_t n_pairs, const pr_refine_params* params, size_t* ws_bytes);

/*  blob_a, blob_b dev   blobs from build_mesh_bvh with width params->bvh_width
 *  n_meshes_a/b         mesh counts of the two blobs (pairs are range-checked
 *                       on the device: an out-of-range pair yields flag 0 and
 *                       dev_status PR_E_ARG)
 *  pairs   dev i32[n_pairs][2]   (i in A, j in B)
 *  flags   dev u8[n_pairs]       out: 1 iff the closed surfaces share a point
 *  params  host
 *  dev_stats dev pr_refine_stats or NULL (counters are overwritten)
 *  dev_status dev i32[1] or NULL  out: PR_OK, or PR_E_ARG / PR_E_UNSUPPORTED
 *                       when a pair index is out of range or a blob was
 *                       built with another width (those pairs get flag 0)
 *  ws, ws_bytes dev     scratch of at least refine_workspace_bytes */
int refine_intersects(const void* blob_a, int64_t n_meshes_a, const void* blob_b,
                      int64_t n_meshes_b, const int32_t* pairs, int64_t n_pairs, uint8_t* flags,
                      const pr_refine_params* params, pr_refine_stats* dev_stats,
                      int32_t* dev_status, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Allocation-free refinement, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): refine_intersects without a workspace argument.
 *
 * Scratch space comes from a static device buffer inside the library, one
 * copy per GPU, of refine_static_scratch_bytes() bytes (64 MiB), held until
 * the process ends.  With queue_cap / survivor_cap 0 the queues default to
 * 2^18 deferred tests and 2^21 surviving groups (overflow falls back to the
 * exact rerun, as with refine_intersects); n_pairs is limited by what fits:
 * a call that would need more scratch returns PR_E_CAPACITY (message in
 * pr_last_error) before enqueuing anything.  The first call on a GPU looks up
 * that GPU's copy of the buffer (with the caller's current device current).
 * Every call on a GPU uses that GPU's single buffer: calls that overlap on
 * one GPU (several streams, several host threads) race and give undefined
 * results, so the caller serialises them.  Each call clears, with a kernel,
 * every counter and state that must start at zero; the buffer keeps the
 * last call's contents otherwise.  Nothing is allocated or freed.  The other
 * arguments and the results are those of refine_intersects. */
size_t refine_static_scratch_bytes(void);
int refine_intersects_static(const void* blob_a, int64_t n_meshes_a, const void* blob_b,
                             int64_t n_meshes_b, const int32_t* pairs, int64_t n_pairs,
                             uint8_t* flags, const pr_refine_params* params,
                             pr_refine_stats* dev_stats, int32_t* dev_status, void* stream);

/* ------------------------------------------------------------------------ */
/* Point-in-mesh test and the containment, within and intersection joins
 * (Section 3.3, Algorithm 2; Section 3.4).
 *
 * For a candidate pair (i in A, j in B) the representative vertex of a mesh
 * is the first corner of its first face (input order; the build stores it
 * in the blob).  "rep(B_j) inside A_i" means the winding number of A_i's
 * surface about that vertex is non-zero: the signed count of crossings of a
 * +z ray from the vertex, each crossing counted with the sign of the
 * crossed triangle's normal z component.  Decisions are exact on the FP32
 * coordinates: orientation signs use the FP64 filter with an exact
 * expansion fallback, and a ray that would meet an edge or a vertex of the
 * target is resolved by symbolic perturbation of the vertex to
 * (x + e, y + e^2, z) for an infinitesimal e > 0 (Simulation of
 * Simplicity), which never changes the winding number of a point off the
 * surface.  A vertex lying on a triangle of the other mesh is reported as
 * such instead.  For closed, embedded, connected surfaces with outward
 * faces, the winding number is 1 inside and 0 outside, which is the paper's
 * odd parity; when the two surfaces share no point, the whole of one lies
 * inside the other iff its representative vertex does. */
typedef struct {
  uint64_t rays;           /* rays cast (pair directions not skipped) */
  uint64_t box_miss;       /* rays that miss the target mesh's box */
  uint64_t node_visits;    /* BVH nodes loaded */
  uint64_t tri_tests;      /* leaf triangles whose box the ray column meets */
  uint64_t crossings;      /* crossings ahead of the vertex (either sign) */
  uint64_t exact_signs;    /* orientation signs the FP64 filter could not certify */
  uint64_t on_surface;     /* representative vertices lying on the other surface */
  uint64_t deep;           /* rays rerun with the full-depth stack */
} pr_inside_stats;

/* Workspace bytes for inside_pairs on n_pairs pairs. */
int inside_workspace_bytes(int64_t n_pairs, size_t* ws_bytes);

/* Point-in-mesh test per candidate pair.
 *  blob_a, blob_b dev   blobs from build_mesh_bvh (any width; both datasets may
 *                       use different widths)
 *  n_meshes_a/b         mesh counts (pairs are range-checked on the device:
 *                       out-of-range pairs get 0 and dev_status PR_E_ARG)
 *  pairs   dev i32[n_pairs][2]
 *  mode    0: raw bits; out[p] = bit 0 rep(B_j) inside A_i, bit 1 rep(A_i)
 *             inside B_j, bit 2 rep(B_j) on A_i's surface, bit 3 rep(A_i)
 *             on B_j's surface (bits 0 / 1 are 0 when 2 / 3 are set);
 *             `cross` is not read (may be NULL).
 *          1: contains      out[p] = !cross[p] && rep(B_j) inside A_i
 *          2: within        out[p] = !cross[p] && rep(A_i) inside B_j
 *          3: intersection  out[p] = cross[p] || rep(B_j) inside A_i
 *                                    || rep(A_i) inside B_j
 *          Modes 1-3 read cross dev u8[n_pairs] (the overlap flags of
 *          refine_intersects for the same pairs) and cast rays only for pairs
 *          with cross[p] == 0; out may alias cross.
 *  out     dev u8[n_pairs]
 *  dev_stats dev pr_inside_stats or NULL (overwritten)
 *  dev_status dev i32[1] or NULL        out: PR_OK, PR_E_ARG (a pair out of range)
 *                       or PR_E_UNSUPPORTED (a blob that is not a blob of this
 *                       library, or n_meshes beyond the blob's count)
 *  ws, ws_bytes dev     scratch of at least inside_workspace_bytes */
int inside_pairs(const void* blob_a, int64_t n_meshes_a, const void* blob_b, int64_t n_meshes_b,
                 const int32_t* pairs, int64_t n_pairs, int32_t mode, const uint8_t* cross,
                 uint8_t* out, pr_inside_stats* dev_stats, int32_t* dev_status, void* ws,
                 size_t ws_bytes, void* stream);

/* One join predicate over candidate pairs: 0 overlap (refine_intersects),
 * 1 contains, 2 within, 3 intersection.  Runs refine_intersects, then, for
 * predicates 1-3, inside_pairs in that mode over the pairs without a shared
 * surface point; flags dev u8[n_pairs] receives the predicate.  The other
 * arguments are those of refine_intersects (params->bvh_width must match
 * both blobs) and inside_pairs (dev_inside_stats is written for predicates
 * 1-3 only); dev_status keeps the first error of either step; ws of at least
 * refine_predicate_workspace_bytes. */
int refine_predicate_workspace_bytes(int64_t n_pairs, const pr_refine_params* params,
                                     size_t* ws_bytes);
int refine_predicate(const void* blob_a, int64_t n_meshes_a, const void* blob_b,
                     int64_t n_meshes_b, const int32_t* pairs, int64_t n_pairs, int32_t predicate,
                     uint8_t* flags, const pr_refine_params* params, pr_refine_stats* dev_stats,
                     pr_inside_stats* dev_inside_stats, int32_t* dev_status, void* ws,
                     size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* The paper's own dataset-level design (Sections 3.2 and 3.5), for
 * comparison with the per-pair path: one BVH over every triangle of the
 * target dataset (a blob built with build_mesh_bvh from ONE mesh holding all
 * of the dataset's triangles, faces in the dataset's order), a
 * triangle-to-object map, each unique source edge traced against that tree
 * with every hit collected (closed, exact segment-triangle tests, as in
 * refine_intersects), and the (source object, target object) records
 * materialised by counting two-pass + sort/unique, or by a single pass into
 * a hashmap that drops duplicates on insert, sized from the selectivity
 * estimate or fixed.  Keys are (i << 32 | j), i in A, j in B. */
typedef struct {
  int32_t op;       /* 0 count: counts[g] = records of source group g, *dev_n = total;
                       1 write: the records of the same trace at the scanned offsets of counts
                         into keys (key_cap entries at least the total);
                       2 hash: insert into keys, a table of key_cap slots (a power of two) cleared
                         by op 3; *dev_n = keys inserted by this call;
                       3 clear: keys[0 .. key_cap) = empty (~0), *dev_n = 0 */
  int32_t flip;     /* 0: source = A, target = B, key (src << 32 | tgt); 1: source = B, key (tgt << 32 | src) */
  int32_t width;    /* BVH width of the target dataset-level blob */
  int32_t reserved;
  int64_t key_cap;
} pr_dataset_params;

typedef struct {
  uint64_t groups;       /* source groups traced */
  uint64_t node_visits;  /* wave-level node visits */
  uint64_t tri_tests;    /* segment-triangle tests */
  uint64_t hits;         /* segment-triangle hits */
  uint64_t records;      /* records emitted (consecutive repeats of one target object dropped per segment) */
  uint64_t exact;        /* tests decided in FP64 / exact arithmetic */
  uint64_t overflow;     /* records that found no room (write beyond the counts, hashmap full) */
  uint64_t new_keys;     /* op 2: keys newly inserted */
} pr_dataset_stats;

/* Object of every leaf-order triangle of a dataset-level blob: tri_obj dev
 * i32[f_total] (out), face_off dev i64[n_objects + 1] (object o owns faces
 * face_off[o] .. face_off[o+1] of the dataset); dev_status: PR_OK or PR_E_ARG
 * when a face lies outside every object. */
int dataset_tri_objects(const void* dblob, const int64_t* face_off, int64_t n_objects, int32_t* tri_obj,
                        int64_t f_total, int32_t* dev_status, void* stream);

/* Workspace of dataset_trace for a source blob of at most max_groups
 * 64-segment groups (3 f_total / 64 + n_meshes bounds it). */
int dataset_trace_ws_bytes(int64_t max_groups, size_t* ws_bytes);

/*  src_blob dev        per-mesh blob of the source dataset (its edges), n_src_objects meshes
 *  dst_blob dev        dataset-level blob of the target dataset, tri_obj its map, n_dst_objects objects
 *  counts   dev u64[max_groups + 1]   op 0 out, op 1 in
 *  keys     dev u64[key_cap]          ops 1-3
 *  dev_n    dev u64[1] or NULL        see pr_dataset_params.op
 *  dev_stats dev or NULL; dev_status dev i32[1]: PR_OK, or PR_E_UNSUPPORTED for a target blob
 *  that is not a one-mesh blob of params->width, or a source of more than max_groups groups. */
int dataset_trace(const void* src_blob, int64_t n_src_objects, const void* dst_blob, const int32_t* tri_obj,
                  int64_t n_dst_objects, const pr_dataset_params* params, uint64_t* counts, int64_t max_groups,
                  uint64_t* keys, uint64_t* dev_n, pr_dataset_stats* dev_stats, int32_t* dev_status, void* ws,
                  size_t ws_bytes, void* stream);

/* Sorted distinct keys of keys[0 .. n_keys) (empty slots ~0 skipped) as i32
 * pairs (i, j) into out_pairs[out_cap][2]; dev_count gets the exact number
 * even beyond out_cap. */
int pairs_unique_ws_bytes(int64_t n_keys, size_t* ws_bytes);
int pairs_unique(const uint64_t* keys, int64_t n_keys, int32_t* out_pairs, int64_t out_cap, int64_t* dev_count,
                 void* ws, size_t ws_bytes, void* stream);

/* Selectivity estimate of Section 3.5 on a cells^3 grid over the union of
 * both datasets' mesh boxes: per cell and dataset the number of meshes whose
 * closed box touches the cell, their mean box side and mean volume ratio
 * (|divergence-theorem volume| / box volume, clamped to [0, 1], 1 for a flat
 * box); per cell N_A N_B min((S_A + S_B + 10^-3)^3 / V_cell *
 * sqrt(R_A R_B)^0.8, 1), summed into *dev_estimate (f64, FP64 throughout). */
int estimate_pairs_ws_bytes(int64_t n_meshes_a, int64_t n_meshes_b, int32_t cells, size_t* ws_bytes);
int estimate_pairs(const void* blob_a, int64_t n_meshes_a, const void* blob_b, int64_t n_meshes_b, int32_t cells,
                   double* dev_estimate, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Result materialisation (Section 3.5): keeps the pairs whose flag is 1, in
 * input order.  pairs dev i32[n_pairs][2], flags dev u8[n_pairs]; dev_n_pairs
 * dev i64[1] or NULL: when given, only the first min(*dev_n_pairs, n_pairs)
 * pairs are considered (n_pairs is then the capacity); out dev i32[cap][2];
 * dev_count dev i64[1] gets the exact total even if it exceeds cap.  ws of
 * at least compact_pairs_ws_bytes. */
int compact_pairs_ws_bytes(int64_t n_pairs, size_t* ws_bytes);
int compact_pairs(const int32_t* pairs, const uint8_t* flags, int64_t n_pairs,
                  const int64_t* dev_n_pairs, int32_t* out, int64_t cap, int64_t* dev_count, void* ws,
                  size_t ws_bytes, void* stream);

/* Batch assembly for serving (Section 3.5 query pipeline): concatenates the
 * leading pairs of n_regions regions, in region order, without a host round
 * trip.  regions dev i32[n_regions * region_cap][2] (region k starts at pair
 * k * region_cap, as left by one filter_aabb_pairs call per query with cap =
 * region_cap); dev_counts dev i64[n_regions], the filter's counts (each
 * clamped to [0, region_cap]); out dev i32[cap][2] receives the
 * concatenation (rows past cap are dropped); dev_total dev i64[1] gets the
 * exact concatenated length, so it can feed refine_intersects as
 * dev_n_pairs.  n_regions <= 2^20 (PR_E_UNSUPPORTED beyond). */
int gather_pair_regions(const int32_t* regions, int64_t region_cap, const int64_t* dev_counts,
                        int64_t n_regions, int32_t* out, int64_t cap, int64_t* dev_total, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PIERCE_H */
