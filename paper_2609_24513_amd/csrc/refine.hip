// refine_intersects: bidirectional edge-segment tracing per candidate pair.
//
// Work unit: one group of 64 segments (64 unique edges of the source mesh,
// consecutive in Morton order of their midpoints) against the target mesh's
// wide BVH (Section 3.1 Steps I-II; both directions as in Section 3.2).  The
// persistent pass first culls every group of every (pair, direction) against
// the top of the target tree (k_cull), then persistent waves trace the
// surviving groups (k_trace), in one of two ways:
//  * wave-per-pair (packet): the wave walks the tree together, one segment
//    per lane; a node is visited once for the whole wave, every still-active
//    lane tests its segment against all W child boxes, and children hit by
//    any lane are pushed with the mask of lanes that hit them onto a per-wave
//    stack (VGPR lanes, then LDS).  At a leaf the lanes of the mask test
//    their segment against each triangle.
//  * wave-per-segment: the lanes are W children x 64/W segment slots; each
//    slot walks its own segment's path with its own stack in LDS, its W lanes
//    testing the W children of its current node (or W leaf triangles) at
//    once.  Suited to groups with few segments near the target, whose paths
//    diverge.
// The automatic schedule picks per group, by how many of its segments meet
// the target box and by the target's size.  A certain hit marks the pair and
// every wave working on it stops (the paper's multi-hit loop is unnecessary:
// one BVH holds one mesh, and any hit decides the pair).

// Segment-box test (conservative): slab test on t in [0, 1] for the segment
// p + t (q - p), with t computed as (plane - p) * fl(1 / fl(q - p)); every t
// carries a relative error of at most gamma_4 = 4 eps / (1 - 4 eps), so
// accepting when t_min <= t_max (1 + 2^-19) + 2^-120 never rejects a box the
// exact segment touches (closed boxes).  A zero direction component uses a
// large finite reciprocal (2^100) and a bias of 2^16 that turns the slab into
// "no constraint" or "empty" exactly.  Valid for FP32-safe coordinates; for
// other meshes every box is accepted and every leaf test is deferred.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <atomic>
#include <climits>
#include <mutex>

#include "common.h"
#include "predicates.h"

namespace pr {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr float kSlabK = 1.0f + 0x1p-19f;
constexpr float kSlabS = 0x1p-120f;
constexpr float kZeroInv = 0x1p100f;
constexpr float kZeroBias = 0x1p16f;

// Entries on a wave's stack: nodes and leaves; a node pops one entry and
// pushes at most W, over at most kMaxDepth node levels plus the leaf level.
template <int W>
constexpr int stack_cap() { return (W - 1) * (kMaxDepth + 1) + 1; }

struct BlobView {
  const MeshDesc* mesh;
  const char* nodes;
  const float* tris;
  const float* seg;
  const float* cbox;
  const float* rbox;
  int64_t n_meshes;
  int32_t width;
  uint32_t magic;
};

__device__ __forceinline__ BlobView view_of(const char* blob) {
  const BlobHeader* h = reinterpret_cast<const BlobHeader*>(blob);
  BlobView v;
  v.mesh = reinterpret_cast<const MeshDesc*>(blob + h->off_mesh);
  v.nodes = blob + h->off_node;
  v.tris = reinterpret_cast<const float*>(blob + h->off_tri);
  v.seg = reinterpret_cast<const float*>(blob + h->off_seg);
  v.cbox = reinterpret_cast<const float*>(blob + h->off_cbox);
  v.rbox = reinterpret_cast<const float*>(blob + h->off_rbox);
  v.n_meshes = h->n_meshes;
  v.width = h->width;
  v.magic = h->magic;
  return v;
}

enum {
  S_SEG = 0, S_VISIT, S_TESTS, S_AMB32, S_AMB64, S_EXACT, S_TRUE, S_QOVER, S_GROUPS, S_TRIF, S_GBOX, S_GTRAV,
  S_MAXV, S_MAXL, S_N
};

struct RefineArgs {
  const char* blob_a;
  const char* blob_b;
  int64_t n_meshes_a, n_meshes_b;
  const int32_t* pairs;
  int64_t n_pairs;            // capacity: pairs[] holds at least this many entries
  const int64_t* np_dev;      // optional device count of the pairs to process
  uint8_t* flags;
  uint32_t* state;            // [P] 0 undecided, 1 intersecting
  unsigned long long* ctr;    // kSlices grab counters of the cull (one per XCD share), 4 KiB apart
  int4* queue;                // deferred tests (pair, dir, segment slot, triangle): kSlices queues
  uint32_t qcap;              // total entries
  uint32_t qsub;              // entries per queue
  uint32_t* qcount;           // kSlices fill counters, kQCtrStride words apart
  unsigned long long* stats;  // [S_N]
  int32_t* status;            // [1]
  int4* surv;                 // kQueues queues of surviving groups (survivor entry layout)
  uint32_t surv_cap;          // entries per queue
  unsigned long long* surv_cnt;  // kQueues fill counters (stride kCtrStride)
  unsigned long long* surv_pop;  // kQueues pop counters (stride kCtrStride)
  int4* tasks;                // kQueues lists of continuation tasks (group, unit, node ref, live | safe << 8)
  uint64_t* tmask;            // lane mask of each task
  uint32_t task_cap;          // tasks per list
  unsigned long long* task_cnt;  // kQueues fill counters (stride kCtrStride)
  unsigned long long* task_pop;  // kQueues pop counters (stride kCtrStride)
  int32_t budget;             // traversal steps before a group hands its stack over (0 = none)
  int32_t share;              // waves of a block share pending stack entries (1 = on)
  int32_t lds_stack;          // 1: the packet traversal's stack lives wholly in LDS
  uint32_t seg_table;         // per target-size bucket: wave-per-segment limit (bytes)
  int32_t* order;             // [P] pairs in cull order (heaviest cost class first), when `ordered`
  uint32_t* ord_cnt;          // kCostClasses class sizes, then kCostClasses fill counters
  int32_t ordered;            // 1: the cull takes its units in `order`
};

constexpr int kSlices = 8;     // one pop counter per XCD
// Survivor queues of the persistent pass: queue blockIdx % kQueues, so every queue is
// filled and drained by the blocks of one XCD (blocks are dealt round-robin
// to the 8 XCDs); 8 queues per XCD keep the atomics on each queue's counters
// below the memory-side serialisation rate.
constexpr int kQueues = 64;
constexpr int kCostClasses = 8;  // cost classes of the cull order (powers of two of the groups)
// Continuation tasks (optional): a group still running after kBudget
// traversal steps hands its pending stack entries over to a third kernel, so
// that the few long groups are spread over many waves instead of ending the
// run alone.  kTaskCap tasks per list.
constexpr int kBudget = 0;  // off by default: measured slower on the pathology-shaped workload
constexpr uint32_t kTaskCap = 1u << 14;
constexpr int kCtrStride = 512; // u64 words between counters (4 KiB: separate memory channels)
// Statistics: kStatCopies copies of the S_N counters (blockIdx % kStatCopies),
// kCtrStride words apart, summed when reported: atomics on one address
// serialise at the memory side (about 11 ns each), and every wave adds its
// counters when it ends.  The overflow counter lives in copy 0 only, so that
// one load tells whether a rerun is needed.
constexpr int kStatCopies = 64;
__device__ __forceinline__ unsigned long long* stat_copy(unsigned long long* stats) {
  return stats + kCtrStride * (blockIdx.x % kStatCopies);
}

__device__ __forceinline__ uint32_t load_state(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void mark_true(uint32_t* p) {
  __hip_atomic_store(p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t ballot(bool b) { return __ballot(b); }

__device__ __forceinline__ int lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ bool box_meet(const float* a, float lx, float ly, float lz, float hx, float hy,
                                         float hz) {
  return a[0] <= hx && lx <= a[3] && a[1] <= hy && ly <= a[4] && a[2] <= hz && lz <= a[5];
}

struct Ray {
  float px, py, pz, ix, iy, iz, bx, by, bz;
};

__device__ __forceinline__ void axis_setup(float d, bool safe, float& inv, float& bias) {
  if (!safe) { inv = 0.f; bias = INFINITY; return; }
  if (d != 0.f) { inv = 1.0f / d; bias = 0.f; }
  else { inv = kZeroInv; bias = kZeroBias; }
}

// t = (plane - p) * inv -+ bias as one fused multiply-add: with bias 0 (a
// non-zero direction component) the value is the rounded product, as two
// separate operations would give; with a zero component the sign of
// (plane - p) is kept exactly and the bias opens the slab to all t, or
// pushes it away from [0, 1].
__device__ __forceinline__ bool slab(const Ray& r, float lx, float ly, float lz, float hx, float hy, float hz) {
  float t0x = fmaf(lx - r.px, r.ix, -r.bx), t1x = fmaf(hx - r.px, r.ix, r.bx);
  float t0y = fmaf(ly - r.py, r.iy, -r.by), t1y = fmaf(hy - r.py, r.iy, r.by);
  float t0z = fmaf(lz - r.pz, r.iz, -r.bz), t1z = fmaf(hz - r.pz, r.iz, r.bz);
  float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.f));
  float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), 1.f));
  return tn <= fmaf(tf, kSlabK, kSlabS);
}

// Per-wave statistics in one VGPR pair: lane k holds counter k (k < S_N), so
// the counters cost no SGPRs in the traversal loops.
struct WaveStats {
  uint64_t acc = 0;
  __device__ __forceinline__ void add(int k, uint64_t x) { acc += (threadIdx.x & 63) == k ? x : 0ull; }
  __device__ __forceinline__ void max(int k, uint64_t x) {
    if ((threadIdx.x & 63) == k && x > acc) acc = x;
  }
};

__device__ __forceinline__ f3 tri_vertex(const float* t, int k) { return f3{t[3 * k], t[3 * k + 1], t[3 * k + 2]}; }
__device__ __forceinline__ f3 tri_vertex(cptr_t<float> t, int k) { return f3{t[3 * k], t[3 * k + 1], t[3 * k + 2]}; }

// Traces group `chunk` of source mesh sm against target mesh tm; the caller
// has checked that the group's box meets the target mesh box.  Returns true
// when the pair is decided (found here or by another wave).
// Per-wave traversal stack of (entry, lane mask) pairs.  The stack top is
// wave-uniform; by default the first kRegStack entries live in VGPR lanes
// (entry k in lane k of three registers, written and read with lane-select
// instructions) and deeper entries in a per-wave LDS array written by lane 0;
// with lds_stack the LDS array holds the first entries and the VGPR lanes the
// deeper ones.
constexpr int kRegStack = 64;

template <int W>
constexpr int lds_stack_cap() { return stack_cap<W>() > kRegStack ? stack_cap<W>() - kRegStack : 1; }

// Wave-per-segment mode: 64 / W segment slots per wave (lanes = W children x
// slots), each slot with its own stack of node references in LDS.
template <int W>
constexpr int seg_slots() { return 64 / W; }
template <int W>
constexpr int seg_cap() { return W == 8 ? 64 : (W == 4 ? 32 : 24); }

// LDS of one wave for the traversal, in 8-byte words: the LDS part of the
// packet stack (lds_stack_cap entries: lane masks, then references), or the
// per-segment stacks of the wave-per-segment mode, which are never in use at
// the same time as the packet stack and share its space.
template <int W>
constexpr int wave_lds_words() {
  return (12 * lds_stack_cap<W>() > 4 * seg_slots<W>() * seg_cap<W>() ? 12 * lds_stack_cap<W>()
                                                                       : 4 * seg_slots<W>() * seg_cap<W>()) / 8 + 1;
}

struct WaveLds {
  int32_t* ref;    // LDS part of the packet stack: node references
  uint64_t* mask;  // ... and their lane masks
  int32_t* seg;    // wave-per-segment stacks (aliases ref / mask), or nullptr
  int lds_first;   // 0: the first kRegStack entries in VGPR lanes, the rest in LDS;
                   // 1: the first lds_cap entries in LDS, the rest in VGPR lanes
  int lds_cap;     // entries the LDS part holds
};

template <int W>
__device__ __forceinline__ WaveLds wave_lds(uint64_t* area, bool lds_first) {
  WaveLds l;
  l.mask = area;
  l.ref = reinterpret_cast<int32_t*>(area + lds_stack_cap<W>());
  l.seg = reinterpret_cast<int32_t*>(area);
  l.lds_first = lds_first ? 1 : 0;
  l.lds_cap = lds_stack_cap<W>();
  return l;
}

// For kernels with only the register stack and its LDS overflow.
__device__ __forceinline__ WaveLds wave_lds(int32_t* ref, uint64_t* mask) {
  return WaveLds{ref, mask, nullptr, 0, 0};
}

// v_writelane_b32: `old` with lane `lane` replaced by the uniform value v
// (the LLVM intrinsic; this clang has no builtin spelling for it).
__device__ int32_t lane_write(int32_t v, int32_t lane, int32_t old) __asm("llvm.amdgcn.writelane.i32");

struct WaveStack {
  int32_t ref;
  int32_t mlo, mhi;
  int32_t* lref;
  uint64_t* lmask;
  int32_t top;
  // entries reg_lo .. reg_lo + kRegStack - 1 live in VGPR lanes 0 .. 63, the
  // others at LDS index i - lds_lo (plain integers, so that the placement
  // of an entry is decided by scalar instructions)
  int32_t reg_lo;
  int32_t lds_lo;
};

__device__ __forceinline__ void stack_layout(WaveStack& s, const WaveLds& l) {
  s.reg_lo = l.lds_first ? l.lds_cap : 0;
  s.lds_lo = l.lds_first ? 0 : kRegStack;
}

// Entry i of the stack: in VGPR lane reg_index(i) or at LDS index lds_index(i).
__device__ __forceinline__ bool in_reg(const WaveStack& s, int32_t i) {
  return (uint32_t)(i - s.reg_lo) < (uint32_t)kRegStack;
}
__device__ __forceinline__ int32_t reg_index(const WaveStack& s, int32_t i) { return i - s.reg_lo; }
__device__ __forceinline__ int32_t lds_index(const WaveStack& s, int32_t i) { return i - s.lds_lo; }

__device__ __forceinline__ void stack_push(WaveStack& s, int32_t ref, uint64_t m) {
  if (in_reg(s, s.top)) {
    const int32_t k = reg_index(s, s.top);
    s.ref = lane_write(ref, k, s.ref);
    s.mlo = lane_write((int32_t)(uint32_t)m, k, s.mlo);
    s.mhi = lane_write((int32_t)(uint32_t)(m >> 32), k, s.mhi);
  } else if ((threadIdx.x & 63) == 0) {
    s.lref[lds_index(s, s.top)] = ref;
    s.lmask[lds_index(s, s.top)] = m;
  }
  ++s.top;
}

__device__ __forceinline__ int32_t stack_ref(const WaveStack& s, int32_t i) {
  return in_reg(s, i) ? __builtin_amdgcn_readlane(s.ref, reg_index(s, i)) : uni(s.lref[lds_index(s, i)]);
}

__device__ __forceinline__ uint64_t stack_mask(const WaveStack& s, int32_t i) {
  if (in_reg(s, i)) {
    const int32_t k = reg_index(s, i);
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(s.mhi, k) << 32) |
           (uint32_t)__builtin_amdgcn_readlane(s.mlo, k);
  }
  return uni64(s.lmask[lds_index(s, i)]);
}

// A wide node read in one burst through the scalar cache.
template <int W>
struct NodeRegs {
  float lo[3][W], hi[3][W];
  int32_t ch[W];
};

template <int W>
__device__ __forceinline__ void load_node(NodeRegs<W>& d, cptr_t<Node<W>> n) {
#pragma unroll
  for (int c = 0; c < W; ++c) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      d.lo[a][c] = n->lo[a][c];
      d.hi[a][c] = n->hi[a][c];
    }
    d.ch[c] = n->child[c];
  }
}

// Lane masks of the children of a node hit by the segments of mask nm: every
// present child is tested by every lane and the result masked.  For
// meshes outside the FP32-safe range the slab test accepts everything and the
// exact uniform test against the group box does the pruning.
template <int W>
__device__ __forceinline__ void test_children(const NodeRegs<W>& d, const Ray& r, uint64_t nm, bool safe,
                                              const float* cb, uint64_t* hm) {
#pragma unroll
  for (int c = 0; c < W; ++c) {
    hm[c] = 0;
    if (d.ch[c] == kEmpty) continue;  // uniform: empty slots cost no vector work
    uint64_t m = ballot(slab(r, d.lo[0][c], d.lo[1][c], d.lo[2][c], d.hi[0][c], d.hi[1][c], d.hi[2][c])) & nm;
    if (!safe && !box_meet(cb, d.lo[0][c], d.lo[1][c], d.lo[2][c], d.hi[0][c], d.hi[1][c], d.hi[2][c])) m = 0;
    hm[c] = m;
  }
}

// Hands the pending entries of a wave's stack over as continuation tasks of
// list tq: entry k sits in lane k of the register stack, so the lanes write
// their own entries; as many as fit are taken from the top.  Returns true
// when the whole stack was handed over.
__device__ bool hand_over(WaveStack& stk, const RefineArgs& ra, int tq, int64_t gc, int32_t unit, int32_t live_safe) {
  const int lane = threadIdx.x & 63;
  const int n = stk.top;
  if (n > kRegStack) return false;  // deeper stacks are finished in place
  unsigned long long b0 = 0;
  if (lane == 0) b0 = atomicAdd(ra.task_cnt + kCtrStride * tq, (unsigned long long)n);
  const uint64_t base = uni64(b0);
  const int fit = base >= ra.task_cap ? 0 : (int)min((uint64_t)n, ra.task_cap - base);
  if (lane < n && lane >= n - fit) {
    const int64_t at = (int64_t)tq * ra.task_cap + (int64_t)(base + (uint64_t)(lane - (n - fit)));
    ra.tasks[at] = make_int4((int32_t)gc, unit, stk.ref, live_safe);
    ra.tmask[at] = ((uint64_t)(uint32_t)stk.mhi << 32) | (uint32_t)stk.mlo;
  }
  stk.top = n - fit;
  return fit == n;
}

// Work sharing inside a block: a wave whose queues are drained
// waits for pending stack entries that its block's tracing waves move into a
// small LDS task list when they see it waiting.  Every counter is monotonic
// within one launch; slots beyond kBlkTasks are never used.
constexpr uint32_t kBlkTasks = 128;

struct BlockShare {
  int4 task[kBlkTasks];       // group, unit, node ref, live | safe << 8
  uint64_t mask[kBlkTasks];   // lane mask of the entry
  uint32_t ready[kBlkTasks];  // 1 once the slot is written
  uint32_t tail;              // slots reserved
  uint32_t head;              // slots taken
  uint32_t idle;              // waves waiting for a task
  uint32_t active;            // waves still on their queues
  uint32_t busy;              // waves tracing a task they took (or about to)
};

__device__ __forceinline__ uint32_t lds_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Moves the `h` oldest pending entries of a wave's stack (entries 0..h-1,
// the subtrees nearest the root; h <= top) to the block's task list: each lane below
// h writes its entry and then marks the slot ready; the rest of the stack
// moves down.  Returns the number of entries moved (fewer when the list is
// full).
__device__ int share_out(WaveStack& stk, BlockShare* sh, int64_t gc, int32_t unit, int32_t live_safe, int h) {
  const int lane = threadIdx.x & 63;
  uint32_t b0 = 0;
  if (lane == 0) b0 = __hip_atomic_fetch_add(&sh->tail, (uint32_t)h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  const uint32_t base = (uint32_t)uni((int32_t)b0);
  const int fit = base >= kBlkTasks ? 0 : (int)min((uint32_t)h, kBlkTasks - base);
  if (fit == 0) return 0;
  if (lane < fit) {
    sh->task[base + lane] = make_int4((int32_t)gc, unit, stk.ref, live_safe);
    sh->mask[base + lane] = ((uint64_t)(uint32_t)stk.mhi << 32) | (uint32_t)stk.mlo;
    __hip_atomic_store(&sh->ready[base + lane], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  const int src = lane + fit < 64 ? lane + fit : 63;
  stk.ref = __shfl(stk.ref, src);
  stk.mlo = __shfl(stk.mlo, src);
  stk.mhi = __shfl(stk.mhi, src);
  stk.top -= fit;
  return fit;
}

// Deferred tests: kSlices queues (one per XCD, the block's XCD taken as
// blockIdx % kSlices), each of qsub entries with its own fill counter, so
// that the waves of different XCDs never contend for one counter.
constexpr int kQCtrStride = 1024;  // u32 words between the fill counters (4 KiB)

// Appends the tests of the lanes with `amb` set (segment slot `slot_idx`,
// triangle `tri`) to the deferred-test queue of the block's XCD.  Returns
// false when the queue is full: the pair is then marked for the exact rerun.
__device__ bool defer_tests(const RefineArgs& ra, bool amb, int32_t pair, int32_t dir, int32_t slot_idx, int32_t tri,
                            WaveStats& st) {
  const int lane = threadIdx.x & 63;
  const uint64_t am = ballot(amb);
  if (!am) return true;
  const int qx = (int)(blockIdx.x % kSlices);
  uint32_t base = 0;
  if (lane == 0) base = atomicAdd(ra.qcount + kQCtrStride * qx, (uint32_t)__popcll(am));
  base = (uint32_t)uni((int32_t)base);
  const uint32_t idx = base + (uint32_t)lanes_below(am);
  if (amb && idx < ra.qsub) ra.queue[(int64_t)qx * ra.qsub + idx] = make_int4(pair, dir, slot_idx, tri);
  const uint64_t over = ballot(amb && idx >= ra.qsub);
  if (over) {
    st.add(S_QOVER, (uint64_t)__popcll(over));
    if (lane == 0) atomicCAS(ra.state + pair, 0u, 2u);
    return false;
  }
  return true;
}

// One closed segment-triangle test at a leaf, first tier: the FP32 filter
// (PREC 0 and 3), FP64/exact (PREC 1) or a forced deferral (PREC 2, test
// mode).
template <int PREC>
__device__ __forceinline__ int leaf_test(f3 p, f3 q, f3 a, f3 b, f3 c, bool safe) {
  if (PREC == 1) {
    ExactCounters ec{0};
    return seg_tri_exact(p, q, a, b, c, ec) ? kHit : kMiss;
  }
  if (PREC == 2) return kAmbig;
  return safe ? seg_tri_f32(p, q, a, b, c) : kAmbig;
}

// Second tier of the FP32 traversal with PREC 3: the lane's tests that the
// FP32 filter left open (bits of `amb`, triangle first + bit * stride) go to
// the exact grid tier; decided ones leave `amb` and hits enter `hit`.  n32
// and ngrid count the FP32-uncertain tests and those decided here.
// The exact tests of one lane, out of line: the expansion arithmetic keeps
// its registers to itself instead of raising the traversal loop's.  Returns
// the still-uncertain bits; hits are added to *hit, decisions to *ngrid.
__device__ __noinline__ uint32_t grid_decide(f3 p, f3 q, const float* tris, int32_t first, int stride, uint32_t amb,
                                             uint32_t* hit, uint32_t* ngrid) {
  for (uint32_t m = amb; m; m &= m - 1) {
    const int k = __builtin_ctz(m);
    const float* tp = tris + 9 * (int64_t)(first + k * stride);
    const int g = seg_tri_grid(p, q, tri_vertex(tp, 0), tri_vertex(tp, 1), tri_vertex(tp, 2));
    if (g != kAmbig) {
      ++*ngrid;
      amb &= ~(1u << k);
      if (g == kHit) *hit |= 1u << k;
    }
  }
  return amb;
}

template <int PREC>
__device__ __forceinline__ void grid_tier(f3 p, f3 q, const float* tris, int32_t first, int stride, uint32_t& hit,
                                          uint32_t& amb, uint32_t& n32, uint32_t& ngrid) {
  n32 += (uint32_t)__popc(amb);
  if (PREC != 3) return;
  amb = grid_decide(p, q, tris, first, stride, amb, &hit, &ngrid);
}

// Wave sum of a per-lane count.
__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// Wave-per-segment traversal of the segments `todo` (lanes of group gc)
// against the target tree from `root`: lanes are W children x 64/W segment
// slots; a slot traces one segment at a time with its own stack of node
// references in LDS (`sstk`), its W lanes testing the W children of the
// slot's current node, or W triangles of a leaf at a time.  Slots that finish
// take the next segment.  A segment whose stack would overflow is left to
// the packet traversal (its bit is set in `overflow`).  Returns true when the
// pair is decided.
template <int W, int PREC>
__device__ bool trace_segments(const BlobView& S, const BlobView& T, int64_t gc, int32_t root, int32_t pair,
                               int32_t dir, bool safe, uint64_t todo, const float* cb, const RefineArgs& ra,
                               int32_t* sstk, WaveStats& st, uint64_t& overflow) {
  constexpr int CAP = seg_cap<W>();
  constexpr uint32_t kWMask = (1u << W) - 1u;
  const int lane = threadIdx.x & 63;
  const int slot = lane / W, c = lane % W;
  int32_t* stk = sstk + slot * CAP;
  const float* sp = S.seg + gc * (6 * kChunk);
  const Node<W>* nodes = reinterpret_cast<const Node<W>*>(T.nodes);
  int seg = -1, top = 0;
  f3 p{0.f, 0.f, 0.f}, q{0.f, 0.f, 0.f};
  Ray r{};
  uint32_t visits = 0, leaves = 0, tests = 0;  // slot events counted by the slot's lane 0
  uint32_t n32 = 0, ngrid = 0;
  // the counts go into the wave's statistics on every way out
  struct Fold {
    WaveStats& st;
    uint32_t &visits, &leaves, &tests, &n32, &ngrid;
    __device__ ~Fold() {
      const uint32_t v = wave_sum(visits), l = wave_sum(leaves), t = wave_sum(tests);
      st.add(S_VISIT, v);
      st.add(S_TRIF, l);
      st.add(S_TESTS, t);
      st.add(S_AMB32, wave_sum(n32));
      st.add(S_EXACT, PREC == 1 ? t : wave_sum(ngrid));
      st.max(S_MAXV, v);
      st.max(S_MAXL, l);
    }
  } fold{st, visits, leaves, tests, n32, ngrid};
  uint32_t poll = 0;
  int iter = 0;
  overflow = 0;
  for (;;) {
    // idle slots take the next segments of `todo`, lowest slot first
    const uint64_t idle = ballot(c == 0 && seg < 0);
    if (idle && todo) {
      uint64_t m = idle;
      int take = -1;
      while (m && todo) {
        const int leader = __builtin_ctzll(m);
        m &= m - 1;
        const int b = __builtin_ctzll(todo);
        todo &= todo - 1;
        if (slot == leader / W) take = b;
      }
      if (take >= 0) {
        seg = take;
        p = f3{sp[seg], sp[kChunk + seg], sp[2 * kChunk + seg]};
        q = f3{sp[3 * kChunk + seg], sp[4 * kChunk + seg], sp[5 * kChunk + seg]};
        r.px = p.x; r.py = p.y; r.pz = p.z;
        axis_setup(q.x - p.x, safe, r.ix, r.bx);
        axis_setup(q.y - p.y, safe, r.iy, r.by);
        axis_setup(q.z - p.z, safe, r.iz, r.bz);
        stk[0] = root;  // every lane of the slot writes the same entry
        top = 1;
      }
    }
    if (!ballot(seg >= 0)) break;
    if ((++iter & 15) == 0) {
      if (uni((int32_t)poll)) return true;
      poll = load_state(ra.state + pair);
    }
    const bool active = seg >= 0;
    int32_t ref = 0;
    if (active) ref = stk[--top];
    const bool is_leaf = active && ref < 0, is_inner = active && ref >= 0;
    // leaf: the slot's lanes test its triangles, W at a time
    uint32_t hitb = 0, ambb = 0;
    int32_t tfirst = 0;
    if (is_leaf) {
      const int32_t lr = ~ref;
      tfirst = lr >> 3;
      const int cnt = (lr & 7) + 1;
      if (c == 0) ++leaves;
      for (int t = c; t < cnt; t += W) {
        const float* tp = T.tris + 9 * (int64_t)(tfirst + t);
        const int res = leaf_test<PREC>(p, q, tri_vertex(tp, 0), tri_vertex(tp, 1), tri_vertex(tp, 2), safe);
        ++tests;
        hitb |= (res == kHit ? 1u : 0u) << (t / W);
        ambb |= (res == kAmbig ? 1u : 0u) << (t / W);
      }
      if (ambb) grid_tier<PREC>(p, q, T.tris, tfirst + c, W, hitb, ambb, n32, ngrid);
    }
    if (ballot(hitb != 0)) {
      if (lane == 0) mark_true(ra.state + pair);
      return true;
    }
    if (ballot(ambb != 0)) {
#pragma unroll
      for (int k = 0; k < (8 + W - 1) / W; ++k) {
        const bool amb = (ambb >> k) & 1u;
        if (!ballot(amb)) continue;
        if (!defer_tests(ra, amb, pair, dir, (int32_t)(gc * kChunk + seg), tfirst + c + k * W, st)) return true;
      }
    }
    // inner node: lane c tests child c against the slot's segment
    bool h = false;
    int32_t child = kEmpty;
    if (is_inner) {
      const Node<W>* n = nodes + ref;
      const float lx = n->lo[0][c], ly = n->lo[1][c], lz = n->lo[2][c];
      const float hx = n->hi[0][c], hy = n->hi[1][c], hz = n->hi[2][c];
      child = n->child[c];
      h = child != kEmpty && slab(r, lx, ly, lz, hx, hy, hz) && (safe || box_meet(cb, lx, ly, lz, hx, hy, hz));
      if (c == 0) ++visits;
    }
    const uint64_t hm = ballot(h);
    bool ovf = false;
    if (is_inner) {
      const uint32_t mine = (uint32_t)(hm >> (slot * W)) & kWMask;
      const int cnt = __popc(mine);
      if (top + cnt > CAP) {
        ovf = true;
      } else {
        if (h) stk[top + __popc(mine & ((1u << c) - 1u))] = child;
        top += cnt;
      }
    }
    // the pushes of one lane are read by the other lanes of its slot
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint64_t om = ballot(ovf && c == 0); om; om &= om - 1)
      overflow |= 1ull << __builtin_amdgcn_readlane(seg, __builtin_ctzll(om));
    if (ovf || (active && top == 0)) seg = -1;
  }
  return false;
}

// The top of a target tree as a frontier of boxes held one per lane: lane
// j W + d holds child d of node root + 1 + j, and lane c < W also holds root
// child c.  The builder numbers the root's internal children root + 1,
// root + 2, ... in child order, so the second level is known from the root's
// index alone and loads together with the root (nodes numbered after them
// lie deeper, and their boxes lie inside second-level boxes).  Every triangle
// lies inside a root leaf-child box or a second-level box, so a box that
// meets none of the frontier meets no triangle.  Absent entries hold
// inverted boxes, which meet nothing.
template <int W>
struct Frontier {
  float b2[6];  // second-level box of this lane
  float b1[6];  // root child box of lane c < W
  bool leaf1;   // lane c < W: root child c is a leaf
  int32_t c1;   // lane c < W: reference of root child c
  int32_t c2;   // reference of this lane's second-level entry (with REFS)
};

__device__ __forceinline__ bool meet6(const float* g, float lx, float ly, float lz, float hx, float hy, float hz) {
  return (g[0] <= hx) & (lx <= g[3]) & (g[1] <= hy) & (ly <= g[4]) & (g[2] <= hz) & (lz <= g[5]);
}

__device__ __forceinline__ float lane_f(float v, int j) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), j));
}

// With REFS the lanes also hold the child references of their entries.
template <int W, bool REFS = false>
__device__ __forceinline__ void load_frontier(Frontier<W>& F, const char* nodes, int32_t troot, int32_t n_nodes) {
  const int lane = threadIdx.x & 63;
  const int j = lane / W, d = lane % W;
  const int32_t n2 = min(W, n_nodes - 1);
#pragma unroll
  for (int a = 0; a < 3; ++a) { F.b2[a] = INFINITY; F.b2[3 + a] = -INFINITY; F.b1[a] = INFINITY; F.b1[3 + a] = -INFINITY; }
  F.leaf1 = false;
  F.c1 = kEmpty;
  F.c2 = kEmpty;
  if (j < n2) {
    const float* nd = reinterpret_cast<const float*>(nodes + sizeof(Node<W>) * ((int64_t)troot + 1 + j));
#pragma unroll
    for (int a = 0; a < 6; ++a) F.b2[a] = nd[a * W + d];
    if (REFS) F.c2 = reinterpret_cast<const int32_t*>(nd)[6 * W + d];
  }
  if (lane < W) {
    const float* nd = reinterpret_cast<const float*>(nodes + sizeof(Node<W>) * (int64_t)troot);
#pragma unroll
    for (int a = 0; a < 6; ++a) F.b1[a] = nd[a * W + lane];
    F.c1 = reinterpret_cast<const int32_t*>(nd)[6 * W + lane];
    F.leaf1 = F.c1 < 0 && F.c1 != kEmpty;
  }
}

// How one group is traced.
struct TraceOpts {
  WaveLds lds;
  bool rerun = false;          // k_fix rerun: no pair-state polling, every test exact
  uint64_t start_mask = 0;     // continue a handed-over task from `root` with these lanes
  int budget = 0;              // steps before the stack is handed over (0 = never)
  int tq = 0;                  // task list for the hand-over
  BlockShare* sh = nullptr;    // block work sharing
  int seg_max = 0;             // wave-per-segment when at most this many segments meet the root box
  int32_t n_nodes = 0;         // target's node count: > 0 starts the packet from the frontier
};

// Frontier entries a group may start from (each a subtree one or two levels
// below the root); with more, the group starts at the root.  At most 2W - 1
// entries, so that the stack bound of a root start (W - 1 entries per level)
// still holds.
template <int W>
constexpr int frontier_start_max() { return 2 * W - 1; }

// Traces segment group gc (global index in the source blob, `live` segments)
// against the target mesh whose root node is `root` and box `tb`.  Returns
// true when the pair is decided (found here or by another wave).  With a
// non-zero start_mask the trace continues a handed-over task instead: the
// stack starts as (root, start_mask) and the group's segments are not counted
// again.  With a budget, a group still running after that many steps hands its
// stack over to task list tq and returns.  Groups with at most seg_max
// segments meeting the target box take the wave-per-segment traversal.
template <int W, int PREC, int SCHED = 1>
__device__ bool trace_core(const BlobView& S, const BlobView& T, int64_t gc, int live, int32_t root,
                           const float* tb, int32_t pair, int32_t dir, bool safe, const RefineArgs& ra,
                           WaveStats& st, const TraceOpts& o) {
  const int lane = threadIdx.x & 63;
  const bool rerun = o.rerun;
  int budget = o.budget;
  BlockShare* const sh = o.sh;
  // issue every load the group needs at once: its box, its segments and the
  // pair's state
  const uint32_t decided = rerun ? 0u : load_state(ra.state + pair);
  float cb[6];
  const cptr_t<float> cbp = cview(S.cbox) + 8 * gc;
#pragma unroll
  for (int k = 0; k < 6; ++k) cb[k] = cbp[k];
  const bool valid = lane < live;
  const float* sp = S.seg + gc * (6 * kChunk);
  f3 p{sp[lane], sp[kChunk + lane], sp[2 * kChunk + lane]};
  f3 q{sp[3 * kChunk + lane], sp[4 * kChunk + lane], sp[5 * kChunk + lane]};
  Ray r;
  r.px = p.x; r.py = p.y; r.pz = p.z;
  axis_setup(q.x - p.x, safe, r.ix, r.bx);
  axis_setup(q.y - p.y, safe, r.iy, r.by);
  axis_setup(q.z - p.z, safe, r.iz, r.bz);
  if (uni((int32_t)decided)) return true;
  uint64_t m0 = o.start_mask;
  bool cont = m0 != 0;
  if (m0 == 0) {
    st.add(S_SEG, (uint64_t)live);
    m0 = ballot(valid && (tb == nullptr || slab(r, tb[0], tb[1], tb[2], tb[3], tb[4], tb[5])));
    if (m0 == 0) return false;
    if (SCHED != 1 && o.seg_max > 0 && o.lds.seg && __popcll(m0) <= o.seg_max) {
      st.add(S_GTRAV, 1);
      uint64_t over = 0;
      if (trace_segments<W, PREC>(S, T, gc, root, pair, dir, safe, m0, cb, ra, o.lds.seg, st, over)) return true;
      if (!over) return false;
      m0 = over;  // segments whose stacks overflowed: packet traversal from the root
      cont = true;
    }
  }
  // per-group counters (uniform, 32 bits), folded into the wave's statistics
  // when the group ends
  struct GroupCount {
    WaveStats& s;
    bool cont;
    uint32_t visits = 0, leaf_tris = 0, tests = 0;
    uint32_t n32 = 0, ngrid = 0;  // per lane
    __device__ ~GroupCount() {
      if (!cont) s.add(S_GTRAV, 1);
      s.add(S_VISIT, visits);
      s.add(S_TRIF, leaf_tris);
      s.add(S_TESTS, tests);
      if (PREC == 1) s.add(S_EXACT, tests);
      if (PREC != 1) {
        s.add(S_AMB32, wave_sum(n32));
        s.add(S_EXACT, wave_sum(ngrid));
      }
      s.max(S_MAXV, visits);
      s.max(S_MAXL, leaf_tris);
    }
  } gcount{st, cont};
  constexpr int CAP = stack_cap<W>();
  WaveStack stk;
  stk.ref = 0; stk.mlo = 0; stk.mhi = 0;
  stk.lref = o.lds.ref; stk.lmask = o.lds.mask; stk.top = 0;
  stack_layout(stk, o.lds);
  bool started = false;
  if (!cont && o.n_nodes > 1) {
    // Start below the root: the second-level children whose boxes the group
    // box meets are tested by every lane and pushed, so the root and the
    // second-level nodes are not visited.  Lane j W + d holds child d of
    // node root + 1 + j; only the root's internal children, nodes root + 1
    // ... root + n_inner, are second-level nodes.  A root with a leaf child
    // (small meshes) starts at the root.
    const int j = lane / W, d = lane % W;
    const int32_t rref = lane < W ? reinterpret_cast<const int32_t*>(T.nodes + sizeof(Node<W>) * (int64_t)root)[6 * W + lane]
                                  : kEmpty;
    float e[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    int32_t eref = kEmpty;
    if (j < min(W, o.n_nodes - 1)) {
      const float* nd = reinterpret_cast<const float*>(T.nodes + sizeof(Node<W>) * ((int64_t)root + 1 + j));
#pragma unroll
      for (int a = 0; a < 6; ++a) e[a] = nd[a * W + d];
      eref = reinterpret_cast<const int32_t*>(nd)[6 * W + d];
    }
    const uint64_t inner = ballot(rref >= 0 && rref != kEmpty);
    const uint64_t leaf = ballot(rref < 0);
    const int n_inner = __popcll(inner);
    const uint64_t f = ballot(lane < n_inner * W && eref != kEmpty && meet6(cb, e[0], e[1], e[2], e[3], e[4], e[5]));
    if (!leaf && __popcll(f) <= frontier_start_max<W>()) {
      started = true;
      // visits: the second-level nodes whose child boxes are tested here
#pragma unroll
      for (int i = 0; i < W; ++i) gcount.visits += ((f >> (i * W)) & ((1ull << W) - 1ull)) ? 1u : 0u;
      for (uint64_t fm = f; fm; fm &= fm - 1) {
        const int k = __builtin_ctzll(fm);
        const float lx = lane_f(e[0], k), ly = lane_f(e[1], k), lz = lane_f(e[2], k);
        const float hx = lane_f(e[3], k), hy = lane_f(e[4], k), hz = lane_f(e[5], k);
        const uint64_t m = safe ? ballot(slab(r, lx, ly, lz, hx, hy, hz)) & m0 : m0;
        if (m) stack_push(stk, __builtin_amdgcn_readlane(eref, k), m);
      }
      if (stk.top == 0) return false;
    }
  }
  if (!started) stack_push(stk, root, m0);
  int iter = 0;
  const cptr_t<Node<W>> nodes = cview(reinterpret_cast<const Node<W>*>(T.nodes));
  // the pair's state is polled every 16 pops; the load is issued one poll
  // ahead so that the traversal never waits for it
  uint32_t poll = 0;
  while (stk.top > 0) {
    if (budget && iter >= budget) {
      if (hand_over(stk, ra, o.tq, gc, (pair << 1) | dir, live | (safe ? 256 : 0))) return false;
      budget = 0;  // the rest did not fit: finish here
      if (stk.top == 0) return false;
    }
    --stk.top;
    const int32_t ref = stack_ref(stk, stk.top);
    const uint64_t nm = stack_mask(stk, stk.top);
    if (!rerun && (++iter & 15) == 0) {
      if (uni((int32_t)poll)) return true;
      poll = load_state(ra.state + pair);
    }
    if (sh && stk.top >= 1 && stk.top <= kRegStack) {
      // waves of the block waiting for work, beyond the tasks already waiting
      const uint32_t idle = lds_load(&sh->idle), tail = lds_load(&sh->tail), head = lds_load(&sh->head);
      const uint32_t n = tail < kBlkTasks ? tail : kBlkTasks;
      const uint32_t waiting = n > head ? n - head : 0u;
      const int want = uni((int32_t)(idle > waiting ? idle - waiting : 0u));
      if (want > 0 && tail < kBlkTasks)
        share_out(stk, sh, gc, (pair << 1) | dir, live | (safe ? 256 : 0), want < stk.top ? want : stk.top);
    }
    if (ref < 0) {
      // leaf: the lanes of the mask test their segment against its
      // triangles, four at a time, read as one contiguous block (the
      // triangle array has three triangles of slack at its end)
      const bool on = (nm >> lane) & 1ull;
      const int32_t lr = ~ref;
      const int32_t first = lr >> 3;
      const int cnt = (lr & 7) + 1;
      gcount.leaf_tris += (uint32_t)cnt;
      gcount.tests += (uint32_t)__popcll(nm) * (uint32_t)cnt;
      uint32_t hitbits = 0, ambbits = 0;
      for (int t0 = 0; t0 < cnt; t0 += 4) {
        const cptr_t<float> tp = cview(T.tris) + 9 * (int64_t)(first + t0);
        float tv[36];
#pragma unroll
        for (int k = 0; k < 36; ++k) tv[k] = tp[k];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (t0 + k >= cnt) break;
          const f3 ta{tv[9 * k], tv[9 * k + 1], tv[9 * k + 2]};
          const f3 tb3{tv[9 * k + 3], tv[9 * k + 4], tv[9 * k + 5]};
          const f3 tc{tv[9 * k + 6], tv[9 * k + 7], tv[9 * k + 8]};
          const int res = on ? leaf_test<PREC>(p, q, ta, tb3, tc, safe) : kMiss;
          hitbits |= (res == kHit ? 1u : 0u) << (t0 + k);
          ambbits |= (res == kAmbig ? 1u : 0u) << (t0 + k);
        }
      }
      if (ambbits) grid_tier<PREC>(p, q, T.tris, first, 1, hitbits, ambbits, gcount.n32, gcount.ngrid);
      if (ballot(hitbits != 0)) {
        if (lane == 0 && !rerun) mark_true(ra.state + pair);
        return true;
      }
      if (ballot(ambbits != 0)) {
        for (int t = 0; t < cnt; ++t) {
          const bool amb = (ambbits >> t) & 1u;
          if (!ballot(amb)) continue;
          // the queue is full: the whole pair is decided again later in FP64/exact
          if (!defer_tests(ra, amb, pair, dir, (int32_t)(gc * kChunk + lane), first + t, st)) return true;
        }
      }
      continue;
    }
    // inner node: all of it is loaded at once, every child is tested
    NodeRegs<W> nd;
    load_node<W>(nd, nodes + ref);
    ++gcount.visits;
    uint64_t hm[W];
    test_children<W>(nd, r, nm, safe, cb, hm);
    if (stk.top + W > CAP) {  // cannot happen for a valid blob (depth <= kMaxDepth)
      if (lane == 0) atomicMin(ra.status, (int32_t)PR_E_UNSUPPORTED);
      return true;
    }
#pragma unroll
    for (int c = 0; c < W; ++c)
      if (hm[c]) stack_push(stk, nd.ch[c], hm[c]);
  }
  return false;
}

// Group `chunk` of source mesh sm against target mesh tm; the caller has
// checked that the group's box meets the target mesh box.
template <int W, int PREC>
__device__ __forceinline__ bool trace_group(const BlobView& S, const BlobView& T, const MeshDesc& sm,
                                            const MeshDesc& tm, int32_t chunk, int32_t pair, int32_t dir, bool safe,
                                            const RefineArgs& ra, int32_t* lref, uint64_t* lmask, WaveStats& st,
                                            bool rerun = false) {
  const int64_t gc = (int64_t)sm.chunk_base + chunk;
  const int live = min(kChunk, sm.n_edges - chunk * kChunk);
  TraceOpts o;
  o.lds = wave_lds(lref, lmask);
  o.rerun = rerun;
  return trace_core<W, PREC>(S, T, gc, live, tm.root, tm.box, pair, dir, safe, ra, st, o);
}

// One group with its own box pre-test (per-pair and rerun kernels).
template <int W, int PREC>
__device__ bool trace_chunk(const BlobView& S, const BlobView& T, const MeshDesc& sm, const MeshDesc& tm,
                            int32_t chunk, int32_t pair, int32_t dir, bool safe, const RefineArgs& ra,
                            int32_t* snode, uint64_t* smask, WaveStats& st, bool rerun = false) {
  st.add(S_GROUPS, 1);
  if (tm.root == kEmpty) return false;
  const float* cbp = S.cbox + 8 * ((int64_t)sm.chunk_base + chunk);
  float cb[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) cb[k] = cbp[k];
  if (!box_meet(cb, tm.box[0], tm.box[1], tm.box[2], tm.box[3], tm.box[4], tm.box[5])) return false;
  st.add(S_GBOX, 1);
  return trace_group<W, PREC>(S, T, sm, tm, chunk, pair, dir, safe, ra, snode, smask, st, rerun);
}

__device__ __forceinline__ void flush_stats(const WaveStats& st, const RefineArgs& ra) {
  const int k = threadIdx.x & 63;
  if (k < S_N && st.acc) {
    unsigned long long* c = k == S_QOVER ? ra.stats : stat_copy(ra.stats);
    if (k == S_MAXV || k == S_MAXL) atomicMax(c + k, (unsigned long long)st.acc);
    else atomicAdd(c + k, (unsigned long long)st.acc);
  }
}

__device__ __forceinline__ bool pair_ok(const RefineArgs& ra, int64_t p, int32_t& i, int32_t& j) {
  i = ra.pairs[2 * p];
  j = ra.pairs[2 * p + 1];
  return i >= 0 && i < ra.n_meshes_a && j >= 0 && j < ra.n_meshes_b;
}

// Pairs processed: n_pairs, or the device count when one is given (clamped
// to [0, n_pairs]).
__device__ __forceinline__ int64_t npairs(const RefineArgs& ra) {
  if (!ra.np_dev) return ra.n_pairs;
  const int64_t v = *ra.np_dev;
  return v < 0 ? 0 : (v < ra.n_pairs ? v : ra.n_pairs);
}

__device__ __forceinline__ bool blobs_ok(const BlobView& A, const BlobView& B, const RefineArgs& ra, int W) {
  return A.magic == kMagic && B.magic == kMagic && A.width == W && B.width == W && A.n_meshes == ra.n_meshes_a &&
         B.n_meshes == ra.n_meshes_b;
}

// ---- setup --------------------------------------------------------------------

// Pair states are cleared for the pairs processed only (every kernel bounds
// its pairs by the device count).
__global__ void k_init(RefineArgs ra) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t np = npairs(ra);
  for (int64_t p = i; p < np; p += (int64_t)gridDim.x * blockDim.x) ra.state[p] = 0u;
  if (i < kStatCopies * S_N) ra.stats[kCtrStride * (i / S_N) + i % S_N] = 0ull;
  if (i < kSlices) {
    ra.ctr[kCtrStride * i] = 0ull;
    ra.qcount[kQCtrStride * i] = 0u;
  }
  if (i < 2 * kCostClasses) ra.ord_cnt[i] = 0u;
  if (i < kQueues) {
    ra.surv_cnt[kCtrStride * i] = 0ull;
    ra.surv_pop[kCtrStride * i] = 0ull;
    if (ra.task_cnt) {
      ra.task_cnt[kCtrStride * i] = 0ull;
      ra.task_pop[kCtrStride * i] = 0ull;
    }
  }
  if (i == 0) {
    *ra.status = PR_OK;
  }
}

// Cull order: many units per wave are taken from shares a few at a time, and
// a share ends with the units taken last; pairs are therefore culled in
// decreasing cost class (the two meshes' groups), so the last units taken are
// short.  Class sizes, then places; within a class the order is arbitrary
// (the results do not depend on it).
__device__ __forceinline__ int cost_class(const BlobView& A, const BlobView& B, const RefineArgs& ra, int64_t p) {
  int32_t i, j;
  if (!pair_ok(ra, p, i, j)) return kCostClasses - 1;
  const int64_t c = (int64_t)A.mesh[i].n_chunks + B.mesh[j].n_chunks;
  // class 0: 4,096 groups or more, then one class per halving, the last below 64
  const int lg = c > 0 ? 63 - __builtin_clzll((uint64_t)c) : 0;
  return lg >= 12 ? 0 : (lg <= 5 ? kCostClasses - 1 : 12 - lg);
}

__global__ void k_order_count(RefineArgs ra) {
  __shared__ uint32_t s_cnt[kCostClasses];
  if (threadIdx.x < kCostClasses) s_cnt[threadIdx.x] = 0u;
  __syncthreads();
  const BlobView A = view_of(ra.blob_a), B = view_of(ra.blob_b);
  const int64_t np = npairs(ra);
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&s_cnt[cost_class(A, B, ra, p)], 1u);
  __syncthreads();
  if (threadIdx.x < kCostClasses && s_cnt[threadIdx.x]) atomicAdd(ra.ord_cnt + threadIdx.x, s_cnt[threadIdx.x]);
}

// Each block places blockDim pairs per step: ranks within the block from LDS
// counters, one range per class reserved with one atomic.
__global__ void k_order_place(RefineArgs ra) {
  __shared__ uint32_t s_cnt[kCostClasses], s_off[kCostClasses];
  const BlobView A = view_of(ra.blob_a), B = view_of(ra.blob_b);
  const int64_t np = npairs(ra);
  uint32_t cbase[kCostClasses];
  cbase[0] = 0u;
  for (int k = 1; k < kCostClasses; ++k) cbase[k] = cbase[k - 1] + ra.ord_cnt[k - 1];
  for (int64_t b0 = blockIdx.x * (int64_t)blockDim.x; b0 < np; b0 += (int64_t)gridDim.x * blockDim.x) {
    if (threadIdx.x < kCostClasses) s_cnt[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t p = b0 + threadIdx.x;
    const bool live = p < np;
    const int c = live ? cost_class(A, B, ra, p) : 0;
    const uint32_t r = live ? atomicAdd(&s_cnt[c], 1u) : 0u;
    __syncthreads();
    if (threadIdx.x < kCostClasses && s_cnt[threadIdx.x])
      s_off[threadIdx.x] = atomicAdd(ra.ord_cnt + kCostClasses + threadIdx.x, s_cnt[threadIdx.x]);
    __syncthreads();
    if (live) ra.order[cbase[c] + s_off[c] + r] = (int32_t)p;
    __syncthreads();  // s_cnt / s_off are rewritten by the next step
  }
}

// Frontier entries (bits of f2 for second-level lanes, of f1 for root
// lanes) that box g meets, for every lane: one uniform step per entry of
// the candidate masks.
template <int W>
__device__ __forceinline__ void frontier_masks(const float* g, uint64_t f2, uint32_t f1, const Frontier<W>& F,
                                               uint64_t& m2, uint32_t& m1) {
  m2 = 0;
  m1 = 0;
  for (; f2; f2 &= f2 - 1) {
    const int j = __builtin_ctzll(f2);
    if (meet6(g, lane_f(F.b2[0], j), lane_f(F.b2[1], j), lane_f(F.b2[2], j), lane_f(F.b2[3], j),
              lane_f(F.b2[4], j), lane_f(F.b2[5], j)))
      m2 |= 1ull << j;
  }
  for (; f1; f1 &= f1 - 1) {
    const int j = __builtin_ctz(f1);
    if (meet6(g, lane_f(F.b1[0], j), lane_f(F.b1[1], j), lane_f(F.b1[2], j), lane_f(F.b1[3], j),
              lane_f(F.b1[4], j), lane_f(F.b1[5], j)))
      m1 |= 1u << j;
  }
}

// Whether box g meets one of the frontier entries of masks f2, f1; stops
// once every active lane has met one.
template <int W>
__device__ __forceinline__ bool meets_frontier(const float* g, uint64_t f2, uint32_t f1, const Frontier<W>& F) {
  bool hit = false;
  for (; f2; f2 &= f2 - 1) {
    const int j = __builtin_ctzll(f2);
    hit = hit | meet6(g, lane_f(F.b2[0], j), lane_f(F.b2[1], j), lane_f(F.b2[2], j), lane_f(F.b2[3], j),
                      lane_f(F.b2[4], j), lane_f(F.b2[5], j));
    if (!ballot(!hit)) return hit;
  }
  for (; f1; f1 &= f1 - 1) {
    const int j = __builtin_ctz(f1);
    hit = hit | meet6(g, lane_f(F.b1[0], j), lane_f(F.b1[1], j), lane_f(F.b1[2], j), lane_f(F.b1[3], j),
                      lane_f(F.b1[4], j), lane_f(F.b1[5], j));
  }
  return hit;
}

__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int j) {
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, j);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), j);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int size_bucket(int32_t n_tris) {
  return n_tris < (1 << 10) ? 0 : (n_tris < (1 << 13) ? 1 : (n_tris < (1 << 16) ? 2 : 3));
}

constexpr int kCullBuf = 256;  // survivor entries buffered per wave in LDS
constexpr int kRunsMin = 4;    // runs of 64 groups from which the cull tests run boxes first
// Multiplier of the pop-order permutation of a survivor queue; a prime above
// any queue length, so coprime with it.
constexpr uint64_t kSpread = 2654435761ull;
// k_cull: up to kCullStatic units per wave are dealt in a fixed stride;
// beyond, waves take kCullGrab units at a time from their XCD's share.
constexpr int kCullStatic = 8;
constexpr int kCullGrab = 4;

// Appends a wave's buffered survivors to its slice queue with one atomic.
// A survivor that does not fit marks its pair for the rerun pass (state 2:
// every group of the pair traced again, exactly), as an overflow of the
// deferred-test queue does.
__device__ void flush_survivors(const int4* buf, int n, int slice, const RefineArgs& ra, WaveStats& st) {
  const int lane = threadIdx.x & 63;
  unsigned long long b0 = 0;
  if (lane == 0) b0 = atomicAdd(ra.surv_cnt + kCtrStride * slice, (unsigned long long)n);
  const uint64_t base = uni64(b0);
  int4* q = ra.surv + (int64_t)slice * ra.surv_cap;
  uint32_t over = 0;
  for (int i = lane; i < n; i += 64) {
    const int4 e = buf[i];
    if (base + i < ra.surv_cap) {
      q[base + i] = e;
    } else {
      atomicCAS(ra.state + (e.y >> 1), 0u, 2u);
      ++over;
    }
  }
  if (base + n > ra.surv_cap) {
    for (int o = 32; o > 0; o >>= 1) over += __shfl_xor(over, o);
    st.add(S_QOVER, (uint64_t)over);
  }
}

// Persistent pass, phase 1: one wave per unit (pair, direction), units dealt to the
// waves in a fixed stride or, with many units per wave, taken from per-XCD
// shares a few at a time.  The wave validates the pair, tests the source
// mesh box against the target mesh box and the frontier of its top two
// levels, then culls the source groups 64 at a time (one group box per
// lane, the next 64 boxes loading while the current ones are tested) and
// buffers the survivors in LDS; full buffers go to the block's queue (blockIdx % kQueues, on
// the XCD the block runs on, so phase 2 mostly finds the pair's data in the
// same L2).  Survivor entry: global group index, unit, target root node,
// live segments | FP32-safe flag << 8 | target size bucket << 9 | target
// node count (at most 2^21 - 1) << 11, so that the tracing wave needs no
// descriptor.
template <int W, int PREC>
__global__ __launch_bounds__(kBlock, 7) void k_cull(RefineArgs ra) {
  __shared__ int4 s_buf[kWaves][kCullBuf];
  const int wv = uni((int32_t)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  const BlobView A = view_of(ra.blob_a), B = view_of(ra.blob_b);
  if (!blobs_ok(A, B, ra, W)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicMin(ra.status, (int32_t)PR_E_UNSUPPORTED);
    return;
  }
  const int slice = (int)(blockIdx.x % kQueues);
  int4* buf = s_buf[wv];
  int nbuf = 0;
  WaveStats st;
  const int64_t U = 2 * npairs(ra);
  const cptr_t<int32_t> pairs = cview(ra.pairs);
  // Culls unit u (pair ids ia, jb).
  auto cull_unit = [&](int64_t u, int32_t ia, int32_t jb) {
    const int32_t pair = (int32_t)(u >> 1), dir = (int32_t)(u & 1);
    if (ia < 0 || ia >= ra.n_meshes_a || jb < 0 || jb >= ra.n_meshes_b) {
      if (lane == 0) atomicMin(ra.status, (int32_t)PR_E_ARG);
      return;
    }
    const BlobView& S = dir == 0 ? A : B;
    const BlobView& T = dir == 0 ? B : A;
    const int32_t sid = dir == 0 ? ia : jb, tid = dir == 0 ? jb : ia;
    const cptr_t<MeshDesc> smd = cview(S.mesh) + sid;
    const cptr_t<MeshDesc> tmd = cview(T.mesh) + tid;
    float sb[6], tb[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) { sb[k] = smd->box[k]; tb[k] = tmd->box[k]; }
    const int32_t troot = tmd->root;
    const int32_t n_chunks = smd->n_chunks, n_edges = smd->n_edges, chunk_base = smd->chunk_base;
    const bool safe = (smd->flags & tmd->flags & kMeshSafe) != 0;
    const int32_t tword = (safe ? 256 : 0) | (size_bucket(tmd->n_tris) << 9) | (min(tmd->n_nodes, (1 << 21) - 1) << 11);
    if (troot == kEmpty || n_chunks <= 0 || !box_meet(sb, tb[0], tb[1], tb[2], tb[3], tb[4], tb[5])) return;
    // Groups come in runs of 64 (one per lane), each with a run box.  With
    // at least kRunsMin runs, the run boxes are tested first, 64 at a time,
    // and only the groups of the runs that pass are read; fewer runs are
    // read group by group (the extra dependent load of the run level costs
    // more than it saves there).  The first boxes load together with the
    // frontier.
    const float* cbox = S.cbox + 8 * (int64_t)chunk_base;
    const float* rbox = S.rbox + 8 * (int64_t)chunk_base;
    const int32_t n_all = (n_chunks + kChunk - 1) / kChunk;
    const bool hier = n_all >= kRunsMin;
    const int32_t n_runs = hier ? n_all : 1;
    float g[6], gn[6];
    {
      const float* cp = hier ? rbox + 8 * (int64_t)kChunk * min(lane, n_runs - 1)
                                   : cbox + 8 * (int64_t)min(lane, n_chunks - 1);
#pragma unroll
      for (int k = 0; k < 6; ++k) g[k] = cp[k];
    }
    Frontier<W> F;
    load_frontier<W>(F, T.nodes, troot, tmd->n_nodes);
    // the whole source mesh against the frontier: the entries it meets are
    // the only ones its runs and groups can meet
    const uint64_t f2m = ballot(meet6(sb, F.b2[0], F.b2[1], F.b2[2], F.b2[3], F.b2[4], F.b2[5]));
    const uint32_t f1m = (uint32_t)ballot(F.leaf1 && meet6(sb, F.b1[0], F.b1[1], F.b1[2], F.b1[3], F.b1[4], F.b1[5]));
    if (!(f2m | f1m)) return;
    // One loop over items, each 64 boxes (one per lane): a batch of run
    // boxes, or the groups of one run.  A run batch records, per run, the
    // frontier entries its box meets; a run's groups are tested against those
    // only.  After a run batch, the groups of its passing runs follow, then
    // the next batch.  While a run's groups are tested, the next item's boxes
    // load.
    uint64_t rm2 = 0;             // per lane (run of the batch): frontier entries met
    uint32_t rm1 = 0;
    uint64_t f2 = f2m;            // entries the groups in g can meet
    uint32_t f1 = f1m;
    int32_t r0 = 0;               // first run of the current batch
    // passing runs of the batch not yet loaded (without the run level:
    // every run after the first, whose groups are in g)
    uint64_t rmask = hier ? 0ull : ((1ull << n_all) - 1ull) & ~1ull;
    auto load_runs = [&](int32_t rb, float* dst) {
      const float* cp = rbox + 8 * (int64_t)kChunk * min(rb + lane, n_runs - 1);
#pragma unroll
      for (int k = 0; k < 6; ++k) dst[k] = cp[k];
    };
    auto load_groups = [&](int32_t r, float* dst) {
      const float* cp = cbox + 8 * (int64_t)min(r * kChunk + lane, n_chunks - 1);
#pragma unroll
      for (int k = 0; k < 6; ++k) dst[k] = cp[k];
    };
    auto next_run = [&]() {
      const int32_t r = r0 + __builtin_ctzll(rmask);
      rmask &= rmask - 1;
      return r;
    };
    float g2[6];                  // boxes of the run after next
    bool batch = hier;            // g holds a batch of run boxes
    int32_t cur = 0;              // run of the groups in g
    while (true) {
      if (batch) {
        frontier_masks<W>(g, f2m, f1m, F, rm2, rm1);
        const bool pass = r0 + lane < n_runs && box_meet(g, tb[0], tb[1], tb[2], tb[3], tb[4], tb[5]) &&
                          (rm2 | rm1) != 0;
        rmask = ballot(pass);
        if (!rmask) {
          if (r0 + kChunk >= n_runs) break;
          r0 += kChunk;
          load_runs(r0, g);
          continue;
        }
        cur = next_run();
        load_groups(cur, g);
      }
      // the groups of the batch's passing runs, with the boxes of the next
      // two runs loading while a run is tested
      int32_t n1 = -1, n2 = -1;
      if (rmask) { n1 = next_run(); load_groups(n1, gn); }
      if (rmask) { n2 = next_run(); load_groups(n2, g2); }
      while (true) {
        if (hier) {
          f2 = lane_u64(rm2, cur - r0);
          f1 = (uint32_t)__builtin_amdgcn_readlane((int)rm1, cur - r0);
        }
        const int32_t idx = cur * kChunk + lane;
        const bool pass = idx < n_chunks && box_meet(g, tb[0], tb[1], tb[2], tb[3], tb[4], tb[5]) &&
                          meets_frontier<W>(g, f2, f1, F);
        const uint64_t mask = ballot(pass);
        st.add(S_GROUPS, (uint64_t)min(kChunk, n_chunks - cur * kChunk));
        if (mask) {
          const int n = __popcll(mask);
          st.add(S_GBOX, (uint64_t)n);
          if (nbuf + n > kCullBuf) {
            flush_survivors(buf, nbuf, slice, ra, st);
            nbuf = 0;
          }
          if (pass) {
            const int live = min(kChunk, n_edges - idx * kChunk);
            buf[nbuf + lanes_below(mask)] = make_int4(chunk_base + idx, (int32_t)u, troot, live | tword);
          }
          nbuf += n;
        }
        if (n1 < 0) break;
        cur = n1;
        n1 = n2;
        n2 = -1;
#pragma unroll
        for (int k = 0; k < 6; ++k) { g[k] = gn[k]; gn[k] = g2[k]; }
        if (rmask) { n2 = next_run(); load_groups(n2, g2); }
      }
      if (!hier || r0 + kChunk >= n_runs) break;
      r0 += kChunk;
      load_runs(r0, g);
      batch = true;
    }
  };
  const int64_t nw = (int64_t)gridDim.x * kWaves;
  if (U <= kCullStatic * nw) {
    // few units per wave: dealt in a fixed stride, the pair of the wave's
    // next unit read while the current one is culled
    const int64_t u0 = (int64_t)blockIdx.x * kWaves + wv;
    int32_t next_a = 0, next_b = 0;
    if (u0 < U) {
      next_a = pairs[2 * (u0 >> 1)];
      next_b = pairs[2 * (u0 >> 1) + 1];
    }
    for (int64_t u = u0; u < U; u += nw) {
      const int32_t ia = next_a, jb = next_b;
      if (u + nw < U) {
        next_a = pairs[2 * ((u + nw) >> 1)];
        next_b = pairs[2 * ((u + nw) >> 1) + 1];
      }
      cull_unit(u, ia, jb);
    }
  } else {
    // many units per wave, of uneven cost: one share per XCD, from which the
    // waves of that XCD take kCullGrab units at a time (the next grab in
    // flight while the current units are culled), so a block that starts
    // late or draws large meshes takes fewer.  With the cull order, share xs
    // holds pairs xs, xs + nsl, ... of the order (both directions of each),
    // the costliest first; otherwise a contiguous range of units.
    const int nsl = gridDim.x < (unsigned)kSlices ? 1 : kSlices;
    const int xs = (int)(blockIdx.x % nsl);
    const int64_t np = U >> 1;
    const int64_t slo = ra.ordered ? 0 : U * xs / nsl;
    const int64_t shi = ra.ordered ? 2 * ((np - xs + nsl - 1) / nsl) : U * (xs + 1) / nsl;
    unsigned long long* const uctr = ra.ctr + kCtrStride * xs;
    unsigned long long g0 = 0;
    if (lane == 0) g0 = atomicAdd(uctr, (unsigned long long)kCullGrab);
    int64_t ub = slo + (int64_t)uni64(g0);
    while (ub < shi) {
      unsigned long long gnext = 0;
      if (lane == 0) gnext = atomicAdd(uctr, (unsigned long long)kCullGrab);
      const int64_t ue = ub + kCullGrab < shi ? ub + kCullGrab : shi;
      int64_t pl = -1;
      int32_t ia = 0, jb = 0;
      for (int64_t k = ub; k < ue; ++k) {
        const int64_t pk = ra.ordered ? (int64_t)ra.order[xs + nsl * (k >> 1)] : (k >> 1);
        const int64_t u = 2 * pk + (k & 1);
        if (pk != pl) {
          pl = pk;
          ia = pairs[2 * pl];
          jb = pairs[2 * pl + 1];
        }
        cull_unit(u, ia, jb);
      }
      ub = slo + (int64_t)uni64(gnext);
    }
  }
  if (nbuf) flush_survivors(buf, nbuf, slice, ra, st);
  flush_stats(st, ra);
}

// After its queues are drained a wave takes tasks from its block's list
// (pending stack entries that the block's tracing waves moved out on seeing
// it wait) until no wave of the block is still on its queues or tracing a
// task and the list is drained.  A wave that moves entries out comes back
// here afterwards and leaves only after seeing the list drained, so no task
// is left behind.  All waiting is on LDS; a wait longer than kHelpSpinLimit
// looks (far beyond any traversal) reports PR_E_DEVICE and leaves.
constexpr uint32_t kHelpSpinLimit = 1u << 22;

template <int W, int PREC>
__device__ void block_help(const BlobView& A, const BlobView& B, const RefineArgs& ra, BlockShare* sh, const WaveLds& lds,
                           WaveStats& st) {
  const int lane = threadIdx.x & 63;
  if (lane == 0) {
    __hip_atomic_fetch_add(&sh->idle, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(&sh->active, ~0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  for (uint32_t spin = 0;; ++spin) {
    if (spin >= kHelpSpinLimit) {
      if (lane == 0) atomicMin(ra.status, (int32_t)PR_E_DEVICE);
      break;
    }
    const uint32_t tail = lds_load(&sh->tail), head = lds_load(&sh->head);
    const uint32_t n = tail < kBlkTasks ? tail : kBlkTasks;
    if (uni((int32_t)(head < n))) {
      // announce the attempt before claiming: a wave deciding whether to
      // leave reads the busy count before the list
      if (lane == 0) __hip_atomic_fetch_add(&sh->busy, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
      uint32_t got = ~0u;
      if (lane == 0) {
        uint32_t h = lds_load(&sh->head);
        for (int t = 0; t < 64; ++t) {
          const uint32_t tl = lds_load(&sh->tail);
          if (h >= (tl < kBlkTasks ? tl : kBlkTasks)) break;
          uint32_t e = h;
          if (__hip_atomic_compare_exchange_strong(&sh->head, &e, h + 1, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP)) {
            got = h;
            break;
          }
          h = e;
        }
      }
      got = (uint32_t)uni((int32_t)got);
      if (got == ~0u) {
        if (lane == 0) __hip_atomic_fetch_add(&sh->busy, ~0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        continue;
      }
      if (lane == 0) __hip_atomic_fetch_add(&sh->idle, ~0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      // the slot was reserved by a wave of this block that writes it next
      uint32_t ok = 0;
      for (uint32_t w = 0; w < kHelpSpinLimit && !ok; ++w) {
        ok = (uint32_t)uni((int32_t)__hip_atomic_load(&sh->ready[got], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
        if (!ok) __builtin_amdgcn_s_sleep(1);
      }
      if (!ok) {
        if (lane == 0) {
          atomicMin(ra.status, (int32_t)PR_E_DEVICE);
          __hip_atomic_fetch_add(&sh->busy, ~0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        break;
      }
      const int4 t = sh->task[got];
      const uint64_t m = sh->mask[got];
      const int32_t pair = t.y >> 1, dir = t.y & 1;
      const BlobView& S = dir == 0 ? A : B;
      const BlobView& T = dir == 0 ? B : A;
      const float tb_unused[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // the root was tested when the group started
      TraceOpts o;
      o.lds = lds;
      o.start_mask = uni64(m);
      o.sh = sh;
      trace_core<W, PREC>(S, T, uni(t.x), uni(t.w) & 0xff, uni(t.z), tb_unused, pair, dir, (uni(t.w) & 256) != 0, ra,
                          st, o);
      if (lane == 0) {
        __hip_atomic_fetch_add(&sh->idle, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(&sh->busy, ~0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      spin = 0;
      continue;
    }
    // nothing to take: leave once no wave of the block is on its queues or
    // tracing a task (read first) and the list is drained (read after)
    if (uni((int32_t)(__hip_atomic_load(&sh->active, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) == 0u &&
                      __hip_atomic_load(&sh->busy, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) == 0u))) {
      const uint32_t tl = lds_load(&sh->tail);
      if (uni((int32_t)(lds_load(&sh->head) >= (tl < kBlkTasks ? tl : kBlkTasks)))) break;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}


// Target-size buckets of the automatic schedule (triangles of the target
// mesh: below 2^10, 2^13, 2^16, and larger) and the per-bucket limit on the
// segments of a group that meet the target box for the group to be traced
// wave-per-segment (byte k of the table).
// Persistent pass, phase 2: waves pop surviving groups kPop at a time from the
// queue of their block (blockIdx % kQueues, on the XCD whose phase-1 blocks
// filled it) and trace them; a wave leaves a queue after its first empty pop
// and then helps with the other queues of its XCD (q + 8, q + 16, ...), so
// the queues of one XCD finish together.  No wave touches another XCD's
// counters (a counter that many waves hit is a memory-side hot spot).  With
// fewer blocks than queues a block drains queues blockIdx, blockIdx +
// gridDim, ...  Pop slot j maps to
// queue slot j * kSpread mod (slots): the queue holds each pair's groups side
// by side, and spreading them over the run lets a hit found in one group
// cancel the pair's later groups.  A wave whose queues are drained then
// takes the pending subtrees that the other waves of its block hand over
// (`block_help`), so the block's long traversals end together.
template <int W, int PREC, int SCHED>
__global__ __launch_bounds__(kBlock, SCHED == 1 ? 6 : 5) void k_trace(RefineArgs ra) {
  __shared__ uint64_t s_area[kWaves][wave_lds_words<W>()];
  __shared__ BlockShare s_share;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (threadIdx.x < kBlkTasks) s_share.ready[threadIdx.x] = 0u;
  if (threadIdx.x == 0) {
    s_share.tail = 0u;
    s_share.head = 0u;
    s_share.idle = 0u;
    s_share.active = kWaves;
    s_share.busy = 0u;
  }
  __syncthreads();
  // with the stack's first entries in LDS there is no hand-over of stack entries
  const bool lds_only = ra.lds_stack != 0;
  BlockShare* const sh = ra.share && !lds_only ? &s_share : nullptr;
  TraceOpts o;
  o.lds = wave_lds<W>(s_area[wv], lds_only);
  o.budget = lds_only ? 0 : ra.budget;
  o.sh = sh;
  const BlobView A = view_of(ra.blob_a), B = view_of(ra.blob_b);
  if (!blobs_ok(A, B, ra, W)) return;
  WaveStats st;
  const int home = (int)(blockIdx.x % kQueues);
  const bool few = gridDim.x < (unsigned)kQueues;
  // with a full grid: home, then the XCD's other queues; with a small one:
  // home, home + gridDim, ... (every queue has a block)
  const int nq = few ? (kQueues - 1 - home) / (int)gridDim.x + 1 : kQueues / kSlices;
  for (int j = 0; j < nq; ++j) {
    const int cid = few ? home + j * (int)gridDim.x : (home + j * kSlices) % kQueues;
    const uint64_t filled = ra.surv_cnt[kCtrStride * cid];
    const uint64_t n = filled < ra.surv_cap ? filled : ra.surv_cap;
    // groups popped at a time: 8 from queues long enough to give every wave
    // that drains them dozens of batches, else 4 (the last batches of a
    // short queue set its end)
    const uint64_t qwaves = (uint64_t)gridDim.x * kWaves / kQueues + 1;
    const int kPop = n >= 64 * qwaves ? 8 : 4;
    const uint64_t slots = (n + kPop - 1) / kPop;
    const cptr_t<int32_t> q = cview(reinterpret_cast<const int32_t*>(ra.surv + (int64_t)cid * ra.surv_cap));
    for (;;) {
      unsigned long long k0 = 0;
      if (lane == 0) k0 = atomicAdd(ra.surv_pop + kCtrStride * cid, (unsigned long long)kPop);
      const uint64_t k = uni64(k0);
      if (k >= n) break;
      const uint64_t e0 = ((k / kPop) * kSpread % slots) * kPop;
      const int cnt = (int)((e0 + kPop < n ? e0 + kPop : n) - e0);
      // lane j < cnt reads entry e0 + j and its pair's state, all at once:
      // groups of pairs already decided are dropped before their segments load
      const int32_t unit_l = lane < cnt ? q[4 * (e0 + lane) + 1] : 0;
      const bool todo_l = lane < cnt && load_state(ra.state + (unit_l >> 1)) == 0u;
      for (uint64_t todo = ballot(todo_l); todo; todo &= todo - 1) {
        const uint64_t e = e0 + __builtin_ctzll(todo);
        const int4 it = make_int4(q[4 * e], q[4 * e + 1], q[4 * e + 2], q[4 * e + 3]);
        const int32_t pair = it.y >> 1, dir = it.y & 1;
        const BlobView& S = dir == 0 ? A : B;
        const BlobView& T = dir == 0 ? B : A;
        o.tq = cid;
        o.n_nodes = (int32_t)((uint32_t)it.w >> 11);
        if (SCHED == 1) {
          // the entry names the target's root and node count: no descriptor
          // read, and no target-box test (the frontier entries lie inside it)
          o.seg_max = 0;
          trace_core<W, PREC, SCHED>(S, T, it.x, it.w & 0xff, it.z, nullptr, pair, dir, (it.w & 256) != 0, ra, st, o);
        } else {
          const int32_t tid = ra.pairs[2 * pair + (dir == 0 ? 1 : 0)];
          const cptr_t<MeshDesc> tmd = cview(T.mesh) + tid;
          float tb[6];
#pragma unroll
          for (int c = 0; c < 6; ++c) tb[c] = tmd->box[c];
          o.seg_max = (int)((ra.seg_table >> (8 * ((it.w >> 9) & 3))) & 0xffu);
          trace_core<W, PREC, SCHED>(S, T, it.x, it.w & 0xff, it.z, tb, pair, dir, (it.w & 256) != 0, ra, st, o);
        }
      }
    }
  }
  if (sh) block_help<W, PREC>(A, B, ra, sh, o.lds, st);
  flush_stats(st, ra);
}

// Persistent pass, optional phase 3: the stacks that phase 2 handed over, one task (node,
// lane mask of its group) at a time, popped like the survivors: task list of
// the block first, then the other lists of its XCD.
template <int W, int PREC>
__global__ __launch_bounds__(kBlock, 5) void k_trace2(RefineArgs ra) {
  constexpr int CAP = lds_stack_cap<W>();
  __shared__ int32_t s_node[kWaves][CAP];
  __shared__ uint64_t s_mask[kWaves][CAP];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const BlobView A = view_of(ra.blob_a), B = view_of(ra.blob_b);
  if (!blobs_ok(A, B, ra, W)) return;
  WaveStats st;
  const int home = (int)(blockIdx.x % kQueues);
  const bool few = gridDim.x < (unsigned)kQueues;
  const int nq = few ? (kQueues - 1 - home) / (int)gridDim.x + 1 : kQueues / kSlices;
  for (int j = 0; j < nq; ++j) {
    const int cid = few ? home + j * (int)gridDim.x : (home + j * kSlices) % kQueues;
    const uint64_t filled = ra.task_cnt[kCtrStride * cid];
    const uint64_t n = filled < ra.task_cap ? filled : ra.task_cap;
    if (n == 0) continue;
    const cptr_t<int32_t> q = cview(reinterpret_cast<const int32_t*>(ra.tasks + (int64_t)cid * ra.task_cap));
    const cptr_t<uint64_t> qm = cview(ra.tmask + (int64_t)cid * ra.task_cap);
    for (;;) {
      unsigned long long k0 = 0;
      if (lane == 0) k0 = atomicAdd(ra.task_pop + kCtrStride * cid, 1ull);
      const uint64_t e = uni64(k0);
      if (e >= n) break;
      const int4 it = make_int4(q[4 * e], q[4 * e + 1], q[4 * e + 2], q[4 * e + 3]);
      const uint64_t m = qm[e];
      const int32_t pair = it.y >> 1, dir = it.y & 1;
      const BlobView& S = dir == 0 ? A : B;
      const BlobView& T = dir == 0 ? B : A;
      const float tb_unused[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // the root test was done in phase 2
      TraceOpts o;
      o.lds = wave_lds(s_node[wv], s_mask[wv]);
      o.start_mask = m;
      trace_core<W, PREC>(S, T, it.x, it.w & 0xff, it.z, tb_unused, pair, dir, (it.w & 256) != 0, ra, st, o);
    }
  }
  flush_stats(st, ra);
}

template <int W, int PREC>
__global__ __launch_bounds__(kBlock) void k_refine_pair(RefineArgs ra, int64_t p) {
  constexpr int CAP = lds_stack_cap<W>();
  __shared__ int32_t s_node[kWaves][CAP];
  __shared__ uint64_t s_mask[kWaves][CAP];
  const int wv = threadIdx.x >> 6;
  const BlobView A = view_of(ra.blob_a), B = view_of(ra.blob_b);
  int32_t i, j;
  if (p >= npairs(ra)) return;  // beyond the device count
  if (!blobs_ok(A, B, ra, W)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicMin(ra.status, (int32_t)PR_E_UNSUPPORTED);
    return;
  }
  if (!pair_ok(ra, p, i, j)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicMin(ra.status, (int32_t)PR_E_ARG);
    return;
  }
  const MeshDesc a = A.mesh[i], b = B.mesh[j];
  if (!box_meet(a.box, b.box[0], b.box[1], b.box[2], b.box[3], b.box[4], b.box[5])) return;
  WaveStats st;
  const int32_t gw = (int32_t)(blockIdx.x * kWaves + wv), nw = (int32_t)(gridDim.x * kWaves);
  const bool safe = (a.flags & b.flags & kMeshSafe) != 0;
  const int32_t pr32 = (int32_t)p;
  for (int dir = 0; dir < 2; ++dir) {
    const MeshDesc& sm = dir == 0 ? a : b;
    const MeshDesc& tm = dir == 0 ? b : a;
    bool done = false;
    for (int32_t c = gw; c < sm.n_chunks; c += nw) {
      if (load_state(ra.state + p)) { done = true; break; }
      if (trace_chunk<W, PREC>(dir == 0 ? A : B, dir == 0 ? B : A, sm, tm, c, pr32, dir, safe, ra, s_node[wv],
                               s_mask[wv], st)) { done = true; break; }
    }
    if (done) break;
  }
  flush_stats(st, ra);
}

__device__ void redecide(const RefineArgs& ra);

// After the traversal: (1) the deferred tests of undecided pairs (state 0) are
// decided in FP64/exact, one thread per test; (2) pairs whose deferred tests
// or survivors overflowed a queue (state 2) are traced again with every leaf
// test decided in place in FP64/exact, one block per pair.  The two parts
// touch disjoint pairs.
template <int W>
__global__ __launch_bounds__(kBlock) void k_fix(RefineArgs ra) {
  constexpr int CAP = lds_stack_cap<W>();
  __shared__ int32_t s_node[kWaves][CAP];
  __shared__ uint64_t s_mask[kWaves][CAP];
  __shared__ uint32_t s_hit;
  redecide(ra);
  const int wv = threadIdx.x >> 6;
  const BlobView A = view_of(ra.blob_a), B = view_of(ra.blob_b);
  if (!blobs_ok(A, B, ra, W)) return;
  WaveStats st;
  if (ra.stats[S_QOVER] == 0) return;  // nothing overflowed: nothing to rerun
  const int64_t np = npairs(ra);
  for (int64_t p = blockIdx.x; p < np; p += gridDim.x) {
    if (load_state(ra.state + p) != 2u) continue;
    if (threadIdx.x == 0) s_hit = 0;
    __syncthreads();
    int32_t i, j;
    pair_ok(ra, p, i, j);
    const MeshDesc a = A.mesh[i], b = B.mesh[j];
    for (int dir = 0; dir < 2; ++dir) {
      const MeshDesc& sm = dir == 0 ? a : b;
      const MeshDesc& tm = dir == 0 ? b : a;
      for (int32_t c = wv; c < sm.n_chunks; c += kWaves) {
        if (s_hit) break;
        if (trace_chunk<W, 1>(dir == 0 ? A : B, dir == 0 ? B : A, sm, tm, c, (int32_t)p, dir,
                              (sm.flags & tm.flags & kMeshSafe) != 0, ra, s_node[wv], s_mask[wv], st, true))
          s_hit = 1;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) ra.state[p] = s_hit ? 1u : 0u;
    __syncthreads();
  }
  flush_stats(st, ra);
}

// ---- deferred FP64 / exact decisions ----------------------------------------------

__device__ void redecide(const RefineArgs& ra) {
  const BlobView A = view_of(ra.blob_a), B = view_of(ra.blob_b);
  uint64_t nexact = 0, namb = 0;
  for (int qx = 0; qx < kSlices; ++qx) {
    const uint32_t qn = ra.qcount[kQCtrStride * qx];
    const uint32_t n = qn < ra.qsub ? qn : ra.qsub;
    const int4* queue = ra.queue + (int64_t)qx * ra.qsub;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
      const int4 e = queue[k];
      if (load_state(ra.state + e.x)) continue;
      const BlobView& S = e.y == 0 ? A : B;
      const BlobView& T = e.y == 0 ? B : A;
      const int64_t slot = e.z;
      const float* sp = S.seg + (slot / kChunk) * (6 * kChunk) + (slot % kChunk);
      const f3 p{sp[0], sp[kChunk], sp[2 * kChunk]}, q{sp[3 * kChunk], sp[4 * kChunk], sp[5 * kChunk]};
      const float* tp = T.tris + 9 * (int64_t)e.w;
      ExactCounters ec{0};
      const bool h = seg_tri_exact(p, q, tri_vertex(tp, 0), tri_vertex(tp, 1), tri_vertex(tp, 2), ec);
      ++nexact;
      if (ec.exact_signs) ++namb;
      if (h) mark_true(ra.state + e.x);
    }
  }
  if (nexact) atomicAdd(stat_copy(ra.stats) + S_EXACT, (unsigned long long)nexact);
  if (namb) atomicAdd(stat_copy(ra.stats) + S_AMB64, (unsigned long long)namb);
}

// Statistics and status out: one wave, lane c reads copy c of the counters
// (agent-scope loads: other XCDs wrote them), then sums (maxima) across lanes.
__device__ void report(const RefineArgs& ra, pr_refine_stats* out, int32_t* dev_status) {
  static_assert(kStatCopies == 64, "one lane per copy");
  const int lane = threadIdx.x & 63;
  if (out) {
    unsigned long long v[S_N];
    // every load issued before the first reduction
#pragma unroll
    for (int k = 0; k < S_N; ++k)
      v[k] = __hip_atomic_load(ra.stats + kCtrStride * lane + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int k = 0; k < S_N; ++k) {
      unsigned long long x = v[k];
      for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(x, o);
        x = (k == S_MAXV || k == S_MAXL) ? (y > x ? y : x) : x + y;
      }
      v[k] = x;
    }
    if (lane == 0) {
      out->segments = v[S_SEG];
      out->node_visits = v[S_VISIT];
      out->tri_tests = v[S_TESTS];
      out->fp32_ambiguous = v[S_AMB32];
      out->fp64_filter_ambiguous = v[S_AMB64];
      out->exact_decided = v[S_EXACT];
      out->pairs_true = v[S_TRUE];
      out->queue_overflow = v[S_QOVER];
      out->groups = v[S_GROUPS];
      out->tri_fetches = v[S_TRIF];
      out->groups_box_pass = v[S_GBOX];
      out->groups_traversed = v[S_GTRAV];
      out->max_group_node_visits = v[S_MAXV];
      out->max_group_leaf_fetches = v[S_MAXL];
    }
  }
  if (dev_status && lane == 0)
    *dev_status = __hip_atomic_load(ra.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Flags from the pair states and the intersecting-pair count; the report
// follows as a kernel of its own (the launch boundary orders the counts
// without device-wide fences in every block).
__global__ __launch_bounds__(kBlock) void k_finalize(RefineArgs ra) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  unsigned long long cnt = 0;
  const int64_t np = npairs(ra);
  for (; p < np; p += (int64_t)gridDim.x * blockDim.x) {
    const uint8_t f = ra.state[p] == 1u ? 1 : 0;
    ra.flags[p] = f;
    cnt += f;
  }
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(stat_copy(ra.stats) + S_TRUE, cnt);
}

// The report alone (no pairs).
__global__ void k_report(RefineArgs ra, pr_refine_stats* out, int32_t* dev_status) { report(ra, out, dev_status); }

// ---- host side ---------------------------------------------------------------------

void carve(Carve& cv, RefineArgs& ra, int64_t P, uint32_t qcap, uint32_t surv_cap, bool with_tasks) {
  ra.state = cv.take<uint32_t>(P);
  ra.ctr = cv.take<unsigned long long>(kSlices * kCtrStride);
  ra.qcount = cv.take<uint32_t>(kSlices * kQCtrStride);
  ra.stats = cv.take<unsigned long long>(kStatCopies * kCtrStride);
  ra.status = cv.take<int32_t>(1);
  ra.queue = cv.take<int4>((int64_t)kSlices * ((qcap + kSlices - 1) / kSlices));
  ra.surv_cnt = cv.take<unsigned long long>(kQueues * kCtrStride);
  ra.surv_pop = cv.take<unsigned long long>(kQueues * kCtrStride);
  ra.surv = cv.take<int4>((int64_t)kQueues * surv_cap);
  ra.order = cv.take<int32_t>(P);
  ra.ord_cnt = cv.take<uint32_t>(64);
  if (with_tasks) {  // continuation task lists: only with a step budget
    ra.task_cap = kTaskCap;
    ra.tasks = cv.take<int4>((int64_t)kQueues * kTaskCap);
    ra.tmask = cv.take<uint64_t>((int64_t)kQueues * kTaskCap);
    ra.task_cnt = cv.take<unsigned long long>(kQueues * kCtrStride);
    ra.task_pop = cv.take<unsigned long long>(kQueues * kCtrStride);
  }
}

int check(int64_t P, const pr_refine_params* p) {
  if (!p) { set_error("params is NULL"); return PR_E_ARG; }
  if (!(p->bvh_width == 2 || p->bvh_width == 4 || p->bvh_width == 8)) { set_error("bvh_width must be 2, 4 or 8"); return PR_E_ARG; }
  if (p->precision < 0 || p->precision > 3) { set_error("precision must be 0, 1, 2 or 3"); return PR_E_ARG; }
  if (p->persistent < 0 || p->persistent > 1) { set_error("persistent must be 0 or 1"); return PR_E_ARG; }
  if (p->queue_cap < 0 || p->grid_blocks < 0) { set_error("negative launch parameter"); return PR_E_ARG; }
  if (p->schedule < 0 || p->schedule > 2) { set_error("schedule must be 0 (auto), 1 (wave-per-pair) or 2 (wave-per-segment)"); return PR_E_ARG; }
  if (p->lds_stack < 0 || p->lds_stack > 1) { set_error("lds_stack must be 0 or 1"); return PR_E_ARG; }
  if (p->survivor_cap < 0) { set_error("survivor_cap < 0"); return PR_E_ARG; }
  if (p->trace_budget < -1) { set_error("trace_budget < -1"); return PR_E_ARG; }
  if (P < 0) { set_error("n_pairs < 0"); return PR_E_ARG; }
  if (P >= ((int64_t)1 << 30)) { set_error("n_pairs >= 2^30"); return PR_E_UNSUPPORTED; }
  return PR_OK;
}

uint32_t qcap_of(const pr_refine_params* p, uint32_t dflt) { return p->queue_cap > 0 ? (uint32_t)p->queue_cap : dflt; }
uint32_t scap_of(const pr_refine_params* p, uint32_t dflt) {
  const uint32_t total = p->survivor_cap > 0 ? (uint32_t)p->survivor_cap : dflt;
  return (total + kQueues - 1) / kQueues;
}
int budget_of(const pr_refine_params* p) {
  return p->trace_budget == 0 ? kBudget : (p->trace_budget < 0 ? 0 : p->trace_budget);
}

// Default capacities of the deferred-test and surviving-group queues: with a
// caller workspace, and with the library's static scratch buffer.
constexpr uint32_t kQcapDefault = 1u << 20, kScapDefault = 1u << 24;
constexpr uint32_t kQcapStatic = 1u << 18, kScapStatic = 1u << 21;

// Launches a kernel whose one argument is the RefineArgs.  The optional
// events take the dispatch's own start and end time stamps, so that timing
// puts no marker packets (and no idle gaps) into the stream.
template <typename K>
int launch_ra(K kernel, int blocks, hipStream_t s, RefineArgs& ra, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  void* args[] = {&ra};
  // the plain launch when no event rides on the dispatch (it is also the
  // form a stream capture records)
  if (!e0 && !e1)
    PR_HIP(hipLaunchKernel(reinterpret_cast<const void*>(kernel), dim3(blocks), dim3(kBlock), args, 0, s));
  else
    PR_HIP(hipExtLaunchKernel(reinterpret_cast<const void*>(kernel), dim3(blocks), dim3(kBlock), args, 0, s, e0, e1, 0));
  return PR_OK;
}

// Resident blocks per compute unit of kernel K, computed once per device
// (one cache per kernel instantiation).
template <auto K>
int blocks_per_cu(int dev) {
  static std::atomic<int> cache[64];
  if (dev < 0 || dev >= 64) return -1;
  int v = cache[dev].load(std::memory_order_relaxed);
  if (v > 0) return v;
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, K, kBlock, 0) != hipSuccess) return -1;
  v = per > 0 ? per : 1;
  cache[dev].store(v, std::memory_order_relaxed);
  return v;
}

int cu_count(int dev) {
  static std::atomic<int> cache[64];
  if (dev < 0 || dev >= 64) return -1;
  int v = cache[dev].load(std::memory_order_relaxed);
  if (v > 0) return v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) return -1;
  cache[dev].store(v, std::memory_order_relaxed);
  return v;
}

template <int W, int PREC>
int launch(RefineArgs& ra, const pr_refine_params* prm, hipStream_t s) {
  const int64_t P = ra.n_pairs;
  hipEvent_t eb = (hipEvent_t)prm->ev_begin, ee = (hipEvent_t)prm->ev_end;
  if (prm->persistent) {
    int dev = 0;
    PR_HIP(hipGetDevice(&dev));
    const int cus = cu_count(dev);
    // the automatic schedule with an all-zero table is the packet traversal
    const int sched = prm->schedule == 0 && ra.seg_table == 0u ? 1 : prm->schedule;
    const int per = sched == 1   ? blocks_per_cu<k_trace<W, PREC, 1>>(dev)
                    : sched == 2 ? blocks_per_cu<k_trace<W, PREC, 2>>(dev)
                                 : blocks_per_cu<k_trace<W, PREC, 0>>(dev);
    const int per_cull = blocks_per_cu<k_cull<W, PREC>>(dev);
    if (cus <= 0 || per <= 0 || per_cull <= 0) { set_error("device attribute query failed"); return PR_E_DEVICE; }
    const int blocks = prm->grid_blocks > 0 ? prm->grid_blocks : cus * per;
    // many units per wave: the cull takes them heaviest class first
    const int64_t cull_waves = (int64_t)cus * per_cull * kWaves;
    ra.ordered = 2 * P > kCullStatic * cull_waves ? 1 : 0;
    if (ra.ordered) {
      hipLaunchKernelGGL(k_order_count, dim3(grid_for(P, kBlock)), dim3(kBlock), 0, s, ra);
      hipLaunchKernelGGL(k_order_place, dim3(grid_for(P, kBlock)), dim3(kBlock), 0, s, ra);
    }
    int r = launch_ra(k_cull<W, PREC>, cus * per_cull, s, ra, eb, nullptr);
    hipEvent_t et = ra.budget > 0 ? nullptr : ee;
    if (r == PR_OK) {
      if (sched == 1) r = launch_ra(k_trace<W, PREC, 1>, blocks, s, ra, nullptr, et);
      else if (sched == 2) r = launch_ra(k_trace<W, PREC, 2>, blocks, s, ra, nullptr, et);
      else r = launch_ra(k_trace<W, PREC, 0>, blocks, s, ra, nullptr, et);
    }
    if (r == PR_OK && ra.budget > 0) r = launch_ra(k_trace2<W, PREC>, blocks, s, ra, nullptr, ee);
    if (r != PR_OK) return r;
  } else {
    const int blocks = prm->grid_blocks > 0 ? prm->grid_blocks : 64;
    if (eb) PR_HIP(hipEventRecord(eb, s));
    for (int64_t p = 0; p < P; ++p) hipLaunchKernelGGL((k_refine_pair<W, PREC>), dim3(blocks), dim3(kBlock), 0, s, ra, p);
    if (ee) PR_HIP(hipEventRecord(ee, s));
  }
  return PR_OK;
}

// Per-bucket wave-per-segment limits of the automatic schedule (one byte per
// target-size bucket, smallest targets in the low byte).  The built-in table
// is all zero: on the workloads measured here (pathology-shaped, batching,
// precision stress) the packet traversal beats wave-per-segment in every
// bucket, because a group's 64 Morton-ordered segments share most of their
// path and one node load serves them all.
uint32_t seg_table_of(const pr_refine_params* p) {
  if (p->schedule == 1) return 0u;
  if (p->schedule == 2) return 0xffffffffu;
  return p->seg_live_max;
}

// Workspace bytes of a refinement of P pairs with the given queue defaults.
int ws_needed(int64_t P, const pr_refine_params* params, uint32_t qdef, uint32_t sdef, size_t* bytes) {
  Carve cv{nullptr, 0};
  RefineArgs ra{};
  carve(cv, ra, P, qcap_of(params, qdef), scap_of(params, sdef), budget_of(params) > 0);
  *bytes = cv.used + 256;
  return PR_OK;
}

int refine_run(const void* blob_a, int64_t n_meshes_a, const void* blob_b, int64_t n_meshes_b,
               const int32_t* pairs, int64_t n_pairs, uint8_t* flags, const pr_refine_params* params,
               pr_refine_stats* dev_stats, int32_t* dev_status, void* ws, size_t ws_bytes, uint32_t qdef,
               uint32_t sdef, hipStream_t s) {
  RefineArgs ra{};
  Carve cv{(char*)ws, ws_bytes};
  const uint32_t qcap = qcap_of(params, qdef);
  const uint32_t scap = scap_of(params, sdef);
  const int budget = budget_of(params);
  carve(cv, ra, n_pairs, qcap, scap, budget > 0);
  if (cv.used > ws_bytes) { set_error("ws_bytes %zu < required %zu", ws_bytes, cv.used); return PR_E_CAPACITY; }
  int r = PR_OK;
  ra.blob_a = (const char*)blob_a;
  ra.blob_b = (const char*)blob_b;
  ra.n_meshes_a = n_meshes_a;
  ra.n_meshes_b = n_meshes_b;
  ra.pairs = pairs;
  ra.n_pairs = n_pairs;
  ra.np_dev = params->dev_n_pairs;
  ra.flags = flags;
  ra.qcap = qcap;
  ra.qsub = (qcap + kSlices - 1) / kSlices;
  ra.surv_cap = scap;
  ra.budget = budget;
  ra.share = params->trace_budget == 0 && budget == 0 ? 1 : 0;
  ra.lds_stack = params->lds_stack;
  ra.seg_table = seg_table_of(params);
  const int64_t init_items = n_pairs > kStatCopies * S_N ? n_pairs : kStatCopies * S_N;
  const int64_t init_blocks = grid_for(init_items, kBlock);
  hipLaunchKernelGGL(k_init, dim3((unsigned)(init_blocks < 1024 ? init_blocks : 1024)), dim3(kBlock), 0, s, ra);
  if (n_pairs > 0) {
    const int W = params->bvh_width, PREC = params->precision;
#define PR_LAUNCH(w, q) if (W == w && PREC == q) r = launch<w, q>(ra, params, s)
    PR_LAUNCH(2, 0); PR_LAUNCH(2, 1); PR_LAUNCH(2, 2); PR_LAUNCH(2, 3);
    PR_LAUNCH(4, 0); PR_LAUNCH(4, 1); PR_LAUNCH(4, 2); PR_LAUNCH(4, 3);
    PR_LAUNCH(8, 0); PR_LAUNCH(8, 1); PR_LAUNCH(8, 2); PR_LAUNCH(8, 3);
#undef PR_LAUNCH
    if (r) return r;
    const int fb = 256;  // enough threads for the deferred tests, blocks for the reruns
    if (W == 2) hipLaunchKernelGGL(k_fix<2>, dim3(fb), dim3(kBlock), 0, s, ra);
    else if (W == 4) hipLaunchKernelGGL(k_fix<4>, dim3(fb), dim3(kBlock), 0, s, ra);
    else hipLaunchKernelGGL(k_fix<8>, dim3(fb), dim3(kBlock), 0, s, ra);
    hipLaunchKernelGGL(k_finalize, dim3(grid_for(n_pairs, kBlock)), dim3(kBlock), 0, s, ra);
    hipLaunchKernelGGL(k_report, dim3(1), dim3(64), 0, s, ra, dev_stats, dev_status);
  } else {
    hipLaunchKernelGGL(k_report, dim3(1), dim3(64), 0, s, ra, dev_stats, dev_status);
  }
  PR_HIP(hipGetLastError());
  return PR_OK;
}

int check_refine_args(const void* blob_a, const void* blob_b, const int32_t* pairs, int64_t n_pairs,
                      const uint8_t* flags, int64_t n_meshes_a, int64_t n_meshes_b) {
  if (!blob_a || !blob_b || (n_pairs > 0 && (!pairs || !flags)) || n_meshes_a < 0 || n_meshes_b < 0) {
    set_error("null pointer or negative size");
    return PR_E_ARG;
  }
  return PR_OK;
}

// ---- allocation-free variant: the library's own static scratch buffer ----------

// Device scratch for refine_intersects_static: one copy per GPU, held until
// the process ends.  Host code never uses this name as an address; it uses
// the per-device address from hipGetSymbolAddress.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

// Address of this GPU's copy of `scratch`, looked up once per device with
// that device current (the caller's current device).
int static_scratch(void** out) {
  int dev = 0;
  PR_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) { set_error("device index %d beyond 63", dev); return PR_E_UNSUPPORTED; }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) { set_error("hipGetSymbolAddress(scratch) returned NULL"); return PR_E_DEVICE; }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PR_OK;
}

}  // namespace
}  // namespace pr

using namespace pr;

extern "C" int refine_workspace_bytes(int64_t n_pairs, const pr_refine_params* params, size_t* ws_bytes) {
  int r = check(n_pairs, params);
  if (r) return r;
  if (!ws_bytes) { set_error("ws_bytes is NULL"); return PR_E_ARG; }
  return ws_needed(n_pairs, params, kQcapDefault, kScapDefault, ws_bytes);
}

extern "C" int refine_intersects(const void* blob_a, int64_t n_meshes_a, const void* blob_b, int64_t n_meshes_b,
                                 const int32_t* pairs, int64_t n_pairs, uint8_t* flags,
                                 const pr_refine_params* params, pr_refine_stats* dev_stats, int32_t* dev_status,
                                 void* ws, size_t ws_bytes, void* stream) {
  int r = check(n_pairs, params);
  if (r) return r;
  r = check_refine_args(blob_a, blob_b, pairs, n_pairs, flags, n_meshes_a, n_meshes_b);
  if (r) return r;
  if (!ws) { set_error("ws is NULL"); return PR_E_ARG; }
  return refine_run(blob_a, n_meshes_a, blob_b, n_meshes_b, pairs, n_pairs, flags, params, dev_stats, dev_status, ws,
                    ws_bytes, kQcapDefault, kScapDefault, (hipStream_t)stream);
}

extern "C" size_t refine_static_scratch_bytes(void) { return kStaticScratchBytes; }

extern "C" int refine_intersects_static(const void* blob_a, int64_t n_meshes_a, const void* blob_b,
                                        int64_t n_meshes_b, const int32_t* pairs, int64_t n_pairs, uint8_t* flags,
                                        const pr_refine_params* params, pr_refine_stats* dev_stats,
                                        int32_t* dev_status, void* stream) {
  int r = check(n_pairs, params);
  if (r) return r;
  r = check_refine_args(blob_a, blob_b, pairs, n_pairs, flags, n_meshes_a, n_meshes_b);
  if (r) return r;
  size_t need = 0;
  r = ws_needed(n_pairs, params, kQcapStatic, kScapStatic, &need);
  if (r) return r;
  if (need > kStaticScratchBytes) {
    set_error("refine_intersects_static: %lld pairs with these queue capacities need %zu bytes of scratch; the "
              "static buffer holds %zu (use refine_intersects with a workspace)",
              (long long)n_pairs, need, kStaticScratchBytes);
    return PR_E_CAPACITY;
  }
  void* ws = nullptr;
  r = static_scratch(&ws);
  if (r) return r;
  return refine_run(blob_a, n_meshes_a, blob_b, n_meshes_b, pairs, n_pairs, flags, params, dev_stats, dev_status, ws,
                    kStaticScratchBytes, kQcapStatic, kScapStatic, (hipStream_t)stream);
}
