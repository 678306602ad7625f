// The paper's own dataset-level design (Sections 3.2 and 3.5), beside the
// per-pair refinement: one BVH over all triangles of the target dataset
// (a blob built from one mesh that holds every triangle), a
// triangle-to-object map, every unique source edge traced against that
// tree with all of its hits collected (the multi-hit loop: a traversal that
// does not stop at the first hit visits every leaf the segment's path
// reaches), and the (source object, target object) records materialised in
// one of the paper's ways:
//  * counting two-pass: a pass counts each source group's records, a scan
//    gives offsets, a second pass writes them, then sort + unique;
//  * single pass into a hashmap that drops duplicates on insert, sized by
//    the selectivity estimate (or a fixed capacity).
// The selectivity estimate (Section 3.5's grid statistics, interaction
// volume, shape factor and cap) runs here too.
//
// Work unit: one group of 64 segments (64 unique edges of one source mesh);
// a wave traces it with the packet traversal: the node loaded once for the
// wave, every active lane testing its segment against every child, a stack
// of (node, lane mask) entries in LDS.  Leaf tests are the closed
// segment-triangle test, FP32 filter with the exact fallback in place.  A
// lane drops a record equal to its previous one (consecutive hits of one
// target object).
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "scan.h"

#include <algorithm>
#include <climits>
#include <cmath>

#include "common.h"
#include "predicates.h"

namespace pr {
namespace {

constexpr int kDB = 256;                       // threads per block
constexpr int kDWaves = kDB / 64;
constexpr int kGrab = 8;                       // groups taken per grab
constexpr int kXcd = 8;
constexpr int kCtrWords = 512;                 // u64 words between counters
constexpr uint64_t kEmptyKey = ~0ull;
constexpr float kSlabKd = 1.0f + 0x1p-19f;
constexpr float kSlabSd = 0x1p-120f;
constexpr float kZeroInvD = 0x1p100f;
constexpr float kZeroBiasD = 0x1p16f;

enum { D_GROUPS = 0, D_VISITS, D_TESTS, D_HITS, D_RECORDS, D_EXACT, D_OVER, D_NEW, D_N };
static_assert(sizeof(pr_dataset_stats) == D_N * 8, "stats layout");

struct DBlob {
  const MeshDesc* mesh;
  const char* nodes;
  const float* tris;
  const float* seg;
  const float* cbox;
  const int32_t* cmesh;
  int64_t n_meshes, n_chunks;
  int32_t width;
  uint32_t magic;
};

__device__ __forceinline__ DBlob dview(const char* b) {
  const BlobHeader* h = reinterpret_cast<const BlobHeader*>(b);
  DBlob v;
  v.mesh = reinterpret_cast<const MeshDesc*>(b + h->off_mesh);
  v.nodes = b + h->off_node;
  v.tris = reinterpret_cast<const float*>(b + h->off_tri);
  v.seg = reinterpret_cast<const float*>(b + h->off_seg);
  v.cbox = reinterpret_cast<const float*>(b + h->off_cbox);
  v.cmesh = reinterpret_cast<const int32_t*>(b + h->off_cmesh);
  v.n_meshes = h->n_meshes;
  v.n_chunks = h->n_chunks;
  v.width = h->width;
  v.magic = h->magic;
  return v;
}

// Conservative closed segment-box test, the same form as the refinement's:
// t = fl(fl(plane - p) * fl(1 / d)) -+ bias with a relative error below
// gamma_4; accept when t_min <= t_max (1 + 2^-19) + 2^-120; a zero direction
// component gets a large reciprocal and a bias that turn its slab into "no
// constraint" or "empty" exactly.  Every box is accepted for meshes outside
// the FP32-safe range (their leaf tests are all exact).
struct DRay {
  float px, py, pz, ix, iy, iz, bx, by, bz;
};

__device__ __forceinline__ void daxis(float d, bool safe, float& inv, float& bias) {
  if (!safe) { inv = 0.f; bias = INFINITY; return; }
  if (d != 0.f) { inv = 1.0f / d; bias = 0.f; }
  else { inv = kZeroInvD; bias = kZeroBiasD; }
}

__device__ __forceinline__ bool dslab(const DRay& r, float lx, float ly, float lz, float hx, float hy, float hz) {
  float t0x = fmaf(lx - r.px, r.ix, -r.bx), t1x = fmaf(hx - r.px, r.ix, r.bx);
  float t0y = fmaf(ly - r.py, r.iy, -r.by), t1y = fmaf(hy - r.py, r.iy, r.by);
  float t0z = fmaf(lz - r.pz, r.iz, -r.bz), t1z = fmaf(hz - r.pz, r.iz, r.bz);
  float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.f));
  float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), 1.f));
  return tn <= fmaf(tf, kSlabKd, kSlabSd);
}

__device__ __forceinline__ uint64_t mix64(uint64_t x) {  // splitmix64 finaliser
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}

struct TraceArgs {
  const char* src;            // per-mesh blob of the source dataset (its edges)
  const char* dst;            // dataset-level blob of the target dataset (one mesh)
  const int32_t* tri_obj;     // target: object of each leaf-order triangle
  int64_t n_src_objects, n_dst_objects;
  int32_t op, flip;
  uint64_t* counts;           // [groups] op 0 out / op 1 in
  const uint64_t* offsets;    // [groups] op 1
  uint64_t* keys;
  int64_t key_cap;
  int64_t max_groups;         // entries of counts / offsets
  unsigned long long* grab;   // kXcd grab counters, kCtrWords apart
  unsigned long long* stats;  // D_N counters
  int32_t* status;
  uint32_t* xlist;            // [max_groups] groups for the exact pass
  uint32_t* xcount;           // [1]
};

// Leaf triangle test of one lane's segment: 1 hit, 0 miss, -1 when the FP32
// bound cannot decide and EXACT is off (the group is then traced again by the
// exact kernel); with EXACT, the FP64 filter and exact expansions decide.
template <bool EXACT>
__device__ __forceinline__ int dleaf(f3 p, f3 q, f3 a, f3 b, f3 c, bool safe, uint32_t& exact) {
  const int r = safe ? seg_tri_f32(p, q, a, b, c) : kAmbig;
  if (r != kAmbig) return r == kHit ? 1 : 0;
  if (!EXACT) return -1;
  ++exact;
  ExactCounters ec{0};
  return seg_tri_exact(p, q, a, b, c, ec) ? 1 : 0;
}

template <int W>
constexpr int dstack_cap() { return (W - 1) * (kMaxDepth + 1) + 1; }

// Traces group g and emits its records for op 0 (count), 1 (write at the
// group's offset) or 2 (hash insert).  Returns false when a test needs the
// exact tier and EXACT is off: the group is then appended to the exact list
// and traced again, whole, by the exact kernel (which rewrites its count,
// rewrites its records at the same offsets, or inserts them again).
template <int W, int OP, bool EXACT>
__device__ bool trace_group_ds(const TraceArgs& a, const DBlob& S, const DBlob& T, int64_t g, int32_t* s_ref,
                               uint64_t* s_mask, uint32_t (&cnt)[D_N]) {
  const int lane = threadIdx.x & 63;
  const int32_t sm = S.cmesh[g];
  const MeshDesc smd = S.mesh[sm];
  const int32_t live = min((int32_t)kChunk, smd.n_edges - (int32_t)(g - smd.chunk_base) * kChunk);
  const MeshDesc tmd = T.mesh[0];
  const bool safe = (smd.flags & tmd.flags & kMeshSafe) != 0;
  const float* sp = S.seg + g * (6 * kChunk);
  const f3 p{sp[lane], sp[kChunk + lane], sp[2 * kChunk + lane]};
  const f3 q{sp[3 * kChunk + lane], sp[4 * kChunk + lane], sp[5 * kChunk + lane]};
  DRay r;
  r.px = p.x; r.py = p.y; r.pz = p.z;
  daxis(q.x - p.x, safe, r.ix, r.bx);
  daxis(q.y - p.y, safe, r.iy, r.by);
  daxis(q.z - p.z, safe, r.iz, r.bz);
  cnt[D_GROUPS] += lane == 0 ? 1u : 0u;
  const bool valid = lane < live;
  uint64_t m0 = __ballot(valid && tmd.root != kEmpty &&
                         dslab(r, tmd.box[0], tmd.box[1], tmd.box[2], tmd.box[3], tmd.box[4], tmd.box[5]) &&
                         (safe || (fminf(p.x, q.x) <= tmd.box[3] && fmaxf(p.x, q.x) >= tmd.box[0] &&
                                   fminf(p.y, q.y) <= tmd.box[4] && fmaxf(p.y, q.y) >= tmd.box[1] &&
                                   fminf(p.z, q.z) <= tmd.box[5] && fmaxf(p.z, q.z) >= tmd.box[2])));
  int32_t last = -1;         // per lane: target object of its previous record
  uint32_t mine = 0;         // per lane: records (op 0)
  uint64_t wrote = 0;        // op 1: records of the group written so far (uniform)
  uint64_t obase = 0, oend = 0;
  if (OP == 1) {
    obase = a.offsets[g];
    oend = obase + a.counts[g];
  }
  const int64_t src_obj = sm;
  auto record = [&](bool hit, int32_t tobj) {
    const bool emit = hit && tobj != last;
    if (hit) last = tobj;
    if (OP == 0) {
      mine += emit ? 1u : 0u;
      return;
    }
    const uint64_t key = a.flip ? ((uint64_t)(uint32_t)tobj << 32) | (uint32_t)src_obj
                                : ((uint64_t)(uint32_t)src_obj << 32) | (uint32_t)tobj;
    if (OP == 1) {
      const uint64_t em = __ballot(emit);
      if (!em) return;
      const uint64_t pos = obase + wrote + (uint64_t)__builtin_amdgcn_mbcnt_hi(
                               (uint32_t)(em >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)em, 0u));
      if (emit) {
        if (pos < oend && pos < (uint64_t)a.key_cap) a.keys[pos] = key;
        else ++cnt[D_OVER];
      }
      wrote += (uint64_t)__popcll(em);
      return;
    }
    // OP == 2: open addressing, linear probing
    cnt[D_RECORDS] += emit ? 1u : 0u;
    if (emit) {
      const uint64_t capm = (uint64_t)a.key_cap - 1;
      uint64_t h = mix64(key) & capm;
      bool done = false;
      for (int64_t probe = 0; probe < a.key_cap; ++probe) {
        const uint64_t prev = atomicCAS(reinterpret_cast<unsigned long long*>(a.keys + h), kEmptyKey, key);
        if (prev == kEmptyKey) { ++cnt[D_NEW]; done = true; break; }
        if (prev == key) { done = true; break; }
        h = (h + 1) & capm;
      }
      if (!done) ++cnt[D_OVER];
    }
  };
  if (m0) {
    const Node<W>* nodes = reinterpret_cast<const Node<W>*>(T.nodes);
    int top = 0;
    if (lane == 0) { s_ref[0] = tmd.root; s_mask[0] = m0; }
    top = 1;
    while (top > 0) {
      --top;
      // lane 0 wrote the entry: make it visible to the whole wave
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int32_t ref = __builtin_amdgcn_readfirstlane(s_ref[top]);
      const uint64_t nm = s_mask[top];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const bool on = (nm >> lane) & 1ull;
      if (ref < 0) {
        const int32_t lr = ~ref;
        const int32_t first = lr >> 3, cnt_t = (lr & 7) + 1;
        for (int t = 0; t < cnt_t; ++t) {
          const float* tp = T.tris + 9 * (int64_t)(first + t);
          const f3 ta{tp[0], tp[1], tp[2]}, tb{tp[3], tp[4], tp[5]}, tc{tp[6], tp[7], tp[8]};
          uint32_t ex = 0;
          const int res = on ? dleaf<EXACT>(p, q, ta, tb, tc, safe, ex) : 0;
          if (!EXACT && __ballot(res < 0)) return false;
          const bool hit = res > 0;
          cnt[D_EXACT] += ex;
          cnt[D_TESTS] += on ? 1u : 0u;
          cnt[D_HITS] += hit ? 1u : 0u;
          int32_t tobj = 0;
          if (__ballot(hit)) tobj = a.tri_obj[first + t];
          record(hit, tobj);
        }
        continue;
      }
      cnt[D_VISITS] += lane == 0 ? 1u : 0u;
      const Node<W>* n = nodes + ref;
      uint64_t hm[W];
#pragma unroll
      for (int c = 0; c < W; ++c) {
        const int32_t ch = n->child[c];
        hm[c] = 0;
        if (ch == kEmpty) continue;
        const float lx = n->lo[0][c], ly = n->lo[1][c], lz = n->lo[2][c];
        const float hx = n->hi[0][c], hy = n->hi[1][c], hz = n->hi[2][c];
        bool hit = on && dslab(r, lx, ly, lz, hx, hy, hz);
        if (!safe)
          hit = hit && fminf(p.x, q.x) <= hx && fmaxf(p.x, q.x) >= lx && fminf(p.y, q.y) <= hy &&
                fmaxf(p.y, q.y) >= ly && fminf(p.z, q.z) <= hz && fmaxf(p.z, q.z) >= lz;
        hm[c] = __ballot(hit);
      }
#pragma unroll
      for (int c = W - 1; c >= 0; --c) {
        if (!hm[c]) continue;
        if (top >= dstack_cap<W>()) {  // not for a valid blob (depth <= kMaxDepth)
          if (lane == 0) atomicMin(a.status, (int32_t)PR_E_UNSUPPORTED);
          return true;
        }
        if (lane == 0) { s_ref[top] = n->child[c]; s_mask[top] = hm[c]; }
        ++top;
      }
    }
  }
  if (OP == 0) {
    uint32_t s = mine;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) a.counts[g] = s;
    cnt[D_RECORDS] += lane == 0 ? s : 0u;
  } else if (OP == 1) {
    cnt[D_RECORDS] += lane == 0 ? (uint32_t)wrote : 0u;
  }
  return true;
}

__device__ __forceinline__ void flush_counts(const TraceArgs& a, const uint32_t (&cnt)[D_N]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < D_N; ++k) {
    uint32_t s = cnt[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0 && s) atomicAdd(a.stats + k, (unsigned long long)s);
  }
}

__device__ __forceinline__ bool dblobs_ok(const TraceArgs& a, const DBlob& S, const DBlob& T, int W) {
  return S.magic == kMagic && T.magic == kMagic && T.n_meshes == 1 && T.width == W &&
         a.n_src_objects <= S.n_meshes && S.n_chunks <= a.max_groups;
}

// Persistent waves over the source groups: one contiguous share per XCD
// (blocks are dealt to the XCDs round-robin), taken kGrab groups at a time.
template <int W, int OP>
__global__ __launch_bounds__(kDB) void k_dtrace(TraceArgs a) {
  __shared__ int32_t s_ref[kDWaves][dstack_cap<W>()];
  __shared__ uint64_t s_mask[kDWaves][dstack_cap<W>()];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const DBlob S = dview(a.src), T = dview(a.dst);
  uint32_t cnt[D_N] = {};
  if (!dblobs_ok(a, S, T, W)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicMin(a.status, (int32_t)PR_E_UNSUPPORTED);
    return;
  }
  const int64_t G = S.n_chunks;
  const int xs = (int)(blockIdx.x % kXcd);
  const int64_t lo = G * xs / kXcd, hi = G * (xs + 1) / kXcd;
  unsigned long long* ctr = a.grab + kCtrWords * xs;
  while (true) {
    unsigned long long b = 0;
    if (lane == 0) b = atomicAdd(ctr, (unsigned long long)kGrab);
    const int64_t g0 = lo + (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)b);
    if (g0 >= hi) break;
    const int64_t g1 = g0 + kGrab < hi ? g0 + kGrab : hi;
    for (int64_t g = g0; g < g1; ++g)
      if (!trace_group_ds<W, OP, false>(a, S, T, g, s_ref[wv], s_mask[wv], cnt)) {
        if (lane == 0) a.xlist[atomicAdd(a.xcount, 1u)] = (uint32_t)g;  // at most one entry per group
      }
  }
  flush_counts(a, cnt);
}

// The groups that met a test the FP32 bound could not decide, traced again
// with the exact tier (one wave per group).
template <int W, int OP>
__global__ __launch_bounds__(kDB) void k_dtrace_exact(TraceArgs a) {
  __shared__ int32_t s_ref[kDWaves][dstack_cap<W>()];
  __shared__ uint64_t s_mask[kDWaves][dstack_cap<W>()];
  const int wv = threadIdx.x >> 6;
  const DBlob S = dview(a.src), T = dview(a.dst);
  uint32_t cnt[D_N] = {};
  if (!dblobs_ok(a, S, T, W)) return;
  const uint32_t n = *a.xcount;
  for (uint32_t k = blockIdx.x * kDWaves + wv; k < n; k += gridDim.x * kDWaves)
    trace_group_ds<W, OP, true>(a, S, T, a.xlist[k], s_ref[wv], s_mask[wv], cnt);
  flush_counts(a, cnt);
}

__global__ void k_dclear(uint64_t* keys, int64_t n, uint64_t* counts, int64_t n_counts, unsigned long long* grab,
                         unsigned long long* stats, int32_t* status, uint64_t* dev_n, int zero_n,
                         uint32_t* xcount = nullptr) {
  const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t i = i0; i < n; i += (int64_t)gridDim.x * blockDim.x) keys[i] = kEmptyKey;
  for (int64_t i = i0; i < n_counts; i += (int64_t)gridDim.x * blockDim.x) counts[i] = 0ull;
  if (grab && i0 < kXcd) grab[kCtrWords * i0] = 0ull;
  if (stats && i0 < D_N) stats[i0] = 0ull;
  if (i0 == 0) {
    *status = PR_OK;
    if (zero_n && dev_n) *dev_n = 0ull;
    if (xcount) *xcount = 0u;
  }
}

__global__ void k_dreport(const unsigned long long* stats, const int32_t* status, const uint64_t* offsets,
                          int64_t groups, pr_dataset_stats* out, int32_t* dev_status, uint64_t* dev_n, int op) {
  const int t = threadIdx.x;
  if (t < D_N && out) reinterpret_cast<uint64_t*>(out)[t] = stats[t];
  if (t == 0) {
    if (dev_status) *dev_status = *status;
    if (dev_n) {
      if (op == 0) *dev_n = offsets[groups];
      else if (op == 2) *dev_n = stats[D_NEW];
    }
  }
}

// ---- triangle -> object --------------------------------------------------

__global__ void k_tri_obj(const char* blob, const int64_t* face_off, int64_t n_obj, int32_t* tri_obj,
                          int64_t f_cap, int32_t* status) {
  const BlobHeader* h = reinterpret_cast<const BlobHeader*>(blob);
  const int32_t* triid = reinterpret_cast<const int32_t*>(blob + h->off_triid);
  if (h->magic != kMagic || h->n_meshes != 1 || h->f_total != f_cap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicMin(status, (int32_t)PR_E_UNSUPPORTED);
    return;
  }
  const int64_t F = f_cap;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < F; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t f = triid[k];
    // last object o with face_off[o] <= f
    int64_t lo = 0, hi = n_obj;  // face_off[lo] <= f < face_off[hi]
    if (f < face_off[0] || f >= face_off[n_obj]) {
      atomicMin(status, (int32_t)PR_E_ARG);
      tri_obj[k] = -1;
      continue;
    }
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (face_off[mid] <= f) lo = mid; else hi = mid;
    }
    tri_obj[k] = (int32_t)lo;
  }
}

// ---- selectivity estimate ------------------------------------------------

constexpr double kEstEps = 1e-3;
constexpr double kEstGamma = 0.8;

struct EstArgs {
  const char* blob[2];
  int64_t n[2];
  int32_t cells;
  double* side[2];    // [n] mean box side
  double* ratio[2];   // [n] volume ratio
  double* ext;        // [6] union box lo xyz, hi xyz (as ordered ints for the reduction)
  double* grid;       // [2][3][cells^3]: count, sum of sides, sum of ratios
  double* out;
};

__device__ __forceinline__ void amin_d(double* p, double v) {
  unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
  unsigned long long old = *q;
  while (__longlong_as_double((long long)old) > v) {
    const unsigned long long prev = atomicCAS(q, old, (unsigned long long)__double_as_longlong(v));
    if (prev == old) break;
    old = prev;
  }
}
__device__ __forceinline__ void amax_d(double* p, double v) {
  unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
  unsigned long long old = *q;
  while (__longlong_as_double((long long)old) < v) {
    const unsigned long long prev = atomicCAS(q, old, (unsigned long long)__double_as_longlong(v));
    if (prev == old) break;
    old = prev;
  }
}

__global__ void k_est_init(EstArgs e, int64_t grid_words) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < grid_words;
       i += (int64_t)gridDim.x * blockDim.x)
    e.grid[i] = 0.0;
  if (blockIdx.x == 0 && threadIdx.x < 6) e.ext[threadIdx.x] = threadIdx.x < 3 ? INFINITY : -INFINITY;
  if (blockIdx.x == 0 && threadIdx.x == 0) *e.out = 0.0;
}

// One block per mesh: volume by the divergence theorem over its triangles
// (FP64), mean box side and volume ratio; the union box.  (The host checks
// nothing on the device blobs: a count above the blob's is cut to it.)
__global__ void k_est_objects(EstArgs e, int d) {
  __shared__ double s_red[kDB / 64];
  const BlobHeader* h = reinterpret_cast<const BlobHeader*>(e.blob[d]);
  if (h->magic != kMagic) return;
  const int64_t nm = e.n[d] < h->n_meshes ? e.n[d] : h->n_meshes;
  const MeshDesc* md = reinterpret_cast<const MeshDesc*>(e.blob[d] + h->off_mesh);
  const float* tris = reinterpret_cast<const float*>(e.blob[d] + h->off_tri);
  for (int64_t m = blockIdx.x; m < nm; m += gridDim.x) {
    const MeshDesc D = md[m];
    double acc = 0.0;
    for (int32_t t = threadIdx.x; t < D.n_tris; t += blockDim.x) {
      const float* p = tris + 9 * ((int64_t)D.tri_base + t);
      const double ax = p[0], ay = p[1], az = p[2], bx = p[3], by = p[4], bz = p[5];
      const double cx = p[6], cy = p[7], cz = p[8];
      acc += ax * (by * cz - bz * cy) + ay * (bz * cx - bx * cz) + az * (bx * cy - by * cx);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double v = 0.0;
      for (int k = 0; k < kDB / 64; ++k) v += s_red[k];
      v = fabs(v / 6.0);
      if (D.n_tris > 0) {
        const double ex = (double)D.box[3] - D.box[0], ey = (double)D.box[4] - D.box[1],
                     ez = (double)D.box[5] - D.box[2];
        e.side[d][m] = (ex + ey + ez) / 3.0;
        const double bv = ex * ey * ez;
        e.ratio[d][m] = bv > 0.0 ? fmin(fmax(v / bv, 0.0), 1.0) : 1.0;
        for (int k = 0; k < 3; ++k) {
          amin_d(e.ext + k, (double)D.box[k]);
          amax_d(e.ext + 3 + k, (double)D.box[3 + k]);
        }
      } else {
        e.side[d][m] = 0.0;
        e.ratio[d][m] = 0.0;
      }
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void grid_frame(const EstArgs& e, double* lo, double* size) {
  for (int k = 0; k < 3; ++k) {
    lo[k] = e.ext[k];
    const double hi = e.ext[3 + k];
    size[k] = hi > lo[k] ? (hi - lo[k]) / e.cells : 1.0;
  }
}

// One thread per object: adds it to every cell its closed box touches.
__global__ void k_est_cells(EstArgs e, int d) {
  const BlobHeader* h = reinterpret_cast<const BlobHeader*>(e.blob[d]);
  if (h->magic != kMagic) return;
  const int64_t nm = e.n[d] < h->n_meshes ? e.n[d] : h->n_meshes;
  const MeshDesc* md = reinterpret_cast<const MeshDesc*>(e.blob[d] + h->off_mesh);
  double lo[3], size[3];
  grid_frame(e, lo, size);
  const int G = e.cells;
  const int64_t C = (int64_t)G * G * G;
  double* cnt = e.grid + (int64_t)d * 3 * C;
  double* sid = cnt + C;
  double* rat = sid + C;
  for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < nm; m += (int64_t)gridDim.x * blockDim.x) {
    const MeshDesc D = md[m];
    if (D.n_tris <= 0) continue;
    int c0[3], c1[3];
    for (int k = 0; k < 3; ++k) {
      double a = ceil(((double)D.box[k] - lo[k]) / size[k] - 1.0);
      double b = floor(((double)D.box[3 + k] - lo[k]) / size[k]);
      a = fmin(fmax(a, 0.0), (double)(G - 1));
      b = fmin(fmax(b, 0.0), (double)(G - 1));
      c0[k] = (int)a;
      c1[k] = (int)b;
    }
    const double s = e.side[d][m], r = e.ratio[d][m];
    for (int x = c0[0]; x <= c1[0]; ++x)
      for (int y = c0[1]; y <= c1[1]; ++y)
        for (int z = c0[2]; z <= c1[2]; ++z) {
          const int64_t c = ((int64_t)x * G + y) * G + z;
          atomicAdd(cnt + c, 1.0);
          atomicAdd(sid + c, s);
          atomicAdd(rat + c, r);
        }
  }
}

__global__ void k_est_sum(EstArgs e) {
  __shared__ double s_red[kDB / 64];
  double lo[3], size[3];
  grid_frame(e, lo, size);
  const double vcell = size[0] * size[1] * size[2];
  const int64_t C = (int64_t)e.cells * e.cells * e.cells;
  const double* n1 = e.grid;
  const double* s1 = n1 + C;
  const double* r1 = s1 + C;
  const double* n2 = e.grid + 3 * C;
  const double* s2 = n2 + C;
  const double* r2 = s2 + C;
  double acc = 0.0;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < C; c += (int64_t)gridDim.x * blockDim.x) {
    if (n1[c] > 0.0 && n2[c] > 0.0) {
      const double S1 = s1[c] / n1[c], S2 = s2[c] / n2[c];
      const double R1 = r1[c] / n1[c], R2 = r2[c] / n2[c];
      const double w = S1 + S2 + kEstEps;
      const double pb = w * w * w / vcell;
      const double fs = pow(sqrt(R1 * R2), kEstGamma);
      acc += n1[c] * n2[c] * fmin(pb * fs, 1.0);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = 0.0;
    for (int k = 0; k < kDB / 64; ++k) v += s_red[k];
    atomicAdd(e.out, v);
  }
}

// ---- sort + unique ---------------------------------------------------------

__global__ void k_unique_flags(const uint64_t* keys, int64_t n, uint32_t* flags) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    flags[i] = (keys[i] != kEmptyKey && (i == 0 || keys[i] != keys[i - 1])) ? 1u : 0u;
}

__global__ void k_unique_write(const uint64_t* keys, int64_t n, const uint32_t* flags, const uint64_t* pos,
                               int32_t* out, int64_t cap, int64_t* count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (flags[i] && (int64_t)pos[i] < cap) {
      out[2 * pos[i]] = (int32_t)(keys[i] >> 32);
      out[2 * pos[i] + 1] = (int32_t)(uint32_t)keys[i];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *count = n > 0 ? (int64_t)(pos[n - 1] + flags[n - 1]) : 0;
}

template <typename T>
T* take(char*& p, size_t& left, int64_t n) {
  const size_t need = (size_t)align256((int64_t)(sizeof(T) * (size_t)(n > 0 ? n : 1)));
  if (need > left) return nullptr;
  T* r = reinterpret_cast<T*>(p);
  p += need;
  left -= need;
  return r;
}

int unique_ws(int64_t n, size_t* bytes) {
  size_t sort_tmp = 0;
  const hipError_t e =
      hipcub::DeviceRadixSort::SortKeys(nullptr, sort_tmp, (const uint64_t*)nullptr, (uint64_t*)nullptr, (int)n, 0, 64);
  if (e != hipSuccess) return hip_fail(e, "hipcub SortKeys size");
  const size_t scan_tmp = (size_t)(8 * (scan_tiles_of(n) + 1));
  *bytes = (size_t)align256(8 * n) + (size_t)align256(4 * n) + (size_t)align256(8 * n) +
           (size_t)align256((int64_t)std::max(sort_tmp, scan_tmp)) + 1024;
  return PR_OK;
}

size_t trace_ws(int64_t groups) {
  const size_t scan_tmp = (size_t)(8 * (scan_tiles_of(groups + 1) + 1));
  return (size_t)align256(8 * (groups + 1)) + (size_t)align256(8 * kXcd * kCtrWords) + (size_t)align256(8 * D_N) +
         256 + 256 + (size_t)align256(4 * (groups > 0 ? groups : 1)) + (size_t)align256((int64_t)scan_tmp) + 1024;
}

size_t est_ws(int64_t na, int64_t nb, int32_t cells) {
  const int64_t C = (int64_t)cells * cells * cells;
  return (size_t)align256(16 * (na > 0 ? na : 1)) + (size_t)align256(16 * (nb > 0 ? nb : 1)) + 256 +
         (size_t)align256(8 * 6 * C) + 1024;
}

}  // namespace
}  // namespace pr

using namespace pr;

extern "C" int dataset_tri_objects(const void* dblob, const int64_t* face_off, int64_t n_objects, int32_t* tri_obj,
                                   int64_t f_total, int32_t* dev_status, void* stream) {
  if (!dblob || !face_off || !tri_obj || !dev_status || n_objects <= 0 || f_total < 0) {
    set_error("null pointer or bad size");
    return PR_E_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_dclear, dim3(1), dim3(64), 0, s, (uint64_t*)nullptr, (int64_t)0, (uint64_t*)nullptr,
                     (int64_t)0, (unsigned long long*)nullptr, (unsigned long long*)nullptr, dev_status,
                     (uint64_t*)nullptr, 0);
  hipLaunchKernelGGL(k_tri_obj, dim3(grid_for(f_total, 256)), dim3(256), 0, s, (const char*)dblob, face_off,
                     n_objects, tri_obj, f_total, dev_status);
  PR_HIP(hipGetLastError());
  return PR_OK;
}

extern "C" int dataset_trace_ws_bytes(int64_t max_groups, size_t* ws_bytes) {
  if (max_groups < 0 || !ws_bytes) { set_error("bad argument"); return PR_E_ARG; }
  if (max_groups >= INT_MAX) { set_error("too many groups"); return PR_E_UNSUPPORTED; }
  *ws_bytes = trace_ws(max_groups);
  return PR_OK;
}

extern "C" int dataset_trace(const void* src_blob, int64_t n_src_objects, const void* dst_blob,
                             const int32_t* tri_obj, int64_t n_dst_objects, const pr_dataset_params* params,
                             uint64_t* counts, int64_t max_groups, uint64_t* keys, uint64_t* dev_n,
                             pr_dataset_stats* dev_stats, int32_t* dev_status, void* ws, size_t ws_bytes,
                             void* stream) {
  if (!src_blob || !dst_blob || !params || !dev_status || !ws || n_src_objects < 0 || n_dst_objects < 0 ||
      max_groups < 0) {
    set_error("null pointer or negative size");
    return PR_E_ARG;
  }
  const int op = params->op;
  if (op < 0 || op > 3 || (params->flip != 0 && params->flip != 1) || params->width < 2 || params->width > 8 ||
      (params->width & (params->width - 1))) {
    set_error("bad params (op %d, flip %d, width %d)", op, params->flip, params->width);
    return PR_E_ARG;
  }
  if ((op == 0 || op == 1) && !counts) { set_error("counts is NULL"); return PR_E_ARG; }
  if (op != 0 && (!keys || params->key_cap <= 0)) { set_error("keys / key_cap"); return PR_E_ARG; }
  if (op == 2 && (params->key_cap & (params->key_cap - 1))) { set_error("key_cap must be a power of two"); return PR_E_ARG; }
  if (op != 3 && !tri_obj) { set_error("tri_obj is NULL"); return PR_E_ARG; }
  if (max_groups >= INT_MAX) { set_error("too many groups"); return PR_E_UNSUPPORTED; }
  if (ws_bytes < trace_ws(max_groups)) { set_error("ws_bytes %zu < required %zu", ws_bytes, trace_ws(max_groups)); return PR_E_CAPACITY; }
  hipStream_t s = (hipStream_t)stream;
  char* p = (char*)ws;
  size_t left = ws_bytes;
  uint64_t* offsets = take<uint64_t>(p, left, max_groups + 1);
  unsigned long long* grab = take<unsigned long long>(p, left, kXcd * kCtrWords);
  unsigned long long* stats = take<unsigned long long>(p, left, D_N);
  int32_t* status = take<int32_t>(p, left, 64);
  uint32_t* xcount = take<uint32_t>(p, left, 64);
  uint32_t* xlist = take<uint32_t>(p, left, max_groups);
  void* scan_tmp = p;
  TraceArgs a{};
  a.src = (const char*)src_blob;
  a.dst = (const char*)dst_blob;
  a.tri_obj = tri_obj;
  a.n_src_objects = n_src_objects;
  a.n_dst_objects = n_dst_objects;
  a.op = op;
  a.flip = params->flip;
  a.counts = counts;
  a.offsets = offsets;
  a.keys = keys;
  a.key_cap = params->key_cap;
  a.max_groups = max_groups;
  a.grab = grab;
  a.stats = stats;
  a.status = status;
  a.xlist = xlist;
  a.xcount = xcount;
  // op 3 clears the table (and the key count), op 0 the per-group counts
  // (every one of max_groups + 1 entries: the scan reads them all); every op
  // clears the grab counters, statistics and status
  const int64_t nclear = op == 3 ? params->key_cap : 0;
  const int64_t ncounts = op == 0 ? max_groups + 1 : 0;
  const int64_t nmax = std::max<int64_t>(std::max<int64_t>(nclear, ncounts), 64);
  hipLaunchKernelGGL(k_dclear, dim3(grid_for(nmax, 256)), dim3(256), 0, s, keys, nclear, counts, ncounts, grab,
                     stats, status, dev_n, op == 3 ? 1 : 0, xcount);
  if (op == 3) {
    hipLaunchKernelGGL(k_dreport, dim3(1), dim3(64), 0, s, (const unsigned long long*)stats, (const int32_t*)status,
                       (const uint64_t*)offsets, (int64_t)0, dev_stats, dev_status, (uint64_t*)nullptr, op);
    PR_HIP(hipGetLastError());
    return PR_OK;
  }
  if (op == 1) {
    PR_HIP(device_exclusive_scan((const uint64_t*)counts, offsets, max_groups, (int64_t*)scan_tmp, (int64_t*)nullptr, s));
  }
  int dev = 0;
  PR_HIP(hipGetDevice(&dev));
  int cus = 0;
  PR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int blocks = cus * 4;
  const int W = params->width;
#define PR_DT(w, o)                                                                     \
  if (W == w && op == o) {                                                              \
    hipLaunchKernelGGL((k_dtrace<w, o>), dim3(blocks), dim3(kDB), 0, s, a);             \
    hipLaunchKernelGGL((k_dtrace_exact<w, o>), dim3(256), dim3(kDB), 0, s, a);          \
  }
  PR_DT(2, 0); PR_DT(2, 1); PR_DT(2, 2);
  PR_DT(4, 0); PR_DT(4, 1); PR_DT(4, 2);
  PR_DT(8, 0); PR_DT(8, 1); PR_DT(8, 2);
#undef PR_DT
  if (op == 0) {
    // offsets of every group and, at [max_groups], the total
    PR_HIP(device_exclusive_scan((const uint64_t*)counts, offsets, max_groups + 1, (int64_t*)scan_tmp, (int64_t*)nullptr, s));
  }
  hipLaunchKernelGGL(k_dreport, dim3(1), dim3(64), 0, s, (const unsigned long long*)stats, (const int32_t*)status,
                     (const uint64_t*)offsets, max_groups, dev_stats, dev_status, dev_n, op);
  PR_HIP(hipGetLastError());
  return PR_OK;
}

extern "C" int pairs_unique_ws_bytes(int64_t n_keys, size_t* ws_bytes) {
  if (n_keys < 0 || !ws_bytes) { set_error("bad argument"); return PR_E_ARG; }
  if (n_keys >= INT_MAX) { set_error("n_keys %lld beyond 2^31", (long long)n_keys); return PR_E_UNSUPPORTED; }
  return unique_ws(n_keys, ws_bytes);
}

extern "C" int pairs_unique(const uint64_t* keys, int64_t n_keys, int32_t* out_pairs, int64_t out_cap,
                            int64_t* dev_count, void* ws, size_t ws_bytes, void* stream) {
  if (n_keys < 0 || out_cap < 0 || !dev_count || !ws || (n_keys > 0 && !keys) || (out_cap > 0 && !out_pairs)) {
    set_error("null pointer or negative size");
    return PR_E_ARG;
  }
  if (n_keys >= INT_MAX) { set_error("n_keys beyond 2^31"); return PR_E_UNSUPPORTED; }
  size_t need = 0;
  const int r = unique_ws(n_keys, &need);
  if (r != PR_OK) return r;
  if (ws_bytes < need) { set_error("ws_bytes %zu < required %zu", ws_bytes, need); return PR_E_CAPACITY; }
  hipStream_t s = (hipStream_t)stream;
  char* p = (char*)ws;
  size_t left = ws_bytes;
  uint64_t* sorted = take<uint64_t>(p, left, n_keys);
  uint32_t* flags = take<uint32_t>(p, left, n_keys);
  uint64_t* pos = take<uint64_t>(p, left, n_keys);
  void* tmp = p;
  size_t tmp_bytes = left;
  if (n_keys == 0) {
    hipLaunchKernelGGL(k_unique_write, dim3(1), dim3(64), 0, s, (const uint64_t*)sorted, (int64_t)0,
                       (const uint32_t*)flags, (const uint64_t*)pos, out_pairs, out_cap, dev_count);
    PR_HIP(hipGetLastError());
    return PR_OK;
  }
  PR_HIP(hipcub::DeviceRadixSort::SortKeys(tmp, tmp_bytes, keys, sorted, (int)n_keys, 0, 64, s));
  hipLaunchKernelGGL(k_unique_flags, dim3(grid_for(n_keys, 256)), dim3(256), 0, s, (const uint64_t*)sorted, n_keys,
                     flags);
  PR_HIP(device_exclusive_scan((const uint32_t*)flags, pos, n_keys, (int64_t*)tmp, (int64_t*)nullptr, s));
  hipLaunchKernelGGL(k_unique_write, dim3(grid_for(n_keys, 256)), dim3(256), 0, s, (const uint64_t*)sorted, n_keys,
                     (const uint32_t*)flags, (const uint64_t*)pos, out_pairs, out_cap, dev_count);
  PR_HIP(hipGetLastError());
  return PR_OK;
}

extern "C" int estimate_pairs_ws_bytes(int64_t n_meshes_a, int64_t n_meshes_b, int32_t cells, size_t* ws_bytes) {
  if (n_meshes_a < 0 || n_meshes_b < 0 || cells < 1 || cells > 256 || !ws_bytes) {
    set_error("bad argument");
    return PR_E_ARG;
  }
  *ws_bytes = est_ws(n_meshes_a, n_meshes_b, cells);
  return PR_OK;
}

extern "C" int estimate_pairs(const void* blob_a, int64_t n_meshes_a, const void* blob_b, int64_t n_meshes_b,
                              int32_t cells, double* dev_estimate, void* ws, size_t ws_bytes, void* stream) {
  if (!blob_a || !blob_b || !dev_estimate || !ws || n_meshes_a < 0 || n_meshes_b < 0 || cells < 1 || cells > 256) {
    set_error("null pointer or bad size");
    return PR_E_ARG;
  }
  if (ws_bytes < est_ws(n_meshes_a, n_meshes_b, cells)) { set_error("ws_bytes too small"); return PR_E_CAPACITY; }
  hipStream_t s = (hipStream_t)stream;
  char* p = (char*)ws;
  size_t left = ws_bytes;
  EstArgs e{};
  e.blob[0] = (const char*)blob_a;
  e.blob[1] = (const char*)blob_b;
  e.n[0] = n_meshes_a;
  e.n[1] = n_meshes_b;
  e.cells = cells;
  e.side[0] = take<double>(p, left, n_meshes_a);
  e.ratio[0] = take<double>(p, left, n_meshes_a);
  e.side[1] = take<double>(p, left, n_meshes_b);
  e.ratio[1] = take<double>(p, left, n_meshes_b);
  e.ext = take<double>(p, left, 8);
  const int64_t C = (int64_t)cells * cells * cells;
  e.grid = take<double>(p, left, 6 * C);
  e.out = dev_estimate;
  if (!e.grid) { set_error("ws_bytes too small"); return PR_E_CAPACITY; }
  hipLaunchKernelGGL(k_est_init, dim3(grid_for(6 * C, 256)), dim3(256), 0, s, e, 6 * C);
  for (int d = 0; d < 2; ++d)
    if (e.n[d] > 0)
      hipLaunchKernelGGL(k_est_objects, dim3((int)std::min<int64_t>(e.n[d], 65536)), dim3(kDB), 0, s, e, d);
  for (int d = 0; d < 2; ++d)
    if (e.n[d] > 0) hipLaunchKernelGGL(k_est_cells, dim3(grid_for(e.n[d], 256)), dim3(256), 0, s, e, d);
  hipLaunchKernelGGL(k_est_sum, dim3(grid_for(C, kDB)), dim3(kDB), 0, s, e);
  PR_HIP(hipGetLastError());
  return PR_OK;
}
