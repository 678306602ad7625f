// refine_intersects: bidirectional edge-segment tracing per candidate pair.
//
// Work unit: one wavefront traces one group of 64 segments (64 unique edges
// of the source mesh, consecutive in Morton order of their midpoints) against
// the target mesh's wide BVH (Section 3.1 Steps I-II; both directions as in
// Section 3.2).  The wave walks the tree together ("packet" traversal): a
// node is visited once for the whole wave, its child boxes are first tested
// against the group's exact box (one uniform test, exact comparisons), then
// every still-active lane tests its own segment; children hit by any lane
// are pushed with the mask of lanes that hit them onto a per-wave stack in
// LDS.  At a leaf the lanes of the mask test their segment against each
// triangle.  A certain hit marks the pair and every wave working on it stops
// (the paper's multi-hit loop is unnecessary: one BVH holds one mesh, and
// any hit decides the pair).
//
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
#include <hipcub/hipcub.hpp>

#include <climits>

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

template <int W>
constexpr int stack_cap() { return (W - 1) * kMaxDepth + 1; }

struct BlobView {
  const MeshDesc* mesh;
  const char* nodes;
  const float* tris;
  const float* seg;
  const float* cbox;
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
  v.n_meshes = h->n_meshes;
  v.width = h->width;
  v.magic = h->magic;
  return v;
}

enum {
  S_SEG = 0, S_VISIT, S_TESTS, S_AMB32, S_AMB64, S_EXACT, S_TRUE, S_QOVER, S_N
};

struct RefineArgs {
  const char* blob_a;
  const char* blob_b;
  int64_t n_meshes_a, n_meshes_b;
  const int32_t* pairs;
  int64_t n_pairs;
  uint8_t* flags;
  uint32_t* state;            // [P] 0 undecided, 1 intersecting
  int64_t* unit_cnt;          // [2P+1]
  int64_t* offs;              // [2P+1]
  unsigned long long* ctr;    // pop counter
  int4* queue;                // deferred tests (pair, dir, segment slot, triangle)
  uint32_t qcap;
  uint32_t* qcount;
  unsigned long long* stats;  // [S_N]
  int32_t* status;            // [1]
  int32_t chunks_per_pop;
};

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

__device__ __forceinline__ bool slab(const Ray& r, float lx, float ly, float lz, float hx, float hy, float hz) {
  float t0x = (lx - r.px) * r.ix - r.bx, t1x = (hx - r.px) * r.ix + r.bx;
  float t0y = (ly - r.py) * r.iy - r.by, t1y = (hy - r.py) * r.iy + r.by;
  float t0z = (lz - r.pz) * r.iz - r.bz, t1z = (hz - r.pz) * r.iz + r.bz;
  float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.f));
  float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), 1.f));
  return tn <= fmaf(tf, kSlabK, kSlabS);
}

struct WaveStats {
  uint64_t v[S_N];
};

__device__ __forceinline__ f3 tri_vertex(const float* t, int k) { return f3{t[3 * k], t[3 * k + 1], t[3 * k + 2]}; }

// Traces group `chunk` of source mesh sm against target mesh tm.  Returns
// true when the pair is decided (found here or by another wave).
template <int W, int PREC>
__device__ bool trace_chunk(const BlobView& S, const BlobView& T, const MeshDesc& sm, const MeshDesc& tm,
                            int32_t chunk, int32_t pair, int32_t dir, bool safe, const RefineArgs& ra,
                            int32_t* snode, uint64_t* smask, WaveStats& st) {
  const int lane = threadIdx.x & 63;
  const int64_t gc = (int64_t)sm.chunk_base + chunk;
  const int live = min(kChunk, sm.n_edges - chunk * kChunk);
  st.v[S_SEG] += (uint64_t)live;
  float cb[6];
  const float* cbp = S.cbox + 8 * gc;
#pragma unroll
  for (int k = 0; k < 6; ++k) cb[k] = cbp[k];
  if (!box_meet(cb, tm.box[0], tm.box[1], tm.box[2], tm.box[3], tm.box[4], tm.box[5])) return false;
  if (tm.root == kEmpty) return false;
  const bool valid = lane < live;
  const float* sp = S.seg + gc * (6 * kChunk);
  f3 p{sp[lane], sp[kChunk + lane], sp[2 * kChunk + lane]};
  f3 q{sp[3 * kChunk + lane], sp[4 * kChunk + lane], sp[5 * kChunk + lane]};
  Ray r;
  r.px = p.x; r.py = p.y; r.pz = p.z;
  axis_setup(q.x - p.x, safe, r.ix, r.bx);
  axis_setup(q.y - p.y, safe, r.iy, r.by);
  axis_setup(q.z - p.z, safe, r.iz, r.bz);
  uint64_t m0 = ballot(valid && slab(r, tm.box[0], tm.box[1], tm.box[2], tm.box[3], tm.box[4], tm.box[5]));
  if (m0 == 0) return false;
  constexpr int CAP = stack_cap<W>();
  int top = 0;
  if (lane == 0) { snode[0] = tm.root; smask[0] = m0; }
  top = 1;
  int iter = 0;
  const Node<W>* nodes = reinterpret_cast<const Node<W>*>(T.nodes);
  while (top > 0) {
    --top;
    const int32_t node = uni(snode[top]);
    const uint64_t nm = uni64(smask[top]);
    if ((++iter & 15) == 0 && load_state(ra.state + pair)) return true;
    st.v[S_VISIT] += 1;
    const Node<W>* nd = nodes + node;
    const bool on = (nm >> lane) & 1ull;
#pragma unroll
    for (int c = 0; c < W; ++c) {
      const int32_t ch = nd->child[c];
      if (ch == kEmpty) continue;
      const float lx = nd->lo[0][c], ly = nd->lo[1][c], lz = nd->lo[2][c];
      const float hx = nd->hi[0][c], hy = nd->hi[1][c], hz = nd->hi[2][c];
      if (!box_meet(cb, lx, ly, lz, hx, hy, hz)) continue;
      const uint64_t hm = ballot(on && slab(r, lx, ly, lz, hx, hy, hz));
      if (hm == 0) continue;
      if (ch >= 0) {
        if (top >= CAP) {  // cannot happen for a valid blob (depth <= kMaxDepth)
          if (lane == 0) atomicMin(ra.status, (int32_t)PR_E_UNSUPPORTED);
          return true;
        }
        if (lane == 0) { snode[top] = ch; smask[top] = hm; }
        ++top;
        continue;
      }
      const int32_t lr = ~ch;
      const int32_t first = lr >> 3;
      const int cnt = (lr & 7) + 1;
      const bool lon = (hm >> lane) & 1ull;
      for (int t = 0; t < cnt; ++t) {
        const float* tp = T.tris + 9 * (int64_t)(first + t);
        const f3 a = tri_vertex(tp, 0), b = tri_vertex(tp, 1), c3 = tri_vertex(tp, 2);
        int res = kMiss;
        if (lon) {
          if (PREC == 0) {
            res = safe ? seg_tri_f32(p, q, a, b, c3) : kAmbig;
          } else if (PREC == 1) {
            ExactCounters ec{0};
            res = seg_tri_exact(p, q, a, b, c3, ec) ? kHit : kMiss;
          } else {
            res = kAmbig;
          }
        }
        st.v[S_TESTS] += (uint64_t)__popcll(hm);
        if (PREC == 1) st.v[S_EXACT] += (uint64_t)__popcll(hm);
        if (ballot(res == kHit)) {
          if (lane == 0) mark_true(ra.state + pair);
          return true;
        }
        const uint64_t am = ballot(res == kAmbig);
        if (am) {
          st.v[S_AMB32] += (uint64_t)__popcll(am);
          uint32_t base = 0;
          if (lane == 0) base = atomicAdd(ra.qcount, (uint32_t)__popcll(am));
          base = (uint32_t)uni((int32_t)base);
          bool inline_hit = false;
          if (res == kAmbig) {
            const uint32_t idx = base + (uint32_t)lanes_below(am);
            if (idx < ra.qcap) {
              ra.queue[idx] = make_int4(pair, dir, (int32_t)(gc * kChunk + lane), first + t);
            } else {
              ExactCounters ec{0};
              inline_hit = seg_tri_exact(p, q, a, b, c3, ec);
            }
          }
          const uint64_t over = ballot(res == kAmbig && base + (uint32_t)lanes_below(am) >= ra.qcap);
          if (over) {
            st.v[S_QOVER] += (uint64_t)__popcll(over);
            st.v[S_EXACT] += (uint64_t)__popcll(over);
          }
          if (ballot(inline_hit)) {
            if (lane == 0) mark_true(ra.state + pair);
            return true;
          }
        }
      }
    }
  }
  return false;
}

__device__ __forceinline__ void flush_stats(const WaveStats& st, const RefineArgs& ra) {
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < S_N; ++k)
      if (st.v[k]) atomicAdd(ra.stats + k, (unsigned long long)st.v[k]);
  }
}

__device__ __forceinline__ bool pair_ok(const RefineArgs& ra, int64_t p, int32_t& i, int32_t& j) {
  i = ra.pairs[2 * p];
  j = ra.pairs[2 * p + 1];
  return i >= 0 && i < ra.n_meshes_a && j >= 0 && j < ra.n_meshes_b;
}

__device__ __forceinline__ bool blobs_ok(const BlobView& A, const BlobView& B, const RefineArgs& ra, int W) {
  return A.magic == kMagic && B.magic == kMagic && A.width == W && B.width == W && A.n_meshes == ra.n_meshes_a &&
         B.n_meshes == ra.n_meshes_b;
}

// ---- setup --------------------------------------------------------------------

__global__ void k_init(RefineArgs ra) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t p = i; p < ra.n_pairs; p += (int64_t)gridDim.x * blockDim.x) ra.state[p] = 0u;
  if (i < S_N) ra.stats[i] = 0ull;
  if (i == 0) {
    *ra.qcount = 0u;
    *ra.ctr = 0ull;
    *ra.status = PR_OK;
  }
}

// Coarse cull of a direction: does box `b` meet any leaf box of the target
// tree within the first levels?  Conservative (true when unsure).
template <int W>
__device__ bool coarse_meet(const float* b, const BlobView& T, const MeshDesc& tm) {
  if (tm.root == kEmpty) return false;
  const Node<W>* nodes = reinterpret_cast<const Node<W>*>(T.nodes);
  int32_t stk[24];
  int32_t dep[24];
  int sp = 0, visits = 0;
  stk[sp] = tm.root; dep[sp] = 1; ++sp;
  while (sp > 0) {
    --sp;
    int32_t n = stk[sp], d = dep[sp];
    if (++visits > 48) return true;
    const Node<W>* nd = nodes + n;
    for (int c = 0; c < W; ++c) {
      int32_t ch = nd->child[c];
      if (ch == kEmpty) continue;
      if (!box_meet(b, nd->lo[0][c], nd->lo[1][c], nd->lo[2][c], nd->hi[0][c], nd->hi[1][c], nd->hi[2][c])) continue;
      if (ch < 0 || d >= 4 || sp >= 24) return true;
      stk[sp] = ch; dep[sp] = d + 1; ++sp;
    }
  }
  return false;
}

template <int W>
__global__ void k_plan(RefineArgs ra) {
  const BlobView A = view_of(ra.blob_a), B = view_of(ra.blob_b);
  const bool bok = blobs_ok(A, B, ra, W);
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p == 0) ra.unit_cnt[2 * ra.n_pairs] = 0;
  for (; p < ra.n_pairs; p += (int64_t)gridDim.x * blockDim.x) {
    int32_t i, j;
    int64_t c0 = 0, c1 = 0;
    if (!bok) {
      if (p == 0) atomicMin(ra.status, (int32_t)PR_E_UNSUPPORTED);
    } else if (!pair_ok(ra, p, i, j)) {
      atomicMin(ra.status, (int32_t)PR_E_ARG);
    } else {
      const MeshDesc a = A.mesh[i], b = B.mesh[j];
      if (box_meet(a.box, b.box[0], b.box[1], b.box[2], b.box[3], b.box[4], b.box[5])) {
        if (coarse_meet<W>(a.box, B, b)) c0 = a.n_chunks;
        if (coarse_meet<W>(b.box, A, a)) c1 = b.n_chunks;
      }
    }
    ra.unit_cnt[2 * p] = c0;
    ra.unit_cnt[2 * p + 1] = c1;
  }
}

// Unit u (a (pair, direction)) holding global group index v: offs[u] <= v < offs[u+1].
__device__ __forceinline__ int64_t find_unit(const int64_t* offs, int64_t U, int64_t v) {
  const int lane = threadIdx.x & 63;
  int64_t lo = 0, hi = U;
  while (hi - lo > 1) {
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t idx = lo + (int64_t)lane * step;
    const bool ok = idx < hi && offs[idx] <= v;
    const uint64_t m = ballot(ok);
    const int last = 63 - __clzll((long long)m);
    lo = lo + (int64_t)last * step;
    const int64_t nh = lo + step;
    hi = nh < hi ? nh : hi;
  }
  return lo;
}

template <int W, int PREC>
__global__ __launch_bounds__(kBlock) void k_refine_persistent(RefineArgs ra) {
  constexpr int CAP = stack_cap<W>();
  __shared__ int32_t s_node[kWaves][CAP];
  __shared__ uint64_t s_mask[kWaves][CAP];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const BlobView A = view_of(ra.blob_a), B = view_of(ra.blob_b);
  if (!blobs_ok(A, B, ra, W)) return;
  const int64_t U = 2 * ra.n_pairs;
  const int64_t total = ra.offs[U];
  const int64_t G = ra.chunks_per_pop;
  WaveStats st;
#pragma unroll
  for (int k = 0; k < S_N; ++k) st.v[k] = 0;
  int64_t cur_lo = 0, cur_hi = 0;
  int32_t pair = 0, dir = 0;
  MeshDesc sm, tm;
  bool safe = false, skip = false;
  for (;;) {
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(ra.ctr, (unsigned long long)G);
    base = uni64(base);
    if ((int64_t)base >= total) break;
    const int64_t end = ((int64_t)base + G < total) ? (int64_t)base + G : total;
    for (int64_t v = (int64_t)base; v < end; ++v) {
      if (v >= cur_hi || v < cur_lo) {
        const int64_t u = find_unit(ra.offs, U, v);
        cur_lo = ra.offs[u];
        cur_hi = ra.offs[u + 1];
        pair = uni((int32_t)(u >> 1));
        dir = uni((int32_t)(u & 1));
        const int32_t i = ra.pairs[2 * (int64_t)pair], j = ra.pairs[2 * (int64_t)pair + 1];
        sm = dir == 0 ? A.mesh[i] : B.mesh[j];
        tm = dir == 0 ? B.mesh[j] : A.mesh[i];
        safe = (sm.flags & tm.flags & kMeshSafe) != 0;
        skip = false;
      }
      if (skip) continue;
      if (load_state(ra.state + pair)) { skip = true; continue; }
      const int32_t chunk = (int32_t)(v - cur_lo);
      if (trace_chunk<W, PREC>(dir == 0 ? A : B, dir == 0 ? B : A, sm, tm, chunk, pair, dir, safe, ra,
                               s_node[wv], s_mask[wv], st))
        skip = true;
    }
  }
  flush_stats(st, ra);
}

template <int W, int PREC>
__global__ __launch_bounds__(kBlock) void k_refine_pair(RefineArgs ra, int64_t p) {
  constexpr int CAP = stack_cap<W>();
  __shared__ int32_t s_node[kWaves][CAP];
  __shared__ uint64_t s_mask[kWaves][CAP];
  const int wv = threadIdx.x >> 6;
  const BlobView A = view_of(ra.blob_a), B = view_of(ra.blob_b);
  int32_t i, j;
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
#pragma unroll
  for (int k = 0; k < S_N; ++k) st.v[k] = 0;
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

// ---- deferred FP64 / exact decisions ----------------------------------------------

__global__ void k_redecide(RefineArgs ra) {
  const BlobView A = view_of(ra.blob_a), B = view_of(ra.blob_b);
  const uint32_t qn = *ra.qcount;
  const uint32_t n = qn < ra.qcap ? qn : ra.qcap;
  uint64_t nexact = 0, namb = 0;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int4 e = ra.queue[k];
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
  if (nexact) atomicAdd(ra.stats + S_EXACT, (unsigned long long)nexact);
  if (namb) atomicAdd(ra.stats + S_AMB64, (unsigned long long)namb);
}

__global__ void k_finalize(RefineArgs ra) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  unsigned long long cnt = 0;
  for (; p < ra.n_pairs; p += (int64_t)gridDim.x * blockDim.x) {
    const uint8_t f = ra.state[p] ? 1 : 0;
    ra.flags[p] = f;
    cnt += f;
  }
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(ra.stats + S_TRUE, cnt);
}

__global__ void k_report(RefineArgs ra, pr_refine_stats* out, int32_t* dev_status) {
  if (out) {
    out->segments = ra.stats[S_SEG];
    out->node_visits = ra.stats[S_VISIT];
    out->tri_tests = ra.stats[S_TESTS];
    out->fp32_ambiguous = ra.stats[S_AMB32];
    out->fp64_filter_ambiguous = ra.stats[S_AMB64];
    out->exact_decided = ra.stats[S_EXACT];
    out->pairs_true = ra.stats[S_TRUE];
    out->queue_overflow = ra.stats[S_QOVER];
  }
  if (dev_status) *dev_status = *ra.status;
}

// ---- host side ---------------------------------------------------------------------

struct WsLayout {
  size_t total;
  size_t scan_bytes;
};

int carve(Carve& cv, RefineArgs& ra, int64_t P, uint32_t qcap, void** scan_tmp, size_t* scan_bytes) {
  ra.state = cv.take<uint32_t>(P);
  ra.unit_cnt = cv.take<int64_t>(2 * P + 1);
  ra.offs = cv.take<int64_t>(2 * P + 1);
  ra.ctr = cv.take<unsigned long long>(1);
  ra.qcount = cv.take<uint32_t>(1);
  ra.stats = cv.take<unsigned long long>(S_N);
  ra.status = cv.take<int32_t>(1);
  ra.queue = cv.take<int4>(qcap);
  size_t b = 0;
  hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, b, (int64_t*)nullptr, (int64_t*)nullptr, (int)(2 * P + 1));
  if (e != hipSuccess) return hip_fail(e, "hipcub scan size");
  *scan_bytes = b;
  *scan_tmp = cv.take<char>((int64_t)b);
  return PR_OK;
}

int check(int64_t P, const pr_refine_params* p) {
  if (!p) { set_error("params is NULL"); return PR_E_ARG; }
  if (!(p->bvh_width == 2 || p->bvh_width == 4 || p->bvh_width == 8)) { set_error("bvh_width must be 2, 4 or 8"); return PR_E_ARG; }
  if (p->precision < 0 || p->precision > 2) { set_error("precision must be 0, 1 or 2"); return PR_E_ARG; }
  if (p->persistent < 0 || p->persistent > 1) { set_error("persistent must be 0 or 1"); return PR_E_ARG; }
  if (p->queue_cap < 0 || p->grid_blocks < 0 || p->chunks_per_pop < 0) { set_error("negative launch parameter"); return PR_E_ARG; }
  if (p->reserved[0] || p->reserved[1]) { set_error("reserved fields must be 0"); return PR_E_ARG; }
  if (P < 0) { set_error("n_pairs < 0"); return PR_E_ARG; }
  if (P >= ((int64_t)1 << 30)) { set_error("n_pairs >= 2^30"); return PR_E_UNSUPPORTED; }
  return PR_OK;
}

uint32_t qcap_of(const pr_refine_params* p) { return p->queue_cap > 0 ? (uint32_t)p->queue_cap : (1u << 20); }

template <int W, int PREC>
int launch(RefineArgs& ra, const pr_refine_params* prm, void* scan_tmp, size_t scan_bytes, hipStream_t s) {
  const int64_t P = ra.n_pairs;
  if (prm->persistent) {
    hipLaunchKernelGGL(k_plan<W>, dim3(grid_for(P, kBlock)), dim3(kBlock), 0, s, ra);
    PR_HIP(hipcub::DeviceScan::ExclusiveSum(scan_tmp, scan_bytes, ra.unit_cnt, ra.offs, (int)(2 * P + 1), s));
    int blocks = prm->grid_blocks;
    if (blocks <= 0) {
      int dev = 0, cus = 0, per = 0;
      PR_HIP(hipGetDevice(&dev));
      PR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
      PR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_refine_persistent<W, PREC>, kBlock, 0));
      blocks = cus * (per > 0 ? per : 1);
    }
    hipLaunchKernelGGL((k_refine_persistent<W, PREC>), dim3(blocks), dim3(kBlock), 0, s, ra);
  } else {
    const int blocks = prm->grid_blocks > 0 ? prm->grid_blocks : 64;
    for (int64_t p = 0; p < P; ++p) hipLaunchKernelGGL((k_refine_pair<W, PREC>), dim3(blocks), dim3(kBlock), 0, s, ra, p);
  }
  return PR_OK;
}

}  // namespace
}  // namespace pr

using namespace pr;

extern "C" int refine_workspace_bytes(int64_t n_pairs, const pr_refine_params* params, size_t* ws_bytes) {
  int r = check(n_pairs, params);
  if (r) return r;
  if (!ws_bytes) { set_error("ws_bytes is NULL"); return PR_E_ARG; }
  Carve cv{nullptr, 0};
  RefineArgs ra{};
  void* t;
  size_t b;
  r = carve(cv, ra, n_pairs, qcap_of(params), &t, &b);
  if (r) return r;
  *ws_bytes = cv.used + 256;
  return PR_OK;
}

extern "C" int refine_intersects(const void* blob_a, int64_t n_meshes_a, const void* blob_b, int64_t n_meshes_b,
                                 const int32_t* pairs, int64_t n_pairs, uint8_t* flags,
                                 const pr_refine_params* params, pr_refine_stats* dev_stats, int32_t* dev_status,
                                 void* ws, size_t ws_bytes, void* stream) {
  int r = check(n_pairs, params);
  if (r) return r;
  if (!blob_a || !blob_b || !ws || (n_pairs > 0 && (!pairs || !flags)) || n_meshes_a < 0 || n_meshes_b < 0) {
    set_error("null pointer or negative size");
    return PR_E_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  RefineArgs ra{};
  Carve cv{(char*)ws, ws_bytes};
  void* scan_tmp = nullptr;
  size_t scan_bytes = 0;
  const uint32_t qcap = qcap_of(params);
  r = carve(cv, ra, n_pairs, qcap, &scan_tmp, &scan_bytes);
  if (r) return r;
  if (cv.used > ws_bytes || !scan_tmp) { set_error("ws_bytes %zu < required %zu", ws_bytes, cv.used); return PR_E_CAPACITY; }
  ra.blob_a = (const char*)blob_a;
  ra.blob_b = (const char*)blob_b;
  ra.n_meshes_a = n_meshes_a;
  ra.n_meshes_b = n_meshes_b;
  ra.pairs = pairs;
  ra.n_pairs = n_pairs;
  ra.flags = flags;
  ra.qcap = qcap;
  ra.chunks_per_pop = params->chunks_per_pop > 0 ? params->chunks_per_pop : 4;
  hipLaunchKernelGGL(k_init, dim3(grid_for(n_pairs > S_N ? n_pairs : S_N, kBlock)), dim3(kBlock), 0, s, ra);
  if (n_pairs > 0) {
    const int W = params->bvh_width, PREC = params->precision;
#define PR_LAUNCH(w, q) if (W == w && PREC == q) r = launch<w, q>(ra, params, scan_tmp, scan_bytes, s)
    PR_LAUNCH(2, 0); PR_LAUNCH(2, 1); PR_LAUNCH(2, 2);
    PR_LAUNCH(4, 0); PR_LAUNCH(4, 1); PR_LAUNCH(4, 2);
    PR_LAUNCH(8, 0); PR_LAUNCH(8, 1); PR_LAUNCH(8, 2);
#undef PR_LAUNCH
    if (r) return r;
    hipLaunchKernelGGL(k_redecide, dim3(1024), dim3(kBlock), 0, s, ra);
    hipLaunchKernelGGL(k_finalize, dim3(grid_for(n_pairs, kBlock)), dim3(kBlock), 0, s, ra);
  }
  hipLaunchKernelGGL(k_report, dim3(1), dim3(1), 0, s, ra, dev_stats, dev_status);
  PR_HIP(hipGetLastError());
  return PR_OK;
}
