// build_mesh_bvh: per-mesh wide BVHs and unique-edge segments for a dataset.
//
// Steps (all on the device, one batched pass over every mesh):
//  1. validate faces (ids in range, finite coordinates, not exactly collinear),
//     exact triangle boxes, per-mesh exact boxes and FP32-safe flags;
//  2. Morton codes of triangle centroids relative to their mesh box, keyed
//     by mesh id, sorted (one radix sort for all meshes);
//  3. per mesh, a binary radix tree over the sorted codes (Karras 2012,
//     "Maximizing parallelism in the construction of BVHs, octrees, and k-d
//     trees"), ties broken by position;
//  4. bottom-up refit with exact min/max boxes;
//  5. collapse to width W: each wide node starts from a binary node and
//     repeatedly opens the child with the largest box surface among those
//     holding more than L triangles, until it has W children; children of at
//     most L triangles become leaves (a Karras subtree is a contiguous range
//     of the sorted order, so a leaf is a range of leaf-order triangles);
//  6. unique edges (Section 3.1: duplicate edges of one mesh are merged), as
//     (min, max) global vertex id keys, sorted and deduplicated, then ordered
//     inside each mesh by the Morton code of their midpoint so that a group of
//     64 consecutive segments is spatially coherent, and written as FP32
//     endpoints in groups of 64 with the exact box of each group.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "scan.h"

#include <climits>
#include <cstdio>

#include "common.h"
#include "predicates.h"

namespace pr {
namespace {

constexpr int kBlock = 256;
// threads of the one-block-per-mesh kernels (refit, collapse): the largest
// mesh's block is the end of those launches
constexpr int kMeshBlock = 1024;

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__device__ __forceinline__ uint32_t quant10(float c, float lo, float hi) {
  float ext = hi - lo;
  if (!(ext > 0.f)) return 0;
  float t = (c - lo) / ext * 1024.f;
  int q = (int)t;
  return (uint32_t)(q < 0 ? 0 : (q > 1023 ? 1023 : q));
}

__device__ __forceinline__ uint32_t morton3(f3 c, const float* box) {
  return (spread10(quant10(c.x, box[0], box[3])) << 2) | (spread10(quant10(c.y, box[1], box[4])) << 1) |
         spread10(quant10(c.z, box[2], box[5]));
}

__device__ __forceinline__ bool safe_coord(float c) {
  float a = fabsf(c);
  return c == 0.f || (a >= kSafeLo && a <= kSafeHi);
}

__device__ __forceinline__ f3 load_v(const float* verts, int64_t g) {
  return f3{verts[3 * g], verts[3 * g + 1], verts[3 * g + 2]};
}

struct BuildArgs {
  const float* verts;
  const int64_t* vert_off;
  const int32_t* faces;
  const int64_t* face_off;
  int64_t n_meshes, v_total, f_total;
  int width, leaf;
  int builder;           // 0: open the largest-area child, 1: the largest area x triangle count
  // blob sections
  char* blob;
  MeshDesc* mesh;
  char* nodes;
  float* tris;
  int32_t* triid;
  float* seg;
  int32_t* edge;
  float* cbox;
  int32_t* cmesh;
  float* rep;            // [M][4] representative vertex of each mesh
  float* rbox;           // [chunk_cap][8] box of each run of 64 groups, at the run's first group
  int64_t node_cap, chunk_cap;
  // workspace
  int32_t* status;       // min bad face (INT_MAX if none)
  int32_t* face_mesh;    // [F]
  float* tbox;           // [F][6]
  uint8_t* fsafe;        // [F]
  uint64_t* key0;        // [F]
  uint64_t* key1;        // [F]
  int32_t* val0;         // [F]
  int32_t* val1;         // [F]
  int32_t* left;         // [F] binary children (bit 31: leaf, payload: global sorted position)
  int32_t* right;        // [F]
  int32_t* parent;       // [F] parent of internal node g
  int32_t* lparent;      // [F] parent of leaf position g
  float* nbox;           // [F][6]
  int32_t* nleaf;        // [F] triangles under each binary node
  int32_t* nfirst;       // [F]
  uint32_t* visit;       // [F]
  int64_t* nbound;       // [M+1] scanned node bounds
  int32_t* stk;          // [F][3] collapse work stacks
  uint64_t* ekey0;       // [3F]
  uint64_t* ekey1;       // [3F]
  int32_t* eval0;        // [3F]
  int32_t* eval1;        // [3F]
  int32_t* eflag;        // [3F + 1]
  int32_t* epos;         // [3F + 1]
  int32_t* estart;       // [M]
  int32_t* eend;         // [M]
  int64_t* cscan;        // [M+1]
  int32_t* meshctr;      // [4] misc device counters: [0] lowest, [1] highest coordinate bit exponent
  uint8_t* mesh_ok;      // [M] offsets of the mesh are consistent
  uint64_t* ekey2;       // [3F] sorted (mesh, Morton) keys of unique edges
  int64_t* nscan;        // [M+1] scanned node bounds
  int64_t* chunk_scan;   // [M+1] scanned group counts
  char* tnodes;          // [node_cap] nodes at bound-sized offsets, before compaction
  int64_t* ncount;       // [M+1] nodes used per mesh, then scanned
  int64_t* tsum;         // tile sums of the prefix sums
  int32_t* morder;       // [M] meshes in decreasing size class (the per-mesh kernels' order)
  int32_t* mcnt;         // [kSizeClasses][order blocks] meshes of each class in each block
  int64_t* mpos;         // the same, scanned
};

// The per-mesh kernels (refit, collapse, node copy) give each mesh one
// block, and a launch ends with its largest mesh; blocks therefore take the
// meshes in decreasing size class (powers of two of the face count), index
// order within a class: a stable counting sort of kMeshOrdTile meshes per
// block (class counts, a scan, then each mesh's place).
constexpr int kSizeClasses = 8;
constexpr int kMeshOrdTile = 1024;  // meshes per block of the order kernels (4 per thread)

// ---- mesh order ----------------------------------------------------------------

__device__ __forceinline__ int size_class(const BuildArgs& a, int64_t m) {
  const int64_t n = a.face_off[m + 1] - a.face_off[m];
  const int lg = n > 0 ? 63 - __builtin_clzll((uint64_t)n) : 0;
  return lg >= 16 ? 0 : (lg <= 9 ? kSizeClasses - 1 : 16 - lg);
}

// Per thread: the classes of its 4 meshes (kSizeClasses for none) and its
// count of each class, 16 bits a class (classes 0-3 in w0, 4-7 in w1).
__device__ __forceinline__ void mesh_items(const BuildArgs& a, int* cls, uint64_t& w0, uint64_t& w1) {
  const int64_t m0 = blockIdx.x * (int64_t)kMeshOrdTile + 4 * (int64_t)threadIdx.x;
  w0 = 0;
  w1 = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = m0 + k < a.n_meshes ? size_class(a, m0 + k) : kSizeClasses;
    cls[k] = c;
    if (c < 4) w0 += 1ull << (16 * c);
    else if (c < kSizeClasses) w1 += 1ull << (16 * (c - 4));
  }
}

__global__ __launch_bounds__(256) void k_mesh_order_count(BuildArgs a, int64_t nb) {
  __shared__ uint64_t s[4];
  int cls[4];
  uint64_t w0, w1;
  mesh_items(a, cls, w0, w1);
  const uint64_t t0 = block_sum<256>(w0, s), t1 = block_sum<256>(w1, s);
  if (threadIdx.x < kSizeClasses) {
    const uint64_t t = threadIdx.x < 4 ? t0 >> (16 * threadIdx.x) : t1 >> (16 * (threadIdx.x - 4));
    a.mcnt[threadIdx.x * nb + blockIdx.x] = (int32_t)(t & 0xffffu);
  }
}

__global__ __launch_bounds__(256) void k_mesh_order_place(BuildArgs a, int64_t nb) {
  __shared__ uint64_t s[4];
  int cls[4];
  uint64_t w0, w1;
  mesh_items(a, cls, w0, w1);
  uint64_t t0, t1;
  const uint64_t e0 = block_exclusive_sum<256>(w0, s, t0), e1 = block_exclusive_sum<256>(w1, s, t1);
  const int64_t m0 = blockIdx.x * (int64_t)kMeshOrdTile + 4 * (int64_t)threadIdx.x;
  uint32_t seen = 0;  // this thread's earlier meshes, 4 bits a class
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = cls[k];
    if (c >= kSizeClasses) continue;
    const uint64_t before = c < 4 ? (e0 >> (16 * c)) & 0xffffu : (e1 >> (16 * (c - 4))) & 0xffffu;
    a.morder[a.mpos[c * nb + blockIdx.x] + (int64_t)before + ((seen >> (4 * c)) & 0xfu)] = (int32_t)(m0 + k);
    seen += 1u << (4 * c);
  }
}

// ---- step 1 ---------------------------------------------------------------

__global__ void k_face_mesh(BuildArgs a) {
  for (int64_t m = blockIdx.x; m < a.n_meshes; m += gridDim.x) {
    int64_t f0 = a.face_off[m], f1 = a.face_off[m + 1];
    int64_t v0 = a.vert_off[m], v1 = a.vert_off[m + 1];
    bool ok = f0 >= 0 && f1 >= f0 && f1 <= a.f_total && v0 >= 0 && v1 >= v0 && v1 <= a.v_total;
    if (m == 0) ok = ok && f0 == 0 && v0 == 0;
    if (m == a.n_meshes - 1) ok = ok && f1 == a.f_total && v1 == a.v_total;
    if (threadIdx.x == 0) {
      a.mesh_ok[m] = ok ? 1 : 0;
      if (!ok) atomicMin(a.status, 0);
    }
    if (!ok) continue;
    for (int64_t f = f0 + threadIdx.x; f < f1; f += blockDim.x) a.face_mesh[f] = (int32_t)m;
  }
}

// Exponents of the lowest and highest set bit of a finite non-zero FP32 value.
__device__ __forceinline__ int bit_lo(float x) {
  const uint32_t b = __float_as_uint(x) & 0x7fffffffu;
  const uint32_t e = b >> 23, m = b & 0x7fffffu;
  return e == 0 ? -149 + __builtin_ctz(m) : (int)e - 150 + __builtin_ctz(m | 0x800000u);
}
__device__ __forceinline__ int bit_hi(float x) {
  const uint32_t b = __float_as_uint(x) & 0x7fffffffu;
  const uint32_t e = b >> 23, m = b & 0x7fffffu;
  return e == 0 ? -149 + (31 - __builtin_clz(m)) : (int)e - 127;
}

__global__ void k_tri_prep(BuildArgs a) {
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int elo = INT_MAX, ehi = INT_MIN;  // bit exponents over this thread's coordinates
  for (; f < a.f_total; f += (int64_t)gridDim.x * blockDim.x) {
    int32_t m = a.face_mesh[f];
    bool mok = a.mesh_ok[m];
    int64_t v0 = mok ? a.vert_off[m] : 0, nv = mok ? a.vert_off[m + 1] - v0 : 0;
    int32_t id[3] = {a.faces[3 * f], a.faces[3 * f + 1], a.faces[3 * f + 2]};
    bool bad = !mok;
    for (int k = 0; k < 3; ++k) bad |= (id[k] < 0 || id[k] >= nv);
    float* tb = a.tbox + 6 * f;
    if (bad) {
      atomicMin(a.status, (int32_t)f);
      for (int k = 0; k < 3; ++k) { tb[k] = 0.f; tb[3 + k] = 0.f; }
      a.fsafe[f] = 0;
      continue;
    }
    f3 p0 = load_v(a.verts, v0 + id[0]), p1 = load_v(a.verts, v0 + id[1]), p2 = load_v(a.verts, v0 + id[2]);
    float cs[9] = {p0.x, p0.y, p0.z, p1.x, p1.y, p1.z, p2.x, p2.y, p2.z};
    bool fin = true, safe = true;
    for (int k = 0; k < 9; ++k) { fin &= isfinite(cs[k]); safe &= safe_coord(cs[k]); }
    for (int k = 0; k < 9; ++k)
      if (fin && cs[k] != 0.f) {
        elo = min(elo, bit_lo(cs[k]));
        ehi = max(ehi, bit_hi(cs[k]));
      }
    if (!fin) {
      atomicMin(a.status, (int32_t)f);
      safe = false;
    } else {
      // exactly collinear iff all three coordinate-plane orientations vanish
      ExactCounters cnt{0};
      bool degen = sign_orient2d(p0, p1, p2, 1, 2, cnt) == 0 && sign_orient2d(p0, p1, p2, 2, 0, cnt) == 0 &&
                   sign_orient2d(p0, p1, p2, 0, 1, cnt) == 0;
      if (degen) atomicMin(a.status, (int32_t)f);
    }
    tb[0] = fminf(fminf(p0.x, p1.x), p2.x);
    tb[1] = fminf(fminf(p0.y, p1.y), p2.y);
    tb[2] = fminf(fminf(p0.z, p1.z), p2.z);
    tb[3] = fmaxf(fmaxf(p0.x, p1.x), p2.x);
    tb[4] = fmaxf(fmaxf(p0.y, p1.y), p2.y);
    tb[5] = fmaxf(fmaxf(p0.z, p1.z), p2.z);
    a.fsafe[f] = safe ? 1 : 0;
  }
  // one atomic pair per wave (the grid is capped so that these stay few)
  for (int o = 32; o > 0; o >>= 1) {
    elo = min(elo, __shfl_xor(elo, o));
    ehi = max(ehi, __shfl_xor(ehi, o));
  }
  if ((threadIdx.x & 63) == 0 && elo != INT_MAX) {
    atomicMin(a.meshctr + 0, elo);
    atomicMax(a.meshctr + 1, ehi);
  }
}

__device__ __forceinline__ float blk_min(float v, float* sh) {
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  float r = sh[0];
  for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = fminf(r, sh[i]);
  return r;
}

__device__ __forceinline__ float blk_max(float v, float* sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  float r = sh[0];
  for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = fmaxf(r, sh[i]);
  return r;
}

__global__ void k_mesh_box(BuildArgs a) {
  __shared__ float sh[16];
  for (int64_t m = blockIdx.x; m < a.n_meshes; m += gridDim.x) {
    int64_t f0 = a.face_off[m], f1 = a.face_off[m + 1];
    if (!a.mesh_ok[m]) { f0 = 0; f1 = 0; }
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    float safe = 1.f;
    for (int64_t f = f0 + threadIdx.x; f < f1; f += blockDim.x) {
      const float* tb = a.tbox + 6 * f;
      for (int k = 0; k < 3; ++k) { lo[k] = fminf(lo[k], tb[k]); hi[k] = fmaxf(hi[k], tb[3 + k]); }
      if (!a.fsafe[f]) safe = 0.f;
    }
    float r[6];
    for (int k = 0; k < 3; ++k) { r[k] = blk_min(lo[k], sh); r[3 + k] = blk_max(hi[k], sh); }
    float s = blk_min(safe, sh);
    if (threadIdx.x == 0) {
      MeshDesc d;
      for (int k = 0; k < 6; ++k) d.box[k] = r[k];
      d.node_base = 0; d.n_nodes = 0;
      d.tri_base = (int32_t)f0;
      d.n_tris = (int32_t)(f1 - f0);
      d.chunk_base = 0; d.n_chunks = 0; d.n_edges = 0; d.depth = 0;
      d.root = kEmpty;
      d.flags = s > 0.f ? kMeshSafe : 0;
      a.mesh[m] = d;
      // representative vertex for the point-in-mesh test: the first corner
      // of the mesh's first face (the face id is range-checked here; a bad
      // id fails the build through the status word anyway)
      float4 rv = make_float4(0.f, 0.f, 0.f, 0.f);
      if (f1 > f0) {
        const int64_t v0 = a.vert_off[m], nv = a.vert_off[m + 1] - v0;
        const int32_t id = a.faces[3 * f0];
        if (id >= 0 && id < nv) {
          const float* x = a.verts + 3 * (v0 + id);
          rv = make_float4(x[0], x[1], x[2], 1.f);
        }
      }
      reinterpret_cast<float4*>(a.rep)[m] = rv;
    }
  }
}

// ---- step 2 ---------------------------------------------------------------

__global__ void k_morton(BuildArgs a) {
  if (*a.status != INT_MAX) return;  // invalid input: the blob is not built
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; f < a.f_total; f += (int64_t)gridDim.x * blockDim.x) {
    int32_t m = a.face_mesh[f];
    const float* tb = a.tbox + 6 * f;
    f3 c{0.5f * (tb[0] + tb[3]), 0.5f * (tb[1] + tb[4]), 0.5f * (tb[2] + tb[5])};
    uint32_t code = morton3(c, a.mesh[m].box);
    a.key0[f] = ((uint64_t)(uint32_t)m << kMortonBits) | code;
    a.val0[f] = (int32_t)f;
  }
}

// ---- step 3: Karras radix tree ---------------------------------------------

__device__ __forceinline__ int delta(const uint64_t* keys, int64_t base, int n, int i, int j) {
  if (j < 0 || j >= n) return -1;
  uint32_t ki = (uint32_t)(keys[base + i] & ((1u << kMortonBits) - 1));
  uint32_t kj = (uint32_t)(keys[base + j] & ((1u << kMortonBits) - 1));
  if (ki != kj) return __clz(ki ^ kj);
  return 32 + __clz((uint32_t)(i ^ j));
}

__global__ void k_karras(BuildArgs a, const uint64_t* keys) {
  if (*a.status != INT_MAX) return;  // invalid input: the blob is not built
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; g < a.f_total; g += (int64_t)gridDim.x * blockDim.x) {
    int32_t m = a.face_mesh[g];
    int64_t base = a.face_off[m];
    int n = (int)(a.face_off[m + 1] - base);
    int i = (int)(g - base);
    if (i == 0) a.parent[g] = -1;  // root (or the single leaf's slot)
    if (n == 1) { a.lparent[g] = -1; continue; }
    if (i >= n - 1) continue;
    int d = (delta(keys, base, n, i, i + 1) - delta(keys, base, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = delta(keys, base, n, i, i - d);
    int lmax = 2;
    while (delta(keys, base, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
      if (delta(keys, base, n, i, i + (l + t) * d) > dmin) l += t;
    int j = i + l * d;
    int dnode = delta(keys, base, n, i, j);
    int s = 0;
    int t = l;
    do {
      t = (t + 1) >> 1;
      if (delta(keys, base, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int split = i + s * d + (d < 0 ? -1 : 0);
    int lo = i < j ? i : j, hi = i < j ? j : i;
    int32_t lc, rc;
    if (lo == split) { lc = (int32_t)(base + split) | INT_MIN; a.lparent[base + split] = (int32_t)g; }
    else { lc = (int32_t)(base + split); a.parent[base + split] = (int32_t)g; }
    if (hi == split + 1) { rc = (int32_t)(base + split + 1) | INT_MIN; a.lparent[base + split + 1] = (int32_t)g; }
    else { rc = (int32_t)(base + split + 1); a.parent[base + split + 1] = (int32_t)g; }
    a.left[g] = lc;
    a.right[g] = rc;
  }
}

// ---- step 4: refit ------------------------------------------------------------

__device__ __forceinline__ void child_info(const BuildArgs& a, int32_t c, const int32_t* sorted_face, float* box,
                                           int32_t& count, int32_t& first) {
  if (c < 0) {
    int32_t pos = c & INT_MAX;
    const float* tb = a.tbox + 6 * (int64_t)sorted_face[pos];
    for (int k = 0; k < 6; ++k) box[k] = tb[k];
    count = 1;
    first = pos;
  } else {
    for (int k = 0; k < 6; ++k) box[k] = a.nbox[6 * (int64_t)c + k];
    count = a.nleaf[c];
    first = a.nfirst[c];
  }
}

// One block per mesh: every climb of a mesh stays inside one workgroup, so
// workgroup-scope acquire/release on the visit counters orders the box
// writes without device-wide cache maintenance.
__global__ __launch_bounds__(kMeshBlock) void k_refit(BuildArgs a, const int32_t* sorted_face) {
  if (*a.status != INT_MAX) return;  // invalid input: the blob is not built
  for (int64_t mi = blockIdx.x; mi < a.n_meshes; mi += gridDim.x) {
    const int64_t m = a.morder[mi];
    const int64_t f0 = a.face_off[m], f1 = a.face_off[m + 1];
    for (int64_t g = f0 + threadIdx.x; g < f1; g += blockDim.x) {
      int32_t p = a.lparent[g];
      while (p >= 0) {
        uint32_t old = __hip_atomic_fetch_add(&a.visit[p], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == 0) break;  // the sibling subtree is not done yet
        float bl[6], br[6];
        int32_t cl, cr, fl, fr;
        child_info(a, a.left[p], sorted_face, bl, cl, fl);
        child_info(a, a.right[p], sorted_face, br, cr, fr);
        for (int k = 0; k < 3; ++k) {
          a.nbox[6 * (int64_t)p + k] = fminf(bl[k], br[k]);
          a.nbox[6 * (int64_t)p + 3 + k] = fmaxf(bl[3 + k], br[3 + k]);
        }
        a.nleaf[p] = cl + cr;
        a.nfirst[p] = fl < fr ? fl : fr;
        p = a.parent[p];
      }
    }
  }
}

// ---- step 5: collapse to width W -------------------------------------------

__global__ void k_node_bound(BuildArgs a) {
  int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; m < a.n_meshes; m += (int64_t)gridDim.x * blockDim.x) {
    int64_t n = a.mesh[m].n_tris;
    a.nbound[m] = nodes_bound(n, a.width, a.leaf);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.nbound[a.n_meshes] = 0;
}

__device__ __forceinline__ float half_area(const float* b) {
  float dx = b[3] - b[0], dy = b[4] - b[1], dz = b[5] - b[2];
  return dx * dy + dy * dz + dz * dx;
}

// Collapse of each mesh's binary tree into a width-W tree, one block per
// mesh, one level of wide nodes per round.  An item is (binary subtree root,
// wide slot, depth); the block's threads take the items of the current
// level one each.  A thread starts from the two children of its binary node
// and keeps opening one of them until it holds W children or none can be
// opened (only subtrees of more than L triangles are opened): builder 0 opens
// the child of largest surface area, builder 1 the child of largest surface
// area x triangle count (its term of the surface-area cost).  It writes the
// wide node and appends an item, with a fresh slot, for every child that
// needs a wide node of its own.  Slots are numbered in creation order (root
// 0), so the top levels of a tree sit together.  Items live in the mesh's
// part of the work array (at most one per internal binary node).
template <int W>
__device__ void collapse_item(const BuildArgs& a, Node<W>* nodes, int64_t nb, int64_t bound, int32_t* items,
                              int it, int32_t* s_used, int32_t* s_tail, int32_t* s_depth, int32_t* s_over) {
  const int32_t x = items[3 * it], w = items[3 * it + 1], dep = items[3 * it + 2];
  atomicMax(s_depth, dep);
  const int L = a.leaf;
  int32_t S[W];
  float Sb[W][6];
  int32_t Sc[W], Sf[W];
  int ns = 2;
  S[0] = a.left[x];
  S[1] = a.right[x];
  child_info(a, S[0], a.val1, Sb[0], Sc[0], Sf[0]);
  child_info(a, S[1], a.val1, Sb[1], Sc[1], Sf[1]);
  while (ns < W) {
    int best = -1;
    float bscore = -1.f;
    for (int k = 0; k < ns; ++k)
      if (S[k] >= 0 && Sc[k] > L) {
        const float ar = half_area(Sb[k]);
        const float score = a.builder == 1 ? ar * (float)Sc[k] : ar;
        if (score > bscore) { bscore = score; best = k; }
      }
    if (best < 0) break;
    const int32_t y = S[best];
    S[best] = a.left[y];
    S[ns] = a.right[y];
    child_info(a, S[best], a.val1, Sb[best], Sc[best], Sf[best]);
    child_info(a, S[ns], a.val1, Sb[ns], Sc[ns], Sf[ns]);
    ++ns;
  }
  Node<W> nd;
  for (int c = 0; c < W; ++c) {
    nd.pad[c] = 0;
    if (c < ns) {
      for (int k = 0; k < 3; ++k) { nd.lo[k][c] = Sb[c][k]; nd.hi[k][c] = Sb[c][3 + k]; }
      if (Sc[c] <= L) {
        nd.child[c] = leaf_ref(Sf[c], Sc[c]);
      } else {
        const int32_t slot = atomicAdd(s_used, 1);
        if (slot >= bound) {
          *s_over = 1;
          nd.child[c] = kEmpty;
          continue;
        }
        nd.child[c] = (int32_t)(nb + slot);
        const int32_t pos = atomicAdd(s_tail, 1);
        items[3 * pos] = S[c];
        items[3 * pos + 1] = slot;
        items[3 * pos + 2] = dep + 1;
      }
    } else {
      for (int k = 0; k < 3; ++k) { nd.lo[k][c] = INFINITY; nd.hi[k][c] = -INFINITY; }
      nd.child[c] = kEmpty;
    }
  }
  nodes[nb + w] = nd;
}

template <int W>
__global__ __launch_bounds__(kMeshBlock) void k_collapse(BuildArgs a, const int64_t* node_base_scan) {
  __shared__ int32_t s_used, s_tail, s_depth, s_over;
  if (*a.status != INT_MAX) return;  // invalid input: the blob is not built
  Node<W>* nodes = reinterpret_cast<Node<W>*>(a.tnodes);
  for (int64_t mi = blockIdx.x; mi < a.n_meshes; mi += gridDim.x) {
    const int64_t m = a.morder[mi];
    const int n = a.mesh[m].n_tris;
    const int64_t fbase = a.face_off[m];
    const int64_t nb = node_base_scan[m];
    const int64_t bound = node_base_scan[m + 1] - nb;
    if (n == 0) {
      if (threadIdx.x == 0) {
        a.mesh[m].root = kEmpty;
        a.mesh[m].n_nodes = 0;
        a.mesh[m].node_base = (int32_t)nb;
      }
      continue;
    }
    if (n <= a.leaf) {
      if (threadIdx.x == 0) {
        const MeshDesc d = a.mesh[m];
        Node<W> nd;
        for (int c = 0; c < W; ++c) {
          for (int k = 0; k < 3; ++k) { nd.lo[k][c] = INFINITY; nd.hi[k][c] = -INFINITY; }
          nd.child[c] = kEmpty;
          nd.pad[c] = 0;
        }
        for (int k = 0; k < 3; ++k) { nd.lo[k][0] = d.box[k]; nd.hi[k][0] = d.box[3 + k]; }
        nd.child[0] = leaf_ref((int32_t)fbase, n);
        nodes[nb] = nd;
        a.mesh[m].node_base = (int32_t)nb;
        a.mesh[m].root = (int32_t)nb;
        a.mesh[m].n_nodes = 1;
        a.mesh[m].depth = 1;
      }
      continue;
    }
    int32_t* items = a.stk + 3 * fbase;
    if (threadIdx.x == 0) {
      items[0] = (int32_t)fbase;  // binary root: internal node 0 of the mesh
      items[1] = 0;
      items[2] = 1;
      s_used = 1;
      s_tail = 1;
      s_depth = 1;
      s_over = 0;
    }
    __syncthreads();
    int head = 0;
    for (;;) {
      const int tail = s_tail;
      __syncthreads();  // every thread has the level's end before items are appended
      if (head >= tail) break;
      for (int it = head + (int)threadIdx.x; it < tail; it += (int)blockDim.x)
        collapse_item<W>(a, nodes, nb, bound, items, it, &s_used, &s_tail, &s_depth, &s_over);
      head = tail;
      __syncthreads();  // the next level's items are written
    }
    if (threadIdx.x == 0) {
      if (s_over || s_depth > kMaxDepth) atomicMin(a.status, (int32_t)fbase);
      a.mesh[m].node_base = (int32_t)nb;
      a.mesh[m].root = (int32_t)nb;
      a.mesh[m].n_nodes = s_used < bound ? s_used : (int32_t)bound;
      a.mesh[m].depth = s_depth;
    }
    __syncthreads();
  }
}

// Compaction: the collapse reserved nodes_bound() slots per mesh; the used
// nodes are copied to consecutive positions of the blob (internal child
// references shifted by the same amount), so a query touches a dense array.
__global__ void k_node_count(BuildArgs a) {
  int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; m < a.n_meshes; m += (int64_t)gridDim.x * blockDim.x) a.ncount[m] = a.mesh[m].n_nodes;
  if (blockIdx.x == 0 && threadIdx.x == 0) a.ncount[a.n_meshes] = 0;
}

template <int W>
__global__ void k_node_copy(BuildArgs a, const int64_t* new_base) {
  if (*a.status != INT_MAX) return;  // invalid input: the blob is not built
  const Node<W>* src = reinterpret_cast<const Node<W>*>(a.tnodes);
  Node<W>* dst = reinterpret_cast<Node<W>*>(a.nodes);
  for (int64_t mi = blockIdx.x; mi < a.n_meshes; mi += gridDim.x) {
    const int64_t m = a.morder[mi];
    const int32_t old_base = a.mesh[m].node_base;
    const int32_t n = a.mesh[m].n_nodes;
    const int64_t nb = new_base[m];
    const int32_t shift = (int32_t)(nb - old_base);
    for (int32_t k = threadIdx.x; k < n; k += blockDim.x) {
      Node<W> nd = src[old_base + k];
      for (int c = 0; c < W; ++c)
        if (nd.child[c] >= 0 && nd.child[c] != kEmpty) nd.child[c] += shift;
      dst[nb + k] = nd;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      a.mesh[m].node_base = (int32_t)nb;
      a.mesh[m].root = n > 0 ? (int32_t)nb : kEmpty;
    }
  }
}

// ---- leaf-order triangles ----------------------------------------------------

__global__ void k_write_tris(BuildArgs a) {
  if (*a.status != INT_MAX) return;  // invalid input: the blob is not built
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; g < a.f_total; g += (int64_t)gridDim.x * blockDim.x) {
    int32_t f = a.val1[g];
    int32_t m = a.face_mesh[f];
    bool mok = a.mesh_ok[m];
    int64_t v0 = mok ? a.vert_off[m] : 0, nv = mok ? a.vert_off[m + 1] - v0 : 0;
    float* t = a.tris + 9 * g;
    for (int k = 0; k < 3; ++k) {
      int32_t id = a.faces[3 * (int64_t)f + k];
      f3 p{0.f, 0.f, 0.f};
      if (id >= 0 && id < nv) p = load_v(a.verts, v0 + id);  // invalid input: status already set
      t[3 * k] = p.x; t[3 * k + 1] = p.y; t[3 * k + 2] = p.z;
    }
    a.triid[g] = (int32_t)(f - (mok ? a.face_off[m] : 0));
  }
}

// ---- step 6: unique edges --------------------------------------------------------

__global__ void k_edge_keys(BuildArgs a) {
  if (*a.status != INT_MAX) return;  // invalid input: the blob is not built
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; f < a.f_total; f += (int64_t)gridDim.x * blockDim.x) {
    int32_t m = a.face_mesh[f];
    bool mok = a.mesh_ok[m];
    int64_t v0 = mok ? a.vert_off[m] : 0, nv = mok ? a.vert_off[m + 1] - v0 : 0;
    for (int k = 0; k < 3; ++k) {
      int32_t i0 = a.faces[3 * f + k], i1 = a.faces[3 * f + (k + 1) % 3];
      // invalid ids become a self-loop on vertex 0 of the dataset, which is dropped
      if (i0 < 0 || i0 >= nv || i1 < 0 || i1 >= nv) { a.ekey0[3 * f + k] = 0; continue; }
      uint64_t u = (uint64_t)(v0 + i0), v = (uint64_t)(v0 + i1);
      uint64_t lo = u < v ? u : v, hi = u < v ? v : u;
      a.ekey0[3 * f + k] = (lo << 32) | hi;
    }
  }
}

__global__ void k_edge_flag(BuildArgs a, const uint64_t* keys, int64_t n) {
  if (*a.status != INT_MAX) return;  // invalid input: the blob is not built
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t k = keys[i];
    bool first = (i == 0 || keys[i - 1] != k) && ((k >> 32) != (k & 0xffffffffu));
    a.eflag[i] = first ? 1 : 0;
  }
}

__device__ __forceinline__ int32_t mesh_of_vertex(const int64_t* vert_off, int64_t n_meshes, int64_t v) {
  int64_t lo = 0, hi = n_meshes;  // vert_off[lo] <= v < vert_off[hi]
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (vert_off[mid] <= v) lo = mid; else hi = mid;
  }
  return (int32_t)lo;
}

// compacts unique keys and builds the (mesh, midpoint Morton) sort keys;
// keys is the sorted raw key array, output goes to ekey0/eval0
__global__ void k_edge_compact(BuildArgs a, const uint64_t* keys, int64_t n) {
  if (*a.status != INT_MAX) return;  // invalid input: the blob is not built
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int32_t total = a.epos[n];
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (a.eflag[i]) {
      int32_t e = a.epos[i];
      uint64_t k = keys[i];
      int64_t u = (int64_t)(k >> 32), v = (int64_t)(k & 0xffffffffu);
      int32_t m = mesh_of_vertex(a.vert_off, a.n_meshes, u);
      f3 p = load_v(a.verts, u), q = load_v(a.verts, v);
      f3 mid{0.5f * (p.x + q.x), 0.5f * (p.y + q.y), 0.5f * (p.z + q.z)};
      a.ekey0[e] = ((uint64_t)(uint32_t)m << kMortonBits) | morton3(mid, a.mesh[m].box);
      a.eval0[e] = (int32_t)i;
    }
    if (i >= total) {
      a.ekey0[i] = ~0ull;
      a.eval0[i] = -1;
    }
  }
}

__global__ void k_edge_ranges(BuildArgs a, const uint64_t* skeys, int64_t n) {
  if (*a.status != INT_MAX) return;  // invalid input: the blob is not built
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t total = a.epos[n];
  for (; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int32_t m = (int32_t)(skeys[e] >> kMortonBits);
    if (e == 0 || (int32_t)(skeys[e - 1] >> kMortonBits) != m) a.estart[m] = (int32_t)e;
    if (e == total - 1 || (int32_t)(skeys[e + 1] >> kMortonBits) != m) a.eend[m] = (int32_t)(e + 1);
  }
}

__global__ void k_chunk_counts(BuildArgs a) {
  if (*a.status != INT_MAX) return;  // invalid input: the blob is not built
  int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; m < a.n_meshes; m += (int64_t)gridDim.x * blockDim.x) {
    int32_t ne = a.eend[m] - a.estart[m];
    a.mesh[m].n_edges = ne;
    a.cscan[m] = (ne + kChunk - 1) / kChunk;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.cscan[a.n_meshes] = 0;
}

__global__ void k_write_segs(BuildArgs a, const int64_t* chunk_scan, const uint64_t* ukeys,
                             const int32_t* order, int64_t n) {
  if (*a.status != INT_MAX) return;  // invalid input: the blob is not built
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t total = a.epos[n];
  for (; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int32_t src = order[e];  // index into the sorted raw key array
    uint64_t k = ukeys[src];
    int64_t u = (int64_t)(k >> 32), v = (int64_t)(k & 0xffffffffu);
    int32_t m = mesh_of_vertex(a.vert_off, a.n_meshes, u);
    int32_t local = (int32_t)(e - a.estart[m]);
    int64_t chunk = chunk_scan[m] + local / kChunk;
    int lane = local % kChunk;
    if (chunk >= a.chunk_cap) { atomicMin(a.status, 0); continue; }
    f3 p = load_v(a.verts, u), q = load_v(a.verts, v);
    float* s = a.seg + chunk * (6 * kChunk);
    s[0 * kChunk + lane] = p.x; s[1 * kChunk + lane] = p.y; s[2 * kChunk + lane] = p.z;
    s[3 * kChunk + lane] = q.x; s[4 * kChunk + lane] = q.y; s[5 * kChunk + lane] = q.z;
    int32_t* ed = a.edge + chunk * (2 * kChunk);
    int64_t v0 = a.vert_off[m];
    ed[lane] = (int32_t)(u - v0);
    ed[kChunk + lane] = (int32_t)(v - v0);
    if (lane == 0) a.cmesh[chunk] = m;
  }
}

__global__ void k_mesh_chunks(BuildArgs a, const int64_t* chunk_scan) {
  if (*a.status != INT_MAX) return;  // invalid input: the blob is not built
  int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; m < a.n_meshes; m += (int64_t)gridDim.x * blockDim.x) {
    a.mesh[m].chunk_base = (int32_t)chunk_scan[m];
    a.mesh[m].n_chunks = (int32_t)(chunk_scan[m + 1] - chunk_scan[m]);
  }
}

// one wavefront per group: exact box of the live segments' endpoints
__global__ void k_chunk_box(BuildArgs a, const int64_t* chunk_scan) {
  if (*a.status != INT_MAX) return;  // invalid input: the blob is not built
  int64_t total = chunk_scan[a.n_meshes];
  int lane = threadIdx.x & 63;
  int64_t c = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  int64_t stride = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (; c < total; c += stride) {
    int32_t m = a.cmesh[c];
    int32_t local0 = (int32_t)(c - a.mesh[m].chunk_base) * kChunk;
    bool live = local0 + lane < a.mesh[m].n_edges;
    const float* s = a.seg + c * (6 * kChunk);
    float lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
      float pv = live ? s[k * kChunk + lane] : INFINITY;
      float qv = live ? s[(3 + k) * kChunk + lane] : INFINITY;
      lo[k] = fminf(pv, qv);
      pv = live ? s[k * kChunk + lane] : -INFINITY;
      qv = live ? s[(3 + k) * kChunk + lane] : -INFINITY;
      hi[k] = fmaxf(pv, qv);
      for (int o = 32; o > 0; o >>= 1) {
        lo[k] = fminf(lo[k], __shfl_xor(lo[k], o));
        hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], o));
      }
    }
    if (lane == 0) {
      float* b = a.cbox + 8 * c;
      for (int k = 0; k < 3; ++k) { b[k] = lo[k]; b[3 + k] = hi[k]; }
      b[6] = 0.f; b[7] = 0.f;
    }
  }
}

// Run boxes: the box of each run of 64 consecutive groups of a mesh, stored
// at the run's first group, so that the cull can skip 64 groups with one test.
__global__ void k_run_box(BuildArgs a, const int64_t* chunk_scan) {
  if (*a.status != INT_MAX) return;
  const int64_t total = chunk_scan[a.n_meshes];
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < total; c += (int64_t)gridDim.x * blockDim.x) {
    const int32_t m = a.cmesh[c];
    const int64_t c0 = a.mesh[m].chunk_base, c1 = c0 + a.mesh[m].n_chunks;
    if ((c - c0) % kChunk != 0) continue;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int64_t e = c + kChunk < c1 ? c + kChunk : c1;
    for (int64_t g = c; g < e; ++g) {
      const float* b = a.cbox + 8 * g;
      for (int k = 0; k < 3; ++k) { lo[k] = fminf(lo[k], b[k]); hi[k] = fmaxf(hi[k], b[3 + k]); }
    }
    float* r = a.rbox + 8 * c;
    for (int k = 0; k < 3; ++k) { r[k] = lo[k]; r[3 + k] = hi[k]; }
    r[6] = 0.f; r[7] = 0.f;
  }
}

__global__ void k_header(BuildArgs a, BlobHeader h, const int64_t* chunk_scan, int64_t n3) {
  h.n_chunks = a.f_total > 0 ? chunk_scan[a.n_meshes] : 0;
  h.n_edges = a.f_total > 0 ? a.epos[n3] : 0;
  h.exp_lo = a.meshctr[0];
  h.exp_hi = a.meshctr[1];
  *reinterpret_cast<BlobHeader*>(a.blob) = h;
}

__global__ void k_status_out(const int32_t* st, int32_t* out) {
  int32_t s = *st;
  *out = (s == INT_MAX) ? -1 : s;
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// ---- sizes ------------------------------------------------------------------

struct Layout {
  int64_t node_cap, chunk_cap;
  int64_t off_mesh, off_node, off_tri, off_triid, off_seg, off_edge, off_cbox, off_cmesh, off_rep, off_rbox, total;
};

Layout blob_layout(int64_t M, int64_t F, int W, int L) {
  Layout y;
  y.node_cap = F / (W - 1) + F / (L + 1) + 2 * M + 1;
  y.chunk_cap = (3 * F) / kChunk + M + 1;
  int64_t o = align256(sizeof(BlobHeader));
  y.off_mesh = o; o = align256(o + M * (int64_t)sizeof(MeshDesc));
  y.off_node = o; o = align256(o + y.node_cap * node_bytes(W));
  // three triangles of slack after the last one: a leaf's triangles are
  // read four at a time as one contiguous block
  y.off_tri = o; o = align256(o + (F + 3) * 36);
  y.off_triid = o; o = align256(o + F * 4);
  y.off_seg = o; o = align256(o + y.chunk_cap * 6 * kChunk * 4);
  y.off_edge = o; o = align256(o + y.chunk_cap * 2 * kChunk * 4);
  y.off_cbox = o; o = align256(o + y.chunk_cap * 32);
  y.off_cmesh = o; o = align256(o + y.chunk_cap * 4);
  y.off_rep = o; o = align256(o + M * 16);
  y.off_rbox = o; o = align256(o + y.chunk_cap * 32);
  y.total = o;
  return y;
}

int end_bit_for(int64_t M) {
  int b = 1;
  while (((int64_t)1 << b) <= M) ++b;  // M <= 2^b - 1, so ids < 2^b - 1
  return kMortonBits + b;
}

// Carves the workspace; with base == nullptr only measures.  Sort temp sizes
// are queried from hipCUB.
int carve_ws(Carve& cv, BuildArgs& a, int64_t M, int64_t F, int64_t node_cap, int W, void** sort_tmp,
             size_t* sort_bytes) {
  int64_t E3 = 3 * F;
  a.status = cv.take<int32_t>(4);
  a.meshctr = cv.take<int32_t>(4);
  a.face_mesh = cv.take<int32_t>(F);
  a.tbox = cv.take<float>(6 * F);
  a.fsafe = cv.take<uint8_t>(F);
  a.key0 = cv.take<uint64_t>(F);
  a.key1 = cv.take<uint64_t>(F);
  a.val0 = cv.take<int32_t>(F);
  a.val1 = cv.take<int32_t>(F);
  a.left = cv.take<int32_t>(F);
  a.right = cv.take<int32_t>(F);
  a.parent = cv.take<int32_t>(F);
  a.lparent = cv.take<int32_t>(F);
  a.nbox = cv.take<float>(6 * F);
  a.nleaf = cv.take<int32_t>(F);
  a.nfirst = cv.take<int32_t>(F);
  a.visit = cv.take<uint32_t>(F);
  a.nbound = cv.take<int64_t>(M + 1);
  a.stk = cv.take<int32_t>(3 * F);
  a.ekey0 = cv.take<uint64_t>(E3);
  a.ekey1 = cv.take<uint64_t>(E3);
  a.eval0 = cv.take<int32_t>(E3);
  a.eval1 = cv.take<int32_t>(E3);
  a.eflag = cv.take<int32_t>(E3 + 1);
  a.epos = cv.take<int32_t>(E3 + 1);
  a.estart = cv.take<int32_t>(M);
  a.eend = cv.take<int32_t>(M);
  a.cscan = cv.take<int64_t>(M + 1);
  a.mesh_ok = cv.take<uint8_t>(M);
  a.ekey2 = cv.take<uint64_t>(E3);
  a.nscan = cv.take<int64_t>(M + 1);
  a.chunk_scan = cv.take<int64_t>(M + 1);
  a.ncount = cv.take<int64_t>(M + 1);
  a.tsum = cv.take<int64_t>(scan_tiles_of((E3 > M ? E3 : M) + 1) + 1);
  a.morder = cv.take<int32_t>(M);
  a.mcnt = cv.take<int32_t>(kSizeClasses * ((M + kMeshOrdTile - 1) / kMeshOrdTile));
  a.mpos = cv.take<int64_t>(kSizeClasses * ((M + kMeshOrdTile - 1) / kMeshOrdTile));
  a.tnodes = cv.take<char>(node_cap * node_bytes(W));
  // temp storage for the library sorts
  size_t need = 0, b = 0;
  int eb = end_bit_for(M);
  hipError_t e;
  e = hipcub::DeviceRadixSort::SortPairs(nullptr, b, (uint64_t*)nullptr, (uint64_t*)nullptr, (int32_t*)nullptr,
                                         (int32_t*)nullptr, (int)(F > 0 ? F : 1), 0, eb);
  if (e != hipSuccess) return hip_fail(e, "hipcub SortPairs size");
  need = need > b ? need : b;
  e = hipcub::DeviceRadixSort::SortKeys(nullptr, b, (uint64_t*)nullptr, (uint64_t*)nullptr, (int)(E3 > 0 ? E3 : 1), 0, 64);
  if (e != hipSuccess) return hip_fail(e, "hipcub SortKeys size");
  need = need > b ? need : b;
  e = hipcub::DeviceRadixSort::SortPairs(nullptr, b, (uint64_t*)nullptr, (uint64_t*)nullptr, (int32_t*)nullptr,
                                         (int32_t*)nullptr, (int)(E3 > 0 ? E3 : 1), 0, eb);
  if (e != hipSuccess) return hip_fail(e, "hipcub SortPairs size");
  need = need > b ? need : b;
  *sort_bytes = need;
  *sort_tmp = cv.take<char>((int64_t)need);
  return PR_OK;
}

int check_params(int64_t M, int64_t F, int64_t V, const pr_bvh_params* p) {
  if (!p) { set_error("params is NULL"); return PR_E_ARG; }
  if (!(p->width == 2 || p->width == 4 || p->width == 8)) { set_error("width must be 2, 4 or 8"); return PR_E_ARG; }
  if (!(p->leaf_size == 1 || p->leaf_size == 2 || p->leaf_size == 4 || p->leaf_size == 8)) {
    set_error("leaf_size must be 1, 2, 4 or 8");
    return PR_E_ARG;
  }
  if (p->builder < 0 || p->builder > 1) { set_error("builder must be 0 or 1"); return PR_E_ARG; }
  if (p->reserved != 0) { set_error("reserved must be 0"); return PR_E_ARG; }
  if (M < 0 || F < 0 || V < 0) { set_error("negative size"); return PR_E_ARG; }
  if (M == 0 && (F > 0 || V > 0)) { set_error("faces or vertices without meshes"); return PR_E_ARG; }
  if (F >= ((int64_t)1 << 28) || V >= ((int64_t)1 << 31) || M >= ((int64_t)1 << 24)) {
    set_error("sizes beyond index ranges (f_total < 2^28, v_total < 2^31, n_meshes < 2^24)");
    return PR_E_UNSUPPORTED;
  }
  return PR_OK;
}

}  // namespace
}  // namespace pr

using namespace pr;

extern "C" int build_mesh_bvh_sizes(int64_t n_meshes, int64_t f_total, int64_t v_total,
                                    const pr_bvh_params* params, size_t* blob_bytes, size_t* ws_bytes) {
  int r = check_params(n_meshes, f_total, v_total, params);
  if (r) return r;
  if (!blob_bytes || !ws_bytes) { set_error("output pointer is NULL"); return PR_E_ARG; }
  Layout y = blob_layout(n_meshes, f_total, params->width, params->leaf_size);
  *blob_bytes = (size_t)y.total;
  Carve cv{nullptr, 0};
  BuildArgs a{};
  void* tmp;
  size_t tb;
  Layout y0 = blob_layout(n_meshes, f_total, params->width, params->leaf_size);
  r = carve_ws(cv, a, n_meshes, f_total, y0.node_cap, params->width, &tmp, &tb);
  if (r) return r;
  *ws_bytes = cv.used + 256;
  return PR_OK;
}

extern "C" size_t build_mesh_bvh_bytes(int64_t n_meshes, int64_t f_total, int64_t v_total,
                                       const pr_bvh_params* params) {
  if (check_params(n_meshes, f_total, v_total, params) != PR_OK) return 0;
  return (size_t)blob_layout(n_meshes, f_total, params->width, params->leaf_size).total;
}

extern "C" int build_mesh_bvh(const float* verts, const int64_t* vert_off, const int32_t* faces,
                              const int64_t* face_off, int64_t n_meshes, int64_t v_total, int64_t f_total,
                              const pr_bvh_params* params, void* blob, size_t blob_bytes, void* ws,
                              size_t ws_bytes, int32_t* dev_status, void* stream) {
  int r = check_params(n_meshes, f_total, v_total, params);
  if (r) return r;
  if (!blob || !ws || !dev_status || !vert_off || !face_off || (f_total > 0 && (!faces || !verts))) {
    set_error("null pointer argument");
    return PR_E_ARG;
  }
  const int W = params->width, L = params->leaf_size;
  Layout y = blob_layout(n_meshes, f_total, W, L);
  if (blob_bytes < (size_t)y.total) { set_error("blob_bytes %zu < required %lld", blob_bytes, (long long)y.total); return PR_E_CAPACITY; }
  hipStream_t s = (hipStream_t)stream;
  BuildArgs a{};
  Carve cv{(char*)ws, ws_bytes};
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  r = carve_ws(cv, a, n_meshes, f_total, y.node_cap, W, &tmp, &tmp_bytes);
  if (r) return r;
  if (cv.used > ws_bytes || !tmp) { set_error("ws_bytes %zu < required %zu", ws_bytes, cv.used); return PR_E_CAPACITY; }
  a.verts = verts; a.vert_off = vert_off; a.faces = faces; a.face_off = face_off;
  a.n_meshes = n_meshes; a.v_total = v_total; a.f_total = f_total; a.width = W; a.leaf = L;
  a.builder = params->builder;
  a.blob = (char*)blob;
  a.mesh = reinterpret_cast<MeshDesc*>(a.blob + y.off_mesh);
  a.nodes = a.blob + y.off_node;
  a.tris = reinterpret_cast<float*>(a.blob + y.off_tri);
  a.triid = reinterpret_cast<int32_t*>(a.blob + y.off_triid);
  a.seg = reinterpret_cast<float*>(a.blob + y.off_seg);
  a.edge = reinterpret_cast<int32_t*>(a.blob + y.off_edge);
  a.cbox = reinterpret_cast<float*>(a.blob + y.off_cbox);
  a.cmesh = reinterpret_cast<int32_t*>(a.blob + y.off_cmesh);
  a.rep = reinterpret_cast<float*>(a.blob + y.off_rep);
  a.rbox = reinterpret_cast<float*>(a.blob + y.off_rbox);
  a.node_cap = y.node_cap;
  a.chunk_cap = y.chunk_cap;

  const int64_t F = f_total, M = n_meshes, E3 = 3 * F;
  const int gF = grid_for(F, kBlock), gM = grid_for(M, kBlock), gE = grid_for(E3, kBlock);
  int eb = end_bit_for(M);

  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, a.status, 1, INT_MAX);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, a.meshctr + 0, 1, INT_MAX);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, a.meshctr + 1, 1, INT_MIN);
  if (M > 0) {
    hipLaunchKernelGGL(k_fill_i32, dim3(gM), dim3(kBlock), 0, s, a.estart, M, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(gM), dim3(kBlock), 0, s, a.eend, M, 0);
    if (F > 0) hipLaunchKernelGGL(k_fill_i32, dim3(gF), dim3(kBlock), 0, s, a.face_mesh, F, 0);
    hipLaunchKernelGGL(k_face_mesh, dim3((int)(M < 65536 ? M : 65536)), dim3(kBlock), 0, s, a);
  }
  if (F > 0) {
    hipLaunchKernelGGL(k_fill_u32, dim3(gF), dim3(kBlock), 0, s, a.visit, F, 0u);
    hipLaunchKernelGGL(k_tri_prep, dim3(gF < 4096 ? gF : 4096), dim3(kBlock), 0, s, a);
  }
  if (M > 0) hipLaunchKernelGGL(k_mesh_box, dim3((int)(M < 65536 ? M : 65536)), dim3(kBlock), 0, s, a);
  if (M > 0) {
    // the per-mesh kernels below take the meshes largest first
    const int64_t nbm = (M + kMeshOrdTile - 1) / kMeshOrdTile;
    hipLaunchKernelGGL(k_mesh_order_count, dim3((unsigned)nbm), dim3(256), 0, s, a, nbm);
    PR_HIP(device_exclusive_scan((const int32_t*)a.mcnt, a.mpos, kSizeClasses * nbm, a.tsum, (int64_t*)nullptr, s));
    hipLaunchKernelGGL(k_mesh_order_place, dim3((unsigned)nbm), dim3(256), 0, s, a, nbm);
  }
  if (F > 0) {
    hipLaunchKernelGGL(k_morton, dim3(gF), dim3(kBlock), 0, s, a);
    PR_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, a.key0, a.key1, a.val0, a.val1, (int)F, 0, eb, s));
    hipLaunchKernelGGL(k_karras, dim3(gF), dim3(kBlock), 0, s, a, (const uint64_t*)a.key1);
    hipLaunchKernelGGL(k_refit, dim3((int)(M < 65536 ? M : 65536)), dim3(kMeshBlock), 0, s, a, (const int32_t*)a.val1);
  }
  if (M > 0) {
    hipLaunchKernelGGL(k_node_bound, dim3(gM), dim3(kBlock), 0, s, a);
    PR_HIP(device_exclusive_scan((const int64_t*)a.nbound, a.nscan, M + 1, a.tsum, (int64_t*)nullptr, s));
    const int gC = (int)(M < 65536 ? M : 65536);  // one block per mesh
    if (W == 2) hipLaunchKernelGGL(k_collapse<2>, dim3(gC), dim3(kMeshBlock), 0, s, a, (const int64_t*)a.nscan);
    else if (W == 4) hipLaunchKernelGGL(k_collapse<4>, dim3(gC), dim3(kMeshBlock), 0, s, a, (const int64_t*)a.nscan);
    else hipLaunchKernelGGL(k_collapse<8>, dim3(gC), dim3(kMeshBlock), 0, s, a, (const int64_t*)a.nscan);
    hipLaunchKernelGGL(k_node_count, dim3(gM), dim3(kBlock), 0, s, a);
    PR_HIP(device_exclusive_scan((const int64_t*)a.ncount, a.nbound, M + 1, a.tsum, (int64_t*)nullptr, s));
    const int gMB = (int)(M < 65536 ? M : 65536);
    if (W == 2) hipLaunchKernelGGL(k_node_copy<2>, dim3(gMB), dim3(kBlock), 0, s, a, (const int64_t*)a.nbound);
    else if (W == 4) hipLaunchKernelGGL(k_node_copy<4>, dim3(gMB), dim3(kBlock), 0, s, a, (const int64_t*)a.nbound);
    else hipLaunchKernelGGL(k_node_copy<8>, dim3(gMB), dim3(kBlock), 0, s, a, (const int64_t*)a.nbound);
  }
  if (F > 0) {
    hipLaunchKernelGGL(k_write_tris, dim3(gF), dim3(kBlock), 0, s, a);
    // unique edges: raw keys -> sorted (ekey1) -> flags/positions -> (mesh, Morton) keys (ekey0)
    hipLaunchKernelGGL(k_edge_keys, dim3(gF), dim3(kBlock), 0, s, a);
    PR_HIP(hipcub::DeviceRadixSort::SortKeys(tmp, tmp_bytes, a.ekey0, a.ekey1, (int)E3, 0, 64, s));
    hipLaunchKernelGGL(k_edge_flag, dim3(gE), dim3(kBlock), 0, s, a, (const uint64_t*)a.ekey1, E3);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, a.eflag + E3, 1, 0);
    PR_HIP(device_exclusive_scan((const int32_t*)a.eflag, a.epos, E3 + 1, a.tsum, (int64_t*)nullptr, s));
    hipLaunchKernelGGL(k_edge_compact, dim3(gE), dim3(kBlock), 0, s, a, (const uint64_t*)a.ekey1, E3);
    PR_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, a.ekey0, a.ekey2, a.eval0, a.eval1, (int)E3, 0, eb, s));
    hipLaunchKernelGGL(k_edge_ranges, dim3(gE), dim3(kBlock), 0, s, a, (const uint64_t*)a.ekey2, E3);
  }
  if (M > 0) {
    hipLaunchKernelGGL(k_chunk_counts, dim3(gM), dim3(kBlock), 0, s, a);
    PR_HIP(device_exclusive_scan((const int64_t*)a.cscan, a.chunk_scan, M + 1, a.tsum, (int64_t*)nullptr, s));
    hipLaunchKernelGGL(k_mesh_chunks, dim3(gM), dim3(kBlock), 0, s, a, (const int64_t*)a.chunk_scan);
  }
  if (F > 0) {
    hipLaunchKernelGGL(k_write_segs, dim3(gE), dim3(kBlock), 0, s, a, (const int64_t*)a.chunk_scan,
                       (const uint64_t*)a.ekey1, (const int32_t*)a.eval1, E3);
    hipLaunchKernelGGL(k_chunk_box, dim3(grid_for(a.chunk_cap * 64, kBlock)), dim3(kBlock), 0, s, a,
                       (const int64_t*)a.chunk_scan);
    hipLaunchKernelGGL(k_run_box, dim3(grid_for(a.chunk_cap, kBlock)), dim3(kBlock), 0, s, a,
                       (const int64_t*)a.chunk_scan);
  }
  BlobHeader h{};
  h.magic = kMagic;
  h.version = PR_ABI_VERSION;
  h.width = W;
  h.leaf_size = L;
  h.n_meshes = M;
  h.f_total = F;
  h.v_total = v_total;
  h.node_cap = y.node_cap;
  h.chunk_cap = y.chunk_cap;
  h.off_mesh = y.off_mesh;
  h.off_node = y.off_node;
  h.off_tri = y.off_tri;
  h.off_triid = y.off_triid;
  h.off_seg = y.off_seg;
  h.off_edge = y.off_edge;
  h.off_cbox = y.off_cbox;
  h.off_cmesh = y.off_cmesh;
  h.off_rep = y.off_rep;
  h.off_rbox = y.off_rbox;
  h.total_bytes = y.total;
  hipLaunchKernelGGL(k_header, dim3(1), dim3(1), 0, s, a, h, (const int64_t*)a.chunk_scan, E3);
  hipLaunchKernelGGL(k_status_out, dim3(1), dim3(1), 0, s, (const int32_t*)a.status, dev_status);
  PR_HIP(hipGetLastError());
  return PR_OK;
}
