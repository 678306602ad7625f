// Internal definitions shared by the library's HIP sources: blob layout,
// launch helpers and error reporting.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/pierce.h"

namespace pr {

constexpr uint32_t kMagic = 0x31425250u;  // "PRB1"
constexpr int kChunk = 64;                // segments per group (one wavefront)
constexpr int kMaxDepth = 64;             // BVH depth bound enforced by the build
constexpr int32_t kEmpty = 0x7fffffff;    // empty child slot
constexpr int kMortonBits = 30;           // 10 bits per axis

// Every coordinate of an "FP32-safe" mesh is 0 or has magnitude in
// [2^-40, 2^40]; the FP32 error bounds of the traversal assume it.
constexpr float kSafeLo = 0x1p-40f;
constexpr float kSafeHi = 0x1p40f;

// Blob header (first 256 bytes of every blob).  Offsets are in bytes from the
// blob start; every section starts on a 256-byte boundary.
struct BlobHeader {
  uint32_t magic;
  uint32_t version;
  int32_t width;
  int32_t leaf_size;
  int64_t n_meshes;
  int64_t f_total;
  int64_t v_total;
  int64_t node_cap;   // wide nodes reserved
  int64_t chunk_cap;  // 64-segment groups reserved
  int64_t off_mesh;   // MeshDesc[n_meshes]
  int64_t off_node;   // node_cap nodes of node_bytes(width); per mesh the root comes first and its
                      // internal children follow it, in child order
  int64_t off_tri;    // f32[f_total][9], leaf order
  int64_t off_triid;  // i32[f_total]: mesh-local face index of each leaf-order triangle
  int64_t off_seg;    // f32[chunk_cap][6][64]: segment endpoints p.xyz, q.xyz, lane-minor
  int64_t off_edge;   // i32[chunk_cap][2][64]: mesh-local vertex ids of each segment
  int64_t off_cbox;   // f32[chunk_cap][8]: box of each group's endpoints (lo3, hi3, pad2)
  int64_t off_cmesh;  // i32[chunk_cap]: mesh of each group
  int64_t total_bytes;
  int64_t n_chunks;   // groups in use (written by the build)
  int64_t n_edges;    // unique edges in use (written by the build)
  int32_t exp_lo;     // lowest exponent of a set bit over every non-zero coordinate of a face
  int32_t exp_hi;     // highest such exponent (every |coordinate| < 2^(exp_hi + 1))
  int64_t off_rep;    // f32[n_meshes][4]: first corner of each mesh's first face (input order), w = 1;
                      // w = 0 for a mesh without faces
  int64_t off_rbox;   // f32[chunk_cap][8]: at the first group of each run of 64 groups of a mesh
                      // (group - chunk_base a multiple of 64), the box of the run's groups
  int64_t reserved[11];
};
static_assert(sizeof(BlobHeader) == 256, "header size");

// Per-mesh descriptor (64 bytes).
struct MeshDesc {
  float box[6];        // exact box of the mesh's triangles: lo xyz, hi xyz
  int32_t node_base;   // index of the root node in the node array
  int32_t n_nodes;     // nodes in use
  int32_t tri_base;    // first leaf-order triangle (= first face of the mesh)
  int32_t n_tris;
  int32_t chunk_base;  // first 64-segment group
  int32_t n_chunks;
  int32_t n_edges;     // unique edges
  int32_t depth;       // node levels on the longest root-to-leaf path
  int32_t root;        // node index of the root, or kEmpty for an empty mesh
  int32_t flags;       // bit 0: all coordinates FP32-safe
};
static_assert(sizeof(MeshDesc) == 64, "mesh desc size");

constexpr int32_t kMeshSafe = 1;

// A node of width W: child boxes in structure-of-arrays order, then child
// references.  child >= 0: node index; child == kEmpty: unused slot;
// child < 0: leaf, ~child = first_triangle << 3 | (count - 1).
template <int W>
struct Node {
  float lo[3][W];
  float hi[3][W];
  int32_t child[W];
  int32_t pad[W];
};
static_assert(sizeof(Node<4>) == 128, "node size");

__host__ __device__ inline int64_t node_bytes(int w) { return 32 * (int64_t)w; }

__host__ __device__ inline int32_t leaf_ref(int32_t first, int32_t count) {
  return ~((first << 3) | (count - 1));
}

// Wide nodes that the build may create for a mesh of n triangles: full nodes
// consume W-1 binary nodes of more than L triangles, partial nodes own
// disjoint subtrees of more than L triangles.
__host__ __device__ inline int64_t nodes_bound(int64_t n, int w, int l) {
  if (n <= 0) return 0;
  if (n <= l) return 1;
  return (n - 1) / (w - 1) + n / (l + 1) + 2;
}

__host__ __device__ inline int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// Library-wide error state.
void set_error(const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

// Data that no kernel writes while it is read (blob contents, filter
// inputs) is read through the constant address space, so that uniform reads
// go through the scalar cache into SGPRs.
template <class T>
using cptr_t = const __attribute__((address_space(4))) T*;

template <class T>
__device__ __forceinline__ cptr_t<T> cview(const T* p) {
  return (cptr_t<T>)(reinterpret_cast<uintptr_t>(p));
}

#define PR_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return pr::hip_fail(e_, #call); \
  } while (0)

// Bump allocator over a caller-provided workspace.
struct Carve {
  char* base;
  size_t cap;
  size_t used = 0;
  template <typename T>
  T* take(int64_t n) {
    size_t off = (size_t)align256((int64_t)used);
    size_t need = off + sizeof(T) * (size_t)(n > 0 ? n : 0);
    used = need;
    if (base == nullptr || need > cap) return nullptr;
    return reinterpret_cast<T*>(base + off);
  }
};

inline int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > (1 << 20)) g = 1 << 20;
  return (int)g;
}

}  // namespace pr
