// inside_pairs / refine_predicate: the point-in-mesh test of the containment
// join (Section 3.3, Algorithm 2) and the containment, within and
// intersection predicates built on it (Sections 3.3 and 3.4).
//
// Work unit: one candidate pair, one thread.  A ray is the representative
// vertex v of one mesh against the other mesh's BVH: the thread walks the
// target tree along the column {(v.x, v.y, z) : z >= v.z} (the +z ray of the
// paper's parity test), counting signed crossings; it casts the rays the
// predicate needs (contains: rep(B_j) in A_i; within: rep(A_i) in B_j;
// intersection: the second only if the first is outside; raw bits: both).  The paper casts one ray
// per object against a BVH of a whole dataset and toggles a parity bit per
// hit object; here each candidate pair has its target mesh's own tree, so
// the ray meets only that mesh and a signed count per unit replaces the
// per-object parity array.
//
// The thread's stack lives in LDS, entry-major with one column per thread so
// that lanes at equal depth use distinct banks.  A pair whose stack would
// overflow is appended to a list and rerun by a second kernel whose threads
// hold a stack of the full depth bound.
//
// Crossing rule (exact on the FP32 coordinates).  The vertex is perturbed to
// v' = (x + e, y + e^2, z) for an infinitesimal e > 0 (Simulation of
// Simplicity, Edelsbrunner and Muecke 1990).  In the xy projection,
// orient2d(a, b, v') = orient2d(a, b, v) + (a.y - b.y) e + (b.x - a.x) e^2,
// so its sign is that of the first non-zero term; it is exactly
// antisymmetric in (a, b), so a column through a shared edge is counted in
// exactly one of the two triangles, and it is zero only for an edge whose
// projection is a point.  The column meets triangle (a, b, c) iff the three
// edge signs are equal and non-zero (never for a triangle whose projection
// is a segment: the three terms sum to its zero projected area); that
// common sign s is the sign of the normal's z component.  The crossing lies
// above v iff orient(a, b, c, v) = -s, and then adds s to the winding
// number.  If orient(a, b, c, v) = 0 while the column meets the triangle, v
// lies on it.  Perturbing v does not change the winding number of a point
// off the surface, because it is constant near such a point.  A vertex on
// the surface is detected separately, exactly: for every triangle whose
// closed box contains v, orient(a, b, c, v) = 0 and v inside the closed
// triangle in a coordinate plane where its projection is not degenerate.
// Orientation signs use the FP64 filter with the exact expansion fallback.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "predicates.h"

namespace pr {
namespace {

constexpr int kIB = 64;                       // threads per block, fast kernel (one wave: small
                                              // launches still reach every compute unit)
constexpr int kFastCap = 32;                  // LDS stack entries per thread there
constexpr int kDeepB = 32;                    // threads per block, deep kernel
constexpr int kDeepCap = 7 * (kMaxDepth + 1) + 1;  // W - 1 <= 7 pending siblings per level (the
                                                   // leaf level too), plus one
constexpr int kDeepGrid = 256;
constexpr int kCopies = 64;                   // statistics copies (blockIdx % kCopies)
constexpr int kStride = 512;                  // u64 words between copies

enum { I_RAYS = 0, I_BOXMISS, I_VISITS, I_TESTS, I_CROSS, I_EXACT, I_ON, I_DEEP, I_N };
static_assert(sizeof(pr_inside_stats) == I_N * 8, "stats layout");

// per-unit result codes
enum : uint8_t { U_OUT = 0, U_IN = 1, U_ON = 2 };

struct Blob {
  const MeshDesc* mesh;
  const char* nodes;
  const float* tris;
  const float4* rep;
  int32_t width;
};

__device__ __forceinline__ Blob blob_of(const char* b) {
  const BlobHeader* h = reinterpret_cast<const BlobHeader*>(b);
  Blob v;
  v.mesh = reinterpret_cast<const MeshDesc*>(b + h->off_mesh);
  v.nodes = b + h->off_node;
  v.tris = reinterpret_cast<const float*>(b + h->off_tri);
  v.rep = reinterpret_cast<const float4*>(b + h->off_rep);
  v.width = h->width;
  return v;
}

struct InsideArgs {
  const char* blob_a;
  const char* blob_b;
  int64_t n_meshes_a, n_meshes_b;
  const int32_t* pairs;
  int64_t n_pairs;
  const uint8_t* cross;       // modes 1-3: overlap flags
  uint8_t* out;
  int32_t mode;
  uint32_t* deep;             // [P] pairs rerun with the full stack
  uint32_t* ctr;              // [0] pairs in deep, [1] deep-kernel blocks finished
  unsigned long long* stats;  // kCopies copies, kStride words apart
  int32_t* status;            // [1] PR_OK or PR_E_ARG
};

struct Counts {
  uint32_t c[I_N];
};

// Sign of orient2d(a, b, v') in the xy plane for the perturbed v'.
__device__ __forceinline__ int sos2(f3 a, f3 b, f3 v, ExactCounters& ec) {
  const int o = sign_orient2d(a, b, v, 0, 1, ec);
  if (o != 0) return o;
  if (a.y != b.y) return a.y > b.y ? 1 : -1;
  if (a.x != b.x) return b.x > a.x ? 1 : -1;
  return 0;
}

// v (in the triangle's plane) lies in the closed triangle: returns
// on | exact_signs << 1 (a call, so the counters stay in registers).
__device__ __noinline__ uint32_t on_triangle(f3 a, f3 b, f3 c, f3 v) {
  ExactCounters ec{0};
  int i = 1, j = 2;
  if (sign_orient2d(a, b, c, 1, 2, ec) == 0) {
    i = 2; j = 0;
    if (sign_orient2d(a, b, c, 2, 0, ec) == 0) { i = 0; j = 1; }
  }
  const int s1 = sign_orient2d(a, b, v, i, j, ec), s2 = sign_orient2d(b, c, v, i, j, ec),
            s3 = sign_orient2d(c, a, v, i, j, ec);
  const bool on = (s1 >= 0 && s2 >= 0 && s3 >= 0) || (s1 <= 0 && s2 <= 0 && s3 <= 0);
  return (on ? 1u : 0u) | (ec.exact_signs << 1);
}

// One leaf triangle against the column above v: returns true when v lies on
// the triangle, else adds the crossing (if any) to wn.
__device__ __forceinline__ bool column_tri(const float* t, f3 v, int& wn, Counts& k) {
  const f3 a{t[0], t[1], t[2]}, b{t[3], t[4], t[5]}, c{t[6], t[7], t[8]};
  const float xlo = fminf(fminf(a.x, b.x), c.x), xhi = fmaxf(fmaxf(a.x, b.x), c.x);
  const float ylo = fminf(fminf(a.y, b.y), c.y), yhi = fmaxf(fmaxf(a.y, b.y), c.y);
  const float zlo = fminf(fminf(a.z, b.z), c.z), zhi = fmaxf(fmaxf(a.z, b.z), c.z);
  // strictly outside the closed column box, or wholly below v: no crossing
  // ahead, and v is not on the triangle
  if (v.x < xlo || v.x > xhi || v.y < ylo || v.y > yhi || v.z > zhi) return false;
  ++k.c[I_TESTS];
  ExactCounters ec{0};
  const int s1 = sos2(a, b, v, ec);
  bool meets = s1 != 0 && sos2(b, c, v, ec) == s1;
  meets = meets && sos2(c, a, v, ec) == s1;
  const bool inbox = v.z >= zlo;
  bool on = false;
  if (meets || inbox) {
    const int o3 = sign_orient3d(a, b, c, v, ec);
    if (o3 == 0) {
      if (meets) {
        on = true;
      } else {
        const uint32_t r = on_triangle(a, b, c, v);
        on = (r & 1u) != 0;
        ec.exact_signs += r >> 1;
      }
    } else if (meets && o3 == -s1) {
      wn += s1;
      ++k.c[I_CROSS];
    }
  }
  k.c[I_EXACT] += ec.exact_signs;
  return on;
}

// Winding test of v against mesh tm of T: U_OUT, U_IN, U_ON, or -1 when the
// stack (cap entries, stride apart) would overflow.
template <int W>
__device__ __forceinline__ int column_walk(const Blob& T, int32_t tm, f3 v, int32_t* stk, int stride, int cap, Counts& k) {
  const MeshDesc* md = T.mesh + tm;
  const int32_t root = md->root;
  if (root == kEmpty || md->n_tris <= 0 || !(md->box[0] <= v.x && v.x <= md->box[3] && md->box[1] <= v.y &&
                                             v.y <= md->box[4] && v.z <= md->box[5])) {
    ++k.c[I_BOXMISS];
    return U_OUT;
  }
  const Node<W>* nodes = reinterpret_cast<const Node<W>*>(T.nodes);
  int sp = 1;
  stk[0] = root;
  int wn = 0;
  // leaves are pushed like nodes, so the leaf code exists once
  while (sp > 0) {
    --sp;
    const int32_t ref = stk[sp * stride];
    if (ref < 0) {
      const int32_t lr = ~ref;
      const int32_t first = lr >> 3, cnt = (lr & 7) + 1;
      for (int t = 0; t < cnt; ++t)
        if (column_tri(T.tris + 9 * (int64_t)(first + t), v, wn, k)) {
          ++k.c[I_ON];
          return U_ON;
        }
      continue;
    }
    const Node<W>* n = nodes + ref;
    ++k.c[I_VISITS];
    // the whole node is loaded at once
    float lx[W], hx[W], ly[W], hy[W], hz[W];
    int32_t ch[W];
#pragma unroll
    for (int q = 0; q < W; ++q) {
      lx[q] = n->lo[0][q]; hx[q] = n->hi[0][q];
      ly[q] = n->lo[1][q]; hy[q] = n->hi[1][q];
      hz[q] = n->hi[2][q];
      ch[q] = n->child[q];
    }
#pragma unroll
    for (int q = 0; q < W; ++q) {
      if (ch[q] == kEmpty || !(lx[q] <= v.x && v.x <= hx[q] && ly[q] <= v.y && v.y <= hy[q] && v.z <= hz[q]))
        continue;
      if (sp == cap) return -1;
      stk[sp * stride] = ch[q];
      ++sp;
    }
  }
  return wn != 0 ? U_IN : U_OUT;
}

__device__ __forceinline__ int walk(const Blob& T, int32_t tm, f3 v, int32_t* stk, int stride, int cap,
                                    Counts& k) {
  if (T.width == 2) return column_walk<2>(T, tm, v, stk, stride, cap, k);
  if (T.width == 4) return column_walk<4>(T, tm, v, stk, stride, cap, k);
  return column_walk<8>(T, tm, v, stk, stride, cap, k);
}

// The two blobs are this library's and hold the meshes the caller names.
__device__ __forceinline__ bool blobs_ok(const InsideArgs& a) {
  const BlobHeader* ha = reinterpret_cast<const BlobHeader*>(a.blob_a);
  const BlobHeader* hb = reinterpret_cast<const BlobHeader*>(a.blob_b);
  return ha->magic == kMagic && hb->magic == kMagic && a.n_meshes_a <= ha->n_meshes &&
         a.n_meshes_b <= hb->n_meshes && (ha->width == 2 || ha->width == 4 || ha->width == 8) &&
         (hb->width == 2 || hb->width == 4 || hb->width == 8);
}

// One ray: the representative vertex r of a source mesh against mesh tm of T.
__device__ __forceinline__ int ray(float4 r, const Blob& T, int32_t tm, int32_t* stk, int stride, int cap,
                                   Counts& k) {
  if (r.w == 0.f) return U_OUT;  // the source mesh has no faces
  ++k.c[I_RAYS];
  return walk(T, tm, f3{r.x, r.y, r.z}, stk, stride, cap, k);
}

// The output byte of pair p in the call's mode, casting only the rays the
// mode needs (rep(B_j) against A_i first), or -1 when a ray's stack would
// overflow.
__device__ __forceinline__ int pair_result(const InsideArgs& a, int64_t p, int32_t* stk, int stride, int cap,
                                            Counts& k) {
  if (a.mode != 0 && a.cross[p] != 0) return a.mode == 3 ? 1 : 0;
  if (!blobs_ok(a)) {
    __hip_atomic_store(a.status, (int32_t)PR_E_UNSUPPORTED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  const int32_t i = a.pairs[2 * p], j = a.pairs[2 * p + 1];
  if (i < 0 || i >= a.n_meshes_a || j < 0 || j >= a.n_meshes_b) {
    __hip_atomic_store(a.status, (int32_t)PR_E_ARG, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  const Blob A = blob_of(a.blob_a), B = blob_of(a.blob_b);
  // d = 0: rep(B_j) against A_i; d = 1: rep(A_i) against B_j
  int r[2] = {U_OUT, U_OUT};
  const int d_lo = a.mode == 2 ? 1 : 0, d_hi = a.mode == 1 ? 0 : 1;
#pragma unroll 1
  for (int d = d_lo; d <= d_hi; ++d) {
    const Blob& T = d == 0 ? A : B;
    const int rd = ray(d == 0 ? B.rep[j] : A.rep[i], T, d == 0 ? i : j, stk, stride, cap, k);
    if (rd < 0) return -1;
    if (a.mode == 3 && rd == U_IN) return 1;
    if (d == 0) r[0] = rd; else r[1] = rd;
  }
  if (a.mode == 1) return r[0] == U_IN;
  if (a.mode != 0) return r[1] == U_IN;
  return (r[0] == U_IN ? 1 : 0) | (r[1] == U_IN ? 2 : 0) | (r[0] == U_ON ? 4 : 0) | (r[1] == U_ON ? 8 : 0);
}

__device__ __forceinline__ uint32_t wave_add(uint32_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

__global__ void k_inside_init(InsideArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < kCopies * I_N) a.stats[kStride * (t / I_N) + (t % I_N)] = 0ull;
  if (t == 0) {
    a.ctr[0] = 0u;  // pairs handed to the deep kernel
    a.ctr[1] = 0u;  // deep-kernel blocks finished
    *a.status = PR_OK;
  }
}

// One thread per pair (one wave per block: small launches still spread over
// every compute unit).
__global__ __launch_bounds__(kIB) void k_inside(InsideArgs a) {
  __shared__ int32_t stk[kFastCap * kIB];
  Counts k{};
  for (int64_t p = blockIdx.x * (int64_t)kIB + threadIdx.x; p < a.n_pairs; p += (int64_t)gridDim.x * kIB) {
    const int res = pair_result(a, p, stk + threadIdx.x, kIB, kFastCap, k);
    if (res < 0) {
      // out[p] is left alone (it may alias cross[p], which the rerun reads)
      a.deep[atomicAdd(a.ctr, 1u)] = (uint32_t)p;  // at most P pairs: the list never overflows
      ++k.c[I_DEEP];
    } else {
      a.out[p] = (uint8_t)res;
    }
  }
  unsigned long long* dst = a.stats + kStride * (blockIdx.x % kCopies);
#pragma unroll
  for (int q = 0; q < I_N; ++q) {
    const uint32_t sum = wave_add(k.c[q]);
    if (threadIdx.x == 0 && sum) atomicAdd(dst + q, (unsigned long long)sum);
  }
}

// Reruns the pairs whose stack overflowed with the full-depth stack, then the
// last block to finish sums the statistics and reports the status.
// keep_ok: leave dev_status alone unless this call found an error
// (refine_predicate: refine_intersects has written it already).
__global__ __launch_bounds__(kDeepB) void k_inside_deep(InsideArgs a, pr_inside_stats* out, int32_t* dev_status,
                                                       int keep_ok) {
  __shared__ int32_t stk[kDeepCap * kDeepB];
  __shared__ int last;
  Counts k{};
  const uint32_t n = __hip_atomic_load(a.ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (uint32_t q = blockIdx.x * kDeepB + threadIdx.x; q < n; q += gridDim.x * kDeepB) {
    const int64_t p = a.deep[q];
    Counts dup{};  // the rays and box tests were counted by the first pass
    int res = pair_result(a, p, stk + threadIdx.x, kDeepB, kDeepCap, dup);
    for (int c = I_VISITS; c < I_N; ++c) k.c[c] += dup.c[c];
    if (res < 0) {  // deeper than the build allows: not for a valid blob
      __hip_atomic_store(a.status, (int32_t)PR_E_UNSUPPORTED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      res = 0;
    }
    a.out[p] = (uint8_t)res;
  }
  // half-wave blocks and few pairs: each thread adds its own counters
  for (int c = 0; c < I_N; ++c)
    if (k.c[c]) atomicAdd(a.stats + c, (unsigned long long)k.c[c]);
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(a.ctr + 1, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!last) return;
  const int t = threadIdx.x;
  if (t < I_N && out) {
    unsigned long long sum = 0;
    for (int c = 0; c < kCopies; ++c)
      sum += __hip_atomic_load(a.stats + kStride * c + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    reinterpret_cast<uint64_t*>(out)[t] = sum;
  }
  if (t == 0 && dev_status) {
    const int32_t st = __hip_atomic_load(a.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (st != PR_OK || !keep_ok) *dev_status = st;
  }
}

void carve_inside(Carve& cv, InsideArgs& a, int64_t P) {
  a.deep = cv.take<uint32_t>(P);
  a.ctr = cv.take<uint32_t>(64);
  a.stats = cv.take<unsigned long long>((int64_t)kCopies * kStride);
  a.status = cv.take<int32_t>(64);
}

int check_inside(int64_t P) {
  if (P < 0) { set_error("n_pairs < 0"); return PR_E_ARG; }
  if (P > ((int64_t)1 << 30)) { set_error("n_pairs %lld beyond 2^30", (long long)P); return PR_E_UNSUPPORTED; }
  return PR_OK;
}

int inside_ws(int64_t P, size_t* bytes) {
  Carve cv{nullptr, 0};
  InsideArgs a{};
  carve_inside(cv, a, P);
  *bytes = cv.used + 256;
  return PR_OK;
}

// With keep_status, dev_status is written only on an error.
int inside_run(const void* blob_a, int64_t n_meshes_a, const void* blob_b, int64_t n_meshes_b,
               const int32_t* pairs, int64_t n_pairs, int32_t mode, const uint8_t* cross, uint8_t* out,
               pr_inside_stats* dev_stats, int32_t* dev_status, void* ws, size_t ws_bytes, bool keep_status,
               hipStream_t s) {
  InsideArgs a{};
  Carve cv{(char*)ws, ws_bytes};
  carve_inside(cv, a, n_pairs);
  if (cv.used > ws_bytes) { set_error("ws_bytes %zu < required %zu", ws_bytes, cv.used); return PR_E_CAPACITY; }
  a.blob_a = (const char*)blob_a;
  a.blob_b = (const char*)blob_b;
  a.n_meshes_a = n_meshes_a;
  a.n_meshes_b = n_meshes_b;
  a.pairs = pairs;
  a.n_pairs = n_pairs;
  a.cross = cross;
  a.out = out;
  a.mode = mode;
  hipLaunchKernelGGL(k_inside_init, dim3((kCopies * I_N + 255) / 256), dim3(256), 0, s, a);
  if (n_pairs > 0) {
    const int g = (int)std::min<int64_t>((n_pairs + kIB - 1) / kIB, 1 << 16);
    hipLaunchKernelGGL(k_inside, dim3(g), dim3(kIB), 0, s, a);
  }
  hipLaunchKernelGGL(k_inside_deep, dim3(kDeepGrid), dim3(kDeepB), 0, s, a, dev_stats, dev_status,
                     keep_status ? 1 : 0);
  PR_HIP(hipGetLastError());
  return PR_OK;
}

int check_inside_args(const void* blob_a, int64_t n_meshes_a, const void* blob_b, int64_t n_meshes_b,
                      const int32_t* pairs, int64_t n_pairs, const void* out) {
  if (!blob_a || !blob_b || n_meshes_a < 0 || n_meshes_b < 0 || (n_pairs > 0 && (!pairs || !out))) {
    set_error("null pointer or negative size");
    return PR_E_ARG;
  }
  return check_inside(n_pairs);
}

}  // namespace
}  // namespace pr

using namespace pr;

extern "C" int inside_workspace_bytes(int64_t n_pairs, size_t* ws_bytes) {
  int r = check_inside(n_pairs);
  if (r) return r;
  if (!ws_bytes) { set_error("ws_bytes is NULL"); return PR_E_ARG; }
  return inside_ws(n_pairs, ws_bytes);
}

extern "C" int inside_pairs(const void* blob_a, int64_t n_meshes_a, const void* blob_b, int64_t n_meshes_b,
                            const int32_t* pairs, int64_t n_pairs, int32_t mode, const uint8_t* cross,
                            uint8_t* out, pr_inside_stats* dev_stats, int32_t* dev_status, void* ws,
                            size_t ws_bytes, void* stream) {
  int r = check_inside_args(blob_a, n_meshes_a, blob_b, n_meshes_b, pairs, n_pairs, out);
  if (r) return r;
  if (mode < 0 || mode > 3) { set_error("mode %d not in 0..3", mode); return PR_E_ARG; }
  if (mode != 0 && n_pairs > 0 && !cross) { set_error("mode %d needs the overlap flags", mode); return PR_E_ARG; }
  if (!ws) { set_error("ws is NULL"); return PR_E_ARG; }
  return inside_run(blob_a, n_meshes_a, blob_b, n_meshes_b, pairs, n_pairs, mode, cross, out, dev_stats, dev_status,
                    ws, ws_bytes, false, (hipStream_t)stream);
}

extern "C" int refine_predicate_workspace_bytes(int64_t n_pairs, const pr_refine_params* params,
                                                size_t* ws_bytes) {
  if (!ws_bytes) { set_error("ws_bytes is NULL"); return PR_E_ARG; }
  size_t a = 0, b = 0;
  int r = refine_workspace_bytes(n_pairs, params, &a);
  if (r) return r;
  r = inside_workspace_bytes(n_pairs, &b);
  if (r) return r;
  *ws_bytes = a > b ? a : b;
  return PR_OK;
}

extern "C" int refine_predicate(const void* blob_a, int64_t n_meshes_a, const void* blob_b, int64_t n_meshes_b,
                                const int32_t* pairs, int64_t n_pairs, int32_t predicate, uint8_t* flags,
                                const pr_refine_params* params, pr_refine_stats* dev_stats,
                                pr_inside_stats* dev_inside_stats, int32_t* dev_status, void* ws, size_t ws_bytes,
                                void* stream) {
  if (predicate < 0 || predicate > 3) { set_error("predicate %d not in 0..3", predicate); return PR_E_ARG; }
  int r = check_inside_args(blob_a, n_meshes_a, blob_b, n_meshes_b, pairs, n_pairs, flags);
  if (r) return r;
  size_t need = 0;
  r = refine_predicate_workspace_bytes(n_pairs, params, &need);
  if (r) return r;
  if (!ws || ws_bytes < need) { set_error("ws_bytes %zu < required %zu", ws_bytes, need); return ws ? PR_E_CAPACITY : PR_E_ARG; }
  // the two steps run one after the other on the stream and share the workspace
  r = refine_intersects(blob_a, n_meshes_a, blob_b, n_meshes_b, pairs, n_pairs, flags, params, dev_stats, dev_status,
                        ws, ws_bytes, stream);
  if (r || predicate == 0) return r;
  return inside_run(blob_a, n_meshes_a, blob_b, n_meshes_b, pairs, n_pairs, predicate, flags, flags, dev_inside_stats,
                    dev_status, ws, ws_bytes, true, (hipStream_t)stream);
}
