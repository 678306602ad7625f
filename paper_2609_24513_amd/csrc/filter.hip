// filter_aabb_pairs and compact_pairs.
//
// Filter: all (i, j) whose closed mesh boxes overlap (touching boxes count),
// optionally restricted to pairs whose common box part meets a closed query
// box.  With a query box the meshes are first reduced to those meeting it
// (an ordered compaction per dataset: one block per dataset up to kSmallScan
// meshes, a flag pass and a device scan beyond).  Up to kFastCols columns
// and kFastRows rows, two kernels produce the pairs (a count pass and a
// write pass over blocks of 64 rows, the block totals summed in front of
// each block); larger datasets take the general path: one wave per kept row
// of A against LDS tiles of the kept boxes of B, a scan of the row counts
// and a second pass that writes each row's pairs.  Either way the output is
// sorted by (i, j) and identical run to run.  The exact total is always
// written; output beyond `cap` is dropped (the caller relaunches with a
// larger buffer, as the paper does for its result structure, Section 3.5).
//
// Compaction (Section 3.5 result materialisation): pairs whose flag is 1,
// in input order, in tiles of kScanTile pairs: the flag count of every tile,
// then every tile writes its pairs from the counts of the tiles before it.
// The prefix sums are the library's own (scan.h).
#include <hip/hip_runtime.h>

#include "common.h"
#include "scan.h"

namespace pr {
namespace {

constexpr int kBlock = 256;
constexpr int kScanBlock = 1024;        // threads of the single-block scans
constexpr int kScanItems = 4;           // consecutive items per thread per tile
constexpr int64_t kSmallScan = 65536;   // single-block scans up to this many items

__device__ __forceinline__ const MeshDesc* meshes_of(const void* blob) {
  const BlobHeader* h = reinterpret_cast<const BlobHeader*>(blob);
  return reinterpret_cast<const MeshDesc*>(reinterpret_cast<const char*>(blob) + h->off_mesh);
}

__device__ __forceinline__ bool meet(const float* a, const float* b) {
  return a[0] <= b[3] && b[0] <= a[3] && a[1] <= b[4] && b[1] <= a[4] && a[2] <= b[5] && b[2] <= a[5];
}

__global__ void k_keep(const void* blob, int64_t M, const float* query, int32_t* flag) {
  const MeshDesc* md = meshes_of(blob);
  int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; m < M; m += (int64_t)gridDim.x * blockDim.x) {
    bool ok = md[m].n_tris > 0;
    if (query) ok = ok && meet(md[m].box, query);
    flag[m] = ok ? 1 : 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) flag[M] = 0;
}

// Kept meshes: their ids and a compact copy of their boxes (24 bytes each,
// read coalesced by the row kernels instead of 64-byte descriptors).
__global__ void k_list(const void* blob, const int32_t* flag, const int32_t* pos, int64_t M, int32_t* ids,
                       float* boxes) {
  const MeshDesc* md = meshes_of(blob);
  int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; m < M; m += (int64_t)gridDim.x * blockDim.x)
    if (flag[m]) {
      const int32_t k = pos[m];
      ids[k] = (int32_t)m;
      for (int c = 0; c < 6; ++c) boxes[6 * (int64_t)k + c] = md[m].box[c];
    }
}

// Without a query box every mesh is a row (A) or a column (B): boxes copied
// in index order, an empty mesh given an inverted box (+inf lows, -inf
// highs) that meets nothing; ids are the identity.
__global__ void k_boxes_all(const void* blob_a, int64_t MA, int32_t* ids_a, float* box_a, int32_t* cnt_a,
                            const void* blob_b, int64_t MB, int32_t* ids_b, float* box_b, int32_t* cnt_b) {
  const int64_t n = MA + MB;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const bool a = i < MA;
    const int64_t m = a ? i : i - MA;
    const MeshDesc& d = meshes_of(a ? blob_a : blob_b)[m];
    float* bx = (a ? box_a : box_b) + 6 * m;
    const bool ok = d.n_tris > 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      bx[c] = ok ? d.box[c] : INFINITY;
      bx[3 + c] = ok ? d.box[3 + c] : -INFINITY;
    }
    (a ? ids_a : ids_b)[m] = (int32_t)m;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *cnt_a = (int32_t)MA;
    *cnt_b = (int32_t)MB;
  }
}

// With a query box: ordered compaction of the meshes that meet it, for
// datasets of at most kSmallScan meshes, in two launches.  k_keep_bits tests
// every mesh of both datasets, one per thread on as many blocks as there are
// tiles of kScanBlock meshes, and stores each wave's ballot (bit l of entry
// tile * kKeepWaves + wave: mesh tile * kScanBlock + wave * 64 + l).
// k_keep_small, one block per dataset (block 0: A, block 1: B), scans the
// entries' counts (one entry per thread) and each thread writes the kept
// meshes of its entry, ids and boxes, in index order; the count goes to cnt.
constexpr int kKeepWaves = kScanBlock / 64;
constexpr int kKeepEntries = (int)(kSmallScan / 64);  // ballot words of a dataset
static_assert(kKeepEntries == kScanBlock, "one ballot word per thread of the scan block");

__global__ __launch_bounds__(kScanBlock) void k_keep_bits(const void* blob_a, int64_t MA, const void* blob_b,
                                                          int64_t MB, const float* query, uint64_t* bits_a,
                                                          uint64_t* bits_b) {
  const int64_t tiles_a = (MA + kScanBlock - 1) / kScanBlock;
  const bool first = (int64_t)blockIdx.x < tiles_a;
  const int64_t tile = first ? (int64_t)blockIdx.x : (int64_t)blockIdx.x - tiles_a;
  const MeshDesc* md = meshes_of(first ? blob_a : blob_b);
  const int64_t M = first ? MA : MB;
  const int64_t m = tile * kScanBlock + threadIdx.x;
  bool ok = false;
  if (m < M) {
    const float4* p4 = reinterpret_cast<const float4*>(md + m);
    const float4 u = p4[0], v = p4[1], w = p4[2];  // box, node base/count, tri base/count
    const float b[6] = {u.x, u.y, u.z, u.w, v.x, v.y};
    float q[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) q[c] = query[c];
    ok = __float_as_int(w.y) > 0 && meet(b, q);
  }
  const uint64_t bm = __ballot(ok);
  if ((threadIdx.x & 63) == 0) (first ? bits_a : bits_b)[tile * kKeepWaves + (threadIdx.x >> 6)] = bm;
}

__global__ __launch_bounds__(kScanBlock) void k_keep_small(const void* blob_a, int64_t MA, const uint64_t* bits_a,
                                                           int32_t* ids_a, float* box_a, int32_t* cnt_a,
                                                           const void* blob_b, int64_t MB, const uint64_t* bits_b,
                                                           int32_t* ids_b, float* box_b, int32_t* cnt_b) {
  __shared__ int32_t s_scan[kKeepWaves];
  const bool first = blockIdx.x == 0;
  const MeshDesc* md = meshes_of(first ? blob_a : blob_b);
  const int64_t M = first ? MA : MB;
  const uint64_t* bits = first ? bits_a : bits_b;
  int32_t* ids = first ? ids_a : ids_b;
  float* boxes = first ? box_a : box_b;
  const int t = threadIdx.x;
  const int ntiles = (int)((M + kScanBlock - 1) / kScanBlock);  // at most 64 (M <= kSmallScan)
  // entry t covers meshes 64 t ... 64 t + 63 (tile t / kKeepWaves, wave
  // t % kKeepWaves), so the entries' order is the meshes' order
  uint64_t word = t < ntiles * kKeepWaves ? bits[t] : 0ull;
  int32_t total = 0;
  int32_t pos = block_exclusive_sum<kScanBlock>((int32_t)__popcll(word), s_scan, total);
  for (; word; word &= word - 1) {
    const int64_t m = 64 * (int64_t)t + __builtin_ctzll(word);
    ids[pos] = (int32_t)m;
#pragma unroll
    for (int c = 0; c < 6; ++c) boxes[6 * (int64_t)pos + c] = md[m].box[c];
    ++pos;
  }
  if (t == 0) *(first ? cnt_a : cnt_b) = total;
}

// Exclusive scan of the row counts (at most kSmallScan rows) in one block,
// over the first *n_live rows only (the kept rows); the total goes to
// off[n] (n the rows scanned) and to the caller's count.
__global__ __launch_bounds__(kScanBlock) void k_rowscan_small(const int64_t* cnt, int64_t rows, const int32_t* n_live,
                                                              int64_t* off, int64_t* total_out) {
  __shared__ int64_t s_scan[kScanBlock / 64];
  const int64_t live = *n_live;
  const int64_t n = live < 0 ? 0 : (live < rows ? live : rows);
  int64_t running = 0;
  for (int64_t base = 0; base < n; base += kScanBlock * kScanItems) {
    const int64_t r0 = base + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      v[i] = r0 + i < n ? cnt[r0 + i] : 0;
      sum += v[i];
    }
    int64_t total = 0;
    int64_t o = running + block_exclusive_sum<kScanBlock>(sum, s_scan, total);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
      if (r0 + i < n) {
        off[r0 + i] = o;
        o += v[i];
      }
    running += total;
  }
  if (threadIdx.x == 0) {
    off[n] = running;
    *total_out = running;
  }
}

struct RowArgs {
  const float* box_a;  // compact boxes of the kept meshes
  const float* box_b;
  const int32_t* ids_a;
  const int32_t* ids_b;
  const int32_t* na;  // device counts
  const int32_t* nb;
  const float* query;
  int64_t rows;       // capacity of the row arrays (n_meshes_a)
  bool live_only;     // counts only for the kept rows (the scan reads no more)
  int64_t* rowcnt;    // [rows + 1]
  const int64_t* rowoff;
  int32_t* pairs;
  int64_t cap;
};

// Row kernels: a block takes kRowsPerBlock kept rows of A (one per wave) and
// walks the kept boxes of B in tiles of kTile staged in LDS (one copy per
// tile for the block's rows instead of one L2 read per row); each wave tests
// its row against the tile, 64 columns at a time.
constexpr int kRowsPerBlock = kBlock / 64;
constexpr int kTile = 1024;

__device__ __forceinline__ bool test_box(const float* a, const float* q, float l0, float l1, float l2, float h0,
                                         float h1, float h2) {
  if (q) {
    return fmaxf(fmaxf(a[0], l0), q[0]) <= fminf(fminf(a[3], h0), q[3]) &&
           fmaxf(fmaxf(a[1], l1), q[1]) <= fminf(fminf(a[4], h1), q[4]) &&
           fmaxf(fmaxf(a[2], l2), q[2]) <= fminf(fminf(a[5], h2), q[5]);
  }
  return a[0] <= h0 && l0 <= a[3] && a[1] <= h1 && l1 <= a[4] && a[2] <= h2 && l2 <= a[5];
}

__device__ __forceinline__ void load_tile(float (*t)[kTile], const float* box_b, int32_t t0, int32_t nb) {
  for (int i = threadIdx.x; i < kTile; i += kBlock) {
    const int32_t k = t0 + i;
    if (k < nb) {
#pragma unroll
      for (int c = 0; c < 6; ++c) t[c][i] = box_b[6 * (int64_t)k + c];
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_row_count(RowArgs r) {
  __shared__ float tile[6][kTile];
  const int32_t na = *r.na, nb = *r.nb;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t nrows = r.live_only ? (na < r.rows ? (int64_t)na : r.rows) : r.rows;
  const int64_t groups = (nrows + kRowsPerBlock - 1) / kRowsPerBlock;
  for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
    const int64_t row = g * kRowsPerBlock + wv;
    const bool live = row < na;
    float a[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) a[c] = live ? r.box_a[6 * row + c] : 0.f;
    unsigned long long cnt = 0;
    if (g * kRowsPerBlock < na) {  // uniform over the block
      for (int32_t t0 = 0; t0 < nb; t0 += kTile) {
        __syncthreads();
        load_tile(tile, r.box_b, t0, nb);
        __syncthreads();
        if (live) {
          const int32_t n = min(kTile, nb - t0);
          for (int32_t i = lane; i < n; i += 64)
            cnt += test_box(a, r.query, tile[0][i], tile[1][i], tile[2][i], tile[3][i], tile[4][i], tile[5][i]) ? 1
                                                                                                             : 0;
        }
      }
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
    if (lane == 0 && row < nrows) r.rowcnt[row] = (int64_t)cnt;
  }
  if (!r.live_only && blockIdx.x == 0 && threadIdx.x == 0) r.rowcnt[r.rows] = 0;
}

__global__ __launch_bounds__(kBlock) void k_row_write(RowArgs r) {
  __shared__ float tile[6][kTile];
  const int32_t na = *r.na, nb = *r.nb;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t groups = ((int64_t)na + kRowsPerBlock - 1) / kRowsPerBlock;
  for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
    const int64_t row = g * kRowsPerBlock + wv;
    const bool live = row < na;
    float a[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) a[c] = live ? r.box_a[6 * row + c] : 0.f;
    const int32_t ia = live ? r.ids_a[row] : 0;
    int64_t out = live ? r.rowoff[row] : 0;
    for (int32_t t0 = 0; t0 < nb; t0 += kTile) {
      __syncthreads();
      load_tile(tile, r.box_b, t0, nb);
      __syncthreads();
      if (!live) continue;
      const int32_t n = min(kTile, nb - t0);
      for (int32_t i0 = 0; i0 < n; i0 += 64) {
        const int32_t i = i0 + lane;
        const bool ok =
            i < n && test_box(a, r.query, tile[0][i], tile[1][i], tile[2][i], tile[3][i], tile[4][i], tile[5][i]);
        const uint64_t m = __ballot(ok);
        if (ok) {
          const int64_t pos = out + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
          if (pos < r.cap) {
            r.pairs[2 * pos] = ia;
            r.pairs[2 * pos + 1] = r.ids_b[t0 + i];
          }
        }
        out += __popcll(m);
      }
    }
  }
}

// Pair kernels for the common shape (at most kFastCols columns, at most
// kFastRows rows).  A block owns kRT = 64 consecutive rows, one per lane;
// each of its kPairWaves waves holds the rows' boxes and walks a contiguous
// slice of the columns, 64 at a time: one vector load per lane stages the
// chunk in the wave's LDS area, then every column is read back as an LDS
// broadcast and tested by all 64 rows at once (six compares per 64 tests),
// each lane counting its row's hits in a register.  The count pass stores
// the (row, slice) counts and the block's total; the write pass scans the
// block's counts in row-major order, adds the totals of the blocks before
// it and walks the slices again, each lane writing its row's pairs in
// ascending column order: the same sorted list as the general path's.
// Without a query box the kernels read the mesh descriptors directly (an
// empty mesh pairs with nothing); with one they read the kept lists.
constexpr int kRT = 64;
constexpr int kPairBlock = 1024;
constexpr int kPairWaves = kPairBlock / 64;
constexpr int64_t kFastCols = 8192;
constexpr int64_t kFastGrid = 2048;
constexpr int64_t kFastRows = kRT * kFastGrid;

struct PairArgs {
  const void* blob_a;  // descriptors (no query box)
  const void* blob_b;
  const float* box_a;  // kept lists (query box)
  const float* box_b;
  const int32_t* ids_a;
  const int32_t* ids_b;
  const int32_t* na;  // kept counts (query box)
  const int32_t* nb;
  int64_t MA, MB;
  int32_t* cnt;       // [grid * kRT * kPairWaves]: (row, slice) counts
  int32_t* blocksum;  // [grid]
  int32_t* pairs;
  int64_t cap;
  int64_t* count;
};

template <bool Q>
__device__ __forceinline__ int64_t rows_of(const PairArgs& a) { return Q ? (int64_t)*a.na : a.MA; }
template <bool Q>
__device__ __forceinline__ int64_t cols_of(const PairArgs& a) { return Q ? (int64_t)*a.nb : a.MB; }

// Box and id of row i of A or column i of B; an empty mesh gets an
// inverted box (+inf lows, -inf highs), which meets nothing.
template <bool Q>
__device__ __forceinline__ int32_t mesh_box(const void* blob, const float* boxes, const int32_t* ids, int64_t i,
                                            float* b) {
  if (Q) {
    const cptr_t<float> p = cview(boxes) + 6 * i;
#pragma unroll
    for (int c = 0; c < 6; ++c) b[c] = p[c];
    return cview(ids)[i];
  }
  const cptr_t<MeshDesc> d = cview(meshes_of(blob)) + i;
  const bool ok = d->n_tris > 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    b[c] = ok ? d->box[c] : INFINITY;
    b[3 + c] = ok ? d->box[3 + c] : -INFINITY;
  }
  return (int32_t)i;
}

// Column slice of wave w: [lo, hi).
__device__ __forceinline__ void slice_of(int64_t nb, int w, int64_t& lo, int64_t& hi) {
  const int64_t per = (nb + kPairWaves - 1) / kPairWaves;
  lo = per * w < nb ? per * w : nb;
  hi = lo + per < nb ? lo + per : nb;
}

// Closed overlap of row box a and a column box, without branches.  With a
// query box the rows and columns are the kept meshes, which each meet the
// query box; two such boxes that overlap share a point with it on every
// axis (three pairwise-meeting intervals have a common point), so the same
// test serves both cases.
__device__ __forceinline__ bool overlap(const float* a, float l0, float l1, float l2, float h0, float h1, float h2) {
  return (a[0] <= h0) & (l0 <= a[3]) & (a[1] <= h1) & (l1 <= a[4]) & (a[2] <= h2) & (l2 <= a[5]);
}

// A staged column: box (lo xyz, hi xyz) and id.
struct alignas(16) ColBox {
  float lo[3];
  float hi0;
  float hi1, hi2;
  int32_t id, pad;
};

// Walks the wave's slice [lo, hi) in chunks of 64 staged in `st` (the
// wave's 64-entry LDS area) for the lane's row box rb; with WRITE, each hit
// (row id ia, column id) goes to pairs[out++] while out < cap.  Returns the
// number of hits.
template <bool Q, bool WRITE>
__device__ __forceinline__ int32_t walk(const PairArgs& a, ColBox* st, int64_t lo, int64_t hi, const float* rb,
                                        int32_t ia, int64_t out) {
  const int lane = threadIdx.x & 63;
  int32_t n = 0;
  for (int64_t c0 = lo; c0 < hi; c0 += 64) {
    const int m = (int)(hi - c0 < 64 ? hi - c0 : 64);
    if (lane < m) {
      float b[6];
      const int32_t id = mesh_box<Q>(a.blob_b, a.box_b, a.ids_b, c0 + lane, b);
      st[lane] = ColBox{{b[0], b[1], b[2]}, b[3], b[4], b[5], id, 0};
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int u = 0; u < m; ++u) {
      const ColBox c = st[u];
      const bool ok = overlap(rb, c.lo[0], c.lo[1], c.lo[2], c.hi0, c.hi1, c.hi2);
      if (WRITE && ok) {
        if (out < a.cap) {
          a.pairs[2 * out] = ia;
          a.pairs[2 * out + 1] = c.id;
        }
        ++out;
      }
      n += ok ? 1 : 0;
    }
    __builtin_amdgcn_wave_barrier();  // the chunk is read before the next one is staged
  }
  return n;
}

template <bool Q, bool WRITE>
__global__ __launch_bounds__(kPairBlock) void k_pairs(PairArgs a) {
  __shared__ int64_t s_red[kPairWaves];
  __shared__ int32_t s_scan[kPairWaves];
  __shared__ ColBox s_col[kPairWaves][64];
  __shared__ int64_t s_base;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
  const int64_t r0 = (int64_t)blockIdx.x * kRT;
  const int64_t na = rows_of<Q>(a), nb = cols_of<Q>(a);
  const int64_t row = r0 + lane;
  float rb[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  int32_t ia = 0;
  if (row < na) ia = mesh_box<Q>(a.blob_a, a.box_a, a.ids_a, row, rb);
  int64_t lo, hi;
  slice_of(nb, w, lo, hi);
  const bool any = r0 < na;  // uniform over the block
  int32_t* cnt = a.cnt + (int64_t)blockIdx.x * kPairBlock;
  if (!WRITE) {
    const int32_t n = any ? walk<Q, false>(a, s_col[w], lo, hi, rb, ia, 0) : 0;
    cnt[lane * kPairWaves + w] = n;  // row-major (row, slice)
    const int64_t t = block_sum<kPairBlock>((int64_t)n, s_red);
    if (threadIdx.x == 0) a.blocksum[blockIdx.x] = (int32_t)t;
    return;
  }
  int32_t total = 0;
  const int32_t pre = block_exclusive_sum<kPairBlock>(cnt[threadIdx.x], s_scan, total);
  int64_t before = 0;
  for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += kPairBlock) before += a.blocksum[b];
  before = block_sum<kPairBlock>(before, s_red);
  if (threadIdx.x == 0) s_base = before;
  __syncthreads();
  // the offset of (row = lane, slice = w) sits with thread lane * kPairWaves + w
  __shared__ int32_t s_off[kPairBlock];
  s_off[threadIdx.x] = pre;
  __syncthreads();
  if (any) walk<Q, true>(a, s_col[w], lo, hi, rb, ia, s_base + s_off[lane * kPairWaves + w]);
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *a.count = s_base + total;
}


__global__ void k_set_i64(int64_t* out, int64_t v) { *out = v; }

__device__ __forceinline__ int64_t clamped_n(int64_t n, const int64_t* n_dev) {
  return n_dev ? (*n_dev < 0 ? 0 : (*n_dev < n ? *n_dev : n)) : n;
}

// Compaction, pass 1: the number of flagged pairs of each tile (pairs at
// or beyond the device count, when one is given, are not flagged).
__global__ __launch_bounds__(kTileThreads) void k_cflag_tiles(const uint8_t* flags, int64_t n, const int64_t* n_dev,
                                                              int64_t* tsum) {
  __shared__ int64_t s[kTileThreads / 64];
  const int64_t m = clamped_n(n, n_dev);
  const int64_t i0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kTileItems;
  int64_t c = 0;
#pragma unroll
  for (int k = 0; k < kTileItems; ++k) c += i0 + k < m && flags[i0 + k] ? 1 : 0;
  const int64_t t = block_sum<kTileThreads>(c, s);
  if (threadIdx.x == 0) tsum[blockIdx.x] = t;
}

// Compaction, pass 2: tile b writes its flagged pairs in order from its
// offset.  TOP: tsum already holds the tiles' offsets (scanned by
// k_scan_top, which also wrote the count); otherwise the tile adds up the
// counts of the tiles before it and the last tile writes the count.
// kTileItems consecutive pairs per thread; their flagged pairs are read
// before the scan, so that every load is in flight at once.
template <bool TOP>
__global__ __launch_bounds__(kTileThreads) void k_cflag_write(const int32_t* pairs, const uint8_t* flags, int64_t n,
                                                              const int64_t* n_dev, const int64_t* tsum, int32_t* out,
                                                              int64_t cap, int64_t* count) {
  __shared__ int64_t s[kTileThreads / 64];
  const int64_t m = clamped_n(n, n_dev);
  const int64_t i0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kTileItems;
  uint32_t f = 0;
#pragma unroll
  for (int k = 0; k < kTileItems; ++k) f |= (i0 + k < m && flags[i0 + k] ? 1u : 0u) << k;
  int32_t pv[kTileItems][2];
#pragma unroll
  for (int k = 0; k < kTileItems; ++k)
    if ((f >> k) & 1u) {
      pv[k][0] = pairs[2 * (i0 + k)];
      pv[k][1] = pairs[2 * (i0 + k) + 1];
    }
  int64_t base;
  if (TOP) {
    base = tsum[blockIdx.x];
  } else {
    int64_t b = 0;
    for (int64_t j = threadIdx.x; j < (int64_t)blockIdx.x; j += kTileThreads) b += tsum[j];
    base = block_sum<kTileThreads>(b, s);
  }
  int64_t all = 0;
  int64_t pos = base + block_exclusive_sum<kTileThreads>((int64_t)__popc(f), s, all);
#pragma unroll
  for (int k = 0; k < kTileItems; ++k)
    if ((f >> k) & 1u) {
      if (pos < cap) {
        out[2 * pos] = pv[k][0];
        out[2 * pos + 1] = pv[k][1];
      }
      ++pos;
    }
  if (!TOP && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *count = base + all;
}

// Tiles up to which pass 2 adds up the earlier tiles' counts itself.
constexpr int64_t kDirectTiles = 1024;

// Concatenation of the leading pairs of n fixed-size regions (the candidate
// lists that one filter call per query leaves in its own region), in region
// order, with the counts read on the device: one block per region sums the
// clamped counts of the regions before it, then copies its rows.
__global__ __launch_bounds__(kBlock) void k_gather(const int32_t* regions, int64_t region_cap, const int64_t* counts,
                                                  int64_t n, int32_t* out, int64_t cap, int64_t* total) {
  __shared__ int64_t s_red[kBlock / 64];
  __shared__ int64_t s_off;
  const int64_t k = blockIdx.x;
  if (n == 0) {
    if (threadIdx.x == 0) *total = 0;
    return;
  }
  auto clamped = [&](int64_t j) {
    const int64_t c = counts[j];
    return c < 0 ? (int64_t)0 : (c < region_cap ? c : region_cap);
  };
  int64_t part = 0;
  for (int64_t j = threadIdx.x; j < k; j += kBlock) part += clamped(j);
  part = block_sum<kBlock>(part, s_red);
  if (threadIdx.x == 0) s_off = part;
  __syncthreads();
  const int64_t off = s_off, c = clamped(k);
  const int32_t* src = regions + 2 * k * region_cap;
  for (int64_t i = threadIdx.x; i < c; i += kBlock)
    if (off + i < cap) {
      out[2 * (off + i)] = src[2 * i];
      out[2 * (off + i) + 1] = src[2 * i + 1];
    }
  if (k == n - 1 && threadIdx.x == 0) *total = off + c;
}

struct FilterWs {
  int32_t *flag_a, *flag_b, *pos_a, *pos_b, *ids_a, *ids_b;
  float *box_a, *box_b;
  int64_t *rowcnt, *rowoff;
  int32_t *blocksum, *paircnt;
  int64_t* tsum;  // tile sums of the device-wide scans
  uint64_t *keep_a, *keep_b;  // query-box ballots of the single-block keep path
};

int carve_filter(Carve& cv, FilterWs& w, int64_t MA, int64_t MB) {
  w.flag_a = cv.take<int32_t>(MA + 1);
  w.flag_b = cv.take<int32_t>(MB + 1);
  w.pos_a = cv.take<int32_t>(MA + 1);
  w.pos_b = cv.take<int32_t>(MB + 1);
  w.ids_a = cv.take<int32_t>(MA + 1);
  w.ids_b = cv.take<int32_t>(MB + 1);
  w.box_a = cv.take<float>(6 * (MA + 1));
  w.box_b = cv.take<float>(6 * (MB + 1));
  w.rowcnt = cv.take<int64_t>(MA + 1);
  w.rowoff = cv.take<int64_t>(MA + 1);
  w.blocksum = cv.take<int32_t>(kFastGrid);
  const int64_t fast_rows = MA <= kFastRows ? MA : 0;
  w.paircnt = cv.take<int32_t>((fast_rows + kRT - 1) / kRT * kPairBlock);
  const int64_t mx = MA > MB ? MA : MB;
  w.tsum = cv.take<int64_t>(scan_tiles_of(mx + 1));
  w.keep_a = cv.take<uint64_t>(kKeepEntries);
  w.keep_b = cv.take<uint64_t>(kKeepEntries);
  return PR_OK;
}

// The meshes of both datasets (each of at most kSmallScan) that meet the
// query box: ids, boxes and counts in the filter workspace.
void launch_keep_small(hipStream_t s, const void* blob_a, int64_t MA, const void* blob_b, int64_t MB,
                       const float* query, const FilterWs& w) {
  const int64_t tiles = (MA + kScanBlock - 1) / kScanBlock + (MB + kScanBlock - 1) / kScanBlock;
  if (tiles > 0)
    hipLaunchKernelGGL(k_keep_bits, dim3((unsigned)tiles), dim3(kScanBlock), 0, s, blob_a, MA, blob_b, MB, query,
                       w.keep_a, w.keep_b);
  hipLaunchKernelGGL(k_keep_small, dim3(2), dim3(kScanBlock), 0, s, blob_a, MA, (const uint64_t*)w.keep_a, w.ids_a,
                     w.box_a, w.pos_a + MA, blob_b, MB, (const uint64_t*)w.keep_b, w.ids_b, w.box_b, w.pos_b + MB);
}

struct CompactWs {
  int64_t* tsum;  // flag count (then offset) of each tile
};

int carve_compact(Carve& cv, CompactWs& w, int64_t n) {
  w.tsum = cv.take<int64_t>(scan_tiles_of(n) + 1);
  return PR_OK;
}

}  // namespace
}  // namespace pr

using namespace pr;

extern "C" int filter_aabb_pairs_ws_bytes(int64_t n_meshes_a, int64_t n_meshes_b, size_t* ws_bytes) {
  if (n_meshes_a < 0 || n_meshes_b < 0 || !ws_bytes) { set_error("bad argument"); return PR_E_ARG; }
  if (n_meshes_a >= ((int64_t)1 << 30) || n_meshes_b >= ((int64_t)1 << 30)) { set_error("too many meshes"); return PR_E_UNSUPPORTED; }
  Carve cv{nullptr, 0};
  FilterWs w{};
  int r = carve_filter(cv, w, n_meshes_a, n_meshes_b);
  if (r) return r;
  *ws_bytes = cv.used + 256;
  return PR_OK;
}

extern "C" int filter_aabb_pairs(const void* blob_a, int64_t n_meshes_a, const void* blob_b, int64_t n_meshes_b,
                                 const float* query_box, int32_t* pairs, int64_t cap, int64_t* dev_count, void* ws,
                                 size_t ws_bytes, void* stream) {
  if (!blob_a || !blob_b || !dev_count || !ws || cap < 0 || (cap > 0 && !pairs) || n_meshes_a < 0 || n_meshes_b < 0) {
    set_error("bad argument");
    return PR_E_ARG;
  }
  if (n_meshes_a >= ((int64_t)1 << 30) || n_meshes_b >= ((int64_t)1 << 30)) { set_error("too many meshes"); return PR_E_UNSUPPORTED; }
  hipStream_t s = (hipStream_t)stream;
  Carve cv{(char*)ws, ws_bytes};
  FilterWs w{};
  int r = carve_filter(cv, w, n_meshes_a, n_meshes_b);
  if (r) return r;
  if (cv.used > ws_bytes) { set_error("ws_bytes %zu < required %zu", ws_bytes, cv.used); return PR_E_CAPACITY; }
  const int64_t MA = n_meshes_a, MB = n_meshes_b;
  if (MA > 0 && MB > 0 && MA <= kFastRows && MB <= kFastCols && (!query_box || MA <= kSmallScan)) {
    PairArgs pa{};
    pa.MA = MA;
    pa.MB = MB;
    pa.blocksum = w.blocksum;
    pa.cnt = w.paircnt;
    pa.pairs = pairs;
    pa.cap = cap;
    pa.count = dev_count;
    const int grid = (int)((MA + kRT - 1) / kRT);
    if (!query_box) {
      pa.blob_a = blob_a;
      pa.blob_b = blob_b;
      hipLaunchKernelGGL((k_pairs<false, false>), dim3(grid), dim3(kPairBlock), 0, s, pa);
      hipLaunchKernelGGL((k_pairs<false, true>), dim3(grid), dim3(kPairBlock), 0, s, pa);
    } else {
      launch_keep_small(s, blob_a, MA, blob_b, MB, query_box, w);
      pa.box_a = w.box_a;
      pa.box_b = w.box_b;
      pa.ids_a = w.ids_a;
      pa.ids_b = w.ids_b;
      pa.na = w.pos_a + MA;
      pa.nb = w.pos_b + MB;
      hipLaunchKernelGGL((k_pairs<true, false>), dim3(grid), dim3(kPairBlock), 0, s, pa);
      hipLaunchKernelGGL((k_pairs<true, true>), dim3(grid), dim3(kPairBlock), 0, s, pa);
    }
    PR_HIP(hipGetLastError());
    return PR_OK;
  }
  if (!query_box) {
    hipLaunchKernelGGL(k_boxes_all, dim3(grid_for(MA + MB, kBlock)), dim3(kBlock), 0, s, blob_a, MA, w.ids_a,
                       w.box_a, w.pos_a + MA, blob_b, MB, w.ids_b, w.box_b, w.pos_b + MB);
  } else if (MA <= kSmallScan && MB <= kSmallScan) {
    launch_keep_small(s, blob_a, MA, blob_b, MB, query_box, w);
  } else {
    hipLaunchKernelGGL(k_keep, dim3(grid_for(MA + 1, kBlock)), dim3(kBlock), 0, s, blob_a, MA, query_box, w.flag_a);
    hipLaunchKernelGGL(k_keep, dim3(grid_for(MB + 1, kBlock)), dim3(kBlock), 0, s, blob_b, MB, query_box, w.flag_b);
    PR_HIP(device_exclusive_scan(w.flag_a, w.pos_a, MA + 1, w.tsum, (int64_t*)nullptr, s));
    PR_HIP(device_exclusive_scan(w.flag_b, w.pos_b, MB + 1, w.tsum, (int64_t*)nullptr, s));
    hipLaunchKernelGGL(k_list, dim3(grid_for(MA, kBlock)), dim3(kBlock), 0, s, blob_a, (const int32_t*)w.flag_a,
                       (const int32_t*)w.pos_a, MA, w.ids_a, w.box_a);
    hipLaunchKernelGGL(k_list, dim3(grid_for(MB, kBlock)), dim3(kBlock), 0, s, blob_b, (const int32_t*)w.flag_b,
                       (const int32_t*)w.pos_b, MB, w.ids_b, w.box_b);
  }
  RowArgs ra{};
  ra.box_a = w.box_a;
  ra.box_b = w.box_b;
  ra.query = query_box;
  ra.ids_a = w.ids_a;
  ra.ids_b = w.ids_b;
  ra.na = w.pos_a + MA;
  ra.nb = w.pos_b + MB;
  ra.rows = MA;
  ra.live_only = MA <= kSmallScan;
  ra.rowcnt = w.rowcnt;
  ra.rowoff = w.rowoff;
  ra.pairs = pairs;
  ra.cap = cap;
  const int64_t row_groups = (MA + kRowsPerBlock - 1) / kRowsPerBlock;
  const int rows_grid = (int)(row_groups < 2048 ? (row_groups > 0 ? row_groups : 1) : 2048);
  hipLaunchKernelGGL(k_row_count, dim3(rows_grid), dim3(kBlock), 0, s, ra);
  if (MA <= kSmallScan) {
    hipLaunchKernelGGL(k_rowscan_small, dim3(1), dim3(kScanBlock), 0, s, (const int64_t*)w.rowcnt, MA,
                       (const int32_t*)(w.pos_a + MA), w.rowoff, dev_count);
    hipLaunchKernelGGL(k_row_write, dim3(rows_grid), dim3(kBlock), 0, s, ra);
  } else {
    PR_HIP(device_exclusive_scan((const int64_t*)w.rowcnt, w.rowoff, MA + 1, w.tsum, dev_count, s));
    hipLaunchKernelGGL(k_row_write, dim3(rows_grid), dim3(kBlock), 0, s, ra);
  }
  PR_HIP(hipGetLastError());
  return PR_OK;
}

extern "C" int compact_pairs_ws_bytes(int64_t n_pairs, size_t* ws_bytes) {
  if (n_pairs < 0 || !ws_bytes) { set_error("bad argument"); return PR_E_ARG; }
  if (n_pairs >= ((int64_t)1 << 30)) { set_error("n_pairs >= 2^30"); return PR_E_UNSUPPORTED; }
  Carve cv{nullptr, 0};
  CompactWs w{};
  int r = carve_compact(cv, w, n_pairs);
  if (r) return r;
  *ws_bytes = cv.used + 256;
  return PR_OK;
}

extern "C" int compact_pairs(const int32_t* pairs, const uint8_t* flags, int64_t n_pairs, const int64_t* dev_n_pairs,
                             int32_t* out, int64_t cap, int64_t* dev_count, void* ws, size_t ws_bytes, void* stream) {
  if (n_pairs < 0 || cap < 0 || !dev_count || !ws || (n_pairs > 0 && (!pairs || !flags)) || (cap > 0 && !out)) {
    set_error("bad argument");
    return PR_E_ARG;
  }
  if (n_pairs >= ((int64_t)1 << 30)) { set_error("n_pairs >= 2^30"); return PR_E_UNSUPPORTED; }
  hipStream_t s = (hipStream_t)stream;
  Carve cv{(char*)ws, ws_bytes};
  CompactWs w{};
  int r = carve_compact(cv, w, n_pairs);
  if (r) return r;
  if (cv.used > ws_bytes) { set_error("ws_bytes %zu < required %zu", ws_bytes, cv.used); return PR_E_CAPACITY; }
  const int64_t nt = scan_tiles_of(n_pairs);
  if (nt == 0) {
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, dev_count, (int64_t)0);
    PR_HIP(hipGetLastError());
    return PR_OK;
  }
  hipLaunchKernelGGL(k_cflag_tiles, dim3((unsigned)nt), dim3(kTileThreads), 0, s, flags, n_pairs, dev_n_pairs, w.tsum);
  if (nt <= kDirectTiles) {
    hipLaunchKernelGGL(k_cflag_write<false>, dim3((unsigned)nt), dim3(kTileThreads), 0, s, pairs, flags, n_pairs,
                       dev_n_pairs, (const int64_t*)w.tsum, out, cap, dev_count);
  } else {
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kTopThreads), 0, s, w.tsum, nt, dev_count);
    hipLaunchKernelGGL(k_cflag_write<true>, dim3((unsigned)nt), dim3(kTileThreads), 0, s, pairs, flags, n_pairs,
                       dev_n_pairs, (const int64_t*)w.tsum, out, cap, dev_count);
  }
  PR_HIP(hipGetLastError());
  return PR_OK;
}

extern "C" int gather_pair_regions(const int32_t* regions, int64_t region_cap, const int64_t* dev_counts,
                                   int64_t n_regions, int32_t* out, int64_t cap, int64_t* dev_total, void* stream) {
  if (region_cap < 0 || n_regions < 0 || cap < 0 || !dev_total ||
      (n_regions > 0 && (!regions || !dev_counts)) || (cap > 0 && !out)) {
    set_error("bad argument");
    return PR_E_ARG;
  }
  if (n_regions > ((int64_t)1 << 20)) { set_error("n_regions > 2^20"); return PR_E_UNSUPPORTED; }
  hipLaunchKernelGGL(k_gather, dim3(n_regions > 0 ? (unsigned)n_regions : 1u), dim3(kBlock), 0, (hipStream_t)stream,
                     regions, region_cap, dev_counts, n_regions, out, cap, dev_total);
  PR_HIP(hipGetLastError());
  return PR_OK;
}
