// Exact CPU oracle for the closed-set mesh-pair intersection predicate.
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
// reference that the HIP library is checked against.  Only the tests, the
// smoke check and the CPU-baseline leg of the benchmark load it; the
// library shares no code, header, table or helper with it.
//
// What is computed (the join's refinement predicate, Section 3.2 "Overlap
// Join" read with closed sets): a candidate pair (A_i, B_j) of closed
// triangle meshes is TRUE iff some closed triangle t of A_i and some closed
// triangle u of B_j share a point.  Vertices are the exact real values of
// the stored FP32 coordinates.  Touching counts (vertex-vertex, vertex on
// face, edge-edge, coplanar contact); a mesh nested inside another without
// contact is FALSE (containment is a separate predicate, Section 3.3).
//
// How: triangle-triangle intersection by the separating axis theorem,
// evaluated in exact integer arithmetic.
//  * Each FP32 value is m * 2^e with |m| < 2^24.  Within one test all values
//    are scaled by 2^-emin (emin = smallest exponent present), which turns
//    them into exact integers; every quantity compared below is a
//    homogeneous polynomial of the same degree, so signs are unchanged.
//  * Two compact convex sets are disjoint iff a plane separates them
//    strictly.  For two non-degenerate triangles, the normal of such a plane
//    can be taken among 17 candidates: the two face normals n_t, n_u, the
//    nine cross products e_t x e_u of their edges, and the six in-plane edge
//    normals n_t x e_t, n_u x e_u (these are the facet normals of the
//    Minkowski difference t - u, whether or not the triangles are coplanar).
//    The three coordinate axes are valid candidates too and are tried first
//    as a cheap exact rejection.
//  * An axis L separates iff max(L.t) < min(L.u) or max(L.u) < min(L.t).
//    Degree of the compared polynomials: <= 4 in the coordinates.
//  * Mesh pair: brute force over all triangle pairs (mode 0), or the same
//    pairs restricted by exact closed-box sweep-and-prune (mode 1; sound
//    because disjoint boxes imply disjoint triangles).  Stops at the first
//    intersecting couple.
// Degenerate triangles (exactly collinear vertices) are rejected with
// ORACLE_E_DEGENERATE: the paper leaves them to preprocessing (Section 3.6).
// The check comes before any other test, so a degenerate triangle is refused
// wherever it lies; at mesh level every pair holding its mesh is refused.
// Face ids outside the mesh's vertex range and non-finite coordinates are
// argument errors (ORACLE_E_ARG).  A value that would not fit the fixed-width
// integers is reported as ORACLE_E_OVERFLOW (never for finite FP32 input:
// 1280 bits cover degree-4 products over the whole FP32 exponent range).

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

enum { ORACLE_OK = 0, ORACLE_E_ARG = -1, ORACLE_E_DEGENERATE = -3, ORACLE_E_OVERFLOW = -6 };

namespace {

constexpr int LIMBS = 20;  // 1280 bits: enough for any finite FP32 input

struct Big {
  int n;       // used limbs of the magnitude (0 <=> zero)
  bool neg;    // sign (false for zero)
  uint64_t d[LIMBS];
};

thread_local bool g_overflow = false;  // set if a value would not fit (never expected)

// Limbs a value may use.  LIMBS in normal operation; a test lowers it
// (oracle_set_limb_budget) to check that a value which does not fit is
// reported as ORACLE_E_OVERFLOW instead of giving a silently wrong sign.
std::atomic<int> g_limb_budget{LIMBS};
inline int limb_budget() { return g_limb_budget.load(std::memory_order_relaxed); }

inline void big_norm(Big& r) {
  while (r.n > 0 && r.d[r.n - 1] == 0) --r.n;
  if (r.n == 0) r.neg = false;
}

inline Big big_zero() {
  Big r;
  r.n = 0; r.neg = false;
  std::memset(r.d, 0, sizeof r.d);
  return r;
}

// value = (neg ? -1 : 1) * mag * 2^shift
Big big_from(uint64_t mag, bool neg, int shift) {
  Big r = big_zero();
  if (mag == 0) return r;
  int q = shift / 64, s = shift % 64;
  if (q + 1 >= limb_budget()) { g_overflow = true; return r; }
  r.d[q] = mag << s;
  if (s) r.d[q + 1] = mag >> (64 - s);
  r.n = q + 2;
  r.neg = neg;
  big_norm(r);
  return r;
}

int mag_cmp(const Big& a, const Big& b) {
  if (a.n != b.n) return a.n < b.n ? -1 : 1;
  for (int i = a.n - 1; i >= 0; --i)
    if (a.d[i] != b.d[i]) return a.d[i] < b.d[i] ? -1 : 1;
  return 0;
}

Big mag_add(const Big& a, const Big& b) {
  Big r = big_zero();
  int n = std::max(a.n, b.n);
  unsigned __int128 carry = 0;
  for (int i = 0; i < n; ++i) {
    unsigned __int128 t = (unsigned __int128)a.d[i] + b.d[i] + carry;
    r.d[i] = (uint64_t)t;
    carry = t >> 64;
  }
  if (carry) {
    if (n >= limb_budget()) { g_overflow = true; return r; }
    r.d[n++] = (uint64_t)carry;
  }
  r.n = n;
  big_norm(r);
  return r;
}

// |a| - |b|, requires |a| >= |b|
Big mag_sub(const Big& a, const Big& b) {
  Big r = big_zero();
  uint64_t borrow = 0;
  for (int i = 0; i < a.n; ++i) {
    uint64_t bi = b.d[i];
    uint64_t t = a.d[i] - bi - borrow;
    borrow = (a.d[i] < bi || (a.d[i] - bi) < borrow) ? 1 : 0;
    r.d[i] = t;
  }
  r.n = a.n;
  big_norm(r);
  return r;
}

Big add(const Big& a, const Big& b) {
  if (a.n == 0) return b;
  if (b.n == 0) return a;
  if (a.neg == b.neg) {
    Big r = mag_add(a, b);
    r.neg = r.n ? a.neg : false;
    return r;
  }
  int c = mag_cmp(a, b);
  if (c == 0) return big_zero();
  if (c > 0) { Big r = mag_sub(a, b); r.neg = r.n ? a.neg : false; return r; }
  Big r = mag_sub(b, a); r.neg = r.n ? b.neg : false; return r;
}

Big negate(Big a) { if (a.n) a.neg = !a.neg; return a; }
Big sub(const Big& a, const Big& b) { return add(a, negate(b)); }

Big mul(const Big& a, const Big& b) {
  Big r = big_zero();
  if (a.n == 0 || b.n == 0) return r;
  if (a.n + b.n > limb_budget()) { g_overflow = true; return r; }
  for (int i = 0; i < a.n; ++i) {
    unsigned __int128 carry = 0;
    for (int j = 0; j < b.n; ++j) {
      unsigned __int128 t = (unsigned __int128)a.d[i] * b.d[j] + r.d[i + j] + carry;
      r.d[i + j] = (uint64_t)t;
      carry = t >> 64;
    }
    r.d[i + b.n] = (uint64_t)carry;
  }
  r.n = a.n + b.n;
  r.neg = a.neg != b.neg;
  big_norm(r);
  return r;
}

inline int sgn(const Big& a) { return a.n == 0 ? 0 : (a.neg ? -1 : 1); }
inline int cmp(const Big& a, const Big& b) { return sgn(sub(a, b)); }

// ---- exact scaling of FP32 values ---------------------------------------

struct Dy { uint64_t m; bool neg; int e; };  // value = (neg?-1:1) * m * 2^e

Dy decompose(float x) {
  Dy r{0, false, 0};
  if (x == 0.0f) return r;
  int e;
  float f = std::frexp(x, &e);             // x = f * 2^e, 0.5 <= |f| < 1
  double m = std::ldexp((double)std::fabs(f), 24);  // exact: 24-bit integer
  r.m = (uint64_t)m;
  r.neg = x < 0;
  r.e = e - 24;
  return r;
}

struct V3 { Big x, y, z; };

V3 vsub(const V3& a, const V3& b) { return {sub(a.x, b.x), sub(a.y, b.y), sub(a.z, b.z)}; }
V3 cross(const V3& a, const V3& b) {
  return {sub(mul(a.y, b.z), mul(a.z, b.y)),
          sub(mul(a.z, b.x), mul(a.x, b.z)),
          sub(mul(a.x, b.y), mul(a.y, b.x))};
}
Big dot(const V3& a, const V3& b) { return add(add(mul(a.x, b.x), mul(a.y, b.y)), mul(a.z, b.z)); }
bool is_zero(const V3& a) { return a.x.n == 0 && a.y.n == 0 && a.z.n == 0; }

// Scale n points (3 floats each) to exact integers sharing one exponent.
void to_ints(const float* const* pts, int n, V3* out) {
  Dy dy[64];
  int emin = 1 << 20;
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k) {
      dy[3 * i + k] = decompose(pts[i][k]);
      if (dy[3 * i + k].m) emin = std::min(emin, dy[3 * i + k].e);
    }
  for (int i = 0; i < n; ++i) {
    Big c[3];
    for (int k = 0; k < 3; ++k) {
      const Dy& q = dy[3 * i + k];
      c[k] = q.m ? big_from(q.m, q.neg, q.e - emin) : big_zero();
    }
    out[i] = {c[0], c[1], c[2]};
  }
}

// Separating-axis test on one axis; pts relative to a common origin.
bool separates(const V3& L, const V3* T, const V3* U) {
  Big pt[3], pu[3];
  for (int i = 0; i < 3; ++i) { pt[i] = dot(L, T[i]); pu[i] = dot(L, U[i]); }
  auto mx = [](Big* p) { Big m = p[0]; for (int i = 1; i < 3; ++i) if (cmp(p[i], m) > 0) m = p[i]; return m; };
  auto mn = [](Big* p) { Big m = p[0]; for (int i = 1; i < 3; ++i) if (cmp(p[i], m) < 0) m = p[i]; return m; };
  if (cmp(mx(pt), mn(pu)) < 0) return true;
  if (cmp(mx(pu), mn(pt)) < 0) return true;
  return false;
}

std::atomic<uint64_t> g_tests{0};

// Exact test of a degenerate triangle: its three vertices are collinear
// (or coincide) iff the cross product of two edge vectors is exactly zero.
bool tri_degenerate(const float* t) {
  const float* pts[3] = {t, t + 3, t + 6};
  V3 X[3];
  to_ints(pts, 3, X);
  return is_zero(cross(vsub(X[1], X[0]), vsub(X[2], X[0])));
}

// 1 = closed triangles share a point, 0 = disjoint.  Both triangles must be
// non-degenerate (checked by the callers before this is reached).
int tri_tri_core(const float* t, const float* u) {
  // coordinate axes first: exact float comparisons
  for (int k = 0; k < 3; ++k) {
    float t0 = std::min(std::min(t[k], t[3 + k]), t[6 + k]);
    float t1 = std::max(std::max(t[k], t[3 + k]), t[6 + k]);
    float u0 = std::min(std::min(u[k], u[3 + k]), u[6 + k]);
    float u1 = std::max(std::max(u[k], u[3 + k]), u[6 + k]);
    if (t1 < u0 || u1 < t0) return 0;
  }
  const float* pts[6] = {t, t + 3, t + 6, u, u + 3, u + 6};
  V3 X[6];
  to_ints(pts, 6, X);
  V3 T[3], U[3];
  for (int i = 0; i < 3; ++i) { T[i] = vsub(X[i], X[0]); U[i] = vsub(X[3 + i], X[0]); }
  V3 et[3] = {vsub(T[1], T[0]), vsub(T[2], T[1]), vsub(T[0], T[2])};
  V3 eu[3] = {vsub(U[1], U[0]), vsub(U[2], U[1]), vsub(U[0], U[2])};
  V3 nt = cross(et[0], vsub(T[2], T[0]));
  V3 nu = cross(eu[0], vsub(U[2], U[0]));
  g_tests.fetch_add(1, std::memory_order_relaxed);
  if (separates(nt, T, U)) return 0;
  if (separates(nu, T, U)) return 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      V3 L = cross(et[i], eu[j]);
      if (!is_zero(L) && separates(L, T, U)) return 0;
    }
  for (int i = 0; i < 3; ++i) {
    V3 L = cross(nt, et[i]);
    if (separates(L, T, U)) return 0;
    L = cross(nu, eu[i]);
    if (separates(L, T, U)) return 0;
  }
  return 1;
}

// 1 = closed triangles share a point, 0 = disjoint, -3 = a degenerate input
// (decided first, whatever the triangles' positions).
int tri_tri(const float* t, const float* u) {
  if (tri_degenerate(t) || tri_degenerate(u)) return ORACLE_E_DEGENERATE;
  return tri_tri_core(t, u);
}

// ---- orientation signs (exported for predicate pins) ----------------------

int orient3d_sign(const float* a, const float* b, const float* c, const float* d) {
  const float* pts[4] = {a, b, c, d};
  V3 X[4];
  to_ints(pts, 4, X);
  return sgn(dot(cross(vsub(X[1], X[0]), vsub(X[2], X[0])), vsub(X[3], X[0])));
}

// ---- mesh level ---------------------------------------------------------

struct MeshView {
  const float* v; const int32_t* f; int64_t nv, nf;
};

struct TriBox { float lo[3], hi[3]; int32_t id; };

void tri_pts(const MeshView& m, int64_t i, float* out9) {
  for (int k = 0; k < 3; ++k) {
    int32_t vi = m.f[3 * i + k];
    for (int c = 0; c < 3; ++c) out9[3 * k + c] = m.v[3 * vi + c];
  }
}

TriBox tri_box(const MeshView& m, int64_t i) {
  float p[9];
  tri_pts(m, i, p);
  TriBox b;
  for (int c = 0; c < 3; ++c) {
    b.lo[c] = std::min(std::min(p[c], p[3 + c]), p[6 + c]);
    b.hi[c] = std::max(std::max(p[c], p[3 + c]), p[6 + c]);
  }
  b.id = (int32_t)i;
  return b;
}

bool boxes_meet(const float* alo, const float* ahi, const float* blo, const float* bhi) {
  for (int c = 0; c < 3; ++c)
    if (ahi[c] < blo[c] || bhi[c] < alo[c]) return false;
  return true;
}

bool mesh_valid(const MeshView& m) {
  for (int64_t i = 0; i < 3 * m.nf; ++i)
    if (m.f[i] < 0 || m.f[i] >= m.nv) return false;
  for (int64_t i = 0; i < 3 * m.nv; ++i)
    if (!std::isfinite(m.v[i])) return false;
  return true;
}

// 0 if every triangle of the mesh is non-degenerate, else ORACLE_E_DEGENERATE.
int mesh_degenerate(const MeshView& m) {
  float t[9];
  for (int64_t i = 0; i < m.nf; ++i) {
    tri_pts(m, i, t);
    if (tri_degenerate(t)) return ORACLE_E_DEGENERATE;
  }
  return 0;
}

// Both meshes have been checked for degenerate triangles; returns 1 / 0.
int pair_brute(const MeshView& A, const MeshView& B) {
  float t[9], u[9];
  for (int64_t i = 0; i < A.nf; ++i) {
    tri_pts(A, i, t);
    for (int64_t j = 0; j < B.nf; ++j) {
      tri_pts(B, j, u);
      int r = tri_tri_core(t, u);
      if (r != 0) return r;
    }
  }
  return 0;
}

int pair_pruned(const MeshView& A, const MeshView& B) {
  std::vector<TriBox> ba(A.nf), bb(B.nf);
  float alo[3] = {INFINITY, INFINITY, INFINITY}, ahi[3] = {-INFINITY, -INFINITY, -INFINITY};
  float blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = 0; i < A.nf; ++i) {
    ba[i] = tri_box(A, i);
    for (int c = 0; c < 3; ++c) { alo[c] = std::min(alo[c], ba[i].lo[c]); ahi[c] = std::max(ahi[c], ba[i].hi[c]); }
  }
  for (int64_t j = 0; j < B.nf; ++j) {
    bb[j] = tri_box(B, j);
    for (int c = 0; c < 3; ++c) { blo[c] = std::min(blo[c], bb[j].lo[c]); bhi[c] = std::max(bhi[c], bb[j].hi[c]); }
  }
  if (A.nf == 0 || B.nf == 0 || !boxes_meet(alo, ahi, blo, bhi)) return 0;
  std::vector<TriBox> sa, sb;
  for (auto& b : ba) if (boxes_meet(b.lo, b.hi, blo, bhi)) sa.push_back(b);
  for (auto& b : bb) if (boxes_meet(b.lo, b.hi, alo, ahi)) sb.push_back(b);
  auto by_x = [](const TriBox& p, const TriBox& q) { return p.lo[0] < q.lo[0] || (p.lo[0] == q.lo[0] && p.id < q.id); };
  std::sort(sa.begin(), sa.end(), by_x);
  std::sort(sb.begin(), sb.end(), by_x);
  float t[9], u[9];
  size_t i = 0, j = 0;
  while (i < sa.size() && j < sb.size()) {
    if (sa[i].lo[0] <= sb[j].lo[0]) {
      const TriBox& a = sa[i];
      for (size_t k = j; k < sb.size() && sb[k].lo[0] <= a.hi[0]; ++k) {
        if (!boxes_meet(a.lo, a.hi, sb[k].lo, sb[k].hi)) continue;
        tri_pts(A, a.id, t); tri_pts(B, sb[k].id, u);
        int r = tri_tri_core(t, u);
        if (r != 0) return r;
      }
      ++i;
    } else {
      const TriBox& b = sb[j];
      for (size_t k = i; k < sa.size() && sa[k].lo[0] <= b.hi[0]; ++k) {
        if (!boxes_meet(b.lo, b.hi, sa[k].lo, sa[k].hi)) continue;
        tri_pts(A, sa[k].id, t); tri_pts(B, b.id, u);
        int r = tri_tri_core(t, u);
        if (r != 0) return r;
      }
      ++j;
    }
  }
  return 0;
}

MeshView view(const float* v, const int32_t* f, const int64_t* vo, const int64_t* fo, int64_t m) {
  return {v + 3 * vo[m], f + 3 * fo[m], vo[m + 1] - vo[m], fo[m + 1] - fo[m]};
}

// ---- point in mesh (containment, Section 3.3) ----------------------------
//
// Winding number of a closed triangle mesh about a point p, computed
// exactly: cast the ray p + t d (t > 0) along an integer direction d and add,
// for every triangle it crosses through the triangle's interior, the sign of
// n . d, n = (b - a) x (c - a).  The line meets the interior iff the triple
// products [a-p, b-p, d], [b-p, c-p, d], [c-p, a-p, d] share one strict sign;
// the crossing lies ahead of p iff orient(a,b,c,p) and n . d have opposite
// signs.  When the line meets an edge or a vertex of a triangle, or lies in a
// triangle's plane, the direction is degenerate for this point and mesh and
// the next direction of a fixed list is used.  A point on a triangle is
// reported as such.  For an embedded closed surface with outward faces the
// winding number is 1 inside and 0 outside.

enum { ORACLE_ON_SURFACE = 2, ORACLE_E_RAY = -7 };

const int kDirs[16][3] = {{1, 2, 3},   {-3, 1, 2},  {2, -1, 5},  {5, 3, -7}, {-2, 7, 1},  {7, -5, 3},
                          {3, 11, -2}, {-13, 4, 9}, {1, -9, -4}, {6, 1, 13}, {-5, -8, 3}, {11, 2, 6},
                          {-1, 17, 5}, {4, -3, -11}, {9, 13, 2}, {-7, -2, -15}};

V3 dir_vec(const int* d) {
  return {big_from((uint64_t)std::abs(d[0]), d[0] < 0, 0), big_from((uint64_t)std::abs(d[1]), d[1] < 0, 0),
          big_from((uint64_t)std::abs(d[2]), d[2] < 0, 0)};
}

// One triangle against the ray from p along d: sets *contrib to +-1 for a
// crossing ahead of p, 0 otherwise; returns 1 when the direction is
// degenerate for this triangle, 2 when p lies on the triangle, else 0.
int ray_triangle(const float* p, const float* t, const V3& D, int* contrib) {
  *contrib = 0;
  const float* pts[4] = {p, t, t + 3, t + 6};
  V3 X[4];
  to_ints(pts, 4, X);
  const V3 A = vsub(X[1], X[0]), B = vsub(X[2], X[0]), C = vsub(X[3], X[0]);  // a-p, b-p, c-p
  const int e1 = sgn(dot(cross(A, B), D)), e2 = sgn(dot(cross(B, C), D)), e3 = sgn(dot(cross(C, A), D));
  const V3 n = cross(vsub(X[2], X[1]), vsub(X[3], X[1]));
  const int f0 = sgn(dot(n, vsub(X[0], X[1])));  // orient(a,b,c,p)
  if (f0 == 0) {
    // p in the triangle's plane: on the triangle iff the 2D tests pass in a
    // coordinate plane where the normal component is non-zero
    int i = 1, j = 2;
    if (n.x.n == 0) { i = 2; j = 0; if (n.y.n == 0) { i = 0; j = 1; } }
    auto o2 = [&](const V3& u, const V3& v, const V3& w) {
      const Big* U[3] = {&u.x, &u.y, &u.z};
      const Big* Vv[3] = {&v.x, &v.y, &v.z};
      const Big* Ww[3] = {&w.x, &w.y, &w.z};
      return sgn(sub(mul(sub(*Vv[i], *U[i]), sub(*Ww[j], *U[j])), mul(sub(*Vv[j], *U[j]), sub(*Ww[i], *U[i]))));
    };
    const int s1 = o2(X[1], X[2], X[0]), s2 = o2(X[2], X[3], X[0]), s3 = o2(X[3], X[1], X[0]);
    if ((s1 >= 0 && s2 >= 0 && s3 >= 0) || (s1 <= 0 && s2 <= 0 && s3 <= 0)) return 2;
  }
  const bool pos = e1 > 0 || e2 > 0 || e3 > 0, neg = e1 < 0 || e2 < 0 || e3 < 0;
  if (pos && neg) return 0;                  // the line misses the closed triangle
  if (e1 == 0 || e2 == 0 || e3 == 0) return 1;  // through an edge or a vertex, or in the plane
  const int nd = sgn(dot(n, D));
  if (nd == 0) return 1;
  if (f0 != 0 && f0 == -nd) *contrib = nd;   // the crossing is ahead of p
  return 0;
}

// Winding number of mesh m about p, or ORACLE_ON_SURFACE (as *on = 1), or an
// error when every direction of the list is degenerate.  Directions are tried
// from kDirs[first] on (cyclically).
int winding(const MeshView& m, const float* p, int* w, int* on, int first = 0) {
  float t[9];
  *on = 0;
  for (int kk = 0; kk < 16; ++kk) {
    const V3 D = dir_vec(kDirs[(first + kk) % 16]);
    int sum = 0;
    bool degenerate = false;
    for (int64_t i = 0; i < m.nf && !degenerate; ++i) {
      tri_pts(m, i, t);
      int c = 0;
      const int r = ray_triangle(p, t, D, &c);
      if (r == 2) { *on = 1; *w = 0; return 0; }
      if (r == 1) degenerate = true;
      sum += c;
    }
    if (!degenerate) { *w = sum; return 0; }
  }
  return ORACLE_E_RAY;
}

}  // namespace

extern "C" {

int oracle_tri_tri(const float* t9, const float* u9) {
  g_overflow = false;
  int r = tri_tri(t9, u9);
  return g_overflow ? ORACLE_E_OVERFLOW : r;
}

// Test hook: limbs a value may use (1..LIMBS); returns the previous budget.
// Lowering it makes large intermediate values overflow on purpose, so that a
// test can see the overflow reported instead of a wrong answer.
int oracle_set_limb_budget(int limbs) {
  if (limbs < 1 || limbs > LIMBS) return ORACLE_E_ARG;
  return g_limb_budget.exchange(limbs);
}

// Winding number of mesh m of a set (verts, faces, offsets) about point p,
// trying the ray directions from number first_dir on; *on_surface = 1 when p
// lies on one of its triangles.  Returns 0 or an error.
int oracle_winding(const float* v, const int32_t* f, const int64_t* vo, const int64_t* fo, int64_t nm, int64_t m,
                   const float* p, int first_dir, int32_t* w, int32_t* on_surface) {
  if (m < 0 || m >= nm || !p || !w || !on_surface || first_dir < 0 || first_dir >= 16) return ORACLE_E_ARG;
  MeshView M = view(v, f, vo, fo, m);
  if (!mesh_valid(M)) return ORACLE_E_ARG;
  g_overflow = false;
  int ww = 0, on = 0;
  const int r = winding(M, p, &ww, &on, first_dir);
  if (g_overflow) return ORACLE_E_OVERFLOW;
  *w = ww;
  *on_surface = on;
  return r;
}

// Per candidate pair (i, j): bit 0 = the first vertex of B_j's first face lies
// inside A_i (winding number non-zero), bit 1 = the first vertex of A_i's first
// face lies inside B_j; bit 2 / bit 3 = that vertex lies on the other surface
// (bits 0 / 1 are then 0).  A mesh without faces has no such vertex: 0.
int oracle_inside_pairs(const float* va, const int32_t* fa, const int64_t* voa, const int64_t* foa, int64_t ma,
                        const float* vb, const int32_t* fb, const int64_t* vob, const int64_t* fob, int64_t mb,
                        const int32_t* pairs, int64_t n_pairs, uint8_t* bits, int n_threads) {
  if (n_pairs < 0 || (n_pairs > 0 && (!pairs || !bits)) || ma < 0 || mb < 0) return ORACLE_E_ARG;
  for (int64_t p = 0; p < n_pairs; ++p)
    if (pairs[2 * p] < 0 || pairs[2 * p] >= ma || pairs[2 * p + 1] < 0 || pairs[2 * p + 1] >= mb) return ORACLE_E_ARG;
  for (int64_t m = 0; m < ma; ++m) if (!mesh_valid(view(va, fa, voa, foa, m))) return ORACLE_E_ARG;
  for (int64_t m = 0; m < mb; ++m) if (!mesh_valid(view(vb, fb, vob, fob, m))) return ORACLE_E_ARG;
  std::atomic<int64_t> next{0};
  std::atomic<int> status{0};
  auto rep = [](const MeshView& m, float* out) {
    const int32_t vi = m.f[0];
    for (int c = 0; c < 3; ++c) out[c] = m.v[3 * vi + c];
  };
  auto worker = [&]() {
    for (;;) {
      const int64_t p = next.fetch_add(1);
      if (p >= n_pairs) break;
      const MeshView A = view(va, fa, voa, foa, pairs[2 * p]);
      const MeshView B = view(vb, fb, vob, fob, pairs[2 * p + 1]);
      uint8_t b = 0;
      g_overflow = false;
      float q[3];
      int w = 0, on = 0;
      if (A.nf > 0 && B.nf > 0) {
        rep(B, q);
        int r = winding(A, q, &w, &on);
        if (r) status.store(r);
        if (on) b |= 4; else if (w != 0) b |= 1;
        rep(A, q);
        r = winding(B, q, &w, &on);
        if (r) status.store(r);
        if (on) b |= 8; else if (w != 0) b |= 2;
      }
      if (g_overflow) status.store(ORACLE_E_OVERFLOW);
      bits[p] = b;
    }
  };
  int nt = n_threads > 0 ? n_threads : (int)std::max(1u, std::thread::hardware_concurrency());
  std::vector<std::thread> pool;
  for (int i = 0; i < nt; ++i) pool.emplace_back(worker);
  for (auto& th : pool) th.join();
  return status.load();
}

int oracle_orient3d(const float* a, const float* b, const float* c, const float* d) {
  g_overflow = false;
  int r = orient3d_sign(a, b, c, d);
  return g_overflow ? ORACLE_E_OVERFLOW : r;
}

// flags[p] = 1 iff meshes A[pairs[p][0]] and B[pairs[p][1]] share a point.
// mode 0: all triangle pairs; mode 1: exact box sweep-and-prune first.
// Returns 0, or a negative code; *n_tests receives the exact triangle tests run.
int oracle_join(const float* va, const int32_t* fa, const int64_t* voa, const int64_t* foa, int64_t ma,
                const float* vb, const int32_t* fb, const int64_t* vob, const int64_t* fob, int64_t mb,
                const int32_t* pairs, int64_t n_pairs, uint8_t* flags, int mode, int n_threads,
                uint64_t* n_tests) {
  if (n_pairs < 0 || (n_pairs > 0 && (!pairs || !flags)) || ma < 0 || mb < 0) return ORACLE_E_ARG;
  for (int64_t p = 0; p < n_pairs; ++p)
    if (pairs[2 * p] < 0 || pairs[2 * p] >= ma || pairs[2 * p + 1] < 0 || pairs[2 * p + 1] >= mb)
      return ORACLE_E_ARG;
  for (int64_t m = 0; m < ma; ++m) if (!mesh_valid(view(va, fa, voa, foa, m))) return ORACLE_E_ARG;
  for (int64_t m = 0; m < mb; ++m) if (!mesh_valid(view(vb, fb, vob, fob, m))) return ORACLE_E_ARG;
  g_tests.store(0);
  // Degenerate triangles are refused for every pair that holds their mesh,
  // whatever the triangles' positions (each mesh is checked once, on first use).
  std::vector<std::atomic<int>> okA(ma), okB(mb);  // 0 unchecked, 1 valid, 2 degenerate
  for (auto& x : okA) x.store(0);
  for (auto& x : okB) x.store(0);
  auto checked = [](std::atomic<int>& st, const MeshView& m) {
    int v = st.load();
    if (v == 0) {
      v = mesh_degenerate(m) == 0 ? 1 : 2;
      st.store(v);
    }
    return v == 1;
  };
  std::atomic<int64_t> next{0};
  std::atomic<int> status{0};
  auto worker = [&]() {
    for (;;) {
      int64_t p = next.fetch_add(1);
      if (p >= n_pairs) break;
      MeshView A = view(va, fa, voa, foa, pairs[2 * p]);
      MeshView B = view(vb, fb, vob, fob, pairs[2 * p + 1]);
      g_overflow = false;
      int r;
      if (!checked(okA[pairs[2 * p]], A) || !checked(okB[pairs[2 * p + 1]], B)) r = ORACLE_E_DEGENERATE;
      else r = mode == 0 ? pair_brute(A, B) : pair_pruned(A, B);
      if (g_overflow) r = ORACLE_E_OVERFLOW;
      if (r < 0) { status.store(r); flags[p] = 0; }
      else flags[p] = (uint8_t)r;
    }
  };
  int nt = n_threads > 0 ? n_threads : (int)std::max(1u, std::thread::hardware_concurrency());
  std::vector<std::thread> pool;
  for (int i = 0; i < nt; ++i) pool.emplace_back(worker);
  for (auto& th : pool) th.join();
  if (n_tests) *n_tests = g_tests.load();
  return status.load();
}

}  // extern "C"
