// Device predicates for the closed segment-triangle test at BVH leaves
// (Section 3.1 Step II: a hit within the edge's extent means the edge
// pierces a face; here read with closed sets, so touching counts).
//
// Three tiers:
//  1. FP32 filter.  Each orientation determinant det[u, v, w] is evaluated as
//     w . (u x v) in FP32 from rounded coordinate differences, with no fused
//     multiply-add.  Its rounding error is below 8 eps * perm + O(eps^2),
//     perm = sum_k |w_k| (|u_i v_j| + |u_j v_i|), eps = 2^-24; we certify a
//     sign only when |det| > 2^-20 perm + 2^-100.  The absolute term covers
//     underflow; the bound holds when every coordinate is 0 or within
//     [2^-40, 2^40] (the "FP32-safe" range, checked per mesh at build time).
//  2. FP64 filter: the same expression in FP64 (eps = 2^-53), certified when
//     |det| > 2^-49 perm.  FP32 inputs cannot overflow or underflow there.
//  2'. Grid: let e be the exponent of the lowest set bit over the fifteen
//     coordinates of a test and h the exponent of the highest; when
//     h - e <= 14, every coordinate difference is an integer below 2^16
//     units of 2^e and is exact in FP32, a product of two is exact in FP64
//     (48-bit operands' product, below 2^32 units), a cross-product component
//     (below 2^33) and a determinant (below 3 * 2^49 units) are exact in
//     FP64, so the signs are exact.  Cheap, so the FP32 traversal decides
//     such tests in place.
//  3. Exact: the determinant expanded into 24 products of three FP32
//     coordinates; each product is an exact pair of doubles (the first
//     product of two FP32 values is exact, the second uses an FMA-based
//     error-free product) and the 48 doubles are summed exactly into a
//     nonoverlapping expansion by repeated Two-Sum (Shewchuk 1997, "Adaptive
//     precision floating-point arithmetic and fast robust geometric
//     predicates").  The sign of the largest component is the exact sign.
//
// Closed segment [p,q] vs closed triangle (a,b,c), non-degenerate triangle:
//  s_p = orient(a,b,c,p), s_q = orient(a,b,c,q)
//  both of one strict sign           -> miss
//  both zero (segment in the plane)  -> 2D separating-axis test in a
//      coordinate projection where the triangle's normal component is
//      non-zero: separated iff a,b,c lie strictly on one side of line pq, or
//      p and q lie strictly outside one edge line (opposite the third vertex)
//  otherwise the segment meets the plane in one point, which lies in the
//      closed triangle iff orient(p,q,a,b), orient(p,q,b,c), orient(p,q,c,a)
//      are all >= 0 or all <= 0.
// orient(x1,x2,x3,x4) = det[x2-x1, x3-x1, x4-x1] throughout.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pr {

struct f3 {
  float x, y, z;
};

enum { kMiss = 0, kHit = 1, kAmbig = 2 };

constexpr float kRel32 = 0x1p-20f;
constexpr float kAbs32 = 0x1p-100f;
constexpr double kRel64 = 0x1p-49;

__device__ __forceinline__ float get(const f3& v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }

// ---------------------------------------------------------------- tier 1: FP32

// det[u, v, w] given u, v, w (already rounded differences); returns value and permanent.
__device__ __forceinline__ void det3_f32(float ux, float uy, float uz, float vx, float vy, float vz,
                                         float wx, float wy, float wz, float& det, float& perm) {
  float m1 = uy * vz, m2 = uz * vy;
  float m3 = uz * vx, m4 = ux * vz;
  float m5 = ux * vy, m6 = uy * vx;
  float nx = m1 - m2, ny = m3 - m4, nz = m5 - m6;
  det = (wx * nx + wy * ny) + wz * nz;
  perm = (fabsf(wx) * (fabsf(m1) + fabsf(m2)) + fabsf(wy) * (fabsf(m3) + fabsf(m4))) +
         fabsf(wz) * (fabsf(m5) + fabsf(m6));
}

__device__ __forceinline__ bool certain32(float det, float perm) {
  return fabsf(det) > kRel32 * perm + kAbs32;
}

// FP32 filter of the closed segment-triangle test: kMiss, kHit or kAmbig.
// Only valid for FP32-safe coordinates.
__device__ __forceinline__ int seg_tri_f32(f3 p, f3 q, f3 a, f3 b, f3 c) {
  float ux = b.x - a.x, uy = b.y - a.y, uz = b.z - a.z;
  float vx = c.x - a.x, vy = c.y - a.y, vz = c.z - a.z;
  // normal and its permanent weights, shared by the two endpoint tests
  float m1 = uy * vz, m2 = uz * vy;
  float m3 = uz * vx, m4 = ux * vz;
  float m5 = ux * vy, m6 = uy * vx;
  float nx = m1 - m2, ny = m3 - m4, nz = m5 - m6;
  float ax = fabsf(m1) + fabsf(m2), ay = fabsf(m3) + fabsf(m4), az = fabsf(m5) + fabsf(m6);
  float px = p.x - a.x, py = p.y - a.y, pz = p.z - a.z;
  float qx = q.x - a.x, qy = q.y - a.y, qz = q.z - a.z;
  float sp = (px * nx + py * ny) + pz * nz;
  float pp = (fabsf(px) * ax + fabsf(py) * ay) + fabsf(pz) * az;
  float sq = (qx * nx + qy * ny) + qz * nz;
  float pq = (fabsf(qx) * ax + fabsf(qy) * ay) + fabsf(qz) * az;
  bool cp = certain32(sp, pp), cq = certain32(sq, pq);
  if (cp && cq && ((sp > 0.f) == (sq > 0.f))) return kMiss;
  // line pq against the three directed edges
  float dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
  float apx = a.x - p.x, apy = a.y - p.y, apz = a.z - p.z;
  float bpx = b.x - p.x, bpy = b.y - p.y, bpz = b.z - p.z;
  float cpx = c.x - p.x, cpy = c.y - p.y, cpz = c.z - p.z;
  float o1, e1, o2, e2, o3, e3;
  det3_f32(dx, dy, dz, apx, apy, apz, bpx, bpy, bpz, o1, e1);  // orient(p,q,a,b)
  det3_f32(dx, dy, dz, bpx, bpy, bpz, cpx, cpy, cpz, o2, e2);  // orient(p,q,b,c)
  det3_f32(dx, dy, dz, cpx, cpy, cpz, apx, apy, apz, o3, e3);  // orient(p,q,c,a)
  bool c1 = certain32(o1, e1), c2 = certain32(o2, e2), c3 = certain32(o3, e3);
  bool pos = (c1 && o1 > 0.f) || (c2 && o2 > 0.f) || (c3 && o3 > 0.f);
  bool neg = (c1 && o1 < 0.f) || (c2 && o2 < 0.f) || (c3 && o3 < 0.f);
  if (pos && neg) return kMiss;
  if (c1 && c2 && c3 && cp && cq && ((sp > 0.f) != (sq > 0.f))) return kHit;
  return kAmbig;
}

// ---------------------------------------------------------------- grid tier

// Exponents of the lowest and of the highest set bit of a non-zero FP32
// value (|x| < 2^(high + 1)).
__device__ __forceinline__ int low_exp(float x) {
  const uint32_t b = __float_as_uint(x) & 0x7fffffffu;
  const uint32_t e = b >> 23, m = b & 0x7fffffu;
  if (e == 0) return -149 + __builtin_ctz(m);            // subnormal: m * 2^-149
  return (int)e - 150 + __builtin_ctz(m | 0x800000u);    // (2^23 + m) * 2^(e - 150)
}
__device__ __forceinline__ int high_exp(float x) {
  const uint32_t b = __float_as_uint(x) & 0x7fffffffu;
  const uint32_t e = b >> 23, m = b & 0x7fffffu;
  if (e == 0) return -149 + (31 - __builtin_clz(m));
  return (int)e - 127;
}

__device__ __forceinline__ void span(float x, int& lo, int& hi) {
  if (x != 0.f) {
    lo = min(lo, low_exp(x));
    hi = max(hi, high_exp(x));
  }
}

// Exact sign of det[b-a, c-a, d-a] on a grid of span <= 14 (see above).
__device__ __forceinline__ int gsign3(f3 a, f3 b, f3 c, f3 d) {
  const float ux = b.x - a.x, uy = b.y - a.y, uz = b.z - a.z;
  const float vx = c.x - a.x, vy = c.y - a.y, vz = c.z - a.z;
  const float wx = d.x - a.x, wy = d.y - a.y, wz = d.z - a.z;
  const double nx = (double)uy * vz - (double)uz * vy;
  const double ny = (double)uz * vx - (double)ux * vz;
  const double nz = (double)ux * vy - (double)uy * vx;
  const double det = ((double)wx * nx + (double)wy * ny) + (double)wz * nz;
  return (det > 0.0) - (det < 0.0);
}

// Exact sign of det[b-a, c-a] in the coordinate plane (i, j), same grid.
__device__ __forceinline__ int gsign2(f3 a, f3 b, f3 c, int i, int j) {
  const double det = (double)(get(b, i) - get(a, i)) * (get(c, j) - get(a, j)) -
                     (double)(get(b, j) - get(a, j)) * (get(c, i) - get(a, i));
  return (det > 0.0) - (det < 0.0);
}

// Exact closed segment-triangle decision when the five points lie on a grid
// of span <= 14 (see above); kAmbig when they do not.  Same decision
// procedure as seg_tri_exact.  Not inlined: the traversal calls it only for
// tests the FP32 filter leaves open, and its registers stay out of the loop.
__device__ __noinline__ int seg_tri_grid(f3 p, f3 q, f3 a, f3 b, f3 c) {
  int lo = 1 << 20, hi = -(1 << 20);
  span(p.x, lo, hi); span(p.y, lo, hi); span(p.z, lo, hi);
  span(q.x, lo, hi); span(q.y, lo, hi); span(q.z, lo, hi);
  span(a.x, lo, hi); span(a.y, lo, hi); span(a.z, lo, hi);
  span(b.x, lo, hi); span(b.y, lo, hi); span(b.z, lo, hi);
  span(c.x, lo, hi); span(c.y, lo, hi); span(c.z, lo, hi);
  if (hi - lo > 14) return kAmbig;
  const int sp = gsign3(a, b, c, p), sq = gsign3(a, b, c, q);
  if (sp != 0 && sp == sq) return kMiss;
  if (sp == 0 && sq == 0) {
    int i = 1, j = 2;
    if (gsign2(a, b, c, 1, 2) == 0) {
      i = 2; j = 0;
      if (gsign2(a, b, c, 2, 0) == 0) { i = 0; j = 1; }
    }
    const int s1 = gsign2(p, q, a, i, j), s2 = gsign2(p, q, b, i, j), s3 = gsign2(p, q, c, i, j);
    if ((s1 > 0 && s2 > 0 && s3 > 0) || (s1 < 0 && s2 < 0 && s3 < 0)) return kMiss;
    // p and q strictly outside one edge line (opposite the third vertex)
    int sz = gsign2(a, b, c, i, j);
    if (gsign2(a, b, p, i, j) == -sz && gsign2(a, b, q, i, j) == -sz) return kMiss;
    sz = gsign2(b, c, a, i, j);
    if (gsign2(b, c, p, i, j) == -sz && gsign2(b, c, q, i, j) == -sz) return kMiss;
    sz = gsign2(c, a, b, i, j);
    if (gsign2(c, a, p, i, j) == -sz && gsign2(c, a, q, i, j) == -sz) return kMiss;
    return kHit;
  }
  const int o1 = gsign3(p, q, a, b), o2 = gsign3(p, q, b, c), o3 = gsign3(p, q, c, a);
  return ((o1 >= 0 && o2 >= 0 && o3 >= 0) || (o1 <= 0 && o2 <= 0 && o3 <= 0)) ? kHit : kMiss;
}

// ---------------------------------------------------------------- tier 3: exact

constexpr int kExpMax = 48;

struct Expansion {
  double e[kExpMax];  // nonoverlapping, increasing magnitude, no zeros
  int n;
};

__device__ __forceinline__ void two_sum(double a, double b, double& s, double& err) {
  s = a + b;
  double bv = s - a;
  double av = s - bv;
  err = (a - av) + (b - bv);
}

// e <- e + b, exactly (Grow-Expansion with zero elimination).
__device__ __forceinline__ void grow(Expansion& x, double b) {
  double q = b;
  int k = 0;
  for (int i = 0; i < x.n; ++i) {
    double s, h;
    two_sum(q, x.e[i], s, h);
    if (h != 0.0) x.e[k++] = h;
    q = s;
  }
  if (q != 0.0) x.e[k++] = q;
  x.n = k;
}

// e <- e + s*x*y*z exactly, for FP32 x, y, z and s = +-1.
__device__ __forceinline__ void add_prod3(Expansion& e, double s, float x, float y, float z) {
  double xy = ((double)x * (double)y) * s;  // exact: 48-bit product
  double hi = xy * (double)z;
  double lo = fma(xy, (double)z, -hi);     // exact remainder
  grow(e, lo);
  grow(e, hi);
}

__device__ __forceinline__ int exp_sign(const Expansion& e) {
  return e.n == 0 ? 0 : (e.e[e.n - 1] > 0.0 ? 1 : -1);
}

// s * x.(y cross z)
__device__ __forceinline__ void add_det3(Expansion& e, double s, f3 x, f3 y, f3 z) {
  add_prod3(e, s, x.x, y.y, z.z);
  add_prod3(e, -s, x.x, y.z, z.y);
  add_prod3(e, s, x.y, y.z, z.x);
  add_prod3(e, -s, x.y, y.x, z.z);
  add_prod3(e, s, x.z, y.x, z.y);
  add_prod3(e, -s, x.z, y.y, z.x);
}

// Exact sign of orient(a,b,c,d) = det[b-a, c-a, d-a]
//   = det(b,c,d) - det(a,c,d) + det(a,b,d) - det(a,b,c).
__device__ __noinline__ int orient3d_exact(f3 a, f3 b, f3 c, f3 d) {
  Expansion e;
  e.n = 0;
  add_det3(e, 1.0, b, c, d);
  add_det3(e, -1.0, a, c, d);
  add_det3(e, 1.0, a, b, d);
  add_det3(e, -1.0, a, b, c);
  return exp_sign(e);
}

// Exact sign of det[b-a, c-a] in the coordinate plane (i, j)
//   = det(b,c) - det(a,c) + det(a,b), det(x,y) = x_i y_j - x_j y_i.
__device__ __noinline__ int orient2d_exact(f3 a, f3 b, f3 c, int i, int j) {
  Expansion e;
  e.n = 0;
  float ai = get(a, i), aj = get(a, j), bi = get(b, i), bj = get(b, j), ci = get(c, i), cj = get(c, j);
  grow(e, (double)bi * (double)cj);
  grow(e, -((double)bj * (double)ci));
  grow(e, -((double)ai * (double)cj));
  grow(e, (double)aj * (double)ci);
  grow(e, (double)ai * (double)bj);
  grow(e, -((double)aj * (double)bi));
  return exp_sign(e);
}

// ---------------------------------------------------------------- tier 2: FP64

struct ExactCounters {
  uint32_t exact_signs;  // signs the FP64 bound could not certify
};

__device__ __forceinline__ int sign_orient3d(f3 a, f3 b, f3 c, f3 d, ExactCounters& cnt) {
  double ux = (double)b.x - a.x, uy = (double)b.y - a.y, uz = (double)b.z - a.z;
  double vx = (double)c.x - a.x, vy = (double)c.y - a.y, vz = (double)c.z - a.z;
  double wx = (double)d.x - a.x, wy = (double)d.y - a.y, wz = (double)d.z - a.z;
  double m1 = uy * vz, m2 = uz * vy, m3 = uz * vx, m4 = ux * vz, m5 = ux * vy, m6 = uy * vx;
  double det = (wx * (m1 - m2) + wy * (m3 - m4)) + wz * (m5 - m6);
  double perm = (fabs(wx) * (fabs(m1) + fabs(m2)) + fabs(wy) * (fabs(m3) + fabs(m4))) +
                fabs(wz) * (fabs(m5) + fabs(m6));
  if (fabs(det) > kRel64 * perm) return det > 0.0 ? 1 : -1;
  cnt.exact_signs++;
  return orient3d_exact(a, b, c, d);
}

__device__ __forceinline__ int sign_orient2d(f3 a, f3 b, f3 c, int i, int j, ExactCounters& cnt) {
  double ui = (double)get(b, i) - get(a, i), uj = (double)get(b, j) - get(a, j);
  double vi = (double)get(c, i) - get(a, i), vj = (double)get(c, j) - get(a, j);
  double m1 = ui * vj, m2 = uj * vi;
  double det = m1 - m2;
  double perm = fabs(m1) + fabs(m2);
  if (fabs(det) > kRel64 * perm) return det > 0.0 ? 1 : -1;
  cnt.exact_signs++;
  return orient2d_exact(a, b, c, i, j);
}

// Exact closed segment-triangle decision (FP64 filter, then exact).
__device__ __noinline__ bool seg_tri_exact(f3 p, f3 q, f3 a, f3 b, f3 c, ExactCounters& cnt) {
  int sp = sign_orient3d(a, b, c, p, cnt);
  int sq = sign_orient3d(a, b, c, q, cnt);
  if (sp != 0 && sp == sq) return false;
  if (sp == 0 && sq == 0) {
    // coplanar: project along an axis where the normal component is non-zero
    int i = 1, j = 2;  // normal x = det over (y, z)
    if (sign_orient2d(a, b, c, 1, 2, cnt) == 0) {
      i = 2; j = 0;    // normal y = det over (z, x)
      if (sign_orient2d(a, b, c, 2, 0, cnt) == 0) { i = 0; j = 1; }
    }
    int s1 = sign_orient2d(p, q, a, i, j, cnt);
    int s2 = sign_orient2d(p, q, b, i, j, cnt);
    int s3 = sign_orient2d(p, q, c, i, j, cnt);
    if ((s1 > 0 && s2 > 0 && s3 > 0) || (s1 < 0 && s2 < 0 && s3 < 0)) return false;
    f3 v[3] = {a, b, c};
    for (int k = 0; k < 3; ++k) {
      f3 x = v[k], y = v[(k + 1) % 3], z = v[(k + 2) % 3];
      int sz = sign_orient2d(x, y, z, i, j, cnt);
      int t1 = sign_orient2d(x, y, p, i, j, cnt);
      int t2 = sign_orient2d(x, y, q, i, j, cnt);
      if (t1 == -sz && t2 == -sz) return false;
    }
    return true;
  }
  int o1 = sign_orient3d(p, q, a, b, cnt);
  int o2 = sign_orient3d(p, q, b, c, cnt);
  int o3 = sign_orient3d(p, q, c, a, cnt);
  return (o1 >= 0 && o2 >= 0 && o3 >= 0) || (o1 <= 0 && o2 <= 0 && o3 <= 0);
}

}  // namespace pr
