// Device-side renderer rules (Section 3.3.1) in binary32, every operation in a
// fixed order with explicit fma, so that the triangle and texel decisions are
// reproducible bit for bit by any implementation that follows the same rules.
// Built with -ffp-contract=off; HIP's float division and sqrt are correctly
// rounded by default.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lf {

// Camera record: fx fy cx cy R[9] (row-major, world -> camera) t[3].
struct Cam {
  float fx, fy, cx, cy;
  float r[9];
  float t[3];
};

struct V3 {
  float x, y, z;
};

__device__ __forceinline__ Cam load_cam(const float* __restrict__ p) {
  Cam c;
  c.fx = p[0]; c.fy = p[1]; c.cx = p[2]; c.cy = p[3];
#pragma unroll
  for (int i = 0; i < 9; ++i) c.r[i] = p[4 + i];
  c.t[0] = p[13]; c.t[1] = p[14]; c.t[2] = p[15];
  return c;
}

// X_cam = R X + t, each row as R0*X + (R1*Y + (R2*Z + t)) with fused steps.
__device__ __forceinline__ V3 to_cam(const Cam& c, float X, float Y, float Z) {
  V3 o;
  o.x = __builtin_fmaf(c.r[0], X, __builtin_fmaf(c.r[1], Y, __builtin_fmaf(c.r[2], Z, c.t[0])));
  o.y = __builtin_fmaf(c.r[3], X, __builtin_fmaf(c.r[4], Y, __builtin_fmaf(c.r[5], Z, c.t[1])));
  o.z = __builtin_fmaf(c.r[6], X, __builtin_fmaf(c.r[7], Y, __builtin_fmaf(c.r[8], Z, c.t[2])));
  return o;
}

__device__ __forceinline__ V3 sub3(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }

// a x b, every component as a1*b2 - a2*b1 = fma(a1, b2, -(a2*b1)).
__device__ __forceinline__ V3 cross3(V3 a, V3 b) {
  return V3{__builtin_fmaf(a.y, b.z, -(a.z * b.y)), __builtin_fmaf(a.z, b.x, -(a.x * b.z)),
            __builtin_fmaf(a.x, b.y, -(a.y * b.x))};
}

// a . b = a0*b0 + (a1*b1 + a2*b2).
__device__ __forceinline__ float dot3(V3 a, V3 b) {
  return __builtin_fmaf(a.x, b.x, __builtin_fmaf(a.y, b.y, a.z * b.z));
}

// Ray-cast constants of a triangle (A, B, C) in camera space for the pixel
// ray r = (rx, ry, 1): hit = A + u (C - A) + v (B - A) at depth z with
// N = (C-A) x (B-A), Nu = (B-A) x A, Nv = A x (C-A), D = A . N,
// den = r.N, u = r.Nu / den, v = r.Nv / den, z = D / den.
struct RayK {
  V3 n, nu, nv;
  float d;
};

__device__ __forceinline__ RayK ray_consts(V3 A, V3 B, V3 C) {
  V3 e1 = sub3(C, A), e2 = sub3(B, A);
  RayK k;
  k.n = cross3(e1, e2);
  k.nu = cross3(e2, A);
  k.nv = cross3(A, e1);
  k.d = dot3(A, k.n);
  return k;
}

// r . n with r = (rx, ry, 1): rx*nx + (ry*ny + nz).
__device__ __forceinline__ float rdot(float rx, float ry, V3 n) {
  return __builtin_fmaf(rx, n.x, __builtin_fmaf(ry, n.y, n.z));
}

__device__ __forceinline__ float ray_x(const Cam& c, int x) { return (((float)x + 0.5f) - c.cx) / c.fx; }
__device__ __forceinline__ float ray_y(const Cam& c, int y) { return (((float)y + 0.5f) - c.cy) / c.fy; }

// Depth of a fragment; returns false when it is not in front of the camera
// (z <= 0, NaN) or not finite.
__device__ __forceinline__ bool frag_depth(const RayK& k, float rx, float ry, float* z) {
  float den = rdot(rx, ry, k.n);
  float zz = k.d / den;
  *z = zz;
  return zz > 0.0f && zz <= 3.402823466e38f;
}

constexpr float kGuard = 1048576.0f;  // clipped polygons stay within |px|, |py| <= 2^20

// Signed distance to clip plane p (inside when >= 0):
// 0: z - z_near; 1: (G-cx) z - fx x; 2: (G+cx) z + fx x; 3: (G-cy) z - fy y; 4: (G+cy) z + fy y.
__device__ __forceinline__ float clip_dist(int p, V3 v, const Cam& c, float z_near) {
  switch (p) {
    case 0: return v.z - z_near;
    case 1: return __builtin_fmaf(kGuard - c.cx, v.z, -(c.fx * v.x));
    case 2: return __builtin_fmaf(kGuard + c.cx, v.z, c.fx * v.x);
    case 3: return __builtin_fmaf(kGuard - c.cy, v.z, -(c.fy * v.y));
    default: return __builtin_fmaf(kGuard + c.cy, v.z, c.fy * v.y);
  }
}

__device__ __forceinline__ bool inside_all(V3 v, const Cam& c, float z_near) {
  bool in = true;
#pragma unroll
  for (int p = 0; p < 5; ++p) in = in && (clip_dist(p, v, c, z_near) >= 0.0f);
  return in;
}

// Sutherland-Hodgman over the five planes in order.  An edge crossing a plane
// contributes the point I + a (O - I), a = dI / (dI - dO), computed from its
// inside end I towards its outside end O, so both triangles that share the
// edge produce identical bits.  Vertex i is kept before the crossing on edge
// (i, i+1).  Returns the polygon size (0..8).
__device__ __forceinline__ int clip_poly(V3 (&P)[8], int n, const Cam& c, float z_near) {
  for (int p = 0; p < 5; ++p) {
    if (n == 0) break;
    V3 Q[8];
    float d[8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (i < n) d[i] = clip_dist(p, P[i], c, z_near);
    int m = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (i < n) {
        int j = (i + 1 == n) ? 0 : i + 1;
        bool ii = d[i] >= 0.0f;
        bool ij = d[j] >= 0.0f;
        if (ii) Q[m++] = P[i];
        if (ii != ij) {
          V3 I = ii ? P[i] : P[j];
          V3 O = ii ? P[j] : P[i];
          float dI = ii ? d[i] : d[j];
          float dO = ii ? d[j] : d[i];
          float a = dI / (dI - dO);
          Q[m++] = V3{__builtin_fmaf(a, O.x - I.x, I.x), __builtin_fmaf(a, O.y - I.y, I.y),
                      __builtin_fmaf(a, O.z - I.z, I.z)};
        }
      }
    }
    n = m;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (i < n) P[i] = Q[i];
  }
  return n;
}

// Projection and snap to 8 sub-pixel bits (round half to even).
__device__ __forceinline__ void snap(const Cam& c, V3 v, int* X, int* Y) {
  float xn = v.x / v.z;
  float yn = v.y / v.z;
  float px = __builtin_fmaf(c.fx, xn, c.cx);
  float py = __builtin_fmaf(c.fy, yn, c.cy);
  *X = (int)__builtin_rintf(px * 256.0f);
  *Y = (int)__builtin_rintf(py * 256.0f);
}

// Texel of (u, v) on a triangle with s steps (Section 3.1, eq. idtexel read as
// a bijection): cell (a, b) = (floor(s u), floor(s v)) clamped into the
// triangle a + b <= s - 1 (NaN -> 0); row r = s - 1 - a holds b = 0..r at
// r (r + 1) / 2 + b.  SPLIT: the upper-right half of a full cell (fractional
// parts summing to >= 1) is numbered after all s (s + 1) / 2 lower cells.
__device__ __forceinline__ int texel_id(int s, int split, float u, float v) {
  const float fs = (float)s;
  const float su = fs * u;
  const float sv = fs * v;
  int a = 0;
  if (su > 0.0f) a = (su >= fs) ? s - 1 : (int)__builtin_floorf(su);
  const int r = s - 1 - a;
  int b = 0;
  if (sv > 0.0f) b = (sv >= (float)(r + 1)) ? r : (int)__builtin_floorf(sv);
  int id = ((r * (r + 1)) >> 1) + b;
  if (split && b < r) {  // a + b <= s - 2: a full square cell
    const float fu = su - (float)a;
    const float fv = sv - (float)b;
    if (fu + fv >= 1.0f) {
      const int r2 = r - 1;
      id = ((s * (s + 1)) >> 1) + ((r2 * (r2 + 1)) >> 1) + b;
    }
  }
  return id;
}

__device__ __forceinline__ int texel_count(int s, int split) { return split ? s * s : (s * (s + 1)) >> 1; }

// Top/left ownership of a pixel centre lying exactly on an edge i->j of a
// positively oriented triangle: left edges (dy < 0) and top edges
// (dy == 0, dx > 0) own it.
__device__ __forceinline__ bool top_left(int dx, int dy) { return dy < 0 || (dy == 0 && dx > 0); }

}  // namespace lf
