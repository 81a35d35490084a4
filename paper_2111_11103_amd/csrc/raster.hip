// Renderer (Section 3.3.1): z-buffered projection of the mesh into per-pixel
// (depth, triangle) keys, then resolution of every pixel's texel row
// l = id_t + id_x (Section 3.3.2, eq. texel-in-array; eq. idtexel).
//
// k_raster: one thread per (frame, triangle); a wave of 64 consecutive
// triangles first tests its cluster box against the view frustum and leaves
// if the whole cluster is outside.  Unclipped triangles are snapped to 8
// sub-pixel bits; a triangle whose pixel-centre bounding box is small is
// rasterized by its own thread with incremental int64 edge functions; larger
// ones (and clipped polygons) are rasterized by the whole wave together, 8x8
// pixel blocks at a time.  Every covered pixel's key (bits(z) << 32 | t) goes
// through a 64-bit atomic minimum, so the result does not depend on the
// order in which fragments arrive.
#include "internal.h"
#include "spec.h"

namespace lf {

__global__ __launch_bounds__(256) void k_raytab(const float* __restrict__ cams, int nf, int H, int W,
                                                float* __restrict__ rx, float* __restrict__ ry) {
  const int f = blockIdx.y;
  const Cam c = load_cam(cams + 16 * (int64_t)f);
  for (int i = blockIdx.x * 256 + threadIdx.x; i < W + H; i += gridDim.x * 256) {
    if (i < W) rx[(int64_t)f * W + i] = ray_x(c, i);
    else ry[(int64_t)f * H + (i - W)] = ray_y(c, i - W);
  }
}

hipError_t launch_raytab(const float* cams, int nf, int H, int W, float* rx, float* ry, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  k_raytab<<<dim3((unsigned)((W + H + 255) / 256), (unsigned)nf), 256, 0, s>>>(cams, nf, H, W, rx, ry);
  return hipGetLastError();
}

namespace {

constexpr int kSmallPx = 48;   // bbox pixel count handled by a single thread

struct Frag {
  unsigned long long* keys;    // this frame's key plane
  const float* rx;
  const float* ry;
  int W;
};

__device__ __forceinline__ void emit(const Frag& fr, const RayK& rk, int x, int y, uint32_t tri) {
  float z;
  if (!frag_depth(rk, fr.rx[x], fr.ry[y], &z)) return;
  const unsigned long long key = ((unsigned long long)__float_as_uint(z) << 32) | tri;
  unsigned long long* slot = fr.keys + (int64_t)y * fr.W + x;
  // keys only decrease within a batch: a stale value that is already smaller
  // proves this fragment loses, so the atomic can be skipped
  if (__builtin_nontemporal_load(slot) <= key) return;
  atomicMin(slot, key);
}

// Oriented sub-triangle with edge data for coverage tests.
struct Edge3 {
  int x0, y0, x1, y1, x2, y2;  // positively oriented vertices
  int b01, b12, b20;           // 1 if the edge does not own on-edge centres
  bool ok;
};

__device__ __forceinline__ Edge3 setup_tri(int ax, int ay, int bx, int by, int cx, int cy) {
  Edge3 e;
  const long long area = (long long)(bx - ax) * (cy - ay) - (long long)(by - ay) * (cx - ax);
  e.ok = area != 0;
  if (area < 0) { int tx = bx, ty = by; bx = cx; by = cy; cx = tx; cy = ty; }
  e.x0 = ax; e.y0 = ay; e.x1 = bx; e.y1 = by; e.x2 = cx; e.y2 = cy;
  e.b01 = top_left(bx - ax, by - ay) ? 0 : 1;
  e.b12 = top_left(cx - bx, cy - by) ? 0 : 1;
  e.b20 = top_left(ax - cx, ay - cy) ? 0 : 1;
  return e;
}

__device__ __forceinline__ long long efn(int xi, int yi, int xj, int yj, int px, int py) {
  return (long long)(xj - xi) * (py - yi) - (long long)(yj - yi) * (px - xi);
}

__device__ __forceinline__ bool covers(const Edge3& e, int px, int py) {
  return efn(e.x0, e.y0, e.x1, e.y1, px, py) >= e.b01 && efn(e.x1, e.y1, e.x2, e.y2, px, py) >= e.b12 &&
         efn(e.x2, e.y2, e.x0, e.y0, px, py) >= e.b20;
}

// Single-thread raster of one positively oriented sub-triangle over a pixel
// box, stepping the three edge functions incrementally.
__device__ __forceinline__ void raster_tri_thread(const Frag& fr, const RayK& rk, uint32_t tri, const Edge3& e, int x0, int x1,
                                  int y0, int y1) {
  const int px0 = 256 * x0 + 128, py0 = 256 * y0 + 128;
  long long r01 = efn(e.x0, e.y0, e.x1, e.y1, px0, py0) - e.b01;
  long long r12 = efn(e.x1, e.y1, e.x2, e.y2, px0, py0) - e.b12;
  long long r20 = efn(e.x2, e.y2, e.x0, e.y0, px0, py0) - e.b20;
  // d/dx of efn(i->j) = -(yj - yi), d/dy = (xj - xi); one pixel = 256 units
  const long long sx01 = -256ll * (e.y1 - e.y0), sy01 = 256ll * (e.x1 - e.x0);
  const long long sx12 = -256ll * (e.y2 - e.y1), sy12 = 256ll * (e.x2 - e.x1);
  const long long sx20 = -256ll * (e.y0 - e.y2), sy20 = 256ll * (e.x0 - e.x2);
  for (int y = y0; y <= y1; ++y) {
    long long a = r01, b = r12, c = r20;
    for (int x = x0; x <= x1; ++x) {
      if ((a | b | c) >= 0) emit(fr, rk, x, y, tri);
      a += sx01; b += sx12; c += sx20;
    }
    r01 += sy01; r12 += sy12; r20 += sy20;
  }
}

// v[i] for a runtime i without dynamic register indexing (keeps the array in VGPRs).
__device__ __forceinline__ int pick8(const int (&v)[8], int i) {
  int r = v[0];
#pragma unroll
  for (int k = 1; k < 8; ++k) r = (i == k) ? v[k] : r;
  return r;
}

}  // namespace

__global__ __launch_bounds__(256) void k_raster(MeshDev m, const float* __restrict__ cams, int H, int W,
                                                unsigned long long* __restrict__ keys,
                                                const float* __restrict__ rxt, const float* __restrict__ ryt) {
  const int fb = blockIdx.y;
  const Cam cam = load_cam(cams + 16 * (int64_t)fb);
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;

  // ---- cluster cull (uniform per wave) ----
  {
    const int64_t cl = t >> 6;
    if (cl >= m.n_clusters) return;
    const float* b = m.cl_box + 8 * cl;
    const float lo[3] = {b[0], b[1], b[2]}, hi[3] = {b[3], b[4], b[5]};
    // bound on |coordinate| magnitudes for a rounding margin
    float mag = fabsf(cam.t[0]) + fabsf(cam.t[1]) + fabsf(cam.t[2]);
    for (int d = 0; d < 3; ++d) mag += 3.0f * fmaxf(fabsf(lo[d]), fabsf(hi[d]));
    const float eps = 1e-5f * mag;
    // planes in camera space (inside >= 0): near, and the image borders
    // widened by 2 px: x: fx*x + (cx + 2) z >= 0, (W + 2 - cx) z - fx*x >= 0 ...
    bool out[5] = {true, true, true, true, true};
    for (int k = 0; k < 8; ++k) {
      V3 p = to_cam(cam, (k & 1) ? hi[0] : lo[0], (k & 2) ? hi[1] : lo[1], (k & 4) ? hi[2] : lo[2]);
      const float magp = eps * (1.0f + fabsf(cam.fx) + fabsf(cam.fy) + fabsf(cam.cx) + fabsf(cam.cy) + W + H);
      out[0] = out[0] && (p.z - m.z_near < -eps);
      out[1] = out[1] && (cam.fx * p.x + (cam.cx + 2.0f) * p.z < -magp);
      out[2] = out[2] && (((float)W + 2.0f - cam.cx) * p.z - cam.fx * p.x < -magp);
      out[3] = out[3] && (cam.fy * p.y + (cam.cy + 2.0f) * p.z < -magp);
      out[4] = out[4] && (((float)H + 2.0f - cam.cy) * p.z - cam.fy * p.y < -magp);
    }
    if (out[0] || out[1] || out[2] || out[3] || out[4]) return;
  }

  Frag fr{keys + (int64_t)fb * H * W, rxt + (int64_t)fb * W, ryt + (int64_t)fb * H, W};
  const bool live = t < m.T;
  int n = 0;
  int PX[8] = {0, 0, 0, 0, 0, 0, 0, 0}, PY[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  RayK rk{};
  if (live) {
    const int i0 = m.faces_uv[3 * t], i1 = m.faces_uv[3 * t + 1], i2 = m.faces_uv[3 * t + 2];
    const float* q0 = m.verts + 3 * (int64_t)i0;
    const float* q1 = m.verts + 3 * (int64_t)i1;
    const float* q2 = m.verts + 3 * (int64_t)i2;
    const V3 A = to_cam(cam, q0[0], q0[1], q0[2]);
    const V3 B = to_cam(cam, q1[0], q1[1], q1[2]);
    const V3 C = to_cam(cam, q2[0], q2[1], q2[2]);
    // trivially outside one plane: nothing survives clipping
    bool gone = false;
#pragma unroll
    for (int p = 0; p < 5; ++p)
      gone = gone || (clip_dist(p, A, cam, m.z_near) < 0.0f && clip_dist(p, B, cam, m.z_near) < 0.0f &&
                      clip_dist(p, C, cam, m.z_near) < 0.0f);
    if (!gone) {
      rk = ray_consts(A, B, C);
      if (inside_all(A, cam, m.z_near) && inside_all(B, cam, m.z_near) && inside_all(C, cam, m.z_near)) {
        snap(cam, A, &PX[0], &PY[0]);
        snap(cam, B, &PX[1], &PY[1]);
        snap(cam, C, &PX[2], &PY[2]);
        n = 3;
      } else {
        V3 P[8];
        P[0] = A; P[1] = B; P[2] = C;
        n = clip_poly(P, 3, cam, m.z_near);
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (i < n) snap(cam, P[i], &PX[i], &PY[i]);
      }
    }
  }
  // pixel-centre bounding box: centre (256x+128) in [min, max]
  int x0 = 0, x1 = -1, y0 = 0, y1 = -1;
  if (n >= 3) {
    int xmin = PX[0], xmax = PX[0], ymin = PY[0], ymax = PY[0];
#pragma unroll
    for (int i = 1; i < 8; ++i)
      if (i < n) {
        xmin = min(xmin, PX[i]); xmax = max(xmax, PX[i]);
        ymin = min(ymin, PY[i]); ymax = max(ymax, PY[i]);
      }
    x0 = max((xmin + 127) >> 8, 0);
    x1 = min((xmax - 128) >> 8, W - 1);
    y0 = max((ymin + 127) >> 8, 0);
    y1 = min((ymax - 128) >> 8, H - 1);
  }
  const bool any = n >= 3 && x0 <= x1 && y0 <= y1;
  const int npx = any ? (x1 - x0 + 1) * (y1 - y0 + 1) : 0;
  const bool small = any && npx <= kSmallPx;
  if (small) {
    for (int i = 1; i + 1 < n; ++i) {
      const Edge3 e = setup_tri(PX[0], PY[0], pick8(PX, i), pick8(PY, i), pick8(PX, i + 1), pick8(PY, i + 1));
      if (e.ok) raster_tri_thread(fr, rk, (uint32_t)t, e, x0, x1, y0, y1);
    }
  }
  // ---- large triangles: the whole wave, one triangle at a time ----
  unsigned long long big = __ballot(any && !small);
  while (big) {
    const int src = __ffsll(big) - 1;
    big &= big - 1;
    const int bn = __shfl(n, src);
    int bx[8], by[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      bx[i] = __shfl(PX[i], src);
      by[i] = __shfl(PY[i], src);
    }
    RayK bk;
    bk.n = V3{__shfl(rk.n.x, src), __shfl(rk.n.y, src), __shfl(rk.n.z, src)};
    bk.d = __shfl(rk.d, src);
    const int bx0 = __shfl(x0, src), bx1 = __shfl(x1, src), by0 = __shfl(y0, src), by1 = __shfl(y1, src);
    const uint32_t btri = (uint32_t)(t - lane + src);
    const int ox = lane & 7, oy = lane >> 3;
    for (int yb = by0; yb <= by1; yb += 8) {
      for (int xb = bx0; xb <= bx1; xb += 8) {
        const int x = xb + ox, y = yb + oy;
        if (x > bx1 || y > by1) continue;
        const int pcx = 256 * x + 128, pcy = 256 * y + 128;
        bool cov = false;
        for (int i = 1; i + 1 < bn; ++i) {
          const Edge3 e = setup_tri(bx[0], by[0], pick8(bx, i), pick8(by, i), pick8(bx, i + 1), pick8(by, i + 1));
          cov = cov || (e.ok && covers(e, pcx, pcy));
        }
        if (cov) emit(fr, bk, x, y, btri);
      }
    }
  }
}

hipError_t launch_raster(const MeshDev& m, const float* cams, int nf, int H, int W, unsigned long long* keys,
                         const float* rx, const float* ry, hipStream_t s) {
  if (nf <= 0 || m.T == 0) return hipSuccess;
  k_raster<<<dim3((unsigned)((m.T + 255) / 256), (unsigned)nf), 256, 0, s>>>(m, cams, H, W, keys, rx, ry);
  return hipGetLastError();
}

// ---- resolve: key -> (triangle, texel row, depth); resets the key --------------
__global__ __launch_bounds__(256) void k_resolve(MeshDev m, const float* __restrict__ cams, int H, int W,
                                                 unsigned long long* __restrict__ keys,
                                                 const float* __restrict__ rxt, const float* __restrict__ ryt,
                                                 int32_t* __restrict__ l_out, int32_t* __restrict__ tri_out,
                                                 float* __restrict__ z_out, const uint8_t* __restrict__ valid,
                                                 int32_t* __restrict__ cnt, int64_t cnt_stride) {
  const int fb = blockIdx.y;
  const int64_t HW = (int64_t)H * W;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= HW) return;
  const int64_t i = (int64_t)fb * HW + p;
  const unsigned long long key = keys[i];
  keys[i] = ~0ull;
  int32_t l = -1, tri = -1;
  float z = __builtin_nanf("");
  if (key != ~0ull) {
    tri = (int32_t)(uint32_t)(key & 0xffffffffull);
    const Cam cam = load_cam(cams + 16 * (int64_t)fb);
    const int x = (int)(p % W), y = (int)(p / W);
    const int i0 = m.faces_uv[3 * (int64_t)tri], i1 = m.faces_uv[3 * (int64_t)tri + 1],
              i2 = m.faces_uv[3 * (int64_t)tri + 2];
    const float* q0 = m.verts + 3 * (int64_t)i0;
    const float* q1 = m.verts + 3 * (int64_t)i1;
    const float* q2 = m.verts + 3 * (int64_t)i2;
    const RayK rk = ray_consts(to_cam(cam, q0[0], q0[1], q0[2]), to_cam(cam, q1[0], q1[1], q1[2]),
                               to_cam(cam, q2[0], q2[1], q2[2]));
    const float rx = rxt[(int64_t)fb * W + x], ry = ryt[(int64_t)fb * H + y];
    const float den = rdot(rx, ry, rk.n);
    z = rk.d / den;
    const float u = rdot(rx, ry, rk.nu) / den;
    const float v = rdot(rx, ry, rk.nv) / den;
    l = (int32_t)(row_offset(m, tri) + texel_id(tri_s(m, tri), m.split, u, v));
    if (cnt && (!valid || valid[i])) atomicAdd(cnt + (int64_t)fb * cnt_stride + l, 1);
  }
  if (l_out) l_out[i] = l;
  if (tri_out) tri_out[i] = tri;
  if (z_out) z_out[i] = z;
}

hipError_t launch_resolve(const MeshDev& m, const float* cams, int nf, int H, int W, unsigned long long* keys,
                          const float* rx, const float* ry, int32_t* l_out, int32_t* tri_out, float* z_out,
                          const uint8_t* valid, int32_t* cnt, int64_t cnt_stride, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  const int64_t HW = (int64_t)H * W;
  k_resolve<<<dim3((unsigned)((HW + 255) / 256), (unsigned)nf), 256, 0, s>>>(m, cams, H, W, keys, rx, ry, l_out,
                                                                             tri_out, z_out, valid, cnt, cnt_stride);
  return hipGetLastError();
}

}  // namespace lf
