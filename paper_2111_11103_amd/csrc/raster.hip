// Renderer (Section 3.3.1): z-buffered projection of the mesh into per-pixel
// triangle ids, then every pixel's texel row l = id_t + id_x (Section 3.3.2,
// eq. texel-in-array; eq. idtexel).
//
// Sort-middle tiled rasterizer, all frames of a batch at once:
//   k_cull_clusters  frame x cluster (64 consecutive triangles): conservative
//                    frustum test of the cluster box, compact list of the
//                    clusters that may be visible;
//   k_bin            one wave per visible cluster: set up every triangle
//                    (transform, clip, 8-bit sub-pixel snap) and append it
//                    to the fixed-capacity list of every tile (16x16 or
//                    32x32 pixels, a tuning knob) its pixel-centre box
//                    overlaps (slots reserved per block through LDS tile
//                    counters);
//   k_tile_raster    one workgroup per (frame, tile): a 64-bit depth|id key
//                    per pixel in LDS, every listed triangle rasterized with
//                    exact integer edge functions and the top-left rule (small
//                    ones by one thread, large ones by the whole wave),
//                    ds_min_u64 on the key; then every pixel resolves its
//                    winner into (triangle, texel row, depth) and writes them
//                    out, with one texel-row count atomic per run of
//                    same-row pixels.
// Triangles are read from a triangle-major copy of their positions built at
// load (one dependent read per triangle).
// The key order (depth bits, then triangle id) makes the result independent
// of the order fragments arrive in.
#include <algorithm>

#include "internal.h"
#include "spec.h"

namespace lf {

namespace {


// Snapped screen triangle of one triangle in one frame.  Only scalars, so
// that it lives in registers: a triangle that crosses a clip plane and
// becomes a polygon of more than three vertices is marked by n and its
// polygon recomputed (same arithmetic, same bits) where it is drawn.
struct Setup {
  int n;                       // 0 = nothing to draw, 3 = triangle, 4..8 = clipped polygon
  int ax, ay, bx, by, cx, cy;  // the triangle (n == 3), 1/256 px
  RayK rk;                     // ray-cast constants of the original triangle
  int x0, x1, y0, y1;          // pixel-centre box, clamped to the image
};

// Camera-space corners of triangle t (uv order) from the triangle-major copy
// of the positions: one dependent read instead of indices, then vertices.
__device__ __forceinline__ void load_tri(const MeshDev& m, const Cam& cam, int64_t t, V3& A, V3& B, V3& C) {
  const float4 p = m.tri_v[3 * t], q = m.tri_v[3 * t + 1], r = m.tri_v[3 * t + 2];
  A = to_cam(cam, p.x, p.y, p.z);
  B = to_cam(cam, p.w, q.x, q.y);
  C = to_cam(cam, q.z, q.w, r.x);
}

// Snapped polygon of the camera-space triangle (A, B, C) clipped by the five
// planes, written to px, py (0..8 vertices; the count is returned).  Out of
// line, with its polygon arrays in per-lane memory: only triangles that
// cross a plane take this path.  It reads the camera record itself, so that
// callers need not keep their copy in memory.
__device__ __noinline__ int clipped_polygon(const float* __restrict__ cam_rec, float z_near, V3 A, V3 B, V3 C,
                                            int* px, int* py) {
  const Cam cam = load_cam(cam_rec);
  V3 P[8];
  P[0] = A; P[1] = B; P[2] = C;
  const int n = clip_poly(P, 3, cam, z_near);
  for (int i = 0; i < n; ++i) snap(cam, P[i], &px[i], &py[i]);
  return n;
}

// Vertex count and pixel-unit bounds of the clipped, snapped polygon, and its
// vertices when it is a triangle (returned in registers).
struct ClipBox {
  int n, xmin, xmax, ymin, ymax;
  int ax, ay, bx, by, cx, cy;
};

__device__ __noinline__ ClipBox clipped_box(const float* __restrict__ cam_rec, float z_near, V3 A, V3 B, V3 C) {
  int PX[8], PY[8];
  ClipBox r{};
  r.n = clipped_polygon(cam_rec, z_near, A, B, C, PX, PY);
  if (r.n < 3) return r;
  r.xmin = r.xmax = PX[0];
  r.ymin = r.ymax = PY[0];
  for (int i = 1; i < r.n; ++i) {
    r.xmin = min(r.xmin, PX[i]); r.xmax = max(r.xmax, PX[i]);
    r.ymin = min(r.ymin, PY[i]); r.ymax = max(r.ymax, PY[i]);
  }
  r.ax = PX[0]; r.ay = PY[0]; r.bx = PX[1]; r.by = PY[1]; r.cx = PX[2]; r.cy = PY[2];
  return r;
}

__device__ __forceinline__ void setup_triangle(const MeshDev& m, const Cam& cam, const float* cam_rec, int64_t t, int H,
                                               int W, Setup& s) {
  s.n = 0;
  s.ax = s.ay = s.bx = s.by = s.cx = s.cy = 0;
  s.x0 = 0; s.x1 = -1; s.y0 = 0; s.y1 = -1;
  V3 A, B, C;
  load_tri(m, cam, t, A, B, C);
  bool gone = false;
#pragma unroll
  for (int p = 0; p < 5; ++p)
    gone = gone || (clip_dist(p, A, cam, m.z_near) < 0.0f && clip_dist(p, B, cam, m.z_near) < 0.0f &&
                    clip_dist(p, C, cam, m.z_near) < 0.0f);
  if (gone) return;
  s.rk = ray_consts(A, B, C);
  int xmin, xmax, ymin, ymax;
  if (inside_all(A, cam, m.z_near) && inside_all(B, cam, m.z_near) && inside_all(C, cam, m.z_near)) {
    snap(cam, A, &s.ax, &s.ay);
    snap(cam, B, &s.bx, &s.by);
    snap(cam, C, &s.cx, &s.cy);
    s.n = 3;
    xmin = min(min(s.ax, s.bx), s.cx); xmax = max(max(s.ax, s.bx), s.cx);
    ymin = min(min(s.ay, s.by), s.cy); ymax = max(max(s.ay, s.by), s.cy);
  } else {
    const ClipBox cb = clipped_box(cam_rec, m.z_near, A, B, C);
    if (cb.n < 3) return;
    s.n = cb.n;
    if (cb.n == 3) {
      s.ax = cb.ax; s.ay = cb.ay; s.bx = cb.bx; s.by = cb.by; s.cx = cb.cx; s.cy = cb.cy;
    }
    xmin = cb.xmin; xmax = cb.xmax; ymin = cb.ymin; ymax = cb.ymax;
  }
  // pixel x is a candidate iff its centre 256x + 128 lies in [xmin, xmax]
  s.x0 = max((xmin + 127) >> 8, 0);
  s.x1 = min((xmax - 128) >> 8, W - 1);
  s.y0 = max((ymin + 127) >> 8, 0);
  s.y1 = min((ymax - 128) >> 8, H - 1);
  if (s.x0 > s.x1 || s.y0 > s.y1) s.n = 0;
}

// Oriented sub-triangle with its top-left biases.
struct Edge3 {
  int x0, y0, x1, y1, x2, y2;
  int b01, b12, b20;          // 1 when the edge does not own centres lying on it
  bool ok;
};

__device__ __forceinline__ Edge3 orient(int ax, int ay, int bx, int by, int cx, int cy) {
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

// Conservative cluster-vs-frustum test: outside if all 8 box corners lie
// beyond one plane (near, or an image border widened by 2 px) by a margin far
// larger than the rounding of the per-vertex arithmetic, so no triangle of a
// culled cluster could have covered a pixel centre.
__device__ bool cluster_outside(const MeshDev& m, const Cam& cam, int64_t cl, int H, int W) {
  const float* b = m.cl_box + 8 * cl;
  const float lo[3] = {b[0], b[1], b[2]}, hi[3] = {b[3], b[4], b[5]};
  float mag = fabsf(cam.t[0]) + fabsf(cam.t[1]) + fabsf(cam.t[2]);
  for (int d = 0; d < 3; ++d) mag += 3.0f * fmaxf(fabsf(lo[d]), fabsf(hi[d]));
  const float eps = 1e-5f * mag;
  const float magp = eps * (1.0f + fabsf(cam.fx) + fabsf(cam.fy) + fabsf(cam.cx) + fabsf(cam.cy) + W + H);
  bool out0 = true, out1 = true, out2 = true, out3 = true, out4 = true;
  for (int k = 0; k < 8; ++k) {
    const V3 p = to_cam(cam, (k & 1) ? hi[0] : lo[0], (k & 2) ? hi[1] : lo[1], (k & 4) ? hi[2] : lo[2]);
    out0 = out0 && (p.z - m.z_near < -eps);
    out1 = out1 && (cam.fx * p.x + (cam.cx + 2.0f) * p.z < -magp);
    out2 = out2 && (((float)W + 2.0f - cam.cx) * p.z - cam.fx * p.x < -magp);
    out3 = out3 && (cam.fy * p.y + (cam.cy + 2.0f) * p.z < -magp);
    out4 = out4 && (((float)H + 2.0f - cam.cy) * p.z - cam.fy * p.y < -magp);
  }
  return out0 || out1 || out2 || out3 || out4;
}

// Wave-aggregated append: this lane's slot where `want`.
__device__ __forceinline__ int wave_append(int32_t* counter, bool want) {
  const unsigned long long mask = __ballot(want);
  if (mask == 0) return -1;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll(mask) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, __popcll(mask));
  base = __shfl(base, leader);
  return base + __popcll(mask & ((1ull << lane) - 1ull));
}

}  // namespace

// ---- 1. visible clusters ------------------------------------------------------
__global__ __launch_bounds__(256) void k_cull_clusters(MeshDev m, const float* __restrict__ cams, int H, int W,
                                                       int32_t* __restrict__ vis, int32_t* __restrict__ vis_n) {
  const int fb = blockIdx.y;
  const Cam cam = load_cam(cams + 16 * (int64_t)fb);
  const int64_t cl = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool keep = cl < m.n_clusters && !cluster_outside(m, cam, cl, H, W);
  const int slot = wave_append(vis_n + fb, keep);
  if (keep) vis[(int64_t)fb * m.n_clusters + slot] = (int32_t)cl;
}

// ---- 2. binning into tiles (one pass into fixed-capacity tile lists) -----------------
// Every tile of a frame owns `cap` list slots.  A triangle takes a slot in
// every tile its pixel-centre box overlaps; the tile's counter keeps counting
// past `cap`, which tells the raster to fall back to walking the frame's
// visible clusters for that tile.
//
// With the frame's tile counts fitting in LDS (dynamic LDS of 2 * ntiles
// ints), a block bins its four clusters together: it counts its triangles
// per tile with LDS atomics, reserves each touched tile's slots with one
// global atomic (all issued at once, none waited for inside a loop), then
// places every triangle at the tile's base plus an LDS rank.  Otherwise the
// lanes of a wave that are on the same tile share one global atomic.
constexpr int kBinLdsTiles = 4096;

template <int TS>
__global__ __launch_bounds__(256) void k_bin(MeshDev m, const float* __restrict__ cams, int H, int W,
                                             const int32_t* __restrict__ vis, const int32_t* __restrict__ vis_n,
                                             int32_t* __restrict__ tcnt, int32_t* __restrict__ tlist, int64_t list_cap,
                                             int cap) {
  extern __shared__ int tile_lds[];       // [ntiles] counts, then bases; [ntiles] ranks
  const int fb = blockIdx.y;
  const Cam cam = load_cam(cams + 16 * (int64_t)fb);
  const int ntx = (W + TS - 1) / TS, nty = (H + TS - 1) / TS;
  const int ntiles = ntx * nty;
  const int lane = threadIdx.x & 63;
  const int nvis = vis_n[fb];
  int32_t* cnt = tcnt + (int64_t)fb * ntiles;
  int32_t* lst = tlist + (int64_t)fb * list_cap;
  if (ntiles <= kBinLdsTiles) {
    int* tb = tile_lds;
    int* tr = tile_lds + ntiles;
    for (int w0 = blockIdx.x * 4; w0 < nvis; w0 += gridDim.x * 4) {   // same trip count for the whole block
      const int w = w0 + (threadIdx.x >> 6);
      int64_t t = m.T;
      Setup s;
      s.n = 0;
      s.x0 = 0; s.x1 = -1; s.y0 = 0; s.y1 = -1;
      if (w < nvis) {
        t = vis[(int64_t)fb * m.n_clusters + w] * (int64_t)kClusterTris + lane;
        if (t < m.T) setup_triangle(m, cam, cams + 16 * (int64_t)fb, t, H, W, s);
      }
      const bool draw = t < m.T && s.n != 0;
      const int tx0 = s.x0 / TS, tx1 = s.x1 / TS, ty0 = s.y0 / TS, ty1 = s.y1 / TS;
      for (int i = threadIdx.x; i < ntiles; i += 256) {
        tb[i] = 0;
        tr[i] = 0;
      }
      __syncthreads();
      if (draw)
        for (int ty = ty0; ty <= ty1; ++ty)
          for (int tx = tx0; tx <= tx1; ++tx) atomicAdd(&tb[ty * ntx + tx], 1);
      __syncthreads();
      for (int i = threadIdx.x; i < ntiles; i += 256) {
        const int n = tb[i];
        if (n) tb[i] = atomicAdd(cnt + i, n);
      }
      __syncthreads();
      if (draw)
        for (int ty = ty0; ty <= ty1; ++ty)
          for (int tx = tx0; tx <= tx1; ++tx) {
            const int tile = ty * ntx + tx;
            const int pos = tb[tile] + atomicAdd(&tr[tile], 1);
            if (pos < cap) lst[(int64_t)tile * cap + pos] = (int32_t)t;
          }
      __syncthreads();                    // the next round clears the arrays
    }
    return;
  }
  for (int w = blockIdx.x * 4 + (threadIdx.x >> 6); w < nvis; w += gridDim.x * 4) {
    const int64_t cl = vis[(int64_t)fb * m.n_clusters + w];
    const int64_t t = cl * kClusterTris + lane;
    Setup s;
    s.n = 0;
    s.x0 = 0; s.x1 = -1; s.y0 = 0; s.y1 = -1;
    if (t < m.T) setup_triangle(m, cam, cams + 16 * (int64_t)fb, t, H, W, s);
    // walk this lane's tile range; lanes currently on the same tile share one atomic
    const int tx0 = s.x0 / TS, tx1 = s.x1 / TS, ty0 = s.y0 / TS, ty1 = s.y1 / TS;
    int tx = tx0, ty = ty0;
    bool more = s.n != 0;
    while (true) {
      const int tile = more ? ty * ntx + tx : -1;
      const unsigned long long act = __ballot(more);
      if (act == 0) break;
      const int leader_tile = __shfl(tile, __ffsll(act) - 1);
      const bool mine = more && tile == leader_tile;
      const unsigned long long grp = __ballot(mine);
      const int leader = __ffsll(grp) - 1;
      const int rank = __popcll(grp & ((1ull << lane) - 1ull));
      int base = 0;
      if (lane == leader) base = atomicAdd(cnt + leader_tile, __popcll(grp));
      base = __shfl(base, leader);
      if (mine) {
        const int pos = base + rank;
        if (pos < cap) lst[(int64_t)leader_tile * cap + pos] = (int32_t)t;
        if (++tx > tx1) { tx = tx0; ++ty; }
        more = ty <= ty1;
      }
    }
  }
}

// ---- 5. tile raster + resolve --------------------------------------------------------
namespace {

struct TileCtx {
  unsigned long long* key;   // LDS [ts*ts]
  const float* rx;           // LDS [ts] ray x of the tile's columns
  const float* ry;           // LDS [ts]
  int tx0, ty0;              // tile origin (pixels)
  int ts;                    // tile edge
  int small_px;              // boxes up to this area: one lane per triangle
  const float* cam_rec;      // the frame's camera record (global memory)
  int* poly;                 // LDS [4 waves][16]: a clipped polygon's snapped x, then y
};

__device__ __forceinline__ void emit_lds(const TileCtx& c, const RayK& rk, int x, int y, uint32_t tri) {
  float z;
  if (!frag_depth(rk, c.rx[x - c.tx0], c.ry[y - c.ty0], &z)) return;
  const unsigned long long k = ((unsigned long long)__float_as_uint(z) << 32) | tri;
  atomicMin(c.key + (y - c.ty0) * c.ts + (x - c.tx0), k);
}

// One thread rasterizes one triangle over a small pixel box, stepping the
// three edge functions incrementally.  Only triangles whose coordinate
// differences are all below 2^14 (64 px) take this path: then every edge
// value fits in int32 exactly, so the narrow arithmetic gives the same
// decisions as the int64 edge functions.
__device__ __forceinline__ void raster_thread(const TileCtx& c, const RayK& rk, uint32_t tri, const Edge3& e, int x0,
                                              int x1, int y0, int y1) {
  const int px0 = 256 * x0 + 128, py0 = 256 * y0 + 128;
  int r01 = (e.x1 - e.x0) * (py0 - e.y0) - (e.y1 - e.y0) * (px0 - e.x0) - e.b01;
  int r12 = (e.x2 - e.x1) * (py0 - e.y1) - (e.y2 - e.y1) * (px0 - e.x1) - e.b12;
  int r20 = (e.x0 - e.x2) * (py0 - e.y2) - (e.y0 - e.y2) * (px0 - e.x2) - e.b20;
  const int sx01 = -256 * (e.y1 - e.y0), sy01 = 256 * (e.x1 - e.x0);
  const int sx12 = -256 * (e.y2 - e.y1), sy12 = 256 * (e.x2 - e.x1);
  const int sx20 = -256 * (e.y0 - e.y2), sy20 = 256 * (e.x0 - e.x2);
  for (int y = y0; y <= y1; ++y) {
    int a = r01, b = r12, d = r20;
    for (int x = x0; x <= x1; ++x) {
      if ((a | b | d) >= 0) emit_lds(c, rk, x, y, tri);
      a += sx01; b += sx12; d += sx20;
    }
    r01 += sy01; r12 += sy12; r20 += sy20;
  }
}

// Whether the triangle this lane holds (box restricted to the tile) is drawn
// by the lane itself; every other drawable triangle is queued for a wave.
__device__ __forceinline__ bool lane_draws(const Setup& s, int x0, int x1, int y0, int y1, int small_px) {
  const int ex = max(max(s.ax, s.bx), s.cx) - min(min(s.ax, s.bx), s.cx);
  const int ey = max(max(s.ay, s.by), s.cy) - min(min(s.ay, s.by), s.cy);
  return s.n == 3 && ex < 16384 && ey < 16384 && (x1 - x0 + 1) * (y1 - y0 + 1) <= small_px;
}

// Draw one (sub-)triangle with the whole wave over the pixel box x0..x1 x
// y0..y1, 8x8 pixels per step, with int64 edge functions.
__device__ __forceinline__ void wave_triangle(const TileCtx& c, const RayK& rk, uint32_t t, int ax, int ay, int bx,
                                              int by, int cx, int cy, int x0, int x1, int y0, int y1) {
  const Edge3 e = orient(ax, ay, bx, by, cx, cy);
  if (!e.ok) return;
  const int lane = threadIdx.x & 63;
  const int ox = lane & 7, oy = lane >> 3;
  for (int yb = y0; yb <= y1; yb += 8) {
    for (int xb = x0; xb <= x1; xb += 8) {
      const int x = xb + ox, y = yb + oy;
      if (x > x1 || y > y1) continue;
      if (covers(e, 256 * x + 128, 256 * y + 128)) emit_lds(c, rk, x, y, t);
    }
  }
}

// A clipped triangle (a polygon of more than three vertices) drawn by the
// whole wave as the fan (v0, vi, vi+1).  The polygon's vertices go to the
// wave's LDS slot (every lane writes the same values, then reads them back).
__device__ __forceinline__ void wave_polygon(const TileCtx& c, const MeshDev& m, const Cam& cam, const RayK& rk,
                                             uint32_t t, int x0, int x1, int y0, int y1) {
  int* PX = c.poly + 16 * (threadIdx.x >> 6);
  int* PY = PX + 8;
  V3 A, B, C;
  load_tri(m, cam, t, A, B, C);
  const int n = clipped_polygon(c.cam_rec, m.z_near, A, B, C, PX, PY);
  for (int i = 1; i + 1 < n; ++i)
    wave_triangle(c, rk, t, PX[0], PY[0], PX[i], PY[i], PX[i + 1], PY[i + 1], x0, x1, y0, y1);
}

// The whole wave draws triangle t (wave-uniform) over its box restricted to
// the tile.
__device__ __forceinline__ void raster_wave(const TileCtx& c, const MeshDev& m, const Cam& cam, uint32_t t, int H,
                                            int W, int tx1, int ty1) {
  Setup s;
  setup_triangle(m, cam, c.cam_rec, t, H, W, s);
  const int x0 = max(s.x0, c.tx0), x1 = min(s.x1, tx1), y0 = max(s.y0, c.ty0), y1 = min(s.y1, ty1);
  if (s.n < 3 || x0 > x1 || y0 > y1) return;
  if (s.n == 3) wave_triangle(c, s.rk, t, s.ax, s.ay, s.bx, s.by, s.cx, s.cy, x0, x1, y0, y1);
  else wave_polygon(c, m, cam, s.rk, t, x0, x1, y0, y1);
}

// One round of up to 256 triangles (one per thread, `have` = this thread
// holds triangle t): small ones are drawn by their lane, the rest queued in
// LDS and drawn by the block's four waves in turn.  Every thread of the
// block must call it.
__device__ __forceinline__ void raster_round(const TileCtx& c, const MeshDev& m, const Cam& cam, bool have,
                                             uint32_t t, int H, int W, int tx1, int ty1, uint32_t* queue,
                                             int* queue_n) {
  bool queued = false;
  if (have) {
    Setup s;
    setup_triangle(m, cam, c.cam_rec, t, H, W, s);
    const int x0 = max(s.x0, c.tx0), x1 = min(s.x1, tx1), y0 = max(s.y0, c.ty0), y1 = min(s.y1, ty1);
    if (s.n >= 3 && x0 <= x1 && y0 <= y1) {
      if (lane_draws(s, x0, x1, y0, y1, c.small_px)) {
        const Edge3 e = orient(s.ax, s.ay, s.bx, s.by, s.cx, s.cy);
        if (e.ok) raster_thread(c, s.rk, t, e, x0, x1, y0, y1);
      } else {
        queued = true;
      }
    }
  }
  if (queued) queue[atomicAdd(queue_n, 1)] = t;
  __syncthreads();
  const int nq = *queue_n;
  __syncthreads();
  if (threadIdx.x == 0) *queue_n = 0;
  for (int i = threadIdx.x >> 6; i < nq; i += 4)
    raster_wave(c, m, cam, (uint32_t)__builtin_amdgcn_readfirstlane((int)queue[i]), H, W, tx1, ty1);
  __syncthreads();
}

}  // namespace

template <int TS>
__global__ __launch_bounds__(256) void k_tile_raster(MeshDev m, const float* __restrict__ cams, int H, int W,
                                                     const int32_t* __restrict__ vis, const int32_t* __restrict__ vis_n,
                                                     int32_t* __restrict__ tcnt, const int32_t* __restrict__ tlist,
                                                     int64_t list_cap, int cap, RasterOut out) {
  __shared__ unsigned long long key[TS * TS];
  __shared__ float rxs[TS], rys[TS];
  __shared__ int hkey[kTileSlots], hcnt[kTileSlots], hbase[kTileSlots];   // the tile's bucket table
  __shared__ uint32_t queue[256];                                          // triangles a wave draws
  __shared__ int queue_n;
  __shared__ int poly[4 * 16];
  const int fb = blockIdx.y;
  const Cam cam = load_cam(cams + 16 * (int64_t)fb);
  const int ntx = (W + TS - 1) / TS, nty = (H + TS - 1) / TS;
  const int ntiles = ntx * nty;
  const int tile = blockIdx.x;
  const int tx0 = (tile % ntx) * TS, ty0 = (tile / ntx) * TS;
  const int tx1 = min(tx0 + TS, W) - 1, ty1 = min(ty0 + TS, H) - 1;
  // entries of this tile's list; the counter is left at zero for the next use
  int32_t* tc = tcnt + (int64_t)fb * ntiles + tile;
  const int n_ent = *tc;
  for (int i = threadIdx.x; i < TS * TS; i += 256) key[i] = ~0ull;
  if (threadIdx.x < TS) rxs[threadIdx.x] = ray_x(cam, tx0 + threadIdx.x);
  else if (threadIdx.x < 2 * TS) rys[threadIdx.x - TS] = ray_y(cam, ty0 + threadIdx.x - TS);
  if (threadIdx.x == 0) queue_n = 0;
  __syncthreads();
  if (threadIdx.x == 0) *tc = 0;
  const TileCtx c{key, rxs, rys, tx0, ty0, TS, m.small_px, cams + 16 * (int64_t)fb, poly};
  const int64_t HW = (int64_t)H * W;

  if (n_ent <= cap) {
    const int32_t* lst = tlist + (int64_t)fb * list_cap + (int64_t)tile * cap;
    for (int base = 0; base < n_ent; base += 256) {   // same trip count for the whole block
      const int e = base + threadIdx.x;
      const bool have = e < n_ent;
      raster_round(c, m, cam, have, have ? (uint32_t)lst[e] : 0u, H, W, tx1, ty1, queue, &queue_n);
    }
  } else {
    // the tile's list overflowed its capacity: walk every triangle of every
    // visible cluster instead (slow, same result)
    const int nvis = vis_n[fb];
    for (int w0 = 0; w0 < nvis; w0 += 4) {
      const int w = w0 + (threadIdx.x >> 6);
      const int64_t t = w < nvis ? (int64_t)vis[(int64_t)fb * m.n_clusters + w] * kClusterTris + (threadIdx.x & 63)
                                 : m.T;
      raster_round(c, m, cam, t < m.T, (uint32_t)t, H, W, tx1, ty1, queue, &queue_n);
    }
  }
  // (every round ends at a barrier: the tile's depth keys are final here)
  // ---- resolve every pixel of the tile: PPT pixels per thread, in groups of
  // G whose memory round trips overlap; triangle, depth and feature outputs
  // are written as soon as they are known ----
  constexpr int PPT = TS * TS / 256;
  int32_t tri[PPT], l[PPT];
  bool use[PPT];
  auto pix_of = [&](int r) {
    const int i = threadIdx.x + 256 * r;
    return (int64_t)fb * HW + (int64_t)(ty0 + i / TS) * W + (tx0 + i % TS);
  };
  auto in_of = [&](int r) {
    const int i = threadIdx.x + 256 * r;
    return tx0 + (i % TS) <= tx1 && ty0 + (i / TS) <= ty1;
  };
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    const unsigned long long k = key[threadIdx.x + 256 * r];
    tri[r] = (in_of(r) && k != ~0ull) ? (int32_t)(uint32_t)(k & 0xffffffffull) : -1;
    l[r] = -1;
  }
  constexpr int G = PPT < 2 ? PPT : 2;   // pixels whose loads are in flight together (16-pixel tiles: 1)
  static_assert(PPT % G == 0, "pixel groups divide the pixels per thread");
#pragma unroll
  for (int h = 0; h < PPT; h += G) {
    float4 tv[G][3];
    bool vis[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const int r = h + q;
      if (tri[r] >= 0) {
        tv[q][0] = m.tri_v[3 * (int64_t)tri[r]];
        tv[q][1] = m.tri_v[3 * (int64_t)tri[r] + 1];
        tv[q][2] = m.tri_v[3 * (int64_t)tri[r] + 2];
      }
      vis[q] = !out.valid || (tri[r] >= 0 && out.valid[pix_of(r)]);
    }
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const int r = h + q;
      use[r] = tri[r] >= 0 && vis[q];
      float z = __builtin_nanf("");
      float4 geo = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (tri[r] >= 0) {
        const int i = threadIdx.x + 256 * r;
        const float4 p = tv[q][0], qq = tv[q][1], t3 = tv[q][2];
        const RayK rk = ray_consts(to_cam(cam, p.x, p.y, p.z), to_cam(cam, p.w, qq.x, qq.y),
                                   to_cam(cam, qq.z, qq.w, t3.x));
        const float rx = rxs[i % TS], ry = rys[i / TS];
        const float den = rdot(rx, ry, rk.n);
        z = rk.d / den;
        const float u = rdot(rx, ry, rk.nu) / den;
        const float v = rdot(rx, ry, rk.nv) / den;
        l[r] = (int32_t)(row_offset(m, tri[r]) + texel_id(tri_s(m, tri[r]), m.split, u, v));
        if (out.geo) {
          // |cos| of the angle between the ray and the triangle normal, depth
          // squashed to [0, 1), 3 * smallest barycentric clamped to [0, 1]
          const float rl = sqrtf(rx * rx + ry * ry + 1.0f);
          const float nl = sqrtf(rk.n.x * rk.n.x + rk.n.y * rk.n.y + rk.n.z * rk.n.z);
          const float cs = nl > 0.0f ? fabsf(den) / (rl * nl) : 0.0f;
          const float b = 3.0f * fminf(fminf(u, v), 1.0f - u - v);
          geo = make_float4(cs, z / (1.0f + z), fminf(fmaxf(b, 0.0f), 1.0f), 0.0f);
        }
      }
      if (in_of(r)) {
        const int64_t px = pix_of(r);
        if (out.tri) out.tri[px] = tri[r];
        if (out.z) out.z[px] = z;
        if (out.geo) out.geo[px] = geo;
      }
    }
  }
  if (out.tricnt) {
#pragma unroll
    for (int r = 0; r < PPT; ++r)
      if (tri[r] >= 0) atomicAdd(out.tricnt + (int64_t)fb * m.T + tri[r], 1);
  }
  if (out.seg || out.cnt) {
    // A wave holds whole tile rows (TS consecutive lanes per row).  Lanes next
    // to each other with the same key form a run; the run's first lane adds
    // the run length to the key's counter with one atomic.  Only rows inside
    // the accumulator's window count (row l is counted at l - win_lo).
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (2ull << lane) - 1ull;   // lanes 0..lane (lane 63: all)
    bool win[PPT];
    int lw[PPT];
#pragma unroll
    for (int r = 0; r < PPT; ++r) {
      const int64_t d = (int64_t)l[r] - m.win_lo;
      win[r] = use[r] && d >= 0 && d < m.n_rows;
      lw[r] = win[r] ? (int)d : -1;
    }
    if (out.cnt) {
      // per-frame pixel counts of every texel row (w^(I) outside the grouped gather)
      constexpr unsigned long long kRowStart = TS == 16 ? 0x0001000100010001ull : 0x0000000100000001ull;
#pragma unroll
      for (int r = 0; r < PPT; ++r) {
        const int key = lw[r];
        const int prev = __shfl_up(key, 1);
        const unsigned long long heads = __ballot(key != prev) | kRowStart;
        const unsigned long long after = heads & ~below;
        const int next = after ? __ffsll(after) - 1 : 64;
        if (win[r] && 63 - __clzll(heads & below) == lane)
          atomicAdd(out.cnt + (int64_t)fb * out.cnt_stride + key, next - lane);
      }
    }
    if (out.seg) {
      // sorted scatter, first level: pixels counted per bucket of
      // 2^kBucketShift texel rows.  Runs of same-bucket lanes add their
      // length to the tile's count of the bucket (an LDS table, open
      // addressing); then one global atomic per (tile, bucket) reserves the
      // tile's slots, and a run's pixels take consecutive ranks from its
      // place in them, so the fill writes them contiguously.  A bucket that
      // finds the table full is counted with a global atomic per run.
      for (int i = threadIdx.x; i < kTileSlots; i += 256) {
        hkey[i] = -1;
        hcnt[i] = 0;
      }
      __syncthreads();
      int slot[PPT], rb[PPT], head[PPT];
#pragma unroll
      for (int r = 0; r < PPT; ++r) {
        const int key = win[r] ? lw[r] >> kBucketShift : -1;
        const int prev = __shfl_up(key, 1);
        const unsigned long long heads = __ballot(key != prev) | 1ull;
        const unsigned long long after = heads & ~below;
        const int next = after ? __ffsll(after) - 1 : 64;
        head[r] = 63 - __clzll(heads & below);
        slot[r] = -1;
        rb[r] = 0;
        if (win[r] && head[r] == lane) {
          int h = (int)(((uint32_t)key * 2654435761u) >> (32 - kTileSlotBits));
          for (int probe = 0; probe < kTileSlots; ++probe) {
            const int old = atomicCAS(&hkey[h], -1, key);
            if (old == -1 || old == key) {
              slot[r] = h;
              break;
            }
            h = (h + 1) & (kTileSlots - 1);
          }
          if (slot[r] >= 0) rb[r] = atomicAdd(&hcnt[slot[r]], next - lane);
          else rb[r] = atomicAdd(out.seg + key, next - lane);   // table full: this run reserves alone
        }
      }
      __syncthreads();
      for (int i = threadIdx.x; i < kTileSlots; i += 256)
        if (hkey[i] >= 0) hbase[i] = atomicAdd(out.seg + hkey[i], hcnt[i]);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < PPT; ++r) {
        const int s = __shfl(slot[r], head[r]);
        const int base = __shfl(rb[r], head[r]) + (s >= 0 ? hbase[s] : 0);
        if (win[r]) out.rank[pix_of(r)] = base + (lane - head[r]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < PPT; ++r)
    if (out.l && in_of(r)) out.l[pix_of(r)] = l[r];
}

// ---- launcher ---------------------------------------------------------------
template <int TS>
hipError_t render_batch_ts(const MeshDev& m, const float* cams, int nb, int H, int W, const RasterWs& ws,
                           const RasterOut& out, hipStream_t s) {
  const int ntx = (W + TS - 1) / TS, nty = (H + TS - 1) / TS;
  const int ntiles = ntx * nty;
  hipError_t e = launch_zero(ws.vis_n, (int64_t)nb * 4, s);
  if (e != hipSuccess) return e;
  if (m.n_clusters > 0)
    k_cull_clusters<<<dim3((unsigned)((m.n_clusters + 255) / 256), (unsigned)nb), 256, 0, s>>>(m, cams, H, W, ws.vis,
                                                                                               ws.vis_n);
  const unsigned gb = (unsigned)std::min<int64_t>((m.n_clusters + 3) / 4 + 1, 256);
  const int cap = (int)std::min<int64_t>(ws.list_cap / ntiles, INT32_MAX);
  const size_t bin_lds = ntiles <= kBinLdsTiles ? (size_t)ntiles * 2 * sizeof(int) : 0;
  k_bin<TS><<<dim3(gb, (unsigned)nb), 256, bin_lds, s>>>(m, cams, H, W, ws.vis, ws.vis_n, ws.tcnt, ws.tlist,
                                                         ws.list_cap, cap);
  k_tile_raster<TS><<<dim3((unsigned)ntiles, (unsigned)nb), 256, 0, s>>>(m, cams, H, W, ws.vis, ws.vis_n, ws.tcnt,
                                                                         ws.tlist, ws.list_cap, cap, out);
  return hipGetLastError();
}

hipError_t launch_render_batch(const MeshDev& m, const float* cams, int nb, int H, int W, const RasterWs& ws,
                               const RasterOut& out, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  return m.tile == 16 ? render_batch_ts<16>(m, cams, nb, H, W, ws, out, s)
                      : render_batch_ts<32>(m, cams, nb, H, W, ws, out, s);
}

}  // namespace lf
