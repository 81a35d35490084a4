/*
 * CPU ORACLE for label fusion in semantically textured meshes
 * (Fervers et al., "Improving Semantic Image Segmentation via Label Fusion in
 * Semantically Textured Meshes").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path (the
 * HIP library) never calls it and shares no code, header, table or helper
 * with it.
 *
 * It is a plain, slow, direct evaluation of what the method computes:
 *
 *   - per-triangle uv frame and texel counts            (Section 3.1)
 *   - renderer: z-buffered projection of every triangle, (Section 3.3.1,
 *     the triangle id and texel id of every pixel          eq. idtexel)
 *   - correspondence sets K_x                            (Section 3.1, eq. projected-pixels)
 *   - row l = id_t + id_x of the texel array              (Section 3.3.2, eq. texel-in-array)
 *   - weighted aggregation f_w-sum / f_w-mul / f_w-maxsum (Section 3.2.1-3.2.2,
 *     eqs. maxsum, mul, sum, w-maxsum, w-mul, w-sum)
 *   - pixel weights w^(P) = 1 and w^(I) = 1/|K_i ∩ K_x|  (Section 3.2.2)
 *   - norm (L1) and the argmax class of every texel      (Section 3.2.1)
 *   - render-back of the fused labels                     (Section 3.2.1, last paragraphs)
 *
 * Precision: integer decisions taken from floating point (which triangle a
 * pixel sees, which texel cell it lands in, the uv origin of a triangle) are
 * taken in IEEE binary32 with every operation written out in a fixed order
 * (explicit fmaf, no contraction: build with -ffp-contract=off, no fast-math),
 * so an independent GPU implementation of the same rules can match them bit
 * for bit.  All fusion arithmetic is binary64.
 *
 * Readings of points the paper leaves open (camera model, fill rule, clipping,
 * tie-breaks, texel index bijection, SPLIT scheme) are stated next to the
 * code that takes them.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define OR_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------ texels */

/* Number of texels of a triangle with s steps per uv dimension.
 * scheme 0 (SQUARE): the paper's (s^2 + s)/2 cells (Section 3.1, Fig. texels).
 * scheme 1 (SPLIT): every full square cell (i + j <= s - 2) is cut along its
 * anti-diagonal into two triangles, giving s^2 texels of equal uv area. */
OR_API int64_t or_texel_count(int32_t s, int32_t scheme) {
    if (s < 1) return -1;
    if (scheme == 0) return (int64_t)s * (s + 1) / 2;
    if (scheme == 1) return (int64_t)s * s;
    return -1;
}

/* Texel id of the point (u, v) of a triangle (eq. idtexel, read as a bijection).
 * The cell of (u, v) is (a, b) = (floor(s u), floor(s v)) restricted to the
 * triangle a + b <= s - 1 (Section 3.1: u, v >= 0, u + v < 1; cell
 * [a/s, (a+1)/s) x [b/s, (b+1)/s)).  The printed formula (a^2 + a)/2 + b is not
 * injective on that domain (it needs b <= a); the bijection used keeps its
 * triangular-number form with the row index r = s - 1 - a, whose row holds
 * b = 0..r:  id = r (r + 1)/2 + b, in [0, s (s + 1)/2).
 * Points outside the triangle (possible at silhouettes, where coverage comes
 * from snapped vertices) are clamped into the nearest valid cell; NaN maps
 * to 0.
 * SPLIT: inside a full cell, the upper-right half (fractional parts summing to
 * >= 1) gets id s (s + 1)/2 + r' (r' + 1)/2 + b with r' = s - 2 - a. */
OR_API int32_t or_texel_id(int32_t s, int32_t scheme, float u, float v) {
    float fs = (float)s;
    float su = fs * u;
    float sv = fs * v;
    int32_t a, b;
    if (!(su > 0.0f)) a = 0;
    else if (su >= fs) a = s - 1;
    else a = (int32_t)floorf(su);
    int32_t bmax = s - 1 - a;
    if (!(sv > 0.0f)) b = 0;
    else if (sv >= (float)(bmax + 1)) b = bmax;
    else b = (int32_t)floorf(sv);
    int32_t r = s - 1 - a;
    int32_t id = r * (r + 1) / 2 + b;
    if (scheme == 1 && a + b <= s - 2) {
        float fu = su - (float)a;
        float fv = sv - (float)b;
        if (fu + fv >= 1.0f) {
            int32_t r2 = s - 2 - a;
            id = s * (s + 1) / 2 + r2 * (r2 + 1) / 2 + b;
        }
    }
    return id;
}

/* --------------------------------------------------------------- mesh prep */

static float dot3f(const float a[3], const float b[3]) {
    return fmaf(a[0], b[0], fmaf(a[1], b[1], a[2] * b[2]));
}

/* uv frame of every triangle (Section 3.1): the origin is the vertex whose
 * interior angle is closest to a right angle, i.e. the smallest
 * cos^2 = (a.b)^2 / ((a.a)(b.b)) with a, b the edges leaving it, in binary32,
 * ties to the lowest local index.  Output order (A, B, C): A is the origin
 * (uv (0,0)), B = next vertex in the input order (uv (0,1)), C = the one after
 * (uv (1,0)), following the order the vertices' uv are listed in.
 * |X_t| per triangle and the exclusive prefix offsets id_t (Section 3.3.2).
 * Returns 0, or -1 if a face index is out of range / s < 1. */
OR_API int32_t or_prepare_mesh(int64_t n_vertices, const float* verts, int64_t n_faces,
                               const int32_t* faces, const int32_t* s_face, int32_t s_uniform,
                               int32_t scheme, int32_t* faces_uv, int32_t* s_out, int64_t* off) {
    int64_t acc = 0;
    for (int64_t t = 0; t < n_faces; ++t) {
        int32_t idx[3];
        for (int m = 0; m < 3; ++m) {
            idx[m] = faces[3 * t + m];
            if (idx[m] < 0 || idx[m] >= n_vertices) return -1;
        }
        float cm[3];
        for (int m = 0; m < 3; ++m) {
            const float* P = verts + 3 * (int64_t)idx[m];
            const float* Q = verts + 3 * (int64_t)idx[(m + 1) % 3];
            const float* R = verts + 3 * (int64_t)idx[(m + 2) % 3];
            float a[3] = {Q[0] - P[0], Q[1] - P[1], Q[2] - P[2]};
            float b[3] = {R[0] - P[0], R[1] - P[1], R[2] - P[2]};
            float ab = dot3f(a, b), aa = dot3f(a, a), bb = dot3f(b, b);
            cm[m] = (ab * ab) / (aa * bb);
        }
        int o = 0;
        if (cm[1] < cm[o]) o = 1;
        if (cm[2] < cm[o]) o = 2;
        faces_uv[3 * t + 0] = idx[o];
        faces_uv[3 * t + 1] = idx[(o + 1) % 3];
        faces_uv[3 * t + 2] = idx[(o + 2) % 3];
        int32_t s = s_face ? s_face[t] : s_uniform;
        if (s < 1) return -1;
        s_out[t] = s;
        off[t] = acc;
        acc += or_texel_count(s, scheme);
    }
    off[n_faces] = acc;
    return 0;
}

/* ------------------------------------------------------------------ raster */

/* Camera record: fx fy cx cy R[9] (row-major, world->camera) t[3].
 * Pinhole, no distortion, OpenCV axes; pixel (x, y) has its centre at
 * (x + 1/2, y + 1/2). */
typedef struct { float fx, fy, cx, cy, R[9], t[3]; } cam_t;

static void to_camera(const cam_t* c, const float* X, float out[3]) {
    out[0] = fmaf(c->R[0], X[0], fmaf(c->R[1], X[1], fmaf(c->R[2], X[2], c->t[0])));
    out[1] = fmaf(c->R[3], X[0], fmaf(c->R[4], X[1], fmaf(c->R[5], X[2], c->t[1])));
    out[2] = fmaf(c->R[6], X[0], fmaf(c->R[7], X[1], fmaf(c->R[8], X[2], c->t[2])));
}

static void cross3f(const float a[3], const float b[3], float o[3]) {
    o[0] = fmaf(a[1], b[2], -(a[2] * b[1]));
    o[1] = fmaf(a[2], b[0], -(a[0] * b[2]));
    o[2] = fmaf(a[0], b[1], -(a[1] * b[0]));
}

/* Ray-cast constants of the ORIGINAL triangle (A, B, C) in camera space:
 * the pixel ray r = (rx, ry, 1) meets A + u (C - A) + v (B - A) at depth z
 * (Cramer's rule): N = e1 x e2, Nu = e2 x A, Nv = A x e1, D = A . N with
 * e1 = C - A, e2 = B - A;  den = r.N, u = r.Nu/den, v = r.Nv/den, z = D/den. */
typedef struct { float N[3], Nu[3], Nv[3], D; } rc_t;

static void raycast_consts(const float A[3], const float B[3], const float C[3], rc_t* k) {
    float e1[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
    float e2[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    cross3f(e1, e2, k->N);
    cross3f(e2, A, k->Nu);
    cross3f(A, e1, k->Nv);
    k->D = dot3f(A, k->N);
}

static float ray_x(const cam_t* c, int32_t x) { return (((float)x + 0.5f) - c->cx) / c->fx; }
static float ray_y(const cam_t* c, int32_t y) { return (((float)y + 0.5f) - c->cy) / c->fy; }

static float rdot(float rx, float ry, const float n[3]) { return fmaf(rx, n[0], fmaf(ry, n[1], n[2])); }

#define GUARD 1048576.0f  /* |projected coordinate| <= 2^20 px after clipping */

/* Clipping planes in camera space, distance d >= 0 means inside:
 *   0: z - z_near
 *   1: (G - cx) z - fx x      (px <= G)
 *   2: (G + cx) z + fx x      (px >= -G)
 *   3: (G - cy) z - fy y      (py <= G)
 *   4: (G + cy) z + fy y      (py >= -G)                                    */
static float plane_dist(int p, const float v[3], const cam_t* c, float z_near) {
    switch (p) {
        case 0: return v[2] - z_near;
        case 1: return fmaf(GUARD - c->cx, v[2], -(c->fx * v[0]));
        case 2: return fmaf(GUARD + c->cx, v[2], c->fx * v[0]);
        case 3: return fmaf(GUARD - c->cy, v[2], -(c->fy * v[1]));
        default: return fmaf(GUARD + c->cy, v[2], c->fy * v[1]);
    }
}

/* Sutherland-Hodgman against the five planes in order.  For each edge
 * (P_i, P_{i+1}) of the current polygon: P_i is kept if inside; if the edge
 * crosses the plane, the crossing point is appended, computed from the inside
 * end I towards the outside end O as I + alpha (O - I), alpha = dI/(dI - dO),
 * each component fmaf(alpha, O - I, I) -- the same bits from both triangles
 * sharing the edge.  Returns the vertex count (0..8). */
static int clip_polygon(float poly[8][3], int n, const cam_t* c, float z_near) {
    float tmp[8][3];
    for (int p = 0; p < 5 && n > 0; ++p) {
        float d[8];
        for (int i = 0; i < n; ++i) d[i] = plane_dist(p, poly[i], c, z_near);
        int m = 0;
        for (int i = 0; i < n; ++i) {
            int j = (i + 1) % n;
            int in_i = d[i] >= 0.0f, in_j = d[j] >= 0.0f;
            if (in_i) { memcpy(tmp[m], poly[i], sizeof(float) * 3); ++m; }
            if (in_i != in_j) {
                const float* I = in_i ? poly[i] : poly[j];
                const float* O = in_i ? poly[j] : poly[i];
                float dI = in_i ? d[i] : d[j];
                float dO = in_i ? d[j] : d[i];
                float alpha = dI / (dI - dO);
                for (int k = 0; k < 3; ++k) tmp[m][k] = fmaf(alpha, O[k] - I[k], I[k]);
                ++m;
            }
        }
        n = m;
        memcpy(poly, tmp, sizeof(float) * 3 * (size_t)n);
    }
    return n;
}

/* Snap to 8 sub-pixel bits, round half to even. */
static void project_snap(const cam_t* c, const float v[3], int32_t* X, int32_t* Y) {
    float xn = v[0] / v[2];
    float yn = v[1] / v[2];
    float px = fmaf(c->fx, xn, c->cx);
    float py = fmaf(c->fy, yn, c->cy);
    *X = (int32_t)rintf(px * 256.0f);
    *Y = (int32_t)rintf(py * 256.0f);
}

/* Edge function of edge i->j at point P (twice the signed area), exact int64. */
static int64_t edge_fn(int64_t Xi, int64_t Yi, int64_t Xj, int64_t Yj, int64_t XP, int64_t YP) {
    return (Xj - Xi) * (YP - Yi) - (Yj - Yi) * (XP - Xi);
}

/* Top-left rule for an edge i->j of a triangle with positive area (interior
 * where all edge functions are > 0, image y pointing down): a pixel centre on
 * the edge belongs to the triangle iff the edge is a left edge (interior on
 * its +x side: dy < 0) or a top edge (horizontal with interior below:
 * dy == 0, dx > 0). */
static int is_top_left(int64_t dx, int64_t dy) { return dy < 0 || (dy == 0 && dx > 0); }

static int64_t floordiv256(int64_t a) { return a >= 0 ? a / 256 : -((-a + 255) / 256); }

/* Visit every pixel centre covered by the snapped triangle (X0..Y2), calling
 * fn(ctx, x, y).  Returns 0 if the triangle has zero area. */
typedef void (*pix_fn)(void* ctx, int32_t x, int32_t y);

static void cover_triangle(int64_t X0, int64_t Y0, int64_t X1, int64_t Y1, int64_t X2, int64_t Y2,
                           int32_t H, int32_t W, pix_fn fn, void* ctx) {
    int64_t area = edge_fn(X0, Y0, X1, Y1, X2, Y2);
    if (area == 0) return;
    if (area < 0) { int64_t tx = X1, ty = Y1; X1 = X2; Y1 = Y2; X2 = tx; Y2 = ty; }
    int64_t xmin = X0 < X1 ? (X0 < X2 ? X0 : X2) : (X1 < X2 ? X1 : X2);
    int64_t xmax = X0 > X1 ? (X0 > X2 ? X0 : X2) : (X1 > X2 ? X1 : X2);
    int64_t ymin = Y0 < Y1 ? (Y0 < Y2 ? Y0 : Y2) : (Y1 < Y2 ? Y1 : Y2);
    int64_t ymax = Y0 > Y1 ? (Y0 > Y2 ? Y0 : Y2) : (Y1 > Y2 ? Y1 : Y2);
    int64_t x0 = floordiv256(xmin) - 1, x1 = floordiv256(xmax) + 1;
    int64_t y0 = floordiv256(ymin) - 1, y1 = floordiv256(ymax) + 1;
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    if (x1 > W - 1) x1 = W - 1;
    if (y1 > H - 1) y1 = H - 1;
    int tl01 = is_top_left(X1 - X0, Y1 - Y0);
    int tl12 = is_top_left(X2 - X1, Y2 - Y1);
    int tl20 = is_top_left(X0 - X2, Y0 - Y2);
    for (int64_t y = y0; y <= y1; ++y) {
        for (int64_t x = x0; x <= x1; ++x) {
            int64_t PX = 256 * x + 128, PY = 256 * y + 128;
            int64_t e01 = edge_fn(X0, Y0, X1, Y1, PX, PY);
            int64_t e12 = edge_fn(X1, Y1, X2, Y2, PX, PY);
            int64_t e20 = edge_fn(X2, Y2, X0, Y0, PX, PY);
            int in01 = e01 > 0 || (e01 == 0 && tl01);
            int in12 = e12 > 0 || (e12 == 0 && tl12);
            int in20 = e20 > 0 || (e20 == 0 && tl20);
            if (in01 && in12 && in20) fn(ctx, (int32_t)x, (int32_t)y);
        }
    }
}

typedef struct {
    const cam_t* cam;
    const rc_t* rc;
    uint64_t* keys;
    int32_t* count;
    uint32_t tri;
    int32_t W;
} frag_ctx;

static float depth_at(const cam_t* c, const rc_t* k, int32_t x, int32_t y) {
    float rx = ray_x(c, x), ry = ray_y(c, y);
    float den = rdot(rx, ry, k->N);
    return k->D / den;
}

/* z-buffer: key = (bits(z) << 32) | triangle id, smallest key wins, i.e. the
 * nearest surface (z > 0 and finite) and, on equal depth, the lower id. */
static void frag_depth(void* vctx, int32_t x, int32_t y) {
    frag_ctx* f = (frag_ctx*)vctx;
    float z = depth_at(f->cam, f->rc, x, y);
    if (!(z > 0.0f) || !(z <= 3.4028234663852886e38f)) return;
    uint32_t zb;
    memcpy(&zb, &z, 4);
    uint64_t key = ((uint64_t)zb << 32) | f->tri;
    uint64_t* slot = &f->keys[(int64_t)y * f->W + x];
    if (key < *slot) *slot = key;
}

static void frag_count(void* vctx, int32_t x, int32_t y) {
    frag_ctx* f = (frag_ctx*)vctx;
    f->count[(int64_t)y * f->W + x] += 1;
}

/* One triangle of one frame: transform, clip, fan-triangulate, cover. */
static void raster_triangle(const cam_t* cam, float z_near, const float* verts, const int32_t* fuv,
                            uint32_t t, int32_t H, int32_t W, pix_fn fn, frag_ctx* ctx) {
    float A[3], B[3], C[3];
    to_camera(cam, verts + 3 * (int64_t)fuv[0], A);
    to_camera(cam, verts + 3 * (int64_t)fuv[1], B);
    to_camera(cam, verts + 3 * (int64_t)fuv[2], C);
    rc_t rc;
    raycast_consts(A, B, C, &rc);
    float poly[8][3];
    memcpy(poly[0], A, 12); memcpy(poly[1], B, 12); memcpy(poly[2], C, 12);
    int n = clip_polygon(poly, 3, cam, z_near);
    if (n < 3) return;
    int32_t X[8], Y[8];
    for (int i = 0; i < n; ++i) project_snap(cam, poly[i], &X[i], &Y[i]);
    ctx->rc = &rc;
    ctx->tri = t;
    for (int i = 1; i + 1 < n; ++i)
        cover_triangle(X[0], Y[0], X[i], Y[i], X[i + 1], Y[i + 1], H, W, fn, ctx);
}

/* Renderer for one frame (Section 3.3.1).  Outputs per pixel: triangle id
 * (-1 = background), texel row l = off[t] + id_x (-1), depth z (NaN), uv.
 * Any of the outputs may be NULL. */
OR_API int32_t or_raster_frame(const float* verts, int64_t n_faces, const int32_t* faces_uv,
                               const int32_t* s_face, const int64_t* off, int32_t scheme,
                               const float* cam16, float z_near, int32_t H, int32_t W,
                               int32_t* tri_out, int32_t* l_out, float* z_out, float* uv_out) {
    cam_t cam;
    memcpy(&cam, cam16, sizeof(cam));
    int64_t npx = (int64_t)H * W;
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)npx);
    if (!keys) return -1;
    for (int64_t i = 0; i < npx; ++i) keys[i] = UINT64_MAX;
    frag_ctx ctx = {&cam, NULL, keys, NULL, 0, W};
    for (int64_t t = 0; t < n_faces; ++t)
        raster_triangle(&cam, z_near, verts, faces_uv + 3 * t, (uint32_t)t, H, W, frag_depth, &ctx);
    for (int32_t y = 0; y < H; ++y) {
        for (int32_t x = 0; x < W; ++x) {
            int64_t i = (int64_t)y * W + x;
            int32_t tri = -1, l = -1;
            float z = NAN, u = NAN, v = NAN;
            if (keys[i] != UINT64_MAX) {
                tri = (int32_t)(keys[i] & 0xffffffffu);
                const int32_t* fuv = faces_uv + 3 * (int64_t)tri;
                float A[3], B[3], C[3];
                to_camera(&cam, verts + 3 * (int64_t)fuv[0], A);
                to_camera(&cam, verts + 3 * (int64_t)fuv[1], B);
                to_camera(&cam, verts + 3 * (int64_t)fuv[2], C);
                rc_t rc;
                raycast_consts(A, B, C, &rc);
                float rx = ray_x(&cam, x), ry = ray_y(&cam, y);
                float den = rdot(rx, ry, rc.N);
                z = rc.D / den;
                u = rdot(rx, ry, rc.Nu) / den;
                v = rdot(rx, ry, rc.Nv) / den;
                l = (int32_t)(off[tri] + or_texel_id(s_face[tri], scheme, u, v));
            }
            if (tri_out) tri_out[i] = tri;
            if (l_out) l_out[i] = l;
            if (z_out) z_out[i] = z;
            if (uv_out) { uv_out[2 * i] = u; uv_out[2 * i + 1] = v; }
        }
    }
    free(keys);
    return 0;
}

/* Coverage count per pixel with the depth test off (watertightness checks). */
OR_API int32_t or_coverage_count(const float* verts, int64_t n_faces, const int32_t* faces_uv,
                                 const float* cam16, float z_near, int32_t H, int32_t W,
                                 int32_t* count) {
    cam_t cam;
    memcpy(&cam, cam16, sizeof(cam));
    memset(count, 0, sizeof(int32_t) * (size_t)H * W);
    frag_ctx ctx = {&cam, NULL, NULL, count, 0, W};
    for (int64_t t = 0; t < n_faces; ++t)
        raster_triangle(&cam, z_near, verts, faces_uv + 3 * t, (uint32_t)t, H, W, frag_count, &ctx);
    return 0;
}

/* Snapped, clipped sub-triangles of one triangle (for brute-force checks):
 * writes up to 6 sub-triangles as 6 ints each; returns their count. */
OR_API int32_t or_snapped_fan(const float* verts, const int32_t* fuv3, const float* cam16,
                              float z_near, int32_t* out) {
    cam_t cam;
    memcpy(&cam, cam16, sizeof(cam));
    float poly[8][3];
    to_camera(&cam, verts + 3 * (int64_t)fuv3[0], poly[0]);
    to_camera(&cam, verts + 3 * (int64_t)fuv3[1], poly[1]);
    to_camera(&cam, verts + 3 * (int64_t)fuv3[2], poly[2]);
    int n = clip_polygon(poly, 3, &cam, z_near);
    if (n < 3) return 0;
    int32_t X[8], Y[8];
    for (int i = 0; i < n; ++i) project_snap(&cam, poly[i], &X[i], &Y[i]);
    int k = 0;
    for (int i = 1; i + 1 < n; ++i, ++k) {
        out[6 * k + 0] = X[0]; out[6 * k + 1] = Y[0];
        out[6 * k + 2] = X[i]; out[6 * k + 3] = Y[i];
        out[6 * k + 4] = X[i + 1]; out[6 * k + 5] = Y[i + 1];
    }
    return k;
}

/* Camera-space polygon of one triangle after the five-plane clip, before
 * projection (for checks of the clipping rules): the world-space corners A,
 * B, C are taken in the order given; out receives up to 8 vertices of 3
 * floats; returns their count (0..8). */
OR_API int32_t or_clip_triangle(const float* cam16, float z_near, const float* A, const float* B, const float* C,
                                float* out) {
    cam_t cam;
    memcpy(&cam, cam16, sizeof(cam));
    float poly[8][3];
    to_camera(&cam, A, poly[0]);
    to_camera(&cam, B, poly[1]);
    to_camera(&cam, C, poly[2]);
    int n = clip_polygon(poly, 3, &cam, z_near);
    memcpy(out, poly, sizeof(float) * 3 * (size_t)n);
    return n;
}

/* ---------------------------------------------------------------- fusion */

/* OCP 8-bit floating point, E4M3FN: 1 sign, 4 exponent (bias 7), 3 mantissa
 * bits; exponent 0 is subnormal (m/8 * 2^-6); S.1111.111 is NaN; no infinity. */
OR_API double or_e4m3_decode(uint8_t q) {
    int sgn = (q >> 7) & 1, e = (q >> 3) & 15, m = q & 7;
    double v;
    if (e == 15 && m == 7) return NAN;
    if (e == 0) v = ldexp((double)m / 8.0, -6);
    else v = ldexp(1.0 + (double)m / 8.0, e - 7);
    return sgn ? -v : v;
}

/* Aggregators (Section 3.2.1/3.2.2):
 *   0 SUM:    A_x = sum_k w_k p_k                        (eq. w-sum)
 *   1 MUL:    A_x = sum_k w_k log p_k  (log of eq. w-mul's product)
 *   2 MAXSUM: A_x = sum_k w_k g(p_k), g keeps the entries equal to max p_k (eq. w-maxsum)
 * Weights (Section 3.2.2): 0 = w^(P) = 1; 1 = w^(I) = 1 / |K_i ∩ K_{x_k}|, the
 * number of valid pixels of the same frame on the same texel; 2 = a given
 * per-pixel weight array.
 * Probabilities: prob_dtype 0 = float32 [F][c][H][W] (strides in elements,
 * order f, c, y, x); 3 = E4M3FN codes with a float32 per-pixel scale
 * [F][H][W] (p = decode(q) * scale).
 * A (binary64, [n_texels][c]) and W_sum ([n_texels], total weight per texel)
 * are accumulated into (not cleared), so frames can be fused incrementally. */
OR_API int32_t or_fuse(int32_t F, int32_t H, int32_t W, int32_t c, const int32_t* l, const uint8_t* valid,
                       const void* probs, int32_t prob_dtype, const int64_t* strides, const float* scale,
                       int32_t aggregator, int32_t weighting, const float* wpix, int64_t n_texels,
                       double* A, double* W_sum) {
    int64_t npx = (int64_t)H * W;
    int32_t* cnt = NULL;
    if (weighting == 1) {
        cnt = (int32_t*)calloc((size_t)n_texels, sizeof(int32_t));
        if (!cnt) return -1;
    }
    double* p = (double*)malloc(sizeof(double) * (size_t)c);
    for (int32_t f = 0; f < F; ++f) {
        const int32_t* lf = l + (int64_t)f * npx;
        const uint8_t* vf = valid ? valid + (int64_t)f * npx : NULL;
        if (weighting == 1) {
            for (int64_t i = 0; i < npx; ++i)
                if (lf[i] >= 0 && (!vf || vf[i])) cnt[lf[i]] += 1;
        }
        for (int32_t y = 0; y < H; ++y) {
            for (int32_t x = 0; x < W; ++x) {
                int64_t i = (int64_t)y * W + x;
                int32_t li = lf[i];
                if (li < 0 || (vf && !vf[i])) continue;
                if (li >= n_texels) { free(p); free(cnt); return -2; }
                double w = 1.0;
                if (weighting == 1) w = 1.0 / (double)cnt[li];
                else if (weighting == 2) w = (double)wpix[(int64_t)f * npx + i];
                for (int32_t j = 0; j < c; ++j) {
                    int64_t e = f * strides[0] + j * strides[1] + y * strides[2] + x * strides[3];
                    if (prob_dtype == 0) p[j] = (double)((const float*)probs)[e];
                    else p[j] = or_e4m3_decode(((const uint8_t*)probs)[e]) * (double)scale[(int64_t)f * npx + i];
                }
                double* row = A + (int64_t)li * c;
                if (aggregator == 0) {
                    for (int32_t j = 0; j < c; ++j) row[j] += w * p[j];
                } else if (aggregator == 1) {
                    for (int32_t j = 0; j < c; ++j) row[j] += w * log(p[j]);
                } else {
                    double mx = p[0];
                    for (int32_t j = 1; j < c; ++j) if (p[j] > mx) mx = p[j];
                    for (int32_t j = 0; j < c; ++j) if (p[j] == mx) row[j] += w * p[j];
                }
                if (W_sum) W_sum[li] += w;
            }
        }
        if (weighting == 1) {
            for (int64_t i = 0; i < npx; ++i)
                if (lf[i] >= 0 && (!vf || vf[i])) cnt[lf[i]] = 0;
        }
    }
    free(p);
    free(cnt);
    return 0;
}

/* norm and argmax (Section 3.2.1).  SUM / MAXSUM: S = sum_j A_j; if S > 0,
 * P = A / S and the label is the first index of the maximum; an unobserved
 * texel (S = 0, no definition in the paper) gets P = 0 and label 255.
 * MUL: the product of eq. w-mul normalised, computed from its logarithm as
 * P_j = exp(A_j - max A) / sum_i exp(A_i - max A); a texel with no weight
 * (W_sum = 0) gets P = 0 and label 255. */
OR_API int32_t or_finalize(int64_t n_texels, int32_t c, const double* A, const double* W_sum,
                           int32_t aggregator, double* P, uint8_t* label) {
    for (int64_t x = 0; x < n_texels; ++x) {
        const double* a = A + x * c;
        double* o = P + x * c;
        if (aggregator == 1) {
            if (!(W_sum[x] > 0.0)) {
                for (int32_t j = 0; j < c; ++j) o[j] = 0.0;
                label[x] = 255;
                continue;
            }
            double mx = a[0];
            for (int32_t j = 1; j < c; ++j) if (a[j] > mx) mx = a[j];
            double s = 0.0;
            for (int32_t j = 0; j < c; ++j) s += exp(a[j] - mx);
            int32_t best = 0;
            for (int32_t j = 0; j < c; ++j) {
                o[j] = exp(a[j] - mx) / s;
                if (a[j] > a[best]) best = j;
            }
            label[x] = (uint8_t)best;
        } else {
            double s = 0.0;
            for (int32_t j = 0; j < c; ++j) s += a[j];
            if (!(s > 0.0)) {
                for (int32_t j = 0; j < c; ++j) o[j] = 0.0;
                label[x] = 255;
                continue;
            }
            int32_t best = 0;
            for (int32_t j = 0; j < c; ++j) {
                o[j] = a[j] / s;
                if (a[j] > a[best]) best = j;
            }
            label[x] = (uint8_t)best;
        }
    }
    return 0;
}

/* Render-back: each pixel gets the fused label of its texel, 255 where no
 * triangle is hit or the pixel is invalid. */
OR_API int32_t or_render(int64_t n_px, const int32_t* l, const uint8_t* valid, const uint8_t* label,
                         uint8_t* out) {
    for (int64_t i = 0; i < n_px; ++i) {
        int32_t li = l[i];
        out[i] = (li >= 0 && (!valid || valid[i])) ? label[li] : 255;
    }
    return 0;
}
