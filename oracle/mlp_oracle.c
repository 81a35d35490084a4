/*
 * CPU ORACLE of the learned per-observation fusion weight (test
 * infrastructure only; see semfuse_oracle.c).
 *
 * The paper weights every observation k of a texel by w_k (Section 3.2.2,
 * eqs. w-maxsum / w-mul / w-sum) with two fixed choices, w^(P) = 1 and
 * w^(I) = 1/|K_i ∩ K_x|.  The learned form replaces w_k by the output of a
 * small network on per-observation features phi_k in R^8:
 *
 *   h1 = relu(W1 q(phi) + b1)         W1: 64 x 8
 *   h2 = relu(W2 q(h1) + b2)          W2: 64 x 64,  q = round to bfloat16
 *   w  = sigmoid(w3 . h2 + b3)        w3: 64
 *
 * with the weights W1, W2, w3 and the inputs of the two matrix products
 * taken as bfloat16 values (biases binary32) and all arithmetic in binary64.  With rounding off (round_mode 0) the same code
 * is a plain binary64 network, which the finite-difference pins use.
 *
 * Training target: y_k = 1 when the observation's own argmax equals the
 * label the plain fusion gives its texel; loss = binary cross-entropy of w
 * against y, averaged over the batch.
 *
 * Features (per valid covered pixel k of frame i, camera ray r = (rx, ry, 1),
 * triangle normal n, uv (u, v) on it, depth z, probabilities p):
 *   0  |r.n| / (|r||n|)             cosine of the viewing angle
 *   1  z / (1 + z)                   depth
 *   2  -sum_j p_j ln p_j / ln c      normalised entropy (p_j <= 0 terms = 0)
 *   3  max_j p_j                      top-1 probability
 *   4  p_(1) - p_(2)                  top-1 minus top-2
 *   5  min(1, 3 min(u, v, 1-u-v))     closeness to the triangle's centroid
 *   6  min(2, ln n / ln 64)           n = pixels of frame i on the same texel
 *   7  |(x+1/2-cx, y+1/2-cy)| / |(cx, cy)|   radial image distance
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OM_API __attribute__((visibility("default")))

enum { NI = 8, NH = 64 };
/* flat parameter layout (binary32): W1[64][8], b1[64], W2[64][64], b2[64], w3[64], b3 */
enum { OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NI, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
       OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH, NPARAM = OFF_B3 + 1 };

OM_API int32_t om_nparam(void) { return NPARAM; }

/* bfloat16 round to nearest even of a binary32 value (returned as binary32). */
static float bf16_rne(float x) {
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) {       /* inf / nan: keep (quiet nan) */
        if (u & 0x007fffffu) u |= 0x00400000u;
        u &= 0xffff0000u;
    } else {
        uint32_t lsb = (u >> 16) & 1u;
        u += 0x7fffu + lsb;
        u &= 0xffff0000u;
    }
    float r;
    memcpy(&r, &u, 4);
    return r;
}

OM_API float om_bf16(float x) { return bf16_rne(x); }

static double q(double v, int round_mode) { return round_mode ? (double)bf16_rne((float)v) : v; }

/* Forward pass of one observation; optional activations out. */
static double forward1(const float* P, const double* phi, int rm, double* h1p, double* h1q, double* h2p, double* h2) {
    for (int o = 0; o < NH; ++o) {
        double a = P[OFF_B1 + o];
        for (int i = 0; i < NI; ++i) a += q(P[OFF_W1 + o * NI + i], rm) * q(phi[i], rm);
        h1p[o] = a;
        h1q[o] = q(a > 0.0 ? a : 0.0, rm);
    }
    double zz = P[OFF_B3];
    for (int o = 0; o < NH; ++o) {
        double a = P[OFF_B2 + o];
        for (int i = 0; i < NH; ++i) a += q(P[OFF_W2 + o * NH + i], rm) * h1q[i];
        h2p[o] = a;
        h2[o] = a > 0.0 ? a : 0.0;
        zz += q(P[OFF_W3 + o], rm) * h2[o];
    }
    return zz;
}

/* Weights w = sigmoid(logit) for N observations (phi: [N][8] binary32). */
OM_API void om_forward(const float* params, const float* phi, int64_t N, int32_t round_mode, double* out) {
    double h1p[NH], h1q[NH], h2p[NH], h2[NH], x[NI];
    for (int64_t n = 0; n < N; ++n) {
        for (int i = 0; i < NI; ++i) x[i] = phi[n * NI + i];
        double zz = forward1(params, x, round_mode, h1p, h1q, h2p, h2);
        out[n] = 1.0 / (1.0 + exp(-zz));
    }
}

/* Mean binary cross-entropy over the batch and its gradient with respect to
 * every parameter (binary64).  With rounding on, the rounding steps are
 * treated as identity in the backward pass (straight-through), as the
 * training kernels do. */
OM_API double om_loss_grad(const float* params, const float* phi, const float* target, int64_t N, int32_t round_mode,
                           double* grad) {
    double h1p[NH], h1q[NH], h2p[NH], h2[NH], x[NI], d2[NH], d1[NH];
    memset(grad, 0, sizeof(double) * NPARAM);
    double loss = 0.0;
    for (int64_t n = 0; n < N; ++n) {
        for (int i = 0; i < NI; ++i) x[i] = phi[n * NI + i];
        double zz = forward1(params, x, round_mode, h1p, h1q, h2p, h2);
        double y = target[n];
        /* BCE with logits: log(1 + e^z) - y z, stable form */
        loss += (zz > 0 ? zz + log1p(exp(-zz)) : log1p(exp(zz))) - y * zz;
        double s = 1.0 / (1.0 + exp(-zz));
        double dz = (s - y) / (double)N;
        grad[OFF_B3] += dz;
        for (int o = 0; o < NH; ++o) {
            grad[OFF_W3 + o] += dz * h2[o];
            d2[o] = h2p[o] > 0.0 ? dz * q(params[OFF_W3 + o], round_mode) : 0.0;
        }
        for (int o = 0; o < NH; ++o) {
            grad[OFF_B2 + o] += d2[o];
            for (int i = 0; i < NH; ++i) grad[OFF_W2 + o * NH + i] += d2[o] * h1q[i];
        }
        for (int i = 0; i < NH; ++i) {
            double a = 0.0;
            for (int o = 0; o < NH; ++o) a += d2[o] * q(params[OFF_W2 + o * NH + i], round_mode);
            d1[i] = h1p[i] > 0.0 ? a : 0.0;
        }
        for (int o = 0; o < NH; ++o) {
            grad[OFF_B1 + o] += d1[o];
            for (int i = 0; i < NI; ++i) grad[OFF_W1 + o * NI + i] += d1[o] * q(x[i], round_mode);
        }
    }
    return loss / (double)N;
}

/* One Adam step (Kingma & Ba 2015) in binary64 on binary32 parameters. */
OM_API void om_adam(float* params, double* m, double* v, const double* grad, int64_t n, double lr, double b1, double b2,
                    double eps, int32_t t) {
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * grad[i];
        v[i] = b2 * v[i] + (1.0 - b2) * grad[i] * grad[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        params[i] = (float)((double)params[i] - lr * mh / (sqrt(vh) + eps));
    }
}

/* Features of one observation (see the header). */
OM_API void om_features(double rx, double ry, const double* nrm, double z, double u, double v, const double* p,
                        int32_t c, int32_t n_same, double x_px, double y_px, double cx, double cy, double* phi) {
    double rn = rx * nrm[0] + ry * nrm[1] + nrm[2];
    double lr = sqrt(rx * rx + ry * ry + 1.0);
    double ln = sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
    phi[0] = ln > 0 ? fabs(rn) / (lr * ln) : 0.0;
    phi[1] = z / (1.0 + z);
    double h = 0.0, p1 = -INFINITY, p2 = -INFINITY;
    for (int j = 0; j < c; ++j) {
        if (p[j] > 0.0) h -= p[j] * log(p[j]);
        if (p[j] > p1) { p2 = p1; p1 = p[j]; }
        else if (p[j] > p2) p2 = p[j];
    }
    if (c < 2) p2 = 0.0;
    phi[2] = c > 1 ? h / log((double)c) : 0.0;
    phi[3] = p1;
    phi[4] = p1 - p2;
    double b = u;
    if (v < b) b = v;
    if (1.0 - u - v < b) b = 1.0 - u - v;
    b *= 3.0;
    phi[5] = b < 0 ? 0.0 : (b > 1 ? 1.0 : b);
    double lc = log((double)(n_same > 0 ? n_same : 1)) / log(64.0);
    phi[6] = lc > 2.0 ? 2.0 : lc;
    double dx = x_px + 0.5 - cx, dy = y_px + 0.5 - cy;
    phi[7] = sqrt(dx * dx + dy * dy) / sqrt(cx * cx + cy * cy);
}

/* Features and training targets of every valid covered pixel of one frame.
 * The renderer is the oracle's own (tri, uv, z per pixel); the normal and
 * ray are recomputed in binary64 from the camera-space triangle.  probs is
 * float32 [c][H][W] of this frame with element strides (sc, sy, sx); labels
 * are the texel labels of the plain fusion (NULL: targets not written).
 * Returns the number of observations written (pixel order), or -1. */
int32_t or_raster_frame(const float* verts, int64_t n_faces, const int32_t* faces_uv, const int32_t* s_face,
                        const int64_t* off, int32_t scheme, const float* cam16, float z_near, int32_t H, int32_t W,
                        int32_t* tri_out, int32_t* l_out, float* z_out, float* uv_out);

OM_API int64_t om_frame_features(const float* verts, int64_t n_faces, const int32_t* faces_uv, const int32_t* s_face,
                                 const int64_t* off, int32_t scheme, int64_t n_texels, const float* cam16, float z_near,
                                 int32_t H, int32_t W, const float* probs, int64_t sc, int64_t sy, int64_t sx,
                                 int32_t c, const uint8_t* valid, const uint8_t* labels, float* phi_out,
                                 float* target_out, int32_t* pix_out) {
    int64_t npx = (int64_t)H * W;
    int32_t* tri = (int32_t*)malloc(sizeof(int32_t) * npx);
    int32_t* l = (int32_t*)malloc(sizeof(int32_t) * npx);
    float* z = (float*)malloc(sizeof(float) * npx);
    float* uv = (float*)malloc(sizeof(float) * 2 * npx);
    int32_t* cnt = (int32_t*)calloc((size_t)n_texels, sizeof(int32_t));
    double* p = (double*)malloc(sizeof(double) * c);
    if (!tri || !l || !z || !uv || !cnt || !p) return -1;
    or_raster_frame(verts, n_faces, faces_uv, s_face, off, scheme, cam16, z_near, H, W, tri, l, z, uv);
    for (int64_t i = 0; i < npx; ++i)
        if (l[i] >= 0 && (!valid || valid[i])) cnt[l[i]] += 1;
    const double fx = cam16[0], fy = cam16[1], cx = cam16[2], cy = cam16[3];
    double R[9], t[3];
    for (int k = 0; k < 9; ++k) R[k] = cam16[4 + k];
    for (int k = 0; k < 3; ++k) t[k] = cam16[13 + k];
    int64_t n = 0;
    for (int32_t y = 0; y < H; ++y) {
        for (int32_t x = 0; x < W; ++x) {
            int64_t i = (int64_t)y * W + x;
            if (l[i] < 0 || (valid && !valid[i])) continue;
            const int32_t* f = faces_uv + 3 * (int64_t)tri[i];
            double P[3][3];
            for (int m = 0; m < 3; ++m) {
                const float* X = verts + 3 * (int64_t)f[m];
                for (int r = 0; r < 3; ++r) P[m][r] = R[3 * r] * X[0] + R[3 * r + 1] * X[1] + R[3 * r + 2] * X[2] + t[r];
            }
            double e1[3], e2[3], nrm[3];
            for (int r = 0; r < 3; ++r) { e1[r] = P[2][r] - P[0][r]; e2[r] = P[1][r] - P[0][r]; }
            nrm[0] = e1[1] * e2[2] - e1[2] * e2[1];
            nrm[1] = e1[2] * e2[0] - e1[0] * e2[2];
            nrm[2] = e1[0] * e2[1] - e1[1] * e2[0];
            for (int j = 0; j < c; ++j) p[j] = probs[j * sc + y * sy + x * sx];
            double rx = (x + 0.5 - cx) / fx, ry = (y + 0.5 - cy) / fy;
            double ph[NI];
            om_features(rx, ry, nrm, z[i], uv[2 * i], uv[2 * i + 1], p, c, cnt[l[i]], x, y, cx, cy, ph);
            for (int k = 0; k < NI; ++k) phi_out[n * NI + k] = (float)ph[k];
            if (target_out) {
                int best = 0;
                for (int j = 1; j < c; ++j) if (p[j] > p[best]) best = j;
                target_out[n] = (labels[l[i]] != 255 && labels[l[i]] == best) ? 1.0f : 0.0f;
            }
            if (pix_out) pix_out[n] = (int32_t)i;
            ++n;
        }
    }
    free(tri); free(l); free(z); free(uv); free(cnt); free(p);
    return n;
}
