/*
 * semfuse: label fusion in semantically textured meshes on AMD Instinct MI355X (gfx950).
 *
 * The method (Fervers et al., "Improving Semantic Image Segmentation via Label
 * Fusion in Semantically Textured Meshes"): a known triangle mesh is rendered
 * with every frame's camera into per-pixel triangle and texel identifiers
 * (Section 3.3.1); each pixel's c-class probability vector is aggregated into
 * the row of a texel-major array P (Section 3.3.2, eq. texel-in-array) with
 * the weighted aggregators of Section 3.2 (eqs. w-sum, w-mul, w-maxsum and
 * the weights w^(P), w^(I)); every row is normalised and its argmax is the
 * texel's class (Section 3.2.1); the fused labels are rendered back into every
 * frame.
 *
 * Conventions shared by every call
 *  - All pointers named d_* are device pointers (hipMalloc / torch CUDA
 *    tensors) owned by the caller; the library allocates no device memory
 *    (its one static array, the scratch of lf_fuse_frames_noalloc, is part of
 *    the loaded code object) and keeps no pointer beyond what the mesh handle
 *    documents.  h_* pointers are host memory.
 *  - Calls enqueue work on `stream` and return without waiting, except
 *    lf_load_mesh, which waits for its validation result.  Inputs must stay
 *    unmodified until the stream has consumed them.
 *  - A handle is not thread-safe; two handles are independent.
 *  - Every call returns an lf_status; on failure lf_last_error() (thread-local)
 *    describes it.  No C++ exception crosses this interface.
 *  - Camera record (16 floats): fx, fy, cx, cy, R[9] (row-major, world to
 *    camera), t[3]; X_cam = R X_world + t; pinhole, no distortion, x right,
 *    y down, z forward; pixel (x, y) has its centre at (x + 1/2, y + 1/2).
 *  - Probability input: a 4-D array indexed [frame][class][y][x] with
 *    arbitrary element strides (NCHW, or channels-last NHWC memory).  float32,
 *    or OCP E4M3FN codes (uint8) with a float32 per-pixel scale
 *    [frame][y][x]: p = decode(q) * scale.  Probabilities are used as given
 *    (not renormalised); NaN propagates into the texels it reaches.
 *  - Limits: 1 <= c <= 255 (labels are uint8, 255 = void); n_texels < 2^31;
 *    H, W <= 8192; triangle count < 2^31.
 */
#ifndef SEMFUSE_H
#define SEMFUSE_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LF_OK = 0,
    LF_EINVAL = -1,   /* bad argument, shape or option                         */
    LF_ESIZE = -2,    /* caller buffer / workspace smaller than required       */
    LF_EHIP = -3,     /* HIP runtime error (launch failure, ...)               */
    LF_ESTATE = -4    /* handle freed or used with mismatching options         */
} lf_status;

typedef enum { LF_TEX_SQUARE = 0, LF_TEX_SPLIT = 1 } lf_texel_scheme;
typedef enum { LF_W_PIXEL = 0, LF_W_IMAGE = 1, LF_W_LEARNED = 2, LF_W_MIX = 3 } lf_weighting;
typedef enum { LF_AGG_SUM = 0, LF_AGG_MUL = 1, LF_AGG_MAXSUM = 2 } lf_aggregator;
typedef enum { LF_F32 = 0, LF_BF16 = 1, LF_F16 = 2, LF_FP8_E4M3 = 3 } lf_dtype;
typedef enum {
    LF_SCATTER_AUTO = 0,     /* SORTED when a pixel's classes are contiguous, else STAGED when allowed, else ATOMIC */
    LF_SCATTER_ATOMIC = 1,   /* LDS-hash pre-reduction, then FP32 atomics (any strides, any dtype) */
    LF_SCATTER_SORTED = 2,   /* texel-sorted gather reading each pixel's classes in place */
    LF_SCATTER_STAGED = 3    /* frames first transposed to pixel-major rows in the frame workspace, then
                                the texel-sorted gather (planar inputs; FP32, c % 4 == 0, c <= 60) */
} lf_scatter_mode;

typedef struct lf_mesh_s* lf_mesh;

/* Mesh options.
 *  scheme     texel layout of a triangle with s steps per uv dimension
 *             (Section 3.1): SQUARE = the paper's (s^2+s)/2 cells; SPLIT cuts
 *             every full square cell along its anti-diagonal (s^2 texels).
 *  s_uniform  s for every triangle when no per-face array is given (>= 1).
 *  n_classes  c.
 *  aggregator f of Section 3.2.1 (eq. sum / mul / maxsum, weighted forms of 3.2.2).
 *  accum_dtype LF_F32 (default) or LF_BF16 / LF_F16 to keep the accumulator
 *             itself in 16 bits (measures accumulation stagnation; SUM only).
 *  z_near     near clipping plane in camera units (> 0). */
typedef struct {
    int32_t scheme;
    int32_t s_uniform;
    int32_t n_classes;
    int32_t aggregator;
    int32_t accum_dtype;
    float z_near;
} lf_mesh_opts;

/* Sizes of the caller-owned buffers of a mesh (Section 3.3.2: n_x = sum of
 * |X_t|).  h_s_face: optional per-face s (host, [n_faces]).  Outputs:
 * *n_texels; *mesh_ws_bytes = workspace lf_load_mesh needs and the handle
 * keeps using.  Errors: LF_EINVAL on bad options or counts. */
lf_status lf_mesh_sizes(const lf_mesh_opts* opts, int64_t n_vertices, int64_t n_faces,
                        const int32_t* h_s_face, int64_t* n_texels, int64_t* mesh_ws_bytes);

/* Load a mesh (Section 3.1 / 3.3.2): picks every triangle's uv origin (the
 * vertex whose interior angle is closest to 90 degrees), its texel count and
 * its row offset id_t, builds culling bounds, and clears the accumulator.
 *  d_vertices [V][3] float32 world coordinates; d_faces [T][3] int32 vertex
 *  indices; d_s_face [T] int32 or NULL (then opts->s_uniform);
 *  d_mesh_ws  >= mesh_ws_bytes, 256-byte aligned, kept by the handle;
 *  d_accum    [n_texels][c] accumulator (FP32 unless opts->accum_dtype), kept;
 *             or NULL for a texture fused window by window only (the mesh
 *             then starts with an empty window: see lf_set_window);
 *  d_wsum     [n_texels] float32 total weight per texel, kept (may be NULL
 *             unless aggregator == MUL and d_accum is given).
 * Waits on `stream` for index validation: LF_EINVAL if a face index is out of
 * range or an s is < 1.  The triangles' vertex positions are copied into the
 * mesh workspace here: later changes to d_vertices are not seen.  The caller
 * keeps vertices, workspace and accumulator alive until lf_free_mesh. */
lf_status lf_load_mesh(const lf_mesh_opts* opts, const float* d_vertices, int64_t n_vertices,
                       const int32_t* d_faces, int64_t n_faces, const int32_t* d_s_face,
                       void* d_mesh_ws, int64_t mesh_ws_bytes, void* d_accum, float* d_wsum,
                       int64_t n_texels, hipStream_t stream, lf_mesh* out);

/* alpha of LF_W_MIX for this mesh (0 = w^(P), 1 = w^(I)); LF_EINVAL outside [0, 1]. */
lf_status lf_set_weight_mix(lf_mesh mesh, float alpha);

/* Texel-row window: out-of-core aggregation for textures larger than a device
 * budget (Section 3.3.2 runs the aggregator on the GPU or, for larger meshes
 * and texel resolutions, on the CPU; here the texture is fused on the GPU a
 * window of rows at a time and the caller moves each window's result where
 * it keeps the texture, e.g. host memory).  After this call the mesh
 * accumulates only texel rows row_lo .. row_lo + n_rows - 1, row r at row
 * r - row_lo of d_accum [n_rows][c] (and d_wsum [n_rows], required for MUL);
 * pixels on other rows are skipped by lf_fuse_frames and lf_fuse_batch;
 * lf_reset clears the window; lf_finalize writes the
 * window's rows (texture [n_rows][c], labels [n_rows], window-relative).
 * The renderer and lf_render_labels keep using whole-texture rows (label
 * images read labels [n_texels]).  Per-row workspace (lf_frame_ws_bytes)
 * shrinks with the window.  The learned weighting and lf_extract_features
 * need the whole texture (LF_ESTATE with a window).  d_accum = NULL with
 * row_lo = 0, n_rows = n_texels, d_wsum = NULL restores the load-time
 * buffers.  The buffers stay the caller's; nothing is cleared here.
 * Errors: LF_EINVAL for a window outside [0, n_texels) or a misaligned
 * buffer. */
lf_status lf_set_window(lf_mesh mesh, int64_t row_lo, int64_t n_rows, void* d_accum, float* d_wsum);

/* Clear the accumulator (and weight sums): start a new fusion. */
lf_status lf_reset(lf_mesh mesh, hipStream_t stream);

/* Workspace bytes lf_fuse_frames / lf_rasterize / lf_render_labels need for
 * frames of H x W processed `batch` at a time (batch >= 1). */
lf_status lf_frame_ws_bytes(lf_mesh mesh, int32_t H, int32_t W, int32_t batch, int32_t weighting,
                            int32_t scatter_mode, int64_t* bytes);

/* Exact workspace bytes of an lf_fuse_frames call with this input dtype and
 * these strides (AUTO resolved as the call resolves it). */
lf_status lf_fuse_ws_bytes(lf_mesh mesh, int32_t H, int32_t W, int32_t batch, int32_t weighting,
                           int32_t scatter_mode, int32_t prob_dtype, const int64_t* h_strides, int64_t* bytes);

/* Fuse F frames into the accumulator (Sections 3.3.1, 3.3.2, 3.2):
 * render every frame to triangle / texel ids, then add w_k * p_k (SUM),
 * w_k * log p_k (MUL) or w_k * g(p_k) (MAXSUM) into row l_k of every valid
 * covered pixel.
 *  d_cams   [F][16] float32 camera records (device);
 *  d_probs  probability input, element strides[4] = (frame, class, y, x);
 *  prob_dtype LF_F32 or LF_FP8_E4M3 (then d_scale [F][H][W] float32);
 *  d_valid  [F][H][W] uint8 (0 = pixel without depth, skipped) or NULL;
 *  weighting LF_W_PIXEL (w = 1), LF_W_IMAGE (w = 1/|K_i ∩ K_x|),
 *           LF_W_LEARNED (w = the bound MLP's output, see lf_mlp_bind) or
 *           LF_W_MIX (w = (1 - alpha) + alpha/|K_i ∩ K_x|, the weights
 *           between w^(P) and w^(I) of the evaluation, Fig. 4a; alpha from
 *           lf_set_weight_mix, default 1/2);
 *  d_l_out  [F][H][W] int32 texel rows (-1 = no triangle) or NULL;
 *  d_ws     workspace of lf_frame_ws_bytes(H, W, batch) bytes, 256-aligned;
 *  scatter_mode  LF_SCATTER_AUTO / ATOMIC / SORTED / STAGED (same result up
 *           to FP32 summation order).
 * Frames may be fused in several calls (fusion is incremental).  Errors:
 * LF_EINVAL (shapes, dtype, strides), LF_ESIZE (workspace), LF_EHIP. */
lf_status lf_fuse_frames(lf_mesh mesh, const float* d_cams, int32_t F, int32_t H, int32_t W,
                         const void* d_probs, int32_t prob_dtype, const int64_t* h_strides,
                         const float* d_scale, const uint8_t* d_valid, int32_t weighting,
                         int32_t* d_l_out, void* d_ws, int64_t ws_bytes, int32_t batch,
                         int32_t scatter_mode, hipStream_t stream);

/* lf_fuse_frames for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same fusion, arguments and results, with the frame workspace taken from
 * a fixed array of LF_NOALLOC_SCRATCH_BYTES that the library holds on every
 * GPU it runs on until the process ends.  The call allocates nothing; the
 * caller still passes the mesh (with its workspace and accumulator), inputs
 * and outputs.  The scratch belongs to the current device (hipSetDevice),
 * which must be the device of the mesh and the stream.  Every call on one GPU
 * shares that GPU's scratch: calls whose work overlaps on the device (two
 * host threads, or two streams not ordered by events) race and give wrong
 * results; calls ordered on one stream do not.  Whatever must start at zero
 * is cleared by the call itself.  Errors: as lf_fuse_frames; LF_ESIZE with
 * the bytes needed when the call's frame workspace (lf_fuse_ws_bytes for the
 * same arguments) exceeds the scratch. */
#define LF_NOALLOC_SCRATCH_BYTES (64ll << 20)
lf_status lf_fuse_frames_noalloc(lf_mesh mesh, const float* d_cams, int32_t F, int32_t H, int32_t W,
                                 const void* d_probs, int32_t prob_dtype, const int64_t* h_strides,
                                 const float* d_scale, const uint8_t* d_valid, int32_t weighting, int32_t* d_l_out,
                                 int32_t batch, int32_t scatter_mode, hipStream_t stream);

/* Normalise every texel and take its class (Section 3.2.1): SUM/MAXSUM
 * P = A / sum_j A_j, MUL P = softmax(A); label = first maximal index; a texel
 * never observed gets P = 0 and label 255.
 *  d_tex_out [n_texels][c] in tex_dtype (LF_F32, LF_BF16 or LF_F16, round to
 *            nearest even) or NULL;  d_labels [n_texels] uint8 (required). */
lf_status lf_finalize(lf_mesh mesh, void* d_tex_out, int32_t tex_dtype, uint8_t* d_labels,
                      hipStream_t stream);

/* Render the fused labels back into F frames (Section 3.2.1): out = label of
 * the pixel's texel, 255 where no triangle is hit or the pixel is invalid.
 *  d_l [F][H][W] rows from lf_fuse_frames, or NULL to re-render with d_cams;
 *  d_labels [n_texels] from lf_finalize; d_out [F][H][W] uint8. */
lf_status lf_render_labels(lf_mesh mesh, const float* d_cams, int32_t F, int32_t H, int32_t W,
                           const int32_t* d_l, const uint8_t* d_valid, const uint8_t* d_labels,
                           uint8_t* d_out, void* d_ws, int64_t ws_bytes, hipStream_t stream);

/* Renderer alone (Section 3.3.1): per pixel triangle id (-1 none), texel row
 * l (-1), depth z (NaN where none).  Any output may be NULL. */
lf_status lf_rasterize(lf_mesh mesh, const float* d_cams, int32_t F, int32_t H, int32_t W,
                       int32_t* d_tri, int32_t* d_l, float* d_z, void* d_ws, int64_t ws_bytes,
                       hipStream_t stream);

/* ---- Tuning ------------------------------------------------------------------
 * Launch parameters of a mesh's kernels that do not change results: the
 * raster tile edge (16 or 32 pixels; default 32), the number of
 * observations each row keeps in flight in the texel-sorted gather (4 or 8;
 * default 8) and the largest pixel-box area a triangle may have to be
 * rasterized by a single lane rather than a whole wave (1..1024; default
 * 48), and the resident waves per compute unit the gather's grid is sized
 * for (1..1024; default 8: fewer leave room for the next batch's raster,
 * which runs concurrently on a second stream; more than fit at once, e.g.
 * 512, balance rows of uneven length when the gather has the device alone),
 * and where LF_W_LEARNED evaluates the network (0, default: in a separate
 * pass over the batch's pixels first; 1: inside the texel-sorted gather
 * where it can).
 * Frame batch size and scatter mode are per-call arguments.
 * lf_frame_ws_bytes depends on the tile: query it after lf_set_tuning. */
typedef struct {
    int32_t tile;
    int32_t gather_unroll;
    int32_t small_px;
    int32_t gather_waves;
    int32_t learned_in_gather;
} lf_tuning;
lf_status lf_set_tuning(lf_mesh mesh, const lf_tuning* tuning);
lf_status lf_get_tuning(lf_mesh mesh, lf_tuning* tuning);

/* Whether the texel-sorted scatter overlaps batches (default 1): each
 * batch's gather runs on the mesh's second stream while the caller's stream
 * renders and sorts the next batch.  0 runs the gathers on the caller's
 * stream, one batch after another, so that a gather has the whole device
 * (used to time the gather kernel alone).  Results do not depend on it.
 * Errors: LF_ESTATE for an invalid mesh handle. */
lf_status lf_set_overlap(lf_mesh mesh, int32_t enabled);

/* ---- Many scenes in one call, and as one captured graph ---------------------
 * One job = one complete fusion of a scene (Sections 3.2 and 3.3): clear its
 * accumulator, fuse its F frames (as lf_fuse_frames), normalise every texel
 * (as lf_finalize) and optionally render the labels back (as
 * lf_render_labels from the stored rows).
 *  pool      0: frame f reads input frame f; > 0: frame f reads input frame
 *            f % pool of d_probs / d_scale / d_valid (a cycled input pool;
 *            cameras, rows and images stay per frame);
 *  d_l_out   [F][H][W] rows or NULL (required when d_images is set);
 *  d_tex_out [n_texels][c] in tex_dtype or NULL;  d_labels [n_texels]
 *            (required);  d_images [F][H][W] uint8 or NULL.
 * The jobs run on up to four scene lanes at once: streams of the library
 * (one set per device) forked from `stream` and joined back into it with
 * events, so that small scenes' kernels fill the compute units a large
 * scene's latency-bound kernels leave idle.  Jobs on one mesh run in one
 * lane, in call order; meshes are dealt to lanes largest first (frames x
 * pixels).  Each lane has its own slice of the workspace:
 * lf_batch_ws_bytes = lanes x the largest frame workspace a job needs.
 * Batched calls on one device enqueue one at a time (a library lock); their
 * work is ordered on the lane streams. */
typedef struct {
    lf_mesh mesh;
    const float* d_cams;
    int32_t F, H, W;
    const void* d_probs;
    int32_t prob_dtype;
    int64_t strides[4];
    const float* d_scale;
    const uint8_t* d_valid;
    int32_t pool;
    int32_t weighting;
    int32_t batch;
    int32_t scatter_mode;
    int32_t* d_l_out;
    void* d_tex_out;
    int32_t tex_dtype;
    uint8_t* d_labels;
    uint8_t* d_images;
} lf_scene_job;

lf_status lf_batch_ws_bytes(const lf_scene_job* jobs, int32_t n_jobs, int64_t* bytes);

/* Run the jobs.  Every job is checked before anything is enqueued. */
lf_status lf_fuse_batch(const lf_scene_job* jobs, int32_t n_jobs, void* d_ws, int64_t ws_bytes,
                        hipStream_t stream);

/* Capture the jobs' whole launch sequence into executable HIP graphs, one per
 * scene lane (on one lane, captured on `stream`, which must not be the
 * legacy default stream); lf_graph_launch replays them on any stream,
 * forking it into the lanes and joining them back.  The sequence holds kernels only (buffers are cleared by
 * kernels, no host synchronisation, no allocation), so replays are
 * independent.  Every buffer the jobs name is baked into the graph: keep them
 * alive and in place while the graph exists; new input values in those
 * buffers are picked up by the next replay.  Profiling must be off. */
typedef struct lf_graph_s* lf_graph;
lf_status lf_graph_capture_batch(const lf_scene_job* jobs, int32_t n_jobs, void* d_ws, int64_t ws_bytes,
                                 hipStream_t stream, lf_graph* out);
lf_status lf_graph_launch(lf_graph graph, hipStream_t stream);
void lf_graph_free(lf_graph graph);

/* ---- Learned per-observation weight ---------------------------------------
 * Section 3.2.2 weights every observation k of a texel by w_k, with the two
 * fixed choices w^(P) = 1 and w^(I) = 1/|K_i ∩ K_x|.  LF_W_LEARNED takes w_k
 * from a small network on per-observation features phi_k (8 floats):
 *   0 |cos| of the angle between the pixel ray and the triangle normal,
 *   1 z / (1 + z) of the depth z,  2 normalised entropy -sum p ln p / ln c,
 *   3 top-1 probability,  4 top-1 minus top-2,
 *   5 min(1, 3 min(u, v, 1-u-v)) (closeness to the triangle's centroid),
 *   6 min(2, ln n / ln 64), n = the frame's pixels on the same texel,
 *   7 |(x + 1/2 - cx, y + 1/2 - cy)| / |(cx, cy)| (radial image distance).
 * Network: h1 = relu(W1 q(phi) + b1), h2 = relu(W2 q(h1) + b2),
 * w = sigmoid(w3 . h2 + b3); W1 64x8, W2 64x64, w3 64; q = round to bfloat16.
 * Master parameters are binary32 in the order W1 (row-major [64][8]), b1,
 * W2 ([64][64]), b2, w3, b3 (n_params floats); the packed form holds W1, W2,
 * w3 in bfloat16 and the biases in binary32 (packed_bytes, 16-byte aligned).
 * Training target: y_k = 1 when the observation's own argmax equals the
 * label plain fusion gives its texel; loss = mean binary cross-entropy.
 * Where the network runs (lf_tuning.learned_in_gather): a separate pass
 * writes per-pixel weights first, from a per-frame count array; or, on the
 * texel-sorted path with contiguous classes (c % 4 == 0, c <= 64,
 * channels-last or staged planar input) and batches of at most 128 frames,
 * the gather evaluates the network for every observation of a texel bucket
 * just before summing them (n from its own per-frame counters).  Both give
 * the same weights. */

/* Number of master parameters and bytes of the packed form. */
lf_status lf_mlp_sizes(int32_t* n_params, int64_t* packed_bytes);

/* Pack binary32 master parameters d_params [n_params] into d_packed
 * (bfloat16 weights, round to nearest even). */
lf_status lf_mlp_pack(const float* d_params, void* d_packed, hipStream_t stream);

/* Bind packed weights to a mesh for LF_W_LEARNED fusion (NULL unbinds).  The
 * handle keeps the pointer: the caller keeps the buffer alive and may repack
 * into it between calls. */
lf_status lf_mlp_bind(lf_mesh mesh, const void* d_packed);

/* w [n] = network output for features d_phi [n][8] (float32). */
lf_status lf_mlp_forward(const void* d_packed, const float* d_phi, int64_t n, float* d_w,
                         hipStream_t stream);

/* Mean binary cross-entropy of the network on (d_phi [n][8], d_target [n]
 * in {0, 1}) and its gradient with respect to every master parameter, in the
 * master order, written to d_grad [n_params] (overwritten) and *d_loss
 * (float, may be NULL).  The rounding q is passed straight through in the
 * backward pass; products use the bfloat16 weights of d_packed. */
lf_status lf_mlp_grad(const void* d_packed, const float* d_phi, const float* d_target, int64_t n,
                      float* d_grad, float* d_loss, hipStream_t stream);

/* One Adam step (Kingma & Ba) on n binary32 parameters with moments d_m,
 * d_v (caller-owned, zero before step 1): step counts from 1. */
lf_status lf_adam_step(float* d_params, float* d_m, float* d_v, const float* d_grad, int64_t n,
                       float lr, float beta1, float beta2, float eps, int32_t step, hipStream_t stream);

/* Features of every valid covered pixel of F frames (arguments as in
 * lf_fuse_frames), appended in unspecified order:
 *  d_phi [cap][8] features; d_target [cap] training targets against the
 *  fused labels d_labels [n_texels] (both may be NULL together); d_pix [cap]
 *  int32 pixel index f*H*W + y*W + x (or NULL; needs F*H*W < 2^31);
 *  *d_count (uint64, device) = number of observations found, which may
 *  exceed cap: only the first cap are written.
 *  d_ws: workspace of lf_frame_ws_bytes(H, W, batch, LF_W_LEARNED,
 *  LF_SCATTER_ATOMIC) for some batch >= 1. */
lf_status lf_extract_features(lf_mesh mesh, const float* d_cams, int32_t F, int32_t H, int32_t W,
                              const void* d_probs, int32_t prob_dtype, const int64_t* h_strides,
                              const float* d_scale, const uint8_t* d_valid, const uint8_t* d_labels,
                              float* d_phi, float* d_target, int32_t* d_pix, int64_t cap,
                              uint64_t* d_count, void* d_ws, int64_t ws_bytes, hipStream_t stream);

/* Agreement of label images with the frames' own labels, the statistic by
 * which plain fusion judges the learned weight on held-out frames (the
 * training target's notion of label error, Section 3.2.1: a pixel's label is
 * the argmax of its distribution, first maximal class on ties):
 * d_counts[0] += pixels of d_images [F][H][W] with a label (not 255) that are
 * valid; d_counts[1] += those whose label equals the argmax of the pixel's
 * own input distribution (probabilities as in lf_fuse_frames).  d_counts is
 * two uint64 on the device, accumulated into (zero them to start). */
lf_status lf_label_agreement(const void* d_probs, int32_t prob_dtype, const int64_t* h_strides, const float* d_scale,
                             const uint8_t* d_valid, int32_t n_classes, int32_t F, int32_t H, int32_t W,
                             const uint8_t* d_images, uint64_t* d_counts, hipStream_t stream);

/* ---- Texel resolution from the worst-case frame (Section 3.1) -------------
 * a_t = the largest number of pixel centres triangle t covers (as the
 * z-buffer's winner) in any frame; s_t = max(1, ceil(gamma * sqrt(a_t))).
 * A mesh loaded with d_s_face = s_t (and the paper's SQUARE scheme) has the
 * paper's texture resolution for that gamma.  Pixels count whether or not
 * they are valid. */

/* Workspace bytes of lf_triangle_max_pixels for frames of H x W, `batch` at a time. */
lf_status lf_area_ws_bytes(lf_mesh mesh, int32_t H, int32_t W, int32_t batch, int64_t* bytes);

/* Raise d_area [T] (int32, caller-owned; zero it to start) to every frame's
 * pixel count of each triangle, over F frames (cameras as in
 * lf_fuse_frames).  Several calls accumulate the maximum. */
lf_status lf_triangle_max_pixels(lf_mesh mesh, const float* d_cams, int32_t F, int32_t H, int32_t W,
                                 int32_t* d_area, void* d_ws, int64_t ws_bytes, hipStream_t stream);

/* d_s_face [n_faces] = max(1, ceil(gamma * sqrt(d_area))) in binary32
 * (correctly rounded square root), capped at 4096. */
lf_status lf_texel_resolution(const int32_t* d_area, int64_t n_faces, float gamma, int32_t* d_s_face,
                              hipStream_t stream);

/* Per-stage kernel timing with HIP events recorded on the launch stream
 * around every kernel of a stage (instrumentation for roofline reports).
 * Stages: 0 ray tables + raster, 1 resolve, 2 scatter, 3 counts, 4 finalize,
 * 5 render, 6 accumulator reset, 7 learned-weight inference / feature extraction.
 * lf_profile_enable(mesh, 1) starts recording (clearing earlier records);
 * lf_profile_read waits for the recorded events and returns, per stage, the
 * summed milliseconds and the number of timed launches. */
#define LF_N_STAGES 8
typedef struct {
    double ms[LF_N_STAGES];
    int64_t launches[LF_N_STAGES];
} lf_profile;
lf_status lf_profile_enable(lf_mesh mesh, int32_t on);
lf_status lf_profile_read(lf_mesh mesh, lf_profile* out);

/* Release a handle (no device memory is freed: the caller owns it all). */
void lf_free_mesh(lf_mesh mesh);

/* Thread-local description of the last failure ("" if none). */
const char* lf_last_error(void);

/* Library version string. */
const char* lf_version(void);

#ifdef __cplusplus
}
#endif
#endif
