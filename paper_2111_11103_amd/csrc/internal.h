// Internal host/device interfaces of the semfuse library (not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lf {

constexpr int kClusterTris = 64;      // triangles per culling cluster (one wave)

// Device view of a loaded mesh.  Every pointer is caller-owned device memory.
struct MeshDev {
  const float* verts;        // [V][3]
  int32_t* faces_uv;         // [T][3] vertex indices in uv order (A, B, C)
  float4* tri_v;             // [T][3] positions of A, B, C in uv order: (A.xyz B.x) (B.yz C.xy) (C.z 0 0 0)
  int32_t* s_face;           // [T] or nullptr (uniform s)
  int64_t* off;              // [T+1] row offsets or nullptr (uniform: t * n_per)
  float* cl_box;             // [n_clusters][8]: lo.xyz, hi.xyz, magnitude bound, pad
  int32_t* err;              // [1] validation flag
  void* accum;               // [n_rows][c]: texel rows win_lo .. win_lo + n_rows - 1
  float* wsum;               // [n_rows] or nullptr
  int64_t V, T, n_texels, n_clusters;
  int64_t win_lo, n_rows;    // the accumulator's texel-row window (0, n_texels unless set)
  int32_t s_uniform, split, c, aggregator, accum_dtype;
  int32_t n_per;             // texels per triangle when uniform
  float z_near;
  int32_t tile;              // raster tile edge: 16 or 32 pixels
  int32_t gather_unroll;     // observations in flight per row in the sorted gather: 4 or 8
  int32_t small_px;          // pixel boxes up to this area are rasterized by one lane
  int32_t gather_waves;      // resident waves per CU the sorted gather's grid is sized for
  float mix;                 // alpha of the mixed weight (1 - alpha) w^(P) + alpha w^(I)
  int32_t learned_in_gather; // the learned weight evaluated inside the sorted gather where it can (1) or never (0)
};

__device__ __forceinline__ int64_t row_offset(const MeshDev& m, int64_t t) {
  return m.off ? m.off[t] : t * (int64_t)m.n_per;
}
__device__ __forceinline__ int tri_s(const MeshDev& m, int64_t t) { return m.s_face ? m.s_face[t] : m.s_uniform; }

constexpr int kTileSize = 32;         // default raster tile edge (pixels)
constexpr int kBucketShift = 4;       // sorted scatter: texel rows per first-level bucket = 2^kBucketShift
constexpr int kTileSlotBits = 9;      // the tile raster's table of buckets seen in the tile: 2^9 slots
constexpr int kTileSlots = 1 << kTileSlotBits;

// Raster workspace of one batch (all caller memory).
struct RasterWs {
  int32_t* vis;              // [B][n_clusters] visible cluster ids
  int32_t* vis_n;            // [B]
  int32_t* tcnt;             // [B][ntiles] tile list lengths (zero between uses)
  int32_t* tlist;            // [B][list_cap]: ntiles lists of list_cap / ntiles triangle ids
  int64_t list_cap;
};

// Per-pixel outputs of the renderer for a batch (batch-relative pointers, any may be null).
struct RasterOut {
  int32_t* l;                // texel rows
  int32_t* tri;              // triangle ids
  float* z;                  // depths
  const uint8_t* valid;      // validity of the batch's pixels
  int32_t* cnt;              // per-frame texel counts [B][cnt_stride] (w^(I))
  int64_t cnt_stride;
  int32_t* seg;              // per-bucket observation counts of the batch (sorted scatter):
                             // bucket = window-relative row >> kBucketShift
  int32_t* rank;             // [B][H][W] rank of the pixel within its bucket's segment
  float4* geo;               // [B][H][W] learned-weight geometry: cos of the viewing angle,
                             // z / (1 + z), centroid closeness, 0 (zeros where no triangle)
  int32_t* tricnt;           // [B][T] pixels covered per triangle (texel-resolution pre-pass)
};

struct ProbIn {
  const void* p;             // probabilities (float32 or E4M3 codes)
  const float* scale;        // per-pixel scale for E4M3 [F][H][W]
  const uint8_t* valid;      // [F][H][W] or nullptr
  int64_t sf, sc, sy, sx;    // element strides
  int32_t dtype;             // 0 = f32, 3 = e4m3
};

// OCP E4M3FN code (sign, 4 exponent bits with bias 7, 3 mantissa bits; 0x7f /
// 0xff are NaN, no infinities) to binary32, exactly, by the gfx950 FP8
// conversion instruction: byte K of a packed word, or a single code.
template <int K>
__device__ __forceinline__ float fp8_e4m3_byte(uint32_t w) {
  return __builtin_amdgcn_cvt_f32_fp8((int)w, K);
}
__device__ __forceinline__ float fp8_e4m3(uint32_t code) { return __builtin_amdgcn_cvt_f32_fp8((int)code, 0); }

// ---- launchers (return hipGetLastError()) ----------------------------------
hipError_t launch_mesh_prep(const MeshDev& m, const int32_t* faces, hipStream_t s);
hipError_t launch_offsets(const MeshDev& m, int32_t* scratch, hipStream_t s);
hipError_t launch_cluster_boxes(const MeshDev& m, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t s);
hipError_t launch_render_batch(const MeshDev& m, const float* cams, int nb, int H, int W, const RasterWs& ws,
                               const RasterOut& out, hipStream_t s);
hipError_t launch_scatter_atomic(const MeshDev& m, const ProbIn& in, int f_first, int nf, int H, int W,
                                 const int32_t* l, int weighting, const int32_t* cnt, int64_t cnt_stride,
                                 const float* wpix, float mix, hipStream_t s);
// Per-frame counts are indexed by window-relative rows l - win_lo (rows
// outside [win_lo, win_lo + cnt_stride) are skipped).
hipError_t launch_clear_counts(const int32_t* l, const uint8_t* valid, int nf, int H, int W, int32_t* cnt,
                               int64_t cnt_stride, int64_t win_lo, hipStream_t s);
hipError_t launch_finalize(const MeshDev& m, void* tex_out, int tex_dtype, uint8_t* labels, hipStream_t s);
// Exclusive scan of n counters into start[0..n] and the list of counters
// that are non-zero (rows[0 .. *nrows)); *nrows must be zero beforehand.
hipError_t launch_seg_scan(const int32_t* seg, int64_t n, int32_t* sums, int32_t* start, int32_t* rows,
                           int32_t* nrows, hipStream_t s);
// Pixels whose row lies outside [win_lo, win_lo + n_rows) are skipped;
// buckets and cnt are indexed by window-relative rows.  Every other valid
// covered pixel writes rec[bstart[bucket] + rank] = (element offset of its
// class-0 value relative to frame f_first, row within the bucket), and its
// weight / E4M3 scale into rec_w / rec_s where those are given.  With
// cnt_zero (the per-frame count array, [nf][cnt_stride], when nothing after
// the fill reads it and the fill's own weights do not) every covered pixel
// in the window also sets its row's count back to zero.
hipError_t launch_seg_fill(const ProbIn& in, int f_first, int nf, int H, int W, const int32_t* l, const int32_t* rank,
                           const int32_t* bstart, uint2* rec, float* rec_w, float* rec_s, int weighting,
                           const int32_t* cnt, int64_t cnt_stride, const float* wpix, float mix, int64_t win_lo,
                           int64_t n_rows, int32_t* cnt_zero, hipStream_t s);
// Second level of the sort through memory (layouts the grouped gather does
// not take): every non-empty bucket's records ordered by row into ent (and
// ent_w / ent_s) within the bucket's range, with one span (window-relative
// row, start, end, 0) per touched row appended to spans; *nspans must be
// zero beforehand.
hipError_t launch_bucket_sort(int64_t n_buckets, const int32_t* bstart, const int32_t* blist, const int32_t* nblist,
                              const uint2* rec, const float* rec_w, const float* rec_s, uint32_t* ent, float* ent_w,
                              float* ent_s, int4* spans, int32_t* nspans, hipStream_t s);
// Frames [f_first, f_first + nf) of planar FP32 input as pixel-major rows of
// c floats: staging[(f - f_first) * H * W + p][j] (c % 4 == 0, c <= 60).
hipError_t launch_planar_rows(const ProbIn& in, int f_first, int nf, int H, int W, int c, float* staging,
                              hipStream_t s);
// Whether the input's classes are contiguous 4-class chunks the grouped
// gather reads (c <= 64, c % 4 == 0, aligned).
bool seg_grouped_ok(const MeshDev& m, const ProbIn& in);
// n / d for every 32-bit unsigned n, with d (>= 1) fixed at launch: the
// round-up multiplier method (Granlund & Montgomery, "Division by invariant
// integers using multiplication", 1994): t = mulhi(m, n),
// q = (t + ((n - t) >> s1)) >> s2.
struct Udiv {
  uint32_t m = 1, s1 = 0, s2 = 0;
  static Udiv make(uint32_t d) {
    Udiv u;
    uint32_t l = 0;
    while (l < 32 && ((uint64_t)1 << l) < d) ++l;   // l = ceil(log2 d)
    u.m = (uint32_t)((((unsigned __int128)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1);
    u.s1 = l < 1 ? l : 1;
    u.s2 = l > 1 ? l - 1 : 0;
    return u;
  }
  __host__ __device__ __forceinline__ uint32_t operator()(uint32_t n) const {
    const uint32_t t = (uint32_t)(((uint64_t)n * m) >> 32);   // v_mul_hi_u32
    return (t + ((n - t) >> s1)) >> s2;
  }
};

// What the grouped gather needs to evaluate the learned weight itself
// (mlp = nullptr: it does not): the packed network, the resolve's per-pixel
// geometry of the batch ([nf][H][W]) and the batch's cameras ([nf][16]).
// The launcher fills in the image size and its dividers.
struct GatherLearn {
  const void* mlp;
  const float4* geo;
  const float* cams;
  uint32_t hw = 0, w = 0;
  Udiv dhw, dw;
};
// Grouped gather from the bucket-ordered records of a batch of nf frames.
// Weights: from rec_w (or 1) when frame_w is 0, wpix is null and learn.mlp
// is null; with frame_w = LF_W_IMAGE or LF_W_MIX the gather counts every
// row's observations per frame itself (only where seg_frame_counts_ok
// holds); with wpix ([nf][H][W] per-pixel weights) it reads them by pixel
// index, as it reads E4M3 scales when rec_s is null (only where
// seg_pixels_dense_ok holds); with learn.mlp it computes every
// observation's learned weight from the observation itself (where both
// hold).
hipError_t launch_bucket_gather(const MeshDev& m, const ProbIn& in, int f_first, int H, int W, int64_t n_buckets,
                                const int32_t* bstart, const int32_t* blist, const int32_t* nblist, const uint2* rec,
                                const float* rec_w, const float* rec_s, int nf, int frame_w, float mix,
                                const float* wpix, const GatherLearn& learn, hipStream_t s);
// Per-class gather over the spans of k_bucket_sort (any strides; weights and
// E4M3 scales per entry).
hipError_t launch_seg_gather(const MeshDev& m, const ProbIn& in, int f_first, const int4* spans,
                             const int32_t* nspans, const uint32_t* ent, const float* ent_w, const float* ent_s,
                             hipStream_t s);
// Whether the gather of input `in` (batches of at most nf frames) can recover
// each observation's frame from its stored element offset and count frames
// itself.
bool seg_frame_counts_ok(const MeshDev& m, const ProbIn& in, int nf, int H, int W);
// Whether the gather of input `in` can recover each observation's pixel
// index from its stored offset, to read E4M3 scales and per-pixel weights by
// it (then the fill stores neither).
bool seg_pixels_dense_ok(const MeshDev& m, const ProbIn& in, int nf, int H, int W);
// Whether the grouped gather can evaluate the learned weight itself for
// input `in` in batches of at most nf frames (frame counts and pixel
// indices recoverable, nf <= 128, its LDS within 64 KB).
bool seg_learned_ok(const MeshDev& m, const ProbIn& in, int nf, int H, int W);
// counts[0] += labelled valid pixels of the label images img [F][H][W],
// counts[1] += those whose label is the argmax of the pixel's own input.
hipError_t launch_agreement(const ProbIn& in, int c, int F, int H, int W, const uint8_t* img,
                            unsigned long long* counts, hipStream_t s);
hipError_t launch_render(const int32_t* l, const uint8_t* valid, const uint8_t* labels, int64_t npx,
                         uint8_t* out, hipStream_t s);

// texel resolution from the worst-case frame (fuse.hip)
hipError_t launch_area_max(const int32_t* tri, int nf, int H, int W, int32_t* tricnt, int64_t T, int32_t* area,
                           hipStream_t s);
hipError_t launch_texel_resolution(const int32_t* area, int64_t T, float gamma, int32_t* s_face, hipStream_t s);

// learned per-observation weight (mlp.hip)
int mlp_nparam();
int mlp_packed_bytes();
hipError_t launch_mlp_pack(const float* params, void* packed, hipStream_t s);
hipError_t launch_adam(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s);
hipError_t launch_mlp_forward(const void* packed, const float* phi, int64_t n, float* w, hipStream_t s);
hipError_t launch_mlp_grad(const void* packed, const float* phi, const float* tgt, int64_t n, float inv_total,
                           float* grad, float* loss, hipStream_t s);
hipError_t launch_mlp_weights(const void* packed, const ProbIn& in, int f_first, int nf, int H, int W,
                              const float* cams, const int32_t* l, const float4* geo, const int32_t* cnt,
                              int64_t cnt_stride, int c, float* wpix, hipStream_t s);
hipError_t launch_extract(const ProbIn& in, int f_first, int nf, int H, int W, const float* cams, const int32_t* l,
                          const float4* geo, const int32_t* cnt, int64_t cnt_stride, int c, const uint8_t* labels,
                          float* phi, float* tgt, int32_t* pix, int64_t cap, unsigned long long* count, hipStream_t s);

}  // namespace lf
