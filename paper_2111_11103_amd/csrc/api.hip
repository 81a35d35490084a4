// C-ABI of the semfuse library: argument checking, workspace carving and the
// per-batch launch sequence.  See include/semfuse.h for the contract.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/semfuse.h"
#include "internal.h"

using namespace lf;

// Event pairs recorded around the kernels of each stage when profiling is on.
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<hipEvent_t> marks[LF_N_STAGES];   // start, end, start, end, ...
  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void recycle() {
    for (auto& v : marks) {
      for (hipEvent_t e : v) pool.push_back(e);
      v.clear();
    }
  }
  ~Profiler() {
    recycle();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

struct lf_mesh_s {
  uint32_t magic;
  MeshDev d;
  lf_mesh_opts opts;
  Profiler prof;
  const void* mlp = nullptr;   // bound packed weights of the learned weighting
};

namespace {
// Records an event pair around the launches in its scope (stage `st`).
struct StageTimer {
  Profiler* p;
  int st;
  hipStream_t s;
  StageTimer(lf_mesh_s* m, int stage, hipStream_t stream) : p(m && m->prof.on ? &m->prof : nullptr), st(stage), s(stream) {
    if (p) {
      hipEvent_t e = p->take();
      if (e && hipEventRecord(e, s) == hipSuccess) p->marks[st].push_back(e);
      else p = nullptr;
    }
  }
  ~StageTimer() {
    if (p) {
      hipEvent_t e = p->take();
      if (e && hipEventRecord(e, s) == hipSuccess) p->marks[st].push_back(e);
      else p->marks[st].pop_back();
    }
  }
};
}  // namespace

namespace {

constexpr uint32_t kMagic = 0x5E4F05E1u;
thread_local char g_err[512] = "";

lf_status fail(lf_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

lf_status hip_check(hipError_t e, const char* where) {
  if (e != hipSuccess) return fail(LF_EHIP, "%s: %s", where, hipGetErrorString(e));
  return LF_OK;
}

#define LF_TRY(expr, where)                                 \
  do {                                                      \
    lf_status _st = hip_check((expr), (where));             \
    if (_st != LF_OK) return _st;                           \
  } while (0)

int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }

int64_t per_tri(int32_t s, int32_t scheme) {
  return scheme == LF_TEX_SPLIT ? (int64_t)s * s : (int64_t)s * (s + 1) / 2;
}

struct MeshLayout {
  int64_t faces_uv, s_face, off, cl_box, err, scan, total;
};

MeshLayout mesh_layout(int64_t T, bool per_face) {
  MeshLayout L{};
  int64_t o = 0;
  L.faces_uv = o; o += align256(T * 3 * 4);
  L.s_face = o; if (per_face) o += align256(T * 4);
  L.off = o; if (per_face) o += align256((T + 1) * 8);
  const int64_t ncl = (T + kClusterTris - 1) / kClusterTris;
  L.cl_box = o; o += align256(ncl * 8 * 4);
  L.err = o; o += 256;
  L.scan = o; if (per_face) o += align256(((T + 4095) / 4096 + 2) * 8);
  L.total = o;
  return L;
}

lf_status check_opts(const lf_mesh_opts* o) {
  if (!o) return fail(LF_EINVAL, "options are NULL");
  if (o->scheme != LF_TEX_SQUARE && o->scheme != LF_TEX_SPLIT) return fail(LF_EINVAL, "unknown texel scheme %d", o->scheme);
  if (o->n_classes < 1 || o->n_classes > 255) return fail(LF_EINVAL, "n_classes must be in [1, 255], got %d", o->n_classes);
  if (o->aggregator < LF_AGG_SUM || o->aggregator > LF_AGG_MAXSUM) return fail(LF_EINVAL, "unknown aggregator %d", o->aggregator);
  if (o->accum_dtype != LF_F32 && o->accum_dtype != LF_BF16 && o->accum_dtype != LF_F16)
    return fail(LF_EINVAL, "accumulator dtype %d not supported", o->accum_dtype);
  if (o->accum_dtype != LF_F32 && o->aggregator == LF_AGG_MUL)
    return fail(LF_EINVAL, "MUL aggregation keeps log-probability sums and needs an FP32 accumulator");
  if (!(o->z_near > 0.0f)) return fail(LF_EINVAL, "z_near must be > 0");
  return LF_OK;
}

lf_status check_mesh(lf_mesh m) {
  if (!m || m->magic != kMagic) return fail(LF_ESTATE, "invalid or freed mesh handle");
  return LF_OK;
}

struct FrameLayout {
  int64_t vis, vis_n, tcnt, toff, over, tlist, l, cnt, geo, wpix, seg, rank, start, sums, rows, nrows, ent_off, ent_w,
      ent_s, total;
  int64_t list_cap, ntiles;
  bool sorted;
};

int64_t tiles_of(int H, int W) {
  return (int64_t)((W + kTileSize - 1) / kTileSize) * ((H + kTileSize - 1) / kTileSize);
}

FrameLayout frame_layout(const MeshDev& m, int H, int W, int B, int weighting, int scatter_mode) {
  FrameLayout L{};
  const int64_t HW = (int64_t)H * W;
  L.ntiles = tiles_of(H, W);
  L.list_cap = 4 * m.T + 64 * L.ntiles + 1024;
  L.sorted = scatter_mode != LF_SCATTER_ATOMIC;
  int64_t o = 0;
  L.vis = o; o += align256(B * std::max<int64_t>(m.n_clusters, 1) * 4);
  L.vis_n = o; o += align256(B * 4);
  L.tcnt = o; o += align256(B * L.ntiles * 4);
  L.toff = o; o += align256(B * (L.ntiles + 1) * 4);
  L.over = o; o += align256(B * 4);
  L.tlist = o; o += align256(B * L.list_cap * 4);
  L.l = o; o += align256(B * HW * 4);
  L.cnt = o; if (weighting == LF_W_IMAGE || weighting == LF_W_LEARNED) o += align256(B * m.n_texels * 4);
  L.geo = o; if (weighting == LF_W_LEARNED) o += align256(B * HW * 16);
  L.wpix = o; if (weighting == LF_W_LEARNED) o += align256(B * HW * 4);
  L.seg = o; if (L.sorted) o += align256(m.n_texels * 4);
  L.rank = o; if (L.sorted) o += align256(B * HW * 4);
  L.start = o; if (L.sorted) o += align256((m.n_texels + 1) * 4);
  L.sums = o; if (L.sorted) o += align256((m.n_texels / 8192 + 2) * 4);
  L.rows = o; if (L.sorted) o += align256(m.n_texels * 4);
  L.nrows = o; if (L.sorted) o += 256;
  L.ent_off = o; if (L.sorted) o += align256(B * HW * 4);
  L.ent_w = o; if (L.sorted) o += align256(B * HW * 4);
  L.ent_s = o; if (L.sorted) o += align256(B * HW * 4);
  L.total = o;
  return L;
}

lf_status check_frames(int32_t F, int32_t H, int32_t W) {
  if (F < 0) return fail(LF_EINVAL, "negative frame count");
  if (H < 1 || W < 1 || H > 8192 || W > 8192) return fail(LF_EINVAL, "image size %dx%d out of range [1, 8192]", W, H);
  return LF_OK;
}

RasterWs raster_ws(const FrameLayout& L, char* ws) {
  RasterWs r;
  r.vis = reinterpret_cast<int32_t*>(ws + L.vis);
  r.vis_n = reinterpret_cast<int32_t*>(ws + L.vis_n);
  r.tcnt = reinterpret_cast<int32_t*>(ws + L.tcnt);
  r.toff = reinterpret_cast<int32_t*>(ws + L.toff);
  r.over = reinterpret_cast<int32_t*>(ws + L.over);
  r.tlist = reinterpret_cast<int32_t*>(ws + L.tlist);
  r.list_cap = L.list_cap;
  return r;
}

// Render frames [f0, f0 + nb) of the call and resolve them into texel rows
// (and optional triangle / depth outputs, per-frame and per-row counts).
lf_status render_batch(lf_mesh_s* mh, const float* cams, int f0, int nb, int H, int W, const FrameLayout& L,
                       char* ws, const RasterOut& out, hipStream_t s) {
  StageTimer tm(mh, 0, s);
  LF_TRY(launch_render_batch(mh->d, cams + 16 * (int64_t)f0, nb, H, W, raster_ws(L, ws), out, s), "render");
  return LF_OK;
}

int pick_batch(const MeshDev& m, int H, int W, int F, int64_t ws_bytes, int weighting, int mode) {
  int B = 1;
  while (B < F && B < 64 && frame_layout(m, H, W, B * 2, weighting, mode).total <= ws_bytes) B *= 2;
  return B > F ? F : B;
}

}  // namespace

extern "C" {

const char* lf_last_error(void) { return g_err; }
const char* lf_version(void) { return "semfuse 0.1 (gfx950)"; }

lf_status lf_mesh_sizes(const lf_mesh_opts* opts, int64_t n_vertices, int64_t n_faces, const int32_t* h_s_face,
                        int64_t* n_texels, int64_t* mesh_ws_bytes) {
  g_err[0] = 0;
  lf_status st = check_opts(opts);
  if (st != LF_OK) return st;
  if (n_vertices < 0 || n_faces < 0 || n_faces >= (int64_t)1 << 31) return fail(LF_EINVAL, "bad vertex/face count");
  int64_t nx = 0;
  if (h_s_face) {
    for (int64_t t = 0; t < n_faces; ++t) {
      if (h_s_face[t] < 1) return fail(LF_EINVAL, "s of face %lld is %d (< 1)", (long long)t, h_s_face[t]);
      nx += per_tri(h_s_face[t], opts->scheme);
    }
  } else {
    if (opts->s_uniform < 1 || opts->s_uniform > 4096) return fail(LF_EINVAL, "s_uniform must be in [1, 4096]");
    nx = n_faces * per_tri(opts->s_uniform, opts->scheme);
  }
  if (nx >= ((int64_t)1 << 31)) return fail(LF_EINVAL, "texel count %lld exceeds 2^31 - 1", (long long)nx);
  if (n_texels) *n_texels = nx;
  if (mesh_ws_bytes) *mesh_ws_bytes = mesh_layout(n_faces, h_s_face != nullptr).total;
  return LF_OK;
}

lf_status lf_load_mesh(const lf_mesh_opts* opts, const float* d_vertices, int64_t n_vertices, const int32_t* d_faces,
                       int64_t n_faces, const int32_t* d_s_face, void* d_mesh_ws, int64_t mesh_ws_bytes,
                       void* d_accum, float* d_wsum, int64_t n_texels, hipStream_t stream, lf_mesh* out) {
  g_err[0] = 0;
  if (!out) return fail(LF_EINVAL, "out handle pointer is NULL");
  *out = nullptr;
  lf_status st = check_opts(opts);
  if (st != LF_OK) return st;
  if (n_vertices < 1 || n_faces < 0 || n_faces >= (int64_t)1 << 31) return fail(LF_EINVAL, "bad vertex/face count");
  if (!d_vertices || (!d_faces && n_faces > 0) || !d_mesh_ws || (!d_accum && n_texels > 0))
    return fail(LF_EINVAL, "NULL device buffer");
  if (reinterpret_cast<uintptr_t>(d_mesh_ws) & 255) return fail(LF_EINVAL, "mesh workspace must be 256-byte aligned");
  if (opts->aggregator == LF_AGG_MUL && !d_wsum) return fail(LF_EINVAL, "MUL aggregation needs the weight-sum buffer");
  const bool per_face = d_s_face != nullptr;
  if (!per_face && (opts->s_uniform < 1 || opts->s_uniform > 4096)) return fail(LF_EINVAL, "s_uniform must be in [1, 4096]");
  const MeshLayout L = mesh_layout(n_faces, per_face);
  if (mesh_ws_bytes < L.total) return fail(LF_ESIZE, "mesh workspace %lld < %lld bytes", (long long)mesh_ws_bytes, (long long)L.total);
  if (!per_face) {
    const int64_t want = n_faces * per_tri(opts->s_uniform, opts->scheme);
    if (want != n_texels) return fail(LF_ESIZE, "n_texels %lld != %lld", (long long)n_texels, (long long)want);
  }
  char* ws = reinterpret_cast<char*>(d_mesh_ws);
  MeshDev d{};
  d.verts = d_vertices;
  d.faces_uv = reinterpret_cast<int32_t*>(ws + L.faces_uv);
  d.s_face = per_face ? reinterpret_cast<int32_t*>(ws + L.s_face) : nullptr;
  d.off = per_face ? reinterpret_cast<int64_t*>(ws + L.off) : nullptr;
  d.cl_box = reinterpret_cast<float*>(ws + L.cl_box);
  d.err = reinterpret_cast<int32_t*>(ws + L.err);
  d.accum = d_accum;
  d.wsum = d_wsum;
  d.V = n_vertices;
  d.T = n_faces;
  d.n_texels = n_texels;
  d.n_clusters = (n_faces + kClusterTris - 1) / kClusterTris;
  d.s_uniform = per_face ? 0 : opts->s_uniform;
  d.split = opts->scheme == LF_TEX_SPLIT;
  d.c = opts->n_classes;
  d.aggregator = opts->aggregator;
  d.accum_dtype = opts->accum_dtype;
  d.n_per = per_face ? 0 : (int32_t)per_tri(opts->s_uniform, opts->scheme);
  d.z_near = opts->z_near;

  LF_TRY(launch_zero(d.err, 4, stream), "clear flag");
  if (per_face)
    LF_TRY(hipMemcpyAsync(d.s_face, d_s_face, n_faces * 4, hipMemcpyDeviceToDevice, stream), "copy s");
  LF_TRY(launch_mesh_prep(d, d_faces, stream), "mesh prep");
  if (per_face) LF_TRY(launch_offsets(d, reinterpret_cast<int32_t*>(ws + L.scan), stream), "offsets");
  LF_TRY(launch_cluster_boxes(d, stream), "cluster boxes");
  LF_TRY(launch_zero(d_accum, n_texels * opts->n_classes * (opts->accum_dtype == LF_F32 ? 4 : 2), stream),
         "clear accumulator");
  if (d_wsum) LF_TRY(launch_zero(d_wsum, n_texels * 4, stream), "clear weights");
  int32_t herr = 0;
  int64_t htot = n_texels;
  LF_TRY(hipMemcpyAsync(&herr, d.err, 4, hipMemcpyDeviceToHost, stream), "read flag");
  if (per_face) LF_TRY(hipMemcpyAsync(&htot, d.off + n_faces, 8, hipMemcpyDeviceToHost, stream), "read total");
  LF_TRY(hipStreamSynchronize(stream), "sync");
  if (herr) return fail(LF_EINVAL, "face index out of range [0, %lld) or s < 1", (long long)n_vertices);
  if (htot != n_texels) return fail(LF_ESIZE, "n_texels %lld != %lld", (long long)n_texels, (long long)htot);
  lf_mesh h = new (std::nothrow) lf_mesh_s;
  if (!h) return fail(LF_EINVAL, "out of host memory");
  h->magic = kMagic;
  h->d = d;
  h->opts = *opts;
  *out = h;
  return LF_OK;
}

lf_status lf_reset(lf_mesh mesh, hipStream_t stream) {
  g_err[0] = 0;
  lf_status st = check_mesh(mesh);
  if (st != LF_OK) return st;
  StageTimer tm(mesh, 6, stream);
  LF_TRY(launch_zero(mesh->d.accum, mesh->d.n_texels * mesh->d.c * (mesh->d.accum_dtype == LF_F32 ? 4 : 2), stream),
         "clear accumulator");
  if (mesh->d.wsum) LF_TRY(launch_zero(mesh->d.wsum, mesh->d.n_texels * 4, stream), "clear weights");
  return LF_OK;
}

lf_status lf_frame_ws_bytes(lf_mesh mesh, int32_t H, int32_t W, int32_t batch, int32_t weighting,
                            int32_t scatter_mode, int64_t* bytes) {
  g_err[0] = 0;
  lf_status st = check_mesh(mesh);
  if (st != LF_OK) return st;
  if ((st = check_frames(1, H, W)) != LF_OK) return st;
  if (batch < 1 || batch > 65535) return fail(LF_EINVAL, "batch must be in [1, 65535]");
  if (bytes) *bytes = frame_layout(mesh->d, H, W, batch, weighting, scatter_mode).total;
  return LF_OK;
}

lf_status lf_fuse_frames(lf_mesh mesh, const float* d_cams, int32_t F, int32_t H, int32_t W, const void* d_probs,
                         int32_t prob_dtype, const int64_t* h_strides, const float* d_scale, const uint8_t* d_valid,
                         int32_t weighting, int32_t* d_l_out, void* d_ws, int64_t ws_bytes, int32_t batch,
                         int32_t scatter_mode, hipStream_t stream) {
  g_err[0] = 0;
  lf_status st = check_mesh(mesh);
  if (st != LF_OK) return st;
  if ((st = check_frames(F, H, W)) != LF_OK) return st;
  if (F == 0) return LF_OK;
  if (!d_cams || !d_probs || !h_strides || !d_ws) return fail(LF_EINVAL, "NULL argument");
  if (prob_dtype != LF_F32 && prob_dtype != LF_FP8_E4M3) return fail(LF_EINVAL, "probabilities must be F32 or FP8_E4M3");
  if (prob_dtype == LF_FP8_E4M3 && !d_scale) return fail(LF_EINVAL, "FP8 input needs the per-pixel scale");
  if (weighting < LF_W_PIXEL || weighting > LF_W_LEARNED) return fail(LF_EINVAL, "unknown weighting %d", weighting);
  if (weighting == LF_W_LEARNED && !mesh->mlp) return fail(LF_ESTATE, "learned weighting needs weights bound by lf_mlp_bind");
  if (scatter_mode < LF_SCATTER_AUTO || scatter_mode > LF_SCATTER_SORTED) return fail(LF_EINVAL, "bad scatter mode");
  for (int i = 0; i < 4; ++i)
    if (h_strides[i] < 0) return fail(LF_EINVAL, "negative stride");
  if (batch < 1) return fail(LF_EINVAL, "batch must be >= 1");
  if (reinterpret_cast<uintptr_t>(d_ws) & 255) return fail(LF_EINVAL, "workspace must be 256-byte aligned");
  const MeshDev& d = mesh->d;
  const int B = batch < F ? batch : F;
  // texel-sorted aggregation when the classes of a pixel are contiguous
  const int mode = scatter_mode != LF_SCATTER_AUTO ? scatter_mode
                                                   : (h_strides[1] == 1 ? LF_SCATTER_SORTED : LF_SCATTER_ATOMIC);
  const FrameLayout L = frame_layout(d, H, W, B, weighting, scatter_mode == LF_SCATTER_AUTO ? LF_SCATTER_SORTED : mode);
  if (ws_bytes < L.total) return fail(LF_ESIZE, "frame workspace %lld < %lld bytes", (long long)ws_bytes, (long long)L.total);
  char* ws = reinterpret_cast<char*>(d_ws);
  const int64_t HW = (int64_t)H * W;
  ProbIn in{d_probs, d_scale, d_valid, h_strides[0], h_strides[1], h_strides[2], h_strides[3], prob_dtype};
  const bool learned = weighting == LF_W_LEARNED;
  int32_t* cnt = weighting != LF_W_PIXEL ? reinterpret_cast<int32_t*>(ws + L.cnt) : nullptr;
  float4* geo = learned ? reinterpret_cast<float4*>(ws + L.geo) : nullptr;
  float* wpix = learned ? reinterpret_cast<float*>(ws + L.wpix) : nullptr;
  // the sorted path stores batch-relative element offsets in 32 bits
  const bool sorted = mode == LF_SCATTER_SORTED &&
                      ((int64_t)(B - 1) * h_strides[0] + (int64_t)(H - 1) * h_strides[2] +
                       (int64_t)(W - 1) * h_strides[3] + (int64_t)d.c * h_strides[1]) < ((int64_t)1 << 32);
  int32_t* seg = sorted ? reinterpret_cast<int32_t*>(ws + L.seg) : nullptr;
  LF_TRY(launch_zero(ws + L.tcnt, B * L.ntiles * 4, stream), "clear tile counts");
  if (cnt) LF_TRY(launch_zero(cnt, (int64_t)B * d.n_texels * 4, stream), "clear counts");
  int32_t* rank = sorted ? reinterpret_cast<int32_t*>(ws + L.rank) : nullptr;
  for (int f0 = 0; f0 < F; f0 += B) {
    const int nb = (F - f0) < B ? (F - f0) : B;
    int32_t* lb = d_l_out ? d_l_out + (int64_t)f0 * HW : reinterpret_cast<int32_t*>(ws + L.l);
    const uint8_t* vb = d_valid ? d_valid + (int64_t)f0 * HW : nullptr;
    if (seg) LF_TRY(launch_zero(seg, d.n_texels * 4, stream), "clear segments");
    RasterOut out{lb, nullptr, nullptr, vb, cnt, d.n_texels, seg, rank, geo};
    if ((st = render_batch(mesh, d_cams, f0, nb, H, W, L, ws, out, stream)) != LF_OK) return st;
    if (learned) {
      StageTimer tm(mesh, 7, stream);
      LF_TRY(launch_mlp_weights(mesh->mlp, in, f0, nb, H, W, d_cams, lb, geo, cnt, d.n_texels, d.c, wpix, stream),
             "learned weights");
    }
    if (sorted) {
      int32_t* start = reinterpret_cast<int32_t*>(ws + L.start);
      uint32_t* eo = reinterpret_cast<uint32_t*>(ws + L.ent_off);
      float* ew = weighting != LF_W_PIXEL ? reinterpret_cast<float*>(ws + L.ent_w) : nullptr;
      float* es = prob_dtype == LF_FP8_E4M3 ? reinterpret_cast<float*>(ws + L.ent_s) : nullptr;
      {
        StageTimer tm(mesh, 3, stream);
        LF_TRY(launch_zero(ws + L.nrows, 4, stream), "clear row count");
        LF_TRY(launch_seg_scan(seg, d.n_texels, reinterpret_cast<int32_t*>(ws + L.sums), start,
                               reinterpret_cast<int32_t*>(ws + L.rows), reinterpret_cast<int32_t*>(ws + L.nrows),
                               stream), "segment scan");
        LF_TRY(launch_seg_fill(in, f0, nb, H, W, lb, rank, start, eo, ew, es, weighting, cnt, d.n_texels, wpix, stream),
               "segment fill");
      }
      StageTimer tm(mesh, 2, stream);
      LF_TRY(launch_seg_gather(d, in, f0, H, W, start, reinterpret_cast<int32_t*>(ws + L.rows),
                               reinterpret_cast<int32_t*>(ws + L.nrows), eo, ew, es, stream), "segment gather");
    } else {
      StageTimer tm(mesh, 2, stream);
      LF_TRY(launch_scatter_atomic(d, in, f0, nb, H, W, lb, weighting, cnt, d.n_texels, wpix, stream), "scatter");
    }
    if (cnt) {
      StageTimer tm(mesh, 3, stream);
      LF_TRY(launch_clear_counts(lb, vb, nb, H, W, cnt, d.n_texels, stream), "clear counts");
    }
  }
  return LF_OK;
}

lf_status lf_finalize(lf_mesh mesh, void* d_tex_out, int32_t tex_dtype, uint8_t* d_labels, hipStream_t stream) {
  g_err[0] = 0;
  lf_status st = check_mesh(mesh);
  if (st != LF_OK) return st;
  if (!d_labels) return fail(LF_EINVAL, "labels buffer is NULL");
  if (tex_dtype != LF_F32 && tex_dtype != LF_BF16 && tex_dtype != LF_F16) return fail(LF_EINVAL, "bad texture dtype");
  StageTimer tm(mesh, 4, stream);
  LF_TRY(launch_finalize(mesh->d, d_tex_out, tex_dtype, d_labels, stream), "finalize");
  return LF_OK;
}

lf_status lf_render_labels(lf_mesh mesh, const float* d_cams, int32_t F, int32_t H, int32_t W, const int32_t* d_l,
                           const uint8_t* d_valid, const uint8_t* d_labels, uint8_t* d_out, void* d_ws,
                           int64_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  lf_status st = check_mesh(mesh);
  if (st != LF_OK) return st;
  if ((st = check_frames(F, H, W)) != LF_OK) return st;
  if (!d_labels || !d_out) return fail(LF_EINVAL, "NULL argument");
  const int64_t HW = (int64_t)H * W;
  if (d_l) {
    StageTimer tm(mesh, 5, stream);
    LF_TRY(launch_render(d_l, d_valid, d_labels, (int64_t)F * HW, d_out, stream), "render");
    return LF_OK;
  }
  if (!d_cams || !d_ws) return fail(LF_EINVAL, "re-rendering needs cameras and a workspace");
  if (F == 0) return LF_OK;
  if (reinterpret_cast<uintptr_t>(d_ws) & 255) return fail(LF_EINVAL, "workspace must be 256-byte aligned");
  const int B = pick_batch(mesh->d, H, W, F, ws_bytes, LF_W_PIXEL, LF_SCATTER_ATOMIC);
  const FrameLayout L = frame_layout(mesh->d, H, W, B, LF_W_PIXEL, LF_SCATTER_ATOMIC);
  if (ws_bytes < L.total) return fail(LF_ESIZE, "frame workspace too small");
  char* ws = reinterpret_cast<char*>(d_ws);
  LF_TRY(launch_zero(ws + L.tcnt, B * L.ntiles * 4, stream), "clear tile counts");
  for (int f0 = 0; f0 < F; f0 += B) {
    const int nb = (F - f0) < B ? (F - f0) : B;
    int32_t* lb = reinterpret_cast<int32_t*>(ws + L.l);
    RasterOut out{lb, nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr};
    if ((st = render_batch(mesh, d_cams, f0, nb, H, W, L, ws, out, stream)) != LF_OK) return st;
    StageTimer tm(mesh, 5, stream);
    LF_TRY(launch_render(lb, d_valid ? d_valid + (int64_t)f0 * HW : nullptr, d_labels, (int64_t)nb * HW,
                         d_out + (int64_t)f0 * HW, stream), "render");
  }
  return LF_OK;
}

lf_status lf_rasterize(lf_mesh mesh, const float* d_cams, int32_t F, int32_t H, int32_t W, int32_t* d_tri,
                       int32_t* d_l, float* d_z, void* d_ws, int64_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  lf_status st = check_mesh(mesh);
  if (st != LF_OK) return st;
  if ((st = check_frames(F, H, W)) != LF_OK) return st;
  if (F == 0) return LF_OK;
  if (!d_cams || !d_ws) return fail(LF_EINVAL, "NULL argument");
  if (reinterpret_cast<uintptr_t>(d_ws) & 255) return fail(LF_EINVAL, "workspace must be 256-byte aligned");
  const int B = pick_batch(mesh->d, H, W, F, ws_bytes, LF_W_PIXEL, LF_SCATTER_ATOMIC);
  const FrameLayout L = frame_layout(mesh->d, H, W, B, LF_W_PIXEL, LF_SCATTER_ATOMIC);
  if (ws_bytes < L.total) return fail(LF_ESIZE, "frame workspace too small");
  char* ws = reinterpret_cast<char*>(d_ws);
  const int64_t HW = (int64_t)H * W;
  LF_TRY(launch_zero(ws + L.tcnt, B * L.ntiles * 4, stream), "clear tile counts");
  for (int f0 = 0; f0 < F; f0 += B) {
    const int nb = (F - f0) < B ? (F - f0) : B;
    const int64_t o = (int64_t)f0 * HW;
    RasterOut out{d_l ? d_l + o : nullptr, d_tri ? d_tri + o : nullptr, d_z ? d_z + o : nullptr, nullptr, nullptr, 0,
                  nullptr, nullptr, nullptr};
    if ((st = render_batch(mesh, d_cams, f0, nb, H, W, L, ws, out, stream)) != LF_OK) return st;
  }
  return LF_OK;
}

lf_status lf_profile_enable(lf_mesh mesh, int32_t on) {
  g_err[0] = 0;
  lf_status st = check_mesh(mesh);
  if (st != LF_OK) return st;
  for (auto& v : mesh->prof.marks)
    for (hipEvent_t e : v) (void)hipEventSynchronize(e);
  mesh->prof.recycle();
  mesh->prof.on = on != 0;
  return LF_OK;
}

lf_status lf_profile_read(lf_mesh mesh, lf_profile* out) {
  g_err[0] = 0;
  lf_status st = check_mesh(mesh);
  if (st != LF_OK) return st;
  if (!out) return fail(LF_EINVAL, "NULL profile");
  for (int k = 0; k < LF_N_STAGES; ++k) {
    double ms = 0.0;
    const auto& v = mesh->prof.marks[k];
    for (size_t i = 0; i + 1 < v.size(); i += 2) {
      LF_TRY(hipEventSynchronize(v[i + 1]), "event sync");
      float t = 0.0f;
      LF_TRY(hipEventElapsedTime(&t, v[i], v[i + 1]), "event time");
      ms += t;
    }
    out->ms[k] = ms;
    out->launches[k] = (int64_t)(v.size() / 2);
  }
  return LF_OK;
}

// ---- learned per-observation weight --------------------------------------------

lf_status lf_mlp_sizes(int32_t* n_params, int64_t* packed_bytes) {
  g_err[0] = 0;
  if (n_params) *n_params = mlp_nparam();
  if (packed_bytes) *packed_bytes = mlp_packed_bytes();
  return LF_OK;
}

lf_status lf_mlp_pack(const float* d_params, void* d_packed, hipStream_t stream) {
  g_err[0] = 0;
  if (!d_params || !d_packed) return fail(LF_EINVAL, "NULL argument");
  if (reinterpret_cast<uintptr_t>(d_packed) & 15) return fail(LF_EINVAL, "packed weights must be 16-byte aligned");
  LF_TRY(launch_mlp_pack(d_params, d_packed, stream), "pack");
  return LF_OK;
}

lf_status lf_mlp_bind(lf_mesh mesh, const void* d_packed) {
  g_err[0] = 0;
  lf_status st = check_mesh(mesh);
  if (st != LF_OK) return st;
  if (d_packed && (reinterpret_cast<uintptr_t>(d_packed) & 15))
    return fail(LF_EINVAL, "packed weights must be 16-byte aligned");
  mesh->mlp = d_packed;
  return LF_OK;
}

lf_status lf_mlp_forward(const void* d_packed, const float* d_phi, int64_t n, float* d_w, hipStream_t stream) {
  g_err[0] = 0;
  if (n < 0) return fail(LF_EINVAL, "negative count");
  if (n == 0) return LF_OK;
  if (!d_packed || !d_phi || !d_w) return fail(LF_EINVAL, "NULL argument");
  if (n > ((int64_t)1 << 40)) return fail(LF_EINVAL, "too many observations");
  LF_TRY(launch_mlp_forward(d_packed, d_phi, n, d_w, stream), "forward");
  return LF_OK;
}

lf_status lf_mlp_grad(const void* d_packed, const float* d_phi, const float* d_target, int64_t n, float* d_grad,
                      float* d_loss, hipStream_t stream) {
  g_err[0] = 0;
  if (n < 0) return fail(LF_EINVAL, "negative count");
  if (!d_grad) return fail(LF_EINVAL, "NULL gradient buffer");
  LF_TRY(launch_zero(d_grad, (int64_t)mlp_nparam() * 4, stream), "clear gradient");
  if (d_loss) LF_TRY(launch_zero(d_loss, 4, stream), "clear loss");
  if (n == 0) return LF_OK;
  if (!d_packed || !d_phi || !d_target) return fail(LF_EINVAL, "NULL argument");
  if (n > ((int64_t)1 << 40)) return fail(LF_EINVAL, "too many observations");
  LF_TRY(launch_mlp_grad(d_packed, d_phi, d_target, n, (float)(1.0 / (double)n), d_grad, d_loss, stream), "gradient");
  return LF_OK;
}

lf_status lf_adam_step(float* d_params, float* d_m, float* d_v, const float* d_grad, int64_t n, float lr,
                       float beta1, float beta2, float eps, int32_t step, hipStream_t stream) {
  g_err[0] = 0;
  if (n < 0) return fail(LF_EINVAL, "negative count");
  if (step < 1) return fail(LF_EINVAL, "Adam step counts from 1");
  if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return fail(LF_EINVAL, "Adam needs 0 <= beta < 1 and eps > 0");
  if (n == 0) return LF_OK;
  if (!d_params || !d_m || !d_v || !d_grad) return fail(LF_EINVAL, "NULL argument");
  LF_TRY(launch_adam(d_params, d_m, d_v, d_grad, n, lr, beta1, beta2, eps, step, stream), "adam");
  return LF_OK;
}

lf_status lf_extract_features(lf_mesh mesh, const float* d_cams, int32_t F, int32_t H, int32_t W, const void* d_probs,
                              int32_t prob_dtype, const int64_t* h_strides, const float* d_scale,
                              const uint8_t* d_valid, const uint8_t* d_labels, float* d_phi, float* d_target,
                              int32_t* d_pix, int64_t cap, uint64_t* d_count, void* d_ws, int64_t ws_bytes,
                              hipStream_t stream) {
  g_err[0] = 0;
  lf_status st = check_mesh(mesh);
  if (st != LF_OK) return st;
  if ((st = check_frames(F, H, W)) != LF_OK) return st;
  if (!d_count) return fail(LF_EINVAL, "NULL count");
  LF_TRY(launch_zero(d_count, 8, stream), "clear count");
  if (F == 0) return LF_OK;
  if (!d_cams || !d_probs || !h_strides || !d_ws || !d_phi) return fail(LF_EINVAL, "NULL argument");
  if (d_target && !d_labels) return fail(LF_EINVAL, "targets need the fused labels");
  if (cap < 0) return fail(LF_EINVAL, "negative capacity");
  if (prob_dtype != LF_F32 && prob_dtype != LF_FP8_E4M3) return fail(LF_EINVAL, "probabilities must be F32 or FP8_E4M3");
  if (prob_dtype == LF_FP8_E4M3 && !d_scale) return fail(LF_EINVAL, "FP8 input needs the per-pixel scale");
  for (int i = 0; i < 4; ++i)
    if (h_strides[i] < 0) return fail(LF_EINVAL, "negative stride");
  const int64_t HW = (int64_t)H * W;
  if (d_pix && (int64_t)F * HW >= ((int64_t)1 << 31)) return fail(LF_EINVAL, "pixel indices exceed int32");
  if (reinterpret_cast<uintptr_t>(d_ws) & 255) return fail(LF_EINVAL, "workspace must be 256-byte aligned");
  const MeshDev& d = mesh->d;
  const int B = pick_batch(d, H, W, F, ws_bytes, LF_W_LEARNED, LF_SCATTER_ATOMIC);
  const FrameLayout L = frame_layout(d, H, W, B, LF_W_LEARNED, LF_SCATTER_ATOMIC);
  if (ws_bytes < L.total) return fail(LF_ESIZE, "frame workspace %lld < %lld bytes", (long long)ws_bytes, (long long)L.total);
  char* ws = reinterpret_cast<char*>(d_ws);
  ProbIn in{d_probs, d_scale, d_valid, h_strides[0], h_strides[1], h_strides[2], h_strides[3], prob_dtype};
  int32_t* cnt = reinterpret_cast<int32_t*>(ws + L.cnt);
  float4* geo = reinterpret_cast<float4*>(ws + L.geo);
  int32_t* lb = reinterpret_cast<int32_t*>(ws + L.l);
  LF_TRY(launch_zero(ws + L.tcnt, B * L.ntiles * 4, stream), "clear tile counts");
  LF_TRY(launch_zero(cnt, (int64_t)B * d.n_texels * 4, stream), "clear counts");
  for (int f0 = 0; f0 < F; f0 += B) {
    const int nb = (F - f0) < B ? (F - f0) : B;
    const uint8_t* vb = d_valid ? d_valid + (int64_t)f0 * HW : nullptr;
    RasterOut out{lb, nullptr, nullptr, vb, cnt, d.n_texels, nullptr, nullptr, geo};
    if ((st = render_batch(mesh, d_cams, f0, nb, H, W, L, ws, out, stream)) != LF_OK) return st;
    StageTimer tm(mesh, 7, stream);
    LF_TRY(launch_extract(in, f0, nb, H, W, d_cams, lb, geo, cnt, d.n_texels, d.c, d_labels, d_phi, d_target, d_pix,
                          cap, reinterpret_cast<unsigned long long*>(d_count), stream), "extract");
    LF_TRY(launch_clear_counts(lb, vb, nb, H, W, cnt, d.n_texels, stream), "clear counts");
  }
  return LF_OK;
}

void lf_free_mesh(lf_mesh mesh) {
  if (mesh && mesh->magic == kMagic) {
    mesh->magic = 0;
    delete mesh;
  }
}

}  // extern "C"
