// C-ABI of the semfuse library: argument checking, workspace carving and the
// per-batch launch sequence.  See include/semfuse.h for the contract.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
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
  void* accum_full = nullptr;  // the load-time accumulator and weight sums (all rows)
  float* wsum_full = nullptr;
  // Second stream of the sorted path: the gather of batch k runs on it while
  // the caller's stream renders and sorts batch k + 1 (events order them).
  hipStream_t side = nullptr;
  hipEvent_t sorted_ev[2] = {nullptr, nullptr};    // batch's entries are ready (caller's stream)
  hipEvent_t gathered_ev[2] = {nullptr, nullptr};  // batch's gather is done (side stream)
  bool overlap = true;                              // false: gathers run on the caller's stream
  ~lf_mesh_s() {
    for (int i = 0; i < 2; ++i) {
      if (sorted_ev[i]) (void)hipEventDestroy(sorted_ev[i]);
      if (gathered_ev[i]) (void)hipEventDestroy(gathered_ev[i]);
    }
    if (side) (void)hipStreamDestroy(side);
  }
};

namespace {
// Records an event pair around the launches in its scope (stage `st`).
struct StageTimer {
  Profiler* p;
  int st;
  hipStream_t s;
  StageTimer(lf_mesh_s* m, int stage, hipStream_t stream)
      : p(m && m->prof.on ? &m->prof : nullptr), st(stage), s(stream) {
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
  int64_t faces_uv, tri_v, s_face, off, cl_box, err, scan, total;
};

MeshLayout mesh_layout(int64_t T, bool per_face) {
  MeshLayout L{};
  int64_t o = 0;
  L.faces_uv = o; o += align256(T * 3 * 4);
  L.tri_v = o; o += align256(T * 48);
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
  int64_t vis, vis_n, tcnt, tlist, l, cnt, geo, wpix, seg, rank, sums, total;
  // what the gather reads, twice: batch k uses set k % 2 (counts: [0] spans, [1] non-empty buckets)
  int64_t bstart[2], blist[2], counts[2], rec[2], rec_w[2], rec_s[2], spans[2], ent_off[2], ent_w[2], ent_s[2],
      stage[2];
  int64_t list_cap, ntiles, n_buckets;
  bool sorted;
};

int64_t tiles_of(int H, int W, int ts) {
  return (int64_t)((W + ts - 1) / ts) * ((H + ts - 1) / ts);
}

// grouped: 1 = the grouped gather reads the bucket records (no second sort
// through memory), 0 = the per-class gather (sorted through memory), -1 =
// not known (room for both).
FrameLayout frame_layout(const MeshDev& m, int H, int W, int B, int weighting, int scatter_mode, int grouped = -1) {
  FrameLayout L{};
  const int64_t HW = (int64_t)H * W;
  L.ntiles = tiles_of(H, W, m.tile);
  L.list_cap = 4 * m.T + 64 * L.ntiles + 1024;
  L.sorted = scatter_mode != LF_SCATTER_ATOMIC;
  L.n_buckets = (m.n_rows + (1 << kBucketShift) - 1) >> kBucketShift;
  const int64_t max_spans = std::min<int64_t>(m.n_rows, B * HW);
  const bool spans = L.sorted && grouped != 1;
  int64_t o = 0;
  L.vis = o; o += align256(B * std::max<int64_t>(m.n_clusters, 1) * 4);
  L.vis_n = o; o += align256(B * 4);
  L.tcnt = o; o += align256(B * L.ntiles * 4);
  L.tlist = o; o += align256(B * L.list_cap * 4);
  L.l = o; o += align256(B * HW * 4);
  L.cnt = o; if (weighting != LF_W_PIXEL) o += align256(B * m.n_rows * 4);
  // learned-weight geometry: two sets on the sorted path, whose gather may read them in place
  L.geo = o; if (weighting == LF_W_LEARNED) o += align256((L.sorted ? 2 : 1) * B * HW * 16);
  // learned weights: two sets on the sorted path, whose gather reads them in place
  L.wpix = o; if (weighting == LF_W_LEARNED) o += align256((L.sorted ? 2 : 1) * B * HW * 4);
  // first level of the sorted path, used on the caller's stream only: bucket
  // counts and ranks (resolve), scan partial sums
  L.seg = o; if (L.sorted) o += align256(L.n_buckets * 4);
  L.rank = o; if (L.sorted) o += align256(B * HW * 4);
  L.sums = o; if (L.sorted) o += align256((L.n_buckets / 8192 + 2) * 4);
  // AUTO may pick the staged form for planar inputs: size for it too
  const bool staged = scatter_mode == LF_SCATTER_STAGED ||
                      (scatter_mode == LF_SCATTER_AUTO && m.c % 4 == 0 && m.c <= 60);
  for (int k = 0; k < 2; ++k) {
    L.bstart[k] = o; if (L.sorted) o += align256((L.n_buckets + 1) * 4);
    L.blist[k] = o; if (L.sorted) o += align256(L.n_buckets * 4);
    L.counts[k] = o; if (L.sorted) o += 256;
    L.rec[k] = o; if (L.sorted) o += align256(B * HW * 8);
    L.rec_w[k] = o; if (L.sorted && weighting != LF_W_PIXEL) o += align256(B * HW * 4);
    L.rec_s[k] = o; if (L.sorted) o += align256(B * HW * 4);
    L.spans[k] = o; if (spans) o += align256(max_spans * 16);
    L.ent_off[k] = o; if (spans) o += align256(B * HW * 4);
    L.ent_w[k] = o; if (spans && weighting != LF_W_PIXEL) o += align256(B * HW * 4);
    L.ent_s[k] = o; if (spans) o += align256(B * HW * 4);
    L.stage[k] = o; if (staged) o += align256(B * HW * m.c * 4);
  }
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
  if (!d_vertices || (!d_faces && n_faces > 0) || !d_mesh_ws) return fail(LF_EINVAL, "NULL device buffer");
  if (!d_accum && d_wsum) return fail(LF_EINVAL, "weight sums without an accumulator");
  if (reinterpret_cast<uintptr_t>(d_mesh_ws) & 255) return fail(LF_EINVAL, "mesh workspace must be 256-byte aligned");
  if (opts->aggregator == LF_AGG_MUL && d_accum && !d_wsum)
    return fail(LF_EINVAL, "MUL aggregation needs the weight-sum buffer");
  const bool per_face = d_s_face != nullptr;
  if (!per_face && (opts->s_uniform < 1 || opts->s_uniform > 4096)) return fail(LF_EINVAL, "s_uniform must be in [1, 4096]");
  const MeshLayout L = mesh_layout(n_faces, per_face);
  if (mesh_ws_bytes < L.total) return fail(LF_ESIZE, "mesh workspace %lld < %lld bytes", (long long)mesh_ws_bytes, (long long)L.total);
  // texel rows are int32 everywhere on the device (l = id_t + id_x)
  if (n_texels < 0 || n_texels >= ((int64_t)1 << 31))
    return fail(LF_EINVAL, "texel count %lld outside [0, 2^31 - 1]", (long long)n_texels);
  if (!per_face) {
    const int64_t want = n_faces * per_tri(opts->s_uniform, opts->scheme);
    if (want >= ((int64_t)1 << 31)) return fail(LF_EINVAL, "texel count %lld exceeds 2^31 - 1", (long long)want);
    if (want != n_texels) return fail(LF_ESIZE, "n_texels %lld != %lld", (long long)n_texels, (long long)want);
  }
  char* ws = reinterpret_cast<char*>(d_mesh_ws);
  MeshDev d{};
  d.verts = d_vertices;
  d.faces_uv = reinterpret_cast<int32_t*>(ws + L.faces_uv);
  d.tri_v = reinterpret_cast<float4*>(ws + L.tri_v);
  d.s_face = per_face ? reinterpret_cast<int32_t*>(ws + L.s_face) : nullptr;
  d.off = per_face ? reinterpret_cast<int64_t*>(ws + L.off) : nullptr;
  d.cl_box = reinterpret_cast<float*>(ws + L.cl_box);
  d.err = reinterpret_cast<int32_t*>(ws + L.err);
  d.accum = d_accum;
  d.wsum = d_wsum;
  d.V = n_vertices;
  d.T = n_faces;
  d.n_texels = n_texels;
  d.win_lo = 0;
  d.n_rows = d_accum ? n_texels : 0;   // no accumulator: an empty window until lf_set_window
  d.n_clusters = (n_faces + kClusterTris - 1) / kClusterTris;
  d.s_uniform = per_face ? 0 : opts->s_uniform;
  d.split = opts->scheme == LF_TEX_SPLIT;
  d.c = opts->n_classes;
  d.aggregator = opts->aggregator;
  d.accum_dtype = opts->accum_dtype;
  d.n_per = per_face ? 0 : (int32_t)per_tri(opts->s_uniform, opts->scheme);
  d.z_near = opts->z_near;
  d.tile = kTileSize;
  d.gather_unroll = 8;
  d.small_px = 48;
  d.gather_waves = 8;
  d.learned_in_gather = 0;
  d.mix = 0.5f;

  LF_TRY(launch_zero(d.err, 4, stream), "clear flag");
  if (per_face)
    LF_TRY(hipMemcpyAsync(d.s_face, d_s_face, n_faces * 4, hipMemcpyDeviceToDevice, stream), "copy s");
  LF_TRY(launch_mesh_prep(d, d_faces, stream), "mesh prep");
  if (per_face) LF_TRY(launch_offsets(d, reinterpret_cast<int32_t*>(ws + L.scan), stream), "offsets");
  LF_TRY(launch_cluster_boxes(d, stream), "cluster boxes");
  if (d_accum)
    LF_TRY(launch_zero(d_accum, n_texels * opts->n_classes * (opts->accum_dtype == LF_F32 ? 4 : 2), stream),
           "clear accumulator");
  if (d_wsum) LF_TRY(launch_zero(d_wsum, n_texels * 4, stream), "clear weights");
  int32_t herr = 0;
  int64_t htot = n_texels;
  LF_TRY(hipMemcpyAsync(&herr, d.err, 4, hipMemcpyDeviceToHost, stream), "read flag");
  if (per_face) LF_TRY(hipMemcpyAsync(&htot, d.off + n_faces, 8, hipMemcpyDeviceToHost, stream), "read total");
  LF_TRY(hipStreamSynchronize(stream), "sync");
  if (herr) return fail(LF_EINVAL, "face index out of range [0, %lld) or s < 1", (long long)n_vertices);
  if (htot >= ((int64_t)1 << 31)) return fail(LF_EINVAL, "texel count %lld exceeds 2^31 - 1", (long long)htot);
  if (htot != n_texels) return fail(LF_ESIZE, "n_texels %lld != %lld", (long long)n_texels, (long long)htot);
  lf_mesh h = new (std::nothrow) lf_mesh_s;
  if (!h) return fail(LF_EINVAL, "out of host memory");
  hipError_t he = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking);
  for (int i = 0; i < 2 && he == hipSuccess; ++i) {
    he = hipEventCreateWithFlags(&h->sorted_ev[i], hipEventDisableTiming);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&h->gathered_ev[i], hipEventDisableTiming);
  }
  if (he != hipSuccess) {
    delete h;
    return fail(LF_EHIP, "stream/event creation: %s", hipGetErrorString(he));
  }
  h->magic = kMagic;
  h->d = d;
  h->opts = *opts;
  h->accum_full = d_accum;
  h->wsum_full = d_wsum;
  *out = h;
  return LF_OK;
}

lf_status lf_reset(lf_mesh mesh, hipStream_t stream) {
  g_err[0] = 0;
  lf_status st = check_mesh(mesh);
  if (st != LF_OK) return st;
  StageTimer tm(mesh, 6, stream);
  LF_TRY(launch_zero(mesh->d.accum, mesh->d.n_rows * mesh->d.c * (mesh->d.accum_dtype == LF_F32 ? 4 : 2), stream),
         "clear accumulator");
  if (mesh->d.wsum) LF_TRY(launch_zero(mesh->d.wsum, mesh->d.n_rows * 4, stream), "clear weights");
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

}  // extern "C"

namespace {

// Everything lf_fuse_frames checks, plus the input pool (0 = none).
struct FuseArgs {
  lf_mesh mesh;
  const float* cams;
  int32_t F, H, W;
  const void* probs;
  int32_t dtype;
  const int64_t* strides;
  const float* scale;
  const uint8_t* valid;
  int32_t pool;
  int32_t weighting;
  int32_t* l_out;
  int32_t batch, scatter_mode;
  bool one_stream = false;   // gathers (and staging) on the call's stream even when the mesh overlaps
};

// Resolved scatter mode (AUTO -> SORTED iff classes are contiguous) and the
// frame layout the call needs.
bool stage_ok(const MeshDev& d, int32_t dtype) { return dtype == LF_F32 && d.c % 4 == 0 && d.c <= 60; }

int resolve_mode(const FuseArgs& a) {
  if (a.scatter_mode != LF_SCATTER_AUTO) return a.scatter_mode;
  if (a.strides[1] == 1) return LF_SCATTER_SORTED;
  return stage_ok(a.mesh->d, a.dtype) ? LF_SCATTER_STAGED : LF_SCATTER_ATOMIC;
}

// Whether the sorted path of these arguments gathers with the grouped gather:
// 1 yes, 0 no (the per-class gather), -1 not known (no input pointer given:
// room for both).
int fuse_grouped(const FuseArgs& a, int mode) {
  if (mode != LF_SCATTER_SORTED && mode != LF_SCATTER_STAGED) return 0;
  const MeshDev& d = a.mesh->d;
  if (mode == LF_SCATTER_STAGED) {
    // staged rows: 256-byte aligned workspace, c floats per pixel
    const int64_t c = d.c;
    const ProbIn st{reinterpret_cast<const void*>(uintptr_t(256)), nullptr, nullptr, (int64_t)a.H * a.W * c, 1,
                    (int64_t)a.W * c, c, LF_F32};
    return seg_grouped_ok(d, st) ? 1 : 0;
  }
  if (!a.probs) return -1;
  const ProbIn in{a.probs, a.scale, a.valid, a.strides[0], a.strides[1], a.strides[2], a.strides[3], a.dtype};
  return seg_grouped_ok(d, in) ? 1 : 0;
}

FrameLayout fuse_layout(const FuseArgs& a) {
  const int B = a.batch < a.F ? a.batch : a.F;
  const int mode = resolve_mode(a);
  return frame_layout(a.mesh->d, a.H, a.W, B > 0 ? B : 1, a.weighting, mode, fuse_grouped(a, mode));
}

lf_status check_fuse(const FuseArgs& a, const void* ws, int64_t ws_bytes) {
  lf_status st = check_mesh(a.mesh);
  if (st != LF_OK) return st;
  if ((st = check_frames(a.F, a.H, a.W)) != LF_OK) return st;
  if (a.F == 0) return LF_OK;
  if (!a.cams || !a.probs || !a.strides || !ws) return fail(LF_EINVAL, "NULL argument");
  if (a.dtype != LF_F32 && a.dtype != LF_FP8_E4M3) return fail(LF_EINVAL, "probabilities must be F32 or FP8_E4M3");
  if (a.dtype == LF_FP8_E4M3 && !a.scale) return fail(LF_EINVAL, "FP8 input needs the per-pixel scale");
  if (a.weighting < LF_W_PIXEL || a.weighting > LF_W_MIX) return fail(LF_EINVAL, "unknown weighting %d", a.weighting);
  if (a.weighting == LF_W_LEARNED && !a.mesh->mlp)
    return fail(LF_ESTATE, "learned weighting needs weights bound by lf_mlp_bind");
  if (a.weighting == LF_W_LEARNED && a.mesh->d.n_rows != a.mesh->d.n_texels)
    return fail(LF_ESTATE, "learned weighting needs the whole texture (no texel-row window)");
  if (a.scatter_mode < LF_SCATTER_AUTO || a.scatter_mode > LF_SCATTER_STAGED) return fail(LF_EINVAL, "bad scatter mode");
  if (a.scatter_mode == LF_SCATTER_STAGED && !stage_ok(a.mesh->d, a.dtype))
    return fail(LF_EINVAL, "the staged scatter needs FP32 input, c %% 4 == 0 and c <= 60");
  for (int i = 0; i < 4; ++i)
    if (a.strides[i] < 0) return fail(LF_EINVAL, "negative stride");
  if (a.batch < 1) return fail(LF_EINVAL, "batch must be >= 1");
  if (a.pool < 0) return fail(LF_EINVAL, "negative input pool");
  if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(LF_EINVAL, "workspace must be 256-byte aligned");
  const FrameLayout L = fuse_layout(a);
  if (ws_bytes < L.total) return fail(LF_ESIZE, "frame workspace %lld < %lld bytes", (long long)ws_bytes, (long long)L.total);
  return LF_OK;
}

// The per-batch launch sequence of a checked call.  With an input pool,
// frame f reads input frame f % pool (cameras and outputs stay per frame);
// batches never straddle the end of the pool.
lf_status fuse_impl(const FuseArgs& a, void* d_ws, hipStream_t stream) {
  if (a.F == 0) return LF_OK;
  lf_mesh mesh = a.mesh;
  const MeshDev& d = mesh->d;
  const int B = a.batch < a.F ? a.batch : a.F;
  const int mode = resolve_mode(a);
  const FrameLayout L = fuse_layout(a);
  char* ws = reinterpret_cast<char*>(d_ws);
  const int64_t HW = (int64_t)a.H * a.W;
  const int H = a.H, W = a.W;
  const int64_t* st = a.strides;
  ProbIn in{a.probs, a.scale, a.valid, st[0], st[1], st[2], st[3], a.dtype};
  const bool learned = a.weighting == LF_W_LEARNED;
  float4* geo_sets = learned ? reinterpret_cast<float4*>(ws + L.geo) : nullptr;   // [1 or 2][B][H][W]
  float* wpix_sets = learned ? reinterpret_cast<float*>(ws + L.wpix) : nullptr;   // [1 or 2][B][H][W]
  // the sorted path stores batch-relative element offsets in 32 bits
  const bool staged = mode == LF_SCATTER_STAGED && (int64_t)B * HW * d.c < ((int64_t)1 << 32);
  const bool sorted = staged || (mode == LF_SCATTER_SORTED &&
                                 ((int64_t)(B - 1) * st[0] + (int64_t)(H - 1) * st[2] + (int64_t)(W - 1) * st[3] +
                                  (int64_t)d.c * st[1]) < ((int64_t)1 << 32));
  // staged rows of a batch: frame stride H*W*c, row stride W*c, pixel stride c
  auto staged_in = [&](const void* rows_p, const uint8_t* valid) {
    return ProbIn{rows_p, nullptr, valid, HW * d.c, 1, (int64_t)W * d.c, d.c, LF_F32};
  };
  // w^(I) and the mixed weight on the grouped gather: it counts each row's
  // observations per frame itself, so no per-frame count array is kept
  const bool frame_counts = sorted && (a.weighting == LF_W_IMAGE || a.weighting == LF_W_MIX) &&
                            seg_frame_counts_ok(d, staged ? staged_in(ws + L.stage[0], nullptr) : in, B, H, W);
  // pixels dense in the gather's input: it reads E4M3 scales and the learned
  // weight by pixel index itself, and the fill copies neither
  const bool pix_direct =
      sorted && seg_pixels_dense_ok(d, staged ? staged_in(ws + L.stage[0], nullptr) : in, B, H, W);
  // the grouped gather reads the bucket records; any other layout is sorted by row through memory first
  const bool grouped = sorted && (staged || seg_grouped_ok(d, in));
  // the learned weight inside the grouped gather: features from the
  // observations it streams, n from its per-frame counters, geometry from
  // the resolve (set k of batch k); no count array and no inference pass
  const bool learn_in_gather =
      learned && d.learned_in_gather && grouped && seg_learned_ok(d, staged ? staged_in(ws + L.stage[0], nullptr) : in, B, H, W);
  int32_t* cnt = (a.weighting != LF_W_PIXEL && !frame_counts && !learn_in_gather)
                     ? reinterpret_cast<int32_t*>(ws + L.cnt)
                     : nullptr;
  int32_t* seg = sorted ? reinterpret_cast<int32_t*>(ws + L.seg) : nullptr;
  LF_TRY(launch_zero(ws + L.tcnt, B * L.ntiles * 4, stream), "clear tile counts");
  if (cnt) LF_TRY(launch_zero(cnt, (int64_t)B * d.n_rows * 4, stream), "clear counts");
  int32_t* rank = sorted ? reinterpret_cast<int32_t*>(ws + L.rank) : nullptr;
  lf_status status;
  int nbatch = 0;      // sorted batches issued: batch k's gather runs on `side`
  hipStream_t side = (mesh->overlap && !a.one_stream) ? mesh->side : stream;
  // batches: frames [f0, f0 + nb) read input frames [fi, fi + nb)
  struct Batch {
    int f0, nb, fi;
  };
  auto batch_at = [&](int f0) {
    int nb = (a.F - f0) < B ? (a.F - f0) : B;
    const int fi = a.pool > 0 ? f0 % a.pool : f0;     // input frame of the batch's first frame
    if (a.pool > 0 && nb > a.pool - fi) nb = a.pool - fi;   // batches never straddle the end of the pool
    return Batch{f0, nb, fi};
  };
  // Planar inputs: the side stream transposes each batch into pixel-major
  // rows (staging set j % 2), batch j + 1 while batch j is sorted on the
  // caller's stream; the fill and the gather then read the rows like
  // channels-last input.  Stream order on the side stream protects a set
  // from being rewritten before its gather has read it.
  auto stage_batch = [&](const Batch& b, int j) -> lf_status {
    StageTimer tm(mesh, 3, side);
    LF_TRY(launch_planar_rows(in, b.fi, b.nb, H, W, d.c, reinterpret_cast<float*>(ws + L.stage[j & 1]), side),
           "planar rows");
    return LF_OK;
  };
  if (staged) {
    // the input may come from work on the caller's stream
    LF_TRY(hipEventRecord(mesh->sorted_ev[1], stream), "record call start");
    LF_TRY(hipStreamWaitEvent(side, mesh->sorted_ev[1], 0), "wait for call start");
    if ((status = stage_batch(batch_at(0), 0)) != LF_OK) return status;
  }
  int j = 0;
  for (Batch cur = batch_at(0); cur.f0 < a.F; cur = batch_at(cur.f0 + cur.nb), ++j) {
    const int f0 = cur.f0, nb = cur.nb, fi = cur.fi;
    const bool more = f0 + nb < a.F;
    const float* cams_in = a.cams + 16 * (int64_t)(f0 - fi);  // camera of input index fi + k is f0 + k
    int32_t* lb = a.l_out ? a.l_out + (int64_t)f0 * HW : reinterpret_cast<int32_t*>(ws + L.l);
    const uint8_t* vb = a.valid ? a.valid + (int64_t)fi * HW : nullptr;
    const int k = nbatch & 1;   // sorted path: buffer set of this batch
    bool cnt_zeroed = false;    // the per-frame counts cleared by the fill
    float4* geo = learned ? geo_sets + (sorted ? (int64_t)k * B * HW : 0) : nullptr;
    // geometry set k may still be read by the gather two batches back
    if (learn_in_gather && nbatch >= 2)
      LF_TRY(hipStreamWaitEvent(stream, mesh->gathered_ev[k], 0), "wait for gather");
    if (seg) LF_TRY(launch_zero(seg, L.n_buckets * 4, stream), "clear bucket counts");
    RasterOut out{lb, nullptr, nullptr, vb, cnt, d.n_rows, seg, rank, geo};
    if ((status = render_batch(mesh, a.cams, f0, nb, H, W, L, ws, out, stream)) != LF_OK) return status;
    float* wpix = (learned && !learn_in_gather) ? wpix_sets + (sorted ? (int64_t)k * B * HW : 0) : nullptr;
    if (learned && !learn_in_gather) {
      // weight set k may still be read by the gather two batches back
      if (sorted && nbatch >= 2) LF_TRY(hipStreamWaitEvent(stream, mesh->gathered_ev[k], 0), "wait for gather");
      StageTimer tm(mesh, 7, stream);
      LF_TRY(launch_mlp_weights(mesh->mlp, in, fi, nb, H, W, cams_in, lb, geo, cnt, d.n_rows, d.c, wpix, stream),
             "learned weights");
    }
    if (sorted) {
      int32_t* counts = reinterpret_cast<int32_t*>(ws + L.counts[k]);   // [0] spans, [1] non-empty buckets
      const bool need_w = a.weighting != LF_W_PIXEL && !frame_counts && !(learned && pix_direct);
      const bool need_s = a.dtype == LF_FP8_E4M3 && !pix_direct;
      uint2* rec = reinterpret_cast<uint2*>(ws + L.rec[k]);
      float* rw = need_w ? reinterpret_cast<float*>(ws + L.rec_w[k]) : nullptr;
      float* rs = need_s ? reinterpret_cast<float*>(ws + L.rec_s[k]) : nullptr;
      int32_t* bstart = reinterpret_cast<int32_t*>(ws + L.bstart[k]);
      int32_t* blist = reinterpret_cast<int32_t*>(ws + L.blist[k]);
      float* stg = staged ? reinterpret_cast<float*>(ws + L.stage[k]) : nullptr;
      // the per-class gather reads rows sorted through memory
      int4* spans = grouped ? nullptr : reinterpret_cast<int4*>(ws + L.spans[k]);
      uint32_t* eo = grouped ? nullptr : reinterpret_cast<uint32_t*>(ws + L.ent_off[k]);
      float* ew = (!grouped && need_w) ? reinterpret_cast<float*>(ws + L.ent_w[k]) : nullptr;
      float* es = (!grouped && need_s) ? reinterpret_cast<float*>(ws + L.ent_s[k]) : nullptr;
      // the fill sets the per-frame counts back to zero where it does not
      // read them itself (nothing after it does)
      cnt_zeroed = cnt && !(rw && (a.weighting == LF_W_IMAGE || a.weighting == LF_W_MIX));
      // set k was last read by the gather two batches ago
      if (nbatch >= 2) LF_TRY(hipStreamWaitEvent(stream, mesh->gathered_ev[k], 0), "wait for gather");
      {
        StageTimer tm(mesh, 3, stream);
        LF_TRY(launch_zero(counts, 8, stream), "clear span and bucket counts");
        LF_TRY(launch_seg_scan(seg, L.n_buckets, reinterpret_cast<int32_t*>(ws + L.sums), bstart, blist, counts + 1,
                               stream),
               "bucket scan");
        const ProbIn sin = staged_in(stg, a.valid ? a.valid + (int64_t)fi * HW : nullptr);
        if (staged)
          LF_TRY(launch_seg_fill(sin, 0, nb, H, W, lb, rank, bstart, rec, rw, nullptr, a.weighting, cnt, d.n_rows,
                                 wpix, d.mix, d.win_lo, d.n_rows, cnt_zeroed ? cnt : nullptr, stream),
                 "bucket fill");
        else
          LF_TRY(launch_seg_fill(in, fi, nb, H, W, lb, rank, bstart, rec, rw, rs, a.weighting, cnt, d.n_rows, wpix,
                                 d.mix, d.win_lo, d.n_rows, cnt_zeroed ? cnt : nullptr, stream),
                 "bucket fill");
        if (!grouped)
          LF_TRY(launch_bucket_sort(L.n_buckets, bstart, blist, counts + 1, rec, rw, rs, eo, ew, es, spans, counts,
                                    stream), "bucket sort");
      }
      LF_TRY(hipEventRecord(mesh->sorted_ev[k], stream), "record sorted");
      if (staged && more && (status = stage_batch(batch_at(f0 + nb), j + 1)) != LF_OK) return status;
      LF_TRY(hipStreamWaitEvent(side, mesh->sorted_ev[k], 0), "wait for sort");
      {
        StageTimer tm(mesh, 2, side);
        if (grouped)
          LF_TRY(launch_bucket_gather(d, staged ? staged_in(stg, nullptr) : in, staged ? 0 : fi, H, W, L.n_buckets,
                                      bstart, blist, counts + 1, rec, rw, rs, nb, frame_counts ? a.weighting : 0,
                                      d.mix, (learned && pix_direct) ? wpix : nullptr,
                                      GatherLearn{learn_in_gather ? mesh->mlp : nullptr, geo,
                                                  a.cams + 16 * (int64_t)f0},
                                      side),
                 "bucket gather");
        else
          LF_TRY(launch_seg_gather(d, in, fi, spans, counts, eo, ew, es, side), "segment gather");
      }
      LF_TRY(hipEventRecord(mesh->gathered_ev[k], side), "record gathered");
      ++nbatch;
    } else {
      StageTimer tm(mesh, 2, stream);
      LF_TRY(launch_scatter_atomic(d, in, fi, nb, H, W, lb, a.weighting, cnt, d.n_rows, wpix, d.mix, stream),
             "scatter");
    }
    if (cnt && !cnt_zeroed) {
      StageTimer tm(mesh, 3, stream);
      LF_TRY(launch_clear_counts(lb, vb, nb, H, W, cnt, d.n_rows, d.win_lo, stream), "clear counts");
    }
  }
  // the call is complete on the caller's stream once the last gather is
  if (nbatch > 0) LF_TRY(hipStreamWaitEvent(stream, mesh->gathered_ev[(nbatch - 1) & 1], 0), "join gathers");
  return LF_OK;
}

FuseArgs job_args(const lf_scene_job& j) {
  return FuseArgs{j.mesh, j.d_cams, j.F, j.H, j.W, j.d_probs, j.prob_dtype, j.strides, j.d_scale, j.d_valid,
                  j.pool, j.weighting, j.d_l_out, j.batch, j.scatter_mode};
}

// Lane of every job, the number of lanes used and one lane's workspace bytes.
struct BatchPlan {
  std::vector<int> lane;
  int lanes = 1;
  int64_t lane_bytes = 256;
};

BatchPlan plan_batch(const lf_scene_job* jobs, int32_t n);

lf_status check_jobs(const lf_scene_job* jobs, int32_t n, const void* ws, int64_t ws_bytes) {
  if (n < 0) return fail(LF_EINVAL, "negative job count");
  if (n > 0 && !jobs) return fail(LF_EINVAL, "NULL jobs");
  for (int i = 0; i < n; ++i) {
    lf_status st = check_mesh(jobs[i].mesh);
    if (st != LF_OK) return fail(st, "job %d: invalid mesh handle", i);
  }
  // every lane of the call has its own slice of the workspace
  const BatchPlan plan = plan_batch(jobs, n);
  if (n > 0 && ws_bytes < plan.lanes * plan.lane_bytes)
    return fail(LF_ESIZE, "batch workspace %lld < %lld bytes (%d scene lanes)", (long long)ws_bytes,
                (long long)(plan.lanes * plan.lane_bytes), plan.lanes);
  for (int i = 0; i < n; ++i) {
    const lf_scene_job& j = jobs[i];
    lf_status st = check_fuse(job_args(j), ws, plan.lane_bytes);
    if (st != LF_OK) return fail(st, "job %d: %s", i, std::string(g_err).c_str());
    if (!j.d_labels) return fail(LF_EINVAL, "job %d: labels buffer is NULL", i);
    if (j.d_tex_out && j.tex_dtype != LF_F32 && j.tex_dtype != LF_BF16 && j.tex_dtype != LF_F16)
      return fail(LF_EINVAL, "job %d: bad texture dtype", i);
    if (j.d_images && !j.d_l_out) return fail(LF_EINVAL, "job %d: label images need d_l_out", i);
  }
  return LF_OK;
}

// One job, complete, on `stream` with workspace d_ws.
// one_stream: the scene runs entirely on `stream` (no side-stream overlap
// within the scene: several scene lanes already fill the device).
lf_status run_job(const lf_scene_job& j, void* d_ws, hipStream_t stream, bool one_stream = false) {
  lf_mesh m = j.mesh;
  {
    StageTimer tm(m, 6, stream);
    LF_TRY(launch_zero(m->d.accum, m->d.n_rows * m->d.c * (m->d.accum_dtype == LF_F32 ? 4 : 2), stream),
           "clear accumulator");
    if (m->d.wsum) LF_TRY(launch_zero(m->d.wsum, m->d.n_rows * 4, stream), "clear weights");
  }
  FuseArgs a = job_args(j);
  a.one_stream = one_stream;
  lf_status st = fuse_impl(a, d_ws, stream);
  if (st != LF_OK) return st;
  {
    StageTimer tm(m, 4, stream);
    LF_TRY(launch_finalize(m->d, j.d_tex_out, j.tex_dtype, j.d_labels, stream), "finalize");
  }
  if (j.d_images) {
    StageTimer tm(m, 5, stream);
    const int64_t HW = (int64_t)j.H * j.W;
    // with an input pool, frame f's validity is input frame f % pool's
    const int chunk = j.pool > 0 ? j.pool : j.F;
    for (int f0 = 0; f0 < j.F; f0 += chunk) {
      const int nf = std::min(chunk, j.F - f0);
      LF_TRY(launch_render(j.d_l_out + f0 * HW, j.d_valid, j.d_labels, nf * HW, j.d_images + f0 * HW, stream),
             "render");
    }
  }
  return LF_OK;
}

// ---- many scenes at once: scene lanes ---------------------------------------------
// The jobs of one batched call run on up to kBatchLanes streams of the
// library at once (forked from and joined back into the caller's stream with
// events): the kernels of small scenes then fill the compute units that a
// large scene's latency-bound kernels leave idle.  With several lanes a
// scene runs on its lane's stream alone (no second stream per scene for the
// gathers: the lanes already overlap one scene's gathers with another's
// raster, and the extra streams cost more than they hide).  Jobs on one mesh
// share a lane (in call order); meshes are dealt to lanes largest first,
// each to the lane with the least work (frames x pixels).  Every lane has
// its own slice of the workspace.
constexpr int kBatchLanes = 4;

struct LanePool {
  hipStream_t s[kBatchLanes] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kBatchLanes] = {};
};
std::mutex g_lane_mu;                 // held while a batched call enqueues its work
LanePool g_lanes[64];                 // per device

lf_status lane_pool(LanePool** out) {
  int dev = -1;
  LF_TRY(hipGetDevice(&dev), "current device");
  if (dev < 0 || dev >= 64) return fail(LF_EINVAL, "device ordinal %d beyond the lane table", dev);
  LanePool& p = g_lanes[dev];
  if (!p.fork) {
    for (int l = 0; l < kBatchLanes; ++l) {
      LF_TRY(hipStreamCreateWithFlags(&p.s[l], hipStreamNonBlocking), "lane stream");
      LF_TRY(hipEventCreateWithFlags(&p.join[l], hipEventDisableTiming), "lane event");
    }
    LF_TRY(hipEventCreateWithFlags(&p.fork, hipEventDisableTiming), "lane event");
  }
  *out = &p;
  return LF_OK;
}

BatchPlan plan_batch(const lf_scene_job* jobs, int32_t n) {
  BatchPlan p;
  p.lane.assign(n, 0);
  std::vector<lf_mesh> meshes;
  std::vector<double> work;
  std::vector<int> mesh_of(n);
  for (int i = 0; i < n; ++i) {
    int k = 0;
    while (k < (int)meshes.size() && meshes[k] != jobs[i].mesh) ++k;
    if (k == (int)meshes.size()) {
      meshes.push_back(jobs[i].mesh);
      work.push_back(0.0);
    }
    mesh_of[i] = k;
    work[k] += (double)jobs[i].F * jobs[i].H * jobs[i].W;
    p.lane_bytes = std::max(p.lane_bytes, align256(fuse_layout(job_args(jobs[i])).total));
  }
  p.lanes = std::max(1, std::min<int>(kBatchLanes, (int)meshes.size()));
  std::vector<int> order(meshes.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
  std::vector<double> load(p.lanes, 0.0);
  std::vector<int> lane_of_mesh(meshes.size(), 0);
  for (int k : order) {
    const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    lane_of_mesh[k] = l;
    load[l] += work[k];
  }
  for (int i = 0; i < n; ++i) p.lane[i] = lane_of_mesh[mesh_of[i]];
  return p;
}

lf_status run_jobs(const lf_scene_job* jobs, int32_t n, void* d_ws, hipStream_t stream) {
  if (n <= 0) return LF_OK;
  const BatchPlan plan = plan_batch(jobs, n);
  char* ws = reinterpret_cast<char*>(d_ws);
  if (plan.lanes == 1) {
    for (int i = 0; i < n; ++i) {
      lf_status st = run_job(jobs[i], ws, stream);
      if (st != LF_OK) return st;
    }
    return LF_OK;
  }
  std::lock_guard<std::mutex> lock(g_lane_mu);
  LanePool* lp = nullptr;
  lf_status st = lane_pool(&lp);
  if (st != LF_OK) return st;
  LF_TRY(hipEventRecord(lp->fork, stream), "fork");
  for (int l = 0; l < plan.lanes; ++l) LF_TRY(hipStreamWaitEvent(lp->s[l], lp->fork, 0), "lane start");
  for (int i = 0; i < n; ++i) {
    const int l = plan.lane[i];
    if ((st = run_job(jobs[i], ws + (int64_t)l * plan.lane_bytes, lp->s[l], true)) != LF_OK) return st;
  }
  for (int l = 0; l < plan.lanes; ++l) {
    LF_TRY(hipEventRecord(lp->join[l], lp->s[l]), "lane end");
    LF_TRY(hipStreamWaitEvent(stream, lp->join[l], 0), "join");
  }
  return LF_OK;
}

}  // namespace

// One executable graph per scene lane: a launch forks the caller's stream
// into the lane streams, replays every lane's graph on its own lane, and
// joins them back.
struct lf_graph_s {
  std::vector<hipGraph_t> graph;
  std::vector<hipGraphExec_t> exec;
};

extern "C" {

lf_status lf_fuse_frames(lf_mesh mesh, const float* d_cams, int32_t F, int32_t H, int32_t W, const void* d_probs,
                         int32_t prob_dtype, const int64_t* h_strides, const float* d_scale, const uint8_t* d_valid,
                         int32_t weighting, int32_t* d_l_out, void* d_ws, int64_t ws_bytes, int32_t batch,
                         int32_t scatter_mode, hipStream_t stream) {
  g_err[0] = 0;
  const FuseArgs a{mesh, d_cams, F, H, W, d_probs, prob_dtype, h_strides, d_scale, d_valid, 0, weighting, d_l_out,
                   batch, scatter_mode};
  lf_status st = check_fuse(a, d_ws, ws_bytes);
  if (st != LF_OK) return st;
  return fuse_impl(a, d_ws, stream);
}

}  // extern "C"

// ---- Fusion through the library's own static scratch (no allocation) -------
// One fixed-size device array per GPU takes the place of the caller's frame
// workspace.  Host code never passes the array's name to a kernel: on the
// host it is only a stand-in, so each device's address is looked up once
// (with that device current) and kept in g_scratch_ptr.
namespace {
static __device__ __align__(256) char scratch[LF_NOALLOC_SCRATCH_BYTES];
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

lf_status scratch_of_current_device(void** out) {
  int dev = -1;
  LF_TRY(hipGetDevice(&dev), "current device");
  if (dev < 0 || dev >= kScratchDevices) return fail(LF_EINVAL, "device ordinal %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    LF_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch address");
    if (!p) return fail(LF_EHIP, "scratch address of device %d is NULL", dev);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LF_OK;
}
}  // namespace

extern "C" {

lf_status lf_fuse_frames_noalloc(lf_mesh mesh, const float* d_cams, int32_t F, int32_t H, int32_t W,
                                 const void* d_probs, int32_t prob_dtype, const int64_t* h_strides,
                                 const float* d_scale, const uint8_t* d_valid, int32_t weighting, int32_t* d_l_out,
                                 int32_t batch, int32_t scatter_mode, hipStream_t stream) {
  g_err[0] = 0;
  const FuseArgs a{mesh, d_cams, F, H, W, d_probs, prob_dtype, h_strides, d_scale, d_valid, 0, weighting, d_l_out,
                   batch, scatter_mode};
  void* ws = nullptr;
  lf_status st = scratch_of_current_device(&ws);
  if (st != LF_OK) return st;
  st = check_fuse(a, ws, LF_NOALLOC_SCRATCH_BYTES);
  if (st == LF_ESIZE)
    return fail(LF_ESIZE, "this call needs %lld bytes of frame workspace; the static scratch holds %lld "
                "(use a smaller batch, or lf_fuse_frames with a caller workspace)",
                (long long)fuse_layout(a).total, (long long)LF_NOALLOC_SCRATCH_BYTES);
  if (st != LF_OK) return st;
  return fuse_impl(a, ws, stream);
}

lf_status lf_area_ws_bytes(lf_mesh mesh, int32_t H, int32_t W, int32_t batch, int64_t* bytes) {
  g_err[0] = 0;
  lf_status st = check_mesh(mesh);
  if (st != LF_OK) return st;
  if ((st = check_frames(1, H, W)) != LF_OK) return st;
  if (batch < 1 || batch > 65535) return fail(LF_EINVAL, "batch must be in [1, 65535]");
  if (bytes)
    *bytes = frame_layout(mesh->d, H, W, batch, LF_W_PIXEL, LF_SCATTER_ATOMIC).total +
             align256((int64_t)batch * std::max<int64_t>(mesh->d.T, 1) * 4);
  return LF_OK;
}

lf_status lf_triangle_max_pixels(lf_mesh mesh, const float* d_cams, int32_t F, int32_t H, int32_t W, int32_t* d_area,
                                 void* d_ws, int64_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  lf_status st = check_mesh(mesh);
  if (st != LF_OK) return st;
  if ((st = check_frames(F, H, W)) != LF_OK) return st;
  if (F == 0 || mesh->d.T == 0) return LF_OK;
  if (!d_cams || !d_area || !d_ws) return fail(LF_EINVAL, "NULL argument");
  if (reinterpret_cast<uintptr_t>(d_ws) & 255) return fail(LF_EINVAL, "workspace must be 256-byte aligned");
  const MeshDev& d = mesh->d;
  auto total = [&](int b) {
    return frame_layout(d, H, W, b, LF_W_PIXEL, LF_SCATTER_ATOMIC).total + align256((int64_t)b * d.T * 4);
  };
  int B = 1;
  while (B < F && B < 64 && total(B * 2) <= ws_bytes) B *= 2;
  if (B > F) B = F;
  if (ws_bytes < total(B)) return fail(LF_ESIZE, "workspace %lld < %lld bytes", (long long)ws_bytes, (long long)total(B));
  const FrameLayout L = frame_layout(d, H, W, B, LF_W_PIXEL, LF_SCATTER_ATOMIC);
  char* ws = reinterpret_cast<char*>(d_ws);
  int32_t* tri = reinterpret_cast<int32_t*>(ws + L.l);
  int32_t* tricnt = reinterpret_cast<int32_t*>(ws + L.total);
  LF_TRY(launch_zero(ws + L.tcnt, B * L.ntiles * 4, stream), "clear tile counts");
  LF_TRY(launch_zero(tricnt, (int64_t)B * d.T * 4, stream), "clear triangle counts");
  for (int f0 = 0; f0 < F; f0 += B) {
    const int nb = (F - f0) < B ? (F - f0) : B;
    RasterOut out{nullptr, tri, nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr, tricnt};
    if ((st = render_batch(mesh, d_cams, f0, nb, H, W, L, ws, out, stream)) != LF_OK) return st;
    LF_TRY(launch_area_max(tri, nb, H, W, tricnt, d.T, d_area, stream), "area max");
  }
  return LF_OK;
}

lf_status lf_texel_resolution(const int32_t* d_area, int64_t n_faces, float gamma, int32_t* d_s_face,
                              hipStream_t stream) {
  g_err[0] = 0;
  if (n_faces < 0) return fail(LF_EINVAL, "negative face count");
  if (!(gamma >= 0.0f) || gamma > 1e6f) return fail(LF_EINVAL, "gamma must be in [0, 1e6]");
  if (n_faces == 0) return LF_OK;
  if (!d_area || !d_s_face) return fail(LF_EINVAL, "NULL argument");
  LF_TRY(launch_texel_resolution(d_area, n_faces, gamma, d_s_face, stream), "texel resolution");
  return LF_OK;
}

lf_status lf_fuse_ws_bytes(lf_mesh mesh, int32_t H, int32_t W, int32_t batch, int32_t weighting,
                           int32_t scatter_mode, int32_t prob_dtype, const int64_t* h_strides, int64_t* bytes) {
  g_err[0] = 0;
  lf_status st = check_mesh(mesh);
  if (st != LF_OK) return st;
  if ((st = check_frames(1, H, W)) != LF_OK) return st;
  if (batch < 1 || batch > 65535) return fail(LF_EINVAL, "batch must be in [1, 65535]");
  if (!h_strides) return fail(LF_EINVAL, "NULL strides");
  const FuseArgs a{mesh, nullptr, batch, H, W, nullptr, prob_dtype, h_strides, nullptr, nullptr, 0, weighting,
                   nullptr, batch, scatter_mode};
  if (bytes) *bytes = fuse_layout(a).total;
  return LF_OK;
}

lf_status lf_batch_ws_bytes(const lf_scene_job* jobs, int32_t n, int64_t* bytes) {
  g_err[0] = 0;
  if (n < 0 || (n > 0 && !jobs)) return fail(LF_EINVAL, "bad job list");
  for (int i = 0; i < n; ++i) {
    lf_status st = check_mesh(jobs[i].mesh);
    if (st != LF_OK) return fail(st, "job %d: invalid mesh handle", i);
    if ((st = check_frames(jobs[i].F, jobs[i].H, jobs[i].W)) != LF_OK) return st;
    if (jobs[i].batch < 1) return fail(LF_EINVAL, "job %d: batch must be >= 1", i);
  }
  const BatchPlan plan = plan_batch(jobs, n);
  if (bytes) *bytes = plan.lanes * plan.lane_bytes;
  return LF_OK;
}

lf_status lf_fuse_batch(const lf_scene_job* jobs, int32_t n, void* d_ws, int64_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  lf_status st = check_jobs(jobs, n, d_ws, ws_bytes);
  if (st != LF_OK) return st;
  return run_jobs(jobs, n, d_ws, stream);
}

lf_status lf_graph_capture_batch(const lf_scene_job* jobs, int32_t n, void* d_ws, int64_t ws_bytes,
                                 hipStream_t stream, lf_graph* out) {
  g_err[0] = 0;
  if (!out) return fail(LF_EINVAL, "NULL graph handle pointer");
  *out = nullptr;
  if (!stream) return fail(LF_EINVAL, "capture needs a non-default stream");
  lf_status st = check_jobs(jobs, n, d_ws, ws_bytes);
  if (st != LF_OK) return st;
  for (int i = 0; i < n; ++i)
    if (jobs[i].mesh->prof.on) return fail(LF_ESTATE, "job %d: turn profiling off before capturing", i);
  const BatchPlan plan = plan_batch(jobs, n);
  lf_graph h = new (std::nothrow) lf_graph_s;
  if (!h) return fail(LF_EINVAL, "out of host memory");
  // on one lane the caller's stream is captured; with several, every lane's
  // jobs on its own lane stream
  std::unique_lock<std::mutex> lock(g_lane_mu, std::defer_lock);
  LanePool* lp = nullptr;
  if (plan.lanes > 1) {
    lock.lock();
    if ((st = lane_pool(&lp)) != LF_OK) {
      delete h;
      return st;
    }
  }
  char* ws = reinterpret_cast<char*>(d_ws);
  for (int l = 0; l < plan.lanes && st == LF_OK; ++l) {
    hipStream_t ls = plan.lanes > 1 ? lp->s[l] : stream;
    hipError_t e = hipStreamBeginCapture(ls, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      st = fail(LF_EHIP, "begin capture: %s", hipGetErrorString(e));
      break;
    }
    for (int i = 0; i < n && st == LF_OK; ++i)
      if (plan.lane[i] == l) st = run_job(jobs[i], ws + (int64_t)l * plan.lane_bytes, ls, plan.lanes > 1);
    hipGraph_t lg = nullptr;
    e = hipStreamEndCapture(ls, &lg);
    if (st == LF_OK && e != hipSuccess) st = fail(LF_EHIP, "end capture: %s", hipGetErrorString(e));
    if (lg) h->graph.push_back(lg);
    if (st == LF_OK) {
      hipGraphExec_t x = nullptr;
      e = hipGraphInstantiate(&x, lg, nullptr, nullptr, 0);
      if (e != hipSuccess) st = fail(LF_EHIP, "instantiate: %s", hipGetErrorString(e));
      else h->exec.push_back(x);
    }
  }
  if (lock.owns_lock()) lock.unlock();
  if (st != LF_OK) {
    lf_graph_free(h);
    return st;
  }
  *out = h;
  return LF_OK;
}

lf_status lf_graph_launch(lf_graph g, hipStream_t stream) {
  g_err[0] = 0;
  if (!g || g->exec.empty()) return fail(LF_ESTATE, "invalid graph handle");
  if (g->exec.size() == 1) {
    LF_TRY(hipGraphLaunch(g->exec[0], stream), "graph launch");
    return LF_OK;
  }
  std::lock_guard<std::mutex> lock(g_lane_mu);
  LanePool* lp = nullptr;
  lf_status st = lane_pool(&lp);
  if (st != LF_OK) return st;
  LF_TRY(hipEventRecord(lp->fork, stream), "fork");
  for (size_t l = 0; l < g->exec.size(); ++l) {
    LF_TRY(hipStreamWaitEvent(lp->s[l], lp->fork, 0), "lane start");
    LF_TRY(hipGraphLaunch(g->exec[l], lp->s[l]), "graph launch");
    LF_TRY(hipEventRecord(lp->join[l], lp->s[l]), "lane end");
    LF_TRY(hipStreamWaitEvent(stream, lp->join[l], 0), "join");
  }
  return LF_OK;
}

void lf_graph_free(lf_graph g) {
  if (!g) return;
  for (hipGraphExec_t x : g->exec) (void)hipGraphExecDestroy(x);
  for (hipGraph_t x : g->graph) (void)hipGraphDestroy(x);
  delete g;
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

lf_status lf_set_tuning(lf_mesh mesh, const lf_tuning* t) {
  g_err[0] = 0;
  lf_status st = check_mesh(mesh);
  if (st != LF_OK) return st;
  if (!t) return fail(LF_EINVAL, "NULL tuning");
  if (t->tile != 16 && t->tile != 32) return fail(LF_EINVAL, "tile must be 16 or 32, got %d", t->tile);
  if (t->gather_unroll != 4 && t->gather_unroll != 8)
    return fail(LF_EINVAL, "gather_unroll must be 4 or 8, got %d", t->gather_unroll);
  if (t->small_px < 1 || t->small_px > 1024) return fail(LF_EINVAL, "small_px must be in [1, 1024], got %d", t->small_px);
  if (t->gather_waves < 1 || t->gather_waves > 1024)
    return fail(LF_EINVAL, "gather_waves must be in [1, 1024], got %d", t->gather_waves);
  if (t->learned_in_gather != 0 && t->learned_in_gather != 1)
    return fail(LF_EINVAL, "learned_in_gather must be 0 or 1, got %d", t->learned_in_gather);
  mesh->d.small_px = t->small_px;
  mesh->d.learned_in_gather = t->learned_in_gather;
  mesh->d.gather_waves = t->gather_waves;
  mesh->d.tile = t->tile;
  mesh->d.gather_unroll = t->gather_unroll;
  return LF_OK;
}

lf_status lf_set_overlap(lf_mesh mesh, int32_t enabled) {
  g_err[0] = 0;
  lf_status st = check_mesh(mesh);
  if (st != LF_OK) return st;
  mesh->overlap = enabled != 0;
  return LF_OK;
}

lf_status lf_set_window(lf_mesh mesh, int64_t row_lo, int64_t n_rows, void* d_accum, float* d_wsum) {
  g_err[0] = 0;
  lf_status st = check_mesh(mesh);
  if (st != LF_OK) return st;
  MeshDev& d = mesh->d;
  if (row_lo < 0 || n_rows < 0 || row_lo + n_rows > d.n_texels)
    return fail(LF_EINVAL, "window [%lld, %lld) outside [0, %lld)", (long long)row_lo, (long long)(row_lo + n_rows),
                (long long)d.n_texels);
  if (!d_accum) {
    if (row_lo != 0 || n_rows != d.n_texels || d_wsum)
      return fail(LF_EINVAL, "a window other than the whole texture needs its own accumulator");
    if (!mesh->accum_full && n_rows > 0)
      return fail(LF_ESTATE, "the mesh was loaded without a whole-texture accumulator");
    d.accum = mesh->accum_full;
    d.wsum = mesh->wsum_full;
  } else {
    if (d.aggregator == LF_AGG_MUL && !d_wsum) return fail(LF_EINVAL, "MUL aggregation needs the weight-sum buffer");
    if (reinterpret_cast<uintptr_t>(d_accum) & 15) return fail(LF_EINVAL, "window accumulator must be 16-byte aligned");
    d.accum = d_accum;
    d.wsum = d_wsum;
  }
  d.win_lo = row_lo;
  d.n_rows = n_rows;
  return LF_OK;
}

lf_status lf_set_weight_mix(lf_mesh mesh, float alpha) {
  g_err[0] = 0;
  lf_status st = check_mesh(mesh);
  if (st != LF_OK) return st;
  if (!(alpha >= 0.0f && alpha <= 1.0f)) return fail(LF_EINVAL, "alpha must be in [0, 1]");
  mesh->d.mix = alpha;
  return LF_OK;
}

lf_status lf_get_tuning(lf_mesh mesh, lf_tuning* t) {
  g_err[0] = 0;
  lf_status st = check_mesh(mesh);
  if (st != LF_OK) return st;
  if (!t) return fail(LF_EINVAL, "NULL tuning");
  t->tile = mesh->d.tile;
  t->gather_unroll = mesh->d.gather_unroll;
  t->small_px = mesh->d.small_px;
  t->gather_waves = mesh->d.gather_waves;
  t->learned_in_gather = mesh->d.learned_in_gather;
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
  if (mesh->d.n_rows != mesh->d.n_texels)
    return fail(LF_ESTATE, "feature extraction needs the whole texture (no texel-row window)");
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
    LF_TRY(launch_clear_counts(lb, vb, nb, H, W, cnt, d.n_texels, 0, stream), "clear counts");
  }
  return LF_OK;
}

lf_status lf_label_agreement(const void* d_probs, int32_t prob_dtype, const int64_t* h_strides, const float* d_scale,
                             const uint8_t* d_valid, int32_t n_classes, int32_t F, int32_t H, int32_t W,
                             const uint8_t* d_images, uint64_t* d_counts, hipStream_t stream) {
  g_err[0] = 0;
  lf_status st = check_frames(F, H, W);
  if (st != LF_OK) return st;
  if (!d_counts) return fail(LF_EINVAL, "NULL counts");
  if (n_classes < 1 || n_classes > 255) return fail(LF_EINVAL, "n_classes must be in [1, 255]");
  if (F == 0) return LF_OK;
  if (!d_probs || !h_strides || !d_images) return fail(LF_EINVAL, "NULL argument");
  if (prob_dtype != LF_F32 && prob_dtype != LF_FP8_E4M3) return fail(LF_EINVAL, "probabilities must be F32 or FP8_E4M3");
  if (prob_dtype == LF_FP8_E4M3 && !d_scale) return fail(LF_EINVAL, "FP8 input needs the per-pixel scale");
  for (int i = 0; i < 4; ++i)
    if (h_strides[i] < 0) return fail(LF_EINVAL, "negative stride");
  ProbIn in{d_probs, d_scale, d_valid, h_strides[0], h_strides[1], h_strides[2], h_strides[3], prob_dtype};
  LF_TRY(launch_agreement(in, n_classes, F, H, W, d_images, reinterpret_cast<unsigned long long*>(d_counts), stream),
         "agreement");
  return LF_OK;
}

void lf_free_mesh(lf_mesh mesh) {
  if (mesh && mesh->magic == kMagic) {
    mesh->magic = 0;
    delete mesh;
  }
}

}  // extern "C"
