// Texel-sorted aggregation (Sections 3.2.1, 3.2.2, 3.3.2) without floating
// point atomics: every batch of frames is counting-sorted by texel row, then
// a group of lanes owns each touched row and adds all of the batch's
// observations of it in registers before a single read-modify-write of the
// row.  The sort has two levels, so that every pass over the batch's pixels
// reads and writes contiguous runs:
//   (resolve)     every pixel counted in its bucket of 2^kBucketShift
//                 consecutive texel rows, with its rank in the bucket (one
//                 atomic per run of same-bucket pixels of a wave);
//   k_seg_scan*   exclusive scan of the bucket counts -> bucket starts and
//                 the list of non-empty buckets;
//   k_seg_fill    every valid covered pixel writes, at its bucket's start
//                 plus its rank, a record of the element offset of its
//                 class-0 value and its row within the bucket (and, where the
//                 gather cannot find them itself, its weight and FP8 scale);
//   (second level) the records of every bucket ordered by row:
//   k_bucket_gather16  contiguous classes (c <= 64, c % 4 == 0): one
//                 workgroup per bucket sorts its records by row in LDS, then
//                 16 lanes per row (4 classes each) stream the row's
//                 observations, sum w * f(p) in registers and update the row
//                 once (with the learned weight, the workgroup first
//                 evaluates the network for every record of the bucket);
//   k_bucket_sort + k_seg_gather  any other layout: the buckets' records
//                 sorted by row through memory (one span (row, start, end)
//                 per touched row), then one wave per 64 touched rows,
//                 lanes = classes (any c, any strides);
//   k_planar_rows planar (NCHW) frames transposed to pixel-major rows first.
// Rows touched by many frames of a batch are read and written once per
// batch instead of once per pixel.
#include <algorithm>

#include "accum.h"
#include <type_traits>

#include "internal.h"
#include "mlp.h"
#include "spec.h"

namespace lf {

// ---- scan of the segment counts ------------------------------------------------
constexpr int kSegChunk = 8192;   // rows per scan block (256 threads x 32)

__global__ __launch_bounds__(256) void k_seg_sums(const int32_t* __restrict__ cnt, int64_t n, int32_t* __restrict__ sums) {
  __shared__ int red[256];
  const int64_t base = (int64_t)blockIdx.x * kSegChunk;
  int acc = 0;
  for (int i = threadIdx.x; i < kSegChunk; i += 256) {
    const int64_t r = base + i;
    if (r < n) acc += cnt[r];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(1024) void k_seg_scan_sums(int32_t* __restrict__ sums, int64_t nblk) {
  __shared__ int part[1024];
  int carry = 0;
  for (int64_t base = 0; base < nblk; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const int v = i < nblk ? sums[i] : 0;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
      const int a = threadIdx.x >= d ? part[threadIdx.x - d] : 0;
      __syncthreads();
      part[threadIdx.x] += a;
      __syncthreads();
    }
    if (i < nblk) sums[i] = carry + part[threadIdx.x] - v;
    carry += part[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[nblk] = carry;
}

// Also appends every row with observations to a compact list (one global
// atomic per block) so the gather visits only touched rows.  A thread scans
// 32 consecutive rows; the block's counts and starts pass through LDS
// (padded rows of 33 words: conflict-free both ways) so that the global
// reads and writes are coalesced.
constexpr int kSegPer = kSegChunk / 256;   // rows per thread
constexpr int kSegPad = kSegPer + 1;

__global__ __launch_bounds__(256) void k_seg_scan(const int32_t* __restrict__ cnt, int64_t n,
                                                  const int32_t* __restrict__ sums, int32_t* __restrict__ start,
                                                  int32_t* __restrict__ rows, int32_t* __restrict__ nrows) {
  __shared__ int sv[256 * kSegPad];
  __shared__ int part[256];
  __shared__ int zpart[256];
  __shared__ int zbase;
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kSegChunk;
  // element e of the chunk sits at (e / 32) * 33 + e % 32
#pragma unroll 8
  for (int i = 0; i < kSegPer; ++i) {
    const int e = i * 256 + t;
    const int64_t r = base + e;
    sv[(e >> 5) * kSegPad + (e & 31)] = r < n ? cnt[r] : 0;
  }
  __syncthreads();
  int* my = sv + t * kSegPad;   // this thread's rows base + 32 t ...
  int acc = 0;
  int nz = 0;
#pragma unroll 8
  for (int i = 0; i < kSegPer; ++i) {
    const int v = my[i];
    acc += v;
    nz += v > 0;
  }
  part[t] = acc;
  zpart[t] = nz;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {
    const int a = t >= d ? part[t - d] : 0;
    const int b = t >= d ? zpart[t - d] : 0;
    __syncthreads();
    part[t] += a;
    zpart[t] += b;
    __syncthreads();
  }
  if (t == 255) zbase = atomicAdd(nrows, zpart[255]);
  __syncthreads();
  int run = sums[blockIdx.x] + part[t] - acc;
  int zpos = zbase + zpart[t] - nz;
  const int64_t r0 = base + (int64_t)t * kSegPer;
#pragma unroll 8
  for (int i = 0; i < kSegPer; ++i) {
    const int v = my[i];
    my[i] = run;                                   // exclusive start of the row
    run += v;
    if (v > 0) rows[zpos++] = (int32_t)(r0 + i);   // v > 0 only for rows below n
  }
  __syncthreads();
#pragma unroll 8
  for (int i = 0; i < kSegPer; ++i) {
    const int e = i * 256 + t;
    const int64_t r = base + e;
    if (r < n) start[r] = sv[(e >> 5) * kSegPad + (e & 31)];
  }
  if (blockIdx.x == gridDim.x - 1 && t == 0) start[n] = sums[gridDim.x];
}

// ---- fill ------------------------------------------------------------------------
// 4 pixels per thread; every phase is issued for all 4 before the next so
// the dependent loads (row, then its bucket's start) overlap.  Pixels of one
// run of the resolve have consecutive ranks, so a wave's record stores are
// contiguous.  Workgroups are dealt to the 8 XCDs in turn and the grid's
// width is a multiple of 8, so block x runs on XCD x % 8; it takes pixel
// chunk (x % 8) * (width / 8) + x / 8, which gives every XCD one band of
// image rows in every frame.
constexpr int kBucketMask = (1 << kBucketShift) - 1;

__global__ __launch_bounds__(256) void k_seg_fill(ProbIn in, int f_first, int H, int W, const int32_t* __restrict__ lbuf,
                                                  const int32_t* __restrict__ rank, const int32_t* __restrict__ bstart,
                                                  uint2* __restrict__ rec, float* __restrict__ rec_w,
                                                  float* __restrict__ rec_s, int weighting,
                                                  const int32_t* __restrict__ cnt, int64_t cnt_stride,
                                                  const float* __restrict__ wpix, float mix, int64_t win_lo,
                                                  int64_t n_rows, int32_t* __restrict__ cnt_zero) {
  constexpr int P = 4;
  const int fb = blockIdx.y;
  const int64_t HW = (int64_t)H * W;
  int l[P], st[P];
  int64_t p[P];
  bool ok[P];
  const int64_t chunk = (int64_t)(blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
#pragma unroll
  for (int k = 0; k < P; ++k) {
    p[k] = (chunk * P + k) * 256 + threadIdx.x;
    ok[k] = p[k] < HW;
    // window-relative row (-1: no triangle, invalid, or outside the window)
    const int64_t lw = ok[k] ? (int64_t)lbuf[(int64_t)fb * HW + p[k]] - win_lo : -1;
    l[k] = (lw >= 0 && lw < n_rows) ? (int)lw : -1;
    // the per-frame count of the row is no longer needed: back to zero
    if (cnt_zero && l[k] >= 0) cnt_zero[(int64_t)fb * cnt_stride + l[k]] = 0;
    if (l[k] >= 0 && in.valid && !in.valid[(int64_t)(f_first + fb) * HW + p[k]]) l[k] = -1;
  }
#pragma unroll
  for (int k = 0; k < P; ++k) st[k] = l[k] >= 0 ? bstart[l[k] >> kBucketShift] + rank[(int64_t)fb * HW + p[k]] : 0;
#pragma unroll
  for (int k = 0; k < P; ++k) {
    if (l[k] < 0) continue;
    const int pos = st[k];
    const int y = (int)(p[k] / W), x = (int)(p[k] - (int64_t)y * W);
    rec[pos] = make_uint2((uint32_t)((int64_t)fb * in.sf + (int64_t)y * in.sy + (int64_t)x * in.sx),
                          (uint32_t)(l[k] & kBucketMask));
    if (rec_w) {
      float w = 1.0f;
      if (weighting == 1) w = 1.0f / (float)cnt[(int64_t)fb * cnt_stride + l[k]];
      else if (weighting == 2) w = wpix[(int64_t)fb * HW + p[k]];
      else if (weighting == 3) w = (1.0f - mix) + mix / (float)cnt[(int64_t)fb * cnt_stride + l[k]];
      rec_w[pos] = w;
    }
    if (rec_s) rec_s[pos] = in.scale[(int64_t)(f_first + fb) * HW + p[k]];
  }
}

// ---- second level, through memory: rows within a bucket -------------------------------
// For the per-class gather (any strides): one workgroup per non-empty bucket
// (walking the list): the bucket's records are counted per row in LDS, the
// counts scanned into the rows' segment starts (within the bucket's own range
// of the entry arrays), every touched row appends its span (row, start,
// end), and every record is moved to its row's next free slot.  Within a
// row, entries keep no particular order.
constexpr int kBucketRows = 1 << kBucketShift;
static_assert(kBucketRows <= 64, "one wave scans a bucket's row counts");

__global__ __launch_bounds__(256) void k_bucket_sort(const int32_t* __restrict__ bstart,
                                                     const int32_t* __restrict__ blist,
                                                     const int32_t* __restrict__ nblist, const uint2* __restrict__ rec,
                                                     const float* __restrict__ rec_w, const float* __restrict__ rec_s,
                                                     uint32_t* __restrict__ ent, float* __restrict__ ent_w,
                                                     float* __restrict__ ent_s, int4* __restrict__ spans,
                                                     int32_t* __restrict__ nspans) {
  __shared__ int hist[kBucketRows];
  const int t = threadIdx.x;
  const int nb = *nblist;
  for (int g = blockIdx.x; g < nb; g += gridDim.x) {
    const int b = blist[g];
    const int s0 = bstart[b], s1 = bstart[b + 1];
    if (t < kBucketRows) hist[t] = 0;
    __syncthreads();
    for (int i = s0 + t; i < s1; i += 256) atomicAdd(&hist[rec[i].y & kBucketMask], 1);
    __syncthreads();
    if (t < 64) {
      const int cnt = t < kBucketRows ? hist[t] : 0;
      int incl = cnt, nz = cnt > 0;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int a = __shfl_up(incl, o), z = __shfl_up(nz, o);
        if (t >= o) {
          incl += a;
          nz += z;
        }
      }
      int base = 0;
      if (t == 63) base = atomicAdd(nspans, nz);
      base = __shfl(base, 63);
      if (t < kBucketRows) {
        const int st = s0 + incl - cnt;
        hist[t] = st;                                   // the row's cursor
        if (cnt > 0) spans[base + nz - 1] = make_int4(b * kBucketRows + t, st, st + cnt, 0);
      }
    }
    __syncthreads();
    for (int i = s0 + t; i < s1; i += 256) {
      const uint2 q = rec[i];
      const int d = atomicAdd(&hist[q.y & kBucketMask], 1);
      ent[d] = q.x;
      if (ent_w) ent_w[d] = rec_w[i];
      if (ent_s) ent_s[d] = rec_s[i];
    }
    __syncthreads();                               // hist is cleared for the next bucket
  }
}

// ---- planar inputs: transpose to rows ----------------------------------------------------
// For inputs whose classes are far apart in memory (NCHW), frames are first
// transposed into a staging array of contiguous class vectors (pixel-major,
// c floats per pixel), which the fill and gather then treat like
// channels-last input.  A block takes 128 consecutive pixels of one frame:
// each class plane is read coalesced into LDS (padded rows; every load of a
// thread issued before its LDS stores), then the block's 128 x c floats are
// written out as contiguous float4 runs (c % 4 == 0, c <= 60, FP32; LDS
// sized by c).
constexpr int kStageMaxC = 60;
constexpr int kStagePixels = 128;   // pixels per block (LDS c x 129 floats: several blocks per CU)

template <int PB>
__global__ __launch_bounds__(256) void k_planar_rows(ProbIn in, int f_first, int H, int W, int c,
                                                     float* __restrict__ staging) {
  constexpr int ROW = PB + 1;                               // padded LDS row of one class
  constexpr int K4 = PB / 4;                                // float4 of a plane per block
  constexpr int JS = 256 / K4;                              // planes read per pass of the block
  extern __shared__ float sv[];                             // [c][ROW]
  const int fb = blockIdx.y;
  const int64_t HW = (int64_t)H * W;
  const int t = threadIdx.x;
  const int64_t p0 = (int64_t)blockIdx.x * PB;
  const float* base = reinterpret_cast<const float*>(in.p) + (int64_t)(f_first + fb) * in.sf;
  if (in.sx == 1 && in.sy == W && (HW & 3) == 0 && (in.sc & 3) == 0 && (in.sf & 3) == 0 &&
      (reinterpret_cast<uintptr_t>(in.p) & 15) == 0) {
    // dense planes: float4 loads of 4 consecutive pixels (thread t: pixels
    // 4 (t % K4) .. + 3 of planes t / K4 + JS i), all issued before the LDS
    // stores
    const int n4 = (int)min<int64_t>(K4, (HW - p0) >> 2);
    const int k = t % K4, j0 = t / K4;
    constexpr int NV = (kStageMaxC + JS - 1) / JS;
    float4 v[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int j = j0 + JS * i;
      if (j < c && k < n4) v[i] = *reinterpret_cast<const float4*>(base + (int64_t)j * in.sc + p0 + 4 * k);
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int j = j0 + JS * i;
      if (j < c && k < n4) {
        float* d = sv + j * ROW + 4 * k;
        d[0] = v[i].x; d[1] = v[i].y; d[2] = v[i].z; d[3] = v[i].w;
      }
    }
  } else if (t < PB && p0 + t < HW) {
    const int64_t p = p0 + t;
    const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
    const float* src = base + (int64_t)y * in.sy + (int64_t)x * in.sx;
    float* dst = sv + t;
#pragma unroll 4
    for (int j = 0; j < c; ++j) {
      dst[j * ROW] = *src;
      src += in.sc;
    }
  }
  __syncthreads();
  // output element i (in float4 units) of the block is (row, q) = (i / nq, i % nq): walk it incrementally
  const int nq = c >> 2;
  const int n = (int)min<int64_t>(PB, HW - p0);
  const int drow = 256 / nq, dq = 256 - drow * nq;
  int row = t / nq, q = t - (t / nq) * nq;
  float4* out = reinterpret_cast<float4*>(staging + ((int64_t)fb * HW + p0) * c);
  for (int i = t; i < n * nq; i += 256) {
    const float* col = sv + 4 * q * ROW + row;
    out[i] = make_float4(col[0], col[ROW], col[2 * ROW], col[3 * ROW]);
    row += drow;
    q += dq;
    if (q >= nq) { q -= nq; ++row; }
  }
}

// ---- gather --------------------------------------------------------------------------
template <int DT>
__device__ __forceinline__ float ld_prob(const void* p, int64_t e) {
  if constexpr (DT == 0) return reinterpret_cast<const float*>(p)[e];
  else return fp8_e4m3(reinterpret_cast<const uint8_t*>(p)[e]);
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// Compensated (Kahan) addition of x to the running sum s, its rounding error
// carried in c (the sum is s - c): the error of a row's sum then stays within
// about 2 * 2^-24 of the sum of magnitudes however many observations the row
// has, where a plain running sum drifts with their number (a texel seen by
// tens of thousands of pixels in a batch).  Finite terms only.
__device__ __forceinline__ void kahan_add(float& s, float& c, float x) {
  const float y = x - c;
  const float t = s + y;
  c = (t - s) - y;
  s = t;
}

// SUM and MAXSUM rows are summed with compensation; MUL rows (sums of logs,
// which may be -inf) with plain additions.
template <int NCH, int DT, int AGG>
__device__ __forceinline__ void accumulate(float (&acc)[NCH], float (&cmp)[NCH], const float (&v)[NCH], float w,
                                           int lane, int c) {
  if constexpr (AGG == 0) {
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) kahan_add(acc[ch], cmp[ch], w * v[ch]);
  } else if constexpr (AGG == 1) {
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) acc[ch] += w * logf(v[ch]);
  } else {
    float mx = -__builtin_inff();
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) mx = fmaxf(mx, (lane + 64 * ch < c) ? v[ch] : -__builtin_inff());
    mx = wave_max(mx);
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) kahan_add(acc[ch], cmp[ch], w * ((v[ch] == mx) ? v[ch] : 0.0f));
  }
}

constexpr int kGatherUnroll = 8;   // observations in flight per wave

// Element offset of an observation's class-0 value: the batch's first frame
// plus the batch-relative offset stored by the fill.
struct PixDecode {
  int64_t base;
  __device__ __forceinline__ int64_t operator()(const ProbIn&, uint32_t q) const { return base + (int64_t)q; }
};

// Lanes = classes (any stride, any c): one wave per 64 consecutive spans
// (touched rows).
template <int NCH, int DT, int AGG, int AT>
__global__ __launch_bounds__(256) void k_seg_gather(MeshDev m, ProbIn in, PixDecode dec, const int4* __restrict__ spans,
                                                    const int32_t* __restrict__ nspans,
                                                    const uint32_t* __restrict__ ent_pix,
                                                    const float* __restrict__ ent_w, const float* __restrict__ ent_s) {
  const int lane = threadIdx.x & 63;
  const int64_t x0 = (((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6) * 64;
  const int ns = *nspans;
  if (x0 >= ns) return;
  const int c = m.c;
  const int64_t xl = x0 + lane;
  int s = 0, e = 0, row = 0;
  if (xl < ns) {
    const int4 sp = spans[xl];
    row = sp.x;
    s = sp.y;
    e = sp.z;
  }
  unsigned long long todo = __ballot(e > s);
  while (todo) {
    const int src = __ffsll(todo) - 1;
    todo &= todo - 1;
    const int seg_s = __builtin_amdgcn_readlane(s, src), seg_e = __builtin_amdgcn_readlane(e, src);
    const int64_t x = __builtin_amdgcn_readlane(row, src);
    // the row's old value is loaded first so its latency hides behind the observations
    float old[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const int j = lane + 64 * ch;
      old[ch] = j < c ? acc_load<AT>(m.accum, x * c + j) : 0.0f;
    }
    float acc[NCH], cmp[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) acc[ch] = cmp[ch] = 0.0f;
    float wsum = 0.0f;
    for (int b = seg_s; b < seg_e; b += 64) {
      const int k = b + lane;
      const bool ok = k < seg_e;
      const int64_t my_off = ok ? dec(in, ent_pix[k]) : 0;
      const float my_w = (ent_w && ok) ? ent_w[k] : 1.0f;
      const float my_s = (ent_s && ok) ? ent_s[k] : 1.0f;
      const int cnt = min(64, seg_e - b);
      const int lo32 = (int)(my_off & 0xffffffffll), hi32 = (int)(my_off >> 32);
      for (int i0 = 0; i0 < cnt; i0 += kGatherUnroll) {
        float v[kGatherUnroll][NCH];
        float w[kGatherUnroll];
#pragma unroll
        for (int u = 0; u < kGatherUnroll; ++u) {
          const int i = i0 + u < cnt ? i0 + u : i0;   // uniform
          const int64_t off = ((int64_t)__builtin_amdgcn_readlane(hi32, i) << 32) |
                              (uint32_t)__builtin_amdgcn_readlane(lo32, i);
          w[u] = i0 + u < cnt ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(my_w), i)) : 0.0f;
          const float sc = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(my_s), i));
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch) {
            const int j = lane + 64 * ch;
            v[u][ch] = (j < c && i0 + u < cnt) ? ld_prob<DT>(in.p, off + (int64_t)j * in.sc) : 1.0f;
            if (DT == 3) v[u][ch] = v[u][ch] * sc;
          }
        }
#pragma unroll
        for (int u = 0; u < kGatherUnroll; ++u) {
          if (i0 + u < cnt) {
            accumulate<NCH, DT, AGG>(acc, cmp, v[u], w[u], lane, c);
            wsum += w[u];
          }
        }
      }
    }
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const int j = lane + 64 * ch;
      if (j < c) acc_store<AT>(m.accum, x * c + j, old[ch] + (acc[ch] - cmp[ch]));
    }
    if (m.wsum && lane == 0) m.wsum[x] += wsum;
  }
}

// 16 lanes per row (classes contiguous, c <= 64, c % 4 == 0): lane i of a
// group owns classes 4i..4i+3 of one texel row and reads them as one float4
// (FP32) or one 32-bit word of four codes (E4M3) per observation, so one wave
// instruction fetches four contiguous class vectors.  The group loads 16
// observation offsets at once (one per lane, shuffled out) and keeps U (4 or
// 8) observations in flight.
//
// Per-frame weights (frame_w = 1: w^(I) = 1 / n, 3: (1 - mix) + mix / n, with
// n the number of pixels of the observation's frame that see the texel,
// Section 3.2.2): a row's observations of one frame are exactly that frame's
// pixels on the texel, so n is counted per row and frame in LDS from the
// row's own observations; an observation's frame is its stored element
// offset divided by the frame stride sfd.  Nothing per frame and texel is
// kept in device memory.
//
// Pixels dense in the input (spix != 0: a stored offset is spix times the
// batch-relative pixel index): E4M3 scales are read from the input's own
// [F][H][W] scale array at sbase + index, and per-pixel weights (wpix, the
// learned weight, [B][H][W]) at the index, instead of from per-observation
// copies written by the fill.
struct GatherCtx {
  int frame_w;
  float mix;
  uint32_t sfd;
  uint32_t spix;
  int64_t sbase;
  const float* wpix;
  const float* ew;   // per-observation weights, or nullptr
  const float* es;   // per-observation E4M3 scales, or nullptr
  Udiv dsfd, dspix;  // division by sfd and by spix (1 where spix = 0)
};

// The observations of one row: element offsets off[0 .. n); observation k's
// weight and scale sit at ibase + (idx ? idx[k] : k) of ew / es; fcnt = the
// row's per-frame counts (frame weights); sw[k] = observation k's learned
// weight when the gather evaluated the network itself.
struct RowObs {
  const uint32_t* off;
  const uint16_t* idx;
  int64_t ibase;
  const int* fcnt;
  const float* sw;
};

// One group (16 lanes) adds the row's observations to texel row x: up to 16
// observations summed plainly, the chunk sums then added to the row with
// compensation (SUM / MAXSUM) or plainly (MUL: sums of logs), the row read
// and written once.
template <int DT, int AGG, int AT, int U>
__device__ __forceinline__ void gather_row(const MeshDev& m, const ProbIn& in, const PixDecode& dec,
                                           const GatherCtx& gc, int64_t x, int n, const RowObs& ro, int gl,
                                           bool act) {
  const int c = m.c;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  float4 cmp = make_float4(0.f, 0.f, 0.f, 0.f);   // compensation of the SUM / MAXSUM sums
  float4 old = make_float4(0.f, 0.f, 0.f, 0.f);
  if (act) {
    if constexpr (AT == 0) {
      old = *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(m.accum) + x * c + 4 * gl);
    } else {
      const int64_t i0 = x * c + 4 * gl;
      old = make_float4(acc_load<AT>(m.accum, i0), acc_load<AT>(m.accum, i0 + 1), acc_load<AT>(m.accum, i0 + 2),
                        acc_load<AT>(m.accum, i0 + 3));
    }
  }
  float wsum = 0.0f;
  for (int k0 = 0; k0 < n; k0 += 16) {
    float4 part = make_float4(0.f, 0.f, 0.f, 0.f);
    const int kk = k0 + gl;
    const bool okl = kk < n;
    const uint32_t my_e = okl ? ro.off[kk] : 0u;
    const uint32_t my_p = gc.spix ? gc.dspix(my_e) : 0u;   // batch-relative pixel index
    const int64_t ei = ro.ibase + (ro.idx ? (int64_t)ro.idx[okl ? kk : 0] : (int64_t)kk);
    float my_w;
    if (ro.sw) {
      my_w = okl ? ro.sw[kk] : 0.0f;
    } else if (gc.frame_w) {
      const float nn = okl ? (float)ro.fcnt[gc.dsfd(my_e)] : 1.0f;
      my_w = okl ? (gc.frame_w == 1 ? 1.0f / nn : (1.0f - gc.mix) + gc.mix / nn) : 0.0f;
    } else if (gc.wpix) {
      my_w = okl ? gc.wpix[my_p] : 0.0f;
    } else {
      my_w = okl ? (gc.ew ? gc.ew[ei] : 1.0f) : 0.0f;
    }
    float my_s = 1.0f;
    if constexpr (DT == 3) {
      if (okl) my_s = gc.spix ? in.scale[gc.sbase + my_p] : gc.es[ei];
    }
    const int cnt = min(16, n - k0);
    for (int h = 0; h < cnt; h += U) {
      float4 v[U];
      float w[U];
      uint32_t q[U];                             // E4M3: raw codes, decoded once every load is issued
      float sc[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int src = h + u;
        const uint32_t e = __shfl(my_e, src, 16);
        w[u] = __shfl(my_w, src, 16);            // 0 past the row's end
        sc[u] = DT == 3 ? __shfl(my_s, src, 16) : 1.0f;
        const int64_t off = dec(in, e);
        v[u] = make_float4(1.f, 1.f, 1.f, 1.f);
        q[u] = 0u;
        if (act && src < cnt) {
          if constexpr (DT == 0)
            v[u] = *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(in.p) + off + 4 * gl);
          else
            q[u] = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const uint8_t*>(in.p) + off + 4 * gl);
        }
      }
      if constexpr (DT == 3) {
        // per-component selects (a select of whole vectors would be turned
        // into a load through a selected address, i.e. scratch memory)
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool okq = act && h + u < cnt;
          v[u].x = okq ? fp8_e4m3_byte<0>(q[u]) * sc[u] : 1.0f;
          v[u].y = okq ? fp8_e4m3_byte<1>(q[u]) * sc[u] : 1.0f;
          v[u].z = okq ? fp8_e4m3_byte<2>(q[u]) * sc[u] : 1.0f;
          v[u].w = okq ? fp8_e4m3_byte<3>(q[u]) * sc[u] : 1.0f;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        float4 t = v[u];
        if constexpr (AGG == 1) {
          t = make_float4(logf(t.x), logf(t.y), logf(t.z), logf(t.w));
        } else if constexpr (AGG == 2) {
          float mx = act ? fmaxf(fmaxf(t.x, t.y), fmaxf(t.z, t.w)) : -__builtin_inff();
#pragma unroll
          for (int o = 8; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 16));
          t = make_float4(t.x == mx ? t.x : 0.f, t.y == mx ? t.y : 0.f, t.z == mx ? t.z : 0.f,
                          t.w == mx ? t.w : 0.f);
        }
        part.x += w[u] * t.x;
        part.y += w[u] * t.y;
        part.z += w[u] * t.z;
        part.w += w[u] * t.w;
        wsum += w[u];
      }
    }
    if constexpr (AGG == 1) {
      acc.x += part.x;
      acc.y += part.y;
      acc.z += part.z;
      acc.w += part.w;
    } else {
      kahan_add(acc.x, cmp.x, part.x);
      kahan_add(acc.y, cmp.y, part.y);
      kahan_add(acc.z, cmp.z, part.z);
      kahan_add(acc.w, cmp.w, part.w);
    }
  }
  if (act) {
    const float4 nv4 = make_float4(old.x + (acc.x - cmp.x), old.y + (acc.y - cmp.y), old.z + (acc.z - cmp.z),
                                   old.w + (acc.w - cmp.w));
    if constexpr (AT == 0) {
      *reinterpret_cast<float4*>(reinterpret_cast<float*>(m.accum) + x * c + 4 * gl) = nv4;
    } else {
      const int64_t i0 = x * c + 4 * gl;
      acc_store<AT>(m.accum, i0, nv4.x);
      acc_store<AT>(m.accum, i0 + 1, nv4.y);
      acc_store<AT>(m.accum, i0 + 2, nv4.z);
      acc_store<AT>(m.accum, i0 + 3, nv4.w);
    }
  }
  if (m.wsum && gl == 0) m.wsum[x] += wsum;
}

// The grouped gather straight from the bucket-ordered records: one workgroup
// per non-empty bucket (walking the list), one group per row of the bucket
// (kBucketRows = 16 groups).  The bucket's records are counted per row and
// frame in LDS (frame weights, learned weight), then taken a chunk at a
// time: counted per row, scanned, and moved into LDS in row order, and every
// group adds its row's observations of the chunk (a row split over chunks is
// read and written once per chunk, by the same workgroup, in order).
constexpr int kBucketChunk = 2048;
constexpr int kLearnChunk = 1024;   // records per chunk with the learned weight

__host__ __device__ inline size_t bucket_gather_lds(int nf, bool frame_counts, bool learned) {
  const size_t ch = learned ? kLearnChunk : kBucketChunk;
  return ch * 4 + (learned ? ch * 4 : 0) + ch * 2 + 4 * kBucketRows * 4 +
         (frame_counts ? (size_t)kBucketRows * nf * 4 : 0);
}

// The learned weight of every record of a chunk (row order, d = 0 .. n):
// wave w takes records 64 (w + 4 i) .. + 63.  Each record's class vector is
// read by four lanes, lane j taking the four-class chunks j, j + 4, ...
// (a load instruction reads four consecutive chunks of each of 16 records:
// 64 contiguous bytes in FP32, 16 in E4M3), summed in the
// separate pass's order and reduced by a butterfly over the quad; the lane
// whose index is the record's place in the wave keeps its entropy sum and
// top-2.  Then lane = record: geometry from the resolve's per-pixel copy, n
// from the bucket's frame counters, the network on the matrix cores for the
// 16-record tiles the records fill, weights into LDS.  Pixels are dense in
// the input (offset = spix * batch-relative pixel index).
template <int DT>
__device__ __forceinline__ void chunk_learned_weights(const MeshDev& m, const ProbIn& in, const PixDecode& dec,
                                                      const GatherCtx& gc, const GatherLearn& lc,
                                                      const uint32_t* soff, const uint16_t* srow, const int* fc,
                                                      int nf, int n, float* sw) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = lane & 3, g4 = lane >> 2;
  const int c = m.c, nq = c >> 2, kmax = (nq + 3) >> 2;   // chunks; chunks per lane
  const uint8_t* pb = reinterpret_cast<const uint8_t*>(in.p);
  for (int base = wv * 64; base < n; base += 256) {
    // the network's parameters are read where they are used (from cache),
    // not held in registers across records
    const void* wp = lc.mlp;
    asm volatile("" : "+s"(wp));
    const MlpW Wt = mlp_view(wp);
    // round r: quad g4 reduces record base + 4 g4 + r.  Two rounds' loads
    // are issued before their sums; loads take no branch (past the chunk or
    // the vector a lane reads an in-bounds chunk and drops it).
    float hk = 0.0f, p1k = -__builtin_inff(), p2k = -__builtin_inff();
#pragma unroll 1
    for (int r0 = 0; r0 < 4; r0 += 2) {
      typename std::conditional<DT == 0, float4, uint32_t>::type v[2][4];
      float sc[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const uint32_t e = soff[min(base + 4 * g4 + r0 + i, n - 1)];
        const int64_t o = dec(in, e);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int q = min(j + 4 * k, nq - 1);
          if constexpr (DT == 0) v[i][k] = reinterpret_cast<const float4*>(pb + o * 4)[q];
          else v[i][k] = reinterpret_cast<const uint32_t*>(pb + o)[q];
        }
        sc[i] = DT == 3 ? in.scale[gc.sbase + gc.dspix(e)] : 1.0f;
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int r = r0 + i;
        float h = 0.0f, p1 = -__builtin_inff(), p2 = -__builtin_inff();
        int best = 0;
        if (base + 4 * g4 + r < n) {
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (k < kmax && j + 4 * k < nq) {
              if constexpr (DT == 0) {
                h = h + chunk_entropy<false>(v[i][k].x, v[i][k].y, v[i][k].z, v[i][k].w, 4 * (j + 4 * k), p1, p2,
                                             best);
              } else {
                const float t = sc[i];
                h = h + chunk_entropy<false>(fp8_e4m3_byte<0>(v[i][k]) * t, fp8_e4m3_byte<1>(v[i][k]) * t,
                                             fp8_e4m3_byte<2>(v[i][k]) * t, fp8_e4m3_byte<3>(v[i][k]) * t,
                                             4 * (j + 4 * k), p1, p2, best);
              }
            }
        }
        butterfly4(h, p1, p2);
        hk = j == r ? h : hk;
        p1k = j == r ? p1 : p1k;
        p2k = j == r ? p2 : p2k;
      }
    }
    const int d = base + lane;
    const bool ok = d < n;
    float phi[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) phi[k] = 0.0f;
    if (ok) {
      const uint32_t e = soff[d];
      const uint32_t p = gc.dspix(e);            // batch-relative pixel index
      const uint32_t fb = lc.dhw(p);
      const uint32_t rem = p - fb * lc.hw;
      const uint32_t y = lc.dw(rem), x = rem - y * lc.w;
      float ent;
      finish_prob_features(hk, c, ent, p2k);
      observation_phi(ent, p1k, p2k, lc.geo[p], fc[srow[d] * nf + gc.dsfd(e)], (int)x, (int)y,
                      lc.cams + 16 * (int64_t)fb, phi);
    }
    const float w = mlp_wave(phi, Wt, min(4, (n - base + 15) >> 4));
    if (ok) sw[d] = w;
  }
}

template <int DT, int AGG, int AT, int U, bool LW>
__device__ __forceinline__ void bucket_gather16(const MeshDev& m, const ProbIn& in, const PixDecode& dec,
                                                const GatherCtx& gc, const GatherLearn& lc, int H, int W,
                                                const int32_t* __restrict__ bstart, const int32_t* __restrict__ blist,
                                                const int32_t* __restrict__ nblist, const uint2* __restrict__ rec,
                                                int nf) {
  static_assert(kBucketRows == 16, "one group of 16 lanes per row of a bucket");
  constexpr int CH = LW ? kLearnChunk : kBucketChunk;
  extern __shared__ int lds[];
  uint32_t* soff = reinterpret_cast<uint32_t*>(lds);                    // [CH] offsets, row order
  float* sw = reinterpret_cast<float*>(soff + CH);                      // LW: [CH] learned weights
  uint16_t* sidx = reinterpret_cast<uint16_t*>(LW ? reinterpret_cast<uint32_t*>(sw + CH) : soff + CH);
                                                                        // [CH] chunk index (LW: row) of each
  int* rcnt2 = reinterpret_cast<int*>(sidx + CH);                       // [2][16] the chunk's count per row
                                                                        // (chunk j uses half j % 2)
  int* rst = rcnt2 + 2 * kBucketRows;                                   // [16] start per row
  int* rcur = rst + kBucketRows;                                        // [16] cursor per row
  int* fc = rcur + kBucketRows;                                         // [16][nf] frame counts
  const int t = threadIdx.x, gl = t & 15, grp = t >> 4;
  const bool act = gl < (m.c >> 2);
  const bool counts = LW || gc.frame_w;
  const int nb = *nblist;
  int g = blockIdx.x;
  int b = 0, s0 = 0, s1 = 0;
  if (g < nb) {
    b = blist[g];
    s0 = bstart[b];
    s1 = bstart[b + 1];
  }
  if (t < 2 * kBucketRows) rcnt2[t] = 0;
  __syncthreads();
  int j = 0;                                           // chunks done by this workgroup
  while (g < nb) {
    // the next bucket's place, read while this one is summed
    const int gn = g + (int)gridDim.x;
    int bn = 0, s0n = 0, s1n = 0;
    if (gn < nb) {
      bn = blist[gn];
      s0n = bstart[bn];
      s1n = bstart[bn + 1];
    }
    if (counts) {
      for (int i = t; i < kBucketRows * nf; i += 256) fc[i] = 0;
      __syncthreads();
      for (int i = s0 + t; i < s1; i += 256) {
        const uint2 q = rec[i];
        atomicAdd(&fc[(q.y & kBucketMask) * nf + gc.dsfd(q.x)], 1);
      }
    }
    for (int c0 = s0; c0 < s1; c0 += CH, ++j) {
      const int n = min(CH, s1 - c0);
      int* rcnt = rcnt2 + (j & 1) * kBucketRows;
      // the chunk's records, read once: counted per row, then placed in row order
      constexpr int PER = CH / 256;
      uint2 q[PER];
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int i = t + 256 * k;
        q[k] = i < n ? rec[c0 + i] : make_uint2(0u, 0u);
      }
#pragma unroll
      for (int k = 0; k < PER; ++k)
        if (t + 256 * k < n) atomicAdd(&rcnt[q[k].y & kBucketMask], 1);
      __syncthreads();
      if (t < 64) {
        const int v = t < kBucketRows ? rcnt[t] : 0;
        int incl = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int a = __shfl_up(incl, o);
          if (t >= o) incl += a;
        }
        if (t < kBucketRows) {
          rst[t] = incl - v;
          rcur[t] = incl - v;
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int i = t + 256 * k;
        if (i < n) {
          const int r = q[k].y & kBucketMask;
          const int d = atomicAdd(&rcur[r], 1);
          soff[d] = q[k].x;
          sidx[d] = (uint16_t)(LW ? r : i);
        }
      }
      // the other half of the row counts is free: clear it for the next chunk
      if (t < kBucketRows) rcnt2[((j + 1) & 1) * kBucketRows + t] = 0;
      __syncthreads();
      if constexpr (LW) {
        chunk_learned_weights<DT>(m, in, dec, gc, lc, soff, sidx, fc, nf, n, sw);
        __syncthreads();
      }
      const int cnt = rcnt[grp];
      if (cnt > 0)
        gather_row<DT, AGG, AT, U>(m, in, dec, gc, (int64_t)b * kBucketRows + grp, cnt,
                                   RowObs{soff + rst[grp], LW ? nullptr : sidx + rst[grp], c0, fc + grp * nf,
                                          LW ? sw + rst[grp] : nullptr},
                                   gl, act);
      __syncthreads();                                 // the chunk's LDS is reused next
    }
    g = gn;
    b = bn;
    s0 = s0n;
    s1 = s1n;
  }
}

template <int DT, int AGG, int AT, int U>
__global__ __launch_bounds__(256) void k_bucket_gather16(MeshDev m, ProbIn in, PixDecode dec, GatherCtx gc,
                                                         GatherLearn lc, int H, int W,
                                                         const int32_t* __restrict__ bstart,
                                                         const int32_t* __restrict__ blist,
                                                         const int32_t* __restrict__ nblist,
                                                         const uint2* __restrict__ rec, int nf) {
  bucket_gather16<DT, AGG, AT, U, false>(m, in, dec, gc, lc, H, W, bstart, blist, nblist, rec, nf);
}

// With the learned weight: registers for four waves per SIMD (no spills).
template <int DT, int AGG, int AT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_bucket_gather16_learned(
    MeshDev m, ProbIn in, PixDecode dec, GatherCtx gc, GatherLearn lc, int H, int W,
    const int32_t* __restrict__ bstart, const int32_t* __restrict__ blist, const int32_t* __restrict__ nblist,
    const uint2* __restrict__ rec, int nf) {
  bucket_gather16<DT, AGG, AT, 8, true>(m, in, dec, gc, lc, H, W, bstart, blist, nblist, rec, nf);
}

constexpr int kCountFrames = 256;   // frames per batch the gather's frame counters cover (16 KB of LDS)

// 4-class chunks of contiguous classes: 16-byte (FP32) / 4-byte (E4M3) aligned
static bool grouped_ok(const MeshDev& m, const ProbIn& in) {
  const int64_t esz = in.dtype == 0 ? 4 : 1;
  const int64_t chunk = 4 * esz;
  return in.sc == 1 && m.c <= 64 && (m.c % 4) == 0 && (reinterpret_cast<uintptr_t>(in.p) % chunk) == 0 &&
         ((in.sf * esz) % chunk) == 0 && ((in.sy * esz) % chunk) == 0 && ((in.sx * esz) % chunk) == 0 &&
         (reinterpret_cast<uintptr_t>(m.accum) % 16) == 0;
}

// The frame of a stored offset fb * sf + y * sy + x * sx is offset / sf when
// every pixel's offset within a frame is below the frame stride.
bool seg_frame_counts_ok(const MeshDev& m, const ProbIn& in, int nf, int H, int W) {
  if (!grouped_ok(m, in) || nf < 1 || nf > kCountFrames) return false;
  return nf == 1 || (in.sf > (int64_t)(H - 1) * in.sy + (int64_t)(W - 1) * in.sx && in.sf < ((int64_t)1 << 32));
}

// A stored offset fb * sf + y * sy + x * sx is sx times the batch-relative
// pixel index (fb * H + y) * W + x when sy = W * sx and sf = H * W * sx.
bool seg_pixels_dense_ok(const MeshDev& m, const ProbIn& in, int nf, int H, int W) {
  if (!grouped_ok(m, in) || in.sx < 1 || in.sx >= ((int64_t)1 << 32)) return false;
  return in.sy == (int64_t)W * in.sx && (nf == 1 || in.sf == (int64_t)H * W * in.sx);
}

bool seg_grouped_ok(const MeshDev& m, const ProbIn& in) { return grouped_ok(m, in); }

constexpr int kLearnFrames = 128;   // frames per batch of the learned gather (per-wave frame counters)

bool seg_learned_ok(const MeshDev& m, const ProbIn& in, int nf, int H, int W) {
  return nf <= kLearnFrames && seg_frame_counts_ok(m, in, nf, H, W) && seg_pixels_dense_ok(m, in, nf, H, W) &&
         bucket_gather_lds(nf, true, true) <= 65536;
}

hipError_t launch_bucket_gather(const MeshDev& m, const ProbIn& in, int f_first, int H, int W, int64_t n_buckets,
                                const int32_t* bstart, const int32_t* blist, const int32_t* nblist, const uint2* rec,
                                const float* rec_w, const float* rec_s, int nf, int frame_w, float mix,
                                const float* wpix, const GatherLearn& learn, hipStream_t s) {
  if (m.n_rows == 0 || n_buckets <= 0) return hipSuccess;
  if (!grouped_ok(m, in)) return hipErrorInvalidValue;
  const bool learned = learn.mlp != nullptr;
  if ((frame_w || learned) && !seg_frame_counts_ok(m, in, nf, H, W)) return hipErrorInvalidValue;
  if (frame_w && frame_w != 1 && frame_w != 3) return hipErrorInvalidValue;
  if (learned && (frame_w || wpix || rec_w || !learn.geo || !learn.cams || !seg_learned_ok(m, in, nf, H, W)))
    return hipErrorInvalidValue;
  // E4M3 without per-observation scales, per-pixel weights or the learned
  // weight: read by pixel index
  const bool direct = (in.dtype == 3 && !rec_s) || wpix || learned;
  if (direct && ((in.dtype == 3 && !in.scale) || (frame_w && wpix) || !seg_pixels_dense_ok(m, in, nf, H, W)))
    return hipErrorInvalidValue;
  const uint32_t sfd = nf > 1 ? (uint32_t)in.sf : 0xffffffffu;   // every stored offset is below 2^32 - 1
  const uint32_t spix = direct ? (uint32_t)in.sx : 0u;
  GatherCtx gc{frame_w, mix, sfd, spix, (int64_t)f_first * H * W, wpix, rec_w, rec_s, Udiv::make(sfd),
               Udiv::make(spix ? spix : 1u)};
  GatherLearn lc = learn;
  lc.hw = (uint32_t)H * (uint32_t)W;
  lc.w = (uint32_t)W;
  lc.dhw = Udiv::make(lc.hw);
  lc.dw = Udiv::make(lc.w);
  const PixDecode dec{(int64_t)f_first * in.sf};
  const size_t lds = bucket_gather_lds(nf, frame_w || learned, learned);
  // gather_waves resident waves (one workgroup = 4 waves) on each of the 256 CUs
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(n_buckets, (int64_t)64 * m.gather_waves));
#define LF_ARGS m, in, dec, gc, lc, H, W, bstart, blist, nblist, rec, nf
#define LF_R(DT, AGG, AT)                                                                   \
  do {                                                                                      \
    if (learned)                                                                            \
      k_bucket_gather16_learned<DT, AGG, AT><<<g, 256, lds, s>>>(LF_ARGS);                  \
    else if (m.gather_unroll == 4)                                                          \
      k_bucket_gather16<DT, AGG, AT, 4><<<g, 256, lds, s>>>(LF_ARGS);                       \
    else                                                                                    \
      k_bucket_gather16<DT, AGG, AT, 8><<<g, 256, lds, s>>>(LF_ARGS);                       \
  } while (0)
#define LF_R2(DT)                                                                                            \
  do {                                                                                                       \
    if (m.aggregator == 1) LF_R(DT, 1, 0);                                                                   \
    else if (m.accum_dtype == 1) { if (m.aggregator == 0) LF_R(DT, 0, 1); else LF_R(DT, 2, 1); }            \
    else if (m.accum_dtype == 2) { if (m.aggregator == 0) LF_R(DT, 0, 2); else LF_R(DT, 2, 2); }            \
    else { if (m.aggregator == 0) LF_R(DT, 0, 0); else LF_R(DT, 2, 0); }                                     \
  } while (0)
  if (in.dtype == 0) LF_R2(0);
  else LF_R2(3);
#undef LF_R2
#undef LF_R
#undef LF_ARGS
  return hipGetLastError();
}

hipError_t launch_seg_gather(const MeshDev& m, const ProbIn& in, int f_first, const int4* spans,
                             const int32_t* nspans, const uint32_t* ent, const float* ent_w, const float* ent_s,
                             hipStream_t s) {
  if (m.n_rows == 0) return hipSuccess;
  if (in.dtype == 3 && !ent_s) return hipErrorInvalidValue;
  const PixDecode dec{(int64_t)f_first * in.sf};
  const int64_t waves = (m.n_rows + 63) / 64;
  dim3 g((unsigned)((waves + 3) / 4));
#define LF_G(NCH, DT, AGG, AT) \
  k_seg_gather<NCH, DT, AGG, AT><<<g, 256, 0, s>>>(m, in, dec, spans, nspans, ent, ent_w, ent_s)
#define LF_G2(NCH, DT)                                                                                       \
  do {                                                                                                       \
    if (m.aggregator == 1) LF_G(NCH, DT, 1, 0);                                                              \
    else if (m.accum_dtype == 1) { if (m.aggregator == 0) LF_G(NCH, DT, 0, 1); else LF_G(NCH, DT, 2, 1); }  \
    else if (m.accum_dtype == 2) { if (m.aggregator == 0) LF_G(NCH, DT, 0, 2); else LF_G(NCH, DT, 2, 2); }  \
    else { if (m.aggregator == 0) LF_G(NCH, DT, 0, 0); else LF_G(NCH, DT, 2, 0); }                          \
  } while (0)
  if (m.c <= 64) {
    if (in.dtype == 0) LF_G2(1, 0); else LF_G2(1, 3);
  } else {
    if (in.dtype == 0) LF_G2(4, 0); else LF_G2(4, 3);
  }
#undef LF_G2
#undef LF_G
  return hipGetLastError();
}

hipError_t launch_seg_scan(const int32_t* seg, int64_t n, int32_t* sums, int32_t* start, int32_t* rows,
                           int32_t* nrows, hipStream_t s) {
  const int64_t nblk = std::max<int64_t>((n + kSegChunk - 1) / kSegChunk, 1);
  k_seg_sums<<<dim3((unsigned)nblk), 256, 0, s>>>(seg, n, sums);
  k_seg_scan_sums<<<1, 1024, 0, s>>>(sums, nblk);
  k_seg_scan<<<dim3((unsigned)nblk), 256, 0, s>>>(seg, n, sums, start, rows, nrows);
  return hipGetLastError();
}

hipError_t launch_planar_rows(const ProbIn& in, int f_first, int nf, int H, int W, int c, float* staging,
                              hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  if (c > kStageMaxC || (c & 3) || in.dtype != 0) return hipErrorInvalidValue;
  const int64_t HW = (int64_t)H * W;
  const size_t lds = (size_t)c * (kStagePixels + 1) * 4;
  k_planar_rows<kStagePixels><<<dim3((unsigned)((HW + kStagePixels - 1) / kStagePixels), (unsigned)nf), 256, lds, s>>>(
      in, f_first, H, W, c, staging);
  return hipGetLastError();
}

hipError_t launch_seg_fill(const ProbIn& in, int f_first, int nf, int H, int W, const int32_t* l, const int32_t* rank,
                           const int32_t* bstart, uint2* rec, float* rec_w, float* rec_s, int weighting,
                           const int32_t* cnt, int64_t cnt_stride, const float* wpix, float mix, int64_t win_lo,
                           int64_t n_rows, int32_t* cnt_zero, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  // the count array is either read here (w^(I), mixed) or cleared here
  if (cnt_zero && rec_w && (weighting == 1 || weighting == 3)) return hipErrorInvalidValue;
  const int64_t HW = (int64_t)H * W;
  const unsigned gx = (unsigned)(((HW + 1023) / 1024 + 7) / 8 * 8);   // chunks, rounded up to a multiple of 8
  k_seg_fill<<<dim3(gx, (unsigned)nf), 256, 0, s>>>(in, f_first, H, W, l, rank, bstart, rec, rec_w, rec_s, weighting,
                                                    cnt, cnt_stride, wpix, mix, win_lo, n_rows, cnt_zero);
  return hipGetLastError();
}

hipError_t launch_bucket_sort(int64_t n_buckets, const int32_t* bstart, const int32_t* blist, const int32_t* nblist,
                              const uint2* rec, const float* rec_w, const float* rec_s, uint32_t* ent, float* ent_w,
                              float* ent_s, int4* spans, int32_t* nspans, hipStream_t s) {
  if (n_buckets <= 0) return hipSuccess;
  const unsigned g = (unsigned)std::min<int64_t>(n_buckets, 4096);
  k_bucket_sort<<<g, 256, 0, s>>>(bstart, blist, nblist, rec, rec_w, rec_s, ent, ent_w, ent_s, spans, nspans);
  return hipGetLastError();
}

}  // namespace lf
