// Aggregation (Sections 3.2.1, 3.2.2, 3.3.2): scatter of weighted pixel
// distributions into texel rows, normalisation + argmax, render-back.
//
// k_scatter_hash: a block owns one screen tile of K consecutive frames.  The
// texel rows its (pixel, frame) observations hit are first gathered into an
// LDS hash table (open addressing on the row index), so every distinct row
// costs one global atomic per class per block instead of one per pixel.
// Classes are processed CC at a time: the block reads one class plane of the
// tile (coalesced along x for NCHW input), adds w * p into the LDS row with
// ds_add_f32, then flushes the used rows to HBM with global_atomic_add_f32.
// Observations that find no free slot fall back to direct global atomics.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "accum.h"
#include <algorithm>

#include "internal.h"
#include "spec.h"

namespace lf {

template <int DT>
__device__ __forceinline__ float load_prob(const ProbIn& in, int64_t e, float scale) {
  if constexpr (DT == 0) {
    return __builtin_nontemporal_load(reinterpret_cast<const float*>(in.p) + e);
  } else {
    return fp8_e4m3(__builtin_nontemporal_load(reinterpret_cast<const uint8_t*>(in.p) + e)) * scale;
  }
}

template <int AGG>
__device__ __forceinline__ float agg_term(float p, float pmax) {
  if constexpr (AGG == 0) return p;
  else if constexpr (AGG == 1) return logf(p);
  else return (p == pmax) ? p : 0.0f;
}

template <int TW, int TH, int K, int CC, int DT, int AGG, int AT>
__global__ __launch_bounds__(TW * TH) void k_scatter_hash(MeshDev m, ProbIn in, int f_first, int nf, int H, int W,
                                                           const int32_t* __restrict__ lbuf, int weighting,
                                                           const int32_t* __restrict__ cnt, int64_t cnt_stride,
                                                           const float* __restrict__ wpix, float mix) {
  constexpr int NT = TW * TH;
  constexpr int HS = 2048;            // hash slots (power of two)
  constexpr int RC = 1024;            // LDS rows
  constexpr int MAXPROBE = 64;
  __shared__ int hkey[HS];
  __shared__ short hpos[HS];
  __shared__ int rowl[RC];
  __shared__ float rows[RC * CC];
  __shared__ int nrow;

  const int c = m.c;
  void* __restrict__ A = m.accum;
  const int tiles_x = (W + TW - 1) / TW;
  const int tile = blockIdx.x;
  const int x = (tile % tiles_x) * TW + (threadIdx.x % TW);
  const int y = (tile / tiles_x) * TH + (threadIdx.x / TW);
  const bool inimg = x < W && y < H;
  const int64_t HW = (int64_t)H * W;
  const int fb0 = blockIdx.y * K;     // first frame of this group, relative to the batch

  for (int i = threadIdx.x; i < HS; i += NT) hkey[i] = -1;
  if (threadIdx.x == 0) nrow = 0;
  __syncthreads();

  int lk[K];
  int sk[K];
  float wk[K];
  float sck[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    lk[k] = -1;
    sk[k] = -1;
    wk[k] = 0.0f;
    sck[k] = 1.0f;
    const int fb = fb0 + k;
    if (fb < nf && inimg) {
      const int64_t pi = (int64_t)fb * HW + (int64_t)y * W + x;
      const int64_t gi = (int64_t)(f_first + fb) * HW + (int64_t)y * W + x;
      // window-relative row (-1: no triangle, invalid, or outside the window)
      const int64_t lw = (int64_t)lbuf[pi] - m.win_lo;
      int l = (lbuf[pi] >= 0 && lw >= 0 && lw < m.n_rows) ? (int)lw : -1;
      if (l >= 0 && in.valid && !in.valid[gi]) l = -1;
      if (l >= 0) {
        float w = 1.0f;
        if (weighting == 1) w = 1.0f / (float)cnt[(int64_t)fb * cnt_stride + l];
        else if (weighting == 2) w = wpix[pi];
        else if (weighting == 3) w = (1.0f - mix) + mix / (float)cnt[(int64_t)fb * cnt_stride + l];
        lk[k] = l;
        wk[k] = w;
        if (DT == 3) sck[k] = in.scale[gi];
        if (m.wsum) unsafeAtomicAdd(m.wsum + l, w);
        // insert l; the thread whose CAS fills an empty slot owns it
        uint32_t h = ((uint32_t)l * 2654435761u) >> (32 - 11);
        for (int probe = 0; probe < MAXPROBE; ++probe) {
          const int prev = atomicCAS(&hkey[h], -1, l);
          if (prev == -1 || prev == l) {
            sk[k] = (prev == -1) ? (int)(h | 0x80000000u) : (int)h;
            break;
          }
          h = (h + 1) & (HS - 1);
        }
      }
    }
  }
  __syncthreads();
  // owners allocate compact rows
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (sk[k] != -1 && (sk[k] & 0x80000000)) {
      const int slot = sk[k] & 0x7fffffff;
      const int pos = atomicAdd(&nrow, 1);
      hpos[slot] = (short)(pos < RC ? pos : -1);
      if (pos < RC) rowl[pos] = lk[k];
      sk[k] = slot;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (sk[k] != -1) sk[k] = hpos[sk[k]];   // -1 when the rows overflowed
  const int nr = min(nrow, RC);

  // per-observation maxima for maxsum
  float pmx[K];
#pragma unroll
  for (int k = 0; k < K; ++k) pmx[k] = 0.0f;
  if constexpr (AGG == 2) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (lk[k] < 0) continue;
      const int64_t base = (int64_t)(f_first + fb0 + k) * in.sf + (int64_t)y * in.sy + (int64_t)x * in.sx;
      float mx = load_prob<DT>(in, base, sck[k]);
      for (int j = 1; j < c; ++j) mx = fmaxf(mx, load_prob<DT>(in, base + (int64_t)j * in.sc, sck[k]));
      pmx[k] = mx;
    }
  }

  for (int j0 = 0; j0 < c; j0 += CC) {
    for (int i = threadIdx.x; i < nr * CC; i += NT) rows[i] = 0.0f;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (lk[k] < 0) continue;
      const int64_t base = (int64_t)(f_first + fb0 + k) * in.sf + (int64_t)y * in.sy + (int64_t)x * in.sx;
#pragma unroll
      for (int jj = 0; jj < CC; ++jj) {
        const int j = j0 + jj;
        if (j >= c) break;
        const float v = wk[k] * agg_term<AGG>(load_prob<DT>(in, base + (int64_t)j * in.sc, sck[k]), pmx[k]);
        if (sk[k] >= 0) atomicAdd(&rows[sk[k] * CC + jj], v);
        else acc_atomic_add<AT>(A, (int64_t)lk[k] * c + j, v);
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nr * CC; i += NT) {
      const int r = i / CC, jj = i - r * CC;
      const int j = j0 + jj;
      const float v = rows[i];
      if (j < c && v != 0.0f) acc_atomic_add<AT>(A, (int64_t)rowl[r] * c + j, v);
    }
    __syncthreads();
  }
}

hipError_t launch_scatter_atomic(const MeshDev& m, const ProbIn& in, int f_first, int nf, int H, int W,
                                 const int32_t* l, int weighting, const int32_t* cnt, int64_t cnt_stride,
                                 const float* wpix, float mix, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  constexpr int TW = 16, TH = 16, K = 4, CC = 8;
  dim3 grid((unsigned)(((W + TW - 1) / TW) * ((H + TH - 1) / TH)), (unsigned)((nf + K - 1) / K));
#define LF_SCATTER(DT, AGG, AT)                                                                     \
  k_scatter_hash<TW, TH, K, CC, DT, AGG, AT><<<grid, TW * TH, 0, s>>>(m, in, f_first, nf, H, W, l, weighting, cnt, \
                                                                       cnt_stride, wpix, mix)
#define LF_SCATTER2(DT)                                                   \
  do {                                                                    \
    if (m.aggregator == 1) LF_SCATTER(DT, 1, 0);                          \
    else if (m.accum_dtype == 0) { if (m.aggregator == 0) LF_SCATTER(DT, 0, 0); else LF_SCATTER(DT, 2, 0); } \
    else if (m.accum_dtype == 1) { if (m.aggregator == 0) LF_SCATTER(DT, 0, 1); else LF_SCATTER(DT, 2, 1); } \
    else { if (m.aggregator == 0) LF_SCATTER(DT, 0, 2); else LF_SCATTER(DT, 2, 2); }                     \
  } while (0)
  if (in.dtype == 0) LF_SCATTER2(0);
  else LF_SCATTER2(3);
#undef LF_SCATTER2
#undef LF_SCATTER
  return hipGetLastError();
}

// ---- w^(I) counts are per frame: clear the entries a batch touched ---------
__global__ __launch_bounds__(256) void k_clear_counts(const int32_t* __restrict__ l, int H, int W,
                                                      int32_t* __restrict__ cnt, int64_t cnt_stride, int64_t win_lo) {
  const int fb = blockIdx.y;
  const int64_t HW = (int64_t)H * W;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= HW) return;
  const int32_t li = l[(int64_t)fb * HW + p];
  const int64_t lw = (int64_t)li - win_lo;
  if (li >= 0 && lw >= 0 && lw < cnt_stride) cnt[(int64_t)fb * cnt_stride + lw] = 0;
}

// ---- texel resolution (Section 3.1): a_t = most pixels triangle t covers in
// any frame; s_t = max(1, ceil(gamma * sqrt(a_t))) ----------------------------------
// Per pixel of each frame: raise area[t] to the frame's count of t (the same
// value from every pixel of t), then a second kernel clears the counts.
__global__ __launch_bounds__(256) void k_area_max(const int32_t* __restrict__ tri, int H, int W,
                                                  const int32_t* __restrict__ tricnt, int64_t T,
                                                  int32_t* __restrict__ area) {
  const int fb = blockIdx.y;
  const int64_t HW = (int64_t)H * W;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= HW) return;
  const int32_t t = tri[(int64_t)fb * HW + p];
  if (t >= 0) atomicMax(area + t, tricnt[(int64_t)fb * T + t]);
}

__global__ __launch_bounds__(256) void k_area_clear(const int32_t* __restrict__ tri, int H, int W,
                                                    int32_t* __restrict__ tricnt, int64_t T) {
  const int fb = blockIdx.y;
  const int64_t HW = (int64_t)H * W;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= HW) return;
  const int32_t t = tri[(int64_t)fb * HW + p];
  if (t >= 0) tricnt[(int64_t)fb * T + t] = 0;
}

hipError_t launch_area_max(const int32_t* tri, int nf, int H, int W, int32_t* tricnt, int64_t T, int32_t* area,
                           hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  const int64_t HW = (int64_t)H * W;
  const dim3 g((unsigned)((HW + 255) / 256), (unsigned)nf);
  k_area_max<<<g, 256, 0, s>>>(tri, H, W, tricnt, T, area);
  k_area_clear<<<g, 256, 0, s>>>(tri, H, W, tricnt, T);
  return hipGetLastError();
}

// binary32 throughout (gamma, correctly rounded sqrt, product, ceil)
__global__ __launch_bounds__(256) void k_texel_resolution(const int32_t* __restrict__ area, int64_t T, float gamma,
                                                          int32_t* __restrict__ s_face) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= T) return;
  const float v = ceilf(gamma * sqrtf((float)area[t]));
  s_face[t] = v > 1.0f ? (int32_t)fminf(v, 4096.0f) : 1;
}

hipError_t launch_texel_resolution(const int32_t* area, int64_t T, float gamma, int32_t* s_face, hipStream_t s) {
  if (T <= 0) return hipSuccess;
  k_texel_resolution<<<dim3((unsigned)((T + 255) / 256)), 256, 0, s>>>(area, T, gamma, s_face);
  return hipGetLastError();
}

hipError_t launch_clear_counts(const int32_t* l, const uint8_t* /*valid*/, int nf, int H, int W, int32_t* cnt,
                               int64_t cnt_stride, int64_t win_lo, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  const int64_t HW = (int64_t)H * W;
  k_clear_counts<<<dim3((unsigned)((HW + 255) / 256), (unsigned)nf), 256, 0, s>>>(l, H, W, cnt, cnt_stride, win_lo);
  return hipGetLastError();
}

// ---- normalise + argmax (one wave per row group) ---------------------------
template <int OUT>
__device__ __forceinline__ void store_tex(void* out, int64_t i, float v) {
  if constexpr (OUT == 0) reinterpret_cast<float*>(out)[i] = v;
  else if constexpr (OUT == 1) reinterpret_cast<__hip_bfloat16*>(out)[i] = __float2bfloat16(v);
  else reinterpret_cast<__half*>(out)[i] = __float2half(v);
}

// A block stages R consecutive rows in LDS with coalesced loads (row stride
// padded to an odd number of words against bank conflicts); one thread per
// row then computes S = sum_j A_j in class order, P = A / S and the first
// maximal class (S == 0: never observed -> P = 0, label 255).  For MUL the row
// holds sum w log p: P = softmax(A), observed iff its weight sum is > 0.
// The normalised rows are written back through LDS, coalesced.
template <int OUT, int AGG, int AT>
__global__ __launch_bounds__(256) void k_finalize(MeshDev m, void* __restrict__ out, uint8_t* __restrict__ labels, int R) {
  extern __shared__ float rows[];
  const int c = m.c;
  const int cp = c | 1;
  const int64_t x0 = (int64_t)blockIdx.x * R;
  const int nr = (int)min<int64_t>(R, m.n_rows - x0);
  const int64_t a0 = x0 * c;
  // element i of the block's rows sits at row i / c: walk (row, class) pairs
  // incrementally instead of dividing per element
  if (AT == 0 && (c & 3) == 0 && (reinterpret_cast<uintptr_t>(m.accum) & 15) == 0) {
    // four classes per load (rows of c % 4 == 0 floats stay 16-byte aligned)
    const float4* src = reinterpret_cast<const float4*>(reinterpret_cast<const float*>(m.accum) + a0);
    const int c4 = c >> 2;
    int r = threadIdx.x / c4, j = 4 * (threadIdx.x - r * c4);
    const int dr = 256 / c4, dj = 4 * (256 - dr * c4);
    for (int i = threadIdx.x; i < nr * c4; i += 256) {
      const float4 v = src[i];
      float* d = rows + r * cp + j;
      d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
      r += dr;
      j += dj;
      if (j >= c) { j -= c; ++r; }
    }
  } else {
    int r = threadIdx.x / c, j = threadIdx.x - (threadIdx.x / c) * c;
    const int dr = 256 / c, dj = 256 - dr * c;
    for (int i = threadIdx.x; i < nr * c; i += 256) {
      rows[r * cp + j] = acc_load<AT>(m.accum, a0 + i);
      r += dr;
      j += dj;
      if (j >= c) { j -= c; ++r; }
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < nr; r += 256) {
    float* row = rows + r * cp;
    float mx = row[0];
    int best = 0;
    for (int j = 1; j < c; ++j) {
      const float v = row[j];
      if (v > mx) { mx = v; best = j; }
    }
    bool seen;
    if constexpr (AGG == 1) {
      seen = m.wsum[x0 + r] > 0.0f;
      float s = 0.0f;
      for (int j = 0; j < c; ++j) s += expf(row[j] - mx);
      for (int j = 0; j < c; ++j) row[j] = seen ? expf(row[j] - mx) / s : 0.0f;
    } else {
      float s = 0.0f;
      for (int j = 0; j < c; ++j) s += row[j];
      seen = s > 0.0f;
      for (int j = 0; j < c; ++j) row[j] = seen ? row[j] / s : 0.0f;
    }
    labels[x0 + r] = seen ? (uint8_t)best : (uint8_t)255;
  }
  if (!out) return;
  __syncthreads();
  if (OUT == 0 && (c & 3) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
    float4* dst = reinterpret_cast<float4*>(reinterpret_cast<float*>(out) + x0 * c);
    const int c4 = c >> 2;
    int r = threadIdx.x / c4, j = 4 * (threadIdx.x - r * c4);
    const int dr = 256 / c4, dj = 4 * (256 - dr * c4);
    for (int i = threadIdx.x; i < nr * c4; i += 256) {
      const float* q = rows + r * cp + j;
      dst[i] = make_float4(q[0], q[1], q[2], q[3]);
      r += dr;
      j += dj;
      if (j >= c) { j -= c; ++r; }
    }
    return;
  }
  int r = threadIdx.x / c, j = threadIdx.x - (threadIdx.x / c) * c;
  const int dr = 256 / c, dj = 256 - dr * c;
  for (int i = threadIdx.x; i < nr * c; i += 256) {
    store_tex<OUT>(out, x0 * c + i, rows[r * cp + j]);
    r += dr;
    j += dj;
    if (j >= c) { j -= c; ++r; }
  }
}

hipError_t launch_finalize(const MeshDev& m, void* tex_out, int tex_dtype, uint8_t* labels, hipStream_t s) {
  if (m.n_rows == 0) return hipSuccess;
  const int cp = m.c | 1;
  // rows per block: up to 128, within 32 KB of LDS (21 KB at c = 40: seven
  // blocks per compute unit keep more row loads in flight than three blocks
  // of 256 rows)
  const int R = std::max(1, std::min(128, 8192 / cp));
  const size_t lds = (size_t)R * cp * sizeof(float);
  dim3 g((unsigned)((m.n_rows + R - 1) / R));
#define LF_FIN(O, A, T) k_finalize<O, A, T><<<g, 256, lds, s>>>(m, tex_out, labels, R)
#define LF_FIN2(O)                                              \
  do {                                                          \
    if (m.aggregator == 1) LF_FIN(O, 1, 0);                     \
    else if (m.accum_dtype == 1) LF_FIN(O, 0, 1);               \
    else if (m.accum_dtype == 2) LF_FIN(O, 0, 2);               \
    else LF_FIN(O, 0, 0);                                       \
  } while (0)
  if (tex_dtype == 1) LF_FIN2(1);
  else if (tex_dtype == 2) LF_FIN2(2);
  else LF_FIN2(0);
#undef LF_FIN2
#undef LF_FIN
  return hipGetLastError();
}

// ---- render-back: a texel label per pixel (255 where unseen or invalid) ------
__global__ __launch_bounds__(256) void k_render(const int32_t* __restrict__ l, const uint8_t* __restrict__ valid,
                                                const uint8_t* __restrict__ labels, int64_t npx,
                                                uint8_t* __restrict__ out) {
  // 8 pixels per thread at a stride of 256: every load, label gather and
  // store instruction of a wave covers 64 neighbouring pixels, which see
  // neighbouring texels, so a gather touches few cache lines.
  constexpr int P = 8;
  const int64_t base = (int64_t)blockIdx.x * (256 * P) + threadIdx.x;
  int32_t li[P];
  bool ok[P];
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const int64_t p = base + (int64_t)k * 256;
    ok[k] = p < npx;
    li[k] = ok[k] ? l[p] : -1;
  }
  if (valid) {
#pragma unroll
    for (int k = 0; k < P; ++k)
      if (ok[k] && !valid[base + (int64_t)k * 256]) li[k] = -1;
  }
  uint8_t lab[P];
#pragma unroll
  for (int k = 0; k < P; ++k) lab[k] = li[k] >= 0 ? labels[li[k]] : (uint8_t)255;
#pragma unroll
  for (int k = 0; k < P; ++k)
    if (ok[k]) out[base + (int64_t)k * 256] = lab[k];
}

// ---- agreement of label images with the frames' own argmax ------------------
// counts[0] += pixels with a label (not 255) and valid; counts[1] += those
// whose label equals the argmax of the pixel's own distribution (first
// maximal class).  One block per 256 pixels of a frame; one atomic pair per
// block.
template <int DT>
__global__ __launch_bounds__(256) void k_agreement(ProbIn in, int c, int H, int W, const uint8_t* __restrict__ img,
                                                   unsigned long long* __restrict__ counts) {
  __shared__ unsigned int part[2][4];
  const int f = blockIdx.y;
  const int64_t HW = (int64_t)H * W;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  unsigned int n = 0, agree = 0;
  if (p < HW) {
    const uint8_t lab = img[(int64_t)f * HW + p];
    const bool ok = lab != 255 && (!in.valid || in.valid[(int64_t)f * HW + p]);
    if (ok) {
      const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
      const int64_t base = (int64_t)f * in.sf + (int64_t)y * in.sy + (int64_t)x * in.sx;
      const float sc = DT == 3 ? in.scale[(int64_t)f * HW + p] : 1.0f;
      float best = -__builtin_inff();
      int arg = 0;
      for (int j = 0; j < c; ++j) {
        float v;
        if constexpr (DT == 0) v = reinterpret_cast<const float*>(in.p)[base + (int64_t)j * in.sc];
        else v = fp8_e4m3(reinterpret_cast<const uint8_t*>(in.p)[base + (int64_t)j * in.sc]) * sc;
        if (v > best) { best = v; arg = j; }
      }
      n = 1;
      agree = arg == lab;
    }
  }
  // wave sums, then one atomic pair per block
  const unsigned long long bn = __ballot(n != 0), ba = __ballot(agree != 0);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    part[0][wv] = (unsigned)__popcll(bn);
    part[1][wv] = (unsigned)__popcll(ba);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned tn = part[0][0] + part[0][1] + part[0][2] + part[0][3];
    const unsigned ta = part[1][0] + part[1][1] + part[1][2] + part[1][3];
    if (tn) atomicAdd(counts, (unsigned long long)tn);
    if (ta) atomicAdd(counts + 1, (unsigned long long)ta);
  }
}

hipError_t launch_agreement(const ProbIn& in, int c, int F, int H, int W, const uint8_t* img,
                            unsigned long long* counts, hipStream_t s) {
  if (F <= 0) return hipSuccess;
  const int64_t HW = (int64_t)H * W;
  const dim3 g((unsigned)((HW + 255) / 256), (unsigned)F);
  if (in.dtype == 0) k_agreement<0><<<g, 256, 0, s>>>(in, c, H, W, img, counts);
  else k_agreement<3><<<g, 256, 0, s>>>(in, c, H, W, img, counts);
  return hipGetLastError();
}

hipError_t launch_render(const int32_t* l, const uint8_t* valid, const uint8_t* labels, int64_t npx, uint8_t* out,
                         hipStream_t s) {
  if (npx <= 0) return hipSuccess;
  k_render<<<dim3((unsigned)((npx + 2047) / 2048)), 256, 0, s>>>(l, valid, labels, npx, out);
  return hipGetLastError();
}

}  // namespace lf
