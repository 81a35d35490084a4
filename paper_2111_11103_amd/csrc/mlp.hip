// Learned per-observation fusion weight: w_k = MLP(phi_k), a generalisation
// of the fixed weights w^(P), w^(I) of Section 3.2.2.
//
//   h1 = relu(W1 q(phi) + b1)   (64 x 8)
//   h2 = relu(W2 q(h1) + b2)    (64 x 64)
//   w  = sigmoid(w3 . h2 + b3)
// q = round to bfloat16; W1, W2, w3 are bfloat16, biases and accumulation
// binary32.  Inference runs both matrix products on the matrix cores
// (v_mfma_f32_16x16x16_bf16 for the 8-input layer, v_mfma_f32_16x16x32_bf16
// for the hidden layer): a wave evaluates 64 observations as four 16-column
// tiles of the transposed layers, q(h1) kept in registers.
// Training gradients are accumulated on the vector ALUs in binary32 (one
// wave per chunk of observations, one lane per hidden unit) and applied
// with Adam on binary32 master parameters.
#include <hip/hip_bf16.h>

#include "internal.h"
#include "mlp.h"
#include "spec.h"

namespace lf {

// ---- packing and Adam ---------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_pack(const float* __restrict__ prm, char* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= NPARAM) return;
  if (i < OB1) reinterpret_cast<uint16_t*>(out + PW1)[i - OW1] = bf16_bits(prm[i]);
  else if (i < OW2) reinterpret_cast<float*>(out + PB1)[i - OB1] = prm[i];
  else if (i < OB2) reinterpret_cast<uint16_t*>(out + PW2)[i - OW2] = bf16_bits(prm[i]);
  else if (i < OW3) reinterpret_cast<float*>(out + PB2)[i - OB2] = prm[i];
  else if (i < OB3) reinterpret_cast<uint16_t*>(out + PW3)[i - OW3] = bf16_bits(prm[i]);
  else reinterpret_cast<float*>(out + PB3)[0] = prm[i];
}

// Adam (Kingma & Ba 2015) in binary32: bias-corrected first and second moments.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, int64_t n, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ __launch_bounds__(256) void k_mlp_forward(const void* __restrict__ packed, const float* __restrict__ phi,
                                                     int64_t n, float* __restrict__ w_out) {
  const MlpW W = mlp_view(packed);
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float x[NI];
#pragma unroll
  for (int k = 0; k < NI; ++k) x[k] = i < n ? phi[i * NI + k] : 0.0f;
  const float w = mlp_wave(x, W);
  if (i < n) w_out[i] = w;
}

// Inference as a pass of its own (layouts the grouped gather does not take):
// weight of every valid covered pixel of the batch (0 elsewhere), from the
// per-frame count array.  A pixel's class vector, geometry and validity are
// read before its coverage is known (they exist for every pixel of the
// frame), so only the frame count waits for the texel row.
template <int DT>
__global__ __launch_bounds__(256) void k_mlp_weights(const void* __restrict__ packed, ProbIn in, int f_first, int H,
                                                     int W, Udiv dw, const float* __restrict__ cams,
                                                     const int32_t* __restrict__ lbuf, const float4* __restrict__ geo,
                                                     const int32_t* __restrict__ cnt, int64_t cnt_stride, int c,
                                                     float* __restrict__ wpix) {
  const MlpW Wt = mlp_view(packed);
  const int fb = blockIdx.y;
  const uint32_t HW = (uint32_t)H * (uint32_t)W;
  const uint32_t p = blockIdx.x * 256u + threadIdx.x;
  const int64_t pi = (int64_t)fb * HW + p;
  const int64_t gi = (int64_t)(f_first + fb) * HW + p;
  float x[NI];
#pragma unroll
  for (int k = 0; k < NI; ++k) x[k] = 0.0f;
  bool use = false;
  if (p < HW) {
    const int y = (int)dw(p), xx = (int)(p - (uint32_t)y * (uint32_t)W);
    const int l = lbuf[pi];
    const bool ok = !in.valid || in.valid[gi];
    const float4 g = geo[pi];
    const int64_t base = (int64_t)(f_first + fb) * in.sf + (int64_t)y * in.sy + (int64_t)xx * in.sx;
    const float sc = DT == 3 ? in.scale[gi] : 1.0f;
    float ent, p1, p2;
    int best;
    prob_features<DT, false>(in, base, sc, c, ent, p1, p2, best);
    use = l >= 0 && ok;
    if (use)
      observation_phi(ent, p1, p2, g, cnt[(int64_t)fb * cnt_stride + l], xx, y, cams + 16 * (int64_t)(f_first + fb),
                      x);
  }
  const float w = mlp_wave(x, Wt);
  if (p < HW) wpix[pi] = use ? w : 0.0f;
}

// The same pass for pixel-dense class vectors (channels-last, rows and
// frames contiguous, c % 4 == 0, c <= 64): one wave per 64 consecutive
// pixels copies their class vectors -- one contiguous byte range -- into LDS
// with 16-byte loads in address order, then each lane reads its own vector
// from LDS.  Read lane by lane from global memory instead, every load
// instruction of the wave would touch a cache line per lane and each line
// would be requested again by the next load instructions.
__device__ const uint8_t kValidAll = 1;   // validity of every pixel when no mask is given

template <int DT>
__global__ __launch_bounds__(64) void k_mlp_weights_staged(const void* __restrict__ packed, ProbIn in, int f_first,
                                                           int H, int W, Udiv dw, const float* __restrict__ cams,
                                                           const int32_t* __restrict__ lbuf,
                                                           const float4* __restrict__ geo,
                                                           const int32_t* __restrict__ cnt, int64_t cnt_stride, int c,
                                                           float* __restrict__ wpix) {
  extern __shared__ float4 stage[];   // [64 * c * esz / 16]
  constexpr int esz = DT == 0 ? 4 : 1;
  const MlpW Wt = mlp_view(packed);
  const int fb = blockIdx.y;
  const int lane = threadIdx.x;
  const uint32_t HW = (uint32_t)H * (uint32_t)W;
  const uint32_t p0 = blockIdx.x * 64u, p = p0 + lane;
  const int n_px = (int)min(64u, HW - p0);
  const int64_t pi = (int64_t)fb * HW + p;
  const int64_t gi = (int64_t)(f_first + fb) * HW + p;
  // the wave's class vectors: bytes [0, n_px c esz) from the first pixel on
  const uint8_t* src8 = reinterpret_cast<const uint8_t*>(in.p) + ((int64_t)(f_first + fb) * in.sf + (int64_t)p0 * c) * esz;
  const int nbytes = n_px * c * esz, n16 = nbytes >> 4;
  const float4* src = reinterpret_cast<const float4*>(src8);
  // global -> LDS without registers: load i puts lane's 16 bytes at
  // stage[64 i + lane]
#pragma unroll
  for (int i = 0; i < 16; ++i)
    if (lane + 64 * i < n16)
      __builtin_amdgcn_global_load_lds(src + lane + 64 * i, (__attribute__((address_space(3))) void*)(stage + 64 * i),
                                       16, 0, 0);
  // a ragged last wave may end in 4-byte words (c esz is a multiple of 4)
  const int tail = (nbytes - 16 * n16) >> 2;
  if (lane < tail)
    reinterpret_cast<uint32_t*>(stage)[4 * n16 + lane] = reinterpret_cast<const uint32_t*>(src8)[4 * n16 + lane];
  // loads whose addresses do not depend on the texel row, issued behind them
  // without branches (lanes past the last pixel read the last pixel's)
  const int64_t back = lane < n_px ? 0 : lane - (n_px - 1);
  const int l = lbuf[pi - back];
  const uint8_t ok = *(in.valid ? in.valid + (gi - back) : &kValidAll);
  const float4 g = geo[pi - back];
  const float sc = DT == 3 ? in.scale[gi - back] : 1.0f;
  __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0): the LDS loads have landed
  __syncthreads();
  // features of every lane without branches (the frame count load then
  // overlaps the class loop); lanes that are not a valid covered pixel
  // enter the network with phi = 0 and write weight 0
  const bool use = lane < n_px && l >= 0 && ok != 0;
  const int n_same = cnt[(int64_t)fb * cnt_stride + max(l, 0)];
  float h = 0.0f, p1 = -__builtin_inff(), p2 = -__builtin_inff(), ent;
  int best = 0;
  vector_features<DT, false>(reinterpret_cast<const uint8_t*>(stage) + min(lane, n_px - 1) * c * esz, sc, c, h, p1,
                             p2, best);
  finish_prob_features(h, c, ent, p2);
  const int y = (int)dw(p), xx = (int)(p - (uint32_t)y * (uint32_t)W);
  float x[NI];
  observation_phi(ent, p1, p2, g, n_same, xx, y, cams + 16 * (int64_t)(f_first + fb), x);
#pragma unroll
  for (int k = 0; k < NI; ++k) x[k] = use ? x[k] : 0.0f;
  const float w = mlp_wave(x, Wt);
  if (lane < n_px) wpix[pi] = use ? w : 0.0f;
}

// Training data: features and targets (own argmax == the texel's fused label)
// of every valid covered pixel of the batch, appended in arbitrary order.
template <int DT>
__global__ __launch_bounds__(256) void k_extract(ProbIn in, int f_first, int H, int W, const float* __restrict__ cams,
                                                 const int32_t* __restrict__ lbuf, const float4* __restrict__ geo,
                                                 const int32_t* __restrict__ cnt, int64_t cnt_stride, int c,
                                                 const uint8_t* __restrict__ labels, float* __restrict__ phi_out,
                                                 float* __restrict__ tgt_out, int32_t* __restrict__ pix_out,
                                                 int64_t cap, unsigned long long* __restrict__ count) {
  const int fb = blockIdx.y;
  const int64_t HW = (int64_t)H * W;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t pi = (int64_t)fb * HW + p;
  const int64_t gi = (int64_t)(f_first + fb) * HW + p;
  bool use = false;
  int l = -1;
  if (p < HW) {
    l = lbuf[pi];
    use = l >= 0 && (!in.valid || in.valid[gi]);
  }
  const unsigned long long mask = __ballot(use);
  if (mask == 0) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll(mask) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(count, (unsigned long long)__popcll(mask));
  base = __shfl(base, leader);
  if (!use) return;
  const unsigned long long slot = base + __popcll(mask & ((1ull << lane) - 1ull));
  if ((int64_t)slot >= cap) return;
  const int y = (int)(p / W), xx = (int)(p - (int64_t)y * W);
  const int64_t pb = (int64_t)(f_first + fb) * in.sf + (int64_t)y * in.sy + (int64_t)xx * in.sx;
  const float sc = DT == 3 ? in.scale[gi] : 1.0f;
  float x[NI];
  int best;
  observation_features<DT>(in, pb, sc, c, geo[pi], cnt[(int64_t)fb * cnt_stride + l], xx, y,
                           cams + 16 * (int64_t)(f_first + fb), x, best);
#pragma unroll
  for (int k = 0; k < NI; ++k) phi_out[slot * NI + k] = x[k];
  if (tgt_out) tgt_out[slot] = (labels && labels[l] != 255 && labels[l] == best) ? 1.0f : 0.0f;
  if (pix_out) pix_out[slot] = (int32_t)((int64_t)(f_first + fb) * HW + p);
}

// ---- training gradients (vector ALU, binary32) --------------------------------------
// One 64-lane block walks `chunks` chunks of 64 observations; lane o owns
// hidden unit o of both layers.  Straight-through rounding: the backward pass
// uses the bfloat16 weights and q(h1), q(phi) of the forward pass.
__global__ __launch_bounds__(64) void k_mlp_grad(const void* __restrict__ packed, const float* __restrict__ phi,
                                                 const float* __restrict__ tgt, int64_t n, int chunks,
                                                 float inv_total, float* __restrict__ grad, float* __restrict__ loss) {
  __shared__ float sx[64][NI];          // q(phi) of the chunk's samples
  __shared__ float sh1[64][NH + 1];     // q(h1)[sample][unit]
  __shared__ float sh2[64][NH + 1];     // relu(h2)[sample][unit]
  __shared__ float sd[64][NH + 1];      // w3*h2, then d(loss)/d(h2 pre-activation)
  __shared__ uint16_t sw2[NH][NH + 2];  // W2 (bfloat16)
  __shared__ float sdz[64];
  const MlpW W = mlp_view(packed);
  const int o = threadIdx.x;
  float w1[NI], w2[NH];
#pragma unroll
  for (int k = 0; k < NI; ++k) w1[k] = bf16_val(W.W1[o * NI + k]);
#pragma unroll
  for (int i = 0; i < NH; ++i) {
    w2[i] = bf16_val(W.W2[o * NH + i]);
    sw2[o][i] = W.W2[o * NH + i];
  }
  const float b1 = W.b1[o], b2 = W.b2[o], w3 = bf16_val(W.w3[o]), b3 = W.b3[0];
  float gW1[NI], gW2[NH];
#pragma unroll
  for (int k = 0; k < NI; ++k) gW1[k] = 0.0f;
#pragma unroll
  for (int i = 0; i < NH; ++i) gW2[i] = 0.0f;
  float gb1 = 0.0f, gb2 = 0.0f, gw3 = 0.0f, gb3 = 0.0f, lsum = 0.0f;
  __syncthreads();
  for (int ch = 0; ch < chunks; ++ch) {
    const int64_t s0 = ((int64_t)blockIdx.x * chunks + ch) * 64;
    if (s0 >= n) break;
    const int64_t si = s0 + o;
    const bool live = si < n;
#pragma unroll
    for (int k = 0; k < NI; ++k) sx[o][k] = live ? bf16_val(bf16_bits(phi[si * NI + k])) : 0.0f;
    const float y = live ? tgt[si] : 0.0f;
    __syncthreads();
    uint64_t m1 = 0, m2 = 0;   // relu masks of unit o over the chunk's samples
    for (int s = 0; s < 64; ++s) {
      float a = b1;
#pragma unroll
      for (int k = 0; k < NI; ++k) a += w1[k] * sx[s][k];
      if (a > 0.0f) m1 |= 1ull << s;
      sh1[s][o] = bf16_val(bf16_bits(fmaxf(a, 0.0f)));
    }
    __syncthreads();
    for (int s = 0; s < 64; ++s) {
      float a = b2;
#pragma unroll
      for (int i = 0; i < NH; ++i) a += w2[i] * sh1[s][i];
      if (a > 0.0f) m2 |= 1ull << s;
      const float h = fmaxf(a, 0.0f);
      sh2[s][o] = h;
      sd[s][o] = w3 * h;
    }
    __syncthreads();
    {
      float z = b3;
      for (int i = 0; i < NH; ++i) z += sd[o][i];
      const float sg = 1.0f / (1.0f + expf(-z));
      // binary cross-entropy with logits, stable form
      const float l = (z > 0.0f ? z + log1pf(expf(-z)) : log1pf(expf(z))) - y * z;
      sdz[o] = live ? (sg - y) * inv_total : 0.0f;
      if (live) lsum += l * inv_total;
    }
    __syncthreads();
    for (int s = 0; s < 64; ++s) {
      const float dz = sdz[s];
      gw3 += dz * sh2[s][o];
      if (o == 0) gb3 += dz;
      const float d2 = ((m2 >> s) & 1ull) ? dz * w3 : 0.0f;
      gb2 += d2;
#pragma unroll
      for (int i = 0; i < NH; ++i) gW2[i] += d2 * sh1[s][i];
      sd[s][o] = d2;
    }
    __syncthreads();
    for (int s = 0; s < 64; ++s) {
      float a = 0.0f;
      for (int q = 0; q < NH; ++q) a += sd[s][q] * bf16_val(sw2[q][o]);
      const float d1 = ((m1 >> s) & 1ull) ? a : 0.0f;
      gb1 += d1;
#pragma unroll
      for (int k = 0; k < NI; ++k) gW1[k] += d1 * sx[s][k];
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < NI; ++k) atomicAdd(grad + OW1 + o * NI + k, gW1[k]);
  atomicAdd(grad + OB1 + o, gb1);
#pragma unroll
  for (int i = 0; i < NH; ++i) atomicAdd(grad + OW2 + o * NH + i, gW2[i]);
  atomicAdd(grad + OB2 + o, gb2);
  atomicAdd(grad + OW3 + o, gw3);
  if (o == 0) atomicAdd(grad + OB3, gb3);
  float v = lsum;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (o == 0 && loss) atomicAdd(loss, v);
}

// ---- launchers --------------------------------------------------------------------
int mlp_nparam() { return NPARAM; }
int mlp_packed_bytes() { return PACKED_BYTES; }

hipError_t launch_mlp_pack(const float* params, void* packed, hipStream_t s) {
  k_mlp_pack<<<dim3((NPARAM + 255) / 256), 256, 0, s>>>(params, reinterpret_cast<char*>(packed));
  return hipGetLastError();
}

hipError_t launch_adam(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  k_adam<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(p, m, v, g, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const void* packed, const float* phi, int64_t n, float* w, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_mlp_forward<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(packed, phi, n, w);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const void* packed, const float* phi, const float* tgt, int64_t n, float inv_total,
                           float* grad, float* loss, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  constexpr int chunks = 4;
  const int64_t blocks = (n + 64 * chunks - 1) / (64 * chunks);
  k_mlp_grad<<<dim3((unsigned)blocks), 64, 0, s>>>(packed, phi, tgt, n, chunks, inv_total, grad, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_weights(const void* packed, const ProbIn& in, int f_first, int nf, int H, int W,
                              const float* cams, const int32_t* l, const float4* g4, const int32_t* cnt,
                              int64_t cnt_stride, int c, float* wpix, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  const int64_t HW = (int64_t)H * W;
  if (HW >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  const Udiv dw = Udiv::make((uint32_t)W);
  const int64_t esz = in.dtype == 0 ? 4 : 1;
  const bool dense = in.sc == 1 && in.sx == c && in.sy == (int64_t)W * c && (c & 3) == 0 && c <= 64 &&
                     (reinterpret_cast<uintptr_t>(in.p) & 15) == 0 && ((in.sf * esz) & 15) == 0;
  if (dense) {
    dim3 g((unsigned)((HW + 63) / 64), (unsigned)nf);
    const size_t lds = (size_t)64 * c * esz;
    if (in.dtype == 0)
      k_mlp_weights_staged<0><<<g, 64, lds, s>>>(packed, in, f_first, H, W, dw, cams, l, g4, cnt, cnt_stride, c, wpix);
    else
      k_mlp_weights_staged<3><<<g, 64, lds, s>>>(packed, in, f_first, H, W, dw, cams, l, g4, cnt, cnt_stride, c, wpix);
    return hipGetLastError();
  }
  dim3 g((unsigned)((HW + 255) / 256), (unsigned)nf);
  if (in.dtype == 0)
    k_mlp_weights<0><<<g, 256, 0, s>>>(packed, in, f_first, H, W, dw, cams, l, g4, cnt, cnt_stride, c, wpix);
  else k_mlp_weights<3><<<g, 256, 0, s>>>(packed, in, f_first, H, W, dw, cams, l, g4, cnt, cnt_stride, c, wpix);
  return hipGetLastError();
}

hipError_t launch_extract(const ProbIn& in, int f_first, int nf, int H, int W, const float* cams, const int32_t* l,
                          const float4* g4, const int32_t* cnt, int64_t cnt_stride, int c, const uint8_t* labels,
                          float* phi, float* tgt, int32_t* pix, int64_t cap, unsigned long long* count, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  const int64_t HW = (int64_t)H * W;
  dim3 g((unsigned)((HW + 255) / 256), (unsigned)nf);
  if (in.dtype == 0)
    k_extract<0><<<g, 256, 0, s>>>(in, f_first, H, W, cams, l, g4, cnt, cnt_stride, c, labels, phi, tgt, pix, cap, count);
  else
    k_extract<3><<<g, 256, 0, s>>>(in, f_first, H, W, cams, l, g4, cnt, cnt_stride, c, labels, phi, tgt, pix, cap, count);
  return hipGetLastError();
}

}  // namespace lf
