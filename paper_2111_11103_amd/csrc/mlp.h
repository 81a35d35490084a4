// The learned per-observation weight's network (a generalisation of the
// fixed weights w^(P), w^(I) of Section 3.2.2): parameter layouts and the
// matrix-core evaluation of 64 observations by one wave, shared by the
// network kernels and the gather that weights observations as it sums them.
//
//   h1 = relu(W1 q(phi) + b1)   (64 x 8)
//   h2 = relu(W2 q(h1) + b2)    (64 x 64)
//   w  = sigmoid(w3 . h2 + b3)
// q = round to bfloat16; W1, W2, w3 are bfloat16, biases and accumulation
// binary32.
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace lf {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int NI = 8, NH = 64;
// master (binary32) layout
constexpr int OW1 = 0, OB1 = OW1 + NH * NI, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH, OB3 = OW3 + NH;
constexpr int NPARAM = OB3 + 1;
// packed compute layout (bytes)
constexpr int PW1 = 0, PW2 = PW1 + NH * NI * 2, PW3 = PW2 + NH * NH * 2, PB1 = PW3 + NH * 2, PB2 = PB1 + NH * 4,
              PB3 = PB2 + NH * 4, PACKED_BYTES = 10240;
static_assert(PB3 + 4 <= PACKED_BYTES, "packed layout");

__device__ __forceinline__ uint16_t bf16_bits(float x) {
  const __hip_bfloat16 b = __float2bfloat16(x);   // round to nearest even
  return *reinterpret_cast<const uint16_t*>(&b);
}
__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

struct MlpW {
  const uint16_t* W1;
  const uint16_t* W2;
  const uint16_t* w3;
  const float* b1;
  const float* b2;
  const float* b3;
};

__host__ __device__ inline MlpW mlp_view(const void* packed) {
  const char* p = reinterpret_cast<const char*>(packed);
  return MlpW{reinterpret_cast<const uint16_t*>(p + PW1), reinterpret_cast<const uint16_t*>(p + PW2),
              reinterpret_cast<const uint16_t*>(p + PW3), reinterpret_cast<const float*>(p + PB1),
              reinterpret_cast<const float*>(p + PB2), reinterpret_cast<const float*>(p + PB3)};
}

// ---- inference on the matrix cores ---------------------------------------------
// Both layers are computed transposed (hidden unit x observation), so that a
// layer's output fragment is, lane for lane, the next layer's B operand: in
// a 16x16x16 product lane (col, grp) holds D[4 grp + r][col], r = 0..3, and
// takes B[4 grp + r][col]; q(h1) never leaves the registers.  The hidden
// layer contracts 32 units per 16x16x32 product: a lane's eight B values are
// its fragments of two unit tiles, and its eight A values are the weights of
// those same eight units (a contraction does not depend on the order in
// which its index is laid over lanes and slots, as long as A and B agree).
// The input fragments take q(phi) of observation 16 t + col from that lane
// by permutes.  No LDS is used, so waves do not wait for each other.

__device__ __forceinline__ s4 pack_s4(uint32_t lo, uint32_t hi) {
  return s4{(short)(lo & 0xffffu), (short)(lo >> 16), (short)(hi & 0xffffu), (short)(hi >> 16)};
}
// eight bfloat16 operands of a 16x16x32 product: tile a's four, then tile b's
__device__ __forceinline__ bf8 join_bf8(s4 a, s4 b) {
  return __builtin_bit_cast(bf8, (s8)__builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7));
}

// Evaluate the network for the observations of a wave (lane = observation).
// Every lane of the wave must reach it.  Only the first nt (wave-uniform,
// 1..4) groups of 16 lanes are evaluated; lanes from 16 nt on get an
// unspecified value.
__device__ inline float mlp_wave(const float (&phi)[NI], const MlpW& W, int nt = 4) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  // q(phi) of this lane, two features per word
  uint32_t qp[NI / 2];
#pragma unroll
  for (int k = 0; k < NI / 2; ++k) qp[k] = (uint32_t)bf16_bits(phi[2 * k]) | ((uint32_t)bf16_bits(phi[2 * k + 1]) << 16);
  // layer 1: A = W1 tile n (unit 16 n + col, inputs 4 grp .. 4 grp + 3; K padded 8 -> 16)
  s4 aw1[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    s4 v = {0, 0, 0, 0};
    if (grp < 2) {
      const uint16_t* w = W.W1 + (n * 16 + col) * NI + 4 * grp;
      v = s4{(short)w[0], (short)w[1], (short)w[2], (short)w[3]};
    }
    aw1[n] = v;
  }
  float b1v[4][4];
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int r = 0; r < 4; ++r) b1v[n][r] = W.b1[n * 16 + 4 * grp + r];
  s4 h1[4][4];   // [unit tile][observation tile]: q(h1) of units 16 n + 4 grp + r, observation 16 t + col
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (t < nt) {
      const int src = t * 16 + col;
      uint32_t q[NI / 2];
#pragma unroll
      for (int k = 0; k < NI / 2; ++k) q[k] = (uint32_t)__shfl((int)qp[k], src);
      const s4 bphi = grp == 0 ? pack_s4(q[0], q[1]) : grp == 1 ? pack_s4(q[2], q[3]) : s4{0, 0, 0, 0};
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        f4 d = {b1v[n][0], b1v[n][1], b1v[n][2], b1v[n][3]};   // bias enters as the accumulator
        d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aw1[n], bphi, d, 0, 0, 0);
        uint32_t lo = (uint32_t)bf16_bits(fmaxf(d[0], 0.0f)) | ((uint32_t)bf16_bits(fmaxf(d[1], 0.0f)) << 16);
        uint32_t hi = (uint32_t)bf16_bits(fmaxf(d[2], 0.0f)) | ((uint32_t)bf16_bits(fmaxf(d[3], 0.0f)) << 16);
        h1[n][t] = pack_s4(lo, hi);
      }
    }
  }
  // layer 2 + output layer: A = W2 tiles (n2, 2 k2), (n2, 2 k2 + 1), B = q(h1)
  // tiles (2 k2, t), (2 k2 + 1, t): units 32 k2 + 4 grp + r and
  // 32 k2 + 16 + 4 grp + r of output unit 16 n2 + col
  float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    bf8 aw2[2];
#pragma unroll
    for (int k2 = 0; k2 < 2; ++k2) {
      const uint16_t* w = W.W2 + (n2 * 16 + col) * NH + k2 * 32 + 4 * grp;
      aw2[k2] = join_bf8(s4{(short)w[0], (short)w[1], (short)w[2], (short)w[3]},
                         s4{(short)w[16], (short)w[17], (short)w[18], (short)w[19]});
    }
    float b2v[4], w3v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      b2v[r] = W.b2[n2 * 16 + 4 * grp + r];
      w3v[r] = bf16_val(W.w3[n2 * 16 + 4 * grp + r]);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t < nt) {
        f4 d = {b2v[0], b2v[1], b2v[2], b2v[3]};
#pragma unroll
        for (int k2 = 0; k2 < 2; ++k2)
          d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw2[k2], join_bf8(h1[2 * k2][t], h1[2 * k2 + 1][t]), d, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) part[t] = fmaf(w3v[r], fmaxf(d[r], 0.0f), part[t]);
      }
    }
  }
  // sum over the four lane groups (units 4 grp + r of every tile); lane
  // 16 grp + col is observation 16 t + col with t = grp
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    part[t] += __shfl_xor(part[t], 16);
    part[t] += __shfl_xor(part[t], 32);
  }
  const float z = (grp == 0 ? part[0] : grp == 1 ? part[1] : grp == 2 ? part[2] : part[3]) + W.b3[0];
  return 1.0f / (1.0f + expf(-z));
}

// ---- features ---------------------------------------------------------------------
// Probability features of pixel (frame f, y, x): normalised entropy, top-1,
// top-1 minus top-2.  Also returns the first maximal class (BEST).
// Running entropy / top-2 / first-argmax update with class j's probability,
// without branches.  The entropy is accumulated in bits with the hardware
// base-2 logarithm (normalised by log2 c below, the same value as nats /
// ln c); a probability below the smallest normal binary32 enters the
// logarithm at that bound (its term is under 1.5e-36, and 0 for p = 0).
// Top-2 counts a repeated maximum twice: p2 = median(p2, p1, p) is the
// second largest of {p2 <= p1, p}.
template <bool BEST>
__device__ __forceinline__ void prob_step(float p, int j, float& h, float& p1, float& p2, int& best) {
  h = fmaf(-p, __log2f(fmaxf(p, 1.17549435e-38f)), h);
  if constexpr (BEST) best = p > p1 ? j : best;
  p2 = __builtin_amdgcn_fmed3f(p2, p1, p);
  p1 = fmaxf(p1, p);
}

// Entropy partial of four consecutive classes j .. j + 3, summed in class
// order from 0, with the running top-2 and first argmax.
template <bool BEST>
__device__ __forceinline__ float chunk_entropy(float a, float b, float cc, float d, int j, float& p1, float& p2,
                                               int& best) {
  float s = 0.0f;
  prob_step<BEST>(a, j, s, p1, p2, best);
  prob_step<BEST>(b, j + 1, s, p1, p2, best);
  prob_step<BEST>(cc, j + 2, s, p1, p2, best);
  prob_step<BEST>(d, j + 3, s, p1, p2, best);
  return s;
}

// The order in which a class vector's entropy is summed (c % 4 == 0,
// c <= 64): partials s[q] of the four-class chunks (slots past the vector
// hold 0); lane sums t_j = ((s[j] + s[j + 4]) + s[j + 8]) + s[j + 12],
// j = 0..3; then (t_0 + t_1) + (t_2 + t_3).  It is the order of four lanes
// each summing chunks j, j + 4, ... of a vector and reducing by a butterfly,
// so a vector read by one lane and a vector read by four give the same bits.
__device__ __forceinline__ float chunk_order_sum(const float (&s)[16]) {
  float t[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) t[j] = ((s[j] + s[j + 4]) + s[j + 8]) + s[j + 12];
  return (t[0] + t[1]) + (t[2] + t[3]);
}

// Entropy sum h, top-2 and first argmax over a contiguous class vector of c
// (c % 4 == 0, c <= 64) values: FP32, or E4M3 codes times `scale`, four per
// 32-bit word.  `src` may point to global memory or LDS; every load of the
// vector is issued first.
template <int DT, bool BEST, typename P>
__device__ __forceinline__ void vector_features(const P* src, float scale, int c, float& h, float& p1, float& p2,
                                                int& best) {
  float s[16];
  if constexpr (DT == 0) {
    const float4* s4p = reinterpret_cast<const float4*>(src);
    float4 v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (4 * q < c) v[q] = s4p[q];
#pragma unroll
    for (int q = 0; q < 16; ++q)
      s[q] = 4 * q < c ? chunk_entropy<BEST>(v[q].x, v[q].y, v[q].z, v[q].w, 4 * q, p1, p2, best) : 0.0f;
  } else {
    const uint32_t* s1p = reinterpret_cast<const uint32_t*>(src);
    uint32_t v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (4 * q < c) v[q] = s1p[q];
#pragma unroll
    for (int q = 0; q < 16; ++q)
      s[q] = 4 * q < c ? chunk_entropy<BEST>(fp8_e4m3_byte<0>(v[q]) * scale, fp8_e4m3_byte<1>(v[q]) * scale,
                                             fp8_e4m3_byte<2>(v[q]) * scale, fp8_e4m3_byte<3>(v[q]) * scale, 4 * q,
                                             p1, p2, best)
                       : 0.0f;
  }
  h = chunk_order_sum(s);
}

// One step of the four-lane butterfly of the chunked order above: this
// lane's entropy partial and top-2 merged with those of the lane DPP control
// CTRL names.  With p1 >= p2 and o1 >= o2 the second largest of the four is
// max(min(p1, o1), max(p2, o2)) = median(p1, o1, max(p2, o2)).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ void butterfly_step(float& h, float& p1, float& p2) {
  const float oh = dpp_f<CTRL>(h), o1 = dpp_f<CTRL>(p1), o2 = dpp_f<CTRL>(p2);
  h = h + oh;
  p2 = __builtin_amdgcn_fmed3f(p1, o1, fmaxf(p2, o2));
  p1 = fmaxf(p1, o1);
}
// Every lane of a wave must take part; afterwards each lane holds its quad's
// entropy sum (lane sums t_j added as (t_0 + t_1) + (t_2 + t_3)) and top-2.
__device__ __forceinline__ void butterfly4(float& h, float& p1, float& p2) {
  butterfly_step<0xb1>(h, p1, p2);   // quad_perm [1, 0, 3, 2]
  butterfly_step<0x4e>(h, p1, p2);   // quad_perm [2, 3, 0, 1]
}

// Normalised entropy from the entropy sum h (bits); top-2 is 0 for c < 2.
// Hardware logarithm and reciprocal (about one unit in the last place each).
__device__ __forceinline__ void finish_prob_features(float h, int c, float& ent, float& p2) {
  if (c < 2) p2 = 0.0f;
  ent = c > 1 ? h * __builtin_amdgcn_rcpf(__log2f((float)c)) : 0.0f;
}

template <int DT, bool BEST>
__device__ __forceinline__ void prob_features(const ProbIn& in, int64_t base, float scale, int c, float& ent, float& p1,
                                              float& p2, int& best) {
  float h = 0.0f;
  p1 = -__builtin_inff();
  p2 = -__builtin_inff();
  best = 0;
  const int64_t esz = DT == 0 ? 4 : 1;
  const bool vec = in.sc == 1 && (c & 3) == 0 && c <= 64 &&
                   ((reinterpret_cast<uintptr_t>(in.p) + base * esz) & (4 * esz - 1)) == 0;
  if (vec) {
    vector_features<DT, BEST>(reinterpret_cast<const uint8_t*>(in.p) + base * esz, scale, c, h, p1, p2, best);
  } else if ((c & 3) == 0 && c <= 64) {
    // strided classes, summed in the chunked order of the vector path
    float s[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      if (4 * q < c) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int64_t o = base + (int64_t)(4 * q + k) * in.sc;
          if constexpr (DT == 0) v[k] = reinterpret_cast<const float*>(in.p)[o];
          else v[k] = fp8_e4m3(reinterpret_cast<const uint8_t*>(in.p)[o]) * scale;
        }
      }
      s[q] = 4 * q < c ? chunk_entropy<BEST>(v[0], v[1], v[2], v[3], 4 * q, p1, p2, best) : 0.0f;
    }
    h = chunk_order_sum(s);
  } else {
    for (int j = 0; j < c; ++j) {
      float p;
      if constexpr (DT == 0) {
        p = reinterpret_cast<const float*>(in.p)[base + (int64_t)j * in.sc];
      } else {
        p = fp8_e4m3(reinterpret_cast<const uint8_t*>(in.p)[base + (int64_t)j * in.sc]) * scale;
      }
      prob_step<BEST>(p, j, h, p1, p2, best);
    }
  }
  finish_prob_features(h, c, ent, p2);
}

// phi of one observation from the renderer's per-pixel geometry (cos of the
// viewing angle, z/(1+z), centroid closeness), its frame count, its pixel
// position and the probability features (normalised entropy, top-1, top-2).
// ln n / ln 64 = log2 n / 6; the radial distance with the hardware square
// root and reciprocal (about one unit in the last place each).
__device__ __forceinline__ void observation_phi(float ent, float p1, float p2, float4 geo, int n_same, int x, int y,
                                                const float* cam, float (&phi)[NI]) {
  phi[0] = geo.x;
  phi[1] = geo.y;
  phi[2] = ent;
  phi[3] = p1;
  phi[4] = p1 - p2;
  phi[5] = geo.z;
  phi[6] = fminf(__log2f((float)max(n_same, 1)) * (1.0f / 6.0f), 2.0f);
  const float cx = cam[2], cy = cam[3];
  const float dx = (float)x + 0.5f - cx, dy = (float)y + 0.5f - cy;
  phi[7] = __builtin_amdgcn_sqrtf(dx * dx + dy * dy) * __builtin_amdgcn_rsqf(cx * cx + cy * cy);
}

template <int DT, bool BEST = true>
__device__ __forceinline__ void observation_features(const ProbIn& in, int64_t base, float scale, int c, float4 geo,
                                                     int n_same, int x, int y, const float* cam, float (&phi)[NI],
                                                     int& best) {
  float ent, p1, p2;
  prob_features<DT, BEST>(in, base, scale, c, ent, p1, p2, best);
  observation_phi(ent, p1, p2, geo, n_same, x, y, cam, phi);
}

}  // namespace lf
