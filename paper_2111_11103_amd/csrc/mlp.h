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

namespace lf {

typedef short s4 __attribute__((ext_vector_type(4)));
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
constexpr int H1S = 68;   // LDS row stride of q(h1) in halfwords (conflict-free fragment reads)

struct WaveLds {
  uint16_t* phi;   // [64][8]
  uint16_t* h1;    // [64][H1S]
  float* logit;    // [64]
};

// Orders the LDS exchanges between the lanes of one wave: the LDS performs a
// wave's operations in issue order, so only the compiler has to keep them in
// program order (fences and a wave-level scheduling barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Evaluate the network for the 64 observations of a wave (lane = observation).
// Every lane of the wave must reach it; L is the wave's own LDS, so waves do
// not wait for each other.
__device__ inline float mlp_wave(const float (&phi)[NI], const MlpW& W, const WaveLds& L) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
#pragma unroll
  for (int k = 0; k < NI; ++k) L.phi[lane * NI + k] = bf16_bits(phi[k]);
  // B fragments: lane holds B[k = 4*grp + r][j = col] of each 16x16 tile
  s4 bw1[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    s4 t = {0, 0, 0, 0};
    if (grp < 2) {
      const uint16_t* w = W.W1 + (n * 16 + col) * NI + 4 * grp;
      t = s4{(short)w[0], (short)w[1], (short)w[2], (short)w[3]};
    }
    bw1[n] = t;
  }
  wave_lds_sync();
  // layer 1: h1[sample][unit] for 4 sample tiles x 4 unit tiles
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    s4 a = {0, 0, 0, 0};
    if (grp < 2) {
      const uint16_t* x = L.phi + (t * 16 + col) * NI + 4 * grp;
      a = s4{(short)x[0], (short)x[1], (short)x[2], (short)x[3]};
    }
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      f4 d = {0.f, 0.f, 0.f, 0.f};
      d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw1[n], d, 0, 0, 0);
      const float bias = W.b1[n * 16 + col];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float h = fmaxf(d[r] + bias, 0.0f);
        L.h1[(t * 16 + 4 * grp + r) * H1S + n * 16 + col] = bf16_bits(h);
      }
    }
  }
  wave_lds_sync();
  // layer 2 + output layer
  float part[4][4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) part[t][r] = 0.0f;
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    s4 bw2[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const uint16_t* w = W.W2 + (n * 16 + col) * NH + ks * 16 + 4 * grp;
      bw2[ks] = s4{(short)w[0], (short)w[1], (short)w[2], (short)w[3]};
    }
    const float bias = W.b2[n * 16 + col];
    const float w3 = bf16_val(W.w3[n * 16 + col]);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const uint16_t* x = L.h1 + (t * 16 + col) * H1S + ks * 16 + 4 * grp;
        const s4 a = s4{(short)x[0], (short)x[1], (short)x[2], (short)x[3]};
        d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw2[ks], d, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) part[t][r] += w3 * fmaxf(d[r] + bias, 0.0f);
    }
  }
  // sum over the 16 units a lane group holds, per sample row
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float v = part[t][r];
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 16);
      if (col == 0) L.logit[t * 16 + 4 * grp + r] = v + W.b3[0];
    }
  wave_lds_sync();
  const float z = L.logit[lane];
  return 1.0f / (1.0f + expf(-z));
}

}  // namespace lf
