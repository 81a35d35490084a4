// Mesh loading: uv frames, texel counts and row offsets (Sections 3.1, 3.3.2),
// culling bounds, small fill kernels.
#include "internal.h"
#include "spec.h"

namespace lf {

// uv origin = the vertex whose interior angle is closest to 90 degrees:
// smallest (a.b)^2 / ((a.a)(b.b)) over the three corners (binary32, first
// minimum wins).  faces_uv = (origin, next, next-next) in input order, and
// tri_v the three positions in that order.
__global__ __launch_bounds__(256) void k_mesh_prep(MeshDev m, const int32_t* __restrict__ faces) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.T) return;
  int idx[3];
  bool bad = false;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    idx[k] = faces[3 * t + k];
    bad |= (idx[k] < 0) | ((int64_t)idx[k] >= m.V);
  }
  if (m.s_face) bad |= m.s_face[t] < 1;
  if (bad) {
    atomicOr(m.err, 1);
    m.faces_uv[3 * t + 0] = 0;
    m.faces_uv[3 * t + 1] = 0;
    m.faces_uv[3 * t + 2] = 0;
    for (int k = 0; k < 3; ++k) m.tri_v[3 * t + k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    return;
  }
  V3 P[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float* q = m.verts + 3 * (int64_t)idx[k];
    P[k] = V3{q[0], q[1], q[2]};
  }
  float cosq[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    V3 a = sub3(P[(k + 1) % 3], P[k]);
    V3 b = sub3(P[(k + 2) % 3], P[k]);
    float ab = dot3(a, b);
    cosq[k] = (ab * ab) / (dot3(a, a) * dot3(b, b));
  }
  int o = 0;
  if (cosq[1] < cosq[o]) o = 1;
  if (cosq[2] < cosq[o]) o = 2;
  m.faces_uv[3 * t + 0] = idx[o];
  m.faces_uv[3 * t + 1] = idx[(o + 1) % 3];
  m.faces_uv[3 * t + 2] = idx[(o + 2) % 3];
  // triangle-major copy of the positions: one 48-byte read per triangle
  const V3 A = P[o], B = P[(o + 1) % 3], C = P[(o + 2) % 3];
  m.tri_v[3 * t + 0] = make_float4(A.x, A.y, A.z, B.x);
  m.tri_v[3 * t + 1] = make_float4(B.y, B.z, C.x, C.y);
  m.tri_v[3 * t + 2] = make_float4(C.z, 0.0f, 0.0f, 0.0f);
}

hipError_t launch_mesh_prep(const MeshDev& m, const int32_t* faces, hipStream_t s) {
  if (m.T == 0) return hipSuccess;
  k_mesh_prep<<<dim3((unsigned)((m.T + 255) / 256)), dim3(256), 0, s>>>(m, faces);
  return hipGetLastError();
}

// ---- exclusive prefix sum of per-face texel counts (int64) ----------------
constexpr int kScanChunk = 4096;

__global__ __launch_bounds__(256) void k_chunk_sums(MeshDev m, int64_t* sums) {
  __shared__ int64_t red[256];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  int64_t acc = 0;
  for (int i = threadIdx.x; i < kScanChunk; i += 256) {
    int64_t t = base + i;
    if (t < m.T) acc += texel_count(max(m.s_face[t], 1), m.split);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

__global__ void k_scan_sums(int64_t* sums, int64_t n) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t acc = 0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t v = sums[i];
    sums[i] = acc;
    acc += v;
  }
  sums[n] = acc;
}

__global__ __launch_bounds__(256) void k_chunk_scan(MeshDev m, const int64_t* sums) {
  __shared__ int64_t part[256];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  constexpr int per = kScanChunk / 256;
  int64_t loc[per];
  int64_t acc = 0;
#pragma unroll
  for (int i = 0; i < per; ++i) {
    int64_t t = base + (int64_t)threadIdx.x * per + i;
    int64_t v = (t < m.T) ? texel_count(max(m.s_face[t], 1), m.split) : 0;
    loc[i] = acc;
    acc += v;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  // inclusive scan of the 256 thread totals
  for (int d = 1; d < 256; d <<= 1) {
    int64_t v = (threadIdx.x >= d) ? part[threadIdx.x - d] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  const int64_t pre = sums[blockIdx.x] + part[threadIdx.x] - acc;
#pragma unroll
  for (int i = 0; i < per; ++i) {
    int64_t t = base + (int64_t)threadIdx.x * per + i;
    if (t < m.T) m.off[t] = pre + loc[i];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) m.off[m.T] = sums[gridDim.x];
}

hipError_t launch_offsets(const MeshDev& m, int32_t* scratch, hipStream_t s) {
  if (!m.off) return hipSuccess;
  int64_t nch = (m.T + kScanChunk - 1) / kScanChunk;
  if (nch == 0) nch = 1;
  int64_t* sums = reinterpret_cast<int64_t*>(scratch);
  k_chunk_sums<<<dim3((unsigned)nch), dim3(256), 0, s>>>(m, sums);
  k_scan_sums<<<1, 1, 0, s>>>(sums, nch);
  k_chunk_scan<<<dim3((unsigned)nch), dim3(256), 0, s>>>(m, sums);
  return hipGetLastError();
}

// ---- culling bounds: axis-aligned box of each cluster of 64 triangles ------
__global__ __launch_bounds__(64) void k_cluster_boxes(MeshDev m) {
  const int64_t cl = blockIdx.x;
  const int64_t t = cl * kClusterTris + threadIdx.x;
  float lo[3] = {3.0e38f, 3.0e38f, 3.0e38f}, hi[3] = {-3.0e38f, -3.0e38f, -3.0e38f};
  if (t < m.T) {
    for (int k = 0; k < 3; ++k) {
      const float* q = m.verts + 3 * (int64_t)m.faces_uv[3 * t + k];
      for (int d = 0; d < 3; ++d) {
        lo[d] = fminf(lo[d], q[d]);
        hi[d] = fmaxf(hi[d], q[d]);
      }
    }
  }
  for (int d = 0; d < 3; ++d) {
    for (int w = 32; w > 0; w >>= 1) {
      lo[d] = fminf(lo[d], __shfl_xor(lo[d], w));
      hi[d] = fmaxf(hi[d], __shfl_xor(hi[d], w));
    }
  }
  if (threadIdx.x == 0) {
    float* b = m.cl_box + 8 * cl;
    b[0] = lo[0]; b[1] = lo[1]; b[2] = lo[2];
    b[3] = hi[0]; b[4] = hi[1]; b[5] = hi[2];
    b[6] = 0.0f; b[7] = 0.0f;
  }
}

hipError_t launch_cluster_boxes(const MeshDev& m, hipStream_t s) {
  if (m.n_clusters == 0) return hipSuccess;
  k_cluster_boxes<<<dim3((unsigned)m.n_clusters), dim3(64), 0, s>>>(m);
  return hipGetLastError();
}

// ---- fills -----------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

__global__ __launch_bounds__(256) void k_zero_u32(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0u;
}

__global__ __launch_bounds__(256) void k_zero_u8(uint8_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0;
}

static unsigned grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill_u64<<<grid_for(n), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

// Zero-fill with a kernel (no memset nodes, so the call is safe under graph capture).
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t s) {
  if (bytes <= 0) return hipSuccess;
  if ((bytes & 3) == 0 && (reinterpret_cast<uintptr_t>(p) & 3) == 0)
    k_zero_u32<<<grid_for(bytes / 4), 256, 0, s>>>(reinterpret_cast<uint32_t*>(p), bytes / 4);
  else
    k_zero_u8<<<grid_for(bytes), 256, 0, s>>>(reinterpret_cast<uint8_t*>(p), bytes);
  return hipGetLastError();
}

}  // namespace lf
