// Measurement aid, not part of the library: the rate at which the GPU
// serves reads of random fixed-size segments.  A CSR sketch that visits rows
// in bucket order reads, per row, one segment of the column array and one of
// the value array at unrelated addresses, so this rate bounds it.
//
// skls_probe_segments: each group of seg_bytes / 16 lanes reads the segment
// idx[k] (16 bytes per lane) for k = 0 .. nseg - 1 and folds it into a sum,
// written to *sink only if it equals an impossible value (so the loads are
// kept).  data holds at least (max idx + 1) * seg_bytes bytes; seg_bytes is
// 16, 32, 64, 128 or 256; the launch is asynchronous on `stream`.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

template <int G>
__global__ __launch_bounds__(256) void k_segments(const float4* __restrict__ data, const int32_t* __restrict__ idx,
                                                  int64_t nseg, float* __restrict__ sink) {
  const int sub = threadIdx.x % G;
  const int64_t grp = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / G;
  const int64_t ngrp = static_cast<int64_t>(gridDim.x) * blockDim.x / G;
  float s = 0.0f;
  for (int64_t k = grp; k < nseg; k += 4 * ngrp) {
    float4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t kk = k + u * ngrp;
      v[u] = kk < nseg ? data[static_cast<int64_t>(idx[kk]) * G + sub] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) s += v[u].x + v[u].y + v[u].z + v[u].w;
  }
  if (s == -1.2345e-30f) sink[0] = s;
}

template <int G>
int launch(const void* data, const int32_t* idx, int64_t nseg, float* sink, hipStream_t s) {
  hipLaunchKernelGGL(k_segments<G>, dim3(256 * 32), dim3(256), 0, s, static_cast<const float4*>(data), idx, nseg,
                     sink);
  return hipGetLastError() == hipSuccess ? 0 : 1;
}

}  // namespace

extern "C" __attribute__((visibility("default"))) int skls_probe_segments(const void* data, const int32_t* idx,
                                                                         int64_t nseg, int32_t seg_bytes,
                                                                         float* sink, void* stream) {
  if (data == nullptr || idx == nullptr || sink == nullptr || nseg < 0) return 1;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  switch (seg_bytes) {
    case 16: return launch<1>(data, idx, nseg, sink, s);
    case 32: return launch<2>(data, idx, nseg, sink, s);
    case 64: return launch<4>(data, idx, nseg, sink, s);
    case 128: return launch<8>(data, idx, nseg, sink, s);
    case 256: return launch<16>(data, idx, nseg, sink, s);
    default: return 1;
  }
}
