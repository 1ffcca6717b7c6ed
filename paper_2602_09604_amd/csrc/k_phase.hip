// Phase-only pass: psi[i] *= exp(2 pi i theta(i)) with theta (in turns) a
// quadratic polynomial of the bits of i, evaluated from LDS chunk tables
// (see phase.cpp).  An elementwise, perfectly coalesced sweep: no groups, no
// matrix, one read and one write per amplitude.
#include "k_common.h"

namespace sv {

namespace {
using kern::gld;
using kern::gst;

struct PhaseArgs {
  uint64_t pairs;                // float4 elements
  int nch;                       // 8-bit chunks that carry index bits
  int nhubs;
  int hub[kPhaseHubs];
};

__device__ __forceinline__ float theta_turns(const float* __restrict__ tl, const PhaseArgs& a, uint64_t i) {
  // every table entry is a fraction of a turn in [0, 1); partial sums are
  // folded back into [0, 1) so the FP32 sum keeps ~2^-23 turn resolution
  float t = 0.f;
  int idx[kPhaseChunks];
#pragma unroll
  for (int c = 0; c < kPhaseChunks; ++c) {
    idx[c] = (int)((i >> (8 * c)) & 255);
    if (c < a.nch) t += tl[c * 256 + idx[c]];
  }
  t -= floorf(t);
  const float* R = tl + kPhaseChunks * 256;
  for (int h = 0; h < a.nhubs; ++h) {
    if (!((i >> a.hub[h]) & 1)) continue;
#pragma unroll
    for (int c = 0; c < kPhaseChunks; ++c)
      if (c < a.nch) t += R[(h * kPhaseChunks + c) * 256 + idx[c]];
    t -= floorf(t);
  }
  return t;
}

__device__ __forceinline__ float2 rotate(const float2 v, float turns) {
  float s, c;
  sincospif(2.f * turns, &s, &c);
  return make_float2(v.x * c - v.y * s, v.x * s + v.y * c);
}

template <bool NT>
__global__ __launch_bounds__(256) void k_phase(float4* __restrict__ psi, const float4* __restrict__ tab,
                                               const PhaseArgs a) {
  extern __shared__ float4 tl4[];
  const float* tl = reinterpret_cast<const float*>(tl4);
  const int floats = kPhaseChunks * 256 * (1 + a.nhubs);
  for (int i = threadIdx.x; i < floats / 4; i += 256) tl4[i] = tab[i];
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < a.pairs; e += stride) {
    const float4 v = gld<NT>(psi + e);
    const float2 lo = rotate(make_float2(v.x, v.y), theta_turns(tl, a, 2 * e));
    const float2 hi = rotate(make_float2(v.z, v.w), theta_turns(tl, a, 2 * e + 1));
    gst<NT>(psi + e, make_float4(lo.x, lo.y, hi.x, hi.y));
  }
}

}  // namespace

void launch_phase(int n, void* psi, const unsigned char* data, int nhubs, const int* hubs, hipStream_t st) {
  PhaseArgs a{};
  a.pairs = (uint64_t)1 << (n - 1);
  a.nch = (n + 7) / 8;
  a.nhubs = nhubs;
  for (int h = 0; h < nhubs; ++h) a.hub[h] = hubs[h];
  uint64_t blocks = (a.pairs + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  const size_t lds = sizeof(float) * kPhaseChunks * 256 * (1 + nhubs);
  if (n >= kern::kNtMinQubits)
    hipLaunchKernelGGL(k_phase<true>, dim3((unsigned)blocks), dim3(256), lds, st, (float4*)psi,
                       (const float4*)data, a);
  else
    hipLaunchKernelGGL(k_phase<false>, dim3((unsigned)blocks), dim3(256), lds, st, (float4*)psi,
                       (const float4*)data, a);
  SV_HIP(hipGetLastError());
}

}  // namespace sv
