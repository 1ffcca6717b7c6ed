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

__device__ __forceinline__ float2 rotate(const float2 v, float turns) {
  float s, c;
  sincospif(2.f * turns, &s, &c);
  return make_float2(v.x * c - v.y * s, v.x * s + v.y * c);
}

// The two amplitudes i0 = 2e and i1 = 2e + 1 of float4 element e.  Chunks
// 1.. of their index are equal, so the chunk-1.. table sums are shared; only
// the chunk-0 entries (and a hub on bit 0) differ.  Within a wavefront the
// 128 indices share chunks 1.., so those LDS reads are broadcasts.  Every
// table entry is a fraction of a turn in [0, 1); partial sums are folded
// back into [0, 1) so the FP32 sum keeps ~2^-23 turn resolution.
__device__ __forceinline__ float4 phase_pair(const float* __restrict__ T, const float* __restrict__ R,
                                             const PhaseArgs& a, uint64_t e, const float4 v) {
  const uint64_t i0 = 2 * e;
  const int lo0 = (int)(i0 & 255);
  int idx[kPhaseChunks];
#pragma unroll
  for (int c = 1; c < kPhaseChunks; ++c) idx[c] = (int)((i0 >> (8 * c)) & 255);
  float u = 0.f;
#pragma unroll
  for (int c = 1; c < kPhaseChunks; ++c)
    if (c < a.nch) u += T[c * 256 + idx[c]];
  u -= floorf(u);
  float t0 = u + T[lo0], t1 = u + T[lo0 + 1];
  for (int h = 0; h < a.nhubs; ++h) {
    const float* Rh = R + h * kPhaseChunks * 256;
    float sh = 0.f;
#pragma unroll
    for (int c = 1; c < kPhaseChunks; ++c)
      if (c < a.nch) sh += Rh[c * 256 + idx[c]];
    const int hb = a.hub[h];
    const float x0 = (float)((i0 >> hb) & 1), x1 = (float)(((i0 | 1) >> hb) & 1);
    t0 = fmaf(x0, sh + Rh[lo0], t0);
    t1 = fmaf(x1, sh + Rh[lo0 + 1], t1);
    t0 -= floorf(t0);
    t1 -= floorf(t1);
  }
  const float2 lo = rotate(make_float2(v.x, v.y), t0);
  const float2 hi = rotate(make_float2(v.z, v.w), t1);
  return make_float4(lo.x, lo.y, hi.x, hi.y);
}

// Two elements per thread per iteration, both loads issued before any math.
template <bool NT>
__global__ __launch_bounds__(256) void k_phase(float4* __restrict__ psi, const float4* __restrict__ tab,
                                               const PhaseArgs a) {
  extern __shared__ float4 tl4[];
  const float* tl = reinterpret_cast<const float*>(tl4);
  const int floats = kPhaseChunks * 256 * (1 + a.nhubs);
  for (int i = threadIdx.x; i < floats / 4; i += 256) tl4[i] = tab[i];
  __syncthreads();
  const float* T = tl;
  const float* R = tl + kPhaseChunks * 256;
  const uint64_t stride = (uint64_t)gridDim.x * 512;
  for (uint64_t e0 = (uint64_t)blockIdx.x * 512 + threadIdx.x; e0 < a.pairs; e0 += stride) {
    const uint64_t e1 = e0 + 256;
    const bool has1 = e1 < a.pairs;
    const float4 v0 = gld<NT>(psi + e0);
    const float4 v1 = has1 ? gld<NT>(psi + e1) : make_float4(0.f, 0.f, 0.f, 0.f);
    gst<NT>(psi + e0, phase_pair(T, R, a, e0, v0));
    if (has1) gst<NT>(psi + e1, phase_pair(T, R, a, e1, v1));
  }
}

}  // namespace

void launch_phase(int n, void* psi, const unsigned char* data, int nhubs, const int* hubs, hipStream_t st) {
  PhaseArgs a{};
  a.pairs = (uint64_t)1 << (n - 1);
  a.nch = (n + 7) / 8;
  a.nhubs = nhubs;
  for (int h = 0; h < nhubs; ++h) a.hub[h] = hubs[h];
  uint64_t blocks = (a.pairs + 511) / 512;
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
