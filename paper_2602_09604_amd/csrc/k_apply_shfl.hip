// Passes whose targets all lie in the low seven bits, with at most two of
// them in bits 1..6: the gate is applied without any gather.  Every lane
// loads one 16-byte element (amplitudes 2e and 2e + 1), so a wavefront reads
// 1 KiB contiguously; element bits 0..5 are the lane bits, i.e. state bits
// 1..6.  A target on bit 0 lives inside the element, a target on bit t in
// 1..6 in the partner lane (lane ^ 2^(t-1)), and the partner values arrive by
// cross-lane permutes (ds_bpermute), never through memory.
#include "k_common.h"

namespace sv {

namespace {
using kern::gld;
using kern::gst;

struct ShflArgs {
  uint64_t elems;   // 2^(n-1) float4 elements
  int m1, m2;       // lane xor masks of the lane targets (m2 = 0 when only one)
  int bit0;         // 1: bit 0 is a target (local bit 0)
};

// value held by lane ^ mask (a cross-lane permute; mask < 64)
__device__ __forceinline__ float lane_xor(float v, int mask) { return __shfl_xor(v, mask, 64); }

__device__ __forceinline__ float4 lane_xor4(const float4 v, int mask) {
  return make_float4(lane_xor(v.x, mask), lane_xor(v.y, mask), lane_xor(v.z, mask), lane_xor(v.w, mask));
}

__device__ __forceinline__ void cmac2(float2& acc, const float2 u, float vx, float vy) {
  acc.x = fmaf(u.x, vx, acc.x);
  acc.x = fmaf(-u.y, vy, acc.x);
  acc.y = fmaf(u.x, vy, acc.y);
  acc.y = fmaf(u.y, vx, acc.y);
}

// MODE 0: one lane target (2x2, local bit 0 = lane target); the element holds
//         two independent groups (bit 0 is not a target).
// MODE 1: bit 0 and one lane target (4x4: local bit 0 = state bit 0, local
//         bit 1 = lane target); the element holds two amplitudes of one group.
// MODE 2: two lane targets (4x4, local bits 0, 1 = lane targets m1 < m2); the
//         element holds two independent groups.
template <int MODE, bool NT>
__global__ __launch_bounds__(256) void k_apply_shfl(float4* __restrict__ psi, const float2* __restrict__ U,
                                                    const ShflArgs a) {
  const uint64_t e = ((uint64_t)blockIdx.y * gridDim.x + blockIdx.x) * 256 + threadIdx.x;
  // the grid covers whole wavefronts of real elements (elems is a multiple of 64)
  const int lane = threadIdx.x & 63;
  const float4 v = gld<NT>(psi + e);
  float4 out;
  if constexpr (MODE == 0) {
    const float4 p = lane_xor4(v, a.m1);
    const int b = (lane & a.m1) ? 1 : 0;
    const float2 us = U[b * 2 + b], up = U[b * 2 + (1 - b)];  // own and partner coefficients of row b
    float2 lo = make_float2(0.f, 0.f), hi = make_float2(0.f, 0.f);
    cmac2(lo, us, v.x, v.y);
    cmac2(lo, up, p.x, p.y);
    cmac2(hi, us, v.z, v.w);
    cmac2(hi, up, p.z, p.w);
    out = make_float4(lo.x, lo.y, hi.x, hi.y);
  } else if constexpr (MODE == 1) {
    const float4 p = lane_xor4(v, a.m1);
    const int b = (lane & a.m1) ? 1 : 0;  // local bit 1
    // own local indices 2b, 2b+1; partner's 2(1-b), 2(1-b)+1
    const int r0 = 2 * b, po = 2 * (1 - b);
    float2 o0 = make_float2(0.f, 0.f), o1 = make_float2(0.f, 0.f);
    cmac2(o0, U[r0 * 4 + r0], v.x, v.y);
    cmac2(o0, U[r0 * 4 + r0 + 1], v.z, v.w);
    cmac2(o0, U[r0 * 4 + po], p.x, p.y);
    cmac2(o0, U[r0 * 4 + po + 1], p.z, p.w);
    cmac2(o1, U[(r0 + 1) * 4 + r0], v.x, v.y);
    cmac2(o1, U[(r0 + 1) * 4 + r0 + 1], v.z, v.w);
    cmac2(o1, U[(r0 + 1) * 4 + po], p.x, p.y);
    cmac2(o1, U[(r0 + 1) * 4 + po + 1], p.z, p.w);
    out = make_float4(o0.x, o0.y, o1.x, o1.y);
  } else {
    float4 x[4];  // x[c] = this lane's group component with local index c
    const int l = ((lane & a.m1) ? 1 : 0) | ((lane & a.m2) ? 2 : 0);
    const float4 p1 = lane_xor4(v, a.m1), p2 = lane_xor4(v, a.m2), p3 = lane_xor4(v, a.m1 | a.m2);
    x[l] = v;
    x[l ^ 1] = p1;
    x[l ^ 2] = p2;
    x[l ^ 3] = p3;
    float2 lo = make_float2(0.f, 0.f), hi = make_float2(0.f, 0.f);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float2 u = U[l * 4 + c];
      cmac2(lo, u, x[c].x, x[c].y);
      cmac2(hi, u, x[c].z, x[c].w);
    }
    out = make_float4(lo.x, lo.y, hi.x, hi.y);
  }
  gst<NT>(psi + e, out);
}

template <int MODE, bool NT>
void launch_t(float4* psi, const float2* U, const ShflArgs& a, hipStream_t st) {
  const uint64_t blocks = a.elems / 256;
  const uint64_t gx = blocks < 65536 ? blocks : 65536;
  const uint64_t gy = blocks / gx;  // elems is a power of two >= 256
  hipLaunchKernelGGL((k_apply_shfl<MODE, NT>), dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, psi, U, a);
}

}  // namespace

bool shfl_eligible(int n, int k, const int* s) {
  if (n < 9 || k < 1 || k > 2) return false;
  int lane = 0, zero = 0;
  for (int j = 0; j < k; ++j) {
    if (s[j] == 0) ++zero;
    else if (s[j] <= 6) ++lane;
    else return false;
  }
  // two lane targets: only within bits 1..5 (a partner across the two halves
  // of the wavefront, bit 6, costs more permute bandwidth than the LDS form)
  if (lane == 2 && (s[0] > 5 || s[1] > 5)) return false;
  return lane >= 1 && (zero == 0 || lane == 1);
}

// The planner has checked shfl_eligible (targets sorted ascending).
void launch_shfl(const Pass& p, int n, void* psi_, const float2* U, hipStream_t st) {
  if (!shfl_eligible(n, p.k, p.s)) throw DeviceError{hipErrorInvalidValue, "k_apply_shfl: targets not in bits 0..6"};
  ShflArgs a{};
  a.elems = (uint64_t)1 << (n - 1);
  int mode;
  if (p.s[0] == 0) {
    mode = 1;
    a.m1 = 1 << (p.s[1] - 1);
  } else if (p.k == 1) {
    mode = 0;
    a.m1 = 1 << (p.s[0] - 1);
  } else {
    mode = 2;
    a.m1 = 1 << (p.s[0] - 1);
    a.m2 = 1 << (p.s[1] - 1);
  }
  float4* psi = reinterpret_cast<float4*>(psi_);
  const bool nt = n >= kern::kNtMinQubits;
  if (mode == 0) nt ? launch_t<0, true>(psi, U, a, st) : launch_t<0, false>(psi, U, a, st);
  else if (mode == 1) nt ? launch_t<1, true>(psi, U, a, st) : launch_t<1, false>(psi, U, a, st);
  else nt ? launch_t<2, true>(psi, U, a, st) : launch_t<2, false>(psi, U, a, st);
}

}  // namespace sv
