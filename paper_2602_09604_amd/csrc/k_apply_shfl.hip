// Gates of up to three qubits whose targets all lie in the low seven bits:
// the gate is applied without any gather.  Every lane
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
  int m[3];         // lane xor masks of the lane targets, ascending
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

// KL lane targets (local bits BIT0 .. BIT0 + KL - 1) and, with BIT0, state
// bit 0 as local bit 0 (inside the element).  Lane l holds lane-local index
// li (its bits at the lane targets); the 2^KL - 1 partners lane ^ M(d) hold
// li ^ d.  Without BIT0 the element carries two independent groups (bit 0 =
// 0 in .xy, 1 in .zw); with BIT0 it carries local indices 2 li and 2 li + 1
// of one group.
template <int KL, bool BIT0, bool NT>
__global__ __launch_bounds__(256) void k_apply_shfl(float4* __restrict__ psi, const float2* __restrict__ U,
                                                    const ShflArgs a) {
  constexpr int DL = 1 << KL;
  constexpr int D = DL << (BIT0 ? 1 : 0);  // matrix dimension
  const uint64_t e = ((uint64_t)blockIdx.y * gridDim.x + blockIdx.x) * 256 + threadIdx.x;
  // the grid covers whole wavefronts of real elements (2^(n-1) is a multiple of 256)
  const int lane = threadIdx.x & 63;
  int li = 0;
#pragma unroll
  for (int j = 0; j < KL; ++j) li |= ((lane & a.m[j]) ? 1 : 0) << j;
  const float4 v = gld<NT>(psi + e);
  float2 lo = make_float2(0.f, 0.f), hi = make_float2(0.f, 0.f);
#pragma unroll
  for (int d = 0; d < DL; ++d) {  // partner lane ^ M(d) holds lane-local index c = li ^ d
    int mask = 0;
#pragma unroll
    for (int j = 0; j < KL; ++j)
      if ((d >> j) & 1) mask |= a.m[j];
    const float4 w = d == 0 ? v : lane_xor4(v, mask);
    const int c = li ^ d;
    if constexpr (!BIT0) {
      const float2 u = U[li * D + c];
      cmac2(lo, u, w.x, w.y);
      cmac2(hi, u, w.z, w.w);
    } else {
      const int r0 = 2 * li;
      cmac2(lo, U[r0 * D + 2 * c], w.x, w.y);
      cmac2(lo, U[r0 * D + 2 * c + 1], w.z, w.w);
      cmac2(hi, U[(r0 + 1) * D + 2 * c], w.x, w.y);
      cmac2(hi, U[(r0 + 1) * D + 2 * c + 1], w.z, w.w);
    }
  }
  gst<NT>(psi + e, make_float4(lo.x, lo.y, hi.x, hi.y));
}

template <int KL, bool BIT0, bool NT>
void launch_t(float4* psi, const float2* U, const ShflArgs& a, uint64_t elems, hipStream_t st) {
  const uint64_t blocks = elems / 256;
  const uint64_t gx = blocks < 65536 ? blocks : 65536;
  const uint64_t gy = blocks / gx;  // elems is a power of two >= 256
  hipLaunchKernelGGL((k_apply_shfl<KL, BIT0, NT>), dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, psi, U, a);
}

template <int KL, bool BIT0>
void launch_kl(float4* psi, const float2* U, const ShflArgs& a, uint64_t elems, bool nt, hipStream_t st) {
  if (nt) launch_t<KL, BIT0, true>(psi, U, a, elems, st);
  else launch_t<KL, BIT0, false>(psi, U, a, elems, st);
}

}  // namespace

// k <= 3 gates on bits 0..6 with one to three lane targets (bits 1..6); two
// or more lane targets only within bits 1..5 (a partner across the two halves
// of the wavefront, bit 6, costs more permute bandwidth than it saves).
bool shfl_eligible(int n, int k, const int* s) {
  if (n < 9 || k < 1 || k > 3) return false;
  int lane = 0, top = 0;
  for (int j = 0; j < k; ++j) {
    if (s[j] == 0) continue;
    if (s[j] <= 6) ++lane, top = s[j] > top ? s[j] : top;
    else return false;
  }
  if (lane == 0 || (lane >= 2 && top > 5)) return false;
  return true;
}

// The planner has checked shfl_eligible (targets sorted ascending).
void launch_shfl(const Pass& p, int n, void* psi_, const float2* U, hipStream_t st) {
  if (!shfl_eligible(n, p.k, p.s)) throw DeviceError{hipErrorInvalidValue, "k_apply_shfl: targets not eligible"};
  ShflArgs a{};
  const bool bit0 = p.s[0] == 0;
  const int kl = p.k - (bit0 ? 1 : 0);
  for (int j = 0; j < kl; ++j) a.m[j] = 1 << (p.s[j + (bit0 ? 1 : 0)] - 1);
  float4* psi = reinterpret_cast<float4*>(psi_);
  const uint64_t elems = (uint64_t)1 << (n - 1);
  const bool nt = n >= kern::kNtMinQubits;
  switch (kl * 2 + (bit0 ? 1 : 0)) {
    case 2: launch_kl<1, false>(psi, U, a, elems, nt, st); break;
    case 3: launch_kl<1, true>(psi, U, a, elems, nt, st); break;
    case 4: launch_kl<2, false>(psi, U, a, elems, nt, st); break;
    case 5: launch_kl<2, true>(psi, U, a, elems, nt, st); break;
    case 6: launch_kl<3, false>(psi, U, a, elems, nt, st); break;
    default: throw DeviceError{hipErrorInvalidValue, "k_apply_shfl: lane targets"};
  }
  SV_HIP(hipGetLastError());
}

}  // namespace sv
