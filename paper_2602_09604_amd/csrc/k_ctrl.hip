// Controlled gate passes (Eq. 4 with the control indicator 1_c): only the
// 2^(n-k-c) groups whose c control bits hold the control values are
// gathered, multiplied and scattered; every other amplitude is never read.
//
// Work item t enumerates the free bits (neither target nor control): zeros
// are inserted at every fixed bit in ascending order, then the control
// values are OR-ed in.  Consecutive work items therefore differ in the
// lowest free bit, which keeps a wavefront's accesses contiguous whenever
// bit 0 is free.
#include "k_common.h"

namespace sv {

namespace {
using namespace kern;

struct CtrlArgs {
  uint64_t groups;             // 2^(n - k - c)
  uint64_t fixed;              // targets | controls
  uint64_t cval;               // control values (bits of the control mask)
  uint64_t stride[SV_MAX_K];   // 1 << s[j], targets ascending
};

template <int K>
__global__ __launch_bounds__(256) void k_apply_ctrl(float2* __restrict__ psi, const float2* __restrict__ U,
                                                    const CtrlArgs a) {
  constexpr int D = 1 << K;
  const uint64_t t = ((uint64_t)blockIdx.y * gridDim.x + blockIdx.x) * 256 + threadIdx.x;
  if (t >= a.groups) return;
  uint64_t base = t;
  for (uint64_t m = a.fixed; m; m &= m - 1) {  // ascending fixed bits (a uniform loop)
    const uint64_t low = (m & (~m + 1)) - 1;   // ones below the lowest remaining fixed bit
    base = ((base & ~low) << 1) | (base & low);
  }
  base |= a.cval;
  float2 v[D];
#pragma unroll
  for (int l = 0; l < D; ++l) v[l] = psi[base + local_offset<K, uint64_t>(l, a.stride)];
#pragma unroll
  for (int r = 0; r < D; ++r) {
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int c = 0; c < D; ++c) cmac(acc, U[r * D + c], v[c]);
    psi[base + local_offset<K, uint64_t>(r, a.stride)] = acc;
  }
}

template <int K>
void launch_ctrl_t(float2* psi, const float2* U, const CtrlArgs& a, hipStream_t st) {
  const uint64_t blocks = (a.groups + 255) / 256;
  const uint64_t gx = blocks < 65536 ? blocks : 65536;
  const uint64_t gy = (blocks + gx - 1) / gx;
  hipLaunchKernelGGL(k_apply_ctrl<K>, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, psi, U, a);
}

}  // namespace

// The planner has checked: targets sorted, distinct and < n; controls < n,
// disjoint from the targets; cval within cmask; k + c <= n.
void launch_ctrl(const Pass& p, int n, void* psi_, const float2* U, hipStream_t st) {
  CtrlArgs a{};
  a.fixed = p.cmask;
  for (int j = 0; j < p.k; ++j) {
    a.stride[j] = (uint64_t)1 << p.s[j];
    a.fixed |= a.stride[j];
  }
  a.cval = p.cval;
  const int free_bits = n - __builtin_popcountll(a.fixed);
  if (free_bits < 0 || __builtin_popcountll(a.fixed) != p.k + __builtin_popcountll(p.cmask) ||
      (p.cval & ~p.cmask) != 0 || (n < 64 && (a.fixed >> n) != 0))
    throw DeviceError{hipErrorInvalidValue, "k_apply_ctrl: inconsistent controls"};
  a.groups = (uint64_t)1 << free_bits;
  float2* psi = reinterpret_cast<float2*>(psi_);
  switch (p.k) {
    case 1: launch_ctrl_t<1>(psi, U, a, st); break;
    case 2: launch_ctrl_t<2>(psi, U, a, st); break;
    case 3: launch_ctrl_t<3>(psi, U, a, st); break;
    case 4: launch_ctrl_t<4>(psi, U, a, st); break;
    case 5: launch_ctrl_t<5>(psi, U, a, st); break;
    case 6: launch_ctrl_t<6>(psi, U, a, st); break;
    default: throw DeviceError{hipErrorInvalidValue, "k_apply_ctrl: k outside 1..6"};
  }
}

}  // namespace sv
