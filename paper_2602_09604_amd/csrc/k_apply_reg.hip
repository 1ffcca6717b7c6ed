// Register-resident gate passes (see k_common.h for the scheme).
#include "k_common.h"

namespace sv {

namespace {
using namespace kern;

template <typename IDX>
struct RegArgs {
  IDX groups;             // number of lane work items
  IDX lowmask[SV_MAX_K];  // insertion masks of the K element-space targets, ascending
  IDX stride[SV_MAX_K];   // element stride of local bit j
};

// MODE 0 (PAIR): no target on bit 0.  Elements are float4 = amplitudes
//   (2p, 2p+1), i.e. two groups that differ only in bit 0; K = k targets in
//   element space at s[j]-1.  Each lane applies U to both groups.
// MODE 1 (Q0):   bit 0 is target 0.  The float4 holds local indices 2l'
//   and 2l'+1; K = k-1 element-space targets at s[j]-1 for j >= 1.
// MODE 2 (ONE):  float2 elements, one group per lane, K = k targets at s[j].
template <int K, int MODE, typename IDX, bool NT>
__global__ __launch_bounds__(256) void k_apply_reg(void* __restrict__ psi_,
                                                   const float2* __restrict__ U,
                                                   const RegArgs<IDX> a) {
  constexpr int D = 1 << K;  // loads per lane
  const IDX g = ((IDX)blockIdx.y * gridDim.x + blockIdx.x) * 256 + threadIdx.x;
  if (g >= a.groups) return;
  const IDX base = insert_zeros<K, IDX>(g, a.lowmask);
  if constexpr (MODE == 2) {
    float2* __restrict__ psi = reinterpret_cast<float2*>(psi_);
    float2 v[D];
#pragma unroll
    for (int l = 0; l < D; ++l) v[l] = gld<NT>(psi + base + local_offset<K, IDX>(l, a.stride));
#pragma unroll
    for (int r = 0; r < D; ++r) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int c = 0; c < D; ++c) cmac(acc, U[r * D + c], v[c]);
      gst<NT>(psi + base + local_offset<K, IDX>(r, a.stride), acc);
    }
  } else {
    float4* __restrict__ psi = reinterpret_cast<float4*>(psi_);
    float4 v[D];
#pragma unroll
    for (int l = 0; l < D; ++l) v[l] = gld<NT>(psi + base + local_offset<K, IDX>(l, a.stride));
#pragma unroll
    for (int r = 0; r < D; ++r) gst<NT>(psi + base + local_offset<K, IDX>(r, a.stride), pair_row<K, MODE>(v, U, r));
  }
}

template <typename IDX, bool NT, int K, int MODE>
void launch_reg_t(void* psi, const float2* U, const RegArgs<IDX>& a, hipStream_t st) {
  // 2-D grid keeps blocks * 256 below 2^32 work-items per dimension
  const uint64_t blocks = ((uint64_t)a.groups + 255) / 256;
  const uint64_t gx = blocks < 65536 ? blocks : 65536;
  const uint64_t gy = (blocks + gx - 1) / gx;
  hipLaunchKernelGGL((k_apply_reg<K, MODE, IDX, NT>), dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, psi,
                     U, a);
}

template <typename IDX, bool NT, int MODE>
void launch_reg_k(int K, void* psi, const float2* U, const RegArgs<IDX>& a, hipStream_t st) {
  switch (K) {
    case 0: if constexpr (MODE == 1) { launch_reg_t<IDX, NT, 0, MODE>(psi, U, a, st); return; } break;
    case 1: launch_reg_t<IDX, NT, 1, MODE>(psi, U, a, st); return;
    case 2: launch_reg_t<IDX, NT, 2, MODE>(psi, U, a, st); return;
    case 3: launch_reg_t<IDX, NT, 3, MODE>(psi, U, a, st); return;
    case 4: launch_reg_t<IDX, NT, 4, MODE>(psi, U, a, st); return;
    case 5: launch_reg_t<IDX, NT, 5, MODE>(psi, U, a, st); return;
    case 6: if constexpr (MODE == 2) { launch_reg_t<IDX, NT, 6, MODE>(psi, U, a, st); return; } break;
    default: break;
  }
  throw DeviceError{hipErrorInvalidValue, "k_apply_reg: unsupported K/mode"};
}

template <typename IDX, bool NT>
void launch_reg(const Pass& p, int n, void* psi, const float2* U, hipStream_t st) {
  RegArgs<IDX> a{};
  int mode, K;
  int pos[SV_MAX_K];
  if (p.s[0] == 0) {           // bit 0 is a target: it lives inside the float4
    mode = 1;
    K = p.k - 1;
    for (int j = 0; j < K; ++j) pos[j] = p.s[j + 1] - 1;
    a.groups = (IDX)1 << (n - 1 - K);
  } else if (p.k <= 5) {       // two groups per lane
    mode = 0;
    K = p.k;
    for (int j = 0; j < K; ++j) pos[j] = p.s[j] - 1;
    a.groups = (IDX)1 << (n - 1 - K);
  } else {                     // k = 6 with no target on bit 0: one group per lane
    mode = 2;
    K = p.k;
    for (int j = 0; j < K; ++j) pos[j] = p.s[j];
    a.groups = (IDX)1 << (n - K);
  }
  for (int j = 0; j < K; ++j) {
    a.lowmask[j] = ((IDX)1 << pos[j]) - 1;
    a.stride[j] = (IDX)1 << pos[j];
  }
  if (mode == 0) launch_reg_k<IDX, NT, 0>(K, psi, U, a, st);
  else if (mode == 1) launch_reg_k<IDX, NT, 1>(K, psi, U, a, st);
  else launch_reg_k<IDX, NT, 2>(K, psi, U, a, st);
}

}  // namespace

void launch_mfma(const Pass& p, int n, void* psi, const unsigned char* data, hipStream_t st);
void launch_lds(const Pass& p, int n, void* psi, const float2* U, hipStream_t st);

// Host checks of the launch geometry happen in the planner (targets sorted,
// distinct, < n; k <= n; LDS tile fits); this only dispatches.
void launch_pass(const Pass& p, int n, void* psi, const unsigned char* arena_dev, hipStream_t st) {
  const unsigned char* data = arena_dev + p.mat_off;
  if (p.variant == V_MFMA) {  // with or without controls
    launch_mfma(p, n, psi, data, st);
  } else if (p.cmask) {
    launch_ctrl(p, n, psi, reinterpret_cast<const float2*>(data), st);
  } else if (p.variant == V_SHFL) {
    launch_shfl(p, n, psi, reinterpret_cast<const float2*>(data), st);
  } else if (p.variant == V_PHASE) {
    launch_phase(n, psi, data, p.nhubs, p.hub, st);
  } else if (p.variant == V_LDS) {
    launch_lds(p, n, psi, reinterpret_cast<const float2*>(data), st);
  } else {
    const bool nt = gather_nt(n, p.k, p.s);
    const float2* U = reinterpret_cast<const float2*>(data);
    if (n <= 32) {
      if (nt) launch_reg<uint32_t, true>(p, n, psi, U, st);
      else launch_reg<uint32_t, false>(p, n, psi, U, st);
    } else {
      if (nt) launch_reg<uint64_t, true>(p, n, psi, U, st);
      else launch_reg<uint64_t, false>(p, n, psi, U, st);
    }
  }
  SV_HIP(hipGetLastError());
}

}  // namespace sv
