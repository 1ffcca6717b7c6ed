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
    if constexpr (K <= 4) {
      // the 3M row products: up to K = 4 the extra input sums and third
      // accumulator still leave room for several waves per SIMD; at K = 5
      // they would leave one (measured slower than the 4M form)
      const float* __restrict__ U3 = u3_of<K, MODE>(U);
      float2 sv[D];
      input_sums<D>(v, sv);
#pragma unroll
      for (int r = 0; r < D; ++r)
        gst<NT>(psi + base + local_offset<K, IDX>(r, a.stride), pair_row3<K, MODE>(v, sv, U3, r));
    } else {
#pragma unroll
      for (int r = 0; r < D; ++r)
        gst<NT>(psi + base + local_offset<K, IDX>(r, a.stride), pair_row<K, MODE>(v, U, r));
    }
  }
}

// MODE 0 / 1 with targets on element bits 0..2 (set TM; amplitude bits 1..3)
// on a streamed state: the lane exchange of k_common.h.  Lane j of a wave owns
// the work item u(j) | c(j) << (6 - m) of the wave's 64 (c(j): j's bits in TM,
// u(j): its other bits); load slot X reads, in lane j, the element of item
// u(j) | X << (6 - m) whose low-target local bits are c(j), so that 8 aligned
// lanes read one whole line; a butterfly over the m targets (m = 1) or a
// transpose through LDS (m = 2, 3) then hands every lane all elements of its
// own item.  Outputs go back the same way, 2^m rows at a time.  The number of
// work items is a multiple of 64.
template <int K, int MODE, int TM>
__global__ __launch_bounds__(256) void k_apply_reg_x(float4* __restrict__ psi, const float2* __restrict__ U,
                                                     const RegArgs<uint64_t> a) {
  constexpr int D = 1 << K;
  constexpr int M = LowBits<TM>::m;
  constexpr int XM = (1 << M) - 1;
  static_assert(M <= K, "every low target is an element-space target");
  const uint64_t wave0 = ((uint64_t)blockIdx.y * gridDim.x + blockIdx.x) * 256 + (threadIdx.x & ~63u);
  if (wave0 >= a.groups) return;  // whole waves: groups is a multiple of 64
  const int j = threadIdx.x & 63;
  const int uj = compress_bits<6>(j, ~TM & 63), cj = compress_bits<6>(j, TM);
  uint64_t offc = 0;
#pragma unroll
  for (int i = 0; i < M; ++i)
    if ((cj >> i) & 1) offc += a.stride[i];
  uint64_t xoff[XM + 1];
#pragma unroll
  for (int X = 0; X <= XM; ++X) xoff[X] = insert_zeros<K, uint64_t>((uint64_t)X << (6 - M), a.lowmask);
  const uint64_t b0 = insert_zeros<K, uint64_t>(wave0 + uj, a.lowmask) + offc;
  float4 v[D];
#pragma unroll
  for (int r = 0; r < D; ++r) v[r] = gld<true>(psi + b0 + xoff[r & XM] + local_offset<K, uint64_t>(r & ~XM, a.stride));
  __shared__ float4 xs[M >= 2 ? 4 * D * 64 : 1];  // the LDS hand-over of m = 2, 3
  float4* t = xs + (M >= 2 ? (threadIdx.x >> 6) * D * 64 : 0);
  if constexpr (M >= 2) xtranspose_lds<TM>(v, t, j, cj);
  else xtranspose<TM>(v, j);
#pragma unroll
  for (int hi = 0; hi < D; hi += XM + 1) {
    float4 o[XM + 1];
#pragma unroll
    for (int x = 0; x <= XM; ++x) o[x] = pair_row<K, MODE>(v, U, hi | x);
    if constexpr (M >= 2) xtranspose_lds_back<TM>(o, t, hi, j, cj);
    else xtranspose<TM>(o, j);
#pragma unroll
    for (int x = 0; x <= XM; ++x) gst<true>(psi + b0 + xoff[x] + local_offset<K, uint64_t>(hi, a.stride), o[x]);
  }
}

template <int K, int MODE, int TM>
void launch_reg_x_t(void* psi, const float2* U, const RegArgs<uint64_t>& a, hipStream_t st) {
  const uint64_t blocks = ((uint64_t)a.groups + 255) / 256;
  const uint64_t gx = blocks < 65536 ? blocks : 65536;
  const uint64_t gy = (blocks + gx - 1) / gx;
  hipLaunchKernelGGL((k_apply_reg_x<K, MODE, TM>), dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, (float4*)psi,
                     U, a);
}

template <int MODE, int TM>
void launch_reg_x_k(int K, void* psi, const float2* U, const RegArgs<uint64_t>& a, hipStream_t st) {
  constexpr int M = LowBits<TM>::m;
  switch (K) {
    case 1: if constexpr (M <= 1) return launch_reg_x_t<1, MODE, TM>(psi, U, a, st); break;
    case 2: if constexpr (M <= 2) return launch_reg_x_t<2, MODE, TM>(psi, U, a, st); break;
    case 3: return launch_reg_x_t<3, MODE, TM>(psi, U, a, st);
    default: break;
  }
  throw DeviceError{hipErrorInvalidValue, "k_apply_reg_x: unsupported K / low targets"};
}

template <int MODE>
void launch_reg_x(int tm, int K, void* psi, const float2* U, const RegArgs<uint64_t>& a, hipStream_t st) {
  switch (tm) {
    case 1: return launch_reg_x_k<MODE, 1>(K, psi, U, a, st);
    case 2: return launch_reg_x_k<MODE, 2>(K, psi, U, a, st);
    case 3: return launch_reg_x_k<MODE, 3>(K, psi, U, a, st);
    case 4: return launch_reg_x_k<MODE, 4>(K, psi, U, a, st);
    case 5: return launch_reg_x_k<MODE, 5>(K, psi, U, a, st);
    case 6: return launch_reg_x_k<MODE, 6>(K, psi, U, a, st);
    case 7: return launch_reg_x_k<MODE, 7>(K, psi, U, a, st);
    default: throw DeviceError{hipErrorInvalidValue, "k_apply_reg_x: low-target mask"};
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

// Low-target mask of the register exchange form (0: the plain kernel): a
// streamed state, a pass with two groups or half a group per 16-byte element
// (MODE 0 / 1) and at most 3 element-space targets, some of them on element
// bits 0..2.
int reg_exchange_mask(int n, int k, const int* s) {
  if (n < kern::kNtMinQubits) return 0;
  const bool q0 = s[0] == 0;
  const int K = q0 ? k - 1 : k;
  if (K < 1 || K > 3 || (!q0 && k > 5)) return 0;
  int tm = 0;
  for (int j = q0 ? 1 : 0; j < k; ++j)
    if (s[j] >= 1 && s[j] <= 3) tm |= 1 << (s[j] - 1);
  return tm;
}

}  // namespace

bool reg_streams(int n, int k, const int* s) { return reg_exchange_mask(n, k, s) != 0 || kern::gather_nt(n, k, s); }

namespace {

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

void launch_reg_exchange(const Pass& p, int n, int tm, void* psi, const float2* U, hipStream_t st) {
  RegArgs<uint64_t> a{};
  const bool q0 = p.s[0] == 0;
  const int K = q0 ? p.k - 1 : p.k;
  for (int j = 0; j < K; ++j) {
    const int pos = p.s[q0 ? j + 1 : j] - 1;
    a.lowmask[j] = ((uint64_t)1 << pos) - 1;
    a.stride[j] = (uint64_t)1 << pos;
  }
  a.groups = (uint64_t)1 << (n - 1 - K);
  if (a.groups % 64) throw DeviceError{hipErrorInvalidValue, "k_apply_reg_x: work items not a multiple of 64"};
  if (q0) launch_reg_x<1>(tm, K, psi, U, a, st);
  else launch_reg_x<0>(tm, K, psi, U, a, st);
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
    launch_phase(n, psi, data, st);
  } else if (p.variant == V_LDS) {
    launch_lds(p, n, psi, reinterpret_cast<const float2*>(data), st);
  } else if (const int tm = reg_exchange_mask(n, p.k, p.s)) {
    launch_reg_exchange(p, n, tm, psi, reinterpret_cast<const float2*>(data), st);
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
