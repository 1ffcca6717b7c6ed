// Gate-application passes on VALU (gfx950): each pass applies one k-qubit
// matrix to all 2^(n-k) groups of the state in place (Sec. II-A, Eq. 4).
//
// Two kernels:
//   k_apply_reg  -- every lane owns whole groups in registers, gathered
//                   straight from HBM.  Lanes are consecutive in the lowest
//                   non-target bits, so each of the 2^K loads of a wavefront
//                   is one contiguous row when no target sits in bits 1..6.
//                   All amplitudes of a group are loaded before the first
//                   output is written (the load-buffer idea of Sec. IV-B), so
//                   each output row is stored as soon as it is computed.
//   k_apply_lds  -- a workgroup copies a tile of 2^T amplitudes (2^h chunks of
//                   2^m contiguous amplitudes, one chunk per combination of the
//                   h targets >= m) into LDS with coalesced 16-byte loads,
//                   applies the gate to the 2^(T-k) groups of the tile from
//                   LDS, and writes the tile back coalesced.  This is the
//                   path for targets in the low bits, where a register-direct
//                   gather would touch partial cache lines.
//
// Matrix entries are wave-uniform and read through the scalar unit; the
// matrix of a pass sits in the device arena, complex64 row-major, already
// permuted so that local bit j is the j-th lowest target.
#include "sv_internal.h"

namespace sv {

namespace {

__device__ __forceinline__ void cmac(float2& acc, const float2 u, const float2 v) {
  acc.x = fmaf(u.x, v.x, acc.x);
  acc.x = fmaf(-u.y, v.y, acc.x);
  acc.y = fmaf(u.x, v.y, acc.y);
  acc.y = fmaf(u.y, v.x, acc.y);
}

// Insert a zero bit below each mask boundary, ascending: turns a group index
// into the index of its first amplitude (all target bits zero).
template <int K, typename IDX>
__device__ __forceinline__ IDX insert_zeros(IDX g, const IDX* lowmask) {
#pragma unroll
  for (int j = 0; j < K; ++j) g = ((g & ~lowmask[j]) << 1) | (g & lowmask[j]);
  return g;
}

template <int K, typename IDX>
__device__ __forceinline__ IDX local_offset(int l, const IDX* stride) {
  IDX off = 0;
#pragma unroll
  for (int j = 0; j < K; ++j)
    if ((l >> j) & 1) off += stride[j];
  return off;
}

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
template <int K, int MODE, typename IDX>
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
    for (int l = 0; l < D; ++l) v[l] = psi[base + local_offset<K, IDX>(l, a.stride)];
#pragma unroll
    for (int r = 0; r < D; ++r) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int c = 0; c < D; ++c) cmac(acc, U[r * D + c], v[c]);
      psi[base + local_offset<K, IDX>(r, a.stride)] = acc;
    }
  } else if constexpr (MODE == 0) {
    float4* __restrict__ psi = reinterpret_cast<float4*>(psi_);
    float4 v[D];
#pragma unroll
    for (int l = 0; l < D; ++l) v[l] = psi[base + local_offset<K, IDX>(l, a.stride)];
#pragma unroll
    for (int r = 0; r < D; ++r) {
      float2 a0 = make_float2(0.f, 0.f), a1 = make_float2(0.f, 0.f);
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const float2 u = U[r * D + c];
        cmac(a0, u, make_float2(v[c].x, v[c].y));
        cmac(a1, u, make_float2(v[c].z, v[c].w));
      }
      psi[base + local_offset<K, IDX>(r, a.stride)] = make_float4(a0.x, a0.y, a1.x, a1.y);
    }
  } else {
    constexpr int DM = 2 * D;  // matrix dimension 2^(K+1)
    float4* __restrict__ psi = reinterpret_cast<float4*>(psi_);
    float4 v[D];
#pragma unroll
    for (int l = 0; l < D; ++l) v[l] = psi[base + local_offset<K, IDX>(l, a.stride)];
#pragma unroll
    for (int r = 0; r < D; ++r) {
      float2 a0 = make_float2(0.f, 0.f), a1 = make_float2(0.f, 0.f);
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const float2 lo = make_float2(v[c].x, v[c].y), hi = make_float2(v[c].z, v[c].w);
        cmac(a0, U[(2 * r) * DM + 2 * c], lo);
        cmac(a0, U[(2 * r) * DM + 2 * c + 1], hi);
        cmac(a1, U[(2 * r + 1) * DM + 2 * c], lo);
        cmac(a1, U[(2 * r + 1) * DM + 2 * c + 1], hi);
      }
      psi[base + local_offset<K, IDX>(r, a.stride)] = make_float4(a0.x, a0.y, a1.x, a1.y);
    }
  }
}

struct LdsArgs {
  uint64_t tiles;      // 2^(n-T)
  int T, m, h;         // tile bits, chunk bits, number of targets >= m
  int hi_pos[SV_MAX_K];  // ascending state bits of the h high targets
  int loc_mask[SV_MAX_K];  // insertion masks of the tile-local targets, ascending
  int loc_stride[SV_MAX_K];  // tile-local stride of local bit j
};

template <int K>
__global__ __launch_bounds__(256) void k_apply_lds(float2* __restrict__ psi,
                                                   const float2* __restrict__ U,
                                                   const LdsArgs a) {
  extern __shared__ float4 tile4[];
  float2* tile2 = reinterpret_cast<float2*>(tile4);
  float4* __restrict__ psi4 = reinterpret_cast<float4*>(psi);
  constexpr int D = 1 << K;
  const int pairs = 1 << (a.T - 1);
  const int mmask = (1 << a.m) - 1;
  const int groups = 1 << (a.T - K);
  for (uint64_t t = blockIdx.x; t < a.tiles; t += gridDim.x) {
    // first amplitude of the tile: tile index in the bits >= m that are not
    // high targets
    uint64_t tb = t << a.m;
    for (int i = 0; i < a.h; ++i) {
      const uint64_t lm = ((uint64_t)1 << a.hi_pos[i]) - 1;
      tb = ((tb & ~lm) << 1) | (tb & lm);
    }
    for (int x2 = threadIdx.x; x2 < pairs; x2 += 256) {
      const int x = x2 << 1;
      const int c = x >> a.m;
      uint64_t gi = tb + (uint64_t)(x & mmask);
      for (int i = 0; i < a.h; ++i)
        if ((c >> i) & 1) gi += (uint64_t)1 << a.hi_pos[i];
      tile4[x2] = psi4[gi >> 1];
    }
    __syncthreads();
    for (int gl = threadIdx.x; gl < groups; gl += 256) {
      const int b = insert_zeros<K, int>(gl, a.loc_mask);
      float2 v[D];
#pragma unroll
      for (int l = 0; l < D; ++l) v[l] = tile2[b + local_offset<K, int>(l, a.loc_stride)];
#pragma unroll
      for (int r = 0; r < D; ++r) {
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int c = 0; c < D; ++c) cmac(acc, U[r * D + c], v[c]);
        tile2[b + local_offset<K, int>(r, a.loc_stride)] = acc;
      }
    }
    __syncthreads();
    for (int x2 = threadIdx.x; x2 < pairs; x2 += 256) {
      const int x = x2 << 1;
      const int c = x >> a.m;
      uint64_t gi = tb + (uint64_t)(x & mmask);
      for (int i = 0; i < a.h; ++i)
        if ((c >> i) & 1) gi += (uint64_t)1 << a.hi_pos[i];
      psi4[gi >> 1] = tile4[x2];
    }
    __syncthreads();
  }
}

template <typename IDX, int K, int MODE>
void launch_reg_t(void* psi, const float2* U, const RegArgs<IDX>& a, hipStream_t st) {
  // 2-D grid keeps blocks * 256 below 2^32 work-items per dimension
  const uint64_t blocks = ((uint64_t)a.groups + 255) / 256;
  const uint64_t gx = blocks < 65536 ? blocks : 65536;
  const uint64_t gy = (blocks + gx - 1) / gx;
  hipLaunchKernelGGL((k_apply_reg<K, MODE, IDX>), dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, psi,
                     U, a);
}

template <typename IDX, int MODE>
void launch_reg_k(int K, void* psi, const float2* U, const RegArgs<IDX>& a, hipStream_t st) {
  switch (K) {
    case 0: if constexpr (MODE == 1) { launch_reg_t<IDX, 0, MODE>(psi, U, a, st); return; } break;
    case 1: launch_reg_t<IDX, 1, MODE>(psi, U, a, st); return;
    case 2: launch_reg_t<IDX, 2, MODE>(psi, U, a, st); return;
    case 3: launch_reg_t<IDX, 3, MODE>(psi, U, a, st); return;
    case 4: launch_reg_t<IDX, 4, MODE>(psi, U, a, st); return;
    case 5: launch_reg_t<IDX, 5, MODE>(psi, U, a, st); return;
    case 6: if constexpr (MODE == 2) { launch_reg_t<IDX, 6, MODE>(psi, U, a, st); return; } break;
    default: break;
  }
  throw DeviceError{hipErrorInvalidValue, "k_apply_reg: unsupported K/mode"};
}

template <typename IDX>
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
  if (mode == 0) launch_reg_k<IDX, 0>(K, psi, U, a, st);
  else if (mode == 1) launch_reg_k<IDX, 1>(K, psi, U, a, st);
  else launch_reg_k<IDX, 2>(K, psi, U, a, st);
}

void launch_lds(const Pass& p, int n, void* psi, const float2* U, hipStream_t st) {
  LdsArgs a{};
  const int T = p.tile_bits < n ? p.tile_bits : n;
  int m = 0;
  const int h = lds_split(T, p.k, p.s, &m);
  a.T = T;
  a.m = m;
  a.h = h;
  a.tiles = (uint64_t)1 << (n - T);
  // targets below m keep their bit; high target i moves to tile bit m + i
  int loc[SV_MAX_K];
  int hi = 0;
  for (int j = 0; j < p.k; ++j) {
    if (p.s[j] < m) {
      loc[j] = p.s[j];
    } else {
      a.hi_pos[hi] = p.s[j];
      loc[j] = m + hi;
      ++hi;
    }
  }
  for (int j = 0; j < p.k; ++j) {
    a.loc_mask[j] = (1 << loc[j]) - 1;
    a.loc_stride[j] = 1 << loc[j];
  }
  const uint64_t max_blocks = 256 * 16;
  const unsigned blocks = (unsigned)(a.tiles < max_blocks ? a.tiles : max_blocks);
  const size_t lds = (size_t)8 << T;
  switch (p.k) {
    case 1: hipLaunchKernelGGL(k_apply_lds<1>, dim3(blocks), dim3(256), lds, st, (float2*)psi, U, a); break;
    case 2: hipLaunchKernelGGL(k_apply_lds<2>, dim3(blocks), dim3(256), lds, st, (float2*)psi, U, a); break;
    case 3: hipLaunchKernelGGL(k_apply_lds<3>, dim3(blocks), dim3(256), lds, st, (float2*)psi, U, a); break;
    case 4: hipLaunchKernelGGL(k_apply_lds<4>, dim3(blocks), dim3(256), lds, st, (float2*)psi, U, a); break;
    case 5: hipLaunchKernelGGL(k_apply_lds<5>, dim3(blocks), dim3(256), lds, st, (float2*)psi, U, a); break;
    case 6: hipLaunchKernelGGL(k_apply_lds<6>, dim3(blocks), dim3(256), lds, st, (float2*)psi, U, a); break;
    default: throw DeviceError{hipErrorInvalidValue, "k_apply_lds: bad k"};
  }
}

}  // namespace

void launch_mfma(const Pass& p, int n, void* psi, const unsigned char* data, hipStream_t st);

// Host checks of the launch geometry happen in the planner (targets sorted,
// distinct, < n; k <= n; LDS tile fits); this only dispatches.
void launch_pass(const Pass& p, int n, void* psi, const unsigned char* arena_dev, hipStream_t st) {
  const unsigned char* data = arena_dev + p.mat_off;
  if (p.variant == V_MFMA) {
    launch_mfma(p, n, psi, data, st);
  } else if (p.variant == V_LDS) {
    launch_lds(p, n, psi, reinterpret_cast<const float2*>(data), st);
  } else if (n <= 32) {
    launch_reg<uint32_t>(p, n, psi, reinterpret_cast<const float2*>(data), st);
  } else {
    launch_reg<uint64_t>(p, n, psi, reinterpret_cast<const float2*>(data), st);
  }
  SV_HIP(hipGetLastError());
}

}  // namespace sv
