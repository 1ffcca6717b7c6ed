// LDS-staged gate passes for low target qubits (see k_common.h).
#include "k_common.h"

namespace sv {

namespace {
using namespace kern;

struct LdsArgs {
  uint64_t tiles;            // 2^(n-T)
  int m, h;                  // chunk bits, number of targets >= m
  int hi_pos[SV_MAX_K];      // ascending state bits of the h high targets
  int pmask[SV_MAX_K];       // insertion masks of the K compute-space targets, ascending
  int pstride[SV_MAX_K];     // compute-space stride of local bit j
  int nt;                    // stream the state non-temporally
};

// Tile slots are float4 (two amplitudes).  XOR-swizzling slot bits 0..3
// with bits 4..7 and 8..11 spreads the strided group reads of the compute
// phase over all LDS banks while keeping every aligned run of 16 slots (one
// 256-byte row, what the coalesced load/store phases touch) a permutation
// of itself.
__device__ __forceinline__ int swz(int x2) { return x2 ^ (((x2 >> 4) ^ (x2 >> 8)) & 15); }

// Global float4 index of tile slot x2.
__device__ __forceinline__ uint64_t tile_global(const LdsArgs& a, uint64_t tb, int x2) {
  const int x = x2 << 1;
  const int c = x >> a.m;
  uint64_t gi = tb + (uint64_t)(x & ((1 << a.m) - 1));
  for (int i = 0; i < a.h; ++i)
    if ((c >> i) & 1) gi += (uint64_t)1 << a.hi_pos[i];
  return gi >> 1;
}

// T: log2 amplitudes per tile.  MODE as in k_apply_reg, over the tile:
// 0 = two groups per lane (bit 0 not a target), 1 = bit 0 is target 0,
// 2 = one group per lane with float2 accesses (k = 6, bit 0 not a target).
template <int T, int K, int MODE, bool NT>
__global__ __launch_bounds__(256) void k_apply_lds(float4* __restrict__ psi4,
                                                   const float2* __restrict__ U,
                                                   const LdsArgs a) {
  extern __shared__ float4 tile[];
  constexpr int SLOTS = 1 << (T - 1);
  constexpr int PER = (SLOTS + 255) / 256;
  constexpr int D = 1 << K;
  constexpr int ITEMS = MODE == 2 ? (1 << (T - K)) : (1 << (T - 1 - K));
  const int tid = threadIdx.x;
  for (uint64_t t = blockIdx.x; t < a.tiles; t += gridDim.x) {
    uint64_t tb = t << a.m;  // tile index spread over the non-target bits >= m
    for (int i = 0; i < a.h; ++i) {
      const uint64_t lm = ((uint64_t)1 << a.hi_pos[i]) - 1;
      tb = ((tb & ~lm) << 1) | (tb & lm);
    }
    float4 r[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int x2 = tid + 256 * i;
      if (SLOTS % 256 == 0 || x2 < SLOTS) r[i] = gld<NT>(psi4 + tile_global(a, tb, x2));
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int x2 = tid + 256 * i;
      if (SLOTS % 256 == 0 || x2 < SLOTS) tile[swz(x2)] = r[i];
    }
    __syncthreads();
    for (int it = tid; it < ITEMS; it += 256) {
      const int b = insert_zeros<K, int>(it, a.pmask);
      if constexpr (MODE == 2) {
        float2* tile2 = reinterpret_cast<float2*>(tile);
        float2 v[D];
#pragma unroll
        for (int l = 0; l < D; ++l) {
          const int x = b + local_offset<K, int>(l, a.pstride);
          v[l] = tile2[2 * swz(x >> 1) + (x & 1)];
        }
#pragma unroll
        for (int rr = 0; rr < D; ++rr) {
          float2 acc = make_float2(0.f, 0.f);
#pragma unroll
          for (int c = 0; c < D; ++c) cmac(acc, U[rr * D + c], v[c]);
          const int x = b + local_offset<K, int>(rr, a.pstride);
          tile2[2 * swz(x >> 1) + (x & 1)] = acc;
        }
      } else {
        float4 v[D];
#pragma unroll
        for (int l = 0; l < D; ++l) v[l] = tile[swz(b + local_offset<K, int>(l, a.pstride))];
#pragma unroll
        for (int rr = 0; rr < D; ++rr)
          tile[swz(b + local_offset<K, int>(rr, a.pstride))] = pair_row<K, MODE>(v, U, rr);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int x2 = tid + 256 * i;
      if (SLOTS % 256 == 0 || x2 < SLOTS) r[i] = tile[swz(x2)];
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int x2 = tid + 256 * i;
      if (SLOTS % 256 == 0 || x2 < SLOTS) gst<NT>(psi4 + tile_global(a, tb, x2), r[i]);
    }
    __syncthreads();
  }
}

template <int T, int K, int MODE, bool NT>
void launch_lds_nt(const LdsArgs& a, void* psi, const float2* U, hipStream_t st) {
  const uint64_t max_blocks = 256 * 8;
  const unsigned blocks = (unsigned)(a.tiles < max_blocks ? a.tiles : max_blocks);
  constexpr size_t lds = (size_t)8 << T;
  hipLaunchKernelGGL((k_apply_lds<T, K, MODE, NT>), dim3(blocks), dim3(256), lds, st, (float4*)psi, U, a);
}

template <int T, int K, int MODE>
void launch_lds_t(const LdsArgs& a, void* psi, const float2* U, hipStream_t st) {
  if (a.nt) return launch_lds_nt<T, K, MODE, true>(a, psi, U, st);
  launch_lds_nt<T, K, MODE, false>(a, psi, U, st);
}

template <int T>
void launch_lds_mode(int K, int mode, const LdsArgs& a, void* psi, const float2* U, hipStream_t st) {
  if (mode == 2) {
    if (K == 6) return launch_lds_t<T, 6, 2>(a, psi, U, st);
  } else if (mode == 0) {
    switch (K) {
      case 1: return launch_lds_t<T, 1, 0>(a, psi, U, st);
      case 2: return launch_lds_t<T, 2, 0>(a, psi, U, st);
      case 3: return launch_lds_t<T, 3, 0>(a, psi, U, st);
      case 4: return launch_lds_t<T, 4, 0>(a, psi, U, st);
      case 5: return launch_lds_t<T, 5, 0>(a, psi, U, st);
      default: break;
    }
  } else {
    switch (K) {
      case 0: return launch_lds_t<T, 0, 1>(a, psi, U, st);
      case 1: return launch_lds_t<T, 1, 1>(a, psi, U, st);
      case 2: return launch_lds_t<T, 2, 1>(a, psi, U, st);
      case 3: return launch_lds_t<T, 3, 1>(a, psi, U, st);
      case 4: return launch_lds_t<T, 4, 1>(a, psi, U, st);
      case 5: return launch_lds_t<T, 5, 1>(a, psi, U, st);
      default: break;
    }
  }
  throw DeviceError{hipErrorInvalidValue, "k_apply_lds: unsupported K/mode"};
}

// Tile sizes built: 2^8, 2^10 and 2^12 amplitudes (2, 8 and 32 KiB of LDS).
}  // namespace

int lds_tile_bits_for(int n, int want) {
  int T = want >= 12 ? 12 : (want >= 10 ? 10 : 8);
  while (T > n) T -= 2;
  return T;
}

void launch_lds(const Pass& p, int n, void* psi, const float2* U, hipStream_t st) {
  LdsArgs a{};
  const int T = lds_tile_bits_for(n, p.tile_bits);
  int m = 0;
  const int h = lds_split(T, p.k, p.s, &m);
  a.m = m;
  a.h = h;
  a.tiles = (uint64_t)1 << (n - T);
  a.nt = n >= kNtMinQubits;
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
  int mode, K;
  int pos[SV_MAX_K];
  if (loc[0] == 0) {
    mode = 1;
    K = p.k - 1;
    for (int j = 0; j < K; ++j) pos[j] = loc[j + 1] - 1;
  } else if (p.k <= 5) {
    mode = 0;
    K = p.k;
    for (int j = 0; j < K; ++j) pos[j] = loc[j] - 1;
  } else {
    mode = 2;
    K = p.k;
    for (int j = 0; j < K; ++j) pos[j] = loc[j];
  }
  for (int j = 0; j < K; ++j) {
    a.pmask[j] = (1 << pos[j]) - 1;
    a.pstride[j] = 1 << pos[j];
  }
  switch (T) {
    case 12: launch_lds_mode<12>(K, mode, a, psi, U, st); break;
    case 10: launch_lds_mode<10>(K, mode, a, psi, U, st); break;
    default: launch_lds_mode<8>(K, mode, a, psi, U, st); break;
  }
}

}  // namespace sv
