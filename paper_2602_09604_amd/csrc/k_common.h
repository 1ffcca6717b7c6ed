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
#pragma once
#include "sv_internal.h"

namespace sv {
namespace kern {

// Global state accesses.  A pass streams the state once; for states beyond
// the last-level cache the non-temporal form (NT = true) keeps the stream
// from evicting useful lines and measured faster for in-place sweeps; small
// states that stay cache-resident across passes use ordinary accesses.
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));

template <bool NT>
__device__ __forceinline__ float4 gld(const float4* p) {
  if constexpr (NT) {
    const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
  } else {
    return *p;
  }
}
template <bool NT>
__device__ __forceinline__ float2 gld(const float2* p) {
  if constexpr (NT) {
    const nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(p));
    return make_float2(v.x, v.y);
  } else {
    return *p;
  }
}
template <bool NT>
__device__ __forceinline__ void gst(float4* p, const float4 v) {
  if constexpr (NT) {
    const nt_f4 w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<nt_f4*>(p));
  } else {
    *p = v;
  }
}
template <bool NT>
__device__ __forceinline__ void gst(float2* p, const float2 v) {
  if constexpr (NT) {
    const nt_f2 w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<nt_f2*>(p));
  } else {
    *p = v;
  }
}

// States of at least 2^26 amplitudes (512 MiB) exceed the 256 MB last-level
// cache: stream them non-temporally.
constexpr int kNtMinQubits = 26;

// Register-gather passes stream non-temporally only when every wavefront
// access covers whole 128-byte lines, i.e. no target in bits 1..3 (bit 0
// lives inside the 16-byte element).  Otherwise the partial lines of one
// access are completed by the lane's other accesses through the L2, which
// non-temporal accesses would bypass (measured 2-10x slower).
inline bool gather_nt(int n, int k, const int* s) {
  if (n < kNtMinQubits) return false;
  for (int j = 0; j < k; ++j)
    if (s[j] >= 1 && s[j] < 4) return false;
  return true;
}

// ---- lane exchange for targets on amplitude bits 1..3 ----------------------
// A target on element bit t in {0, 1, 2} (16-byte elements; amplitude bit
// t + 1) splits every 128-byte line between the loads of different local
// indices.  The exchange forms let 8 aligned lanes read one whole line per
// load (each lane the element of another group whose low-target bits are the
// lane's own bits there) and then transpose the loaded elements across those
// lanes with a butterfly of lane swaps, so that every lane holds its own
// group; stores undo it.  TM is the set of such target bits (element bits),
// m = popcount(TM); register r of a unit has the low-target local bits in
// its bits 0..m-1.
template <int TM>
struct LowBits {
  static constexpr int m = (TM & 1) + ((TM >> 1) & 1) + ((TM >> 2) & 1);
  static constexpr int t(int i) {
    int c = 0;
    for (int b = 0; b < 3; ++b)
      if ((TM >> b) & 1) {
        if (c == i) return b;
        ++c;
      }
    return 0;
  }
};

// value of the lane j ^ 2^T (T in 0..2; within aligned groups of 8 lanes)
template <int T>
__device__ __forceinline__ float lane_xor(float v) {
  const int x = __float_as_int(v);
  if constexpr (T == 0) return __int_as_float(__builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, true));  // quad_perm 1,0,3,2
  else if constexpr (T == 1) return __int_as_float(__builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, true));  // 2,3,0,1
  else return __int_as_float(__builtin_amdgcn_ds_swizzle(x, (4 << 10) | 0x1F));  // bit mode: xor 4
}

template <int TM, int I, int N>
__device__ __forceinline__ void xstage(float4 (&R)[N], int j) {
  constexpr int T = LowBits<TM>::t(I);
  const bool hi = (j >> T) & 1;
#pragma unroll
  for (int r = 0; r < N; ++r) {
    if (r & (1 << I)) continue;
    const int r1 = r | (1 << I);
    // component-wise selects on values (a select between the two array
    // elements themselves would take their addresses)
    const float4 a0 = R[r], a1 = R[r1];
    const float4 snd = make_float4(hi ? a0.x : a1.x, hi ? a0.y : a1.y, hi ? a0.z : a1.z, hi ? a0.w : a1.w);
    const float4 rcv = make_float4(lane_xor<T>(snd.x), lane_xor<T>(snd.y), lane_xor<T>(snd.z), lane_xor<T>(snd.w));
    R[r] = make_float4(hi ? rcv.x : a0.x, hi ? rcv.y : a0.y, hi ? rcv.z : a0.z, hi ? rcv.w : a0.w);
    R[r1] = make_float4(hi ? a1.x : rcv.x, hi ? a1.y : rcv.y, hi ? a1.z : rcv.z, hi ? a1.w : rcv.w);
  }
}

// register r of a unit: bits 0..m-1 the low-target local bits (before the
// butterfly: the slot X), the rest the unit's other local bits
template <int TM, int N>
__device__ __forceinline__ void xtranspose(float4 (&R)[N], int j) {
  constexpr int M = LowBits<TM>::m;
  if constexpr (M >= 1) xstage<TM, 0, N>(R, j);
  if constexpr (M >= 2) xstage<TM, 1, N>(R, j);
  if constexpr (M >= 3) xstage<TM, 2, N>(R, j);
}

// the low bits of x placed at the positions of the set bits of TM, ascending
template <int TM>
__host__ __device__ constexpr int spread_bits(int x) {
  int o = 0, c = 0;
  for (int b = 0; b < 3; ++b)
    if ((TM >> b) & 1) o |= ((x >> c++) & 1) << b;
  return o;
}

// orders the LDS accesses of one wavefront around it (lanes of a wave
// exchange data through LDS without a workgroup barrier)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The same hand-over through LDS, for m = 2 or 3, where the butterfly's
// stages cost more lane swaps and selects than a trip through LDS.  t holds
// N * 64 float4 per wavefront.  Register r goes to row r, column
// j ^ spread(r & XM); lane j then reads row (r & ~XM) | c(j) at the same
// column.  The XOR keeps the writes and the reads free of bank conflicts.
template <int TM, int N>
__device__ __forceinline__ void xtranspose_lds(float4 (&R)[N], float4* t, int j, int cj) {
  constexpr int XM = (1 << LowBits<TM>::m) - 1;
#pragma unroll
  for (int r = 0; r < N; ++r) t[r * 64 + (j ^ spread_bits<TM>(r & XM))] = R[r];
  wave_sync();
#pragma unroll
  for (int r = 0; r < N; ++r) R[r] = t[((r & ~XM) | cj) * 64 + (j ^ spread_bits<TM>(r & XM))];
}

// Its inverse for the 2^m outputs O[x] = row hb | x of this lane's own item
// (hb a multiple of 2^m): afterwards O[X] is slot X's element, as loaded.
template <int TM, int N>
__device__ __forceinline__ void xtranspose_lds_back(float4 (&O)[N], float4* t, int hb, int j, int cj) {
  wave_sync();  // every lane has read what these writes replace
#pragma unroll
  for (int x = 0; x < N; ++x) t[(hb | cj) * 64 + (j ^ spread_bits<TM>(x))] = O[x];
  wave_sync();
#pragma unroll
  for (int x = 0; x < N; ++x) O[x] = t[(hb | x) * 64 + (j ^ spread_bits<TM>(x))];
}

// bits of v at the positions of mask (BITS-bit values), packed ascending
template <int BITS>
__device__ __forceinline__ int compress_bits(int v, int mask) {
  int o = 0, c = 0;
#pragma unroll
  for (int b = 0; b < BITS; ++b)
    if ((mask >> b) & 1) o |= ((v >> b) & 1) << c++;
  return o;
}

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

// Output row r of the pair layout.  MODE 0: v[c] holds local index c of two
// groups (bit 0 = 0 in .xy, bit 0 = 1 in .zw); MODE 1: v[c] holds local
// indices 2c (.xy) and 2c+1 (.zw) of one group, and the result holds rows
// 2r and 2r+1.
template <int K, int MODE>
__device__ __forceinline__ float4 pair_row(const float4* v, const float2* __restrict__ U, const int r) {
  constexpr int D = 1 << K;
  float2 a0 = make_float2(0.f, 0.f), a1 = make_float2(0.f, 0.f);
  if constexpr (MODE == 0) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const float2 u = U[r * D + c];
      cmac(a0, u, make_float2(v[c].x, v[c].y));
      cmac(a1, u, make_float2(v[c].z, v[c].w));
    }
  } else {
    constexpr int DM = 2 * D;  // matrix dimension 2^(K+1)
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const float2 lo = make_float2(v[c].x, v[c].y), hi = make_float2(v[c].z, v[c].w);
      cmac(a0, U[(2 * r) * DM + 2 * c], lo);
      cmac(a0, U[(2 * r) * DM + 2 * c + 1], hi);
      cmac(a1, U[(2 * r + 1) * DM + 2 * c], lo);
      cmac(a1, U[(2 * r + 1) * DM + 2 * c + 1], hi);
    }
  }
  return make_float4(a0.x, a0.y, a1.x, a1.y);
}

// The 3M form of the same row products (three real products per complex
// multiply-accumulate instead of four), for the register kernel, whose
// larger passes are bound by the vector ALUs.  With s = vr + vi per input
// and the matrix stored as u3 = (ur, ur + ui, ui - ur) per element:
// T += ur s, R += vi (ur + ui), I += vr (ui - ur); then Re = T - R and
// Im = T + I (T - R = sum ur vr - ui vi, T + I = sum ur vi + ui vr).
struct Acc3 {
  float t = 0.f, r = 0.f, i = 0.f;
};

__device__ __forceinline__ void cmac3(Acc3& a, const float* __restrict__ u3, const float vr, const float vi,
                                      const float s) {
  a.t = fmaf(u3[0], s, a.t);
  a.r = fmaf(vi, u3[1], a.r);
  a.i = fmaf(vr, u3[2], a.i);
}

__device__ __forceinline__ float2 fin3(const Acc3& a) { return make_float2(a.t - a.r, a.t + a.i); }

// where the 3M copy starts in a register pass's data: after the d x d
// complex64 matrix, d = 2^K (MODE 0, 2) or 2^(K+1) (MODE 1)
template <int K, int MODE>
__device__ __forceinline__ const float* u3_of(const float2* U) {
  constexpr int d = MODE == 1 ? 2 << K : 1 << K;
  return reinterpret_cast<const float*>(U + d * d);
}

// s = vr + vi of both amplitudes of every input element
template <int D>
__device__ __forceinline__ void input_sums(const float4* v, float2* s) {
#pragma unroll
  for (int c = 0; c < D; ++c) s[c] = make_float2(v[c].x + v[c].y, v[c].z + v[c].w);
}

// pair_row in the 3M form; s from input_sums
template <int K, int MODE>
__device__ __forceinline__ float4 pair_row3(const float4* v, const float2* s, const float* __restrict__ U3,
                                            const int r) {
  constexpr int D = 1 << K;
  Acc3 a0, a1;
  if constexpr (MODE == 0) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const float* u = U3 + 3 * (r * D + c);
      cmac3(a0, u, v[c].x, v[c].y, s[c].x);
      cmac3(a1, u, v[c].z, v[c].w, s[c].y);
    }
  } else {
    constexpr int DM = 2 * D;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      cmac3(a0, U3 + 3 * ((2 * r) * DM + 2 * c), v[c].x, v[c].y, s[c].x);
      cmac3(a0, U3 + 3 * ((2 * r) * DM + 2 * c + 1), v[c].z, v[c].w, s[c].y);
      cmac3(a1, U3 + 3 * ((2 * r + 1) * DM + 2 * c), v[c].x, v[c].y, s[c].x);
      cmac3(a1, U3 + 3 * ((2 * r + 1) * DM + 2 * c + 1), v[c].z, v[c].w, s[c].y);
    }
  }
  const float2 o0 = fin3(a0), o1 = fin3(a1);
  return make_float4(o0.x, o0.y, o1.x, o1.y);
}

}  // namespace kern
}  // namespace sv
