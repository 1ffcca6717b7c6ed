// Phase-only pass: psi[i] *= exp(2 pi i theta(i)) with theta (in turns) a
// quadratic polynomial of the bits of i: c + sum_q alpha_q x_q +
// sum_{a<b} beta_ab x_a x_b (phase.cpp builds it from a run of diagonal
// gates).  An elementwise, perfectly coalesced sweep: one read and one write
// per amplitude, any number of interacting pairs in one pass.
//
// The grid covers a low span of 2^lb amplitudes (lb = min(n, 28)) and walks
// it 2^(n - lb) times, once per value k of the high bits, so a thread's low
// index bits never change.  (Measured at 34 qubits: spans of 2^21, 2^22,
// 2^24, 2^26, 2^28, 2^30 amplitudes ran at 0.64, 0.67, 0.72, 0.74, 0.76,
// 0.77 of HBM peak; the whole state as one span, 0.28 at 32 qubits, pays
// the per-thread setup for every four amplitudes.)  Split x = xL + (k << lb):
//   theta(x) = theta(xL) + theta_high(k) + sum_j k_j gamma_j(xL),
//   gamma_j(xL) = sum_{a in L} beta_{a, lb+j} x_a.
// A thread owns the amplitudes base + {0, 1, 512, 513} (bits 0 and 9 free in
// base), so it evaluates theta(base), the two bit-0 / bit-9 increments and
// gamma_j(base) once, in FP64, from the coefficients in LDS; bits 10.. of
// base are the block's, and their sums are formed once per block.  Each sweep
// then costs a few adds per amplitude plus the sine and cosine: the bit-0 and
// bit-9 parts of sum_j k_j gamma_j come from the per-k table.
#include "k_common.h"

namespace sv {

namespace {
using kern::gld;
using kern::gst;

struct PhaseArgs {
  uint64_t pairs;  // float4 elements of the state
  int n;
  int lb;          // low span: 2^lb amplitudes per sweep of the grid
  int nh;          // high bits n - lb
};

__device__ __forceinline__ float2 rotate(const float2 v, float turns) {
  float s, c;
  sincospif(2.f * turns, &s, &c);
  return make_float2(v.x * c - v.y * s, v.x * s + v.y * c);
}

__device__ __forceinline__ float fold(double t) { return (float)(t - rint(t)); }

template <bool NT>
__global__ __launch_bounds__(256) void k_phase(float4* __restrict__ psi, const unsigned char* __restrict__ data,
                                               const PhaseArgs a) {
  __shared__ double s_beta[kPhaseMaxQ * kPhaseMaxQ];
  __shared__ double s_alpha[kPhaseMaxQ];
  __shared__ double s_rho[kPhaseMaxQ];  // sum over the block's set bits b >= 10 of beta[q][b]
  __shared__ double s_theta_p;          // c + the polynomial on the block's bits alone
  const double* coef = reinterpret_cast<const double*>(data);
  for (int i = threadIdx.x; i < kPhaseMaxQ * kPhaseMaxQ; i += 256) s_beta[i] = coef[1 + kPhaseMaxQ + i];
  if (threadIdx.x < kPhaseMaxQ) s_alpha[threadIdx.x] = coef[1 + threadIdx.x];
  __syncthreads();
  const uint64_t pbits = (uint64_t)blockIdx.x << 10;  // amplitude bits 10 .. lb-1 of this block
  if (threadIdx.x < kPhaseMaxQ) {
    const int q = threadIdx.x;
    double r = 0.0;
    for (int b = 10; b < a.lb; ++b)
      if ((pbits >> b) & 1) r += s_beta[q * kPhaseMaxQ + b];
    s_rho[q] = r;
  } else if (threadIdx.x == 64) {
    double t = coef[0];
    for (int b = 10; b < a.lb; ++b) {
      if (!((pbits >> b) & 1)) continue;
      t += s_alpha[b];
      for (int b2 = 10; b2 < b; ++b2)
        if ((pbits >> b2) & 1) t += s_beta[b * kPhaseMaxQ + b2];
    }
    s_theta_p = t;
  }
  __syncthreads();

  // this thread's low part: bits 1..8 from the thread, 10.. from the block
  const uint64_t e0 = (uint64_t)blockIdx.x * 512 + threadIdx.x;
  const uint64_t base = 2 * e0;
  const int lq = a.lb < 9 ? a.lb : 9;  // thread bits 1 .. lq-1
  double th = s_theta_p, g0 = s_alpha[0] + s_rho[0], g9 = s_alpha[9] + s_rho[9];
  for (int q = 1; q < lq; ++q) {
    if (!((base >> q) & 1)) continue;
    double r = s_alpha[q] + s_rho[q];
    for (int q2 = 1; q2 < q; ++q2)
      if ((base >> q2) & 1) r += s_beta[q * kPhaseMaxQ + q2];
    th += r;
    g0 += s_beta[q];
    g9 += s_beta[9 * kPhaseMaxQ + q];
  }
  // bit 9 exists only from 10 qubits up; its coefficients are zero below
  const double b09 = s_beta[9];
  const float t00 = fold(th), t10 = fold(th + g0), t01 = fold(th + g9), t11 = fold(th + g0 + g9 + b09);
  float gam[kPhaseMaxHigh];
#pragma unroll
  for (int j = 0; j < kPhaseMaxHigh; ++j) {
    gam[j] = 0.f;
    if (j < a.nh) {
      const int b = a.lb + j;
      double r = s_rho[b];
      for (int q = 1; q < lq; ++q)
        if ((base >> q) & 1) r += s_beta[b * kPhaseMaxQ + q];
      gam[j] = fold(r);
    }
  }

  const float4* tab = reinterpret_cast<const float4*>(data + kPhaseCoefBytes);
  const uint64_t span = (uint64_t)1 << (a.lb - 1);  // elements per sweep of the grid
  const uint64_t sweeps = (uint64_t)1 << a.nh;
  const bool ok0 = e0 < a.pairs, ok1 = e0 + 256 < a.pairs;  // false only below 10 qubits
  const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
  // the next sweep's two elements and table entry are loaded before this
  // sweep's math, so a wave keeps four 16-byte loads in flight and never
  // waits on the table
  float4 v0 = ok0 ? gld<NT>(psi + e0) : zero;
  float4 v1 = ok1 ? gld<NT>(psi + e0 + 256) : zero;
  float4 hk = tab[0];
  for (uint64_t k = 0; k < sweeps; ++k) {
    const uint64_t f0 = e0 + k * span, f1 = f0 + 256;
    float4 n0 = zero, n1 = zero, nk = zero;
    if (k + 1 < sweeps) {  // ok0 and ok1 hold whenever there is a next sweep
      n0 = gld<NT>(psi + f0 + span);
      n1 = gld<NT>(psi + f1 + span);
      nk = tab[k + 1];
    }
    float G = hk.x;
#pragma unroll
    for (int j = 0; j < kPhaseMaxHigh; ++j) {
      if (j < a.nh && ((k >> j) & 1)) G += gam[j];
      if ((j & 3) == 3) G -= rintf(G);  // keep the sum small: full FP32 resolution
    }
    if (ok0) {
      const float2 lo = rotate(make_float2(v0.x, v0.y), t00 + G);
      const float2 hi = rotate(make_float2(v0.z, v0.w), t10 + G + hk.y);
      gst<NT>(psi + f0, make_float4(lo.x, lo.y, hi.x, hi.y));
    }
    if (ok1) {
      const float2 lo = rotate(make_float2(v1.x, v1.y), t01 + G + hk.z);
      const float2 hi = rotate(make_float2(v1.z, v1.w), t11 + G + hk.y + hk.z);
      gst<NT>(psi + f1, make_float4(lo.x, lo.y, hi.x, hi.y));
    }
    v0 = n0;
    v1 = n1;
    hk = nk;
  }
}

}  // namespace

void launch_phase(int n, void* psi, const unsigned char* data, hipStream_t st) {
  PhaseArgs a{};
  a.pairs = (uint64_t)1 << (n - 1);
  a.n = n;
  a.lb = phase_low_bits(n);
  a.nh = n - a.lb;
  const unsigned blocks = a.lb > 10 ? 1u << (a.lb - 10) : 1u;  // 512 elements (1024 amplitudes) per block
  if (n >= kern::kNtMinQubits)
    hipLaunchKernelGGL(k_phase<true>, dim3(blocks), dim3(256), 0, st, (float4*)psi, data, a);
  else
    hipLaunchKernelGGL(k_phase<false>, dim3(blocks), dim3(256), 0, st, (float4*)psi, data, a);
  SV_HIP(hipGetLastError());
}

}  // namespace sv
