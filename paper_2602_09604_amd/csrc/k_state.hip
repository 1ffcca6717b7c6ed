// State initialisation and the FP64 norm reduction sum |c_i|^2 (Eq. 1).
#include <mutex>

#include "k_common.h"

namespace sv {

namespace {
using kern::gld;
using kern::gst;

constexpr int kNormBlocks = 2048;  // partials of the first level
constexpr int kThreads = 256;

// Write |index>: a single coalesced sweep of 16-byte stores.
template <bool NT>
__global__ __launch_bounds__(256) void k_init_basis(float4* __restrict__ psi, uint64_t pairs,
                                                    uint64_t index) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < pairs; i += stride) {
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (i == (index >> 1)) {
      if (index & 1) v.z = 1.f;
      else v.x = 1.f;
    }
    gst<NT>(psi + i, v);
  }
}

// Streamed states (26 qubits and more): the same sweep walked in 32 KiB
// chunks per wave (wave W of NW takes chunks W, W + NW, ...), so the waves
// in flight write a moving window of the state, each its own contiguous
// run: 5.8 against 6.7 ms at 32 qubits, the same at 34 (the norm's read
// sweep gained nothing from the same walk).  Needs pairs to be a multiple
// of NW * kChunk.
constexpr uint64_t kChunk = 2048;  // float4 pairs per chunk

__global__ __launch_bounds__(256) void k_init_chunks(float4* __restrict__ psi, uint64_t pairs, uint64_t index) {
  const uint64_t NW = (uint64_t)gridDim.x * (256 / 64);
  const uint64_t W = (uint64_t)blockIdx.x * (256 / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const uint64_t rounds = pairs / (NW * kChunk);
  for (uint64_t c = 0; c < rounds; ++c) {
    const uint64_t e0 = (c * NW + W) * kChunk + lane;
#pragma unroll 8
    for (int k = 0; k < (int)(kChunk / 64); ++k) {
      const uint64_t i = e0 + (uint64_t)k * 64;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (i == (index >> 1)) {
        if (index & 1) v.z = 1.f;
        else v.x = 1.f;
      }
      gst<true>(psi + i, v);
    }
  }
}

__global__ __launch_bounds__(256) void k_init_basis_1q(float2* __restrict__ psi, uint64_t index) {
  if (threadIdx.x < 2) psi[threadIdx.x] = make_float2(threadIdx.x == index ? 1.f : 0.f, 0.f);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

__device__ double block_sum(double v) {
  __shared__ double part[kThreads / 64];
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) part[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kThreads / 64; ++i) s += part[i];
  return s;
}

// Level 1: each block owns a contiguous slice of float4 pairs; FP32 squares
// promoted to FP64 before accumulation.
template <bool NT>
__global__ __launch_bounds__(256) void k_norm_partial(const float4* __restrict__ psi, uint64_t pairs,
                                                      double* __restrict__ partials) {
  const uint64_t per = (pairs + gridDim.x - 1) / gridDim.x;
  const uint64_t lo = (uint64_t)blockIdx.x * per;
  const uint64_t hi = lo + per < pairs ? lo + per : pairs;
  double acc = 0.0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
    const float4 v = gld<NT>(psi + i);
    acc = fma((double)v.x, (double)v.x, acc);
    acc = fma((double)v.y, (double)v.y, acc);
    acc = fma((double)v.z, (double)v.z, acc);
    acc = fma((double)v.w, (double)v.w, acc);
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// Level 2: one block sums the partials in a fixed order.
__global__ __launch_bounds__(256) void k_norm_final(const double* __restrict__ partials, int parts,
                                                    double* __restrict__ out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < parts; i += kThreads) acc += partials[i];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) *out = s;
}

__global__ void k_norm_1q(const float2* __restrict__ psi, double* __restrict__ out) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < 2; ++i) s += (double)psi[i].x * psi[i].x + (double)psi[i].y * psi[i].y;
    *out = s;
  }
}

// Scratch of the allocation-free norm: the first-level partials, one copy per
// device (the runtime places it when the code object loads; it stays until the
// process ends).  Host code never passes this name to a kernel: it is a host
// stand-in, not a device address.  The device address comes from
// hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) double scratch[kNormBlocks];

}  // namespace

int norm_partials_needed() { return kNormBlocks; }

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on the current device (looked up on the first
// call per device).
static double* scratch_on_current_device() {
  int dev = 0;
  SV_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw DeviceError{hipErrorInvalidDevice, "scratch: device index"};
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    SV_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}

void launch_norm_noalloc(const void* psi, int n, double* out, hipStream_t st) {
  // launch_norm caps its first level at kNormBlocks partials and writes every
  // partial the second level reads, so the scratch needs no clearing
  launch_norm(psi, n, scratch_on_current_device(), kNormBlocks, out, st);
}

void launch_init_basis(void* psi, int n, uint64_t index, hipStream_t st) {
  if (n == 1) {
    hipLaunchKernelGGL(k_init_basis_1q, dim3(1), dim3(64), 0, st, (float2*)psi, index);
  } else {
    const uint64_t pairs = (uint64_t)1 << (n - 1);
    uint64_t blocks = (pairs + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (n >= kern::kNtMinQubits && pairs % ((uint64_t)kNormBlocks * 4 * kChunk) == 0)
      hipLaunchKernelGGL(k_init_chunks, dim3(kNormBlocks), dim3(256), 0, st, (float4*)psi, pairs, index);
    else if (n >= kern::kNtMinQubits)
      hipLaunchKernelGGL(k_init_basis<true>, dim3((unsigned)blocks), dim3(256), 0, st, (float4*)psi, pairs, index);
    else
      hipLaunchKernelGGL(k_init_basis<false>, dim3((unsigned)blocks), dim3(256), 0, st, (float4*)psi, pairs, index);
  }
  SV_HIP(hipGetLastError());
}

void launch_norm(const void* psi, int n, double* partials, int max_parts, double* out, hipStream_t st) {
  if (n == 1) {
    hipLaunchKernelGGL(k_norm_1q, dim3(1), dim3(64), 0, st, (const float2*)psi, out);
  } else {
    const uint64_t pairs = (uint64_t)1 << (n - 1);
    uint64_t blocks = (pairs + 1023) / 1024;  // at least 4 pairs per thread
    if (blocks > (uint64_t)max_parts) blocks = max_parts;
    if (blocks < 1) blocks = 1;
    if (n >= kern::kNtMinQubits)
      hipLaunchKernelGGL(k_norm_partial<true>, dim3((unsigned)blocks), dim3(256), 0, st, (const float4*)psi, pairs,
                         partials);
    else
      hipLaunchKernelGGL(k_norm_partial<false>, dim3((unsigned)blocks), dim3(256), 0, st, (const float4*)psi, pairs,
                         partials);
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(256), 0, st, (const double*)partials, (int)blocks, out);
  }
  SV_HIP(hipGetLastError());
}

}  // namespace sv
