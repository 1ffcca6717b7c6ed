// Fusion cost model: a 3-layer MLP (F -> W -> W -> 1, ReLU) trained on the
// GPU with mean squared error and Adam, all in hand-written kernels.
//
// Parameter layout (row-major): W1 [W x F], b1 [W], W2 [W x W], b2 [W],
// W3 [1 x W], b3 [1].
//
// k_mlp_grad: one workgroup per chunk of 64 samples keeps the inputs and both
// hidden activations in LDS, runs the forward pass, the loss and the whole
// backward pass, and writes its chunk's gradient (sum over its samples of
// dL/dparam) to a partial buffer.  k_mlp_reduce sums the partials in a fixed
// order (deterministic), k_mlp_adam applies the update.
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "sv_internal.h"

struct sv_mlp {
  int width = 64;
  int nparams = 0;
  hipStream_t stream = nullptr;
  float* params = nullptr;  // device
  float* grad = nullptr;    // device, last loss_grad
  float* m = nullptr;       // Adam moments
  float* v = nullptr;
  float* partial = nullptr;  // [max_blocks][nparams + 1]
  int max_blocks = 0;
  float* loss_dev = nullptr;
  float* host_pinned = nullptr;  // nparams + 1
  int step = 0;
};

namespace sv {

namespace {

constexpr int F = SV_COST_FEATURES;
constexpr int CH = 64;  // samples per workgroup

int num_params(int w) { return w * F + w + w * w + w + w + 1; }

template <int W>
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ P, const float* __restrict__ X,
                                                  const float* __restrict__ T, int B, float* __restrict__ partial,
                                                  int stride) {
  __shared__ float xs[CH][F + 1];
  __shared__ float h1[CH][W + 1];
  __shared__ float h2[CH][W + 1];
  __shared__ float dy[CH];
  const float* W1 = P;
  const float* b1 = W1 + W * F;
  const float* W2 = b1 + W;
  const float* b2 = W2 + W * W;
  const float* W3 = b2 + W;
  const float* b3 = W3 + W;
  const int tid = threadIdx.x;
  const int s0 = blockIdx.x * CH;
  const int ns = min(CH, B - s0);
  float* out = partial + (size_t)blockIdx.x * stride;
  for (int i = tid; i < CH * F; i += 256) {
    const int s = i / F, f = i % F;
    xs[s][f] = s < ns ? X[(size_t)(s0 + s) * F + f] : 0.f;
  }
  __syncthreads();
  // forward, layer 1 and 2
  for (int i = tid; i < CH * W; i += 256) {
    const int s = i / W, j = i % W;
    float a = b1[j];
    for (int f = 0; f < F; ++f) a = fmaf(W1[j * F + f], xs[s][f], a);
    h1[s][j] = a > 0.f ? a : 0.f;
  }
  __syncthreads();
  for (int i = tid; i < CH * W; i += 256) {
    const int s = i / W, j = i % W;
    float a = b2[j];
    for (int q = 0; q < W; ++q) a = fmaf(W2[j * W + q], h1[s][q], a);
    h2[s][j] = a > 0.f ? a : 0.f;
  }
  __syncthreads();
  // output, loss and dL/dy = 2 (y - t) / B
  if (tid < CH) {
    float d = 0.f;
    if (tid < ns) {
      float y = b3[0];
      for (int q = 0; q < W; ++q) y = fmaf(W3[q], h2[tid][q], y);
      d = y - T[s0 + tid];
    }
    dy[tid] = d;
  }
  __syncthreads();
  if (tid == 0) {
    float l = 0.f;
    for (int s = 0; s < ns; ++s) l += dy[s] * dy[s];
    out[stride - 1] = l;  // sum of squared errors of the chunk
  }
  if (tid < CH) dy[tid] *= 2.f / (float)B;
  __syncthreads();
  float* gW1 = out;
  float* gb1 = gW1 + W * F;
  float* gW2 = gb1 + W;
  float* gb2 = gW2 + W * W;
  float* gW3 = gb2 + W;
  float* gb3 = gW3 + W;
  // layer 3 gradients
  if (tid < W) {
    float a = 0.f;
    for (int s = 0; s < CH; ++s) a = fmaf(dy[s], h2[s][tid], a);
    gW3[tid] = a;
  }
  if (tid == W) {
    float a = 0.f;
    for (int s = 0; s < CH; ++s) a += dy[s];
    gb3[0] = a;
  }
  __syncthreads();
  // dh2 (in place of h2): dy * W3 where the unit was active
  for (int i = tid; i < CH * W; i += 256) {
    const int s = i / W, j = i % W;
    h2[s][j] = h2[s][j] > 0.f ? dy[s] * W3[j] : 0.f;
  }
  __syncthreads();
  // layer 2 gradients: gW2[i][j] = sum_s dh2[s][i] h1[s][j]
  for (int i = tid; i < W * W; i += 256) {
    const int r = i / W, c = i % W;
    float a = 0.f;
    for (int s = 0; s < CH; ++s) a = fmaf(h2[s][r], h1[s][c], a);
    gW2[i] = a;
  }
  for (int r = tid; r < W; r += 256) {
    float a = 0.f;
    for (int s = 0; s < CH; ++s) a += h2[s][r];
    gb2[r] = a;
  }
  __syncthreads();
  // dh1 = (dh2 W2) where the unit was active; computed into registers first
  // because the mask reads h1 in place
  float tmp[CH * W / 256];
#pragma unroll
  for (int t = 0; t < CH * W / 256; ++t) {
    const int i = tid + 256 * t;
    const int s = i / W, j = i % W;
    float a = 0.f;
    for (int q = 0; q < W; ++q) a = fmaf(h2[s][q], W2[q * W + j], a);
    tmp[t] = h1[s][j] > 0.f ? a : 0.f;
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < CH * W / 256; ++t) {
    const int i = tid + 256 * t;
    h1[i / W][i % W] = tmp[t];
  }
  __syncthreads();
  // layer 1 gradients: gW1[i][f] = sum_s dh1[s][i] x[s][f]
  for (int i = tid; i < W * F; i += 256) {
    const int r = i / F, c = i % F;
    float a = 0.f;
    for (int s = 0; s < CH; ++s) a = fmaf(h1[s][r], xs[s][c], a);
    gW1[i] = a;
  }
  for (int r = tid; r < W; r += 256) {
    float a = 0.f;
    for (int s = 0; s < CH; ++s) a += h1[s][r];
    gb1[r] = a;
  }
}

// Sum the per-chunk partials in chunk order: grad[i] = sum_b partial[b][i].
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ partial, int blocks, int stride,
                                                    float* __restrict__ grad, float* __restrict__ loss, int B) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < stride) {
    float a = 0.f;
    for (int b = 0; b < blocks; ++b) a += partial[(size_t)b * stride + i];
    if (i == stride - 1) *loss = a / (float)B;
    else grad[i] = a;
  }
}

__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ p, const float* __restrict__ g,
                                                  float* __restrict__ m, float* __restrict__ v, int n, float lr,
                                                  float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

template <int W>
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ P, const float* __restrict__ X, int B,
                                                     float* __restrict__ Y) {
  __shared__ float h1[4][W];
  __shared__ float h2[4][W];
  const float* W1 = P;
  const float* b1 = W1 + W * F;
  const float* W2 = b1 + W;
  const float* b2 = W2 + W * W;
  const float* W3 = b2 + W;
  const float* b3 = W3 + W;
  const int w = threadIdx.x / 64, j = threadIdx.x % 64;  // one wave per sample
  const int s = blockIdx.x * 4 + w;
  const bool ok = s < B;
  if (j < W) {
    float a = b1[j];
    if (ok)
      for (int f = 0; f < F; ++f) a = fmaf(W1[j * F + f], X[(size_t)s * F + f], a);
    h1[w][j] = a > 0.f ? a : 0.f;
  }
  __syncthreads();
  if (j < W) {
    float a = b2[j];
    for (int q = 0; q < W; ++q) a = fmaf(W2[j * W + q], h1[w][q], a);
    h2[w][j] = a > 0.f ? a : 0.f;
  }
  __syncthreads();
  if (j == 0 && ok) {
    float y = b3[0];
    for (int q = 0; q < W; ++q) y = fmaf(W3[q], h2[w][q], y);
    Y[s] = y;
  }
}

uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

void cost_model_set(const std::vector<float>& params, int width);

}  // namespace sv

using namespace sv;

#define MLP_GUARD_BEGIN try {
#define MLP_GUARD_END                                                                    \
  }                                                                                      \
  catch (const DeviceError& e) {                                                         \
    return fail(SV_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.err));      \
  }                                                                                      \
  catch (const std::bad_alloc&) {                                                        \
    return fail(SV_ENOMEM, "host allocation failed");                                    \
  }                                                                                      \
  catch (...) {                                                                          \
    return fail(SV_EINVAL, "unknown failure");                                           \
  }

extern "C" {

int sv_mlp_create(int width, uint64_t seed, void* hip_stream, sv_mlp** out) {
  if (!out) return fail(SV_EINVAL, "out is NULL");
  *out = nullptr;
  if (width != 64) return fail(SV_EINVAL, "width must be 64 (the kernels are built for it)");
  sv_mlp* m = new sv_mlp();
  MLP_GUARD_BEGIN
  m->width = width;
  m->nparams = num_params(width);
  m->stream = (hipStream_t)hip_stream;
  const size_t pb = sizeof(float) * m->nparams;
  SV_HIP(hipMalloc(&m->params, pb));
  SV_HIP(hipMalloc(&m->grad, pb));
  SV_HIP(hipMalloc(&m->m, pb));
  SV_HIP(hipMalloc(&m->v, pb));
  SV_HIP(hipMalloc(&m->loss_dev, sizeof(float)));
  SV_HIP(hipHostMalloc(&m->host_pinned, pb + sizeof(float), hipHostMallocDefault));
  // He-uniform weights from a SplitMix64 stream, zero biases
  std::vector<float> p(m->nparams, 0.f);
  uint64_t st = seed;
  auto fill = [&](size_t off, int count, int fan_in) {
    const double lim = std::sqrt(6.0 / fan_in);
    for (int i = 0; i < count; ++i) {
      const double u = (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0);
      p[off + i] = (float)((2.0 * u - 1.0) * lim);
    }
  };
  const int W = width;
  fill(0, W * F, F);
  fill((size_t)W * F + W, W * W, W);
  fill((size_t)W * F + W + W * W + W, W, W);
  SV_HIP(hipMemcpy(m->params, p.data(), pb, hipMemcpyHostToDevice));
  std::vector<float> z(m->nparams, 0.f);
  SV_HIP(hipMemcpy(m->m, z.data(), pb, hipMemcpyHostToDevice));
  SV_HIP(hipMemcpy(m->v, z.data(), pb, hipMemcpyHostToDevice));
  SV_HIP(hipMemcpy(m->grad, z.data(), pb, hipMemcpyHostToDevice));
  *out = m;
  return SV_OK;
  }
  catch (const DeviceError& e) {
    sv_mlp_free(m);
    return fail(SV_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.err));
  }
  catch (...) {
    sv_mlp_free(m);
    return fail(SV_ENOMEM, "host allocation failed");
  }
}

int sv_mlp_free(sv_mlp* m) {
  if (!m) return SV_OK;
  (void)hipStreamSynchronize(m->stream);
  if (m->params) (void)hipFree(m->params);
  if (m->grad) (void)hipFree(m->grad);
  if (m->m) (void)hipFree(m->m);
  if (m->v) (void)hipFree(m->v);
  if (m->partial) (void)hipFree(m->partial);
  if (m->loss_dev) (void)hipFree(m->loss_dev);
  if (m->host_pinned) (void)hipHostFree(m->host_pinned);
  delete m;
  return SV_OK;
}

int sv_mlp_num_params(const sv_mlp* m, size_t* count) {
  if (!m || !count) return fail(SV_EINVAL, "NULL argument");
  *count = (size_t)m->nparams;
  return SV_OK;
}

int sv_mlp_get_params(sv_mlp* m, float* host_params) {
  if (!m || !host_params) return fail(SV_EINVAL, "NULL argument");
  MLP_GUARD_BEGIN
  SV_HIP(hipMemcpyAsync(m->host_pinned, m->params, sizeof(float) * m->nparams, hipMemcpyDeviceToHost, m->stream));
  SV_HIP(hipStreamSynchronize(m->stream));
  std::memcpy(host_params, m->host_pinned, sizeof(float) * m->nparams);
  return SV_OK;
  MLP_GUARD_END
}

int sv_mlp_set_params(sv_mlp* m, const float* host_params) {
  if (!m || !host_params) return fail(SV_EINVAL, "NULL argument");
  MLP_GUARD_BEGIN
  std::memcpy(m->host_pinned, host_params, sizeof(float) * m->nparams);
  SV_HIP(hipMemcpyAsync(m->params, m->host_pinned, sizeof(float) * m->nparams, hipMemcpyHostToDevice, m->stream));
  SV_HIP(hipStreamSynchronize(m->stream));
  m->step = 0;
  return SV_OK;
  MLP_GUARD_END
}

int sv_mlp_forward(sv_mlp* m, const float* x_dev, int batch, float* y_dev) {
  if (!m || !x_dev || !y_dev || batch < 1) return fail(SV_EINVAL, "bad arguments");
  MLP_GUARD_BEGIN
  hipLaunchKernelGGL(k_mlp_forward<64>, dim3((batch + 3) / 4), dim3(256), 0, m->stream, m->params, x_dev, batch,
                     y_dev);
  SV_HIP(hipGetLastError());
  SV_HIP(hipStreamSynchronize(m->stream));
  return SV_OK;
  MLP_GUARD_END
}

static void mlp_loss_grad_async(sv_mlp* m, const float* x_dev, const float* y_dev, int batch) {
  const int blocks = (batch + CH - 1) / CH;
  const int stride = m->nparams + 1;
  if (blocks > m->max_blocks) {
    SV_HIP(hipStreamSynchronize(m->stream));
    if (m->partial) SV_HIP(hipFree(m->partial));
    m->partial = nullptr;
    SV_HIP(hipMalloc(&m->partial, sizeof(float) * (size_t)stride * blocks));
    m->max_blocks = blocks;
  }
  hipLaunchKernelGGL(k_mlp_grad<64>, dim3(blocks), dim3(256), 0, m->stream, m->params, x_dev, y_dev, batch,
                     m->partial, stride);
  SV_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_mlp_reduce, dim3((stride + 255) / 256), dim3(256), 0, m->stream, m->partial, blocks, stride,
                     m->grad, m->loss_dev, batch);
  SV_HIP(hipGetLastError());
}

int sv_mlp_loss_grad(sv_mlp* m, const float* x_dev, const float* y_dev, int batch, float* loss_host,
                     float* grad_host) {
  if (!m || !x_dev || !y_dev || batch < 1) return fail(SV_EINVAL, "bad arguments");
  MLP_GUARD_BEGIN
  mlp_loss_grad_async(m, x_dev, y_dev, batch);
  SV_HIP(hipMemcpyAsync(m->host_pinned, m->grad, sizeof(float) * m->nparams, hipMemcpyDeviceToHost, m->stream));
  SV_HIP(hipMemcpyAsync(m->host_pinned + m->nparams, m->loss_dev, sizeof(float), hipMemcpyDeviceToHost, m->stream));
  SV_HIP(hipStreamSynchronize(m->stream));
  if (loss_host) *loss_host = m->host_pinned[m->nparams];
  if (grad_host) std::memcpy(grad_host, m->host_pinned, sizeof(float) * m->nparams);
  return SV_OK;
  MLP_GUARD_END
}

static void mlp_adam_async(sv_mlp* m, float lr, float b1, float b2, float eps) {
  m->step += 1;
  const float c1 = 1.f - std::pow(b1, (float)m->step);
  const float c2 = 1.f - std::pow(b2, (float)m->step);
  hipLaunchKernelGGL(k_mlp_adam, dim3((m->nparams + 255) / 256), dim3(256), 0, m->stream, m->params, m->grad, m->m,
                     m->v, m->nparams, lr, b1, b2, eps, c1, c2);
  SV_HIP(hipGetLastError());
}

int sv_mlp_adam_step(sv_mlp* m, float lr, float beta1, float beta2, float eps) {
  if (!m || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(SV_EINVAL, "bad Adam arguments");
  MLP_GUARD_BEGIN
  mlp_adam_async(m, lr, beta1, beta2, eps);
  SV_HIP(hipStreamSynchronize(m->stream));
  return SV_OK;
  MLP_GUARD_END
}

int sv_mlp_train(sv_mlp* m, const float* x_dev, const float* y_dev, int n, int epochs, float lr, float* final_loss) {
  if (!m || !x_dev || !y_dev || n < 1 || epochs < 1 || !(lr > 0)) return fail(SV_EINVAL, "bad arguments");
  MLP_GUARD_BEGIN
  for (int e = 0; e < epochs; ++e) {
    mlp_loss_grad_async(m, x_dev, y_dev, n);
    mlp_adam_async(m, lr, 0.9f, 0.999f, 1e-8f);
  }
  mlp_loss_grad_async(m, x_dev, y_dev, n);  // loss at the final parameters
  SV_HIP(hipMemcpyAsync(m->host_pinned + m->nparams, m->loss_dev, sizeof(float), hipMemcpyDeviceToHost, m->stream));
  SV_HIP(hipStreamSynchronize(m->stream));
  if (final_loss) *final_loss = m->host_pinned[m->nparams];
  return SV_OK;
  MLP_GUARD_END
}

int sv_cost_model_install(sv_mlp* m) {
  return host_guard([&]() -> int {
    if (!m) return fail(SV_EINVAL, "NULL model");
    std::vector<float> p(m->nparams);
    if (int rc = sv_mlp_get_params(m, p.data())) return rc;
    cost_model_set(p, m->width);
    return SV_OK;
  });
}

}  // extern "C"
