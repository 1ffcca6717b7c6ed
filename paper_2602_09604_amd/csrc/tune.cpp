// Autotuner: per pass class, time every candidate kernel variant and tile
// shape on the device and keep the fastest.
//
// A pass class is (precision, k, bit 0 is a target, number of targets in
// bits 1..6).  That is what decides coalescing (targets in the low bits split
// the contiguous wavefront rows), the LDS tile split, and whether a matrix-core
// variant applies.  Candidates: the register kernel, the LDS kernel with 2^10
// and 2^12 amplitude tiles, and the MFMA kernel for k >= 4 in MFMA precisions.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <random>
#include <sstream>
#include <tuple>

#include "sv_internal.h"

namespace sv {

void* state_psi(sv_state* s);
int state_n(sv_state* s);
hipStream_t state_stream(sv_state* s);
bool state_poisoned(sv_state* s);
void state_poison(sv_state* s);
int batch_lds_max_n();
void set_batch_lds_max_n(int n);
int batch_lds_cap();
void batch_run_impl(void* const* psis, const int* ns, const sv_gate* const* circuits, const size_t* n_gates,
                    size_t n_circ, const sv_run_opts& o, hipStream_t st, int lds_max_n, double* gpu_s,
                    uint64_t* passes_out, double* fuse_s, uint64_t* bytes_out, uint64_t* launches_out);

namespace {

struct Choice {
  int variant;
  int tile_bits;
  double ms;
};
using Key = std::tuple<int, int, int, int>;  // precision, k, q0, nlow

std::mutex g_mu;
std::map<Key, Choice> g_table;

int count_low(int k, const int* s) {
  int c = 0;
  for (int j = 0; j < k; ++j)
    if (s[j] >= 1 && s[j] < 7) ++c;
  return c;
}

Key key_of(int precision, int k, const int* s) {
  // below k = 4 every precision runs on the VALU kernels
  const int p = k >= 4 ? precision : SV_PREC_FP32_VALU;
  return Key{p, k, s[0] == 0 ? 1 : 0, count_low(k, s)};
}

bool lookup(int precision, int k, const int* s, Choice* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_table.find(key_of(precision, k, s));
  if (it == g_table.end()) return false;
  *out = it->second;
  return true;
}

}  // namespace

Shape tuned_shape(int variant, int n, int k, const int* s, int precision) {
  (void)n;
  Shape sh;
  sh.tile_bits = 12;
  Choice c;
  if (lookup(precision, k, s, &c) && c.variant == variant && variant == V_LDS) sh.tile_bits = c.tile_bits;
  return sh;
}

// AUTO choice from the tuned table; -1 when the class has not been tuned.
int tuned_variant(int n, int k, const int* s, int precision) {
  (void)n;
  Choice c;
  if (!lookup(precision, k, s, &c)) return -1;
  return c.variant;
}

}  // namespace sv

using namespace sv;

extern "C" {

int sv_autotune(sv_state* s, int budget_ms) {
  if (!s) return fail(SV_EINVAL, "state handle is NULL");
  if (state_poisoned(s)) return fail(SV_ESTATE, "handle poisoned by an earlier device failure");
  const int n = state_n(s);
  if (n < 16) return fail(SV_EINVAL, "autotune needs a state of at least 16 qubits");
  const auto t_start = std::chrono::steady_clock::now();
  unsigned char* dev = nullptr;
  unsigned char* host = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  try {
    SV_HIP(hipMalloc(&dev, 1 << 17));
    SV_HIP(hipHostMalloc(&host, 1 << 17, hipHostMallocDefault));
    SV_HIP(hipEventCreate(&e0));
    SV_HIP(hipEventCreate(&e1));
    hipStream_t st = state_stream(s);
    void* psi = state_psi(s);
    launch_init_basis(psi, n, 0, st);
    std::mt19937_64 rng(12345);
    std::normal_distribution<double> nd;
    std::map<Key, Choice> found;
    const int precs[4] = {SV_PREC_FP32_VALU, SV_PREC_FP32_MFMA, SV_PREC_BF16X3, SV_PREC_FP16X3};
    for (int pi = 0; pi < 4; ++pi) {
      const int prec = precs[pi];
      for (int k = (prec == SV_PREC_FP32_VALU ? 1 : 4); k <= SV_MAX_K; ++k) {
        // a random (not unitary; timing does not depend on it) matrix
        const int d = 1 << k;
        std::vector<double> mat((size_t)2 * d * d);
        for (auto& v : mat) v = nd(rng) / d;
        for (int q0 = 0; q0 <= 1; ++q0) {
          for (int nlow = 0; nlow + q0 <= k && nlow <= 6; ++nlow) {
            if (k - q0 - nlow > n - 7) continue;  // not enough high bits
            Pass p;
            p.k = k;
            p.precision = prec;
            int c = 0;
            if (q0) p.s[c++] = 0;
            for (int i = 0; i < nlow; ++i) p.s[c++] = 1 + i;
            for (; c < k; ++c) p.s[c] = n - k + c;  // the rest on the top qubits
            std::sort(p.s, p.s + k);
            std::vector<std::pair<int, int>> cands = {{V_REG, 12}, {V_LDS, 10}, {V_LDS, 12}};
            if (mfma_supported(k, prec) && n >= k + 6) cands.push_back({V_MFMA, 12});
            if (shfl_eligible(n, k, p.s)) cands.push_back({V_SHFL, 12});
            Choice best{V_REG, 12, 1e30};
            for (auto& cand : cands) {
              p.variant = cand.first;
              p.tile_bits = cand.second;
              p.mfma_x = p.variant == V_MFMA ? mfma_exchange_mask(n, p) : 0;
              p.mat_bytes = pass_data_bytes(p);
              p.mat_off = 0;
              encode_pass_data(p, mat.data(), host);
              SV_HIP(hipMemcpyAsync(dev, host, p.mat_bytes, hipMemcpyHostToDevice, st));
              launch_pass(p, n, psi, dev, st);  // warm-up
              std::vector<float> t;
              for (int r = 0; r < 3; ++r) {
                SV_HIP(hipEventRecord(e0, st));
                launch_pass(p, n, psi, dev, st);
                SV_HIP(hipEventRecord(e1, st));
                SV_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                SV_HIP(hipEventElapsedTime(&ms, e0, e1));
                t.push_back(ms);
              }
              std::sort(t.begin(), t.end());
              if (t[1] < best.ms) best = Choice{cand.first, cand.second, t[1]};
              // renormalise occasionally: random matrices grow the state
              launch_init_basis(psi, n, 0, st);
            }
            found[key_of(prec, k, p.s)] = best;
            if (budget_ms > 0 &&
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count() >
                    budget_ms)
              goto done;
          }
        }
      }
    }
  done:
    SV_HIP(hipStreamSynchronize(st));
    {
      // Batched kernel: largest state kept LDS-resident.  A batch of 64
      // two-layer RY-RZ + CNOT-ladder circuits per size, timed LDS-resident
      // against level-synchronous sweeps; the limit grows while LDS wins.
      const double pi = 3.14159265358979323846;
      std::uniform_real_distribution<double> ang(0.0, 2 * pi);
      int thr = 9;
      for (int nb = 10; nb <= std::min(14, batch_lds_cap()); ++nb) {
        const int copies = 64;
        if (((size_t)copies << nb) > ((size_t)1 << n)) break;
        std::vector<std::vector<double>> mats;
        std::vector<sv_gate> gates;
        for (int layer = 0; layer < 2; ++layer) {
          for (int q = 0; q < nb; ++q) {
            const double t = ang(rng), f = ang(rng);
            mats.push_back({std::cos(t / 2), 0, -std::sin(t / 2), 0, std::sin(t / 2), 0, std::cos(t / 2), 0});
            mats.push_back({std::cos(f / 2), -std::sin(f / 2), 0, 0, 0, 0, std::cos(f / 2), std::sin(f / 2)});
          }
          for (int q = 0; q + 1 < nb; ++q) {
            std::vector<double> cx(32, 0.0);
            cx[2 * 0] = cx[2 * (2 * 4 + 2)] = cx[2 * (3 * 4 + 1)] = cx[2 * (1 * 4 + 3)] = 1.0;
            mats.push_back(cx);
          }
        }
        size_t mi = 0;
        for (int layer = 0; layer < 2; ++layer) {
          for (int q = 0; q < nb; ++q)
            for (int r = 0; r < 2; ++r) {
              sv_gate g{};
              g.k = 1;
              g.qubits[0] = q;
              g.matrix = mats[mi++].data();
              gates.push_back(g);
            }
          for (int q = 0; q + 1 < nb; ++q) {
            sv_gate g{};
            g.k = 2;
            g.qubits[0] = q;
            g.qubits[1] = q + 1;
            g.matrix = mats[mi++].data();
            gates.push_back(g);
          }
        }
        std::vector<void*> psis(copies);
        std::vector<int> ns(copies, nb);
        std::vector<const sv_gate*> circs(copies, gates.data());
        std::vector<size_t> counts(copies, gates.size());
        for (int c = 0; c < copies; ++c) psis[c] = (float2*)psi + ((size_t)c << nb);
        sv_run_opts o{};
        o.max_k = 4;
        o.fusion = SV_FUSE_GREEDY;
        double t_lds = 0, t_lvl = 0, best_lds = 1e30, best_lvl = 1e30;
        for (int r = 0; r < 3; ++r) {
          batch_run_impl(psis.data(), ns.data(), circs.data(), counts.data(), copies, o, st, 14, &t_lds, nullptr,
                         nullptr, nullptr, nullptr);
          batch_run_impl(psis.data(), ns.data(), circs.data(), counts.data(), copies, o, st, 0, &t_lvl, nullptr,
                         nullptr, nullptr, nullptr);
          best_lds = std::min(best_lds, t_lds);
          best_lvl = std::min(best_lvl, t_lvl);
        }
        if (best_lds <= best_lvl) thr = nb;
        else break;
      }
      set_batch_lds_max_n(thr);
    }
    launch_init_basis(psi, n, 0, st);
    {
      std::lock_guard<std::mutex> lk(g_mu);
      for (auto& kv : found) g_table[kv.first] = kv.second;
    }
    bump_plan_epoch();
    (void)hipFree(dev);
    (void)hipHostFree(host);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return SV_OK;
  } catch (const DeviceError& e) {
    state_poison(s);
    if (dev) (void)hipFree(dev);
    if (host) (void)hipHostFree(host);
    return fail(SV_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.err));
  } catch (...) {
    (void)hipStreamSynchronize(state_stream(s));
    if (dev) (void)hipFree(dev);
    if (host) (void)hipHostFree(host);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return fail(SV_ENOMEM, "host failure during tuning");
  }
}

// JSON: {"entries": [[precision, k, q0, nlow, variant, tile_bits, ms], ...]}
int sv_tune_save(const char* path) {
  return host_guard([&]() -> int {
    if (!path) return fail(SV_EINVAL, "path is NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    std::ofstream f(path);
    if (!f) return fail(SV_EINVAL, std::string("cannot write ") + path);
    f << "{\"format\": \"libsv-tune-1\", \"batch_lds_max_n\": " << batch_lds_max_n() << ", \"entries\": [";
    bool first = true;
    for (auto& kv : g_table) {
      f << (first ? "" : ", ") << "[" << std::get<0>(kv.first) << ", " << std::get<1>(kv.first) << ", "
        << std::get<2>(kv.first) << ", " << std::get<3>(kv.first) << ", " << kv.second.variant << ", "
        << kv.second.tile_bits << ", " << kv.second.ms << "]";
      first = false;
    }
    f << "]}\n";
    return f ? SV_OK : fail(SV_EINVAL, "write failed");
  });
}

int sv_tune_load(const char* path) {
  return host_guard([&]() -> int {
    if (!path) return fail(SV_EINVAL, "path is NULL");
    std::ifstream f(path);
    if (!f) return fail(SV_EINVAL, std::string("cannot read ") + path);
    std::stringstream ss;
    ss << f.rdbuf();
    std::string text = ss.str();
    const size_t at = text.find("\"entries\"");
    if (text.find("libsv-tune-1") == std::string::npos || at == std::string::npos)
      return fail(SV_EINVAL, "not a libsv tuning file");
    std::map<Key, Choice> parsed;
    size_t pos = text.find('[', at);
    if (pos == std::string::npos) return fail(SV_EINVAL, "malformed tuning file");
    ++pos;
    while (true) {
      const size_t open = text.find('[', pos);
      if (open == std::string::npos) break;
      const size_t close = text.find(']', open);
      if (close == std::string::npos) return fail(SV_EINVAL, "malformed tuning file");
      int p, k, q0, nlow, var, tb;
      double ms;
      if (std::sscanf(text.c_str() + open, "[%d, %d, %d, %d, %d, %d, %lf]", &p, &k, &q0, &nlow, &var, &tb, &ms) != 7)
        return fail(SV_EINVAL, "malformed tuning entry");
      if (p < 0 || p > 3 || k < 1 || k > SV_MAX_K || q0 < 0 || q0 > 1 || nlow < 0 || nlow > 6 || var < V_REG ||
          var > V_SHFL || var == V_PHASE || (tb != 10 && tb != 12))
        return fail(SV_EINVAL, "tuning entry out of range");
      parsed[Key{p, k, q0, nlow}] = Choice{var, tb, ms};
      pos = close + 1;
    }
    const size_t bl = text.find("\"batch_lds_max_n\"");
    if (bl != std::string::npos) {
      int v = 0;
      if (std::sscanf(text.c_str() + text.find(':', bl) + 1, "%d", &v) != 1 || v < 1 || v > 14)
        return fail(SV_EINVAL, "batch_lds_max_n out of range");
      set_batch_lds_max_n(v);
    }
    {
      std::lock_guard<std::mutex> lk(g_mu);
      for (auto& kv : parsed) g_table[kv.first] = kv.second;
    }
    bump_plan_epoch();
    return SV_OK;
  });
}

}  // extern "C"
