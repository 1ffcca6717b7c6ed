// Internal declarations shared by the library's translation units (not part
// of the ABI).  Conventions: qubit q = bit q of the amplitude index; a pass's
// targets are held sorted ascending (s[0] < s[1] < ...) and its matrix has
// been permuted to match, so local bit j of the matrix index is state bit s[j].
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "../../include/sv.h"

namespace sv {

// ---------------------------------------------------------------- errors --
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

struct DeviceError {
  hipError_t err;
  const char* what;
};

// Run a host-only entry point body so that no C++ exception crosses the ABI.
template <class F>
int host_guard(F&& body) {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return fail(SV_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(SV_EINVAL, e.what());
  } catch (...) {
    return fail(SV_EINVAL, "unknown failure");
  }
}

#define SV_HIP(call)                                          \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) throw ::sv::DeviceError{e_, #call}; \
  } while (0)

// ---------------------------------------------------------------- passes --
// One in-place sweep of the state by a k-qubit gate.
enum Variant { V_AUTO = 0, V_REG = 1, V_LDS = 2, V_MFMA = 3, V_PHASE = 4, V_SHFL = 5 };
// Kernel family of a variant in sv_run_stats (the shuffle kernel keeps whole
// groups in registers: family 1 with the register kernel).
inline int variant_family(int v) { return v == V_SHFL ? V_REG : v; }

struct Pass {
  int k = 0;
  int s[SV_MAX_K] = {0, 0, 0, 0, 0, 0};  // sorted targets
  int variant = V_REG;                   // resolved (never AUTO)
  int precision = SV_PREC_FP32_VALU;
  size_t mat_off = 0;                    // byte offset of the pass data in the matrix arena
  size_t mat_bytes = 0;
  // launch shape (from the tuner or defaults)
  int tile_bits = 13;                    // LDS: log2 amplitudes per tile
  int reg_iters = 1;                     // REG: groups per thread
  int mfma_cols = 32;                    // MFMA: groups per wavefront tile
  // controlled passes: act only where (index & cmask) == cval
  uint64_t cmask = 0;
  uint64_t cval = 0;
  // nmux > 1 (matrix cores only): one launch applies 2^c matrices, one per
  // value of the c control bits in cmask (value v: control t = bit t of v),
  // their data one after another; cval is unused
  int nmux = 0;
  // matrix cores on a streamed state with targets on amplitude bits 1..3:
  // the bits (t - 1) of those targets, for the lane-exchange kernel and its
  // permuted encoding (0: the plain kernel); set by mfma_exchange_mask
  int mfma_x = 0;
};

// Launch shape defaults / tuned values.
struct Shape {
  int tile_bits = 13;
  int reg_iters = 1;
  int mfma_cols = 32;
};

// Kernel launchers (k_apply.hip, k_mfma.hip, k_state.hip).
void launch_pass(const Pass& p, int n, void* psi, const unsigned char* arena_dev, hipStream_t st);
void launch_init_basis(void* psi, int n, uint64_t index, hipStream_t st);
void launch_norm(const void* psi, int n, double* partials, int max_parts, double* out, hipStream_t st);
int norm_partials_needed();
// The same reduction with its partials in the library's static per-device
// scratch (no allocation); `out` is a device double.
void launch_norm_noalloc(const void* psi, int n, double* out, hipStream_t st);

// Bytes of device data a pass needs in the arena for its precision/variant,
// and the host-side encoder that writes it (matrix already normalised,
// complex128 row-major in sorted-target order).
size_t pass_data_bytes(const Pass& p);
void encode_pass_data(const Pass& p, const double* mat, unsigned char* dst);
bool mfma_supported(int k, int precision);
int mfma_exchange_mask(int n, const Pass& p);
// The register kernel streams a pass non-temporally with whole-line accesses:
// no target on amplitude bits 1..3, or at most three element-space targets
// with the lane exchange (k_apply_reg.hip).
bool reg_streams(int n, int k, const int* s);
// Controls the matrix-core kernel takes: at most three, none on bit 0, and at
// least one 32-group tile left.
bool mfma_ctrl_supported(int n, int k, uint64_t cmask);

// Planning helpers (plan.cpp).
void normalise_gate(int k, const int32_t* qubits, const double* mat, int* sorted_out,
                    std::vector<double>& mat_out);
int choose_variant(int n, int k, const int* s, int precision, int requested);
Shape tuned_shape(int variant, int n, int k, const int* s, int precision);
int lds_split(int tile_bits, int k, const int* s, int* m_out);
int lds_tile_bits_for(int n, int want);

// Fusion (fuse.cpp).
struct FusedGate {
  int k = 0;
  int q[SV_MAX_K] = {0, 0, 0, 0, 0, 0};  // ascending
  std::vector<double> mat;     // 2 * 4^k doubles, row-major, local bit j = q[j]
  uint64_t cmask = 0;          // controls of a controlled pass (0: none)
  uint64_t cval = 0;
};
// Controlled gates that fit in max_k qubits together with their controls,
// lifted to dense gates on the union; the others are kept (and later run as
// controlled passes).  `store` owns the lifted matrices.
void lower_controlled(const sv_gate* g, size_t n, int max_k, std::vector<sv_gate>& out,
                      std::vector<std::vector<double>>& store);
inline uint64_t gate_span(const sv_gate& g) {
  uint64_t m = g.cmask;
  for (int j = 0; j < g.k; ++j) m |= (uint64_t)1 << g.qubits[j];
  return m;
}
int validate_gates(const sv_gate* g, size_t n, int n_qubits);
void fuse_greedy(const sv_gate* g, size_t n, int max_k, std::vector<FusedGate>& out,
                 std::vector<int32_t>& block_of);
void fuse_none(const sv_gate* g, size_t n, std::vector<FusedGate>& out, std::vector<int32_t>& block_of);
void fuse_maxblock(const sv_gate* g, size_t n, int max_k, std::vector<FusedGate>& out,
                   std::vector<int32_t>& block_of);
// Partition searches.  max_ctrl > 0 lets a block take diagonal gates that
// reach outside its qubits as controls (see block_split).
void maxblock_partition(const sv_gate* g, size_t n, int max_k, bool narrow, std::vector<std::vector<int>>& blocks,
                        int max_ctrl = 0);
void beam_partition(const sv_gate* g, size_t n, int max_k, int width, int topm,
                    std::vector<std::vector<int>>& blocks, int max_ctrl = 0);
// Fused gates of a partition, in block order; block_of[i] is the index of
// the first fused gate of gate i's block.  With max_ctrl > 0 a block may come
// out as 2^c controlled gates on the same targets, one per control value.
void fuse_blocks(const sv_gate* g, size_t n, const std::vector<std::vector<int>>& blocks,
                 std::vector<FusedGate>& out, std::vector<int32_t>& block_of, int max_ctrl = 0);
// Control bits a block may use: at or above kCtrlMinBit, so that every
// control value covers whole 128-byte lines (runs of at least 16 amplitudes)
// and the matrix-core passes keep their streaming stores.
constexpr int kCtrlMinBit = 4;
constexpr uint64_t kCtrlLowBits = ((uint64_t)1 << kCtrlMinBit) - 1;
// Controls a fused block takes when the search allows them, and the smallest
// state where it does (with k < 4 targets a block with c controls runs as 2^c
// register launches, each over 2^-c of the state, which must still fill the
// GPU).
constexpr int kBlockCtrl = 3;
constexpr int kBlockCtrlMinQubits = 28;
bool is_diagonal_gate(const sv_gate& g);
// Targets and controls of a block: every qubit that only diagonal members
// touch, at or above kCtrlMinBit, may be a control (the block's unitary is
// block-diagonal in it); the highest such qubits become controls, at most
// max_ctrl of them, and at least one qubit stays a target.
void block_split(const sv_gate* g, const std::vector<int>& members, int max_ctrl, uint64_t& targets,
                 uint64_t& controls);
// Set on threads of a host worker pool so that the work they call does not
// start threads of its own.
bool host_pool_worker();
void set_host_pool_worker(bool on);
void fuse_phase(const sv_gate* g, size_t n, int max_k, std::vector<FusedGate>& out, std::vector<int32_t>& block_of);
bool is_phase_matrix(int k, const double* mat);

// Quadratic phase polynomial theta(x) = c + sum_q alpha_q x_q + sum_{a<b} beta_ab x_a x_b
// (angles in radians) of a run of pure-phase diagonal gates.
struct PhasePoly {
  double c = 0.0;
  std::vector<double> alpha;                    // per qubit
  std::vector<std::vector<double>> beta;        // beta[a][b], a < b
  explicit PhasePoly(int n = 0) : alpha(n, 0.0), beta(n, std::vector<double>(n, 0.0)) {}
  void add_gate(int k, const int* q, const double* mat);
};
// Device data of one phase pass (angles in turns, each folded into
// [-1/2, 1/2)): the polynomial's coefficients as doubles -- c, alpha[q] and
// beta[a][b] stored symmetrically, kPhaseMaxQ wide -- then, for the index
// bits above the low span of 2^lb amplitudes one grid sweep covers
// (lb = phase_low_bits(n)), one float4 per value k of those bits:
// (theta_high(k), sum_j k_j beta[0][lb + j], sum_j k_j beta[9][lb + j], 0),
// where theta_high is the polynomial on the high bits alone without c.
constexpr int kPhaseMaxQ = SV_MAX_QUBITS;
constexpr int kPhaseLowBits = 28;
constexpr int kPhaseMaxHigh = kPhaseMaxQ - kPhaseLowBits;
constexpr size_t kPhaseCoefBytes = ((1 + kPhaseMaxQ + (size_t)kPhaseMaxQ * kPhaseMaxQ) * sizeof(double) + 15) / 16 * 16;
inline int phase_low_bits(int n) { return n < kPhaseLowBits ? n : kPhaseLowBits; }
inline size_t phase_data_bytes(int n) { return kPhaseCoefBytes + 16 * ((size_t)1 << (n - phase_low_bits(n))); }
void phase_data(const PhasePoly& p, int n, unsigned char* out);
void launch_phase(int n, void* psi, const unsigned char* data, hipStream_t st);
void launch_ctrl(const Pass& p, int n, void* psi, const float2* U, hipStream_t st);
bool shfl_eligible(int n, int k, const int* s);
void launch_shfl(const Pass& p, int n, void* psi, const float2* U, hipStream_t st);

// State reads (k_measure.hip).
size_t pauli_scratch_bytes();
void launch_pauli(const void* psi, int n, uint64_t f, int nt, const uint64_t* z, double* scratch, double* out,
                  hipStream_t st);
int marginal_max_qubits();
size_t marginal_scratch_bytes(int m);
void launch_marginal(const void* psi, int n, int m, const int* qubits, double* scratch, double* out,
                     hipStream_t st);
size_t sample_scratch_bytes(int n);
void launch_sample(const void* psi, int n, bool prepare, const double* uniforms, uint64_t shots, uint64_t* out,
                   double* scratch, hipStream_t st);
// Planning epoch: bumped whenever something fusion or variant choice reads
// changes (the installed cost model, the tuned launch table), so that a kept
// graph is never relaunched for a plan that would now come out different.
uint64_t plan_epoch();
void bump_plan_epoch();
// Learned fusion; max_ctrl > 0 adds candidates whose blocks take controls.
bool fuse_learned(const sv_gate* g, size_t n, int n_qubits, int max_k, int precision,
                  std::vector<FusedGate>& out, std::vector<int32_t>& block_of, int max_ctrl);

// Cost model (cost_model.cpp).
void cost_features(int k, const int* qubits, int n, int precision, float* out);
bool cost_model_ready();
double cost_model_predict_log(int k, const int* qubits, int n, int precision);

}  // namespace sv
