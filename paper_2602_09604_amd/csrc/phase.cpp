// Diagonal specialisation: pure-phase gates as phase polynomials.
//
// A diagonal unitary on at most two qubits a, b is exp(i theta) with
// theta = c + alpha_a x_a + alpha_b x_b + beta x_a x_b (four diagonal entries,
// four parameters), so any run of such gates (CZ, CP, RZ, Z, S, T, ...)
// multiplies amplitude i by exp(i theta(i)) with theta a quadratic polynomial
// in the bits of i.  Such gates commute with one another; fusion exploits it
// (fuse_phase) and the device applies a whole run as one elementwise pass
// (k_phase).
//
// The device receives the coefficients themselves (every pair, no limit on
// how many pairs interact) plus a small table over the index bits above the
// span one grid sweep covers; k_phase evaluates the rest per thread.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>

#include "sv_internal.h"

namespace sv {


namespace {
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kUnitTol = 1e-12;

uint64_t qmask_of(const sv_gate& g) { return gate_span(g); }

double wrap(double a) {
  a = std::fmod(a, kTwoPi);
  return a < 0 ? a + kTwoPi : a;
}
}  // namespace

bool is_phase_matrix(int k, const double* mat) {
  if (k < 1 || k > 2 || !mat) return false;
  const int d = 1 << k;
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c) {
      const double re = mat[2 * (r * d + c)], im = mat[2 * (r * d + c) + 1];
      if (r == c) {
        if (std::fabs(std::hypot(re, im) - 1.0) > kUnitTol) return false;
      } else if (re != 0.0 || im != 0.0) {
        return false;
      }
    }
  return true;
}

void PhasePoly::add_gate(int k, const int* q, const double* mat) {
  auto arg = [&](int l) { return std::atan2(mat[2 * (l * ((1 << k) + 1)) + 1], mat[2 * (l * ((1 << k) + 1))]); };
  if (k == 1) {
    const double t0 = arg(0), t1 = arg(1);
    c += t0;
    alpha[q[0]] += t1 - t0;
  } else {
    // local index l = b0 + 2 b1, b0 = bit of q[0], b1 = bit of q[1]
    const double t00 = arg(0), t10 = arg(1), t01 = arg(2), t11 = arg(3);
    c += t00;
    alpha[q[0]] += t10 - t00;
    alpha[q[1]] += t01 - t00;
    const int a = std::min(q[0], q[1]), b = std::max(q[0], q[1]);
    beta[a][b] += t11 - t10 - t01 + t00;
  }
}

void phase_data(const PhasePoly& p, int n, unsigned char* out) {
  // angles in turns, folded into [-1/2, 1/2) (sums of a few stay small, so
  // FP32 keeps ~2^-24 turn resolution on the device)
  auto turns = [](double a) {
    double t = wrap(a) / kTwoPi;
    return t >= 0.5 ? t - 1.0 : t;
  };
  std::memset(out, 0, kPhaseCoefBytes);
  double* coef = reinterpret_cast<double*>(out);
  double* alpha = coef + 1;
  double* beta = alpha + kPhaseMaxQ;
  const int m = std::min(n, (int)p.alpha.size());
  coef[0] = turns(p.c);
  for (int a = 0; a < m; ++a) {
    alpha[a] = turns(p.alpha[a]);
    for (int b = a + 1; b < m; ++b) beta[(size_t)a * kPhaseMaxQ + b] = beta[(size_t)b * kPhaseMaxQ + a] = turns(p.beta[a][b]);
  }
  const int lb = phase_low_bits(n), nh = n - lb;
  float* tab = reinterpret_cast<float*>(out + kPhaseCoefBytes);
  auto B = [&](int a, int b) { return beta[(size_t)a * kPhaseMaxQ + b]; };
  for (uint64_t k = 0; k < ((uint64_t)1 << nh); ++k) {
    double th = 0.0, b0 = 0.0, b9 = 0.0;
    for (int j = 0; j < nh; ++j) {
      if (!((k >> j) & 1)) continue;
      const int q = lb + j;
      th += alpha[q];
      for (int j2 = 0; j2 < j; ++j2)
        if ((k >> j2) & 1) th += B(lb + j2, q);
      b0 += B(0, q);
      if (n > 9) b9 += B(9, q);
    }
    tab[4 * k + 0] = (float)(th - std::nearbyint(th));
    tab[4 * k + 1] = (float)(b0 - std::nearbyint(b0));
    tab[4 * k + 2] = (float)(b9 - std::nearbyint(b9));
    tab[4 * k + 3] = 0.f;
  }
}

// Greedy max-k fusion in which pure-phase gates do not block one another.
// Two blocked sets: qubits a dense gate may not touch (every skipped gate)
// and qubits a phase gate may not touch (skipped dense gates only, since
// phase gates commute).  A dense seed grows a dense block that also takes the
// phase gates that fit; a phase seed collects every phase gate it can reach
// into a phase block (any width).
void fuse_phase(const sv_gate* g, size_t n, int max_k, std::vector<FusedGate>& out, std::vector<int32_t>& block_of) {
  out.clear();
  block_of.assign(n, -1);
  int nq = 1;
  std::vector<uint64_t> masks(n);
  std::vector<char> ph(n), consumed(n, 0);
  for (size_t i = 0; i < n; ++i) {
    masks[i] = qmask_of(g[i]);
    ph[i] = !g[i].cmask && is_phase_matrix(g[i].k, g[i].matrix);
    for (int q = 0; q < 64; ++q)
      if ((masks[i] >> q) & 1) nq = std::max(nq, q + 1);
  }
  std::vector<std::vector<int>> dense_blocks;
  for (size_t seed = 0; seed < n; ++seed) {
    if (consumed[seed]) continue;
    std::vector<int> members{(int)seed};
    consumed[seed] = 1;
    uint64_t block_dense = 0, block_phase = 0;
    if (ph[seed]) {
      for (size_t h = seed + 1; h < n; ++h) {
        if (consumed[h]) continue;
        if (ph[h] && (masks[h] & block_phase) == 0) {
          members.push_back((int)h);
          consumed[h] = 1;
        } else if (!ph[h]) {
          block_phase |= masks[h];
        }
      }
      PhasePoly poly(nq);
      for (int i : members) poly.add_gate(g[i].k, g[i].qubits, g[i].matrix);
      // canonical gates: CP(beta) per pair, diag(1, e^{i alpha}) per qubit, global phase on the first
      const size_t first = out.size();
      for (int a = 0; a < nq; ++a)
        for (int b = a + 1; b < nq; ++b) {
          const double bb = wrap(poly.beta[a][b]);
          if (bb == 0.0) continue;
          FusedGate f;
          f.k = 2;
          f.q[0] = a;
          f.q[1] = b;
          f.mat.assign(32, 0.0);
          f.mat[0] = f.mat[2 * 5] = f.mat[2 * 10] = 1.0;
          f.mat[2 * 15] = std::cos(bb);
          f.mat[2 * 15 + 1] = std::sin(bb);
          out.push_back(std::move(f));
        }
      for (int a = 0; a < nq; ++a) {
        const double aa = wrap(poly.alpha[a]);
        if (aa == 0.0) continue;
        FusedGate f;
        f.k = 1;
        f.q[0] = a;
        f.mat = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0, std::cos(aa), std::sin(aa)};
        out.push_back(std::move(f));
      }
      if (out.size() == first) {  // the block is a global phase only
        FusedGate f;
        f.k = 1;
        f.q[0] = g[seed].qubits[0];
        f.mat = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0};
        out.push_back(std::move(f));
      }
      const std::complex<double> gp = std::polar(1.0, poly.c);
      for (size_t e = 0; e < out[first].mat.size(); e += 2) {
        const std::complex<double> v = std::complex<double>(out[first].mat[e], out[first].mat[e + 1]) * gp;
        out[first].mat[e] = v.real();
        out[first].mat[e + 1] = v.imag();
      }
      for (int i : members) block_of[i] = (int32_t)first;
      continue;
    }
    uint64_t S = masks[seed];
    for (size_t h = seed + 1; h < n && !g[seed].cmask; ++h) {  // a controlled pass stays alone
      if (consumed[h]) continue;
      const uint64_t qh = masks[h];
      const bool fits = !g[h].cmask && __builtin_popcountll(S | qh) <= max_k;
      if (ph[h]) {
        if ((qh & block_phase) == 0 && fits) {
          S |= qh;
          members.push_back((int)h);
          consumed[h] = 1;
        } else {
          block_dense |= qh;
        }
      } else {
        if ((qh & block_dense) == 0 && fits) {
          S |= qh;
          members.push_back((int)h);
          consumed[h] = 1;
        } else {
          block_dense |= qh;
          block_phase |= qh;
        }
      }
      if (__builtin_popcountll(S) >= max_k && (S & ~block_dense) == 0 && (S & ~block_phase) == 0) break;
    }
    std::vector<FusedGate> one;
    std::vector<int32_t> tmp;
    std::vector<std::vector<int>> blocks{members};
    fuse_blocks(g, n, blocks, one, tmp);
    for (int i : members) block_of[i] = (int32_t)out.size();
    out.push_back(std::move(one[0]));
  }
}

}  // namespace sv
