/*
 * CPU complex128 state-vector oracle.  TEST INFRASTRUCTURE ONLY: it exists so
 * that tests, the smoke check and the benchmark's CPU-baseline leg can check
 * and time the GPU library against a plain, slow, obviously correct
 * implementation.  It shares no code with the GPU library and nothing in the
 * product may call it.
 *
 * Everything here is written straight from the paper's definitions:
 *   - the state is 2^n complex amplitudes, norm sum |c_i|^2 (Sec. II-A, Eq. 1-2);
 *   - a k-qubit gate is a 2^k x 2^k matrix applied by matrix-vector product to
 *     each of the 2^(n-k) groups of amplitudes that agree on all non-target bits
 *     and enumerate the target bits (Sec. II-A, Eq. 4);
 *   - a controlled gate acts only on the groups whose control bits hold the
 *     control values (the indicator 1_c of Eq. 4) and leaves the rest alone.
 * Gates are applied one at a time, in order, never fused and never reordered.
 *
 * Layout: psi[2*i] = Re c_i, psi[2*i+1] = Im c_i (IEEE binary64, no fast-math,
 * no FMA contraction).  Qubit q is bit q of the index; local bit j of the gate
 * matrix index is state bit qubits[j]; U is row-major, interleaved re/im.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)

int orc_threads(void) { return omp_get_max_threads(); }

/* |x> : all zero except amplitude x = 1 (Eq. 1 with one non-zero c_i). */
void orc_init_basis(double* psi, int n, uint64_t x) {
  const int64_t len = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < 2 * len; ++i) psi[i] = 0.0;
  psi[2 * x] = 1.0;
}

/* Eq. 4 with the control indicator 1_c: for each group g of the 2^(n-k)
 * groups, gather the 2^k amplitudes whose target bits enumerate
 * l = 0..2^k-1, multiply by U, scatter back -- but only for groups whose
 * control bits (cmask) equal cval; every other group is left as it is.
 * cmask = 0 is the plain gate. */
int orc_apply_controlled_gate(double* psi, int n, int k, const int32_t* qubits, const double* U,
                              uint64_t cmask, uint64_t cval) {
  if (k < 1 || k > 10 || k > n || !psi || !qubits || !U) return ORC_EINVAL;
  if ((cval & ~cmask) != 0 || (n < 64 && (cmask >> n) != 0)) return ORC_EINVAL;
  int sorted[10];
  for (int j = 0; j < k; ++j) {
    if (qubits[j] < 0 || qubits[j] >= n) return ORC_EINVAL;
    if ((cmask >> qubits[j]) & 1) return ORC_EINVAL; /* a qubit is a control or a target */
    for (int i = 0; i < j; ++i)
      if (qubits[i] == qubits[j]) return ORC_EINVAL;
    sorted[j] = qubits[j];
  }
  for (int a = 1; a < k; ++a) /* insertion sort, ascending */
    for (int b = a; b > 0 && sorted[b - 1] > sorted[b]; --b) {
      int t = sorted[b];
      sorted[b] = sorted[b - 1];
      sorted[b - 1] = t;
    }
  const int dim = 1 << k;
  uint64_t* off = (uint64_t*)malloc(sizeof(uint64_t) * dim);
  for (int l = 0; l < dim; ++l) {
    off[l] = 0;
    for (int j = 0; j < k; ++j)
      if ((l >> j) & 1) off[l] |= (uint64_t)1 << qubits[j];
  }
  const int64_t groups = (int64_t)1 << (n - k);
#pragma omp parallel
  {
    double* vr = (double*)malloc(sizeof(double) * dim);
    double* vi = (double*)malloc(sizeof(double) * dim);
#pragma omp for schedule(static)
    for (int64_t g = 0; g < groups; ++g) {
      /* base index: the bits of g with a zero inserted at every target bit */
      uint64_t base = (uint64_t)g;
      for (int j = 0; j < k; ++j) {
        const int s = sorted[j];
        const uint64_t low = base & (((uint64_t)1 << s) - 1);
        base = ((base >> s) << (s + 1)) | low;
      }
      if ((base & cmask) != cval) continue; /* 1_c = 0: the group is untouched */
      for (int l = 0; l < dim; ++l) {
        vr[l] = psi[2 * (base + off[l])];
        vi[l] = psi[2 * (base + off[l]) + 1];
      }
      for (int r = 0; r < dim; ++r) {
        double wr = 0.0, wi = 0.0;
        for (int c = 0; c < dim; ++c) {
          const double ur = U[2 * (r * dim + c)], ui = U[2 * (r * dim + c) + 1];
          wr += ur * vr[c] - ui * vi[c];
          wi += ur * vi[c] + ui * vr[c];
        }
        psi[2 * (base + off[r])] = wr;
        psi[2 * (base + off[r]) + 1] = wi;
      }
    }
    free(vr);
    free(vi);
  }
  free(off);
  return ORC_OK;
}

/* Eq. 4 for an uncontrolled gate. */
int orc_apply_gate(double* psi, int n, int k, const int32_t* qubits, const double* U) {
  return orc_apply_controlled_gate(psi, n, k, qubits, U, 0, 0);
}

/* Apply a serialised gate list in order (k[g], qubits[6*g..], matrices at
 * mats + 2*mat_off[g]; control mask and values cmask[g], cval[g], or no
 * controls at all when cmask is NULL). */
int orc_apply_circuit(double* psi, int n, int64_t n_gates, const int32_t* ks,
                      const int32_t* qubits6, const int64_t* mat_off, const double* mats,
                      const uint64_t* cmask, const uint64_t* cval) {
  for (int64_t g = 0; g < n_gates; ++g) {
    int rc = orc_apply_controlled_gate(psi, n, ks[g], qubits6 + 6 * g, mats + 2 * mat_off[g],
                                       cmask ? cmask[g] : 0, cmask ? cval[g] : 0);
    if (rc != ORC_OK) return rc;
  }
  return ORC_OK;
}

/* Pairwise (cascade) summation of |c_i|^2 over [lo, hi). */
static double norm_pairwise(const double* psi, int64_t lo, int64_t hi) {
  if (hi - lo <= 256) {
    double s = 0.0;
    for (int64_t i = lo; i < hi; ++i) s += psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
    return s;
  }
  const int64_t mid = lo + (hi - lo) / 2;
  return norm_pairwise(psi, lo, mid) + norm_pairwise(psi, mid, hi);
}

/* sum_i |c_i|^2 (Eq. 1).  The range is split into 2^p equal parts summed in
 * parallel, then combined pairwise, so the result does not depend on the
 * thread count. */
double orc_norm_sq(const double* psi, int64_t len) {
  int64_t parts = 1;
  while (parts < 256 && parts * 4096 <= len) parts *= 2;
  double* part = (double*)malloc(sizeof(double) * parts);
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < parts; ++p)
    part[p] = norm_pairwise(psi, p * (len / parts), p == parts - 1 ? len : (p + 1) * (len / parts));
  for (int64_t w = 1; w < parts; w *= 2)
    for (int64_t p = 0; p + w < parts; p += 2 * w) part[p] += part[p + w];
  double s = part[0];
  free(part);
  return s;
}

/* Comparison statistics between a complex64 state g (interleaved floats) and
 * a complex128 state o over `count` amplitudes.  out[0] = max |g_i - o_i|,
 * out[1] = sum |g-o|^2, out[2] = sum |o|^2, out[3] = sum |g|^2,
 * out[4], out[5] = Re, Im of <o|g> = sum conj(o_i) g_i. */
typedef struct {
  double mx, d2, o2, g2, ipr, ipi;
} cmp_acc;

static cmp_acc cmp_pairwise(const float* g, const double* o, int64_t lo, int64_t hi) {
  cmp_acc a = {0, 0, 0, 0, 0, 0};
  if (hi - lo <= 256) {
    for (int64_t i = lo; i < hi; ++i) {
      const double gr = g[2 * i], gi = g[2 * i + 1], orr = o[2 * i], oi = o[2 * i + 1];
      const double dr = gr - orr, di = gi - oi;
      const double d = sqrt(dr * dr + di * di);
      if (d > a.mx) a.mx = d;
      a.d2 += dr * dr + di * di;
      a.o2 += orr * orr + oi * oi;
      a.g2 += gr * gr + gi * gi;
      a.ipr += orr * gr + oi * gi;
      a.ipi += orr * gi - oi * gr;
    }
    return a;
  }
  const int64_t mid = lo + (hi - lo) / 2;
  cmp_acc x = cmp_pairwise(g, o, lo, mid), y = cmp_pairwise(g, o, mid, hi);
  a.mx = x.mx > y.mx ? x.mx : y.mx;
  a.d2 = x.d2 + y.d2;
  a.o2 = x.o2 + y.o2;
  a.g2 = x.g2 + y.g2;
  a.ipr = x.ipr + y.ipr;
  a.ipi = x.ipi + y.ipi;
  return a;
}

void orc_compare(const float* g, const double* o, int64_t count, double* out) {
  int64_t parts = 1;
  while (parts < 256 && parts * 4096 <= count) parts *= 2;
  cmp_acc* part = (cmp_acc*)malloc(sizeof(cmp_acc) * parts);
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < parts; ++p)
    part[p] = cmp_pairwise(g, o, p * (count / parts), p == parts - 1 ? count : (p + 1) * (count / parts));
  for (int64_t w = 1; w < parts; w *= 2)
    for (int64_t p = 0; p + w < parts; p += 2 * w) {
      cmp_acc* x = &part[p];
      const cmp_acc* y = &part[p + w];
      x->mx = x->mx > y->mx ? x->mx : y->mx;
      x->d2 += y->d2;
      x->o2 += y->o2;
      x->g2 += y->g2;
      x->ipr += y->ipr;
      x->ipi += y->ipi;
    }
  out[0] = part[0].mx;
  out[1] = part[0].d2;
  out[2] = part[0].o2;
  out[3] = part[0].g2;
  out[4] = part[0].ipr;
  out[5] = part[0].ipi;
  free(part);
}
