// PEPS evolution on the host in FP64 (main text, "Quantum Circuit Simulator
// Based on PEPS"): one-qubit gates act on the physical index (eq. 3); a
// two-qubit gate O = sum_s U_s (x) V_s (eq. 4) puts U_s on the left/upper
// site and V_s on the right/lower site, bundling s with the shared bond
// (eqs. 5-6) as new = old * chi_o + s on both sides.
//
// CZ uses its exact rank-2 split CZ = sum_s |s><s| (x) Z^s: the left/upper
// site keeps the entries with sigma = s, the right/lower one flips the sign
// of the entries with sigma = s = 1.  Only copies and sign changes, so the
// tensors stay exact.  General U2 gates are split with a one-sided Jacobi SVD
// of the 4x4 operator reshaped as (tau_n sigma_n) x (tau_m sigma_m), with
// sqrt(S) given to each factor.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "psim_internal.hpp"

namespace psim {

namespace {

enum Leg { LEG_L = 0, LEG_R = 1, LEG_U = 2, LEG_D = 3 };

void apply_1q(Site& a, const cd U[4]) {
  const size_t half = a.size() / 2;
  for (size_t x = 0; x < half; ++x) {
    const cd a0 = a.t[x], a1 = a.t[half + x];
    a.t[x] = U[0] * a0 + U[1] * a1;
    a.t[half + x] = U[2] * a0 + U[3] * a1;
  }
}

Site widen(const Site& a, Leg leg, int k) {
  Site b = a;
  switch (leg) {
    case LEG_L: b.dl *= k; break;
    case LEG_R: b.dr *= k; break;
    case LEG_U: b.du *= k; break;
    case LEG_D: b.dd *= k; break;
  }
  b.t.assign((size_t)2 * b.dl * b.dr * b.du * b.dd, cd(0.0));
  return b;
}

// new flat index of (tau, l, r, u, d) with the widened leg's index old*k + s
inline size_t widened_at(const Site& b, Leg leg, int k, int tau, int l, int r, int u, int d, int s) {
  switch (leg) {
    case LEG_L: l = l * k + s; break;
    case LEG_R: r = r * k + s; break;
    case LEG_U: u = u * k + s; break;
    case LEG_D: d = d * k + s; break;
  }
  return b.at(tau, l, r, u, d);
}

// A'[tau; .., (old, s), ..] = sum_sigma F[tau][sigma][s] A[sigma; .., old, ..]
Site absorb_factor(const Site& a, Leg leg, int k, const std::vector<cd>& F) {
  Site b = widen(a, leg, k);
  for (int tau = 0; tau < 2; ++tau)
    for (int sg = 0; sg < 2; ++sg)
      for (int l = 0; l < a.dl; ++l)
        for (int r = 0; r < a.dr; ++r)
          for (int u = 0; u < a.du; ++u)
            for (int d = 0; d < a.dd; ++d) {
              const cd v = a.t[a.at(sg, l, r, u, d)];
              if (v == cd(0.0)) continue;
              for (int s = 0; s < k; ++s) {
                const cd f = F[((size_t)tau * 2 + sg) * k + s];
                if (f != cd(0.0)) b.t[widened_at(b, leg, k, tau, l, r, u, d, s)] += f * v;
              }
            }
  return b;
}

// CZ, left/upper factor |s><s|: entry kept where sigma = tau = s.
Site cz_left(const Site& a, Leg leg) {
  Site b = widen(a, leg, 2);
  for (int tau = 0; tau < 2; ++tau)
    for (int l = 0; l < a.dl; ++l)
      for (int r = 0; r < a.dr; ++r)
        for (int u = 0; u < a.du; ++u)
          for (int d = 0; d < a.dd; ++d)
            b.t[widened_at(b, leg, 2, tau, l, r, u, d, tau)] = a.t[a.at(tau, l, r, u, d)];
  return b;
}

// CZ, right/lower factor Z^s: entry copied for s = 0, sign (-1)^tau for s = 1.
Site cz_right(const Site& a, Leg leg) {
  Site b = widen(a, leg, 2);
  for (int tau = 0; tau < 2; ++tau)
    for (int l = 0; l < a.dl; ++l)
      for (int r = 0; r < a.dr; ++r)
        for (int u = 0; u < a.du; ++u)
          for (int d = 0; d < a.dd; ++d) {
            const cd v = a.t[a.at(tau, l, r, u, d)];
            b.t[widened_at(b, leg, 2, tau, l, r, u, d, 0)] = v;
            b.t[widened_at(b, leg, 2, tau, l, r, u, d, 1)] = tau ? -v : v;
          }
  return b;
}

}  // namespace

// One-sided (Hestenes) Jacobi SVD of a complex 4x4 matrix: M = U diag(S) V^H,
// singular values in decreasing order.
void jacobi_svd4(const cd M[16], cd U[16], double S[4], cd V[16]) {
  cd W[16], Vm[16];
  for (int i = 0; i < 16; ++i) { W[i] = M[i]; Vm[i] = (i % 5 == 0) ? 1.0 : 0.0; }
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < 3; ++p)
      for (int q = p + 1; q < 4; ++q) {
        double alpha = 0, beta = 0;
        cd gamma = 0;
        for (int i = 0; i < 4; ++i) {
          alpha += std::norm(W[i * 4 + p]);
          beta += std::norm(W[i * 4 + q]);
          gamma += std::conj(W[i * 4 + p]) * W[i * 4 + q];
        }
        const double g = std::abs(gamma);
        if (g == 0.0 || g <= 1e-300 + 1e-17 * std::sqrt(alpha * beta)) continue;
        off = std::max(off, g / std::sqrt(alpha * beta));
        const cd ph = std::conj(gamma) / g;  // multiply column q by e^{-i phi}
        const double zeta = (beta - alpha) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::abs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int i = 0; i < 4; ++i) {
          const cd wp = W[i * 4 + p], wq = W[i * 4 + q] * ph;
          W[i * 4 + p] = c * wp - s * wq;
          W[i * 4 + q] = s * wp + c * wq;
          const cd vp = Vm[i * 4 + p], vq = Vm[i * 4 + q] * ph;
          Vm[i * 4 + p] = c * vp - s * vq;
          Vm[i * 4 + q] = s * vp + c * vq;
        }
      }
    if (off < 1e-16) break;
  }
  double nrm[4];
  for (int j = 0; j < 4; ++j) {
    double a = 0;
    for (int i = 0; i < 4; ++i) a += std::norm(W[i * 4 + j]);
    nrm[j] = std::sqrt(a);
  }
  int ord[4] = {0, 1, 2, 3};
  std::sort(ord, ord + 4, [&](int x, int y) { return nrm[x] > nrm[y]; });
  for (int jj = 0; jj < 4; ++jj) {
    const int j = ord[jj];
    S[jj] = nrm[j];
    for (int i = 0; i < 4; ++i) {
      U[i * 4 + jj] = nrm[j] > 0 ? W[i * 4 + j] / nrm[j] : cd(0.0);
      V[i * 4 + jj] = Vm[i * 4 + j];
    }
  }
}

namespace {

void apply_2q(psim_peps_t& P, int kind, const double* m, int q0, int q1) {
  const int r0 = q0 / P.lh, c0 = q0 % P.lh, r1 = q1 / P.lh, c1 = q1 % P.lh;
  cd O[16];
  gate_matrix_2q(kind, m, O);
  int n, mm;
  bool horizontal;
  cd Op[16];
  if ((r0 == r1 && c1 == c0 + 1) || (c0 == c1 && r1 == r0 + 1)) {
    n = q0; mm = q1; horizontal = (r0 == r1);
    std::copy(O, O + 16, Op);
  } else if ((r0 == r1 && c0 == c1 + 1) || (c0 == c1 && r0 == r1 + 1)) {
    // left/upper qubit first: swap the qubits of rows and columns
    n = q1; mm = q0; horizontal = (r0 == r1);
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int c = 0; c < 2; ++c)
          for (int d = 0; d < 2; ++d) Op[(2 * b + a) * 4 + (2 * d + c)] = O[(2 * a + b) * 4 + (2 * c + d)];
  } else {
    fail(PSIM_EINVAL, "two-qubit gate on qubits " + std::to_string(q0) + ", " + std::to_string(q1) +
                          " that are not lattice neighbours");
  }
  const Leg ln = horizontal ? LEG_R : LEG_D, lm = horizontal ? LEG_L : LEG_U;
  if (kind == PSIM_CZ) {
    P.sites[n] = cz_left(P.sites[n], ln);
    P.sites[mm] = cz_right(P.sites[mm], lm);
    return;
  }
  // eq. (4): M[(tn sn), (tm sm)] = O[(tn tm), (sn sm)]
  cd M[16], U[16], V[16];
  double S[4];
  for (int tn = 0; tn < 2; ++tn)
    for (int sn = 0; sn < 2; ++sn)
      for (int tm = 0; tm < 2; ++tm)
        for (int sm = 0; sm < 2; ++sm) M[(2 * tn + sn) * 4 + (2 * tm + sm)] = Op[(2 * tn + tm) * 4 + (2 * sn + sm)];
  jacobi_svd4(M, U, S, V);
  int k = 0;
  while (k < 4 && S[k] > 1e-12 * S[0]) ++k;
  if (k == 0) fail(PSIM_EINVAL, "two-qubit gate matrix is zero");
  std::vector<cd> Fl((size_t)4 * k), Fr((size_t)4 * k);
  for (int s = 0; s < k; ++s) {
    const double rt = std::sqrt(S[s]);
    for (int t = 0; t < 2; ++t)
      for (int sg = 0; sg < 2; ++sg) {
        Fl[((size_t)t * 2 + sg) * k + s] = U[(2 * t + sg) * 4 + s] * rt;
        Fr[((size_t)t * 2 + sg) * k + s] = std::conj(V[(2 * t + sg) * 4 + s]) * rt;
      }
  }
  P.sites[n] = absorb_factor(P.sites[n], ln, k, Fl);
  P.sites[mm] = absorb_factor(P.sites[mm], lm, k, Fr);
}

}  // namespace

}  // namespace psim

using namespace psim;

// Gates in array order on an existing PEPS (eqs. 3-6).
static void apply_gates(psim_peps_t& P, const psim_gate* gates, size_t n_gates) {
  if (n_gates && !gates) fail(PSIM_EINVAL, "gates is NULL");
  const int n = P.lv * P.lh;
  int last_cycle = INT32_MIN;
  for (size_t g = 0; g < n_gates; ++g) {
    const psim_gate& G = gates[g];
    if (G.cycle < last_cycle) fail(PSIM_EINVAL, "gate cycles must be non-decreasing");
    last_cycle = G.cycle;
    if (G.q0 < 0 || G.q0 >= n) fail(PSIM_EINVAL, "gate " + std::to_string(g) + ": qubit out of range");
    if (is_two_qubit(G.kind)) {
      if (G.q1 < 0 || G.q1 >= n || G.q1 == G.q0)
        fail(PSIM_EINVAL, "gate " + std::to_string(g) + ": bad second qubit");
      apply_2q(P, G.kind, G.m, G.q0, G.q1);
    } else {
      cd U[4];
      gate_matrix_1q(G.kind, G.m, U);
      apply_1q(P.sites[G.q0], U);
    }
  }
}

psim_peps_t* build_peps(int32_t lv, int32_t lh, const psim_gate* gates, size_t n_gates) {
  if (lv < 1 || lh < 1 || (int64_t)lv * lh > 4096) fail(PSIM_EINVAL, "lattice size out of range");
  if (n_gates && !gates) fail(PSIM_EINVAL, "gates is NULL");
  const int n = lv * lh;
  auto* P = new psim_peps_t();
  P->lv = lv;
  P->lh = lh;
  P->sites.resize(n);
  for (auto& s : P->sites) {
    s.t.assign(2, cd(0.0));
    s.t[0] = 1.0;  // |0>
  }
  try {
    apply_gates(*P, gates, n_gates);
  } catch (...) {
    delete P;
    throw;
  }
  return P;
}

// More gates on an existing state (the remark after eq. 7: gates may follow
// a measurement); applied to a copy, so a failing gate leaves P unchanged.
void apply_more_gates(psim_peps_t& P, const psim_gate* gates, size_t n_gates) {
  psim_peps_t tmp = P;
  apply_gates(tmp, gates, n_gates);
  P = std::move(tmp);
}

// Measurement outcome |value> on one qubit: the physical slice sigma != value
// of its site tensor is set to zero (unnormalised: the new squared norm is
// the outcome's probability times the old one).
void project_qubit(psim_peps_t& P, int32_t qubit, int32_t value) {
  if (qubit < 0 || qubit >= P.lv * P.lh) fail(PSIM_EINVAL, "qubit out of range");
  if (value != 0 && value != 1) fail(PSIM_EINVAL, "value must be 0 or 1");
  Site& s = P.sites[(size_t)qubit];
  const size_t half = s.t.size() / 2;  // sigma is the slowest index
  std::fill(s.t.begin() + (value ? 0 : half), s.t.begin() + (value ? half : 2 * half), cd(0.0));
}
