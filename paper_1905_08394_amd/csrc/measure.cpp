// Observables and measurements (main text: the simulator keeps the whole
// state, so besides single amplitudes it gives expectation values and
// sequences of measurements).
//
// Both rest on the double-layer network: the norm <psi|psi> of the PEPS is
// the contraction, bond by bond, of the bra layer (complex conjugate tensors)
// with the ket layer, with a one-qubit operator O_n between the two physical
// legs of site n:
//   E_n[(l l')][(r r')][(u u')][(d d')] = sum_{s, s'} conj(A_n[s][l][r][u][d]) O_n[s][s'] A_n[s'][l'][r'][u'][d']
// (the bra index first in every doubled leg).  Such a network is again a
// lattice of rank-4 tensors with the squared bond sizes, so it is handed to
// the amplitude machinery as a PEPS whose two "physical" slices at site n are
// E_n for two operators O_{n,0}, O_{n,1}: the "amplitude" of bitstring b is
// then <psi| prod_n O_{n,b_n} |psi>, contracted by the same plans, schemes,
// precisions and kernels as ordinary amplitudes.
//
// Sequential measurement in the computational basis (qubit 0 first): with
// the prefix t_0 .. t_{k-1} already drawn, qubit k takes 0 with probability
// p(t_0 .. t_{k-1}, 0) / (p(.., 0) + p(.., 1)), where p(prefix) is the
// double-layer value with projectors |t><t| on the measured sites and the
// identity elsewhere.  One double-layer PEPS per k serves every sample: sites
// n <= k carry the slices (|0><0|, |1><1|), sites n > k the slices (I, I).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include "psim_internal.hpp"

psim_plan_t* make_plan(const psim_peps_t* P, const psim_plan_opts* o);
void free_plan(psim_plan_t* pl);

namespace psim {

psim_peps_t* double_layer(const psim_peps_t& P, const double* ops) {
  if (!ops) fail(PSIM_EINVAL, "ops is NULL");
  const size_t n = P.sites.size();
  for (size_t x = 0; x < n * 2 * 8; ++x)
    if (!std::isfinite(ops[x])) fail(PSIM_EINVAL, "ops entry " + std::to_string(x) + " is not finite");
  auto* out = new psim_peps_t();
  out->lv = P.lv;
  out->lh = P.lh;
  out->sites.resize(n);
  for (size_t q = 0; q < n; ++q) {
    const Site& a = P.sites[q];
    Site& e = out->sites[q];
    e.dl = a.dl * a.dl;
    e.dr = a.dr * a.dr;
    e.du = a.du * a.du;
    e.dd = a.dd * a.dd;
    const size_t legs = (size_t)e.dl * e.dr * e.du * e.dd;
    if (legs > ((size_t)1 << 28)) {
      delete out;
      fail(PSIM_EUNSUPPORTED, "double-layer site tensor too large (" + std::to_string(legs) + " elements per slice)");
    }
    e.t.assign(2 * legs, cd(0.0));
    for (int s = 0; s < 2; ++s) {
      const double* m = ops + (q * 2 + s) * 8;
      for (int s1 = 0; s1 < 2; ++s1)
        for (int s2 = 0; s2 < 2; ++s2) {
          const cd o(m[2 * (s1 * 2 + s2)], m[2 * (s1 * 2 + s2) + 1]);
          if (o == cd(0.0)) continue;
          for (int l1 = 0; l1 < a.dl; ++l1)
            for (int r1 = 0; r1 < a.dr; ++r1)
              for (int u1 = 0; u1 < a.du; ++u1)
                for (int d1 = 0; d1 < a.dd; ++d1) {
                  const cd x = std::conj(a.t[a.at(s1, l1, r1, u1, d1)]) * o;
                  if (x == cd(0.0)) continue;
                  for (int l2 = 0; l2 < a.dl; ++l2)
                    for (int r2 = 0; r2 < a.dr; ++r2)
                      for (int u2 = 0; u2 < a.du; ++u2)
                        for (int d2 = 0; d2 < a.dd; ++d2)
                          e.t[e.at(s, l1 * a.dl + l2, r1 * a.dr + r2, u1 * a.du + u2, d1 * a.dd + d2)] +=
                              x * a.t[a.at(s2, l2, r2, u2, d2)];
                }
        }
    }
  }
  return out;
}

namespace {

// slices of site n for measurement step k: projectors on n <= k, identity above
std::vector<double> step_ops(size_t n_sites, size_t k) {
  std::vector<double> ops(n_sites * 16, 0.0);
  for (size_t q = 0; q < n_sites; ++q) {
    double* m0 = ops.data() + q * 16;
    double* m1 = m0 + 8;
    if (q <= k) {
      m0[0] = 1.0;  // |0><0|
      m1[6] = 1.0;  // |1><1|
    } else {
      m0[0] = m0[6] = 1.0;  // I
      m1[0] = m1[6] = 1.0;
    }
  }
  return ops;
}

}  // namespace

uint64_t sample_workspace(const psim_peps_t& P, const psim_plan_opts& o) {
  std::unique_ptr<psim_peps_t> V(double_layer(P, step_ops(P.sites.size(), 0).data()));
  psim_plan_opts h = o;
  h.flags |= PSIM_PLAN_HOST_ONLY;
  psim_plan_t* pl = make_plan(V.get(), &h);
  const uint64_t b = pl->ws_total;
  free_plan(pl);
  return b;
}

void sample(const psim_peps_t& P, const psim_plan_opts& o, const double* u, size_t n_samples, void* ws,
            size_t ws_bytes, void* stream, uint8_t* bits, double* prob) {
  if (!u || !bits) fail(PSIM_EINVAL, "u or bits is NULL");
  const size_t N = P.sites.size();
  for (size_t x = 0; x < n_samples * N; ++x)
    if (!(u[x] >= 0.0 && u[x] < 1.0)) fail(PSIM_EINVAL, "u[" + std::to_string(x) + "] is not in [0, 1)");
  if (n_samples == 0) return;
  std::vector<uint8_t> cur(n_samples * N, 0), q(2 * n_samples * N);
  std::vector<double> p(n_samples, 1.0), amp(4 * n_samples);
  for (size_t k = 0; k < N; ++k) {
    std::unique_ptr<psim_peps_t> V(double_layer(P, step_ops(N, k).data()));
    psim_plan_t* pl = make_plan(V.get(), &o);
    try {
      for (size_t s = 0; s < n_samples; ++s)
        for (int b = 0; b < 2; ++b) {
          uint8_t* r = q.data() + (2 * s + b) * N;
          std::memcpy(r, cur.data() + s * N, N);
          r[k] = (uint8_t)b;
        }
      run_amplitudes(pl, q.data(), 2 * n_samples, ws, ws_bytes, stream, amp.data());
    } catch (...) {
      free_plan(pl);
      throw;
    }
    free_plan(pl);
    for (size_t s = 0; s < n_samples; ++s) {
      // the values are real and non-negative up to rounding
      const double p0 = std::max(amp[4 * s], 0.0), p1 = std::max(amp[4 * s + 2], 0.0);
      const double t = p0 + p1 > 0 ? p0 / (p0 + p1) : 0.5;
      const uint8_t b = u[s * N + k] < t ? 0 : 1;
      cur[s * N + k] = b;
      p[s] = b ? p1 : p0;
    }
  }
  std::memcpy(bits, cur.data(), n_samples * N);
  if (prob) std::memcpy(prob, p.data(), n_samples * sizeof(double));
}

}  // namespace psim
