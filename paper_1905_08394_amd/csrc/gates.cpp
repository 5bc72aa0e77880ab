// Gate matrices used by the builder (supplement S-I gate set).
// H = (1/sqrt2)[[1,1],[1,-1]], T = diag(1, e^{i pi/4}),
// sqrt(X) = 1/2 [[1+i, 1-i], [1-i, 1+i]], sqrt(Y) = 1/2 [[1+i, -1-i], [1+i, 1+i]]
// (principal square roots), CZ = diag(1, 1, 1, -1).
#include <cmath>

#include "psim_internal.hpp"

namespace psim {

bool is_two_qubit(int kind) { return kind == PSIM_CZ || kind == PSIM_U2; }

void gate_matrix_1q(int kind, const double* m, cd out[4]) {
  const double s = 1.0 / std::sqrt(2.0);
  switch (kind) {
    case PSIM_H:
      out[0] = s; out[1] = s; out[2] = s; out[3] = -s;
      return;
    case PSIM_T:
      out[0] = 1.0; out[1] = 0.0; out[2] = 0.0; out[3] = cd(s, s);
      return;
    case PSIM_SQRT_X:
      out[0] = cd(0.5, 0.5); out[1] = cd(0.5, -0.5); out[2] = cd(0.5, -0.5); out[3] = cd(0.5, 0.5);
      return;
    case PSIM_SQRT_Y:
      out[0] = cd(0.5, 0.5); out[1] = cd(-0.5, -0.5); out[2] = cd(0.5, 0.5); out[3] = cd(0.5, 0.5);
      return;
    case PSIM_U1:
      if (!m) fail(PSIM_EINVAL, "U1 gate without a matrix");
      for (int i = 0; i < 4; ++i) out[i] = cd(m[2 * i], m[2 * i + 1]);
      return;
    default:
      fail(PSIM_EINVAL, "not a one-qubit gate kind: " + std::to_string(kind));
  }
}

void gate_matrix_2q(int kind, const double* m, cd out[16]) {
  if (kind == PSIM_CZ) {
    for (int i = 0; i < 16; ++i) out[i] = 0.0;
    out[0] = 1; out[5] = 1; out[10] = 1; out[15] = -1;
    return;
  }
  if (kind == PSIM_U2) {
    if (!m) fail(PSIM_EINVAL, "U2 gate without a matrix");
    for (int i = 0; i < 16; ++i) out[i] = cd(m[2 * i], m[2 * i + 1]);
    return;
  }
  fail(PSIM_EINVAL, "not a two-qubit gate kind: " + std::to_string(kind));
}

}  // namespace psim
