/* A plain C client of libpsim on the GPU, without PyTorch: device workspace
 * from hipMalloc, all 512 amplitudes of a 3x3 random-style circuit (H layer,
 * CZ on every edge, T on every qubit, H layer) in FP64 and FP32 3M, checked
 * for normalisation (sum |a|^2 = 1) and against each other; the plan's
 * reported sizes and the per-amplitude error estimates (NaN for FP64, finite
 * and of the size of the FP32 error for FP32 3M). */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "psim.h"

static int run(psim_peps_t *peps, int32_t prec, const uint8_t *bits, size_t nb, double *amp, double *err) {
  psim_plan_opts o;
  memset(&o, 0, sizeof o);
  o.prec = prec;
  o.max_batch = (int32_t)nb;
  psim_plan_t *plan = NULL;
  if (psim_plan(peps, &o, &plan) != PSIM_OK) {
    fprintf(stderr, "psim_plan: %s\n", psim_last_error());
    return 1;
  }
  psim_plan_stats s;
  psim_plan_info(plan, &s);
  if (s.peak_bytes != s.workspace_bytes + s.weights_bytes || s.n_tasks < (int64_t)s.R * (s.L + 1)) {
    fprintf(stderr, "plan stats: peak %llu, tasks %lld\n", (unsigned long long)s.peak_bytes, (long long)s.n_tasks);
    psim_plan_free(plan);
    return 1;
  }
  void *ws = NULL;
  if (hipMalloc(&ws, s.workspace_bytes) != hipSuccess) {
    fprintf(stderr, "hipMalloc failed\n");
    psim_plan_free(plan);
    return 1;
  }
  hipStream_t st;
  hipStreamCreate(&st);
  const psim_status r = psim_amplitudes(plan, bits, nb, ws, s.workspace_bytes, st, amp, err);
  if (r != PSIM_OK) fprintf(stderr, "psim_amplitudes: %s\n", psim_last_error());
  hipStreamDestroy(st);
  hipFree(ws);
  psim_plan_free(plan);
  return r == PSIM_OK ? 0 : 1;
}

int main(void) {
  psim_gate g[64];
  size_t n = 0;
  for (int q = 0; q < 9; ++q) g[n++] = (psim_gate){PSIM_H, 0, q, -1, NULL};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      const int q = r * 3 + c;
      if (c + 1 < 3) g[n++] = (psim_gate){PSIM_CZ, 1, q, q + 1, NULL};
      if (r + 1 < 3) g[n++] = (psim_gate){PSIM_CZ, 1, q, q + 3, NULL};
    }
  for (int q = 0; q < 9; ++q) g[n++] = (psim_gate){PSIM_T, 2, q, -1, NULL};
  for (int q = 0; q < 9; ++q) g[n++] = (psim_gate){PSIM_H, 3, q, -1, NULL};
  psim_peps_t *peps = NULL;
  if (psim_build(3, 3, g, n, &peps) != PSIM_OK) {
    fprintf(stderr, "psim_build: %s\n", psim_last_error());
    return 1;
  }
  const size_t nb = 512;
  uint8_t *bits = malloc(nb * 9);
  for (size_t b = 0; b < nb; ++b)
    for (int q = 0; q < 9; ++q) bits[b * 9 + q] = (uint8_t)((b >> (8 - q)) & 1);
  double *a64 = malloc(2 * nb * sizeof(double)), *a32 = malloc(2 * nb * sizeof(double));
  double *e64 = malloc(nb * sizeof(double)), *e32 = malloc(nb * sizeof(double));
  int bad = run(peps, PSIM_FP64, bits, nb, a64, e64) || run(peps, PSIM_FP32_3M, bits, nb, a32, e32);
  /* error estimates: NaN without a companion (FP64); finite, non-negative and
     below 1e-3 for FP32 3M on amplitudes that are not tiny */
  for (size_t b = 0; !bad && b < nb; ++b) {
    const double mag = hypot(a64[2 * b], a64[2 * b + 1]);
    if (!isnan(e64[b]) || !(e32[b] >= 0) || (mag > 1e-3 && e32[b] > 1e-3)) {
      fprintf(stderr, "error estimate %zu: fp64 %g fp32 %g (|a| %g)\n", b, e64[b], e32[b], mag);
      bad = 1;
    }
  }
  double n64 = 0, n32 = 0, diff = 0;
  for (size_t b = 0; !bad && b < nb; ++b) {
    n64 += a64[2 * b] * a64[2 * b] + a64[2 * b + 1] * a64[2 * b + 1];
    n32 += a32[2 * b] * a32[2 * b] + a32[2 * b + 1] * a32[2 * b + 1];
    diff = fmax(diff, hypot(a64[2 * b] - a32[2 * b], a64[2 * b + 1] - a32[2 * b + 1]));
  }
  if (!bad && (fabs(n64 - 1) > 1e-12 || fabs(n32 - 1) > 1e-5 || diff * sqrt((double)nb) > 1e-5)) {
    fprintf(stderr, "norms %.15f %.15f, max difference %.3e\n", n64, n32, diff);
    bad = 1;
  }
  if (!bad) printf("c gpu client ok: sum |a|^2 FP64 %.15f, FP32 3M %.9f, max |a64 - a32| %.2e\n", n64, n32, diff);
  free(bits);
  free(a64);
  free(a32);
  free(e64);
  free(e32);
  psim_peps_free(peps);
  return bad;
}
