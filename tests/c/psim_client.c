/* A plain C client of libpsim: builds the PEPS of a 3x3 circuit (an H layer,
 * CZ on every horizontal and vertical edge, an H layer), plans its row
 * contraction on the host only, and checks the plan's sizes and the error
 * paths through the C ABI alone (no device needed). */
#include <stdio.h>
#include <string.h>

#include "psim.h"

static int fail_count = 0;
#define CHECK(cond, ...)                  \
  do {                                    \
    if (!(cond)) {                        \
      fprintf(stderr, __VA_ARGS__);       \
      fprintf(stderr, "\n");              \
      ++fail_count;                       \
    }                                     \
  } while (0)

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
  for (int q = 0; q < 9; ++q) g[n++] = (psim_gate){PSIM_H, 2, q, -1, NULL};

  psim_peps_t *peps = NULL;
  psim_status st = psim_build(3, 3, g, n, &peps);
  CHECK(st == PSIM_OK && peps, "psim_build: %d %s", (int)st, psim_last_error());

  int32_t lv = 0, lh = 0, chi = 0;
  int64_t bonds[12];
  st = psim_peps_info(peps, &lv, &lh, &chi, bonds, 12);
  CHECK(st == PSIM_OK && lv == 3 && lh == 3 && chi == 2, "psim_peps_info: %d lv %d lh %d chi %d", (int)st, lv,
        lh, chi);
  for (int b = 0; b < 12; ++b) CHECK(bonds[b] == 2, "bond %d has size %lld", b, (long long)bonds[b]);

  psim_plan_opts o;
  memset(&o, 0, sizeof o);
  o.prec = PSIM_FP32_3M;
  o.flags = PSIM_PLAN_HOST_ONLY;
  o.max_batch = 4;
  psim_plan_t *plan = NULL;
  st = psim_plan(peps, &o, &plan);
  CHECK(st == PSIM_OK && plan, "psim_plan: %d %s", (int)st, psim_last_error());
  psim_plan_stats s;
  st = psim_plan_info(plan, &s);
  CHECK(st == PSIM_OK && s.L == 3 && s.R == 3 && s.chi == 2 && s.cmac_per_amplitude > 0 && s.n_gemm_steps == 9,
        "psim_plan_info: %d L %d R %d chi %d steps %lld", (int)st, s.L, s.R, s.chi, (long long)s.n_gemm_steps);
  /* peak device bytes = workspace + packed site matrices; tasks: per row, v chunks x sites + a rescale */
  CHECK(s.peak_bytes == s.workspace_bytes + s.weights_bytes && s.peak_bytes > 0, "peak_bytes %llu",
        (unsigned long long)s.peak_bytes);
  CHECK(s.n_tasks >= (int64_t)s.R * (s.L + 1), "n_tasks %lld", (long long)s.n_tasks);

  /* a host-only plan cannot run; nothing is written */
  uint8_t bits[9] = {0};
  double out[2] = {-7.0, -7.0};
  double err[1] = {-7.0};
  st = psim_amplitudes(plan, bits, 1, NULL, 0, NULL, out, err);
  CHECK(st == PSIM_EINVAL && out[0] == -7.0 && err[0] == -7.0, "host-only psim_amplitudes: %d", (int)st);

  /* a CZ between non-neighbours is rejected with a message */
  psim_gate bad = {PSIM_CZ, 0, 0, 4, NULL};
  psim_peps_t *p2 = NULL;
  st = psim_build(3, 3, &bad, 1, &p2);
  CHECK(st == PSIM_EINVAL && p2 == NULL && strstr(psim_last_error(), "neighbour"), "bad gate: %d %s", (int)st,
        psim_last_error());

  /* psim_contract_site: a tile or split choice the precision lacks, or a
     bit that names nothing, is refused before any device work */
  double w[32] = {0};
  int32_t bad_prec[3] = {PSIM_FP64 | PSIM_CONTRACT_SPLIT_ACC, PSIM_FP32_3M | (4 << PSIM_CONTRACT_TILE_SHIFT),
                         PSIM_FP32_4M | 0x200};
  for (int i = 0; i < 3; ++i) {
    st = psim_contract_site(bad_prec[i], 1, 8, 2, 2, 4, (const void *)w, 32, w, (void *)w, 0, NULL);
    CHECK(st == PSIM_EINVAL, "contract_site choice %d: %d", i, (int)st);
  }

  psim_plan_free(plan);
  psim_peps_free(peps);
  psim_plan_free(NULL);
  psim_peps_free(NULL);
  if (fail_count == 0) printf("c client ok (%s)\n", psim_version());
  return fail_count == 0 ? 0 : 1;
}
