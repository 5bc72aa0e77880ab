// C ABI of libpsim: status codes, thread-local error messages, handles.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "psim_internal.hpp"

psim_peps_t* build_peps(int32_t lv, int32_t lh, const psim_gate* gates, size_t n_gates);
void apply_more_gates(psim_peps_t& P, const psim_gate* gates, size_t n_gates);
void project_qubit(psim_peps_t& P, int32_t qubit, int32_t value);
psim_plan_t* make_plan(const psim_peps_t* P, const psim_plan_opts* o);
void free_plan(psim_plan_t* pl);
void tune_plan(psim_plan_t* pl, void* ws, size_t ws_bytes, void* stream, int reps, double* best_ms);
psim_group_s* make_group(psim_plan_t* const* plans, int np);
void free_group(psim_group_s* G);
void run_group(psim_group_s* G, const uint8_t* const* bits, const size_t* n, void* const* ws, const size_t* ws_bytes,
               void* stream, double* const* out);

namespace psim {

static thread_local std::string g_last_error = "no error";

void set_last_error(const std::string& msg) { g_last_error = msg; }

[[noreturn]] void fail(psim_status st, const std::string& msg) { throw Error{st, msg}; }

}  // namespace psim

using namespace psim;

template <typename F>
static psim_status guarded(F&& f) {
  try {
    f();
    return PSIM_OK;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return PSIM_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(std::string("internal error: ") + e.what());
    return PSIM_EINTERNAL;
  } catch (...) {
    set_last_error("internal error");
    return PSIM_EINTERNAL;
  }
}

extern "C" {

psim_status psim_build(int32_t lv, int32_t lh, const psim_gate* gates, size_t n_gates, psim_peps_t** out) {
  return guarded([&] {
    if (!out) fail(PSIM_EINVAL, "out is NULL");
    *out = build_peps(lv, lh, gates, n_gates);
  });
}

psim_status psim_peps_info(const psim_peps_t* P, int32_t* lv, int32_t* lh, int32_t* chi, int64_t* bond_dims,
                           size_t n_bonds) {
  return guarded([&] {
    if (!P) fail(PSIM_EINVAL, "peps is NULL");
    const size_t nb = (size_t)P->lv * (P->lh - 1) + (size_t)(P->lv - 1) * P->lh;
    if (bond_dims && n_bonds < nb) fail(PSIM_EINVAL, "bond_dims needs " + std::to_string(nb) + " entries");
    int c = 1;
    for (const Site& s : P->sites) c = std::max({c, s.dl, s.dr, s.du, s.dd});
    if (lv) *lv = P->lv;
    if (lh) *lh = P->lh;
    if (chi) *chi = c;
    if (bond_dims) {
      size_t x = 0;
      for (int r = 0; r < P->lv; ++r)
        for (int col = 0; col + 1 < P->lh; ++col) bond_dims[x++] = P->sites[r * P->lh + col].dr;
      for (int r = 0; r + 1 < P->lv; ++r)
        for (int col = 0; col < P->lh; ++col) bond_dims[x++] = P->sites[r * P->lh + col].dd;
    }
  });
}

void psim_peps_free(psim_peps_t* P) { delete P; }

psim_status psim_apply(psim_peps_t* P, const psim_gate* gates, size_t n_gates) {
  return guarded([&] {
    if (!P) fail(PSIM_EINVAL, "peps is NULL");
    apply_more_gates(*P, gates, n_gates);
  });
}

psim_status psim_project(psim_peps_t* P, int32_t qubit, int32_t value) {
  return guarded([&] {
    if (!P) fail(PSIM_EINVAL, "peps is NULL");
    project_qubit(*P, qubit, value);
  });
}

psim_status psim_double_layer(const psim_peps_t* P, const double* ops, psim_peps_t** out) {
  return guarded([&] {
    if (!P || !out) fail(PSIM_EINVAL, "peps or out is NULL");
    *out = double_layer(*P, ops);
  });
}

psim_status psim_sample_workspace(const psim_peps_t* P, const psim_plan_opts* opts, uint64_t* bytes) {
  return guarded([&] {
    if (!P || !opts || !bytes) fail(PSIM_EINVAL, "peps, opts or bytes is NULL");
    *bytes = sample_workspace(*P, *opts);
  });
}

psim_status psim_sample(const psim_peps_t* P, const psim_plan_opts* opts, const double* u, size_t n_samples,
                        void* d_workspace, size_t workspace_bytes, void* hip_stream, uint8_t* bits,
                        double* out_prob) {
  return guarded([&] {
    if (!P || !opts) fail(PSIM_EINVAL, "peps or opts is NULL");
    if (opts->flags & PSIM_PLAN_HOST_ONLY) fail(PSIM_EINVAL, "sampling needs a device plan");
    sample(*P, *opts, u, n_samples, d_workspace, workspace_bytes, hip_stream, bits, out_prob);
  });
}

psim_status psim_plan(const psim_peps_t* P, const psim_plan_opts* opts, psim_plan_t** out) {
  return guarded([&] {
    if (!out) fail(PSIM_EINVAL, "out is NULL");
    *out = make_plan(P, opts);
  });
}

psim_status psim_plan_info(const psim_plan_t* pl, psim_plan_stats* s) {
  return guarded([&] {
    if (!pl || !s) fail(PSIM_EINVAL, "NULL argument");
    psim_plan_stats o{};
    o.workspace_bytes = pl->ws_total;
    o.weights_bytes = pl->weights_bytes;
    o.peak_tensor_elems = (uint64_t)pl->peak_elems;
    o.cmac_per_amplitude = pl->cmac;
    o.n_gemm_steps = pl->sq ? pl->sq_steps : (int64_t)pl->steps.size();
    o.peak_bytes = pl->ws_total + pl->weights_bytes;
    o.w_chunk = 0;
    for (const auto& lev : pl->levels)
      if (w_cut(lev)) o.w_chunk = o.w_chunk ? std::min(o.w_chunk, lev.wchunk) : lev.wchunk;
    if (pl->sq) {
      o.n_tasks = pl->sq_steps;
    } else {
      o.n_tasks = 0;
      for (const auto& lev : pl->levels)
        o.n_tasks += (pl->L == 1 ? 1 : (lev.Dv + lev.vchunk - 1) / lev.vchunk) * (w_cut(lev) ? lev.Dw / lev.wchunk : 1) *
                         pl->L + 1;
    }
    o.L = pl->L;
    o.R = pl->R;
    o.chi = pl->chi;
    int vc = 0;
    for (const auto& lev : pl->levels) vc = std::max(vc, lev.vchunk);
    o.v_chunk = vc;
    for (const auto& lev : pl->levels)
      if (lev.Dv > 1) o.v_chunk = std::min(o.v_chunk, lev.vchunk);
    o.sweep = pl->sweep;
    o.prec = pl->opts.prec;
    double worst = -1;
    for (const auto& st : pl->steps) {
      const double cm = (double)st.M * st.K1 * st.K2 * st.N * (st.kind == 2 ? 1 : pl->levels[st.i].Dv);
      if (cm > worst) { worst = cm; o.hot_cfg = st.kind == 1 ? st.cfg : 0; }
    }
    *s = o;
  });
}

void psim_plan_free(psim_plan_t* pl) { free_plan(pl); }

psim_status psim_amplitudes(psim_plan_t* pl, const uint8_t* bits, size_t n, void* ws, size_t ws_bytes,
                            void* stream, double* out, double* out_rel_err) {
  return guarded([&] {
    if (!pl) fail(PSIM_EINVAL, "plan is NULL");
    run_amplitudes(pl, bits, n, ws, ws_bytes, stream, out, false, out_rel_err);
  });
}

psim_status psim_contract_site(int32_t prec, int64_t batch, int64_t M, int64_t K1, int64_t K2, int64_t N,
                               const void* dA, int64_t a_batch_stride, const double* W, void* dC,
                               int32_t transpose_out, void* stream) {
  return guarded([&] {
    // optional bits above the precision: split accumulation and a tile candidate
    if (prec & ~(0xff | PSIM_CONTRACT_SPLIT_ACC | (0xff << PSIM_CONTRACT_TILE_SHIFT)))
      fail(PSIM_EINVAL, "unknown bits in the precision argument");
    const int split = (prec & PSIM_CONTRACT_SPLIT_ACC) ? 1 : 0;
    const int cfg = (prec >> PSIM_CONTRACT_TILE_SHIFT) & 0xff;
    prec &= 0xff;
    if (prec != PSIM_FP64 && prec != PSIM_FP32_4M && prec != PSIM_FP32_3M && prec != PSIM_BF16X3)
      fail(PSIM_EUNSUPPORTED, "precision not available");
    if (cfg >= config_count(prec) || (split && (prec == PSIM_FP64 || prec == PSIM_BF16X3 || !split_candidate(prec, cfg))))
      fail(PSIM_EINVAL, "tile candidate or split accumulation not available for this precision");
    if (batch < 1 || M < 1 || K1 < 1 || K2 < 1 || N < 1) fail(PSIM_EINVAL, "non-positive size");
    if (!dA || !W || !dC) fail(PSIM_EINVAL, "NULL buffer");
    const int eb = prec == PSIM_FP64 ? 16 : 8;
    if (((uintptr_t)dA | (uintptr_t)dC) % eb) fail(PSIM_EINVAL, "device buffers must be aligned to one complex");
    if (batch > 1 && a_batch_stride < K1 * M * K2) fail(PSIM_EINVAL, "a_batch_stride must be at least K1*M*K2");
    const int64_t K = K1 * K2;
    std::vector<cd> Wc((size_t)(K * N));
    for (int64_t x = 0; x < K * N; ++x) Wc[x] = cd(W[2 * x], W[2 * x + 1]);
    std::vector<char> packed, packed_b;
    int64_t ld = 0, ld_b = 0, plane_b = 0;
    pack_site_matrix(prec == PSIM_BF16X3 ? PSIM_FP32_4M : prec, Wc.data(), K, N, packed, ld);
    if (prec == PSIM_BF16X3) pack_site_matrix_bf16(Wc.data(), K, N, packed_b, ld_b, plane_b);
    void* dW = nullptr;
    void* dWb = nullptr;
    hip_check(hipMalloc(&dW, packed.size() + packed_b.size()), "hipMalloc(W)");
    try {
      hipStream_t st = (hipStream_t)stream;
      hip_check(hipMemcpyAsync(dW, packed.data(), packed.size(), hipMemcpyHostToDevice, st), "upload W");
      if (!packed_b.empty()) {
        dWb = (char*)dW + packed.size();
        hip_check(hipMemcpyAsync(dWb, packed_b.data(), packed_b.size(), hipMemcpyHostToDevice, st), "upload W");
      }
      GemmLaunch g;
      g.Wb0 = dWb;
      g.ldwb = ld_b;
      g.planeb = plane_b;
      g.prec = prec;
      g.A = dA;
      g.C = dC;
      g.W0 = dW;
      g.ldw = ld;
      g.M = M;
      g.K1 = K1;
      g.K2 = K2;
      g.N = N;
      g.nodes = batch;
      g.Bz = 1;
      g.sA_node = a_batch_stride;
      g.sC_node = M * N;
      g.trans_out = transpose_out ? 1 : 0;
      g.split = split;
      g.cfg = transpose_out ? 0 : cfg;
      launch_site_gemm(g, st);
      hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    } catch (...) {
      (void)hipFree(dW);
      throw;
    }
    hip_check(hipFree(dW), "hipFree(W)");
  });
}

psim_status psim_tune(psim_plan_t* pl, void* ws, size_t ws_bytes, void* stream, int32_t reps, double* best_ms) {
  return guarded([&] {
    if (!pl) fail(PSIM_EINVAL, "plan is NULL");
    tune_plan(pl, ws, ws_bytes, stream, reps, best_ms);
  });
}

psim_status psim_profile(psim_plan_t* pl, int32_t op, psim_kernel_stats* out) {
  return guarded([&] {
    if (!pl) fail(PSIM_EINVAL, "plan is NULL");
    if (op == 1) {
      pl->profile = true;
      for (auto& k : pl->prof) k = psim_kernel_stats{};
    } else if (op == 2) {
      if (!out) fail(PSIM_EINVAL, "out is NULL");
      for (int i = 0; i < 4; ++i) out[i] = pl->prof[i];
    } else if (op == 0) {
      pl->profile = false;
    } else {
      fail(PSIM_EINVAL, "op must be 0, 1 or 2");
    }
  });
}

psim_status psim_group(psim_plan_t* const* plans, int32_t n_plans, psim_group_t** out) {
  return guarded([&] {
    if (!out) fail(PSIM_EINVAL, "out is NULL");
    *out = make_group(plans, n_plans);
  });
}

psim_status psim_group_info(const psim_group_t* g, psim_group_stats* out) {
  return guarded([&] {
    if (!g || !out) fail(PSIM_EINVAL, "group or out is NULL");
    psim_group_stats o{};
    o.n_plans = (int32_t)g->plans.size();
    o.descriptor_bytes = g->desc_bytes;
    o.grouped_launches = g->grouped_launches;
    *out = o;
  });
}

psim_status psim_group_amplitudes(psim_group_t* g, const uint8_t* const* bits, const size_t* n_bitstrings,
                                  void* const* workspaces, const size_t* workspace_bytes, void* stream,
                                  double* const* out) {
  return guarded([&] {
    if (!g) fail(PSIM_EINVAL, "group is NULL");
    run_group(g, bits, n_bitstrings, workspaces, workspace_bytes, stream, out);
  });
}

void psim_group_free(psim_group_t* g) { free_group(g); }

const char* psim_last_error(void) { return g_last_error.c_str(); }

const char* psim_version(void) { return "psim 0.1 (gfx950)"; }

}  // extern "C"
