// Amplitude scheduler: runs the planned row sweep for a batch of bitstrings.
//
// Bitstrings that agree on their first i+1 swept rows share the boundary F_i
// (the reuse idea of the "fast sampling" remark in S-II), so the batch is
// organised as a trie: level i holds one node per distinct prefix of rows
// 0..i, and each node's row is computed once from its parent's boundary.
// Nodes of a level are processed in groups and the v leg in chunks (both
// sized by the planner for the memory budget); every site contraction is
// one batched GEMM launch over (node, v).  After each row the boundary of
// every node is rescaled by an exact power of two chosen from its largest
// component, and the exponents are carried along the trie; the amplitude is
// mantissa * 2^(row exponents + site-matrix exponents), assembled in FP64.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <unordered_map>

#include <hip/hip_runtime_api.h>

#include "psim_internal.hpp"

using namespace psim;

namespace {

struct Trie {
  // per level: parent index of each node and the bits of its row
  std::vector<std::vector<int32_t>> parent;
  std::vector<std::vector<uint8_t>> tau;  // nodes x L
  std::vector<int32_t> leaf;              // per bitstring: node at the last level
};

Trie build_trie(const psim_plan_t& pl, const uint8_t* bits, size_t n) {
  const int R = pl.R, L = pl.L, nq = pl.lv * pl.lh;
  Trie t;
  t.parent.resize(R);
  t.tau.resize(R);
  std::vector<int32_t> cur(n, 0);  // node of each bitstring at the previous level (root = 0)
  for (int i = 0; i < R; ++i) {
    std::map<std::pair<int32_t, uint64_t>, int32_t> index;
    std::vector<int32_t> next(n);
    for (size_t b = 0; b < n; ++b) {
      uint64_t key = 0;
      for (int j = 0; j < L; ++j) key |= (uint64_t)bits[b * nq + pl.cs[(size_t)i * L + j].qubit] << j;
      auto k = std::make_pair(cur[b], key);
      auto it = index.find(k);
      if (it == index.end()) {
        const int32_t id = (int32_t)t.parent[i].size();
        index.emplace(k, id);
        t.parent[i].push_back(cur[b]);
        for (int j = 0; j < L; ++j) t.tau[i].push_back((uint8_t)((key >> j) & 1));
        next[b] = id;
      } else {
        next[b] = it->second;
      }
    }
    cur.swap(next);
  }
  t.leaf = cur;
  return t;
}

// Workspace layout: per-level trie tables, exponents, row maxima (the table
// region, pl.ws_tab bytes at the start), the two boundary buffers (even / odd
// rows) and the two intermediate buffers.  A grouped run may place the table
// region elsewhere (tab != NULL); the boundary and intermediate buffers stay
// where they are.
struct WsLayout {
  char* tab;
  std::vector<int32_t*> parent;
  std::vector<uint8_t*> tau;
  int32_t* exp[2];
  uint32_t* mx;
  char* F[2];
  char* G[2];
};

WsLayout layout(const psim_plan_t& pl, void* ws, char* tab = nullptr) {
  auto al = [](uint64_t x) { return (x + 255) / 256 * 256; };
  char* base = (char*)(((uintptr_t)ws + 255) / 256 * 256);
  char* p = tab ? tab : base;
  WsLayout w;
  w.tab = p;
  const int R = pl.R, L = pl.L;
  w.parent.resize(R);
  w.tau.resize(R);
  int64_t nmax_all = 1;
  for (int i = 0; i < R; ++i) {
    const Level& lev = pl.levels[i];
    w.parent[i] = (int32_t*)p;
    p += al((uint64_t)lev.nmax * 4);
    w.tau[i] = (uint8_t*)p;
    p += al((uint64_t)lev.nmax * L);
    nmax_all = std::max(nmax_all, lev.nmax);
  }
  w.exp[0] = (int32_t*)p; p += al((uint64_t)nmax_all * 4);
  w.exp[1] = (int32_t*)p; p += al((uint64_t)nmax_all * 4);
  w.mx = (uint32_t*)p; p += al((uint64_t)nmax_all * 4);
  p = base + pl.ws_tab;
  w.F[0] = p + pl.levels[0].F_off;
  w.F[1] = p + (R > 1 ? pl.levels[1].F_off : 0);
  p += pl.ws_F;
  w.G[0] = p;
  w.G[1] = p + pl.ws_G / 2;
  return w;
}

}  // namespace

void clear_graphs(psim_plan_t* pl) {
  for (auto& kv : pl->graphs) (void)hipGraphExecDestroy((hipGraphExec_t)kv.second);
  pl->graphs.clear();
}

void tune_plan(psim_plan_t* pl, void* ws, size_t ws_bytes, void* stream, int reps, double* best_ms) {
  if (pl->host_only) fail(PSIM_EINVAL, "plan was made with PSIM_PLAN_HOST_ONLY");
  if (!ws || ws_bytes < pl->ws_total) fail(PSIM_EINVAL, "workspace is NULL or smaller than the plan needs");
  if (reps < 1) fail(PSIM_EINVAL, "reps must be at least 1");
  if (best_ms) *best_ms = 0;
  if (pl->sq) return;
  const bool split = (pl->opts.flags & PSIM_PLAN_SPLIT_ACC) != 0;
  std::vector<int> cands;
  for (int cfg = 0; cfg < config_count(pl->opts.prec); ++cfg)
    if (!split || split_candidate(pl->opts.prec, cfg)) cands.push_back(cfg);
  if (cands.size() < 2) return;
  hip_check(hipSetDevice(pl->opts.device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  WsLayout W = layout(*pl, ws);
  const int L = pl->L;
  double worst_cmac = 0;
  // distinct shapes of the interior-site contractions
  std::map<std::vector<int64_t>, std::vector<size_t>> shapes;
  for (size_t x = 0; x < pl->steps.size(); ++x) {
    const Step& s = pl->steps[x];
    if (s.kind != 1 || s.K2 % 2) continue;
    const Level& lev = pl->levels[s.i];
    shapes[{interior_rows(lev, s), s.K1, s.K2, s.N, interior_batch(lev)}].push_back(x);
  }
  hipEvent_t a, b;
  hip_check(hipEventCreate(&a), "hipEventCreate");
  hip_check(hipEventCreate(&b), "hipEventCreate");
  bool changed = false;
  const std::string arch = device_arch(pl->opts.device);
  std::map<std::string, std::pair<int, double>> store;  // for PSIM_TUNE_CACHE
  for (auto& kv : shapes) {
    const Step& s = pl->steps[kv.second.front()];
    const Level& lev = pl->levels[s.i];
    const int64_t c = interior_batch(lev), Ms = interior_rows(lev, s);
    GemmLaunch g;
    g.prec = pl->opts.prec;
    g.A = W.G[0];
    g.C = W.G[1];
    const DevMatrix& dm = pl->w[((size_t)s.i * L + s.j) * 2];
    g.W0 = g.W1 = dm.ptr;
    g.ldw = dm.ld;
    if (dm.ptr_b) {  // BF16x3: the pre-split planes
      g.Wb0 = g.Wb1 = dm.ptr_b;
      g.ldwb = dm.ld_b;
      g.planeb = dm.plane_b;
    }
    g.M = Ms; g.K1 = s.K1; g.K2 = s.K2; g.N = s.N;
    g.nodes = 1; g.Bz = (int32_t)c;
    g.sA_v = s.K1 * Ms * s.K2; g.sA_node = c * g.sA_v;
    g.sC_v = Ms * s.N; g.sC_node = c * g.sC_v;
    int best = 0;
    double best_t = 1e300;
    g.split = split ? 1 : 0;
    for (int cfg : cands) {
      g.cfg = cfg;
      launch_site_gemm(g, st);  // warm
      hip_check(hipEventRecord(a, st), "hipEventRecord");
      for (int r = 0; r < reps; ++r) launch_site_gemm(g, st);
      hip_check(hipEventRecord(b, st), "hipEventRecord");
      hip_check(hipEventSynchronize(b), "hipEventSynchronize");
      float ms = 0;
      hip_check(hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
      const double t = ms / reps;
      if (t < best_t) { best_t = t; best = cfg; }
    }
    store[tune_key(arch, pl->opts.prec, Ms, s.K1, s.K2, s.N, c, split)] = {best, best_t};
    for (size_t x : kv.second) {
      if (pl->steps[x].cfg != best) changed = true;
      pl->steps[x].cfg = best;
    }
    const double cm = (double)c * Ms * s.K1 * s.K2 * s.N;
    if (cm > worst_cmac) {
      worst_cmac = cm;
      if (best_ms) *best_ms = best_t;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  tune_cache_store(store);
  if (changed) {
    // captured sweeps replay the old tile configurations: drop them, and make
    // every group that holds this plan re-capture (its graph key has tune_gen)
    clear_graphs(pl);
    ++pl->tune_gen;
  }
}

namespace {

void check_batch(const psim_plan_t* pl, const uint8_t* bits, size_t n, void* ws, size_t ws_bytes, double* out) {
  if (pl->host_only) fail(PSIM_EINVAL, "plan was made with PSIM_PLAN_HOST_ONLY");
  if (!bits || !out) fail(PSIM_EINVAL, "bits or out is NULL");
  if (n == 0) return;
  if (!ws) fail(PSIM_EINVAL, "workspace is NULL");
  if (ws_bytes < pl->ws_total)
    fail(PSIM_EINVAL, "workspace has " + std::to_string(ws_bytes) + " bytes, plan needs " +
                          std::to_string(pl->ws_total));
  const size_t nq = (size_t)pl->lv * pl->lh;
  for (size_t x = 0; x < n * nq; ++x)
    if (bits[x] > 1) fail(PSIM_EINVAL, "bit " + std::to_string(x) + " is not 0 or 1");
}

// Sub-batches whose prefix trie fits the planned capacities: sort the
// bitstrings by their swept rows (row 0 first) so that neighbours share the
// longest prefixes, then cut greedily.  Returns lists of bitstring indices.
std::vector<std::vector<size_t>> split_batches(const psim_plan_t* pl, const uint8_t* bits, size_t n) {
  const int nq = pl->lv * pl->lh;
  std::vector<size_t> order(n);
  for (size_t b = 0; b < n; ++b) order[b] = b;
  auto rowkey = [&](size_t b, int i) {
    uint64_t key = 0;
    for (int j = 0; j < pl->L; ++j) key |= (uint64_t)bits[b * nq + pl->cs[(size_t)i * pl->L + j].qubit] << j;
    return key;
  };
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
    for (int i = 0; i < pl->R; ++i) {
      const uint64_t a = rowkey(x, i), b = rowkey(y, i);
      if (a != b) return a < b;
    }
    return false;
  });
  std::vector<std::vector<size_t>> out;
  std::vector<int64_t> count(pl->R, 0);
  size_t start = 0;
  for (size_t x = 0; x < n; ++x) {
    // first swept row where this bitstring leaves the previous one's path
    int first = 0;
    if (x > start) {
      while (first < pl->R && rowkey(order[x], first) == rowkey(order[x - 1], first)) ++first;
    }
    bool fits = (int64_t)(x - start + 1) <= (int64_t)pl->opts.max_batch;
    for (int i = (x > start ? first : 0); i < pl->R && fits; ++i) fits = count[i] + 1 <= pl->levels[i].cap;
    if (!fits) {
      out.emplace_back(order.begin() + start, order.begin() + x);
      start = x;
      std::fill(count.begin(), count.end(), 0);
      first = 0;
    }
    for (int i = (x > start ? first : 0); i < pl->R; ++i) ++count[i];
  }
  if (n > start) out.emplace_back(order.begin() + start, order.end());
  return out;
}

// One device operation of the row sweep: a site contraction or a row rescale.
struct Op {
  bool rescale = false;
  int cls = 0;  // 0 first site, 1 interior site, 2 last site, 3 rescale
  double cmac = 0;
  double bytes = 0;  // algorithmic device-memory traffic
  GemmLaunch g;
  // rescale arguments
  void* F = nullptr;
  int64_t F_elems = 0, nodes = 0;
  const int32_t* parent = nullptr;
  const int32_t* e_in = nullptr;
  int32_t* e_out = nullptr;
  uint32_t* mx = nullptr;
  int row = 0;
};

// One sub-batch of one plan, ready to run: its trie (uploaded to the
// workspace) and the ordered operations that contract it.
struct Prepared {
  psim_plan_t* pl = nullptr;
  std::vector<uint8_t> bits;  // the sub-batch's bitstrings, nq bytes each
  size_t n = 0;
  Trie t;
  WsLayout W;
  std::vector<Op> ops;
  std::vector<char> vals;     // downloaded leaf boundaries (scalars)
  std::vector<int32_t> ex;    // and their exponents
};

// Builds the trie and the operation list of one sub-batch.  The trie tables
// and the root exponent are written to tab_img, the host image of the table
// region (pl->ws_tab bytes, zero-filled by the caller); the caller uploads it
// to P.W.tab before the operations run.
void prepare(psim_plan_t* pl, const uint8_t* bits, const std::vector<size_t>& idx, void* ws, char* tab_dev,
             char* tab_img, Prepared& P) {
  const int R = pl->R, L = pl->L, prec = pl->opts.prec, nq = pl->lv * pl->lh;
  const uint64_t eb = pl->elem_bytes;
  P.pl = pl;
  P.n = idx.size();
  P.bits.resize(P.n * nq);
  for (size_t x = 0; x < P.n; ++x) std::memcpy(&P.bits[x * nq], bits + idx[x] * nq, nq);
  P.t = build_trie(*pl, P.bits.data(), P.n);
  P.W = layout(*pl, ws, tab_dev);
  const Trie& t = P.t;
  WsLayout& W = P.W;
  for (int i = 0; i < R; ++i) {
    if ((int64_t)t.parent[i].size() > pl->levels[i].cap) fail(PSIM_EINTERNAL, "trie larger than planned");
    std::memcpy(tab_img + ((char*)W.parent[i] - W.tab), t.parent[i].data(), t.parent[i].size() * 4);
    std::memcpy(tab_img + ((char*)W.tau[i] - W.tab), t.tau[i].data(), t.tau[i].size());
  }
  // root exponent 0
  std::memset(tab_img + ((char*)W.exp[1] - W.tab), 0, 4);

  P.ops.clear();
  for (int i = 0; i < R; ++i) {
    const Level& lev = pl->levels[i];
    const int64_t nodes = (int64_t)t.parent[i].size();
    const void* Fprev = i == 0 ? pl->d_ones : (const void*)W.F[(i - 1) % 2];
    const int64_t Fprev_elems = i == 0 ? 1 : pl->levels[i - 1].F_elems;
    char* Fcur = W.F[i % 2];
    const int c = lev.vchunk;
    const bool wc = w_cut(lev);
    const int cw = wc ? lev.wchunk : 1;
    const int64_t rows_per_col = (prec == PSIM_FP32_3M) ? 1 : 2;  // packed rows per complex column (first site)
    for (int64_t g0 = 0; g0 < nodes; g0 += lev.group) {
      const int64_t gn = std::min<int64_t>(lev.group, nodes - g0);
      for (int v0 = 0; v0 < lev.Dv; v0 += c) {
        for (int w0 = 0; w0 < (wc ? lev.Dw : 1); w0 += cw) {
          for (int j = 0; j < L; ++j) {
            const Step& s = pl->steps[(size_t)i * L + j];
            const DevMatrix& w0m = pl->w[((size_t)i * L + j) * 2];
            const DevMatrix& w1m = pl->w[((size_t)i * L + j) * 2 + 1];
            Op op;
            GemmLaunch& g = op.g;
            g.prec = (prec == PSIM_FP32_3M && s.kind == 2) ? PSIM_FP32_4M : prec;  // see the packing
            g.cfg = s.kind == 1 ? s.cfg : 0;
            g.split = (pl->opts.flags & PSIM_PLAN_SPLIT_ACC) ? 1 : 0;
            const bool bf16_companion = pl->companion && prec == PSIM_BF16X3;
            if (pl->companion && !bf16_companion) {  // the other K-loop accumulation
              g.split ^= 1;
              if (g.split && !split_candidate(prec, g.cfg)) g.cfg = 0;  // the split kernels' tiles
            }
            if (bf16_companion) g.prec = PSIM_FP32_4M;           // the FP32 4M matrices every BF16x3 site has
            if (s.kind == 1 && w0m.ptr_b && !bf16_companion) {
              g.Wb0 = w0m.ptr_b;
              g.Wb1 = w1m.ptr_b;
              g.ldwb = w0m.ld_b;
              g.planeb = w0m.plane_b;
            }
            g.W0 = w0m.ptr;
            g.W1 = w1m.ptr;
            g.ldw = w0m.ld;
            g.tau = W.tau[i] + g0 * L + j;
            g.tau_stride = L;
            g.nodes = gn;
            g.N = s.N;
            g.K2 = s.K2;
            g.M = s.M;
            if (s.kind == 2) {
              g.trans_out = 1;
              g.C = Fcur + (uint64_t)g0 * lev.F_elems * eb;
              g.sC_node = lev.F_elems;
              if (L == 1) {  // the only site: contracts the parent's boundary directly
                g.Bz = 1;
                g.A = Fprev;
                g.a_index = W.parent[i] + g0;
                g.sA_node = Fprev_elems;
                g.K1 = lev.Dv;
                g.beta = 0;
              } else if (!wc) {
                g.Bz = 1;
                g.A = W.G[(L - 2) % 2];
                g.sA_node = (int64_t)c * s.M * s.K2;
                g.K1 = c;
                g.w_koff = (int64_t)v0 * s.K2;
                g.beta = v0 > 0;
              } else {
                // one batch entry per w of the chunk: its c v values are the
                // K1 blocks; F[d_last][w][d_1 ..] receives C^T at column w
                const int64_t Mt = s.M / lev.Dw;
                g.M = Mt;
                g.Bz = cw;
                g.A = W.G[(L - 2) % 2];
                g.sA_v = (int64_t)c * Mt * s.K2;
                g.sA_node = (int64_t)cw * g.sA_v;
                g.K1 = c;
                g.w_koff = (int64_t)v0 * s.K2;
                g.beta = v0 > 0;
                g.C = (char*)g.C + (uint64_t)w0 * Mt * eb;
                g.sC_v = Mt;
                g.ldct = (int64_t)lev.Dw * Mt;
              }
            } else if (!wc) {
              g.Bz = c;
              g.K1 = s.K1;
              g.C = W.G[j % 2];
              g.sC_v = s.g_out;
              g.sC_node = (int64_t)c * s.g_out;
              if (s.kind == 0) {
                g.A = (const char*)Fprev + (uint64_t)v0 * s.K1 * s.M * eb;
                g.a_index = W.parent[i] + g0;
                g.sA_node = Fprev_elems;
                g.sA_v = s.K1 * s.M;
              } else {
                g.A = W.G[(j - 1) % 2];
                g.sA_v = s.K1 * s.M * s.K2;
                g.sA_node = (int64_t)c * g.sA_v;
              }
            } else if (s.kind == 0) {
              // the columns (w, r_0) of the w chunk: packed rows from w0 * dr on;
              // results stored per (w, v) pair as [w][v][m][r_0]
              const int64_t dr = pl->cs[(size_t)i * L].dr;
              const uint64_t off = (uint64_t)w0 * dr * rows_per_col * w0m.ld * (prec == PSIM_FP64 ? 8 : 4);
              g.W0 = (const char*)w0m.ptr + off;
              g.W1 = (const char*)w1m.ptr + off;
              g.N = (int64_t)cw * dr;
              g.Bz = c;
              g.K1 = s.K1;
              g.A = (const char*)Fprev + (uint64_t)v0 * s.K1 * s.M * eb;
              g.a_index = W.parent[i] + g0;
              g.sA_node = Fprev_elems;
              g.sA_v = s.K1 * s.M;
              g.C = W.G[0];
              g.sC_v = s.M * dr;
              g.nb = dr;
              g.sCw = (int64_t)c * s.M * dr;
              g.sC_node = (int64_t)cw * g.sCw;
            } else {
              // interior site on every (w, v) pair of the pass, d_0 out of the rows
              const int64_t Mt = s.M / lev.Dw;
              g.M = Mt;
              g.Bz = c * cw;
              g.K1 = s.K1;
              g.A = W.G[(j - 1) % 2];
              g.sA_v = s.K1 * Mt * s.K2;
              g.sA_node = (int64_t)c * cw * g.sA_v;
              g.C = W.G[j % 2];
              g.sC_v = Mt * s.N;
              g.sC_node = (int64_t)c * cw * g.sC_v;
            }
            // class 1 is eq. S4 proper: interior sites of interior rows; the
            // first and last rows' interior sites (small M or N) join class 0
            op.cls = (s.kind == 1 && (i == 0 || i == R - 1)) ? 0 : s.kind;
            op.cmac = (double)g.nodes * g.Bz * g.M * g.K1 * g.K2 * g.N;
            op.bytes = (double)eb * ((double)g.nodes * g.Bz * g.K1 * g.M * g.K2 +
                                     (double)g.nodes * g.Bz * g.M * g.N * (g.beta ? 2 : 1) +
                                     (double)g.K1 * g.K2 * g.N);
            op.row = i;
            P.ops.push_back(op);
          }
        }
        if (L == 1) break;  // the single site consumed every v at once
      }
    }
    // exact power-of-two rescale of every node's boundary; exponents along the trie
    Op op;
    op.rescale = true;
    op.cls = 3;
    op.bytes = 3.0 * eb * (double)nodes * lev.F_elems;
    op.F = Fcur;
    op.F_elems = lev.F_elems;
    op.nodes = nodes;
    op.parent = W.parent[i];
    op.e_in = W.exp[(i + 1) % 2];
    op.e_out = W.exp[i % 2];
    op.mx = W.mx;
    op.row = i;
    P.ops.push_back(op);
  }
  if ((int64_t)P.ops.size() > pl->max_ops) fail(PSIM_EINTERNAL, "more operations than planned");
}

void run_op(const psim_plan_t* pl, const Op& op, hipStream_t st) {
  if (op.rescale)
    launch_rowscale(pl->opts.prec, op.F, op.F_elems, op.nodes, op.parent, const_cast<int32_t*>(op.e_in), op.e_out,
                    op.mx, st);
  else
    launch_site_gemm(op.g, st);
}

void enqueue_download(Prepared& P, hipStream_t st) {
  const psim_plan_t* pl = P.pl;
  const int R = pl->R;
  const int64_t leaves = (int64_t)P.t.parent[R - 1].size();
  P.vals.resize((size_t)leaves * pl->elem_bytes);
  P.ex.resize((size_t)leaves);
  hip_check(hipMemcpyAsync(P.vals.data(), P.W.F[(R - 1) % 2], P.vals.size(), hipMemcpyDeviceToHost, st), "download");
  hip_check(hipMemcpyAsync(P.ex.data(), P.W.exp[(R - 1) % 2], P.ex.size() * 4, hipMemcpyDeviceToHost, st),
            "download");
}

// amplitude b = mantissa * 2^(row exponents + site-matrix exponents), in FP64
void assemble(const Prepared& P, const std::vector<size_t>& idx, double* out) {
  const psim_plan_t* pl = P.pl;
  const int R = pl->R, L = pl->L, nq = pl->lv * pl->lh;
  for (size_t b = 0; b < P.n; ++b) {
    const int32_t leaf = P.t.leaf[b];
    double re, im;
    if (pl->elem_bytes == 16) {
      const double* v = (const double*)P.vals.data();
      re = v[2 * leaf];
      im = v[2 * leaf + 1];
    } else {
      const float* v = (const float*)P.vals.data();
      re = v[2 * leaf];
      im = v[2 * leaf + 1];
    }
    int64_t e = P.ex[leaf];
    for (int i = 0; i < R; ++i)
      for (int j = 0; j < L; ++j) {
        const int tau = P.bits[b * nq + pl->cs[(size_t)i * L + j].qubit];
        e += pl->w[((size_t)i * L + j) * 2 + tau].exp2;
      }
    out[2 * idx[b]] = std::ldexp(re, (int)e);
    out[2 * idx[b] + 1] = std::ldexp(im, (int)e);
  }
}

// One sub-batch of one plan on its own: optional event timing, row progress
// log, or graph capture / replay of the operation list.
void run_one(psim_plan_t* pl, const uint8_t* bits, const std::vector<size_t>& idx, void* ws, hipStream_t st,
             double* out, bool no_alloc) {
  Prepared P;
  std::vector<char> img(pl->ws_tab, 0);
  prepare(pl, bits, idx, ws, nullptr, img.data(), P);
  hip_check(hipMemcpyAsync(P.W.tab, img.data(), img.size(), hipMemcpyHostToDevice, st), "upload tables");

  struct Timed {
    hipEvent_t a, b;
    int cls;
    double cmac, bytes;
  };
  std::vector<Timed> timed;
  const char* env_log = std::getenv("PSIM_LOG");
  const bool log_rows = env_log && env_log[0] == '1';
  const auto t_begin = std::chrono::steady_clock::now();

  // The launch sequence depends only on the workspace address and the number
  // of nodes per level; the tables it reads were uploaded by prepare().
  // events are created per launch while profiling; the companion sweep of an
  // error estimate is not profiled
  const bool profile = pl->profile && !no_alloc && !pl->companion;
  const bool use_graph = (pl->opts.flags & PSIM_PLAN_GRAPH) && !profile && !log_rows && !no_alloc;
  hipGraphExec_t gexec = nullptr;
  bool capturing = false;
  std::vector<int64_t> gkey;
  if (use_graph) {
    gkey.push_back((int64_t)(uintptr_t)ws);
    gkey.push_back(pl->companion);
    for (int i = 0; i < pl->R; ++i) gkey.push_back((int64_t)P.t.parent[i].size());
    auto it = pl->graphs.find(gkey);
    if (it != pl->graphs.end()) {
      gexec = (hipGraphExec_t)it->second;
    } else {
      if (!pl->cap_stream) {
        hipStream_t cs;
        hip_check(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
        pl->cap_stream = cs;
      }
      hip_check(hipStreamBeginCapture((hipStream_t)pl->cap_stream, hipStreamCaptureModeRelaxed),
                "hipStreamBeginCapture");
      capturing = true;
    }
  }
  hipStream_t lst = capturing ? (hipStream_t)pl->cap_stream : st;  // stream the sweep is recorded on
  if (!gexec) {
    try {
      for (const Op& op : P.ops) {
        if (profile) {
          Timed tm{};
          tm.cls = op.cls;
          tm.cmac = op.cmac;
          tm.bytes = op.bytes;
          hip_check(hipEventCreate(&tm.a), "hipEventCreate");
          hip_check(hipEventCreate(&tm.b), "hipEventCreate");
          hip_check(hipEventRecord(tm.a, lst), "hipEventRecord");
          timed.push_back(tm);
        }
        run_op(pl, op, lst);
        if (profile) hip_check(hipEventRecord(timed.back().b, lst), "hipEventRecord");
        if (log_rows && op.rescale) {  // progress for long runs: wait for the row, then report it
          hip_check(hipStreamSynchronize(lst), "hipStreamSynchronize");
          std::fprintf(stderr, "psim: row %d/%d done (%lld nodes) at %.2f s\n", op.row + 1, pl->R,
                       (long long)op.nodes,
                       std::chrono::duration<double>(std::chrono::steady_clock::now() - t_begin).count());
          std::fflush(stderr);
        }
      }
    } catch (...) {
      if (capturing) {
        hipGraph_t graph = nullptr;
        (void)hipStreamEndCapture(lst, &graph);
        if (graph) (void)hipGraphDestroy(graph);
      }
      throw;
    }
  }
  if (capturing) {
    hipGraph_t graph = nullptr;
    hip_check(hipStreamEndCapture(lst, &graph), "hipStreamEndCapture");
    const hipError_t e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    hip_check(e, "hipGraphInstantiate");
    if (pl->graphs.size() >= kMaxPlanGraphs) clear_graphs(pl);  // bounded cache: start over
    pl->graphs[gkey] = (void*)gexec;
  }
  if (gexec) hip_check(hipGraphLaunch(gexec, st), "hipGraphLaunch");

  enqueue_download(P, st);
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
  for (Timed& tm : timed) {
    float ms = 0;
    hip_check(hipEventElapsedTime(&ms, tm.a, tm.b), "hipEventElapsedTime");
    pl->prof[tm.cls].ms += ms;
    pl->prof[tm.cls].launches += 1;
    pl->prof[tm.cls].cmac += tm.cmac;
    pl->prof[tm.cls].bytes += tm.bytes;
    (void)hipEventDestroy(tm.a);
    (void)hipEventDestroy(tm.b);
  }
  assemble(P, idx, out);
}

}  // namespace

namespace {

void sweep(psim_plan_t* pl, const uint8_t* bits, size_t n, void* ws, void* stream, double* res, bool no_alloc) {
  if (pl->sq) {
    run_square(pl, bits, n, ws, stream, res, no_alloc);
  } else {
    hip_check(hipSetDevice(pl->opts.device), "hipSetDevice");
    for (const auto& idx : split_batches(pl, bits, n)) run_one(pl, bits, idx, ws, (hipStream_t)stream, res, no_alloc);
  }
}

}  // namespace

void run_amplitudes(psim_plan_t* pl, const uint8_t* bits, size_t n, void* ws, size_t ws_bytes, void* stream,
                    double* out, bool no_alloc, double* out_err) {
  check_batch(pl, bits, n, ws, ws_bytes, out);
  if (n == 0) return;
  // results are assembled in host memory and copied to the outputs only once
  // every sub-batch has succeeded, so a failing call leaves them untouched
  std::vector<double> res(2 * n);
  sweep(pl, bits, n, ws, stream, res.data(), no_alloc);
  std::vector<double> err;
  if (out_err) {
    err.assign(n, std::nan(""));
    if (pl->opts.prec != PSIM_FP64) {
      std::vector<double> alt(2 * n);
      pl->companion = 1;
      try {
        sweep(pl, bits, n, ws, stream, alt.data(), no_alloc);
      } catch (...) {
        pl->companion = 0;
        throw;
      }
      pl->companion = 0;
      for (size_t b = 0; b < n; ++b) {
        const double dr = res[2 * b] - alt[2 * b], di = res[2 * b + 1] - alt[2 * b + 1];
        err[b] = std::hypot(dr, di) / std::hypot(alt[2 * b], alt[2 * b + 1]);
      }
    }
  }
  std::memcpy(out, res.data(), res.size() * sizeof(double));
  if (out_err) std::memcpy(out_err, err.data(), err.size() * sizeof(double));
}

// ------------------------------------------------------------------ groups
// Several plans (different circuits, lattices, depths) advance together:
// pass p runs sub-batch p of every plan, and step k of a pass issues
// operation k of every plan's list.  Site contractions of one step that share
// a kernel variant go into one grouped launch (one grid over all their
// tiles); the others are launched one by one.  Every plan's operations stay
// in their own order on the one stream, so each plan computes exactly what
// psim_amplitudes computes for it.
void free_group(psim_group_s* G);

psim_group_s* make_group(psim_plan_t* const* plans, int np) {
  if (!plans || np < 1) fail(PSIM_EINVAL, "plans is NULL or empty");
  auto* G = new psim_group_s();
  try {
    auto al = [](uint64_t x) { return (x + 255) / 256 * 256; };
    uint64_t off = 0;
    const uint64_t kb = (uint64_t)kargs_bytes();
    for (int p = 0; p < np; ++p) {
      psim_plan_t* pl = plans[p];
      if (!pl) fail(PSIM_EINVAL, "plan " + std::to_string(p) + " is NULL");
      if (pl->host_only) fail(PSIM_EINVAL, "plan " + std::to_string(p) + " was made with PSIM_PLAN_HOST_ONLY");
      if (pl->opts.device != plans[0]->opts.device) fail(PSIM_EINVAL, "plans are on different devices");
      if (pl->sq) fail(PSIM_EUNSUPPORTED, "plan " + std::to_string(p) + " uses the square partition (not groupable)");
      G->plans.push_back(pl);
      G->desc_off.push_back(off);
      off += al((uint64_t)pl->max_ops * kb);
      G->tab_off.push_back(off);
      off += al(pl->ws_tab);
    }
    G->seg_off = off;
    off += al((uint64_t)np * 2 * sizeof(CopySeg));
    G->res_begin = off;
    for (int p = 0; p < np; ++p) {
      const psim_plan_t* pl = plans[p];
      const uint64_t leaves = (uint64_t)pl->levels[pl->R - 1].cap;
      G->res_off.push_back(off);
      off += al(leaves * pl->elem_bytes);
      G->res_exp_off.push_back(off);
      off += al(leaves * 4);
    }
    G->bytes = off;
    G->device = plans[0]->opts.device;
    G->desc_bytes = off;
    hip_check(hipSetDevice(G->device), "hipSetDevice");
    hip_check(hipMalloc(&G->d_buf, off), "hipMalloc(group buffer)");
    hip_check(hipHostMalloc((void**)&G->h_buf, off, hipHostMallocDefault), "hipHostMalloc(group staging)");
  } catch (...) {
    free_group(G);
    throw;
  }
  return G;
}

void free_group(psim_group_s* G) {
  if (!G) return;
  for (auto& kv : G->graphs) (void)hipGraphExecDestroy((hipGraphExec_t)kv.second.first);
  if (G->cap_stream) (void)hipStreamDestroy((hipStream_t)G->cap_stream);
  if (G->d_buf) (void)hipFree(G->d_buf);
  if (G->h_buf) (void)hipHostFree(G->h_buf);
  delete G;
}

void run_group(psim_group_s* G, const uint8_t* const* bits, const size_t* n, void* const* ws, const size_t* ws_bytes,
               void* stream, double* const* out) {
  const int np = (int)G->plans.size();
  if (!bits || !n || !ws || !ws_bytes || !out) fail(PSIM_EINVAL, "an argument array is NULL");
  for (int p = 0; p < np; ++p) {
    try {
      check_batch(G->plans[p], bits[p], n[p], ws[p], ws_bytes[p], out[p]);
    } catch (const Error& e) {
      fail(e.status, "plan " + std::to_string(p) + ": " + e.msg);
    }
  }
  // workspaces must not overlap (each plan's sweep writes its own)
  for (int p = 0; p < np; ++p)
    for (int q = p + 1; q < np; ++q) {
      if (!n[p] || !n[q]) continue;
      const uintptr_t a0 = (uintptr_t)ws[p], a1 = a0 + G->plans[p]->ws_total;
      const uintptr_t b0 = (uintptr_t)ws[q], b1 = b0 + G->plans[q]->ws_total;
      if (a0 < b1 && b0 < a1) fail(PSIM_EINVAL, "workspaces of plans " + std::to_string(p) + " and " +
                                                    std::to_string(q) + " overlap");
    }
  hip_check(hipSetDevice(G->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  std::vector<std::vector<std::vector<size_t>>> subs(np);
  size_t passes = 0;
  for (int p = 0; p < np; ++p) {
    if (n[p]) subs[p] = split_batches(G->plans[p], bits[p], n[p]);
    passes = std::max(passes, subs[p].size());
  }
  const int kb = kargs_bytes();
  const int maxg = max_group();
  const int maxs = max_scale_group();
  // every plan's results in host memory until the last pass has succeeded
  std::vector<std::vector<double>> res(np);
  for (int p = 0; p < np; ++p) res[p].resize(2 * n[p]);
  char* dbuf = (char*)G->d_buf;
  char* hbuf = G->h_buf;
  CopySeg* hseg = (CopySeg*)(hbuf + G->seg_off);
  for (size_t pass = 0; pass < passes; ++pass) {
    // host image of everything the pass reads: trie tables (relocated into
    // the group buffer), launch descriptors, the result-gather segments
    std::vector<Prepared> P;
    std::vector<int> who;
    for (int p = 0; p < np; ++p)
      if (pass < subs[p].size()) {
        P.emplace_back();
        who.push_back(p);
        std::memset(hbuf + G->tab_off[p], 0, G->plans[p]->ws_tab);
        prepare(G->plans[p], bits[p], subs[p][pass], ws[p], dbuf + G->tab_off[p], hbuf + G->tab_off[p], P.back());
      }
    const size_t m = P.size();
    std::vector<std::vector<int>> variant(m);
    std::vector<std::vector<long long>> tiles(m);
    size_t steps = 0;
    int64_t max_seg = 0;
    for (size_t q = 0; q < m; ++q) {
      const int p = who[q];
      const auto& ops = P[q].ops;
      steps = std::max(steps, ops.size());
      variant[q].assign(ops.size(), -1);
      tiles[q].assign(ops.size(), 0);
      for (size_t k = 0; k < ops.size(); ++k)
        if (!ops[k].rescale) variant[q][k] = group_variant(ops[k].g, hbuf + G->desc_off[p] + k * kb, &tiles[q][k]);
      const psim_plan_t* pl = P[q].pl;
      const int64_t leaves = (int64_t)P[q].t.parent[pl->R - 1].size();
      hseg[2 * q] = CopySeg{P[q].W.F[(pl->R - 1) % 2], dbuf + G->res_off[p], leaves * pl->elem_bytes};
      hseg[2 * q + 1] = CopySeg{P[q].W.exp[(pl->R - 1) % 2], dbuf + G->res_exp_off[p], leaves * 4};
      max_seg = std::max(max_seg, leaves * (int64_t)pl->elem_bytes);
    }
    hip_check(hipMemcpyAsync(dbuf, hbuf, G->res_begin, hipMemcpyHostToDevice, st), "upload group tables");
    // the interleaved sweep; returns the number of merged launches issued
    auto issue = [&](hipStream_t ls) {
      int64_t merged = 0;
      for (size_t k = 0; k < steps; ++k) {
        std::map<int, std::vector<std::pair<size_t, size_t>>> byvar;  // variant -> (plan slot, op)
        std::map<int, std::vector<RescaleJob>> scale;  // storage (FP64 or FP32) -> fused rescales
        for (size_t q = 0; q < m; ++q) {
          if (k >= P[q].ops.size()) continue;
          const Op& op = P[q].ops[k];
          if (op.rescale && rescale_fusable(op.F_elems))
            scale[P[q].pl->elem_bytes == 16 ? PSIM_FP64 : PSIM_FP32_4M].push_back(
                RescaleJob{op.F, op.F_elems, op.nodes, op.parent, op.e_in, op.e_out});
          else if (variant[q][k] < 0)
            run_op(P[q].pl, op, ls);
          else
            byvar[variant[q][k]].emplace_back(q, k);
        }
        for (auto& kv : scale)
          for (size_t a = 0; a < kv.second.size(); a += maxs) {
            const int cnt = (int)std::min<size_t>(maxs, kv.second.size() - a);
            launch_rescale_group(kv.first, kv.second.data() + a, cnt, ls);
          }
        for (auto& kv : byvar) {
          const auto& lst = kv.second;
          if (lst.size() == 1) {  // nothing to merge with
            run_op(P[lst[0].first].pl, P[lst[0].first].ops[lst[0].second], ls);
            continue;
          }
          for (size_t a = 0; a < lst.size(); a += maxg) {
            const int cnt = (int)std::min<size_t>(maxg, lst.size() - a);
            std::vector<const void*> probs(cnt);
            std::vector<long long> start(cnt + 1, 0);
            for (int x = 0; x < cnt; ++x) {
              const size_t q = lst[a + x].first, kk = lst[a + x].second;
              probs[x] = dbuf + G->desc_off[who[q]] + kk * kb;
              start[x + 1] = start[x] + tiles[q][kk];
            }
            launch_group(kv.first, probs.data(), start.data(), cnt, ls);
            merged += 1;
          }
        }
      }
      // every plan's leaf values and exponents into the group buffer
      launch_copy_segments((const CopySeg*)(dbuf + G->seg_off), (int)(2 * m), max_seg, ls);
      return merged;
    };
    // Graph replay when every plan asks for it: the launch sequence depends
    // only on which plans take part, their workspaces and their trie shapes
    // (the descriptors and tables it reads were uploaded above).
    bool use_graph = true;
    for (size_t q = 0; q < m; ++q) use_graph = use_graph && (P[q].pl->opts.flags & PSIM_PLAN_GRAPH);
    if (!use_graph) {
      G->grouped_launches += issue(st);
    } else {
      std::vector<int64_t> key;
      for (size_t q = 0; q < m; ++q) {
        key.push_back(who[q]);
        key.push_back(P[q].pl->tune_gen);   // tile configurations as tuned when captured
        key.push_back((int64_t)(uintptr_t)ws[who[q]]);
        for (const auto& lev : P[q].t.parent) key.push_back((int64_t)lev.size());
      }
      auto it = G->graphs.find(key);
      if (it == G->graphs.end()) {
        if (!G->cap_stream) {
          hipStream_t cs;
          hip_check(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
          G->cap_stream = cs;
        }
        hipStream_t cs = (hipStream_t)G->cap_stream;
        hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
        int64_t merged = 0;
        try {
          merged = issue(cs);
        } catch (...) {
          hipGraph_t graph = nullptr;
          (void)hipStreamEndCapture(cs, &graph);
          if (graph) (void)hipGraphDestroy(graph);
          throw;
        }
        hipGraph_t graph = nullptr;
        hip_check(hipStreamEndCapture(cs, &graph), "hipStreamEndCapture");
        hipGraphExec_t gexec = nullptr;
        const hipError_t e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        hip_check(e, "hipGraphInstantiate");
        it = G->graphs.emplace(key, std::make_pair((void*)gexec, merged)).first;
      }
      hip_check(hipGraphLaunch((hipGraphExec_t)it->second.first, st), "hipGraphLaunch");
      G->grouped_launches += it->second.second;
    }
    hip_check(hipMemcpyAsync(hbuf + G->res_begin, dbuf + G->res_begin, G->bytes - G->res_begin,
                             hipMemcpyDeviceToHost, st), "download group results");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    for (size_t q = 0; q < m; ++q) {
      const int p = who[q];
      const psim_plan_t* pl = P[q].pl;
      const size_t leaves = P[q].t.parent[pl->R - 1].size();
      P[q].vals.assign(hbuf + G->res_off[p], hbuf + G->res_off[p] + leaves * pl->elem_bytes);
      P[q].ex.resize(leaves);
      std::memcpy(P[q].ex.data(), hbuf + G->res_exp_off[p], leaves * 4);
      assemble(P[q], subs[who[q]][pass], res[who[q]].data());
    }
  }
  for (int p = 0; p < np; ++p)
    if (n[p]) std::memcpy(out[p], res[p].data(), res[p].size() * sizeof(double));
}
