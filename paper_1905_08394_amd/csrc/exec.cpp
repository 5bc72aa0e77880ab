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

// Workspace layout: per-level trie tables, exponents, row maxima, the two
// boundary buffers (even / odd rows) and the two intermediate buffers.
struct WsLayout {
  std::vector<int32_t*> parent;
  std::vector<uint8_t*> tau;
  int32_t* exp[2];
  uint32_t* mx;
  char* F[2];
  char* G[2];
};

WsLayout layout(const psim_plan_t& pl, void* ws) {
  auto al = [](uint64_t x) { return (x + 255) / 256 * 256; };
  char* p = (char*)(((uintptr_t)ws + 255) / 256 * 256);
  WsLayout w;
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
  w.F[0] = p + pl.levels[0].F_off;
  w.F[1] = p + (R > 1 ? pl.levels[1].F_off : 0);
  p += pl.ws_F;
  w.G[0] = p;
  w.G[1] = p + pl.ws_G / 2;
  return w;
}

}  // namespace

void tune_plan(psim_plan_t* pl, void* ws, size_t ws_bytes, void* stream, int reps, double* best_ms) {
  if (pl->host_only) fail(PSIM_EINVAL, "plan was made with PSIM_PLAN_HOST_ONLY");
  if (!ws || ws_bytes < pl->ws_total) fail(PSIM_EINVAL, "workspace is NULL or smaller than the plan needs");
  if (reps < 1) fail(PSIM_EINVAL, "reps must be at least 1");
  if (best_ms) *best_ms = 0;
  if ((pl->opts.prec != PSIM_FP32_4M && pl->opts.prec != PSIM_FP32_3M) || (pl->opts.flags & PSIM_PLAN_SPLIT_ACC))
    return;
  const int ncfg = pl->opts.prec == PSIM_FP32_3M ? fp32_3m_config_count() : fp32_config_count();
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
    shapes[{s.M, s.K1, s.K2, s.N, (int64_t)lev.vchunk}].push_back(x);
  }
  hipEvent_t a, b;
  hip_check(hipEventCreate(&a), "hipEventCreate");
  hip_check(hipEventCreate(&b), "hipEventCreate");
  for (auto& kv : shapes) {
    const Step& s = pl->steps[kv.second.front()];
    const int c = pl->levels[s.i].vchunk;
    GemmLaunch g;
    g.prec = pl->opts.prec;
    g.A = W.G[0];
    g.C = W.G[1];
    g.W0 = g.W1 = pl->w[((size_t)s.i * L + s.j) * 2].ptr;
    g.ldw = pl->w[((size_t)s.i * L + s.j) * 2].ld;
    g.M = s.M; g.K1 = s.K1; g.K2 = s.K2; g.N = s.N;
    g.nodes = 1; g.Bz = c;
    g.sA_v = s.K1 * s.M * s.K2; g.sA_node = c * g.sA_v;
    g.sC_v = s.g_out; g.sC_node = c * s.g_out;
    int best = 0;
    double best_t = 1e300;
    for (int cfg = 0; cfg < ncfg; ++cfg) {
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
    for (size_t x : kv.second) pl->steps[x].cfg = best;
    const double cm = (double)c * s.M * s.K1 * s.K2 * s.N;
    if (cm > worst_cmac) {
      worst_cmac = cm;
      if (best_ms) *best_ms = best_t;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
}

void run_amplitudes(psim_plan_t* pl, const uint8_t* bits, size_t n, void* ws, size_t ws_bytes, void* stream,
                    double* out) {
  if (pl->host_only) fail(PSIM_EINVAL, "plan was made with PSIM_PLAN_HOST_ONLY");
  if (!bits || !out) fail(PSIM_EINVAL, "bits or out is NULL");
  if (n == 0) return;
  if (!ws) fail(PSIM_EINVAL, "workspace is NULL");
  if (ws_bytes < pl->ws_total)
    fail(PSIM_EINVAL, "workspace has " + std::to_string(ws_bytes) + " bytes, plan needs " +
                          std::to_string(pl->ws_total));
  const int nq = pl->lv * pl->lh;
  for (size_t x = 0; x < n * (size_t)nq; ++x)
    if (bits[x] > 1) fail(PSIM_EINVAL, "bit " + std::to_string(x) + " is not 0 or 1");
  // Split into sub-batches whose prefix trie fits the planned capacities:
  // sort the bitstrings by their swept rows (row 0 first) so that neighbours
  // share the longest prefixes, then cut greedily.
  if (!pl->in_subbatch) {
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
    std::vector<uint8_t> sb;
    std::vector<double> so;
    std::vector<int64_t> count(pl->R, 0);
    size_t start = 0;
    auto flush = [&](size_t end) {
      const size_t m = end - start;
      sb.resize(m * nq);
      so.resize(2 * m);
      for (size_t x = 0; x < m; ++x) std::memcpy(&sb[x * nq], bits + order[start + x] * nq, nq);
      pl->in_subbatch = true;
      try {
        run_amplitudes(pl, sb.data(), m, ws, ws_bytes, stream, so.data());
      } catch (...) {
        pl->in_subbatch = false;
        throw;
      }
      pl->in_subbatch = false;
      for (size_t x = 0; x < m; ++x) {
        out[2 * order[start + x]] = so[2 * x];
        out[2 * order[start + x] + 1] = so[2 * x + 1];
      }
      start = end;
    };
    for (size_t x = 0; x < n; ++x) {
      // first swept row where this bitstring leaves the previous one's path
      int first = 0;
      if (x > start) {
        while (first < pl->R && rowkey(order[x], first) == rowkey(order[x - 1], first)) ++first;
      }
      bool fits = (int64_t)(x - start + 1) <= (int64_t)pl->opts.max_batch;
      for (int i = (x > start ? first : 0); i < pl->R && fits; ++i) fits = count[i] + 1 <= pl->levels[i].cap;
      if (!fits) {
        flush(x);
        std::fill(count.begin(), count.end(), 0);
        first = 0;
      }
      for (int i = (x > start ? first : 0); i < pl->R; ++i) ++count[i];
    }
    flush(n);
    return;
  }
  hip_check(hipSetDevice(pl->opts.device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  const int R = pl->R, L = pl->L, prec = pl->opts.prec;
  const uint64_t eb = pl->elem_bytes;
  Trie t = build_trie(*pl, bits, n);

  // ------------------------------------------------------------ workspace
  WsLayout W = layout(*pl, ws);
  std::vector<int32_t*>& d_parent = W.parent;
  std::vector<uint8_t*>& d_tau = W.tau;
  int32_t** d_exp = W.exp;
  uint32_t* d_max = W.mx;
  char** dF = W.F;
  char** dG = W.G;

  for (int i = 0; i < R; ++i) {
    if ((int64_t)t.parent[i].size() > pl->levels[i].cap) fail(PSIM_EINTERNAL, "trie larger than planned");
    hip_check(hipMemcpyAsync(d_parent[i], t.parent[i].data(), t.parent[i].size() * 4, hipMemcpyHostToDevice, st),
              "upload parents");
    hip_check(hipMemcpyAsync(d_tau[i], t.tau[i].data(), t.tau[i].size(), hipMemcpyHostToDevice, st),
              "upload bits");
  }
  // root exponent 0
  const int32_t zero = 0;
  hip_check(hipMemcpyAsync(d_exp[1], &zero, 4, hipMemcpyHostToDevice, st), "upload exponent");

  // ------------------------------------------------------------ event timing (optional)
  struct Timed {
    hipEvent_t a, b;
    int cls;
    double cmac;
  };
  std::vector<Timed> timed;
  auto tstart = [&](int cls, double cmac) {
    if (!pl->profile) return;
    Timed t{};
    t.cls = cls;
    t.cmac = cmac;
    hip_check(hipEventCreate(&t.a), "hipEventCreate");
    hip_check(hipEventCreate(&t.b), "hipEventCreate");
    hip_check(hipEventRecord(t.a, st), "hipEventRecord");
    timed.push_back(t);
  };
  auto tstop = [&]() {
    if (!pl->profile) return;
    hip_check(hipEventRecord(timed.back().b, st), "hipEventRecord");
  };

  const char* env_log = std::getenv("PSIM_LOG");
  const bool log_rows = env_log && env_log[0] == '1';
  const auto t_begin = std::chrono::steady_clock::now();

  // ------------------------------------------------------------ graph replay (optional)
  // The launch sequence below depends only on the workspace address and the
  // number of nodes per level; the tables it reads were uploaded above.
  const bool use_graph = (pl->opts.flags & PSIM_PLAN_GRAPH) && !pl->profile && !log_rows;
  hipGraphExec_t gexec = nullptr;
  bool capturing = false;
  std::vector<int64_t> gkey;
  if (use_graph) {
    gkey.push_back((int64_t)(uintptr_t)ws);
    for (int i = 0; i < R; ++i) gkey.push_back((int64_t)t.parent[i].size());
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
  hipStream_t ust = st;  // stream the uploads and results use
  if (capturing) st = (hipStream_t)pl->cap_stream;

  // ------------------------------------------------------------ rows
  for (int i = 0; i < R && !gexec; ++i) {
    const Level& lev = pl->levels[i];
    const int64_t nodes = (int64_t)t.parent[i].size();
    const void* Fprev = i == 0 ? pl->d_ones : (const void*)dF[(i - 1) % 2];
    const int64_t Fprev_elems = i == 0 ? 1 : pl->levels[i - 1].F_elems;
    char* Fcur = dF[i % 2];
    const int c = lev.vchunk;
    for (int64_t g0 = 0; g0 < nodes; g0 += lev.group) {
      const int64_t gn = std::min<int64_t>(lev.group, nodes - g0);
      for (int v0 = 0; v0 < lev.Dv; v0 += c) {
        for (int j = 0; j < L; ++j) {
          const Step& s = pl->steps[(size_t)i * L + j];
          const DevMatrix& w0 = pl->w[((size_t)i * L + j) * 2];
          const DevMatrix& w1 = pl->w[((size_t)i * L + j) * 2 + 1];
          GemmLaunch g;
          g.prec = (prec == PSIM_FP32_3M && s.kind == 2) ? PSIM_FP32_4M : prec;  // see the packing
          g.cfg = s.kind == 1 ? s.cfg : 0;
          g.split = (pl->opts.flags & PSIM_PLAN_SPLIT_ACC) ? 1 : 0;
          if (s.kind == 1 && w0.ptr_b) {
            g.Wb0 = w0.ptr_b;
            g.Wb1 = w1.ptr_b;
            g.ldwb = w0.ld_b;
            g.planeb = w0.plane_b;
          }
          g.W0 = w0.ptr;
          g.W1 = w1.ptr;
          g.ldw = w0.ld;
          g.tau = d_tau[i] + g0 * L + j;
          g.tau_stride = L;
          g.nodes = gn;
          g.N = s.N;
          g.K2 = s.K2;
          g.M = s.M;
          if (s.kind == 2) {
            g.trans_out = 1;
            g.Bz = 1;
            g.C = Fcur + (uint64_t)g0 * lev.F_elems * eb;
            g.sC_node = lev.F_elems;
            if (L == 1) {  // the only site: contracts the parent's boundary directly
              g.A = Fprev;
              g.a_index = d_parent[i] + g0;
              g.sA_node = Fprev_elems;
              g.K1 = lev.Dv;
              g.beta = 0;
            } else {
              g.A = dG[(L - 2) % 2];
              g.sA_node = (int64_t)c * s.M * s.K2;
              g.K1 = c;
              g.w_koff = (int64_t)v0 * s.K2;
              g.beta = v0 > 0;
            }
          } else {
            g.Bz = c;
            g.K1 = s.K1;
            g.C = dG[j % 2];
            g.sC_v = s.g_out;
            g.sC_node = (int64_t)c * s.g_out;
            if (s.kind == 0) {
              g.A = (const char*)Fprev + (uint64_t)v0 * s.K1 * s.M * eb;
              g.a_index = d_parent[i] + g0;
              g.sA_node = Fprev_elems;
              g.sA_v = s.K1 * s.M;
            } else {
              g.A = dG[(j - 1) % 2];
              g.sA_v = s.K1 * s.M * s.K2;
              g.sA_node = (int64_t)c * g.sA_v;
            }
          }
          tstart(s.kind, (double)g.nodes * g.Bz * g.M * g.K1 * g.K2 * g.N);
          launch_site_gemm(g, st);
          tstop();
        }
        if (L == 1) break;  // the single site consumed every v at once
      }
    }
    // exact power-of-two rescale of every node's boundary; exponents along the trie
    tstart(3, 0.0);
    launch_rowscale(prec, Fcur, lev.F_elems, nodes, d_parent[i], d_exp[(i + 1) % 2], d_exp[i % 2], d_max, st);
    tstop();
    if (log_rows) {  // progress for long runs: wait for the row, then report it
      hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
      std::fprintf(stderr, "psim: row %d/%d done (%lld nodes) at %.2f s\n", i + 1, R, (long long)nodes,
                   std::chrono::duration<double>(std::chrono::steady_clock::now() - t_begin).count());
      std::fflush(stderr);
    }
  }

  if (capturing) {
    hipGraph_t graph = nullptr;
    const hipError_t e1 = hipStreamEndCapture(st, &graph);
    st = ust;
    hip_check(e1, "hipStreamEndCapture");
    hip_check(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    (void)hipGraphDestroy(graph);
    pl->graphs[gkey] = (void*)gexec;
  }
  if (gexec) hip_check(hipGraphLaunch(gexec, st), "hipGraphLaunch");

  // ------------------------------------------------------------ results
  const int64_t leaves = (int64_t)t.parent[R - 1].size();
  std::vector<char> vals((size_t)leaves * eb);
  std::vector<int32_t> ex((size_t)leaves);
  hip_check(hipMemcpyAsync(vals.data(), dF[(R - 1) % 2], vals.size(), hipMemcpyDeviceToHost, st), "download");
  hip_check(hipMemcpyAsync(ex.data(), d_exp[(R - 1) % 2], ex.size() * 4, hipMemcpyDeviceToHost, st), "download");
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
  for (Timed& t : timed) {
    float ms = 0;
    hip_check(hipEventElapsedTime(&ms, t.a, t.b), "hipEventElapsedTime");
    pl->prof[t.cls].ms += ms;
    pl->prof[t.cls].launches += 1;
    pl->prof[t.cls].cmac += t.cmac;
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (size_t b = 0; b < n; ++b) {
    const int32_t leaf = t.leaf[b];
    double re, im;
    if (eb == 16) {
      const double* v = (const double*)vals.data();
      re = v[2 * leaf];
      im = v[2 * leaf + 1];
    } else {
      const float* v = (const float*)vals.data();
      re = v[2 * leaf];
      im = v[2 * leaf + 1];
    }
    int64_t e = ex[leaf];
    for (int i = 0; i < R; ++i)
      for (int j = 0; j < L; ++j) {
        const int tau = bits[b * nq + pl->cs[(size_t)i * L + j].qubit];
        e += pl->w[((size_t)i * L + j) * 2 + tau].exp2;
      }
    out[2 * b] = std::ldexp(re, (int)e);
    out[2 * b + 1] = std::ldexp(im, (int)e);
  }
}
