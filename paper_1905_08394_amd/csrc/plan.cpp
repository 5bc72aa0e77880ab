// Contraction planner for the generic row scheme (supplement S-II, eqs.
// S2-S6, Fig. S2(a)).
//
// Geometry.  The lattice is swept along its long side so the boundary has
// L = min(Lv, Lh) legs and the largest tensor has rank L+1 (S-II).  In the
// sweep frame, contraction row i / column j is site (i, j) with legs l, r, u,
// d; u/d point along the sweep.  Each site's projected tensor E = A[tau]
// (eq. 7) is stored as a K x N complex matrix W[(u, l)][(d, r)].
//
// Leg order ("rotating" layout).  The boundary after row i is stored as
// F_i[d_{L-1}][d_0 .. d_{L-2}].  Inside row i the leg v = u_{L-1} (the input
// leg the last site contracts) is held fixed as a batch index: it is not
// touched before the last site, so the row splits into independent
// per-v pieces (a cut loop over v, the "cut" technique of the conclusions),
// summed by the last site.  Per v the running tensor after site j is
//   G_j[u_{j+1} .. u_{L-2}][d_0 .. d_j][r_j],
// so every site is one complex GEMM (eq. S4) with no transposes:
//   C[m][(d_j, r_j)] = sum_{u_j, r_{j-1}} A[u_j][m][r_{j-1}] W[(u_j, l_j)][(d_j, r_j)],
// where K1 = u_j is the slowest leg of A and K2 = r_{j-1} the fastest.  Site
// 0 has K2 = 1 (A read K-major); the last site takes v itself as K1 and
// writes F_i transposed into the layout above, accumulating over v chunks in
// a fixed order.  Row 0 starts from the scalar 1 (all u legs have size 1);
// the last row has d legs of size 1 and ends in the scalar amplitude.
//
// Work count.  Each step costs M K1 K2 N complex multiply-adds per (node, v);
// the sum over the sweep is the exact count whose leading term is eq. (S8).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include <hip/hip_runtime_api.h>

#include "psim_internal.hpp"

namespace psim {

static int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

int64_t packed_ld(int prec, int64_t K) {
  (void)prec;
  return round_up(2 * K, 32) + 32;
}
int64_t packed_rows(int prec, int64_t N) {
  return prec == PSIM_FP32_3M ? round_up(N, 128) : round_up(2 * N, 256);
}

// Real expansion of a complex K x N matrix for the 4M scheme, stored
// transposed: P[n'][k'] = B'[k'][n'] with
//   B'[2k][2n] = Re W, B'[2k][2n+1] = Im W, B'[2k+1][2n] = -Im W, B'[2k+1][2n+1] = Re W,
// so that an interleaved complex row a (re, im, re, im, ...) times B' gives
// the interleaved complex row a W.  Zero padded to packed_rows x packed_ld.
void pack_site_matrix(int prec, const cd* W, int64_t K, int64_t N, std::vector<char>& out, int64_t& ld) {
  ld = packed_ld(prec, K);
  const int64_t rows = packed_rows(prec, N);
  if (prec == PSIM_FP32_3M) {
    // 3M: one row per complex column n, (Re, Im) of W[k][n] interleaved along k
    out.assign((size_t)(rows * ld) * sizeof(float), 0);
    float* P = reinterpret_cast<float*>(out.data());
    for (int64_t k = 0; k < K; ++k)
      for (int64_t n = 0; n < N; ++n) {
        const cd w = W[k * N + n];
        P[n * ld + 2 * k] = (float)w.real();
        P[n * ld + 2 * k + 1] = (float)w.imag();
      }
  } else if (prec == PSIM_FP64) {
    out.assign((size_t)(rows * ld) * sizeof(double), 0);
    double* P = reinterpret_cast<double*>(out.data());
    for (int64_t k = 0; k < K; ++k)
      for (int64_t n = 0; n < N; ++n) {
        const cd w = W[k * N + n];
        P[(2 * n) * ld + 2 * k] = w.real();
        P[(2 * n + 1) * ld + 2 * k] = w.imag();
        P[(2 * n) * ld + 2 * k + 1] = -w.imag();
        P[(2 * n + 1) * ld + 2 * k + 1] = w.real();
      }
  } else {
    out.assign((size_t)(rows * ld) * sizeof(float), 0);
    float* P = reinterpret_cast<float*>(out.data());
    for (int64_t k = 0; k < K; ++k)
      for (int64_t n = 0; n < N; ++n) {
        const cd w = W[k * N + n];
        const float re = (float)w.real(), im = (float)w.imag();  // round to nearest even
        P[(2 * n) * ld + 2 * k] = re;
        P[(2 * n + 1) * ld + 2 * k] = im;
        P[(2 * n) * ld + 2 * k + 1] = -im;
        P[(2 * n + 1) * ld + 2 * k + 1] = re;
      }
  }
}

// bfloat16 by round-to-nearest-even of an FP32 value (IEEE binary32 with the
// low 16 bits rounded away); NaN stays NaN.
static uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
static float bf16_to_float(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// BF16x3: the FP32 4M expansion split into hi = bf16(x) and lo = bf16(x - hi)
// planes, each stored like pack_site_matrix's FP32 layout (P[n'][k']).
void pack_site_matrix_bf16(const cd* W, int64_t K, int64_t N, std::vector<char>& out, int64_t& ld, int64_t& plane) {
  std::vector<char> f32;
  int64_t ld32 = 0;
  pack_site_matrix(PSIM_FP32_4M, W, K, N, f32, ld32);
  ld = ld32;
  const int64_t rows = packed_rows(PSIM_FP32_4M, N);
  plane = rows * ld;
  out.assign((size_t)(2 * plane) * 2, 0);
  const float* P = reinterpret_cast<const float*>(f32.data());
  uint16_t* H = reinterpret_cast<uint16_t*>(out.data());
  uint16_t* Lo = H + plane;
  for (int64_t x = 0; x < plane; ++x) {
    const uint16_t h = bf16_rne(P[x]);
    H[x] = h;
    Lo[x] = bf16_rne(P[x] - bf16_to_float(h));
  }
}

namespace {

// contraction-frame site (i, j) -> original site and leg sizes
void frame_sites(const psim_peps_t& P, int sweep, int R, int L, std::vector<CSite>& cs) {
  cs.resize((size_t)R * L);
  for (int i = 0; i < R; ++i)
    for (int j = 0; j < L; ++j) {
      CSite c;
      const int r = sweep == 1 ? i : j, col = sweep == 1 ? j : i;
      c.qubit = r * P.lh + col;
      const Site& s = P.sites[c.qubit];
      if (sweep == 1) {
        c.dl = s.dl; c.dr = s.dr; c.du = s.du; c.dd = s.dd;
      } else {  // columns: frame-u = left, frame-d = right, frame-l = up, frame-r = down
        c.dl = s.du; c.dr = s.dd; c.du = s.dl; c.dd = s.dr;
      }
      cs[(size_t)i * L + j] = c;
    }
}

// W[(u, l)][(d, r)] of the projected site in the sweep frame
void site_matrix(const psim_peps_t& P, int sweep, const CSite& c, int tau, std::vector<cd>& W) {
  const Site& s = P.sites[c.qubit];
  const int64_t K = (int64_t)c.du * c.dl, N = (int64_t)c.dd * c.dr;
  W.assign((size_t)(K * N), cd(0.0));
  for (int u = 0; u < c.du; ++u)
    for (int l = 0; l < c.dl; ++l)
      for (int d = 0; d < c.dd; ++d)
        for (int r = 0; r < c.dr; ++r) {
          // frame legs -> original legs
          const int ol = sweep == 1 ? l : u, orr = sweep == 1 ? r : d;
          const int ou = sweep == 1 ? u : l, od = sweep == 1 ? d : r;
          W[(size_t)((u * c.dl + l) * N + d * c.dr + r)] = s.t[s.at(tau, ol, orr, ou, od)];
        }
}

int exponent_of_max(const std::vector<cd>& W) {
  double mx = 0;
  for (const cd& w : W) mx = std::max(mx, std::max(std::abs(w.real()), std::abs(w.imag())));
  if (mx == 0) return 0;
  int e;
  std::frexp(mx, &e);  // mx = f 2^e, f in [0.5, 1)
  return e;
}

}  // namespace

}  // namespace psim

using namespace psim;

psim_plan_t* make_plan(const psim_peps_t* P, const psim_plan_opts* o) {
  if (!P) fail(PSIM_EINVAL, "peps is NULL");
  psim_plan_opts opts{};
  if (o) opts = *o;
  if (opts.prec != PSIM_FP64 && opts.prec != PSIM_FP32_4M && opts.prec != PSIM_FP32_3M && opts.prec != PSIM_BF16X3)
    fail(PSIM_EUNSUPPORTED, "precision " + std::to_string(opts.prec) + " is not available in this library");
  if (opts.mem_budget_bytes == 0) opts.mem_budget_bytes = 200ull << 30;
  if (opts.max_batch <= 0) opts.max_batch = 1;
  if (opts.tile_cfg < 0 || opts.tile_cfg >= config_count(opts.prec))
    fail(PSIM_EINVAL, "tile_cfg " + std::to_string(opts.tile_cfg) + " is not a candidate of this precision");
  // the split-accumulation kernels come in one tile configuration (FP32 3M: two)
  if ((opts.flags & PSIM_PLAN_SPLIT_ACC) && !split_candidate(opts.prec, opts.tile_cfg))
    fail(PSIM_EINVAL, "tile_cfg " + std::to_string(opts.tile_cfg) + " has no split-accumulation form");
  int sweep = opts.sweep;
  if (sweep == 0) sweep = (P->lh <= P->lv) ? 1 : 2;
  if (sweep < 1 || sweep > 3) fail(PSIM_EINVAL, "sweep must be 0, 1, 2 or 3");
  if (sweep == 3) {  // square partition (square.cpp)
    auto* pl = new psim_plan_t();
    try {
      pl->opts = opts;
      pl->lv = P->lv;
      pl->lh = P->lh;
      pl->sweep = 3;
      pl->R = P->lv;
      pl->L = P->lh;
      pl->host_only = (opts.flags & PSIM_PLAN_HOST_ONLY) != 0;
      pl->elem_bytes = opts.prec == PSIM_FP64 ? 16 : 8;
      pl->chi = 1;
      for (const Site& s : P->sites) pl->chi = std::max({pl->chi, s.dl, s.dr, s.du, s.dd});
      if (!pl->host_only) hip_check(hipSetDevice(opts.device), "hipSetDevice");
      make_square_plan(pl, *P);
      if (!pl->host_only) {
        hip_check(hipMalloc(&pl->d_ones, 16), "hipMalloc(ones)");
        launch_fill_ones(opts.prec, pl->d_ones, nullptr);
        hip_check(hipDeviceSynchronize(), "fill ones");
      }
    } catch (...) {
      if (pl->d_ones) (void)hipFree(pl->d_ones);
      delete pl;
      throw;
    }
    return pl;
  }

  auto* pl = new psim_plan_t();
  try {
    pl->opts = opts;
    pl->lv = P->lv;
    pl->lh = P->lh;
    pl->sweep = sweep;
    pl->R = sweep == 1 ? P->lv : P->lh;
    pl->L = sweep == 1 ? P->lh : P->lv;
    pl->host_only = (opts.flags & PSIM_PLAN_HOST_ONLY) != 0;
    pl->elem_bytes = opts.prec == PSIM_FP64 ? 16 : 8;
    const int R = pl->R, L = pl->L;
    if (L > 64) fail(PSIM_EUNSUPPORTED, "boundary wider than 64 sites");
    frame_sites(*P, sweep, R, L, pl->cs);
    pl->chi = 1;
    for (const Site& s : P->sites) pl->chi = std::max({pl->chi, s.dl, s.dr, s.du, s.dd});

    // ---------------------------------------------------------- steps
    auto cs = [&](int i, int j) -> const CSite& { return pl->cs[(size_t)i * L + j]; };
    pl->levels.resize(R);
    pl->steps.resize((size_t)R * L);
    double cmac = 0;
    int64_t peak = 1;
    for (int i = 0; i < R; ++i) {
      Level& lev = pl->levels[i];
      lev.Dv = cs(i, L - 1).du;
      int64_t F = 1;
      for (int j = 0; j < L; ++j) F *= cs(i, j).dd;
      lev.F_elems = F;
      for (int j = 0; j < L; ++j) {
        Step& st = pl->steps[(size_t)i * L + j];
        st.i = i;
        st.j = j;
        const CSite& c = cs(i, j);
        if (j == L - 1) {
          st.kind = 2;
          st.K1 = lev.Dv;
          st.K2 = c.dl;
          int64_t M = 1;
          for (int jj = 0; jj < L - 1; ++jj) M *= cs(i, jj).dd;
          st.M = M;
          st.N = (int64_t)c.dd * c.dr;
          if (c.dr != 1) fail(PSIM_EINTERNAL, "last site with an open right leg");
          cmac += (double)st.M * st.K1 * st.K2 * st.N;
        } else {
          st.kind = j == 0 ? 0 : 1;
          st.K1 = c.du;
          st.K2 = c.dl;
          int64_t M = 1;
          for (int jj = j + 1; jj <= L - 2; ++jj) M *= cs(i, jj).du;
          for (int jj = 0; jj < j; ++jj) M *= cs(i, jj).dd;
          st.M = M;
          st.N = (int64_t)c.dd * c.dr;
          st.g_out = st.M * st.N;
          st.cfg = opts.tile_cfg;
          lev.Gmax = std::max(lev.Gmax, st.g_out);
          if (!(i == 0 && j == 0)) cmac += (double)lev.Dv * st.M * st.K1 * st.K2 * st.N;
        }
      }
      peak = std::max({peak, lev.F_elems, lev.Gmax * lev.Dv});
      // most distinct prefixes (nodes) at this level
      const double cap = std::ldexp(1.0, std::min(62, (i + 1) * L));
      lev.nmax = (int64_t)std::min<double>(opts.max_batch, cap);
    }
    pl->cmac = cmac;
    pl->peak_elems = peak;

    // ---------------------------------------------------------- memory plan
    // Workspace = tables + two boundary buffers (even / odd levels) + two
    // intermediate buffers (ping-pong inside a row).  Per level i the plan
    // fixes: vchunk (v values per pass), group (nodes per pass) and cap
    // (nodes whose boundary can be held); batches whose prefix trie exceeds a
    // cap are split by the scheduler.  Passes are sized toward kParElems
    // elements per intermediate buffer, enough work to fill the GPU.
    const uint64_t eb = pl->elem_bytes;
    const uint64_t budget = opts.mem_budget_bytes;
    const uint64_t kParElems = 1ull << 31;
    // rows whose per-v intermediate exceeds this many elements are cut over
    // the first output leg w as well (intermediates of D^(L-1) per (v, w))
    const uint64_t kWCutElems = 1ull << 29;
    auto al = [](uint64_t x) { return (x + 255) / 256 * 256; };
    int64_t nmax_all = 1;
    uint64_t tab = 0;
    uint64_t Fmin[2] = {0, 0};
    for (int i = 0; i < R; ++i) {
      const Level& lev = pl->levels[i];
      nmax_all = std::max(nmax_all, lev.nmax);
      tab += al((uint64_t)lev.nmax * 4) + al((uint64_t)lev.nmax * L);
      Fmin[i % 2] = std::max(Fmin[i % 2], al((uint64_t)lev.F_elems * eb));
    }
    tab += 3 * al((uint64_t)nmax_all * 4);  // exponents (two levels) and row maxima
    pl->ws_tab = tab;
    if (tab + Fmin[0] + Fmin[1] > budget)
      fail(PSIM_ENOMEM, "plan needs at least " + std::to_string(tab + Fmin[0] + Fmin[1]) +
                            " bytes for boundaries; budget is " + std::to_string(budget));
    const uint64_t gbud = budget - tab - Fmin[0] - Fmin[1];
    uint64_t G = 0;
    for (int i = 0; i < R; ++i) {
      Level& lev = pl->levels[i];
      if (L == 1 || lev.Gmax == 0) {
        lev.vchunk = lev.Dv;
        lev.group = (int)std::min<int64_t>(lev.nmax, 1 << 16);
        continue;
      }
      const int64_t K2 = cs(i, L - 1).dl;
      // keep the last site's packed-matrix offset 16-byte aligned
      auto v_ok = [&](int cand) { return lev.Dv % cand == 0 && (cand == lev.Dv || ((int64_t)cand * K2) % 2 == 0); };
      // per-(node, v, w) intermediates of a row cut over w as well (w = d of
      // the first site, held fixed from its creation to the end of the row)
      lev.Dw = cs(i, 0).dd;
      lev.Gtask = 0;
      for (int j = 0; j < L - 1; ++j) {
        const Step& st = pl->steps[(size_t)i * L + j];
        const int64_t t = j == 0 ? st.M * cs(i, 0).dr : st.M / lev.Dw * st.N;
        lev.Gtask = std::max(lev.Gtask, t);
      }
      const bool cut_w = lev.Dw > 1 && (lev.Gmax > kWCutElems || 2ull * lev.Gmax * eb > gbud);
      if (!cut_w) {
        const uint64_t per = 2ull * lev.Gmax * eb;  // ping-pong, one (node, v)
        const uint64_t par = std::max<uint64_t>(kParElems, lev.Gmax);
        int c = 0;
        for (int cand = lev.Dv; cand >= 1; --cand)
          if (v_ok(cand) && (uint64_t)cand * per <= gbud && (uint64_t)cand * lev.Gmax <= par) { c = cand; break; }
        if (c == 0)
          fail(PSIM_ENOMEM, "plan needs at least " + std::to_string(tab + Fmin[0] + Fmin[1] + per) + " bytes (row " +
                                std::to_string(i) + "); budget is " + std::to_string(budget));
        lev.vchunk = c;
        lev.wchunk = lev.Dw;
        uint64_t g = std::max<uint64_t>(1, par / ((uint64_t)c * lev.Gmax));
        g = std::min<uint64_t>({g, (uint64_t)lev.nmax, gbud / ((uint64_t)c * per), 1u << 16});
        lev.group = (int)std::max<uint64_t>(g, 1);
        G = std::max(G, 2 * al((uint64_t)lev.group * c * lev.Gmax * eb));
        continue;
      }
      // cut over w: (v, w) pairs per pass up to `target` elements per buffer,
      // v chunk first (fewer accumulation passes of the last site), leaving
      // room for at least two w values when possible
      const uint64_t task = (uint64_t)lev.Gtask;
      const uint64_t target = std::min<uint64_t>(std::max<uint64_t>(kWCutElems, task), gbud / (2 * eb));
      int c = 0;
      for (int cand = lev.Dv; cand >= 1 && !c; --cand)
        if (v_ok(cand) && 2 * cand * task <= target) c = cand;
      for (int cand = lev.Dv; cand >= 1 && !c; --cand)
        if (v_ok(cand) && cand * task <= target) c = cand;
      if (c == 0)
        fail(PSIM_ENOMEM, "plan needs at least " + std::to_string(tab + Fmin[0] + Fmin[1] + 2 * task * eb) +
                              " bytes (row " + std::to_string(i) + ", cut over v and w); budget is " +
                              std::to_string(budget));
      int cw = 1;
      for (int cand = lev.Dw - 1; cand >= 1; --cand)
        if (lev.Dw % cand == 0 && (uint64_t)c * cand * task <= target) { cw = cand; break; }
      lev.vchunk = c;
      lev.wchunk = cw;
      uint64_t g = std::max<uint64_t>(1, target / ((uint64_t)c * cw * task));
      g = std::min<uint64_t>({g, (uint64_t)lev.nmax, 1u << 16});
      lev.group = (int)std::max<uint64_t>(g, 1);
      G = std::max(G, 2 * al((uint64_t)lev.group * c * cw * task * eb));
    }
    // boundaries: what is left, split between even and odd levels
    if (tab + G + Fmin[0] + Fmin[1] > budget)
      fail(PSIM_ENOMEM, "plan needs at least " + std::to_string(tab + G + Fmin[0] + Fmin[1]) +
                            " bytes; budget is " + std::to_string(budget));
    const uint64_t rest = budget - tab - G;
    const uint64_t spare = rest - Fmin[0] - Fmin[1];
    uint64_t Fb[2] = {0, 0};
    for (int par = 0; par < 2; ++par) {
      const uint64_t avail = par == 0 ? Fmin[0] + spare / 2 : rest - Fb[0];
      for (int i = par; i < R; i += 2) {
        Level& lev = pl->levels[i];
        const uint64_t one = al((uint64_t)lev.F_elems * eb);
        lev.cap = (int64_t)std::min<uint64_t>((uint64_t)lev.nmax, std::max<uint64_t>(1, avail / one));
        Fb[par] = std::max(Fb[par], al((uint64_t)lev.cap * lev.F_elems * eb));
      }
    }
    for (int i = 0; i < R; ++i) {
      Level& lev = pl->levels[i];
      lev.group = (int)std::min<int64_t>(lev.group, lev.cap);
      lev.F_off = (i % 2) ? Fb[0] : 0;
    }
    // device operations per sub-batch: per level, every node group runs L
    // site contractions per v chunk, then one rescale
    pl->max_ops = 0;
    for (int i = 0; i < R; ++i) {
      const Level& lev = pl->levels[i];
      const int64_t groups = (lev.cap + lev.group - 1) / lev.group;
      const int64_t chunks = L == 1 ? 1 : (lev.Dv + lev.vchunk - 1) / lev.vchunk;
      const int64_t wchunks = w_cut(lev) ? lev.Dw / lev.wchunk : 1;
      pl->max_ops += groups * chunks * wchunks * L + 1;
    }
    pl->ws_F = Fb[0] + Fb[1];
    pl->ws_G = G;
    pl->ws_total = pl->ws_tab + pl->ws_F + pl->ws_G + 256;
    if (pl->ws_total > budget + 256) fail(PSIM_EINTERNAL, "memory plan exceeds its budget");

    // ---------------------------------------------------------- stored tile choices
    // psim_tune's earlier measurements (PSIM_TUNE_CACHE) for these interior
    // shapes on this device architecture; an explicit tile_cfg wins
    if (!pl->host_only && opts.tile_cfg == 0 && std::getenv("PSIM_TUNE_CACHE")) {
      const bool split = (opts.flags & PSIM_PLAN_SPLIT_ACC) != 0;
      const std::string arch = device_arch(opts.device);
      for (Step& st : pl->steps) {
        if (st.kind != 1) continue;
        int cfg = 0;
        const Level& lv_ = pl->levels[st.i];
        if (tune_cache_lookup(tune_key(arch, opts.prec, interior_rows(lv_, st), st.K1, st.K2, st.N, interior_batch(lv_),
                                       split),
                              &cfg) &&
            cfg >= 0 && cfg < config_count(opts.prec) && (!split || split_candidate(opts.prec, cfg)))
          st.cfg = cfg;
      }
    }

    // ---------------------------------------------------------- pack + upload
    pl->w.resize((size_t)R * L * 2);
    std::vector<cd> W;
    std::vector<char> buf;
    for (int i = 0; i < R; ++i)
      for (int j = 0; j < L; ++j) {
        const CSite& c = cs(i, j);
        for (int tau = 0; tau < 2; ++tau) {
          DevMatrix& dm = pl->w[((size_t)i * L + j) * 2 + tau];
          site_matrix(*P, sweep, c, tau, W);
          dm.exp2 = exponent_of_max(W);
          const double sc = std::ldexp(1.0, -dm.exp2);  // exact power of two
          for (cd& x : W) x *= sc;
          // the last site of a row always runs the 4M transposed-store kernel
          // in FP32 plans (its 256 x 64 tile suits the few output columns)
          const bool last = (j == L - 1);
          const int pack_prec =
              (opts.prec == PSIM_BF16X3 || (opts.prec == PSIM_FP32_3M && last)) ? PSIM_FP32_4M : opts.prec;
          pack_site_matrix(pack_prec, W.data(), (int64_t)c.du * c.dl, (int64_t)c.dd * c.dr, buf, dm.ld);
          // a row cut over w reads the first site's matrix from an offset
          // (the columns of one w chunk): 256 zero rows keep the last
          // chunk's full tiles inside the allocation
          if (j == 0) buf.resize(buf.size() + (size_t)256 * dm.ld * (opts.prec == PSIM_FP64 ? 8 : 4), 0);
          pl->weights_bytes += buf.size();
          if (!pl->host_only) {
            hip_check(hipSetDevice(opts.device), "hipSetDevice");
            hip_check(hipMalloc(&dm.ptr, buf.size()), "hipMalloc(site matrix)");
            hip_check(hipMemcpy(dm.ptr, buf.data(), buf.size(), hipMemcpyHostToDevice), "hipMemcpy(site matrix)");
          }
          if (opts.prec == PSIM_BF16X3) {  // interior sites also get the split planes
            pack_site_matrix_bf16(W.data(), (int64_t)c.du * c.dl, (int64_t)c.dd * c.dr, buf, dm.ld_b, dm.plane_b);
            pl->weights_bytes += buf.size();
            if (!pl->host_only) {
              hip_check(hipMalloc(&dm.ptr_b, buf.size()), "hipMalloc(site matrix)");
              hip_check(hipMemcpy(dm.ptr_b, buf.data(), buf.size(), hipMemcpyHostToDevice), "hipMemcpy(site matrix)");
            }
          }
        }
      }
    if (!pl->host_only) {
      hip_check(hipMalloc(&pl->d_ones, 16), "hipMalloc(ones)");
      launch_fill_ones(opts.prec, pl->d_ones, nullptr);
      hip_check(hipDeviceSynchronize(), "fill ones");
    }
  } catch (...) {
    for (auto& dm : pl->w) {
      if (dm.ptr) (void)hipFree(dm.ptr);
      if (dm.ptr_b) (void)hipFree(dm.ptr_b);
    }
    if (pl->d_ones) (void)hipFree(pl->d_ones);
    delete pl;
    throw;
  }
  return pl;
}

void free_plan(psim_plan_t* pl) {
  if (!pl) return;
  for (auto& kv : pl->graphs) (void)hipGraphExecDestroy((hipGraphExec_t)kv.second);
  if (pl->cap_stream) (void)hipStreamDestroy((hipStream_t)pl->cap_stream);
  for (auto& dm : pl->w) {
    if (dm.ptr) (void)hipFree(dm.ptr);
    if (dm.ptr_b) (void)hipFree(dm.ptr_b);
  }
  if (pl->d_ones) (void)hipFree(pl->d_ones);
  delete pl;
}
