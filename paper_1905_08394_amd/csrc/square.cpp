// Square partition (supplement S-II, Fig. S2(b); eqs. S9-S10 for an L x L
// lattice with L even, S11-S12 for L odd), for any Lv x Lh lattice with both
// sides at least 2.
//
// The lattice is cut into four blocks ("quadrants") by the middle horizontal
// cut (a = floor(Lv/2) rows above it) and the middle vertical cut (b =
// floor(Lh/2) columns left of it).  Each quadrant is contracted on its own
// from its lattice corner inward; what is left open are the bonds it shares
// with the two neighbouring quadrants.  The four quadrant tensors are then
// joined, each join being one complex GEMM (for L x L, L even, both joins are
// D^(L/2) x D^(L/2) x D^(L/2): the leading term 2 D^(3L/2) of eq. S10; for L
// odd the two joins are D^((L+1)/2) x D^((L-1)/2) x D^((L-1)/2) and
// D^((L+1)/2) x D^((L-1)/2) x D^((L+1)/2), whose sum is eq. S12):
//   T[vUR][vUL] = sum_hU   Q_UR[vUR][hU]  Q_UL[vUL][hU]
//   Y[vUR][hL]  = sum_vUL  T[vUR][vUL]    Q_LL[hL][vUL]
//   <tau|psi>   = sum      Y[vUR][hL]     Q_LR[vUR][hL].
// Bitstrings that agree on the upper half share T, those that also agree on
// the lower-left quadrant share Y (the reuse of the fast-sampling remark).
//
// Quadrant frames.  Quadrant q (nr x nc sites) is walked in a frame (i, j)
// that
// starts at its lattice corner: rows are mirrored for the lower quadrants
// (bottom-up) and columns for the right ones (right to left), with the legs
// l/r and u/d swapped accordingly.  Frame row 0 lies on the lattice edge and
// frame column 0 too, so their u and l legs have size 1; the frame-r legs of
// column nc-1 (o_i) and the frame-d legs of row nr-1 stay open.
//
// Leg order inside a quadrant.  Before frame row i the running tensor is
//   [u_0 .. u_{nc-1}][o_0 .. o_{i-1}]   (u_j = frame-d leg of site (i-1, j)),
// and site j of the row is one GEMM of the row scheme's rotating layout,
//   C[m][(d_j, r_j)] = sum_{u_j, r_{j-1}} A[u_j][m][r_{j-1}] W[(u_j, l_j)][(d_j, r_j)],
// with m = [u_{j+1} .. u_{nc-1}][o_0 .. o_{i-1}][d_0 .. d_{j-1}] untouched.
// After the row the tensor is [o_0 .. o_{i-1}][d_0 .. d_{nc-1}][o_i]; one
// permute brings it to [d ...][o_0 .. o_i] for the next row.  The finished
// quadrant is stored as [d ...][o ...] (UL, UR, LR) or [o ...][d ...] (LL),
// the layouts the joins read (a quadrant tensor Q[n][k] is the packed W
// operand of W[k][n] = Q[n][k]).
//
// Every tensor is rescaled by an exact power of two after each row and each
// join; the exponents are summed on the host in FP64 with the site-matrix
// exponents.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>

#include <hip/hip_runtime_api.h>

#include "psim_internal.hpp"

namespace psim {

struct SqSite {
  int qubit = 0;
  int dl = 1, dr = 1, du = 1, dd = 1;  // frame leg sizes
  DevMatrix w[2];                       // packed W[(u, l)][(d, r)] for tau = 0, 1
};

struct SqQuad {
  int mr = 0, mc = 0;          // mirrored rows / columns
  int nr = 1, nc = 1;          // frame rows / columns
  std::vector<SqSite> s;       // frame (i, j) at i * nc + j
  int64_t dv = 1, dh = 1;      // sizes of the open vertical-cut / horizontal-cut legs
  double cmac = 0;
};

struct SquarePlan {
  int lv = 0, lh = 0;
  SqQuad q[4];                 // UL, UR, LL, LR
  int64_t tmax = 1;            // largest running tensor (complex elements)
  int64_t qmax = 1;            // largest quadrant / joined tensor
  int64_t prow[2] = {0, 0}, pld[2] = {0, 0};  // packed operands of the two joins
  uint64_t off_w1 = 0, off_w2 = 0, off_a = 0, off_b = 0, off_c = 0, off_p = 0, off_small = 0, off_y = 0;
  int ycap = 1;                // Y tensors held at once (lower-left patterns joined per pass)
  double cmac_quads = 0, cmac_joins = 0;
  int64_t n_steps = 0;
  ~SquarePlan() {
    for (auto& qd : q)
      for (auto& st : qd.s)
        for (auto& w : st.w)
          if (w.ptr) (void)hipFree(w.ptr);
  }
};

namespace {

int exponent_of_max_sq(const std::vector<cd>& W) {
  double mx = 0;
  for (const cd& w : W) mx = std::max(mx, std::max(std::abs(w.real()), std::abs(w.imag())));
  if (mx == 0) return 0;
  int e;
  std::frexp(mx, &e);
  return e;
}

// Running-tensor shapes of frame site (i, j): M, K1, K2, N as in the header.
struct Shape {
  int64_t M, K1, K2, N;
};

Shape site_shape(const SqQuad& Q, int i, int j) {
  const int nc = Q.nc;
  auto at = [&](int a, int b) -> const SqSite& { return Q.s[(size_t)a * nc + b]; };
  Shape sh;
  sh.K1 = at(i, j).du;
  sh.K2 = at(i, j).dl;
  sh.N = (int64_t)at(i, j).dd * at(i, j).dr;
  int64_t M = 1;
  for (int jj = j + 1; jj < nc; ++jj) M *= at(i, jj).du;
  for (int k = 0; k < i; ++k) M *= at(k, nc - 1).dr;
  for (int jj = 0; jj < j; ++jj) M *= at(i, jj).dd;
  sh.M = M;
  return sh;
}

}  // namespace

void make_square_plan(psim_plan_t* pl, const psim_peps_t& P) {
  const int Lv = P.lv, Lh = P.lh;
  if (Lv < 2 || Lh < 2) fail(PSIM_EUNSUPPORTED, "the square partition needs at least 2 rows and 2 columns");
  const int prec = pl->opts.prec;
  if (prec == PSIM_BF16X3) fail(PSIM_EUNSUPPORTED, "the square partition runs in FP64, FP32 4M or FP32 3M");
  auto sq = std::make_shared<SquarePlan>();
  sq->lv = Lv;
  sq->lh = Lh;
  const int a = Lv / 2, b = Lh / 2;  // rows above / columns left of the cuts
  const int mirror[4][2] = {{0, 0}, {0, 1}, {1, 0}, {1, 1}};
  for (int qi = 0; qi < 4; ++qi) {
    SqQuad& Q = sq->q[qi];
    Q.mr = mirror[qi][0];
    Q.mc = mirror[qi][1];
    Q.nr = Q.mr ? Lv - a : a;
    Q.nc = Q.mc ? Lh - b : b;
    const int nr = Q.nr, nc = Q.nc;
    Q.s.resize((size_t)nr * nc);
    for (int i = 0; i < nr; ++i)
      for (int j = 0; j < nc; ++j) {
        const int r = Q.mr ? Lv - 1 - i : i, c = Q.mc ? Lh - 1 - j : j;
        SqSite& st = Q.s[(size_t)i * nc + j];
        st.qubit = r * Lh + c;
        const Site& s = P.sites[st.qubit];
        st.dl = Q.mc ? s.dr : s.dl;
        st.dr = Q.mc ? s.dl : s.dr;
        st.du = Q.mr ? s.dd : s.du;
        st.dd = Q.mr ? s.du : s.dd;
      }
    for (int j = 0; j < nc; ++j) Q.dv *= Q.s[(size_t)(nr - 1) * nc + j].dd;
    for (int i = 0; i < nr; ++i) Q.dh *= Q.s[(size_t)i * nc + nc - 1].dr;
    for (int i = 0; i < nr; ++i)
      for (int j = 0; j < nc; ++j) {
        const Shape sh = site_shape(Q, i, j);
        Q.cmac += (double)sh.M * sh.K1 * sh.K2 * sh.N;
        sq->tmax = std::max({sq->tmax, sh.M * sh.K1 * sh.K2, sh.M * sh.N});
        ++sq->n_steps;
      }
    sq->qmax = std::max(sq->qmax, Q.dv * Q.dh);
    sq->cmac_quads += Q.cmac;
  }
  const int64_t vUL = sq->q[0].dv, vUR = sq->q[1].dv, hU = sq->q[0].dh, hL = sq->q[2].dh;
  if (sq->q[1].dh != hU || sq->q[2].dv != vUL || sq->q[3].dv != vUR || sq->q[3].dh != hL)
    fail(PSIM_EINTERNAL, "quadrant cut legs do not match");
  sq->qmax = std::max({sq->qmax, vUR * vUL, vUR * hL});
  sq->cmac_joins = (double)vUR * hU * vUL + (double)vUR * vUL * hL + (double)vUR * hL;
  sq->n_steps += 2;
  // packed W operands: join 1 reads Q_UL as (N = vUL) x (K = hU), join 2 reads Q_LL as (N = hL) x (K = vUL)
  sq->prow[0] = packed_rows(prec, vUL);
  sq->pld[0] = packed_ld(prec, hU);
  sq->prow[1] = packed_rows(prec, hL);
  sq->pld[1] = packed_ld(prec, vUL);

  // ---------------------------------------------------------- workspace
  const uint64_t eb = pl->elem_bytes;  // bytes per complex element
  const uint64_t rb = eb / 2;          // bytes per real
  auto al = [](uint64_t x) { return (x + 255) / 256 * 256; };
  uint64_t off = 0;
  sq->off_w1 = off; off += al((uint64_t)sq->tmax * eb);
  sq->off_w2 = off; off += al((uint64_t)sq->tmax * eb);
  sq->off_a = off; off += al((uint64_t)sq->qmax * eb);
  sq->off_b = off; off += al((uint64_t)sq->qmax * eb);
  sq->off_c = off; off += al((uint64_t)sq->qmax * eb);
  sq->off_p = off;
  off += al((uint64_t)std::max(sq->prow[0] * sq->pld[0], sq->prow[1] * sq->pld[1]) * rb);
  sq->off_small = off;
  off += al(16 + (uint64_t)cdot_blocks() * 16);
  // more Y tensors (one per lower-left pattern of a pass) from what the
  // budget leaves, so each lower-right quadrant is contracted once per pass
  sq->off_y = off;
  const uint64_t ysz = al((uint64_t)sq->qmax * eb);
  const uint64_t budget = pl->opts.mem_budget_bytes;
  uint64_t extra = budget > off + 256 ? (budget - off - 256) / ysz : 0;
  extra = std::min<uint64_t>({extra, 15, (uint64_t)std::max(pl->opts.max_batch, 1) - 1});
  sq->ycap = 1 + (int)extra;
  off += extra * ysz;
  pl->ws_total = off + 256;
  if (pl->ws_total > pl->opts.mem_budget_bytes)
    fail(PSIM_ENOMEM, "square partition needs " + std::to_string(pl->ws_total) + " bytes; budget is " +
                          std::to_string(pl->opts.mem_budget_bytes));
  pl->peak_elems = std::max(sq->tmax, sq->qmax);
  pl->cmac = sq->cmac_quads + sq->cmac_joins;

  // ---------------------------------------------------------- site matrices
  std::vector<cd> W;
  std::vector<char> buf;
  for (auto& Q : sq->q)
    for (auto& st : Q.s) {
      const Site& s = P.sites[st.qubit];
      const int64_t K = (int64_t)st.du * st.dl, N = (int64_t)st.dd * st.dr;
      for (int tau = 0; tau < 2; ++tau) {
        W.assign((size_t)(K * N), cd(0.0));
        for (int u = 0; u < st.du; ++u)
          for (int l = 0; l < st.dl; ++l)
            for (int d = 0; d < st.dd; ++d)
              for (int r = 0; r < st.dr; ++r) {
                const int ol = Q.mc ? r : l, orr = Q.mc ? l : r;
                const int ou = Q.mr ? d : u, od = Q.mr ? u : d;
                W[(size_t)((u * st.dl + l) * N + d * st.dr + r)] = s.t[s.at(tau, ol, orr, ou, od)];
              }
        DevMatrix& dm = st.w[tau];
        dm.exp2 = exponent_of_max_sq(W);
        const double sc = std::ldexp(1.0, -dm.exp2);
        for (cd& x : W) x *= sc;
        pack_site_matrix(prec, W.data(), K, N, buf, dm.ld);
        pl->weights_bytes += buf.size();
        if (!pl->host_only) {
          hip_check(hipMalloc(&dm.ptr, buf.size()), "hipMalloc(site matrix)");
          hip_check(hipMemcpy(dm.ptr, buf.data(), buf.size(), hipMemcpyHostToDevice), "hipMemcpy(site matrix)");
        }
      }
    }
  pl->sq = sq;
  pl->sq_steps = sq->n_steps;
}

namespace {

struct SqRun {
  const psim_plan_t* pl;
  const SquarePlan* sq;
  hipStream_t st;
  char* base;
  int prec;
  uint64_t eb;
  int32_t* d_zero;
  int32_t* d_e;
  uint32_t* d_mx;
  double* d_part;
  // optional event timing (psim_profile): class 0 quadrant site contractions,
  // 1 joins, 2 permutes / packing / inner products, 3 rescales
  struct Timed {
    hipEvent_t a, b;
    int cls;
    double cmac, bytes;
  };
  std::vector<Timed> timed;
  bool profile = false;

  char* buf(uint64_t off) const { return base + off; }

  template <typename F>
  void run(int cls, double cmac, double bytes, F&& f) {
    if (!profile) {
      f();
      return;
    }
    Timed t{};
    t.cls = cls;
    t.cmac = cmac;
    t.bytes = bytes;
    hip_check(hipEventCreate(&t.a), "hipEventCreate");
    hip_check(hipEventCreate(&t.b), "hipEventCreate");
    hip_check(hipEventRecord(t.a, st), "hipEventRecord");
    f();
    hip_check(hipEventRecord(t.b, st), "hipEventRecord");
    timed.push_back(t);
  }

  void collect(psim_plan_t* p) {
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    for (Timed& t : timed) {
      float ms = 0;
      hip_check(hipEventElapsedTime(&ms, t.a, t.b), "hipEventElapsedTime");
      p->prof[t.cls].ms += ms;
      p->prof[t.cls].launches += 1;
      p->prof[t.cls].cmac += t.cmac;
      p->prof[t.cls].bytes += t.bytes;
      (void)hipEventDestroy(t.a);
      (void)hipEventDestroy(t.b);
    }
    timed.clear();
  }

  // exact power-of-two rescale of one tensor; returns the exponent taken out
  int64_t rescale(void* T, int64_t elems) {
    run(3, 0, 3.0 * eb * elems, [&] { launch_rowscale(prec, T, elems, 1, d_zero, d_zero, d_e, d_mx, st); });
    int32_t e = 0;
    hip_check(hipMemcpyAsync(&e, d_e, 4, hipMemcpyDeviceToHost, st), "download exponent");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    return e;
  }

  // Contract quadrant qi for bits into dst; returns its exponent.
  int64_t quad(int qi, const uint8_t* bits, char* dst) {
    const SqQuad& Q = sq->q[qi];
    const int nr = Q.nr, nc = Q.nc;
    char* cur = buf(sq->off_w1);
    char* nxt = buf(sq->off_w2);
    int64_t e = 0;
    int64_t cur_elems = 1;
    for (int i = 0; i < nr; ++i) {
      for (int j = 0; j < nc; ++j) {
        const SqSite& st_ = Q.s[(size_t)i * nc + j];
        const int tau = bits[st_.qubit];
        const DevMatrix& w = st_.w[tau];
        const Shape sh = site_shape(Q, i, j);
        GemmLaunch g;
        g.prec = prec;
        g.A = (i == 0 && j == 0) ? pl->d_ones : (const void*)cur;
        g.C = nxt;
        g.W0 = g.W1 = w.ptr;
        g.ldw = w.ld;
        g.M = sh.M;
        g.K1 = sh.K1;
        g.K2 = sh.K2;
        g.N = sh.N;
        g.nodes = 1;
        g.Bz = 1;
        g.sA_node = sh.K1 * sh.M * sh.K2;
        g.sC_node = sh.M * sh.N;
        run(0, (double)sh.M * sh.K1 * sh.K2 * sh.N, (double)eb * (sh.M * sh.K1 * sh.K2 + sh.M * sh.N),
            [&] { launch_site_gemm(g, st); });
        e += w.exp2;
        std::swap(cur, nxt);
        cur_elems = sh.M * sh.N;
      }
      e += rescale(cur, cur_elems);
      // [o_0 .. o_{i-1}][d_0 .. d_{h-1}][o_i] -> next layout
      int64_t X = 1, Y = 1;
      for (int k = 0; k < i; ++k) X *= Q.s[(size_t)k * nc + nc - 1].dr;
      for (int j = 0; j < nc; ++j) Y *= Q.s[(size_t)i * nc + j].dd;
      const int64_t Z = Q.s[(size_t)i * nc + nc - 1].dr;
      if (i + 1 < nr) {
        if (X > 1) {
          run(2, 0, 2.0 * eb * X * Y * Z, [&] { launch_permute3(prec, cur, nxt, X, Y, Z, 0, st); });
          std::swap(cur, nxt);
        }
      } else {
        run(2, 0, 2.0 * eb * X * Y * Z, [&] { launch_permute3(prec, cur, dst, X, Y, Z, qi == 2 ? 1 : 0, st); });
      }
    }
    return e;
  }

  void gemm(const void* A, int64_t M, int64_t K, const void* P, int64_t ld, int64_t N, void* C) {
    GemmLaunch g;
    g.prec = prec;
    g.A = A;
    g.C = C;
    g.W0 = g.W1 = P;
    g.ldw = ld;
    g.M = M;
    g.K1 = 1;
    g.K2 = K;
    g.N = N;
    g.nodes = 1;
    g.Bz = 1;
    g.sA_node = M * K;
    g.sC_node = M * N;
    run(1, (double)M * K * N, (double)eb * (M * K + K * N + M * N), [&] { launch_site_gemm(g, st); });
  }
  void pack(const void* Q, void* P, int64_t N, int64_t K, int64_t rows, int64_t ld) {
    run(2, 0, (double)eb * N * K + (double)(eb / 2) * rows * ld, [&] { launch_pack_w(prec, Q, P, N, K, rows, ld, st); });
  }
};

}  // namespace

void run_square(psim_plan_t* pl, const uint8_t* bits, size_t n, void* ws, void* stream, double* out) {
  const SquarePlan* sq = pl->sq.get();
  const int nq = sq->lv * sq->lh;
  hip_check(hipSetDevice(pl->opts.device), "hipSetDevice");
  SqRun R;
  R.pl = pl;
  R.sq = sq;
  R.st = (hipStream_t)stream;
  R.base = (char*)(((uintptr_t)ws + 255) / 256 * 256);
  R.profile = pl->profile;
  R.prec = pl->opts.prec;
  R.eb = pl->elem_bytes;
  char* small = R.buf(sq->off_small);
  R.d_zero = (int32_t*)small;
  R.d_e = (int32_t*)(small + 4);
  R.d_mx = (uint32_t*)(small + 8);
  R.d_part = (double*)(small + 16);
  static const int32_t zero = 0;
  hip_check(hipMemcpyAsync(R.d_zero, &zero, 4, hipMemcpyHostToDevice, R.st), "upload zero");

  // key of a bitstring: the bits of UL, UR, LL, LR sites in frame order;
  // koff[q] = where quadrant q's bits start
  size_t koff[5] = {0, 0, 0, 0, 0};
  for (int qi = 0; qi < 4; ++qi) koff[qi + 1] = koff[qi] + sq->q[qi].s.size();
  std::vector<size_t> order(n);
  for (size_t b = 0; b < n; ++b) order[b] = b;
  std::vector<std::vector<uint8_t>> keys(n);
  for (size_t b = 0; b < n; ++b) {
    std::vector<uint8_t>& k = keys[b];
    k.reserve(koff[4]);
    for (int qi = 0; qi < 4; ++qi)
      for (const SqSite& st_ : sq->q[qi].s) k.push_back(bits[b * nq + st_.qubit]);
  }
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return keys[x] < keys[y]; });
  auto same = [&](size_t x, size_t y, int upto) {  // keys agree on quadrants 0 .. upto-1
    return std::equal(keys[x].begin(), keys[x].begin() + koff[upto], keys[y].begin());
  };

  const int64_t vUL = sq->q[0].dv, vUR = sq->q[1].dv, hU = sq->q[0].dh, hL = sq->q[2].dh;
  char* A = R.buf(sq->off_a);
  char* B = R.buf(sq->off_b);
  char* C = R.buf(sq->off_c);
  char* P = R.buf(sq->off_p);
  const uint64_t ysz = ((uint64_t)sq->qmax * R.eb + 255) / 256 * 256;
  auto ybuf = [&](int k) { return k == 0 ? B : R.buf(sq->off_y) + (uint64_t)(k - 1) * ysz; };
  const int nblk = cdot_blocks();
  std::vector<double> part((size_t)nblk * 2);
  size_t x = 0;
  while (x < n) {
    // bitstrings [x, xe) share the upper half: T once
    size_t xe = x + 1;
    while (xe < n && same(order[x], order[xe], 2)) ++xe;
    const uint8_t* b0 = bits + order[x] * nq;
    const int64_t eUL = R.quad(0, b0, A);       // Q_UL [vUL][hU]
    const int64_t eUR = R.quad(1, b0, B);       // Q_UR [vUR][hU]
    R.pack(A, P, vUL, hU, sq->prow[0], sq->pld[0]);
    R.gemm(B, vUR, hU, P, sq->pld[0], vUL, C);  // T [vUR][vUL]
    const int64_t eT = eUL + eUR + R.rescale(C, vUR * vUL);
    size_t y = x;
    while (y < xe) {
      // one pass: up to ycap lower-left patterns, each joined into its Y
      std::vector<int64_t> eY;
      std::vector<int> slot(xe - y);  // Y of each bitstring of the pass
      size_t ye = y;
      while (ye < xe && (int)eY.size() < sq->ycap) {
        const uint8_t* bb = bits + order[ye] * nq;
        const int k = (int)eY.size();
        const int64_t eLL = R.quad(2, bb, A);   // Q_LL [hL][vUL]
        R.pack(A, P, hL, vUL, sq->prow[1], sq->pld[1]);
        R.gemm(C, vUR, vUL, P, sq->pld[1], hL, ybuf(k));  // Y [vUR][hL]
        eY.push_back(eT + eLL + R.rescale(ybuf(k), vUR * hL));
        size_t z = ye;
        while (z < xe && same(order[ye], order[z], 3)) slot[z++ - y] = k;
        ye = z;
      }
      // each lower-right pattern of the pass once, dotted with the Y's that need it
      std::map<std::vector<uint8_t>, std::vector<size_t>> lr;
      for (size_t z = y; z < ye; ++z)
        lr[std::vector<uint8_t>(keys[order[z]].begin() + koff[3], keys[order[z]].end())].push_back(z);
      for (auto& kv : lr) {
        const uint8_t* bb = bits + order[kv.second.front()] * nq;
        const int64_t eLR = R.quad(3, bb, A);   // Q_LR [vUR][hL]
        std::map<int, std::pair<double, double>> done;
        for (size_t z : kv.second) {
          const int k = slot[z - y];
          if (!done.count(k)) {
            R.run(2, (double)vUR * hL, 2.0 * R.eb * vUR * hL,
                  [&] { launch_cdot(R.prec, ybuf(k), A, vUR * hL, R.d_part, R.st); });
            hip_check(hipMemcpyAsync(part.data(), R.d_part, part.size() * 8, hipMemcpyDeviceToHost, R.st),
                      "download");
            hip_check(hipStreamSynchronize(R.st), "hipStreamSynchronize");
            double re = 0, im = 0;
            for (int t = 0; t < nblk; ++t) {
              re += part[2 * t];
              im += part[2 * t + 1];
            }
            done[k] = {re, im};
          }
          const size_t b = order[z];
          const int64_t e = eY[k] + eLR;
          out[2 * b] = std::ldexp(done[k].first, (int)e);
          out[2 * b + 1] = std::ldexp(done[k].second, (int)e);
        }
      }
      y = ye;
    }
    x = xe;
  }
  R.collect(pl);
}

}  // namespace psim
