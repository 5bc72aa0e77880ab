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
// Every quadrant tensor is rescaled by an exact power of two after each of
// its rows (its largest component in [1/2, 1)).  The joins are not: T and Y
// are sums of at most D^h products of such components, far inside the FP32
// range, and their magnitudes only pass into the final FP64 inner product.
// The exponents stay on the device (one slot per rescale) with the
// inner products (one slot per amplitude) until a flush downloads them all at
// once, so the host does not wait on the stream between launches; each
// amplitude's exponent is then summed on the host with the site-matrix
// exponents.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>

#include <hip/hip_runtime_api.h>

#include "psim_internal.hpp"

namespace psim {

// device slots for rescale exponents and inner products between flushes
constexpr int64_t kSqExpSlots = 8192;
constexpr int64_t kSqDotSlots = 1024;
// batched form: at most this many bitstrings per chunk, and used only when
// the budget holds at least kSqMinChunk
constexpr int64_t kSqChunk = 32;
constexpr int64_t kSqMinChunk = 8;

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
  // join j reads its quadrant tensor itself as the W operand (ld = 2K, no
  // packing): FP32 3M with every tile interior (the direct-to-LDS kernel)
  bool direct[2] = {false, false};
  uint64_t off_w1 = 0, off_w2 = 0, off_a = 0, off_b = 0, off_c = 0, off_p = 0, off_small = 0, off_y = 0;
  int ycap = 1;                // Y tensors held at once (lower-left patterns joined per pass)
  // batched form (chunk > 0): the bitstrings of a chunk have every quadrant
  // pattern contracted in one set of launches (the pattern is the node
  // index), each join per pattern pair; buffers [node][elements] with
  // exact node strides
  int64_t chunk = 0;
  uint64_t boff_run[2] = {0, 0}, boff_q[4] = {0, 0, 0, 0}, boff_t = 0, boff_y = 0, boff_pk[2] = {0, 0};
  uint64_t boff_tau = 0, boff_zeros = 0, boff_mx = 0, boff_desc[2] = {0, 0};
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
  // join 1 reads Q_UL as W (N = vUL, K = hU), join 2 reads Q_LL (N = hL, K = vUL); M = vUR for both
  const int64_t jn[2] = {vUL, hL}, jk[2] = {hU, vUL};
  for (int j = 0; j < 2; ++j) {
    sq->direct[j] = prec == PSIM_FP32_3M && vUR % 128 == 0 && jn[j] % 128 == 0 && jk[j] % 32 == 0;
    sq->prow[j] = sq->direct[j] ? 0 : packed_rows(prec, jn[j]);
    sq->pld[j] = sq->direct[j] ? 2 * jk[j] : packed_ld(prec, jk[j]);
  }

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
  off += al(16 + (uint64_t)cdot_blocks() * 16 + (uint64_t)kSqExpSlots * 4 + (uint64_t)kSqDotSlots * 16);
  // more Y tensors (one per lower-left pattern of a pass) from what the
  // budget leaves, so each lower-right quadrant is contracted once per pass
  sq->off_y = off;
  const uint64_t ysz = al((uint64_t)sq->qmax * eb);
  const uint64_t budget = pl->opts.mem_budget_bytes;
  uint64_t extra = budget > off + 256 ? (budget - off - 256) / ysz : 0;
  extra = std::min<uint64_t>({extra, 15, (uint64_t)std::max(pl->opts.max_batch, 1) - 1});
  sq->ycap = 1 + (int)extra;
  off += extra * ysz;
  const uint64_t seq_total = off + 256;

  // batched form, when the budget holds a chunk of at least kSqMinChunk
  {
    const int64_t sq_[4] = {sq->q[0].dv * sq->q[0].dh, sq->q[1].dv * sq->q[1].dh, sq->q[2].dv * sq->q[2].dh,
                            sq->q[3].dv * sq->q[3].dh};
    const uint64_t per = eb * (2 * (uint64_t)sq->tmax + sq_[0] + sq_[1] + sq_[2] + sq_[3] + (uint64_t)vUR * vUL +
                               (uint64_t)vUR * hL) +
                         rb * (uint64_t)(sq->prow[0] * sq->pld[0] + sq->prow[1] * sq->pld[1]) + (uint64_t)Lv * Lh + 8;
    const uint64_t fixed = sq->off_y + 16 * 256 + 256 +  // small region and per-region alignment
                           2 * (uint64_t)max_group() * kargs_bytes();
    int64_t c = budget > fixed ? (int64_t)((budget - fixed) / per) : 0;
    c = std::min<int64_t>({c, kSqChunk, (int64_t)std::max(pl->opts.max_batch, 1)});
    if (c >= kSqMinChunk) {
      sq->chunk = c;
      uint64_t bo = sq->off_y;
      auto take = [&](uint64_t bytes) {
        const uint64_t at = bo;
        bo += al(bytes);
        return at;
      };
      sq->boff_run[0] = take((uint64_t)c * sq->tmax * eb);
      sq->boff_run[1] = take((uint64_t)c * sq->tmax * eb);
      for (int qi = 0; qi < 4; ++qi) sq->boff_q[qi] = take((uint64_t)c * sq_[qi] * eb);
      sq->boff_t = take((uint64_t)c * vUR * vUL * eb);
      sq->boff_y = take((uint64_t)c * vUR * hL * eb);
      sq->boff_pk[0] = take((uint64_t)c * sq->prow[0] * sq->pld[0] * rb);
      sq->boff_pk[1] = take((uint64_t)c * sq->prow[1] * sq->pld[1] * rb);
      sq->boff_tau = take((uint64_t)c * Lv * Lh);
      sq->boff_zeros = take((uint64_t)c * 4);
      sq->boff_mx = take((uint64_t)c * 4);
      sq->boff_desc[0] = take((uint64_t)max_group() * kargs_bytes());
      sq->boff_desc[1] = take((uint64_t)max_group() * kargs_bytes());
      sq->ycap = 1;
      off = bo;
    }
  }
  pl->ws_total = sq->chunk ? off + 256 : seq_total;
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
  int split = 0;         // per-stage partial sums in the FP32 site and join kernels
  uint64_t eb;
  int32_t* d_zero;
  uint32_t* d_mx;
  double* d_part;
  int32_t* d_exps;       // kSqExpSlots exponent slots
  double* d_dots;        // kSqDotSlots (re, im) inner products
  double* out = nullptr;

  // Exponent of a tensor: a host part (site matrices) plus device slots
  // (rescales), identified by ids that are never reused within a call.
  struct Exp {
    int64_t host = 0;
    std::vector<int64_t> slots;
    Exp& operator+=(const Exp& o) {
      host += o.host;
      slots.insert(slots.end(), o.slots.begin(), o.slots.end());
      return *this;
    }
  };
  int64_t exp_next = 0, exp_base = 0, dot_next = 0, dot_base = 0;
  std::vector<int64_t> exp_val;   // downloaded exponent of every slot id below exp_base
  std::vector<double> dot_val;    // downloaded (re, im) of every dot id below dot_base
  struct Pend {
    size_t b;                     // output index
    int64_t dot;
    Exp e;
  };
  std::vector<Pend> pend;         // amplitudes waiting for the next flush
  // optional event timing (psim_profile): class 0 quadrant site contractions,
  // 1 joins, 2 permutes / packing / inner products, 3 rescales
  struct Timed {
    hipEvent_t a, b;
    int cls;
    double cmac, bytes;
  };
  std::vector<Timed> timed;
  bool profile = false;

  SqRun() = default;
  SqRun(const SqRun&) = delete;
  SqRun& operator=(const SqRun&) = delete;
  ~SqRun() {  // events left by a run that ended in an error
    for (Timed& t : timed) {
      (void)hipEventDestroy(t.a);
      (void)hipEventDestroy(t.b);
    }
  }

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

  // Download every slot written since the last flush (one synchronisation)
  // and write the amplitudes that waited for them.
  void flush() {
    const int64_t ne = exp_next - exp_base, nd = dot_next - dot_base;
    if (ne == 0 && nd == 0 && pend.empty()) return;
    std::vector<int32_t> he((size_t)ne);
    std::vector<double> hd((size_t)(2 * nd));
    if (ne) hip_check(hipMemcpyAsync(he.data(), d_exps, (size_t)ne * 4, hipMemcpyDeviceToHost, st), "download exponents");
    if (nd) hip_check(hipMemcpyAsync(hd.data(), d_dots, (size_t)nd * 16, hipMemcpyDeviceToHost, st), "download dots");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    exp_val.insert(exp_val.end(), he.begin(), he.end());
    dot_val.insert(dot_val.end(), hd.begin(), hd.end());
    exp_base = exp_next;
    dot_base = dot_next;
    for (const Pend& p : pend) {
      int64_t e = p.e.host;
      for (int64_t id : p.e.slots) e += exp_val[(size_t)id];
      out[2 * p.b] = std::ldexp(dot_val[(size_t)(2 * p.dot)], (int)e);
      out[2 * p.b + 1] = std::ldexp(dot_val[(size_t)(2 * p.dot + 1)], (int)e);
    }
    pend.clear();
  }

  // End of a quadrant row for `nodes` running tensors T (per_node elements
  // apart): exact power-of-two rescale, one exponent slot per node, then,
  // when out is set, the permute [X][Y][Z] -> out (mode as launch_permute3).
  // Small tensors are scaled in place by the fused kernel; for large ones
  // only the exponents are found here and the permute applies the scaling
  // (one pass over the tensor fewer).  parents: `nodes` zeros; mx: `nodes`
  // scratch words.  Returns the first slot id.
  int64_t row_end(void* T, int64_t per_node, int64_t nodes, const int32_t* parents, uint32_t* mx, void* out,
                  int64_t X, int64_t Y, int64_t Z, int mode) {
    if (exp_next - exp_base + nodes > kSqExpSlots) flush();
    int32_t* slot = d_exps + (exp_next - exp_base);
    const bool fold = out && !rescale_fusable(per_node);
    if (fold)
      run(3, 0, 1.0 * eb * per_node * nodes,
          [&] { launch_row_exponents(prec, T, per_node, nodes, parents, d_zero, slot, mx, st); });
    else
      run(3, 0, 3.0 * eb * per_node * nodes,
          [&] { launch_rowscale(prec, T, per_node, nodes, parents, d_zero, slot, mx, st); });
    if (out)
      run(2, 0, 2.0 * eb * X * Y * Z * nodes,
          [&] { launch_permute3(prec, T, out, X, Y, Z, mode, st, nodes, fold ? mx : nullptr); });
    const int64_t first = exp_next;
    exp_next += nodes;
    return first;
  }

  // sum_i a[i] b[i] over n complex elements into a dot slot; returns its id
  int64_t dot(const void* a, const void* b, int64_t n) {
    if (dot_next - dot_base == kSqDotSlots) flush();
    double* o = d_dots + 2 * (dot_next - dot_base);
    run(2, (double)n, 2.0 * eb * n, [&] { launch_cdot(prec, a, b, n, d_part, o, st); });
    return dot_next++;
  }

  // Contract quadrant qi for bits into dst; returns its exponent.
  Exp quad(int qi, const uint8_t* bits, char* dst) {
    const SqQuad& Q = sq->q[qi];
    const int nr = Q.nr, nc = Q.nc;
    char* cur = buf(sq->off_w1);
    char* nxt = buf(sq->off_w2);
    Exp e;
    int64_t cur_elems = 1;
    for (int i = 0; i < nr; ++i) {
      for (int j = 0; j < nc; ++j) {
        const SqSite& st_ = Q.s[(size_t)i * nc + j];
        const int tau = bits[st_.qubit];
        const DevMatrix& w = st_.w[tau];
        const Shape sh = site_shape(Q, i, j);
        GemmLaunch g;
        g.prec = prec;
        g.split = split;
        g.cfg = (split && prec == PSIM_FP32_3M) ? 3 : 0;  // the 64 x 128 split tile, as for the joins
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
        e.host += w.exp2;
        std::swap(cur, nxt);
        cur_elems = sh.M * sh.N;
      }
      // rescale; [o_0 .. o_{i-1}][d_0 .. d_{h-1}][o_i] -> next layout
      int64_t X = 1, Y = 1;
      for (int k = 0; k < i; ++k) X *= Q.s[(size_t)k * nc + nc - 1].dr;
      for (int j = 0; j < nc; ++j) Y *= Q.s[(size_t)i * nc + j].dd;
      const int64_t Z = Q.s[(size_t)i * nc + nc - 1].dr;
      const bool last = i + 1 == nr;
      char* out = last ? dst : (X > 1 ? nxt : nullptr);
      e.slots.push_back(row_end(cur, cur_elems, 1, d_zero, d_mx, out, X, Y, Z, last && qi == 2 ? 1 : 0));
      if (out == nxt) std::swap(cur, nxt);
    }
    return e;
  }

  int32_t* d_zeros = nullptr;  // batched form: parent index 0 for every node
  uint32_t* d_mxn = nullptr;   // batched form: per-node rescale scratch

  // Batched form: quadrant qi for `nodes` patterns at once (pattern p's bits
  // at d_tau[p * sites + s], s in frame order), running tensors in r0 / r1,
  // the finished tensors in dst (node stride dv * dh).  Returns the first
  // exponent slot of each frame row; pattern p's slot of row i is
  // row_slot[i] + p.
  std::vector<int64_t> quad_nodes(int qi, int64_t nodes, const uint8_t* d_tau, char* r0, char* r1, char* dst) {
    const SqQuad& Q = sq->q[qi];
    const int nr = Q.nr, nc = Q.nc;
    const int64_t sites = (int64_t)Q.s.size();
    char* cur = r0;
    char* nxt = r1;
    std::vector<int64_t> row_slot;
    int64_t cur_elems = 1;
    for (int i = 0; i < nr; ++i) {
      for (int j = 0; j < nc; ++j) {
        const SqSite& st_ = Q.s[(size_t)i * nc + j];
        if (st_.w[0].ld != st_.w[1].ld) fail(PSIM_EINTERNAL, "site matrices of one site differ in layout");
        const Shape sh = site_shape(Q, i, j);
        const bool first = i == 0 && j == 0;
        GemmLaunch g;
        g.prec = prec;
        g.split = split;
        g.cfg = (split && prec == PSIM_FP32_3M) ? 3 : 0;  // the 64 x 128 split tile, as for the joins
        g.A = first ? pl->d_ones : (const void*)cur;
        g.C = nxt;
        g.W0 = st_.w[0].ptr;
        g.W1 = st_.w[1].ptr;
        g.tau = d_tau + (i * nc + j);
        g.tau_stride = sites;
        g.ldw = st_.w[0].ld;
        g.M = sh.M;
        g.K1 = sh.K1;
        g.K2 = sh.K2;
        g.N = sh.N;
        g.nodes = nodes;
        g.Bz = 1;
        g.sA_node = first ? 0 : sh.K1 * sh.M * sh.K2;  // every node reads the scalar 1 first
        g.sC_node = sh.M * sh.N;
        run(0, (double)nodes * sh.M * sh.K1 * sh.K2 * sh.N,
            (double)eb * nodes * (sh.M * sh.K1 * sh.K2 + sh.M * sh.N), [&] { launch_site_gemm(g, st); });
        std::swap(cur, nxt);
        cur_elems = sh.M * sh.N;
      }
      int64_t X = 1, Y = 1;
      for (int k = 0; k < i; ++k) X *= Q.s[(size_t)k * nc + nc - 1].dr;
      for (int j = 0; j < nc; ++j) Y *= Q.s[(size_t)i * nc + j].dd;
      const int64_t Z = Q.s[(size_t)i * nc + nc - 1].dr;
      const bool last = i + 1 == nr;
      char* out = last ? dst : (X > 1 ? nxt : nullptr);
      row_slot.push_back(row_end(cur, cur_elems, nodes, d_zeros, d_mxn, out, X, Y, Z, last && qi == 2 ? 1 : 0));
      if (out == nxt) std::swap(cur, nxt);
    }
    return row_slot;
  }

  static GemmLaunch join_launch(int prec, int split, const void* A, int64_t M, int64_t K, const void* P, int64_t ld,
                                int64_t N, void* C) {
    GemmLaunch g;
    g.prec = prec;
    g.split = split;
    // split 3M joins: the 64 x 128 split tile (no spills, three workgroups
    // per CU; the 128 x 128 one is taken where M is not a multiple of 64)
    g.cfg = (split && prec == PSIM_FP32_3M) ? 3 : 0;
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
    return g;
  }

  // Several joins of one shape: one grouped launch (the same kernel body and
  // tiles as separate launches) when the kernel has a grouped form, else one
  // launch each.  d_desc holds max_group() descriptors; host copies of the
  // descriptors are appended to keep (alive until the next synchronisation).
  void joins(const std::vector<GemmLaunch>& gl, char* d_desc, std::vector<std::vector<uint8_t>>& keep) {
    if (gl.empty()) return;
    const int kb = kargs_bytes();
    double cmac = 0, bytes = 0;
    for (const GemmLaunch& g : gl) {
      cmac += (double)g.M * g.K2 * g.N;
      bytes += (double)eb * (g.M * g.K2 + g.K2 * g.N + g.M * g.N);
    }
    if (gl.size() > 1 && (int)gl.size() <= max_group()) {
      keep.emplace_back(gl.size() * (size_t)kb);
      std::vector<uint8_t>& desc = keep.back();
      std::vector<long long> start(gl.size() + 1, 0);
      std::vector<const void*> probs(gl.size());
      int var = -1;
      bool ok = true;
      for (size_t i = 0; i < gl.size() && ok; ++i) {
        long long tiles = 0;
        const int v = group_variant(gl[i], desc.data() + i * kb, &tiles);
        ok = v >= 0 && (var < 0 || v == var);
        var = v;
        start[i + 1] = start[i] + tiles;
        probs[i] = d_desc + i * kb;
      }
      if (ok) {
        hip_check(hipMemcpyAsync(d_desc, desc.data(), desc.size(), hipMemcpyHostToDevice, st), "upload join descriptors");
        run(1, cmac, bytes, [&] { launch_group(var, probs.data(), start.data(), (int)gl.size(), st); });
        return;
      }
    }
    for (const GemmLaunch& g : gl)
      run(1, (double)g.M * g.K2 * g.N, (double)eb * (g.M * g.K2 + g.K2 * g.N + g.M * g.N),
          [&] { launch_site_gemm(g, st); });
  }

  void gemm(const void* A, int64_t M, int64_t K, const void* P, int64_t ld, int64_t N, void* C) {
    GemmLaunch g;
    g.prec = prec;
    g.split = split;
    // split 3M joins: the 64 x 128 split tile (no spills, three workgroups
    // per CU; the 128 x 128 one is taken where M is not a multiple of 64)
    g.cfg = (split && prec == PSIM_FP32_3M) ? 3 : 0;
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
  void pack(const void* Q, void* P, int64_t N, int64_t K, int64_t rows, int64_t ld, int64_t nodes = 1) {
    run(2, 0, nodes * ((double)eb * N * K + (double)(eb / 2) * rows * ld),
        [&] { launch_pack_w(prec, Q, P, N, K, rows, ld, st, nodes); });
  }
};

}  // namespace

namespace {

// Batched form: consecutive bitstrings of the sorted order in chunks of up to
// sq->chunk.  Per chunk, each quadrant's distinct patterns are contracted
// together (the pattern is the node index of every launch), then one join per
// distinct (UL, UR) pair (T) and per distinct (pair, LL) (Y), then one inner
// product per distinct (Y, LR); a chunk whose (UL, UR) pairs, and (UL, UR,
// LL) triples, were all in the previous chunk reuses its T, and Y, tensors
// (bitstrings that differ only in the lower quadrants: the fast-sampling
// reuse of the square partition).  Each tensor is computed by the same kernel
// body on the same tiles as in the one-by-one form (the joins of a chunk in
// one grouped launch where the kernel has a grouped form), so the results
// are the same bit for bit.
void run_chunks(SqRun& R, const uint8_t* bits, const std::vector<size_t>& order,
                const std::vector<std::vector<uint8_t>>& keys, const size_t koff[5]) {
  const SquarePlan* sq = R.sq;
  const int nq = sq->lv * sq->lh;
  const size_t n = order.size();
  const int64_t vUL = sq->q[0].dv, vUR = sq->q[1].dv, hU = sq->q[0].dh, hL = sq->q[2].dh;
  const uint64_t eb = R.eb, rb = R.eb / 2;
  int64_t qsz[4];
  for (int qi = 0; qi < 4; ++qi) qsz[qi] = sq->q[qi].dv * sq->q[qi].dh;
  char* run0 = R.buf(sq->boff_run[0]);
  char* run1 = R.buf(sq->boff_run[1]);
  char* Tst = R.buf(sq->boff_t);
  char* Yst = R.buf(sq->boff_y);
  R.d_zeros = (int32_t*)R.buf(sq->boff_zeros);
  R.d_mxn = (uint32_t*)R.buf(sq->boff_mx);
  hip_check(hipMemsetAsync(R.d_zeros, 0, (size_t)sq->chunk * 4, R.st), "clear parents");
  uint8_t* d_tau = (uint8_t*)R.buf(sq->boff_tau);
  std::vector<std::vector<uint8_t>> uploads;  // host copies stay alive until the final flush
  using Key = std::vector<uint8_t>;
  using Pair = std::pair<Key, Key>;     // (UL, UR) patterns
  using Tri = std::array<Key, 3>;       // (UL, UR, LL) patterns
  // T and Y tensors left in their stores by the previous chunk; a chunk all
  // of whose pairs (triples) are among them reuses them instead of
  // recomputing (bitstrings that differ only in the lower quadrants)
  std::map<Pair, int> t_of;
  std::vector<SqRun::Exp> eT;
  std::map<Tri, int> y_of;
  std::vector<SqRun::Exp> eY;
  for (size_t c0 = 0; c0 < n; c0 += (size_t)sq->chunk) {
    const size_t c1 = std::min(n, c0 + (size_t)sq->chunk);
    std::vector<std::array<Key, 4>> kq(c1 - c0);
    for (size_t z = c0; z < c1; ++z)
      for (int qi = 0; qi < 4; ++qi)
        kq[z - c0][qi] = Key(keys[order[z]].begin() + koff[qi], keys[order[z]].begin() + koff[qi + 1]);
    bool new_t = false, new_y = false;
    for (const auto& k : kq) {
      new_t = new_t || !t_of.count(Pair(k[0], k[1]));
      new_y = new_y || !y_of.count(Tri{k[0], k[1], k[2]});
    }
    new_y = new_y || new_t;
    // distinct patterns of the quadrants to contract
    const bool need[4] = {new_t, new_t, new_y, true};
    std::map<Key, int> pid[4];
    std::vector<size_t> rep[4];  // a bitstring of each pattern
    std::vector<std::array<int, 4>> bp(c1 - c0, std::array<int, 4>{-1, -1, -1, -1});
    for (size_t z = c0; z < c1; ++z)
      for (int qi = 0; qi < 4; ++qi) {
        if (!need[qi]) continue;
        auto it = pid[qi].find(kq[z - c0][qi]);
        if (it == pid[qi].end()) {
          it = pid[qi].emplace(kq[z - c0][qi], (int)rep[qi].size()).first;
          rep[qi].push_back(order[z]);
        }
        bp[z - c0][qi] = it->second;
      }
    // bits of every pattern in frame order, the quadrants to contract in one upload
    uploads.emplace_back();
    std::vector<uint8_t>& tab = uploads.back();
    size_t toff[4];
    std::vector<int64_t> host_e[4];
    for (int qi = 0; qi < 4; ++qi) {
      toff[qi] = tab.size();
      for (size_t b : rep[qi]) {
        int64_t e = 0;
        for (const SqSite& st_ : sq->q[qi].s) {
          const uint8_t t = bits[b * nq + st_.qubit];
          tab.push_back(t);
          e += st_.w[t].exp2;
        }
        host_e[qi].push_back(e);
      }
    }
    hip_check(hipMemcpyAsync(d_tau, tab.data(), tab.size(), hipMemcpyHostToDevice, R.st), "upload pattern bits");
    auto quad = [&](int qi) {
      return R.quad_nodes(qi, (int64_t)rep[qi].size(), d_tau + toff[qi], run0, run1, R.buf(sq->boff_q[qi]));
    };
    auto qptr = [&](int qi, int p) { return R.buf(sq->boff_q[qi]) + (uint64_t)p * qsz[qi] * eb; };
    auto pattern_exp = [&](int qi, int p, const std::vector<int64_t>& row_slot) {
      SqRun::Exp e;
      e.host = host_e[qi][p];
      for (int64_t x : row_slot) e.slots.push_back(x + p);
      return e;
    };
    std::vector<GemmLaunch> gl;
    if (new_t) {
      // upper half: T per distinct (UL, UR)
      const std::vector<int64_t> sUL = quad(0), sUR = quad(1);
      if (!sq->direct[0])
        R.pack(qptr(0, 0), R.buf(sq->boff_pk[0]), vUL, hU, sq->prow[0], sq->pld[0], (int64_t)rep[0].size());
      auto w_ul = [&](int p) -> const char* {
        return sq->direct[0] ? qptr(0, p) : R.buf(sq->boff_pk[0]) + (uint64_t)p * sq->prow[0] * sq->pld[0] * rb;
      };
      t_of.clear();
      eT.clear();
      std::vector<std::pair<int, int>> pairs;
      for (size_t z = c0; z < c1; ++z) {
        const auto& b = bp[z - c0];
        if (t_of.emplace(Pair(kq[z - c0][0], kq[z - c0][1]), (int)pairs.size()).second) {
          pairs.emplace_back(b[0], b[1]);
          SqRun::Exp e = pattern_exp(0, b[0], sUL);
          e += pattern_exp(1, b[1], sUR);
          eT.push_back(e);
        }
      }
      for (size_t t = 0; t < pairs.size(); ++t)
        gl.push_back(SqRun::join_launch(
            R.prec, R.split, qptr(1, pairs[t].second), vUR, hU,
            w_ul(pairs[t].first), sq->pld[0], vUL,
            Tst + (uint64_t)t * vUR * vUL * eb));
      R.joins(gl, R.buf(sq->boff_desc[0]), uploads);
    }
    if (new_y) {
      // lower-left: Y per distinct (pair, LL)
      const std::vector<int64_t> sLL = quad(2);
      if (!sq->direct[1])
        R.pack(qptr(2, 0), R.buf(sq->boff_pk[1]), hL, vUL, sq->prow[1], sq->pld[1], (int64_t)rep[2].size());
      auto w_ll = [&](int p) -> const char* {
        return sq->direct[1] ? qptr(2, p) : R.buf(sq->boff_pk[1]) + (uint64_t)p * sq->prow[1] * sq->pld[1] * rb;
      };
      y_of.clear();
      eY.clear();
      std::vector<std::pair<int, int>> tris;  // (T index, LL pattern)
      for (size_t z = c0; z < c1; ++z) {
        const auto& k = kq[z - c0];
        const int ti = t_of.at(Pair(k[0], k[1]));
        if (y_of.emplace(Tri{k[0], k[1], k[2]}, (int)tris.size()).second) {
          tris.emplace_back(ti, bp[z - c0][2]);
          SqRun::Exp e = eT[ti];
          e += pattern_exp(2, bp[z - c0][2], sLL);
          eY.push_back(e);
        }
      }
      gl.clear();
      for (size_t t = 0; t < tris.size(); ++t)
        gl.push_back(SqRun::join_launch(
            R.prec, R.split, Tst + (uint64_t)tris[t].first * vUR * vUL * eb, vUR, vUL,
            w_ll(tris[t].second), sq->pld[1], hL,
            Yst + (uint64_t)t * vUR * hL * eb));
      R.joins(gl, R.buf(sq->boff_desc[1]), uploads);
    }
    // lower-right, then one inner product per distinct (Y, LR)
    const std::vector<int64_t> sLR = quad(3);
    std::map<std::pair<int, int>, int64_t> dot_id;
    for (size_t z = c0; z < c1; ++z) {
      const auto& k = kq[z - c0];
      const int lr = bp[z - c0][3];
      const int yi = y_of.at(Tri{k[0], k[1], k[2]});
      auto it = dot_id.find(std::make_pair(yi, lr));
      if (it == dot_id.end())
        it = dot_id.emplace(std::make_pair(yi, lr),
                            R.dot(Yst + (uint64_t)yi * vUR * hL * eb, qptr(3, lr), vUR * hL)).first;
      SqRun::Pend p{order[z], it->second, eY[yi]};
      p.e += pattern_exp(3, lr, sLR);
      R.pend.push_back(std::move(p));
    }
  }
  R.flush();
}

}  // namespace

void run_square(psim_plan_t* pl, const uint8_t* bits, size_t n, void* ws, void* stream, double* out, bool no_alloc) {
  const SquarePlan* sq = pl->sq.get();
  const int nq = sq->lv * sq->lh;
  hip_check(hipSetDevice(pl->opts.device), "hipSetDevice");
  SqRun R;
  R.pl = pl;
  R.sq = sq;
  R.st = (hipStream_t)stream;
  R.base = (char*)(((uintptr_t)ws + 255) / 256 * 256);
  R.profile = pl->profile && !no_alloc && !pl->companion;
  R.prec = pl->opts.prec;
  R.split = (pl->opts.flags & PSIM_PLAN_SPLIT_ACC) ? 1 : 0;
  if (pl->companion) R.split ^= 1;  // error estimate: the other K-loop accumulation
  R.eb = pl->elem_bytes;
  char* small = R.buf(sq->off_small);
  R.d_zero = (int32_t*)small;
  R.d_mx = (uint32_t*)(small + 8);
  R.d_part = (double*)(small + 16);
  R.d_exps = (int32_t*)(small + 16 + (size_t)cdot_blocks() * 16);
  R.d_dots = (double*)(small + 16 + (size_t)cdot_blocks() * 16 + (size_t)kSqExpSlots * 4);
  R.out = out;
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
  if (sq->chunk > 0) {
    run_chunks(R, bits, order, keys, koff);
    R.flush();
    R.collect(pl);
    return;
  }
  char* A = R.buf(sq->off_a);
  char* B = R.buf(sq->off_b);
  char* C = R.buf(sq->off_c);
  char* P = R.buf(sq->off_p);
  const uint64_t ysz = ((uint64_t)sq->qmax * R.eb + 255) / 256 * 256;
  auto ybuf = [&](int k) { return k == 0 ? B : R.buf(sq->off_y) + (uint64_t)(k - 1) * ysz; };
  size_t x = 0;
  while (x < n) {
    // bitstrings [x, xe) share the upper half: T once
    size_t xe = x + 1;
    while (xe < n && same(order[x], order[xe], 2)) ++xe;
    const uint8_t* b0 = bits + order[x] * nq;
    SqRun::Exp eT = R.quad(0, b0, A);           // Q_UL [vUL][hU]
    eT += R.quad(1, b0, B);                     // Q_UR [vUR][hU]
    if (!sq->direct[0]) R.pack(A, P, vUL, hU, sq->prow[0], sq->pld[0]);
    R.gemm(B, vUR, hU, sq->direct[0] ? A : P, sq->pld[0], vUL, C);  // T [vUR][vUL]
    size_t y = x;
    while (y < xe) {
      // one pass: up to ycap lower-left patterns, each joined into its Y
      std::vector<SqRun::Exp> eY;
      std::vector<int> slot(xe - y);  // Y of each bitstring of the pass
      size_t ye = y;
      while (ye < xe && (int)eY.size() < sq->ycap) {
        const uint8_t* bb = bits + order[ye] * nq;
        const int k = (int)eY.size();
        SqRun::Exp e = eT;
        e += R.quad(2, bb, A);                  // Q_LL [hL][vUL]
        if (!sq->direct[1]) R.pack(A, P, hL, vUL, sq->prow[1], sq->pld[1]);
        R.gemm(C, vUR, vUL, sq->direct[1] ? A : P, sq->pld[1], hL, ybuf(k));  // Y [vUR][hL]
        eY.push_back(e);
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
        const SqRun::Exp eLR = R.quad(3, bb, A);  // Q_LR [vUR][hL]
        std::map<int, int64_t> done;            // Y slot -> dot id
        for (size_t z : kv.second) {
          const int k = slot[z - y];
          if (!done.count(k)) done[k] = R.dot(ybuf(k), A, vUR * hL);
          SqRun::Pend p{order[z], done[k], eY[k]};
          p.e += eLR;
          R.pend.push_back(std::move(p));
        }
      }
      y = ye;
    }
    x = xe;
  }
  R.flush();
  R.collect(pl);
}

}  // namespace psim
