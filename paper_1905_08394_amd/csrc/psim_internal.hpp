// Internal types of libpsim: PEPS, contraction plan, kernel launch interface.
#pragma once

#include <complex>
#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "psim.h"

namespace psim {

using cd = std::complex<double>;

// ---------------------------------------------------------------- errors
struct Error {
  psim_status status;
  std::string msg;
};
[[noreturn]] void fail(psim_status st, const std::string& msg);
void set_last_error(const std::string& msg);

// ---------------------------------------------------------------- PEPS
// Rank-5 site tensor A[sigma][l][r][u][d] (eq. 1), row-major in that order.
struct Site {
  int dl = 1, dr = 1, du = 1, dd = 1;
  std::vector<cd> t;  // 2 * dl * dr * du * dd
  size_t size() const { return t.size(); }
  size_t at(int s, int l, int r, int u, int d) const {
    return ((((size_t)s * dl + l) * dr + r) * du + u) * dd + d;
  }
};

}  // namespace psim

struct psim_peps_s {
  int lv = 0, lh = 0;
  std::vector<psim::Site> sites;  // qubit n = r * lh + c
};

namespace psim {

// gates.cpp
void gate_matrix_1q(int kind, const double* m, cd out[4]);
void gate_matrix_2q(int kind, const double* m, cd out[16]);
bool is_two_qubit(int kind);

// build.cpp
void jacobi_svd4(const cd M[16], cd U[16], double S[4], cd V[16]);

// ---------------------------------------------------------------- plan
// Site of the swept lattice: contraction row i (0..R-1), column j (0..L-1).
// Legs are named in the sweep frame (l, r, u, d); u/d run along the sweep.
struct CSite {
  int qubit = 0;
  int dl = 1, dr = 1, du = 1, dd = 1;
};

// One site contraction (eqs. S3-S5) for one node (prefix) and one v value.
struct Step {
  int i = 0, j = 0;
  int kind = 0;          // 0 first site, 1 interior, 2 last site (K1 = v chunk)
  int64_t M = 1, K1 = 1, K2 = 1, N = 1;
  int64_t g_out = 0;     // elements of the output per (node, v) (kind 0/1)
  int cfg = 0;           // kernel tile candidate chosen by the tuner
};

struct Level {
  int64_t F_elems = 1;   // elements of F_i (boundary after row i)
  int64_t Gmax = 0;      // largest per-(node, v) intermediate of this row
  int Dv = 1;            // size of the leg v = u of the last site in this row
  int vchunk = 1;        // v values per pass
  int Dw = 1;            // size of the leg w = d of the first site (the first output leg)
  int wchunk = 1;        // w values per pass; wchunk < Dw: the row is cut over w as well as v
  int64_t Gtask = 0;     // largest per-(node, v, w) intermediate when the row is cut over w
  int group = 1;         // nodes per pass
  int64_t nmax = 1;      // most nodes (distinct prefixes) this level can have
  int64_t cap = 1;       // nodes whose boundary fits the workspace at once
  uint64_t F_off = 0;    // byte offset of this level's boundary buffer in the F region
};

struct DevMatrix {
  void* ptr = nullptr;   // packed, on device
  int64_t ld = 0;        // leading dimension (real elements) of the packed layout
  int exp2 = 0;          // site matrix was scaled by 2^-exp2
  void* ptr_b = nullptr; // BF16x3 plans: hi and lo bf16 planes of the 4M expansion
  int64_t ld_b = 0, plane_b = 0;
};

}  // namespace psim

namespace psim {
struct SquarePlan;
}

struct psim_plan_s {
  psim_plan_opts opts{};
  int lv = 0, lh = 0;
  int R = 0, L = 0;
  int sweep = 1;                         // 1 rows, 2 columns
  int chi = 1;
  std::vector<psim::CSite> cs;           // R * L, index i * L + j
  std::vector<psim::Level> levels;       // R
  std::vector<psim::Step> steps;         // per row i: L steps (index i * L + j)
  std::vector<psim::DevMatrix> w;        // per site and tau: (i * L + j) * 2 + tau
  double cmac = 0;
  int64_t peak_elems = 0;
  uint64_t weights_bytes = 0;
  uint64_t ws_F = 0, ws_G = 0, ws_tab = 0, ws_total = 0;
  bool host_only = false;
  int elem_bytes = 8;
  void* d_ones = nullptr;                // device scalar 1 (the empty boundary before row 0)
  bool profile = false;                  // time launches with events
  psim_kernel_stats prof[4] = {};
  // PSIM_PLAN_GRAPH: instantiated graphs of the row sweep, keyed by workspace
  // address and node count per level, and the stream they are captured on
  std::map<std::vector<int64_t>, void*> graphs;
  void* cap_stream = nullptr;
  int64_t tune_gen = 0;                  // bumped whenever psim_tune changes a tile configuration
  // 1 while the companion sweep of an error estimate runs: FP32 plans toggle
  // split accumulation, BF16x3 plans run their FP32 4M matrices
  int companion = 0;
  int64_t max_ops = 0;                   // most device operations one sub-batch can need
  // square partition (sweep 3): quadrant frames, packed site matrices, workspace plan
  std::shared_ptr<psim::SquarePlan> sq;
  int64_t sq_steps = 0;
};

namespace psim {
// Launch shape of an interior-site step (kind 1): rows per batch entry and
// batch entries per node.  A row cut over w (wchunk < Dw) runs every (v, w)
// pair as its own batch entry, with d_0 = w taken out of the rows.
inline bool w_cut(const Level& lev) { return lev.wchunk < lev.Dw; }
inline int64_t interior_rows(const Level& lev, const Step& s) { return w_cut(lev) ? s.M / lev.Dw : s.M; }
inline int64_t interior_batch(const Level& lev) { return (int64_t)lev.vchunk * (w_cut(lev) ? lev.wchunk : 1); }
}  // namespace psim

// Plans run together (psim_group): the plans are borrowed; the group owns the
// device array of launch descriptors (max_ops slots per plan).
struct psim_group_s {
  std::vector<psim_plan_s*> plans;
  // One device buffer and a pinned host mirror at the same offsets: per plan
  // the launch descriptors (max_ops slots) and the trie-table region, the
  // result-gather segment table, then per plan the gathered leaf values and
  // exponents.  [0, res_off) is uploaded once per pass, [res_off, bytes)
  // downloaded once per pass.
  std::vector<uint64_t> desc_off, tab_off, res_off, res_exp_off;
  uint64_t seg_off = 0, res_begin = 0, bytes = 0;
  void* d_buf = nullptr;
  char* h_buf = nullptr;
  uint64_t desc_bytes = 0;
  int device = 0;
  int64_t grouped_launches = 0;
  // all plans with PSIM_PLAN_GRAPH: instantiated graphs of a pass, keyed by
  // (plan slot, workspace address, nodes per level) of every plan in it, with
  // the number of merged launches each holds; the stream they are captured on
  std::map<std::vector<int64_t>, std::pair<void*, int64_t>> graphs;
  void* cap_stream = nullptr;
};

namespace psim {

// pack.cpp / kernels: sizes of the packed site matrix for a precision
int64_t packed_ld(int prec, int64_t K);
int64_t packed_rows(int prec, int64_t N);
void pack_site_matrix(int prec, const cd* W, int64_t K, int64_t N, std::vector<char>& out, int64_t& ld);
void pack_site_matrix_bf16(const cd* W, int64_t K, int64_t N, std::vector<char>& out, int64_t& ld, int64_t& plane);

// kernels.hip: launch interface (host side)
struct GemmLaunch {
  int prec = PSIM_FP32_4M;
  const void* A = nullptr;
  void* C = nullptr;
  const void* W0 = nullptr;
  const void* W1 = nullptr;
  const int32_t* a_index = nullptr;   // per node: block of A to read (nullable: node itself)
  const uint8_t* tau = nullptr;       // per node: 0/1 selects W0/W1 (nullable: W0)
  int64_t tau_stride = 0;
  int64_t M = 1, K1 = 1, K2 = 1, N = 1;
  int64_t ldw = 0;                    // packed W leading dimension
  int64_t w_koff = 0;                 // complex k offset into W (v chunk of the last site)
  int64_t sA_node = 0, sA_v = 0;      // strides in complex elements
  int64_t sC_node = 0, sC_v = 0;
  int64_t nodes = 1;
  int32_t Bz = 1;                     // batch entries per node
  int32_t trans_out = 0;
  int32_t beta = 0;
  int32_t cfg = 0;                    // tile candidate of the FP32 row-major kernel (0 = default)
  int32_t split = 0;                  // FP32 4M: per-stage partial sums (more accurate K-loop)
  const void* Wb0 = nullptr;          // BF16x3: pre-split bf16 planes of W (hi then lo)
  const void* Wb1 = nullptr;
  int64_t ldwb = 0, planeb = 0;
  int64_t ldct = 0;                   // transposed stores: row stride of C^T in complex elements (0 = M)
  int64_t nb = 0, sCw = 0;            // plain stores with nb > 0: C[n / nb][m][n % nb], blocks sCw apart
};
int fp32_config_count();
int fp32_3m_config_count();
int fp64_config_count();
int bf16x3_config_count();
// tile candidates of a precision (1 = a single configuration)
int config_count(int prec);
// candidates that have a split-accumulation form (FP32 3M: 0 and the 64 x 128
// direct-to-LDS tile; every other precision: 0)
inline bool split_candidate(int prec, int cfg) { return cfg == 0 || (prec == PSIM_FP32_3M && cfg == 3); }
// tune_cache.cpp: autotuner choices kept in the JSON file PSIM_TUNE_CACHE names
std::string device_arch(int device);
std::string tune_key(const std::string& arch, int prec, int64_t M, int64_t K1, int64_t K2, int64_t N, int64_t Bz,
                     bool split = false);
bool tune_cache_lookup(const std::string& key, int* cfg);
void tune_cache_store(const std::map<std::string, std::pair<int, double>>& entries);
void launch_site_gemm(const GemmLaunch& g, void* stream);
// Grouped launches (several problems, one grid): returns the variant id and
// writes the problem descriptor (kargs_bytes() bytes) to out and its tile
// count to *tiles, or returns -1 when the launch is not groupable.
int group_variant(const GemmLaunch& g, void* out, long long* tiles);
int kargs_bytes();
int max_group();
// d_probs[i]: device address of problem i's descriptor; start[0..nprob]: tile offsets
void launch_group(int variant, const void* const* d_probs, const long long* start, int nprob, void* stream);
void launch_rowscale(int prec, void* F, int64_t elems_per_node, int64_t nodes, const int32_t* parent,
                     const int32_t* exp_prev, int32_t* exp_cur, uint32_t* scratch_max, void* stream);
void launch_fill_ones(int prec, void* p, void* stream);
// Rescale of small boundaries (at most kFusedScaleReals reals per node) in one
// fused launch, for up to max_scale_group() boundaries of one precision.
constexpr int64_t kFusedScaleReals = 1 << 18;
struct RescaleJob {
  void* F;
  int64_t per_node, nodes;
  const int32_t* parent;
  const int32_t* exp_prev;
  int32_t* exp_cur;
};
// Device-side gather of small segments (one workgroup row per segment).
struct CopySeg {
  const void* src;
  void* dst;
  int64_t bytes;
};
void launch_copy_segments(const CopySeg* d_segs, int n, int64_t max_bytes, void* stream);
// square partition: complex in[X][Y][Z] -> out[Y][X][Z] (mode 0) or out[X][Z][Y]
// (mode 1), for `nodes` tensors X*Y*Z elements apart
// (mx, nullable: per-node exponent + 4096 from launch_row_exponents; the
// permute then also scales each node by 2^-exponent)
void launch_permute3(int prec, const void* in, void* out, int64_t X, int64_t Y, int64_t Z, int mode, void* stream,
                     int64_t nodes = 1, const uint32_t* mx = nullptr);
// the exponent half of launch_rowscale (nothing scaled; mx keeps exponent + 4096)
void launch_row_exponents(int prec, const void* F, int64_t per_node, int64_t nodes, const int32_t* parent,
                          const int32_t* exp_prev, int32_t* exp_cur, uint32_t* mx, void* stream);
// device Q[n][k] (N x K complex) -> packed W operand for W[k][n] = Q[n][k]
// (rows x ld, zero padded), for `nodes` matrices N*K complex / rows*ld reals apart
void launch_pack_w(int prec, const void* Q, void* P, int64_t N, int64_t K, int64_t rows, int64_t ld, void* stream,
                   int64_t nodes = 1);
// sum_i a[i] b[i] over n complex elements in FP64: cdot_blocks() (re, im)
// partial sums in part, their sum in out[0..1]
int cdot_blocks();
// square.cpp
void make_square_plan(psim_plan_t* pl, const psim_peps_t& P);
// no_alloc: no profiling events (the call creates nothing on the device)
void run_square(psim_plan_t* pl, const uint8_t* bits, size_t n, void* ws, void* stream, double* out,
                bool no_alloc = false);

void launch_cdot(int prec, const void* a, const void* b, int64_t n, double* part, double* out, void* stream);
bool rescale_fusable(int64_t per_node);
int max_scale_group();
void launch_rescale_group(int prec, const RescaleJob* jobs, int n, void* stream);

void hip_check(int err, const char* what);

// measure.cpp: double-layer networks and sequential measurement
psim_peps_t* double_layer(const psim_peps_t& P, const double* ops);
uint64_t sample_workspace(const psim_peps_t& P, const psim_plan_opts& o);
void sample(const psim_peps_t& P, const psim_plan_opts& o, const double* u, size_t n_samples, void* ws,
            size_t ws_bytes, void* stream, uint8_t* bits, double* prob);

}  // namespace psim

// exec.cpp: the row sweep (or the square partition) for a batch; out is
// written only when every sub-batch succeeded.  no_alloc: eager launches only
// (no graph capture or instantiation, no profiling events).
// out_err (nullable): per-amplitude relative-error estimates from a second
// sweep in the companion form (NaN for FP64 plans).
void run_amplitudes(psim_plan_t* pl, const uint8_t* bits, size_t n, void* ws, size_t ws_bytes, void* stream,
                    double* out, bool no_alloc = false, double* out_err = nullptr);
// instantiated graphs a plan keeps at most (the cache is emptied when full)
constexpr size_t kMaxPlanGraphs = 64;
void clear_graphs(psim_plan_t* pl);

