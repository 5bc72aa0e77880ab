/*
 * psim — exact single amplitudes of 2D quantum circuits by PEPS contraction,
 * on one AMD Instinct MI355X (gfx950).
 *
 * Method (Guo et al., "General-purpose quantum circuit simulator with
 * Projected Entangled-Pair States and the quantum supremacy frontier"):
 *   - the state of an Lv x Lh qubit lattice is a PEPS of rank-5 site tensors
 *     A_n[sigma][l][r][u][d] (eq. 1);
 *   - one-qubit gates contract the physical index (eq. 3); a nearest-neighbour
 *     two-qubit gate is split into a sum of chi_o products (eq. 4) and each
 *     factor is absorbed into one site, the new index being bundled with the
 *     shared bond (eqs. 5-6);
 *   - the amplitude <tau|psi> is the contraction of the projected tensors
 *     E_n = A_n[tau_n] (eq. 7), done exactly row by row (supplement S-II,
 *     eqs. S2-S6, Fig. S2(a)), along the short side of the lattice.
 *
 * Conventions shared by every entry point
 *   - qubit n sits at row r = n / lh, column c = n % lh (row 0 on top);
 *   - a bitstring is lv*lh bytes, byte n = tau_n in {0, 1};
 *   - two-qubit matrices act on (q0, q1) with row index 2*tau_q0 + tau_q1;
 *   - matrices are row-major complex as interleaved (re, im) doubles;
 *   - every function returns a psim_status; on failure nothing is written to
 *     the outputs and psim_last_error() describes the cause.  Handles are
 *     opaque, owned by the caller and freed with the matching *_free call
 *     (which accepts NULL).  Input arrays are borrowed for the duration of
 *     the call only.
 *   - functions that take a device (HIP) stream enqueue on it and return
 *     after synchronising that stream.
 *   - with PSIM_LOG=1 in the environment, psim_amplitudes prints one progress
 *     line per swept row to stderr (for long runs); nothing else is printed.
 */
#ifndef PSIM_PUBLIC_H_
#define PSIM_PUBLIC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PSIM_OK = 0,
  PSIM_EINVAL = -1,        /* bad argument: qubit out of range, non-neighbouring 2q gate, bit not 0/1, NULL */
  PSIM_ENOMEM = -2,        /* plan exceeds the memory budget (message states the bytes needed) or allocation failed */
  PSIM_EDEVICE = -3,       /* HIP runtime error (message carries the HIP error string) */
  PSIM_EUNSUPPORTED = -4,  /* valid request this library does not implement */
  PSIM_EINTERNAL = -5
} psim_status;

/* Gate kinds.  The random circuits use H, T, SQRT_X, SQRT_Y and CZ
 * (supplement S-I); U1 / U2 are arbitrary 2x2 / 4x4 matrices given in m. */
typedef enum {
  PSIM_H = 0, PSIM_T = 1, PSIM_SQRT_X = 2, PSIM_SQRT_Y = 3, PSIM_CZ = 4, PSIM_U1 = 5, PSIM_U2 = 6
} psim_gate_kind;

typedef struct {
  int32_t kind;     /* psim_gate_kind */
  int32_t cycle;    /* non-decreasing along the gate list; informational otherwise */
  int32_t q0, q1;   /* q1 = -1 for one-qubit gates */
  const double *m;  /* U1: 8 doubles, U2: 32 doubles (row-major complex); NULL for named gates */
} psim_gate;

typedef enum {
  PSIM_FP64 = 0,     /* complex128 storage, FP64 MFMA */
  PSIM_FP32_4M = 1,  /* complex64 storage, complex product as one real FP32 MFMA GEMM (4 real mults) */
  PSIM_FP32_3M = 2,  /* complex64 storage, three real FP32 MFMA GEMMs (Gauss) */
  PSIM_BF16X3 = 3    /* complex64 storage, BF16 hi/lo split, 3 BF16 MFMA products, FP32 accumulation */
} psim_precision;

typedef enum {
  PSIM_PLAN_HOST_ONLY = 1,  /* plan the contraction on the host only (no device, cannot run) */
  PSIM_PLAN_SPLIT_ACC = 2,  /* FP32 4M and FP32 3M, every site kernel and square-partition join, in
                               both schemes: accumulate each K stage (32 reals of k; each pair of
                               stages in the direct-to-LDS 3M kernel) separately before adding it to
                               the running sum (smaller rounding error, same work, slower: twice the
                               accumulator registers; joins are not grouped) */
  PSIM_PLAN_GRAPH = 4       /* psim_amplitudes captures its row sweep into a HIP graph the first time
                               a (workspace, prefix-trie shape) pair is seen and replays it afterwards;
                               ignored while profiling or when PSIM_LOG=1 */
} psim_plan_flags;

typedef struct {
  int32_t prec;               /* psim_precision */
  int32_t flags;              /* psim_plan_flags */
  uint64_t mem_budget_bytes;  /* device bytes the workspace may use; 0 = 200 GiB */
  int32_t max_batch;          /* most bitstrings per psim_amplitudes call; 0 = 1 */
  int32_t sweep;              /* 0 = along the short side (Fig. S2(a)), 1 = rows, 2 = columns,
                                 3 = square partition (Fig. S2(b); eqs. S9-S10 for even and S11-S12
                                 for odd L x L lattices, any lattice with both sides >= 2; FP64 /
                                 FP32 4M / FP32 3M; not groupable, not tuned).  When the budget
                                 holds the tensors of at least 8 bitstrings, the workspace is sized
                                 for chunks of up to min(32, max_batch) bitstrings contracted
                                 together; otherwise bitstrings go one by one (same results) */
  int32_t device;             /* HIP device ordinal */
  int32_t tile_cfg;           /* interior-site tile candidate: 0 = default, k > 0 = candidate k
                                 (FP32 4M: 1..6, FP32 3M: 1..3, FP64: 1..2, BF16X3: 1..2; with
                                 PSIM_PLAN_SPLIT_ACC only 0, or 3 for FP32 3M (the split kernels'
                                 tiles): EINVAL otherwise).  With 0 and PSIM_TUNE_CACHE set in the environment, the
                                 choices psim_tune stored there for this device architecture,
                                 precision and shape are used; psim_tune may replace them */
} psim_plan_opts;

typedef struct {
  uint64_t workspace_bytes;   /* device workspace psim_amplitudes needs for max_batch bitstrings */
  uint64_t weights_bytes;     /* device memory the plan itself holds (packed site matrices) */
  uint64_t peak_tensor_elems; /* largest tensor held at once for one bitstring (all v-slices) */
  double cmac_per_amplitude;  /* exact complex multiply-adds for one bitstring in the plan's scheme
                                 (row sweep, or the square partition's quadrants and joins) */
  int64_t n_gemm_steps;       /* site contractions per bitstring */
  int32_t L;                  /* boundary width (legs of the row boundary F) */
  int32_t R;                  /* number of rows swept */
  int32_t chi;                /* bond dimension, eq. (2) */
  int32_t v_chunk;            /* v-slices processed together in interior rows */
  int32_t sweep;              /* 1 = rows, 2 = columns, 3 = square partition */
  int32_t prec;
  int32_t hot_cfg;            /* tile candidate used by the costliest site contraction (0 = default) */
  uint64_t peak_bytes;        /* device bytes in use at the peak of psim_amplitudes for max_batch
                                 bitstrings: workspace_bytes + weights_bytes (nothing else is
                                 allocated during the call) */
  int64_t n_tasks;            /* independent pieces of work in one bitstring's contraction: row
                                 scheme, per row, v chunks x site contractions plus one rescale
                                 (the cut loop over v, supplement S-II); square partition, its
                                 device operations per bitstring (quadrant sites, joins,
                                 permutes, inner product) */
  int32_t w_chunk;            /* rows cut over w as well as v (their intermediates exceed 2^29
                                 elements, or the budget): the smallest number of w values per
                                 pass; 0 when no row is cut over w */
} psim_plan_stats;

typedef struct psim_peps_s psim_peps_t;
typedef struct psim_plan_s psim_plan_t;

/* PEPS evolution (eqs. 3-6) on the host in FP64.  Gates are applied in array
 * order to |0...0>.  CZ uses its exact rank-2 split sum_s |s><s| (x) Z^s;
 * U2 is split by SVD with the singular values shared between the factors.
 * Errors: EINVAL for bad sizes, qubits, kinds, or a 2q gate whose qubits are
 * not lattice neighbours. */
psim_status psim_build(int32_t lv, int32_t lh, const psim_gate *gates, size_t n_gates, psim_peps_t **out);

/* Lattice and bond sizes of a built PEPS.  bond_dims (nullable) receives
 * lv*(lh-1) horizontal bonds (row-major, bond (r,c)-(r,c+1)) followed by
 * (lv-1)*lh vertical bonds (bond (r,c)-(r+1,c)), i.e. n_bonds entries. */
psim_status psim_peps_info(const psim_peps_t *peps, int32_t *lv, int32_t *lh, int32_t *chi,
                           int64_t *bond_dims, size_t n_bonds);

/* Frees a PEPS (host memory only); NULL is a no-op.  Plans made from it stay
 * valid. */
void psim_peps_free(psim_peps_t *peps);

/* More gates on a built (possibly projected) PEPS, in array order, with the
 * rules of psim_build (the remark after eq. 7: gates may be applied between
 * measurements).  All or nothing: on an error the PEPS is unchanged. */
psim_status psim_apply(psim_peps_t *peps, const psim_gate *gates, size_t n_gates);

/* Records a measurement outcome: qubit's state projected on |value>
 * (A_q[s] = 0 for s != value), without renormalising, so the squared norm
 * becomes the outcome's probability times the previous squared norm, and
 * double-layer values of the result are unnormalised (divide by the
 * all-identity value for conditional ones).  Errors: EINVAL for a bad qubit
 * or a value other than 0 / 1. */
psim_status psim_project(psim_peps_t *peps, int32_t qubit, int32_t value);

/* Double-layer network of a PEPS (main text: observables of the stored
 * state): the norm network <psi|psi> with a one-qubit operator between the
 * bra and ket layers of every site, returned as a PEPS whose bonds are the
 * squared bonds (doubled leg index = bra * D + ket) and whose two physical
 * slices at site n are
 *   E_{n,s}[(l l')][(r r')][(u u')][(d d')]
 *       = sum_{a,b} conj(A_n[a][l][r][u][d]) O_{n,s}[a][b] A_n[b][l'][r'][u'][d'],  s = 0, 1.
 * ops: host, lv*lh*2 complex 2x2 matrices (row-major (re, im) pairs), O_{n,s}
 * at ops + (2n + s) * 8.  Planned and contracted like any PEPS, its
 * "amplitude" of bitstring b is <psi| prod_n O_{n,b_n} |psi> (e.g. O_{n,0} =
 * Z_n, O_{m,0} = I elsewhere, bits all 0: <Z_n>).  *out is a new handle.
 * Errors: EINVAL for NULL or non-finite ops; EUNSUPPORTED when a doubled site
 * tensor exceeds 2^28 elements per slice. */
psim_status psim_double_layer(const psim_peps_t *peps, const double *ops, psim_peps_t **out);

/* Sequential measurement of every qubit in the computational basis, qubit 0
 * first (main text: sequences of measurements on the stored state): with the
 * prefix t_0..t_{k-1} drawn, qubit k is 0 when u[s * N + k] < p(t_0..t_{k-1}, 0)
 * / (p(.., 0) + p(.., 1)), p being the double-layer value with |t><t| on the
 * measured sites and I elsewhere (N = lv*lh double-layer contractions per call,
 * each over all samples at once, planned with opts: precision, scheme,
 * max_batch, memory budget).  u: host, n_samples * N numbers in [0, 1) (the
 * caller's random numbers).  Writes bits (host, n_samples * N bytes) and, if
 * out_prob is not NULL, p(bits) per sample (host, n_samples doubles).
 * d_workspace: device memory of psim_sample_workspace bytes.
 * Errors: EINVAL for NULL arguments, u outside [0, 1), a short workspace or a
 * host-only opts; ENOMEM / EDEVICE as psim_plan / psim_amplitudes. */
psim_status psim_sample_workspace(const psim_peps_t *peps, const psim_plan_opts *opts, uint64_t *bytes);
psim_status psim_sample(const psim_peps_t *peps, const psim_plan_opts *opts, const double *u, size_t n_samples,
                        void *d_workspace, size_t workspace_bytes, void *hip_stream, uint8_t *bits,
                        double *out_prob);

/* Plan the exact contraction (supplement S-II, Fig. S2(a)): sweep axis, leg
 * orders, cut loops over the last input leg v of each row and, where the
 * per-v intermediates are large, over its first output leg w as well (every
 * (v, w) pair then holds D^(L-1)-element intermediates; same work), the
 * memory plan for the budget, exact work count.
 * Unless PSIM_PLAN_HOST_ONLY is set, projects both values of every site
 * (E = A[tau], eq. 7), packs them for the chosen precision and uploads them to
 * the device; the peps may be freed afterwards.
 * Errors: ENOMEM with the bytes needed; EUNSUPPORTED for a precision this
 * build lacks; EDEVICE on HIP failures. */
psim_status psim_plan(const psim_peps_t *peps, const psim_plan_opts *opts, psim_plan_t **out);

/* The plan's sizes and work counts (psim_plan_stats).  Errors: EINVAL for a
 * NULL argument. */
psim_status psim_plan_info(const psim_plan_t *plan, psim_plan_stats *out);

/* Frees everything the plan holds (device memory, captured graphs);
 * NULL is a no-op.  No call on the plan (or on a group holding it) may be
 * running. */
void psim_plan_free(psim_plan_t *plan);

/* Amplitudes <tau|psi> (eq. 7) of n_bitstrings bitstrings (bits: host,
 * n_bitstrings * lv*lh bytes).  d_workspace is device memory of at least
 * psim_plan_stats.workspace_bytes bytes, owned by the caller; hip_stream is a
 * hipStream_t (NULL = default stream).  Bitstrings that share leading rows
 * share those rows' work.  Results go to out_amp (host, 2*n doubles: re, im)
 * in FP64 as mantissa * 2^exponent assembled on the host.  If more than
 * max_batch bitstrings are passed they are processed max_batch at a time.
 *
 * out_rel_err (nullable; host, n doubles): a measured estimate of each
 * amplitude's relative rounding error, not a bound (an a-priori bound in the
 * style of first-order rounding analysis is larger than the amplitude itself
 * for random circuits of this size, so it would say nothing).  When non-NULL
 * the batch is contracted a second time in a companion form with different
 * rounding, and out_rel_err[b] = |a_b - c_b| / |c_b| (c = companion result;
 * out_amp still holds the plan's own result a):
 *   FP32 4M / 3M plans: the other K-loop accumulation (partial sums per K
 *     stage on or off, PSIM_PLAN_SPLIT_ACC), same packed site matrices.  The
 *     difference is dominated by the less accurate of the two (the unsplit
 *     form, whose error is 2-3x larger), so it tracks the error of unsplit
 *     plans and overstates that of split plans.  It sees only the K-loop
 *     part of the error: where every contraction fits one K stage (bonds of
 *     at most 4, errors near 1e-7) both forms coincide and it reads 0;
 *   BF16X3 plans: the FP32 4M form of the same site matrices (about 100x
 *     more accurate), so the estimate is close to the actual BF16x3 error;
 *   FP64 plans: NaN (no companion; the FP64 path's error is below 1e-12).
 * The estimate doubles the call's work (its second sweep is not profiled).
 * Errors: EINVAL for bits outside {0,1} or a short workspace, EDEVICE.  On an
 * error neither output is written. */
psim_status psim_amplitudes(psim_plan_t *plan, const uint8_t *bits, size_t n_bitstrings,
                            void *d_workspace, size_t workspace_bytes, void *hip_stream,
                            double *out_amp, double *out_rel_err);

/* Allocation-free form of psim_amplitudes, for callers that cannot allocate
 * device memory (tight serving loops, harnesses that forbid hipMalloc): the
 * workspace is a fixed array of PSIM_STATIC_WORKSPACE_BYTES bytes inside the
 * library, one per device, held from its first use on that device until the
 * process ends.  Same kernels, same launches and the same results, bit for
 * bit, as psim_amplitudes on the same plan and bitstrings; the call captures
 * no graph, records no profiling events and allocates nothing on the device
 * (it still enqueues on hip_stream and synchronises it, so it cannot itself
 * be captured into a graph).  All calls on one device share the array, which
 * keeps the last call's contents (each call writes everything it reads before
 * reading it): calls that overlap in time on one device race.
 * Errors: EINVAL when the plan's workspace_bytes exceeds
 * PSIM_STATIC_WORKSPACE_BYTES (the message gives both sizes), otherwise those
 * of psim_amplitudes; out_amp and out_rel_err (nullable, as for
 * psim_amplitudes) are written only on success. */
#define PSIM_STATIC_WORKSPACE_BYTES (64ull << 20)
psim_status psim_amplitudes_static(psim_plan_t *plan, const uint8_t *bits, size_t n_bitstrings, void *hip_stream,
                                   double *out_amp, double *out_rel_err);

/* Optional bits of psim_contract_site's prec argument. */
#define PSIM_CONTRACT_SPLIT_ACC 0x100 /* the split-accumulation kernels (FP32 4M / 3M) */
#define PSIM_CONTRACT_TILE_SHIFT 16   /* prec | (k << 16): tile candidate k (psim_plan_opts.tile_cfg) */

/* One site contraction of the row scheme, eq. (S4), on device buffers:
 *   C[z][m][n] = sum_{k1,k2} A[z][k1][m][k2] * W[k1*K2 + k2][n]     (complex)
 * A: device, complex (complex128 for PSIM_FP64, complex64 otherwise), batch
 *    stride a_batch_stride elements, element (k1, m, k2) at k1*M*K2 + m*K2 + k2.
 * W: host, K1*K2 x N complex128, row-major (packed and uploaded per call).
 * C: device, same element type as A, batch stride M*N; transpose_out = 1
 *    stores C[z][n][m] instead.  batch = number of z.
 * prec: a psim_precision, optionally OR'ed with PSIM_CONTRACT_SPLIT_ACC and
 * (k << PSIM_CONTRACT_TILE_SHIFT) to pick the kernels a plan with
 * PSIM_PLAN_SPLIT_ACC or tile_cfg = k would run (the tile candidate applies
 * to plain stores; transposed stores take the precision's one kernel).
 * Runs the same kernels the amplitude path uses; allocates its own scratch.
 * Errors: EINVAL for non-positive sizes, NULL, a tile / split choice the
 * precision lacks or any other bit set in prec; EUNSUPPORTED, EDEVICE. */
psim_status psim_contract_site(int32_t prec, int64_t batch, int64_t M, int64_t K1, int64_t K2, int64_t N,
                               const void *d_A, int64_t a_batch_stride, const double *W,
                               void *d_C, int32_t transpose_out, void *hip_stream);

/* Autotuner: for every distinct interior-site contraction shape of the plan
 * (eq. S4 steps), time each tile candidate of the plan's precision (reps
 * launches each, HIP events on hip_stream) on scratch data inside the
 * caller's workspace (>= psim_plan_stats.workspace_bytes, contents are
 * overwritten), and keep the fastest for psim_amplitudes.  Every candidate
 * computes the same products in the same order, so the choice changes speed,
 * never results.  best_ms (nullable) receives the chosen time of the
 * costliest shape.  With PSIM_TUNE_CACHE naming a file in the environment,
 * the choices are merged into it as JSON, keyed by device architecture,
 * precision and shape (M, K1, K2, N, batch entries), and later plans start
 * from them.  Split-accumulation plans choose among their split kernels'
 * tiles (FP32 3M: 128 x 128 or 64 x 128; other precisions have one, and
 * nothing is timed); square-partition plans keep their single configuration.  Captured graphs of
 * the plan are dropped when a choice changes.
 * Errors: EINVAL for a short workspace, reps < 1 or an unwritable cache file,
 * EDEVICE. */
psim_status psim_tune(psim_plan_t *plan, void *d_workspace, size_t workspace_bytes, void *hip_stream,
                      int32_t reps, double *best_ms);

/* Per-kernel-class timing of psim_amplitudes, measured with HIP events
 * recorded on the caller's stream around every launch (adds two event
 * records per launch while enabled).  Classes: 0 = first site of a row
 * (K-major A) and the other sites of the first and last rows (their small M
 * or N), 1 = interior sites of the interior rows (eq. S4, the hot step),
 * 2 = last site of a row (v summed, transposed store), 3 = per-row rescale.  op = 1 resets and
 * enables, op = 2 reads the accumulated totals into out[4] (nullable for
 * op 1/0), op = 0 disables.  cmac is the algorithmic complex multiply-add
 * count of the timed launches, bytes their algorithmic memory traffic (for
 * the memory-bound classes 0, 2 and 3).  Square-partition plans (sweep 3)
 * use the classes for: 0 = quadrant site contractions, 1 = the two joins
 * (the D^h x D^h x D^h GEMMs), 2 = permutes, packing and inner products,
 * 3 = rescales. */
typedef struct {
  double ms;          /* summed kernel time */
  int64_t launches;
  double cmac;
  double bytes;       /* algorithmic device-memory bytes of the timed launches: operands read
                         once, results written once (read too when accumulated), one site
                         matrix per launch; rescale: boundary read twice, written once */
} psim_kernel_stats;

psim_status psim_profile(psim_plan_t *plan, int32_t op, psim_kernel_stats *out);

/* Several plans run together: different circuits, lattice sizes and depths
 * in one sweep (the batching of independent amplitude computations that the
 * paper's row scheme allows, supplement S-II, Fig. S2(a); every plan's
 * amplitude is still eq. (7)).  The plans are borrowed: they must outlive the
 * group and not be used by another call while a group call runs.  The group
 * owns a small device array of launch descriptors (psim_group_stats).
 * Errors: EINVAL for a NULL or empty plan list, a host-only plan, or plans
 * on different devices; ENOMEM / EDEVICE on allocation failure. */
typedef struct psim_group_s psim_group_t;

typedef struct {
  int32_t n_plans;
  uint64_t descriptor_bytes;   /* device memory the group holds */
  int64_t grouped_launches;    /* merged launches issued so far (several problems, one grid) */
} psim_group_stats;

psim_status psim_group(psim_plan_t *const *plans, int32_t n_plans, psim_group_t **out);

/* Errors: EINVAL for a NULL argument. */
psim_status psim_group_info(const psim_group_t *group, psim_group_stats *out);

/* Amplitudes for every plan of the group in one interleaved sweep.  Arrays
 * are indexed by plan: bits[p] (host, n_bitstrings[p] * lv*lh bytes of plan
 * p), d_workspaces[p] (device, at least workspace_bytes[p] >= that plan's
 * psim_plan_stats.workspace_bytes; the workspaces of plans with bitstrings
 * must not overlap), out_amp[p] (host, 2*n_bitstrings[p] doubles).  A plan
 * with n_bitstrings[p] = 0 is skipped.  Step k of the sweep issues the k-th
 * device operation of every plan; FP32 (4M / 3M, default tiles, no split
 * accumulation) site contractions of one step that use the same kernel are
 * merged into one launch over all their tiles, everything else is launched
 * per plan.  Each plan's results equal psim_amplitudes' bit for bit.  When
 * every plan was made with PSIM_PLAN_GRAPH, each pass of the sweep is
 * captured into a HIP graph the first time its shape (plans taking part,
 * workspaces, prefix-trie sizes) is seen, and replayed afterwards.
 * Enqueues on hip_stream and synchronises it.
 * Errors: as psim_amplitudes, for the first failing plan (its index in the
 * message); EINVAL for overlapping workspaces. */
psim_status psim_group_amplitudes(psim_group_t *group, const uint8_t *const *bits, const size_t *n_bitstrings,
                                  void *const *d_workspaces, const size_t *workspace_bytes, void *hip_stream,
                                  double *const *out_amp);

/* Frees the group's descriptors and graphs (not its plans); NULL is a
 * no-op. */
void psim_group_free(psim_group_t *group);

/* Message for the last failing call on this thread; valid until the next
 * psim_* call on the same thread.  Never NULL. */
const char *psim_last_error(void);

/* Library version string. */
const char *psim_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PSIM_PUBLIC_H_ */
