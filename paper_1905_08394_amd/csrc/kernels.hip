// Site-contraction kernels for gfx950 (CDNA4).
//
// One launch computes, for every batch entry z = (node, v):
//   C[m][n] = sum_{k1, k2} A[k1][m][k2] * W[k1*K2 + k2][n]        (complex, eq. S4)
// A and C are interleaved complex (re, im).  The complex product is done as a
// single real GEMM (the 4M scheme): the interleaved row of A (length 2K) times
// the real 2K x 2N expansion B' of W (packed on the host, stored transposed
// as P[n'][k']) yields the interleaved row of C.  B' has 4 real entries per
// complex entry of W, so the real GEMM does exactly the 8 real flops of a
// complex multiply-add.
//
// Tiling: 256 threads = 4 waves in a 2 x 2 grid; each wave owns a
// (BM/2) x (BN/2) block of real outputs held in MFMA accumulators.  Tiles of
// A (BM x BK) and P (BN x BK) are staged through LDS with double buffering:
// global loads for stage k+1 are issued before the MFMAs of stage k and
// written to the other LDS buffer afterwards, one barrier per stage.  Inside
// a stage each lane reads 16-byte fragments (4 consecutive k for FP32, 2 for
// FP64) so that one LDS read feeds several MFMAs; the k order inside a group
// of 8 is permuted identically for A and B, which leaves the sum unchanged.
//
// Workgroups are assigned XCD-aware: hardware dispatches workgroup b to XCD
// b mod 8, so tile t = (b mod 8) * ceil(T/8) + b / 8 gives each XCD a
// contiguous range of tiles, and the N-tiles of one M-block (which share the
// same rows of A) run on the same XCD and its L2.
//
// A-tile loaders: ROWMAJOR reads 16 bytes along k (needs an even K2 for
// FP32), KMAJOR reads along m when K2 == 1 (A stored as A[k][m]: the first
// site of a row) and transposes into LDS, GENERIC reads one complex at a time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>

#include "psim_internal.hpp"

namespace psim {

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// ROWFAST: ROWMAJOR for launches where every tile is interior (M % BM == 0,
// 2K % BK == 0) and a stage never straddles two k1 values (2 K2 % BK == 0):
// no bounds checks, one k1/k2 split per stage.
enum AMode { ROWMAJOR = 0, KMAJOR = 1, GENERIC = 2, ROWFAST = 3 };

struct KArgs {
  const void* A;
  void* C;
  const void* W0;
  const void* W1;
  const int32_t* a_index;
  const uint8_t* tau;
  long long tau_stride;
  long long M, K1, K2, N;
  long long K;        // complex K = K1 * K2
  long long Kr, Nr;   // real 2K, 2N
  long long ldw, w_koff_r;
  long long sA_node, sA_v, sC_node, sC_v;
  long long MT, NT, T;
  long long plane;    // BF16x3: elements between the hi and lo planes of W
  long long ldct;     // transposed stores: complex elements between rows n of C (M for a dense C^T)
  long long nb, sCw;  // nb > 0: plain stores split N into blocks of nb columns, block b at b * sCw
                      // (C[n / nb][m][n % nb]); 0: row-major C[m][n]
  int Bz, trans_out, beta;
};

// ---------------------------------------------------------------- traits
template <typename T>
struct Mfma;

template <>
struct Mfma<float> {
  static constexpr int MB = 32;       // block edge
  static constexpr int KPI = 2;       // k per instruction
  static constexpr int NACC = 16;     // accumulators per lane per block
  static constexpr int KV = 4;        // k per lane per group of 8
  typedef f32x16 acc_t;
  typedef f32x4 frag_t;
  __device__ static inline void mma(const frag_t& a, const frag_t& b, acc_t& c, int s) {
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], b[s], c, 0, 0, 0);
  }
  // row of output element r held by lane
  __device__ static inline int out_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }
  __device__ static inline int out_col(int lane) { return lane & 31; }
};

template <>
struct Mfma<double> {
  static constexpr int MB = 16;
  static constexpr int KPI = 4;
  static constexpr int NACC = 4;
  static constexpr int KV = 2;
  typedef f64x4 acc_t;
  typedef f64x2 frag_t;
  __device__ static inline void mma(const frag_t& a, const frag_t& b, acc_t& c, int s) {
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], c, 0, 0, 0);
  }
  // measured on gfx950: accumulator r of lane l holds row 4r + l/16, column l%16
  __device__ static inline int out_row(int lane, int r) { return 4 * r + (lane >> 4); }
  __device__ static inline int out_col(int lane) { return lane & 15; }
};

// 16-byte vector of T
template <typename T>
struct V16;
template <>
struct V16<float> { typedef f32x4 t; static constexpr int n = 4; };
template <>
struct V16<double> { typedef f64x2 t; static constexpr int n = 2; };

// ---------------------------------------------------------------- kernel
// SCH = 4: the 4M scheme above.  SCH = 3 (FP32 only): the Gauss 3M scheme,
//   T1 = Ar Wr, T2 = Ai Wi, T3 = (Ar + Ai)(Wr + Wi),  Re C = T1 - T2,  Im C = T3 - T1 - T2,
// three real MFMA products per complex multiply-add instead of four.  The
// LDS A tile is the same interleaved (re, im) tile; each lane reads four
// consecutive complex k (8 floats), splits re / im in registers and forms
// re + im there.  W is packed as P[n][2k] = Re W[k][n], P[n][2k+1] = Im W[k][n].
// SPLIT (FP32, 4M or 3M): each stage of BK real k accumulates into a fresh
// partial sum that is then added to the running accumulator, so the FP32
// rounding of the K-loop sum grows like sqrt(BK) + sqrt(K/BK) instead of
// sqrt(K) (about 3x smaller at K = 2048).
template <typename T, int BM, int BN, int BK, int AMODE, bool TRANS, int SCH, bool SPLIT>
__device__ __forceinline__ void site_gemm_body(const KArgs& p, const long long t) {
  typedef Mfma<T> MF;
  typedef typename V16<T>::t vec_t;
  static_assert(SCH == 4 || (SCH == 3 && sizeof(T) == 4), "3M is FP32 only");
  // transposed FP32 stores: compute C^T blocks so that lanes run along m and
  // each lane stores (Re, Im) pairs contiguous with its neighbours
  constexpr bool SWAP = TRANS && sizeof(T) == 4 && !SPLIT;
  constexpr int VN = V16<T>::n;          // reals per 16-byte vector
  constexpr int LDS_LD = BK + VN;        // padded row length (reals)
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int MBLK = WM / MF::MB, NBLK = WN / MF::MB;
  constexpr int NBLK3 = WN / 2 / MF::MB;  // 3M: complex columns per wave / 32
  constexpr int GROUPS = BK / 8;
  constexpr int BROWS = SCH == 4 ? BN : BN / 2;   // rows of the packed W per tile
  // A tile: BM x BK reals = BM * BK / VN vectors
  constexpr int A_VECS = BM * BK / VN / 256;
  constexpr int B_VECS = BROWS * BK / VN / 256;
  static_assert(A_VECS * VN * 256 == BM * BK, "A tile");
  static_assert(B_VECS * VN * 256 == BROWS * BK, "B tile");
  static_assert(SCH == 4 || (NBLK3 >= 1 && BK % 16 == 0), "3M tile");
  // GENERIC loader works on single complex numbers (2 reals)
  constexpr int A_CPLX = BM * BK / 2 / 256;

  __shared__ __attribute__((aligned(16))) T sA[2][BM * LDS_LD];
  __shared__ __attribute__((aligned(16))) T sB[2][BROWS * LDS_LD];

  const long long nt = t % p.NT;
  const long long rest = t / p.NT;
  const long long mt = rest % p.MT;
  const long long z = rest / p.MT;
  const long long node = z / p.Bz, vb = z % p.Bz;
  const long long ablk = p.a_index ? (long long)p.a_index[node] : node;
  const T* __restrict__ A = (const T*)p.A + 2 * (ablk * p.sA_node + vb * p.sA_v);
  const int tauv = p.tau ? (int)p.tau[node * p.tau_stride] : 0;
  const T* __restrict__ W = (const T*)(tauv ? p.W1 : p.W0) + p.w_koff_r;
  T* __restrict__ C = (T*)p.C + 2 * (node * p.sC_node + vb * p.sC_v);
  const long long m0 = mt * BM, n0 = nt * BN;
  const long long brow0 = nt * BROWS;  // first packed-W row of this tile

  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const long long sK1 = p.M * p.K2;    // complex stride of k1 in A
  const unsigned K2u = (unsigned)p.K2;

  vec_t ra[AMODE == GENERIC ? 1 : A_VECS];  // ROWMAJOR / ROWFAST / KMAJOR staging
  T rc[AMODE == GENERIC ? A_CPLX * 2 : 1];
  vec_t rb[B_VECS];

  // ROWFAST: (k1, k2) of the next stage, advanced one stage per load (stages
  // are loaded in order and never straddle a k1 block), so no division
  long long fk1 = 0, fk2 = 0;
  auto load_a = [&](long long kr0) {
    if constexpr (AMODE == ROWFAST) {
      const T* base = A + 2 * (fk1 * sK1 + m0 * p.K2 + fk2);
#pragma unroll
      for (int it = 0; it < A_VECS; ++it) {
        const int lin = it * 256 + tid;
        const int row = lin / (BK / VN), kq = lin % (BK / VN);
        ra[it] = *(const vec_t*)(base + 2 * (long long)row * p.K2 + kq * VN);
      }
      fk2 += BK / 2;
      if (fk2 == p.K2) {
        fk2 = 0;
        ++fk1;
      }
    } else if constexpr (AMODE == ROWMAJOR) {
#pragma unroll
      for (int it = 0; it < A_VECS; ++it) {
        const int lin = it * 256 + tid;
        const int row = lin / (BK / VN), kq = lin % (BK / VN);
        const long long m = m0 + row, kr = kr0 + kq * VN;
        vec_t v = {};
        if (m < p.M && kr < p.Kr) {
          const unsigned k = (unsigned)(kr >> 1);
          const unsigned k1 = k / K2u, k2 = k - k1 * K2u;
          v = *(const vec_t*)(A + 2 * ((long long)k1 * sK1 + m * p.K2 + k2));
        }
        ra[it] = v;
      }
    } else if constexpr (AMODE == KMAJOR) {
      // VN/2 complex along m per vector, BK/2 complex k per tile
      constexpr int CPV = VN / 2;
#pragma unroll
      for (int it = 0; it < A_VECS; ++it) {
        const int lin = it * 256 + tid;
        const int kk = lin / (BM / CPV), mp = lin % (BM / CPV);
        const long long m = m0 + mp * CPV, k = (kr0 >> 1) + kk;
        vec_t v = {};
        if (m < p.M && k < p.K) v = *(const vec_t*)(A + 2 * (k * p.M + m));
        ra[it] = v;
      }
    } else {
#pragma unroll
      for (int it = 0; it < A_CPLX; ++it) {
        const int lin = it * 256 + tid;
        const int row = lin / (BK / 2), kc = lin % (BK / 2);
        const long long m = m0 + row, k = (kr0 >> 1) + kc;
        T re = 0, im = 0;
        if (m < p.M && k < p.K) {
          const unsigned k1 = (unsigned)k / K2u, k2 = (unsigned)k - k1 * K2u;
          const T* q = A + 2 * ((long long)k1 * sK1 + m * p.K2 + k2);
          re = q[0];
          im = q[1];
        }
        rc[2 * it] = re;
        rc[2 * it + 1] = im;
      }
    }
  };
  auto store_a = [&](int buf) {
    T* s = sA[buf];
    if constexpr (AMODE == ROWMAJOR || AMODE == ROWFAST) {
#pragma unroll
      for (int it = 0; it < A_VECS; ++it) {
        const int lin = it * 256 + tid;
        const int row = lin / (BK / VN), kq = lin % (BK / VN);
        *(vec_t*)(s + row * LDS_LD + kq * VN) = ra[it];
      }
    } else if constexpr (AMODE == KMAJOR) {
      constexpr int CPV = VN / 2;
#pragma unroll
      for (int it = 0; it < A_VECS; ++it) {
        const int lin = it * 256 + tid;
        const int kk = lin / (BM / CPV), mp = lin % (BM / CPV);
#pragma unroll
        for (int c = 0; c < CPV; ++c) {
          s[(mp * CPV + c) * LDS_LD + 2 * kk] = ra[it][2 * c];
          s[(mp * CPV + c) * LDS_LD + 2 * kk + 1] = ra[it][2 * c + 1];
        }
      }
    } else {
#pragma unroll
      for (int it = 0; it < A_CPLX; ++it) {
        const int lin = it * 256 + tid;
        const int row = lin / (BK / 2), kc = lin % (BK / 2);
        s[row * LDS_LD + 2 * kc] = rc[2 * it];
        s[row * LDS_LD + 2 * kc + 1] = rc[2 * it + 1];
      }
    }
  };
  auto load_b = [&](long long kr0) {
#pragma unroll
    for (int it = 0; it < B_VECS; ++it) {
      const int lin = it * 256 + tid;
      const int row = lin / (BK / VN), kq = lin % (BK / VN);
      rb[it] = *(const vec_t*)(W + (brow0 + row) * p.ldw + kr0 + kq * VN);
    }
  };
  auto store_b = [&](int buf) {
    T* s = sB[buf];
#pragma unroll
    for (int it = 0; it < B_VECS; ++it) {
      const int lin = it * 256 + tid;
      const int row = lin / (BK / VN), kq = lin % (BK / VN);
      *(vec_t*)(s + row * LDS_LD + kq * VN) = rb[it];
    }
  };

  typename MF::acc_t acc[SCH == 4 ? MBLK : 1][SCH == 4 ? NBLK : 1];
  typename MF::acc_t acc3[SCH == 3 ? MBLK : 1][SCH == 3 ? NBLK3 : 1][3];
  if constexpr (SCH == 4) {
#pragma unroll
    for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
      for (int bj = 0; bj < NBLK; ++bj)
#pragma unroll
        for (int r = 0; r < MF::NACC; ++r) acc[bi][bj][r] = 0;
  } else {
#pragma unroll
    for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
      for (int bj = 0; bj < NBLK3; ++bj)
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
          for (int r = 0; r < MF::NACC; ++r) acc3[bi][bj][q][r] = 0;
  }

  const long long nk = (p.Kr + BK - 1) / BK;
  load_a(0);
  load_b(0);
  store_a(0);
  store_b(0);
  __syncthreads();

  // lane's fragment position inside a group of 8 k
  const int frow = lane % MF::MB;
  const int fk = (lane / MF::MB) * MF::KV;

  for (long long kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    const bool more = kt + 1 < nk;
    if (more) {
      load_a((kt + 1) * BK);
      load_b((kt + 1) * BK);
    }
    const T* a_s = sA[cur];
    const T* b_s = sB[cur];
    if constexpr (SCH == 4) {
      typename MF::acc_t part[SPLIT ? MBLK : 1][SPLIT ? NBLK : 1];
      if constexpr (SPLIT) {
#pragma unroll
        for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
          for (int bj = 0; bj < NBLK; ++bj)
#pragma unroll
            for (int r = 0; r < MF::NACC; ++r) part[bi][bj][r] = 0;
      }
#pragma unroll
      for (int g = 0; g < GROUPS; ++g) {
        typename MF::frag_t af[MBLK], bf[NBLK];
#pragma unroll
        for (int bi = 0; bi < MBLK; ++bi)
          af[bi] = *(const typename MF::frag_t*)(a_s + (wr * WM + bi * MF::MB + frow) * LDS_LD + g * 8 + fk);
#pragma unroll
        for (int bj = 0; bj < NBLK; ++bj)
          bf[bj] = *(const typename MF::frag_t*)(b_s + (wc * WN + bj * MF::MB + frow) * LDS_LD + g * 8 + fk);
#pragma unroll
        for (int s = 0; s < MF::KV; ++s)
#pragma unroll
          for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
            for (int bj = 0; bj < NBLK; ++bj) {
              if constexpr (SPLIT)
                MF::mma(af[bi], bf[bj], part[bi][bj], s);
              else if constexpr (SWAP)
                MF::mma(bf[bj], af[bi], acc[bi][bj], s);  // block holds C^T: rows n', columns m
              else
                MF::mma(af[bi], bf[bj], acc[bi][bj], s);
            }
      }
      if constexpr (SPLIT) {
#pragma unroll
        for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
          for (int bj = 0; bj < NBLK; ++bj) acc[bi][bj] += part[bi][bj];
      }
    } else {
      // groups of 8 complex k (16 floats); lane half h covers complex k 4h .. 4h+3
      const int f8 = (lane / MF::MB) * 8;
      // SPLIT: this stage's three products summed apart, then added to acc3
      typename MF::acc_t part3[SPLIT ? MBLK : 1][SPLIT ? NBLK3 : 1][3];
      auto& tgt = [&]() -> auto& {
        if constexpr (SPLIT) return part3;
        else return acc3;
      }();
      if constexpr (SPLIT) {
#pragma unroll
        for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
          for (int bj = 0; bj < NBLK3; ++bj)
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
              for (int r = 0; r < MF::NACC; ++r) part3[bi][bj][q][r] = 0;
      }
#pragma unroll
      for (int g = 0; g < BK / 16; ++g) {
        f32x4 ar[MBLK], ai[MBLK], as[MBLK], br[NBLK3], bim[NBLK3], bs[NBLK3];
#pragma unroll
        for (int bi = 0; bi < MBLK; ++bi) {
          const T* q = a_s + (wr * WM + bi * MF::MB + frow) * LDS_LD + g * 16 + f8;
          const f32x4 x0 = *(const f32x4*)q, x1 = *(const f32x4*)(q + 4);
          ar[bi] = f32x4{x0[0], x0[2], x1[0], x1[2]};
          ai[bi] = f32x4{x0[1], x0[3], x1[1], x1[3]};
          as[bi] = ar[bi] + ai[bi];
        }
#pragma unroll
        for (int bj = 0; bj < NBLK3; ++bj) {
          const T* q = b_s + (wc * (WN / 2) + bj * MF::MB + frow) * LDS_LD + g * 16 + f8;
          const f32x4 x0 = *(const f32x4*)q, x1 = *(const f32x4*)(q + 4);
          br[bj] = f32x4{x0[0], x0[2], x1[0], x1[2]};
          bim[bj] = f32x4{x0[1], x0[3], x1[1], x1[3]};
          bs[bj] = br[bj] + bim[bj];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
            for (int bj = 0; bj < NBLK3; ++bj) {
              if constexpr (SWAP) {  // C^T blocks: rows n, columns m
                tgt[bi][bj][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(br[bj][s], ar[bi][s], tgt[bi][bj][0], 0, 0, 0);
                tgt[bi][bj][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(bim[bj][s], ai[bi][s], tgt[bi][bj][1], 0, 0, 0);
                tgt[bi][bj][2] = __builtin_amdgcn_mfma_f32_32x32x2f32(bs[bj][s], as[bi][s], tgt[bi][bj][2], 0, 0, 0);
              } else {
                tgt[bi][bj][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[bi][s], br[bj][s], tgt[bi][bj][0], 0, 0, 0);
                tgt[bi][bj][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[bi][s], bim[bj][s], tgt[bi][bj][1], 0, 0, 0);
                tgt[bi][bj][2] = __builtin_amdgcn_mfma_f32_32x32x2f32(as[bi][s], bs[bj][s], tgt[bi][bj][2], 0, 0, 0);
              }
            }
      }
      if constexpr (SPLIT) {
#pragma unroll
        for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
          for (int bj = 0; bj < NBLK3; ++bj)
#pragma unroll
            for (int q = 0; q < 3; ++q) acc3[bi][bj][q] += part3[bi][bj][q];
      }
    }
    if (more) {
      store_a(cur ^ 1);
      store_b(cur ^ 1);
    }
    __syncthreads();
  }

  // ------------------------------------------------------------ epilogue
  if constexpr (SWAP && SCH == 4) {
    // block (bi, bj) holds C^T: lane -> m, registers r / r+1 -> (Re, Im) of one n
#pragma unroll
    for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
      for (int bj = 0; bj < NBLK; ++bj)
#pragma unroll
        for (int r = 0; r < MF::NACC; r += 2) {
          const long long m = m0 + wr * WM + bi * MF::MB + (lane & 31);
          const long long nr = n0 + wc * WN + bj * MF::MB + MF::out_row(lane, r);  // even
          if (m < p.M && nr < p.Nr) {
            f32x2 v = {acc[bi][bj][r], acc[bi][bj][r + 1]};
            f32x2* dst = (f32x2*)(C + 2 * ((nr >> 1) * p.ldct + m));
            if (p.beta) v += *dst;
            *dst = v;
          }
        }
  } else if constexpr (SWAP && SCH == 3) {
    const long long c0 = n0 / 2;
#pragma unroll
    for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
      for (int bj = 0; bj < NBLK3; ++bj)
#pragma unroll
        for (int r = 0; r < MF::NACC; ++r) {
          const long long m = m0 + wr * WM + bi * MF::MB + (lane & 31);
          const long long n = c0 + wc * (WN / 2) + bj * MF::MB + MF::out_row(lane, r);
          if (m < p.M && n < p.N) {
            const T t1 = acc3[bi][bj][0][r], t2 = acc3[bi][bj][1][r], t3 = acc3[bi][bj][2][r];
            f32x2 v = {t1 - t2, t3 - t1 - t2};
            f32x2* dst = (f32x2*)(C + 2 * (n * p.ldct + m));
            if (p.beta) v += *dst;
            *dst = v;
          }
        }
  } else if constexpr (SCH == 4) {
#pragma unroll
    for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
      for (int bj = 0; bj < NBLK; ++bj)
#pragma unroll
        for (int r = 0; r < MF::NACC; ++r) {
          const long long row = m0 + wr * WM + bi * MF::MB + MF::out_row(lane, r);
          const long long col = n0 + wc * WN + bj * MF::MB + MF::out_col(lane);
          if (row < p.M && col < p.Nr) {
            const T v = acc[bi][bj][r];
            if constexpr (!TRANS) {
              if (p.nb) {
                const long long cc = col >> 1;
                C[2 * ((cc / p.nb) * p.sCw + row * p.nb + cc % p.nb) + (col & 1)] = v;
              } else {
                C[row * p.Nr + col] = v;
              }
            } else {
              T* dst = C + 2 * ((col >> 1) * p.ldct + row) + (col & 1);
              *dst = p.beta ? *dst + v : v;
            }
          }
        }
  } else {
    const long long c0 = n0 / 2;  // first complex column of the tile
#pragma unroll
    for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
      for (int bj = 0; bj < NBLK3; ++bj)
#pragma unroll
        for (int r = 0; r < MF::NACC; ++r) {
          const long long row = m0 + wr * WM + bi * MF::MB + MF::out_row(lane, r);
          const long long col = c0 + wc * (WN / 2) + bj * MF::MB + MF::out_col(lane);
          if (row < p.M && col < p.N) {
            const T t1 = acc3[bi][bj][0][r], t2 = acc3[bi][bj][1][r], t3 = acc3[bi][bj][2][r];
            f32x2 v = {t1 - t2, t3 - t1 - t2};
            f32x2* dst = (f32x2*)(C + 2 * (TRANS  ? col * p.ldct + row
                                           : p.nb ? (col / p.nb) * p.sCw + row * p.nb + col % p.nb
                                                  : row * p.N + col));
            if constexpr (TRANS) {
              if (p.beta) v += *dst;
            }
            *dst = v;
          }
        }
  }
}

// XCD-aware tile order: workgroup b runs on XCD b mod 8; tile
// (b mod 8) * ceil(T/8) + b / 8 gives each XCD a contiguous range of tiles.
__device__ __forceinline__ long long xcd_tile(long long T) {
  const long long per_xcd = (T + 7) / 8;
  const long long bid = blockIdx.x;
  return (bid % 8) * per_xcd + bid / 8;
}

template <typename T, int BM, int BN, int BK, int AMODE, bool TRANS, int SCH>
__global__ __launch_bounds__(256) void site_gemm(KArgs p) {
  const long long t = xcd_tile(p.T);
  if (t >= p.T) return;
  site_gemm_body<T, BM, BN, BK, AMODE, TRANS, SCH, false>(p, t);
}

// split-accumulation variant, held to two waves per SIMD
template <typename T, int BM, int BN, int BK, int AMODE, bool TRANS, int SCH>
__global__ __launch_bounds__(256, 2) void site_gemm_split(KArgs p) {
  const long long t = xcd_tile(p.T);
  if (t >= p.T) return;
  site_gemm_body<T, BM, BN, BK, AMODE, TRANS, SCH, true>(p, t);
}

// Grouped launch: one grid over the tiles of several independent problems
// (site contractions of different circuits).  Problem i owns global tiles
// [start[i], start[i+1]); the descriptors live in device memory, their
// addresses and the tile offsets travel in the kernel arguments.  Every
// workgroup finds its problem by a binary search over uniform values and
// reads the descriptor into scalar registers.
constexpr int kMaxGroup = 32;
struct GroupArgs {
  const KArgs* probs[kMaxGroup];
  long long start[kMaxGroup + 1];  // start[nprob] = total tiles
  int nprob;
};

__device__ __forceinline__ int find_problem(const GroupArgs& ga, long long g) {
  int lo = 0, hi = ga.nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ga.start[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

template <typename T, int BM, int BN, int BK, int AMODE, bool TRANS, int SCH>
__global__ __launch_bounds__(256) void site_gemm_group(GroupArgs ga) {
  const long long total = ga.start[ga.nprob];
  const long long g = xcd_tile(total);
  if (g >= total) return;
  const int i = find_problem(ga, g);
  KArgs p;
  const int* src = (const int*)ga.probs[i];
  int* dst = (int*)&p;
#pragma unroll
  for (int w = 0; w < (int)(sizeof(KArgs) / 4); ++w) dst[w] = __builtin_amdgcn_readfirstlane(src[w]);
  site_gemm_body<T, BM, BN, BK, AMODE, TRANS, SCH, false>(p, g - ga.start[i]);
}

// ---------------------------------------------------------------- 3M, direct-to-LDS
// The 3M interior-site contraction for launches where every tile is interior
// and every stage lies inside one k1 block (the ROWFAST conditions), with
// operands copied global -> LDS by the load unit itself
// (global_load_lds_dwordx4): no register staging and no LDS store
// instructions.  Each wave-wide copy writes 64 x 16 bytes contiguously, so the
// LDS tiles are unpadded rows of BK floats (8 chunks of 16 bytes) and the lane
// that fills physical chunk p of row r fetches logical chunk p ^ swz(r); the
// fragment reads apply the same permutation, which spreads 16 consecutive
// rows over distinct banks.  The two LDS buffers are separate arrays and the
// K loop is unrolled by two, so each copy and each read names its buffer.
#define PSIM_LDS(p) ((__attribute__((address_space(3))) void*)(p))

__device__ __forceinline__ int dtl_swz(int r) { return (r ^ (r >> 3)) & 7; }

template <int BM, int BN, bool SPLIT = false>
__device__ __forceinline__ void dtl3m_body(const KArgs& p, const long long t) {
  constexpr int BK = 32;                 // floats per stage row = 8 chunks
  constexpr int MB = 32;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int MBLK = WM / MB;
  constexpr int NBLK3 = WN / 2 / MB;
  constexpr int BROWS = BN / 2;          // packed-W rows (complex columns) per tile
  constexpr int A_INS = BM * BK / 4 / 64 / 4;     // wave-wide 1 KB copies per wave
  constexpr int B_INS = BROWS * BK / 4 / 64 / 4;
  static_assert(A_INS >= 1 && B_INS >= 1 && NBLK3 >= 1, "tile");
  __shared__ __attribute__((aligned(1024))) float sA0[BM * BK];
  __shared__ __attribute__((aligned(1024))) float sA1[BM * BK];
  __shared__ __attribute__((aligned(1024))) float sB0[BROWS * BK];
  __shared__ __attribute__((aligned(1024))) float sB1[BROWS * BK];

  const long long nt = t % p.NT;
  const long long rest = t / p.NT;
  const long long mt = rest % p.MT;
  const long long z = rest / p.MT;
  const long long node = z / p.Bz, vb = z % p.Bz;
  const long long ablk = p.a_index ? (long long)p.a_index[node] : node;
  const float* __restrict__ A = (const float*)p.A + 2 * (ablk * p.sA_node + vb * p.sA_v);
  const int tauv = p.tau ? (int)p.tau[node * p.tau_stride] : 0;
  const float* __restrict__ W = (const float*)(tauv ? p.W1 : p.W0) + p.w_koff_r;
  float* __restrict__ C = (float*)p.C + 2 * (node * p.sC_node + vb * p.sC_v);
  const long long m0 = mt * BM;
  const long long brow0 = nt * BROWS;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const long long sK1 = p.M * p.K2;

  // Copy `it` of this wave fills tile rows (it * 4 + wid) * 8 + lane / 8,
  // physical chunk lane % 8; the lane fetches logical chunk p ^ swz(row).
  // Byte offsets from the uniform stage base stay below 2^31.
  const unsigned a_rs = (unsigned)(2 * p.K2 * 4);  // bytes between rows of A
  const unsigned b_rs = (unsigned)(p.ldw * 4);     // bytes between rows of packed W
  auto src_off = [&](int it, unsigned row_stride) {
    const int row = (it * 4 + wid) * 8 + (lane >> 3);
    const int chk = (lane & 7) ^ dtl_swz(row);
    return (unsigned)row * row_stride + (unsigned)chk * 16u;
  };
  long long fk1 = 0, fk2 = 0, kr = 0;  // next stage: (k1, k2) of A, real k of W
  auto issue = [&](float* sa, float* sb) {
    const char* abase = (const char*)(A + 2 * (fk1 * sK1 + m0 * p.K2 + fk2));
    const char* bbase = (const char*)(W + brow0 * p.ldw + kr);
#pragma unroll
    for (int it = 0; it < A_INS; ++it)
      __builtin_amdgcn_global_load_lds((const void*)(abase + src_off(it, a_rs)), PSIM_LDS(sa + (it * 4 + wid) * 256),
                                       16, 0, 0);
#pragma unroll
    for (int it = 0; it < B_INS; ++it)
      __builtin_amdgcn_global_load_lds((const void*)(bbase + src_off(it, b_rs)), PSIM_LDS(sb + (it * 4 + wid) * 256),
                                       16, 0, 0);
    fk2 += BK / 2;
    if (fk2 == p.K2) {
      fk2 = 0;
      ++fk1;
    }
    kr += BK;
  };

  f32x16 acc3[MBLK][NBLK3][3];
#pragma unroll
  for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
    for (int bj = 0; bj < NBLK3; ++bj)
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc3[bi][bj][q][r] = 0;
  // SPLIT: the products of each pair of stages (64 reals of k) are summed on
  // their own (fresh partial accumulators, opened by the pair's first stage)
  // and then added to the running sums (by its second), which shortens the
  // FP32 rounding chains of the K loop
  f32x16 part[SPLIT ? MBLK : 1][SPLIT ? NBLK3 : 1][SPLIT ? 3 : 1];

  const int frow = lane % MB;
  const int fh = (lane / MB) * 2;  // first logical chunk of this lane half within a group of 4
  auto compute = [&](const float* a_s, const float* b_s, const bool open, const bool close) {
    if (SPLIT && open) {
#pragma unroll
      for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
        for (int bj = 0; bj < NBLK3; ++bj)
#pragma unroll
          for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int r = 0; r < 16; ++r) part[bi][bj][q][r] = 0;
    }
    auto& dst = [&]() -> auto& {
      if constexpr (SPLIT) return part;
      else return acc3;
    }();
#pragma unroll
    for (int g = 0; g < BK / 16; ++g) {
      f32x4 ar[MBLK], ai[MBLK], as[MBLK], br[NBLK3], bim[NBLK3], bs[NBLK3];
#pragma unroll
      for (int bi = 0; bi < MBLK; ++bi) {
        const int r = wr * WM + bi * MB + frow;
        const int c0 = g * 4 + fh, sw = dtl_swz(r);
        const f32x4 x0 = *(const f32x4*)(a_s + r * BK + ((c0 ^ sw) << 2));
        const f32x4 x1 = *(const f32x4*)(a_s + r * BK + (((c0 + 1) ^ sw) << 2));
        ar[bi] = f32x4{x0[0], x0[2], x1[0], x1[2]};
        ai[bi] = f32x4{x0[1], x0[3], x1[1], x1[3]};
        as[bi] = ar[bi] + ai[bi];
      }
#pragma unroll
      for (int bj = 0; bj < NBLK3; ++bj) {
        const int r = wc * (WN / 2) + bj * MB + frow;
        const int c0 = g * 4 + fh, sw = dtl_swz(r);
        const f32x4 x0 = *(const f32x4*)(b_s + r * BK + ((c0 ^ sw) << 2));
        const f32x4 x1 = *(const f32x4*)(b_s + r * BK + (((c0 + 1) ^ sw) << 2));
        br[bj] = f32x4{x0[0], x0[2], x1[0], x1[2]};
        bim[bj] = f32x4{x0[1], x0[3], x1[1], x1[3]};
        bs[bj] = br[bj] + bim[bj];
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
          for (int bj = 0; bj < NBLK3; ++bj) {
            dst[bi][bj][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[bi][s], br[bj][s], dst[bi][bj][0], 0, 0, 0);
            dst[bi][bj][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[bi][s], bim[bj][s], dst[bi][bj][1], 0, 0, 0);
            dst[bi][bj][2] = __builtin_amdgcn_mfma_f32_32x32x2f32(as[bi][s], bs[bj][s], dst[bi][bj][2], 0, 0, 0);
          }
    }
    if (SPLIT && close) {
#pragma unroll
      for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
        for (int bj = 0; bj < NBLK3; ++bj)
#pragma unroll
          for (int q = 0; q < 3; ++q) acc3[bi][bj][q] += part[bi][bj][q];
    }
  };
  // vmcnt(0), other counters unconstrained: the copies into LDS have landed
  constexpr unsigned kWaitVm0 = 0x3f70;

  // the launcher guarantees an even number of stages
  const int npair = (int)(p.Kr / (2 * BK));
  issue(sA0, sB0);
  __builtin_amdgcn_s_waitcnt(kWaitVm0);
  __syncthreads();
  for (int kp = 0; kp < npair; ++kp) {
    issue(sA1, sB1);
    compute(sA0, sB0, true, false);
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
    if (kp + 1 < npair) issue(sA0, sB0);
    compute(sA1, sB1, false, true);
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
  }

  const long long c0 = nt * (BN / 2);  // first complex column of the tile
#pragma unroll
  for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
    for (int bj = 0; bj < NBLK3; ++bj)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const long long row = m0 + wr * WM + bi * MB + Mfma<float>::out_row(lane, r);
        const long long col = c0 + wc * (WN / 2) + bj * MB + Mfma<float>::out_col(lane);
        if (col < p.N) {
          const float t1 = acc3[bi][bj][0][r], t2 = acc3[bi][bj][1][r], t3 = acc3[bi][bj][2][r];
          f32x2 v = {t1 - t2, t3 - t1 - t2};
          *(f32x2*)(C + 2 * (row * p.N + col)) = v;
        }
      }
}

template <int BM, int BN>
__global__ __launch_bounds__(256, 3) void site_gemm_3m_dtl(KArgs p) {
  const long long t = xcd_tile(p.T);
  if (t >= p.T) return;
  dtl3m_body<BM, BN>(p, t);
}

// split-accumulation form (PSIM_PLAN_SPLIT_ACC): twice the accumulators, two
// workgroups per CU
template <int BM, int BN, int OCC = 2>
__global__ __launch_bounds__(256, OCC) void site_gemm_3m_dtl_split(KArgs p) {
  const long long t = xcd_tile(p.T);
  if (t >= p.T) return;
  dtl3m_body<BM, BN, true>(p, t);
}

// grouped form (see site_gemm_group)
template <int BM, int BN>
__global__ __launch_bounds__(256, 3) void site_gemm_3m_dtl_group(GroupArgs ga) {
  const long long total = ga.start[ga.nprob];
  const long long g = xcd_tile(total);
  if (g >= total) return;
  const int i = find_problem(ga, g);
  KArgs p;
  const int* src = (const int*)ga.probs[i];
  int* dst = (int*)&p;
#pragma unroll
  for (int w = 0; w < (int)(sizeof(KArgs) / 4); ++w) dst[w] = __builtin_amdgcn_readfirstlane(src[w]);
  dtl3m_body<BM, BN>(p, g - ga.start[i]);
}

// ---------------------------------------------------------------- 4M, direct-to-LDS
// 4M form of the direct-to-LDS interior kernel (FP32 on v_mfma_f32_32x32x2f32,
// FP64 on v_mfma_f64_16x16x4f64): the real expansion of the complex product,
// stage rows of 128 bytes (32 floats or 16 doubles: the same chunks and
// swizzle as above), BM x BN real outputs per workgroup.  A lane's fragment
// (KV consecutive k) is one 16-byte chunk.  The products and their order are
// those of the row-major kernel with the same tile.
template <typename T, int BM, int BN, int OCC>
__global__ __launch_bounds__(256, OCC) void site_gemm_4m_dtl(KArgs p) {
  typedef Mfma<T> MF;
  constexpr int BK = 128 / (int)sizeof(T);  // elements per stage row = 8 chunks
  constexpr int KV = MF::KV;                 // elements per chunk
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int MBLK = WM / MF::MB, NBLK = WN / MF::MB;
  constexpr int A_INS = BM * 128 / 1024 / 4;
  constexpr int B_INS = BN * 128 / 1024 / 4;
  static_assert(A_INS >= 1 && B_INS >= 1 && MBLK >= 1 && NBLK >= 1, "tile");
  static_assert(KV * (int)sizeof(T) == 16, "one chunk per fragment");
  __shared__ __attribute__((aligned(1024))) T sA0[BM * BK];
  __shared__ __attribute__((aligned(1024))) T sA1[BM * BK];
  __shared__ __attribute__((aligned(1024))) T sB0[BN * BK];
  __shared__ __attribute__((aligned(1024))) T sB1[BN * BK];

  const long long t = xcd_tile(p.T);
  if (t >= p.T) return;
  const long long nt = t % p.NT;
  const long long rest = t / p.NT;
  const long long mt = rest % p.MT;
  const long long z = rest / p.MT;
  const long long node = z / p.Bz, vb = z % p.Bz;
  const long long ablk = p.a_index ? (long long)p.a_index[node] : node;
  const T* __restrict__ A = (const T*)p.A + 2 * (ablk * p.sA_node + vb * p.sA_v);
  const int tauv = p.tau ? (int)p.tau[node * p.tau_stride] : 0;
  const T* __restrict__ W = (const T*)(tauv ? p.W1 : p.W0) + p.w_koff_r;
  T* __restrict__ C = (T*)p.C + 2 * (node * p.sC_node + vb * p.sC_v);
  const long long m0 = mt * BM, n0 = nt * BN;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const long long sK1 = p.M * p.K2;
  const unsigned a_rs = (unsigned)(2 * p.K2 * (long long)sizeof(T));
  const unsigned b_rs = (unsigned)(p.ldw * (long long)sizeof(T));
  auto src_off = [&](int it, unsigned row_stride) {
    const int row = (it * 4 + wid) * 8 + (lane >> 3);
    const int chk = (lane & 7) ^ dtl_swz(row);
    return (unsigned)row * row_stride + (unsigned)chk * 16u;
  };
  long long fk1 = 0, fk2 = 0, kr = 0;
  auto issue = [&](T* sa, T* sb) {
    const char* abase = (const char*)(A + 2 * (fk1 * sK1 + m0 * p.K2 + fk2));
    const char* bbase = (const char*)(W + n0 * p.ldw + kr);
#pragma unroll
    for (int it = 0; it < A_INS; ++it)
      __builtin_amdgcn_global_load_lds((const void*)(abase + src_off(it, a_rs)), PSIM_LDS(sa + (it * 4 + wid) * (1024 / (int)sizeof(T))),
                                       16, 0, 0);
#pragma unroll
    for (int it = 0; it < B_INS; ++it)
      __builtin_amdgcn_global_load_lds((const void*)(bbase + src_off(it, b_rs)), PSIM_LDS(sb + (it * 4 + wid) * (1024 / (int)sizeof(T))),
                                       16, 0, 0);
    fk2 += BK / 2;
    if (fk2 == p.K2) {
      fk2 = 0;
      ++fk1;
    }
    kr += BK;
  };

  typename MF::acc_t acc[MBLK][NBLK];
#pragma unroll
  for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
    for (int bj = 0; bj < NBLK; ++bj)
#pragma unroll
      for (int r = 0; r < MF::NACC; ++r) acc[bi][bj][r] = 0;

  const int frow = lane % MF::MB;
  const int fq = lane / MF::MB;  // which chunk of a group of 8 k this lane reads
  auto compute = [&](const T* a_s, const T* b_s) {
#pragma unroll
    for (int g = 0; g < BK / 8; ++g) {
      typename MF::frag_t af[MBLK], bf[NBLK];
#pragma unroll
      for (int bi = 0; bi < MBLK; ++bi) {
        const int r = wr * WM + bi * MF::MB + frow;
        af[bi] = *(const typename MF::frag_t*)(a_s + r * BK + (((g * (8 / KV) + fq) ^ dtl_swz(r)) * KV));
      }
#pragma unroll
      for (int bj = 0; bj < NBLK; ++bj) {
        const int r = wc * WN + bj * MF::MB + frow;
        bf[bj] = *(const typename MF::frag_t*)(b_s + r * BK + (((g * (8 / KV) + fq) ^ dtl_swz(r)) * KV));
      }
#pragma unroll
      for (int s = 0; s < MF::KV; ++s)
#pragma unroll
        for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
          for (int bj = 0; bj < NBLK; ++bj) MF::mma(af[bi], bf[bj], acc[bi][bj], s);
    }
  };
  constexpr unsigned kWaitVm0 = 0x3f70;

  const int npair = (int)(p.Kr / (2 * BK));
  issue(sA0, sB0);
  __builtin_amdgcn_s_waitcnt(kWaitVm0);
  __syncthreads();
  for (int kp = 0; kp < npair; ++kp) {
    issue(sA1, sB1);
    compute(sA0, sB0);
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
    if (kp + 1 < npair) issue(sA0, sB0);
    compute(sA1, sB1);
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
  }

#pragma unroll
  for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
    for (int bj = 0; bj < NBLK; ++bj)
#pragma unroll
      for (int r = 0; r < MF::NACC; ++r) {
        const long long row = m0 + wr * WM + bi * MF::MB + MF::out_row(lane, r);
        const long long col = n0 + wc * WN + bj * MF::MB + MF::out_col(lane);
        if (col < p.Nr) C[row * p.Nr + col] = acc[bi][bj][r];
      }
}

// ---------------------------------------------------------------- BF16x3
// Split-precision variant of the 4M kernel for row-major A and a plain store:
// every FP32 operand x is split as x = hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) (round to nearest even), and
//   a b ~= a_hi b_hi + a_hi b_lo + a_lo b_hi
// is accumulated in FP32 with v_mfma_f32_32x32x16_bf16 (the a_lo b_lo term,
// ~2^-18 relative, is dropped).  W arrives pre-split (two bf16 planes of the
// transposed 4M expansion); A is split while it is staged into LDS.  Lane
// half h of a 32x32x16 MFMA supplies 8 consecutive k (k = 8h .. 8h+7).
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int BM, int BN, bool FAST>
__global__ __launch_bounds__(256) void site_gemm_bf16x3(KArgs p) {
  constexpr int BK = 16;                 // reals per stage: one MFMA k-step
  constexpr int LD = BK + 8;             // padded LDS row (bf16), 48 bytes
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int MBLK = WM / 32, NBLK = WN / 32;
  constexpr int A_VECS = BM * BK / 4 / 256;     // float4 loads of A per thread
  constexpr int B_VECS = BN * BK / 8 / 256;     // 16-byte loads per bf16 plane per thread
  static_assert(A_VECS >= 1 && A_VECS * 4 * 256 == BM * BK, "A tile");
  static_assert(B_VECS >= 1 && B_VECS * 8 * 256 == BN * BK, "B tile");

  __shared__ __attribute__((aligned(16))) __bf16 sAh[2][BM * LD];
  __shared__ __attribute__((aligned(16))) __bf16 sAl[2][BM * LD];
  __shared__ __attribute__((aligned(16))) __bf16 sBh[2][BN * LD];
  __shared__ __attribute__((aligned(16))) __bf16 sBl[2][BN * LD];

  const long long per_xcd = (p.T + 7) / 8;
  const long long bid = blockIdx.x;
  const long long t = (bid % 8) * per_xcd + bid / 8;
  if (t >= p.T) return;
  const long long nt = t % p.NT;
  const long long rest = t / p.NT;
  const long long mt = rest % p.MT;
  const long long z = rest / p.MT;
  const long long node = z / p.Bz, vb = z % p.Bz;
  const long long ablk = p.a_index ? (long long)p.a_index[node] : node;
  const float* __restrict__ A = (const float*)p.A + 2 * (ablk * p.sA_node + vb * p.sA_v);
  const int tauv = p.tau ? (int)p.tau[node * p.tau_stride] : 0;
  // bf16 planes: hi at W, lo at W + plane (elements); p.ldw is the row length in bf16
  const __bf16* __restrict__ Wh = (const __bf16*)(tauv ? p.W1 : p.W0) + p.w_koff_r;
  const __bf16* __restrict__ Wl = Wh + p.plane;
  float* __restrict__ C = (float*)p.C + 2 * (node * p.sC_node + vb * p.sC_v);
  const long long m0 = mt * BM, n0 = nt * BN;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const long long sK1 = p.M * p.K2;
  const unsigned K2u = (unsigned)p.K2;

  // Staging registers, two sets: the global loads run two stages ahead of
  // the MFMAs (stage s is loaded into set s % 2), so a load has about two
  // stages of MFMA work to arrive before its data is converted and stored.
  struct Stage {
    f32x4 a[A_VECS];
    f32x4 bh[B_VECS], bl[B_VECS];  // 16 bytes = 8 bf16 each
  };
  Stage set0, set1;

  long long fk1 = 0, fk2 = 0;  // FAST: next stage's (k1, k2), as in ROWFAST; loads are issued in stage order
  auto load = [&](long long kr0, Stage& r) {
    if constexpr (FAST) {  // interior tile, stage inside one k1 (see ROWFAST)
      const float* base = A + 2 * (fk1 * sK1 + m0 * p.K2 + fk2);
#pragma unroll
      for (int it = 0; it < A_VECS; ++it) {
        const int lin = it * 256 + tid;
        const int row = lin / (BK / 4), kq = lin % (BK / 4);
        r.a[it] = *(const f32x4*)(base + 2 * (long long)row * p.K2 + kq * 4);
      }
      fk2 += BK / 2;
      if (fk2 == p.K2) {
        fk2 = 0;
        ++fk1;
      }
    } else {
#pragma unroll
      for (int it = 0; it < A_VECS; ++it) {
        const int lin = it * 256 + tid;
        const int row = lin / (BK / 4), kq = lin % (BK / 4);
        const long long m = m0 + row, kr = kr0 + kq * 4;
        f32x4 v = {};
        if (m < p.M && kr < p.Kr) {
          const unsigned k = (unsigned)(kr >> 1);
          const unsigned k1 = k / K2u, k2 = k - k1 * K2u;
          v = *(const f32x4*)(A + 2 * ((long long)k1 * sK1 + m * p.K2 + k2));
        }
        r.a[it] = v;
      }
    }
#pragma unroll
    for (int it = 0; it < B_VECS; ++it) {
      const int lin = it * 256 + tid;
      const int row = lin / (BK / 8), kq = lin % (BK / 8);
      const long long off = (n0 + row) * p.ldw + kr0 + kq * 8;
      r.bh[it] = *(const f32x4*)(Wh + off);
      r.bl[it] = *(const f32x4*)(Wl + off);
    }
  };
  auto store = [&](int buf, const Stage& r) {
#pragma unroll
    for (int it = 0; it < A_VECS; ++it) {
      const int lin = it * 256 + tid;
      const int row = lin / (BK / 4), kq = lin % (BK / 4);
      bf16x4 hi, lo;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        hi[e] = (__bf16)r.a[it][e];
        lo[e] = (__bf16)(r.a[it][e] - (float)hi[e]);
      }
      *(bf16x4*)(&sAh[buf][row * LD + kq * 4]) = hi;
      *(bf16x4*)(&sAl[buf][row * LD + kq * 4]) = lo;
    }
#pragma unroll
    for (int it = 0; it < B_VECS; ++it) {
      const int lin = it * 256 + tid;
      const int row = lin / (BK / 8), kq = lin % (BK / 8);
      *(f32x4*)(&sBh[buf][row * LD + kq * 8]) = r.bh[it];
      *(f32x4*)(&sBl[buf][row * LD + kq * 8]) = r.bl[it];
    }
  };

  f32x16 acc[MBLK][NBLK];
#pragma unroll
  for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
    for (int bj = 0; bj < NBLK; ++bj)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[bi][bj][r] = 0;

  const long long nk = (p.Kr + BK - 1) / BK;
  load(0, set0);
  store(0, set0);
  if (nk > 1) load(BK, set1);
  __syncthreads();
  const int frow = lane & 31, fk = (lane >> 5) * 8;
  // One stage: its fragments come from LDS buffer kt & 1; NEXT holds stage
  // kt + 1 (stored into the other buffer halfway through the MFMAs, where the
  // conversion and the LDS stores overlap the matrix work), FREE receives the
  // loads of stage kt + 2.  Each accumulator sees its products in the same
  // order as with one staging set.
#define PSIM_BF16X3_STAGE(KT, NEXT, FREE)                                                                   \
  {                                                                                                       \
    const long long kt_ = (KT);                                                                           \
    const int cur = (int)(kt_ & 1);                                                                       \
    if (kt_ + 2 < nk) load((kt_ + 2) * BK, FREE);                                                         \
    bf16x8 ah[MBLK], al[MBLK], bh[NBLK], bl[NBLK];                                                        \
    _Pragma("unroll") for (int bi = 0; bi < MBLK; ++bi) {                                                 \
      const int o = (wr * WM + bi * 32 + frow) * LD + fk;                                                 \
      ah[bi] = *(const bf16x8*)(&sAh[cur][o]);                                                            \
      al[bi] = *(const bf16x8*)(&sAl[cur][o]);                                                            \
    }                                                                                                     \
    _Pragma("unroll") for (int bj = 0; bj < NBLK; ++bj) {                                                 \
      const int o = (wc * WN + bj * 32 + frow) * LD + fk;                                                 \
      bh[bj] = *(const bf16x8*)(&sBh[cur][o]);                                                            \
      bl[bj] = *(const bf16x8*)(&sBl[cur][o]);                                                            \
    }                                                                                                     \
    _Pragma("unroll") for (int bi = 0; bi < MBLK / 2; ++bi)                                               \
      _Pragma("unroll") for (int bj = 0; bj < NBLK; ++bj) {                                               \
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[bi], bh[bj], acc[bi][bj], 0, 0, 0);      \
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[bi], bl[bj], acc[bi][bj], 0, 0, 0);      \
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[bi], bh[bj], acc[bi][bj], 0, 0, 0);      \
      }                                                                                                   \
    if (kt_ + 1 < nk) store(cur ^ 1, NEXT);                                                               \
    _Pragma("unroll") for (int bi = MBLK / 2; bi < MBLK; ++bi)                                            \
      _Pragma("unroll") for (int bj = 0; bj < NBLK; ++bj) {                                               \
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[bi], bh[bj], acc[bi][bj], 0, 0, 0);      \
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[bi], bl[bj], acc[bi][bj], 0, 0, 0);      \
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[bi], bh[bj], acc[bi][bj], 0, 0, 0);      \
      }                                                                                                   \
    __syncthreads();                                                                                      \
  }
  long long kt = 0;
  for (; kt + 1 < nk; kt += 2) {
    PSIM_BF16X3_STAGE(kt, set1, set0)
    PSIM_BF16X3_STAGE(kt + 1, set0, set1)
  }
  if (kt < nk) PSIM_BF16X3_STAGE(kt, set1, set0)
#undef PSIM_BF16X3_STAGE

#pragma unroll
  for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
    for (int bj = 0; bj < NBLK; ++bj)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const long long row = m0 + wr * WM + bi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const long long col = n0 + wc * WN + bj * 32 + (lane & 31);
        if (row < p.M && col < p.Nr) C[row * p.Nr + col] = acc[bi][bj][r];
      }
}

// Direct-to-LDS form of the BF16x3 kernel for interior launches (every tile
// interior, every 16-real stage inside one k1 block, a multiple of four
// stages).  A is copied global -> LDS in FP32 by the load unit and split into
// hi / lo as its fragments are read; W's two pre-split planes are copied side
// by side into one 64-byte LDS row per output column (hi k 0..15, then lo
// k 0..15).  Rows are unpadded, their four 16-byte chunks permuted by
// (row >> 2) & 3 so the fragment reads of 16 consecutive rows hit distinct
// banks.  Four LDS buffers form a ring: the copies of a stage are issued
// three stages before its products, so about 2 us of matrix work covers the
// latency of a copy that misses L2.  512 threads: 8 waves as 4 (m) x 2 (n)
// blocks of 64 x 128 outputs, 128 accumulator registers each, two waves per
// SIMD.  The split, the products and their order for each output element
// are those of site_gemm_bf16x3, so the two agree bit for bit.
// x = hi + lo for 8 floats (x0 then x1) with hi = bf16(x) and lo =
// bf16(x - hi), both rounded to nearest even, as the operand registers of a
// 32x32x16 MFMA hold them.  Each pair is rounded in one packed conversion and
// its hi values are widened back to FP32 by a shift and a mask of the packed
// word (bf16 is the upper half of an FP32), so x - hi is exact as in the
// scalar form.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split_bf16x8(const f32x4 x0, const f32x4 x1, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const f32x4& x = q < 2 ? x0 : x1;
    const int e = 2 * (q & 1);
    const bf16x2 h = __builtin_convertvector(f32x2{x[e], x[e + 1]}, bf16x2);
    const unsigned u = __builtin_bit_cast(unsigned, h);
    const float f0 = __builtin_bit_cast(float, u << 16), f1 = __builtin_bit_cast(float, u & 0xffff0000u);
    const bf16x2 l = __builtin_convertvector(f32x2{x[e] - f0, x[e + 1] - f1}, bf16x2);
    hi[2 * q] = h[0];
    hi[2 * q + 1] = h[1];
    lo[2 * q] = l[0];
    lo[2 * q + 1] = l[1];
  }
}

__device__ __forceinline__ int ring_swz(int r) { return (r >> 2) & 3; }

template <int BM, int BN>
__global__ __launch_bounds__(512) void site_gemm_bf16x3_dtl(KArgs p) {
  constexpr int BK = 16;                 // reals per stage: one MFMA k-step
  constexpr int NW = 8;                  // waves per workgroup
  constexpr int WM = BM / 4, WN = BN / 2;
  constexpr int MBLK = WM / 32, NBLK = WN / 32;
  constexpr int A_INS = BM * 64 / 1024 / NW;  // wave-wide 1 KiB copies per wave and stage
  constexpr int B_INS = BN * 64 / 1024 / NW;
  static_assert(A_INS >= 1 && B_INS >= 1 && A_INS * NW * 1024 == BM * 64 && B_INS * NW * 1024 == BN * 64, "tile");
  __shared__ __attribute__((aligned(1024))) float sA0[BM * BK];
  __shared__ __attribute__((aligned(1024))) float sA1[BM * BK];
  __shared__ __attribute__((aligned(1024))) float sA2[BM * BK];
  __shared__ __attribute__((aligned(1024))) float sA3[BM * BK];
  __shared__ __attribute__((aligned(1024))) __bf16 sB0[BN * 2 * BK];
  __shared__ __attribute__((aligned(1024))) __bf16 sB1[BN * 2 * BK];
  __shared__ __attribute__((aligned(1024))) __bf16 sB2[BN * 2 * BK];
  __shared__ __attribute__((aligned(1024))) __bf16 sB3[BN * 2 * BK];

  const long long t = xcd_tile(p.T);
  if (t >= p.T) return;
  const long long nt = t % p.NT;
  const long long rest = t / p.NT;
  const long long mt = rest % p.MT;
  const long long z = rest / p.MT;
  const long long node = z / p.Bz, vb = z % p.Bz;
  const long long ablk = p.a_index ? (long long)p.a_index[node] : node;
  const float* __restrict__ A = (const float*)p.A + 2 * (ablk * p.sA_node + vb * p.sA_v);
  const int tauv = p.tau ? (int)p.tau[node * p.tau_stride] : 0;
  const __bf16* __restrict__ Wh = (const __bf16*)(tauv ? p.W1 : p.W0) + p.w_koff_r;
  const __bf16* __restrict__ Wl = Wh + p.plane;
  float* __restrict__ C = (float*)p.C + 2 * (node * p.sC_node + vb * p.sC_v);
  const long long m0 = mt * BM, n0 = nt * BN;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const long long sK1 = p.M * p.K2;

  // Copy `it` of this wave fills tile rows (it * NW + wid) * 16 + lane / 4,
  // physical chunk lane % 4, from logical chunk (lane % 4) ^ swz(row); for W
  // logical chunks 0-1 are the hi plane's k 0..15 and 2-3 the lo plane's.
  // Byte offsets from the uniform stage bases stay below 2^31.
  const unsigned a_rs = (unsigned)(2 * p.K2 * 4);  // bytes between rows of A
  const unsigned b_rs = (unsigned)(p.ldw * 2);     // bytes between rows of a W plane
  long long fk1 = 0, fk2 = 0, kr = 0;              // next stage: (k1, k2) of A, real k of W
  auto issue = [&](float* sa, __bf16* sb) {
    const char* abase = (const char*)(A + 2 * (fk1 * sK1 + m0 * p.K2 + fk2));
    const char* hbase = (const char*)(Wh + n0 * p.ldw + kr);
    const char* lbase = (const char*)(Wl + n0 * p.ldw + kr);
#pragma unroll
    for (int it = 0; it < A_INS; ++it) {
      const int row = (it * NW + wid) * 16 + (lane >> 2);
      const int chk = (lane & 3) ^ ring_swz(row);
      __builtin_amdgcn_global_load_lds((const void*)(abase + (unsigned)row * a_rs + (unsigned)chk * 16u),
                                       PSIM_LDS(sa + (it * NW + wid) * 256), 16, 0, 0);
    }
#pragma unroll
    for (int it = 0; it < B_INS; ++it) {
      const int row = (it * NW + wid) * 16 + (lane >> 2);
      const int chk = (lane & 3) ^ ring_swz(row);
      const char* src = ((chk & 2) ? lbase : hbase) + (unsigned)row * b_rs + (unsigned)(chk & 1) * 16u;
      __builtin_amdgcn_global_load_lds((const void*)src, PSIM_LDS(sb + (it * NW + wid) * 512), 16, 0, 0);
    }
    fk2 += BK / 2;
    if (fk2 == p.K2) {
      fk2 = 0;
      ++fk1;
    }
    kr += BK;
  };

  f32x16 acc[MBLK][NBLK];
#pragma unroll
  for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
    for (int bj = 0; bj < NBLK; ++bj)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[bi][bj][r] = 0;

  const int frow = lane & 31, h = lane >> 5;  // lane half h supplies k 8h .. 8h+7 of the k-step
  auto compute = [&](const float* a_s, const __bf16* b_s) {
    bf16x8 ah[MBLK], al[MBLK], bh[NBLK], bl[NBLK];
#pragma unroll
    for (int bi = 0; bi < MBLK; ++bi) {
      const int r = wr * WM + bi * 32 + frow;
      const int sw = ring_swz(r);
      const f32x4 x0 = *(const f32x4*)(a_s + r * BK + (((2 * h) ^ sw) << 2));
      const f32x4 x1 = *(const f32x4*)(a_s + r * BK + (((2 * h + 1) ^ sw) << 2));
      split_bf16x8(x0, x1, ah[bi], al[bi]);
    }
#pragma unroll
    for (int bj = 0; bj < NBLK; ++bj) {
      const int r = wc * WN + bj * 32 + frow;
      const int sw = ring_swz(r);
      bh[bj] = *(const bf16x8*)(b_s + r * 2 * BK + ((h ^ sw) << 3));
      bl[bj] = *(const bf16x8*)(b_s + r * 2 * BK + (((2 + h) ^ sw) << 3));
    }
#pragma unroll
    for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
      for (int bj = 0; bj < NBLK; ++bj) {
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[bi], bh[bj], acc[bi][bj], 0, 0, 0);
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[bi], bl[bj], acc[bi][bj], 0, 0, 0);
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[bi], bh[bj], acc[bi][bj], 0, 0, 0);
      }
  };
  // vmcnt(n), other counters unconstrained: all but this wave's n most recent
  // copies into LDS have landed (A_INS + B_INS copies per stage)
  constexpr int PER = A_INS + B_INS;
  static_assert(2 * PER <= 15, "vmcnt field");
  constexpr unsigned kWaitVm0 = 0x3f70, kWaitVm1 = 0x3f70 | PER, kWaitVm2 = 0x3f70 | (2 * PER);

  // one stage: wait for its copies (the copies of up to two later stages
  // may still be in flight), barrier (every wave's copies have landed and
  // every wave is done with the buffer the next issue overwrites), issue the
  // copies of stage s + 3 into that buffer, then the stage's products
  const int nst = (int)(p.Kr / BK);  // the launcher guarantees a multiple of 4
#define PSIM_BF16X3_RING(S, SA, SB, NA, NB)                     \
  {                                                             \
    const int s_ = (S);                                         \
    if (s_ + 2 < nst)                                           \
      __builtin_amdgcn_s_waitcnt(kWaitVm2);                     \
    else if (s_ + 1 < nst)                                      \
      __builtin_amdgcn_s_waitcnt(kWaitVm1);                     \
    else                                                        \
      __builtin_amdgcn_s_waitcnt(kWaitVm0);                     \
    __syncthreads();                                            \
    if (s_ + 3 < nst) issue(NA, NB);                            \
    compute(SA, SB);                                            \
  }
  issue(sA0, sB0);
  issue(sA1, sB1);
  issue(sA2, sB2);
  for (int s0 = 0; s0 < nst; s0 += 4) {
    PSIM_BF16X3_RING(s0, sA0, sB0, sA3, sB3)
    PSIM_BF16X3_RING(s0 + 1, sA1, sB1, sA0, sB0)
    PSIM_BF16X3_RING(s0 + 2, sA2, sB2, sA1, sB1)
    PSIM_BF16X3_RING(s0 + 3, sA3, sB3, sA2, sB2)
  }
#undef PSIM_BF16X3_RING

#pragma unroll
  for (int bi = 0; bi < MBLK; ++bi)
#pragma unroll
    for (int bj = 0; bj < NBLK; ++bj)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const long long row = m0 + wr * WM + bi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const long long col = n0 + wc * WN + bj * 32 + (lane & 31);
        if (col < p.Nr) C[row * p.Nr + col] = acc[bi][bj][r];
      }
}

// ---------------------------------------------------------------- rescale
// Per node: largest binary exponent of any component (as exponent + 4096,
// so that unsigned atomicMax orders it), 0 when the node is all zeros.
template <typename T>
__global__ void row_absmax(const T* __restrict__ F, long long per_node, uint32_t* mx) {
  const long long node = blockIdx.y;
  const T* f = F + 2 * node * per_node;
  T m = 0;
  for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < 2 * per_node;
       x += (long long)gridDim.x * blockDim.x)
    m = fmax(m, fabs(f[x]));
  // wave reduction
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  __shared__ T red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
    if (m > 0) {
      int e;
      frexp(m, &e);  // m = f 2^e, f in [0.5, 1)
      atomicMax(mx + node, (uint32_t)(e + 4096));
    }
  }
}

__global__ void row_exponent(long long nodes, const int32_t* parent, const int32_t* exp_prev, int32_t* exp_cur,
                             uint32_t* mx) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  const int e = mx[n] ? (int)mx[n] - 4096 : 0;
  exp_cur[n] = exp_prev[parent[n]] + e;
  mx[n] = (uint32_t)(e + 4096);  // keep the shift for row_apply
}

template <typename T>
__global__ void row_apply(T* __restrict__ F, long long per_node, const uint32_t* mx) {
  const long long node = blockIdx.y;
  const int e = (int)mx[node] - 4096;
  if (e == 0) return;
  T* f = F + 2 * node * per_node;
  for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < 2 * per_node;
       x += (long long)gridDim.x * blockDim.x)
    f[x] = ldexp(f[x], -e);
}

// Fused rescale for small boundaries, several problems per launch: one
// workgroup per node finds the node's largest component, its exponent e,
// the node's running exponent (parent's plus e) and scales the node by 2^-e.
// Same results as row_absmax + row_exponent + row_apply.
constexpr int kMaxScale = 32;
struct ScaleProb {
  void* F;
  long long per_node;  // complex elements per node
  const int32_t* parent;
  const int32_t* exp_prev;
  int32_t* exp_cur;
};
struct ScaleArgs {
  ScaleProb p[kMaxScale];
  long long start[kMaxScale + 1];  // first global node of each problem; start[n] = total
  int n;
};

template <typename T>
__global__ __launch_bounds__(256) void row_rescale_fused(ScaleArgs a) {
  const long long g = blockIdx.x;
  int lo = 0, hi = a.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.start[mid] <= g) lo = mid; else hi = mid - 1;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  const long long node = g - a.start[lo];
  const long long len = 2 * a.p[lo].per_node;
  T* f = (T*)a.p[lo].F + node * len;
  T m = 0;
  for (long long x = threadIdx.x; x < len; x += blockDim.x) m = fmax(m, fabs(f[x]));
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  __shared__ T red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  int e = 0;
  if (m > 0) frexp(m, &e);
  if (threadIdx.x == 0) a.p[lo].exp_cur[node] = a.p[lo].exp_prev[a.p[lo].parent[node]] + e;
  if (e == 0) return;
  for (long long x = threadIdx.x; x < len; x += blockDim.x) f[x] = ldexp(f[x], -e);
}

__global__ void copy_segments(const CopySeg* __restrict__ segs) {
  const CopySeg sg = segs[blockIdx.y];
  const unsigned char* a = (const unsigned char*)sg.src;
  unsigned char* b = (unsigned char*)sg.dst;
  for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < sg.bytes;
       x += (long long)gridDim.x * blockDim.x)
    b[x] = a[x];
}

// ---------------------------------------------------------------- square partition helpers
// Three-index permutes of a complex tensor in[X][Y][Z] (E = float2 or
// double2, one complex element): mode 0 writes out[Y][X][Z], mode 1
// out[X][Z][Y].  One thread per output element; blockIdx.y = node, nodes
// X*Y*Z elements apart in both tensors.  With mx (per node: exponent + 4096,
// as row_exponent leaves it) every element is scaled by 2^-exponent on the
// way, exactly as row_apply would have done in place.
template <typename E>
__global__ void permute3(const E* __restrict__ in, E* __restrict__ out, long long X, long long Y, long long Z,
                         int mode, const uint32_t* __restrict__ mx) {
  const long long total = X * Y * Z;
  in += blockIdx.y * total;
  out += blockIdx.y * total;
  const int e = mx ? (int)mx[blockIdx.y] - 4096 : 0;
  for (long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x; o < total;
       o += (long long)gridDim.x * blockDim.x) {
    long long x, y, z;
    if (mode == 0) {  // o = (y X + x) Z + z
      z = o % Z;
      const long long q = o / Z;
      x = q % X;
      y = q / X;
    } else {          // o = (x Z + z) Y + y
      y = o % Y;
      const long long q = o / Y;
      z = q % Z;
      x = q / Z;
    }
    E v = in[(x * Y + y) * Z + z];
    if (e != 0) {
      v.x = ldexp(v.x, -e);
      v.y = ldexp(v.y, -e);
    }
    out[o] = v;
  }
}

// A device complex matrix Q[n][k] (row-major, N x K) as the packed W operand
// of the site kernels for W[k][n] = Q[n][k], zero padded to rows x ld:
// 3M: P[n][2k + c] = component c of Q[n][k]; 4M (float or double): the real
// expansion P[2n + a][2k + b] = [[Re, -Im], [Im, Re]][a][b] of Q[n][k].
// blockIdx.y = node: N*K complex elements apart in Q, rows*ld reals in P.
template <typename T>
__global__ void pack_w(const T* __restrict__ Q, T* __restrict__ P, long long N, long long K, long long rows,
                       long long ld, int three_m) {
  const long long total = rows * ld;
  Q += blockIdx.y * 2 * N * K;
  P += blockIdx.y * total;
  for (long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x; o < total;
       o += (long long)gridDim.x * blockDim.x) {
    const long long row = o / ld, c = o - row * ld;
    T v = 0;
    if (three_m) {
      if (row < N && c < 2 * K) v = Q[2 * (row * K + (c >> 1)) + (c & 1)];
    } else if (row < 2 * N && c < 2 * K) {
      const long long n = row >> 1, k = c >> 1;
      const int a = (int)(row & 1), b = (int)(c & 1);
      const T re = Q[2 * (n * K + k)], im = Q[2 * (n * K + k) + 1];
      v = (a == b) ? re : (a ? im : -im);
    }
    P[o] = v;
  }
}

// Partial sums of sum_i a[i] b[i] (complex, no conjugation) in FP64: one
// (re, im) pair per workgroup in part[2 * blockIdx.x].
template <typename T>
__global__ __launch_bounds__(256) void cdot_partial(const T* __restrict__ a, const T* __restrict__ b, long long n,
                                                    double* __restrict__ part) {
  double re = 0, im = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double ar = a[2 * i], ai = a[2 * i + 1], br = b[2 * i], bi = b[2 * i + 1];
    re += ar * br - ai * bi;
    im += ar * bi + ai * br;
  }
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off);
    im += __shfl_xor(im, off);
  }
  __shared__ double red[2][4];
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = re;
    red[1][threadIdx.x >> 6] = im;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    part[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

// Sum of the nblk (re, im) partials of cdot_partial into out[0..1], in a
// fixed order (one workgroup: strided per-thread sums, then a tree).
__global__ __launch_bounds__(256) void cdot_finish(const double* __restrict__ part, int nblk,
                                                   double* __restrict__ out) {
  __shared__ double red[2][256];
  double re = 0, im = 0;
  for (int t = threadIdx.x; t < nblk; t += 256) {
    re += part[2 * t];
    im += part[2 * t + 1];
  }
  red[0][threadIdx.x] = re;
  red[1][threadIdx.x] = im;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      red[0][threadIdx.x] += red[0][threadIdx.x + h];
      red[1][threadIdx.x] += red[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0][0];
    out[1] = red[1][0];
  }
}

__global__ void zero_u32(uint32_t* p, long long n) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < n) p[x] = 0;
}

template <typename T>
__global__ void fill_one(T* p) {
  p[0] = 1;
  p[1] = 0;
}

// ---------------------------------------------------------------- host side
void hip_check(int err, const char* what) {
  if (err != hipSuccess)
    fail(PSIM_EDEVICE, std::string(what) + ": " + hipGetErrorString((hipError_t)err));
}

// Tile candidates (BM x BN real outputs per workgroup, BK reals per stage) of
// the FP32 row-major interior-site kernel; index 0 is the default.
struct FCfg {
  int bm, bn, bk;
};
// 6 = the direct-to-LDS 4M kernel with 128 x 64 tiles (0 is its 128 x 128 form)
static const FCfg kFp32Configs[] = {{128, 128, 32}, {256, 128, 16}, {128, 256, 16},
                                    {256, 256, 16}, {128, 128, 64}, {256, 128, 32}, {128, 64, 32}};
int fp32_config_count() { return (int)(sizeof(kFp32Configs) / sizeof(kFp32Configs[0])); }
// 3M candidates: 0 = 128 x 128 x 32 (two waves per SIMD), 1 = 256 x 128 x 32,
// 2 = 128 x 256 x 32 (one wave per SIMD, twice the work per LDS stage)
// 3 = the direct-to-LDS kernel with 64 x 128 tiles (more workgroups per CU)
static const FCfg kFp32_3mConfigs[] = {{128, 128, 32}, {256, 128, 32}, {128, 256, 32}, {64, 128, 32}};
int fp32_3m_config_count() { return (int)(sizeof(kFp32_3mConfigs) / sizeof(kFp32_3mConfigs[0])); }
// FP64 candidates: 0 = direct-to-LDS 128 x 64, 1 = direct-to-LDS 64 x 64,
// 2 = row-major 128 x 64 x 16 (LDS through registers)
int fp64_config_count() { return 3; }
// BF16x3 candidates: 0 = 256 x 256 tiles, 1 = 128 x 256, 2 = the direct-to-LDS
// kernel with 256 x 256 tiles and two waves per SIMD
int bf16x3_config_count() { return 3; }
int config_count(int prec) {
  switch (prec) {
    case PSIM_FP32_4M: return fp32_config_count();
    case PSIM_FP32_3M: return fp32_3m_config_count();
    case PSIM_FP64: return fp64_config_count();
    case PSIM_BF16X3: return bf16x3_config_count();
    default: return 1;
  }
}

template <typename T, int BM, int BN, int BK, int AMODE, bool TRANS, int SCH = 4, bool SPLIT = false>
static void launch(const KArgs& a, long long blocks, hipStream_t st) {
  if constexpr (SPLIT)
    hipLaunchKernelGGL((site_gemm_split<T, BM, BN, BK, AMODE, TRANS, SCH>), dim3((unsigned)blocks), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((site_gemm<T, BM, BN, BK, AMODE, TRANS, SCH>), dim3((unsigned)blocks), dim3(256), 0, st, a);
}

static KArgs make_kargs(const GemmLaunch& g) {
  if (g.M < 1 || g.K1 < 1 || g.K2 < 1 || g.N < 1 || g.nodes < 1 || g.Bz < 1)
    fail(PSIM_EINVAL, "site gemm: non-positive size");
  if (g.M >= (1LL << 31) || g.K1 * g.K2 >= (1LL << 30))
    fail(PSIM_EUNSUPPORTED, "site gemm: M or K too large for one batch entry");
  KArgs a{};
  a.A = g.A;
  a.C = g.C;
  a.W0 = g.W0;
  a.W1 = g.W1 ? g.W1 : g.W0;
  a.a_index = g.a_index;
  a.tau = g.tau;
  a.tau_stride = g.tau_stride;
  a.M = g.M;
  a.K1 = g.K1;
  a.K2 = g.K2;
  a.N = g.N;
  a.K = g.K1 * g.K2;
  a.Kr = 2 * a.K;
  a.Nr = 2 * g.N;
  a.ldw = g.ldw;
  a.w_koff_r = 2 * g.w_koff;
  a.sA_node = g.sA_node;
  a.sA_v = g.sA_v;
  a.sC_node = g.sC_node;
  a.sC_v = g.sC_v;
  a.Bz = g.Bz;
  a.trans_out = g.trans_out;
  a.beta = g.beta;
  a.ldct = g.ldct ? g.ldct : g.M;
  a.nb = g.nb;
  a.sCw = g.sCw;
  if (g.nb && (g.trans_out || g.nb < 1)) fail(PSIM_EINVAL, "site gemm: split-N stores need a plain store");
  return a;
}

// 16-byte vector loads need every batch entry's A to start 16-byte aligned
static int fp32_mode(const GemmLaunch& g) {
  const bool even_base = ((uintptr_t)g.A % 16 == 0) && (g.sA_node % 2 == 0) && (g.sA_v % 2 == 0);
  return (g.K2 % 2 == 0 && even_base) ? ROWMAJOR
         : (g.K2 == 1 && g.M % 2 == 0 && g.K1 > 1 && even_base) ? KMAJOR : GENERIC;
}

// The direct-to-LDS 3M kernel applies: interior tiles only, every K stage
// inside one k1 block, an even number of stages, 32-bit copy offsets.
static bool dtl3m_ok(const GemmLaunch& g, int mode, int bm = 128) {
  return g.prec == PSIM_FP32_3M && !g.trans_out && !g.nb && mode == ROWMAJOR && g.M % bm == 0 &&
         (2 * g.K2) % 32 == 0 && (2 * g.K1 * g.K2) % 64 == 0 && g.K2 < (1 << 20) && g.ldw < (1 << 22);
}

// Grouped-launch variants (FP32 only), the kernels launch_site_gemm picks for
// default tiles: id = 8 * (3M ? 1 : 0) + 2 * mode + trans with 128 x 128 x 32
// tiles (mode: ROWMAJOR, KMAJOR, GENERIC, ROWFAST); 16 / 17 = 4M transposed
// small-N tiles (256 x 64 x 16, ROWMAJOR / KMAJOR); 18 = 3M direct-to-LDS.
// -1: not groupable.
int group_variant(const GemmLaunch& g, void* out, long long* tiles) {
  if ((g.prec != PSIM_FP32_4M && g.prec != PSIM_FP32_3M) || g.split || g.cfg > 0) return -1;
  int mode = fp32_mode(g);
  KArgs a = make_kargs(g);
  const long long Z = g.nodes * g.Bz;
  int id, bm, bn;
  if (g.prec == PSIM_FP32_4M && g.trans_out && g.N <= 32 && mode != GENERIC) {
    id = mode == ROWMAJOR ? 16 : 17;
    bm = 256;
    bn = 64;
  } else if (dtl3m_ok(g, mode)) {
    id = 18;
    bm = 128;
    bn = 128;
  } else {
    if (mode == ROWMAJOR && g.M % 128 == 0 && (2 * g.K1 * g.K2) % 32 == 0 && (2 * g.K2) % 32 == 0) mode = ROWFAST;
    id = 8 * (g.prec == PSIM_FP32_3M ? 1 : 0) + 2 * mode + (g.trans_out ? 1 : 0);
    bm = 128;
    bn = 128;
  }
  a.MT = (a.M + bm - 1) / bm;
  a.NT = (a.Nr + bn - 1) / bn;
  a.T = a.MT * a.NT * Z;
  std::memcpy(out, &a, sizeof(KArgs));
  *tiles = a.T;
  return id;
}

template <int SCH, int AMODE, bool TRANS>
static void glaunch(const GroupArgs& ga, long long blocks, hipStream_t st) {
  hipLaunchKernelGGL((site_gemm_group<float, 128, 128, 32, AMODE, TRANS, SCH>), dim3((unsigned)blocks), dim3(256), 0,
                     st, ga);
}

template <int SCH>
static void glaunch_mode(int mode, bool trans, const GroupArgs& ga, long long blocks, hipStream_t st) {
  switch (mode) {
    case ROWMAJOR: trans ? glaunch<SCH, ROWMAJOR, true>(ga, blocks, st) : glaunch<SCH, ROWMAJOR, false>(ga, blocks, st); break;
    case KMAJOR: trans ? glaunch<SCH, KMAJOR, true>(ga, blocks, st) : glaunch<SCH, KMAJOR, false>(ga, blocks, st); break;
    case GENERIC: trans ? glaunch<SCH, GENERIC, true>(ga, blocks, st) : glaunch<SCH, GENERIC, false>(ga, blocks, st); break;
    default: trans ? glaunch<SCH, ROWFAST, true>(ga, blocks, st) : glaunch<SCH, ROWFAST, false>(ga, blocks, st); break;
  }
}

void launch_group(int variant, const void* const* d_probs, const long long* start, int nprob, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (nprob < 1 || nprob > kMaxGroup) fail(PSIM_EINTERNAL, "group size out of range");
  if (variant < 0 || variant > 18) fail(PSIM_EINTERNAL, "unknown group variant");
  GroupArgs ga{};
  for (int i = 0; i < nprob; ++i) {
    ga.probs[i] = (const KArgs*)d_probs[i];
    ga.start[i] = start[i];
  }
  ga.start[nprob] = start[nprob];
  ga.nprob = nprob;
  const long long total = start[nprob];
  if (total < 1) return;
  const long long blocks = (total + 7) / 8 * 8;
  if (blocks > 0x7fffffffLL) fail(PSIM_EUNSUPPORTED, "grid too large");
  if (variant == 18)
    hipLaunchKernelGGL((site_gemm_3m_dtl_group<128, 128>), dim3((unsigned)blocks), dim3(256), 0, st, ga);
  else if (variant == 16)
    hipLaunchKernelGGL((site_gemm_group<float, 256, 64, 16, ROWMAJOR, true, 4>), dim3((unsigned)blocks), dim3(256), 0,
                       st, ga);
  else if (variant == 17)
    hipLaunchKernelGGL((site_gemm_group<float, 256, 64, 16, KMAJOR, true, 4>), dim3((unsigned)blocks), dim3(256), 0,
                       st, ga);
  else if (variant < 8)
    glaunch_mode<4>((variant >> 1) & 3, variant & 1, ga, blocks, st);
  else
    glaunch_mode<3>((variant >> 1) & 3, variant & 1, ga, blocks, st);
  hip_check(hipGetLastError(), "grouped site_gemm launch");
}

int kargs_bytes() { return (int)sizeof(KArgs); }
int max_group() { return kMaxGroup; }

// FP32 launch arguments with 128 x 128 tiles over Z batch entries
static KArgs default_tiles(const KArgs& a, long long Z) {
  KArgs d = a;
  d.MT = (d.M + 128 - 1) / 128;
  d.NT = (d.Nr + 128 - 1) / 128;
  d.T = d.MT * d.NT * Z;
  return d;
}
static long long default_blocks(const KArgs& a, long long Z) { return (default_tiles(a, Z).T + 7) / 8 * 8; }

void launch_site_gemm(const GemmLaunch& g, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  KArgs a = make_kargs(g);
  // batch entries = nodes * Bz; the kernel splits z = node * Bz + v
  const long long Z = g.nodes * g.Bz;
  if (g.prec == PSIM_FP64) {
    KArgs b = a;
    b.MT = (b.M + 64 - 1) / 64;
    b.NT = (b.Nr + 64 - 1) / 64;
    b.T = b.MT * b.NT * Z;
    const long long blocks = (b.T + 7) / 8 * 8;
    if (blocks > 0x7fffffffLL) fail(PSIM_EUNSUPPORTED, "grid too large");
    const bool kmajor = g.K2 == 1 && g.K1 > 1;
    // interior-only row-major launches (every stage inside one k1 block):
    // 128 x 64 tiles with the division-free loader
    const bool fastd = !g.trans_out && !g.nb && g.K2 % 8 == 0 && g.M % 128 == 0;
    const bool dtl_ok = fastd && (g.K1 * g.K2) % 16 == 0 && g.K2 < (1 << 20) && g.ldw < (1 << 22);
    if (dtl_ok && g.cfg == 1) {
      // candidate 1: 64 x 64 tiles
      KArgs f = a;
      f.MT = f.M / 64;
      f.NT = (f.Nr + 64 - 1) / 64;
      f.T = f.MT * f.NT * Z;
      const long long fb = (f.T + 7) / 8 * 8;
      if (fb > 0x7fffffffLL) fail(PSIM_EUNSUPPORTED, "grid too large");
      hipLaunchKernelGGL((site_gemm_4m_dtl<double, 64, 64, 4>), dim3((unsigned)fb), dim3(256), 0, st, f);
    } else if (dtl_ok && g.cfg != 2) {
      // an even number of 16-double stages, 32-bit copy offsets: direct-to-LDS
      KArgs f = a;
      f.MT = f.M / 128;
      f.NT = (f.Nr + 64 - 1) / 64;
      f.T = f.MT * f.NT * Z;
      const long long fb = (f.T + 7) / 8 * 8;
      if (fb > 0x7fffffffLL) fail(PSIM_EUNSUPPORTED, "grid too large");
      hipLaunchKernelGGL((site_gemm_4m_dtl<double, 128, 64, 3>), dim3((unsigned)fb), dim3(256), 0, st, f);
    } else if (fastd) {
      KArgs f = a;
      f.MT = f.M / 128;
      f.NT = (f.Nr + 64 - 1) / 64;
      f.T = f.MT * f.NT * Z;
      const long long fb = (f.T + 7) / 8 * 8;
      if (fb > 0x7fffffffLL) fail(PSIM_EUNSUPPORTED, "grid too large");
      launch<double, 128, 64, 16, ROWFAST, false>(f, fb, st);
    } else if (kmajor && g.trans_out)
      launch<double, 64, 64, 16, KMAJOR, true>(b, blocks, st);
    else if (kmajor)
      launch<double, 64, 64, 16, KMAJOR, false>(b, blocks, st);
    else if (g.trans_out)
      launch<double, 64, 64, 16, GENERIC, true>(b, blocks, st);
    else
      launch<double, 64, 64, 16, GENERIC, false>(b, blocks, st);
  } else {
    KArgs b = a;
    b.MT = (b.M + 128 - 1) / 128;
    b.NT = (b.Nr + 128 - 1) / 128;
    b.T = b.MT * b.NT * Z;
    const long long blocks = (b.T + 7) / 8 * 8;
    if (blocks > 0x7fffffffLL) fail(PSIM_EUNSUPPORTED, "grid too large");
    const int mode = fp32_mode(g);
    // interior-only tiles of bm rows and bk reals per stage
    auto fast = [&](int bm, int bk) {
      return mode == ROWMAJOR && g.M % bm == 0 && (2 * g.K1 * g.K2) % bk == 0 && (2 * g.K2) % bk == 0;
    };
    if (g.split && g.prec == PSIM_FP32_4M) {
      if (g.trans_out && g.N <= 32 && fast(128, 32)) {
        // last sites of a row (N <= 32 complex): tiles 64 reals wide, so
        // none of a 128-wide tile's columns are padding; the same products
        // in the same k order as the 128 x 128 tiles
        KArgs f = b;
        f.NT = (f.Nr + 63) / 64;
        f.T = f.MT * f.NT * Z;
        const long long fb = (f.T + 7) / 8 * 8;
        if (fb > 0x7fffffffLL) fail(PSIM_EUNSUPPORTED, "grid too large");
        launch<float, 128, 64, 32, ROWFAST, true, 4, true>(f, fb, st);
      } else if (fast(128, 32))
        g.trans_out ? launch<float, 128, 128, 32, ROWFAST, true, 4, true>(b, blocks, st)
                    : launch<float, 128, 128, 32, ROWFAST, false, 4, true>(b, blocks, st);
      else if (mode == ROWMAJOR)
        g.trans_out ? launch<float, 128, 128, 32, ROWMAJOR, true, 4, true>(b, blocks, st)
                    : launch<float, 128, 128, 32, ROWMAJOR, false, 4, true>(b, blocks, st);
      else if (mode == KMAJOR)
        g.trans_out ? launch<float, 128, 128, 32, KMAJOR, true, 4, true>(b, blocks, st)
                    : launch<float, 128, 128, 32, KMAJOR, false, 4, true>(b, blocks, st);
      else
        g.trans_out ? launch<float, 128, 128, 32, GENERIC, true, 4, true>(b, blocks, st)
                    : launch<float, 128, 128, 32, GENERIC, false, 4, true>(b, blocks, st);
    } else if (g.split && g.prec == PSIM_FP32_3M && !dtl3m_ok(g, mode)) {
      // 3M launches outside the direct-to-LDS kernel, per-stage partial sums
      if (fast(128, 32))
        g.trans_out ? launch<float, 128, 128, 32, ROWFAST, true, 3, true>(b, blocks, st)
                    : launch<float, 128, 128, 32, ROWFAST, false, 3, true>(b, blocks, st);
      else if (mode == ROWMAJOR)
        g.trans_out ? launch<float, 128, 128, 32, ROWMAJOR, true, 3, true>(b, blocks, st)
                    : launch<float, 128, 128, 32, ROWMAJOR, false, 3, true>(b, blocks, st);
      else if (mode == KMAJOR && !g.trans_out) {
        // first sites of a row: 64-row tiles, half the accumulators of a
        // wave, so more workgroups share a CU (same products, same order)
        KArgs f = b;
        f.MT = (f.M + 63) / 64;
        f.T = f.MT * f.NT * Z;
        const long long fb = (f.T + 7) / 8 * 8;
        if (fb > 0x7fffffffLL) fail(PSIM_EUNSUPPORTED, "grid too large");
        launch<float, 64, 128, 32, KMAJOR, false, 3, true>(f, fb, st);
      } else if (mode == KMAJOR)
        launch<float, 128, 128, 32, KMAJOR, true, 3, true>(b, blocks, st);
      else
        g.trans_out ? launch<float, 128, 128, 32, GENERIC, true, 3, true>(b, blocks, st)
                    : launch<float, 128, 128, 32, GENERIC, false, 3, true>(b, blocks, st);
    } else if (g.prec == PSIM_BF16X3 && mode == ROWMAJOR && !g.trans_out && !g.nb && g.Wb0) {
      // split-precision kernel on the pre-split planes
      b.W0 = g.Wb0;
      b.W1 = g.Wb1 ? g.Wb1 : g.Wb0;
      b.ldw = g.ldwb;
      b.plane = g.planeb;
      const bool big = g.cfg != 1;
      const int bm = big ? 256 : 128, bn = 256;
      b.MT = (b.M + bm - 1) / bm;
      b.NT = (b.Nr + bn - 1) / bn;
      b.T = b.MT * b.NT * Z;
      const long long bl = (b.T + 7) / 8 * 8;
      if (bl > 0x7fffffffLL) fail(PSIM_EUNSUPPORTED, "grid too large");
      const bool f = g.M % bm == 0 && (2 * g.K1 * g.K2) % 16 == 0 && (2 * g.K2) % 16 == 0;
      // candidate 2: the direct-to-LDS form (16-real stages inside one k1
      // block, a multiple of four of them, 32-bit copy offsets); other
      // shapes take candidate 0's kernel, which gives the same results
      const bool dtl = g.cfg == 2 && g.M % 256 == 0 && (2 * g.K2) % 16 == 0 && (2 * g.K1 * g.K2) % 64 == 0 &&
                       g.K2 < (1 << 20) && g.ldwb < (1 << 22);
      if (dtl)
        hipLaunchKernelGGL((site_gemm_bf16x3_dtl<256, 256>), dim3((unsigned)bl), dim3(512), 0, st, b);
      else if (big && f)
        hipLaunchKernelGGL((site_gemm_bf16x3<256, 256, true>), dim3((unsigned)bl), dim3(256), 0, st, b);
      else if (big)
        hipLaunchKernelGGL((site_gemm_bf16x3<256, 256, false>), dim3((unsigned)bl), dim3(256), 0, st, b);
      else if (f)
        hipLaunchKernelGGL((site_gemm_bf16x3<128, 256, true>), dim3((unsigned)bl), dim3(256), 0, st, b);
      else
        hipLaunchKernelGGL((site_gemm_bf16x3<128, 256, false>), dim3((unsigned)bl), dim3(256), 0, st, b);
    } else if (g.prec == PSIM_FP32_3M && !g.trans_out && g.cfg > 0 && !g.split && mode == ROWMAJOR) {
      const FCfg& c = kFp32_3mConfigs[g.cfg];
      b.MT = (b.M + c.bm - 1) / c.bm;
      b.NT = (b.Nr + c.bn - 1) / c.bn;
      b.T = b.MT * b.NT * Z;
      const long long bl = (b.T + 7) / 8 * 8;
      if (bl > 0x7fffffffLL) fail(PSIM_EUNSUPPORTED, "grid too large");
      const bool f = fast(c.bm, c.bk);
      switch (g.cfg) {
        case 1: f ? launch<float, 256, 128, 32, ROWFAST, false, 3>(b, bl, st)
                  : launch<float, 256, 128, 32, ROWMAJOR, false, 3>(b, bl, st); break;
        case 2: f ? launch<float, 128, 256, 32, ROWFAST, false, 3>(b, bl, st)
                  : launch<float, 128, 256, 32, ROWMAJOR, false, 3>(b, bl, st); break;
        case 3:
          if (dtl3m_ok(g, mode, 64))
            hipLaunchKernelGGL((site_gemm_3m_dtl<64, 128>), dim3((unsigned)bl), dim3(256), 0, st, b);
          else  // shapes the direct-to-LDS kernel does not take: 128 x 128 tiles
            launch<float, 128, 128, 32, ROWMAJOR, false, 3>(default_tiles(a, Z), default_blocks(a, Z), st);
          break;
        default: fail(PSIM_EINVAL, "unknown kernel config");
      }
    } else if (dtl3m_ok(g, mode)) {
      // interior tiles, an even number of K stages, 32-bit copy offsets:
      // the direct-to-LDS kernel (same products in the same order as the
      // ROWFAST 3M kernel, so the same results bit for bit)
      if (g.split && g.cfg == 3) {
        // split accumulation with 64 x 128 tiles: half the accumulators per
        // wave, three workgroups per CU instead of two
        KArgs f = b;
        f.MT = f.M / 64;
        f.T = f.MT * f.NT * Z;
        const long long fb = (f.T + 7) / 8 * 8;
        if (fb > 0x7fffffffLL) fail(PSIM_EUNSUPPORTED, "grid too large");
        hipLaunchKernelGGL((site_gemm_3m_dtl_split<64, 128, 3>), dim3((unsigned)fb), dim3(256), 0, st, f);
      } else if (g.split)
        hipLaunchKernelGGL((site_gemm_3m_dtl_split<128, 128>), dim3((unsigned)blocks), dim3(256), 0, st, b);
      else
        hipLaunchKernelGGL((site_gemm_3m_dtl<128, 128>), dim3((unsigned)blocks), dim3(256), 0, st, b);
  } else if (g.prec == PSIM_FP32_3M) {
      if (fast(128, 32))
        g.trans_out ? launch<float, 128, 128, 32, ROWFAST, true, 3>(b, blocks, st)
                    : launch<float, 128, 128, 32, ROWFAST, false, 3>(b, blocks, st);
      else if (mode == ROWMAJOR)
        g.trans_out ? launch<float, 128, 128, 32, ROWMAJOR, true, 3>(b, blocks, st)
                    : launch<float, 128, 128, 32, ROWMAJOR, false, 3>(b, blocks, st);
      else if (mode == KMAJOR)
        g.trans_out ? launch<float, 128, 128, 32, KMAJOR, true, 3>(b, blocks, st)
                    : launch<float, 128, 128, 32, KMAJOR, false, 3>(b, blocks, st);
      else
        g.trans_out ? launch<float, 128, 128, 32, GENERIC, true, 3>(b, blocks, st)
                    : launch<float, 128, 128, 32, GENERIC, false, 3>(b, blocks, st);
    } else if (mode == ROWMAJOR && !g.trans_out && g.cfg > 0) {
      // tile candidates of the hot (interior-site) kernel; see kFp32Configs
      const FCfg& c = kFp32Configs[g.cfg];
      b.MT = (b.M + c.bm - 1) / c.bm;
      b.NT = (b.Nr + c.bn - 1) / c.bn;
      b.T = b.MT * b.NT * Z;
      const long long bl = (b.T + 7) / 8 * 8;
      if (bl > 0x7fffffffLL) fail(PSIM_EUNSUPPORTED, "grid too large");
      const bool f = fast(c.bm, c.bk);
      switch (g.cfg) {
        case 1: f ? launch<float, 256, 128, 16, ROWFAST, false>(b, bl, st)
                  : launch<float, 256, 128, 16, ROWMAJOR, false>(b, bl, st); break;
        case 2: f ? launch<float, 128, 256, 16, ROWFAST, false>(b, bl, st)
                  : launch<float, 128, 256, 16, ROWMAJOR, false>(b, bl, st); break;
        case 3: f ? launch<float, 256, 256, 16, ROWFAST, false>(b, bl, st)
                  : launch<float, 256, 256, 16, ROWMAJOR, false>(b, bl, st); break;
        case 4: f ? launch<float, 128, 128, 64, ROWFAST, false>(b, bl, st)
                  : launch<float, 128, 128, 64, ROWMAJOR, false>(b, bl, st); break;
        case 5: f ? launch<float, 256, 128, 32, ROWFAST, false>(b, bl, st)
                  : launch<float, 256, 128, 32, ROWMAJOR, false>(b, bl, st); break;
        case 6:
          if (f && (2 * g.K1 * g.K2) % 64 == 0 && g.K2 < (1 << 20) && g.ldw < (1 << 22))
            hipLaunchKernelGGL((site_gemm_4m_dtl<float, 128, 64, 3>), dim3((unsigned)bl), dim3(256), 0, st, b);
          else
            launch<float, 128, 128, 32, ROWMAJOR, false>(default_tiles(a, Z), default_blocks(a, Z), st);
          break;
        default: fail(PSIM_EINVAL, "unknown kernel config");
      }
    } else if (g.trans_out && g.N <= 32 && mode != GENERIC) {
      // last site of a row: few output columns, tall M -> 256 x 64 tiles
      b.MT = (b.M + 256 - 1) / 256;
      b.NT = (b.Nr + 64 - 1) / 64;
      b.T = b.MT * b.NT * Z;
      const long long bl = (b.T + 7) / 8 * 8;
      if (bl > 0x7fffffffLL) fail(PSIM_EUNSUPPORTED, "grid too large");
      if (mode == ROWMAJOR)
        launch<float, 256, 64, 16, ROWMAJOR, true>(b, bl, st);
      else
        launch<float, 256, 64, 16, KMAJOR, true>(b, bl, st);
    } else if (!g.trans_out && !g.nb && fast(128, 32) && (2 * g.K1 * g.K2) % 64 == 0 && g.K2 < (1 << 20) &&
               g.ldw < (1 << 22)) {
      // interior tiles, an even number of K stages: direct-to-LDS 4M kernel
      hipLaunchKernelGGL((site_gemm_4m_dtl<float, 128, 128, 2>), dim3((unsigned)blocks), dim3(256), 0, st, b);
    } else if (fast(128, 32))
      g.trans_out ? launch<float, 128, 128, 32, ROWFAST, true>(b, blocks, st)
                  : launch<float, 128, 128, 32, ROWFAST, false>(b, blocks, st);
    else if (mode == ROWMAJOR)
      g.trans_out ? launch<float, 128, 128, 32, ROWMAJOR, true>(b, blocks, st)
                  : launch<float, 128, 128, 32, ROWMAJOR, false>(b, blocks, st);
    else if (mode == KMAJOR)
      g.trans_out ? launch<float, 128, 128, 32, KMAJOR, true>(b, blocks, st)
                  : launch<float, 128, 128, 32, KMAJOR, false>(b, blocks, st);
    else
      g.trans_out ? launch<float, 128, 128, 32, GENERIC, true>(b, blocks, st)
                  : launch<float, 128, 128, 32, GENERIC, false>(b, blocks, st);
  }
  hip_check(hipGetLastError(), "site_gemm launch");
}

static unsigned grid_for(long long total) {
  return (unsigned)std::max<long long>(1, std::min<long long>((total + 255) / 256, 1 << 20));
}

void launch_permute3(int prec, const void* in, void* out, int64_t X, int64_t Y, int64_t Z, int mode, void* stream,
                     int64_t nodes, const uint32_t* mx) {
  if (X < 1 || Y < 1 || Z < 1 || (mode != 0 && mode != 1) || nodes < 1 || nodes > 65535)
    fail(PSIM_EINTERNAL, "permute3: bad arguments");
  hipStream_t st = (hipStream_t)stream;
  const long long total = X * Y * Z;
  const dim3 grid(grid_for(total), (unsigned)nodes);
  if (prec == PSIM_FP64)
    hipLaunchKernelGGL(permute3<double2>, grid, dim3(256), 0, st, (const double2*)in, (double2*)out, (long long)X,
                       (long long)Y, (long long)Z, mode, mx);
  else
    hipLaunchKernelGGL(permute3<float2>, grid, dim3(256), 0, st, (const float2*)in, (float2*)out, (long long)X,
                       (long long)Y, (long long)Z, mode, mx);
  hip_check(hipGetLastError(), "permute3 launch");
}

void launch_pack_w(int prec, const void* Q, void* P, int64_t N, int64_t K, int64_t rows, int64_t ld, void* stream,
                   int64_t nodes) {
  if (nodes < 1 || nodes > 65535) fail(PSIM_EINTERNAL, "pack_w: bad node count");
  hipStream_t st = (hipStream_t)stream;
  const long long total = rows * ld;
  const dim3 grid(grid_for(total), (unsigned)nodes);
  if (prec == PSIM_FP64)
    hipLaunchKernelGGL(pack_w<double>, grid, dim3(256), 0, st, (const double*)Q, (double*)P, (long long)N,
                       (long long)K, (long long)rows, (long long)ld, 0);
  else
    hipLaunchKernelGGL(pack_w<float>, grid, dim3(256), 0, st, (const float*)Q, (float*)P, (long long)N, (long long)K,
                       (long long)rows, (long long)ld, prec == PSIM_FP32_3M ? 1 : 0);
  hip_check(hipGetLastError(), "pack_w launch");
}

int cdot_blocks() { return 1024; }

void launch_cdot(int prec, const void* a, const void* b, int64_t n, double* part, double* out, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (prec == PSIM_FP64)
    hipLaunchKernelGGL(cdot_partial<double>, dim3(cdot_blocks()), dim3(256), 0, st, (const double*)a, (const double*)b,
                       (long long)n, part);
  else
    hipLaunchKernelGGL(cdot_partial<float>, dim3(cdot_blocks()), dim3(256), 0, st, (const float*)a, (const float*)b,
                       (long long)n, part);
  hipLaunchKernelGGL(cdot_finish, dim3(1), dim3(256), 0, st, (const double*)part, cdot_blocks(), out);
  hip_check(hipGetLastError(), "cdot launch");
}

void launch_copy_segments(const CopySeg* d_segs, int n, int64_t max_bytes, void* stream) {
  if (n < 1) return;
  if (n > 65535) fail(PSIM_EUNSUPPORTED, "too many segments for one gather");
  const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((max_bytes + 255) / 256, 64));
  hipLaunchKernelGGL(copy_segments, dim3(gx, (unsigned)n), dim3(256), 0, (hipStream_t)stream, d_segs);
  hip_check(hipGetLastError(), "gather launch");
}

bool rescale_fusable(int64_t per_node) { return 2 * per_node <= kFusedScaleReals; }
int max_scale_group() { return kMaxScale; }

void launch_rescale_group(int prec, const RescaleJob* jobs, int n, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (n < 1 || n > kMaxScale) fail(PSIM_EINTERNAL, "rescale group size out of range");
  ScaleArgs a{};
  long long total = 0;
  for (int i = 0; i < n; ++i) {
    if (!rescale_fusable(jobs[i].per_node)) fail(PSIM_EINTERNAL, "boundary too large for the fused rescale");
    a.p[i] = ScaleProb{jobs[i].F, jobs[i].per_node, jobs[i].parent, jobs[i].exp_prev, jobs[i].exp_cur};
    a.start[i] = total;
    total += jobs[i].nodes;
  }
  a.start[n] = total;
  a.n = n;
  if (total < 1) return;
  if (total > 0x7fffffffLL) fail(PSIM_EUNSUPPORTED, "grid too large");
  if (prec == PSIM_FP64)
    hipLaunchKernelGGL(row_rescale_fused<double>, dim3((unsigned)total), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(row_rescale_fused<float>, dim3((unsigned)total), dim3(256), 0, st, a);
  hip_check(hipGetLastError(), "fused rescale launch");
}

void launch_rowscale(int prec, void* F, int64_t per_node, int64_t nodes, const int32_t* parent,
                     const int32_t* exp_prev, int32_t* exp_cur, uint32_t* mx, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (rescale_fusable(per_node)) {  // small boundaries: one launch
    RescaleJob j{F, per_node, nodes, parent, exp_prev, exp_cur};
    launch_rescale_group(prec, &j, 1, stream);
    return;
  }
  const unsigned nb = (unsigned)((nodes + 255) / 256);
  hipLaunchKernelGGL(zero_u32, dim3(nb), dim3(256), 0, st, mx, nodes);
  long long per_block = 256 * 16;
  unsigned gx = (unsigned)std::min<long long>((2 * per_node + per_block - 1) / per_block, 4096);
  if (gx == 0) gx = 1;
  if (nodes > 65535) fail(PSIM_EUNSUPPORTED, "too many nodes for one rescale launch");
  if (prec == PSIM_FP64)
    hipLaunchKernelGGL(row_absmax<double>, dim3(gx, (unsigned)nodes), dim3(256), 0, st, (const double*)F, per_node, mx);
  else
    hipLaunchKernelGGL(row_absmax<float>, dim3(gx, (unsigned)nodes), dim3(256), 0, st, (const float*)F, per_node, mx);
  hipLaunchKernelGGL(row_exponent, dim3(nb), dim3(256), 0, st, nodes, parent, exp_prev, exp_cur, mx);
  if (prec == PSIM_FP64)
    hipLaunchKernelGGL(row_apply<double>, dim3(gx, (unsigned)nodes), dim3(256), 0, st, (double*)F, per_node, mx);
  else
    hipLaunchKernelGGL(row_apply<float>, dim3(gx, (unsigned)nodes), dim3(256), 0, st, (float*)F, per_node, mx);
  hip_check(hipGetLastError(), "rowscale launch");
}

void launch_row_exponents(int prec, const void* F, int64_t per_node, int64_t nodes, const int32_t* parent,
                          const int32_t* exp_prev, int32_t* exp_cur, uint32_t* mx, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const unsigned nb = (unsigned)((nodes + 255) / 256);
  if (nodes > 65535) fail(PSIM_EUNSUPPORTED, "too many nodes for one rescale launch");
  hipLaunchKernelGGL(zero_u32, dim3(nb), dim3(256), 0, st, mx, nodes);
  long long per_block = 256 * 16;
  unsigned gx = (unsigned)std::min<long long>((2 * per_node + per_block - 1) / per_block, 4096);
  if (gx == 0) gx = 1;
  if (prec == PSIM_FP64)
    hipLaunchKernelGGL(row_absmax<double>, dim3(gx, (unsigned)nodes), dim3(256), 0, st, (const double*)F, per_node, mx);
  else
    hipLaunchKernelGGL(row_absmax<float>, dim3(gx, (unsigned)nodes), dim3(256), 0, st, (const float*)F, per_node, mx);
  hipLaunchKernelGGL(row_exponent, dim3(nb), dim3(256), 0, st, nodes, parent, exp_prev, exp_cur, mx);
  hip_check(hipGetLastError(), "row exponent launch");
}

void launch_fill_ones(int prec, void* p, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (prec == PSIM_FP64)
    hipLaunchKernelGGL(fill_one<double>, dim3(1), dim3(1), 0, st, (double*)p);
  else
    hipLaunchKernelGGL(fill_one<float>, dim3(1), dim3(1), 0, st, (float*)p);
  hip_check(hipGetLastError(), "fill ones launch");
}

}  // namespace psim
