// Complex GEMMs on the CDNA matrix cores (MFMA 16x16x4, fp64 or fp32).
//
// The dense contractions of the step (Section II-B: S = Psi^*(H Psi), and the
// per-atom pseudopotential application of Section III-A recast as projector
// GEMMs) all reduce to two shapes:
//   * "cn": C = A^H B with a very long inner dimension K = N_pw (projections
//     beta^H Y, Gram Y^H Y, projected Hamiltonian Y^H W).  Split over K; each
//     split writes complex-double partials that a second kernel sums in a
//     fixed order (deterministic, no atomics).  In fp32 the MFMA accumulators
//     are moved into fp64 registers every 256 K values, so the long sums keep
//     fp64-like accuracy.
//   * "nn": C = A B with K = N_proj or N_b and M = N_pw rows (beta (D P),
//     rotation Y C).  A fused epilogue assembles H Y or the Chebyshev update.
//
// Complex products run as four real MFMAs on the (re, im) planes:
//   conj(a) b: re += ar br + ai bi, im += ar bi - ai br
//   a b:       re += ar br - ai bi, im += ar bi + ai br
// MFMA 16x16x4 lane layout: operand A[i][k] comes from lane i + 16 k and
// operand B[k][j] from lane j + 16 k for both precisions; accumulator element r
// of lane l holds C[4 (l / 16) + r][l % 16] for f32 but C[l / 16 + 4 r][l % 16]
// for f64 (measured with one-hot operands on gfx950).
//
// Structure of one workgroup (4 waves in a 2 x 2 arrangement): global loads of
// the next K tile go to registers (16-byte loads where the leading dimension
// allows) while the MFMAs run on the current tile; the tiles live in two LDS
// buffers, so each K tile costs one barrier.  Tiles are handed out XCD by XCD:
// consecutive tiles, which share operand panels, run on the same L2.

#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace pw {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct MF;
template <> struct MF<double> {
  using acc = v4d;
  static __device__ __forceinline__ acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct MF<float> {
  using acc = v4f;
  static __device__ __forceinline__ acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int kBK = 16;     // K per tile (complex elements)
constexpr int kFlush = 16;  // fp32 cn: K tiles per move into fp64 registers
constexpr int kXcd = 8;     // XCDs per MI355X

// 16 bytes = U complex elements (U = 2 for fp32, 1 for fp64)
template <typename T> struct Vec16;
template <> struct Vec16<float> {
  using type = float4;
  static constexpr int U = 2;
};
template <> struct Vec16<double> {
  using type = double2;
  static constexpr int U = 1;
};

// Tile index -> (tm, tn, split) with the tiles of one XCD contiguous.  Launch order
// sends workgroup w to XCD w % 8.
__device__ __forceinline__ int xcd_tile(int w, int total) {
  const int per = total / kXcd, rem = total % kXcd;
  const int x = w % kXcd, i = w / kXcd;
  // XCDs 0..rem-1 get per + 1 tiles, the others per
  return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

// Loader of a K-contiguous operand panel: kBK values of NC columns starting at (k0, c0).
// Element (k, c) goes to S[k * LDS_LD + c].
template <typename T, int NC, bool VEC>
struct KcLoader {
  static constexpr int U = VEC ? Vec16<T>::U : 1;
  static constexpr int UNITS = kBK / U * NC;  // loads per tile
  static constexpr int PER = (UNITS + 255) / 256;
  cplx<T> r[PER][U];
  __device__ __forceinline__ void load(const cplx<T>* __restrict__ P, long ld, const cplx<T>* __restrict__ P2, long ld2,
                                       int ncol1, int ncols, int c0, int k0, int kend, int tid) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * 256;
      const int ku = idx % (kBK / U), c = idx / (kBK / U);
      const int gc = c0 + c, gk = k0 + ku * U;
#pragma unroll
      for (int u = 0; u < U; ++u) r[q][u] = mk<T>(0, 0);
      if (idx < UNITS && gc < ncols) {
        const cplx<T>* col = gc < ncol1 ? P + (long)gc * ld : P2 + (long)(gc - ncol1) * ld2;
        if (VEC && gk + U <= kend) {
          const typename Vec16<T>::type v = *reinterpret_cast<const typename Vec16<T>::type*>(col + gk);
          if constexpr (std::is_same<T, float>::value) {
            r[q][0] = mk<T>(v.x, v.y);
            r[q][U - 1] = mk<T>(v.z, v.w);
          } else {
            r[q][0] = mk<T>(v.x, v.y);
          }
        } else {
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (gk + u < kend) r[q][u] = col[gk + u];
        }
      }
    }
  }
  template <int LDS_LD>
  __device__ __forceinline__ void store(cplx<T>* S, int tid) const {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * 256;
      if (idx < UNITS) {
        const int ku = idx % (kBK / U), c = idx / (kBK / U);
#pragma unroll
        for (int u = 0; u < U; ++u) S[(ku * U + u) * LDS_LD + c] = r[q][u];
      }
    }
  }
};

// Loader of an M-contiguous operand panel (nn A): NR rows x kBK columns of a column-major matrix.
template <typename T, int NR, bool VEC>
struct McLoader {
  static constexpr int U = VEC ? Vec16<T>::U : 1;
  static constexpr int UNITS = NR / U * kBK;
  static constexpr int PER = (UNITS + 255) / 256;
  cplx<T> r[PER][U];
  __device__ __forceinline__ void load(const cplx<T>* __restrict__ P, long ld, int nrows, int r0, int k0, int kend,
                                       int tid) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * 256;
      const int mu = idx % (NR / U), k = idx / (NR / U);
      const int gm = r0 + mu * U, gk = k0 + k;
#pragma unroll
      for (int u = 0; u < U; ++u) r[q][u] = mk<T>(0, 0);
      if (idx < UNITS && gk < kend) {
        const cplx<T>* col = P + (long)gk * ld;
        if (VEC && gm + U <= nrows) {
          const typename Vec16<T>::type v = *reinterpret_cast<const typename Vec16<T>::type*>(col + gm);
          if constexpr (std::is_same<T, float>::value) {
            r[q][0] = mk<T>(v.x, v.y);
            r[q][U - 1] = mk<T>(v.z, v.w);
          } else {
            r[q][0] = mk<T>(v.x, v.y);
          }
        } else {
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (gm + u < nrows) r[q][u] = col[gm + u];
        }
      }
    }
  }
  template <int LDS_LD>
  __device__ __forceinline__ void store(cplx<T>* S, int tid) const {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * 256;
      if (idx < UNITS) {
        const int mu = idx % (NR / U), k = idx / (NR / U);
#pragma unroll
        for (int u = 0; u < U; ++u) S[k * LDS_LD + mu * U + u] = r[q][u];
      }
    }
  }
};

// A-operand loaders of one interface: load(A, lda, bg, extent, offset, k0, kend, tid) and
// store<LDS_LD>(S, tid).  The table loaders ignore bg; the generator loaders ignore A.
template <typename T, int NC, bool VEC>
struct CnATable {  // cn A: NC columns of a table
  KcLoader<T, NC, VEC> l;
  __device__ __forceinline__ void load(const cplx<T>* A, long lda, const BetaGen&, int ncols, int c0, int k0, int kend,
                                       int tid) {
    l.load(A, lda, A, lda, ncols, ncols, c0, k0, kend, tid);
  }
  template <int LDS_LD>
  __device__ __forceinline__ void store(cplx<T>* S, int tid) const {
    l.template store<LDS_LD>(S, tid);
  }
};
template <typename T, int NR, bool VEC>
struct NnATable {  // nn A: NR rows of a table
  McLoader<T, NR, VEC> l;
  __device__ __forceinline__ void load(const cplx<T>* A, long lda, const BetaGen&, int nrows, int r0, int k0, int kend,
                                       int tid) {
    l.load(A, lda, nrows, r0, k0, kend, tid);
  }
  template <int LDS_LD>
  __device__ __forceinline__ void store(cplx<T>* S, int tid) const {
    l.template store<LDS_LD>(S, tid);
  }
};

// The four projectors of atom a at plane wave g (zero outside the sphere / atom range).
template <typename T>
__device__ __forceinline__ void beta_gen4(const BetaGen& bg, int g, int a, cplx<T> (&v)[4]) {
  if (g >= bg.npw || a >= bg.natoms) {
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] = mk<T>(0, 0);
    return;
  }
  const int n1 = bg.miller[3 * g], n2 = bg.miller[3 * g + 1], n3 = bg.miller[3 * g + 2];
  const double2* p = bg.ph + (long)a * bg.w;
  const double2 e1 = p[n1 + bg.h1], e2 = p[bg.o2 + n2 + bg.h2], e3 = p[bg.o3 + n3 + bg.h3];
  const double2 e12 = make_double2(e1.x * e2.x - e1.y * e2.y, e1.x * e2.y + e1.y * e2.x);
  const double2 e = make_double2(e12.x * e3.x - e12.y * e3.y, e12.x * e3.y + e12.y * e3.x);
  const double4 r = *reinterpret_cast<const double4*>(bg.rad + 4 * (long)g);
  v[0] = mk<T>((T)(r.x * e.x), (T)(r.x * e.y));
  v[1] = mk<T>((T)(r.y * e.x), (T)(r.y * e.y));
  v[2] = mk<T>((T)(r.z * e.x), (T)(r.z * e.y));
  v[3] = mk<T>((T)(r.w * e.x), (T)(r.w * e.y));
}

template <typename T, int NC, bool VEC>
struct CnABeta {  // cn A = beta: NC columns (NC / 4 atoms from column c0) x kBK plane waves
  static constexpr int UNITS = kBK * (NC / 4);
  static constexpr int PER = (UNITS + 255) / 256;
  cplx<T> r[PER][4];
  __device__ __forceinline__ void load(const cplx<T>*, long, const BetaGen& bg, int, int c0, int k0, int kend,
                                       int tid) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * 256;
      const int k = idx % kBK, al = idx / kBK;
      const int g = k0 + k;
      beta_gen4<T>(bg, (idx < UNITS && g < kend) ? g : bg.npw, c0 / 4 + al, r[q]);
    }
  }
  template <int LDS_LD>
  __device__ __forceinline__ void store(cplx<T>* S, int tid) const {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * 256;
      if (idx < UNITS) {
        const int k = idx % kBK, al = idx / kBK;
#pragma unroll
        for (int m = 0; m < 4; ++m) S[k * LDS_LD + 4 * al + m] = r[q][m];
      }
    }
  }
};

template <typename T, int NR, bool VEC>
struct NnABeta {  // nn A = beta: NR plane waves from r0 x kBK columns (kBK / 4 atoms from k0)
  static constexpr int UNITS = NR * (kBK / 4);
  static constexpr int PER = (UNITS + 255) / 256;
  cplx<T> r[PER][4];
  __device__ __forceinline__ void load(const cplx<T>*, long, const BetaGen& bg, int nrows, int r0, int k0, int kend,
                                       int tid) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * 256;
      const int mu = idx % NR, al = idx / NR;
      const int g = r0 + mu, a = k0 / 4 + al;
      beta_gen4<T>(bg, (idx < UNITS && g < nrows && 4 * a < kend) ? g : bg.npw, a, r[q]);
    }
  }
  template <int LDS_LD>
  __device__ __forceinline__ void store(cplx<T>* S, int tid) const {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * 256;
      if (idx < UNITS) {
        const int mu = idx % NR, al = idx / NR;
#pragma unroll
        for (int m = 0; m < 4; ++m) S[(4 * al + m) * LDS_LD + mu] = r[q][m];
      }
    }
  }
};

// Wave-level MFMA accumulation over one K tile held in LDS.
// sA: kBK x (BM + 1) (m contiguous), sB: kBK x (BN + 1) (n contiguous).
template <typename T, int WBM, int WBN, bool CONJ_A>
__device__ __forceinline__ void mma_tile(const cplx<T>* sA, const cplx<T>* sB, int lda_s, int ldb_s, int mo, int no,
                                         int lane, typename MF<T>::acc (&cr)[WBM][WBN],
                                         typename MF<T>::acc (&ci)[WBM][WBN]) {
#pragma unroll
  for (int kk = 0; kk < kBK; kk += 4) {
    cplx<T> av[WBM], bv[WBN];
    const int kr = kk + (lane >> 4);
#pragma unroll
    for (int a = 0; a < WBM; ++a) av[a] = sA[kr * lda_s + mo + a * 16 + (lane & 15)];
#pragma unroll
    for (int b = 0; b < WBN; ++b) bv[b] = sB[kr * ldb_s + no + b * 16 + (lane & 15)];
#pragma unroll
    for (int a = 0; a < WBM; ++a)
#pragma unroll
      for (int b = 0; b < WBN; ++b) cr[a][b] = MF<T>::mma(av[a].x, bv[b].x, cr[a][b]);
#pragma unroll
    for (int a = 0; a < WBM; ++a)
#pragma unroll
      for (int b = 0; b < WBN; ++b) ci[a][b] = MF<T>::mma(av[a].x, bv[b].y, ci[a][b]);
#pragma unroll
    for (int a = 0; a < WBM; ++a) {
      const T ai = CONJ_A ? av[a].y : -av[a].y;
#pragma unroll
      for (int b = 0; b < WBN; ++b) cr[a][b] = MF<T>::mma(ai, bv[b].y, cr[a][b]);
    }
#pragma unroll
    for (int a = 0; a < WBM; ++a) {
      const T ai = CONJ_A ? -av[a].y : av[a].y;
#pragma unroll
      for (int b = 0; b < WBN; ++b) ci[a][b] = MF<T>::mma(ai, bv[b].x, ci[a][b]);
    }
  }
}

// ------------------------------------------------------------------------------------------
// cn: part[s] = A^H B over K chunk s.  Workgroup tile BM x BN (waves 2 x 2).
// ------------------------------------------------------------------------------------------
template <typename T, int BM, int BN, bool VEC, class AL>
__global__ __launch_bounds__(256) void k_gemm_cn(const cplx<T>* __restrict__ A, long lda,
                                                 const cplx<T>* __restrict__ B, long ldb,
                                                 const cplx<T>* __restrict__ B2, long ldb2, int ncol1, int M, int N,
                                                 int K, int kchunk, int tiles_m, int tiles_n,
                                                 double2* __restrict__ part, BetaGen bg) {
  constexpr int WBM = BM / 32, WBN = BN / 32;  // 16x16 blocks per wave
  constexpr int LA = BM + 1, LB = BN + 1;
  using acc_t = typename MF<T>::acc;
  __shared__ cplx<T> sA[2][kBK * LA];
  __shared__ cplx<T> sB[2][kBK * LB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nsplit = gridDim.x / (tiles_m * tiles_n);
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  // tiles of one split are contiguous; inside a split, n fastest
  const int sp = t / (tiles_m * tiles_n);
  const int tr = t - sp * tiles_m * tiles_n;
  const int tm = tr / tiles_n, tn = tr - tm * tiles_n;
  (void)nsplit;
  const int i0 = tm * BM, j0 = tn * BN;
  const int kb = sp * kchunk, ke = min(K, kb + kchunk);
  const int mo = (wave & 1) * (BM / 2), no = (wave >> 1) * (BN / 2);
  acc_t cr[WBM][WBN], ci[WBM][WBN];
  double dr[WBM][WBN][4], di[WBM][WBN][4];
#pragma unroll
  for (int a = 0; a < WBM; ++a)
#pragma unroll
    for (int b = 0; b < WBN; ++b) {
      cr[a][b] = acc_t{0, 0, 0, 0};
      ci[a][b] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int r = 0; r < 4; ++r) dr[a][b][r] = di[a][b][r] = 0.0;
    }
  AL la;
  KcLoader<T, BN, VEC> lb;
  const int ntiles = ke > kb ? (ke - kb + kBK - 1) / kBK : 0;
  if (ntiles > 0) {
    la.load(A, lda, bg, M, i0, kb, ke, tid);
    lb.load(B, ldb, B2, ldb2, ncol1, N, j0, kb, ke, tid);
    la.template store<LA>(sA[0], tid);
    lb.template store<LB>(sB[0], tid);
  }
  __syncthreads();
  for (int it = 0; it < ntiles; ++it) {
    const int cur = it & 1;
    const bool more = it + 1 < ntiles;
    if (more) {
      const int kn = kb + (it + 1) * kBK;
      la.load(A, lda, bg, M, i0, kn, ke, tid);
      lb.load(B, ldb, B2, ldb2, ncol1, N, j0, kn, ke, tid);
    }
    mma_tile<T, WBM, WBN, true>(sA[cur], sB[cur], LA, LB, mo, no, lane, cr, ci);
    if constexpr (std::is_same<T, float>::value) {
      if ((it % kFlush) == kFlush - 1) {
#pragma unroll
        for (int a = 0; a < WBM; ++a)
#pragma unroll
          for (int b = 0; b < WBN; ++b) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              dr[a][b][r] += (double)cr[a][b][r];
              di[a][b][r] += (double)ci[a][b][r];
            }
            cr[a][b] = acc_t{0, 0, 0, 0};
            ci[a][b] = acc_t{0, 0, 0, 0};
          }
      }
    }
    if (more) {
      la.template store<LA>(sA[cur ^ 1], tid);
      lb.template store<LB>(sB[cur ^ 1], tid);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < WBM; ++a)
#pragma unroll
    for (int b = 0; b < WBN; ++b) {
      const int col = j0 + no + b * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + mo + a * 16 + MF<T>::row(lane, r);
        if (row < M && col < N) {
          double2 v;
          v.x = dr[a][b][r] + (double)cr[a][b][r];
          v.y = di[a][b][r] + (double)ci[a][b][r];
          part[((long)sp * N + col) * M + row] = v;
        }
      }
    }
}

template <typename T>
__global__ void k_reduce_parts(const double2* __restrict__ part, int nsplit, int M, int N,
                               const double* __restrict__ dscale, int dper, double2* __restrict__ out64,
                               long ldo64, cplx<T>* __restrict__ outT, long ldoT) {
  PW_GRID_STRIDE(idx, (long)M * N) {
    const int j = (int)(idx / M), i = (int)(idx - (long)j * M);
    double2 s = part[idx];
    for (int p = 1; p < nsplit; ++p) {
      const double2 v = part[(long)p * M * N + idx];
      s.x += v.x;
      s.y += v.y;
    }
    if (dscale) {
      const double d = dscale[i % dper];
      s.x *= d;
      s.y *= d;
    }
    if (out64) out64[(long)j * ldo64 + i] = s;
    if (outT) outT[(long)j * ldoT + i] = mk<T>((T)s.x, (T)s.y);
  }
}

// ------------------------------------------------------------------------------------------
// nn: out = epilogue(A B).  A: M x K (m contiguous), B: K x N (k contiguous).
// ------------------------------------------------------------------------------------------
template <typename T, int BM, int BN, bool VEC, class AL>
__global__ __launch_bounds__(256) void k_gemm_nn(const cplx<T>* __restrict__ A, long lda,
                                                 const cplx<T>* __restrict__ B, long ldb, int M, int N, int K,
                                                 int tiles_n, cplx<T>* out, long ldo, EpiH e, BetaGen bg) {
  constexpr int WBM = BM / 32, WBN = BN / 32;
  constexpr int LA = BM + 1, LB = BN + 1;
  using acc_t = typename MF<T>::acc;
  __shared__ cplx<T> sA[2][kBK * LA];
  __shared__ cplx<T> sB[2][kBK * LB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int tm = t / tiles_n, tn = t - tm * tiles_n;  // n fastest: workgroups sharing an A panel are adjacent
  const int i0 = tm * BM, j0 = tn * BN;
  const int mo = (wave & 1) * (BM / 2), no = (wave >> 1) * (BN / 2);
  acc_t cr[WBM][WBN], ci[WBM][WBN];
#pragma unroll
  for (int a = 0; a < WBM; ++a)
#pragma unroll
    for (int b = 0; b < WBN; ++b) {
      cr[a][b] = acc_t{0, 0, 0, 0};
      ci[a][b] = acc_t{0, 0, 0, 0};
    }
  AL la;
  KcLoader<T, BN, VEC> lb;
  const int ntiles = (K + kBK - 1) / kBK;
  if (ntiles > 0) {
    la.load(A, lda, bg, M, i0, 0, K, tid);
    lb.load(B, ldb, B, ldb, N, N, j0, 0, K, tid);
    la.template store<LA>(sA[0], tid);
    lb.template store<LB>(sB[0], tid);
  }
  __syncthreads();
  for (int it = 0; it < ntiles; ++it) {
    const int cur = it & 1;
    const bool more = it + 1 < ntiles;
    if (more) {
      const int kn = (it + 1) * kBK;
      la.load(A, lda, bg, M, i0, kn, K, tid);
      lb.load(B, ldb, B, ldb, N, N, j0, kn, K, tid);
    }
    mma_tile<T, WBM, WBN, false>(sA[cur], sB[cur], LA, LB, mo, no, lane, cr, ci);
    if (more) {
      la.template store<LA>(sA[cur ^ 1], tid);
      lb.template store<LB>(sB[cur ^ 1], tid);
    }
    __syncthreads();
  }
  const T* kin = static_cast<const T*>(e.kin);
  const cplx<T>* Y = static_cast<const cplx<T>*>(e.Y);
  const cplx<T>* Zl = static_cast<const cplx<T>*>(e.Zl);
  const cplx<T>* Yp = static_cast<const cplx<T>*>(e.Yp);
  const T alpha = (T)e.alpha, cc = (T)e.c, beta = (T)e.beta;
#pragma unroll
  for (int a = 0; a < WBM; ++a)
#pragma unroll
    for (int b = 0; b < WBN; ++b) {
      const int col = j0 + no + b * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + mo + a * 16 + MF<T>::row(lane, r);
        if (row < M && col < N) {
          cplx<T> v = mk<T>(cr[a][b][r], ci[a][b][r]);
          if (e.mode == 1) {
            const cplx<T> y = Y[(long)col * e.ldy + row];
            const cplx<T> z = Zl[(long)col * e.ldz + row];
            const T kc = kin[row] - cc;
            v.x = alpha * (kc * y.x + z.x + v.x);
            v.y = alpha * (kc * y.y + z.y + v.y);
            if (Yp) {
              const cplx<T> p = Yp[(long)col * e.ldp + row];
              v.x -= beta * p.x;
              v.y -= beta * p.y;
            }
          }
          if (e.mode == 2) {
            const auto z = Zl[(long)col * e.ldz + row];
            v.x += z.x;
            v.y += z.y;
          }
          out[(long)col * ldo + row] = v;
        }
      }
    }
}

// ------------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------------
template <typename T> struct CnShape;
template <> struct CnShape<float> {
  static constexpr int BM = 128, BN = 64;
};
template <> struct CnShape<double> {
  static constexpr int BM = 64, BN = 64;
};
template <typename T> struct NnShape;
template <> struct NnShape<float> {
  static constexpr int BM = 128, BN = 128;
};
template <> struct NnShape<double> {
  static constexpr int BM = 128, BN = 64;
};

static inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

template <typename T>
static bool vec_ok(const void* p, long ld) {
  return aligned16(p) && (sizeof(T) == 8 || (ld % 2) == 0);
}

int gemm_cn_tiles(int M, int N, bool fp64) {
  const int bm = fp64 ? CnShape<double>::BM : CnShape<float>::BM;
  const int bn = fp64 ? CnShape<double>::BN : CnShape<float>::BN;
  return ceil_div(M, bm) * ceil_div(N, bn);
}

template <typename T>
hipError_t launch_gemm_cn(const cplx<T>* A, long lda, const cplx<T>* B, long ldb, const cplx<T>* B2, long ldb2,
                          int ncol1, int M, int N, int K, int nsplit, double2* part, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  constexpr int BM = CnShape<T>::BM, BN = CnShape<T>::BN;
  int kchunk = ceil_div(K, nsplit);
  kchunk = ceil_div(kchunk, kBK) * kBK;
  if (kchunk <= 0) kchunk = kBK;
  const int tm = ceil_div(M, BM), tn = ceil_div(N, BN);
  const cplx<T>* b2 = B2 ? B2 : B;
  const long l2 = B2 ? ldb2 : ldb;
  const bool vec = vec_ok<T>(A, lda) && vec_ok<T>(B, ldb) && vec_ok<T>(b2, l2);
  dim3 grid(tm * tn * nsplit);
  const BetaGen none{};
  if (vec)
    hipLaunchKernelGGL((k_gemm_cn<T, BM, BN, true, CnATable<T, BM, true>>), grid, dim3(256), 0, s, A, lda, B, ldb, b2,
                       l2, ncol1, M, N, K, kchunk, tm, tn, part, none);
  else
    hipLaunchKernelGGL((k_gemm_cn<T, BM, BN, false, CnATable<T, BM, false>>), grid, dim3(256), 0, s, A, lda, B, ldb,
                       b2, l2, ncol1, M, N, K, kchunk, tm, tn, part, none);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gemm_cn_beta(const BetaGen& bg, const cplx<T>* B, long ldb, int N, int nsplit, double2* part,
                               hipStream_t s) {
  const int M = 4 * bg.natoms, K = bg.npw;
  if (M <= 0 || N <= 0) return hipSuccess;
  constexpr int BM = CnShape<T>::BM, BN = CnShape<T>::BN;
  static_assert(BM % 4 == 0, "tile must hold whole atoms");
  int kchunk = ceil_div(K, nsplit);
  kchunk = ceil_div(kchunk, kBK) * kBK;
  if (kchunk <= 0) kchunk = kBK;
  const int tm = ceil_div(M, BM), tn = ceil_div(N, BN);
  const cplx<T>* A = nullptr;
  dim3 grid(tm * tn * nsplit);
  if (vec_ok<T>(B, ldb))
    hipLaunchKernelGGL((k_gemm_cn<T, BM, BN, true, CnABeta<T, BM, true>>), grid, dim3(256), 0, s, A, 0L, B, ldb, B,
                       ldb, N, M, N, K, kchunk, tm, tn, part, bg);
  else
    hipLaunchKernelGGL((k_gemm_cn<T, BM, BN, false, CnABeta<T, BM, false>>), grid, dim3(256), 0, s, A, 0L, B, ldb, B,
                       ldb, N, M, N, K, kchunk, tm, tn, part, bg);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_reduce_parts(const double2* part, int nsplit, int M, int N, const double* dscale, int dper,
                               double2* out64, long ldo64, cplx<T>* outT, long ldoT, hipStream_t s) {
  const long n = (long)M * N;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_parts<T>, dim3(stride_blocks(n)), dim3(256), 0, s, part, nsplit, M, N, dscale,
                     dper > 0 ? dper : 1, out64, ldo64, outT, ldoT);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gemm_nn(const cplx<T>* A, long lda, const cplx<T>* B, long ldb, int M, int N, int K,
                          cplx<T>* out, long ldo, const EpiH& e, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  constexpr int BM = NnShape<T>::BM, BN = NnShape<T>::BN;
  const int tm = ceil_div(M, BM), tn = ceil_div(N, BN);
  const bool vec = vec_ok<T>(A, lda) && vec_ok<T>(B, ldb);
  dim3 grid(tm * tn);
  const BetaGen none{};
  if (vec)
    hipLaunchKernelGGL((k_gemm_nn<T, BM, BN, true, NnATable<T, BM, true>>), grid, dim3(256), 0, s, A, lda, B, ldb, M,
                       N, K, tn, out, ldo, e, none);
  else
    hipLaunchKernelGGL((k_gemm_nn<T, BM, BN, false, NnATable<T, BM, false>>), grid, dim3(256), 0, s, A, lda, B, ldb,
                       M, N, K, tn, out, ldo, e, none);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gemm_nn_beta(const BetaGen& bg, const cplx<T>* B, long ldb, int N, cplx<T>* out, long ldo,
                               const EpiH& e, hipStream_t s) {
  const int M = bg.npw, K = 4 * bg.natoms;
  if (M <= 0 || N <= 0) return hipSuccess;
  constexpr int BM = NnShape<T>::BM, BN = NnShape<T>::BN;
  static_assert(kBK % 4 == 0, "K tile must hold whole atoms");
  const int tm = ceil_div(M, BM), tn = ceil_div(N, BN);
  const cplx<T>* A = nullptr;
  dim3 grid(tm * tn);
  if (vec_ok<T>(B, ldb))
    hipLaunchKernelGGL((k_gemm_nn<T, BM, BN, true, NnABeta<T, BM, true>>), grid, dim3(256), 0, s, A, 0L, B, ldb, M, N,
                       K, tn, out, ldo, e, bg);
  else
    hipLaunchKernelGGL((k_gemm_nn<T, BM, BN, false, NnABeta<T, BM, false>>), grid, dim3(256), 0, s, A, 0L, B, ldb, M,
                       N, K, tn, out, ldo, e, bg);
  return hipGetLastError();
}

#define PW_INST_GEMM(T)                                                                                      \
  template hipError_t launch_gemm_cn<T>(const cplx<T>*, long, const cplx<T>*, long, const cplx<T>*, long,   \
                                        int, int, int, int, int, double2*, hipStream_t);                     \
  template hipError_t launch_reduce_parts<T>(const double2*, int, int, int, const double*, int, double2*,   \
                                             long, cplx<T>*, long, hipStream_t);                             \
  template hipError_t launch_gemm_nn<T>(const cplx<T>*, long, const cplx<T>*, long, int, int, int, cplx<T>*, \
                                        long, const EpiH&, hipStream_t);                                     \
  template hipError_t launch_gemm_cn_beta<T>(const BetaGen&, const cplx<T>*, long, int, int, double2*,      \
                                             hipStream_t);                                                   \
  template hipError_t launch_gemm_nn_beta<T>(const BetaGen&, const cplx<T>*, long, int, cplx<T>*, long,     \
                                             const EpiH&, hipStream_t);
PW_INST_GEMM(float)
PW_INST_GEMM(double)

}  // namespace pw
