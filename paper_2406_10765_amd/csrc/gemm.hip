// Complex GEMMs on the CDNA matrix cores (MFMA 16x16x4, fp64 or fp32).
//
// The dense contractions of the step (Section II-B: S = Psi^*(H Psi), and the
// per-atom pseudopotential application of Section III-A recast as projector
// GEMMs) all reduce to two shapes:
//   * "cn": C = A^H B with a very long inner dimension K = N_pw (projections
//     beta^H Y, Gram Y^H Y, projected Hamiltonian Y^H W).  Split over K; each
//     split writes complex-double partials that a second kernel sums in a
//     fixed order (deterministic, no atomics).
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

constexpr int G_WM = 2, G_WN = 2;          // 16x16 blocks per wave (rows, cols)
constexpr int G_BM = 32 * G_WM, G_BN = 32 * G_WN, G_BK = 16;
constexpr int G_FLUSH = 16;                // fp32: move partial sums to fp64 every 16 K tiles

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_cn(const cplx<T>* __restrict__ A, long lda,
                                                 const cplx<T>* __restrict__ B, long ldb,
                                                 const cplx<T>* __restrict__ B2, long ldb2, int ncol1, int M,
                                                 int N, int K, int kchunk, double2* __restrict__ part) {
  using acc_t = typename MF<T>::acc;
  __shared__ cplx<T> sA[G_BK][G_BM + 1];
  __shared__ cplx<T> sB[G_BK][G_BN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int i0 = blockIdx.x * G_BM, j0 = blockIdx.y * G_BN, sp = blockIdx.z;
  const int kb = sp * kchunk, ke = min(K, kb + kchunk);
  acc_t cr[G_WM][G_WN], ci[G_WM][G_WN];
  double dr[G_WM][G_WN][4], di[G_WM][G_WN][4];
#pragma unroll
  for (int a = 0; a < G_WM; ++a)
#pragma unroll
    for (int b = 0; b < G_WN; ++b) {
      cr[a][b] = acc_t{0, 0, 0, 0};
      ci[a][b] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int r = 0; r < 4; ++r) dr[a][b][r] = di[a][b][r] = 0.0;
    }
  const cplx<T> zero = mk<T>(0, 0);
  int tile = 0;
  for (int k0 = kb; k0 < ke; k0 += G_BK, ++tile) {
#pragma unroll
    for (int r = 0; r < G_BK * G_BM / 256; ++r) {
      const int idx = tid + r * 256;
      const int kk = idx & (G_BK - 1), ii = idx / G_BK;
      const int gi = i0 + ii, gk = k0 + kk;
      sA[kk][ii] = (gi < M && gk < ke) ? A[(long)gi * lda + gk] : zero;
    }
#pragma unroll
    for (int r = 0; r < G_BK * G_BN / 256; ++r) {
      const int idx = tid + r * 256;
      const int kk = idx & (G_BK - 1), jj = idx / G_BK;
      const int gj = j0 + jj, gk = k0 + kk;
      cplx<T> v = zero;
      if (gj < N && gk < ke) v = gj < ncol1 ? B[(long)gj * ldb + gk] : B2[(long)(gj - ncol1) * ldb2 + gk];
      sB[kk][jj] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < G_BK; kk += 4) {
      cplx<T> av[G_WM], bv[G_WN];
#pragma unroll
      for (int a = 0; a < G_WM; ++a) av[a] = sA[kk + (lane >> 4)][wm * 16 * G_WM + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < G_WN; ++b) bv[b] = sB[kk + (lane >> 4)][wn * 16 * G_WN + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < G_WM; ++a)
#pragma unroll
        for (int b = 0; b < G_WN; ++b) {
          cr[a][b] = MF<T>::mma(av[a].x, bv[b].x, cr[a][b]);
          cr[a][b] = MF<T>::mma(av[a].y, bv[b].y, cr[a][b]);
          ci[a][b] = MF<T>::mma(av[a].x, bv[b].y, ci[a][b]);
          ci[a][b] = MF<T>::mma(-av[a].y, bv[b].x, ci[a][b]);
        }
    }
    __syncthreads();
    if constexpr (std::is_same<T, float>::value) {
      if ((tile & (G_FLUSH - 1)) == G_FLUSH - 1) {
#pragma unroll
        for (int a = 0; a < G_WM; ++a)
#pragma unroll
          for (int b = 0; b < G_WN; ++b) {
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
  }
#pragma unroll
  for (int a = 0; a < G_WM; ++a)
#pragma unroll
    for (int b = 0; b < G_WN; ++b) {
      const int col = j0 + wn * 16 * G_WN + b * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + wm * 16 * G_WM + a * 16 + MF<T>::row(lane, r);
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
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)M * N) return;
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

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_nn(const cplx<T>* __restrict__ A, long lda,
                                                 const cplx<T>* __restrict__ B, long ldb, int M, int N, int K,
                                                 cplx<T>* out, long ldo, EpiH e) {
  using acc_t = typename MF<T>::acc;
  __shared__ cplx<T> sA[G_BK][G_BM + 1];
  __shared__ cplx<T> sB[G_BK][G_BN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int i0 = blockIdx.x * G_BM, j0 = blockIdx.y * G_BN;
  acc_t cr[G_WM][G_WN], ci[G_WM][G_WN];
#pragma unroll
  for (int a = 0; a < G_WM; ++a)
#pragma unroll
    for (int b = 0; b < G_WN; ++b) {
      cr[a][b] = acc_t{0, 0, 0, 0};
      ci[a][b] = acc_t{0, 0, 0, 0};
    }
  const cplx<T> zero = mk<T>(0, 0);
  for (int k0 = 0; k0 < K; k0 += G_BK) {
#pragma unroll
    for (int r = 0; r < G_BK * G_BM / 256; ++r) {
      const int idx = tid + r * 256;
      const int ii = idx & (G_BM - 1), kk = idx / G_BM;
      const int gi = i0 + ii, gk = k0 + kk;
      sA[kk][ii] = (gi < M && gk < K) ? A[(long)gk * lda + gi] : zero;
    }
#pragma unroll
    for (int r = 0; r < G_BK * G_BN / 256; ++r) {
      const int idx = tid + r * 256;
      const int kk = idx & (G_BK - 1), jj = idx / G_BK;
      const int gj = j0 + jj, gk = k0 + kk;
      sB[kk][jj] = (gj < N && gk < K) ? B[(long)gj * ldb + gk] : zero;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < G_BK; kk += 4) {
      cplx<T> av[G_WM], bv[G_WN];
#pragma unroll
      for (int a = 0; a < G_WM; ++a) av[a] = sA[kk + (lane >> 4)][wm * 16 * G_WM + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < G_WN; ++b) bv[b] = sB[kk + (lane >> 4)][wn * 16 * G_WN + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < G_WM; ++a)
#pragma unroll
        for (int b = 0; b < G_WN; ++b) {
          cr[a][b] = MF<T>::mma(av[a].x, bv[b].x, cr[a][b]);
          cr[a][b] = MF<T>::mma(-av[a].y, bv[b].y, cr[a][b]);
          ci[a][b] = MF<T>::mma(av[a].x, bv[b].y, ci[a][b]);
          ci[a][b] = MF<T>::mma(av[a].y, bv[b].x, ci[a][b]);
        }
    }
    __syncthreads();
  }
  const T* kin = static_cast<const T*>(e.kin);
  const cplx<T>* Y = static_cast<const cplx<T>*>(e.Y);
  const cplx<T>* Zl = static_cast<const cplx<T>*>(e.Zl);
  const cplx<T>* Yp = static_cast<const cplx<T>*>(e.Yp);
  const T alpha = (T)e.alpha, cc = (T)e.c, beta = (T)e.beta;
#pragma unroll
  for (int a = 0; a < G_WM; ++a)
#pragma unroll
    for (int b = 0; b < G_WN; ++b) {
      const int col = j0 + wn * 16 * G_WN + b * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + wm * 16 * G_WM + a * 16 + MF<T>::row(lane, r);
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
          out[(long)col * ldo + row] = v;
        }
      }
    }
}

template <typename T>
hipError_t launch_gemm_cn(const cplx<T>* A, long lda, const cplx<T>* B, long ldb, const cplx<T>* B2, long ldb2,
                          int ncol1, int M, int N, int K, int nsplit, double2* part, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  int kchunk = ceil_div(K, nsplit);
  kchunk = ceil_div(kchunk, G_BK) * G_BK;
  if (kchunk <= 0) kchunk = G_BK;
  dim3 grid(ceil_div(M, G_BM), ceil_div(N, G_BN), nsplit);
  hipLaunchKernelGGL(k_gemm_cn<T>, grid, dim3(256), 0, s, A, lda, B, ldb, B2 ? B2 : B, ldb2, ncol1, M, N, K,
                     kchunk, part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_reduce_parts(const double2* part, int nsplit, int M, int N, const double* dscale, int dper,
                               double2* out64, long ldo64, cplx<T>* outT, long ldoT, hipStream_t s) {
  const long n = (long)M * N;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_parts<T>, dim3(ceil_div(n, 256)), dim3(256), 0, s, part, nsplit, M, N, dscale,
                     dper > 0 ? dper : 1, out64, ldo64, outT, ldoT);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gemm_nn(const cplx<T>* A, long lda, const cplx<T>* B, long ldb, int M, int N, int K,
                          cplx<T>* out, long ldo, const EpiH& e, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid(ceil_div(M, G_BM), ceil_div(N, G_BN));
  hipLaunchKernelGGL(k_gemm_nn<T>, grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, out, ldo, e);
  return hipGetLastError();
}

#define PW_INST_GEMM(T)                                                                                      \
  template hipError_t launch_gemm_cn<T>(const cplx<T>*, long, const cplx<T>*, long, const cplx<T>*, long,   \
                                        int, int, int, int, int, double2*, hipStream_t);                     \
  template hipError_t launch_reduce_parts<T>(const double2*, int, int, int, const double*, int, double2*,   \
                                             long, cplx<T>*, long, hipStream_t);                             \
  template hipError_t launch_gemm_nn<T>(const cplx<T>*, long, const cplx<T>*, long, int, int, int, cplx<T>*, \
                                        long, const EpiH&, hipStream_t);
PW_INST_GEMM(float)
PW_INST_GEMM(double)

}  // namespace pw
