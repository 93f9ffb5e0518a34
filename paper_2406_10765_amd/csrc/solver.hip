// Kernels of the PPCG step and of the basis-selecting Rayleigh-Ritz (Section II-A names CG, PPCG
// and LOBPCG as the inner eigensolvers): per-column inner products in FP64, the per-column
// Rayleigh-Ritz on span{x_j, w_j, p_j} (at most 3 x 3, one thread per column, FP64 Jacobi), the
// column update, and the scaling kernels of the truncated SVQB basis of the large Rayleigh-Ritz.

#include <cmath>

#include "common.hpp"
#include "kernels.hpp"

namespace pw {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// conj(a) b accumulated into s
__device__ __forceinline__ void cdot_acc(double2& s, double2 a, double2 b) {
  s.x += a.x * b.x + a.y * b.y;
  s.y += a.x * b.y - a.y * b.x;
}
__device__ __forceinline__ double2 ld2(const float2* p, long i) {
  const float2 v = p[i];
  return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ double2 ld2(const double2* p, long i) { return p[i]; }

// Cyclic Jacobi on an n x n Hermitian matrix (n <= 3): A becomes diagonal (eigenvalues on the
// diagonal), V accumulates the unitary eigenvector matrix (columns).  Each rotation first takes
// the phase out of a_pq (A <- D^H A D, D = diag(.., e^{-i phi} at q, ..)) and then zeroes the now
// real a_pq by a real plane rotation.
__device__ void jacobi_herm(double2 (&A)[3][3], double2 (&V)[3][3], int n) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) V[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  for (int sweep = 0; sweep < 12; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int p = 0; p < n; ++p) {
      diag += A[p][p].x * A[p][p].x;
      for (int q = p + 1; q < n; ++q) off += A[p][q].x * A[p][q].x + A[p][q].y * A[p][q].y;
    }
    if (off <= 1e-32 * diag || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double b = hypot(A[p][q].x, A[p][q].y);
        if (b == 0.0) continue;
        // phase: column q times e^{-i phi}, row q times e^{+i phi}
        const double2 ph = make_double2(A[p][q].x / b, -A[p][q].y / b);  // e^{-i phi}
        for (int k = 0; k < n; ++k) {
          A[k][q] = cmul(A[k][q], ph);
          V[k][q] = cmul(V[k][q], ph);
        }
        for (int k = 0; k < n; ++k) A[q][k] = cmul(A[q][k], cconj(ph));
        A[p][q] = make_double2(b, 0.0);
        A[q][p] = make_double2(b, 0.0);
        // real rotation R = [[c, s], [-s, c]] in the (p, q) plane: A <- R^T A R, V <- V R
        const double tau = (A[q][q].x - A[p][p].x) / (2.0 * b);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double2 akp = A[k][p], akq = A[k][q];
          A[k][p] = cadd(cscale(akp, c), cscale(akq, -s));
          A[k][q] = cadd(cscale(akp, s), cscale(akq, c));
          const double2 vkp = V[k][p], vkq = V[k][q];
          V[k][p] = cadd(cscale(vkp, c), cscale(vkq, -s));
          V[k][q] = cadd(cscale(vkp, s), cscale(vkq, c));
        }
        for (int k = 0; k < n; ++k) {
          const double2 apk = A[p][k], aqk = A[q][k];
          A[p][k] = cadd(cscale(apk, c), cscale(aqk, -s));
          A[q][k] = cadd(cscale(apk, s), cscale(aqk, c));
        }
        A[p][q] = A[q][p] = make_double2(0.0, 0.0);
        A[p][p].y = A[q][q].y = 0.0;
      }
  }
}

}  // namespace

// Per column j: dots[j * 11 + e] for e = x^H x, x^H w, x^H p, w^H w, w^H p, p^H p,
// x^H (H w), x^H (H p), w^H (H w), w^H (H p), p^H (H p), FP64 accumulation in a fixed order
// (deterministic).  Without p (have_p == 0) its entries are zero.
template <typename T>
__global__ __launch_bounds__(256) void k_ppcg_dots(const cplx<T>* __restrict__ X, long ldx,
                                                   const cplx<T>* __restrict__ W, const cplx<T>* __restrict__ Pp,
                                                   const cplx<T>* __restrict__ HW, const cplx<T>* __restrict__ HP,
                                                   long ldz, int rows, int have_p, double2* __restrict__ dots) {
  constexpr int NE = 11;
  __shared__ double2 red[4][NE];
  const int j = blockIdx.x;
  const cplx<T>* x = X + (long)j * ldx;
  const cplx<T>* w = W + (long)j * ldz;
  const cplx<T>* p = Pp + (long)j * ldz;
  const cplx<T>* hw = HW + (long)j * ldz;
  const cplx<T>* hp = HP + (long)j * ldz;
  double2 s[NE];
  for (int e = 0; e < NE; ++e) s[e] = make_double2(0.0, 0.0);
  for (int i = threadIdx.x; i < rows; i += blockDim.x) {
    const double2 xv = ld2(x, i), wv = ld2(w, i), hwv = ld2(hw, i);
    cdot_acc(s[0], xv, xv);
    cdot_acc(s[1], xv, wv);
    cdot_acc(s[3], wv, wv);
    cdot_acc(s[6], xv, hwv);
    cdot_acc(s[8], wv, hwv);
    if (have_p) {
      const double2 pv = ld2(p, i), hpv = ld2(hp, i);
      cdot_acc(s[2], xv, pv);
      cdot_acc(s[4], wv, pv);
      cdot_acc(s[5], pv, pv);
      cdot_acc(s[7], xv, hpv);
      cdot_acc(s[9], wv, hpv);
      cdot_acc(s[10], pv, hpv);
    }
  }
  for (int e = 0; e < NE; ++e)
    for (int off = 32; off > 0; off >>= 1) {
      s[e].x += __shfl_down(s[e].x, off, 64);
      s[e].y += __shfl_down(s[e].y, off, 64);
    }
  if ((threadIdx.x & 63) == 0)
    for (int e = 0; e < NE; ++e) red[threadIdx.x >> 6][e] = s[e];
  __syncthreads();
  if (threadIdx.x < NE) {
    double2 t = make_double2(0.0, 0.0);
    for (int wv = 0; wv < 4; ++wv) t = cadd(t, red[wv][threadIdx.x]);
    dots[(long)j * NE + threadIdx.x] = t;
  }
}

// Per column j (one thread): the lowest Ritz vector of H on span{x_j, w_j, p_j} from the Gram
// matrix G and the matrix A of H on that basis (A_00 = lam_j, the Ritz value of x_j):
//   D = diag(G)^-1/2 (0 for a zero vector), D G D = U diag(sigma) U^H, the directions with
//   sigma <= drop_tol * max(sigma) dropped, T = D U_kept diag(sigma_kept)^-1/2,
//   T^H A T = V diag(mu) V^H, c = T v_min, phase fixed so that c_0 is real and >= 0.
// coef[j * 3 + i] = c_i (c_2 = 0 without p).
__global__ void k_ppcg_small(const double2* __restrict__ dots, const double* __restrict__ lam, int nb, int have_p,
                             double drop_tol, double2* __restrict__ coef) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nb) return;
  const double2* d = dots + (long)j * 11;
  const int n = have_p ? 3 : 2;
  double2 G[3][3], A[3][3];
  const double2 z = make_double2(0.0, 0.0);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) G[a][b] = A[a][b] = z;
  // upper triangles from the dots, lower by conjugation
  G[0][0] = d[0];
  G[0][1] = d[1];
  G[0][2] = d[2];
  G[1][1] = d[3];
  G[1][2] = d[4];
  G[2][2] = d[5];
  A[0][0] = make_double2(lam[j], 0.0);
  A[0][1] = d[6];
  A[0][2] = d[7];
  A[1][1] = d[8];
  A[1][2] = d[9];
  A[2][2] = d[10];
  for (int a = 0; a < 3; ++a) {
    G[a][a].y = 0.0;
    A[a][a].y = 0.0;
    for (int b = 0; b < a; ++b) {
      G[a][b] = cconj(G[b][a]);
      A[a][b] = cconj(A[b][a]);
    }
  }
  double sc[3];
  for (int a = 0; a < 3; ++a) sc[a] = (a < n && G[a][a].x > 0.0) ? 1.0 / sqrt(G[a][a].x) : 0.0;
  double2 Gt[3][3], U[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Gt[a][b] = cscale(G[a][b], sc[a] * sc[b]);
  jacobi_herm(Gt, U, n);
  double smax = 0.0;
  for (int a = 0; a < n; ++a) smax = fmax(smax, Gt[a][a].x);
  // T: kept columns of D U diag(sigma)^-1/2
  double2 Tm[3][3];
  int nk = 0;
  for (int c = 0; c < n; ++c) {
    const double sg = Gt[c][c].x;
    if (!(sg > drop_tol * smax) || !(smax > 0.0)) continue;
    const double f = 1.0 / sqrt(sg);
    for (int r = 0; r < 3; ++r) Tm[r][nk] = cscale(U[r][c], sc[r] * f);
    ++nk;
  }
  double2 c3[3] = {z, z, z};
  if (nk > 0) {
    // At = T^H A T (nk x nk)
    double2 AT[3][3], At[3][3], Vv[3][3];
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < nk; ++c) {
        double2 s = z;
        for (int k = 0; k < n; ++k) s = cadd(s, cmul(A[r][k], Tm[k][c]));
        AT[r][c] = s;
      }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) At[a][b] = z;
    for (int a = 0; a < nk; ++a)
      for (int b = 0; b < nk; ++b) {
        double2 s = z;
        for (int k = 0; k < n; ++k) s = cadd(s, cmul(cconj(Tm[k][a]), AT[k][b]));
        At[a][b] = s;
      }
    for (int a = 0; a < nk; ++a) {
      At[a][a].y = 0.0;
      for (int b = 0; b < a; ++b) {
        const double2 h = cscale(cadd(At[a][b], cconj(At[b][a])), 0.5);
        At[a][b] = h;
        At[b][a] = cconj(h);
      }
    }
    jacobi_herm(At, Vv, nk);
    int im = 0;
    for (int a = 1; a < nk; ++a)
      if (At[a][a].x < At[im][im].x) im = a;
    for (int r = 0; r < n; ++r) {
      double2 s = z;
      for (int k = 0; k < nk; ++k) s = cadd(s, cmul(Tm[r][k], Vv[k][im]));
      c3[r] = s;
    }
    const double a0 = hypot(c3[0].x, c3[0].y);
    if (a0 > 0.0) {
      const double2 ph = make_double2(c3[0].x / a0, -c3[0].y / a0);  // conj(c0) / |c0|
      for (int r = 0; r < n; ++r) c3[r] = cmul(c3[r], ph);
      c3[0].y = 0.0;
    }
  }
  for (int r = 0; r < 3; ++r) coef[(long)j * 3 + r] = c3[r];
}

// X[:, j] <- a_j x_j + b_j w_j + g_j p_j, Pd[:, j] <- b_j w_j + g_j p_j (coefficients in FP64,
// the sums in the data precision).
template <typename T>
__global__ void k_ppcg_update(cplx<T>* __restrict__ X, long ldx, cplx<T>* __restrict__ Pd, long ldp,
                              const cplx<T>* __restrict__ W, const cplx<T>* __restrict__ Pp, long ldz, int rows,
                              int cols, int have_p, const double2* __restrict__ coef) {
  PW_GRID_STRIDE(idx, (long)rows * cols) {
    const int j = (int)(idx / rows), g = (int)(idx - (long)j * rows);
    const double2 a = coef[(long)j * 3], b = coef[(long)j * 3 + 1], c = coef[(long)j * 3 + 2];
    const double2 x = ld2(X, (long)j * ldx + g), w = ld2(W, (long)j * ldz + g);
    double2 p = cmul(b, w);
    if (have_p) p = cadd(p, cmul(c, ld2(Pp, (long)j * ldz + g)));
    const double2 xn = cadd(cmul(a, x), p);
    X[(long)j * ldx + g] = mk<T>((T)xn.x, (T)xn.y);
    Pd[(long)j * ldp + g] = mk<T>((T)p.x, (T)p.y);
  }
}

template <typename T>
hipError_t launch_ppcg_dots(const cplx<T>* X, long ldx, const cplx<T>* W, const cplx<T>* Pp, const cplx<T>* HW,
                            const cplx<T>* HP, long ldz, int rows, int cols, int have_p, double2* dots,
                            hipStream_t s) {
  if (cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ppcg_dots<T>, dim3(cols), dim3(256), 0, s, X, ldx, W, Pp, HW, HP, ldz, rows, have_p, dots);
  return hipGetLastError();
}

hipError_t launch_ppcg_small(const double2* dots, const double* lam, int nb, int have_p, double drop_tol,
                             double2* coef, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ppcg_small, dim3((nb + 63) / 64), dim3(64), 0, s, dots, lam, nb, have_p, drop_tol, coef);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ppcg_update(cplx<T>* X, long ldx, cplx<T>* Pd, long ldp, const cplx<T>* W, const cplx<T>* Pp,
                              long ldz, int rows, int cols, int have_p, const double2* coef, hipStream_t s) {
  const long n = (long)rows * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ppcg_update<T>, dim3(stride_blocks(n)), dim3(256), 0, s, X, ldx, Pd, ldp, W, Pp, ldz, rows,
                     cols, have_p, coef);
  return hipGetLastError();
}

// ---- truncated SVQB basis of a k x k Gram matrix S (column-major, lds) -----------------------
// d_i = S_ii^-1/2 (0 when S_ii <= 0)
__global__ void k_svqb_diag(const double2* __restrict__ S, long lds, int k, double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const double v = S[(long)i * lds + i].x;
  d[i] = v > 0.0 ? 1.0 / sqrt(v) : 0.0;
}
// S <- D S D
__global__ void k_svqb_scale(double2* __restrict__ S, long lds, int k, const double* __restrict__ d) {
  PW_GRID_STRIDE(idx, (long)k * k) {
    const int j = (int)(idx / k), i = (int)(idx - (long)j * k);
    S[(long)j * lds + i] = cscale(S[(long)j * lds + i], d[i] * d[j]);
  }
}
// T[:, c] = D U[:, first + c] / sqrt(sigma[first + c]), c < kept
__global__ void k_svqb_basis(const double2* __restrict__ U, long ldu, int k, const double* __restrict__ sigma,
                             const double* __restrict__ d, int first, int kept, double2* __restrict__ Tm, long ldt) {
  PW_GRID_STRIDE(idx, (long)k * kept) {
    const int c = (int)(idx / k), i = (int)(idx - (long)c * k);
    const double f = d[i] / sqrt(sigma[first + c]);
    Tm[(long)c * ldt + i] = cscale(U[(long)(first + c) * ldu + i], f);
  }
}

// d_i = Re S_ii (before the factorisation overwrites S)
__global__ void k_diag_copy(const double2* __restrict__ S, long lds, int k, double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) d[i] = S[(long)i * lds + i].x;
}
// out = min_i |L_ii|^2 / d_i over the Cholesky factor L (one block; min is independent of order)
__global__ __launch_bounds__(256) void k_min_pivot(const double2* __restrict__ L, long ldl, int k,
                                                   const double* __restrict__ d, double* __restrict__ out) {
  __shared__ double red[256];
  double m = 1.0e300;
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    const double2 v = L[(long)i * ldl + i];
    const double r = d[i] > 0.0 ? (v.x * v.x + v.y * v.y) / d[i] : 0.0;
    m = fmin(m, r);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_diag_copy(const double2* S, long lds, int k, double* d, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag_copy, dim3((k + 255) / 256), dim3(256), 0, s, S, lds, k, d);
  return hipGetLastError();
}

hipError_t launch_min_pivot(const double2* L, long ldl, int k, const double* d, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_min_pivot, dim3(1), dim3(256), 0, s, L, ldl, k, d, out);
  return hipGetLastError();
}

hipError_t launch_svqb_scale(double2* S, long lds, int k, double* d, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_svqb_diag, dim3((k + 255) / 256), dim3(256), 0, s, S, lds, k, d);
  hipLaunchKernelGGL(k_svqb_scale, dim3(stride_blocks((long)k * k)), dim3(256), 0, s, S, lds, k, d);
  return hipGetLastError();
}

hipError_t launch_svqb_basis(const double2* U, long ldu, int k, const double* sigma, const double* d, int first,
                             int kept, double2* Tm, long ldt, hipStream_t s) {
  const long n = (long)k * kept;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_svqb_basis, dim3(stride_blocks(n)), dim3(256), 0, s, U, ldu, k, sigma, d, first, kept, Tm,
                     ldt);
  return hipGetLastError();
}

template hipError_t launch_ppcg_dots<float>(const float2*, long, const float2*, const float2*, const float2*,
                                            const float2*, long, int, int, int, double2*, hipStream_t);
template hipError_t launch_ppcg_dots<double>(const double2*, long, const double2*, const double2*, const double2*,
                                             const double2*, long, int, int, int, double2*, hipStream_t);
template hipError_t launch_ppcg_update<float>(float2*, long, float2*, long, const float2*, const float2*, long, int,
                                              int, int, const double2*, hipStream_t);
template hipError_t launch_ppcg_update<double>(double2*, long, double2*, long, const double2*, const double2*, long,
                                               int, int, int, const double2*, hipStream_t);

}  // namespace pw
