// Setup kernels (local potential on the sphere, projector table) and the small
// per-step kernels (conversions, Hermitian part, residual norms).

#include <cmath>

#include "../../include/pw.h"
#include "bf16split.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace pw {

constexpr double kPi = 3.14159265358979323846;

template <typename T>
__global__ void k_fill_zero(cplx<T>* p, long n) {
  PW_GRID_STRIDE(i, n) p[i] = mk<T>(0, 0);
}

// exp(-2 pi i t) with t reduced to [-1/2, 1/2] first (exact phase from Miller indices)
__device__ __forceinline__ double2 expm2pi(double t) {
  t -= rint(t);
  double s, c;
  sincospi(2.0 * t, &s, &c);
  return make_double2(c, -s);
}

// V(G) = S(G) v(|G|) + dV(G) on the sphere, with
//   v(G) = (1/Omega)(-4 pi Z e^{-G^2 rc^2/4}/G^2 + c e^{-G^2 rc^2/4}),  S(G) = sum_a e^{-i G.tau_a},
//   dV(+-G_k) = (amp_k / 2) e^{+-i phase_k};  V(0) = 0.
__global__ void k_vg_sphere(const int* __restrict__ miller, int npw, const double* __restrict__ frac,
                            const int* __restrict__ mm, const double* __restrict__ ma, const double* __restrict__ mp,
                            PotParams p, double2* __restrict__ vg) {
  __shared__ double sf[3 * 256];
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  int n1 = 0, n2 = 0, n3 = 0;
  if (g < npw) {
    n1 = miller[3 * g];
    n2 = miller[3 * g + 1];
    n3 = miller[3 * g + 2];
  }
  const double gx = 2.0 * kPi * n1 / p.L[0], gy = 2.0 * kPi * n2 / p.L[1], gz = 2.0 * kPi * n3 / p.L[2];
  const double g2 = gx * gx + gy * gy + gz * gz;
  double sre = 0.0, sim = 0.0;
  for (int a0 = 0; a0 < p.natoms; a0 += 256) {
    const int na = min(256, p.natoms - a0);
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * na; i += blockDim.x) sf[i] = frac[3 * a0 + i];
    __syncthreads();
    for (int a = 0; a < na; ++a) {
      const double2 e = expm2pi(n1 * sf[3 * a] + n2 * sf[3 * a + 1] + n3 * sf[3 * a + 2]);
      sre += e.x;
      sim += e.y;
    }
  }
  if (g >= npw) return;
  double2 out = make_double2(0.0, 0.0);
  if (g2 > 0.0 && 0.5 * g2 <= p.ecut) {
    const double omega = p.L[0] * p.L[1] * p.L[2];
    const double gauss = exp(-g2 * p.rc * p.rc / 4.0);
    const double v = (-4.0 * kPi * p.zval * gauss / g2 + p.gauss_c * gauss) / omega;
    out.x = v * sre;
    out.y = v * sim;
    for (int k = 0; k < p.nmodes; ++k) {
      const int m1 = mm[3 * k], m2 = mm[3 * k + 1], m3 = mm[3 * k + 2];
      if (n1 == m1 && n2 == m2 && n3 == m3) {
        out.x += 0.5 * ma[k] * cos(mp[k]);
        out.y += 0.5 * ma[k] * sin(mp[k]);
      } else if (n1 == -m1 && n2 == -m2 && n3 == -m3) {
        out.x += 0.5 * ma[k] * cos(mp[k]);
        out.y -= 0.5 * ma[k] * sin(mp[k]);
      }
    }
  }
  vg[g] = out;
}

// beta[g, 4a+m] = (c/sqrt(Omega)) e^{-sigma^2 |G|^2/2} Y_m(G) e^{-i G.tau_a},
// c = sqrt(32 pi^{5/2} sigma^3); Y_0 = 1/(2 sqrt(pi)), Y_{1x,y,z} = sqrt(3/(4 pi)) G_{x,y,z}/|G| (0 at G=0).
// form PW_PROJ_LOCALIZED: Y_{1m} = -i sigma G_m / sqrt(2 pi) (the transform of a Gaussian times r_m).
__device__ __forceinline__ void beta_values(const int* __restrict__ miller, int g, const double* __restrict__ frac,
                                            int a, double L0, double L1, double L2, double sigma, int form,
                                            double2 out[4]) {
  const int n1 = miller[3 * g], n2 = miller[3 * g + 1], n3 = miller[3 * g + 2];
  const double gx = 2.0 * kPi * n1 / L0, gy = 2.0 * kPi * n2 / L1, gz = 2.0 * kPi * n3 / L2;
  const double g2 = gx * gx + gy * gy + gz * gz;
  const double omega = L0 * L1 * L2;
  const double c = sqrt(32.0 * pow(kPi, 2.5) * sigma * sigma * sigma);
  const double radial = c / sqrt(omega) * exp(-0.5 * sigma * sigma * g2);
  const double y0 = 0.5 / sqrt(kPi);
  const double c1 = sqrt(3.0 / (4.0 * kPi));
  const double gn = sqrt(g2);
  const double inv = gn > 0.0 ? c1 / gn : 0.0;
  const double2 e = expm2pi(n1 * frac[3 * a] + n2 * frac[3 * a + 1] + n3 * frac[3 * a + 2]);
  if (form == PW_PROJ_LOCALIZED) {
    const double c2 = sigma / sqrt(2.0 * kPi);
    const double ym[4] = {y0, gx * c2, gy * c2, gz * c2};
    out[0] = make_double2(radial * y0 * e.x, radial * y0 * e.y);
#pragma unroll
    for (int m = 1; m < 4; ++m) {
      const double sc = radial * ym[m];
      out[m] = make_double2(sc * e.y, -sc * e.x);  // -i (e.x + i e.y)
    }
    return;
  }
  const double ym[4] = {y0, gx * inv, gy * inv, gz * inv};
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const double sc = radial * ym[m];
    out[m] = make_double2(sc * e.x, sc * e.y);
  }
}

template <typename T>
__global__ void k_beta_table(const int* __restrict__ miller, int npw, const double* __restrict__ frac, double L0,
                             double L1, double L2, double sigma, int form, cplx<T>* __restrict__ beta, long ld) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (g >= npw) return;
  double2 v[4];
  beta_values(miller, g, frac, a, L0, L1, L2, sigma, form, v);
#pragma unroll
  for (int m = 0; m < 4; ++m) beta[(long)(4 * a + m) * ld + g] = mk<T>((T)v[m].x, (T)v[m].y);
}

// The fp32 table stored as two bf16 planes: word (re, im) of hi = bf16(x) and of lo = bf16(x - hi),
// x the fp32 value; rows npw..ld-1 of every column are zero.
__global__ void k_beta_planes(const int* __restrict__ miller, int npw, const double* __restrict__ frac, double L0,
                              double L1, double L2, double sigma, int form, unsigned int* __restrict__ hi,
                              unsigned int* __restrict__ lo, long ld) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (g >= ld) return;
  double2 v[4] = {};
  if (g < npw) beta_values(miller, g, frac, a, L0, L1, L2, sigma, form, v);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const Split2 re = split((float)v[m].x), im = split((float)v[m].y);
    const long o = (long)(4 * a + m) * ld + g;
    hi[o] = pack(re.h, im.h);
    lo[o] = pack(re.l, im.l);
  }
}

// Tables of the on-the-fly projector generator: rad[4g+m] = (c/sqrt(Omega)) e^{-sigma^2|G|^2/2} Y_m(G)
// and, per atom, e^{-2 pi i n f_d} for each axis d and n in [-h_d, h_d].
__global__ void k_beta_rad(const int* __restrict__ miller, int npw, double L0, double L1, double L2, double sigma,
                           double* __restrict__ rad) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= npw) return;
  const int n1 = miller[3 * g], n2 = miller[3 * g + 1], n3 = miller[3 * g + 2];
  const double gx = 2.0 * kPi * n1 / L0, gy = 2.0 * kPi * n2 / L1, gz = 2.0 * kPi * n3 / L2;
  const double g2 = gx * gx + gy * gy + gz * gz;
  const double c = sqrt(32.0 * pow(kPi, 2.5) * sigma * sigma * sigma);
  const double radial = c / sqrt(L0 * L1 * L2) * exp(-0.5 * sigma * sigma * g2);
  const double c1 = sqrt(3.0 / (4.0 * kPi));
  const double gn = sqrt(g2);
  const double inv = gn > 0.0 ? c1 / gn : 0.0;
  rad[4 * (long)g] = radial * (0.5 / sqrt(kPi));
  rad[4 * (long)g + 1] = radial * gx * inv;
  rad[4 * (long)g + 2] = radial * gy * inv;
  rad[4 * (long)g + 3] = radial * gz * inv;
}

__global__ void k_beta_phase(BetaGen bg, const double* __restrict__ frac, double2* __restrict__ ph) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (i >= bg.w) return;
  int d, n;
  if (i < bg.o2) {
    d = 0;
    n = i - bg.h1;
  } else if (i < bg.o3) {
    d = 1;
    n = i - bg.o2 - bg.h2;
  } else {
    d = 2;
    n = i - bg.o3 - bg.h3;
  }
  ph[(long)a * bg.w + i] = expm2pi(n * frac[3 * a + d]);
}

hipError_t launch_beta_gen_tables(const BetaGen& bg, const double* frac, const double* L, double sigma, double* rad,
                                  double2* ph, hipStream_t s) {
  if (bg.npw > 0)
    hipLaunchKernelGGL(k_beta_rad, dim3(ceil_div(bg.npw, 256)), dim3(256), 0, s, bg.miller, bg.npw, L[0], L[1], L[2],
                       sigma, rad);
  if (bg.natoms > 0)
    hipLaunchKernelGGL(k_beta_phase, dim3(ceil_div(bg.w, 256), bg.natoms), dim3(256), 0, s, bg, frac, ph);
  return hipGetLastError();
}

template <typename T>
__global__ void k_convert(const double2* __restrict__ in, long ldi, cplx<T>* __restrict__ out, long ldo, int rows,
                          int cols) {
  PW_GRID_STRIDE(idx, (long)rows * cols) {
    const int j = (int)(idx / rows), i = (int)(idx - (long)j * rows);
    const double2 v = in[(long)j * ldi + i];
    out[(long)j * ldo + i] = mk<T>((T)v.x, (T)v.y);
  }
}

template <typename T>
__global__ void k_copy_cols(const cplx<T>* __restrict__ in, long ldi, cplx<T>* __restrict__ out, long ldo, int rows,
                            int cols) {
  PW_GRID_STRIDE(idx, (long)rows * cols) {
    const int j = (int)(idx / rows), i = (int)(idx - (long)j * rows);
    out[(long)j * ldo + i] = in[(long)j * ldi + i];
  }
}

template <typename T>
__global__ void k_scale_cols_lam(const double2* __restrict__ in, long ldi, cplx<T>* __restrict__ out, long ldo, int n,
                                 const double* __restrict__ lam, double sc) {
  PW_GRID_STRIDE(idx, (long)n * n) {
    const int j = (int)(idx / n), i = (int)(idx - (long)j * n);
    const double f = sc * lam[j];
    const double2 v = in[(long)j * ldi + i];
    out[(long)j * ldo + i] = mk<T>((T)(f * v.x), (T)(f * v.y));
  }
}

__global__ void k_hermitize(double2* A, long lda, int n) {
  PW_GRID_STRIDE(idx, (long)n * n) {
    const int j = (int)(idx / n), i = (int)(idx - (long)j * n);
    if (i < j) continue;
    double2 a = A[(long)j * lda + i];
    if (i == j) {
      a.y = 0.0;
      A[(long)j * lda + i] = a;
      continue;
    }
    const double2 b = A[(long)i * lda + j];
    const double2 m = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    A[(long)j * lda + i] = m;
    A[(long)i * lda + j] = make_double2(m.x, -m.y);
  }
}

// One workgroup per column; fp64 accumulation, wavefront shuffles then LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_resid(const cplx<T>* __restrict__ W, long ldw, const cplx<T>* __restrict__ X,
                                               long ldx, const double* __restrict__ lam, int rows,
                                               double* __restrict__ resid) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  const double l = lam ? lam[j] : 0.0;
  const cplx<T>* w = W + (long)j * ldw;
  const cplx<T>* x = X + (long)j * ldx;
  const double lj = lam ? l : 0.0;
  double s = 0.0;
  for (int i = threadIdx.x; i < rows; i += blockDim.x) {
    const cplx<T> a = w[i], b = x[i];
    const double rx = (double)a.x - lj * (double)b.x;
    const double ry = (double)a.y - lj * (double)b.y;
    s += rx * rx + ry * ry;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w2 = 0; w2 < (int)(blockDim.x >> 6); ++w2) t += red[w2];
    resid[j] = sqrt(t);
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_lanczos(cplx<T>* __restrict__ w, const cplx<T>* __restrict__ v,
                                                  const cplx<T>* __restrict__ vp, double bprev_h,
                                                  const double* __restrict__ bprev_d, int n,
                                                  double* __restrict__ sc) {
  __shared__ double red[16];
  __shared__ double alpha_s;
  const double bprev = bprev_d ? *bprev_d : bprev_h;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += (double)v[i].x * w[i].x + (double)v[i].y * w[i].y;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += red[k];
    alpha_s = t;
  }
  __syncthreads();
  const double a = alpha_s;
  double q = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    cplx<T> x = w[i];
    const double rx = (double)x.x - a * v[i].x - bprev * vp[i].x;
    const double ry = (double)x.y - a * v[i].y - bprev * vp[i].y;
    w[i] = mk<T>((T)rx, (T)ry);
    q += rx * rx + ry * ry;
  }
  __syncthreads();
  for (int off = 32; off > 0; off >>= 1) q += __shfl_down(q, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += red[k];
    sc[0] = a;
    sc[1] = sqrt(t);
  }
}

// out = in / beta with beta read from the device.  A beta below 1e-12 ends the recurrence on the
// host, which discards the later steps; the vector is then zeroed so that they stay finite.
template <typename T>
__global__ void k_scale_copy_inv(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                 const double* __restrict__ beta, int n) {
  const double b = *beta;
  const double scale = b < 1e-12 ? 0.0 : 1.0 / b;
  PW_GRID_STRIDE(i, (long)n) out[i] = mk<T>((T)(in[i].x * scale), (T)(in[i].y * scale));
}

template <typename T>
hipError_t launch_lanczos_step(cplx<T>* w, const cplx<T>* v, const cplx<T>* vp, double beta_prev,
                               const double* beta_prev_dev, int n, double* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_lanczos<T>, dim3(1), dim3(1024), 0, s, w, v, vp, beta_prev, beta_prev_dev, n, sc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scale_copy_inv(const cplx<T>* in, cplx<T>* out, const double* beta, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy_inv<T>, dim3(stride_blocks(n)), dim3(256), 0, s, in, out, beta, n);
  return hipGetLastError();
}

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

template <typename T>
__global__ void k_random_block(cplx<T>* __restrict__ X, long ld, int npw, int nb, const T* __restrict__ kin,
                               unsigned long long seed) {
  PW_GRID_STRIDE(idx, (long)npw * nb) {
    const int j = (int)(idx / npw), g = (int)(idx - (long)j * npw);
    const unsigned long long c = splitmix64(seed ^ splitmix64(((unsigned long long)j << 32) | (unsigned)g));
    const unsigned long long d = splitmix64(c);
    const double u1 = ((c >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = ((d >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double r = sqrt(-2.0 * log(u1)) / (1.0 + 2.0 * (double)kin[g]);
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    X[(long)j * ld + g] = mk<T>((T)(r * cs), (T)(r * sn));
  }
}

template <typename T>
__global__ void k_scale_cols_inv(cplx<T>* __restrict__ X, long ld, int npw, int nb, const double* __restrict__ nrm) {
  PW_GRID_STRIDE(idx, (long)npw * nb) {
    const int j = (int)(idx / npw), g = (int)(idx - (long)j * npw);
    const T s = (T)(1.0 / nrm[j]);
    cplx<T> v = X[(long)j * ld + g];
    X[(long)j * ld + g] = mk<T>(v.x * s, v.y * s);
  }
}

template <typename T>
hipError_t launch_random_block(cplx<T>* X, long ld, int npw, int nb, const T* kin, unsigned long long seed,
                               hipStream_t s) {
  const long n = (long)npw * nb;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_random_block<T>, dim3(stride_blocks(n)), dim3(256), 0, s, X, ld, npw, nb, kin, seed);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scale_cols_inv(cplx<T>* X, long ld, int npw, int nb, const double* norms, hipStream_t s) {
  const long n = (long)npw * nb;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_cols_inv<T>, dim3(stride_blocks(n)), dim3(256), 0, s, X, ld, npw, nb, norms);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_zero(cplx<T>* p, long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero<T>, dim3(stride_blocks(n)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_vg_sphere(const int* miller, int npw, const double* frac, const int* mode_miller,
                            const double* mode_amp, const double* mode_phase, PotParams p, double2* vg,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_vg_sphere, dim3(ceil_div(npw, 256)), dim3(256), 0, s, miller, npw, frac, mode_miller, mode_amp,
                     mode_phase, p, vg);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_beta_table(const int* miller, int npw, const double* frac, int natoms, const double* L,
                             double sigma, int form, cplx<T>* beta, long ld, hipStream_t s) {
  if (natoms <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_beta_table<T>, dim3(ceil_div(npw, 256), natoms), dim3(256), 0, s, miller, npw, frac, L[0], L[1],
                     L[2], sigma, form, beta, ld);
  return hipGetLastError();
}

hipError_t launch_beta_planes(const int* miller, int npw, const double* frac, int natoms, const double* L,
                              double sigma, int form, unsigned int* hi, unsigned int* lo, long ld, hipStream_t s) {
  if (natoms <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_beta_planes, dim3(ceil_div(ld, 256), natoms), dim3(256), 0, s, miller, npw, frac, L[0], L[1],
                     L[2], sigma, form, hi, lo, ld);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_convert_c64_to(const double2* in, long ldi, cplx<T>* out, long ldo, int rows, int cols,
                                 hipStream_t s) {
  const long n = (long)rows * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_convert<T>, dim3(stride_blocks(n)), dim3(256), 0, s, in, ldi, out, ldo, rows, cols);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy_cols(const cplx<T>* in, long ldi, cplx<T>* out, long ldo, int rows, int cols, hipStream_t s) {
  const long n = (long)rows * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_cols<T>, dim3(stride_blocks(n)), dim3(256), 0, s, in, ldi, out, ldo, rows, cols);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scale_cols_lam(const double2* in, long ldi, cplx<T>* out, long ldo, int n, const double* lam,
                                 double sc, hipStream_t st) {
  const long m = (long)n * n;
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_cols_lam<T>, dim3(stride_blocks(m)), dim3(256), 0, st, in, ldi, out, ldo, n, lam, sc);
  return hipGetLastError();
}

// theta[j] = Re(x_j^H w_j) / (x_j^H x_j) per column (FP64 accumulation), one block per column
template <typename T>
__global__ __launch_bounds__(256) void k_rayleigh(const cplx<T>* __restrict__ W, long ldw, const cplx<T>* __restrict__ X,
                                                  long ldx, int rows, double* __restrict__ theta) {
  __shared__ double red[2][4];
  const int j = blockIdx.x;
  const cplx<T>* w = W + (long)j * ldw;
  const cplx<T>* x = X + (long)j * ldx;
  double d = 0.0, n = 0.0;
  for (int i = threadIdx.x; i < rows; i += blockDim.x) {
    const cplx<T> a = w[i], b = x[i];
    d += (double)b.x * a.x + (double)b.y * a.y;
    n += (double)b.x * b.x + (double)b.y * b.y;
  }
  for (int off = 32; off > 0; off >>= 1) {
    d += __shfl_down(d, off, 64);
    n += __shfl_down(n, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = d;
    red[1][threadIdx.x >> 6] = n;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double td = 0.0, tn = 0.0;
    for (int w2 = 0; w2 < (int)(blockDim.x >> 6); ++w2) {
      td += red[0][w2];
      tn += red[1][w2];
    }
    theta[j] = td / tn;
  }
}

template <typename T>
hipError_t launch_rayleigh(const cplx<T>* W, long ldw, const cplx<T>* X, long ldx, int rows, int cols, double* theta,
                           hipStream_t s) {
  if (cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rayleigh<T>, dim3(cols), dim3(256), 0, s, W, ldw, X, ldx, rows, theta);
  return hipGetLastError();
}

// R[g, j] = (W[g, j] - theta_j X[g, j]) / (1 + kin[g]): preconditioned residual block
template <typename T>
__global__ void k_precond_resid(const cplx<T>* __restrict__ W, long ldw, const cplx<T>* __restrict__ X, long ldx,
                                const double* __restrict__ theta, const T* __restrict__ kin, int rows, int cols,
                                cplx<T>* __restrict__ R, long ldr) {
  PW_GRID_STRIDE(idx, (long)rows * cols) {
    const int j = (int)(idx / rows), g = (int)(idx - (long)j * rows);
    const double t = theta[j], p = 1.0 / (1.0 + (double)kin[g]);
    const cplx<T> w = W[(long)j * ldw + g], x = X[(long)j * ldx + g];
    R[(long)j * ldr + g] = mk<T>((T)(((double)w.x - t * x.x) * p), (T)(((double)w.y - t * x.y) * p));
  }
}

template <typename T>
hipError_t launch_precond_resid(const cplx<T>* W, long ldw, const cplx<T>* X, long ldx, const double* theta,
                                const T* kin, int rows, int cols, cplx<T>* R, long ldr, hipStream_t s) {
  const long n = (long)rows * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_precond_resid<T>, dim3(stride_blocks(n)), dim3(256), 0, s, W, ldw, X, ldx, theta, kin, rows,
                     cols, R, ldr);
  return hipGetLastError();
}
template hipError_t launch_rayleigh<float>(const float2*, long, const float2*, long, int, int, double*, hipStream_t);
template hipError_t launch_rayleigh<double>(const double2*, long, const double2*, long, int, int, double*,
                                            hipStream_t);
template hipError_t launch_precond_resid<float>(const float2*, long, const float2*, long, const double*,
                                                const float*, int, int, float2*, long, hipStream_t);
template hipError_t launch_precond_resid<double>(const double2*, long, const double2*, long, const double*,
                                                 const double*, int, int, double2*, long, hipStream_t);

// rho[r] (+)= sum over the nbt bands of occ[b] psq[b][r], bands in order (deterministic)
template <typename T>
__global__ void k_density_acc(const T* __restrict__ psq, int nbt, long nr, const double* __restrict__ occ,
                              double* __restrict__ rho, int first) {
  PW_GRID_STRIDE(r, nr) {
    double acc = first ? 0.0 : rho[r];
    for (int b = 0; b < nbt; ++b) acc += occ[b] * (double)psq[(long)b * nr + r];
    rho[r] = acc;
  }
}

template <typename T>
hipError_t launch_density_acc(const T* psq, int nbt, long nr, const double* occ, double* rho, bool first,
                              hipStream_t s) {
  if (nr <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_density_acc<T>, dim3(stride_blocks(nr)), dim3(256), 0, s, psq, nbt, nr, occ, rho,
                     first ? 1 : 0);
  return hipGetLastError();
}
template hipError_t launch_density_acc<float>(const float*, int, long, const double*, double*, bool, hipStream_t);
template hipError_t launch_density_acc<double>(const double*, int, long, const double*, double*, bool, hipStream_t);

__global__ void k_mirror_upper(double2* A, long lda, int n) {
  PW_GRID_STRIDE(idx, (long)n * n) {
    const int j = (int)(idx / n), i = (int)(idx - (long)j * n);
    if (i < j) continue;
    if (i == j) {
      A[(long)j * lda + i].y = 0.0;
      continue;
    }
    const double2 u = A[(long)i * lda + j];  // (j, i), upper
    A[(long)j * lda + i] = make_double2(u.x, -u.y);
  }
}

hipError_t launch_mirror_upper(double2* A, long lda, int n, hipStream_t s) {
  const long m = (long)n * n;
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mirror_upper, dim3(stride_blocks(m)), dim3(256), 0, s, A, lda, n);
  return hipGetLastError();
}

hipError_t launch_hermitize(double2* A, long lda, int n, hipStream_t s) {
  const long m = (long)n * n;
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hermitize, dim3(stride_blocks(m)), dim3(256), 0, s, A, lda, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_resid(const cplx<T>* W, long ldw, const cplx<T>* X, long ldx, const double* lam, int rows, int cols,
                        double* resid, hipStream_t s) {
  if (cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_resid<T>, dim3(cols), dim3(256), 0, s, W, ldw, X, ldx, lam, rows, resid);
  return hipGetLastError();
}

#define PW_INST_MISC(T)                                                                                         \
  template hipError_t launch_fill_zero<T>(cplx<T>*, long, hipStream_t);                                         \
  template hipError_t launch_beta_table<T>(const int*, int, const double*, int, const double*, double, int,      \
                                           cplx<T>*, long, hipStream_t);                                        \
  template hipError_t launch_convert_c64_to<T>(const double2*, long, cplx<T>*, long, int, int, hipStream_t);    \
  template hipError_t launch_copy_cols<T>(const cplx<T>*, long, cplx<T>*, long, int, int, hipStream_t);         \
  template hipError_t launch_lanczos_step<T>(cplx<T>*, const cplx<T>*, const cplx<T>*, double, const double*, int, \
                                             double*, hipStream_t);                                             \
  template hipError_t launch_scale_copy_inv<T>(const cplx<T>*, cplx<T>*, const double*, int, hipStream_t);     \
  template hipError_t launch_random_block<T>(cplx<T>*, long, int, int, const T*, unsigned long long, hipStream_t); \
  template hipError_t launch_scale_cols_inv<T>(cplx<T>*, long, int, int, const double*, hipStream_t);          \
  template hipError_t launch_scale_cols_lam<T>(const double2*, long, cplx<T>*, long, int, const double*, double,  \
                                               hipStream_t);                                                     \
  template hipError_t launch_resid<T>(const cplx<T>*, long, const cplx<T>*, long, const double*, int, int,      \
                                      double*, hipStream_t);
PW_INST_MISC(float)
PW_INST_MISC(double)

}  // namespace pw
