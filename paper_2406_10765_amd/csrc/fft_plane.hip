// Fused plane pass with compile-time sizes: for one z plane of one band, inverse 2D FFT of
// the stick data, multiplication by V(r), forward 2D FFT, gather of the stick positions.
//
// Each 1D FFT of length N = A * B is done in two register stages with one LDS exchange:
//   n = B n1 + n2:  Y[n2][k1] = W_N^{s n2 k1} * sum_n1 x[B n1 + n2] W_A^{s n1 k1}     (stage 1)
//                   X[k1 + A k2] = sum_n2 Y[n2][k1] W_B^{s n2 k2}                      (stage 2)
// (s = +1 inverse, -1 forward; W_M = exp(2 pi i / M)).  T = gcd(A, B) threads share a line:
// thread t takes n2 = t + T i in stage 1 and k1 = t + T j in stage 2.
// Along x the inverse transform, the V(r) multiplication and the forward transform run back to
// back: after the inverse stage 2 a thread holds y[m1 + A m2] for its m1 and every m2, which is
// exactly the input of the forward split m = m1 + A m2, q = B q1 + q2:
//   Z[m1][q2] = W_N^{-m1 q2} sum_m2 y[m1 + A m2] W_B^{-m2 q2}                        (in registers)
//   F[B q1 + q2] = sum_m1 Z[m1][q2] W_A^{-m1 q1}                                       (after one exchange)
// The small DFTs are fully unrolled with compile-time twiddles.

#include <type_traits>
#include <utility>

#include "common.hpp"
#include "kernels.hpp"

namespace pw {

// static loop: f(std::integral_constant<int, i>) for i in [0, N)
template <typename F, int... I>
__device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// ---- compile-time trigonometry (twiddles of the small DFTs) ------------------------------
constexpr double kPiC = 3.14159265358979323846264338327950288;
constexpr double csin(double x) {
  // reduce to [-pi, pi]
  while (x > kPiC) x -= 2 * kPiC;
  while (x < -kPiC) x += 2 * kPiC;
  double term = x, sum = x;
  for (int n = 1; n < 30; ++n) {
    term *= -x * x / ((2 * n) * (2 * n + 1));
    sum += term;
  }
  return sum;
}
constexpr double ccos(double x) { return csin(x + kPiC / 2); }

// In-register DFT of compile-time size S with sign SG (+1 inverse, -1 forward), natural order.
template <typename T, int S, int SG>
struct SmallDft {
  static __device__ __forceinline__ void run(cplx<T>* v) {
    if constexpr (S == 1) {
      return;
    } else if constexpr (S == 2) {
      const cplx<T> a = v[0], b = v[1];
      v[0] = cadd<T>(a, b);
      v[1] = csub<T>(a, b);
    } else if constexpr (S == 3) {
      const T h = (T)0.86602540378443864676;
      const cplx<T> t1 = cadd<T>(v[1], v[2]), t2 = csub<T>(v[1], v[2]);
      const cplx<T> m = mk<T>(v[0].x - (T)0.5 * t1.x, v[0].y - (T)0.5 * t1.y);
      const cplx<T> r = cmuli<T>(cscale<T>(t2, h), SG);
      v[0] = cadd<T>(v[0], t1);
      v[1] = cadd<T>(m, r);
      v[2] = csub<T>(m, r);
    } else if constexpr (S == 4) {
      const cplx<T> s02 = cadd<T>(v[0], v[2]), d02 = csub<T>(v[0], v[2]);
      const cplx<T> s13 = cadd<T>(v[1], v[3]);
      const cplx<T> d13 = cmuli<T>(csub<T>(v[1], v[3]), SG);
      v[0] = cadd<T>(s02, s13);
      v[2] = csub<T>(s02, s13);
      v[1] = cadd<T>(d02, d13);
      v[3] = csub<T>(d02, d13);
    } else {
      // S = F * G with F the first radix (4, 2 or 3): n = G f + g, k = kf + F kg
      constexpr int F = (S % 4 == 0) ? 4 : (S % 2 == 0) ? 2 : 3;
      constexpr int G = S / F;
      cplx<T> t[G][F];
      sfor<G>([&](auto gi) {
        constexpr int g = decltype(gi)::value;
        cplx<T> u[F];
#pragma unroll
        for (int f = 0; f < F; ++f) u[f] = v[G * f + g];
        SmallDft<T, F, SG>::run(u);
        sfor<F>([&](auto ki) {
          constexpr int kf = decltype(ki)::value;
          if constexpr (g * kf != 0) {
            constexpr double ang = SG * 2.0 * kPiC * (double)(g * kf) / (double)S;
            constexpr T wc = (T)ccos(ang), ws = (T)csin(ang);
            u[kf] = cmul<T>(u[kf], mk<T>(wc, ws));
          }
          t[g][kf] = u[kf];
        });
      });
#pragma unroll
      for (int kf = 0; kf < F; ++kf) {
        cplx<T> w[G];
#pragma unroll
        for (int g = 0; g < G; ++g) w[g] = t[g][kf];
        SmallDft<T, G, SG>::run(w);
#pragma unroll
        for (int kg = 0; kg < G; ++kg) v[kf + F * kg] = w[kg];
      }
    }
  }
};

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }

// One line FFT of length N = A B held in LDS (element e at base + e * es), T threads per line.
// In: natural order; out: natural order.  Barriers are executed by every thread of the block
// (active = false threads take part in the barriers only).
template <typename T, int A, int B, int SG>
__device__ __forceinline__ void line_fft(cplx<T>* buf, int base, int es, int t, bool active, const cplx<T>* twN) {
  constexpr int N = A * B, TT = cgcd(A, B), I1 = B / TT, J2 = A / TT;
  cplx<T> r1[I1][A];
  if (active) {
#pragma unroll
    for (int i = 0; i < I1; ++i)
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) r1[i][n1] = buf[base + (B * n1 + t + TT * i) * es];
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int i = 0; i < I1; ++i) {
      const int n2 = t + TT * i;
      SmallDft<T, A, SG>::run(r1[i]);
#pragma unroll
      for (int k1 = 1; k1 < A; ++k1) {
        cplx<T> w = twN[(n2 * k1) % N];
        if (SG > 0) w.y = -w.y;
        r1[i][k1] = cmul<T>(r1[i][k1], w);
      }
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) buf[base + (k1 * B + n2) * es] = r1[i][k1];
    }
  }
  __syncthreads();
  cplx<T> r2[J2][B];
  if (active) {
#pragma unroll
    for (int j = 0; j < J2; ++j) {
      const int k1 = t + TT * j;
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) r2[j][n2] = buf[base + (k1 * B + n2) * es];
      SmallDft<T, B, SG>::run(r2[j]);
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int j = 0; j < J2; ++j) {
      const int k1 = t + TT * j;
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) buf[base + (k1 + A * k2) * es] = r2[j][k2];
    }
  }
  __syncthreads();
}

// Row pass: inverse FFT, * V, forward FFT, in place on a row held in LDS (element stride 1).
template <typename T, int A, int B>
__device__ __forceinline__ void row_ivf(cplx<T>* buf, int base, int t, bool active, const cplx<T>* twN,
                                        const T* __restrict__ vrow) {
  constexpr int N = A * B, TT = cgcd(A, B), I1 = B / TT, J2 = A / TT;
  // inverse stage 1
  cplx<T> r1[I1][A];
  if (active) {
#pragma unroll
    for (int i = 0; i < I1; ++i)
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) r1[i][n1] = buf[base + B * n1 + t + TT * i];
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int i = 0; i < I1; ++i) {
      const int n2 = t + TT * i;
      SmallDft<T, A, +1>::run(r1[i]);
#pragma unroll
      for (int k1 = 1; k1 < A; ++k1) {
        cplx<T> w = twN[(n2 * k1) % N];
        w.y = -w.y;
        r1[i][k1] = cmul<T>(r1[i][k1], w);
      }
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) buf[base + k1 * B + n2] = r1[i][k1];
    }
  }
  __syncthreads();
  // inverse stage 2, * V, forward stage 1 (all in registers)
  cplx<T> r2[J2][B];
  if (active) {
#pragma unroll
    for (int j = 0; j < J2; ++j) {
      const int k1 = t + TT * j;
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) r2[j][n2] = buf[base + k1 * B + n2];
      SmallDft<T, B, +1>::run(r2[j]);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) r2[j][k2] = cscale<T>(r2[j][k2], vrow[k1 + A * k2]);
      SmallDft<T, B, -1>::run(r2[j]);  // over m2 = k2, output q2
#pragma unroll
      for (int q2 = 1; q2 < B; ++q2) r2[j][q2] = cmul<T>(r2[j][q2], twN[(k1 * q2) % N]);
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int j = 0; j < J2; ++j) {
      const int m1 = t + TT * j;
#pragma unroll
      for (int q2 = 0; q2 < B; ++q2) buf[base + q2 * A + m1] = r2[j][q2];
    }
  }
  __syncthreads();
  // forward stage 2: for each q2 of this thread, A-point DFT over m1
  cplx<T> r3[I1][A];
  if (active) {
#pragma unroll
    for (int i = 0; i < I1; ++i) {
      const int q2 = t + TT * i;
#pragma unroll
      for (int m1 = 0; m1 < A; ++m1) r3[i][m1] = buf[base + q2 * A + m1];
      SmallDft<T, A, -1>::run(r3[i]);
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int i = 0; i < I1; ++i) {
      const int q2 = t + TT * i;
#pragma unroll
      for (int q1 = 0; q1 < A; ++q1) buf[base + B * q1 + q2] = r3[i][q1];
    }
  }
  __syncthreads();
}

__device__ __forceinline__ int wrapn(int n, int N) { return n < 0 ? n + N : n; }

// Plane kernel for an N x N plane, N = A B.  Grid (n3, nbatch), NT threads.
// LDS: plane [y][x] with row stride N + 1, then the twiddle table W_N (forward sign).
template <typename T, int A, int B, int NT>
__global__ __launch_bounds__(NT) void k_plane_n(cplx<T>* __restrict__ SB, const T* __restrict__ V,
                                                const Stick* __restrict__ st, GridDesc g,
                                                const cplx<T>* __restrict__ twg, T scale) {
  constexpr int N = A * B, TT = cgcd(A, B), R = N + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* plane = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* tw = plane + N * R;
  const int tid = threadIdx.x;
  const int z = blockIdx.x, b = blockIdx.y;
  for (int i = tid; i < N * R; i += NT) plane[i] = mk<T>(0, 0);
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];
  __syncthreads();
  cplx<T>* sb = SB + ((long)b * g.n3 + z) * g.nst;
  for (int s = tid; s < g.nst; s += NT) {
    const Stick t = st[s];
    plane[wrapn(t.n2, N) * R + wrapn(t.n1, N)] = sb[s];
  }
  __syncthreads();
  // inverse along y on the active columns (lines = x, element stride R)
  {
    const int L = g.n1a;
    for (int l0 = 0; l0 < L; l0 += NT / TT) {
      const int l = l0 + tid % (NT / TT), t = min(tid / (NT / TT), TT);
      const bool act = l < L && t < TT;
      const int x = act ? (l <= g.n1max ? l : l + N - g.n1a) : 0;
      line_fft<T, A, B, +1>(plane, x, R, t, act, tw);
    }
  }
  // along x: inverse, * V, forward (lines = y rows)
  {
    const T* vz = V + (long)z * N * N;
    for (int l0 = 0; l0 < N; l0 += NT / TT) {
      const int y = l0 + tid % (NT / TT), t = min(tid / (NT / TT), TT);
      const bool act = y < N && t < TT;
      row_ivf<T, A, B>(plane, (act ? y : 0) * R, t, act, tw, vz + (long)(act ? y : 0) * N);
    }
  }
  // forward along y on the active columns
  {
    const int L = g.n1a;
    for (int l0 = 0; l0 < L; l0 += NT / TT) {
      const int l = l0 + tid % (NT / TT), t = min(tid / (NT / TT), TT);
      const bool act = l < L && t < TT;
      const int x = act ? (l <= g.n1max ? l : l + N - g.n1a) : 0;
      line_fft<T, A, B, -1>(plane, x, R, t, act, tw);
    }
  }
  for (int s = tid; s < g.nst; s += NT) {
    const Stick t = st[s];
    sb[s] = cscale<T>(plane[wrapn(t.n2, N) * R + wrapn(t.n1, N)], scale);
  }
}

// Sizes with a compile-time plane kernel: N = A B and threads per block.
template <typename T>
static bool launch_plane_n_sized(int N, cplx<T>* SB, const T* V, int nbatch, const Stick* st, const GridDesc& g,
                                 const cplx<T>* tw, T scale, hipStream_t s, hipError_t* err) {
  dim3 grid(g.n3, nbatch);
  const size_t lds = (size_t)(N * (N + 1) + N) * sizeof(cplx<T>);
#define PW_PLANE_CASE(NN, AA, BB, NTT)                                                                   \
  case NN:                                                                                               \
    hipLaunchKernelGGL((k_plane_n<T, AA, BB, NTT>), grid, dim3(NTT), lds, s, SB, V, st, g, tw, scale); \
    *err = hipGetLastError();                                                                            \
    return true;
  switch (N) {
    PW_PLANE_CASE(24, 4, 6, 256)
    PW_PLANE_CASE(27, 3, 9, 256)
    PW_PLANE_CASE(32, 4, 8, 256)
    PW_PLANE_CASE(48, 4, 12, 256)
    PW_PLANE_CASE(54, 6, 9, 256)
    PW_PLANE_CASE(64, 8, 8, 512)
    PW_PLANE_CASE(81, 9, 9, 768)
    PW_PLANE_CASE(96, 8, 12, 512)
    PW_PLANE_CASE(128, 8, 16, 1024)
    default:
      return false;
  }
#undef PW_PLANE_CASE
}

bool plane_n_supported(int n1, int n2, int real_bytes, size_t max_lds) {
  if (n1 != n2) return false;
  switch (n1) {
    case 24: case 27: case 32: case 48: case 54: case 64: case 81: case 96: case 128:
      break;
    default:
      return false;
  }
  const size_t lds = (size_t)(n1 * (n1 + 1) + n1) * 2 * real_bytes;
  return lds <= max_lds;
}

template <typename T>
hipError_t launch_plane_n(cplx<T>* SB, const T* V, int nbatch, const Stick* st, const GridDesc& g,
                          const cplx<T>* tw, T scale, hipStream_t s) {
  hipError_t e = hipErrorInvalidValue;
  if (!launch_plane_n_sized<T>(g.n1, SB, V, nbatch, st, g, tw, scale, s, &e)) return hipErrorInvalidValue;
  return e;
}

void pw_allow_large_lds_plane_n() {
  const int bytes = (int)(160 * 1024);
#define PW_ALLOW(AA, BB, NTT)                                                                                    \
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_plane_n<float, AA, BB, NTT>),                      \
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);                                 \
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_plane_n<double, AA, BB, NTT>),                     \
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  PW_ALLOW(4, 6, 256)
  PW_ALLOW(3, 9, 256)
  PW_ALLOW(4, 8, 256)
  PW_ALLOW(4, 12, 256)
  PW_ALLOW(6, 9, 256)
  PW_ALLOW(8, 8, 512)
  PW_ALLOW(9, 9, 768)
  PW_ALLOW(8, 12, 512)
  PW_ALLOW(8, 16, 1024)
#undef PW_ALLOW
}

template hipError_t launch_plane_n<float>(cplx<float>*, const float*, int, const Stick*, const GridDesc&,
                                          const cplx<float>*, float, hipStream_t);
template hipError_t launch_plane_n<double>(cplx<double>*, const double*, int, const Stick*, const GridDesc&,
                                           const cplx<double>*, double, hipStream_t);

}  // namespace pw
