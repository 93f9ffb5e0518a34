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
// vr[j][k2] = V at x = k1 + A k2 with k1 = t + gcd(A, B) j (loaded by the caller ahead of time).
template <typename T, int A, int B>
__device__ __forceinline__ void row_ivf(cplx<T>* buf, int base, int t, bool active, const cplx<T>* twN,
                                        const T (&vr)[A / cgcd(A, B)][B]) {
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
      for (int k2 = 0; k2 < B; ++k2) r2[j][k2] = cscale<T>(r2[j][k2], vr[j][k2]);
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
  constexpr int N = A * B, TT = cgcd(A, B), R = N + 1, J2 = A / TT;
  static_assert(NT / TT >= N, "one row per thread group");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* plane = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* tw = plane + N * R;
  const int tid = threadIdx.x;
  const int z = blockIdx.x, b = blockIdx.y;
  // V(r) of this thread's row, fetched first so that its latency hides behind the y pass
  const int yrow = tid % (NT / TT), trow = min(tid / (NT / TT), TT);
  const bool row_act = yrow < N && trow < TT;
  T vr[J2][B];
  {
    const T* vz = V + ((long)z * N + (row_act ? yrow : 0)) * N;
#pragma unroll
    for (int j = 0; j < J2; ++j)
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) vr[j][k2] = row_act ? vz[(trow + TT * j) + A * k2] : (T)0;
  }
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
  // along x: inverse, * V, forward (lines = y rows, one per thread group)
  row_ivf<T, A, B>(plane, (row_act ? yrow : 0) * R, trow, row_act, tw, vr);
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

// ---- real-space projectors on 128 x 128 FP32 planes --------------------------------------------
// The projectors are truncated to the grid points within a radius R of their atom (Section III-A:
// a projector acts only near its atom).  An entry (atom, plane) holds unwrapped ranges of columns
// x0 .. x0+nx-1 and rows y0 .. y0+ny-1 (mod 128 on the plane) that contain every point of the disc
// the ball cuts from the plane; a point lies in the ball when dx^2 + (dy^2 + dz^2) <= R^2.  The
// Gaussian factors as e^{-dx^2/(2 s^2)} e^{-(dy^2 + dz^2)/(2 s^2)}.  Both passes evaluate points
// through rs_colpart / rs_row / rs_in, so they see the same points and the same values.
//  * The projection pass holds the plane in LDS (row y in natural x order, word y * 128 + x) and
//    gives each wave whole (atom, plane) entries: its lanes cover the disc, 16, 32 or 64 columns
//    at a time, and one reduction across the wave ends each entry.
//  * The pass of V(r) adds D P on the x pass itself, where lane (l, t) of wave w holds the 16 values
//    of row y = 8w + l at x = t + 8k in registers: the wave walks the entries of its 8-row band and
//    visits only the 8-column blocks that an entry's columns meet (a wave-uniform mask).
// value of lane k of v (k uniform over the wave)
__device__ __forceinline__ float rs_lane(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ __forceinline__ int rs_lane(int v, int k) { return __builtin_amdgcn_readlane(v, k); }

// One entry's data, loaded by lane k of the wave, then read by the whole wave with rs_entry.
struct RsLaneEnt {
  float dz, bx, by;
  int xr, yr;  // x0 | nx << 16 and y0 | ny << 16 (x0, y0 as 16-bit two's complement)
  int mask;
};
__device__ __forceinline__ RsLaneEnt rs_load(const RsEnt& en) {
  RsLaneEnt l;
  l.dz = en.dz;
  l.bx = en.bx;
  l.by = en.by;
  l.xr = (int)(unsigned short)en.x0 | ((int)en.nx << 16);
  l.yr = (int)(unsigned short)en.y0 | ((int)en.ny << 16);
  l.mask = en.mask;
  return l;
}
__device__ __forceinline__ RsLaneEnt rs_empty() {
  RsLaneEnt l;
  l.dz = l.bx = l.by = 0.f;
  l.xr = l.yr = 0;
  l.mask = 0;
  return l;
}

struct RsEntry {
  float dz, dz2, bx, by;
  int x0, nx, y0, ny;
  unsigned mask;  // bit k: columns 8k .. 8k+7 meet x0 .. x0+nx-1 (mod 128)
};
__device__ __forceinline__ RsEntry rs_entry(const RsLaneEnt& l, int k) {
  RsEntry e;
  e.dz = rs_lane(l.dz, k);
  e.dz2 = e.dz * e.dz;
  e.bx = rs_lane(l.bx, k);
  e.by = rs_lane(l.by, k);
  const int xr = rs_lane(l.xr, k), yr = rs_lane(l.yr, k);
  e.x0 = (int)(short)(xr & 0xffff);
  e.nx = xr >> 16;
  e.y0 = (int)(short)(yr & 0xffff);
  e.ny = yr >> 16;
  e.mask = (unsigned)rs_lane(l.mask, k);
  return e;
}

// Row part of row y (0 .. 127): whether it is in the entry's rows, dy, dy^2 + dz^2 and
// e^{-(dy^2 + dz^2)/(2 s^2)}.
struct RsRow {
  bool ok;
  float dy, s, gyz;
};
__device__ __forceinline__ RsRow rs_row(const RsDesc& d, const RsEntry& e, int y) {
  RsRow w;
  const int oy = (y - e.y0) & 127;
  w.ok = oy < e.ny;
  w.dy = fmaf((float)oy, d.hy, e.by);
  w.s = fmaf(w.dy, w.dy, e.dz2);
  w.gyz = __builtin_amdgcn_exp2f(w.s * d.k2);
  return w;
}
// Column part of column x (0 .. 127): dx, dx^2 and e^{-dx^2/(2 s^2)}.  A column outside the entry's
// range needs no test of its own: its dx exceeds the disc radius of the enlarged range radius, so
// the ball test below rejects it (by a margin of 2e-4 of R^2, far above FP32 rounding).
struct RsCol {
  float dx, dx2, gx;
};
__device__ __forceinline__ RsCol rs_colpart(const RsDesc& d, const RsEntry& e, int x) {
  RsCol c;
  const int ox = (x - e.x0) & 127;
  c.dx = fmaf((float)ox, d.hx, e.bx);
  c.dx2 = c.dx * c.dx;
  c.gx = __builtin_amdgcn_exp2f(c.dx2 * d.k2);
  return c;
}
__device__ __forceinline__ bool rs_in(const RsDesc& d, const RsCol& c, const RsRow& w) {
  return w.ok && c.dx2 + w.s <= d.r2;
}

__device__ __forceinline__ float rs_wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Adds sum_a sum_m sqrt(Omega) p_m(r - tau_a) dp_{a,m} to this lane's 16 values of row y (x = t + 8k),
// atoms in the order of the band's entry list.  With p_0 = c0 g, p_m = c1 d_m g and g = gx gyz the
// term is gx (w0 + dx w1), w0 = gyz (c0 dp_0 + c1 (dy dp_y + dz dp_z)), w1 = gyz c1 dp_x.
__device__ __forceinline__ void rs_add_regs(float2 (&r)[16], const RsDesc& rd, int z, int w, int y, int t,
                                            const float2* dp, int lane) {
  const int e0 = rd.boff[16 * z + w], e1 = rd.boff[16 * z + w + 1];
  for (int base = e0; base < e1; base += 64) {
    RsLaneEnt le = rs_empty();
    float2 q0 = make_float2(0.f, 0.f), q1 = q0, q2 = q0, q3 = q0;
    if (base + lane < e1) {
      const RsEnt en = rd.bent[base + lane];
      le = rs_load(en);
      const float2* c = dp + 4 * en.atom;
      q0 = c[0];
      q1 = c[1];
      q2 = c[2];
      q3 = c[3];
    }
    const int cnt = min(64, e1 - base);
    for (int k = 0; k < cnt; ++k) {
      const RsEntry e = rs_entry(le, k);
      const RsRow rw = rs_row(rd, e, y);
      // dp holds (c0 D P_0, c1 D P_x, c1 D P_y, c1 D P_z)
      const float ax = fmaf(e.dz, rs_lane(q3.x, k), rs_lane(q0.x, k));
      const float ay = fmaf(e.dz, rs_lane(q3.y, k), rs_lane(q0.y, k));
      const float w0x = rw.gyz * fmaf(rw.dy, rs_lane(q2.x, k), ax);
      const float w0y = rw.gyz * fmaf(rw.dy, rs_lane(q2.y, k), ay);
      const float w1x = rw.gyz * rs_lane(q1.x, k), w1y = rw.gyz * rs_lane(q1.y, k);
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        if (e.mask & (1u << kk)) {
          const RsCol cc = rs_colpart(rd, e, t + 8 * kk);
          const float gx = rs_in(rd, cc, rw) ? cc.gx : 0.f;
          r[kk].x += gx * fmaf(cc.dx, w1x, w0x);
          r[kk].y += gx * fmaf(cc.dx, w1y, w0y);
        }
      }
    }
  }
}

// ---- 128 x 128 FP32 planes with wave-local lines ---------------------------------------------
// The same transform as k_plane_n (inverse along y on the active columns, inverse along x, * V,
// forward along x, forward along y on the active columns), arranged so that the 8 threads of a
// line sit in one wave: the exchange between the two stages of a line is ordered by the wave
// itself and needs no workgroup barrier, and the plane needs no zero fill, scatter or gather:
//   y passes read their input straight from the sticks (zeros off the stick's n2 range) and the
//   forward one writes its stick positions straight back;
//   the plane in LDS holds only the active columns xa = n1 + n1max, at column xa ^ sy(row) of
//   each 128-word row (sy(r) = 8 ((r >> 4 ^ r) & 1));
//   the x pass uses its row as exchange space: stage-1 word (n2, k1) of the inverse at
//   16 k1 + (n2 ^ k1 ^ 8 (y & 1)), word (m1, q2) of the forward at (8 q2 + (m1 ^ (q2 & 7))) ^ 8 (y & 1).
// Each swizzle spreads the 64 lanes of a wave (8 lines x 8 threads) over all 16 eight-byte bank
// slots in every access of the three passes.  Three workgroup barriers per plane.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ int p128_col(int row, int xa) { return xa ^ ((((row >> 4) ^ row) & 1) << 3); }

// NL: the real-space projectors' D P term is added to V psi between the x passes (rs_add_regs).
template <bool NL>
__global__ __launch_bounds__(1024) void k_plane128(float2* __restrict__ SB, const float* __restrict__ V,
                                                   const int* __restrict__ colstart, GridDesc g,
                                                   const float2* __restrict__ twg, float scale, RsDesc rd,
                                                   const float2* __restrict__ dp, int nproj) {
  using T = float;
  constexpr int N = 128, A = 8, B = 16, LPW = 8, NW = 16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float2* plane = reinterpret_cast<float2*>(smem_raw);
  float2* tw = plane + N * N;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int l = lane >> 3, t = lane & 7;
  const int z = blockIdx.x, b = blockIdx.y;
  const int n1max = g.n1max, n1a = g.n1a;
  const int yrow = wv * LPW + l;
  for (int i = tid; i < N; i += 1024) tw[i] = twg[i];
  float2* sb = SB + ((long)b * g.n3 + z) * g.nst;
  __syncthreads();
  const float2 zero = mk<T>(0, 0);
  // ---- inverse along y, active columns ----
  for (int grp = wv; grp * LPW < n1a; grp += NW) {
    const int xa = grp * LPW + l;
    const bool act = xa < n1a;
    int cs = 0, m = -1;
    if (act) {
      cs = colstart[xa];
      m = (colstart[xa + 1] - cs - 1) >> 1;
    }
    float2 r1[2][A];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) {
        const int y = B * n1 + t + 8 * i;
        const int n2 = y < N / 2 ? y : y - N;
        r1[i][n1] = (n2 <= m && -n2 <= m) ? sb[cs + n2 + m] : zero;
      }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int n2 = t + 8 * i;
      SmallDft<T, A, +1>::run(r1[i]);
#pragma unroll
      for (int k1 = 1; k1 < A; ++k1) {
        float2 w = tw[(n2 * k1) % N];
        w.y = -w.y;
        r1[i][k1] = cmul<T>(r1[i][k1], w);
      }
      if (act)
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) {
          const int e = B * k1 + n2;
          plane[e * N + p128_col(e, xa)] = r1[i][k1];
        }
    }
    wave_sync();
    float2 r2[B];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
      const int e = B * t + n2;
      r2[n2] = plane[e * N + p128_col(e, xa)];
    }
    SmallDft<T, B, +1>::run(r2);
    wave_sync();
    if (act)
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) {
        const int e = t + A * k2;
        plane[e * N + p128_col(e, xa)] = r2[k2];
      }
  }
  __syncthreads();
  // ---- along x on every row: inverse, * V, forward ----
  {
    // V(r) of this thread's row (x = t + 8 k2), issued before the inverse stages that hide it
    T vr[B];
    {
      const T* vz = V + ((long)z * N + yrow) * N + t;
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) vr[k2] = vz[A * k2];
    }
    const int y = yrow;
    const int sy = (((y >> 4) ^ y) & 1) << 3, py = (y & 1) << 3;
    float2* row = plane + y * N;
    float2 r1[2][A];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) {
        const int x = B * n1 + t + 8 * i;
        const int k = x < N / 2 ? x : x - N;
        r1[i][n1] = (k <= n1max && -k <= n1max) ? row[(k + n1max) ^ sy] : zero;
      }
    wave_sync();
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int n2 = t + 8 * i;
      SmallDft<T, A, +1>::run(r1[i]);
#pragma unroll
      for (int k1 = 1; k1 < A; ++k1) {
        float2 w = tw[(n2 * k1) % N];
        w.y = -w.y;
        r1[i][k1] = cmul<T>(r1[i][k1], w);
      }
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) row[B * k1 + (n2 ^ k1 ^ py)] = r1[i][k1];
    }
    wave_sync();
    float2 r2[B];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) r2[n2] = row[B * t + (n2 ^ t ^ py)];
    SmallDft<T, B, +1>::run(r2);  // r2[k2] = value at x = t + 8 k2
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) r2[k2] = cscale<T>(r2[k2], vr[k2]);
    if constexpr (NL) rs_add_regs(r2, rd, z, wv, y, t, dp + (long)b * nproj, lane);
    SmallDft<T, B, -1>::run(r2);  // over m2, output q2
#pragma unroll
    for (int q2 = 1; q2 < B; ++q2) r2[q2] = cmul<T>(r2[q2], tw[(t * q2) % N]);
    wave_sync();
#pragma unroll
    for (int q2 = 0; q2 < B; ++q2) row[(A * q2 + (t ^ (q2 & 7))) ^ py] = r2[q2];
    wave_sync();
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int q2 = t + 8 * i;
#pragma unroll
      for (int m1 = 0; m1 < A; ++m1) r1[i][m1] = row[(A * q2 + (m1 ^ (q2 & 7))) ^ py];
      SmallDft<T, A, -1>::run(r1[i]);  // r1[i][q1] = F[16 q1 + q2]
    }
    wave_sync();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q1 = 0; q1 < A; ++q1) {
        const int x = B * q1 + t + 8 * i;
        const int k = x < N / 2 ? x : x - N;
        if (k <= n1max && -k <= n1max) row[(k + n1max) ^ sy] = r1[i][q1];
      }
  }
  __syncthreads();
  // ---- forward along y, active columns, into the sticks ----
  for (int grp = wv; grp * LPW < n1a; grp += NW) {
    const int xa = grp * LPW + l;
    const bool act = xa < n1a;
    int cs = 0, m = -1;
    if (act) {
      cs = colstart[xa];
      m = (colstart[xa + 1] - cs - 1) >> 1;
    }
    float2 r1[2][A];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) {
        const int e = B * n1 + t + 8 * i;
        r1[i][n1] = plane[e * N + p128_col(e, xa)];
      }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int n2 = t + 8 * i;
      SmallDft<T, A, -1>::run(r1[i]);
#pragma unroll
      for (int k1 = 1; k1 < A; ++k1) r1[i][k1] = cmul<T>(r1[i][k1], tw[(n2 * k1) % N]);
    }
    wave_sync();
    if (act)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) {
          const int e = B * k1 + t + 8 * i;
          plane[e * N + p128_col(e, xa)] = r1[i][k1];
        }
    wave_sync();
    float2 r2[B];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
      const int e = B * t + n2;
      r2[n2] = plane[e * N + p128_col(e, xa)];
    }
    SmallDft<T, B, -1>::run(r2);  // r2[k2] = value at y = t + 8 k2
    if (act)
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) {
        const int y = t + A * k2;
        const int n2 = y < N / 2 ? y : y - N;
        if (n2 <= m && -n2 <= m) sb[cs + n2 + m] = cscale<T>(r2[k2], scale);
      }
  }
}

namespace p128 {
constexpr int N = 128, A = 8, B = 16, LPW = 8;

__device__ __forceinline__ void yinv_load(const float2* __restrict__ sb, const int* __restrict__ colstart, int n1a,
                                          int grp, int l, int t, float2 (&r)[2][A]) {
  const int xa = grp * LPW + l;
  int cs = 0, m = -1;
  if (xa < n1a) {
    cs = colstart[xa];
    m = (colstart[xa + 1] - cs - 1) >> 1;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) {
      const int y = B * n1 + t + 8 * i;
      const int n2 = y < N / 2 ? y : y - N;
      r[i][n1] = (n2 <= m && -n2 <= m) ? sb[cs + n2 + m] : make_float2(0.f, 0.f);
    }
}

__device__ __forceinline__ void yinv_compute(float2* plane, const float2* tw, int n1a, int grp, int l, int t,
                                             float2 (&r1)[2][A]) {
  const int xa = grp * LPW + l;
  const bool act = xa < n1a;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int n2 = t + 8 * i;
    SmallDft<float, A, +1>::run(r1[i]);
#pragma unroll
    for (int k1 = 1; k1 < A; ++k1) {
      float2 w = tw[(n2 * k1) % N];
      w.y = -w.y;
      r1[i][k1] = cmul<float>(r1[i][k1], w);
    }
    if (act)
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) {
        const int e = B * k1 + n2;
        plane[e * N + p128_col(e, xa)] = r1[i][k1];
      }
  }
  wave_sync();
  float2 r2[B];
#pragma unroll
  for (int n2 = 0; n2 < B; ++n2) {
    const int e = B * t + n2;
    r2[n2] = plane[e * N + p128_col(e, xa)];
  }
  SmallDft<float, B, +1>::run(r2);
  wave_sync();
  if (act)
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) {
      const int e = t + A * k2;
      plane[e * N + p128_col(e, xa)] = r2[k2];
    }
}
}  // namespace p128

// Charge density on 128 x 128 FP32 planes, fused: a workgroup takes one z plane and a group of the
// batch's bands, runs the inverse y pass (as k_plane128) and the inverse x pass of each band, and
// adds occ_b |psi_b(r)|^2 to FP64 registers of its rows' grid points, bands in order; the group's
// sum goes out once (part[group][z][y][x]) instead of one |psi|^2 grid per band.  8 waves; each
// wave owns two rows per line (y0 = 8 w + l,
// y1 = 8 (w + 8) + l), so a thread keeps 32 sums.
__device__ __forceinline__ void xinv_row_acc(float2* plane, const float2* tw, int y, int t, int n1max, double occ,
                                             double (&acc)[16]) {
  constexpr int N = 128, A = 8, B = 16;
  const int sy = (((y >> 4) ^ y) & 1) << 3, py = (y & 1) << 3;
  float2* row = plane + y * N;
  float2 r1[2][A];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) {
      const int x = B * n1 + t + 8 * i;
      const int k = x < N / 2 ? x : x - N;
      r1[i][n1] = (k <= n1max && -k <= n1max) ? row[(k + n1max) ^ sy] : make_float2(0.f, 0.f);
    }
  wave_sync();
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int n2 = t + 8 * i;
    SmallDft<float, A, +1>::run(r1[i]);
#pragma unroll
    for (int k1 = 1; k1 < A; ++k1) {
      float2 w = tw[(n2 * k1) % N];
      w.y = -w.y;
      r1[i][k1] = cmul<float>(r1[i][k1], w);
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) row[B * k1 + (n2 ^ k1 ^ py)] = r1[i][k1];
  }
  wave_sync();
  float2 r2[B];
#pragma unroll
  for (int n2 = 0; n2 < B; ++n2) r2[n2] = row[B * t + (n2 ^ t ^ py)];
  SmallDft<float, B, +1>::run(r2);  // r2[k2] = psi at x = t + 8 k2
#pragma unroll
  for (int k2 = 0; k2 < B; ++k2) acc[k2] += occ * ((double)r2[k2].x * r2[k2].x + (double)r2[k2].y * r2[k2].y);
}

__global__ __launch_bounds__(512) void k_density128(const float2* __restrict__ SB, const int* __restrict__ colstart,
                                                    GridDesc g, const float2* __restrict__ twg,
                                                    const double* __restrict__ occ, int nbt, int per,
                                                    double* __restrict__ part, int add) {
  constexpr int N = 128, A = 8, LPW = 8, NW = 8;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float2* plane = reinterpret_cast<float2*>(smem_raw);
  float2* tw = plane + N * N;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int l = lane >> 3, t = lane & 7;
  const int z = blockIdx.x, grp = blockIdx.y;
  const int n1max = g.n1max, n1a = g.n1a;
  const int ngrp = (n1a + LPW - 1) / LPW;
  const int y0 = wv * LPW + l, y1 = (wv + NW) * LPW + l;
  const int b_lo = grp * per, b_hi = min(nbt, b_lo + per);
  for (int i = tid; i < N; i += 64 * NW) tw[i] = twg[i];
  double acc0[16], acc1[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc0[k] = acc1[k] = 0.0;
  __syncthreads();
  for (int b = b_lo; b < b_hi; ++b) {
    const float2* sb = SB + ((long)b * g.n3 + z) * g.nst;
    for (int cg = wv; cg < ngrp; cg += NW) {
      float2 r[2][A];
      p128::yinv_load(sb, colstart, n1a, cg, l, t, r);
      p128::yinv_compute(plane, tw, n1a, cg, l, t, r);
    }
    __syncthreads();
    const double o = occ[b];
    xinv_row_acc(plane, tw, y0, t, n1max, o, acc0);
    __builtin_amdgcn_sched_barrier(0);
    xinv_row_acc(plane, tw, y1, t, n1max, o, acc1);
    __syncthreads();
  }
  double* pz = part + ((long)grp * g.n3 + z) * N * N;
#pragma unroll
  for (int k2 = 0; k2 < 16; ++k2) {
    double* q0 = pz + (long)y0 * N + t + A * k2;
    double* q1 = pz + (long)y1 * N + t + A * k2;
    *q0 = add ? *q0 + acc0[k2] : acc0[k2];
    *q1 = add ? *q1 + acc1[k2] : acc1[k2];
  }
}

// rho[r] = (first ? 0 : rho[r]) + sum over groups of part[group][r], groups in order
__global__ void k_density_groups(const double* __restrict__ part, int ngroups, long nr, double* __restrict__ rho,
                                 int first) {
  PW_GRID_STRIDE(r, nr) {
    double s = first ? 0.0 : rho[r];
    for (int q = 0; q < ngroups; ++q) s += part[(long)q * nr + r];
    rho[r] = s;
  }
}

bool density128_supported(const GridDesc& g, int real_bytes) {
  return real_bytes == 4 && g.n1 == 128 && g.n2 == 128 && g.n1a <= 128;
}

hipError_t launch_density128(const float2* SB, const int* colstart, const GridDesc& g, const float2* tw,
                             const double* occ, int nbt, int ngroups, double* part, double* rho, bool first,
                             hipStream_t s) {
  if (nbt <= 0) return hipSuccess;
  const size_t lds = (size_t)(128 * 128 + 128) * sizeof(float2);
  if (!part || ngroups <= 1) {
    // one group per plane: its sum goes straight into rho
    hipLaunchKernelGGL(k_density128, dim3(g.n3, 1), dim3(512), lds, s, SB, colstart, g, tw, occ, nbt, nbt, rho,
                       first ? 0 : 1);
    return hipGetLastError();
  }
  if (ngroups > nbt) ngroups = nbt;
  const int per = (nbt + ngroups - 1) / ngroups;
  ngroups = (nbt + per - 1) / per;
  hipLaunchKernelGGL(k_density128, dim3(g.n3, ngroups), dim3(512), lds, s, SB, colstart, g, tw, occ, nbt, per, part,
                     0);
  const long nr = 128L * 128 * g.n3;
  hipLaunchKernelGGL(k_density_groups, dim3(stride_blocks(nr)), dim3(256), 0, s, part, ngroups, nr, rho,
                     first ? 1 : 0);
  return hipGetLastError();
}

// Inverse x pass of row y (as in xinv_row_acc); the row then holds psi in natural x order.
__device__ __forceinline__ void xinv_row_store(float2* plane, const float2* tw, int y, int t, int n1max) {
  constexpr int N = 128, A = 8, B = 16;
  const int sy = (((y >> 4) ^ y) & 1) << 3, py = (y & 1) << 3;
  float2* row = plane + y * N;
  float2 r1[2][A];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) {
      const int x = B * n1 + t + 8 * i;
      const int k = x < N / 2 ? x : x - N;
      r1[i][n1] = (k <= n1max && -k <= n1max) ? row[(k + n1max) ^ sy] : make_float2(0.f, 0.f);
    }
  wave_sync();
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int n2 = t + 8 * i;
    SmallDft<float, A, +1>::run(r1[i]);
#pragma unroll
    for (int k1 = 1; k1 < A; ++k1) {
      float2 w = tw[(n2 * k1) % N];
      w.y = -w.y;
      r1[i][k1] = cmul<float>(r1[i][k1], w);
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) row[B * k1 + (n2 ^ k1 ^ py)] = r1[i][k1];
  }
  wave_sync();
  float2 r2[B];
#pragma unroll
  for (int n2 = 0; n2 < B; ++n2) r2[n2] = row[B * t + (n2 ^ t ^ py)];
  SmallDft<float, B, +1>::run(r2);  // r2[k2] = psi at x = t + 8 k2
  wave_sync();
  // natural x order (no swizzle): the projection loop then addresses a point as y * 128 + x
#pragma unroll
  for (int k2 = 0; k2 < B; ++k2) row[t + A * k2] = r2[k2];
}

// log2 of the lanes per row of an entry: 16, 32 or 64 columns at a time (64 / lx rows per step).
__device__ __forceinline__ int rs_lxs(int nx) { return nx <= 16 ? 4 : (nx <= 32 ? 5 : 6); }

// Inverse pass with the projections: a workgroup takes plane z of band b, transforms it inside LDS
// (inverse y on the active columns, inverse x on every row), then each wave takes entries of the
// plane (one atom each), sums g psi, g dx psi and g dy psi over the entry's points with its 64
// lanes (p_z = c1 dz g needs no sum of its own) and writes the four projector sums, reduced
// across the wave in a fixed order, to part[(b nent + e) 4 + m].
__global__ __launch_bounds__(1024) void k_rs_proj128(const float2* __restrict__ SB, const int* __restrict__ colstart,
                                                     GridDesc g, const float2* __restrict__ twg, RsDesc rd,
                                                     float2* __restrict__ part) {
  constexpr int N = 128, LPW = 8, NW = 16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float2* plane = reinterpret_cast<float2*>(smem_raw);
  float2* tw = plane + N * N;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int l = lane >> 3, t = lane & 7;
  const int z = blockIdx.x, b = blockIdx.y;
  const int e0 = rd.zoff[z], e1 = rd.zoff[z + 1];
  if (e0 == e1) return;  // no atom within reach of this plane (uniform over the workgroup)
  const int n1a = g.n1a;
  const int ngrp = (n1a + LPW - 1) / LPW;
  for (int i = tid; i < N; i += 1024) tw[i] = twg[i];
  const float2* sb = SB + ((long)b * g.n3 + z) * g.nst;
  __syncthreads();
  for (int cg = wv; cg < ngrp; cg += NW) {
    float2 r[2][8];
    p128::yinv_load(sb, colstart, n1a, cg, l, t, r);
    p128::yinv_compute(plane, tw, n1a, cg, l, t, r);
  }
  __syncthreads();
  xinv_row_store(plane, tw, wv * LPW + l, t, g.n1max);
  __syncthreads();
  float2* pb = part + (long)b * rd.nent * 4;
  // this wave's entries e0 + wv + 16 k, their data loaded one entry per lane
  for (int base = e0 + wv; base < e1; base += NW * 64) {
    RsLaneEnt le = rs_empty();
    if (base + NW * lane < e1) le = rs_load(rd.zent[base + NW * lane]);
    const int cnt = min(64, (e1 - base + NW - 1) / NW);
    for (int k = 0; k < cnt; ++k) {
      const int e = base + NW * k;
      const RsEntry en = rs_entry(le, k);
      float s0x = 0.f, s0y = 0.f, sxx = 0.f, sxy = 0.f, syx = 0.f, syy = 0.f;
      const int lxs = rs_lxs(en.nx), lx = 1 << lxs, rps = 64 >> lxs;
      const int lr = lane >> lxs, lc = lane & (lx - 1);
      if (en.nx > 16 && en.nx <= 32) {
        // 16 lanes per row, each with two columns 16 apart, four rows per step: one row factor
        // serves two points
        const int lr4 = lane >> 4, lc4 = lane & 15;
        const int xa = (en.x0 + lc4) & (N - 1), xb = (en.x0 + lc4 + 16) & (N - 1);
        const RsCol ca = rs_colpart(rd, en, xa), cb = rs_colpart(rd, en, xb);
        const bool okb = lc4 + 16 < en.nx;  // the first column is always in the range
        for (int q = lr4; q < en.ny; q += 4) {
          const int y = (en.y0 + q) & (N - 1);
          const RsRow rw = rs_row(rd, en, y);
          const float ga = rs_in(rd, ca, rw) ? ca.gx * rw.gyz : 0.f;
          const float gb = (okb && rs_in(rd, cb, rw)) ? cb.gx * rw.gyz : 0.f;
          const float2 va = plane[y * N + xa], vb = plane[y * N + xb];
          const float gxa = ga * ca.dx, gxb = gb * cb.dx;
          s0x = fmaf(ga, va.x, fmaf(gb, vb.x, s0x));
          s0y = fmaf(ga, va.y, fmaf(gb, vb.y, s0y));
          sxx = fmaf(gxa, va.x, fmaf(gxb, vb.x, sxx));
          sxy = fmaf(gxa, va.y, fmaf(gxb, vb.y, sxy));
          // sum of g psi over the row's two points, times dy for p_y
          const float tx = fmaf(ga, va.x, gb * vb.x), ty = fmaf(ga, va.y, gb * vb.y);
          syx = fmaf(rw.dy, tx, syx);
          syy = fmaf(rw.dy, ty, syy);
        }
      } else {
        for (int xc = 0; xc < en.nx; xc += lx) {
          const int x = (en.x0 + xc + lc) & (N - 1);
          const RsCol cc = rs_colpart(rd, en, x);
          const bool colok = xc + lc < en.nx;  // lanes past the range would alias its first columns
          for (int q = lr; q < en.ny; q += rps) {
            const int y = (en.y0 + q) & (N - 1);
            const RsRow rw = rs_row(rd, en, y);
            const float gg = (colok && rs_in(rd, cc, rw)) ? cc.gx * rw.gyz : 0.f;
            const float2 v = plane[y * N + x];
            const float gxv = gg * cc.dx, gyv = gg * rw.dy;
            s0x = fmaf(gg, v.x, s0x);
            s0y = fmaf(gg, v.y, s0y);
            sxx = fmaf(gxv, v.x, sxx);
            sxy = fmaf(gxv, v.y, sxy);
            syx = fmaf(gyv, v.x, syx);
            syy = fmaf(gyv, v.y, syy);
          }
        }
      }
      s0x = rs_wave_sum(s0x);
      s0y = rs_wave_sum(s0y);
      sxx = rs_wave_sum(sxx);
      sxy = rs_wave_sum(sxy);
      syx = rs_wave_sum(syx);
      syy = rs_wave_sum(syy);
      if (lane == 0) {
        const float c0 = rd.c0, c1 = rd.c1, c1z = rd.c1 * en.dz;
        float4* o = reinterpret_cast<float4*>(pb + (long)e * 4);
        o[0] = make_float4(c0 * s0x, c0 * s0y, c1 * sxx, c1 * sxy);
        o[1] = make_float4(c1 * syx, c1 * syy, c1z * s0x, c1z * s0y);
      }
    }
  }
}

// dp[b nproj + 4a + m] = c_m dscale[m] inv_nr sum over atom a's entries (plane order) of part, in FP64
// (c_0 = c0, c_m = c1: the prefactor the addition would otherwise apply per point).
__global__ void k_rs_reduce(const float2* __restrict__ part, RsDesc rd, int nbt, const double* __restrict__ dscale,
                            double inv_nr, float2* __restrict__ dp, int nproj) {
  PW_GRID_STRIDE(idx, (long)nbt * rd.natoms) {
    const int j = (int)(idx / rd.natoms), a = (int)(idx - (long)j * rd.natoms);
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = rd.aoff[a]; k < rd.aoff[a + 1]; ++k) {
      const float4* q = reinterpret_cast<const float4*>(part + ((long)j * rd.nent + rd.aent[k]) * 4);
      const float4 u = q[0], v = q[1];
      s[0] += u.x;
      s[1] += u.y;
      s[2] += u.z;
      s[3] += u.w;
      s[4] += v.x;
      s[5] += v.y;
      s[6] += v.z;
      s[7] += v.w;
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      // D P times the projector prefactor, as the addition uses it
      const double f = dscale[m] * inv_nr * (m == 0 ? (double)rd.c0 : (double)rd.c1);
      dp[(long)j * nproj + 4 * a + m] = make_float2((float)(s[2 * m] * f), (float)(s[2 * m + 1] * f));
    }
  }
}

hipError_t launch_rs_proj128(const float2* SB, const int* colstart, const GridDesc& g, const float2* tw,
                             const RsDesc& rd, int nbatch, float2* part, hipStream_t s) {
  if (nbatch <= 0 || rd.nent <= 0) return hipSuccess;
  if (g.n1 != 128 || g.n2 != 128 || g.n1a > 128) return hipErrorInvalidValue;
  const size_t lds = (size_t)(128 * 128 + 128) * sizeof(float2);
  hipLaunchKernelGGL(k_rs_proj128, dim3(g.n3, nbatch), dim3(1024), lds, s, SB, colstart, g, tw, rd, part);
  return hipGetLastError();
}

hipError_t launch_rs_reduce(const float2* part, const RsDesc& rd, int nbt, const double* dscale, double inv_nr,
                            float2* dp, int nproj, hipStream_t s) {
  if (nbt <= 0 || rd.natoms <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rs_reduce, dim3(stride_blocks((long)nbt * rd.natoms)), dim3(256), 0, s, part, rd, nbt, dscale,
                     inv_nr, dp, nproj);
  return hipGetLastError();
}

hipError_t launch_plane128_nl(float2* SB, const float* V, int nbatch, const int* colstart, const GridDesc& g,
                              const float2* tw, float scale, const RsDesc& rd, const float2* dp, int nproj,
                              hipStream_t s) {
  if (nbatch <= 0) return hipSuccess;
  if (g.n1 != 128 || g.n2 != 128 || g.n1a > 128) return hipErrorInvalidValue;
  const size_t lds = (size_t)(128 * 128 + 128) * sizeof(float2);
  hipLaunchKernelGGL(k_plane128<true>, dim3(g.n3, nbatch), dim3(1024), lds, s, SB, V, colstart, g, tw, scale, rd, dp,
                     nproj);
  return hipGetLastError();
}

// ---- z transforms of the sticks with compile-time N = A B ---------------------------------
// gcd(A, B) threads share a stick; a block takes SPW sticks of one band (at most 256 threads and
// 48 KB of LDS).  Stick element i (0 <= i < len, h = (len - 1) / 2) sits at z = i - h mod N.
template <typename T, int A, int B>
struct StickShape {
  static constexpr int N = A * B, TT = cgcd(A, B);
  static constexpr int SPW0 = 256 / TT, SPWL = (48 * 1024) / (N * (int)sizeof(cplx<T>));
  static constexpr int SPW = SPW0 < SPWL ? SPW0 : SPWL;
  static constexpr int NT = SPW * TT;
  // LDS swizzle.  Lane = TT s + t: a half-wave (32 lanes, the unit in which the LDS serves a
  // 64-lane access of 8-byte elements) holds Gh = 32 / TT sticks, and its TT threads of one
  // stick touch TT positions at once, 1 or B apart, which in a plain [position][stick] layout
  // all fall in the same banks.  Stick s of position p is stored at column s ^ (Gh x(p)),
  // x(p) = (p + p / B) mod X with X = E / Gh slices of Gh sticks per 256-byte bank row (E
  // elements): the TT positions then occupy distinct slices (checked by enumeration for every
  // compiled size).  Used where the shapes allow it (32 % TT == 0, SPW a multiple of E).
  static constexpr int E = 256 / (int)sizeof(cplx<T>);
  static constexpr int Gh = 32 % TT == 0 ? 32 / TT : 0;
  static constexpr bool SWZ = Gh > 0 && E > Gh && SPW % E == 0;
  static constexpr int X = SWZ ? E / Gh : 1;
  __device__ __forceinline__ static int at(int p, int s) {
    if constexpr (SWZ) return p * SPW + (s ^ (Gh * ((p + p / B) % X)));
    else return p * SPW + s;
  }
};

__device__ __forceinline__ int stick_index(int z, int h, int N) {
  return z <= h ? z + h : (z >= N - h ? z - N + h : -1);
}

// sphere -> sticks, inverse FFT along z.  Grid (ceil(nst / SPW), nbatch).  SB layout [band][z][stick].
template <typename T, int A, int B>
__global__ __launch_bounds__(256) void k_sticks_inv_n(const cplx<T>* __restrict__ X, long ldx,
                                                      cplx<T>* __restrict__ SB, const Stick* __restrict__ st,
                                                      GridDesc g, const cplx<T>* __restrict__ twg) {
  using SS = StickShape<T, A, B>;
  constexpr int N = A * B, TT = SS::TT, SPW = SS::SPW, NT = SS::NT, I1 = B / TT, J2 = A / TT;
  __shared__ cplx<T> buf[N * SPW];  // [position][stick]
  __shared__ cplx<T> tw[N];
  const int tid = threadIdx.x, b = blockIdx.y;
  const int s = tid / TT, t = tid % TT;  // stick within the block, thread within the stick
  const int s0 = blockIdx.x * SPW;
  const bool act = s0 + s < g.nst;
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];
  Stick sk{0, 0, 0, 0};
  if (act) sk = st[s0 + s];
  const int h = (sk.len - 1) >> 1;
  const cplx<T>* xs = X + (long)b * ldx + sk.off;
  // stage 1 input straight from the sphere: x[B n1 + n2], n2 = t + TT i
  cplx<T> r1[I1][A];
#pragma unroll
  for (int i = 0; i < I1; ++i)
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) {
      const int e = act ? stick_index(B * n1 + t + TT * i, h, N) : -1;
      r1[i][n1] = e >= 0 ? xs[e] : mk<T>(0, 0);
    }
  __syncthreads();  // twiddles
#pragma unroll
  for (int i = 0; i < I1; ++i) {
    const int n2 = t + TT * i;
    SmallDft<T, A, +1>::run(r1[i]);
#pragma unroll
    for (int k1 = 1; k1 < A; ++k1) {
      cplx<T> w = tw[(n2 * k1) % N];
      w.y = -w.y;
      r1[i][k1] = cmul<T>(r1[i][k1], w);
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) buf[SS::at(k1 * B + n2, s)] = r1[i][k1];
  }
  __syncthreads();
  cplx<T> r2[J2][B];
#pragma unroll
  for (int j = 0; j < J2; ++j) {
    const int k1 = t + TT * j;
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) r2[j][n2] = buf[SS::at(k1 * B + n2, s)];
    SmallDft<T, B, +1>::run(r2[j]);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < J2; ++j) {
    const int k1 = t + TT * j;
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) buf[SS::at(k1 + A * k2, s)] = r2[j][k2];
  }
  __syncthreads();
  // rows of SPW consecutive sticks per z
  const int ns = min(SPW, g.nst - s0);
  cplx<T>* sb = SB + (long)b * N * g.nst + s0;
  for (int i = tid; i < N * SPW; i += NT) {
    const int z = i / SPW, l = i - z * SPW;
    if (l < ns) sb[(long)z * g.nst + l] = buf[SS::at(z, l)];
  }
}

// sticks -> sphere, forward FFT along z.  UPD (FP32): the Chebyshev update of StickUpd is applied to
// each value as it is written (Z is then the updated block).
template <typename T, int A, int B, bool UPD = false>
__global__ __launch_bounds__(256) void k_sticks_fwd_n(const cplx<T>* __restrict__ SB, cplx<T>* __restrict__ Z,
                                                      long ldz, const Stick* __restrict__ st, GridDesc g,
                                                      const cplx<T>* __restrict__ twg, StickUpd u) {
  using SS = StickShape<T, A, B>;
  constexpr int N = A * B, TT = SS::TT, SPW = SS::SPW, NT = SS::NT, I1 = B / TT, J2 = A / TT;
  __shared__ cplx<T> buf[N * SPW];
  __shared__ cplx<T> tw[N];
  const int tid = threadIdx.x, b = blockIdx.y;
  const int s = tid / TT, t = tid % TT;
  const int s0 = blockIdx.x * SPW;
  const int ns = min(SPW, g.nst - s0);
  const bool act = s < ns;
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];
  const cplx<T>* sb = SB + (long)b * N * g.nst + s0;
  for (int i = tid; i < N * SPW; i += NT) {
    const int z = i / SPW, l = i - z * SPW;
    buf[SS::at(z, l)] = l < ns ? sb[(long)z * g.nst + l] : mk<T>(0, 0);
  }
  Stick sk{0, 0, 0, 0};
  if (act) sk = st[s0 + s];
  __syncthreads();
  cplx<T> r1[I1][A];
#pragma unroll
  for (int i = 0; i < I1; ++i)
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) r1[i][n1] = buf[SS::at(B * n1 + t + TT * i, s)];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < I1; ++i) {
    const int n2 = t + TT * i;
    SmallDft<T, A, -1>::run(r1[i]);
#pragma unroll
    for (int k1 = 1; k1 < A; ++k1) r1[i][k1] = cmul<T>(r1[i][k1], tw[(n2 * k1) % N]);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) buf[SS::at(k1 * B + n2, s)] = r1[i][k1];
  }
  __syncthreads();
  if (!act) return;
  const int h = (sk.len - 1) >> 1;
  cplx<T>* zs = Z + (long)b * ldz + sk.off;
#pragma unroll
  for (int j = 0; j < J2; ++j) {
    const int k1 = t + TT * j;
    cplx<T> r2[B];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) r2[n2] = buf[SS::at(k1 * B + n2, s)];
    SmallDft<T, B, -1>::run(r2);
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) {
      const int e = stick_index(k1 + A * k2, h, N);
      if (e >= 0) {
        if constexpr (UPD) {
          const long i = (long)sk.off + e;
          const float2 y = u.Y[(long)b * u.ldy + i];
          const float kc = u.kin[i] - u.c;
          float2 v;
          v.x = u.alpha * (kc * y.x + r2[k2].x);
          v.y = u.alpha * (kc * y.y + r2[k2].y);
          if (u.Yp) {
            const float2 p = u.Yp[(long)b * u.ldp + i];
            v.x -= u.beta * p.x;
            v.y -= u.beta * p.y;
          }
          zs[e] = v;
        } else {
          zs[e] = r2[k2];
        }
      }
    }
  }
}

#define PW_STICK_SIZES(X) \
  X(24, 4, 6) X(27, 3, 9) X(32, 4, 8) X(48, 4, 12) X(54, 6, 9) X(64, 8, 8) X(81, 9, 9) X(96, 8, 12) X(128, 8, 16) \
  X(192, 12, 16)

bool sticks_n_supported(int n3) {
  switch (n3) {
#define PW_CASE(NN, AA, BB) case NN:
    PW_STICK_SIZES(PW_CASE)
#undef PW_CASE
    return true;
    default:
      return false;
  }
}

template <typename T>
hipError_t launch_sticks_inv_n(const cplx<T>* X, long ldx, cplx<T>* SB, int nbatch, const Stick* st,
                               const GridDesc& g, const cplx<T>* tw3, hipStream_t s) {
  switch (g.n3) {
#define PW_CASE(NN, AA, BB)                                                                                   \
  case NN:                                                                                                    \
    hipLaunchKernelGGL((k_sticks_inv_n<T, AA, BB>), dim3(ceil_div(g.nst, StickShape<T, AA, BB>::SPW), nbatch),  \
                       dim3(StickShape<T, AA, BB>::NT), 0, s, X, ldx, SB, st, g, tw3);                         \
    return hipGetLastError();
    PW_STICK_SIZES(PW_CASE)
#undef PW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_sticks_fwd_n(const cplx<T>* SB, cplx<T>* Z, long ldz, int nbatch, const Stick* st,
                               const GridDesc& g, const cplx<T>* tw3, hipStream_t s) {
  switch (g.n3) {
#define PW_CASE(NN, AA, BB)                                                                                   \
  case NN:                                                                                                    \
    hipLaunchKernelGGL((k_sticks_fwd_n<T, AA, BB>), dim3(ceil_div(g.nst, StickShape<T, AA, BB>::SPW), nbatch),  \
                       dim3(StickShape<T, AA, BB>::NT), 0, s, SB, Z, ldz, st, g, tw3, StickUpd{});             \
    return hipGetLastError();
    PW_STICK_SIZES(PW_CASE)
#undef PW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_sticks_fwd_upd(const float2* SB, float2* out, long ldo, int nbatch, const Stick* st,
                                 const GridDesc& g, const float2* tw3, const StickUpd& u, hipStream_t s) {
  switch (g.n3) {
#define PW_CASE(NN, AA, BB)                                                                                     \
  case NN:                                                                                                      \
    hipLaunchKernelGGL((k_sticks_fwd_n<float, AA, BB, true>),                                                   \
                       dim3(ceil_div(g.nst, StickShape<float, AA, BB>::SPW), nbatch),                           \
                       dim3(StickShape<float, AA, BB>::NT), 0, s, SB, out, ldo, st, g, tw3, u);                 \
    return hipGetLastError();
    PW_STICK_SIZES(PW_CASE)
#undef PW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template hipError_t launch_sticks_inv_n<float>(const cplx<float>*, long, cplx<float>*, int, const Stick*,
                                               const GridDesc&, const cplx<float>*, hipStream_t);
template hipError_t launch_sticks_inv_n<double>(const cplx<double>*, long, cplx<double>*, int, const Stick*,
                                                const GridDesc&, const cplx<double>*, hipStream_t);
template hipError_t launch_sticks_fwd_n<float>(const cplx<float>*, cplx<float>*, long, int, const Stick*,
                                               const GridDesc&, const cplx<float>*, hipStream_t);
template hipError_t launch_sticks_fwd_n<double>(const cplx<double>*, cplx<double>*, long, int, const Stick*,
                                                const GridDesc&, const cplx<double>*, hipStream_t);

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
hipError_t launch_plane_n(cplx<T>* SB, const T* V, int nbatch, const Stick* st, const int* colstart,
                          const GridDesc& g, const cplx<T>* tw, T scale, hipStream_t s) {
  if constexpr (std::is_same<T, float>::value) {
    if (g.n1 == 128 && g.n2 == 128 && g.n1a <= 128) {
      const size_t lds = (size_t)(128 * 128 + 128) * sizeof(float2);
      hipLaunchKernelGGL(k_plane128<false>, dim3(g.n3, nbatch), dim3(1024), lds, s, SB, V, colstart, g, tw, scale,
                         RsDesc{}, (const float2*)nullptr, 0);
      return hipGetLastError();
    }
  }
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
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_plane128<false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_plane128<true>), hipFuncAttributeMaxDynamicSharedMemorySize,
                            bytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rs_proj128), hipFuncAttributeMaxDynamicSharedMemorySize,
                            bytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_density128), hipFuncAttributeMaxDynamicSharedMemorySize,
                            bytes);
}

template hipError_t launch_plane_n<float>(cplx<float>*, const float*, int, const Stick*, const int*,
                                          const GridDesc&, const cplx<float>*, float, hipStream_t);
template hipError_t launch_plane_n<double>(cplx<double>*, const double*, int, const Stick*, const int*,
                                           const GridDesc&, const cplx<double>*, double, hipStream_t);

}  // namespace pw
