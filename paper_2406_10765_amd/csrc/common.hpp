// Shared types and small device helpers for the plane-wave eigensolver library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace pw {

// Complex number types: interleaved (re, im) pairs.
template <typename T> struct cvec;
template <> struct cvec<float> { using type = float2; };
template <> struct cvec<double> { using type = double2; };
template <typename T> using cplx = typename cvec<T>::type;

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T x, T y) {
  cplx<T> r;
  r.x = x;
  r.y = y;
  return r;
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// multiply by +i (s = +1) or -i (s = -1)
template <typename T>
__device__ __forceinline__ cplx<T> cmuli(cplx<T> a, int s) {
  return s > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}

// One stick of the G sphere: all plane waves with Miller (n1, n2, n3), n3 in [-h, h],
// stored contiguously from `off` (len = 2h + 1).
struct Stick {
  int off;
  int len;
  int n1;
  int n2;
};

// Real-space projectors: one (atom, z plane) pair, or (atom, z plane, 8-row band) triple: the plane's
// z displacement from the atom (bohr); unwrapped grid ranges that hold every point of the disc the
// ball cuts from the plane: columns x0 .. x0+nx-1, rows y0 .. y0+ny-1; the displacements of the
// first column and row from the atom, bx = x0 hx - x_a and by = y0 hy - y_a (bohr); and the mask of
// the 8-column blocks (columns 8k .. 8k+7 of the plane) that the columns meet.
struct RsEnt {
  int atom;
  float dz, bx, by;
  short x0, nx, y0, ny;
  unsigned short mask, pad;
};

// Tables of the real-space projectors on a 128 x 128 x n3 grid (PW_FLAG_RSPACE_KB).
struct RsDesc {
  const float4* atoms;  // per atom: x, y, z (bohr, inside the cell), w unused
  const int* zoff;      // entries of plane z: zent[zoff[z] .. zoff[z + 1]); entry index = partial slot
  const RsEnt* zent;
  const int* boff;      // entries of plane z and row band w (rows 8w .. 8w+7): bent[boff[16z+w] ..)
  const RsEnt* bent;
  const int* aoff;      // the zent indices of atom a, in plane order: aent[aoff[a] .. aoff[a + 1])
  const int* aent;
  int nent, natoms;     // nent: zent entries
  float hx, hy;         // grid steps along x and y (bohr)
  float r2;             // truncation radius squared (bohr^2)
  float k2;             // -log2(e) / (2 sigma^2): e^{-d^2/(2 sigma^2)} = 2^{k2 d^2}
  float c0, c1;         // sqrt(Omega) times the unit-norm prefactors of p_0 and p_m
};

// Chebyshev update fused into the forward stick pass: out = alpha ((kin - c) Y + z) - beta Yp, z the
// transform written at a sphere position (Yp may be null).
struct StickUpd {
  const float* kin;
  const float2* Y;
  long ldy;
  const float2* Yp;
  long ldp;
  float alpha, c, beta;
};

// Radix plan of one 1D FFT length (radices in order of application).
struct FftPlan {
  int n;
  int nrad;
  int rad[10];
};

// Geometry of the transform: the plane-wave sphere, its sticks and the grid.
struct GridDesc {
  int n1, n2, n3;     // grid
  int nst;            // number of sticks
  int npw;            // plane waves
  int n1max;          // max |n1| over sticks; active x columns xa = n1 + n1max in [0, n1a)
  int n1a;            // 2 * n1max + 1
  FftPlan p1, p2, p3; // radix plans for the three axes
};

inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// Blocks for a grid-stride loop over n elements with 256-thread blocks.  A dispatch counts
// work-items per grid dimension in 32 bits, so element-wise kernels over blocks of billions of
// entries loop instead of launching one work-item per element.
inline int stride_blocks(long long n) {
  const long long b = (n + 255) / 256;
  return (int)(b < (1 << 20) ? (b > 0 ? b : 1) : (1 << 20));
}
#define PW_GRID_STRIDE(idx, total) \
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < (total); idx += (long)gridDim.x * blockDim.x)

}  // namespace pw
