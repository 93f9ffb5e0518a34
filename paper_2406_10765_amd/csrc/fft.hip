// Batched 3D FFTs of the plane-wave sphere with the local potential applied in
// real space: Z = P_sphere FFT_fwd[ V(r) FFT_inv[ P_sphere^T Y ] ] per band.
//
// The local-potential term of H is a multiplication in real space; the
// wavefunction of one band lives on the sphere |G|^2/2 <= E_cut (Section II-A).
// The transform runs in three stages so that only non-zero data moves:
//   1. sticks:  sphere -> 1D inverse FFT along z for every (n1, n2) stick
//   2. planes:  for every z plane, 2D inverse FFT, multiply by V(r), 2D forward
//               FFT, keep only the stick positions
//   3. sticks:  1D forward FFT along z, gather back onto the sphere
// Every 1D FFT is a Stockham radix-2/3/4 transform held in LDS; twiddles come
// from tables computed in double precision on the host.
//
// Conventions: psi(r_j) = sum_G c_G exp(+i G.r_j) (unnormalised inverse) and
// c_G = (1/N_r) sum_j f(r_j) exp(-i G.r_j); the 1/N_r is applied in stage 2.

#include <cstdlib>

#include "common.hpp"
#include "kernels.hpp"

namespace pw {

// In-register DFT of size R with sign sgn (+1 inverse, -1 forward).
template <typename T, int R>
__device__ __forceinline__ void dft_r(cplx<T>* a, int sgn) {
  if constexpr (R == 2) {
    const cplx<T> t0 = a[0], t1 = a[1];
    a[0] = cadd<T>(t0, t1);
    a[1] = csub<T>(t0, t1);
  } else if constexpr (R == 3) {
    const T h = (T)0.86602540378443864676;  // sqrt(3)/2
    const cplx<T> t1 = cadd<T>(a[1], a[2]);
    const cplx<T> t2 = csub<T>(a[1], a[2]);
    const cplx<T> m = mk<T>(a[0].x - (T)0.5 * t1.x, a[0].y - (T)0.5 * t1.y);
    const cplx<T> r = cmuli<T>(cscale<T>(t2, h), sgn);
    a[0] = cadd<T>(a[0], t1);
    a[1] = cadd<T>(m, r);
    a[2] = csub<T>(m, r);
  } else {
    const cplx<T> s02 = cadd<T>(a[0], a[2]), d02 = csub<T>(a[0], a[2]);
    const cplx<T> s13 = cadd<T>(a[1], a[3]);
    const cplx<T> d13 = cmuli<T>(csub<T>(a[1], a[3]), sgn);
    a[0] = cadd<T>(s02, s13);
    a[2] = csub<T>(s02, s13);
    a[1] = cadd<T>(d02, d13);
    a[3] = csub<T>(d02, d13);
  }
}

// One Stockham pass of radix R over `nlines` lines of length n in LDS.
// Element e of line l is at buf[base(l) + e*es], base(l) = (l < split ? l : l + skip) * ls.
// Pass state: Ls = product of the radices already applied.
// Butterfly j (k = j mod Ls) reads x[j + t n/R], twiddles by w^(t k) with
// w = exp(sgn 2 pi i / (Ls R)), and writes y[(j - k) R + k + u Ls].
// line_fast picks the thread -> (line, j) order so that neighbouring lanes
// touch neighbouring LDS words for both strided and contiguous lines.
template <typename T, int R, int MAXBF>
__device__ __forceinline__ void fft_pass(cplx<T>* buf, int n, int nlines, int split, int skip, int es,
                                         int ls, bool line_fast, int Ls, const cplx<T>* tw, int sgn,
                                         int tid, int nthr) {
  const int nbf = n / R;
  const int total = nbf * nlines;
  const int tws = n / (Ls * R);
  cplx<T> v[MAXBF][R];
  int ob[MAXBF];
#pragma unroll
  for (int q = 0; q < MAXBF; ++q) {
    const int bid = tid + q * nthr;
    if (bid < total) {
      int l, j;
      if (line_fast) {
        l = bid % nlines;
        j = bid / nlines;
      } else {
        l = bid / nbf;
        j = bid - l * nbf;
      }
      const int k = j % Ls;
      const int base = (l < split ? l : l + skip) * ls;
      const cplx<T>* src = buf + base + j * es;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        cplx<T> a = src[t * nbf * es];
        if (t > 0 && k > 0) {
          cplx<T> w = tw[t * k * tws];
          if (sgn > 0) w.y = -w.y;
          a = cmul<T>(a, w);
        }
        v[q][t] = a;
      }
      dft_r<T, R>(v[q], sgn);
      ob[q] = base + ((j - k) * R + k) * es;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXBF; ++q) {
    const int bid = tid + q * nthr;
    if (bid < total) {
#pragma unroll
      for (int u = 0; u < R; ++u) buf[ob[q] + u * Ls * es] = v[q][u];
    }
  }
  __syncthreads();
}

template <typename T, int MAXE>
__device__ void fft_lines(cplx<T>* buf, const FftPlan& p, int nlines, int split, int skip, int es, int ls,
                          bool line_fast, const cplx<T>* tw, int sgn, int tid, int nthr) {
  int Ls = 1;
  for (int i = 0; i < p.nrad; ++i) {
    const int R = p.rad[i];
    if (R == 4)
      fft_pass<T, 4, MAXE / 4>(buf, p.n, nlines, split, skip, es, ls, line_fast, Ls, tw, sgn, tid, nthr);
    else if (R == 2)
      fft_pass<T, 2, MAXE / 2>(buf, p.n, nlines, split, skip, es, ls, line_fast, Ls, tw, sgn, tid, nthr);
    else
      fft_pass<T, 3, MAXE / 3>(buf, p.n, nlines, split, skip, es, ls, line_fast, Ls, tw, sgn, tid, nthr);
    Ls *= R;
  }
}

__device__ __forceinline__ int wrap(int n, int N) { return n < 0 ? n + N : n; }

// ---------------------------------------------------------------------------
// Stage 1: sphere -> sticks, inverse FFT along z.  Grid (ceil(nst/spw), nbatch).
// SB layout: [band][z][stick].
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_sticks_inv(const cplx<T>* __restrict__ X, long ldx, cplx<T>* __restrict__ SB,
                             const Stick* __restrict__ st, GridDesc g, const cplx<T>* __restrict__ tw3,
                             int spw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* tw = buf + spw * g.n3;
  int* soff = reinterpret_cast<int*>(tw + g.n3);
  int* slen = soff + spw;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int b = blockIdx.y;
  const int s0 = blockIdx.x * spw;
  const int ns = min(spw, g.nst - s0);
  const int n3 = g.n3;
  for (int i = tid; i < spw * n3; i += nthr) buf[i] = mk<T>(0, 0);
  for (int i = tid; i < n3; i += nthr) tw[i] = tw3[i];
  for (int i = tid; i < ns; i += nthr) {
    soff[i] = st[s0 + i].off;
    slen[i] = st[s0 + i].len;
  }
  __syncthreads();
  const int g0 = soff[0];
  const int g1 = soff[ns - 1] + slen[ns - 1];
  const cplx<T>* xb = X + (long)b * ldx;
  for (int gi = g0 + tid; gi < g1; gi += nthr) {
    int lo = 0, hi = ns - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (soff[mid] <= gi) lo = mid; else hi = mid - 1;
    }
    const int h = (slen[lo] - 1) >> 1;
    const int z = wrap(gi - soff[lo] - h, n3);
    buf[z * spw + lo] = xb[gi];
  }
  __syncthreads();
  fft_lines<T, 16>(buf, g.p3, spw, spw, 0, spw, 1, true, tw, +1, tid, nthr);
  cplx<T>* sb = SB + (long)b * n3 * g.nst;
  for (int i = tid; i < spw * n3; i += nthr) {
    const int z = i / spw, l = i - z * spw;
    if (l < ns) sb[(long)z * g.nst + s0 + l] = buf[i];
  }
}

// ---------------------------------------------------------------------------
// Stage 3: sticks -> sphere, forward FFT along z.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_sticks_fwd(const cplx<T>* __restrict__ SB, cplx<T>* __restrict__ Z, long ldz,
                             const Stick* __restrict__ st, GridDesc g, const cplx<T>* __restrict__ tw3,
                             int spw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* tw = buf + spw * g.n3;
  int* soff = reinterpret_cast<int*>(tw + g.n3);
  int* slen = soff + spw;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int b = blockIdx.y;
  const int s0 = blockIdx.x * spw;
  const int ns = min(spw, g.nst - s0);
  const int n3 = g.n3;
  const cplx<T>* sb = SB + (long)b * n3 * g.nst;
  for (int i = tid; i < spw * n3; i += nthr) {
    const int z = i / spw, l = i - z * spw;
    buf[i] = l < ns ? sb[(long)z * g.nst + s0 + l] : mk<T>(0, 0);
  }
  for (int i = tid; i < n3; i += nthr) tw[i] = tw3[i];
  for (int i = tid; i < ns; i += nthr) {
    soff[i] = st[s0 + i].off;
    slen[i] = st[s0 + i].len;
  }
  __syncthreads();
  fft_lines<T, 16>(buf, g.p3, spw, spw, 0, spw, 1, true, tw, -1, tid, nthr);
  const int g0 = soff[0];
  const int g1 = soff[ns - 1] + slen[ns - 1];
  cplx<T>* zb = Z + (long)b * ldz;
  for (int gi = g0 + tid; gi < g1; gi += nthr) {
    int lo = 0, hi = ns - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (soff[mid] <= gi) lo = mid; else hi = mid - 1;
    }
    const int h = (slen[lo] - 1) >> 1;
    const int z = wrap(gi - soff[lo] - h, n3);
    zb[gi] = buf[z * spw + lo];
  }
}

// ---------------------------------------------------------------------------
// Stage 2, fused: one workgroup per (z plane, band); the whole N1 x N2 plane
// sits in LDS, layout [y][x].  mode 0: inverse, * V, forward, gather * scale.
// mode 1: inverse only, write the real part to vout[z][y][x] (potential setup).
// mode 2: inverse only, write |psi|^2 to vout[band][z][y][x] (charge density).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(1024) void k_plane(cplx<T>* __restrict__ SB, const T* __restrict__ V, const Stick* __restrict__ st,
                        GridDesc g, const cplx<T>* __restrict__ tw1g, const cplx<T>* __restrict__ tw2g,
                        T scale, int mode, T* __restrict__ vout) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n1 = g.n1, n2 = g.n2, n3 = g.n3;
  const int np = n1 * n2;
  cplx<T>* plane = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* tw1 = plane + np;
  cplx<T>* tw2 = tw1 + n1;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int z = blockIdx.x, b = blockIdx.y;
  for (int i = tid; i < np; i += nthr) plane[i] = mk<T>(0, 0);
  for (int i = tid; i < n1; i += nthr) tw1[i] = tw1g[i];
  for (int i = tid; i < n2; i += nthr) tw2[i] = tw2g[i];
  __syncthreads();
  cplx<T>* sb = SB + ((long)b * n3 + z) * g.nst;
  for (int s = tid; s < g.nst; s += nthr) {
    const Stick t = st[s];
    plane[wrap(t.n2, n2) * n1 + wrap(t.n1, n1)] = sb[s];
  }
  __syncthreads();
  // y lines (columns), only the active x columns n1 in [-n1max, n1max]
  fft_lines<T, 16>(plane, g.p2, g.n1a, g.n1max + 1, n1 - g.n1a, n1, 1, true, tw2, +1, tid, nthr);
  // x lines (rows)
  fft_lines<T, 16>(plane, g.p1, n2, n2, 0, 1, n1, false, tw1, +1, tid, nthr);
  const long zoff = (long)z * np;
  if (mode == 1) {
    for (int i = tid; i < np; i += nthr) vout[zoff + i] = plane[i].x;
    return;
  }
  if (mode == 2) {
    T* vb = vout + (long)b * n3 * np + zoff;
    for (int i = tid; i < np; i += nthr) vb[i] = plane[i].x * plane[i].x + plane[i].y * plane[i].y;
    return;
  }
  for (int i = tid; i < np; i += nthr) plane[i] = cscale<T>(plane[i], V[zoff + i]);
  __syncthreads();
  fft_lines<T, 16>(plane, g.p1, n2, n2, 0, 1, n1, false, tw1, -1, tid, nthr);
  fft_lines<T, 16>(plane, g.p2, g.n1a, g.n1max + 1, n1 - g.n1a, n1, 1, true, tw2, -1, tid, nthr);
  for (int s = tid; s < g.nst; s += nthr) {
    const Stick t = st[s];
    sb[s] = cscale<T>(plane[wrap(t.n2, n2) * n1 + wrap(t.n1, n1)], scale);
  }
}

// ---------------------------------------------------------------------------
// Stage 2, pencil form for planes larger than LDS.  The intermediate G1 holds
// only the active x columns: G1[band][z][y][xa], xa = n1 + n1max.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_ycols_inv(const cplx<T>* __restrict__ SB, cplx<T>* __restrict__ G1,
                            const Stick* __restrict__ st, const int* __restrict__ colstart, GridDesc g,
                            const cplx<T>* __restrict__ tw2g, int cx) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n2 = g.n2, n3 = g.n3;
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);  // [y][c]
  cplx<T>* tw = buf + n2 * cx;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int xa0 = blockIdx.x * cx, z = blockIdx.y, b = blockIdx.z;
  const int nc = min(cx, g.n1a - xa0);
  for (int i = tid; i < n2 * cx; i += nthr) buf[i] = mk<T>(0, 0);
  for (int i = tid; i < n2; i += nthr) tw[i] = tw2g[i];
  __syncthreads();
  const cplx<T>* sb = SB + ((long)b * n3 + z) * g.nst;
  const int sbeg = colstart[xa0], send = colstart[xa0 + nc];
  for (int s = sbeg + tid; s < send; s += nthr) {
    const Stick t = st[s];
    buf[wrap(t.n2, n2) * cx + (t.n1 + g.n1max - xa0)] = sb[s];
  }
  __syncthreads();
  fft_lines<T, 16>(buf, g.p2, cx, cx, 0, cx, 1, true, tw, +1, tid, nthr);
  cplx<T>* out = G1 + ((long)b * n3 + z) * n2 * g.n1a;
  for (int i = tid; i < n2 * cx; i += nthr) {
    const int y = i / cx, c = i - y * cx;
    if (c < nc) out[(long)y * g.n1a + xa0 + c] = buf[i];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_xrows(cplx<T>* __restrict__ G1, const T* __restrict__ V, GridDesc g,
                        const cplx<T>* __restrict__ tw1g, int cy, int mode, T* __restrict__ vout) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n1 = g.n1, n2 = g.n2, n3 = g.n3;
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);  // [r][x]
  cplx<T>* tw = buf + cy * n1;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int y0 = blockIdx.x * cy, z = blockIdx.y, b = blockIdx.z;
  const int ny = min(cy, n2 - y0);
  for (int i = tid; i < cy * n1; i += nthr) buf[i] = mk<T>(0, 0);
  for (int i = tid; i < n1; i += nthr) tw[i] = tw1g[i];
  __syncthreads();
  cplx<T>* gb = G1 + (((long)b * n3 + z) * n2 + y0) * g.n1a;
  for (int i = tid; i < ny * g.n1a; i += nthr) {
    const int r = i / g.n1a, xa = i - r * g.n1a;
    buf[r * n1 + wrap(xa - g.n1max, n1)] = gb[i];
  }
  __syncthreads();
  fft_lines<T, 16>(buf, g.p1, cy, cy, 0, 1, n1, false, tw, +1, tid, nthr);
  const long voff = ((long)z * n2 + y0) * n1;
  if (mode == 1) {
    for (int i = tid; i < ny * n1; i += nthr) vout[voff + i] = buf[i].x;
    return;
  }
  if (mode == 2) {
    T* vb = vout + (long)b * n3 * n2 * n1 + voff;
    for (int i = tid; i < ny * n1; i += nthr) vb[i] = buf[i].x * buf[i].x + buf[i].y * buf[i].y;
    return;
  }
  for (int i = tid; i < ny * n1; i += nthr) buf[i] = cscale<T>(buf[i], V[voff + i]);
  __syncthreads();
  fft_lines<T, 16>(buf, g.p1, cy, cy, 0, 1, n1, false, tw, -1, tid, nthr);
  for (int i = tid; i < ny * g.n1a; i += nthr) {
    const int r = i / g.n1a, xa = i - r * g.n1a;
    gb[i] = buf[r * n1 + wrap(xa - g.n1max, n1)];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_ycols_fwd(cplx<T>* __restrict__ SB, const cplx<T>* __restrict__ G1,
                            const Stick* __restrict__ st, const int* __restrict__ colstart, GridDesc g,
                            const cplx<T>* __restrict__ tw2g, int cx, T scale) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n2 = g.n2, n3 = g.n3;
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* tw = buf + n2 * cx;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int xa0 = blockIdx.x * cx, z = blockIdx.y, b = blockIdx.z;
  const int nc = min(cx, g.n1a - xa0);
  const cplx<T>* in = G1 + ((long)b * n3 + z) * n2 * g.n1a;
  for (int i = tid; i < n2 * cx; i += nthr) {
    const int y = i / cx, c = i - y * cx;
    buf[i] = c < nc ? in[(long)y * g.n1a + xa0 + c] : mk<T>(0, 0);
  }
  for (int i = tid; i < n2; i += nthr) tw[i] = tw2g[i];
  __syncthreads();
  fft_lines<T, 16>(buf, g.p2, cx, cx, 0, cx, 1, true, tw, -1, tid, nthr);
  cplx<T>* sb = SB + ((long)b * n3 + z) * g.nst;
  const int sbeg = colstart[xa0], send = colstart[xa0 + nc];
  for (int s = sbeg + tid; s < send; s += nthr) {
    const Stick t = st[s];
    sb[s] = cscale<T>(buf[wrap(t.n2, n2) * cx + (t.n1 + g.n1max - xa0)], scale);
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

// Largest threads-per-line budget check: every pass must fit MAXE=16 registers.
static bool fits_maxe(const FftPlan& p, int nlines, int nthr) {
  for (int i = 0; i < p.nrad; ++i) {
    const int R = p.rad[i];
    const long total = (long)(p.n / R) * nlines;
    const long per = (total + nthr - 1) / nthr;
    if (per > 16 / R) return false;
  }
  return true;
}

int fft_pick_threads(const FftPlan& p, int nlines, int min_thr) {
  for (int t = min_thr; t <= 1024; t += 64)
    if (fits_maxe(p, nlines, t)) return t;
  return -1;
}

template <typename T>
hipError_t launch_sticks_inv(const cplx<T>* X, long ldx, cplx<T>* SB, int nbatch, const Stick* st,
                             const GridDesc& g, const cplx<T>* tw3, const FftLaunch& L, hipStream_t s) {
  if (L.sized_sticks) return launch_sticks_inv_n<T>(X, ldx, SB, nbatch, st, g, tw3, s);
  const size_t lds = (size_t)L.spw * g.n3 * sizeof(cplx<T>) + g.n3 * sizeof(cplx<T>) + 2 * L.spw * sizeof(int);
  dim3 grid(ceil_div(g.nst, L.spw), nbatch);
  hipLaunchKernelGGL(k_sticks_inv<T>, grid, dim3(L.stick_thr), lds, s, X, ldx, SB, st, g, tw3, L.spw);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sticks_fwd(const cplx<T>* SB, cplx<T>* Z, long ldz, int nbatch, const Stick* st,
                             const GridDesc& g, const cplx<T>* tw3, const FftLaunch& L, hipStream_t s) {
  if (L.sized_sticks) return launch_sticks_fwd_n<T>(SB, Z, ldz, nbatch, st, g, tw3, s);
  const size_t lds = (size_t)L.spw * g.n3 * sizeof(cplx<T>) + g.n3 * sizeof(cplx<T>) + 2 * L.spw * sizeof(int);
  dim3 grid(ceil_div(g.nst, L.spw), nbatch);
  hipLaunchKernelGGL(k_sticks_fwd<T>, grid, dim3(L.stick_thr), lds, s, SB, Z, ldz, st, g, tw3, L.spw);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_plane_fused(cplx<T>* SB, const T* V, int nbatch, const Stick* st, const GridDesc& g,
                              const cplx<T>* tw1, const cplx<T>* tw2, T scale, int mode, T* vout, const FftLaunch& L,
                              hipStream_t s) {
  const size_t lds = (size_t)(g.n1 * g.n2 + g.n1 + g.n2) * sizeof(cplx<T>);
  dim3 grid(g.n3, nbatch);
  hipLaunchKernelGGL(k_plane<T>, grid, dim3(L.plane_thr), lds, s, SB, V, st, g, tw1, tw2, scale, mode, vout);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pencil_yinv(const cplx<T>* SB, cplx<T>* G1, int nbatch, const Stick* st, const int* colstart,
                              const GridDesc& g, const cplx<T>* tw2, const FftLaunch& L, hipStream_t s) {
  const size_t lds = (size_t)(g.n2 * L.cx + g.n2) * sizeof(cplx<T>);
  dim3 grid(ceil_div(g.n1a, L.cx), g.n3, nbatch);
  hipLaunchKernelGGL(k_ycols_inv<T>, grid, dim3(L.col_thr), lds, s, SB, G1, st, colstart, g, tw2, L.cx);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pencil_x(cplx<T>* G1, const T* V, int nbatch, const GridDesc& g, const cplx<T>* tw1, int mode,
                           T* vout, const FftLaunch& L, hipStream_t s) {
  const size_t lds = (size_t)(L.cy * g.n1 + g.n1) * sizeof(cplx<T>);
  dim3 grid(ceil_div(g.n2, L.cy), g.n3, nbatch);
  hipLaunchKernelGGL(k_xrows<T>, grid, dim3(L.row_thr), lds, s, G1, V, g, tw1, L.cy, mode, vout);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pencil_yfwd(cplx<T>* SB, const cplx<T>* G1, int nbatch, const Stick* st, const int* colstart,
                              const GridDesc& g, const cplx<T>* tw2, T scale, const FftLaunch& L, hipStream_t s) {
  const size_t lds = (size_t)(g.n2 * L.cx + g.n2) * sizeof(cplx<T>);
  dim3 grid(ceil_div(g.n1a, L.cx), g.n3, nbatch);
  hipLaunchKernelGGL(k_ycols_fwd<T>, grid, dim3(L.col_thr), lds, s, SB, G1, st, colstart, g, tw2, L.cx, scale);
  return hipGetLastError();
}

bool fft_plan_launch(const GridDesc& g, int real_bytes, size_t max_lds, FftLaunch* L) {
  const int cb = 2 * real_bytes;
  // sticks: spw lines of n3, at most 48 KB of LDS and 16 elements per thread at 256 threads
  int spw = 64;
  while (spw > 4 && ((size_t)spw * g.n3 * cb > 48 * 1024 || (long)spw * g.n3 > 256 * 16)) spw /= 2;
  L->spw = spw;
  L->stick_thr = fits_maxe(g.p3, spw, 256) ? 256 : -1;
  if (L->stick_thr < 0) return false;
  // fused plane if it fits in LDS
  const size_t plane_lds = (size_t)(g.n1 * g.n2 + g.n1 + g.n2) * cb;
  L->fused = false;
  if (plane_lds <= max_lds) {
    int t1 = fft_pick_threads(g.p2, g.n1a, 64);
    int t2 = fft_pick_threads(g.p1, g.n2, 64);
    int t = t1 > t2 ? t1 : t2;
    const int want = ((g.n1 * g.n2 / 4 + 63) / 64) * 64;
    if (t > 0 && want > t) t = want > 1024 ? 1024 : want;
    if (t > 0 && fits_maxe(g.p2, g.n1a, t) && fits_maxe(g.p1, g.n2, t)) {
      L->fused = true;
      L->plane_thr = t;
    }
  }
  L->sized = L->fused && plane_n_supported(g.n1, g.n2, real_bytes, max_lds) && std::getenv("PW_GENERIC_PLANE") == nullptr;
  L->sized_sticks = sticks_n_supported(g.n3) && std::getenv("PW_GENERIC_STICKS") == nullptr;
  L->cx = 16;
  while (L->cx > 1 && L->cx * g.n2 > 4096) L->cx /= 2;
  L->cy = 16;
  while (L->cy > 1 && L->cy * g.n1 > 4096) L->cy /= 2;
  L->col_thr = fits_maxe(g.p2, L->cx, 256) ? 256 : -1;
  L->row_thr = fits_maxe(g.p1, L->cy, 256) ? 256 : -1;
  if (!L->fused && (L->col_thr < 0 || L->row_thr < 0)) return false;
  return true;
}

void pw_allow_large_lds() {
  const int bytes = (int)(160 * 1024);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_plane<float>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_plane<double>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

#define PW_INST_FFT(T)                                                                                         \
  template hipError_t launch_sticks_inv<T>(const cplx<T>*, long, cplx<T>*, int, const Stick*, const GridDesc&, \
                                           const cplx<T>*, const FftLaunch&, hipStream_t);                      \
  template hipError_t launch_sticks_fwd<T>(const cplx<T>*, cplx<T>*, long, int, const Stick*, const GridDesc&, \
                                           const cplx<T>*, const FftLaunch&, hipStream_t);                      \
  template hipError_t launch_plane_fused<T>(cplx<T>*, const T*, int, const Stick*, const GridDesc&,           \
                                            const cplx<T>*, const cplx<T>*, T, int, T*, const FftLaunch&,      \
                                            hipStream_t);                                                      \
  template hipError_t launch_pencil_yinv<T>(const cplx<T>*, cplx<T>*, int, const Stick*, const int*,          \
                                            const GridDesc&, const cplx<T>*, const FftLaunch&, hipStream_t);   \
  template hipError_t launch_pencil_x<T>(cplx<T>*, const T*, int, const GridDesc&, const cplx<T>*, int, T*,   \
                                         const FftLaunch&, hipStream_t);                                       \
  template hipError_t launch_pencil_yfwd<T>(cplx<T>*, const cplx<T>*, int, const Stick*, const int*,          \
                                            const GridDesc&, const cplx<T>*, T, const FftLaunch&, hipStream_t);
PW_INST_FFT(float)
PW_INST_FFT(double)

}  // namespace pw
