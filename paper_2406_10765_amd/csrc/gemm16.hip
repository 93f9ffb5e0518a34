// Split-precision complex GEMMs on the bf16 matrix cores (MFMA 16x16x32 bf16, fp32 accumulation).
//
// Every fp32 operand x is split into hi = bf16(x) and lo = bf16(x - hi) (round to nearest even;
// x - hi is exact in fp32).  A real product is formed as hi*hi' + hi*lo' + lo*hi' (three terms),
// which drops lo*lo' and the residual of the two-term split (about 2^-18 relative each), or with
// lo*lo' added (four terms).  The four-term form is used for the Gram / projected matrices: in a
// self product such as sum |y|^2 the dropped lo*lo' has one sign and would bias the sums, while
// the split residual left by the four-term form has no preferred sign.
//
// Complex products are written as real products over the interleaved (re, im) dimension k':
//   cn, C = A^H B:  Re C = sum_k' A'_k' B'_k',   Im C = sum_k' A'_k' B''_k'
//                   A' = (ar, ai), B' = (br, bi), B'' = (bi, -br)  per complex k
//   nn, C = A B:    Re C = sum_k' A'_k' Br_k',   Im C = sum_k' A'_k' Bi_k'
//                   A' = (ar, ai), Br = (br, -bi), Bi = (bi, br)
// so the raw interleaved columns of the big operands are the MFMA operands; B'' comes from B' by
// swapping the 16-bit halves of each word and flipping one sign bit, in registers.
//
// MFMA 16x16x32 bf16: lane l supplies 8 consecutive k' values of row/column l % 16 from k' slot
// l / 16; the accumulator layout is that of the fp32 16x16x4 instruction (C[4 (l/16) + r][l % 16]).
// LDS planes are stored [slot][row][8] (rows swizzled within groups of 16) so the 16 lanes of a
// slot read 256 contiguous bytes.

#include <type_traits>

#include "bf16split.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace pw {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f16 __attribute__((ext_vector_type(4)));

constexpr int hBK = 16;  // complex K per tile = 32 real k' = one MFMA slab
constexpr int hFlush = 256;  // K tiles (4096 complex K) per fp32 MFMA accumulation before fp64
constexpr int hXcd = 8;

__device__ __forceinline__ int xcd_tile16(int w, int total) {
  const int per = total / hXcd, rem = total % hXcd;
  const int x = w % hXcd, i = w / hXcd;
  return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

// (re, im) words -> (im, -re)
__device__ __forceinline__ v8bf swapneg(v8bf v) {
  uint4 u = __builtin_bit_cast(uint4, v);
  u.x = ((u.x >> 16) | (u.x << 16)) ^ 0x80000000u;
  u.y = ((u.y >> 16) | (u.y << 16)) ^ 0x80000000u;
  u.z = ((u.z >> 16) | (u.z << 16)) ^ 0x80000000u;
  u.w = ((u.w >> 16) | (u.w << 16)) ^ 0x80000000u;
  return __builtin_bit_cast(v8bf, u);
}

__device__ __forceinline__ v4f16 mma16(v8bf a, v8bf b, v4f16 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Plane of one K tile: [4 slots][NR rows][8 bf16]; element (row, k') at (k'/8)*NR*8 + row*8 + k'%8.
template <int NR>
__device__ __forceinline__ int plane_off(int row, int kp) {
  // Rows are permuted within aligned groups of 16 by XOR with 4 * slot, so that writers whose lanes
  // span several slots and few rows still reach all 64 banks; a 16-row fragment read stays one
  // conflict-free 256-byte group.
  const int slot = kp >> 3;
  return (slot * NR + (row ^ (4 * (slot & 3)))) * 8 + (kp & 7);
}

// Loader of a K-contiguous complex operand (cn A, cn B): kBK complex = 32 reals per column.
// Writes hi and lo planes of the raw interleaved values.
template <int NC, bool VEC>
struct KcSplit {
  static constexpr int UNITS = 8 * NC;  // 4 reals (2 complex) per unit
  static constexpr int PER = (UNITS + 255) / 256;
  float v[PER][4];
  __device__ __forceinline__ void load(const float2* __restrict__ P, long ld, const float2* __restrict__ P2,
                                       long ld2, int ncol1, int ncols, int c0, int k0, int kend, int tid) {
    if (VEC && c0 + NC <= ncols && k0 + hBK <= kend && (UNITS % 256) == 0) {
      // whole tile inside the operand: no per-element checks
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int idx = tid + q * 256;
        const int u = idx & 7, c = idx >> 3;
        const int gc = c0 + c;
        const float2* col = gc < ncol1 ? P + (long)gc * ld : P2 + (long)(gc - ncol1) * ld2;
        const float4 x = *reinterpret_cast<const float4*>(col + k0 + 2 * u);
        v[q][0] = x.x;
        v[q][1] = x.y;
        v[q][2] = x.z;
        v[q][3] = x.w;
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * 256;
      const int u = idx & 7, c = idx >> 3;
      const int gc = c0 + c, gk = k0 + 2 * u;
      v[q][0] = v[q][1] = v[q][2] = v[q][3] = 0.f;
      if (idx < UNITS && gc < ncols) {
        const float2* col = gc < ncol1 ? P + (long)gc * ld : P2 + (long)(gc - ncol1) * ld2;
        if (VEC && gk + 2 <= kend) {
          const float4 x = *reinterpret_cast<const float4*>(col + gk);
          v[q][0] = x.x;
          v[q][1] = x.y;
          v[q][2] = x.z;
          v[q][3] = x.w;
        } else {
          if (gk < kend) {
            const float2 x = col[gk];
            v[q][0] = x.x;
            v[q][1] = x.y;
          }
          if (gk + 1 < kend) {
            const float2 x = col[gk + 1];
            v[q][2] = x.x;
            v[q][3] = x.y;
          }
        }
      }
    }
  }
  __device__ __forceinline__ void store(unsigned short* Hp, unsigned short* Lp, int tid) const {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * 256;
      if (idx < UNITS) {
        const int u = idx & 7, c = idx >> 3;
        const int off = plane_off<NC>(c, 4 * u);
        Split2 s0 = split(v[q][0]), s1 = split(v[q][1]), s2 = split(v[q][2]), s3 = split(v[q][3]);
        uint2 hh, ll;
        hh.x = pack(s0.h, s1.h);
        hh.y = pack(s2.h, s3.h);
        ll.x = pack(s0.l, s1.l);
        ll.y = pack(s2.l, s3.l);
        *reinterpret_cast<uint2*>(Hp + off) = hh;
        *reinterpret_cast<uint2*>(Lp + off) = ll;
      }
    }
  }
};

// Loader of the nn A operand (M-contiguous columns): NR rows x kBK complex.  Each unit is two
// complex values of rows (m, m+1) at one k.
template <int NR, bool VEC>
struct McSplit {
  static constexpr int UNITS = (NR / 2) * hBK;
  static constexpr int PER = (UNITS + 255) / 256;
  float v[PER][4];
  // unit idx -> row pair mu, k: four consecutive k per group of four lanes, so that a wave covers
  // 16 consecutive row pairs at 4 k (256 contiguous bytes per column)
  __device__ __forceinline__ static void unit(int idx, int& mu, int& k) {
    constexpr int NP = NR / 2;
    k = (idx & 3) + 4 * (idx / (4 * NP));
    mu = (idx >> 2) % NP;
  }
  __device__ __forceinline__ void load(const float2* __restrict__ P, long ld, int nrows, int r0, int k0, int kend,
                                       int tid) {
    if (VEC && r0 + NR <= nrows && k0 + hBK <= kend && (UNITS % 256) == 0) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int idx = tid + q * 256;
        int mu, k;
        unit(idx, mu, k);
        const float4 x = *reinterpret_cast<const float4*>(P + (long)(k0 + k) * ld + r0 + 2 * mu);
        v[q][0] = x.x;
        v[q][1] = x.y;
        v[q][2] = x.z;
        v[q][3] = x.w;
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * 256;
      int mu, k;
      unit(idx, mu, k);
      const int gm = r0 + 2 * mu, gk = k0 + k;
      v[q][0] = v[q][1] = v[q][2] = v[q][3] = 0.f;
      if (idx < UNITS && gk < kend) {
        const float2* col = P + (long)gk * ld;
        if (VEC && gm + 2 <= nrows) {
          const float4 x = *reinterpret_cast<const float4*>(col + gm);
          v[q][0] = x.x;
          v[q][1] = x.y;
          v[q][2] = x.z;
          v[q][3] = x.w;
        } else {
          if (gm < nrows) {
            const float2 x = col[gm];
            v[q][0] = x.x;
            v[q][1] = x.y;
          }
          if (gm + 1 < nrows) {
            const float2 x = col[gm + 1];
            v[q][2] = x.x;
            v[q][3] = x.y;
          }
        }
      }
    }
  }
  __device__ __forceinline__ void store(unsigned short* Hp, unsigned short* Lp, int tid) const {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * 256;
      if (idx < UNITS) {
        int mu, k;
        unit(idx, mu, k);
        const Split2 a = split(v[q][0]), b = split(v[q][1]), c = split(v[q][2]), d = split(v[q][3]);
        const unsigned int w[4] = {pack(a.h, b.h), pack(a.l, b.l), pack(c.h, d.h), pack(c.l, d.l)};
        // the two rows are written in an order that alternates every 8 units, which spreads
        // each write instruction over 16 distinct rows modulo 16
        const int f = (mu >> 3) & 1;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int r = e ^ f;
          const int o = plane_off<NR>(2 * mu + r, 2 * k);
          *reinterpret_cast<unsigned int*>(Hp + o) = w[2 * r];
          *reinterpret_cast<unsigned int*>(Lp + o) = w[2 * r + 1];
        }
      }
    }
  }
};

// Loader of the nn B operand (small K x N, k contiguous): writes the four planes
// Br = (br, -bi) hi/lo and Bi = (bi, br) hi/lo.
template <int NC>
struct KcSplitB {
  static constexpr int UNITS = 8 * NC;
  static constexpr int PER = (UNITS + 255) / 256;
  float v[PER][4];
  __device__ __forceinline__ void load(const float2* __restrict__ P, long ld, int ncols, int c0, int k0, int kend,
                                       int tid) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * 256;
      const int u = idx & 7, c = idx >> 3;
      const int gc = c0 + c, gk = k0 + 2 * u;
      v[q][0] = v[q][1] = v[q][2] = v[q][3] = 0.f;
      if (idx < UNITS && gc < ncols) {
        const float2* col = P + (long)gc * ld;
        if (gk < kend) {
          const float2 x = col[gk];
          v[q][0] = x.x;
          v[q][1] = x.y;
        }
        if (gk + 1 < kend) {
          const float2 x = col[gk + 1];
          v[q][2] = x.x;
          v[q][3] = x.y;
        }
      }
    }
  }
  __device__ __forceinline__ void store(unsigned short* RH, unsigned short* RL, unsigned short* IH,
                                        unsigned short* IL, int tid) const {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * 256;
      if (idx < UNITS) {
        const int u = idx & 7, c = idx >> 3;
        const int off = plane_off<NC>(c, 4 * u);
        const Split2 r0 = split(v[q][0]), i0 = split(v[q][1]), r1 = split(v[q][2]), i1 = split(v[q][3]);
        const Split2 n0 = split(-v[q][1]), n1 = split(-v[q][3]);
        uint2 w;
        w.x = pack(r0.h, n0.h);
        w.y = pack(r1.h, n1.h);
        *reinterpret_cast<uint2*>(RH + off) = w;
        w.x = pack(r0.l, n0.l);
        w.y = pack(r1.l, n1.l);
        *reinterpret_cast<uint2*>(RL + off) = w;
        w.x = pack(i0.h, r0.h);
        w.y = pack(i1.h, r1.h);
        *reinterpret_cast<uint2*>(IH + off) = w;
        w.x = pack(i0.l, r0.l);
        w.y = pack(i1.l, r1.l);
        *reinterpret_cast<uint2*>(IL + off) = w;
      }
    }
  }
};

// A-operand loaders with one interface: load(A0, A1, lda, extent, offset, k0, kend, tid) fetches
// one K tile into registers, store(H, L, tid) writes its hi and lo planes.
template <int NC, bool VEC>
struct CnAF32 {  // cn A from fp32 data (NC columns of A), split on the fly
  KcSplit<NC, VEC> l;
  __device__ __forceinline__ void load(const void* A0, const void*, long lda, int ncols, int c0, int k0, int kend,
                                       int tid) {
    const float2* P = static_cast<const float2*>(A0);
    l.load(P, lda, P, lda, ncols, ncols, c0, k0, kend, tid);
  }
  __device__ __forceinline__ void store(unsigned short* H, unsigned short* L, int tid) const { l.store(H, L, tid); }
};

template <int NR, bool VEC>
struct NnAF32 {  // nn A from fp32 data (NR rows of A), split on the fly
  McSplit<NR, VEC> l;
  __device__ __forceinline__ void load(const void* A0, const void*, long lda, int nrows, int r0, int k0, int kend,
                                       int tid) {
    l.load(static_cast<const float2*>(A0), lda, nrows, r0, k0, kend, tid);
  }
  __device__ __forceinline__ void store(unsigned short* H, unsigned short* L, int tid) const { l.store(H, L, tid); }
};

// cn A from pre-split planes: a unit is 4 complex k (16 bytes) of one column in each plane, which
// is one 8-value k' group of the LDS plane.
template <int NC, bool VEC>
struct CnAPlanes {
  static constexpr int UNITS = 4 * NC;
  static constexpr int PER = (UNITS + 255) / 256;
  uint4 h[PER], l[PER];
  __device__ __forceinline__ void load(const void* A0, const void* A1, long lda, int ncols, int c0, int k0, int kend,
                                       int tid) {
    const unsigned int* Hp = static_cast<const unsigned int*>(A0);
    const unsigned int* Lp = static_cast<const unsigned int*>(A1);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * 256;
      const int sl = idx & 3, c = idx >> 2;
      const int gc = c0 + c, gk = k0 + 4 * sl;
      h[q] = l[q] = uint4{0, 0, 0, 0};
      if (idx < UNITS && gc < ncols) {
        const long o = (long)gc * lda + gk;
        if (VEC && gk + 4 <= kend) {
          h[q] = *reinterpret_cast<const uint4*>(Hp + o);
          l[q] = *reinterpret_cast<const uint4*>(Lp + o);
        } else {
          unsigned int th[4] = {0, 0, 0, 0}, tl[4] = {0, 0, 0, 0};
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (gk + e < kend) {
              th[e] = Hp[o + e];
              tl[e] = Lp[o + e];
            }
          h[q] = uint4{th[0], th[1], th[2], th[3]};
          l[q] = uint4{tl[0], tl[1], tl[2], tl[3]};
        }
      }
    }
  }
  __device__ __forceinline__ void store(unsigned short* H, unsigned short* L, int tid) const {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * 256;
      if (idx < UNITS) {
        const int sl = idx & 3, c = idx >> 2;
        const int off = plane_off<NC>(c, 8 * sl);
        *reinterpret_cast<uint4*>(H + off) = h[q];
        *reinterpret_cast<uint4*>(L + off) = l[q];
      }
    }
  }
};

// nn A from pre-split planes: a unit is 4 consecutive rows at one k in each plane; each word is
// the (re, im) pair at k' = 2k of its row.
template <int NR, bool VEC>
struct NnAPlanes {
  static constexpr int UNITS = (NR / 4) * hBK;
  static constexpr int PER = (UNITS + 255) / 256;
  uint4 h[PER], l[PER];
  // unit idx -> row quad mu, k: four consecutive k per group of four lanes; a wave covers 16
  // consecutive row quads (256 contiguous bytes per column and plane) at 4 k
  __device__ __forceinline__ static void unit(int idx, int& mu, int& k) {
    constexpr int NQ = NR / 4;
    k = (idx & 3) + 4 * (idx / (4 * NQ));
    mu = (idx >> 2) % NQ;
  }
  __device__ __forceinline__ void load(const void* A0, const void* A1, long lda, int nrows, int r0, int k0, int kend,
                                       int tid) {
    const unsigned int* Hp = static_cast<const unsigned int*>(A0);
    const unsigned int* Lp = static_cast<const unsigned int*>(A1);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * 256;
      int mu, k;
      unit(idx, mu, k);
      const int gm = r0 + 4 * mu, gk = k0 + k;
      h[q] = l[q] = uint4{0, 0, 0, 0};
      if (idx < UNITS && gk < kend) {
        const long o = (long)gk * lda + gm;
        if (VEC && gm + 4 <= nrows) {
          h[q] = *reinterpret_cast<const uint4*>(Hp + o);
          l[q] = *reinterpret_cast<const uint4*>(Lp + o);
        } else {
          unsigned int th[4] = {0, 0, 0, 0}, tl[4] = {0, 0, 0, 0};
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (gm + e < nrows) {
              th[e] = Hp[o + e];
              tl[e] = Lp[o + e];
            }
          h[q] = uint4{th[0], th[1], th[2], th[3]};
          l[q] = uint4{tl[0], tl[1], tl[2], tl[3]};
        }
      }
    }
  }
  __device__ __forceinline__ void store(unsigned short* H, unsigned short* L, int tid) const {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * 256;
      if (idx < UNITS) {
        int mu, k;
        unit(idx, mu, k);
        const unsigned int hv[4] = {h[q].x, h[q].y, h[q].z, h[q].w};
        const unsigned int lv[4] = {l[q].x, l[q].y, l[q].z, l[q].w};
        // rotate the row order by mu / 4 so that each write instruction covers 16 distinct rows
        // modulo 16
        const int f = (mu >> 2) & 3;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = (e + f) & 3;
          const int off = plane_off<NR>(4 * mu + r, 2 * k);
          unsigned int hw = hv[0], lw = lv[0];
#pragma unroll
          for (int j = 1; j < 4; ++j)
            if (r == j) {
              hw = hv[j];
              lw = lv[j];
            }
          *reinterpret_cast<unsigned int*>(H + off) = hw;
          *reinterpret_cast<unsigned int*>(L + off) = lw;
        }
      }
    }
  }
};

template <int NR>
__device__ __forceinline__ v8bf frag(const unsigned short* plane, int row, int lane) {
  return *reinterpret_cast<const v8bf*>(plane + plane_off<NR>(row + (lane & 15), 8 * (lane >> 4)));
}

// ------------------------------------------------------------------------------------------
// cn: part[s] = A^H B over K chunk s (fp32 data, bf16x3 products, fp64 partials).
// ------------------------------------------------------------------------------------------
template <int BM, int BN, bool VEC, int NTERM, class AL>
__global__ __launch_bounds__(256) void k_gemm_cn_bf16x3(const void* __restrict__ A0, const void* __restrict__ A1,
                                                        long lda, const float2* __restrict__ B, long ldb,
                                                        const float2* __restrict__ B2, long ldb2, int ncol1, int M,
                                                        int N, int K, int kchunk, int tiles_m, int tiles_n,
                                                        double2* __restrict__ part) {
  constexpr int WBM = BM / 32, WBN = BN / 32;
  constexpr int PA = 4 * BM * 8, PB = 4 * BN * 8;  // plane sizes (bf16 elements)
  __shared__ unsigned short sAh[2][PA], sAl[2][PA], sBh[2][PB], sBl[2][PB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int t = xcd_tile16(blockIdx.x, gridDim.x);
  const int sp = t / (tiles_m * tiles_n);
  const int tr = t - sp * tiles_m * tiles_n;
  const int tm = tr / tiles_n, tn = tr - tm * tiles_n;
  const int i0 = tm * BM, j0 = tn * BN;
  const int kb = sp * kchunk, ke = min(K, kb + kchunk);
  const int mo = (wave & 1) * (BM / 2), no = (wave >> 1) * (BN / 2);
  // Two accumulation levels: the MFMA accumulators (fp32) over hFlush K tiles, then the fp64
  // partial in global memory, which this workgroup alone owns.
  v4f16 cr[WBM][WBN], ci[WBM][WBN];
  AL la;
  KcSplit<BN, VEC> lb;
  const int ntiles = ke > kb ? (ke - kb + hBK - 1) / hBK : 0;
  if (ntiles > 0) {
    la.load(A0, A1, lda, M, i0, kb, ke, tid);
    lb.load(B, ldb, B2, ldb2, ncol1, N, j0, kb, ke, tid);
    la.store(sAh[0], sAl[0], tid);
    lb.store(sBh[0], sBl[0], tid);
  }
  __syncthreads();
  bool stored = false;
  int it = 0;
  do {
    const int fend = min(ntiles, it + hFlush);
#pragma unroll
    for (int a = 0; a < WBM; ++a)
#pragma unroll
      for (int b = 0; b < WBN; ++b) cr[a][b] = ci[a][b] = v4f16{0, 0, 0, 0};
    for (; it < fend; ++it) {
      const int cur = it & 1;
      const bool more = it + 1 < ntiles;
      if (more) {
        const int kn = kb + (it + 1) * hBK;
        la.load(A0, A1, lda, M, i0, kn, ke, tid);
        lb.load(B, ldb, B2, ldb2, ncol1, N, j0, kn, ke, tid);
      }
      v8bf ah[WBM], al[WBM];
#pragma unroll
      for (int a = 0; a < WBM; ++a) {
        ah[a] = frag<BM>(sAh[cur], mo + a * 16, lane);
        al[a] = frag<BM>(sAl[cur], mo + a * 16, lane);
      }
#pragma unroll
      for (int b = 0; b < WBN; ++b) {
        const v8bf bh = frag<BN>(sBh[cur], no + b * 16, lane);
        const v8bf bl = frag<BN>(sBl[cur], no + b * 16, lane);
        const v8bf bh2 = swapneg(bh), bl2 = swapneg(bl);
#pragma unroll
        for (int a = 0; a < WBM; ++a) {
          cr[a][b] = mma16(ah[a], bh, cr[a][b]);
          ci[a][b] = mma16(ah[a], bh2, ci[a][b]);
          cr[a][b] = mma16(ah[a], bl, cr[a][b]);
          ci[a][b] = mma16(ah[a], bl2, ci[a][b]);
          cr[a][b] = mma16(al[a], bh, cr[a][b]);
          ci[a][b] = mma16(al[a], bh2, ci[a][b]);
          if constexpr (NTERM == 4) {
            cr[a][b] = mma16(al[a], bl, cr[a][b]);
            ci[a][b] = mma16(al[a], bl2, ci[a][b]);
          }
        }
      }
      if (more) {
        la.store(sAh[cur ^ 1], sAl[cur ^ 1], tid);
        lb.store(sBh[cur ^ 1], sBl[cur ^ 1], tid);
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
          const int row = i0 + mo + a * 16 + 4 * (lane >> 4) + r;
          if (row < M && col < N) {
            double2* dst = part + ((long)sp * N + col) * M + row;
            double2 v;
            v.x = (double)cr[a][b][r];
            v.y = (double)ci[a][b][r];
            if (stored) {
              const double2 o = *dst;
              v.x += o.x;
              v.y += o.y;
            }
            *dst = v;
          }
        }
      }
    stored = true;
  } while (it < ntiles);
}

// ------------------------------------------------------------------------------------------
// nn: out = epilogue(A B) (fp32 data, bf16x3 products).
// ------------------------------------------------------------------------------------------
template <int BM, int BN, class AL>
__global__ __launch_bounds__(256) void k_gemm_nn_bf16x3(const void* __restrict__ A0, const void* __restrict__ A1,
                                                        long lda, const float2* __restrict__ B, long ldb, int M, int N,
                                                        int K,
                                                        int tiles_n, float2* out, long ldo, EpiH e) {
  constexpr int WBM = BM / 32, WBN = BN / 32;
  constexpr int PA = 4 * BM * 8, PB = 4 * BN * 8;
  __shared__ unsigned short sAh[2][PA], sAl[2][PA], sRH[2][PB], sRL[2][PB], sIH[2][PB], sIL[2][PB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int t = xcd_tile16(blockIdx.x, gridDim.x);
  const int tm = t / tiles_n, tn = t - tm * tiles_n;
  const int i0 = tm * BM, j0 = tn * BN;
  const int mo = (wave & 1) * (BM / 2), no = (wave >> 1) * (BN / 2);
  v4f16 cr[WBM][WBN], ci[WBM][WBN];
#pragma unroll
  for (int a = 0; a < WBM; ++a)
#pragma unroll
    for (int b = 0; b < WBN; ++b) {
      cr[a][b] = v4f16{0, 0, 0, 0};
      ci[a][b] = v4f16{0, 0, 0, 0};
    }
  AL la;
  KcSplitB<BN> lb;
  const int ntiles = (K + hBK - 1) / hBK;
  if (ntiles > 0) {
    la.load(A0, A1, lda, M, i0, 0, K, tid);
    lb.load(B, ldb, N, j0, 0, K, tid);
    la.store(sAh[0], sAl[0], tid);
    lb.store(sRH[0], sRL[0], sIH[0], sIL[0], tid);
  }
  __syncthreads();
  for (int it = 0; it < ntiles; ++it) {
    const int cur = it & 1;
    const bool more = it + 1 < ntiles;
    if (more) {
      const int kn = (it + 1) * hBK;
      la.load(A0, A1, lda, M, i0, kn, K, tid);
      lb.load(B, ldb, N, j0, kn, K, tid);
    }
    v8bf ah[WBM], al[WBM];
#pragma unroll
    for (int a = 0; a < WBM; ++a) {
      ah[a] = frag<BM>(sAh[cur], mo + a * 16, lane);
      al[a] = frag<BM>(sAl[cur], mo + a * 16, lane);
    }
#pragma unroll
    for (int b = 0; b < WBN; ++b) {
      const v8bf rh = frag<BN>(sRH[cur], no + b * 16, lane);
      const v8bf rl = frag<BN>(sRL[cur], no + b * 16, lane);
      const v8bf ih = frag<BN>(sIH[cur], no + b * 16, lane);
      const v8bf il = frag<BN>(sIL[cur], no + b * 16, lane);
#pragma unroll
      for (int a = 0; a < WBM; ++a) {
        cr[a][b] = mma16(ah[a], rh, cr[a][b]);
        ci[a][b] = mma16(ah[a], ih, ci[a][b]);
        cr[a][b] = mma16(ah[a], rl, cr[a][b]);
        ci[a][b] = mma16(ah[a], il, ci[a][b]);
        cr[a][b] = mma16(al[a], rh, cr[a][b]);
        ci[a][b] = mma16(al[a], ih, ci[a][b]);
      }
    }
    if (more) {
      la.store(sAh[cur ^ 1], sAl[cur ^ 1], tid);
      lb.store(sRH[cur ^ 1], sRL[cur ^ 1], sIH[cur ^ 1], sIL[cur ^ 1], tid);
    }
    __syncthreads();
  }
  const float* kin = static_cast<const float*>(e.kin);
  const float2* Y = static_cast<const float2*>(e.Y);
  const float2* Zl = static_cast<const float2*>(e.Zl);
  const float2* Yp = static_cast<const float2*>(e.Yp);
  const float alpha = (float)e.alpha, cc = (float)e.c, beta = (float)e.beta;
#pragma unroll
  for (int a = 0; a < WBM; ++a)
#pragma unroll
    for (int b = 0; b < WBN; ++b) {
      const int col = j0 + no + b * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + mo + a * 16 + 4 * (lane >> 4) + r;
        if (row < M && col < N) {
          float2 v = make_float2(cr[a][b][r], ci[a][b][r]);
          if (e.mode == 1) {
            const float2 y = Y[(long)col * e.ldy + row];
            const float2 z = Zl[(long)col * e.ldz + row];
            const float kc = kin[row] - cc;
            v.x = alpha * (kc * y.x + z.x + v.x);
            v.y = alpha * (kc * y.y + z.y + v.y);
            if (Yp) {
              const float2 p = Yp[(long)col * e.ldp + row];
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

static inline bool ok16(const void* p, long ld) {
  return (reinterpret_cast<uintptr_t>(p) & 15) == 0 && (ld % 2) == 0;
}

constexpr int kCnBM = 128, kCnBN = 64, kNnBM = 128, kNnBN = 64;

int gemm_cn_bf16_tiles(int M, int N) { return ceil_div(M, kCnBM) * ceil_div(N, kCnBN); }

hipError_t launch_gemm_cn_bf16x3(const float2* A, long lda, const float2* B, long ldb, const float2* B2, long ldb2,
                                 int ncol1, int M, int N, int K, int nsplit, double2* part, int nterm, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  int kchunk = ceil_div(K, nsplit);
  kchunk = ceil_div(kchunk, hBK) * hBK;
  if (kchunk <= 0) kchunk = hBK;
  const int tm = ceil_div(M, kCnBM), tn = ceil_div(N, kCnBN);
  const float2* b2 = B2 ? B2 : B;
  const long l2 = B2 ? ldb2 : ldb;
  const bool vec = ok16(A, lda) && ok16(B, ldb) && ok16(b2, l2);
  dim3 grid(tm * tn * nsplit);
#define PW_CN16(V, NT)                                                                                            \
  hipLaunchKernelGGL((k_gemm_cn_bf16x3<kCnBM, kCnBN, V, NT, CnAF32<kCnBM, V>>), grid, dim3(256), 0, s,          \
                     static_cast<const void*>(A), static_cast<const void*>(nullptr), lda, B, ldb, b2, l2, ncol1, M, \
                     N, K, kchunk, tm, tn, part)
  if (nterm == 4) {
    if (vec) PW_CN16(true, 4); else PW_CN16(false, 4);
  } else {
    if (vec) PW_CN16(true, 3); else PW_CN16(false, 3);
  }
#undef PW_CN16
  return hipGetLastError();
}

static inline bool ok_planes(const void* h, const void* l, long lda) {
  return (reinterpret_cast<uintptr_t>(h) & 15) == 0 && (reinterpret_cast<uintptr_t>(l) & 15) == 0 && (lda % 4) == 0;
}

hipError_t launch_gemm_cn_bf16x3_planes(const unsigned int* Ahi, const unsigned int* Alo, long lda, const float2* B,
                                        long ldb, int M, int N, int K, int nsplit, double2* part, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  int kchunk = ceil_div(K, nsplit);
  kchunk = ceil_div(kchunk, hBK) * hBK;
  if (kchunk <= 0) kchunk = hBK;
  const int tm = ceil_div(M, kCnBM), tn = ceil_div(N, kCnBN);
  const bool vec = ok_planes(Ahi, Alo, lda) && ok16(B, ldb);
  dim3 grid(tm * tn * nsplit);
  if (vec)
    hipLaunchKernelGGL((k_gemm_cn_bf16x3<kCnBM, kCnBN, true, 3, CnAPlanes<kCnBM, true>>), grid, dim3(256), 0, s,
                       static_cast<const void*>(Ahi), static_cast<const void*>(Alo), lda, B, ldb, B, ldb, N, M, N, K,
                       kchunk, tm, tn, part);
  else
    hipLaunchKernelGGL((k_gemm_cn_bf16x3<kCnBM, kCnBN, false, 3, CnAPlanes<kCnBM, false>>), grid, dim3(256), 0, s,
                       static_cast<const void*>(Ahi), static_cast<const void*>(Alo), lda, B, ldb, B, ldb, N, M, N, K,
                       kchunk, tm, tn, part);
  return hipGetLastError();
}

hipError_t launch_gemm_nn_bf16x3(const float2* A, long lda, const float2* B, long ldb, int M, int N, int K,
                                 float2* out, long ldo, const EpiH& e, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int tm = ceil_div(M, kNnBM), tn = ceil_div(N, kNnBN);
  const bool vec = ok16(A, lda);
  dim3 grid(tm * tn);
  const void* a0 = A;
  if (vec)
    hipLaunchKernelGGL((k_gemm_nn_bf16x3<kNnBM, kNnBN, NnAF32<kNnBM, true>>), grid, dim3(256), 0, s, a0, nullptr,
                       lda, B, ldb, M, N, K, tn, out, ldo, e);
  else
    hipLaunchKernelGGL((k_gemm_nn_bf16x3<kNnBM, kNnBN, NnAF32<kNnBM, false>>), grid, dim3(256), 0, s, a0, nullptr,
                       lda, B, ldb, M, N, K, tn, out, ldo, e);
  return hipGetLastError();
}

hipError_t launch_gemm_nn_bf16x3_planes(const unsigned int* Ahi, const unsigned int* Alo, long lda, const float2* B,
                                        long ldb, int M, int N, int K, float2* out, long ldo, const EpiH& e,
                                        hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int tm = ceil_div(M, kNnBM), tn = ceil_div(N, kNnBN);
  const bool vec = ok_planes(Ahi, Alo, lda);
  dim3 grid(tm * tn);
  const void* a0 = Ahi;
  const void* a1 = Alo;
  if (vec)
    hipLaunchKernelGGL((k_gemm_nn_bf16x3<kNnBM, kNnBN, NnAPlanes<kNnBM, true>>), grid, dim3(256), 0, s, a0, a1, lda,
                       B, ldb, M, N, K, tn, out, ldo, e);
  else
    hipLaunchKernelGGL((k_gemm_nn_bf16x3<kNnBM, kNnBN, NnAPlanes<kNnBM, false>>), grid, dim3(256), 0, s, a0, a1, lda,
                       B, ldb, M, N, K, tn, out, ldo, e);
  return hipGetLastError();
}

}  // namespace pw
