// Split-precision complex GEMMs on the bf16 matrix cores (MFMA 16x16x32 bf16, fp32 accumulation).
//
// Every fp32 operand x is split into hi = bf16(x) and lo = bf16(x - hi) (round to nearest even;
// x - hi is exact in fp32).  A real product is formed as hi*hi' + hi*lo' + lo*hi' (three terms),
// which drops lo*lo' and the residual of the two-term split (2^-16 relative at most), or with
// lo*lo' added (four terms).  The four-term form is used for the Gram / projected matrices: in a
// self product such as sum |y|^2 the dropped lo*lo' has one sign and would bias the sums, while
// the split residual left by the four-term form has no preferred sign.
//
// Complex products are written as real products over the interleaved (re, im) dimension k':
//   cn, C = A^H B:  Re C = sum_k' A'_k' B'_k',   Im C = sum_k' A'_k' B''_k'
//                   A' = (ar, ai), B' = (br, bi), B'' = (bi, -br)  per complex k
//   nn, C = A B:    Re C = sum_k' A'_k' Br_k',   Im C = sum_k' A'_k' Bi_k'
//                   A' = (ar, ai), Br = (br, -bi), Bi = (bi, br)
// Only A' and B' (cn) or A' and Br (nn) are stored; B'' and Bi come from them in registers by
// rotating each 32-bit word by 16 bits and flipping one sign bit.
//
// Workgroup: 4 waves, tile 128 x 128, each wave 64 x 64 (4 x 4 MFMA blocks, 128 accumulator
// registers).  K tiles of 16 complex (32 k') are staged through two LDS buffers; the next tile is
// fetched into registers while the MFMAs run on the current one, so each tile costs one barrier.
//
// MFMA 16x16x32 bf16: lane l supplies 8 consecutive k' values of row/column l % 16 from k' slot
// l / 16; the accumulator layout is that of the fp32 16x16x4 instruction (C[4 (l/16) + r][l % 16]).
// LDS plane of one operand tile (NR rows x 32 k'): 16-byte chunks (8 k' of one row), chunk of
// (row, slot) at ((row / 16) * 4 + slot) * 16 + ((row % 16) ^ slot).  A 16-row fragment is then
// one contiguous kilobyte read lane by lane, and every loader below maps its lanes so that each
// LDS write instruction touches distinct banks.

#include <type_traits>

#include "bf16split.hpp"
#include "common.hpp"
#include "kernels.hpp"
#include "pipe_addr.hpp"

namespace pw {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f16 __attribute__((ext_vector_type(4)));

constexpr int hBK = 16;       // complex K per tile = 32 real k' = one MFMA slab
constexpr int hFlush = 256;   // K tiles (4096 complex K) per fp32 MFMA accumulation before fp64
constexpr int hXcd = 8;
constexpr int hTM = 128, hTN = 128;  // workgroup tile

__device__ __forceinline__ int chunk_of(int row, int slot) {
  return (((row >> 4) << 2) + slot) * 16 + ((row & 15) ^ slot);
}

__device__ __forceinline__ int xcd_tile16(int w, int total) {
  const int per = total / hXcd, rem = total % hXcd;
  const int x = w % hXcd, i = w / hXcd;
  return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

// (re, im) words -> (im, -re): B'' from B' (cn)
__device__ __forceinline__ v8bf swapneg_hi(v8bf v) {
  uint4 u = __builtin_bit_cast(uint4, v);
  u.x = ((u.x >> 16) | (u.x << 16)) ^ 0x80000000u;
  u.y = ((u.y >> 16) | (u.y << 16)) ^ 0x80000000u;
  u.z = ((u.z >> 16) | (u.z << 16)) ^ 0x80000000u;
  u.w = ((u.w >> 16) | (u.w << 16)) ^ 0x80000000u;
  return __builtin_bit_cast(v8bf, u);
}
// (br, -bi) words -> (bi, br): Bi from Br (nn)
__device__ __forceinline__ v8bf swapneg_lo(v8bf v) {
  uint4 u = __builtin_bit_cast(uint4, v);
  u.x = ((u.x >> 16) | (u.x << 16)) ^ 0x00008000u;
  u.y = ((u.y >> 16) | (u.y << 16)) ^ 0x00008000u;
  u.z = ((u.z >> 16) | (u.z << 16)) ^ 0x00008000u;
  u.w = ((u.w >> 16) | (u.w << 16)) ^ 0x00008000u;
  return __builtin_bit_cast(v8bf, u);
}

__device__ __forceinline__ v4f16 mma16(v8bf a, v8bf b, v4f16 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Fragment of rows row0..row0+15 (row0 a multiple of 16): lane l reads chunk (row0 + l % 16, l / 16).
__device__ __forceinline__ v8bf frag(const uint4* plane, int row0, int lane) {
  const int slot = lane >> 4, i = lane & 15;
  return __builtin_bit_cast(v8bf, plane[((row0 >> 4) << 6) + slot * 16 + (i ^ slot)]);
}

// ------------------------------------------------------------------------------------------
// Loaders.  load() fetches one K tile into registers, store() writes the hi and lo planes.
// ------------------------------------------------------------------------------------------

// K-contiguous fp32 complex columns (cn A or B; NC columns, optional second matrix for columns
// >= ncol1), split on the fly.  Unit: 2 complex (16 bytes) of one column -> 8 bytes per plane.
// Lanes: bit 0 half of the chunk, bits 1-4 column within 16, bits 5-6 slot, higher bits column
// group: a wave writes 512 contiguous bytes per plane.  NEG negates the imaginary parts (nn B).
template <int NC, bool VEC, bool NEG, int NTH = 256>
struct SplitK {
  static constexpr int UNITS = 8 * NC;
  static constexpr int PER = UNITS / NTH;
  static_assert(UNITS % NTH == 0, "whole units per thread");
  float v[PER][4];
  __device__ __forceinline__ static void unit(int idx, int& c, int& half, int& slot) {
    half = idx & 1;
    slot = (idx >> 5) & 3;
    c = ((idx >> 7) << 4) + ((idx >> 1) & 15);
  }
  __device__ __forceinline__ void load(const float2* __restrict__ P, long ld, const float2* __restrict__ P2,
                                       long ld2, int ncol1, int ncols, int c0, int k0, int kend, int tid) {
    const bool full = VEC && c0 + NC <= ncols && k0 + hBK <= kend;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      int c, half, slot;
      unit(tid + q * NTH, c, half, slot);
      const int gc = c0 + c, gk = k0 + 4 * slot + 2 * half;
      const float2* col = gc < ncol1 ? P + (long)gc * ld : P2 + (long)(gc - ncol1) * ld2;
      if (full) {
        const float4 x = *reinterpret_cast<const float4*>(col + gk);
        v[q][0] = x.x;
        v[q][1] = x.y;
        v[q][2] = x.z;
        v[q][3] = x.w;
      } else {
        v[q][0] = v[q][1] = v[q][2] = v[q][3] = 0.f;
        if (gc < ncols) {
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
  }
  __device__ __forceinline__ void store(uint4* H, uint4* L, int tid) const {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      int c, half, slot;
      unit(tid + q * NTH, c, half, slot);
      const Split2 r0 = split(v[q][0]), i0 = split(NEG ? -v[q][1] : v[q][1]);
      const Split2 r1 = split(v[q][2]), i1 = split(NEG ? -v[q][3] : v[q][3]);
      const int o = chunk_of(c, slot);
      reinterpret_cast<uint2*>(H + o)[half] = uint2{pack(r0.h, i0.h), pack(r1.h, i1.h)};
      reinterpret_cast<uint2*>(L + o)[half] = uint2{pack(r0.l, i0.l), pack(r1.l, i1.l)};
    }
  }
};

// M-contiguous fp32 complex columns (nn A), split on the fly.  Unit: rows (2 mu, 2 mu + 1) at one
// k.  Lanes: bits 0-1 k within 4, then 16 consecutive row pairs; the two rows are written in an
// order that alternates every 8 pairs, so each write instruction covers 16 distinct rows modulo 16
// and 4 words of each chunk (all 64 banks).
template <int NR, bool VEC>
struct SplitM {
  static constexpr int NP = NR / 2;
  static constexpr int UNITS = NP * hBK;
  static constexpr int PER = UNITS / 256;
  static_assert(UNITS % 256 == 0, "whole units per thread");
  float v[PER][4];
  __device__ __forceinline__ static void unit(int idx, int& mu, int& k) {
    k = (idx & 3) + 4 * (idx / (4 * NP));
    mu = (idx >> 2) % NP;
  }
  __device__ __forceinline__ void load(const float2* __restrict__ P, long ld, int nrows, int r0, int k0, int kend,
                                       int tid) {
    const bool full = VEC && r0 + NR <= nrows && k0 + hBK <= kend;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      int mu, k;
      unit(tid + q * 256, mu, k);
      const int gm = r0 + 2 * mu, gk = k0 + k;
      const float2* col = P + (long)gk * ld;
      if (full) {
        const float4 x = *reinterpret_cast<const float4*>(col + gm);
        v[q][0] = x.x;
        v[q][1] = x.y;
        v[q][2] = x.z;
        v[q][3] = x.w;
      } else {
        v[q][0] = v[q][1] = v[q][2] = v[q][3] = 0.f;
        if (gk < kend) {
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
  }
  __device__ __forceinline__ void store(uint4* H, uint4* L, int tid) const {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      int mu, k;
      unit(tid + q * 256, mu, k);
      const Split2 a = split(v[q][0]), b = split(v[q][1]), c = split(v[q][2]), d = split(v[q][3]);
      const unsigned int w[4] = {pack(a.h, b.h), pack(a.l, b.l), pack(c.h, d.h), pack(c.l, d.l)};
      const int f = (mu >> 3) & 1;
      const int slot = k >> 2, word = k & 3;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int r = e ^ f;
        const int o = chunk_of(2 * mu + r, slot);
        reinterpret_cast<unsigned int*>(H + o)[word] = r ? w[2] : w[0];
        reinterpret_cast<unsigned int*>(L + o)[word] = r ? w[3] : w[1];
      }
    }
  }
};

// K-contiguous pre-split planes (cn A = projector planes): unit = 4 complex k (one chunk) of one
// column per plane.  Lanes: bits 0-3 column within 16, bits 4-5 slot: a wave writes one
// contiguous kilobyte per plane.
template <int NC, bool VEC, int NTH = 256>
struct PlanesK {
  static constexpr int UNITS = 4 * NC;
  static constexpr int PER = UNITS / NTH;
  static_assert(UNITS % NTH == 0, "whole units per thread");
  uint4 h[PER], l[PER];
  __device__ __forceinline__ void load(const unsigned int* __restrict__ Hp, const unsigned int* __restrict__ Lp,
                                       long lda, int ncols, int c0, int k0, int kend, int tid) {
    const bool full = VEC && c0 + NC <= ncols && k0 + hBK <= kend;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * NTH;
      const int c = ((idx >> 6) << 4) + (idx & 15), slot = (idx >> 4) & 3;
      const int gc = c0 + c, gk = k0 + 4 * slot;
      const long o = (long)gc * lda + gk;
      if (full) {
        h[q] = *reinterpret_cast<const uint4*>(Hp + o);
        l[q] = *reinterpret_cast<const uint4*>(Lp + o);
      } else {
        h[q] = l[q] = uint4{0, 0, 0, 0};
        if (gc < ncols) {
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
  }
  __device__ __forceinline__ void store(uint4* H, uint4* L, int tid) const {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * NTH;
      const int c = ((idx >> 6) << 4) + (idx & 15), slot = (idx >> 4) & 3;
      const int o = chunk_of(c, slot);
      H[o] = h[q];
      L[o] = l[q];
    }
  }
};

// M-contiguous pre-split planes (nn A = projector planes): unit = 4 rows x 4 k of one plane,
// loaded as four 16-byte row quads (one per k) and transposed in registers into four chunks (one
// per row).  The first NR threads take the hi plane, the others the lo plane.  Lanes: bits 0-1 k quad,
// bits 2-5 row quad; with the chunk swizzle each write instruction covers 16 distinct chunks.
template <int NR, bool VEC, int NTH = 256>
struct PlanesM {
  static_assert(NTH == 2 * NR && hBK == 16, "one unit per thread");
  uint4 t[4];
  __device__ __forceinline__ void load(const unsigned int* __restrict__ Hp, const unsigned int* __restrict__ Lp,
                                       long lda, int nrows, int r0, int k0, int kend, int tid) {
    const unsigned int* Pp = tid < NR ? Hp : Lp;
    const int u = tid % NR;
    const int kq = u & 3, gq = u >> 2;
    const int gm = r0 + 4 * gq;
    const bool full = VEC && r0 + NR <= nrows && k0 + hBK <= kend;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gk = k0 + 4 * kq + j;
      const long o = (long)gk * lda + gm;
      if (full) {
        t[j] = *reinterpret_cast<const uint4*>(Pp + o);
      } else {
        t[j] = uint4{0, 0, 0, 0};
        if (gk < kend) {
          if (VEC && gm + 4 <= nrows) {
            t[j] = *reinterpret_cast<const uint4*>(Pp + o);
          } else {
            unsigned int w[4] = {0, 0, 0, 0};
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (gm + e < nrows) w[e] = Pp[o + e];
            t[j] = uint4{w[0], w[1], w[2], w[3]};
          }
        }
      }
    }
  }
  __device__ __forceinline__ void store(uint4* H, uint4* L, int tid) const {
    uint4* D = tid < NR ? H : L;
    const int u = tid % NR;
    const int kq = u & 3, gq = u >> 2;
    D[chunk_of(4 * gq + 0, kq)] = uint4{t[0].x, t[1].x, t[2].x, t[3].x};
    D[chunk_of(4 * gq + 1, kq)] = uint4{t[0].y, t[1].y, t[2].y, t[3].y};
    D[chunk_of(4 * gq + 2, kq)] = uint4{t[0].z, t[1].z, t[2].z, t[3].z};
    D[chunk_of(4 * gq + 3, kq)] = uint4{t[0].w, t[1].w, t[2].w, t[3].w};
  }
};

// A-operand adapters with one interface (the kernels take two untyped pointers).
template <int NC, bool VEC>
struct CnAF32 {
  SplitK<NC, VEC, false> l;
  __device__ __forceinline__ void load(const void* A0, const void*, long lda, int ncols, int c0, int k0, int kend,
                                       int tid) {
    const float2* P = static_cast<const float2*>(A0);
    l.load(P, lda, P, lda, ncols, ncols, c0, k0, kend, tid);
  }
  __device__ __forceinline__ void store(uint4* H, uint4* L, int tid) const { l.store(H, L, tid); }
};
template <int NC, bool VEC, int NTH = 256>
struct CnAPlanes {
  PlanesK<NC, VEC, NTH> l;
  __device__ __forceinline__ void load(const void* A0, const void* A1, long lda, int ncols, int c0, int k0, int kend,
                                       int tid) {
    l.load(static_cast<const unsigned int*>(A0), static_cast<const unsigned int*>(A1), lda, ncols, c0, k0, kend,
           tid);
  }
  __device__ __forceinline__ void store(uint4* H, uint4* L, int tid) const { l.store(H, L, tid); }
};
template <int NR, bool VEC>
struct NnAF32 {
  SplitM<NR, VEC> l;
  __device__ __forceinline__ void load(const void* A0, const void*, long lda, int nrows, int r0, int k0, int kend,
                                       int tid) {
    l.load(static_cast<const float2*>(A0), lda, nrows, r0, k0, kend, tid);
  }
  __device__ __forceinline__ void store(uint4* H, uint4* L, int tid) const { l.store(H, L, tid); }
};
template <int NR, bool VEC, int NTH = 256>
struct NnAPlanes {
  PlanesM<NR, VEC, NTH> l;
  __device__ __forceinline__ void load(const void* A0, const void* A1, long lda, int nrows, int r0, int k0, int kend,
                                       int tid) {
    l.load(static_cast<const unsigned int*>(A0), static_cast<const unsigned int*>(A1), lda, nrows, r0, k0, kend,
           tid);
  }
  __device__ __forceinline__ void store(uint4* H, uint4* L, int tid) const { l.store(H, L, tid); }
};

// cn B-operand adapters: fp32 columns split on the fly (with the optional second matrix of the
// Gram product), or pre-split planes.
template <int NC, bool VEC>
struct CnBF32 {
  SplitK<NC, VEC, false> l;
  __device__ __forceinline__ void load(const void* B0, const void*, long ldb, const void* B2, long ldb2, int ncol1,
                                       int ncols, int c0, int k0, int kend, int tid) {
    l.load(static_cast<const float2*>(B0), ldb, static_cast<const float2*>(B2), ldb2, ncol1, ncols, c0, k0, kend,
           tid);
  }
  __device__ __forceinline__ void store(uint4* H, uint4* L, int tid) const { l.store(H, L, tid); }
};
template <int NC, bool VEC, int NTH = 256>
struct CnBPlanes {
  PlanesK<NC, VEC, NTH> l;
  __device__ __forceinline__ void load(const void* B0, const void* B1, long ldb, const void*, long, int, int ncols,
                                       int c0, int k0, int kend, int tid) {
    l.load(static_cast<const unsigned int*>(B0), static_cast<const unsigned int*>(B1), ldb, ncols, c0, k0, kend, tid);
  }
  __device__ __forceinline__ void store(uint4* H, uint4* L, int tid) const { l.store(H, L, tid); }
};

// nn B-operand adapters: the K-contiguous columns of B as Br = (br, -bi) words, either fp32 split on
// the fly or planes already holding those words (launch_reduce_planes).
template <int NC, int NTH = 256>
struct NnBF32 {
  SplitK<NC, false, true, NTH> l;  // B rows are small, scalar loads
  __device__ __forceinline__ void load(const void* B0, const void*, long ldb, int ncols, int c0, int k0, int kend,
                                       int tid) {
    const float2* P = static_cast<const float2*>(B0);
    l.load(P, ldb, P, ldb, ncols, ncols, c0, k0, kend, tid);
  }
  __device__ __forceinline__ void store(uint4* H, uint4* L, int tid) const { l.store(H, L, tid); }
};
template <int NC, bool VEC, int NTH = 256>
struct NnBPlanes {
  PlanesK<NC, VEC, NTH> l;
  __device__ __forceinline__ void load(const void* B0, const void* B1, long ldb, int ncols, int c0, int k0, int kend,
                                       int tid) {
    l.load(static_cast<const unsigned int*>(B0), static_cast<const unsigned int*>(B1), ldb, ncols, c0, k0, kend, tid);
  }
  __device__ __forceinline__ void store(uint4* H, uint4* L, int tid) const { l.store(H, L, tid); }
};

// ------------------------------------------------------------------------------------------
// cn: part[s] = A^H B over K chunk s (fp32 accumulation per hFlush tiles, fp64 partials).
// ------------------------------------------------------------------------------------------
// Workgroup of NT threads (NT / 64 waves of 64 x 64), tile TM x TN with TM / 64 waves along M.
template <int NTERM, class AL, class BL, int TM = hTM, int NT = 256>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_gemm_cn_bf16x3(
    const void* __restrict__ A0, const void* __restrict__ A1, long lda, const void* __restrict__ B0,
    const void* __restrict__ B1, long ldb, const void* __restrict__ B2, long ldb2, int ncol1, int M, int N, int K,
    int kchunk, int tiles_m, int tiles_n, double2* __restrict__ part) {
  constexpr int WM = TM / 64, TN = 64 * (NT / 64) / WM;
  constexpr int PA = TM * 4, PB = TN * 4;  // chunks per plane
  __shared__ uint4 sAh[2][PA], sAl[2][PA], sBh[2][PB], sBl[2][PB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int t = xcd_tile16(blockIdx.x, gridDim.x);
  const int sp = t / (tiles_m * tiles_n);
  const int tr = t - sp * tiles_m * tiles_n;
  const int tm = tr / tiles_n, tn = tr - tm * tiles_n;
  const int i0 = tm * TM, j0 = tn * TN;
  const int kb = sp * kchunk, ke = min(K, kb + kchunk);
  const int mo = (wave % WM) * 64, no = (wave / WM) * 64;
  v4f16 cr[4][4], ci[4][4];
  AL la;
  BL lb;
  const int ntiles = ke > kb ? (ke - kb + hBK - 1) / hBK : 0;
  if (ntiles > 0) {
    la.load(A0, A1, lda, M, i0, kb, ke, tid);
    lb.load(B0, B1, ldb, B2, ldb2, ncol1, N, j0, kb, ke, tid);
    la.store(sAh[0], sAl[0], tid);
    lb.store(sBh[0], sBl[0], tid);
  }
  __syncthreads();
  bool stored = false;
  int it = 0;
  do {
    const int fend = min(ntiles, it + hFlush);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) cr[a][b] = ci[a][b] = v4f16{0, 0, 0, 0};
    for (; it < fend; ++it) {
      const int cur = it & 1;
      const bool more = it + 1 < ntiles;
      if (more) {
        const int kn = kb + (it + 1) * hBK;
        la.load(A0, A1, lda, M, i0, kn, ke, tid);
        lb.load(B0, B1, ldb, B2, ldb2, ncol1, N, j0, kn, ke, tid);
      }
      v8bf ah[4], al[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        ah[a] = frag(sAh[cur], mo + a * 16, lane);
        al[a] = frag(sAl[cur], mo + a * 16, lane);
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const v8bf bh = frag(sBh[cur], no + b * 16, lane);
        const v8bf bl = frag(sBl[cur], no + b * 16, lane);
        const v8bf bh2 = swapneg_hi(bh), bl2 = swapneg_hi(bl);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
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
    // fp64 partial, owned by this workgroup
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
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

// Epilogue of the nn products for a wave's AT x BT blocks of 16 x 16 (accumulator layout of the
// 16 x 16 MFMA: lane l holds rows 4 (l / 16) + r, column l % 16): out = update(acc) as EpiH says,
// plus the bf16 planes of out when e.ph is set.
template <int AT, int BT>
__device__ __forceinline__ void epi_tile(const v4f16 (&cr)[AT][BT], const v4f16 (&ci)[AT][BT], int row_base,
                                         int col_base, int lane, int M, int N, float2* out, long ldo,
                                         const EpiH& e) {
  const float* kin = static_cast<const float*>(e.kin);
  const float2* Y = static_cast<const float2*>(e.Y);
  const float2* Zl = static_cast<const float2*>(e.Zl);
  const float2* Yp = static_cast<const float2*>(e.Yp);
  const float alpha = (float)e.alpha, cc = (float)e.c, beta = (float)e.beta;
  const float2 zero2 = make_float2(0.f, 0.f);
  // one entry: v = accumulator, kr = kin[row], y, z, p = Y, Zl, Yp at (row, col)
  auto update = [&](float2 v, float kr, float2 y, float2 z, float2 p) {
    if (e.mode == 1) {
      const float kc = kr - cc;
      v.x = alpha * (kc * y.x + z.x + v.x);
      v.y = alpha * (kc * y.y + z.y + v.y);
      if (Yp) {
        v.x -= beta * p.x;
        v.y -= beta * p.y;
      }
    }
    if (e.mode == 2) {
      v.x += z.x;
      v.y += z.y;
    }
    return v;
  };
#pragma unroll
  for (int a = 0; a < AT; ++a)
#pragma unroll
    for (int b = 0; b < BT; ++b) {
      // one 16 x 16 block at a time: no loads hoisted across blocks (bounded register use)
      __builtin_amdgcn_sched_barrier(0);
      const int col = col_base + b * 16 + (lane & 15);
      const int row0 = row_base + a * 16 + 4 * (lane >> 4);
      if (e.vec4 && col < N && row0 + 4 <= M) {
        // the lane's four consecutive rows of one column: 16-byte accesses
        float2 v[4], y[4], z[4], q[4];
        float kr[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < 4; ++r) y[r] = z[r] = q[r] = zero2;
        if (e.mode == 1) {
          const float4 k4 = *reinterpret_cast<const float4*>(kin + row0);
          kr[0] = k4.x;
          kr[1] = k4.y;
          kr[2] = k4.z;
          kr[3] = k4.w;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const float4 yy = reinterpret_cast<const float4*>(Y + (long)col * e.ldy + row0)[h];
            y[2 * h] = make_float2(yy.x, yy.y);
            y[2 * h + 1] = make_float2(yy.z, yy.w);
            if (Yp) {
              const float4 pp = reinterpret_cast<const float4*>(Yp + (long)col * e.ldp + row0)[h];
              q[2 * h] = make_float2(pp.x, pp.y);
              q[2 * h + 1] = make_float2(pp.z, pp.w);
            }
          }
        }
        if (e.mode >= 1) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const float4 zz = reinterpret_cast<const float4*>(Zl + (long)col * e.ldz + row0)[h];
            z[2 * h] = make_float2(zz.x, zz.y);
            z[2 * h + 1] = make_float2(zz.z, zz.w);
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = update(make_float2(cr[a][b][r], ci[a][b][r]), kr[r], y[r], z[r], q[r]);
        float4* oq = reinterpret_cast<float4*>(out + (long)col * ldo + row0);
        oq[0] = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
        oq[1] = make_float4(v[2].x, v[2].y, v[3].x, v[3].y);
        if (e.ph) {
          unsigned int wh[4], wl[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const Split2 sr = split(v[r].x), si = split(v[r].y);
            wh[r] = pack(sr.h, si.h);
            wl[r] = pack(sr.l, si.l);
          }
          const long o = (long)col * e.ldpl + row0;
          *reinterpret_cast<uint4*>(static_cast<unsigned int*>(e.ph) + o) = uint4{wh[0], wh[1], wh[2], wh[3]};
          *reinterpret_cast<uint4*>(static_cast<unsigned int*>(e.pl) + o) = uint4{wl[0], wl[1], wl[2], wl[3]};
        }
        continue;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + r;
        if (row < M && col < N) {
          const bool m1 = e.mode == 1;
          const float2 y = m1 ? Y[(long)col * e.ldy + row] : zero2;
          const float2 z = e.mode >= 1 ? Zl[(long)col * e.ldz + row] : zero2;
          const float2 q = m1 && Yp ? Yp[(long)col * e.ldp + row] : zero2;
          const float2 v = update(make_float2(cr[a][b][r], ci[a][b][r]), m1 ? kin[row] : 0.f, y, z, q);
          out[(long)col * ldo + row] = v;
          if (e.ph) {
            const Split2 sr = split(v.x), si = split(v.y);
            const long o = (long)col * e.ldpl + row;
            static_cast<unsigned int*>(e.ph)[o] = pack(sr.h, si.h);
            static_cast<unsigned int*>(e.pl)[o] = pack(sr.l, si.l);
          }
        }
      }
    }
}


// ------------------------------------------------------------------------------------------
// nn: out = epilogue(A B) (fp32 data, bf16x3 products).
// ------------------------------------------------------------------------------------------
// Each wave owns a WR x (4096 / WR) block of the tile: WR = 64 holds the A fragments and streams
// the B ones; WR = 128 (one wave per 32 columns) holds the B fragments and their (bi, br) forms
// and streams A, so that no two waves of a workgroup form the same (bi, br) words.
template <class AL, class BL, int TM = hTM, int NT = 256, int WR = 64>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_gemm_nn_bf16x3(
    const void* __restrict__ A0, const void* __restrict__ A1, long lda, const void* __restrict__ B0,
    const void* __restrict__ B1, long ldb, int M, int N, int K, int tiles_n, float2* out, long ldo, EpiH e) {
  constexpr int WC = 4096 / WR, AT = WR / 16, BT = WC / 16;
  constexpr int WM = TM / WR, TN = WC * (NT / 64) / WM;
  constexpr int PA = TM * 4, PB = TN * 4;
  __shared__ uint4 sAh[2][PA], sAl[2][PA], sBh[2][PB], sBl[2][PB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int t = xcd_tile16(blockIdx.x, gridDim.x);
  const int tm = t / tiles_n, tn = t - tm * tiles_n;
  const int i0 = tm * TM, j0 = tn * TN;
  const int mo = (wave % WM) * WR, no = (wave / WM) * WC;
  v4f16 cr[AT][BT], ci[AT][BT];
#pragma unroll
  for (int a = 0; a < AT; ++a)
#pragma unroll
    for (int b = 0; b < BT; ++b) cr[a][b] = ci[a][b] = v4f16{0, 0, 0, 0};
  AL la;
  BL lb;  // Br = (br, -bi)
  const int ntiles = (K + hBK - 1) / hBK;
  if (ntiles > 0) {
    la.load(A0, A1, lda, M, i0, 0, K, tid);
    lb.load(B0, B1, ldb, N, j0, 0, K, tid);
    la.store(sAh[0], sAl[0], tid);
    lb.store(sBh[0], sBl[0], tid);
  }
  __syncthreads();
  for (int it = 0; it < ntiles; ++it) {
    const int cur = it & 1;
    const bool more = it + 1 < ntiles;
    if (more) {
      const int kn = (it + 1) * hBK;
      la.load(A0, A1, lda, M, i0, kn, K, tid);
      lb.load(B0, B1, ldb, N, j0, kn, K, tid);
    }
    if constexpr (WR == 64) {
      v8bf ah[AT], al[AT];
#pragma unroll
      for (int a = 0; a < AT; ++a) {
        ah[a] = frag(sAh[cur], mo + a * 16, lane);
        al[a] = frag(sAl[cur], mo + a * 16, lane);
      }
#pragma unroll
      for (int b = 0; b < BT; ++b) {
        const v8bf rh = frag(sBh[cur], no + b * 16, lane);
        const v8bf rl = frag(sBl[cur], no + b * 16, lane);
        const v8bf ih = swapneg_lo(rh), il = swapneg_lo(rl);
#pragma unroll
        for (int a = 0; a < AT; ++a) {
          cr[a][b] = mma16(ah[a], rh, cr[a][b]);
          ci[a][b] = mma16(ah[a], ih, ci[a][b]);
          cr[a][b] = mma16(ah[a], rl, cr[a][b]);
          ci[a][b] = mma16(ah[a], il, ci[a][b]);
          cr[a][b] = mma16(al[a], rh, cr[a][b]);
          ci[a][b] = mma16(al[a], ih, ci[a][b]);
        }
      }
    } else {
      v8bf rh[BT], rl[BT], ih[BT], il[BT];
#pragma unroll
      for (int b = 0; b < BT; ++b) {
        rh[b] = frag(sBh[cur], no + b * 16, lane);
        rl[b] = frag(sBl[cur], no + b * 16, lane);
        ih[b] = swapneg_lo(rh[b]);
        il[b] = swapneg_lo(rl[b]);
      }
#pragma unroll
      for (int a = 0; a < AT; ++a) {
        const v8bf ah = frag(sAh[cur], mo + a * 16, lane);
        const v8bf al = frag(sAl[cur], mo + a * 16, lane);
#pragma unroll
        for (int b = 0; b < BT; ++b) {
          cr[a][b] = mma16(ah, rh[b], cr[a][b]);
          ci[a][b] = mma16(ah, ih[b], ci[a][b]);
          cr[a][b] = mma16(ah, rl[b], cr[a][b]);
          ci[a][b] = mma16(ah, il[b], ci[a][b]);
          cr[a][b] = mma16(al, rh[b], cr[a][b]);
          ci[a][b] = mma16(al, ih[b], ci[a][b]);
        }
      }
    }
    if (more) {
      la.store(sAh[cur ^ 1], sAl[cur ^ 1], tid);
      lb.store(sBh[cur ^ 1], sBl[cur ^ 1], tid);
    }
    __syncthreads();
  }
  epi_tile<AT, BT>(cr, ci, i0 + mo, j0 + no, lane, M, N, out, ldo, e);
}

// ------------------------------------------------------------------------------------------
// Pipelined nn form on pre-split planes (the nonlocal product and the rotations).  Operand tiles
// go from global memory straight into LDS (the direct global-to-LDS loads of gfx950, 16 bytes per
// lane), three K tiles of 256 x 128 in a ring, so a tile's loads have two tiles of MFMA work to
// arrive in.  One workgroup per CU (the ring takes 149 KB of LDS).  NW = 8 waves of 64 x 64
// (two per SIMD, which hide each other's LDS reads) or NW = 4 waves of 128 x 64 (one per SIMD,
// the next tile's fragments read into registers while the current ones are used).
//   B (K-contiguous planes, the D P or coefficient words): lane i of a load of 16 columns fetches
//     chunk (column, slot) with slot = i / 16 and column = (i % 16) ^ slot, so the LDS image is
//     the chunk layout of chunk_of() and fragments are read lane-linearly without bank conflicts.
//   A (M-contiguous planes, the projector or block words): one load per (plane, k) copies 256
//     consecutive rows (1 KB) into a row of 260 words; a fragment is four 32-bit reads (k = 4 (l / 16)
//     + j for row l % 16), whose four lane groups fall 16 banks apart.
// Rows and columns beyond the operands are clamped to the last ones (their results are dropped;
// pipe_addr.hpp holds the arithmetic, checked by a host test over every load).
// ------------------------------------------------------------------------------------------
constexpr int pTM = 256, pTN = 128, pST = 3;
constexpr int pApitch = 260;                       // words per (plane, k) row of the A tile
constexpr int pAbytes = 2 * hBK * pApitch * 4;     // 33,280 B
constexpr int pBbytes = 2 * pTN * hBK * 4;         // 16,384 B
constexpr int pStage = pAbytes + pBbytes;

__device__ __forceinline__ void dma16(const unsigned int* g, void* l) {
  __builtin_amdgcn_global_load_lds(g, l, 16, 0, 0);
}
// s_waitcnt vmcnt(N) alone (expcnt and lgkmcnt left at their maxima)
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}
__device__ __forceinline__ void wait_lds() { __builtin_amdgcn_s_waitcnt(0xc07f); }  // lgkmcnt(0)

// Address of the 16 bytes a lane loads: a wave-uniform base plus a per-lane 32-bit byte offset.
__device__ __forceinline__ const unsigned int* at_off(const unsigned int* base, unsigned int byte_off) {
  return reinterpret_cast<const unsigned int*>(reinterpret_cast<const unsigned char*>(base) + byte_off);
}

// K-contiguous tile: NC columns x 16 k, hi and lo planes, 2 NC / 16 loads of 1 KB (16 columns
// each), this wave issuing those with index wave, wave + NW, ...  (the B tile, and the A tile of
// the cn form).  The columns a lane loads are the same for every K tile; off[q] is computed once.
template <int NC, int NW>
struct KTile {
  static constexpr int G = NC / 16, Q = 2 * G / NW;
  unsigned int off[Q];
  __device__ __forceinline__ void offsets(long ld, int c0, int ncols, int wave, int lane) {
#pragma unroll
    for (int q = 0; q < Q; ++q) off[q] = pipe_koff_bytes(c0, (wave + NW * q) % G, ncols, ld, lane);
  }
  __device__ __forceinline__ void load(const unsigned int* __restrict__ H, const unsigned int* __restrict__ L, long ld,
                                       int c0, int ncols, int k0, unsigned char* dst, int wave) const {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int j = wave + NW * q, pl = j / G, g = j % G;
      const unsigned int* base = (pl ? L : H) + (long)pipe_kbase_col(c0, g, ncols) * ld + k0;
      dma16(at_off(base, off[q]), dst + (pl * G + g) * 1024);
    }
  }
};
// M-contiguous A tile (nn form): 256 rows x 16 k, hi and lo planes, 32 loads of 1 KB (one per
// plane and k).
template <int NW>
struct ATile {
  static constexpr int Q = 32 / NW;
  unsigned int off;
  __device__ __forceinline__ void offsets(long ld, int r0, int lane) { off = pipe_moff_bytes(ld, r0, lane); }
  __device__ __forceinline__ void load(const unsigned int* __restrict__ H, const unsigned int* __restrict__ L, long ld,
                                       int r0, int k0, unsigned char* dst, int wave) const {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int j = wave + NW * q, pl = j >> 4, k = j & 15;
      const unsigned int* base = (pl ? L : H) + (long)(k0 + k) * ld + r0;
      dma16(at_off(base, off), dst + (pl * 16 + k) * (pApitch * 4));
    }
  }
};

// A fragment (rows ra .. ra + 15 of the tile) from the A tile plane.
__device__ __forceinline__ v8bf frag_m(const unsigned int* plane, int ra, int lane) {
  const int row = ra + (lane & 15), kg = lane >> 4;
  uint4 u;
  u.x = plane[(4 * kg + 0) * pApitch + row];
  u.y = plane[(4 * kg + 1) * pApitch + row];
  u.z = plane[(4 * kg + 2) * pApitch + row];
  u.w = plane[(4 * kg + 3) * pApitch + row];
  return __builtin_bit_cast(v8bf, u);
}

// The fragments a wave needs from one K tile: AT A blocks and 4 B blocks, hi and lo.  CN: the cn
// form (A tile in the chunk layout, AB bytes of A before the B tile), else the nn form.
template <int AT, bool CN>
struct TileFrags {
  static constexpr int AB = CN ? 2 * pTM * hBK * 4 : pAbytes;
  v8bf ah[AT], al[AT], bh[4], bl[4];
  __device__ __forceinline__ void read(const unsigned char* st, int ra0, int cb0, int lane) {
    const uint4* Bh = reinterpret_cast<const uint4*>(st + AB);
    const uint4* Bl = Bh + pTN * 4;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      bh[b] = frag(Bh, cb0 + b * 16, lane);
      bl[b] = frag(Bl, cb0 + b * 16, lane);
    }
#pragma unroll
    for (int a = 0; a < AT; ++a) {
      if constexpr (CN) {
        const uint4* Ah = reinterpret_cast<const uint4*>(st);
        ah[a] = frag(Ah, ra0 + a * 16, lane);
        al[a] = frag(Ah + pTM * 4, ra0 + a * 16, lane);
      } else {
        const unsigned int* Ah = reinterpret_cast<const unsigned int*>(st);
        ah[a] = frag_m(Ah, ra0 + a * 16, lane);
        al[a] = frag_m(Ah + hBK * pApitch, ra0 + a * 16, lane);
      }
    }
  }
  // Re C += A' B, Im C += A'' B with the A words rotated (only the B fragments stay in registers
  // across the blocks):
  //   nn  C = A B:    A'' = (ai, -ar), B as stored (br, -bi)
  //   cn  C = A^H B:  A'' = (-ai, ar), B as stored (br, bi)
  template <int NTERM>
  __device__ __forceinline__ void mfma(v4f16 (&cr)[AT][4], v4f16 (&ci)[AT][4]) const {
#pragma unroll
    for (int a = 0; a < AT; ++a) {
      const v8bf h = ah[a], l = al[a];
      const v8bf h2 = CN ? swapneg_lo(h) : swapneg_hi(h);
      const v8bf l2 = CN ? swapneg_lo(l) : swapneg_hi(l);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        cr[a][b] = mma16(h, bh[b], cr[a][b]);
        ci[a][b] = mma16(h2, bh[b], ci[a][b]);
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        cr[a][b] = mma16(h, bl[b], cr[a][b]);
        ci[a][b] = mma16(h2, bl[b], ci[a][b]);
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        cr[a][b] = mma16(l, bh[b], cr[a][b]);
        ci[a][b] = mma16(l2, bh[b], ci[a][b]);
      }
      if constexpr (NTERM == 4) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          cr[a][b] = mma16(l, bl[b], cr[a][b]);
          ci[a][b] = mma16(l2, bl[b], ci[a][b]);
        }
      }
    }
  }
};

// out = epilogue(A B), A M-contiguous planes (lda words per k), B K-contiguous (br, -bi) planes
// (ldb words per column).  K a multiple of 16.
template <int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW / 4, NW / 4))) void k_gemm_nn_pipe(
    const unsigned int* __restrict__ Ah, const unsigned int* __restrict__ Al, long lda,
    const unsigned int* __restrict__ Bh, const unsigned int* __restrict__ Bl, long ldb, int M, int N, int K,
    int tiles_n, float2* out, long ldo, EpiH e) {
  constexpr int WM = NW / 2, RT = pTM / WM, AT = RT / 16;  // waves along M, rows per wave
  constexpr int LPW = ATile<NW>::Q + KTile<pTN, NW>::Q;    // direct loads per wave per K tile
  constexpr bool DB = NW == 4;                             // fragments double-buffered in registers
  __shared__ __align__(16) unsigned char smem[pST * pStage];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int t = xcd_tile16(blockIdx.x, gridDim.x);
  const int tm = t / tiles_n, tn = t - tm * tiles_n;
  const int i0 = tm * pTM, j0 = tn * pTN;
  const int wm = wave % WM, wn = wave / WM;
  const int ra0 = wm * RT, cb0 = wn * 64;
  v4f16 cr[AT][4], ci[AT][4];
#pragma unroll
  for (int a = 0; a < AT; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) cr[a][b] = ci[a][b] = v4f16{0, 0, 0, 0};
  const int ntiles = K / hBK;
  ATile<NW> ta;
  KTile<pTN, NW> tb;
  ta.offsets(lda, i0, lane);
  tb.offsets(ldb, j0, N, wave, lane);
  auto issue = [&](int kt) {
    unsigned char* st = smem + (kt % pST) * pStage;
    ta.load(Ah, Al, lda, i0, kt * hBK, st, wave);
    tb.load(Bh, Bl, ldb, j0, N, kt * hBK, st + pAbytes, wave);
  };
  if constexpr (DB) {
    // Iteration it: wait for tile it + 1, barrier (every wave has read tile it into registers, so
    // its stage is free), issue tile it + 3 into it, read tile it + 1's fragments, then run tile
    // it's MFMAs while those reads land.
    for (int p = 0; p < pST && p < ntiles; ++p) issue(p);
    TileFrags<AT, false> cur, nxt;
    if (ntiles > 0) {
      if (ntiles > 2) wait_vm<2 * LPW>();
      else if (ntiles > 1) wait_vm<LPW>();
      else wait_vm<0>();
      __builtin_amdgcn_s_barrier();
      cur.read(smem, ra0, cb0, lane);
    }
    for (int it = 0; it < ntiles; ++it) {
      const bool more = it + 1 < ntiles;
      if (more) {
        if (it + 2 < ntiles) wait_vm<LPW>();
        else wait_vm<0>();
        wait_lds();
        __builtin_amdgcn_s_barrier();
        if (it + 3 < ntiles) issue(it + 3);
        nxt.read(smem + ((it + 1) % pST) * pStage, ra0, cb0, lane);
      }
      cur.template mfma<3>(cr, ci);
      if (more) cur = nxt;
    }
  } else {
    // Iteration it: wait for tile it (tile it + 1 may be in flight), barrier (every wave is done
    // with tile it - 1), issue tile it + 2 into tile it - 1's stage, read and use tile it.
    if (ntiles > 0) issue(0);
    if (ntiles > 1) issue(1);
    for (int it = 0; it < ntiles; ++it) {
      if (it + 1 < ntiles) wait_vm<LPW>();
      else wait_vm<0>();
      wait_lds();
      __builtin_amdgcn_s_barrier();
      if (it + 2 < ntiles) issue(it + 2);
      TileFrags<AT, false> f;
      f.read(smem + (it % pST) * pStage, ra0, cb0, lane);
      f.template mfma<3>(cr, ci);
    }
  }
  epi_tile<AT, 4>(cr, ci, i0 + ra0, j0 + cb0, lane, M, N, out, ldo, e);
}

// cn on planes, pipelined like the nn form: part[s] = A^H B over K chunk s, A (256-column tiles)
// and B (128-column tiles) both K-contiguous planes, NW = 8 waves of 64 x 64; fp32 accumulation
// moved to the fp64 partial every hFlush tiles (one owner per partial entry, no atomics).  The K
// range is covered by whole tiles of 16: the words of each column from K up to its leading
// dimension must be zero in both operands (the launcher checks that the leading dimensions reach
// K rounded up to 16; the planes this library writes hold zeros there).
// herm > 0: the first herm columns of B are A itself (a Gram matrix A^H A in them); tiles of those
// columns that lie wholly below the diagonal are not computed (their partials are left as they
// are: the caller takes that block from its upper triangle).
template <int NTERM>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_gemm_cn_pipe(
    const unsigned int* __restrict__ Ah, const unsigned int* __restrict__ Al, long lda,
    const unsigned int* __restrict__ Bh, const unsigned int* __restrict__ Bl, long ldb, int M, int N, int K,
    int kchunk, int tiles_m, int tiles_n, double2* __restrict__ part, int herm) {
  constexpr int NW = 8, AT = 4;
  constexpr int AB = TileFrags<AT, true>::AB, SB = AB + pBbytes;
  constexpr int LPW = KTile<pTM, NW>::Q + KTile<pTN, NW>::Q;
  __shared__ __align__(16) unsigned char smem[pST * SB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int t = xcd_tile16(blockIdx.x, gridDim.x);
  const int sp = t / (tiles_m * tiles_n);
  const int tr = t - sp * tiles_m * tiles_n;
  const int tm = tr / tiles_n, tn = tr - tm * tiles_n;
  const int i0 = tm * pTM, j0 = tn * pTN;
  if (j0 + pTN <= herm && i0 > j0 + pTN - 1) return;  // strictly lower tile of the Gram block
  const int kb = sp * kchunk, ke = min(K, kb + kchunk);
  const int ra0 = (wave & 3) * 64, cb0 = (wave >> 2) * 64;
  const int ntiles = ke > kb ? (ke - kb + hBK - 1) / hBK : 0;
  KTile<pTM, NW> ta;
  KTile<pTN, NW> tb;
  ta.offsets(lda, i0, M, wave, lane);
  tb.offsets(ldb, j0, N, wave, lane);
  auto issue = [&](int kt) {
    unsigned char* st = smem + (kt % pST) * SB;
    const int k0 = kb + kt * hBK;
    ta.load(Ah, Al, lda, i0, M, k0, st, wave);
    tb.load(Bh, Bl, ldb, j0, N, k0, st + AB, wave);
  };
  if (ntiles > 0) issue(0);
  if (ntiles > 1) issue(1);
  v4f16 cr[AT][4], ci[AT][4];
  bool stored = false;
  int it = 0;
  do {
    const int fend = min(ntiles, it + hFlush);
#pragma unroll
    for (int a = 0; a < AT; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) cr[a][b] = ci[a][b] = v4f16{0, 0, 0, 0};
    for (; it < fend; ++it) {
      // tile it has landed (tile it + 1 may be in flight); every wave is done with tile it - 1,
      // whose stage receives tile it + 2
      if (it + 1 < ntiles) wait_vm<LPW>();
      else wait_vm<0>();
      wait_lds();
      __builtin_amdgcn_s_barrier();
      if (it + 2 < ntiles) issue(it + 2);
      TileFrags<AT, true> f;
      f.read(smem + (it % pST) * SB, ra0, cb0, lane);
      f.template mfma<NTERM>(cr, ci);
    }
#pragma unroll
    for (int a = 0; a < AT; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int col = j0 + cb0 + b * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = i0 + ra0 + a * 16 + 4 * (lane >> 4) + r;
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

// Zero words [r0, ld) of each of cols columns of a pair of planes (the padding the pipelined cn
// form reads past the last row).
__global__ void k_zero_plane_rows(unsigned int* __restrict__ H, unsigned int* __restrict__ L, long ld, int r0,
                                  int cols) {
  const long pad = ld - r0;
  PW_GRID_STRIDE(idx, pad * cols) {
    const long c = idx / pad, r = r0 + (idx - c * pad);
    H[c * ld + r] = 0u;
    L[c * ld + r] = 0u;
  }
}

hipError_t launch_zero_plane_rows(unsigned int* H, unsigned int* L, long ld, int r0, int cols, hipStream_t s) {
  const long n = (ld - r0) * (long)cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_plane_rows, dim3(stride_blocks(n)), dim3(256), 0, s, H, L, ld, r0, cols);
  return hipGetLastError();
}

// hi/lo planes of fp32 complex columns: word (re, im) of bf16(x) and of bf16(x - hi).
__global__ void k_split_planes(const float2* __restrict__ X, long ldx, int rows, int cols, unsigned int* __restrict__ H,
                               unsigned int* __restrict__ L, long ldp) {
  PW_GRID_STRIDE(idx, (long)rows * cols) {
    const int j = (int)(idx / rows), i = (int)(idx - (long)j * rows);
    const float2 v = X[(long)j * ldx + i];
    const Split2 sr = split(v.x), si = split(v.y);
    H[(long)j * ldp + i] = pack(sr.h, si.h);
    L[(long)j * ldp + i] = pack(sr.l, si.l);
  }
}

hipError_t launch_split_planes(const float2* X, long ldx, int rows, int cols, unsigned int* H, unsigned int* L,
                               long ldp, hipStream_t s) {
  const long n = (long)rows * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_split_planes, dim3(stride_blocks(n)), dim3(256), 0, s, X, ldx, rows, cols, H, L, ldp);
  return hipGetLastError();
}

// Sum of the split-K partials, scaled per row by dscale[i % dper], rounded to fp32 and stored as the
// nn B operand's planes: words (re, -im) of bf16(x) and of bf16(x - hi), k = row contiguous.
__global__ void k_reduce_planes(const double2* __restrict__ part, int nsplit, int M, int N,
                                const double* __restrict__ dscale, int dper, unsigned int* __restrict__ H,
                                unsigned int* __restrict__ L, long ldp) {
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
    const float re = (float)s.x, im = (float)s.y;
    const Split2 sr = split(re), si = split(-im);
    H[(long)j * ldp + i] = pack(sr.h, si.h);
    L[(long)j * ldp + i] = pack(sr.l, si.l);
  }
}

hipError_t launch_reduce_planes(const double2* part, int nsplit, int M, int N, const double* dscale, int dper,
                                unsigned int* H, unsigned int* L, long ldp, hipStream_t s) {
  const long n = (long)M * N;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_planes, dim3(stride_blocks(n)), dim3(256), 0, s, part, nsplit, M, N, dscale,
                     dper > 0 ? dper : 1, H, L, ldp);
  return hipGetLastError();
}

// n x n FP64 coefficients (columns optionally scaled by sc * lam[j]) as the nn B planes: rounded to
// fp32, then words (re, -im) of bf16(x) and bf16(x - hi).
__global__ void k_coef_planes(const double2* __restrict__ C, long ldc, int n, const double* __restrict__ lam,
                              double sc, unsigned int* __restrict__ H, unsigned int* __restrict__ L, long ldp) {
  PW_GRID_STRIDE(idx, (long)n * n) {
    const int j = (int)(idx / n), i = (int)(idx - (long)j * n);
    const double2 v = C[(long)j * ldc + i];
    const double f = lam ? sc * lam[j] : 1.0;
    const float re = (float)(f * v.x), im = (float)(f * v.y);
    const Split2 sr = split(re), si = split(-im);
    H[(long)j * ldp + i] = pack(sr.h, si.h);
    L[(long)j * ldp + i] = pack(sr.l, si.l);
  }
}

hipError_t launch_coef_planes(const double2* C, long ldc, int n, const double* lam, double sc, unsigned int* H,
                              unsigned int* L, long ldp, hipStream_t s) {
  const long m = (long)n * n;
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_coef_planes, dim3(stride_blocks(m)), dim3(256), 0, s, C, ldc, n, lam, sc, H, L, ldp);
  return hipGetLastError();
}

// Whether every array of the nn epilogue allows 16-byte accesses of a lane's four rows (row0 a
// multiple of 4): 16-byte aligned bases, even complex leading dimensions, planes' a multiple of 4.
static EpiH epi_vec4(const EpiH& e, const void* out, long ldo) {
  auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  bool ok = al(out) && ldo % 2 == 0;
  if (e.mode >= 1) ok = ok && al(e.Zl) && e.ldz % 2 == 0;
  if (e.mode == 1) ok = ok && al(e.kin) && al(e.Y) && e.ldy % 2 == 0 && (!e.Yp || (al(e.Yp) && e.ldp % 2 == 0));
  if (e.ph) ok = ok && al(e.ph) && al(e.pl) && e.ldpl % 4 == 0;
  EpiH r = e;
  r.vec4 = ok ? 1 : 0;
  return r;
}

static inline bool ok16(const void* p, long ld) {
  return (reinterpret_cast<uintptr_t>(p) & 15) == 0 && (ld % 2) == 0;
}
static inline bool ok_planes(const void* h, const void* l, long lda) {
  return (reinterpret_cast<uintptr_t>(h) & 15) == 0 && (reinterpret_cast<uintptr_t>(l) & 15) == 0 && (lda % 4) == 0;
}

int gemm_cn_bf16_tiles(int M, int N) { return ceil_div(M, hTM) * ceil_div(N, hTN); }

static int cn_chunk(int K, int nsplit) {
  int kchunk = ceil_div(K, nsplit);
  kchunk = ceil_div(kchunk, hBK) * hBK;
  return kchunk > 0 ? kchunk : hBK;
}

hipError_t launch_gemm_cn_bf16x3(const float2* A, long lda, const float2* B, long ldb, const float2* B2, long ldb2,
                                 int ncol1, int M, int N, int K, int nsplit, double2* part, int nterm, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int kchunk = cn_chunk(K, nsplit);
  const int tm = ceil_div(M, hTM), tn = ceil_div(N, hTN);
  const float2* b2 = B2 ? B2 : B;
  const long l2 = B2 ? ldb2 : ldb;
  const bool vec = ok16(A, lda) && ok16(B, ldb) && ok16(b2, l2);
  dim3 grid(tm * tn * nsplit);
  const void* a0 = A;
  const void* b0 = B;
  const void* bb = b2;
  const void* nul = nullptr;
#define PW_CN16(V, NT)                                                                                             \
  hipLaunchKernelGGL((k_gemm_cn_bf16x3<NT, CnAF32<hTM, V>, CnBF32<hTN, V>>), grid, dim3(256), 0, s, a0, nul, lda, \
                     b0, nul, ldb, bb, l2, ncol1, M, N, K, kchunk, tm, tn, part)
  if (nterm == 4) {
    if (vec) PW_CN16(true, 4); else PW_CN16(false, 4);
  } else {
    if (vec) PW_CN16(true, 3); else PW_CN16(false, 3);
  }
#undef PW_CN16
  return hipGetLastError();
}

// The projection with pre-split planes uses a 256-row tile with 8 waves when M is large: the block
// is then re-read by half as many workgroups.  (The nonlocal product, whose K is short, keeps two
// 128 x 128 workgroups per CU, which overlap one's epilogue with the other's MFMAs.)
constexpr int hWM = 256, hWT = 512;
// wave tile rows of the nonlocal product on planes
constexpr int hNnWR = 128;
static bool planes_wide(int M) { return M >= 512; }

int gemm_cn_bf16_planes_tiles(int M, int N) {
  return planes_wide(M) ? ceil_div(M, hWM) * ceil_div(N, hTN) : gemm_cn_bf16_tiles(M, N);
}


// The pipelined forms need 16-byte aligned planes with leading dimensions a multiple of 4 words,
// and enough work to fill the chip with 256 x 128 tiles.
constexpr int kPipeWaves = 8;
static bool use_pipe(const void* a, const void* a2, long lda, const void* b, const void* b2, long ldb, long M,
                     long N) {
  return ok_planes(a, a2, lda) && ok_planes(b, b2, ldb) && lda >= 4 && ldb >= 4 && M * N >= (1L << 20);
}

hipError_t launch_gemm_cn_bf16x3_planes(const unsigned int* Ahi, const unsigned int* Alo, long lda,
                                        const unsigned int* Bhi, const unsigned int* Blo, long ldb, int M, int N, int K,
                                        int nsplit, double2* part, hipStream_t s, int nterm, int herm_cols) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int kchunk = cn_chunk(K, nsplit);
  const long kpad = (long)ceil_div(K, hBK) * hBK;  // the last tile reads the zero words up to here
  if (kpad <= lda && kpad <= ldb && use_pipe(Ahi, Alo, lda, Bhi, Blo, ldb, M, N)) {
    const int tm = ceil_div(M, pTM), tn = ceil_div(N, pTN);
    dim3 grid(tm * tn * nsplit);
    if (nterm == 4)
      hipLaunchKernelGGL(k_gemm_cn_pipe<4>, grid, dim3(512), 0, s, Ahi, Alo, lda, Bhi, Blo, ldb, M, N, K, kchunk, tm,
                         tn, part, herm_cols);
    else
      hipLaunchKernelGGL(k_gemm_cn_pipe<3>, grid, dim3(512), 0, s, Ahi, Alo, lda, Bhi, Blo, ldb, M, N, K, kchunk, tm,
                         tn, part, herm_cols);
    return hipGetLastError();
  }
  const bool vec = ok_planes(Ahi, Alo, lda) && ok_planes(Bhi, Blo, ldb);
  const void* a0 = Ahi;
  const void* a1 = Alo;
  const void* b0 = Bhi;
  const void* b1 = Blo;
  const void* nul = nullptr;
#define PW_CNP(NTERM, V, TM, NT)                                                                                  \
  hipLaunchKernelGGL((k_gemm_cn_bf16x3<NTERM, CnAPlanes<TM, V, NT>, CnBPlanes<hTN, V, NT>, TM, NT>), grid, dim3(NT), \
                     0, s, a0, a1, lda, b0, b1, ldb, nul, 0L, N, M, N, K, kchunk, tm, tn, part)
  if (planes_wide(M)) {
    const int tm = ceil_div(M, hWM), tn = ceil_div(N, hTN);
    dim3 grid(tm * tn * nsplit);
    if (nterm == 4) {
      if (vec) PW_CNP(4, true, hWM, hWT); else PW_CNP(4, false, hWM, hWT);
    } else {
      if (vec) PW_CNP(3, true, hWM, hWT); else PW_CNP(3, false, hWM, hWT);
    }
    return hipGetLastError();
  }
  const int tm = ceil_div(M, hTM), tn = ceil_div(N, hTN);
  dim3 grid(tm * tn * nsplit);
  if (nterm == 4) {
    if (vec) PW_CNP(4, true, hTM, 256); else PW_CNP(4, false, hTM, 256);
  } else {
    if (vec) PW_CNP(3, true, hTM, 256); else PW_CNP(3, false, hTM, 256);
  }
#undef PW_CNP
  return hipGetLastError();
}

hipError_t launch_gemm_nn_bf16x3(const float2* A, long lda, const float2* B, long ldb, int M, int N, int K,
                                 float2* out, long ldo, const EpiH& e, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const EpiH ev = epi_vec4(e, out, ldo);
  const int tm = ceil_div(M, hTM), tn = ceil_div(N, hTN);
  const bool vec = ok16(A, lda);
  dim3 grid(tm * tn);
  const void* a0 = A;
  const void* a1 = nullptr;
  const void* b0 = B;
  if (vec)
    hipLaunchKernelGGL((k_gemm_nn_bf16x3<NnAF32<hTM, true>, NnBF32<hTN>>), grid, dim3(256), 0, s, a0, a1, lda, b0,
                       a1, ldb, M, N, K, tn, out, ldo, ev);
  else
    hipLaunchKernelGGL((k_gemm_nn_bf16x3<NnAF32<hTM, false>, NnBF32<hTN>>), grid, dim3(256), 0, s, a0, a1, lda, b0,
                       a1, ldb, M, N, K, tn, out, ldo, ev);
  return hipGetLastError();
}

hipError_t launch_gemm_nn_bf16x3_bplanes(const float2* A, long lda, const unsigned int* Bhi, const unsigned int* Blo,
                                         long ldb, int M, int N, int K, float2* out, long ldo, const EpiH& e,
                                         hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const EpiH ev = epi_vec4(e, out, ldo);
  const int tm = ceil_div(M, hTM), tn = ceil_div(N, hTN);
  const bool vec = ok16(A, lda) && ok_planes(Bhi, Blo, ldb);
  dim3 grid(tm * tn);
  const void* a0 = A;
  const void* a1 = nullptr;
  const void* b0 = Bhi;
  const void* b1 = Blo;
  if (vec)
    hipLaunchKernelGGL((k_gemm_nn_bf16x3<NnAF32<hTM, true>, NnBPlanes<hTN, true>>), grid, dim3(256), 0, s, a0, a1,
                       lda, b0, b1, ldb, M, N, K, tn, out, ldo, ev);
  else
    hipLaunchKernelGGL((k_gemm_nn_bf16x3<NnAF32<hTM, false>, NnBPlanes<hTN, false>>), grid, dim3(256), 0, s, a0, a1,
                       lda, b0, b1, ldb, M, N, K, tn, out, ldo, ev);
  return hipGetLastError();
}

hipError_t launch_gemm_nn_bf16x3_planes(const unsigned int* Ahi, const unsigned int* Alo, long lda,
                                        const unsigned int* Bhi, const unsigned int* Blo, long ldb, int M, int N, int K,
                                        float2* out, long ldo, const EpiH& e, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const EpiH ev = epi_vec4(e, out, ldo);
  if (K % hBK == 0 && K > 0 && lda >= M && use_pipe(Ahi, Alo, lda, Bhi, Blo, ldb, M, N)) {
    const int tm = ceil_div(M, pTM), tn = ceil_div(N, pTN);
    hipLaunchKernelGGL(k_gemm_nn_pipe<kPipeWaves>, dim3(tm * tn), dim3(64 * kPipeWaves), 0, s, Ahi, Alo, lda, Bhi, Blo,
                       ldb, M, N, K, tn, out, ldo, ev);
    return hipGetLastError();
  }
  const int tm = ceil_div(M, hTM), tn = ceil_div(N, hTN);
  const bool vec = ok_planes(Ahi, Alo, lda) && ok_planes(Bhi, Blo, ldb);
  dim3 grid(tm * tn);
  const void* a0 = Ahi;
  const void* a1 = Alo;
  const void* b0 = Bhi;
  const void* b1 = Blo;
  if (vec)
    hipLaunchKernelGGL((k_gemm_nn_bf16x3<NnAPlanes<hTM, true>, NnBPlanes<hTN, true>, hTM, 256, hNnWR>), grid, dim3(256),
                       0, s, a0, a1, lda, b0, b1, ldb, M, N, K, tn, out, ldo, ev);
  else
    hipLaunchKernelGGL((k_gemm_nn_bf16x3<NnAPlanes<hTM, false>, NnBPlanes<hTN, false>, hTM, 256, hNnWR>), grid,
                       dim3(256), 0, s, a0, a1, lda, b0, b1, ldb, M, N, K, tn, out, ldo, ev);
  return hipGetLastError();
}

}  // namespace pw
