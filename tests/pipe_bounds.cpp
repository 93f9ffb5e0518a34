// Host-side bounds test of the direct global-to-LDS loads of the pipelined split-bf16 GEMMs: for a
// GEMM shape it enumerates every load of the first and the last K tile of every workgroup tile
// (addresses are affine in the K tile, so these bound all others) with the kernels' own address
// arithmetic (pipe_addr.hpp), and checks that each 16-byte load lies inside its operand.
// Usage: pipe_bounds nn M N K lda ldb | pipe_bounds cn M N K lda ldb nsplit
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>

#define __host__
#define __device__
#include "../paper_2406_10765_amd/csrc/pipe_addr.hpp"

using namespace pw;

static long bad = 0, checked = 0;

static void check(long word, long lo, long hi, const char* what) {
  ++checked;
  if (word < lo || word + 3 >= hi) {
    if (bad < 5) std::printf("out of bounds: %s word %ld not in [%ld, %ld)\n", what, word, lo, hi);
    ++bad;
  }
}

// K-contiguous tile of NC columns: every lane of every wave, both planes (same arithmetic).
static void ktile(int NC, int c0, int ncols, long ld, int k0, long colwords_limit) {
  const int G = NC / 16, Q = 2 * G / 4;
  for (int wave = 0; wave < 4; ++wave)
    for (int q = 0; q < Q; ++q) {
      const int g = (wave + 4 * q) % G;
      for (int lane = 0; lane < 64; ++lane) {
        const long word = (long)pipe_kbase_col(c0, g, ncols) * ld + k0 + pipe_koff_bytes(c0, g, ncols, ld, lane) / 4;
        check(word, 0, (long)ncols * ld, "K-contiguous operand");
        // and inside its own column (the K tile never runs past the column's padded length)
        const long col = word / ld, inword = word - col * ld;
        check(inword, 0, colwords_limit, "column");
      }
    }
}

int main(int argc, char** argv) {
  if (argc < 7) return 2;
  const bool nn = std::strcmp(argv[1], "nn") == 0;
  const int M = std::atoi(argv[2]), N = std::atoi(argv[3]), K = std::atoi(argv[4]);
  const long lda = std::atol(argv[5]), ldb = std::atol(argv[6]);
  const int TM = 256, TN = 128;
  const int tm = (M + TM - 1) / TM, tn = (N + TN - 1) / TN;
  if (nn) {
    const int ntiles = K / 16;
    for (int a = 0; a < tm; ++a)
      for (int b = 0; b < tn; ++b)
        for (int kt : {0, ntiles - 1}) {
          const int k0 = kt * 16, r0 = a * TM;
          for (int wave = 0; wave < 4; ++wave)
            for (int q = 0; q < 8; ++q) {
              const int k = (wave + 4 * q) & 15;
              for (int lane = 0; lane < 64; ++lane)
                check((long)(k0 + k) * lda + r0 + pipe_moff_bytes(lda, r0, lane) / 4, 0, lda * K,
                      "M-contiguous operand");
            }
          ktile(TN, b * TN, N, ldb, k0, ldb);
        }
  } else {
    const int nsplit = argc > 7 ? std::atoi(argv[7]) : 1;
    int kchunk = (K + nsplit - 1) / nsplit;
    kchunk = (kchunk + 15) / 16 * 16;
    for (int sp = 0; sp < nsplit; ++sp) {
      const int kb = sp * kchunk, ke = kb + kchunk < K ? kb + kchunk : K;
      if (ke <= kb) continue;
      const int ntiles = (ke - kb + 15) / 16;
      for (int a = 0; a < tm; ++a)
        for (int b = 0; b < tn; ++b)
          for (int kt : {0, ntiles - 1}) {
            const int k0 = kb + kt * 16;
            ktile(TM, a * TM, M, lda, k0, lda);
            ktile(TN, b * TN, N, ldb, k0, ldb);
          }
    }
  }
  std::printf("%s M=%d N=%d K=%d: %ld loads checked, %ld out of bounds\n", argv[1], M, N, K, checked, bad);
  return bad ? 1 : 0;
}
