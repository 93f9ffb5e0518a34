// Handle, setup, H application, one block-eigensolver step and the C ABI.
//
// One step (pw_eig_step) follows the structure of the inner eigensolver of
// Section II-A and the subspace products of Section II-B:
//   filter:   Y = p_m(H) X with the scaled three-term Chebyshev recurrence,
//             every degree one H application whose last GEMM writes the update
//   project:  W = H Y; [S | H_s] = Y^H [Y | W] in one split-K GEMM
//   solve:    FP64 generalised Hermitian eigensolve: Cholesky of S, reduction to standard
//             form by two triangular solves, Hermitian eigensolve, back-substitution
//             (rocSOLVER/rocBLAS), the one-device analogue of the Syevd of Section III-D
//   rotate:   X' = Y C, W' = W C; residual norms ||W'_i - lambda_i X'_i||
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <new>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/pw.h"
#include "kernels.hpp"
#include "slots.hpp"
#include "plan.hpp"

using namespace pw;

static thread_local std::string g_last_error;

// Work array of pw_apply_h_noalloc, for callers that cannot allocate device memory.  Each device
// the library runs on holds its own copy for the life of the process; host code reaches it only
// through the device address hipGetSymbolAddress returns (kept per device below), never through
// the array's name.
constexpr size_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char* g_scratch[kMaxDevices] = {};

// Device address of this device's work array (the device must be current); null on failure.
static unsigned char* scratch_address(int dev, std::string* err) {
  if (dev < 0 || dev >= kMaxDevices) {
    *err = "device ordinal beyond the library's table";
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch[dev] = static_cast<unsigned char*>(ptr);
  }
  return g_scratch[dev];
}

struct pw_handle_s {
  Plan plan;
  unsigned char* arena = nullptr;
  size_t arena_bytes = 0;
  hipStream_t stream = nullptr;
  rocblas_handle blas = nullptr;
  int device = 0;
  size_t max_lds = kDefaultMaxLds;
  std::string err;
  double bmax_cached = NAN;
  // lambda_1 and lambda_nb of the last successful pw_eig_step on this handle (NaN before one)
  double last_lo = NAN, last_hi = NAN;
  bool lent = false;            // rocBLAS handle, second stream and events belong to a request-loop slot
  int solve_retries = 0;        // steps of the last pw_solve taken again after a failed Cholesky
  std::string solve_retry_msg;  // the text of that failure
  // PW_PROGRESS=1 in the environment: report each completed filter block of a band-blocked
  // step on stderr (the stream is synchronised at each report).
  bool progress = false;
  // Block whose bf16 planes the planes buffer holds (split-precision projectors), or null, and
  // the number of its leading columns they cover.
  const void* yp_src = nullptr;
  int yp_n = 0;
  // Block whose planes follow those of yp_src (the Gram product's second operand), or null.
  const void* wp_src = nullptr;
  // This device's copy of the library's static work array (device address), and, while a call of
  // pw_apply_h_noalloc runs, the work buffers of its H applications placed in it: stick and
  // pencil intermediates, split-K partials, D P and the bf16 planes of the block, for ws_cols
  // columns per H application and ws_fft_batch bands per FFT launch.
  unsigned char* scratch = nullptr;
  unsigned char* ws = nullptr;
  size_t ws_sb = 0, ws_g1 = 0, ws_parts = 0, ws_pt = 0, ws_yp = 0;
  int ws_cols = 0, ws_fft_batch = 0;
  std::chrono::steady_clock::time_point t_step;
  void report(const char* what, int i, int n) {
    if (!progress) return;
    (void)hipStreamSynchronize(stream);
    const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_step).count();
    std::fprintf(stderr, "pw: %s %d/%d done at %.1f s\n", what, i, n, t);
    std::fflush(stderr);
  }
  // phase timers
  bool timing = false;
  hipEvent_t open_ev = nullptr;
  struct Rec {
    int ph;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Rec> pending;
  pw_phase_stat stats[PW_NPHASES] = {};

  template <typename X>
  X* at(size_t off) const { return reinterpret_cast<X*>(arena + off); }

  hipEvent_t take_event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void tbegin() { tbegin(stream); }
  void tend(int ph) { tend(ph, stream); }
  void tbegin(hipStream_t s) {
    if (!timing) return;
    open_ev = take_event();
    if (open_ev) hipEventRecord(open_ev, s);
  }
  void tend(int ph, hipStream_t s) {
    if (!timing || !open_ev) return;
    hipEvent_t b = take_event();
    if (!b) return;
    hipEventRecord(b, s);
    pending.push_back({ph, open_ev, b});
    open_ev = nullptr;
  }
  // Requires the stream to be synchronised.
  void resolve() {
    for (const Rec& r : pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
        stats[r.ph].ms += ms;
        stats[r.ph].launches += 1;
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  // Second stream of the handle (default priority): the FFT part of each H application runs on
  // it, forked from and joined back into the caller's stream, concurrently with the projection.
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  ~pw_handle_s() {
    if (aux) {
      hipStreamSynchronize(aux);
      if (!lent) hipStreamDestroy(aux);
    }
    if (ev_fork && !lent) hipEventDestroy(ev_fork);
    if (ev_join && !lent) hipEventDestroy(ev_join);
    for (const Rec& r : pending) {
      hipEventDestroy(r.a);
      hipEventDestroy(r.b);
    }
    for (hipEvent_t e : pool) hipEventDestroy(e);
  }
};

namespace {

#define PW_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      h->err = std::string(#call) + ": " + hipGetErrorString(e_);                     \
      return PW_EDEVICE;                                                              \
    }                                                                                 \
  } while (0)

// Launch `call` bracketed by the phase timer of `ph`.
#define PW_TIMED(ph, call) \
  do {                     \
    h->tbegin();           \
    PW_HIP(call);          \
    h->tend(ph);           \
  } while (0)
#define PW_TIMED_ON(ph, st, call) \
  do {                            \
    h->tbegin(st);                \
    PW_HIP(call);                 \
    h->tend(ph, st);              \
  } while (0)

pw_status fail(pw_handle_s* h, pw_status s, const std::string& m) {
  if (h) h->err = m;
  g_last_error = m;
  return s;
}

template <typename T>
struct Engine {
  enum { PLANES_NONE = 0, PLANES_NEXT = 1, PLANES_GRAM = 2, PLANES_KEEP = 3 };
  pw_handle_s* h;
  const Plan& P;
  explicit Engine(pw_handle_s* hh) : h(hh), P(hh->plan) {}

  cplx<T>* beta() const { return h->at<cplx<T>>(P.lay.beta); }
  cplx<T>* u0() const { return h->at<cplx<T>>(P.lay.u0); }
  cplx<T>* u1() const { return h->at<cplx<T>>(P.lay.u1); }
  cplx<T>* zb() const { return h->at<cplx<T>>(P.lay.zb); }

  bool flag(unsigned f) const { return (P.flags & f) != 0; }
  // With split-precision projector products the table is stored as bf16 hi and lo planes of
  // one (re, im) word per entry, leading dimension ldw words, in the same arena bytes.
  bool beta_planes() const { return std::is_same<T, float>::value && flag(PW_FLAG_BF16_KB); }
  bool beta_otf() const { return flag(PW_FLAG_BETA_OTF); }
  BetaGen beta_gen() const {
    BetaGen bg;
    bg.miller = h->at<int>(P.lay.miller);
    bg.rad = h->at<double>(P.lay.brad);
    bg.ph = h->at<double2>(P.lay.bph);
    bg.h1 = P.hmax[0];
    bg.h2 = P.hmax[1];
    bg.h3 = P.hmax[2];
    bg.o2 = 2 * P.hmax[0] + 1;
    bg.o3 = bg.o2 + 2 * P.hmax[1] + 1;
    bg.w = P.bwidth;
    bg.npw = P.npw;
    bg.natoms = P.natoms;
    return bg;
  }
  RsDesc rs_desc() const {
    RsDesc d{};
    d.atoms = h->at<float4>(P.lay.rsat);
    d.zoff = h->at<int>(P.lay.rszo);
    d.zent = h->at<RsEnt>(P.lay.rsze);
    d.boff = h->at<int>(P.lay.rsbo);
    d.bent = h->at<RsEnt>(P.lay.rsbe);
    d.aoff = h->at<int>(P.lay.rsao);
    d.aent = h->at<int>(P.lay.rsae);
    d.nent = (int)P.rs_zent.size();
    d.natoms = P.natoms;
    d.hx = (float)(P.L[0] / P.g.n1);
    d.hy = (float)(P.L[1] / P.g.n2);
    d.r2 = (float)(P.rs_radius * P.rs_radius);
    d.k2 = (float)(-1.4426950408889634 * 0.5 / (P.beta_sigma * P.beta_sigma));
    const double so = std::sqrt(P.L[0] * P.L[1] * P.L[2]);
    d.c0 = (float)(so * std::pow(3.14159265358979323846, -0.75) * std::pow(P.beta_sigma, -1.5));
    d.c1 = (float)(so * std::sqrt(2.0) * std::pow(3.14159265358979323846, -0.75) * std::pow(P.beta_sigma, -2.5));
    return d;
  }
  unsigned int* beta_hi() const { return h->at<unsigned int>(P.lay.beta); }
  unsigned int* beta_lo() const { return beta_hi() + (size_t)P.ldw * P.nproj; }
  // Work buffers of an H application: the arena's, or the static work array's during
  // pw_apply_h_noalloc.
  template <typename X>
  X* work(size_t arena_off, size_t ws_off) const {
    return h->ws ? reinterpret_cast<X*>(h->ws + ws_off) : h->at<X>(arena_off);
  }
  cplx<T>* sb_buf() const { return work<cplx<T>>(P.lay.sb, h->ws_sb); }
  cplx<T>* g1_buf() const { return work<cplx<T>>(P.lay.g1, h->ws_g1); }
  double2* parts_buf() const { return work<double2>(P.lay.parts, h->ws_parts); }
  int fft_batch() const { return h->ws ? h->ws_fft_batch : P.fft_batch; }
  unsigned int* yp_hi() const { return work<unsigned int>(P.lay.yp, h->ws_yp); }
  unsigned int* yp_lo() const { return yp_hi() + (size_t)P.ldw * (h->ws ? h->ws_cols : P.yp_cols); }
  // the unblocked step keeps the planes of W = H Y beside those of Y for the Gram product
  bool gram_planes() const {
    return std::is_same<T, float>::value && (beta_planes() || P.rspace) && flag(PW_FLAG_BF16_GRAM) &&
           P.yp_cols >= 2 * P.nbb;
  }
  // with projector planes, D B^H Y is kept as the nonlocal product's B planes in the bytes of PT
  unsigned int* pt_hi() const { return work<unsigned int>(P.lay.pt, h->ws_pt); }
  unsigned int* pt_lo() const { return pt_hi() + (size_t)P.nproj * (h->ws ? h->ws_cols : P.nbb); }
  bool planes_of(const void* Y, int nb) const { return Y && h->yp_src == Y && nb <= h->yp_n; }
  void set_planes(const void* Y, int nb) {
    h->yp_src = Y;
    h->yp_n = Y ? nb : 0;
    h->wp_src = nullptr;
  }
  // Rotation coefficients (n x n, leading dimension n) as the nn product's B operand: with
  // split-precision rotation, bf16 planes (hi, then lo) in the bytes of the fp32 table at off;
  // otherwise the table in the compute precision.  Column j is scaled by sc * lambda_j when lam is
  // given.
  const cplx<T>* coef_table(size_t off, int n, const double* lam, double sc) {
    double2* Hs = h->at<double2>(P.lay.sh) + (size_t)n * n;
    if constexpr (std::is_same<T, float>::value) {
      if (flag(PW_FLAG_BF16_ROT)) {
        unsigned int* hi = h->at<unsigned int>(off);
        h->tbegin();
        (void)launch_coef_planes(Hs, n, n, lam, sc, hi, hi + (size_t)n * n, n, h->stream);
        h->tend(PW_PH_OTHER);
        return h->at<cplx<T>>(off);
      }
    }
    if (lam) {
      cplx<T>* t = h->at<cplx<T>>(off);
      h->tbegin();
      (void)launch_scale_cols_lam<T>(Hs, n, t, n, n, lam, sc, h->stream);
      h->tend(PW_PH_OTHER);
      return t;
    }
    return coeffs(n);
  }
  // out = epilogue(A C[:, c0 : c0 + w]), C from coef_table (n x n).
  hipError_t rot(const cplx<T>* A, long lda, const cplx<T>* C, int n, int c0, int w, cplx<T>* out, long ldo,
                 const EpiH& e) {
    if constexpr (std::is_same<T, float>::value) {
      if (flag(PW_FLAG_BF16_ROT)) {
        const unsigned int* hi = reinterpret_cast<const unsigned int*>(C);
        const unsigned int* ch = hi + (size_t)c0 * n;
        const unsigned int* cl = hi + (size_t)n * n + (size_t)c0 * n;
        if ((beta_planes() || P.rspace) && planes_of(A, n))
          return launch_gemm_nn_bf16x3_planes(yp_hi(), yp_lo(), P.ldw, ch, cl, n, P.npw, w, n, out, ldo, e,
                                              h->stream);
        // W = H Y of the unblocked step keeps its planes beside those of Y for the Gram product
        if (gram_planes() && A && static_cast<const void*>(A) == h->wp_src && h->yp_src && n <= h->yp_n) {
          const size_t pc = (size_t)P.ldw * h->yp_n;
          return launch_gemm_nn_bf16x3_planes(yp_hi() + pc, yp_lo() + pc, P.ldw, ch, cl, n, P.npw, w, n, out, ldo,
                                              e, h->stream);
        }
        return launch_gemm_nn_bf16x3_bplanes(A, lda, ch, cl, n, P.npw, w, n, out, ldo, e, h->stream);
      }
    }
    return launch_gemm_nn<T>(A, lda, C + (long)c0 * n, n, P.npw, w, n, out, ldo, e, h->stream);
  }

  hipError_t cn(bool split16, const cplx<T>* A, long lda, const cplx<T>* B, long ldb, const cplx<T>* B2, long ldb2,
                int ncol1, int M, int N, int K, int nsplit, double2* part, int nterm = 3) {
    if constexpr (std::is_same<T, float>::value) {
      if (split16)
        return launch_gemm_cn_bf16x3(A, lda, B, ldb, B2, ldb2, ncol1, M, N, K, nsplit, part, nterm, h->stream);
    }
    return launch_gemm_cn<T>(A, lda, B, ldb, B2, ldb2, ncol1, M, N, K, nsplit, part, h->stream);
  }
  hipError_t nn(bool split16, const cplx<T>* A, long lda, const cplx<T>* B, long ldb, int M, int N, int K,
                cplx<T>* out, long ldo, const EpiH& e) {
    if constexpr (std::is_same<T, float>::value) {
      if (split16) return launch_gemm_nn_bf16x3(A, lda, B, ldb, M, N, K, out, ldo, e, h->stream);
    }
    return launch_gemm_nn<T>(A, lda, B, ldb, M, N, K, out, ldo, e, h->stream);
  }

  // Local potential part: Z = P_sphere FFT_fwd[V FFT_inv[P_sphere^T Y]] for nb columns.
  pw_status local_part(const cplx<T>* Y, long ldy, cplx<T>* Z, long ldz, int nb, hipStream_t sm) {
    const GridDesc& g = P.g;
    const T scale = (T)(1.0 / ((double)g.n1 * g.n2 * g.n3));
    cplx<T>* SB = sb_buf();
    cplx<T>* G1 = g1_buf();
    const Stick* st = h->at<Stick>(P.lay.sticks);
    const int* cs = h->at<int>(P.lay.colstart);
    const T* V = h->at<T>(P.lay.vr);
    const cplx<T>* tw1 = h->at<cplx<T>>(P.lay.tw1);
    const cplx<T>* tw2 = h->at<cplx<T>>(P.lay.tw2);
    const cplx<T>* tw3 = h->at<cplx<T>>(P.lay.tw3);
    const int fb = fft_batch();
    for (int b0 = 0; b0 < nb; b0 += fb) {
      const int nbt = std::min(fb, nb - b0);
      PW_TIMED_ON(PW_PH_STICKS_INV, sm,
                  launch_sticks_inv<T>(Y + (long)b0 * ldy, ldy, SB, nbt, st, g, tw3, P.fl, sm));
      if (P.fl.sized) {
        PW_TIMED_ON(PW_PH_PLANE, sm, launch_plane_n<T>(SB, V, nbt, st, cs, g, tw1, scale, sm));
      } else if (P.fl.fused) {
        PW_TIMED_ON(PW_PH_PLANE, sm,
                    launch_plane_fused<T>(SB, V, nbt, st, g, tw1, tw2, scale, 0, (T*)nullptr, P.fl, sm));
      } else {
        PW_TIMED_ON(PW_PH_PENCIL_YINV, sm, launch_pencil_yinv<T>(SB, G1, nbt, st, cs, g, tw2, P.fl, sm));
        PW_TIMED_ON(PW_PH_PENCIL_X, sm, launch_pencil_x<T>(G1, V, nbt, g, tw1, 0, (T*)nullptr, P.fl, sm));
        PW_TIMED_ON(PW_PH_PENCIL_YFWD, sm, launch_pencil_yfwd<T>(SB, G1, nbt, st, cs, g, tw2, scale, P.fl, sm));
      }
      PW_TIMED_ON(PW_PH_STICKS_FWD, sm,
                  launch_sticks_fwd<T>(SB, Z + (long)b0 * ldz, ldz, nbt, st, g, tw3, P.fl, sm));
    }
    return PW_OK;
  }

  // The whole H application with real-space projectors (PW_FLAG_RSPACE_KB), per FFT batch: sticks,
  // then the inverse plane pass with the projections (SB only read), their sum over planes into
  // D P (the batch's columns of PT), then the plane pass adding D P at the atoms' points to V psi
  // before the forward transforms, then the forward sticks, which apply the Chebyshev update
  // out = alpha ((kin - c) Y + V psi + V_NL psi) - beta Yp as they write the sphere.
  pw_status local_part_rs(const cplx<T>* Y, long ldy, cplx<T>* out, long ldo, int nb, double alpha, double c,
                          double beta_c, const cplx<T>* Yp, long ldp, hipStream_t sm) {
    if constexpr (std::is_same<T, float>::value) {
      const GridDesc& g = P.g;
      const float scale = (float)(1.0 / ((double)g.n1 * g.n2 * g.n3));
      cplx<T>* SB = sb_buf();
      const Stick* st = h->at<Stick>(P.lay.sticks);
      const int* cs = h->at<int>(P.lay.colstart);
      const T* V = h->at<T>(P.lay.vr);
      const cplx<T>* tw1 = h->at<cplx<T>>(P.lay.tw1);
      const cplx<T>* tw3 = h->at<cplx<T>>(P.lay.tw3);
      const RsDesc rd = rs_desc();
      float2* part = h->at<float2>(P.lay.rsp);
      cplx<T>* PT = h->at<cplx<T>>(P.lay.pt);
      const double* dsc = h->at<double>(P.lay.dscale);
      const double inv_nr = 1.0 / ((double)g.n1 * g.n2 * g.n3);
      const int fb = P.fft_batch;
      for (int b0 = 0; b0 < nb; b0 += fb) {
        const int nbt = std::min(fb, nb - b0);
        PW_TIMED_ON(PW_PH_STICKS_INV, sm,
                    launch_sticks_inv<T>(Y + (long)b0 * ldy, ldy, SB, nbt, st, g, tw3, P.fl, sm));
        PW_TIMED_ON(PW_PH_PROJ, sm, launch_rs_proj128(SB, cs, g, tw1, rd, nbt, part, sm));
        PW_TIMED_ON(PW_PH_PROJ_REDUCE, sm,
                    launch_rs_reduce(part, rd, nbt, dsc, inv_nr, PT + (long)b0 * P.nproj, P.nproj, sm));
        PW_TIMED_ON(PW_PH_PLANE, sm,
                    launch_plane128_nl(SB, V, nbt, cs, g, tw1, scale, rd, PT + (long)b0 * P.nproj, P.nproj, sm));
        StickUpd u;
        u.kin = h->at<float>(P.lay.kin);
        u.Y = Y + (long)b0 * ldy;
        u.ldy = ldy;
        u.Yp = Yp ? Yp + (long)b0 * ldp : nullptr;
        u.ldp = ldp;
        u.alpha = (float)alpha;
        u.c = (float)c;
        u.beta = (float)beta_c;
        PW_TIMED_ON(PW_PH_STICKS_FWD, sm,
                    launch_sticks_fwd_upd(SB, out + (long)b0 * ldo, ldo, nbt, st, g, tw3, u, sm));
      }
      return PW_OK;
    } else {
      return fail(h, PW_EINVAL, "real-space projectors need PW_MIXED");
    }
  }

  // out = alpha ((kin - c) Y + Zl + B D B^H Y) - beta Yp, where Zl is first filled with the
  // local potential part.  Zl may equal out (apply_h); Yp may equal out (in-place update).
  // planes_out (split-precision projectors): PLANES_NEXT writes the bf16 planes of out for a
  // following hop on out; PLANES_GRAM writes them beside those of Y for the Gram product and keeps
  // Y's; PLANES_KEEP keeps Y's (the caller leaves Y unchanged while it uses them); PLANES_NONE
  // drops them.
  pw_status hop(const cplx<T>* Y, long ldy, int nb, cplx<T>* out, long ldo, cplx<T>* Zl, long ldz, double alpha,
                double c, double beta_c, const cplx<T>* Yp, long ldp, int planes_out = PLANES_NONE) {
    // the local part (FFTs, memory bound) on the second stream, the projection (matrix cores)
    // on the caller's stream; both only read Y, and the nonlocal GEMM waits for both.  With
    // phase timing on, everything stays on the caller's stream so that phase times are not
    // inflated by sharing the device.
    // Small blocks (serving-size cells) gain nothing from it and would only add streams.
    const bool overlap = !P.rspace && !h->timing && (double)P.npw * nb >= (double)(1 << 26);
    if (P.rspace) {
      // the forward sticks write the updated block: nothing else to do
      set_planes(nullptr, 0);
      return local_part_rs(Y, ldy, out, ldo, nb, alpha, c, beta_c, Yp, ldp, h->stream);
    }
    if (overlap) {
      PW_HIP(hipEventRecord(h->ev_fork, h->stream));
      PW_HIP(hipStreamWaitEvent(h->aux, h->ev_fork, 0));
    }
    if (!P.rspace) {
      pw_status s = local_part(Y, ldy, Zl, ldz, nb, overlap ? h->aux : h->stream);
      if (s != PW_OK) return s;
    }
    if (overlap) PW_HIP(hipEventRecord(h->ev_join, h->aux));
    cplx<T>* PT = work<cplx<T>>(P.lay.pt, h->ws_pt);
    if (P.nproj > 0 && !P.rspace) {
      double2* parts = parts_buf();
      if constexpr (std::is_same<T, float>::value) {
        if (beta_planes()) {
          if (!planes_of(Y, nb)) {
            PW_TIMED(PW_PH_OTHER, launch_split_planes(Y, ldy, P.npw, nb, yp_hi(), yp_lo(), P.ldw, h->stream));
            set_planes(Y, nb);
          }
          PW_TIMED(PW_PH_PROJ, launch_gemm_cn_bf16x3_planes(beta_hi(), beta_lo(), P.ldw, yp_hi(), yp_lo(), P.ldw,
                                                            P.nproj, nb, P.npw, P.nsplit_proj, parts, h->stream));
        }
      }
      if (beta_otf())
        PW_TIMED(PW_PH_PROJ, launch_gemm_cn_beta<T>(beta_gen(), Y, ldy, nb, P.nsplit_proj, parts, h->stream));
      else if (!beta_planes())
        PW_TIMED(PW_PH_PROJ, cn(false, beta(), P.ldw, Y, ldy, nullptr, 0, nb, P.nproj, nb, P.npw, P.nsplit_proj, parts));
      if (beta_planes())
        PW_TIMED(PW_PH_PROJ_REDUCE, launch_reduce_planes(parts, P.nsplit_proj, P.nproj, nb,
                                                         h->at<double>(P.lay.dscale), 4, pt_hi(), pt_lo(), P.nproj,
                                                         h->stream));
      else
        PW_TIMED(PW_PH_PROJ_REDUCE, launch_reduce_parts<T>(parts, P.nsplit_proj, P.nproj, nb,
                                                           h->at<double>(P.lay.dscale), 4, nullptr, 0, PT, P.nproj,
                                                           h->stream));
    }
    if (overlap) PW_HIP(hipStreamWaitEvent(h->stream, h->ev_join, 0));
    EpiH e;
    e.mode = 1;
    e.alpha = alpha;
    e.c = c;
    e.beta = beta_c;
    e.kin = h->at<T>(P.lay.kin);
    e.Y = Y;
    e.ldy = ldy;
    e.Zl = Zl;
    e.ldz = ldz;
    e.Yp = Yp;
    e.ldp = ldp;
    e.ph = e.pl = nullptr;
    e.ldpl = 0;
    e.vec4 = 0;
    const bool keep_y = (planes_out == PLANES_GRAM || planes_out == PLANES_KEEP) && planes_of(Y, nb) &&
                        static_cast<const void*>(out) != static_cast<const void*>(Y) &&
                        static_cast<const void*>(Zl) != static_cast<const void*>(Y);
    const void* ysrc = h->yp_src;
    set_planes(keep_y ? ysrc : nullptr, keep_y ? nb : 0);
    if constexpr (std::is_same<T, float>::value) {
      if (beta_planes()) {
        const bool w_gram = planes_out == PLANES_GRAM && keep_y && gram_planes();
        if (planes_out == PLANES_NEXT || w_gram) {
          const size_t pc = w_gram ? (size_t)P.ldw * nb : 0;  // W's columns follow Y's
          e.ph = yp_hi() + pc;
          e.pl = yp_lo() + pc;
          e.ldpl = P.ldw;
        }
        PW_TIMED(PW_PH_NL, launch_gemm_nn_bf16x3_planes(beta_hi(), beta_lo(), P.ldw, pt_hi(), pt_lo(), P.nproj,
                                                        P.npw, nb, P.nproj, out, ldo, e, h->stream));
        if (planes_out == PLANES_NEXT) set_planes(out, nb);
        if (w_gram) h->wp_src = out;
        return PW_OK;
      }
    }
    if (beta_otf()) {
      PW_TIMED(PW_PH_NL, launch_gemm_nn_beta<T>(beta_gen(), PT, P.nproj, nb, out, ldo, e, h->stream));
      return PW_OK;
    }
    PW_TIMED(PW_PH_NL, nn(false, beta(), P.ldw, PT, P.nproj, P.npw, nb, P.nproj, out, ldo, e));
    return PW_OK;
  }

  // rho(r) = sum_j occ_j |psi_j(r)|^2 on the FFT grid ([z][y][x], FP64), psi_j the unnormalised
  // inverse transform of column j: sticks -> inverse plane (or pencil) pass writing |psi|^2 per band
  // into u0, then a band-ordered weighted sum.  occ is on the device.
  pw_status density(const cplx<T>* X, int nb, long ld, const double* occ, double* rho) {
    const GridDesc& g = P.g;
    const long nr = (long)g.n1 * g.n2 * g.n3;
    cplx<T>* SB = h->at<cplx<T>>(P.lay.sb);
    cplx<T>* G1 = h->at<cplx<T>>(P.lay.g1);
    const Stick* st = h->at<Stick>(P.lay.sticks);
    const int* cs = h->at<int>(P.lay.colstart);
    const cplx<T>* tw1 = h->at<cplx<T>>(P.lay.tw1);
    const cplx<T>* tw2 = h->at<cplx<T>>(P.lay.tw2);
    const cplx<T>* tw3 = h->at<cplx<T>>(P.lay.tw3);
    T* psq = h->at<T>(P.lay.u0);
    const long u0_elems = 2L * P.ldw * P.nbb;
    if constexpr (std::is_same<T, float>::value) {
      if (P.fl.fused && density128_supported(g, P.real_bytes)) {
        // fused: one FP64 grid per band group (about two groups per compute unit in all), summed
        // into rho per batch
        int cus = 256;
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        int ngroups = std::max(1, (cus + g.n3 - 1) / g.n3);
        double* part = reinterpret_cast<double*>(psq);  // ngroups grids of nr doubles
        if ((long)ngroups * nr * 2 > u0_elems) {
          ngroups = 1;  // the group sums do not fit the work buffer: one group, straight into rho
          part = nullptr;
        }
        for (int b0 = 0; b0 < nb; b0 += P.fft_batch) {
          const int nbt = std::min(P.fft_batch, nb - b0);
          PW_TIMED(PW_PH_STICKS_INV,
                   launch_sticks_inv<T>(X + (long)b0 * ld, ld, SB, nbt, st, g, tw3, P.fl, h->stream));
          PW_TIMED(PW_PH_PLANE, launch_density128(SB, cs, g, tw1, occ + b0, nbt, ngroups, part, rho, b0 == 0,
                                                  h->stream));
        }
        return PW_OK;
      }
    }
    // bands per pass: the stick batch, and as many |psi|^2 grids as u0 holds
    const int per = (int)std::min<long>(P.fft_batch, u0_elems / nr);
    if (per < 1) return fail(h, PW_EINVAL, "density: the work buffer cannot hold one real-space grid");
    for (int b0 = 0; b0 < nb; b0 += per) {
      const int nbt = std::min(per, nb - b0);
      PW_TIMED(PW_PH_STICKS_INV, launch_sticks_inv<T>(X + (long)b0 * ld, ld, SB, nbt, st, g, tw3, P.fl, h->stream));
      if (P.fl.fused) {
        PW_TIMED(PW_PH_PLANE, launch_plane_fused<T>(SB, (const T*)nullptr, nbt, st, g, tw1, tw2, (T)1, 2, psq, P.fl,
                                                    h->stream));
      } else {
        PW_TIMED(PW_PH_PENCIL_YINV, launch_pencil_yinv<T>(SB, G1, nbt, st, cs, g, tw2, P.fl, h->stream));
        PW_TIMED(PW_PH_PENCIL_X, launch_pencil_x<T>(G1, (const T*)nullptr, nbt, g, tw1, 2, psq, P.fl, h->stream));
      }
      PW_TIMED(PW_PH_OTHER, launch_density_acc<T>(psq, nbt, nr, occ + b0, rho, b0 == 0, h->stream));
    }
    return PW_OK;
  }

  // HX = H X in column groups of `step` bands (the filter block, or what the static work array
  // holds during pw_apply_h_noalloc).
  pw_status apply_h(const cplx<T>* X, cplx<T>* HX, int nb, int ld, int step) {
    set_planes(nullptr, 0);
    for (int c0 = 0; c0 < nb; c0 += step) {
      const int w = std::min(step, nb - c0);
      pw_status s = hop(X + (long)c0 * ld, ld, w, HX + (long)c0 * ld, ld, HX + (long)c0 * ld, ld, 1.0, 0.0, 0.0,
                        nullptr, 0);
      if (s != PW_OK) return s;
    }
    return PW_OK;
  }

  // Chebyshev filter of w columns Y0 (ld0) in place: on return the columns hold Y_m.
  // Uses u0, u1 and zb (nbb columns each).
  pw_status filter_block(cplx<T>* Y0, long ld0, int w, const pw_step_params& prm) {
    const int m = prm.degree;
    const long ldw = P.ldw;
    if (m < 1) return PW_OK;
    const double e = 0.5 * (prm.b - prm.a), c = 0.5 * (prm.b + prm.a);
    const double s1 = e / (prm.a_lo - c), tau = 2.0 / s1;
    pw_status s = hop(Y0, ld0, w, u1(), ldw, zb(), ldw, s1 / e, c, 0.0, nullptr, 0, PLANES_NEXT);
    if (s != PW_OK) return s;
    const cplx<T>* prev = Y0;
    long ldprev = ld0;
    cplx<T>* cur = u1();
    double sg = s1;
    for (int k = 1; k < m; ++k) {
      const double sn = 1.0 / (tau - sg);
      cplx<T>* dst = (prev == Y0) ? u0() : const_cast<cplx<T>*>(prev);
      s = hop(cur, ldw, w, dst, ldw, zb(), ldw, 2.0 * sn / e, c, sg * sn, prev, ldprev, PLANES_NEXT);
      if (s != PW_OK) return s;
      prev = cur;
      ldprev = ldw;
      cur = dst;
      sg = sn;
    }
    PW_TIMED(PW_PH_OTHER, launch_copy_cols<T>(cur, ldw, Y0, ld0, P.npw, w, h->stream));
    if (h->yp_src == static_cast<const void*>(cur)) h->yp_src = Y0;  // same values, same columns
    return PW_OK;
  }

  // Band-blocked step: the filter and W = H Y run on column blocks; residuals from W C - X (C Lambda).
  pw_status eig_step_blocked(cplx<T>* X, cplx<T>* HX, int nb, int ld, const pw_step_params& prm, double* eig_host,
                             double* resid_host, double* bounds_out) {
    const long ldw = P.ldw;
    cplx<T>* W = h->at<cplx<T>>(P.lay.wf);
    pw_status s;
    const int nblk = (nb + P.nbb - 1) / P.nbb;
    h->t_step = std::chrono::steady_clock::now();
    for (int c0 = 0; c0 < nb; c0 += P.nbb) {
      const int w = std::min(P.nbb, nb - c0);
      s = filter_block(X + (long)c0 * ld, ld, w, prm);
      if (s != PW_OK) return s;
      s = hop(X + (long)c0 * ld, ld, w, W + (long)c0 * ldw, ldw, zb(), ldw, 1.0, 0.0, 0.0, nullptr, 0);
      if (s != PW_OK) return s;
      h->report("filter block", c0 / P.nbb + 1, nblk);
    }
    s = project_solve(X, ld, W, ldw, nb);
    if (s != PW_OK) return s;
    h->report("Gram and eigensolve", 1, 1);
    double* eig_d = h->at<double>(P.lay.eig);
    double* resid_d = h->at<double>(P.lay.resid);
    const cplx<T>* C = coef_table(P.lay.ct, nb, nullptr, 1.0);
    // CL = -C diag(lambda)
    const cplx<T>* CL = coef_table(P.lay.ct2, nb, eig_d, -1.0);
    EpiH st;
    std::memset(&st, 0, sizeof(st));
    for (int c0 = 0; c0 < nb; c0 += P.nbb) {
      const int w = std::min(P.nbb, nb - c0);
      // zb = W C[:, blk];  u0 = X CL[:, blk] + zb;  resid = ||u0 columns||
      PW_TIMED(PW_PH_ROTATE, rot(W, ldw, C, nb, c0, w, zb(), ldw, st));
      EpiH ad = st;
      ad.mode = 2;
      ad.Zl = zb();
      ad.ldz = ldw;
      PW_TIMED(PW_PH_ROTATE, rot(X, ld, CL, nb, c0, w, u0(), ldw, ad));
      PW_TIMED(PW_PH_RESID, launch_resid<T>(u0(), ldw, u0(), ldw, (const double*)nullptr, P.npw, w, resid_d + c0,
                                            h->stream));
      if (prm.want_hx && HX) {
        PW_TIMED(PW_PH_OTHER, launch_copy_cols<T>(zb(), ldw, HX + (long)c0 * ld, ld, P.npw, w, h->stream));
      }
    }
    // X' = X C into W's storage, then back into X
    PW_TIMED(PW_PH_ROTATE, rot(X, ld, C, nb, 0, nb, W, ldw, st));
    PW_TIMED(PW_PH_OTHER, launch_copy_cols<T>(W, ldw, X, ld, P.npw, nb, h->stream));
    set_planes(nullptr, 0);
    return finish(nb, eig_host, resid_host, bounds_out, prm.b);
  }

  pw_status rotate(const cplx<T>* A, long lda, const cplx<T>* C, int nb, cplx<T>* out, long ldo) {
    EpiH e;
    std::memset(&e, 0, sizeof(e));
    e.mode = 0;
    PW_TIMED(PW_PH_ROTATE, rot(A, lda, C, nb, 0, nb, out, ldo, e));
    if (h->yp_src == static_cast<const void*>(out)) set_planes(nullptr, 0);
    return PW_OK;
  }

  pw_status eig_step(cplx<T>* X, cplx<T>* HX, int nb, int ld, const pw_step_params& prm, double* eig_host,
                     double* resid_host, double* bounds_out) {
    set_planes(nullptr, 0);
    if (P.nbb < P.nbands) return eig_step_blocked(X, HX, nb, ld, prm, eig_host, resid_host, bounds_out);
    const int m = prm.degree;
    double bmax = prm.b;
    const long ldw = P.ldw;
    const cplx<T>* Y = X;
    long ldy = ld;
    cplx<T>* dead = u0();  // buffer free to receive W
    pw_status s;
    if (m >= 1) {
      const double e = 0.5 * (prm.b - prm.a), c = 0.5 * (prm.b + prm.a);
      const double s1 = e / (prm.a_lo - c), tau = 2.0 / s1;
      s = hop(X, ld, nb, u1(), ldw, zb(), ldw, s1 / e, c, 0.0, nullptr, 0, PLANES_NEXT);
      if (s != PW_OK) return s;
      const cplx<T>* prev = X;
      long ldprev = ld;
      cplx<T>* cur = u1();
      double sg = s1;
      for (int k = 1; k < m; ++k) {
        const double sn = 1.0 / (tau - sg);
        cplx<T>* dst = (prev == X) ? u0() : const_cast<cplx<T>*>(prev);
        s = hop(cur, ldw, nb, dst, ldw, zb(), ldw, 2.0 * sn / e, c, sg * sn, prev, ldprev, PLANES_NEXT);
        if (s != PW_OK) return s;
        prev = cur;
        ldprev = ldw;
        cur = dst;
        sg = sn;
      }
      Y = cur;
      ldy = ldw;
      dead = (prev == X) ? u0() : const_cast<cplx<T>*>(prev);
    }
    // W = H Y
    cplx<T>* W = dead;
    s = hop(Y, ldy, nb, W, ldw, zb(), ldw, 1.0, 0.0, 0.0, nullptr, 0, gram_planes() ? PLANES_GRAM : PLANES_KEEP);
    if (s != PW_OK) return s;
    s = project_solve(Y, ldy, W, ldw, nb);
    if (s != PW_OK) return s;
    const cplx<T>* C = coef_table(P.lay.ct, nb, nullptr, 1.0);
    double* eig_d = h->at<double>(P.lay.eig);
    // X' = Y C (never in place), W' = W C
    cplx<T>* Wr = (prm.want_hx && HX) ? HX : zb();
    const long ldwr = (prm.want_hx && HX) ? ld : ldw;
    if (Y == X) {
      s = rotate(Y, ldy, C, nb, u1(), ldw);
      if (s != PW_OK) return s;
      PW_TIMED(PW_PH_OTHER, launch_copy_cols<T>(u1(), ldw, X, ld, P.npw, nb, h->stream));
      if (h->yp_src == static_cast<const void*>(X)) set_planes(nullptr, 0);
    } else {
      s = rotate(Y, ldy, C, nb, X, ld);
      if (s != PW_OK) return s;
    }
    s = rotate(W, ldw, C, nb, Wr, ldwr);
    if (s != PW_OK) return s;
    double* resid_d = h->at<double>(P.lay.resid);
    PW_TIMED(PW_PH_RESID, launch_resid<T>(Wr, ldwr, X, ld, eig_d, P.npw, nb, resid_d, h->stream));
    set_planes(nullptr, 0);
    return finish(nb, eig_host, resid_host, bounds_out, bmax);
  }

  // [S | H_s] = Y^H [Y | W], Hermitian parts, FP64 generalised eigensolve (C in the H_s storage).
  pw_status project_solve(const cplx<T>* Y, long ldy, const cplx<T>* W, long ldw, int nb) {
    double2* parts = h->at<double2>(P.lay.parts);
    double2* SH = h->at<double2>(P.lay.sh);
    if (gram_planes() && planes_of(Y, nb) && h->wp_src == static_cast<const void*>(W)) {
      // S = Y^H Y is Hermitian: its tiles below the diagonal are skipped and mirrored afterwards
      PW_TIMED(PW_PH_GRAM, launch_gemm_cn_bf16x3_planes(yp_hi(), yp_lo(), P.ldw, yp_hi(), yp_lo(), P.ldw, nb, 2 * nb,
                                                        P.npw, P.nsplit_gram, parts, h->stream, 4, nb));
      return dense_solve(nb, P.nsplit_gram, 0.0, true);
    }
    if constexpr (std::is_same<T, float>::value) {
      if (P.rspace && gram_planes() && nb <= P.nbb) {
        // real-space projectors write no planes: split Y and W here for the planes' Gram product
        const size_t pc = (size_t)P.ldw * nb;
        PW_TIMED(PW_PH_OTHER, launch_split_planes(Y, ldy, P.npw, nb, yp_hi(), yp_lo(), P.ldw, h->stream));
        PW_TIMED(PW_PH_OTHER, launch_split_planes(W, ldw, P.npw, nb, yp_hi() + pc, yp_lo() + pc, P.ldw, h->stream));
        set_planes(Y, nb);
        h->wp_src = W;
        PW_TIMED(PW_PH_GRAM, launch_gemm_cn_bf16x3_planes(yp_hi(), yp_lo(), P.ldw, yp_hi(), yp_lo(), P.ldw, nb,
                                                          2 * nb, P.npw, P.nsplit_gram, parts, h->stream, 4, nb));
        return dense_solve(nb, P.nsplit_gram, 0.0, true);
      }
    }
    PW_TIMED(PW_PH_GRAM, cn(flag(PW_FLAG_BF16_GRAM), Y, ldy, Y, ldy, W, ldw, nb, nb, 2 * nb, P.npw, P.nsplit_gram,
                            parts, 4));
    return dense_solve(nb, P.nsplit_gram);
  }

  // Sum the split-K partials of [S | H_s] (n x 2n), take Hermitian parts, and solve
  // H_s C = S C diag(lambda), C^H S C = I in FP64 (C in the H_s storage, lambda ascending).
  // With min_pivot > 0 a factor whose smallest pivot keeps no more than min_pivot of its diagonal
  // entry (|L_ii|^2 <= min_pivot S_ii) counts as a failed factorisation (PW_ENOTPD).
  // s_upper: only S's upper triangle was computed (the lower one is taken from it).
  pw_status dense_solve(int nb, int nsplit, double min_pivot = 0.0, bool s_upper = false) {
    double2* parts = h->at<double2>(P.lay.parts);
    double2* SH = h->at<double2>(P.lay.sh);
    double2* S = SH;
    double2* Hs = SH + (size_t)nb * nb;
    h->tbegin();
    PW_HIP(launch_reduce_parts<T>(parts, nsplit, nb, 2 * nb, nullptr, 0, SH, nb, (cplx<T>*)nullptr, 0,
                                  h->stream));
    if (s_upper)
      PW_HIP(launch_mirror_upper(S, nb, nb, h->stream));
    else
      PW_HIP(launch_hermitize(S, nb, nb, h->stream));
    PW_HIP(launch_hermitize(Hs, nb, nb, h->stream));
    h->tend(PW_PH_GRAM_REDUCE);
    // Hs C = S C diag(lambda), C^H S C = I: S = L L^H, A = L^{-1} Hs L^{-H} by two triangular
    // solves (level 3; the library's unblocked reduction to standard form took half the time),
    // A V = V diag(lambda), C = L^{-H} V in the Hs storage.
    double* eig_d = h->at<double>(P.lay.eig);
    int* info_d = h->at<int>(P.lay.info);
    auto* Sz = reinterpret_cast<rocblas_double_complex*>(S);
    auto* Hz = reinterpret_cast<rocblas_double_complex*>(Hs);
    const rocblas_double_complex one(1.0, 0.0);
    h->tbegin();
    double* dS = h->at<double>(P.lay.ework);
    double* piv_d = h->at<double>(P.lay.scal) + 3;  // [8, 8 + 2 kLanczosChunk) hold the Lanczos pairs
    if (min_pivot > 0.0) PW_HIP(launch_diag_copy(S, nb, nb, dS, h->stream));
    rocblas_status rs = rocsolver_zpotrf(h->blas, rocblas_fill_lower, nb, Sz, nb, info_d);
    if (rs != rocblas_status_success)
      return fail(h, PW_EDEVICE, std::string("rocsolver_zpotrf: ") + rocblas_status_to_string(rs));
    if (min_pivot > 0.0) PW_HIP(launch_min_pivot(S, nb, nb, dS, piv_d, h->stream));
    int info[2] = {0, 0};
    double piv = 1.0;
    PW_HIP(hipMemcpyAsync(&info[0], info_d, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    if (min_pivot > 0.0) PW_HIP(hipMemcpyAsync(&piv, piv_d, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    PW_HIP(hipStreamSynchronize(h->stream));
    if (info[0] > 0) {
      h->tend(PW_PH_EIGSOLVE);
      return fail(h, PW_ENOTPD, "Cholesky of the Gram matrix failed (rank-deficient block)");
    }
    if (min_pivot > 0.0 && !(piv > min_pivot)) {
      h->tend(PW_PH_EIGSOLVE);
      return fail(h, PW_ENOTPD, "Gram matrix numerically singular (a Cholesky pivot below the drop tolerance)");
    }
    rs = rocblas_ztrsm(h->blas, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none,
                       rocblas_diagonal_non_unit, nb, nb, &one, Sz, nb, Hz, nb);
    if (rs == rocblas_status_success)
      rs = rocblas_ztrsm(h->blas, rocblas_side_right, rocblas_fill_lower, rocblas_operation_conjugate_transpose,
                         rocblas_diagonal_non_unit, nb, nb, &one, Sz, nb, Hz, nb);
    if (rs != rocblas_status_success)
      return fail(h, PW_EDEVICE, std::string("rocblas_ztrsm: ") + rocblas_status_to_string(rs));
    rs = rocsolver_zheevd(h->blas, rocblas_evect_original, rocblas_fill_lower, nb, Hz, nb, eig_d,
                          h->at<double>(P.lay.ework), info_d + 1);
    if (rs != rocblas_status_success)
      return fail(h, PW_EDEVICE, std::string("rocsolver_zheevd: ") + rocblas_status_to_string(rs));
    rs = rocblas_ztrsm(h->blas, rocblas_side_left, rocblas_fill_lower, rocblas_operation_conjugate_transpose,
                       rocblas_diagonal_non_unit, nb, nb, &one, Sz, nb, Hz, nb);
    if (rs != rocblas_status_success)
      return fail(h, PW_EDEVICE, std::string("rocblas_ztrsm: ") + rocblas_status_to_string(rs));
    h->tend(PW_PH_EIGSOLVE);
    PW_HIP(hipMemcpyAsync(&info[1], info_d + 1, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    PW_HIP(hipStreamSynchronize(h->stream));
    if (info[1] > 0) return fail(h, PW_ENUMERIC, "dense eigensolver did not converge");
    return PW_OK;
  }

  // Rayleigh-Ritz on the kept part of a basis whose Gram matrix failed the Cholesky test: the
  // split-K partials of [S | H_s] are summed again, S is scaled to unit diagonal
  // (D = diag(S)^-1/2), D S D = U diag(sigma) U^H, the directions with sigma <= tol * max(sigma)
  // dropped, T = D U_kept diag(sigma_kept)^-1/2 (T^H S T = I), T^H H_s T = V diag(lambda) V^H
  // and C = T V (the nb lowest columns, in the H_s storage with leading dimension k).  *kept is
  // the dimension of the kept span; PW_ENOTPD when it is below nb.
  pw_status dense_solve_svqb(int k, int nb, int nsplit, double tol, int* kept_out) {
    double2* parts = h->at<double2>(P.lay.parts);
    double2* SH = h->at<double2>(P.lay.sh);
    double2* S = SH;
    double2* Hs = SH + (size_t)k * k;
    double* d = h->at<double>(P.lay.ct);  // k doubles; the coefficient table is written later
    double* sig = h->at<double>(P.lay.eig);
    int* info_d = h->at<int>(P.lay.info);
    h->tbegin();
    PW_HIP(launch_reduce_parts<T>(parts, nsplit, k, 2 * k, nullptr, 0, SH, k, (cplx<T>*)nullptr, 0, h->stream));
    PW_HIP(launch_hermitize(S, k, k, h->stream));
    PW_HIP(launch_hermitize(Hs, k, k, h->stream));
    PW_HIP(launch_svqb_scale(S, k, k, d, h->stream));
    auto* Sz = reinterpret_cast<rocblas_double_complex*>(S);
    auto* Hz = reinterpret_cast<rocblas_double_complex*>(Hs);
    rocblas_status rs = rocsolver_zheevd(h->blas, rocblas_evect_original, rocblas_fill_lower, k, Sz, k, sig,
                                         h->at<double>(P.lay.ework), info_d + 1);
    if (rs != rocblas_status_success)
      return fail(h, PW_EDEVICE, std::string("rocsolver_zheevd: ") + rocblas_status_to_string(rs));
    std::vector<double> sh(k);
    int info = 0;
    PW_HIP(hipMemcpyAsync(sh.data(), sig, sizeof(double) * k, hipMemcpyDeviceToHost, h->stream));
    PW_HIP(hipMemcpyAsync(&info, info_d + 1, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    PW_HIP(hipStreamSynchronize(h->stream));
    if (info > 0) return fail(h, PW_ENUMERIC, "eigensolver of the basis Gram matrix did not converge");
    const double smax = sh[k - 1];
    int first = 0;
    while (first < k && !(sh[first] > tol * smax)) ++first;
    const int kept = k - first;
    if (kept_out) *kept_out = kept;
    if (!(smax > 0.0) || kept < nb) {
      h->tend(PW_PH_EIGSOLVE);
      return fail(h, PW_ENOTPD, "basis spans fewer directions than the block has columns");
    }
    // T (k x kept) and H_s T (k x kept) in the partials' storage, T^H H_s T in the S storage
    double2* Tm = parts;
    double2* HT = parts + (size_t)k * kept;
    PW_HIP(launch_svqb_basis(S, k, k, sig, d, first, kept, Tm, k, h->stream));
    auto* Tz = reinterpret_cast<rocblas_double_complex*>(Tm);
    auto* HTz = reinterpret_cast<rocblas_double_complex*>(HT);
    const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
    rs = rocblas_zgemm(h->blas, rocblas_operation_none, rocblas_operation_none, k, kept, k, &one, Hz, k, Tz, k,
                       &zero, HTz, k);
    if (rs == rocblas_status_success)
      rs = rocblas_zgemm(h->blas, rocblas_operation_conjugate_transpose, rocblas_operation_none, kept, kept, k, &one,
                         Tz, k, HTz, k, &zero, Sz, kept);
    if (rs != rocblas_status_success)
      return fail(h, PW_EDEVICE, std::string("rocblas_zgemm: ") + rocblas_status_to_string(rs));
    PW_HIP(launch_hermitize(S, kept, kept, h->stream));
    rs = rocsolver_zheevd(h->blas, rocblas_evect_original, rocblas_fill_lower, kept, Sz, kept, sig,
                          h->at<double>(P.lay.ework), info_d + 1);
    if (rs != rocblas_status_success)
      return fail(h, PW_EDEVICE, std::string("rocsolver_zheevd: ") + rocblas_status_to_string(rs));
    rs = rocblas_zgemm(h->blas, rocblas_operation_none, rocblas_operation_none, k, nb, kept, &one, Tz, k, Sz, kept,
                       &zero, Hz, k);
    if (rs != rocblas_status_success)
      return fail(h, PW_EDEVICE, std::string("rocblas_zgemm: ") + rocblas_status_to_string(rs));
    h->tend(PW_PH_EIGSOLVE);
    PW_HIP(hipMemcpyAsync(&info, info_d + 1, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    PW_HIP(hipStreamSynchronize(h->stream));
    if (info > 0) return fail(h, PW_ENUMERIC, "dense eigensolver did not converge");
    return PW_OK;
  }

  // Basis directions whose scaled Gram eigenvalue is below this fraction of the largest are
  // dropped (the Gram matrix of FP32 data is accurate to about 1e-7 of its diagonal).
  static constexpr double drop_tol() { return sizeof(T) == 8 ? PW_DROP_TOL_FP64 : PW_DROP_TOL_MIXED; }

  // One LOBPCG step (the C ABI's pw_lobpcg_step): Z = [X R P], HZ = [HX HR HP] in the arena,
  // Rayleigh-Ritz on span Z, X' = Z C_1 into X, P' = [R P] C_1(R and P rows) into Pd.
  pw_status lobpcg_step(cplx<T>* X, cplx<T>* Pd, int nb, long ld, bool have_p, double* eig_host,
                        double* resid_host, int* kept) {
    set_planes(nullptr, 0);
    const long ldw = P.ldw;
    cplx<T>* Z = h->at<cplx<T>>(P.lay.lz);
    cplx<T>* HZ = Z + (size_t)3 * P.nbands * ldw;
    double* theta = h->at<double>(P.lay.eig);  // Rayleigh quotients of X (before the eigensolve)
    double* resid_d = h->at<double>(P.lay.resid);
    double* nrm = h->at<double>(P.lay.ework);
    const T* kin = h->at<T>(P.lay.kin);
    // X and W = H X
    PW_TIMED(PW_PH_OTHER, launch_copy_cols<T>(X, ld, Z, ldw, P.npw, nb, h->stream));
    pw_status s = hop(Z, ldw, nb, HZ, ldw, HZ, ldw, 1.0, 0.0, 0.0, nullptr, 0);
    if (s != PW_OK) return s;
    // theta, residual norms of X, preconditioned residuals R (unit columns) and H R
    cplx<T>* R = Z + (size_t)nb * ldw;
    PW_TIMED(PW_PH_OTHER, launch_rayleigh<T>(HZ, ldw, Z, ldw, P.npw, nb, theta, h->stream));
    PW_TIMED(PW_PH_RESID, launch_resid<T>(HZ, ldw, Z, ldw, theta, P.npw, nb, resid_d, h->stream));
    PW_HIP(hipMemcpyAsync(resid_host, resid_d, sizeof(double) * nb, hipMemcpyDeviceToHost, h->stream));
    PW_TIMED(PW_PH_OTHER, launch_precond_resid<T>(HZ, ldw, Z, ldw, theta, kin, P.npw, nb, R, ldw, h->stream));
    PW_TIMED(PW_PH_OTHER, launch_resid<T>(R, ldw, R, ldw, (const double*)nullptr, P.npw, nb, nrm, h->stream));
    PW_TIMED(PW_PH_OTHER, launch_scale_cols_inv<T>(R, ldw, P.npw, nb, nrm, h->stream));
    s = hop(R, ldw, nb, HZ + (size_t)nb * ldw, ldw, HZ + (size_t)nb * ldw, ldw, 1.0, 0.0, 0.0, nullptr, 0);
    if (s != PW_OK) return s;
    if (have_p) {
      cplx<T>* Pz = Z + (size_t)2 * nb * ldw;
      PW_TIMED(PW_PH_OTHER, launch_copy_cols<T>(Pd, ld, Pz, ldw, P.npw, nb, h->stream));
      PW_TIMED(PW_PH_OTHER, launch_resid<T>(Pz, ldw, Pz, ldw, (const double*)nullptr, P.npw, nb, nrm, h->stream));
      PW_TIMED(PW_PH_OTHER, launch_scale_cols_inv<T>(Pz, ldw, P.npw, nb, nrm, h->stream));
      s = hop(Pz, ldw, nb, HZ + (size_t)2 * nb * ldw, ldw, HZ + (size_t)2 * nb * ldw, ldw, 1.0, 0.0, 0.0, nullptr, 0);
      if (s != PW_OK) return s;
    }
    // Rayleigh-Ritz on span Z; when the basis is numerically dependent (its Gram matrix fails the
    // Cholesky test), on the part of the span that the truncated SVQB basis keeps
    double2* parts = h->at<double2>(P.lay.parts);
    const int k = (have_p ? 3 : 2) * nb;
    PW_TIMED(PW_PH_GRAM, cn(flag(PW_FLAG_BF16_GRAM), Z, ldw, Z, ldw, HZ, ldw, k, k, 2 * k, P.npw, P.nsplit_lob,
                            parts, 4));
    if (kept) *kept = k;
    s = dense_solve(k, P.nsplit_lob, drop_tol());
    if (s == PW_ENOTPD) s = dense_solve_svqb(k, nb, P.nsplit_lob, drop_tol(), kept);
    if (s != PW_OK) return s;
    const cplx<T>* C = coeffs(k);
    EpiH e;
    std::memset(&e, 0, sizeof(e));
    e.mode = 0;
    PW_TIMED(PW_PH_ROTATE, nn(flag(PW_FLAG_BF16_ROT), Z, ldw, C, k, P.npw, nb, k, X, ld, e));
    PW_TIMED(PW_PH_ROTATE, nn(flag(PW_FLAG_BF16_ROT), R, ldw, C + nb, k, P.npw, nb, k - nb, Pd, ld, e));
    PW_HIP(hipMemcpyAsync(eig_host, h->at<double>(P.lay.eig), sizeof(double) * nb, hipMemcpyDeviceToHost,
                          h->stream));
    PW_HIP(hipStreamSynchronize(h->stream));
    for (int i = 0; i < nb; ++i)
      if (!std::isfinite(eig_host[i]) || !std::isfinite(resid_host[i]))
        return fail(h, PW_ENUMERIC, "non-finite Ritz value or residual");
    return PW_OK;
  }

  // One PPCG step (the C ABI's pw_ppcg_step).  Arena: Z = [X0 | W | P] and HZ = [H X0 | H W | H P]
  // (the LOBPCG buffers).  Rayleigh-Ritz on span X (X <- X C, P <- P C), residuals of the Ritz
  // vectors, W = T R, [W P] <- [W P] - X (X^H [W P]), H W and H P, then per column the Ritz vector
  // of span{x_j, w_j, p_j}: X <- a X + b W + g P, P <- b W + g P.
  pw_status ppcg_step(cplx<T>* X, cplx<T>* Pd, int nb, long ld, bool have_p, double* eig_host, double* resid_host) {
    set_planes(nullptr, 0);
    const long ldw = P.ldw;
    cplx<T>* Z = h->at<cplx<T>>(P.lay.lz);
    cplx<T>* HZ = Z + (size_t)3 * P.nbands * ldw;
    cplx<T>* Zw = Z + (size_t)nb * ldw;
    cplx<T>* Zp = Z + (size_t)2 * nb * ldw;
    cplx<T>* HZw = HZ + (size_t)nb * ldw;
    cplx<T>* HZp = HZ + (size_t)2 * nb * ldw;
    double* eig_d = h->at<double>(P.lay.eig);
    double* resid_d = h->at<double>(P.lay.resid);
    const T* kin = h->at<T>(P.lay.kin);
    double2* parts = h->at<double2>(P.lay.parts);
    // Rayleigh-Ritz on span X
    PW_TIMED(PW_PH_OTHER, launch_copy_cols<T>(X, ld, Z, ldw, P.npw, nb, h->stream));
    pw_status s = hop(Z, ldw, nb, HZ, ldw, HZ, ldw, 1.0, 0.0, 0.0, nullptr, 0);
    if (s != PW_OK) return s;
    PW_TIMED(PW_PH_GRAM, cn(flag(PW_FLAG_BF16_GRAM), Z, ldw, Z, ldw, HZ, ldw, nb, nb, 2 * nb, P.npw, P.nsplit_gram,
                            parts, 4));
    s = dense_solve(nb, P.nsplit_gram);
    if (s != PW_OK) return s;
    const cplx<T>* C = coeffs(nb);
    EpiH e;
    std::memset(&e, 0, sizeof(e));
    e.mode = 0;
    const bool r16 = flag(PW_FLAG_BF16_ROT);
    PW_TIMED(PW_PH_ROTATE, nn(r16, Z, ldw, C, nb, P.npw, nb, nb, X, ld, e));    // Ritz vectors
    PW_TIMED(PW_PH_ROTATE, nn(r16, HZ, ldw, C, nb, P.npw, nb, nb, Zw, ldw, e));  // H times them
    if (have_p) PW_TIMED(PW_PH_ROTATE, nn(r16, Pd, ld, C, nb, P.npw, nb, nb, Zp, ldw, e));
    // residual norms, then W = T (H X - X Lambda) in place of H X
    PW_TIMED(PW_PH_RESID, launch_resid<T>(Zw, ldw, X, ld, eig_d, P.npw, nb, resid_d, h->stream));
    PW_TIMED(PW_PH_OTHER, launch_precond_resid<T>(Zw, ldw, X, ld, eig_d, kin, P.npw, nb, Zw, ldw, h->stream));
    // [W P] <- [W P] - X (X^H [W P]): the coefficients summed with the factor -1
    const int ncols = have_p ? 2 * nb : nb;
    double* neg = h->at<double>(P.lay.scal) + 2;
    static const double kMinusOne = -1.0;
    PW_HIP(hipMemcpyAsync(neg, &kMinusOne, sizeof(double), hipMemcpyHostToDevice, h->stream));
    PW_TIMED(PW_PH_GRAM, cn(flag(PW_FLAG_BF16_GRAM), X, ld, Zw, ldw, nullptr, 0, ncols, nb, ncols, P.npw,
                            P.nsplit_gram, parts, 4));
    cplx<T>* Cp = h->at<cplx<T>>(P.lay.ct);
    PW_TIMED(PW_PH_GRAM_REDUCE, launch_reduce_parts<T>(parts, P.nsplit_gram, nb, ncols, neg, 1, nullptr, 0, Cp, nb,
                                                       h->stream));
    e.mode = 2;
    e.Zl = Zw;
    e.ldz = ldw;
    PW_TIMED(PW_PH_ROTATE, nn(r16, X, ld, Cp, nb, P.npw, ncols, nb, Zw, ldw, e));
    // H W and H P
    s = hop(Zw, ldw, nb, HZw, ldw, HZw, ldw, 1.0, 0.0, 0.0, nullptr, 0);
    if (s != PW_OK) return s;
    if (have_p) {
      s = hop(Zp, ldw, nb, HZp, ldw, HZp, ldw, 1.0, 0.0, 0.0, nullptr, 0);
      if (s != PW_OK) return s;
    }
    // per-column Rayleigh-Ritz and the update
    double2* dots = parts;
    double2* coef = parts + (size_t)11 * nb;
    PW_TIMED(PW_PH_OTHER, launch_ppcg_dots<T>(X, ld, Zw, Zp, HZw, HZp, ldw, P.npw, nb, have_p ? 1 : 0, dots,
                                              h->stream));
    PW_TIMED(PW_PH_OTHER, launch_ppcg_small(dots, eig_d, nb, have_p ? 1 : 0, drop_tol(), coef, h->stream));
    PW_TIMED(PW_PH_OTHER, launch_ppcg_update<T>(X, ld, Pd, ld, Zw, Zp, ldw, P.npw, nb, have_p ? 1 : 0, coef,
                                                h->stream));
    PW_HIP(hipGetLastError());
    PW_HIP(hipMemcpyAsync(eig_host, eig_d, sizeof(double) * nb, hipMemcpyDeviceToHost, h->stream));
    PW_HIP(hipMemcpyAsync(resid_host, resid_d, sizeof(double) * nb, hipMemcpyDeviceToHost, h->stream));
    PW_HIP(hipStreamSynchronize(h->stream));
    for (int i = 0; i < nb; ++i)
      if (!std::isfinite(eig_host[i]) || !std::isfinite(resid_host[i]))
        return fail(h, PW_ENUMERIC, "non-finite Ritz value or residual");
    return PW_OK;
  }

  // Eigenvector coefficients C in the compute precision.
  const cplx<T>* coeffs(int nb) {
    double2* Hs = h->at<double2>(P.lay.sh) + (size_t)nb * nb;
    if constexpr (sizeof(T) == 8) {
      return reinterpret_cast<const cplx<T>*>(Hs);
    } else {
      cplx<T>* ct = h->at<cplx<T>>(P.lay.ct);
      h->tbegin();
      (void)launch_convert_c64_to<T>(Hs, nb, ct, nb, nb, nb, h->stream);
      h->tend(PW_PH_OTHER);
      return ct;
    }
  }

  pw_status finish(int nb, double* eig_host, double* resid_host, double* bounds_out, double bmax) {
    double* eig_d = h->at<double>(P.lay.eig);
    double* resid_d = h->at<double>(P.lay.resid);
    PW_HIP(hipGetLastError());
    PW_HIP(hipMemcpyAsync(eig_host, eig_d, sizeof(double) * nb, hipMemcpyDeviceToHost, h->stream));
    PW_HIP(hipMemcpyAsync(resid_host, resid_d, sizeof(double) * nb, hipMemcpyDeviceToHost, h->stream));
    PW_HIP(hipStreamSynchronize(h->stream));
    h->resolve();
    for (int i = 0; i < nb; ++i)
      if (!std::isfinite(eig_host[i]) || !std::isfinite(resid_host[i]))
        return fail(h, PW_ENUMERIC, "non-finite eigenvalue or residual");
    if (bounds_out) {
      bounds_out[0] = eig_host[0];
      bounds_out[1] = eig_host[nb - 1];
      bounds_out[2] = bmax;
    }
    return PW_OK;
  }

  pw_status random_block(cplx<T>* X, int nb, int ld, unsigned long long seed) {
    double* nrm = h->at<double>(P.lay.resid);
    PW_HIP(launch_random_block<T>(X, ld, P.npw, nb, h->at<T>(P.lay.kin), seed, h->stream));
    PW_HIP(launch_resid<T>(X, ld, X, ld, (const double*)nullptr, P.npw, nb, nrm, h->stream));
    PW_HIP(launch_scale_cols_inv<T>(X, ld, P.npw, nb, nrm, h->stream));
    return PW_OK;
  }

  // Lanczos estimate of the top of the spectrum (filter bound b).
  pw_status spectrum_bound(int steps, unsigned long long seed, double* out) {
    const int n = P.npw;
    cplx<T>* V0 = h->at<cplx<T>>(P.lay.lanc);
    cplx<T>* V1 = V0 + P.ldw;
    cplx<T>* Wv = V1 + P.ldw;
    double* lab = h->at<double>(P.lay.scal) + 8;  // (alpha, beta) of each step of a chunk
    // seeded start vector (splitmix64 + Box-Muller), normalised on the host
    std::vector<cplx<T>> v(n);
    uint64_t x = seed ? seed : 0x9e3779b97f4a7c15ull;
    auto next = [&]() {
      x += 0x9e3779b97f4a7c15ull;
      uint64_t z = x;
      z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
      z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
      z ^= z >> 31;
      return ((z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    };
    double nrm = 0.0;
    std::vector<double> tmp(2 * n);
    for (int i = 0; i < n; ++i) {
      const double u1 = next(), u2 = next();
      const double r = std::sqrt(-2.0 * std::log(u1));
      tmp[2 * i] = r * std::cos(6.283185307179586 * u2);
      tmp[2 * i + 1] = r * std::sin(6.283185307179586 * u2);
      nrm += tmp[2 * i] * tmp[2 * i] + tmp[2 * i + 1] * tmp[2 * i + 1];
    }
    nrm = 1.0 / std::sqrt(nrm);
    for (int i = 0; i < n; ++i) v[i] = mk<T>((T)(tmp[2 * i] * nrm), (T)(tmp[2 * i + 1] * nrm));
    PW_HIP(hipMemcpyAsync(V1, v.data(), sizeof(cplx<T>) * n, hipMemcpyHostToDevice, h->stream));
    PW_HIP(launch_fill_zero<T>(V0, P.ldw, h->stream));
    // The recurrence runs on the device, each step reading the previous beta there; the host reads
    // the (alpha, beta) pairs once per chunk of kLanczosChunk steps.  A beta below 1e-12 ends the
    // recurrence: the steps after it in its chunk are discarded.
    std::vector<double> al, be;
    double bprev = 0.0;
    const int total = std::min(steps, n);
    bool ended = false;
    for (int c0 = 0; c0 < total && !ended; c0 += kLanczosChunk) {
      const int c1 = std::min(total, c0 + kLanczosChunk);
      for (int it = c0; it < c1; ++it) {
        pw_status s = apply_h(V1, Wv, 1, (int)P.ldw, P.nbb);
        if (s != PW_OK) return s;
        double* ab = lab + 2 * (it - c0);
        PW_HIP(launch_lanczos_step<T>(Wv, V1, V0, bprev, it > c0 ? ab - 1 : nullptr, n, ab, h->stream));
        // V0 <- V1, V1 <- W / beta
        PW_HIP(launch_copy_cols<T>(V1, P.ldw, V0, P.ldw, n, 1, h->stream));
        PW_HIP(launch_scale_copy_inv<T>(Wv, V1, ab + 1, n, h->stream));
      }
      std::vector<double> hs(2 * (size_t)(c1 - c0));
      PW_HIP(hipMemcpyAsync(hs.data(), lab, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, h->stream));
      PW_HIP(hipStreamSynchronize(h->stream));
      for (int i = 0; i < c1 - c0; ++i) {
        al.push_back(hs[2 * i]);
        be.push_back(hs[2 * i + 1]);
        if (hs[2 * i + 1] < 1e-12) {
          ended = true;
          break;
        }
      }
      bprev = be.back();
    }
    // largest eigenvalue of the tridiagonal matrix by bisection (Sturm count)
    const int k = (int)al.size();
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < k; ++i) {
      const double r = (i > 0 ? std::fabs(be[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(be[i]) : 0.0);
      lo = std::min(lo, al[i] - r);
      hi = std::max(hi, al[i] + r);
    }
    auto count_below = [&](double xv) {
      int cnt = 0;
      double d = 1.0;
      for (int i = 0; i < k; ++i) {
        const double b2 = i > 0 ? be[i - 1] * be[i - 1] : 0.0;
        d = al[i] - xv - (i > 0 ? b2 / d : 0.0);
        if (d == 0.0) d = -1e-300;
        if (d < 0) ++cnt;
      }
      return cnt;
    };
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (count_below(mid) >= k) hi = mid; else lo = mid;
    }
    *out = 1.01 * (hi + std::fabs(be[k - 1]));
    return PW_OK;
  }

  pw_status setup() {
    const Plan& p = P;
    const GridDesc& g = p.g;
    hipStream_t st = h->stream;
    // tables
    PW_HIP(hipMemcpyAsync(h->at<int>(p.lay.miller), p.miller.data(), sizeof(int) * p.miller.size(),
                          hipMemcpyHostToDevice, st));
    PW_HIP(hipMemcpyAsync(h->at<Stick>(p.lay.sticks), p.sticks.data(), sizeof(Stick) * p.sticks.size(),
                          hipMemcpyHostToDevice, st));
    PW_HIP(hipMemcpyAsync(h->at<int>(p.lay.colstart), p.colstart.data(), sizeof(int) * p.colstart.size(),
                          hipMemcpyHostToDevice, st));
    std::vector<T> kin(p.npw);
    for (int i = 0; i < p.npw; ++i) kin[i] = (T)p.kin[i];
    PW_HIP(hipMemcpyAsync(h->at<T>(p.lay.kin), kin.data(), sizeof(T) * p.npw, hipMemcpyHostToDevice, st));
    auto twid = [&](int n, size_t off) -> pw_status {
      std::vector<cplx<T>> tw(n);
      for (int m = 0; m < n; ++m) {
        const long double a = -2.0L * 3.14159265358979323846264338327950288L * m / n;
        tw[m] = mk<T>((T)std::cos(a), (T)std::sin(a));
      }
      PW_HIP(hipMemcpyAsync(h->at<cplx<T>>(off), tw.data(), sizeof(cplx<T>) * n, hipMemcpyHostToDevice, st));
      PW_HIP(hipStreamSynchronize(st));
      return PW_OK;
    };
    if (twid(g.n1, p.lay.tw1) != PW_OK || twid(g.n2, p.lay.tw2) != PW_OK || twid(g.n3, p.lay.tw3) != PW_OK)
      return PW_EDEVICE;
    const int nmodes = (int)p.mode_amp.size();
    if (p.natoms)
      PW_HIP(hipMemcpyAsync(h->at<double>(p.lay.frac), p.frac.data(), sizeof(double) * p.frac.size(),
                            hipMemcpyHostToDevice, st));
    if (nmodes) {
      PW_HIP(hipMemcpyAsync(h->at<int>(p.lay.mmil), p.mode_miller.data(), sizeof(int) * 3 * nmodes,
                            hipMemcpyHostToDevice, st));
      PW_HIP(hipMemcpyAsync(h->at<double>(p.lay.mamp), p.mode_amp.data(), sizeof(double) * nmodes,
                            hipMemcpyHostToDevice, st));
      PW_HIP(hipMemcpyAsync(h->at<double>(p.lay.mpha), p.mode_phase.data(), sizeof(double) * nmodes,
                            hipMemcpyHostToDevice, st));
    }
    const double ds[4] = {p.d0, p.d1, p.d1, p.d1};
    PW_HIP(hipMemcpyAsync(h->at<double>(p.lay.dscale), ds, sizeof(ds), hipMemcpyHostToDevice, st));
    // V(G) on the sphere -> V(r) on the grid (inverse FFT through the same stick/plane machinery)
    PotParams pp;
    for (int i = 0; i < 3; ++i) pp.L[i] = p.L[i];
    pp.zval = p.natoms ? p.zval : 0.0;
    pp.rc = p.rc;
    pp.gauss_c = p.natoms ? p.gauss_c : 0.0;
    pp.ecut = p.ecut;
    pp.natoms = p.natoms;
    pp.nmodes = nmodes;
    double2* vg = h->at<double2>(p.lay.vg);
    PW_HIP(launch_vg_sphere(h->at<int>(p.lay.miller), p.npw, h->at<double>(p.lay.frac), h->at<int>(p.lay.mmil),
                            h->at<double>(p.lay.mamp), h->at<double>(p.lay.mpha), pp, vg, st));
    cplx<T>* vgT = u0();
    PW_HIP(launch_convert_c64_to<T>(vg, p.npw, vgT, p.npw, p.npw, 1, st));
    {
      cplx<T>* SB = h->at<cplx<T>>(p.lay.sb);
      cplx<T>* G1 = h->at<cplx<T>>(p.lay.g1);
      const Stick* sti = h->at<Stick>(p.lay.sticks);
      const cplx<T>* tw1 = h->at<cplx<T>>(p.lay.tw1);
      const cplx<T>* tw2 = h->at<cplx<T>>(p.lay.tw2);
      T* vr = h->at<T>(p.lay.vr);
      PW_HIP(launch_sticks_inv<T>(vgT, p.npw, SB, 1, sti, g, h->at<cplx<T>>(p.lay.tw3), p.fl, st));
      if (p.fl.fused) {
        PW_HIP(launch_plane_fused<T>(SB, (const T*)nullptr, 1, sti, g, tw1, tw2, (T)1, 1, vr, p.fl, st));
      } else {
        PW_HIP(launch_pencil_yinv<T>(SB, G1, 1, sti, h->at<int>(p.lay.colstart), g, tw2, p.fl, st));
        PW_HIP(launch_pencil_x<T>(G1, (const T*)nullptr, 1, g, tw1, 1, vr, p.fl, st));
      }
    }
    if (p.nproj && beta_otf())
      PW_HIP(launch_beta_gen_tables(beta_gen(), h->at<double>(p.lay.frac), p.L, p.beta_sigma,
                                    h->at<double>(p.lay.brad), h->at<double2>(p.lay.bph), st));
    else if (p.nproj && beta_planes())
      PW_HIP(launch_beta_planes(h->at<int>(p.lay.miller), p.npw, h->at<double>(p.lay.frac), p.natoms, p.L,
                                p.beta_sigma, p.proj_form, beta_hi(), beta_lo(), p.ldw, st));
    else if (p.nproj && !p.rspace)
      PW_HIP(launch_beta_table<T>(h->at<int>(p.lay.miller), p.npw, h->at<double>(p.lay.frac), p.natoms, p.L,
                                  p.beta_sigma, p.proj_form, beta(), p.ldw, st));
    if (p.rspace) {
      auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpyAsync(h->at<char>(off), src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
      };
      PW_HIP(up(p.lay.rsat, p.rs_atoms.data(), sizeof(float) * p.rs_atoms.size()));
      PW_HIP(up(p.lay.rszo, p.rs_zoff.data(), sizeof(int) * p.rs_zoff.size()));
      PW_HIP(up(p.lay.rsze, p.rs_zent.data(), sizeof(RsEnt) * p.rs_zent.size()));
      PW_HIP(up(p.lay.rsbo, p.rs_boff.data(), sizeof(int) * p.rs_boff.size()));
      PW_HIP(up(p.lay.rsbe, p.rs_bent.data(), sizeof(RsEnt) * p.rs_bent.size()));
      PW_HIP(up(p.lay.rsao, p.rs_aoff.data(), sizeof(int) * p.rs_aoff.size()));
      PW_HIP(up(p.lay.rsae, p.rs_aent.data(), sizeof(int) * p.rs_aent.size()));
    }
    // the block planes' words past the last plane wave stay zero from here on (the cn products read them)
    if (p.yp_cols > 0) PW_HIP(launch_zero_plane_rows(yp_hi(), yp_lo(), p.ldw, p.npw, p.yp_cols, st));
    PW_HIP(hipStreamSynchronize(st));
    return PW_OK;
  }
};

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char* pw_status_string(pw_status s) {
  switch (s) {
    case PW_OK: return "ok";
    case PW_PENDING: return "pending";
    case PW_EINVAL: return "invalid argument";
    case PW_ENOMEM: return "out of memory";
    case PW_EDEVICE: return "device error";
    case PW_ENOTPD: return "Gram matrix not positive definite";
    case PW_ENUMERIC: return "non-finite result";
    case PW_ENOTCONV: return "not converged";
    case PW_EBUSY: return "busy";
  }
  return "unknown status";
}

const char* pw_last_error(const pw_handle* h) {
  if (h) return h->err.c_str();
  return g_last_error.c_str();
}

// LDS per workgroup of the current device (gfx950: 160 KB); the default when no device is visible.
static size_t device_max_lds() {
  int dev = 0, n = 0, lds = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return kDefaultMaxLds;
  }
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
    return std::min((size_t)lds, kDefaultMaxLds);
  (void)hipGetLastError();
  return kDefaultMaxLds;
}

static void fill_info(const Plan& p, pw_info* out) {
  out->npw = p.npw;
  out->nst = p.nst;
  out->nr = (long long)p.n[0] * p.n[1] * p.n[2];
  out->nproj = p.nproj;
  out->footprint_bytes = p.lay.total;
  for (int i = 0; i < 3; ++i) out->fft_n[i] = p.n[i];
  out->nbands = p.nbands;
  out->prec = p.prec;
  out->fused_planes = p.fl.fused ? 1 : 0;
  out->filter_block = p.nbb;
}

pw_status pw_plan(const pw_cell_desc* desc, pw_info* out) {
  if (!out) return fail(nullptr, PW_EINVAL, "null output");
  try {
    Plan p;
    std::string err;
    pw_status s = make_plan(desc, device_max_lds(), &p, &err);
    if (s != PW_OK) return fail(nullptr, s, err);
    fill_info(p, out);
    return PW_OK;
  } catch (const std::bad_alloc&) {
    return fail(nullptr, PW_ENOMEM, "host allocation failed");
  }
}

pw_status pw_plan_gvectors(const pw_cell_desc* desc, int* miller) {
  if (!miller) return fail(nullptr, PW_EINVAL, "null output");
  try {
    Plan p;
    std::string err;
    pw_status s = make_plan(desc, kDefaultMaxLds, &p, &err);
    if (s != PW_OK) return fail(nullptr, s, err);
    std::memcpy(miller, p.miller.data(), sizeof(int) * p.miller.size());
    return PW_OK;
  } catch (const std::bad_alloc&) {
    return fail(nullptr, PW_ENOMEM, "host allocation failed");
  }
}

pw_status pw_setup(const pw_cell_desc* desc, void* arena_dev, size_t arena_bytes, void* hip_stream,
                   pw_handle** out) {
  return pw::setup_handle(desc, arena_dev, arena_bytes, hip_stream, nullptr, out);
}

}  // extern "C"

namespace pw {

pw_status slot_resources_create(hipStream_t stream, SlotResources* r) {
  *r = SlotResources{};
  if (rocblas_create_handle(&r->blas) != rocblas_status_success) {
    r->blas = nullptr;
    return fail(nullptr, PW_EDEVICE, "rocblas_create_handle failed");
  }
  rocblas_set_stream(r->blas, stream);
  if (hipStreamCreateWithFlags(&r->aux, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&r->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&r->ev_join, hipEventDisableTiming) != hipSuccess) {
    slot_resources_destroy(r);
    return fail(nullptr, PW_EDEVICE, "stream or event creation failed");
  }
  return PW_OK;
}

void slot_resources_destroy(SlotResources* r) {
  if (r->aux) {
    hipStreamSynchronize(r->aux);
    hipStreamDestroy(r->aux);
  }
  if (r->ev_fork) hipEventDestroy(r->ev_fork);
  if (r->ev_join) hipEventDestroy(r->ev_join);
  if (r->blas) rocblas_destroy_handle(r->blas);
  *r = SlotResources{};
}

pw_status setup_handle(const pw_cell_desc* desc, void* arena_dev, size_t arena_bytes, void* hip_stream,
                       const SlotResources* res, pw_handle** out) {
  if (!out) return fail(nullptr, PW_EINVAL, "null handle pointer");
  *out = nullptr;
  if (!arena_dev) return fail(nullptr, PW_EINVAL, "null arena");
  if (reinterpret_cast<uintptr_t>(arena_dev) % kArenaAlign) return fail(nullptr, PW_EINVAL, "arena not 256-byte aligned");
  pw_handle_s* h = nullptr;
  try {
    h = new pw_handle_s();
  } catch (const std::bad_alloc&) {
    return fail(nullptr, PW_ENOMEM, "host allocation failed");
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    delete h;
    return fail(nullptr, PW_EDEVICE, "no HIP device");
  }
  h->device = dev;
  {
    std::string serr;
    h->scratch = scratch_address(dev, &serr);
    if (!h->scratch) {
      delete h;
      return fail(nullptr, PW_EDEVICE, serr);
    }
  }
  h->max_lds = device_max_lds();
  if (const char* e = std::getenv("PW_PROGRESS")) h->progress = e[0] == '1';
  std::string err;
  pw_status s;
  try {
    s = make_plan(desc, h->max_lds, &h->plan, &err);
  } catch (const std::bad_alloc&) {
    delete h;
    return fail(nullptr, PW_ENOMEM, "host allocation failed");
  }
  if (s != PW_OK) {
    delete h;
    return fail(nullptr, s, err);
  }
  if (arena_bytes < h->plan.lay.total) {
    const std::string m = "arena too small: need " + std::to_string(h->plan.lay.total) + " bytes";
    delete h;
    return fail(nullptr, PW_ENOMEM, m);
  }
  h->arena = static_cast<unsigned char*>(arena_dev);
  h->arena_bytes = arena_bytes;
  h->stream = static_cast<hipStream_t>(hip_stream);
  if (res) {
    // lent by a request-loop slot (same stream): no creation, no destruction per request
    h->lent = true;
    h->blas = res->blas;
    h->aux = res->aux;
    h->ev_fork = res->ev_fork;
    h->ev_join = res->ev_join;
  } else {
    if (rocblas_create_handle(&h->blas) != rocblas_status_success) {
      delete h;
      return fail(nullptr, PW_EDEVICE, "rocblas_create_handle failed");
    }
    rocblas_set_stream(h->blas, h->stream);
    if (hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess) {
      rocblas_destroy_handle(h->blas);
      delete h;
      return fail(nullptr, PW_EDEVICE, "stream or event creation failed");
    }
  }
  if (h->plan.fl.fused) {
    // allow large dynamic LDS for the fused plane kernels: once per process, so that no thread
    // changes a kernel's attributes while another (request loop worker) launches it
    static std::once_flag lds_once;
    std::call_once(lds_once, [] {
      pw_allow_large_lds();
      pw_allow_large_lds_plane_n();
    });
  }
  s = h->plan.prec == PW_FP64 ? Engine<double>(h).setup() : Engine<float>(h).setup();
  if (s != PW_OK) {
    g_last_error = h->err;
    if (!h->lent) rocblas_destroy_handle(h->blas);
    delete h;
    return s;
  }
  *out = h;
  return PW_OK;
}

}  // namespace pw

extern "C" {

pw_status pw_query(const pw_handle* h, pw_info* out) {
  if (!h || !out) return fail(nullptr, PW_EINVAL, "null argument");
  fill_info(h->plan, out);
  return PW_OK;
}

pw_status pw_get_gvectors(const pw_handle* h, int* miller) {
  if (!h || !miller) return fail(nullptr, PW_EINVAL, "null argument");
  std::memcpy(miller, h->plan.miller.data(), sizeof(int) * h->plan.miller.size());
  return PW_OK;
}

static pw_status check_block(pw_handle* h, const void* X, int nb, int ld) {
  if (!X) return fail(h, PW_EINVAL, "null block");
  if (nb < 1 || nb > h->plan.nbands) return fail(h, PW_EINVAL, "nb out of range [1, nbands]");
  if (ld < h->plan.npw) return fail(h, PW_EINVAL, "ld < npw");
  return PW_OK;
}

pw_status pw_apply_h(pw_handle* h, const void* X, void* HX, int nb, int ld) {
  if (!h) return fail(nullptr, PW_EINVAL, "null handle");
  pw_status s = check_block(h, X, nb, ld);
  if (s != PW_OK) return s;
  if (!HX) return fail(h, PW_EINVAL, "null output");
  const size_t cb = 2 * (size_t)h->plan.real_bytes;
  const char* x0 = static_cast<const char*>(X);
  const char* y0 = static_cast<const char*>(HX);
  const size_t span = ((size_t)(nb - 1) * ld + h->plan.npw) * cb;
  if (x0 < y0 + span && y0 < x0 + span) return fail(h, PW_EINVAL, "X and HX overlap");
  if (h->plan.prec == PW_FP64)
    return Engine<double>(h).apply_h(static_cast<const double2*>(X), static_cast<double2*>(HX), nb, ld,
                                     h->plan.nbb);
  return Engine<float>(h).apply_h(static_cast<const float2*>(X), static_cast<float2*>(HX), nb, ld, h->plan.nbb);
}

// Columns per H application that the static work array holds, and the placement of the work
// buffers in it; 0 when not even one column fits.
static int noalloc_layout(pw_handle* h, int nb) {
  const Plan& P = h->plan;
  const GridDesc& g = P.g;
  const size_t cb = 2 * (size_t)P.real_bytes;
  const size_t sb1 = (size_t)P.nst * g.n3 * cb;
  const size_t g11 = P.fl.fused ? 0 : (size_t)g.n3 * g.n2 * g.n1a * cb;
  const bool planes = P.real_bytes == 4 && (P.flags & PW_FLAG_BF16_KB) && P.nproj > 0;
  const size_t per_col = sb1 + g11 + (P.nproj ? 16 * (size_t)P.nsplit_proj * P.nproj + cb * P.nproj : 0) +
                         (planes ? 8 * (size_t)P.ldw : 0);
  const size_t slack = 5 * kArenaAlign;
  if (kScratchBytes <= slack) return 0;
  long w = (long)((kScratchBytes - slack) / per_col);
  w = std::min<long>(w, std::min(nb, P.nbb));
  if (w < 1) return 0;
  auto al = [](size_t x) { return (x + kArenaAlign - 1) / kArenaAlign * kArenaAlign; };
  const size_t fb = (size_t)std::min<long>(P.fft_batch, w);
  size_t off = 0;
  h->ws_sb = off;
  off = al(off + sb1 * fb);
  h->ws_g1 = off;
  off = al(off + g11 * fb);
  h->ws_parts = off;
  off = al(off + (P.nproj ? 16 * (size_t)P.nsplit_proj * P.nproj * w : 0));
  h->ws_pt = off;
  off = al(off + (P.nproj ? cb * P.nproj * w : 0));
  h->ws_yp = off;
  off = al(off + (planes ? 8 * (size_t)P.ldw * w : 0));
  if (off > kScratchBytes) return 0;
  h->ws_cols = (int)w;
  h->ws_fft_batch = (int)fb;
  return (int)w;
}

pw_status pw_apply_h_noalloc(pw_handle* h, const void* X, void* HX, int nb, int ld) {
  if (!h) return fail(nullptr, PW_EINVAL, "null handle");
  pw_status s = check_block(h, X, nb, ld);
  if (s != PW_OK) return s;
  if (!HX) return fail(h, PW_EINVAL, "null output");
  const size_t cb = 2 * (size_t)h->plan.real_bytes;
  const char* x0 = static_cast<const char*>(X);
  const char* y0 = static_cast<const char*>(HX);
  const size_t span = ((size_t)(nb - 1) * ld + h->plan.npw) * cb;
  if (x0 < y0 + span && y0 < x0 + span) return fail(h, PW_EINVAL, "X and HX overlap");
  if (!h->scratch) return fail(h, PW_EDEVICE, "no static work array on this device");
  if (h->plan.rspace)
    return fail(h, PW_EINVAL, "pw_apply_h_noalloc does not take handles with PW_FLAG_RSPACE_KB");
  const int w = noalloc_layout(h, nb);
  if (w < 1)
    return fail(h, PW_ENOMEM, "one band of this cell needs more than the " + std::to_string(kScratchBytes >> 20) +
                                  " MiB static work array of pw_apply_h_noalloc");
  // phase timers would create events: not recorded during this call
  const bool timing = h->timing;
  h->timing = false;
  h->ws = h->scratch;
  // the bf16 planes of the block live in the shared array: clear the words past the last plane
  // wave, which the projection reads as zeros
  if (h->plan.real_bytes == 4 && (h->plan.flags & PW_FLAG_BF16_KB) && h->plan.nproj > 0) {
    unsigned int* yh = reinterpret_cast<unsigned int*>(h->ws + h->ws_yp);
    if (launch_zero_plane_rows(yh, yh + (size_t)h->plan.ldw * w, h->plan.ldw, h->plan.npw, w, h->stream) !=
        hipSuccess) {
      h->ws = nullptr;
      h->timing = timing;
      return fail(h, PW_EDEVICE, "clearing the work array failed");
    }
  }
  if (h->plan.prec == PW_FP64)
    s = Engine<double>(h).apply_h(static_cast<const double2*>(X), static_cast<double2*>(HX), nb, ld, w);
  else
    s = Engine<float>(h).apply_h(static_cast<const float2*>(X), static_cast<float2*>(HX), nb, ld, w);
  // the planes bookkeeping refers to the work array only during this call
  h->ws = nullptr;
  h->timing = timing;
  h->yp_src = nullptr;
  h->yp_n = 0;
  h->wp_src = nullptr;
  return s;
}

pw_status pw_density(pw_handle* h, const void* X, int nb, int ld, const double* occ_host, void* rho_dev) {
  if (!h) return fail(nullptr, PW_EINVAL, "null handle");
  pw_status s = check_block(h, X, nb, ld);
  if (s != PW_OK) return s;
  if (!occ_host || !rho_dev) return fail(h, PW_EINVAL, "null occupations or output");
  for (int i = 0; i < nb; ++i)
    if (!std::isfinite(occ_host[i])) return fail(h, PW_EINVAL, "non-finite occupation");
  double* occ = h->at<double>(h->plan.lay.occ);
  if (hipMemcpyAsync(occ, occ_host, sizeof(double) * nb, hipMemcpyHostToDevice, h->stream) != hipSuccess)
    return fail(h, PW_EDEVICE, "occupation upload failed");
  s = h->plan.prec == PW_FP64
          ? Engine<double>(h).density(static_cast<const double2*>(X), nb, ld, occ, static_cast<double*>(rho_dev))
          : Engine<float>(h).density(static_cast<const float2*>(X), nb, ld, occ, static_cast<double*>(rho_dev));
  if (s != PW_OK) return s;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(h, PW_EDEVICE, "stream synchronise failed");
  return PW_OK;
}

pw_status pw_lobpcg_step(pw_handle* h, void* X, void* Pd, int nb, int ld, int have_p, double* eig, double* resid,
                         int* kept) {
  if (!h) return fail(nullptr, PW_EINVAL, "null handle");
  pw_status s = check_block(h, X, nb, ld);
  if (s != PW_OK) return s;
  if (!Pd || !eig || !resid) return fail(h, PW_EINVAL, "null directions or output");
  if (!(h->plan.flags & PW_FLAG_LOBPCG)) return fail(h, PW_EINVAL, "handle not planned with PW_FLAG_LOBPCG");
  const size_t cb = 2 * (size_t)h->plan.real_bytes;
  const char* x0 = static_cast<const char*>(X);
  const char* p0 = static_cast<const char*>(Pd);
  const size_t span = ((size_t)(nb - 1) * ld + h->plan.npw) * cb;
  if (x0 < p0 + span && p0 < x0 + span) return fail(h, PW_EINVAL, "X and P overlap");
  if (h->plan.prec == PW_FP64)
    return Engine<double>(h).lobpcg_step(static_cast<double2*>(X), static_cast<double2*>(Pd), nb, ld, have_p != 0,
                                         eig, resid, kept);
  return Engine<float>(h).lobpcg_step(static_cast<float2*>(X), static_cast<float2*>(Pd), nb, ld, have_p != 0, eig,
                                      resid, kept);
}

pw_status pw_ppcg_step(pw_handle* h, void* X, void* Pd, int nb, int ld, int have_p, double* eig, double* resid) {
  if (!h) return fail(nullptr, PW_EINVAL, "null handle");
  pw_status s = check_block(h, X, nb, ld);
  if (s != PW_OK) return s;
  if (!Pd || !eig || !resid) return fail(h, PW_EINVAL, "null directions or output");
  if (!(h->plan.flags & PW_FLAG_LOBPCG)) return fail(h, PW_EINVAL, "handle not planned with PW_FLAG_LOBPCG");
  const size_t cb = 2 * (size_t)h->plan.real_bytes;
  const char* x0 = static_cast<const char*>(X);
  const char* p0 = static_cast<const char*>(Pd);
  const size_t span = ((size_t)(nb - 1) * ld + h->plan.npw) * cb;
  if (x0 < p0 + span && p0 < x0 + span) return fail(h, PW_EINVAL, "X and P overlap");
  if (h->plan.prec == PW_FP64)
    return Engine<double>(h).ppcg_step(static_cast<double2*>(X), static_cast<double2*>(Pd), nb, ld, have_p != 0, eig,
                                       resid);
  return Engine<float>(h).ppcg_step(static_cast<float2*>(X), static_cast<float2*>(Pd), nb, ld, have_p != 0, eig,
                                    resid);
}

pw_status pw_eig_step(pw_handle* h, void* X, void* HX, int nb, int ld, const pw_step_params* p, double* eig,
                      double* resid, double bounds_out[3]) {
  if (!h) return fail(nullptr, PW_EINVAL, "null handle");
  pw_status s = check_block(h, X, nb, ld);
  if (s != PW_OK) return s;
  if (!p || !eig || !resid) return fail(h, PW_EINVAL, "null argument");
  if (p->degree < 0 || p->degree > 1000) return fail(h, PW_EINVAL, "degree out of range");
  if (p->want_hx && !HX) return fail(h, PW_EINVAL, "want_hx without HX");
  pw_step_params q = *p;
  if (q.degree > 0) {
    if (std::isnan(q.a_lo) || std::isnan(q.a)) {
      if (!std::isfinite(h->last_lo) || !std::isfinite(h->last_hi))
        return fail(h, PW_EINVAL, "NaN filter bounds need a previous step on this handle");
      if (std::isnan(q.a_lo)) q.a_lo = h->last_lo;
      if (std::isnan(q.a)) q.a = h->last_hi;
    }
    if (std::isnan(q.b)) {
      if (!std::isfinite(h->bmax_cached)) {
        double bb = 0.0;
        s = pw_spectrum_bound(h, 20, 1, &bb);
        if (s != PW_OK) return s;
        h->bmax_cached = bb;
      }
      q.b = h->bmax_cached;
    }
    if (!(std::isfinite(q.a_lo) && std::isfinite(q.a) && std::isfinite(q.b) && q.a_lo < q.a && q.a < q.b))
      return fail(h, PW_EINVAL, "filter bounds must satisfy a_lo < a < b");
  }
  if (h->plan.prec == PW_FP64)
    s = Engine<double>(h).eig_step(static_cast<double2*>(X), static_cast<double2*>(HX), nb, ld, q, eig, resid,
                                   bounds_out);
  else
    s = Engine<float>(h).eig_step(static_cast<float2*>(X), static_cast<float2*>(HX), nb, ld, q, eig, resid,
                                  bounds_out);
  if (s == PW_OK) {
    h->last_lo = eig[0];
    h->last_hi = eig[nb - 1];
  }
  return s;
}

pw_status pw_solve(pw_handle* h, void* X, int nb, int ld, int nconv, double tol, int degree, int max_steps,
                   double b, double* eig, double* resid, int* steps) {
  if (!h) return fail(nullptr, PW_EINVAL, "null handle");
  pw_status s = check_block(h, X, nb, ld);
  if (s != PW_OK) return s;
  if (!eig || !resid) return fail(h, PW_EINVAL, "null output");
  if (!(tol > 0.0) || degree < 1 || degree > 1000 || max_steps < 1 || nconv < 0 || nconv > nb)
    return fail(h, PW_EINVAL, "bad solve parameters (tol > 0, 1 <= degree <= 1000, max_steps >= 1, "
                              "0 <= nconv <= nb)");
  if (steps) *steps = 0;
  if (std::isnan(b)) {
    if (!std::isfinite(h->bmax_cached)) {
      s = pw_spectrum_bound(h, 20, 1, &h->bmax_cached);
      if (s != PW_OK) return s;
    }
    b = h->bmax_cached;
  }
  if (!std::isfinite(b)) return fail(h, PW_EINVAL, "non-finite filter bound b");
  const int nc = nconv > 0 ? nconv : nb;
  auto converged = [&]() {
    for (int i = 0; i < nc; ++i)
      if (!(resid[i] <= tol)) return false;
    return true;
  };
  pw_step_params p{0, NAN, NAN, b, 0};
  double bnd[3] = {0, 0, 0};
  int k = 0;
  h->solve_retries = 0;
  h->solve_retry_msg.clear();
  s = pw_eig_step(h, X, nullptr, nb, ld, &p, eig, resid, bnd);
  if (s == PW_OK) k = 1;
  const bool x_kept_on_failure = h->plan.nbb >= h->plan.nbands;  // the unblocked filter never writes X
  while (s == PW_OK && !converged() && k < max_steps) {
    p.degree = degree;
    p.a_lo = bnd[0];
    p.a = bnd[1];
    p.b = b;
    s = pw_eig_step(h, X, nullptr, nb, ld, &p, eig, resid, bnd);
    if (s == PW_ENOTPD && x_kept_on_failure && h->solve_retries == 0) {
      // X still holds the previous iterate: take the step again at half the degree (a smaller
      // spread of the filter's amplification), once
      h->solve_retries = 1;
      h->solve_retry_msg = "step " + std::to_string(k + 1) + ": " + h->err;
      p.degree = degree > 1 ? degree / 2 : 1;
      s = pw_eig_step(h, X, nullptr, nb, ld, &p, eig, resid, bnd);
    }
    if (s == PW_OK) ++k;
  }
  if (steps) *steps = k;
  if (s != PW_OK) {
    h->err = "step " + std::to_string(k + 1) + ": " + h->err;
    g_last_error = h->err;
    return s;
  }
  if (!converged()) return fail(h, PW_ENOTCONV, "max_steps reached before the tolerance");
  return PW_OK;
}

int pw_solve_retries(pw_handle* h, const char** msg) {
  if (!h) return -1;
  if (msg) *msg = h->solve_retries ? h->solve_retry_msg.c_str() : nullptr;
  return h->solve_retries;
}

pw_status pw_random_block(pw_handle* h, void* X, int nb, int ld, unsigned long long seed) {
  if (!h) return fail(nullptr, PW_EINVAL, "null handle");
  pw_status s = check_block(h, X, nb, ld);
  if (s != PW_OK) return s;
  if (h->plan.prec == PW_FP64) return Engine<double>(h).random_block(static_cast<double2*>(X), nb, ld, seed);
  return Engine<float>(h).random_block(static_cast<float2*>(X), nb, ld, seed);
}

pw_status pw_spectrum_bound(pw_handle* h, int steps, unsigned long long seed, double* bmax) {
  if (!h || !bmax) return fail(nullptr, PW_EINVAL, "null argument");
  if (steps < 2 || steps > 1000) return fail(h, PW_EINVAL, "steps out of range [2, 1000]");
  if (h->plan.prec == PW_FP64) return Engine<double>(h).spectrum_bound(steps, seed, bmax);
  return Engine<float>(h).spectrum_bound(steps, seed, bmax);
}

pw_status pw_set_timing(pw_handle* h, int on) {
  if (!h) return fail(nullptr, PW_EINVAL, "null handle");
  if (!on && !h->pending.empty()) {
    if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(h, PW_EDEVICE, "stream synchronise failed");
    h->resolve();
  }
  h->timing = on != 0;
  return PW_OK;
}

pw_status pw_get_stats(pw_handle* h, pw_phase_stat* out) {
  if (!h || !out) return fail(nullptr, PW_EINVAL, "null argument");
  if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(h, PW_EDEVICE, "stream synchronise failed");
  h->resolve();
  for (int i = 0; i < PW_NPHASES; ++i) out[i] = h->stats[i];
  return PW_OK;
}

pw_status pw_reset_stats(pw_handle* h) {
  if (!h) return fail(nullptr, PW_EINVAL, "null handle");
  if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(h, PW_EDEVICE, "stream synchronise failed");
  h->resolve();
  for (int i = 0; i < PW_NPHASES; ++i) h->stats[i] = pw_phase_stat{0, 0.0};
  return PW_OK;
}

pw_status pw_destroy(pw_handle* h) {
  if (!h) return PW_OK;
  if (h->stream) hipStreamSynchronize(h->stream);
  if (h->blas && !h->lent) rocblas_destroy_handle(h->blas);
  delete h;
  return PW_OK;
}

}  // extern "C"
