// Host-side launchers of the HIP kernels (all asynchronous on the given stream).
#pragma once

#include "common.hpp"

namespace pw {

// ---------------------------------------------------------------- FFT ------
struct FftLaunch {
  int spw;        // sticks per workgroup in the z pass
  int stick_thr;  // threads per workgroup in the z pass
  bool fused;     // whole plane in LDS
  bool sized;     // fused plane with a compile-time size kernel (register FFT stages)
  bool sized_sticks;  // z transforms with a compile-time size kernel
  int plane_thr;
  int cx, cy;     // columns / rows per workgroup in the pencil form
  int col_thr, row_thr;
};

bool fft_plan_launch(const GridDesc& g, int real_bytes, size_t max_lds, FftLaunch* L);

template <typename T>
hipError_t launch_sticks_inv(const cplx<T>* X, long ldx, cplx<T>* SB, int nbatch, const Stick* st,
                             const GridDesc& g, const cplx<T>* tw3, const FftLaunch& L, hipStream_t s);
template <typename T>
hipError_t launch_sticks_fwd(const cplx<T>* SB, cplx<T>* Z, long ldz, int nbatch, const Stick* st,
                             const GridDesc& g, const cplx<T>* tw3, const FftLaunch& L, hipStream_t s);
// Plane stage.  Fused form (whole plane in LDS): mode 0 = inverse 2D FFT, * V, forward 2D FFT,
// gather * scale; mode 1 = inverse only, real part to vout[z][y][x].
template <typename T>
hipError_t launch_plane_fused(cplx<T>* SB, const T* V, int nbatch, const Stick* st, const GridDesc& g,
                              const cplx<T>* tw1, const cplx<T>* tw2, T scale, int mode, T* vout, const FftLaunch& L,
                              hipStream_t s);
// Compile-time-size fused plane (square planes of supported sizes); mode 0 only.
bool sticks_n_supported(int n3);
template <typename T>
hipError_t launch_sticks_inv_n(const cplx<T>* X, long ldx, cplx<T>* SB, int nbatch, const Stick* st,
                               const GridDesc& g, const cplx<T>* tw3, hipStream_t s);
template <typename T>
hipError_t launch_sticks_fwd_n(const cplx<T>* SB, cplx<T>* Z, long ldz, int nbatch, const Stick* st,
                               const GridDesc& g, const cplx<T>* tw3, hipStream_t s);
bool plane_n_supported(int n1, int n2, int real_bytes, size_t max_lds);
// colstart: first stick of each active column xa = n1 + n1max (n1a + 1 entries; a column's sticks
// run over n2 = -m .. m in order).
template <typename T>
hipError_t launch_plane_n(cplx<T>* SB, const T* V, int nbatch, const Stick* st, const int* colstart,
                          const GridDesc& g, const cplx<T>* tw, T scale, hipStream_t s);
void pw_allow_large_lds_plane_n();
// Real-space projectors on 128 x 128 FP32 planes (sticks in SB as for the plane pass).
// Inverse pass: the projections of nbatch bands, one partial of 4 complex sums per band and
// (atom, plane) entry: part[(b nent + e) 4 + m].  SB is only read.
hipError_t launch_rs_proj128(const float2* SB, const int* colstart, const GridDesc& g, const float2* tw,
                             const RsDesc& rd, int nbatch, float2* part, hipStream_t s);
// Forward stick pass (sized sticks) with the Chebyshev update of u applied as the sphere values are
// written: out[b ldo + i] = alpha ((kin[i] - c) Y[b ldy + i] + z) - beta Yp[b ldp + i].
hipError_t launch_sticks_fwd_upd(const float2* SB, float2* out, long ldo, int nbatch, const Stick* st,
                                 const GridDesc& g, const float2* tw3, const StickUpd& u, hipStream_t s);
// dp[b nproj + 4a + m] = c_m dscale[m] inv_nr (sum over atom a's entries of part), b < nbt, with
// c_0 = rd.c0 and c_m = rd.c1 for m = 1, 2, 3 (the form the addition of D P reads).
hipError_t launch_rs_reduce(const float2* part, const RsDesc& rd, int nbt, const double* dscale, double inv_nr,
                            float2* dp, int nproj, hipStream_t s);
// The plane pass of k_plane128 with sum_a p_m(r - tau_a) dp[b nproj + 4a + m] added to V psi at the
// atoms' points before the forward transforms.
hipError_t launch_plane128_nl(float2* SB, const float* V, int nbatch, const int* colstart, const GridDesc& g,
                              const float2* tw, float scale, const RsDesc& rd, const float2* dp, int nproj,
                              hipStream_t s);
// Fused charge density of nbt bands on 128 x 128 FP32 planes (sticks in SB as for the plane
// pass): ngroups band groups per z plane, each group's FP64 sum of occ_b |psi_b|^2 in part
// (ngroups x 128 x 128 x n3 doubles), then rho = (first ? 0 : rho) + the group sums in order;
// with part == nullptr (or one group) the single group's sum goes straight into rho.
bool density128_supported(const GridDesc& g, int real_bytes);
hipError_t launch_density128(const float2* SB, const int* colstart, const GridDesc& g, const float2* tw,
                             const double* occ, int nbt, int ngroups, double* part, double* rho, bool first,
                             hipStream_t s);
// Pencil form: y inverse (sticks -> G1), x rows (inverse, * V, forward; mode 1: inverse only to vout),
// y forward (G1 -> sticks * scale).
template <typename T>
hipError_t launch_pencil_yinv(const cplx<T>* SB, cplx<T>* G1, int nbatch, const Stick* st, const int* colstart,
                              const GridDesc& g, const cplx<T>* tw2, const FftLaunch& L, hipStream_t s);
template <typename T>
hipError_t launch_pencil_x(cplx<T>* G1, const T* V, int nbatch, const GridDesc& g, const cplx<T>* tw1, int mode,
                           T* vout, const FftLaunch& L, hipStream_t s);
template <typename T>
hipError_t launch_pencil_yfwd(cplx<T>* SB, const cplx<T>* G1, int nbatch, const Stick* st, const int* colstart,
                              const GridDesc& g, const cplx<T>* tw2, T scale, const FftLaunch& L, hipStream_t s);

// --------------------------------------------------------------- GEMM ------
// C_part[s] = A^H B over the s-th K chunk.  A: K x M, B: K x N (column-major; columns of B
// with index >= nsplit_col come from B2).  Partials are complex double, [s][N][M].
// Number of output tiles of the cn kernel for an M x N result (used to choose the K split).
int gemm_cn_tiles(int M, int N, bool fp64);


template <typename T>
hipError_t launch_gemm_cn(const cplx<T>* A, long lda, const cplx<T>* B, long ldb, const cplx<T>* B2,
                          long ldb2, int ncol1, int M, int N, int K, int nsplit, double2* part, hipStream_t s);

// Sum the split partials: out[j*ldo + i] = scale_i * sum_s part[s][j][i]  (scale_i = dscale[i % dper]
// when dscale != null), written as complex double to out64 (if non-null) and as T to outT (if non-null).
template <typename T>
hipError_t launch_reduce_parts(const double2* part, int nsplit, int M, int N, const double* dscale, int dper,
                               double2* out64, long ldo64, cplx<T>* outT, long ldoT, hipStream_t s);

// Epilogue parameters of the row-major-tile GEMM C = A B:
//   out = alpha * ((kin_i - c) Y + Zl + acc) - beta * Yp      (EPI_H)
//   out = acc                                                  (EPI_STORE)
struct EpiH {
  int mode;  // 0 = store, 1 = H / Chebyshev update, 2 = out = acc + Zl
  double alpha, c, beta;
  const void* kin;  // T[M]
  const void* Y;
  long ldy;
  const void* Zl;
  long ldz;
  const void* Yp;  // may be null when beta == 0
  long ldp;
  // split-precision nn only, optional: bf16 hi/lo planes of out (one (re, im) word per entry,
  // leading dimension ldpl), for the next projector product
  void* ph;
  void* pl;
  long ldpl;
  // split-precision nn: set by the launcher when every epilogue array allows 16-byte accesses
  int vec4;
};

// Generator of the projector matrix inside the GEMM loaders, for cells whose table would not
// fit:  beta[g, 4a+m] = rad[4g+m] * ph_a(n1) ph_a(n2) ph_a(n3), where rad holds
// (c/sqrt(Omega)) e^{-sigma^2|G|^2/2} Y_m(G) per plane wave and ph_a the per-atom factors
// e^{-2 pi i n f_d(a)} of each axis d (f = fractional position), n from -h_d to h_d.
struct BetaGen {
  const int* miller;    // 3 * npw
  const double* rad;    // 4 * npw
  const double2* ph;    // natoms * w
  int h1, h2, h3;       // offsets of n = 0 in the three axis tables
  int o2, o3;           // start of the axis-2 and axis-3 tables within one atom's row
  int w;                // (2 h1 + 1) + (2 h2 + 1) + (2 h3 + 1)
  int npw, natoms;
};
// part[s] = beta^H B over K chunk s with beta generated on the fly (M = 4 natoms columns).
template <typename T>
hipError_t launch_gemm_cn_beta(const BetaGen& bg, const cplx<T>* B, long ldb, int N, int nsplit, double2* part,
                               hipStream_t s);
// out = epilogue(beta B) with beta generated on the fly (K = 4 natoms).
template <typename T>
hipError_t launch_gemm_nn_beta(const BetaGen& bg, const cplx<T>* B, long ldb, int N, cplx<T>* out, long ldo,
                               const EpiH& e, hipStream_t s);
// Tables of BetaGen: rad (npw x 4) and the per-atom axis factors (natoms x w).
hipError_t launch_beta_gen_tables(const BetaGen& bg, const double* frac, const double* L, double sigma,
                                  double* rad, double2* ph, hipStream_t s);
template <typename T>
hipError_t launch_gemm_nn(const cplx<T>* A, long lda, const cplx<T>* B, long ldb, int M, int N, int K,
                          cplx<T>* out, long ldo, const EpiH& e, hipStream_t s);


// Split-precision (bf16x3) forms of the two GEMM shapes, fp32 data.
int gemm_cn_bf16_tiles(int M, int N);
// tiles of the projection product with pre-split planes (launch_gemm_cn_bf16x3_planes)
int gemm_cn_bf16_planes_tiles(int M, int N);
// nterm = 3: hi*hi' + hi*lo' + lo*hi'; nterm = 4 adds lo*lo'.
hipError_t launch_gemm_cn_bf16x3(const float2* A, long lda, const float2* B, long ldb, const float2* B2, long ldb2,
                                 int ncol1, int M, int N, int K, int nsplit, double2* part, int nterm, hipStream_t s);
hipError_t launch_gemm_nn_bf16x3(const float2* A, long lda, const float2* B, long ldb, int M, int N, int K,
                                 float2* out, long ldo, const EpiH& e, hipStream_t s);
// The same products with pre-split bf16 planes (launch_beta_planes layout): cn with A and B given
// as planes of M and N columns of length K, nn with A = planes of K columns of length M.  Leading
// dimensions of planes count 32-bit words.
// herm_cols > 0: B's first herm_cols columns are A itself; the pipelined form may then skip the
// tiles of that Gram block that lie wholly below its diagonal (their partials are not written), so
// the caller must take the block's lower triangle from its upper one (launch_mirror_upper).
hipError_t launch_gemm_cn_bf16x3_planes(const unsigned int* Ahi, const unsigned int* Alo, long lda,
                                        const unsigned int* Bhi, const unsigned int* Blo, long ldb, int M, int N, int K,
                                        int nsplit, double2* part, hipStream_t s, int nterm = 3, int herm_cols = 0);
// The cn form on planes reads the words of each column from K up to the next multiple of 16 when
// both leading dimensions reach that far: those words must be zero.  The projector planes are
// written with zeros there; the block planes are cleared once (at set-up, or by
// launch_zero_plane_rows for planes in other memory) and never written there afterwards.
hipError_t launch_zero_plane_rows(unsigned int* H, unsigned int* L, long ld, int r0, int cols, hipStream_t s);
// hi/lo planes (one (re, im) word per entry, leading dimension ldp) of rows x cols fp32 complex.
hipError_t launch_split_planes(const float2* X, long ldx, int rows, int cols, unsigned int* H, unsigned int* L,
                               long ldp, hipStream_t s);
// nn with A = planes of K columns of length M and B = planes of N columns of length K holding
// (re, -im) words (launch_reduce_planes).
hipError_t launch_gemm_nn_bf16x3_planes(const unsigned int* Ahi, const unsigned int* Alo, long lda,
                                        const unsigned int* Bhi, const unsigned int* Blo, long ldb, int M, int N, int K,
                                        float2* out, long ldo, const EpiH& e, hipStream_t s);
// nn with fp32 A (M contiguous) and B planes as above.
hipError_t launch_gemm_nn_bf16x3_bplanes(const float2* A, long lda, const unsigned int* Bhi, const unsigned int* Blo,
                                         long ldb, int M, int N, int K, float2* out, long ldo, const EpiH& e,
                                         hipStream_t s);
// n x n FP64 matrix C (ldc), column j scaled by sc * lam[j] when lam is given, as nn B planes (ldp).
hipError_t launch_coef_planes(const double2* C, long ldc, int n, const double* lam, double sc, unsigned int* H,
                              unsigned int* L, long ldp, hipStream_t s);
// launch_reduce_parts into the nn B planes: the M x N sum over nsplit partials, row i scaled by
// dscale[i % dper], rounded to fp32 and split into words (re, -im) of hi and lo (leading dimension
// ldp, a multiple of 4 words).
hipError_t launch_reduce_planes(const double2* part, int nsplit, int M, int N, const double* dscale, int dper,
                                unsigned int* H, unsigned int* L, long ldp, hipStream_t s);

// --------------------------------------------------------------- misc ------
// LOBPCG pieces: per-column Rayleigh quotients theta_j = Re(x_j^H w_j) / |x_j|^2 (FP64), and the
// preconditioned residual block R = (W - X diag(theta)) / (1 + kin) (rows: plane waves).
template <typename T>
hipError_t launch_rayleigh(const cplx<T>* W, long ldw, const cplx<T>* X, long ldx, int rows, int cols, double* theta,
                           hipStream_t s);
template <typename T>
hipError_t launch_precond_resid(const cplx<T>* W, long ldw, const cplx<T>* X, long ldx, const double* theta,
                                const T* kin, int rows, int cols, cplx<T>* R, long ldr, hipStream_t s);
// PPCG pieces (solver.hip): per-column FP64 inner products of x_j, w_j, p_j and H w_j, H p_j
// (11 per column, see k_ppcg_dots), the per-column Rayleigh-Ritz on span{x_j, w_j, p_j} (coef:
// 3 per column), and the update X <- a X + b W + g P, Pd <- b W + g P.
template <typename T>
hipError_t launch_ppcg_dots(const cplx<T>* X, long ldx, const cplx<T>* W, const cplx<T>* Pp, const cplx<T>* HW,
                            const cplx<T>* HP, long ldz, int rows, int cols, int have_p, double2* dots,
                            hipStream_t s);
hipError_t launch_ppcg_small(const double2* dots, const double* lam, int nb, int have_p, double drop_tol,
                             double2* coef, hipStream_t s);
template <typename T>
hipError_t launch_ppcg_update(cplx<T>* X, long ldx, cplx<T>* Pd, long ldp, const cplx<T>* W, const cplx<T>* Pp,
                              long ldz, int rows, int cols, int have_p, const double2* coef, hipStream_t s);
// Truncated SVQB basis of a k x k Gram matrix: S <- D S D with d_i = S_ii^-1/2 (d: k doubles), and
// T[:, c] = D U[:, first + c] / sqrt(sigma[first + c]) for c < kept.
// Pivot test of a Cholesky factor: d = Re diag(S) before the factorisation, then
// out = min_i |L_ii|^2 / d_i (one double, device).
hipError_t launch_diag_copy(const double2* S, long lds, int k, double* d, hipStream_t s);
hipError_t launch_min_pivot(const double2* L, long ldl, int k, const double* d, double* out, hipStream_t s);
hipError_t launch_svqb_scale(double2* S, long lds, int k, double* d, hipStream_t s);
hipError_t launch_svqb_basis(const double2* U, long ldu, int k, const double* sigma, const double* d, int first,
                             int kept, double2* Tm, long ldt, hipStream_t s);
// Charge density: rho[r] = (first ? 0 : rho[r]) + sum_b occ[b] psq[b * nr + r], bands in order.
template <typename T>
hipError_t launch_density_acc(const T* psq, int nbt, long nr, const double* occ, double* rho, bool first,
                              hipStream_t s);
template <typename T>
hipError_t launch_fill_zero(cplx<T>* p, long n, hipStream_t s);

// V(G) on the sphere (complex double) from the analytic pseudopotential and structure factors
struct PotParams {
  double L[3];
  double zval, rc, gauss_c, ecut;
  int natoms;
  int nmodes;
};
hipError_t launch_vg_sphere(const int* miller, int npw, const double* frac, const int* mode_miller,
                            const double* mode_amp, const double* mode_phase, PotParams p, double2* vg,
                            hipStream_t s);
// beta[g, 4a+m] table (column-major, ld)
template <typename T>
hipError_t launch_beta_table(const int* miller, int npw, const double* frac, int natoms, const double* L,
                             double sigma, int form, cplx<T>* beta, long ld, hipStream_t s);
// Projector table as bf16 hi/lo planes (one 32-bit (re, im) word per entry, column-major, leading
// dimension ld; rows npw..ld-1 zero), for the split-precision projector GEMMs.
hipError_t launch_beta_planes(const int* miller, int npw, const double* frac, int natoms, const double* L,
                              double sigma, int form, unsigned int* hi, unsigned int* lo, long ld, hipStream_t s);
template <typename T>
hipError_t launch_convert_c64_to(const double2* in, long ldi, cplx<T>* out, long ldo, int rows, int cols,
                                 hipStream_t s);
template <typename T>
hipError_t launch_copy_cols(const cplx<T>* in, long ldi, cplx<T>* out, long ldo, int rows, int cols,
                            hipStream_t s);
// out[:, j] = s * lam[j] * in[:, j] (complex double in, T out), n x n
template <typename T>
hipError_t launch_scale_cols_lam(const double2* in, long ldi, cplx<T>* out, long ldo, int n, const double* lam,
                                 double s, hipStream_t st);
// Hermitian part: A <- (A + A^H)/2, n x n complex double
hipError_t launch_hermitize(double2* A, long lda, int n, hipStream_t s);
// Hermitian matrix from its upper triangle: A(i, j) <- conj(A(j, i)) for i > j, Im A(i, i) <- 0
hipError_t launch_mirror_upper(double2* A, long lda, int n, hipStream_t s);
// r_j = || W_j - lam_j X_j ||_2 with double accumulation; flag[0] |= non-finite seen
template <typename T>
hipError_t launch_resid(const cplx<T>* W, long ldw, const cplx<T>* X, long ldx, const double* lam, int rows,
                        int cols, double* resid, hipStream_t s);

// Lanczos: alpha = Re<v, w>; w <- w - alpha v - beta_prev v_prev; beta = ||w||.  sc[0..1] = alpha, beta.
// beta_prev is read from beta_prev_dev when that is not null (the previous step's sc[1]).
template <typename T>
hipError_t launch_lanczos_step(cplx<T>* w, const cplx<T>* v, const cplx<T>* vp, double beta_prev,
                               const double* beta_prev_dev, int n, double* sc, hipStream_t s);
// out = in / *beta (zero when *beta < 1e-12, where the recurrence ends)
template <typename T>
hipError_t launch_scale_copy_inv(const cplx<T>* in, cplx<T>* out, const double* beta, int n, hipStream_t s);
// Seeded random block (see pw_random_block) and per-column scaling by 1 / norm.
template <typename T>
hipError_t launch_random_block(cplx<T>* X, long ld, int npw, int nb, const T* kin, unsigned long long seed,
                               hipStream_t s);
template <typename T>
hipError_t launch_scale_cols_inv(cplx<T>* X, long ld, int npw, int nb, const double* norms, hipStream_t s);
// Opt the fused plane kernels in to the full LDS of a workgroup.
void pw_allow_large_lds();

}  // namespace pw
