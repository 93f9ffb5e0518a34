// Host planner: plane-wave sphere, sticks, grid, radix plans and arena layout.
#pragma once

#include <string>
#include <vector>

#include "../../include/pw.h"
#include "common.hpp"
#include "kernels.hpp"

namespace pw {

constexpr size_t kArenaAlign = 256;
constexpr size_t kDefaultMaxLds = 160 * 1024;  // LDS per workgroup on gfx950
constexpr int kLanczosChunk = 64;  // Lanczos steps whose (alpha, beta) stay on the device between host reads

struct ArenaLayout {
  size_t miller, sticks, colstart, kin, tw1, tw2, tw3, vr, frac, mmil, mamp, mpha, vg, dscale;
  size_t beta, brad, bph, yp, u0, u1, zb, wf, sb, g1, pt, parts, sh, ct, ct2, eig, ework, resid, info, scal, lanc,
      occ, lz;
  size_t rsat, rszo, rsze, rsbo, rsbe, rsao, rsae, rsp;  // real-space projector tables and partials
  size_t total;
};

struct Plan {
  // copy of the description
  double L[3];
  double ecut;
  int natoms;
  std::vector<double> tau;  // 3 * natoms, Cartesian
  std::vector<double> frac; // 3 * natoms, fractional (tau / L)
  int nbands;
  double zval, rc, gauss_c, beta_sigma, d0, d1;
  std::vector<int> mode_miller;
  std::vector<double> mode_amp, mode_phase;
  int prec;
  unsigned flags;
  int real_bytes;  // 8 (FP64) or 4 (mixed)
  // basis
  int nmax[3];
  int n[3];
  int npw, nst, nproj;
  long ldw;  // internal leading dimension (npw rounded up to 16)
  std::vector<int> miller;     // 3 * npw, stick order
  std::vector<Stick> sticks;   // nst
  std::vector<int> colstart;   // n1a + 1: first stick of each active x column
  std::vector<double> kin;     // npw: |G|^2 / 2
  GridDesc g;
  FftLaunch fl;
  int fft_batch;               // bands per FFT launch group
  int nbb;                     // bands per filter block (== nbands: unblocked step)
  int nsplit_proj, nsplit_gram;
  int nsplit_lob;  // K splits of the LOBPCG basis Gram product (PW_FLAG_LOBPCG), else 0
  // bf16 plane columns held per plane: nbb, or 2 nbb when the unblocked step also keeps the
  // planes of H Y beside those of Y (split-precision projectors and Gram product)
  int yp_cols;
  int hmax[3];                 // max |n_d| over the sphere (projector generator tables)
  int bwidth;                  // per-atom axis-factor table length
  int proj_form;               // PW_PROJ_GSPACE or PW_PROJ_LOCALIZED
  // real-space projectors (PW_FLAG_RSPACE_KB): per-atom positions, the (atom, plane) entries per
  // plane and per (plane, 8-row band), and each atom's per-plane entries; see RsDesc
  bool rspace;
  double rs_radius;
  std::vector<float> rs_atoms;  // 4 per atom
  std::vector<int> rs_zoff, rs_boff, rs_aoff, rs_aent;
  std::vector<RsEnt> rs_zent, rs_bent;
  ArenaLayout lay;
};

// Fills `p` from `d`; returns PW_OK or PW_EINVAL with a message.
pw_status make_plan(const pw_cell_desc* d, size_t max_lds, Plan* p, std::string* err);

// 2^p 3^q test and radix plan
bool is_23_smooth(int n);
FftPlan radix_plan(int n);

}  // namespace pw
