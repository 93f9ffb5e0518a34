// Host planner.  The basis is every G = 2 pi (n1/L1, n2/L2, n3/L3) with |G|^2/2 <= ecut
// (Section II-A: the cutoff selects the plane waves and fixes the grid).  The grid
// follows the alias-free reading N_i = min 2^p 3^q >= 3 floor(nmax_i) + 1, which is
// the smallest grid on which the FFT application of a potential band-limited to the
// same sphere equals the textbook matrix element V(G - G') exactly.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

namespace pw {

static const double kTwoPi = 6.283185307179586476925;

bool is_23_smooth(int n) {
  if (n < 1) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

FftPlan radix_plan(int n) {
  FftPlan p;
  p.n = n;
  p.nrad = 0;
  int m = n, c2 = 0, c3 = 0;
  while (m % 2 == 0) { m /= 2; ++c2; }
  while (m % 3 == 0) { m /= 3; ++c3; }
  for (int i = 0; i < c2 / 2; ++i) p.rad[p.nrad++] = 4;
  if (c2 % 2) p.rad[p.nrad++] = 2;
  for (int i = 0; i < c3; ++i) p.rad[p.nrad++] = 3;
  return p;
}

static int smallest_23_at_least(int need) {
  int best = -1;
  for (long p2 = 1; p2 < 8L * need + 8; p2 *= 2)
    for (long p3 = p2; p3 < 8L * need + 8; p3 *= 3)
      if (p3 >= need && (best < 0 || p3 < best)) best = (int)p3;
  return best;
}

static size_t align_up(size_t x) { return (x + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }

// Tables of the real-space projectors.  Atom a (position wrapped into the cell) reaches the planes
// iz = ceil((z_a - R) / h_z) .. floor((z_a + R) / h_z) (unwrapped; plane iz mod n3), and within
// plane iz the columns and rows of the disc of radius sqrt(R^2 - dz^2), dz = iz h_z - z_a: one
// per-plane entry, and one per-band entry for each 8-row band the disc's rows meet.  The ranges
// use a radius enlarged by a relative 1e-4, so that they hold every point the kernels' FP32 test
// can accept; the kernels decide which points lie in the ball.  Each atom's per-plane entries are
// listed in plane order for the reduction.
static void build_rspace_tables(Plan& P) {
  const GridDesc& g = P.g;
  const int n3 = g.n3, nbr = 16;  // 128 rows in bands of 8
  const double h[3] = {P.L[0] / g.n1, P.L[1] / g.n2, P.L[2] / g.n3};
  const double R = P.rs_radius, Rs = R * (1.0 + 1e-4);
  P.rs_atoms.assign(4 * (size_t)P.natoms, 0.f);
  std::vector<std::vector<RsEnt>> per_z(n3), per_band((size_t)n3 * nbr);
  for (int a = 0; a < P.natoms; ++a) {
    double t[3];
    for (int i = 0; i < 3; ++i) {
      double v = std::fmod(P.tau[3 * a + i], P.L[i]);
      if (v < 0) v += P.L[i];
      t[i] = v;
      P.rs_atoms[4 * a + i] = (float)v;
    }
    const int z0 = (int)std::ceil((t[2] - Rs) / h[2]), z1 = (int)std::floor((t[2] + Rs) / h[2]);
    for (int iz = z0; iz <= z1; ++iz) {
      const int z = ((iz % n3) + n3) % n3;
      const float dz = (float)(iz * h[2] - t[2]);
      const double rho2 = Rs * Rs - (double)dz * dz;
      if (rho2 < 0) continue;
      const double rho = std::sqrt(rho2);
      const int x0 = (int)std::ceil((t[0] - rho) / h[0]), x1 = (int)std::floor((t[0] + rho) / h[0]);
      const int y0 = (int)std::ceil((t[1] - rho) / h[1]), y1 = (int)std::floor((t[1] + rho) / h[1]);
      if (x1 < x0 || y1 < y0) continue;
      RsEnt e{a, dz, (float)(x0 * h[0] - t[0]), (float)(y0 * h[1] - t[1]),
              (short)x0, (short)(x1 - x0 + 1), (short)y0, (short)(y1 - y0 + 1), 0, 0};
      for (int ix = x0; ix <= x1; ++ix) e.mask |= (unsigned short)(1u << ((((ix % 128) + 128) % 128) >> 3));
      per_z[z].push_back(e);
      std::vector<char> hit(nbr, 0);
      for (int iy = y0; iy <= y1; ++iy) hit[(((iy % 128) + 128) % 128) / 8] = 1;
      for (int w = 0; w < nbr; ++w)
        if (hit[w]) per_band[(size_t)z * nbr + w].push_back(e);
    }
  }
  // Balance the projection pass: wave w of a plane's workgroup takes positions w, w + 16, w + 32, ...
  // of the plane's list, so the entries are sorted by size (columns x rows) and dealt to the waves
  // in snake order (largest to waves 0 .. 15, the next 16 to waves 15 .. 0, ...).
  for (int z = 0; z < n3; ++z) {
    std::vector<RsEnt>& v = per_z[z];
    std::stable_sort(v.begin(), v.end(), [](const RsEnt& a, const RsEnt& b) {
      return (int)a.nx * a.ny > (int)b.nx * b.ny;
    });
    std::vector<RsEnt> dealt(v.size());
    const size_t full = v.size() / 16 * 16;  // entries in whole rounds; the rest go in order
    for (size_t r = 0; r < v.size(); ++r) {
      const size_t k = r / 16, i = r % 16;
      const size_t pos = r < full ? 16 * k + ((k % 2 == 0) ? i : 15 - i) : r;
      dealt[pos] = v[r];
    }
    v.swap(dealt);
  }
  P.rs_zoff.assign(n3 + 1, 0);
  P.rs_zent.clear();
  std::vector<std::vector<std::pair<int, int>>> of_atom(P.natoms);  // (unwrapped order key, zent index)
  for (int z = 0; z < n3; ++z) {
    P.rs_zoff[z] = (int)P.rs_zent.size();
    for (const RsEnt& e : per_z[z]) {
      of_atom[e.atom].push_back({z, (int)P.rs_zent.size()});
      P.rs_zent.push_back(e);
    }
  }
  P.rs_zoff[n3] = (int)P.rs_zent.size();
  P.rs_aoff.assign(P.natoms + 1, 0);
  P.rs_aent.clear();
  for (int a = 0; a < P.natoms; ++a) {
    P.rs_aoff[a] = (int)P.rs_aent.size();
    for (const auto& pr : of_atom[a]) P.rs_aent.push_back(pr.second);
  }
  P.rs_aoff[P.natoms] = (int)P.rs_aent.size();
  P.rs_boff.assign(per_band.size() + 1, 0);
  P.rs_bent.clear();
  for (size_t k = 0; k < per_band.size(); ++k) {
    P.rs_boff[k] = (int)P.rs_bent.size();
    P.rs_bent.insert(P.rs_bent.end(), per_band[k].begin(), per_band[k].end());
  }
  P.rs_boff[per_band.size()] = (int)P.rs_bent.size();
}

pw_status make_plan(const pw_cell_desc* d, size_t max_lds, Plan* p, std::string* err) {
  if (!d) { *err = "null description"; return PW_EINVAL; }
  for (int i = 0; i < 3; ++i)
    if (!(d->L[i] > 0.0) || !std::isfinite(d->L[i])) { *err = "cell lengths must be positive"; return PW_EINVAL; }
  if (!(d->ecut > 0.0) || !std::isfinite(d->ecut)) { *err = "ecut must be positive"; return PW_EINVAL; }
  if (d->natoms < 0 || (d->natoms > 0 && !d->tau)) { *err = "bad atoms"; return PW_EINVAL; }
  if (d->nbands < 1) { *err = "nbands must be >= 1"; return PW_EINVAL; }
  if (d->prec != PW_FP64 && d->prec != PW_MIXED) { *err = "unknown precision"; return PW_EINVAL; }
  const unsigned known = PW_FLAG_PENCIL_FFT | PW_FLAG_BF16_GRAM | PW_FLAG_BF16_KB | PW_FLAG_BF16_ROT |
                         PW_FLAG_BETA_OTF | PW_FLAG_LOBPCG | PW_FLAG_RSPACE_KB;
  if (d->flags & ~known) { *err = "unknown flag bits"; return PW_EINVAL; }
  if ((d->flags & PW_FLAG_BETA_OTF) && (d->flags & PW_FLAG_BF16_KB)) {
    *err = "PW_FLAG_BETA_OTF cannot be combined with PW_FLAG_BF16_KB";
    return PW_EINVAL;
  }
  if (d->prec == PW_FP64 && (d->flags & (PW_FLAG_BF16_GRAM | PW_FLAG_BF16_KB | PW_FLAG_BF16_ROT))) {
    *err = "bf16 split products need PW_MIXED";
    return PW_EINVAL;
  }
  if (d->nmodes < 0 || (d->nmodes > 0 && (!d->mode_miller || !d->mode_amp || !d->mode_phase))) {
    *err = "bad perturbation modes";
    return PW_EINVAL;
  }
  for (int k = 0; k < d->nmodes; ++k)
    if (!std::isfinite(d->mode_amp[k]) || !std::isfinite(d->mode_phase[k])) {
      *err = "non-finite perturbation mode";
      return PW_EINVAL;
    }
  if (!std::isfinite(d->zval) || !std::isfinite(d->rc) || !std::isfinite(d->gauss_c) || !std::isfinite(d->beta_sigma) ||
      !std::isfinite(d->d0) || !std::isfinite(d->d1)) {
    *err = "non-finite pseudopotential parameter";
    return PW_EINVAL;
  }
  const bool have_proj = (d->d0 != 0.0 || d->d1 != 0.0) && d->natoms > 0;
  if (have_proj && !(d->beta_sigma > 0.0)) { *err = "beta_sigma must be positive"; return PW_EINVAL; }
  if (d->proj_form != PW_PROJ_GSPACE && d->proj_form != PW_PROJ_LOCALIZED) {
    *err = "unknown projector form";
    return PW_EINVAL;
  }
  if (d->proj_form == PW_PROJ_LOCALIZED && (d->flags & PW_FLAG_BETA_OTF)) {
    *err = "PW_FLAG_BETA_OTF generates the PW_PROJ_GSPACE projectors only";
    return PW_EINVAL;
  }
  const bool rspace = (d->flags & PW_FLAG_RSPACE_KB) != 0;
  if (rspace) {
    if (d->proj_form != PW_PROJ_LOCALIZED) {
      *err = "PW_FLAG_RSPACE_KB needs proj_form = PW_PROJ_LOCALIZED";
      return PW_EINVAL;
    }
    if (d->prec != PW_MIXED) { *err = "PW_FLAG_RSPACE_KB needs PW_MIXED"; return PW_EINVAL; }
    if (d->flags & (PW_FLAG_BF16_KB | PW_FLAG_BETA_OTF | PW_FLAG_PENCIL_FFT)) {
      *err = "PW_FLAG_RSPACE_KB cannot be combined with PW_FLAG_BF16_KB, PW_FLAG_BETA_OTF or PW_FLAG_PENCIL_FFT";
      return PW_EINVAL;
    }
    if (!have_proj) { *err = "PW_FLAG_RSPACE_KB needs projectors (atoms and d0 or d1 nonzero)"; return PW_EINVAL; }
    if (!(d->rs_radius > 0.0) || !std::isfinite(d->rs_radius)) {
      *err = "PW_FLAG_RSPACE_KB needs rs_radius > 0";
      return PW_EINVAL;
    }
    for (int i = 0; i < 3; ++i)
      if (!(2.0 * d->rs_radius * (1.0 + 1e-4) < d->L[i])) {
        *err = "rs_radius must stay below half of every cell length";
        return PW_EINVAL;
      }
  }
  if (d->natoms > 0 && d->zval != 0.0 && !(d->rc > 0.0)) { *err = "rc must be positive"; return PW_EINVAL; }

  Plan& P = *p;
  for (int i = 0; i < 3; ++i) P.L[i] = d->L[i];
  P.ecut = d->ecut;
  P.natoms = d->natoms;
  P.tau.assign(d->tau ? d->tau : nullptr, d->tau ? d->tau + 3 * d->natoms : nullptr);
  P.frac.resize(3 * P.natoms);
  for (int a = 0; a < P.natoms; ++a)
    for (int i = 0; i < 3; ++i) {
      const double t = P.tau[3 * a + i];
      if (!std::isfinite(t)) { *err = "non-finite atom position"; return PW_EINVAL; }
      P.frac[3 * a + i] = t / P.L[i];
    }
  P.nbands = d->nbands;
  P.zval = d->zval;
  P.rc = d->rc;
  P.gauss_c = d->gauss_c;
  P.beta_sigma = d->beta_sigma;
  P.d0 = d->d0;
  P.d1 = d->d1;
  P.mode_miller.assign(d->mode_miller ? d->mode_miller : nullptr,
                       d->mode_miller ? d->mode_miller + 3 * d->nmodes : nullptr);
  P.mode_amp.assign(d->mode_amp ? d->mode_amp : nullptr, d->mode_amp ? d->mode_amp + d->nmodes : nullptr);
  P.mode_phase.assign(d->mode_phase ? d->mode_phase : nullptr, d->mode_phase ? d->mode_phase + d->nmodes : nullptr);
  P.prec = d->prec;
  P.flags = d->flags;
  P.proj_form = d->proj_form;
  P.rspace = rspace;
  P.rs_radius = rspace ? d->rs_radius : 0.0;
  P.real_bytes = d->prec == PW_FP64 ? 8 : 4;

  // --- sphere in stick order: n1, then n2, then n3 ascending -------------------
  const double r2 = 2.0 * P.ecut;  // |G|^2 <= 2 ecut
  for (int i = 0; i < 3; ++i) {
    P.nmax[i] = (int)std::floor(std::sqrt(r2) * P.L[i] / kTwoPi);
    if (P.nmax[i] > 4000) { *err = "cutoff too large for this cell"; return PW_EINVAL; }
  }
  P.miller.clear();
  P.sticks.clear();
  P.kin.clear();
  const double b0 = kTwoPi / P.L[0], b1 = kTwoPi / P.L[1], b2 = kTwoPi / P.L[2];
  for (int n1 = -P.nmax[0]; n1 <= P.nmax[0]; ++n1) {
    for (int n2 = -P.nmax[1]; n2 <= P.nmax[1]; ++n2) {
      const double g12 = (n1 * b0) * (n1 * b0) + (n2 * b1) * (n2 * b1);
      if (g12 > r2) continue;
      int h = (int)std::floor(std::sqrt(r2 - g12) / b2);
      while (g12 + ((h + 1) * b2) * ((h + 1) * b2) <= r2) ++h;
      while (h >= 0 && g12 + (h * b2) * (h * b2) > r2) --h;
      if (h < 0) continue;
      Stick s;
      s.off = (int)(P.miller.size() / 3);
      s.len = 2 * h + 1;
      s.n1 = n1;
      s.n2 = n2;
      P.sticks.push_back(s);
      for (int n3 = -h; n3 <= h; ++n3) {
        P.miller.push_back(n1);
        P.miller.push_back(n2);
        P.miller.push_back(n3);
        const double g2 = g12 + (n3 * b2) * (n3 * b2);
        P.kin.push_back(0.5 * g2);
      }
    }
  }
  P.npw = (int)P.kin.size();
  P.nst = (int)P.sticks.size();
  if (P.nbands > P.npw) { *err = "nbands exceeds the number of plane waves"; return PW_EINVAL; }
  P.nproj = have_proj ? 4 * P.natoms : 0;
  P.ldw = (P.npw + 15) / 16 * 16;

  // --- grid ----------------------------------------------------------------------
  const bool user_grid = d->fft_n[0] || d->fft_n[1] || d->fft_n[2];
  for (int i = 0; i < 3; ++i) {
    const int need = 3 * P.nmax[i] + 1;
    if (user_grid) {
      const int ni = d->fft_n[i];
      if (ni < need) { *err = "fft_n below the alias-free size 3*nmax+1"; return PW_EINVAL; }
      if (!is_23_smooth(ni)) { *err = "fft_n must be of the form 2^p 3^q"; return PW_EINVAL; }
      P.n[i] = ni;
    } else {
      P.n[i] = smallest_23_at_least(need);
    }
    if (P.n[i] > 512) { *err = "grid dimension above 512 is not supported"; return PW_EINVAL; }
  }
  int n1max = 0;
  for (const Stick& s : P.sticks) n1max = std::max(n1max, std::abs(s.n1));
  GridDesc& g = P.g;
  g.n1 = P.n[0];
  g.n2 = P.n[1];
  g.n3 = P.n[2];
  g.nst = P.nst;
  g.npw = P.npw;
  g.n1max = n1max;
  g.n1a = 2 * n1max + 1;
  g.p1 = radix_plan(g.n1);
  g.p2 = radix_plan(g.n2);
  g.p3 = radix_plan(g.n3);
  P.colstart.assign(g.n1a + 1, 0);
  {
    int s = 0;
    for (int xa = 0; xa < g.n1a; ++xa) {
      P.colstart[xa] = s;
      while (s < P.nst && P.sticks[s].n1 + n1max == xa) ++s;
    }
    P.colstart[g.n1a] = s;
  }
  if (!fft_plan_launch(g, P.real_bytes, (d->flags & PW_FLAG_PENCIL_FFT) ? 0 : max_lds, &P.fl)) {
    *err = "no FFT launch shape fits this grid";
    return PW_EINVAL;
  }
  if (P.rspace) {
    if (!P.fl.sized || g.n1 != 128 || g.n2 != 128 || g.n1a > 128) {
      *err = "PW_FLAG_RSPACE_KB needs a 128 x 128 x n3 grid whose planes fit in LDS";
      return PW_EINVAL;
    }
    build_rspace_tables(P);
  }

  // --- filter blocking -------------------------------------------------------------
  {
    const size_t col = (size_t)P.ldw * 2 * P.real_bytes;
    if (d->filter_block < 0) { *err = "filter_block must be >= 0"; return PW_EINVAL; }
    if (d->filter_block > 0) {
      P.nbb = std::min(d->filter_block, P.nbands);
    } else if (3 * col * (size_t)P.nbands <= (64ull << 30)) {
      P.nbb = P.nbands;
    } else {
      long b = (long)((16ull << 30) / (3 * col)) / 64 * 64;
      if (b < 64) b = 64;
      P.nbb = (int)std::min<long>(b, P.nbands);
    }
  }

  // --- batching ------------------------------------------------------------------
  const size_t cb = 2 * (size_t)P.real_bytes;
  const size_t per_band_sb = (size_t)P.nst * g.n3 * cb;
  const size_t per_band_g1 = P.fl.fused ? 0 : (size_t)g.n3 * g.n2 * g.n1a * cb;
  size_t budget = 192ull << 20;  // keep the stick/pencil intermediates of one batch cache-sized
  if (const char* e = std::getenv("PW_FFT_BATCH_MB")) budget = (size_t)std::atol(e) << 20;
  int fb = (int)(budget / (per_band_sb + per_band_g1));
  if (fb < 1) fb = 1;
  if (fb > P.nbb) fb = P.nbb;
  P.fft_batch = fb;
  // K splits: enough workgroups to fill the chip several times over (the pipelined split-bf16
  // forms run one workgroup per CU, and more, shorter chunks balance their tail: measured at
  // Si512, 57 splits of the projection and 49 of the Gram take 1.0 and 2 ms less than 29 and 25)
  auto pick_split = [](int tiles, int K, int target = 2048) {
    int s = (target + tiles - 1) / tiles;
    int kmax = K / 512;
    if (s > kmax) s = kmax;
    if (s > 64) s = 64;
    if (s < 1) s = 1;
    return s;
  };
  const bool f64 = P.prec == PW_FP64;
  const bool bkb = (P.flags & PW_FLAG_BF16_KB) != 0, bgr = (P.flags & PW_FLAG_BF16_GRAM) != 0;
  P.nsplit_proj = P.nproj ? (bkb ? pick_split(gemm_cn_bf16_planes_tiles(P.nproj, P.nbb), P.npw, 4096)
                                  : pick_split(gemm_cn_tiles(P.nproj, P.nbb, f64), P.npw))
                          : 1;
  // planes of Y and W for the Gram product: written by the nonlocal product's epilogue with
  // split-precision projectors, split from Y and W before the Gram product with real-space ones
  const bool gram_planes = (bkb || P.rspace) && bgr && P.nbb >= P.nbands;
  P.yp_cols = bkb ? P.nbb * (gram_planes ? 2 : 1) : (gram_planes ? 2 * P.nbb : 0);
  P.nsplit_gram = gram_planes ? pick_split(gemm_cn_bf16_planes_tiles(P.nbands, 2 * P.nbands), P.npw, 4096)
                  : pick_split(bgr ? gemm_cn_bf16_tiles(P.nbands, 2 * P.nbands)
                                   : gemm_cn_tiles(P.nbands, 2 * P.nbands, f64),
                               P.npw);
  const bool lob = (P.flags & PW_FLAG_LOBPCG) != 0;
  if (lob && P.nbb < P.nbands) {
    *err = "PW_FLAG_LOBPCG needs every band in one block (the plan would filter in blocks)";
    return PW_EINVAL;
  }
  P.nsplit_lob = lob ? pick_split(bgr ? gemm_cn_bf16_tiles(3 * P.nbands, 6 * P.nbands)
                                      : gemm_cn_tiles(3 * P.nbands, 6 * P.nbands, f64),
                                  P.npw)
                     : 0;
  const size_t kb = lob ? 3 * (size_t)P.nbands : (size_t)P.nbands;  // largest dense problem

  // --- arena layout --------------------------------------------------------------
  ArenaLayout& L = P.lay;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const size_t rb = P.real_bytes;
  const size_t nb = P.nbands;
  const size_t nr = (size_t)g.n1 * g.n2 * g.n3;
  L.miller = take(sizeof(int) * 3 * P.npw);
  L.sticks = take(sizeof(Stick) * P.nst);
  L.colstart = take(sizeof(int) * (g.n1a + 1));
  L.kin = take(rb * P.npw);
  L.tw1 = take(cb * g.n1);
  L.tw2 = take(cb * g.n2);
  L.tw3 = take(cb * g.n3);
  L.vr = take(rb * nr);
  L.frac = take(sizeof(double) * 3 * std::max(1, P.natoms));
  L.mmil = take(sizeof(int) * 3 * std::max<size_t>(1, P.mode_amp.size()));
  L.mamp = take(sizeof(double) * std::max<size_t>(1, P.mode_amp.size()));
  L.mpha = take(sizeof(double) * std::max<size_t>(1, P.mode_amp.size()));
  L.vg = take(sizeof(double) * 2 * P.npw);
  L.dscale = take(sizeof(double) * 4);
  const bool otf = (P.flags & PW_FLAG_BETA_OTF) != 0;
  for (int i = 0; i < 3; ++i) P.hmax[i] = 0;
  for (int gi = 0; gi < P.npw; ++gi)
    for (int i = 0; i < 3; ++i) P.hmax[i] = std::max(P.hmax[i], std::abs(P.miller[3 * gi + i]));
  P.bwidth = (2 * P.hmax[0] + 1) + (2 * P.hmax[1] + 1) + (2 * P.hmax[2] + 1);
  L.beta = take(otf || P.rspace ? 0 : cb * P.ldw * P.nproj);
  L.brad = take(otf ? sizeof(double) * 4 * P.npw : 0);
  L.bph = take(otf ? 16 * (size_t)P.natoms * P.bwidth : 0);
  const bool blocked = P.nbb < P.nbands;
  L.u0 = take(cb * P.ldw * P.nbb);
  L.u1 = take(cb * P.ldw * P.nbb);
  L.zb = take(cb * P.ldw * P.nbb);
  L.wf = take(blocked ? cb * P.ldw * nb : 0);
  L.sb = take(per_band_sb * P.fft_batch);
  L.g1 = take(per_band_g1 * P.fft_batch);
  L.pt = take(cb * std::max(1, P.nproj) * P.nbb);
  // bf16 hi/lo planes of the block entering the projector product (split-precision projectors)
  L.yp = take(8 * (size_t)P.ldw * P.yp_cols);
  const size_t parts = std::max({(size_t)P.nsplit_proj * P.nproj * P.nbb, (size_t)P.nsplit_gram * nb * 2 * nb,
                                  (size_t)P.nsplit_lob * kb * 2 * kb});
  L.parts = take(16 * parts);
  L.sh = take(16 * kb * 2 * kb);
  L.ct = take(cb * kb * kb);
  L.ct2 = take(blocked ? cb * nb * nb : 0);
  L.eig = take(sizeof(double) * kb);
  L.ework = take(sizeof(double) * kb);
  L.resid = take(sizeof(double) * nb);
  L.info = take(sizeof(int) * 4);
  L.scal = take(sizeof(double) * (8 + 2 * kLanczosChunk));  // scalars, then the Lanczos (alpha, beta) pairs
  L.lanc = take(cb * P.ldw * 3);
  L.occ = take(sizeof(double) * nb);  // band weights of the charge density
  // LOBPCG basis Z = [X R P] and HZ = [HX HR HP] (3 nbands columns each)
  L.lz = take(lob ? 2 * cb * P.ldw * 3 * nb : 0);
  const size_t nent = P.rs_zent.size();
  L.rsat = take(sizeof(float) * P.rs_atoms.size());
  L.rszo = take(sizeof(int) * P.rs_zoff.size());
  L.rsze = take(sizeof(RsEnt) * nent);
  L.rsbo = take(sizeof(int) * P.rs_boff.size());
  L.rsbe = take(sizeof(RsEnt) * P.rs_bent.size());
  L.rsao = take(sizeof(int) * P.rs_aoff.size());
  L.rsae = take(sizeof(int) * P.rs_aent.size());
  L.rsp = take(32 * nent * (size_t)(P.rspace ? P.fft_batch : 0));  // 4 complex FP32 per band and entry
  L.total = off;
  return PW_OK;
}

}  // namespace pw
