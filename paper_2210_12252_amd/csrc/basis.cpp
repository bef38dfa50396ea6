// Host set-up of a helical-wave basis and the host-only C ABI entry points.
//
// Index set (Sec. 3.2, eq. Energy_cutoff, applied at the Bloch parameter eta
// with the shifted kinetic energy): every (m, n, k) with
//   kappa = 1/2 [ (b_k^{|n|}/R)^2 + (2 pi/tau)^2 (m - alpha n - eta)^2 ] <= E_cut
// inside the clamps.  Because kappa grows with k at fixed (m, n), the kept k
// of a mode form a prefix 1..K (the mask of Sec. 3.2 becomes a ragged length).
// Radial functions (App. B): xi_{n,k}(r) = J_n(b r/R) / (sqrt(pi tau) R
// J_{n+1}(b)); with J_{-n} = (-1)^n J_n and J_{n-1}(b) = -J_{n+1}(b) at a zero
// of J_n, xi_{-n,k} = xi_{n,k}, so one table per |n| serves both signs.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "helic_internal.h"
#include "setup_math.h"

namespace helic {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

helic_status fail(helic_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

namespace {

constexpr double TIE_TOL = 1e-10;
constexpr double PI = 3.14159265358979323846;

// Nearest bfloat16 (ties to even) of a finite double, via its float value.
uint16_t bf16_round(double v) {
  const float f = (float)v;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

std::vector<int32_t> radix_plan(int n) {
  std::vector<int32_t> f;
  while (n % 4 == 0) { f.push_back(4); n /= 4; }
  while (n % 3 == 0) { f.push_back(3); n /= 3; }
  while (n % 5 == 0) { f.push_back(5); n /= 5; }
  while (n % 2 == 0) { f.push_back(2); n /= 2; }
  if (n != 1) f.clear();
  return f;
}

helic_status build(helic_basis_s* h) {
  const helic_params& p = h->p;
  if (p.ncyc < 1 || p.ncyc > 64) return fail(HELIC_ERR_INVALID, "cyclic order must be 1..64");
  if (p.nu < 0 || p.nu >= p.ncyc) return fail(HELIC_ERR_INVALID, "cyclic Bloch index nu must be 0..ncyc-1");
  if (!(p.R > 0) || !(p.tau > 0) || !(p.ecut > 0) || !(p.alpha >= 0.0 && p.alpha < 1.0) ||
      !(p.eta >= -0.5 && p.eta < 0.5) || !std::isfinite(p.R) || !std::isfinite(p.tau) ||
      !std::isfinite(p.ecut))
    return fail(HELIC_ERR_INVALID, "invalid R, tau, alpha, ecut or eta");
  if ((p.n_t1 > 0) != (p.n_t2 > 0) || p.n_t1 < 0 || p.n_t2 < 0 || p.n_r < 0)
    return fail(HELIC_ERR_INVALID, "give both angular grid sizes (> 0) or neither (0)");
  const bool grid_given = p.n_t1 > 0;
  int m_max = p.m_max, n_max = p.n_max;
  if (grid_given) {
    if (m_max < 0) m_max = (p.n_t1 - 1) / 2;
    if (n_max < 0) n_max = (p.n_t2 - 1) / 2;
  }
  const double R = p.R, tau = p.tau, ecut = p.ecut, alpha = p.alpha, eta = p.eta;
  // cyclic order N and index nu: mode (m, n) carries exp(i 2 pi (m theta1 +
  // n N theta2)) (Sec. 2.3; theta2 spans [0, 1/N)) and the radial functions of
  // order p = n N - nu.  At nu = 0 these are the paper's J_{|n| N}.  For
  // nu != 0 the paper keeps J_{nN} and adds the nu^2 / (2 r^2) and
  // (i nu / (2 pi r^2)) d/dtheta2 terms of eq. Simplify_2 through the
  // integrals of eq. I_nkk_prime, which diverge for n = 0; on
  // exp(i 2 pi n N theta2) those terms turn the Bessel operator of order nN
  // into that of order nN - nu, so order |nN - nu| diagonalises the same
  // operator's kinetic part (no integral table).  A group holds the modes of
  // one Bessel order: n = +-g at nu = 0, usually a single n otherwise.
  const int N = p.ncyc, nu = p.nu;
  const double w = 2.0 * PI / tau;
  const double xmax = R * std::sqrt(2.0 * ecut);   // largest admissible zero
  auto order = [&](int n) { return std::abs(n * N - nu); };
  int n_lo = -n_max, n_hi = n_max;
  if (n_max < 0) {
    n_hi = 0;
    while (bessel_zeros(order(n_hi + 1), 1)[0] <= xmax * (1.0 + 1e-15)) ++n_hi;
    n_lo = 0;
    while (bessel_zeros(order(n_lo - 1), 1)[0] <= xmax * (1.0 + 1e-15)) --n_lo;
  }
  // orders in increasing value, each with its angular indices (larger n first)
  std::vector<std::pair<int, std::vector<int>>> ords;
  for (int n = n_hi; n >= n_lo; --n) {
    const int o = order(n);
    auto it = std::find_if(ords.begin(), ords.end(), [&](const std::pair<int, std::vector<int>>& e) {
      return e.first == o;
    });
    if (it == ords.end()) ords.push_back({o, {n}});
    else it->second.push_back(n);
  }
  std::sort(ords.begin(), ords.end(),
            [](const std::pair<int, std::vector<int>>& a, const std::pair<int, std::vector<int>>& b) {
              return a.first < b.first;
            });
  h->modes.clear();
  h->groups.clear();
  int64_t row = 0;
  for (const auto& on : ords) {
    const int po = on.first;
    // zeros of J_po below xmax (at most k_max of them)
    int cnt = (int)(xmax / PI) + 4;
    if (p.k_max > 0) cnt = std::min(cnt, p.k_max);
    std::vector<double> z = bessel_zeros(po, cnt);
    while (p.k_max <= 0 && z.back() <= xmax) {
      cnt *= 2;
      z = bessel_zeros(po, cnt);
    }
    Group grp;
    grp.g = po;
    grp.mode0 = (int32_t)h->modes.size();
    grp.row0 = row;
    grp.Kmax = 0;
    const double span = std::sqrt(2.0 * ecut) / w + 1.0;
    for (const int n : on.second) {
      const double c0 = alpha * (n * N - nu) + eta;
      int mlo = (int)std::floor(c0 - span), mhi = (int)std::ceil(c0 + span);
      if (m_max >= 0) { mlo = std::max(mlo, -m_max); mhi = std::min(mhi, m_max); }
      for (int m = mlo; m <= mhi; ++m) {
        const double ax = w * (m - alpha * (n * N - nu) - eta);
        int K = 0;
        for (size_t k = 0; k < z.size(); ++k) {
          const double kap = 0.5 * ((z[k] / R) * (z[k] / R) + ax * ax);
          if (std::fabs(kap - ecut) < TIE_TOL)
            return fail(HELIC_ERR_CUTOFF_TIE, "cutoff tie: a kinetic energy equals E_cut within 1e-10 Ha");
          if (kap <= ecut) K = (int)k + 1; else break;
        }
        if (K == 0) continue;
        Mode md;
        md.m = m; md.n = n; md.g = std::abs(n); md.K = K; md.row0 = row;
        md.bin1 = md.bin2 = 0;
        h->modes.push_back(md);
        row += K;
        grp.Kmax = std::max(grp.Kmax, K);
      }
    }
    grp.nmodes = (int32_t)h->modes.size() - grp.mode0;
    grp.nrows = row - grp.row0;
    if (grp.nmodes == 0) continue;
    // Storage order of the group's modes (the slab layout of the
    // intermediates; rows keep the compact order through row0): K
    // descending, so the 8 modes of a 16-column MFMA tile of the radial
    // stages have similar K, and a tile's work ends at the K of its first
    // mode (the radial kernels rely on this order).
    std::stable_sort(h->modes.begin() + grp.mode0, h->modes.end(),
                     [](const Mode& a, const Mode& b) { return a.K > b.K; });
    grp.zeros.assign(z.begin(), z.begin() + grp.Kmax);
    h->groups.push_back(grp);
  }
  h->L = row;
  if (h->L == 0) return fail(HELIC_ERR_INVALID, "empty basis: no function below the cutoff");
  int mlo = 1 << 30, mhi = -(1 << 30), nabs = 0, kmx = 0;
  for (const Mode& md : h->modes) {
    mlo = std::min(mlo, md.m); mhi = std::max(mhi, md.m);
    nabs = std::max(nabs, md.g); kmx = std::max(kmx, md.K);
  }
  if (grid_given) {
    h->n_t1 = p.n_t1; h->n_t2 = p.n_t2;
  } else {
    int mabs = std::max(std::abs(mlo), std::abs(mhi));
    h->n_t1 = smooth_at_least(2 * mabs + 2);
    h->n_t2 = smooth_at_least(2 * nabs + 2);
  }
  h->n_r = p.n_r > 0 ? p.n_r : 4 * kmx;
  if (mhi - mlo + 1 > h->n_t1 || 2 * nabs + 1 > h->n_t2)
    return fail(HELIC_ERR_GRID, "angular grid does not resolve the index set");
  h->fac1 = radix_plan(h->n_t1);
  h->fac2 = radix_plan(h->n_t2);
  if (h->fac1.empty() || h->fac2.empty())
    return fail(HELIC_ERR_GRID, "angular grid sizes must have prime factors 2, 3, 5 only");
  if (h->n_r > 4096) return fail(HELIC_ERR_GRID, "n_r above 4096");

  // compact index list, kinetic diagonal, per-row (local mode, k) and bins
  h->mnk.resize(3 * h->L);
  h->kappa.resize(h->L);
  h->row_ck.resize(h->L);
  std::vector<char> has_row1(h->n_t1, 0);
  for (const Group& grp : h->groups) {
    for (int c = 0; c < grp.nmodes; ++c) {
      Mode& md = h->modes[grp.mode0 + c];
      md.bin1 = ((md.m % h->n_t1) + h->n_t1) % h->n_t1;
      md.bin2 = ((md.n % h->n_t2) + h->n_t2) % h->n_t2;
      has_row1[md.bin1] = 1;
      const double ax = w * (md.m - alpha * (md.n * N - nu) - eta);
      for (int k = 0; k < md.K; ++k) {
        const int64_t r = md.row0 + k;
        h->mnk[3 * r] = md.m; h->mnk[3 * r + 1] = md.n; h->mnk[3 * r + 2] = k + 1;
        const double b = grp.zeros[k] / R;
        h->kappa[r] = 0.5 * (b * b + ax * ax);
        h->row_ck[r] = (c << 16) | k;
      }
    }
  }
  h->rows1.clear();
  for (int i = 0; i < h->n_t1; ++i)
    if (has_row1[i]) h->rows1.push_back(i);

  // grid
  h->theta1.resize(h->n_t1);
  h->theta2.resize(h->n_t2);
  for (int i = 0; i < h->n_t1; ++i) h->theta1[i] = (double)i / h->n_t1;
  for (int j = 0; j < h->n_t2; ++j) h->theta2[j] = (double)j / ((double)N * h->n_t2);
  h->q.resize(h->n_r);
  h->wq.resize(h->n_r);
  gauss_jacobi01(h->n_r, h->q.data(), h->wq.data());

  // radial tables, packed in MFMA fragment order per group
  const int nr = h->n_r;
  const int nrt = (nr + 15) / 16, nrs = (nr + 3) / 4;
  int64_t inv_total = 0, fwd_total = 0;
  h->max_kpad = 0;
  h->max_colpad = 0;
  int64_t inv16_total = 0, fwd16_total = 0;
  for (Group& grp : h->groups) {
    const int nks = (grp.Kmax + 3) / 4, nkt = (grp.Kmax + 15) / 16;
    grp.tinv_off = inv_total;
    grp.tfwd_off = fwd_total;
    inv_total += (int64_t)nrt * nks * FRAG;
    fwd_total += (int64_t)nkt * nrs * FRAG;
    grp.tinv16_off = inv16_total;
    grp.tfwd16_off = fwd16_total;
    inv16_total += (int64_t)nrt * nkt * FRAG;
    fwd16_total += (int64_t)nkt * ((nr + 15) / 16) * FRAG;
    h->max_kpad = std::max(h->max_kpad, 4 * nks);
    h->max_colpad = std::max(h->max_colpad, 16 * ((2 * grp.nmodes + 15) / 16));
  }
  h->tab_inv.assign(inv_total, 0.0);
  h->tab_dinv.assign(inv_total, 0.0);
  h->tab_fwd.assign(fwd_total, 0.0);
  h->tab_inv16.assign(inv16_total * 4, 0);
  h->tab_fwd16.assign(fwd16_total * 4, 0);
  const double norm0 = std::sqrt((double)N / (PI * tau)) / R;
  std::vector<double> jv(2);
  for (const Group& grp : h->groups) {
    const int nks = (grp.Kmax + 3) / 4;
    const int g = grp.g;   // Bessel order of the group
    std::vector<double> xi((size_t)nr * grp.Kmax);   // xi[l * Kmax + k]
    std::vector<double> dxi((size_t)nr * grp.Kmax);  // d xi / dr
    std::vector<double> buf(g + 2), buf2(g + 2);
    for (int k = 0; k < grp.Kmax; ++k) {
      const double b = grp.zeros[k];
      bessel_j_all(g + 1, b, buf.data());
      const double c = norm0 / buf[g + 1];
      for (int l = 0; l < nr; ++l) {
        bessel_j_all(g, b * h->q[l], buf.data());
        xi[(size_t)l * grp.Kmax + k] = c * buf[g];
        // J_g' = (J_{g-1} - J_{g+1}) / 2, with J_{-1} = -J_1
        bessel_j_all(g + 1, b * h->q[l], buf2.data());
        const double jm1 = g > 0 ? buf2[g - 1] : -buf2[1];
        dxi[(size_t)l * grp.Kmax + k] = c * (b / R) * 0.5 * (jm1 - buf2[g + 1]);
      }
    }
    for (int t = 0; t < nrt; ++t)
      for (int s = 0; s < nks; ++s)
        for (int ln = 0; ln < FRAG; ++ln) {
          const int l = 16 * t + ln % 16, k = 4 * s + ln / 16;
          if (l < nr && k < grp.Kmax) {
            h->tab_inv[grp.tinv_off + ((int64_t)t * nks + s) * FRAG + ln] = xi[(size_t)l * grp.Kmax + k];
            h->tab_dinv[grp.tinv_off + ((int64_t)t * nks + s) * FRAG + ln] = dxi[(size_t)l * grp.Kmax + k];
          }
        }
    const double pref = 2.0 * PI * tau / N;   // 2 pi tau / N (Alg. 3)
    for (int t = 0; t < (grp.Kmax + 15) / 16; ++t)
      for (int s = 0; s < nrs; ++s)
        for (int ln = 0; ln < FRAG; ++ln) {
          const int k = 16 * t + ln % 16, l = 4 * s + ln / 16;
          if (l < nr && k < grp.Kmax)
            h->tab_fwd[grp.tfwd_off + ((int64_t)t * nrs + s) * FRAG + ln] =
                pref * R * R * h->wq[l] * xi[(size_t)l * grp.Kmax + k];
        }
    // BF16 tables (16x16x16 fragments): inverse rows r, contraction k;
    // forward rows k, contraction r
    const int nk16 = (grp.Kmax + 15) / 16, nr16 = (nr + 15) / 16;
    for (int t = 0; t < nrt; ++t)
      for (int s = 0; s < nk16; ++s)
        for (int ln = 0; ln < FRAG; ++ln)
          for (int j = 0; j < 4; ++j) {
            const int l = 16 * t + ln % 16, k = 16 * s + 4 * (ln / 16) + j;
            if (l < nr && k < grp.Kmax)
              h->tab_inv16[(grp.tinv16_off + ((int64_t)t * nk16 + s) * FRAG + ln) * 4 + j] =
                  bf16_round(xi[(size_t)l * grp.Kmax + k]);
          }
    for (int t = 0; t < nk16; ++t)
      for (int s = 0; s < nr16; ++s)
        for (int ln = 0; ln < FRAG; ++ln)
          for (int j = 0; j < 4; ++j) {
            const int k = 16 * t + ln % 16, l = 16 * s + 4 * (ln / 16) + j;
            if (l < nr && k < grp.Kmax)
              h->tab_fwd16[(grp.tfwd16_off + ((int64_t)t * nr16 + s) * FRAG + ln) * 4 + j] =
                  bf16_round(pref * R * R * h->wq[l] * xi[(size_t)l * grp.Kmax + k]);
          }
  }
  return HELIC_OK;
}

}  // namespace
}  // namespace helic

using namespace helic;

extern "C" {

const char* helic_last_error(void) { return g_last_error.c_str(); }

helic_status helic_basis_create(const helic_params* p, helic_basis* out) {
  if (!p || !out) return fail(HELIC_ERR_INVALID, "null argument");
  *out = nullptr;
  helic_basis_s* h = new (std::nothrow) helic_basis_s();
  if (!h) return fail(HELIC_ERR_NOMEM, "host allocation failed");
  h->p = *p;
  helic_status s;
  try {
    s = build(h);
  } catch (const std::bad_alloc&) {
    s = fail(HELIC_ERR_NOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    s = fail(HELIC_ERR_INVALID, e.what());
  }
  if (s != HELIC_OK) {
    delete h;
    return s;
  }
  *out = h;
  return HELIC_OK;
}

helic_status helic_basis_destroy(helic_basis h) {
  if (!h) return HELIC_OK;
  device_release(h);
  delete h;
  return HELIC_OK;
}

helic_status helic_basis_info(helic_basis h, int64_t* L, int32_t* n_t1, int32_t* n_t2,
                              int32_t* n_r, int32_t* n_modes) {
  if (!h) return fail(HELIC_ERR_INVALID, "null handle");
  if (L) *L = h->L;
  if (n_t1) *n_t1 = h->n_t1;
  if (n_t2) *n_t2 = h->n_t2;
  if (n_r) *n_r = h->n_r;
  if (n_modes) *n_modes = (int32_t)h->modes.size();
  return HELIC_OK;
}

helic_status helic_basis_indices(helic_basis h, int32_t* mnk, double* kappa) {
  if (!h) return fail(HELIC_ERR_INVALID, "null handle");
  if (mnk) std::memcpy(mnk, h->mnk.data(), sizeof(int32_t) * h->mnk.size());
  if (kappa) std::memcpy(kappa, h->kappa.data(), sizeof(double) * h->kappa.size());
  return HELIC_OK;
}

helic_status helic_grid(helic_basis h, double* theta1, double* theta2, double* r, double* w_r) {
  if (!h) return fail(HELIC_ERR_INVALID, "null handle");
  if (theta1) std::memcpy(theta1, h->theta1.data(), sizeof(double) * h->n_t1);
  if (theta2) std::memcpy(theta2, h->theta2.data(), sizeof(double) * h->n_t2);
  for (int l = 0; l < h->n_r; ++l) {
    if (r) r[l] = h->p.R * h->q[l];
    if (w_r) w_r[l] = h->wq[l];
  }
  return HELIC_OK;
}

helic_status helic_util_bessel_j(int32_t p, int32_t n, const double* x, double* out) {
  if (n < 0 || (n > 0 && (!x || !out))) return fail(HELIC_ERR_INVALID, "bad arguments");
  for (int i = 0; i < n; ++i) {
    if (!(x[i] >= 0.0) || !std::isfinite(x[i])) return fail(HELIC_ERR_INVALID, "x must be finite and >= 0");
  }
  for (int i = 0; i < n; ++i) out[i] = bessel_j(p, x[i]);
  return HELIC_OK;
}

helic_status helic_util_bessel_zeros(int32_t p, int32_t count, double* out) {
  if (count < 0 || (count > 0 && !out)) return fail(HELIC_ERR_INVALID, "bad arguments");
  std::vector<double> z = bessel_zeros(p, count);
  std::copy(z.begin(), z.end(), out);
  return HELIC_OK;
}

helic_status helic_util_gauss_jacobi(int32_t n, double* q, double* w) {
  if (n < 0 || (n > 0 && (!q || !w))) return fail(HELIC_ERR_INVALID, "bad arguments");
  try {
    gauss_jacobi01(n, q, w);
  } catch (const std::exception& e) {
    return fail(HELIC_ERR_INVALID, e.what());
  }
  return HELIC_OK;
}

}  // extern "C"
