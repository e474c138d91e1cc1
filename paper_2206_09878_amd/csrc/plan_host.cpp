// Host tables of the y-discretisation (App. C) and of the x-z transforms.
//
// B-spline values and derivatives at a point come from the triangular
// "nonzero functions of one knot span" evaluation with its derivative table
// (Piegl & Tiller, The NURBS Book, algorithm A2.3), written here for
// clamped knot vectors.  Collocation rows are stored band-packed.
#include "plan_host.h"

#include <algorithm>
#include <cmath>
#include <random>

namespace lmvd {
namespace {

std::vector<double> clamped(const std::vector<double>& xi, int order) {
  std::vector<double> t;
  t.insert(t.end(), order - 1, xi.front());
  t.insert(t.end(), xi.begin(), xi.end());
  t.insert(t.end(), order - 1, xi.back());
  return t;
}

std::vector<double> greville_points(const std::vector<double>& t, int order) {
  int n = int(t.size()) - order;
  std::vector<double> g(n);
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int q = 1; q < order; ++q) s += t[i + q];
    g[i] = s / double(order - 1);
  }
  return g;
}

// Knot span s with t[s] <= x < t[s+1]; the right end belongs to the last span.
int span_of(const std::vector<double>& t, int order, double x) {
  int n = int(t.size()) - order;
  if (x >= t[n]) return n - 1;
  int lo = order - 1, hi = n;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (x < t[mid]) hi = mid; else lo = mid;
  }
  return lo;
}

// Nonzero functions N_{s-deg+r} (r = 0..deg) of degree `deg` at x in span s
// and their first `nd` derivatives: ders[k][r].
void span_basis(const std::vector<double>& t, int deg, int s, double x, int nd,
                double ders[3][kMaxW]) {
  double ndu[kMaxW][kMaxW], left[kMaxW], right[kMaxW], a[2][kMaxW];
  ndu[0][0] = 1.0;
  for (int j = 1; j <= deg; ++j) {
    left[j] = x - t[s + 1 - j];
    right[j] = t[s + j] - x;
    double saved = 0.0;
    for (int r = 0; r < j; ++r) {
      ndu[j][r] = right[r + 1] + left[j - r];
      double temp = ndu[r][j - 1] / ndu[j][r];
      ndu[r][j] = saved + right[r + 1] * temp;
      saved = left[j - r] * temp;
    }
    ndu[j][j] = saved;
  }
  for (int j = 0; j <= deg; ++j) ders[0][j] = ndu[j][deg];
  for (int r = 0; r <= deg; ++r) {
    int s1 = 0, s2 = 1;
    a[0][0] = 1.0;
    for (int k = 1; k <= nd; ++k) {
      double d = 0.0;
      int rk = r - k, pk = deg - k;
      if (r >= k) {
        a[s2][0] = a[s1][0] / ndu[pk + 1][rk];
        d = a[s2][0] * ndu[rk][pk];
      }
      int j1 = (rk >= -1) ? 1 : -rk;
      int j2 = (r - 1 <= pk) ? k - 1 : deg - r;
      for (int j = j1; j <= j2; ++j) {
        a[s2][j] = (a[s1][j] - a[s1][j - 1]) / ndu[pk + 1][rk + j];
        d += a[s2][j] * ndu[rk + j][pk];
      }
      if (r <= pk) {
        a[s2][k] = -a[s1][k - 1] / ndu[pk + 1][r];
        d += a[s2][k] * ndu[r][pk];
      }
      ders[k][r] = d;
      std::swap(s1, s2);
    }
  }
  double f = deg;
  for (int k = 1; k <= nd; ++k) {
    for (int j = 0; j <= deg; ++j) ders[k][j] *= f;
    f *= double(deg - k);
  }
}

// Row tables of derivatives 0..nd of the order-`order` basis on knots t at pts.
void rows_at(const std::vector<double>& t, int order, const std::vector<double>& pts, int nd,
             RowTable* out) {
  int n = int(t.size()) - order;
  for (int d = 0; d <= nd; ++d) {
    out[d].rows = int(pts.size());
    out[d].cols = n;
    out[d].lo.assign(pts.size(), 0);
    out[d].w.assign(pts.size() * kMaxW, 0.0);
  }
  for (size_t i = 0; i < pts.size(); ++i) {
    int s = span_of(t, order, pts[i]);
    double ders[3][kMaxW] = {{0}};
    span_basis(t, order - 1, s, pts[i], nd, ders);
    for (int d = 0; d <= nd; ++d) {
      out[d].lo[i] = s - order + 1;
      for (int r = 0; r < order; ++r) out[d].w[i * kMaxW + r] = ders[d][r];
    }
  }
}

// No-pivot LU of a dense n x n matrix (row-major), returned band-packed.
lmvd_status band_lu(std::vector<double> A, int n, BandLU& lu, std::string& msg) {
  int lower = 0, upper = 0;
  double amax = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (A[size_t(i) * n + j] != 0.0) {
        lower = std::max(lower, i - j);
        upper = std::max(upper, j - i);
        amax = std::max(amax, std::fabs(A[size_t(i) * n + j]));
      }
  if (lower > kMaxBand || upper > kMaxBand) {
    msg = "bandwidth exceeds the LU table limit";
    return LMVD_EUNSUPPORTED;
  }
  std::vector<double> Aorig = A;
  for (int k = 0; k < n; ++k) {
    double piv = A[size_t(k) * n + k];
    if (!(std::fabs(piv) > 1e-12 * amax)) {
      msg = "near-zero pivot in a no-pivot LU";
      return LMVD_ENUMERIC;
    }
    for (int i = k + 1; i < std::min(n, k + lower + 1); ++i) {
      double m = A[size_t(i) * n + k] / piv;
      A[size_t(i) * n + k] = m;
      for (int j = k + 1; j < std::min(n, k + upper + 1); ++j) A[size_t(i) * n + j] -= m * A[size_t(k) * n + j];
    }
  }
  lu.n = n;
  lu.lower = lower;
  lu.upper = upper;
  lu.lmul.assign(size_t(n) * kMaxBand, 0.0);
  lu.u.assign(size_t(n) * (kMaxBand + 1), 0.0);
  lu.uinv.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    for (int m = 1; m <= lower && i - m >= 0; ++m) lu.lmul[size_t(i) * kMaxBand + m - 1] = A[size_t(i) * n + i - m];
    for (int q = 1; q <= upper && i + q < n; ++q) lu.u[size_t(i) * (kMaxBand + 1) + q] = A[size_t(i) * n + i + q];
    lu.uinv[i] = 1.0 / A[size_t(i) * n + i];
    lu.u[size_t(i) * (kMaxBand + 1)] = A[size_t(i) * n + i];
  }
  // residual check of the factorisation on a random vector
  std::mt19937_64 rng(12345);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  std::vector<double> x(n), b(n, 0.0), y(n);
  for (auto& v : x) v = U(rng);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) b[i] += Aorig[size_t(i) * n + j] * x[j];
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int m = 1; m <= lower && i - m >= 0; ++m) s -= lu.lmul[size_t(i) * kMaxBand + m - 1] * y[i - m];
    y[i] = s;
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = y[i];
    for (int q = 1; q <= upper && i + q < n; ++q) s -= lu.u[size_t(i) * (kMaxBand + 1) + q] * y[i + q];
    y[i] = s * lu.uinv[i];
  }
  double err = 0.0, xm = 0.0;
  for (int i = 0; i < n; ++i) {
    err = std::max(err, std::fabs(y[i] - x[i]));
    xm = std::max(xm, std::fabs(x[i]));
  }
  if (!(err <= 1e-9 * xm)) {
    msg = "no-pivot LU is inaccurate";
    return LMVD_ENUMERIC;
  }
  return LMVD_OK;
}

bool factor23(int n, FftPlan& f) {
  if (n < 1) return false;
  int a = 0, b = 0, m = n;
  while (m % 2 == 0) { m /= 2; ++a; }
  while (m % 3 == 0) { m /= 3; ++b; }
  if (m != 1) return false;
  f.n = n;
  f.nstages = 0;
  while (a >= 3) { f.radix[f.nstages++] = 8; a -= 3; }
  if (a == 2) f.radix[f.nstages++] = 4;
  if (a == 1) f.radix[f.nstages++] = 2;
  for (int i = 0; i < b; ++i) f.radix[f.nstages++] = 3;
  if (f.nstages == 0) f.radix[f.nstages++] = 1;
  int ns = 1;
  for (int s = 0; s < f.nstages; ++s) {
    f.ns[s] = ns;
    ns *= f.radix[s];
  }
  f.tw.resize(size_t(2) * n);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int t = 0; t < n; ++t) {
    long double ang = -2.0L * pi * (long double)t / (long double)n;
    f.tw[2 * t] = double(cosl(ang));
    f.tw[2 * t + 1] = double(sinl(ang));
  }
  return true;
}

}  // namespace

std::vector<double> dense(const RowTable& r) {
  std::vector<double> D(size_t(r.rows) * r.cols, 0.0);
  for (int i = 0; i < r.rows; ++i)
    for (int q = 0; q < kMaxW; ++q) {
      int j = r.lo[i] + q;
      if (j >= 0 && j < r.cols) D[size_t(i) * r.cols + j] = r.w[size_t(i) * kMaxW + q];
    }
  return D;
}

lmvd_status build_host_tables(const lmvd_config& cfg, HostTables& H, std::string& msg) {
  H.cfg = cfg;
  const int p = cfg.order;
  if (p < 3 || p > 9) { msg = "order must be in 3..9"; return LMVD_EUNSUPPORTED; }
  if (cfg.n1 < 2 || cfg.n3 < 2 || cfg.n1 % 2 || cfg.n3 % 2) { msg = "n1, n3 must be even >= 2"; return LMVD_EINVAL; }
  if (cfg.n2 < p) { msg = "n2 must be >= order"; return LMVD_EINVAL; }
  if (cfg.m1 < cfg.n1 || cfg.m3 < cfg.n3 || cfg.m1 % 2) { msg = "m1 >= n1 (even) and m3 >= n3 required"; return LMVD_EINVAL; }
  if (!(cfg.L1 > 0 && cfg.L2 > 0 && cfg.L3 > 0 && cfg.dt > 0 && cfg.rho_l > 0 && cfg.rho_h > 0)) {
    msg = "lengths, dt and densities must be positive";
    return LMVD_EINVAL;
  }
  if (cfg.kf < 0 || cfg.plane_batch < 0) { msg = "kf and plane_batch must be >= 0"; return LMVD_EINVAL; }
  if (cfg.rhoD_form != 0 && cfg.rhoD_form != 1) { msg = "rhoD_form must be 0 or 1"; return LMVD_EINVAL; }
  if (cfg.check_finite != 0 && cfg.check_finite != 1) { msg = "check_finite must be 0 or 1"; return LMVD_EINVAL; }
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(cfg.mu_z[k]) || !std::isfinite(cfg.rhoD_z[k])) {
      msg = "transport-law coefficients must be finite";
      return LMVD_EINVAL;
    }
  if (!cfg.breakpoints) { msg = "breakpoints is NULL"; return LMVD_EINVAL; }
  const int nb = cfg.n2 - p + 2;
  H.breakpoints.assign(cfg.breakpoints, cfg.breakpoints + nb);
  for (int i = 1; i < nb; ++i)
    if (!(H.breakpoints[i] > H.breakpoints[i - 1])) { msg = "breakpoints must increase"; return LMVD_EINVAL; }
  if (std::fabs(H.breakpoints.front() + 0.5 * cfg.L2) > 1e-12 * cfg.L2 ||
      std::fabs(H.breakpoints.back() - 0.5 * cfg.L2) > 1e-12 * cfg.L2) {
    msg = "breakpoints must end at -L2/2 and +L2/2";
    return LMVD_EINVAL;
  }
  H.n2 = cfg.n2;
  H.p = p;
  H.nl = cfg.n1 / 2;
  H.nn = cfg.n3 - 1;
  H.hx = cfg.m1 / 2;
  H.t = clamped(H.breakpoints, p);
  H.ts = clamped(H.breakpoints, p + 1);
  H.tau = greville_points(H.t, p);
  H.tau_s = greville_points(H.ts, p + 1);
  rows_at(H.t, p, H.tau, 2, H.E);
  rows_at(H.ts, p + 1, H.tau, 0, &H.F0);
  rows_at(H.t, p, H.tau_s, 1, H.G);
  rows_at(H.ts, p + 1, H.tau_s, 2, H.Es);
  H.dstar.resize(H.n2);
  for (int j = 0; j < H.n2; ++j) H.dstar[j] = double(p) / (H.ts[j + p + 1] - H.ts[j + 1]);

  // shared projections (values -> coefficients), end rows replaced
  const int n2 = H.n2;
  std::vector<double> E0 = dense(H.E[0]), E1 = dense(H.E[1]);
  for (int kind = 0; kind < 3; ++kind) {
    std::vector<double> A = E0;
    if (kind > 0) {
      for (int end : {0, n2 - 1}) {
        for (int j = 0; j < n2; ++j) {
          double v = (kind == 1) ? (j == end ? 1.0 : 0.0) : E1[size_t(end) * n2 + j];
          A[size_t(end) * n2 + j] = v;
        }
      }
    }
    lmvd_status st = band_lu(A, n2, H.proj[kind], msg);
    if (st != LMVD_OK) return st;
  }

  // band of A(k): union of E*_0, E*_1, E*_2 row supports
  {
    int lower = 0, upper = 0;
    for (int i = 0; i <= n2; ++i)
      for (int d = 0; d < 3; ++d)
        for (int q = 0; q < kMaxW; ++q) {
          int j = H.Es[d].lo[i] + q;
          if (j < 0 || j > n2 || H.Es[d].w[size_t(i) * kMaxW + q] == 0.0) continue;
          lower = std::max(lower, i - j);
          upper = std::max(upper, j - i);
        }
    H.a_lower = lower;
    H.a_upper = upper;
    if (lower > 8 || upper > 8) { msg = "A(k) bandwidth exceeds 8"; return LMVD_EUNSUPPORTED; }
    H.fac_nm.assign(n2 + 1, 0);
    H.fac_ns.assign(n2 + 1, 0);
    // no-pivot stability of A(k) over the range of k of this grid
    double kmax = std::sqrt(std::pow(2 * M_PI * (H.nl - 1) / cfg.L1, 2) +
                            std::pow(2 * M_PI * (cfg.n3 / 2 - 1) / cfg.L3, 2));
    double kmin = 2 * M_PI / std::max(cfg.L1, cfg.L3);
    std::vector<double> ks;
    for (int s = 0; s <= 6; ++s) ks.push_back(kmin * std::pow(kmax / kmin, s / 6.0));
    std::vector<double> Es0 = dense(H.Es[0]), Es1 = dense(H.Es[1]), Es2 = dense(H.Es[2]);
    const int n = n2 + 1;
    for (double k : ks) {
      if (!(k > 0)) continue;
      std::vector<double> A(size_t(n) * n);
      for (size_t e = 0; e < A.size(); ++e) A[e] = Es2[e] - k * k * Es0[e];
      for (int j = 0; j < n; ++j) {
        A[j] = k * Es0[j] - Es1[j];
        A[size_t(n2) * n + j] = k * Es0[size_t(n2) * n + j] + Es1[size_t(n2) * n + j];
      }
      BandLU tmp;
      lmvd_status st = band_lu(A, n, tmp, msg);
      if (st != LMVD_OK) { msg = "A(k): " + msg; return st; }
      // the m^c solve eliminates from the last row upwards: LU of the reversed matrix
      std::vector<double> Ar(A.size());
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ar[size_t(i) * n + j] = A[size_t(n - 1 - i) * n + (n - 1 - j)];
      st = band_lu(Ar, n, tmp, msg);
      if (st != LMVD_OK) { msg = "A(k) reversed: " + msg; return st; }
      // nonzero structure of the bottom-up elimination
      std::vector<double> a = A;
      for (int i = n - 1; i >= 0; --i) {
        for (int m = upper; m >= 1; --m) {
          if (i + m >= n) continue;
          const double e = a[size_t(i) * n + i + m];
          if (e == 0.0) continue;
          H.fac_nm[i] = std::max(H.fac_nm[i], m);
          const double lm = e / a[size_t(i + m) * n + i + m];
          for (int j = std::max(0, i + m - lower - upper); j <= i + m; ++j)
            a[size_t(i) * n + j] -= lm * a[size_t(i + m) * n + j];
          a[size_t(i) * n + i + m] = 0.0;
        }
        for (int q = 1; q <= i; ++q)
          if (a[size_t(i) * n + i - q] != 0.0) H.fac_ns[i] = std::max(H.fac_ns[i], q);
      }
    }
    H.fac_off.assign(n, 0);
    int off = 0;
    for (int i = n - 1; i >= 0; --i) {  // in the order of the bottom-up sweep
      if (H.fac_nm[i] > upper || H.fac_ns[i] > lower) { msg = "A(k) elimination exceeds its band"; return LMVD_ENUMERIC; }
      H.fac_off[i] = off;
      off += H.fac_nm[i] + H.fac_ns[i] + 1;
    }
    H.fac_slots = off;
  }

  H.k1.resize(H.nl);
  H.k3.resize(H.nn);
  for (int l = 0; l < H.nl; ++l) H.k1[l] = 2.0 * M_PI * l / cfg.L1;
  for (int i = 0; i < H.nn; ++i) {
    int n = (i < cfg.n3 / 2) ? i : i - (cfg.n3 - 1);
    H.k3[i] = 2.0 * M_PI * n / cfg.L3;
  }
  if (!factor23(cfg.m3, H.fz) || !factor23(H.hx, H.fx) || cfg.m3 > 1024 || H.hx > 1024) {
    msg = "m3 and m1/2 must be 2^a 3^b <= 1024";
    return LMVD_EUNSUPPORTED;
  }
  H.emit_first.assign(H.n2, 0);
  H.emit_cnt.assign(H.n2, 0);
  for (int i = H.n2 - 1; i >= 0; --i) {
    const int lo = H.E[0].lo[i];
    if (lo < 0 || lo >= H.n2) { msg = "E0 band start out of range"; return LMVD_ENUMERIC; }
    H.emit_first[lo] = i;  // the smallest i with this lo, after the descending loop
    H.emit_cnt[lo] += 1;
  }
  // G_1 rows at interior tau*, emitted by the descending sweep of a projection
  H.g1e_first.assign(H.n2, 0);
  H.g1e_cnt.assign(H.n2, 0);
  for (int i = H.n2 - 1; i >= 1; --i) {
    const int lo = H.G[1].lo[i];
    if (lo < 0 || lo >= H.n2) { msg = "G1 band start out of range"; return LMVD_ENUMERIC; }
    if (i < H.n2 - 1 && lo > H.G[1].lo[i + 1]) { msg = "G1 band starts not monotone"; return LMVD_ENUMERIC; }
    H.g1e_first[lo] = i;
    H.g1e_cnt[lo] += 1;
  }
  // F_0 (B* at tau) and F_1 = E_0 D* (derivative of a B* spline at tau), emitted by an
  // ascending sweep over B* coefficients once their last column is known
  {
    const int ns = H.n2 + 1;
    std::vector<double> F0d = dense(H.F0), E0d = dense(H.E[0]);
    H.asc_first.assign(ns, 0);
    H.asc_cnt.assign(ns, 0);
    H.asc_w.assign(size_t(2) * H.n2 * kMaxW, 0.0);
    int prev_last = -1;
    for (int i = 0; i < H.n2; ++i) {
      std::vector<double> f1(ns, 0.0);
      for (int j = 0; j < ns; ++j) {
        double v = 0.0;
        if (j >= 1) v += E0d[size_t(i) * H.n2 + j - 1] * H.dstar[j - 1];
        if (j < H.n2) v -= E0d[size_t(i) * H.n2 + j] * H.dstar[j];
        f1[j] = v;
      }
      int first = ns, last = -1;
      for (int j = 0; j < ns; ++j)
        if (F0d[size_t(i) * ns + j] != 0.0 || f1[j] != 0.0) {
          first = std::min(first, j);
          last = std::max(last, j);
        }
      if (last < 0 || last - first >= kMaxW) { msg = "F0/F1 row support exceeds the window"; return LMVD_ENUMERIC; }
      if (last < prev_last) { msg = "F0/F1 row ends not monotone"; return LMVD_ENUMERIC; }
      prev_last = last;
      if (H.asc_cnt[last] == 0) H.asc_first[last] = i;
      H.asc_cnt[last] += 1;
      for (int q = 0; q < kMaxW && last - q >= 0; ++q) {
        H.asc_w[size_t(i) * kMaxW + q] = F0d[size_t(i) * ns + last - q];
        H.asc_w[(size_t(H.n2) + i) * kMaxW + q] = f1[last - q];
      }
    }
  }
  // wall rows of E_0 P_N: x solves P^T x = e with e = (row 0 or n2-1 of E_0)^T,
  // P = L U the Neumann matrix (U^T z = e, then L^T x = z)
  {
    const BandLU& B = H.proj[2];
    const int n = H.n2;
    auto wall = [&](int row, std::vector<double>& x) {
      std::vector<double> z(n, 0.0);
      x.assign(n, 0.0);
      for (int i = 0; i < n; ++i) {
        double s = H.E[0].at(row, i);
        for (int q = 1; q <= B.upper && i - q >= 0; ++q) s -= B.u[size_t(i - q) * (kMaxBand + 1) + q] * z[i - q];
        z[i] = s * B.uinv[i];
      }
      for (int i = n - 1; i >= 0; --i) {
        double s = z[i];
        for (int m = 1; m <= B.lower && i + m < n; ++m) s -= B.lmul[size_t(i + m) * kMaxBand + (m - 1)] * x[i + m];
        x[i] = s;
      }
    };
    auto cut = [&](const std::vector<double>& x, bool from_top) {
      // interior rows by distance d = 1 .. n-2 from the wall; tails summed from the far end
      std::vector<double> tail(size_t(n), 0.0);  // tail[d] = sum over distances > d
      for (int d = n - 3; d >= 0; --d) tail[d] = tail[d + 1] + std::fabs(x[from_top ? n - 2 - d : d + 1]);
      const double tot = tail[0];
      int k = 0;
      while (k < n - 2 && tail[k] > std::ldexp(tot, -60)) ++k;
      return k;
    };
    std::vector<double> x0, x1;
    wall(0, x0);
    wall(n - 1, x1);
    H.wall_k0 = cut(x0, false);
    H.wall_k1 = cut(x1, true);
    H.wall_w.assign(size_t(H.wall_k0) + H.wall_k1 + 2, 0.0);
    for (int d = 1; d <= H.wall_k0; ++d) H.wall_w[d] = x0[d];
    for (int d = 1; d <= H.wall_k1; ++d) H.wall_w[size_t(H.wall_k0) + 1 + d] = x1[n - 1 - d];
  }
  H.xtw.resize(size_t(2) * H.hx);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int k = 0; k < H.hx; ++k) {
    long double ang = -2.0L * pi * (long double)k / (long double)cfg.m1;
    H.xtw[2 * k] = double(cosl(ang));
    H.xtw[2 * k + 1] = double(sinl(ang));
  }
  return LMVD_OK;
}

}  // namespace lmvd

namespace lmvd {

// The bottom-up no-pivot elimination of A(k) (rows n2 .. 0) for every distinct k^2 = k1^2 + k3^2 of the
// grid, with the row check of the device factorisation: s = largest magnitude of row i of A; the pivot
// must reach 1e-12 s and the eliminated row may not exceed growth_max s.
lmvd_status factor_check_host(const HostTables& H, double growth_max, FactorCheck& out) {
  const int n2 = H.n2, N = n2 + 1, LA = H.a_lower, UA = H.a_upper, W = LA + UA + 1;
  std::vector<double> ks;
  for (int l = 0; l < H.nl; ++l)
    for (int n = 0; n < (H.nn + 1) / 2; ++n) ks.push_back(H.k1[l] * H.k1[l] + H.k3[n] * H.k3[n]);
  std::sort(ks.begin(), ks.end());
  ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
  out = FactorCheck{};
  out.min_pivot_ratio = INFINITY;
  std::vector<double> piv(size_t(UA) * LA), pinv(UA), a(W);
  for (double ksq : ks) {
    if (ksq == 0.0) continue;
    ++out.distinct_k;
    const double k = std::sqrt(ksq);
    std::fill(piv.begin(), piv.end(), 0.0);
    std::fill(pinv.begin(), pinv.end(), 0.0);
    for (int i = N - 1; i >= 0; --i) {
      const bool robin = (i == 0 || i == n2);
      const double sg = (i == 0) ? -1.0 : 1.0;
      double rs = 0.0;
      for (int w = 0; w < W; ++w) {
        const int col = i - LA + w;
        a[w] = robin ? k * H.Es[0].at(i, col) + sg * H.Es[1].at(i, col)
                     : H.Es[2].at(i, col) - ksq * H.Es[0].at(i, col);
        rs = std::max(rs, std::fabs(a[w]));
      }
      for (int m = UA; m >= 1; --m) {
        const double lm = a[LA + m] * pinv[m - 1];
        for (int q = 1; q <= LA; ++q) a[LA + m - q] -= lm * piv[size_t(m - 1) * LA + q - 1];
      }
      double big = 0.0;
      for (int w = 0; w <= LA; ++w) big = std::max(big, std::fabs(a[w]));
      const double growth = big / rs, ratio = std::fabs(a[LA]) / rs;
      if (!(ratio >= 1e-12) || !(growth <= growth_max)) ++out.bad_rows;
      if (growth > out.max_growth) out.max_growth = growth;
      if (ratio < out.min_pivot_ratio) out.min_pivot_ratio = ratio;
      for (int m = UA - 1; m > 0; --m) {
        pinv[m] = pinv[m - 1];
        for (int q = 0; q < LA; ++q) piv[size_t(m) * LA + q] = piv[size_t(m - 1) * LA + q];
      }
      pinv[0] = 1.0 / a[LA];
      for (int q = 1; q <= LA; ++q) piv[q - 1] = a[LA - q];
    }
  }
  return out.bad_rows ? LMVD_ENUMERIC : LMVD_OK;
}

}  // namespace lmvd

namespace lmvd {

// Values of the B basis (order p, star = 0) or the B* basis (order p + 1, star = 1) at the points y, all
// within [-L2/2, L2/2]: out[i * ncols + j] = B_j(y_i), ncols = n2 (n2 + 1 for B*).
lmvd_status basis_values(const HostTables& H, int star, const std::vector<double>& y, std::vector<double>& out) {
  const double h = 0.5 * H.cfg.L2;
  for (double v : y)
    if (!(v >= -h && v <= h)) return LMVD_EINVAL;
  RowTable rt;
  rows_at(star ? H.ts : H.t, star ? H.p + 1 : H.p, y, 0, &rt);
  out = dense(rt);
  return LMVD_OK;
}

}  // namespace lmvd
