// Host FP64 table builders of a Yin-Yang plan (the density-independent terms,
// computed once per grid as the paper prescribes at the end of Sect. 3).
#include "yyg_tables.h"

#include <algorithm>
#include <cmath>
#include <thread>

namespace yyg {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kHalfPi = 1.57079632679489661923;

// Run body(i) for i in [0, n) over the available host threads.
template <class F>
void parallel_for(long n, F body) {
  unsigned nt = std::max(1u, std::min(std::thread::hardware_concurrency(), 32u));
  if (n < 64 || nt == 1) {
    for (long i = 0; i < n; ++i) body(i);
    return;
  }
  std::vector<std::thread> pool;
  long chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    long lo = t * chunk, hi = std::min(n, lo + chunk);
    if (lo >= hi) break;
    pool.emplace_back([=] {
      for (long i = lo; i < hi; ++i) body(i);
    });
  }
  for (auto &th : pool) th.join();
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration.
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_n(z), p0 = P_{n-1}(z)
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// ---- overlap geometry -----------------------------------------------------
// Along the meridian phi of one patch, the other patch leaves uncovered the
// theta band (pi/2 - e, pi/2 + e), e = max(e1, e2):
//   e1: the other patch's colatitude limit, |sin t sin p| <= c,
//       c = cos(pi/4 - delta_theta) -> e1 = pi/2 - asin(c/|sin p|), |sin p| > c;
//   e2: the other patch's longitude limit, excluded where cos p > 0 and
//       |cos t| < tan(pi/4 - delta_phi) sin t cos p -> e2 = atan(t cos p).
// sin e1 and sin e2 have elementary antiderivatives in phi (F1, F2), so
// the covered area of a cell is exact once phi is split where the
// integrand changes form.
struct Band {
  double c, a, t;  // c = cos(pi/4 - d_t), a = sin(pi/4 - d_t), t = tan(pi/4 - d_p)
};

inline double band_e1(double phi, const Band &b) {
  double s = std::fabs(std::sin(phi));
  return s > b.c ? kHalfPi - std::asin(b.c / s) : 0.0;
}
inline double band_e2(double phi, const Band &b) {
  double cp = std::cos(phi);
  return (cp > 0.0 && b.t > 0.0) ? std::atan(b.t * cp) : 0.0;
}
// d/dphi F1 = sin(e1(phi)) = sqrt(1 - c^2/sin^2 phi) where |sin phi| >= c.
// With u = cos phi: integral of sqrt(a^2-u^2)/(1-u^2) du
//   = asin(u/a) - c atan(c u / sqrt(a^2 - u^2)).
// Both terms are written as atan2(., r) with r = sqrt(a^2 - u^2) =
// sqrt(sin^2 phi - c^2): at the band's onset (r -> 0) their square-root
// parts then cancel analytically instead of through rounded asin near 1.
inline double band_F1(double phi, const Band &b) {
  double s = std::fabs(std::sin(phi));
  double u = std::cos(phi);
  double r = std::sqrt(std::max(0.0, (s - b.c) * (s + b.c)));
  double v = std::atan2(u, r) - b.c * std::atan2(b.c * u, r);
  return std::sin(phi) >= 0.0 ? -v : v;
}
// d/dphi F2 = sin(atan(t cos phi)) = t cos phi / sqrt(1 + t^2 cos^2 phi).
inline double band_F2(double phi, const Band &b) {
  return std::asin(b.t * std::sin(phi) / std::sqrt(1.0 + b.t * b.t));
}

// Integral over [pa, pb] of the part of the cell's theta range [ta, tb]
// (weighted by sin t) that the band (pi/2-e, pi/2+e) removes.
double excluded_integral(double ta, double tb, double pa, double pb, const Band &b) {
  std::vector<double> pts = {pa, pb};
  auto add = [&](double x) {
    if (x > pa && x < pb) pts.push_back(x);
  };
  auto add_sin = [&](double s) {  // |sin phi| = s
    if (s > 1.0) return;
    double base = std::asin(s);
    add(base); add(-base); add(kPi - base); add(-kPi + base);
  };
  auto add_cos = [&](double cv) {  // cos phi = cv >= 0
    if (cv > 1.0 || cv < 0.0) return;
    double base = std::acos(cv);
    add(base); add(-base);
  };
  add_sin(b.c);
  add(kHalfPi); add(-kHalfPi); add(0.0);
  if (b.t > 0.0) add_cos(std::sqrt((1.0 - b.c * b.c) / (1.0 + b.c * b.c * b.t * b.t)));  // e1 = e2
  const double vs[2] = {std::fabs(kHalfPi - ta), std::fabs(kHalfPi - tb)};
  for (double v : vs) {
    if (v <= 0.0) continue;
    add_sin(b.c / std::cos(v));
    if (b.t > 0.0) add_cos(std::tan(v) / b.t);
  }
  std::sort(pts.begin(), pts.end());
  const double cta = std::cos(ta), ctb = std::cos(tb);
  const double full = cta - ctb;
  double total = 0.0;
  for (size_t i = 0; i + 1 < pts.size(); ++i) {
    double x0 = pts[i], x1 = pts[i + 1];
    if (!(x1 > x0)) continue;
    double xm = 0.5 * (x0 + x1);
    double e1 = band_e1(xm, b), e2 = band_e2(xm, b);
    int branch = (e1 >= e2) ? (e1 > 0.0 ? 1 : 0) : 2;
    double e = std::max(e1, e2);
    double k0 = 0.0, k1 = 0.0;  // excluded = k0 + k1 sin(e)
    if (tb <= kHalfPi) {
      double d = kHalfPi - tb, D = kHalfPi - ta;
      if (e <= d) {
      } else if (e >= D) {
        k0 = full;
      } else {
        k0 = -ctb;
        k1 = 1.0;
      }
    } else if (ta >= kHalfPi) {
      double d = ta - kHalfPi, D = tb - kHalfPi;
      if (e <= d) {
      } else if (e >= D) {
        k0 = full;
      } else {
        k0 = cta;
        k1 = 1.0;
      }
    } else {
      if (e >= kHalfPi - ta) k0 += cta; else k1 += 1.0;
      if (e >= tb - kHalfPi) k0 -= ctb; else k1 += 1.0;
    }
    double piece = k0 * (x1 - x0);
    if (k1 != 0.0 && branch != 0) {
      double F = branch == 1 ? band_F1(x1, b) - band_F1(x0, b) : band_F2(x1, b) - band_F2(x0, b);
      piece += k1 * F;
    }
    total += piece;
  }
  return total;
}

}  // namespace

std::vector<ColInfo> column_table(int L) {
  std::vector<ColInfo> cols((L + 1) * (L + 1));
  for (int l = 0; l <= L; ++l)
    for (int m = 0; m <= l; ++m)
      for (int s = 0; s < (m == 0 ? 1 : 2); ++s) cols[qcol(l, m, s)] = {l, m, s};
  return cols;
}

PatchGeom make_patch(int n_t, int n_p, double d_t, double d_p) {
  PatchGeom g;
  g.n_t = n_t;
  g.n_p = n_p;
  g.d_t = d_t;
  g.d_p = d_p;
  g.th.resize(n_t + 1);
  g.ph.resize(n_p + 1);
  const double t0 = 0.25 * kPi - d_t, tspan = 0.5 * kPi + 2 * d_t;
  const double p0 = -0.75 * kPi - d_p, pspan = 1.5 * kPi + 2 * d_p;
  for (int j = 0; j <= n_t; ++j) g.th[j] = t0 + tspan * j / n_t;
  for (int k = 0; k <= n_p; ++k) g.ph[k] = p0 + pspan * k / n_p;
  return g;
}

PatchGeom make_polar_patch(int n_t, int n_p) {
  PatchGeom g;
  g.n_t = n_t;
  g.n_p = n_p;
  g.polar = true;
  g.th.resize(n_t + 1);
  g.ph.resize(n_p + 1);
  for (int j = 0; j <= n_t; ++j) g.th[j] = kPi * j / n_t;
  for (int k = 0; k <= n_p; ++k) g.ph[k] = 2.0 * kPi * k / n_p;
  return g;
}

void dims_from_resolution(double res_deg, int *n_t, int *n_p, double *d_t, double *d_p) {
  const double spans[2] = {90.0, 270.0};
  int n[2];
  double d[2];
  for (int i = 0; i < 2; ++i) {
    n[i] = (int)std::ceil(spans[i] / res_deg - 1e-9) + 2;
    d[i] = (n[i] * res_deg - spans[i]) * 0.5 * kPi / 180.0;
  }
  *n_t = n[0];
  *n_p = n[1];
  *d_t = d[0];
  *d_p = d[1];
}

void overlap_weights(const PatchGeom &g, double *w) {
  if (g.polar) {
    std::fill(w, w + (long)g.n_t * g.n_p, 1.0);
    return;
  }
  Band b;
  b.c = std::cos(0.25 * kPi - g.d_t);
  b.a = std::sin(0.25 * kPi - g.d_t);
  b.t = std::tan(0.25 * kPi - g.d_p);
  parallel_for((long)g.n_t * g.n_p, [&](long idx) {
    int j = (int)(idx / g.n_p), k = (int)(idx % g.n_p);
    double ta = g.th[j], tb = g.th[j + 1], pa = g.ph[k], pb = g.ph[k + 1];
    double full = (std::cos(ta) - std::cos(tb)) * (pb - pa);
    double excl = excluded_integral(ta, tb, pa, pb, b);
    double covered = (full - excl) / full;  // fraction inside the other patch
    covered = std::min(1.0, std::max(0.0, covered));
    w[idx] = 1.0 - 0.5 * covered;
  });
}

void legendre_normalised(int L, double x, double s, double *out) {
  const int W = L + 1;
  double smm = 1.0;
  for (int m = 0; m <= L; ++m) {
    if (m > 0) smm *= -s * std::sqrt((2.0 * m - 1.0) / (2.0 * m));
    out[m * W + m] = smm;
    if (m + 1 <= L) out[(m + 1) * W + m] = std::sqrt(2.0 * m + 1.0) * x * smm;
    for (int l = m + 2; l <= L; ++l) {
      out[l * W + m] = ((2.0 * l - 1.0) * x * out[(l - 1) * W + m] -
                        std::sqrt((double)(l + m - 1) * (l - m - 1)) * out[(l - 2) * W + m]) /
                       std::sqrt((double)(l - m) * (l + m));
    }
  }
  const double r2 = std::sqrt(2.0);
  for (int l = 1; l <= L; ++l)
    for (int m = 1; m <= l; ++m) out[l * W + m] *= r2;
}

std::vector<double> norm_sqrt(int L) {
  std::vector<double> s((L + 1) * (L + 1), 0.0);
  for (int l = 0; l <= L; ++l)
    for (int m = 0; m <= l; ++m) {
      double v = (m == 0) ? 1.0 : 2.0;
      for (int k = l - m + 1; k <= l + m; ++k) v /= k;
      s[l * (L + 1) + m] = std::sqrt(v);
    }
  return s;
}

void theta_table_normalised(const PatchGeom &g, int L, double *out) {
  const int Q = (L + 1) * (L + 1), W = L + 1;
  double dmax = 0.0;
  for (int j = 0; j < g.n_t; ++j) dmax = std::max(dmax, g.th[j + 1] - g.th[j]);
  int n = 24 + (int)std::ceil((L + 2) * dmax);
  std::vector<double> xg, wg;
  gauss_legendre(n, xg, wg);
  auto cols = column_table(L);
  parallel_for(g.n_t, [&](long j) {
    std::vector<double> acc(W * W, 0.0), P(W * W);
    double ta = g.th[j], tb = g.th[j + 1];
    double h = 0.5 * (tb - ta), mid = 0.5 * (ta + tb);
    for (int i = 0; i < n; ++i) {
      double t = mid + h * xg[i];
      double st = std::sin(t);
      legendre_normalised(L, std::cos(t), st, P.data());
      double wt = wg[i] * h * st;
      for (int l = 0; l <= L; ++l)
        for (int m = 0; m <= l; ++m) acc[l * W + m] += wt * P[l * W + m];
    }
    for (int q = 0; q < Q; ++q) out[j * Q + q] = acc[cols[q].l * W + cols[q].m];
  });
}

void phi_table(const PatchGeom &g, int L, double *out) {
  const int Q = (L + 1) * (L + 1);
  auto cols = column_table(L);
  for (int k = 0; k < g.n_p; ++k) {
    double pa = g.ph[k], pb = g.ph[k + 1];
    double c = 0.5 * (pa + pb), h = 0.5 * (pb - pa);
    for (int q = 0; q < Q; ++q) {
      int m = cols[q].m;
      double v;
      if (m == 0) {
        v = pb - pa;
      } else {
        // product forms of the differences in Eqs. (14)-(15)
        double sh = std::sin(m * h);
        v = cols[q].is_sin ? 2.0 * std::sin(m * c) * sh / m : 2.0 * std::cos(m * c) * sh / m;
      }
      out[k * Q + q] = v;
    }
  }
}

void radial_coefficients(int n_r, const double *r, int L, double *out) {
  for (int n = 0; n < n_r; ++n) {
    double rlo = r[n], rhi = r[n + 1];
    for (int l = 0; l <= L; ++l) {
      double *o = out + ((size_t)n * (L + 1) + l) * 4;
      if (rlo > 0.0) {
        double lq = std::log(rlo / rhi);
        o[0] = std::pow(rlo / rhi, l + 1);
        o[1] = rhi * rhi * (-std::expm1((l + 3) * lq)) / (l + 3);
      } else {
        o[0] = 0.0;
        o[1] = rhi * rhi / (l + 3);
      }
      if (n + 1 < n_r) {
        double rn = r[n + 1], sig = rn / r[n + 2];
        double ls = std::log(sig);
        o[2] = std::pow(sig, l);
        o[3] = (l == 2) ? -rn * rn * ls : rn * rn * (-std::expm1((l - 2) * ls)) / (l - 2);
      } else {
        o[2] = 0.0;
        o[3] = 0.0;
      }
    }
  }
}

void cross_points(const PatchGeom &g, double *out) {
  for (int j = 0; j < g.n_t; ++j) {
    double tc = 0.5 * (g.th[j] + g.th[j + 1]);
    double st = std::sin(tc), ct = std::cos(tc);
    for (int k = 0; k < g.n_p; ++k) {
      double pc = 0.5 * (g.ph[k] + g.ph[k + 1]);
      double sp = std::sin(pc), cp = std::cos(pc);
      double *o = out + ((size_t)j * g.n_p + k) * 3;
      // Eqs. (23)-(24) as the map (x, y, z) -> (-x, z, y)
      o[0] = st * sp;
      o[1] = std::hypot(ct, st * cp);
      o[2] = std::atan2(ct, -st * cp);
    }
  }
}

void self_legendre_table(const PatchGeom &g, int L, double *out) {
  const int Q = (L + 1) * (L + 1), W = L + 1;
  auto cols = column_table(L);
  std::vector<double> P(W * W);
  for (int j = 0; j < g.n_t; ++j) {
    double tc = 0.5 * (g.th[j] + g.th[j + 1]);
    legendre_normalised(L, std::cos(tc), std::sin(tc), P.data());
    for (int q = 0; q < Q; ++q) out[(size_t)j * Q + q] = P[cols[q].l * W + cols[q].m];
  }
}

void self_trig_table(const PatchGeom &g, int L, double *out) {
  const int Q = (L + 1) * (L + 1);
  auto cols = column_table(L);
  for (int k = 0; k < g.n_p; ++k) {
    double pc = 0.5 * (g.ph[k] + g.ph[k + 1]);
    for (int q = 0; q < Q; ++q) {
      int m = cols[q].m;
      out[(size_t)k * Q + q] = cols[q].is_sin ? std::sin(m * pc) : std::cos(m * pc);
    }
  }
}

void cross_basis(const PatchGeom &g, int L, double *out) {
  const int Q = (L + 1) * (L + 1), W = L + 1;
  auto cols = column_table(L);
  std::vector<double> pts((size_t)g.n_t * g.n_p * 3);
  cross_points(g, pts.data());
  parallel_for((long)g.n_t * g.n_p, [&](long a) {
    thread_local std::vector<double> P, cm, sm;
    P.resize(W * W);
    cm.resize(W);
    sm.resize(W);
    const double *pt = &pts[a * 3];
    legendre_normalised(L, pt[0], pt[1], P.data());
    for (int m = 0; m <= L; ++m) {
      cm[m] = std::cos(m * pt[2]);
      sm[m] = std::sin(m * pt[2]);
    }
    double *o = out + (size_t)a * Q;
    for (int q = 0; q < Q; ++q) {
      const ColInfo &c = cols[q];
      o[q] = P[c.l * W + c.m] * (c.is_sin ? sm[c.m] : cm[c.m]);
    }
  });
}

void separable_cs(const PatchGeom &g, int L, long ldk, double *out) {
  const int Q = (L + 1) * (L + 1), nmc = 2 * L + 1;
  std::vector<double> cs((size_t)g.n_p * Q);
  phi_table(g, L, cs.data());
  for (int mc = 0; mc < nmc; ++mc) {
    const int m = (mc + 1) / 2;
    const int q = m * m + mc;  // column (l = m, m, c)
    double *o = out + (size_t)mc * ldk;
    for (long k = 0; k < ldk; ++k) o[k] = k < g.n_p ? cs[(size_t)k * Q + q] : 0.0;
  }
}

void separable_trig(const PatchGeom &g, int L, long ldm, double *out) {
  const int nmc = 2 * L + 1;
  for (int k = 0; k < g.n_p; ++k) {
    const double pc = 0.5 * (g.ph[k] + g.ph[k + 1]);
    for (long mc = 0; mc < ldm; ++mc) {
      double v = 0.0;
      if (mc < nmc) {
        const int m = (int)(mc + 1) / 2;
        v = (mc == 0 || (mc & 1)) ? std::cos(m * pc) : std::sin(m * pc);
      }
      out[(size_t)k * ldm + mc] = v;
    }
  }
}

long rotation_blocks_size(int L) {
  long n = 0;
  for (int l = 0; l <= L; ++l) n += (long)(2 * l + 1) * (2 * l + 1);
  return n;
}

void rotation_blocks(int L, double *out) {
  const int W = L + 1, Q = W * W;
  // nodes: Gauss-Legendre in cos(theta) (L+1 nodes integrate degree 2L+1)
  // times 2L+2 equally spaced longitudes (exact for trig degree <= 2L+1)
  const int nt = L + 1, np = 2 * L + 2;
  std::vector<double> xg, wg;
  gauss_legendre(nt, xg, wg);
  auto cols = column_table(L);
  std::vector<long> off(L + 2, 0);
  for (int l = 0; l <= L; ++l) off[l + 1] = off[l] + (long)(2 * l + 1) * (2 * l + 1);
  // basis values at every node and at its image under the rotation
  const long npts = (long)nt * np;
  std::vector<double> Y((size_t)npts * Q), YR((size_t)npts * Q), wt(npts);
  parallel_for(npts, [&](long idx) {
    thread_local std::vector<double> P, PR;
    P.resize(W * W);
    PR.resize(W * W);
    const int it = (int)(idx / np), ip = (int)(idx % np);
    const double ct = xg[it], st = std::sqrt(std::max(0.0, (1.0 - ct) * (1.0 + ct)));
    const double ph = 2.0 * kPi * (ip + 0.5) / np;
    wt[idx] = wg[it] * 2.0 * kPi / np;
    const double sp = std::sin(ph), cp = std::cos(ph);
    // image point (x, y, z) -> (-x, z, y)
    const double ct2 = st * sp, st2 = std::hypot(ct, st * cp), ph2 = std::atan2(ct, -st * cp);
    legendre_normalised(L, ct, st, P.data());
    legendre_normalised(L, ct2, st2, PR.data());
    double *y = &Y[(size_t)idx * Q], *yr = &YR[(size_t)idx * Q];
    for (int q = 0; q < Q; ++q) {
      const ColInfo &c = cols[q];
      const double a1 = c.m * ph, a2 = c.m * ph2;
      y[q] = P[c.l * W + c.m] * (c.is_sin ? std::sin(a1) : std::cos(a1));
      yr[q] = PR[c.l * W + c.m] * (c.is_sin ? std::sin(a2) : std::cos(a2));
    }
  });
  // D_l[a][b] = (2l+1)/(4 pi) sum_nodes w YR_a Y_b   (the basis has norm 4 pi/(2l+1))
  parallel_for(L + 1, [&](long l) {
    const int d = 2 * (int)l + 1, q0 = (int)(l * l);
    double *blk = out + off[l];
    for (int i = 0; i < d * d; ++i) blk[i] = 0.0;
    for (long idx = 0; idx < npts; ++idx) {
      const double *y = &Y[(size_t)idx * Q + q0], *yr = &YR[(size_t)idx * Q + q0];
      const double w0 = wt[idx];
      for (int a = 0; a < d; ++a) {
        const double f = w0 * yr[a];
        for (int b = 0; b < d; ++b) blk[a * d + b] += f * y[b];
      }
    }
    const double s = (2.0 * l + 1.0) / (4.0 * kPi);
    for (int i = 0; i < d * d; ++i) blk[i] *= s;
  });
}

}  // namespace yyg
