// Host-only checks of the plan-table builders and of descriptor validation,
// compiled with AddressSanitizer and UndefinedBehaviorSanitizer (no HIP, no
// GPU).  Every builder writes into a buffer of exactly the size its
// declaration documents, so a write past it, a read of freed or
// uninitialised heap memory, an integer overflow or a misaligned access in
// the host code fails the run.  Exit status 0 and "0 failures" on success.
#include <cmath>
#include <cstdio>
#include <vector>

#include "yyg.h"
#include "yyg_tables.h"

namespace {

int fails = 0;

void expect(bool ok, const char *what, int line) {
  if (!ok) {
    ++fails;
    std::printf("FAIL line %d: %s\n", line, what);
  }
}
#define EXPECT(c) expect((c), #c, __LINE__)

bool all_finite(const std::vector<double> &v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

std::vector<double> log_edges(int n, double r0, double r1) {
  std::vector<double> r(n + 1);
  for (int i = 0; i <= n; ++i) r[i] = r0 * std::pow(r1 / r0, (double)i / n);
  return r;
}

yyg_grid_desc make(int n_r, const double *r, int nt, int np, double dt, double dp, int L, int kind) {
  yyg_grid_desc d{};
  d.n_r = n_r;
  d.r_edges = r;
  d.n_theta = nt;
  d.n_phi = np;
  d.delta_theta = dt;
  d.delta_phi = dp;
  d.lmax = L;
  d.G = 1.0;
  d.kind = kind;
  return d;
}

size_t table_size(const yyg_grid_desc &d, int which) {
  const size_t Q = (size_t)(d.lmax + 1) * (d.lmax + 1), nang = (size_t)d.n_theta * d.n_phi;
  switch (which) {
    case YYG_TABLE_WEIGHTS: return nang;
    case YYG_TABLE_THETA: return d.n_theta * Q;
    case YYG_TABLE_PHI: return d.n_phi * Q;
    case YYG_TABLE_RADIAL: return 4 * (size_t)d.n_r * (d.lmax + 1);
    case YYG_TABLE_CROSS: return 3 * nang;
    default: return (size_t)yyg::rotation_blocks_size(d.lmax);
  }
}

// every table of the C ABI's host export, at its exact size; wrong sizes
// and a null output are refused
void check_exports(const yyg_grid_desc &d) {
  for (int which = YYG_TABLE_WEIGHTS; which <= YYG_TABLE_ROTATION; ++which) {
    const size_t n = table_size(d, which);
    std::vector<double> out(n, -7.0);
    const int st = yyg_host_table(&d, which, out.data(), n);
    if (which == YYG_TABLE_CROSS && d.kind == YYG_GRID_POLAR) {
      EXPECT(st == YYG_ERR_UNSUPPORTED);
      continue;
    }
    EXPECT(st == YYG_OK);
    EXPECT(all_finite(out));
    if (which == YYG_TABLE_WEIGHTS)
      for (double w : out) EXPECT(d.kind == YYG_GRID_POLAR ? w == 1.0 : (w >= 0.5 && w <= 1.0));
    std::vector<double> big(n + 1);
    EXPECT(yyg_host_table(&d, which, big.data(), n + 1) == YYG_ERR_INVALID_ARG);
    if (n > 0) EXPECT(yyg_host_table(&d, which, out.data(), n - 1) == YYG_ERR_INVALID_ARG);
    EXPECT(yyg_host_table(&d, which, nullptr, n) == YYG_ERR_INVALID_ARG);
  }
  std::vector<double> one(1);
  EXPECT(yyg_host_table(&d, 99, one.data(), 1) == YYG_ERR_INVALID_ARG);
  EXPECT(yyg_host_table(&d, -1, one.data(), 1) == YYG_ERR_INVALID_ARG);
}

// the builders a plan uses beyond the exported ones, at their documented sizes
void check_builders(const yyg_grid_desc &d) {
  const int L = d.lmax, Q = (L + 1) * (L + 1), nmc = 2 * L + 1;
  const yyg::PatchGeom g = d.kind == YYG_GRID_POLAR ? yyg::make_polar_patch(d.n_theta, d.n_phi)
                                                    : yyg::make_patch(d.n_theta, d.n_phi, d.delta_theta, d.delta_phi);
  EXPECT((int)g.th.size() == d.n_theta + 1 && (int)g.ph.size() == d.n_phi + 1);
  const size_t nang = (size_t)d.n_theta * d.n_phi;
  EXPECT((int)yyg::column_table(L).size() == Q);
  EXPECT((int)yyg::norm_sqrt(L).size() == (L + 1) * (L + 1));
  std::vector<double> p((size_t)(L + 1) * (L + 1));
  yyg::legendre_normalised(L, 0.3, std::sqrt(1.0 - 0.09), p.data());
  EXPECT(all_finite(p));
  std::vector<double> sl((size_t)d.n_theta * Q), st((size_t)d.n_phi * Q);
  yyg::self_legendre_table(g, L, sl.data());
  yyg::self_trig_table(g, L, st.data());
  EXPECT(all_finite(sl) && all_finite(st));
  const long ldk = (d.n_phi + 15) / 16 * 16, ldm = (nmc + 15) / 16 * 16;
  std::vector<double> cs((size_t)nmc * ldk), trig((size_t)d.n_phi * ldm);
  yyg::separable_cs(g, L, ldk, cs.data());
  yyg::separable_trig(g, L, ldm, trig.data());
  EXPECT(all_finite(cs) && all_finite(trig));
  if (d.kind == YYG_GRID_YINYANG) {
    std::vector<double> cb(nang * Q), cp(3 * nang);
    yyg::cross_basis(g, L, cb.data());
    yyg::cross_points(g, cp.data());
    EXPECT(all_finite(cb) && all_finite(cp));
  }
}

}  // namespace

int main() {
  const std::vector<double> r3 = log_edges(3, 1.0, 10.0), r1 = {0.0, 2.0}, r40 = log_edges(40, 1e5, 1e10);
  const double dt = 0.0349, dp = 0.0349;
  const yyg_grid_desc good[] = {
      make(3, r3.data(), 6, 16, 0.1, 0.1, 4, YYG_GRID_YINYANG),
      make(40, r40.data(), 47, 137, dt, dp, 25, YYG_GRID_YINYANG),
      make(3, r3.data(), 12, 34, dt, dp, 64, YYG_GRID_YINYANG),
      make(1, r1.data(), 5, 7, 0.0, 0.0, 0, YYG_GRID_YINYANG),
      make(3, r3.data(), 8, 16, 0.0, 0.0, 6, YYG_GRID_POLAR),
      make(1, r1.data(), 1, 1, 0.0, 0.0, 3, YYG_GRID_POLAR),
  };
  for (const auto &d : good) {
    EXPECT(yyg::validate_desc(&d) == YYG_OK);
    check_exports(d);
    check_builders(d);
  }
  // descriptors outside their documented ranges
  const std::vector<double> dec = {1.0, 3.0, 2.0}, neg = {-1.0, 1.0, 2.0}, nan_e = {0.0, NAN, 2.0};
  std::vector<yyg_grid_desc> bad;
  bad.push_back(make(3, nullptr, 6, 16, 0.1, 0.1, 4, YYG_GRID_YINYANG));
  bad.push_back(make(0, r3.data(), 6, 16, 0.1, 0.1, 4, YYG_GRID_YINYANG));
  bad.push_back(make(3, r3.data(), 0, 16, 0.1, 0.1, 4, YYG_GRID_YINYANG));
  bad.push_back(make(3, r3.data(), 6, -2, 0.1, 0.1, 4, YYG_GRID_YINYANG));
  bad.push_back(make(3, r3.data(), 6, 16, 0.1, 0.1, -1, YYG_GRID_YINYANG));
  bad.push_back(make(3, r3.data(), 6, 16, 0.1, 0.1, YYG_LMAX_CAP + 1, YYG_GRID_YINYANG));
  bad.push_back(make(2, dec.data(), 6, 16, 0.1, 0.1, 4, YYG_GRID_YINYANG));
  bad.push_back(make(2, neg.data(), 6, 16, 0.1, 0.1, 4, YYG_GRID_YINYANG));
  bad.push_back(make(2, nan_e.data(), 6, 16, 0.1, 0.1, 4, YYG_GRID_YINYANG));
  bad.push_back(make(3, r3.data(), 6, 16, 0.8, 0.1, 4, YYG_GRID_YINYANG));
  bad.push_back(make(3, r3.data(), 6, 16, 0.1, -0.1, 4, YYG_GRID_YINYANG));
  bad.push_back(make(3, r3.data(), 6, 16, 0.1, 0.0, 4, YYG_GRID_POLAR));
  bad.push_back(make(3, r3.data(), 6, 16, 0.1, 0.1, 4, 7));
  bad.push_back(make(3, r3.data(), 1 << 14, 1 << 13, 0.1, 0.1, 4, YYG_GRID_YINYANG));
  yyg_grid_desc gnan = make(3, r3.data(), 6, 16, 0.1, 0.1, 4, YYG_GRID_YINYANG);
  gnan.G = NAN;
  bad.push_back(gnan);
  std::vector<double> out(64);
  for (const auto &d : bad) {
    EXPECT(yyg::validate_desc(&d) == YYG_ERR_INVALID_ARG);
    EXPECT(yyg_host_table(&d, YYG_TABLE_WEIGHTS, out.data(), out.size()) == YYG_ERR_INVALID_ARG);
  }
  EXPECT(yyg::validate_desc(nullptr) == YYG_ERR_INVALID_ARG);
  EXPECT(yyg_host_table(nullptr, YYG_TABLE_WEIGHTS, out.data(), out.size()) == YYG_ERR_INVALID_ARG);
  // resolution rule and status strings
  int nt = 0, np = 0;
  double ddt = -1, ddp = -1;
  yyg::dims_from_resolution(0.5, &nt, &np, &ddt, &ddp);
  EXPECT(nt == 182 && np == 542 && ddt >= 0 && ddp >= 0);
  for (int s = -8; s <= 1; ++s) EXPECT(yyg_status_string(s) != nullptr);
  std::printf("host checks: %d failures\n", fails);
  return fails != 0;
}
