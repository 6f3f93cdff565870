// Host-only part of the C ABI: descriptor validation, status strings and
// the host exports of the plan tables.  Built without HIP, so that it and
// yyg_tables.cpp also compile for host sanitizer runs.
#include <cmath>
#include <cstddef>
#include <new>

#include "yyg.h"
#include "yyg_tables.h"

namespace yyg {

// A descriptor's fields within the documented ranges (yyg_grid_desc).
int validate_desc(const yyg_grid_desc *d) {
  if (!d || !d->r_edges) return YYG_ERR_INVALID_ARG;
  if (d->kind != YYG_GRID_YINYANG && d->kind != YYG_GRID_POLAR) return YYG_ERR_INVALID_ARG;
  if (d->kind == YYG_GRID_POLAR && (d->delta_theta != 0.0 || d->delta_phi != 0.0)) return YYG_ERR_INVALID_ARG;
  if (d->n_r < 1 || d->n_theta < 1 || d->n_phi < 1) return YYG_ERR_INVALID_ARG;
  if (d->lmax < 0 || d->lmax > YYG_LMAX_CAP) return YYG_ERR_INVALID_ARG;
  const double q = 0.78539816339744830962;
  if (!(d->delta_theta >= 0.0 && d->delta_theta < q) || !(d->delta_phi >= 0.0 && d->delta_phi < q))
    return YYG_ERR_INVALID_ARG;
  if (!std::isfinite(d->G)) return YYG_ERR_INVALID_ARG;
  if (!(d->r_edges[0] >= 0.0) || !std::isfinite(d->r_edges[0])) return YYG_ERR_INVALID_ARG;
  for (int i = 0; i < d->n_r; ++i)
    if (!(d->r_edges[i + 1] > d->r_edges[i]) || !std::isfinite(d->r_edges[i + 1])) return YYG_ERR_INVALID_ARG;
  if ((long)d->n_theta * d->n_phi > (1L << 26)) return YYG_ERR_INVALID_ARG;
  return YYG_OK;
}

}  // namespace yyg

extern "C" {

const char *yyg_status_string(int status) {
  switch (status) {
    case YYG_OK: return "ok";
    case YYG_ERR_INVALID_ARG: return "invalid argument";
    case YYG_ERR_OUT_OF_MEMORY: return "out of memory";
    case YYG_ERR_DEVICE: return "HIP device error";
    case YYG_ERR_NOT_READY: return "not ready (no density uploaded or precision not prepared)";
    case YYG_ERR_UNSUPPORTED: return "unsupported";
    case YYG_ERR_NONFINITE: return "non-finite input";
    default: return "unknown status";
  }
}

int yyg_host_table(const yyg_grid_desc *d, int which, double *out, size_t n) {
  int st = yyg::validate_desc(d);
  if (st != YYG_OK) return st;
  if (!out) return YYG_ERR_INVALID_ARG;
  const int L = d->lmax, Q = (L + 1) * (L + 1);
  const size_t nang = (size_t)d->n_theta * d->n_phi;
  yyg::PatchGeom g = d->kind == YYG_GRID_POLAR ? yyg::make_polar_patch(d->n_theta, d->n_phi)
                                               : yyg::make_patch(d->n_theta, d->n_phi, d->delta_theta, d->delta_phi);
  try {
    switch (which) {
      case YYG_TABLE_WEIGHTS:
        if (n != nang) return YYG_ERR_INVALID_ARG;
        yyg::overlap_weights(g, out);
        return YYG_OK;
      case YYG_TABLE_THETA: {
        if (n != (size_t)d->n_theta * Q) return YYG_ERR_INVALID_ARG;
        yyg::theta_table_normalised(g, L, out);
        auto s = yyg::norm_sqrt(L);
        auto cols = yyg::column_table(L);
        for (int j = 0; j < d->n_theta; ++j)
          for (int q = 0; q < Q; ++q) out[(size_t)j * Q + q] /= s[cols[q].l * (L + 1) + cols[q].m];
        return YYG_OK;
      }
      case YYG_TABLE_PHI:
        if (n != (size_t)d->n_phi * Q) return YYG_ERR_INVALID_ARG;
        yyg::phi_table(g, L, out);
        return YYG_OK;
      case YYG_TABLE_RADIAL:
        if (n != (size_t)4 * d->n_r * (L + 1)) return YYG_ERR_INVALID_ARG;
        yyg::radial_coefficients(d->n_r, d->r_edges, L, out);
        return YYG_OK;
      case YYG_TABLE_CROSS:
        if (n != 3 * nang) return YYG_ERR_INVALID_ARG;
        if (g.polar) return YYG_ERR_UNSUPPORTED;
        yyg::cross_points(g, out);
        return YYG_OK;
      case YYG_TABLE_ROTATION:
        if (n != (size_t)yyg::rotation_blocks_size(L)) return YYG_ERR_INVALID_ARG;
        yyg::rotation_blocks(L, out);
        return YYG_OK;
      default:
        return YYG_ERR_INVALID_ARG;
    }
  } catch (const std::bad_alloc &) {
    return YYG_ERR_OUT_OF_MEMORY;
  }
}

}  // extern "C"
