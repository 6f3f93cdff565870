// Host FP64 builders of the density-independent tables of a Yin-Yang plan.
#pragma once

#include <cstddef>
#include <vector>

#include "yyg.h"

namespace yyg {

// YYG_OK, or YYG_ERR_INVALID_ARG when a field of d is outside its documented
// range (yyg.h, yyg_grid_desc).
int validate_desc(const yyg_grid_desc *d);

// Column index of (l, m, cos/sin) in the Q = (L+1)^2 spherical-harmonic
// columns: q(l,0) = l^2, q(l,m,cos) = l^2 + 2m - 1, q(l,m,sin) = l^2 + 2m.
inline int qcol(int l, int m, int is_sin) { return m == 0 ? l * l : l * l + 2 * m - 1 + is_sin; }

struct ColInfo {
  int l, m, is_sin;
};
std::vector<ColInfo> column_table(int L);

struct PatchGeom {
  int n_t = 0, n_p = 0;
  double d_t = 0, d_p = 0;
  bool polar = false;          // full-sphere polar grid (one patch, no overlap)
  std::vector<double> th, ph;  // edges, n+1 each
};
PatchGeom make_patch(int n_t, int n_p, double d_t, double d_p);
// spherical polar grid of Sect. 2: theta in [0, pi], phi in [0, 2 pi]
PatchGeom make_polar_patch(int n_t, int n_p);

// resolution rule n = ceil(span/res) + 2, buffers split the surplus
void dims_from_resolution(double res_deg, int *n_t, int *n_p, double *d_t, double *d_p);

// exact overlap weights w[j*n_p + k] (Sect. 4, Eq. 25), closed-form areas;
// 1 everywhere on the polar grid
void overlap_weights(const PatchGeom &g, double *w);

// Schmidt-type normalised Legendre values pbar[q-independent index lm]
// pbar_l^m(x) = sqrt((2 - delta_m0) (l-m)!/(l+m)!) P_l^m(x), Condon-Shortley
// phase; out indexed [l*(L+1) + m].
void legendre_normalised(int L, double x, double s, double *out);

// sqrt((2 - delta_m0) (l-m)!/(l+m)!) for l, m <= L, indexed [l*(L+1)+m]
std::vector<double> norm_sqrt(int L);

// T-bar_j^(q) = sqrt(N^(lm)) T_j^(lm) at [j*Q + q] (same in cos/sin cols),
// Gauss-Legendre quadrature in theta of sin(t) pbar_l^m(cos t).
void theta_table_normalised(const PatchGeom &g, int L, double *out);

// C_k^(m) / S_k^(m) (Eqs. 14-15) at [k*Q + q]
void phi_table(const PatchGeom &g, int L, double *out);

// radial coefficients [n][l][4] = alpha, beta, gamma, kappa (see yyg.h)
void radial_coefficients(int n_r, const double *r, int L, double *out);

// (cos t', sin t', phi') of every cell midpoint in the other frame, [a][3]
void cross_points(const PatchGeom &g, double *out);

// Synthesis bases: self part pbar(cos t_j) at [j*Q+q], trig(m phi_k) at [k*Q+q];
// cross part pbar(cos t') trig(m phi') at [a*Q+q].
void self_legendre_table(const PatchGeom &g, int L, double *out);
void self_trig_table(const PatchGeom &g, int L, double *out);
void cross_basis(const PatchGeom &g, int L, double *out);

// ---- separable form (phi transform, theta transform, patch rotation) -----
// Azimuthal column index of (m, cos/sin): mc = 0 for m = 0, 2m-1 / 2m for
// cos / sin, so that q(l, m, c) = l^2 + mc.  2L+1 columns.


// CS[mc][k] = C_k^(m) or S_k^(m) (Eqs. 14-15), rows of length ldk (zero padded)
void separable_cs(const PatchGeom &g, int L, long ldk, double *out);

// trig[k][mc] = cos / sin (m phi_k) at the cell midpoints, rows of length ldm
void separable_trig(const PatchGeom &g, int L, long ldm, double *out);

// Per degree l, the (2l+1) x (2l+1) block D_l with
//   Ybar_q(R x) = sum_q' D_l[q - l^2][q' - l^2] Ybar_q'(x),
// where R is the Yin <-> Yang map (x, y, z) -> (-x, z, y) and Ybar_q are the
// sqrt(N)-normalised real harmonics of the plan.  Blocks are stored one
// after the other (offset of block l: sum_{l' < l} (2l'+1)^2), row-major.
// Computed by Gauss-Legendre x uniform-phi quadrature, exact for the
// degree-2l products.
void rotation_blocks(int L, double *out);
long rotation_blocks_size(int L);

}  // namespace yyg
