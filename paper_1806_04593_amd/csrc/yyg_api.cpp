// C ABI of the Yin-Yang multipole solver: plan creation (tables), density
// upload, solve, exports.  See include/yyg.h for the contract.
#include "yyg.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <new>
#include <vector>

#include "yyg_internal.h"
#include "yyg_tables.h"

namespace {

constexpr int kSlots = 8;

struct TimedLaunch {
  int slot;
  hipEvent_t start, stop;
};

long round_up(long v, long m) { return (v + m - 1) / m * m; }

// Device memory the library holds, process-wide, against an optional cap:
// the environment variable YYG_MAX_DEVICE_BYTES (a decimal byte count; unset,
// empty, 0 or not a plain number: no cap), read at every allocation.  An
// allocation that would take the total past the cap fails like a failed
// hipMalloc, before the runtime is asked.
std::mutex g_mem_mu;
std::unordered_map<void *, size_t> g_mem_sizes;
size_t g_mem_held = 0;

size_t mem_cap() {
  const char *e = std::getenv("YYG_MAX_DEVICE_BYTES");
  if (!e || !*e) return 0;
  char *end = nullptr;
  const unsigned long long v = std::strtoull(e, &end, 10);
  return (end && *end == '\0' && e[0] != '-') ? (size_t)v : 0;
}

hipError_t dev_malloc(void **p, size_t bytes) {
  std::lock_guard<std::mutex> lock(g_mem_mu);
  const size_t cap = mem_cap();
  if (cap && (bytes > cap || g_mem_held > cap - bytes)) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  const hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return e;
  }
  if (*p) {
    g_mem_sizes[*p] = bytes;
    g_mem_held += bytes;
  }
  return hipSuccess;
}

hipError_t dev_free(void *p) {
  if (!p) return hipSuccess;
  {
    std::lock_guard<std::mutex> lock(g_mem_mu);
    auto it = g_mem_sizes.find(p);
    if (it != g_mem_sizes.end()) {
      g_mem_held -= it->second;
      g_mem_sizes.erase(it);
    }
  }
  return hipFree(p);
}

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace

struct yyg_grid {
  int device = 0;
  int kind = YYG_GRID_YINYANG;
  int n_patch = 2;       // patches: 2 (Yin-Yang) or 1 (polar)
  int n_r = 0, n_t = 0, n_p = 0, L = 0, Q = 0;
  double G = 1.0;
  long nang = 0, ldb = 0, ldy = 0;
  int nsplit = 1;        // split-K factor of the analysis contraction
  int var_ana = 0;       // tile variant of the analysis contraction
  int var_syn = 0;       // tile variant of the synthesis contraction
  int part_cap = 1;      // splits the partial-moment buffer can hold
  int part_gen = 0;      // bumped whenever the partial-moment buffer moves
  std::vector<double> r_edges, w_host, nrm_q;
  yyg::PatchGeom geom;

  double *d_Bt = nullptr;    // analysis basis [Q][ldb]
  double *d_Y = nullptr;     // synthesis basis [nang][ldy], self | cross (cross on Yin-Yang only)
  double *d_coef = nullptr;  // radial coefficients [n_r][L+1][4]
  int *d_qdeg = nullptr;     // degree l of each column
  double *d_part = nullptr;  // split-K partial moments [nsplit][P n_r][Q]
  double *d_Ahat = nullptr;  // reduced moments (sqrt(N) scaled) [P n_r][Q], or [Q][P n_r] after a separable solve
  bool ahat_cols = false;    // d_Ahat holds the column-major layout
  double *d_U = nullptr;     // synthesis operand [P n_r][ldy]
  double *d_rho_owned = nullptr;
  int cus = 256;  // compute units of the device (persistent grids)
  // opt-in check of the density for NaN / infinity before each solve
  bool check_finite = false;
  int *d_flag = nullptr;
  const double *rho = nullptr;

  // reduced-precision tables, index prec - 1 (FP32, BF16x3, FP16x2)
  struct Lp {
    bool ready = false;
    void *Bt = nullptr;  // analysis basis planes [parts][Q][ldb]
    int *eBt = nullptr;  // row exponents of the analysis basis
    long ldb = 0;
    void *Y = nullptr;   // synthesis basis planes [parts][nang][ldy]
    int *eY = nullptr;
    long ldy = 0;
    void *Ar = nullptr;  // density planes [parts][2 n_r][lda], split per solve
    long lda = 0;
    void *Ur = nullptr;  // synthesis-operand planes [parts][2 n_r][ldu]
    long ldu = 0;
    int var_ana = 0, nsplit = 1, var_syn = 0;
  } lp[3];
  int *d_eA = nullptr;  // row exponents of the density (FP16x2)
  int *d_eU = nullptr;  // row exponents of the synthesis operand (FP16x2)

  // separable form
  int method = YYG_METHOD_DENSE;
  struct Sep {
    bool ready = false;
    long ldk = 0, ldm = 0, ldl = 0;
    double *Wcs = nullptr;   // weighted phi-analysis basis [n_t][2L+1][ldk]: w_jk C/S_k^(m)
    double *trig = nullptr;  // phi-synthesis basis [n_p][ldm]
    double *T2 = nullptr;    // theta-analysis basis [mc][l][n_t]: sqrt(N) T_j^(lm)
    double *P2 = nullptr;    // theta-synthesis basis [mc][j][ldl]: sqrt(N) P_l^m(cos t_j)
    double *Drot = nullptr;  // per degree l: the rotation block D_l (d x d), one after the other
    double *X2 = nullptr;    // phi-analysis output [mc][j][row]
    double *V = nullptr;     // theta-synthesis output [mc][j][row]
    double *At = nullptr;    // own + rotated other moments, column-major [Q][row] (Yin-Yang)
    double *Ut = nullptr;    // potential coefficients of own + rotated other moments [mc][l][row]
    double *coefS = nullptr; // radial recurrence coefficients [L+1][4][n_r]
    // phi phases, strided batches over the colatitudes j: analysis (C
    // stored column-major) and synthesis (A stored k-major)
    yyg::GemmF64Args phi_ana{}, phi_syn{};
    // the same two as LDS-basis kernels
    yyg::PhiDirectArgs phi_ana_d{}, phi_syn_d{};
    // the same two folded about the patch's central meridian (the tile
    // variants use these when the grid is mirror-symmetric: fold = true)
    bool fold = false;
    long h = 0, ldkh = 0, ks = 0, ldtf = 0;  // folded length, its row stride; synthesis split and row stride
    long kca = 0, nba = 0, kcs = 0, nks = 0;  // folded LDS-basis kernels: cos rows / slots and totals
    double *WF = nullptr;    // folded analysis basis [n_t][2][L+1][ldkh]: even (cos) / odd (sin) halves
    double *TF = nullptr;    // folded synthesis basis [h][ldtf]: cos m at m, sin m at ks + m - 1
    yyg::GemmF64Args phi_ana_f{}, phi_syn_f{};
    yyg::PhiStreamArgs phi_syn_s{};  // streaming folded synthesis
    yyg::PhiAnaStreamArgs phi_ana_s{};  // streaming folded analysis
    double *CSF = nullptr;  // its colatitude-independent folded basis [16 (nte + nto)][ldcs]
    double *Wt = nullptr;   // its folded overlap weights [n_t][ldcs]
    // folded analysis, both halves per block: basis rows cos m at slot m
    // (m <= L), sin m at slot ks + m - 1, [n_t][ks + L][ldkh], exact weights
    double *WFAB = nullptr;
    yyg::GemmF64Args phi_ana_ab{};
    // folded LDS-basis kernels: the cos / sin halves without padding each to
    // the tile width
    double *WFD = nullptr;   // analysis basis [n_t][kca + 16 ceil(L/16)][h]: cos m at row m, sin m at kca + m - 1
    double *TFD = nullptr;   // synthesis basis [h][kcs + 4 ceil(L/4)]: cos m at slot m, sin m at kcs + m - 1
    yyg::PhiDirectArgs phi_ana_fd{}, phi_syn_fd{};
    // folded phi synthesis with the fragments loaded straight from memory
    double *BK = nullptr;    // its basis, slot-major [kcs + 4 ceil(L/4)][hp]
    long hp = 0;             // h padded to a multiple of 32
    yyg::PhiLeanArgs phi_syn_l{};
    // theta phases and rotation: one launch each over their problems
    yyg::SepPhaseArgs args{};
    // variant per phase (0 phi analysis, 1 theta analysis, 2 moment
    // rotation, 3 theta synthesis, 4 phi synthesis): v < V the tile v,
    // V + v the same with the deep prefetch, 2V + d (phi phases) the
    // LDS-basis kernel d, 2V + D + f (phi phases, fold) the folded
    // LDS-basis kernel f, 2V + D + F + e (phi synthesis, fold) the LDS-free
    // kernel e
    // defaults (before autotuning): 32 x 32 tiles, 64 x 32 for the theta
    // synthesis
    int var[5] = {10, 10, 10, 9, 10};
    // reduced-precision phi transforms (FP32, BF16 x 3): tile of the phi
    // analysis and of the phi synthesis (yyg::sep_lp_tile_count() shapes)
    int lpt[2][2] = {{0, 1}, {0, 1}};
  } sep;

  bool timing = false;
  std::vector<TimedLaunch> launches;
};

namespace {


hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Release the separable form's device buffers (after a failed build too,
// so that a retry starts from nothing).
void sep_release(yyg_grid *g) {
  auto &S = g->sep;
  double **b[] = {&S.Wcs, &S.trig, &S.T2, &S.P2, &S.Drot, &S.X2, &S.V,   &S.Ut,  &S.coefS,
                  &S.At,  &S.WF,   &S.TF, &S.WFD, &S.TFD,  &S.BK, &S.WFAB, &S.CSF, &S.Wt};
  for (double **x : b) {
    if (*x) (void)dev_free(*x);
    *x = nullptr;
  }
}

// Release the operand planes of one reduced precision of the dense form.
template <class LpPlan>
void lp_release(LpPlan &l) {
  void **b[] = {reinterpret_cast<void **>(&l.Bt), reinterpret_cast<void **>(&l.eBt), reinterpret_cast<void **>(&l.Y),
                reinterpret_cast<void **>(&l.eY), reinterpret_cast<void **>(&l.Ar), reinterpret_cast<void **>(&l.Ur)};
  for (void **x : b) {
    if (*x) (void)dev_free(*x);
    *x = nullptr;
  }
}

void free_grid(yyg_grid *g) {
  if (!g) return;
  double *bufs[] = {g->d_Bt, g->d_Y, g->d_coef, g->d_part, g->d_Ahat, g->d_U, g->d_rho_owned};
  (void)dev_free(g->d_flag);
  for (double *b : bufs)
    if (b) (void)dev_free(b);
  if (g->d_qdeg) (void)dev_free(g->d_qdeg);
  for (auto &l : g->lp) lp_release(l);
  if (g->d_eA) (void)dev_free(g->d_eA);
  if (g->d_eU) (void)dev_free(g->d_eU);
  sep_release(g);
  for (auto &t : g->launches) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  delete g;
}

template <class T>
int dmalloc(T **p, size_t count) {
  if (dev_malloc(reinterpret_cast<void **>(p), count * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return YYG_ERR_OUT_OF_MEMORY;
  }
  return YYG_OK;
}

// Record a start event if timing is on; returns the index of the record.
int timing_begin(yyg_grid *g, int slot, hipStream_t s) {
  if (!g->timing) return -1;
  TimedLaunch t{slot, nullptr, nullptr};
  if (hipEventCreate(&t.start) != hipSuccess || hipEventCreate(&t.stop) != hipSuccess) return -1;
  (void)hipEventRecord(t.start, s);
  g->launches.push_back(t);
  return (int)g->launches.size() - 1;
}
void timing_end(yyg_grid *g, int idx, hipStream_t s) {
  if (idx >= 0) (void)hipEventRecord(g->launches[idx].stop, s);
}

}  // namespace

namespace yyg {
int choose_split(long tiles, long K) {
  // Blocks resident at once: 256 CUs x 2 blocks.  Pick the smallest split
  // whose wave-quantised cost is within 10% of the best, keeping at least
  // four 16-wide k stages per split.
  const long slots = 512;
  long smax = std::max(1L, std::min(32L, K / 64));
  double best = 1e30;
  std::vector<double> cost(smax + 1);
  for (long s = 1; s <= smax; ++s) {
    long waves = (tiles * s + slots - 1) / slots;
    cost[s] = (double)waves / s;
    best = std::min(best, cost[s]);
  }
  for (long s = 1; s <= smax; ++s)
    if (cost[s] <= 1.1 * best) return (int)s;
  return 1;
}
}  // namespace yyg

namespace {

// Timing of one launch configuration: one warm-up, then the
// minimum over `reps` event-timed launches (timings are data-independent).
template <class F>
double time_launch(F launch, hipStream_t s, int reps) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return 1e30;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return 1e30;
  }
  double best = 1e30;
  if (launch() == hipSuccess && hipStreamSynchronize(s) == hipSuccess) {
    for (int r = 0; r < reps; ++r) {
      (void)hipEventRecord(a, s);
      hipError_t e = launch();
      (void)hipEventRecord(b, s);
      if (e != hipSuccess || hipEventSynchronize(b) != hipSuccess) {
        best = 1e30;
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, a, b);
      best = std::min(best, (double)ms);
    }
  }
  (void)hipGetLastError();
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return best;
}

std::string tune_key(int prec, int role, long M, long N, long K) {
  char buf[128];
  std::snprintf(buf, sizeof buf, "p%d r%d %ld %ld %ld", prec, role, M, N, K);
  return buf;
}

std::map<std::string, std::pair<int, int>> read_tune_cache(const char *path) {
  std::map<std::string, std::pair<int, int>> m;
  if (!path) return m;
  std::FILE *f = std::fopen(path, "r");
  if (!f) return m;
  char line[256];
  while (std::fgets(line, sizeof line, f)) {
    int p, r, v, sp;
    long M, N, K;
    if (std::sscanf(line, "p%d r%d %ld %ld %ld -> %d %d", &p, &r, &M, &N, &K, &v, &sp) == 7)
      m[tune_key(p, r, M, N, K)] = {v, sp};
  }
  std::fclose(f);
  return m;
}

}  // namespace


namespace {

// Variants of separable phase r: v < V the tile v, V + v the same with
// three stages of loads in flight (V = the FP64 tile variants); the phi
// phases (0, 4) also 2V + d, the LDS-basis kernel variant d (d < D), and
// 2V + D + f, its folded form f (F of them; mirror-symmetric grids only);
// the phi synthesis also 2V + D + F + e, the LDS-free folded kernel e.
// Every phase then takes X = yyg::x4_variant_count() tiles on the 4x4x4
// FP64 MFMA at the end of its range (sep_x4_base).
int sep_x4_base(int r) {
  const int v = 2 * yyg::gemm_f64_variant_count();
  const int phi = yyg::phi_direct_variant_count() + yyg::phi_fold_variant_count();
  return r == 0 ? v + phi : r == 4 ? v + phi + yyg::phi_lean_variant_count() : v;
}

// The phi transforms then take the streaming kernels after those (folded
// grids only): yyg::phi_ana_stream_variant_count() for the analysis,
// yyg::phi_stream_variant_count() for the synthesis.
int sep_stream_base(int r) { return sep_x4_base(r) + yyg::x4_variant_count(r); }

int sep_stream_count(int r) {
  return r == 0 ? yyg::phi_ana_stream_variant_count() : r == 4 ? yyg::phi_stream_variant_count() : 0;
}

// The phi analysis last takes yyg::fold_xcol_variant_count() folded tiles
// whose last output column is summed on the vector units (folded grids only).
int sep_xcol_base(int r) { return sep_stream_base(r) + sep_stream_count(r); }

int sep_variant_count(int r) { return sep_xcol_base(r) + (r == 0 ? yyg::fold_xcol_variant_count() : 0); }

bool sep_fold_variant(int r, int v) {
  if ((r == 0 || r == 4) && v >= sep_stream_base(r)) return true;
  if (v >= sep_x4_base(r)) return yyg::x4_fold_only(r, v - sep_x4_base(r)) != 0;
  return (r == 0 || r == 4) && v >= 2 * yyg::gemm_f64_variant_count() + yyg::phi_direct_variant_count();
}

// Whether variant v of phase r can run on this plan's grid and degree.
bool sep_variant_available(const yyg_grid *g, int r, int v) {
  if (r < 0 || r > 4 || v < 0 || v >= sep_variant_count(r)) return false;
  if (sep_fold_variant(r, v) && !g->sep.fold) return false;
  if (r == 4 && v >= sep_stream_base(4)) return yyg::phi_stream_supports(v - sep_stream_base(4), g->L);
  if (r == 0 && v >= sep_xcol_base(0)) return true;
  if (r == 0 && v >= sep_stream_base(0))
    return yyg::phi_ana_stream_supports(v - sep_stream_base(0), (int)g->sep.h, g->n_p);
  return true;
}

int sep_set_variant(yyg_grid *g, int r, int v) {
  if (r < 0 || r > 4 || v < 0 || v >= sep_variant_count(r)) return YYG_ERR_INVALID_ARG;
  if (!sep_variant_available(g, r, v)) return YYG_ERR_UNSUPPORTED;
  g->sep.var[r] = v;
  return YYG_OK;
}

hipError_t sep_launch_phase(yyg_grid *g, int r, hipStream_t s) {
  auto &S = g->sep;
  const int nv = yyg::gemm_f64_variant_count(), nd = yyg::phi_direct_variant_count();
  const int nf = yyg::phi_fold_variant_count();
  if (r == 4 && S.var[r] >= sep_stream_base(4))
    return yyg::launch_phi_syn_stream(S.var[r] - sep_stream_base(4), S.phi_syn_s, g->cus, s);
  if (r == 0 && S.var[r] >= sep_xcol_base(0)) return yyg::launch_fold_xcol(S.var[r] - sep_xcol_base(0), S.phi_ana_f, s);
  if (r == 0 && S.var[r] >= sep_stream_base(0))
    return yyg::launch_phi_ana_stream(S.var[r] - sep_stream_base(0), S.phi_ana_s, g->cus, s);
  if (S.var[r] >= sep_x4_base(r)) {
    if (r == 2 && g->n_patch != 2) return hipSuccess;
    const yyg::GemmF64Args &phi = r == 0 ? (S.fold ? S.phi_ana_f : S.phi_ana) : (S.fold ? S.phi_syn_f : S.phi_syn);
    return yyg::launch_x4_sep_phase(S.var[r] - sep_x4_base(r), r, S.fold, phi, S.phi_ana_ab, S.args, s);
  }
  if (r == 4 && S.var[r] >= 2 * nv + nd + nf) return yyg::launch_phi_syn_lean(S.var[r] - 2 * nv - nd - nf, S.phi_syn_l, s);
  if (sep_fold_variant(r, S.var[r]))
    return yyg::launch_phi_fold(S.var[r] - 2 * nv - nd, r == 0, r == 0 ? S.phi_ana_fd : S.phi_syn_fd, s);
  if ((r == 0 || r == 4) && S.var[r] >= 2 * nv)
    return yyg::launch_phi_direct(S.var[r] - 2 * nv, r == 0, r == 0 ? S.phi_ana_d : S.phi_syn_d, s);
  const int v = S.var[r] % nv;
  const bool deep = S.var[r] >= nv;
  const int dr = deep ? yyg::kRoleDeep : 0;
  if (r == 0) return yyg::launch_gemm_f64_batched(v, (S.fold ? 2 : 0) + dr, S.fold ? S.phi_ana_f : S.phi_ana, s);
  if (r == 4) return yyg::launch_gemm_f64_batched(v, (S.fold ? 3 : 1) + dr, S.fold ? S.phi_syn_f : S.phi_syn, s);
  if (r == 2 && g->n_patch != 2) return hipSuccess;  // one patch: nothing to rotate
  return yyg::launch_gemm_f64_sep(v, r, deep, S.args, s);
}

// Work buffers of the separable form: the plan's own, or (allocation-free
// solve) regions of the device scratch array.
struct SepWork {
  double *X2, *V, *Ut, *At, *Ahat;
};

SepWork sep_work(const yyg_grid *g) { return {g->sep.X2, g->sep.V, g->sep.Ut, g->sep.At, g->d_Ahat}; }

// Point every launch argument of the separable form at the work buffers w.
void sep_bind_work(yyg_grid *g, const SepWork &w) {
  auto &S = g->sep;
  S.X2 = w.X2;
  S.V = w.V;
  S.Ut = w.Ut;
  S.At = w.At;
  g->d_Ahat = w.Ahat;
  S.phi_ana.C = S.phi_ana_f.C = S.phi_ana_ab.C = w.X2;
  S.phi_ana_d.C = S.phi_ana_fd.C = w.X2;
  S.phi_syn.A = S.phi_syn_f.A = w.V;
  S.phi_syn_s.V = w.V;
  S.phi_ana_s.X2 = w.X2;
  S.phi_syn_d.X = S.phi_syn_fd.X = w.V;
  S.phi_syn_l.V = w.V;
  S.args.X2 = w.X2;
  S.args.Ut = w.Ut;
  S.args.Ahat = w.Ahat;
  S.args.At = w.At;
  S.args.V = w.V;
}

// Doubles of the separable form's work buffers, each region rounded up to
// 256 bytes.
size_t sep_work_doubles(const yyg_grid *g) {
  const long M = (long)g->n_patch * g->n_r, nmc = 2L * g->L + 1;
  auto r32 = [](long v) { return (size_t)((v + 31) / 32 * 32); };
  return 2 * r32(nmc * g->n_t * M) + r32(nmc * (g->L + 1) * M) + (g->n_patch == 2 ? r32(M * g->Q) : 0) +
         r32(M * g->Q);
}

// Point the phi phases at this solve's density and potential (kernel
// arguments: nothing is copied).
int sep_set_pointers(yyg_grid *g, const double *rho, double *phi, hipStream_t) {
  g->sep.phi_ana.A = rho;
  g->sep.phi_syn.C = phi;
  g->sep.phi_ana_d.X = rho;
  g->sep.phi_syn_d.C = phi;
  g->sep.phi_ana_f.A = rho;
  g->sep.phi_ana_s.rho = rho;
  g->sep.phi_ana_ab.A = rho;
  g->sep.phi_syn_f.C = phi;
  g->sep.phi_syn_s.phi = phi;
  g->sep.phi_ana_fd.X = rho;
  g->sep.phi_syn_fd.C = phi;
  g->sep.phi_syn_l.C = phi;
  return YYG_OK;
}

int sep_build(yyg_grid *g) {
  auto &S = g->sep;
  const int L = g->L, Q = g->Q, nmc = 2 * L + 1, nt = g->n_t, np = g->n_p;
  const long M = (long)g->n_patch * g->n_r;
  const long MJ = M * nt;  // (row, j) pairs
  S.ldk = round_up(np, 16);
  S.ldm = round_up(nmc, 16);
  S.ldl = round_up(L + 1, 16);
  if (!yyg::radial_scan_q_supports(g->n_r, g->n_patch)) return YYG_ERR_UNSUPPORTED;
  std::vector<double> CSt, Wcs, trig, T, P, T2, P2, D, coef, coefS, WF, TF, WFD, TFD, BK, WFAB, CSF, WTF;
  int nte = 0, nto = 0, ldcs = 0;
  try {
    coef.resize((size_t)4 * g->n_r * (L + 1));
    yyg::radial_coefficients(g->n_r, g->r_edges.data(), L, coef.data());
    coefS.resize(coef.size());
    for (int n = 0; n < g->n_r; ++n)
      for (int l = 0; l <= L; ++l)
        for (int k = 0; k < 4; ++k)
          coefS[((size_t)l * 4 + k) * g->n_r + n] = coef[((size_t)n * (L + 1) + l) * 4 + k];
    CSt.resize((size_t)nmc * S.ldk);
    yyg::separable_cs(g->geom, L, S.ldk, CSt.data());
    // the overlap weights folded into one basis copy per colatitude
    Wcs.assign((size_t)nt * nmc * S.ldk, 0.0);
    for (int j = 0; j < nt; ++j)
      for (int mc = 0; mc < nmc; ++mc)
        for (int k = 0; k < np; ++k)
          Wcs[((size_t)j * nmc + mc) * S.ldk + k] = g->w_host[(size_t)j * np + k] * CSt[(size_t)mc * S.ldk + k];
    trig.resize((size_t)np * S.ldm);
    yyg::separable_trig(g->geom, L, S.ldm, trig.data());
    // Mirror symmetry about the central meridian: the cell centres, overlap
    // weights and cos / sin bases are even / odd under k -> n_p - 1 - k (up
    // to rounding), so each phi transform folds into an even and an odd
    // half of ceil(n_p / 2) points.  The bases are closed forms, symmetric
    // to a few ulps; a weight is the covered fraction of a cell, the
    // difference of O(1) terms over the cell's solid angle, so its rounding
    // grows as the cells shrink (1.5e-12 between mirror cells at 0.5 deg):
    // the weights are checked to 1e-10 (an asymmetric grid is off by the
    // partial cells' O(1e-3) and more) and each mirror pair takes their mean,
    // as close to the exact fraction as either.
    {
      double cmax = 0.0, tmax = 0.0, wbad = 0.0, cbad = 0.0, tbad = 0.0;
      for (int mc = 0; mc < nmc; ++mc)
        for (int k = 0; k < np; ++k) {
          cmax = std::max(cmax, std::fabs(CSt[(size_t)mc * S.ldk + k]));
          tmax = std::max(tmax, std::fabs(trig[(size_t)k * S.ldm + mc]));
        }
      for (int k = 0; k < np; ++k) {
        const int km = np - 1 - k;
        for (int j = 0; j < nt; ++j)
          wbad = std::max(wbad, std::fabs(g->w_host[(size_t)j * np + k] - g->w_host[(size_t)j * np + km]));
        for (int mc = 0; mc < nmc; ++mc) {
          const double sg = (mc > 0 && mc % 2 == 0) ? -1.0 : 1.0;  // sin columns are odd
          cbad = std::max(cbad, std::fabs(CSt[(size_t)mc * S.ldk + k] - sg * CSt[(size_t)mc * S.ldk + km]));
          tbad = std::max(tbad, std::fabs(trig[(size_t)k * S.ldm + mc] - sg * trig[(size_t)km * S.ldm + mc]));
        }
      }
      S.fold = np >= 2 && wbad <= 1e-10 && cbad <= 1e-12 * cmax && tbad <= 1e-12 * tmax;
    }
    S.h = (np + 1) / 2;
    S.ldkh = round_up(S.h, 16);
    S.ks = round_up(L + 1, 16);
    S.ldtf = S.ks + round_up(L, 16);
    if (S.fold) {
      const int h = S.h, mid = np % 2 ? h - 1 : -1;
      WF.assign((size_t)2 * nt * (L + 1) * S.ldkh, 0.0);
      TF.assign((size_t)h * S.ldtf, 0.0);
      for (int j = 0; j < nt; ++j)
        for (int k = 0; k < h; ++k) {
          // one weight per mirror pair (equal up to rounding); the middle
          // cell enters the even half twice
          const double wb = 0.5 * (g->w_host[(size_t)j * np + k] + g->w_host[(size_t)j * np + np - 1 - k]);
          const double f = (k == mid ? 0.5 : 1.0) * wb;
          for (int m = 0; m <= L; ++m) {
            WF[(((size_t)j * 2 + 0) * (L + 1) + m) * S.ldkh + k] = f * CSt[(size_t)(m ? 2 * m - 1 : 0) * S.ldk + k];
            if (m > 0)
              WF[(((size_t)j * 2 + 1) * (L + 1) + m - 1) * S.ldkh + k] = f * CSt[(size_t)(2 * m) * S.ldk + k];
          }
        }
      for (int k = 0; k < h; ++k)
        for (int m = 0; m <= L; ++m) {
          TF[(size_t)k * S.ldtf + m] = trig[(size_t)k * S.ldm + (m ? 2 * m - 1 : 0)];
          if (m > 0) TF[(size_t)k * S.ldtf + S.ks + m - 1] = trig[(size_t)k * S.ldm + 2 * m];
        }
      // the streaming analysis: the folded C / S rows without the weights
      // (cos outputs m = 0..L in tiles of 16, then sin outputs m = 1..L) and
      // the weights per colatitude, the middle cell's half in the weight
      nte = (L + 16) / 16;
      nto = (L + 15) / 16;
      ldcs = (int)round_up(h, 16);
      CSF.assign((size_t)16 * (nte + nto) * ldcs, 0.0);
      WTF.assign((size_t)nt * ldcs, 0.0);
      for (int k = 0; k < h; ++k) {
        for (int m = 0; m <= L; ++m) {
          CSF[(size_t)m * ldcs + k] = CSt[(size_t)(m ? 2 * m - 1 : 0) * S.ldk + k];
          if (m > 0) CSF[((size_t)16 * nte + m - 1) * ldcs + k] = CSt[(size_t)(2 * m) * S.ldk + k];
        }
        for (int j = 0; j < nt; ++j)
          WTF[(size_t)j * ldcs + k] =
              (k == mid ? 0.5 : 1.0) * 0.5 * (g->w_host[(size_t)j * np + k] + g->w_host[(size_t)j * np + np - 1 - k]);
      }
      // both halves in one basis for kGemmFoldAB: slot s < ks the cos half,
      // ks <= s < ks + L the sin half
      WFAB.assign((size_t)nt * (S.ks + L) * S.ldkh, 0.0);
      for (int j = 0; j < nt; ++j)
        for (int m = 0; m <= L; ++m)
          for (int k = 0; k < h; ++k) {
            const size_t base = (size_t)j * (S.ks + L);
            WFAB[(base + m) * S.ldkh + k] = WF[(((size_t)j * 2 + 0) * (L + 1) + m) * S.ldkh + k];
            if (m > 0) WFAB[(base + S.ks + m - 1) * S.ldkh + k] = WF[(((size_t)j * 2 + 1) * (L + 1) + m - 1) * S.ldkh + k];
          }
      // the same for the folded LDS-basis kernels: the cos half padded to a
      // multiple of 16 rows (analysis) / 4 slots (synthesis), the sin half
      // after it
      S.kca = round_up(L + 1, 16);
      S.kcs = round_up(L + 1, 4);
      S.nba = S.kca + round_up(L, 16);
      S.nks = S.kcs + round_up(L, 4);
      WFD.assign((size_t)nt * S.nba * h, 0.0);
      TFD.assign((size_t)h * S.nks, 0.0);
      for (int j = 0; j < nt; ++j)
        for (int m = 0; m <= L; ++m)
          for (int k = 0; k < h; ++k) {
            const double *wf = &WF[((size_t)j * 2 * (L + 1)) * S.ldkh + k];
            WFD[((size_t)j * S.nba + m) * h + k] = wf[(size_t)m * S.ldkh];
            if (m > 0) WFD[((size_t)j * S.nba + S.kca + m - 1) * h + k] = wf[(size_t)(L + 1 + m - 1) * S.ldkh];
          }
      for (int k = 0; k < h; ++k)
        for (int m = 0; m <= L; ++m) {
          TFD[(size_t)k * S.nks + m] = TF[(size_t)k * S.ldtf + m];
          if (m > 0) TFD[(size_t)k * S.nks + S.kcs + m - 1] = TF[(size_t)k * S.ldtf + S.ks + m - 1];
        }
      // the same synthesis basis slot-major, cells padded to a multiple of 32
      S.hp = round_up(h, 32);
      BK.assign((size_t)S.nks * S.hp, 0.0);
      for (long sl = 0; sl < S.nks; ++sl)
        for (int k = 0; k < h; ++k) BK[(size_t)sl * S.hp + k] = TFD[(size_t)k * S.nks + sl];
    }
    T.resize((size_t)nt * Q);
    yyg::theta_table_normalised(g->geom, L, T.data());
    P.resize((size_t)nt * Q);
    yyg::self_legendre_table(g->geom, L, P.data());
    // azimuthal-column-major copies for the theta GEMMs
    T2.assign((size_t)nmc * (L + 1) * nt, 0.0);
    P2.assign((size_t)nmc * nt * S.ldl, 0.0);
    for (int mc = 0; mc < nmc; ++mc) {
      const int m = (mc + 1) / 2;
      for (int l = m; l <= L; ++l)
        for (int j = 0; j < nt; ++j) {
          T2[((size_t)mc * (L + 1) + l) * nt + j] = T[(size_t)j * Q + l * l + mc];
          P2[((size_t)mc * nt + j) * S.ldl + l] = P[(size_t)j * Q + l * l + mc];
        }
    }
    // per degree: D_l (the rotation phase starts its accumulators from a
    // patch's own moments and adds the other patch's moments times D_l)
    D.resize(yyg::rotation_blocks_size(L));
    yyg::rotation_blocks(L, D.data());
  } catch (const std::bad_alloc &) {
    return YYG_ERR_OUT_OF_MEMORY;
  }
  int st = YYG_OK;
  if (st == YYG_OK) st = dmalloc(&S.Wcs, Wcs.size());
  if (st == YYG_OK) st = dmalloc(&S.trig, trig.size());
  if (st == YYG_OK) st = dmalloc(&S.T2, T2.size());
  if (st == YYG_OK) st = dmalloc(&S.P2, P2.size());
  if (st == YYG_OK) st = dmalloc(&S.Drot, D.size());
  if (st == YYG_OK) st = dmalloc(&S.X2, (size_t)nmc * MJ);
  if (st == YYG_OK) st = dmalloc(&S.V, (size_t)nmc * MJ);
  if (st == YYG_OK) st = dmalloc(&S.Ut, (size_t)nmc * (L + 1) * M);
  if (st == YYG_OK && g->n_patch == 2) st = dmalloc(&S.At, (size_t)M * Q);
  if (st == YYG_OK) st = dmalloc(&S.coefS, coefS.size());
  if (st == YYG_OK && S.fold) st = dmalloc(&S.WF, WF.size());
  if (st == YYG_OK && S.fold) st = dmalloc(&S.TF, TF.size());
  if (st == YYG_OK && S.fold) st = dmalloc(&S.WFD, WFD.size());
  if (st == YYG_OK && S.fold) st = dmalloc(&S.TFD, TFD.size());
  if (st == YYG_OK && S.fold) st = dmalloc(&S.BK, BK.size());
  if (st == YYG_OK && S.fold) st = dmalloc(&S.WFAB, WFAB.size());
  if (st == YYG_OK && S.fold) st = dmalloc(&S.CSF, CSF.size());
  if (st == YYG_OK && S.fold) st = dmalloc(&S.Wt, WTF.size());
  if (st != YYG_OK) {
    sep_release(g);
    return st;
  }
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t r) {
    if (e == hipSuccess && r != hipSuccess) e = r;
  };
  chk(hipMemcpy(S.Wcs, Wcs.data(), Wcs.size() * sizeof(double), hipMemcpyHostToDevice));
  chk(hipMemcpy(S.trig, trig.data(), trig.size() * sizeof(double), hipMemcpyHostToDevice));
  chk(hipMemcpy(S.T2, T2.data(), T2.size() * sizeof(double), hipMemcpyHostToDevice));
  chk(hipMemcpy(S.P2, P2.data(), P2.size() * sizeof(double), hipMemcpyHostToDevice));
  chk(hipMemcpy(S.Drot, D.data(), D.size() * sizeof(double), hipMemcpyHostToDevice));
  chk(hipMemcpy(S.coefS, coefS.data(), coefS.size() * sizeof(double), hipMemcpyHostToDevice));
  if (S.fold) {
    chk(hipMemcpy(S.WF, WF.data(), WF.size() * sizeof(double), hipMemcpyHostToDevice));
    chk(hipMemcpy(S.TF, TF.data(), TF.size() * sizeof(double), hipMemcpyHostToDevice));
    chk(hipMemcpy(S.WFD, WFD.data(), WFD.size() * sizeof(double), hipMemcpyHostToDevice));
    chk(hipMemcpy(S.TFD, TFD.data(), TFD.size() * sizeof(double), hipMemcpyHostToDevice));
    chk(hipMemcpy(S.BK, BK.data(), BK.size() * sizeof(double), hipMemcpyHostToDevice));
    chk(hipMemcpy(S.WFAB, WFAB.data(), WFAB.size() * sizeof(double), hipMemcpyHostToDevice));
    chk(hipMemcpy(S.CSF, CSF.data(), CSF.size() * sizeof(double), hipMemcpyHostToDevice));
    chk(hipMemcpy(S.Wt, WTF.data(), WTF.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    sep_release(g);
    return YYG_ERR_DEVICE;
  }
  auto kround = [](long k) { return (int)((k + 15) / 16 * 16); };
  // per colatitude j: X2[mc][j][row] = sum_k rho[row][j][k] w_jk CS_k^(mc)   (rho set per solve)
  S.phi_ana = yyg::GemmF64Args{(int)M, nmc, np, nullptr, (long)nt * np, S.Wcs, S.ldk, S.X2, MJ, M, kround(np), 1};
  S.phi_ana.batch = nt;
  S.phi_ana.a_batch = np;
  S.phi_ana.b_batch = (long)nmc * S.ldk;
  // per colatitude j: phi[row][j][k] = sum_mc V[mc][j][row] trig[k][mc]        (phi set per solve)
  S.phi_syn = yyg::GemmF64Args{(int)M, np, nmc, S.V, MJ, S.trig, S.ldm, nullptr, (long)nt * np, np, kround(nmc), 1};
  S.phi_syn.batch = nt;
  S.phi_syn.a_batch = M;
  // folded: even (cos) and odd (sin) halves of every row, h = ceil(n_p / 2)
  S.phi_ana_f = yyg::GemmF64Args{(int)M, L + 1, (int)S.h, nullptr, (long)nt * np, S.WF, S.ldkh, S.X2, MJ, M, kround(S.h), 1};
  S.phi_ana_f.batch = 2 * nt;
  S.phi_ana_f.a_batch = np;
  S.phi_ana_f.b_batch = (long)(L + 1) * S.ldkh;
  S.phi_ana_f.fold_k = np;
  S.phi_ana_f.fold_mc = nmc;
  // both halves per block: slots ks + L, the same density rows and output
  S.phi_ana_ab = yyg::GemmF64Args{(int)M, (int)(S.ks + L), (int)S.h, nullptr, (long)nt * np, S.WFAB, S.ldkh, S.X2, MJ,
                                  M, kround(S.h), 1};
  S.phi_ana_ab.batch = nt;
  S.phi_ana_ab.a_batch = np;
  S.phi_ana_ab.b_batch = (long)(S.ks + L) * S.ldkh;
  S.phi_ana_ab.k_split = (int)S.ks;
  S.phi_ana_ab.fold_k = np;
  S.phi_ana_ab.fold_mc = nmc;
  S.phi_syn_f = yyg::GemmF64Args{(int)M, (int)S.h, (int)S.ldtf, S.V, MJ, S.TF, S.ldtf, nullptr, (long)nt * np, np,
                                 kround(S.ldtf), 1};
  S.phi_syn_f.batch = nt;
  S.phi_syn_f.a_batch = M;
  S.phi_syn_f.k_split = (int)S.ks;
  S.phi_syn_f.fold_k = np;
  S.phi_syn_f.fold_mc = nmc;
  S.phi_syn_s = yyg::PhiStreamArgs{S.V, S.TF, nullptr, MJ, (long)nt * np, (int)M, nt, np, (int)S.h, L, nmc,
                                   (int)S.ldtf, (int)S.ks};
  S.phi_ana_s = yyg::PhiAnaStreamArgs{nullptr, S.CSF, S.Wt, S.X2, MJ, (long)nt * np, (int)M, nt, np, (int)S.h, L,
                                      nmc, ldcs, nte, nto};
  S.phi_ana_d = yyg::PhiDirectArgs{nullptr, S.Wcs, S.X2, (int)M, nt, nmc, np, S.ldk, (long)nmc * S.ldk};
  S.phi_syn_d = yyg::PhiDirectArgs{S.V, S.trig, nullptr, (int)M, nt, np, nmc, S.ldm, 0};
  S.phi_ana_fd = yyg::PhiDirectArgs{nullptr, S.WFD, S.X2, (int)M, nt, (int)S.nba, (int)S.h, S.h, S.nba * S.h,
                                    np, (int)S.kca, nmc};
  S.phi_syn_fd = yyg::PhiDirectArgs{S.V, S.TFD, nullptr, (int)M, nt, (int)S.h, (int)S.nks, S.nks, 0,
                                    np, (int)S.kcs, nmc};
  S.phi_syn_l = yyg::PhiLeanArgs{S.V, S.BK, nullptr, (int)M, nt, np, (int)S.h, (int)S.hp, (int)S.nks, (int)S.kcs, nmc};
  // theta analysis, rotation (Yin-Yang) and theta synthesis: problem
  // operands derived in the kernels from these
  S.args = yyg::SepPhaseArgs{L,    g->n_r, g->n_patch, nt,  S.ldl, S.X2, S.T2, S.P2,
                             S.Ut, S.Drot,   g->d_Ahat,  S.At, S.V};
  S.ready = true;
  return YYG_OK;
}

// Separable solve: phi analysis (a strided batch over the colatitudes),
// theta analysis (one problem per azimuthal column) into the column-major
// moments, own plus rotated other moments (Yin-Yang; one problem per degree
// and patch), radial scan into the azimuthal-column-major coefficients,
// theta synthesis (one problem per azimuthal column), phi synthesis (a
// strided batch over the colatitudes).
// A phi phase (0 or 4) in `precision`: the FP64 variant of the plan, or the
// plan's reduced-precision tile for FP32 / BF16 x 3.
// The opt-in input check: YYG_ERR_NONFINITE if rho holds a NaN or an
// infinity, YYG_OK if not or if the check is off.  Waits for the check on
// stream s; allocates nothing (the flag is the plan's).
int check_rho(yyg_grid *g, const double *rho, hipStream_t s) {
  if (!g->check_finite) return YYG_OK;
  const long n = (long)g->n_patch * g->n_r * g->nang;
  int h = 0;
  hipError_t e = yyg::launch_check_finite(rho, n, g->d_flag, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&h, g->d_flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return YYG_ERR_DEVICE;
  }
  return h ? YYG_ERR_NONFINITE : YYG_OK;
}

// Choices of a reduced-precision phi transform (side 0 analysis, 1
// synthesis): the tile shapes, and in FP32 on a folded grid also the FP32
// streaming kernels after them.
int sep_lp_choices(const yyg_grid *g, int precision, int side) {
  if (precision != YYG_FP32 || !g->sep.fold) return yyg::sep_lp_tile_count();
  return yyg::sep_lp_tile_count() +
         (side == 1 ? yyg::phi_stream32_variant_count() : yyg::phi_ana_stream32_variant_count());
}

bool sep_lp_available(const yyg_grid *g, int precision, int side, int t) {
  if (t < 0 || t >= sep_lp_choices(g, precision, side)) return false;
  const int u = t - yyg::sep_lp_tile_count();
  if (u < 0) return true;
  return side == 1 ? yyg::phi_stream32_supports(u, g->L) : yyg::phi_ana_stream32_supports(u, (int)g->sep.h, g->n_p);
}

hipError_t sep_launch_phi(yyg_grid *g, int r, int precision, hipStream_t s) {
  auto &S = g->sep;
  if (precision == YYG_FP64) return sep_launch_phase(g, r, s);
  if (r == 4 && precision == YYG_FP32 && S.lpt[0][1] >= yyg::sep_lp_tile_count())
    return yyg::launch_phi_syn_stream32(S.lpt[0][1] - yyg::sep_lp_tile_count(), S.phi_syn_s, g->cus, s);
  if (r == 0 && precision == YYG_FP32 && S.lpt[0][0] >= yyg::sep_lp_tile_count())
    return yyg::launch_phi_ana_stream32(S.lpt[0][0] - yyg::sep_lp_tile_count(), S.phi_ana_s, g->cus, s);
  const yyg::GemmF64Args &phi = r == 0 ? (S.fold ? S.phi_ana_f : S.phi_ana) : (S.fold ? S.phi_syn_f : S.phi_syn);
  return yyg::launch_sep_lp_phase(precision, S.lpt[precision - 1][r == 0 ? 0 : 1], r, S.fold, phi, s);
}

hipError_t sep_solve(yyg_grid *g, hipStream_t s, int precision = YYG_FP64) {
  auto &S = g->sep;
  hipError_t e = hipSuccess;
  g->ahat_cols = true;
  int t = timing_begin(g, 4, s);
  e = sep_launch_phi(g, 0, precision, s);
  timing_end(g, t, s);
  // the scan's input: the moments, or with two patches their rotated sum
  const double *scan_in = g->n_patch == 2 ? S.At : g->d_Ahat;
  if (e == hipSuccess) {
    t = timing_begin(g, 5, s);
    e = sep_launch_phase(g, 1, s);
    if (e == hipSuccess) e = sep_launch_phase(g, 2, s);
    timing_end(g, t, s);
  }
  if (e == hipSuccess) {
    t = timing_begin(g, 1, s);
    e = yyg::launch_radial_scan_q(scan_in, S.coefS, g->d_qdeg, g->n_r, g->L, -g->G, g->n_patch, S.Ut, s);
    timing_end(g, t, s);
  }
  if (e == hipSuccess) {
    t = timing_begin(g, 6, s);
    e = sep_launch_phase(g, 3, s);
    timing_end(g, t, s);
  }
  if (e == hipSuccess) {
    t = timing_begin(g, 7, s);
    e = sep_launch_phi(g, 4, precision, s);
    timing_end(g, t, s);
  }
  return e;
}

}  // namespace


struct yyg_batch {
  int device = 0;
  int precision = 0;
  std::vector<yyg_grid *> grids;
  std::vector<const double *> rho;
  std::vector<double *> phi;
  // per-field argument arrays: pinned host copies (pointer-patched per
  // solve) and their device mirrors, refreshed by a copy at the head of
  // the recorded graph
  yyg::GemmF64Args *h_f64[2] = {nullptr, nullptr}, *d_f64[2] = {nullptr, nullptr};
  yyg::GemmLpArgs *h_lp[2] = {nullptr, nullptr}, *d_lp[2] = {nullptr, nullptr};
  yyg::ScanArgs *d_scan = nullptr;
  yyg::SplitArgs *h_split[2] = {nullptr, nullptr}, *d_split[2] = {nullptr, nullptr};
  int4 *d_items[2] = {nullptr, nullptr};  // analysis / synthesis work items
  int n_items[2] = {0, 0};
  int var[2] = {0, 0};                    // tile variants
  int blocks[2] = {0, 0};                 // resident persistent blocks
  int4 *d_scan_items = nullptr;
  int n_scan_items = 0;
  int2 *d_split_items[2] = {nullptr, nullptr};
  int n_split_items[2] = {0, 0};
  int cus = 256;
  hipGraphExec_t exec = nullptr;
  hipStream_t exec_stream = nullptr;
  hipEvent_t done = nullptr;
  hipStream_t stream = nullptr;  // used when the caller passes the default stream
  bool launched = false;
  std::vector<int> part_gen;     // plans' partial-buffer generations the arguments hold
  // separable batches (FP64, every plan in the separable form): the five
  // phases and the column scans as grouped launches over all plans
  bool sep = false, sep_fold = false;
  yyg::GemmF64Args *h_phi[2] = {nullptr, nullptr}, *d_phi[2] = {nullptr, nullptr};  // phi analysis / synthesis
  yyg::SepPhaseArgs *d_sargs = nullptr;
  yyg::ScanQArgs *d_qscan = nullptr;
  int2 *d_qitems = nullptr;
  int n_qitems = 0, max_nr = 0;
  int4 *d_sitems[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int n_sitems[5] = {0, 0, 0, 0, 0};
  int svar[5] = {0, 0, 0, 0, 0};    // tile of each phase (yyg::sep_batch_tile)
  int sblocks[5] = {0, 0, 0, 0, 0};
};

namespace {

void batch_drop_graph(yyg_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
  b->exec_stream = nullptr;
}

void batch_free(yyg_batch *b) {
  if (!b) return;
  batch_drop_graph(b);
  for (int r = 0; r < 2; ++r) {
    if (b->h_f64[r]) (void)hipHostFree(b->h_f64[r]);
    if (b->h_lp[r]) (void)hipHostFree(b->h_lp[r]);
    if (b->h_split[r]) (void)hipHostFree(b->h_split[r]);
    void *d[] = {b->d_f64[r], b->d_lp[r], b->d_split[r], b->d_items[r], b->d_split_items[r]};
    for (void *x : d)
      if (x) (void)dev_free(x);
  }
  if (b->d_scan) (void)dev_free(b->d_scan);
  if (b->d_scan_items) (void)dev_free(b->d_scan_items);
  for (int r = 0; r < 2; ++r) {
    if (b->h_phi[r]) (void)hipHostFree(b->h_phi[r]);
    if (b->d_phi[r]) (void)dev_free(b->d_phi[r]);
  }
  for (int r = 0; r < 5; ++r)
    if (b->d_sitems[r]) (void)dev_free(b->d_sitems[r]);
  if (b->d_sargs) (void)dev_free(b->d_sargs);
  if (b->d_qscan) (void)dev_free(b->d_qscan);
  if (b->d_qitems) (void)dev_free(b->d_qitems);
  if (b->done) (void)hipEventDestroy(b->done);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

template <class T>
int upload(T **dst, const std::vector<T> &src) {
  if (*dst) (void)dev_free(*dst);
  *dst = nullptr;
  if (src.empty()) return YYG_OK;
  if (dev_malloc(reinterpret_cast<void **>(dst), src.size() * sizeof(T)) != hipSuccess) {
    *dst = nullptr;
    (void)hipGetLastError();
    return YYG_ERR_OUT_OF_MEMORY;
  }
  if (hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return YYG_ERR_DEVICE;
  }
  return YYG_OK;
}

// Work items of one contraction phase for tile variant v, largest K first
// so the persistent blocks finish together.
int batch_set_items(yyg_batch *b, int role, int v) {
  const bool lp = b->precision != YYG_FP64;
  int bm, bn;
  if (lp)
    yyg::gemm_lp_variant_tile(v, &bm, &bn);
  else
    yyg::gemm_f64_variant_tile(v, &bm, &bn);
  std::vector<std::pair<long, int4>> work;
  const int n = (int)b->grids.size();
  for (int f = 0; f < n; ++f) {
    const yyg_grid *g = b->grids[f];
    const long M = (long)g->n_patch * g->n_r, N = role == 0 ? g->Q : g->nang, K = role == 0 ? g->nang : (long)g->n_patch * g->Q;
    const int tm = (int)((M + bm - 1) / bm), tn = (int)((N + bn - 1) / bn);
    if (lp) {
      b->h_lp[role][f].tiles_m = tm;
    } else {
      b->h_f64[role][f].tiles_m = tm;
    }
    for (int j = 0; j < tn; ++j)
      for (int i = 0; i < tm; ++i) work.push_back({K, int4{f, i, j, 0}});
  }
  std::stable_sort(work.begin(), work.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
  std::vector<int4> items(work.size());
  for (size_t i = 0; i < work.size(); ++i) items[i] = work[i].second;
  int st = upload(&b->d_items[role], items);
  if (st != YYG_OK) return st;
  b->n_items[role] = (int)items.size();
  b->var[role] = v;
  // resident blocks: LDS-limited occupancy of the variant, four at most
  const int eb = lp ? yyg::lp_elem_bytes(b->precision) : 8;
  const int parts = lp ? yyg::lp_parts(b->precision) : 1;
  const int bk = lp ? yyg::lp_stage_k(b->precision) : 16;
  const long lds = 2L * parts * (bm + bn) * (bk + 16 / eb) * eb;
  int per_cu = (int)std::max(1L, std::min(4L, 160L * 1024 / std::max(1L, lds)));
  b->blocks[role] = std::max(1, std::min(b->n_items[role], b->cus * per_cu));
  // the per-problem tiles_m lives in the argument arrays
  if (lp) {
    std::vector<yyg::GemmLpArgs> h(b->h_lp[role], b->h_lp[role] + n);
    if (hipMemcpy(b->d_lp[role], h.data(), n * sizeof(yyg::GemmLpArgs), hipMemcpyHostToDevice) != hipSuccess)
      return YYG_ERR_DEVICE;
  } else {
    std::vector<yyg::GemmF64Args> h(b->h_f64[role], b->h_f64[role] + n);
    if (hipMemcpy(b->d_f64[role], h.data(), n * sizeof(yyg::GemmF64Args), hipMemcpyHostToDevice) != hipSuccess)
      return YYG_ERR_DEVICE;
  }
  return YYG_OK;
}

hipError_t batch_launch_gemm(yyg_batch *b, int role, hipStream_t s) {
  if (b->precision == YYG_FP64)
    return yyg::launch_gemm_f64_grouped(b->var[role], role, b->d_f64[role], b->d_items[role], b->n_items[role],
                                        b->blocks[role], s);
  return yyg::launch_gemm_lp_grouped(b->precision, b->var[role], role, b->d_lp[role], b->d_items[role],
                                     b->n_items[role], b->blocks[role], s);
}

// Write the current density / potential pointers into the pinned argument
// arrays (their device mirrors are refreshed by the graph's first nodes).
void batch_patch_pointers(yyg_batch *b) {
  const int n = (int)b->grids.size();
  for (int f = 0; f < n; ++f) {
    if (b->sep) {
      b->h_phi[0][f].A = b->rho[f];
      b->h_phi[1][f].C = b->phi[f];
    } else if (b->precision == YYG_FP64) {
      b->h_f64[0][f].A = b->rho[f];
      b->h_f64[1][f].C = b->phi[f];
    } else {
      b->h_split[0][f].X = b->rho[f];
      b->h_lp[1][f].C = b->phi[f];
    }
  }
}

hipError_t sep_batch_enqueue(yyg_batch *b, hipStream_t s, hipEvent_t *ev);

// Enqueue the whole batched solve on s (recorded into the graph).
hipError_t batch_enqueue(yyg_batch *b, hipStream_t s) {
  if (b->sep) return sep_batch_enqueue(b, s, nullptr);
  const int n = (int)b->grids.size();
  hipError_t e = hipSuccess;
  const bool lp = b->precision != YYG_FP64;
  if (!lp) {
    e = hipMemcpyAsync(b->d_f64[0], b->h_f64[0], n * sizeof(yyg::GemmF64Args), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->d_f64[1], b->h_f64[1], n * sizeof(yyg::GemmF64Args), hipMemcpyHostToDevice, s);
  } else {
    e = hipMemcpyAsync(b->d_split[0], b->h_split[0], n * sizeof(yyg::SplitArgs), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->d_lp[1], b->h_lp[1], n * sizeof(yyg::GemmLpArgs), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = yyg::launch_split_rows_grouped(b->precision, b->d_split[0], b->d_split_items[0], b->n_split_items[0],
                                         std::min(b->n_split_items[0], b->cus * 8), s);
  }
  if (e == hipSuccess) e = batch_launch_gemm(b, 0, s);
  if (e == hipSuccess)
    e = yyg::launch_radial_scan_grouped(b->d_scan, b->d_scan_items, b->n_scan_items,
                                        std::min(b->n_scan_items, b->cus * 2), s);
  if (e == hipSuccess && lp)
    e = yyg::launch_split_rows_grouped(b->precision, b->d_split[1], b->d_split_items[1], b->n_split_items[1],
                                       std::min(b->n_split_items[1], b->cus * 8), s);
  if (e == hipSuccess) e = batch_launch_gemm(b, 1, s);
  return e;
}

int batch_build(yyg_batch *b) {
  const int n = (int)b->grids.size();
  const bool lp = b->precision != YYG_FP64;
  const bool scaled = b->precision == YYG_FP16X2;
  b->rho.assign(n, nullptr);
  b->phi.assign(n, nullptr);
  b->part_gen.resize(n);
  for (int f = 0; f < n; ++f) b->part_gen[f] = b->grids[f]->part_gen;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) == hipSuccess && cus > 0)
    b->cus = cus;
  if (hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) return YYG_ERR_DEVICE;
  if (hipStreamCreate(&b->stream) != hipSuccess) return YYG_ERR_DEVICE;
  for (int r = 0; r < 2; ++r) {
    if (lp) {
      if (hipHostMalloc(reinterpret_cast<void **>(&b->h_lp[r]), n * sizeof(yyg::GemmLpArgs), 0) != hipSuccess ||
          hipHostMalloc(reinterpret_cast<void **>(&b->h_split[r]), n * sizeof(yyg::SplitArgs), 0) != hipSuccess ||
          dev_malloc(reinterpret_cast<void **>(&b->d_lp[r]), n * sizeof(yyg::GemmLpArgs)) != hipSuccess ||
          dev_malloc(reinterpret_cast<void **>(&b->d_split[r]), n * sizeof(yyg::SplitArgs)) != hipSuccess) {
        (void)hipGetLastError();
        return YYG_ERR_OUT_OF_MEMORY;
      }
    } else {
      if (hipHostMalloc(reinterpret_cast<void **>(&b->h_f64[r]), n * sizeof(yyg::GemmF64Args), 0) != hipSuccess ||
          dev_malloc(reinterpret_cast<void **>(&b->d_f64[r]), n * sizeof(yyg::GemmF64Args)) != hipSuccess) {
        (void)hipGetLastError();
        return YYG_ERR_OUT_OF_MEMORY;
      }
    }
  }
  std::vector<yyg::ScanArgs> scan(n);
  std::vector<int4> scan_items;
  std::vector<int2> split_items[2];
  for (int f = 0; f < n; ++f) {
    yyg_grid *g = b->grids[f];
    const int Q = g->Q;
    const long M = (long)g->n_patch * g->n_r;
    if (!lp) {
      yyg::GemmF64Args &a = b->h_f64[0][f];
      a = yyg::GemmF64Args{(int)M, Q, (int)g->nang, nullptr, g->nang, g->d_Bt, g->ldb, g->d_part, Q, 0,
                           (int)(((g->nang + 15) / 16) * 16), 1};
      yyg::GemmF64Args &c = b->h_f64[1][f];
      c = yyg::GemmF64Args{(int)M, (int)g->nang, g->n_patch * Q, g->d_U, g->ldy, g->d_Y, g->ldy, nullptr, g->nang, 0,
                           (int)(((g->n_patch * Q + 15) / 16) * 16), 1};
    } else {
      auto &L = g->lp[b->precision - 1];
      const int bk = yyg::lp_stage_k(b->precision);
      b->h_split[0][f] = yyg::SplitArgs{nullptr, g->nang, (int)g->nang, scaled ? g->d_eA : nullptr, L.Ar, L.lda,
                                        M * L.lda};
      b->h_split[1][f] = yyg::SplitArgs{g->d_U, g->ldy, g->n_patch * Q, scaled ? g->d_eU : nullptr, L.Ur, L.ldu, M * L.ldu};
      b->h_lp[0][f] = yyg::GemmLpArgs{(int)M, Q, (int)g->nang, L.Ar, L.lda, M * L.lda, scaled ? g->d_eA : nullptr,
                                      L.Bt, L.ldb, (long)Q * L.ldb, L.eBt, g->d_part, Q, 0,
                                      (int)((g->nang + bk - 1) / bk * bk), 1};
      b->h_lp[1][f] = yyg::GemmLpArgs{(int)M, (int)g->nang, g->n_patch * Q, L.Ur, L.ldu, M * L.ldu,
                                      scaled ? g->d_eU : nullptr, L.Y, L.ldy, (long)g->nang * L.ldy, L.eY, nullptr,
                                      g->nang, 0, (int)((g->n_patch * Q + bk - 1) / bk * bk), 1};
      for (long r = 0; r < M; ++r) {
        split_items[0].push_back(int2{f, (int)r});
        split_items[1].push_back(int2{f, (int)r});
      }
    }
    scan[f] = yyg::ScanArgs{g->d_part, 1, M * Q, g->d_Ahat, g->d_coef, g->d_qdeg, g->n_r, Q, g->L, -g->G, g->d_U,
                            g->ldy, g->n_patch == 2 ? 1 : 0};
    for (int p = 0; p < g->n_patch; ++p)
      for (int cb = 0; cb < (Q + 15) / 16; ++cb) scan_items.push_back(int4{f, cb, p, 0});
  }
  int st = upload(&b->d_scan, scan);
  if (st == YYG_OK) st = upload(&b->d_scan_items, scan_items);
  b->n_scan_items = (int)scan_items.size();
  if (lp) {
    for (int r = 0; r < 2 && st == YYG_OK; ++r) {
      st = upload(&b->d_split_items[r], split_items[r]);
      b->n_split_items[r] = (int)split_items[r].size();
      if (st == YYG_OK &&
          hipMemcpy(b->d_split[r], b->h_split[r], n * sizeof(yyg::SplitArgs), hipMemcpyHostToDevice) != hipSuccess)
        st = YYG_ERR_DEVICE;
    }
  }
  // default tile variant 64 x 64 (index 3 of the FP64 list, 0 of the others)
  for (int role = 0; role < 2 && st == YYG_OK; ++role) st = batch_set_items(b, role, lp ? 0 : 3);
  return st;
}

// Work items of separable phase r over every plan for batch tile t, the
// longest contractions first so that the persistent blocks finish together:
// (plan, tile row, tile column, z), z the strided-batch index (phi phases)
// or the problem of the phase (theta phases, rotation).
int sep_batch_set_items(yyg_batch *b, int r, int t) {
  int bm, bn, threads;
  yyg::sep_batch_tile(t, &bm, &bn, &threads);
  std::vector<std::pair<long, int4>> work;
  const int n = (int)b->grids.size();
  auto tiles = [&](long M, long N, long K, int f, int z) {
    const int tm = (int)((M + bm - 1) / bm), tn = (int)((N + bn - 1) / bn);
    for (int j = 0; j < tn; ++j)
      for (int i = 0; i < tm; ++i) work.push_back({K, int4{f, i, j, z}});
  };
  for (int f = 0; f < n; ++f) {
    const yyg_grid *g = b->grids[f];
    const long Mr = (long)g->n_patch * g->n_r;
    const int L = g->L, nmc = 2 * L + 1;
    if (r == 0 || r == 4) {
      const yyg::GemmF64Args &a = b->h_phi[r == 0 ? 0 : 1][f];
      for (int z = 0; z < a.batch; ++z) tiles(a.M, a.N, a.K, f, z);
    } else if (r == 1) {
      for (int z = 0; z < nmc; ++z) tiles(Mr, L + 1 - (z + 1) / 2, g->n_t, f, z);
    } else if (r == 2) {
      if (g->n_patch == 2)
        for (int z = 0; z < 2 * (L + 1); ++z) tiles(g->n_r, 2 * (L - z / 2) + 1, 2 * (L - z / 2) + 1, f, z);
    } else {
      for (int z = 0; z < nmc; ++z) tiles(g->n_t, Mr, L + 1 - (z + 1) / 2, f, z);
    }
  }
  std::stable_sort(work.begin(), work.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
  std::vector<int4> items(work.size());
  for (size_t i = 0; i < work.size(); ++i) items[i] = work[i].second;
  int st = upload(&b->d_sitems[r], items);
  if (st != YYG_OK) return st;
  b->n_sitems[r] = (int)items.size();
  b->svar[r] = t;
  // resident blocks: LDS-limited occupancy of the tile, four at most
  const long lds = 2L * (bm + bn) * 18 * 8;
  const int per_cu = (int)std::max(1L, std::min(4L, 160L * 1024 / lds));
  b->sblocks[r] = std::max(1, std::min(b->n_sitems[r], b->cus * per_cu));
  return YYG_OK;
}

int sep_batch_build(yyg_batch *b) {
  const int n = (int)b->grids.size();
  b->rho.assign(n, nullptr);
  b->phi.assign(n, nullptr);
  b->part_gen.resize(n);
  for (int f = 0; f < n; ++f) b->part_gen[f] = b->grids[f]->part_gen;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) == hipSuccess && cus > 0)
    b->cus = cus;
  if (hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) return YYG_ERR_DEVICE;
  if (hipStreamCreate(&b->stream) != hipSuccess) return YYG_ERR_DEVICE;
  // folded phi transforms when every plan is mirror-symmetric (one launch
  // mode for all plans)
  b->sep_fold = true;
  for (int f = 0; f < n; ++f) b->sep_fold = b->sep_fold && b->grids[f]->sep.fold;
  for (int r = 0; r < 2; ++r)
    if (hipHostMalloc(reinterpret_cast<void **>(&b->h_phi[r]), n * sizeof(yyg::GemmF64Args), 0) != hipSuccess ||
        dev_malloc(reinterpret_cast<void **>(&b->d_phi[r]), n * sizeof(yyg::GemmF64Args)) != hipSuccess) {
      (void)hipGetLastError();
      return YYG_ERR_OUT_OF_MEMORY;
    }
  std::vector<yyg::SepPhaseArgs> sargs(n);
  std::vector<yyg::ScanQArgs> qscan(n);
  std::vector<int2> qitems;
  for (int f = 0; f < n; ++f) {
    yyg_grid *g = b->grids[f];
    auto &S = g->sep;
    b->h_phi[0][f] = b->sep_fold ? S.phi_ana_f : S.phi_ana;
    b->h_phi[1][f] = b->sep_fold ? S.phi_syn_f : S.phi_syn;
    sargs[f] = S.args;
    const int chunk = ((g->n_r + 63) / 64) | 1;
    qscan[f] = yyg::ScanQArgs{g->n_patch == 2 ? S.At : g->d_Ahat, S.coefS, g->d_qdeg, g->n_r, g->L, chunk,
                              g->n_patch, -g->G, S.Ut};
    b->max_nr = std::max(b->max_nr, g->n_r);
    for (int q = 0; q < g->Q; ++q) qitems.push_back(int2{f, q});
  }
  int st = upload(&b->d_sargs, sargs);
  if (st == YYG_OK) st = upload(&b->d_qscan, qscan);
  if (st == YYG_OK) st = upload(&b->d_qitems, qitems);
  b->n_qitems = (int)qitems.size();
  // default tiles: 64 x 80 for the phi analysis, 128 x 48 for the phi
  // synthesis, 32 x 32 for the theta phases and the rotation
  const int def[5] = {3, 0, 0, 0, 4};
  for (int r = 0; r < 5 && st == YYG_OK; ++r) st = sep_batch_set_items(b, r, def[r]);
  return st;
}

// The batched separable solve on s; with ev (6 events) recorded before
// the argument copies and after each of the six launches.
hipError_t sep_batch_enqueue(yyg_batch *b, hipStream_t s, hipEvent_t *ev) {
  const int n = (int)b->grids.size();
  hipError_t e = hipSuccess;
  auto mark = [&](int i) {
    if (ev && e == hipSuccess) e = hipEventRecord(ev[i], s);
  };
  mark(0);
  e = hipMemcpyAsync(b->d_phi[0], b->h_phi[0], n * sizeof(yyg::GemmF64Args), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_phi[1], b->h_phi[1], n * sizeof(yyg::GemmF64Args), hipMemcpyHostToDevice, s);
  auto phase = [&](int r) {
    if (e == hipSuccess)
      e = yyg::launch_sep_batch_phase(b->svar[r], r, b->sep_fold, b->d_phi[r == 0 ? 0 : 1], b->d_sargs, b->d_sitems[r],
                                      b->n_sitems[r], b->sblocks[r], s);
  };
  phase(0);
  mark(1);
  phase(1);
  phase(2);
  mark(2);
  if (e == hipSuccess)
    e = yyg::launch_radial_scan_q_grouped(b->d_qscan, b->d_qitems, b->n_qitems, std::min(b->n_qitems, b->cus * 4),
                                          b->max_nr, s);
  mark(3);
  phase(3);
  mark(4);
  phase(4);
  mark(5);
  return e;
}

}  // namespace

extern "C" {

int yyg_grid_create(const yyg_grid_desc *d, int device, yyg_grid **out) {
  if (!out) return YYG_ERR_INVALID_ARG;
  *out = nullptr;
  int st = yyg::validate_desc(d);
  if (st != YYG_OK) return st;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return YYG_ERR_DEVICE;
  }
  if (device < 0 || device >= ndev) return YYG_ERR_INVALID_ARG;

  yyg_grid *g = new (std::nothrow) yyg_grid;
  if (!g) return YYG_ERR_OUT_OF_MEMORY;
  g->device = device;
  g->kind = d->kind;
  g->n_patch = d->kind == YYG_GRID_POLAR ? 1 : 2;
  g->n_r = d->n_r;
  g->n_t = d->n_theta;
  g->n_p = d->n_phi;
  g->L = d->lmax;
  g->Q = (d->lmax + 1) * (d->lmax + 1);
  g->G = d->G;
  g->nang = (long)g->n_t * g->n_p;
  g->ldb = round_up(g->nang, 16);
  g->ldy = round_up((long)g->n_patch * g->Q, 16);
  g->r_edges.assign(d->r_edges, d->r_edges + d->n_r + 1);
  g->geom = d->kind == YYG_GRID_POLAR ? yyg::make_polar_patch(g->n_t, g->n_p)
                                      : yyg::make_patch(g->n_t, g->n_p, d->delta_theta, d->delta_phi);
  const int L = g->L, Q = g->Q, n_r = g->n_r;
  const long M = (long)g->n_patch * n_r;
  {
    int bm, bn;
    yyg::gemm_f64_variant_tile(g->var_ana, &bm, &bn);
    g->nsplit = yyg::choose_split(((M + bm - 1) / bm) * ((Q + bn - 1) / bn), g->nang);
    g->part_cap = g->nsplit;
  }

  std::vector<double> Tt, CS, coef, P, Tr, Yx;
  std::vector<int> qdeg(Q);
  try {
    g->w_host.resize(g->nang);
    yyg::overlap_weights(g->geom, g->w_host.data());
    Tt.resize((size_t)g->n_t * Q);
    yyg::theta_table_normalised(g->geom, L, Tt.data());
    CS.resize((size_t)g->n_p * Q);
    yyg::phi_table(g->geom, L, CS.data());
    coef.resize((size_t)4 * n_r * (L + 1));
    yyg::radial_coefficients(n_r, g->r_edges.data(), L, coef.data());
    P.resize((size_t)g->n_t * Q);
    yyg::self_legendre_table(g->geom, L, P.data());
    Tr.resize((size_t)g->n_p * Q);
    yyg::self_trig_table(g->geom, L, Tr.data());
    if (g->n_patch == 2) {
      Yx.resize((size_t)g->nang * Q);
      yyg::cross_basis(g->geom, L, Yx.data());
    }
    auto cols = yyg::column_table(L);
    auto s = yyg::norm_sqrt(L);
    g->nrm_q.resize(Q);
    for (int q = 0; q < Q; ++q) {
      qdeg[q] = cols[q].l;
      g->nrm_q[q] = s[cols[q].l * (L + 1) + cols[q].m];
    }
  } catch (const std::bad_alloc &) {
    free_grid(g);
    return YYG_ERR_OUT_OF_MEMORY;
  }

  DeviceGuard dg(device);
  if (!dg.ok) {
    free_grid(g);
    return YYG_ERR_DEVICE;
  }
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
      g->cus = cus;
  }
  double *d_w = nullptr, *d_Tt = nullptr, *d_CS = nullptr, *d_P = nullptr, *d_Tr = nullptr;
  auto cleanup_tmp = [&] {
    double *t[] = {d_w, d_Tt, d_CS, d_P, d_Tr};
    for (double *b : t)
      if (b) (void)dev_free(b);
  };
  st = YYG_OK;
  if (st == YYG_OK) st = dmalloc(&g->d_Bt, (size_t)Q * g->ldb);
  if (st == YYG_OK) st = dmalloc(&g->d_Y, (size_t)g->nang * g->ldy);
  if (st == YYG_OK) st = dmalloc(&g->d_coef, coef.size());
  if (st == YYG_OK) st = dmalloc(&g->d_qdeg, (size_t)Q);
  if (st == YYG_OK) st = dmalloc(&g->d_part, (size_t)g->nsplit * M * Q);
  if (st == YYG_OK) st = dmalloc(&g->d_Ahat, (size_t)M * Q);
  if (st == YYG_OK) st = dmalloc(&g->d_U, (size_t)M * g->ldy);
  if (st == YYG_OK) st = dmalloc(&d_w, (size_t)g->nang);
  if (st == YYG_OK) st = dmalloc(&d_Tt, Tt.size());
  if (st == YYG_OK) st = dmalloc(&d_CS, CS.size());
  if (st == YYG_OK) st = dmalloc(&d_P, P.size());
  if (st == YYG_OK) st = dmalloc(&d_Tr, Tr.size());
  if (st != YYG_OK) {
    cleanup_tmp();
    free_grid(g);
    return st;
  }
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t r) {
    if (e == hipSuccess && r != hipSuccess) e = r;
  };
  chk(hipMemcpy(g->d_coef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice));
  chk(hipMemcpy(g->d_qdeg, qdeg.data(), qdeg.size() * sizeof(int), hipMemcpyHostToDevice));
  chk(hipMemcpy(d_w, g->w_host.data(), g->nang * sizeof(double), hipMemcpyHostToDevice));
  chk(hipMemcpy(d_Tt, Tt.data(), Tt.size() * sizeof(double), hipMemcpyHostToDevice));
  chk(hipMemcpy(d_CS, CS.data(), CS.size() * sizeof(double), hipMemcpyHostToDevice));
  chk(hipMemcpy(d_P, P.data(), P.size() * sizeof(double), hipMemcpyHostToDevice));
  chk(hipMemcpy(d_Tr, Tr.data(), Tr.size() * sizeof(double), hipMemcpyHostToDevice));
  chk(hipMemset(g->d_U, 0, (size_t)M * g->ldy * sizeof(double)));
  chk(hipMemset(g->d_Ahat, 0, (size_t)M * Q * sizeof(double)));
  if (e == hipSuccess) chk(yyg::launch_expand_analysis_basis(d_w, d_Tt, d_CS, g->n_t, g->n_p, Q, g->d_Bt, g->ldb, 0));
  if (e == hipSuccess) chk(yyg::launch_expand_self_basis(d_P, d_Tr, g->n_t, g->n_p, Q, g->d_Y, g->ldy, g->n_patch * Q, 0));
  // cross part: columns [Q, 2Q) of every row
  if (e == hipSuccess && g->n_patch == 2)
    chk(hipMemcpy2D(g->d_Y + Q, g->ldy * sizeof(double), Yx.data(), (size_t)Q * sizeof(double),
                    (size_t)Q * sizeof(double), g->nang, hipMemcpyHostToDevice));
  chk(hipDeviceSynchronize());
  cleanup_tmp();
  if (e != hipSuccess) {
    (void)hipGetLastError();
    free_grid(g);
    return YYG_ERR_DEVICE;
  }
  *out = g;
  return YYG_OK;
}

int yyg_grid_create_res(int n_r, const double *r_edges, double res_deg, int lmax, double G, int device,
                        yyg_grid **out) {
  if (!(res_deg > 0.0) || !std::isfinite(res_deg) || res_deg > 90.0) return YYG_ERR_INVALID_ARG;
  yyg_grid_desc d;
  std::memset(&d, 0, sizeof(d));
  d.kind = YYG_GRID_YINYANG;
  d.n_r = n_r;
  d.r_edges = r_edges;
  yyg::dims_from_resolution(res_deg, &d.n_theta, &d.n_phi, &d.delta_theta, &d.delta_phi);
  d.lmax = lmax;
  d.G = G;
  return yyg_grid_create(&d, device, out);
}

int yyg_grid_dims(const yyg_grid *g, int *n_r, int *n_theta, int *n_phi, int *Q) {
  if (!g) return YYG_ERR_INVALID_ARG;
  if (n_r) *n_r = g->n_r;
  if (n_theta) *n_theta = g->n_t;
  if (n_phi) *n_phi = g->n_p;
  if (Q) *Q = g->Q;
  return YYG_OK;
}

int yyg_grid_kind(const yyg_grid *g, int *kind, int *patches) {
  if (!g) return YYG_ERR_INVALID_ARG;
  if (kind) *kind = g->kind;
  if (patches) *patches = g->n_patch;
  return YYG_OK;
}

int yyg_prepare(yyg_grid *g, int precision) {
  if (!g) return YYG_ERR_INVALID_ARG;
  if (precision == YYG_FP64) return YYG_OK;
  if (precision < 0 || precision > YYG_FP16X2) return YYG_ERR_INVALID_ARG;
  auto &L = g->lp[precision - 1];
  if (L.ready) return YYG_OK;
  DeviceGuard dg(g->device);
  if (!dg.ok) return YYG_ERR_DEVICE;
  const int Q = g->Q;
  const long M = (long)g->n_patch * g->n_r;
  const int parts = yyg::lp_parts(precision), eb = yyg::lp_elem_bytes(precision), bk = yyg::lp_stage_k(precision);
  L.ldb = round_up(g->nang, std::max(bk, 16));
  L.ldy = round_up((long)g->n_patch * Q, std::max(bk, 16));
  L.lda = L.ldb;
  L.ldu = L.ldy;
  const size_t bt_plane = (size_t)Q * L.ldb, y_plane = (size_t)g->nang * L.ldy;
  int st = YYG_OK;
  auto bmalloc = [&](void **ptr, size_t bytes) {
    if (st != YYG_OK) return;
    if (dev_malloc(ptr, bytes) != hipSuccess) {
      *ptr = nullptr;
      (void)hipGetLastError();
      st = YYG_ERR_OUT_OF_MEMORY;
    }
  };
  bmalloc(&L.Bt, bt_plane * parts * eb);
  bmalloc(reinterpret_cast<void **>(&L.eBt), (size_t)Q * sizeof(int));
  bmalloc(&L.Y, y_plane * parts * eb);
  bmalloc(reinterpret_cast<void **>(&L.eY), (size_t)g->nang * sizeof(int));
  bmalloc(&L.Ar, (size_t)M * L.lda * parts * eb);
  bmalloc(&L.Ur, (size_t)M * L.ldu * parts * eb);
  if (!g->d_eA) bmalloc(reinterpret_cast<void **>(&g->d_eA), (size_t)M * sizeof(int));
  if (!g->d_eU) bmalloc(reinterpret_cast<void **>(&g->d_eU), (size_t)M * sizeof(int));
  if (st != YYG_OK) {
    lp_release(L);
    return st;
  }
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t r) {
    if (e == hipSuccess && r != hipSuccess) e = r;
  };
  chk(yyg::launch_row_exponent(g->d_Bt, g->ldb, Q, (int)g->nang, L.eBt, 0));
  chk(yyg::launch_split_rows(precision, g->d_Bt, g->ldb, Q, (int)g->nang, L.eBt, L.Bt, L.ldb, (long)bt_plane, 0));
  chk(yyg::launch_row_exponent(g->d_Y, g->ldy, (int)g->nang, g->n_patch * Q, L.eY, 0));
  chk(yyg::launch_split_rows(precision, g->d_Y, g->ldy, (int)g->nang, g->n_patch * Q, L.eY, L.Y, L.ldy, (long)y_plane, 0));
  chk(hipDeviceSynchronize());
  if (e != hipSuccess) {
    (void)hipGetLastError();
    lp_release(L);
    return YYG_ERR_DEVICE;
  }
  int bm, bn;
  yyg::gemm_lp_variant_tile(0, &bm, &bn);
  L.var_ana = 0;
  L.var_syn = 0;
  L.nsplit = yyg::choose_split(((M + bm - 1) / bm) * ((Q + bn - 1) / bn), g->nang);
  if (L.nsplit > g->part_cap) {
    double *np = nullptr;
    if (dmalloc(&np, (size_t)L.nsplit * M * Q) != YYG_OK) {
      lp_release(L);
      return YYG_ERR_OUT_OF_MEMORY;
    }
    (void)dev_free(g->d_part);
    g->d_part = np;
    g->part_gen += 1;
    g->part_cap = L.nsplit;
  }
  L.ready = true;
  return YYG_OK;
}

int yyg_upload_rho(yyg_grid *g, const double *rho, int rho_is_device, void *stream) {
  if (!g || !rho) return YYG_ERR_INVALID_ARG;
  if (rho_is_device) {
    g->rho = rho;
    return YYG_OK;
  }
  DeviceGuard dg(g->device);
  if (!dg.ok) return YYG_ERR_DEVICE;
  const size_t bytes = (size_t)g->n_patch * g->n_r * g->nang * sizeof(double);
  if (!g->d_rho_owned) {
    int st = dmalloc(&g->d_rho_owned, bytes / sizeof(double));
    if (st != YYG_OK) return st;
  }
  if (hipMemcpyAsync(g->d_rho_owned, rho, bytes, hipMemcpyHostToDevice, as_stream(stream)) != hipSuccess) {
    (void)hipGetLastError();
    return YYG_ERR_DEVICE;
  }
  g->rho = g->d_rho_owned;
  return YYG_OK;
}

int yyg_solve(yyg_grid *g, double *phi, int phi_is_device, int precision, void *stream) {
  if (!g || !phi) return YYG_ERR_INVALID_ARG;
  if (precision < 0 || precision > YYG_FP16X2) return YYG_ERR_INVALID_ARG;
  const bool sep_form = g->method == YYG_METHOD_SEPARABLE;
  // the separable form converts its operands in the kernels (nothing to
  // prepare); FP16's exponent range would need row scaling it does not do
  if (sep_form && precision == YYG_FP16X2) return YYG_ERR_UNSUPPORTED;
  if (!sep_form && precision != YYG_FP64 && !g->lp[precision - 1].ready) return YYG_ERR_NOT_READY;
  if (!g->rho) return YYG_ERR_NOT_READY;
  DeviceGuard dg(g->device);
  if (!dg.ok) return YYG_ERR_DEVICE;
  hipStream_t s = as_stream(stream);
  if (int st = check_rho(g, g->rho, s); st != YYG_OK) return st;
  const int Q = g->Q, n_r = g->n_r;
  const long M = (long)g->n_patch * n_r;
  double *out = phi;
  double *tmp = nullptr;
  if (!phi_is_device) {
    if (dmalloc(&tmp, (size_t)M * g->nang) != YYG_OK) return YYG_ERR_OUT_OF_MEMORY;
    out = tmp;
  }
  hipError_t e = hipSuccess;
  int t;
  const bool lp = precision != YYG_FP64;
  const bool scaled = precision == YYG_FP16X2;
  if (g->method == YYG_METHOD_SEPARABLE) {
    int st = sep_set_pointers(g, g->rho, out, s);
    if (st != YYG_OK) {
      if (tmp) (void)dev_free(tmp);
      return st;
    }
    e = sep_solve(g, s, precision);
    if (!phi_is_device) {
      if (e == hipSuccess)
        e = hipMemcpyAsync(phi, out, (size_t)M * g->nang * sizeof(double), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      (void)dev_free(tmp);
      g->sep.phi_syn.C = nullptr;  // the temporary is gone
      g->sep.phi_syn_d.C = nullptr;
      g->sep.phi_syn_f.C = nullptr;
      g->sep.phi_syn_s.phi = nullptr;
      g->sep.phi_syn_fd.C = nullptr;
      g->sep.phi_syn_l.C = nullptr;
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return YYG_ERR_DEVICE;
    }
    return YYG_OK;
  }
  g->ahat_cols = false;
  const int nsplit = lp ? g->lp[precision - 1].nsplit : g->nsplit;
  if (lp) {
    // split the density into operand planes (rows scaled for FP16)
    const auto &L = g->lp[precision - 1];
    t = timing_begin(g, 3, s);
    if (scaled) e = yyg::launch_row_exponent(g->rho, g->nang, (int)M, (int)g->nang, g->d_eA, s);
    if (e == hipSuccess)
      e = yyg::launch_split_rows(precision, g->rho, g->nang, (int)M, (int)g->nang, scaled ? g->d_eA : nullptr, L.Ar,
                                 L.lda, M * L.lda, s);
    timing_end(g, t, s);
  }
  if (e == hipSuccess) {
    t = timing_begin(g, 0, s);
    if (!lp) {
      e = yyg::launch_gemm_nt_f64(g->var_ana, 0, (int)M, Q, (int)g->nang, g->rho, g->nang, g->d_Bt, g->ldb,
                                  g->d_part, Q, nsplit, M * Q, s);
    } else {
      const auto &L = g->lp[precision - 1];
      e = yyg::launch_gemm_nt_lp(precision, L.var_ana, 0, (int)M, Q, (int)g->nang, L.Ar, L.lda, M * L.lda,
                                 scaled ? g->d_eA : nullptr, L.Bt, L.ldb, (long)Q * L.ldb, L.eBt, g->d_part, Q,
                                 nsplit, M * Q, s);
    }
    timing_end(g, t, s);
  }
  if (e == hipSuccess) {
    t = timing_begin(g, 1, s);
    e = yyg::launch_radial_scan(g->d_part, nsplit, M * Q, g->d_Ahat, g->d_coef, g->d_qdeg, n_r, Q, g->L, -g->G,
                                g->d_U, g->ldy, g->n_patch, s);
    timing_end(g, t, s);
  }
  if (e == hipSuccess && lp) {
    const auto &L = g->lp[precision - 1];
    t = timing_begin(g, 3, s);
    if (scaled) e = yyg::launch_row_exponent(g->d_U, g->ldy, (int)M, g->n_patch * Q, g->d_eU, s);
    if (e == hipSuccess)
      e = yyg::launch_split_rows(precision, g->d_U, g->ldy, (int)M, g->n_patch * Q, scaled ? g->d_eU : nullptr, L.Ur, L.ldu,
                                 M * L.ldu, s);
    timing_end(g, t, s);
  }
  if (e == hipSuccess) {
    t = timing_begin(g, 2, s);
    if (!lp) {
      e = yyg::launch_gemm_nt_f64(g->var_syn, 1, (int)M, (int)g->nang, g->n_patch * Q, g->d_U, g->ldy, g->d_Y, g->ldy, out,
                                  g->nang, 1, 0, s);
    } else {
      const auto &L = g->lp[precision - 1];
      e = yyg::launch_gemm_nt_lp(precision, L.var_syn, 1, (int)M, (int)g->nang, g->n_patch * Q, L.Ur, L.ldu, M * L.ldu,
                                 scaled ? g->d_eU : nullptr, L.Y, L.ldy, (long)g->nang * L.ldy, L.eY, out, g->nang,
                                 1, 0, s);
    }
    timing_end(g, t, s);
  }
  if (!phi_is_device) {
    if (e == hipSuccess)
      e = hipMemcpyAsync(phi, out, (size_t)M * g->nang * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)dev_free(tmp);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return YYG_ERR_DEVICE;
  }
  return YYG_OK;
}

int yyg_solve_noalloc(yyg_grid *g, const double *rho, double *phi, void *stream) {
  if (!g || !rho || !phi) return YYG_ERR_INVALID_ARG;
  if (g->method != YYG_METHOD_SEPARABLE || !g->sep.ready) return YYG_ERR_NOT_READY;
  DeviceGuard dg(g->device);
  if (!dg.ok) return YYG_ERR_DEVICE;
  double *base = nullptr;
  size_t bytes = 0;
  if (yyg::scratch_region(g->device, &base, &bytes) != hipSuccess) {
    (void)hipGetLastError();
    return YYG_ERR_DEVICE;
  }
  if (sep_work_doubles(g) * sizeof(double) > bytes) return YYG_ERR_UNSUPPORTED;
  if (int st = check_rho(g, rho, as_stream(stream)); st != YYG_OK) return st;
  // carve the work buffers out of the scratch array; every one of them is
  // written in full by its phase before any later phase reads it, so none
  // needs clearing
  const long M = (long)g->n_patch * g->n_r, nmc = 2L * g->L + 1;
  auto r32 = [](long v) { return (v + 31) / 32 * 32; };
  SepWork w{};
  double *p = base;
  w.X2 = p, p += r32(nmc * g->n_t * M);
  w.V = p, p += r32(nmc * g->n_t * M);
  w.Ut = p, p += r32(nmc * (g->L + 1) * M);
  w.At = g->n_patch == 2 ? p : nullptr, p += g->n_patch == 2 ? r32(M * g->Q) : 0;
  w.Ahat = p;
  const SepWork own = sep_work(g);
  const bool timing = g->timing, cols = g->ahat_cols;
  g->timing = false;  // no events: nothing is created
  sep_bind_work(g, w);
  hipStream_t s = as_stream(stream);
  hipError_t e = hipSuccess;
  if (sep_set_pointers(g, rho, phi, s) != YYG_OK) e = hipErrorInvalidValue;
  if (e == hipSuccess) e = sep_solve(g, s);
  sep_bind_work(g, own);
  g->timing = timing;
  g->ahat_cols = cols;  // the plan's moments buffer still holds the last yyg_solve's
  sep_set_pointers(g, nullptr, nullptr, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return YYG_ERR_DEVICE;
  }
  return YYG_OK;
}

int yyg_set_check_finite(yyg_grid *g, int on) {
  if (!g) return YYG_ERR_INVALID_ARG;
  if (on && !g->d_flag) {
    DeviceGuard dg(g->device);
    if (!dg.ok) return YYG_ERR_DEVICE;
    if (int st = dmalloc(&g->d_flag, 1); st != YYG_OK) return st;
  }
  g->check_finite = on != 0;
  return YYG_OK;
}

int yyg_device_bytes(size_t *held) {
  if (!held) return YYG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_mem_mu);
  *held = g_mem_held;
  return YYG_OK;
}

int yyg_get_moments(yyg_grid *g, double *A_host) {
  if (!g || !A_host) return YYG_ERR_INVALID_ARG;
  DeviceGuard dg(g->device);
  if (!dg.ok) return YYG_ERR_DEVICE;
  const long M = (long)g->n_patch * g->n_r;
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(A_host, g->d_Ahat, (size_t)M * g->Q * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
    (void)hipGetLastError();
    return YYG_ERR_DEVICE;
  }
  if (g->ahat_cols) {
    std::vector<double> t(A_host, A_host + M * g->Q);
    for (long r = 0; r < M; ++r)
      for (int q = 0; q < g->Q; ++q) A_host[r * g->Q + q] = t[q * M + r];
  }
  for (long r = 0; r < M; ++r)
    for (int q = 0; q < g->Q; ++q) A_host[r * g->Q + q] /= g->nrm_q[q];
  return YYG_OK;
}

int yyg_get_weights(const yyg_grid *g, double *w_host) {
  if (!g || !w_host) return YYG_ERR_INVALID_ARG;
  std::memcpy(w_host, g->w_host.data(), g->w_host.size() * sizeof(double));
  return YYG_OK;
}

int yyg_grid_destroy(yyg_grid *g) {
  if (!g) return YYG_ERR_INVALID_ARG;
  DeviceGuard dg(g->device);
  (void)hipDeviceSynchronize();
  free_grid(g);
  return YYG_OK;
}

int yyg_set_timing(yyg_grid *g, int enable) {
  if (!g) return YYG_ERR_INVALID_ARG;
  DeviceGuard dg(g->device);
  (void)hipDeviceSynchronize();
  for (auto &t : g->launches) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  g->launches.clear();
  g->timing = enable != 0;
  return YYG_OK;
}

int yyg_get_timing(yyg_grid *g, double *ms, long *counts, int n_slots) {
  if (!g || !ms || !counts || n_slots < 1 || n_slots > kSlots) return YYG_ERR_INVALID_ARG;
  DeviceGuard dg(g->device);
  for (int i = 0; i < n_slots; ++i) {
    ms[i] = 0.0;
    counts[i] = 0;
  }
  for (auto &t : g->launches) {
    if (hipEventSynchronize(t.stop) != hipSuccess) {
      (void)hipGetLastError();
      return YYG_ERR_DEVICE;
    }
    float v = 0.f;
    if (hipEventElapsedTime(&v, t.start, t.stop) != hipSuccess) {
      (void)hipGetLastError();
      return YYG_ERR_DEVICE;
    }
    if (t.slot < n_slots) {
      ms[t.slot] += v;
      counts[t.slot] += 1;
    }
  }
  return YYG_OK;
}

int yyg_set_method(yyg_grid *g, int method) {
  if (!g || (method != YYG_METHOD_DENSE && method != YYG_METHOD_SEPARABLE)) return YYG_ERR_INVALID_ARG;
  if (method == YYG_METHOD_SEPARABLE && !g->sep.ready) {
    DeviceGuard dg(g->device);
    if (!dg.ok) return YYG_ERR_DEVICE;
    if (hipDeviceSynchronize() != hipSuccess) {
      (void)hipGetLastError();
      return YYG_ERR_DEVICE;
    }
    int st = sep_build(g);
    if (st != YYG_OK) return st;
  }
  g->method = method;
  return YYG_OK;
}

int yyg_autotune(yyg_grid *g, int precision, void *stream) {
  if (!g) return YYG_ERR_INVALID_ARG;
  if (precision < 0 || precision > YYG_FP16X2) return YYG_ERR_INVALID_ARG;
  const bool lp = precision != YYG_FP64;
  const bool sep_form = g->method == YYG_METHOD_SEPARABLE;
  if (sep_form && precision == YYG_FP16X2) return YYG_ERR_UNSUPPORTED;
  if (lp && !sep_form && !g->lp[precision - 1].ready) return YYG_ERR_NOT_READY;
  DeviceGuard dg(g->device);
  if (!dg.ok) return YYG_ERR_DEVICE;
  hipStream_t s = as_stream(stream);
  if (lp && sep_form) {
    // the reduced-precision phi transforms of the separable form: each
    // tile shape timed inside whole solves, phi analysis then synthesis
    if (!g->sep.ready) return YYG_ERR_NOT_READY;
    const long Mt = (long)g->n_patch * g->n_r;
    double *phi_t = nullptr, *rho_t = nullptr;
    int st = dmalloc(&phi_t, (size_t)Mt * g->nang);
    if (st == YYG_OK && !g->rho) {
      st = dmalloc(&rho_t, (size_t)Mt * g->nang);
      if (st == YYG_OK) (void)hipMemsetAsync(rho_t, 0, (size_t)Mt * g->nang * sizeof(double), s);
    }
    if (st == YYG_OK) st = sep_set_pointers(g, g->rho ? g->rho : rho_t, phi_t, s);
    const bool timing = g->timing;
    g->timing = false;
    auto solve_ms = [&]() { return time_launch([&] { return sep_solve(g, s, precision); }, s, 5); };
    for (int r = 0; r < 2 && st == YYG_OK; ++r) {
      int &cur = g->sep.lpt[precision - 1][r];
      int best = cur;
      double bt = solve_ms() - 1e-4;
      const int t0 = cur;
      for (int t = 0; t < sep_lp_choices(g, precision, r); ++t) {
        if (t == t0 || !sep_lp_available(g, precision, r, t)) continue;
        cur = t;
        const double tm = solve_ms();
        if (tm < bt) {
          bt = tm;
          best = t;
        }
      }
      cur = best;
    }
    g->timing = timing;
    (void)hipStreamSynchronize(s);
    if (phi_t) (void)dev_free(phi_t);
    if (rho_t) (void)dev_free(rho_t);
    sep_set_pointers(g, nullptr, nullptr, s);
    return st;
  }
  const int Q = g->Q;
  const long M = (long)g->n_patch * g->n_r;
  int *cur_va = lp ? &g->lp[precision - 1].var_ana : &g->var_ana;
  int *cur_sp = lp ? &g->lp[precision - 1].nsplit : &g->nsplit;
  int *cur_vs = lp ? &g->lp[precision - 1].var_syn : &g->var_syn;
  const int nv = lp ? yyg::gemm_lp_variant_count() : yyg::gemm_f64_variant_count();
  auto tile = [&](int v, int *bm, int *bn) {
    if (lp)
      yyg::gemm_lp_variant_tile(v, bm, bn);
    else
      yyg::gemm_f64_variant_tile(v, bm, bn);
  };
  const char *cache_path = std::getenv("YYG_TUNE_CACHE");
  auto cache = read_tune_cache(cache_path);
  const std::string ka = tune_key(precision, 0, M, Q, g->nang), ks = tune_key(precision, 1, M, g->nang, (long)g->n_patch * Q);
  int best_va = *cur_va, best_sp = *cur_sp, best_vs = *cur_vs;
  // a plan in the separable form tunes that form's phases only (FP64): the
  // dense contractions keep their configuration
  const bool sep_only = !lp && sep_form;
  bool have_a = sep_only, have_s = sep_only;
  if (!sep_only && cache.count(ka)) {
    best_va = cache[ka].first;
    best_sp = cache[ka].second;
    have_a = best_va >= 0 && best_va < nv && best_sp >= 1 && best_sp <= 32;
  }
  if (!sep_only && cache.count(ks)) {
    best_vs = cache[ks].first;
    have_s = best_vs >= 0 && best_vs < nv;
  }
  double *tmp_in = nullptr, *tmp_out = nullptr, *tmp_part = nullptr;
  const int smax = 32;
  int st = YYG_OK;
  if (!have_a || !have_s) {
    if (!g->rho) st = dmalloc(&tmp_in, (size_t)M * g->nang);
    if (st == YYG_OK) st = dmalloc(&tmp_out, (size_t)M * g->nang);
    if (st == YYG_OK) st = dmalloc(&tmp_part, (size_t)smax * M * Q);
    if (st == YYG_OK && tmp_in) (void)hipMemsetAsync(tmp_in, 0, (size_t)M * g->nang * sizeof(double), s);
    if (st != YYG_OK) {
      if (tmp_in) (void)dev_free(tmp_in);
      if (tmp_out) (void)dev_free(tmp_out);
      if (tmp_part) (void)dev_free(tmp_part);
      return st;
    }
  }
  const double *rho = g->rho ? g->rho : tmp_in;
  const bool scaled = precision == YYG_FP16X2;
  if (lp && (!have_a || !have_s)) {
    const auto &L = g->lp[precision - 1];
    if (scaled) {
      (void)yyg::launch_row_exponent(rho, g->nang, (int)M, (int)g->nang, g->d_eA, s);
      (void)yyg::launch_row_exponent(g->d_U, g->ldy, (int)M, g->n_patch * Q, g->d_eU, s);
    }
    (void)yyg::launch_split_rows(precision, rho, g->nang, (int)M, (int)g->nang, scaled ? g->d_eA : nullptr, L.Ar,
                                 L.lda, M * L.lda, s);
    (void)yyg::launch_split_rows(precision, g->d_U, g->ldy, (int)M, g->n_patch * Q, scaled ? g->d_eU : nullptr, L.Ur, L.ldu,
                                 M * L.ldu, s);
  }
  auto ana = [&](int v, int sp) -> hipError_t {
    if (!lp)
      return yyg::launch_gemm_nt_f64(v, 0, (int)M, Q, (int)g->nang, rho, g->nang, g->d_Bt, g->ldb, tmp_part, Q, sp,
                                     M * Q, s);
    const auto &L = g->lp[precision - 1];
    return yyg::launch_gemm_nt_lp(precision, v, 0, (int)M, Q, (int)g->nang, L.Ar, L.lda, M * L.lda,
                                  scaled ? g->d_eA : nullptr, L.Bt, L.ldb, (long)Q * L.ldb, L.eBt, tmp_part, Q, sp,
                                  M * Q, s);
  };
  auto syn = [&](int v) -> hipError_t {
    if (!lp)
      return yyg::launch_gemm_nt_f64(v, 1, (int)M, (int)g->nang, g->n_patch * Q, g->d_U, g->ldy, g->d_Y, g->ldy, tmp_out,
                                     g->nang, 1, 0, s);
    const auto &L = g->lp[precision - 1];
    return yyg::launch_gemm_nt_lp(precision, v, 1, (int)M, (int)g->nang, g->n_patch * Q, L.Ur, L.ldu, M * L.ldu,
                                  scaled ? g->d_eU : nullptr, L.Y, L.ldy, (long)g->nang * L.ldy, L.eY, tmp_out,
                                  g->nang, 1, 0, s);
  };
  if (!have_a) {
    double best = 1e30;
    for (int v = 0; v < nv; ++v) {
      int bm, bn;
      tile(v, &bm, &bn);
      long tiles = ((M + bm - 1) / bm) * ((Q + bn - 1) / bn);
      int base = yyg::choose_split(tiles, g->nang);
      int cands[] = {1, 2, 4, 8, 16, 32, base};
      for (int sp : cands) {
        if (sp > smax || (long)sp * 64 > g->nang + 64) continue;
        double t = time_launch([&] { return ana(v, sp); }, s, 3);
        // the scan reads every partial once more: charge it at HBM speed
        t += (double)sp * M * Q * 8.0 / 5.0e9;
        if (t < best) {
          best = t;
          best_va = v;
          best_sp = sp;
        }
      }
    }
  }
  if (!have_s) {
    double best = 1e30;
    for (int v = 0; v < nv; ++v) {
      double t = time_launch([&] { return syn(v); }, s, 3);
      if (t < best) {
        best = t;
        best_vs = v;
      }
    }
  }
  if (tmp_in) (void)dev_free(tmp_in);
  if (tmp_out) (void)dev_free(tmp_out);
  if (tmp_part) (void)dev_free(tmp_part);
  if (best_sp > g->part_cap) {
    double *np = nullptr;
    if (dmalloc(&np, (size_t)best_sp * M * Q) != YYG_OK) return YYG_ERR_OUT_OF_MEMORY;
    (void)hipDeviceSynchronize();
    (void)dev_free(g->d_part);
    g->d_part = np;
    g->part_gen += 1;
    g->part_cap = best_sp;
  }
  *cur_va = best_va;
  *cur_sp = best_sp;
  *cur_vs = best_vs;
  // separable form (FP64): tile variant of each grouped phase
  if (sep_only && g->sep.ready) {
    double *phi_t = nullptr, *rho_t = nullptr;
    int st3 = dmalloc(&phi_t, (size_t)M * g->nang);
    if (st3 == YYG_OK && !g->rho) {
      st3 = dmalloc(&rho_t, (size_t)M * g->nang);
      if (st3 == YYG_OK) (void)hipMemsetAsync(rho_t, 0, (size_t)M * g->nang * sizeof(double), s);
    }
    if (st3 == YYG_OK) st3 = sep_set_pointers(g, g->rho ? g->rho : rho_t, phi_t, s);
    // Each phase in turn (the others at their current choice): every
    // variant is timed inside whole back-to-back solves, where the kernels
    // meet the caches and clocks they run under in use (timed alone, the
    // short phases rank differently); a variant replaces the current one only
    // when the solve gets faster by more than 0.5% (at least 0.3 us), so that
    // near-ties do not flip between runs.
    auto solve_ms = [&]() { return time_launch([&] { return sep_solve(g, s); }, s, 5); };
    const bool timing = g->timing;
    g->timing = false;  // no per-phase events while tuning
    for (int r = 0; r < 5 && st3 == YYG_OK; ++r) {
      if (r == 2 && g->n_patch != 2) continue;  // one patch: no rotation
      const int v0 = g->sep.var[r];
      const double t0 = solve_ms();
      double best = t0 - std::max(0.0003, 0.005 * t0);
      int bv = v0;
      for (int v = 0; v < sep_variant_count(r) && st3 == YYG_OK; ++v) {
        if (v == v0 || !sep_variant_available(g, r, v)) continue;
        st3 = sep_set_variant(g, r, v);
        if (st3 != YYG_OK) break;
        const double t = solve_ms();
        if (t < best) {
          best = t;
          bv = v;
        }
      }
      if (st3 == YYG_OK) st3 = sep_set_variant(g, r, bv);
    }
    g->timing = timing;
    (void)hipStreamSynchronize(s);
    if (phi_t) (void)dev_free(phi_t);
    if (rho_t) (void)dev_free(rho_t);
    g->sep.phi_ana.A = nullptr;  // the next solve writes its own pointers
    g->sep.phi_syn.C = nullptr;
    g->sep.phi_ana_d.X = nullptr;
    g->sep.phi_syn_d.C = nullptr;
    g->sep.phi_ana_f.A = nullptr;
    g->sep.phi_ana_s.rho = nullptr;
    g->sep.phi_ana_ab.A = nullptr;
    g->sep.phi_syn_f.C = nullptr;
    g->sep.phi_syn_s.phi = nullptr;
    g->sep.phi_ana_fd.X = nullptr;
    g->sep.phi_syn_fd.C = nullptr;
    g->sep.phi_syn_l.C = nullptr;
    if (st3 != YYG_OK) return st3;
  }
  if (cache_path && !sep_only && (!have_a || !have_s)) {
    if (std::FILE *f = std::fopen(cache_path, "a")) {
      if (!have_a) std::fprintf(f, "%s -> %d %d\n", ka.c_str(), best_va, best_sp);
      if (!have_s) std::fprintf(f, "%s -> %d %d\n", ks.c_str(), best_vs, 1);
      std::fclose(f);
    }
  }
  return YYG_OK;
}

int yyg_plan_config(yyg_grid *g, int precision, int var_ana, int split_ana, int var_syn) {
  if (!g || precision < 0 || precision > YYG_FP16X2) return YYG_ERR_INVALID_ARG;
  const bool lp = precision != YYG_FP64;
  if (lp && !g->lp[precision - 1].ready) return YYG_ERR_NOT_READY;
  const int nv = lp ? yyg::gemm_lp_variant_count() : yyg::gemm_f64_variant_count();
  if (var_ana < 0 || var_ana >= nv || var_syn < 0 || var_syn >= nv || split_ana < 1 || split_ana > 64)
    return YYG_ERR_INVALID_ARG;
  DeviceGuard dg(g->device);
  if (!dg.ok) return YYG_ERR_DEVICE;
  if (split_ana > g->part_cap) {
    const long M = (long)g->n_patch * g->n_r;
    double *np = nullptr;
    if (dmalloc(&np, (size_t)split_ana * M * g->Q) != YYG_OK) return YYG_ERR_OUT_OF_MEMORY;
    (void)hipDeviceSynchronize();
    (void)dev_free(g->d_part);
    g->d_part = np;
    g->part_gen += 1;
    g->part_cap = split_ana;
  }
  if (lp) {
    auto &L = g->lp[precision - 1];
    L.var_ana = var_ana;
    L.nsplit = split_ana;
    L.var_syn = var_syn;
  } else {
    g->var_ana = var_ana;
    g->nsplit = split_ana;
    g->var_syn = var_syn;
  }
  return YYG_OK;
}

int yyg_plan_info(const yyg_grid *g, int precision, int *info, int n) {
  if (!g || !info || n < 1 || precision < 0 || precision > YYG_FP16X2) return YYG_ERR_INVALID_ARG;
  const bool lp = precision != YYG_FP64;
  int va = g->var_ana, sp = g->nsplit, vs = g->var_syn;
  if (lp) {
    va = g->lp[precision - 1].var_ana;
    sp = g->lp[precision - 1].nsplit;
    vs = g->lp[precision - 1].var_syn;
  }
  int ba, bn_a, bs, bn_s;
  if (lp) {
    yyg::gemm_lp_variant_tile(va, &ba, &bn_a);
    yyg::gemm_lp_variant_tile(vs, &bs, &bn_s);
  } else {
    yyg::gemm_f64_variant_tile(va, &ba, &bn_a);
    yyg::gemm_f64_variant_tile(vs, &bs, &bn_s);
  }
  const int vals[7] = {va, sp, vs, ba, bn_a, bs, bn_s};
  for (int i = 0; i < n && i < 7; ++i) info[i] = vals[i];
  return YYG_OK;
}

int yyg_sep_config(yyg_grid *g, int phase, int variant) {
  if (!g || phase < 0 || phase > 4) return YYG_ERR_INVALID_ARG;
  if (!g->sep.ready) return YYG_ERR_NOT_READY;
  if (variant < 0 || variant >= sep_variant_count(phase)) return YYG_ERR_INVALID_ARG;
  DeviceGuard dg(g->device);
  if (!dg.ok) return YYG_ERR_DEVICE;
  if (hipDeviceSynchronize() != hipSuccess) {  // the work items may be in use
    (void)hipGetLastError();
    return YYG_ERR_DEVICE;
  }
  return sep_set_variant(g, phase, variant);
}

int yyg_sep_variant_count(int phase) {
  if (phase < 0 || phase > 4) return YYG_ERR_INVALID_ARG;
  return sep_variant_count(phase);
}

int yyg_sep_info(const yyg_grid *g, int *variants, int n) {
  if (!g || !variants || n < 1) return YYG_ERR_INVALID_ARG;
  for (int i = 0; i < n && i < 5; ++i)
    variants[i] = (!g->sep.ready || (i == 2 && g->n_patch != 2)) ? -1 : g->sep.var[i];
  return YYG_OK;
}

int yyg_sep_phase(yyg_grid *g, int phase, double *phi, void *stream) {
  if (!g || !phi || phase < 0 || phase > 4) return YYG_ERR_INVALID_ARG;
  if (g->method != YYG_METHOD_SEPARABLE || !g->sep.ready || !g->rho) return YYG_ERR_NOT_READY;
  DeviceGuard dg(g->device);
  if (!dg.ok) return YYG_ERR_DEVICE;
  hipStream_t s = as_stream(stream);
  const int st = sep_set_pointers(g, g->rho, phi, s);
  if (st != YYG_OK) return st;
  if (sep_launch_phase(g, phase, s) != hipSuccess) {
    (void)hipGetLastError();
    return YYG_ERR_DEVICE;
  }
  return YYG_OK;
}

int yyg_sep_kernel(const yyg_grid *g, int phase, char *name, size_t n) {
  if (!g || !name || n < 1 || phase < 0 || phase > 4) return YYG_ERR_INVALID_ARG;
  if (!g->sep.ready) return YYG_ERR_NOT_READY;
  if (phase == 2 && g->n_patch != 2) {
    name[0] = 0;
    return YYG_OK;
  }
  const int v = g->sep.var[phase], x0 = sep_x4_base(phase);
  const int r = phase == 4 && v >= sep_stream_base(4) ? yyg::phi_stream_kernel_name(v - sep_stream_base(4), name, n)
                : phase == 0 && v >= sep_xcol_base(0) ? yyg::fold_xcol_kernel_name(v - sep_xcol_base(0), name, n)
                : phase == 0 && v >= sep_stream_base(0)
                    ? yyg::phi_ana_stream_kernel_name(v - sep_stream_base(0), name, n)
                : v >= x0 ? yyg::x4_kernel_name(v - x0, phase, g->sep.fold, name, n)
                          : yyg::sep_kernel_name(phase, v, g->sep.fold, name, n);
  return r == 0 ? YYG_OK : YYG_ERR_INVALID_ARG;
}

int yyg_sep_lp_config(yyg_grid *g, int precision, int phase, int tile) {
  if (!g || (phase != 0 && phase != 4)) return YYG_ERR_INVALID_ARG;
  if (precision != YYG_FP32 && precision != YYG_BF16X3) return YYG_ERR_INVALID_ARG;
  if (!g->sep.ready) return YYG_ERR_NOT_READY;
  const int side = phase == 0 ? 0 : 1;
  if (tile < 0 || tile >= yyg::sep_lp_tile_count() +
                              std::max(yyg::phi_stream32_variant_count(), yyg::phi_ana_stream32_variant_count()))
    return YYG_ERR_INVALID_ARG;
  if (!sep_lp_available(g, precision, side, tile)) return YYG_ERR_UNSUPPORTED;
  g->sep.lpt[precision - 1][side] = tile;
  return YYG_OK;
}

int yyg_sep_lp_kernel(const yyg_grid *g, int precision, int phase, char *name, size_t n) {
  if (!g || !name || n < 1 || (phase != 0 && phase != 4)) return YYG_ERR_INVALID_ARG;
  if (precision != YYG_FP32 && precision != YYG_BF16X3) return YYG_ERR_INVALID_ARG;
  if (!g->sep.ready) return YYG_ERR_NOT_READY;
  const int t = g->sep.lpt[precision - 1][phase == 0 ? 0 : 1], u = t - yyg::sep_lp_tile_count();
  const int r = u < 0        ? yyg::sep_lp_kernel_name(precision, t, phase, g->sep.fold, name, n)
                : phase == 4 ? yyg::phi_stream32_kernel_name(u, name, n)
                             : yyg::phi_ana_stream32_kernel_name(u, name, n);
  return r == 0 ? YYG_OK : YYG_ERR_INVALID_ARG;
}

int yyg_batch_create(yyg_grid *const *grids, int n, int precision, yyg_batch **out) {
  if (!out) return YYG_ERR_INVALID_ARG;
  *out = nullptr;
  if (!grids || n < 1 || precision < 0 || precision > YYG_FP16X2) return YYG_ERR_INVALID_ARG;
  // the separable form when every plan is in it (FP64), the dense form otherwise
  bool sep = precision == YYG_FP64;
  for (int f = 0; f < n; ++f) {
    if (!grids[f] || grids[f]->device != grids[0]->device) return YYG_ERR_INVALID_ARG;
    sep = sep && grids[f]->method == YYG_METHOD_SEPARABLE && grids[f]->sep.ready;
  }
  for (int f = 0; f < n; ++f) {
    if (!sep && grids[f]->n_r > 1024) return YYG_ERR_UNSUPPORTED;
    if (precision != YYG_FP64 && !grids[f]->lp[precision - 1].ready) return YYG_ERR_NOT_READY;
  }
  yyg_batch *b = new (std::nothrow) yyg_batch;
  if (!b) return YYG_ERR_OUT_OF_MEMORY;
  b->device = grids[0]->device;
  b->precision = precision;
  b->sep = sep;
  b->grids.assign(grids, grids + n);
  DeviceGuard dg(b->device);
  if (!dg.ok) {
    delete b;
    return YYG_ERR_DEVICE;
  }
  int st = sep ? sep_batch_build(b) : batch_build(b);
  if (st != YYG_OK) {
    batch_free(b);
    return st;
  }
  *out = b;
  return YYG_OK;
}

int yyg_batch_autotune(yyg_batch *b, void *stream) {
  if (!b) return YYG_ERR_INVALID_ARG;
  // the timed launches read the densities and write the potentials of the
  // last batched solve
  if (!b->launched) return YYG_ERR_NOT_READY;
  DeviceGuard dg(b->device);
  if (!dg.ok) return YYG_ERR_DEVICE;
  hipStream_t s = as_stream(stream);
  if (hipStreamSynchronize(b->stream) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    (void)hipGetLastError();
    return YYG_ERR_DEVICE;
  }
  if (b->sep) {
    // each phase in turn, the others at their current tile: whole eager
    // batched solves, the fastest of three per tile
    for (int r = 0; r < 5; ++r) {
      if (r == 2 && b->n_sitems[2] == 0) continue;  // no two-patch plan: nothing to rotate
      int best = b->svar[r];
      double bt = 1e30;
      for (int t = 0; t < yyg::sep_batch_tile_count(); ++t) {
        int st = sep_batch_set_items(b, r, t);
        if (st != YYG_OK) return st;
        const double tm = time_launch([&] { return sep_batch_enqueue(b, s, nullptr); }, s, 3);
        if (tm < bt) {
          bt = tm;
          best = t;
        }
      }
      int st = sep_batch_set_items(b, r, best);
      if (st != YYG_OK) return st;
    }
    batch_drop_graph(b);
    return YYG_OK;
  }
  const bool lp = b->precision != YYG_FP64;
  const int nv = lp ? yyg::gemm_lp_variant_count() : yyg::gemm_f64_variant_count();
  // time each phase's contraction per tile variant on the batch's own
  // problems (density pointers of the last solve, or whatever the plans
  // hold: timings do not depend on the values)
  int best[2] = {b->var[0], b->var[1]};
  for (int role = 0; role < 2; ++role) {
    double bt = 1e30;
    for (int v = 0; v < nv; ++v) {
      int st = batch_set_items(b, role, v);
      if (st != YYG_OK) return st;
      double t = time_launch([&] { return batch_launch_gemm(b, role, s); }, s, 3);
      if (t < bt) {
        bt = t;
        best[role] = v;
      }
    }
  }
  for (int role = 0; role < 2; ++role) {
    int st = batch_set_items(b, role, best[role]);
    if (st != YYG_OK) return st;
  }
  batch_drop_graph(b);
  return YYG_OK;
}

int yyg_batch_info(const yyg_batch *b, int *info, int n) {
  if (!b || !info || n < 1) return YYG_ERR_INVALID_ARG;
  if (b->sep) {
    const int vals[9] = {(int)b->grids.size(), b->precision, b->svar[0], b->svar[4], b->n_sitems[0], b->n_sitems[4],
                         b->svar[1], b->svar[2], b->svar[3]};
    for (int i = 0; i < n && i < 9; ++i) info[i] = vals[i];
    return YYG_OK;
  }
  const int vals[9] = {(int)b->grids.size(), b->precision, b->var[0], b->var[1], b->n_items[0], b->n_items[1],
                       -1, -1, -1};
  for (int i = 0; i < n && i < 9; ++i) info[i] = vals[i];
  return YYG_OK;
}

int yyg_batch_solve(yyg_batch *b, const double *const *d_rho, double *const *d_phi, void *stream) {
  if (!b || !d_rho || !d_phi) return YYG_ERR_INVALID_ARG;
  const int n = (int)b->grids.size();
  for (int f = 0; f < n; ++f)
    if (!d_rho[f] || !d_phi[f]) return YYG_ERR_INVALID_ARG;
  // a plan's work buffer moved (autotune / plan_config after the batch was
  // built): the recorded arguments are stale
  for (int f = 0; f < n; ++f)
    if (b->grids[f]->part_gen != b->part_gen[f]) return YYG_ERR_NOT_READY;
  DeviceGuard dg(b->device);
  if (!dg.ok) return YYG_ERR_DEVICE;
  // a graph cannot be recorded on the legacy default stream: use the
  // batch's own blocking stream, which that stream orders against
  hipStream_t s = stream ? as_stream(stream) : b->stream;
  for (int f = 0; f < n; ++f)
    if (int st = check_rho(b->grids[f], d_rho[f], s); st != YYG_OK) return st;
  for (int f = 0; f < n; ++f) b->grids[f]->ahat_cols = b->sep;  // the moments' layout the batch leaves
  bool changed = false;
  for (int f = 0; f < n; ++f)
    if (b->rho[f] != d_rho[f] || b->phi[f] != d_phi[f]) changed = true;
  if (changed) {
    // the previous launch may still read the staged arguments
    if (b->launched && hipEventSynchronize(b->done) != hipSuccess) {
      (void)hipGetLastError();
      return YYG_ERR_DEVICE;
    }
    for (int f = 0; f < n; ++f) {
      b->rho[f] = d_rho[f];
      b->phi[f] = d_phi[f];
    }
    batch_patch_pointers(b);
  }
  hipError_t e = hipSuccess;
  if (!b->exec || b->exec_stream != s) {
    batch_drop_graph(b);
    // record the whole batched solve once, replay it afterwards
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t e2 = batch_enqueue(b, s);
      hipGraph_t graph = nullptr;
      e = hipStreamEndCapture(s, &graph);
      if (e == hipSuccess) e = e2;
      if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      if (e == hipSuccess) b->exec_stream = s;
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      batch_drop_graph(b);
      return YYG_ERR_DEVICE;
    }
  }
  e = hipGraphLaunch(b->exec, s);
  if (e == hipSuccess) e = hipEventRecord(b->done, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return YYG_ERR_DEVICE;
  }
  b->launched = true;
  return YYG_OK;
}

int yyg_batch_profile(yyg_batch *b, void *stream, double *ms, int n) {
  if (!b || !ms || n < 1) return YYG_ERR_INVALID_ARG;
  if (!b->launched) return YYG_ERR_NOT_READY;
  DeviceGuard dg(b->device);
  if (!dg.ok) return YYG_ERR_DEVICE;
  hipStream_t s = stream ? as_stream(stream) : b->stream;
  hipEvent_t ev[6];
  for (auto &x : ev)
    if (hipEventCreate(&x) != hipSuccess) return YYG_ERR_DEVICE;
  if (b->sep) {
    // phases 0-2 (phi and theta analysis, rotation), the scans, phases 3-4
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = sep_batch_enqueue(b, s, ev);
    if (e == hipSuccess) e = hipEventSynchronize(ev[5]);
    float t[5] = {0, 0, 0, 0, 0};
    for (int i = 0; i < 5 && e == hipSuccess; ++i) e = hipEventElapsedTime(&t[i], ev[i], ev[i + 1]);
    for (auto &x : ev) (void)hipEventDestroy(x);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return YYG_ERR_DEVICE;
    }
    const double vals[4] = {(double)t[0] + t[1], t[2], (double)t[3] + t[4], 0.0};
    for (int i = 0; i < n && i < 4; ++i) ms[i] = vals[i];
    return YYG_OK;
  }
  const int nf = (int)b->grids.size();
  const bool lp = b->precision != YYG_FP64;
  hipError_t e = hipStreamSynchronize(s);
  // the same launches as the recorded graph, eagerly, with events between
  if (e == hipSuccess) {
    if (!lp) {
      e = hipMemcpyAsync(b->d_f64[0], b->h_f64[0], nf * sizeof(yyg::GemmF64Args), hipMemcpyHostToDevice, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_f64[1], b->h_f64[1], nf * sizeof(yyg::GemmF64Args), hipMemcpyHostToDevice, s);
    } else {
      e = hipMemcpyAsync(b->d_split[0], b->h_split[0], nf * sizeof(yyg::SplitArgs), hipMemcpyHostToDevice, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_lp[1], b->h_lp[1], nf * sizeof(yyg::GemmLpArgs), hipMemcpyHostToDevice, s);
    }
  }
  if (e == hipSuccess) e = hipEventRecord(ev[0], s);
  if (e == hipSuccess && lp)
    e = yyg::launch_split_rows_grouped(b->precision, b->d_split[0], b->d_split_items[0], b->n_split_items[0],
                                       std::min(b->n_split_items[0], b->cus * 8), s);
  if (e == hipSuccess) e = hipEventRecord(ev[1], s);
  if (e == hipSuccess) e = batch_launch_gemm(b, 0, s);
  if (e == hipSuccess) e = hipEventRecord(ev[2], s);
  if (e == hipSuccess)
    e = yyg::launch_radial_scan_grouped(b->d_scan, b->d_scan_items, b->n_scan_items,
                                        std::min(b->n_scan_items, b->cus * 2), s);
  if (e == hipSuccess) e = hipEventRecord(ev[3], s);
  if (e == hipSuccess && lp)
    e = yyg::launch_split_rows_grouped(b->precision, b->d_split[1], b->d_split_items[1], b->n_split_items[1],
                                       std::min(b->n_split_items[1], b->cus * 8), s);
  if (e == hipSuccess) e = hipEventRecord(ev[4], s);
  if (e == hipSuccess) e = batch_launch_gemm(b, 1, s);
  if (e == hipSuccess) e = hipEventRecord(ev[5], s);
  if (e == hipSuccess) e = hipEventSynchronize(ev[5]);
  float t[5] = {0, 0, 0, 0, 0};
  for (int i = 0; i < 5 && e == hipSuccess; ++i) e = hipEventElapsedTime(&t[i], ev[i], ev[i + 1]);
  for (auto &x : ev) (void)hipEventDestroy(x);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return YYG_ERR_DEVICE;
  }
  // slots as for plans: 0 analysis, 1 scan, 2 synthesis, 3 operand splits
  const double vals[4] = {t[1], t[2], t[4], (double)t[0] + t[3]};
  for (int i = 0; i < n && i < 4; ++i) ms[i] = vals[i];
  return YYG_OK;
}

int yyg_batch_destroy(yyg_batch *b) {
  if (!b) return YYG_ERR_INVALID_ARG;
  DeviceGuard dg(b->device);
  (void)hipDeviceSynchronize();
  batch_free(b);
  return YYG_OK;
}

}  // extern "C"
