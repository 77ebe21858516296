// Host implementation of the C ABI declared in include/lbm.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_adjoint.h"
#include "lbm_internal.h"
#include "lbm_site.h"

using namespace lbm;

namespace {

thread_local std::string g_err;

lbm_status fail(lbm_status s, const std::string& msg) {
  g_err = msg;
  return s;
}
lbm_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return LBM_EHIP;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int elem_bytes(int storage) { return storage == LBM_F64 ? 8 : storage == LBM_F32 ? 4 : 2; }
bool is_f64(int storage) { return storage == LBM_F64; }

struct Layout {
  int Q = 0, pitch = 0;
  long long qs = 0, n_sites = 0, cap = 0, k = 0, bcap = 0;
  size_t lat_bytes = 0;
  int rows = 0;            // ny, or nz * ny for D3Q27
  size_t off_nl = 0;       // nonlocal filter coefficients (27 values of the compute type)
  size_t off_lat[2] = {0, 0}, off_omega = 0, off_sel = 0, off_cnt = 0, off_partial = 0,
         off_stats = 0, off_div = 0, off_ckey = 0, off_cidx = 0, off_cmom = 0, off_hist = 0,
         off_coarse = 0, off_wcount = 0, off_ccount = 0, off_stage = 0, off_blist = 0,
         off_selected = 0, off_f64list = 0, off_f64cnt = 0, off_ens = 0, off_ens_dsb = 0,
         off_ens_cnt = 0, off_ens_sum = 0;
  AdjointLayout adj;
  size_t total = 0;
};

// Rows of the stored lattice: ny, or nz * ny for D3Q27 (row z * ny + y).
long long rows_of(const lbm_config* c) {
  return c->lattice == LBM_D3Q27 ? (long long)c->ny * c->nz : c->ny;
}
int q_of(const lbm_config* c) { return c->lattice == LBM_D3Q27 ? 27 : (c->lattice == LBM_D2Q9 ? 9 : 3); }

bool validate(const lbm_config* c, std::string& why) {
  if (!c) { why = "config is NULL"; return false; }
  if (c->lattice != LBM_D1Q3 && c->lattice != LBM_D2Q9 && c->lattice != LBM_D3Q27) {
    why = "lattice must be LBM_D1Q3, LBM_D2Q9 or LBM_D3Q27"; return false;
  }
  if (c->nx < 1 || c->ny < 1) { why = "nx and ny must be positive"; return false; }
  if (c->lattice != LBM_D3Q27 && c->nz > 1) { why = "nz > 1 needs LBM_D3Q27"; return false; }
  if (c->lattice == LBM_D3Q27 && c->nz < 1) { why = "nz must be positive"; return false; }
  if ((long long)c->nx * rows_of(c) >= (1ll << 31)) { why = "nx*ny*nz must be below 2^31"; return false; }
  if (c->lattice == LBM_D3Q27) {
    // population planes are addressed with 32-bit byte offsets
    const long long plane = (long long)(c->nx + 63) / 64 * 64 * rows_of(c) * elem_bytes(c->storage);
    if (plane >= (1ll << 32)) { why = "a D3Q27 population plane must stay below 4 GiB"; return false; }
    if (c->bc != LBM_BC_PERIODIC) { why = "D3Q27 lattices are periodic"; return false; }
    if (c->collision != LBM_LBGK) { why = "D3Q27 lattices collide with LBGK"; return false; }
    if (c->limiters & LBM_LIM_EHRENFEST) { why = "D3Q27 has no Ehrenfest selection"; return false; }
    if (c->ens_limiter != LBM_ENS_NONE || c->checkpoint_every > 0 || c->omega_field || c->nl_filter) {
      why = "D3Q27 excludes the ensemble limiters, the adjoint, the omega field and the nonlocal filter";
      return false;
    }
  }
  if (c->nl_filter) {
    if (c->lattice == LBM_D3Q27 || c->bc != LBM_BC_PERIODIC) {
      why = "the nonlocal filter needs a periodic D1Q3 or D2Q9 lattice"; return false;
    }
    if (c->limiters & (LBM_LIM_MEDIAN | LBM_LIM_EHRENFEST) || c->ens_limiter != LBM_ENS_NONE ||
        c->checkpoint_every > 0) {
      why = "the nonlocal filter excludes the median filter, the Ehrenfest selection, the "
            "ensemble limiters and the adjoint";
      return false;
    }
    for (int k = 0; k < 27; ++k)
      if (!std::isfinite(c->nl_coef[k])) { why = "nl_coef must be finite"; return false; }
  }
  if (c->lattice == LBM_D1Q3 && c->ny != 1) { why = "D1Q3 needs ny = 1"; return false; }
  if (c->lattice == LBM_D1Q3 && c->bc != LBM_BC_PERIODIC && c->bc != LBM_BC_BOUNCEBACK) {
    why = "D1Q3 supports periodic and bounce-back ends only"; return false;
  }
  if (c->bc < 0 || c->bc > 4) { why = "unknown boundary"; return false; }
  if (c->bc == LBM_BC_DIFFUSIVE) {
    if (c->lattice != LBM_D2Q9 || c->nx < 3 || c->ny < 3) {
      why = "the diffusive wall needs D2Q9 with nx, ny >= 3"; return false;
    }
    if (c->ens_limiter != LBM_ENS_NONE) { why = "the diffusive wall excludes the ensemble limiters"; return false; }
    if (c->checkpoint_every > 0) {
      why = "the adjoint does not cover the diffusive wall (checkpoint_every must be 0)"; return false;
    }
  }
  if (c->collision < 0 || c->collision > 2) { why = "unknown collision"; return false; }
  if (c->collision == LBM_MRT && c->lattice != LBM_D2Q9) { why = "MRT is defined for D2Q9"; return false; }
  if (c->storage < 0 || c->storage > 3) { why = "unknown storage"; return false; }
  if (c->nu < 0 && !(c->omega > 0 && c->omega < 2.0000001)) { why = "omega must lie in (0, 2]"; return false; }
  if ((c->limiters & LBM_LIM_EHRENFEST) && (c->ehr_k < 0 || !(c->ehr_delta >= 0))) {
    why = "ehr_k and ehr_delta must be >= 0"; return false;
  }
  if (c->collision == LBM_ELBM && c->elbm_max_iter < 1) { why = "elbm_max_iter must be >= 1"; return false; }
  if (c->mrt_preset < LBM_RATES_GIVEN || c->mrt_preset > LBM_RATES_SHEAR) { why = "unknown mrt_preset"; return false; }
  if (c->mrt_preset != LBM_RATES_GIVEN && c->mrt_basis != LBM_MRT_M1) {
    why = "the rate presets are rates of the M1 basis"; return false;
  }
  if (c->sel_action != LBM_SEL_EQUILIBRIUM && c->sel_action != LBM_SEL_MRT) { why = "unknown sel_action"; return false; }
  if (c->sel_action == LBM_SEL_MRT &&
      (!(c->limiters & LBM_LIM_EHRENFEST) || c->collision != LBM_LBGK || c->lattice != LBM_D2Q9)) {
    why = "the MRT limiter (sel_action = LBM_SEL_MRT) needs the Ehrenfest selection, LBGK and D2Q9";
    return false;
  }
  if (c->ens_limiter < LBM_ENS_NONE || c->ens_limiter > LBM_ENS_POINTWISE) { why = "unknown ens_limiter"; return false; }
  if (c->ens_limiter != LBM_ENS_NONE) {
    if (c->limiters & LBM_LIM_MEDIAN) { why = "the ensemble limiters and the median filter exclude each other"; return false; }
    if (c->checkpoint_every > 0) { why = "the adjoint does not cover the ensemble limiters (checkpoint_every must be 0)"; return false; }
    if (!(c->ens_k > 0) || !(c->ens_alpha > 0) || !(c->ens_delta >= 0)) {
      why = "ens_k and ens_alpha must be > 0 and ens_delta >= 0"; return false;
    }
    if ((c->ens_limiter == LBM_ENS_THRESHOLD || c->ens_limiter == LBM_ENS_DOUBLE_MONOTONE) &&
        !(c->ens_delta0 > 0) && !(c->ens_delta > 0)) {
      why = "a threshold needs ens_delta0 > 0 (eq. EntThresh) or ens_delta > 0"; return false;
    }
  }
  if (c->checkpoint_every < 0 || c->max_steps < 0) { why = "checkpoint_every/max_steps must be >= 0"; return false; }
  if (c->checkpoint_every > 0 && c->max_steps < 1) { why = "checkpoint_every > 0 needs max_steps >= 1"; return false; }
  return true;
}

// lattices = false: the two lattices are the caller's (not in the
// workspace), densely packed (row pitch nx), and no adjoint is recorded.
Layout make_layout(const lbm_config* c, bool lattices = true) {
  Layout L;
  L.Q = q_of(c);
  L.rows = (int)rows_of(c);
  L.pitch = lattices ? (c->nx + 63) / 64 * 64 : c->nx;
  L.qs = (long long)L.rows * L.pitch;
  L.n_sites = (long long)c->nx * L.rows;
  L.lat_bytes = (size_t)L.Q * L.qs * elem_bytes(c->storage);
  const size_t rb = is_f64(c->storage) ? 8 : 4;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o += align256(bytes); return at; };
  if (lattices) {
    L.off_lat[0] = take(L.lat_bytes);
    L.off_lat[1] = take(L.lat_bytes);
  }
  L.off_omega = c->omega_field ? take((size_t)L.qs * rb) : 0;
  L.off_sel = take(sizeof(SelState));
  L.off_cnt = take((size_t)kCntSlots * CNT_N * sizeof(unsigned long long));
  L.off_partial = take(stats_partial_doubles(c->nx, L.rows) * sizeof(double));
  L.off_nl = c->nl_filter ? take(27 * rb) : 0;
  L.off_stats = take(8 * sizeof(double));
  L.off_div = take(sizeof(long long));
  if (c->limiters & LBM_LIM_EHRENFEST) {
    L.k = c->ehr_k < L.n_sites ? c->ehr_k : L.n_sites;
    // every wavefront of the step kernel owns 64 candidate entries
    const TileShape ts = tile_shape(L.Q, (c->limiters & LBM_LIM_MEDIAN) != 0, c->nx);
    const long long tiles = (long long)((c->nx + ts.tx - 1) / ts.tx) * ((c->ny + ts.ty - 1) / ts.ty);
    L.cap = tiles * 256;
    L.off_ckey = take((size_t)L.cap * rb);
    L.off_cidx = take((size_t)L.cap * 4);
    L.off_cmom = take((size_t)L.cap * 3 * rb);
    L.off_wcount = take((size_t)tiles * 4 * 4);
    L.off_hist = take((size_t)kHistWords * 4);
    L.off_coarse = take(kCoarse * 4);
    L.off_ccount = take((size_t)kCountSlots * kCountStride * 8);
    // kSweepRegions regions x 64 entries per k_fix_regions workgroup
    L.off_stage = take((size_t)((tiles * 4 + kSweepRegions - 1) / kSweepRegions) * kSweepRegions * 64 * 4);
    L.bcap = std::min<long long>(L.cap, 1ll << 20);
    L.off_blist = take((size_t)L.bcap * 4);
    L.off_selected = take((size_t)std::max<long long>(L.k, 1) * 4);
  }
  if (c->collision == LBM_ELBM && !is_f64(c->storage)) {
    L.off_f64list = take((size_t)L.n_sites * 4);
    L.off_f64cnt = take(2 * sizeof(unsigned int));
  }
  if (c->ens_limiter != LBM_ENS_NONE) {
    L.off_ens = take(sizeof(EnsState));
    L.off_ens_dsb = take((size_t)L.qs * rb);
    L.off_ens_cnt = take((size_t)kEnsBins * 4);
    L.off_ens_sum = take((size_t)kEnsBins * 8);
  }
  if (lattices) {
    L.adj = adjoint_layout(c, L.lat_bytes, L.qs, L.k, o);
    o = L.adj.end;
  }
  L.total = o;
  return L;
}

double omega_of(const lbm_config* c) { return c->nu >= 0 ? 1.0 / (3.0 * c->nu + 0.5) : c->omega; }

// MRT change of basis (section 5), rebuilt from its velocity polynomials in
// tensor order; inverse by Gauss-Jordan elimination with partial pivoting.
void mrt_matrices(int basis, double M[81], double Minv[81]) {
  for (int i = 0; i < 9; ++i) {
    const double vx = (i % 3) - 1, vy = (i / 3) - 1, v2 = vx * vx + vy * vy;
    double r[9];
    if (basis == LBM_MRT_M1) {
      r[0] = 1; r[1] = -4 + 3 * v2; r[2] = 4 - 10.5 * v2 + 4.5 * v2 * v2; r[3] = vx;
      r[4] = (-5 + 3 * v2) * vx; r[5] = vy; r[6] = (-5 + 3 * v2) * vy; r[7] = vx * vx - vy * vy;
      r[8] = vx * vy;
    } else {
      r[0] = 1; r[1] = vx; r[2] = vy; r[3] = v2; r[4] = vx * vx - vy * vy; r[5] = vx * vy;
      r[6] = vx * vx * vy; r[7] = vx * vy * vy; r[8] = vx * vx * vy * vy;
    }
    for (int k = 0; k < 9; ++k) M[k * 9 + i] = r[k];
  }
  double a[9][18];
  for (int r = 0; r < 9; ++r)
    for (int c = 0; c < 18; ++c) a[r][c] = c < 9 ? M[r * 9 + c] : (c - 9 == r ? 1.0 : 0.0);
  for (int c = 0; c < 9; ++c) {
    int p = c;
    for (int r = c + 1; r < 9; ++r) if (std::fabs(a[r][c]) > std::fabs(a[p][c])) p = r;
    if (p != c) for (int k = 0; k < 18; ++k) std::swap(a[p][k], a[c][k]);
    const double piv = a[c][c];
    for (int k = 0; k < 18; ++k) a[c][k] /= piv;
    for (int r = 0; r < 9; ++r) {
      if (r == c) continue;
      const double f = a[r][c];
      if (f != 0.0) for (int k = 0; k < 18; ++k) a[r][k] -= f * a[c][k];
    }
  }
  for (int r = 0; r < 9; ++r)
    for (int c = 0; c < 9; ++c) Minv[r * 9 + c] = a[r][c + 9];
}

template <class R>
void fill_args(StepArgs<R>& A, const lbm_config* c, const Layout& L, char* ws) {
  std::memset((void*)&A, 0, sizeof(A));
  A.qs = L.qs; A.nx = c->nx; A.ny = L.rows; A.pitch = L.pitch;
  A.ny3 = c->ny;
  A.nz = c->lattice == LBM_D3Q27 ? c->nz : 1;
  A.nl_coef = L.off_nl ? (const R*)(ws + L.off_nl) : nullptr;
  const TileShape ts = tile_shape(L.Q, (c->limiters & LBM_LIM_MEDIAN) != 0, c->nx);
  A.tiles_x = (c->nx + ts.tx - 1) / ts.tx;
  A.tiles_y = (c->ny + ts.ty - 1) / ts.ty;
  A.tile_tx = ts.tx;
  A.bc = c->bc;
  A.eq_kind = c->collision == LBM_ELBM ? LBM_EQ_ENTROPIC : c->equilibrium;
  A.positivity = (c->limiters & LBM_LIM_POSITIVITY) ? 1 : 0;
  A.ehrenfest = (c->limiters & LBM_LIM_EHRENFEST) ? 1 : 0;
  A.count_events = 1;
  A.rho0 = (R)c->rho0;
  const double om = omega_of(c);
  A.omega = (R)om;
  A.omega_field = c->omega_field ? (const R*)(ws + L.off_omega) : nullptr;
  for (int i = 0; i < 9; ++i) A.lid[i] = 0;
  A.lid_u = c->bc == LBM_BC_DIFFUSIVE ? (R)c->u_lid : R(0);
  if (c->bc == LBM_BC_CAVITY || c->bc == LBM_BC_COUETTE) {
    for (int i = 0; i < L.Q; ++i) {
      const int a = L.Q == 9 ? (i % 3) - 1 : i - 1;
      const int b = L.Q == 9 ? (i / 3) - 1 : 0;
      const double w = (L.Q == 9 ? (a == 0 ? 2.0 / 3.0 : 1.0 / 6.0) * (b == 0 ? 2.0 / 3.0 : 1.0 / 6.0)
                                 : (a == 0 ? 2.0 / 3.0 : 1.0 / 6.0));
      A.lid[i] = (R)(6.0 * w * c->rho_wall * a * c->u_lid);
    }
  }
  // MRT: the collision itself, or the MRT limiter at the selected sites of
  // an LBGK lattice (section 5)
  A.sel_mrt = c->sel_action == LBM_SEL_MRT ? 1 : 0;
  if (c->collision == LBM_MRT || A.sel_mrt) {
    double M[81], Mi[81];
    mrt_matrices(c->mrt_basis, M, Mi);
    for (int i = 0; i < 81; ++i) { A.M[i] = (R)M[i]; A.Minv[i] = (R)Mi[i]; }
    double rates[9];
    if (c->mrt_basis == LBM_MRT_M1) {
      // rows rho, e, epsilon, j_x, q_x, j_y, q_y, p_xx, p_xy
      double se = c->s_e, seps = c->s_eps, sq = c->s_q;
      A.nu_rows = (1u << 7) | (1u << 8);
      A.q_rows = 0;
      A.q_mode = 0;
      switch (c->mrt_preset) {
        case LBM_RATES_TRT:        // s_e = s_eps = s_nu, s_q = 8 (2 - s_nu) / (8 - s_nu)
          A.nu_rows |= (1u << 1) | (1u << 2);
          A.q_rows = (1u << 4) | (1u << 6);
          A.q_mode = 1;
          break;
        case LBM_RATES_MRT_TRTQ:   // s_e = 1.64, s_eps = 1.54, TRT third-order rate
          se = 1.64; seps = 1.54;
          A.q_rows = (1u << 4) | (1u << 6);
          A.q_mode = 1;
          break;
        case LBM_RATES_MRT1:
          se = 1.64; seps = 1.54; sq = 1.9;
          break;
        case LBM_RATES_SHEAR:      // s_q = 3 (2 - s_nu) / (3 - s_nu)
          se = 1.64; seps = 1.54;
          A.q_rows = (1u << 4) | (1u << 6);
          A.q_mode = 2;
          break;
        default:
          break;
      }
      const double r1[9] = {1, se, seps, 1, sq, 1, sq, om, om};
      std::memcpy(rates, r1, sizeof(rates));
    } else {
      const double r2[9] = {1, 1, 1, 1, om, om, 1, 1, 1};
      std::memcpy(rates, r2, sizeof(rates));
      A.nu_rows = (1u << 4) | (1u << 5);
    }
    for (int i = 0; i < 9; ++i) A.rates[i] = (R)rates[i];
  }
  A.eps = (R)c->elbm_eps;
  A.atol = sizeof(R) == 4 ? (R)5e-7 : (R)0;
  A.dS_cut = (R)c->elbm_dS_cut;
  A.max_iter = c->elbm_max_iter;
  A.norm = c->elbm_norm;
  A.fallback = c->elbm_fallback;
  A.eps64 = c->elbm_eps;
  A.dS_cut64 = c->elbm_dS_cut;
  A.f64_below = (R)c->elbm_f64_below;
  A.med_delta = (R)c->med_delta;
  A.ehr_delta = (R)c->ehr_delta;
  A.sel = (SelState*)(ws + L.off_sel);
  A.counters = (unsigned long long*)(ws + L.off_cnt);
  A.ens_mode = c->ens_limiter;
  A.ens_alpha = (R)c->ens_alpha;
  A.ens_k = (R)c->ens_k;
  A.ens_delta = (R)c->ens_delta;
  if (c->ens_limiter != LBM_ENS_NONE) {
    A.ens = (EnsState*)(ws + L.off_ens);
    A.ens_dsb = (R*)(ws + L.off_ens_dsb);
    A.ens_cnt = (unsigned int*)(ws + L.off_ens_cnt);
    A.ens_sum = (double*)(ws + L.off_ens_sum);
  }
  A.f64_sites = L.off_f64list ? (uint32_t*)(ws + L.off_f64list) : nullptr;
  A.f64_count = L.off_f64cnt ? (unsigned int*)(ws + L.off_f64cnt) : nullptr;
  if (A.ehrenfest) {
    A.cand_key = (typename KeyOf<R>::T*)(ws + L.off_ckey);
    A.cand_idx = (uint32_t*)(ws + L.off_cidx);
    A.cand_mom = (R*)(ws + L.off_cmom);
    A.cap = L.cap;
    A.wcount = (uint32_t*)(ws + L.off_wcount);
    A.ccount = (unsigned long long*)(ws + L.off_ccount);
    A.hist = (unsigned int*)(ws + L.off_hist);
  }
}

}  // namespace

// Steps per captured graph (even: a replay starts and ends on the same lattice).
constexpr int kGraphSteps = 16;

struct lbm_ctx {
  lbm_config cfg;
  Layout L;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int cur = 0;               // lattice holding the current state
  long long steps = 0;
  bool recorded = false;     // a rollout usable by lbm_backward exists
  StepArgs<double> a64;
  StepArgs<float> a32;
  // kGraphSteps steps captured once per starting lattice and replayed by
  // lbm_step (kernels only; every argument is the same at each replay)
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [recording][lattice]
  void* lat(int i) { return ws + L.off_lat[i]; }
  bool f64() const { return cfg.storage == LBM_F64; }
  ~lbm_ctx() {
    for (auto& gg : graph)
      for (auto& g : gg)
        if (g) hipGraphExecDestroy(g);
    if (cap_stream) hipStreamDestroy(cap_stream);
  }
};

static SelectArgs select_args(lbm_ctx* c, const void* args);
static hipError_t capture_graph(lbm_ctx* c);

extern "C" {

void lbm_config_default(lbm_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->lattice = LBM_D2Q9; c->nx = 64; c->ny = 64; c->bc = LBM_BC_PERIODIC;
  c->rho_wall = 1.0; c->collision = LBM_LBGK; c->equilibrium = LBM_EQ_POLY;
  c->nu = -1.0; c->omega = 1.0; c->mrt_basis = LBM_MRT_M1;
  c->s_e = 1.64; c->s_eps = 1.54; c->s_q = 1.9;
  c->med_delta = 1e-3; c->elbm_norm = LBM_NORM_ENTROPIC; c->elbm_fallback = LBM_FB_POSITIVITY;
  c->elbm_eps = 1e-14; c->elbm_max_iter = 32; c->elbm_dS_cut = 1e-15; c->elbm_f64_below = 3.0;
  c->storage = LBM_F32; c->rho0 = 1.0; c->nz = 1;
}

size_t lbm_workspace_bytes(const lbm_config* cfg) {
  std::string why;
  if (!validate(cfg, why)) { g_err = why; return 0; }
  return make_layout(cfg).total;
}

lbm_status lbm_init(const lbm_config* cfg, void* ws, size_t ws_bytes, void* stream,
                    lbm_ctx** out) {
  g_err.clear();
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  std::string why;
  if (!validate(cfg, why)) return fail(LBM_EINVAL, why);
  Layout L = make_layout(cfg);
  if (!ws || ws_bytes < L.total)
    return fail(LBM_EWORKSPACE, "workspace needs " + std::to_string(L.total) + " bytes");
  if (((uintptr_t)ws & 255) != 0) return fail(LBM_EWORKSPACE, "workspace must be 256-byte aligned");
  lbm_ctx* c = new lbm_ctx();
  c->cfg = *cfg;
  c->L = L;
  c->ws = (char*)ws;
  c->stream = (hipStream_t)stream;
  if (c->f64()) fill_args<double>(c->a64, cfg, L, c->ws);
  else fill_args<float>(c->a32, cfg, L, c->ws);
  // selection state, counters and divergence flag
  SelState s0;
  init_select_state(&s0, c->f64());
  hipError_t e = hipMemcpyAsync(c->ws + L.off_sel, &s0, sizeof(SelState), hipMemcpyHostToDevice, c->stream);
  double coef64[27];
  float coef32[27];
  if (e == hipSuccess && L.off_nl) {
    for (int k = 0; k < 27; ++k) { coef64[k] = cfg->nl_coef[k]; coef32[k] = (float)cfg->nl_coef[k]; }
    e = hipMemcpyAsync(c->ws + L.off_nl, c->f64() ? (const void*)coef64 : (const void*)coef32,
                       27 * (c->f64() ? 8 : 4), hipMemcpyHostToDevice, c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->ws + L.off_cnt, 0, (size_t)kCntSlots * CNT_N * 8, c->stream);
  if (e == hipSuccess && L.off_ens) e = hipMemsetAsync(c->ws + L.off_ens, 0, sizeof(EnsState), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->ws + L.off_div, 0xff, sizeof(long long), c->stream);
  if (e == hipSuccess && L.off_f64cnt)
    e = hipMemsetAsync(c->ws + L.off_f64cnt, 0, 2 * sizeof(unsigned int), c->stream);
  if (e == hipSuccess && (cfg->limiters & LBM_LIM_EHRENFEST)) {
    e = hipMemsetAsync(c->ws + L.off_hist, 0, (size_t)kHistWords * 4, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + L.off_coarse, 0, kCoarse * 4, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + L.off_wcount, 0, (size_t)(L.cap / 64) * 4, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + L.off_ccount, 0, (size_t)kCountSlots * kCountStride * 8, c->stream);
  }
  // Capture the graphs that lbm_step replays (kGraphSteps steps from either
  // lattice) now, so that no later lbm_step call pays for a capture.
  for (int l = 0; l < 2 && e == hipSuccess; ++l) {
    c->cur = l;
    e = capture_graph(c);
  }
  c->cur = 0;
  if (e != hipSuccess) { delete c; return hip_fail(e, "lbm_init"); }
  *out = c;
  return LBM_OK;
}

static lbm_status reset_rollout(lbm_ctx* c) {
  c->steps = 0;
  c->recorded = false;
  hipError_t e = hipMemsetAsync(c->ws + c->L.off_div, 0xff, sizeof(long long), c->stream);
  if (e == hipSuccess)
    e = hipMemsetAsync(c->ws + c->L.off_sel + offsetof(SelState, tape_t), 0, sizeof(long long),
                       c->stream);
  if (e != hipSuccess) return hip_fail(e, "reset");
  if (c->cfg.limiters & LBM_LIM_EHRENFEST) {
    const void* args;
    if (c->f64()) { c->a64.src = c->lat(c->cur); c->a64.dst = c->lat(1 - c->cur); args = &c->a64; }
    else { c->a32.src = c->lat(c->cur); c->a32.dst = c->lat(1 - c->cur); args = &c->a32; }
    SelectArgs sa = select_args(c, args);
    e = launch_select_calibrate(sa, c->stream);
    if (e != hipSuccess) return hip_fail(e, "selection calibration");
  }
  if (c->cfg.checkpoint_every > 0) {
    e = adjoint_begin_record(c->L.adj, c->ws, c->lat(c->cur), c->L.lat_bytes, c->stream);
    if (e != hipSuccess) return hip_fail(e, "checkpoint");
    c->recorded = true;
  }
  return LBM_OK;
}

lbm_status lbm_set_equilibrium(lbm_ctx* c, const void* rho, const void* ux, const void* uy,
                               int dtype) {
  g_err.clear();
  if (!c || !rho || !ux) return fail(LBM_EINVAL, "NULL argument");
  if (dtype != LBM_F64 && dtype != LBM_F32) return fail(LBM_EINVAL, "dtype must be LBM_F64 or LBM_F32");
  if (c->L.Q == 27) return fail(LBM_EUNSUPPORTED, "D3Q27: use lbm_set_equilibrium3d");
  if (c->L.Q == 9 && !uy) return fail(LBM_EINVAL, "uy is required for D2Q9");
  const int kind = c->cfg.collision == LBM_ELBM ? LBM_EQ_ENTROPIC : c->cfg.equilibrium;
  hipError_t e = launch_set_eq(c->cfg.storage, c->L.Q, rho, ux, uy, nullptr, dtype == LBM_F64,
                               c->lat(c->cur), c->L.qs, c->cfg.nx, c->L.rows, c->L.pitch, kind,
                               c->cfg.rho0, c->stream);
  if (e != hipSuccess) return hip_fail(e, "lbm_set_equilibrium");
  return reset_rollout(c);
}

lbm_status lbm_set_equilibrium3d(lbm_ctx* c, const void* rho, const void* ux, const void* uy,
                                 const void* uz, int dtype) {
  g_err.clear();
  if (!c || !rho || !ux || !uy || !uz) return fail(LBM_EINVAL, "NULL argument");
  if (dtype != LBM_F64 && dtype != LBM_F32) return fail(LBM_EINVAL, "dtype must be LBM_F64 or LBM_F32");
  if (c->L.Q != 27) return fail(LBM_EINVAL, "lbm_set_equilibrium3d needs a D3Q27 lattice");
  hipError_t e = launch_set_eq(c->cfg.storage, 27, rho, ux, uy, uz, dtype == LBM_F64,
                               c->lat(c->cur), c->L.qs, c->cfg.nx, c->L.rows, c->L.pitch,
                               c->cfg.equilibrium, c->cfg.rho0, c->stream);
  if (e != hipSuccess) return hip_fail(e, "lbm_set_equilibrium3d");
  return reset_rollout(c);
}

lbm_status lbm_set_populations(lbm_ctx* c, const void* f, int dtype) {
  g_err.clear();
  if (!c || !f) return fail(LBM_EINVAL, "NULL argument");
  if (dtype != LBM_F64 && dtype != LBM_F32) return fail(LBM_EINVAL, "dtype must be LBM_F64 or LBM_F32");
  hipError_t e = launch_set_pop(c->cfg.storage, c->L.Q, f, dtype == LBM_F64, c->lat(c->cur),
                                c->L.qs, c->cfg.nx, c->L.rows, c->L.pitch, c->cfg.rho0, c->stream);
  if (e != hipSuccess) return hip_fail(e, "lbm_set_populations");
  return reset_rollout(c);
}

lbm_status lbm_get_populations(lbm_ctx* c, void* f, int dtype) {
  g_err.clear();
  if (!c || !f) return fail(LBM_EINVAL, "NULL argument");
  if (dtype != LBM_F64 && dtype != LBM_F32) return fail(LBM_EINVAL, "dtype must be LBM_F64 or LBM_F32");
  hipError_t e = launch_get_pop(c->cfg.storage, c->L.Q, f, dtype == LBM_F64, c->lat(c->cur),
                                c->L.qs, c->cfg.nx, c->L.rows, c->L.pitch, c->cfg.rho0, c->stream);
  if (e != hipSuccess) return hip_fail(e, "lbm_get_populations");
  return LBM_OK;
}

lbm_status lbm_set_omega(lbm_ctx* c, const void* omega, int dtype) {
  g_err.clear();
  if (!c || !omega) return fail(LBM_EINVAL, "NULL argument");
  if (!c->cfg.omega_field) return fail(LBM_EINVAL, "config has omega_field = 0");
  if (dtype != LBM_F64 && dtype != LBM_F32) return fail(LBM_EINVAL, "dtype must be LBM_F64 or LBM_F32");
  const size_t rb = c->f64() ? 8 : 4;
  const size_t eb = dtype == LBM_F64 ? 8 : 4;
  char* dst = c->ws + c->L.off_omega;
  if (rb == eb) {
    hipError_t e = hipMemcpy2DAsync(dst, c->L.pitch * rb, omega, c->cfg.nx * eb, c->cfg.nx * eb,
                                    c->cfg.ny, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(e, "lbm_set_omega");
    return LBM_OK;
  }
  hipError_t e = launch_convert_field(omega, dtype == LBM_F64, dst, c->f64(), c->cfg.nx, c->cfg.ny,
                                      c->L.pitch, c->stream);
  if (e != hipSuccess) return hip_fail(e, "lbm_set_omega");
  return LBM_OK;
}

static hipError_t one_step(lbm_ctx* c, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
  const int src = c->cur, dst = 1 - c->cur;
  const bool med = (c->cfg.limiters & LBM_LIM_MEDIAN) != 0;
  const void* args;
  if (c->f64()) { c->a64.src = c->lat(src); c->a64.dst = c->lat(dst); args = &c->a64; }
  else { c->a32.src = c->lat(src); c->a32.dst = c->lat(dst); args = &c->a32; }
  hipError_t e = hipSuccess;
  if (c->cfg.ens_limiter != LBM_ENS_NONE)
    e = launch_ensemble(c->cfg.storage, c->L.Q, args, c->cfg.ens_delta0, c->cfg.ens_delta,
                        c->stream);
  if (e == hipSuccess) {
    if (c->L.Q == 27) e = launch_step3(c->cfg.storage, med, args, c->stream, ev0, ev1);
    else if (c->cfg.nl_filter) e = launch_step_nl(c->cfg.storage, c->L.Q, c->cfg.collision, args, c->stream, ev0, ev1);
    else e = launch_step(c->cfg.storage, c->L.Q, c->cfg.collision, med, args, c->stream, ev0, ev1);
  }
  if (e != hipSuccess) return e;
  if (c->cfg.limiters & LBM_LIM_EHRENFEST) {
    SelectArgs sa = select_args(c, args);
    e = launch_select(sa, c->stream);
    if (e != hipSuccess) return e;
  }
  c->cur = dst;
  c->steps += 1;
  return hipSuccess;
}

static SelectArgs select_args(lbm_ctx* c, const void* args) {
    SelectArgs sa;
    sa.storage = c->cfg.storage; sa.Q = c->L.Q; sa.coll = c->cfg.collision; sa.step_args = args;
    sa.k = c->L.k; sa.n_sites = c->L.n_sites;
    sa.selected = (int32_t*)(c->ws + c->L.off_selected);
    sa.segsel = (int32_t*)(c->ws + c->L.off_stage);
    sa.blist = (uint32_t*)(c->ws + c->L.off_blist);
    sa.bcap = c->L.bcap;
    sa.coarse = (unsigned int*)(c->ws + c->L.off_coarse);
    sa.n_sel_out = nullptr;
    // recording: the selection kernels index the tape by the device's step
    // count since the rollout began
    sa.tape_sel = adjoint_selected_slot(c->L.adj, c->ws, 0, nullptr);
    sa.tape_cnt = adjoint_count_slot(c->L.adj, c->ws, 0);
    sa.tape_len = sa.tape_sel ? c->L.adj.max_steps : 0;
    return sa;
}

// Capture kGraphSteps steps from lattice c->cur on the library's own stream
// (the caller's may be the legacy default stream, which cannot be
// captured); the host-side step state is restored afterwards.
static hipError_t capture_graph(lbm_ctx* c) {
  hipError_t e = hipSuccess;
  if (!c->cap_stream) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  const hipStream_t user = c->stream;
  const int cur0 = c->cur;
  const long long steps0 = c->steps;
  c->stream = c->cap_stream;
  hipGraph_t g = nullptr;
  e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    for (int s = 0; s < kGraphSteps && e == hipSuccess; ++s) e = one_step(c);
    const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
    if (e == hipSuccess) e = e2;
  }
  c->stream = user;
  c->cur = cur0;
  c->steps = steps0;
  if (e == hipSuccess)
    e = hipGraphInstantiate(&c->graph[c->L.adj.on ? 1 : 0][cur0], g, nullptr, nullptr, 0);
  if (g) hipGraphDestroy(g);
  return e;
}

// Replay kGraphSteps steps from the captured graph (capturing it first).
static lbm_status replay_graph(lbm_ctx* c) {
  hipGraphExec_t& g = c->graph[c->L.adj.on ? 1 : 0][c->cur];
  if (!g) {
    const hipError_t e = capture_graph(c);
    if (e != hipSuccess) return hip_fail(e, "graph capture");
  }
  const hipError_t e = hipGraphLaunch(g, c->stream);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  c->steps += kGraphSteps;
  return LBM_OK;
}

// The periodic divergence check (FP64 reduction) after a step.
static hipError_t check_now(lbm_ctx* c) {
  return launch_stats(c->cfg.storage, c->L.Q, c->lat(c->cur), c->L.qs, c->cfg.nx, c->L.rows,
                      c->L.pitch, c->cfg.bc == LBM_BC_PERIODIC, c->cfg.rho0,
                      (double*)(c->ws + c->L.off_partial),
                      (double*)(c->ws + c->L.off_stats), (long long*)(c->ws + c->L.off_div),
                      c->steps, c->stream);
}

static lbm_status run_steps(lbm_ctx* c, long long n, hipEvent_t* ev) {
  // Launch-bound lattices gain most: whole groups of kGraphSteps steps
  // replay a captured graph (not with events, which time each step).  The
  // work that falls between steps stays outside the graph, and a replay
  // never spans it: the checkpoint copies and the end of the tape of a
  // recorded rollout (the tape itself is indexed on the device), and the
  // periodic divergence checks.
  const bool rec = c->recorded && c->L.adj.on;
  const bool graphs = !ev && (rec || !c->L.adj.on);
  const long long ci = c->cfg.check_interval;
  long long eager = 0;   // eager steps of this call (index into ev)
  while (n > 0) {
    bool fits = graphs && n >= kGraphSteps;
    if (fits && rec) {
      const long long K = c->L.adj.K;
      fits = c->steps + kGraphSteps <= c->cfg.max_steps && K - c->steps % K >= kGraphSteps;
    }
    if (fits && ci > 0) fits = ci - c->steps % ci >= kGraphSteps;
    if (fits) {
      const lbm_status st = replay_graph(c);
      if (st != LBM_OK) return st;
      n -= kGraphSteps;
      if (rec) {
        const hipError_t e = adjoint_after_step(c->L.adj, c->ws, c->steps, c->lat(c->cur),
                                                c->L.lat_bytes, c->stream);
        if (e != hipSuccess) return hip_fail(e, "checkpoint");
      }
      if (ci > 0 && c->steps % ci == 0) {
        const hipError_t e = check_now(c);
        if (e != hipSuccess) return hip_fail(e, "check");
      }
      continue;
    }
    if (c->recorded && c->steps >= c->cfg.max_steps)
      return fail(LBM_ESTATE, "rollout longer than cfg.max_steps; lbm_backward could not cover it");
    hipError_t e = ev ? one_step(c, ev[2 * eager], ev[2 * eager + 1]) : one_step(c);
    if (e != hipSuccess) return hip_fail(e, "lbm_step");
    ++eager;
    --n;
    if (c->recorded) {
      e = adjoint_after_step(c->L.adj, c->ws, c->steps, c->lat(c->cur), c->L.lat_bytes, c->stream);
      if (e != hipSuccess) return hip_fail(e, "checkpoint");
    }
    if (ci > 0 && c->steps % ci == 0) {
      e = check_now(c);
      if (e != hipSuccess) return hip_fail(e, "check");
    }
  }
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, long long n) {
  g_err.clear();
  if (!c) return fail(LBM_EINVAL, "ctx is NULL");
  if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
  return run_steps(c, n, nullptr);
}

lbm_status lbm_profile_step(lbm_ctx* c, long long n, double out[2]) {
  g_err.clear();
  if (!c || !out) return fail(LBM_EINVAL, "NULL argument");
  if (n < 1) return fail(LBM_EINVAL, "n must be >= 1");
  std::vector<hipEvent_t> ev((size_t)(2 * n + 1), nullptr);
  hipError_t e = hipSuccess;
  for (auto& x : ev) {
    e = hipEventCreate(&x);
    if (e != hipSuccess) break;
  }
  lbm_status st = LBM_OK;
  if (e == hipSuccess) {
    st = run_steps(c, n, ev.data());
    if (st == LBM_OK) {
      e = hipEventRecord(ev[2 * n], c->stream);
      if (e == hipSuccess) e = hipEventSynchronize(ev[2 * n]);
    }
  }
  double kern = 0.0, total = 0.0;
  if (e == hipSuccess && st == LBM_OK) {
    for (long long s = 0; s < n && e == hipSuccess; ++s) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, ev[2 * s], ev[2 * s + 1]);
      kern += ms;
    }
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[2 * n]);
    total = ms;
  }
  for (auto& x : ev)
    if (x) hipEventDestroy(x);
  if (st != LBM_OK) return st;
  if (e != hipSuccess) return hip_fail(e, "lbm_profile_step");
  out[0] = kern;
  out[1] = total;
  return LBM_OK;
}

lbm_status lbm_moments(lbm_ctx* c, void* rho, void* ux, void* uy, int dtype) {
  g_err.clear();
  if (!c || !rho || !ux) return fail(LBM_EINVAL, "NULL argument");
  if (dtype != LBM_F64 && dtype != LBM_F32) return fail(LBM_EINVAL, "dtype must be LBM_F64 or LBM_F32");
  if (c->L.Q == 27) return fail(LBM_EUNSUPPORTED, "D3Q27: read the populations (lbm_get_populations)");
  hipError_t e = launch_moments(c->cfg.storage, c->L.Q, c->lat(c->cur), c->L.qs, c->cfg.nx,
                                c->cfg.ny, c->L.pitch, c->cfg.rho0, rho, ux, uy,
                                dtype == LBM_F64, c->stream);
  if (e != hipSuccess) return hip_fail(e, "lbm_moments");
  return LBM_OK;
}

lbm_status lbm_stats_get(lbm_ctx* c, lbm_stats* out) {
  g_err.clear();
  if (!c || !out) return fail(LBM_EINVAL, "NULL argument");
  hipError_t e = launch_stats(c->cfg.storage, c->L.Q, c->lat(c->cur), c->L.qs, c->cfg.nx,
                              c->L.rows, c->L.pitch, c->cfg.bc == LBM_BC_PERIODIC, c->cfg.rho0,
                              (double*)(c->ws + c->L.off_partial),
                              (double*)(c->ws + c->L.off_stats),
                              (long long*)(c->ws + c->L.off_div), c->steps, c->stream);
  if (e != hipSuccess) return hip_fail(e, "lbm_stats");
  double st[8];
  long long div = -1;
  SelState sel;
  std::memset(&sel, 0, sizeof(sel));
  e = hipMemcpyAsync(st, c->ws + c->L.off_stats, 8 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&div, c->ws + c->L.off_div, sizeof(div), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&sel, c->ws + c->L.off_sel, sizeof(sel), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "lbm_stats");
  std::memset(out, 0, sizeof(*out));
  out->mass = st[0]; out->mom_x = st[1]; out->mom_y = st[2]; out->entropy = st[3];
  out->min_rho = st[4]; out->nonfinite = st[5] != 0.0;
  if (c->L.Q == 27) out->mom_z = st[6];   // the z momentum takes the enstrophy slots in 3D
  else out->enstrophy = st[7] > 0.0 ? st[6] / st[7] : 0.0;
  out->steps = c->steps;
  out->diverged_step = div;
  out->n_selected = sel.n_sel;
  out->select_fallbacks = (long long)sel.fallbacks;
  out->select_overflow = (long long)sel.overflows;
  out->select_candidates = (long long)sel.cand_total;
  if (c->cfg.ens_limiter != LBM_ENS_NONE) {
    EnsState es;
    e = hipMemcpy(&es, c->ws + c->L.off_ens, sizeof(es), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "lbm_stats");
    const bool thr = c->cfg.ens_limiter == LBM_ENS_THRESHOLD ||
                     c->cfg.ens_limiter == LBM_ENS_DOUBLE_MONOTONE;
    out->ens_threshold = thr ? es.threshold : __builtin_huge_val();
    double sdS = 0.0, n = 0.0;
    for (int k = 0; k < kEnsSlots; ++k) {
      out->lbgk_production += es.step_acc[k][0];
      out->limiter_production += es.step_acc[k][1];
      sdS += es.step_acc[k][2];
      n += es.step_acc[k][3];
    }
    out->ens_mean = n > 0.0 ? sdS / n : 0.0;
  }
  if (div >= 0) return fail(LBM_EDIVERGED, "non-finite value or rho <= 0 found at step " + std::to_string(div));
  if (sel.overflows) return fail(LBM_ESELECT, "Ehrenfest boundary list overflowed: more than 2^20 sites tie within one histogram bucket");
  return LBM_OK;
}

lbm_status lbm_counters(lbm_ctx* c, unsigned long long* out, int n) {
  g_err.clear();
  if (!c || !out || n < 1) return fail(LBM_EINVAL, "bad argument");
  std::vector<unsigned long long> all((size_t)kCntSlots * CNT_N);
  hipError_t e = hipMemcpyAsync(all.data(), c->ws + c->L.off_cnt, all.size() * 8,
                                hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "lbm_counters");
  for (int k = 0; k < n; ++k) {
    unsigned long long sum = 0;
    if (k < CNT_N)
      for (int slot = 0; slot < kCntSlots; ++slot) sum += all[(size_t)slot * CNT_N + k];
    out[k] = sum;
  }
  return LBM_OK;
}

lbm_status lbm_selected(lbm_ctx* c, long long* idx, long long cap, long long* count) {
  g_err.clear();
  if (!c || !count) return fail(LBM_EINVAL, "NULL argument");
  *count = 0;
  if (!(c->cfg.limiters & LBM_LIM_EHRENFEST)) return LBM_OK;
  SelState sel;
  hipError_t e = hipMemcpyAsync(&sel, c->ws + c->L.off_sel, sizeof(sel), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "lbm_selected");
  const long long n = sel.n_sel;
  *count = n;
  if (!idx || n == 0) return LBM_OK;
  std::vector<int32_t> tmp((size_t)n);
  const int32_t* src = adjoint_selected_slot(c->L.adj, c->ws, c->steps - 1,
                                             (int32_t*)(c->ws + c->L.off_selected));
  e = hipMemcpy(tmp.data(), src, (size_t)n * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "lbm_selected");
  std::sort(tmp.begin(), tmp.end());
  for (long long i = 0; i < n && i < cap; ++i) idx[i] = tmp[(size_t)i];
  return LBM_OK;
}

static lbm_status backward_impl(lbm_ctx* c, const void* dL_dfT, void* dL_df0, void* dL_domega,
                                int dtype, std::vector<hipEvent_t>* ev);

lbm_status lbm_backward(lbm_ctx* c, const void* dL_dfT, void* dL_df0, void* dL_domega, int dtype) {
  g_err.clear();
  return backward_impl(c, dL_dfT, dL_df0, dL_domega, dtype, nullptr);
}

lbm_status lbm_profile_backward(lbm_ctx* c, const void* dL_dfT, void* dL_df0, void* dL_domega,
                                int dtype, double out[2]) {
  g_err.clear();
  if (!c || !out) return fail(LBM_EINVAL, "NULL argument");
  const long long T = c->steps;
  std::vector<hipEvent_t> ev((size_t)(2 * T + 2), nullptr);
  hipError_t e = hipSuccess;
  for (auto& x : ev) {
    e = hipEventCreate(&x);
    if (e != hipSuccess) break;
  }
  lbm_status st = e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_profile_backward");
  if (st == LBM_OK) {
    e = hipEventRecord(ev[2 * T], c->stream);
    st = e == hipSuccess ? backward_impl(c, dL_dfT, dL_df0, dL_domega, dtype, &ev)
                         : hip_fail(e, "lbm_profile_backward");
  }
  if (st == LBM_OK) {
    e = hipEventRecord(ev[2 * T + 1], c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev[2 * T + 1]);
    double kern = 0.0;
    for (long long s = 0; s < T && e == hipSuccess; ++s) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, ev[2 * s], ev[2 * s + 1]);
      kern += ms;
    }
    float tot = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&tot, ev[2 * T], ev[2 * T + 1]);
    if (e != hipSuccess) st = hip_fail(e, "lbm_profile_backward");
    out[0] = kern;
    out[1] = tot;
  }
  for (auto& x : ev)
    if (x) hipEventDestroy(x);
  return st;
}

}  // extern "C"

static lbm_status backward_impl(lbm_ctx* c, const void* dL_dfT, void* dL_df0, void* dL_domega,
                                int dtype, std::vector<hipEvent_t>* ev) {
  if (!c || !dL_dfT || !dL_df0) return fail(LBM_EINVAL, "NULL argument");
  if (dtype != LBM_F64 && dtype != LBM_F32) return fail(LBM_EINVAL, "dtype must be LBM_F64 or LBM_F32");
  if (c->cfg.checkpoint_every <= 0 || !c->recorded)
    return fail(LBM_ESTATE, "no recorded rollout (set checkpoint_every > 0 and call lbm_set_* first)");
  const AdjointLayout& A = c->L.adj;
  const long long T = c->steps;
  const int Q = c->L.Q, nx = c->cfg.nx, ny = c->cfg.ny, pitch = c->L.pitch;
  const long long qs = c->L.qs;
  const bool r64 = c->f64();
  const bool med = (c->cfg.limiters & LBM_LIM_MEDIAN) != 0;
  const int din = dtype == LBM_F64;
  hipStream_t st = c->stream;
  char* ws = c->ws;
  void* lam[2] = {ws + A.off_lam[0], ws + A.off_lam[1]};
  void* gom = ws + A.off_gom;
  unsigned char* mask = A.k > 0 ? (unsigned char*)(ws + A.off_mask) : nullptr;
  MedianAdjoint mad;
  if (A.median) {
    mad.gs = ws + A.off_med_gs;
    mad.h = ws + A.off_med_h;
    mad.am = (unsigned char*)(ws + A.off_med_am);
  }
  auto seg = [&](long long j) { return (void*)(ws + A.off_seg + (size_t)j * align256(c->L.lat_bytes)); };
  auto ckpt = [&](long long s) { return (const void*)(ws + A.off_ckpt + (size_t)s * align256(c->L.lat_bytes)); };
  // Step arguments of the recompute: no selection, no counters.
  StepArgs<double> a64 = c->a64;
  StepArgs<float> a32 = c->a32;
  a64.ehrenfest = a32.ehrenfest = 0;
  a64.count_events = a32.count_events = 0;
  auto args_for = [&](const void* src, void* dst, void* alpha = nullptr,
                      unsigned char* branch = nullptr) -> const void* {
    if (r64) {
      a64.src = src; a64.dst = dst; a64.alpha_out = (double*)alpha; a64.branch_out = branch;
      return &a64;
    }
    a32.src = src; a32.dst = dst; a32.alpha_out = (float*)alpha; a32.branch_out = branch;
    return &a32;
  };
  // ELBM: alpha and branch of step t0 + j of the segment being reversed
  const size_t fbytes = align256((size_t)qs * (r64 ? 8 : 4)), bbytes = align256((size_t)qs);
  auto alpha_slot = [&](long long j) -> void* {
    return A.store_alpha ? (void*)(ws + A.off_alpha + (size_t)j * fbytes) : nullptr;
  };
  auto branch_slot = [&](long long j) -> unsigned char* {
    return A.store_alpha ? (unsigned char*)(ws + A.off_branch + (size_t)j * bbytes) : nullptr;
  };
  hipError_t e = launch_to_pitch(dL_dfT, din, lam[0], r64, Q, nx, ny, pitch, qs, st);
  if (e == hipSuccess) e = hipMemsetAsync(gom, 0, (size_t)qs * (r64 ? 8 : 4), st);
  if (e == hipSuccess && mask) e = hipMemsetAsync(mask, 0, (size_t)nx * ny, st);
  int cur = 0;
  for (long long s = T > 0 ? (T - 1) / A.K : -1; s >= 0 && e == hipSuccess; --s) {
    const long long t0 = s * A.K, t1 = std::min(T, t0 + A.K);
    // states g_t0 .. g_{t1-1} of the segment, from its checkpoint (ELBM: the
    // last step too, into a spare slot, for its alpha)
    e = hipMemcpyAsync(seg(0), ckpt(s), c->L.lat_bytes, hipMemcpyDeviceToDevice, st);
    const long long t_end = A.store_alpha ? t1 : t1 - 1;
    for (long long t = t0; t < t_end && e == hipSuccess; ++t) {
      const bool last = t + 1 == t1;
      const void* args = args_for(seg(t - t0), last ? seg(A.K) : seg(t + 1 - t0),
                                  alpha_slot(t - t0), branch_slot(t - t0));
      e = launch_step(c->cfg.storage, Q, c->cfg.collision, med, args, st);
      if (e == hipSuccess && A.k > 0 && !last)
        e = launch_tape_fix(c->cfg.storage, Q, args, adjoint_selected_slot(A, ws, t, nullptr),
                            adjoint_count_slot(A, ws, t), A.k, st);
    }
    // reverse sweep over the segment
    for (long long t = t1 - 1; t >= t0 && e == hipSuccess; --t) {
      const int32_t* list = A.k > 0 ? adjoint_selected_slot(A, ws, t, nullptr) : nullptr;
      const long long* cnt = A.k > 0 ? adjoint_count_slot(A, ws, t) : nullptr;
      // short lists go to the adjoint kernel itself; long ones through the mask
      const bool short_list = list && A.k <= kAdjListMax;
      if (mask && !short_list) e = launch_mark(mask, list, cnt, A.k, 1, st);
      const void* args = args_for(seg(t - t0), nullptr);
      if (e == hipSuccess)
        e = launch_adjoint(c->cfg.storage, Q, c->cfg.collision, args, lam[cur], lam[1 - cur],
                           dL_domega ? gom : nullptr, short_list ? nullptr : mask,
                           alpha_slot(t - t0), branch_slot(t - t0),
                           short_list ? list : nullptr, cnt, A.k, mad, st,
                           ev ? (*ev)[2 * t] : nullptr, ev ? (*ev)[2 * t + 1] : nullptr);
      if (e == hipSuccess && mask && !short_list) e = launch_mark(mask, list, cnt, A.k, 0, st);
      cur = 1 - cur;
    }
  }
  if (e == hipSuccess) e = launch_from_pitch(lam[cur], r64, dL_df0, din, Q, nx, ny, pitch, qs, st);
  if (e == hipSuccess && dL_domega)
    e = launch_from_pitch(gom, r64, dL_domega, din, 1, nx, ny, pitch, qs, st);
  if (e != hipSuccess) return hip_fail(e, "lbm_backward");
  return LBM_OK;
}

// ---------------------------------------------------------------------------
// One step without any allocation (lbm_step_noalloc).  Every buffer besides
// the caller's two lattices lives in `scratch`, a static device array that
// each device holds from the library's load until the process ends.  In
// host code `scratch` names a host-side stand-in, not device memory: its
// device address comes from hipGetSymbolAddress, looked up once per device
// (with that device current) and kept in g_scratch_ptr; only that address
// is ever passed to kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[LBM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Everything a step reads before writing it, cleared in the scratch array
// with a kernel (no memset nodes when the caller captures the call): the
// selection state (its floor back at the threshold), the histograms, the
// candidate counters and region counts, the limiter counters and the FP64
// site list's count.
struct ScratchReset {
  SelState sel;
  SelState* sel_dst;
  unsigned long long* counters;   // kCntSlots * CNT_N
  unsigned int* hist;             // kHistWords
  unsigned int* coarse;           // kCoarse
  unsigned long long* ccount;     // kCountSlots * kCountStride
  uint32_t* wcount;               // n_wcount
  long long n_wcount;
  unsigned int* f64_count;        // 2
};

__global__ void k_scratch_reset(const ScratchReset r) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  if (t == 0) *r.sel_dst = r.sel;
  for (long long i = t; i < (long long)kCntSlots * CNT_N; i += stride) r.counters[i] = 0;
  if (r.hist) {
    for (long long i = t; i < kHistWords; i += stride) r.hist[i] = 0;
    for (long long i = t; i < kCoarse; i += stride) r.coarse[i] = 0;
    for (long long i = t; i < (long long)kCountSlots * kCountStride; i += stride) r.ccount[i] = 0;
    for (long long i = t; i < r.n_wcount; i += stride) r.wcount[i] = 0;
  }
  if (r.f64_count && t < 2) r.f64_count[t] = 0;
}

}  // namespace

extern "C" lbm_status lbm_step_noalloc(const lbm_config* cfg, const void* f_src, void* f_dst,
                                       void* stream) {
  g_err.clear();
  std::string why;
  if (!validate(cfg, why)) return fail(LBM_EINVAL, why);
  if (!f_src || !f_dst || f_src == f_dst)
    return fail(LBM_EINVAL, "f_src and f_dst must be distinct device buffers");
  if (cfg->checkpoint_every != 0 || cfg->omega_field != 0)
    return fail(LBM_EINVAL, "lbm_step_noalloc needs checkpoint_every = 0 and omega_field = 0");
  if (cfg->lattice == LBM_D3Q27 || cfg->nl_filter)
    return fail(LBM_EUNSUPPORTED, "lbm_step_noalloc covers the D1Q3 and D2Q9 steps without the nonlocal filter");
  const Layout L = make_layout(cfg, false);
  if (L.total > (size_t)LBM_NOALLOC_SCRATCH_BYTES)
    return fail(LBM_EWORKSPACE, "lbm_step_noalloc: this configuration needs " +
                                    std::to_string(L.total) + " bytes of scratch, above the " +
                                    std::to_string((long long)LBM_NOALLOC_SCRATCH_BYTES) +
                                    "-byte static array (use lbm_init with a workspace)");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "lbm_step_noalloc");
  if (dev < 0 || dev >= kMaxDevices) return fail(LBM_EINVAL, "device ordinal out of range");
  void* base = nullptr;
  e = scratch_address(dev, &base);
  if (e != hipSuccess) return hip_fail(e, "lbm_step_noalloc: scratch address");
  char* ws = (char*)base;
  const hipStream_t st = (hipStream_t)stream;
  const bool f64 = cfg->storage == LBM_F64;
  StepArgs<double> a64;
  StepArgs<float> a32;
  const void* args;
  if (f64) {
    fill_args<double>(a64, cfg, L, ws);
    a64.src = f_src;
    a64.dst = f_dst;
    args = &a64;
  } else {
    fill_args<float>(a32, cfg, L, ws);
    a32.src = f_src;
    a32.dst = f_dst;
    args = &a32;
  }
  const bool ehr = (cfg->limiters & LBM_LIM_EHRENFEST) != 0;
  ScratchReset r;
  std::memset((void*)&r, 0, sizeof(r));
  init_select_state(&r.sel, f64);
  r.sel_dst = (SelState*)(ws + L.off_sel);
  r.counters = (unsigned long long*)(ws + L.off_cnt);
  if (ehr) {
    r.hist = (unsigned int*)(ws + L.off_hist);
    r.coarse = (unsigned int*)(ws + L.off_coarse);
    r.ccount = (unsigned long long*)(ws + L.off_ccount);
    r.wcount = (uint32_t*)(ws + L.off_wcount);
    r.n_wcount = L.cap / 64;
  }
  r.f64_count = L.off_f64cnt ? (unsigned int*)(ws + L.off_f64cnt) : nullptr;
  hipLaunchKernelGGL(k_scratch_reset, dim3(64), dim3(256), 0, st, r);
  e = hipGetLastError();
  if (e == hipSuccess)
    e = launch_step(cfg->storage, L.Q, cfg->collision, (cfg->limiters & LBM_LIM_MEDIAN) != 0,
                    args, st);
  if (e == hipSuccess && ehr) {
    SelectArgs sa;
    sa.storage = cfg->storage; sa.Q = L.Q; sa.coll = cfg->collision; sa.step_args = args;
    sa.k = L.k; sa.n_sites = L.n_sites;
    sa.selected = (int32_t*)(ws + L.off_selected);
    sa.segsel = (int32_t*)(ws + L.off_stage);
    sa.blist = (uint32_t*)(ws + L.off_blist);
    sa.bcap = L.bcap;
    sa.coarse = (unsigned int*)(ws + L.off_coarse);
    sa.n_sel_out = nullptr;
    sa.tape_sel = nullptr;
    sa.tape_cnt = nullptr;
    sa.tape_len = 0;
    e = launch_select(sa, st);
  }
  if (e != hipSuccess) return hip_fail(e, "lbm_step_noalloc");
  return LBM_OK;
}

extern "C" {

void lbm_destroy(lbm_ctx* c) { delete c; }

const char* lbm_last_error(void) { return g_err.c_str(); }

}  // extern "C"
