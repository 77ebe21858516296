// Per-site preparation shared by the step kernel, the median halo and the
// Ehrenfest selection rescans: pull-stream with boundaries, moments,
// equilibrium and nonequilibrium entropy.  One definition, so every caller
// sees bit-identical values for a site.
#pragma once

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

struct TileShape { int tx, ty; };
// Workgroup tile of 256 sites: whole 256-site row segments when rows are
// long enough, 64 x 4 blocks otherwise and for the median filter's LDS tile.
inline __host__ __device__ TileShape tile_shape(int Q, bool median, int nx) {
  if (Q == 3) return TileShape{256, 1};
  if (median) return TileShape{64, 4};
  return nx >= 256 ? TileShape{256, 1} : TileShape{64, 4};
}

// Velocity components of population i in tensor order: D1Q3 i = a + 1;
// D2Q9 i = 3 (b + 1) + (a + 1); D3Q27 i = 9 (c + 1) + 3 (b + 1) + (a + 1).
template <int Q> __device__ __forceinline__ int vx_of(int i) {
  return Q == 27 ? i % 3 - 1 : (Q == 9 ? kAx9[i] : i - 1);
}
template <int Q> __device__ __forceinline__ int vy_of(int i) {
  return Q == 27 ? (i / 3) % 3 - 1 : (Q == 9 ? kBy9[i] : 0);
}
template <int Q> __device__ __forceinline__ int vz_of(int i) { return Q == 27 ? i / 9 - 1 : 0; }
template <class R, int Q> __device__ __forceinline__ R wt(int i) {
  if constexpr (Q == 27) return w1<R>(vx_of<27>(i)) * w1<R>(vy_of<27>(i)) * w1<R>(vz_of<27>(i));
  return Q == 9 ? w9<R>(i) : w1<R>(i - 1);
}

// a / b from rb, a reciprocal of b within an ulp, corrected once by the
// exact residual a - q b: within a small fraction of an ulp of the
// correctly rounded quotient and, unlike a * rb, without a bias.  A biased
// velocity or equilibrium scale (a * rcp(rho), rho * fl(1/36)) is a
// systematic momentum error at every step; at omega near 2 it accumulates
// (the FP32 shear layer then lost most of its entropy production over 20k
// steps).
template <class R>
__device__ __forceinline__ R qdiv(R a, R b, R rb) {
  const R q = a * rb;
  return fma(fma(-q, b, a), rb, q);
}

// Equilibrium in the storage representation (unshifted f*_i, or the
// deviation f*_i - w_i rho0) from m0 (rho, or rho - rho0 when shifted):
// the product of the 1D equilibria (section 8), f*_ab = rho phi_a phi_b,
// evaluated as (rho/36) (c_a + dt_a)(c_b + dt_b) with integer weights.
// dx, dy: the deviations dt_a of u_x and u_y, for a caller that goes on to
// Delta S (site_dS_dev takes them instead of evaluating them again).
template <class R, int Q, bool SH>
__device__ __forceinline__ void equilibrium_v(R m0, R rho0, R ux, R uy, int kind, R feq[Q], R dx[3],
                                              R dy[3]) {
  eq_dev6<R>(ux, kind, dx);
  if constexpr (Q == 9) eq_dev6<R>(uy, kind, dy);
  const R rho = SH ? rho0 + m0 : m0;
  constexpr R S = Q == 9 ? R(36) : R(6);
  constexpr R iS = R(1) / S;
  const R rs = qdiv<R>(rho, S, iS);
  const R ms = qdiv<R>(m0, S, iS);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if constexpr (Q == 9) {
      const int a = vx_of<Q>(i), b = vy_of<Q>(i);
      const R ca = (R)c1(a), cb = (R)c1(b);
      const R da = dx[a + 1], db = dy[b + 1];
      feq[i] = SH ? ms * (ca * cb) + rs * (ca * db + da * cb + da * db)
                  : rs * ((ca + da) * (cb + db));
    } else {
      const R ca = (R)c1(i - 1);
      feq[i] = SH ? ms * ca + rs * dx[i] : rs * (ca + dx[i]);
    }
  }
}
template <class R, int Q, bool SH>
__device__ __forceinline__ void equilibrium_v(R m0, R rho0, R ux, R uy, int kind, R feq[Q]) {
  R dx[3], dy[3];
  equilibrium_v<R, Q, SH>(m0, rho0, ux, uy, kind, feq, dx, dy);
}

// Element `off` of an array whose base is the same for the whole wavefront:
// a 32-bit byte offset on a scalar base (one vector register per address).
template <class S>
__device__ __forceinline__ const S* at(const S* base, unsigned off) {
  return (const S*)((const char*)base + off * (unsigned)sizeof(S));
}
template <class S>
__device__ __forceinline__ S* at(S* base, unsigned off) {
  return (S*)((char*)base + off * (unsigned)sizeof(S));
}

// Pull on a periodic lattice, branch-free: three source rows and three source
// columns per site, each population at a scalar base plus a 32-bit offset.
// CACHED: cached loads (the caller reads some populations twice).
template <class S, int Q, bool CACHED = false>
__device__ __forceinline__ void pull_periodic(const S* __restrict__ src, long long qs, int pitch,
                                              int nx, int ny, int x, int y,
                                              typename StoreT<S>::R v[Q]) {
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const unsigned r[3] = {(unsigned)(yp * pitch), (unsigned)(y * pitch), (unsigned)(ym * pitch)};
  const unsigned c[3] = {(unsigned)xp, (unsigned)x, (unsigned)xm};   // a = -1, 0, +1
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const S* p = at(src + (long long)i * qs, r[vy_of<Q>(i) + 1] + c[vx_of<Q>(i) + 1]);
    v[i] = CACHED ? StoreT<S>::ldc(p) : StoreT<S>::ld(p);
  }
}

// Pull f_i(x) = f_i(x - v_i) with the boundary rules: periodic wrap, or
// halfway bounce-back f_i(x) = f_opp(i)(x) plus the moving-wall term when
// the source lies above the top row.  Branch-free: the plane and offset are
// selected and every population is one unconditional load (both candidate
// addresses lie inside the lattice), so that the nine loads issue together
// instead of each waiting at the join of an if/else.  CACHED: cached loads.
template <class S, int Q, bool CACHED = false>
__device__ __forceinline__ void pull(const S* __restrict__ src, long long qs, int pitch, int nx,
                                     int ny, int bc, int x, int y,
                                     const typename StoreT<S>::R* lid,
                                     typename StoreT<S>::R v[Q]) {
  using R = typename StoreT<S>::R;
  const bool wrap_x = bc == BC_PERIODIC || bc == BC_COUETTE, wrap_y = bc == BC_PERIODIC;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int sx = x - vx_of<Q>(i), sy = y - vy_of<Q>(i);
    if (wrap_x) sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
    if (wrap_y) sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
    const bool out = (sx < 0) | (sx >= nx) | (sy < 0) | (sy >= ny);
    const int plane = out ? Q - 1 - i : i;
    const unsigned off = out ? (unsigned)(y * pitch + x) : (unsigned)(sy * pitch + sx);
    const S* p = at(src + (long long)plane * qs, off);
    const R val = CACHED ? StoreT<S>::ldc(p) : StoreT<S>::ld(p);
    v[i] = sy >= ny ? val + lid[i] : val;
  }
}

// A node of the diffusive wall (the outer ring of the lattice).
template <class R>
__device__ __forceinline__ bool on_wall(const StepArgs<R>& A, int x, int y) {
  return A.bc == BC_DIFFUSIVE && (x == 0 || y == 0 || x == A.nx - 1 || y == A.ny - 1);
}

// Diffusive Maxwell wall (section 8, First Hopf bifurcation) at wall node
// (x, y) of the streamed state v (storage representation): with n the
// inward normal, the incoming directions are those with v_i . n > 0 (at a
// corner only v_i = n, which makes the rule bounce-back), gamma = sum of
// f_opp(i) over them / sum of f*_i(1, u_wall) over them, and every
// population whose source lies outside (v_i . n > 0 along either axis)
// becomes gamma f*_i(1, u_wall).  The lid row moves at (lid_u, 0); the other
// walls and the corners rest.
template <class S, int Q>
__device__ __forceinline__ void diffusive_wall(const StepArgs<typename StoreT<S>::R>& A, int x, int y,
                                            typename StoreT<S>::R v[Q]) {
  using R = typename StoreT<S>::R;
  constexpr bool SH = StoreT<S>::shifted;
  if constexpr (Q == 9) {
    const int n_x = x == 0 ? 1 : (x == A.nx - 1 ? -1 : 0);
    const int n_y = y == 0 ? 1 : (y == A.ny - 1 ? -1 : 0);
    const bool corner = n_x != 0 && n_y != 0;
    const R uw = (n_y == -1 && n_x == 0) ? A.lid_u : R(0);
    R fw[Q];
    equilibrium_v<R, Q, false>(R(1), A.rho0, uw, R(0), A.eq_kind, fw);
    R num = R(0), den = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int a = vx_of<Q>(i), b = vy_of<Q>(i);
      const bool in = corner ? (a == n_x && b == n_y) : (a * n_x + b * n_y > 0);
      if (in) {
        const int o = Q - 1 - i;
        num += v[o] + (SH ? wt<R, Q>(o) * A.rho0 : R(0));
        den += fw[i];
      }
    }
    const R gamma = num / den;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int a = vx_of<Q>(i), b = vy_of<Q>(i);
      if (a * n_x > 0 || b * n_y > 0) v[i] = gamma * fw[i] - (SH ? wt<R, Q>(i) * A.rho0 : R(0));
    }
  }
}

template <class R, int Q, bool SH>
__device__ __forceinline__ void moments_v(const R v[Q], R rho0, R& m0, R& ux, R& uy) {
  R s = R(0), jx = R(0), jy = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    s += v[i];
    if (vx_of<Q>(i) != 0) jx += vx_of<Q>(i) > 0 ? v[i] : -v[i];
    if (vy_of<Q>(i) != 0) jy += vy_of<Q>(i) > 0 ? v[i] : -v[i];
  }
  m0 = s;
  const R rho = SH ? rho0 + s : s;
  const R ir = rcp<R>(rho);
  ux = qdiv<R>(jx, rho, ir);
  uy = qdiv<R>(jy, rho, ir);
}

// Nonequilibrium entropy of a site (section 4, eq. DelS), sum_i f_i
// ln(f_i / f*_i), evaluated as sum_i f*_i h(x_i), x_i = (f_i - f*_i) / f*_i
// (same value because f and f* share rho).  With the product form of f*,
// 1/f*_ab = (S/rho) / ((c_a + dt_a)(c_b + dt_b)), so 1 + 2*3 reciprocals
// replace nine divisions.  +inf if some f_i < 0 or f*_i <= 0.
//
// Screening: for x >= -1/2, h(x) <= x^2/2 + max(-x, 0)^3/3 (for x >= 0 since
// h'' <= 1; for -1/2 <= x < 0 the series terms beyond the cubic one sum to
// less than the cubic term).  With y_i = -x_i = d_i / f*_i the bound on
// f*_i h(x_i) reads d_i y_i (1/2 + max(y_i, 0)/3) <= d_i y_i (1/2 +
// max(ymax, 0)/3) (d_i y_i = f*_i y_i^2 >= 0), so U = (sum_i d_i y_i)
// (1/2 + max(ymax, 0)/3) bounds Delta S from above.  When U < screen (and
// every y_i <= 1/2) the exact sum is skipped and U is returned: the caller
// only needs to know that Delta S is below `screen`.  screen = 0 always
// evaluates the exact sum.
// D3Q27 (uz): the same with three factors, 1/f*_abc = (216/rho) /
// ((c_a + dt_a)(c_b + dt_b)(c_c + dt_c)).
// site_dS_dev takes the equilibrium's deviations dt_a of u_x, u_y, u_z
// (eq_dev6) from the caller; site_dS_q evaluates them.  `screened`, when
// given, is set when the value returned is the bound U (below `screen`)
// rather than Delta S itself.
template <class R, int Q, bool SH>
__device__ __forceinline__ R site_dS_dev(const R v[Q], const R d[Q], R m0, R rho0, const R dx[3],
                                         const R dy[3], const R dz[3], R screen,
                                         bool* screened = nullptr) {
  R fx[3], fy[3], fz[3], rx[3], ry[3], rz[3];
  const R rho = SH ? rho0 + m0 : m0;
  constexpr R S = Q == 27 ? R(216) : (Q == 9 ? R(36) : R(6));
  const R irs = S * rcp<R>(rho);
  bool bad = rho <= R(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    fx[a] = (R)c1(a - 1) + dx[a];
    rx[a] = irs * rcp<R>(fx[a]);       // S / (rho (c_a + dt_a))
    bad |= fx[a] <= R(0);
    if constexpr (Q >= 9) {
      fy[a] = (R)c1(a - 1) + dy[a];
      ry[a] = rcp<R>(fy[a]);
      bad |= fy[a] <= R(0);
    }
    if constexpr (Q == 27) {
      fz[a] = (R)c1(a - 1) + dz[a];
      rz[a] = rcp<R>(fz[a]);
      bad |= fz[a] <= R(0);
    }
  }
  R y[Q];
  R sdy = R(0), ymax = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int a = vx_of<Q>(i) + 1, b = vy_of<Q>(i) + 1, cz = vz_of<Q>(i) + 1;
    const R sh = SH ? wt<R, Q>(i) * rho0 : R(0);
    // D3Q27 (whose callers take the exact sum everywhere) tests for negative
    // populations here; deferring the test costs that kernel spilled
    // registers
    if constexpr (Q == 27) bad |= (v[i] + sh) < R(0);
    const R inv = Q == 27 ? rx[a] * ry[b] * rz[cz] : (Q == 9 ? rx[a] * ry[b] : rx[a]);   // 1 / f*_i
    y[i] = d[i] * inv;
    ymax = fmax(ymax, y[i]);
    sdy += d[i] * y[i];
  }
  if (bad) return r_inf<R>();
  // the bound is non-negative, so a screen of 0 (a literal in the callers
  // that need every value exact) never returns it: the test, and with it
  // the bound, drop out of their code
  if (screen > R(0)) {
    const R ub = sdy * (R(0.5) + ymax * R(1.0 / 3.0));   // ymax >= 0 (it starts at 0)
    // the margin covers the rounding of the bound itself
    if (!(ymax > R(0.5)) && ub * R(1.0001) < screen) {
      if (screened) *screened = true;
      return ub;
    }
  }
  // A negative population f_i = v_i + w_i rho0 < 0 has y_i = (f*_i - f_i) /
  // f*_i > 1 (f*_i > 0 here), so the screen above never returns for it and
  // the test is needed only from here on.  f_i < 0 exactly when v_i < -sh (a
  // nonzero sum does not round to zero), one instruction fewer.
  if constexpr (Q != 27) {
    bool neg = false;
#pragma unroll
    for (int i = 0; i < Q; ++i) neg |= v[i] < -(SH ? wt<R, Q>(i) * rho0 : R(0));
    if (neg) return r_inf<R>();
  }
  // h_fn takes the Taylor series wherever |x| < 0.1; when that holds for
  // every component of every active lane of the wavefront, the logarithms
  // are skipped for all of them (same values, the series either way).
  R ya = R(0);                           // max |y_i|
#pragma unroll
  for (int i = 0; i < Q; ++i) ya = fmax(ya, fabs(y[i]));
  const bool big = !(ya < R(0.1));
  // FP32: a site with every |y_i| < 0.01 takes the short series in every
  // component (h_poly_short), chosen by the site's own values only.
  const bool tiny = sizeof(R) == 4 && ya < R(0.01);
  auto hp = [&](R x) {
    if constexpr (sizeof(R) == 4) return tiny ? (R)h_poly_short((float)x) : h_poly<R>(x);
    else return h_poly<R>(x);
  };
  // Each component adds fma(a_i, b_i, acc): (d_i y_i, h_poly(-y_i)) where
  // |y_i| < 0.1 (f*_i h(x_i) = f*_i y_i^2 h_poly(-y_i) = d_i y_i h_poly), else
  // (f*_i, h(-y_i)); both branches below form the same terms in the same
  // order, so a site's value does not depend on the other lanes.
  R acc = R(0);
  if (__ballot(big) == 0ull) {
    if (sizeof(R) == 4 && tiny) {
#pragma unroll
      for (int i = 0; i < Q; ++i) acc = fma(d[i] * y[i], hp(-y[i]), acc);
    } else {
#pragma unroll
      for (int i = 0; i < Q; ++i) acc = fma(d[i] * y[i], h_poly<R>(-y[i]), acc);
    }
  } else {
    const R rs = rho * (R(1) / S);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int a = vx_of<Q>(i) + 1, b = vy_of<Q>(i) + 1, cz = vz_of<Q>(i) + 1;
      const R fq = Q == 27 ? fx[a] * fy[b] * fz[cz] : (Q == 9 ? fx[a] * fy[b] : fx[a]);
      const bool small = fabs(y[i]) < R(0.1);
      const R ta = small ? d[i] * y[i] : fq * rs;
      const R tb = small ? hp(-y[i]) : h_fn<R>(-y[i]);
      acc = fma(ta, tb, acc);
    }
  }
  return acc;
}
template <class R, int Q, bool SH>
__device__ __forceinline__ R site_dS_q(const R v[Q], const R d[Q], R m0, R rho0, R ux, R uy, R uz,
                                       int kind, R screen) {
  R dx[3], dy[3], dz[3];
  eq_dev6<R>(ux, kind, dx);
  if constexpr (Q >= 9) eq_dev6<R>(uy, kind, dy);
  if constexpr (Q == 27) eq_dev6<R>(uz, kind, dz);
  return site_dS_dev<R, Q, SH>(v, d, m0, rho0, dx, dy, dz, screen);
}
template <class R, int Q, bool SH>
__device__ __forceinline__ R site_dS(const R v[Q], const R d[Q], R m0, R rho0, R ux, R uy,
                                     int kind, R screen = R(0)) {
  return site_dS_q<R, Q, SH>(v, d, m0, rho0, ux, uy, R(0), kind, screen);
}

// Ranking key of a non-negative Delta S: its bit pattern (monotone in the
// value); NaN ranks as +inf.
template <class R> __device__ __forceinline__ typename KeyOf<R>::T key_of(R x);
template <> __device__ __forceinline__ uint32_t key_of<float>(float x) {
  return x != x ? 0x7f800000u : __float_as_uint(x);   // NaN ranks as +inf
}
template <> __device__ __forceinline__ unsigned long long key_of<double>(double x) {
  return x != x ? 0x7ff0000000000000ull : (unsigned long long)__double_as_longlong(x);
}
// The Delta S value whose key is k.
template <class R> __device__ __forceinline__ R value_of_key(unsigned long long k);
template <> __device__ __forceinline__ float value_of_key<float>(unsigned long long k) {
  return __uint_as_float((uint32_t)k);
}
template <> __device__ __forceinline__ double value_of_key<double>(unsigned long long k) {
  return __longlong_as_double((long long)k);
}

// Everything up to Delta S for one site: used by the step, the median halo
// and the selection rescans, so that all of them see bit-identical values.
// PER: the caller knows the lattice is periodic (branch-free pull).  WALL:
// the configuration may have the diffusive wall (configurations with the
// adjoint or an ensemble limiter never do, and their kernels leave it out).
// CACHED: cached loads (the median kernel pulls halo sites that neighbouring
// tiles pull too).
template <class S, int Q, bool PER = false, bool WALL = !PER, bool CACHED = false>
__device__ __forceinline__ typename StoreT<S>::R site_prep(
    const StepArgs<typename StoreT<S>::R>& A, int x, int y, typename StoreT<S>::R v[Q],
    typename StoreT<S>::R feq[Q], typename StoreT<S>::R d[Q], typename StoreT<S>::R& m0,
    typename StoreT<S>::R& ux, typename StoreT<S>::R& uy, bool need_dS,
    typename StoreT<S>::R screen = typename StoreT<S>::R(0), bool* screened = nullptr) {
  using R = typename StoreT<S>::R;
  constexpr bool SH = StoreT<S>::shifted;
  if constexpr (PER) pull_periodic<S, Q, CACHED>((const S*)A.src, A.qs, A.pitch, A.nx, A.ny, x, y, v);
  else pull<S, Q, CACHED>((const S*)A.src, A.qs, A.pitch, A.nx, A.ny, A.bc, x, y, A.lid, v);
  // a diffusive wall node: the wall rule, and Delta S 0 (never a candidate)
  const bool wall = WALL && on_wall<R>(A, x, y);
  if (wall) diffusive_wall<S, Q>(A, x, y, v);
  moments_v<R, Q, SH>(v, A.rho0, m0, ux, uy);
  R dx[3], dy[3];
  equilibrium_v<R, Q, SH>(m0, A.rho0, ux, uy, A.eq_kind, feq, dx, dy);
#pragma unroll
  for (int i = 0; i < Q; ++i) d[i] = feq[i] - v[i];
  return (need_dS && !wall) ? site_dS_dev<R, Q, SH>(v, d, m0, A.rho0, dx, dy, dx, screen, screened)
                            : R(0);
}

template <class R> struct KeyInf;
template <> struct KeyInf<float> { static constexpr unsigned long long v = 0x7f800000ull; };
template <> struct KeyInf<double> { static constexpr unsigned long long v = 0x7ff0000000000000ull; };

// Histogram bucket of a key in the frame (base, shift); +inf keys and keys
// beyond the frame go to the top bucket.
template <class R>
__device__ __forceinline__ int bucket_of(unsigned long long key, unsigned long long base,
                                         unsigned int shift) {
  if (key >= KeyInf<R>::v) return kBuckets - 1;
  if (key < base) return 0;
  const unsigned long long b = (key - base) >> shift;
  return b >= (unsigned long long)kBuckets ? kBuckets - 1 : (int)b;
}

// Candidate floor and histogram frame of this step's parity.  Both
// parities' fields and the step count are read unconditionally (the state
// always exists), so that the loads issue together.
struct StepFrame {
  unsigned long long floor, base;
  unsigned int shift;
};
__device__ __forceinline__ StepFrame step_frame(const SelState* sel) {
  const unsigned long long f0 = sel->floor_key[0], f1 = sel->floor_key[1];
  const unsigned long long b0 = sel->base_key[0], b1 = sel->base_key[1];
  const unsigned int s0 = sel->shift[0], s1 = sel->shift[1];
  const bool odd = (sel->step & 1ull) != 0;
  return StepFrame{odd ? f1 : f0, odd ? b1 : b0, odd ? s1 : s0};
}

// h[bin] += 1 for every active lane with `on` (h in LDS or global memory).
// The lanes whose bin equals the first such lane's add with one atomic: a
// group of exactly tied keys sends whole wavefronts to one bin, where 64
// atomics on one address would queue behind each other.
__device__ __forceinline__ void hist_add(unsigned int* h, unsigned int bin, bool on) {
  const unsigned long long act = __ballot(on);
  if (!act) return;
  const int leader = __ffsll((long long)act) - 1;
  const unsigned int b0 = (unsigned int)__shfl((int)bin, leader);
  const unsigned long long same = __ballot(on && bin == b0);
  if (on && bin != b0) atomicAdd(&h[bin], 1u);
  else if ((int)__lane_id() == leader) atomicAdd(&h[b0], (unsigned int)__popcll(same));
}

// Append of Ehrenfest candidates by one wavefront (all its lanes call it):
// the wavefront owns 64 entries of the candidate buffer (its region), so a
// ballot gives every candidate its slot without a global counter; the
// region's count goes to wcount and each key's bucket count to the
// histogram.
template <class R>
__device__ __forceinline__ void append_candidates(const StepArgs<R>& A, const StepFrame& fr,
                                                  long long region, bool is_c,
                                                  typename KeyOf<R>::T key, uint32_t idx,
                                                  R m0, R ux, R uy) {
  const unsigned long long mask = __ballot(is_c);
  if (!mask) return;
  const int lane = __lane_id();
  if (lane == __ffsll((long long)mask) - 1) {
    A.wcount[region] = (uint32_t)__popcll(mask);
    atomicAdd(&A.ccount[(region & (kCountSlots - 1)) * kCountStride], (unsigned long long)__popcll(mask));
  }
  if (is_c) {
    const long long pos = region * 64 + __popcll(mask & ((1ull << lane) - 1ull));
    A.cand_key[pos] = key;
    A.cand_idx[pos] = idx;
    A.cand_mom[pos] = m0;
    A.cand_mom[A.cap + pos] = ux;
    A.cand_mom[2 * A.cap + pos] = uy;
  }
  hist_add(A.hist, (unsigned int)hist_pos(bucket_of<R>((unsigned long long)key, fr.base, fr.shift)), is_c);
}

template <class S, int Q, bool CACHED = false>
__device__ typename StoreT<S>::R slot_dS(const StepArgs<typename StoreT<S>::R>& A, int gx,
                                         int gy) {
  using R = typename StoreT<S>::R;
  const bool wrap_x = A.bc == BC_PERIODIC || A.bc == BC_COUETTE;
  const bool wrap_y = A.bc == BC_PERIODIC;
  if (wrap_x) gx = gx < 0 ? gx + A.nx : (gx >= A.nx ? gx - A.nx : gx);
  if (wrap_y) gy = gy < 0 ? gy + A.ny : (gy >= A.ny ? gy - A.ny : gy);
  if (gx < 0 || gx >= A.nx || gy < 0 || gy >= A.ny) return __builtin_nan("");  // outside
  if (on_wall<R>(A, gx, gy)) return __builtin_nan("");   // a diffusive wall node
  R v[Q], feq[Q], d[Q], m0, ux, uy;
  return site_prep<S, Q, false, true, CACHED>(A, gx, gy, v, feq, d, m0, ux, uy, true);
}

}  // namespace lbm
