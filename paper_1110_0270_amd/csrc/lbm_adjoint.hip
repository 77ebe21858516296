// Adjoint of the regularised LBM step (reverse mode).
//
// A step maps the stored lattice g_t to g_{t+1}(x) = C(p(x); omega(x)), where
// p = pull(g_t) is the streamed pre-collision state (section 2) and C the
// site-local collision with its limiters.  The pull with periodic wrap and
// halfway bounce-back is a permutation of the populations (plus constants
// from the moving wall), so its transpose is a push that writes every entry
// of the adjoint lattice exactly once: with mu(x) = J(x)^T lambda_{t+1}(x),
//   lambda_t[i](x - v_i) = mu_i(x)   when x - v_i is the pull source,
//   lambda_t[opp(i)](x)  = mu_i(x)   when the pull bounced back.
// J(x) is differentiated along the branch the forward step took: a site
// sent to equilibrium by the Ehrenfest limiter contributes d f*/d p; the
// positivity rule through its homothety coefficient and the component that
// attained it; ELBM through alpha, by implicit differentiation of
// S(p + alpha (f* - p)) = S(p) on the root branch (section 3) or through the
// attaining component of alpha_max on the positivity branch.
#include <hip/hip_ext.h>

#include "lbm_adjoint.h"
#include "lbm_collide.h"

namespace lbm {

// 1D equilibrium factors phi_a(u) and their derivatives (section 6):
//   polynomial: phi_0 = 2/3 - u^2, phi_+- = 1/6 +- u/2 + u^2/2;
//   entropic:   phi_0 = (2/3)(2 - s), phi_+- = +-u/2 + (2s - 1)/6, s = sqrt(1+3u^2).
template <class R>
__device__ __forceinline__ void eq_phi(R u, int kind, R phi[3], R dphi[3]) {
  R dt[3];
  eq_dev6<R>(u, kind, dt);
#pragma unroll
  for (int a = 0; a < 3; ++a) phi[a] = ((R)c1(a - 1) + dt[a]) / R(6);
  const R g = kind == EQ_POLY ? u : u / sqrt(R(1) + R(3) * u * u);
  dphi[0] = R(-0.5) + g;
  dphi[1] = R(-2) * g;
  dphi[2] = R(0.5) + g;
}

// out = (d f*/d p)^T a for f*_i = rho phi_a(u_x) phi_b(u_y), rho = sum p,
// rho u = sum v p: out_k = a0 + v_kx ax + v_ky ay with
// ax = sum_i a_i phi_a' phi_b, ay = sum_i a_i phi_a phi_b',
// a0 = sum_i a_i phi_a phi_b - u_x ax - u_y ay.
template <class R, int Q>
__device__ __forceinline__ void feq_vjp(const R a[Q], R ux, R uy, int kind, R out[Q]) {
  R px[3], dpx[3], py[3], dpy[3];
  eq_phi<R>(ux, kind, px, dpx);
  if constexpr (Q == 9) eq_phi<R>(uy, kind, py, dpy);
  R s0 = R(0), sx = R(0), sy = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int ia = vx_of<Q>(i) + 1, ib = vy_of<Q>(i) + 1;
    if constexpr (Q == 9) {
      s0 += a[i] * (px[ia] * py[ib]);
      sx += a[i] * (dpx[ia] * py[ib]);
      sy += a[i] * (px[ia] * dpy[ib]);
    } else {
      s0 += a[i] * px[ia];
      sx += a[i] * dpx[ia];
    }
  }
  const R a0 = s0 - ux * sx - uy * sy;
#pragma unroll
  for (int k = 0; k < Q; ++k) out[k] = a0 + (R)vx_of<Q>(k) * sx + (R)vy_of<Q>(k) * sy;
}

template <class R>
struct AdjArgs {
  const R* lam_in;          // lambda_{t+1}, [Q][ny][pitch]
  R* lam_out;               // lambda_t
  R* gom;                   // dL/d omega accumulator [ny][pitch] or nullptr
  const unsigned char* mask;// 1 at sites the Ehrenfest limiter sent to f* (or nullptr)
  const R* alpha;           // ELBM: the step's alpha per site [ny][pitch]
  const unsigned char* branch;  // ELBM: the step's branch per site
  // Short Ehrenfest lists (k <= kAdjListLds) replace the mask: the step's
  // selected sites and their count, read into LDS by every workgroup.
  const int32_t* list;
  const long long* count;
  long long k;
  // Median filter ([ny][pitch] each, or nullptr): per site, the derivative
  // of the loss with respect to its own Delta S through its homothety
  // (med_gs), the derivative with respect to its median neighbour's Delta S
  // (med_h), and which neighbour that is (med_am: offset code, 255 = none).
  R* med_gs;
  R* med_h;
  unsigned char* med_am;
};
constexpr int kAdjListLds = (int)kAdjListMax;

// The step's adjoint at one site: a = dL/dv for the state v that entered
// the collision (the pulled state, after the median filter when it is on),
// given lam = dL/d(the site's post-collision state), along the branch the
// forward step took; gw receives dL/d omega(x).  d = f* - v.
// SELMRT: an LBGK lattice whose selected sites took the MRT collision (the
// MRT limiter); a compile-time variant, so that the other kernels do not
// carry the MRT code.
template <class S, int Q, int COLL, bool SELMRT = false>
__device__ __forceinline__ void adjoint_site(const StepArgs<typename StoreT<S>::R>& A,
                                             const AdjArgs<typename StoreT<S>::R>& B, long long o,
                                             bool ehr, const typename StoreT<S>::R v[Q],
                                             const typename StoreT<S>::R feq[Q],
                                             const typename StoreT<S>::R d[Q],
                                             typename StoreT<S>::R ux, typename StoreT<S>::R uy,
                                             typename StoreT<S>::R om,
                                             const typename StoreT<S>::R lam[Q],
                                             typename StoreT<S>::R a[Q],
                                             typename StoreT<S>::R& gw) {
  using R = typename StoreT<S>::R;
  constexpr bool SH = StoreT<S>::shifted;
  R mu[Q], lf[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) lf[i] = R(0);
  gw = R(0);
  // on an MRT-limited lattice a selected site took the MRT collision
  const bool mrt_here = COLL == COLL_MRT || (Q == 9 && SELMRT && ehr);
  if (ehr && !SELMRT) {
    // Ehrenfest step: g' = f*(p)
#pragma unroll
    for (int i = 0; i < Q; ++i) { lf[i] = lam[i]; mu[i] = R(0); }
  } else {
    R q[Q];
    CollInfo<R> ci;
    if constexpr (COLL == COLL_ELBM) {
      // alpha and branch of the forward step, kept by the recompute: the
      // collided state is the forward's bit for bit without a second root solve
      ci.alpha = B.alpha[o];
      ci.branch = B.branch[o];
      const R ab = ci.alpha * (om * R(0.5));
#pragma unroll
      for (int i = 0; i < Q; ++i) q[i] = v[i] + ab * d[i];
    } else if constexpr (Q == 9) {
      if (mrt_here) collide_site<S, Q, COLL_MRT>(A, v, feq, d, om, q, ci);
      else collide_site<S, Q, COLL>(A, v, feq, d, om, q, ci);
    } else {
      collide_site<S, Q, COLL>(A, v, feq, d, om, q, ci);
    }
    // positivity rule: g'' = f* + phi (q - f*), phi = f*_a / (f*_a - q_a)
    R lq[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) lq[i] = lam[i];
    if (A.positivity) {
      R q2[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) q2[i] = q[i];
      CollInfo<R> cp;
      positivity_site<S, Q>(A, feq, q2, cp);
      if (cp.pos_arg >= 0) {
        const int a = cp.pos_arg;
        const R phi = cp.phi;
        R se = R(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) se += (q[i] - feq[i]) * lam[i];
        const R sha = SH ? wt<R, Q>(a) * A.rho0 : R(0);
        const R qa = q[a] + sha, fa = feq[a] + sha;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          lq[i] = phi * lam[i];
          lf[i] = (R(1) - phi) * lam[i];
        }
        lq[a] += se * phi * phi / fa;
        lf[a] -= se * phi * phi * qa / (fa * fa);
      }
    }
    if (COLL == COLL_MRT || mrt_here) {
      // q = p + B (f* - p), B = Minv diag(rates(omega)) M; the rates of the
      // presets depend on the shear rate too
      R z[Q], m[Q];
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        R sz = R(0), sm = R(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          sz += A.Minv[i * Q + k] * lq[i];
          sm += A.M[k * Q + i] * d[i];
        }
        z[k] = sz;
        m[k] = sm;
        gw += mrt_drate<R>(A, k, om) * sz * sm;
      }
#pragma unroll
      for (int k = 0; k < Q; ++k) z[k] *= mrt_rate<R>(A, k, om);
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        R w = R(0);
#pragma unroll
        for (int k = 0; k < Q; ++k) w += A.M[k * Q + j] * z[k];
        mu[j] = lq[j] - w;
        lf[j] += w;
      }
    } else if constexpr (COLL == COLL_LBGK) {
      // q = p + omega (f* - p)
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        mu[i] = (R(1) - om) * lq[i];
        lf[i] += om * lq[i];
        gw += lq[i] * d[i];
      }
    } else {
      // q = p + alpha beta (f* - p), beta = omega / 2
      const R alpha = ci.alpha, ab = alpha * (om * R(0.5));
      R lal = R(0);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        mu[i] = (R(1) - ab) * lq[i];
        lf[i] += ab * lq[i];
        gw += lq[i] * (alpha * R(0.5)) * d[i];
        lal += lq[i] * d[i];
      }
      lal *= om * R(0.5);                       // dL/d alpha
      R fa[Q], qa[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const R sh = SH ? wt<R, Q>(i) * A.rho0 : R(0);
        fa[i] = v[i] + sh;
        qa[i] = feq[i] + sh;
      }
      if (ci.branch == EB_ROOT) {
        // implicit derivative: d alpha = -(dS_f/dp dp + dS_f/df* df*) / S_f',
        // with ln((p + alpha D)/w) = ln(p/w) + ln(1 + alpha D/p)
        R d1 = R(0), l1[Q], lw[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const R xx = alpha * d[i] / fa[i];
          l1[i] = lg1p<R>(xx < R(-1) ? R(-1) : xx);
          lw[i] = log(fa[i] / wt<R, Q>(i));
          d1 -= d[i] * (l1[i] + lg1p<R>(-d[i] / qa[i]));
        }
        const R c = -lal / d1;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const R gs = -(lw[i] + l1[i] + R(1));   // dS/dy at p + alpha D
          const R ps = -(lw[i] + R(1));           // dS/dy at p
          mu[i] += c * ((R(1) - alpha) * gs - ps);
          lf[i] += c * (alpha * gs);
        }
      } else if (ci.branch == EB_NOROOT && A.fallback == 0) {
        // alpha = alpha_max = p_a / (p_a - f*_a) at the attaining component
        R amin = r_inf<R>();
        int a = -1;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          if (d[i] < R(0)) {
            const R r = fa[i] / (-d[i]);
            if (r < amin) { amin = r; a = i; }
          }
        }
        if (a >= 0) {
          const R den = fa[a] - qa[a];
          mu[a] += lal * (-qa[a] / (den * den));
          lf[a] += lal * (fa[a] / (den * den));
        }
      }
    }
  }
  R tf[Q];
  feq_vjp<R, Q>(lf, ux, uy, A.eq_kind, tf);
#pragma unroll
  for (int i = 0; i < Q; ++i) a[i] = mu[i] + tf[i];
}

// Transpose of the pull: val_i, the derivative with respect to the
// population that site (x, y) pulled in direction i, goes to that
// population's slot of the adjoint lattice (add = true adds it to what is
// there).  Every slot is reached from exactly one site.
template <class R, int Q, bool ADD = false>
__device__ __forceinline__ void push_adjoint(const StepArgs<R>& A, R* lam_out, int x, int y,
                                             const R val[Q]) {
  const long long o = (long long)y * A.pitch + x;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int sx = x - vx_of<Q>(i), sy = y - vy_of<Q>(i);
    bool out;
    if (A.bc == BC_PERIODIC) {
      sx = sx < 0 ? sx + A.nx : (sx >= A.nx ? sx - A.nx : sx);
      sy = sy < 0 ? sy + A.ny : (sy >= A.ny ? sy - A.ny : sy);
      out = false;
    } else if (A.bc == BC_COUETTE) {
      sx = sx < 0 ? sx + A.nx : (sx >= A.nx ? sx - A.nx : sx);
      out = (sy < 0) | (sy >= A.ny);
    } else {
      out = (sx < 0) | (sx >= A.nx) | (sy < 0) | (sy >= A.ny);
    }
    R* dst = !out ? &lam_out[(long long)i * A.qs + (long long)sy * A.pitch + sx]
                  : &lam_out[(long long)(Q - 1 - i) * A.qs + o];
    if constexpr (ADD) *dst += val[i];
    else __builtin_nontemporal_store(val[i], dst);
  }
}

// Reads a short Ehrenfest list into LDS (every thread of the workgroup
// calls it) and returns its length; 0 without a list.
template <class R>
__device__ __forceinline__ int load_short_list(const AdjArgs<R>& B, int32_t* lsel) {
  if (!B.list) return 0;
  // the list's k slots (k <= kAdjListLds) are loaded with its count: one
  // round trip
  const long long c = *B.count;
  const int32_t v = (long long)threadIdx.x < B.k ? B.list[threadIdx.x] : 0;
  const int nl = (int)(c < B.k ? c : B.k);
  if ((int)threadIdx.x < nl) lsel[threadIdx.x] = v;
  __syncthreads();
  return nl;
}

// LBGK in FP32 arithmetic keeps seven wavefronts per SIMD (at most 72
// registers, 8 bytes of spills): the 4096^2 FP32 adjoint step took 359
// against 368 us with six (75 registers, no spills) and 553 us with five;
// eight (64 registers) spill 112 bytes.
template <class S, int Q, int COLL, bool SELMRT = false>
__global__ __launch_bounds__(256, (COLL == COLL_LBGK && !SELMRT && sizeof(S) <= 4) ? 7 : 1)
void k_adjoint(const StepArgs<typename StoreT<S>::R> A, const AdjArgs<typename StoreT<S>::R> B) {
  using R = typename StoreT<S>::R;
  // Workgroups go round-robin to the 8 XCDs; each XCD takes pairs of
  // adjacent 256-site segments, which share the lines that the pull and the
  // push reach across their edge (the last, incomplete group of 16 keeps
  // launch order).
  const long long nb = gridDim.x, b = blockIdx.x;
  const long long tb = (b / 16 * 16 + 16 <= nb) ? (b / 16) * 16 + (b % 8) * 2 + (b / 8) % 2 : b;
  const long long s = tb * blockDim.x + threadIdx.x;
  __shared__ int32_t lsel[kAdjListLds];
  const int nl = load_short_list<R>(B, lsel);
  if (s >= (long long)A.nx * A.ny) return;
  bool ehr = B.mask && B.mask[s];
  for (int j = 0; j < nl; ++j) ehr |= lsel[j] == (int32_t)s;
  const int y = (int)(s / A.nx), x = (int)(s % A.nx);
  R v[Q], feq[Q], d[Q], m0, ux, uy;
  site_prep<S, Q, false, false>(A, x, y, v, feq, d, m0, ux, uy, false);
  const long long o = (long long)y * A.pitch + x;
  const R om = A.omega_field ? A.omega_field[o] : A.omega;
  R lam[Q], a[Q], gw;
#pragma unroll
  for (int i = 0; i < Q; ++i)
    // the adjoint lattices, like the populations, are streamed once per
    // step: nontemporal loads and stores
    lam[i] = __builtin_nontemporal_load(&B.lam_in[(long long)i * A.qs + o]);
  adjoint_site<S, Q, COLL, SELMRT>(A, B, o, ehr, v, feq, d, ux, uy, om, lam, a, gw);
  push_adjoint<R, Q>(A, B.lam_out, x, y, a);
  if (B.gom) __builtin_nontemporal_store(__builtin_nontemporal_load(&B.gom[o]) + gw, &B.gom[o]);
}

// Adjoint of a step with the median entropy filter (section 4), first part.
// The forward step replaced the pulled state p of a site by
//   p~ = f* + c (p - f*),  c = sqrt(med / Delta S)
// where the site was accepted (Delta S > delta and med < Delta S; med the
// median Delta S of its neighbourhood), and collided p~; f* is the same for
// p and p~ (same moments).  With a = dL/dp~ from the collision's adjoint:
//   dL/dp = c a + (df*/dp)^T ((1 - c) a)          (through p and f*)
//         + dL/dc dc/d Delta S(x) grad Delta S(x)  (through the site's own Delta S)
// and dL/dc dc/dmed flows to the median neighbour y's Delta S.  Each
// workgroup recomputes Delta S of its tile and a one-site halo in LDS (as
// the forward kernel does), finds the median and which neighbour holds it
// (stable ranks: among equal values the lowest offset code, -1..1 in y then
// x), pushes the first line into the adjoint lattice and records, per site,
// the two Delta S derivatives and the median neighbour's code for
// k_median_gather.  dL/dc = sum_i a_i (p_i - f*_i); dc/dDelta S = -c /
// (2 Delta S); dc/dmed = c / (2 med), taken as 0 where med = 0 (the site
// was mapped onto f*; the one-sided derivative is infinite).
template <class S, int Q, int COLL, int TX, int TY, bool SELMRT = false>
__global__ __launch_bounds__(256) void k_adjoint_med(const StepArgs<typename StoreT<S>::R> A,
                                                     const AdjArgs<typename StoreT<S>::R> B) {
  using R = typename StoreT<S>::R;
  static_assert(TX * TY == 256, "tile must hold 256 sites");
  const int t = blockIdx.x;
  const int tile_x = t % A.tiles_x, tile_y = t / A.tiles_x;
  const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
  const int x = tile_x * TX + lx, y = tile_y * TY + ly;
  const bool valid = x < A.nx && y < A.ny;
  __shared__ int32_t lsel[kAdjListLds];
  const int nl = load_short_list<R>(B, lsel);
  R v[Q], feq[Q], d[Q], m0 = R(0), ux = R(0), uy = R(0), dS = R(0);
  if (valid) dS = site_prep<S, Q, false, false>(A, x, y, v, feq, d, m0, ux, uy, true);
  constexpr int HY = (Q == 9) ? 1 : 0;
  constexpr int SW = TX + 2, SH_ = TY + 2 * HY;
  __shared__ R sdS[SH_ * SW];
  sdS[(ly + HY) * SW + lx + 1] = valid ? dS : slot_dS<S, Q>(A, x, y);
  constexpr int NHALO = SH_ * SW - TX * TY;
  for (int s = threadIdx.x; s < NHALO; s += 256) {
    int hx, hy;
    if constexpr (HY == 1) {
      if (s < SW) { hx = s; hy = 0; }
      else if (s < 2 * SW) { hx = s - SW; hy = SH_ - 1; }
      else { const int r = s - 2 * SW; hy = 1 + r / 2; hx = (r & 1) ? SW - 1 : 0; }
    } else {
      hy = 0;
      hx = (s == 0) ? 0 : SW - 1;
    }
    sdS[hy * SW + hx] = slot_dS<S, Q>(A, tile_x * TX + hx - 1, tile_y * TY + hy - HY);
  }
  __syncthreads();
  if (!valid) return;
  constexpr int NN = (Q == 9) ? 9 : 3;
  R nb[NN];
  int n = 0;
#pragma unroll
  for (int k = 0; k < NN; ++k) {
    const int dy = (Q == 9) ? k / 3 - 1 : 0, dx = (Q == 9) ? k % 3 - 1 : k - 1;
    const R val = sdS[(ly + HY + dy) * SW + lx + 1 + dx];
    const bool in = !(val != val);
    n += in ? 1 : 0;
    nb[k] = in ? val : r_inf<R>();
  }
  // the median (the ceil(n/2)-th smallest) and the neighbour that holds it
  const int rank = (n + 1) / 2 - 1;
  int am = -1;
  R med = r_inf<R>();
#pragma unroll
  for (int k = 0; k < NN; ++k) {
    int r = 0;
#pragma unroll
    for (int j = 0; j < NN; ++j) r += (nb[j] < nb[k] || (j < k && nb[j] == nb[k])) ? 1 : 0;
    if (r == rank) { am = k; med = nb[k]; }
  }
  const bool acc = (dS > A.med_delta) & (med < dS) & (dS < r_inf<R>());
  const R c = acc ? sqrt(med / dS) : R(1);
  // the filtered state, as the forward step formed it
  R vt[Q], dt[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    vt[i] = acc ? feq[i] + c * (v[i] - feq[i]) : v[i];
    dt[i] = feq[i] - vt[i];
  }
  const long long s = (long long)y * A.nx + x;
  bool ehr = B.mask && B.mask[s];
  for (int j = 0; j < nl; ++j) ehr |= lsel[j] == (int32_t)s;
  const long long o = (long long)y * A.pitch + x;
  const R om = A.omega_field ? A.omega_field[o] : A.omega;
  R lam[Q], a[Q], gw;
#pragma unroll
  for (int i = 0; i < Q; ++i) lam[i] = B.lam_in[(long long)i * A.qs + o];
  adjoint_site<S, Q, COLL, SELMRT>(A, B, o, ehr, vt, feq, dt, ux, uy, om, lam, a, gw);
  R gs = R(0), h = R(0);
  if (acc) {
    R sc = R(0), ra[Q], tf[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      sc -= a[i] * d[i];                  // dL/dc = sum a_i (p_i - f*_i)
      ra[i] = (R(1) - c) * a[i];
    }
    feq_vjp<R, Q>(ra, ux, uy, A.eq_kind, tf);
#pragma unroll
    for (int i = 0; i < Q; ++i) a[i] = c * a[i] + tf[i];
    gs = -sc * c / (R(2) * dS);
    h = med > R(0) ? sc * c / (R(2) * med) : R(0);
  }
  push_adjoint<R, Q>(A, B.lam_out, x, y, a);
  B.med_gs[o] = gs;
  B.med_h[o] = h;
  B.med_am[o] = (acc && h != R(0)) ? (unsigned char)am : (unsigned char)255;
  if (B.gom) B.gom[o] += gw;
}

// Second part: site y collects G = dL/dDelta S(y), its own term plus the
// terms of the neighbours whose median it held, and adds G grad_p Delta S(y)
// to the adjoint slots that its pulled populations came from.  With
// Delta S = sum_i p_i ln(p_i / f*_i) and f* a function of the moments of p:
//   grad_p Delta S = ln(p / f*) + (df*/dp)^T ((f* - p) / f*)
// (the 1 from differentiating p ln p cancels against sum_j df*_j/dp =
// d rho / dp = 1).  For the entropic equilibrium the second term vanishes:
// ln f* is affine in the velocity and f*, p share their moments.  A
// population at 0 (left there by the positivity rule) contributes 0 ln 0 =
// 0 to Delta S with no derivative (the one-sided one is infinite).
template <class S, int Q>
__global__ __launch_bounds__(256) void k_median_gather(const StepArgs<typename StoreT<S>::R> A,
                                                       const AdjArgs<typename StoreT<S>::R> B) {
  using R = typename StoreT<S>::R;
  constexpr bool SH = StoreT<S>::shifted;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (long long)A.nx * A.ny) return;
  const int y = (int)(s / A.nx), x = (int)(s % A.nx);
  const long long o = (long long)y * A.pitch + x;
  R G = B.med_gs[o];
  constexpr int NN = (Q == 9) ? 9 : 3;
  const bool wrap_x = A.bc == BC_PERIODIC || A.bc == BC_COUETTE;
  const bool wrap_y = A.bc == BC_PERIODIC;
#pragma unroll
  for (int k = 0; k < NN; ++k) {
    const int dy = (Q == 9) ? k / 3 - 1 : 0, dx = (Q == 9) ? k % 3 - 1 : k - 1;
    int gx = x + dx, gy = y + dy;
    if (wrap_x) gx = gx < 0 ? gx + A.nx : (gx >= A.nx ? gx - A.nx : gx);
    if (wrap_y) gy = gy < 0 ? gy + A.ny : (gy >= A.ny ? gy - A.ny : gy);
    if (gx < 0 || gx >= A.nx || gy < 0 || gy >= A.ny) continue;
    const long long on = (long long)gy * A.pitch + gx;
    // neighbour (gx, gy) = (x, y) + e had its median at offset -e
    if (B.med_am[on] == (unsigned char)(NN - 1 - k)) G += B.med_h[on];
  }
  if (G == R(0)) return;
  R v[Q], feq[Q], d[Q], m0, ux, uy;
  site_prep<S, Q, false, false>(A, x, y, v, feq, d, m0, ux, uy, false);
  R r[Q], tf[Q], g[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R sh = SH ? wt<R, Q>(i) * A.rho0 : R(0);
    r[i] = d[i] / (feq[i] + sh);           // (f* - p) / f*
  }
  feq_vjp<R, Q>(r, ux, uy, A.eq_kind, tf);
#pragma unroll
  for (int i = 0; i < Q; ++i) g[i] = G * ((r[i] < R(1) ? lg1p<R>(-r[i]) : R(0)) + tf[i]);
  push_adjoint<R, Q, true>(A, B.lam_out, x, y, g);
}

// Recompute of an Ehrenfest step from its tape: the selected state (f*, or
// the MRT limiter's collision) at the listed sites, from the pulled state
// exactly as the selection kernels computed it.
template <class S, int Q>
__global__ void k_tape_fix(const StepArgs<typename StoreT<S>::R> A, const int32_t* list,
                           const long long* count, long long k) {
  using R = typename StoreT<S>::R;
  // the list's slots (k of them) are loaded with its count: one round trip
  // fewer than loading them after it
  const long long c = *count;
  const long long n = c < k ? c : k;
  for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < k;
       j += (long long)gridDim.x * blockDim.x) {
    const int idx = list[j];
    if (j >= n) continue;
    const int y = idx / A.nx, x = idx % A.nx;
    R v[Q], feq[Q], d[Q], m0, ux, uy;
    site_prep<S, Q, false, false>(A, x, y, v, feq, d, m0, ux, uy, false);
    if (A.sel_mrt) selected_state<S, Q>(A, x, y, m0, ux, uy, feq);
    S* dst = (S*)A.dst;
#pragma unroll
    for (int i = 0; i < Q; ++i)
      StoreT<S>::st(dst + (long long)i * A.qs + (long long)y * A.pitch + x, feq[i]);
  }
}

__global__ void k_mark(unsigned char* mask, const int32_t* list, const long long* count,
                       long long k, unsigned char val) {
  const long long n = *count < k ? *count : k;
  for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (long long)gridDim.x * blockDim.x)
    mask[list[j]] = val;
}

// Dense caller arrays <-> pitched compute-precision arrays.
template <class R>
__global__ void k_to_pitch(const void* src, int src_f64, R* dst, int nf, int nx, int ny,
                           int pitch, long long qs) {
  const long long n = (long long)nx * ny;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n * nf;
       s += (long long)gridDim.x * blockDim.x) {
    const int f = (int)(s / n);
    const long long r = s % n;
    const int y = (int)(r / nx), x = (int)(r % nx);
    const double v = src_f64 ? ((const double*)src)[s] : (double)((const float*)src)[s];
    dst[(long long)f * qs + (long long)y * pitch + x] = (R)v;
  }
}
template <class R>
__global__ void k_from_pitch(const R* src, void* dst, int dst_f64, int nf, int nx, int ny,
                             int pitch, long long qs) {
  const long long n = (long long)nx * ny;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n * nf;
       s += (long long)gridDim.x * blockDim.x) {
    const int f = (int)(s / n);
    const long long r = s % n;
    const int y = (int)(r / nx), x = (int)(r % nx);
    const double v = (double)src[(long long)f * qs + (long long)y * pitch + x];
    if (dst_f64) ((double*)dst)[s] = v;
    else ((float*)dst)[s] = (float)v;
  }
}

// ---------------------------------------------------------------------------
static int grid_of(long long n) {
  long long g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 65535 * 16 ? 65535 * 16 : g));
}

template <class S, int Q, int COLL, bool SELMRT>
static void launch_adj_k(const StepArgs<typename StoreT<S>::R>& A,
                         const AdjArgs<typename StoreT<S>::R>& B, int g, hipStream_t s,
                         hipEvent_t e0, hipEvent_t e1) {
  if (B.med_am) {
    // median filter: the 64 x 4 (D1Q3: 256 x 1) tiles of the forward median
    // kernel, then the gather; the events bracket both
    constexpr int TX = Q == 9 ? 64 : 256, TY = 256 / TX;
    const dim3 gt(A.tiles_x * A.tiles_y);
    const int gs = (int)(((long long)A.nx * A.ny + 255) / 256);
    if (e0 || e1) {
      hipExtLaunchKernelGGL((k_adjoint_med<S, Q, COLL, TX, TY, SELMRT>), gt, dim3(256), 0, s, e0, nullptr, 0, A, B);
      hipExtLaunchKernelGGL((k_median_gather<S, Q>), dim3(gs), dim3(256), 0, s, nullptr, e1, 0, A, B);
    } else {
      hipLaunchKernelGGL((k_adjoint_med<S, Q, COLL, TX, TY, SELMRT>), gt, dim3(256), 0, s, A, B);
      hipLaunchKernelGGL((k_median_gather<S, Q>), dim3(gs), dim3(256), 0, s, A, B);
    }
    return;
  }
  if (e0 || e1)
    hipExtLaunchKernelGGL((k_adjoint<S, Q, COLL, SELMRT>), dim3(g), dim3(256), 0, s, e0, e1, 0, A, B);
  else
    hipLaunchKernelGGL((k_adjoint<S, Q, COLL, SELMRT>), dim3(g), dim3(256), 0, s, A, B);
}

template <class S, int Q>
static hipError_t launch_adj_q(int coll, const void* sargs, const void* aargs, hipStream_t s,
                               hipEvent_t e0, hipEvent_t e1) {
  using R = typename StoreT<S>::R;
  const StepArgs<R>& A = *(const StepArgs<R>*)sargs;
  const AdjArgs<R>& B = *(const AdjArgs<R>*)aargs;
  const int g = (int)(((long long)A.nx * A.ny + 255) / 256);
  if (coll == COLL_LBGK) {
    if constexpr (Q == 9) {
      if (A.sel_mrt) {
        launch_adj_k<S, Q, COLL_LBGK, true>(A, B, g, s, e0, e1);
        return hipGetLastError();
      }
    }
    launch_adj_k<S, Q, COLL_LBGK, false>(A, B, g, s, e0, e1);
  } else if (coll == COLL_ELBM) {
    launch_adj_k<S, Q, COLL_ELBM, false>(A, B, g, s, e0, e1);
  } else if constexpr (Q == 9) {
    launch_adj_k<S, Q, COLL_MRT, false>(A, B, g, s, e0, e1);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class S>
static hipError_t launch_adj_s(int Q, int coll, const void* sargs, const void* aargs, hipStream_t s,
                               hipEvent_t e0, hipEvent_t e1) {
  return Q == 9 ? launch_adj_q<S, 9>(coll, sargs, aargs, s, e0, e1)
                : launch_adj_q<S, 3>(coll, sargs, aargs, s, e0, e1);
}

hipError_t launch_adjoint(int storage, int Q, int coll, const void* step_args, const void* lam_in,
                          void* lam_out, void* gom, const unsigned char* mask,
                          const void* alpha, const unsigned char* branch, const int32_t* list,
                          const long long* count, long long k, const MedianAdjoint& med,
                          hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (coll == COLL_ELBM && (!alpha || !branch)) return hipErrorInvalidValue;
  if (list && (!count || k > kAdjListLds)) return hipErrorInvalidValue;
  if (med.am && (!med.gs || !med.h)) return hipErrorInvalidValue;
  if (storage == 0) {
    AdjArgs<double> B{(const double*)lam_in, (double*)lam_out, (double*)gom, mask,
                      (const double*)alpha, branch, list, count, k,
                      (double*)med.gs, (double*)med.h, med.am};
    return launch_adj_s<double>(Q, coll, step_args, &B, s, e0, e1);
  }
  AdjArgs<float> B{(const float*)lam_in, (float*)lam_out, (float*)gom, mask,
                   (const float*)alpha, branch, list, count, k,
                   (float*)med.gs, (float*)med.h, med.am};
  if (storage == 1) return launch_adj_s<float>(Q, coll, step_args, &B, s, e0, e1);
  if (storage == 2) return launch_adj_s<_Float16>(Q, coll, step_args, &B, s, e0, e1);
  return launch_adj_s<bf16_t>(Q, coll, step_args, &B, s, e0, e1);
}

template <class S, int Q>
static void tape_fix_q(const void* sargs, const int32_t* list, const long long* cnt, long long k,
                       hipStream_t s) {
  using R = typename StoreT<S>::R;
  const StepArgs<R>& A = *(const StepArgs<R>*)sargs;
  hipLaunchKernelGGL((k_tape_fix<S, Q>), dim3(grid_of(k)), dim3(256), 0, s, A, list, cnt, k);
}

hipError_t launch_tape_fix(int storage, int Q, const void* step_args, const int32_t* list,
                           const long long* count, long long k, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  switch (storage * 16 + Q) {
    case 0 * 16 + 9: tape_fix_q<double, 9>(step_args, list, count, k, s); break;
    case 0 * 16 + 3: tape_fix_q<double, 3>(step_args, list, count, k, s); break;
    case 1 * 16 + 9: tape_fix_q<float, 9>(step_args, list, count, k, s); break;
    case 1 * 16 + 3: tape_fix_q<float, 3>(step_args, list, count, k, s); break;
    case 2 * 16 + 9: tape_fix_q<_Float16, 9>(step_args, list, count, k, s); break;
    case 2 * 16 + 3: tape_fix_q<_Float16, 3>(step_args, list, count, k, s); break;
    case 3 * 16 + 9: tape_fix_q<bf16_t, 9>(step_args, list, count, k, s); break;
    default: tape_fix_q<bf16_t, 3>(step_args, list, count, k, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_mark(unsigned char* mask, const int32_t* list, const long long* count,
                       long long k, unsigned char val, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mark, dim3(grid_of(k)), dim3(256), 0, s, mask, list, count, k, val);
  return hipGetLastError();
}

hipError_t launch_to_pitch(const void* src, int src_f64, void* dst, int dst_f64, int nf, int nx,
                           int ny, int pitch, long long qs, hipStream_t s) {
  const int g = grid_of((long long)nf * nx * ny);
  if (dst_f64) hipLaunchKernelGGL((k_to_pitch<double>), dim3(g), dim3(256), 0, s, src, src_f64, (double*)dst, nf, nx, ny, pitch, qs);
  else hipLaunchKernelGGL((k_to_pitch<float>), dim3(g), dim3(256), 0, s, src, src_f64, (float*)dst, nf, nx, ny, pitch, qs);
  return hipGetLastError();
}

hipError_t launch_from_pitch(const void* src, int src_f64, void* dst, int dst_f64, int nf, int nx,
                             int ny, int pitch, long long qs, hipStream_t s) {
  const int g = grid_of((long long)nf * nx * ny);
  if (src_f64) hipLaunchKernelGGL((k_from_pitch<double>), dim3(g), dim3(256), 0, s, (const double*)src, dst, dst_f64, nf, nx, ny, pitch, qs);
  else hipLaunchKernelGGL((k_from_pitch<float>), dim3(g), dim3(256), 0, s, (const float*)src, dst, dst_f64, nf, nx, ny, pitch, qs);
  return hipGetLastError();
}

}  // namespace lbm
