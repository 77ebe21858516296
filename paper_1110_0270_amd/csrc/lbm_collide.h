// Collision of one site (LBGK, MRT, ELBM) and the positivity rule, shared by
// the step kernel, the adjoint's recompute and the adjoint kernel so that all
// of them take bit-identical branches.
#pragma once

#include "lbm_site.h"

namespace lbm {

struct ElbmF64Site { float f[9], q[9]; };
struct ElbmF64Result { float alpha; int branch; int iters; };

// The FP64 root solve for a site of an FP32 lattice from its FP32 state, out
// of line (the kernels carry its code once, away from their hot path): used
// by the median filter's kernel, which has no deferred list; the other FP32
// ELBM kernels defer such sites to k_elbm_f64, which rebuilds them in FP64.
template <int Q>
__device__ __noinline__ ElbmF64Result elbm_alpha_fp64(ElbmF64Site s, double eps, double dS_cut,
                                                      int max_iter, int norm, int fallback) {
  double fd[Q], qd[Q], Dd[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    fd[i] = (double)s.f[i];
    qd[i] = (double)s.q[i];
    Dd[i] = qd[i] - fd[i];
  }
  ElbmParams<double> e64{eps, 0.0, dS_cut, max_iter, norm, fallback};
  ElbmF64Result r;
  r.alpha = (float)elbm_alpha<double, Q>(fd, qd, Dd, alpha_max<double, Q>(fd, Dd), e64,
                                         r.branch, r.iters);
  return r;
}

// The same FP64 root solve with one site spread over a group of 16 lanes of
// the wavefront: lane c of the group holds component c of f and f* (idle
// lanes, c >= Q or a group without a site, hold f = f* = 1 and add zero to
// every sum).  The sums over the components are butterfly reductions within
// the group, which leave the same bits in every lane of it, so every lane
// takes the same branches and returns the same result.  Each iteration costs
// one logarithm and two divisions per lane instead of Q of each in one lane.
__device__ __forceinline__ double group16_sum(double v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double group16_min(double v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double group16_max(double v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ bool group16_any(bool b) {
  int v = b ? 1 : 0;
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v |= __shfl_xor(v, o);
  return v != 0;
}

struct ElbmGroupResult { double alpha; int branch; int iters; };

static __device__ ElbmGroupResult elbm_alpha_fp64_group(double f_c, double q_c, bool act,
                                                        double eps, double dS_cut, int max_iter,
                                                        int norm, int fallback) {
  const double f = act ? f_c : 1.0, q = act ? q_c : 1.0, D = q - f;
  ElbmGroupResult r;
  r.iters = 0;
  if (group16_any(act && f <= 0.0)) {
    r.alpha = 1.0;
    r.branch = EB_NONPOS;
    return r;
  }
  const double x = -D / q;
  const double U = group16_sum(q * x * x);
  const double xmax = group16_max(act ? x : -1.0);
  if (U < 2.0 * dS_cut * (1.0 + xmax / 3.0)) {
    const double dS = group16_sum(q * h_fn<double>(x));
    if (dS < dS_cut) {
      r.alpha = 2.0;
      r.branch = EB_CUTOFF;
      return r;
    }
  }
  const double lnr = log1p(x);
  const double nrm = norm == 0 ? sqrt(U) : group16_sum(fabs(D));
  const double s1 = group16_sum(D * lnr);
  const double amax = group16_min(D < 0.0 ? f / (-D) : __builtin_huge_val());
  bool probe = amax < __builtin_huge_val();
  double a = amax > 2.0 ? 2.0 : 0.5 * (1.0 + amax);
  double prev = __builtin_huge_val();
  constexpr double kNoise = 64.0 * 2.220446049250313e-16;
  for (int it = 0;;) {
    const double aa = probe ? amax : a;
    const double xa = aa * D / f;
    const double l = log1p(xa < -1.0 ? -1.0 : xa);
    const double s0 = group16_sum(f * h_log<double>(xa, l));
    const double t1 = group16_sum(D * (l + lnr));
    const double t2 = group16_sum(D * D / (f + aa * D));
    const double sf = -s0 - aa * s1, d1 = -t1, d2 = -t2;
    if (probe) {
      if (sf >= 0.0) {
        r.alpha = fallback == 0 ? amax : 1.0;
        r.branch = EB_NOROOT;
        return r;
      }
      probe = false;
      continue;
    }
    const double step_est = fabs(sf / d1);
    const bool stalled = it >= 2 && step_est >= 0.5 * prev && step_est < kNoise * a;
    if (step_est * nrm < eps || it >= max_iter || stalled) {
      if (sf < 0.0) a = a - 2.0 * sf / d1;
      break;
    }
    ++it;
    ++r.iters;
    prev = step_est;
    const double disc = d1 * d1 - 2.0 * sf * d2;
    const double delta = disc >= 0.0 ? 2.0 * sf / (-d1 + sqrt(disc)) : -sf / d1;
    double an = a + delta;
    if (an >= amax) an = 0.5 * (a + amax);
    if (an <= 1.0) an = 0.5 * (a + 1.0);
    a = an;
  }
  r.alpha = a;
  r.branch = EB_ROOT;
  return r;
}

// Relaxation rate of MRT row k at shear rate om (section 5, with the rate
// presets of sections 5, 7 and 8), and its derivative in om.
template <class R>
__device__ __forceinline__ R mrt_rate(const StepArgs<R>& A, int k, R om) {
  if ((A.nu_rows >> k) & 1u) return om;
  if ((A.q_rows >> k) & 1u)
    return A.q_mode == 1 ? R(8) * (R(2) - om) / (R(8) - om) : R(3) * (R(2) - om) / (R(3) - om);
  return A.rates[k];
}
template <class R>
__device__ __forceinline__ R mrt_drate(const StepArgs<R>& A, int k, R om) {
  if ((A.nu_rows >> k) & 1u) return R(1);
  if ((A.q_rows >> k) & 1u) {
    const R c = A.q_mode == 1 ? R(8) : R(3), t = c - om;
    return -c * (c - R(2)) / (t * t);
  }
  return R(0);
}

// Wavefront-aggregated event counter: one atomic per wavefront that has
// events.
__device__ __forceinline__ void count_event(bool ev, unsigned long long* ctr) {
  const unsigned long long m = __ballot(ev);
  if (m && __lane_id() == (unsigned)(__ffsll((long long)m) - 1))
    atomicAdd(ctr, (unsigned long long)__popcll(m));
}

// Sum of a per-lane count over the wavefront, added once.
__device__ __forceinline__ void count_sum(int v, unsigned long long* ctr) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (v && __lane_id() == 0) atomicAdd(ctr, (unsigned long long)v);
}

template <class R>
struct CollInfo {
  R alpha = R(2);   // ELBM alpha (2 elsewhere)
  int branch = EB_ROOT;
  bool f64 = false; // ELBM root solved in FP64
  int pos_arg = -1; // positivity rule: component set to 0, -1 if inactive
  R phi = R(1);     // positivity rule: homothety coefficient
  int iters = 0;    // ELBM root iterations
  bool deferred = false;  // FP64 solve left to k_elbm_f64
};

// Collision (eq. CollisionIntegral; section 5 MRT in moment space; section
// 3 ELBM), in the storage representation: d = f* - f, om the relaxation rate
// (LBGK omega, MRT shear rate s_nu, ELBM 2 beta).
// DEFER (FP32 ELBM only): a site that needs the FP64 solve is not collided;
// ci.deferred is set and post[] is left unset (k_elbm_f64 rebuilds it).
template <class S, int Q, int COLL, bool DEFER = false>
__device__ __forceinline__ void collide_site(const StepArgs<typename StoreT<S>::R>& A,
                                             const typename StoreT<S>::R v[Q],
                                             const typename StoreT<S>::R feq[Q],
                                             const typename StoreT<S>::R d[Q],
                                             typename StoreT<S>::R om,
                                             typename StoreT<S>::R post[Q],
                                             CollInfo<typename StoreT<S>::R>& ci) {
  using R = typename StoreT<S>::R;
  constexpr bool SH = StoreT<S>::shifted;
  if constexpr (COLL == COLL_LBGK) {
#pragma unroll
    for (int i = 0; i < Q; ++i) post[i] = v[i] + om * d[i];
  } else if constexpr (COLL == COLL_MRT) {
    R m[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      R s = R(0);
#pragma unroll
      for (int j = 0; j < Q; ++j) s += A.M[k * Q + j] * d[j];
      m[k] = s * mrt_rate<R>(A, k, om);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      R s = R(0);
#pragma unroll
      for (int k = 0; k < Q; ++k) s += A.Minv[i * Q + k] * m[k];
      post[i] = v[i] + s;
    }
  } else {  // ELBM
    R fa[Q], qa[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R sh = SH ? wt<R, Q>(i) * A.rho0 : R(0);
      fa[i] = v[i] + sh;
      qa[i] = feq[i] + sh;
    }
    const R amax = alpha_max<R, Q>(fa, d);
    int br = EB_ROOT;
    R alpha;
    ElbmParams<R> ep{A.eps, A.atol, A.dS_cut, A.max_iter, A.norm, A.fallback};
    bool f64 = false;
    if constexpr (sizeof(R) == 4) {
      if (amax < A.f64_below) {
        if constexpr (DEFER) {
          ci.deferred = true;
          return;
        }
        // FP64 solve near the no-root (degenerate) branch.
        ElbmF64Site st;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          st.f[i] = fa[i];
          st.q[i] = qa[i];
        }
        const ElbmF64Result r =
            elbm_alpha_fp64<Q>(st, A.eps64, A.dS_cut64, A.max_iter, A.norm, A.fallback);
        alpha = r.alpha;
        br = r.branch;
        ci.iters = r.iters;
        f64 = true;
      } else {
        alpha = elbm_alpha<R, Q>(fa, qa, d, amax, ep, br, ci.iters);
      }
    } else {
      alpha = elbm_alpha<R, Q>(fa, qa, d, amax, ep, br, ci.iters);
    }
    const R ab = alpha * (om * R(0.5));
#pragma unroll
    for (int i = 0; i < Q; ++i) post[i] = v[i] + ab * d[i];
    ci.alpha = alpha;
    ci.branch = br;
    ci.f64 = f64;
  }
}

// Positivity rule (section 4): a collided state with a negative component
// moves along the line to f* until the first component reaches 0.
template <class S, int Q>
__device__ __forceinline__ void positivity_site(const StepArgs<typename StoreT<S>::R>& A,
                                                const typename StoreT<S>::R feq[Q],
                                                typename StoreT<S>::R post[Q],
                                                CollInfo<typename StoreT<S>::R>& ci) {
  using R = typename StoreT<S>::R;
  constexpr bool SH = StoreT<S>::shifted;
  R phi = r_inf<R>();
  int arg = -1;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R sh = SH ? wt<R, Q>(i) * A.rho0 : R(0);
    const R pa = post[i] + sh, qa = feq[i] + sh;
    if (pa < R(0) && qa > R(0)) {
      const R r = qa / (qa - pa);
      if (r < phi) { phi = r; arg = i; }
    }
  }
  if (arg >= 0) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R sh = SH ? wt<R, Q>(i) * A.rho0 : R(0);
      post[i] = (i == arg) ? -sh : feq[i] + phi * (post[i] - feq[i]);
    }
    ci.pos_arg = arg;
    ci.phi = phi;
  }
}

// The state the Ehrenfest selection gives a selected site (section 4, and
// the MRT limiter of section 5): f* from the moments the step recorded for
// it, or, on an MRT-limited lattice, the MRT collision of its pulled state
// (the step's source lattice, intact while the selection runs) followed by
// the positivity rule when that is on.
template <class S, int Q>
__device__ __forceinline__ void selected_state(const StepArgs<typename StoreT<S>::R>& A, int x,
                                               int y, typename StoreT<S>::R m0,
                                               typename StoreT<S>::R ux,
                                               typename StoreT<S>::R uy,
                                               typename StoreT<S>::R out[Q]) {
  using R = typename StoreT<S>::R;
  constexpr bool SH = StoreT<S>::shifted;
  if constexpr (Q == 9) {
    if (A.sel_mrt) {
      R v[Q], feq[Q], d[Q], mm, vx, vy;
      site_prep<S, Q, false, false>(A, x, y, v, feq, d, mm, vx, vy, false);
      const R om = A.omega_field ? A.omega_field[(long long)y * A.pitch + x] : A.omega;
      CollInfo<R> ci;
      collide_site<S, Q, COLL_MRT>(A, v, feq, d, om, out, ci);
      if (A.positivity) positivity_site<S, Q>(A, feq, out, ci);
      return;
    }
  }
  equilibrium_v<R, Q, SH>(m0, A.rho0, ux, uy, A.eq_kind, out);
}

// The step after the pull (and the median filter): Ehrenfest candidacy
// (eligible, Delta S > delta, and above the floor), collision, positivity
// rule, store into the second lattice, and the limiter counters.  Every lane
// of the wavefront calls it.
// DEFER (FP32 ELBM): sites whose root solve needs FP64 are listed for
// k_elbm_f64 instead of being collided, limited and stored here.
template <class S, int Q, int COLL, bool EHR = true, bool DEFER = false>
__device__ __forceinline__ void site_finish(const StepArgs<typename StoreT<S>::R>& A, int x, int y,
                                            bool valid, bool wall, long long region,
                                            typename StoreT<S>::R v[Q],
                                            typename StoreT<S>::R feq[Q],
                                            typename StoreT<S>::R d[Q], typename StoreT<S>::R m0,
                                            typename StoreT<S>::R ux, typename StoreT<S>::R uy,
                                            typename StoreT<S>::R dS,
                                            const StepFrame& fr,
                                            unsigned long long* cnt) {
  using R = typename StoreT<S>::R;
  // Ehrenfest candidates: eligible (Delta S > delta) and above the floor.
  if (EHR && A.ehrenfest) {
    using K = typename KeyOf<R>::T;
    const K key = key_of<R>(dS);
    const bool is_c = valid && !wall && (dS > A.ehr_delta) && (key >= (K)fr.floor);
    append_candidates<R>(A, fr, region, is_c, key, (uint32_t)(y * A.nx + x), m0, ux, uy);
  }

  R post[Q];
  bool pos_event = false, deferred = false;
  if (valid && wall) {
    // a diffusive wall node keeps its streamed state after the wall rule
    S* dst = (S*)A.dst;
    const unsigned o = (unsigned)(y * A.pitch + x);
#pragma unroll
    for (int i = 0; i < Q; ++i) StoreT<S>::st(at(dst + (long long)i * A.qs, o), v[i]);
  }
  if (valid && !wall) {
    const R om = A.omega_field ? A.omega_field[(long long)y * A.pitch + x] : A.omega;
    CollInfo<R> ci;
    collide_site<S, Q, COLL, DEFER>(A, v, feq, d, om, post, ci);
    deferred = ci.deferred;
    if constexpr (COLL == COLL_ELBM) {
      // a deferred site counts no event here (its CollInfo is the default)
      if (A.alpha_out && !deferred) {
        const long long o = (long long)y * A.pitch + x;
        A.alpha_out[o] = ci.alpha;
        A.branch_out[o] = (unsigned char)ci.branch;
      }
      if (A.count_events) {
        count_event(ci.branch == EB_NOROOT, cnt + CNT_ELBM_NOROOT);
        count_event(ci.f64, cnt + CNT_ELBM_F64);
        count_event(ci.branch == EB_NONPOS, cnt + CNT_ELBM_NONPOS);
        count_sum(ci.iters, cnt + CNT_ELBM_ITERS);
      }
    }
    if (!deferred) {
      if (A.positivity) {
        positivity_site<S, Q>(A, feq, post, ci);
        pos_event = ci.pos_arg >= 0;
      }
      S* dst = (S*)A.dst;
      const unsigned o = (unsigned)(y * A.pitch + x);
#pragma unroll
      for (int i = 0; i < Q; ++i) StoreT<S>::st(at(dst + (long long)i * A.qs, o), post[i]);
    }
  } else if constexpr (COLL == COLL_ELBM) {
    // an empty lane or a wall node: no collision, no events
    if (A.count_events) {
      count_event(false, cnt + CNT_ELBM_NOROOT);
      count_event(false, cnt + CNT_ELBM_F64);
      count_event(false, cnt + CNT_ELBM_NONPOS);
      count_sum(0, cnt + CNT_ELBM_ITERS);
    }
  }
  if (A.positivity && A.count_events) count_event(pos_event, cnt + CNT_POSITIVITY);
  if constexpr (DEFER) {
    // wave-aggregated append to the FP64 list
    const unsigned long long m = __ballot(deferred);
    if (m) {
      const int lane = __lane_id(), leader = __ffsll((long long)m) - 1;
      unsigned int base = 0;
      if (lane == leader) base = atomicAdd(A.f64_count, (unsigned int)__popcll(m));
      base = __shfl(base, leader);
      if (deferred) A.f64_sites[base + __popcll(m & ((1ull << lane) - 1ull))] = (uint32_t)(y * A.nx + x);
    }
  }
}

}  // namespace lbm
