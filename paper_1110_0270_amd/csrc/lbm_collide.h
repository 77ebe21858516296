// Collision of one site (LBGK, MRT, ELBM) and the positivity rule, shared by
// the step kernel, the adjoint's recompute and the adjoint kernel so that all
// of them take bit-identical branches.
#pragma once

#include "lbm_site.h"

namespace lbm {

struct ElbmF64Site { float f[9], q[9]; };
struct ElbmF64Result { float alpha; int branch; int iters; };

// The FP64 root solve for a site of an FP32 lattice, out of line: the FP32
// kernels carry its code once, away from their hot path (few sites take it).
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
// ci.deferred is set and post[] is left unset.
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
      m[k] = s * (((A.nu_rows >> k) & 1u) ? om : A.rates[k]);
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

}  // namespace lbm
