// Device-side building blocks of the regularised LBM step for gfx950:
// lattice constants, storage forms, equilibria, nonequilibrium entropy,
// the ELBM root solve and the positivity rule.  Everything here is
// __device__ inline and templated on the compute type R (double or float).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// ---------------------------------------------------------------------------
// Lattices (section 2; section 6 for D1Q3, section 5 for D2Q9).  Tensor
// order: D2Q9 i = 3 (b + 1) + (a + 1) for velocity (a, b), opposite 8 - i;
// D1Q3 i = a + 1, opposite 2 - i.  Weights are the products of the D1Q3
// weights (1/6, 2/3, 1/6), which the 1D equilibria take at u = 0.
// ---------------------------------------------------------------------------
__device__ constexpr int kAx9[9] = {-1, 0, 1, -1, 0, 1, -1, 0, 1};
__device__ constexpr int kBy9[9] = {-1, -1, -1, 0, 0, 0, 1, 1, 1};

template <class R>
__device__ __forceinline__ R w1(int a) {  // D1Q3 weight of velocity a
  return a == 0 ? R(2) / R(3) : R(1) / R(6);
}
template <class R>
__device__ __forceinline__ R w9(int i) {
  return w1<R>(kAx9[i]) * w1<R>(kBy9[i]);
}

enum Bc : int { BC_PERIODIC = 0, BC_BOUNCEBACK = 1, BC_CAVITY = 2, BC_COUETTE = 3, BC_DIFFUSIVE = 4 };
enum Coll : int { COLL_LBGK = 0, COLL_MRT = 1, COLL_ELBM = 2 };
enum EqKind : int { EQ_POLY = 0, EQ_ENTROPIC = 1 };
enum ElbmBranch : int { EB_ROOT = 0, EB_CUTOFF = 1, EB_NOROOT = 2, EB_NONPOS = 3, EB_F64 = 4 };

// ---------------------------------------------------------------------------
// Storage forms.  FP64 holds f_i.  FP32, FP16 and BF16 hold the shifted
// deviation g_i = f_i - w_i rho0, rounded to nearest even, so that their
// precision is spent on the small deviations from rest.  Populations are
// loaded and stored nontemporally: a step reads and writes each one once,
// and the two lattices are far larger than the caches (measured 5 % faster
// steps at 4096^2 than with cached loads).  ldc is the cached load, for the
// kernels that read a population again (halos staged in LDS).
// ---------------------------------------------------------------------------
struct bf16_t { uint16_t bits; };

template <class S> struct StoreT;
template <> struct StoreT<double> {
  using R = double;
  static constexpr bool shifted = false;
  static __device__ __forceinline__ double cvt(double v) { return v; }
  static __device__ __forceinline__ double raw(const double* p) { return __builtin_nontemporal_load(p); }
  static __device__ __forceinline__ double ld(const double* p) { return __builtin_nontemporal_load(p); }
  static __device__ __forceinline__ double ldc(const double* p) { return *p; }
  static __device__ __forceinline__ void st(double* p, double v) { __builtin_nontemporal_store(v, p); }
};
template <> struct StoreT<float> {
  using R = float;
  static constexpr bool shifted = true;
  static __device__ __forceinline__ float cvt(float v) { return v; }
  static __device__ __forceinline__ float raw(const float* p) { return __builtin_nontemporal_load(p); }
  static __device__ __forceinline__ float ld(const float* p) { return __builtin_nontemporal_load(p); }
  static __device__ __forceinline__ float ldc(const float* p) { return *p; }
  static __device__ __forceinline__ void st(float* p, float v) { __builtin_nontemporal_store(v, p); }
};
template <> struct StoreT<_Float16> {
  using R = float;
  static constexpr bool shifted = true;
  static __device__ __forceinline__ float cvt(_Float16 v) { return (float)v; }
  static __device__ __forceinline__ _Float16 raw(const _Float16* p) { return __builtin_nontemporal_load(p); }
  static __device__ __forceinline__ float ld(const _Float16* p) { return (float)__builtin_nontemporal_load(p); }
  static __device__ __forceinline__ float ldc(const _Float16* p) { return (float)*p; }
  static __device__ __forceinline__ void st(_Float16* p, float v) { __builtin_nontemporal_store((_Float16)v, p); }
};
template <> struct StoreT<bf16_t> {
  using R = float;
  static constexpr bool shifted = true;
  static __device__ __forceinline__ float cvt(bf16_t v) { return __uint_as_float(((uint32_t)v.bits) << 16); }
  static __device__ __forceinline__ bf16_t raw(const bf16_t* p) {
    bf16_t r;
    r.bits = __builtin_nontemporal_load(&p->bits);
    return r;
  }
  static __device__ __forceinline__ float ld(const bf16_t* p) {
    return __uint_as_float(((uint32_t)__builtin_nontemporal_load(&p->bits)) << 16);
  }
  static __device__ __forceinline__ float ldc(const bf16_t* p) {
    return __uint_as_float(((uint32_t)p->bits) << 16);
  }
  static __device__ __forceinline__ void st(bf16_t* p, float v) {
    // gfx950's conversion instruction: round to nearest even, NaN stays NaN
    const uint16_t r = __builtin_bit_cast(uint16_t, (__bf16)v);
    __builtin_nontemporal_store(r, &p->bits);
  }
};

// ---------------------------------------------------------------------------
// 1D equilibria (section 6), scaled by 6 so that the weights become the
// integers c = (1, 4, 1), and written as deviations dt_a = 6 phi_a(u) - c_a:
//   polynomial: phi_0 = (2/3)(1 - 3u^2/2)  ->  dt_0 = -6 u^2
//   entropic:   phi_0 = (2/3)(2 - s), s = sqrt(1 + 3u^2)  ->  dt_0 = -4 (s - 1)
//   both:       phi_+- = (1 - phi_0)/2 +- u/2  ->  dt_+- = -dt_0/2 +- 3u
// (the same identities as the printed phi_-, phi_+).  With exact integer
// weights, sum_a (c_a + dt_a) = 6 and sum_a a (c_a + dt_a) = 6u hold up to
// unbiased rounding, so the discrete equilibrium adds no systematic mass or
// momentum drift in FP32.
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ void eq_dev6(R u, int kind, R dt[3]) {
  R d0;
  if (kind == EQ_POLY) {
    d0 = R(-6) * u * u;
  } else {
    const R t = R(3) * u * u;
    d0 = R(-4) * (t / (sqrt(R(1) + t) + R(1)));  // -4 (s - 1) without cancellation
  }
  const R h = R(-0.5) * d0;
  dt[0] = h - R(3) * u;
  dt[1] = d0;
  dt[2] = h + R(3) * u;
}

__device__ __forceinline__ int c1(int a) { return a == 0 ? 4 : 1; }  // 6 w_a

// h(x) = (1 + x) ln(1 + x) - x, h(-1) = 1; Taylor series for |x| < 0.1.
// h_series is the series part, x^2 h_poly(x); h_log(x, l) takes
// l = ln(1 + x) from the caller (so that a sum that also needs ln(1 + x)
// evaluates it once).
template <class R>
__device__ __forceinline__ R h_poly(R x);
template <>
__device__ __forceinline__ double h_poly<double>(double x) {
  double acc = 0.0;
#pragma unroll
  for (int n = 16; n >= 3; --n) {
    double c = ((n & 1) ? -1.0 : 1.0) / (double)(n * (n - 1));
    acc = (acc + c) * x;
  }
  return acc + 0.5;
}
template <>
__device__ __forceinline__ float h_poly<float>(float x) {
  // terms up to x^8 (truncation below 4e-8 of the leading term), Horner's
  // rule in fused multiply-adds: sum_{n=2..8} (-1)^n x^(n-2) / (n (n-1))
  float p = 1.0f / 56.0f;
#pragma unroll
  for (int n = 7; n >= 2; --n) p = fmaf(p, x, ((n & 1) ? -1.0f : 1.0f) / (float)(n * (n - 1)));
  return p;
}
// FP32, |x| < 0.01: the terms up to x^3 (n <= 5); the rest of the series is
// below |x|^4 / 30 / (1 - |x|) < 3.4e-10, i.e. 6.7e-10 of the leading 1/2,
// under FP32's rounding and under h_poly's own truncation.
__device__ __forceinline__ float h_poly_short(float x) {
  return fmaf(fmaf(fmaf(-1.0f / 20.0f, x, 1.0f / 12.0f), x, -1.0f / 6.0f), x, 0.5f);
}
template <class R>
__device__ __forceinline__ R h_series(R x) { return h_poly<R>(x) * x * x; }
// Branch-free selects: both forms are evaluated and one is kept, so that the
// nine components of a site interleave instead of running as nine divergent
// branches one after another.
template <class R>
__device__ __forceinline__ R h_log(R x, R l) {
  const R ser = h_series<R>(x);
  const R lgv = (R(1) + x) * l - x;
  return fabs(x) < R(0.1) ? ser : (x <= R(-1) ? R(1) : lgv);
}
// ln(1 + x) for x >= -1.  FP64: the library log1p.  FP32: for |x| < 0.1 its
// Taylor series to x^8 (truncation below 1.2e-9 relative); otherwise the
// hardware logarithm of u = 1 + x times x / (u - 1), which removes the
// rounding of u (D. Goldberg, What every computer scientist should know
// about floating-point arithmetic, 1991, theorem 4): a few units in the last
// place, against the several hundred instructions of the extended-precision
// library routine.
template <class R> __device__ __forceinline__ R lg1p(R x);
template <> __device__ __forceinline__ double lg1p<double>(double x) { return log1p(x); }
// The series part of lg1p<float> (|x| < 0.1).
template <class R> __device__ __forceinline__ R lg1p_series(R x);
template <> __device__ __forceinline__ float lg1p_series<float>(float x) {
  // x sum_{n=1..8} (-1)^(n+1) x^(n-1) / n by Horner's rule in fused
  // multiply-adds
  float p = -1.0f / 8.0f;
#pragma unroll
  for (int n = 7; n >= 1; --n) p = fmaf(p, x, ((n & 1) ? 1.0f : -1.0f) / (float)n);
  return p * x;
}
template <> __device__ __forceinline__ double lg1p_series<double>(double x) { return log1p(x); }
template <> __device__ __forceinline__ float lg1p<float>(float x) {
  const float ser = lg1p_series<float>(x);
  const float u = 1.0f + x;
  const float lgv = __logf(u) * (x * __builtin_amdgcn_rcpf(u - 1.0f));
  return fabsf(x) < 0.1f ? ser : lgv;
}

// a / b: correctly rounded in FP64; in FP32 a times the hardware reciprocal
// (within 2 units in the last place).
template <class R> __device__ __forceinline__ R fdiv(R a, R b);
template <> __device__ __forceinline__ double fdiv<double>(double a, double b) { return a / b; }
template <> __device__ __forceinline__ float fdiv<float>(float a, float b) {
  return a * __builtin_amdgcn_rcpf(b);
}
template <class R>
__device__ __forceinline__ R h_fn(R x) {
  if constexpr (sizeof(R) == 4) {
    return h_log<R>(x, lg1p<R>(x < R(-1) ? R(-1) : x));
  } else {
    if (fabs(x) < R(0.1)) return h_series<R>(x);
    if (x <= R(-1)) return R(1);
    return (R(1) + x) * lg1p<R>(x) - x;
  }
}

template <class R> __device__ __forceinline__ R rcp(R x);
template <> __device__ __forceinline__ double rcp<double>(double x) { return 1.0 / x; }
template <> __device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

template <class R> __device__ __forceinline__ R r_inf();
template <> __device__ __forceinline__ double r_inf<double>() { return __builtin_huge_val(); }
template <> __device__ __forceinline__ float r_inf<float>() { return __builtin_huge_valf(); }

// ---------------------------------------------------------------------------
// ELBM root (section 3).  S_f(alpha) = S(f + alpha D) - S(f), D = f* - f,
// with entropic f*, in the cancellation-free form
//   S_f   = -sum f_i h(alpha D_i / f_i) - alpha sum D_i ln(f_i / f*_i)
//   S_f'  = -sum D_i ln((f_i + alpha D_i) / f*_i)
//   S_f'' = -sum D_i^2 / (f_i + alpha D_i)
// ---------------------------------------------------------------------------
// x = num / f: in FP32 num times rf = rcp(f), the value fdiv gives, with the
// reciprocal taken once per site instead of once per evaluation; in FP64 the
// correctly rounded quotient.
template <class R>
__device__ __forceinline__ R over_f(R num, R f, R rf) {
  if constexpr (sizeof(R) == 4) return num * rf;
  else return num / f;
}

// True when b holds on every active lane of the wavefront.
__device__ __forceinline__ bool wave_all(bool b) { return __all(b) != 0; }

// S_f and its derivatives at alpha = a.  s1 = sum_i D_i ln(f_i / f*_i), the
// same for every alpha.  With r_i = D_i / (f_i + a D_i) the higher
// derivatives are S_f^(2) = -sum D r, S_f^(3) = sum D r^2 and
// S_f^(4) = -2 sum D r^3 (d2, d3, d4); rmax = max |r_i| bounds the ratio of
// consecutive terms of the Taylor series of S_f in alpha around a.
// m = max_i |D_i| / f_i (FP32; from rf): a m < 0.0999999 guarantees every
// computed |x_i| = |fl(fl(a D_i) rf_i)| < 0.1 (the margin of 1e-6 covers
// the two roundings), so that the wavefront can take the series alone.
template <class R, int Q>
__device__ __forceinline__ void sf_parts(const R f[Q], const R rf[Q], const R D[Q], R s1, R m,
                                         R a, R& sf, R& d1, R& d2, R& d3, R& d4, R& rmax) {
  R s0 = R(0), t1 = R(0), t2 = R(0), t3 = R(0), t4 = R(0);
  rmax = R(0);
  auto higher = [&](int i) {
    const R r = D[i] * rcp<R>(f[i] + a * D[i]);
    const R u = D[i] * r, u2 = u * r;
    t2 += u;
    t3 += u2;
    t4 += u2 * r;
    rmax = fmax(rmax, fabs(r));
  };
  if (sizeof(R) == 4 && wave_all(a * m < R(0.0999999))) {
    // every |x_i| < 0.1 on the wavefront: ln(1 + x) and h(x) are their
    // series, the values the selects below would keep
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R x = over_f<R>(a * D[i], f[i], rf[i]);
      s0 += f[i] * h_series<R>(x);
      t1 += D[i] * lg1p_series<R>(x);
      higher(i);
    }
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R x = over_f<R>(a * D[i], f[i], rf[i]);
      const R xl = x < R(-1) ? R(-1) : x;
      const R l = lg1p<R>(xl);
      s0 += f[i] * h_log<R>(x, l);
      t1 += D[i] * l;
      if constexpr (sizeof(R) == 4) {
        higher(i);
      } else {
        t2 += fdiv<R>(D[i] * D[i], f[i] + a * D[i]);
      }
    }
  }
  sf = -s0 - a * s1;
  d1 = -(t1 + s1);
  d2 = -t2;
  d3 = t3;
  d4 = R(-2) * t4;
}

template <class R>
struct ElbmParams {
  R eps;        // stop when |S_f / S_f'| * ||D|| < eps
  R atol;       // or when |S_f / S_f'| < atol (the resolution of alpha; 0 in FP64)
  R dS_cut;     // Delta S below: plain LBGK (alpha = 2)
  int max_iter;
  int norm;     // 0 entropic, 1 L1
  int fallback; // 0 positivity (alpha_max), 1 Ehrenfest rule (alpha = 1)
};

// Returns alpha and the branch taken.  f: populations, feq: entropic
// equilibrium, D = feq - f, amax: largest alpha with f + alpha D >= 0
// (computed by the caller).
//
// The cutoff test Delta S < dS_cut needs the exact Delta S =
// sum f*_i h(x_i), x_i = (f_i - f*_i) / f*_i, only near equilibrium:
// h(x) >= x^2 / (2 (1 + x/3)) for x >= -1 (the bound behind Bernstein's
// inequality), so sum f*_i x_i^2 / (2 (1 + max x/3)) <= Delta S decides it
// for every other site.  The same x_i give ln(f_i / f*_i) and the entropic
// norm.
template <class R, int Q>
__device__ R elbm_alpha(const R f[Q], const R feq[Q], const R D[Q], R amax,
                        const ElbmParams<R>& p, int& branch, int& iters) {
  iters = 0;
  bool nonpos = false;
#pragma unroll
  for (int i = 0; i < Q; ++i) nonpos |= (f[i] <= R(0));
  if (nonpos) { branch = EB_NONPOS; return R(1); }
  R x[Q], U = R(0), xmax = R(-1);
  bool xsmall = true;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    x[i] = fdiv<R>(-D[i], feq[i]);
    U += feq[i] * x[i] * x[i];
    xmax = fmax(xmax, x[i]);
    xsmall &= fabs(x[i]) < R(0.1);
  }
  if (U < R(2) * p.dS_cut * (R(1) + xmax / R(3))) {
    R dS = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) dS += feq[i] * h_fn<R>(x[i]);
    if (dS < p.dS_cut) { branch = EB_CUTOFF; return R(2); }
  }
  // s1 = sum_i D_i ln(f_i / f*_i), ln(f_i / f*_i) = ln(1 + x_i)
  R s1 = R(0);
  if (sizeof(R) == 4 && wave_all(xsmall)) {
#pragma unroll
    for (int i = 0; i < Q; ++i) s1 += D[i] * lg1p_series<R>(x[i]);
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) s1 += D[i] * lg1p<R>(x[i]);
  }
  R nrm = R(0);
  if (p.norm == 0) {
    nrm = sqrt(U);
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) nrm += fabs(D[i]);
  }
  R rf[Q], m = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    rf[i] = sizeof(R) == 4 ? rcp<R>(f[i]) : R(0);
    m = fmax(m, fabs(D[i]) * rf[i]);
  }
  // One evaluation site for S_f and its derivatives (the kernel's code size
  // decides its speed).  A root exists iff S_f(alpha_max) < 0 (alpha_max
  // finite).  S_f is concave (S is concave, f + alpha D affine) with
  // S_f(0) = 0, so the first iterate's evaluation at a settles that in most
  // sites: the tangent there bounds S_f from above, and if it reaches 0
  // within the first half of [a, alpha_max], S_f(alpha_max) <= d1
  // (alpha_max - a) / 2 < 0, a margin far above rounding.  Otherwise the
  // next evaluation is the probe at alpha_max, after which the iteration
  // resumes from the saved first one.  The evaluation that stops the
  // iteration also serves the final sign check.
  // FP32: after a full evaluation at c, S_f and its first two derivatives at
  // c + dl come from the Taylor series in alpha to the fourth derivative
  // while |dl| rmax <= 2^-10 (the first omitted term is below 1e-9 of the
  // second-order one, under FP32 rounding); further away, a full evaluation.
  constexpr bool TAYLOR = sizeof(R) == 4;
  bool need_probe = amax < r_inf<R>();
  bool saved = false, full = true;
  R a = amax > R(2) ? R(2) : R(0.5) * (R(1) + amax);
  R c = a, F0 = R(0), F1 = R(0), F2 = R(0), F3 = R(0), F4 = R(0), rmax = r_inf<R>();
  R prev = r_inf<R>();
  // a Newton step within 64 units in the last place of alpha that no longer
  // halves is rounding noise: the iteration has converged as far as this
  // precision allows (otherwise such a site spins to max_iter and holds up
  // its whole wavefront)
  constexpr R kNoise = R(64) * (sizeof(R) == 4 ? R(1.1920929e-7) : R(2.220446049250313e-16));
  for (int it = 0;;) {
    R sf, d1, d2;
    const bool probing = need_probe && saved;
    if (full || probing) {
      R e0, e1, e2, e3, e4, em;
      sf_parts<R, Q>(f, rf, D, s1, m, probing ? amax : a, e0, e1, e2, e3, e4, em);
      if (probing) {
        if (e0 >= R(0)) {
          branch = EB_NOROOT;
          return p.fallback == 0 ? amax : R(1);
        }
        need_probe = false;   // resume at a = c
        sf = F0;
        d1 = F1;
        d2 = F2;
      } else {
        c = a;
        F0 = e0; F1 = e1; F2 = e2; F3 = e3; F4 = e4;
        rmax = em;
        sf = e0;
        d1 = e1;
        d2 = e2;
        if (need_probe) {
          const R gap = amax - a;
          if (d1 < R(0) && gap >= R(0.25) * a && sf + R(0.5) * d1 * gap < R(0)) {
            need_probe = false;   // the tangent proves the root
          } else {
            saved = true;
            continue;
          }
        }
      }
    } else {
      const R dl = a - c;
      sf = F0 + dl * (F1 + dl * (R(0.5) * F2 + dl * (F3 * R(1.0 / 6.0) + dl * (F4 * R(1.0 / 24.0)))));
      d1 = F1 + dl * (F2 + dl * (R(0.5) * F3 + dl * (F4 * R(1.0 / 6.0))));
      d2 = F2 + dl * (F3 + dl * (R(0.5) * F4));
    }
    const R step_est = fabs(fdiv<R>(sf, d1));
    const bool stalled = it >= 2 && step_est >= R(0.5) * prev && step_est < kNoise * a;
    if (step_est * nrm < p.eps || step_est < p.atol || it >= p.max_iter || stalled) {
      if (sf < R(0)) a = a - fdiv<R>(R(2) * sf, d1);
      break;
    }
    ++it;
    ++iters;
    prev = step_est;
    R disc = d1 * d1 - R(2) * sf * d2;
    R delta = disc >= R(0) ? fdiv<R>(R(2) * sf, -d1 + sqrt(disc)) : fdiv<R>(-sf, d1);
    R an = a + delta;
    if (an >= amax) an = R(0.5) * (a + amax);
    if (an <= R(1)) an = R(0.5) * (a + R(1));
    a = an;
    full = !TAYLOR || !(fabs(a - c) * rmax <= R(0x1p-10));
  }
  branch = EB_ROOT;
  return a;
}

// Largest alpha keeping f + alpha D >= 0 (inf if no D_i < 0).
template <class R, int Q>
__device__ __forceinline__ R alpha_max(const R f[Q], const R D[Q]) {
  R amax = r_inf<R>();
#pragma unroll
  for (int i = 0; i < Q; ++i)
    if (D[i] < R(0)) amax = fmin(amax, fdiv<R>(f[i], -D[i]));
  return amax;
}

}  // namespace lbm
