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

enum Bc : int { BC_PERIODIC = 0, BC_BOUNCEBACK = 1, BC_CAVITY = 2, BC_COUETTE = 3 };
enum Coll : int { COLL_LBGK = 0, COLL_MRT = 1, COLL_ELBM = 2 };
enum EqKind : int { EQ_POLY = 0, EQ_ENTROPIC = 1 };
enum ElbmBranch : int { EB_ROOT = 0, EB_CUTOFF = 1, EB_NOROOT = 2, EB_NONPOS = 3, EB_F64 = 4 };

// ---------------------------------------------------------------------------
// Storage forms.  FP64 holds f_i.  FP32, FP16 and BF16 hold the shifted
// deviation g_i = f_i - w_i rho0, rounded to nearest even, so that their
// precision is spent on the small deviations from rest.
// ---------------------------------------------------------------------------
struct bf16_t { uint16_t bits; };

template <class S> struct StoreT;
template <> struct StoreT<double> {
  using R = double;
  static constexpr bool shifted = false;
  static __device__ __forceinline__ double ld(const double* p) { return *p; }
  static __device__ __forceinline__ void st(double* p, double v) { __builtin_nontemporal_store(v, p); }
};
template <> struct StoreT<float> {
  using R = float;
  static constexpr bool shifted = true;
  static __device__ __forceinline__ float ld(const float* p) { return *p; }
  static __device__ __forceinline__ void st(float* p, float v) { __builtin_nontemporal_store(v, p); }
};
template <> struct StoreT<_Float16> {
  using R = float;
  static constexpr bool shifted = true;
  static __device__ __forceinline__ float ld(const _Float16* p) { return (float)*p; }
  static __device__ __forceinline__ void st(_Float16* p, float v) { *p = (_Float16)v; }
};
template <> struct StoreT<bf16_t> {
  using R = float;
  static constexpr bool shifted = true;
  static __device__ __forceinline__ float ld(const bf16_t* p) {
    return __uint_as_float(((uint32_t)p->bits) << 16);
  }
  static __device__ __forceinline__ void st(bf16_t* p, float v) {
    uint32_t u = __float_as_uint(v);
    uint16_t r;
    if ((u & 0x7fffffffu) > 0x7f800000u) {
      r = (uint16_t)((u >> 16) | 0x40u);              // quiet NaN
    } else {
      u += 0x7fffu + ((u >> 16) & 1u);                // round to nearest even
      r = (uint16_t)(u >> 16);
    }
    p->bits = r;
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
template <class R>
__device__ __forceinline__ R h_fn(R x);
template <>
__device__ __forceinline__ double h_fn<double>(double x) {
  if (fabs(x) < 0.1) {
    double acc = 0.0;
#pragma unroll
    for (int n = 16; n >= 3; --n) {
      double c = ((n & 1) ? -1.0 : 1.0) / (double)(n * (n - 1));
      acc = (acc + c) * x;
    }
    return (acc + 0.5) * x * x;
  }
  if (x <= -1.0) return 1.0;
  return (1.0 + x) * log1p(x) - x;
}
template <>
__device__ __forceinline__ float h_fn<float>(float x) {
  if (fabsf(x) < 0.1f) {
    // terms up to x^8: truncation below 4e-8 of the leading term
    float acc = 0.0f;
#pragma unroll
    for (int n = 8; n >= 3; --n) {
      float c = ((n & 1) ? -1.0f : 1.0f) / (float)(n * (n - 1));
      acc = (acc + c) * x;
    }
    return (acc + 0.5f) * x * x;
  }
  if (x <= -1.0f) return 1.0f;
  return (1.0f + x) * log1pf(x) - x;
}

template <class R> __device__ __forceinline__ R rcp(R x);
template <> __device__ __forceinline__ double rcp<double>(double x) { return 1.0 / x; }
template <> __device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

template <class R> __device__ __forceinline__ R lg1p(R x);
template <> __device__ __forceinline__ double lg1p<double>(double x) { return log1p(x); }
template <> __device__ __forceinline__ float lg1p<float>(float x) { return log1pf(x); }

template <class R> __device__ __forceinline__ R r_inf();
template <> __device__ __forceinline__ double r_inf<double>() { return __builtin_huge_val(); }
template <> __device__ __forceinline__ float r_inf<float>() { return __builtin_huge_valf(); }

// Nonequilibrium entropy (section 4, eq. DelS): sum_i f_i ln(f_i / f*_i),
// evaluated as sum_i f*_i h((f_i - f*_i) / f*_i) (same value since f and
// f* share rho).  d = f* - f.  +inf if some f_i < 0 or f*_i <= 0.
template <class R, int Q>
__device__ __forceinline__ R delta_s(const R f[Q], const R feq[Q], const R d[Q]) {
  R s = R(0);
  bool bad = false;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    bad |= (f[i] < R(0)) | (feq[i] <= R(0));
    s += feq[i] * h_fn<R>(-d[i] / feq[i]);
  }
  return bad ? r_inf<R>() : s;
}

// ---------------------------------------------------------------------------
// ELBM root (section 3).  S_f(alpha) = S(f + alpha D) - S(f), D = f* - f,
// with entropic f*, in the cancellation-free form
//   S_f   = -sum f_i h(alpha D_i / f_i) - alpha sum D_i ln(f_i / f*_i)
//   S_f'  = -sum D_i ln((f_i + alpha D_i) / f*_i)
//   S_f'' = -sum D_i^2 / (f_i + alpha D_i)
// ---------------------------------------------------------------------------
template <class R, int Q>
__device__ __forceinline__ void sf_parts(const R f[Q], const R D[Q], const R lnr[Q], R a,
                                         R& sf, R& d1, R& d2) {
  R s0 = R(0), s1 = R(0), t1 = R(0), t2 = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    R x = a * D[i] / f[i];
    s0 += f[i] * h_fn<R>(x);
    s1 += D[i] * lnr[i];
    R xl = x < R(-1) ? R(-1) : x;
    t1 += D[i] * (lg1p<R>(xl) + lnr[i]);
    t2 += D[i] * D[i] / (f[i] + a * D[i]);
  }
  sf = -s0 - a * s1;
  d1 = -t1;
  d2 = -t2;
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
// equilibrium, D = feq - f, dS: nonequilibrium entropy, amax: largest alpha
// with f + alpha D >= 0 (computed by the caller).
template <class R, int Q>
__device__ R elbm_alpha(const R f[Q], const R feq[Q], const R D[Q], R dS, R amax,
                        const ElbmParams<R>& p, int& branch) {
  bool nonpos = false;
#pragma unroll
  for (int i = 0; i < Q; ++i) nonpos |= (f[i] <= R(0));
  if (nonpos) { branch = EB_NONPOS; return R(1); }
  if (dS < p.dS_cut) { branch = EB_CUTOFF; return R(2); }
  R lnr[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) lnr[i] = lg1p<R>(-D[i] / feq[i]);
  const bool finite = amax < r_inf<R>();
  if (finite) {
    R sf, d1, d2;
    sf_parts<R, Q>(f, D, lnr, amax, sf, d1, d2);
    if (sf >= R(0)) {
      branch = EB_NOROOT;
      return p.fallback == 0 ? amax : R(1);
    }
  }
  R nrm = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) nrm += p.norm == 0 ? D[i] * D[i] / feq[i] : fabs(D[i]);
  if (p.norm == 0) nrm = sqrt(nrm);
  R a = amax > R(2) ? R(2) : R(0.5) * (R(1) + amax);
  for (int it = 0; it < p.max_iter; ++it) {
    R sf, d1, d2;
    sf_parts<R, Q>(f, D, lnr, a, sf, d1, d2);
    const R step_est = fabs(sf / d1);
    if (step_est * nrm < p.eps || step_est < p.atol) break;
    R disc = d1 * d1 - R(2) * sf * d2;
    R delta = disc >= R(0) ? R(2) * sf / (-d1 + sqrt(disc)) : -sf / d1;
    R an = a + delta;
    if (an >= amax) an = R(0.5) * (a + amax);
    if (an <= R(1)) an = R(0.5) * (a + R(1));
    a = an;
  }
  {
    R sf, d1, d2;
    sf_parts<R, Q>(f, D, lnr, a, sf, d1, d2);
    if (sf < R(0)) a = a - R(2) * sf / d1;
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
    if (D[i] < R(0)) amax = fmin(amax, f[i] / (-D[i]));
  return amax;
}

}  // namespace lbm
