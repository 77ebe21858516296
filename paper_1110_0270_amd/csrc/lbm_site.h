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

template <int Q> __device__ __forceinline__ int vx_of(int i) { return Q == 9 ? kAx9[i] : i - 1; }
template <int Q> __device__ __forceinline__ int vy_of(int i) { return Q == 9 ? kBy9[i] : 0; }
template <class R, int Q> __device__ __forceinline__ R wt(int i) {
  return Q == 9 ? w9<R>(i) : w1<R>(i - 1);
}

// Equilibrium in the storage representation (unshifted f*_i, or the
// deviation f*_i - w_i rho0) from m0 (rho, or rho - rho0 when shifted):
// the product of the 1D equilibria (section 8), f*_ab = rho phi_a phi_b,
// evaluated as (rho/36) (c_a + dt_a)(c_b + dt_b) with integer weights.
template <class R, int Q, bool SH>
__device__ __forceinline__ void equilibrium_v(R m0, R rho0, R ux, R uy, int kind, R feq[Q]) {
  R dx[3], dy[3];
  eq_dev6<R>(ux, kind, dx);
  if constexpr (Q == 9) eq_dev6<R>(uy, kind, dy);
  const R rho = SH ? rho0 + m0 : m0;
  constexpr R S = Q == 9 ? R(36) : R(6);
  const R rs = rho / S;
  const R ms = m0 / S;
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

// Pull f_i(x) = f_i(x - v_i) with the boundary rules: periodic wrap, or
// halfway bounce-back f_i(x) = f_opp(i)(x) plus the moving-wall term when
// the source lies above the top row.
template <class S, int Q>
__device__ __forceinline__ void pull(const S* __restrict__ src, long long qs, int pitch, int nx,
                                     int ny, int bc, int x, int y,
                                     const typename StoreT<S>::R* lid,
                                     typename StoreT<S>::R v[Q]) {
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int sx = x - vx_of<Q>(i), sy = y - vy_of<Q>(i);
    bool out;
    if (bc == BC_PERIODIC) {
      sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
      sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
      out = false;
    } else if (bc == BC_COUETTE) {
      sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
      out = (sy < 0) | (sy >= ny);
    } else {
      out = (sx < 0) | (sx >= nx) | (sy < 0) | (sy >= ny);
    }
    if (!out) {
      v[i] = StoreT<S>::ld(src + (long long)i * qs + (long long)sy * pitch + sx);
    } else {
      v[i] = StoreT<S>::ld(src + (long long)(Q - 1 - i) * qs + (long long)y * pitch + x);
      if (sy >= ny) v[i] += lid[i];
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
  ux = jx / rho;
  uy = jy / rho;
}

template <class R, int Q, bool SH>
__device__ __forceinline__ R site_dS(const R v[Q], const R feq[Q], const R d[Q], R rho0) {
  R fa[Q], qa[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R sh = SH ? wt<R, Q>(i) * rho0 : R(0);
    fa[i] = v[i] + sh;
    qa[i] = feq[i] + sh;
  }
  return delta_s<R, Q>(fa, qa, d);
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

// Everything up to Delta S for one site: used by the step, the median halo
// and the selection rescans, so that all of them see bit-identical values.
template <class S, int Q>
__device__ __forceinline__ typename StoreT<S>::R site_prep(
    const StepArgs<typename StoreT<S>::R>& A, int x, int y, typename StoreT<S>::R v[Q],
    typename StoreT<S>::R feq[Q], typename StoreT<S>::R d[Q], typename StoreT<S>::R& m0,
    typename StoreT<S>::R& ux, typename StoreT<S>::R& uy, bool need_dS) {
  using R = typename StoreT<S>::R;
  constexpr bool SH = StoreT<S>::shifted;
  pull<S, Q>((const S*)A.src, A.qs, A.pitch, A.nx, A.ny, A.bc, x, y, A.lid, v);
  moments_v<R, Q, SH>(v, A.rho0, m0, ux, uy);
  equilibrium_v<R, Q, SH>(m0, A.rho0, ux, uy, A.eq_kind, feq);
#pragma unroll
  for (int i = 0; i < Q; ++i) d[i] = feq[i] - v[i];
  return need_dS ? site_dS<R, Q, SH>(v, feq, d, A.rho0) : R(0);
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

// Wave-aggregated append of Ehrenfest candidates (all lanes of the wave must
// call it): one atomic per wave reserves the slots; the candidate's key, site
// index and moments go to the buffer and its bucket count to the histogram.
template <class R>
__device__ __forceinline__ void append_candidates(const StepArgs<R>& A, bool is_c,
                                                  typename KeyOf<R>::T key, uint32_t idx,
                                                  R m0, R ux, R uy) {
  const unsigned long long mask = __ballot(is_c);
  if (!mask) return;
  SelState* st = A.sel;
  const int lane = __lane_id();
  const int leader = __ffsll((long long)mask) - 1;
  unsigned long long kmax = (is_c && (unsigned long long)key < KeyInf<R>::v) ? (unsigned long long)key : 0ull;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(kmax, off);
    kmax = o > kmax ? o : kmax;
  }
  unsigned long long base = ~0ull;
  if (lane == leader) {
    // once the buffer has overflowed the step goes to a rescan anyway; stop
    // contending for the counter
    const unsigned long long seen = __hip_atomic_load(&st->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (seen <= (unsigned long long)A.cap) {
      base = atomicAdd(&st->count, (unsigned long long)__popcll(mask));
      if (kmax) atomicMax(&st->max_key, kmax);
    }
  }
  base = __shfl(base, leader);
  if (is_c && base != ~0ull) {
    const unsigned long long pos = base + (unsigned long long)__popcll(mask & ((1ull << lane) - 1ull));
    if (pos < (unsigned long long)A.cap) {
      A.cand_key[pos] = key;
      A.cand_idx[pos] = idx;
      A.cand_mom[pos] = m0;
      A.cand_mom[A.cap + pos] = ux;
      A.cand_mom[2 * A.cap + pos] = uy;
      atomicAdd(&A.hist[bucket_of<R>((unsigned long long)key, st->base_key, st->shift)], 1u);
    }
  }
}

template <class S, int Q>
__device__ typename StoreT<S>::R slot_dS(const StepArgs<typename StoreT<S>::R>& A, int gx,
                                         int gy) {
  using R = typename StoreT<S>::R;
  const bool wrap_x = A.bc == BC_PERIODIC || A.bc == BC_COUETTE;
  const bool wrap_y = A.bc == BC_PERIODIC;
  if (wrap_x) gx = gx < 0 ? gx + A.nx : (gx >= A.nx ? gx - A.nx : gx);
  if (wrap_y) gy = gy < 0 ? gy + A.ny : (gy >= A.ny ? gy - A.ny : gy);
  if (gx < 0 || gx >= A.nx || gy < 0 || gy >= A.ny) return __builtin_nan("");  // outside
  R v[Q], feq[Q], d[Q], m0, ux, uy;
  return site_prep<S, Q>(A, gx, gy, v, feq, d, m0, ux, uy, true);
}

}  // namespace lbm
