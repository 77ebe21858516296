// Ehrenfest regularisation with a budget (section 4): after the collision,
// the k sites of largest nonequilibrium entropy Delta S > delta (ties to the
// lower site index) are sent to their equilibrium f*.  Since every collision
// keeps rho and u, f* is rebuilt from the moments that the step kernel
// recorded with each candidate and written over the collided state.
//
// The step kernel appends only sites whose key (the bit pattern of Delta S,
// monotone for non-negative floats) is at least a floor carried over from
// the previous step, so selection works on a short candidate list instead
// of the whole lattice:
//   k_fb_scan   (only if the candidates cannot contain the answer: too few
//                above a raised floor, or more than the buffer holds) rescans
//                the lattice, builds a coarse Delta S histogram and picks a
//                safe floor bin;
//   k_fb_append (same condition) rescans and appends from that bin up;
//   k_hist      builds a 4096-bucket histogram of the candidate keys and
//                finds the boundary bucket holding the k-th largest key;
//   k_fix       writes f* at candidates above the boundary bucket and
//                resolves the boundary bucket exactly by a radix select on
//                (key descending, site index ascending).
// The last workgroup of each kernel (atomic ticket) does its serial part.
#include "lbm_site.h"

namespace lbm {

template <class R> struct KeyTraits;
template <> struct KeyTraits<float> {
  static constexpr int bits = 32;
  static constexpr unsigned long long quarter = 2ull << 23;   // Delta S / 4
};
template <> struct KeyTraits<double> {
  static constexpr int bits = 64;
  static constexpr unsigned long long quarter = 2ull << 52;
};

__device__ __forceinline__ unsigned int coarse_bin(float v) {
  const uint32_t u = v != v ? 0x7f800000u : __float_as_uint(v);
  const uint32_t b = u >> 19;  // exponent and 4 mantissa bits: 0 .. 4080 for v >= 0
  return b < (uint32_t)kCoarse ? b : 0u;
}
__device__ __forceinline__ unsigned long long ld_acq(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned int ld_acq(const unsigned int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Returns true in every thread of the last workgroup to arrive.
__device__ __forceinline__ bool last_block(unsigned int* ticket) {
  __shared__ bool is_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) is_last = atomicAdd(ticket, 1u) == gridDim.x - 1;
  __syncthreads();
  if (is_last) __threadfence();
  return is_last;
}

template <class R>
__device__ __forceinline__ bool need_rescan(const SelState* st, long long k, long long cap) {
  const unsigned long long n = st->count;
  return n > (unsigned long long)cap || ((long long)n < k && st->floor_raised);
}

template <class R>
__device__ __forceinline__ unsigned long long delta_key(R delta) {
  return delta <= R(0) ? 0ull : (unsigned long long)key_of<R>(delta);
}

// ---------------------------------------------------------------------------
template <class S, int Q>
__global__ __launch_bounds__(256) void k_fb_scan(const StepArgs<typename StoreT<S>::R> A,
                                                 long long k, unsigned int* coarse) {
  using R = typename StoreT<S>::R;
  SelState* st = A.sel;
  if (!need_rescan<R>(st, k, A.cap)) return;
  __shared__ unsigned int h[kCoarse];
  for (int i = threadIdx.x; i < kCoarse; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const long long n = (long long)A.nx * A.ny;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(s / A.nx), x = (int)(s % A.nx);
    R v[Q], feq[Q], d[Q], m0, ux, uy;
    const R dS = site_prep<S, Q>(A, x, y, v, feq, d, m0, ux, uy, true);
    if (dS > A.ehr_delta) atomicAdd(&h[coarse_bin((float)dS)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kCoarse; i += blockDim.x)
    if (h[i]) atomicAdd(&coarse[i], h[i]);
  if (!last_block(&st->ticket)) return;
  // Serial part: the coarse bin that holds the k-th largest Delta S.
  if (threadIdx.x == 0) {
    unsigned long long cum = 0;
    int b = kCoarse - 1;
    for (; b > 0; --b) {
      cum += ld_acq(&coarse[b]);
      if (cum >= (unsigned long long)k) break;
    }
    if (b == 0) cum += ld_acq(&coarse[0]);
    st->fb_bin = b;
    st->fallback = 1;
    st->fallbacks += 1;
    if (cum > (unsigned long long)A.cap) st->overflows += 1;
    st->count = 0;
    st->max_key = 0;
    st->ticket = 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kCoarse; i += blockDim.x) coarse[i] = 0;
}

template <class S, int Q>
__global__ __launch_bounds__(256) void k_fb_append(const StepArgs<typename StoreT<S>::R> A) {
  using R = typename StoreT<S>::R;
  using K = typename KeyOf<R>::T;
  SelState* st = A.sel;
  if (!st->fallback) return;
  const unsigned int fb = (unsigned int)st->fb_bin;
  const long long n = (long long)A.nx * A.ny;
  const long long nthreads = (long long)gridDim.x * blockDim.x;
  const long long iters = (n + nthreads - 1) / nthreads;
  for (long long it = 0; it < iters; ++it) {
    const long long s = it * nthreads + (long long)blockIdx.x * blockDim.x + threadIdx.x;
    bool is_c = false;
    R dS = R(0), m0 = R(0), ux = R(0), uy = R(0);
    int x = 0, y = 0;
    if (s < n) {
      y = (int)(s / A.nx);
      x = (int)(s % A.nx);
      R v[Q], feq[Q], d[Q];
      dS = site_prep<S, Q>(A, x, y, v, feq, d, m0, ux, uy, true);
      is_c = (dS > A.ehr_delta) && coarse_bin((float)dS) >= fb;
    }
    const unsigned long long mask = __ballot(is_c);
    if (!mask) continue;
    const int lane = __lane_id();
    const int leader = __ffsll((long long)mask) - 1;
    const K key = key_of<R>(dS);
    unsigned long long kmax = is_c ? (unsigned long long)key : 0ull;
    for (int off = 32; off > 0; off >>= 1) {
      const unsigned long long o = __shfl_xor(kmax, off);
      kmax = o > kmax ? o : kmax;
    }
    unsigned long long base = 0;
    if (lane == leader) {
      base = atomicAdd(&st->count, (unsigned long long)__popcll(mask));
      atomicMax(&st->max_key, kmax);
    }
    base = __shfl(base, leader);
    if (is_c) {
      const unsigned long long pos =
          base + (unsigned long long)__popcll(mask & ((1ull << lane) - 1ull));
      if (pos < (unsigned long long)A.cap) {
        A.cand_key[pos] = key;
        A.cand_idx[pos] = (uint32_t)(y * A.nx + x);
        A.cand_mom[pos] = m0;
        A.cand_mom[A.cap + pos] = ux;
        A.cand_mom[2 * A.cap + pos] = uy;
      }
    }
  }
}

// Lower edge of the candidate keys and the bucket width for this step.
template <class R>
__device__ __forceinline__ void bucket_frame(const SelState* st, R delta,
                                             unsigned long long& base, unsigned int& shift) {
  if (st->fallback) {
    const float edge = __uint_as_float(((uint32_t)st->fb_bin) << 19);
    base = (unsigned long long)key_of<R>((R)edge);
  } else {
    base = st->floor_raised ? st->floor_key : delta_key<R>(delta);
  }
  const unsigned long long mx = st->max_key;
  const unsigned long long span = mx > base ? mx - base : 0ull;
  shift = 0;
  while (shift < 62 && (span >> shift) >= (unsigned long long)kBuckets) ++shift;
}

__device__ __forceinline__ int bucket_of(unsigned long long key, unsigned long long base,
                                         unsigned int shift) {
  if (key < base) return 0;
  const unsigned long long b = (key - base) >> shift;
  return b >= (unsigned long long)kBuckets ? kBuckets - 1 : (int)b;
}

template <class R>
__global__ __launch_bounds__(256) void k_hist(const StepArgs<R> A, long long k,
                                              long long n_sites, unsigned int* hist) {
  SelState* st = A.sel;
  const unsigned long long nc_all = st->count;
  const long long nc = (long long)(nc_all < (unsigned long long)A.cap ? nc_all : A.cap);
  unsigned long long base;
  unsigned int shift;
  bucket_frame<R>(st, A.ehr_delta, base, shift);
  __shared__ unsigned int h[kBuckets];
  for (int i = threadIdx.x; i < kBuckets; i += blockDim.x) h[i] = 0;
  __syncthreads();
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < nc;
       p += (long long)gridDim.x * blockDim.x)
    atomicAdd(&h[bucket_of((unsigned long long)A.cand_key[p], base, shift)], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < kBuckets; i += blockDim.x)
    if (h[i]) atomicAdd(&hist[i], h[i]);
  if (!last_block(&st->ticket)) return;
  if (threadIdx.x == 0) {
    const long long need = k < nc ? k : nc;
    int boundary = -1;
    long long take = 0;
    if (nc > k && k > 0) {
      unsigned long long cum = 0;
      for (int b = kBuckets - 1; b >= 0; --b) {
        const unsigned long long c = ld_acq(&hist[b]);
        if (cum + c >= (unsigned long long)need) {
          boundary = b;
          take = need - (long long)cum;
          break;
        }
        cum += c;
      }
    } else if (k <= 0) {
      boundary = kBuckets;  // take nothing
    }
    st->boundary = boundary;
    st->take = take;
    st->base_key = base;
    st->shift = shift;
    // Floor for the next step: keep about 2k candidates (never raised when
    // the buffer can hold every site).
    const unsigned long long dk = delta_key<R>(A.ehr_delta);
    unsigned long long fnext = dk;
    if (A.cap < n_sites && k > 0) {
      const unsigned long long target = 2ull * (unsigned long long)k;
      unsigned long long cum = 0;
      int t = -1;
      for (int b = kBuckets - 1; b >= 0; --b) {
        cum += ld_acq(&hist[b]);
        if (cum >= target) { t = b; break; }
      }
      if (t >= 0) fnext = base + ((unsigned long long)t << shift);
      else fnext = base > KeyTraits<R>::quarter ? base - KeyTraits<R>::quarter : 0ull;
      if (fnext < dk) fnext = dk;
    }
    st->floor_key = fnext;
    st->floor_raised = fnext > dk ? 1 : 0;
    st->ticket = 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kBuckets; i += blockDim.x) hist[i] = 0;
}

template <class S, int Q>
__device__ __forceinline__ void write_feq(const StepArgs<typename StoreT<S>::R>& A, long long p) {
  using R = typename StoreT<S>::R;
  constexpr bool SH = StoreT<S>::shifted;
  const uint32_t idx = A.cand_idx[p];
  const int y = (int)(idx / (uint32_t)A.nx), x = (int)(idx % (uint32_t)A.nx);
  R feq[Q];
  equilibrium_v<R, Q, SH>(A.cand_mom[p], A.rho0, A.cand_mom[A.cap + p],
                          A.cand_mom[2 * A.cap + p], A.eq_kind, feq);
  S* dst = (S*)A.dst;
#pragma unroll
  for (int i = 0; i < Q; ++i)
    StoreT<S>::st(dst + (long long)i * A.qs + (long long)y * A.pitch + x, feq[i]);
}

template <class S, int Q>
__global__ __launch_bounds__(1024) void k_fix(const StepArgs<typename StoreT<S>::R> A,
                                              long long k, int32_t* selected, uint32_t* blist,
                                              long long* n_sel_out) {
  using R = typename StoreT<S>::R;
  SelState* st = A.sel;
  const unsigned long long nc_all = st->count;
  const long long nc = (long long)(nc_all < (unsigned long long)A.cap ? nc_all : A.cap);
  const int boundary = st->boundary;
  const unsigned long long base = st->base_key;
  const unsigned int shift = st->shift;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < nc;
       p += (long long)gridDim.x * blockDim.x) {
    const int b = bucket_of((unsigned long long)A.cand_key[p], base, shift);
    if (boundary < 0 || b > boundary) {
      write_feq<S, Q>(A, p);
      const unsigned long long slot = atomicAdd((unsigned long long*)&st->n_sel, 1ull);
      if (slot < (unsigned long long)k) selected[slot] = (int32_t)A.cand_idx[p];
    } else if (b == boundary) {
      const unsigned long long q = atomicAdd(&st->bcount, 1ull);
      if (q < (unsigned long long)kBoundaryCap) blist[q] = (uint32_t)p;
    }
  }
  if (!last_block(&st->ticket)) return;

  // Boundary bucket: take the `take` largest (key desc, index asc) by an MSD
  // radix select over 8-bit digits of the key, then of the complemented index.
  __shared__ unsigned int dh[256];
  __shared__ unsigned long long s_key_pref;
  __shared__ uint32_t s_idx_pref;
  __shared__ long long s_need;
  const long long m_all = (long long)ld_acq(&st->bcount);
  const long long m = m_all < kBoundaryCap ? m_all : kBoundaryCap;
  long long take = st->take;
  if (boundary >= 0 && boundary < kBuckets && take > 0) {
    if (threadIdx.x == 0) { s_key_pref = 0; s_idx_pref = 0; s_need = take; }
    constexpr int KB = KeyTraits<R>::bits;
    // digits: KB/8 of the key then 4 of ~index, most significant first
    for (int dgt = 0; dgt < KB / 8 + 4; ++dgt) {
      for (int i = threadIdx.x; i < 256; i += blockDim.x) dh[i] = 0;
      __syncthreads();
      const bool on_key = dgt < KB / 8;
      const int shiftb = on_key ? KB - 8 * (dgt + 1) : 32 - 8 * (dgt - KB / 8 + 1);
      const unsigned long long kp = s_key_pref;
      const uint32_t ip = s_idx_pref;
      for (long long q = threadIdx.x; q < m; q += blockDim.x) {
        const uint32_t p = blist[q];
        const unsigned long long key = (unsigned long long)A.cand_key[p];
        const uint32_t ni = ~A.cand_idx[p];
        bool match;
        unsigned int digit;
        if (on_key) {
          const unsigned long long hi_mask = dgt == 0 ? 0ull : (~0ull << (shiftb + 8)) & (KB == 64 ? ~0ull : 0xffffffffull);
          match = (key & hi_mask) == (kp & hi_mask);
          digit = (unsigned int)((key >> shiftb) & 0xffu);
        } else {
          const uint32_t hi_mask = (shiftb + 8 >= 32) ? 0u : (~0u << (shiftb + 8));
          match = key == kp && (ni & hi_mask) == (ip & hi_mask);
          digit = (ni >> shiftb) & 0xffu;
        }
        if (match) atomicAdd(&dh[digit], 1u);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        long long need = s_need, cum = 0;
        int dsel = 0;
        for (int dd = 255; dd >= 0; --dd) {
          if (cum + (long long)dh[dd] >= need) { dsel = dd; break; }
          cum += dh[dd];
        }
        s_need = need - cum;
        if (on_key) s_key_pref |= ((unsigned long long)dsel) << shiftb;
        else s_idx_pref |= ((uint32_t)dsel) << shiftb;
      }
      __syncthreads();
    }
    const unsigned long long tk = s_key_pref;
    const uint32_t ti = s_idx_pref;
    for (long long q = threadIdx.x; q < m; q += blockDim.x) {
      const uint32_t p = blist[q];
      const unsigned long long key = (unsigned long long)A.cand_key[p];
      const uint32_t ni = ~A.cand_idx[p];
      if (key > tk || (key == tk && ni >= ti)) {
        write_feq<S, Q>(A, p);
        const unsigned long long slot = atomicAdd((unsigned long long*)&st->n_sel, 1ull);
        if (slot < (unsigned long long)k) selected[slot] = (int32_t)A.cand_idx[p];
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (n_sel_out) *n_sel_out = ld_acq((const unsigned long long*)&st->n_sel);
    if (m_all > kBoundaryCap) st->overflows += 1;
    st->count = 0;
    st->max_key = 0;
    st->bcount = 0;
    st->fallback = 0;
    st->ticket = 0;
  }
}

// Reset of the per-step selection counter before a step's fix-up.
__global__ void k_sel_begin(SelState* st) {
  st->n_sel = 0;
}

template <class S, int Q>
static hipError_t launch_select_t(const SelectArgs& a, hipStream_t s) {
  using R = typename StoreT<S>::R;
  const StepArgs<R>& A = *(const StepArgs<R>*)a.step_args;
  hipLaunchKernelGGL((k_fb_scan<S, Q>), dim3(512), dim3(256), 0, s, A, a.k, a.coarse);
  hipLaunchKernelGGL((k_fb_append<S, Q>), dim3(512), dim3(256), 0, s, A);
  hipLaunchKernelGGL((k_hist<R>), dim3(128), dim3(256), 0, s, A, a.k, a.n_sites, a.hist);
  hipLaunchKernelGGL(k_sel_begin, dim3(1), dim3(1), 0, s, A.sel);
  hipLaunchKernelGGL((k_fix<S, Q>), dim3(64), dim3(1024), 0, s, A, a.k, a.selected,
                     (uint32_t*)a.boundary_idx, a.n_sel_out);
  return hipGetLastError();
}

hipError_t launch_select(const SelectArgs& a, hipStream_t s) {
  switch (a.storage * 16 + a.Q) {
    case 0 * 16 + 9: return launch_select_t<double, 9>(a, s);
    case 0 * 16 + 3: return launch_select_t<double, 3>(a, s);
    case 1 * 16 + 9: return launch_select_t<float, 9>(a, s);
    case 1 * 16 + 3: return launch_select_t<float, 3>(a, s);
    case 2 * 16 + 9: return launch_select_t<_Float16, 9>(a, s);
    case 2 * 16 + 3: return launch_select_t<_Float16, 3>(a, s);
    case 3 * 16 + 9: return launch_select_t<bf16_t, 9>(a, s);
    default: return launch_select_t<bf16_t, 3>(a, s);
  }
}

}  // namespace lbm
