// The D3Q27 step on a periodic lattice for gfx950:
//   pull-stream (section 2, free flight)
//   -> moments and the product equilibrium (section 6's 1D equilibria)
//   -> median entropy filter over the 27-site neighbourhood (section 4: the
//      14th of the 27 sorted Delta S values)
//   -> LBGK collision (eq. CollisionIntegral) -> positivity rule (section 4)
//   -> store into the second lattice.
// Without the median filter every lane takes one site of a 256-site row
// segment.  With it, a workgroup takes a TX x TY column of sites and marches
// along z through ZC layers, keeping Delta S of three layers (the tile plus
// a one-site halo) in an LDS ring: each layer's Delta S is evaluated once
// per column, not once per neighbour.
#include <hip/hip_ext.h>

#include "lbm_collide.h"
#include "lbm_internal.h"
#include "lbm_site3.h"

namespace lbm {

// g mod n for the tile and halo coordinates, which lie within one lattice
// width of [0, n) unless the lattice is narrower than a tile (then the
// remainder)
__device__ __forceinline__ int wrap_mod(int g, int n) {
  const int r = g < 0 ? g + n : (g >= n ? g - n : g);
  return (r < 0 || r >= n) ? ((g % n) + n) % n : r;
}

// After the filter: LBGK, the positivity rule, the store.
template <class S>
__device__ __forceinline__ void finish27(const StepArgs<typename StoreT<S>::R>& A, unsigned off,
                                         bool valid, typename StoreT<S>::R v[27],
                                         typename StoreT<S>::R feq[27], unsigned long long* cnt) {
  using R = typename StoreT<S>::R;
  bool pos_event = false;
  if (valid) {
#pragma unroll
    for (int i = 0; i < 27; ++i) v[i] = v[i] + A.omega * (feq[i] - v[i]);   // collided in place
    if (A.positivity) {
      CollInfo<R> ci;
      positivity_site<S, 27>(A, feq, v, ci);
      pos_event = ci.pos_arg >= 0;
    }
    S* dst = (S*)A.dst;
#pragma unroll
    for (int i = 0; i < 27; ++i) StoreT<S>::st(at(dst + (long long)i * A.qs, off), v[i]);
  }
  if (A.positivity && A.count_events) count_event(pos_event, cnt + CNT_POSITIVITY);
}

template <class S>
__global__ __launch_bounds__(256) void k_step3(const StepArgs<typename StoreT<S>::R> A) {
  using R = typename StoreT<S>::R;
  constexpr bool SH = StoreT<S>::shifted;
  // workgroup -> (256-site segment of a row, row z * ny + y)
  const int segs = (A.nx + 255) / 256;
  const int row = (int)blockIdx.x / segs, x = ((int)blockIdx.x % segs) * 256 + (int)threadIdx.x;
  const int y = row % A.ny3, z = row / A.ny3;
  const bool valid = x < A.nx;
  unsigned long long* const cnt = A.counters + (blockIdx.x % kCntSlots) * CNT_N;
  R v[27], feq[27];
  if (valid) {
    R m0, ux, uy, uz;
    pull27<S>((const S*)A.src, A.qs, A.pitch, A.nx, A.ny3, A.nz, x, y, z, v);
    moments27<R, SH>(v, A.rho0, m0, ux, uy, uz);
    equilibrium27<R, SH>(m0, A.rho0, ux, uy, uz, A.eq_kind, feq);
  }
  finish27<S>(A, (unsigned)(row * A.pitch + x), valid, v, feq, cnt);
}

template <class R>
__device__ __forceinline__ void cswap(R& a, R& b) {
  const R lo = fmin(a, b), hi = fmax(a, b);
  a = lo;
  b = hi;
}

// The 14th smallest of 27 values by forgetful selection: a window of 15
// values; each round moves the window's minimum to its first slot and its
// maximum to its last, drops both (neither can be the median of the values
// not yet dropped) and takes the next value into the last slot.  After
// twelve rounds three values remain, and their middle one is the median.
// All indices are compile-time, so the array stays in registers.
template <class R>
__device__ __forceinline__ R median27(R a[27]) {
#pragma unroll
  for (int r = 0; r < 13; ++r) {
#pragma unroll
    for (int k = r + 1; k < 15; ++k) cswap(a[r], a[k]);        // minimum -> a[r]
#pragma unroll
    for (int k = r + 1; k < 14; ++k) cswap(a[k], a[14]);       // maximum -> a[14]
    if (r < 12) a[14] = a[15 + r];
  }
  return a[13];
}

template <class S, int TX, int TY, int ZC>
__global__ __launch_bounds__(TX * TY, (sizeof(typename StoreT<S>::R) == 4 && TX * TY <= 512) ? 4 : 1) void k_step3_median(const StepArgs<typename StoreT<S>::R> A,
                                                          int tiles_x, int tiles_y) {
  using R = typename StoreT<S>::R;
  constexpr bool SH = StoreT<S>::shifted;
  constexpr int NT = TX * TY, SW = TX + 2, NS = (TX + 2) * (TY + 2);
  __shared__ R ring[3][NS];

  // Workgroup -> (tile, chunk of layers).  Consecutive workgroups are dealt
  // round-robin to the 8 XCDs; each XCD takes a contiguous band of tiles
  // (neighbouring rows of tiles in the same layers), whose halos it reads
  // from its own L2.
  const int T = tiles_x * tiles_y * ((A.nz + ZC - 1) / ZC);
  const int b = blockIdx.x;
  const int tb = (T % 8 == 0) ? (b % 8) * (T / 8) + b / 8 : b;
  const int tile_x = tb % tiles_x, tile_y = (tb / tiles_x) % tiles_y, chunk = tb / (tiles_x * tiles_y);
  const int x0 = tile_x * TX, y0 = tile_y * TY, z0 = chunk * ZC;
  const int z1 = min(z0 + ZC, A.nz);
  const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
  const int x = x0 + lx, y = y0 + ly;
  const bool valid = x < A.nx && y < A.ny3;
  unsigned long long* const cnt = A.counters + (b % kCntSlots) * CNT_N;

  // Delta S of layer z (periodic) over the tile and its halo into ring slot
  // `slot`; positions beyond the lattice wrap, so ragged tiles need no
  // special case.
  auto layer = [&](int z, int slot) {
    const int zz = wrap_mod(z, A.nz);
#pragma unroll 1
    for (int s = tid; s < NS; s += NT) {
      const int gx = wrap_mod(x0 + s % SW - 1, A.nx), gy = wrap_mod(y0 + s / SW - 1, A.ny3);
      R v[27], d[27], m0, ux, uy, uz;
      pull27<S, true>((const S*)A.src, A.qs, A.pitch, A.nx, A.ny3, A.nz, gx, gy, zz, v);
      moments27<R, SH>(v, A.rho0, m0, ux, uy, uz);
      equilibrium27<R, SH>(m0, A.rho0, ux, uy, uz, A.eq_kind, d);
#pragma unroll
      for (int i = 0; i < 27; ++i) d[i] -= v[i];                      // f* - f
      ring[slot][s] = site_dS_q<R, 27, SH>(v, d, m0, A.rho0, ux, uy, uz, A.eq_kind, R(0));
    }
  };

  layer(z0 - 1, 2);
  layer(z0, 0);
  for (int z = z0; z < z1; ++z) {
    const int sc = (z - z0) % 3, sm = (z - z0 + 2) % 3, sp = (z - z0 + 1) % 3;
    layer(z + 1, sp);
    __syncthreads();
    // The median decision first, from LDS alone (the site's own state is
    // not yet live): median < Delta S exactly when at least 14 of the 27
    // values lie below Delta S; wavefronts without a site above delta skip
    // the count, and only wavefronts with an accepted site select the 14th.
    const R dS = valid ? ring[sc][(ly + 1) * SW + lx + 1] : R(0);
    const bool cand = valid && (dS > A.med_delta) && (dS < r_inf<R>());
    bool acc = false;
    R med = R(0);
    auto nbr = [&](int k) {
      const int dz = k / 9 - 1, dy = (k / 3) % 3 - 1, dx = k % 3 - 1;
      return ring[dz < 0 ? sm : (dz > 0 ? sp : sc)][(ly + 1 + dy) * SW + lx + 1 + dx];
    };
    if (__ballot(cand)) {
      int below = 0;
#pragma unroll
      for (int k = 0; k < 27; ++k) below += nbr(k) < dS ? 1 : 0;
      acc = cand && below >= 14;
      if (__ballot(acc)) {
        R nb[27];
#pragma unroll
        for (int k = 0; k < 27; ++k) nb[k] = nbr(k);
        med = median27<R>(nb);
      }
    }
    // every lane pulls (a lane past the lattice edge an in-range site that
    // it does not store), so that nothing stays undefined from one layer to
    // the next: the compiler would otherwise carry those values through the
    // next layer's Delta S and run out of registers
    R v[27], feq[27], m0, ux, uy, uz;
    pull27<S, true>((const S*)A.src, A.qs, A.pitch, A.nx, A.ny3, A.nz, valid ? x : x0, valid ? y : y0, z, v);
    moments27<R, SH>(v, A.rho0, m0, ux, uy, uz);
    equilibrium27<R, SH>(m0, A.rho0, ux, uy, uz, A.eq_kind, feq);
    if (acc) {
      const R c = sqrt(med / dS);
#pragma unroll
      for (int i = 0; i < 27; ++i) v[i] = feq[i] + c * (v[i] - feq[i]);
    }
    if (A.count_events) count_event(acc, cnt + CNT_MEDIAN);
    finish27<S>(A, (unsigned)((z * A.ny3 + y) * A.pitch + x), valid, v, feq, cnt);
    __syncthreads();   // the next layer overwrites the ring slot of z - 1
  }
}

// ---------------------------------------------------------------------------
template <class S>
static hipError_t launch3(bool median, const void* args, hipStream_t s, hipEvent_t e0,
                          hipEvent_t e1) {
  using R = typename StoreT<S>::R;
  const StepArgs<R>& A = *(const StepArgs<R>*)args;
  if (median) {
    // 64 x 8 columns of 32 layers: 1.29 halo sites per site, 1.06 layers
    // per layer (FP32 arithmetic: 64 x 16 tiles measured no faster)
    constexpr int TX = 64, TY = 8, ZC = sizeof(R) == 4 ? 32 : 16;
    const int tx = (A.nx + TX - 1) / TX, ty = (A.ny3 + TY - 1) / TY;
    const dim3 grid(tx * ty * ((A.nz + ZC - 1) / ZC)), block(TX * TY);
    auto kern = k_step3_median<S, TX, TY, ZC>;
    if (e0 && e1) hipExtLaunchKernelGGL(kern, grid, block, 0, s, e0, e1, 0, A, tx, ty);
    else hipLaunchKernelGGL(kern, grid, block, 0, s, A, tx, ty);
  } else {
    const dim3 grid((unsigned)((A.nx + 255) / 256 * (long long)A.ny3 * A.nz)), block(256);
    if (e0 && e1) hipExtLaunchKernelGGL(k_step3<S>, grid, block, 0, s, e0, e1, 0, A);
    else hipLaunchKernelGGL(k_step3<S>, grid, block, 0, s, A);
  }
  return hipGetLastError();
}

hipError_t launch_step3(int storage, bool median, const void* args, hipStream_t s, hipEvent_t e0,
                        hipEvent_t e1) {
  switch (storage) {
    case 0: return launch3<double>(median, args, s, e0, e1);
    case 1: return launch3<float>(median, args, s, e0, e1);
    case 2: return launch3<_Float16>(median, args, s, e0, e1);
    default: return launch3<bf16_t>(median, args, s, e0, e1);
  }
}

}  // namespace lbm
