// Fused per-site step of the regularised LBM for gfx950 (one thread per
// site, 256-thread workgroups of 64-wide wavefronts):
//   pull-stream with boundaries (section 2, free flight)
//   -> moments and equilibrium (sections 2, 6, 8)
//   -> nonequilibrium entropy (section 4, eq. DelS) when a limiter needs it
//   -> median entropy filter (section 4), Delta S of the tile and a one-site
//      halo staged in LDS
//   -> collision: LBGK (eq. CollisionIntegral), MRT (section 5) or ELBM
//      (section 3)
//   -> positivity rule (section 4)
//   -> store into the second lattice, and append Ehrenfest candidates
//      (section 4) for the selection kernels.
#include "lbm_device.h"
#include "lbm_internal.h"
#include <hip/hip_ext.h>

#include "lbm_collide.h"

namespace lbm {

template <class R>
__device__ __forceinline__ void sort_net9(R a[9]) {
#pragma unroll
  for (int pass = 0; pass < 9; ++pass) {
#pragma unroll
    for (int j = pass & 1; j + 1 < 9; j += 2) {
      const R lo = fmin(a[j], a[j + 1]), hi = fmax(a[j], a[j + 1]);
      a[j] = lo;
      a[j + 1] = hi;
    }
  }
}

// Sites of an FP32 ELBM step that need the FP64 root solve, listed by the
// step kernel (alpha_max < f64_below: near the no-root branch, where
// alpha = alpha_max = f_a / (f_a - f*_a) hangs on a small population and the
// FP32 forms' absolute rounding of the shifted representation, about
// ulp(w_a rho0), would move it by a relative 1e-4).  Each is rebuilt from the
// source lattice in FP64: the stored values (exact in FP64) plus w_i rho0,
// moments, entropic f*, the root solve, the collision and the positivity
// rule, rounded only when stored; its counters and adjoint records are
// taken as the step kernel would have.  The last workgroup clears the list:
// every workgroup has used the list length (its loop bounds) before it
// takes its ticket, and nothing else that a workgroup wrote is read here,
// so no device-scope fence is needed (on gfx950 one writes back the XCD's
// L2).
template <class S, int Q>
__global__ __launch_bounds__(256) void k_elbm_f64(const StepArgs<typename StoreT<S>::R> A) {
  using R = typename StoreT<S>::R;
  constexpr bool SH = StoreT<S>::shifted;
  const unsigned int n = A.f64_count[0];
  unsigned long long* const cnt = A.counters + (blockIdx.x % kCntSlots) * CNT_N;
  // 16 sites per workgroup, one per group of 16 lanes: every lane of the
  // group rebuilds the site, lane c takes component c into the group's
  // root solve, and lane 0 collides, limits and stores it.
  const unsigned int grp = threadIdx.x / 16, c = threadIdx.x % 16;
  const double rho0 = (double)A.rho0;
  for (unsigned int b0 = blockIdx.x * 16u; b0 < n; b0 += gridDim.x * 16u) {
    const unsigned int i = b0 + grp;
    const bool on = i < n;
    const uint32_t idx = on ? A.f64_sites[i] : 0u;
    const int x = (int)(idx % (uint32_t)A.nx), y = (int)(idx / (uint32_t)A.nx);
    double f[Q], q[Q];
    ElbmGroupResult r{2.0, EB_CUTOFF, 0};
    if (on) {
      R v[Q];
      pull<S, Q>((const S*)A.src, A.qs, A.pitch, A.nx, A.ny, A.bc, x, y, A.lid, v);
#pragma unroll
      for (int k = 0; k < Q; ++k) f[k] = (double)v[k] + (SH ? wt<double, Q>(k) * rho0 : 0.0);
      double m0, ux, uy;
      moments_v<double, Q, false>(f, rho0, m0, ux, uy);
      equilibrium_v<double, Q, false>(m0, rho0, ux, uy, EQ_ENTROPIC, q);
      double f_c = 1.0, q_c = 1.0;
#pragma unroll
      for (int k = 0; k < Q; ++k)
        if ((int)c == k) { f_c = f[k]; q_c = q[k]; }
      r = elbm_alpha_fp64_group(f_c, q_c, (int)c < Q, A.eps64, A.dS_cut64, A.max_iter, A.norm,
                                A.fallback);
    }
    const bool mine = on && c == 0;
    bool pos_event = false;
    if (mine) {
      const long long o = (long long)y * A.pitch + x;
      const double om = A.omega_field ? (double)A.omega_field[o] : (double)A.omega;
      const double ab = r.alpha * (om * 0.5);
      double post[Q];
#pragma unroll
      for (int k = 0; k < Q; ++k) post[k] = f[k] + ab * (q[k] - f[k]);
      if (A.positivity) {
        // positivity rule (section 4) in FP64
        double phi = __builtin_huge_val();
        int arg = -1;
#pragma unroll
        for (int k = 0; k < Q; ++k)
          if (post[k] < 0.0 && q[k] > 0.0) {
            const double t = q[k] / (q[k] - post[k]);
            if (t < phi) { phi = t; arg = k; }
          }
        if (arg >= 0) {
#pragma unroll
          for (int k = 0; k < Q; ++k) post[k] = (k == arg) ? 0.0 : q[k] + phi * (post[k] - q[k]);
          pos_event = true;
        }
      }
      S* dst = (S*)A.dst;
#pragma unroll
      for (int k = 0; k < Q; ++k)
        StoreT<S>::st(at(dst + (long long)k * A.qs, (unsigned)o),
                      (R)(post[k] - (SH ? wt<double, Q>(k) * rho0 : 0.0)));
      if (A.alpha_out) {
        A.alpha_out[o] = (R)r.alpha;
        A.branch_out[o] = (unsigned char)r.branch;
      }
    }
    if (A.count_events) {
      count_event(mine && r.branch == EB_NOROOT, cnt + CNT_ELBM_NOROOT);
      count_event(mine, cnt + CNT_ELBM_F64);
      count_event(mine && r.branch == EB_NONPOS, cnt + CNT_ELBM_NONPOS);
      count_sum(mine ? r.iters : 0, cnt + CNT_ELBM_ITERS);
      if (A.positivity) count_event(pos_event, cnt + CNT_POSITIVITY);
    }
  }
  __shared__ bool last;
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(&A.f64_count[1], 1u) == gridDim.x - 1;
  __syncthreads();
  if (last && threadIdx.x == 0) {
    A.f64_count[0] = 0;
    A.f64_count[1] = 0;
  }
}

// LBGK in FP32/16-bit storage on row tiles fits 64 registers: keep the full
// occupancy of 8 wavefronts per SIMD (the compiler would otherwise take a few
// more).
// ENS: the ensemble or smooth limiter of section 4 acts on the pulled state
// (f* + phi (f - f*), phi from the site's Delta S and the step's threshold
// and mean), and the workgroup adds the dissipation monitor's sums.
// NB (median filter only): the workgroup takes NB tiles stacked vertically
// (TX x NB TY sites, 256 NB threads) and shares one LDS tile of Delta S
// with a one-site halo: 156 halo sites per 768 with NB = 3 against 140 per
// 256, whose populations are pulled a second time.  Each wavefront keeps
// the candidate region of its own 256-site tile.
template <class S, int Q, int COLL, bool MEDIAN, int TX, int TY, bool PER, bool ENS = false,
          int NB = 1>
__global__ __launch_bounds__(256 * NB, ((COLL == COLL_LBGK && sizeof(S) <= 4 && !MEDIAN && !ENS && TX == 256) ? 8 : 1))
void k_step(const StepArgs<typename StoreT<S>::R> A) {
  using R = typename StoreT<S>::R;
  constexpr bool SH = StoreT<S>::shifted;
  static_assert(TX * TY == 256, "tile must hold 256 sites");
  static_assert(NB == 1 || MEDIAN, "stacked tiles serve the median filter's halo");

  // Tile order.  Consecutive workgroups are dealt round-robin to the 8
  // XCDs.  The median filter re-reads its halo, so each XCD gets a
  // contiguous band of tiles (the rows above and below a tile in the same
  // L2).  Otherwise every population is read once and the loads bypass the
  // caches: tiles nearly in launch order, all XCDs streaming the same
  // stretch of the lattice (measured 5 % (FP32) and 10 % (FP64) faster
  // than the bands).  With 4-byte storage each XCD takes pairs of
  // horizontally adjacent tiles, which share the line the pull reaches
  // across their edge (2 % faster again; FP64 gains nothing from pairs).
  const int T = A.tiles_x * ((A.tiles_y + NB - 1) / NB);   // workgroups
  const int b = blockIdx.x;
  constexpr int G = sizeof(S) == 4 ? 2 : 1;
  const int tb = (MEDIAN && T % 8 == 0) ? (b % 8) * (T / 8) + b / 8
               : ((T % (8 * G) == 0) ? (b / (8 * G)) * (8 * G) + (b % 8) * G + (b / 8) % G : b);
  const int sub = (int)threadIdx.x / 256, tid = (int)threadIdx.x % 256;
  const int tile_x = tb % A.tiles_x, tile_y = (tb / A.tiles_x) * NB + sub;
  const int t = tile_y * A.tiles_x + tile_x;   // this thread's 256-site tile
  const int lx = tid % TX, ly = tid / TX;
  const int x = tile_x * TX + lx, y = tile_y * TY + ly;
  const bool valid = x < A.nx && y < A.ny;
  const bool wall = valid && !PER && on_wall<typename StoreT<S>::R>(A, x, y);

  unsigned long long* const cnt = A.counters + (blockIdx.x % kCntSlots) * CNT_N;
  const bool need_dS = MEDIAN || ENS || A.ehrenfest;
  // Sites provably below the Ehrenfest floor skip the exact Delta S; with
  // the median filter, sites provably below delta as well (below both,
  // a site is no candidate of either), and a workgroup that holds a
  // median candidate evaluates them exactly further down.
  const StepFrame fr = step_frame(A.sel);
  const R ehr_screen = A.ehrenfest ? value_of_key<R>(fr.floor) : r_inf<R>();
  const R screen = ENS ? R(0)
                       : (MEDIAN ? fmin(A.med_delta, ehr_screen) : (A.ehrenfest ? ehr_screen : R(0)));
  R v[Q], feq[Q], d[Q], m0 = R(0), ux = R(0), uy = R(0), dS = R(0);
  bool screened = false;
  // the median kernel's pulls are cached: its halo sites are pulled again,
  // here or by the neighbouring tiles
  if (valid)
    dS = site_prep<S, Q, PER, !PER, MEDIAN>(A, x, y, v, feq, d, m0, ux, uy, need_dS, screen,
                                            &screened);

  if constexpr (ENS) {
    double prod = 0.0, lim = 0.0, sdS = 0.0, nfin = 0.0;
    if (valid) {
      const EnsState* E = A.ens;
      const R t = (R)E->threshold;
      R phi;
      if (!(dS < r_inf<R>())) {
        phi = R(0);                               // a non-positive population: f*
      } else if (A.ens_mode == ENS_THRESHOLD) {   // eq. entrHom
        phi = dS >= t ? sqrt(t / (dS > R(0) ? dS : R(1))) : R(1);
      } else if (A.ens_mode == ENS_SMOOTH) {      // eq. phiExamp
        const R r = dS / (A.ens_alpha * (R)E->mean);
        phi = (R(1) + pow(r, A.ens_k - R(0.5))) / (R(1) + pow(r, A.ens_k));
      } else if (A.ens_mode == ENS_DOUBLE_MONOTONE) {  // eq. DoublMonSpec
        phi = pow(R(1) + pow(dS / t, A.ens_k), R(-0.5) / A.ens_k);
      } else {                                    // pointwise 1 / (1 + alpha Delta S^k)
        phi = R(1) / (R(1) + A.ens_alpha * pow(dS, A.ens_k));
      }
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        v[i] = feq[i] + phi * (v[i] - feq[i]);
        d[i] = feq[i] - v[i];
      }
      if (dS < r_inf<R>()) {
        const R om = A.omega_field ? A.omega_field[(long long)y * A.pitch + x] : A.omega;
        prod = (1.0 - ((double)om - 1.0) * ((double)om - 1.0)) * (double)dS;
        lim = (1.0 - (double)phi * (double)phi) * (double)dS;
        sdS = (double)dS;
        nfin = 1.0;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      prod += __shfl_xor(prod, o);
      lim += __shfl_xor(lim, o);
      sdS += __shfl_xor(sdS, o);
      nfin += __shfl_xor(nfin, o);
    }
    if (__lane_id() == 0) {
      double* acc = A.ens->step_acc[blockIdx.x % kEnsSlots];
      atomicAdd(&acc[0], prod);
      atomicAdd(&acc[1], lim);
      atomicAdd(&acc[2], sdS);
      atomicAdd(&acc[3], nfin);
    }
  }

  if constexpr (MEDIAN) {
    // Median entropy filter: Delta S of the tile plus a one-site halo in LDS.
    constexpr int HY = (Q == 9) ? 1 : 0;
    constexpr int SW = TX + 2, SH_ = TY * NB + 2 * HY;
    __shared__ R sdS[SH_ * SW];
    const int by = sub * TY + ly;                         // row within the workgroup
    const int x0 = tile_x * TX, y0 = (tb / A.tiles_x) * NB * TY;
    // only a site above delta can be filtered: a workgroup without one needs
    // neither the halo's Delta S nor the neighbourhoods
    const bool cand = valid && !wall && (dS > A.med_delta) && (dS < r_inf<R>());
    if (__syncthreads_or(cand)) {
      // the neighbourhoods need every Delta S exact
      if (screened) dS = site_dS<R, Q, SH>(v, d, m0, A.rho0, ux, uy, A.eq_kind, R(0));
      sdS[(by + HY) * SW + lx + 1] = valid ? (wall ? R(__builtin_nan("")) : dS) : slot_dS<S, Q, true>(A, x, y);
      constexpr int NHALO = SH_ * SW - TX * TY * NB;
      for (int s = threadIdx.x; s < NHALO; s += 256 * NB) {
        // halo slot s -> LDS coordinates: top row, bottom row, then the left
        // and right columns (2D); the two end slots of the single row (1D)
        int hx, hy;
        if constexpr (HY == 1) {
          if (s < SW) { hx = s; hy = 0; }
          else if (s < 2 * SW) { hx = s - SW; hy = SH_ - 1; }
          else { const int r = s - 2 * SW; hy = 1 + r / 2; hx = (r & 1) ? SW - 1 : 0; }
        } else {
          hy = 0;
          hx = (s == 0) ? 0 : SW - 1;
        }
        sdS[hy * SW + hx] = slot_dS<S, Q, true>(A, x0 + hx - 1, y0 + hy - HY);
      }
      __syncthreads();
      if (valid && !wall) {
        // wavefronts without a site above delta skip the neighbourhood's sort
        R med = R(0);
        if (__ballot(cand)) {
          R nb[9];
          int n = 0;
          constexpr int NN = (Q == 9) ? 9 : 3;
#pragma unroll
          for (int k = 0; k < NN; ++k) {
            const int dy = (Q == 9) ? k / 3 - 1 : 0, dx = (Q == 9) ? k % 3 - 1 : k - 1;
            const R val = sdS[(by + HY + dy) * SW + lx + 1 + dx];
            const bool in = !(val != val);
            n += in ? 1 : 0;
            nb[k] = in ? val : r_inf<R>();
          }
          if constexpr (Q == 9) {
            sort_net9<R>(nb);
            const int rank = (n + 1) / 2 - 1;
            med = nb[0];
#pragma unroll
            for (int k = 1; k < 9; ++k) med = rank == k ? nb[k] : med;
          } else {
            R a0 = fmin(nb[0], nb[1]), a1 = fmax(nb[0], nb[1]);
            const R a2 = fmax(a1, nb[2]);
            a1 = fmin(a1, nb[2]);
            const R b0 = fmin(a0, a1), b1 = fmax(a0, a1);
            (void)a2;
            med = ((n + 1) / 2 - 1) == 0 ? b0 : b1;
          }
        }
        const bool acc = cand & (med < dS);
        if (acc) {
          const R c = sqrt(med / dS);
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            v[i] = feq[i] + c * (v[i] - feq[i]);
            d[i] = feq[i] - v[i];
          }
        }
        if (A.count_events) count_event(acc, cnt + CNT_MEDIAN);
      } else if (A.count_events) {
        count_event(false, cnt + CNT_MEDIAN);
      }
    }
  }

  constexpr bool DEFER = COLL == COLL_ELBM && sizeof(R) == 4 && !MEDIAN && !ENS;
  site_finish<S, Q, COLL, true, DEFER>(A, x, y, valid, wall, (long long)t * 4 + tid / 64, v, feq, d,
                                       m0, ux, uy, dS, fr, cnt);
}

// The step on a periodic lattice without the median filter, in rows of 256
// sites: each workgroup takes ROWS consecutive rows of one 256-column strip,
// and with ROWS > 1 every thread issues the loads of its next row before it
// computes the current one (two rows of loads in flight per wavefront).
// Per-site arithmetic is the one-site kernel's, so the results are
// bit-identical.  Used for the 16-bit storage forms and for ELBM in FP32,
// with a compile-time variant without the Ehrenfest code.  16-bit LBGK is
// held to 64 registers (eight wavefronts per SIMD; the Ehrenfest variant
// would take 65 and run seven): three spilled values cost less than the
// lost wavefront (FP16 115.2 -> 112.3 us, BF16 133.6 -> 128.2 us at 4096^2
// with the limiter).
template <class S, int Q, int COLL, int ROWS, bool EHR>
__global__ __launch_bounds__(256, (COLL == COLL_LBGK && sizeof(S) == 2) ? 8 : 1) void k_step_rows(const StepArgs<typename StoreT<S>::R> A) {
  using R = typename StoreT<S>::R;
  constexpr bool SH = StoreT<S>::shifted;
  const int nyc = (A.ny + ROWS - 1) / ROWS;
  const int T = A.tiles_x * nyc;
  const int b = blockIdx.x;
  // Workgroups go round-robin to the 8 XCDs; each XCD takes pairs of
  // adjacent row segments, which share the line the pull reaches across
  // their edge (the last, incomplete group of 16 keeps launch order).  With
  // nontemporal loads this beats one contiguous band of rows per XCD:
  // FP16 108.4 -> 103.2 us, BF16 111.4 -> 107.3 us without limiters.
  const int t = (b / 16 * 16 + 16 <= T) ? (b / 16) * 16 + (b % 8) * 2 + (b / 8) % 2 : b;
  const int tile_x = t % A.tiles_x, y0 = (t / A.tiles_x) * ROWS;
  const int x = tile_x * 256 + (int)threadIdx.x;
  const bool valid = x < A.nx;
  const int xl = valid ? x : 0;
  const unsigned c[3] = {(unsigned)(xl == A.nx - 1 ? 0 : xl + 1), (unsigned)xl,
                         (unsigned)(xl == 0 ? A.nx - 1 : xl - 1)};   // source columns, a = -1, 0, +1
  unsigned long long* const cnt = A.counters + (blockIdx.x % kCntSlots) * CNT_N;
  const StepFrame fr = step_frame(A.sel);
  const R screen = (EHR && A.ehrenfest) ? value_of_key<R>(fr.floor) : R(0);
  const S* __restrict__ src = (const S*)A.src;

  auto load_row = [&](int y, S raw[Q]) {
    const int ym = y == 0 ? A.ny - 1 : y - 1, yp = y == A.ny - 1 ? 0 : y + 1;
    const unsigned r[3] = {(unsigned)(yp * A.pitch), (unsigned)(y * A.pitch),
                           (unsigned)(ym * A.pitch)};                // source rows, b = -1, 0, +1
#pragma unroll
    for (int i = 0; i < Q; ++i)
      raw[i] = StoreT<S>::raw(at(src + (long long)i * A.qs, r[vy_of<Q>(i) + 1] + c[vx_of<Q>(i) + 1]));
  };

  S nxt[Q];
  load_row(y0, nxt);
#pragma unroll 1
  for (int rr = 0; rr < ROWS; ++rr) {
    const int y = y0 + rr;
    if (y >= A.ny) break;                    // uniform over the workgroup
    S cur[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) cur[i] = nxt[i];
    if (rr + 1 < ROWS && y + 1 < A.ny) load_row(y + 1, nxt);
    R v[Q], feq[Q], d[Q], m0, ux, uy;
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = StoreT<S>::cvt(cur[i]);
    moments_v<R, Q, SH>(v, A.rho0, m0, ux, uy);
    R dx[3], dy[3];
    equilibrium_v<R, Q, SH>(m0, A.rho0, ux, uy, A.eq_kind, feq, dx, dy);
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = feq[i] - v[i];
    const R dS = (EHR && A.ehrenfest && valid)
                     ? site_dS_dev<R, Q, SH>(v, d, m0, A.rho0, dx, dy, dx, screen)
                     : R(0);
    const long long region = ((long long)y * A.tiles_x + tile_x) * 4 + threadIdx.x / 64;
    site_finish<S, Q, COLL, EHR, COLL == COLL_ELBM && sizeof(R) == 4>(A, x, y, valid, false, region,
                                                                       v, feq, d, m0, ux, uy, dS, fr,
                                                                       cnt);
  }
}

// ---------------------------------------------------------------------------
// Launch dispatch.
// ---------------------------------------------------------------------------
template <class S, int Q, int COLL, bool MEDIAN, int TX, int TY, bool PER = false, bool ENS = false,
          int NB = 1>
static void launch_k(const StepArgs<typename StoreT<S>::R>& A, hipStream_t s, hipEvent_t e0,
                     hipEvent_t e1) {
  const dim3 grid(A.tiles_x * ((A.tiles_y + NB - 1) / NB)), block(256 * NB);
  if (e0 && e1)  // events taken at the kernel's own start and end
    hipExtLaunchKernelGGL((k_step<S, Q, COLL, MEDIAN, TX, TY, PER, ENS, NB>), grid, block, 0, s, e0, e1, 0, A);
  else
    hipLaunchKernelGGL((k_step<S, Q, COLL, MEDIAN, TX, TY, PER, ENS, NB>), grid, block, 0, s, A);
}

template <class S, int Q, int COLL, bool MEDIAN>
static hipError_t launch_t(const void* args, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  using R = typename StoreT<S>::R;
  const StepArgs<R>& A = *(const StepArgs<R>*)args;
  if constexpr (!MEDIAN) {
    if (A.ens_mode != ENS_NONE) {
      // the ensemble limiters run on the one-site kernel (no row pipeline,
      // no deferred FP64 list: the limiter changed the state the list would
      // rebuild)
      if constexpr (Q == 3) launch_k<S, Q, COLL, false, 256, 1, false, true>(A, s, e0, e1);
      else if (tile_shape(Q, false, A.nx).tx == 256) launch_k<S, Q, COLL, false, 256, 1, false, true>(A, s, e0, e1);
      else launch_k<S, Q, COLL, false, 64, 4, false, true>(A, s, e0, e1);
      return hipGetLastError();
    }
  }
  if constexpr (Q == 3) {
    launch_k<S, Q, COLL, MEDIAN, 256, 1>(A, s, e0, e1);
  } else if constexpr (MEDIAN) {
    // Three stacked tiles with FP32 arithmetic (LBGK, MRT): 12 wavefronts,
    // two workgroups per CU at 74 registers.  4096^2 FP32 on one box: one
    // tile 412 us, two 379, three 353; four 457 on another (one workgroup
    // per CU).  FP64 and ELBM (over 128 registers) keep one tile.
    constexpr int NB = (COLL != COLL_ELBM && sizeof(typename StoreT<S>::R) == 4) ? 3 : 1;
    // periodic lattices: the branch-free pull of the tile's own sites
    if (A.bc == BC_PERIODIC) launch_k<S, Q, COLL, MEDIAN, 64, 4, true, false, NB>(A, s, e0, e1);
    else launch_k<S, Q, COLL, MEDIAN, 64, 4, false, false, NB>(A, s, e0, e1);
  } else {
    if (tile_shape(Q, MEDIAN, A.nx).tx == 256) {
      // 16-bit storage and ELBM.  With cached loads the one-site-per-lane
      // kernel left the memory system idle in 16-bit storage (2.4 TB/s
      // against 4.2 TB/s with four rows per workgroup and the next row's
      // loads in flight); with nontemporal loads one row per workgroup is
      // fastest (FP16 plain 123 -> 109 us, BF16 Ehrenfest 188 -> 154 us,
      // 4096^2 ELBM 1.11 -> 1.06 ms against four rows).
      bool rows = false;
      if constexpr (sizeof(S) == 2 || (sizeof(S) == 4 && COLL == COLL_ELBM)) {
        if (A.bc == BC_PERIODIC) {
          constexpr int ROWS = 1;
          const dim3 grid(A.tiles_x * ((A.ny + ROWS - 1) / ROWS)), block(256);
          // without Ehrenfest, a kernel compiled without the candidate code
          // (fewer registers, one more wavefront per SIMD in 16-bit storage)
          auto kern = A.ehrenfest ? k_step_rows<S, Q, COLL, ROWS, true>
                                  : k_step_rows<S, Q, COLL, ROWS, false>;
          if (e0 && e1)
            hipExtLaunchKernelGGL(kern, grid, block, 0, s, e0, e1, 0, A);
          else
            hipLaunchKernelGGL(kern, grid, block, 0, s, A);
          rows = true;
        }
      }
      if (!rows) {
        if constexpr (COLL != COLL_ELBM) {
          if (A.bc == BC_PERIODIC) launch_k<S, Q, COLL, MEDIAN, 256, 1, true>(A, s, e0, e1);
          else launch_k<S, Q, COLL, MEDIAN, 256, 1>(A, s, e0, e1);
        } else {
          launch_k<S, Q, COLL, MEDIAN, 256, 1>(A, s, e0, e1);
        }
      }
    } else {
      launch_k<S, Q, COLL, MEDIAN, 64, 4>(A, s, e0, e1);
    }
  }
  if constexpr (COLL == COLL_ELBM && sizeof(R) == 4 && !MEDIAN) {
    // the sites the step kernel left for the FP64 root solve (few; the
    // kernel returns at once when there are none)
    if (A.f64_sites)
      hipLaunchKernelGGL((k_elbm_f64<S, Q>), dim3(256), dim3(256), 0, s, A);
  }
  return hipGetLastError();
}

template <class S>
static hipError_t launch_s(int Q, int coll, bool median, const void* args, hipStream_t s,
                           hipEvent_t e0, hipEvent_t e1) {
  if (Q == 3) {
    if (coll == COLL_LBGK)
      return median ? launch_t<S, 3, COLL_LBGK, true>(args, s, e0, e1) : launch_t<S, 3, COLL_LBGK, false>(args, s, e0, e1);
    if (coll == COLL_ELBM)
      return median ? launch_t<S, 3, COLL_ELBM, true>(args, s, e0, e1) : launch_t<S, 3, COLL_ELBM, false>(args, s, e0, e1);
    return hipErrorInvalidValue;
  }
  switch (coll) {
    case COLL_LBGK:
      return median ? launch_t<S, 9, COLL_LBGK, true>(args, s, e0, e1) : launch_t<S, 9, COLL_LBGK, false>(args, s, e0, e1);
    case COLL_MRT:
      return median ? launch_t<S, 9, COLL_MRT, true>(args, s, e0, e1) : launch_t<S, 9, COLL_MRT, false>(args, s, e0, e1);
    default:
      return median ? launch_t<S, 9, COLL_ELBM, true>(args, s, e0, e1) : launch_t<S, 9, COLL_ELBM, false>(args, s, e0, e1);
  }
}

hipError_t launch_step(int storage, int Q, int coll, bool median, const void* args,
                       hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  switch (storage) {
    case 0: return launch_s<double>(Q, coll, median, args, s, e0, e1);
    case 1: return launch_s<float>(Q, coll, median, args, s, e0, e1);
    case 2: return launch_s<_Float16>(Q, coll, median, args, s, e0, e1);
    default: return launch_s<bf16_t>(Q, coll, median, args, s, e0, e1);
  }
}

}  // namespace lbm
