// The step with the general nonlocal filter of section 4 ("General nonlocal
// filters") on a periodic D1Q3 or D2Q9 lattice, for gfx950:
//   pull-stream -> moments and equilibrium
//   -> f(x) = f*(x) + sum_y d(y) f_neq(x + y), f_neq = f - f* of the streamed
//      state, over the neighbourhood shifts y (3 in 1D, 3 x 3 in 2D)
//   -> collision (LBGK, MRT or ELBM) -> positivity rule -> store.
// Each f_neq(x + y) carries no density or momentum, so f*(x) is also the
// equilibrium of the filtered state.  A workgroup stages f_neq of its tile
// and a one-site halo in LDS: every thread first evaluates its own site
// (whose f* it keeps), then the halo ring is shared out.
#include <hip/hip_ext.h>

#include "lbm_collide.h"
#include "lbm_internal.h"

namespace lbm {

// g mod n for the tile and halo coordinates, which lie within one lattice
// width of [0, n) unless the lattice is narrower than a tile (then the
// remainder)
__device__ __forceinline__ int wrap1(int g, int n) {
  const int r = g < 0 ? g + n : (g >= n ? g - n : g);
  return (r < 0 || r >= n) ? ((g % n) + n) % n : r;
}

template <class S, int Q, int COLL, int TX, int TY>
__global__ __launch_bounds__(TX * TY) void k_step_nl(const StepArgs<typename StoreT<S>::R> A,
                                                     int tiles_x) {
  using R = typename StoreT<S>::R;
  constexpr bool SH = StoreT<S>::shifted;
  constexpr int NT = TX * TY;
  constexpr int HY = Q == 9 ? 1 : 0, SW = TX + 2, SHH = TY + 2 * HY, NS = SW * SHH;
  constexpr int NRING = NS - NT, NK = Q == 9 ? 9 : 3;
  __shared__ R neq[Q][NS];

  // Consecutive workgroups are dealt round-robin to the 8 XCDs; each XCD
  // takes a contiguous band of tiles, so that the halo rows a tile shares
  // with the tiles above and below come from its own L2.
  const int T = (int)gridDim.x, b = blockIdx.x;
  const int tb = (T % 8 == 0) ? (b % 8) * (T / 8) + b / 8 : b;
  const int tile_x = tb % tiles_x, tile_y = tb / tiles_x;
  const int x0 = tile_x * TX, y0 = tile_y * TY;
  const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
  const int x = x0 + lx, y = y0 + ly;
  const bool valid = x < A.nx && y < A.ny;
  unsigned long long* const cnt = A.counters + (blockIdx.x % kCntSlots) * CNT_N;

  // one site of the tile or halo (periodic wrap, so ragged tiles need no
  // special case): its f_neq into LDS slot s
  R v[Q], feq[Q], m0, ux, uy;
  auto stage = [&](int gx, int gy, int s) {
    pull_periodic<S, Q, true>((const S*)A.src, A.qs, A.pitch, A.nx, A.ny, wrap1(gx, A.nx),
                        wrap1(gy, A.ny), v);
    moments_v<R, Q, SH>(v, A.rho0, m0, ux, uy);
    equilibrium_v<R, Q, SH>(m0, A.rho0, ux, uy, A.eq_kind, feq);
#pragma unroll
    for (int i = 0; i < Q; ++i) neq[i][s] = v[i] - feq[i];
  };
  stage(x, y, (ly + HY) * SW + lx + 1);
  R feq_c[Q], m0_c = m0, ux_c = ux, uy_c = uy;
#pragma unroll
  for (int i = 0; i < Q; ++i) feq_c[i] = feq[i];
  // the halo ring: top row, bottom row, then the left and right columns
  // (2D); the two end slots of the single row (1D)
  for (int r = tid; r < NRING; r += NT) {
    int hx, hy;
    if constexpr (Q == 9) {
      if (r < SW) { hx = r; hy = 0; }
      else if (r < 2 * SW) { hx = r - SW; hy = SHH - 1; }
      else { const int k = r - 2 * SW; hy = 1 + k / 2; hx = (k & 1) ? SW - 1 : 0; }
    } else {
      hy = 0;
      hx = r == 0 ? 0 : SW - 1;
    }
    stage(x0 + hx - 1, y0 + hy - HY, hy * SW + hx);
  }
  __syncthreads();

  R d[Q];
  if (valid) {
    R c[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) c[k] = A.nl_coef[k];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      R acc = R(0);
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        const int dy = Q == 9 ? k / 3 - 1 : 0, dx = Q == 9 ? k % 3 - 1 : k - 1;
        acc += c[k] * neq[i][(ly + HY + dy) * SW + lx + 1 + dx];
      }
      v[i] = feq_c[i] + acc;
      d[i] = feq_c[i] - v[i];
    }
  }
  const StepFrame fr{0, 0, 0};   // no Ehrenfest selection with this filter
  site_finish<S, Q, COLL, false, false>(A, x, y, valid, false, 0, v, feq_c, d, m0_c, ux_c, uy_c,
                                        R(0), fr, cnt);
}

template <class S, int Q, int COLL>
static hipError_t launch_nl(const void* args, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  using R = typename StoreT<S>::R;
  const StepArgs<R>& A = *(const StepArgs<R>*)args;
  // 2D: 64 x 8 tiles (1.29 halo sites per site, against 1.55 for 64 x 4;
  // 64 x 16 with 1.16 measured 4 % slower: fewer workgroups per CU to
  // overlap one's loads with another's LDS phase); FP32 ELBM keeps 64 x 4
  // (the root solve's registers); 1D: rows of 256
  constexpr int TX = Q == 9 ? 64 : 256;
  constexpr int TY = Q != 9 ? 1 : (sizeof(R) == 8 ? 8 : (COLL == COLL_ELBM ? 4 : 8));
  const int tx = (A.nx + TX - 1) / TX, ty = (A.ny + TY - 1) / TY;
  const dim3 grid(tx * ty), block(TX * TY);
  auto kern = k_step_nl<S, Q, COLL, TX, TY>;
  if (e0 && e1) hipExtLaunchKernelGGL(kern, grid, block, 0, s, e0, e1, 0, A, tx);
  else hipLaunchKernelGGL(kern, grid, block, 0, s, A, tx);
  return hipGetLastError();
}

template <class S>
static hipError_t launch_nl_s(int Q, int coll, const void* args, hipStream_t s, hipEvent_t e0,
                              hipEvent_t e1) {
  if (Q == 3) {
    if (coll == COLL_LBGK) return launch_nl<S, 3, COLL_LBGK>(args, s, e0, e1);
    if (coll == COLL_ELBM) return launch_nl<S, 3, COLL_ELBM>(args, s, e0, e1);
    return hipErrorInvalidValue;
  }
  switch (coll) {
    case COLL_LBGK: return launch_nl<S, 9, COLL_LBGK>(args, s, e0, e1);
    case COLL_MRT: return launch_nl<S, 9, COLL_MRT>(args, s, e0, e1);
    default: return launch_nl<S, 9, COLL_ELBM>(args, s, e0, e1);
  }
}

hipError_t launch_step_nl(int storage, int Q, int coll, const void* args, hipStream_t s,
                          hipEvent_t e0, hipEvent_t e1) {
  switch (storage) {
    case 0: return launch_nl_s<double>(Q, coll, args, s, e0, e1);
    case 1: return launch_nl_s<float>(Q, coll, args, s, e0, e1);
    case 2: return launch_nl_s<_Float16>(Q, coll, args, s, e0, e1);
    default: return launch_nl_s<bf16_t>(Q, coll, args, s, e0, e1);
  }
}

}  // namespace lbm
