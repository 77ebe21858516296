// Ehrenfest regularisation with a budget (section 4): after the collision,
// the k sites of largest nonequilibrium entropy Delta S > delta (ties to the
// lower site index) are sent to their equilibrium f*.  Every collision keeps
// rho and u, so f* is rebuilt from the moments that the step kernel recorded
// with each candidate and written over the collided state.
//
// The step kernel appends only sites whose key (the bit pattern of Delta S)
// is at least a floor carried over from the previous step, and counts them
// in a 4096-bucket histogram whose frame also comes from the previous step.
// Selection then touches the short candidate list only:
//   k_fb_scan   counts the candidates in every workgroup; unless a rescan
//               is needed, its first workgroup finds the boundary bucket
//               (holding the k-th largest key) from the histogram and the
//               others return.  Only when the candidates cannot hold the
//               answer (fewer than k above a raised floor) all of them
//               rescan the lattice, histogram the top 12 bits of Delta S
//               and pick a floor bin that holds at least k sites;
//   k_fb_append same condition: rescans and appends from that bin up;
//               its last workgroup then finds the boundary bucket;
//   k_fix_regions writes f* at candidates above the boundary bucket and
//               lists those inside it;
//   k_fix_tail  resolves the boundary bucket exactly by an MSD radix select
//               on (key descending, site index ascending), sets the next
//               step's floor and frame, and resets the counters;
//   k_sel_mrt   (MRT limiter only) replaces f* at the selected sites by the
//               MRT collision.
#include "lbm_collide.h"

namespace lbm {

template <class R> struct KeyTraits;
template <> struct KeyTraits<float> {
  static constexpr int bits = 32;
  static constexpr unsigned long long quarter = 1ull << 21;   // a quarter octave of Delta S
};
template <> struct KeyTraits<double> {
  static constexpr int bits = 64;
  static constexpr unsigned long long quarter = 1ull << 50;
};

__device__ __forceinline__ unsigned int coarse_bin(float v) {
  const uint32_t u = v != v ? 0x7f800000u : __float_as_uint(v);
  const uint32_t b = u >> 19;  // exponent and 4 mantissa bits: 0 .. 4080 for v >= 0
  return b < (uint32_t)kCoarse ? b : 0u;
}
template <class R>
__device__ __forceinline__ unsigned long long coarse_edge_key(int bin) {
  const float edge = __uint_as_float(((uint32_t)bin) << 19);
  return (unsigned long long)key_of<R>((R)edge);
}
__device__ __forceinline__ unsigned long long ld_rlx(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned int ld_rlx(const unsigned int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// True in every thread of the last workgroup to arrive.
__device__ __forceinline__ bool last_block(unsigned int* ticket) {
  __shared__ bool is_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) is_last = atomicAdd(ticket, 1u) == gridDim.x - 1;
  __syncthreads();
  if (is_last) __threadfence();
  return is_last;
}

// Block-wide search of an LDS histogram h[0..NB) from the top bin down: *bin
// receives the bin where the running count first reaches `need` (-1 if the
// histogram holds fewer), *above the count in the bins above it.  Every
// thread of the block calls it (blockDim.x a multiple of 64, at most 1024).
// Thread t sums a contiguous run of bins from the top; the running counts
// come from a shuffle scan in each wavefront plus the wavefront totals.
template <int NB>
__device__ void find_from_top(const unsigned int* h, unsigned long long need, int* bin,
                              unsigned long long* above) {
  __shared__ unsigned long long wsum[16];
  __shared__ int s_bin;
  __shared__ unsigned long long s_above;
  const int T = blockDim.x, t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int C = (NB + T - 1) / T;
  const int hi = NB - t * C;
  const int lo = hi - C > 0 ? hi - C : 0;
  unsigned long long s = 0;
  for (int b = lo; b < hi; ++b) s += h[b];
  unsigned long long incl = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long v = __shfl_up(incl, o);
    if (lane >= o) incl += v;
  }
  if (lane == 63) wsum[wv] = incl;
  if (t == 0) { s_bin = -1; s_above = 0; }
  __syncthreads();
  for (int j = 0; j < wv; ++j) incl += wsum[j];
  const unsigned long long excl = incl - s;
  if (s > 0 && need > 0 && excl < need && need <= incl) {
    unsigned long long c = excl;
    for (int b = hi - 1; b >= lo; --b) {
      if (c + h[b] >= need) { s_bin = b; s_above = c; break; }
      c += h[b];
    }
  }
  __syncthreads();
  *bin = s_bin;
  *above = s_above;
  __syncthreads();
}

template <class R>
__device__ __forceinline__ unsigned long long delta_key(R delta) {
  return delta <= R(0) ? 0ull : (unsigned long long)key_of<R>(delta);
}

// Frame for a histogram of keys in [base, top): about 2048 buckets, leaving
// half of the 4096 as margin for keys that grow in the next step.
__device__ __forceinline__ unsigned int frame_shift(unsigned long long base, unsigned long long top) {
  const unsigned long long span = top > base ? top - base : 0ull;
  unsigned int sh = 0;
  while (sh < 62 && (span >> sh) >= (unsigned long long)(kBuckets / 2)) ++sh;
  return sh;
}

// Site of lane `lane` of wavefront w in logical tile t (the step kernel's
// layout).
__device__ __forceinline__ void tile_site(int t, int w, int lane, int tiles_x, int tx, int& x, int& y) {
  const int tid = w * 64 + lane;
  x = (t % tiles_x) * tx + tid % tx;
  y = (t / tiles_x) * (256 / tx) + tid / tx;
}

// ---------------------------------------------------------------------------
// Sum of the spread candidate counters; every lane of the calling wavefront
// takes part (one counter per lane) and receives the sum.
__device__ __forceinline__ unsigned long long candidate_count(const unsigned long long* cc) {
  const int lane = __lane_id();
  unsigned long long n = lane < kCountSlots ? ld_rlx(&cc[lane * kCountStride]) : 0ull;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o);
  return n;
}

// The bucket holding the k-th largest candidate key, from the step's
// histogram (in LDS) and candidate count; stored in the selection state
// for the region sweep.  Every thread of one workgroup calls it.
template <class R>
__device__ void boundary_from(const unsigned int* h, long long nc, long long k, SelState* st) {
  int boundary = -1;
  unsigned long long above = 0;
  if (k <= 0) {
    boundary = kBuckets;                 // take nothing
  } else if (nc > k) {
    find_from_top<kBuckets>(h, (unsigned long long)k, &boundary, &above);
    if (boundary < 0) boundary = -1;
  }
  if (threadIdx.x == 0) {
    st->b_bin = boundary;
    st->b_nc = (unsigned long long)nc;
    st->b_above = above;
  }
}

// calibrate = 0: the step's first selection kernel; 1: first floor of a
// freshly set lattice.
template <class S, int Q>
__global__ __launch_bounds__(1024) void k_fb_scan(const StepArgs<typename StoreT<S>::R> A,
                                                 long long k, unsigned int* coarse,
                                                 int calibrate) {
  using R = typename StoreT<S>::R;
  SelState* st = A.sel;
  static_assert(kCoarse == kBuckets, "one LDS histogram serves both uses");
  __shared__ unsigned int h[kCoarse];
  if (!calibrate) {
    // Every workgroup takes the same decision from the same counters.  The
    // first one loads the histogram with them (one memory round trip) and,
    // unless the step rescans, finds the boundary bucket.
    __shared__ unsigned long long s_nc;
    if (blockIdx.x == 0)
      for (int i = threadIdx.x; i < kBuckets; i += blockDim.x) h[i] = ld_rlx(&A.hist[hist_pos(i)]);
    if (threadIdx.x < 64) {
      const unsigned long long n = candidate_count(A.ccount);
      if (threadIdx.x == 0) s_nc = n;
    }
    const unsigned long long step = st->step;
    const int fr0 = st->floor_raised[0], fr1 = st->floor_raised[1];
    const bool raised = ((step & 1ull) ? fr1 : fr0) != 0;
    __syncthreads();
    // a rescan is needed when the floor was raised and fewer than k sites
    // reached it
    const long long nc = (long long)s_nc;
    if (!(nc < k && raised)) {
      if (blockIdx.x == 0) boundary_from<R>(h, nc, k, st);
      return;
    }
    __syncthreads();
  }
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
  // The coarse bin that holds the k-th largest Delta S, and the frame of the
  // fallback candidates' histogram.
  for (int i = threadIdx.x; i < kCoarse; i += blockDim.x) h[i] = ld_rlx(&coarse[i]);
  __syncthreads();
  int b;
  unsigned long long above;
  const unsigned long long want = calibrate ? 3ull * (unsigned long long)k : (unsigned long long)k;
  find_from_top<kCoarse>(h, want > 0 ? want : 1ull, &b, &above);
  if (b < 0) b = 0;                                   // fewer eligible sites: take all
  __shared__ int top;
  if (threadIdx.x == 0) top = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < kCoarse - 16; i += blockDim.x)   // highest finite bin
    if (h[i]) atomicMax(&top, i);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long edge = coarse_edge_key<R>(b);
    const int par = (int)(st->step & 1ull);
    if (calibrate) {
      const unsigned long long dk = delta_key<R>(A.ehr_delta);
      const unsigned long long f = edge > dk ? edge : dk;
      const unsigned int sh = frame_shift(f, coarse_edge_key<R>(top + 1));
      for (int q = 0; q < 2; ++q) {
        st->floor_key[q] = f;
        st->floor_raised[q] = f > dk ? 1 : 0;
        st->base_key[q] = f;
        st->shift[q] = sh;
      }
      st->fallback = 0;
    } else {
      st->fb_bin = b;
      st->fallback = 1;
      st->fallbacks += 1;
      st->base_key[par] = edge;
      st->shift[par] = frame_shift(edge, coarse_edge_key<R>(top + 1));
    }
    st->ticket = 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kCoarse; i += blockDim.x) coarse[i] = 0;
  for (int i = threadIdx.x; i < kHistWords; i += blockDim.x) A.hist[i] = 0;
  for (int i = threadIdx.x; i < kCountSlots; i += blockDim.x) A.ccount[i * kCountStride] = 0;
}

template <class R>
__device__ void find_boundary(const StepArgs<R>& A, long long k) {
  __shared__ unsigned int h[kBuckets];
  __shared__ unsigned long long s_nc;
  for (int i = threadIdx.x; i < kBuckets; i += blockDim.x) h[i] = ld_rlx(&A.hist[hist_pos(i)]);
  if (threadIdx.x < 64) {
    const unsigned long long n = candidate_count(A.ccount);
    if (threadIdx.x == 0) s_nc = n;
  }
  __syncthreads();
  boundary_from<R>(h, (long long)s_nc, k, A.sel);
}

// Rescan append, in the step kernel's tile layout so that every wavefront
// region is rewritten (stale counts of the step kernel included).
template <class S, int Q>
__global__ __launch_bounds__(256) void k_fb_append(const StepArgs<typename StoreT<S>::R> A,
                                                   long long k) {
  using R = typename StoreT<S>::R;
  SelState* st = A.sel;
  if (!st->fallback) return;
  const unsigned int fb = (unsigned int)st->fb_bin;
  const int T = A.tiles_x * A.tiles_y;
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  for (int t = blockIdx.x; t < T; t += gridDim.x) {
    int x, y;
    tile_site(t, w, lane, A.tiles_x, A.tile_tx, x, y);
    const bool valid = x < A.nx && y < A.ny;
    bool is_c = false;
    R dS = R(0), m0 = R(0), ux = R(0), uy = R(0);
    if (valid) {
      R v[Q], feq[Q], d[Q];
      dS = site_prep<S, Q>(A, x, y, v, feq, d, m0, ux, uy, true);
      is_c = (dS > A.ehr_delta) && coarse_bin((float)dS) >= fb;
    }
    const long long region = (long long)t * 4 + w;
    const unsigned long long mask = __ballot(is_c);
    if (lane == 0) {
      A.wcount[region] = (uint32_t)__popcll(mask);
      if (mask)
        atomicAdd(&A.ccount[(region & (kCountSlots - 1)) * kCountStride], (unsigned long long)__popcll(mask));
    }
    if (is_c) {
      const long long pos = region * 64 + __popcll(mask & ((1ull << lane) - 1ull));
      A.cand_key[pos] = key_of<R>(dS);
      A.cand_idx[pos] = (uint32_t)(y * A.nx + x);
      A.cand_mom[pos] = m0;
      A.cand_mom[A.cap + pos] = ux;
      A.cand_mom[2 * A.cap + pos] = uy;
      const int par = (int)(st->step & 1ull);
      atomicAdd(&A.hist[hist_pos(bucket_of<R>((unsigned long long)key_of<R>(dS), st->base_key[par], st->shift[par]))], 1u);
    }
  }
  if (last_block(&st->ticket)) {
    find_boundary<R>(A, k);
    if (threadIdx.x == 0) st->ticket = 0;
  }
}

// f* of site idx from the moments recorded with its candidate entry,
// written over the collided state.
template <class S, int Q>
__device__ __forceinline__ void write_feq_at(const StepArgs<typename StoreT<S>::R>& A,
                                             uint32_t idx, typename StoreT<S>::R m0,
                                             typename StoreT<S>::R ux, typename StoreT<S>::R uy) {
  using R = typename StoreT<S>::R;
  constexpr bool SH = StoreT<S>::shifted;
  const int y = (int)(idx / (uint32_t)A.nx), x = (int)(idx % (uint32_t)A.nx);
  R feq[Q];
  equilibrium_v<R, Q, SH>(m0, A.rho0, ux, uy, A.eq_kind, feq);
  S* dst = (S*)A.dst;
#pragma unroll
  for (int i = 0; i < Q; ++i)
    StoreT<S>::st(dst + (long long)i * A.qs + (long long)y * A.pitch + x, feq[i]);
}

// Wave-aggregated reservation of one slot per set lane on an LDS counter.
__device__ __forceinline__ unsigned int lds_slot(bool on, unsigned int* ctr) {
  const unsigned long long mask = __ballot(on);
  if (!mask) return 0;
  const int lane = __lane_id();
  const int leader = __ffsll((long long)mask) - 1;
  unsigned int base = 0;
  if (lane == leader) base = atomicAdd(ctr, (unsigned int)__popcll(mask));
  base = __shfl(base, leader);
  return base + (unsigned int)__popcll(mask & ((1ull << lane) - 1ull));
}

// Boundary-bucket entries that the exact resolution stages in LDS; lists of
// up to kTailRank entries are ranked directly.
constexpr int kTailStage = 2048;
constexpr int kTailRank = 256;

// Exact resolution of the boundary bucket and the next step's floor and
// frame, by one workgroup.
template <class S, int Q>
__device__ void fix_tail(const StepArgs<typename StoreT<S>::R>& A, long long k, long long n_sites,
                         int32_t* selected, uint32_t* blist, long long bcap,
                         long long* n_sel_out, int32_t* tape_sel, long long* tape_cnt,
                         long long tape_len, uint32_t* scratch, long long scratch_len) {
  using R = typename StoreT<S>::R;
  SelState* st = A.sel;
  __shared__ unsigned int h[kBuckets];
  __shared__ unsigned int dh[256];
  __shared__ unsigned long long s_off_pref;
  __shared__ uint32_t s_idx_pref;
  __shared__ unsigned int s_tot;
  __shared__ unsigned long long t_off[kTailStage];
  __shared__ uint32_t t_ni[kTailStage], t_p[kTailStage];
  // every load is issued before the first barrier; both parities' fields
  // are loaded with the step count (one round trip)
  const unsigned long long step = st->step;
  const unsigned long long base_p[2] = {st->base_key[0], st->base_key[1]};
  const unsigned int shift_p[2] = {st->shift[0], st->shift[1]};
  const int raised_p[2] = {st->floor_raised[0], st->floor_raised[1]};
  const unsigned long long floor_p[2] = {st->floor_key[0], st->floor_key[1]};
  for (int i = threadIdx.x; i < kBuckets; i += blockDim.x) h[i] = ld_rlx(&A.hist[hist_pos(i)]);
  // candidate count, boundary bucket and the count above it, as found by
  // k_fb_scan (or by the rescan's last workgroup)
  const long long nc = (long long)st->b_nc;
  const int b_bin = st->b_bin;
  const unsigned long long b_above = st->b_above;
  const unsigned long long sel_bnd = st->sel_bnd;
  const long long m_all = (long long)(sel_bnd & 0xffffffffull);
  // state the epilogue updates
  const bool fell_back = st->fallback != 0;
  const long long tape_t = st->tape_t;
  if (tape_sel && tape_t < tape_len) {
    selected = tape_sel + tape_t * k;
    n_sel_out = tape_cnt + tape_t;
  }
  const unsigned long long overflows = st->overflows, cand_total = st->cand_total;
  // this thread's boundary-list entry, loaded with the state (the short-list
  // path below needs it; past the list's length it is not used)
  const uint32_t p_mine = (long long)threadIdx.x < bcap ? blist[threadIdx.x] : 0u;
  if (threadIdx.x == 0) s_tot = (unsigned int)(sel_bnd >> 32);
  __syncthreads();
  const int par = (int)(step & 1ull);
  const unsigned long long base = par ? base_p[1] : base_p[0];
  const unsigned int shift = par ? shift_p[1] : shift_p[0];
  const bool raised = (par ? raised_p[1] : raised_p[0]) != 0;
  const unsigned long long floor_prev = par ? floor_p[1] : floor_p[0];
  const long long need = k < nc ? k : nc;
  const int boundary = (k > 0 && nc > k) ? b_bin : -1;
  const unsigned long long above = (k > 0 && nc > k) ? b_above : 0ull;
  const long long take = (boundary >= 0 && k > 0 && nc > k) ? need - (long long)above : 0;
  const long long m = m_all < bcap ? m_all : bcap;
  if (take > 0 && m > 0 && m <= kTailRank && (int)blockDim.x >= 4 * kTailRank) {
    // Short list: the rank of each entry in (key descending, site index
    // ascending) order is the number of entries that beat it.  Entry q is
    // counted by `slices` threads, each against a contiguous slice of the
    // list in LDS; the entries of rank below `take` are selected.  The
    // moments are loaded with the key, so f* needs no further round trip.
    const unsigned long long edge = base + ((unsigned long long)boundary << shift);
    const int mq = (int)((m + 63) & ~63ll);          // entries rounded up to whole wavefronts
    const int slices = (int)blockDim.x / mq;         // >= 4
    const int q = (int)threadIdx.x % mq, sl = (int)threadIdx.x / mq;
    unsigned long long oq = 0;
    uint32_t nq = 0;
    R m0 = R(0), ux = R(0), uy = R(0);
    if ((int)threadIdx.x < m) {
      const uint32_t p = p_mine;
      const unsigned long long key = (unsigned long long)A.cand_key[p];
      oq = key >= edge ? key - edge : 0ull;
      nq = ~A.cand_idx[p];
      m0 = A.cand_mom[p];
      ux = A.cand_mom[A.cap + p];
      uy = A.cand_mom[2 * A.cap + p];
      t_off[threadIdx.x] = oq;
      t_ni[threadIdx.x] = nq;
      t_p[threadIdx.x] = 0;                         // rank counter of entry threadIdx.x
    }
    __syncthreads();
    if (sl < slices && q < m) {
      const unsigned long long o = t_off[q];
      const uint32_t ni = t_ni[q];
      const int per = ((int)m + slices - 1) / slices;
      const int j0 = sl * per, j1 = j0 + per < (int)m ? j0 + per : (int)m;
      unsigned int beat = 0;
#pragma unroll 4
      for (int j = j0; j < j1; ++j) {
        const unsigned long long oj = t_off[j];
        beat += (oj > o || (oj == o && t_ni[j] > ni)) ? 1u : 0u;
      }
      if (beat) atomicAdd(&t_p[q], beat);
    }
    __syncthreads();
    // thread q < m (slice 0 when blockDim.x / mq >= 1) holds entry q's moments
    const bool sel = (int)threadIdx.x < m && (long long)t_p[threadIdx.x] < take;
    if (sel) write_feq_at<S, Q>(A, ~nq, m0, ux, uy);
    const unsigned int slot = lds_slot(sel, &s_tot);
    if (sel && (long long)slot < k) selected[slot] = (int32_t)~nq;
  } else if (take > 0 && m > 0) {
    // keys of the bucket differ only in their offset from its lower edge:
    // `shift` bits, or all bits in the open-ended top bucket
    const unsigned long long edge = base + ((unsigned long long)boundary << shift);
    const int nb = boundary == kBuckets - 1 ? KeyTraits<R>::bits : (int)shift;
    const int kd = (nb + 7) / 8;
    // MSD radix select, one byte per pass: the key digits from the top, then
    // the site index digits.  Up to kTailStage entries are read from the
    // candidate buffer once into LDS and every pass works there.  Longer
    // lists (large groups of exactly tied keys, frequent with 16-bit
    // storage) are written once as 16-byte records (offset, ~index,
    // position) to a global scratch array, the region sweep's stage (unused
    // once the sweep has finished), so that every pass reads one record per
    // entry instead of two dependent loads; without room there the passes
    // read the candidate buffer.  The staging read also takes the first
    // digit's histogram (every entry matches the empty prefix), and once the
    // entries matching the prefix fit in LDS, one more pass over the list
    // gathers them there for the remaining digits.
    const bool staged = m <= kTailStage;
    const bool recs = !staged && scratch && 4 * m <= scratch_len;
    // index digits: the bytes that site indices below n_sites use; above
    // them every ~index holds ones, and so does the prefix from the start
    const int kdi = n_sites <= 256 ? 1 : (32 - __clz((unsigned int)(n_sites - 1)) + 7) / 8;
    const uint32_t ip0 = kdi >= 4 ? 0u : ~((1u << (8 * kdi)) - 1u);
    auto digit_shift = [&](int dgt) { return dgt < kd ? 8 * (kd - 1 - dgt) : 8 * (kdi - 1 - (dgt - kd)); };
    const int sb0 = digit_shift(0);
    __shared__ unsigned int s_last_cnt, s_gather;
    if (threadIdx.x == 0) { s_off_pref = 0; s_idx_pref = ip0; s_last_cnt = (unsigned int)m; s_gather = 0; }
    for (int i = threadIdx.x; i < 256; i += blockDim.x) dh[i] = 0;
    __syncthreads();
    if (staged || recs) {
      for (long long b0 = 0; b0 < m; b0 += 4 * (long long)blockDim.x) {
        const long long q0 = b0 + threadIdx.x;
        uint32_t pu[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const long long q = q0 + u * (long long)blockDim.x;
          pu[u] = q < m ? blist[q] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const long long q = q0 + u * (long long)blockDim.x;
          unsigned long long off = 0;
          uint32_t ni = 0;
          if (q < m) {
            const unsigned long long key = (unsigned long long)A.cand_key[pu[u]];
            off = key >= edge ? key - edge : 0ull;
            ni = ~A.cand_idx[pu[u]];
            if (staged) {
              t_off[q] = off;
              t_ni[q] = ni;
              t_p[q] = pu[u];
            } else {
              *reinterpret_cast<uint4*>(scratch + 4 * q) =
                  make_uint4((uint32_t)off, (uint32_t)(off >> 32), ni, pu[u]);
            }
          }
          hist_add(dh, kd > 0 ? (unsigned int)((off >> sb0) & 0xffu) : (ni >> sb0) & 0xffu, q < m);
        }
      }
      __syncthreads();
    }
    // entry q of the list, from LDS (`lds`) or from the records / the
    // candidate buffer
    auto entry = [&](bool lds, long long q, unsigned long long& off, uint32_t& ni, uint32_t& p) {
      if (lds) {
        off = t_off[q];
        ni = t_ni[q];
        p = t_p[q];
      } else if (recs) {
        const uint4 r = *reinterpret_cast<const uint4*>(scratch + 4 * q);
        off = (unsigned long long)r.x | ((unsigned long long)r.y << 32);
        ni = r.z;
        p = r.w;
      } else {
        p = blist[q];
        const unsigned long long key = (unsigned long long)A.cand_key[p];
        off = key >= edge ? key - edge : 0ull;
        ni = ~A.cand_idx[p];
      }
    };
    // does (off, ni) match the prefix found so far, down to bit `sb` of the
    // key digits (on_key) or of the index digits
    auto matches = [](bool on_key, int sb, unsigned long long off, uint32_t ni,
                      unsigned long long op, uint32_t ip) {
      if (on_key) {
        const unsigned long long hm = sb >= 64 ? 0ull : (~0ull << sb);
        return (off & hm) == (op & hm);
      }
      const uint32_t hm = sb >= 32 ? 0u : (~0u << sb);
      return off == op && (ni & hm) == (ip & hm);
    };
    bool local = staged;      // the entries still matching are all in LDS
    long long ml = m;         // the entries a pass visits
    unsigned long long need_left = (unsigned long long)take;
    for (int dgt = 0; dgt < kd + kdi; ++dgt) {
      // after the key digits: if every entry sharing the threshold key is
      // taken, the site-index digits cannot change the set
      if (dgt == kd && s_last_cnt == need_left) break;
      const bool on_key = dgt < kd;
      const int sb = digit_shift(dgt);
      if (!(dgt == 0 && (staged || recs))) {
        for (int i = threadIdx.x; i < 256; i += blockDim.x) dh[i] = 0;
        __syncthreads();
        const unsigned long long op = s_off_pref;
        const uint32_t ip = s_idx_pref;
        // four entries per thread in flight
        for (long long b0 = 0; b0 < ml; b0 += 4 * (long long)blockDim.x) {
          const long long q0 = b0 + threadIdx.x;
          unsigned long long offs[4] = {0ull, 0ull, 0ull, 0ull};
          uint32_t nis[4] = {0u, 0u, 0u, 0u}, ps[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const long long q = q0 + u * (long long)blockDim.x;
            if (q < ml) entry(local, q, offs[u], nis[u], ps[u]);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const long long q = q0 + u * (long long)blockDim.x;
            const bool on = q < ml && matches(on_key, sb + 8, offs[u], nis[u], op, ip);
            hist_add(dh, on_key ? (unsigned int)((offs[u] >> sb) & 0xffu) : (nis[u] >> sb) & 0xffu, on);
          }
        }
        __syncthreads();
      }
      int dsel;
      unsigned long long dabove;
      find_from_top<256>(dh, need_left, &dsel, &dabove);
      if (dsel < 0) dsel = 0;
      need_left -= dabove;
      if (threadIdx.x == 0) {
        if (on_key) s_off_pref |= ((unsigned long long)dsel) << sb;
        else s_idx_pref |= ((uint32_t)dsel) << sb;
        s_last_cnt = dh[dsel];
      }
      __syncthreads();
      // the entries matching the extended prefix fit in LDS, and a further
      // pass follows: gather them (p is not needed, the final pass reads
      // the list itself)
      const bool more = dgt + 1 < kd + kdi && !(dgt + 1 == kd && s_last_cnt == need_left);
      if (!local && more && s_last_cnt <= (unsigned int)kTailStage) {
        const unsigned long long op = s_off_pref;
        const uint32_t ip = s_idx_pref;
        // the same trip count in every thread (the slots come from ballots)
        for (long long b0 = 0; b0 < m; b0 += 4 * (long long)blockDim.x) {
          const long long q0 = b0 + threadIdx.x;
          unsigned long long offs[4] = {0ull, 0ull, 0ull, 0ull};
          uint32_t nis[4] = {0u, 0u, 0u, 0u}, ps[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const long long q = q0 + u * (long long)blockDim.x;
            if (q < m) entry(false, q, offs[u], nis[u], ps[u]);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const long long q = q0 + u * (long long)blockDim.x;
            const bool on = q < m && matches(on_key, sb, offs[u], nis[u], op, ip);
            const unsigned int slot = lds_slot(on, &s_gather);
            if (on && slot < (unsigned int)kTailStage) {   // slot < s_last_cnt
              t_off[slot] = offs[u];
              t_ni[slot] = nis[u];
            }
          }
        }
        __syncthreads();
        local = true;
        ml = s_gather;
      }
    }
    // The selected entries: four per thread, every load issued before the
    // first store (the records, then the moments of the selected ones), so
    // that a long list costs a quarter of the round trips.
    const unsigned long long to = s_off_pref;
    const uint32_t ti = s_idx_pref;
    for (long long b0 = 0; b0 < m; b0 += 4 * (long long)blockDim.x) {
      const long long q0 = b0 + threadIdx.x;
      unsigned long long offs[4] = {0ull, 0ull, 0ull, 0ull};
      uint32_t nis[4] = {0u, 0u, 0u, 0u}, ps[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const long long q = q0 + u * (long long)blockDim.x;
        if (q < m) entry(staged, q, offs[u], nis[u], ps[u]);
      }
      bool sel[4];
      R m0s[4], uxs[4], uys[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const long long q = q0 + u * (long long)blockDim.x;
        sel[u] = q < m && (offs[u] > to || (offs[u] == to && nis[u] >= ti));
        m0s[u] = uxs[u] = uys[u] = R(0);
        if (sel[u]) {
          m0s[u] = A.cand_mom[ps[u]];
          uxs[u] = A.cand_mom[A.cap + ps[u]];
          uys[u] = A.cand_mom[2 * A.cap + ps[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (sel[u]) write_feq_at<S, Q>(A, ~nis[u], m0s[u], uxs[u], uys[u]);   // ~ni: the site
        const unsigned int slot = lds_slot(sel[u], &s_tot);
        if (sel[u] && (long long)slot < k) selected[slot] = (int32_t)~nis[u];
      }
    }
  }
  __syncthreads();

  // --- floor and frame for the next step of this parity --------------------
  // Keep between 2k and 3.5k candidates (aim at 3k); the floor is never
  // raised when k is at least a tenth of the lattice.  (A window up to 6k
  // let the count drift to 4.5-4.7k, each extra candidate an exact Delta S
  // in the step kernel and an entry for the selection kernels to sort; one
  // up to 3k re-aims almost every step, which cost more than it saved.)  The frame spans twice the
  // current candidates' range above the floor.
  const unsigned long long dk = delta_key<R>(A.ehr_delta);
  unsigned long long fnext = dk;
  if (10 * k < n_sites && k > 0) {
    const bool keep = raised && !fell_back && nc >= 2 * k && nc <= 7 * k / 2;
    if (keep) {
      fnext = floor_prev;
    } else {
      int t2;
      unsigned long long a2;
      find_from_top<kBuckets>(h, 3ull * (unsigned long long)k, &t2, &a2);
      if (t2 >= 0 && t2 < kBuckets - 1) fnext = base + ((unsigned long long)t2 << shift);
      else if (t2 < 0) fnext = base > 2 * KeyTraits<R>::quarter ? base - 2 * KeyTraits<R>::quarter : 0ull;
      else fnext = floor_prev;
    }
    if (fnext < dk) fnext = dk;
  }
  // top nonempty bucket: per-thread maximum, wavefront maximum by
  // shuffles, one LDS atomic per wavefront
  __shared__ int s_top;
  if (threadIdx.x == 0) s_top = -1;
  __syncthreads();
  {
    int tmax = -1;
    for (int i = threadIdx.x; i < kBuckets; i += blockDim.x)
      if (h[i]) tmax = i;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const int v = __shfl_xor(tmax, o);
      tmax = v > tmax ? v : tmax;
    }
    if (__lane_id() == 0 && tmax >= 0) atomicMax(&s_top, tmax);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // upper end of this step's keys: the top nonempty bucket's upper edge,
    // or twice the frame when keys ran past it
    const unsigned long long span = (unsigned long long)kBuckets << shift;
    const unsigned long long hi_key = s_top < 0 ? fnext + 1
        : (s_top < kBuckets - 1 ? base + ((unsigned long long)(s_top + 1) << shift) : base + 2 * span);
    st->floor_key[par] = fnext;
    st->floor_raised[par] = fnext > dk ? 1 : 0;
    st->base_key[par] = fnext;
    st->shift[par] = frame_shift(fnext, hi_key > fnext ? fnext + 2 * (hi_key - fnext) : fnext + 1);
    const unsigned int ns = s_tot < (unsigned int)k ? s_tot : (unsigned int)k;
    st->n_sel = (long long)ns;
    if (n_sel_out) *n_sel_out = (long long)ns;
    if (m_all > bcap) st->overflows = overflows + 1;
    st->cand_total = cand_total + (unsigned long long)nc;
    st->fallback = 0;
    st->sel_bnd = 0;
    st->step += 1;
    st->tape_t = tape_t + 1;
  }
  for (int i = threadIdx.x; i < kHistWords; i += blockDim.x) A.hist[i] = 0;
  for (int i = threadIdx.x; i < kCountSlots; i += blockDim.x) A.ccount[i * kCountStride] = 0;
}

// LDS staging of a k_fix_regions workgroup: selected sites and boundary
// entries (the rest, up to kSweepRegions x 64 entries, go to its global
// stage).
constexpr int kRegSel = 6144;
constexpr int kRegBnd = 2048;
// Regions with at most this many candidates are walked lane by lane.
constexpr int kFewCand = 4;

// Selection: k_fix_regions sends every candidate above the boundary bucket to
// equilibrium and lists the boundary bucket; k_fix_tail (one workgroup of
// 1024: the exact resolution is a chain of dependent loads over the list)
// resolves the boundary bucket exactly and prepares the next step.
template <class S, int Q>
__global__ __launch_bounds__(kSweepRegions) void k_fix_regions(const StepArgs<typename StoreT<S>::R> A,
                                                     long long k, int32_t* selected,
                                                     int32_t* stage, uint32_t* blist,
                                                     long long bcap, int32_t* tape_sel,
                                                     long long tape_len) {
  using R = typename StoreT<S>::R;
  SelState* st = A.sel;
  __shared__ unsigned int s_sel, s_bnd;
  __shared__ unsigned long long s_base_sel, s_base_bnd;
  __shared__ int32_t l_sel[kRegSel], l_bnd[kRegBnd];
  // both parities' frames are loaded with the step count (one round trip)
  const unsigned long long step = st->step;
  const unsigned long long base0 = st->base_key[0], base1 = st->base_key[1];
  const unsigned int shift0 = st->shift[0], shift1 = st->shift[1];
  const int boundary = st->b_bin;          // -1: take every candidate
  const long long tape_t = st->tape_t;
  if (tape_sel && tape_t < tape_len) selected = tape_sel + tape_t * k;
  const unsigned long long base = (step & 1ull) ? base1 : base0;
  const unsigned int shift = (step & 1ull) ? shift1 : shift0;
  if (threadIdx.x == 0) { s_sel = 0; s_bnd = 0; }
  __syncthreads();
  // 64 regions per wavefront, spread over the whole lattice with a stride of
  // the wavefront count (candidates crowd into whole rows of a shear layer;
  // a contiguous assignment would hand one wavefront an entire dense row).
  // One read of the 64 counts, then the non-empty regions in turn with one
  // lane per entry.
  const long long nreg = (long long)A.tiles_x * A.tiles_y * 4;
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  constexpr int kWaves = kSweepRegions / 64;
  const long long g = (long long)blockIdx.x * kWaves + w, nwave = (long long)gridDim.x * kWaves;
  const long long my_r = (long long)lane * nwave + g;
  int32_t* my_stage = stage + (long long)blockIdx.x * kSweepRegions * 64;
  uint32_t cnt = 0;
  if (my_r < nreg) cnt = A.wcount[my_r];
  // One candidate entry p (when `on`): f* at the selected, staging of the
  // selected and of the boundary entries.  Every lane of the wavefront calls
  // it (the LDS slots come from ballots).
  auto visit = [&](bool on, long long p) {
    bool sel = false, bnd = false;
    uint32_t idx = 0;
    R m0 = R(0), ux = R(0), uy = R(0);
    if (on) {
      // the whole entry in one round trip
      const unsigned long long key = (unsigned long long)A.cand_key[p];
      idx = A.cand_idx[p];
      m0 = A.cand_mom[p];
      ux = A.cand_mom[A.cap + p];
      uy = A.cand_mom[2 * A.cap + p];
      const int b = bucket_of<R>(key, base, shift);
      sel = boundary < 0 || b > boundary;
      bnd = b == boundary;
    }
    if (sel) write_feq_at<S, Q>(A, idx, m0, ux, uy);
    // staged in LDS, or past its capacity in the workgroup's global stage
    const unsigned int slot = lds_slot(sel, &s_sel);
    if (sel) {
      if (slot < (unsigned int)kRegSel) l_sel[slot] = (int32_t)idx;
      else my_stage[slot] = (int32_t)idx;
    }
    const unsigned int q = lds_slot(bnd, &s_bnd);
    if (bnd) {                                  // boundary entries fill from the end
      if (q < (unsigned int)kRegBnd) l_bnd[q] = (int32_t)p;
      else my_stage[kSweepRegions * 64 - 1 - q] = (int32_t)p;
    }
  };
  // Sparse regions (at most kFewCand entries, where candidates are scattered
  // over the lattice) are walked by their own lane, all lanes at once; dense
  // regions (candidates crowding into the rows of a shear layer) one after
  // another with one lane per entry.
  const uint32_t few = cnt <= (uint32_t)kFewCand ? cnt : 0u;
  uint32_t fmax_c = few;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t v = __shfl_xor(fmax_c, o);
    fmax_c = v > fmax_c ? v : fmax_c;
  }
  for (uint32_t e = 0; e < fmax_c; ++e) visit(e < few, my_r * 64 + e);
  unsigned long long nz = __ballot(cnt > (uint32_t)kFewCand);
  while (nz) {
    const int j = __ffsll((long long)nz) - 1;
    nz &= nz - 1;
    const uint32_t c = __shfl(cnt, j);
    const long long rj = __shfl(my_r, j);
    visit((uint32_t)lane < c, rj * 64 + lane);
  }
  if (cnt) A.wcount[my_r] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    // one atomic reserves both lists' slots (same-address atomics from
    // every workgroup queue behind each other); neither count reaches 2^31,
    // the limit on the lattice's sites, so no carry crosses the halves
    const unsigned long long both = ((unsigned long long)s_sel << 32) | s_bnd;
    const unsigned long long old = both ? atomicAdd(&st->sel_bnd, both) : 0ull;
    s_base_sel = old >> 32;
    s_base_bnd = old & 0xffffffffull;
  }
  __syncthreads();
  for (unsigned int i = threadIdx.x; i < s_sel; i += blockDim.x)
    if ((long long)(s_base_sel + i) < k)
      selected[s_base_sel + i] = i < (unsigned int)kRegSel ? l_sel[i] : my_stage[i];
  for (unsigned int i = threadIdx.x; i < s_bnd; i += blockDim.x)
    if ((long long)(s_base_bnd + i) < bcap)
      blist[s_base_bnd + i] = (uint32_t)(i < (unsigned int)kRegBnd ? l_bnd[i] : my_stage[kSweepRegions * 64 - 1 - i]);
}

template <class S, int Q>
__global__ __launch_bounds__(1024) void k_fix_tail(const StepArgs<typename StoreT<S>::R> A,
                                                   long long k, long long n_sites,
                                                   int32_t* selected, uint32_t* blist,
                                                   long long bcap, long long* n_sel_out,
                                                   int32_t* tape_sel, long long* tape_cnt,
                                                   long long tape_len, uint32_t* scratch,
                                                   long long scratch_len) {
  fix_tail<S, Q>(A, k, n_sites, selected, blist, bcap, n_sel_out, tape_sel, tape_cnt, tape_len,
                 scratch, scratch_len);
}

// The MRT limiter (section 5) on an LBGK lattice: the step's selected sites,
// which the sweep has just sent to f*, receive the MRT collision of their
// pulled state instead (the source lattice is intact until the next step),
// then the positivity rule when it is on.  The list is where k_fix_tail
// wrote it: the tape slot of the step when recording, else `selected`.
template <class S, int Q>
__global__ __launch_bounds__(256) void k_sel_mrt(const StepArgs<typename StoreT<S>::R> A,
                                                 long long k, const int32_t* selected,
                                                 const int32_t* tape_sel, long long tape_len) {
  using R = typename StoreT<S>::R;
  const SelState* st = A.sel;
  const long long n = st->n_sel;
  const long long t = st->tape_t - 1;
  const int32_t* list = (tape_sel && t >= 0 && t < tape_len) ? tape_sel + t * k : selected;
  for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (long long)gridDim.x * blockDim.x) {
    const int idx = list[j];
    const int y = idx / A.nx, x = idx % A.nx;
    R out[Q];
    selected_state<S, Q>(A, x, y, R(0), R(0), R(0), out);
    S* dst = (S*)A.dst;
#pragma unroll
    for (int i = 0; i < Q; ++i)
      StoreT<S>::st(dst + (long long)i * A.qs + (long long)y * A.pitch + x, out[i]);
  }
}

template <class S, int Q>
static hipError_t launch_select_t(const SelectArgs& a, hipStream_t s) {
  using R = typename StoreT<S>::R;
  const StepArgs<R>& A = *(const StepArgs<R>*)a.step_args;
  // All but the first workgroup of k_fb_scan, and all of k_fb_append,
  // return at once unless this step rescans (rare).  k_fb_scan runs 64
  // workgroups of 1024 threads: its first one reads the 4096-bucket
  // histogram four words per thread (1.2 us per step less than 256 x 256).
  hipLaunchKernelGGL((k_fb_scan<S, Q>), dim3(64), dim3(1024), 0, s, A, a.k, a.coarse, 0);
  hipLaunchKernelGGL((k_fb_append<S, Q>), dim3(256), dim3(256), 0, s, A, a.k);
  const long long nreg = (long long)A.tiles_x * A.tiles_y * 4;
  const int gfix = (int)((nreg + kSweepRegions - 1) / kSweepRegions);
  hipLaunchKernelGGL((k_fix_regions<S, Q>), dim3(gfix), dim3(kSweepRegions), 0, s, A, a.k, a.selected,
                     a.segsel, a.blist, a.bcap, a.tape_sel, a.tape_len);
  // the region sweep's stage: gfix workgroups x kSweepRegions regions x 64
  // entries
  hipLaunchKernelGGL((k_fix_tail<S, Q>), dim3(1), dim3(1024), 0, s, A, a.k, a.n_sites,
                     a.selected, a.blist, a.bcap, a.n_sel_out, a.tape_sel, a.tape_cnt,
                     a.tape_len, (uint32_t*)a.segsel, (long long)gfix * kSweepRegions * 64);
  if (A.sel_mrt) {
    const long long g = (a.k + 255) / 256;
    hipLaunchKernelGGL((k_sel_mrt<S, Q>), dim3((unsigned)(g < 1 ? 1 : (g > 1024 ? 1024 : g))),
                       dim3(256), 0, s, A, a.k, a.selected, a.tape_sel, a.tape_len);
  }
  return hipGetLastError();
}

template <class S, int Q>
static hipError_t launch_calibrate_t(const SelectArgs& a, hipStream_t s) {
  using R = typename StoreT<S>::R;
  const StepArgs<R>& A = *(const StepArgs<R>*)a.step_args;
  // the floor is only ever raised when k is below a tenth of the lattice
  if (!(10 * a.k < a.n_sites && a.k > 0)) return hipSuccess;
  hipLaunchKernelGGL((k_fb_scan<S, Q>), dim3(1024), dim3(256), 0, s, A, a.k, a.coarse, 1);
  return hipGetLastError();
}

hipError_t launch_select_calibrate(const SelectArgs& a, hipStream_t s) {
  switch (a.storage * 16 + a.Q) {
    case 0 * 16 + 9: return launch_calibrate_t<double, 9>(a, s);
    case 0 * 16 + 3: return launch_calibrate_t<double, 3>(a, s);
    case 1 * 16 + 9: return launch_calibrate_t<float, 9>(a, s);
    case 1 * 16 + 3: return launch_calibrate_t<float, 3>(a, s);
    case 2 * 16 + 9: return launch_calibrate_t<_Float16, 9>(a, s);
    case 2 * 16 + 3: return launch_calibrate_t<_Float16, 3>(a, s);
    case 3 * 16 + 9: return launch_calibrate_t<bf16_t, 9>(a, s);
    default: return launch_calibrate_t<bf16_t, 3>(a, s);
  }
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

// Initial selection state: floor at the threshold, a frame spanning every
// positive key (bucket = the top 12 bits of the key).
void init_select_state(SelState* h, int f64) {
  *h = SelState{};
  h->shift[0] = h->shift[1] = f64 ? 51u : 19u;
}

}  // namespace lbm
