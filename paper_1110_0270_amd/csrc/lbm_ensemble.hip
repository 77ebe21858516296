// Ensemble-dependent limiters of section 4 ("Smooth limiters", "Monitoring
// total dissipation"): the statistics of the step's pre-collision Delta S
// field that the limiter f* + phi (f - f*) needs before the collision.
//   k_ens_reset   clears the sums and the histogram, sets the fixed
//                 threshold;
//   k_ens_pre     Delta S of every site (the step kernel's own site
//                 preparation, so both see the same values) into a buffer,
//                 the sums behind E(Delta S) and the LBGK production
//                 P = sum [1 - (omega - 1)^2] Delta S, and the first level of
//                 a histogram of Delta S keys (counts and FP64 sums);
//   k_ens_reduce  (one workgroup) after the pre-pass: E and delta_0 P; then,
//                 per level of a radix descent over the keys (12 bits at a
//                 time, FP32 keys in 3 levels, FP64 in 6), the bin in which
//                 L(s) = sum max(Delta S - s, 0) crosses delta_0 P (eq.
//                 EntThresh); at a bin's lower edge e, L(e) = S(>= e) - e
//                 N(>= e) from the counts and sums of the bins above;
//   k_ens_hist    the next level's histogram of the keys inside that bin.
// When every key bit is resolved the crossing lies between the key v* and
// the next larger value, where L(s) = S(> v*) - s N(> v*) is linear:
// Delta S_0 = (S(> v*) - delta_0 P) / N(> v*), and Delta S_t =
// max(Delta S_0, delta).
#include <algorithm>

#include "lbm_site.h"

namespace lbm {

template <class R> struct EnsBits;
template <> struct EnsBits<float> { static constexpr int total = 32; };
template <> struct EnsBits<double> { static constexpr int total = 64; };

__host__ __device__ inline int ens_level_bits(int total, int done) {
  const int rem = total - done;
  return rem < 12 ? rem : 12;
}

template <class R>
__device__ __forceinline__ bool ens_finite(R v) { return v == v && v < r_inf<R>(); }

__global__ void k_ens_reset(EnsState* E, unsigned int* cnt, double* sum, int descent,
                            double delta, int fixed) {
  const int t = threadIdx.x;
  for (int b = t; b < kEnsBins; b += blockDim.x) { cnt[b] = 0; sum[b] = 0.0; }
  for (int i = t; i < kEnsSlots * 4; i += blockDim.x) (&E->step_acc[0][0])[i] = 0.0;
  if (t == 0) {
    E->sum_dS = 0.0; E->production = 0.0; E->n_finite = 0.0;
    E->mean = 0.0; E->rhs = 0.0; E->above_n = 0.0; E->above_s = 0.0;
    E->prefix = 0ull; E->prefix_bits = 0; E->active = descent;
    E->threshold = fixed ? delta : __builtin_huge_val();
  }
}

// Sum over the workgroup (256 threads) into LDS slot w[0..2].
__device__ __forceinline__ void block_sum3(double a, double b, double c, double* out) {
  __shared__ double part[4][3];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
    c += __shfl_xor(c, o);
  }
  const int w = threadIdx.x / 64;
  if (__lane_id() == 0) { part[w][0] = a; part[w][1] = b; part[w][2] = c; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < 3; ++k) out[k] = part[0][k] + part[1][k] + part[2][k] + part[3][k];
  }
}

template <class S, int Q, bool HIST>
__global__ __launch_bounds__(256) void k_ens_pre(const StepArgs<typename StoreT<S>::R> A) {
  using R = typename StoreT<S>::R;
  using K = typename KeyOf<R>::T;
  constexpr int TB = EnsBits<R>::total;
  __shared__ unsigned int hc[HIST ? kEnsBins : 1];
  __shared__ double hs[HIST ? kEnsBins : 1];
  if constexpr (HIST) {
    for (int b = threadIdx.x; b < kEnsBins; b += blockDim.x) { hc[b] = 0; hs[b] = 0.0; }
    __syncthreads();
  }
  const long long n = (long long)A.nx * A.ny;
  double s_dS = 0.0, s_prod = 0.0, s_n = 0.0;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(s / A.nx), x = (int)(s % A.nx);
    R v[Q], feq[Q], d[Q], m0, ux, uy;
    const R dS = site_prep<S, Q, false, false>(A, x, y, v, feq, d, m0, ux, uy, true);
    const long long o = (long long)y * A.pitch + x;
    A.ens_dsb[o] = dS;
    if (ens_finite<R>(dS)) {
      const R om = A.omega_field ? A.omega_field[o] : A.omega;
      const double c = 1.0 - ((double)om - 1.0) * ((double)om - 1.0);
      s_dS += (double)dS;
      s_prod += c * (double)dS;
      s_n += 1.0;
      if constexpr (HIST) {
        const unsigned b = (unsigned)((unsigned long long)key_of<R>(dS) >> (TB - 12));
        atomicAdd(&hc[b], 1u);
        atomicAdd(&hs[b], (double)dS);
      }
    }
  }
  __shared__ double tot[3];
  block_sum3(s_dS, s_prod, s_n, tot);
  if (threadIdx.x == 0) {
    if (tot[2] > 0.0) {
      atomicAdd(&A.ens->sum_dS, tot[0]);
      atomicAdd(&A.ens->production, tot[1]);
      atomicAdd(&A.ens->n_finite, tot[2]);
    }
  }
  if constexpr (HIST) {
    __syncthreads();
    for (int b = threadIdx.x; b < kEnsBins; b += blockDim.x)
      if (hc[b]) {
        atomicAdd(&A.ens_cnt[b], hc[b]);
        atomicAdd(&A.ens_sum[b], hs[b]);
      }
  }
}

// Histogram of the next level: keys inside the bin resolved so far.
template <class R>
__global__ __launch_bounds__(256) void k_ens_hist(const R* dsb, int nx, int ny, int pitch,
                                                  const EnsState* E, unsigned int* cnt,
                                                  double* sum) {
  constexpr int TB = EnsBits<R>::total;
  if (!E->active) return;
  __shared__ unsigned int hc[kEnsBins];
  __shared__ double hs[kEnsBins];
  const unsigned long long prefix = E->prefix;
  const int pb = E->prefix_bits;
  const int nb = ens_level_bits(TB, pb);
  const int rem = TB - pb;
  for (int b = threadIdx.x; b < kEnsBins; b += blockDim.x) { hc[b] = 0; hs[b] = 0.0; }
  __syncthreads();
  const long long n = (long long)nx * ny;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(s / nx), x = (int)(s % nx);
    const R v = dsb[(long long)y * pitch + x];
    if (!ens_finite<R>(v)) continue;
    const unsigned long long key = (unsigned long long)key_of<R>(v);
    if ((rem >= 64 ? 0ull : (key >> rem)) != prefix) continue;
    const unsigned b = (unsigned)((key >> (rem - nb)) & ((1ull << nb) - 1ull));
    atomicAdd(&hc[b], 1u);
    atomicAdd(&hs[b], (double)v);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kEnsBins; b += blockDim.x)
    if (hc[b]) {
      atomicAdd(&cnt[b], hc[b]);
      atomicAdd(&sum[b], hs[b]);
    }
}

// One workgroup of 1024 threads.  first: after the pre-pass (mean, delta_0 P
// and the level-0 bins).  Bin b of the level spans keys [e_b, e_{b+1}).
template <class R>
__global__ __launch_bounds__(1024) void k_ens_reduce(EnsState* E, unsigned int* cnt, double* sum,
                                                     int first, double delta0, double delta) {
  constexpr int TB = EnsBits<R>::total;
  const int t = threadIdx.x;
  if (first && t == 0) {
    E->mean = E->n_finite > 0.0 ? E->sum_dS / E->n_finite : 0.0;
    E->rhs = delta0 * E->production;
  }
  __syncthreads();
  const int active = E->active;
  const double rhs = E->rhs;
  if (first && active && t == 0) {
    // the budget covers all of it: every limited site goes to Delta S_t = delta
    if (rhs >= E->sum_dS) { E->threshold = delta > 0.0 ? delta : 0.0; E->active = 0; }
    else if (!(rhs > 0.0)) { E->threshold = __builtin_huge_val(); E->active = 0; }
  }
  __syncthreads();
  if (!active || !E->active) {
    for (int b = t; b < kEnsBins; b += blockDim.x) { cnt[b] = 0; sum[b] = 0.0; }
    return;
  }
  const unsigned long long prefix = E->prefix;
  const int pb = E->prefix_bits;
  const int nb = ens_level_bits(TB, pb);
  const int rem = TB - pb;
  const int nbins = 1 << nb;
  const double an = E->above_n, as = E->above_s;
  // thread t owns bins [4t, 4t + 4) of the level's nbins (<= 4096)
  double cn[4], cs[4], tn = 0.0, ts = 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int b = 4 * t + j;
    cn[j] = b < nbins ? (double)cnt[b] : 0.0;
    cs[j] = b < nbins ? sum[b] : 0.0;
    tn += cn[j];
    ts += cs[j];
  }
  // exclusive suffix sums over threads (bins above thread t's)
  __shared__ double wn[16], ws[16];
  double sn = tn, ss = ts;        // inclusive suffix within the wavefront
  const int lane = t & 63, w = t >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double a = __shfl_down(sn, o), c = __shfl_down(ss, o);
    if (lane + o < 64) { sn += a; ss += c; }
  }
  if (lane == 0) { wn[w] = sn; ws[w] = ss; }
  __syncthreads();
  double en = sn - tn, es = ss - ts;  // exclusive, within the wavefront
  for (int j = w + 1; j < 16; ++j) { en += wn[j]; es += ws[j]; }
  __shared__ int best;
  if (t == 0) best = -1;
  __syncthreads();
  // bins from the top: L(e_b) = S(>= e_b) - e_b N(>= e_b) is non-increasing in b
  {
    double rn = en, rs = es;
    for (int j = 3; j >= 0; --j) {
      const int b = 4 * t + j;
      rn += cn[j];
      rs += cs[j];
      if (b >= nbins) continue;
      const unsigned long long ek = (pb == 0 ? 0ull : (prefix << rem)) | ((unsigned long long)b << (rem - nb));
      const double e = (double)value_of_key<R>(ek);
      if (e >= 0.0 && (rs + as) - e * (rn + an) >= rhs) atomicMax(&best, b);
    }
  }
  __syncthreads();
  const int bb = best < 0 ? 0 : best;
  if (t == bb / 4) {
    // counts and sums of the bins above the chosen one
    double rn = en, rs = es;
    for (int j = 3; j > bb % 4; --j) { rn += cn[j]; rs += cs[j]; }
    const double nan_ = an + rn, nas = as + rs;
    const unsigned long long np = (pb == 0 ? 0ull : (prefix << nb)) | (unsigned long long)bb;
    const int npb = pb + nb;
    E->above_n = nan_;
    E->above_s = nas;
    E->prefix = np;
    E->prefix_bits = npb;
    if (npb >= TB) {
      // every key bit resolved: the crossing lies between the value v* and
      // the next larger value, where L is linear
      const double vstar = (double)value_of_key<R>(np);
      const double s0 = nan_ > 0.0 ? (nas - rhs) / nan_ : vstar;
      E->threshold = s0 > delta ? s0 : delta;
      E->active = 0;
    }
  }
  __syncthreads();
  for (int b = t; b < kEnsBins; b += blockDim.x) { cnt[b] = 0; sum[b] = 0.0; }
}

template <class S, int Q>
static hipError_t launch_ens_t(const StepArgs<typename StoreT<S>::R>& A, double delta0,
                               double delta, hipStream_t s) {
  using R = typename StoreT<S>::R;
  const bool need_t = A.ens_mode == ENS_THRESHOLD || A.ens_mode == ENS_DOUBLE_MONOTONE;
  const bool descent = need_t && delta0 > 0.0;
  const bool pre = descent || A.ens_mode == ENS_SMOOTH;
  hipLaunchKernelGGL(k_ens_reset, dim3(1), dim3(1024), 0, s, A.ens, A.ens_cnt, A.ens_sum,
                     descent ? 1 : 0, delta, (need_t && !descent) ? 1 : 0);
  if (!pre) return hipGetLastError();
  const long long n = (long long)A.nx * A.ny;
  const int g = (int)std::min<long long>((n + 255) / 256, 2048);
  if (descent)
    hipLaunchKernelGGL((k_ens_pre<S, Q, true>), dim3(g), dim3(256), 0, s, A);
  else
    hipLaunchKernelGGL((k_ens_pre<S, Q, false>), dim3(g), dim3(256), 0, s, A);
  hipLaunchKernelGGL((k_ens_reduce<R>), dim3(1), dim3(1024), 0, s, A.ens, A.ens_cnt, A.ens_sum,
                     1, delta0, delta);
  if (descent) {
    constexpr int TB = EnsBits<R>::total;
    for (int done = 12; done < TB; done += ens_level_bits(TB, done)) {
      hipLaunchKernelGGL((k_ens_hist<R>), dim3(g), dim3(256), 0, s, (const R*)A.ens_dsb, A.nx,
                         A.ny, A.pitch, (const EnsState*)A.ens, A.ens_cnt, A.ens_sum);
      hipLaunchKernelGGL((k_ens_reduce<R>), dim3(1), dim3(1024), 0, s, A.ens, A.ens_cnt,
                         A.ens_sum, 0, delta0, delta);
    }
  }
  return hipGetLastError();
}

hipError_t launch_ensemble(int storage, int Q, const void* args, double delta0, double delta,
                           hipStream_t s) {
  switch (storage * 16 + Q) {
    case 0 * 16 + 9: return launch_ens_t<double, 9>(*(const StepArgs<double>*)args, delta0, delta, s);
    case 0 * 16 + 3: return launch_ens_t<double, 3>(*(const StepArgs<double>*)args, delta0, delta, s);
    case 1 * 16 + 9: return launch_ens_t<float, 9>(*(const StepArgs<float>*)args, delta0, delta, s);
    case 1 * 16 + 3: return launch_ens_t<float, 3>(*(const StepArgs<float>*)args, delta0, delta, s);
    case 2 * 16 + 9: return launch_ens_t<_Float16, 9>(*(const StepArgs<float>*)args, delta0, delta, s);
    case 2 * 16 + 3: return launch_ens_t<_Float16, 3>(*(const StepArgs<float>*)args, delta0, delta, s);
    case 3 * 16 + 9: return launch_ens_t<bf16_t, 9>(*(const StepArgs<float>*)args, delta0, delta, s);
    default: return launch_ens_t<bf16_t, 3>(*(const StepArgs<float>*)args, delta0, delta, s);
  }
}

}  // namespace lbm
