// Lattice initialisation, population I/O, moments and the whole-lattice
// FP64 reductions (mass, momentum, entropy, divergence check).
#include "lbm_site3.h"

namespace lbm {

template <class T>
__device__ __forceinline__ double rd(const void* p, long long i, int f64) {
  return f64 ? ((const double*)p)[i] : (double)((const float*)p)[i];
}
__device__ __forceinline__ void wr(void* p, long long i, double v, int f64) {
  if (f64) ((double*)p)[i] = v;
  else ((float*)p)[i] = (float)v;
}

// f = f*(rho, u) of the configured kind (sections 6 and 8).
template <class S, int Q>
__global__ void k_set_eq(const void* rho, const void* ux, const void* uy, const void* uz, int in_f64, S* lat,
                         long long qs, int nx, int ny, int pitch, int kind, double rho0) {
  using R = typename StoreT<S>::R;
  constexpr bool SH = StoreT<S>::shifted;
  const long long n = (long long)nx * ny;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(s / nx), x = (int)(s % nx);
    const R r = (R)rd<R>(rho, s, in_f64);
    const R u = (R)rd<R>(ux, s, in_f64);
    const R w = (Q >= 9 && uy) ? (R)rd<R>(uy, s, in_f64) : R(0);
    R feq[Q];
    if constexpr (Q == 27) {
      const R wz = uz ? (R)rd<R>(uz, s, in_f64) : R(0);
      equilibrium27<R, SH>(SH ? r - (R)rho0 : r, (R)rho0, u, w, wz, kind, feq);
    } else {
      equilibrium_v<R, Q, SH>(SH ? r - (R)rho0 : r, (R)rho0, u, w, kind, feq);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) StoreT<S>::st(lat + (long long)i * qs + (long long)y * pitch + x, feq[i]);
  }
}

template <class S, int Q>
__global__ void k_set_pop(const void* f, int in_f64, S* lat, long long qs, int nx, int ny,
                          int pitch, double rho0) {
  constexpr bool SH = StoreT<S>::shifted;
  const long long n = (long long)nx * ny;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(s / nx), x = (int)(s % nx);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      double v = rd<double>(f, (long long)i * n + s, in_f64);
      if (SH) v -= wt<double, Q>(i) * rho0;
      StoreT<S>::st(lat + (long long)i * qs + (long long)y * pitch + x,
                    (typename StoreT<S>::R)v);
    }
  }
}

template <class S, int Q>
__global__ void k_get_pop(void* f, int out_f64, const S* lat, long long qs, int nx, int ny,
                          int pitch, double rho0) {
  constexpr bool SH = StoreT<S>::shifted;
  const long long n = (long long)nx * ny;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(s / nx), x = (int)(s % nx);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      double v = (double)StoreT<S>::ld(lat + (long long)i * qs + (long long)y * pitch + x);
      if (SH) v += wt<double, Q>(i) * rho0;
      wr(f, (long long)i * n + s, v, out_f64);
    }
  }
}

// rho = sum f_i, u = sum v_i f_i / rho (section 2), evaluated in FP64.
template <class S, int Q>
__device__ __forceinline__ void site_moments64(const S* lat, long long qs, int pitch, int x, int y,
                                               double rho0, double f[Q], double& rho,
                                               double& jx, double& jy) {
  constexpr bool SH = StoreT<S>::shifted;
  rho = 0.0; jx = 0.0; jy = 0.0;
  double dr = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double g = (double)StoreT<S>::ld(lat + (long long)i * qs + (long long)y * pitch + x);
    f[i] = SH ? g + wt<double, Q>(i) * rho0 : g;
    dr += g;
    jx += vx_of<Q>(i) * g;
    jy += vy_of<Q>(i) * g;
  }
  rho = SH ? rho0 + dr : dr;
}

template <class S, int Q>
__global__ void k_moments(const S* lat, long long qs, int nx, int ny, int pitch, double rho0,
                          void* rho, void* ux, void* uy, int out_f64) {
  const long long n = (long long)nx * ny;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(s / nx), x = (int)(s % nx);
    double f[Q], r, jx, jy;
    site_moments64<S, Q>(lat, qs, pitch, x, y, rho0, f, r, jx, jy);
    wr(rho, s, r, out_f64);
    wr(ux, s, jx / r, out_f64);
    if (uy) wr(uy, s, jy / r, out_f64);
  }
}

// Per-block partial sums in a fixed order (deterministic), then one block
// combines them in a fixed order.
constexpr int kStatsBlocks = 1024;
constexpr int kStatsThreads = 256;

// u at site (x, y) in FP64 (for the vorticity)
template <class S, int Q>
__device__ __forceinline__ void site_u64(const S* lat, long long qs, int pitch, int x, int y,
                                         double rho0, double& ux, double& uy) {
  double f[Q], r, jx, jy;
  site_moments64<S, Q>(lat, qs, pitch, x, y, rho0, f, r, jx, jy);
  ux = jx / r;
  uy = jy / r;
}

template <class S, int Q>
__global__ __launch_bounds__(kStatsThreads) void k_stats(const S* lat, long long qs, int nx,
                                                         int ny, int pitch, int periodic,
                                                         double rho0, double* partial) {
  __shared__ double sm[8][kStatsThreads];
  const long long n = (long long)nx * ny;
  double a_m = 0, a_x = 0, a_y = 0, a_s = 0, a_min = __builtin_huge_val(), a_bad = 0;
  double a_w = 0, a_n = 0;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(s / nx), x = (int)(s % nx);
    double f[Q], r, jx, jy;
    site_moments64<S, Q>(lat, qs, pitch, x, y, rho0, f, r, jx, jy);
    double ent = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (!isfinite(f[i])) a_bad = 1.0;
      if (f[i] > 0.0) ent -= f[i] * log(f[i] / wt<double, Q>(i));
    }
    a_m += r; a_x += jx; a_y += jy; a_s += ent;
    if constexpr (Q == 27) {
      // the z momentum (D3Q27) in the slot of the vorticity sum
#pragma unroll
      for (int i = 0; i < Q; ++i) a_w += vz_of<Q>(i) * (f[i] - (StoreT<S>::shifted ? wt<double, Q>(i) * rho0 : 0.0));
    }
    a_min = fmin(a_min, r);
    // vorticity du_y/dx - du_x/dy by central differences (D2Q9)
    if (Q == 9 && (periodic || (x > 0 && y > 0 && x < nx - 1 && y < ny - 1))) {
      const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
      const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
      double ux_a, uy_a, ux_b, uy_b, ux_c, uy_c, ux_d, uy_d;
      site_u64<S, Q>(lat, qs, pitch, xp, y, rho0, ux_a, uy_a);
      site_u64<S, Q>(lat, qs, pitch, xm, y, rho0, ux_b, uy_b);
      site_u64<S, Q>(lat, qs, pitch, x, yp, rho0, ux_c, uy_c);
      site_u64<S, Q>(lat, qs, pitch, x, ym, rho0, ux_d, uy_d);
      const double w = (uy_a - uy_b) / 2.0 - (ux_c - ux_d) / 2.0;
      a_w += w * w;
      a_n += 1.0;
    }
  }
  const int t = threadIdx.x;
  sm[0][t] = a_m; sm[1][t] = a_x; sm[2][t] = a_y; sm[3][t] = a_s; sm[4][t] = a_min; sm[5][t] = a_bad;
  sm[6][t] = a_w; sm[7][t] = a_n;
  __syncthreads();
  for (int off = kStatsThreads / 2; off > 0; off >>= 1) {
    if (t < off) {
      for (int k = 0; k < 4; ++k) sm[k][t] += sm[k][t + off];
      sm[4][t] = fmin(sm[4][t], sm[4][t + off]);
      sm[5][t] = fmax(sm[5][t], sm[5][t + off]);
      sm[6][t] += sm[6][t + off];
      sm[7][t] += sm[7][t + off];
    }
    __syncthreads();
  }
  if (t < 8) partial[(long long)blockIdx.x * 8 + t] = sm[t][0];
}

__global__ __launch_bounds__(kStatsThreads) void k_stats_final(const double* partial, int nb,
                                                               double* out,
                                                               long long* diverged_step,
                                                               long long step) {
  __shared__ double sm[8][kStatsThreads];
  const int t = threadIdx.x;
  double a[8] = {0, 0, 0, 0, __builtin_huge_val(), 0, 0, 0};
  for (int b = t; b < nb; b += kStatsThreads) {
    for (int k = 0; k < 4; ++k) a[k] += partial[(long long)b * 8 + k];
    a[4] = fmin(a[4], partial[(long long)b * 8 + 4]);
    a[5] = fmax(a[5], partial[(long long)b * 8 + 5]);
    a[6] += partial[(long long)b * 8 + 6];
    a[7] += partial[(long long)b * 8 + 7];
  }
  for (int k = 0; k < 8; ++k) sm[k][t] = a[k];
  __syncthreads();
  for (int off = kStatsThreads / 2; off > 0; off >>= 1) {
    if (t < off) {
      for (int k = 0; k < 4; ++k) sm[k][t] += sm[k][t + off];
      sm[4][t] = fmin(sm[4][t], sm[4][t + off]);
      sm[5][t] = fmax(sm[5][t], sm[5][t + off]);
      sm[6][t] += sm[6][t + off];
      sm[7][t] += sm[7][t + off];
    }
    __syncthreads();
  }
  if (t == 0) {
    for (int k = 0; k < 8; ++k) out[k] = sm[k][0];
    const bool bad = sm[5][0] != 0.0 || !(sm[4][0] > 0.0) || !isfinite(sm[0][0]);
    if (bad && *diverged_step < 0) *diverged_step = step;
  }
}

// ---------------------------------------------------------------------------
static inline int grid_for(long long n) {
  long long g = (n + 255) / 256;
  return (int)(g < 4096 ? (g < 1 ? 1 : g) : 4096);
}

#define LBM_QSWITCH(Q, ...)                                                              \
  if (Q == 27) { constexpr int QQ = 27; __VA_ARGS__; }                                   \
  else if (Q == 9) { constexpr int QQ = 9; __VA_ARGS__; }                                \
  else { constexpr int QQ = 3; __VA_ARGS__; }
#define LBM_DISPATCH(storage, Q, ...)                                                    \
  do {                                                                                   \
    if (storage == 0) { using S = double; LBM_QSWITCH(Q, __VA_ARGS__) }                   \
    else if (storage == 1) { using S = float; LBM_QSWITCH(Q, __VA_ARGS__) }               \
    else if (storage == 2) { using S = _Float16; LBM_QSWITCH(Q, __VA_ARGS__) }            \
    else { using S = bf16_t; LBM_QSWITCH(Q, __VA_ARGS__) }                                \
  } while (0)

hipError_t launch_set_eq(int storage, int Q, const void* rho, const void* ux, const void* uy,
                         const void* uz, int in_f64, void* lat, long long qs, int nx, int ny, int pitch,
                         int eq_kind, double rho0, hipStream_t s) {
  const int g = grid_for((long long)nx * ny);
  LBM_DISPATCH(storage, Q, hipLaunchKernelGGL((k_set_eq<S, QQ>), dim3(g), dim3(256), 0, s, rho, ux, uy, uz, in_f64, (S*)lat, qs, nx, ny, pitch, eq_kind, rho0));
  return hipGetLastError();
}

hipError_t launch_set_pop(int storage, int Q, const void* f, int in_f64, void* lat, long long qs,
                          int nx, int ny, int pitch, double rho0, hipStream_t s) {
  const int g = grid_for((long long)nx * ny);
  LBM_DISPATCH(storage, Q, hipLaunchKernelGGL((k_set_pop<S, QQ>), dim3(g), dim3(256), 0, s, f, in_f64, (S*)lat, qs, nx, ny, pitch, rho0));
  return hipGetLastError();
}

hipError_t launch_get_pop(int storage, int Q, void* f, int out_f64, const void* lat, long long qs,
                          int nx, int ny, int pitch, double rho0, hipStream_t s) {
  const int g = grid_for((long long)nx * ny);
  LBM_DISPATCH(storage, Q, hipLaunchKernelGGL((k_get_pop<S, QQ>), dim3(g), dim3(256), 0, s, f, out_f64, (const S*)lat, qs, nx, ny, pitch, rho0));
  return hipGetLastError();
}

hipError_t launch_moments(int storage, int Q, const void* lat, long long qs, int nx, int ny,
                          int pitch, double rho0, void* rho, void* ux, void* uy, int out_f64,
                          hipStream_t s) {
  const int g = grid_for((long long)nx * ny);
  LBM_DISPATCH(storage, Q, hipLaunchKernelGGL((k_moments<S, QQ>), dim3(g), dim3(256), 0, s, (const S*)lat, qs, nx, ny, pitch, rho0, rho, ux, uy, out_f64));
  return hipGetLastError();
}

long long stats_partial_doubles(int, int) { return (long long)kStatsBlocks * 8; }

hipError_t launch_stats(int storage, int Q, const void* lat, long long qs, int nx, int ny,
                        int pitch, int periodic, double rho0, double* partial, double* out,
                        long long* diverged_step, long long step, hipStream_t s) {
  LBM_DISPATCH(storage, Q, hipLaunchKernelGGL((k_stats<S, QQ>), dim3(kStatsBlocks), dim3(kStatsThreads), 0, s, (const S*)lat, qs, nx, ny, pitch, periodic, rho0, partial));
  hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(kStatsThreads), 0, s, (const double*)partial,
                     kStatsBlocks, out, diverged_step, step);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
}

}  // namespace lbm
