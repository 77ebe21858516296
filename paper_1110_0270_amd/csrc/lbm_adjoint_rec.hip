// Recording side of the adjoint: checkpoint store and selection tape.
#include "lbm_adjoint.h"
#include "lbm_internal.h"

namespace lbm {

static size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

AdjointLayout adjoint_layout(const lbm_config* c, size_t lat_bytes, long long qs, long long k,
                             size_t offset) {
  AdjointLayout L;
  L.end = offset;
  if (c->checkpoint_every <= 0 || c->max_steps <= 0) return L;
  L.on = true;
  L.K = c->checkpoint_every;
  L.max_steps = c->max_steps;
  L.n_ckpt = c->max_steps / L.K + 1;
  L.k = (c->limiters & LBM_LIM_EHRENFEST) ? k : 0;
  L.lat_bytes = lat_bytes;
  const int Q = c->lattice == LBM_D2Q9 ? 9 : 3;
  const size_t rb = c->storage == LBM_F64 ? 8 : 4;
  L.lam_bytes = (size_t)Q * qs * rb;
  size_t o = offset;
  auto take = [&](size_t b) { size_t at = o; o += a256(b); return at; };
  L.off_ckpt = take((size_t)L.n_ckpt * a256(lat_bytes));
  // ELBM: one more state slot, so that the last step of a segment can be
  // recomputed for its alpha
  L.store_alpha = c->collision == LBM_ELBM;
  L.off_seg = take((size_t)(L.K + (L.store_alpha ? 1 : 0)) * a256(lat_bytes));
  if (L.store_alpha) {
    L.off_alpha = take((size_t)L.K * a256((size_t)qs * rb));
    L.off_branch = take((size_t)L.K * a256((size_t)qs));
  }
  L.median = (c->limiters & LBM_LIM_MEDIAN) != 0;
  if (L.median) {
    L.off_med_gs = take((size_t)qs * rb);
    L.off_med_h = take((size_t)qs * rb);
    L.off_med_am = take((size_t)qs);
  }
  L.off_lam[0] = take(L.lam_bytes);
  L.off_lam[1] = take(L.lam_bytes);
  L.off_gom = take((size_t)qs * rb);
  if (L.k > 0) {
    L.off_tape_sel = take((size_t)L.max_steps * L.k * 4);
    L.off_tape_cnt = take((size_t)L.max_steps * 8);
    L.off_mask = take((size_t)c->nx * c->ny);
  }
  L.end = o;
  return L;
}

hipError_t adjoint_begin_record(const AdjointLayout& L, char* ws, const void* lat,
                                size_t lat_bytes, hipStream_t s) {
  if (!L.on) return hipSuccess;
  return hipMemcpyAsync(ws + L.off_ckpt, lat, lat_bytes, hipMemcpyDeviceToDevice, s);
}

hipError_t adjoint_after_step(const AdjointLayout& L, char* ws, long long steps_done,
                              const void* lat, size_t lat_bytes, hipStream_t s) {
  if (!L.on || steps_done % L.K != 0) return hipSuccess;
  const long long slot = steps_done / L.K;
  if (slot >= L.n_ckpt) return hipSuccess;
  return hipMemcpyAsync(ws + L.off_ckpt + (size_t)slot * a256(lat_bytes), lat, lat_bytes,
                        hipMemcpyDeviceToDevice, s);
}

int32_t* adjoint_selected_slot(const AdjointLayout& L, char* ws, long long t, int32_t* dflt) {
  if (!L.on || L.k <= 0 || t < 0 || t >= L.max_steps) return dflt;
  return (int32_t*)(ws + L.off_tape_sel) + (size_t)t * L.k;
}

long long* adjoint_count_slot(const AdjointLayout& L, char* ws, long long t) {
  if (!L.on || L.k <= 0 || t < 0 || t >= L.max_steps) return nullptr;
  return (long long*)(ws + L.off_tape_cnt) + t;
}

__global__ void k_convert_field(const void* src, int src_f64, void* dst, int dst_f64, int nx,
                                int ny, int pitch) {
  const long long n = (long long)nx * ny;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(s / nx), x = (int)(s % nx);
    const double v = src_f64 ? ((const double*)src)[s] : (double)((const float*)src)[s];
    const long long o = (long long)y * pitch + x;
    if (dst_f64) ((double*)dst)[o] = v;
    else ((float*)dst)[o] = (float)v;
  }
}

hipError_t launch_convert_field(const void* src, int src_f64, void* dst, int dst_f64, int nx,
                                int ny, int pitch, hipStream_t s) {
  long long n = (long long)nx * ny;
  int g = (int)std::min<long long>((n + 255) / 256, 4096);
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_convert_field, dim3(g), dim3(256), 0, s, src, src_f64, dst, dst_f64, nx, ny,
                     pitch);
  return hipGetLastError();
}

}  // namespace lbm
