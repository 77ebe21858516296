// D3Q27 site arithmetic: the tensor product of D1Q3 (velocities (a, b, c)
// in {-1, 0, 1}^3, weights w_a w_b w_c, tensor order i = 9 (c + 1) +
// 3 (b + 1) + (a + 1), opposite 26 - i) with the product of the 1D
// equilibria of section 6.  The lattice is stored as 27 planes of nz * ny
// rows of `pitch` elements, row z * ny + y.
#pragma once

#include "lbm_site.h"

namespace lbm {

// Pull on the periodic 3D lattice, branch-free: three source columns, rows
// and layers, each population at a scalar base plus a 32-bit offset.
// CACHED: cached loads (the caller reads populations again).
template <class S, bool CACHED = false>
__device__ __forceinline__ void pull27(const S* __restrict__ src, long long qs, int pitch, int nx,
                                       int ny, int nz, int x, int y, int z,
                                       typename StoreT<S>::R v[27]) {
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
  const unsigned c[3] = {(unsigned)xp, (unsigned)x, (unsigned)xm};   // a = -1, 0, +1
  const int ys[3] = {yp, y, ym}, zs[3] = {zp, z, zm};
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const unsigned row = (unsigned)((zs[vz_of<27>(i) + 1] * ny + ys[vy_of<27>(i) + 1]) * pitch);
    const S* p = at(src + (long long)i * qs, row + c[vx_of<27>(i) + 1]);
    v[i] = CACHED ? StoreT<S>::ldc(p) : StoreT<S>::ld(p);
  }
}

// m0 = sum_i v_i (rho, or rho - rho0 when shifted) and u = sum_i v_i g_i / rho.
template <class R, bool SH>
__device__ __forceinline__ void moments27(const R v[27], R rho0, R& m0, R& ux, R& uy, R& uz) {
  R s = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    s += v[i];
    if (vx_of<27>(i) != 0) jx += vx_of<27>(i) > 0 ? v[i] : -v[i];
    if (vy_of<27>(i) != 0) jy += vy_of<27>(i) > 0 ? v[i] : -v[i];
    if (vz_of<27>(i) != 0) jz += vz_of<27>(i) > 0 ? v[i] : -v[i];
  }
  m0 = s;
  const R rho = SH ? rho0 + s : s;
  const R ir = rcp<R>(rho);
  ux = qdiv<R>(jx, rho, ir);
  uy = qdiv<R>(jy, rho, ir);
  uz = qdiv<R>(jz, rho, ir);
}

// f*_abc = (rho/216) (c_a + dt_a)(c_b + dt_b)(c_c + dt_c) with the integer
// weights c = (1, 4, 1) (eq_dev6), in the storage representation: with
// P_ab = (c_a + dt_a)(c_b + dt_b), C_ab = c_a c_b and D_ab = P_ab - C_ab,
// f*_abc - w_abc rho0 = (m0/216) C_ab c_c + (rho/216) (D_ab c_c + P_ab dt_c).
template <class R, bool SH>
__device__ __forceinline__ void equilibrium27(R m0, R rho0, R ux, R uy, R uz, int kind,
                                              R feq[27]) {
  R dx[3], dy[3], dz[3];
  eq_dev6<R>(ux, kind, dx);
  eq_dev6<R>(uy, kind, dy);
  eq_dev6<R>(uz, kind, dz);
  const R rho = SH ? rho0 + m0 : m0;
  constexpr R S = R(216), iS = R(1) / S;
  const R rs = qdiv<R>(rho, S, iS);
  const R ms = qdiv<R>(m0, S, iS);
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const int a = vx_of<27>(i), b = vy_of<27>(i), c = vz_of<27>(i);
    const R ca = (R)c1(a), cb = (R)c1(b), cc = (R)c1(c);
    const R da = dx[a + 1], db = dy[b + 1], dc = dz[c + 1];
    if (SH) {
      const R cab = ca * cb;
      const R pab = (ca + da) * (cb + db);
      const R dab = ca * db + da * cb + da * db;
      feq[i] = ms * (cab * cc) + rs * (dab * cc + pab * dc);
    } else {
      feq[i] = rs * ((ca + da) * (cb + db) * (cc + dc));
    }
  }
}

}  // namespace lbm
