// Node update of the D2Q9 step shared by the single-lattice and the batched
// kernels: pull streaming with half-way bounce-back (Sec. 2.1 Eq. 1,
// Sec. 2.3 Eq. 12), Zou & He inlet / outlet columns (Sec. 2.2), the
// momentum-exchange force (Eqs. 14-15) and the collision (Eq. 2 or MRT).
#pragma once

#include "d2q9_dev.hpp"
#include "lbm_internal.hpp"

namespace lbm {

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <typename T, int MRT, typename P>
__device__ __forceinline__ void collide(T g[9], const P& L) {
  if constexpr (MRT) {
    const MrtRates<T> r{T(L.s_e), T(L.s_eps), T(L.s_q), T(L.omega)};
    collide_mrt(g, r);
  } else {
    collide_bgk(g, T(L.omega));
  }
}

// Momentum exchange of one node: population q was bounced back off a body
// node in direction -c_q; the link carries 2 f*_qbar (-c_q) into the body.
template <typename T>
__device__ __forceinline__ void add_force(uint32_t lk, const T g[9], T& fx, T& fy) {
  const uint32_t fb = (lk >> LINK_FORCE_SHIFT) & 0x1FFu;
  if (fb) {
#pragma unroll
    for (int q = 1; q < 9; ++q) {
      if ((fb >> q) & 1u) {
        const T f = g[q] + wgt<T>(q);
        fx -= T(2 * cx(q)) * f;
        fy -= T(2 * cy(q)) * f;
      }
    }
  }
}

// Element access through a wave-uniform plane pointer and a 32-bit byte offset.
template <typename S>
__device__ __forceinline__ typename Store<S>::T ld_at(const S* plane, uint32_t byte_off) {
  return Store<S>::ld_nt(reinterpret_cast<const S*>(reinterpret_cast<const char*>(plane) + byte_off));
}
template <typename S>
__device__ __forceinline__ void st_at(S* plane, uint32_t byte_off, typename Store<S>::T v) {
  Store<S>::st(reinterpret_cast<S*>(reinterpret_cast<char*>(plane) + byte_off), v);
}

// A no-op observer of the pre-collision populations of a node.
struct NoHook {
  template <typename T>
  __device__ void operator()(int, int, const T*) const {}
};

// One node per thread: the pull reads each plane at x - c_q directly (one
// element off alignment for c_x != 0; the neighbouring wave's cache line),
// with the non-temporal hint.
// P is any parameter struct with the fields of StepLaunch that a node uses
// (buffers, geometry, sizes, boundary flags, rates); `hook` sees the
// completed pre-collision populations of every updated node.
template <typename S, int MRT, typename P, typename Hook = NoHook>
__device__ __forceinline__ void bulk_node(const P& L, int tx, int x, int y,
                                          typename Store<S>::T& fx, typename Store<S>::T& fy,
                                          typename Store<S>::T& dm, const Hook& hook = Hook()) {
  using T = typename Store<S>::T;
  const S* __restrict__ A = static_cast<const S*>(L.A);
  S* __restrict__ B = static_cast<S*>(L.B);
  constexpr uint32_t es = sizeof(S);
  const uint32_t pitch = uint32_t(L.pitch);
  const uint32_t self = (uint32_t(y) * pitch + uint32_t(x)) * es;
  uint32_t lk = 0;
  if (L.chunk[y * L.nchunk + tx]) lk = L.links[uint32_t(y) * pitch + uint32_t(x)];
  if (lk & LINK_SOLID) return;
  if ((lk & LINK_OUTLET) && L.n_nn) return;   // done by the neural blocks

  int xm = x - 1, xp = x + 1, ym = y - 1, yp = y + 1;
  if (xm < 0) xm = L.xper ? L.nx - 1 : 0;
  if (xp >= L.nx) xp = L.xper ? 0 : L.nx - 1;
  if (ym < 0) ym = L.yper ? L.ny - 1 : 0;
  if (yp >= L.ny) yp = L.yper ? 0 : L.ny - 1;
  const uint32_t rm = uint32_t(ym) * pitch, r0 = uint32_t(y) * pitch, rp = uint32_t(yp) * pitch;

  T g[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const uint32_t sx = uint32_t(cx(q) == 1 ? xm : (cx(q) == -1 ? xp : x));
    const uint32_t sr = cy(q) == 1 ? rm : (cy(q) == -1 ? rp : r0);
    g[q] = ld_at(A + int64_t(q) * L.plane, (sr + sx) * es);
  }
  if (lk & 0x1FFu) {
#pragma unroll
    for (int q = 1; q < 9; ++q)
      if ((lk >> q) & 1u) g[q] = ld_at(A + int64_t(opp(q)) * L.plane, self);
  }
  if (lk & (LINK_INLET | LINK_OUTLET)) {
    if (lk & LINK_INLET)
      zouhe_inlet(g, L.inlet ? T(L.inlet[y]) : T(L.u_in));
    else
      zouhe_outlet(g, T(L.one_minus_rho_out));
  }
  add_force(lk, g, fx, fy);
  dm += macro(g).drho;
  hook(x, y, g);
  collide<T, MRT>(g, L);
#pragma unroll
  for (int q = 0; q < 9; ++q) st_at(B + int64_t(q) * L.plane, self, g[q]);
}

}  // namespace lbm
