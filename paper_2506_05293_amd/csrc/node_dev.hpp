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
#pragma clang fp contract(off)
  const uint32_t fb = (lk >> LINK_FORCE_SHIFT) & 0x1FFu;
  if (fb) {
#pragma unroll
    for (int q = 1; q < 9; ++q) {
      if ((fb >> q) & 1u) {
        const T f = g[q] + wgt<T>(q);
        if (cx(q) != 0) fx = fmadd(T(-2 * cx(q)), f, fx);
        if (cy(q) != 0) fy = fmadd(T(-2 * cy(q)), f, fy);
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

// ---- bulk tile ------------------------------------------------------------------
// A bulk workgroup is four wave64, one lattice row each, over the same
// kChunk columns: every lane owns kVec consecutive nodes.  Each population
// plane is read with one aligned vector load per lane; the +-1 column shift of the
// pull is done across lanes (one neighbour element per lane through
// ds_bpermute, plus one halo element at each wave edge), so all global
// traffic is 8- to 32-byte wide per lane and fully coalesced.
//
// Loads and stores address a plane through a wave-uniform base pointer plus a
// 32-bit offset, so no 64-bit address is built per lane.
static_assert(kChunk == 64 * kVec, "one vector row per wave spans a chunk");
constexpr int kV = kVec;

// Vector load / store of kV consecutive elements of one plane: plain loads,
// non-temporal stores.
template <typename V>
__device__ __forceinline__ V ld_vec(const V* p) { return *p; }
template <typename V>
__device__ __forceinline__ void st_vec_nt(V* p, V v) { __builtin_nontemporal_store(v, p); }

template <typename S> struct VecIO;
template <> struct VecIO<float> {
  typedef float v __attribute__((ext_vector_type(kV)));
  __device__ static void ld(const float* p, float* e) {
    const v a = ld_vec(reinterpret_cast<const v*>(p));
#pragma unroll
    for (int i = 0; i < kV; ++i) e[i] = a[i];
  }
  __device__ static void st(float* p, const float* e) {
    v a;
#pragma unroll
    for (int i = 0; i < kV; ++i) a[i] = e[i];
    st_vec_nt(reinterpret_cast<v*>(p), a);
  }
};
template <> struct VecIO<double> {
  typedef double v __attribute__((ext_vector_type(2)));
  __device__ static void ld(const double* p, double* e) {
#pragma unroll
    for (int k = 0; k < kV / 2; ++k) {
      const v a = ld_vec(reinterpret_cast<const v*>(p) + k);
      e[2 * k] = a[0];
      e[2 * k + 1] = a[1];
    }
  }
  __device__ static void st(double* p, const double* e) {
#pragma unroll
    for (int k = 0; k < kV / 2; ++k) {
      const v a = {e[2 * k], e[2 * k + 1]};
      st_vec_nt(reinterpret_cast<v*>(p) + k, a);
    }
  }
};
template <> struct VecIO<__half> {
  typedef unsigned short v __attribute__((ext_vector_type(kV)));
  __device__ static void ld(const __half* p, float* e) {
    const v a = ld_vec(reinterpret_cast<const v*>(p));
#pragma unroll
    for (int i = 0; i < kV; ++i) e[i] = __half2float(__ushort_as_half(a[i]));
  }
  __device__ static void st(__half* p, const float* e) {
    v a;
#pragma unroll
    for (int i = 0; i < kV; ++i) a[i] = __half_as_ushort(to_half(e[i]));
    st_vec_nt(reinterpret_cast<v*>(p), a);
  }
};

template <typename S, int MRT, typename P, typename Hook = NoHook>
__device__ __forceinline__ void bulk_row(const P& L, int tx, int y, int lane,
                                         typename Store<S>::T& fx, typename Store<S>::T& fy,
                                         typename Store<S>::T& dm, const Hook& hook = Hook()) {
  using T = typename Store<S>::T;
  const S* __restrict__ A = static_cast<const S*>(L.A);
  S* __restrict__ B = static_cast<S*>(L.B);
  const uint32_t pitch = uint32_t(L.pitch);
  const int xw = tx * kChunk;                 // first column of this wave
  const int x0 = xw + lane * kV;              // first column of this lane

  int ym = y - 1, yp = y + 1;
  if (ym < 0) ym = L.yper ? L.ny - 1 : 0;
  if (yp >= L.ny) yp = L.yper ? 0 : L.ny - 1;
  const uint32_t r0 = uint32_t(y) * pitch, rm = uint32_t(ym) * pitch, rp = uint32_t(yp) * pitch;
  int hm = xw - 1, hp = xw + kChunk;          // halo columns of the wave
  if (hm < 0) hm = L.xper ? L.nx - 1 : 0;
  if (hp >= L.nx) hp = L.xper ? 0 : L.nx - 1;

  // 1. pull every plane: g[i][q] = A_q(x0 + i - cx_q, y - cy_q)
  T g[kV][9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const S* Aq = A + int64_t(q) * L.plane;
    const uint32_t ro = cy(q) == 1 ? rm : (cy(q) == -1 ? rp : r0);
    T e[kV];
    VecIO<S>::ld(Aq + ro + uint32_t(x0), e);
    if (cx(q) == 0) {
#pragma unroll
      for (int i = 0; i < kV; ++i) g[i][q] = e[i];
    } else if (cx(q) == 1) {
      T prev = __shfl_up(e[kV - 1], 1, 64);
      if (lane == 0) prev = Store<S>::ld(Aq + ro + uint32_t(hm));
      g[0][q] = prev;
#pragma unroll
      for (int i = 1; i < kV; ++i) g[i][q] = e[i - 1];
    } else {
      T next = __shfl_down(e[0], 1, 64);
      if (lane == 63) next = Store<S>::ld(Aq + ro + uint32_t(hp));
      g[kV - 1][q] = next;
#pragma unroll
      for (int i = 0; i < kV - 1; ++i) g[i][q] = e[i + 1];
    }
  }

  // 2. link words of the lane's nodes (only in chunks that have any)
  uint32_t lk[kV];
#pragma unroll
  for (int i = 0; i < kV; ++i) lk[i] = 0u;
  if (L.chunk[y * L.nchunk + tx]) {
#pragma unroll
    for (int i = 0; i < kV; ++i) lk[i] = L.links[r0 + uint32_t(x0 + i)];
  }

  // 3. per node: fix-ups, boundary columns, force, collision
  bool keep[kV];
  bool vec = true;        // the lane's nodes are all updated here or padding
  bool any = false;       // the lane holds at least one node updated here
#pragma unroll
  for (int i = 0; i < kV; ++i) {
    const int x = x0 + i;
    keep[i] = x < L.nx && !(lk[i] & LINK_SOLID) && !((lk[i] & LINK_OUTLET) && L.n_nn);
    vec = vec && (keep[i] || x >= L.nx);
    any = any || keep[i];
    if (!keep[i]) continue;
    if (L.xper && x == L.nx - 1) {            // last column wraps to column 0
#pragma unroll
      for (int q = 0; q < 9; ++q)
        if (cx(q) == -1)
          g[i][q] = Store<S>::ld(A + int64_t(q) * L.plane +
                                 (cy(q) == 1 ? rm : (cy(q) == -1 ? rp : r0)));
    }
    if (lk[i] & 0x1FFu) {                     // half-way bounce-back
#pragma unroll
      for (int q = 1; q < 9; ++q)
        if ((lk[i] >> q) & 1u) g[i][q] = Store<S>::ld(A + int64_t(opp(q)) * L.plane + r0 + uint32_t(x));
    }
    if (lk[i] & (LINK_INLET | LINK_OUTLET)) {
      if (lk[i] & LINK_INLET)
        zouhe_inlet(g[i], L.inlet ? T(L.inlet[y]) : T(L.u_in));
      else
        zouhe_outlet(g[i], T(L.one_minus_rho_out));
    }
    add_force(lk[i], g[i], fx, fy);
    dm += macro(g[i]).drho;
    hook(x, y, g[i]);
    collide<T, MRT>(g[i], L);
  }

  // 4. store: one vector store per plane where the lane's nodes are all
  // updated here or padding (columns nx .. pitch-1 are never read as a valid
  // node's source: the outlet and wrap-around columns replace those pulls),
  // else per node; a lane of padding only stores nothing
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    S* Bq = B + int64_t(q) * L.plane + r0 + uint32_t(x0);
    T e[kV];
#pragma unroll
    for (int i = 0; i < kV; ++i) e[i] = g[i][q];
    if (vec) {
      if (any) VecIO<S>::st(Bq, e);
    } else {
#pragma unroll
      for (int i = 0; i < kV; ++i)
        if (keep[i]) Store<S>::st(Bq + i, e[i]);
    }
  }
}

}  // namespace lbm
